/*
 * bsort oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of bsort (Guzman,
 * "bsort: A theoretically efficient non-comparison-based sorting algorithm
 * for integer and floating-point numbers", arXiv 2603.08929), written from
 * the paper's Sections II and III (Algorithms 1-5).  It exists to check the
 * GPU library; only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code with the GPU path.
 *
 * Keys are raw w-bit patterns (1 <= w <= 64) held in the low bits of a
 * uint64_t.  All bit work is done on the unsigned pattern, never on a
 * signed or floating-point interpretation.
 */
#ifndef BSORT_ORACLE_H
#define BSORT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key interpretation (which top-level routine of Section III runs). */
#define BSO_UNSIGNED 0 /* Algorithm 2 on the whole array              */
#define BSO_SIGNED   1 /* Algorithm 3: two's complement               */
#define BSO_FLOAT    2 /* Algorithms 4+5: sign | exponent | mantissa  */

/* Partition flavour of Algorithm 1. */
#define BSO_LOMUTO 0 /* the paper's swap loop (unstable, in place)    */
#define BSO_STABLE 1 /* same split, both sides keep their input order */

/*
 * Sort keys[0..n) in place.
 *   w          bits per key (1..64; float mode needs w >= 2)
 *   mode       BSO_UNSIGNED / BSO_SIGNED / BSO_FLOAT
 *   mant_bits  float mode only: mantissa width (0 <= mant_bits <= w-2)
 *   asc        1 ascending, 0 descending
 *   flavour    BSO_LOMUTO or BSO_STABLE
 *   idx        nullable; if given, must hold 0..n-1 on entry (or any
 *              payload) and is permuted along with the keys
 *   snap       nullable; (w+1) x n row-major.  Row 0 is the input, row d
 *              the array after every partition on bit w-d has run
 *              (breadth-first view of the recursion).
 *   snap_idx   nullable; same layout for the index payload.
 * Returns 0, or -1 on bad arguments (nothing is written then).
 */
int bso_sort(uint64_t *keys, int64_t *idx, uint64_t n, int w, int mode,
             int mant_bits, int asc, int flavour, uint64_t *snap,
             int64_t *snap_idx);

/*
 * Key and payload found at sorted position j after a stable sort of
 * keys[0..n) with idx = 0..n-1, computed by following only the branch of
 * the recursion that holds position j (binary quickselect with the same
 * partition).  keys is not modified.  Returns 0 or -1.
 */
int bso_select(const uint64_t *keys, uint64_t n, int w, int mode,
               int mant_bits, int asc, uint64_t j, uint64_t *key_out,
               int64_t *idx_out);

/*
 * 128-bit keys: the same algorithms with w = 128, stable flavour.  Key i is
 * the pattern hi[i] * 2^64 + lo[i]; lo and hi are sorted in place, idx
 * (nullable) is permuted with them.  Float mode: sign bit 127, mantissa of
 * mant_bits bits (0 <= mant_bits <= 126; 112 for IEEE binary128).
 * Returns 0 or -1.
 */
int bso_sort128(uint64_t *lo, uint64_t *hi, int64_t *idx, uint64_t n, int mode,
                int mant_bits, int asc);

/* Backward of values = x[idx] along each row: grad_in[r, idx[r,j]] =
 * grad_out[r,j] (the derivative of a gather by a permutation).  Doubles.
 * Returns 0, or -1 if a row of idx is not a permutation. */
int bso_permute_backward(const double *grad_out, const int64_t *idx,
                         uint64_t rows, uint64_t cols, double *grad_in);

#ifdef __cplusplus
}
#endif

#endif
