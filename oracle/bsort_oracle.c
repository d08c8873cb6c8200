/*
 * bsort oracle -- TEST INFRASTRUCTURE ONLY (see bsort_oracle.h).
 *
 * Written from the paper's text, in its notation: a key is a w-bit pattern,
 * m is a single-bit mask, [ps, pe) a half-open partition and asc the sort
 * direction.  Readings taken where the paper is ambiguous:
 *   - ranges are half-open [ps, pe) with 0 <= ps <= pe <= n (Alg. 1 input
 *     spec vs. the call with pe = |a| in Alg. 3);
 *   - a partition of fewer than two elements returns at once (Alg. 2 and 5
 *     have no base case; without it the recursion makes 2^w calls, against
 *     the O(nw) bound of Theorem 4; the result is unchanged);
 *   - the negative half of a float array is sorted in the inverse
 *     direction (Section III-B's three-pass description, Theorem 3 part 3,
 *     and the Fig. 3 trace), not with the literal asc of Algorithm 4;
 *   - the mask is shifted logically (the unsigned pattern is used throughout).
 *
 * Built with -DBSO_MUTANT=k (k > 0) it compiles a deliberately wrong variant
 * used only by the tests that show the paper's pins catch such mistakes.
 */
#include "bsort_oracle.h"

#include <stdlib.h>
#include <string.h>

#ifndef BSO_MUTANT
#define BSO_MUTANT 0
#endif

typedef struct {
  uint64_t *a;       /* keys (w-bit patterns)                       */
  int64_t *idx;      /* payload moved with the keys, or NULL        */
  uint64_t n;
  int w;
  int flavour;       /* BSO_LOMUTO / BSO_STABLE                     */
  uint64_t *tmp_a;   /* stable flavour: staging for the second side */
  int64_t *tmp_i;
  uint64_t *snap;    /* (w+1) x n or NULL                           */
  int64_t *snap_i;
  unsigned char *touched; /* (w+1) x n, set where a row was written */
} bso_ctx;

/* Row of the breadth-first snapshot written after partitioning on mask m:
 * the top bit (m = 2^(w-1)) is row 1, bit 0 is row w. */
static int row_of(const bso_ctx *c, uint64_t m) {
  int b = 0;
  while ((m >> b) != 1) b++;
  return c->w - b;
}

static void record(bso_ctx *c, uint64_t m, uint64_t ps, uint64_t pe) {
  if (!c->snap && !c->snap_i) return;
  const uint64_t r = (uint64_t)row_of(c, m);
  for (uint64_t i = ps; i < pe; ++i) {
    if (c->snap) c->snap[r * c->n + i] = c->a[i];
    if (c->snap_i && c->idx) c->snap_i[r * c->n + i] = c->idx[i];
    c->touched[r * c->n + i] = 1;
  }
}

/*
 * Algorithm 1 (singlePassBSort).  An element goes to the front part
 * [ps, k) when (asc and its masked bit is 0) or (not asc and the bit is 1);
 * returns k.  Lomuto flavour: the paper's swap loop.  Stable flavour: the
 * same split with both sides in their input order (the order shown in the
 * traces of Figs. 1 and 2).
 */
static uint64_t single_pass_bsort(bso_ctx *c, uint64_t m, uint64_t ps,
                                  uint64_t pe, int asc) {
  uint64_t *a = c->a;
  int64_t *idx = c->idx;
  uint64_t k = ps;
  if (c->flavour == BSO_LOMUTO) {
    for (uint64_t i = ps; i < pe; ++i) {
      const int set = (a[i] & m) != 0;
      if ((asc && !set) || (!asc && set)) {
        uint64_t t = a[i]; a[i] = a[k]; a[k] = t;
        if (idx) { int64_t u = idx[i]; idx[i] = idx[k]; idx[k] = u; }
        k++;
      }
    }
  } else {
    uint64_t nsecond = 0;
    for (uint64_t i = ps; i < pe; ++i) {
      const int set = (a[i] & m) != 0;
      if ((asc && !set) || (!asc && set)) {
        a[k] = a[i];
        if (idx) idx[k] = idx[i];
        k++;
      } else {
        c->tmp_a[nsecond] = a[i];
        if (idx) c->tmp_i[nsecond] = idx[i];
        nsecond++;
      }
    }
    memcpy(a + k, c->tmp_a, nsecond * sizeof(uint64_t));
    if (idx) memcpy(idx + k, c->tmp_i, nsecond * sizeof(int64_t));
  }
  record(c, m, ps, pe);
  return k;
}

/* Algorithm 2 (binaryQuickSort): partition on m, then sort both sides on
 * the next lower bit until the mask is exhausted. */
static void binary_quick_sort(bso_ctx *c, uint64_t m, uint64_t ps,
                              uint64_t pe, int asc) {
  if (pe - ps < 2 || m == 0) return;
  const uint64_t k = single_pass_bsort(c, m, ps, pe, asc);
  const uint64_t m2 = m >> 1;
#if BSO_MUTANT == 8
  /* mutant: stops one bit early (bit 0 never partitioned) */
  if (m2 == 1) return;
#endif
  if (m2 == 0) return;
  binary_quick_sort(c, m2, ps, k, asc);
  binary_quick_sort(c, m2, k, pe, asc);
}

/* Algorithm 5 (bsortF): exponent bits by recursion; once the mask reaches
 * the lowest exponent bit (m = 1 << mant_bits) the mantissa is sorted as an
 * unsigned integer with Algorithm 2. */
static void bsort_f(bso_ctx *c, uint64_t m, uint64_t ps, uint64_t pe,
                    int asc, int mant_bits) {
  if (pe - ps < 2 || m == 0) return;
  const uint64_t k = single_pass_bsort(c, m, ps, pe, asc);
  const uint64_t m2 = m >> 1;
  if (m == ((uint64_t)1 << mant_bits)) {
    binary_quick_sort(c, m2, ps, k, asc);
    binary_quick_sort(c, m2, k, pe, asc);
    return;
  }
  bsort_f(c, m2, ps, k, asc, mant_bits);
  bsort_f(c, m2, k, pe, asc, mant_bits);
}

#if BSO_MUTANT >= 3 && BSO_MUTANT <= 5
/* Mutants 3-5 sort the float fields in a wrong hierarchical order (the
 * cases refuted by Theorem 2).  masks[] lists the bits level by level. */
static void gen_order(bso_ctx *c, const uint64_t *masks, int nm, int lvl,
                      uint64_t sign_m, uint64_t ps, uint64_t pe, int asc,
                      int neg) {
  if (pe - ps < 2 || lvl >= nm) return;
  const uint64_t m = masks[lvl];
  int dir = asc;
  if (m == sign_m) dir = !asc;
  else if (neg) dir = !asc;
  const uint64_t k = single_pass_bsort(c, m, ps, pe, dir);
  int neg_lo = neg, neg_hi = neg;
  if (m == sign_m) { neg_lo = asc ? 1 : 0; neg_hi = asc ? 0 : 1; }
  gen_order(c, masks, nm, lvl + 1, sign_m, ps, k, asc, neg_lo);
  gen_order(c, masks, nm, lvl + 1, sign_m, k, pe, asc, neg_hi);
}
#endif

int bso_sort(uint64_t *keys, int64_t *idx, uint64_t n, int w, int mode,
             int mant_bits, int asc, int flavour, uint64_t *snap,
             int64_t *snap_idx) {
  if (w < 1 || w > 64) return -1;
  if (mode != BSO_UNSIGNED && mode != BSO_SIGNED && mode != BSO_FLOAT)
    return -1;
  if (mode == BSO_FLOAT && (w < 2 || mant_bits < 0 || mant_bits > w - 2))
    return -1;
  if (flavour != BSO_LOMUTO && flavour != BSO_STABLE) return -1;
  if (n > 0 && !keys) return -1;
  if (snap_idx && !idx) return -1;
  const uint64_t wmask = (w == 64) ? ~(uint64_t)0 : (((uint64_t)1 << w) - 1);
  for (uint64_t i = 0; i < n; ++i)
    if (keys[i] & ~wmask) return -1;

  bso_ctx c;
  memset(&c, 0, sizeof c);
  c.a = keys; c.idx = idx; c.n = n; c.w = w; c.flavour = flavour;
  c.snap = snap; c.snap_i = snap_idx;
  if (flavour == BSO_STABLE && n > 0) {
    c.tmp_a = (uint64_t *)malloc(n * sizeof(uint64_t));
    c.tmp_i = (int64_t *)malloc(n * sizeof(int64_t));
    if (!c.tmp_a || !c.tmp_i) { free(c.tmp_a); free(c.tmp_i); return -1; }
  }
  if (snap || snap_idx) {
    c.touched = (unsigned char *)calloc((size_t)(w + 1) * (n ? n : 1), 1);
    if (!c.touched) { free(c.tmp_a); free(c.tmp_i); return -1; }
    for (uint64_t i = 0; i < n; ++i) {
      if (snap) snap[i] = keys[i];
      if (snap_idx) snap_idx[i] = idx[i];
      c.touched[i] = 1;
    }
  }

  const uint64_t top = (uint64_t)1 << (w - 1);
  if (n >= 2) {
    if (mode == BSO_UNSIGNED) {
      binary_quick_sort(&c, top, 0, n, asc);
    } else if (mode == BSO_SIGNED) {
      /* Algorithm 3: the sign pass runs in the inverse direction, then both
       * halves are sorted as unsigned on the remaining bits. */
#if BSO_MUTANT == 2
      const uint64_t k = single_pass_bsort(&c, top, 0, n, asc);
#else
      const uint64_t k = single_pass_bsort(&c, top, 0, n, !asc);
#endif
#if BSO_MUTANT == 9
      binary_quick_sort(&c, top >> 1, 0, k, !asc);
      binary_quick_sort(&c, top >> 1, k, n, !asc);
#else
      binary_quick_sort(&c, top >> 1, 0, k, asc);
      binary_quick_sort(&c, top >> 1, k, n, asc);
#endif
    } else {
#if BSO_MUTANT >= 3 && BSO_MUTANT <= 5
      uint64_t masks[64];
      int nm = 0;
      const int e_hi = w - 2, e_lo = mant_bits; /* exponent bits */
      const int m_hi = mant_bits - 1;           /* mantissa bits */
#if BSO_MUTANT == 3 /* sign, mantissa, exponent (Theorem 2, case 2) */
      masks[nm++] = top;
      for (int b = m_hi; b >= 0; --b) masks[nm++] = (uint64_t)1 << b;
      for (int b = e_hi; b >= e_lo; --b) masks[nm++] = (uint64_t)1 << b;
#elif BSO_MUTANT == 4 /* exponent, sign, mantissa (case 1) */
      for (int b = e_hi; b >= e_lo; --b) masks[nm++] = (uint64_t)1 << b;
      masks[nm++] = top;
      for (int b = m_hi; b >= 0; --b) masks[nm++] = (uint64_t)1 << b;
#else /* mantissa, exponent, sign (case 1) */
      for (int b = m_hi; b >= 0; --b) masks[nm++] = (uint64_t)1 << b;
      for (int b = e_hi; b >= e_lo; --b) masks[nm++] = (uint64_t)1 << b;
      masks[nm++] = top;
#endif
      gen_order(&c, masks, nm, 0, top, 0, n, asc, 0);
#else
      /* Algorithm 4: sign pass in the inverse direction.  With !asc the
       * front part [0, k) holds the set sign bits (negatives) when sorting
       * ascending and the clear ones when sorting descending. */
#if BSO_MUTANT == 2
      const uint64_t k = single_pass_bsort(&c, top, 0, n, asc);
#else
      const uint64_t k = single_pass_bsort(&c, top, 0, n, !asc);
#endif
      uint64_t neg_ps = asc ? 0 : k, neg_pe = asc ? k : n;
      uint64_t pos_ps = asc ? k : 0, pos_pe = asc ? n : k;
#if BSO_MUTANT == 1
      /* mutant: the literal pseudocode passes asc to both halves */
      bsort_f(&c, top >> 1, neg_ps, neg_pe, asc, mant_bits);
#else
      bsort_f(&c, top >> 1, neg_ps, neg_pe, !asc, mant_bits);
#endif
      bsort_f(&c, top >> 1, pos_ps, pos_pe, asc, mant_bits);
#endif
    }
  }

  if (c.touched) {
    for (int r = 1; r <= w; ++r)
      for (uint64_t i = 0; i < n; ++i)
        if (!c.touched[(uint64_t)r * n + i]) {
          if (snap) snap[(uint64_t)r * n + i] = snap[(uint64_t)(r - 1) * n + i];
          if (snap_idx)
            snap_idx[(uint64_t)r * n + i] = snap_idx[(uint64_t)(r - 1) * n + i];
        }
  }
  free(c.touched);
  free(c.tmp_a);
  free(c.tmp_i);
  return 0;
}

/* ---------------------------------------------------------------- w = 128
 * The same steps for 128-bit patterns (Section III-C: the method holds for
 * any word size), stable flavour: Algorithm 1 splits on a single-bit mask
 * m, Algorithm 2 recurses to the next lower bit, Algorithm 3 inverts the
 * sign pass, Algorithms 4 and 5 also invert the negative half. */
typedef unsigned __int128 bso_u128;

typedef struct {
  bso_u128 *a;
  int64_t *idx;
  bso_u128 *tmp_a;
  int64_t *tmp_i;
} bso_ctx128;

static uint64_t split128(bso_ctx128 *c, bso_u128 m, uint64_t ps, uint64_t pe, int asc) {
  uint64_t k = ps, nsecond = 0;
  for (uint64_t i = ps; i < pe; ++i) {
    const int set = (c->a[i] & m) != 0;
    if ((asc && !set) || (!asc && set)) {
      c->a[k] = c->a[i];
      if (c->idx) c->idx[k] = c->idx[i];
      k++;
    } else {
      c->tmp_a[nsecond] = c->a[i];
      if (c->idx) c->tmp_i[nsecond] = c->idx[i];
      nsecond++;
    }
  }
  memcpy(c->a + k, c->tmp_a, nsecond * sizeof(bso_u128));
  if (c->idx) memcpy(c->idx + k, c->tmp_i, nsecond * sizeof(int64_t));
  return k;
}

static void bqs128(bso_ctx128 *c, bso_u128 m, uint64_t ps, uint64_t pe, int asc) {
  if (pe - ps < 2 || m == 0) return;
  const uint64_t k = split128(c, m, ps, pe, asc);
  bqs128(c, m >> 1, ps, k, asc);
  bqs128(c, m >> 1, k, pe, asc);
}

static void bsortf128(bso_ctx128 *c, bso_u128 m, uint64_t ps, uint64_t pe, int asc,
                      int mant_bits) {
  if (pe - ps < 2 || m == 0) return;
  const uint64_t k = split128(c, m, ps, pe, asc);
  if (m == ((bso_u128)1 << mant_bits)) {
    bqs128(c, m >> 1, ps, k, asc);
    bqs128(c, m >> 1, k, pe, asc);
    return;
  }
  bsortf128(c, m >> 1, ps, k, asc, mant_bits);
  bsortf128(c, m >> 1, k, pe, asc, mant_bits);
}

int bso_sort128(uint64_t *lo, uint64_t *hi, int64_t *idx, uint64_t n, int mode,
                int mant_bits, int asc) {
  if (mode != BSO_UNSIGNED && mode != BSO_SIGNED && mode != BSO_FLOAT) return -1;
  if (mode == BSO_FLOAT && (mant_bits < 0 || mant_bits > 126)) return -1;
  if (n > 0 && (!lo || !hi)) return -1;
  bso_ctx128 c;
  memset(&c, 0, sizeof c);
  c.idx = idx;
  if (n > 0) {
    c.a = (bso_u128 *)malloc(n * sizeof(bso_u128));
    c.tmp_a = (bso_u128 *)malloc(n * sizeof(bso_u128));
    c.tmp_i = (int64_t *)malloc(n * sizeof(int64_t));
    if (!c.a || !c.tmp_a || !c.tmp_i) {
      free(c.a); free(c.tmp_a); free(c.tmp_i);
      return -1;
    }
    for (uint64_t i = 0; i < n; ++i) c.a[i] = ((bso_u128)hi[i] << 64) | lo[i];
  }
  const bso_u128 top = (bso_u128)1 << 127;
  if (n >= 2) {
    if (mode == BSO_UNSIGNED) {
      bqs128(&c, top, 0, n, asc);
    } else if (mode == BSO_SIGNED) {
      const uint64_t k = split128(&c, top, 0, n, !asc);
      bqs128(&c, top >> 1, 0, k, asc);
      bqs128(&c, top >> 1, k, n, asc);
    } else {
      const uint64_t k = split128(&c, top, 0, n, !asc);
      const uint64_t neg_ps = asc ? 0 : k, neg_pe = asc ? k : n;
      const uint64_t pos_ps = asc ? k : 0, pos_pe = asc ? n : k;
      bsortf128(&c, top >> 1, neg_ps, neg_pe, !asc, mant_bits);
      bsortf128(&c, top >> 1, pos_ps, pos_pe, asc, mant_bits);
    }
  }
  for (uint64_t i = 0; i < n; ++i) {
    lo[i] = (uint64_t)c.a[i];
    hi[i] = (uint64_t)(c.a[i] >> 64);
  }
  free(c.a);
  free(c.tmp_a);
  free(c.tmp_i);
  return 0;
}

/*
 * Quickselect with the paper's partition: run the same sequence of
 * partitions as bso_sort (stable flavour) but descend only into the side
 * that holds sorted position j.  The mask sequence and directions are those
 * of Algorithms 2-5, tracked explicitly instead of by recursion.
 */
int bso_select(const uint64_t *keys, uint64_t n, int w, int mode,
               int mant_bits, int asc, uint64_t j, uint64_t *key_out,
               int64_t *idx_out) {
  if (!keys || !key_out || !idx_out || j >= n) return -1;
  if (w < 1 || w > 64) return -1;
  if (mode != BSO_UNSIGNED && mode != BSO_SIGNED && mode != BSO_FLOAT)
    return -1;
  if (mode == BSO_FLOAT && (w < 2 || mant_bits < 0 || mant_bits > w - 2))
    return -1;
  uint64_t *a = (uint64_t *)malloc(n * sizeof(uint64_t));
  int64_t *ix = (int64_t *)malloc(n * sizeof(int64_t));
  if (!a || !ix) { free(a); free(ix); return -1; }
  memcpy(a, keys, n * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; ++i) ix[i] = (int64_t)i;

  bso_ctx c;
  memset(&c, 0, sizeof c);
  c.a = a; c.idx = ix; c.n = n; c.w = w; c.flavour = BSO_STABLE;
  c.tmp_a = (uint64_t *)malloc(n * sizeof(uint64_t));
  c.tmp_i = (int64_t *)malloc(n * sizeof(int64_t));
  if (!c.tmp_a || !c.tmp_i) {
    free(a); free(ix); free(c.tmp_a); free(c.tmp_i); return -1;
  }

  uint64_t ps = 0, pe = n;
  uint64_t m = (uint64_t)1 << (w - 1);
  int dir = asc;
  if (mode != BSO_UNSIGNED) dir = !asc; /* sign pass of Alg. 3 / Alg. 4 */
  int first = 1;
  while (pe - ps >= 2 && m != 0) {
    const uint64_t k = single_pass_bsort(&c, m, ps, pe, dir);
    if (j < k) pe = k; else ps = k;
    if (first && mode != BSO_UNSIGNED) {
      /* after the sign pass: the chosen half's direction */
      int chose_front = (j < k);
      if (mode == BSO_SIGNED) {
        dir = asc;
      } else {
        /* front half is negative iff asc (see bso_sort) */
        int negative = asc ? chose_front : !chose_front;
        dir = negative ? !asc : asc;
      }
    }
    first = 0;
    m >>= 1;
  }
  *key_out = a[j];
  *idx_out = ix[j];
  free(a); free(ix); free(c.tmp_a); free(c.tmp_i);
  (void)mant_bits; /* the field switch of Alg. 5 does not change the order */
  return 0;
}

int bso_permute_backward(const double *grad_out, const int64_t *idx,
                         uint64_t rows, uint64_t cols, double *grad_in) {
  if ((rows * cols) > 0 && (!grad_out || !idx || !grad_in)) return -1;
  unsigned char *seen = (unsigned char *)calloc(cols ? cols : 1, 1);
  if (!seen) return -1;
  for (uint64_t r = 0; r < rows; ++r) {
    memset(seen, 0, cols ? cols : 1);
    for (uint64_t j = 0; j < cols; ++j) {
      const int64_t s = idx[r * cols + j];
      if (s < 0 || (uint64_t)s >= cols || seen[s]) { free(seen); return -1; }
      seen[s] = 1;
      grad_in[r * cols + (uint64_t)s] = grad_out[r * cols + j];
    }
  }
  free(seen);
  return 0;
}
