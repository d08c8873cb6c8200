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

/* Section II: the i-th partitioning step (1 <= i <= s, s = the key width)
 * tests the single-bit mask m = 1 << (s - i), most significant bit first.
 * The breadth-first snapshot row written after step i is row i. */
static uint64_t step_mask(const bso_ctx *c, int i) {
  return (uint64_t)1 << (c->w - i);
}

static void record(bso_ctx *c, int i, uint64_t ps, uint64_t pe) {
  if (!c->snap && !c->snap_i) return;
  const uint64_t r = (uint64_t)i;
  for (uint64_t j = ps; j < pe; ++j) {
    if (c->snap) c->snap[r * c->n + j] = c->a[j];
    if (c->snap_i && c->idx) c->snap_i[r * c->n + j] = c->idx[j];
    c->touched[r * c->n + j] = 1;
  }
}

/*
 * The two sub-arrays of a step (Section II's invariants): a' holds the
 * elements with (a AND m) != 0, a'' those with (a AND m) == 0.  The
 * direction decides which one comes first: a'' when ascending (a clear bit
 * is the smaller value), a' when descending.
 */
static int joins_first(uint64_t key, uint64_t m, int asc) {
  const int in_a1 = (key & m) != 0; /* a' */
  return asc ? !in_a1 : in_a1;
}

static void exchange(bso_ctx *c, uint64_t x, uint64_t y) {
  const uint64_t t = c->a[x];
  c->a[x] = c->a[y];
  c->a[y] = t;
  if (c->idx) {
    const int64_t u = c->idx[x];
    c->idx[x] = c->idx[y];
    c->idx[y] = u;
  }
}

/*
 * One partitioning step (Algorithm 1, singlePassBSort) on [ps, pe): the
 * sub-array that comes first ends up in [ps, k), the other in [k, pe);
 * returns k.
 *  - BSO_LOMUTO, in place: [ps, k) always holds exactly the first-part
 *    elements met so far, so each further one is exchanged into slot k.
 *  - BSO_STABLE: both sub-arrays in their input order (the order the traces
 *    of Figs. 1 and 2 show), the second one through a staging buffer.
 */
static uint64_t partition_step(bso_ctx *c, int i, uint64_t ps, uint64_t pe,
                               int asc) {
  const uint64_t m = step_mask(c, i);
  uint64_t k = ps;
  if (c->flavour == BSO_LOMUTO) {
    for (uint64_t j = ps; j < pe; ++j)
      if (joins_first(c->a[j], m, asc)) exchange(c, j, k++);
  } else {
    /* first-part elements move down to slot k in input order; the others
     * wait in the staging buffer, in input order, and follow them */
    uint64_t nsecond = 0;
    for (uint64_t j = ps; j < pe; ++j) {
      if (joins_first(c->a[j], m, asc)) {
        c->a[k] = c->a[j];
        if (c->idx) c->idx[k] = c->idx[j];
        k++;
      } else {
        c->tmp_a[nsecond] = c->a[j];
        if (c->idx) c->tmp_i[nsecond] = c->idx[j];
        nsecond++;
      }
    }
    memcpy(c->a + k, c->tmp_a, nsecond * sizeof(uint64_t));
    if (c->idx) memcpy(c->idx + k, c->tmp_i, nsecond * sizeof(int64_t));
  }
  record(c, i, ps, pe);
  return k;
}

/* Algorithm 2 (binaryQuickSort): a step splits the range, then both
 * sub-arrays are sorted from the next step on.  A range of fewer than two
 * elements, or a step past s, is left as it is: splitting it changes
 * nothing, and stopping there avoids the 2^s calls a literal recursion
 * makes (Theorem 4's linear bound assumes it stops). */
static void sort_from_step(bso_ctx *c, int i, uint64_t ps, uint64_t pe,
                           int asc) {
  if (pe - ps < 2 || i > c->w) return;
#if BSO_MUTANT == 8
  /* mutant: stops one bit early (the last step, bit 0, never runs) */
  if (i == c->w) return;
#endif
  const uint64_t k = partition_step(c, i, ps, pe, asc);
  sort_from_step(c, i + 1, ps, k, asc);
  sort_from_step(c, i + 1, k, pe, asc);
}

/* Algorithm 5 (bsortF): the exponent bits by recursion; after the step on
 * the lowest exponent bit (bit mant_bits, step s - mant_bits) the mantissa
 * is sorted as an unsigned integer with Algorithm 2. */
static void bsort_f(bso_ctx *c, int i, uint64_t ps, uint64_t pe, int asc,
                    int mant_bits) {
  if (pe - ps < 2 || i > c->w) return;
  const uint64_t k = partition_step(c, i, ps, pe, asc);
  if (c->w - i == mant_bits) {
    sort_from_step(c, i + 1, ps, k, asc);
    sort_from_step(c, i + 1, k, pe, asc);
    return;
  }
  bsort_f(c, i + 1, ps, k, asc, mant_bits);
  bsort_f(c, i + 1, k, pe, asc, mant_bits);
}

#if BSO_MUTANT >= 3 && BSO_MUTANT <= 5
/* Mutants 3-5 sort the float fields in a wrong hierarchical order (the
 * cases refuted by Theorem 2).  masks[] lists the bits level by level. */
static void gen_order(bso_ctx *c, const int *steps, int nm, int lvl,
                      uint64_t ps, uint64_t pe, int asc, int neg) {
  if (pe - ps < 2 || lvl >= nm) return;
  const int i = steps[lvl];
  int dir = asc;
  if (i == 1) dir = !asc; /* the sign bit */
  else if (neg) dir = !asc;
  const uint64_t k = partition_step(c, i, ps, pe, dir);
  int neg_lo = neg, neg_hi = neg;
  if (i == 1) { neg_lo = asc ? 1 : 0; neg_hi = asc ? 0 : 1; }
  gen_order(c, steps, nm, lvl + 1, ps, k, asc, neg_lo);
  gen_order(c, steps, nm, lvl + 1, k, pe, asc, neg_hi);
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

  if (n >= 2) {
    if (mode == BSO_UNSIGNED) {
      sort_from_step(&c, 1, 0, n, asc);
    } else if (mode == BSO_SIGNED) {
      /* Algorithm 3: the sign pass (step 1) runs in the inverse direction,
       * then both halves are sorted as unsigned from step 2 on. */
#if BSO_MUTANT == 2
      const uint64_t k = partition_step(&c, 1, 0, n, asc);
#else
      const uint64_t k = partition_step(&c, 1, 0, n, !asc);
#endif
#if BSO_MUTANT == 9
      sort_from_step(&c, 2, 0, k, !asc);
      sort_from_step(&c, 2, k, n, !asc);
#else
      sort_from_step(&c, 2, 0, k, asc);
      sort_from_step(&c, 2, k, n, asc);
#endif
    } else {
#if BSO_MUTANT >= 3 && BSO_MUTANT <= 5
      int steps[64]; /* the step of bit b is w - b */
      int nm = 0;
      const int e_hi = w - 2, e_lo = mant_bits; /* exponent bits */
      const int m_hi = mant_bits - 1;           /* mantissa bits */
#if BSO_MUTANT == 3 /* sign, mantissa, exponent (Theorem 2, case 2) */
      steps[nm++] = 1;
      for (int b = m_hi; b >= 0; --b) steps[nm++] = w - b;
      for (int b = e_hi; b >= e_lo; --b) steps[nm++] = w - b;
#elif BSO_MUTANT == 4 /* exponent, sign, mantissa (case 1) */
      for (int b = e_hi; b >= e_lo; --b) steps[nm++] = w - b;
      steps[nm++] = 1;
      for (int b = m_hi; b >= 0; --b) steps[nm++] = w - b;
#else /* mantissa, exponent, sign (case 1) */
      for (int b = m_hi; b >= 0; --b) steps[nm++] = w - b;
      for (int b = e_hi; b >= e_lo; --b) steps[nm++] = w - b;
      steps[nm++] = 1;
#endif
      gen_order(&c, steps, nm, 0, 0, n, asc, 0);
#else
      /* Algorithm 4: sign pass (step 1) in the inverse direction.  With
       * !asc the first part [0, k) holds the set sign bits (negatives) when
       * sorting ascending and the clear ones when sorting descending. */
#if BSO_MUTANT == 2
      const uint64_t k = partition_step(&c, 1, 0, n, asc);
#else
      const uint64_t k = partition_step(&c, 1, 0, n, !asc);
#endif
      uint64_t neg_ps = asc ? 0 : k, neg_pe = asc ? k : n;
      uint64_t pos_ps = asc ? k : 0, pos_pe = asc ? n : k;
#if BSO_MUTANT == 1
      /* mutant: the literal pseudocode passes asc to both halves */
      bsort_f(&c, 2, neg_ps, neg_pe, asc, mant_bits);
#else
      bsort_f(&c, 2, neg_ps, neg_pe, !asc, mant_bits);
#endif
      bsort_f(&c, 2, pos_ps, pos_pe, asc, mant_bits);
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
 * that holds sorted position j.  The step sequence and directions are those
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
  int dir = asc;
  if (mode != BSO_UNSIGNED) dir = !asc; /* sign pass of Alg. 3 / Alg. 4 */
  int first = 1;
  for (int i = 1; pe - ps >= 2 && i <= w; ++i) {
    const uint64_t k = partition_step(&c, i, ps, pe, dir);
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
