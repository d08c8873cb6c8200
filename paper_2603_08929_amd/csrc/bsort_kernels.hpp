// Device side of libbsort: HIP kernels for gfx950 (CDNA4, wave64).
//
// The method (bsort, arXiv 2603.08929, Section II, Algorithms 1-2, and
// Section III, Algorithms 3-5) splits every live part of the array on one
// bit, most significant first, into a front part and a back part, and
// recurses into both.  Here the recursion runs breadth first: one global
// "level" processes the current bit of every live segment at once.
//
// A level is ONE pass over the live keys: each workgroup takes a tile of
// one segment, ranks its keys front/back with wave ballots and an LDS scan,
// finds how many front keys precede the tile through a decoupled look-back
// over the segment's earlier tiles, and scatters the tile as two contiguous
// runs.  The split point of a segment is not needed before its back part is
// written: back keys are placed from the segment's right end leftwards, so
// the back child is stored in reverse order and the next level reads it
// right to left (a per-segment "rev" flag).  The same pass folds the AND and
// OR of each child's keys into per-child accumulators, from which the next
// level picks the child's next bit (bits on which a child is constant are
// skipped: a split with an empty side is the identity) or retires it.
// Segments of at most T keys finish all their remaining bits inside one
// workgroup, in LDS (the hybrid switch to a cache-resident routine that the
// paper proposes in Sections IV-B and V).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsort {

enum : int { MODE_U = 0, MODE_I = 1, MODE_F = 2 };

// Segment descriptor meta bits.
constexpr uint32_t BIT_MASK = 0x7Fu;   // bit to split on next (0..63)
constexpr uint32_t BIT_NONE = 0x7Fu;   // no bit left: copy only
constexpr uint32_t META_REV = 1u << 7; // stored right to left
constexpr uint32_t META_SIGN = 1u << 8;  // float keys of this segment are negative
constexpr uint32_t META_BUF = 1u << 9;   // data lives in the scratch buffers
constexpr uint32_t META_IOTA = 1u << 10; // index payload not materialized yet

constexpr uint32_t STATUS_WAIT_TIMEOUT = 1u;
constexpr uint32_t STATUS_BAD_OFFSETS = 2u;

constexpr int MAX_LEVELS = 66;

// A live, finishing or retired segment: keys [start, start+len) of one of
// the two buffers.  tile0 is its first tile id within its level.
struct Seg {
  uint64_t start;
  uint64_t len;
  uint32_t meta;
  uint32_t tile0;
  uint64_t pad_;
};
static_assert(sizeof(Seg) == 32, "Seg layout");

// Per live segment: AND/OR of the keys that went to the front (lo) and back
// (hi) child, and the split (number of front keys), written by the level.
struct Acc {
  uint64_t and_lo, or_lo, and_hi, or_hi;
  uint64_t split;
};

// Work-list counters, zeroed at the start of every call.
struct Header {
  uint64_t packed[MAX_LEVELS]; // per level: (live segments << 32) | tiles
  uint32_t grab[MAX_LEVELS];   // per level: next tile id handed out
  uint32_t n_finish;
  uint32_t n_copy;
  uint32_t status;
  uint32_t pad_;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_add_u32(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t atomic_add_u64(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_and_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
__device__ __forceinline__ uint64_t wave_and_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v &= __shfl_xor(v, d);
  return v;
}
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d);
  return v;
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(v, d);
    if (lane >= d) v += y;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(v, d);
    if (lane >= d) v += y;
  }
  return v;
}

// Which side a key goes to (Algorithm 1's test, with the direction rules of
// Algorithms 3-5): 1 = back part.  Ascending puts the 0-side first; the sign
// pass of signed and float keys runs in the inverse direction; the lower
// bits of negative floats run in the inverse direction too.  `f` is the
// segment's flip: back = bit XOR f.
__device__ __forceinline__ int flip_of(int bit, int w, int mode, int desc, int negative) {
  const int top = (bit == w - 1);
  return desc ^ (top ? (mode != MODE_U) : (mode == MODE_F && negative));
}

// Look-back status words: epoch (level + 1) | status | 48-bit value.
constexpr uint64_t LB_AGG = 1, LB_INCL = 2;
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t st, uint64_t v) {
  return ((uint64_t)epoch << 50) | (st << 48) | (v & ((1ull << 48) - 1));
}
__device__ __forceinline__ uint64_t lb_status(uint64_t w, uint32_t epoch) {
  return ((w >> 50) == epoch) ? ((w >> 48) & 3) : 0;
}

// Decoupled look-back within one segment (run by one whole wave): publishes
// this tile's front count, then sums the counts of the segment's earlier
// tiles until one with a published inclusive prefix.  Returns the number of
// front keys in the segment's tiles before tile t.  Tiles are handed out in
// increasing order, so every tile waited on is held by a running
// workgroup; the wait is bounded all the same, and a timeout is recorded in
// the status word instead of hanging.
__device__ uint64_t look_back(uint64_t *flags, uint32_t t, uint32_t tile0, uint32_t count,
                              uint32_t epoch, uint32_t *status) {
  const int lane = threadIdx.x & 63;
  if (lane == 0) st_relaxed(&flags[t], lb_pack(epoch, t == tile0 ? LB_INCL : LB_AGG, count));
  if (t == tile0) return 0;
  uint64_t acc = 0;
  int64_t look = (int64_t)t - 1;
  for (;;) {
    const int64_t pred = look - lane;
    const bool in = pred >= (int64_t)tile0;
    uint64_t word = 0, st = 0;
    uint32_t spins = 0;
    for (;;) {
      if (in) {
        word = ld_relaxed(&flags[pred]);
        st = lb_status(word, epoch);
      }
      if (__all(!in || st != 0)) break;
      if (++spins > (1u << 20) ||
          (spins > 64 && (__hip_atomic_load(status, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT) & STATUS_WAIT_TIMEOUT))) {
        if (lane == 0) atomic_or_u32(status, STATUS_WAIT_TIMEOUT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    const uint64_t incl = __ballot(in && st == LB_INCL);
    uint64_t val = (in && st != 0) ? (word & ((1ull << 48) - 1)) : 0;
    if (incl) {
      const int stop = __ffsll((unsigned long long)incl) - 1;
      if (lane > stop) val = 0;
      acc += wave_sum_u64(val);
      break;
    }
    acc += wave_sum_u64(val);
    look -= 64;
    if (look < (int64_t)tile0) break;  // only reachable after a timeout
  }
  if (lane == 0) st_relaxed(&flags[t], lb_pack(epoch, LB_INCL, acc + count));
  return acc;
}

// ------------------------------------------------------------------- init

__global__ void init_kernel(Header *hdr, uint64_t *flags, uint64_t nflags) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t *h = reinterpret_cast<uint32_t *>(hdr);
  for (uint64_t i = i0; i < sizeof(Header) / 4; i += stride) h[i] = 0;
  for (uint64_t i = i0; i < nflags; i += stride) flags[i] = 0;
}

// offsets[0] = 0, non-decreasing, offsets[B] = n; otherwise flag it.
__global__ void validate_kernel(const int64_t *offsets, uint64_t B, uint64_t n, Header *hdr) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s <= B; s += stride) {
    const int64_t v = offsets[s];
    bool bad = v < 0 || (uint64_t)v > n;
    if (s == 0) bad |= v != 0;
    if (s == B) bad |= (uint64_t)v != n;
    if (s < B) bad |= offsets[s + 1] < v;
    if (bad) atomic_or_u32(&hdr->status, STATUS_BAD_OFFSETS);
  }
}

// ------------------------------------------------------- work-list building

constexpr int KIND_NONE = 0, KIND_LIVE = 1, KIND_FINISH = 2, KIND_COPY = 3;

struct ListArgs {
  Header *hdr;
  Seg *live_next;       // level (lvl+1) live list
  Acc *acc_next;
  uint32_t *tile_map_next;
  Seg *fin;
  Seg *cpy;
  int next_level;
  uint32_t tile;        // keys per level tile
  uint32_t t_fin;       // finish threshold (keys)
};

struct Child {
  uint64_t start, len;
  uint32_t meta;
  uint32_t tiles;
  int kind;
};

// Allocates slots for the children of one wave (two per lane) with one
// atomic per list, writes the descriptors and the tile -> segment map.
__device__ void emit_children(const ListArgs &a, Child (&ch)[2]) {
  const int lane = threadIdx.x & 63;
  // live: slots and tiles packed in one 64-bit counter so that slot order
  // and tile order agree
  uint64_t mine = 0;
  uint32_t nfin = 0, ncpy = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (ch[c].kind == KIND_LIVE) mine += (1ull << 32) | ch[c].tiles;
    nfin += ch[c].kind == KIND_FINISH;
    ncpy += ch[c].kind == KIND_COPY;
  }
  const uint64_t inc_live = wave_incl_scan_u64(mine);
  const uint32_t inc_fin = wave_incl_scan_u32(nfin);
  const uint32_t inc_cpy = wave_incl_scan_u32(ncpy);
  const uint64_t tot_live = __shfl(inc_live, 63);
  const uint32_t tot_fin = __shfl(inc_fin, 63);
  const uint32_t tot_cpy = __shfl(inc_cpy, 63);
  uint64_t b_live = 0;
  uint32_t b_fin = 0, b_cpy = 0;
  if (lane == 0) {
    if (tot_live) b_live = atomic_add_u64(&a.hdr->packed[a.next_level], tot_live);
    if (tot_fin) b_fin = atomic_add_u32(&a.hdr->n_finish, tot_fin);
    if (tot_cpy) b_cpy = atomic_add_u32(&a.hdr->n_copy, tot_cpy);
  }
  b_live = __shfl(b_live, 0);
  b_fin = __shfl(b_fin, 0);
  b_cpy = __shfl(b_cpy, 0);
  uint64_t pos = b_live + (inc_live - mine);
  uint32_t fpos = b_fin + (inc_fin - nfin);
  uint32_t cpos = b_cpy + (inc_cpy - ncpy);
  uint32_t slot[2] = {0, 0}, tile0[2] = {0, 0};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    Seg s;
    s.start = ch[c].start;
    s.len = ch[c].len;
    s.meta = ch[c].meta;
    s.tile0 = 0;
    s.pad_ = 0;
    if (ch[c].kind == KIND_LIVE) {
      slot[c] = (uint32_t)(pos >> 32);
      tile0[c] = (uint32_t)pos;
      s.tile0 = tile0[c];
      a.live_next[slot[c]] = s;
      Acc z;
      z.and_lo = ~0ull; z.or_lo = 0; z.and_hi = ~0ull; z.or_hi = 0; z.split = 0;
      a.acc_next[slot[c]] = z;
      pos += (1ull << 32) | ch[c].tiles;
    } else if (ch[c].kind == KIND_FINISH) {
      a.fin[fpos++] = s;
    } else if (ch[c].kind == KIND_COPY) {
      a.cpy[cpos++] = s;
    }
  }
  // tile -> segment map, written cooperatively by the wave
  if (__ballot(ch[0].kind == KIND_LIVE || ch[1].kind == KIND_LIVE) == 0) return;
  for (int src = 0; src < 64; ++src) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t nt = __shfl(ch[c].kind == KIND_LIVE ? ch[c].tiles : 0u, src);
      if (nt == 0) continue;
      const uint32_t t0 = __shfl(tile0[c], src);
      const uint32_t sl = __shfl(slot[c], src);
      for (uint32_t k = lane; k < nt; k += 64) a.tile_map_next[t0 + k] = sl;
    }
  }
}

// Level 0: every user segment becomes a live segment (split on the top bit,
// the first pass of Algorithms 2, 3 and 4), or goes straight to the finish
// list when it is small.
struct SeedArgs {
  ListArgs l;
  const int64_t *offsets; // nullable: one segment [0, n)
  uint64_t B, n;
  int w;
  int with_idx;
  int no_finish;
};

__global__ void seed_kernel(SeedArgs a) {
  if (a.l.hdr->status & STATUS_BAD_OFFSETS) return;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t base0 = (uint64_t)blockIdx.x * blockDim.x;
  for (uint64_t base = base0; base < a.B; base += stride) {
    const uint64_t s = base + threadIdx.x;
    Child ch[2];
    ch[0].kind = ch[1].kind = KIND_NONE;
    ch[0].tiles = ch[1].tiles = 0;
    if (s < a.B) {
      uint64_t st = 0, en = a.n;
      if (a.offsets) {
        int64_t o0 = a.offsets[s], o1 = a.offsets[s + 1];
        o0 = o0 < 0 ? 0 : o0;
        o1 = o1 < o0 ? o0 : o1;
        st = (uint64_t)o0 > a.n ? a.n : (uint64_t)o0;
        en = (uint64_t)o1 > a.n ? a.n : (uint64_t)o1;
      }
      const uint64_t len = en - st;
      ch[0].start = st;
      ch[0].len = len;
      ch[0].meta = META_IOTA | (uint32_t)(a.w - 1);
      if (len == 1) {
        if (a.with_idx) { ch[0].kind = KIND_FINISH; ch[0].meta = META_IOTA | BIT_NONE; }
      } else if (len >= 2) {
        if (!a.no_finish && len <= a.l.t_fin) {
          ch[0].kind = KIND_FINISH;
        } else {
          ch[0].kind = KIND_LIVE;
          ch[0].tiles = (uint32_t)((len + a.l.tile - 1) / a.l.tile);
        }
      }
    }
    emit_children(a.l, ch);
  }
}

// After level `level`: turn each parent's two children into next-level
// segments, finish entries, copy entries or nothing (already in place).
struct PlanArgs {
  ListArgs l;
  const Seg *live;
  const Acc *acc;
  int level;
  int w;
  int with_idx;
  int idx64;
  int no_skip;
  int no_finish;
};

__global__ void plan_kernel(PlanArgs a) {
  const uint32_t S = (uint32_t)(a.l.hdr->packed[a.level] >> 32);
  const uint32_t buf_out = (uint32_t)((a.level + 1) & 1) ? META_BUF : 0u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < S; base += stride) {
    const uint64_t q = base + threadIdx.x;
    Child ch[2];
    ch[0].kind = ch[1].kind = KIND_NONE;
    ch[0].tiles = ch[1].tiles = 0;
    if (q < S) {
      const Seg p = a.live[q];
      const Acc ac = a.acc[q];
      const int bit = (int)(p.meta & BIT_MASK);
      const uint64_t F = ac.split;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint64_t len = c ? p.len - F : F;
        const uint64_t andv = c ? ac.and_hi : ac.and_lo;
        const uint64_t orv = c ? ac.or_hi : ac.or_lo;
        const uint32_t rev = c ? META_REV : 0u;
        ch[c].start = c ? p.start + F : p.start;
        ch[c].len = len;
        if (len == 0) continue;
        int nb = -1;
        if (len >= 2 && bit > 0) {
          if (a.no_skip) {
            nb = bit - 1;
          } else {
            const uint64_t d = (andv ^ orv) & ((1ull << bit) - 1);
            if (d) nb = 63 - __clzll((long long)d);
          }
        }
        const uint32_t sign = ((andv >> (a.w - 1)) & 1) ? META_SIGN : 0u;
        const uint32_t meta = rev | sign | buf_out;
        if (nb < 0) {
          // retired: every key of the child is the same pattern
          const bool need = buf_out || (a.with_idx && (rev || a.idx64));
          if (need) {
            ch[c].meta = meta | BIT_NONE;
            ch[c].kind = len <= a.l.t_fin ? KIND_FINISH : KIND_COPY;
          }
        } else if (!a.no_finish && len <= a.l.t_fin) {
          ch[c].meta = meta | (uint32_t)nb;
          ch[c].kind = KIND_FINISH;
        } else {
          ch[c].meta = meta | (uint32_t)nb;
          ch[c].kind = KIND_LIVE;
          ch[c].tiles = (uint32_t)((len + a.l.tile - 1) / a.l.tile);
        }
      }
    }
    emit_children(a.l, ch);
  }
}

// ------------------------------------------------------------ global level

template <typename KT>
struct LevelArgs {
  const KT *keys_in;
  KT *keys_out;
  const uint32_t *idx_in;
  uint32_t *idx_out;
  const Seg *segs;
  Acc *acc;
  const uint32_t *tile_map;
  uint64_t *lookback;
  Header *hdr;
  int w, mode, desc, level;
};

template <typename KT, bool IDX, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void level_kernel(LevelArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr int TILE = BLOCK * IPT;
  constexpr int NCNT = IPT * WAVES;
  constexpr int CPL = (NCNT + 63) / 64;
  __shared__ KT s_key[TILE];
  __shared__ uint32_t s_idx[IDX ? TILE : 1];
  __shared__ uint32_t s_cnt[NCNT];
  __shared__ uint64_t s_red[4][WAVES];
  __shared__ Seg s_seg;
  __shared__ uint32_t s_tile, s_slot, s_c1;
  __shared__ uint64_t s_prefix;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t ntiles = (uint32_t)(a.hdr->packed[a.level] & 0xffffffffu);
  const uint32_t epoch = (uint32_t)a.level + 1;

  for (;;) {
    if (tid == 0) {
      const uint32_t t = atomic_add_u32(&a.hdr->grab[a.level], 1u);
      s_tile = t;
      if (t < ntiles) {
        const uint32_t slot = a.tile_map[t];
        s_slot = slot;
        s_seg = a.segs[slot];
      }
    }
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= ntiles) break;
    const uint32_t slot = s_slot;
    const uint64_t start = s_seg.start, len = s_seg.len;
    const uint32_t meta = s_seg.meta, tile0 = s_seg.tile0;
    const int bit = (int)(meta & BIT_MASK);
    const bool rev = (meta & META_REV) != 0;
    const bool iota = (meta & META_IOTA) != 0;
    const int f = flip_of(bit, a.w, a.mode, a.desc, (meta & META_SIGN) ? 1 : 0);
    const uint32_t j = t - tile0;
    const uint64_t lo = (uint64_t)j * TILE;
    const uint32_t cnt = (uint32_t)((len - lo) < (uint64_t)TILE ? (len - lo) : (uint64_t)TILE);
    const uint64_t end = start + len;

    // load the tile in logical order (right to left for a reversed segment)
    KT key[IPT];
    uint32_t ix[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t q = (uint32_t)(i * BLOCK + tid);
      const uint64_t pos = lo + q;
      key[i] = 0;
      ix[i] = 0;
      if (q < cnt) {
        const uint64_t addr = rev ? (end - 1 - pos) : (start + pos);
        key[i] = a.keys_in[addr];
        if (IDX) ix[i] = iota ? (uint32_t)pos : a.idx_in[addr];
      }
    }
    // front/back test, per-(item, wave) front counts, child AND/OR
    uint64_t fm[IPT];
    uint64_t and_lo = ~0ull, or_lo = 0, and_hi = ~0ull, or_hi = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t q = (uint32_t)(i * BLOCK + tid);
      const bool valid = q < cnt;
      const uint64_t k = (uint64_t)key[i];
      const bool back = valid && ((((k >> bit) & 1ull) ^ (uint64_t)f) != 0);
      const bool front = valid && !back;
      fm[i] = __ballot(front);
      if (lane == 0) s_cnt[i * WAVES + wave] = (uint32_t)__popcll(fm[i]);
      if (front) { and_lo &= k; or_lo |= k; }
      if (back) { and_hi &= k; or_hi |= k; }
    }
    and_lo = wave_and_u64(and_lo);
    or_lo = wave_or_u64(or_lo);
    and_hi = wave_and_u64(and_hi);
    or_hi = wave_or_u64(or_hi);
    if (lane == 0) {
      s_red[0][wave] = and_lo;
      s_red[1][wave] = or_lo;
      s_red[2][wave] = and_hi;
      s_red[3][wave] = or_hi;
    }
    __syncthreads();

    if (wave == 0) {
      // exclusive scan of the (item, wave) front counts; position order is
      // item-major, then wave, then lane
      uint32_t v[CPL];
      uint32_t sum = 0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int e = lane * CPL + c;
        v[c] = e < NCNT ? s_cnt[e] : 0u;
        sum += v[c];
      }
      const uint32_t incl = wave_incl_scan_u32(sum);
      uint32_t ex = incl - sum;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int e = lane * CPL + c;
        if (e < NCNT) s_cnt[e] = ex;
        ex += v[c];
      }
      const uint32_t c1 = __shfl(incl, 63);
      const uint64_t P1 = look_back(a.lookback, t, tile0, c1, epoch, &a.hdr->status);
      if (lane == 0) {
        s_prefix = P1;
        s_c1 = c1;
        uint64_t al = ~0ull, ol = 0, ah = ~0ull, oh = 0;
#pragma unroll
        for (int w2 = 0; w2 < WAVES; ++w2) {
          al &= s_red[0][w2];
          ol |= s_red[1][w2];
          ah &= s_red[2][w2];
          oh |= s_red[3][w2];
        }
        Acc *ac = &a.acc[slot];
        if (c1 > 0) {
          atomic_and_u64(&ac->and_lo, al);
          atomic_or_u64(&ac->or_lo, ol);
        }
        if (cnt > c1) {
          atomic_and_u64(&ac->and_hi, ah);
          atomic_or_u64(&ac->or_hi, oh);
        }
        if (lo + cnt == len) ac->split = P1 + c1;
      }
    }
    __syncthreads();

    // stage the tile as [front run | back run reversed] in LDS
    const uint64_t P1 = s_prefix;
    const uint32_t c1 = s_c1;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t q = (uint32_t)(i * BLOCK + tid);
      if (q < cnt) {
        const uint32_t r1 = s_cnt[i * WAVES + wave] + lanes_below(fm[i]);
        const bool front = (fm[i] >> lane) & 1ull;
        const uint32_t x = front ? r1 : (cnt - 1 - (q - r1));
        s_key[x] = key[i];
        if (IDX) s_idx[x] = ix[i];
      }
    }
    __syncthreads();

    // two contiguous runs: front keys at start + P1 + x, back keys counted
    // from the segment's right end (P2 back keys precede this tile)
    const uint64_t P2 = lo - P1;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t x = (uint32_t)(i * BLOCK + tid);
      if (x < cnt) {
        const uint64_t dst = (x < c1) ? (start + P1 + x) : (end - P2 - (cnt - x));
        a.keys_out[dst] = s_key[x];
        if (IDX) a.idx_out[dst] = s_idx[x];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- LDS finish

template <typename KT>
struct FinishArgs {
  const KT *keys_buf[2];
  const uint32_t *idx_buf[2];
  KT *keys_final;
  void *idx_final;
  const Seg *list;
  Header *hdr;
  int w, mode, desc, idx64, no_skip;
};

// One workgroup per segment of at most BLOCK*IPT keys: all remaining bits
// are split in LDS, MSB first, each split stable within every group of keys
// that share the bits above (the groups are tracked with head flags that
// travel with the keys).  Writes the final keys and indices to the caller's
// buffers.
template <typename KT, bool IDX, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void finish_kernel(FinishArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr int T = BLOCK * IPT;
  constexpr int NCH = IPT * WAVES;  // 64-key chunks
  constexpr int CPL = (NCH + 63) / 64;
  __shared__ KT s_key[T];
  __shared__ uint32_t s_idx[IDX ? T : 1];
  __shared__ uint8_t s_head[T];
  __shared__ uint32_t s_tot[T];
  __shared__ uint32_t s_ccnt[NCH];
  __shared__ int32_t s_chead[NCH];
  __shared__ uint8_t s_cfirst[NCH + 1];
  __shared__ uint64_t s_red[2][WAVES];
  __shared__ Seg s_seg;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nf = a.hdr->n_finish;
  const uint64_t lt = (1ull << lane) - 1;
  const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  if (tid == 0) s_cfirst[NCH] = 1;

  for (uint32_t e = blockIdx.x; e < nf; e += gridDim.x) {
    if (tid == 0) s_seg = a.list[e];
    __syncthreads();
    const uint64_t start = s_seg.start;
    const uint32_t len = (uint32_t)s_seg.len;
    const uint32_t meta = s_seg.meta;
    const int bit0 = (int)(meta & BIT_MASK);
    const bool rev = (meta & META_REV) != 0;
    const bool iota = (meta & META_IOTA) != 0;
    const int buf = (meta & META_BUF) ? 1 : 0;
    const KT *kin = a.keys_buf[buf];
    const uint32_t *iin = a.idx_buf[buf];

    KT key[IPT];
    uint32_t ix[IPT];
    bool head[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t p = (uint32_t)(i * BLOCK + tid);
      key[i] = 0;
      ix[i] = 0;
      head[i] = p == 0;
      if (p < len) {
        const uint64_t addr = rev ? (start + len - 1 - p) : (start + p);
        key[i] = kin[addr];
        if (IDX) ix[i] = iota ? p : iin[addr];
      }
    }

    if (bit0 != (int)BIT_NONE && len >= 2) {
      // bits on which the whole segment agrees are skipped
      uint64_t andv = ~0ull, orv = 0;
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        if ((uint32_t)(i * BLOCK + tid) < len) {
          andv &= (uint64_t)key[i];
          orv |= (uint64_t)key[i];
        }
      }
      andv = wave_and_u64(andv);
      orv = wave_or_u64(orv);
      if (lane == 0) {
        s_red[0][wave] = andv;
        s_red[1][wave] = orv;
      }
      __syncthreads();
      andv = ~0ull;
      orv = 0;
#pragma unroll
      for (int w2 = 0; w2 < WAVES; ++w2) {
        andv &= s_red[0][w2];
        orv |= s_red[1][w2];
      }
      const uint64_t below = (bit0 == 63) ? ~0ull : ((2ull << bit0) - 1);
      const uint64_t todo = a.no_skip ? below : ((andv ^ orv) & below);

      for (int b = bit0; b >= 0; --b) {
        if (!((todo >> b) & 1ull)) continue;
        uint64_t fm[IPT], hm[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          const bool valid = p < len;
          const uint64_t k = (uint64_t)key[i];
          const int fl = flip_of(b, a.w, a.mode, a.desc, (int)((k >> (a.w - 1)) & 1ull));
          const bool back = valid && ((((k >> b) & 1ull) ^ (uint64_t)fl) != 0);
          fm[i] = __ballot(valid && !back);
          hm[i] = __ballot(valid && head[i]);
          if (lane == 0) {
            const int c = i * WAVES + wave;
            if (hm[i]) {
              const int h = 63 - __clzll((long long)hm[i]);
              s_chead[c] = c * 64 + h;
              s_ccnt[c] = (uint32_t)__popcll(fm[i] >> h);
            } else {
              s_chead[c] = -1;
              s_ccnt[c] = (uint32_t)__popcll(fm[i]);
            }
            s_cfirst[c] = (uint8_t)(hm[i] & 1ull);
          }
        }
        __syncthreads();
        if (wave == 0) {
          // segmented exclusive scan of the chunk summaries: carry-in = the
          // last head before the chunk and the front keys counted since it
          int32_t hv[CPL];
          uint32_t cv[CPL];
          int32_t ah = -1;
          uint32_t ac = 0;
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const int e2 = lane * CPL + c;
            hv[c] = e2 < NCH ? s_chead[e2] : -1;
            cv[c] = e2 < NCH ? s_ccnt[e2] : 0u;
            if (hv[c] >= 0) { ah = hv[c]; ac = cv[c]; } else { ac += cv[c]; }
          }
          // inclusive scan of (ah, ac) with the segmented operator
#pragma unroll
          for (int d = 1; d < 64; d <<= 1) {
            const int32_t uh = __shfl_up(ah, d);
            const uint32_t uc = __shfl_up(ac, d);
            if (lane >= d && ah < 0) { ah = uh; ac += uc; }
          }
          int32_t xh = __shfl_up(ah, 1);
          uint32_t xc = __shfl_up(ac, 1);
          if (lane == 0) { xh = -1; xc = 0; }
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const int e2 = lane * CPL + c;
            if (e2 < NCH) {
              // reuse the chunk arrays for the exclusive carry-in
              s_chead[e2] = xh;
              s_ccnt[e2] = xc;
            }
            if (hv[c] >= 0) { xh = hv[c]; xc = cv[c]; } else { xc += cv[c]; }
          }
        }
        __syncthreads();
        uint32_t gs[IPT], r1[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          const int c = i * WAVES + wave;
          const uint64_t hle = hm[i] & le;
          if (hle) {
            const int h = 63 - __clzll((long long)hle);
            gs[i] = (uint32_t)(c * 64 + h);
            r1[i] = (uint32_t)__popcll(fm[i] & lt & ~((1ull << h) - 1));
          } else {
            gs[i] = (uint32_t)s_chead[c];
            r1[i] = s_ccnt[c] + (uint32_t)__popcll(fm[i] & lt);
          }
          const bool front = (fm[i] >> lane) & 1ull;
          if (p < len) {
            const bool nxt_head = (p + 1 == len) ||
                                  (lane < 63 ? ((hm[i] >> (lane + 1)) & 1ull) != 0
                                             : s_cfirst[c + 1] != 0);
            if (nxt_head) s_tot[gs[i]] = r1[i] + (front ? 1u : 0u);
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          if (p < len) {
            const bool front = (fm[i] >> lane) & 1ull;
            const uint32_t F = s_tot[gs[i]];
            const uint32_t r2 = (p - gs[i]) - r1[i];
            const uint32_t dst = front ? gs[i] + r1[i] : gs[i] + F + r2;
            s_key[dst] = key[i];
            if (IDX) s_idx[dst] = ix[i];
            s_head[dst] = (uint8_t)(front ? (r1[i] == 0) : (r2 == 0));
          }
        }
        __syncthreads();
        bool all_heads = true;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          if (p < len) {
            key[i] = s_key[p];
            if (IDX) ix[i] = s_idx[p];
            head[i] = s_head[p] != 0;
            all_heads &= head[i];
          }
        }
        // also the barrier that protects LDS before the next bit
        if (__syncthreads_and(all_heads)) break;
      }
    }

#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t p = (uint32_t)(i * BLOCK + tid);
      if (p < len) {
        a.keys_final[start + p] = key[i];
        if (IDX) {
          if (a.idx64) static_cast<int64_t *>(a.idx_final)[start + p] = (int64_t)ix[i];
          else static_cast<uint32_t *>(a.idx_final)[start + p] = ix[i];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- copy-back

template <typename KT>
struct CopyArgs {
  const KT *keys_buf[2];
  uint32_t *idx_buf[2];
  KT *keys_final;
  void *idx_final;
  const Seg *list;
  Header *hdr;
  int idx64;
};

// Retired segments larger than the finish threshold whose data is not yet
// final (in scratch, stored right to left, or needing 64-bit indices).  All
// keys of a retired segment are the same pattern, so keys are filled.
template <typename KT, bool IDX>
__global__ void copy_kernel(CopyArgs<KT> a) {
  const uint32_t nc = a.hdr->n_copy;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t e = 0; e < nc; ++e) {
    const Seg s = a.list[e];
    const bool rev = (s.meta & META_REV) != 0;
    const int buf = (s.meta & META_BUF) ? 1 : 0;
    if (buf) {
      const KT kv = a.keys_buf[1][s.start];
      for (uint64_t i = i0; i < s.len; i += stride) a.keys_final[s.start + i] = kv;
    }
    if (!IDX) continue;
    if (buf == 0 && rev && !a.idx64) {
      uint32_t *x = a.idx_buf[0] + s.start;
      for (uint64_t i = i0; i < s.len / 2; i += stride) {
        const uint32_t u = x[i], v = x[s.len - 1 - i];
        x[i] = v;
        x[s.len - 1 - i] = u;
      }
    } else {
      const uint32_t *src = a.idx_buf[buf] + s.start;
      for (uint64_t i = i0; i < s.len; i += stride) {
        const uint32_t v = src[rev ? (s.len - 1 - i) : i];
        if (a.idx64) static_cast<int64_t *>(a.idx_final)[s.start + i] = (int64_t)v;
        else static_cast<uint32_t *>(a.idx_final)[s.start + i] = v;
      }
    }
  }
}

// -------------------------------------------------------- backward scatter

// grad_in[r, idx[r, j]] = grad_sorted[r, j]; values are moved as raw bits.
template <typename ET, bool I64>
__global__ void backward_scatter_kernel(const ET *g, const void *idx, uint64_t rows,
                                        uint64_t cols, ET *out) {
  for (uint64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const uint64_t row = r * cols;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols;
         c += (uint64_t)gridDim.x * blockDim.x) {
      const uint64_t d = I64 ? (uint64_t) static_cast<const int64_t *>(idx)[row + c]
                             : (uint64_t) static_cast<const uint32_t *>(idx)[row + c];
      if (d < cols) out[row + d] = g[row + c];
    }
  }
}

}  // namespace bsort
