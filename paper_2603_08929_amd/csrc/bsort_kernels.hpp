// Device side of libbsort: HIP kernels for gfx950 (CDNA4, wave64).
//
// The method (bsort, arXiv 2603.08929, Section II, Algorithms 1-2, and
// Section III, Algorithms 3-5) splits every live part of the array on one
// bit, most significant first, into a front part and a back part, and
// recurses into both.  Here the recursion runs breadth first: one global
// "level" processes the current bit of every live segment at once.
//
// A level is ONE pass over the live keys: each wave takes a tile of one
// segment, ranks its keys front/back with ballots and lane masks, takes
// how many front keys precede the tile (and the segment's total) from
// per-tile counts made before the level -- by the previous level while it
// wrote the keys, or by the prep pass for segments whose bit was reached by
// skipping -- and a scan of them by the prep pass, and writes the front keys
// from the segment's start and the back keys after all its front keys.  The
// same pass folds the AND and OR of each child's keys into per-child
// accumulators, from which the next level picks the child's next bit (bits
// on which a child is constant are skipped: a split with an empty side is
// the identity) or retires it.  Segments of at most T keys finish all their
// remaining bits inside one workgroup, in LDS (the hybrid switch to a
// cache-resident routine that the paper proposes in Sections IV-B and V).
//
// Every load of a tile is issued on every path (empty ranges where there is
// nothing to read), so that the in-order counter of outstanding loads lets
// the current tile's work wait only for its own data.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include <cstddef>

namespace bsort {

enum : int { MODE_U = 0, MODE_I = 1, MODE_F = 2 };

// Segment descriptor meta bits.
constexpr uint32_t BIT_MASK = 0x7Fu;   // bit to split on next (0..63)
constexpr uint32_t BIT_NONE = 0x7Fu;   // no bit left: copy only
constexpr uint32_t META_SIGN = 1u << 8;  // float keys of this segment are negative
constexpr uint32_t META_BUF = 1u << 9;   // data lives in the scratch buffers
constexpr uint32_t META_IOTA = 1u << 10; // index payload not materialized yet
constexpr uint32_t META_PRE = 1u << 11;  // the previous level counted `bit` per tile (at cbase)

constexpr uint32_t STATUS_OVERSIZE = 1u;  // a finish entry larger than the workgroup's capacity
constexpr uint32_t STATUS_BAD_OFFSETS = 2u;
constexpr uint32_t STATUS_BAD_COUNTS = 4u;  // a tile's precomputed prefix exceeded its position
constexpr uint32_t STATUS_BARRIER = 8u;  // a grid barrier of the tail kernel timed out

constexpr int MAX_LEVELS = 66;

// A live, finishing or retired segment: keys [start, start+len) of one of
// the two buffers.  tile0 is its first tile id within its level.
struct Seg {
  uint64_t start;
  uint64_t len;
  uint32_t meta;
  uint32_t tile0;
  uint32_t cbase;  // front counts of this level's tiles: at cbase + j
  uint32_t slot;   // per-tile copies: the segment's slot in its level's list
};
static_assert(sizeof(Seg) == 32, "Seg layout");

// A segment of the tiny lists (2 to TINY_MAX keys, no tiles): the fields a
// tiny pass reads, in half the bytes of a Seg.
struct TinySeg {
  uint64_t start;
  uint32_t len;
  uint32_t meta;
};
static_assert(sizeof(TinySeg) == 16, "TinySeg layout");

// Per live segment: AND/OR of the keys that went to the front (lo) and back
// (hi) child, written by the level's tiles, and the split (number of front
// keys, one word per segment slot).  The AND/OR words are replicated (with a
// single copy every tile of a big segment would contend for the same line):
// a segment of nt tiles keeps R = acc_repl(len) replicas, tile j updating
// replica j mod R, and replica r lives at entry tile0 + ACC_STRIDE * r of the
// level's per-tile array.  Since ACC_STRIDE * (R - 1) < nt, segments never
// share entries, and the replicas of one segment sit on distinct 128-byte
// lines.  The array is sized by tiles, not by segments x ACC_REPL.
constexpr int ACC_REPL = 16;
constexpr uint32_t ACC_STRIDE = 4;
struct AccRep {
  uint64_t and_lo, or_lo, and_hi, or_hi;
};
static_assert(sizeof(AccRep) * ACC_STRIDE == 128, "AccRep layout");

// Work-list counters, zeroed at the start of every call.
struct Header {
  uint32_t status;             // kept first: read by bsort_device_status
  uint32_t n_finish;
  uint32_t n_copy;
  uint32_t n_finish_small;     // entries of the small-segment finish list
  uint32_t n_finish_tiny;      // ... and of the tiny-segment one
  uint32_t n_finish_med;       // ... and of the medium-segment one
  uint64_t finish_keys;        // keys handed to the LDS finish (all levels)
  uint64_t copy_keys;          // keys of retired segments copied back
  uint64_t packed[MAX_LEVELS]; // per level: (live segments << 32) | tiles
  uint32_t prep_ticket[MAX_LEVELS]; // per level: prep workgroups done
  uint64_t live_keys[MAX_LEVELS]; // per level: keys in live segments
  uint32_t bar_grp[8];         // tail-kernel grid barrier: arrivals per block group
  uint32_t bar_top;            // ... and groups complete
  uint64_t iota_keys[MAX_LEVELS];  // per level: live keys whose indices are still the identity
  uint64_t moved_keys[MAX_LEVELS]; // per level: keys of segments whose split moved them
  uint32_t n_tiny[MAX_LEVELS];     // per level: entries of the tiny-segment list (no-finish mode)
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed_u32(const uint32_t *p) {
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

// Values that are the same in every lane (read back from LDS, say) made
// provably uniform, so that addresses and buffer descriptors derived from
// them live in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
  return (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v) |
         ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32);
}

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Raw buffer access: a per-tile descriptor (base in SGPRs, byte range) and
// 32-bit lane offsets.  Loads past the range return 0 and stores past it
// are dropped by the hardware.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ uint8_t buf_load<uint8_t>(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ uint16_t buf_load<uint16_t>(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ uint32_t buf_load<uint32_t>(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ uint64_t buf_load<uint64_t>(rsrc_t r, uint32_t off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return (uint64_t)v[0] | ((uint64_t)v[1] << 32);
}
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, uint8_t v) {
  __builtin_amdgcn_raw_buffer_store_b8(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(rsrc_t r, uint32_t off, uint64_t v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  u32x2 w;
  w[0] = (uint32_t)v;
  w[1] = (uint32_t)(v >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 0);
}

// Wave-wide reductions and scans with DPP row shifts and row broadcasts
// (rows of 16 lanes, then rows 0-1 into 1 and 3, then 0-2 into 2-3), so the
// lane exchange stays in the VALU.  Lane 63 ends with the full result.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_src(uint32_t identity, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  v += dpp_src<0x111, 0xf>(0u, v);  // row_shr:1
  v += dpp_src<0x112, 0xf>(0u, v);  // row_shr:2
  v += dpp_src<0x114, 0xf>(0u, v);  // row_shr:4
  v += dpp_src<0x118, 0xf>(0u, v);  // row_shr:8
  v += dpp_src<0x142, 0xa>(0u, v);  // row_bcast:15
  v += dpp_src<0x143, 0xc>(0u, v);  // row_bcast:31
  return v;
}
__device__ __forceinline__ uint32_t wave_and_dpp32(uint32_t v) {
  v &= dpp_src<0x111, 0xf>(~0u, v);
  v &= dpp_src<0x112, 0xf>(~0u, v);
  v &= dpp_src<0x114, 0xf>(~0u, v);
  v &= dpp_src<0x118, 0xf>(~0u, v);
  v &= dpp_src<0x142, 0xa>(~0u, v);
  v &= dpp_src<0x143, 0xc>(~0u, v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_or_dpp32(uint32_t v) {
  v |= dpp_src<0x111, 0xf>(0u, v);
  v |= dpp_src<0x112, 0xf>(0u, v);
  v |= dpp_src<0x114, 0xf>(0u, v);
  v |= dpp_src<0x118, 0xf>(0u, v);
  v |= dpp_src<0x142, 0xa>(0u, v);
  v |= dpp_src<0x143, 0xc>(0u, v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint64_t wave_and_dpp(uint64_t v) {
  const uint32_t lo = wave_and_dpp32((uint32_t)v);
  const uint32_t hi = wave_and_dpp32((uint32_t)(v >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t wave_or_dpp(uint64_t v) {
  return (uint64_t)wave_or_dpp32((uint32_t)v) | ((uint64_t)wave_or_dpp32((uint32_t)(v >> 32)) << 32);
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

// Largest i in [0, n) with le(i), for a predicate that holds on a prefix of
// [0, n) and at 0: a 64-ary search by one whole wave (every lane probes one
// point per round), so a search over 2^14 entries takes three dependent
// loads instead of fourteen.  All 64 lanes must call it.
template <typename Le>
__device__ __forceinline__ uint32_t wave_search_le(uint32_t n, Le le) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const uint32_t step = (hi - lo + 64) / 64;
    const uint32_t idx = lo + lane * step;
    const uint64_t ok = __ballot(idx <= hi && le(idx));
    lo += ((uint32_t)__popcll(ok) - 1) * step;
    hi = lo + step - 1 < hi ? lo + step - 1 : hi;
  }
  return lo;
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

// ------------------------------------------------------------------- init

__global__ void init_kernel(Header *hdr, uint32_t *cnts, uint64_t ncnts) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t *h = reinterpret_cast<uint32_t *>(hdr);
  for (uint64_t i = i0; i < sizeof(Header) / 4; i += stride) h[i] = 0;
  for (uint64_t i = i0; i < ncnts; i += stride) cnts[i] = 0;
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

constexpr int KIND_NONE = 0, KIND_LIVE = 1, KIND_FINISH = 2, KIND_COPY = 3, KIND_TINY = 4;

// Without the LDS finish (every bit a global level), a segment of at most
// this many keys leaves the level tiles for the tiny-segment pass, which
// splits many such segments per wave instead of one per level tile.
constexpr uint32_t TINY_MAX = 256;

struct ListArgs {
  Header *hdr;
  Seg *live_next;       // level (lvl+1) live list, in tile order
  AccRep *acc_next;     // per-tile AND/OR replicas of level (lvl+1)
  uint64_t *split_next;  // per-slot split of level (lvl+1)
  Seg *fin;
  Seg *fin_small;       // finish entries of at most t_small keys
  Seg *fin_tiny;        // finish entries of at most t_tiny keys
  Seg *fin_med;         // finish entries of at most t_med keys
  Seg *cpy;
  int next_level;
  uint32_t tile;        // keys per level tile
  uint32_t t_fin;       // finish threshold (keys)
  uint32_t t_small;     // finish entries up to this size take the one-wave finish
  uint32_t t_tiny;      // ... and up to this size, one key per lane
  uint32_t t_med;       // ... and up to this size, half the full finish shape
  uint32_t recount;     // count base of segments whose counts the level did not make
  TinySeg *tiny_next;   // level (lvl+1) tiny-segment list (nullptr: none)
};

struct Child {
  uint64_t start, len;
  uint32_t meta;
  uint32_t tiles;
  uint32_t cbase;     // count base, or CBASE_OWN: not counted by the level, at recount + tile0
  int kind;
};
constexpr uint32_t CBASE_OWN = 0xFFFFFFFFu;

// Replicas of a segment's AND/OR words in use: many only for segments with
// many tiles (the ones whose tiles would contend).
__device__ __forceinline__ uint32_t acc_repl(uint64_t len, uint32_t tile) {
  const uint64_t nt = (len + tile - 1) / tile;
  return nt >= 256 ? (uint32_t)ACC_REPL : (nt >= 64 ? 4u : 1u);
}

// Allocates slots for the children of one wave (two per lane) with one
// atomic per list and writes their descriptors.
__device__ void emit_children(const ListArgs &a, Child (&ch)[2]) {
  const int lane = threadIdx.x & 63;
  // live: slots and tiles packed in one 64-bit counter so that slot order
  // and tile order agree
  uint64_t mine = 0, klive = 0, kiota = 0, kfin = 0, kcpy = 0;
  uint32_t nfin = 0, nfs = 0, nft = 0, nfm = 0, ncpy = 0, ntiny = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (ch[c].kind == KIND_LIVE) {
      mine += (1ull << 32) | ch[c].tiles;
      klive += ch[c].len;
      if (ch[c].meta & META_IOTA) kiota += ch[c].len;
    }
    if (ch[c].kind == KIND_FINISH) {
      if (ch[c].len <= a.t_tiny) nft++;
      else if (ch[c].len <= a.t_small) nfs++;
      else if (ch[c].len <= a.t_med) nfm++;
      else nfin++;
      kfin += ch[c].len;
    }
    if (ch[c].kind == KIND_COPY) { ncpy++; kcpy += ch[c].len; }
    if (ch[c].kind == KIND_TINY) {
      ntiny++;
      klive += ch[c].len;
      if (ch[c].meta & META_IOTA) kiota += ch[c].len;
    }
  }
  // statistics (keys per list), one atomic per wave and list
  klive = wave_sum_u64(klive);
  kiota = wave_sum_u64(kiota);
  kfin = wave_sum_u64(kfin);
  kcpy = wave_sum_u64(kcpy);
  if (lane == 0) {
    if (klive) atomic_add_u64(&a.hdr->live_keys[a.next_level], klive);
    if (kiota) atomic_add_u64(&a.hdr->iota_keys[a.next_level], kiota);
    if (kfin) atomic_add_u64(&a.hdr->finish_keys, kfin);
    if (kcpy) atomic_add_u64(&a.hdr->copy_keys, kcpy);
  }
  const uint64_t inc_live = wave_incl_scan_u64(mine);
  const uint32_t inc_fin = wave_incl_scan_u32(nfin);
  const uint32_t inc_fs = wave_incl_scan_u32(nfs);
  const uint32_t inc_ft = wave_incl_scan_u32(nft);
  const uint32_t inc_fm = wave_incl_scan_u32(nfm);
  const uint32_t inc_cpy = wave_incl_scan_u32(ncpy);
  const uint32_t inc_tiny = wave_incl_scan_u32(ntiny);
  const uint64_t tot_live = __shfl(inc_live, 63);
  const uint32_t tot_fin = __shfl(inc_fin, 63);
  const uint32_t tot_fs = __shfl(inc_fs, 63);
  const uint32_t tot_ft = __shfl(inc_ft, 63);
  const uint32_t tot_fm = __shfl(inc_fm, 63);
  const uint32_t tot_cpy = __shfl(inc_cpy, 63);
  const uint32_t tot_tiny = __shfl(inc_tiny, 63);
  uint64_t b_live = 0;
  uint32_t b_fin = 0, b_fs = 0, b_ft = 0, b_fm = 0, b_cpy = 0, b_tiny = 0;
  if (lane == 0) {
    if (tot_live) b_live = atomic_add_u64(&a.hdr->packed[a.next_level], tot_live);
    if (tot_fin) b_fin = atomic_add_u32(&a.hdr->n_finish, tot_fin);
    if (tot_fs) b_fs = atomic_add_u32(&a.hdr->n_finish_small, tot_fs);
    if (tot_ft) b_ft = atomic_add_u32(&a.hdr->n_finish_tiny, tot_ft);
    if (tot_fm) b_fm = atomic_add_u32(&a.hdr->n_finish_med, tot_fm);
    if (tot_cpy) b_cpy = atomic_add_u32(&a.hdr->n_copy, tot_cpy);
    if (tot_tiny) b_tiny = atomic_add_u32(&a.hdr->n_tiny[a.next_level], tot_tiny);
  }
  b_live = __shfl(b_live, 0);
  b_fin = __shfl(b_fin, 0);
  b_fs = __shfl(b_fs, 0);
  b_ft = __shfl(b_ft, 0);
  b_fm = __shfl(b_fm, 0);
  b_cpy = __shfl(b_cpy, 0);
  b_tiny = __shfl(b_tiny, 0);
  uint64_t pos = b_live + (inc_live - mine);
  uint32_t fpos = b_fin + (inc_fin - nfin);
  uint32_t fspos = b_fs + (inc_fs - nfs);
  uint32_t ftpos = b_ft + (inc_ft - nft);
  uint32_t fmpos = b_fm + (inc_fm - nfm);
  uint32_t cpos = b_cpy + (inc_cpy - ncpy);
  uint32_t tpos = b_tiny + (inc_tiny - ntiny);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    Seg s;
    s.start = ch[c].start;
    s.len = ch[c].len;
    s.meta = ch[c].meta;
    s.tile0 = 0;
    s.cbase = 0;
    s.slot = 0;
    if (ch[c].kind == KIND_LIVE) {
      const uint32_t slot = (uint32_t)(pos >> 32);
      s.tile0 = (uint32_t)pos;
      s.cbase = ch[c].cbase == CBASE_OWN ? a.recount + s.tile0 : ch[c].cbase;
      s.slot = slot;
      a.live_next[slot] = s;
      const uint32_t nr = acc_repl(ch[c].len, a.tile);
      for (uint32_t k = 0; k < nr; ++k) {
        AccRep *z = &a.acc_next[s.tile0 + ACC_STRIDE * k];
        z->and_lo = ~0ull;
        z->or_lo = 0;
        z->and_hi = ~0ull;
        z->or_hi = 0;
      }
      a.split_next[slot] = 0;
      pos += (1ull << 32) | ch[c].tiles;
    } else if (ch[c].kind == KIND_FINISH) {
      if (ch[c].len <= a.t_tiny) a.fin_tiny[ftpos++] = s;
      else if (ch[c].len <= a.t_small) a.fin_small[fspos++] = s;
      else if (ch[c].len <= a.t_med) a.fin_med[fmpos++] = s;
      else a.fin[fpos++] = s;
    } else if (ch[c].kind == KIND_COPY) {
      a.cpy[cpos++] = s;
    } else if (ch[c].kind == KIND_TINY) {
      a.tiny_next[tpos++] = TinySeg{s.start, (uint32_t)s.len, s.meta};
    }
  }
}

// Level 0: every user segment becomes a live segment (split on the top bit,
// the first pass of Algorithms 2, 3 and 4), or goes straight to the finish
// list when it is small.  Its front counts are not known yet, so the prep
// pass before the level counts its tiles.
struct SeedArgs {
  ListArgs l;
  const int64_t *offsets; // nullable: one segment [0, n)
  uint64_t B, n;
  int w;
  int with_idx;
  int no_finish;
  void *idx_final;  // the caller's indices (uint32, or int64 with idx64)
  int idx64;
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
    ch[0].cbase = ch[1].cbase = 0;
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
        // sorted as it stands: only its index (0) is written
        if (a.with_idx) {
          if (a.idx64) static_cast<int64_t *>(a.idx_final)[st] = 0;
          else static_cast<uint32_t *>(a.idx_final)[st] = 0;
        }
      } else if (len >= 2) {
        if (!a.no_finish && len <= a.l.t_fin) {
          ch[0].kind = KIND_FINISH;
        } else if (a.l.tiny_next && len <= TINY_MAX) {
          ch[0].kind = KIND_TINY;
        } else {
          ch[0].kind = KIND_LIVE;
          ch[0].tiles = (uint32_t)((len + a.l.tile - 1) / a.l.tile);
          ch[0].cbase = CBASE_OWN;
        }
      }
    }
    emit_children(a.l, ch);
  }
}

// After level `level`: turn each parent's two children into next-level
// segments, finish entries, copy entries or nothing (already in place).
// The level wrote the children into the other buffer, front child first;
// a split with an empty side moved nothing, so that child stays where its
// parent was (and keeps an index payload that is still the identity).
struct PlanArgs {
  ListArgs l;
  const Seg *live;
  const AccRep *acc;
  const uint64_t *split;
  uint32_t *zero_a;  // count arrays the next level accumulates into (zero_b nullable)
  uint32_t *zero_b;
  uint64_t zero_n;
  // 0: clear zero_n entries; k > 0: only the first k * (T + S) + 1, where T
  // and S are this level's tiles and segments (the next level's tiles are
  // at most T + S, and its counts land below 2 * its tiles)
  uint32_t zero_per_tile;
  int level;
  int w;
  int with_idx;
  int idx64;
  int no_skip;
  int no_finish;
  int inplace;  // the level partitioned in place: no buffers, no counts
};

__device__ __forceinline__ void plan_body(const PlanArgs &a) {
  const uint64_t packed = ld_relaxed(&a.l.hdr->packed[a.level]);
  const uint32_t S = (uint32_t)(packed >> 32);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t zn = a.zero_n;
  if (a.zero_per_tile) {
    const uint64_t need = (uint64_t)a.zero_per_tile * ((uint64_t)(uint32_t)packed + S) + 1;
    if (need < zn) zn = need;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < zn; i += stride) {
    a.zero_a[i] = 0;
    if (a.zero_b) a.zero_b[i] = 0;
  }
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < S; base += stride) {
    const uint64_t q = base + threadIdx.x;
    Child ch[2];
    ch[0].kind = ch[1].kind = KIND_NONE;
    ch[0].tiles = ch[1].tiles = 0;
    ch[0].cbase = ch[1].cbase = 0;
    uint64_t kmoved = 0;
    if (q < S) {
      const Seg p = a.live[q];
      uint64_t and_lo = ~0ull, or_lo = 0, and_hi = ~0ull, or_hi = 0;
      const uint32_t nr = acc_repl(p.len, a.l.tile);
      if (nr == 1) {
        const AccRep r0 = a.acc[p.tile0];
        and_lo = r0.and_lo;
        or_lo = r0.or_lo;
        and_hi = r0.and_hi;
        or_hi = r0.or_hi;
      } else {
        // all replicas in flight at once; indices past the last replica
        // read the last one again, which AND and OR absorb
        AccRep rep[ACC_REPL];
#pragma unroll
        for (uint32_t k = 0; k < (uint32_t)ACC_REPL; ++k)
          rep[k] = a.acc[p.tile0 + ACC_STRIDE * (k < nr ? k : nr - 1)];
#pragma unroll
        for (uint32_t k = 0; k < (uint32_t)ACC_REPL; ++k) {
          and_lo &= rep[k].and_lo;
          or_lo |= rep[k].or_lo;
          and_hi &= rep[k].and_hi;
          or_hi |= rep[k].or_hi;
        }
      }
      const int bit = (int)(p.meta & BIT_MASK);
      const uint64_t F = a.split[q];
      const uint32_t nt_p = (uint32_t)((p.len + a.l.tile - 1) / a.l.tile);
      // where the children's keys are: moved to the other buffer, or left
      // in place by a split with an empty side
      const bool moved = !a.inplace && F != 0 && F != p.len;
      kmoved = moved ? p.len : 0ull;
      const uint32_t cbuf = moved ? ((p.meta & META_BUF) ^ META_BUF) : (p.meta & META_BUF);
      const uint32_t ciota = (moved || a.inplace) ? 0u : (p.meta & META_IOTA);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint64_t len = c ? p.len - F : F;
        const uint64_t andv = c ? and_hi : and_lo;
        const uint64_t orv = c ? or_hi : or_lo;
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
        const uint32_t meta = sign | cbuf | ciota;
        if (nb < 0) {
          // retired: every key of the child is the same pattern; it still
          // has to reach the caller's buffers if it sits in scratch or its
          // indices are not written there yet
          const bool need = cbuf || (a.with_idx && (ciota || a.idx64));
          if (need) {
            ch[c].meta = meta | BIT_NONE;
            ch[c].kind = len <= a.l.t_fin ? KIND_FINISH : KIND_COPY;
          }
        } else if (!a.no_finish && len <= a.l.t_fin) {
          ch[c].meta = meta | (uint32_t)nb;
          ch[c].kind = KIND_FINISH;
        } else if (a.l.tiny_next && len <= TINY_MAX) {
          ch[c].meta = meta | (uint32_t)nb;
          ch[c].kind = KIND_TINY;
        } else {
          // the level counted this child's front keys on bit - 1 per tile;
          // a child that skipped to a lower bit is counted by the prep pass
          const bool pre = nb == bit - 1 && !a.inplace;
          ch[c].meta = meta | (pre ? META_PRE : 0u) | (uint32_t)nb;
          ch[c].kind = KIND_LIVE;
          ch[c].tiles = (uint32_t)((len + a.l.tile - 1) / a.l.tile);
          ch[c].cbase = pre ? 2 * p.tile0 + (uint32_t)c * nt_p : CBASE_OWN;
        }
      }
    }
    kmoved = wave_sum_u64(kmoved);
    if ((threadIdx.x & 63) == 0 && kmoved) atomic_add_u64(&a.l.hdr->moved_keys[a.level], kmoved);
    emit_children(a.l, ch);
  }
}

__global__ void plan_kernel(PlanArgs a) { plan_body(a); }


// ------------------------------------------------------------ global level
//
// One level splits every live segment on its bit.  A level tile is one
// wave's work: TILE = 64 * IPT consecutive keys of one segment, tile key q
// at lane q % 64 of item q / 64, so that every load reads 64 consecutive
// keys.  What a tile needs from other tiles is made before the level by the
// prep pass: its segment's descriptor, the number of front keys in the tile
// and in the segment before it, and the segment's total F.  So no tile
// waits for another and a wave works alone: no block barrier, no LDS.
//
// A front key of front rank r (counted in input order over the segment)
// lands at start + r, a back key of back rank r at start + F + r: both
// children keep input order, as the stable partitions of Figs. 1-2 do.  A
// split with an empty side (F = 0 or F = len) is the identity (Algorithm 1
// with k = ps or k = pe): its tiles write nothing and the child stays in
// the parent's buffer.
//
// While it places the keys, a tile also counts, for each child tile of the
// next level, the keys that go front on bit - 1 (the usual next bit), and
// folds the AND and OR of each child's keys into the segment's replicated
// words, from which the plan picks each child's next bit.

constexpr int PREP_TILES = 256;  // level tiles per prep workgroup: a chunk

// The per-tile prefix words a level tile reads with per-lane buffer loads:
// one descriptor covers both arrays (byte offsets from the first).
struct LevelMeta {
  uint32_t pc;     // uint2 per tile: (front keys of its segment before it in its chunk, its front keys)
  uint32_t carry;  // uint64 per chunk: front keys of the segment open at its start, before it
  uint32_t range;  // bytes the descriptor covers
};

template <typename KT>
struct PrepArgs {
  const KT *keys[2];       // key buffers 0 (the caller's) and 1 (scratch)
  const Seg *live;         // this level's live segments, in tile order
  Seg *tmap;               // out: per tile, its segment's descriptor
  uint2 *pc;               // out: see LevelMeta
  uint64_t *agg;           // per chunk: front keys after its last segment start (or all), bit 63 = has one
  uint64_t *carry;         // out: see LevelMeta
  const uint32_t *cnt_in;  // front keys per tile of counted segments, at cbase + j (previous level)
  Header *hdr;
  int w, mode, desc, level;
};

// Front keys of one level tile, counted by the whole wave from its keys:
// loads only; the caller reduces (so several tiles' loads are in flight).
template <typename KT, int IPT>
__device__ __forceinline__ void tile_keys(const KT *keys, uint64_t start, uint64_t len,
                                          uint64_t lo, KT (&k)[IPT], uint32_t &cnt) {
  constexpr uint32_t TILE = 64 * IPT;
  const int lane = threadIdx.x & 63;
  cnt = lo < len ? (uint32_t)(len - lo < TILE ? len - lo : TILE) : 0u;
  const rsrc_t kr = make_rsrc(keys + start + lo, cnt * (uint32_t)sizeof(KT));
#pragma unroll
  for (int i = 0; i < IPT; ++i) k[i] = buf_load<KT>(kr, (uint32_t)(i * 64 + lane) * (uint32_t)sizeof(KT));
}

// Before each level.  Workgroup b takes the chunk of level tiles
// [256 b, 256 b + 256), a wave 64 of them, a lane one:
//  - the tile's segment (one 64-ary wave search for the wave's first tile,
//    then the segments that start among its tiles) and descriptor;
//  - its front keys: made by the previous level for segments split on the
//    bit below their parent's, else counted here from the keys (level 0,
//    and segments that reached their bit by skipping);
//  - an exclusive scan of the counts over the chunk that restarts at every
//    segment start; and the chunk's sum after its last segment start.
// The last workgroup to finish (a ticket) turns the chunk sums into each
// chunk's carry, the front keys of the segment that is open at the chunk's
// start, before it.  A tile's front prefix is then its scan value plus,
// when its segment started in an earlier chunk, its chunk's carry.
template <typename KT, int IPT>
__device__ __forceinline__ void prep_body(const PrepArgs<KT> &a, uint32_t chunk) {
  constexpr uint32_t TILE = 64 * IPT;
  constexpr int RB = 4;  // tiles counted at once by a wave
  using RT = typename std::conditional<sizeof(KT) == 8, uint64_t, uint32_t>::type;
  __shared__ uint32_t s_tail[4], s_hh[4], s_last;
  __shared__ uint64_t s_v[256];
  __shared__ uint32_t s_f[256];
  // the chunk's tiles that have to be counted here, for the whole workgroup
  __shared__ uint64_t s_need[4];
  __shared__ uint64_t s_tst[PREP_TILES], s_tln[PREP_TILES];
  __shared__ uint32_t s_tmt[PREP_TILES], s_tj[PREP_TILES], s_list[PREP_TILES], s_cres[PREP_TILES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t pk = ld_relaxed(&a.hdr->packed[a.level]);
  const uint32_t S = (uint32_t)(pk >> 32), ntiles = (uint32_t)pk;
  const uint32_t nchunks = (ntiles + PREP_TILES - 1) / PREP_TILES;
  if (chunk >= nchunks) return;
  const bool spread = nchunks < 64;  // few workgroups: the chunk's waves share its counting
  const uint32_t t0 = chunk * PREP_TILES + (uint32_t)wave * 64;
  const uint32_t t = t0 + (uint32_t)lane;
  const bool valid = t < ntiles;
  uint32_t c = 0;
  bool head = false, need = false;
  if (t0 < ntiles) {
    const uint32_t s0 = wave_search_le(S, [&](uint32_t i) { return a.live[i].tile0 <= t0; });
    // bit d of M: a segment starts at tile t0 + d (d >= 1)
    const uint32_t sl = s0 + 1 + (uint32_t)lane;
    const uint32_t e = sl < S ? a.live[sl].tile0 : 0xffffffffu;
    const uint32_t d = e - t0;
    const uint64_t M = wave_or_dpp(d < 64u ? 1ull << d : 0ull);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const uint32_t s = s0 + (uint32_t)__popcll(M & upto);
    Seg sg = {};
    if (valid) {
      sg = a.live[s];
      a.tmap[t] = sg;
    }
    const uint32_t j = t - sg.tile0;
    head = valid && j == 0;
    const bool counted = (sg.meta & META_PRE) != 0;
    if (valid && counted) c = a.cnt_in[sg.cbase + j];
    need = valid && !counted;
    if (!spread) {
      // a wave counts its own tiles
      uint64_t todo = __ballot(need);
      while (todo) {
        uint32_t who[RB], cnt[RB];
        KT k[RB][IPT];
        int bit[RB];
        uint32_t f[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          who[u] = todo ? (uint32_t)(__ffsll((unsigned long long)todo) - 1) : 64u;
          todo &= todo ? todo - 1 : 0ull;
          const int wl = who[u] < 64u ? (int)who[u] : 0;
          const uint32_t mt = (uint32_t)__builtin_amdgcn_readlane((int)sg.meta, wl);
          const uint64_t st =
              (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sg.start, wl) |
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sg.start >> 32), wl)
               << 32);
          const uint64_t ln =
              who[u] < 64u
                  ? ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sg.len, wl) |
                     ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sg.len >> 32),
                                                                    wl)
                      << 32))
                  : 0ull;
          const uint32_t jj = (uint32_t)__builtin_amdgcn_readlane((int)j, wl);
          bit[u] = (int)(mt & BIT_MASK);
          f[u] = (uint32_t)flip_of(bit[u], a.w, a.mode, a.desc, (mt & META_SIGN) ? 1 : 0);
          tile_keys<KT, IPT>(a.keys[(mt & META_BUF) ? 1 : 0], st, ln, (uint64_t)jj * TILE, k[u],
                             cnt[u]);
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          uint32_t n = 0;
#pragma unroll
          for (int i = 0; i < IPT; ++i) {
            const bool fr = (uint32_t)(i * 64 + lane) < cnt[u] &&
                            ((((RT)k[u][i] >> bit[u]) & 1u) ^ f[u]) == 0;
            n += (uint32_t)__popcll(__ballot(fr));
          }
          if ((uint32_t)lane == who[u]) c = n;
        }
      }
    } else if (need) {
      s_tst[tid] = sg.start;
      s_tln[tid] = sg.len;
      s_tmt[tid] = sg.meta;
      s_tj[tid] = j;
    }
  }
  // Tiles whose counts the previous level did not make (level 0, segments
  // that reached their bit by skipping) are counted from their keys: by
  // their own wave when the level has many chunks, else by the whole
  // workgroup, RB tiles at a time per wave, so that a chunk whose tiles to
  // count sit in one wave does not wait on that wave alone.
  if (!spread) need = false;
  const uint64_t nm = spread ? __ballot(need) : 0ull;
  if (spread && lane == 0) s_need[wave] = nm;
  if (spread) __syncthreads();
  uint32_t total = 0, off = 0;
  if (spread) {
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) {
      const uint32_t k = (uint32_t)__popcll(s_need[w2]);
      if (w2 < wave) off += k;
      total += k;
    }
  }
  if (total) {
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (need) s_list[off + (uint32_t)__popcll(nm & below)] = (uint32_t)tid;
    __syncthreads();
    for (uint32_t base = (uint32_t)wave * RB; base < total; base += 4 * RB) {
      uint32_t who[RB], cnt[RB];
      KT k[RB][IPT];
      int bit[RB];
      uint32_t f[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const bool v = base + u < total;
        who[u] = v ? s_list[base + u] : 0u;
        const uint32_t mt = s_tmt[who[u]];
        bit[u] = (int)(mt & BIT_MASK);
        f[u] = (uint32_t)flip_of(bit[u], a.w, a.mode, a.desc, (mt & META_SIGN) ? 1 : 0);
        tile_keys<KT, IPT>(a.keys[(mt & META_BUF) ? 1 : 0], s_tst[who[u]], v ? s_tln[who[u]] : 0ull,
                           (uint64_t)s_tj[who[u]] * TILE, k[u], cnt[u]);
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        uint32_t n = 0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const bool fr = (uint32_t)(i * 64 + lane) < cnt[u] &&
                          ((((RT)k[u][i] >> bit[u]) & 1u) ^ f[u]) == 0;
          n += (uint32_t)__popcll(__ballot(fr));
        }
        if (lane == 0 && base + u < total) s_cres[who[u]] = n;
      }
    }
    __syncthreads();
    if (need) c = s_cres[tid];
  }
  // exclusive scan of c over the chunk, restarting at segment starts
  const uint32_t inc = wave_incl_scan_dpp(c);
  const uint32_t exc = inc - c;
  const uint64_t hm = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const uint64_t hb = hm & upto;
  const int hl = hb ? 63 - __clzll((long long)hb) : -1;  // last segment start at or before the lane
  uint32_t pre = exc - (hl >= 0 ? (uint32_t)__shfl((int)exc, hl) : 0u);
  const int hlast = hm ? 63 - __clzll((long long)hm) : -1;
  const uint32_t wtot = (uint32_t)__shfl((int)inc, 63);
  const uint32_t wtail = wtot - (hlast >= 0 ? (uint32_t)__shfl((int)exc, hlast) : 0u);
  if (lane == 0) {
    s_tail[wave] = wtail;
    s_hh[wave] = hm != 0;
  }
  __syncthreads();
  if (hl < 0) {
    // the segment started in an earlier wave (or chunk): add the earlier
    // waves' fronts back to its start
    uint32_t cw = 0;
    for (int w2 = wave - 1; w2 >= 0; --w2) {
      cw += s_tail[w2];
      if (s_hh[w2]) break;
    }
    pre += cw;
  }
  if (valid) a.pc[t] = make_uint2(pre, c);
  if (tid == 0) {
    uint64_t A = 0;
    bool hh = false;
    for (int w2 = 3; w2 >= 0 && !hh; --w2) {
      A += s_tail[w2];
      hh = s_hh[w2] != 0;
    }
    a.agg[chunk] = A | (hh ? 1ull << 63 : 0ull);
    __threadfence();
    s_last = atomic_add_u32(&a.hdr->prep_ticket[a.level], 1u) == nchunks - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // carry[0] = 0; carry[i + 1] = sum_i + (chunk i has a segment start ? 0 : carry[i]):
  // per thread a run of chunks, then a scan of the runs' (restart, sum) pairs
  constexpr uint64_t HEAD = 1ull << 63;
  const uint32_t per = (nchunks + 255) / 256;
  const uint32_t c0 = (uint32_t)tid * per, c1 = c0 + per < nchunks ? c0 + per : nchunks;
  uint64_t v = 0;
  uint32_t fl = 0;
  for (uint32_t i = c0; i < c1; ++i) {
    const uint64_t x = ld_relaxed(&a.agg[i]);
    if (x & HEAD) {
      fl = 1;
      v = x & ~HEAD;
    } else {
      v += x;
    }
  }
  s_v[tid] = v;
  s_f[tid] = fl;
  for (int dd = 1; dd < 256; dd <<= 1) {
    __syncthreads();
    const uint64_t pv = tid >= dd ? s_v[tid - dd] : 0ull;
    const uint32_t pf = tid >= dd ? s_f[tid - dd] : 0u;
    __syncthreads();
    if (!fl) {
      v += pv;
      fl = pf;
    }
    s_v[tid] = v;
    s_f[tid] = fl;
  }
  __syncthreads();
  uint64_t cin = tid ? s_v[tid - 1] : 0ull;
  for (uint32_t i = c0; i < c1; ++i) {
    a.carry[i] = cin;
    const uint64_t x = ld_relaxed(&a.agg[i]);
    cin = (x & HEAD) ? (x & ~HEAD) : cin + x;
  }
}

template <typename KT, int IPT>
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs<KT> a) {
  prep_body<KT, IPT>(a, blockIdx.x);
}

template <typename KT>
struct LevelArgs {
  KT *keys[2];             // key buffers 0 (the caller's) and 1 (scratch)
  uint32_t *idx[2];        // the index buffers paired with them
  const Seg *tmap;         // per tile: its segment's descriptor (from the prep pass)
  const char *meta;        // base of the prefix arrays of LevelMeta
  LevelMeta off;
  AccRep *acc;             // the replicas again, for the atomics
  uint64_t *split;         // per segment slot: its front keys F (for the plan)
  Header *hdr;
  uint32_t *cnt_out;       // next level: front keys on bit - 1 per child tile
  int w, mode, desc, level;
};

// A tile's registers, loaded one tile ahead of its use.
template <typename KT, int IPT>
struct WaveRegs {
  uint32_t mw;        // lanes 8-15: its prefix words (see issue_tile)
  KT key[IPT];
  uint32_t ix[IPT];
};

// Uniform description of a tile, from its descriptor dwords (lanes 0-7).
struct WaveTile {
  uint64_t start, len, lo;
  uint32_t meta, tile0, cbase, slot, t, j, cnt, nt;
  bool valid;
};

// A wave's AND/OR of the keys of its current segment's two children, per
// lane, carried across the wave's tiles while they belong to one segment
// and folded into one of the segment's replicas when the segment changes
// (once per wave and segment, not once per tile).
template <typename RT>
struct WaveAcc {
  uint32_t slot;  // segment slot, or ~0 for none
  uint32_t rep;   // replica entry the wave folds into
  RT and_lo, or_lo, and_hi, or_hi;
};

__device__ __forceinline__ uint32_t rl(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// The descriptor dword of tile t for lanes 0-7 (0 elsewhere or past the end).
__device__ __forceinline__ uint32_t load_desc(const Seg *tmap, uint32_t t, uint32_t ntiles) {
  const uint32_t lane = threadIdx.x & 63;
  const bool v = t < ntiles;
  const rsrc_t r = make_rsrc(tmap + (v ? t : 0u), v ? (uint32_t)sizeof(Seg) : 0u);
  return buf_load<uint32_t>(r, lane < 8u ? lane * 4u : ~0u);
}

template <int TILE>
__device__ __forceinline__ WaveTile wave_tile(uint32_t dsc, uint32_t t, uint32_t ntiles) {
  WaveTile w;
  w.t = t;
  w.valid = t < ntiles;
  w.start = (uint64_t)rl(dsc, 0) | ((uint64_t)rl(dsc, 1) << 32);
  w.len = (uint64_t)rl(dsc, 2) | ((uint64_t)rl(dsc, 3) << 32);
  w.meta = rl(dsc, 4);
  w.tile0 = rl(dsc, 5);
  w.cbase = rl(dsc, 6);
  w.slot = rl(dsc, 7);
  w.j = t - w.tile0;
  w.lo = (uint64_t)w.j * TILE;
  w.cnt = w.valid ? (uint32_t)(w.len - w.lo < (uint64_t)TILE ? w.len - w.lo : (uint64_t)TILE) : 0u;
  w.nt = (uint32_t)((w.len + TILE - 1) / TILE);
  return w;
}

// Every load of a tile is issued on every path -- a tile past the end, an
// index that is an iota, or a lane with nothing to fetch gets an empty range,
// whose reads return 0 without a memory access -- so that the number of
// loads in flight does not depend on the path and each use waits only for
// its own loads (the counter of outstanding loads retires in order).
// Lanes 8-15 fetch: 8-9 the tile's (prefix, count), 10-11 its chunk's carry,
// 12-13 the (prefix, count) of the segment's last tile, 14-15 that tile's
// chunk carry.
template <typename KT, bool IDX, int IPT>
__device__ __forceinline__ void issue_tile(const LevelArgs<KT> &a, rsrc_t mr, const WaveTile &w,
                                           WaveRegs<KT, IPT> &r) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t L = w.tile0 + w.nt - 1;
  // one selected offset per lane (selects, not branches)
  const uint32_t odd = (lane & 1u) * 4u;
  uint32_t o = ~0u;
  o = lane - 8u < 2u ? a.off.pc + w.t * 8u + odd : o;
  o = lane - 10u < 2u ? a.off.carry + (w.t / PREP_TILES) * 8u + odd : o;
  o = lane - 12u < 2u ? a.off.pc + L * 8u + odd : o;
  o = lane - 14u < 2u ? a.off.carry + (L / PREP_TILES) * 8u + odd : o;
  o = w.valid ? o : ~0u;
  r.mw = buf_load<uint32_t>(mr, o);
  const bool iota = (w.meta & META_IOTA) != 0;
  const int buf = (w.meta & META_BUF) ? 1 : 0;
  const uint64_t sbase = w.valid ? w.start + w.lo : 0u;
  const rsrc_t kr = make_rsrc(a.keys[buf] + sbase, w.cnt * (uint32_t)sizeof(KT));
  const rsrc_t ir = make_rsrc(IDX ? a.idx[buf] + sbase : nullptr, IDX && !iota ? w.cnt * 4u : 0u);
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t q = (uint32_t)(i * 64) + lane;  // past cnt: out of range, reads 0
    r.key[i] = buf_load<KT>(kr, q * (uint32_t)sizeof(KT));
    if (IDX) r.ix[i] = buf_load<uint32_t>(ir, q * 4u);  // an iota is added at use
  }
}

// Folds the wave's AND/OR words into its replica of the segment's children
// and starts over.
template <typename KT, typename RT>
__device__ __forceinline__ void flush_acc(const LevelArgs<KT> &a, WaveAcc<RT> &acc) {
  if (acc.slot != ~0u) {
    uint64_t al, ol, ah, oh;
    if (sizeof(RT) == 8) {
      al = wave_and_dpp((uint64_t)acc.and_lo);
      ol = wave_or_dpp((uint64_t)acc.or_lo);
      ah = wave_and_dpp((uint64_t)acc.and_hi);
      oh = wave_or_dpp((uint64_t)acc.or_hi);
    } else {
      al = (uint64_t)wave_and_dpp32((uint32_t)acc.and_lo) | (~0ull << 32);
      ol = (uint64_t)wave_or_dpp32((uint32_t)acc.or_lo);
      ah = (uint64_t)wave_and_dpp32((uint32_t)acc.and_hi) | (~0ull << 32);
      oh = (uint64_t)wave_or_dpp32((uint32_t)acc.or_hi);
    }
    if ((threadIdx.x & 63) == 0) {
      AccRep *ac = &a.acc[acc.rep];
      if (al != ~0ull) atomic_and_u64(&ac->and_lo, al);
      if (ol != 0) atomic_or_u64(&ac->or_lo, ol);
      if (ah != ~0ull) atomic_and_u64(&ac->and_hi, ah);
      if (oh != 0) atomic_or_u64(&ac->or_hi, oh);
    }
  }
  acc.and_lo = (RT)~(RT)0;
  acc.or_lo = 0;
  acc.and_hi = (RT)~(RT)0;
  acc.or_hi = 0;
}

// The per-key work of a tile: rank each key on its side, store it (and its
// index), fold it into its child's AND/OR words, and count the keys that go
// front on the next bit per child tile.  NEAR: byte offsets from the
// segment's start fit 32 bits (one descriptor per array); otherwise each of
// the tile's two runs, which are far apart, gets its own.
struct TileConsts {
  uint32_t pf, pb;      // offset of the tile's first front / back key from its descriptor
  uint32_t cnt, len32;  // keys in the tile; out-of-range offset for NEAR
  uint32_t xf, xb;      // ranks from which a key lies in its child's following tile
  uint32_t ibase;       // index of an iota input (position), or 0
  int bit, nbit;
  uint32_t f, fnf, fnb;
  bool iota;
};

template <bool NEAR, typename KT, bool IDX, int IPT, typename RT>
__device__ __forceinline__ void tile_keys_pass(const WaveRegs<KT, IPT> &r, const TileConsts &c,
                                               rsrc_t kwf, rsrc_t kwb, rsrc_t iwf, rsrc_t iwb,
                                               uint32_t &cf, RT &and_lo, RT &or_lo, RT &and_hi,
                                               RT &or_hi, uint32_t &nfr, uint32_t &nbk) {
  constexpr uint32_t TILE = 64 * IPT;
  const uint32_t lane = threadIdx.x & 63;
  // A key goes front when its bit equals the flip f: with bm the bit spread
  // over the word (0 or all ones), the front mask is bm XNOR (f ? ~0 : 0)
  // -- selects and masks, no branches
  const RT fx = c.f ? (RT)0 : (RT)~(RT)0;
  const uint32_t xs0 = c.xf, xs1 = c.xb;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t q = (uint32_t)(i * 64) + lane;
    const RT k = (RT)r.key[i];
    const RT vm = q < c.cnt ? (RT)~(RT)0 : (RT)0;
    const RT bm = (RT)0 - (RT)((k >> c.bit) & 1u);
    const RT mf = (bm ^ fx) & vm;   // front key
    const RT mb = ~(bm ^ fx) & vm;  // back key
    const bool front = mf != 0;
    const bool valid = vm != 0;
    const uint64_t fm = __ballot(front);
    const uint32_t r1 = cf + lanes_below(fm);
    const uint32_t r2 = q - r1;
    cf += (uint32_t)__popcll(fm);
    // a lane past the tile's end stores out of range (dropped); so does,
    // with two descriptors, the store of the other side
    const uint32_t iv = r.ix[i] + c.ibase + (c.iota ? (uint32_t)(i * 64) : 0u);
    if (NEAR) {
      const uint32_t dst = valid ? (front ? c.pf + r1 : c.pb + r2) : c.len32;
      buf_store(kwf, dst * (uint32_t)sizeof(KT), r.key[i]);
      if (IDX) buf_store(iwf, dst * 4u, iv);
    } else {
      const uint32_t of = front ? c.pf + r1 : TILE, ob = (valid && !front) ? c.pb + r2 : TILE;
      buf_store(kwf, of * (uint32_t)sizeof(KT), r.key[i]);
      buf_store(kwb, ob * (uint32_t)sizeof(KT), r.key[i]);
      if (IDX) {
        buf_store(iwf, of * 4u, iv);
        buf_store(iwb, ob * 4u, iv);
      }
    }
    and_lo &= k | ~mf;
    or_lo |= k & mf;
    and_hi &= k | ~mb;
    or_hi |= k & mb;
    // next-level counts per lane, two 16-bit fields a side: keys before and
    // after the child tile boundary
    const uint32_t nb = (uint32_t)(k >> c.nbit) & 1u;
    const bool nf = valid && nb == (front ? c.fnf : c.fnb);
    const uint32_t rk = front ? r1 : r2;
    const uint32_t inc = nf ? (rk >= (front ? xs0 : xs1) ? 0x10000u : 1u) : 0u;
    nfr += front ? inc : 0u;
    nbk += front ? 0u : inc;
  }
}

template <typename KT, bool IDX, int IPT, typename RT>
__device__ __forceinline__ void process_tile(const LevelArgs<KT> &a, const WaveTile &w,
                                             const WaveRegs<KT, IPT> &r, WaveAcc<RT> &acc,
                                             uint32_t wave_id) {
  constexpr uint32_t TILE = 64 * IPT;
  const uint32_t lane = threadIdx.x & 63;
  if (!w.valid) return;
  if (w.slot != acc.slot) {
    flush_acc<KT, RT>(a, acc);
    acc.slot = w.slot;
    acc.rep = w.tile0 + ACC_STRIDE * (wave_id & (acc_repl(w.len, TILE) - 1));
  }
  TileConsts c;
  c.bit = (int)(w.meta & BIT_MASK);
  c.f = (uint32_t)flip_of(c.bit, a.w, a.mode, a.desc, (w.meta & META_SIGN) ? 1 : 0);
  // the tile's front prefix P and the segment's front total F
  const uint32_t h = w.tile0 / PREP_TILES;
  const uint32_t L = w.tile0 + w.nt - 1;
  const uint32_t c_t = rl(r.mw, 9);
  const uint64_t car_t = (uint64_t)rl(r.mw, 10) | ((uint64_t)rl(r.mw, 11) << 32);
  const uint64_t car_L = (uint64_t)rl(r.mw, 14) | ((uint64_t)rl(r.mw, 15) << 32);
  const uint64_t P = (uint64_t)rl(r.mw, 8) + (w.t / PREP_TILES != h ? car_t : 0ull);
  const uint64_t F = (uint64_t)rl(r.mw, 12) + rl(r.mw, 13) + (L / PREP_TILES != h ? car_L : 0ull);
  const bool moved = F != 0 && F != w.len;
  c.iota = (w.meta & META_IOTA) != 0;
  const int out = (w.meta & META_BUF) ? 0 : 1;
  const uint64_t B0 = w.lo - P;  // back keys before the tile (with a sane prefix)
  c.ibase = c.iota ? (uint32_t)w.lo + lane : 0u;
  c.cnt = w.cnt;
  c.len32 = (uint32_t)w.len;
  // next level (bit - 1): a child's keys have the segment's sign, or their
  // side's when this level splits the sign bit
  c.nbit = c.bit > 0 ? c.bit - 1 : 0;
  uint32_t sgn_f = (w.meta & META_SIGN) ? 1u : 0u, sgn_b = sgn_f;
  if (c.bit == a.w - 1) {
    sgn_f = c.f;
    sgn_b = 1u - c.f;
  }
  c.fnf = (uint32_t)a.desc ^ (uint32_t)(a.mode == MODE_F && sgn_f);
  c.fnb = (uint32_t)a.desc ^ (uint32_t)(a.mode == MODE_F && sgn_b);
  c.xf = (uint32_t)((P / TILE + 1) * TILE - P);
  c.xb = (uint32_t)((B0 / TILE + 1) * TILE - B0);
  uint32_t nfr = 0, nbk = 0;
  uint32_t cf = 0;  // front keys so far in the tile
  RT and_lo = acc.and_lo, or_lo = acc.or_lo, and_hi = acc.and_hi, or_hi = acc.or_hi;
  // Descriptors are bounded to the segment, so that no store can leave it,
  // and empty when the split has an empty side.
  if (w.len * (sizeof(KT) > 4 ? sizeof(KT) : 4) < (1ull << 32)) {
    const uint32_t rg = moved ? (uint32_t)w.len : 0u;
    const rsrc_t kw = make_rsrc(a.keys[out] + w.start, rg * (uint32_t)sizeof(KT));
    const rsrc_t iw = make_rsrc(IDX ? a.idx[out] + w.start : nullptr, IDX ? rg * 4u : 0u);
    c.pf = (uint32_t)P;
    c.pb = (uint32_t)(F + B0);
    tile_keys_pass<true, KT, IDX, IPT, RT>(r, c, kw, kw, iw, iw, cf, and_lo, or_lo, and_hi, or_hi,
                                           nfr, nbk);
  } else {
    const uint64_t fo = P < w.len ? P : w.len, bo = F + B0 < w.len ? F + B0 : w.len;
    const uint32_t fr = moved ? (uint32_t)((w.len - fo) < TILE ? (w.len - fo) : TILE) : 0u;
    const uint32_t br = moved ? (uint32_t)((w.len - bo) < TILE ? (w.len - bo) : TILE) : 0u;
    const rsrc_t kwf = make_rsrc(a.keys[out] + w.start + fo, fr * (uint32_t)sizeof(KT));
    const rsrc_t kwb = make_rsrc(a.keys[out] + w.start + bo, br * (uint32_t)sizeof(KT));
    const rsrc_t iwf = make_rsrc(IDX ? a.idx[out] + w.start + fo : nullptr, IDX ? fr * 4u : 0u);
    const rsrc_t iwb = make_rsrc(IDX ? a.idx[out] + w.start + bo : nullptr, IDX ? br * 4u : 0u);
    c.pf = 0;
    c.pb = 0;
    tile_keys_pass<false, KT, IDX, IPT, RT>(r, c, kwf, kwb, iwf, iwb, cf, and_lo, or_lo, and_hi,
                                            or_hi, nfr, nbk);
  }
  acc.and_lo = and_lo;
  acc.or_lo = or_lo;
  acc.and_hi = and_hi;
  acc.or_hi = or_hi;
  // counts that broke the prefix would be an internal error: the status
  // word says so (the stores above stayed inside the segment regardless)
  const bool sane = cf == c_t && P <= w.lo && P + cf <= F && F + B0 + (w.cnt - cf) <= w.len;
  // wave totals: at most 64 * IPT per field, so the 16-bit halves do not carry
  const uint32_t tf = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(nfr), 63);
  const uint32_t tb = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(nbk), 63);
  const uint32_t tsel = (lane >> 1) ? tb : tf;
  const uint32_t v = (lane & 1u) ? (tsel >> 16) : (tsel & 0xffffu);
  if (lane < 4u && c.bit > 0 && sane && v) {
    // child c's tile jj of the next level counts at 2 * tile0 + c * nt + jj
    const uint32_t base = (lane >> 1) ? 2 * w.tile0 + w.nt : 2 * w.tile0;
    const uint32_t jj = (uint32_t)(((lane >> 1) ? B0 : P) / TILE) + (lane & 1u);
    atomic_add_u32(&a.cnt_out[base + jj], v);
  }
  if (lane == 0) {
    if (!sane) atomic_or_u32(&a.hdr->status, STATUS_BAD_COUNTS);
    if (w.j == 0) a.split[w.slot] = F;
  }
}

// One global level.  Waves take tiles t = g, g + G, g + 2G, ... (G waves in
// the grid).  A tile's descriptor is fetched two tiles ahead and its counts
// and keys one tile ahead of its use.
template <typename KT, bool IDX, int IPT>
__device__ __forceinline__ void level_body(const LevelArgs<KT> &a) {
  constexpr int TILE = 64 * IPT;
  using RT = typename std::conditional<sizeof(KT) == 8, uint64_t, uint32_t>::type;
  const uint32_t ntiles = (uint32_t)(ld_relaxed(&a.hdr->packed[a.level]) & 0xffffffffu);
  const rsrc_t mr = make_rsrc(a.meta, a.off.range);
  const uint32_t G = gridDim.x * 4u;
  // Workgroups go to the eight XCDs in turn (block b to XCD b % 8), each
  // with its own L2.  Numbering the waves XCD by XCD gives every XCD runs of
  // G/8 consecutive tiles per round, so the cache lines that two adjacent
  // tiles' output runs share are mostly written through one L2.
  const uint32_t nb = gridDim.x;
  const uint32_t bx = (nb & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3);
  const uint32_t g = uni(bx * 4u + (threadIdx.x >> 6));
  uint32_t t = g;
  WaveAcc<RT> acc;
  acc.slot = ~0u;
  acc.rep = 0;
  acc.and_lo = (RT)~(RT)0;
  acc.or_lo = 0;
  acc.and_hi = (RT)~(RT)0;
  acc.or_hi = 0;
  uint32_t dA = load_desc(a.tmap, t, ntiles);
  uint32_t dB = load_desc(a.tmap, t + G, ntiles);
  WaveTile A = wave_tile<TILE>(dA, t, ntiles), B;
  WaveRegs<KT, IPT> rA, rB;
  issue_tile<KT, IDX, IPT>(a, mr, A, rA);
  for (;;) {
    if (!A.valid) break;
    const uint32_t dC = load_desc(a.tmap, t + 2 * G, ntiles);
    B = wave_tile<TILE>(dB, t + G, ntiles);
    issue_tile<KT, IDX, IPT>(a, mr, B, rB);
    process_tile<KT, IDX, IPT, RT>(a, A, rA, acc, g);
    if (!B.valid) break;
    dB = load_desc(a.tmap, t + 3 * G, ntiles);
    A = wave_tile<TILE>(dC, t + 2 * G, ntiles);
    issue_tile<KT, IDX, IPT>(a, mr, A, rA);
    process_tile<KT, IDX, IPT, RT>(a, B, rB, acc, g);
    t += 2 * G;
  }
  flush_acc<KT, RT>(a, acc);
}

template <typename KT, bool IDX, int IPT>
__global__ __launch_bounds__(256) void level_kernel(LevelArgs<KT> a) {
  level_body<KT, IDX, IPT>(a);
}

// ------------------------------------------------------------- tail levels
//
// The last levels of a sort are usually empty: once every part is small
// enough for the LDS finish, no segment is live, yet prep, level and plan
// would each still be launched per level.  From a depth the host picks
// from n on, the levels run in one launch that walks them itself: it stops
// at the first level with no live tile (one header read) and otherwise runs
// the same three phases, separated by grid barriers.  The grid is at most
// what the device holds at once (occupancy x CUs), so a barrier waits only
// for running workgroups; each wait is still bounded in time, and one that
// runs out sets STATUS_BARRIER, after which no barrier waits, so the launch
// always ends.
template <typename KT>
struct TailArgs {
  // the arguments of levels first + 2i (set 0) and first + 2i + 1 (set 1):
  // buffers alternate by level parity; the level number is set per level
  PrepArgs<KT> prep0, prep1;
  LevelArgs<KT> lvl0, lvl1;
  PlanArgs plan0, plan1;
  Header *hdr;
  int first, last;       // levels [first, last)
};

// Barrier number `epoch` (1, 2, ...) of the launch.  Workgroups arrive in
// eight per-group counters, so that no single counter takes every arrival;
// the last of a group counts the group complete.  Each XCD has its own L2:
// the fences make every write before the barrier visible after it in every
// workgroup (L2 written back before the arrival, caches invalidated after
// the wait).
__device__ void grid_sync(Header *hdr, uint32_t epoch) {
  // every wave's stores reach L2 before the workgroup's one write-back: a
  // barrier alone does not wait for them
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __builtin_amdgcn_s_waitcnt(0);  // the write-back done before the arrival
    const uint32_t nb = gridDim.x;
    const uint32_t grp = blockIdx.x & 7u;
    const uint32_t gsize = (nb - grp + 7u) / 8u;
    const uint32_t ngrp = nb < 8u ? nb : 8u;
    if (atomic_add_u32(&hdr->bar_grp[grp], 1u) + 1u == epoch * gsize)
      atomic_add_u32(&hdr->bar_top, 1u);
    const uint64_t t0 = wall_clock64();
    while (ld_relaxed_u32(&hdr->bar_top) < epoch * ngrp &&
           !(ld_relaxed_u32(&hdr->status) & STATUS_BARRIER)) {
      __builtin_amdgcn_s_sleep(4);
      if (wall_clock64() - t0 > 20000000ull) {  // 0.2 s of the 100 MHz clock
        atomic_or_u32(&hdr->status, STATUS_BARRIER);
        break;
      }
    }
    __threadfence();
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
}

// One level of the tail: false when it has no live tile (nor has any
// later level).
template <typename KT, bool IDX, int IPT>
__device__ __forceinline__ bool tail_level(const PrepArgs<KT> &p, const LevelArgs<KT> &l,
                                           const PlanArgs &q, Header *hdr, int lvl,
                                           uint32_t &epoch) {
  // final since the barrier after the previous level's plan (or the
  // previous launch): the same value in every workgroup
  const uint64_t pk = ld_relaxed(&hdr->packed[lvl]);
  if ((uint32_t)pk == 0u) return false;
  PrepArgs<KT> pa = p;
  pa.level = lvl;
  const uint32_t nchunks = ((uint32_t)pk + PREP_TILES - 1) / PREP_TILES;
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    prep_body<KT, IPT>(pa, c);
    __syncthreads();
  }
  grid_sync(hdr, ++epoch);
  LevelArgs<KT> la = l;
  la.level = lvl;
  level_body<KT, IDX, IPT>(la);
  grid_sync(hdr, ++epoch);
  PlanArgs qa = q;
  qa.level = lvl;
  qa.l.next_level = lvl + 1;
  plan_body(qa);
  grid_sync(hdr, ++epoch);
  return true;
}

template <typename KT, bool IDX, int IPT>
__global__ __launch_bounds__(256) void tail_kernel(TailArgs<KT> a) {
  uint32_t epoch = 0;
  for (int lvl = a.first; lvl < a.last; ++lvl) {
    const bool odd = ((lvl - a.first) & 1) != 0;  // uniform: picks a whole argument set
    if (!tail_level<KT, IDX, IPT>(odd ? a.prep1 : a.prep0, odd ? a.lvl1 : a.lvl0,
                                  odd ? a.plan1 : a.plan0, a.hdr, lvl, epoch))
      break;
  }
}

// ------------------------------------------------------------ tiny segments
//
// Without the LDS finish every bit is a global level, and late levels hold
// many segments of a few keys: giving each one a whole level tile would
// make such a level cost a tile per segment.  Segments of at most TINY_MAX
// keys go to a list of their own instead (16-byte entries), which a wave
// takes 64 entries (a window) at a time.  An entry of at most TINY_LANE
// keys is split by its own lane: its keys in registers, a front mask, ranks
// by popcount.  The longer entries are moved to the window's first lanes
// and packed, whole, into batches of 64 x TINY_IPT positions (key position
// q at lane q % 64, item q / 64, as in a level tile); a key finds its
// segment from the batch's segment starts (one mask per item) and ranks are
// counted within the segment from the items' ballots.  Either way the split
// is a level tile's: front keys, then back keys, both in input order, into
// the other buffer (a split with an empty side moves nothing).  Children go
// to the next level's tiny list in the order of their parents, or, once
// done (one key, or bit 0 split), straight to the caller's buffers.  With
// `snapshot` set the segments are only written out as they stand (a sort
// stopped at this level).
constexpr int TINY_IPT = 4;

template <typename KT>
struct TinyArgs {
  KT *keys[2];
  uint32_t *idx[2];
  KT *keys_final;
  void *idx_final;
  const TinySeg *list;  // this level's tiny segments
  ListArgs l;       // the next level's tiny list (tiny_next, next_level, hdr)
  int level, w, mode, desc, idx64, snapshot;
};

// Front keys of a batch at positions below x, from the items' ballots.
__device__ __forceinline__ uint32_t batch_fronts_below(const uint64_t (&b)[TINY_IPT], uint32_t x) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < TINY_IPT; ++i) {
    const uint32_t lo = (uint32_t)i * 64u;
    if (x >= lo + 64u) c += (uint32_t)__popcll(b[i]);
    else if (x > lo) c += (uint32_t)__popcll(b[i] & (~0ull >> (64u - (x - lo))));
  }
  return c;
}

// A split tiny segment's part c (0: front, F keys; 1: back, len - F keys)
// as a segment of the next level, if it has two keys or more and bits remain
// (a part of one key, or split on bit 0, is in its final place already).
__device__ __forceinline__ bool tiny_child(uint64_t start, uint32_t meta, uint32_t len, uint32_t F, int c,
                                           int w, int mode, int desc, uint64_t &cst, uint32_t &clen,
                                           uint32_t &cmeta) {
  const int bit = (int)(meta & BIT_MASK);
  clen = c ? len - F : F;
  cst = start + (c ? F : 0u);
  if (clen < 2 || bit == 0) return false;
  const bool moved = F != 0 && F != len;
  const bool cio = !moved && (meta & META_IOTA) != 0;
  const uint32_t cbuf = moved ? ((meta & META_BUF) ^ META_BUF) : (meta & META_BUF);
  uint32_t sign = meta & META_SIGN;
  if (bit == w - 1)
    sign = ((uint32_t)c ^ (uint32_t)flip_of(bit, w, mode, desc, sign ? 1 : 0)) ? META_SIGN : 0u;
  cmeta = sign | cbuf | (cio ? META_IOTA : 0u) | (uint32_t)(bit - 1);
  return true;
}

// The next level's tiny segments made by a workgroup's TINY_WIN windows
// (per wave, window and lane, in LDS: the entry's start, and its meta,
// length and front count packed in a word, length 0 for none), listed with one list atomic for the whole workgroup: at the
// deepest levels nearly every entry has children, and one atomic per wave
// and window would be the level's serial bottleneck.  The key counts add up
// in thread 0 (klive_wg, kiota_wg) until the workgroup ends.
constexpr int TINY_WIN = 4;
// Entries of at most this many keys are split by their own lane, without
// the batch's lane exchanges.
constexpr uint32_t TINY_LANE = 8;

struct TinyRecs {
  uint64_t st[4][TINY_WIN][64];
  uint32_t pk[4][TINY_WIN][64];  // meta bits 0-10 | len << 11 | F << 20
};
static_assert(TINY_MAX < 512, "a tiny length and front count take 9 bits each");
__device__ __forceinline__ uint32_t tiny_pack(uint32_t meta, uint32_t len, uint32_t F) {
  return (meta & 0x7FFu) | len << 11 | F << 20;
}

__device__ __forceinline__ void emit_tiny_block(const ListArgs &a, int w, int mode, int desc,
                                                const TinyRecs &r, uint32_t (&s_n)[4],
                                                uint64_t (&s_k)[2][4], uint32_t &s_base,
                                                uint64_t &klive_wg, uint64_t &kiota_wg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // children in the order of their parents (window, lane, part), so that a
  // window of the next level covers neighbouring keys
  uint32_t at[TINY_WIN];  // the lane's first position in window v's run
  uint32_t n = 0;
  uint64_t klive = 0, kiota = 0;
  for (int v = 0; v < TINY_WIN; ++v) {
    uint32_t nv = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t cst;
      uint32_t clen, cmeta;
      const uint32_t pk = r.pk[wave][v][lane];
      if (tiny_child(r.st[wave][v][lane], pk & 0x7FFu, (pk >> 11) & 0x1FFu, pk >> 20, c, w, mode, desc,
                     cst, clen, cmeta)) {
        ++nv;
        klive += clen;
        if (cmeta & META_IOTA) kiota += clen;
      }
    }
    const uint32_t inc = wave_incl_scan_dpp(nv);
    at[v] = n + inc - nv;
    n += (uint32_t)__shfl((int)inc, 63);
  }
  klive = wave_sum_u64(klive);
  kiota = wave_sum_u64(kiota);
  if (lane == 0) {
    s_n[wave] = n;
    s_k[0][wave] = klive;
    s_k[1][wave] = kiota;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t tot = s_n[0] + s_n[1] + s_n[2] + s_n[3];
    s_base = tot ? atomic_add_u32(&a.hdr->n_tiny[a.next_level], tot) : 0u;
    klive_wg += s_k[0][0] + s_k[0][1] + s_k[0][2] + s_k[0][3];
    kiota_wg += s_k[1][0] + s_k[1][1] + s_k[1][2] + s_k[1][3];
  }
  __syncthreads();
  uint32_t wbase = s_base;
  for (int w2 = 0; w2 < wave; ++w2) wbase += s_n[w2];
  for (int v = 0; v < TINY_WIN; ++v) {
    uint32_t pos = wbase + at[v];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t cst;
      uint32_t clen, cmeta;
      const uint32_t pk = r.pk[wave][v][lane];
      if (tiny_child(r.st[wave][v][lane], pk & 0x7FFu, (pk >> 11) & 0x1FFu, pk >> 20, c, w, mode, desc,
                     cst, clen, cmeta)) {
        a.tiny_next[pos++] = TinySeg{cst, clen, cmeta};
      }
    }
  }
  __syncthreads();  // the counts in LDS are reused by the next call
}

template <typename KT, bool IDX>
__global__ __launch_bounds__(256) void tiny_kernel(TinyArgs<KT> a) {
  constexpr uint32_t BATCH = 64u * TINY_IPT;
  static_assert(TINY_MAX <= BATCH, "a tiny segment fits one batch");
  __shared__ uint32_t s_n[4], s_base;
  __shared__ uint64_t s_k[2][4];
  __shared__ TinyRecs s_rec;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nt = ld_relaxed_u32(&a.l.hdr->n_tiny[a.level]);
  // waves take equal runs of list entries, 64 at a time (a window), and
  // list the children of TINY_WIN windows with the rest of the workgroup;
  // every wave of a workgroup takes the same number of steps
  const uint32_t G = gridDim.x * (blockDim.x / 64u);
  const uint32_t g = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6);
  const uint32_t per = (nt + G - 1) / G;
  const uint32_t e_end = (g + 1) * per < nt ? (g + 1) * per : nt;
  const uint32_t steps = (per + 64u * TINY_WIN - 1) / (64u * TINY_WIN);
  uint64_t klive_wg = 0, kiota_wg = 0;
  // window t of the wave: list entries [g * per + 64 t, ...) up to e_end;
  // the next window's entries load while the wave works on the current one
  auto window_of = [&](uint32_t t) {
    const uint32_t e = g * per + t * 64u;
    return e < e_end ? (e_end - e < 64u ? e_end - e : 64u) : 0u;
  };
  auto load_entry = [&](uint32_t t, uint64_t &st, uint32_t &ln, uint32_t &mt) {
    st = 0;
    ln = 0;
    mt = 0;
    if (lane < window_of(t)) {
      // one 16-byte load whose every word is used (a loaded word left
      // unused is a register the compiler reuses at once, which makes it
      // wait for the load on the spot)
      const TinySeg q = a.list[g * per + t * 64u + lane];
      st = q.start;
      ln = q.len;
      mt = q.meta;
    }
  };
  uint64_t nst;
  uint32_t nln, nmt;
  load_entry(0, nst, nln, nmt);
  asm volatile("" ::"v"(nst), "v"(nln), "v"(nmt));  // the first window's entries, awaited here
  for (uint32_t step = 0; step < steps; ++step) {
#pragma unroll 1
   for (int v = 0; v < TINY_WIN; ++v) {
    const uint32_t t = step * TINY_WIN + (uint32_t)v;
    // the lane's own entry (length 0 past the window)
    const uint64_t est = nst;
    const uint32_t emt = nmt, elen = nln;
    load_entry(t + 1, nst, nln, nmt);
    uint32_t eF = 0;  // its front count
    // an entry of at most TINY_LANE keys: its lane splits it alone
    const bool sm = elen <= TINY_LANE;
    if (__ballot(sm && elen > 0)) {
      const int bb = (int)(emt & BIT_MASK);
      const uint32_t ff = (uint32_t)flip_of(bb, a.w, a.mode, a.desc, (emt & META_SIGN) ? 1 : 0);
      const int kb = (emt & META_BUF) ? 1 : 0;
      const bool io = (emt & META_IOTA) != 0;
      const KT *kp = kb ? a.keys[1] : a.keys[0];
      const uint32_t *xp = kb ? a.idx[1] : a.idx[0];
      KT kk[TINY_LANE];
      uint32_t xx[TINY_LANE];
#pragma unroll
      for (uint32_t j = 0; j < TINY_LANE; ++j) {
        kk[j] = 0;
        xx[j] = 0;
        if (sm && j < elen) {
          kk[j] = kp[est + j];
          if (IDX) xx[j] = io ? j : xp[est + j];
        }
      }
      uint32_t fm = 0;  // bit j: key j goes to the front part
#pragma unroll
      for (uint32_t j = 0; j < TINY_LANE; ++j) {
        const uint32_t side = (uint32_t)(((uint64_t)kk[j] >> bb) & 1u) ^ ff;
        fm |= ((j < elen ? 1u : 0u) & (side ^ 1u)) << j;
        if (IDX) asm volatile("" ::"v"(xx[j]));
      }
      const uint32_t F = (uint32_t)__popc(fm);
      if (sm) eF = F;
      const bool mv = F != 0 && F != elen;
      const int cb = mv ? 1 - kb : kb;
#pragma unroll
      for (uint32_t j = 0; j < TINY_LANE; ++j) {
        if (!(sm && j < elen)) continue;
        if (a.snapshot) {
          // as it stands: to the caller's buffers
          if (kb) a.keys_final[est + j] = kk[j];
          if (IDX && (kb || io || a.idx64)) {
            if (a.idx64) static_cast<int64_t *>(a.idx_final)[est + j] = (int64_t)xx[j];
            else static_cast<uint32_t *>(a.idx_final)[est + j] = xx[j];
          }
          continue;
        }
        const bool front = (fm >> j) & 1u;
        const uint32_t r = (uint32_t)__popc(fm & ((1u << j) - 1u));
        const uint32_t dst = mv ? (front ? r : F + (j - r)) : j;
        const uint32_t clen = front ? F : elen - F;
        if (clen >= 2 && bb > 0) {
          // a live part: its keys to the buffer the next level reads
          if (mv) {
            (cb ? a.keys[1] : a.keys[0])[est + dst] = kk[j];
            if (IDX) (cb ? a.idx[1] : a.idx[0])[est + dst] = xx[j];
          }
        } else {
          // a done part: straight to the caller's buffers (buffer 0 holds
          // the caller's keys), unless the key is there already
          const bool cio = !mv && io;
          if (mv || kb) a.keys_final[est + dst] = kk[j];
          if (IDX && (mv || cb || cio || a.idx64)) {
            const uint32_t vv = cio ? dst : xx[j];
            if (a.idx64) static_cast<int64_t *>(a.idx_final)[est + dst] = (int64_t)vv;
            else static_cast<uint32_t *>(a.idx_final)[est + dst] = vv;
          }
        }
      }
    }
    // the next window's entries are complete here when the lane path ran
    // (its wait covered them); saying so keeps the loop head from waiting
    // for them behind this window's stores
    asm volatile("" ::"v"(nst), "v"(nln), "v"(nmt));
    // the other entries go through batches, moved to the window's first
    // lanes (a permutation: those entries first, in order, then the rest)
    const uint64_t bigm = __ballot(!sm);
    const uint32_t nb = (uint32_t)__popcll(bigm);
    const uint64_t below = lane ? (~0ull >> (64u - lane)) : 0ull;
    const uint32_t rk = !sm ? (uint32_t)__popcll(bigm & below) : nb + (uint32_t)__popcll(~bigm & below);
    Seg sg = {};
    uint32_t len = 0;
    uint32_t myF = 0;  // the front count of the batch entry in this lane
    if (nb) {
      const int to = (int)(rk * 4u);
      sg.start = (uint64_t)(uint32_t)__builtin_amdgcn_ds_permute(to, (int)(uint32_t)est) |
                 ((uint64_t)(uint32_t)__builtin_amdgcn_ds_permute(to, (int)(uint32_t)(est >> 32)) << 32);
      sg.meta = (uint32_t)__builtin_amdgcn_ds_permute(to, (int)emt);
      const uint32_t pl = (uint32_t)__builtin_amdgcn_ds_permute(to, (int)elen);
      len = lane < nb ? pl : 0u;
    }
    const uint32_t nwin = nb;
    const uint32_t cum = wave_incl_scan_dpp(len);  // over the window
    const uint32_t s0w = cum - len;                  // the entry's first window position
    // batches: successive runs of the window's entries whose keys fit BATCH
    for (uint32_t b0 = 0; b0 < nwin;) {
      const uint32_t base = b0 ? (uint32_t)__shfl((int)cum, (int)b0 - 1) : 0u;
      const uint64_t fits = __ballot(lane >= b0 && lane < nwin && cum - base <= BATCH);
      const uint32_t m = (uint32_t)__popcll(fits);  // >= 1: every entry fits alone
      const bool mine = lane >= b0 && lane < b0 + m;
      const uint32_t s0 = s0w - base;                // batch positions of the lane's entry
      const uint32_t s1 = cum - base;
      // per item, a bit at every segment start inside it
      uint64_t starts[TINY_IPT];
#pragma unroll
      for (int i = 0; i < TINY_IPT; ++i) {
        const uint32_t d = s0 - (uint32_t)i * 64u;
        starts[i] = wave_or_dpp(mine && d < 64u ? 1ull << d : 0ull);
      }
      const uint32_t total = (uint32_t)__shfl((int)cum, (int)(b0 + m) - 1) - base;
      // every key: its segment (a lane of the batch), its place in it, its
      // key and index -- every load issued before any is used
      KT k[TINY_IPT];
      uint32_t x[TINY_IPT], segi[TINY_IPT], jj[TINY_IPT], mts[TINY_IPT];
      uint64_t sts[TINY_IPT], fb[TINY_IPT];
      uint32_t before = 0;  // segment starts in earlier items
#pragma unroll
      for (int i = 0; i < TINY_IPT; ++i) {
        const uint32_t q = (uint32_t)i * 64u + lane;
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        const uint32_t si = b0 + before + (uint32_t)__popcll(starts[i] & upto) - 1u;
        before += (uint32_t)__popcll(starts[i]);
        const bool valid = q < total;
        const int sl = valid ? (int)si : 0;
        segi[i] = (uint32_t)sl;
        sts[i] = (uint64_t)(uint32_t)__shfl((int)(uint32_t)sg.start, sl) |
                 ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(sg.start >> 32), sl) << 32);
        mts[i] = (uint32_t)__shfl((int)sg.meta, sl);
        jj[i] = q - (uint32_t)__shfl((int)s0, sl);
        const int kb = (mts[i] & META_BUF) ? 1 : 0;
        const bool io = (mts[i] & META_IOTA) != 0;
        // the buffer by a select: an index into the argument's array
        // differs per lane and would load the pointer from memory first
        const KT *kp = kb ? a.keys[1] : a.keys[0];
        k[i] = valid ? kp[sts[i] + jj[i]] : (KT)0;
        x[i] = 0;
        if (IDX) {
          const uint32_t *xp = kb ? a.idx[1] : a.idx[0];
          x[i] = !valid ? 0u : (io ? jj[i] : xp[sts[i] + jj[i]]);
        }
      }
      // the keys' sides without a branch, so that every later use finds
      // the loads complete on every path (a wait inside a branch would be
      // repeated before each store, and a wait there also waits for the
      // stores already issued)
#pragma unroll
      for (int i = 0; i < TINY_IPT; ++i) {
        const uint32_t valid = (uint32_t)i * 64u + lane < total ? 1u : 0u;
        const int bb = (int)(mts[i] & BIT_MASK);
        const uint32_t ff = (uint32_t)flip_of(bb, a.w, a.mode, a.desc, (mts[i] & META_SIGN) ? 1 : 0);
        const uint32_t side = (uint32_t)(((uint64_t)k[i] >> bb) & 1u) ^ ff;
        fb[i] = __ballot((valid & (side ^ 1u)) != 0u);
        if (IDX) asm volatile("" ::"v"(x[i]));
      }
      // per entry of the batch: its front keys before it and in it
      const uint32_t Ps = batch_fronts_below(fb, mine ? s0 : 0u);
      const uint32_t Fs = batch_fronts_below(fb, mine ? s1 : 0u) - Ps;
#pragma unroll
      for (int i = 0; i < TINY_IPT; ++i) {
        const uint32_t q = (uint32_t)i * 64u + lane;
        // the lane exchanges first, with every lane active; then the keys
        const int sl = (int)segi[i];
        const uint32_t F = (uint32_t)__shfl((int)Fs, sl);
        const uint32_t P0 = (uint32_t)__shfl((int)Ps, sl);
        const uint32_t ln = (uint32_t)__shfl((int)len, sl);
        const uint64_t st = sts[i];
        const uint32_t mt = mts[i];
        if (q >= total) continue;
        const int kb = (mt & META_BUF) ? 1 : 0;
        const bool io = (mt & META_IOTA) != 0;
        const int bb = (int)(mt & BIT_MASK);
        const uint32_t j = jj[i];
        if (a.snapshot) {
          // as it stands: to the caller's buffers
          if (kb) a.keys_final[st + j] = k[i];
          if (IDX && (kb || io || a.idx64)) {
            if (a.idx64) static_cast<int64_t *>(a.idx_final)[st + j] = (int64_t)x[i];
            else static_cast<uint32_t *>(a.idx_final)[st + j] = x[i];
          }
          continue;
        }
        const bool front = (fb[i] >> lane) & 1u;
        const uint32_t r = batch_fronts_below(fb, q) - P0;  // front keys before it in its segment
        const bool mv = F != 0 && F != ln;
        const uint32_t dst = mv ? (front ? r : F + (j - r)) : j;
        const int cb = mv ? 1 - kb : kb;
        const uint32_t clen = front ? F : ln - F;
        if (clen >= 2 && bb > 0) {
          // a live part: its keys to the buffer the next level reads
          if (mv) {
            (cb ? a.keys[1] : a.keys[0])[st + dst] = k[i];
            if (IDX) (cb ? a.idx[1] : a.idx[0])[st + dst] = x[i];
          }
        } else {
          // a done part: straight to the caller's buffers (buffer 0 holds
          // the caller's keys), unless the key is there already
          const bool cio = !mv && io;
          if (mv || kb) a.keys_final[st + dst] = k[i];
          if (IDX && (mv || cb || cio || a.idx64)) {
            // an identity index is the key's place in its user segment,
            // which a segment that has never moved starts
            const uint32_t v = cio ? dst : x[i];
            if (a.idx64) static_cast<int64_t *>(a.idx_final)[st + dst] = (int64_t)v;
            else static_cast<uint32_t *>(a.idx_final)[st + dst] = v;
          }
        }
      }
      if (mine) myF = Fs;
      b0 += m;
    }
    // back to the entry's own lane
    const uint32_t bF = (uint32_t)__shfl((int)myF, (int)rk);
    if (!sm) eF = bF;
    // lane l: entry l of the window, whose parts the workgroup lists below
    const uint32_t wv = threadIdx.x >> 6;
    s_rec.st[wv][v][lane] = est;
    s_rec.pk[wv][v][lane] = a.snapshot ? 0u : tiny_pack(emt, elen, eF);
   }
   emit_tiny_block(a.l, a.w, a.mode, a.desc, s_rec, s_n, s_k, s_base, klive_wg, kiota_wg);
  }
  if (threadIdx.x == 0) {
    if (klive_wg) atomic_add_u64(&a.l.hdr->live_keys[a.l.next_level], klive_wg);
    if (kiota_wg) atomic_add_u64(&a.l.hdr->iota_keys[a.l.next_level], kiota_wg);
  }
}

// Level launch shape: keys per lane of a level tile.  16 (8 for 64-bit keys)
// in the default shape -- two waves per SIMD, each with a 1024-key tile in
// flight -- and half that in the smaller one.
template <typename KT, int V>
struct LevelShape {
  static constexpr int LIPT = (V == 0 ? 16 : 8) / (sizeof(KT) == 8 ? 2 : 1);
  static constexpr uint32_t TILE = 64 * LIPT;
};

// ------------------------------------------------------------- LDS finish

template <typename KT>
struct FinishArgs {
  const KT *keys_buf[2];
  const uint32_t *idx_buf[2];
  KT *keys_final;
  void *idx_final;
  const Seg *list;
  const uint32_t *count;  // entries in list (a header counter)
  Header *hdr;
  int w, mode, desc, idx64, no_skip;
};

// Rank word of a key: bit b is 1 exactly when the key goes to the back part
// in a split on bit b (the test of Algorithm 1 with the direction rules of
// Algorithms 3-5), so sorting by it ascending is the method's order.  The
// sign decides the direction of the lower bits of float keys.
template <typename KT>
__device__ __forceinline__ KT rank_word(KT k, int w, int mode, int desc) {
  const KT top = (KT)((KT)1 << (w - 1));
  KT m = desc ? (KT)~(KT)0 : (KT)0;
  if (mode != MODE_U) m ^= top;
  if (mode == MODE_F && (k & top)) m ^= (KT)~top;
  return (KT)(k ^ m);
}
// Its inverse: the top bit of the key follows from the top bit of the word.
template <typename KT>
__device__ __forceinline__ KT key_of_rank_word(KT u, int w, int mode, int desc) {
  const KT top = (KT)((KT)1 << (w - 1));
  KT m = desc ? (KT)~(KT)0 : (KT)0;
  if (mode != MODE_U) m ^= top;
  const bool ktop = ((u ^ m) & top) != 0;
  if (mode == MODE_F && ktop) m ^= (KT)~top;
  return (KT)(u ^ m);
}

// Waves per SIMD the finish kernel is built for: narrow keys with at most
// 8192 per block are held to 128 registers so that two blocks share a CU
// (their LDS fits twice); the rest take what they need.
template <typename KT>
constexpr int finish_waves_per_eu(int block, int ipt) {
  return (sizeof(KT) <= 4 && block * ipt <= 8192) ? 4 : 1;
}

// One workgroup per segment of at most BLOCK*IPT keys: the keys are loaded
// once, all remaining bits are resolved in LDS, and the final keys and
// indices go to the caller's buffers (the switch to a cache-resident routine
// for small parts that the paper proposes in Sections IV-B and V).  The
// segment's keys share every bit above its current bit, so a stable sort of
// the rank words on the bits where the segment's keys differ is the same
// result as the remaining bit-by-bit splits.  Those bits are packed into a
// contiguous code, sorted in stable passes of 4 bits, least significant
// first, with per-(digit, thread) counters in LDS and one block-wide scan per
// pass.  The constant bits are put back at the end.
template <typename KT, bool IDX, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(finish_waves_per_eu<KT>(BLOCK, IPT))))
void finish_kernel(FinishArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr int T = BLOCK * IPT;
  using RT = typename std::conditional<sizeof(KT) == 8, uint64_t, uint32_t>::type;
  // LDS: the codes, the indices, then the (digit, thread) counters (two
  // 16-bit counters a word).  For keys of at most 4 bytes the segment record
  // and the AND/OR partials live in the counter words, which are unused
  // until the first pass, and the per-wave scan totals in the code words,
  // which every pass has read into registers before it writes them; so two
  // 8192-key blocks fit one CU's LDS.
  constexpr bool NARROW = sizeof(KT) <= 4;
  constexpr int CNTW = 8 * BLOCK;
  constexpr int SEGW = (int)(sizeof(Seg) / 4);
  constexpr int XW = SEGW + 4 * WAVES + WAVES;  // segment record, AND/OR partials, scan totals
  __shared__ RT s_code[T];
  __shared__ uint32_t s_idx[IDX ? T : 1];
  __shared__ __attribute__((aligned(16))) uint32_t s_cnt[CNTW + (NARROW ? 0 : XW)];
  static_assert(!NARROW || CNTW >= SEGW + 4 * WAVES, "segment record and partials fit the counters");
  Seg &s_seg = *reinterpret_cast<Seg *>(NARROW ? s_cnt : s_cnt + CNTW);
  uint64_t(*const s_red)[WAVES] =
      reinterpret_cast<uint64_t(*)[WAVES]>(s_cnt + (NARROW ? SEGW : CNTW + SEGW));
  uint32_t *const s_wsum =
      NARROW ? reinterpret_cast<uint32_t *>(s_code) : s_cnt + CNTW + SEGW + 4 * WAVES;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nf = *a.count;

  for (uint32_t e = blockIdx.x; e < nf; e += gridDim.x) {
    if (tid == 0) s_seg = a.list[e];
    __syncthreads();
    const uint64_t start = uni(s_seg.start);
    const uint64_t slen = uni(s_seg.len);
    const uint32_t len = (uint32_t)(slen < (uint64_t)T ? slen : (uint64_t)T);
    const uint32_t meta = uni(s_seg.meta);
    const int bit0 = (int)(meta & BIT_MASK);
    const bool iota = (meta & META_IOTA) != 0;
    const int buf = (meta & META_BUF) ? 1 : 0;
    if (tid == 0 && slen > (uint64_t)T) atomic_or_u32(&a.hdr->status, STATUS_OVERSIZE);

    const rsrc_t kr = make_rsrc(a.keys_buf[buf] + start, len * (uint32_t)sizeof(KT));
    const rsrc_t ir = make_rsrc(IDX ? a.idx_buf[buf] + start : nullptr, IDX && !iota ? len * 4u : 0u);
    RT u[IPT];
    uint32_t ix[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t p = (uint32_t)(i * BLOCK + tid);
      const uint32_t o = p;  // past len: out of range, reads 0
      u[i] = (RT)rank_word<KT>(buf_load<KT>(kr, o * (uint32_t)sizeof(KT)), a.w, a.mode, a.desc);
      ix[i] = 0;
      if (IDX) ix[i] = iota ? p : buf_load<uint32_t>(ir, o * 4u);
    }

    RT constw = 0;  // the bits all keys share, at their place in the word
    RT todo = 0;    // the bits still to sort by, at or below bit0
    if (bit0 != (int)BIT_NONE && len >= 2) {
      RT andv = (RT)~(RT)0, orv = 0;
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        if ((uint32_t)(i * BLOCK + tid) < len) {
          andv &= u[i];
          orv |= u[i];
        }
      }
      const uint64_t aw = wave_and_dpp((uint64_t)andv | (sizeof(RT) == 8 ? 0ull : ~0ull << 32));
      const uint64_t ow = wave_or_dpp((uint64_t)orv);
      if (lane == 0) {
        s_red[0][wave] = aw;
        s_red[1][wave] = ow;
      }
      __syncthreads();
      uint64_t at = ~0ull, ot = 0;
#pragma unroll
      for (int w2 = 0; w2 < WAVES; ++w2) {
        at &= s_red[0][w2];
        ot |= s_red[1][w2];
      }
      const uint64_t below = (bit0 == 63) ? ~0ull : ((2ull << bit0) - 1);
      todo = (RT)(a.no_skip ? below : ((at ^ ot) & below));
      constw = (RT)(at & ~(uint64_t)todo);
    }

    if (todo) {
      // pack the bits to sort by into a contiguous code (runs of set bits
      // of `todo`, low to high)
      const int nbits = (int)__popcll((uint64_t)todo);
      RT code[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) code[i] = 0;
      {
        RT m = todo;
        int pos = 0;
        while (m) {
          const int lo = __ffsll((unsigned long long)m) - 1;
          const RT run = (RT)(m >> lo);
          const int rl = (~run == 0) ? (int)(8 * sizeof(RT)) - lo : __ffsll((unsigned long long)~run) - 1;
          const RT rmask = rl >= (int)(8 * sizeof(RT)) ? (RT)~(RT)0 : (RT)(((RT)1 << rl) - 1);
#pragma unroll
          for (int i = 0; i < IPT; ++i) code[i] |= ((u[i] >> lo) & rmask) << pos;
          pos += rl;
          m &= ~(RT)(rmask << lo);
        }
      }
      {
        // Stable LSD passes of CRB bits over the packed codes, ranked in
        // blocked order (thread t holds positions t*IPT .. t*IPT + IPT - 1):
        // each item bumps its (digit, thread) counter in LDS in position
        // order -- an LDS atomic that returns the count so far -- then an
        // exclusive scan over the counters in (digit, thread) order turns
        // every counter into its base, and an item's rank is its counter's
        // base plus its count so far.  Positions past the segment's end
        // carry the largest code and stay last.  Digit d's counter of thread
        // t is the (d >> 3) half of word (d & 7) * BLOCK + t: one scan of the
        // words in (word, thread) order yields, in the low halves, the bases
        // of digits 0..7 and, in the high halves, those of digits 8..15 less
        // the count of digits 0..7 (the low half of the total).
        constexpr int CRB = 4, CDIG = 1 << CRB, CW = CDIG / 2;
        static_assert(T < 65536, "16-bit counter halves");
        static_assert((T & (T - 1)) == 0, "power-of-two finish size");
        constexpr int PB = __builtin_ctz((unsigned)T);  // bits of a position
        const RT maxc = (nbits >= (int)(8 * sizeof(RT))) ? (RT)~(RT)0 : (RT)(((RT)1 << nbits) - 1);
        // With indices, a code that leaves PB bits of its word free travels
        // with its position in one word (code above, position below): the passes
        // then move one word per key, and each index is fetched once, by
        // position, at the end.
        const bool pk = IDX && nbits + PB <= (int)(8 * sizeof(RT));
        const int dsh = pk ? PB : 0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          const RT c = p < len ? code[i] : maxc;
          s_code[p] = pk ? (RT)((c << PB) | p) : c;
          if (IDX) s_idx[p] = ix[i];
        }
        auto passes = [&](auto carry) {
          constexpr bool CARRY = decltype(carry)::value;
          for (int sh = 0; sh < nbits; sh += CRB) {
            __syncthreads();
            RT c[IPT];
            uint32_t x[IPT], loc[IPT];
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
              c[j] = s_code[tid * IPT + j];
              if (CARRY) x[j] = s_idx[tid * IPT + j];
            }
#pragma unroll
            for (int d = 0; d < CW; ++d) s_cnt[d * BLOCK + tid] = 0;
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
              const uint32_t d = (uint32_t)(c[j] >> (sh + dsh)) & (uint32_t)(CDIG - 1);
              const uint32_t hs = (d >> 3) << 4;
              loc[j] = (atomicAdd(&s_cnt[(d & (CW - 1)) * BLOCK + tid], 1u << hs) >> hs) & 0xffffu;
            }
            __syncthreads();
            uint32_t lowtot;
            {
              uint32_t v[CW];
              uint32_t sum = 0;
#pragma unroll
              for (int k = 0; k < CW; ++k) {
                v[k] = s_cnt[tid * CW + k];
                sum += v[k];
              }
              const uint32_t inc = wave_incl_scan_dpp(sum);
              if (lane == 63) s_wsum[wave] = inc;
              __syncthreads();
              uint32_t ex = inc - sum, tot = 0;
#pragma unroll
              for (int w2 = 0; w2 < WAVES; ++w2) {
                const uint32_t ws = s_wsum[w2];
                if (w2 < wave) ex += ws;
                tot += ws;
              }
              lowtot = tot & 0xffffu;
#pragma unroll
              for (int k = 0; k < CW; ++k) {
                s_cnt[tid * CW + k] = ex;
                ex += v[k];
              }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
              const uint32_t d = (uint32_t)(c[j] >> (sh + dsh)) & (uint32_t)(CDIG - 1);
              const uint32_t wv = s_cnt[(d & (CW - 1)) * BLOCK + tid];
              const uint32_t base = (d >> 3) ? (wv >> 16) + lowtot : (wv & 0xffffu);
              const uint32_t dst = base + loc[j];
              s_code[dst] = c[j];
              if (CARRY) s_idx[dst] = x[j];
            }
          }
        };
        if (IDX && !pk)
          passes(std::true_type{});
        else
          passes(std::false_type{});
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          const uint32_t p = (uint32_t)(i * BLOCK + tid);
          const RT wv = s_code[p];
          if (pk) {
            code[i] = wv >> PB;
            ix[i] = s_idx[wv & (RT)(T - 1)];
          } else {
            code[i] = wv;
            if (IDX) ix[i] = s_idx[p];
          }
        }
        __syncthreads();
      }
      // unpack: the sorted bits back into place, the shared bits around them
      {
        RT m = todo;
        int pos = 0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) u[i] = constw;
        while (m) {
          const int lo = __ffsll((unsigned long long)m) - 1;
          const RT run = (RT)(m >> lo);
          const int rl = (~run == 0) ? (int)(8 * sizeof(RT)) - lo : __ffsll((unsigned long long)~run) - 1;
          const RT rmask = rl >= (int)(8 * sizeof(RT)) ? (RT)~(RT)0 : (RT)(((RT)1 << rl) - 1);
#pragma unroll
          for (int i = 0; i < IPT; ++i) u[i] |= ((code[i] >> pos) & rmask) << lo;
          pos += rl;
          m &= ~(RT)(rmask << lo);
        }
      }
    }

    const rsrc_t kw = make_rsrc(a.keys_final + start, len * (uint32_t)sizeof(KT));
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t p = (uint32_t)(i * BLOCK + tid);
      buf_store(kw, p * (uint32_t)sizeof(KT), key_of_rank_word<KT>((KT)u[i], a.w, a.mode, a.desc));
    }
    if (IDX) {
      if (a.idx64) {
        const rsrc_t iw = make_rsrc(static_cast<int64_t *>(a.idx_final) + start, len * 8u);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
          buf_store(iw, (uint32_t)(i * BLOCK + tid) * 8u, (uint64_t)ix[i]);
      } else {
        const rsrc_t iw = make_rsrc(static_cast<uint32_t *>(a.idx_final) + start, len * 4u);
#pragma unroll
        for (int i = 0; i < IPT; ++i) buf_store(iw, (uint32_t)(i * BLOCK + tid) * 4u, ix[i]);
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
// final: in scratch, or with indices not yet in the caller's buffer (still
// the identity, or to be widened).  All keys of a retired segment are the
// same pattern, so keys are filled.
template <typename KT, bool IDX>
__global__ void copy_kernel(CopyArgs<KT> a) {
  const uint32_t nc = a.hdr->n_copy;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t e = 0; e < nc; ++e) {
    const Seg s = a.list[e];
    const bool iota = (s.meta & META_IOTA) != 0;
    const int buf = (s.meta & META_BUF) ? 1 : 0;
    if (buf) {
      const KT kv = a.keys_buf[1][s.start];
      for (uint64_t i = i0; i < s.len; i += stride) a.keys_final[s.start + i] = kv;
    }
    if (!IDX) continue;
    if (iota) {
      for (uint64_t i = i0; i < s.len; i += stride) {
        if (a.idx64) static_cast<int64_t *>(a.idx_final)[s.start + i] = (int64_t)i;
        else static_cast<uint32_t *>(a.idx_final)[s.start + i] = (uint32_t)i;
      }
    } else if (buf || a.idx64) {
      const uint32_t *src = a.idx_buf[buf] + s.start;
      for (uint64_t i = i0; i < s.len; i += stride) {
        const uint32_t v = src[i];
        if (a.idx64) static_cast<int64_t *>(a.idx_final)[s.start + i] = (int64_t)v;
        else static_cast<uint32_t *>(a.idx_final)[s.start + i] = v;
      }
    }
  }
}

// --------------------------------------------------------- level snapshot
//
// The per-level property of Theorem 3's induction (after the k most
// significant bits, the array is ordered by its k-bit prefix) made visible:
// a sort stopped after `level` global levels leaves every live segment of
// that level in the buffer its meta names, its indices possibly still the
// identity.  One wave per level tile writes the tile's keys and indices to
// the caller's buffers; retired segments reach them through the copy and
// finish lists as in a full sort.
template <typename KT>
struct SnapArgs {
  const KT *keys_buf[2];
  const uint32_t *idx_buf[2];
  KT *keys_final;
  void *idx_final;
  const Seg *live;  // the live list of level `level`, in tile order
  const Header *hdr;
  int level;
  uint32_t tile;    // keys per level tile
  int idx64;
};

template <typename KT, bool IDX>
__global__ __launch_bounds__(256) void snapshot_kernel(SnapArgs<KT> a) {
  const uint64_t pk = a.hdr->packed[a.level];
  const uint32_t S = (uint32_t)(pk >> 32), ntiles = (uint32_t)pk;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t G = gridDim.x * 4;
  for (uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6); t < ntiles; t += G) {
    const uint32_t s = wave_search_le(S, [&](uint32_t i) { return a.live[i].tile0 <= t; });
    const Seg sg = a.live[s];
    const uint64_t lo = (uint64_t)(t - sg.tile0) * a.tile;
    const uint64_t hi = lo + a.tile < sg.len ? lo + a.tile : sg.len;
    const int buf = (sg.meta & META_BUF) ? 1 : 0;
    const bool iota = (sg.meta & META_IOTA) != 0;
    for (uint64_t q = lo + lane; q < hi; q += 64) {
      const uint64_t p = sg.start + q;
      if (buf) a.keys_final[p] = a.keys_buf[1][p];
      if (IDX && (iota || buf || a.idx64)) {
        const uint32_t v = iota ? (uint32_t)q : a.idx_buf[buf][p];
        if (a.idx64) static_cast<int64_t *>(a.idx_final)[p] = (int64_t)v;
        else static_cast<uint32_t *>(a.idx_final)[p] = v;
      }
    }
  }
}

// ------------------------------------------------------- in-place levels
//
// A keys-only variant whose scratch is O(n / tile): each level partitions
// every live segment in place, exchanging misplaced keys as Algorithm 1's
// swap loop does, instead of scattering into a second buffer.  Equal keys
// are indistinguishable, so the sorted keys equal the stable path's; the
// exchange is not stable, so no permutation is produced.
//
// With F front keys the split point is k = start + F.  The c back keys left
// of k and the c front keys right of k are exchanged in pairs: the r-th
// back key left of k, counted from the left, with the r-th front key right
// of k, counted from the segment's right end.  Tiles cut both rank
// sequences: a tile left of k starts its back ranks at a_j (back keys
// before it), a tile right of k starts its front ranks at b_i (front keys
// after it).  A work item starts at every such boundary r0 and runs to the
// next one, so it meets at most one tile on each side whatever the key
// distribution: it takes the back keys of one tile from its left start and
// the front keys of one tile from its right start, and exchanges as many
// pairs as the shorter list holds.  The side whose tile ends at the next
// boundary lists exactly the item's keys; the other side lists them first
// and keys of later items after them.  An item reads only its own keys and
// keys no block writes (back keys right of k, front keys left of k), apart
// from those later keys, which it never uses.  Per level:
//  count:  per tile, the front keys on the segment's bit (tcnt, sums per
//          64-tile group in scnt, the segment total F in split) and the
//          AND/OR of the front and of the back keys.  Those are properties
//          of the two key sets, not of their positions, so they are taken
//          before any key moves.
//  prefix: per tile, the front keys in the segment's earlier tiles.
//  locate: per tile, up to two items (one at its first back key left of k,
//          one at its last front key right of k) and the partner position
//          of each start, found before any key moves: one wave per tile
//          searches the tile prefixes, then the partner tile's per-chunk
//          counts, and reads a single 64 * IPT-key chunk.  An item at a right
//          tile's boundary that is also a left tile's is left to the latter.
//  (count also records each tile's first back and last front key and the
//  front keys of each wave's chunk: wave w of the block reads the tile's
//  keys [w * 64 * IPT, (w + 1) * 64 * IPT).)
//  swap:   per item, list both sides in LDS and exchange.

constexpr uint64_t LOC_NONE = ~0ull;

template <typename KT>
struct InplaceArgs {
  KT *keys;
  const Seg *live;   // this level's live segments, in tile order
  Seg *tiles;        // per tile: its segment (written by the count pass)
  Header *hdr;
  uint32_t *tcnt;    // per tile, at the segment's cbase + j
  uint32_t *scnt;    // per 64-tile group, at cbase + j / 64
  uint32_t *pre;     // per tile: front keys in the segment's earlier tiles
  uint32_t *sub;     // per tile and wave: front keys of the wave's 64 * IPT-key chunk
  uint32_t *ends;    // per tile: first back key, last front key + 1 (tile positions)
  uint64_t *items;   // per tile: two items, each {left start, right start}
  AccRep *acc;       // AND/OR replicas of the front (lo) and back (hi) keys
  uint64_t *split;   // per segment slot: front keys F
  int w, mode, desc, level;
};

// Exclusive prefix over the block; `total` gets the block's sum.  Uses
// s_w[WAVES] and leaves it free for the next call.
template <int WAVES>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan_dpp(v);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < WAVES; ++q) {
    const uint32_t x = s_w[q];
    before += q < wave ? x : 0u;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + inc - v;
}

// Position of the r-th key (from 0, in position order) of the given side
// (front or back) among a tile's keys [base, base + cnt), or LOC_NONE if
// there are not that many.  sub[0, WAVES) holds the front keys of each
// 64 * IPT-key chunk of the tile (as the count pass reads it), so one wave
// finds the chunk from the counts and reads that chunk only.  All 64 lanes
// must call it; every lane gets the answer.
template <typename KT, int WAVES, int IPT>
__device__ uint64_t wave_select(const KT *keys, uint64_t base, uint32_t cnt, const uint32_t *sub,
                                uint32_t r, bool want_front, int bit, uint64_t f) {
  constexpr uint32_t SUB = 64 * IPT;
  const uint32_t lane = threadIdx.x & 63;
  uint32_t cw = 0;
  if (lane < (uint32_t)WAVES) {
    const uint32_t c0 = lane * SUB;
    const uint32_t clen = cnt > c0 ? (cnt - c0 < SUB ? cnt - c0 : SUB) : 0u;
    const uint32_t fr = sub[lane];
    cw = want_front ? fr : clen - fr;
  }
  const uint32_t inc = wave_incl_scan_u32(cw);
  const uint64_t past = __ballot(lane < (uint32_t)WAVES && inc > r);
  if (!past) return LOC_NONE;
  const int sc = __ffsll((unsigned long long)past) - 1;
  uint32_t rr = r - (uint32_t)__shfl((int)(inc - cw), sc);
  const uint32_t c0 = (uint32_t)sc * SUB;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t q = c0 + (uint32_t)(i * 64) + lane;
    bool hit = false;
    if (q < cnt) {
      const uint64_t k = (uint64_t)keys[base + q];
      hit = ((((k >> bit) & 1ull) == f) == want_front);
    }
    const uint64_t m = __ballot(hit);
    const uint32_t pc = (uint32_t)__popcll(m);
    if (rr < pc) {
      uint64_t mm = m;
      for (uint32_t z = 0; z < rr; ++z) mm &= mm - 1;
      return base + c0 + (uint64_t)(i * 64) + (uint64_t)(__ffsll((unsigned long long)mm) - 1);
    }
    rr -= pc;
  }
  return LOC_NONE;
}

// Each half of the block takes its own tile (so two tiles' searches and
// loads are in flight per block); a wave reads two of the tile's chunks,
// 2 * IPT keys per lane.  The outputs are per tile and per chunk as if one
// wave had read each chunk.
template <typename KT, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void ip_count_kernel(InplaceArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;  // chunks per tile
  constexpr int HW = WAVES / 2;      // waves per half-block
  constexpr uint32_t TILE = BLOCK * IPT, SUB = 64 * IPT;
  __shared__ Seg s_seg[2];
  __shared__ uint32_t s_c[2][WAVES], s_fb[2][HW], s_lf[2][HW];
  __shared__ uint64_t s_acc[2][HW][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = wave / HW, hw = wave % HW;
  if (blockIdx.x == 0 && tid == 0) {
    // the previous step's finish lists have been consumed
    a.hdr->n_finish = 0;
    a.hdr->n_finish_small = 0;
    a.hdr->n_finish_tiny = 0;
    a.hdr->n_finish_med = 0;
  }
  const uint64_t pk = a.hdr->packed[a.level];
  const uint32_t S = (uint32_t)(pk >> 32), ntiles = (uint32_t)pk;
  for (uint32_t t0 = 2 * blockIdx.x; t0 < ntiles; t0 += 2 * gridDim.x) {
    const uint32_t t = t0 + (uint32_t)h;
    const bool valid = t < ntiles;
    if (hw == 0 && valid) {
      const uint32_t q = wave_search_le(S, [&](uint32_t i) { return a.live[i].tile0 <= t; });
      if (lane == 0) {
        s_seg[h] = a.live[q];
        a.tiles[t] = s_seg[h];
      }
    }
    __syncthreads();
    uint64_t start = 0, len = 0;
    uint32_t meta = 0, tile0 = t, cbase = 0, slot = 0;
    if (valid) {
      start = s_seg[h].start;
      len = s_seg[h].len;
      meta = s_seg[h].meta;
      tile0 = s_seg[h].tile0;
      cbase = s_seg[h].cbase;
      slot = s_seg[h].slot;
    }
    const uint32_t j = t - tile0;
    const int bit = (int)(meta & BIT_MASK);
    const uint64_t f = (uint64_t)flip_of(bit, a.w, a.mode, a.desc, (meta & META_SIGN) ? 1 : 0);
    const uint64_t lo = (uint64_t)j * TILE;
    const uint32_t cnt =
        valid ? (uint32_t)(len - lo < (uint64_t)TILE ? len - lo : (uint64_t)TILE) : 0u;
    const rsrc_t kr = make_rsrc(a.keys + start + lo, cnt * (uint32_t)sizeof(KT));
    KT key[2 * IPT];
#pragma unroll
    for (int i = 0; i < 2 * IPT; ++i) {
      const uint32_t q = (uint32_t)((2 * hw + i / IPT) * SUB + (i % IPT) * 64 + lane);
      key[i] = buf_load<KT>(kr, q * (uint32_t)sizeof(KT));
    }
    uint32_t c[2] = {0, 0}, fb = ~0u, lf = 0;
    uint64_t and_f = ~0ull, or_f = 0, and_b = ~0ull, or_b = 0;
#pragma unroll
    for (int i = 0; i < 2 * IPT; ++i) {
      const uint32_t q = (uint32_t)((2 * hw + i / IPT) * SUB + (i % IPT) * 64 + lane);
      const uint64_t k = (uint64_t)key[i];
      if (q < cnt) {
        if (((k >> bit) & 1ull) == f) {
          ++c[i / IPT];
          and_f &= k;
          or_f |= k;
          lf = q + 1;
        } else {
          and_b &= k;
          or_b |= k;
          fb = fb < q ? fb : q;
        }
      }
    }
    c[0] = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(c[0]), 63);
    c[1] = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_dpp(c[1]), 63);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const uint32_t ofb = (uint32_t)__shfl_xor((int)fb, d), olf = (uint32_t)__shfl_xor((int)lf, d);
      fb = ofb < fb ? ofb : fb;
      lf = olf > lf ? olf : lf;
    }
    and_f = wave_and_dpp(and_f);
    or_f = wave_or_dpp(or_f);
    and_b = wave_and_dpp(and_b);
    or_b = wave_or_dpp(or_b);
    if (lane == 0) {
      s_c[h][2 * hw] = c[0];
      s_c[h][2 * hw + 1] = c[1];
      s_fb[h][hw] = fb;
      s_lf[h][hw] = lf;
      s_acc[h][hw][0] = and_f;
      s_acc[h][hw][1] = or_f;
      s_acc[h][hw][2] = and_b;
      s_acc[h][hw][3] = or_b;
    }
    __syncthreads();
    const int ht = tid - h * (BLOCK / 2);  // thread index within the half
    if (valid && ht == 0) {
      uint32_t sum = 0, tfb = ~0u, tlf = 0;
      uint64_t af = ~0ull, of = 0, ab = ~0ull, ob = 0;
#pragma unroll
      for (int q = 0; q < WAVES; ++q) sum += s_c[h][q];
#pragma unroll
      for (int q = 0; q < HW; ++q) {
        tfb = tfb < s_fb[h][q] ? tfb : s_fb[h][q];
        tlf = tlf > s_lf[h][q] ? tlf : s_lf[h][q];
        af &= s_acc[h][q][0];
        of |= s_acc[h][q][1];
        ab &= s_acc[h][q][2];
        ob |= s_acc[h][q][3];
      }
      a.tcnt[cbase + j] = sum;
      a.ends[2ull * t] = tfb;
      a.ends[2ull * t + 1] = tlf;
      AccRep *z = &a.acc[tile0 + ACC_STRIDE * (j % acc_repl(len, TILE))];
      if (sum) {
        atomic_add_u32(&a.scnt[cbase + (j >> 6)], sum);
        atomic_add_u64(&a.split[slot], sum);
        atomic_and_u64(&z->and_lo, af);
        atomic_or_u64(&z->or_lo, of);
      }
      if (sum < cnt) {
        atomic_and_u64(&z->and_hi, ab);
        atomic_or_u64(&z->or_hi, ob);
      }
    }
    if (valid && ht < WAVES) a.sub[(uint64_t)t * WAVES + ht] = s_c[h][ht];
    __syncthreads();
  }
}

// One wave per tile: the sum of the group sums before the tile's group and
// of the tile counts before it within the group.
template <typename KT>
__global__ __launch_bounds__(256) void ip_prefix_kernel(InplaceArgs<KT> a) {
  const int lane = threadIdx.x & 63;
  const uint32_t ntiles = (uint32_t)a.hdr->packed[a.level];
  const uint32_t wpb = blockDim.x / 64;
  for (uint32_t t = blockIdx.x * wpb + (threadIdx.x >> 6); t < ntiles; t += gridDim.x * wpb) {
    const Seg s = a.tiles[t];
    const uint32_t j = t - s.tile0;
    uint32_t p = 0;
    for (uint32_t g = (uint32_t)lane; g < (j >> 6); g += 64) p += a.scnt[s.cbase + g];
    if ((uint32_t)lane < (j & 63u)) p += a.tcnt[s.cbase + (j & ~63u) + lane];
    p = (uint32_t)wave_sum_u64(p);
    if (lane == 0) a.pre[t] = p;
  }
}

// One wave per tile.  BLOCK and IPT are the count pass's shape (the tile
// and its chunks).
template <typename KT, int BLOCK, int IPT>
__global__ __launch_bounds__(256) void ip_locate_kernel(InplaceArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr uint32_t TILE = BLOCK * IPT;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wpb = blockDim.x / 64;
  const uint32_t ntiles = (uint32_t)a.hdr->packed[a.level];
  for (uint32_t t = blockIdx.x * wpb + (threadIdx.x >> 6); t < ntiles; t += gridDim.x * wpb) {
    const Seg sg = a.tiles[t];
    const uint64_t start = uni(sg.start), len = uni(sg.len);
    const uint32_t tile0 = uni(sg.tile0), j = t - tile0;
    const uint64_t F = uni(a.split[uni(sg.slot)]);
    const int bit = (int)(uni(sg.meta) & BIT_MASK);
    const uint64_t f =
        (uint64_t)flip_of(bit, a.w, a.mode, a.desc, (uni(sg.meta) & META_SIGN) ? 1 : 0);
    const uint64_t lo = (uint64_t)j * TILE;
    const uint32_t cnt = (uint32_t)(len - lo < (uint64_t)TILE ? len - lo : (uint64_t)TILE);
    // the tile's left part is [0, lend), its right part [lend, cnt)
    const uint32_t lend = lo < F ? (uint32_t)(F - lo < cnt ? F - lo : cnt) : 0u;
    const uint32_t fb = uni(a.ends[2ull * t]), lf = uni(a.ends[2ull * t + 1]);
    const uint32_t pre_t = uni(a.pre[t]);
    const uint32_t nt = (uint32_t)((len + TILE - 1) / TILE);
    uint64_t item[4] = {LOC_NONE, LOC_NONE, LOC_NONE, LOC_NONE};
    if (fb < lend) {
      // item at this tile's first back key left of k: rank r0 = back keys before the tile
      const uint64_t r0 = lo - pre_t;
      const uint32_t g = (uint32_t)(F - 1 - r0);  // front keys left of its partner
      const uint32_t i = wave_search_le(nt, [&](uint32_t x) { return a.pre[tile0 + x] <= g; });
      const uint64_t ilo = (uint64_t)i * TILE;
      const uint32_t icnt = (uint32_t)(len - ilo < (uint64_t)TILE ? len - ilo : (uint64_t)TILE);
      item[0] = start + lo + fb;
      item[1] = wave_select<KT, WAVES, IPT>(a.keys, start + ilo, icnt,
                                            &a.sub[(uint64_t)(tile0 + i) * WAVES],
                                            g - uni(a.pre[tile0 + i]), true, bit, f);
    }
    if (lf > lend) {
      // item at this tile's last front key right of k: rank r0 = front keys after the tile
      const uint64_t r0 = F - pre_t - uni(a.tcnt[uni(sg.cbase) + j]);
      const uint32_t nl = (uint32_t)((F + TILE - 1) / TILE);  // tiles with a left part
      const uint32_t jj = wave_search_le(
          nl, [&](uint32_t x) { return (uint64_t)x * TILE - a.pre[tile0 + x] <= r0; });
      const uint64_t jlo = (uint64_t)jj * TILE;
      const uint64_t aj = jlo - uni(a.pre[tile0 + jj]);
      if (aj != r0) {  // else the left tile's own item starts here
        const uint32_t jcnt = (uint32_t)(len - jlo < (uint64_t)TILE ? len - jlo : (uint64_t)TILE);
        item[2] = wave_select<KT, WAVES, IPT>(a.keys, start + jlo, jcnt,
                                              &a.sub[(uint64_t)(tile0 + jj) * WAVES],
                                              (uint32_t)(r0 - aj), false, bit, f);
        item[3] = start + lo + (lf - 1);
      }
    }
    if (lane == 0) {
      uint64_t *o = &a.items[4ull * t];
      o[0] = item[0];
      o[1] = item[1];
      o[2] = item[2];
      o[3] = item[3];
    }
  }
}

// Lists are built with coalesced loads: item position d = i * BLOCK + tid
// (row i of IPT), so position order is (row, wave, lane).  A key's rank in
// its list is the keys flagged in earlier (row, wave) slots -- one wave scan
// over the IPT * WAVES slot counts -- plus the flagged lanes below it.
template <typename KT, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void ip_swap_kernel(InplaceArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr int NS = IPT * WAVES;  // (row, wave) slots
  static_assert(NS <= 64, "one wave scans the slot counts");
  constexpr uint32_t TILE = BLOCK * IPT;
  static_assert(TILE <= 65536, "list offsets are 16-bit");
  __shared__ uint16_t s_a[TILE];  // back keys left of k: offsets from the item's left start
  __shared__ uint16_t s_b[TILE];  // front keys right of k: offsets left of its right start
  __shared__ uint32_t s_ca[NS], s_cb[NS];  // slot counts, then their exclusive prefixes
  __shared__ uint32_t s_n[2];              // list lengths
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t ntiles = (uint32_t)a.hdr->packed[a.level];
  for (uint32_t u = blockIdx.x; u < 2 * ntiles; u += gridDim.x) {
    const uint32_t t = u >> 1;
    const uint64_t ls = uni(a.items[4ull * t + 2 * (u & 1)]);
    const uint64_t rs = uni(a.items[4ull * t + 2 * (u & 1) + 1]);
    if (ls == LOC_NONE || rs == LOC_NONE) continue;
    const Seg sg = a.tiles[t];
    const uint64_t start = uni(sg.start);
    const uint64_t k = start + uni(a.split[uni(sg.slot)]);
    if (ls >= k || rs < k) {
      if (tid == 0) atomic_or_u32(&a.hdr->status, STATUS_BAD_COUNTS);
      continue;
    }
    const int bit = (int)(uni(sg.meta) & BIT_MASK);
    const uint64_t f =
        (uint64_t)flip_of(bit, a.w, a.mode, a.desc, (uni(sg.meta) & META_SIGN) ? 1 : 0);
    // left: [ls, end of ls's tile) below k; right: (start of rs's tile, rs] at or above k
    const uint64_t lte = start + ((ls - start) / TILE + 1) * TILE;
    const uint32_t ln = (uint32_t)((lte < k ? lte : k) - ls);
    const uint64_t rtb = start + ((rs - start) / TILE) * TILE;
    const uint32_t rn = (uint32_t)(rs + 1 - (rtb > k ? rtb : k));
    const rsrc_t kl = make_rsrc(a.keys + ls, ln * (uint32_t)sizeof(KT));
    // the right list runs leftwards from rs: offset d is at rs - d, so its
    // range starts rn - 1 keys left of rs and is read back to front
    const rsrc_t kr = make_rsrc(a.keys + (rs + 1 - rn), rn * (uint32_t)sizeof(KT));
    uint32_t ba = 0, bb = 0, ra[IPT], rb[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t d = (uint32_t)(i * BLOCK + tid);
      const uint64_t kA = (uint64_t)buf_load<KT>(kl, d * (uint32_t)sizeof(KT));
      const uint64_t kB = (uint64_t)buf_load<KT>(kr, (rn - 1 - d) * (uint32_t)sizeof(KT));
      const bool fa = d < ln && ((kA >> bit) & 1ull) != f;
      const bool fb = d < rn && ((kB >> bit) & 1ull) == f;
      const uint64_t ma = __ballot(fa), mb = __ballot(fb);
      ra[i] = lanes_below(ma);
      rb[i] = lanes_below(mb);
      ba |= (uint32_t)fa << i;
      bb |= (uint32_t)fb << i;
      if (lane == 0) {
        s_ca[i * WAVES + wave] = (uint32_t)__popcll(ma);
        s_cb[i * WAVES + wave] = (uint32_t)__popcll(mb);
      }
    }
    __syncthreads();
    if (wave < 2) {
      uint32_t *sc = wave ? s_cb : s_ca;
      const uint32_t v = lane < NS ? sc[lane] : 0u;
      const uint32_t inc = wave_incl_scan_dpp(v);
      if (lane < NS) sc[lane] = inc - v;
      if (lane == 63) s_n[wave] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint16_t d = (uint16_t)(i * BLOCK + tid);
      if ((ba >> i) & 1u) s_a[s_ca[i * WAVES + wave] + ra[i]] = d;
      if ((bb >> i) & 1u) s_b[s_cb[i * WAVES + wave] + rb[i]] = d;
    }
    const uint32_t na = s_n[0], nb = s_n[1];
    const uint32_t pairs = uni(na < nb ? na : nb);
    __syncthreads();
    for (uint32_t i = tid; i < pairs; i += BLOCK) {
      const uint64_t pa = ls + s_a[i], pb = rs - s_b[i];
      const KT ka = a.keys[pa], kb = a.keys[pb];
      a.keys[pa] = kb;
      a.keys[pb] = ka;
    }
    __syncthreads();
  }
}

// The same exchange with each lane taking IPT consecutive positions and
// block-wide scans for the ranks; faster than the coalesced form for 1- and
// 8-byte keys on MI355X.
template <typename KT, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void ip_swap_blocked_kernel(InplaceArgs<KT> a) {
  constexpr int WAVES = BLOCK / 64;
  constexpr uint32_t TILE = BLOCK * IPT;
  __shared__ uint32_t s_a[TILE];  // back keys left of k, from the item's left start
  __shared__ uint32_t s_b[TILE];  // front keys right of k, from its right start leftwards
  __shared__ uint32_t s_w[WAVES];
  const int tid = threadIdx.x;
  const uint32_t ntiles = (uint32_t)a.hdr->packed[a.level];
  for (uint32_t u = blockIdx.x; u < 2 * ntiles; u += gridDim.x) {
    const uint32_t t = u >> 1;
    const uint64_t ls = uni(a.items[4ull * t + 2 * (u & 1)]);
    const uint64_t rs = uni(a.items[4ull * t + 2 * (u & 1) + 1]);
    if (ls == LOC_NONE || rs == LOC_NONE) continue;
    const Seg sg = a.tiles[t];
    const uint64_t start = uni(sg.start);
    const uint64_t k = start + uni(a.split[uni(sg.slot)]);
    if (ls >= k || rs < k) {
      if (tid == 0) atomic_or_u32(&a.hdr->status, STATUS_BAD_COUNTS);
      continue;
    }
    const int bit = (int)(uni(sg.meta) & BIT_MASK);
    const uint64_t f =
        (uint64_t)flip_of(bit, a.w, a.mode, a.desc, (uni(sg.meta) & META_SIGN) ? 1 : 0);
    // left: [ls, end of ls's tile) below k; right: (start of rs's tile, rs] at or above k
    const uint64_t lte = start + ((ls - start) / TILE + 1) * TILE;
    const uint32_t ln = (uint32_t)((lte < k ? lte : k) - ls);
    const uint64_t rtb = start + ((rs - start) / TILE) * TILE;
    const uint32_t rn = (uint32_t)(rs + 1 - (rtb > k ? rtb : k));
    const rsrc_t kl = make_rsrc(a.keys + ls, ln * (uint32_t)sizeof(KT));
    uint32_t mb = 0, mf = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
      const uint32_t d = (uint32_t)(tid * IPT + q);
      const uint64_t key = (uint64_t)buf_load<KT>(kl, d * (uint32_t)sizeof(KT));
      if (d < ln && ((key >> bit) & 1ull) != f) mb |= 1u << q;
      if (d < rn) {
        const uint64_t kr = (uint64_t)a.keys[rs - d];
        if (((kr >> bit) & 1ull) == f) mf |= 1u << q;
      }
    }
    uint32_t na, nb;
    uint32_t ea = block_excl_scan<WAVES>((uint32_t)__builtin_popcount(mb), s_w, na);
    uint32_t eb = block_excl_scan<WAVES>((uint32_t)__builtin_popcount(mf), s_w, nb);
    for (uint32_t m = mb; m; m &= m - 1) s_a[ea++] = (uint32_t)(ls + tid * IPT + __builtin_ctz(m));
    for (uint32_t m = mf; m; m &= m - 1) s_b[eb++] = (uint32_t)(rs - (tid * IPT + __builtin_ctz(m)));
    const uint32_t pairs = uni(na < nb ? na : nb);
    __syncthreads();
    for (uint32_t i = tid; i < pairs; i += BLOCK) {
      const uint64_t pa = s_a[i], pb = s_b[i];
      const KT ka = a.keys[pa], kb = a.keys[pb];
      a.keys[pa] = kb;
      a.keys[pb] = ka;
    }
    __syncthreads();
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

// The same scatter staged through LDS.  A block owns a run of output
// positions that fits in LDS (S = SB / sizeof(ET) elements): m whole rows
// when a row fits (m = S / cols, "packed"), else one slice [s0, s0 + S) of
// one row.  It reads the indices and gradients that can land there in order
// (coalesced loads: its own m rows, or the slice's whole row), drops each
// value whose destination falls in its run into LDS and sets the
// destination's bit in an LDS bitmap, then writes the run out in order, only
// at marked positions: entries outside [0, cols) leave their output
// untouched, as in the direct kernel.  The random writes thus go to LDS and
// HBM sees whole lines.  A row of P > 1 slices is read P times; the blocks
// of one row's slices are then given consecutive dispatch slots of one XCD
// (blocks are dealt to the 8 XCDs round-robin; the grid is 8 ceil(units/8)),
// so they run together and the re-reads hit that XCD's L2.
//
// Work item w (0 <= w < units): packed (slices == 0), rows [w m, w m + m)
// clipped to rows; sliced, row w / slices, slice w % slices.  rcp_cols =
// 1 / cols in fp32, used to find the row of a packed position (exact after
// one correction, positions being below 2^17).
template <typename ET, bool I64, uint32_t SB, uint32_t BLOCK>
__global__ __launch_bounds__(BLOCK) void backward_staged_kernel(const ET *g, const void *idx,
                                                                uint64_t rows, uint64_t cols,
                                                                uint64_t m, uint64_t slices,
                                                                uint64_t units, float rcp_cols,
                                                                ET *out) {
  constexpr uint32_t S = SB / sizeof(ET);
  constexpr uint32_t U = 4;
  static_assert(S <= (1u << 17), "packed positions must stay below 2^17");
  __shared__ ET s_val[S];
  __shared__ uint32_t s_mark[S / 32];
  const uint32_t t = threadIdx.x;
  const uint64_t w = slices > 1 ? (blockIdx.x & 7) * ((units + 7) / 8) + (blockIdx.x >> 3)
                                 : (uint64_t)blockIdx.x;
  if (w >= units) return;
  const bool packed = slices == 0;
  uint64_t q0, in0, nin, s0 = 0;
  uint32_t len;
  if (packed) {
    const uint64_t r0 = w * m;
    const uint64_t mr = rows - r0 < m ? rows - r0 : m;
    q0 = in0 = r0 * cols;
    nin = mr * cols;
    len = (uint32_t)nin;
  } else {
    const uint64_t r = w / slices;
    s0 = (w - r * slices) * S;
    in0 = r * cols;
    q0 = in0 + s0;
    nin = cols;
    len = (uint32_t)(cols - s0 < S ? cols - s0 : S);
  }
  const uint32_t c32 = (uint32_t)cols;
  for (uint32_t i = t; i < (len + 31) / 32; i += BLOCK) s_mark[i] = 0;
  __syncthreads();
  const ET *gr = g + in0;
  auto dest = [&](uint64_t l) -> uint64_t {
    return I64 ? (uint64_t) static_cast<const int64_t *>(idx)[in0 + l]
               : (uint64_t) static_cast<const uint32_t *>(idx)[in0 + l];
  };
  // LDS position of input l with row-local destination d (>= len: none)
  auto target = [&](uint64_t l, uint64_t d) -> uint64_t {
    if (!packed) return d - s0;  // wraps above len when d < s0
    const uint32_t l32 = (uint32_t)l;
    uint32_t rr = (uint32_t)((float)l32 * rcp_cols);
    if (rr * c32 > l32) --rr;
    else if ((rr + 1) * c32 <= l32) ++rr;
    return d < cols ? (uint64_t)rr * cols + d : ~(uint64_t)0;
  };
  auto place = [&](uint64_t o, ET v) {
    if (o < len) {
      s_val[o] = v;
      atomicOr(&s_mark[o >> 5], 1u << (o & 31));
    }
  };
  uint64_t l = t;
  for (; l + (U - 1) * BLOCK < nin; l += U * BLOCK) {
    uint64_t d[U];
    ET v[U];
#pragma unroll
    for (uint32_t k = 0; k < U; ++k) {
      d[k] = dest(l + k * BLOCK);
      v[k] = gr[l + k * BLOCK];
    }
#pragma unroll
    for (uint32_t k = 0; k < U; ++k) place(target(l + k * BLOCK, d[k]), v[k]);
  }
  for (; l < nin; l += BLOCK) place(target(l, dest(l)), gr[l]);
  __syncthreads();
  ET *o = out + q0;
  for (uint32_t i = t; i < len; i += BLOCK)
    if ((s_mark[i >> 5] >> (i & 31)) & 1u) o[i] = s_val[i];
}

// ---------------------------------------------------------- payload gather

// Segment of position x: the last s < B with offsets[s] <= x, searched in
// [lo, hi].  With offsets that are not non-decreasing the answer is some s in
// [lo, hi]; every read stays inside offsets[0, B].
__device__ __forceinline__ uint64_t segment_of(const int64_t *offsets, uint64_t lo, uint64_t hi,
                                               uint64_t x) {
  while (lo < hi) {
    const uint64_t m = lo + (hi - lo + 1) / 2;
    if ((uint64_t)offsets[m] <= x) lo = m;
    else hi = m - 1;
  }
  return lo;
}

// Values that travel with the keys (a key-value sort, or any further tensor
// permuted like the keys): out[j] = values[base + idx[j]], base being 0 for
// a single array and the start of j's segment otherwise.  VT is the value
// word (1, 2, 4, 8 or 16 bytes), moved as raw bits.  A block takes chunks
// of GCH positions; thread 0 finds the segments of the chunk's first and
// last position, and each position searches only between them.  A source
// outside its segment (indices that are not a permutation) is skipped.
// With SCATTER the same pairs move the other way, out[base + idx[j]] =
// values[j]: the inverse permutation, which is the backward of a segmented
// sort or of the gather (targets outside their segment are skipped).
constexpr uint32_t GCH = 4096;
template <typename VT, bool I64, bool SCATTER = false>
__global__ __launch_bounds__(256) void gather_kernel(const VT *values, const void *indices,
                                                     const int64_t *offsets, uint64_t B,
                                                     uint64_t n, VT *out,
                                                     const uint32_t *status) {
  __shared__ uint64_t s_rng[2];
  // after a sort that rejected its offsets the indices are undefined: the
  // values are passed through unchanged
  if (!SCATTER && status && (*status & STATUS_BAD_OFFSETS)) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (uint64_t)gridDim.x * blockDim.x)
      out[j] = values[j];
    return;
  }
  for (uint64_t c0 = (uint64_t)blockIdx.x * GCH; c0 < n; c0 += (uint64_t)gridDim.x * GCH) {
    const uint64_t c1 = c0 + GCH < n ? c0 + GCH : n;
    uint64_t lo = 0, hi = 0;
    if (offsets) {
      if (threadIdx.x == 0) {
        s_rng[0] = segment_of(offsets, 0, B - 1, c0);
        s_rng[1] = segment_of(offsets, 0, B - 1, c1 - 1);
      }
      __syncthreads();
      lo = s_rng[0];
      hi = s_rng[1] < lo ? lo : s_rng[1];
      __syncthreads();
    }
    for (uint64_t j = c0 + threadIdx.x; j < c1; j += blockDim.x) {
      const uint64_t ix = I64 ? (uint64_t) static_cast<const int64_t *>(indices)[j]
                              : (uint64_t) static_cast<const uint32_t *>(indices)[j];
      uint64_t base = 0, len = n;
      if (offsets) {
        const uint64_t s = segment_of(offsets, lo, hi, j);
        base = (uint64_t)offsets[s];
        len = (uint64_t)offsets[s + 1] - base;
      }
      const uint64_t src = base + ix;
      if (ix < len && src < n) {
        if (SCATTER) out[src] = values[j];
        else out[j] = values[src];
      }
    }
  }
}

// ------------------------------------------------------------- bit layouts
//
// Keys whose order bits are not stored most significant first (a sign in
// the lowest bit, fields in another order): a layout lists, from the most
// significant order bit down, the stored bit that holds it.  The bits are
// gathered into that order, the keys sorted, and the bits put back.
struct BitLayout {
  uint8_t src[64];  // src[i]: stored bit of order bit w - 1 - i
};

template <typename KT>
__global__ void layout_kernel(KT *keys, uint64_t n, int w, BitLayout lay, int inverse) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = (uint64_t)keys[i];
    uint64_t out = 0;
    for (int j = 0; j < w; ++j) {
      const int ob = w - 1 - j, sb = lay.src[j];
      if (!inverse) out |= ((k >> sb) & 1ull) << ob;  // stored -> order
      else out |= ((k >> ob) & 1ull) << sb;            // order -> stored
    }
    keys[i] = (KT)out;
  }
}

// ------------------------------------------------------------ 128-bit keys
//
// A 128-bit key (low word first) is sorted most significant word first, as
// the method recurses on the lower bits within each part that agrees on the
// higher ones: the high words are sorted (the low words travel with them),
// the runs of equal high words become segments, and the low words are sorted
// within them.  Both sorts run on the rank word v of the key, whose bit b is
// 1 exactly when the key goes back in a split on bit b (Algorithms 1 and 3-5
// with the direction rules of Section III), so the words are sorted as
// unsigned in ascending order.

__device__ __forceinline__ void rank_word128(uint64_t &lo, uint64_t &hi, int mode, int desc) {
  const uint64_t top = 1ull << 63;
  uint64_t ml = desc ? ~0ull : 0ull, mh = ml;
  if (mode != MODE_U) mh ^= top;
  if (mode == MODE_F && (hi & top)) {
    ml = ~ml;
    mh ^= ~top;
  }
  lo ^= ml;
  hi ^= mh;
}

__global__ void wide_split_kernel(const uint64_t *keys, uint64_t n, int mode, int desc,
                                  uint64_t *hi, uint64_t *lo) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t l = keys[2 * i], h = keys[2 * i + 1];
    rank_word128(l, h, mode, desc);
    lo[i] = l;
    hi[i] = h;
  }
}

// Keys back from sorted rank words: the rank word is the key with bits
// flipped by a mask that depends only on the sign, so flipping again by the
// mask of the key's sign restores it.
__global__ void wide_merge_kernel(const uint64_t *hi, const uint64_t *lo, uint64_t n, int mode,
                                  int desc, uint64_t *keys) {
  const uint64_t top = 1ull << 63;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t l = lo[i], h = hi[i];
    if (desc) {
      l = ~l;
      h = ~h;
    }
    if (mode == MODE_I) {
      h ^= top;
    } else if (mode == MODE_F) {
      if (h & top) {
        h ^= top;  // was a non-negative key
      } else {
        l = ~l;  // was negative: every bit was flipped
        h = ~h;
      }
    }
    keys[2 * i] = l;
    keys[2 * i + 1] = h;
  }
}

// Segments of the low-word sort: offs[j] = start of the run of equal high
// words holding position j (a prefix maximum of the run starts), offs[n] =
// n.  Segment j is then [offs[j], offs[j + 1]): empty inside a run, the
// whole run at its last position.  Three steps: a maximum within each block
// of RCH positions, an exclusive maximum over the blocks, and the final
// maximum of both.
constexpr uint32_t RCH = 4096;
__global__ __launch_bounds__(256) void run_start_local_kernel(const uint64_t *hi, uint64_t n,
                                                              int64_t *offs, int64_t *bmax) {
  __shared__ int64_t s_m[256];
  constexpr uint32_t PER = RCH / 256;
  const uint64_t b0 = (uint64_t)blockIdx.x * RCH;
  const uint64_t t0 = b0 + (uint64_t)threadIdx.x * PER;
  int64_t m = 0;
  for (uint32_t k = 0; k < PER; ++k) {
    const uint64_t j = t0 + k;
    if (j < n && (j == 0 || hi[j] != hi[j - 1])) m = (int64_t)j;
  }
  s_m[threadIdx.x] = m;
  __syncthreads();
  // inclusive maximum scan over the threads (Hillis-Steele)
  for (int d = 1; d < 256; d <<= 1) {
    const int64_t o = threadIdx.x >= (unsigned)d ? s_m[threadIdx.x - d] : 0;
    __syncthreads();
    if (o > s_m[threadIdx.x]) s_m[threadIdx.x] = o;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? s_m[threadIdx.x - 1] : 0;
  for (uint32_t k = 0; k < PER; ++k) {
    const uint64_t j = t0 + k;
    if (j < n) {
      if (j == 0 || hi[j] != hi[j - 1]) run = (int64_t)j;
      offs[j] = run;
    }
  }
  if (threadIdx.x == 255) bmax[blockIdx.x] = s_m[255];
}

__global__ __launch_bounds__(1024) void run_start_blocks_kernel(int64_t *bmax, uint64_t nb) {
  // exclusive maximum over the block maxima, one block, PER blocks a thread
  __shared__ int64_t s_m[1024];
  const uint64_t per = (nb + 1023) / 1024;
  const uint64_t t0 = (uint64_t)threadIdx.x * per;
  int64_t m = 0;
  for (uint64_t k = 0; k < per; ++k)
    if (t0 + k < nb && bmax[t0 + k] > m) m = bmax[t0 + k];
  s_m[threadIdx.x] = m;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t o = threadIdx.x >= (unsigned)d ? s_m[threadIdx.x - d] : 0;
    __syncthreads();
    if (o > s_m[threadIdx.x]) s_m[threadIdx.x] = o;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? s_m[threadIdx.x - 1] : 0;
  for (uint64_t k = 0; k < per; ++k) {
    if (t0 + k < nb) {
      const int64_t v = bmax[t0 + k];
      bmax[t0 + k] = run;
      if (v > run) run = v;
    }
  }
}

__global__ void run_start_final_kernel(int64_t *offs, const int64_t *bexc, uint64_t n) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n;
       j += (uint64_t)gridDim.x * blockDim.x) {
    if (j == n) {
      offs[n] = (int64_t)n;
    } else {
      const int64_t e = bexc[j / RCH];
      if (e > offs[j]) offs[j] = e;
    }
  }
}

}  // namespace bsort
