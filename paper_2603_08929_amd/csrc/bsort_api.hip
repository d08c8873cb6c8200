// Host side of libbsort: argument validation, scratch layout and the launch
// sequence behind the C ABI declared in include/bsort.h.
//
// One call enqueues, on the caller's stream and without any host readback:
//   init   -- zero the work-list counters and the per-tile count arrays
//   (validate offsets, segmented calls only)
//   seed   -- level-0 work lists: each user segment is split on its top bit
//             (the first pass of Algorithms 2-4) or finished in LDS
//   w x { count, level, plan } -- one breadth-first level of the recursion
//             each: tile map and missing per-tile counts, the split pass,
//             then the children's lists
//   copy   -- large retired segments not yet in the caller's buffer
//   finish -- small segments: all remaining bits in LDS, final write
// Grids are sized from upper bounds; the kernels read their real work from
// device memory and loop until it is exhausted.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "bsort.h"
#include "bsort_kernels.hpp"

using namespace bsort;

namespace {

thread_local char g_hip_err[256] = "";

// Benchmark instrumentation: hipEvent pairs around level-kernel launches.
struct Timing {
  int armed = 0;
  int cap = 0;
  int count = 0;
  hipEvent_t *ev = nullptr;
  int *lvl = nullptr;
};
Timing g_timing;
thread_local int g_capturing = 0;  // set while a call is recorded into a graph

void timing_free() {
  if (g_timing.ev) {
    for (int i = 0; i < 2 * g_timing.cap; ++i) (void)hipEventDestroy(g_timing.ev[i]);
    delete[] g_timing.ev;
    delete[] g_timing.lvl;
  }
  g_timing = Timing();
}

int hip_fail(hipError_t e, const char *what) {
  snprintf(g_hip_err, sizeof g_hip_err, "%s: %s", what, hipGetErrorString(e));
  return BSORT_EHIP;
}

struct DevState {
  int checked;
  int ok;
  int cus;
};
DevState g_dev[64];

int device_check(int *cus, int *device = nullptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return BSORT_ENODEV;
  DevState &d = g_dev[dev];
  if (!d.checked) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    d.ok = strncmp(p.gcnArchName, "gfx950", 6) == 0;
    d.cus = p.multiProcessorCount;
    d.checked = 1;
  }
  if (!d.ok) return BSORT_ENODEV;
  *cus = d.cus;
  if (device) *device = dev;
  return BSORT_OK;
}

// Launch configurations.  A configuration fixes the level tile (one wave
// of 64 lanes x LIPT keys), the finish kernel's block and threshold (T =
// FB * FIPT keys) and the grids (every resident workgroup, or half).
// Configuration 0 is the default; bsort_autotune times all of them on the
// caller's data and remembers the fastest per key width, index mode and
// size class.
constexpr int N_LEVEL_SHAPES = 2, N_FINISH_SHAPES = 3, N_GRIDS = 2;
constexpr int N_CONFIGS = N_LEVEL_SHAPES * N_FINISH_SHAPES * N_GRIDS;

// The in-place path's tile: a 512-thread workgroup.
template <typename KT>
struct InplaceShape {
  static constexpr int LB = 512;
  static constexpr int LIPT = sizeof(KT) == 8 ? 4 : 8;
  static constexpr uint32_t TILE = LB * LIPT;
};
template <typename KT, int V>
struct FinishShape {
  static constexpr int FB = V == 1 ? 256 : 512;
  static constexpr int FIPT = (V == 2 ? 8 : 16) / (sizeof(KT) == 8 ? 2 : 1);
  static constexpr uint32_t TFIN = FB * FIPT;
};

// The finish shape for segments of at most T keys: one wave.
template <typename KT>
struct SmallFinish {
  static constexpr int B = 64;
  static constexpr int IPT = sizeof(KT) == 8 ? 4 : 8;
  static constexpr uint32_t T = B * IPT;
};

struct TinyFinish {
  static constexpr int B = 64;
  static constexpr int IPT = 1;
  static constexpr uint32_t T = 64;
};

struct Config {
  int lv, fv, grid;  // level shape, finish shape, grid (0 full, 1 half)
};
Config config_of(int id) { return Config{id / 6, (id / 2) % 3, id % 2}; }
constexpr int CONFIG_DRY_RUN = -2;  // validate the arguments and the device, launch nothing

// Level tile of a configuration's level shape (the smaller one is lv = 1).
constexpr uint32_t tile_of(int key_bytes, int lv) {
  return 64u * ((lv == 0 ? 16u : 8u) / (key_bytes == 8 ? 2u : 1u));
}
static_assert(tile_of(1, 0) == LevelShape<uint8_t, 0>::TILE &&
                  tile_of(2, 1) == LevelShape<uint16_t, 1>::TILE &&
                  tile_of(4, 0) == LevelShape<uint32_t, 0>::TILE &&
                  tile_of(8, 0) == LevelShape<uint64_t, 0>::TILE &&
                  tile_of(8, 1) == LevelShape<uint64_t, 1>::TILE,
              "layout tile and launch tile agree");
uint32_t inplace_tile_of(int key_bytes) { return 512u * (key_bytes == 8 ? 4u : 8u); }
uint32_t tfin_of(int key_bytes, int fv) {
  const uint32_t fb = fv == 1 ? 256 : 512;
  return fb * ((fv == 2 ? 8 : 16) / (key_bytes == 8 ? 2 : 1));
}

constexpr uint32_t ALL_FLAGS =
    BSORT_DESCENDING | BSORT_NO_SKIP | BSORT_NO_FINISH | BSORT_IDX64 | BSORT_KEYS_UNCHANGED;

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch layout.  The header sits at offset 0 (bsort_device_status reads
// it there).  Bounds: a live segment holds more than T keys (more than
// TINY_MAX with BSORT_NO_FINISH, whose tiny lists hold the parts of 2 to
// TINY_MAX keys); a level's tiles are at most n/TILE + segments;
// every parent yields at most two finish entries per level; copy entries
// hold more than T keys each.  The level kernel reads the per-tile prefix
// words and the chunk carries through one buffer descriptor with 32-bit
// offsets (`meta` bytes from the start of pc).
struct Layout {
  size_t hdr, cnts, segs[2], acc[2], split[2], tmap, pc, agg, carry, fin, fins, fint, finm, cpy,
      tiny[2], meta, keys1, idx0, idx1, keys0, total;
  uint64_t smax, tnmax, tmax, fmax, cmax, cn, nchunks;
};

bool make_layout(int key_bytes, uint64_t n, uint64_t B, bool with_idx, uint32_t flags,
                 uint32_t tile, uint32_t tfin, Layout *L) {
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return false;
  const uint64_t w = 8ull * key_bytes;
  const bool no_finish = (flags & BSORT_NO_FINISH) != 0;
  // without the LDS finish, parts of at most TINY_MAX keys go to the tiny
  // lists (each entry at least 2 keys), so a live segment holds more
  L->smax = (no_finish ? n / (TINY_MAX + 1ull) : n / (tfin + 1ull)) + 1;
  L->tnmax = no_finish ? n / 2 + 1 : 0;
  L->tmax = n / tile + L->smax + 1;
  const uint64_t fb = B + 2 * w * L->smax + 1;
  L->fmax = (fb < n + 1 ? fb : n + 1);
  L->cmax = n / (tfin + 1ull) + 1;
  // next-level front counts per tile, two level parities: child c of a
  // parent with tiles [tile0, tile0 + nt) counts at 2 tile0 + c nt + j
  L->cn = 2 * L->tmax + 1;
  L->nchunks = L->tmax / PREP_TILES + 1;
  size_t off = 0;
  L->hdr = off; off = up256(off + sizeof(Header));
  L->cnts = off; off = up256(off + 2 * L->cn * 4);
  for (int i = 0; i < 2; ++i) { L->segs[i] = off; off = up256(off + L->smax * sizeof(Seg)); }
  for (int i = 0; i < 2; ++i) { L->acc[i] = off; off = up256(off + L->tmax * sizeof(AccRep)); }
  for (int i = 0; i < 2; ++i) { L->split[i] = off; off = up256(off + L->smax * 8); }
  L->tmap = off; off = up256(off + L->tmax * sizeof(Seg));
  L->agg = off; off = up256(off + L->nchunks * 8);
  L->pc = off; off = up256(off + L->tmax * 8);
  L->carry = off; off = up256(off + L->nchunks * 8);
  L->meta = off - L->pc;  // bytes of pc and carry, read through one 32-bit descriptor
  L->fin = off; off = up256(off + L->fmax * sizeof(Seg));
  L->fins = off; off = up256(off + L->fmax * sizeof(Seg));
  L->fint = off; off = up256(off + L->fmax * sizeof(Seg));
  L->finm = off; off = up256(off + L->fmax * sizeof(Seg));
  L->cpy = off; off = up256(off + L->cmax * sizeof(Seg));
  // without the LDS finish: the tiny-segment lists of two level parities
  L->tiny[0] = L->tiny[1] = 0;
  if (no_finish)
    for (int i = 0; i < 2; ++i) { L->tiny[i] = off; off = up256(off + L->tnmax * sizeof(TinySeg)); }
  L->keys1 = off; off = up256(off + n * (size_t)key_bytes);
  L->idx0 = L->idx1 = 0;
  if (with_idx) {
    if (flags & BSORT_IDX64) { L->idx0 = off; off = up256(off + n * 4); }
    L->idx1 = off; off = up256(off + n * 4);
  }
  // BSORT_KEYS_UNCHANGED: the keys are sorted in a copy
  L->keys0 = 0;
  if (flags & BSORT_KEYS_UNCHANGED) { L->keys0 = off; off = up256(off + n * (size_t)key_bytes); }
  L->total = off;
  return L->meta < (1ull << 32);
}

template <typename K>
int occupancy(K kernel, int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

uint32_t clamp_grid(uint64_t want, uint64_t cap) {
  if (want < 1) want = 1;
  if (cap < 1) cap = 1;
  return (uint32_t)(want < cap ? want : cap);
}

template <typename KT, bool IDX, int LV, int FV>
int launch_all(KT *keys, uint64_t n, const int64_t *offsets, uint64_t B, int mode,
               uint32_t flags, void *indices, char *scr, const Layout &L, int cus, int half,
               hipStream_t st, int stop) {
  using LS = LevelShape<KT, LV>;
  using FS = FinishShape<KT, FV>;
  const uint64_t gdiv = half ? 2 : 1;
  const int w = 8 * (int)sizeof(KT);
  const int desc = (flags & BSORT_DESCENDING) ? 1 : 0;
  const int idx64 = (IDX && (flags & BSORT_IDX64)) ? 1 : 0;
  const int no_skip = (flags & BSORT_NO_SKIP) ? 1 : 0;
  const int no_finish = (flags & BSORT_NO_FINISH) ? 1 : 0;

  Header *hdr = reinterpret_cast<Header *>(scr + L.hdr);
  Seg *segs[2] = {reinterpret_cast<Seg *>(scr + L.segs[0]),
                  reinterpret_cast<Seg *>(scr + L.segs[1])};
  AccRep *acc[2] = {reinterpret_cast<AccRep *>(scr + L.acc[0]),
                    reinterpret_cast<AccRep *>(scr + L.acc[1])};
  uint64_t *split[2] = {reinterpret_cast<uint64_t *>(scr + L.split[0]),
                        reinterpret_cast<uint64_t *>(scr + L.split[1])};
  Seg *tmap = reinterpret_cast<Seg *>(scr + L.tmap);
  uint2 *pc = reinterpret_cast<uint2 *>(scr + L.pc);
  uint64_t *agg = reinterpret_cast<uint64_t *>(scr + L.agg);
  uint64_t *carry = reinterpret_cast<uint64_t *>(scr + L.carry);
  Seg *fin = reinterpret_cast<Seg *>(scr + L.fin);
  Seg *fins = reinterpret_cast<Seg *>(scr + L.fins);
  Seg *fint = reinterpret_cast<Seg *>(scr + L.fint);
  Seg *finm = reinterpret_cast<Seg *>(scr + L.finm);
  Seg *cpy = reinterpret_cast<Seg *>(scr + L.cpy);
  KT *kbuf[2] = {keys, reinterpret_cast<KT *>(scr + L.keys1)};
  uint32_t *ibuf[2] = {nullptr, nullptr};
  if (IDX) {
    ibuf[0] = idx64 ? reinterpret_cast<uint32_t *>(scr + L.idx0)
                    : static_cast<uint32_t *>(indices);
    ibuf[1] = reinterpret_cast<uint32_t *>(scr + L.idx1);
  }

  const uint64_t cap = (uint64_t)cus * 16;
  uint32_t *cnt_base = reinterpret_cast<uint32_t *>(scr + L.cnts);
  const uint64_t cn = L.cn;  // entries per count array
  uint32_t *cnt[2] = {cnt_base, cnt_base + cn};
  hipLaunchKernelGGL(init_kernel, dim3(clamp_grid((2 * cn + 255) / 256, 2048)), dim3(256), 0,
                     st, hdr, cnt_base, 2 * cn);
  if (offsets)
    hipLaunchKernelGGL(validate_kernel, dim3(clamp_grid((B + 256) / 256, 1024)), dim3(256), 0,
                       st, offsets, B, n, hdr);

  ListArgs la;
  la.hdr = hdr;
  la.fin = fin;
  la.fin_small = fins;
  la.fin_tiny = fint;
  la.fin_med = finm;
  la.cpy = cpy;
  la.tile = LS::TILE;
  la.t_fin = FS::TFIN;
  la.t_small = SmallFinish<KT>::T;
  la.t_tiny = TinyFinish::T;
  la.t_med = FS::TFIN / 2;
  la.recount = (uint32_t)(2 * L.tmax);  // never read: the prep pass counts such segments
  la.tiny_next = nullptr;
  TinySeg *tiny[2] = {nullptr, nullptr};
  if (no_finish) {
    tiny[0] = reinterpret_cast<TinySeg *>(scr + L.tiny[0]);
    tiny[1] = reinterpret_cast<TinySeg *>(scr + L.tiny[1]);
  }

  SeedArgs sa;
  sa.l = la;
  sa.l.live_next = segs[0];
  sa.l.acc_next = acc[0];
  sa.l.split_next = split[0];
  sa.l.next_level = 0;
  sa.l.tiny_next = tiny[0];
  sa.offsets = offsets;
  sa.B = B;
  sa.n = n;
  sa.w = w;
  sa.with_idx = IDX ? 1 : 0;
  sa.no_finish = no_finish;
  sa.idx_final = indices;
  sa.idx64 = idx64;
  hipLaunchKernelGGL(seed_kernel, dim3(clamp_grid((B + 255) / 256, cap)), dim3(256), 0, st, sa);

  auto lk = level_kernel<KT, IDX, LS::LIPT>;
  static const int occ_level = occupancy(lk, 256);
  const uint32_t lgrid = clamp_grid((L.tmax + 3) / 4, (uint64_t)cus * occ_level / gdiv);
  const uint32_t pgrid = clamp_grid((L.smax + 255) / 256, cap);
  auto pk = prep_kernel<KT, LS::LIPT>;
  const uint32_t cgrid = clamp_grid(L.nchunks, L.nchunks);
  // A single array that fits the LDS finish never has a live segment: the
  // seed hands it straight to the finish, so the level passes and the copy
  // would all find empty lists.
  int levels = (!offsets && !no_finish && n <= FS::TFIN) ? 0 : w;
  // a stop before the last level: the level-`stop` live segments are
  // written out as they stand (bsort_levels)
  const bool snapshot = stop < levels;
  if (snapshot) levels = stop;

  // the arguments of level lvl's three kernels (they alternate by parity)
  auto level_args = [&](int lvl, PrepArgs<KT> &ca, LevelArgs<KT> &a, PlanArgs &pa) {
    ca.keys[0] = kbuf[0];
    ca.keys[1] = kbuf[1];
    ca.live = segs[lvl & 1];
    ca.tmap = tmap;
    ca.pc = pc;
    ca.agg = agg;
    ca.carry = carry;
    ca.cnt_in = cnt[lvl & 1];
    ca.hdr = hdr;
    ca.w = w;
    ca.mode = mode;
    ca.desc = desc;
    ca.level = lvl;

    a.keys[0] = kbuf[0];
    a.keys[1] = kbuf[1];
    a.idx[0] = ibuf[0];
    a.idx[1] = ibuf[1];
    a.tmap = tmap;
    a.meta = scr + L.pc;
    a.off.pc = 0;
    a.off.carry = (uint32_t)(L.carry - L.pc);
    a.off.range = (uint32_t)L.meta;
    a.acc = acc[lvl & 1];
    a.split = split[lvl & 1];
    a.hdr = hdr;
    a.cnt_out = cnt[(lvl + 1) & 1];
    a.w = w;
    a.mode = mode;
    a.desc = desc;
    a.level = lvl;

    pa.l = la;
    pa.l.live_next = segs[(lvl + 1) & 1];
    pa.l.acc_next = acc[(lvl + 1) & 1];
    pa.l.split_next = split[(lvl + 1) & 1];
    pa.l.tiny_next = tiny[(lvl + 1) & 1];
    pa.l.next_level = lvl + 1;
    pa.live = segs[lvl & 1];
    pa.acc = acc[lvl & 1];
    pa.split = split[lvl & 1];
    pa.zero_a = cnt[lvl & 1];  // read by this level's prep, filled by the next level
    pa.zero_b = nullptr;
    pa.zero_n = cn;
    pa.zero_per_tile = 2;
    pa.level = lvl;
    pa.w = w;
    pa.with_idx = IDX ? 1 : 0;
    pa.idx64 = idx64;
    pa.no_skip = no_skip;
    pa.no_finish = no_finish;
    pa.inplace = 0;
  };

  // the tiny-segment pass of a level (without the LDS finish), or the
  // write-out of a stopped sort's tiny segments
  auto tiny_args = [&](int lvl, int snap) {
    TinyArgs<KT> ta;
    ta.keys[0] = kbuf[0];
    ta.keys[1] = kbuf[1];
    ta.idx[0] = ibuf[0];
    ta.idx[1] = ibuf[1];
    ta.keys_final = keys;
    ta.idx_final = indices;
    ta.list = tiny[lvl & 1];
    ta.l = la;
    ta.l.tiny_next = tiny[(lvl + 1) & 1];
    ta.l.next_level = lvl + 1;
    ta.level = lvl;
    ta.w = w;
    ta.mode = mode;
    ta.desc = desc;
    ta.idx64 = idx64;
    ta.snapshot = snap;
    return ta;
  };
  // the tiny pass: one resident round of workgroups (a second, partial
  // round would leave most of the chip idle at its end)
  static const int occ_tsp = occupancy(tiny_kernel<KT, IDX>, 256);
  const uint32_t tsgrid = clamp_grid((L.tnmax + 255) / 256, (uint64_t)cus * occ_tsp);

  // Levels below `first_tail` are launched one kernel per phase; the rest
  // run in one tail launch, which ends at the first empty level (its live
  // levels run at lower occupancy than a level launch, so the depth leaves
  // room for skewed data).  Parts of uniform keys reach the finish size
  // after about log2(n / T) levels (T = finish size); six more levels cover
  // the skew of normal floats and presorted runs.  Below 2^22 keys a live
  // tail level is cheap and the launches are most of the cost: one more.
  int first_tail = levels;
  if (!no_finish && !snapshot) {
    const uint64_t parts = (n + FS::TFIN - 1) / FS::TFIN;
    const int depth = parts > 1 ? 64 - __builtin_clzll(parts - 1) : 0;  // ceil(log2(parts))
    const int margin = n >= (1ull << 22) ? 6 : 1;
    first_tail = depth + margin < levels ? depth + margin : levels;
  }
  for (int lvl = 0; lvl < first_tail; ++lvl) {
    PrepArgs<KT> ca;
    LevelArgs<KT> a;
    PlanArgs pa;
    level_args(lvl, ca, a, pa);
    hipLaunchKernelGGL(pk, dim3(cgrid), dim3(256), 0, st, ca);
    const bool timed = g_timing.armed && !g_capturing && g_timing.count < g_timing.cap;
    if (timed) {
      // the events take the kernel's own start and end times from its
      // dispatch: no marker packets between the launches
      hipExtLaunchKernelGGL(lk, dim3(lgrid), dim3(256), 0, st, g_timing.ev[2 * g_timing.count],
                            g_timing.ev[2 * g_timing.count + 1], 0u, a);
      g_timing.lvl[g_timing.count++] = lvl;
    } else {
      hipLaunchKernelGGL(lk, dim3(lgrid), dim3(256), 0, st, a);
    }
    hipLaunchKernelGGL(plan_kernel, dim3(pgrid), dim3(256), 0, st, pa);
    if (no_finish) {
      TinyArgs<KT> ta = tiny_args(lvl, 0);
      hipLaunchKernelGGL((tiny_kernel<KT, IDX>), dim3(tsgrid), dim3(256), 0, st, ta);
    }
  }
  if (first_tail < levels) {
    TailArgs<KT> ta;
    level_args(first_tail, ta.prep0, ta.lvl0, ta.plan0);
    level_args(first_tail + 1, ta.prep1, ta.lvl1, ta.plan1);
    ta.hdr = hdr;
    ta.first = first_tail;
    ta.last = levels;
    auto tk = tail_kernel<KT, IDX, LS::LIPT>;
    // every workgroup resident at once: the barriers wait for all of them
    static const int occ_tail = occupancy(tk, 256);
    hipLaunchKernelGGL(tk, dim3((uint32_t)(cus * occ_tail)), dim3(256), 0, st, ta);
  }

  if (snapshot) {
    SnapArgs<KT> sn;
    sn.keys_buf[0] = kbuf[0];
    sn.keys_buf[1] = kbuf[1];
    sn.idx_buf[0] = ibuf[0];
    sn.idx_buf[1] = ibuf[1];
    sn.keys_final = keys;
    sn.idx_final = indices;
    sn.live = segs[levels & 1];
    sn.hdr = hdr;
    sn.level = levels;
    sn.tile = LS::TILE;
    sn.idx64 = idx64;
    hipLaunchKernelGGL((snapshot_kernel<KT, IDX>), dim3(lgrid), dim3(256), 0, st, sn);
    if (no_finish) {
      TinyArgs<KT> ta = tiny_args(levels, 1);
      hipLaunchKernelGGL((tiny_kernel<KT, IDX>), dim3(tsgrid), dim3(256), 0, st, ta);
    }
  }

  CopyArgs<KT> ca;
  ca.keys_buf[0] = kbuf[0];
  ca.keys_buf[1] = kbuf[1];
  ca.idx_buf[0] = ibuf[0];
  ca.idx_buf[1] = ibuf[1];
  ca.keys_final = keys;
  ca.idx_final = indices;
  ca.list = cpy;
  ca.hdr = hdr;
  ca.idx64 = idx64;
  if (levels > 0)
    hipLaunchKernelGGL((copy_kernel<KT, IDX>), dim3(clamp_grid(cus * 4, cap)), dim3(256), 0, st,
                       ca);

  FinishArgs<KT> fa;
  fa.keys_buf[0] = kbuf[0];
  fa.keys_buf[1] = kbuf[1];
  fa.idx_buf[0] = ibuf[0];
  fa.idx_buf[1] = ibuf[1];
  fa.keys_final = keys;
  fa.idx_final = indices;
  fa.list = fin;
  fa.hdr = hdr;
  fa.w = w;
  fa.mode = mode;
  fa.desc = desc;
  fa.idx64 = idx64;
  fa.no_skip = no_skip;
  fa.count = &hdr->n_finish;
  auto fk = finish_kernel<KT, IDX, FS::FB, FS::FIPT>;
  static const int occ_fin = occupancy(fk, FS::FB);
  const uint32_t fgrid = clamp_grid(L.fmax, (uint64_t)cus * occ_fin / gdiv);
  hipLaunchKernelGGL(fk, dim3(fgrid), dim3(FS::FB), 0, st, fa);
  // segments of at most SmallFinish::T keys: one wave each
  using SF = SmallFinish<KT>;
  FinishArgs<KT> fs = fa;
  fs.list = fins;
  fs.count = &hdr->n_finish_small;
  auto sk = finish_kernel<KT, IDX, SF::B, SF::IPT>;
  static const int occ_small = occupancy(sk, SF::B);
  const uint32_t sgrid = clamp_grid(L.fmax, (uint64_t)cus * occ_small / gdiv);
  hipLaunchKernelGGL(sk, dim3(sgrid), dim3(SF::B), 0, st, fs);
  // segments of at most half the full shape: half the keys per lane
  FinishArgs<KT> fm = fa;
  fm.list = finm;
  fm.count = &hdr->n_finish_med;
  auto mk = finish_kernel<KT, IDX, FS::FB, FS::FIPT / 2>;
  static const int occ_med = occupancy(mk, FS::FB);
  const uint32_t mgrid = clamp_grid(L.fmax, (uint64_t)cus * occ_med / gdiv);
  hipLaunchKernelGGL(mk, dim3(mgrid), dim3(FS::FB), 0, st, fm);
  // segments of at most 64 keys: one key per lane
  FinishArgs<KT> ft = fa;
  ft.list = fint;
  ft.count = &hdr->n_finish_tiny;
  auto tk = finish_kernel<KT, IDX, TinyFinish::B, TinyFinish::IPT>;
  static const int occ_tiny = occupancy(tk, TinyFinish::B);
  const uint32_t tgrid = clamp_grid(L.fmax, (uint64_t)cus * occ_tiny / gdiv);
  hipLaunchKernelGGL(tk, dim3(tgrid), dim3(TinyFinish::B), 0, st, ft);

  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BSORT_OK;
}

// Configuration choice: a process-wide override (tests), else what the
// autotuner found for this device, key width, index mode and size class
// (log2 of the mean segment length), else configuration 0.
int g_override = -1;
signed char g_tuned[64][4][2][48];  // configuration + 1; 0 = not tuned

int kb_slot(int key_bytes) { return key_bytes == 1 ? 0 : key_bytes == 2 ? 1 : key_bytes == 4 ? 2 : 3; }
int size_class(uint64_t n, uint64_t B) {
  const uint64_t mean = n / (B ? B : 1);
  const int c = 63 - __builtin_clzll(mean | 1);
  return c < 47 ? c : 47;
}
int choose_config(int dev, int key_bytes, bool with_idx, uint64_t n, uint64_t B) {
  if (g_override >= 0) return g_override;
  const int t = g_tuned[dev][kb_slot(key_bytes)][with_idx ? 1 : 0][size_class(n, B)];
  return t > 0 ? t - 1 : 0;
}

template <typename KT, bool IDX>
int launch_cfg(const Config &c, KT *k, uint64_t n, const int64_t *off, uint64_t b, int mode,
               uint32_t flags, void *indices, char *scr, const Layout &L, int cus,
               hipStream_t st, int stop) {
#define BSORT_CFG(LV, FV)                                                                    \
  case LV * 3 + FV:                                                                          \
    return launch_all<KT, IDX, LV, FV>(k, n, off, b, mode, flags, indices, scr, L, cus,      \
                                       c.grid, st, stop)
  switch (c.lv * 3 + c.fv) {
    BSORT_CFG(0, 0);
    BSORT_CFG(0, 1);
    BSORT_CFG(0, 2);
    BSORT_CFG(1, 0);
    BSORT_CFG(1, 1);
    BSORT_CFG(1, 2);
    default: return BSORT_EINVAL;
  }
#undef BSORT_CFG
}

template <typename KT>
int run(void *keys, uint64_t n, const int64_t *offsets, uint64_t B, bool segmented, int mode,
        uint32_t flags, void *indices, void *scratch, size_t scratch_bytes, void *stream,
        int force_config, int stop) {
  if (flags & ~ALL_FLAGS) return BSORT_EINVAL;
  if (segmented && B > 0 && !offsets) return BSORT_EINVAL;
  if (segmented && B == 0 && n != 0) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!keys || !scratch) return BSORT_EINVAL;
  const bool with_idx = indices != nullptr;
  if ((flags & BSORT_KEYS_UNCHANGED) && !with_idx) return BSORT_EINVAL;
  // 2^32 keys or more are refused, with or without indices: that size has
  // not passed its tests on the GPU
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  const uint64_t b = segmented ? B : 1;
  // the scratch check uses the largest layout of any configuration, so a
  // buffer sized by bsort_scratch_bytes fits every one of them
  Layout L;
  if (!make_layout((int)sizeof(KT), n, b, with_idx, flags, tile_of((int)sizeof(KT), 1),
                   tfin_of((int)sizeof(KT), 1), &L))
    return BSORT_EINVAL;
  if (scratch_bytes < L.total) return BSORT_ESCRATCH;
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return BSORT_EINVAL;
  int cus = 0, dev = 0;
  const int rc = device_check(&cus, &dev);
  if (rc != BSORT_OK) return rc;
  if (force_config == CONFIG_DRY_RUN) return BSORT_OK;
  const int id = force_config >= 0 ? force_config
                                   : choose_config(dev, (int)sizeof(KT), with_idx, n, b);
  const Config c = config_of(id);
  make_layout((int)sizeof(KT), n, b, with_idx, flags, tile_of((int)sizeof(KT), c.lv),
              tfin_of((int)sizeof(KT), c.fv), &L);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *scr = static_cast<char *>(scratch);
  KT *k = static_cast<KT *>(keys);
  if (flags & BSORT_KEYS_UNCHANGED) {
    k = reinterpret_cast<KT *>(scr + L.keys0);
    const hipError_t e = hipMemcpyAsync(k, keys, n * sizeof(KT), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "key copy");
  }
  const int64_t *off = segmented ? offsets : nullptr;
  if (with_idx)
    return launch_cfg<KT, true>(c, k, n, off, b, mode, flags, indices, scr, L, cus, st, stop);
  return launch_cfg<KT, false>(c, k, n, off, b, mode, flags, indices, scr, L, cus, st, stop);
}

int dispatch(void *keys, int key_type, int key_bytes, uint64_t n, const int64_t *offsets,
             uint64_t B, bool segmented, uint32_t flags, void *indices, void *scratch,
             size_t scratch_bytes, void *stream, int force_config = -1, int stop = 64) {
  if (key_type != BSORT_KEY_U && key_type != BSORT_KEY_I && key_type != BSORT_KEY_F)
    return BSORT_EINVAL;
  switch (key_bytes) {
    case 1:
      return run<uint8_t>(keys, n, offsets, B, segmented, key_type, flags, indices, scratch,
                          scratch_bytes, stream, force_config, stop);
    case 2:
      return run<uint16_t>(keys, n, offsets, B, segmented, key_type, flags, indices, scratch,
                           scratch_bytes, stream, force_config, stop);
    case 4:
      return run<uint32_t>(keys, n, offsets, B, segmented, key_type, flags, indices, scratch,
                           scratch_bytes, stream, force_config, stop);
    case 8:
      return run<uint64_t>(keys, n, offsets, B, segmented, key_type, flags, indices, scratch,
                           scratch_bytes, stream, force_config, stop);
    default:
      return BSORT_EINVAL;
  }
}

// Validation shared by the gather and the key-value entry points.
bool value_args_ok(const void *p, int value_bytes) {
  if (value_bytes != 1 && value_bytes != 2 && value_bytes != 4 && value_bytes != 8 &&
      value_bytes != 16)
    return false;
  return (reinterpret_cast<uintptr_t>(p) & (uintptr_t)(value_bytes - 1)) == 0;
}

int launch_gather(const void *values, int value_bytes, const void *indices, bool i64,
                  const int64_t *offsets, uint64_t B, uint64_t n, void *out, int cus,
                  hipStream_t st, bool scatter = false, const uint32_t *status = nullptr) {
  const uint32_t grid = clamp_grid((n + GCH - 1) / GCH, (uint64_t)cus * 8);
#define BG_ONE(VT, I, S)                                                                    \
  hipLaunchKernelGGL((gather_kernel<VT, I, S>), dim3(grid), dim3(256), 0, st,               \
                     static_cast<const VT *>(values), indices, offsets, B, n,               \
                     static_cast<VT *>(out), status)
#define BG_LAUNCH(VT)                                                                       \
  do {                                                                                      \
    if (i64 && scatter) BG_ONE(VT, true, true);                                             \
    else if (i64) BG_ONE(VT, true, false);                                                  \
    else if (scatter) BG_ONE(VT, false, true);                                              \
    else BG_ONE(VT, false, false);                                                          \
  } while (0)
  switch (value_bytes) {
    case 1: BG_LAUNCH(uint8_t); break;
    case 2: BG_LAUNCH(uint16_t); break;
    case 4: BG_LAUNCH(uint32_t); break;
    case 8: BG_LAUNCH(uint64_t); break;
    default: BG_LAUNCH(uint4); break;
  }
#undef BG_LAUNCH
#undef BG_ONE
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BSORT_OK;
}

// Scratch of a key-value call: the sort's own, then the index buffer when
// the caller passes none, then the gathered values.
struct PairLayout {
  size_t sort, idx, vals, total;
};
bool pair_layout(int key_bytes, uint64_t n, uint64_t B, int value_bytes, bool caller_idx,
                 uint32_t flags, PairLayout *P) {
  if (flags & ~ALL_FLAGS) return false;
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return false;
  if (value_bytes != 1 && value_bytes != 2 && value_bytes != 4 && value_bytes != 8 &&
      value_bytes != 16)
    return false;
  Layout L;
  if (!make_layout(key_bytes, n, B ? B : 1, true, flags, tile_of(key_bytes, 1),
                   tfin_of(key_bytes, 1), &L))
    return false;
  P->sort = L.total;
  size_t off = up256(L.total);
  P->idx = off;
  if (!caller_idx) off = up256(off + n * ((flags & BSORT_IDX64) ? 8 : 4));
  P->vals = off;
  off = up256(off + n * (size_t)value_bytes);
  P->total = off;
  return true;
}

int sort_pairs(void *keys, int key_type, int key_bytes, const int64_t *offsets, uint64_t B,
               bool segmented, uint64_t n, uint32_t flags, void *values, int value_bytes,
               void *indices, void *scratch, size_t scratch_bytes, void *stream) {
  if (flags & ~ALL_FLAGS) return BSORT_EINVAL;
  if (value_bytes != 1 && value_bytes != 2 && value_bytes != 4 && value_bytes != 8 &&
      value_bytes != 16)
    return BSORT_EINVAL;
  if (segmented && B > 0 && !offsets) return BSORT_EINVAL;
  if (segmented && B == 0 && n != 0) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!keys || !values || !scratch || !value_args_ok(values, value_bytes)) return BSORT_EINVAL;
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  PairLayout P;
  if (!pair_layout(key_bytes, n, segmented ? B : 1, value_bytes, indices != nullptr, flags, &P))
    return BSORT_EINVAL;
  if (scratch_bytes < P.total) return BSORT_ESCRATCH;
  char *scr = static_cast<char *>(scratch);
  void *idx = indices ? indices : static_cast<void *>(scr + P.idx);
  int rc = dispatch(keys, key_type, key_bytes, n, offsets, segmented ? B : 1, segmented, flags,
                    idx, scratch, P.sort, stream, CONFIG_DRY_RUN);
  if (rc != BSORT_OK) return rc;
  rc = dispatch(keys, key_type, key_bytes, n, offsets, segmented ? B : 1, segmented, flags, idx,
                scratch, P.sort, stream);
  if (rc != BSORT_OK) return rc;
  int cus = 0;
  rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  void *tmp = scr + P.vals;
  // the sort's status word (its header starts the scratch): bad offsets
  // leave the values as they were, like the keys
  const uint32_t *status = &reinterpret_cast<const Header *>(scr)->status;
  rc = launch_gather(values, value_bytes, idx, (flags & BSORT_IDX64) != 0,
                     segmented ? offsets : nullptr, segmented ? B : 1, n, tmp, cus, st, false,
                     status);
  if (rc != BSORT_OK) return rc;
  const hipError_t e =
      hipMemcpyAsync(values, tmp, n * (size_t)value_bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "value copy");
  return BSORT_OK;
}

// 128-bit keys: scratch for the high and low words, the two permutations,
// the run offsets, the block maxima of their scan, then the scratch of the
// inner sorts (the larger of the key-value sort and the segmented sort).
struct WideLayout {
  size_t hi, lo, idx1, idx2, offs, bmax, inner, inner_bytes, total;
};
constexpr uint32_t WIDE_FLAGS = BSORT_DESCENDING | BSORT_NO_SKIP | BSORT_NO_FINISH |
                                BSORT_IDX64 | BSORT_KEYS_UNCHANGED;
bool wide_layout(uint64_t n, uint32_t flags, WideLayout *W) {
  if (flags & ~WIDE_FLAGS) return false;
  const uint32_t inner = flags & (BSORT_NO_SKIP | BSORT_NO_FINISH | BSORT_IDX64);
  const size_t ib = (flags & BSORT_IDX64) ? 8 : 4;
  size_t off = 0;
  W->hi = off; off = up256(off + n * 8);
  W->lo = off; off = up256(off + n * 8);
  W->idx1 = off; off = up256(off + n * ib);
  W->idx2 = off; off = up256(off + n * ib);
  W->offs = off; off = up256(off + (n + 1) * 8);
  W->bmax = off; off = up256(off + ((n + RCH - 1) / RCH + 1) * 8);
  PairLayout P;
  if (!pair_layout(8, n, 1, 8, true, inner, &P)) return false;
  Layout L;
  if (!make_layout(8, n, n ? n : 1, true, inner, tile_of(8, 1), tfin_of(8, 1), &L)) return false;
  W->inner = off;
  W->inner_bytes = P.total > L.total ? P.total : L.total;
  off = up256(off + W->inner_bytes);
  W->total = off;
  return true;
}

int sort128(void *keys, int key_type, uint64_t n, uint32_t flags, void *indices, void *scratch,
            size_t scratch_bytes, void *stream) {
  if (key_type != BSORT_KEY_U && key_type != BSORT_KEY_I && key_type != BSORT_KEY_F)
    return BSORT_EINVAL;
  if (flags & ~WIDE_FLAGS) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!keys || !scratch) return BSORT_EINVAL;
  if ((flags & BSORT_KEYS_UNCHANGED) && !indices) return BSORT_EINVAL;
  if ((reinterpret_cast<uintptr_t>(keys) & 15) || (reinterpret_cast<uintptr_t>(scratch) & 255) ||
      (reinterpret_cast<uintptr_t>(indices) & ((flags & BSORT_IDX64) ? 7 : 3)))
    return BSORT_EINVAL;
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  WideLayout W;
  if (!wide_layout(n, flags, &W)) return BSORT_EINVAL;
  if (scratch_bytes < W.total) return BSORT_ESCRATCH;
  int cus = 0;
  int rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *scr = static_cast<char *>(scratch);
  uint64_t *hi = reinterpret_cast<uint64_t *>(scr + W.hi);
  uint64_t *lo = reinterpret_cast<uint64_t *>(scr + W.lo);
  void *idx1 = scr + W.idx1;
  void *idx2 = scr + W.idx2;
  int64_t *offs = reinterpret_cast<int64_t *>(scr + W.offs);
  int64_t *bmax = reinterpret_cast<int64_t *>(scr + W.bmax);
  void *inner = scr + W.inner;
  const uint32_t iflags = flags & (BSORT_NO_SKIP | BSORT_NO_FINISH | BSORT_IDX64);
  const int desc = (flags & BSORT_DESCENDING) ? 1 : 0;
  // the inner calls are validated before anything is enqueued
  rc = dispatch(lo, BSORT_KEY_U, 8, n, offs, n, true, iflags, idx2, inner, W.inner_bytes,
                stream, CONFIG_DRY_RUN);
  if (rc != BSORT_OK) return rc;
  const uint32_t g = clamp_grid((n + 255) / 256, (uint64_t)cus * 8);
  hipLaunchKernelGGL(wide_split_kernel, dim3(g), dim3(256), 0, st,
                     static_cast<const uint64_t *>(keys), n, key_type, desc, hi, lo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  // high words first, the low words moving with them
  rc = sort_pairs(hi, BSORT_KEY_U, 8, nullptr, 1, false, n, iflags, lo, 8, idx1, inner,
                  W.inner_bytes, stream);
  if (rc != BSORT_OK) return rc;
  // runs of equal high words -> segments; the low words sorted within them
  const uint64_t nb = (n + RCH - 1) / RCH;
  hipLaunchKernelGGL(run_start_local_kernel, dim3((uint32_t)nb), dim3(256), 0, st, hi, n, offs,
                     bmax);
  hipLaunchKernelGGL(run_start_blocks_kernel, dim3(1), dim3(1024), 0, st, bmax, nb);
  hipLaunchKernelGGL(run_start_final_kernel, dim3(clamp_grid((n + 256) / 256, (uint64_t)cus * 8)),
                     dim3(256), 0, st, offs, bmax, n);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  rc = dispatch(lo, BSORT_KEY_U, 8, n, offs, n, true, iflags, idx2, inner, W.inner_bytes, stream);
  if (rc != BSORT_OK) return rc;
  // the key's permutation: first the high-word sort's, within each run the
  // low-word sort's
  if (indices) {
    rc = launch_gather(idx1, (flags & BSORT_IDX64) ? 8 : 4, idx2, (flags & BSORT_IDX64) != 0,
                       offs, n, n, indices, cus, st);
    if (rc != BSORT_OK) return rc;
  }
  if (!(flags & BSORT_KEYS_UNCHANGED)) {
    hipLaunchKernelGGL(wide_merge_kernel, dim3(g), dim3(256), 0, st, hi, lo, n, key_type, desc,
                       static_cast<uint64_t *>(keys));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return BSORT_OK;
}

// ---- in-place (keys-only, low-scratch) sort
//
// Scratch: the header, per-level lists and per-tile arrays only, O(n / tile
// + segments).  Bounds as for the main layout, except that the finish lists
// are consumed after every step that fills them (the seed and each plan),
// so they hold one step's entries: the seed's (at most B) or two per parent.
constexpr uint32_t IP_FLAGS = BSORT_DESCENDING | BSORT_NO_SKIP | BSORT_NO_FINISH;

struct InplaceLayout {
  size_t hdr, cnts, segs[2], acc[2], split[2], tmap, pre, sub, ends, items, fin, fins,
      fint, finm, cpy, total;
  uint64_t smax, tmax, fmax;
};

bool inplace_layout(int key_bytes, uint64_t n, uint64_t B, uint32_t flags, InplaceLayout *L) {
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return false;
  const uint64_t tile = inplace_tile_of(key_bytes), tfin = tfin_of(key_bytes, 0);
  const bool no_finish = (flags & BSORT_NO_FINISH) != 0;
  L->smax = (no_finish ? n / 2 : n / (tfin + 1)) + 1;
  L->tmax = n / tile + L->smax + 1;
  const uint64_t fb = B + 2 * L->smax + 1;
  L->fmax = fb < n + 1 ? fb : n + 1;
  size_t off = 0;
  L->hdr = off; off = up256(off + sizeof(Header));
  L->cnts = off; off = up256(off + 4 * (3 * L->tmax) * 4);
  for (int i = 0; i < 2; ++i) { L->segs[i] = off; off = up256(off + L->smax * sizeof(Seg)); }
  for (int i = 0; i < 2; ++i) { L->acc[i] = off; off = up256(off + L->tmax * sizeof(AccRep)); }
  for (int i = 0; i < 2; ++i) { L->split[i] = off; off = up256(off + L->smax * 8); }
  L->tmap = off; off = up256(off + L->tmax * sizeof(Seg));
  L->pre = off; off = up256(off + L->tmax * 4);
  L->sub = off; off = up256(off + L->tmax * 8 * 4);   // front keys per wave chunk (8 waves)
  L->ends = off; off = up256(off + L->tmax * 8);
  L->items = off; off = up256(off + L->tmax * 32);  // two {left, right} starts per tile
  L->fin = off; off = up256(off + L->fmax * sizeof(Seg));
  L->fins = off; off = up256(off + L->fmax * sizeof(Seg));
  L->fint = off; off = up256(off + L->fmax * sizeof(Seg));
  L->finm = off; off = up256(off + L->fmax * sizeof(Seg));
  L->cpy = off; off = up256(off + sizeof(Seg));  // never filled: nothing sits in a second buffer
  L->total = off;
  return true;
}

template <typename KT>
void launch_finishes(FinishArgs<KT> fa, Header *hdr, Seg *fin, Seg *fins, Seg *fint, Seg *finm,
                     uint64_t fmax, int cus, hipStream_t st) {
  using FS = FinishShape<KT, 0>;
  using SF = SmallFinish<KT>;
  auto fk = finish_kernel<KT, false, FS::FB, FS::FIPT>;
  auto mk = finish_kernel<KT, false, FS::FB, FS::FIPT / 2>;
  auto sk = finish_kernel<KT, false, SF::B, SF::IPT>;
  auto tk = finish_kernel<KT, false, TinyFinish::B, TinyFinish::IPT>;
  static const int occ_f = occupancy(fk, FS::FB), occ_m = occupancy(mk, FS::FB);
  static const int occ_s = occupancy(sk, SF::B), occ_t = occupancy(tk, TinyFinish::B);
  fa.list = fin;
  fa.count = &hdr->n_finish;
  hipLaunchKernelGGL(fk, dim3(clamp_grid(fmax, (uint64_t)cus * occ_f)), dim3(FS::FB), 0, st, fa);
  fa.list = finm;
  fa.count = &hdr->n_finish_med;
  hipLaunchKernelGGL(mk, dim3(clamp_grid(fmax, (uint64_t)cus * occ_m)), dim3(FS::FB), 0, st, fa);
  fa.list = fins;
  fa.count = &hdr->n_finish_small;
  hipLaunchKernelGGL(sk, dim3(clamp_grid(fmax, (uint64_t)cus * occ_s)), dim3(SF::B), 0, st, fa);
  fa.list = fint;
  fa.count = &hdr->n_finish_tiny;
  hipLaunchKernelGGL(tk, dim3(clamp_grid(fmax, (uint64_t)cus * occ_t)), dim3(TinyFinish::B), 0,
                     st, fa);
}

template <typename KT>
int launch_inplace(KT *keys, uint64_t n, const int64_t *offsets, uint64_t B, int mode,
                   uint32_t flags, char *scr, const InplaceLayout &L, int cus, hipStream_t st) {
  using LS = InplaceShape<KT>;
  using FS = FinishShape<KT, 0>;
  const int w = 8 * (int)sizeof(KT);
  const int desc = (flags & BSORT_DESCENDING) ? 1 : 0;
  const int no_skip = (flags & BSORT_NO_SKIP) ? 1 : 0;
  const int no_finish = (flags & BSORT_NO_FINISH) ? 1 : 0;
  Header *hdr = reinterpret_cast<Header *>(scr + L.hdr);
  Seg *segs[2] = {reinterpret_cast<Seg *>(scr + L.segs[0]),
                  reinterpret_cast<Seg *>(scr + L.segs[1])};
  AccRep *acc[2] = {reinterpret_cast<AccRep *>(scr + L.acc[0]),
                    reinterpret_cast<AccRep *>(scr + L.acc[1])};
  uint64_t *split[2] = {reinterpret_cast<uint64_t *>(scr + L.split[0]),
                        reinterpret_cast<uint64_t *>(scr + L.split[1])};
  Seg *fin = reinterpret_cast<Seg *>(scr + L.fin);
  Seg *fins = reinterpret_cast<Seg *>(scr + L.fins);
  Seg *fint = reinterpret_cast<Seg *>(scr + L.fint);
  Seg *finm = reinterpret_cast<Seg *>(scr + L.finm);
  const uint64_t cap = (uint64_t)cus * 16;
  uint32_t *cnt_base = reinterpret_cast<uint32_t *>(scr + L.cnts);
  const uint64_t cn = 3 * L.tmax;
  uint32_t *tcnt[2] = {cnt_base, cnt_base + 2 * cn};
  uint32_t *scnt[2] = {cnt_base + cn, cnt_base + 3 * cn};
  hipLaunchKernelGGL(init_kernel, dim3(clamp_grid((4 * cn + 255) / 256, 2048)), dim3(256), 0,
                     st, hdr, cnt_base, 4 * cn);
  if (offsets)
    hipLaunchKernelGGL(validate_kernel, dim3(clamp_grid((B + 256) / 256, 1024)), dim3(256), 0,
                       st, offsets, B, n, hdr);

  ListArgs la;
  la.hdr = hdr;
  la.fin = fin;
  la.fin_small = fins;
  la.fin_tiny = fint;
  la.fin_med = finm;
  la.cpy = reinterpret_cast<Seg *>(scr + L.cpy);
  la.tile = LS::TILE;
  la.t_fin = FS::TFIN;
  la.t_small = SmallFinish<KT>::T;
  la.t_tiny = TinyFinish::T;
  la.t_med = FS::TFIN / 2;
  la.recount = (uint32_t)(2 * L.tmax);
  la.tiny_next = nullptr;  // the in-place levels take every segment in tiles

  SeedArgs sa;
  sa.l = la;
  sa.l.live_next = segs[0];
  sa.l.acc_next = acc[0];
  sa.l.split_next = split[0];
  sa.l.next_level = 0;
  sa.offsets = offsets;
  sa.B = B;
  sa.n = n;
  sa.w = w;
  sa.with_idx = 0;
  sa.no_finish = no_finish;
  sa.idx_final = nullptr;
  sa.idx64 = 0;
  hipLaunchKernelGGL(seed_kernel, dim3(clamp_grid((B + 255) / 256, cap)), dim3(256), 0, st, sa);

  FinishArgs<KT> fa;
  fa.keys_buf[0] = keys;
  fa.keys_buf[1] = keys;
  fa.idx_buf[0] = nullptr;
  fa.idx_buf[1] = nullptr;
  fa.keys_final = keys;
  fa.idx_final = nullptr;
  fa.hdr = hdr;
  fa.w = w;
  fa.mode = mode;
  fa.desc = desc;
  fa.idx64 = 0;
  fa.no_skip = no_skip;
  launch_finishes<KT>(fa, hdr, fin, fins, fint, finm, L.fmax, cus, st);

  auto ck = ip_count_kernel<KT, LS::LB, LS::LIPT>;
  auto lk = ip_locate_kernel<KT, LS::LB, LS::LIPT>;
  // the coalesced swap for 2- and 4-byte keys, the blocked one for 1- and 8-byte keys
  // (the faster of the two for each width)
  auto sk = (sizeof(KT) == 2 || sizeof(KT) == 4) ? ip_swap_kernel<KT, LS::LB, LS::LIPT>
                                                 : ip_swap_blocked_kernel<KT, LS::LB, LS::LIPT>;
  static const int occ_c = occupancy(ck, LS::LB), occ_s = occupancy(sk, LS::LB);
  const uint32_t cgrid = clamp_grid((L.tmax + 1) / 2, (uint64_t)cus * occ_c);  // two tiles a block
  const uint32_t sgrid = clamp_grid(2 * L.tmax, (uint64_t)cus * occ_s);
  const uint32_t xgrid = clamp_grid((L.tmax + 3) / 4, cap);
  const uint32_t pgrid = clamp_grid((L.smax + 255) / 256, cap);
  const int levels = (!offsets && !no_finish && n <= FS::TFIN) ? 0 : w;
  for (int lvl = 0; lvl < levels; ++lvl) {
    InplaceArgs<KT> a;
    a.keys = keys;
    a.live = segs[lvl & 1];
    a.tiles = reinterpret_cast<Seg *>(scr + L.tmap);
    a.hdr = hdr;
    a.tcnt = tcnt[lvl & 1];
    a.scnt = scnt[lvl & 1];
    a.pre = reinterpret_cast<uint32_t *>(scr + L.pre);
    a.sub = reinterpret_cast<uint32_t *>(scr + L.sub);
    a.ends = reinterpret_cast<uint32_t *>(scr + L.ends);
    a.items = reinterpret_cast<uint64_t *>(scr + L.items);
    a.acc = acc[lvl & 1];
    a.split = split[lvl & 1];
    a.w = w;
    a.mode = mode;
    a.desc = desc;
    a.level = lvl;
    hipLaunchKernelGGL(ck, dim3(cgrid), dim3(LS::LB), 0, st, a);
    hipLaunchKernelGGL((ip_prefix_kernel<KT>), dim3(xgrid), dim3(256), 0, st, a);
    hipLaunchKernelGGL(lk, dim3(xgrid), dim3(256), 0, st, a);
    hipLaunchKernelGGL(sk, dim3(sgrid), dim3(LS::LB), 0, st, a);

    PlanArgs pa;
    pa.l = la;
    pa.l.live_next = segs[(lvl + 1) & 1];
    pa.l.acc_next = acc[(lvl + 1) & 1];
    pa.l.split_next = split[(lvl + 1) & 1];
    pa.l.next_level = lvl + 1;
    pa.live = segs[lvl & 1];
    pa.acc = acc[lvl & 1];
    pa.split = split[lvl & 1];
    pa.zero_a = tcnt[lvl & 1];  // counted again two levels on
    pa.zero_b = scnt[lvl & 1];
    pa.zero_n = cn;
    pa.zero_per_tile = 0;
    pa.level = lvl;
    pa.w = w;
    pa.with_idx = 0;
    pa.idx64 = 0;
    pa.no_skip = no_skip;
    pa.no_finish = no_finish;
    pa.inplace = 1;
    hipLaunchKernelGGL(plan_kernel, dim3(pgrid), dim3(256), 0, st, pa);
    launch_finishes<KT>(fa, hdr, fin, fins, fint, finm, L.fmax, cus, st);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BSORT_OK;
}

template <typename KT>
int run_inplace(void *keys, uint64_t n, const int64_t *offsets, uint64_t B, bool segmented,
                int mode, uint32_t flags, void *scratch, size_t scratch_bytes, void *stream) {
  if (flags & ~IP_FLAGS) return BSORT_EINVAL;
  if (segmented && B > 0 && !offsets) return BSORT_EINVAL;
  if (segmented && B == 0 && n != 0) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!keys || !scratch) return BSORT_EINVAL;
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  const uint64_t b = segmented ? B : 1;
  InplaceLayout L;
  if (!inplace_layout((int)sizeof(KT), n, b, flags, &L)) return BSORT_EINVAL;
  if (scratch_bytes < L.total) return BSORT_ESCRATCH;
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return BSORT_EINVAL;
  int cus = 0;
  const int rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  return launch_inplace<KT>(static_cast<KT *>(keys), n, segmented ? offsets : nullptr, b, mode,
                            flags, static_cast<char *>(scratch), L, cus,
                            static_cast<hipStream_t>(stream));
}

int dispatch_inplace(void *keys, int key_type, int key_bytes, uint64_t n, const int64_t *offsets,
                     uint64_t B, bool segmented, uint32_t flags, void *scratch,
                     size_t scratch_bytes, void *stream) {
  if (key_type != BSORT_KEY_U && key_type != BSORT_KEY_I && key_type != BSORT_KEY_F)
    return BSORT_EINVAL;
  switch (key_bytes) {
    case 1:
      return run_inplace<uint8_t>(keys, n, offsets, B, segmented, key_type, flags, scratch,
                                  scratch_bytes, stream);
    case 2:
      return run_inplace<uint16_t>(keys, n, offsets, B, segmented, key_type, flags, scratch,
                                   scratch_bytes, stream);
    case 4:
      return run_inplace<uint32_t>(keys, n, offsets, B, segmented, key_type, flags, scratch,
                                   scratch_bytes, stream);
    case 8:
      return run_inplace<uint64_t>(keys, n, offsets, B, segmented, key_type, flags, scratch,
                                   scratch_bytes, stream);
    default:
      return BSORT_EINVAL;
  }
}

constexpr uint64_t BWD_MAX_SLICES = 8;
constexpr uint32_t BWD_BLOCK = 1024;

int launch_status() {
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? hip_fail(e, "kernel launch") : BSORT_OK;
}

template <typename ET, uint32_t SB>
void launch_staged(const void *g, const void *idx, uint64_t rows, uint64_t cols, uint64_t m,
                   uint64_t slices, uint64_t units, uint64_t grid, void *out, bool i64,
                   hipStream_t st) {
  const float rcp = 1.0f / (float)cols;
  if (i64)
    hipLaunchKernelGGL((backward_staged_kernel<ET, true, SB, BWD_BLOCK>), dim3((uint32_t)grid),
                       dim3(BWD_BLOCK), 0, st, static_cast<const ET *>(g), idx, rows, cols, m,
                       slices, units, rcp, static_cast<ET *>(out));
  else
    hipLaunchKernelGGL((backward_staged_kernel<ET, false, SB, BWD_BLOCK>), dim3((uint32_t)grid),
                       dim3(BWD_BLOCK), 0, st, static_cast<const ET *>(g), idx, rows, cols, m,
                       slices, units, rcp, static_cast<ET *>(out));
}

// Launches the LDS-staged scatter when the shape suits it; false otherwise.
template <typename ET>
bool backward_staged(const void *g, const void *idx, uint64_t rows, uint64_t cols, void *out,
                     bool i64, hipStream_t st) {
  constexpr uint64_t S64 = 65536 / sizeof(ET), S128 = 131072 / sizeof(ET);
  constexpr uint64_t MAX_GRID = 0xFFFFFFFFull / BWD_BLOCK;
  if (cols <= S64) {
    const uint64_t m = S64 / cols, units = (rows + m - 1) / m;
    if (units > MAX_GRID) return false;
    launch_staged<ET, 65536>(g, idx, rows, cols, m, 0, units, units, out, i64, st);
    return true;
  }
  const uint64_t slices = (cols + S128 - 1) / S128;
  if (slices > BWD_MAX_SLICES || rows > MAX_GRID / slices) return false;
  const uint64_t units = rows * slices;
  const uint64_t grid = slices > 1 ? 8 * ((units + 7) / 8) : units;
  if (grid > MAX_GRID) return false;
  if (slices == 1)  // one whole row per block
    launch_staged<ET, 131072>(g, idx, rows, cols, 1, 0, units, grid, out, i64, st);
  else
    launch_staged<ET, 131072>(g, idx, rows, cols, 1, slices, units, grid, out, i64, st);
  return true;
}

// ---- allocation-free calls
//
// bsort_segmented_noalloc takes its scratch from this fixed array instead of
// from the caller.  Every GPU the library runs on holds its own copy, at its
// own address, from the first such call until the process ends.  On the host
// the array's name is only a stand-in: its device address is fetched once
// per device with hipGetSymbolAddress (with that device current) and kept,
// and only that address is ever handed to kernels.
static __device__ __align__(256) char noalloc_scratch[BSORT_NOALLOC_SCRATCH_BYTES];
void *g_noalloc_ptr[64];
std::atomic<int> g_noalloc_ready[64];
std::mutex g_noalloc_mu;

int noalloc_scratch_of(int dev, void **out) {
  if (!g_noalloc_ready[dev].load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ready[dev].load(std::memory_order_relaxed)) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
      if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return BSORT_EHIP;
      g_noalloc_ptr[dev] = p;
      g_noalloc_ready[dev].store(1, std::memory_order_release);
    }
  }
  *out = g_noalloc_ptr[dev];
  return BSORT_OK;
}

}  // namespace

extern "C" {

size_t bsort_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments, int with_indices,
                           uint32_t flags) {
  if (flags & ~ALL_FLAGS) return 0;
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return 0;
  // the largest layout of any configuration: the smallest tile and threshold
  Layout L;
  if (!make_layout(key_bytes, n, num_segments ? num_segments : 1, with_indices != 0, flags,
                   tile_of(key_bytes, 1), tfin_of(key_bytes, 1), &L))
    return 0;
  return L.total;
}

int bsort_sort(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
               void *indices, void *scratch, size_t scratch_bytes, void *stream) {
  return dispatch(keys, key_type, key_bytes, n, nullptr, 1, false, flags, indices, scratch,
                  scratch_bytes, stream);
}

int bsort_segmented(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                    uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                    void *scratch, size_t scratch_bytes, void *stream) {
  return dispatch(keys, key_type, key_bytes, n, offsets, num_segments, true, flags, indices,
                  scratch, scratch_bytes, stream);
}

int bsort_levels(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                 uint64_t num_segments, uint64_t n, uint32_t flags, int levels, void *indices,
                 void *scratch, size_t scratch_bytes, void *stream) {
  if (levels < 0 || levels > 8 * key_bytes) return BSORT_EINVAL;
  const bool seg = offsets != nullptr;
  return dispatch(keys, key_type, key_bytes, n, offsets, seg ? num_segments : 1, seg,
                  flags | BSORT_PLAIN, indices, scratch, scratch_bytes, stream, -1, levels);
}

#define BSORT_TYPED(name, T, kt, kb)                                                        \
  int name(T *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,               \
           size_t scratch_bytes, void *stream) {                                            \
    return dispatch(keys, kt, kb, n, nullptr, 1, false, flags, indices, scratch,            \
                    scratch_bytes, stream);                                                 \
  }
BSORT_TYPED(bsort_u8, uint8_t, BSORT_KEY_U, 1)
BSORT_TYPED(bsort_u16, uint16_t, BSORT_KEY_U, 2)
BSORT_TYPED(bsort_u32, uint32_t, BSORT_KEY_U, 4)
BSORT_TYPED(bsort_u64, uint64_t, BSORT_KEY_U, 8)
BSORT_TYPED(bsort_i8, int8_t, BSORT_KEY_I, 1)
BSORT_TYPED(bsort_i16, int16_t, BSORT_KEY_I, 2)
BSORT_TYPED(bsort_i32, int32_t, BSORT_KEY_I, 4)
BSORT_TYPED(bsort_i64, int64_t, BSORT_KEY_I, 8)
BSORT_TYPED(bsort_f8, uint8_t, BSORT_KEY_F, 1)
BSORT_TYPED(bsort_f16, uint16_t, BSORT_KEY_F, 2)
BSORT_TYPED(bsort_f32, float, BSORT_KEY_F, 4)
BSORT_TYPED(bsort_f64, double, BSORT_KEY_F, 8)
#undef BSORT_TYPED

int bsort_segmented_f32(float *keys, const int64_t *offsets, uint64_t num_segments, uint64_t n,
                        uint32_t flags, void *indices, void *scratch, size_t scratch_bytes,
                        void *stream) {
  return dispatch(keys, BSORT_KEY_F, 4, n, offsets, num_segments, true, flags, indices,
                  scratch, scratch_bytes, stream);
}

int bsort_segmented_i32(int32_t *keys, const int64_t *offsets, uint64_t num_segments,
                        uint64_t n, uint32_t flags, void *indices, void *scratch,
                        size_t scratch_bytes, void *stream) {
  return dispatch(keys, BSORT_KEY_I, 4, n, offsets, num_segments, true, flags, indices,
                  scratch, scratch_bytes, stream);
}

int bsort_backward_scatter(const void *grad_sorted, const void *indices, uint64_t rows,
                           uint64_t cols, int elem_bytes, void *grad_in, uint32_t flags,
                           void *stream) {
  if (flags & ~(uint32_t)BSORT_IDX64) return BSORT_EINVAL;
  if (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) return BSORT_EINVAL;
  if (rows == 0 || cols == 0) return BSORT_OK;
  if (!grad_sorted || !indices || !grad_in) return BSORT_EINVAL;
  int cus = 0;
  const int rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool i64 = (flags & BSORT_IDX64) != 0;
  // Rows of at most 64 KB: runs of whole rows staged in 64 KB of LDS (two
  // blocks per CU).  Up to BWD_MAX_SLICES slices of 128 KB: one slice per
  // block.  Wider rows: the direct kernel (each extra slice re-reads the row).
  if (elem_bytes == 2) {
    if (backward_staged<uint16_t>(grad_sorted, indices, rows, cols, grad_in, i64, st))
      return launch_status();
  } else if (elem_bytes == 4) {
    if (backward_staged<uint32_t>(grad_sorted, indices, rows, cols, grad_in, i64, st))
      return launch_status();
  } else if (backward_staged<uint64_t>(grad_sorted, indices, rows, cols, grad_in, i64, st)) {
    return launch_status();
  }
  const uint64_t bx = (cols + 255) / 256;
  dim3 grid(clamp_grid(bx, 4096), clamp_grid(rows, 65535));
#define BS_LAUNCH(ET)                                                                       \
  do {                                                                                      \
    if (i64)                                                                                \
      hipLaunchKernelGGL((backward_scatter_kernel<ET, true>), grid, dim3(256), 0, st,       \
                         static_cast<const ET *>(grad_sorted), indices, rows, cols,         \
                         static_cast<ET *>(grad_in));                                       \
    else                                                                                    \
      hipLaunchKernelGGL((backward_scatter_kernel<ET, false>), grid, dim3(256), 0, st,      \
                         static_cast<const ET *>(grad_sorted), indices, rows, cols,         \
                         static_cast<ET *>(grad_in));                                       \
  } while (0)
  if (elem_bytes == 2) BS_LAUNCH(uint16_t);
  else if (elem_bytes == 4) BS_LAUNCH(uint32_t);
  else BS_LAUNCH(uint64_t);
#undef BS_LAUNCH
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BSORT_OK;
}

size_t bsort_pairs_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments,
                                 int value_bytes, int with_indices, uint32_t flags) {
  PairLayout P;
  if (!pair_layout(key_bytes, n, num_segments ? num_segments : 1, value_bytes, with_indices != 0,
                   flags, &P))
    return 0;
  return P.total;
}

int bsort_sort_pairs(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                     void *values, int value_bytes, void *indices, void *scratch,
                     size_t scratch_bytes, void *stream) {
  return sort_pairs(keys, key_type, key_bytes, nullptr, 1, false, n, flags, values, value_bytes,
                    indices, scratch, scratch_bytes, stream);
}

int bsort_segmented_pairs(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                          uint64_t num_segments, uint64_t n, uint32_t flags, void *values,
                          int value_bytes, void *indices, void *scratch, size_t scratch_bytes,
                          void *stream) {
  return sort_pairs(keys, key_type, key_bytes, offsets, num_segments, true, n, flags, values,
                    value_bytes, indices, scratch, scratch_bytes, stream);
}

int bsort_gather(const void *values, int value_bytes, const void *indices,
                 const int64_t *offsets, uint64_t num_segments, uint64_t n, uint32_t flags,
                 void *out, void *stream) {
  if (flags & ~(uint32_t)BSORT_IDX64) return BSORT_EINVAL;
  if (offsets && num_segments == 0 && n != 0) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!values || !indices || !out) return BSORT_EINVAL;
  if (!value_args_ok(values, value_bytes) || !value_args_ok(out, value_bytes))
    return BSORT_EINVAL;
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  int cus = 0;
  const int rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  return launch_gather(values, value_bytes, indices, (flags & BSORT_IDX64) != 0, offsets,
                       offsets ? num_segments : 1, n, out, cus, static_cast<hipStream_t>(stream));
}

int bsort_scatter(const void *values, int value_bytes, const void *indices,
                  const int64_t *offsets, uint64_t num_segments, uint64_t n, uint32_t flags,
                  void *out, void *stream) {
  if (flags & ~(uint32_t)BSORT_IDX64) return BSORT_EINVAL;
  if (offsets && num_segments == 0 && n != 0) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!values || !indices || !out) return BSORT_EINVAL;
  if (!value_args_ok(values, value_bytes) || !value_args_ok(out, value_bytes))
    return BSORT_EINVAL;
  if (n >= (1ull << 32)) return BSORT_ETOOBIG;
  int cus = 0;
  const int rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  return launch_gather(values, value_bytes, indices, (flags & BSORT_IDX64) != 0, offsets,
                       offsets ? num_segments : 1, n, out, cus, static_cast<hipStream_t>(stream),
                       true);
}

size_t bsort_inplace_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments,
                                   uint32_t flags) {
  if (flags & ~IP_FLAGS) return 0;
  InplaceLayout L;
  if (!inplace_layout(key_bytes, n, num_segments ? num_segments : 1, flags, &L)) return 0;
  return L.total;
}

int bsort_sort_inplace(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                       void *scratch, size_t scratch_bytes, void *stream) {
  return dispatch_inplace(keys, key_type, key_bytes, n, nullptr, 1, false, flags, scratch,
                          scratch_bytes, stream);
}

int bsort_segmented_inplace(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                            uint64_t num_segments, uint64_t n, uint32_t flags, void *scratch,
                            size_t scratch_bytes, void *stream) {
  return dispatch_inplace(keys, key_type, key_bytes, n, offsets, num_segments, true, flags,
                          scratch, scratch_bytes, stream);
}

size_t bsort_scratch_bytes128(uint64_t n, int with_indices, uint32_t flags) {
  (void)with_indices;  // the permutation is always built
  WideLayout W;
  if (!wide_layout(n, flags, &W)) return 0;
  return W.total;
}

int bsort_sort128(void *keys, int key_type, uint64_t n, uint32_t flags, void *indices,
                  void *scratch, size_t scratch_bytes, void *stream) {
  return sort128(keys, key_type, n, flags, indices, scratch, scratch_bytes, stream);
}

int bsort_sort_layout(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                      const uint8_t *bit_order, void *indices, void *scratch,
                      size_t scratch_bytes, void *stream) {
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return BSORT_EINVAL;
  if (n == 0) return BSORT_OK;
  if (!bit_order) return BSORT_EINVAL;
  const int w = 8 * key_bytes;
  BitLayout lay;
  uint64_t seen = 0;
  for (int j = 0; j < w; ++j) {
    if (bit_order[j] >= w) return BSORT_EINVAL;
    seen |= 1ull << bit_order[j];
    lay.src[j] = bit_order[j];
  }
  if (seen != (w == 64 ? ~0ull : ((1ull << w) - 1))) return BSORT_EINVAL;  // not a permutation
  if (reinterpret_cast<uintptr_t>(keys) & (uintptr_t)(key_bytes - 1)) return BSORT_EINVAL;
  // the sort's own checks, before anything is enqueued
  int rc = dispatch(keys, key_type, key_bytes, n, nullptr, 1, false, flags, indices, scratch,
                    scratch_bytes, stream, CONFIG_DRY_RUN);
  if (rc != BSORT_OK) return rc;
  int cus = 0;
  rc = device_check(&cus);
  if (rc != BSORT_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t g = clamp_grid((n + 255) / 256, (uint64_t)cus * 8);
  auto transform = [&](int inverse) {
    switch (key_bytes) {
      case 1: hipLaunchKernelGGL(layout_kernel<uint8_t>, dim3(g), dim3(256), 0, st,
                                 static_cast<uint8_t *>(keys), n, w, lay, inverse); break;
      case 2: hipLaunchKernelGGL(layout_kernel<uint16_t>, dim3(g), dim3(256), 0, st,
                                 static_cast<uint16_t *>(keys), n, w, lay, inverse); break;
      case 4: hipLaunchKernelGGL(layout_kernel<uint32_t>, dim3(g), dim3(256), 0, st,
                                 static_cast<uint32_t *>(keys), n, w, lay, inverse); break;
      default: hipLaunchKernelGGL(layout_kernel<uint64_t>, dim3(g), dim3(256), 0, st,
                                  static_cast<uint64_t *>(keys), n, w, lay, inverse); break;
    }
    return hipGetLastError();
  };
  hipError_t e = transform(0);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  rc = dispatch(keys, key_type, key_bytes, n, nullptr, 1, false, flags, indices, scratch,
                scratch_bytes, stream);
  if (rc != BSORT_OK) return rc;
  e = transform(1);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BSORT_OK;
}

int bsort_config_count(void) { return N_CONFIGS; }

const char *bsort_config_name(int config) {
  static char names[N_CONFIGS][96];
  if (config < 0 || config >= N_CONFIGS) return "invalid configuration";
  if (!names[config][0]) {
    const Config c = config_of(config);
    snprintf(names[config], sizeof names[config],
             "level one wave x %d (tile %u keys), finish %dx%d (T %u keys of 4 B), %s grid",
             (int)tile_of(4, c.lv) / 64, tile_of(4, c.lv), c.fv == 1 ? 256 : 512,
             c.fv == 2 ? 8 : 16, tfin_of(4, c.fv), c.grid ? "half" : "full");
  }
  return names[config];
}

int bsort_config_override(int config) {
  if (config < -1 || config >= N_CONFIGS) return BSORT_EINVAL;
  g_override = config;
  return BSORT_OK;
}

int bsort_tuned_config(int key_bytes, int with_indices, uint64_t n, uint64_t num_segments) {
  if (key_bytes != 1 && key_bytes != 2 && key_bytes != 4 && key_bytes != 8) return BSORT_EINVAL;
  int cus = 0, dev = 0;
  const int rc = device_check(&cus, &dev);
  if (rc != BSORT_OK) return rc;
  return choose_config(dev, key_bytes, with_indices != 0, n, num_segments ? num_segments : 1);
}

void bsort_autotune_reset(void) { memset(g_tuned, 0, sizeof g_tuned); }

// Tuning cache: a text file, "bsort-autotune 1" and then one line per
// choice, "<arch> <CUs> <key bytes> <with indices> <size class> <config>".
// Entries name the device type rather than its index, so a file made on
// one machine applies to every GPU of the same type.
int bsort_autotune_save(const char *path) {
  if (!path) return BSORT_EINVAL;
  FILE *fp = fopen(path, "w");
  if (!fp) return BSORT_EINVAL;
  int rc = fprintf(fp, "bsort-autotune 1\n") > 0 ? BSORT_OK : BSORT_EINVAL;
  static const int kbs[4] = {1, 2, 4, 8};
  for (int dev = 0; dev < 64 && rc == BSORT_OK; ++dev) {
    bool any = false;
    for (int k = 0; k < 4 && !any; ++k)
      for (int x = 0; x < 2 && !any; ++x)
        for (int c = 0; c < 48 && !any; ++c) any = g_tuned[dev][k][x][c] > 0;
    if (!any) continue;
    hipDeviceProp_t p;
    const hipError_t e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) {
      rc = hip_fail(e, "hipGetDeviceProperties");
      break;
    }
    char arch[64];
    snprintf(arch, sizeof arch, "%s", p.gcnArchName);
    for (char *q = arch; *q; ++q)
      if (*q == ' ') *q = '_';
    for (int k = 0; k < 4 && rc == BSORT_OK; ++k)
      for (int x = 0; x < 2 && rc == BSORT_OK; ++x)
        for (int c = 0; c < 48 && rc == BSORT_OK; ++c)
          if (g_tuned[dev][k][x][c] > 0 &&
              fprintf(fp, "%s %d %d %d %d %d\n", arch, p.multiProcessorCount, kbs[k], x, c,
                      g_tuned[dev][k][x][c] - 1) <= 0)
            rc = BSORT_EINVAL;
  }
  if (fclose(fp) != 0 && rc == BSORT_OK) rc = BSORT_EINVAL;
  return rc;
}

int bsort_autotune_load(const char *path) {
  if (!path) return BSORT_EINVAL;
  FILE *fp = fopen(path, "r");
  if (!fp) return BSORT_EINVAL;
  struct Entry {
    char arch[64];
    int cus, kb, idx, cls, cfg;
  };
  static Entry entries[64 * 4 * 2 * 48];
  int ne = 0, rc = BSORT_OK;
  char line[256];
  if (!fgets(line, sizeof line, fp) || strcmp(line, "bsort-autotune 1\n") != 0) rc = BSORT_EINVAL;
  while (rc == BSORT_OK && fgets(line, sizeof line, fp)) {
    Entry en;
    char tail;
    if (ne >= (int)(sizeof entries / sizeof entries[0]) ||
        sscanf(line, "%63s %d %d %d %d %d %c", en.arch, &en.cus, &en.kb, &en.idx, &en.cls,
               &en.cfg, &tail) != 6 ||
        (en.kb != 1 && en.kb != 2 && en.kb != 4 && en.kb != 8) || en.idx < 0 || en.idx > 1 ||
        en.cls < 0 || en.cls >= 48 || en.cfg < 0 || en.cfg >= N_CONFIGS || en.cus <= 0) {
      rc = BSORT_EINVAL;
      break;
    }
    entries[ne++] = en;
  }
  fclose(fp);
  if (rc != BSORT_OK || ne == 0) return rc;  // a malformed file changes nothing
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  for (int dev = 0; dev < ndev && dev < 64; ++dev) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    char arch[64];
    snprintf(arch, sizeof arch, "%s", p.gcnArchName);
    for (char *q = arch; *q; ++q)
      if (*q == ' ') *q = '_';
    for (int i = 0; i < ne; ++i)
      if (strcmp(entries[i].arch, arch) == 0 && entries[i].cus == p.multiProcessorCount)
        g_tuned[dev][kb_slot(entries[i].kb)][entries[i].idx][entries[i].cls] =
            (signed char)(entries[i].cfg + 1);
  }
  return BSORT_OK;
}

int bsort_autotune(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                   uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                   void *scratch, size_t scratch_bytes, void *stream, int reps) {
  if (g_capturing) return BSORT_EINVAL;
  const bool seg = offsets != nullptr;
  const uint64_t B = seg ? num_segments : 1;
  // arguments checked as a sort would check them, nothing launched
  int rc = dispatch(keys, key_type, key_bytes, n, offsets, B, seg, flags, indices, scratch,
                    scratch_bytes, stream, CONFIG_DRY_RUN);
  if (rc != BSORT_OK) return rc;
  if (n == 0) return 0;
  int cus = 0, dev = 0;
  rc = device_check(&cus, &dev);
  if (rc != BSORT_OK) return rc;
  if (reps < 1) reps = 1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = n * (size_t)key_bytes;
  void *orig = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&orig, bytes);
  if (e != hipSuccess) return hip_fail(e, "bsort_autotune: hipMalloc");
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemcpyAsync(orig, keys, bytes, hipMemcpyDeviceToDevice, st);
  const int armed = g_timing.armed;
  g_timing.armed = 0;  // tuning launches are not benchmark launches
  int best = -1;
  float best_ms = 0.f;
  for (int id = 0; id < N_CONFIGS && e == hipSuccess && rc == BSORT_OK; ++id) {
    float t_min = 0.f;
    for (int r = 0; r < reps && e == hipSuccess && rc == BSORT_OK; ++r) {
      e = hipMemcpyAsync(keys, orig, bytes, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e != hipSuccess) break;
      rc = dispatch(keys, key_type, key_bytes, n, offsets, B, seg, flags, indices, scratch,
                    scratch_bytes, stream, id);
      if (rc != BSORT_OK) break;
      e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (r == 0 || ms < t_min)) t_min = ms;
    }
    if (e == hipSuccess && rc == BSORT_OK && (best < 0 || t_min < best_ms)) {
      best = id;
      best_ms = t_min;
    }
  }
  // leave the caller's buffers as a sort with the chosen configuration would
  if (e == hipSuccess && rc == BSORT_OK) {
    g_tuned[dev][kb_slot(key_bytes)][indices ? 1 : 0][size_class(n, B)] = (signed char)(best + 1);
    e = hipMemcpyAsync(keys, orig, bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      rc = dispatch(keys, key_type, key_bytes, n, offsets, B, seg, flags, indices, scratch,
                    scratch_bytes, stream, best);
  }
  g_timing.armed = armed;
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(orig);
  if (e != hipSuccess) return hip_fail(e, "bsort_autotune");
  return rc != BSORT_OK ? rc : best;
}

// A whole call recorded once into a HIP graph and replayed by one launch.
struct bsort_graph {
  hipGraphExec_t exec;
};

int bsort_graph_create(bsort_graph **out, void *keys, int key_type, int key_bytes,
                       const int64_t *offsets, uint64_t num_segments, uint64_t n,
                       uint32_t flags, void *indices, void *scratch, size_t scratch_bytes) {
  if (!out) return BSORT_EINVAL;
  *out = nullptr;
  if (g_capturing) return BSORT_EINVAL;
  const bool seg = offsets != nullptr;
  const uint64_t B = seg ? num_segments : 1;
  int rc = dispatch(keys, key_type, key_bytes, n, offsets, B, seg, flags, indices, scratch,
                    scratch_bytes, nullptr, CONFIG_DRY_RUN);
  if (rc != BSORT_OK) return rc;
  bsort_graph *g = new bsort_graph{nullptr};
  if (n == 0) {  // nothing to record: launching it does nothing
    *out = g;
    return BSORT_OK;
  }
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    g_capturing = 1;
    rc = dispatch(keys, key_type, key_bytes, n, offsets, B, seg, flags, indices, scratch,
                  scratch_bytes, cs);
    g_capturing = 0;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = ee;
  }
  if (e == hipSuccess && rc == BSORT_OK) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess || rc != BSORT_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;
    return e != hipSuccess ? hip_fail(e, "bsort_graph_create") : rc;
  }
  *out = g;
  return BSORT_OK;
}

int bsort_graph_launch(const bsort_graph *graph, void *stream) {
  if (!graph) return BSORT_EINVAL;
  if (!graph->exec) return BSORT_OK;
  const hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return BSORT_OK;
}

int bsort_graph_destroy(bsort_graph *graph) {
  if (!graph) return BSORT_OK;
  hipError_t e = hipSuccess;
  if (graph->exec) e = hipGraphExecDestroy(graph->exec);
  delete graph;
  if (e != hipSuccess) return hip_fail(e, "hipGraphExecDestroy");
  return BSORT_OK;
}

int bsort_segmented_noalloc(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                            uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                            void *stream) {
  if (n == 0)  // validated and done without any scratch, as bsort_segmented does
    return dispatch(keys, key_type, key_bytes, n, offsets, num_segments, true, flags, indices,
                    nullptr, 0, stream);
  // the same bound as bsort_segmented's check of a caller's scratch
  const size_t need = bsort_scratch_bytes(key_bytes, n, num_segments, indices != nullptr, flags);
  if (need == 0) return BSORT_EINVAL;
  if (n < (1ull << 32) && need > (size_t)BSORT_NOALLOC_SCRATCH_BYTES) return BSORT_ENOSPACE;
  int cus = 0, dev = 0;
  int rc = device_check(&cus, &dev);
  if (rc != BSORT_OK) return rc;
  void *scr = nullptr;
  rc = noalloc_scratch_of(dev, &scr);
  if (rc != BSORT_OK) return rc;
  return dispatch(keys, key_type, key_bytes, n, offsets, num_segments, true, flags, indices, scr,
                  (size_t)BSORT_NOALLOC_SCRATCH_BYTES, stream);
}

const char *bsort_strerror(int status) {
  switch (status) {
    case BSORT_OK: return "ok";
    case BSORT_EINVAL: return "invalid argument";
    case BSORT_ESCRATCH: return "scratch buffer too small";
    case BSORT_ETOOBIG: return "too many keys (2^32 or more)";
    case BSORT_EHIP: return g_hip_err[0] ? g_hip_err : "HIP runtime error";
    case BSORT_ENODEV: return "current device is not a gfx950 GPU";
    case BSORT_ENOSPACE:
      return "the call needs more scratch than the allocation-free entry point's built-in "
             "buffer (BSORT_NOALLOC_SCRATCH_BYTES) holds";
    default: return "unknown status";
  }
}

int bsort_level_stats(const void *scratch, void *stream, uint64_t *live_keys,
                      uint32_t *live_segments, uint32_t *tiles, int max_levels,
                      uint64_t *finish_keys, uint64_t *copy_keys) {
  if (!scratch || max_levels < 0) return BSORT_EINVAL;
  Header h;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&h, scratch, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "bsort_level_stats");
  const int m = max_levels < MAX_LEVELS ? max_levels : MAX_LEVELS;
  for (int i = 0; i < m; ++i) {
    if (live_keys) live_keys[i] = h.live_keys[i];
    if (live_segments) live_segments[i] = (uint32_t)(h.packed[i] >> 32);
    if (tiles) tiles[i] = (uint32_t)h.packed[i];
  }
  if (finish_keys) *finish_keys = h.finish_keys;
  if (copy_keys) *copy_keys = h.copy_keys;
  return m;
}

int bsort_level_bytes(const void *scratch, void *stream, uint64_t *iota_keys,
                      uint64_t *moved_keys, int max_levels) {
  if (!scratch || max_levels < 0) return BSORT_EINVAL;
  Header h;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&h, scratch, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "bsort_level_bytes");
  const int m = max_levels < MAX_LEVELS ? max_levels : MAX_LEVELS;
  for (int i = 0; i < m; ++i) {
    if (iota_keys) iota_keys[i] = h.iota_keys[i];
    if (moved_keys) moved_keys[i] = h.moved_keys[i];
  }
  return m;
}

int bsort_timing_arm(int capacity) {
  timing_free();
  if (capacity <= 0) return BSORT_OK;
  g_timing.ev = new hipEvent_t[2 * capacity];
  g_timing.lvl = new int[capacity];
  g_timing.cap = capacity;
  for (int i = 0; i < 2 * capacity; ++i) {
    const hipError_t e = hipEventCreate(&g_timing.ev[i]);
    if (e != hipSuccess) {
      g_timing.cap = i / 2;
      timing_free();
      return hip_fail(e, "hipEventCreate");
    }
  }
  g_timing.armed = 1;
  return BSORT_OK;
}

int bsort_timing_read(float *ms, int *levels, int capacity) {
  const int n = g_timing.count < capacity ? g_timing.count : capacity;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(g_timing.ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], g_timing.ev[2 * i], g_timing.ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    if (levels) levels[i] = g_timing.lvl[i];
  }
  g_timing.count = 0;
  return n;
}

void bsort_timing_disarm(void) { timing_free(); }

int bsort_device_status(const void *scratch, void *stream) {
  if (!scratch) return BSORT_EINVAL;
  uint32_t v = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char *p = static_cast<const char *>(scratch) + offsetof(Header, status);
  hipError_t e = hipMemcpyAsync(&v, p, sizeof v, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "bsort_device_status");
  return (int)v;
}

}  // extern "C"
