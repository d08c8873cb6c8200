/*
 * bsort.h -- C ABI of libbsort, an MI355X (gfx950) implementation of the
 * bsort bit-partition sort (Guzman, arXiv 2603.08929).
 *
 * The operation (Section II, Algorithms 1-2; Section III, Algorithms 3-5):
 * keys are split, most significant bit first, into a front and a back part
 * on one bit at a time; every part is split again on the next lower bit.
 * Ascending puts the 0-side first (Algorithm 1).  Two's-complement keys run
 * the sign-bit pass in the inverse direction (Algorithm 3); IEEE-754 style
 * keys (sign | exponent | mantissa) do the same and also sort the negative
 * half in the inverse direction on all lower bits (Section III-B's three-pass
 * procedure and the Fig. 3 trace).  Resulting order, ascending:
 *   unsigned: numeric;  signed: numeric;
 *   float: -NaN (largest payload first) < -inf < ... < -0 < +0 < ... < +inf
 *          < +NaN (smallest payload first)   (Section III-C special values)
 * Descending is the exact reverse on distinct keys.  Keys are compared as
 * raw bit patterns only -- never loaded as floating point -- so subnormals
 * and NaN payloads keep their bits.
 *
 * Every split is stable (both parts keep input order, as in the traces of
 * Figs. 1 and 2), so the optional index output is THE stable permutation:
 * equal bit patterns keep their input order in both directions.
 *
 * Common conventions
 * ------------------
 * - All pointers except `stream` are DEVICE pointers owned by the caller.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *   asynchronous on that stream: they enqueue kernels and return; they never
 *   allocate device memory and never synchronize.  Calls on one scratch
 *   buffer must not overlap; distinct scratch buffers may run concurrently.
 * - `keys` is sorted in place (the result lands in the caller's buffer).
 * - `indices` (nullable): receives the gather permutation out[j] = in[idx[j]],
 *   0-based and local to each segment (as torch.sort returns it).  uint32
 *   by default; int64 with BSORT_IDX64.
 * - `scratch` of at least bsort_scratch_bytes(...) bytes; 256-byte aligned.
 *   Its contents are undefined afterwards.
 * - Arguments are validated before anything is enqueued; on an error
 *   nothing is written to any buffer.
 */
#ifndef BSORT_H
#define BSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define BSORT_OK 0
#define BSORT_EINVAL (-1)   /* null pointer with n > 0, unknown flag bits, bad key type */
#define BSORT_ESCRATCH (-2) /* scratch smaller than bsort_scratch_bytes()                */
#define BSORT_ETOOBIG (-3)  /* n of 2^32 keys or more (any call)                         */
#define BSORT_EHIP (-4)     /* the HIP runtime refused a launch (see bsort_strerror)     */
#define BSORT_ENODEV (-5)   /* the current device is not a gfx950 GPU                    */
#define BSORT_ENOSPACE (-6) /* more scratch than bsort_segmented_noalloc's buffer holds   */

/* ---- flags ---- */
#define BSORT_DESCENDING 1u /* non-increasing order                                       */
#define BSORT_NO_SKIP 2u    /* partition on every bit; no AND/OR skip of constant bits     */
#define BSORT_NO_FINISH 4u  /* no in-LDS finish of small parts: every bit is a global pass */
#define BSORT_PLAIN (BSORT_NO_SKIP | BSORT_NO_FINISH) /* the paper's w full passes         */
#define BSORT_IDX64 8u      /* indices are int64 instead of uint32                         */
#define BSORT_KEYS_UNCHANGED 16u /* argsort: only the indices are written (indices required);
                                  * the keys are sorted in a scratch copy                  */

/* ---- key types (for bsort_scratch_bytes and the generic entry point) ---- */
#define BSORT_KEY_U 0 /* unsigned integer                     */
#define BSORT_KEY_I 1 /* two's-complement integer             */
#define BSORT_KEY_F 2 /* sign | exponent | mantissa float      */

/*
 * Bytes of device scratch a call needs.  key_bytes in {1,2,4,8};
 * num_segments = 1 for the single-array entry points.  with_indices != 0
 * when `indices` will be non-NULL.  The figure is O(n): a second key buffer
 * (n * key_bytes), a second index buffer (4n, or 8n with BSORT_IDX64), and
 * O(n/4096 + num_segments) bytes of work lists; BSORT_NO_FINISH raises the
 * work-list part to O(n), and BSORT_KEYS_UNCHANGED adds n * key_bytes for
 * the copy that is sorted.  Returns 0 for invalid arguments.
 */
size_t bsort_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments,
                           int with_indices, uint32_t flags);

/*
 * Single-array sort of keys[0, n) (Algorithms 2, 3 and 4 of the paper for
 * the U, I and F families).  f8 serves both e4m3 and e5m2 and f16 serves
 * both fp16 and bfloat16: the order only needs "sign bit first, then a
 * magnitude in sign-magnitude form", not the exponent width (Section III-C).
 * n = 0 is a no-op; n = 1 writes index 0.
 */
int bsort_u8(uint8_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
             size_t scratch_bytes, void *stream);
int bsort_u16(uint16_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_u32(uint32_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_u64(uint64_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_i8(int8_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
             size_t scratch_bytes, void *stream);
int bsort_i16(int16_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_i32(int32_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_i64(int64_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_f8(uint8_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
             size_t scratch_bytes, void *stream);
int bsort_f16(uint16_t *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_f32(float *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);
int bsort_f64(double *keys, uint64_t n, uint32_t flags, void *indices, void *scratch,
              size_t scratch_bytes, void *stream);

/*
 * Segmented (batched) sort: num_segments independent arrays stored back to
 * back in keys[0, n), segment s being [offsets[s], offsets[s+1]).  offsets is
 * a DEVICE array of num_segments+1 int64 with offsets[0] = 0,
 * non-decreasing, offsets[num_segments] = n.  Each segment is sorted as by
 * the single-array call (the same result, bit for bit), in one pass over
 * all of them.  Indices are local to each segment.  Offsets are read and
 * checked on the device: if offsets[0] != 0, offsets[num_segments] != n, or
 * any offset is outside [0, n] or smaller than its predecessor, nothing is
 * sorted (keys and indices are left as they were) and bsort_device_status
 * reports bit 1.  key_type is BSORT_KEY_U/I/F, key_bytes in {1,2,4,8}.
 */
int bsort_segmented(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                    uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                    void *scratch, size_t scratch_bytes, void *stream);

/* Same as bsort_segmented, typed for float32 and int32 keys. */
int bsort_segmented_f32(float *keys, const int64_t *offsets, uint64_t num_segments,
                        uint64_t n, uint32_t flags, void *indices, void *scratch,
                        size_t scratch_bytes, void *stream);
int bsort_segmented_i32(int32_t *keys, const int64_t *offsets, uint64_t num_segments,
                        uint64_t n, uint32_t flags, void *indices, void *scratch,
                        size_t scratch_bytes, void *stream);

/*
 * The sort stopped after its first `levels` global levels, for checking the
 * per-level property of Theorem 3's induction (after the k most significant
 * bits, the array is ordered by its k-bit prefix; Algorithm 2's recursion
 * run breadth first).  Runs the BSORT_PLAIN path (forced on, whatever flags
 * say: every bit is a partition of every part of two keys or more), splits
 * every part on bits w-1 .. w-levels of the order key (the inverse direction
 * on the sign pass of signed and float keys, and on the lower bits of
 * negative floats, as in Algorithms 3-5), and writes the array as it then
 * stands to keys and indices: ordered by the top `levels` bits of the order
 * key, keys with an equal prefix in input order.  levels = 0 writes the
 * input and the identity permutation; levels = w is the full sort.  offsets
 * NULL sorts one array of n keys (num_segments ignored), else as
 * bsort_segmented.  Scratch as for the full sort
 * (bsort_scratch_bytes(key_bytes, n, offsets ? num_segments : 1,
 * indices != NULL, flags | BSORT_PLAIN)).  levels outside [0, w] returns
 * BSORT_EINVAL; other arguments and errors as bsort_sort / bsort_segmented.
 */
int bsort_levels(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                 uint64_t num_segments, uint64_t n, uint32_t flags, int levels, void *indices,
                 void *scratch, size_t scratch_bytes, void *stream);

/*
 * Allocation-free form of bsort_segmented, for callers that cannot allocate
 * device memory or pass a workspace: code recorded under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * result and errors as bsort_segmented, without scratch and scratch_bytes:
 * the scratch is a fixed array of BSORT_NOALLOC_SCRATCH_BYTES bytes in device
 * memory that the library holds on every GPU it runs on, from the first
 * call on that GPU until the process ends.  The call itself allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).
 * A call that would need more scratch than that -- i.e. whenever
 * bsort_scratch_bytes(key_bytes, n, num_segments, indices != NULL, flags)
 * exceeds BSORT_NOALLOC_SCRATCH_BYTES -- returns BSORT_ENOSPACE before
 * anything is enqueued.  All calls on one GPU share its array, which keeps
 * the last call's contents (each call clears what it needs with a kernel):
 * calls that overlap on one GPU (two streams, two threads) race and must be
 * ordered by the caller.  The device status word of bsort_device_status is
 * not available to these calls.
 */
#define BSORT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int bsort_segmented_noalloc(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                            uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                            void *stream);

/* Generic single-array form of the typed entry points above. */
int bsort_sort(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
               void *indices, void *scratch, size_t scratch_bytes, void *stream);

/*
 * Backward of values = x.gather(-1, idx) for rows of length cols (the
 * derivative of a sort is the inverse permutation of its gradient):
 *   grad_in[r, idx[r, j]] = grad_sorted[r, j]     for r < rows, j < cols.
 * elem_bytes 2 (fp16 / bf16, moved bit for bit), 4 (f32) or 8 (f64);
 * indices uint32, or int64 with BSORT_IDX64 in flags.  idx must hold a
 * permutation of 0..cols-1 in every row (as a sort returns it); entries
 * outside [0, cols) are skipped: their output positions keep the caller's
 * bits.  No arithmetic is done on the values.  Rows of up to 8 x 128 KB are
 * staged in LDS (coalesced writes); wider rows are scattered directly.
 * Allocates nothing and does not synchronise.
 */
int bsort_backward_scatter(const void *grad_sorted, const void *indices, uint64_t rows,
                           uint64_t cols, int elem_bytes, void *grad_in, uint32_t flags,
                           void *stream);

/* ---- in-place sort with small scratch ----
 *
 * Keys only.  Every level partitions each live segment in place by
 * exchanging misplaced keys in pairs, as Algorithm 1's swap loop does
 * (Section II; Theorem 5 bounds that loop's auxiliary space), instead of
 * scattering stably into a second buffer.  The scratch then holds only
 * per-level lists and per-tile counts: bsort_inplace_scratch_bytes(...)
 * is O(n / 2048 + num_segments) words, a few percent of the keys.  Equal
 * keys are indistinguishable, so the sorted keys equal those of
 * bsort_sort; no permutation is produced (the exchange is not stable).
 * Each level reads the live keys about twice (a count pass, then the
 * exchange) and writes the exchanged pairs, so this takes about twice as
 * long as bsort_sort without indices.  key_type, key_bytes, offsets and validation as for
 * bsort_sort / bsort_segmented; flags: BSORT_DESCENDING, BSORT_NO_SKIP,
 * BSORT_NO_FINISH (others give BSORT_EINVAL).  Scratch 256-byte aligned.
 */
size_t bsort_inplace_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments,
                                   uint32_t flags);
int bsort_sort_inplace(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                       void *scratch, size_t scratch_bytes, void *stream);
int bsort_segmented_inplace(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                            uint64_t num_segments, uint64_t n, uint32_t flags, void *scratch,
                            size_t scratch_bytes, void *stream);

/* ---- values that travel with the keys ----
 *
 * A key-value sort permutes a payload exactly as the keys: after the sort,
 * values[j] holds the value that came with keys[j] (the stable order of
 * Section II's splits, so equal keys keep their values in input order).
 * value_bytes in {1, 2, 4, 8, 16}; values are moved as raw bits, in place.
 * `values` must be aligned to value_bytes.  `indices` (nullable) receives the
 * permutation as in the sorts above; without it the permutation is kept in
 * scratch.  Flags as for the sorts (BSORT_KEYS_UNCHANGED leaves the keys as
 * they were and permutes only the values).  Scratch: at least
 * bsort_pairs_scratch_bytes(...) bytes, 256-byte aligned.  Offsets as for
 * bsort_segmented: offsets that fail the device-side check leave keys and
 * values as they were (bsort_device_status on this scratch reports bit 1;
 * the indices are then undefined).  Arguments are validated before
 * anything is enqueued.
 */
size_t bsort_pairs_scratch_bytes(int key_bytes, uint64_t n, uint64_t num_segments,
                                 int value_bytes, int with_indices, uint32_t flags);
int bsort_sort_pairs(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                     void *values, int value_bytes, void *indices, void *scratch,
                     size_t scratch_bytes, void *stream);
int bsort_segmented_pairs(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                          uint64_t num_segments, uint64_t n, uint32_t flags, void *values,
                          int value_bytes, void *indices, void *scratch, size_t scratch_bytes,
                          void *stream);

/*
 * Applies a permutation from a sort to another tensor (a second payload):
 *   out[j] = values[base(j) + indices[j]]     for j < n,
 * base(j) = 0 without offsets, else offsets[s] for the segment s holding
 * position j (indices are segment-local, as the sorts return them).
 * value_bytes in {1, 2, 4, 8, 16}; values and out aligned to value_bytes and
 * not overlapping; indices uint32, or int64 with BSORT_IDX64 (the only flag).
 * Positions whose index falls outside their segment are not written.
 */
int bsort_gather(const void *values, int value_bytes, const void *indices,
                 const int64_t *offsets, uint64_t num_segments, uint64_t n, uint32_t flags,
                 void *out, void *stream);

/*
 * The inverse: the backward of a segmented sort (its gradient flows from the
 * sorted order back to each key's input position) or of bsort_gather:
 *   out[base(j) + indices[j]] = values[j]     for j < n,
 * base(j) as above.  For row-shaped sorts bsort_backward_scatter is the
 * faster form; this one takes any segments (ragged rows, the batched sort).
 * Arguments and validation as for bsort_gather; targets outside their
 * segment are skipped (their output keeps the caller's bits), and indices
 * must be a permutation within each segment for every target to be written.
 */
int bsort_scatter(const void *values, int value_bytes, const void *indices,
                  const int64_t *offsets, uint64_t num_segments, uint64_t n, uint32_t flags,
                  void *out, void *stream);

/* ---- keys whose order bits are stored in another layout ----
 *
 * Section III-C notes that other bit arrangements (a sign that is not the
 * top bit, fields in another order) sort with small changes.  bit_order
 * (HOST array of 8 * key_bytes entries, a permutation of 0 .. w-1) lists,
 * from the most significant order bit down, the stored bit that holds it:
 * the key is sorted as the w-bit word whose bit w-1-i is stored bit
 * bit_order[i], read as key_type (for BSORT_KEY_I / BSORT_KEY_F, bit_order[0]
 * is the sign).  The keys' stored layout is kept in the result.  The bits
 * are rearranged in place before and after the sort (with
 * BSORT_KEYS_UNCHANGED the keys come back as they were).  Flags, indices and
 * scratch as for bsort_sort (scratch from bsort_scratch_bytes).
 */
int bsort_sort_layout(void *keys, int key_type, int key_bytes, uint64_t n, uint32_t flags,
                      const uint8_t *bit_order, void *indices, void *scratch,
                      size_t scratch_bytes, void *stream);

/* ---- 128-bit keys ----
 *
 * Section III-C notes that the method carries over to any word size.  Key i
 * is the 16 bytes keys[2i] (low word) and keys[2i+1] (high word), 16-byte
 * aligned; key_type BSORT_KEY_U, BSORT_KEY_I (two's complement) or
 * BSORT_KEY_F (sign | exponent | mantissa, e.g. IEEE binary128).  The order
 * and the stable permutation are those of the sorts above at w = 128.  The
 * keys are sorted most significant word first: the high words (the low
 * words moving with them), then the low words within each run of equal high
 * words.  Flags: BSORT_DESCENDING, BSORT_IDX64, BSORT_KEYS_UNCHANGED (then
 * indices are required) and BSORT_NO_SKIP / BSORT_NO_FINISH, which apply to
 * both word sorts.  Scratch: at least bsort_scratch_bytes128(...) bytes,
 * 256-byte aligned; indices aligned to their width.
 */
size_t bsort_scratch_bytes128(uint64_t n, int with_indices, uint32_t flags);
int bsort_sort128(void *keys, int key_type, uint64_t n, uint32_t flags, void *indices,
                  void *scratch, size_t scratch_bytes, void *stream);

/* ---- launch configurations and the autotuner ----
 *
 * Section V proposes handing partitions to a cache-resident routine once
 * they are small enough; how small is a tuning question.  Here that size is
 * the LDS-finish threshold T, tuned together with the level tile, the block
 * sizes and the grid:
 * a configuration fixes
 *   level kernel: 512 or 256 threads x 8 keys (4 with 8-byte keys) per tile,
 *   finish: 512 x 16, 256 x 16 or 512 x 8 keys per workgroup (halved for
 *           8-byte keys) -- T = 8192, 4096 or 4096 keys of 4 B,
 *   grids: every resident workgroup, or half of them.
 * Configuration 0 is the default.  Every configuration gives the same
 * result, bit for bit; only the time differs. */
int bsort_config_count(void);
/* Static text describing a configuration. */
const char *bsort_config_name(int config);
/* Force one configuration for every later call of this process (-1 clears
 * the override).  For tests and measurements. */
int bsort_config_override(int config);
/* The configuration a call with these parameters would use on the current
 * device (the override, else the tuned one, else 0), or a negative status. */
int bsort_tuned_config(int key_bytes, int with_indices, uint64_t n, uint64_t num_segments);
/* Times every configuration `reps` times on the caller's data (the arguments
 * of bsort_segmented; offsets == NULL means one array of n keys) and keeps
 * the fastest for this device, key width, index mode and size class
 * (log2 of n / num_segments).  On return the buffers hold the sorted result,
 * as after a normal call.  Unlike the sort calls it allocates a copy of the
 * keys (hipMalloc) and synchronizes `stream`; not thread-safe.  Returns the
 * chosen configuration, or a negative status. */
int bsort_autotune(void *keys, int key_type, int key_bytes, const int64_t *offsets,
                   uint64_t num_segments, uint64_t n, uint32_t flags, void *indices,
                   void *scratch, size_t scratch_bytes, void *stream, int reps);
/* Forget every tuned choice. */
void bsort_autotune_reset(void);
/* A tuning cache, so that a later process need not tune again.  save writes
 * every choice of this process to a text file, one line per device type
 * (architecture name and CU count), key width, index mode and size class.
 * load reads such a file and applies its entries to every visible GPU of
 * the same type; the whole file is checked first, and a malformed one
 * changes nothing.  Both return BSORT_OK, BSORT_EINVAL (path unreadable or
 * unwritable, malformed file) or BSORT_EHIP; neither is thread-safe with
 * bsort_autotune. */
int bsort_autotune_save(const char *path);
int bsort_autotune_load(const char *path);

/* ---- HIP graphs ----
 * For callers that sort buffers of the same shape again and again (batched
 * workloads, training loops): the whole launch sequence of one call is
 * recorded once into a HIP graph and replayed with a single launch, so the
 * host submits one command per sort instead of about 3w + 5.  The graph is
 * bound to the pointers, sizes, flags and configuration given at creation;
 * every launch sorts whatever the buffers hold then.  The sequence records no
 * memset or host callback.  Launches that share a scratch buffer must not
 * overlap.  bsort_graph_create validates like bsort_segmented (offsets ==
 * NULL: one array of n keys); it records on a private stream and enqueues
 * nothing. */
typedef struct bsort_graph bsort_graph;
int bsort_graph_create(bsort_graph **graph, void *keys, int key_type, int key_bytes,
                       const int64_t *offsets, uint64_t num_segments, uint64_t n,
                       uint32_t flags, void *indices, void *scratch, size_t scratch_bytes);
int bsort_graph_launch(const bsort_graph *graph, void *stream);
int bsort_graph_destroy(bsort_graph *graph);

/* Text for a status code (for BSORT_EHIP, the last HIP error seen). */
const char *bsort_strerror(int status);

/* Device status word written by the last call that used this scratch:
 * 0 = fine; bit 0 = a part handed to the in-LDS finish exceeded its capacity
 * (an internal error: the result is invalid); bit 1 = the segment offsets
 * failed the device-side check (nothing was sorted); bit 2 = a level tile's
 * precomputed count prefix was inconsistent (an internal error: that tile
 * wrote nothing, the result is invalid); bit 3 = a grid barrier of the tail
 * launch (the levels past the depth chosen from n) waited longer than its
 * bound, 0.2 s, and went on (the result is invalid).  Reads
 * it synchronously on `stream`.  Returns the word, or a negative status. */
int bsort_device_status(const void *scratch, void *stream);

/* ---- instrumentation (benchmarks and tests; not needed to sort) ---- */

/* Work statistics of the last call that used this scratch, read
 * synchronously on `stream`: per level, the keys in live segments, the live
 * segments and the tiles; keys handed to the LDS finish and keys of retired
 * segments copied back.  Any output may be NULL.  Returns the number of
 * levels filled (<= max_levels), or a negative status. */
int bsort_level_stats(const void *scratch, void *stream, uint64_t *live_keys,
                      uint32_t *live_segments, uint32_t *tiles, int max_levels,
                      uint64_t *finish_keys, uint64_t *copy_keys);

/* The same call's byte accounting, per level, read synchronously on
 * `stream`: the live keys whose indices are still the identity (never
 * moved, so the level reads no index for them) and the keys of segments
 * whose split moved them (a split with an empty side moves nothing).  A
 * level reads K bytes per live key and I per live key with real indices,
 * and writes K + I per moved key.  Either output may be NULL.  Returns the
 * number of levels filled (<= max_levels), or a negative status. */
int bsort_level_bytes(const void *scratch, void *stream, uint64_t *iota_keys,
                      uint64_t *moved_keys, int max_levels);

/* While armed, each launch of the global-level kernel (by any call of this
 * process) carries a pair of hipEvents that take the kernel's own start and
 * end times from its dispatch on the call's stream, for the first
 * `capacity` launches.  Levels past the depth chosen from n run in one tail
 * launch, which is not timed.  bsort_timing_read waits for the events,
 * writes each launch's elapsed milliseconds and level index, and restarts
 * the count.  Host-side event objects only; not thread-safe. */
int bsort_timing_arm(int capacity);
int bsort_timing_read(float *ms, int *levels, int capacity);
void bsort_timing_disarm(void);

#ifdef __cplusplus
}
#endif

#endif /* BSORT_H */
