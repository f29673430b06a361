/*
 * ips4o.h -- C ABI of an MI355X (gfx950) in-place super scalar samplesort.
 *
 * The library sorts an array that already lives in device memory, in place,
 * following "In-place Parallel Super Scalar Samplesort (IPS4o)" (Axtmann,
 * Witt, Ferizovic, Sanders; arXiv 1705.02257).  Problem statement (Section 1):
 * arrange A[0..n) so that the keys are non-decreasing under a total order.
 * Extra device memory is O(k * b) per workgroup (Theorem 2), independent of n
 * for a bounded workgroup count; it is owned by the handle and reused.
 *
 * Element types (Section 5, data types):
 *   IPS4O_U64       8-byte unsigned keys.
 *   IPS4O_F64       8-byte IEEE binary64 keys ordered by IEEE 754 totalOrder
 *                   (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN); output
 *                   bit patterns are the input bit patterns, permuted.
 *   IPS4O_PAIR      16-byte records {u64 key, u64 payload}, ordered by key.
 *   IPS4O_QUARTET   32-byte records {u64 w0, w1, w2, u64 payload}, ordered
 *                   lexicographically by (w0, w1, w2).
 *   IPS4O_BYTES100  100-byte records {u8 key[10], u8 payload[90]}, ordered
 *                   lexicographically by the key bytes read as unsigned.
 * Records with equal keys keep their payloads but in no defined order
 * (samplesort is not stable).
 *
 * Pointers: "device" pointers are addresses in the memory of the handle's
 * HIP device (hipMalloc or a torch tensor's data_ptr()); "host" pointers are
 * ordinary process memory.  Alignment: 8 bytes for U64/F64/PAIR/QUARTET,
 * 4 bytes for BYTES100.  The caller owns all arrays it passes.
 *
 * Streams: `hip_stream` is a hipStream_t (NULL = the null stream).  Work is
 * enqueued on that stream, after whatever the caller enqueued before.  The
 * recursion is planned on the host: a level's bucket bounds are copied back
 * as soon as they exist and the next level is enqueued while the current
 * one still runs.  Which calls return after enqueue: ips4o_sort_small and
 * ips4o_sort_segmented_small.  The others (ips4o_sort,
 * ips4o_sort_segmented[_dev], ips4o_distribute[_dev], ips4o_classify,
 * ips4o_select_splitters) wait for their work on the stream before they
 * return, so that device faults are reported by the call itself.  A handle
 * serves one call at a time (it owns
 * the workspace and pinned staging buffers); use one handle per host thread.
 *
 * Errors: every call validates its arguments before touching the device and
 * returns IPS4O_OK (0) or a negative status (ips4o_status_string describes
 * it).  n = 0 and n = 1 are valid no-ops.  IPS4O_ERR_DEVICE_FAULT means a
 * kernel detected an inconsistent state (a bounded wait ran out, counts that
 * do not add up, bucket bounds out of range); the contents of the array are
 * then undefined: blocks held in flight by the permutation may be lost.
 */
#ifndef IPS4O_H
#define IPS4O_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPS4O_OK                    0
#define IPS4O_ERR_INVALID_ARG      -1  /* NULL / misaligned pointer, unknown dtype, bad parameter */
#define IPS4O_ERR_OUT_OF_MEMORY    -2  /* workspace allocation failed */
#define IPS4O_ERR_HIP              -3  /* a HIP runtime call failed */
#define IPS4O_ERR_NOT_SUPPORTED    -4  /* device is not gfx950, or n too large */
#define IPS4O_ERR_DEVICE_FAULT     -5  /* a kernel found an inconsistent state; data undefined */

typedef enum {
    IPS4O_U64 = 0,
    IPS4O_F64 = 1,
    IPS4O_PAIR = 2,
    IPS4O_QUARTET = 3,
    IPS4O_BYTES100 = 4
} ips4o_dtype;

/* Tuning parameters (Section 4, Implementation Details).  A zero field takes
 * the default; a NULL params pointer takes all defaults.
 *   k           buckets of the first level, a power of two in [2, 1024]
 *               (default 256, and 128 for arrays of fewer than 2^27
 *               elements).  Deeper levels choose k adaptively.
 *   block_bytes target block size in bytes; b = max(1, 2^floor(log2(
 *               block_bytes / s))) elements (default 2048, as in the paper).
 *   base_cap    largest subproblem (elements) sorted by the base case
 *               (default and maximum depend on the dtype).
 *   alpha_x100  oversampling factor times 100, used on every level (default:
 *               0.2 * log2 m for a subproblem of m elements, raised to
 *               min(32, sample capacity / k)).
 *   stripes     classification workgroups for the first level of one array
 *               (default: chosen from n; a segmented sort shares its own
 *               count among the segments and ignores this field).
 *   workers     permutation workers (wavefronts) per level, rounded up to a
 *               multiple of four, at most 16380 (default 8192: one round of
 *               the permutation kernel's workgroups on the device).  A level shares them
 *               among its subproblems in groups of four, in proportion to
 *               their blocks, at least one group each (so a level with more
 *               subproblems than groups uses more).
 *   seed        sampling seed (default a fixed constant).
 *   flags       IPS4O_FLAG_* bits.
 *   spin_limit  iterations a kernel may wait for another workgroup before it
 *               reports IPS4O_ERR_DEVICE_FAULT (default 2^16, about 0.1 s;
 *               a legitimate wait lasts microseconds). */
typedef struct {
    uint32_t k;
    uint32_t block_bytes;
    uint32_t base_cap;
    uint32_t alpha_x100;
    uint32_t stripes;
    uint32_t workers;
    uint64_t seed;
    uint32_t flags;
    uint32_t spin_limit;
} ips4o_params;

#define IPS4O_FLAG_NO_SKIP 1u   /* do not skip blocks already in place during the permutation */
#define IPS4O_FLAG_TIMING  2u   /* time every kernel launch with HIP events on the call's stream */
#define IPS4O_FLAG_CHECK   4u   /* debug: verify the phase invariants on the device after
                                   classification and after the permutation (slow) */
#define IPS4O_FLAG_FUSE    8u   /* the base-case kernels clean the buckets of the bins they sort,
                                   instead of a cleanup pass over every bucket of the level (Section
                                   4, Implementation Details: a bucket is sorted as soon as its
                                   cleanup is done).  Same results; slower on gfx950 (the cleanup of
                                   a bin is a chain of dependent memory accesses inside one
                                   workgroup), so it is off by default */
#define IPS4O_FLAG_STRICT  16u  /* strictly in-place hand-off between levels (Section 4.6): after a
                                   level's cleanup every bucket's largest element is moved to its
                                   first entry (ips4o_mark_bucket_max), and the next level is planned
                                   from the buckets a walk over those marks finds with
                                   searchNextLargest (ips4o_search_next_largest), not from the
                                   partition's own boundaries.  The walk does not know which
                                   buckets were equality buckets: the sort's marking also moves each
                                   bucket's smallest element to its last entry, and a bucket above
                                   the base-case capacity whose two ends hold equal keys is taken as
                                   one key value and not partitioned again.  Requires k >= 4;
                                   same results, slower (a read pass and a walk per level, and the
                                   next level is planned only after the cleanup) */

typedef struct ips4o_handle ips4o_handle;

/* Create a handle bound to HIP device `hip_device`.  Fails with
 * IPS4O_ERR_NOT_SUPPORTED unless the device is gfx950.  *out is set to NULL
 * on failure. */
int ips4o_create(int hip_device, ips4o_handle **out);

/* Release the handle and its workspace.  NULL is ignored. */
void ips4o_destroy(ips4o_handle *h);

/* Default parameters of the handle for one element type (an autotuner's
 * choice): every later call on h for that type takes a parameter field the
 * call leaves 0 (or passes no params) from here, before the library's own
 * default; flags are never defaulted.  params = NULL clears them.  Errors:
 * IPS4O_ERR_INVALID_ARG for a NULL handle, an unknown dtype or parameters
 * ips4o_sort would refuse. */
int ips4o_set_default_params(ips4o_handle *h, int dtype, const ips4o_params *params);

/* Device bytes of workspace the handle holds after the calls so far. */
int ips4o_workspace_bytes(const ips4o_handle *h, size_t *bytes);

/* Upper bound of the device workspace (bytes, into *bytes on the host) that
 * a fresh handle holds after ips4o_sort of n elements of `dtype` with these
 * parameters, after ips4o_sort_segmented over n elements in all, or after
 * ips4o_distribute of n elements; computed on the host from n, the element
 * type and the parameters (with h, its default parameters and CU count;
 * h may be NULL: 256 CUs), before any device work.  Theorem 2 bounds the
 * extra space by O(k b) per thread; here a level's stripe buffers stay
 * within max(n/8 elements, 2 k b per CU) (or one stripe per subproblem,
 * when that needs more), so for large n the bound is about n*s/8 plus
 * O(n/base_cap) of per-bucket state.  A handle keeps what it has allocated:
 * after several calls it holds at most the largest of their bounds.
 * Errors: IPS4O_ERR_INVALID_ARG (NULL bytes, unknown dtype, bad params),
 * IPS4O_ERR_NOT_SUPPORTED (n beyond the limit of ips4o_sort). */
int ips4o_workspace_size(const ips4o_handle *h, int dtype, uint64_t n, const ips4o_params *params,
                         size_t *bytes);

/* Sort d_data[0..n) of `dtype` in place (the whole method: sampling,
 * classification, block permutation, cleanup, recursion, base case;
 * Sections 3 and 4).  d_data: device pointer to n elements.
 * Size limit: n < 2^40, and a subproblem must have fewer than 2^25 - 2^16
 * blocks (the permutation's pointer word, Section 4.2): a level whose
 * largest subproblem has more doubles its block size, up to 2048 words
 * (16 KiB), so n stays below about 2^36 u64/f64 keys, 2^35 pairs, 2^34
 * quartets and 2^31 100-byte records; beyond: IPS4O_ERR_NOT_SUPPORTED. */
int ips4o_sort(ips4o_handle *h, void *d_data, uint64_t n, int dtype,
               const ips4o_params *params, void *hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ips4o_sort of a small
 * array that allocates nothing.  d_data[0..n) (device) is sorted in place as
 * one base-case bin, for n <= ips4o_small_max(dtype) elements (16384 u64/f64
 * keys, 8192 pairs, 4096 quartets or 100-byte records); larger n returns
 * IPS4O_ERR_NOT_SUPPORTED before any device work.  The bin list, the
 * counters and the record scratch live in a fixed 512 KiB device array per
 * GPU that the library holds until the process ends, set up by a kernel on
 * `hip_stream` (no memset, no host staging); the call returns after
 * enqueueing its kernels and makes no hipMalloc, hipFree or other
 * allocating call.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (different streams or threads) race; calls on one
 * stream are ordered and safe. */
int ips4o_sort_small(ips4o_handle *h, void *d_data, uint64_t n, int dtype, void *hip_stream);

/* Largest n ips4o_sort_small accepts for `dtype` (0 for an unknown dtype). */
uint64_t ips4o_small_max(int dtype);

/* Segmented sort of many small segments planned on the device, so that it
 * can be captured in a HIP graph and replayed (the recursion of Section 4
 * reduced to its base case: every segment is one bin).  Segment i is
 * d_data[d_offsets[i] .. d_offsets[i+1]) (d_offsets: device, 8-byte aligned,
 * num_segments + 1 offsets), each at most ips4o_small_max(dtype) elements.
 * Kernels on hip_stream turn the table into bins and sort them; the call
 * returns after enqueue, with no host round trip.  A segment above the
 * capacity, or a decreasing pair of offsets, is left as it is and the next
 * ips4o_sync(h, hip_stream) returns IPS4O_ERR_DEVICE_FAULT with fault bit 128
 * (ips4o_last_stats).  The first call for a segment count allocates the bin
 * lists (and, for records, the scratch) on the handle: make it outside a
 * capture; calls for as many segments or fewer then allocate nothing.  One
 * handle serves one call at a time. */
int ips4o_sort_segmented_small(ips4o_handle *h, void *d_data, int dtype, const uint64_t *d_offsets,
                               uint32_t num_segments, void *hip_stream);

/* Sort each of num_segments independent segments of one array in place:
 * segment i is d_data[h_offsets[i] .. h_offsets[i+1]).  The recursion of
 * Section 4 already treats the buckets of a level as independent
 * subproblems; here the caller's segments are the subproblems of the top
 * level, and every level runs one set of launches over all of them.
 * Segments within the base-case capacity go straight to the base case,
 * each on its own; larger ones are distributed with k chosen from their
 * size (at most params->k).  Elements outside [h_offsets[0],
 * h_offsets[num_segments]) are not touched.
 * h_offsets: host pointer to num_segments + 1 non-decreasing element
 * offsets, read before the call returns (NULL allowed when num_segments is
 * 0).  d_data: device pointer holding h_offsets[num_segments] elements.
 * Errors: IPS4O_ERR_INVALID_ARG for decreasing offsets or the checks of
 * ips4o_sort; IPS4O_ERR_NOT_SUPPORTED when h_offsets[num_segments] exceeds
 * the size limit of ips4o_sort.
 * Same stream and handle rules as ips4o_sort. */
int ips4o_sort_segmented(ips4o_handle *h, void *d_data, int dtype, const uint64_t *h_offsets,
                         uint32_t num_segments, const ips4o_params *params, void *hip_stream);

/* ips4o_sort_segmented with the offset table in device memory: d_offsets
 * (device pointer, 8-byte aligned) holds num_segments + 1 non-decreasing
 * element offsets; it is copied to the host in stream order (so earlier
 * work on hip_stream may write it) before the recursion is planned there.
 * Errors and return as for ips4o_sort_segmented. */
int ips4o_sort_segmented_dev(ips4o_handle *h, void *d_data, int dtype, const uint64_t *d_offsets,
                             uint32_t num_segments, const ips4o_params *params, void *hip_stream);

/* One distribution step with caller-given splitters (Section 4: local
 * classification, block permutation, cleanup; no sampling, no recursion).
 * h_splitters: host pointer to num_splitters whole elements of `dtype`
 * whose keys are non-decreasing; only their keys are read.
 * equality_buckets: 0 -> K = num_splitters + 1 buckets with
 * s_{i-1} <= e < s_i (Section 3); 1 -> duplicates are removed and K = 2u + 1
 * buckets over the u unique keys, equal keys in buckets of their own
 * (Section 4, "The Case of Many Identical Keys").
 * h_bounds_out: host pointer to K + 1 uint64 values receiving the bucket
 * boundaries (bounds[0] = 0, bounds[K] = n).  On return d_data[bounds[i] ..
 * bounds[i+1]) holds exactly the elements of bucket i, in no defined order.
 * *num_buckets_out (host, may be NULL) receives K.
 * Limits: 1 <= num_splitters <= 511 (K <= 1023). */
int ips4o_distribute(ips4o_handle *h, void *d_data, uint64_t n, int dtype,
                     const void *h_splitters, uint32_t num_splitters, int equality_buckets,
                     uint64_t *h_bounds_out, uint32_t *num_buckets_out,
                     const ips4o_params *params, void *hip_stream);

/* ips4o_distribute with the splitters and the results in device memory:
 * d_splitters (device, aligned for dtype) holds num_splitters elements
 * whose keys are non-decreasing (copied to the host in stream order, where
 * the search tree is built); d_bounds_out (device, 8-byte aligned) receives
 * K + 1 uint64 bucket boundaries -- room for 2 * num_splitters + 2 is
 * enough -- and *d_num_buckets_out (device, may be NULL) receives K.  The
 * call returns once they are written.  Errors as for ips4o_distribute. */
int ips4o_distribute_dev(ips4o_handle *h, void *d_data, uint64_t n, int dtype, const void *d_splitters,
                         uint32_t num_splitters, int equality_buckets, uint64_t *d_bounds_out,
                         uint32_t *d_num_buckets_out, const ips4o_params *params, void *hip_stream);

/* Bucket index of every element for caller-given splitters: #{s_i <= e}
 * (Section 3), with the equality test of Section 4, computed by the same
 * code the distribution step classifies with (a table over the splitters'
 * leading words narrows each key to a few splitters, a branch-free binary
 * search finishes; the result is the implicit search tree's).
 * Splitter rules as for ips4o_distribute.  d_bucket_out: device pointer to n
 * uint32 values.  d_data is not modified. */
int ips4o_classify(ips4o_handle *h, const void *d_data, uint64_t n, int dtype,
                   const void *h_splitters, uint32_t num_splitters, int equality_buckets,
                   uint32_t *d_bucket_out, void *hip_stream);

/* The sampling step of a sort's first level (Section 3 and Section 4,
 * "Sampling" and "Implementation Details"): alpha*k - 1 elements drawn at
 * positions floor(h_i * n / 2^64), h_i the i-th output of splitmix64 started
 * at `seed` (params->seed, or the default); the sample is sorted and the
 * splitters s_i = sample[i*alpha - 1], i = 1..k-1, are picked; duplicates are
 * removed and equality buckets switched on when there were any.  The first
 * level's buffers hold min(2k, 1024) buckets: should the u unique splitters
 * need more (2u + 1 > min(2k, 1024), only for k = 1024), every second pick of
 * the same sorted sample is used instead and equality buckets stay on.
 * h_splitters_out: host buffer of k - 1 elements of `dtype` (k: the call's,
 * else the handle's default from ips4o_set_default_params; whole elements,
 * only the key fields meaningful) receiving the u unique splitters;
 * *num_unique_out and *equality_out (host) receive u and the flag.
 * d_data is not modified.  Requires n >= 1. */
int ips4o_select_splitters(ips4o_handle *h, const void *d_data, uint64_t n, int dtype,
                           const ips4o_params *params, void *h_splitters_out,
                           uint32_t *num_unique_out, int *equality_out, void *hip_stream);

/* The argument checks that ips4o_sort applies before any device work,
 * without a handle: returns IPS4O_OK, or the status ips4o_sort would return
 * for these arguments (d_data is only inspected for NULL and alignment). */
int ips4o_check_args(const void *d_data, uint64_t n, int dtype, const ips4o_params *params);

/* The argument checks that ips4o_sort_segmented applies before any device
 * work, without a handle: the offsets (NULL allowed only for 0 segments,
 * non-decreasing), then those of ips4o_check_args for the
 * h_offsets[num_segments] elements. */
int ips4o_check_segments(const void *d_data, int dtype, const uint64_t *h_offsets, uint32_t num_segments,
                         const ips4o_params *params);

/* The marking the strictly in-place recursion needs from a partition
 * (Section 4.6, From Almost In-Place to Strictly In-Place): for every bucket
 * b < num_buckets, elements [d_bounds[b], d_bounds[b+1]) of d_data, the first
 * element with the largest key of the bucket trades places with the
 * bucket's first element (buckets of fewer than two elements are left
 * alone).  d_bounds: device pointer to num_buckets + 1 positions (8-byte
 * aligned), non-decreasing and at most n; others are skipped and reported
 * as IPS4O_ERR_DEVICE_FAULT with fault bit 256.  Waits for the stream.
 * Buckets may be in any order and need not cover the array. */
int ips4o_mark_bucket_max(ips4o_handle *h, void *d_data, uint64_t n, int dtype, const uint64_t *d_bounds,
                          uint32_t num_buckets, void *hip_stream);

/* searchNextLargest (Section 4.6) for `count` positions: d_out[q] = the first
 * position j > d_pos[q], j < n, whose key is larger than the key of
 * d_data[d_pos[q]], or n if there is none (also for d_pos[q] >= n).  Each
 * query is an exponential search followed by a 64-way search, which finds
 * that first position whenever the positions after d_pos[q] holding larger
 * keys form a suffix of [d_pos[q]+1, n), as after a partition marked by
 * ips4o_mark_bucket_max when d_pos[q] is a bucket's first entry; for other
 * inputs the result is some position in (d_pos[q], n] whose key is larger
 * (or n).  d_pos, d_out: device pointers to `count` uint64 (8-byte aligned).
 * Reads only d_data[0, n).  Waits for the stream. */
int ips4o_search_next_largest(ips4o_handle *h, const void *d_data, uint64_t n, int dtype, const uint64_t *d_pos,
                              uint64_t count, uint64_t *d_out, void *hip_stream);

/* The checks ips4o_distribute and ips4o_classify apply to caller-given
 * splitters (host pointer to num_splitters elements of `dtype`): count in
 * [1, 511], keys non-decreasing, equality_buckets 0 or 1. */
int ips4o_check_splitters(const void *h_splitters, uint32_t num_splitters, int dtype,
                          int equality_buckets);

/* Wait for the stream and report a device fault raised by an earlier call. */
int ips4o_sync(ips4o_handle *h, void *hip_stream);

/* Static text for a status code. */
const char *ips4o_status_string(int status);

/* Statistics of the most recent ips4o_sort / ips4o_distribute on `h`
 * (host values, filled when the call returns):
 *   levels         distribution levels run
 *   fault_bits     device error bits of the last call (0 = none): 1 a wait
 *                  expired, 2 cleanup counts disagreed, 4 a permutation
 *                  pointer left its bucket, 8 empty-block fix counts
 *                  disagreed; with IPS4O_FLAG_CHECK also 16 a full block
 *                  mixed buckets, 32 recounted buckets differed, 64 a placed
 *                  block held another bucket; 128 ips4o_sort_segmented_small got a
 *                  segment above the capacity or decreasing offsets; 256
 *                  bucket bounds out of range (ips4o_mark_bucket_max), or a
 *                  strictly in-place walk found more buckets than the
 *                  partition made
 *   block_moves    blocks written by the permutations (all levels)
 *   block_skips    blocks found already in place and left there
 *   elements_base  elements sorted by the base case
 *   elements_distributed  sum over levels of the elements partitioned */
typedef struct {
    uint32_t levels;
    uint32_t fault_bits;
    uint64_t block_moves;
    uint64_t block_skips;
    uint64_t elements_base;
    uint64_t elements_distributed;
} ips4o_stats;

int ips4o_last_stats(const ips4o_handle *h, ips4o_stats *out);

/* Per-kernel device time of the most recent ips4o_sort / ips4o_distribute
 * made with IPS4O_FLAG_TIMING (zeros otherwise), from HIP events recorded
 * around each launch on the call's stream.  out[] has IPS4O_KERNEL_KINDS
 * entries in this order: sample, classify, scan, fix_empty, permute,
 * cleanup, basecase, mark (the bucket maxima and the walk of
 * IPS4O_FLAG_STRICT).  alg_bytes is the data the launches had to move by the
 * method's definition: 2*s per element classified, per element of a moved
 * block (permutation and empty-block fix), per element placed by cleanup and
 * per element sorted by the base case; s per element marked. */
#define IPS4O_KERNEL_KINDS 8
typedef struct {
    uint32_t launches;
    uint32_t reserved;
    double ms;
    double alg_bytes;
} ips4o_kernel_stat;

int ips4o_last_kernel_stats(const ips4o_handle *h, ips4o_kernel_stat *out);

/* The same device time and algorithmic bytes per pass over the data of the
 * most recent call made with IPS4O_FLAG_TIMING (none otherwise): one entry
 * per distribution level (Section 4: sampling, classification, empty-block
 * movement, permutation and cleanup of every subproblem of that level),
 * then one for the base case if it ran (base_case = 1).  elements: the
 * elements the pass partitioned or sorted.  Up to max_passes entries are
 * written to out (host); *num_passes (host) receives the number of passes
 * the call made. */
typedef struct {
    uint32_t launches;
    uint32_t base_case;
    double ms;
    double alg_bytes;
    uint64_t elements;
} ips4o_pass_stat;

int ips4o_last_pass_stats(const ips4o_handle *h, ips4o_pass_stat *out, uint32_t max_passes,
                          uint32_t *num_passes);

#ifdef __cplusplus
}
#endif

#endif /* IPS4O_H */
