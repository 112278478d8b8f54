/*
 * corank_merge.h -- C ABI of the MI355X (gfx950) stable-merge library.
 *
 * The operations follow C. Siebert and J. L. Traeff, "Perfectly
 * load-balanced, optimal, stable, parallel merge" (arXiv:1303.4312):
 *
 *   stable merge (Sections 1 and 2): C = stable_merge(A, B) for sorted A (m
 *     elements) and B (n elements); C has m + n elements in nondecreasing
 *     key order, and among equal keys every element of A comes before every
 *     element of B, each side keeping its input order.
 *   co-rank (Section 2, Lemma 1, Algorithm 1): for an output rank i with
 *     0 <= i <= m + n, the unique (j, k) with j + k = i such that the first
 *     i outputs of the stable merge are exactly A[0..j) and B[0..k).
 *   parallel merge (Section 3, Algorithm 2, Proposition 2): the output is
 *     cut into equal blocks, both ends of every block are co-ranked, and each
 *     block is merged on its own; every block merges exactly the same number
 *     of elements (the last may be shorter).
 *
 * Conventions shared by every call:
 *   - Indices are 0-based; sizes are element counts (uint64_t).
 *   - Keys are uint32, uint64 or float32 (cm_key_type).  float32 keys are
 *     compared as IEEE floats, so -0.0 and +0.0 are equal keys (the tie rule
 *     orders them and their bits are copied unchanged); NaN keys are not
 *     allowed.  Payloads, where taken, are uint32 and move with their key.
 *   - Inputs must already be sorted (nondecreasing).  This is a precondition
 *     the merge calls do not check; cm_check_sorted checks it on request.
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer,
 *     including the workspace; the library keeps no pointer after a call
 *     returns and allocates nothing on the merge path.
 *   - Calls that take a stream enqueue work on it and return at once.
 *     Argument errors are found before anything is enqueued and leave the
 *     stream untouched.  A failed kernel launch returns CM_EHIP.
 *   - Output arrays must not overlap input arrays (CM_EALIAS).  A and B may
 *     overlap each other (both are only read).  A null pointer with a
 *     nonzero length is CM_EINVAL.  Zero lengths are valid.
 *   - Every device array holds fewer than 2^48 elements (CM_EINVAL
 *     otherwise), and a call's tile count stays below 2^31.
 */
#ifndef CORANK_MERGE_H
#define CORANK_MERGE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every int-valued call. */
enum cm_status {
    CM_OK = 0,
    CM_EINVAL = -1,    /* bad argument: null pointer, bad size, bad handle */
    CM_ERANGE = -2,    /* rank outside [0, m + n] */
    CM_EDTYPE = -3,    /* unknown key type */
    CM_EALIAS = -4,    /* an output overlaps an input */
    CM_ENOSPC = -5,    /* workspace smaller than the *_workspace_size result, or a
                          server request larger than the server's arena */
    CM_EHIP = -6,      /* a HIP runtime call or kernel launch failed */
    CM_EUNSORTED = -7, /* cm_check_sorted: the array is not sorted */
    CM_ECONFIG = -8,   /* unknown tile configuration */
    CM_EBUSY = -9,     /* server: every request slot is taken */
    CM_ECANCELED = -10, /* server: request dropped at shutdown without running */
    CM_ESTALE = -11     /* tuning file made for another device, HIP runtime or
                           library build (or with no such identity) */
};

/*
 * Key types.  The first three merge and sort in nondecreasing key order; the
 * _DESC types hold the same bits and use the reversed order (nonincreasing;
 * ties still go A first in a merge and keep input order in a sort).  Float
 * keys compare as IEEE values either way (-0.0 == +0.0; no NaN).
 */
enum cm_key_type {
    CM_KEY_U32 = 0,
    CM_KEY_U64 = 1,
    CM_KEY_F32 = 2,
    CM_KEY_U32_DESC = 3,
    CM_KEY_U64_DESC = 4,
    CM_KEY_F32_DESC = 5
};

/* Human-readable name of a status code (static string, never NULL). */
const char *cm_status_string(int status);

/* Library ABI version (increases when a signature changes). */
int cm_version(void);

/*
 * Co-rank on host arrays: Lemma 1 / Algorithm 1 (Section 2), run on the CPU.
 * A (m keys) and B (n keys) are host arrays of key type `key_type`.
 * On CM_OK, *j and *k hold the co-ranks of rank i (j + k = i).
 * Errors: CM_ERANGE if i > m + n; CM_EINVAL for a null pointer with a
 * nonzero length or null j/k; CM_EDTYPE for an unknown key type.
 */
int cm_co_rank_host(int key_type, uint64_t i,
                    const void *A, uint64_t m, const void *B, uint64_t n,
                    uint64_t *j, uint64_t *k);

/*
 * Co-rank of q ranks on device arrays: Algorithm 1 (Section 2), one GPU
 * thread per rank.  ranks[r] (device, q entries) are output ranks; the call
 * writes j_out[r] (device, q entries) with the A co-rank of ranks[r]; the B
 * co-rank is ranks[r] - j_out[r].  A rank above m + n cannot be reported
 * synchronously (the ranks live on the device): its j_out entry is set to
 * UINT64_MAX.
 * Errors (synchronous): CM_EINVAL, CM_EDTYPE, CM_EALIAS (j_out overlapping
 * ranks, A or B), CM_EHIP.
 */
int cm_co_rank(int key_type, const uint64_t *ranks, uint64_t q,
               const void *A, uint64_t m, const void *B, uint64_t n,
               uint64_t *j_out, hipStream_t stream);

/*
 * Workspace bytes a single merge of m and n elements needs: one uint64
 * co-rank per block boundary (Algorithm 2) and one per coarse boundary of
 * the two-level boundary pass, sized for the smallest block of any tile
 * configuration (so one workspace serves every configuration), each array
 * rounded up to 256 bytes.
 * Returns 0 for m + n = 0 or an unknown key type.
 */
size_t cm_merge_workspace_size(int key_type, int with_payload, uint64_t m, uint64_t n);

/*
 * Stable merge of keys (Sections 1-3).  A: m keys, B: n keys, C: m + n keys,
 * all device arrays of key type `key_type`.  workspace: device memory of at
 * least cm_merge_workspace_size(key_type, 0, m, n) bytes (may be NULL when
 * that size is 0); its contents are scratch.
 * Errors: CM_EINVAL, CM_EDTYPE, CM_EALIAS, CM_ENOSPC, CM_EHIP.
 */
int cm_stable_merge(int key_type,
                    const void *A, uint64_t m, const void *B, uint64_t n,
                    void *C, void *workspace, size_t workspace_bytes,
                    hipStream_t stream);

/*
 * Stable merge of key + payload pairs (Sections 1-3).  Like cm_stable_merge;
 * A_val (m), B_val (n) and C_val (m + n) are uint32 device arrays and every
 * payload ends up beside its key.  Keys and payloads are separate arrays
 * (structure of arrays).  workspace: cm_merge_workspace_size(key_type, 1,
 * m, n) bytes.
 * Errors: CM_EINVAL, CM_EDTYPE, CM_EALIAS, CM_ENOSPC, CM_EHIP.
 */
int cm_stable_merge_pairs(int key_type,
                          const void *A, const uint32_t *A_val, uint64_t m,
                          const void *B, const uint32_t *B_val, uint64_t n,
                          void *C, uint32_t *C_val,
                          void *workspace, size_t workspace_bytes,
                          hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the merge
 * of cm_stable_merge_pairs (payload pointers all NULL: cm_stable_merge)
 * with no workspace argument.  Its block co-ranks go to a scratch array of
 * CM_NOALLOC_SCRATCH_BYTES (4 MiB) in the library's device code, one per
 * GPU, held from the first call on that GPU until the process ends.  The
 * call allocates nothing and runs the same kernels with the same tile and
 * boundary choice, so the results are those of cm_stable_merge_pairs.
 * Limit: merges whose cm_merge_workspace_size fits the scratch array (up to
 * about 4.4e8 outputs); larger ones are refused with CM_ENOSPC before
 * anything is enqueued.  Every call on one GPU shares that GPU's array and
 * leaves its contents behind (each call writes every co-rank it reads, so
 * nothing needs clearing): calls whose kernels may overlap on one GPU (on
 * different streams, or from different threads) race and must not be
 * made.  Errors: those of cm_stable_merge_pairs, and CM_EHIP if the
 * scratch array's device address cannot be found.
 */
#define CM_NOALLOC_SCRATCH_BYTES (4u << 20)
int cm_stable_merge_pairs_noalloc(int key_type,
                                  const void *A, const uint32_t *A_val, uint64_t m,
                                  const void *B, const uint32_t *B_val, uint64_t n,
                                  void *C, uint32_t *C_val, hipStream_t stream);

/*
 * Stable merge of (key, uint64 payload) pairs (Sections 1-3): as
 * cm_stable_merge_pairs with 8-byte payloads (A_val: m, B_val: n, C_val:
 * m + n uint64 device arrays), moved by the same kernels; for 8-byte
 * records (a pointer, an index, two packed 4-byte fields) without an
 * origin-code pass and a gather.  Same workspace
 * (cm_merge_workspace_size(key_type, 1, m, n)), tile and boundary choice
 * as cm_stable_merge_pairs, except that boundary mode 3 (the streaming
 * kernel, 4-byte payloads only) runs as mode 2.
 * Errors: CM_EINVAL, CM_EDTYPE, CM_EALIAS, CM_ENOSPC, CM_EHIP.
 */
int cm_stable_merge_pairs64(int key_type,
                            const void *A, const uint64_t *A_val, uint64_t m,
                            const void *B, const uint64_t *B_val, uint64_t n,
                            void *C, uint64_t *C_val,
                            void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/*
 * Batch of separately allocated merges (each one instance of the problem of
 * Section 2), run in one pass of Algorithm 2: every merge is cut into
 * blocks of the batch's block size, blocks never span two merges, and one
 * kernel merges all blocks of all merges.  Used to serve many requests
 * with one launch.
 *
 * cm_merge_desc describes merge r: A (m keys), B (n keys), C (m + n keys)
 * are device key arrays; A_val, B_val, C_val uint32 device payload arrays
 * (all three NULL when with_payload is 0).  first_block is filled by
 * cm_batch_prepare.
 *
 * cm_batch_prepare(key_type, with_payload, descs, count, &total_blocks):
 *   host-only; fills descs[r].first_block (blocks of the merges before r)
 *   for the block size the batch call will use, and the total block count.
 * cm_batch_workspace_size(total_blocks, count): workspace bytes (one uint64
 *   co-rank per block end of every merge, one per 16th of those for the
 *   two-level pass, one uint32 per block and one per block end naming its
 *   merge, and a copy of the count descriptors), each part rounded up to
 *   256.
 * cm_stable_merge_batch(key_type, with_payload, descs_host, descs_dev,
 *   count, total_blocks, workspace, workspace_bytes, stream):
 *   descs_host is the prepared host array (used to check the arguments);
 *   descs_dev is a byte-identical copy of it that the device reads: device
 *   memory, or host memory mapped for the device (hipHostMalloc; its
 *   device address), so that no upload is needed; the call's first kernel
 *   copies it into the workspace, and it must stay alive and unchanged
 *   until the stream has run the call.  With count <= CM_BATCH_INLINE_MAX,
 *   descs_dev may be NULL: the descriptors then travel in the kernel
 *   arguments (copied at the call).  No output may overlap an input or
 *   another output of the batch.  count = 0 is a no-op.  Block ends are
 *   co-ranked as the boundary mode says (cm_set_partition, or the tuning
 *   table's entry for operation 2): 0 = one thread per block end over its
 *   merge's diagonal; 1, 2 = two levels (every 64th block end of the whole
 *   batch searched by 64 or 16 lanes over its merge, the others by
 *   bisection between the nearest of those in the same merge, or the
 *   merge's own ends); 4 = no pass, every block co-ranks its two ends
 *   itself (one wave each; a batch of at most CM_BATCH_INLINE_MAX merges
 *   then runs as a single kernel launch); 3 is taken as 2.
 * Errors: CM_EDTYPE, CM_EINVAL (null pointer with nonzero length, counts
 *   or first_block that do not match cm_batch_prepare), CM_EALIAS,
 *   CM_ENOSPC, CM_EHIP.
 */
#define CM_BATCH_INLINE_MAX 16
typedef struct cm_merge_desc {
    const void *A;
    const uint32_t *A_val;
    uint64_t m;
    const void *B;
    const uint32_t *B_val;
    uint64_t n;
    void *C;
    uint32_t *C_val;
    uint64_t first_block;
} cm_merge_desc;

int cm_batch_prepare(int key_type, int with_payload, cm_merge_desc *descs, uint32_t count,
                     uint64_t *total_blocks);
size_t cm_batch_workspace_size(uint64_t total_blocks, uint32_t count);
int cm_stable_merge_batch(int key_type, int with_payload,
                          const cm_merge_desc *descs_host, const cm_merge_desc *descs_dev,
                          uint32_t count, uint64_t total_blocks,
                          void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Workspace bytes for a segmented merge of num_seg segments with total_a
 * and total_b elements: a status word, and per block boundary and per
 * coarse boundary one uint64 co-rank and one uint32 segment index (sized
 * for the smallest block of any configuration), each part rounded up to
 * 256 bytes.
 */
size_t cm_segmented_workspace_size(int key_type, int with_payload,
                                   uint64_t total_a, uint64_t total_b,
                                   uint64_t num_seg);

/*
 * Batch of num_seg independent stable merges in one pass (each segment is
 * one instance of the problem of Section 2; the batch is partitioned as one
 * merge under the order (segment, key), so blocks of Algorithm 2 run across
 * segment ends and every block still merges the same number of elements).
 *
 * Segment s merges A[a_off[s] .. a_off[s+1]) with B[b_off[s] .. b_off[s+1])
 * into C[a_off[s] + b_off[s] .. a_off[s+1] + b_off[s+1]).
 *   A, B, C: device key arrays (total_a, total_b, total_a + total_b keys).
 *   A_val, B_val, C_val: uint32 device payload arrays, or all three NULL.
 *   a_off, b_off: device uint64 arrays of num_seg + 1 nondecreasing entries
 *     with a_off[0] = b_off[0] = 0, a_off[num_seg] = total_a and
 *     b_off[num_seg] = total_b (the host passes total_a and total_b because
 *     the offsets are on the device).  Empty sides are allowed.  The offsets
 *     are checked on the device before any merging: if they break these
 *     rules, C is left unwritten and the first uint32 of the workspace is
 *     nonzero after the stream completes (it is zero after a good call).
 *   workspace: cm_segmented_workspace_size(...) bytes of device memory.
 * Errors: CM_EINVAL (also num_seg = 0 with nonzero totals, or num_seg at or
 * above 2**32), CM_EDTYPE, CM_EALIAS, CM_ENOSPC, CM_EHIP.
 */
int cm_stable_merge_segmented(int key_type,
                              const void *A, const uint32_t *A_val, const uint64_t *a_off,
                              uint64_t total_a,
                              const void *B, const uint32_t *B_val, const uint64_t *b_off,
                              uint64_t total_b,
                              uint64_t num_seg,
                              void *C, uint32_t *C_val,
                              void *workspace, size_t workspace_bytes,
                              hipStream_t stream);

/*
 * Check on the device that a key array is sorted (the precondition of
 * Section 2).  flag: device uint32 that the call first sets to 0 and that
 * ends up nonzero if some X[x-1] > X[x].  Read it after the stream is done.
 * Errors: CM_EINVAL, CM_EDTYPE, CM_EHIP.
 */
int cm_check_sorted(int key_type, const void *X, uint64_t len, uint32_t *flag,
                    hipStream_t stream);

/*
 * Tile configurations.  A configuration fixes the threads per workgroup (NT)
 * and the outputs per thread (E); one block of Algorithm 2 is NT * E
 * outputs.  Every configuration gives bit-identical results; they differ
 * only in speed.  cm_config_count() configurations are numbered from 0.
 *   cm_config_info: NT and E of configuration id (CM_ECONFIG if unknown).
 *   cm_set_config: the configuration used by the merge calls
 *     for (key_type, with_payload) in this process (not thread-safe against
 *     concurrent merges; set it before launching); config_id -1 returns the
 *     pair to the per-operation defaults.  Until cm_set_config is
 *     called for (key_type, with_payload), or after it is called with -1,
 *     single merges with payloads use configuration 0 (256 x 7), those
 *     without payloads 6 (256 x 9), both 7 (512 x 11) where the automatic
 *     boundary mode skips the pass from 2^21 outputs (2^22 without
 *     payloads); sorts use 6 (256 x 9; 1, 256 x 11, for 4-byte keys
 *     without payloads); segmented batches and batches of separate merges
 *     2 (256 x 15).
 *   cm_set_search: co-rank search of the per-thread searches inside a
 *     block and of the one-level boundary pass: 0 = Algorithm 1, 1 = plain
 *     bisection over the diagonal (default).  Both return the unique pair
 *     of Lemma 1.
 *   cm_set_partition: how block boundaries are co-ranked (Algorithm 2):
 *     -1 (default) = automatic: mode 4 for single merges of fewer than
 *     2^24 outputs (from 2^21 outputs with payloads, 2^22 keys only, with
 *     the 512 x 11 tile unless a configuration is set), else mode 2;
 *     0 = one GPU thread per boundary over the whole diagonal; 1 = two levels: every coarse boundary by a whole wave
 *     with a 64-ary search, then the others by bisection between their two
 *     coarse neighbours; 2 = two levels with 16 lanes (a 16-ary search) per
 *     coarse boundary; 3 = Algorithm 2 with one block per resident workgroup:
 *     only those P + 1 boundaries are co-ranked (a whole wave each), and
 *     each workgroup merges its whole block in steps through LDS ring
 *     buffers (single merges only); 4 = no boundary pass: every block
 *     co-ranks its own two ends (a whole wave each, 64-ary search) and then
 *     merges, as Algorithm 2 has every processing element do (single merges
 *     only; saves a launch on small merges).  The segmented batch uses two
 *     levels (segment search and co-rank narrowed by coarse neighbours) for
 *     any nonzero mode and one level for 0; the batch of separate merges
 *     takes modes 0, 1, 2 and 4 as above (3 as 2) and, automatically,
 *     mode 4 when it has at most CM_BATCH_INLINE_MAX merges, each of fewer
 *     than 2^24 outputs, else mode 2 (cm_tuning_get reports 2 for it: the
 *     rule depends on the merges).  All give the same results.
 *   cm_set_coarse_stride: blocks between coarse boundaries of the two-level
 *     pass (default 64; at least 16).
 *   cm_set_fine_lanes: lanes that search each boundary of the two-level
 *     pass's fine step inside its coarse window: 1 = bisection, 2 or 4 = a
 *     ternary or 5-ary search (fewer dependent rounds, more lanes).
 *   cm_set_block_order: the order in which a single merge, a batch of
 *     separate merges, a sort pass and cm_copy_tiles hand blocks to the
 *     chip's 8 XCDs (workgroups reach the XCDs round-robin), so that
 *     neighbouring blocks, which share the cache lines at their window
 *     edges, run under one L2: c >= 2 (default 32) = runs of c blocks per
 *     XCD, the XCDs side by side (the blocks in flight stay within one
 *     address range); 1 = one contiguous run per XCD; 0 = workgroup order.
 *     At most 2^20 (else CM_EINVAL).  Segmented batches keep workgroup
 *     order.
 *   cm_set_grid: workgroups of every block-merge kernel launch (single
 *     merges, segmented batches, batches of separate merges, sort runs and
 *     passes): 0 (default) = one workgroup per block of Algorithm 2; -1 =
 *     a persistent grid of as many workgroups as the device holds at once
 *     (CUs x occupancy of that kernel), each striding over the blocks, as
 *     Algorithm 2 with p = the resident workgroups deals blocks to them;
 *     g > 0 = at most g workgroups.  Never more workgroups than blocks.
 *     CM_EINVAL below -1.
 *   cm_get_config / cm_get_search / cm_get_partition / cm_get_block_order /
 *     cm_get_coarse_stride / cm_get_fine_lanes / cm_get_grid return the
 *     current setting
 *     (cm_get_config: the value set for the pair, or -1 while none is set
 *     and the per-operation defaults above apply; cm_tuning_get reports the
 *     choice a call would actually make).
 *   (Settings are process-wide and not thread-safe against concurrent
 *   merges; set them before launching.)
 */
int cm_config_count(void);
int cm_config_info(int config_id, int *threads, int *items_per_thread);
int cm_set_config(int key_type, int with_payload, int config_id);
int cm_get_config(int key_type, int with_payload);
int cm_set_search(int search_mode);
int cm_get_search(void);
int cm_set_partition(int partition_mode);
int cm_get_partition(void);
int cm_set_coarse_stride(uint32_t blocks);
int cm_set_block_order(int order);
int cm_get_block_order(void);
int cm_get_coarse_stride(void);
int cm_get_fine_lanes(void);
int cm_set_fine_lanes(int lanes);
int cm_set_grid(int workgroups);
int cm_get_grid(void);

/*
 * Autotuner (self-written; not part of the method).  Times every tile
 * configuration x co-rank search x boundary pass on the caller's buffers
 * (each candidate: one warm call, then `reps` calls between two HIP events
 * on `stream`; the call synchronises), times the four fastest three times
 * more, round-robin, keeps each one's best time, stores the fastest in the
 * tuning table under (operation, key type, payload, size class of m + n) and, if
 * best is not NULL, writes best[0..2] = {config, search, partition}.  Every
 * candidate produces the same output, so C (and C_val) hold the merge
 * afterwards.  Arguments are those of cm_stable_merge_pairs (payload
 * pointers all NULL for keys only) / cm_stable_merge_segmented.  The
 * segmented tuner tries the one-level and two-level boundary passes.
 * Errors: those of the merge calls; CM_EINVAL for reps outside [1, 10000]
 * or an empty merge.
 */
int cm_autotune_merge(int key_type,
                      const void *A, const uint32_t *A_val, uint64_t m,
                      const void *B, const uint32_t *B_val, uint64_t n,
                      void *C, uint32_t *C_val,
                      void *workspace, size_t workspace_bytes,
                      int reps, hipStream_t stream, int *best);
int cm_autotune_segmented(int key_type,
                          const void *A, const uint32_t *A_val, const uint64_t *a_off,
                          uint64_t total_a,
                          const void *B, const uint32_t *B_val, const uint64_t *b_off,
                          uint64_t total_b, uint64_t num_seg,
                          void *C, uint32_t *C_val,
                          void *workspace, size_t workspace_bytes,
                          int reps, hipStream_t stream, int *best);

/*
 * Tuning table.  Entries map (op, key_type, with_payload, size class) to
 * {config, search, partition}; op 0 = single merge, 1 = segmented batch,
 * 2 = batch of separate merges (size class of its total output count),
 * 3 = stable sort (size class of n; partition 0 = one-level boundary pass,
 * any other value = two-level for pairs longer than the coarse stride).  A
 * segmented batch takes partition 0 as the one-level pass and any other
 * value as the two-level pass; a batch of separate merges takes the modes
 * of cm_stable_merge_batch;
 * the size class of a merge of N outputs is the bit length of N (0..64).
 * A merge call uses the entry of its size class when there is one, else
 * the settings of cm_set_config / cm_set_search / cm_set_partition.
 *   cm_tuning_set: add or replace one entry.
 *   cm_tuning_get: choice[0..2] that a call of N outputs would use now
 *     (CM_EINVAL for an unknown op).
 *   cm_tuning_save / cm_tuning_load: text file, one entry per line
 *     "op key_type with_payload size_class config search partition ms",
 *     after a header naming what the timings hold for: the device
 *     architecture (gcnArchName of the current device), the HIP runtime
 *     version and the library's build id (cm_build_id).  load merges the
 *     file into the table; CM_EINVAL on a malformed line, CM_ESTALE if the
 *     header is missing or names another device, runtime or build (either
 *     way the table is unchanged).  path NULL: the file named by the
 *     environment variable CM_TUNING_FILE, else
 *     $XDG_CACHE_HOME/corank_merge/tuning.txt, else
 *     $HOME/.cache/corank_merge/tuning.txt (save creates its directories).
 *   cm_build_id: the library's build id, a hash of its sources.
 *   cm_tuning_clear / cm_tuning_count: empty / size of the table.
 */
int cm_tuning_set(int op, int key_type, int with_payload, int size_class,
                  int config_id, int search_mode, int partition_mode);
int cm_tuning_get(int op, int key_type, int with_payload, uint64_t num_outputs, int *choice);
int cm_tuning_save(const char *path);
int cm_tuning_load(const char *path);
const char *cm_build_id(void);
int cm_tuning_clear(void);
int cm_tuning_count(void);

/*
 * Graph plans: the whole kernel sequence of one merge call, captured once
 * into a HIP graph (on a private stream; the capture records no memory
 * sets) and replayed with one launch.  The plan keeps the caller's
 * pointers and sizes: the buffers must outlive the plan, and a replay reads
 * their contents at replay time.  The tuning choice is fixed at creation.
 * Arguments are those of cm_stable_merge_pairs / cm_stable_merge_segmented
 * (payload pointers all NULL for keys only).
 *   cm_plan_create_*: CM_OK and *plan set, or an error of the merge call,
 *     or CM_EHIP if capture or instantiation failed (*plan = NULL).
 *   cm_plan_launch: one graph launch on `stream`.
 *   cm_plan_update_merge / cm_plan_update_segmented: re-point a plan made by
 *     the matching create call at other buffers and sizes (same arguments
 *     as create, tuning choice made anew): the call is captured again and
 *     applied to the plan's executable graph in place when only kernel
 *     arguments and grid sizes change, else a new executable graph replaces
 *     it.  Not while a launch of the plan may still run.  CM_EINVAL for a
 *     plan of the other kind, an error of the merge call (the plan is then
 *     unchanged), or CM_EHIP.
 *   cm_plan_destroy: frees the plan (not while a launch may still run).
 */
typedef struct cm_plan cm_plan;
int cm_plan_create_merge(int key_type,
                         const void *A, const uint32_t *A_val, uint64_t m,
                         const void *B, const uint32_t *B_val, uint64_t n,
                         void *C, uint32_t *C_val,
                         void *workspace, size_t workspace_bytes, cm_plan **plan);
int cm_plan_create_segmented(int key_type,
                             const void *A, const uint32_t *A_val, const uint64_t *a_off,
                             uint64_t total_a,
                             const void *B, const uint32_t *B_val, const uint64_t *b_off,
                             uint64_t total_b, uint64_t num_seg,
                             void *C, uint32_t *C_val,
                             void *workspace, size_t workspace_bytes, cm_plan **plan);
int cm_plan_launch(cm_plan *plan, hipStream_t stream);
int cm_plan_update_merge(cm_plan *plan, int key_type,
                         const void *A, const uint32_t *A_val, uint64_t m,
                         const void *B, const uint32_t *B_val, uint64_t n,
                         void *C, uint32_t *C_val,
                         void *workspace, size_t workspace_bytes);
int cm_plan_update_segmented(cm_plan *plan, int key_type,
                             const void *A, const uint32_t *A_val, const uint64_t *a_off,
                             uint64_t total_a,
                             const void *B, const uint32_t *B_val, const uint64_t *b_off,
                             uint64_t total_b, uint64_t num_seg,
                             void *C, uint32_t *C_val,
                             void *workspace, size_t workspace_bytes);
int cm_plan_destroy(cm_plan *plan);

/*
 * Per-merge-launch form of cm_stable_merge_segmented: the same batch run as
 * one single-merge call per segment (two kernel launches each), the
 * baseline the one-pass batch is measured against.  a_off_host / b_off_host
 * are host copies of the offsets (num_seg + 1 entries); the key and payload
 * arrays are device arrays as in cm_stable_merge_segmented; workspace must
 * hold cm_merge_workspace_size(key_type, with_payload, m_s, n_s) bytes for
 * the largest segment.  Output is identical to cm_stable_merge_segmented.
 * Errors: as cm_stable_merge_pairs, plus CM_EINVAL for inconsistent host
 * offsets (checked before anything is launched).
 */
int cm_stable_merge_segmented_each(int key_type,
                                   const void *A, const uint32_t *A_val, const uint64_t *a_off_host,
                                   uint64_t total_a,
                                   const void *B, const uint32_t *B_val, const uint64_t *b_off_host,
                                   uint64_t total_b,
                                   uint64_t num_seg,
                                   void *C, uint32_t *C_val,
                                   void *workspace, size_t workspace_bytes,
                                   hipStream_t stream);

/*
 * Measurement helpers (not part of the method).
 *
 * cm_copy: copies `bytes` bytes from device src to device dst on `stream`
 *   with 16-byte vector loads and stores (a plain streaming copy; used to
 *   calibrate hardware byte counters and to measure the copy ceiling).
 *   src and dst must not overlap (CM_EALIAS); both must be 16-byte aligned
 *   and bytes a multiple of 16 (CM_EINVAL).
 * cm_timing_start(capacity): from now on, each of the next `capacity` merge
 *   calls (single or segmented; not the per-merge-launch form) records HIP
 *   events on its stream before its first kernel, between its co-rank pass
 *   and its block-merge kernel, and after the block-merge kernel.  Creates
 *   the events (no device memory is allocated).  CM_EINVAL if capacity is 0
 *   or above 2^20, or timing is already on.
 * cm_timing_stop: waits for the recorded events, writes the number of timed
 *   calls and the mean duration in milliseconds of the co-rank pass and of
 *   the block-merge kernel over them, and releases the events.  If
 *   call_start_ms / call_ms / merge_ms are given (host arrays of at least
 *   `capacity` floats), entry c receives call c's start relative to call
 *   0's start / its whole duration (first event to last) / its block-merge
 *   kernel's duration, in milliseconds (calls on different streams may
 *   overlap).  Every output may be NULL.  CM_EINVAL if timing is off.
 */
int cm_copy(const void *src, void *dst, uint64_t bytes, hipStream_t stream);

/*
 * cm_copy_tiles(config, A, A_val, m, B, B_val, n, C, C_val, stream): the
 *   data movement of a block merge of uint32 keys with uint32 payloads under
 *   tile configuration `config` (T = threads x items outputs per workgroup,
 *   as cm_config_info reports), without the merge (a measurement aid: the
 *   speed of the merge's own traffic pattern).  Workgroup t stages two
 *   windows of the inputs in LDS with 16-byte loads, waits at a barrier and
 *   stores T outputs with 16-byte stores: counting in 16-byte units (4
 *   elements), tile t covers units [q0, q1) = [t T/4, min((t+1) T/4, N/4))
 *   of C and copies A units [j(q0), j(q1)) followed by B units [q0 - j(q0),
 *   q1 - j(q1)), where j(q) = floor(q (m/4) / (N/4)) is A's share; the same
 *   for the payloads into C_val.  Every tile thus reads exactly what it
 *   writes, split between A and B in proportion m : n (Proposition 2's equal
 *   blocks with linear windows instead of co-ranks).  Device arrays; every
 *   base 16-byte aligned, m and n multiples of 4, m + n < 2^34, config in
 *   [0, cm_config_count()) (else CM_EINVAL); C and C_val must not overlap an
 *   input (CM_EALIAS).  m + n = 0 is a no-op.
 */
int cm_copy_tiles(int config, const void *A, const uint32_t *A_val, uint64_t m, const void *B,
                  const uint32_t *B_val, uint64_t n, void *C, uint32_t *C_val, hipStream_t stream);
int cm_timing_start(uint32_t capacity);
int cm_timing_stop(uint32_t *calls, double *co_rank_ms_mean, double *merge_ms_mean,
                   float *call_start_ms, float *call_ms, float *merge_ms);

/*
 * Payloads of any width.  The merge moves one uint32 per key; wider payloads
 * (uint64, structs) travel as origin codes instead: merge the keys with
 * A_codes / B_codes as payloads, then move W-byte records by the merged
 * codes.  Element x of A has code x, element y of B code 2^31 + y (m, n <
 * 2^31), so the codes in C_val name each output's source.
 * cm_origin_codes(m, n, A_codes, B_codes, stream): fills A_codes[x] = x and
 *   B_codes[y] = 2^31 + y (device arrays of m and n uint32).
 * cm_gather_records(codes, N, A_rec, m, B_rec, n, width, out, stream):
 *   out[i] = the width-byte record A_rec[codes[i]] or B_rec[codes[i] - 2^31]
 *   for i < N (device arrays; records contiguous).  Moves 16-, 8- or 4-byte
 *   words when width and every base allow.  A code past its array leaves
 *   out[i] untouched.  CM_EINVAL (width 0, null pointer with a nonzero
 *   size, m or n >= 2^31, N or m + n records of `width` bytes past 2^64
 *   bytes), CM_EALIAS (out overlaps an input), CM_EHIP.
 */
int cm_origin_codes(uint64_t m, uint64_t n, uint32_t *A_codes, uint32_t *B_codes,
                    hipStream_t stream);
int cm_gather_records(const uint32_t *codes, uint64_t N, const void *A_rec, uint64_t m,
                      const void *B_rec, uint64_t n, uint64_t width, void *out,
                      hipStream_t stream);

/*
 * Partition ablation (the prior art the paper improves on, Section 1).  The
 * merge with P processing elements, each a workgroup merging one contiguous
 * output segment through LDS ring buffers (the streaming kernel of
 * boundary mode 3), with the segments cut in one of two ways:
 *   partition 0: P segments of equal length, cut by co-ranking their ends
 *     (Lemma 1 / Algorithm 2 of the paper);
 *   partition 1: the classic cross-rank partition: P / 2 equidistant
 *     samples of A and P / 2 of B, each ranked in the other array by
 *     binary search; the P sample cuts in output order bound the segments,
 *     which hold at most ceil(2m / P) elements of A and ceil(2n / P) of B
 *     and may differ in length by a factor of two.
 * Both produce the merge of cm_stable_merge_pairs (payload pointers all NULL
 * for keys only); only the balance of the segments differs.
 * cm_partition_ablation_workspace_size(P): workspace bytes.
 * cm_merge_partition_ablation(key_type, A, A_val, m, B, B_val, n, C, C_val,
 *   P, partition, bounds, workspace, bytes, stream): P even in [2, 2^20];
 *   bounds: device array of P + 1 uint64 that receives the segment starts
 *   (bounds[P] = m + n).  Timing events (cm_timing_start) separate the
 *   partition kernels from the merge kernel.  Errors as for
 *   cm_stable_merge_pairs; CM_EINVAL for a bad P or partition.
 */
size_t cm_partition_ablation_workspace_size(uint32_t P);
int cm_merge_partition_ablation(int key_type, const void *A, const uint32_t *A_val, uint64_t m,
                                const void *B, const uint32_t *B_val, uint64_t n, void *C,
                                uint32_t *C_val, uint32_t P, int partition, uint64_t *bounds,
                                void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Stable merge sort built from the co-rank merge (Section 1: merging is the
 * step of merge sort; Sections 2-3 give the perfectly balanced parallel
 * merge each pass uses).  Sorts n keys (and their uint32 payloads) into
 * keys_out (vals_out) in nondecreasing key order; equal keys keep their
 * input order (stable).  Float keys compare as IEEE values (-0.0 == +0.0,
 * NaN not allowed).
 *   Runs of 4, 2 or 1 blocks (as many as fit two workgroups' LDS per CU:
 *   4 for 4-byte keys with payloads in the default 256 x 9 tile, runs of
 *   9,216) are first sorted inside LDS (per-thread sorting networks, then
 *   co-rank merges in LDS); then ceil(log2(n / run)) passes merge runs
 *   pairwise, each pass a boundary pass and one block merge over all pairs
 *   (Algorithm 2 per pair).  The boundary pass co-ranks every block start in
 *   its pair: one thread each (partition 0), or, for pairs longer than the
 *   coarse stride, every coarse_stride-th start first by 16-lane groups and
 *   the others inside those brackets (cm_set_fine_lanes lanes each).  Passes
 *   alternate between the output and the workspace.
 * cm_sort_workspace_size(key_type, with_payload, n): bytes (a second key and
 *   payload buffer of n entries, one uint64 per block and one per 16
 *   blocks), 0 for n == 0.
 * cm_sort_run_length(key_type, with_payload, n): elements per run of the
 *   LDS run sort in the configuration a sort of n keys would use now (the
 *   passes then number ceil(log2(n / run))); 0 for an unknown key type.
 *   Host-only; no GPU work.
 * cm_stable_sort(key_type, keys, n, keys_out, workspace, bytes, stream)
 * cm_stable_sort_pairs(key_type, keys, vals, n, keys_out, vals_out,
 *   workspace, bytes, stream)
 *   Device pointers; enqueued on `stream`.  keys_out may be keys itself and
 *   vals_out vals itself (in place); any other overlap of outputs with
 *   inputs, with each other or with the workspace is CM_EALIAS.  n == 0 is a
 *   no-op.  Errors: CM_EDTYPE, CM_EINVAL (null pointer with n > 0),
 *   CM_ENOSPC, CM_EALIAS, CM_EHIP.  The tile configuration and search come
 *   from the tuning table (operation 3) or the process defaults.
 */
size_t cm_sort_workspace_size(int key_type, int with_payload, uint64_t n);
uint64_t cm_sort_run_length(int key_type, int with_payload, uint64_t n);
int cm_stable_sort(int key_type, const void *keys, uint64_t n, void *keys_out, void *workspace,
                   size_t workspace_bytes, hipStream_t stream);
int cm_stable_sort_pairs(int key_type, const void *keys, const uint32_t *vals, uint64_t n,
                         void *keys_out, uint32_t *vals_out, void *workspace,
                         size_t workspace_bytes, hipStream_t stream);

/*
 * Serving runtime (not part of the method; it feeds the batch call above).
 * A server owns a scheduler thread.  Clients submit single merges (device
 * inputs, sizes; or host data, see cm_server_submit_host); the scheduler
 * admits them in arrival order while their outputs fit in an output arena in
 * HBM (the caller's device buffer), packs the admitted ones whose inputs are
 * in place (the producer's work, or the runtime's copy in, has completed)
 * into one cm_stable_merge_batch launch per step (at most max_batch merges;
 * at most max_inflight batches in flight, each on its own stream), and
 * reports each finished merge once.  A finished merge's outputs
 * stay in the arena until the client releases its ticket.  Results are
 * those of cm_stable_merge_pairs / cm_stable_merge on the same inputs.
 *
 * cm_server_create(key_type, with_payload, arena, arena_bytes, max_batch,
 *   max_inflight, max_requests, &server): arena is a device buffer of
 *   arena_bytes (>= 256; the caller keeps it alive until destroy; it must not
 *   overlap any request's inputs); max_batch in [1, 65536], max_inflight in
 *   [1, 16], max_requests in [1, 65535] (submitted and not yet released).
 *   Creates streams (default priority; one per batch in flight and two for
 *   host requests' copies), events, pinned host descriptor buffers and
 *   per-batch device workspaces on the current device once; nothing is
 *   allocated afterwards.  CM_EINVAL / CM_EDTYPE / CM_EHIP.
 * cm_server_submit(server, A, A_val, m, B, B_val, n, inputs_stream,
 *   inputs_pending, &ticket): payload pointers all NULL iff the server has
 *   no payloads.  With inputs_pending set, the merge waits for the work
 *   enqueued on inputs_stream so far (the inputs' producer); otherwise the
 *   inputs must already be in place.  Inputs must stay unchanged until the
 *   merge is reported.  Thread-safe.  CM_EINVAL (bad pointers or sizes),
 *   CM_ENOSPC (the outputs can never fit in the arena), CM_EBUSY (all
 *   max_requests slots are taken: poll and release, then retry),
 *   CM_ECANCELED (the server is shutting down).
 * cm_server_submit_host(server, A, A_val, m, B, B_val, n, C, C_val,
 *   &ticket): the same merge for data in host memory (pinned memory, from
 *   hipHostMalloc, lets the copies overlap; pageable memory works but each
 *   copy then blocks the scheduler thread while it is staged).  The request
 *   is admitted when its outputs and its inputs both fit in the arena (the
 *   inputs are staged there: keys of A and B, then their payloads); at
 *   admission the runtime copies the inputs in on a copy stream of its own,
 *   the batch waits for that copy, and after the batch the outputs are
 *   copied to C (N keys) and C_val (N payloads) on a second copy stream.
 *   The request is reported once its outputs are in C / C_val; until then
 *   the caller keeps every host array alive, the inputs unchanged and the
 *   outputs untouched.  Payload pointers all NULL iff the server has no
 *   payloads.  CM_EINVAL (bad pointers or sizes), CM_EALIAS (C or C_val
 *   overlaps an input or each other), CM_ENOSPC (inputs plus outputs can
 *   never fit in the arena), CM_EBUSY, CM_ECANCELED as for submit.
 * cm_server_poll(server, done, capacity, &count, wait_us): moves up to
 *   `capacity` finished merges into done[] and sets count; waits up to
 *   wait_us microseconds for the first one if none is ready (0: do not
 *   wait).  Each entry: ticket; status (CM_OK, or the batch call's error, or
 *   CM_ECANCELED); C / C_val: the outputs (inside the arena; NULL for an
 *   empty merge; for a host request the caller's host arrays, the arena
 *   copy staying at the offsets until release); keys_offset / vals_offset:
 *   their byte offsets in the arena; queued_ns: submit to launch;
 *   latency_ns: submit to completion as seen by the scheduler (for a host
 *   request: outputs back in host memory); ended_ns: submit to the moment
 *   the scheduler saw the request's batch end on the device (before any
 *   copy back); device_ns: that batch's device time (from HIP events
 *   around its upload and kernels; 0 if they could not be read).
 *   Thread-safe.
 * cm_server_release(server, ticket): the client is done with a reported
 *   merge's outputs; its arena space and slot are reused.  CM_EINVAL for an
 *   unknown, unreported or already released ticket.
 * cm_server_get_stats(server, &stats): counters since creation; busy_ms is the
 *   total time at least one batch was running on the GPU (from HIP events
 *   recorded around each batch's upload and kernels, union over streams) and
 *   span_ms the time from the first batch's start to the last one's end.
 * cm_server_destroy(server): finishes every admitted and launched merge,
 *   cancels submitted merges that can no longer be admitted (arena held by
 *   unreleased outputs), joins the thread and frees the server's resources
 *   (not the arena).
 */
typedef struct cm_server cm_server;
typedef struct cm_server_done {
    uint64_t ticket;
    int32_t status;
    int32_t reserved;
    void *C;
    uint32_t *C_val;
    uint64_t keys_offset;
    uint64_t vals_offset;
    uint64_t queued_ns;
    uint64_t latency_ns;
    uint64_t ended_ns;
    uint64_t device_ns;
} cm_server_done;
typedef struct cm_server_stats {
    uint64_t submitted, completed, failed, canceled, batches, max_batch_seen;
    uint64_t arena_bytes, arena_peak_bytes;
    double busy_ms, span_ms;
} cm_server_stats;

int cm_server_create(int key_type, int with_payload, void *arena, uint64_t arena_bytes,
                     uint32_t max_batch, uint32_t max_inflight, uint32_t max_requests,
                     cm_server **server);
int cm_server_submit(cm_server *server, const void *A, const uint32_t *A_val, uint64_t m,
                     const void *B, const uint32_t *B_val, uint64_t n, hipStream_t inputs_stream,
                     int inputs_pending, uint64_t *ticket);
int cm_server_submit_host(cm_server *server, const void *A, const uint32_t *A_val, uint64_t m,
                          const void *B, const uint32_t *B_val, uint64_t n, void *C,
                          uint32_t *C_val, uint64_t *ticket);
int cm_server_poll(cm_server *server, cm_server_done *done, uint32_t capacity, uint32_t *count,
                   int64_t wait_us);
int cm_server_release(cm_server *server, uint64_t ticket);
int cm_server_get_stats(cm_server *server, cm_server_stats *stats);
int cm_server_destroy(cm_server *server);

#ifdef __cplusplus
}
#endif

#endif /* CORANK_MERGE_H */
