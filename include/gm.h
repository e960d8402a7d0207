/*
 * gm.h -- C ABI of the MI355X Gumbel-Max sketch library (libgm.so).
 *
 * The library computes k-register Gumbel-Max sketches of sparse non-negative
 * vectors ("Fast Gumbel-Max Sketch and its Applications", Zhang, Qi, Wang et
 * al., arXiv:2302.05176) and the two estimators built on them.
 *
 *   s_j(v) = argmin_{i in N+(v)} E_ij / v_i,   y_j(v) = min_{i in N+(v)} E_ij / v_i,
 *
 * j = 0..k-1, with E_ij ~ Exp(1) consistent across vectors (Sec. 1, Eq. (1)
 * and Eq. (2); N+(v) is the set of indices with v_i > 0).  s is the
 * Gumbel-ArgMax sketch (probability-Jaccard estimation), y the Lemiesz sketch
 * (weighted cardinality estimation); x_j = -ln y_j is the Gumbel-Max variable.
 *
 * Two forms with identical distributions but different concrete draws:
 *   FastGM form  -- element i's k variables are generated as ascending order
 *                   statistics (Eq. (7)-(8)) routed to registers by a
 *                   Fisher-Yates permutation (Sec. 2.2); an element stops at
 *                   its first arrival later than the largest register
 *                   (FastPrune), giving O(k ln k + n+) work (Sec. 2.5).
 *   plain form   -- E_ij drawn independently per (i, j); O(k n+) work
 *                   (Sec. 1, the straightforward method).
 * The draws are fixed by the library's draw specification (splitmix64 hash
 * of (seed, i, step), uniform (x>>11 + 1/2) 2^-53, a fixed-order -ln), so a
 * sketch is a pure function of (multiset of (index, weight) entries, k, seed,
 * form): it does not depend on entry order, batch composition, stream or
 * launch configuration.  Sketches are comparable only when built with the
 * same (k, seed, form).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers on the current HIP device,
 *     owned by the caller, and must stay valid until `stream` reaches the
 *     call.  Every call is asynchronous on `stream` (0 = null stream), except
 *     gm_get_data_errors, which synchronises `stream`.
 *   - Input vectors are CSR rows: vector v holds entries
 *     [offsets[v], offsets[v+1]) of `indices` (int32, must be >= 0) and
 *     `weights` (fp32).  offsets has nvec+1 int64 entries and offsets[0] is
 *     the base (need not be 0).  Duplicate indices are allowed (a stream
 *     element seen twice changes nothing when its weight repeats).
 *   - Outputs are row-major: register j of vector v is out_idx[v*k + j]
 *     (int32 index s_j) and out_val[v*k + j] (fp64 key y_j).
 *   - Weight 0 means "not in N+" and the entry is skipped.  A vector with no
 *     positive weight gets empty registers (index -1, value +inf).
 *   - Argument errors (null pointer with nvec > 0, nvec < 0, k outside
 *     [1, GM_K_MAX]) are detected on the host; the call returns
 *     GM_ERR_INVALID_ARG and enqueues nothing.
 *   - Data errors (a negative, NaN or infinite weight, a negative index, or
 *     offsets[v+1] < offsets[v]) are detected on the device: the vector's
 *     registers become (index -2, value NaN) and a sticky per-device counter
 *     is incremented once per bad vector (read it with gm_get_data_errors).
 *   - The library keeps a workspace per device and per stream (for the
 *     FastGM form a planner list of nvec int32 and the walk's lists, for the
 *     plain form a split scratch), created or grown by the first call that
 *     needs it -- make that call outside any stream capture -- and released
 *     by gm_release().  The per-device error counter is static device memory
 *     and survives gm_release().
 */
#ifndef GM_H
#define GM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GM_OK = 0,
    GM_ERR_INVALID_ARG = 1,
    GM_ERR_OUT_OF_MEMORY = 2,
    GM_ERR_DEVICE = 3,
    GM_ERR_UNSUPPORTED = 4
} gm_status;

typedef enum { GM_FORM_FASTGM = 0, GM_FORM_PLAIN = 1 } gm_form;

/* Largest register count supported by the kernels. */
#define GM_K_MAX 4096

/*
 * gm_sketch -- FastGM form (Algorithm 1 / Algorithm 2 semantics: ascending
 * arrivals per element, Fisher-Yates routing, FastPrune against the running
 * maximum register), for nvec CSR vectors with the same k.
 *   indices  [nnz] int32   element indices (>= 0)
 *   weights  [nnz] fp32    element weights (>= 0, finite)
 *   offsets  [nvec+1] int64
 *   nvec     number of vectors (0 is allowed: nothing is launched)
 *   k        registers per sketch, 1..GM_K_MAX
 *   seed     sketch seed (the hash key of every draw)
 *   out_idx  [nvec*k] int32  s_j
 *   out_val  [nvec*k] fp64   y_j
 */
gm_status gm_sketch(const int32_t *indices, const float *weights, const int64_t *offsets,
                    int64_t nvec, int32_t k, uint64_t seed,
                    int32_t *out_idx, double *out_val, hipStream_t stream);

/*
 * gm_sketch_update -- streaming update (Sec. 3, Algorithm 2; mergeability,
 * Sec. 2.3): sk_idx/sk_val (device, row-major [nvec][k], caller-owned) hold
 * the FastGM-form sketches, under the same k and seed, of the entries seen
 * so far (an all-empty row, (-1, +inf), stands for none); vector v's new
 * entries [offsets[v], offsets[v+1]) are merged in place, so that the row
 * becomes the sketch of the union of old and new entries -- bit for bit the
 * result of gm_sketch over that union.  Each vector's walk stops at its
 * stored sketch's largest register (an arrival above it cannot change the
 * result), so updates get cheaper as a stream goes on.  Repeated entries
 * (same index and weight) change nothing.  Data errors poison the row
 * (-2, NaN); a poisoned row stays poisoned; a vector with no positive entry
 * leaves its row unchanged.  Argument errors as for gm_sketch.
 */
gm_status gm_sketch_update(const int32_t *indices, const float *weights, const int64_t *offsets,
                           int64_t nvec, int32_t k, uint64_t seed, int32_t *sk_idx, double *sk_val,
                           hipStream_t stream);

/*
 * gm_sketch_plain -- plain form of Eq. (1)/(2): every (entry, register) key
 * is drawn and the minimum kept; O(k n+) per vector.  Same arguments and
 * layout as gm_sketch.  Register j of a k-register plain sketch equals
 * register j of any larger plain sketch with the same seed.  A call with
 * few vectors splits each vector's entries over several workgroups and
 * merges their minima (Sec. 2.3) in a per-stream scratch area of the
 * library (about 12 * 1536 * CUs * 256 bytes, created by the first such
 * call or by gm_reserve).
 */
gm_status gm_sketch_plain(const int32_t *indices, const float *weights, const int64_t *offsets,
                          int64_t nvec, int32_t k, uint64_t seed,
                          int32_t *out_idx, double *out_val, hipStream_t stream);

/*
 * gm_sketch_plain_noalloc -- gm_sketch_plain for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, layout, results and
 * error rules as gm_sketch_plain; it calls no hipMalloc, hipFree or other
 * allocating routine, not even on its first call on a device.
 *   Scratch: the partial registers of a split launch live in one static
 *   device array per device of 6 MiB + 64 KiB (2^19 partial registers,
 *   2 x 4096 int32 counters and a 32 KiB split plan for batches of many
 *   vectors), held until the process ends.  A call splits
 *   its vectors only as far as that array holds (one vector at any k fits
 *   the full split); a call that would need more runs with fewer entry
 *   ranges, so no input is rejected for its size.  The counters are cleared
 *   by a fill kernel on `stream` at the start of each split call.
 *   Concurrency: every call on a device shares that device's array, so
 *   calls on one device that overlap in time (different streams, or host
 *   threads) race and may return wrong registers; serialise them.
 */
gm_status gm_sketch_plain_noalloc(const int32_t *indices, const float *weights,
                                  const int64_t *offsets, int64_t nvec, int32_t k, uint64_t seed,
                                  int32_t *out_idx, double *out_val, hipStream_t stream);

/*
 * gm_sketch_batched -- vectors with individual register counts, in one call.
 *   k_per_vec    [nvec] int32 (device)  k of vector v, 1..k_max
 *   out_offsets  [nvec+1] int64 (device) registers of vector v are written to
 *                out_*[out_offsets[v] .. out_offsets[v] + k_per_vec[v])
 *   k_max        host-side upper bound of k_per_vec (1..GM_K_MAX)
 *   form         GM_FORM_FASTGM or GM_FORM_PLAIN
 * A vector whose k_per_vec is outside [1, k_max] is a data error (its first
 * out_offsets[v+1]-out_offsets[v] registers are poisoned).
 */
gm_status gm_sketch_batched(const int32_t *indices, const float *weights, const int64_t *offsets,
                            int64_t nvec, const int32_t *k_per_vec, const int64_t *out_offsets,
                            int32_t k_max, uint64_t seed, gm_form form,
                            int32_t *out_idx, double *out_val, hipStream_t stream);

/*
 * gm_reserve -- create, on the current device, the workspace that FastGM
 * calls on `stream` with up to nvec vectors need (planner lists, big-vector
 * candidate pool), and the plain form's split scratch, so that later calls
 * allocate nothing.  Call it before capturing sketch calls into a HIP graph
 * on `stream`.  Synchronous.
 */
gm_status gm_reserve(int64_t nvec, hipStream_t stream);

/*
 * gm_workspace_bytes -- device bytes of the workspace that gm_reserve(nvec,
 * stream) creates for one stream on the current device: the FastGM planner
 * list and per-vector records (about 200 bytes per vector), the big-vector
 * candidate pool (256 MiB), the walk's per-wave lists (64 KiB per resident
 * wave), the split-walk scratch and the plain form's split scratch.  For
 * admission control: each stream that sketches concurrently holds one.
 * Allocates nothing; nvec in [0, 2^31).
 */
gm_status gm_workspace_bytes(int64_t nvec, int64_t *bytes);

/*
 * gm_jaccard_est -- probability-Jaccard estimate of Sec. 1:
 *   out[p] = #{ j : a[p*k+j] == b[p*k+j] and a[p*k+j] >= 0 } / k
 * for npairs row-major pairs of Gumbel-ArgMax sketches (Theorem 1: unbiased
 * for J_P with variance J_P (1 - J_P) / k).  Empty (-1) and poisoned (-2)
 * registers never match.
 */
gm_status gm_jaccard_est(const int32_t *idx_a, const int32_t *idx_b, int64_t npairs, int32_t k,
                         double *out, hipStream_t stream);

/*
 * gm_jaccard_est_pairs -- same estimate for pairs of rows of a device-resident
 * sketch store: out[p] = J_hat(store[ia[p]], store[ib[p]]), rows of k int32.
 *   store_idx [nstore*k] int32, ia/ib [npairs] int64 row numbers (device).
 * Row numbers outside [0, nstore) give out[p] = NaN and count as data errors.
 */
gm_status gm_jaccard_est_pairs(const int32_t *store_idx, int64_t nstore, int32_t k,
                               const int64_t *ia, const int64_t *ib, int64_t npairs,
                               double *out, hipStream_t stream);

/*
 * gm_wcard_est -- weighted-cardinality estimate of Sec. 1 (Lemiesz):
 *   out[v] = (k - 1) / (y_0 + y_1 + ... + y_{k-1})
 * with the sum taken left to right in fp64 (Theorem 2: unbiased).  k >= 2.
 * An empty sketch (+inf registers) gives 0; a poisoned one gives NaN.
 */
gm_status gm_wcard_est(const double *val, int64_t nvec, int32_t k, double *out,
                       hipStream_t stream);

/*
 * gm_setops -- weighted cardinalities of two sets from their sketches.  For
 * sets whose objects carry fixed positive weights (the weighted-cardinality
 * setting of Sec. 1), row p of (idx_a, val_a) and of (idx_b, val_b) are the
 * sketches of A_p and B_p (same k, seed and form; row-major [npairs][k]),
 * and out[p*5 + c] (fp64, device) receives
 *   c = 0  |A u B|_w = (k-1) / sum_j m_j, m_j the lexicographically smaller
 *          of the two registers (the union's sketch, Sec. 2.3; Theorem 2),
 *          summed left to right;
 *   c = 1  |A n B|_w = union * (#{j : registers equal and filled} / k);
 *   c = 2  |A \ B|_w = union * (#{j : A's register smaller} / k);
 *   c = 3  |B \ A|_w = union * (#{j : B's register smaller} / k);
 *   c = 4  J_W(A, B) = #{j : registers equal and filled} / k.
 * The union's register is won by one object with probability proportional
 * to its weight (Sec. 1), in both sets exactly when the registers are equal;
 * the paper applies these estimates (Lemiesz's algebra) in Sec. 4.5 without
 * stating them, so this is the library's reading of them.  Each estimate is
 * unbiased.  Two empty sketches give zeros; a poisoned register (index -2)
 * makes all five NaN.  k >= 2; argument errors as elsewhere.
 */
gm_status gm_setops(const int32_t *idx_a, const double *val_a, const int32_t *idx_b,
                    const double *val_b, int64_t npairs, int32_t k, double *out,
                    hipStream_t stream);

/*
 * gm_rate_probe -- issue-rate probe for the roofline of the sketch kernels.
 * Every one of `lanes` lanes draws `steps` (1..GM_K_MAX) arrivals
 * (what = 0: Renyi prefix of Eq. (7)-(8) with the Fisher-Yates target, as
 * the FastGM walk draws them, k = steps) or plain keys (what = 1: Eq. (1),
 * registers 0..steps-1) of its own synthetic element, with no memory traffic
 * but one fp64 result per lane in out[lanes] (device, caller-owned).  Time it
 * with events on `stream`; the rate is the VALU ceiling of the per-arrival
 * arithmetic.  Invalid what/steps or a null out with lanes > 0 ->
 * GM_ERR_INVALID_ARG.
 */
gm_status gm_rate_probe(int32_t what, int64_t lanes, int32_t steps, uint64_t seed, double *out,
                        hipStream_t stream);

/*
 * gm_merge -- sketch of a union from sketches of its parts (Sec. 2.3):
 * register j of the result is the lexicographic (y, s) minimum over the r
 * input sketches' register j (r row-major sketches of k registers in
 * in_idx/in_val, result in out_idx/out_val).  r >= 1.
 */
gm_status gm_merge(const int32_t *in_idx, const double *in_val, int64_t r, int32_t k,
                   int32_t *out_idx, double *out_val, hipStream_t stream);

/*
 * LSH index over stored sketches (Sec. 1: each register maps similar vectors
 * to the same element with probability J_P, so the registers can key a
 * locality-sensitive index that finds similar vectors in sub-linear time).
 *
 * Band b (0 <= b < bands) of a sketch is its registers b*rows .. b*rows +
 * rows - 1.  A stored row is a candidate for a query when, in at least one
 * band, all `rows` register indices are equal and non-negative (an empty or
 * poisoned register never matches).  A pair at probability-Jaccard J is a
 * candidate with probability 1 - (1 - J^rows)^bands.
 *
 * gm_lsh_build -- indexes store_idx [nstore][k] int32 (device, caller-owned;
 *   it must stay allocated and unchanged while the index is used: queries
 *   verify candidates against it).  1 <= bands <= 64, rows >= 1, bands*rows
 *   <= k.  Allocates the index (12 bytes per row and band, plus the sort's
 *   temporaries during the call) with hipMalloc and synchronises `stream`:
 *   not for graph capture.  *out receives an index owned by the library;
 *   release it with gm_lsh_free.  GM_ERR_UNSUPPORTED when nstore*bands >
 *   2^31 - 1.
 * gm_lsh_query -- for nq queries query_idx [nq][k] int32 (device): count[q]
 *   (device int32) = the number of distinct candidate rows, and cand[q][0 ..
 *   min(count, max_cand) - 1] (device int32, [nq][max_cand]) = the smallest
 *   of them in ascending order.  A query with more than 2048 band matches
 *   (before duplicates across bands are removed) gets count = -1 and no
 *   candidates.  Asynchronous on `stream`.
 * gm_lsh_info -- the index's shape (any output pointer may be null).
 * gm_lsh_free -- releases an index (null is ignored).
 */
typedef struct gm_lsh_index gm_lsh_index;
gm_status gm_lsh_build(const int32_t *store_idx, int64_t nstore, int32_t k, int32_t bands,
                       int32_t rows, gm_lsh_index **out, hipStream_t stream);
gm_status gm_lsh_query(const gm_lsh_index *index, const int32_t *query_idx, int64_t nq,
                       int32_t max_cand, int32_t *cand, int32_t *count, hipStream_t stream);
gm_status gm_lsh_info(const gm_lsh_index *index, int64_t *nstore, int32_t *k, int32_t *bands,
                      int32_t *rows);
void gm_lsh_free(gm_lsh_index *index);

/*
 * gm_get_data_errors -- synchronises `stream`, then stores in *host_count the
 * number of poisoned vectors (and invalid store rows) seen on the current
 * device since the library was loaded or last reset.
 */
gm_status gm_get_data_errors(int64_t *host_count, hipStream_t stream);

/* gm_reset_data_errors -- zero the current device's data-error counter
 * (asynchronous on `stream`). */
gm_status gm_reset_data_errors(hipStream_t stream);

/*
 * gm_set_option -- process-wide tuning and testing knobs (defaults in
 * brackets).  They change how much work is done or which internal path runs,
 * never the result:
 *   GM_OPT_POS_BITS      [31] element-index bits in a packed FastGM register
 *                        (the index sits below the key's top bits), 31..62;
 *                        more bits means fewer key bits and more exact
 *                        re-resolutions of tied prefixes.
 *   GM_OPT_T0_SCALE_PPM  [1000000] scale of the closed-form pruning threshold
 *                        in parts per million; small values force the
 *                        enlarge-and-repeat fallback.
 *   GM_OPT_MAP_LOAD      [14] displaced permutation positions a lane may
 *                        track, 0..16; beyond it an element moves to the
 *                        segment path, where 16 or 64 lanes walk it
 *                        together (0 sends almost every element there).
 *   GM_OPT_REPUBLISH     [8] light iterations between republishes of the
 *                        running maximum register at k <= 256, a power of
 *                        two; scaled by k/256 above (a republish reads all
 *                        k registers).  The segment path republishes every
 *                        max(4, k/64) batches, rounded up to a power of two.
 *   GM_OPT_SEG_REST      [12] an element whose expected number of further
 *                        arrivals below the threshold (k v_i (T - t_1))
 *                        exceeds this goes to the segment path straight
 *                        from its first arrival, 0..1000000 (0: every
 *                        continuing element does).
 *   GM_OPT_SMALL_WAVES   [0] waves per workgroup of the kernels for vectors
 *                        of up to 32768 entries (0: chosen from k; else
 *                        1, 2, 4 or 8).
 *   GM_OPT_WAVE_LIM      [8191] registers-per-block tiling of the k <= 256
 *                        kernel: vectors of at most this many entries are
 *                        sketched one per wave, each wave with a register
 *                        set of its own; larger ones by the whole workgroup
 *                        sharing one set.  0 (one set per workgroup for
 *                        every vector) or 2^m - 1 for m = 4..15.
 *   GM_OPT_TIMING        [0] 1 brackets every launch of a sketch call with
 *                        HIP events on its stream (read with gm_get_timing);
 *                        2 only the sketch kernels themselves (FastGM class
 *                        kernels and the plain kernel), not the planning and
 *                        big-vector passes: fewer events in a timed loop.
 *   GM_OPT_STATS         [0] 1 makes FastGM calls accumulate work counters
 *                        (read them with gm_get_stats); costs a few atomics
 *                        per vector.
 * Options are process-wide and read once per call (atomics): a change made
 * by another host thread, gm_autotune's included, applies from some later
 * call on.  Returns GM_ERR_INVALID_ARG for an unknown option or out-of-range
 * value.
 */
typedef enum {
    GM_OPT_POS_BITS = 0,
    GM_OPT_T0_SCALE_PPM = 1,
    GM_OPT_MAP_LOAD = 2,
    GM_OPT_REPUBLISH = 3,
    GM_OPT_STATS = 4,
    GM_OPT_SEG_REST = 5,
    GM_OPT_SMALL_WAVES = 6,
    GM_OPT_TIMING = 7,
    GM_OPT_WAVE_LIM = 8
} gm_option;
gm_status gm_set_option(gm_option opt, int64_t value);

/*
 * gm_get_stats -- synchronises `stream`, then copies the first n (<= 16)
 * FastGM work counters of the current device, summed over calls made while
 * GM_OPT_STATS was 1: [0] vectors, [1] light-path wave iterations, [2]
 * probe and light arrivals drawn, [3] of which at or below the pruning
 * threshold, [4] elements continued on the light path, [5] elements handed
 * to the segment path, [6] its 16-lane (or 64-lane) batches, [7] extra
 * passes after an unfilled register, [8] exact index resolutions; wave
 * clock cycles (summed over waves) spent in [9] register init, validation
 * and sum, [10] the first walk, [11] the segment path (part of [10] and
 * [12]), [12] repeated walks, [13] completion checks and writeback.
 * gm_reset_stats -- synchronises `stream` and zeroes the counters.
 */
gm_status gm_get_stats(int64_t *host_counters, int32_t n, hipStream_t stream);
gm_status gm_reset_stats(hipStream_t stream);

/*
 * gm_get_timing -- waits for the timed launches made while GM_OPT_TIMING
 * was 1 or 2, then copies up to n entries: kernel name (as the profiler names the
 * instance), total milliseconds and launch count.  Returns the number of
 * entries copied.  gm_reset_timing clears the totals.
 */
int32_t gm_get_timing(int32_t n, char (*names)[64], double *total_ms, int64_t *launches);
void gm_reset_timing(void);

/*
 * gm_autotune -- pick the FastGM schedule options (GM_OPT_SMALL_WAVES,
 * GM_OPT_SEG_REST, GM_OPT_MAP_LOAD, GM_OPT_REPUBLISH and the
 * registers-per-block tiling GM_OPT_WAVE_LIM) for a batch like this
 * one by timing it: coordinate descent over each option's grid, median of
 * `reps` timed runs per point (HIP events on `stream`), then the best
 * setting is applied process-wide.  Arguments as gm_sketch (k_per_vec and
 * out_offsets null) or gm_sketch_batched (both non-null, k_max bounds k).
 * With use_cache != 0 a JSON-lines cache ($GM_TUNE_CACHE, default
 * ~/.cache/gm_tune.jsonl) keyed by (GPU arch, k_max, log2 nvec, log2 nnz,
 * uniform or per-vector k) is consulted first and updated after tuning.
 * The options change the work split, never the sketch.  Synchronises
 * `stream`; runs the batch many times (outputs are overwritten).
 */
typedef struct {
    int32_t small_waves, map_load, seg_rest, republish;
    double ms;          /* median time of the chosen setting */
    int32_t from_cache; /* 1 if taken from the cache without timing */
    int32_t wave_lim;   /* GM_OPT_WAVE_LIM chosen */
} gm_tune_result;
gm_status gm_autotune(const int32_t *indices, const float *weights, const int64_t *offsets,
                      int64_t nvec, const int32_t *k_per_vec, const int64_t *out_offsets,
                      int32_t k_max, uint64_t seed, int32_t *out_idx, double *out_val,
                      int32_t reps, int32_t use_cache, gm_tune_result *result,
                      hipStream_t stream);

/*
 * gm_serve_run -- continuous-batching request loop (sketch requests and
 * probability-Jaccard queries against a device-resident sketch store).
 * The trace `reqs` (nondecreasing arrival_us) is replayed open-loop against
 * the host clock (config.realtime = 1) or with every request present at
 * start (0).  Up to config.slots batches are in flight, one HIP stream each;
 * a free slot admits pending requests in arrival order while the batch holds
 * at most max_batch_requests requests and max_batch_entries sketch entries
 * and the in-flight device bytes stay within device_budget_bytes.  A busy
 * slot counts its staging buffers plus its stream's library workspace
 * (gm_workspace_bytes(max_batch_requests)); fewer slots than asked are used
 * when the budget holds fewer, and a budget below one slot is an argument
 * error.  A partial
 * batch waits for more requests until its oldest one has waited max_wait_us
 * (0: it launches at once; while every slot is busy, arrivals accumulate and
 * the next free slot takes them together).
 *   host_idx/host_w   host CSR entries of the sketch requests (request r
 *                     sketches entries [a, b); b - a <= max_batch_entries)
 *   store_idx         device [nstore * k] int32 sketch indices; a Jaccard
 *                     request compares store rows a and b
 *   out_sketch_idx/val  optional host [n_sketch * k] results, row i for the
 *                     i-th sketch request of the trace
 *   out_jaccard       host [nreq]: estimate of each Jaccard request
 *   out_done_us       host [nreq]: completion time from trace start
 * A request's sketch does not depend on what it was batched with.
 * Synchronous; allocates and frees its own slots.
 */
enum { GM_REQ_SKETCH = 0, GM_REQ_JACCARD = 1 };
typedef struct {
    double arrival_us;
    int32_t kind;
    int32_t pad;
    int64_t a, b;
} gm_request;
typedef struct {
    int32_t k;
    int32_t slots;
    int32_t max_batch_requests;
    int32_t realtime;
    int64_t max_batch_entries;
    int64_t device_budget_bytes;
    double max_wait_us;
    uint64_t seed;
} gm_serve_config;
typedef struct {
    int64_t batches, sketch_requests, jaccard_requests, entries;
    int64_t max_inflight_bytes, max_slots_busy, slots;
    double wall_us;
    int64_t slot_bytes;       /* device bytes one busy slot counts: staging + workspace */
    int64_t workspace_bytes;  /* of which the slot stream's library workspace */
} gm_serve_stats;
gm_status gm_serve_run(const gm_serve_config *cfg, const gm_request *reqs, int64_t nreq,
                       const int32_t *host_idx, const float *host_w,
                       const int32_t *store_idx, int64_t nstore,
                       int32_t *out_sketch_idx, double *out_sketch_val,
                       double *out_jaccard, double *out_done_us, gm_serve_stats *stats);

/* gm_status_string -- static text for a status code. */
const char *gm_status_string(gm_status status);

/* gm_release -- free the library's per-device workspaces (call when no
 * stream still has library work queued). */
void gm_release(void);

/* gm_release_stream -- free the workspace that FastGM calls created for
 * `stream` on the current device (synchronises the stream first); call it
 * before destroying a stream that ran FastGM calls. */
void gm_release_stream(hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GM_H */
