/*
 * mclahe.h -- C ABI of the MI355X (gfx950) multidimensional CLAHE library.
 *
 * Multidimensional contrast limited adaptive histogram equalisation (MCLAHE,
 * Stimper, Bauer, Ernstorfer, Schoelkopf and Xian, 2019).  The method takes
 * an N-dimensional array, a kernel size per dimension, a number of histogram
 * bins, a clip limit normalised to [0, 1] and a choice of global or adaptive
 * (per-kernel) histogram range (Algorithm 1 and Sec. III.D), and computes:
 *
 *   1. the padding of Eq. 1 and its split of Eq. 2, as virtual symmetric
 *      (edge-repeating) padding; nothing is materialised;
 *   2. per-kernel histograms over the padded kernel grid (Alg. 1);
 *   3. clipping with equal redistribution of the excess (Alg. 1);
 *   4. the inclusive CDF, min-max normalised, as a per-kernel mapping table
 *      (LUT) (Alg. 1, Sec. III.C);
 *   5. Lagrange multilinear interpolation of the 2^D neighbouring kernels'
 *      mappings at every voxel (Sec. III.C).
 *
 * Readings of points the paper leaves open, identical to the test oracle:
 *   - Eq. 1 with the minus sign: p = 2b - 1 - ((s - 1) mod b), split
 *     p0 = p / 2 before, p1 = (p + 1) / 2 after; kernel_size[i] <= shape[i];
 *   - symmetric padding repeats the edge sample ([a b c] -> [b a|a b c|c b]);
 *   - bin of value v in single precision, no contraction:
 *       scale = (float)n_bins / (hi - lo);   t = (v - lo) * scale;
 *       bin = !(t > 0) ? 0 : (t >= n_bins ? n_bins - 1 : (int)t);
 *     (for hi == lo, scale is +inf and this gives v > lo ? n_bins-1 : 0);
 *   - global range = min and max of the input, unless the caller gives one;
 *     adaptive range = min and max over the kernel's padded voxels;
 *   - clip count C = floor(clip_limit * K), K = prod(kernel_size), for the
 *     decimal the caller wrote: a double product that falls short of the next
 *     integer by at most 2^-40 of itself counts as that integer (0.02 with
 *     K = 270000 gives 5400); C is capped at K (nothing is clipped there);
 *     excess E = sum_j max(h_j - C, 0) shared equally by all bins once; the
 *     library keeps it exact in units of 1/n_bins count:
 *       H_j = n_bins * min(h_j, C) + E;
 *   - LUT_j = (float)((double)(cdf_j - cdf_0) / (double)(cdf_last - cdf_0))
 *     with the inclusive cdf of H; a zero denominator gives j / (n_bins - 1);
 *   - kernel centres at k*b + (b-1)/2 in padded coordinates; a voxel x lies
 *     in the interpolation cell c = floor(m / 2b), m = 2(x + p0) - (b - 1),
 *     with weight (m - 2bc) / 2b towards kernel c + 1;
 *   - each of the 2^D kernels maps the voxel through its own LUT at the bin
 *     of the voxel under that kernel's range; contributions are summed;
 *   - float output lies in [0, 1]; u8/u16 output is
 *     min(M, floor(y * M + 0.5)) in single precision, M = 255 or 65535.
 *
 * Precision: histograms and clipped counts are exact integers; LUTs are
 * rounded once from double; the interpolated value is accumulated in float
 * (|error| <= 1e-5 of full scale), integer output within one level.
 *
 * Memory and ownership.  The caller owns every device buffer: input, output
 * and a workspace of mclahe_workspace_size() bytes (256-byte aligned).  The
 * library never allocates device memory in a run call (the batched calls
 * allocate pinned host staging buffers and keep cached graphs);
 * mclahe_plan allocates host memory only.  Arrays are C-contiguous, last axis
 * fastest.  Input and output may alias only if their element sizes match.
 * All run calls are asynchronous on the given HIP stream (NULL = the default
 * stream); a kernel fault surfaces at the caller's next synchronisation.
 *
 * Errors.  Every function returns an mclahe_status; no exception crosses the
 * ABI.  mclahe_last_error() returns a thread-local message describing the
 * last failure on the calling thread.
 */
#ifndef MCLAHE_H_
#define MCLAHE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCLAHE_SUCCESS = 0,
    MCLAHE_ERROR_INVALID_VALUE = 1,  /* bad argument (null, range, shape)      */
    MCLAHE_ERROR_NOT_SUPPORTED = 2,  /* valid but outside this build's limits  */
    MCLAHE_ERROR_OUT_OF_MEMORY = 3,  /* host allocation failed                 */
    MCLAHE_ERROR_WORKSPACE = 4,      /* workspace too small or misaligned      */
    MCLAHE_ERROR_HIP = 5             /* a HIP runtime call failed              */
} mclahe_status;

typedef enum { MCLAHE_U8 = 0, MCLAHE_U16 = 1, MCLAHE_F32 = 2 } mclahe_dtype;

/* Global histogram range (GHR) or adaptive, per-kernel range (AHR), Sec. III.D */
typedef enum { MCLAHE_RANGE_GLOBAL = 0, MCLAHE_RANGE_KERNEL = 1 } mclahe_range_mode;

typedef struct mclahe_plan_s *mclahe_plan_t;

/* Byte offsets into the workspace of the per-plan intermediate arrays, so
 * that tests can read them back.  N_k = number of kernels of the padded grid
 * (row-major over the kernel grid, last axis fastest), n = n_bins.
 *   hist    : u32 [N_k][n]   per-kernel histograms
 *   clipped : u64 [N_k][n]   H = n*min(h, C) + E (clip step, units of 1/n)
 *   lut     : f32 [N_k][n]   normalised CDF maps
 *   range   : f32 [N_k][2] (AHR) or [2] (GHR), lo then hi
 *   scale   : f32 [N_k] (AHR) or [1] (GHR), (float)n / (hi - lo)
 *   total   : bytes needed
 * These arrays come first; per-work-unit partials follow them.  The offsets
 * are the same when the plan runs in a batch (whose default work units are
 * coarser, so its per-volume workspace is at most `total`).                */
typedef struct {
    uint64_t hist, clipped, lut, range, scale, total;
} mclahe_layout;

/* Geometry of a plan, for inspection: per axis the padding p (Eq. 1), its
 * split p0/p1 (Eq. 2) and the number of kernels n = (s + p) / b; K = voxels
 * per kernel; clip_count = C; n_kernels = N_k; n_cells = number of
 * interpolation cells (prod(n_i - 1)).                                      */
typedef struct {
    int32_t ndim;
    int64_t pad[8], pad0[8], pad1[8], n_kernels_axis[8];
    int64_t n_kernels, kernel_voxels, clip_count, n_voxels, n_cells;
} mclahe_geometry;

/* Work decomposition knobs.  Any setting yields bit-identical results; only
 * speed changes.  Zero fields mean "library default".
 *   hist_rows_split   : row chunks per kernel column in the histogram pass
 *   hist_copies       : LDS histogram replicas (1, 2, 4, 8) against bin collisions
 *   hist_peel         : wavefront aggregation of colliding bins: 1 = off,
 *                       2 or 3 = one round (0 = default, off)
 *   map_rows_split    : row chunks per cell column in the interpolation pass
 *   map_group         : interpolation cells per work unit along the last axis
 *   map_unit_chunks   : row chunks an interpolation unit runs on one staging of
 *                       its LUTs (1 .. map_rows_split)                        */
typedef struct {
    int32_t hist_rows_split, hist_copies, hist_peel;
    int32_t map_rows_split, map_group, map_unit_chunks;
} mclahe_tuning;

/* Create a plan (host only; no device call).  Arguments follow the paper's
 * statement of the problem (Alg. 1 inputs and parameters; Sec. III.D):
 *   ndim         : 1..8
 *   shape        : ndim sizes s_i >= 1 (total voxels < 2^40)
 *   kernel_size  : ndim sizes 1 <= b_i <= s_i; prod(b) < 2^32
 *   n_bins       : 2..8192
 *   clip_limit   : finite, >= 0 (>= 1 disables clipping, 0 = uniform); a
 *                  double, so that a decimal limit keeps its exact count
 *   mode         : MCLAHE_RANGE_GLOBAL or MCLAHE_RANGE_KERNEL
 *   user_range   : NULL, or {lo, hi} finite with lo < hi (GLOBAL only)
 *   in_dtype     : u8, u16 or f32 (f32 input must be finite)
 *   out_dtype    : f32 (values in [0,1]) or u8/u16 codes
 * Returns INVALID_VALUE for arguments outside these ranges.                 */
mclahe_status mclahe_plan(mclahe_plan_t *plan, int ndim, const int64_t *shape,
                          const int64_t *kernel_size, int n_bins, double clip_limit,
                          mclahe_range_mode mode, const float *user_range,
                          mclahe_dtype in_dtype, mclahe_dtype out_dtype);

/* Release a plan (NULL is accepted).                                        */
mclahe_status mclahe_plan_destroy(mclahe_plan_t plan);

/* Geometry of Eq. 1-2 and the kernel grid for a plan.                       */
mclahe_status mclahe_plan_geometry(mclahe_plan_t plan, mclahe_geometry *geom);

/* Read or replace the plan's work decomposition.  Changing it changes the
 * workspace size; results stay bit-identical.  Not thread-safe against
 * concurrent runs of the same plan.                                         */
mclahe_status mclahe_plan_get_tuning(mclahe_plan_t plan, mclahe_tuning *tuning);
mclahe_status mclahe_plan_set_tuning(mclahe_plan_t plan, const mclahe_tuning *tuning);

/* Method variants for comparison with other CLAHE codes (a plan setting;
 * the default is the paper's method as read above):
 *   redistribution MCLAHE_REDIST_EQUAL    : the excess shared equally once;
 *                  MCLAHE_REDIST_REPEATED : shared equally, then the bins
 *                      above the clip level clipped again and the new excess
 *                      shared again, at most `rounds` (1..8) rounds, stopping
 *                      once no bin exceeds the level; round r counts in
 *                      integer units of 1/n_bins^r (clipped array likewise,
 *                      per kernel in the units of its last round); needs
 *                      n_bins^rounds * K < 2^63 (else NOT_SUPPORTED);
 *                  MCLAHE_REDIST_INTEGER  : integer counts: every bin gets
 *                      floor(E / n_bins), and the remainder R = E mod n_bins
 *                      one count each in bins 0, s, 2s, ... (R bins),
 *                      s = max(n_bins / R, 1) (clipped array in counts);
 *   centre MCLAHE_CENTRE_MIDDLE: kernel centres at k*b + (b-1)/2 (default);
 *          MCLAHE_CENTRE_HALF  : at k*b + b/2 (integer division), the
 *                                convention of some 2D codes (same for odd b).
 * Setting a variant re-derives the plan; workspace sizes do not change.
 * Errors: INVALID_VALUE for unknown values or rounds outside 1..8. */
typedef enum {
    MCLAHE_REDIST_EQUAL = 0, MCLAHE_REDIST_REPEATED = 1, MCLAHE_REDIST_INTEGER = 2
} mclahe_redistribution;
typedef enum { MCLAHE_CENTRE_MIDDLE = 0, MCLAHE_CENTRE_HALF = 1 } mclahe_centre;
typedef struct {
    int32_t redistribution;   /* mclahe_redistribution                      */
    int32_t rounds;           /* repeated redistribution: most rounds (1..8) */
    int32_t centre;           /* mclahe_centre                               */
} mclahe_variant;
mclahe_status mclahe_plan_get_variant(mclahe_plan_t plan, mclahe_variant *variant);
mclahe_status mclahe_plan_set_variant(mclahe_plan_t plan, const mclahe_variant *variant);

/* Workspace bytes for mclahe_run with the plan's current tuning.            */
mclahe_status mclahe_workspace_size(mclahe_plan_t plan, size_t *bytes);

/* Offsets of the intermediate arrays inside the workspace (see above).     */
mclahe_status mclahe_workspace_layout(mclahe_plan_t plan, mclahe_layout *layout);

/* Enhance one volume: d_in -> d_out, all four passes enqueued on hip_stream
 * (range, histogram, clip/CDF/LUT, interpolation).  d_workspace must be
 * 256-byte aligned and hold workspace_bytes >= mclahe_workspace_size();
 * d_in/d_out must be aligned to their element size (16 bytes enables wide
 * loads).  Returns WORKSPACE if the workspace is too small or misaligned. */
mclahe_status mclahe_run(mclahe_plan_t plan, const void *d_in, void *d_out,
                         void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* mclahe_run without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array
 * of MCLAHE_NOALLOC_SCRATCH_BYTES inside the library: every GPU the library
 * runs on holds its own copy from the first call on it until the process
 * ends.  The call allocates nothing (no hipMalloc, no hipFree); its first
 * call on a device looks up that device's copy.  Same kernels, work units
 * and bits as mclahe_run; the intermediate arrays are not readable.  Every
 * call on one GPU shares that GPU's array, which keeps the last call's
 * contents (no clearing is needed: each pass writes what the next reads):
 * calls that overlap on one GPU (different streams, or threads) race and
 * must be ordered by the caller.  d_in/d_out as for mclahe_run.
 * Errors: WORKSPACE if mclahe_workspace_size(plan) exceeds the array (the
 * call then touches no device), INVALID_VALUE for NULL or misaligned
 * buffers, HIP if the device or the array's address cannot be queried.     */
#define MCLAHE_NOALLOC_SCRATCH_BYTES (128ull << 20)
mclahe_status mclahe_run_noalloc(mclahe_plan_t plan, const void *d_in, void *d_out, void *hip_stream);

/* Workspace bytes for a batched call over n plans (sum of the per-volume
 * workspaces plus the descriptor table).                                    */
mclahe_status mclahe_batched_workspace_size(int n, const mclahe_plan_t *plans, size_t *bytes);

/* Per-volume workspace offsets inside a batched workspace: offsets[i] is the
 * byte offset of volume i's own workspace (laid out as mclahe_workspace_layout
 * of plans[i]).                                                             */
mclahe_status mclahe_batched_workspace_offsets(int n, const mclahe_plan_t *plans,
                                               uint64_t *offsets);

/* Enhance n independent volumes (mixed ndim, shape, dtype, parameters) as
 * one batch: each pass is ONE launch per kernel class (volumes that run the
 * same kernel template) over the work units of all its volumes, after one
 * stream-ordered copy of the batch's descriptor table into the workspace.
 * A batch whose structure (table address; kernel, volume count, grid, block
 * and LDS size of every launch) was seen before is replayed from a hipGraph
 * (LRU cache of 16); a new one is launched directly.  Each output (and each
 * intermediate array) is bit-identical to mclahe_run of the same plan.
 * Calls are stream-ordered; two calls in flight on different streams must
 * not share a workspace.                                                    */
mclahe_status mclahe_run_batched(int n, const mclahe_plan_t *plans,
                                 const void *const *d_in, void *const *d_out,
                                 void *d_workspace, size_t workspace_bytes,
                                 void *hip_stream);

/* The same batch as ONE persistent launch (after a kernel that clears the
 * run's counters, both replayed from a hipGraph when the batch repeats):
 * as many work-groups as fit the chip take tickets in order from one
 * counter, every ticket one work unit of one pass of one volume, passes in
 * order (range, histogram, clip/CDF/LUT, interpolation), volumes in batch
 * order within a pass.  A unit waits, polling an atomic completion counter,
 * until every unit of its volume's previous pass has finished; tickets come
 * in dependency order, so the lowest unfinished ticket never waits and the
 * run cannot deadlock.  Every wait is bounded as well: after max_spins polls
 * (0 = library default, about a second) it sets one abort word of the run;
 * every later wait sees the word and ends, every later unit is skipped, and
 * the kernel drains its tickets and ends normally.  mclahe_persistent_status
 * reads the word.  Same workspace and bits as mclahe_run_batched.
 * opts may be NULL.  flags MCLAHE_PERSIST_ABORT_TICKET makes ticket
 * abort_ticket give up without waiting (to exercise the abort path).       */
#define MCLAHE_PERSIST_ABORT_TICKET 1u
typedef struct {
    uint32_t max_spins;      /* polls of one wait before the run gives up; 0 = default */
    uint32_t abort_ticket;   /* with MCLAHE_PERSIST_ABORT_TICKET: this ticket gives up */
    uint32_t flags;
    uint32_t reserved;
} mclahe_persistent_opts;
mclahe_status mclahe_run_batched_persistent(int n, const mclahe_plan_t *plans,
                                            const void *const *d_in, void *const *d_out,
                                            void *d_workspace, size_t workspace_bytes,
                                            const mclahe_persistent_opts *opts, void *hip_stream);

/* After a persistent run on d_workspace (synchronises hip_stream): *aborted
 * = 0 if every unit ran, else 1 + the ticket whose wait gave up (the
 * outputs are then incomplete); *tickets (may be NULL) = tickets handed out
 * (at least the run's total: each work-group takes one more to learn the
 * queue is empty).                                                          */
mclahe_status mclahe_persistent_status(int n, const mclahe_plan_t *plans, const void *d_workspace,
                                       uint32_t *aborted, uint32_t *tickets, void *hip_stream);

/* Bytes of a batch's descriptor table (the head of a batched workspace,
 * before the first volume's own workspace).                                 */
mclahe_status mclahe_batched_table_size(int n, const mclahe_plan_t *plans, size_t *bytes);

/* mclahe_run_batched with the workspace split: volume i keeps its
 * histograms, clipped counts, LUTs and range in its own workspace d_ws[i]
 * of ws_bytes[i] >= mclahe_workspace_size(plans[i]) bytes, and the table
 * goes to d_table (table_bytes >= mclahe_batched_table_size, 256-byte
 * aligned).  For a serving loop that gives each request its own device
 * state.  The buffers must not overlap each other or any input/output
 * (except an in-place volume's own input and output).  Same kernels and the
 * same bits as mclahe_run_batched; errors as there, per volume.  Launches
 * directly every time (no graph capture: a serving loop's batches differ
 * from step to step).                                                       */
mclahe_status mclahe_run_batched_split(int n, const mclahe_plan_t *plans,
                                       const void *const *d_in, void *const *d_out,
                                       void *const *d_ws, const size_t *ws_bytes,
                                       void *d_table, size_t table_bytes,
                                       void *hip_stream);

/* Host image of the batch descriptor table that mclahe_run_batched would
 * upload for these arguments (no device call), for inspection and tests.
 * Copies min(image_bytes, *needed) bytes to host_image (may be NULL) and
 * stores the table size in *needed.  The image holds the library's internal
 * batch header, per-pass unit prefix sums and volume descriptors.           */
mclahe_status mclahe_batched_table(int n, const mclahe_plan_t *plans,
                                   const void *const *d_in, void *const *d_out,
                                   void *d_workspace, void *host_image,
                                   size_t image_bytes, size_t *needed);

/* Out-of-core run (the paper's Sec. V outlook: chunked processing of data
 * that do not fit in memory).  Input and output stay in HOST memory
 * (C-contiguous; pinned memory lets the copies run asynchronously; they must
 * not alias); the volume passes through the device workspace in slabs of
 * slab_layers kernel layers along axis 0 (rows of whole padded kernels).  A
 * global range is one streamed min/max pass over all slabs first; then each
 * slab is uploaded, histogrammed, clipped and turned into LUTs, and the
 * interpolation cells whose two kernel layers are ready are mapped, keeping
 * the last LUT layer of the previous slab as a one-layer halo; the output
 * rows go back to the host.  The result is bit-identical to mclahe_run.
 * Needs ndim >= 2.  The workspace (device, 256-byte aligned) holds one slab
 * of input and output rows, the slab's histograms and LUTs plus the halo:
 * mclahe_chunked_workspace_size().  Asynchronous on hip_stream like
 * mclahe_run: copies run on two internal copy streams of the library that
 * are ordered against hip_stream by events, and hip_stream completes only
 * after the last copy; host buffers must stay valid until then.  Calls on
 * one device are enqueued one at a time.
 * Errors: NOT_SUPPORTED for ndim < 2, INVALID_VALUE for slab_layers < 1,
 * NULL or aliasing buffers, WORKSPACE for a small or misaligned workspace. */
mclahe_status mclahe_chunked_workspace_size(mclahe_plan_t plan, int slab_layers, size_t *bytes);
mclahe_status mclahe_run_chunked(mclahe_plan_t plan, const void *h_in, void *h_out, int slab_layers,
                                 void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* Autotune the plan's work decomposition on the current device: times the
 * candidate settings on the given buffers (which it overwrites) and keeps
 * the fastest.  Needs workspace_bytes >= mclahe_autotune_workspace_size().
 * Synchronises hip_stream.  Results are cached per problem class in memory
 * and, if the environment variable MCLAHE_TUNE_CACHE names a file, there. */
mclahe_status mclahe_autotune_workspace_size(mclahe_plan_t plan, size_t *bytes);
mclahe_status mclahe_autotune(mclahe_plan_t plan, const void *d_in, void *d_out,
                              void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* Batch tuning: the work decomposition a plan uses inside batched calls
 * (mclahe_run_batched and friends), kept apart from the per-volume tuning
 * above.  Same fields and rules as mclahe_plan_get/set_tuning.              */
mclahe_status mclahe_plan_get_batch_tuning(mclahe_plan_t plan, mclahe_tuning *tuning);
mclahe_status mclahe_plan_set_batch_tuning(mclahe_plan_t plan, const mclahe_tuning *tuning);

/* Autotune the batch tuning of n plans together, on the given buffers
 * (overwritten), by timing whole mclahe_run_batched calls (graph replays):
 * per class of volumes that run the same kernels, the histogram row split
 * (default, 2 or 4 times fewer units) with 1, 2 or 4 LDS replicas, then the
 * interpolation row chunks per unit.  A result is kept only if it is faster
 * than the default batch tuning when both are timed again, so a tuned batch
 * is never slower than an untuned one; either way the outputs keep their
 * bits.  Batched workspace sizes may shrink afterwards (re-query
 * mclahe_batched_workspace_size).  The workspace must hold
 * mclahe_autotune_batched_workspace_size() bytes (the batch under default
 * batch tuning).  Synchronises hip_stream.  Results are cached per problem
 * class like mclahe_autotune's.                                             */
mclahe_status mclahe_autotune_batched_workspace_size(int n, const mclahe_plan_t *plans, size_t *bytes);
mclahe_status mclahe_autotune_batched(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                      void *const *d_out, void *d_workspace, size_t workspace_bytes,
                                      void *hip_stream);

/* Per-pass timing for benchmarks.  A timer holds HIP events for up to
 * max_runs calls; mclahe_run_timed is mclahe_run that also records an event
 * before each of the four passes and after the last (no synchronisation).
 * mclahe_timer_read synchronises on the last event and returns, per pass
 * (range, histogram, clip/CDF/LUT, interpolation), the mean milliseconds over
 * the recorded runs, and the number of runs; mclahe_timer_reset forgets them.
 * Calls past max_runs return INVALID_VALUE.                                 */
typedef struct mclahe_timer_s *mclahe_timer_t;
mclahe_status mclahe_timer_create(mclahe_timer_t *timer, int max_runs);
mclahe_status mclahe_timer_destroy(mclahe_timer_t timer);
mclahe_status mclahe_timer_reset(mclahe_timer_t timer);
mclahe_status mclahe_run_timed(mclahe_plan_t plan, const void *d_in, void *d_out, void *d_workspace,
                               size_t workspace_bytes, void *hip_stream, mclahe_timer_t timer);
mclahe_status mclahe_timer_read(mclahe_timer_t timer, float *pass_ms, int *runs);

/* Contrast metrics (the paper's Sec. II measures, used in Tables I and II to
 * judge enhancement): for a volume x, and optionally a second volume y of the
 * same voxel count (e.g. an enhanced result) judged against x:
 *   - lo, hi: minimum and maximum; each volume is min-max normalised to
 *     u = (v - lo) / (hi - lo) in [0, 1] (u = 0 where hi == lo) first;
 *   - mean and std: mean and population standard deviation (RMS contrast)
 *     of u;
 *   - entropy: Shannon entropy in bits, -sum p_j log2 p_j, of the n_bins-bin
 *     grey-level histogram of the raw values over [lo, hi], binned as the
 *     CLAHE histograms are (single precision: t = (v - lo) * (n_bins /
 *     (hi - lo)), bin = t > 0 ? min(floor(t), n_bins - 1) : 0);
 *   - mse = mean((u_x - u_y)^2) and psnr = 10 log10(peak^2 / mse) dB (+inf
 *     for mse = 0).  Both tables of the paper follow from peak = 2^23.
 * Sums are accumulated in double; results are reproducible bit for bit.
 * Without y (d_y = NULL), the [1] entries, mse and psnr are 0.
 * d_x, d_y: device arrays of nvox >= 1 elements of their dtypes, finite
 * values.  d_result: device pointer to one mclahe_metrics_result (written
 * when the stream reaches the last launch).  d_hist: optional device array
 * of 2 * n_bins uint64 receiving the histogram counts of x then y (NULL:
 * not written).  d_workspace: device, 256-byte aligned, at least
 * mclahe_metrics_workspace_size() bytes; owned by the caller, clobbered.
 * Asynchronous on hip_stream (four launches, no synchronisation).
 * Errors: INVALID_VALUE for nvox < 1, n_bins outside [2, 8192], NULL x or
 * result, an unknown dtype or a peak not positive and finite; WORKSPACE for
 * a small or misaligned workspace. */
typedef struct {
    double lo[2], hi[2];   /* minimum and maximum of x ([0]) and y ([1])      */
    double mean[2];        /* mean of the normalised volume                  */
    double std[2];         /* population standard deviation of it            */
    double entropy[2];     /* grey-level Shannon entropy in bits             */
    double mse;            /* mean squared difference of the normalised x, y */
    double psnr;           /* 10 log10(peak^2 / mse) in dB                    */
    uint64_t count;        /* voxels per volume                               */
} mclahe_metrics_result;
mclahe_status mclahe_metrics_workspace_size(int64_t nvox, int n_bins, size_t *bytes);

/* mclahe_run that also computes the contrast metrics (Sec. II; Tables I and
 * II) of the input x = d_in and the enhanced output y = d_out (its stored
 * values: codes for u8/u16 output), as mclahe_metrics(d_in, in_dtype, d_out,
 * out_dtype, ...) defines them, without its separate first pass: the
 * interpolation units write each unit's minimum, maximum and float64 sum of
 * x and y as they map; then one pass over both volumes takes the centred
 * sums and the grey-level histograms (their bins need the ranges first).
 * Same output bits as mclahe_run.  d_workspace: 256-byte aligned, at least
 * mclahe_run_metrics_workspace_size() bytes; its head is laid out as
 * mclahe_workspace_layout() describes.  n_bins, peak, d_result, d_hist as
 * for mclahe_metrics.  Not in place (d_in != d_out).
 * Errors: as mclahe_run and mclahe_metrics.                                */
mclahe_status mclahe_run_metrics_workspace_size(mclahe_plan_t plan, int n_bins, size_t *bytes);
mclahe_status mclahe_run_metrics(mclahe_plan_t plan, const void *d_in, void *d_out, void *d_workspace,
                                 size_t workspace_bytes, int n_bins, double peak,
                                 mclahe_metrics_result *d_result, uint64_t *d_hist, void *hip_stream);
mclahe_status mclahe_metrics(const void *d_x, mclahe_dtype x_dtype, const void *d_y, mclahe_dtype y_dtype,
                             int64_t nvox, int n_bins, double peak, mclahe_metrics_result *d_result,
                             uint64_t *d_hist, void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* Pre-denoising filters of the paper's experiments (Sec. IV): the
 * photoemission volume is smoothed by a Gaussian filter with a standard
 * deviation per axis, the microscopy volume by a median filter over a
 * (2, 2, 2, 1) window, before CLAHE.  Both take C-contiguous device arrays
 * of ndim (1..8) axes; input and output must not overlap.  Outside the array
 * the data continue by edge-repeating reflection ([a b c] -> [.. b a | a b c
 * | c b ..], repeated for windows longer than the axis), as in the CLAHE
 * padding.
 *
 * mclahe_gaussian: separable; one pass per axis with sigma[i] > 0, axes in
 * order 0..ndim-1 (sigma[i] = 0 leaves axis i alone).  Radius
 * r = (int)(truncate * sigma + 0.5) (truncate 4 is the common choice; r at
 * most 64); weights exp(-0.5 / sigma^2 * j^2) for j = -r..r divided by
 * their sum, in double, rounded to float.  Each output of a pass is the
 * single-precision fused multiply-add chain over j = -r..r starting from 0,
 * so results are reproducible bit for bit.  Input u8, u16 or f32; output
 * f32.  With two or more axes to smooth, a workspace of
 * mclahe_gaussian_workspace_size() bytes (one float volume, device,
 * 256-byte aligned, must not overlap the output) holds the intermediate
 * passes; otherwise it may be NULL.  Asynchronous on hip_stream.
 * Errors: INVALID_VALUE for a bad shape, NULL buffers, an unknown dtype, a
 * negative or non-finite sigma or truncate, or overlapping buffers;
 * NOT_SUPPORTED for a radius over 64; WORKSPACE for a small or misaligned
 * workspace.
 *
 * mclahe_median: window[i] >= 1 samples along axis i at offsets
 * -(window[i] / 2) .. window[i] - 1 - window[i] / 2 (for 2: the sample and
 * its predecessor); the output is the window value of rank N / 2 (0-based,
 * ascending), N = prod window[i] <= 64: the median for odd N, the upper of
 * the two middle values for even N.  Output in the input dtype, exact.
 * Asynchronous on hip_stream.  Errors: INVALID_VALUE for a bad shape or
 * window, NULL buffers, an unknown dtype or overlapping buffers;
 * NOT_SUPPORTED for N > 64. */
mclahe_status mclahe_gaussian_workspace_size(int ndim, const int64_t *shape, const double *sigma, size_t *bytes);
mclahe_status mclahe_gaussian(const void *d_in, mclahe_dtype in_dtype, int ndim, const int64_t *shape,
                              const double *sigma, double truncate, float *d_out, void *d_workspace,
                              size_t workspace_bytes, void *hip_stream);
mclahe_status mclahe_median(const void *d_in, mclahe_dtype dtype, int ndim, const int64_t *shape,
                            const int32_t *window, void *d_out, void *hip_stream);

/* Smoothing, then the method: mclahe_gaussian(d_in, in_dtype, plan's shape,
 * sigma, truncate) into d_smooth (float, the plan's input: the plan must
 * take f32), then mclahe_run(plan, d_smooth, d_out) -- the paper's pipeline
 * (Sec. IV: the photoemission volume is smoothed before CLAHE).  Under a
 * global range computed from the data, when the Gaussian's last pass is the
 * fused pass over the last two axes, that pass also takes the minimum and
 * maximum of what it writes, and the method's own range pass (a read of the
 * whole smoothed volume) is skipped.  Same bits as the two calls in order.
 * d_workspace: 256-byte aligned, mclahe_run_smoothed_workspace_size()
 * bytes; its head is laid out as mclahe_workspace_layout() describes.
 * d_smooth must not overlap d_in, d_out or the workspace.
 * Errors: as mclahe_gaussian and mclahe_run.                               */
mclahe_status mclahe_run_smoothed_workspace_size(mclahe_plan_t plan, const double *sigma, double truncate,
                                                 size_t *bytes);
mclahe_status mclahe_run_smoothed(mclahe_plan_t plan, const void *d_in, mclahe_dtype in_dtype,
                                  const double *sigma, double truncate, float *d_smooth, void *d_out,
                                  void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* Human-readable name of a status code (static storage).                   */
const char *mclahe_status_string(mclahe_status s);

/* Thread-local message for the last failure on this thread ("" if none).   */
const char *mclahe_last_error(void);

/* Library version, e.g. "0.1.0".                                            */
const char *mclahe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MCLAHE_H_ */
