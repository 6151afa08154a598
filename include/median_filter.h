/*
 * median_filter.h -- C ABI of the MI355X (gfx950) exact median-filter library.
 *
 * Method: B. Weiss, "Fast Isotropic Median Filtering" (SIGGRAPH 2025).  The
 * library filters an image with a disc, ellipse or convex-polygon window and
 * returns, for every pixel, the element of zero-based rank (N-1)/2 of the N
 * window values (section "Core concepts: Histograms, Pivots, and Counts":
 * for a 7x7 window, the 25th of 49).  The result is exact: it is always one
 * of the input values, bit for bit.  It is computed per tile with the
 * ordinal transform, the omnigram and pivot/count sliding (sections "The
 * Omnigram", "Method Summary", "Implementation" and "GPU").
 *
 * Conventions shared by every entry point
 *  - Image and output buffers are DEVICE pointers owned by the caller.  They
 *    are single-plane, row-major, with the same row stride in bytes; the
 *    stride must be >= w * element size and a multiple of the element size.
 *    Multi-channel (planar) images are filtered one plane per call or per
 *    batch entry.
 *  - Offsets are (dx, dy) with dx to the right and dy down the rows.
 *  - Pixels outside the image are taken from inside by the boundary rule:
 *    MF_CLAMP repeats the edge pixel; MF_MIRROR reflects about the edge pixel
 *    without repeating it (index -1 -> 1, w -> w-2), folding again as often
 *    as needed, so any radius is legal for any image size (w == 1 mirrors to
 *    index 0).
 *  - float32 values are ordered by IEEE 754 totalOrder: -0 < +0, and NaNs of
 *    either sign sort beyond the infinities of that sign.
 *  - Calls are asynchronous on `stream` (0 = the null stream).  Argument
 *    errors are returned before anything is queued; launch errors come back
 *    as MF_ERR_HIP.  No C++ exception crosses this interface.
 *  - `out` must not overlap `img` (MF_ERR_ALIAS): tiles read their
 *    neighbours' halo pixels while other tiles write.
 *  - w == 0 or h == 0 is a successful no-op.
 */
#ifndef MEDIAN_FILTER_H
#define MEDIAN_FILTER_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;

typedef enum { MF_U8 = 0, MF_U16 = 1, MF_F32 = 2 } mf_dtype;
typedef enum { MF_CLAMP = 0, MF_MIRROR = 1 } mf_boundary;
typedef enum {
  MF_OK = 0,
  MF_ERR_INVALID_ARG = -1, /* null pointer, bad size/stride/enum value          */
  MF_ERR_ALIAS = -2,       /* out overlaps img                                   */
  MF_ERR_UNSUPPORTED = -3, /* footprint not row- and column-convex, or too big   */
  MF_ERR_NOMEM = -4,       /* device or host allocation failed                   */
  MF_ERR_HIP = -5,         /* a HIP runtime call or kernel launch failed         */
  MF_ERR_SCRATCH_LIMIT = -6 /* needs more than the fixed scratch buffer holds    */
} mf_status;

/* Human-readable name of a status code (static storage; never NULL). */
const char* mf_status_string(int status);

/* ------------------------------------------------------------------------
 * Footprints (paper, Eq. 3 and "Arbitrary Convex Kernel Shapes").
 *
 * A footprint is an immutable host object owned by the caller.  It is
 * rasterised once into integer row spans; the GPU never evaluates geometry.
 * It must be row- and column-convex (each row and column of the window is
 * one run of pixels), which holds for every convex shape; the constructors
 * return MF_ERR_UNSUPPORTED otherwise.  Its offsets are limited to 255 in
 * each direction from the centre; the filter itself needs the window's
 * width and height to be at most 247 pixels (a disc of radius <= 123) and
 * returns MF_ERR_UNSUPPORTED beyond.  The library uploads the spans to each
 * device the first time the footprint is used there and keeps that copy
 * until mf_footprint_destroy.
 * ------------------------------------------------------------------------ */
typedef struct mf_footprint mf_footprint;

/* Disc of radius r: offsets with dx^2 + dy^2 <= r^2 (Eq. 3). r >= 0. */
int mf_footprint_disc(int r, mf_footprint** out);

/* Disc with an explicit squared limit: dx^2 + dy^2 <= limit.  limit = r(r+1)
 * gives the sets the paper's figures count (21 taps at radius 2). */
int mf_footprint_disc_limit(long long limit, mf_footprint** out);

/* Ellipse with semi-axes a, b (> 0) rotated by theta_deg (+x turns towards
 * +dy).  Member iff (u/a)^2 + (v/b)^2 <= 1 + 1e-9, u = dx cos + dy sin,
 * v = -dx sin + dy cos: lattice points on the boundary are members. */
int mf_footprint_ellipse(double a, double b, double theta_deg, mf_footprint** out);

/* Convex polygon from n_vertices (x, y) pairs in `xy`, either winding;
 * inclusive: points within 1e-9 * (max vertex radius) of an edge are members.
 * Collinear consecutive vertices are allowed.  A vertex list that is not
 * convex (a turn against the winding, or a star that winds more than once),
 * has zero area, a repeated vertex or a non-finite coordinate returns
 * MF_ERR_INVALID_ARG. */
int mf_footprint_polygon(const double* xy, int n_vertices, mf_footprint** out);

/* Regular polygon: vertices at angles rot_deg + 360 k / n_sides on a circle
 * of radius `circumradius` (a vertex on +x when rot_deg == 0). */
int mf_footprint_regular_polygon(int n_sides, double circumradius, double rot_deg,
                                 mf_footprint** out);

/* Tap count N, median rank (N-1)/2 and bounding offsets.  Any output
 * pointer may be NULL. */
int mf_footprint_info(const mf_footprint* fp, int* taps, int* rank, int* dx_min,
                      int* dx_max, int* dy_min, int* dy_max);

/* Host copy of the row spans: for row dy = dy_min + i, the window holds
 * dx in [x_lo[i], x_hi[i]].  Arrays have dy_max - dy_min + 1 entries. */
int mf_footprint_row_spans(const mf_footprint* fp, int* x_lo, int* x_hi);

void mf_footprint_destroy(mf_footprint* fp);

/* ------------------------------------------------------------------------
 * Plain filter (paper, "Method Summary" steps 1-5 and 7; "GPU").
 *
 * Filters one plane: out(x, y) = rank-(N-1)/2 element of the window values
 * around (x, y).  img/out: device pointers, stride_bytes as above; dtype is
 * an mf_dtype and boundary an mf_boundary.
 *
 * Memory: the first call with a footprint on a device uploads its span
 * table (kept until mf_footprint_destroy).  Large windows (global-scratch
 * tiles) use a scratch buffer cached per (device, stream), allocated on first
 * need and replaced by a larger one when a later call on that stream needs
 * more (2 bytes per box pixel and concurrent tile for 8/16-bit images, 8
 * for float32: 33 MB for radius 100 uint16, 133 MB for float32);
 * mf_release_scratch frees it.
 *
 * Graph capture: while `stream` is being captured the call never allocates.
 * It returns MF_ERR_UNSUPPORTED instead if the footprint's table is not yet
 * on the device or the stream's scratch is too small, so a call to be
 * captured needs one uncaptured call with the same footprint, dtype and an
 * image at least as large on that stream first.  Scratch used by a captured
 * call stays allocated (and is not reused for a larger size) until
 * mf_release_scratch.
 * ------------------------------------------------------------------------ */
int median_filter(const void* img, int w, int h, size_t stride_bytes, int dtype,
                  const mf_footprint* fp, int boundary, void* out, hipStream_t stream);

/* As median_filter, with an explicit zero-based rank in [0, N) instead of
 * the median: a percentile filter (paper, Conclusion and the percentile
 * figures of the appendix). */
int median_filter_rank(const void* img, int w, int h, size_t stride_bytes, int dtype,
                       const mf_footprint* fp, int boundary, int rank, void* out,
                       hipStream_t stream);

/* ------------------------------------------------------------------------
 * Chained tiles (paper, "Method Summary" step 6, forwarding last-row
 * solutions to the tile below; "Limitations and Future Work", ordinal
 * transform redundancy: reusing the ranking of the overlap of adjacent
 * input tiles).
 *
 * Same result as median_filter.  One workgroup walks `chain` (>= 1) tiles
 * of a tile column top to bottom.  Each tile after the first keeps the
 * part of its input box it shares with the tile above, already in ordinal
 * order, sorts only its new rows and merges the two by rank, and starts
 * its first band from the medians of the row above it, whose pixels'
 * offsets from their window centres carry over (the kept part keeps its
 * relative order, so each forwarded pixel has exactly the median rank's
 * count below it).  Windows whose box needs the global-scratch sort
 * (MF_ERR_UNSUPPORTED) are not chained.  On this GPU it is slower than
 * median_filter (tiles of a column run one after another and the merge
 * costs about what the saved sort did); it is provided for completeness
 * and measurement.
 * ------------------------------------------------------------------------ */
int median_filter_chained(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          const mf_footprint* fp, int boundary, int chain, void* out,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * Allocation-free median filter, for callers that cannot allocate device
 * memory: code under graph capture, tight serving loops, hosts that forbid
 * hipMalloc.
 *
 * Same arguments, result and kernels as median_filter.  It never calls
 * hipMalloc, hipFree or an allocating library routine: the footprint's span
 * table and the global-scratch sort slots of large windows live in one
 * fixed device array of MF_NOALLOC_SCRATCH_BYTES per GPU (64 KiB for the
 * span table, the rest for sort slots), held from the first call on that
 * GPU until the process ends.  The span table is written into it by a small
 * kernel on `stream` at every call (no host-to-device copy).  A large
 * window's persistent grid is shrunk to the sort slots that fit the array
 * (speed only; the output is unchanged); MF_ERR_SCRATCH_LIMIT if not even
 * one slot fits (no plan of this library needs that much today).
 *
 * The array is shared by every call on that GPU and keeps the last call's
 * contents; calls on one stream are ordered, but calls that overlap on one
 * GPU (other streams, other host threads) race on it and must be
 * serialised by the caller.  The first call on a GPU looks the array up
 * (hipGetSymbolAddress) with that GPU current.
 * ------------------------------------------------------------------------ */
#define MF_NOALLOC_SCRATCH_BYTES ((size_t)128 * 1024 * 1024 + (size_t)64 * 1024)
int median_filter_noalloc(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          const mf_footprint* fp, int boundary, void* out,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * General rank outputs (paper, Limitations and Future Work > Future Work >
 * Multi-Parameter Filtering: one ordinal transform can serve several
 * percentiles; Conclusion and the varying-percentile figure: the percentile
 * may change across the image).
 *
 * median_filter_ranks writes `nouts` planes (1..MF_MAX_RANK_OUTPUTS) from
 * one pass: each tile's box is loaded and sorted once, then its bands run
 * once per plane.  Plane q goes to outs[q].out (same shape and stride as
 * img) and holds, at pixel (x, y), the window element of zero-based rank
 *   rank_map[y * (rank_map_stride_bytes / 4) + x], clamped to [0, N - 1],
 *   where outs[q].rank_map is not NULL (device int32 plane, w x h, stride a
 *   multiple of 4 and >= 4 w), or
 *   outs[q].rank (0 <= rank < N, else MF_ERR_INVALID_ARG) where it is NULL.
 * A clamped entry below 0 selects the window minimum, one above N - 1 the
 * maximum.  Each output must not overlap the image, another output or any
 * rank map (MF_ERR_ALIAS); rank maps may overlap each other and the image.
 * Asynchronous on `stream`, like median_filter.
 *
 * median_filter_rank_map = median_filter_ranks with one plane whose rank
 * map is `rank_map` (not NULL).
 * ------------------------------------------------------------------------ */
#define MF_MAX_RANK_OUTPUTS 8
typedef struct {
  void* out;                    /* device plane */
  int rank;                     /* used where rank_map is NULL */
  const int* rank_map;          /* device int32 plane or NULL */
  size_t rank_map_stride_bytes; /* row stride of rank_map */
} mf_rank_output;

int median_filter_ranks(const void* img, int w, int h, size_t stride_bytes, int dtype,
                        const mf_footprint* fp, int boundary, const mf_rank_output* outs,
                        int nouts, hipStream_t stream);
int median_filter_rank_map(const void* img, int w, int h, size_t stride_bytes, int dtype,
                           const mf_footprint* fp, int boundary, const int* rank_map,
                           size_t rank_map_stride_bytes, void* out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Several windows from one ordinal transform (paper, Limitations and Future
 * Work > Future Work > Multi-Parameter Filtering: one ordinal transform can
 * serve filters of several radii, as long as each tile's box holds all their
 * windows).
 *
 * median_filter_windows writes `nouts` planes (1..MF_MAX_RANK_OUTPUTS) of
 * img, each with its own footprint: plane q (outs[q].out, same shape and
 * stride as img) holds at pixel (x, y) the element of zero-based rank
 *   rank_map[y * (rank_map_stride_bytes / 4) + x], clamped to [0, N_q - 1],
 *   where outs[q].rank_map is not NULL (as in mf_rank_output), else
 *   outs[q].rank (must be < N_q, else MF_ERR_INVALID_ARG; a negative rank
 *   selects the median (N_q - 1) / 2)
 * of the window outs[q].footprint (N_q taps) centred there.  Every
 * footprint must be non-NULL (MF_ERR_INVALID_ARG).
 *
 * The windows are grouped into passes: in decreasing order of the box
 * their own single-window plan loads (T_q pixels, for tiles of P_q), window
 * q joins the current pass, whose first window's box has T_0 pixels, while
 * (T_q / P_q) * N_q >= 0.25 * (T_0 - T_q), else it starts a new pass (a
 * small window in a much larger box walks over the extra pixels in every
 * omnigram scan, which can cost more than the shared sort saves; similar
 * windows share one pass).  A pass of one window is a median_filter_rank /
 * median_filter_rank_map call.  A pass of several loads and sorts each
 * tile's box (that of the smallest offset rectangle holding the pass's
 * windows) once and runs its bands once per plane with that plane's
 * window; if all of them are discs the disc membership test is used,
 * otherwise the span test.  Windows whose common rectangle exceeds the
 * largest box (off-centre shapes on opposite sides) run one pass each.
 * Passes are queued in order on `stream`.  The
 * planes equal, bit for bit, separate median_filter_rank /
 * median_filter_rank_map calls.  Aliasing rules, errors and stream
 * semantics as median_filter_ranks.
 *
 * mf_set_window_fusion(1) makes every later call use one pass for all its
 * windows (measurement and tests); 0 restores the grouping.  Process-wide;
 * returns MF_OK.
 * ------------------------------------------------------------------------ */
typedef struct {
  void* out;                        /* device plane */
  const mf_footprint* footprint;    /* this plane's window */
  int rank;                         /* used where rank_map is NULL; < 0: median */
  const int* rank_map;              /* device int32 plane or NULL */
  size_t rank_map_stride_bytes;     /* row stride of rank_map */
} mf_window_output;

int median_filter_windows(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          int boundary, const mf_window_output* outs, int nouts,
                          hipStream_t stream);
int mf_set_window_fusion(int all);

/* ------------------------------------------------------------------------
 * Batched filtering (not in the paper): many images of any sizes, dtypes
 * and footprints in one persistent launch.
 *
 * mf_plan_create validates every entry (as median_filter does, plus no
 * output may overlap any input or other output: MF_ERR_ALIAS), plans each
 * image exactly as median_filter would (the tuned tile shape for its dtype
 * and footprint when the tuned table has one -- loaded first from
 * `tune_cache_path` if not NULL -- else the default choice), groups all
 * tiles by kernel variant (dtype, footprint form, register capacity or
 * global scratch), orders each group longest-estimated-first, and allocates
 * the device tables: a descriptor per image, the tile queue, two counters
 * per group and, if some image needs it, global scratch; it also creates up
 * to three streams and four events of its own (default priority).  The plan
 * keeps the buffer pointers of `descs` (the device images themselves are
 * not copied): they must stay valid for every launch.  The footprints must
 * outlive the plan.  Synchronous.
 *
 * mf_plan_launch queues one kernel per group: global-scratch groups run a
 * persistent grid (CUs x occupancy workgroups popping tiles; the last one
 * resets the group's counters), the others one workgroup per tile.  With
 * more than one group it records an event on `stream`, makes the plan's
 * streams wait for it, spreads the groups over `stream` and those streams
 * (largest estimated total first, each onto the least loaded), and makes
 * `stream` wait for all of them again, so the whole launch is ordered on
 * `stream` like a single kernel.  Launches need no memset, allocate
 * nothing, and may be captured in a graph.  Launches of one plan must not
 * overlap in time.
 *
 * mf_plan_capture captures mf_plan_launch on `stream` (not the null
 * stream) into a hipGraph owned by the plan; mf_plan_replay launches that
 * graph on `stream`.
 *
 * median_filter_batched = create + launch + stream synchronize + destroy.
 * ------------------------------------------------------------------------ */
typedef struct {
  const void* img; /* device */
  void* out;       /* device, same stride as img */
  int w, h;
  size_t stride_bytes;
  int dtype;       /* mf_dtype */
  const mf_footprint* fp;
  int boundary;    /* mf_boundary */
} mf_image_desc;

typedef struct mf_plan mf_plan;

int mf_plan_create(const mf_image_desc* descs, int n, const char* tune_cache_path,
                   mf_plan** out);
int mf_plan_launch(mf_plan* plan, hipStream_t stream);
int mf_plan_capture(mf_plan* plan, hipStream_t stream);
int mf_plan_replay(mf_plan* plan, hipStream_t stream);
/* Total tiles, workgroups per launch (summed over groups), the largest LDS
 * bytes per workgroup, scratch bytes.  Any output pointer may be NULL. */
int mf_plan_info(const mf_plan* plan, int* tiles, int* grid, int* lds_bytes,
                 long long* scratch_bytes);
/* Number of kernel groups a launch runs and of streams it spreads them over
 * (0 and 0 for an empty plan).  Any output pointer may be NULL. */
int mf_plan_groups(const mf_plan* plan, int* groups, int* streams);
void mf_plan_destroy(mf_plan* plan);
int median_filter_batched(const mf_image_desc* descs, int n, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tile-shape control, for measurement and tuning.  tile_w/tile_h are the
 * output tile size, 1..64 by 1..256 (each of the 16 waves owns 64/tile_w
 * bands side by side, bands of ceil(tile_h / (16 * (64/tile_w))) rows, the
 * last one possibly shorter).  A shape whose input box exceeds 255 x 256
 * pixels, 65535 pixels or the LDS makes later calls return
 * MF_ERR_UNSUPPORTED.  (0, 0) restores the automatic choice.  Affects later
 * calls from every thread.
 * ------------------------------------------------------------------------ */
int mf_set_tile_override(int tile_w, int tile_h);

/* Free every scratch buffer the plain, general-rank and learned filters have
 * cached (all devices and streams).  Waits for each device to go idle.  No
 * filter call may be running and no graph captured around one may be
 * replayed afterwards (its scratch is gone); later calls allocate again. */
int mf_release_scratch(void);

/* Work counters of the tile engine, for the benchmark's work model.
 * enable = 1: allocate (once) and zero ten device counters that later calls
 * accumulate into: [0] wave-cooperative omnigram blocks scanned (64
 * ordinals each), [1] seed windows solved, [2] [3] [4] shader clocks summed
 * over waves spent in load + sort, in seeds and first band rows, and in
 * vertical sweeps, [5] number of waves summed, [6] lane-parallel 8-ordinal
 * groups tested, [7] box pixels ranked by the ordinal transforms, [8]
 * shader clocks in seed solves (part of [3]), [9] shader clocks from tile start
 * to the box loaded (part of [2]; 0 for global-scratch tiles).  The
 * learned and bracketed filters count into the same counters.  enable = 0:
 * stop counting and free them.  enable = -1: copy the ten counters to the
 * host array `out10` (synchronous).  Not thread-safe against concurrent
 * filter calls.  Counting adds a few scalar instructions per block. */
int mf_work_counters(int enable, unsigned long long* out10);

/* ------------------------------------------------------------------------
 * Autotuner (not in the paper).  Times every valid tile shape of the plain
 * filter for this (dtype, footprint) on the caller's image: img/out as in
 * median_filter (device buffers; out is overwritten), `reps` timed runs per
 * shape after one warm-up, on `stream` (synchronous: returns when timing
 * is done).  The fastest shape is recorded in the library's tuned-shape
 * table, which later plain calls and batched plans consult for the same
 * dtype and footprint.  Outputs (any may be NULL): the shape and its mean
 * time in milliseconds.
 * ------------------------------------------------------------------------ */
int mf_autotune(const void* img, int w, int h, size_t stride_bytes, int dtype,
                const mf_footprint* fp, int boundary, void* out, hipStream_t stream, int reps,
                int* best_tile_w, int* best_tile_h, float* best_ms);

/* Batch-aware tuning (not in the paper): tile shapes tuned one image at a
 * time can slow a batch down (fewer, longer tiles balance worse across the
 * batch's launches).  For each (dtype, footprint) of the batch, costliest
 * first, times the batch (mf_plan_create + `reps` mf_plan_launch calls on
 * `stream` after one warm-up) with that footprint's recorded shape and
 * with the default shape, and keeps in the tuned-shape table whichever
 * makes the whole batch faster; footprints without a recorded shape are
 * left alone.  Synchronous.  Outputs (any may be NULL): batch time before
 * and after (ms), and the number of footprints whose recorded shape was
 * dropped.  Later plain calls and plans use the table as left. */
int mf_plan_autotune(const mf_image_desc* descs, int n, hipStream_t stream, int reps,
                     float* before_ms, float* after_ms, int* dropped);

/* Tuned-shape table persistence: a JSON array, one object per line with
 * "key", "tile_w", "tile_h", "ms".  Load merges into the table (existing
 * keys are replaced); save writes the whole table.  MF_ERR_INVALID_ARG if
 * the file cannot be opened. */
int mf_tune_cache_load(const char* path);
int mf_tune_cache_save(const char* path);

/* The tile shape and launch the plain filter would use for this image and
 * footprint: output tile size, input box size (tile + window extent) and
 * the LDS bytes per workgroup.  Host-only; runs no GPU code. */
int mf_query_plan(int w, int h, int dtype, const mf_footprint* fp, int* tile_w, int* tile_h,
                  int* box_w, int* box_h, int* lds_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MEDIAN_FILTER_H */
