/*
 * fr_api.h -- C ABI of libflowroute, flow routing on a gridded DEM for AMD
 * MI355X (gfx950).
 *
 * What is computed (W. Bangerth, "Massively parallel flow routing and
 * drainage area determination"):
 *   - local flow routing (Section 2.1; Appendix A): for every cell, the
 *     neighbour(s) that receive its water;
 *   - global flow routing / drainage area (Section 1, Section 2.1): the water
 *     q that flows through every cell, i.e. the unique solution of
 *     (I - W^T) q = r (Section 2.2, eq. linear-system and eq. Aw=f), where r
 *     is the rain on each cell and W[i][k] the fraction of cell i's water that
 *     goes to cell k;
 *   - the adjoint: rbar = (I - W)^{-1} qbar, the gradient of a linear
 *     functional <qbar, q> with respect to the rain.
 *
 * Grids.  Row-major, C-contiguous, row 0 first in memory; cell (r, c) has
 * linear index r * ncols + c.  Neighbour k = 0..7 of a cell is, in
 * (drow, dcol): (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1) (+1,-1) (+1,0) (+1,+1)
 * ("row-major window order").  Off-grid neighbours do not exist.  Cell size
 * is 1; diagonal neighbours are at distance sqrt(2).
 *
 * Routing rules.
 *   FR_D8  -- each cell gives all its water to the strictly lower neighbour
 *             with the steepest slope s_k = fl(fl(z_i - z_k) * c_k),
 *             c_k = 1 (cardinal) or fl(1/sqrt(2)) (diagonal), computed in
 *             float32; ties go to the lowest k (Section 2.1, D8 scheme).
 *   FR_D4  -- as FR_D8 over the four cardinal neighbours (Section 2.1).
 *   FR_MFD -- each cell splits its water among all strictly lower neighbours
 *             with fractions f_k = s_k^p / sum_j s_j^p, s_k = (z_i - z_k)/d_k,
 *             d_k = 1 or sqrt(2) (Appendix A, multiple-flow-direction
 *             schemes).
 *   A cell with no strictly lower neighbour (boundary outlet, pit or flat)
 *   is a sink: its water leaves the grid there (Section 2.1 footnotes).
 *
 * Memory ownership.  Every pointer argument is caller-owned memory; the
 * library never allocates or frees caller memory.  Pointers documented as
 * "device" must be device (HBM) pointers valid on the current HIP device.
 * Scratch memory comes only through the (ws, ws_bytes) workspace argument,
 * sized by fr_workspace_bytes().  Calls on different streams must use
 * different workspaces.
 *
 * Streams.  All device work is ordered on the given stream, and
 * fr_receivers, fr_accumulate, fr_accumulate_adjoint and
 * fr_accumulate_batched never synchronise the host with it: they enqueue a
 * fixed sequence of kernels whose decisions (how many pointer-doubling
 * rounds, how many sweep passes, whether a fallback path runs) are taken on
 * the device, and return.  Such a call can be captured in a HIP graph and
 * replayed.  Results are complete when the stream reaches the point after
 * the call.  The block iterations and the depression fill read a small flag
 * back between iterations and say so below.
 *
 * Errors.  Return value: FR_OK (0) or a negative FR_ERR_* code from host-side
 * validation of the arguments, or a HIP error seen while enqueueing.
 * Conditions only the device can see (non-finite values, malformed codes,
 * cyclic routing) are reported through the optional device status word
 * `dev_status` (one int32 in device memory, which the caller zeroes before
 * the call): the library stores the first such FR_ERR_* code there; the
 * caller reads it after synchronising the stream.
 */
#ifndef FR_API_H
#define FR_API_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Routing rules. */
#define FR_D8 0
#define FR_MFD 1
#define FR_D4 2

/* Element types of water / rain / adjoint vectors. */
#define FR_NONE 0
#define FR_F32 1
#define FR_F64 2

/* Direction code of a sink in D8/D4 code arrays. */
#define FR_SINK 0xFF

/* Function identifiers for fr_workspace_bytes. */
#define FR_FN_ACCUMULATE 1
#define FR_FN_ADJOINT 2
#define FR_FN_BLOCK_ITER 3      /* block iterations, scheme FR_SCHEME_IX     */
#define FR_FN_BLOCK_ITER_PRE 4  /* block iterations, scheme FR_SCHEME_IMX_IX */
#define FR_FN_FILL 5            /* depression filling (dtype FR_F32)         */

/* Iteration schemes of fr_accumulate_block_iterations. */
#define FR_SCHEME_IX 0      /* Richardson on I + X                         */
#define FR_SCHEME_IMX_IX 1  /* Richardson on (I - X)(I + X)                */

/* Tile orders of fr_batch_plan.order. */
#define FR_ORDER_GIVEN 0
#define FR_ORDER_ROWS_DESC 1   /* tiles with more rows first              */
#define FR_ORDER_CELLS_DESC 2  /* tiles with more cells first             */

/* Status codes. */
#define FR_OK 0
#define FR_ERR_ARG -1        /* null pointer, negative size, bad flag        */
#define FR_ERR_RULE -2       /* unknown rule, or output not valid for rule   */
#define FR_ERR_WORKSPACE -3  /* workspace missing or smaller than required   */
#define FR_ERR_HIP -4        /* a HIP runtime call failed                    */
#define FR_ERR_NONFINITE -5  /* device: NaN or Inf in elevation or rain      */
#define FR_ERR_NOTDAG -6     /* device: routing has a cycle (bad codes)      */
#define FR_ERR_BADCODE -7    /* device: code not 0..7/0xFF or leaves the grid */
#define FR_ERR_TOOLARGE -8   /* grid larger than the library supports        */
#define FR_ERR_STALL -9      /* device: a persistent launch's workgroups could
                                not all run at once (barrier wait timed out) */
#define FR_ERR_CAPACITY -10  /* device: block iterations found more exits than
                                their workspace holds                        */

/*
 * fr_receivers -- local flow routing (Section 2.1; Appendix A for FR_MFD).
 *
 *   z         device, float32[nrows*ncols], elevations.
 *   nrows,
 *   ncols     grid shape, >= 0 each (an empty grid is a no-op); at most
 *             2^31 - 1 cells in total.
 *   rule      FR_D8, FR_D4 or FR_MFD.
 *   code_out  device, uint8[nrows*ncols], written:
 *               D8/D4: direction code k = 0..7 of the receiver, or FR_SINK;
 *               MFD:   bit k set when neighbour k is strictly lower
 *                      (0 = sink).
 *   dev_status optional device int32 (see Errors): FR_ERR_NONFINITE if z
 *             holds NaN or Inf (codes are then unspecified).
 *   stream    HIP stream.
 * Reads z once and writes code_out once.  Needs no workspace.
 */
int fr_receivers(const float* z, int64_t nrows, int64_t ncols, int rule, uint8_t* code_out,
                 int32_t* dev_status, hipStream_t stream);

/*
 * fr_accumulate -- global flow routing (Section 2.1 high-to-low algorithm,
 * Section 2.2 linear system, Appendix A for FR_MFD): solves
 * (I - W^T) q = r for q.  The result equals the high-to-low push; the GPU
 * reaches it without sorting: a cell is computed once all cells that give
 * it water are final, visiting rows in flow order (row sweeps with an exit
 * forest for D8/D4, wavefront sweeps for MFD, a peeling engine as the last
 * resort).
 *
 *   z         device float32 elevations; required for FR_MFD (fractions are
 *             recomputed from it), ignored (may be NULL) for FR_D8/FR_D4.
 *   code      device uint8 codes as written by fr_receivers for this rule.
 *   rule      FR_D8, FR_D4 or FR_MFD.
 *   mfd_p     slope exponent p of FR_MFD (> 0; 1.1 by default); ignored
 *             otherwise.
 *   rain      device rain per cell, element type rain_dtype, or NULL for
 *             unit rain (drainage area, Section 1).
 *   rain_dtype FR_F32 or FR_F64 (ignored when rain is NULL).
 *   q_dtype   FR_F32 (compensated float-float accumulation, float32 output),
 *             FR_F64 (float64 arithmetic and output) or FR_NONE (no q).
 *   q_out     device float32 or float64 [nrows*ncols] per q_dtype, or NULL
 *             when q_dtype is FR_NONE.
 *   counts_out device uint64 [nrows*ncols] exact number of cells draining
 *             through each cell (unit rain), or NULL.  FR_D8/FR_D4 only.
 *   mass_out  device float64[2] or NULL: {sum of q over sinks, sum of rain},
 *             both accumulated in float64 (Section 4 verification check).
 *             Requires q_dtype != FR_NONE.
 *   dev_status optional device int32: FR_ERR_NONFINITE (rain not finite),
 *             FR_ERR_BADCODE, FR_ERR_NOTDAG.
 *   ws, ws_bytes workspace, at least fr_workspace_bytes(FR_FN_ACCUMULATE,..).
 *   stream    HIP stream.
 * Enqueues its kernels and returns without synchronising (see Streams); the
 * outputs are complete when the stream has passed the call.  For FR_F32 and
 * FR_F64 the outputs are the same, bit for bit, on every run with the same
 * inputs.  q_out, counts_out and mass_out must not overlap z, code, rain,
 * the workspace or one another (no in-place routing: the solvers read the
 * inputs after they have written outputs): FR_ERR_ARG otherwise.
 */
int fr_accumulate(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                  double mfd_p, const void* rain, int rain_dtype, int q_dtype, void* q_out,
                  uint64_t* counts_out,
                  double* mass_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                  hipStream_t stream);

/*
 * fr_accumulate_noalloc -- fr_accumulate without a workspace argument, for
 * callers that cannot allocate device memory: code under HIP graph capture
 * that must not allocate, tight serving loops, harnesses that forbid
 * hipMalloc.  Scratch memory is a fixed array inside the library,
 * FR_NOALLOC_SCRATCH_BYTES on every GPU the library runs on, held until the
 * process ends; the call itself allocates nothing.  A grid whose workspace
 * (fr_workspace_bytes(FR_FN_ACCUMULATE, ...)) exceeds the array returns
 * FR_ERR_TOOLARGE.  All calls on one GPU share its array, which keeps the
 * last call's contents (every call clears what must start at zero): calls
 * that overlap on one GPU -- on different streams, or from different host
 * threads -- race, and must be serialised by the caller.  Arguments,
 * results, streams and errors otherwise as fr_accumulate.
 */
#define FR_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int fr_accumulate_noalloc(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                          double mfd_p, const void* rain, int rain_dtype, int q_dtype, void* q_out,
                          uint64_t* counts_out, double* mass_out, int32_t* dev_status, hipStream_t stream);

/*
 * fr_accumulate_adjoint -- transpose solve (I - W) rbar = qbar, i.e.
 * rbar_i = qbar_i + sum_k f_{i->k} rbar_k over the receivers k of i, swept
 * from sinks to sources.  rbar is the gradient of <qbar, q> with respect to
 * the rain r (A = I - W^T from Section 2.2, transposed).
 *
 *   z, code, rule, mfd_p   as for fr_accumulate.
 *   qbar      device vector of element type dtype (FR_F32 or FR_F64).
 *   dtype     FR_F32 (float-float accumulation, float32 output) or FR_F64.
 *   rbar_out  device vector of element type dtype, written.
 *   dev_status, ws, ws_bytes (FR_FN_ADJOINT), stream as above.
 */
int fr_accumulate_adjoint(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols,
                          int rule, double mfd_p, const void* qbar, int dtype, void* rbar_out,
                          int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fr_accumulate_block_iterations -- the paper's parallel scheme (Section
 * 3.3; Appendix B): block Richardson iterations.  The grid is cut into
 * blocks of block_rows x block_cols cells (the paper's per-process
 * subdomains).  Write A = I - W^T as D - R, where D holds every routing pair
 * inside a block and R every pair from one block into another; D^-1 is the
 * exact solve of each block on its own (the same row sweeps and exit forest
 * as fr_accumulate, with forest links kept inside the block), and R passes
 * each cell's water to a receiver in another block.  With X = -D^-1 R the
 * system reads (I + X) q = b, b = D^-1 r, and from w = 0:
 *   FR_SCHEME_IX      w <- D^-1 (r + R w)                      (eq. I+X)
 *   FR_SCHEME_IMX_IX  w <- w + (I - X)(b - (I + X) w): two block solves per
 *                     iteration plus one for b       (eq. (I-X)(I+X))
 * Iterates until one equals the previous one (on the counts where given):
 * the exact solution, reached after C + 1 (FR_SCHEME_IX) or
 * ceil((C + 1) / 2) (FR_SCHEME_IMX_IX) iterations when no flow path crosses
 * a block boundary more than C times (Appendix B).  Single-receiver rules.
 *
 *   z, mfd_p  reserved (pass NULL and 0).
 *   code      device uint8 codes (FR_D8 or FR_D4), as for fr_accumulate.
 *   block_rows, block_cols  block shape: block_cols a multiple of 256 or at
 *             least ncols; block_rows a multiple of 16 or at least nrows.
 *   scheme    FR_SCHEME_IX or FR_SCHEME_IMX_IX.
 *   rain, rain_dtype   as for fr_accumulate (NULL = unit rain).
 *   q_dtype   FR_F64 (float64 water into q_out) or FR_NONE (counts only).
 *   counts_out device uint64 cell counts, or NULL (FR_SCHEME_IX with
 *             q_dtype FR_F64 only: FR_SCHEME_IMX_IX decides convergence on
 *             the counts).  At least one output.
 *   max_iter  iteration budget (>= 1); no fixed point within max_iter + 1
 *             iterations sets FR_ERR_NOTDAG in dev_status.
 *   iters_out host int32: the number of iterations after which the iterate
 *             was exact (0 on an empty grid).
 *   ws, ws_bytes  workspace of fr_workspace_bytes(FR_FN_BLOCK_ITER or
 *             FR_FN_BLOCK_ITER_PRE for the scheme, ...).
 * Synchronises with the stream after every iteration (reads the change
 * flag).  Errors: FR_ERR_ARG (also a block shape not as above), FR_ERR_RULE
 * (not D8/D4), FR_ERR_WORKSPACE, FR_ERR_TOOLARGE, FR_ERR_HIP; in dev_status
 * as for fr_accumulate, and FR_ERR_CAPACITY when more cells leave their
 * tile than the exit list holds (an eighth of the cells on grids above 2^22
 * cells).
 */
int fr_accumulate_block_iterations(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                                   double mfd_p, int64_t block_rows, int64_t block_cols, int scheme,
                                   const void* rain, int rain_dtype, int q_dtype, void* q_out,
                                   uint64_t* counts_out, int32_t max_iter, int32_t* iters_out,
                                   int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fr_fill_depressions -- depression filling before routing (Section 4: the
 * DEM is filled by the priority-flood method so that all water reaches the
 * domain boundary).  Writes the filled surface F: F = z on the grid
 * boundary, elsewhere F(c) = max(z(c), min over neighbours n of next(F(n))),
 * next(x) being the next float32 above x when eps = 1 (then every interior
 * cell has a strictly lower neighbour and the rule routes it to the
 * boundary) or x itself when eps = 0 (depressions become flats).  This is
 * the priority-flood result, computed by tiled relaxation; it is exact (no
 * rounding), bit for bit.
 *
 *   z         device float32[nrows*ncols] elevations, all finite; -0 is read
 *             as +0.
 *   rule      FR_D8 or FR_MFD: 8 neighbours; FR_D4: the 4 cardinal ones
 *             (the neighbours the rule can route to).
 *   eps       1 (epsilon variant) or 0 (plain).
 *   f_out     device float32[nrows*ncols], written; must not alias z.
 *   launches_out  host int32 or NULL: tile launches until nothing changed
 *             (diagnostic).
 *   dev_status optional device int32: FR_ERR_NONFINITE if z holds NaN or Inf
 *             (f_out is then unspecified).
 *   ws, ws_bytes  workspace of fr_workspace_bytes(FR_FN_FILL, nrows, ncols,
 *             rule, FR_F32), a few bytes per 62 x 62 tile.
 * Synchronises with the stream every few launches.  Errors: FR_ERR_ARG,
 * FR_ERR_RULE, FR_ERR_WORKSPACE, FR_ERR_TOOLARGE, FR_ERR_HIP.
 */
int fr_fill_depressions(const float* z, int64_t nrows, int64_t ncols, int rule, int eps, float* f_out,
                        int32_t* launches_out, int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fr_workspace_bytes -- workspace size for fn = FR_FN_ACCUMULATE,
 * FR_FN_ADJOINT, FR_FN_BLOCK_ITER, FR_FN_BLOCK_ITER_PRE or FR_FN_FILL on an
 * nrows x ncols grid with this rule and dtype (FR_NONE means counts only).
 * Returns 0 for invalid arguments.
 */
size_t fr_workspace_bytes(int fn, int64_t nrows, int64_t ncols, int rule, int dtype);

/*
 * Phase timing (instrumentation).  fr_timing_enable(1) makes subsequent
 * fr_receivers / fr_accumulate / fr_accumulate_adjoint calls on this process
 * record HIP events around each of their GPU phases, on the call's stream;
 * fr_timing_enable(0) stops it (the default).  fr_timing_last fills up to
 * `max` entries of names[] (static strings) and ms[] (device milliseconds)
 * for the phases of the most recent timed call and returns how many it
 * filled; the call is complete when it returns, so reading is synchronous.
 * Phases: "receivers"; "d8_up", "d8_forest", "d8_down", "mass" (row-sweep
 * single-receiver path); "sweep" (wavefront sweep passes); "engine"
 * (peeling engine); "batch" (fr_accumulate_batched); "block_iterations"
 * (fr_accumulate_block_iterations); "fill" (fr_fill_depressions).  Not
 * thread-safe.
 */
int fr_timing_enable(int on);
int fr_timing_last(const char** names, float* ms, int max);

/*
 * Batched routing: many independent DEM tiles of uneven size routed by one
 * persistent kernel launch (receivers and accumulation, as fr_receivers +
 * fr_accumulate per tile), without any host synchronisation, so that the
 * call can be captured in a HIP graph.
 *
 * fr_tile describes one tile; all pointers are device pointers:
 *   z          float32[nrows*ncols] elevations (required).
 *   rain       float32[nrows*ncols] rain, or NULL for unit rain.
 *   q_out      float32[nrows*ncols] water (compensated float-float sums), or
 *              NULL; required for FR_MFD.
 *   counts_out uint64[nrows*ncols] drainage counts, or NULL; FR_D8/FR_D4
 *              only.  A D8/D4 tile gives exactly one of q_out and
 *              counts_out.
 *   code_out   uint8[nrows*ncols] receivers as fr_receivers writes them, or
 *              NULL (they are then kept in the workspace).
 *   nrows, ncols  tile shape, >= 1 each, at most 2^31 - 1 cells.
 *   rule       FR_D8, FR_D4 or FR_MFD (slope exponent 1.1).
 */
typedef struct fr_tile {
  const float* z;
  const float* rain;
  float* q_out;
  uint64_t* counts_out;
  uint8_t* code_out;
  int64_t nrows;
  int64_t ncols;
  int32_t rule;
  int32_t reserved;
} fr_tile;

/*
 * fr_batch_plan -- schedule of a batch: `workers` persistent workgroups
 * (0: two per compute unit; at least ceil(ncols / 48) of the widest tile,
 * whose column strips must all run at once -- a tile that needs more is
 * reported as FR_ERR_ARG in dev_status) and the tile `order`
 * (FR_ORDER_GIVEN, FR_ORDER_ROWS_DESC or FR_ORDER_CELLS_DESC).
 * fr_batch_autotune picks one by timing candidates.
 */
typedef struct fr_batch_plan {
  int32_t workers;
  int32_t order;
} fr_batch_plan;

/*
 * fr_batched_workspace_bytes -- workspace for a batch; tiles_host is a host
 * copy of the tile array (only shapes, rules and which outputs are NULL are
 * read).  Returns 0 for an invalid tile.
 */
size_t fr_batched_workspace_bytes(const fr_tile* tiles_host, int32_t ntiles);

/*
 * fr_accumulate_batched -- routes ntiles tiles.
 *   tiles_dev  device copy of the fr_tile array (read by the kernels).
 *   ntiles     >= 0.
 *   plan       schedule, or NULL for the default.
 *   dev_status optional device int32: FR_ERR_NONFINITE, FR_ERR_BADCODE,
 *              FR_ERR_NOTDAG as for fr_accumulate (first error of any tile).
 *   ws, ws_bytes workspace of at least fr_batched_workspace_bytes(); the
 *              caller passes the value it computed on the host copy.
 *   stream     HIP stream.
 * Enqueues three kernels (set-up, workspace fill, the persistent router) and
 * returns without synchronising.  Tile shapes are read on the device; the
 * caller guarantees that they match the ones ws_bytes was computed for.
 */
int fr_accumulate_batched(const fr_tile* tiles_dev, int32_t ntiles, const fr_batch_plan* plan,
                          int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fr_batch_autotune -- picks a plan for this batch: times
 * fr_accumulate_batched for every candidate plan -- one, one and a half and
 * two workgroups per compute unit, times the three tile orders; `reps`
 * timed runs each after one warm-up -- and writes the fastest to
 * *plan_out.  Plans are cached by the batch's signature (device, compute
 * units, and every tile's shape, rule and which of its pointers are NULL):
 * a batch with a cached signature gets its plan without timing.  The cache
 * lives in the process, and in the file set by fr_set_autotune_cache when
 * there is one.  Synchronises the stream; outputs of the tiles are
 * overwritten when it times.
 */
int fr_batch_autotune(const fr_tile* tiles_dev, int32_t ntiles, int32_t* dev_status, void* ws,
                      size_t ws_bytes, int reps, fr_batch_plan* plan_out, hipStream_t stream);

/*
 * fr_set_autotune_cache -- file that keeps fr_batch_autotune's plans across
 * processes (one "signature workers order" line per batch, read when set and
 * appended to when a new plan is found), or NULL for the process cache
 * alone.  Not thread-safe.  Errors: FR_ERR_ARG if the file cannot be read
 * or created.
 */
int fr_set_autotune_cache(const char* path);

/*
 * fr_set_accumulate_path -- process-wide choice of the accumulation path of
 * fr_accumulate and fr_accumulate_adjoint, for tests and diagnostics:
 * FR_PATH_AUTO (the default: row sweeps and exit forest for single
 * receivers -- the tile forest when a sample of the codes predicts flow in
 * every direction (more than 1.5x an eighth of the cells draining sideways
 * or to the next row, on grids of 2^18 cells and more) or their exit list
 * overflows --, the row
 * sweep or the wavefront sweep for MFD, the peeling engine when a sweep
 * gives up), FR_PATH_SWEEP (wavefront sweep, then the engine),
 * FR_PATH_ENGINE (the peeling engine alone) or FR_PATH_TILES (the tile
 * forest for single receivers at once, for terrain known to drain in every
 * direction such as a depression-filled DEM; MFD as FR_PATH_AUTO).  Every
 * path computes the same solution; only the time differs.  Not thread-safe.
 * Errors: FR_ERR_ARG.
 */
#define FR_PATH_AUTO 0
#define FR_PATH_SWEEP 1
#define FR_PATH_ENGINE 2
#define FR_PATH_TILES 3
int fr_set_accumulate_path(int path);

/*
 * fr_served_by -- which solver finished the most recent fr_accumulate or
 * fr_accumulate_adjoint call that used the workspace `ws` (diagnostics and
 * tests; the paths are those of fr_set_accumulate_path):
 *   FR_SERVED_ROWS       row sweeps and exit forest (D8 / D4, Section 2.1)
 *   FR_SERVED_TILES      tile forest: 32 x 64-cell tiles solved in LDS, joined
 *                        by the exit forest (D8 / D4 with flow in every
 *                        direction: predicted by the code sample, or the
 *                        row sweeps' exit list overflowed)
 *   FR_SERVED_ROW_SWEEP  MFD row sweep
 *   FR_SERVED_SWEEP      wavefront sweep
 *   FR_SERVED_ENGINE     peeling engine
 *   FR_SERVED_NONE       not known
 * Reads the workspace's control block with a copy on `stream` and waits for
 * it, so the answer covers every call enqueued before on that stream (calls
 * on empty grids use no workspace; a workspace that no call has used yet
 * gives an unspecified answer).  The workspace stays owned by the caller.  Errors: FR_ERR_ARG (NULL pointer,
 * ws_bytes below one control block), FR_ERR_HIP.
 */
#define FR_SERVED_NONE 0
#define FR_SERVED_ROWS 1
#define FR_SERVED_TILES 2
#define FR_SERVED_ROW_SWEEP 3
#define FR_SERVED_SWEEP 4
#define FR_SERVED_ENGINE 5
int fr_served_by(const void* ws, size_t ws_bytes, int32_t* served_out, hipStream_t stream);

/* fr_status_string -- static text for a status code. */
const char* fr_status_string(int code);

/* fr_version -- library version string. */
const char* fr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FR_API_H */
