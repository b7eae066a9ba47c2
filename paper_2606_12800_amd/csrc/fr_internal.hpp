// Internal declarations of libflowroute (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fr_api.h"

namespace fr {

// Neighbour k = 0..7 in row-major window order; the neighbour in direction
// 7 - k is the opposite one, so cell j = i + off[k] reaches i by direction
// 7 - k.
__host__ __device__ constexpr int nb_dr(int k) { return k < 3 ? -1 : (k < 5 ? 0 : 1); }
__host__ __device__ constexpr int nb_dc(int k) {
  return (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
}
__host__ __device__ constexpr bool nb_diag(int k) { return k == 0 || k == 2 || k == 5 || k == 7; }

constexpr uint8_t SINK = 0xFF;

// Rule families inside the engine: one receiver per cell (D8 / D4 codes) or
// several (MFD lower-neighbour masks).
enum RuleKind { RK_SINGLE = 0, RK_MULTI = 1 };
// Sweep direction: forward accumulation (sources -> sinks) or adjoint
// (sinks -> sources).
enum Dir { DIR_FWD = 0, DIR_ADJ = 1 };
// Value arithmetic: none (counts only), float-float (float32 output), float64.
enum ValKind { VK_NONE = 0, VK_FF = 1, VK_F64 = 2 };

// Tile shape of the peeling engine (cells held in LDS by one workgroup).
constexpr int ENG_TH = 32;
constexpr int ENG_TW = 64;
constexpr int ENG_THREADS = 256;

struct EngineParams {
  int64_t nrows, ncols;
  int32_t ntr, ntc;            // tile grid
  const uint8_t* code;         // D8/D4 direction codes or MFD masks
  const float* z;              // elevations (MFD)
  double p;                    // MFD slope exponent
  const float* src32;          // source term (rain or qbar), float32, or NULL
  const double* src64;         // source term float64, or NULL (both NULL: unit)
  float* vhi;                  // float-float value, high part (= float32 output)
  float* vlo;                  // float-float value, low part (workspace)
  double* v64;                 // float64 value (output)
  uint64_t* cnt;               // exact counts (D8 forward), or NULL
  float* rs32;                 // MFD: 1 / steepest slope of the cell (float32 mode)
  float* iw32;                 // MFD: 1 / sum of normalised weights (float32 mode)
  float* d32;                  // MFD: 1 - sum of the cell's float32 fractions (float32 mode)
  double* iw64;                // MFD: 1 / sum of weights (float64 mode)
  uint8_t* ext;                // per cell: inputs in other tiles not yet finished
  uint8_t* done;               // per cell: 1 once its value is final
  int32_t* stamp;              // per tile: last iteration it was queued for
  int32_t* list0;              // active tile lists (ping-pong)
  int32_t* list1;
  int32_t* nlist;              // [3] ring of list lengths
  unsigned long long* remaining;  // cells not yet finished
  int32_t* status;             // device status word or NULL
  const int32_t* gate;         // run only when *gate != 0 (NULL: always)
  unsigned long long* bar;     // grid barrier arrivals of the persistent launch
};

// Row-sweep single-receiver path (fr_d8.hip): tile = D8Params::th rows x
// D8_TW columns, one wavefront per tile with 4 columns per lane.
constexpr int D8_TW = 256;
// Tile height: taller tiles mean fewer exits (fewer, shallower forest
// rounds); shorter tiles mean more wavefronts, and a tile's rows are swept
// one after another.  Grids below 2^28 cells get tiles short enough for
// about 2048 wavefronts (down to 16 rows).
inline int d8_tile_height(int64_t nrows, int64_t ncols) {
  if (nrows * ncols >= ((int64_t)1 << 28)) return 512;
  const int64_t tcols = (ncols + D8_TW - 1) / D8_TW;
  int th = 256;
  while (th > 16 && ((nrows + th - 1) / th) * tcols < 2048) th /= 2;
  return th;
}
// Blocks of the block iterations: 256 columns x this many rows.
inline int block_iter_height(int64_t nrows, int64_t ncols) {
  return nrows * ncols >= ((int64_t)1 << 28) ? 512 : 256;
}

// Control words of one call, at the start of its workspace (first 256
// bytes): the decisions that would otherwise need the host -- whether the
// exit list overflowed, whether the sweep is done, which way its next pass
// goes -- are taken on the device, so that a call is ordered on its stream
// alone and can be captured in a HIP graph.  Zeroed by the call's first
// kernel.
struct CallCtl {
  int32_t fallback;          // 1: the peeling engine runs (exit list overflow, sweep budget spent)
  int32_t sweep_stop;        // 1: no further sweep pass runs
  int32_t sweep_dir;         // row direction of the next sweep pass (-1 or +1)
  uint32_t sweep_fin[2];     // cells the last pass going up / down finished
  uint32_t loc_max_f;        // D8 forest: largest |local sum| of an exit, float32 bits
  int64_t sweep_remaining;   // cells not yet final
  uint64_t loc_max_d;        // D8 forest: largest |local sum| of an exit, float64 bits
  unsigned long long bar;    // persistent engine: grid barrier arrivals
  int32_t forest_final;      // D8 forest: the pending-additions buffer of the last round
  int32_t ms_flags;          // MFD row sweep: MS_* bits from the check and the decision
  int32_t ms_skip;           // 1: the row sweep does not serve this call (gate of the general mass)
  int32_t d8_tiles;          // 1: the tile-forest path serves this call (the row sweeps' exits overflowed)
  int32_t served;            // FR_SERVED_* of the path the host enqueued first (device gates may override)
  uint32_t probe_cnt;        // D8 probe: sampled cells that drain sideways or to the next row
};
static_assert(sizeof(CallCtl) <= 256, "control block fits its 256-byte slot");
constexpr int CTL_WORDS = 64;  // 32-bit words zeroed at the start of a call

struct D8Params {
  int64_t nrows, ncols;
  int32_t ntr, ntc;
  int32_t th;                  // tile height
  const uint8_t* code;
  const float* rain32;         // or NULL
  const double* rain64;        // or NULL (both NULL: unit rain)
  float* q32;                  // outputs (NULL when not requested)
  double* q64;
  uint64_t* cnt;
  uint32_t* root_of;           // per cell, written for inlets: root cell
  uint32_t* node_of;           // per cell, written for exits: exit index
  uint32_t* ex_cell;           // exit list [cap]
  float* ex_hi;                // local (in-tile) sums of the exits: float-float
  float* ex_lo;
  double* ex_d;                // float64
  uint64_t* ex_cnt[3];         // exit counts: sums [0], additions pending [1], [2]
  unsigned __int128* ex_fx[3]; // exit water as 128-bit fixed point (unit 2^E), likewise
  float* tot_hi;               // forest totals for phase C: float-float
  float* tot_lo;
  double* tot_d;               // float64
  uint32_t* anc[2];
  uint32_t* n_exits;           // exit counter
  uint32_t cap;
  int32_t* flags;              // pointer-doubling round flags
  CallCtl* ctl;
  double* mass_part;           // per tile {sum over sinks, sum of rain}, or NULL
  int32_t* status;
  // Block iterations (the paper's I+X scheme): blocks of bt_r x bt_c tiles
  // (0: a plain solve, no blocks); the previous iterate, read at donors in
  // other blocks; a flag set when an iterate differs from the previous one.
  int32_t bt_r, bt_c;
  const double* it_q64;
  const uint64_t* it_cnt;
  int32_t* it_changed;
  int32_t it_first;            // first iteration: no water crosses a block boundary yet
  int32_t it_nosrc;            // apply D^-1 R only: no rain, no unit count source
  int32_t it_detect;           // compare with the previous iterate (set it_changed)
};

// Exit-list slots reserved per atomic in phase A (at least).  A phase-A
// wavefront leaves unused slots only in its last chunk, so a tile's exits
// take at most their number plus D8_EXIT_CHUNK slots.
constexpr uint32_t D8_EXIT_CHUNK = 32;


// Tile-forest path (fr_d8_tiles.hip): single-receiver solves for flow in
// every direction, tiles of D8T_ROWS x D8T_COLS cells solved in LDS, joined
// by the exit forest.  Its exit list never holds more than
// d8t_exit_bound() entries; its mass partials (d8t_mass_words() doubles) are
// reduced in runs of D8T_MASS_RUN tiles, then once more.
constexpr int D8T_ROWS = 32;
constexpr int D8T_COLS = 64;
constexpr int D8T_MASS_RUN = 4096;
int64_t d8t_tiles(int64_t nrows, int64_t ncols);
uint64_t d8t_exit_bound(int64_t nrows, int64_t ncols);
size_t d8t_mass_words(int64_t nrows, int64_t ncols);
// Opens the path's gate (C->d8_tiles) when the row sweeps' exit list
// overflowed (C->fallback) or `force`, closing the engine's gate again.
hipError_t launch_d8t_gate(CallCtl* C, bool force, hipStream_t s);
// Phase A (up) or C (down) of every tile; both return at once while the
// gate is closed.
hipError_t launch_d8t(bool up, ValKind vk, bool cnt, const D8Params& P, hipStream_t s);
// Samples every 64th row of the codes before the row sweeps: when the cells
// that drain sideways or to the next row predict an overflow of the row
// sweeps' exit list, the list is marked overflowed at once (its count set
// above capacity), so that the row sweeps return at once and the tile
// forest serves the call.
hipError_t launch_d8_probe(const D8Params& P, double limit, hipStream_t s);
// Sums the tiles' mass partials into out[0..1] when the gate is open.
hipError_t launch_d8t_mass(const double* part, int64_t ntiles, double* out, CallCtl* C, hipStream_t s);

// Launchers (defined in the .hip files).
// Phase A (local sums and roots), phase B (exit forest: link, then enough
// pointer-doubling rounds for a forest of P.cap exits -- each a no-op once
// the forest is done or when the exit list overflowed -- then the totals),
// phase C (final sweep).  `iter`: the block
// iteration variants (blocks of P.bt_r x P.bt_c tiles).
hipError_t launch_d8_up(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s);
hipError_t launch_d8_forest(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s);
// The same forest by a work queue over the exits (the tile-forest path).
hipError_t launch_d8_forest_queue(ValKind vk, bool cnt, const D8Params& P, hipStream_t s);
hipError_t launch_d8_down(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s);
// Element-wise steps of the (I - X)(I + X) iteration on float64 values and
// uint64 (wrap-around) counts; either array pair may be NULL.
//   mode 0 (residual): t = b - w + t
//   mode 1 (update):   o = w + t + o, *changed = 1 where o's counts differ from w's
//   mode 2 (clear):    o = 0
hipError_t launch_bi_combine(int mode, int64_t n, const double* bq, const uint64_t* bc, const double* wq,
                             const uint64_t* wc, double* tq, uint64_t* tc, double* oq, uint64_t* oc,
                             int32_t* changed, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s);
// Final mass reduction of per-block partials; skipped when `skip` is given
// and *skip != 0 (the result then comes from another path).
hipError_t launch_mass_final(const double* partial, int nblocks, double* out, const int32_t* skip,
                             hipStream_t s);
// As launch_mass_final, but the reduction runs only when *open != 0.
hipError_t launch_mass_final_if(const double* partial, int nblocks, double* out, const int32_t* open,
                                hipStream_t s);
hipError_t launch_receivers(const float* z, int64_t nrows, int64_t ncols, int rule, uint8_t* code,
                            int32_t* status, hipStream_t s);

struct EngineConfig {
  RuleKind rk;
  Dir dir;
  ValKind vk;
  bool counts;
};

// Receiver code of a cell at elevation zi whose neighbours (row-major window
// order) are at zk[8], +inf off the grid: D8/D4 -- the strictly lower
// neighbour with the steepest float32 slope fl(fl(zi - zk) * c_k), ties to
// the lowest k, or SINK; MFD -- the mask of strictly lower neighbours.
template <int RULE>
__device__ __forceinline__ uint8_t route_code(float zi, const float zk[8]) {
  if (RULE == FR_MFD) {
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) m |= (zk[k] < zi) ? (1u << k) : 0u;
    return (uint8_t)m;
  }
  int best = -1;
  float bs = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (RULE == FR_D4 && nb_diag(k)) continue;
    if (!(zk[k] < zi)) continue;
    const float drop = zi - zk[k];
    const float sl = nb_diag(k) ? drop * 0x1.6a09e6p-1f : drop;
    if (best < 0 || sl > bs) {
      best = k;
      bs = sl;
    }
  }
  return best < 0 ? SINK : (uint8_t)best;
}

// Windowed wavefront sweep (fr_wsweep.hip): one wavefront per strip of
// WS_OWN owned columns (64 computed), rows visited in passes of alternating
// direction.
constexpr int WS_EW = 4;      // 64-bit words per edge record
constexpr int WS_GHOST = 8;   // columns recomputed on each side of a strip
constexpr int WS_OWN = 64 - 2 * WS_GHOST;
constexpr int BATCH_MAXPASS = 32;
constexpr int BATCH_CTR_WORDS = 64;  // per tile: [pass] finished, then the words below
constexpr int BCTR_BAR = 32, BCTR_UP = 33, BCTR_DN = 34;

inline __host__ __device__ size_t ws_align(size_t x) { return (x + 255) / 256 * 256; }
inline __host__ __device__ int64_t ws_strip_count(int64_t ncols) { return (ncols + WS_OWN - 1) / WS_OWN; }

// Workspace of one tile of a batch (offsets within the tile's block).
struct BatchTileLayout {
  size_t code, vhi, vlo, edge, progress, ctr, total;
};
// ff: the tile has a float32 water output (else its float-float values live
// in the workspace and only counts are written).
inline __host__ __device__ BatchTileLayout batch_tile_layout(int64_t nrows, int64_t ncols, bool own_codes,
                                                             bool ff) {
  BatchTileLayout L{};
  const size_t n = (size_t)(nrows * ncols);
  const size_t strips = (size_t)ws_strip_count(ncols);
  size_t o = 0;
  L.code = o; if (own_codes) o += ws_align(n);
  L.vhi = o; if (!ff) o += ws_align(n * 4);
  L.vlo = o; o += ws_align(n * 4);
  L.edge = o; o += ws_align(strips * (size_t)nrows * 2 * WS_EW * 8);
  L.progress = o; o += ws_align(strips * BATCH_MAXPASS * 4);
  L.ctr = o; o += ws_align(BATCH_CTR_WORDS * 4);
  L.total = o;
  return L;
}

// Per-tile record the set-up kernel writes into the batch workspace.
struct BatchTileInfo {
  const float* z;
  const float* rain;
  float* q;
  uint64_t* cnt;
  uint8_t* code;
  float* vhi;
  float* vlo;
  uint64_t* edge;
  int32_t* progress;
  uint32_t* ctr;
  int64_t nrows, ncols;
  int64_t strip_base;  // first work item of the tile in schedule order
  int32_t nstrips, rule;
};

struct BatchHeader {
  unsigned long long ticket;  // next work item
  int64_t total_items;
  int64_t ws_needed;
  int32_t ntiles, order;
};

// Batch workspace: header, tile records, schedule (tile index by position),
// first work item by position (ntiles + 1 entries), then the tile blocks.
inline __host__ __device__ size_t batch_head_bytes(int64_t ntiles) {
  return ws_align(sizeof(BatchHeader)) + ws_align((size_t)ntiles * sizeof(BatchTileInfo)) +
         ws_align((size_t)ntiles * 4) + ws_align((size_t)(ntiles + 1) * 8);
}
inline __host__ __device__ bool batch_tile_ff(int rule, bool has_q) { return rule == FR_MFD || has_q; }

struct WsParams {
  int64_t nrows, ncols;
  const uint8_t* code;
  const float* z;          // elevations (MFD)
  double p;                // MFD slope exponent
  const float* src32;      // source term float32, or NULL
  const double* src64;     // source term float64, or NULL (both NULL: unit)
  float* vhi;              // float-float value, high part (= float32 output)
  float* vlo;              // float-float low part (workspace; NaN = unfinished)
  double* v64;             // float64 value (output; NaN = unfinished)
  uint64_t* cnt;           // counts (output; all ones = unfinished when no value)
  uint64_t* edge;          // [strip][row][side][WS_EW] edge records
  int32_t* progress;       // [strip] last row step finished in this pass (-1 before)
  uint32_t* ctr;           // [0] cells finished by the last pass, [1]/[2] probe counts
  int32_t* status;
  int debug;               // float64 value: unfinished cells carry their state in the NaN payload
  // MFD float-float variant only: codes are D8/D4 directions (turned into
  // one-bit masks, fraction 1), and counts written from the (integer)
  // float-float values, exact below 2^31.
  int codes_single;
  uint64_t* cnt_ff;
};

size_t ws_edge_words(int64_t nrows, int64_t ncols);
hipError_t launch_batch(const void* tiles_dev, int32_t ntiles, int order, int workers, int32_t* status,
                        char* ws, size_t ws_bytes, hipStream_t s);
// Row sweep for MFD masks (fr_msweep.hip): one wavefront per strip of
// MS_OWN columns, computing MS_G ghost columns on each side; owned results
// published in a ring of MS_RING rows per strip.
constexpr int MS_G = 16;
constexpr int MS_OWN = 64 - 2 * MS_G;
constexpr int MS_NB = (MS_G + MS_OWN - 1) / MS_OWN;  // strips on each side that hold ghost columns
constexpr int MS_RING = 64;
enum : int32_t {
  MS_UP = 2,        // check: some cell sends to row r - 1
  MS_DN = 4,        // check: some cell sends to row r + 1
  MS_TAKEN = 8,     // decision: the row sweep serves the call
  MS_FLOW_UP = 16,  // decision: receivers lie in row r - 1
};
struct MsParams {
  int64_t nrows, ncols;
  const uint8_t* code;     // MFD masks
  const float* z;
  double p;
  const float* src32;      // rain / qbar, float32, or NULL
  const double* src64;     // float64, or NULL (both NULL: unit)
  float* vhi;              // float32 output (float-float accumulation), or NULL
  double* v64;             // float64 output, or NULL
  uint64_t* ring;          // [strip][MS_RING][MS_OWN] published words
  int32_t* progress;       // [strip] rows finished
  double* partial;         // [strip][2] mass partials (forward), or NULL
  int32_t* status;
  int32_t nstrips;
};
int64_t ms_strips(int64_t ncols);
size_t ms_ring_words(int64_t ncols);
int64_t ms_max_strips(ValKind vk);
// Check, decision and the sweep; every kernel after the decision is gated by
// the control block.
hipError_t launch_ms(ValKind vk, bool adjoint, const MsParams& P, CallCtl* C, hipStream_t s);
int64_t ws_strips(int64_t ncols);
// Wavefront sweep: set-up (edge records, direction probe, first pass's
// control), then passes, each followed by a control step that counts the
// cells finished, picks the next direction and stops the sequence (done,
// cycle, device error) or, after the last pass of the budget, opens the
// engine's gate.  Passes return at once after a stop.
hipError_t launch_ws_setup(const EngineConfig& cfg, const WsParams& P, CallCtl* C, hipStream_t s);
hipError_t launch_ws_pass(const EngineConfig& cfg, const WsParams& P, const CallCtl* C, int first,
                          hipStream_t s);
hipError_t launch_ws_ctl(const WsParams& P, CallCtl* C, int pass, bool last, hipStream_t s);

// The peeling engine: set-up, then one persistent launch that runs its
// iterations with grid barriers until every cell is final (or a cycle
// leaves the queue empty).  Both return at once when P.gate is closed.
hipError_t launch_engine_init(const EngineConfig& cfg, const EngineParams& P, hipStream_t s);
hipError_t launch_engine_run(const EngineConfig& cfg, const EngineParams& P, hipStream_t s);
hipError_t launch_mass(RuleKind rk, ValKind vk, const EngineParams& P, double* partial,
                       int nblocks, double* mass_out, hipStream_t s);
hipError_t launch_set_status(int32_t* status, int32_t code, hipStream_t s);
// Depression filling: tile grid and work lists (workspace).
struct FillState {
  int32_t ntr, ntc;  // tiles of 62 x 62 cells
  int32_t* queued;   // per tile: latest launch it was queued for
  int32_t* list;     // three lists of ntr * ntc tile indices (ring)
  int32_t* nlist;    // [3] their lengths
  int32_t* last;     // latest launch in which a tile changed
};
hipError_t launch_fill_init(const float* z, float* F, int64_t nr, int64_t nc, const FillState& S, int32_t* status,
                            hipStream_t s);
hipError_t launch_fill_tiles(const float* z, float* F, int64_t nr, int64_t nc, bool eps, bool c8,
                             const FillState& S, int32_t k, hipStream_t s);
hipError_t launch_zero_f64(double* p, int n, hipStream_t s);

}  // namespace fr
