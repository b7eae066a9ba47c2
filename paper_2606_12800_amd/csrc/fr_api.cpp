// Host side of the C ABI declared in fr_api.h: argument validation,
// workspace carving, kernel enqueue and the iteration driver.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fr_internal.hpp"

// Scratch of fr_accumulate_noalloc: one copy on every GPU the library runs
// on.  Host code never passes this name to a kernel (in host code it is a
// stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[FR_NOALLOC_SCRATCH_BYTES];

namespace fr {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMassBlocks = 1024;
constexpr int64_t kMaxCells = 2147483647;  // cell indices fit in int32

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Every workspace of fr_accumulate, fr_accumulate_adjoint and the block
// iterations starts (at its first 256-byte aligned address) with the call's
// control block; the layouts below are relative to the byte after it.
constexpr size_t kCtlBytes = kAlign;

struct Layout {
  size_t vlo, ext, done, rs32, iw32, d32, iw64, stamp, list0, list1, ctr, partial, total;
};

int64_t tiles_of(int64_t nrows, int64_t ncols) {
  return ((nrows + ENG_TH - 1) / ENG_TH) * ((ncols + ENG_TW - 1) / ENG_TW);
}

// Peeling engine.  The float-float low part comes first, at the same offset
// as the wavefront sweep's, so that the mass reduction after either path
// reads it from one place.
Layout layout(int64_t nrows, int64_t ncols, int rule, int vdtype) {
  Layout L{};
  const size_t n = (size_t)(nrows * ncols);
  const size_t nt = (size_t)tiles_of(nrows, ncols);
  size_t o = 0;
  L.vlo = o; if (vdtype == FR_F32) o += up(n * sizeof(float));
  L.ext = o; o += up(n + 4);
  L.done = o; o += up(n + 4);
  L.rs32 = o; if (rule == FR_MFD && vdtype == FR_F32) o += up(n * sizeof(float));
  L.iw32 = o; if (rule == FR_MFD && vdtype == FR_F32) o += up(n * sizeof(float));
  L.d32 = o; if (rule == FR_MFD && vdtype == FR_F32) o += up(n * sizeof(float));
  L.iw64 = o; if (rule == FR_MFD && vdtype == FR_F64) o += up(n * sizeof(double));
  L.stamp = o; o += up(nt * sizeof(int32_t));
  L.list0 = o; o += up(nt * sizeof(int32_t));
  L.list1 = o; o += up(nt * sizeof(int32_t));
  L.ctr = o; o += kAlign;
  L.partial = o; o += up(2 * kMassBlocks * sizeof(double));
  L.total = o;
  return L;
}

// Row-sweep single-receiver path (fr_d8.hip).  The engine's layout overlays
// it: the engine only runs once this path gave up (exit list overflow), and
// then nothing reads this path's data any more.
struct D8Layout {
  size_t root_of, node_of, ex_cell, cnt[3], fx[3], anc, loc, ctr, mass, total;
  uint32_t cap;
};

// Exit capacity, plus a chunk of slack per tile (a phase-A wavefront leaves
// unused slots only in its last chunk): every cell on grids up to 2^22
// cells, so that the list cannot overflow there, else an eighth of the
// cells (at least 2^22).
constexpr int64_t kFullCapacityCells = (int64_t)1 << 22;
// Grids from this size on are probed for flow in every direction (below it
// the row sweeps serve every call).
constexpr int64_t kProbeCells = (int64_t)1 << 18;
uint32_t d8_capacity(int64_t n, int64_t ntiles) {
  const int64_t slack = (int64_t)D8_EXIT_CHUNK * ntiles;
  if (n <= kFullCapacityCells) return (uint32_t)((n > 0 ? n : 1) + slack);
  const int64_t c = n / 8;
  return (uint32_t)((c > kFullCapacityCells ? c : kFullCapacityCells) + slack);
}

// th: tile height (the mass partials are per tile).  Per exit: its cell,
// the sum and two buffers of pending additions (counts and 128-bit fixed
// point), two pointers, and the local sum of phase A (float-float or
// float64); the totals for phase C go into the two pointer buffers
// (contiguous, 8 bytes per exit) once the rounds are over.
D8Layout d8_layout(int64_t nrows, int64_t ncols, int th, int vdtype, bool counts) {
  D8Layout L{};
  const size_t n = (size_t)(nrows * ncols);
  const size_t nt = (size_t)(((nrows + th - 1) / th) * ((ncols + D8_TW - 1) / D8_TW));
  L.cap = d8_capacity((int64_t)n, (int64_t)nt);
  // The list also holds the tile-forest path's exits (fr_d8_tiles.hip).
  const uint64_t tb = d8t_exit_bound(nrows, ncols);
  if (tb > L.cap) L.cap = (uint32_t)tb;
  const size_t cap = L.cap;
  const bool vals = vdtype == FR_F32 || vdtype == FR_F64;
  size_t o = 0;
  L.root_of = o; o += up(n * 4);
  L.node_of = o; o += up(n * 4);
  L.ex_cell = o; o += up(cap * 4);
  for (int b = 0; b < 3; ++b) {
    L.cnt[b] = o;
    if (counts) o += up(cap * 8);
  }
  for (int b = 0; b < 3; ++b) {
    L.fx[b] = o;
    if (vals) o += up(cap * 16);
  }
  L.anc = o; o += up(cap * 8);
  L.loc = o; if (vals) o += up(cap * 8);
  L.ctr = o; o += kAlign;
  const size_t mw = d8t_mass_words(nrows, ncols) > nt * 2 ? d8t_mass_words(nrows, ncols) : nt * 2;
  L.mass = o; o += up(mw * sizeof(double));
  L.total = o;
  return L;
}

// Wavefront sweep (fr_wsweep.hip).  The engine overlays it too.
struct WsLayout {
  size_t vlo, edge, progress, ctr, partial, ms_ring, ms_progress, ms_partial, total;
};

WsLayout ws_layout(int64_t nrows, int64_t ncols, int vdtype) {
  WsLayout L{};
  const size_t n = (size_t)(nrows * ncols);
  size_t o = 0;
  L.vlo = o; if (vdtype == FR_F32) o += up(n * sizeof(float));
  L.edge = o; o += up(ws_edge_words(nrows, ncols) * sizeof(uint64_t));
  L.progress = o; o += up((size_t)ws_strips(ncols) * sizeof(int32_t));
  L.ctr = o; o += kAlign;
  L.partial = o; o += up(2 * kMassBlocks * sizeof(double));
  // Row sweep (MFD): published rows, progress and mass partials per strip.
  L.ms_ring = o; o += up(ms_ring_words(ncols) * sizeof(uint64_t));
  L.ms_progress = o; o += up((size_t)ms_strips(ncols) * sizeof(int32_t));
  L.ms_partial = o; o += up((size_t)ms_strips(ncols) * 2 * sizeof(double));
  L.total = o;
  return L;
}

// Row sweep parameters over the sweep's workspace; NULL outputs stay NULL.
MsParams ms_params(int64_t nrows, int64_t ncols, const uint8_t* code, const float* z, double p, char* body,
                   const WsLayout& L, int32_t* status) {
  MsParams M{};
  M.nrows = nrows;
  M.ncols = ncols;
  M.code = code;
  M.z = z;
  M.p = p;
  M.ring = reinterpret_cast<uint64_t*>(body + L.ms_ring);
  M.progress = reinterpret_cast<int32_t*>(body + L.ms_progress);
  M.partial = reinterpret_cast<double*>(body + L.ms_partial);
  M.status = status;
  M.nstrips = (int32_t)ms_strips(ncols);
  return M;
}

struct Counters {
  int32_t nlist[3];
  int32_t pad;
  unsigned long long remaining;
  unsigned long long bar;
};

bool valid_rule(int rule) { return rule == FR_D8 || rule == FR_D4 || rule == FR_MFD; }

// True when the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

int cu_count() {
  static int cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cache[dev] = v;
  }
  return cache[dev];
}

// ---------------------------------------------------------------------------
// Phase timing (instrumentation only; off by default).
constexpr int kMaxPhases = 8;
struct Timing {
  bool on = false;
  int n = 0;
  const char* names[kMaxPhases];
  hipEvent_t ev[kMaxPhases][2];
  bool created = false;
  int device = -1;
};
Timing g_timing;

bool timing_ready() {
  if (!g_timing.on) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (!g_timing.created || g_timing.device != dev) {
    for (int i = 0; i < kMaxPhases; ++i)
      for (int j = 0; j < 2; ++j)
        if (hipEventCreate(&g_timing.ev[i][j]) != hipSuccess) return false;
    g_timing.created = true;
    g_timing.device = dev;
  }
  return true;
}

void timing_reset() { g_timing.n = 0; }

// Returns the slot of a new phase, or -1 when timing is off.
int phase_begin(const char* name, hipStream_t s) {
  if (!timing_ready() || g_timing.n >= kMaxPhases) return -1;
  const int i = g_timing.n++;
  g_timing.names[i] = name;
  (void)hipEventRecord(g_timing.ev[i][0], s);
  return i;
}

void phase_end(int i, hipStream_t s) {
  if (i >= 0) (void)hipEventRecord(g_timing.ev[i][1], s);
}

// Accumulation path (fr_set_accumulate_path): every path computes the same
// result; the default picks the row sweeps for single receivers.
int g_path = FR_PATH_AUTO;

// The row sweep is tried for MFD masks under the automatic path choice when
// all of its strips can be resident at once.
bool ms_applicable(RuleKind rk, ValKind vk, int64_t ncols) {
  return rk == RK_MULTI && (g_path == FR_PATH_AUTO || g_path == FR_PATH_TILES) &&
         ms_strips(ncols) <= ms_max_strips(vk);
}

constexpr int kMaxSweepPasses = 32;

char* aligned_base(void* ws) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<char*>((a + kAlign - 1) / kAlign * kAlign);
}

EngineParams engine_params(int64_t nrows, int64_t ncols, const uint8_t* code, const float* z, double p,
                           char* body, const Layout& L, int32_t* status, const int32_t* gate) {
  EngineParams P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.ntr = (int32_t)((nrows + ENG_TH - 1) / ENG_TH);
  P.ntc = (int32_t)((ncols + ENG_TW - 1) / ENG_TW);
  P.code = code;
  P.z = z;
  P.p = p;
  P.ext = reinterpret_cast<uint8_t*>(body + L.ext);
  P.done = reinterpret_cast<uint8_t*>(body + L.done);
  P.vlo = reinterpret_cast<float*>(body + L.vlo);
  P.rs32 = reinterpret_cast<float*>(body + L.rs32);
  P.iw32 = reinterpret_cast<float*>(body + L.iw32);
  P.d32 = reinterpret_cast<float*>(body + L.d32);
  P.iw64 = reinterpret_cast<double*>(body + L.iw64);
  P.stamp = reinterpret_cast<int32_t*>(body + L.stamp);
  P.list0 = reinterpret_cast<int32_t*>(body + L.list0);
  P.list1 = reinterpret_cast<int32_t*>(body + L.list1);
  Counters* c = reinterpret_cast<Counters*>(body + L.ctr);
  P.nlist = c->nlist;
  P.remaining = &c->remaining;
  P.bar = &c->bar;
  P.status = status;
  P.gate = gate;
  return P;
}

// The peeling engine behind a gate: its kernels run only when *gate != 0.
int enqueue_engine(const EngineConfig& cfg, const EngineParams& P, hipStream_t s) {
  const int ph = phase_begin("engine", s);
  if (launch_engine_init(cfg, P, s) != hipSuccess || launch_engine_run(cfg, P, s) != hipSuccess) return FR_ERR_HIP;
  phase_end(ph, s);
  return FR_OK;
}

D8Params d8_params(const uint8_t* code, int64_t nrows, int64_t ncols, int th, const void* rain, int rain_dtype,
                   ValKind vk, bool counts, char* body, CallCtl* C, int32_t* status, D8Layout* Lout) {
  const D8Layout L = d8_layout(nrows, ncols, th, vk == VK_FF ? FR_F32 : (vk == VK_F64 ? FR_F64 : FR_NONE), counts);
  D8Params P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.th = th;
  P.ntr = (int32_t)((nrows + P.th - 1) / P.th);
  P.ntc = (int32_t)((ncols + D8_TW - 1) / D8_TW);
  P.code = code;
  P.rain32 = (rain && rain_dtype == FR_F32) ? static_cast<const float*>(rain) : nullptr;
  P.rain64 = (rain && rain_dtype == FR_F64) ? static_cast<const double*>(rain) : nullptr;
  P.root_of = reinterpret_cast<uint32_t*>(body + L.root_of);
  P.node_of = reinterpret_cast<uint32_t*>(body + L.node_of);
  P.ex_cell = reinterpret_cast<uint32_t*>(body + L.ex_cell);
  for (int b = 0; b < 3; ++b) {
    P.ex_cnt[b] = reinterpret_cast<uint64_t*>(body + L.cnt[b]);
    P.ex_fx[b] = reinterpret_cast<unsigned __int128*>(body + L.fx[b]);
  }
  P.ex_hi = reinterpret_cast<float*>(body + L.loc);
  P.ex_lo = P.ex_hi + L.cap;
  P.ex_d = reinterpret_cast<double*>(body + L.loc);
  P.anc[0] = reinterpret_cast<uint32_t*>(body + L.anc);
  P.anc[1] = P.anc[0] + L.cap;
  P.tot_hi = reinterpret_cast<float*>(body + L.anc);
  P.tot_lo = P.tot_hi + L.cap;
  P.tot_d = reinterpret_cast<double*>(body + L.anc);
  uint32_t* ctr = reinterpret_cast<uint32_t*>(body + L.ctr);
  P.n_exits = ctr;
  P.flags = reinterpret_cast<int32_t*>(ctr + 4);
  P.cap = L.cap;
  P.ctl = C;
  P.status = status;
  if (Lout) *Lout = L;
  return P;
}

// Row-sweep path for single-receiver codes, forward solve: phases A, B, C
// and the mass reduction, every one of them ordered on the stream.  An exit
// list overflow opens C->fallback, which the enqueued engine then serves.
int enqueue_d8(const uint8_t* code, int64_t nrows, int64_t ncols, const void* rain, int rain_dtype, ValKind vk,
               float* q32, double* q64, uint64_t* cnt, double* mass_out, int32_t* status, char* body, CallCtl* C,
               bool tiles_only, hipStream_t s) {
  const bool counts = cnt != nullptr;
  D8Layout L{};
  D8Params P = d8_params(code, nrows, ncols, d8_tile_height(nrows, ncols), rain, rain_dtype, vk, counts, body, C,
                         status, &L);
  P.q32 = q32;
  P.q64 = q64;
  P.cnt = cnt;
  P.mass_part = mass_out ? reinterpret_cast<double*>(body + L.mass) : nullptr;
  if (launch_zero_u32(P.n_exits, 32, s) != hipSuccess) return FR_ERR_HIP;
  const bool probe = nrows * ncols >= kProbeCells;
  int ph = -1;
  if (!tiles_only) {
    // From 2^18 cells on, a sample of the codes (every 64th row) first
    // decides whether the row sweeps are worth trying: where more than 1.5x
    // an eighth of the cells (or of the list's capacity) would be exits --
    // flow in every direction, as on a depression-filled DEM -- the tile
    // forest serves the call (on filled DEMs of 2^18 to 2^22 cells it is
    // 1.6 to 4x faster; on tilted ones the row sweeps are).
    if (probe) {
      const double cells = (double)(nrows * ncols);
      const double lim = 1.5 * (cells / 8.0 < (double)P.cap ? cells / 8.0 : (double)P.cap);
      if (launch_d8_probe(P, lim, s) != hipSuccess) return FR_ERR_HIP;
    }
    ph = phase_begin("d8_up", s);
    if (launch_d8_up(vk, counts, false, P, s) != hipSuccess) return FR_ERR_HIP;
    phase_end(ph, s);
    ph = phase_begin("d8_forest", s);
    if (launch_d8_forest(vk, counts, false, P, s) != hipSuccess) return FR_ERR_HIP;
    phase_end(ph, s);
    ph = phase_begin("d8_down", s);
    if (launch_d8_down(vk, counts, false, P, s) != hipSuccess) return FR_ERR_HIP;
    phase_end(ph, s);
    if (mass_out) {
      ph = phase_begin("mass", s);
      if (launch_mass_final(P.mass_part, P.ntr * P.ntc, mass_out, &C->fallback, s) != hipSuccess) return FR_ERR_HIP;
      phase_end(ph, s);
    }
    if (!probe) return FR_OK;  // small grid: the row sweeps' list holds every cell
  }
  // Exit list overflow (flow in every direction), or the path chosen: the
  // tile-forest path, behind its gate, with an exit count and round flags of
  // its own.
  D8Params T = P;
  T.n_exits = P.n_exits + 16;
  T.flags = reinterpret_cast<int32_t*>(P.n_exits + 20);
  ph = phase_begin("d8_tiles", s);
  if (launch_d8t_gate(C, tiles_only, s) != hipSuccess || launch_d8t(true, vk, counts, T, s) != hipSuccess ||
      launch_d8_forest_queue(vk, counts, T, s) != hipSuccess || launch_d8t(false, vk, counts, T, s) != hipSuccess)
    return FR_ERR_HIP;
  if (mass_out && launch_d8t_mass(T.mass_part, d8t_tiles(nrows, ncols), mass_out, C, s) != hipSuccess)
    return FR_ERR_HIP;
  phase_end(ph, s);
  return FR_OK;
}

WsParams ws_params(int64_t nrows, int64_t ncols, const uint8_t* code, const float* z, double p, char* body,
                   const WsLayout& L, ValKind vk, int32_t* status) {
  WsParams P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.code = code;
  P.z = z;
  P.p = p;
  P.vlo = vk == VK_FF ? reinterpret_cast<float*>(body + L.vlo) : nullptr;
  P.edge = reinterpret_cast<uint64_t*>(body + L.edge);
  P.progress = reinterpret_cast<int32_t*>(body + L.progress);
  P.ctr = reinterpret_cast<uint32_t*>(body + L.ctr);
  P.status = status;
  P.debug = 0;
  return P;
}

// Wavefront-sweep passes, each followed by its control step: after the last
// pass of the budget, cells still unfinished open C->fallback.
int enqueue_ws(const EngineConfig& cfg, const WsParams& P, CallCtl* C, hipStream_t s) {
  const int ph = phase_begin("sweep", s);
  if (launch_ws_setup(cfg, P, C, s) != hipSuccess) return FR_ERR_HIP;
  for (int pass = 0; pass < kMaxSweepPasses; ++pass) {
    if (launch_ws_pass(cfg, P, C, pass == 0 ? 1 : 0, s) != hipSuccess ||
        launch_ws_ctl(P, C, pass, pass == kMaxSweepPasses - 1, s) != hipSuccess)
      return FR_ERR_HIP;
  }
  phase_end(ph, s);
  return FR_OK;
}

// Sets the control block's fallback word from the host's path choice
// (FR_PATH_ENGINE): the engine then serves the call on its own.
__global__ void k_open_gate(CallCtl* C) {
  if (threadIdx.x == 0) C->fallback = 1;
}

// Clears the control block at the start of a call and records the path the
// host enqueues first.
__global__ void k_ctl_init(CallCtl* C, int32_t served) {
  uint32_t* w = reinterpret_cast<uint32_t*>(C);
  for (int i = threadIdx.x; i < CTL_WORDS; i += blockDim.x) w[i] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) C->served = served;
}

hipError_t launch_ctl_init(CallCtl* C, int32_t served, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, C, served);
  return hipGetLastError();
}

}  // namespace
}  // namespace fr

using namespace fr;

extern "C" {

const char* fr_version(void) { return "libflowroute 0.1 (gfx950)"; }

int fr_timing_enable(int on) {
  g_timing.on = on != 0;
  g_timing.n = 0;
  return FR_OK;
}

int fr_timing_last(const char** names, float* ms, int max) {
  if (!names || !ms || max < 0) return FR_ERR_ARG;
  int k = 0;
  for (int i = 0; i < g_timing.n && k < max; ++i) {
    float t = 0.0f;
    if (hipEventSynchronize(g_timing.ev[i][1]) != hipSuccess) return FR_ERR_HIP;
    if (hipEventElapsedTime(&t, g_timing.ev[i][0], g_timing.ev[i][1]) != hipSuccess) return FR_ERR_HIP;
    names[k] = g_timing.names[i];
    ms[k] = t;
    ++k;
  }
  return k;
}

const char* fr_status_string(int code) {
  switch (code) {
    case FR_OK: return "ok";
    case FR_ERR_ARG: return "invalid argument";
    case FR_ERR_RULE: return "invalid routing rule or output for this rule";
    case FR_ERR_WORKSPACE: return "workspace missing or too small";
    case FR_ERR_HIP: return "HIP runtime error";
    case FR_ERR_NONFINITE: return "non-finite elevation or rain";
    case FR_ERR_NOTDAG: return "routing graph has a cycle";
    case FR_ERR_BADCODE: return "malformed routing code";
    case FR_ERR_TOOLARGE: return "grid too large";
    case FR_ERR_STALL: return "a persistent launch could not run all its workgroups at once";
    case FR_ERR_CAPACITY: return "more exits than the block iterations' workspace holds";
    default: return "unknown status";
  }
}

// Depression filling: per 62 x 62 tile a queue mark and three list slots,
// plus the list lengths and the last-change word.
constexpr int64_t kFillTile = 62;
size_t fill_bytes(int64_t nrows, int64_t ncols) {
  const size_t ntiles = (size_t)((nrows + kFillTile - 1) / kFillTile) * (size_t)((ncols + kFillTile - 1) / kFillTile);
  return up((4 * ntiles + 4) * sizeof(int32_t)) + kAlign;
}

// Block iterations: the control block, the row-sweep layout (tiles as
// short as 16 rows bound its per-tile words), then `vectors` float64 values
// and counts per cell (I+X: the other iterate; (I-X)(I+X): also D^-1 r and a
// temporary) and the change flag.
size_t block_iter_bytes(int64_t nrows, int64_t ncols, int vectors, int dtype) {
  const size_t n = (size_t)(nrows * ncols);
  const size_t d8 = d8_layout(nrows, ncols, 16, dtype, true).total;
  return kCtlBytes + d8 + (size_t)vectors * (up(n * sizeof(double)) + up(n * sizeof(uint64_t))) + 2 * kAlign;
}

size_t fr_workspace_bytes(int fn, int64_t nrows, int64_t ncols, int rule, int dtype) {
  if (nrows < 0 || ncols < 0 || !valid_rule(rule)) return 0;
  if (nrows > 0 && ncols > kMaxCells / (nrows > 0 ? nrows : 1)) return 0;
  if (fn == FR_FN_ACCUMULATE) {
    if (dtype != FR_NONE && dtype != FR_F32 && dtype != FR_F64) return 0;
    if (rule == FR_MFD && dtype == FR_NONE) return 0;
  } else if (fn == FR_FN_ADJOINT) {
    if (dtype != FR_F32 && dtype != FR_F64) return 0;
  } else if (fn == FR_FN_BLOCK_ITER || fn == FR_FN_BLOCK_ITER_PRE) {
    if (rule == FR_MFD || (dtype != FR_NONE && dtype != FR_F64)) return 0;
    return block_iter_bytes(nrows, ncols, fn == FR_FN_BLOCK_ITER_PRE ? 3 : 1, dtype);
  } else if (fn == FR_FN_FILL) {
    if (dtype != FR_F32) return 0;
    return fill_bytes(nrows, ncols);
  } else {
    return 0;
  }
  size_t t = layout(nrows, ncols, rule, dtype).total;
  const size_t tw = ws_layout(nrows, ncols, dtype).total;
  if (tw > t) t = tw;
  if (fn == FR_FN_ACCUMULATE && rule != FR_MFD) {
    // The counts buffers are sized in, whether or not counts are requested.
    const size_t t8 = d8_layout(nrows, ncols, d8_tile_height(nrows, ncols), dtype, true).total;
    if (t8 > t) t = t8;
  }
  return kCtlBytes + t + kAlign;
}

int fr_served_by(const void* ws, size_t ws_bytes, int32_t* served_out, hipStream_t stream) {
  if (!ws || !served_out || ws_bytes < kCtlBytes + kAlign) return FR_ERR_ARG;
  CallCtl c{};
  char* base = aligned_base(const_cast<void*>(ws));
  if (hipMemcpyAsync(&c, base, sizeof c, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return FR_ERR_HIP;
  int32_t v = c.served;
  if (c.fallback) v = FR_SERVED_ENGINE;
  else if (c.d8_tiles) v = FR_SERVED_TILES;
  else if (c.ms_flags & MS_TAKEN) v = FR_SERVED_ROW_SWEEP;
  *served_out = v >= FR_SERVED_NONE && v <= FR_SERVED_ENGINE ? v : FR_SERVED_NONE;
  return FR_OK;
}

int fr_set_accumulate_path(int path) {
  if (path != FR_PATH_AUTO && path != FR_PATH_SWEEP && path != FR_PATH_ENGINE && path != FR_PATH_TILES)
    return FR_ERR_ARG;
  g_path = path;
  return FR_OK;
}

int fr_receivers(const float* z, int64_t nrows, int64_t ncols, int rule, uint8_t* code_out,
                 int32_t* dev_status, hipStream_t stream) {
  if (nrows < 0 || ncols < 0) return FR_ERR_ARG;
  if (!valid_rule(rule)) return FR_ERR_RULE;
  if (nrows == 0 || ncols == 0) return FR_OK;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!z || !code_out) return FR_ERR_ARG;
  timing_reset();
  const int ph = phase_begin("receivers", stream);
  const hipError_t e = launch_receivers(z, nrows, ncols, rule, code_out, dev_status, stream);
  phase_end(ph, stream);
  return e == hipSuccess ? FR_OK : FR_ERR_HIP;
}

int fr_fill_depressions(const float* z, int64_t nrows, int64_t ncols, int rule, int eps, float* f_out,
                        int32_t* launches_out, int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nrows < 0 || ncols < 0 || (eps != 0 && eps != 1)) return FR_ERR_ARG;
  if (!valid_rule(rule)) return FR_ERR_RULE;
  if (launches_out) *launches_out = 0;
  if (nrows == 0 || ncols == 0) return FR_OK;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!z || !f_out || static_cast<const void*>(z) == static_cast<const void*>(f_out)) return FR_ERR_ARG;
  if (!ws || ws_bytes < fill_bytes(nrows, ncols)) return FR_ERR_WORKSPACE;
  timing_reset();
  const int32_t ntr = (int32_t)((nrows + kFillTile - 1) / kFillTile);
  const int32_t ntc = (int32_t)((ncols + kFillTile - 1) / kFillTile);
  const size_t ntiles = (size_t)ntr * ntc;
  FillState S;
  S.ntr = ntr;
  S.ntc = ntc;
  S.queued = reinterpret_cast<int32_t*>(aligned_base(ws));
  S.list = S.queued + ntiles;
  S.nlist = S.list + 3 * ntiles;
  S.last = S.nlist + 3;
  const bool c8 = rule != FR_D4;
  const int ph = phase_begin("fill", stream);
  int rc = FR_OK;
  if (launch_fill_init(z, f_out, nrows, ncols, S, dev_status, stream) != hipSuccess) rc = FR_ERR_HIP;
  // Launches go out in batches; after each the host reads the length of the
  // next work list: empty means no tile changed in the batch's final launch,
  // so none can change any more.  Every launch lowers values or changes
  // nothing, so this ends.
  constexpr int32_t kBatch = 8;
  for (int32_t k = 0; rc == FR_OK; k += kBatch) {
    for (int32_t j = k; j < k + kBatch && rc == FR_OK; ++j)
      if (launch_fill_tiles(z, f_out, nrows, ncols, eps != 0, c8, S, j, stream) != hipSuccess) rc = FR_ERR_HIP;
    int32_t pending = 0, lastk = 0, st = 0;
    if (rc != FR_OK ||
        hipMemcpyAsync(&pending, S.nlist + (k + kBatch) % 3, sizeof pending, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipMemcpyAsync(&lastk, S.last, sizeof lastk, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (dev_status && hipMemcpyAsync(&st, dev_status, sizeof st, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
      rc = FR_ERR_HIP;
      break;
    }
    if (st != 0) break;
    if (pending == 0) {
      if (launches_out) *launches_out = lastk + 2;  // through the first launch without a change
      break;
    }
  }
  phase_end(ph, stream);
  return rc;
}

int fr_accumulate(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule, double mfd_p,
                  const void* rain, int rain_dtype, int q_dtype, void* q_out, uint64_t* counts_out,
                  double* mass_out, int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nrows < 0 || ncols < 0) return FR_ERR_ARG;
  if (!valid_rule(rule)) return FR_ERR_RULE;
  if (rain && rain_dtype != FR_F32 && rain_dtype != FR_F64) return FR_ERR_ARG;
  if (q_dtype != FR_NONE && q_dtype != FR_F32 && q_dtype != FR_F64) return FR_ERR_ARG;
  if (mass_out && q_dtype == FR_NONE) return FR_ERR_ARG;
  if (rule == FR_MFD) {
    if (counts_out) return FR_ERR_RULE;
    if (q_dtype == FR_NONE) return FR_ERR_RULE;
    if (!(mfd_p > 0.0) || !isfinite(mfd_p)) return FR_ERR_ARG;
  }
  if (nrows == 0 || ncols == 0) {
    // Empty grid: nothing to route (zero-size buffers may be NULL).
    if (mass_out && launch_zero_f64(mass_out, 2, stream) != hipSuccess) return FR_ERR_HIP;
    return FR_OK;
  }
  if ((q_dtype == FR_NONE) != (q_out == nullptr)) return FR_ERR_ARG;
  if (q_dtype == FR_NONE && !counts_out) return FR_ERR_ARG;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!code || (rule == FR_MFD && !z)) return FR_ERR_ARG;
  {
    // No output may share memory with an input, the workspace or another
    // output: the solvers read inputs after writing outputs (the tile forest
    // keeps per-cell structure in q or counts between its two passes).
    const size_t n = (size_t)(nrows * ncols);
    const void* in[4] = {z, code, rain, ws};
    const size_t in_b[4] = {4 * n, n, rain_dtype == FR_F64 ? 8 * n : 4 * n, ws_bytes};
    const void* out[3] = {q_out, counts_out, mass_out};
    const size_t out_b[3] = {q_dtype == FR_F64 ? 8 * n : 4 * n, 8 * n, 16};
    for (int o = 0; o < 3; ++o) {
      for (int i = 0; i < 4; ++i)
        if (overlaps(out[o], out_b[o], in[i], in_b[i])) return FR_ERR_ARG;
      for (int o2 = o + 1; o2 < 3; ++o2)
        if (overlaps(out[o], out_b[o], out[o2], out_b[o2])) return FR_ERR_ARG;
    }
  }
  if (!ws || ws_bytes < fr_workspace_bytes(FR_FN_ACCUMULATE, nrows, ncols, rule, q_dtype)) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);
  CallCtl* C = reinterpret_cast<CallCtl*>(base);
  char* body = base + kCtlBytes;
  timing_reset();

  EngineConfig cfg;
  cfg.rk = rule == FR_MFD ? RK_MULTI : RK_SINGLE;
  cfg.dir = DIR_FWD;
  cfg.vk = q_dtype == FR_F32 ? VK_FF : (q_dtype == FR_F64 ? VK_F64 : VK_NONE);
  cfg.counts = counts_out != nullptr;
  const float* r32 = (rain && rain_dtype == FR_F32) ? static_cast<const float*>(rain) : nullptr;
  const double* r64 = (rain && rain_dtype == FR_F64) ? static_cast<const double*>(rain) : nullptr;
  float* q32 = q_dtype == FR_F32 ? static_cast<float*>(q_out) : nullptr;
  double* q64 = q_dtype == FR_F64 ? static_cast<double*>(q_out) : nullptr;
  const Layout L = layout(nrows, ncols, rule, q_dtype);
  EngineParams P = engine_params(nrows, ncols, code, z, mfd_p, body, L, dev_status, &C->fallback);
  P.src32 = r32;
  P.src64 = r64;
  P.vhi = q32;
  P.v64 = q64;
  P.cnt = counts_out;
  double* partial = reinterpret_cast<double*>(body + L.partial);

  // Every kernel below is ordered on the stream; decisions between them
  // (exit overflow, sweep passes, the engine's gate) are taken on the
  // device through the control block, which starts zeroed.
  const bool tiles_only = cfg.rk == RK_SINGLE && g_path == FR_PATH_TILES;
  const int32_t first = g_path == FR_PATH_ENGINE ? FR_SERVED_ENGINE
                        : (tiles_only ? FR_SERVED_TILES
                                      : (cfg.rk == RK_SINGLE && g_path == FR_PATH_AUTO ? FR_SERVED_ROWS
                                                                                       : FR_SERVED_SWEEP));
  if (launch_ctl_init(C, first, stream) != hipSuccess) return FR_ERR_HIP;
  int rc = FR_OK;
  const int64_t n = nrows * ncols;
  bool ms_on = false;
  double* ms_partial = nullptr;
  int32_t ms_nstrips = 0;
  if (g_path == FR_PATH_ENGINE) {
    hipLaunchKernelGGL(k_open_gate, dim3(1), dim3(64), 0, stream, C);
    if (hipGetLastError() != hipSuccess) return FR_ERR_HIP;
  } else if (cfg.rk == RK_SINGLE && (g_path == FR_PATH_AUTO || tiles_only)) {
    rc = enqueue_d8(code, nrows, ncols, rain, rain_dtype, cfg.vk, q32, q64, counts_out, mass_out, dev_status, body,
                    C, tiles_only, stream);
    if (rc != FR_OK) return rc;
    // Neither list can overflow: the row sweeps' holds every cell on grids
    // up to 2^22 cells, the tile forest's every cell on a tile perimeter.
    if (n <= kFullCapacityCells || tiles_only) return FR_OK;
    // Overflow fallback: the engine and its mass reduction, behind the gate.
    if ((rc = enqueue_engine(cfg, P, stream)) != FR_OK) return rc;
    if (mass_out && launch_mass(cfg.rk, cfg.vk, P, partial, kMassBlocks, mass_out, stream) != hipSuccess)
      return FR_ERR_HIP;
    return FR_OK;
  } else {
    const WsLayout WL = ws_layout(nrows, ncols, q_dtype);
    if (ms_applicable(cfg.rk, cfg.vk, ncols)) {
      MsParams M = ms_params(nrows, ncols, code, z, mfd_p, body, WL, dev_status);
      M.src32 = r32;
      M.src64 = r64;
      M.vhi = q32;
      M.v64 = q64;
      ms_on = true;
      ms_partial = M.partial;
      ms_nstrips = M.nstrips;
      const int ph = phase_begin("row_sweep", stream);
      if (launch_ms(cfg.vk, false, M, C, stream) != hipSuccess) return FR_ERR_HIP;
      phase_end(ph, stream);
    }
    WsParams W = ws_params(nrows, ncols, code, z, mfd_p, body, WL, cfg.vk, dev_status);
    W.src32 = r32;
    W.src64 = r64;
    W.vhi = q32;
    W.v64 = q64;
    W.cnt = counts_out;
    if ((rc = enqueue_ws(cfg, W, C, stream)) != FR_OK) return rc;
  }
  if ((rc = enqueue_engine(cfg, P, stream)) != FR_OK) return rc;
  if (mass_out) {
    // After the sweep or the engine, whichever finished the solve: both keep
    // the float-float low part at the same place.  When the row sweep served
    // the call, its own partials are summed instead.
    EngineParams M = P;
    M.gate = ms_on ? &C->ms_skip : nullptr;
    const int ph = phase_begin("mass", stream);
    if (launch_mass(cfg.rk, cfg.vk, M, partial, kMassBlocks, mass_out, stream) != hipSuccess) return FR_ERR_HIP;
    if (ms_on && launch_mass_final(ms_partial, ms_nstrips, mass_out, &C->ms_skip, stream) != hipSuccess)
      return FR_ERR_HIP;
    phase_end(ph, stream);
  }
  return FR_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int scratch_address(void** out) {
  constexpr int kMaxDevices = 64;
  static void* addr[kMaxDevices];
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FR_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FR_ERR_HIP;
    addr[dev] = p;
  }
  *out = addr[dev];
  return FR_OK;
}

int fr_accumulate_noalloc(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                          double mfd_p, const void* rain, int rain_dtype, int q_dtype, void* q_out,
                          uint64_t* counts_out, double* mass_out, int32_t* dev_status, hipStream_t stream) {
  // The array holds a workspace of this many bytes at its first 256-byte
  // boundary (it is 256-byte aligned itself).
  const size_t need = fr_workspace_bytes(FR_FN_ACCUMULATE, nrows, ncols, rule, q_dtype);
  if (need > FR_NOALLOC_SCRATCH_BYTES) return FR_ERR_TOOLARGE;
  void* ws = nullptr;
  // Empty grids and invalid arguments need no scratch: fr_accumulate
  // answers them as usual.
  if (need > 0 && nrows > 0 && ncols > 0) {
    const int rc = scratch_address(&ws);
    if (rc != FR_OK) return rc;
  }
  return fr_accumulate(z, code, nrows, ncols, rule, mfd_p, rain, rain_dtype, q_dtype, q_out, counts_out, mass_out,
                       dev_status, ws, ws ? FR_NOALLOC_SCRATCH_BYTES : 0, stream);
}

int fr_accumulate_block_iterations(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                                   double mfd_p, int64_t block_rows, int64_t block_cols, int scheme,
                                   const void* rain, int rain_dtype, int q_dtype, void* q_out,
                                   uint64_t* counts_out, int32_t max_iter, int32_t* iters_out,
                                   int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  (void)z;
  (void)mfd_p;
  if (nrows < 0 || ncols < 0 || !iters_out || max_iter < 1 || block_rows < 1 || block_cols < 1) return FR_ERR_ARG;
  if (rule != FR_D8 && rule != FR_D4) return FR_ERR_RULE;
  if (scheme != FR_SCHEME_IX && scheme != FR_SCHEME_IMX_IX) return FR_ERR_ARG;
  if (rain && rain_dtype != FR_F32 && rain_dtype != FR_F64) return FR_ERR_ARG;
  if (q_dtype != FR_NONE && q_dtype != FR_F64) return FR_ERR_ARG;
  *iters_out = 0;
  if (nrows == 0 || ncols == 0) return FR_OK;
  if ((q_dtype == FR_NONE) != (q_out == nullptr)) return FR_ERR_ARG;
  // Convergence is decided on the exact counts for (I-X)(I+X), whose float
  // iterate keeps moving in its last bits.
  if (!counts_out && (q_dtype == FR_NONE || scheme == FR_SCHEME_IMX_IX)) return FR_ERR_ARG;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!code) return FR_ERR_ARG;
  // Blocks are unions of row-sweep tiles: block_cols a multiple of 256 (or
  // the whole width), block_rows a multiple of 16 (or the whole height); the
  // tile height is the largest power of two up to 512 dividing block_rows.
  int th = 512;
  int64_t bt_r = 0, bt_c = 0;
  if (block_rows >= nrows) {
    th = d8_tile_height(nrows, ncols);
    bt_r = (nrows + th - 1) / th;
  } else {
    if (block_rows % 16 != 0) return FR_ERR_ARG;
    while (block_rows % th != 0) th /= 2;
    bt_r = block_rows / th;
  }
  if (block_cols >= ncols) {
    bt_c = (ncols + D8_TW - 1) / D8_TW;
  } else {
    if (block_cols % D8_TW != 0) return FR_ERR_ARG;
    bt_c = block_cols / D8_TW;
  }
  const int fn = scheme == FR_SCHEME_IX ? FR_FN_BLOCK_ITER : FR_FN_BLOCK_ITER_PRE;
  if (!ws || ws_bytes < fr_workspace_bytes(fn, nrows, ncols, rule, q_dtype)) return FR_ERR_WORKSPACE;
  timing_reset();
  char* base = aligned_base(ws);
  CallCtl* C = reinterpret_cast<CallCtl*>(base);
  char* body = base + kCtlBytes;
  const ValKind vk = q_dtype == FR_F64 ? VK_F64 : VK_NONE;
  const bool counts = counts_out != nullptr;
  D8Layout DL{};
  D8Params P = d8_params(code, nrows, ncols, th, rain, rain_dtype, vk, counts, body, C, dev_status, &DL);
  P.bt_r = (int32_t)bt_r;
  P.bt_c = (int32_t)bt_c;
  char* vecs = body + d8_layout(nrows, ncols, 16, q_dtype, true).total;
  const size_t n = (size_t)(nrows * ncols);
  const size_t vb = up(n * sizeof(double)) + up(n * sizeof(uint64_t));
  const int nvec = scheme == FR_SCHEME_IX ? 1 : 3;
  auto vq = [&](int v) { return vk == VK_F64 ? reinterpret_cast<double*>(vecs + v * vb) : nullptr; };
  auto vc = [&](int v) {
    return counts ? reinterpret_cast<uint64_t*>(vecs + v * vb + up(n * sizeof(double))) : nullptr;
  };
  int32_t* flag = reinterpret_cast<int32_t*>(vecs + nvec * vb);
  // The two iterates alternate between the caller's outputs (even
  // iterations) and workspace vector 0 (odd ones); once an iterate equals
  // the previous one both hold the solution.
  double* qbuf[2] = {static_cast<double*>(q_out), vq(0)};
  uint64_t* cbuf[2] = {counts_out, vc(0)};
  // One block solve into (oq, oc): D^-1 (src + R prev) -- src is the rain
  // (unit counts) unless nosrc; prev NULL means no water across block
  // boundaries.  Phases A, B and C with the forest cut at block boundaries.
  auto solve = [&](const double* pq, const uint64_t* pc, bool nosrc, bool detect, double* oq,
                   uint64_t* oc) -> bool {
    P.q64 = oq;
    P.cnt = oc;
    P.it_q64 = pq;
    P.it_cnt = pc;
    P.it_first = (pq == nullptr && pc == nullptr) ? 1 : 0;
    P.it_nosrc = nosrc ? 1 : 0;
    P.it_detect = detect ? 1 : 0;
    P.it_changed = flag;
    return launch_zero_u32(reinterpret_cast<uint32_t*>(C), CTL_WORDS, stream) == hipSuccess &&
           launch_zero_u32(P.n_exits, 16, stream) == hipSuccess &&
           launch_d8_up(vk, counts, true, P, stream) == hipSuccess &&
           launch_d8_forest(vk, counts, true, P, stream) == hipSuccess &&
           launch_d8_down(vk, counts, true, P, stream) == hipSuccess;
  };
  const int ph = phase_begin("block_iterations", stream);
  int rc = FR_OK;
  if (scheme == FR_SCHEME_IMX_IX) {
    // b = D^-1 r (vector 1); the iterate starts at 0 in the slot the first
    // iteration reads.
    if (!solve(nullptr, nullptr, false, false, vq(1), vc(1)) ||
        launch_bi_combine(2, (int64_t)n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, qbuf[0], cbuf[0],
                          nullptr, stream) != hipSuccess)
      rc = FR_ERR_HIP;
  }
  for (int32_t l = 1; rc == FR_OK; ++l) {
    if (l > max_iter + 1) {
      // No fixed point within the budget: a cycle in the codes, or too few
      // iterations allowed for the block crossings of this grid.
      if (dev_status && launch_set_status(dev_status, FR_ERR_NOTDAG, stream) != hipSuccess) rc = FR_ERR_HIP;
      break;
    }
    const int cur = l & 1, prev = cur ^ 1;
    bool ok = launch_zero_u32(reinterpret_cast<uint32_t*>(flag), 1, stream) == hipSuccess;
    if (scheme == FR_SCHEME_IX) {
      // w <- D^-1 (r + R w); the first iteration has no previous iterate.
      ok = ok && (l == 1 ? solve(nullptr, nullptr, false, false, qbuf[cur], cbuf[cur])
                         : solve(qbuf[prev], cbuf[prev], false, true, qbuf[cur], cbuf[cur]));
    } else {
      // res = b - (I + X) w = b - w + D^-1 R w   (vector 2)
      // w  <- w + (I - X) res = w + res + D^-1 R res
      double* w_q = qbuf[prev];
      uint64_t* w_c = cbuf[prev];
      ok = ok && solve(w_q, w_c, true, false, vq(2), vc(2)) &&
           launch_bi_combine(0, (int64_t)n, vq(1), vc(1), w_q, w_c, vq(2), vc(2), nullptr, nullptr, nullptr,
                             stream) == hipSuccess &&
           solve(vq(2), vc(2), true, false, qbuf[cur], cbuf[cur]) &&
           launch_bi_combine(1, (int64_t)n, nullptr, nullptr, w_q, w_c, vq(2), vc(2), qbuf[cur], cbuf[cur], flag,
                             stream) == hipSuccess;
    }
    if (!ok) {
      rc = FR_ERR_HIP;
      break;
    }
    // The convergence test needs the flag on the host: one read-back per
    // iteration (this entry point measures the paper's scheme; the
    // production solve is fr_accumulate).
    int32_t changed = 0, st = 0;
    if (hipMemcpyAsync(&changed, flag, sizeof changed, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (dev_status && hipMemcpyAsync(&st, dev_status, sizeof st, hipMemcpyDeviceToHost, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
      rc = FR_ERR_HIP;
      break;
    }
    if (st != 0) break;
    if (l > 1 && !changed) {
      *iters_out = l - 1;
      break;
    }
  }
  phase_end(ph, stream);
  return rc;
}

int fr_accumulate_adjoint(const float* z, const uint8_t* code, int64_t nrows, int64_t ncols, int rule,
                          double mfd_p, const void* qbar, int dtype, void* rbar_out, int32_t* dev_status,
                          void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nrows < 0 || ncols < 0) return FR_ERR_ARG;
  if (!valid_rule(rule)) return FR_ERR_RULE;
  if (dtype != FR_F32 && dtype != FR_F64) return FR_ERR_ARG;
  if (rule == FR_MFD && (!(mfd_p > 0.0) || !isfinite(mfd_p))) return FR_ERR_ARG;
  if (nrows == 0 || ncols == 0) return FR_OK;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!code || !qbar || !rbar_out || (rule == FR_MFD && !z)) return FR_ERR_ARG;
  if (!ws || ws_bytes < fr_workspace_bytes(FR_FN_ADJOINT, nrows, ncols, rule, dtype)) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);
  CallCtl* C = reinterpret_cast<CallCtl*>(base);
  char* body = base + kCtlBytes;
  timing_reset();

  EngineConfig cfg;
  cfg.rk = rule == FR_MFD ? RK_MULTI : RK_SINGLE;
  cfg.dir = DIR_ADJ;
  cfg.vk = dtype == FR_F32 ? VK_FF : VK_F64;
  cfg.counts = false;
  const float* s32 = dtype == FR_F32 ? static_cast<const float*>(qbar) : nullptr;
  const double* s64 = dtype == FR_F64 ? static_cast<const double*>(qbar) : nullptr;
  float* o32 = dtype == FR_F32 ? static_cast<float*>(rbar_out) : nullptr;
  double* o64 = dtype == FR_F64 ? static_cast<double*>(rbar_out) : nullptr;
  if (launch_ctl_init(C, g_path == FR_PATH_ENGINE ? FR_SERVED_ENGINE : FR_SERVED_SWEEP, stream) != hipSuccess)
    return FR_ERR_HIP;
  int rc = FR_OK;
  if (g_path == FR_PATH_ENGINE) {
    hipLaunchKernelGGL(k_open_gate, dim3(1), dim3(64), 0, stream, C);
    if (hipGetLastError() != hipSuccess) return FR_ERR_HIP;
  } else {
    const WsLayout WL = ws_layout(nrows, ncols, dtype);
    if (ms_applicable(cfg.rk, cfg.vk, ncols)) {
      MsParams M = ms_params(nrows, ncols, code, z, mfd_p, body, WL, dev_status);
      M.src32 = s32;
      M.src64 = s64;
      M.vhi = o32;
      M.v64 = o64;
      M.partial = nullptr;
      const int ph = phase_begin("row_sweep", stream);
      if (launch_ms(cfg.vk, true, M, C, stream) != hipSuccess) return FR_ERR_HIP;
      phase_end(ph, stream);
    }
    WsParams W = ws_params(nrows, ncols, code, z, mfd_p, body, WL, cfg.vk, dev_status);
    W.src32 = s32;
    W.src64 = s64;
    W.vhi = o32;
    W.v64 = o64;
    if ((rc = enqueue_ws(cfg, W, C, stream)) != FR_OK) return rc;
  }
  const Layout L = layout(nrows, ncols, rule, dtype);
  EngineParams P = engine_params(nrows, ncols, code, z, mfd_p, body, L, dev_status, &C->fallback);
  P.src32 = s32;
  P.src64 = s64;
  P.vhi = o32;
  P.v64 = o64;
  P.cnt = nullptr;
  return enqueue_engine(cfg, P, stream);
}

size_t fr_batched_workspace_bytes(const fr_tile* tiles_host, int32_t ntiles) {
  if (ntiles < 0 || (ntiles > 0 && !tiles_host)) return 0;
  size_t off = batch_head_bytes(ntiles);
  for (int32_t i = 0; i < ntiles; ++i) {
    const fr_tile& t = tiles_host[i];
    if (t.nrows < 1 || t.ncols < 1 || !valid_rule(t.rule)) return 0;
    if (t.ncols > kMaxCells / t.nrows) return 0;
    if (t.rule == FR_MFD && !t.q_out) return 0;
    if (t.rule != FR_MFD && (t.q_out != nullptr) == (t.counts_out != nullptr)) return 0;
    const BatchTileLayout L =
        batch_tile_layout(t.nrows, t.ncols, t.code_out == nullptr, batch_tile_ff(t.rule, t.q_out != nullptr));
    off += L.total;
  }
  return off + kAlign;
}

int fr_accumulate_batched(const fr_tile* tiles_dev, int32_t ntiles, const fr_batch_plan* plan,
                          int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (ntiles < 0) return FR_ERR_ARG;
  timing_reset();
  if (ntiles == 0) return FR_OK;
  if (!tiles_dev) return FR_ERR_ARG;
  if (plan && (plan->workers < 0 || (plan->order != FR_ORDER_GIVEN && plan->order != FR_ORDER_ROWS_DESC &&
                                     plan->order != FR_ORDER_CELLS_DESC)))
    return FR_ERR_ARG;
  if (!ws || ws_bytes < batch_head_bytes(ntiles) + kAlign) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);
  const size_t avail = ws_bytes - (size_t)(base - static_cast<char*>(ws));
  const int workers = (plan && plan->workers > 0) ? plan->workers : 2 * cu_count();
  const int order = plan ? plan->order : FR_ORDER_ROWS_DESC;
  const int ph = phase_begin("batch", stream);
  const hipError_t e = launch_batch(tiles_dev, ntiles, order, workers, dev_status, base, avail, stream);
  phase_end(ph, stream);
  return e == hipSuccess ? FR_OK : FR_ERR_HIP;
}

// Autotune cache: batch signature -> plan, in the process and optionally in
// a file (fr_set_autotune_cache).
static std::map<uint64_t, fr_batch_plan> g_plans;
static std::string g_plan_file;

static void fnv(uint64_t& h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xFFu;
    h *= 0x100000001b3ull;
  }
}

int fr_set_autotune_cache(const char* path) {
  g_plan_file = path ? path : "";
  if (!path) return FR_OK;
  FILE* f = fopen(path, "a+");
  if (!f) return FR_ERR_ARG;
  rewind(f);
  unsigned long long sig = 0;
  int w = 0, o = 0;
  while (fscanf(f, "%llx %d %d", &sig, &w, &o) == 3)
    if (w > 0 && (o == FR_ORDER_GIVEN || o == FR_ORDER_ROWS_DESC || o == FR_ORDER_CELLS_DESC))
      g_plans[(uint64_t)sig] = fr_batch_plan{w, o};
  fclose(f);
  return FR_OK;
}

int fr_batch_autotune(const fr_tile* tiles_dev, int32_t ntiles, int32_t* dev_status, void* ws, size_t ws_bytes,
                      int reps, fr_batch_plan* plan_out, hipStream_t stream) {
  if (!plan_out || reps < 1 || ntiles < 0 || (ntiles > 0 && !tiles_dev)) return FR_ERR_ARG;
  const int cu = cu_count();
  // Signature of the batch (its tile table, read back from the device).
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FR_ERR_HIP;
  std::vector<fr_tile> host((size_t)ntiles);
  if (ntiles > 0 && (hipMemcpyAsync(host.data(), tiles_dev, sizeof(fr_tile) * (size_t)ntiles,
                                    hipMemcpyDeviceToHost, stream) != hipSuccess ||
                     hipStreamSynchronize(stream) != hipSuccess))
    return FR_ERR_HIP;
  uint64_t sig = 0xcbf29ce484222325ull;
  fnv(sig, (uint64_t)dev);
  fnv(sig, (uint64_t)cu);
  fnv(sig, (uint64_t)ntiles);
  for (const fr_tile& t : host) {
    fnv(sig, (uint64_t)t.nrows);
    fnv(sig, (uint64_t)t.ncols);
    fnv(sig, ((uint64_t)t.rule << 8) | ((t.rain != nullptr) << 0) | ((t.q_out != nullptr) << 1) |
                 ((t.counts_out != nullptr) << 2) | ((t.code_out != nullptr) << 3));
  }
  const auto hit = g_plans.find(sig);
  if (hit != g_plans.end()) {
    *plan_out = hit->second;
    return FR_OK;
  }
  std::vector<fr_batch_plan> cand;
  for (int w : {2 * cu, cu + cu / 2, cu})
    for (int o : {FR_ORDER_ROWS_DESC, FR_ORDER_CELLS_DESC, FR_ORDER_GIVEN}) cand.push_back(fr_batch_plan{w, o});
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FR_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FR_ERR_HIP;
  }
  float best = -1.0f;
  int rc = FR_OK;
  for (const fr_batch_plan& p : cand) {
    rc = fr_accumulate_batched(tiles_dev, ntiles, &p, dev_status, ws, ws_bytes, stream);
    if (rc != FR_OK) break;
    if (hipEventRecord(e0, stream) != hipSuccess) { rc = FR_ERR_HIP; break; }
    for (int r = 0; r < reps && rc == FR_OK; ++r)
      rc = fr_accumulate_batched(tiles_dev, ntiles, &p, dev_status, ws, ws_bytes, stream);
    if (rc != FR_OK) break;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = FR_ERR_HIP;
      break;
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = FR_ERR_HIP; break; }
    if (best < 0.0f || ms < best) {
      best = ms;
      *plan_out = p;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == FR_OK && best >= 0.0f) {
    g_plans[sig] = *plan_out;
    if (!g_plan_file.empty()) {
      FILE* f = fopen(g_plan_file.c_str(), "a");
      if (f) {
        fprintf(f, "%llx %d %d\n", (unsigned long long)sig, plan_out->workers, plan_out->order);
        fclose(f);
      }
    }
  }
  return rc;
}

}  // extern "C"
