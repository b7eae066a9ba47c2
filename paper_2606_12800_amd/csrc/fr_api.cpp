// Host side of the C ABI declared in fr_api.h: argument validation,
// workspace carving, kernel enqueue and the iteration driver.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fr_internal.hpp"

namespace fr {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMassBlocks = 1024;
constexpr int64_t kMaxCells = 2147483647;  // cell indices fit in int32

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t ext, done, vlo, rs32, iw32, iw64, stamp, list0, list1, ctr, partial, total;
};

int64_t tiles_of(int64_t nrows, int64_t ncols) {
  return ((nrows + ENG_TH - 1) / ENG_TH) * ((ncols + ENG_TW - 1) / ENG_TW);
}

// Offsets relative to the first 256-byte aligned address inside ws; the
// total includes kAlign bytes of slack for that alignment.
Layout layout(int64_t nrows, int64_t ncols, int rule, int vdtype) {
  Layout L{};
  const size_t n = (size_t)(nrows * ncols);
  const size_t nt = (size_t)tiles_of(nrows, ncols);
  size_t o = 0;
  L.ext = o; o += up(n + 4);
  L.done = o; o += up(n + 4);
  L.vlo = o; if (vdtype == FR_F32) o += up(n * sizeof(float));
  L.rs32 = o; if (rule == FR_MFD && vdtype == FR_F32) o += up(n * sizeof(float));
  L.iw32 = o; if (rule == FR_MFD && vdtype == FR_F32) o += up(n * sizeof(float));
  L.iw64 = o; if (rule == FR_MFD && vdtype == FR_F64) o += up(n * sizeof(double));
  L.stamp = o; o += up(nt * sizeof(int32_t));
  L.list0 = o; o += up(nt * sizeof(int32_t));
  L.list1 = o; o += up(nt * sizeof(int32_t));
  L.ctr = o; o += kAlign;
  L.partial = o; o += up(2 * kMassBlocks * sizeof(double));
  L.total = o + kAlign;
  return L;
}

// Workspace of the row-sweep single-receiver path (fr_d8.hip).  It shares
// the workspace with the engine: the engine only runs when this path gives up
// (exit list overflow), after which this path's data is dead.
struct D8Layout {
  size_t root_of, node_of, ex_cell, anc0, anc1, cnt0, cnt1, hi0, hi1, lo0, lo1, q0, q1, ctr, mass, total;
  uint32_t cap;
};

uint32_t d8_capacity(int64_t n) {
  if (n <= ((int64_t)1 << 22)) return (uint32_t)(n > 0 ? n : 1);
  const int64_t c = n / 8;
  return (uint32_t)(c > ((int64_t)1 << 22) ? c : ((int64_t)1 << 22));
}

D8Layout d8_layout(int64_t nrows, int64_t ncols, int vdtype, bool counts) {
  D8Layout L{};
  const size_t n = (size_t)(nrows * ncols);
  const int th = d8_tile_height(nrows, ncols);
  const size_t nt = (size_t)(((nrows + th - 1) / th) * ((ncols + D8_TW - 1) / D8_TW));
  L.cap = d8_capacity((int64_t)n);
  const size_t cap = L.cap;
  size_t o = 0;
  L.root_of = o; o += up(n * 4);
  L.node_of = o; o += up(n * 4);
  L.ex_cell = o; o += up(cap * 4);
  L.anc0 = o; o += up(cap * 4);
  L.anc1 = o; o += up(cap * 4);
  L.cnt0 = o; if (counts) o += up(cap * 8);
  L.cnt1 = o; if (counts) o += up(cap * 8);
  L.hi0 = o; if (vdtype == FR_F32) o += up(cap * 4);
  L.hi1 = o; if (vdtype == FR_F32) o += up(cap * 4);
  L.lo0 = o; if (vdtype == FR_F32) o += up(cap * 4);
  L.lo1 = o; if (vdtype == FR_F32) o += up(cap * 4);
  L.q0 = o; if (vdtype == FR_F64) o += up(cap * 8);
  L.q1 = o; if (vdtype == FR_F64) o += up(cap * 8);
  L.ctr = o; o += kAlign;
  L.mass = o; o += up(nt * 2 * sizeof(double));
  L.total = o + kAlign;
  return L;
}

// Workspace of the wavefront sweep (fr_wsweep.hip).  Like the row-sweep
// path it overlays the engine's workspace; the engine only runs after the
// sweep gave up.
struct WsLayout {
  size_t vlo, edge, progress, ctr, partial, total;
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
  L.total = o + kAlign;
  return L;
}

struct Counters {
  int32_t nlist[3];
  int32_t pad;
  unsigned long long remaining;
};

bool valid_rule(int rule) { return rule == FR_D8 || rule == FR_D4 || rule == FR_MFD; }

int cu_count() {
  static int cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
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

int run_engine_body(const EngineConfig& cfg, EngineParams P, char* base, const Layout& L, int32_t* status,
                    hipStream_t s);

// Runs the peeling engine to completion (see fr_engine.hip).
int run_engine(const EngineConfig& cfg, EngineParams P, char* base, const Layout& L, int32_t* status,
               hipStream_t s) {
  const int ph = phase_begin("engine", s);
  const int rc = run_engine_body(cfg, P, base, L, status, s);
  phase_end(ph, s);
  return rc;
}

int run_engine_body(const EngineConfig& cfg, EngineParams P, char* base, const Layout& L, int32_t* status,
                    hipStream_t s) {
  if (launch_engine_init(cfg, P, s) != hipSuccess) return FR_ERR_HIP;
  const int64_t ntiles = (int64_t)P.ntr * P.ntc;
  int grid = 2 * cu_count();
  if ((int64_t)grid > ntiles) grid = (int)ntiles;
  Counters* dctr = reinterpret_cast<Counters*>(base + L.ctr);
  int it = 0;
  int batch = 4;
  const int max_it = 1 << 30;
  for (;;) {
    for (int b = 0; b < batch; ++b, ++it)
      if (launch_engine_iter(cfg, P, it, grid, s) != hipSuccess) return FR_ERR_HIP;
    Counters h{};
    if (hipMemcpyAsync(&h, dctr, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) return FR_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FR_ERR_HIP;
    if (h.remaining == 0) break;
    if (h.nlist[it % 3] == 0 || it >= max_it) {
      // Nothing queued but cells unfinished: the routing graph has a cycle.
      if (status && launch_set_status(status, FR_ERR_NOTDAG, s) != hipSuccess) return FR_ERR_HIP;
      break;
    }
    if (batch < 64) batch *= 2;
  }
  return FR_OK;
}

// Row-sweep path for single-receiver codes, forward solve.  Returns FR_OK,
// an error, or 1 when the exit list overflowed (the caller then runs the
// engine).
int run_d8(const uint8_t* code, int64_t nrows, int64_t ncols, const float* rain32, const double* rain64,
           ValKind vk, float* q32, double* q64, uint64_t* cnt, double* mass_out, int32_t* status, char* base,
           hipStream_t s) {
  const bool counts = cnt != nullptr;
  const D8Layout L = d8_layout(nrows, ncols, vk == VK_FF ? FR_F32 : (vk == VK_F64 ? FR_F64 : FR_NONE), counts);
  D8Params P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.th = d8_tile_height(nrows, ncols);
  P.ntr = (int32_t)((nrows + P.th - 1) / P.th);
  P.ntc = (int32_t)((ncols + D8_TW - 1) / D8_TW);
  P.code = code;
  P.rain32 = rain32;
  P.rain64 = rain64;
  P.q32 = q32;
  P.q64 = q64;
  P.cnt = cnt;
  P.root_of = reinterpret_cast<uint32_t*>(base + L.root_of);
  P.node_of = reinterpret_cast<uint32_t*>(base + L.node_of);
  P.ex_cell = reinterpret_cast<uint32_t*>(base + L.ex_cell);
  P.anc[0] = reinterpret_cast<uint32_t*>(base + L.anc0);
  P.anc[1] = reinterpret_cast<uint32_t*>(base + L.anc1);
  P.ex_cnt[0] = reinterpret_cast<uint64_t*>(base + L.cnt0);
  P.ex_cnt[1] = reinterpret_cast<uint64_t*>(base + L.cnt1);
  P.ex_hi[0] = reinterpret_cast<float*>(base + L.hi0);
  P.ex_hi[1] = reinterpret_cast<float*>(base + L.hi1);
  P.ex_lo[0] = reinterpret_cast<float*>(base + L.lo0);
  P.ex_lo[1] = reinterpret_cast<float*>(base + L.lo1);
  P.ex_q64[0] = reinterpret_cast<double*>(base + L.q0);
  P.ex_q64[1] = reinterpret_cast<double*>(base + L.q1);
  uint32_t* ctr = reinterpret_cast<uint32_t*>(base + L.ctr);
  P.n_exits = ctr;
  P.flags = reinterpret_cast<int32_t*>(ctr + 4);
  P.cap = L.cap;
  P.mass_part = mass_out ? reinterpret_cast<double*>(base + L.mass) : nullptr;
  P.status = status;

  if (launch_zero_u32(ctr, 16, s) != hipSuccess) return FR_ERR_HIP;
  int ph = phase_begin("d8_up", s);
  if (launch_d8_up(vk, counts, P, s) != hipSuccess) return FR_ERR_HIP;
  phase_end(ph, s);
  uint32_t n = 0;
  if (hipMemcpyAsync(&n, ctr, sizeof n, hipMemcpyDeviceToHost, s) != hipSuccess) return FR_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FR_ERR_HIP;
  if (n > L.cap) return 1;
  P.n_ex = n;
  int round = 0;
  ph = phase_begin("d8_forest", s);
  if (n > 0) {
    if (launch_d8_link(P, n, s) != hipSuccess) return FR_ERR_HIP;
    // A forest of n nodes is at most n deep: 33 rounds always suffice; more
    // means the exits form a cycle (malformed codes).  Rounds go out four
    // at a time (a round after the last one with work returns at once);
    // the host then reads the flag of the last round queued.
    constexpr int kRoundBatch = 4;
    for (;;) {
      for (int q = 0; q < kRoundBatch; ++q, ++round)
        if (launch_d8_round(vk, counts, P, n, round, s) != hipSuccess) return FR_ERR_HIP;
      int32_t flag = 0;
      if (hipMemcpyAsync(&flag, P.flags + 4 + (round - 1) % 3, sizeof flag, hipMemcpyDeviceToHost, s) !=
          hipSuccess)
        return FR_ERR_HIP;
      if (hipStreamSynchronize(s) != hipSuccess) return FR_ERR_HIP;
      if (!flag) break;
      if (round > 33) {
        if (status && launch_set_status(status, FR_ERR_NOTDAG, s) != hipSuccess) return FR_ERR_HIP;
        break;
      }
    }
  }
  phase_end(ph, s);
  ph = phase_begin("d8_down", s);
  if (launch_d8_down(vk, counts, P, s) != hipSuccess) return FR_ERR_HIP;
  phase_end(ph, s);
  if (mass_out) {
    const int nt = P.ntr * P.ntc;
    ph = phase_begin("mass", s);
    if (launch_mass_final(P.mass_part, nt, mass_out, s) != hipSuccess) return FR_ERR_HIP;
    phase_end(ph, s);
  }
  return FR_OK;
}

// Accumulation path: "auto" (row sweeps for D8/D4 forward, the wavefront
// sweep otherwise), "sweep" (the wavefront sweep for everything) or
// "engine" (the peeling engine for everything), from FLOWROUTE_ACC.
enum AccPath { ACC_AUTO, ACC_SWEEP, ACC_ENGINE };
AccPath acc_path() {
  const char* e = getenv("FLOWROUTE_ACC");
  if (e && strcmp(e, "engine") == 0) return ACC_ENGINE;
  if (e && strcmp(e, "sweep") == 0) return ACC_SWEEP;
  return ACC_AUTO;
}

constexpr int kMaxSweepPasses = 32;

// Diagnostics on stderr when FLOWROUTE_VERBOSE is set.
bool verbose() {
  static const bool v = getenv("FLOWROUTE_VERBOSE") != nullptr;
  return v;
}

// Wavefront-sweep passes until every cell is final.  Returns FR_OK, an
// error, or 1 when the pass budget ran out (the caller then runs the
// engine from scratch).
int run_ws(const EngineConfig& cfg, WsParams P, int32_t* status, hipStream_t s) {
  if (launch_ws_setup(cfg, P, s) != hipSuccess) return FR_ERR_HIP;
  uint32_t h[4] = {0, 0, 0, 0};
  if (hipMemcpyAsync(h, P.ctr, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) return FR_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FR_ERR_HIP;
  // Visit the rows holding most inputs first: forward inputs are donors,
  // upstream of their receivers; adjoint inputs are the receivers.
  const bool flows_up = h[1] >= h[2];
  int dir = ((cfg.dir == DIR_FWD) == flows_up) ? -1 : 1;
  int64_t remaining = P.nrows * P.ncols;
  uint32_t last_fin[2] = {0, 0};  // cells finished by the last pass going up (dir -1) / down (dir +1)
  // FLOWROUTE_WS_MAXPASS (diagnostics): stop after that many passes and
  // leave unfinished cells as they are.
  const char* mp = getenv("FLOWROUTE_WS_MAXPASS");
  const int max_pass = mp ? atoi(mp) : -1;
  for (int pass = 0;; ++pass) {
    if (max_pass >= 0 && pass >= max_pass) return FR_OK;
    if (pass >= kMaxSweepPasses) return 1;
    if (launch_zero_u32(P.ctr, 1, s) != hipSuccess) return FR_ERR_HIP;
    if (P.debug && launch_zero_u32(P.ctr + 3, 25, s) != hipSuccess) return FR_ERR_HIP;
    if (launch_ws_progress_reset(P, s) != hipSuccess) return FR_ERR_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (verbose() && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
      (void)hipEventRecord(e0, s);
    if (launch_ws_pass(cfg, P, dir, pass == 0 ? 1 : 0, s) != hipSuccess) return FR_ERR_HIP;
    if (e1) (void)hipEventRecord(e1, s);
    uint32_t fin = 0;
    int32_t st = 0;
    if (hipMemcpyAsync(&fin, P.ctr, sizeof fin, hipMemcpyDeviceToHost, s) != hipSuccess) return FR_ERR_HIP;
    if (status && hipMemcpyAsync(&st, status, sizeof st, hipMemcpyDeviceToHost, s) != hipSuccess)
      return FR_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FR_ERR_HIP;
    remaining -= fin;
    if (verbose()) {
      float ms = 0.0f;
      if (e1) (void)hipEventElapsedTime(&ms, e0, e1);
      uint32_t d[28] = {0};
      if (P.debug && hipMemcpy(d, P.ctr, sizeof d, hipMemcpyDeviceToHost) != hipSuccess) return FR_ERR_HIP;
      fprintf(stderr,
              "flowroute: sweep pass %d dir %+d finished %u remaining %lld (%.3f ms) edge-waits %u pace-spins %u "
              "resolves %u row-iterations %u\n",
              pass, dir, fin, (long long)remaining, ms, d[3], d[4], d[5], d[6]);
      if (P.debug) {
        const uint64_t* tm = reinterpret_cast<const uint64_t*>(d + 8);
        const double steps = (double)P.nrows * (double)ws_strips(P.ncols);
        fprintf(stderr,
                "flowroute:   per strip-step (us): wait-staged %.3f pace %.3f settle %.3f (resolve %.3f, row loop %.3f) freeze %.3f "
                "all %.3f | io stage %.3f poll %.3f iterations/step %.2f\n",
                tm[0] / steps / 100.0, tm[1] / steps / 100.0, tm[2] / steps / 100.0, tm[8] / steps / 100.0, tm[9] / steps / 100.0,
                tm[3] / steps / 100.0, tm[4] / steps / 100.0, tm[5] / steps / 100.0, tm[6] / steps / 100.0,
                tm[7] / steps);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (remaining <= 0 || st != 0) break;
    if (fin == 0) {
      // A pass finishes at least the highest unfinished cell of a DAG.
      if (status && launch_set_status(status, FR_ERR_NOTDAG, s) != hipSuccess) return FR_ERR_HIP;
      break;
    }
    // Either direction finishes the highest unfinished cell, so the next
    // pass may go either way: after one pass each way, repeat the direction
    // whose last pass finished more (terrain that drains mostly one way
    // leaves cells that the reverse sweep barely touches).
    last_fin[dir > 0] = fin;
    if (pass == 0 || last_fin[0] == last_fin[1]) dir = -dir;
    else dir = last_fin[1] > last_fin[0] ? 1 : -1;
  }
  return FR_OK;
}

WsParams ws_params(const EngineConfig& cfg, int64_t nrows, int64_t ncols, const uint8_t* code, const float* z,
                   double p, char* base, const WsLayout& L, int32_t* status) {
  WsParams P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.code = code;
  P.z = z;
  P.p = p;
  P.vlo = cfg.vk == VK_FF ? reinterpret_cast<float*>(base + L.vlo) : nullptr;
  P.edge = reinterpret_cast<uint64_t*>(base + L.edge);
  P.progress = reinterpret_cast<int32_t*>(base + L.progress);
  P.ctr = reinterpret_cast<uint32_t*>(base + L.ctr);
  P.status = status;
  P.debug = getenv("FLOWROUTE_WS_DEBUG") != nullptr;
  return P;
}

char* aligned_base(void* ws) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<char*>((a + kAlign - 1) / kAlign * kAlign);
}

EngineParams common_params(int64_t nrows, int64_t ncols, const uint8_t* code, const float* z, double p,
                           char* base, const Layout& L, int32_t* status) {
  EngineParams P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.ntr = (int32_t)((nrows + ENG_TH - 1) / ENG_TH);
  P.ntc = (int32_t)((ncols + ENG_TW - 1) / ENG_TW);
  P.code = code;
  P.z = z;
  P.p = p;
  P.ext = reinterpret_cast<uint8_t*>(base + L.ext);
  P.done = reinterpret_cast<uint8_t*>(base + L.done);
  P.vlo = reinterpret_cast<float*>(base + L.vlo);
  P.rs32 = reinterpret_cast<float*>(base + L.rs32);
  P.iw32 = reinterpret_cast<float*>(base + L.iw32);
  P.iw64 = reinterpret_cast<double*>(base + L.iw64);
  P.stamp = reinterpret_cast<int32_t*>(base + L.stamp);
  P.list0 = reinterpret_cast<int32_t*>(base + L.list0);
  P.list1 = reinterpret_cast<int32_t*>(base + L.list1);
  Counters* c = reinterpret_cast<Counters*>(base + L.ctr);
  P.nlist = c->nlist;
  P.remaining = &c->remaining;
  P.status = status;
  return P;
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

// Block iterations: `vectors` float64 values and counts per cell (I+X: the
// other iterate; (I-X)(I+X): also D^-1 r and a temporary) and the change
// flag.
size_t block_iter_bytes(int64_t nrows, int64_t ncols, int vectors) {
  const size_t n = (size_t)(nrows * ncols);
  return (size_t)vectors * (up(n * sizeof(double)) + up(n * sizeof(uint64_t))) + 2 * kAlign;
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
    return block_iter_bytes(nrows, ncols, fn == FR_FN_BLOCK_ITER_PRE ? 3 : 1);
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
    const size_t t8 = d8_layout(nrows, ncols, dtype, true).total;
    if (t8 > t) t = t8;
  }
  return t;
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
  const Layout L = layout(nrows, ncols, rule, q_dtype);
  if (!ws || ws_bytes < fr_workspace_bytes(FR_FN_ACCUMULATE, nrows, ncols, rule, q_dtype))
    return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);
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
  const AccPath path = acc_path();
  if (cfg.rk == RK_SINGLE && path == ACC_AUTO) {
    const int rc = run_d8(code, nrows, ncols, r32, r64, cfg.vk, q32, q64, counts_out, mass_out, dev_status,
                          base, stream);
    if (rc != 1) return rc;  // 1: exit list overflow, fall back to the wavefront sweep
  }
  EngineParams P = common_params(nrows, ncols, code, z, mfd_p, base, L, dev_status);
  P.src32 = r32;
  P.src64 = r64;
  P.vhi = q32;
  P.v64 = q64;
  P.cnt = counts_out;
  int rc = 1;
  if (path != ACC_ENGINE) {
    const WsLayout WL = ws_layout(nrows, ncols, q_dtype);
    WsParams W = ws_params(cfg, nrows, ncols, code, z, mfd_p, base, WL, dev_status);
    W.src32 = r32;
    W.src64 = r64;
    W.vhi = q32;
    W.v64 = q64;
    W.cnt = counts_out;
    const int ph = phase_begin("sweep", stream);
    rc = run_ws(cfg, W, dev_status, stream);
    phase_end(ph, stream);
    if (rc != FR_OK && rc != 1) return rc;
    if (rc == FR_OK) P.vlo = W.vlo;  // the float-float low parts the mass sum reads
  }
  if (rc == 1) rc = run_engine(cfg, P, base, L, dev_status, stream);
  if (rc != FR_OK) return rc;
  if (mass_out) {
    double* partial = reinterpret_cast<double*>(base + L.partial);
    const int ph = phase_begin("mass", stream);
    if (launch_mass(cfg.rk, cfg.vk, P, partial, kMassBlocks, mass_out, stream) != hipSuccess) return FR_ERR_HIP;
    phase_end(ph, stream);
  }
  return FR_OK;
}

int fr_accumulate_block_iterations(const uint8_t* code, int64_t nrows, int64_t ncols, int rule, int scheme,
                                   const void* rain, int rain_dtype, int q_dtype, void* q_out,
                                   uint64_t* counts_out, int32_t max_iter, int32_t* iters_out,
                                   int32_t* dev_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nrows < 0 || ncols < 0 || !iters_out || max_iter < 1) return FR_ERR_ARG;
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
  const int fn = scheme == FR_SCHEME_IX ? FR_FN_BLOCK_ITER : FR_FN_BLOCK_ITER_PRE;
  if (!ws || ws_bytes < fr_workspace_bytes(fn, nrows, ncols, rule, q_dtype)) return FR_ERR_WORKSPACE;
  timing_reset();
  char* base = aligned_base(ws);
  const size_t n = (size_t)(nrows * ncols);
  const size_t vb = up(n * sizeof(double)) + up(n * sizeof(uint64_t));
  const int nvec = scheme == FR_SCHEME_IX ? 1 : 3;
  const ValKind vk = q_dtype == FR_F64 ? VK_F64 : VK_NONE;
  const bool counts = counts_out != nullptr;
  auto vq = [&](int v) { return vk == VK_F64 ? reinterpret_cast<double*>(base + v * vb) : nullptr; };
  auto vc = [&](int v) {
    return counts ? reinterpret_cast<uint64_t*>(base + v * vb + up(n * sizeof(double))) : nullptr;
  };
  int32_t* flag = reinterpret_cast<int32_t*>(base + nvec * vb);
  D8Params P{};
  P.nrows = nrows;
  P.ncols = ncols;
  P.th = block_iter_height(nrows, ncols);
  P.ntr = (int32_t)((nrows + P.th - 1) / P.th);
  P.ntc = (int32_t)((ncols + D8_TW - 1) / D8_TW);
  P.code = code;
  P.rain32 = (rain && rain_dtype == FR_F32) ? static_cast<const float*>(rain) : nullptr;
  P.rain64 = (rain && rain_dtype == FR_F64) ? static_cast<const double*>(rain) : nullptr;
  P.status = dev_status;
  // The two iterates alternate between the caller's outputs (even
  // iterations) and workspace vector 0 (odd ones); once an iterate equals
  // the previous one both hold the solution.
  double* qbuf[2] = {static_cast<double*>(q_out), vq(0)};
  uint64_t* cbuf[2] = {counts_out, vc(0)};
  // One block solve into (oq, oc): D^-1 (src + R prev) -- src is the rain
  // (unit counts) unless nosrc; prev NULL means no water across cut pairs.
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
    return launch_d8_iter(vk, counts, P, stream) == hipSuccess;
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
  const Layout L = layout(nrows, ncols, rule, dtype);
  if (!ws || ws_bytes < fr_workspace_bytes(FR_FN_ADJOINT, nrows, ncols, rule, dtype)) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);
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
  int rc = 1;
  if (acc_path() != ACC_ENGINE) {
    const WsLayout WL = ws_layout(nrows, ncols, dtype);
    WsParams W = ws_params(cfg, nrows, ncols, code, z, mfd_p, base, WL, dev_status);
    W.src32 = s32;
    W.src64 = s64;
    W.vhi = o32;
    W.v64 = o64;
    const int ph = phase_begin("sweep", stream);
    rc = run_ws(cfg, W, dev_status, stream);
    phase_end(ph, stream);
    if (rc != 1) return rc;
  }
  EngineParams P = common_params(nrows, ncols, code, z, mfd_p, base, L, dev_status);
  P.src32 = s32;
  P.src64 = s64;
  P.vhi = o32;
  P.v64 = o64;
  P.cnt = nullptr;
  return run_engine(cfg, P, base, L, dev_status, stream);
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
  if (plan && (plan->workers < 0 || (plan->order != FR_ORDER_GIVEN && plan->order != FR_ORDER_ROWS_DESC)))
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

int fr_batch_autotune(const fr_tile* tiles_dev, int32_t ntiles, int32_t* dev_status, void* ws, size_t ws_bytes,
                      int reps, fr_batch_plan* plan_out, hipStream_t stream) {
  if (!plan_out || reps < 1) return FR_ERR_ARG;
  const int cu = cu_count();
  const fr_batch_plan cand[] = {{2 * cu, FR_ORDER_ROWS_DESC}, {2 * cu, FR_ORDER_GIVEN}, {cu, FR_ORDER_ROWS_DESC},
                                {cu, FR_ORDER_GIVEN}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FR_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) return FR_ERR_HIP;
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
    if (verbose()) fprintf(stderr, "flowroute: batch plan workers %d order %d: %.3f ms\n", p.workers, p.order, ms / reps);
    if (best < 0.0f || ms < best) {
      best = ms;
      *plan_out = p;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
