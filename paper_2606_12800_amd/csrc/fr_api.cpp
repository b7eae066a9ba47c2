// Host side of the C ABI declared in fr_api.h: argument validation,
// workspace carving, kernel enqueue and the iteration driver.
#include <math.h>
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

// Runs the peeling engine to completion (see fr_engine.hip).
int run_engine(const EngineConfig& cfg, EngineParams P, char* base, const Layout& L, int32_t* status,
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

size_t fr_workspace_bytes(int fn, int64_t nrows, int64_t ncols, int rule, int dtype) {
  if (nrows < 0 || ncols < 0 || !valid_rule(rule)) return 0;
  if (nrows > 0 && ncols > kMaxCells / (nrows > 0 ? nrows : 1)) return 0;
  if (fn == FR_FN_ACCUMULATE) {
    if (dtype != FR_NONE && dtype != FR_F32 && dtype != FR_F64) return 0;
    if (rule == FR_MFD && dtype == FR_NONE) return 0;
  } else if (fn == FR_FN_ADJOINT) {
    if (dtype != FR_F32 && dtype != FR_F64) return 0;
  } else {
    return 0;
  }
  return layout(nrows, ncols, rule, dtype).total;
}

int fr_receivers(const float* z, int64_t nrows, int64_t ncols, int rule, uint8_t* code_out,
                 int32_t* dev_status, hipStream_t stream) {
  if (nrows < 0 || ncols < 0) return FR_ERR_ARG;
  if (!valid_rule(rule)) return FR_ERR_RULE;
  if (nrows == 0 || ncols == 0) return FR_OK;
  if (ncols > kMaxCells / nrows) return FR_ERR_TOOLARGE;
  if (!z || !code_out) return FR_ERR_ARG;
  return launch_receivers(z, nrows, ncols, rule, code_out, dev_status, stream) == hipSuccess ? FR_OK
                                                                                           : FR_ERR_HIP;
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
  if (!ws || ws_bytes < L.total) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);

  EngineConfig cfg;
  cfg.rk = rule == FR_MFD ? RK_MULTI : RK_SINGLE;
  cfg.dir = DIR_FWD;
  cfg.vk = q_dtype == FR_F32 ? VK_FF : (q_dtype == FR_F64 ? VK_F64 : VK_NONE);
  cfg.counts = counts_out != nullptr;
  EngineParams P = common_params(nrows, ncols, code, z, mfd_p, base, L, dev_status);
  P.src32 = (rain && rain_dtype == FR_F32) ? static_cast<const float*>(rain) : nullptr;
  P.src64 = (rain && rain_dtype == FR_F64) ? static_cast<const double*>(rain) : nullptr;
  P.vhi = q_dtype == FR_F32 ? static_cast<float*>(q_out) : nullptr;
  P.v64 = q_dtype == FR_F64 ? static_cast<double*>(q_out) : nullptr;
  P.cnt = counts_out;
  int rc = run_engine(cfg, P, base, L, dev_status, stream);
  if (rc != FR_OK) return rc;
  if (mass_out) {
    double* partial = reinterpret_cast<double*>(base + L.partial);
    if (launch_mass(cfg.rk, cfg.vk, P, partial, kMassBlocks, mass_out, stream) != hipSuccess) return FR_ERR_HIP;
  }
  return FR_OK;
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
  if (!ws || ws_bytes < L.total) return FR_ERR_WORKSPACE;
  char* base = aligned_base(ws);

  EngineConfig cfg;
  cfg.rk = rule == FR_MFD ? RK_MULTI : RK_SINGLE;
  cfg.dir = DIR_ADJ;
  cfg.vk = dtype == FR_F32 ? VK_FF : VK_F64;
  cfg.counts = false;
  EngineParams P = common_params(nrows, ncols, code, z, mfd_p, base, L, dev_status);
  P.src32 = dtype == FR_F32 ? static_cast<const float*>(qbar) : nullptr;
  P.src64 = dtype == FR_F64 ? static_cast<const double*>(qbar) : nullptr;
  P.vhi = dtype == FR_F32 ? static_cast<float*>(rbar_out) : nullptr;
  P.v64 = dtype == FR_F64 ? static_cast<double*>(rbar_out) : nullptr;
  P.cnt = nullptr;
  return run_engine(cfg, P, base, L, dev_status, stream);
}

}  // extern "C"
