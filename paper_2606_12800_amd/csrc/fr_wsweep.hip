// Windowed wavefront sweep: general accumulation for any routing rule,
// forward (I - W^T) q = r or adjoint (I - W) rbar = qbar (Section 2.1,
// Section 2.2, Appendix A).
//
// The paper's sequential algorithm visits cells high-to-low so that every
// cell comes after all cells that feed it (Section 2.1); any order with that
// property gives the same solution (Section 3.2).  On terrain that drains
// mostly along one grid axis, visiting rows in flow order is almost such an
// order: a cell's inputs lie in the row visited before it, in its own row
// (chains resolved inside the row), or -- rarely, where the terrain locally
// rises against the row order -- in a row visited later.
//
// GPU mapping.  One wavefront owns a strip of 64 columns (lane = column) and
// visits the strip's rows in one direction.  Rows enter a ring of RING rows
// in LDS (state, value, MFD fractions).  A cell is computed once all of its
// inputs are final, by pulling them in fixed neighbour order, so results do
// not depend on timing.  Cells whose inputs are not yet final stay pending
// for up to WIN rows after their row entered; every newly final cell marks
// the neighbouring rows whose pending cells wait for it, which are then
// retried.  Columns next to a strip boundary read the neighbouring strip's
// edge cells from per-row records in HBM (written with device-coherent
// 64-bit stores of words that start out all ones, polled without blocking).
// No wavefront ever waits for another, so no schedule can hang.
//
// Cells still pending when their row leaves the window are left for a later
// pass; passes alternate the row direction and each one finishes at least
// the highest unfinished cell, so a valid DAG always completes and a pass
// that finishes nothing proves a cycle (FR_ERR_NOTDAG).  A pass marks the
// cells it leaves unfinished with a sentinel in a value array (NaN in the
// float-float low part or the float64 value, all ones in counts), so no
// separate done flags are stored.
//
// Precision: float-float (VK_FF, float32 output = hi), float64 (VK_F64),
// exact uint64 counts (CNT).  MFD fractions are computed as in the engine:
// float32 (s / s_max)^p via exp2/log2, or float64 pow.
#include <math.h>

#include "fr_internal.hpp"

namespace fr {
namespace {

// Real-time clock for the sweep's diagnostic counters, read only when they
// are switched on (each read waits for the scalar memory path).
__device__ __forceinline__ uint64_t diag_now(const WsParams& P) {
  return P.debug ? __builtin_amdgcn_s_memrealtime() : 0;
}

constexpr int LW = 66;         // LDS row: side cell, 64 lanes, side cell
// Strips overlap: a wavefront computes 64 columns, owns the middle WS_OWN
// and recomputes GHOST columns of each neighbour (as GHOST columns of its
// own are recomputed by the neighbours).  A value handed across a strip
// boundary then reaches the other strip's owned columns only after passing
// 2 * GHOST columns, which along lateral flow takes as many rows: the
// exchange has that many rows of slack.
constexpr int GHOST = WS_GHOST;
// Lanes whose cells the neighbours read as their side cells.
constexpr int REC_LANE_L = 2 * GHOST;    // read by the left neighbour's lane 63
constexpr int REC_LANE_R = WS_OWN - 1;   // read by the right neighbour's lane 0
// A strip does not start a row more than LEAD rows ahead of a neighbour
// (bounded wait), so neighbours stay within the exchange's slack.
constexpr int LEAD = 4;
constexpr int LEAD_SPIN = 1 << 14;  // polls before a neighbour counts as absent
// Before a row leaves the window with edge cells still waiting for side
// cells, the strip waits while the neighbour keeps making progress: a cell
// left unfinished here holds back everything downstream of it until a later
// pass.  The wait ends when the neighbour froze the rows in question, or
// made no progress for EDGE_STALL_TICKS (100 MHz ticks), or after
// EDGE_WAIT_MAX_TICKS in all.
constexpr uint64_t EDGE_STALL_TICKS = 2000;
constexpr uint64_t EDGE_WAIT_MAX_TICKS = 200000;
// Waits a strip may start before it must see some of them succeed (each
// failed wait costs 4, each successful one returns 1).
constexpr int WAIT_CREDIT = 16;
// Side cells delivered by the I/O wavefront are taken every ARRIVE_EVERY
// steps: edge lanes are ghost columns, so their cells may lag a few rows,
// and taking several deliveries at once retries each affected row once.
constexpr int ARRIVE_EVERY = 4;

constexpr uint32_t S_DONE = 1u << 8;
constexpr uint32_t S_PRIOR = 1u << 9;  // finished in an earlier pass

// ---------------------------------------------------------------------------
// Float-float arithmetic (Dekker 1971; Knuth TAOCP vol. 2, 4.2.2).
struct ff {
  float hi, lo;
};
__device__ __forceinline__ ff ff_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ff ff_fast_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ ff ff_add(ff x, ff y) {
  const ff s = ff_two_sum(x.hi, y.hi);
  return ff_fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
__device__ __forceinline__ ff ff_mul_f(ff x, float f) {
  const float p = x.hi * f;
  return ff_fast_two_sum(p, fmaf(x.hi, f, -p) + x.lo * f);
}

__device__ constexpr float kInvSqrt2f = 0x1.6a09e6p-1f;
__device__ constexpr double kSqrt2 = 1.4142135623730950488;

template <int VK>
struct ValOf {
  using T = float;  // VK_NONE: unused placeholder
};
template <>
struct ValOf<VK_FF> {
  using T = ff;
};
template <>
struct ValOf<VK_F64> {
  using T = double;
};
template <int RK, int VK>
struct FracOf {
  using T = float;
};
template <>
struct FracOf<RK_MULTI, VK_F64> {
  using T = double;
};

__device__ __forceinline__ void vzero(float& v) { v = 0.0f; }
__device__ __forceinline__ void vzero(ff& v) { v = {0.0f, 0.0f}; }
__device__ __forceinline__ void vzero(double& v) { v = 0.0; }
__device__ __forceinline__ void vadd(float&, float) {}
__device__ __forceinline__ void vadd(ff& a, ff b) { a = ff_add(a, b); }
__device__ __forceinline__ void vadd(double& a, double b) { a += b; }
__device__ __forceinline__ float vmul(float v, float) { return v; }
__device__ __forceinline__ ff vmul(ff v, float f) { return ff_mul_f(v, f); }
__device__ __forceinline__ double vmul(double v, double f) { return v * f; }
// v * f * (1 + d): a float32 fraction with the sender's conservation
// correction d (see the staging of MFD fractions).
__device__ __forceinline__ ff vmulc(ff v, float f, float d) {
  const ff p = ff_mul_f(v, f);
  return ff_fast_two_sum(p.hi, fmaf(p.hi, d, p.lo));
}
__device__ __forceinline__ double vmulc(double v, double f, float) { return v * f; }
__device__ __forceinline__ float vmulc(float v, float, float) { return v; }
// cond ? v : 0.
__device__ __forceinline__ float vsel(bool c, float v) { return c ? v : 0.0f; }
__device__ __forceinline__ ff vsel(bool c, ff v) { return {c ? v.hi : 0.0f, c ? v.lo : 0.0f}; }
__device__ __forceinline__ double vsel(bool c, double v) { return c ? v : 0.0; }
// What a donor with value v passes on along an edge of fraction f (with
// the sender's conservation correction d); a single receiver takes all.
template <int RK, typename V, typename F>
__device__ __forceinline__ V contrib(V v, F f, float d) {
  if constexpr (RK == RK_MULTI) return vmulc(v, f, d);
  else return v;
}

// Lane shifts across the whole wavefront (DPP wave_shr:1 / wave_shl:1); the
// lane shifted in receives 0.
__device__ __forceinline__ uint32_t from_left(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float from_left(float x) { return __uint_as_float(from_left(__float_as_uint(x))); }
__device__ __forceinline__ float from_right(float x) { return __uint_as_float(from_right(__float_as_uint(x))); }
__device__ __forceinline__ uint64_t from_left(uint64_t x) {
  return ((uint64_t)from_left((uint32_t)(x >> 32)) << 32) | from_left((uint32_t)x);
}
__device__ __forceinline__ uint64_t from_right(uint64_t x) {
  return ((uint64_t)from_right((uint32_t)(x >> 32)) << 32) | from_right((uint32_t)x);
}
__device__ __forceinline__ double from_left(double x) {
  return __longlong_as_double((long long)from_left((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ double from_right(double x) {
  return __longlong_as_double((long long)from_right((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ ff from_left(ff x) { return {from_left(x.hi), from_left(x.lo)}; }
__device__ __forceinline__ ff from_right(ff x) { return {from_right(x.hi), from_right(x.lo)}; }

template <int RK>
__device__ __forceinline__ bool sends(uint32_t code, int k) {
  return RK == RK_SINGLE ? (code == (uint32_t)k) : (((code >> k) & 1u) != 0);
}

// Edge records: 64-bit payload words, initialised to all ones -- a pattern
// no payload takes (finite values and fractions, counts below 2^63).  Each
// word is written and read with one 64-bit atomic access, so a word that is
// no longer all ones holds its final payload.
constexpr uint64_t REC_EMPTY = ~0ull;
__device__ __forceinline__ void rec_put(uint64_t* p, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t rec_get(const uint64_t* p) {
  return (uint64_t)__hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p)),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void prog_put(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t prog_get(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t pack2(float a, float b) {
  return (uint64_t)__float_as_uint(a) | ((uint64_t)__float_as_uint(b) << 32);
}
__device__ __forceinline__ float lo_f(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ __forceinline__ float hi_f(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32)); }
__device__ __forceinline__ uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(uint64_t w) { return __longlong_as_double((long long)w); }

// Record words of a configuration: the value (one word, float-float packed)
// then, MFD forward, the three fractions toward the neighbouring column
// (float32: two words; float64: three); D8 forward with counts: the count.
template <int RK, int DK, int VK, bool CNT>
constexpr int rec_words() {
  return DK == DIR_ADJ ? 1
                       : (RK == RK_MULTI ? 1 + (VK == VK_F64 ? 3 : 2) : (VK != VK_NONE ? 1 : 0) + (CNT ? 1 : 0));
}
static_assert(rec_words<RK_MULTI, DIR_FWD, VK_F64, false>() <= WS_EW, "edge record too small");

// Ring geometry per configuration (LDS per workgroup stays below 80 KB so
// that two workgroups fit on a compute unit): RING rows in LDS; a row may
// finish during the WIN steps after it became the newest; rows up to
// RING - WIN - 2 ahead of the newest are staged; BATCH rows are staged at a
// time.
template <int RK, int VK>
struct Dims {
  static constexpr bool F64M = RK == RK_MULTI && VK == VK_F64;
  static constexpr int RING = RK == RK_SINGLE ? 32 : (F64M ? 15 : 24);
  static constexpr int WIN = RK == RK_SINGLE ? 22 : (F64M ? 9 : 14);
  static constexpr int BATCH = (RING - WIN - 2) / 2;
};

template <int RK, int VK, bool CNT>
struct WsShared {
  using V = typename ValOf<VK>::T;
  using F = typename FracOf<RK, VK>::T;
  static constexpr int R = Dims<RK, VK>::RING;
  uint32_t st[R][LW];   // bits 0-7 routing code, S_DONE, S_PRIOR
  uint8_t miss[R][LW];  // pending cells: directions of inputs not yet final
  V val[R][LW];         // final value, or the source term while pending
  uint64_t cnt[CNT ? R : 1][LW];
  F frac[RK == RK_MULTI ? R : 1][8][LW];  // MFD: fraction sent in direction k
  // MFD float32: d with (sum_k frac_k) * (1 + d) = 1 to float-float accuracy,
  // so that a cell passes on exactly the water it holds.
  float fd[RK == RK_MULTI && VK == VK_FF ? R : 1][LW];
  // Hand-over between the two wavefronts.
  int staged;         // rows (steps) 0 .. staged-1 are in the ring
  int tcomp;          // the compute wavefront's current step
  int done;           // the compute wavefront has finished
  uint32_t arrived;   // slots whose side cell was delivered since last taken
  int nbp[2];         // neighbours' progress (left, right) as last read
};

// One row of geometry for this lane: own cell and (lanes 0, 63) the cell
// across the strip boundary.
struct Geo {
  uint32_t code, scode;
  float z, sz;
};

template <int VK>
struct Src {
  typename ValOf<VK>::T v;
  uint64_t n;
  bool prior;
};

// Orders one wavefront's LDS accesses: a wavefront executes its LDS
// instructions in order, so only the compiler must not move them across.
__device__ __forceinline__ void lds_sync() { asm volatile("" ::: "memory"); }
// Hand-over words between the two wavefronts live in LDS; the accesses name
// the LDS address space so that they compile to ds_read / ds_write (a
// volatile access through a generic pointer becomes a flat, system-coherent
// access that waits for all of the wavefront's outstanding memory traffic).
typedef __attribute__((address_space(3))) int lds_int;
__device__ __forceinline__ int lds_ld(const int* p) { return *(const volatile lds_int*)p; }
__device__ __forceinline__ void lds_st(int* p, int v) { *(volatile lds_int*)p = v; }

// Two wavefronts per workgroup.  Wavefront 1 (I/O) stages rows into the
// ring ahead of use -- codes, elevations, source terms, earlier passes'
// results, MFD fractions -- polls the neighbours' edge records and progress,
// and delivers them into LDS.  Wavefront 0 (compute) only reads and writes
// LDS and stores results, so it never waits for global memory.
// One pass over one strip by a workgroup of two wavefronts (see above);
// returns when both have finished.
template <int RK, int DK, int VK, bool CNT>
__device__ void ws_strip(WsShared<RK, VK, CNT>& S, const WsParams& P, const int64_t strip, const int dir,
                         const int first) {
  using V = typename ValOf<VK>::T;
  using F = typename FracOf<RK, VK>::T;
  constexpr int R = Dims<RK, VK>::RING;
  constexpr int WIN = Dims<RK, VK>::WIN;
  constexpr int BATCH = Dims<RK, VK>::BATCH;
  constexpr int EWN = rec_words<RK, DK, VK, CNT>();
  constexpr uint32_t NOC = RK == RK_SINGLE ? (uint32_t)SINK : 0u;

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int li = lane + 1;
  const int nr = (int)P.nrows;
  const int64_t nc = P.ncols;
  const int64_t nstrips = (nc + WS_OWN - 1) / WS_OWN;
  const int64_t c = strip * WS_OWN - GHOST + lane;
  const bool live = c >= 0 && c < nc;
  const bool owned = live && lane >= GHOST && lane < GHOST + WS_OWN;
  const bool sideL = lane == 0 && c - 1 >= 0 && c - 1 < nc;
  const bool sideR = lane == 63 && c + 1 >= 0 && c + 1 < nc;
  const bool has_side = sideL || sideR;
  const bool edge_lane = lane == 0 || lane == 63;
  const int64_t cs = lane == 0 ? c - 1 : c + 1;
  const int sidx = lane == 0 ? 0 : LW - 1;
  // Neighbour strips exist (per side) with an edge cell next to ours.
  const int64_t c_first = strip * WS_OWN - GHOST, c_last = c_first + 63;
  const bool nb_exists[2] = {c_first - 1 >= 0 && c_first - 1 < nc, c_last + 1 >= 0 && c_last + 1 < nc};
  const float pf = (float)P.p;

  auto row_of = [&](int t) -> int64_t { return dir < 0 ? (int64_t)nr - 1 - t : (int64_t)t; };
  auto slot = [&](int t) -> int { return t % R; };

  if (threadIdx.x == 0) {
    S.staged = 0;
    S.tcomp = -1;
    S.done = 0;
    S.arrived = 0u;
    S.nbp[0] = nb_exists[0] ? -1 : 0x3FFFFFFF;
    S.nbp[1] = nb_exists[1] ? -1 : 0x3FFFFFFF;
  }
  __syncthreads();

  if (wave == 1) {
    // ======================= I/O wavefront ===============================
    // Direction codes run as one-bit masks (fraction 1) in the MFD variant.
    auto as_mask = [&](uint32_t code) -> uint32_t {
      if (RK == RK_MULTI && P.codes_single) return code <= 7u ? (1u << code) : 0u;
      return code;
    };
    auto load_geo = [&](int t) -> Geo {
      Geo g{NOC, NOC, INFINITY, INFINITY};
      if (t < 0 || t >= nr) return g;
      const int64_t rb = row_of(t) * nc;
      if (live) {
        g.code = as_mask(P.code[rb + c]);
        if (RK == RK_MULTI) g.z = P.z[rb + c];
      }
      if (has_side) {
        g.scode = as_mask(P.code[rb + cs]);
        if (RK == RK_MULTI) g.sz = P.z[rb + cs];
      }
      return g;
    };
    auto load_src = [&](int t) -> Src<VK> {
      Src<VK> sr;
      vzero(sr.v);
      sr.n = 1;
      sr.prior = false;
      if (t < 0 || t >= nr || !live) return sr;
      const int64_t i = row_of(t) * nc + c;
      if constexpr (VK == VK_FF) {
        if (P.src64) {
          const double d = P.src64[i];
          sr.v.hi = (float)d;
          sr.v.lo = (float)(d - (double)sr.v.hi);
        } else {
          sr.v = {P.src32 ? P.src32[i] : 1.0f, 0.0f};
        }
        if (!first) {
          const float lo = P.vlo[i];
          if (!isnan(lo)) {
            sr.v = {P.vhi[i], lo};
            sr.prior = true;
          }
        }
      } else if constexpr (VK == VK_F64) {
        sr.v = P.src64 ? P.src64[i] : (P.src32 ? (double)P.src32[i] : 1.0);
        if (!first) {
          const double y = P.v64[i];
          if (!isnan(y)) {
            sr.v = y;
            sr.prior = true;
          }
        }
      } else {
        if (CNT && !first && P.cnt[i] != ~0ull) sr.prior = true;
      }
      if (CNT && sr.prior) sr.n = P.cnt[i];
      return sr;
    };

    bool bad = false, nonfinite = false;
    // Wanted side cells not yet delivered, per side (left, right), by slot.
    uint32_t want0 = 0u, want1 = 0u;
    // Adjoint: an edge cell gives water to the side cell one step ahead
    // (kept in the edge lane itself).
    bool want_next = false;

    // Writes the row at step y (geometry of steps y-1, y, y+1) into its slot.
    auto stage_row = [&](int y, const Geo& ga, const Geo& gb, const Geo& gc, const Src<VK>& sr) {
      const int sb = slot(y);
      const uint32_t code = gb.code;
      if constexpr (RK == RK_MULTI) {
        const Geo& gu = dir < 0 ? gc : ga;  // grid row r - 1
        const Geo& gd = dir < 0 ? ga : gc;  // grid row r + 1
        float zn[8];
        zn[0] = from_left(gu.z);
        zn[1] = gu.z;
        zn[2] = from_right(gu.z);
        zn[3] = from_left(gb.z);
        zn[4] = from_right(gb.z);
        zn[5] = from_left(gd.z);
        zn[6] = gd.z;
        zn[7] = from_right(gd.z);
        if (lane == 0) {
          zn[0] = sideL ? gu.sz : INFINITY;
          zn[3] = sideL ? gb.sz : INFINITY;
          zn[5] = sideL ? gd.sz : INFINITY;
        }
        if (lane == 63) {
          zn[2] = sideR ? gu.sz : INFINITY;
          zn[4] = sideR ? gb.sz : INFINITY;
          zn[7] = sideR ? gd.sz : INFINITY;
        }
        const float zi = gb.z;
        if (live && !isfinite(zi)) nonfinite = true;
        F fr[8];
        if constexpr (VK == VK_F64) {
          double w[8], sum = 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            w[k] = 0.0;
            if (!live || !sends<RK>(code, k)) continue;
            if (!(zn[k] < zi)) {
              bad = true;
              continue;
            }
            const double sl = ((double)zi - (double)zn[k]) / (nb_diag(k) ? kSqrt2 : 1.0);
            w[k] = pow(sl, P.p);
            sum += w[k];
          }
          const double iw = sum > 0.0 ? 1.0 / sum : 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k) fr[k] = w[k] * iw;
        } else {
          float sl[8], smax = 0.0f;
          bool rcv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            sl[k] = 0.0f;
            rcv[k] = false;
            if (!live || !sends<RK>(code, k)) continue;
            if (!(zn[k] < zi)) {
              bad = true;
              continue;
            }
            rcv[k] = true;
            const float drop = zi - zn[k];
            sl[k] = nb_diag(k) ? drop * kInvSqrt2f : drop;
            smax = sl[k] > smax ? sl[k] : smax;
          }
          // t_k = (s_k / s_max)^p from a correctly rounded quotient (the
          // steepest direction gets exactly 1), f_k = t_k / sum t: a few ulp
          // per fraction.
          float tk[8], sum = 0.0f;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            tk[k] = rcv[k] ? exp2f(pf * log2f(sl[k] / smax)) : 0.0f;
            sum += tk[k];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) fr[k] = sum > 0.0f ? tk[k] / sum : 0.0f;
          // Rounded fractions do not sum to 1 exactly; over thousands of
          // cells along a flow path the excess would compound.  With the
          // exact sum s (float-float), d = 1/s - 1 ~ -(s - 1) restores it.
          ff es = {0.0f, 0.0f};
#pragma unroll
          for (int k = 0; k < 8; ++k) es = ff_add(es, ff{fr[k], 0.0f});
          S.fd[sb][li] = sum > 0.0f ? -((es.hi - 1.0f) + es.lo) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) S.frac[sb][k][li] = fr[k];
      } else {
        if (live && code != SINK) {
          if (code > 7) {
            bad = true;
          } else {
            const int k = (int)code;
            const int64_t rr = row_of(y) + nb_dr(k), cc = c + nb_dc(k);
            if (rr < 0 || rr >= nr || cc < 0 || cc >= nc) bad = true;
          }
        }
      }
      if constexpr (VK == VK_FF) {
        if (live && !isfinite(sr.v.hi)) nonfinite = true;
      } else if constexpr (VK == VK_F64) {
        if (live && !isfinite(sr.v)) nonfinite = true;
      }
      uint32_t st = live ? (code & 0xFFu) : (NOC | S_DONE);
      if (live && sr.prior) st |= S_DONE | S_PRIOR;
      S.st[sb][li] = st;
      S.miss[sb][li] = 0;
      V v = sr.v;
      if (!live) vzero(v);
      S.val[sb][li] = v;
      if constexpr (CNT) S.cnt[sb][li] = live ? sr.n : 0;
      if (edge_lane) {
        S.st[sb][sidx] = has_side ? (gb.scode & 0xFFu) : (NOC | S_DONE);
        V v0;
        vzero(v0);
        S.val[sb][sidx] = v0;
        if constexpr (CNT) S.cnt[sb][sidx] = 0;
        if constexpr (RK == RK_MULTI) {
#pragma unroll
          for (int k = 0; k < 8; ++k) S.frac[sb][k][sidx] = (F)0;
          if constexpr (VK == VK_FF) S.fd[sb][sidx] = 0.0f;
        }
      }
      // Wanted side cells (uniform masks from the edge lanes).
      bool wl = false, wprev = false;
      if (has_side) {
        if (DK == DIR_FWD) {
          // The side cell gives water toward this strip's edge column.
          wl = lane == 0 ? (sends<RK>(gb.scode, 2) || sends<RK>(gb.scode, 4) || sends<RK>(gb.scode, 7))
                         : (sends<RK>(gb.scode, 0) || sends<RK>(gb.scode, 3) || sends<RK>(gb.scode, 5));
        } else {
          // The edge cell gives water to side cells at grid rows r-1, r, r+1.
          const int ka = lane == 0 ? 0 : 2, kb = lane == 0 ? 3 : 4, kc = lane == 0 ? 5 : 7;
          const bool up = sends<RK>(code, ka), mid = sends<RK>(code, kb), dn = sends<RK>(code, kc);
          const bool prev = dir < 0 ? dn : up, next = dir < 0 ? up : dn;  // steps y-1, y+1
          wl = mid || want_next;
          wprev = prev && y >= 1;
          want_next = next;
        }
      }
      const uint64_t bw = __ballot(wl), bp = __ballot(wprev);
      want0 &= ~(1u << sb);
      want1 &= ~(1u << sb);
      if (bw & 1ull) want0 |= 1u << sb;
      if ((bw >> 63) & 1ull) want1 |= 1u << sb;
      if (y >= 1) {
        if (bp & 1ull) want0 |= 1u << slot(y - 1);
        if ((bp >> 63) & 1ull) want1 |= 1u << slot(y - 1);
      }
    };

    Geo gp = load_geo(-1), gcur = load_geo(0);
    int y = 0;  // next step to stage
    // The next batch is loaded one iteration ahead of its use.
    Geo g[BATCH];
    Src<VK> sr[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      g[j] = load_geo(1 + j);
      sr[j] = load_src(j);
    }
    int idle = 0;
    uint64_t io_stage = 0, io_poll = 0, io_iter = 0;  // diagnostics
    for (;;) {
      if (lds_ld(&S.done)) break;
      const int tc = lds_ld(&S.tcomp);
      bool busy = false;
      ++io_iter;
      uint64_t q0 = diag_now(P);
      // Stage a batch once its slots are free: the compute wavefront reads
      // steps tc - WIN .. tc + 1.
      if (y < nr && y + BATCH - 1 <= tc - WIN - 1 + R) {
#pragma unroll
        for (int j = 0; j < BATCH; ++j) {
          const Geo& ga = j == 0 ? gp : (j == 1 ? gcur : g[j - 2]);
          const Geo& gb = j == 0 ? gcur : g[j - 1];
          if (y + j < nr) stage_row(y + j, ga, gb, g[j], sr[j]);
        }
        gp = BATCH >= 2 ? g[BATCH - 2] : gcur;
        gcur = g[BATCH - 1];
        y += BATCH;
        lds_sync();
        if (lane == 0) lds_st(&S.staged, y < nr ? y : nr);
        busy = true;
        if (y < nr) {
#pragma unroll
          for (int j = 0; j < BATCH; ++j) {
            g[j] = load_geo(y + 1 + j);
            sr[j] = load_src(y + j);
          }
        }
      }
      uint64_t q1 = diag_now(P);
      io_stage += q1 - q0;
      q0 = q1;
      // Poll the neighbours' records for wanted rows still in the ring,
      // lane-parallel: lanes 0-31 the left neighbour, 32-63 the right one;
      // four lanes (words) per row, eight rows per load.
      const int plo = tc - WIN > 0 ? tc - WIN : 0;
      const int phi = (y < nr ? y : nr) - 1;
      if ((want0 | want1) && plo <= phi) {
        const int sd = lane >> 5, j = lane & 31, r8 = j >> 2, w = j & 3;
        const int64_t rstrip = sd == 0 ? strip - 1 : strip + 1;
        const int rside = sd == 0 ? 1 : 0;
        const int ksd0 = sd == 0 ? 2 : 0, ksd1 = sd == 0 ? 4 : 3, ksd2 = sd == 0 ? 7 : 5;
        const int sx_idx = sd == 0 ? 0 : LW - 1;
        uint32_t arr = 0;
        constexpr int NB = (R + 7) / 8;
        uint64_t wd[NB];
        bool actb[NB];
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
          const int x = plo + bb * 8 + r8;
          actb[bb] = w < EWN && x <= phi && nb_exists[sd] && ((((sd == 0 ? want0 : want1)) >> slot(x)) & 1u);
          wd[bb] = actb[bb] ? rec_get(P.edge + ((rstrip * P.nrows + row_of(x)) * 2 + rside) * WS_EW + w)
                            : REC_EMPTY;
        }
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
          const int b0 = plo + bb * 8;
          if (b0 > phi) break;
          const int x = b0 + r8;
          const bool act = actb[bb];
          const uint64_t word = wd[bb];
          const uint64_t okm = __ballot(act && word != REC_EMPTY);
          const uint64_t rowm = (((1ull << EWN) - 1ull) << (sd * 32 + r8 * 4));
          const bool complete = act && (okm & rowm) == rowm;
          if (complete) {
            const int sx = slot(x);
            if (w == 0) {
              V v;
              vzero(v);
              if constexpr (VK == VK_FF) {
                v.hi = lo_f(word);
                v.lo = hi_f(word);
              } else if constexpr (VK == VK_F64) {
                v = bitsd(word);
              }
              if constexpr (VK != VK_NONE) S.val[sx][sx_idx] = v;
              if constexpr (DK == DIR_FWD && RK == RK_SINGLE && CNT && VK == VK_NONE) S.cnt[sx][sx_idx] = word;
            } else if constexpr (DK == DIR_FWD && RK == RK_MULTI) {
              if constexpr (VK == VK_F64) {
                S.frac[sx][w == 1 ? ksd0 : (w == 2 ? ksd1 : ksd2)][sx_idx] = bitsd(word);
              } else {
                if (w == 1) {
                  S.frac[sx][ksd0][sx_idx] = lo_f(word);
                  S.frac[sx][ksd1][sx_idx] = hi_f(word);
                } else {
                  S.frac[sx][ksd2][sx_idx] = lo_f(word);
                  S.fd[sx][sx_idx] = hi_f(word);
                }
              }
            } else if constexpr (DK == DIR_FWD && RK == RK_SINGLE && CNT) {
              S.cnt[sx][sx_idx] = word;
            }
          }
          lds_sync();
          if (complete && w == 0) {
            const int sx = slot(x);
            S.st[sx][sx_idx] |= S_DONE;
            arr |= 1u << sx;
          }
          // Delivered rows leave the wanted sets.
          const uint64_t done_rows = __ballot(complete && w == 0);
          for (int qr = 0; qr < 8; ++qr) {
            if ((done_rows >> (qr * 4)) & 1ull) want0 &= ~(1u << slot(b0 + qr));
            if ((done_rows >> (32 + qr * 4)) & 1ull) want1 &= ~(1u << slot(b0 + qr));
          }
        }
        // Publish deliveries after their payload.
        for (int off = 32; off > 0; off >>= 1) arr |= (uint32_t)__shfl_xor((int)arr, off, 64);
        lds_sync();
        if (lane == 0 && arr) {
          atomicOr(&S.arrived, arr);
          busy = true;
        }
      }
      // Neighbours' progress, for pacing and for knowing what they froze.
      if ((lane == 0 && nb_exists[0]) || (lane == 32 && nb_exists[1])) {
        const int sd = lane == 0 ? 0 : 1;
        const int v = prog_get(P.progress + (sd == 0 ? strip - 1 : strip + 1));
        if (v != lds_ld(&S.nbp[sd])) {
          lds_st(&S.nbp[sd], v);
        }
      }
      io_poll += diag_now(P) - q0;
      if (!busy) {
        if (++idle > 4) __builtin_amdgcn_s_sleep(2);
      } else {
        idle = 0;
      }
    }
    if (lane == 0 && P.debug) {
      unsigned long long* tm = reinterpret_cast<unsigned long long*>(P.ctr + 8);
      atomicAdd(tm + 5, (unsigned long long)io_stage);
      atomicAdd(tm + 6, (unsigned long long)io_poll);
      atomicAdd(tm + 7, (unsigned long long)io_iter);
    }
    if (first && P.status) {
      if (__ballot(bad) && lane == 0) atomicCAS(P.status, 0, FR_ERR_BADCODE);
      if (__ballot(nonfinite) && lane == 0) atomicCAS(P.status, 0, FR_ERR_NONFINITE);
    }
  } else {
  // ======================== compute wavefront ============================
  const int my_side = lane == REC_LANE_L ? 0 : 1;
  const bool has_record = live && ((lane == REC_LANE_L && strip > 0) || (lane == REC_LANE_R && strip + 1 < nstrips));
  uint32_t pend_rows = 0, nfin = 0;
  uint32_t n_wait = 0, n_pace = 0, n_resolve = 0, n_iter = 0;  // diagnostics
  uint64_t tm_resolve = 0, tm_loop = 0;
  bool fail = false;

  // Publishes a newly final cell that a neighbour reads as its side cell.
  auto put_record = [&](int x, int sb, const V& v, uint64_t n) {
    uint64_t* rec = P.edge + ((strip * P.nrows + row_of(x)) * 2 + my_side) * WS_EW;
    int w = 0;
    if constexpr (VK == VK_FF) rec_put(rec + w++, pack2(v.hi, v.lo));
    else if constexpr (VK == VK_F64) rec_put(rec + w++, dbits(v));
    if constexpr (DK == DIR_FWD && RK == RK_MULTI) {
      // Fractions toward the neighbouring column, grid rows r-1, r, r+1.
      const F f0 = S.frac[sb][my_side == 0 ? 0 : 2][li];
      const F f1 = S.frac[sb][my_side == 0 ? 3 : 4][li];
      const F f2 = S.frac[sb][my_side == 0 ? 5 : 7][li];
      if constexpr (VK == VK_F64) {
        rec_put(rec + w++, dbits(f0));
        rec_put(rec + w++, dbits(f1));
        rec_put(rec + w++, dbits(f2));
      } else {
        rec_put(rec + w++, pack2(f0, f1));
        rec_put(rec + w++, pack2(f2, S.fd[sb][li]));
      }
    }
    if constexpr (DK == DIR_FWD && RK == RK_SINGLE && CNT) rec_put(rec + w++, n);
    (void)n;
  };

  // Tries to finish the pending cells of the row at step x (slot sb).
  // Returns the lanes finished.
  auto resolve = [&](int x, int sb) -> uint64_t {
    const uint32_t me = S.st[sb][li];
    const bool pend = !(me & S_DONE);
    const uint32_t code = me & 0xFFu;
    V acc = S.val[sb][li];
    uint64_t accn = CNT ? S.cnt[sb][li] : 0;
    bool ok = pend;
    uint32_t miss = 0;
    // Gather the six neighbours in the rows before and after without
    // branches, so that all LDS reads are in flight together; rows off the
    // grid read as finished cells that give nothing.
    uint32_t sj[8];
    V vj[8];
    F fj[8];
    float dj[8];
    uint64_t nj[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k == 3 || k == 4) continue;
      const int xn = x + nb_dr(k) * dir;
      const bool row_ok = xn >= 0 && xn < nr;
      const int sn = slot(row_ok ? xn : x);
      const int ln = li + nb_dc(k);
      sj[k] = row_ok ? S.st[sn][ln] : (NOC | S_DONE);
      if constexpr (VK != VK_NONE) vj[k] = S.val[sn][ln];
      if constexpr (RK == RK_MULTI) fj[k] = DK == DIR_FWD ? S.frac[sn][7 - k][ln] : S.frac[sb][k][li];
      if constexpr (RK == RK_MULTI && VK == VK_FF) dj[k] = DK == DIR_FWD ? S.fd[sn][ln] : S.fd[sb][li];
      else dj[k] = 0.0f;
      if constexpr (CNT) nj[k] = S.cnt[sn][ln];
    }
    // Contributions of the final inputs (zero for the others), summed
    // pairwise in a fixed order: shorter dependency chains than a running
    // sum, and the same result whichever resolve finishes the cell.
    V cj[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k == 3 || k == 4) continue;
      const bool input = pend && (DK == DIR_FWD ? sends<RK>(sj[k] & 0xFFu, 7 - k) : sends<RK>(code, k)) &&
                         x + nb_dr(k) * dir >= 0 && x + nb_dr(k) * dir < nr;
      const bool fin = (sj[k] & S_DONE) != 0;
      if (input && !fin) {
        ok = false;
        miss |= 1u << k;
      }
      const bool take = input && fin;
      if constexpr (VK != VK_NONE) cj[k] = vsel(take, contrib<RK>(vj[k], fj[k], dj[k]));
      if constexpr (CNT) accn += take ? nj[k] : 0;
    }
    if constexpr (VK != VK_NONE) {
      V s0 = cj[0], s1 = cj[2], s2 = cj[6];
      vadd(s0, cj[1]);
      vadd(s1, cj[5]);
      vadd(s2, cj[7]);
      vadd(s0, s1);
      vadd(s0, s2);
      vadd(acc, s0);
    }
    // Same-row inputs, iterated along the row with lane shifts.
    const uint32_t sl = S.st[sb][li - 1], sr = S.st[sb][li + 1];
    const bool in_l = pend && (DK == DIR_FWD ? sends<RK>(sl & 0xFFu, 4) : sends<RK>(code, 3));
    const bool in_r = pend && (DK == DIR_FWD ? sends<RK>(sr & 0xFFu, 3) : sends<RK>(code, 4));
    F fl = (F)1, fr_ = (F)1;
    float dfl = 0.0f, dfr = 0.0f;
    if constexpr (RK == RK_MULTI) {
      fl = DK == DIR_FWD ? S.frac[sb][4][li - 1] : S.frac[sb][3][li];
      fr_ = DK == DIR_FWD ? S.frac[sb][3][li + 1] : S.frac[sb][4][li];
    }
    if constexpr (RK == RK_MULTI && VK == VK_FF) {
      dfl = DK == DIR_FWD ? S.fd[sb][li - 1] : S.fd[sb][li];
      dfr = DK == DIR_FWD ? S.fd[sb][li + 1] : S.fd[sb][li];
    }
    // Side cells of lanes 0 and 63 (another strip) come from LDS.
    bool dside = false;
    V vside;
    vzero(vside);
    uint64_t nside = 0;
    if (edge_lane) {
      dside = ((lane == 0 ? sl : sr) & S_DONE) != 0;
      vside = S.val[sb][sidx];
      if constexpr (CNT) nside = S.cnt[sb][sidx];
    }
    uint32_t cd = pend ? 0u : 1u;
    V cv = S.val[sb][li];
    uint64_t cn = CNT ? S.cnt[sb][li] : 0;
    bool newly = false, dl = false, dr = false;
    const uint64_t tl0 = P.debug ? __builtin_amdgcn_s_memrealtime() : 0;
    for (int it = 0; it < 66; ++it) {
      dl = from_left(cd) != 0;
      dr = from_right(cd) != 0;
      V vl = from_left(cv), vr = from_right(cv);
      uint64_t nl = 0, nrr = 0;
      if constexpr (CNT) {
        nl = from_left(cn);
        nrr = from_right(cn);
      }
      if (lane == 0) {
        dl = dside;
        vl = vside;
        nl = nside;
      }
      if (lane == 63) {
        dr = dside;
        vr = vside;
        nrr = nside;
      }
      const bool can = ok && !cd && (!in_l || dl) && (!in_r || dr);
      if (can) {
        V w = acc;
        uint64_t wn = accn;
        if (in_l) {
          vadd(w, contrib<RK>(vl, fl, dfl));
          wn += nl;
        }
        if (in_r) {
          vadd(w, contrib<RK>(vr, fr_, dfr));
          wn += nrr;
        }
        cv = w;
        cn = wn;
        cd = 1u;
        newly = true;
      }
      ++n_iter;
      if (__ballot(can) == 0) break;
    }
    if (P.debug) tm_loop += __builtin_amdgcn_s_memrealtime() - tl0;
    if (newly) {
      S.st[sb][li] = me | S_DONE;
      S.val[sb][li] = cv;
      if constexpr (CNT) S.cnt[sb][li] = cn;
      if (has_record) put_record(x, sb, cv, cn);
    } else if (pend) {
      if (in_l && !dl) miss |= 1u << 3;
      if (in_r && !dr) miss |= 1u << 4;
      S.miss[sb][li] = (uint8_t)miss;
    }
    return __ballot(newly);
  };

  // Whether pending cells of row y wait for cells of row x finished in D.
  auto affected = [&](int y, int x, uint64_t D) -> bool {
    const int sy = slot(y);
    const uint32_t m = S.miss[sy][li];
    const bool pend = !(S.st[sy][li] & S_DONE);
    const int kb = ((x - y) * dir) < 0 ? 0 : 5;
    bool a = false;
    if (pend) {
      a = a || (((m >> kb) & 1u) && lane >= 1 && ((D >> (lane - 1)) & 1ull));
      a = a || (((m >> (kb + 1)) & 1u) && ((D >> lane) & 1ull));
      a = a || (((m >> (kb + 2)) & 1u) && lane <= 62 && ((D >> (lane + 1)) & 1ull));
    }
    return __ballot(a) != 0;
  };

  // Step of the row held in slot sb among steps t - R + 1 .. t.
  auto step_of = [&](int sb, int t) -> int { return t - (((t % R) - sb + R) % R); };

  // Retries rows until nothing changes; window = steps lo..t.
  auto settle = [&](uint32_t dirty, int lo, int t) {
    while (dirty) {
      const int sb = __builtin_ctz(dirty);
      dirty &= dirty - 1;
      const int x = step_of(sb, t);
      if (x < lo || !((pend_rows >> sb) & 1u)) continue;
      lds_sync();
      ++n_resolve;
      const uint64_t tr0 = P.debug ? __builtin_amdgcn_s_memrealtime() : 0;
      const uint64_t D = resolve(x, sb);
      if (P.debug) tm_resolve += __builtin_amdgcn_s_memrealtime() - tr0;
      lds_sync();
      const bool still = __ballot(!(S.st[sb][li] & S_DONE)) != 0;
      pend_rows = still ? (pend_rows | (1u << sb)) : (pend_rows & ~(1u << sb));
      if (D) {
#pragma unroll
        for (int d = -1; d <= 1; d += 2) {
          const int yy = x + d;
          if (yy < lo || yy > t) continue;
          const int sy = slot(yy);
          if (((pend_rows >> sy) & 1u) && affected(yy, x, D)) dirty |= 1u << sy;
        }
      }
    }
  };

  // Side cells delivered since the last call: rows lo..t whose edge cell
  // waits for one of them.
  auto take_arrivals = [&](int lo, int t) -> uint32_t {
    uint32_t arr = 0;
    if (lane == 0) arr = atomicExch(&S.arrived, 0u);
    arr = (uint32_t)__builtin_amdgcn_readfirstlane((int)arr);
    if (!arr) return 0u;
    lds_sync();
    uint32_t dirty = 0;
    while (arr) {
      const int sx = __builtin_ctz(arr);
      arr &= arr - 1;
      const int x = step_of(sx, t + R - WIN - 1);  // deliveries reach up to the staged rows
#pragma unroll
      for (int d = -1; d <= 1; ++d) {
        const int yy = x + d;
        if (yy < lo || yy > t || !has_side) continue;
        const int sy = slot(yy);
        const int dr = (x - yy) * dir;
        const int k = lane == 0 ? (dr < 0 ? 0 : (dr == 0 ? 3 : 5)) : (dr < 0 ? 2 : (dr == 0 ? 4 : 7));
        if (!(S.st[sy][li] & S_DONE) && ((S.miss[sy][li] >> k) & 1u)) dirty |= 1u << sy;
      }
    }
    return (uint32_t)__builtin_amdgcn_readlane((int)dirty, 0) | (uint32_t)__builtin_amdgcn_readlane((int)dirty, 63);
  };

  // Neighbours that stopped answering are not waited for.
  bool absent[2] = {false, false};
  int nb_last[2] = {-2, -2}, nb_same[2] = {0, 0};

  // Whether the edge lanes of row f still wait for side cells that the
  // neighbour has not given up on (it freezes row x at step x + WIN - 1).
  auto edge_wait_needed = [&](int f) -> bool {
    const int sf = slot(f);
    bool need = false;
    const int sd = lane == 0 ? 0 : 1;
    if (has_side && !absent[sd] && !(S.st[sf][li] & S_DONE)) {
      const uint32_t m = S.miss[sf][li] & (lane == 0 ? 0x29u : 0x94u);
      const int nb = lds_ld(&S.nbp[sd]);
      need = m != 0 && nb < f + 1 + WIN + 1;
    }
    return __ballot(need) != 0;
  };

  // Whether edge cells of row f still wait for side cells.
  auto edge_missing = [&](int f) -> bool {
    const int sf = slot(f);
    const uint32_t m = S.miss[sf][li] & (lane == 0 ? 0x29u : 0x94u);
    return __ballot(has_side && !(S.st[sf][li] & S_DONE) && m != 0) != 0;
  };

  // Waiting pays off where the neighbour is about to deliver; where its
  // side cells cannot finish in this pass (terrain draining against the
  // sweep) the wait only holds everyone back.  A strip stops waiting once
  // its waits keep ending without the side cells.
  int wait_credit = WAIT_CREDIT;
  auto wait_edges = [&](int f, int lo, int t) {
    if (wait_credit <= 0) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    uint64_t t_last = t0;
    int seen0 = lds_ld(&S.nbp[0]), seen1 = lds_ld(&S.nbp[1]);
    for (int it = 0; it < (1 << 20); ++it) {
      if (!edge_wait_needed(f)) break;
      const uint64_t now = __builtin_amdgcn_s_memrealtime();
      const int p0 = lds_ld(&S.nbp[0]), p1 = lds_ld(&S.nbp[1]);
      if (p0 != seen0 || p1 != seen1) {
        seen0 = p0;
        seen1 = p1;
        t_last = now;
      }
      if (now - t_last > EDGE_STALL_TICKS || now - t0 > EDGE_WAIT_MAX_TICKS) break;
      ++n_wait;
      const uint32_t dirty = take_arrivals(lo, t);
      if (dirty) {
        settle(dirty, lo, t);
        t_last = now;
      } else {
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (edge_missing(f)) wait_credit -= 4;
    else if (wait_credit < WAIT_CREDIT) ++wait_credit;
  };

  // Writes a row leaving the window to HBM; in the first pass unfinished
  // cells get the sentinel so a later pass can tell them apart.
  auto freeze = [&](int f) {
    const int sf = slot(f);
    const uint32_t me = S.st[sf][li];
    pend_rows &= ~(1u << sf);
    if (!owned) return;
    const int64_t i = row_of(f) * nc + c;
    if ((me & S_DONE) && !(me & S_PRIOR)) {
      ++nfin;
      if constexpr (VK == VK_FF) {
        const ff v = S.val[sf][li];
        P.vhi[i] = v.hi;
        P.vlo[i] = v.lo;
        if (RK == RK_MULTI && P.cnt_ff) P.cnt_ff[i] = (uint64_t)((int64_t)v.hi + (int64_t)v.lo);
      } else if constexpr (VK == VK_F64) {
        P.v64[i] = S.val[sf][li];
      }
      if constexpr (CNT) P.cnt[i] = S.cnt[sf][li];
    } else if ((first || P.debug) && !(me & S_DONE)) {
      if constexpr (VK == VK_FF) {
        P.vlo[i] = __uint_as_float(0x7FC00000u);
      } else if constexpr (VK == VK_F64) {
        const uint64_t tag = P.debug ? (((uint64_t)S.miss[sf][li] << 24) | (me & 0xFFFFFFu)) : 0ull;
        P.v64[i] = __longlong_as_double((long long)(0x7FF8000000000000ull | tag));
      } else if constexpr (CNT) {
        P.cnt[i] = ~0ull;
      }
    }
  };

  // Bounded wait for the I/O wavefront to stage rows up to step need - 1.
  auto wait_staged = [&](int need) -> bool {
    for (int it = 0; it < (1 << 24); ++it) {
      if (lds_ld(&S.staged) >= need) return true;
      __builtin_amdgcn_s_sleep(1);
    }
    return false;
  };

  uint64_t tm_stage = 0, tm_pace = 0, tm_settle = 0, tm_freeze = 0, tm_all = 0;  // diagnostics
  const uint64_t tm_begin = diag_now(P);
  for (int t = 0; t < nr && !fail; ++t) {
    lds_st(&S.tcomp, t);
    uint64_t tm0 = diag_now(P);
    if (!wait_staged(t + 2 < nr ? t + 2 : nr)) {
      fail = true;
      break;
    }
    lds_sync();
    uint64_t tm1 = diag_now(P);
    tm_stage += tm1 - tm0;
    tm0 = tm1;
    // Pacing: wait while a neighbour is more than LEAD rows behind.
    if (t > LEAD) {
      for (int it = 0; it < (1 << 24); ++it) {
        bool behind = false;
        for (int sd = 0; sd < 2; ++sd) {
          if (absent[sd]) continue;
          const int nb = lds_ld(&S.nbp[sd]);
          if (nb >= t - 1 - LEAD) continue;
          behind = true;
          if (nb == nb_last[sd]) {
            if (++nb_same[sd] > LEAD_SPIN) absent[sd] = true;
          } else {
            nb_last[sd] = nb;
            nb_same[sd] = 0;
          }
        }
        if (!behind) break;
        ++n_pace;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    tm1 = diag_now(P);
    tm_pace += tm1 - tm0;
    tm0 = tm1;
    const int lo = t - WIN + 1 > 0 ? t - WIN + 1 : 0;
    if (t == 0 && __ballot(!(S.st[slot(0)][li] & S_DONE))) pend_rows |= 1u << slot(0);
    if (t + 1 < nr) {
      const int sn = slot(t + 1);
      pend_rows &= ~(1u << sn);
      if (__ballot(!(S.st[sn][li] & S_DONE))) pend_rows |= 1u << sn;
    }
    const uint32_t dirty = ((t % ARRIVE_EVERY) == 0 ? take_arrivals(lo, t) : 0u) | (1u << slot(t));
    settle(dirty, lo, t);
    tm1 = diag_now(P);
    tm_settle += tm1 - tm0;
    tm0 = tm1;
    if (t - WIN + 1 >= 0) {
      const int f = t - WIN + 1;
      if ((pend_rows >> slot(f)) & 1u) {
        // Deliveries not yet taken may finish this row's cells.
        const uint32_t d2 = take_arrivals(lo, t);
        if (d2) settle(d2, lo, t);
        if ((pend_rows >> slot(f)) & 1u) wait_edges(f, lo, t);
      }
      lds_sync();
      freeze(f);
    }
    if (lane == 0) prog_put(P.progress + strip, t);
    tm1 = diag_now(P);
    tm_freeze += tm1 - tm0;
  }
  tm_all = diag_now(P) - tm_begin;

  // Drain: the last rows wait (bounded) for their side cells, then leave.
  if (!fail) {
    const int t = nr - 1;
    const int lo = t - WIN + 2 > 0 ? t - WIN + 2 : 0;
    const uint32_t d2 = take_arrivals(lo, t);
    if (d2) settle(d2, lo, t);
    for (int f = lo; f <= t; ++f) {
      if ((pend_rows >> slot(f)) & 1u) wait_edges(f, lo, t);
    }
    lds_sync();
    for (int f = lo; f <= t; ++f) freeze(f);
  }
  if (lane == 0) prog_put(P.progress + strip, nr + WIN + LEAD + 2);
  lds_sync();
  if (lane == 0) lds_st(&S.done, 1);
  if (fail && lane == 0 && P.status) atomicCAS(P.status, 0, FR_ERR_HIP);
  uint32_t tot = nfin;
  for (int off = 32; off > 0; off >>= 1) tot += (uint32_t)__shfl_xor((int)tot, off, 64);
  if (lane == 0 && tot) atomicAdd(P.ctr, tot);
  if (lane == 0 && P.debug) {
    atomicAdd(P.ctr + 3, n_wait);
    atomicAdd(P.ctr + 4, n_pace);
    atomicAdd(P.ctr + 5, n_resolve);
    atomicAdd(P.ctr + 6, n_iter);
    // Time in 100 MHz ticks, summed over strips.
    unsigned long long* tm = reinterpret_cast<unsigned long long*>(P.ctr + 8);
    atomicAdd(tm + 0, (unsigned long long)tm_stage);
    atomicAdd(tm + 1, (unsigned long long)tm_pace);
    atomicAdd(tm + 2, (unsigned long long)tm_settle);
    atomicAdd(tm + 3, (unsigned long long)tm_freeze);
    atomicAdd(tm + 4, (unsigned long long)tm_all);
    atomicAdd(tm + 8, (unsigned long long)tm_resolve);
    atomicAdd(tm + 9, (unsigned long long)tm_loop);
  }
  }
  __syncthreads();
}

// One pass; returns at once after the control step stopped the sequence.
template <int RK, int DK, int VK, bool CNT>
__global__ __launch_bounds__(128) void k_ws_pass(WsParams P, const CallCtl* C, int first) {
  __shared__ WsShared<RK, VK, CNT> S;
  if (C->sweep_stop) return;  // uniform
  ws_strip<RK, DK, VK, CNT>(S, P, (int64_t)blockIdx.x, C->sweep_dir, first);
}

// Control step before the first pass (pass < 0) and after each pass: counts
// the cells the pass finished and decides the next pass -- stop when every
// cell is final or a device error was reported, report a cycle when a pass
// finished nothing (a pass always finishes the highest unfinished cell of a
// DAG), open the engine's gate when the budget is spent, otherwise pick the
// direction (after one pass each way, the one whose last pass finished more
// cells) -- and clears the pass counter and progress words for it.
__global__ __launch_bounds__(256) void k_ws_ctl(WsParams P, CallCtl* C, int pass, int fwd, int last) {
  __shared__ int s_run;
  if (threadIdx.x == 0) {
    int run = 0;
    if (pass < 0 && (C->ms_flags & MS_TAKEN)) {
      // The row sweep has served the call: no pass runs.
      C->sweep_stop = 1;
    } else if (pass < 0) {
      // Visit first the rows holding most inputs: forward inputs are donors,
      // upstream of their receivers; adjoint inputs are the receivers.
      const bool flows_up = P.ctr[1] >= P.ctr[2];
      C->sweep_dir = ((fwd != 0) == flows_up) ? -1 : 1;
      C->sweep_remaining = P.nrows * P.ncols;
      C->sweep_fin[0] = 0u;
      C->sweep_fin[1] = 0u;
      C->sweep_stop = 0;
      run = 1;
    } else if (!C->sweep_stop) {
      const uint32_t fin = P.ctr[0];
      const int32_t st = P.status ? *(volatile int32_t*)P.status : 0;
      const int64_t rem = C->sweep_remaining - (int64_t)fin;
      C->sweep_remaining = rem;
      if (rem <= 0 || st != 0) {
        C->sweep_stop = 1;
      } else if (fin == 0) {
        C->sweep_stop = 1;
        if (P.status) atomicCAS(P.status, 0, FR_ERR_NOTDAG);
      } else if (last) {
        C->sweep_stop = 1;
        C->fallback = 1;
      } else {
        int dir = C->sweep_dir;
        C->sweep_fin[dir > 0 ? 1 : 0] = fin;
        const uint32_t up = C->sweep_fin[0], dn = C->sweep_fin[1];
        if (pass == 0 || up == dn) dir = -dir;
        else dir = dn > up ? 1 : -1;
        C->sweep_dir = dir;
        run = 1;
      }
    }
    s_run = run;
  }
  __syncthreads();
  if (!s_run) return;
  if (threadIdx.x == 0) P.ctr[0] = 0u;
  if (P.debug)
    for (int i = threadIdx.x; i < 25; i += blockDim.x) P.ctr[3 + i] = 0u;
  const int64_t ns = (P.ncols + WS_OWN - 1) / WS_OWN;
  for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) P.progress[i] = -1;
}

// Samples rows for the prevailing vertical flow direction: ctr[1] counts
// receivers in the row above (r - 1), ctr[2] in the row below.
template <int RK>
__global__ __launch_bounds__(256) void k_ws_probe(WsParams P, int nsample) {
  const int64_t r = (int64_t)blockIdx.x * P.nrows / nsample;
  uint32_t up = 0, dn = 0;
  for (int64_t c = threadIdx.x; c < P.ncols; c += blockDim.x) {
    const uint32_t code = P.code[r * P.ncols + c];
    if (RK == RK_SINGLE) {
      up += code <= 2u ? 1u : 0u;
      dn += (code >= 5u && code <= 7u) ? 1u : 0u;
    } else {
      up += (uint32_t)__popc(code & 0x07u);
      dn += (uint32_t)__popc(code & 0xE0u);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    up += (uint32_t)__shfl_xor((int)up, off, 64);
    dn += (uint32_t)__shfl_xor((int)dn, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (up) atomicAdd(P.ctr + 1, up);
    if (dn) atomicAdd(P.ctr + 2, dn);
  }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Batched routing: one persistent launch for many tiles.  Work items are the
// tiles' strips in schedule order; a workgroup takes the next item from a
// ticket counter.  For its strip it computes the receivers of its owned
// columns, meets the tile's other strips at a barrier (items of a tile are
// consecutive tickets and a tile has far fewer strips than there are
// workgroups, so every strip of a tile is running before any waits long),
// then runs wavefront-sweep passes, with a barrier after each, until the
// tile is complete.

// Bounded barrier of the strips of one tile: release this workgroup's
// global writes, count in, wait for `target` arrivals, acquire.
__device__ bool tile_barrier(uint32_t* bar, uint32_t target) {
  __threadfence();
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 0;
    atomicAdd(bar, 1u);
    for (int it = 0; it < (1 << 22); ++it) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  __syncthreads();
  __threadfence();
  return ok != 0;
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Receivers of the strip's owned columns, every row; the two wavefronts
// take half of the rows each.  Adds the receivers in the row above / below
// to *up / *dn (prevailing flow direction of the tile).
template <int RULE>
__device__ void batch_receivers(const BatchTileInfo& T, int64_t strip, uint32_t* up, uint32_t* dn,
                                int32_t* status) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nr = T.nrows, nc = T.ncols;
  const int64_t c = strip * WS_OWN - WS_GHOST + lane;
  const bool live = c >= 0 && c < nc;
  const bool owned = live && lane >= WS_GHOST && lane < WS_GHOST + WS_OWN;
  const bool sideL = lane == 0 && c - 1 >= 0 && c - 1 < nc;
  const bool sideR = lane == 63 && c + 1 >= 0 && c + 1 < nc;
  const int64_t cs = lane == 0 ? c - 1 : c + 1;
  const int64_t r0 = wave == 0 ? 0 : nr / 2, r1 = wave == 0 ? nr / 2 : nr;
  struct Z {
    float own, side;
  };
  auto ld = [&](int64_t r) -> Z {
    Z v{INFINITY, INFINITY};
    if (r < 0 || r >= nr) return v;
    if (live) v.own = T.z[r * nc + c];
    if (sideL || sideR) v.side = T.z[r * nc + cs];
    return v;
  };
  uint32_t nu = 0, nd = 0;
  bool nonfinite = false;
  // Rows r-1 .. r+4 in W; the next four rows are loaded one iteration early.
  Z W[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) W[j] = ld(r0 - 1 + j);
  for (int64_t r = r0; r < r1; r += 4) {
    Z N[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) N[j] = ld(r + 5 + j);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const Z& u = W[j];
      const Z& m = W[j + 1];
      const Z& d = W[j + 2];
      float zk[8];
      zk[0] = from_left(u.own);
      zk[1] = u.own;
      zk[2] = from_right(u.own);
      zk[3] = from_left(m.own);
      zk[4] = from_right(m.own);
      zk[5] = from_left(d.own);
      zk[6] = d.own;
      zk[7] = from_right(d.own);
      if (lane == 0) {
        zk[0] = sideL ? u.side : INFINITY;
        zk[3] = sideL ? m.side : INFINITY;
        zk[5] = sideL ? d.side : INFINITY;
      }
      if (lane == 63) {
        zk[2] = sideR ? u.side : INFINITY;
        zk[4] = sideR ? m.side : INFINITY;
        zk[7] = sideR ? d.side : INFINITY;
      }
      const uint8_t code = route_code<RULE>(m.own, zk);
      if (owned && r + j < r1 && !isfinite(m.own)) nonfinite = true;
      if (owned && r + j < r1) {
        T.code[(r + j) * nc + c] = code;
        if (RULE == FR_MFD) {
          nu += (uint32_t)__popc(code & 0x07u);
          nd += (uint32_t)__popc(code & 0xE0u);
        } else {
          nu += code <= 2u ? 1u : 0u;
          nd += (code >= 5u && code <= 7u) ? 1u : 0u;
        }
      }
    }
    W[0] = W[4];
    W[1] = W[5];
#pragma unroll
    for (int j = 0; j < 4; ++j) W[2 + j] = N[j];
  }
  for (int off = 32; off > 0; off >>= 1) {
    nu += (uint32_t)__shfl_xor((int)nu, off, 64);
    nd += (uint32_t)__shfl_xor((int)nd, off, 64);
  }
  if (lane == 0) {
    if (nu) atomicAdd(up, nu);
    if (nd) atomicAdd(dn, nd);
  }
  if (__ballot(nonfinite) && lane == 0 && status) atomicCAS(status, 0, FR_ERR_NONFINITE);
}

// Receivers of one strip for any rule.  Kept out of line: it runs once per
// work item and touches no LDS, and inlining it into the router would
// crowd the sweep's registers.
__device__ __attribute__((noinline)) void batch_receivers_any(const BatchTileInfo* Tp, int64_t strip,
                                                              int32_t* status) {
  const BatchTileInfo& T = *Tp;
  if (T.rule == FR_MFD) batch_receivers<FR_MFD>(T, strip, T.ctr + BCTR_UP, T.ctr + BCTR_DN, status);
  else if (T.rule == FR_D4) batch_receivers<FR_D4>(T, strip, T.ctr + BCTR_UP, T.ctr + BCTR_DN, status);
  else batch_receivers<FR_D8>(T, strip, T.ctr + BCTR_UP, T.ctr + BCTR_DN, status);
}

// Bytes of LDS the persistent kernel reserves: the largest sweep variant.
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t BATCH_LDS = sizeof(WsShared<RK_MULTI, VK_FF, false>);

struct BatchParams {
  BatchHeader* hdr;
  const BatchTileInfo* info;
  const int32_t* sched;
  const int64_t* base;
  int32_t* status;
};

template <int RK, int VK, bool CNT>
__device__ __forceinline__ void batch_sweep(unsigned char* lds, const WsParams& P, int64_t strip, int dir,
                                            int first) {
  ws_strip<RK, DIR_FWD, VK, CNT>(*reinterpret_cast<WsShared<RK, VK, CNT>*>(lds), P, strip, dir, first);
}

__global__ __launch_bounds__(128) void k_batch(BatchParams B) {
  __shared__ __align__(16) unsigned char lds[BATCH_LDS];
  __shared__ long long item_sh;
  const int64_t total = B.hdr->total_items;
  const int ntiles = B.hdr->ntiles;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (long long)atomicAdd(&B.hdr->ticket, 1ull);
    __syncthreads();
    // Uniform across the workgroup: keep it (and all tile data) in scalars.
    const uint64_t iu = (uint64_t)item_sh;
    const int64_t item = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(iu >> 32)) << 32) |
                                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)iu));
    __syncthreads();
    if (item >= total) break;
    // Schedule position k with base[k] <= item < base[k + 1].
    int lo = 0, hi = ntiles - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.base[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const BatchTileInfo* Tp = B.info + B.sched[lo];
    const BatchTileInfo T = *Tp;
    const int64_t strip = item - B.base[lo];
    const uint32_t ns = (uint32_t)T.nstrips;
    if (ns > gridDim.x) {
      // The tile's strips could never all run at once on this many workers.
      if (threadIdx.x == 0 && B.status && strip == 0) atomicCAS(B.status, 0, FR_ERR_ARG);
      continue;
    }
    batch_receivers_any(Tp, strip, B.status);
    if (!tile_barrier(T.ctr + BCTR_BAR, ns)) {
      if (threadIdx.x == 0 && B.status) atomicCAS(B.status, 0, FR_ERR_HIP);
      continue;
    }
    // Forward inputs are donors: visit first the rows water comes from.
    int dir = ld_agent(T.ctr + BCTR_UP) >= ld_agent(T.ctr + BCTR_DN) ? -1 : 1;
    const int64_t ncell = T.nrows * T.ncols;
    int64_t done = 0;
    bool complete = false;
    uint32_t fin_up = 0, fin_dn = 0;  // cells finished by the last pass each way
    for (int pass = 0; pass < BATCH_MAXPASS; ++pass) {
      WsParams P{};
      P.nrows = T.nrows;
      P.ncols = T.ncols;
      P.code = T.code;
      P.z = T.z;
      P.p = 1.1;
      P.src32 = T.rule == FR_MFD || T.q ? T.rain : nullptr;
      P.src64 = nullptr;
      P.vhi = T.q ? T.q : T.vhi;
      P.vlo = T.vlo;
      P.v64 = nullptr;
      P.cnt = nullptr;
      P.codes_single = T.rule != FR_MFD;
      P.cnt_ff = T.cnt;
      P.edge = T.edge;
      P.progress = T.progress + (int64_t)pass * T.nstrips;
      P.ctr = T.ctr + pass;
      P.status = B.status;
      P.debug = 0;
      const int first = pass == 0 ? 1 : 0;
      // Every tile runs the MFD float-float variant; a D8/D4 code is a
      // one-bit mask whose fraction is exactly 1, and counts are the
      // float-float values of unit rain, exact integers below 2^31.
      batch_sweep<RK_MULTI, VK_FF, false>(lds, P, strip, dir, first);
      if (!tile_barrier(T.ctr + BCTR_BAR, (uint32_t)(2 + pass) * ns)) {
        if (threadIdx.x == 0 && B.status) atomicCAS(B.status, 0, FR_ERR_HIP);
        break;
      }
      const uint32_t fin = ld_agent(T.ctr + pass);
      done += fin;
      if (done >= ncell) {
        complete = true;
        break;
      }
      if (fin == 0) break;
      // After one pass each way, repeat the direction whose last pass
      // finished more (either direction finishes the highest unfinished cell).
      if (dir > 0) fin_dn = fin;
      else fin_up = fin;
      if (pass == 0 || fin_up == fin_dn) dir = -dir;
      else dir = fin_dn > fin_up ? 1 : -1;
    }
    // A pass that finished nothing, or too many passes: a cycle (or a tile
    // the sweep cannot finish, reported the same way).
    if (!complete && threadIdx.x == 0 && B.status && strip == 0) atomicCAS(B.status, 0, FR_ERR_NOTDAG);
  }
}

// Set-up (one workgroup): tile records, schedule and work-item bases.
__global__ __launch_bounds__(1024) void k_batch_setup(const fr_tile* tiles, int32_t ntiles, int order,
                                                     char* ws, size_t ws_bytes, int32_t* status) {
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(ws);
  char* p = ws + ws_align(sizeof(BatchHeader));
  BatchTileInfo* info = reinterpret_cast<BatchTileInfo*>(p);
  p += ws_align((size_t)ntiles * sizeof(BatchTileInfo));
  int32_t* sched = reinterpret_cast<int32_t*>(p);
  p += ws_align((size_t)ntiles * 4);
  int64_t* base = reinterpret_cast<int64_t*>(p);
  // Schedule: given order, or more rows (cells) first, stable, by parallel
  // ranking.
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
    int rank = i;
    if (order != FR_ORDER_GIVEN && ntiles <= 16384) {
      rank = 0;
      const bool rows = order == FR_ORDER_ROWS_DESC;
      const int64_t ki = rows ? tiles[i].nrows : tiles[i].nrows * tiles[i].ncols;
      for (int j = 0; j < ntiles; ++j) {
        const int64_t kj = rows ? tiles[j].nrows : tiles[j].nrows * tiles[j].ncols;
        rank += (kj > ki || (kj == ki && j < i)) ? 1 : 0;
      }
    }
    sched[rank] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    size_t off = batch_head_bytes(ntiles);
    bool bad = false;
    for (int i = 0; i < ntiles; ++i) {
      const fr_tile& t = tiles[i];
      const bool has_q = t.q_out != nullptr;
      const BatchTileLayout L = batch_tile_layout(t.nrows, t.ncols, t.code_out == nullptr, batch_tile_ff(t.rule, has_q));
      BatchTileInfo I{};
      I.z = t.z;
      I.rain = t.rain;
      I.q = t.q_out;
      I.cnt = t.rule == FR_MFD ? nullptr : t.counts_out;
      if (t.rule != FR_MFD && t.q_out) I.cnt = nullptr;
      I.code = t.code_out ? t.code_out : reinterpret_cast<uint8_t*>(ws + off + L.code);
      I.vhi = reinterpret_cast<float*>(ws + off + L.vhi);
      I.vlo = reinterpret_cast<float*>(ws + off + L.vlo);
      I.edge = reinterpret_cast<uint64_t*>(ws + off + L.edge);
      I.progress = reinterpret_cast<int32_t*>(ws + off + L.progress);
      I.ctr = reinterpret_cast<uint32_t*>(ws + off + L.ctr);
      I.nrows = t.nrows;
      I.ncols = t.ncols;
      I.nstrips = (int32_t)ws_strip_count(t.ncols);
      I.rule = t.rule;
      if (t.nrows < 1 || t.ncols < 1 || !t.z || (t.rule == FR_MFD && !t.q_out) ||
          (t.rule != FR_MFD && (t.q_out != nullptr) == (t.counts_out != nullptr)))
        bad = true;
      info[i] = I;
      off += L.total;
    }
    int64_t item = 0;
    for (int k = 0; k < ntiles; ++k) {
      base[k] = item;
      info[sched[k]].strip_base = item;
      item += info[sched[k]].nstrips;
    }
    base[ntiles] = item;
    hdr->ticket = 0ull;
    hdr->ntiles = ntiles;
    hdr->order = order;
    hdr->ws_needed = (int64_t)off;
    const bool fits = off <= ws_bytes && !bad;
    hdr->total_items = fits ? item : 0;
    if (!fits && status) atomicCAS(status, 0, bad ? FR_ERR_ARG : FR_ERR_WORKSPACE);
  }
}

// Fills each tile's edge records (empty), progress (-1) and counters (0).
__global__ __launch_bounds__(256) void k_batch_fill(const BatchHeader* hdr, const BatchTileInfo* info) {
  if (hdr->total_items == 0) return;
  const BatchTileInfo& T = info[blockIdx.x];
  const int64_t ne = (int64_t)T.nstrips * T.nrows * 2 * WS_EW;
  for (int64_t i = threadIdx.x; i < ne; i += blockDim.x) T.edge[i] = REC_EMPTY;
  for (int64_t i = threadIdx.x; i < (int64_t)T.nstrips * BATCH_MAXPASS; i += blockDim.x) T.progress[i] = -1;
  for (int i = threadIdx.x; i < BATCH_CTR_WORDS; i += blockDim.x) T.ctr[i] = 0u;
}

template <int RK, int DK, int VK, bool CNT>
hipError_t pass_t(const WsParams& P, const CallCtl* C, int first, hipStream_t s) {
  const unsigned strips = (unsigned)((P.ncols + WS_OWN - 1) / WS_OWN);
  hipLaunchKernelGGL((k_ws_pass<RK, DK, VK, CNT>), dim3(strips), dim3(128), 0, s, P, C, first);
  return hipGetLastError();
}

}  // namespace

int64_t ws_strips(int64_t ncols) { return (ncols + WS_OWN - 1) / WS_OWN; }

size_t ws_edge_words(int64_t nrows, int64_t ncols) {
  return (size_t)((ncols + WS_OWN - 1) / WS_OWN) * (size_t)nrows * 2 * WS_EW;
}

hipError_t launch_ws_setup(const EngineConfig& cfg, const WsParams& P, CallCtl* C, hipStream_t s) {
  const int64_t n = (int64_t)ws_edge_words(P.nrows, P.ncols);
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P.edge, n, REC_EMPTY);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(P.ctr), (int64_t)2, 0ull);
  const int ns = P.nrows < 64 ? (int)P.nrows : 64;
  if (cfg.rk == RK_SINGLE)
    hipLaunchKernelGGL(k_ws_probe<RK_SINGLE>, dim3(ns), dim3(256), 0, s, P, ns);
  else
    hipLaunchKernelGGL(k_ws_probe<RK_MULTI>, dim3(ns), dim3(256), 0, s, P, ns);
  hipLaunchKernelGGL(k_ws_ctl, dim3(1), dim3(256), 0, s, P, C, -1, cfg.dir == DIR_FWD ? 1 : 0, 0);
  return hipGetLastError();
}

hipError_t launch_ws_ctl(const WsParams& P, CallCtl* C, int pass, bool last, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_ctl, dim3(1), dim3(256), 0, s, P, C, pass, 0, last ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ws_pass(const EngineConfig& cfg, const WsParams& P, const CallCtl* C, int first, hipStream_t s) {
  if (cfg.dir == DIR_FWD) {
    if (cfg.rk == RK_MULTI) {
      if (cfg.vk == VK_F64) return pass_t<RK_MULTI, DIR_FWD, VK_F64, false>(P, C, first, s);
      return pass_t<RK_MULTI, DIR_FWD, VK_FF, false>(P, C, first, s);
    }
    if (cfg.counts) {
      if (cfg.vk == VK_FF) return pass_t<RK_SINGLE, DIR_FWD, VK_FF, true>(P, C, first, s);
      if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_FWD, VK_F64, true>(P, C, first, s);
      return pass_t<RK_SINGLE, DIR_FWD, VK_NONE, true>(P, C, first, s);
    }
    if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_FWD, VK_F64, false>(P, C, first, s);
    return pass_t<RK_SINGLE, DIR_FWD, VK_FF, false>(P, C, first, s);
  }
  if (cfg.rk == RK_MULTI) {
    if (cfg.vk == VK_F64) return pass_t<RK_MULTI, DIR_ADJ, VK_F64, false>(P, C, first, s);
    return pass_t<RK_MULTI, DIR_ADJ, VK_FF, false>(P, C, first, s);
  }
  if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_ADJ, VK_F64, false>(P, C, first, s);
  return pass_t<RK_SINGLE, DIR_ADJ, VK_FF, false>(P, C, first, s);
}

hipError_t launch_batch(const void* tiles_dev, int32_t ntiles, int order, int workers, int32_t* status,
                        char* ws, size_t ws_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_setup, dim3(1), dim3(1024), 0, s, static_cast<const fr_tile*>(tiles_dev), ntiles,
                     order, ws, ws_bytes, status);
  char* p = ws + ws_align(sizeof(BatchHeader));
  const BatchTileInfo* info = reinterpret_cast<const BatchTileInfo*>(p);
  p += ws_align((size_t)ntiles * sizeof(BatchTileInfo));
  const int32_t* sched = reinterpret_cast<const int32_t*>(p);
  p += ws_align((size_t)ntiles * 4);
  const int64_t* base = reinterpret_cast<const int64_t*>(p);
  hipLaunchKernelGGL(k_batch_fill, dim3((unsigned)ntiles), dim3(256), 0, s,
                     reinterpret_cast<const BatchHeader*>(ws), info);
  BatchParams B{reinterpret_cast<BatchHeader*>(ws), info, sched, base, status};
  hipLaunchKernelGGL(k_batch, dim3((unsigned)workers), dim3(128), 0, s, B);
  return hipGetLastError();
}

}  // namespace fr
