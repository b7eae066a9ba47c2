// Row sweep for routing with several receivers per cell (MFD masks), forward
// (I - W^T) q = r or adjoint (I - W) rbar = qbar (Section 2.1, Section 2.2;
// the fractions as in Appendix A).
//
// Any order that puts every cell after all cells feeding it solves the
// system in one pass (Section 3.2).  When no cell sends water into the row
// before it in some fixed row order -- terrain that drains along the row
// axis -- visiting rows in that order is such an order, except for flow
// between neighbours of the same row.  A cell then depends only on three
// cells of the previous row and on chains of same-row neighbours, so the
// grid is solved row by row: every column of a row at once.
//
// GPU mapping.  One wavefront owns a strip of MS_OWN columns and computes a
// window of 64 columns, lane = column: the owned columns and MS_G columns of
// each neighbouring strip ("ghost" columns), recomputed from the same
// inputs.  A row step pulls the previous row's values of the three upslope
// neighbours through lane shifts (DPP), then resolves same-row chains by
// repeated lane-shifted pulls until no value changes (chains on this kind of
// terrain are a few cells long).  No value leaves the wavefront except the
// owned results.
//
// Ghost columns cannot see beyond the window: the two edge columns never
// know all of their inputs, and what they compute spreads inward along the
// flow (about two columns per row).  Every lane carries a "dirty" bit for
// values that may depend on such an unknown (two 64-bit masks, one per
// side, updated with the same shifts along the same edges).  As long as no
// owned column is dirty, the row is exact.  When the dirt reaches an owned
// column, the strip refreshes that side's ghost columns from the values the
// neighbouring strip published for the previous row, and recomputes the
// row; if a same-row chain still carries dirt in from beyond the window, it
// takes the neighbour's values of the current row for those ghost columns.
// A chain crossing a strip edge runs one way across it, so two strips never
// wait for each other's current row; a strip waits only for rows its
// neighbours have finished or are finishing, and the least advanced strip
// never waits, so every wait ends.
//
// Every strip publishes its owned results of each row in a ring of MS_RING
// rows in HBM, as 64-bit words whose low 8 bits carry the row number
// (device-scope stores and loads, no fences): a reader polls until the tags
// match.  A strip does not overwrite a ring slot before both neighbours have
// passed the row it holds.
//
// The pass applies only when the codes admit it: a check before it reads
// every code and elevation and takes the pass only if the masks are valid
// (receivers strictly lower, on the grid, elevations finite) and no cell
// sends to the row before it in one of the two row orders.  Otherwise the
// general wavefront sweep runs instead.  Results are exact up to rounding
// and do not depend on timing: which ghost columns are refreshed, and with
// what, depends only on the data.
//
// Precision: float-float accumulation for float32 output (hi written; the
// low part stays in registers), float64 otherwise; fractions as in the
// general sweep (float32 (s / s_max)^p with a conservation correction, or
// float64 pow).
#include <math.h>

#include "fr_ff.hpp"
#include "fr_internal.hpp"

namespace fr {
namespace {

using ffa::ff;

constexpr int MS_LANES = 64;
constexpr uint64_t MS_EMPTY = ~0ull;
// Polls of a ring word or progress word before a wait gives up (each poll
// sleeps about 64 clocks): far beyond any legitimate wait.
constexpr uint32_t MS_SPIN_LIMIT = 1u << 20;
constexpr uint64_t kGhostL = (1ull << MS_G) - 1ull;
constexpr uint64_t kGhostR = ~0ull << (MS_G + MS_OWN);
constexpr uint64_t kOwn = ~(kGhostL | kGhostR);

__device__ constexpr float kInvSqrt2f = 0x1.6a09e6p-1f;
__device__ constexpr double kSqrt2 = 1.4142135623730950488;

// Lane shifts across the whole wavefront (DPP wave_shr:1 / wave_shl:1); the
// lane shifted in reads 0 (bound_ctrl).
__device__ __forceinline__ uint32_t sh_l(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t sh_r(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float sh_l(float x) { return __uint_as_float(sh_l(__float_as_uint(x))); }
__device__ __forceinline__ float sh_r(float x) { return __uint_as_float(sh_r(__float_as_uint(x))); }
__device__ __forceinline__ double sh_l(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return __longlong_as_double((long long)(((uint64_t)sh_l((uint32_t)(u >> 32)) << 32) | sh_l((uint32_t)u)));
}
__device__ __forceinline__ double sh_r(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return __longlong_as_double((long long)(((uint64_t)sh_r((uint32_t)(u >> 32)) << 32) | sh_r((uint32_t)u)));
}
__device__ __forceinline__ ff sh_l(ff x) { return {sh_l(x.hi), sh_l(x.lo)}; }
__device__ __forceinline__ ff sh_r(ff x) { return {sh_r(x.hi), sh_r(x.lo)}; }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__builtin_amdgcn_ballot_w64(p); }

// Value arithmetic of the two precisions.
template <int VK>
struct Arith;

template <>
struct Arith<VK_FF> {
  using V = ff;
  using F = float;
  static __device__ __forceinline__ V zero() { return {0.0f, 0.0f}; }
  static __device__ __forceinline__ V one() { return {1.0f, 0.0f}; }
  static __device__ __forceinline__ V from_src(float r) { return {r, 0.0f}; }
  static __device__ __forceinline__ V from_src(double r) {
    const float h = (float)r;
    return {h, (float)(r - (double)h)};
  }
  static __device__ __forceinline__ V add(V a, V b) { return ffa::add(a, b); }
  static __device__ __forceinline__ V contrib(V v, F f, float d) { return ffa::mul_fd(v, f, d); }
  static __device__ __forceinline__ bool nz(V v) { return v.hi != 0.0f; }
  // Unnormalised variants for inner loops (|lo| may exceed ulp(hi)/2 by a
  // few units; the sum is renormalised once at the end): x * f * (1 + d),
  // and a + b.
  static __device__ __forceinline__ V contrib_lean(V x, F f, float d) {
    const float p = x.hi * f;
    float e = fmaf(x.hi, f, -p);
    e = fmaf(x.lo, f, e);
    return {p, fmaf(p, d, e)};
  }
  static __device__ __forceinline__ V add_lean(V a, V b) {
    const ff s = ffa::two_sum(a.hi, b.hi);
    return {s.hi, s.lo + (a.lo + b.lo)};
  }
  static __device__ __forceinline__ V norm(V v) { return ffa::fast_two_sum(v.hi, v.lo); }
  // Either part nonzero (signs ignored).
  static __device__ __forceinline__ bool nz_any(V v) {
    return ((__float_as_uint(v.hi) | __float_as_uint(v.lo)) << 1) != 0u;
  }
  static __device__ __forceinline__ bool finite(V v) { return isfinite(v.hi) && isfinite(v.lo); }
  static __device__ __forceinline__ double wide(V v) { return (double)v.hi + (double)v.lo; }
  // The low part's last 8 bits carry the tag (a change of at most 2^-40 of
  // the value).
  static __device__ __forceinline__ uint64_t pack(V v, uint32_t tag) {
    return ((uint64_t)__float_as_uint(v.hi) << 32) | ((__float_as_uint(v.lo) & ~0xFFu) | tag);
  }
  static __device__ __forceinline__ V unpack(uint64_t w) {
    return {__uint_as_float((uint32_t)(w >> 32)), __uint_as_float((uint32_t)w & ~0xFFu)};
  }
};

template <>
struct Arith<VK_F64> {
  using V = double;
  using F = double;
  static __device__ __forceinline__ V zero() { return 0.0; }
  static __device__ __forceinline__ V one() { return 1.0; }
  static __device__ __forceinline__ V from_src(float r) { return (double)r; }
  static __device__ __forceinline__ V from_src(double r) { return r; }
  static __device__ __forceinline__ V add(V a, V b) { return a + b; }
  static __device__ __forceinline__ V contrib(V v, F f, float) { return v * f; }
  static __device__ __forceinline__ bool nz(V v) { return v != 0.0; }
  static __device__ __forceinline__ V contrib_lean(V x, F f, float) { return x * f; }
  static __device__ __forceinline__ V add_lean(V a, V b) { return a + b; }
  static __device__ __forceinline__ V norm(V v) { return v; }
  static __device__ __forceinline__ bool nz_any(V v) { return v != 0.0; }
  static __device__ __forceinline__ bool finite(V v) { return isfinite(v); }
  static __device__ __forceinline__ double wide(V v) { return v; }
  // The last 8 bits of the significand carry the tag (2^-45 relative).
  static __device__ __forceinline__ uint64_t pack(V v, uint32_t tag) {
    return ((uint64_t)__double_as_longlong(v) & ~0xFFull) | tag;
  }
  static __device__ __forceinline__ V unpack(uint64_t w) {
    return __longlong_as_double((long long)(w & ~0xFFull));
  }
};

__device__ __forceinline__ void st_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_word(const uint64_t* p) {
  return (uint64_t)__hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p)),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_i32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_i32(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fractions of one cell toward its receivers among five candidates, in
// ascending direction order: the three cells of the receiving row (dc = -1,
// 0, +1) and the two same-row neighbours.  FLOW_UP: the receiving row is
// r - 1 (directions 0, 1, 2, then 3, 4); otherwise r + 1 (3, 4, then 5, 6,
// 7).  The arithmetic and its order are those of the general sweep.
template <int VK, bool FLOW_UP>
struct Frac {
  typename Arith<VK>::F nm, n0, np, l, r;  // toward next-row dc -1, 0, +1; left; right
  float d;                                 // conservation correction (float32 mode)
};

template <int VK, bool FLOW_UP>
__device__ __forceinline__ Frac<VK, FLOW_UP> fractions(float zc, float znm, float zn0, float znp, float zl,
                                                       float zr, uint32_t rcv, float pf, double p) {
  // rcv bit j: candidate j (order nm, n0, np, l, r) receives.
  Frac<VK, FLOW_UP> out;
  out.d = 0.0f;
  const float zz[5] = {znm, zn0, znp, zl, zr};
  const bool dg[5] = {true, false, true, false, false};
  // Direction order: FLOW_UP 0,1,2 (next row), 3, 4; else 3, 4, 5,6,7.
  constexpr int ord[5] = {FLOW_UP ? 0 : 3, FLOW_UP ? 1 : 4, FLOW_UP ? 2 : 0, FLOW_UP ? 3 : 1, FLOW_UP ? 4 : 2};
  if constexpr (VK == VK_F64) {
    // w_j = (s_j / s_max)^p = 2^(p log2(s_j / s_max)): the common factor
    // s_max^p cancels in the fractions, and the exponent stays small (a few
    // 1e-16 relative, far cheaper than a general power).
    double sl[5], smax = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      sl[j] = 0.0;
      if ((rcv >> j) & 1u) {
        sl[j] = ((double)zc - (double)zz[j]) / (dg[j] ? kSqrt2 : 1.0);
        smax = sl[j] > smax ? sl[j] : smax;
      }
    }
    const double ism = smax > 0.0 ? 1.0 / smax : 0.0;
    double w[5], sum = 0.0;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int j = ord[o];
      w[j] = ((rcv >> j) & 1u) ? exp2(p * log2(sl[j] * ism)) : 0.0;
      sum += w[j];
    }
    const double iw = sum > 0.0 ? 1.0 / sum : 0.0;
    out.nm = w[0] * iw;
    out.n0 = w[1] * iw;
    out.np = w[2] * iw;
    out.l = w[3] * iw;
    out.r = w[4] * iw;
  } else {
    // Branch-free: t_j = 2^(p log2(s_j / s_max)) with the hardware log2 and
    // exp2 (about 1 ulp each; the ratio is held above the float32 normal
    // range, where t_j is negligible anyway), f_j = t_j / sum t.
    float sl[5], smax = 0.0f;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const float drop = zc - zz[j];
      const float sj = dg[j] ? drop * kInvSqrt2f : drop;
      sl[j] = ((rcv >> j) & 1u) ? sj : 0.0f;
      smax = fmaxf(smax, sl[j]);
    }
    const float ism = smax > 0.0f ? __builtin_amdgcn_rcpf(smax) : 0.0f;
    float tk[5], sum = 0.0f;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int j = ord[o];
      const float r = fmaxf(sl[j] * ism, 0x1p-126f);
      tk[j] = ((rcv >> j) & 1u) ? __builtin_amdgcn_exp2f(pf * __builtin_amdgcn_logf(r)) : 0.0f;
      sum += tk[j];
    }
    const float isum = sum > 0.0f ? __builtin_amdgcn_rcpf(sum) : 0.0f;
    float f[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) f[j] = tk[j] * isum;
    // Rounded fractions do not sum to 1 exactly; over thousands of cells
    // along a flow path the excess would compound.  With the exact sum s
    // (float-float), d = -(s - 1) restores it to first order.
    ff es = {0.0f, 0.0f};
#pragma unroll
    for (int o = 0; o < 5; ++o) es = ffa::add(es, ff{f[ord[o]], 0.0f});
    out.d = sum > 0.0f ? -((es.hi - 1.0f) + es.lo) : 0.0f;
    out.nm = f[0];
    out.n0 = f[1];
    out.np = f[2];
    out.l = f[3];
    out.r = f[4];
  }
  return out;
}

// Resolves same-row chains: q = a + sum over same-row inputs of their
// contributions, by pulls repeated until no increment is left (exact: an
// increment travels one cell per pull and chains end).  fin_l / fin_r:
// fraction of the left / right neighbour's value this cell takes (0: no
// such input), with the sender's correction din_l / din_r.
template <int VK>
__device__ __forceinline__ typename Arith<VK>::V lateral(typename Arith<VK>::V a, typename Arith<VK>::F fin_l,
                                                        float din_l, typename Arith<VK>::F fin_r, float din_r) {
  using A = Arith<VK>;
  using V = typename A::V;
  V q = a, d0 = a, d1;
  // Two pulls per trip (ping-pong increments, no register copies); an
  // increment moves one cell per pull, so 64 pulls cross any window.
  for (int it = 0; it < MS_LANES / 2; ++it) {
    d1 = A::add_lean(A::contrib_lean(sh_l(d0), fin_l, din_l), A::contrib_lean(sh_r(d0), fin_r, din_r));
    if (ballot(A::nz_any(d1)) == 0ull) break;
    q = A::add_lean(q, d1);
    d0 = A::add_lean(A::contrib_lean(sh_l(d1), fin_l, din_l), A::contrib_lean(sh_r(d1), fin_r, din_r));
    if (ballot(A::nz_any(d0)) == 0ull) break;
    q = A::add_lean(q, d0);
  }
  return A::norm(q);
}

// Dirt carried along same-row chains (hl / hr: lanes taking input from the
// left / right).
__device__ __forceinline__ uint64_t spread(uint64_t d, uint64_t hl, uint64_t hr) {
  for (int it = 0; it < MS_LANES; ++it) {
    const uint64_t n = d | ((d << 1) & hl) | ((d >> 1) & hr);
    if (n == d) break;
    d = n;
  }
  return d;
}

// Polls until every lane in `need` reads a word tagged `tag` at its address;
// returns false after the spin limit (the status word then says so).
template <int VK>
__device__ __forceinline__ bool wait_words(const uint64_t* addr, bool need, uint32_t tag,
                                           typename Arith<VK>::V& out) {
  for (uint32_t it = 0;; ++it) {
    uint64_t w = 0;
    if (need) w = ld_word(addr);
    const bool ok = !need || (uint32_t)(w & 0xFFu) == tag;
    if (need && ok) out = Arith<VK>::unpack(w);
    if (ballot(!ok) == 0ull) return true;
    if (it >= MS_SPIN_LIMIT) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

__device__ __forceinline__ bool wait_progress(const int32_t* p, int32_t target) {
  for (uint32_t it = 0;; ++it) {
    if (ld_i32(p) >= target) return true;
    if (it >= MS_SPIN_LIMIT) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Kinds of source term (rain, or qbar for the adjoint).
enum SrcKind { SRC_UNIT = 0, SRC_F32 = 1, SRC_F64 = 2 };
template <int SRC>
struct SrcT {
  using T = float;
};
template <>
struct SrcT<SRC_F64> {
  using T = double;
};

// Inputs of one row step, loaded two steps ahead: the code and source of
// row y(t), and the elevation the step needs next (forward: row y(t + 1),
// the receiving row; adjoint: row y(t)).
template <int SRC>
struct RowIn {
  float z;
  uint32_t code;
  typename SrcT<SRC>::T src;
};

// One wavefront per strip.  FLOW_UP: receivers lie in row r - 1 (forward
// sweep visits rows from the last to the first); else in row r + 1.  ADJ:
// the adjoint, visiting rows the other way and pulling from receivers.
//
// Every global load and store of a row step is issued by every lane (loads
// of columns or rows off the grid read a clamped address and are
// discarded; stores of lanes that own no column go to a scratch slot), so
// the compiler can count outstanding memory operations exactly and a step
// never waits for the loads it issued for a later row.
template <int VK, bool ADJ, bool FLOW_UP, int SRC>
__global__ __launch_bounds__(64) void k_ms(MsParams P, const CallCtl* C) {
  using A = Arith<VK>;
  using V = typename A::V;
  using F = typename A::F;
  using In = RowIn<SRC>;
  const int32_t gate = C->ms_flags;
  if (!(gate & MS_TAKEN) || ((gate & MS_FLOW_UP) != 0) != FLOW_UP) return;

  const int lane = (int)threadIdx.x;
  const int s = (int)blockIdx.x;
  const int64_t nr = P.nrows, nc = P.ncols;
  const int64_t col = (int64_t)s * MS_OWN - MS_G + lane;
  const bool valid = col >= 0 && col < nc;
  const bool owned = valid && lane >= MS_G && lane < MS_G + MS_OWN;
  const uint64_t vmask = ballot(valid);
  const uint64_t own_mask = kOwn & vmask;
  // Edge lanes with a grid column beyond the window: never exact by
  // themselves.
  const int64_t col0 = (int64_t)s * MS_OWN - MS_G;
  const uint64_t edge_l = (col0 >= 1 && col0 < nc) ? 1ull : 0ull;
  const uint64_t edge_r = (col0 + 63 >= 0 && col0 + 64 < nc) ? (1ull << 63) : 0ull;
  // Strips whose owned columns are ghost columns here (MS_NB on each side).
  const int nb_lo = s - MS_NB < 0 ? 0 : s - MS_NB;
  const int nb_hi = s + MS_NB > P.nstrips - 1 ? P.nstrips - 1 : s + MS_NB;
  // Rows in visiting order: step t visits row y(t).
  const bool rows_down = ADJ ? FLOW_UP : !FLOW_UP;  // true: y = t
  auto row_of = [&](int64_t t) { return rows_down ? t : nr - 1 - t; };
  const int64_t ccol = valid ? col : 0;
  const float pf = (float)P.p;

  // Window-edge lanes do not see the column beyond: that candidate is
  // dropped from their masks (their fractions are then wrong, and their
  // values dirty anyway).
  uint32_t drop_mask = 0;
  if (lane == 0) drop_mask |= (1u << 0) | (1u << 3);   // nm, l
  if (lane == 63) drop_mask |= (1u << 2) | (1u << 4);  // np, r
  // Direction bits of the candidates (nm, n0, np, l, r).
  constexpr int kn0 = FLOW_UP ? 0 : 5;
  auto cand = [&](uint32_t code) -> uint32_t {
    uint32_t m = ((code >> kn0) & 7u) | (((code >> 3) & 3u) << 3);
    return valid ? (m & ~drop_mask) : 0u;
  };

  // Ring words: a ghost lane reads the owner of its column.
  uint64_t* ring_mine = P.ring + (size_t)s * MS_RING * MS_OWN;
  const bool ghost_l = lane < MS_G, ghost_r = lane >= MS_G + MS_OWN;
  const int64_t owner = valid ? col / MS_OWN : 0;
  const uint64_t* ring_ghost = P.ring + (size_t)owner * MS_RING * MS_OWN + (size_t)(ccol - owner * MS_OWN);
  int32_t nb_prog = 0;  // smallest neighbour progress seen (rows finished)
  // Store addresses: owned lanes write their cell and ring word, the others
  // a scratch slot of this strip.
  uint64_t* junk = P.junk + (size_t)s * 2 * MS_LANES + lane;
  uint64_t* pub = owned ? ring_mine + (lane - MS_G) : junk + MS_LANES;

  // Previous row state.
  V vp = A::zero();
  F fpm = 0, fp0 = 0, fpp = 0;  // forward: the previous cell's fractions toward this row
  float dp = 0.0f;
  uint64_t dpl = 0, dpr = 0;           // dirt of the previous row's values, by side of origin
  uint64_t spm = 0, sp0 = 0, spp = 0;  // forward: previous-row lanes sending dc -1, 0, +1
  float z_keep = 0.0f;                 // forward: z of this row; adjoint: z of the previous row

  double msum = 0.0, rsum = 0.0;
  bool nonfinite = false, stalled = false;

  auto load_in = [&](int64_t t) -> In {
    In in;
    const int64_t tc = t < nr ? t : nr - 1;
    const int64_t i = row_of(tc) * nc + ccol;
    in.code = P.code[i];
    if constexpr (SRC == SRC_F32) in.src = P.src32[i];
    else if constexpr (SRC == SRC_F64) in.src = P.src64[i];
    else in.src = 0;
    const int64_t tz = ADJ ? tc : (t + 1 < nr ? t + 1 : nr - 1);
    in.z = P.z[row_of(tz) * nc + ccol];
    return in;
  };

  // One row step; false when a wait gave up.
  auto step = [&](int64_t t, In& in) -> bool {
    const int64_t y = row_of(t);
    const int64_t i = y * nc + ccol;
    // This step's inputs (loaded two steps ago); the loads for the step
    // after next are issued at once, so the row's work hides their latency.
    const In cur = in;
    in = load_in(t + 2);
    const uint32_t code = cur.code;
    V srcv;
    if constexpr (SRC == SRC_UNIT) srcv = A::one();
    else srcv = A::from_src(cur.src);
    if (!valid) srcv = A::zero();
    if (!A::finite(srcv)) {
      nonfinite = true;
      srcv = A::zero();
    }
    float zc, zo;  // this row; the receiving row
    if (!ADJ) {
      zc = z_keep;
      zo = t + 1 < nr ? cur.z : 0.0f;
      z_keep = zo;
    } else {
      zc = cur.z;
      zo = z_keep;
      z_keep = zc;
    }
    const uint32_t rcv = cand(code);
    const Frac<VK, FLOW_UP> fr =
        fractions<VK, FLOW_UP>(zc, sh_l(zo), zo, sh_r(zo), sh_l(zc), sh_r(zc), rcv, pf, P.p);

    // Same-row inputs: fraction taken from the left / right neighbour.
    F fin_l, fin_r;
    float din_l, din_r;
    if (!ADJ) {
      fin_l = sh_l(fr.r);
      din_l = sh_l(fr.d);
      fin_r = sh_r(fr.l);
      din_r = sh_r(fr.d);
    } else {
      fin_l = fr.l;
      din_l = fr.d;
      fin_r = fr.r;
      din_r = fr.d;
    }
    const uint64_t hl = ballot(fin_l != (F)0), hr = ballot(fin_r != (F)0);
    // Previous-row inputs and their dirt.
    uint64_t tm, t0, tp;  // lanes taking from the previous row at dc -1, 0, +1 (relative to the taker)
    if (!ADJ) {
      tm = spp << 1;
      t0 = sp0;
      tp = spm >> 1;
    } else {
      tm = ballot(fr.nm != (F)0);
      t0 = ballot(fr.n0 != (F)0);
      tp = ballot(fr.np != (F)0);
    }
    auto pull_prev = [&](V vprev) -> V {
      const V vl = sh_l(vprev), vr = sh_r(vprev);
      V cl, cm, cr;
      if (!ADJ) {
        cl = A::contrib_lean(vl, sh_l(fpp), sh_l(dp));
        cm = A::contrib_lean(vprev, fp0, dp);
        cr = A::contrib_lean(vr, sh_r(fpm), sh_r(dp));
      } else {
        cl = A::contrib_lean(vl, fr.nm, fr.d);
        cm = A::contrib_lean(vprev, fr.n0, fr.d);
        cr = A::contrib_lean(vr, fr.np, fr.d);
      }
      return A::norm(A::add_lean(srcv, A::add_lean(A::add_lean(cl, cm), cr)));
    };
    auto dirt_prev = [&](uint64_t d) -> uint64_t { return ((d << 1) & tm) | (d & t0) | ((d >> 1) & tp); };

    V a = pull_prev(vp);
    uint64_t dl = spread(dirt_prev(dpl) | edge_l, hl, hr);
    uint64_t dr = spread(dirt_prev(dpr) | edge_r, hl, hr);
    V q = lateral<VK>(a, fin_l, din_l, fin_r, din_r);

    if ((dl | dr) & own_mask) {
      // Stage 1: exact previous-row ghost values of the dirty side(s).
      const bool need_l = (dl & own_mask) != 0, need_r = (dr & own_mask) != 0;
      if (t > 0) {
        const uint32_t tag = (uint32_t)((t - 1) & 0xFF);
        const int slot = (int)((t - 1) % MS_RING);
        const bool ld = valid && ((need_l && ghost_l) || (need_r && ghost_r));
        V got = vp;
        if (!wait_words<VK>(ld ? ring_ghost + (size_t)slot * MS_OWN : nullptr, ld, tag, got)) return false;
        vp = got;
        if (need_l) dpl = edge_l;
        if (need_r) dpr = edge_r;
        a = pull_prev(vp);
        dl = spread(dirt_prev(dpl) | edge_l, hl, hr);
        dr = spread(dirt_prev(dpr) | edge_r, hl, hr);
        q = lateral<VK>(a, fin_l, din_l, fin_r, din_r);
      }
      // Stage 2: a same-row chain from beyond the window -- the
      // neighbour's values of this row for that side's ghost columns.
      const bool need2_l = (dl & own_mask) != 0, need2_r = (dr & own_mask) != 0;
      if (need2_l || need2_r) {
        const uint32_t tag = (uint32_t)(t & 0xFF);
        const int slot = (int)(t % MS_RING);
        const bool ld = valid && ((need2_l && ghost_l) || (need2_r && ghost_r));
        V got = a;
        if (!wait_words<VK>(ld ? ring_ghost + (size_t)slot * MS_OWN : nullptr, ld, tag, got)) return false;
        // Fixed ghost values take no same-row input.
        F gl = fin_l, gr = fin_r;
        if (ld) {
          a = got;
          gl = 0;
          gr = 0;
        }
        const uint64_t fixed = ballot(ld);
        const uint64_t hl2 = hl & ~fixed, hr2 = hr & ~fixed;
        q = lateral<VK>(a, gl, din_l, gr, din_r);
        dl = spread((dirt_prev(dpl) | edge_l) & ~fixed, hl2, hr2);
        dr = spread((dirt_prev(dpr) | edge_r) & ~fixed, hl2, hr2);
        if ((dl | dr) & own_mask) return false;  // cannot happen: the fixed columns separate the owned ones
      }
    }

    // Before publishing, the strips reading this one must be past the row
    // the ring slot holds (they may still read rows from their own current
    // row - 1 on).
    const int64_t need_prog = t - MS_RING + 2;
    if (need_prog > nb_prog && nb_hi > nb_lo) {
      int32_t m = INT32_MAX;
      for (int k = nb_lo; k <= nb_hi; ++k) {
        if (k == s) continue;
        if (!wait_progress(P.progress + k, (int32_t)need_prog)) return false;
        m = min(m, ld_i32(P.progress + k));
      }
      nb_prog = m;
    }

    // Results: the owned cells, the ring word, the progress word.
    if constexpr (VK == VK_FF) {
      float* dst = owned ? P.vhi + i : reinterpret_cast<float*>(junk);
      *dst = q.hi;
    } else {
      double* dst = owned ? P.v64 + i : reinterpret_cast<double*>(junk);
      *dst = q;
    }
    st_word(pub + (size_t)(t % MS_RING) * (owned ? MS_OWN : 0), A::pack(q, (uint32_t)(t & 0xFF)));
    st_i32(P.progress + s, (int32_t)(t + 1));
    if (owned) {
      if (!ADJ && code == 0u) msum += A::wide(q);
      rsum += A::wide(srcv);
    }

    // This row becomes the previous one.
    vp = q;
    dpl = dl | edge_l;
    dpr = dr | edge_r;
    if (!ADJ) {
      fpm = fr.nm;
      fp0 = fr.n0;
      fpp = fr.np;
      dp = fr.d;
      spm = ballot(fr.nm != (F)0);
      sp0 = ballot(fr.n0 != (F)0);
      spp = ballot(fr.np != (F)0);
    }
    return true;
  };

  if (!ADJ) z_keep = P.z[row_of(0) * nc + ccol];
  In b0 = load_in(0), b1 = load_in(1);
  for (int64_t t = 0; t < nr; t += 2) {
    if (!step(t, b0)) {
      stalled = true;
      break;
    }
    if (t + 1 >= nr) break;
    if (!step(t + 1, b1)) {
      stalled = true;
      break;
    }
  }

  if (ballot(nonfinite && valid) && lane == 0 && P.status) atomicCAS(P.status, 0, FR_ERR_NONFINITE);
  if (ballot(stalled)) {
    if (lane == 0 && P.status) atomicCAS(P.status, 0, FR_ERR_STALL);
    // Let the neighbours see this strip as finished, so their waits for it
    // end too (their results are void, the status says so).
    if (lane == 0) st_i32(P.progress + s, INT32_MAX);
    return;
  }
  // Mass balance partials in a fixed order (Section 4 verification).
  if (!ADJ && P.partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      msum += __shfl_xor(msum, off);
      rsum += __shfl_xor(rsum, off);
    }
    if (lane == 0) {
      P.partial[2 * s] = msum;
      P.partial[2 * s + 1] = rsum;
    }
  }
}

// Checks the codes and elevations for the row sweep and resets its ring,
// progress and partial words: MS_BAD for an invalid mask (receiver off the
// grid or not strictly lower) or a non-finite elevation, MS_UP / MS_DN when
// some cell sends to row r - 1 / r + 1.
__global__ __launch_bounds__(256) void k_ms_check(MsParams P, CallCtl* C) {
  const int64_t nr = P.nrows, nc = P.ncols, n = nr * nc;
  const int64_t ring_words = (int64_t)P.nstrips * MS_RING * MS_OWN;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t fl = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t m = P.code[i];
    const float zi = P.z[i];
    if (!isfinite(zi)) fl |= MS_BAD;
    if (m & 0x07u) fl |= MS_UP;
    if (m & 0xE0u) fl |= MS_DN;
    if (m) {
      const int64_t r = i / nc, c = i - r * nc;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (!((m >> k) & 1u)) continue;
        const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
        if (rr < 0 || rr >= nr || cc < 0 || cc >= nc || !(P.z[rr * nc + cc] < zi)) fl |= MS_BAD;
      }
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ring_words; i += stride) P.ring[i] = MS_EMPTY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.nstrips; i += stride) P.progress[i] = 0;
  // One atomic per wavefront.
  uint32_t w = fl;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) w |= (uint32_t)__shfl_xor((int)w, off);
  if ((threadIdx.x & 63) == 0 && w) atomicOr(reinterpret_cast<uint32_t*>(&C->ms_flags), w);
}

// The row sweep serves the call when every mask is valid and no cell sends
// against one of the two row orders.
__global__ void k_ms_decide(CallCtl* C) {
  if (threadIdx.x != 0) return;
  const int32_t f = C->ms_flags;
  const bool taken = !(f & MS_BAD) && !((f & MS_UP) && (f & MS_DN));
  const bool flow_up = (f & MS_UP) || !(f & MS_DN);
  C->ms_flags = f | (taken ? MS_TAKEN : 0) | (flow_up ? MS_FLOW_UP : 0);
  C->ms_skip = taken ? 0 : 1;
}

template <int VK, bool ADJ, int SRC>
hipError_t ms_launch_src(const MsParams& P, const CallCtl* C, hipStream_t s) {
  // Both row orientations are launched; the one the check did not pick
  // returns at once.
  hipLaunchKernelGGL((k_ms<VK, ADJ, true, SRC>), dim3((unsigned)P.nstrips), dim3(64), 0, s, P, C);
  hipLaunchKernelGGL((k_ms<VK, ADJ, false, SRC>), dim3((unsigned)P.nstrips), dim3(64), 0, s, P, C);
  return hipGetLastError();
}

template <int VK, bool ADJ>
hipError_t ms_launch_t(const MsParams& P, const CallCtl* C, hipStream_t s) {
  if (P.src32) return ms_launch_src<VK, ADJ, SRC_F32>(P, C, s);
  if (P.src64) return ms_launch_src<VK, ADJ, SRC_F64>(P, C, s);
  return ms_launch_src<VK, ADJ, SRC_UNIT>(P, C, s);
}

}  // namespace

int64_t ms_strips(int64_t ncols) { return (ncols + MS_OWN - 1) / MS_OWN; }

size_t ms_ring_words(int64_t ncols) { return (size_t)ms_strips(ncols) * MS_RING * MS_OWN; }

hipError_t launch_ms(ValKind vk, bool adjoint, const MsParams& P, CallCtl* C, hipStream_t s) {
  const int64_t n = P.nrows * P.ncols;
  const int64_t work = n > (int64_t)ms_ring_words(P.ncols) ? n : (int64_t)ms_ring_words(P.ncols);
  int64_t b = (work + 255) / 256;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_ms_check, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P, C);
  hipLaunchKernelGGL(k_ms_decide, dim3(1), dim3(64), 0, s, C);
  if (vk == VK_F64) return adjoint ? ms_launch_t<VK_F64, true>(P, C, s) : ms_launch_t<VK_F64, false>(P, C, s);
  return adjoint ? ms_launch_t<VK_FF, true>(P, C, s) : ms_launch_t<VK_FF, false>(P, C, s);
}

// Largest number of strips whose wavefronts can all be resident at once
// (the pass waits between neighbouring strips).
int64_t ms_max_strips() {
  static int64_t cached = -1;
  if (cached >= 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_ms<VK_F64, true, true, SRC_F64>),
                                                   64, 0) != hipSuccess)
    return 0;
  int pc2 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc2, reinterpret_cast<const void*>(&k_ms<VK_FF, false, true, SRC_F32>), 64,
                                                   0) == hipSuccess &&
      pc2 < per_cu)
    per_cu = pc2;
  cached = (int64_t)cus * per_cu;
  return cached;
}

}  // namespace fr
