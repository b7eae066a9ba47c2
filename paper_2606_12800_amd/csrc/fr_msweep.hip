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
// GPU mapping.  One workgroup owns a strip of MS_OWN columns and computes a
// window of 64 columns, lane = column: the owned columns and MS_G columns of
// each neighbouring strip ("ghost" columns), recomputed from the same
// inputs.  Producer wavefronts load each row's codes, elevations and source
// terms and compute the cells' fractions into a ring of rows in LDS, ahead
// of the consumer wavefront, which runs the recurrence: a row step pulls
// the previous row's values of the three upslope neighbours through lane
// shifts (DPP), then resolves same-row chains by repeated lane-shifted
// pulls until no value changes (chains on this kind of terrain are a few
// cells long).  No value leaves the consumer except the owned results.
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
// every code and takes the pass only if no cell sends to the row before it
// in one of the two row orders; otherwise the general wavefront sweep runs
// instead.  The pass itself reports masks whose receivers are off the grid
// or not strictly lower, and non-finite elevations, as the general sweep
// does.  Results are exact up to rounding and do not depend on timing:
// which ghost columns are refreshed, and with what, depends only on the
// data.
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

// Waits until strips lo..hi other than s have finished `target` rows;
// returns the smallest progress seen then (below target after the spin
// limit).
__device__ __noinline__ int32_t wait_strips(const int32_t* progress, int lo, int hi, int s, int32_t target) {
  int32_t m = INT32_MAX;
  for (int k = lo; k <= hi; ++k) {
    if (k == s) continue;
    int32_t v = ld_i32(progress + k);
    for (uint32_t it = 0; v < target && it < MS_SPIN_LIMIT; ++it) {
      __builtin_amdgcn_s_sleep(1);
      v = ld_i32(progress + k);
    }
    m = min(m, v);
  }
  return m;
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

// Producer wavefronts per strip: float64 fractions (two transcendental
// functions per candidate) cost more than the consumer's row step, so two
// wavefronts share them (alternate rows).
template <int VK>
constexpr int ms_producers() {
  return VK == VK_F64 ? 2 : 1;
}
constexpr int MS_PR = 6;  // staged rows per strip (LDS ring)

// One staged row, per lane: the cell's fractions toward its five candidate
// receivers (next-row dc -1, 0, +1; left; right), its conservation
// correction, its source term and its code.
template <int VK>
struct Stage {
  typename Arith<VK>::F nm[MS_LANES], n0[MS_LANES], np[MS_LANES], l[MS_LANES], r[MS_LANES];
  float d[MS_LANES];
  typename Arith<VK>::V src[MS_LANES];
  uint32_t code[MS_LANES];
};

__device__ __forceinline__ int32_t lds_ld(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// LDS operations of one wavefront are performed in issue order; these keep
// the compiler from moving the staged data across the flag words.
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Workgroup b runs on XCD b % 8; XCD x takes the x-th contiguous range of
// strips (the first n % 8 ranges one strip longer), so that only 7 strip
// boundaries cross XCDs.  A bijection of 0 .. n - 1.
constexpr int MS_XCDS = 8;
__device__ __forceinline__ int ms_strip_of_block(int b, int n) {
  const int x = b % MS_XCDS, k = b / MS_XCDS;
  const int q = n / MS_XCDS, r = n % MS_XCDS;
  return x * q + (x < r ? x : r) + k;
}

// One workgroup per strip: wavefront 0 is the consumer, which runs the row
// recurrence for the strip's 64-column window; the others are producers,
// which load each row's codes, elevations and source terms and compute the
// fractions into an LDS ring of MS_PR rows ahead of the consumer.
// FLOW_UP: receivers lie in row r - 1 (the forward sweep visits rows from
// the last to the first); else in row r + 1.  ADJ: the adjoint, visiting
// rows the other way and pulling from receivers.
//
// Strips are numbered so that neighbouring strips run on the same XCD (the
// hardware deals workgroups to the 8 XCDs in turn): their overlapping
// columns and exchanged words then meet in one L2.
template <int VK, bool ADJ, bool FLOW_UP, int SRC>
__global__ __launch_bounds__(64 * (1 + ms_producers<VK>())) void k_ms(MsParams P, const CallCtl* C) {
  using A = Arith<VK>;
  using V = typename A::V;
  using F = typename A::F;
  constexpr int NP = ms_producers<VK>();
  const int32_t gate = C->ms_flags;
  if (!(gate & MS_TAKEN) || ((gate & MS_FLOW_UP) != 0) != FLOW_UP) return;

  __shared__ Stage<VK> stage[MS_PR];
  __shared__ int32_t slot_row[MS_PR];  // row held by each slot (-1: none yet)
  __shared__ int32_t cons_row;         // rows the consumer has taken
  __shared__ int32_t abort_flag;       // set by the consumer when it gives up
  if (threadIdx.x < MS_PR) slot_row[threadIdx.x] = -1;
  if (threadIdx.x == 0) {
    cons_row = -1;
    abort_flag = 0;
  }
  __syncthreads();

  const int wave = (int)threadIdx.x >> 6;
  const int lane = (int)threadIdx.x & 63;
  const int s = ms_strip_of_block((int)blockIdx.x, P.nstrips);
  const int64_t nr = P.nrows, nc = P.ncols;
  const int64_t col = (int64_t)s * MS_OWN - MS_G + lane;
  const bool valid = col >= 0 && col < nc;
  const int64_t ccol = valid ? col : 0;
  // Rows in visiting order: step t visits row y(t).
  const bool rows_down = ADJ ? FLOW_UP : !FLOW_UP;  // true: y = t
  auto row_of = [&](int64_t t) { return rows_down ? t : nr - 1 - t; };

  if (wave > 0) {
    // ------------------------------------------------------------ producer
    // Window-edge lanes do not see the column beyond: that candidate is
    // dropped from their masks (their fractions are then wrong, and the
    // consumer treats their values as dirty anyway).
    uint32_t drop_mask = 0;
    if (lane == 0) drop_mask |= (1u << 0) | (1u << 3);   // nm, l
    if (lane == 63) drop_mask |= (1u << 2) | (1u << 4);  // np, r
    constexpr int kn0 = FLOW_UP ? 0 : 5;
    const float pf = (float)P.p;
    // The receiving row of step t: forward the next row visited, adjoint
    // the previous one.
    auto recv_step = [&](int64_t t) -> int64_t { return ADJ ? t - 1 : t + 1; };
    struct Raw {
      float zc, zo;
      uint32_t code;
      typename SrcT<SRC>::T src;
    };
    // A single producer visits every row and loads each elevation row
    // once, carrying the other row of a step over from the step before.
    constexpr bool CARRY = NP == 1;
    auto load_raw = [&](int64_t t) -> Raw {
      Raw w;
      const int64_t tc = t < nr ? t : nr - 1;
      const int64_t i = row_of(tc) * nc + ccol;
      w.code = P.code[i];
      int64_t tr = recv_step(tc);
      tr = tr < 0 ? 0 : (tr >= nr ? nr - 1 : tr);
      // Carrying: forward loads only the receiving (next) row, adjoint only
      // this row.
      if (!CARRY || ADJ) w.zc = P.z[i];
      if (!CARRY || !ADJ) w.zo = P.z[row_of(tr) * nc + ccol];
      if constexpr (SRC == SRC_F32) w.src = P.src32[i];
      else if constexpr (SRC == SRC_F64) w.src = P.src64[i];
      else w.src = 0;
      return w;
    };
    const int k = wave - 1;
    bool bad = false, nonfin = false;
    float zcarry = 0.0f;  // forward: this row's z (last step's next row); adjoint: the previous row's z
    if (CARRY && !ADJ) zcarry = P.z[row_of(0) * nc + ccol];
    Raw nx = load_raw(k);
    for (int64_t t = k; t < nr; t += NP) {
      Raw cur = nx;
      nx = load_raw(t + NP);
      if (CARRY) {
        if (!ADJ) {
          cur.zc = zcarry;
          zcarry = cur.zo;
        } else {
          cur.zo = zcarry;
          zcarry = cur.zc;
        }
      }
      const int slot = (int)(t % MS_PR);
      // Wait until the consumer has released the row this slot held (it
      // keeps its current row and the one before).
      while (lds_ld(&cons_row) <= t - MS_PR) {
        if (lds_ld(&abort_flag)) return;
        __builtin_amdgcn_s_sleep(1);
      }
      const int64_t tr = recv_step(t);
      const bool has_recv_row = tr >= 0 && tr < nr;
      const float zo = has_recv_row ? cur.zo : 0.0f;
      const uint32_t m_all = ((cur.code >> kn0) & 7u) | (((cur.code >> 3) & 3u) << 3);
      uint32_t m = valid ? (m_all & ~drop_mask) : 0u;
      if (valid) {
        // Each receiver must be a strictly lower cell of the grid (the
        // general sweep reports the same errors); the window's edge lanes
        // are checked by the strips that own those columns.
        const float zr[5] = {sh_l(zo), zo, sh_r(zo), sh_l(cur.zc), sh_r(cur.zc)};
        const bool on_grid[5] = {has_recv_row && col >= 1, has_recv_row, has_recv_row && col + 1 < nc, col >= 1,
                                 col + 1 < nc};
        bool badc = false;
#pragma unroll
        for (int j = 0; j < 5; ++j)
          if ((m_all >> j) & 1u) badc |= !on_grid[j] || (((m >> j) & 1u) && !(zr[j] < cur.zc));
        if (!isfinite(cur.zc)) nonfin = true;
        if (badc) bad = true;
      }
      const Frac<VK, FLOW_UP> fr =
          fractions<VK, FLOW_UP>(cur.zc, sh_l(zo), zo, sh_r(zo), sh_l(cur.zc), sh_r(cur.zc), m, pf, P.p);
      V sv;
      if constexpr (SRC == SRC_UNIT) sv = A::one();
      else sv = A::from_src(cur.src);
      Stage<VK>& S = stage[slot];
      S.nm[lane] = fr.nm;
      S.n0[lane] = fr.n0;
      S.np[lane] = fr.np;
      S.l[lane] = fr.l;
      S.r[lane] = fr.r;
      S.d[lane] = fr.d;
      S.src[lane] = sv;
      S.code[lane] = valid ? cur.code : 0u;
      compiler_fence();
      if (lane == 0) lds_st(&slot_row[slot], (int32_t)t);
    }
    if (P.status) {
      if (ballot(bad) && lane == 0) atomicCAS(P.status, 0, FR_ERR_BADCODE);
      if (ballot(nonfin) && lane == 0) atomicCAS(P.status, 0, FR_ERR_NONFINITE);
    }
    return;
  }

  // -------------------------------------------------------------- consumer
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

  // Ring words: a ghost lane reads the owner of its column.
  uint64_t* ring_mine = P.ring + (size_t)s * MS_RING * MS_OWN;
  const bool ghost_l = lane < MS_G, ghost_r = lane >= MS_G + MS_OWN;
  const int64_t owner = valid ? col / MS_OWN : 0;
  const uint64_t* ring_ghost = P.ring + (size_t)owner * MS_RING * MS_OWN + (size_t)(ccol - owner * MS_OWN);
  int32_t nb_prog = 0;  // smallest neighbour progress seen (rows finished)
  uint64_t* pub = ring_mine + (owned ? lane - MS_G : 0);

  // A row's inputs in the form the recurrence takes them: pull weights
  // toward the previous row's three cells (lane shifts -1, 0, +1), same-row
  // input fractions from the left / right, with the senders' corrections,
  // the source term and the masks of lanes taking each input.
  struct Ctx {
    F wl, w0, wr, fl, fr;
    float dwl, dw0, dwr, dfl, dfr;
    V src;
    uint32_t code;
    uint64_t tm, t0, tp, hl, hr;
  };
  // The staged rows t - 1 and t stay in the ring while row t is computed.
  auto load_ctx = [&](int64_t tt) -> Ctx {
    const Stage<VK>& S = stage[tt % MS_PR];
    Ctx c;
    const F nm = S.nm[lane], n0 = S.n0[lane], np = S.np[lane], l = S.l[lane], r = S.r[lane];
    const float d = S.d[lane];
    c.src = S.src[lane];
    c.code = S.code[lane];
    if (!ADJ) {
      // Forward: a cell takes a fraction of each upslope neighbour in the
      // previous row (that cell's own fractions) and of its same-row donors.
      F pnm = 0, pn0 = 0, pnp = 0;
      float pd = 0.0f;
      if (tt > 0) {
        const Stage<VK>& Q = stage[(tt - 1) % MS_PR];
        pnm = Q.nm[lane];
        pn0 = Q.n0[lane];
        pnp = Q.np[lane];
        pd = Q.d[lane];
      }
      c.wl = sh_l(pnp);
      c.dwl = sh_l(pd);
      c.w0 = pn0;
      c.dw0 = pd;
      c.wr = sh_r(pnm);
      c.dwr = sh_r(pd);
      c.fl = sh_l(r);
      c.dfl = sh_l(d);
      c.fr = sh_r(l);
      c.dfr = sh_r(d);
    } else {
      // Adjoint: a cell takes its own fractions of its receivers' values.
      c.wl = nm;
      c.w0 = n0;
      c.wr = np;
      c.fl = l;
      c.fr = r;
      c.dwl = c.dw0 = c.dwr = c.dfl = c.dfr = d;
    }
    c.tm = ballot(c.wl != (F)0);
    c.t0 = ballot(c.w0 != (F)0);
    c.tp = ballot(c.wr != (F)0);
    c.hl = ballot(c.fl != (F)0);
    c.hr = ballot(c.fr != (F)0);
    return c;
  };
  auto pull_prev = [&](const Ctx& c, V vprev) -> V {
    const V cl = A::contrib_lean(sh_l(vprev), c.wl, c.dwl);
    const V cm = A::contrib_lean(vprev, c.w0, c.dw0);
    const V cr = A::contrib_lean(sh_r(vprev), c.wr, c.dwr);
    return A::norm(A::add_lean(c.src, A::add_lean(A::add_lean(cl, cm), cr)));
  };
  auto dirt_prev = [&](const Ctx& c, uint64_t d) -> uint64_t {
    return ((d << 1) & c.tm) | (d & c.t0) | ((d >> 1) & c.tp);
  };
  // One row from the previous row's values and dirt: q and its dirt.
  auto solve_row = [&](const Ctx& c, V vprev, uint64_t pl, uint64_t pr, V& a, V& q, uint64_t& dl, uint64_t& dr) {
    a = pull_prev(c, vprev);
    dl = spread(dirt_prev(c, pl) | edge_l, c.hl, c.hr);
    dr = spread(dirt_prev(c, pr) | edge_r, c.hl, c.hr);
    q = lateral<VK>(a, c.fl, c.dfl, c.fr, c.dfr);
  };

  // Previous row: values and dirt by side of origin.
  V vp = A::zero();
  uint64_t dpl = 0, dpr = 0;

  double msum = 0.0, rsum = 0.0;
  bool nonfinite = false, stalled = false;

  for (int64_t t = 0; t < nr && !stalled; ++t) {
    const int64_t y = row_of(t);
    const int64_t i = y * nc + ccol;
    // Before this row is published, the strips reading this one must be
    // past the row its ring slot holds (they may still read rows from their
    // own current row - 1 on).  Checked first, before any of the row's work.
    const int32_t need_prog = (int32_t)(t - MS_RING + 2);
    if (need_prog > nb_prog && nb_hi > nb_lo) {
      nb_prog = wait_strips(P.progress, nb_lo, nb_hi, s, need_prog);
      if (nb_prog < need_prog) {
        stalled = true;
        break;
      }
    }
    // This row's staged inputs; rows up to t - 2 are released (forward, the
    // previous row's fractions are read again with this row's).
    const int slot = (int)(t % MS_PR);
    while (lds_ld(&slot_row[slot]) != (int32_t)t) __builtin_amdgcn_s_sleep(1);
    compiler_fence();
    Ctx cx = load_ctx(t);
    compiler_fence();
    if (lane == 0) lds_st(&cons_row, (int32_t)(t - 1));
    if (!valid) cx.src = A::zero();
    if (!A::finite(cx.src)) {
      nonfinite = true;
      cx.src = A::zero();
    }

    V a, q;
    uint64_t dl, dr;
    solve_row(cx, vp, dpl, dpr, a, q, dl, dr);

    if ((dl | dr) & own_mask) {
      // Stage 1: exact previous-row ghost values of the dirty side(s).
      if (t >= 1) {
        const bool need_l = (dl & own_mask) != 0, need_r = (dr & own_mask) != 0;
        const bool ld = valid && ((need_l && ghost_l) || (need_r && ghost_r));
        const uint32_t tag = (uint32_t)((t - 1) & 0xFF);
        const int rs = (int)((t - 1) % MS_RING);
        V got = vp;
        if (!wait_words<VK>(ld ? ring_ghost + (size_t)rs * MS_OWN : nullptr, ld, tag, got)) {
          stalled = true;
          break;
        }
        vp = got;
        if (need_l) dpl = edge_l;
        if (need_r) dpr = edge_r;
        solve_row(cx, vp, dpl, dpr, a, q, dl, dr);
      }
      // Stage 2: a same-row chain from beyond the window -- the
      // neighbour's values of this row for that side's ghost columns.
      const bool need2_l = (dl & own_mask) != 0, need2_r = (dr & own_mask) != 0;
      if (need2_l || need2_r) {
        const uint32_t tag = (uint32_t)(t & 0xFF);
        const int rs = (int)(t % MS_RING);
        const bool ld = valid && ((need2_l && ghost_l) || (need2_r && ghost_r));
        V got = a;
        if (!wait_words<VK>(ld ? ring_ghost + (size_t)rs * MS_OWN : nullptr, ld, tag, got)) {
          stalled = true;
          break;
        }
        // Fixed ghost values take no same-row input.
        F gl = cx.fl, gr = cx.fr;
        if (ld) {
          a = got;
          gl = 0;
          gr = 0;
        }
        const uint64_t fixed = ballot(ld);
        const uint64_t hl2 = cx.hl & ~fixed, hr2 = cx.hr & ~fixed;
        q = lateral<VK>(a, gl, cx.dfl, gr, cx.dfr);
        dl = spread((dirt_prev(cx, dpl) | edge_l) & ~fixed, hl2, hr2);
        dr = spread((dirt_prev(cx, dpr) | edge_r) & ~fixed, hl2, hr2);
        if ((dl | dr) & own_mask) {
          stalled = true;  // cannot happen: the fixed columns separate the owned ones
          break;
        }
      }
    }

    // Results: the owned cells, their ring words, the progress word.
    if (owned) {
      if constexpr (VK == VK_FF) P.vhi[i] = q.hi;
      else P.v64[i] = q;
      st_word(pub + (size_t)(t % MS_RING) * MS_OWN, A::pack(q, (uint32_t)(t & 0xFF)));
      if (!ADJ && cx.code == 0u) msum += A::wide(q);
      rsum += A::wide(cx.src);
    }
    if (lane == 0) st_i32(P.progress + s, (int32_t)(t + 1));

    // This row becomes the previous one.
    vp = q;
    dpl = dl | edge_l;
    dpr = dr | edge_r;
  }

  if (ballot(nonfinite && valid) && lane == 0 && P.status) atomicCAS(P.status, 0, FR_ERR_NONFINITE);
  if (ballot(stalled)) {
    if (lane == 0) {
      lds_st(&abort_flag, 1);
      if (P.status) atomicCAS(P.status, 0, FR_ERR_STALL);
      // Let the neighbours see this strip as finished, so their waits for
      // it end too (their results are void, the status says so).
      st_i32(P.progress + s, INT32_MAX);
    }
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

// Reads the codes for the row sweep and resets its ring, progress and
// partial words: MS_UP / MS_DN when some cell sends to row r - 1 / r + 1.
// (The masks' other properties -- receivers on the grid and strictly lower,
// elevations finite -- are checked by the sweep's producers, which read
// every candidate receiver's elevation anyway.)
__global__ __launch_bounds__(256) void k_ms_check(MsParams P, CallCtl* C) {
  const int64_t n = P.nrows * P.ncols;
  const int64_t ring_words = (int64_t)P.nstrips * MS_RING * MS_OWN;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t any = 0;
  // Four codes per load where the row length allows it.
  const int64_t n4 = (P.ncols % 4 == 0 && (reinterpret_cast<uintptr_t>(P.code) & 3) == 0) ? n / 4 : 0;
  const uint32_t* c4 = reinterpret_cast<const uint32_t*>(P.code);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) any |= c4[i];
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) any |= P.code[i];
  any = any | (any >> 8) | (any >> 16) | (any >> 24);
  const uint32_t fl = ((any & 0x07u) ? MS_UP : 0u) | ((any & 0xE0u) ? MS_DN : 0u);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ring_words; i += stride) P.ring[i] = MS_EMPTY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.nstrips; i += stride) P.progress[i] = 0;
  // One atomic per workgroup, and only for bits not set yet (every
  // workgroup of a tilted grid finds the same bit).
  __shared__ uint32_t blk;
  if (threadIdx.x == 0) blk = 0u;
  __syncthreads();
  if (fl) atomicOr(&blk, fl);
  __syncthreads();
  if (threadIdx.x == 0 && blk) {
    uint32_t* f = reinterpret_cast<uint32_t*>(&C->ms_flags);
    if ((__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & blk) != blk) atomicOr(f, blk);
  }
}

// The row sweep serves the call when no cell sends against one of the two
// row orders.
__global__ void k_ms_decide(CallCtl* C) {
  if (threadIdx.x != 0) return;
  const int32_t f = C->ms_flags;
  const bool taken = !((f & MS_UP) && (f & MS_DN));
  const bool flow_up = (f & MS_UP) || !(f & MS_DN);
  C->ms_flags = f | (taken ? MS_TAKEN : 0) | (flow_up ? MS_FLOW_UP : 0);
  C->ms_skip = taken ? 0 : 1;
}

template <int VK, bool ADJ, int SRC>
hipError_t ms_launch_src(const MsParams& P, const CallCtl* C, hipStream_t s) {
  // Both row orientations are launched; the one the check did not pick
  // returns at once.
  const dim3 block(64 * (1 + ms_producers<VK>()));
  hipLaunchKernelGGL((k_ms<VK, ADJ, true, SRC>), dim3((unsigned)P.nstrips), block, 0, s, P, C);
  hipLaunchKernelGGL((k_ms<VK, ADJ, false, SRC>), dim3((unsigned)P.nstrips), block, 0, s, P, C);
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
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_ms_check, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P, C);
  hipLaunchKernelGGL(k_ms_decide, dim3(1), dim3(64), 0, s, C);
  if (vk == VK_F64) return adjoint ? ms_launch_t<VK_F64, true>(P, C, s) : ms_launch_t<VK_F64, false>(P, C, s);
  return adjoint ? ms_launch_t<VK_FF, true>(P, C, s) : ms_launch_t<VK_FF, false>(P, C, s);
}

// Largest number of strips whose workgroups can all be resident at once
// (the pass waits between neighbouring strips), for the given precision:
// the smallest occupancy over the kernel variants of that precision.
int64_t ms_max_strips(ValKind vk) {
  static int64_t cached[3] = {-1, -1, -1};
  const int idx = vk == VK_F64 ? 2 : 1;
  if (cached[idx] >= 0) return cached[idx];
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const void* kf[4];
  int block;
  if (vk == VK_F64) {
    kf[0] = reinterpret_cast<const void*>(&k_ms<VK_F64, false, true, SRC_UNIT>);
    kf[1] = reinterpret_cast<const void*>(&k_ms<VK_F64, false, true, SRC_F64>);
    kf[2] = reinterpret_cast<const void*>(&k_ms<VK_F64, true, true, SRC_F64>);
    kf[3] = reinterpret_cast<const void*>(&k_ms<VK_F64, true, false, SRC_F32>);
    block = 64 * (1 + ms_producers<VK_F64>());
  } else {
    kf[0] = reinterpret_cast<const void*>(&k_ms<VK_FF, false, true, SRC_UNIT>);
    kf[1] = reinterpret_cast<const void*>(&k_ms<VK_FF, false, true, SRC_F64>);
    kf[2] = reinterpret_cast<const void*>(&k_ms<VK_FF, true, true, SRC_F64>);
    kf[3] = reinterpret_cast<const void*>(&k_ms<VK_FF, true, false, SRC_F32>);
    block = 64 * (1 + ms_producers<VK_FF>());
  }
  int per_cu = 1 << 30;
  for (const void* k : kf) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, 0) != hipSuccess) return 0;
    per_cu = n < per_cu ? n : per_cu;
  }
  cached[idx] = (int64_t)cus * per_cu;
  return cached[idx];
}

}  // namespace fr
