// Accumulation engine: solves (I - W^T) q = r (forward) or (I - W) rbar =
// qbar (adjoint) on the grid's routing DAG without sorting.
//
// The paper's sequential algorithm processes cells high-to-low so that every
// cell is visited after all cells that give it water (Section 2.1); its
// "optimization 2" notes that only this processing order matters, not the
// numbering (Section 3.2).  Here the order comes from dependency counting,
// the shared-memory idea the paper cites as prior art (Section 1, Section
// 2.1): a cell is ready once all of its inputs (donors for the forward
// solve, receivers for the adjoint) are final, and then its value is
//   forward:  v_i = r_i + sum_{donors j} f_{j->i} v_j
//   adjoint:  v_i = qbar_i + sum_{receivers k} f_{i->k} v_k,
// pulled in fixed neighbour order, so results do not depend on scheduling.
//
// GPU layout.  The grid is cut into ENG_TH x ENG_TW tiles.  A workgroup
// loads a tile (codes with a one-cell halo, per-cell state) into LDS and
// peels it: ready cells form a frontier, compacted with wavefront ballots;
// processing a frontier cell decrements the in-tile pending counts of its
// outputs in LDS, and cells that reach zero form the next frontier.  Inputs
// in other tiles are tracked by a per-cell counter in HBM; when a tile
// finishes a cell whose output lies in another tile it decrements that
// counter atomically and, at zero, queues the other tile for the next
// iteration.  Iterations repeat until every cell is final.  On a valid DAG
// each iteration finishes at least the cells whose inputs were all final, so
// the number of iterations is bounded by the number of tile boundaries on
// the longest flow path; on a cyclic input the queue drains with cells left
// over, which the host reports as FR_ERR_NOTDAG.
//
// Precision.  VK_FF keeps every value as an unevaluated float-float sum
// (hi + lo) so that long rivers accumulate with ~2^-44 relative error while
// all arithmetic stays in float32; the float32 output is hi.  VK_F64 uses
// float64.  Counts (unit rain, D8/D4 forward) are exact uint64.
#include <math.h>

#include "fr_internal.hpp"

namespace fr {
namespace {

// ---------------------------------------------------------------------------
// Float-float arithmetic (Dekker 1971; Knuth TAOCP vol. 2, 4.2.2): a value is
// the unevaluated sum hi + lo with |lo| <= ulp(hi)/2.
struct ff {
  float hi, lo;
};

__device__ __forceinline__ ff ff_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ ff ff_fast_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ ff ff_add(ff x, ff y) {
  ff s = ff_two_sum(x.hi, y.hi);
  const float e = s.lo + (x.lo + y.lo);
  return ff_fast_two_sum(s.hi, e);
}

// x * f * (1 + d) for a float32 fraction f and the small correction d of
// its cell's fractions (the d term goes into the low part).
__device__ __forceinline__ ff ff_mul_fd(ff x, float f, float d) {
  const float p = x.hi * f;
  float e = fmaf(x.hi, f, -p);
  e = fmaf(x.lo, f, e);
  e = fmaf(p, d, e);
  return ff_fast_two_sum(p, e);
}

// float32 nearest to 1/sqrt(2).
__device__ constexpr float kInvSqrt2f = 0x1.6a09e6p-1f;
__device__ constexpr double kSqrt2 = 1.4142135623730950488;

__device__ __forceinline__ void set_status(int32_t* st, int32_t code) {
  if (st) atomicCAS(st, 0, code);
}

__device__ __forceinline__ bool is_recv(int rk, uint8_t code, int k) {
  return rk == RK_SINGLE ? (code == (uint8_t)k) : (((code >> k) & 1u) != 0);
}

// Weight of the edge from a cell at elevation zh down to a neighbour at zl in
// direction k (MFD), float32 mode: (s / s_ref)^p with s_ref the cell's
// steepest slope, so the exponent stays small and exp2/log2 keep ~1 ulp.
__device__ __forceinline__ float mfd_t32(float zh, float zl, int k, float rs, float p) {
  const float drop = zh - zl;
  const float s = nb_diag(k) ? drop * kInvSqrt2f : drop;
  return exp2f(p * log2f(s * rs));
}

__device__ __forceinline__ double mfd_w64(float zh, float zl, int k, double p) {
  const double s = ((double)zh - (double)zl) / (nb_diag(k) ? kSqrt2 : 1.0);
  return pow(s, p);
}

// ---------------------------------------------------------------------------
// Initialisation: per-cell external pending counts, done flags, MFD split
// constants, argument checks that need the data.
template <int RK, int DIR, int VK>
__global__ __launch_bounds__(256) void k_engine_init(EngineParams P) {
  if (P.gate && *P.gate == 0) return;  // another path finished the solve
  const int64_t n = P.nrows * P.ncols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool badcode = false, nonfinite = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t r = i / P.ncols, c = i - r * P.ncols;
    const int64_t tr = r / ENG_TH, tc = c / ENG_TW;
    const uint8_t ci = P.code[i];
    int ext = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
      const bool in_grid = rr >= 0 && rr < P.nrows && cc >= 0 && cc < P.ncols;
      const int64_t j = rr * P.ncols + cc;
      const bool recv = is_recv(RK, ci, k);
      if (recv && !in_grid) badcode = true;
      if (!in_grid) continue;
      bool input;
      if (DIR == DIR_FWD)
        input = is_recv(RK, P.code[j], 7 - k);  // neighbour gives water to i
      else
        input = recv;  // i gives water to the neighbour
      if (input && (rr / ENG_TH != tr || cc / ENG_TW != tc)) ++ext;
      if (RK == RK_MULTI && recv && !(P.z[j] < P.z[i])) badcode = true;
    }
    if (RK == RK_SINGLE && ci != SINK && ci > 7) badcode = true;
    P.ext[i] = (uint8_t)ext;
    P.done[i] = 0;
    if (P.src32 && !isfinite(P.src32[i])) nonfinite = true;
    if (P.src64 && !isfinite(P.src64[i])) nonfinite = true;
    if (RK == RK_MULTI) {
      const float zi = P.z[i];
      if (!isfinite(zi)) nonfinite = true;
      if (VK == VK_FF) {
        float smax = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (!is_recv(RK, ci, k)) continue;
          const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
          if (rr < 0 || rr >= P.nrows || cc < 0 || cc >= P.ncols) continue;
          const float drop = zi - P.z[rr * P.ncols + cc];
          const float s = nb_diag(k) ? drop * kInvSqrt2f : drop;
          smax = s > smax ? s : smax;
        }
        const float rs = smax > 0.0f ? 1.0f / smax : 0.0f;
        float sum = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (!is_recv(RK, ci, k)) continue;
          const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
          if (rr < 0 || rr >= P.nrows || cc < 0 || cc >= P.ncols) continue;
          sum += mfd_t32(zi, P.z[rr * P.ncols + cc], k, rs, (float)P.p);
        }
        const float iw = sum > 0.0f ? 1.0f / sum : 0.0f;
        // The rounded fractions f_k = t_k * iw do not sum to 1 exactly, and
        // along a long flow path the excess would compound: with their
        // exact (float-float) sum s, every contribution is scaled by
        // 1 + d, d = 1 - s, which restores the sum to first order.  The
        // f_k here are computed exactly as the edges recompute them.
        ff es{0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (!is_recv(RK, ci, k)) continue;
          const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
          if (rr < 0 || rr >= P.nrows || cc < 0 || cc >= P.ncols) continue;
          es = ff_add(es, ff{mfd_t32(zi, P.z[rr * P.ncols + cc], k, rs, (float)P.p) * iw, 0.0f});
        }
        P.rs32[i] = rs;
        P.iw32[i] = iw;
        P.d32[i] = sum > 0.0f ? -((es.hi - 1.0f) + es.lo) : 0.0f;
      } else if (VK == VK_F64) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (!is_recv(RK, ci, k)) continue;
          const int64_t rr = r + nb_dr(k), cc = c + nb_dc(k);
          if (rr < 0 || rr >= P.nrows || cc < 0 || cc >= P.ncols) continue;
          sum += mfd_w64(zi, P.z[rr * P.ncols + cc], k, P.p);
        }
        P.iw64[i] = sum > 0.0 ? 1.0 / sum : 0.0;
      }
    }
  }
  if (badcode) set_status(P.status, FR_ERR_BADCODE);
  if (nonfinite) set_status(P.status, FR_ERR_NONFINITE);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int ntiles = P.ntr * P.ntc;
    P.nlist[0] = ntiles;
    P.nlist[1] = 0;
    P.nlist[2] = 0;
    *P.remaining = (unsigned long long)n;
    *P.bar = 0ull;
  }
  const int64_t ntiles = (int64_t)P.ntr * P.ntc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride) {
    P.stamp[t] = 0;
    P.list0[t] = (int32_t)t;
  }
}

// ---------------------------------------------------------------------------
// Per-tile LDS storage.
template <int RK, int VK, bool CNT>
struct TileLds {
  static constexpr int TH = ENG_TH, TW = ENG_TW, HW = ENG_TW + 2;
  static constexpr int NC = ENG_TH * ENG_TW;
  static constexpr int NH = (ENG_TH + 2) * (ENG_TW + 2);
  uint8_t code[NH];
  // bits 0-7: in-tile inputs not final; bit 8: final; bits 16-23: external
  // inputs not final when the tile was loaded.
  uint32_t st[NC];
  uint16_t front[2][NC];
  int nf[2];
  int ndone;
  ff vff[VK == VK_FF ? NC : 1];
  double v64[VK == VK_F64 ? NC : 1];
  uint64_t cnt[CNT ? NC : 1];
  float z[RK == RK_MULTI ? NH : 1];
  float rs[(RK == RK_MULTI && VK == VK_FF) ? NH : 1];
  float iw[(RK == RK_MULTI && VK == VK_FF) ? NH : 1];
  float dd[(RK == RK_MULTI && VK == VK_FF) ? NH : 1];
  double iw64[(RK == RK_MULTI && VK == VK_F64) ? NH : 1];
};

// Device-coherent (agent scope) loads and stores.  The L2 of each XCD is
// not coherent with the others inside a launch; these accesses are, without
// the whole-L2 write-back / invalidate that device-scope fences cost.
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_dev(const float* p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<uint32_t*>(const_cast<float*>(p)),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
  return (uint64_t)__hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p)),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wavefront's outstanding memory operations have completed.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

constexpr uint32_t ST_DONE = 1u << 8;
// Final before this activation loaded the tile: its value is in HBM only.
constexpr uint32_t ST_PREV = 1u << 9;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Append local index l to frontier f when pred holds (wavefront ballot +
// prefix; one LDS atomic per wavefront).  Must be called by all lanes.
template <class L>
__device__ __forceinline__ void push_front(L& S, int f, bool pred, int l) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0) base = atomicAdd(&S.nf[f], __popcll(m));
  base = __shfl(base, 0, 64);
  if (pred) S.front[f][base + __popcll(m & lanemask_lt())] = (uint16_t)l;
}

// Queue tile t for iteration it + 1 (at most once).
__device__ __forceinline__ void activate(const EngineParams& P, int it, int64_t t) {
  if (atomicMax(&P.stamp[t], it + 1) < it + 1) {
    const int pos = atomicAdd(&P.nlist[(it + 1) % 3], 1);
    int32_t* next = (it & 1) ? P.list0 : P.list1;
    next[pos] = (int32_t)t;
  }
}

// One output edge of a finished cell leaves the tile: decrement the
// receiving cell's external counter (byte inside a 32-bit word).
__device__ __forceinline__ void signal_external(const EngineParams& P, int it, int64_t g, int64_t gr,
                                                int64_t gc) {
  uint32_t* w = reinterpret_cast<uint32_t*>(P.ext + (g & ~(int64_t)3));
  const int sh = 8 * (int)(g & 3);
  const uint32_t old = atomicSub(w, 1u << sh);
  if (((old >> sh) & 0xFFu) == 1u) activate(P, it, (gr / ENG_TH) * P.ntc + gc / ENG_TW);
}

// Fraction of the water on the edge between cell h and its neighbour hn in
// direction k (from h): forward solves pull along donor -> h edges (the
// donor's split), adjoint solves along h -> receiver edges (h's split).
// Float32 mode: x times the fraction, with the splitting cell's correction.
template <int DIR, class L>
__device__ __forceinline__ ff edge_ff(const L& S, ff x, int h, int hn, int k, float p) {
  if (DIR == DIR_FWD) return ff_mul_fd(x, mfd_t32(S.z[hn], S.z[h], 7 - k, S.rs[hn], p) * S.iw[hn], S.dd[hn]);
  return ff_mul_fd(x, mfd_t32(S.z[h], S.z[hn], k, S.rs[h], p) * S.iw[h], S.dd[h]);
}
template <int DIR, class L>
__device__ __forceinline__ double edge_f64(const L& S, int h, int hn, int k, double p) {
  if (DIR == DIR_FWD) return mfd_w64(S.z[hn], S.z[h], 7 - k, p) * S.iw64[hn];
  return mfd_w64(S.z[h], S.z[hn], k, p) * S.iw64[h];
}

// Does cell (lr, lc) have an output outside the tile?
template <int RK, int DIR, class L>
__device__ __forceinline__ bool leaves(const L& S, int h, int lr, int lc, int th, int tw) {
  const uint8_t ci = S.code[h];
  bool any = false;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int hn = h + nb_dr(k) * L::HW + nb_dc(k);
    const bool out = (DIR == DIR_FWD) ? is_recv(RK, ci, k) : is_recv(RK, S.code[hn], 7 - k);
    const int nr = lr + nb_dr(k), nc = lc + nb_dc(k);
    if (out && !(nr >= 0 && nr < th && nc >= 0 && nc < tw)) any = true;
  }
  return any;
}

__device__ __forceinline__ int32_t ld_dev(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One iteration: every tile of list it % 3 (grid-stride over workgroups).
template <int RK, int DIR, int VK, bool CNT>
__device__ __forceinline__ void engine_iter(TileLds<RK, VK, CNT>& S, const EngineParams& P, int it) {
  using L = TileLds<RK, VK, CNT>;
  constexpr int TH = L::TH, TW = L::TW, HW = L::HW, NC = L::NC, NH = L::NH;
  const int tid = threadIdx.x;
  const float pf = (float)P.p;
  const int n_active = ld_dev(P.nlist + it % 3);
  const int32_t* list = (it & 1) ? P.list1 : P.list0;
  // List (it + 2) % 3 was read in the previous iteration and is filled in
  // the next one: clear it now (an atomic store, like the additions).
  if (blockIdx.x == 0 && tid == 0)
    __hip_atomic_store(P.nlist + (it + 2) % 3, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  for (int e = blockIdx.x; e < n_active; e += gridDim.x) {
    const int64_t t = list[e];
    const int64_t tr = t / P.ntc, tc = t - tr * P.ntc;
    const int64_t r0 = tr * TH, c0 = tc * TW;
    const int th = (int)(P.nrows - r0 < TH ? P.nrows - r0 : TH);
    const int tw = (int)(P.ncols - c0 < TW ? P.ncols - c0 : TW);

    // 1. Load codes (and MFD split data) with a one-cell halo.
    for (int h = tid; h < NH; h += ENG_THREADS) {
      const int hr = h / HW - 1, hc = h % HW - 1;
      const int64_t gr = r0 + hr, gc = c0 + hc;
      const bool in_grid = gr >= 0 && gr < P.nrows && gc >= 0 && gc < P.ncols;
      const int64_t g = gr * P.ncols + gc;
      S.code[h] = in_grid ? P.code[g] : (RK == RK_SINGLE ? SINK : (uint8_t)0);
      if (RK == RK_MULTI) {
        S.z[h] = in_grid ? P.z[g] : INFINITY;
        if (VK == VK_FF) {
          S.rs[h] = in_grid ? P.rs32[g] : 0.0f;
          S.iw[h] = in_grid ? P.iw32[g] : 0.0f;
          S.dd[h] = in_grid ? P.d32[g] : 0.0f;
        } else if (VK == VK_F64) {
          S.iw64[h] = in_grid ? P.iw64[g] : 0.0;
        }
      }
    }
    // 2. Cell state.
    for (int l = tid; l < NC; l += ENG_THREADS) {
      const int lr = l / TW, lc = l % TW;
      uint32_t st = ST_DONE | ST_PREV;  // outside the grid: never written
      if (lr < th && lc < tw) {
        const int64_t g = (r0 + lr) * P.ncols + (c0 + lc);
        st = P.done[g] ? (ST_DONE | ST_PREV) : ((uint32_t)P.ext[g] << 16);
      }
      S.st[l] = st;
    }
    if (tid == 0) {
      S.nf[0] = 0;
      S.nf[1] = 0;
      S.ndone = 0;
    }
    __syncthreads();

    // 3. For each unfinished cell: in-tile inputs still pending, and the
    //    part of its value that is already known -- its source term plus
    //    every input that was final when the tile was loaded (inputs in
    //    other tiles, inputs of this tile finished in earlier launches).  A
    //    cell with an unfinished input in another tile cannot finish in this
    //    activation; it is skipped.
    for (int l = tid; l < NC; l += ENG_THREADS) {
      const uint32_t st = S.st[l];
      if (st & ST_DONE) continue;
      const bool ext_ready = ((st >> 16) & 0xFFu) == 0u;
      const int lr = l / TW, lc = l % TW;
      const int h = (lr + 1) * HW + (lc + 1);
      const int64_t gr = r0 + lr, gc = c0 + lc;
      const int64_t g = gr * P.ncols + gc;
      const uint8_t ci = S.code[h];
      uint32_t pend = 0;
      ff vf = {0.0f, 0.0f};
      double vd = 0.0;
      uint64_t cn = 1;
      if (ext_ready) {
        if (VK == VK_FF) {
          if (P.src64) {
            const double d = P.src64[g];
            vf.hi = (float)d;
            vf.lo = (float)(d - (double)vf.hi);
          } else {
            vf.hi = P.src32 ? P.src32[g] : 1.0f;
          }
        }
        if (VK == VK_F64) vd = P.src64 ? P.src64[g] : (P.src32 ? (double)P.src32[g] : 1.0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int hn = h + nb_dr(k) * HW + nb_dc(k);
        const bool input = (DIR == DIR_FWD) ? is_recv(RK, S.code[hn], 7 - k) : is_recv(RK, ci, k);
        if (!input) continue;
        const int nr = lr + nb_dr(k), nc = lc + nb_dc(k);
        if (gr + nb_dr(k) < 0 || gr + nb_dr(k) >= P.nrows || gc + nb_dc(k) < 0 || gc + nb_dc(k) >= P.ncols)
          continue;  // malformed code pointing off the grid
        const bool same = nr >= 0 && nr < th && nc >= 0 && nc < tw;
        if (same && !(S.st[nr * TW + nc] & ST_DONE)) {
          ++pend;
          continue;
        }
        if (!ext_ready) continue;
        // Final input: this tile from an earlier launch (plain load) or
        // another tile, possibly finished during this launch (coherent load).
        const int64_t gn = g + nb_dr(k) * P.ncols + nb_dc(k);
        if (VK == VK_FF) {
          ff vj = same ? ff{P.vhi[gn], P.vlo[gn]} : ff{ld_dev(P.vhi + gn), ld_dev(P.vlo + gn)};
          if (RK == RK_MULTI) vj = edge_ff<DIR>(S, vj, h, hn, k, pf);
          vf = ff_add(vf, vj);
        }
        if (VK == VK_F64) {
          double vj = same ? P.v64[gn] : ld_dev(P.v64 + gn);
          if (RK == RK_MULTI) vj *= edge_f64<DIR>(S, h, hn, k, P.p);
          vd += vj;
        }
        if (CNT) cn += same ? P.cnt[gn] : ld_dev(P.cnt + gn);
      }
      S.st[l] = st | pend;
      if (ext_ready) {
        if (VK == VK_FF) S.vff[l] = vf;
        if (VK == VK_F64) S.v64[l] = vd;
        if (CNT) S.cnt[l] = cn;
      }
    }
    __syncthreads();

    // 4. Initial frontier: unfinished cells with no pending input.
    for (int l0 = 0; l0 < NC; l0 += ENG_THREADS) {
      const int l = l0 + tid;
      const uint32_t st = S.st[l];
      push_front(S, 0, !(st & ST_DONE) && (st & 0xFFu) == 0 && ((st >> 16) & 0xFFu) == 0, l);
    }

    // 5. Peel, in LDS only: a frontier cell adds the values of its in-tile
    //    inputs finished in this activation (in neighbour order) to its known
    //    part, then releases its in-tile outputs.
    int cur = 0;
    for (;;) {
      __syncthreads();
      const int nf = S.nf[cur];
      if (nf == 0) break;
      if (tid == 0) S.ndone += nf;
      for (int i0 = 0; i0 < nf; i0 += ENG_THREADS) {
        const int idx = i0 + tid;
        const bool act = idx < nf;
        const int l = act ? S.front[cur][idx] : 0;
        const int lr = l / TW, lc = l % TW;
        const int h = (lr + 1) * HW + (lc + 1);
        const uint8_t ci = act ? S.code[h] : (uint8_t)0;
        if (act) {
          ff vf = {0.0f, 0.0f};
          double vd = 0.0;
          uint64_t cn = 0;
          if (VK == VK_FF) vf = S.vff[l];
          if (VK == VK_F64) vd = S.v64[l];
          if (CNT) cn = S.cnt[l];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int hn = h + nb_dr(k) * HW + nb_dc(k);
            const bool input = (DIR == DIR_FWD) ? is_recv(RK, S.code[hn], 7 - k) : is_recv(RK, ci, k);
            if (!input) continue;
            const int nr = lr + nb_dr(k), nc = lc + nb_dc(k);
            if (!(nr >= 0 && nr < th && nc >= 0 && nc < tw)) continue;
            const int ln = nr * TW + nc;
            if (S.st[ln] & ST_PREV) continue;  // already in the known part
            if (VK == VK_FF) {
              ff vj = S.vff[ln];
              if (RK == RK_MULTI) vj = edge_ff<DIR>(S, vj, h, hn, k, pf);
              vf = ff_add(vf, vj);
            }
            if (VK == VK_F64) {
              double vj = S.v64[ln];
              if (RK == RK_MULTI) vj *= edge_f64<DIR>(S, h, hn, k, P.p);
              vd += vj;
            }
            if (CNT) cn += S.cnt[ln];
          }
          if (VK == VK_FF) S.vff[l] = vf;
          if (VK == VK_F64) S.v64[l] = vd;
          if (CNT) S.cnt[l] = cn;
          atomicOr(&S.st[l], ST_DONE);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          bool ready = false;
          int ln = 0;
          if (act) {
            const int hn = h + nb_dr(k) * HW + nb_dc(k);
            const bool out = (DIR == DIR_FWD) ? is_recv(RK, ci, k) : is_recv(RK, S.code[hn], 7 - k);
            const int nr = lr + nb_dr(k), nc = lc + nb_dc(k);
            if (out && nr >= 0 && nr < th && nc >= 0 && nc < tw) {
              ln = nr * TW + nc;
              const uint32_t old = atomicSub(&S.st[ln], 1u);
              ready = (old & 0xFFu) == 1u && ((old >> 16) & 0xFFu) == 0u;
            }
          }
          push_front(S, cur ^ 1, ready, ln);
        }
      }
      __syncthreads();
      if (tid == 0) S.nf[cur] = 0;
      cur ^= 1;
    }

    // 6. Write the cells finished in this activation (coalesced rows).
    //    Values that other tiles consume go out device-coherently, and the
    //    stores complete before their consumers' counters are released.
    for (int l = tid; l < NC; l += ENG_THREADS) {
      const uint32_t st = S.st[l];
      if (!(st & ST_DONE) || (st & ST_PREV)) continue;
      const int lr = l / TW, lc = l % TW;
      const int h = (lr + 1) * HW + (lc + 1);
      const int64_t g = (r0 + lr) * P.ncols + (c0 + lc);
      const bool lv = leaves<RK, DIR>(S, h, lr, lc, th, tw);
      if (VK == VK_FF) {
        if (lv) {
          st_dev(P.vhi + g, S.vff[l].hi);
          st_dev(P.vlo + g, S.vff[l].lo);
        } else {
          P.vhi[g] = S.vff[l].hi;
          P.vlo[g] = S.vff[l].lo;
        }
      }
      if (VK == VK_F64) {
        if (lv) st_dev(P.v64 + g, S.v64[l]);
        else P.v64[g] = S.v64[l];
      }
      if (CNT) {
        if (lv) st_dev(P.cnt + g, S.cnt[l]);
        else P.cnt[g] = S.cnt[l];
      }
      P.done[g] = 1;
    }
    wait_stores();
    // 7. Release the external outputs of the newly finished cells.
    for (int l = tid; l < NC; l += ENG_THREADS) {
      const uint32_t st = S.st[l];
      if (!(st & ST_DONE) || (st & ST_PREV)) continue;
      const int lr = l / TW, lc = l % TW;
      const int h = (lr + 1) * HW + (lc + 1);
      const int64_t gr = r0 + lr, gc = c0 + lc;
      const uint8_t ci = S.code[h];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int hn = h + nb_dr(k) * HW + nb_dc(k);
        const bool out = (DIR == DIR_FWD) ? is_recv(RK, ci, k) : is_recv(RK, S.code[hn], 7 - k);
        const int nr = lr + nb_dr(k), nc = lc + nb_dc(k);
        if (!out || (nr >= 0 && nr < th && nc >= 0 && nc < tw)) continue;
        const int64_t ngr = gr + nb_dr(k), ngc = gc + nb_dc(k);
        if (ngr >= 0 && ngr < P.nrows && ngc >= 0 && ngc < P.ncols)
          signal_external(P, it, ngr * P.ncols + ngc, ngr, ngc);
      }
    }
    if (tid == 0 && S.ndone) atomicAdd(P.remaining, (unsigned long long)(-(long long)S.ndone));
    __syncthreads();
  }
}

// Barrier of all workgroups of a persistent launch: arrivals only count up,
// and iteration `epoch` is complete once (epoch + 1) * gridDim.x have
// arrived.  The fences make every global write before the barrier visible
// to every workgroup after it (the L2 of one XCD is not coherent with the
// others).  The wait is bounded: false when some workgroup never arrived
// (the launch's workgroups were not all resident).
__device__ bool grid_sync(unsigned long long* bar, int epoch) {
  __threadfence();
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    const unsigned long long target = (unsigned long long)(epoch + 1) * gridDim.x;
    atomicAdd(bar, 1ull);
    ok = 0;
    for (int i = 0; i < (1 << 24); ++i) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
  }
  __syncthreads();
  __threadfence();
  return ok != 0;
}

// The whole peeling run in one launch: iterations separated by grid
// barriers, until an iteration queues no tile for the next one -- every
// cell is final, or (cells left over) the routing has a cycle.  Every
// workgroup reads the same list length after the same barrier, so all of
// them leave together.
template <int RK, int DIR, int VK, bool CNT>
__global__ __launch_bounds__(ENG_THREADS) void k_engine_run(EngineParams P) {
  __shared__ TileLds<RK, VK, CNT> S;
  if (P.gate && *P.gate == 0) return;  // uniform: another path finished the solve
  for (int it = 0;; ++it) {
    engine_iter<RK, DIR, VK, CNT>(S, P, it);
    if (!grid_sync(P.bar, it)) {
      if (threadIdx.x == 0) set_status(P.status, FR_ERR_STALL);
      return;
    }
    if (ld_dev(P.nlist + (it + 1) % 3) == 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0 && ld_dev(reinterpret_cast<const uint64_t*>(P.remaining)) != 0)
        set_status(P.status, FR_ERR_NOTDAG);
      return;
    }
  }
}

// ---------------------------------------------------------------------------
// Mass balance (Section 4 verification): {sum over sinks of q, sum of rain},
// float64, two deterministic stages.
template <int RK, int VK>
__global__ __launch_bounds__(256) void k_mass_partial(EngineParams P, double* partial) {
  if (P.gate && *P.gate == 0) return;
  const int64_t n = P.nrows * P.ncols;
  double s = 0.0, t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t ci = P.code[i];
    const bool sink = RK == RK_SINGLE ? (ci > 7) : (ci == 0);
    if (sink) s += VK == VK_FF ? (double)P.vhi[i] + (double)P.vlo[i] : P.v64[i];
    t += P.src64 ? P.src64[i] : (P.src32 ? (double)P.src32[i] : 1.0);
  }
  __shared__ double rs[256], rt[256];
  rs[threadIdx.x] = s;
  rt[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rt[threadIdx.x] += rt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = rs[0];
    partial[2 * blockIdx.x + 1] = rt[0];
  }
}

// Runs when gate is NULL, or when (*gate != 0) == open.
__global__ __launch_bounds__(256) void k_mass_final(const double* partial, int nblocks, double* out,
                                                    const int32_t* gate, int open) {
  if (gate && ((*gate != 0) != (open != 0))) return;
  __shared__ double rs[256], rt[256];
  double s = 0.0, t = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    s += partial[2 * b];
    t += partial[2 * b + 1];
  }
  rs[threadIdx.x] = s;
  rt[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rt[threadIdx.x] += rt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rs[0];
    out[1] = rt[0];
  }
}

__global__ void k_set_status(int32_t* st, int32_t code) {
  if (threadIdx.x == 0) atomicCAS(st, 0, code);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ void k_zero_f64(double* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

int init_grid(const EngineParams& P) {
  const int64_t n = P.nrows * P.ncols;
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (int)(b < 1 ? 1 : b);
}

template <int RK, int DIR>
hipError_t init_dispatch_vk(ValKind vk, const EngineParams& P, hipStream_t s) {
  const int g = init_grid(P);
  switch (vk) {
    case VK_FF: hipLaunchKernelGGL((k_engine_init<RK, DIR, VK_FF>), dim3(g), dim3(256), 0, s, P); break;
    case VK_F64: hipLaunchKernelGGL((k_engine_init<RK, DIR, VK_F64>), dim3(g), dim3(256), 0, s, P); break;
    default: hipLaunchKernelGGL((k_engine_init<RK, DIR, VK_NONE>), dim3(g), dim3(256), 0, s, P); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_engine_init(const EngineConfig& cfg, const EngineParams& P, hipStream_t s) {
  if (cfg.rk == RK_SINGLE)
    return cfg.dir == DIR_FWD ? init_dispatch_vk<RK_SINGLE, DIR_FWD>(cfg.vk, P, s)
                              : init_dispatch_vk<RK_SINGLE, DIR_ADJ>(cfg.vk, P, s);
  return cfg.dir == DIR_FWD ? init_dispatch_vk<RK_MULTI, DIR_FWD>(cfg.vk, P, s)
                            : init_dispatch_vk<RK_MULTI, DIR_ADJ>(cfg.vk, P, s);
}

// Workgroups of the persistent engine: as many as can be resident at once
// (at most two per compute unit), so that its grid barriers always complete.
template <int RK, int DIR, int VK, bool CNT>
hipError_t run_t(const EngineParams& P, hipStream_t s) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_engine_run<RK, DIR, VK, CNT>, ENG_THREADS, 0);
  if (e != hipSuccess) return e;
  if (per < 1 || cus < 1) return hipErrorLaunchFailure;
  int64_t grid = (int64_t)cus * (per > 2 ? 2 : per);
  const int64_t ntiles = (int64_t)P.ntr * P.ntc;
  if (grid > ntiles) grid = ntiles;
  hipLaunchKernelGGL((k_engine_run<RK, DIR, VK, CNT>), dim3((unsigned)(grid < 1 ? 1 : grid)), dim3(ENG_THREADS), 0, s,
                     P);
  return hipGetLastError();
}

hipError_t launch_engine_run(const EngineConfig& cfg, const EngineParams& P, hipStream_t s) {
  if (cfg.rk == RK_SINGLE) {
    if (cfg.dir == DIR_FWD) {
      if (cfg.counts) {
        switch (cfg.vk) {
          case VK_FF: return run_t<RK_SINGLE, DIR_FWD, VK_FF, true>(P, s);
          case VK_F64: return run_t<RK_SINGLE, DIR_FWD, VK_F64, true>(P, s);
          default: return run_t<RK_SINGLE, DIR_FWD, VK_NONE, true>(P, s);
        }
      }
      if (cfg.vk == VK_FF) return run_t<RK_SINGLE, DIR_FWD, VK_FF, false>(P, s);
      return run_t<RK_SINGLE, DIR_FWD, VK_F64, false>(P, s);
    }
    if (cfg.vk == VK_FF) return run_t<RK_SINGLE, DIR_ADJ, VK_FF, false>(P, s);
    return run_t<RK_SINGLE, DIR_ADJ, VK_F64, false>(P, s);
  }
  if (cfg.dir == DIR_FWD) {
    if (cfg.vk == VK_FF) return run_t<RK_MULTI, DIR_FWD, VK_FF, false>(P, s);
    return run_t<RK_MULTI, DIR_FWD, VK_F64, false>(P, s);
  }
  if (cfg.vk == VK_FF) return run_t<RK_MULTI, DIR_ADJ, VK_FF, false>(P, s);
  return run_t<RK_MULTI, DIR_ADJ, VK_F64, false>(P, s);
}

hipError_t launch_mass(RuleKind rk, ValKind vk, const EngineParams& P, double* partial, int nblocks,
                       double* mass_out, hipStream_t s) {
  if (rk == RK_SINGLE) {
    if (vk == VK_FF) hipLaunchKernelGGL((k_mass_partial<RK_SINGLE, VK_FF>), dim3(nblocks), dim3(256), 0, s, P, partial);
    else hipLaunchKernelGGL((k_mass_partial<RK_SINGLE, VK_F64>), dim3(nblocks), dim3(256), 0, s, P, partial);
  } else {
    if (vk == VK_FF) hipLaunchKernelGGL((k_mass_partial<RK_MULTI, VK_FF>), dim3(nblocks), dim3(256), 0, s, P, partial);
    else hipLaunchKernelGGL((k_mass_partial<RK_MULTI, VK_F64>), dim3(nblocks), dim3(256), 0, s, P, partial);
  }
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, partial, nblocks, mass_out, P.gate, 1);
  return hipGetLastError();
}

hipError_t launch_mass_final(const double* partial, int nblocks, double* out, const int32_t* skip,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, partial, nblocks, out, skip, 0);
  return hipGetLastError();
}

hipError_t launch_mass_final_if(const double* partial, int nblocks, double* out, const int32_t* open,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, partial, nblocks, out, open, 1);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_set_status(int32_t* status, int32_t code, hipStream_t s) {
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, status, code);
  return hipGetLastError();
}

}  // namespace fr
