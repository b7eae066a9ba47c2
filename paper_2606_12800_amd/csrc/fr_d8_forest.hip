// Phase B of the row-sweep path: the exit forest (see fr_d8_a.hip), and the
// element-wise steps of the (I - X)(I + X) block iteration.
#include "fr_d8.hpp"

namespace fr {
namespace {
// ---------------------------------------------------------------------------
// Phase B: exit forest.  The link step turns each exit's local sum into
// fixed point and points it at the exit its water reaches next (block
// iterations: only inside its block).  An exit list that overflowed its
// capacity opens the engine's gate instead (block iterations: an error).
__device__ __forceinline__ int64_t blk_row(const D8Params& P, int64_t r) { return r / ((int64_t)P.th * P.bt_r); }
__device__ __forceinline__ int64_t blk_col(const D8Params& P, int64_t c) { return c / ((int64_t)TW * P.bt_c); }

// Link: each exit's local sum into fixed point (sum buffer 0; both
// pending buffers cleared), and its parent -- the exit its water reaches
// next (block iterations: only inside its block).  An exit list that
// overflowed its capacity opens the engine's gate instead (block
// iterations: an error).
template <int VK, bool CNT, bool ITER>
__global__ __launch_bounds__(256) void k_d8_link(D8Params P) {
  const uint32_t n = *P.n_exits;
  if (n > P.cap) {  // uniform
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (ITER) set_status(P.status, FR_ERR_CAPACITY);
      else P.ctl->fallback = 1;
    }
    return;
  }
  const int E = VK != VK_NONE ? fx_exponent<VK>(P, n) : 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (VK != VK_NONE) {
      P.ex_fx[1][i] = 0;
      P.ex_fx[2][i] = 0;
    }
    if (CNT) {
      P.ex_cnt[1][i] = 0;
      P.ex_cnt[2][i] = 0;
    }
    const uint32_t ec = P.ex_cell[i];
    uint32_t a = NONE;
    if (ec == NONE) {  // a hole of a phase-A chunk: no water, no parent
      if (VK != VK_NONE) P.ex_fx[0][i] = 0;
      if (CNT) P.ex_cnt[0][i] = 0;
      P.anc[0][i] = NONE;
      continue;
    }
    if (VK == VK_FF) P.ex_fx[0][i] = (u128)(fx_from(P.ex_hi[i], E) + fx_from(P.ex_lo[i], E));
    if (VK == VK_F64) P.ex_fx[0][i] = (u128)fx_from(P.ex_d[i], E);
    const int64_t e = ec;
    const int cd = P.code[e];
    const int64_t x = e + (int64_t)nb_dr(cd) * P.ncols + nb_dc(cd);
    bool leave = false;
    if (ITER) {
      const int64_t er = e / P.ncols, xr = x / P.ncols;
      leave = blk_row(P, er) != blk_row(P, xr) || blk_col(P, e - er * P.ncols) != blk_col(P, x - xr * P.ncols);
    }
    const int64_t rt = leave ? -1 : (int64_t)P.root_of[x];
    if (leave) {
      // Water leaving the block: passed on by the next iteration.
    } else if (rt >= 0 && rt < P.nrows * P.ncols) {
      const int64_t rr = rt / P.ncols, rc = rt - rr * P.ncols;
      const int rcd = P.code[rt];
      bool sink = rcd > 7;
      if (!sink) {
        const int64_t tr = rr + nb_dr(rcd), tc = rc + nb_dc(rcd);
        sink = tr < 0 || tr >= P.nrows || tc < 0 || tc >= P.ncols;
      }
      if (!sink) {
        a = P.node_of[rt];
        if (a >= n) {  // inconsistent bookkeeping: never follow it
          a = NONE;
          set_status(P.status, FR_ERR_BADCODE);
        }
      }
    } else {
      set_status(P.status, FR_ERR_BADCODE);
    }
    P.anc[0][i] = a;
  }
}

// Round j of pointer doubling, one launch.  anc[j & 1] points 2^j exits
// down (or NONE).  Each exit first takes in the additions round j - 1 left
// for it in pending buffer 1 + ((j - 1) & 1) (clearing them): its sum is
// then its subtree within distance < 2^j.  It adds that sum to its
// ancestor's pending buffer 1 + (j & 1) (exact integer additions: the
// result does not depend on their order) and jumps its pointer into
// anc[(j + 1) & 1].  Nothing else reads or writes an exit's own sum, so
// one launch per round suffices.  Flag slot j % 3 says round j left work; a
// round whose predecessor left none returns at once, so the fixed sequence
// of launches stops early on the device.  The last round with work records
// its pending buffer (the totals add it); work left after the last launch
// (a forest deeper than its exit count) proves a cycle.
__device__ __forceinline__ int32_t* round_flag(const D8Params& P, int j) { return &P.flags[4 + j % 3]; }

template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_round(D8Params P, int j, int last) {
  // Slot j + 1 (last set by round j - 2, read by round j - 1) is cleared by
  // every round, idle or not, so that an idle round's successor is idle too.
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(round_flag(P, j + 1), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t n = *P.n_exits;
  if (n > P.cap) return;  // uniform
  if (j > 0 && __hip_atomic_load(round_flag(P, j - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.ctl->forest_final = 1 + (j & 1);
  const int in = 1 + ((j + 1) & 1), out = 1 + (j & 1);  // (j - 1) & 1 == (j + 1) & 1
  const uint32_t* anc = P.anc[j & 1];
  uint32_t* anc2 = P.anc[(j + 1) & 1];
  __shared__ int s_active;
  if (threadIdx.x == 0) s_active = 0;
  __syncthreads();
  bool active = false;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t a = anc[i];
    // An exit's own sum is read only when it changes or is passed on.
    u128 v = 0;
    unsigned long long c = 0;
    if (VK != VK_NONE) {
      const u128 d = j > 0 ? P.ex_fx[in][i] : (u128)0;
      if (d != 0 || a != NONE) v = P.ex_fx[0][i];
      if (d != 0) {
        v += d;
        P.ex_fx[0][i] = v;
        P.ex_fx[in][i] = 0;
      }
    }
    if (CNT) {
      const unsigned long long d = j > 0 ? P.ex_cnt[in][i] : 0ull;
      if (d != 0 || a != NONE) c = P.ex_cnt[0][i];
      if (d != 0) {
        c += d;
        P.ex_cnt[0][i] = c;
        P.ex_cnt[in][i] = 0;
      }
    }
    uint32_t a2 = NONE;
    if (a != NONE) {
      if (VK != VK_NONE && v != 0) atomic_add_fx(&P.ex_fx[out][a], v);
      if (CNT && c != 0) atomicAdd(reinterpret_cast<unsigned long long*>(&P.ex_cnt[out][a]), c);
      a2 = anc[a];
    }
    anc2[i] = a2;
    active |= (a2 != NONE);
  }
  // One store per workgroup, and only while the flag is still clear: an
  // atomic from every wavefront on one word serialises the whole kernel.
  if (__ballot(active) && (threadIdx.x & 63) == 0) s_active = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_active) {
    if (last) set_status(P.status, FR_ERR_NOTDAG);
    else if (__hip_atomic_load(round_flag(P, j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      __hip_atomic_store(round_flag(P, j), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The totals -- sums plus the last round's pending additions -- back from
// fixed point into float-float or float64, where phase C reads them (the
// pointer buffers' memory, free again); counts into sum buffer 0.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_totals(D8Params P) {
  const uint32_t n = *P.n_exits;
  if (n > P.cap) return;  // uniform
  const int f = P.ctl->forest_final;
  const int E = VK != VK_NONE ? fx_exponent<VK>(P, n) : 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (CNT) P.ex_cnt[0][i] += P.ex_cnt[f][i];
    if (VK == VK_NONE) continue;
    const i128 v = (i128)(P.ex_fx[0][i] + P.ex_fx[f][i]);
    if (VK == VK_FF) {
      const ff t = fx_to_ff(v, E);
      P.tot_hi[i] = t.hi;
      P.tot_lo[i] = t.lo;
    } else {
      P.tot_d[i] = fx_to_double(v, E);
    }
  }
}

__global__ __launch_bounds__(256) void k_bi_combine(int mode, int64_t n, const double* bq, const uint64_t* bc,
                                                    const double* wq, const uint64_t* wc, double* tq,
                                                    uint64_t* tc, double* oq, uint64_t* oc, int32_t* changed) {
  bool chg = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (mode == 0) {
      if (tq) tq[i] = bq[i] - wq[i] + tq[i];
      if (tc) tc[i] = bc[i] - wc[i] + tc[i];
    } else if (mode == 1) {
      if (oq) oq[i] = wq[i] + tq[i] + oq[i];
      if (oc) {
        const uint64_t v = wc[i] + tc[i] + oc[i];
        oc[i] = v;
        chg |= v != wc[i];
      }
    } else {
      if (oq) oq[i] = 0.0;
      if (oc) oc[i] = 0;
    }
  }
  if (mode == 1 && __ballot(chg) && (threadIdx.x & 63) == 0 && changed && *(volatile int32_t*)changed == 0)
    *changed = 1;
}

}  // namespace

// Workgroups of the forest kernels: enough for the exits of a large grid,
// few enough that a launch with nothing to do costs little.
unsigned forest_grid(uint32_t cap) {
  const uint32_t b = (cap + 255) / 256;
  return b < 1 ? 1u : (b > 2048 ? 2048u : b);
}

// Rounds enqueued: a forest of cap exits is at most cap deep, and after
// round j every pointer spans 2^(j+1) exits; one more round than that
// bound needs, so that work left in the last one proves a cycle.
int forest_rounds(uint32_t cap) {
  int r = 0;
  while (r < 32 && ((uint64_t)1 << r) < (uint64_t)cap + 1) ++r;
  return r + 1;
}

template <int VK, bool CNT, bool ITER>
hipError_t forest_t(const D8Params& P, hipStream_t s) {
  const dim3 g(forest_grid(P.cap)), b(256);
  hipLaunchKernelGGL((k_d8_link<VK, CNT, ITER>), g, b, 0, s, P);
  const int R = forest_rounds(P.cap);
  for (int j = 0; j < R; ++j) hipLaunchKernelGGL((k_d8_round<VK, CNT>), g, b, 0, s, P, j, j == R - 1 ? 1 : 0);
  hipLaunchKernelGGL((k_d8_totals<VK, CNT>), g, b, 0, s, P);
  return hipGetLastError();
}

hipError_t launch_d8_forest(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s) {
  if (vk == VK_FF) {
    if (iter) return hipErrorInvalidValue;
    return cnt ? forest_t<VK_FF, true, false>(P, s) : forest_t<VK_FF, false, false>(P, s);
  }
  if (vk == VK_F64) {
    if (iter) return cnt ? forest_t<VK_F64, true, true>(P, s) : forest_t<VK_F64, false, true>(P, s);
    return cnt ? forest_t<VK_F64, true, false>(P, s) : forest_t<VK_F64, false, false>(P, s);
  }
  return iter ? forest_t<VK_NONE, true, true>(P, s) : forest_t<VK_NONE, true, false>(P, s);
}

hipError_t launch_bi_combine(int mode, int64_t n, const double* bq, const uint64_t* bc, const double* wq,
                             const uint64_t* wc, double* tq, uint64_t* tc, double* oq, uint64_t* oc,
                             int32_t* changed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_bi_combine, dim3((unsigned)blocks), dim3(256), 0, s, mode, n, bq, bc, wq, wc, tq, tc, oq,
                     oc, changed);
  return hipGetLastError();
}


}  // namespace fr
