// Phase C of the row-sweep path: the final sweep of every tile with its cut
// donors' forest totals (see fr_d8_a.hip).
#include "fr_d8.hpp"

namespace fr {
namespace {
// ---------------------------------------------------------------------------
// Phase C (and the block solve's final sweep).  Returns at once when the
// exit list overflowed: the engine, or an error, takes over.
template <int VK, bool CNT, int RAIN, bool VEC, bool ITER>
__global__ __launch_bounds__(64) void k_d8_c(D8Params P) {
  __shared__ double s_mass[2][64];
  // Row exchange for grids whose rows are not aligned to 4 cells.
  __shared__ float s_q32[VEC || VK != VK_FF ? 1 : TW];
  __shared__ double s_q64[VEC || VK != VK_F64 ? 1 : TW];
  __shared__ uint64_t s_cnt[VEC || !CNT ? 1 : TW];
  if (*P.n_exits > P.cap) return;  // uniform
  const int lane = threadIdx.x;
  const Tile T = tile_of(P, blockIdx.x);
  SweepOut o;
  if (T.border) sweep<false, VK, CNT, RAIN, VEC, true, ITER>(P, T, o, s_q32, s_q64, s_cnt);
  else sweep<false, VK, CNT, RAIN, VEC, false, ITER>(P, T, o, s_q32, s_q64, s_cnt);
  if (ITER) {
    if (__ballot(o.changed) && lane == 0 && P.it_changed) *P.it_changed = 1;
    if (o.badcode) set_status(P.status, FR_ERR_BADCODE);
    if (o.nonfinite) set_status(P.status, FR_ERR_NONFINITE);
  } else if (P.mass_part) {
    s_mass[0][lane] = o.mass[0];
    s_mass[1][lane] = o.mass[1];
    __syncthreads();
    if (lane == 0) {
      double a = 0.0, b = 0.0;
      for (int l = 0; l < 64; ++l) {
        a += s_mass[0][l];
        b += s_mass[1][l];
      }
      // Indexed by workgroup: the final reduction runs in one fixed order.
      P.mass_part[2 * blockIdx.x] = a;
      P.mass_part[2 * blockIdx.x + 1] = b;
    }
  }
}
}  // namespace

template <int VK, bool CNT, int RAIN, bool VEC, bool ITER>
struct KernelC {
  static void launch(const D8Params& P, hipStream_t s) {
    hipLaunchKernelGGL((k_d8_c<VK, CNT, RAIN, VEC, ITER>), dim3((unsigned)((int64_t)P.ntr * P.ntc)), dim3(64), 0,
                       s, P);
  }
};

hipError_t launch_d8_down(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s) {
  return d8_sweep_dispatch<KernelC>(vk, cnt, iter, P, s);
}


}  // namespace fr
