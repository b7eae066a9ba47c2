// Single-receiver (D8 / D4) accumulation by row sweeps plus a reduced exit
// forest.
//
// The water at a cell is its rain plus the water of every cell upstream of it
// (Section 2.1; the unique solution of (I - W^T) q = r, Section 2.2).  On
// tilted terrain nearly every receiver lies in the previous row (row - 1), so
// a sweep over the rows in decreasing index order visits donors before
// receivers -- it is the paper's high-to-low order restricted to that edge
// class, and like the paper's per-process solves (Section 2.4, Section 3.3)
// the grid is cut into blocks whose solves are independent:
//
//   A. Each tile (th rows x 256 columns) is swept by one wavefront, four
//      columns per lane.  Edges from row r+1 to row r inside the tile are
//      followed in registers (cross-lane shifts); every other edge --
//      leaving the tile, within a row, or toward a higher row index -- is
//      "cut".  A top-down sweep yields each cut cell's (exit's) local
//      upstream sum; a bottom-up sweep by a second wavefront of the same
//      workgroup yields, for every cell that receives over a cut edge
//      (inlet), the exit or sink where its in-tile path ends (its root).
//   B. The exits form a forest: exit e drains into exit root(receiver(e)),
//      or nowhere when that root is a sink.  Subtree sums over this forest are
//      computed by pointer doubling in ceil(log2(depth)) rounds.  These stand
//      in for the paper's C + 1 block iterations across block boundaries
//      (Section 3.3, Appendix B), collapsed to a logarithmic number of rounds.
//   C. Each tile is swept again with the totals of its cut donors added: the
//      result is final.  The float64 mass balance is reduced in the same pass.
//
// Every kernel reads the exit count from device memory, and the pointer-
// doubling rounds are a fixed sequence of launches that return at once when
// there is nothing left to do, so a solve never waits for the host.  When the
// exit list overflows its capacity (flow in every direction, as on filled
// terrain), the tile-forest path (fr_d8_tiles.hip) serves the call instead.
//
// Block iterations (the paper's I+X scheme, Section 3.3, Appendix B): with
// blocks made of bt_r x bt_c tiles, the same three phases are the exact
// block solve D^-1 -- the forest keeps only links inside a block, and water
// from donors in other blocks enters as the previous iterate (R w).
//
// Numerics.  Float32 water uses float-float (hi, lo) sums in the sweeps.  The
// forest adds exit sums as 128-bit integers in units of 2^E (E fixed per
// call from the largest exit sum and the exit count, so no sum can
// overflow); integer addition is exact and commutative, so the result does
// not depend on the order in which the atomics land, and the totals go back
// to float-float / float64 once, after the last round: every output is the
// same, bit for bit, from run to run.  Counts are exact uint64.
#include "fr_d8.hpp"

namespace fr {
namespace {
// ---------------------------------------------------------------------------
// Phase A: one workgroup of two wavefronts per tile.  Wavefront 0 runs the
// top-down local sweep (bound by HBM), wavefront 1 the bottom-up root sweep
// (bound by its instruction count); neither reads what the other writes, so
// they overlap on the compute unit.  The local sweep also reports the
// largest |local sum| of its exits, which fixes the forest's fixed-point
// unit.
// The root sweep's wavefront.
template <bool VEC>
__device__ __forceinline__ void root_wave(const D8Params& P, const Tile& T) {
  bool badcode = false;
  if (T.border) root_sweep<VEC, true>(P, T, &badcode);
  else root_sweep_interior<VEC>(P, T, &badcode);
  if (badcode) set_status(P.status, FR_ERR_BADCODE);
}

template <int VK, bool CNT, int RAIN, bool VEC, bool ITER>
__global__ __launch_bounds__(128) void k_d8_a(D8Params P) {
  // Once the exit list has overflowed, the rest of the pass is wasted: the
  // tiles not started yet return at once.
  if (__hip_atomic_load(P.n_exits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > P.cap) return;  // uniform
  const Tile T = tile_of(P, blockIdx.x);
  if (threadIdx.x >= 64) {
    root_wave<VEC>(P, T);
    return;
  }
  SweepOut o;
  if (T.border) sweep<true, VK, CNT, RAIN, VEC, true, ITER>(P, T, o);
  else sweep<true, VK, CNT, RAIN, VEC, false, ITER>(P, T, o);
  if (o.nonfinite) set_status(P.status, FR_ERR_NONFINITE);
  if (VK == VK_FF) {
    float m = o.lmax_f;
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0 && m > 0.0f) atomicMax(&P.ctl->loc_max_f, __float_as_uint(m));
  }
  if (VK == VK_F64) {
    double m = o.lmax_d;
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (threadIdx.x == 0 && m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(&P.ctl->loc_max_d), (unsigned long long)__double_as_longlong(m));
  }
}

}  // namespace

template <int VK, bool CNT, int RAIN, bool VEC, bool ITER>
struct KernelA {
  static void launch(const D8Params& P, hipStream_t s) {
    hipLaunchKernelGGL((k_d8_a<VK, CNT, RAIN, VEC, ITER>), dim3((unsigned)((int64_t)P.ntr * P.ntc)), dim3(128), 0,
                       s, P);
  }
};

hipError_t launch_d8_up(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s) {
  return d8_sweep_dispatch<KernelA>(vk, cnt, iter, P, s);
}


}  // namespace fr
