// Local flow routing kernels (Section 2.1 D8/D4 receivers; Appendix A
// lower-neighbour sets for multiple-flow-direction routing).
//
// Streaming 3x3 stencil.  A workgroup owns a strip of 1024 columns x RPB
// rows; each lane owns 4 consecutive columns and slides a 3-row window down
// the strip in registers, so every elevation is read from HBM once (plus one
// halo row per strip).  Left/right neighbours come from the adjacent lanes by
// cross-lane shuffles; only wave-edge lanes load them from memory.  Off-grid
// neighbours are represented by +inf, which is never "lower".
#include <math.h>

#include "fr_internal.hpp"

namespace fr {
namespace {

constexpr int RCV_THREADS = 256;
constexpr int RCV_COLS = RCV_THREADS * 4;  // columns per workgroup
constexpr int RCV_RPB = 32;                // rows per workgroup

struct Row6 {
  float v[6];  // columns c0-1 .. c0+4
};

// A row as loaded: this lane's four columns, plus (lanes 0 and 63) the
// column just outside the lane group.  Cross-lane assembly happens later, so
// the load can stay in flight while other rows are computed.
struct RawRow {
  float a[4];
  float side;
};

template <bool VEC>
__device__ __forceinline__ RawRow load_raw(const float* __restrict__ z, int64_t nrows, int64_t ncols,
                                           int64_t r, int64_t c0, int lane) {
  RawRow x;
  x.a[0] = x.a[1] = x.a[2] = x.a[3] = INFINITY;
  x.side = INFINITY;
  if (r >= 0 && r < nrows) {
    const float* rp = z + r * ncols;
    if (VEC && c0 + 3 < ncols) {
      const float4 q = *reinterpret_cast<const float4*>(rp + c0);
      x.a[0] = q.x; x.a[1] = q.y; x.a[2] = q.z; x.a[3] = q.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (c0 + j < ncols) x.a[j] = rp[c0 + j];
    }
    if (lane == 0 && c0 - 1 >= 0 && c0 - 1 < ncols) x.side = rp[c0 - 1];
    if (lane == 63 && c0 + 4 < ncols) x.side = rp[c0 + 4];
  }
  return x;
}

__device__ __forceinline__ Row6 assemble(const RawRow& x, int lane) {
  Row6 out;
  float left = __shfl_up(x.a[3], 1, 64);
  float right = __shfl_down(x.a[0], 1, 64);
  if (lane == 0) left = x.side;
  if (lane == 63) right = x.side;
  out.v[0] = left; out.v[1] = x.a[0]; out.v[2] = x.a[1]; out.v[3] = x.a[2]; out.v[4] = x.a[3];
  out.v[5] = right;
  return out;
}

// Code of the cell at column offset j (1..4) of the middle row.
template <int RULE>
__device__ __forceinline__ uint8_t cell_code(const Row6& up, const Row6& mid, const Row6& dn, int j) {
  // Neighbour elevations in row-major window order; "up" is the previous row
  // in memory (row - 1).
  const float zk[8] = {up.v[j - 1], up.v[j], up.v[j + 1], mid.v[j - 1],
                       mid.v[j + 1], dn.v[j - 1], dn.v[j], dn.v[j + 1]};
  return route_code<RULE>(mid.v[j], zk);
}

template <int RULE, bool VEC>
__global__ __launch_bounds__(RCV_THREADS) void k_receivers(const float* __restrict__ z, int64_t nrows,
                                                           int64_t ncols, uint8_t* __restrict__ code,
                                                           int32_t* status) {
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * RCV_COLS + (int64_t)threadIdx.x * 4;
  const int64_t r0 = (int64_t)blockIdx.y * RCV_RPB;
  const int64_t r1 = r0 + RCV_RPB < nrows ? r0 + RCV_RPB : nrows;
  Row6 up = assemble(load_raw<VEC>(z, nrows, ncols, r0 - 1, c0, lane), lane);
  Row6 mid = assemble(load_raw<VEC>(z, nrows, ncols, r0, c0, lane), lane);
  RawRow dn_raw = load_raw<VEC>(z, nrows, ncols, r0 + 1, c0, lane);
  bool bad = false;
  for (int64_t r = r0; r < r1; ++r) {
    // Row r+2 is fetched now and used two iterations later.
    const RawRow nn_raw = load_raw<VEC>(z, nrows, ncols, r + 2, c0, lane);
    const Row6 dn = assemble(dn_raw, lane);
    uint8_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      o[j] = cell_code<RULE>(up, mid, dn, j + 1);
      if (c0 + j < ncols && !isfinite(mid.v[j + 1])) bad = true;
    }
    uint8_t* op = code + r * ncols + c0;
    if (VEC && c0 + 3 < ncols) {
      *reinterpret_cast<uint32_t*>(op) =
          (uint32_t)o[0] | ((uint32_t)o[1] << 8) | ((uint32_t)o[2] << 16) | ((uint32_t)o[3] << 24);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (c0 + j < ncols) op[j] = o[j];
    }
    up = mid;
    mid = dn;
    dn_raw = nn_raw;
  }
  if (bad && status) atomicCAS(status, 0, FR_ERR_NONFINITE);
}

template <int RULE>
hipError_t launch_rule(const float* z, int64_t nrows, int64_t ncols, uint8_t* code, int32_t* status,
                       hipStream_t s) {
  const dim3 grid((unsigned)((ncols + RCV_COLS - 1) / RCV_COLS),
                  (unsigned)((nrows + RCV_RPB - 1) / RCV_RPB));
  const bool vec = (ncols % 4 == 0) && ((uintptr_t)z % 16 == 0) && ((uintptr_t)code % 4 == 0);
  if (vec)
    hipLaunchKernelGGL((k_receivers<RULE, true>), grid, dim3(RCV_THREADS), 0, s, z, nrows, ncols, code,
                       status);
  else
    hipLaunchKernelGGL((k_receivers<RULE, false>), grid, dim3(RCV_THREADS), 0, s, z, nrows, ncols, code,
                       status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_receivers(const float* z, int64_t nrows, int64_t ncols, int rule, uint8_t* code,
                            int32_t* status, hipStream_t s) {
  switch (rule) {
    case FR_D8: return launch_rule<FR_D8>(z, nrows, ncols, code, status, s);
    case FR_D4: return launch_rule<FR_D4>(z, nrows, ncols, code, status, s);
    default: return launch_rule<FR_MFD>(z, nrows, ncols, code, status, s);
  }
}

}  // namespace fr
