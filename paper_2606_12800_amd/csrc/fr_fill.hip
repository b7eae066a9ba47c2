// Depression filling on the GPU: the surface the priority-flood method
// produces (Section 4 fills the DEM that way before routing), computed by
// tiled relaxation instead of a global priority queue.
//
// The filled surface F solves F = z on the grid boundary and
//     F(c) = max(z(c), min over neighbours n of next(F(n)))
// elsewhere, next(x) being the next float32 above x (epsilon variant) or x.
// Starting from F = +inf inside, every update F(c) <- max(z(c), min(F(c),
// next(F(n)) ...)) can only lower F and never below the solution, so any
// order of updates, stale neighbour values included, ends at the solution;
// a state in which no update changes anything is the solution.
//
// Layout: one wavefront owns a tile of 62 x 62 cells and holds it, with its
// one-cell halo ring, as a 64 x 64 window of order-preserving uint32 keys (so
// min, max and next are integer operations, exact for subnormals): lane =
// window column while sweeping down and up the rows, lane = window row
// (after a transpose through LDS) while sweeping right and left.  Neighbours
// in other lanes arrive by DPP wavefront shifts; the halo lanes and steps are
// read once per launch and never updated, so no lane needs an edge case.
// Elevations stay in LDS, read in either orientation.  A tile repeats its
// four sweeps until a round changes nothing (or a round cap is reached),
// then writes its own cells back.  Launch k runs only the tiles next to a
// tile that changed in launch k - 1 (per-tile stamps); the host stops after
// a launch in which no tile changed.
#include "fr_internal.hpp"

namespace fr {
namespace {

constexpr int FT = 64;                     // window side = wavefront width
constexpr int FO = FT - 2;                 // cells owned per tile side
constexpr uint32_t KEY_INF = 0xFF800000u;  // key of +inf
constexpr int FILL_ROUNDS = 256;           // sweep rounds per tile and launch

// Order-preserving map of float32 to uint32 (-0 read as +0) and back.
__device__ __forceinline__ uint32_t fkey(float x) {
  uint32_t b = __float_as_uint(x);
  if (b == 0x80000000u) b = 0;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fval(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Lane i receives x of lane i - 1, or of lane i + 1; the halo lanes at the
// wavefront's ends keep their own value (never used).
__device__ __forceinline__ uint32_t from_lower(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_upper(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

// One sweep over steps 1..62 of the window, forward or backward; lanes 1..62
// update.  zk(s) is the elevation key of this lane's cell at step s.
// Returns whether any cell of this lane changed.
template <bool EPS, bool C8, bool FWD, typename ZK>
__device__ __forceinline__ bool sweep(uint32_t (&f)[FT], bool inner, ZK zk) {
  bool changed = false;
#pragma unroll
  for (int i = 1; i < FT - 1; ++i) {
    const int s = FWD ? i : FT - 1 - i;
    const uint32_t prev = f[s - 1], next = f[s + 1];
    uint32_t m = umin(prev, next);
    m = umin(m, umin(from_lower(f[s]), from_upper(f[s])));
    if (C8) {
      m = umin(m, umin(from_lower(prev), from_upper(prev)));
      m = umin(m, umin(from_lower(next), from_upper(next)));
    }
    // m <= KEY_INF, so m + 1 cannot wrap; min with f (<= KEY_INF) keeps
    // every value a valid key.
    const uint32_t cand = EPS ? m + 1u : m;
    const uint32_t nv = umax(zk(s), umin(f[s], cand));
    const bool ch = inner && nv != f[s];
    changed |= ch;
    f[s] = ch ? nv : f[s];
  }
  return changed;
}

// a[s] of lane l becomes a[l] of lane s (64 x 64 transpose through LDS).
__device__ __forceinline__ void transpose(uint32_t (&a)[FT], uint32_t (*sT)[FT + 1], int lane) {
  __syncthreads();
#pragma unroll
  for (int s = 0; s < FT; ++s) sT[s][lane] = a[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < FT; ++s) a[s] = sT[lane][s];
}

// F = z on the grid boundary, +inf elsewhere; stamps cleared.
__global__ __launch_bounds__(256) void k_fill_init(const float* __restrict__ z, float* __restrict__ F,
                                                   int64_t nr, int64_t nc, int32_t* stamp, int32_t ntiles,
                                                   int32_t* last, int32_t* status) {
  bool bad = false;
  const int64_t n = nr * nc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = z[i];
    bad |= !isfinite(v);
    const int64_t r = i / nc, c = i - r * nc;
    const bool edge = r == 0 || c == 0 || r == nr - 1 || c == nc - 1;
    F[i] = edge ? v + 0.0f : __uint_as_float(0x7F800000u);
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x)
    stamp[t] = -10;
  if (blockIdx.x == 0 && threadIdx.x == 0) *last = -1;
  if (bad && status) atomicCAS(status, 0, FR_ERR_NONFINITE);
}

// Launch k.  stamp[t] = 2k when tile t changed in launch k and converged,
// 2k + 1 when it stopped at the round cap (it then runs again itself).
template <bool EPS, bool C8>
__global__ __launch_bounds__(FT) void k_fill_tile(const float* __restrict__ z, float* F, int64_t nr, int64_t nc,
                                                  int32_t ntr, int32_t ntc, int32_t* stamp, int32_t* last,
                                                  int32_t k) {
  __shared__ uint32_t sT[FT][FT + 1];
  __shared__ uint32_t sZ[FT][FT + 1];  // [window row][window column]
  const int lane = threadIdx.x;
  const int32_t t = blockIdx.x;
  const int32_t tr = t / ntc, tc = t - tr * ntc;
  if (k > 0) {
    bool act = false;
    if (lane < 9) {
      const int32_t rr = tr + lane / 3 - 1, cc = tc + lane % 3 - 1;
      if (rr >= 0 && rr < ntr && cc >= 0 && cc < ntc) {
        const int32_t st = __hip_atomic_load(&stamp[rr * ntc + cc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        act = lane == 4 ? st == 2 * (k - 1) + 1 : (st >> 1) == k - 1;
      }
    }
    if (!__any(act)) return;
  }
  // Window row w is grid row wr0 + w; window column lane is grid column
  // wc0 + lane.  Cells off the grid are +inf with elevation +inf: they never
  // change and lower nothing.
  const int64_t wr0 = (int64_t)tr * FO - 1, wc0 = (int64_t)tc * FO - 1;
  const int64_t col = wc0 + lane;
  const bool col_in = col >= 0 && col < nc;
  uint32_t f[FT];
#pragma unroll
  for (int s = 0; s < FT; ++s) {
    const int64_t row = wr0 + s;
    const bool in = col_in && row >= 0 && row < nr;
    f[s] = in ? fkey(F[row * nc + col]) : KEY_INF;
    sZ[s][lane] = in ? fkey(z[row * nc + col]) : KEY_INF;
  }
  const bool inner = lane >= 1 && lane <= FT - 2;
  bool any = false, capped = true;
  for (int round = 0; round < FILL_ROUNDS; ++round) {
    // Column orientation: steps = window rows, lanes = window columns.
    __syncthreads();
    const auto zcol = [&](int s) { return sZ[s][lane]; };
    bool ch = sweep<EPS, C8, true>(f, inner, zcol);
    ch |= sweep<EPS, C8, false>(f, inner, zcol);
    transpose(f, sT, lane);
    // Row orientation: steps = window columns, lanes = window rows.
    const auto zrow = [&](int s) { return sZ[lane][s]; };
    ch |= sweep<EPS, C8, true>(f, inner, zrow);
    ch |= sweep<EPS, C8, false>(f, inner, zrow);
    transpose(f, sT, lane);
    if (!__any(ch)) {
      capped = false;
      break;
    }
    any = true;
  }
  if (!any) return;
#pragma unroll
  for (int s = 1; s < FT - 1; ++s) {
    const int64_t row = wr0 + s;
    if (inner && col_in && row < nr) F[row * nc + col] = fval(f[s]);
  }
  if (lane == 0) {
    __hip_atomic_store(&stamp[t], 2 * k + (capped ? 1 : 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(last, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

hipError_t launch_fill_init(const float* z, float* F, int64_t nr, int64_t nc, int32_t* stamp, int32_t ntiles,
                            int32_t* last, int32_t* status, hipStream_t s) {
  const int64_t n = nr * nc > ntiles ? nr * nc : ntiles;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_init, dim3((unsigned)blocks), dim3(256), 0, s, z, F, nr, nc, stamp, ntiles, last,
                     status);
  return hipGetLastError();
}

hipError_t launch_fill_tiles(const float* z, float* F, int64_t nr, int64_t nc, int32_t ntr, int32_t ntc,
                             bool eps, bool c8, int32_t* stamp, int32_t* last, int32_t k, hipStream_t s) {
  const dim3 grid((unsigned)(ntr * ntc)), block(FT);
  if (eps) {
    if (c8) hipLaunchKernelGGL((k_fill_tile<true, true>), grid, block, 0, s, z, F, nr, nc, ntr, ntc, stamp, last, k);
    else hipLaunchKernelGGL((k_fill_tile<true, false>), grid, block, 0, s, z, F, nr, nc, ntr, ntc, stamp, last, k);
  } else {
    if (c8) hipLaunchKernelGGL((k_fill_tile<false, true>), grid, block, 0, s, z, F, nr, nc, ntr, ntc, stamp, last, k);
    else hipLaunchKernelGGL((k_fill_tile<false, false>), grid, block, 0, s, z, F, nr, nc, ntr, ntc, stamp, last, k);
  }
  return hipGetLastError();
}

}  // namespace fr
