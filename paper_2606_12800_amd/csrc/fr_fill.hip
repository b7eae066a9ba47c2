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
// four sweeps until one sweep changes nothing (or a round cap is reached),
// then writes its own cells back.  Launch k works through a list of the
// tiles next to a tile that changed in launch k - 1 (the first list: the
// tiles on the grid's perimeter); the host stops once a list is empty.
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

// What one sweep changed in this lane: any cell, the cell at step 1, the
// cell at step 62.
struct SweepChange {
  bool any, lo, hi;
};

// One sweep over steps 1..62 of the window, forward or backward; lanes 1..62
// update.  zk(s) is the elevation key of this lane's cell at step s.  Every
// cell is evaluated with all its neighbours, so a sweep that changes nothing
// has found a fixed point of the tile (for its halo).
template <bool EPS, bool C8, bool FWD, typename ZK>
__device__ __forceinline__ SweepChange sweep(uint32_t (&f)[FT], bool inner, ZK zk) {
  SweepChange c{false, false, false};
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
    if (s == 1) c.lo = ch;
    if (s == FT - 2) c.hi = ch;
    f[s] = ch ? nv : f[s];
  }
  c.any = changed;
  return c;
}

// Which owned cells on the tile's sides changed: the neighbour tile on that
// side reads them as its halo.  Bits: 0 top-left corner, 1 top row, 2
// top-right corner, 3 left column, 5 right column, 6 bottom-left corner, 7
// bottom row, 8 bottom-right corner (the neighbour tile at (dr, dc) is bit
// 3 (dr + 1) + dc + 1); bit 4 (the tile itself) marks a stop at the round
// cap.
struct EdgeChange {
  bool tl = false, t = false, tr = false, l = false, r = false, bl = false, b = false, br = false;
  // Column orientation: steps = rows, lanes = columns.
  __device__ void col(const SweepChange& c, int lane) {
    t |= c.lo;
    b |= c.hi;
    l |= lane == 1 && c.any;
    r |= lane == FT - 2 && c.any;
    tl |= lane == 1 && c.lo;
    tr |= lane == FT - 2 && c.lo;
    bl |= lane == 1 && c.hi;
    br |= lane == FT - 2 && c.hi;
  }
  // Row orientation: steps = columns, lanes = rows.
  __device__ void row(const SweepChange& c, int lane) {
    l |= c.lo;
    r |= c.hi;
    t |= lane == 1 && c.any;
    b |= lane == FT - 2 && c.any;
    tl |= lane == 1 && c.lo;
    tr |= lane == 1 && c.hi;
    bl |= lane == FT - 2 && c.lo;
    br |= lane == FT - 2 && c.hi;
  }
  __device__ uint32_t bits() const {
    return (__any(tl) ? 1u : 0u) | (__any(t) ? 2u : 0u) | (__any(tr) ? 4u : 0u) | (__any(l) ? 8u : 0u) |
           (__any(r) ? 32u : 0u) | (__any(bl) ? 64u : 0u) | (__any(b) ? 128u : 0u) | (__any(br) ? 256u : 0u);
  }
};

// a[s] of lane l becomes a[l] of lane s (64 x 64 transpose through LDS).
__device__ __forceinline__ void transpose(uint32_t (&a)[FT], uint32_t (*sT)[FT + 1], int lane) {
  __syncthreads();
#pragma unroll
  for (int s = 0; s < FT; ++s) sT[s][lane] = a[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < FT; ++s) a[s] = sT[lane][s];
}

// Position of tile (tr, tc) in the list of tiles on the grid's perimeter,
// or -1 inside.
__device__ __forceinline__ int32_t perimeter_slot(int32_t tr, int32_t tc, int32_t ntr, int32_t ntc) {
  if (ntr == 1) return tc;
  if (tr == 0) return tc;
  if (tr == ntr - 1) return ntc + tc;
  if (ntc == 1) return 2 * ntc + (tr - 1);
  if (tc == 0) return 2 * ntc + 2 * (tr - 1);
  if (tc == ntc - 1) return 2 * ntc + 2 * (tr - 1) + 1;
  return -1;
}

// F = z on the grid boundary, +inf elsewhere.  The first work list holds the
// tiles on the grid's perimeter (inside, +inf cells next to +inf cells
// cannot change).
__global__ __launch_bounds__(256) void k_fill_init(const float* __restrict__ z, float* __restrict__ F,
                                                   int64_t nr, int64_t nc, FillState S, int32_t* status) {
  bool bad = false;
  const int64_t n = nr * nc;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float v = z[i];
    bad |= !isfinite(v);
    const int64_t r = i / nc, c = i - r * nc;
    const bool edge = r == 0 || c == 0 || r == nr - 1 || c == nc - 1;
    F[i] = edge ? v + 0.0f : __uint_as_float(0x7F800000u);
  }
  const int32_t ntiles = S.ntr * S.ntc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride) {
    const int32_t tr = (int32_t)(t / S.ntc), tc = (int32_t)(t - (int64_t)tr * S.ntc);
    const int32_t p = perimeter_slot(tr, tc, S.ntr, S.ntc);
    S.queued[t] = p >= 0 ? 0 : -1;
    if (p >= 0) S.list[p] = (int32_t)t;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.nlist[0] = S.ntr == 1 ? S.ntc : (S.ntc == 1 ? S.ntr : 2 * S.ntc + 2 * (S.ntr - 2));
    S.nlist[1] = 0;
    S.nlist[2] = 0;
    *S.last = -1;
  }
  if (bad && status) atomicCAS(status, 0, FR_ERR_NONFINITE);
}

// Relaxes tile t until a sweep changes nothing or the round cap is hit and
// writes its cells back if any changed.  Returns the EdgeChange bits (0: no
// change on the sides) and whether any cell changed.
template <bool EPS, bool C8>
__device__ __forceinline__ uint32_t fill_tile(const float* __restrict__ z, float* F, int64_t nr, int64_t nc,
                                         int32_t tr, int32_t tc, uint32_t (*sT)[FT + 1], uint32_t (*sZ)[FT + 1],
                                         int lane) {
  // Window row w is grid row wr0 + w; window column lane is grid column
  // wc0 + lane.  Cells off the grid are +inf with elevation +inf: they never
  // change and lower nothing.
  const int64_t wr0 = (int64_t)tr * FO - 1, wc0 = (int64_t)tc * FO - 1;
  const int64_t col = wc0 + lane;
  const bool col_in = col >= 0 && col < nc;
  uint32_t f[FT];
  __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
  for (int s = 0; s < FT; ++s) {
    const int64_t row = wr0 + s;
    const bool in = col_in && row >= 0 && row < nr;
    f[s] = in ? fkey(F[row * nc + col]) : KEY_INF;
    sZ[s][lane] = in ? fkey(z[row * nc + col]) : KEY_INF;
  }
  const bool inner = lane >= 1 && lane <= FT - 2;
  const auto zcol = [&](int s) { return sZ[s][lane]; };
  const auto zrow = [&](int s) { return sZ[lane][s]; };
  EdgeChange e;
  bool any = false, capped = true;
  for (int round = 0; round < FILL_ROUNDS && capped; ++round) {
    // Column orientation: steps = window rows, lanes = window columns.
    __syncthreads();
    SweepChange c = sweep<EPS, C8, true>(f, inner, zcol);
    e.col(c, lane);
    if (!__any(c.any)) {
      capped = false;
      break;
    }
    any = true;
    c = sweep<EPS, C8, false>(f, inner, zcol);
    e.col(c, lane);
    if (!__any(c.any)) {
      capped = false;
      break;
    }
    transpose(f, sT, lane);
    // Row orientation: steps = window columns, lanes = window rows.
    c = sweep<EPS, C8, true>(f, inner, zrow);
    e.row(c, lane);
    if (!__any(c.any)) capped = false;
    if (capped) {
      c = sweep<EPS, C8, false>(f, inner, zrow);
      e.row(c, lane);
      if (!__any(c.any)) capped = false;
    }
    transpose(f, sT, lane);
  }
  if (!any) return 0;
#pragma unroll
  for (int s = 1; s < FT - 1; ++s) {
    const int64_t row = wr0 + s;
    if (inner && col_in && row < nr) F[row * nc + col] = fval(f[s]);
  }
  return e.bits() | (capped ? 16u : 0u) | 0x200u;
}

// Launch k works through list k (built by launch k - 1) and builds list
// k + 1: the neighbours of every tile whose cells on the shared side
// changed, and the tile itself when it stopped at the round cap, each once (queued[] holds the latest launch
// a tile was queued for).  List k + 2's length is cleared here: launch k + 1
// fills it, and list k - 1, which shares its slot, is spent.
template <bool EPS, bool C8>
__global__ __launch_bounds__(FT) void k_fill_tile(const float* __restrict__ z, float* F, int64_t nr, int64_t nc,
                                                  FillState S, int32_t k) {
  __shared__ uint32_t sT[FT][FT + 1];
  __shared__ uint32_t sZ[FT][FT + 1];  // [window row][window column]
  const int lane = threadIdx.x;
  const int32_t ntiles = S.ntr * S.ntc;
  const int32_t cur = k % 3, nxt = (k + 1) % 3;
  if (blockIdx.x == 0 && lane == 0) S.nlist[(k + 2) % 3] = 0;
  const int32_t n = S.nlist[cur];
  const int32_t* list = S.list + (size_t)cur * ntiles;
  int32_t* out = S.list + (size_t)nxt * ntiles;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int32_t t = list[i];
    const int32_t tr = t / S.ntc, tc = t - tr * S.ntc;
    const uint32_t res = fill_tile<EPS, C8>(z, F, nr, nc, tr, tc, sT, sZ, lane);
    if (res == 0) continue;
    // Queue the neighbours whose halo changed (and the tile itself after a
    // stop at the round cap).
    if (lane < 9 && ((res >> lane) & 1u)) {
      const int32_t rr = tr + lane / 3 - 1, cc = tc + lane % 3 - 1;
      if (rr >= 0 && rr < S.ntr && cc >= 0 && cc < S.ntc) {
        const int32_t u = rr * S.ntc + cc;
        if (atomicMax(&S.queued[u], k + 1) < k + 1) out[atomicAdd(&S.nlist[nxt], 1)] = u;
      }
    }
    if (lane == 0) __hip_atomic_store(S.last, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

hipError_t launch_fill_init(const float* z, float* F, int64_t nr, int64_t nc, const FillState& S, int32_t* status,
                            hipStream_t s) {
  const int64_t ntiles = (int64_t)S.ntr * S.ntc;
  const int64_t n = nr * nc > ntiles ? nr * nc : ntiles;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_init, dim3((unsigned)blocks), dim3(256), 0, s, z, F, nr, nc, S, status);
  return hipGetLastError();
}

hipError_t launch_fill_tiles(const float* z, float* F, int64_t nr, int64_t nc, bool eps, bool c8,
                             const FillState& S, int32_t k, hipStream_t s) {
  // Enough single-wavefront workgroups for every SIMD of the chip; each
  // walks the list with a grid stride.
  int64_t blocks = (int64_t)S.ntr * S.ntc;
  if (blocks > 2048) blocks = 2048;
  const dim3 grid((unsigned)blocks), block(FT);
  if (eps) {
    if (c8) hipLaunchKernelGGL((k_fill_tile<true, true>), grid, block, 0, s, z, F, nr, nc, S, k);
    else hipLaunchKernelGGL((k_fill_tile<true, false>), grid, block, 0, s, z, F, nr, nc, S, k);
  } else {
    if (c8) hipLaunchKernelGGL((k_fill_tile<false, true>), grid, block, 0, s, z, F, nr, nc, S, k);
    else hipLaunchKernelGGL((k_fill_tile<false, false>), grid, block, 0, s, z, F, nr, nc, S, k);
  }
  return hipGetLastError();
}

}  // namespace fr
