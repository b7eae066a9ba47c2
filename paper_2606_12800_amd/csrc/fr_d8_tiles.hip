// Tile-forest path for single-receiver codes (D8 / D4) whose flow runs in
// every direction, as on depression-filled terrain (the paper's workflow,
// Section 4: fill, then route).
//
// The row sweeps (fr_d8_a.hip) follow only the edges toward the previous
// row; every other cell becomes an exit of the forest, and on filled terrain
// so many do that the exit list overflows.  Here each tile of 32 x 64 cells
// solves its own part of (I - W^T) q = r (Section 2.2) for any flow
// direction, in LDS, so that only the cells whose receiver lies in another
// tile are exits -- at most the tile's perimeter, 188 of its 2048 cells.
// Like the paper's per-process solves (Section 2.4, Section 3.3), the tiles
// are independent blocks; the exits then feed the same fixed-point forest
// as the row sweeps (link, pointer-doubling rounds, totals), which joins
// them, and a second pass over every tile adds its donors' totals.
//
// Inside a tile (one workgroup of 256 threads, 8 cells each):
//   1. the codes with a one-cell halo into LDS; each cell's receiver inside
//      the tile, or none (a sink, or an exit);
//   2. pointer jumping over those receivers: each cell's root -- the sink or
//      exit where its in-tile path ends -- and its depth, the number of
//      in-tile edges to the root, in about log2(depth) rounds;
//   3. the cells by levels of depth, deepest first.  A cell's donors inside
//      the tile lie exactly one level deeper, so with one barrier per level
//      every cell adds its finished donors' values, in neighbour order: a
//      fixed order, so results repeat bit for bit.
// Phase A (up) stores the local sums of the exits in the exit list and, for
// every cell receiving water over the tile's edge (inlet), its root.  Phase C
// (down) starts the inlets from their out-of-tile donors' forest totals;
// its values are final and go out with the tile's mass-balance partial.
//
// The path runs only after the row sweeps' exit list overflowed: every
// launch first reads the control block's gate and returns at once when it is
// closed, and each workgroup walks a stride of tiles, so that a closed gate
// costs a few thousand short workgroups.
#include "fr_d8.hpp"

namespace fr {
namespace {

constexpr int HR = D8T_ROWS;   // tile rows
constexpr int HC = D8T_COLS;   // tile columns
constexpr int HN = HR * HC;    // cells per tile
constexpr int HT = 256;        // threads per workgroup
constexpr int HK = HN / HT;    // cells per thread
constexpr int HW = HC + 2;     // halo row width
constexpr uint32_t PT_TERM = 0x8000u;  // pointer flag: the target is a root
constexpr int NO_LEVEL = 0x7FFF;       // not on a path to a root (cycle) or off the grid
static_assert(HC == 64, "a tile row is one wavefront");
static_assert(HN % HT == 0 && HN <= 0x8000, "pointers fit 15 bits");

struct TT {
  int64_t r0, c0;
  int h, w, id;
};

// Virtual tile t runs on XCD t % 8 (the grid is a multiple of 8 workgroups,
// dispatched round-robin): give each XCD a contiguous run of tiles, whose
// shared halo rows and columns then meet in one L2.
__device__ __forceinline__ TT tile_at(const D8Params& P, int t, int ntiles) {
  const int q = ntiles / 8;
  const int id = t < 8 * q ? (t % 8) * q + t / 8 : t;
  const int ntc = (int)((P.ncols + HC - 1) / HC);
  const int tr = id / ntc, tc = id - tr * ntc;
  TT T;
  T.id = id;
  T.r0 = (int64_t)tr * HR;
  T.c0 = (int64_t)tc * HC;
  T.h = (int)min((int64_t)HR, P.nrows - T.r0);
  T.w = (int)min((int64_t)HC, P.ncols - T.c0);
  return T;
}

template <int VK>
struct TV;
template <>
struct TV<VK_FF> {
  using T = ff;
  __device__ static T zero() { return {0.0f, 0.0f}; }
  __device__ static T add(T a, T b) { return ff_add(a, b); }
  __device__ static double mass(T a) { return (double)a.hi + (double)a.lo; }
};
template <>
struct TV<VK_F64> {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static double mass(T a) { return a; }
};
template <>
struct TV<VK_NONE> {
  using T = int;  // unused
  __device__ static T zero() { return 0; }
  __device__ static T add(T a, T) { return a; }
  __device__ static double mass(T) { return 0.0; }
};

template <int RAIN>
__device__ __forceinline__ double rain_at(const D8Params& P, int64_t g) {
  if (RAIN == RAIN_F32) return (double)P.rain32[g];
  if (RAIN == RAIN_F64) return P.rain64[g];
  return 1.0;
}

template <int VK, int RAIN>
__device__ __forceinline__ typename TV<VK>::T src_of(const D8Params& P, int64_t g) {
  if constexpr (VK == VK_FF) {
    if (RAIN == RAIN_F32) return ff{P.rain32[g], 0.0f};
    if (RAIN == RAIN_F64) {
      const double r = P.rain64[g];
      const float hi = (float)r;
      return ff{hi, (float)(r - (double)hi)};
    }
    return ff{1.0f, 0.0f};
  } else if constexpr (VK == VK_F64) {
    return rain_at<RAIN>(P, g);
  } else {
    return 0;
  }
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

template <bool UP, int VK, bool CNT, int RAIN>
__global__ __launch_bounds__(HT) void k_d8t(D8Params P, int ntiles) {
  if (__hip_atomic_load(&P.ctl->d8_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;  // uniform
  const uint32_t n_ex = *P.n_exits;
  if (!UP && n_ex > P.cap) return;  // uniform: the engine takes over
  using V = typename TV<VK>::T;
  constexpr int VB = VK == VK_NONE ? 0 : HN * 8;
  constexpr int CB = CNT ? HN * 8 : 0;
  constexpr int SB = VB + CB > HN * 4 ? VB + CB : HN * 4;
  __shared__ __align__(16) unsigned char s_buf[SB];
  __shared__ uint8_t s_code[(HR + 2) * HW];
  __shared__ int s_int[16];
  __shared__ double s_dbl[8];
  __shared__ float s_flt[4];
  V* s_v = reinterpret_cast<V*>(s_buf);
  uint64_t* s_c = reinterpret_cast<uint64_t*>(s_buf + VB);
  uint16_t* s_ptr = reinterpret_cast<uint16_t*>(s_buf);  // pointer jumping: aliases the values
  uint16_t* s_dist = s_ptr + HN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nr = P.nrows, nc = P.ncols;

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TT T = tile_at(P, t, ntiles);
    // 1. Codes with a one-cell halo; off the grid reads as a sink.
    for (int e = tid; e < (HR + 2) * HW; e += HT) {
      const int hr = e / HW, hc = e - hr * HW;
      const int64_t r = T.r0 + hr - 1, c = T.c0 + hc - 1;
      uint8_t v = SINK;
      if (r >= 0 && r < nr && c >= 0 && c < nc) v = P.code[r * nc + c];
      s_code[e] = v;
    }
    __syncthreads();
    // 2. Each own cell: in-tile receiver, donor masks (bit n: the neighbour
    // in direction n gives this cell water; inside / outside the tile).
    uint32_t din[HK], dout[HK], ptr[HK], dist[HK];
    bool sink[HK], valid[HK], ex[HK];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int lr = wave + 4 * k, lc = lane;
      const int i = lr * HC + lc;
      valid[k] = lr < T.h && lc < T.w;
      const uint32_t cd = s_code[(lr + 1) * HW + lc + 1];
      bool sk = true, inside = false;
      int rcv = i;
      if (valid[k]) {
        if (cd <= 7u) {
          const int tr = lr + nb_dr((int)cd), tc = lc + nb_dc((int)cd);
          const int64_t gr = T.r0 + tr, gc = T.c0 + tc;
          if (gr < 0 || gr >= nr || gc < 0 || gc >= nc) {
            bad = true;  // receiver off the grid: malformed, treated as a sink
          } else {
            sk = false;
            inside = tr >= 0 && tr < HR && tc >= 0 && tc < HC;
            if (inside) rcv = tr * HC + tc;
          }
        } else if (cd != SINK) {
          bad = true;
        }
      }
      sink[k] = sk;
      ex[k] = valid[k] && !sk && !inside;  // receiver in another tile
      uint32_t mi = 0, mo = 0;
      if (valid[k]) {
#pragma unroll
        for (int n = 0; n < 8; ++n) {
          const int ar = lr + nb_dr(n), ac = lc + nb_dc(n);
          if (s_code[(ar + 1) * HW + ac + 1] == (uint8_t)(7 - n)) {
            if (ar >= 0 && ar < HR && ac >= 0 && ac < HC) mi |= 1u << n;
            else mo |= 1u << n;
          }
        }
      }
      din[k] = mi;
      dout[k] = mo;
      ptr[k] = inside ? (uint32_t)rcv : ((uint32_t)i | PT_TERM);
      dist[k] = inside ? 1u : 0u;
      s_ptr[i] = (uint16_t)ptr[k];
      s_dist[i] = (uint16_t)dist[k];
    }
    if (UP && bad) set_status(P.status, FR_ERR_BADCODE);
    __syncthreads();
    // 3. Pointer jumping: after round j every pointer spans 2^(j+1) edges
    // or ends at a root; a path inside the tile has fewer than HN edges.
    for (int j = 0; j <= 12; ++j) {
      uint32_t np[HK], nd[HK];
      int open = 0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        np[k] = ptr[k];
        nd[k] = dist[k];
        if (!(ptr[k] & PT_TERM)) {
          np[k] = s_ptr[ptr[k]];
          nd[k] = dist[k] + s_dist[ptr[k]];
          open = 1;
        }
      }
      if (!__syncthreads_or(open) || j == 12) break;  // uniform; every read above is done
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        ptr[k] = np[k];
        dist[k] = nd[k];
        const int i = (wave + 4 * k) * HC + lane;
        s_ptr[i] = (uint16_t)np[k];
        s_dist[i] = (uint16_t)nd[k];
      }
      __syncthreads();
    }
    // Depths; a cell whose path never reaches a root lies on or above a
    // cycle (malformed codes).
    int level[HK];
    int dmax = 0;
    bool cyc = false;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const bool ok = valid[k] && (ptr[k] & PT_TERM);
      cyc |= valid[k] && !(ptr[k] & PT_TERM);
      level[k] = ok ? (int)dist[k] : NO_LEVEL;
      if (ok) dmax = max(dmax, (int)dist[k]);
    }
    if (UP && cyc) set_status(P.status, FR_ERR_NOTDAG);
    dmax = wave_max(dmax);
    if (lane == 0) s_int[wave] = dmax;
    // 4. Sources: rain (unit rain: 1), and in phase C the forest totals of
    // the out-of-tile donors, in neighbour order.  The pointer arrays are
    // dead: every thread passed the last barrier after reading them.
    V val[HK];
    uint64_t cnt[HK];
    double m_rain = 0.0;
    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int lr = wave + 4 * k;
      const int64_t g = (T.r0 + lr) * nc + T.c0 + lane;
      V v = TV<VK>::zero();
      uint64_t c = 0;
      if (valid[k]) {
        if (RAIN != RAIN_UNIT) {
          const double r = rain_at<RAIN>(P, g);
          if (UP) nonfinite |= !isfinite(r);
          else m_rain += r;
        } else if (!UP) {
          m_rain += 1.0;
        }
        v = src_of<VK, RAIN>(P, g);
        c = 1;
        if (!UP && dout[k]) {
          uint32_t m = dout[k];
          while (m) {
            const int n = __builtin_ctz(m);
            m &= m - 1;
            const uint32_t nd = P.node_of[g + (int64_t)nb_dr(n) * nc + nb_dc(n)];
            if (nd >= n_ex) {  // inconsistent bookkeeping: never follow it
              set_status(P.status, FR_ERR_BADCODE);
              continue;
            }
            if constexpr (VK == VK_FF) v = ff_add(v, ff{P.tot_hi[nd], P.tot_lo[nd]});
            if constexpr (VK == VK_F64) v += P.tot_d[nd];
            if (CNT) c += P.ex_cnt[0][nd];
          }
        }
      }
      val[k] = v;
      cnt[k] = c;
      const int i = lr * HC + lane;
      if (VK != VK_NONE) s_v[i] = v;
      if (CNT) s_c[i] = c;
    }
    if (UP && nonfinite) set_status(P.status, FR_ERR_NONFINITE);
    __syncthreads();
    const int D = max(max(s_int[0], s_int[1]), max(s_int[2], s_int[3]));
    // 5. Levels, deepest first: a cell's in-tile donors are one level deeper
    // and final; each cell adds them in neighbour order.
    for (int L = D - 1; L >= 0; --L) {
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (level[k] == L && din[k]) {
          const int i = (wave + 4 * k) * HC + lane;
          uint32_t m = din[k];
          V v = val[k];
          uint64_t c = cnt[k];
          while (m) {
            const int n = __builtin_ctz(m);
            m &= m - 1;
            const int a = i + nb_dr(n) * HC + nb_dc(n);
            if (VK != VK_NONE) v = TV<VK>::add(v, s_v[a]);
            if (CNT) c += s_c[a];
          }
          val[k] = v;
          cnt[k] = c;
          if (VK != VK_NONE) s_v[i] = v;
          if (CNT) s_c[i] = c;
        }
      }
      __syncthreads();
    }
    if (UP) {
      // 6a. Exits (a root that is not a sink) into consecutive slots of the
      // list: one atomic per tile.
      const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      // Slot order inside the wavefront: cell k of every lane before cell
      // k + 1 of any lane.
      uint32_t off[HK], wtot = 0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        const uint64_t m = __ballot(ex[k]);
        off[k] = wtot + (uint32_t)__popcll(m & lower);
        wtot += (uint32_t)__popcll(m);
      }
      float lmf = 0.0f;
      double lmd = 0.0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!ex[k]) continue;
        if constexpr (VK == VK_FF) lmf = fmaxf(lmf, fabsf(val[k].hi));
        if constexpr (VK == VK_F64) lmd = fmax(lmd, fabs(val[k]));
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        lmf = fmaxf(lmf, __shfl_xor(lmf, o, 64));
        lmd = fmax(lmd, __shfl_xor(lmd, o, 64));
      }
      if (lane == 0) {
        s_int[4 + wave] = (int)wtot;
        s_flt[wave] = lmf;
        s_dbl[wave] = lmd;
      }
      __syncthreads();
      if (tid == 0) {
        const uint32_t tot = (uint32_t)(s_int[4] + s_int[5] + s_int[6] + s_int[7]);
        s_int[8] = tot ? (int)atomicAdd(P.n_exits, tot) : 0;
        if constexpr (VK == VK_FF) {
          const float m = fmaxf(fmaxf(s_flt[0], s_flt[1]), fmaxf(s_flt[2], s_flt[3]));
          if (m > 0.0f) atomicMax(&P.ctl->loc_max_f, __float_as_uint(m));
        }
        if constexpr (VK == VK_F64) {
          const double m = fmax(fmax(s_dbl[0], s_dbl[1]), fmax(s_dbl[2], s_dbl[3]));
          if (m > 0.0)
            atomicMax(reinterpret_cast<unsigned long long*>(&P.ctl->loc_max_d),
                      (unsigned long long)__double_as_longlong(m));
        }
      }
      __syncthreads();
      uint32_t base = (uint32_t)s_int[8];
      for (int w = 0; w < wave; ++w) base += (uint32_t)s_int[4 + w];
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        const int lr = wave + 4 * k;
        const int64_t g = (T.r0 + lr) * nc + T.c0 + lane;
        if (ex[k]) {
          const uint32_t idx = base + off[k];
          if (idx < P.cap) {
            P.node_of[g] = idx;
            P.ex_cell[idx] = (uint32_t)g;
            if constexpr (VK == VK_FF) {
              P.ex_hi[idx] = val[k].hi;
              P.ex_lo[idx] = val[k].lo;
            }
            if constexpr (VK == VK_F64) P.ex_d[idx] = val[k];
            if (CNT) P.ex_cnt[0][idx] = cnt[k];
          }
        }
        // 6b. Inlets: the root of their in-tile path (NONE on a cycle).
        if (valid[k] && dout[k]) {
          uint32_t rt = NONE;
          if (ptr[k] & PT_TERM) {
            const int p = (int)(ptr[k] & 0x7FFFu);
            rt = (uint32_t)((T.r0 + p / HC) * nc + T.c0 + (p % HC));
          }
          P.root_of[g] = rt;
        }
      }
    } else {
      // 6c. Final values and the tile's {sum over sinks, sum of rain}.
      double m_sink = 0.0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!valid[k]) continue;
        const int64_t g = (T.r0 + wave + 4 * k) * nc + T.c0 + lane;
        if constexpr (VK == VK_FF) {
          if (P.q32) P.q32[g] = val[k].hi + val[k].lo;
        }
        if constexpr (VK == VK_F64) {
          if (P.q64) P.q64[g] = val[k];
        }
        if (CNT) P.cnt[g] = cnt[k];
        if (sink[k]) m_sink += TV<VK>::mass(val[k]);
      }
      if (P.mass_part) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          m_sink += __shfl_xor(m_sink, o, 64);
          m_rain += __shfl_xor(m_rain, o, 64);
        }
        if (lane == 0) {
          s_dbl[2 * wave] = m_sink;
          s_dbl[2 * wave + 1] = m_rain;
        }
        __syncthreads();
        if (tid == 0) {
          P.mass_part[2 * (int64_t)T.id] = (s_dbl[0] + s_dbl[2]) + (s_dbl[4] + s_dbl[6]);
          P.mass_part[2 * (int64_t)T.id + 1] = (s_dbl[1] + s_dbl[3]) + (s_dbl[5] + s_dbl[7]);
        }
      }
    }
    __syncthreads();  // the next tile reuses every LDS array
  }
}

// The gate: the tile-forest path serves the call when the row sweeps' exit
// list overflowed (or the caller chose it: `force`).  It starts from a clean
// forest state (its own exit count and round flags are separate words; the
// fixed-point unit is re-derived) and closes the engine's gate again.
__global__ void k_d8t_gate(CallCtl* C, int force) {
  if (threadIdx.x == 0 && (force || C->fallback)) {
    C->d8_tiles = 1;
    C->fallback = 0;
    C->loc_max_f = 0u;
    C->loc_max_d = 0ull;
  }
}

// Mass-balance partials of the tiles, first stage: each workgroup sums a
// fixed run of D8T_MASS_RUN tiles in a fixed order.
__global__ __launch_bounds__(256) void k_d8t_mass(const double* part, int ntiles, double* out, const CallCtl* C) {
  if (__hip_atomic_load(&C->d8_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  __shared__ double rs[256], rt[256];
  const int b0 = blockIdx.x * D8T_MASS_RUN;
  const int b1 = min(ntiles, b0 + D8T_MASS_RUN);
  double s = 0.0, t = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += 256) {
    s += part[2 * (int64_t)b];
    t += part[2 * (int64_t)b + 1];
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
    out[2 * blockIdx.x] = rs[0];
    out[2 * blockIdx.x + 1] = rt[0];
  }
}

// Workgroups of a tile launch: as many as fit on the device at once (a
// multiple of 8, for the XCD mapping), at most one per tile.
template <bool UP, int VK, bool CNT, int RAIN>
int d8t_grid(int ntiles) {
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_d8t<UP, VK, CNT, RAIN>, HT, 0) != hipSuccess ||
        cus <= 0 || per <= 0) {
      cus = 256;
      per = 2;
    }
    resident = cus * per;
  }
  int g = resident < ntiles ? resident : ntiles;
  if (g >= 8) g -= g % 8;
  return g < 1 ? 1 : g;
}

template <bool UP, int VK, bool CNT, int RAIN>
void d8t_launch(const D8Params& P, int ntiles, hipStream_t s) {
  hipLaunchKernelGGL((k_d8t<UP, VK, CNT, RAIN>), dim3((unsigned)d8t_grid<UP, VK, CNT, RAIN>(ntiles)), dim3(HT), 0,
                     s, P, ntiles);
}

template <bool UP, int VK, bool CNT>
void d8t_rain(const D8Params& P, int ntiles, hipStream_t s) {
  if (VK == VK_NONE || (!P.rain32 && !P.rain64)) d8t_launch<UP, VK, CNT, RAIN_UNIT>(P, ntiles, s);
  else if (P.rain32) d8t_launch<UP, VK, CNT, RAIN_F32>(P, ntiles, s);
  else d8t_launch<UP, VK, CNT, RAIN_F64>(P, ntiles, s);
}

template <bool UP>
void d8t_dispatch(ValKind vk, bool cnt, const D8Params& P, int ntiles, hipStream_t s) {
  if (vk == VK_FF) {
    if (cnt) d8t_rain<UP, VK_FF, true>(P, ntiles, s);
    else d8t_rain<UP, VK_FF, false>(P, ntiles, s);
  } else if (vk == VK_F64) {
    if (cnt) d8t_rain<UP, VK_F64, true>(P, ntiles, s);
    else d8t_rain<UP, VK_F64, false>(P, ntiles, s);
  } else {
    d8t_rain<UP, VK_NONE, true>(P, ntiles, s);
  }
}

}  // namespace

int64_t d8t_tiles(int64_t nrows, int64_t ncols) {
  return ((nrows + D8T_ROWS - 1) / D8T_ROWS) * ((ncols + D8T_COLS - 1) / D8T_COLS);
}

// Cells that can be exits: those on a tile's perimeter (every cell of a tile
// one cell high or wide).
uint64_t d8t_exit_bound(int64_t nrows, int64_t ncols) {
  auto per = [](int64_t h, int64_t w) -> uint64_t {
    return (uint64_t)(h <= 2 || w <= 2 ? h * w : 2 * (h + w) - 4);
  };
  const int64_t fr = nrows / D8T_ROWS, fc = ncols / D8T_COLS;
  const int64_t hr = nrows % D8T_ROWS, hc = ncols % D8T_COLS;
  uint64_t b = (uint64_t)(fr * fc) * per(D8T_ROWS, D8T_COLS);
  if (hr) b += (uint64_t)fc * per(hr, D8T_COLS);
  if (hc) b += (uint64_t)fr * per(D8T_ROWS, hc);
  if (hr && hc) b += per(hr, hc);
  return b;
}

size_t d8t_mass_words(int64_t nrows, int64_t ncols) {
  const int64_t nt = d8t_tiles(nrows, ncols);
  return (size_t)(2 * (nt + (nt + D8T_MASS_RUN - 1) / D8T_MASS_RUN));
}

hipError_t launch_d8t_gate(CallCtl* C, bool force, hipStream_t s) {
  hipLaunchKernelGGL(k_d8t_gate, dim3(1), dim3(64), 0, s, C, force ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_d8t(bool up, ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  const int64_t nt = d8t_tiles(P.nrows, P.ncols);
  if (nt <= 0 || nt > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (up) d8t_dispatch<true>(vk, cnt, P, (int)nt, s);
  else d8t_dispatch<false>(vk, cnt, P, (int)nt, s);
  return hipGetLastError();
}

hipError_t launch_d8t_mass(const double* part, int64_t ntiles, double* out, CallCtl* C, hipStream_t s) {
  const int64_t nb = (ntiles + D8T_MASS_RUN - 1) / D8T_MASS_RUN;
  double* stage = const_cast<double*>(part) + 2 * ntiles;
  hipLaunchKernelGGL(k_d8t_mass, dim3((unsigned)nb), dim3(256), 0, s, part, (int)ntiles, stage, C);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  return launch_mass_final_if(stage, (int)nb, out, &C->d8_tiles, s);
}

}  // namespace fr
