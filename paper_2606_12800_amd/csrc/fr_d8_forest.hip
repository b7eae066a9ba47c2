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

// The work-queue forest's sums (below) are held split, v = hi * 2^56 + lo
// with 0 <= lo < 2^56 for every term added, so that the low word never
// carries: an exit receives its own term and at most 196 children's (one per
// cell of the ring around its tile), below 2^64 together, and both words
// take their additions with no returned value to wait for.  Its unit is 2^6
// coarser than the doubling forest's (sums below 2^118 units), so that the
// high words stay below 2^62 in magnitude.
constexpr int KF_FX_HEAD = 6;
constexpr unsigned long long KF_LO_MASK = (1ull << 56) - 1ull;
__device__ __forceinline__ u128 kf_split(i128 v) {
  const unsigned long long lo = (unsigned long long)(u128)v & KF_LO_MASK;
  const unsigned long long hi = (unsigned long long)(long long)(v >> 56);
  return (u128)lo | ((u128)hi << 64);
}
__device__ __forceinline__ i128 kf_join(u128 w) {
  return (i128)(long long)(unsigned long long)(w >> 64) * ((i128)1 << 56) + (i128)(unsigned long long)w;
}

// The work-queue forest's queue (below): one 32-bit word per exit in the
// second pending-additions buffer, which that forest does not use otherwise.
template <int VK>
__device__ __forceinline__ uint32_t* kf_queue(const D8Params& P) {
  return VK != VK_NONE ? reinterpret_cast<uint32_t*>(P.ex_fx[1]) : reinterpret_cast<uint32_t*>(P.ex_cnt[1]);
}

// Link: each exit's local sum into fixed point (sum buffer 0; both
// pending buffers cleared -- for the work-queue forest only its queue
// word), and its parent -- the exit its water reaches
// next (block iterations: only inside its block).  An exit list that
// overflowed its capacity opens the engine's gate instead (block
// iterations: an error).  For the work-queue forest (QUEUE) each exit also
// counts itself among its parent's children (kf_children_of), starting
// from the zero that the tile pass that listed the exits left there.
template <int VK, bool CNT, bool ITER, bool QUEUE = false>
__global__ __launch_bounds__(256) void k_d8_link(D8Params P) {
  const uint32_t n = *P.n_exits;
  if (n > P.cap) {  // uniform
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (ITER) set_status(P.status, FR_ERR_CAPACITY);
      else P.ctl->fallback = 1;
    }
    return;
  }
  const int E = VK != VK_NONE ? fx_exponent<VK>(P, n) + (QUEUE ? KF_FX_HEAD : 0) : 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (QUEUE) {
      kf_queue<VK>(P)[i] = 0u;
    } else {
      if (VK != VK_NONE) {
        P.ex_fx[1][i] = 0;
        P.ex_fx[2][i] = 0;
      }
      if (CNT) {
        P.ex_cnt[1][i] = 0;
        P.ex_cnt[2][i] = 0;
      }
    }
    const uint32_t ec = P.ex_cell[i];
    uint32_t a = NONE;
    if (ec == NONE) {  // a hole of a phase-A chunk: no water, no parent
      if (VK != VK_NONE) P.ex_fx[0][i] = 0;
      if (CNT) P.ex_cnt[0][i] = 0;
      P.anc[0][i] = NONE;
      continue;
    }
    if (VK != VK_NONE) {
      const i128 v = VK == VK_FF ? fx_from(P.ex_hi[i], E) + fx_from(P.ex_lo[i], E) : fx_from(P.ex_d[i], E);
      P.ex_fx[0][i] = QUEUE ? kf_split(v) : (u128)v;
    }
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
    if (QUEUE && a < n) {
      if (CNT) atomicAdd(reinterpret_cast<unsigned long long*>(&P.ex_cnt[0][a]), 1ull);
      else atomicAdd(&P.anc[1][a], 1u);
    }
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

// ---------------------------------------------------------------------------
// The exit forest by a work queue (tile-forest path, where the forest holds
// tens of millions of exits and is about a thousand deep, so that pointer
// doubling would move every exit's sum through ten rounds of random
// atomics).  Each exit waits for its children; once the last one has added
// its total, the exit is final and enters the queue; whoever takes it adds
// its total to its parent, once.  Sums stay 128-bit integers (the order of
// the atomics changes no bit).  Children are counted by the link step
// (kf_children_of), the queue holds exit + 1 (0: not yet written)
// (kf_queue, cleared by the link step), and no addition is left pending
// for the totals.  Every access to the forest's shared words here is a
// device-coherent atomic, so the XCDs' caches need no write-back or
// invalidation; a finished exit's reads of its sums depend on the queue
// word that named it.  Every wait ends: a wavefront that sees the queue's
// tail stand still for KF_STALL_TICKS gives up (a cycle of exits, from
// malformed codes) and reports FR_ERR_NOTDAG.
constexpr int KF_HEAD = 8, KF_TAIL = 9;          // slots of P.flags
constexpr uint64_t KF_STALL_TICKS = 5000000ull;  // 50 ms of the 100 MHz clock

// An exit's count of children not yet final.  With counts it shares the
// 64-bit word of the exit's count sum (count << 32 | children; counts stay
// below 2^31), so that one atomic both adds a child's count and counts the
// child off; without counts it lives in anc[1].
template <bool CNT>
__device__ __forceinline__ uint32_t kf_children_of(const D8Params& P, uint32_t i) {
  return CNT ? (uint32_t)P.ex_cnt[0][i] : P.anc[1][i];
}

// Appends up to KF_PER_LANE items per lane (bit k of `mask`: par[k]) with
// one atomic per wavefront.
template <int K>
__device__ __forceinline__ void kf_push_many(const D8Params& P, uint32_t* q, uint32_t mask, const uint32_t (&par)[K]) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t incl = (uint32_t)__popc(mask);
  const uint32_t mine = incl;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
    if (lane >= (uint32_t)o) incl += y;
  }
  const uint32_t tot = (uint32_t)__shfl((int)incl, 63, 64);
  if (tot == 0u) return;  // uniform
  uint32_t base = 0;
  if (lane == 0)
    base = __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(&P.flags[KF_TAIL]), tot, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  uint32_t at = (uint32_t)__shfl((int)base, 0, 64) + incl - mine;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if ((mask >> k) & 1u) {
      __hip_atomic_store(&q[at], par[k] + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ++at;
    }
  }
}

// The leaves (holes included) into the queue: each workgroup scans a chunk
// of KF_LEAF_CHUNK exits and reserves its slots with one atomic (the queue's
// tail is one word: atomics on it serialise).
constexpr uint32_t KF_LEAF_PER_THREAD = 16;
constexpr uint32_t KF_LEAF_CHUNK = 256u * KF_LEAF_PER_THREAD;

template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_kf_leaves(D8Params P) {
  const uint32_t n = *P.n_exits;
  if (n > P.cap || n == 0u) return;  // uniform
  uint32_t* q = kf_queue<VK>(P);
  __shared__ uint32_t s_cnt[4], s_base;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (uint32_t c0 = blockIdx.x * KF_LEAF_CHUNK; c0 < n; c0 += gridDim.x * KF_LEAF_CHUNK) {  // uniform
    // Item j of the thread: exit c0 + 256 j + threadIdx.x.
    uint32_t mine = 0, leaf = 0;
#pragma unroll
    for (uint32_t j = 0; j < KF_LEAF_PER_THREAD; ++j) {
      const uint32_t i = c0 + 256u * j + threadIdx.x;
      if (i < n && kf_children_of<CNT>(P, i) == 0u) {
        leaf |= 1u << j;
        ++mine;
      }
    }
    // Exclusive prefix of the counts over the workgroup (wave scan, then
    // the four wave totals).
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == 63) s_cnt[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
      s_base = tot ? __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(&P.flags[KF_TAIL]), tot, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                   : 0u;
    }
    __syncthreads();
    uint32_t at = s_base + incl - mine;
    for (uint32_t w = 0; w < wave; ++w) at += s_cnt[w];
#pragma unroll
    for (uint32_t j = 0; j < KF_LEAF_PER_THREAD; ++j) {
      if ((leaf >> j) & 1u) {
        __hip_atomic_store(&q[at], c0 + 256u * j + threadIdx.x + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++at;
      }
    }
    __syncthreads();  // s_cnt and s_base are reused
  }
}

__device__ __forceinline__ u128 kf_load_fx(const u128* p) {
  const unsigned long long* w = reinterpret_cast<const unsigned long long*>(p);
  const u128 lo = __hip_atomic_load(const_cast<unsigned long long*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const u128 hi = __hip_atomic_load(const_cast<unsigned long long*>(w + 1), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
  return lo | (hi << 64);
}

// Persistent: each wavefront takes KF_SLOTS queue slots at a time (lane l
// holds slots base + 64 k + l) and each lane finishes the exits its slots
// receive, in whatever order they arrive; a slot is written only once its
// exit is final, and every exit is written exactly once, so all n slots
// fill (a cycle aside).
constexpr int KF_PER_LANE = 8;
constexpr uint32_t KF_SLOTS = 64u * KF_PER_LANE;

template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_kf_run(D8Params P) {
  constexpr int K = KF_PER_LANE;
  const uint32_t n = *P.n_exits;
  if (n > P.cap || n == 0u) return;  // uniform
  uint32_t* q = kf_queue<VK>(P);
  uint32_t* head = reinterpret_cast<uint32_t*>(&P.flags[KF_HEAD]);
  const uint32_t* tail = reinterpret_cast<const uint32_t*>(&P.flags[KF_TAIL]);
  const uint32_t lane = threadIdx.x & 63;
  uint32_t tail_seen = 0;
  uint64_t t_seen = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    uint32_t base = 0;
    if (lane == 0) base = __hip_atomic_fetch_add(head, KF_SLOTS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = (uint32_t)__shfl((int)base, 0, 64);
    if (base >= n) return;  // uniform: every slot has been taken
    uint32_t todo = 0;  // bit k: slot base + 64 k + lane not finished
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (base + 64u * k + lane < n) todo |= 1u << k;
    uint32_t avail = n;  // slots below the tail seen last (the others cannot be written yet)
    while (__ballot(todo != 0u)) {  // uniform
      // The lane's exits that have arrived are finished together, each step
      // issued for all of them before its results are waited for: the
      // queue words, the parents, the sums, the additions to the parents
      // (both words at once: they never carry), then one wait, then the
      // count-downs.  The parents made final go into the queue together.
      uint32_t e[K], par[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        e[k] = 0u;
        if (((todo >> k) & 1u) && base + 64u * k + lane < avail)
          e[k] = __hip_atomic_load(&q[base + 64u * k + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // The arrived exits' parents, sums and counts, loaded together (none
      // of them depends on another; a root's sums are loaded and unused).
      uint32_t got = 0;
      u128 x[K];
      unsigned long long c[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        par[k] = NONE;
        x[k] = 0;
        c[k] = 0ull;
        if (e[k] != 0u) {
          got |= 1u << k;
          e[k] -= 1u;
          par[k] = P.anc[0][e[k]];
          if (VK != VK_NONE) x[k] = kf_load_fx(&P.ex_fx[0][e[k]]);
          if (CNT)  // the exit's count (its children are all final: the low word is 0)
            c[k] = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&P.ex_cnt[0][e[k]]), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) >> 32;
        }
      }
      todo &= ~got;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (par[k] >= n) par[k] = NONE;
      if (VK != VK_NONE) {
        // The exit's total, split again, into its parent's two words: no
        // carry, no returned value.
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (par[k] != NONE) {
            const u128 w = kf_split(kf_join(x[k]));
            unsigned long long* pw = reinterpret_cast<unsigned long long*>(&P.ex_fx[0][par[k]]);
            if ((unsigned long long)w != 0ull)
              __hip_atomic_fetch_add(pw, (unsigned long long)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned long long)(w >> 64) != 0ull)
              __hip_atomic_fetch_add(pw + 1, (unsigned long long)(w >> 64), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      // The last child makes the parent final: the additions above have
      // completed (every access to the forest here is a device-coherent
      // atomic, so no cache needs writing back) before the children go
      // down, and a parent is queued only after its children have reached
      // zero.  With counts, one atomic adds the count and counts the child
      // off (count << 32, minus one).
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      uint32_t pmask = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (par[k] != NONE) {
          uint32_t left;
          if (CNT)
            left = (uint32_t)__hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(&P.ex_cnt[0][par[k]]),
                                                    (c[k] << 32) - 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          else
            left = __hip_atomic_fetch_add(&P.anc[1][par[k]], 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (left == 1u) pmask |= 1u << k;
        }
      }
      kf_push_many(P, q, pmask, par);
      if (__ballot(todo != 0u)) {
        // Waiting for slots still empty: give up when the queue stops
        // growing (the exits left form a cycle).
        uint32_t tl = 0;
        if (lane == 0) tl = __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tl = (uint32_t)__shfl((int)tl, 0, 64);
        avail = tl;
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        if (tl != tail_seen) {
          tail_seen = tl;
          t_seen = now;
        } else if (now - t_seen > KF_STALL_TICKS) {
          if (lane == 0) set_status(P.status, FR_ERR_NOTDAG);
          return;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
}

// The totals -- sums plus the last round's pending additions -- back from
// fixed point into float-float or float64, where phase C reads them (the
// pointer buffers' memory, free again); counts into sum buffer 0.  The
// work-queue forest leaves no pending additions, its count words are
// shifted down past their children, and with values each exit's total and
// count go out as one 16-byte record (tile_total_rec), so that the tile
// pass gathers one cache line per exit instead of three.
template <int VK, bool CNT, bool QUEUE = false>
__global__ __launch_bounds__(256) void k_d8_totals(D8Params P) {
  const uint32_t n = *P.n_exits;
  if (n > P.cap) return;  // uniform
  const int f = QUEUE ? 0 : P.ctl->forest_final;
  const int E = VK != VK_NONE ? fx_exponent<VK>(P, n) + (QUEUE ? KF_FX_HEAD : 0) : 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (QUEUE && VK != VK_NONE) {
      const i128 v = kf_join(P.ex_fx[0][i]);
      uint64_t w0;
      if (VK == VK_FF) {
        const ff t = fx_to_ff(v, E);
        w0 = (uint64_t)__float_as_uint(t.hi) | ((uint64_t)__float_as_uint(t.lo) << 32);
      } else {
        w0 = (uint64_t)__double_as_longlong(fx_to_double(v, E));
      }
      const uint64_t w1 = CNT ? P.ex_cnt[0][i] >> 32 : 0ull;
      *reinterpret_cast<ulonglong2*>(tile_total_rec(P, i)) = make_ulonglong2(w0, w1);
      continue;
    }
    if (CNT) P.ex_cnt[0][i] = QUEUE ? P.ex_cnt[0][i] >> 32 : P.ex_cnt[0][i] + P.ex_cnt[f][i];
    if (VK == VK_NONE) continue;
    const i128 v = (i128)(QUEUE ? P.ex_fx[0][i] : P.ex_fx[0][i] + P.ex_fx[f][i]);
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

// Workgroups of the queue kernel: as many as stay resident.
template <int VK, bool CNT>
unsigned kf_grid() {
  static unsigned g = 0;
  if (g == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_kf_run<VK, CNT>, 256, 0) != hipSuccess ||
        cus <= 0 || per <= 0) {
      cus = 256;
      per = 2;
    }
    g = (unsigned)(cus * per);
  }
  return g;
}

template <int VK, bool CNT>
hipError_t forest_queue_t(const D8Params& P, hipStream_t s) {
  const dim3 g(forest_grid(P.cap)), b(256);
  hipLaunchKernelGGL((k_d8_link<VK, CNT, false, true>), g, b, 0, s, P);
  hipLaunchKernelGGL((k_kf_leaves<VK, CNT>), g, b, 0, s, P);
  hipLaunchKernelGGL((k_kf_run<VK, CNT>), dim3(kf_grid<VK, CNT>()), b, 0, s, P);
  hipLaunchKernelGGL((k_d8_totals<VK, CNT, true>), g, b, 0, s, P);
  return hipGetLastError();
}

hipError_t launch_d8_forest_queue(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  if (vk == VK_FF) return cnt ? forest_queue_t<VK_FF, true>(P, s) : forest_queue_t<VK_FF, false>(P, s);
  if (vk == VK_F64) return cnt ? forest_queue_t<VK_F64, true>(P, s) : forest_queue_t<VK_F64, false>(P, s);
  return forest_queue_t<VK_NONE, true>(P, s);
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
