// Wavefront (64 lanes) and workgroup primitives shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fi_internal.h"

namespace fi {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-wide reductions with DPP lane moves (no LDS round trips): pairs and
// quads, half rows and rows, then rows 1 and 3 take the row before and rows 2
// and 3 take row 1, so lane 63 ends with the whole wave's result, which is
// returned to every lane.  Lanes a move leaves alone get `old` (the identity
// of a sum, or the lane's own value for idempotent operations).  Every lane of
// the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t x, uint32_t old) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t x, uint64_t old) {
  return ((uint64_t)dpp32<CTRL, ROWS>((uint32_t)(x >> 32), (uint32_t)(old >> 32)) << 32) |
         dpp32<CTRL, ROWS>((uint32_t)x, (uint32_t)old);
}
template <int CTRL, int ROWS, class T>
__device__ __forceinline__ T dpp_t(T x, T old) {
  if constexpr (sizeof(T) == 8) return (T)dpp64<CTRL, ROWS>((uint64_t)x, (uint64_t)old);
  else return (T)dpp32<CTRL, ROWS>((uint32_t)x, (uint32_t)old);
}
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror,
// row_bcast:15 (rows 1, 3), row_bcast:31 (rows 2, 3); lane 63's result
template <bool kZeroOld, class T, class Op>
__device__ __forceinline__ T wave_reduce(T x, Op op) {
  x = op(x, dpp_t<0xB1, 0xF>(x, kZeroOld ? T(0) : x));
  x = op(x, dpp_t<0x4E, 0xF>(x, kZeroOld ? T(0) : x));
  x = op(x, dpp_t<0x141, 0xF>(x, kZeroOld ? T(0) : x));
  x = op(x, dpp_t<0x140, 0xF>(x, kZeroOld ? T(0) : x));
  x = op(x, dpp_t<0x142, 0xA>(x, kZeroOld ? T(0) : x));
  x = op(x, dpp_t<0x143, 0xC>(x, kZeroOld ? T(0) : x));
  if constexpr (sizeof(T) == 8) {
    return (T)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), 63)
                << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, 63));
  } else {
    return (T)__builtin_amdgcn_readlane((int)x, 63);
  }
}

// Inclusive prefix sum over the wave: row shifts by 1, 2, 4 and 8 lanes, then
// the row broadcasts as above.  Every lane of the wave must be active.
__device__ __forceinline__ int wave_incl_sum_i32(int x) {
  x += (int)dpp32<0x111, 0xF>((uint32_t)x, 0u);
  x += (int)dpp32<0x112, 0xF>((uint32_t)x, 0u);
  x += (int)dpp32<0x114, 0xF>((uint32_t)x, 0u);
  x += (int)dpp32<0x118, 0xF>((uint32_t)x, 0u);
  x += (int)dpp32<0x142, 0xA>((uint32_t)x, 0u);
  x += (int)dpp32<0x143, 0xC>((uint32_t)x, 0u);
  return x;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
  return wave_reduce<false>(x, [](uint32_t a, uint32_t b) { return a | b; });
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  return wave_reduce<false>(x, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
  return wave_reduce<true>(x, [](uint64_t a, uint64_t b) { return a + b; });
}
// (LDS permutes here: the one hot caller, the randomized DFS step, shares its
// kernel with the one-tree-per-workgroup BFS, which ran a quarter slower when
// this minimum used DPP moves.)
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const uint64_t y = __shfl_xor(x, d);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ int wave_min_i32(int x) {
  return wave_reduce<false>(x, [](int a, int b) { return a < b ? a : b; });
}
__device__ __forceinline__ int wave_max_i32(int x) {
  return wave_reduce<false>(x, [](int a, int b) { return a > b ? a : b; });
}

// Wave-aggregated append: lanes with `pred` write `val` to consecutive slots
// of `list`, reserved with one atomicAdd on `counter` per wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t val, int32_t* list,
                                            uint32_t* counter) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) list[base + lanes_below(mask)] = val;
}

// Exclusive prefix sum over the workgroup.  `s_tmp` needs NT/64 + 1 ints of
// LDS.  Returns this thread's exclusive prefix; `total` gets the block sum.
// Ends with a barrier; callers may reuse s_tmp only after another barrier.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int x, int& total, int* s_tmp) {
  constexpr int NW = NT / 64;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  int inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == 63) s_tmp[w] = inc;
  __syncthreads();
  if (w == 0) {
    int v = lane < NW ? s_tmp[lane] : 0;
    int iv = v;
#pragma unroll
    for (int d = 1; d < NW; d <<= 1) {
      int y = __shfl_up(iv, d);
      if (lane >= d) iv += y;
    }
    if (lane < NW) s_tmp[lane] = iv - v;
    if (lane == NW - 1) s_tmp[NW] = iv;
  }
  __syncthreads();
  total = s_tmp[NW];
  return inc - x + s_tmp[w];
}

// Sum over the workgroup, valid in thread 0.  `s_tmp` needs NT/64 words.
template <int NT>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t* s_tmp) {
  x = wave_sum_u64(x);
  if (lane_id() == 0) s_tmp[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t r = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += s_tmp[i];
  }
  __syncthreads();
  return r;
}

// Largest k in [0, len) with a[k] <= x, for a non-decreasing a with a[0] <= x.
__device__ __forceinline__ int upper_index(const int* a, int len, int x) {
  int lo = 0, hi = len;  // answer in [lo, hi)
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_agent_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a cooperative launch (all workgroups co-resident).
// Arrival counter and generation live in separate cache lines of the
// control block; the generation is read before arriving so the release by
// the last workgroup cannot be missed.  Agent-scope fences on both sides make
// every store before the barrier visible to every load after it.
__device__ __forceinline__ void grid_barrier(uint64_t* ctl, uint32_t nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t* bar = ctl + C_BAR;
    uint64_t* gen = ctl + C_GEN;
    uint64_t g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    uint64_t arrived = __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(bar, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g)
        __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
  }
  __syncthreads();
}

// Insert one tree's result into the cloud (single thread).  New key: the
// first claimer of a slot sets its tag; every inserter then folds its fields
// in with commutative atomics.
__device__ __forceinline__ void cloud_insert(const DevGraph& G, uint64_t khi, uint64_t klo,
                                             uint64_t S, uint64_t t) {
  if (klo == kEmpty) {  // reserved tag value
    atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_COLLISION);
    return;
  }
  uint64_t idx = klo & G.cloud_mask;
  for (uint64_t probe = 0; probe <= G.cloud_mask; ++probe) {
    CloudSlot* s = G.cloud + idx;
    uint64_t old = atomicCAS((unsigned long long*)&s->tag, (unsigned long long)kEmpty,
                             (unsigned long long)klo);
    if (old == kEmpty || old == klo) {
      if (old == kEmpty) {
        uint64_t c = atomicAdd((unsigned long long*)(G.ctl + C_COUNT), 1ull);
        if (c + 1 > G.cloud_cap)
          atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_CAPACITY);
      }
      atomicMin((unsigned long long*)&s->khi_min, (unsigned long long)khi);
      atomicMax((unsigned long long*)&s->khi_max, (unsigned long long)khi);
      atomicMin((unsigned long long*)&s->s_min, (unsigned long long)S);
      atomicMax((unsigned long long*)&s->s_max, (unsigned long long)S);
      atomicAdd((unsigned long long*)&s->freq, 1ull);
      atomicMin((unsigned long long*)&s->first, (unsigned long long)t);
      atomicAdd((unsigned long long*)(G.ctl + C_TREES), 1ull);
      atomicMin((unsigned long long*)(G.ctl + C_BEST), (unsigned long long)((S << 32) | t));
      return;
    }
    idx = (idx + 1) & G.cloud_mask;
  }
  atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_CAPACITY);
}

// Barrier among `nb` workgroups of a cooperative launch (local ranks
// 0..nb-1): they arrive in groups of kBarGroup, the last of each group
// arrives at the root, the last root arrival bumps the generation.  bar:
// [0] generation, [16] root, [32 + 16 g] group g (each on its own line).
constexpr int kBarGroup = 16;
__device__ __forceinline__ void group_sync(uint64_t* bar, uint32_t rank, uint32_t nb) {
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t* gen = bar;
    uint64_t* root = bar + 16;
    const uint32_t g = rank / kBarGroup;
    const uint32_t ngroups = (nb + kBarGroup - 1) / kBarGroup;
    const uint32_t gsize = min((uint32_t)kBarGroup, nb - g * kBarGroup);
    uint64_t* grp = bar + 32 + 16 * g;
    const uint64_t g0 = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const uint64_t a = __hip_atomic_fetch_add(grp, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == gsize - 1) {
      __hip_atomic_store(grp, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t b = __hip_atomic_fetch_add(root, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (b == ngroups - 1) {
        __hip_atomic_store(root, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g0)
      __builtin_amdgcn_s_sleep(1);
    __threadfence();
  }
  __syncthreads();
}

}  // namespace fi
