// Which trees share a pass of the multi-tree sweep.
//
// A pass walks the rows of every vertex that some of its trees have not yet
// visited, once per BFS level, and the walk costs about one step per edge
// that hits at least one of its trees.  Trees whose levels agree on most
// vertices share those steps; trees whose roots lie at different distances
// from the graph's core reach each vertex at different levels and so need
// separate steps.  The sweep therefore takes the trees of a block (up to
// kOrderMax) in the order of their roots' distance to the core, measured as
// the sum of BFS distances to the kHubs vertices of highest degree, then by
// decreasing root degree, then by tree index.  Every tree's result depends
// only on (graph, seed, tree), and the cloud combines trees with
// commutative atomics, so the order changes the speed and nothing else.
//
// At upload: the distance sums (one multi-source BFS, one bit per hub).
// Per block of trees: the root of each tree in the component with the most
// vertices (its minimum-key vertex, the root rule of the sampler), then the
// sort; the pass reads these roots instead of searching that component again.
// A large component's roots come from inverting the key (k_main_roots_inv).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {
namespace {

constexpr int kHubs = 8;
constexpr int32_t kCentMinVertices = 65536;  // main components below this keep tree order
constexpr int kChunk = 4096;                  // vertices per root-search task
constexpr int32_t kInvertMin = 1 << 18;       // main components from this size invert the key
constexpr int kInvPerLane = 4;                // candidate keys per lane and step
constexpr int32_t kCentWide = 256;            // rows longer than this take a wave each

// Inverse of an odd a mod 2^32 by Newton's iteration x <- x (2 - a x): a is
// its own inverse mod 8, and every step doubles the number of correct bits.
__host__ __device__ constexpr uint32_t inv_odd(uint32_t a) {
  uint32_t x = a;
  for (int i = 0; i < 4; ++i) x *= 2u - a * x;
  return x;
}

// Inverse of fmix32: its five steps undone in reverse order.  A shift-xor
// y = x ^ (x >> s) is undone by x = y ^ (y >> s) ^ (y >> 2s) ^ ... while
// the shifts stay below 32 bits.
__host__ __device__ constexpr uint32_t fmix32_inv(uint32_t h) {
  h ^= h >> 16;
  h *= inv_odd(0xC2B2AE35u);
  h ^= (h >> 13) ^ (h >> 26);
  h *= inv_odd(0x85EBCA6Bu);
  h ^= h >> 16;
  return h;
}
static_assert(inv_odd(0x85EBCA6Bu) * 0x85EBCA6Bu == 1u && inv_odd(0xC2B2AE35u) * 0xC2B2AE35u == 1u,
              "inverse of an odd multiplier");
static_assert(fmix32_inv(fmix32(0u)) == 0u && fmix32_inv(fmix32(1u)) == 1u &&
                  fmix32_inv(fmix32(0x7FFFFFFFu)) == 0x7FFFFFFFu &&
                  fmix32_inv(fmix32(0xDEADBEEFu)) == 0xDEADBEEFu &&
                  fmix32_inv(fmix32(16000000u)) == 16000000u,
              "fmix32 inverse");

inline int grid_for(int64_t work, int block, int cap = 65536) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + block - 1) / block, cap));
}

__global__ void k_cent_clear(int32_t n, uint8_t* vis, uint8_t* front, uint16_t* dsum) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    vis[v] = 0;
    front[v] = 0;
    dsum[v] = 0;
  }
}

// Hub h (distinct vertices) starts its BFS: bit h of its visit and frontier bytes.
__global__ void k_cent_seed(const int32_t* hubs, int nh, uint8_t* vis, uint8_t* front) {
  const int h = threadIdx.x;
  if (h < nh) {
    vis[hubs[h]] = (uint8_t)(1u << h);
    front[hubs[h]] = (uint8_t)(1u << h);
  }
}

// One BFS level for all hubs at once: a vertex not yet reached by every hub
// takes the hubs that reached one of its neighbours at the previous level,
// and adds `level` for each of them to its distance sum.  Rows longer than
// kCentWide are left to k_cent_wide.
__device__ __forceinline__ void cent_take(int32_t v, uint8_t have, uint8_t nb, uint8_t* next,
                                          uint8_t* vis, uint16_t* dsum, uint32_t level, bool& grew) {
  const uint8_t fresh = (uint8_t)(nb & ~have);
  next[v] = fresh;
  if (fresh) {
    vis[v] = (uint8_t)(have | fresh);
    dsum[v] = (uint16_t)min(65535u, (uint32_t)dsum[v] + level * (uint32_t)__popc(fresh));
    grew = true;
  }
}

__global__ void k_cent_level(const int32_t* rp, const uint32_t* adj, int32_t n, uint8_t full,
                             const uint8_t* front, uint8_t* next, uint8_t* vis, uint16_t* dsum,
                             uint32_t level, uint32_t* any) {
  bool grew = false;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (rp[v + 1] - rp[v] > kCentWide) continue;
    const uint8_t have = vis[v];
    uint8_t nb = 0;
    if (have != full) {
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
        nb |= front[adj[e] & kVertexMask];
        if ((uint8_t)(nb | have) == full) break;
      }
    }
    cent_take((int32_t)v, have, nb, next, vis, dsum, level, grew);
  }
  if (__ballot(grew) && lane_id() == 0) atomicOr(any, 1u);
}

// The same step for the rows longer than kCentWide (rows[0, nrows)), one
// wave per row, its lanes over the row's entries.
__global__ void k_cent_wide(const int32_t* rp, const uint32_t* adj, const int32_t* rows,
                            int32_t nrows, uint8_t full, const uint8_t* front, uint8_t* next,
                            uint8_t* vis, uint16_t* dsum, uint32_t level, uint32_t* any) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool grew = false;
  for (int64_t k = wave; k < nrows; k += nwaves) {
    const int32_t v = rows[k];
    const uint8_t have = vis[v];
    uint32_t nb = 0;
    if (have != full) {
      const int32_t e1 = rp[v + 1];
      for (int32_t c = rp[v]; c < e1; c += 64) {
        if (c + lane < e1) nb |= front[adj[c + lane] & kVertexMask];
        if ((uint8_t)(wave_or_u32(nb) | have) == full) break;
      }
      nb = wave_or_u32(nb);
    }
    if (lane == 0) cent_take(v, have, (uint8_t)nb, next, vis, dsum, level, grew);
  }
  if (lane == 0 && grew) atomicOr(any, 1u);
}

__global__ void k_fill64(uint64_t* p, int64_t len, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Root candidates (key << 32 | vertex << 1) of trees t0 .. t0 + count - 1 in
// the main component (cverts[b, e)): one wave per (64 trees, kChunk
// vertices), lane t the minimum for its tree, then one atomic minimum per
// tree.  Two running minima keep two compare chains in flight.
__global__ void k_main_roots(const int32_t* cverts, int32_t b, int32_t e, uint64_t seed,
                             uint64_t t0, uint32_t count, uint64_t* oroot) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t nchunks = ((int64_t)e - b + kChunk - 1) / kChunk;
  const int64_t ngroups = (count + 63) / 64;
  for (int64_t task = wave; task < nchunks * ngroups; task += nwaves) {
    const int64_t gi = task / nchunks, ci = task - gi * nchunks;
    const uint32_t slot = (uint32_t)(gi * 64 + lane);
    const KeyMix km = key_mix(tree_salt(seed, t0 + slot));
    uint64_t best = kUnvisited, alt = kUnvisited;
    const int32_t c0 = b + (int32_t)(ci * kChunk), c1 = min(e, c0 + kChunk);
    for (int32_t c = c0; c < c1; c += 64) {
      const int32_t mine = c + lane < c1 ? cverts[c + lane] : 0;
      const uint32_t hm = fmix32((uint32_t)mine);
      const int cnt = min(64, c1 - c);
      int j = 0;
      for (; j + 1 < cnt; j += 2) {
        const uint32_t v0 = (uint32_t)__builtin_amdgcn_readlane(mine, j);
        const uint32_t h0 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j);
        const uint32_t v1 = (uint32_t)__builtin_amdgcn_readlane(mine, j + 1);
        const uint32_t h1 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j + 1);
        const uint64_t k0 = root_candidate(vkey_of(km, h0), v0);
        const uint64_t k1 = root_candidate(vkey_of(km, h1), v1);
        best = k0 < best ? k0 : best;
        alt = k1 < alt ? k1 : alt;
      }
      if (j < cnt) {
        const uint32_t v0 = (uint32_t)__builtin_amdgcn_readlane(mine, j);
        const uint32_t h0 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j);
        const uint64_t k0 = root_candidate(vkey_of(km, h0), v0);
        best = k0 < best ? k0 : best;
      }
    }
    best = alt < best ? alt : best;
    if (slot < count) atomicMin((unsigned long long*)(oroot + slot), (unsigned long long)best);
  }
}

// The same root candidates for a main component of at least kInvertMin
// vertices, by inverting the key instead of scanning the component.  A
// tree's key is a bijection of the 32-bit vertex id, so its smallest key on
// the component is the first k = 0, 1, 2, ... whose preimage
// u = fmix32^-1((k * m^-1) xor x) is a vertex (u < n) of that component:
// about 2^32 / |component| candidates per tree instead of |component|.  One
// wave per tree tests 64 kInvPerLane consecutive keys per step; every key
// has a preimage and some vertex of the component holds a key, so the walk
// ends by k = 2^32 - 1 at the latest.
__global__ void k_main_roots_inv(const int32_t* comp, const int32_t* cverts, int32_t b, int32_t n,
                                 uint64_t seed, uint64_t t0, uint32_t count, uint64_t* oroot) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int32_t label = comp[cverts[b]];
  for (int64_t t = wave; t < count; t += nwaves) {
    const KeyMix km = key_mix(tree_salt(seed, t0 + (uint64_t)t));
    const uint32_t minv = inv_odd(km.m);
    uint64_t found = kUnvisited;
    for (uint64_t base = 0; base < (1ull << 32) && found == kUnvisited; base += 64 * kInvPerLane) {
      uint32_t u[kInvPerLane];
      bool hit[kInvPerLane];
#pragma unroll
      for (int i = 0; i < kInvPerLane; ++i)
        u[i] = fmix32_inv(((uint32_t)base + (uint32_t)(64 * i + lane)) * minv ^ km.x);
#pragma unroll
      for (int i = 0; i < kInvPerLane; ++i) hit[i] = u[i] < (uint32_t)n && comp[u[i]] == label;
#pragma unroll
      for (int i = 0; i < kInvPerLane; ++i) {
        const uint64_t bal = __ballot(hit[i]);
        if (bal && found == kUnvisited) {
          const int j = __ffsll((unsigned long long)bal) - 1;
          const uint32_t k = (uint32_t)base + (uint32_t)(64 * i + j);
          found = root_candidate(k, (uint32_t)__builtin_amdgcn_readlane((int)u[i], j));
        }
      }
    }
    if (lane == 0) oroot[t] = found;
  }
}

// Sort keys of the block's trees and their order: (distance sum of the
// root, 0xFFFF - min(root degree, 0xFFFF), tree offset), ascending, by a
// bitonic sort of the next power of two entries in LDS (padding sorts last).
constexpr int kSortThreads = 1024;
__global__ void __launch_bounds__(kSortThreads) k_order(const uint64_t* oroot, const uint16_t* dsum,
                                                        const int32_t* rp, uint32_t count,
                                                        uint32_t npow, uint64_t t0, uint32_t* perm) {
  __shared__ uint64_t key[kOrderMax];
  for (uint32_t i = threadIdx.x; i < npow; i += kSortThreads) {
    uint64_t k = ~0ull;
    if (i < count) {
      const uint32_t r = word_vertex(oroot[i]);
      const uint32_t deg = (uint32_t)min(0xFFFF, rp[r + 1] - rp[r]);
      k = ((uint64_t)dsum[r] << 48) | ((uint64_t)(0xFFFFu - deg) << 32) | i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= npow; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < npow; i += kSortThreads) {
        const uint32_t p = i ^ j;
        if (p > i) {
          const uint64_t a = key[i], c = key[p];
          if ((a > c) == ((i & k) == 0)) {
            key[i] = c;
            key[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < count; i += kSortThreads)
    perm[i] = (uint32_t)(t0 + (uint32_t)key[i]);
}

}  // namespace

int centrality_setup(fi_graph* g, hipStream_t s) {
  g->cent = false;
  const int32_t n = g->dg.n;
  if (g->main_big < 0 || g->main_end - g->main_begin < kCentMinVertices) return FI_OK;
  // the kHubs vertices of highest degree (ties to the smaller id)
  std::vector<int32_t> rp((size_t)n + 1);
  if (hipMemcpyAsync(rp.data(), g->dg.row_ptr, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FI_EDEVICE;
  std::vector<int32_t> order(n);
  for (int32_t v = 0; v < n; ++v) order[v] = v;
  const int nh = std::min<int32_t>(kHubs, n);
  std::partial_sort(order.begin(), order.begin() + nh, order.end(), [&](int32_t a, int32_t b) {
    const int32_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
    return da != db ? da > db : a < b;
  });
  uint8_t* vis = (uint8_t*)(g->ws + g->L.scratch);
  uint8_t* front = vis + n;
  uint8_t* next = front + n;
  uint32_t* any = (uint32_t*)(g->ws + g->L.oroot);
  int32_t* hubs = (int32_t*)(g->ws + g->L.operm);
  uint16_t* dsum = (uint16_t*)(g->ws + g->L.cent);
  // the long rows, after the three byte maps (the scratch region holds 8 (n + 64) bytes)
  std::vector<int32_t> wide;
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] - rp[v] > kCentWide) wide.push_back(v);
  int32_t* rows = (int32_t*)(g->ws + g->L.scratch + ((3 * (size_t)n + 255) & ~(size_t)255));
  if (hipMemcpyAsync(hubs, order.data(), 4 * nh, hipMemcpyHostToDevice, s) != hipSuccess ||
      (!wide.empty() && hipMemcpyAsync(rows, wide.data(), 4 * wide.size(), hipMemcpyHostToDevice,
                                       s) != hipSuccess))
    return FI_EDEVICE;
  const int32_t nwide = (int32_t)wide.size();
  hipLaunchKernelGGL(k_cent_clear, dim3(grid_for(n, 256)), dim3(256), 0, s, n, vis, front, dsum);
  hipLaunchKernelGGL(k_cent_seed, dim3(1), dim3(64), 0, s, (const int32_t*)hubs, nh, vis, front);
  const uint8_t full = (uint8_t)((1u << nh) - 1);
  for (uint32_t level = 1;; ++level) {
    uint32_t grew = 0;
    if (hipMemsetAsync(any, 0, 4, s) != hipSuccess) return FI_EDEVICE;
    hipLaunchKernelGGL(k_cent_level, dim3(grid_for(n, 256)), dim3(256), 0, s, g->dg.row_ptr, g->dg.adj,
                       n, full, (const uint8_t*)front, next, vis, dsum, level, any);
    if (nwide > 0)
      hipLaunchKernelGGL(k_cent_wide, dim3(grid_for((int64_t)nwide * 64, 256)), dim3(256), 0, s,
                         g->dg.row_ptr, g->dg.adj, (const int32_t*)rows, nwide, full,
                         (const uint8_t*)front, next, vis, dsum, level, any);
    if (hipMemcpyAsync(&grew, any, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FI_EDEVICE;
    std::swap(front, next);
    if (!grew) break;
  }
  if (hipGetLastError() != hipSuccess) return FI_EDEVICE;
  g->cent = true;
  return FI_OK;
}

hipError_t order_trees(fi_graph* g, uint64_t seed, uint64_t t0, uint32_t count, hipStream_t s) {
  if (count == 0 || count > (uint32_t)kOrderMax) return hipErrorInvalidValue;
  uint64_t* oroot = (uint64_t*)(g->ws + g->L.oroot);
  uint32_t* perm = (uint32_t*)(g->ws + g->L.operm);
  const int32_t* cverts = (const int32_t*)(g->ws + g->L.cverts);
  if (g->main_end - g->main_begin >= kInvertMin) {
    hipLaunchKernelGGL(k_main_roots_inv, dim3(grid_for((int64_t)count * 64, 256)), dim3(256), 0, s,
                       g->dg.comp, cverts, g->main_begin, g->dg.n, seed, t0, count, oroot);
  } else {
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(count, 256)), dim3(256), 0, s, oroot, (int64_t)count,
                       kUnvisited);
    const int64_t nchunks = ((int64_t)g->main_end - g->main_begin + kChunk - 1) / kChunk;
    const int64_t tasks = nchunks * (((int64_t)count + 63) / 64);
    hipLaunchKernelGGL(k_main_roots, dim3(grid_for(tasks * 64, 256, 8192)), dim3(256), 0, s, cverts,
                       g->main_begin, g->main_end, seed, t0, count, oroot);
  }
  uint32_t npow = 1;
  while (npow < count) npow <<= 1;
  hipLaunchKernelGGL(k_order, dim3(1), dim3(kSortThreads), 0, s, (const uint64_t*)oroot,
                     (const uint16_t*)(g->ws + g->L.cent), g->dg.row_ptr, count, npow, t0, perm);
  return hipGetLastError();
}

}  // namespace fi
