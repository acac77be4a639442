// The balanced state Sigma' as a list of edges to switch: for a vertex state
// (n bits, set = -1), the undirected edges it frustrates, which are exactly
// the edges Alg. alg-balance switches when the state is a tree's (Theorem
// t:HararyCut), and the edges Alg. alg-gradient flips when it is a rounded
// graphL state.  The list keeps the upper-triangle edge order (u < v,
// increasing (u, v)), so it is unique.
//
// Ordered compaction in three launches over tiles of kTile edges:
// count each tile, scan the tile counts in one workgroup, then write each
// tile's edges in order (rounds of kBlock consecutive edges, ranked by a
// ballot prefix inside waves and a workgroup scan across them).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"
#include "frustration.h"

namespace fi {
namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 16;
constexpr int kTile = kBlock * kRounds;  // edges per tile
constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint32_t frustrated(const uint2 uv, const uint64_t* bits) {
  const uint32_t u = uv.x, v = uv.y & kVertexMask;
  const uint32_t bu = (uint32_t)(bits[u >> 6] >> (u & 63)) & 1u;
  const uint32_t bv = (uint32_t)(bits[v >> 6] >> (v & 63)) & 1u;
  return (uv.y >> 31) ^ bu ^ bv;
}

// Bit r of the result: edge base + r * kBlock + threadIdx.x is frustrated.
// All kRounds edge loads are issued before the state gathers that depend on
// them, so each thread has kRounds independent chains in flight.
__device__ __forceinline__ uint32_t tile_flags(const uint2* edges, int64_t m, int64_t base,
                                               const uint64_t* bits, uint2* uv) {
  // the edge list streams once: non-temporal loads keep the state bitmap,
  // which every edge gathers from twice, resident in L2
  const uint64_t* ev = reinterpret_cast<const uint64_t*>(edges);
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = base + r * kBlock + threadIdx.x;
    const uint64_t w = e < m ? __builtin_nontemporal_load(ev + e) : 0ull;
    uv[r] = make_uint2((uint32_t)w, (uint32_t)(w >> 32));
  }
  uint32_t f = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t e = base + r * kBlock + threadIdx.x;
    if (e < m) f |= frustrated(uv[r], bits) << r;
  }
  return f;
}

__global__ void __launch_bounds__(kBlock) k_sw_count(const uint2* edges, int64_t m,
                                                      const uint64_t* bits, uint32_t* tile_cnt) {
  __shared__ uint64_t s_tmp[kBlock / 64];
  uint2 uv[kRounds];
  const uint32_t f = tile_flags(edges, m, (int64_t)blockIdx.x * kTile, bits, uv);
  const uint64_t tot = block_sum_u64<kBlock>((uint64_t)__popc(f), s_tmp);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = (uint32_t)tot;
}

// Exclusive offsets of the tiles (one workgroup) and the total.
__global__ void __launch_bounds__(kScanThreads) k_sw_scan(const uint32_t* tile_cnt, int64_t ntiles,
                                                           uint64_t* tile_off, uint64_t* total) {
  __shared__ uint64_t s_w[kScanThreads / 64 + 1];
  const int64_t per = (ntiles + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  const int64_t b1 = min(ntiles, b0 + per);
  uint64_t mine = 0;
  for (int64_t i = b0; i < b1; ++i) mine += tile_cnt[i];
  // workgroup exclusive scan of `mine`
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint64_t inc = mine;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      const uint64_t t = s_w[i];
      s_w[i] = run;
      run += t;
    }
    s_w[kScanThreads / 64] = run;
  }
  __syncthreads();
  uint64_t off = inc - mine + s_w[w];
  for (int64_t i = b0; i < b1; ++i) {
    tile_off[i] = off;
    off += tile_cnt[i];
  }
  if (threadIdx.x == 0) *total = s_w[kScanThreads / 64];
}

__global__ void __launch_bounds__(kBlock) k_sw_write(const uint2* edges, int64_t m,
                                                      const uint64_t* bits, const uint64_t* tile_off,
                                                      int32_t* out, int64_t cap) {
  __shared__ uint32_t s_w[kRounds][kBlock / 64];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint2 uv[kRounds];
  const uint32_t f = tile_flags(edges, m, (int64_t)blockIdx.x * kTile, bits, uv);
  uint64_t mask[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    mask[r] = __ballot((f >> r) & 1u);
    if (lane == 0) s_w[r][w] = (uint32_t)__popcll(mask[r]);
  }
  __syncthreads();
  // edges are ordered by (round, wave, lane) inside the tile
  uint64_t off = tile_off[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    uint32_t before = 0, round = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
      const uint32_t c = s_w[r][i];
      before += i < w ? c : 0u;
      round += c;
    }
    if ((f >> r) & 1u) {
      const uint64_t at = off + before + lanes_below(mask[r]);
      if ((int64_t)at < cap) {
        out[2 * at] = (int32_t)uv[r].x;
        out[2 * at + 1] = (int32_t)(uv[r].y & kVertexMask);
      }
    }
    off += round;
  }
}

__global__ void k_edge_list(const uint2* edges, int64_t m, int32_t* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint2 uv = edges[e];
    out[2 * e] = (int32_t)uv.x;
    out[2 * e + 1] = (int32_t)(uv.y & kVertexMask);
  }
}

}  // namespace

int64_t switch_tiles(int64_t m) { return (m + kTile - 1) / kTile; }

}  // namespace fi

using namespace fi;

extern "C" {

int fi_edge_list(fi_graph* g, int32_t* d_uv_out, void* stream) {
  if (!g || g->is_batch || !d_uv_out) return FI_EINVAL;
  const int64_t m = g->dg.m;
  if (m == 0) return FI_OK;
  const int grid = (int)std::min<int64_t>((m + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL(k_edge_list, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, g->dg.edges, m,
                     d_uv_out);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_switch_list(fi_graph* g, const uint64_t* d_bits, int32_t* d_uv_out, int64_t cap,
                   uint64_t* d_count, void* stream) {
  if (!g || g->is_batch || !d_bits || !d_count || cap < 0 || (cap > 0 && !d_uv_out))
    return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t m = g->dg.m;
  const int64_t ntiles = switch_tiles(m);
  uint32_t* cnt = (uint32_t*)(g->ws + g->L.swtile);
  uint64_t* off = (uint64_t*)(g->ws + g->L.swtile + 8 * (size_t)(ntiles + 1));
  if (ntiles > 0)
    hipLaunchKernelGGL(k_sw_count, dim3((unsigned)ntiles), dim3(kBlock), 0, s, g->dg.edges, m,
                       d_bits, cnt);
  hipLaunchKernelGGL(k_sw_scan, dim3(1), dim3(kScanThreads), 0, s, cnt, ntiles, off, d_count);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_sw_write, dim3((unsigned)ntiles), dim3(kBlock), 0, s, g->dg.edges, m,
                       d_bits, off, d_uv_out, cap);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
