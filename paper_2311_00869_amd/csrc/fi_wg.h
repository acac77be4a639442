// One tree on one workgroup: shared by the single-graph sweep (sweep.hip)
// and the batched sweep of many graphs (batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {
namespace wg {

__device__ __forceinline__ uint64_t amin64(uint64_t* p, uint64_t v) {
  return atomicMin((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void set_err(const DevGraph& G, uint64_t bit) {
  atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)bit);
}

template <int NT>
struct WgShared {
  int off[NT];
  int start[NT];
  uint64_t base[NT];
  int scan[NT / 64 + 1];
  uint64_t red[NT / 64];
  uint32_t tail;
};

// One tree on one workgroup.  pw[n] are the tree words, q[n] the BFS queue
// (level L occupies a contiguous range of it).
template <int NT>
__device__ __forceinline__ void wg_tree(const DevGraph& G, const SweepArgs& A, uint64_t t, uint64_t* pw,
                        int32_t* q, WgShared<NT>& sh) {
  const int tid = threadIdx.x;
  const int32_t n = G.n;
  const int32_t* rp = G.row_ptr;
  const KeyMix km = key_mix(tree_salt(A.seed, t));

  // (a) every vertex unreached
  for (int32_t v = tid; v < n; v += NT) pw[v] = kUnvisited;
  if (tid == 0) sh.tail = 0;
  __syncthreads();
  // (b) component roots: minimum key, accumulated in the anchor's word
  for (int32_t v = tid; v < n; v += NT)
    if (rp[v + 1] > rp[v]) amin64(pw + G.comp[v], root_candidate(vkey(km, v), v));
  __syncthreads();
  // (c) collect the roots of components with an edge
  for (int32_t v = tid; v < n; v += NT) {
    bool anchor = rp[v + 1] > rp[v] && G.comp[v] == v;
    int32_t r = anchor ? (int32_t)word_vertex(pw[v]) : 0;
    wave_append(anchor, r, q, &sh.tail);
  }
  __syncthreads();
  for (int32_t v = tid; v < n; v += NT)
    if (rp[v + 1] > rp[v] && G.comp[v] == v) pw[v] = kUnvisited;
  __syncthreads();
  const uint32_t nroots = sh.tail;
  for (uint32_t i = tid; i < nroots; i += NT) {
    int32_t r = q[i];
    pw[r] = tree_word(0, vkey(km, r), 0);
  }
  for (int32_t v = tid; v < n; v += NT)
    if (rp[v + 1] == rp[v]) pw[v] = tree_word(0, vkey(km, v), 0);
  __syncthreads();

  // (d) BFS, level by level; the frontier is q[lo, hi)
  uint32_t lo = 0, hi = nroots, L = 0;
  while (lo < hi) {
    if (L + 1 > kMaxLevel) {
      if (tid == 0) set_err(G, E_DEPTH);
      break;
    }
    for (uint32_t c0 = lo; c0 < hi; c0 += NT) {
      const uint32_t i = c0 + tid;
      int d = 0, st = 0;
      uint64_t base = 0;
      if (i < hi) {
        const int32_t u = q[i];
        st = rp[u];
        d = rp[u + 1] - st;
        base = tree_word(L + 1, vkey(km, u), (uint32_t)(pw[u] & 1));
      }
      int total;
      const int off = block_exclusive_scan<NT>(d, total, sh.scan);
      sh.off[tid] = off;
      sh.start[tid] = st;
      sh.base[tid] = base;
      __syncthreads();
      for (int j0 = 0; j0 < total; j0 += NT) {
        const int j = j0 + tid;
        bool found = false;
        int32_t v = 0;
        if (j < total) {
          const int k = upper_index(sh.off, NT, j);
          const uint32_t a = G.adj[sh.start[k] + (j - sh.off[k])];
          v = (int32_t)(a & kVertexMask);
          const uint64_t nw = sh.base[k] ^ (uint64_t)(a >> 31);
          if (pw[v] > nw) found = amin64(pw + v, nw) == kUnvisited;
        }
        wave_append(found, v, q, &sh.tail);
      }
      __syncthreads();
    }
    lo = hi;
    hi = sh.tail;
    ++L;
  }
  __syncthreads();

  // (e) canonical words (one wave per 64 vertices) and their key terms
  uint64_t khi = 0, klo = 0, S = 0;
  const int lane = lane_id(), wave = tid >> 6;
  for (int32_t i = wave; i < G.nwords; i += NT / 64) {
    const int32_t v = i * 64 + lane;
    uint32_t bit = 0;
    if (v < n) bit = (uint32_t)((pw[v] ^ pw[G.comp[v]]) & 1);
    const uint64_t W = __ballot(bit);
    if (lane == 0) {
      key_terms((uint64_t)i, W, khi, klo);
      if (A.bits_out) A.bits_out[i] = W;
    }
  }
  // (f) the exact count: frustrated iff neg xor b_u xor b_v
  for (int64_t e = tid; e < G.m; e += NT) {
    const uint2 uv = G.edges[e];
    const uint32_t v = uv.y & kVertexMask;
    S += ((uv.y >> 31) ^ (uint32_t)(pw[uv.x] ^ pw[v])) & 1u;
  }
  khi = block_sum_u64<NT>(khi, sh.red);
  klo = block_sum_u64<NT>(klo, sh.red);
  S = block_sum_u64<NT>(S, sh.red);
  if (tid == 0) {
    if (A.insert) cloud_insert(G, khi, klo, S, t);
    if (A.tree_switches) A.tree_switches[t - A.t0] = S;
  }
  __syncthreads();
}


}  // namespace wg
}  // namespace fi
