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

template <int NT>
__device__ __forceinline__ void wg_finish(const DevGraph& G, const SweepArgs& A, uint64_t t,
                                          const uint64_t* pw, WgShared<NT>& sh);

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
  wg_finish<NT>(G, A, t, pw, sh);
}

// (e), (f) and the cloud insert for a tree whose states are bit 0 of pw.
template <int NT>
__device__ __forceinline__ void wg_finish(const DevGraph& G, const SweepArgs& A, uint64_t t,
                                          const uint64_t* pw, WgShared<NT>& sh) {
  const int tid = threadIdx.x;
  const int32_t n = G.n;
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

// ------------------------------------------------------------ other samplers
// Section "Tree-Sampling techniques for graphBpp" and Alg. alg-hybrid, with
// all randomness from the tree's salt as for BFS.  Only bit 0 of pw (the
// state, 1 = -1) matters to wg_finish; other bits mark visited vertices.
constexpr uint64_t kVisited = 1ull << 62;

// Alg. alg-hybrid's 0/1: the top bit of the SplitMix64 finalizer of the salt.
__device__ __forceinline__ int hybrid_coin(uint64_t salt) { return (int)(mix64(salt) >> 63); }

// Randomized DFS: from the current vertex, move to the unvisited neighbour
// of smallest key (the shuffled adjacency order), back up when there is
// none; one search per component from its minimum-key vertex.  A wave runs
// one component at a time (lanes scan the adjacency, a wave minimum picks);
// the waves of the workgroup take components in turn.  The search stack of
// component k lives in q[cptr[k] ..), one slot per vertex of the component.
template <int NT>
__device__ __forceinline__ void wg_tree_rdfs(const DevGraph& G, const SweepArgs& A, uint64_t t,
                                             uint64_t* pw, int32_t* q, WgShared<NT>& sh) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int32_t n = G.n;
  const int32_t* rp = G.row_ptr;
  const KeyMix km = key_mix(tree_salt(A.seed, t));
  const int32_t nanch = (int32_t)G.ctl[C_NANCH];
  (void)sh;
  for (int32_t v = tid; v < n; v += NT) pw[v] = rp[v + 1] > rp[v] ? kUnvisited : kVisited;
  __syncthreads();
  for (int32_t v = tid; v < n; v += NT)
    if (rp[v + 1] > rp[v]) amin64(pw + G.comp[v], root_candidate(vkey(km, v), v));
  __syncthreads();
  for (int32_t k = tid; k < nanch; k += NT) q[A.cptr[k]] = (int32_t)word_vertex(pw[G.anchors[k]]);
  __syncthreads();
  for (int32_t k = tid; k < nanch; k += NT) pw[G.anchors[k]] = kUnvisited;
  __syncthreads();
  for (int32_t k = wave; k < nanch; k += NT / 64) {
    int32_t* stk = q + A.cptr[k];
    int32_t u = stk[0];
    uint32_t bu = 0;
    if (lane == 0) pw[u] = kVisited;
    __threadfence_block();
    int32_t top = 0;
    while (true) {
      const int64_t e0 = rp[u], e1 = rp[u + 1];
      uint64_t best = ~0ull;
      for (int64_t e = e0 + lane; e < e1; e += 64) {
        const uint32_t v = G.adj[e] & kVertexMask;
        if (pw[v] == kUnvisited) {
          const uint64_t c = (uint64_t)vkey(km, v) << 32 | (uint64_t)(e - e0);
          best = c < best ? c : best;
        }
      }
      // the smallest key wins (the keys of one row's neighbours are
      // distinct): a 32-bit wave minimum, then the lane that holds it
      const bool has = best != ~0ull;
      if (!__ballot(has)) {  // every neighbour visited: back up
        if (top == 0) break;
        --top;
        u = stk[top];
        bu = (uint32_t)(pw[u] & 1);
        continue;
      }
      const uint32_t bk = (uint32_t)(best >> 32);
      const uint32_t kmin = wave_reduce<false>(has ? bk : 0xFFFFFFFFu,
                                               [](uint32_t x, uint32_t y) { return x < y ? x : y; });
      const int wl = __builtin_ctzll(__ballot(has && bk == kmin));
      const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)best, wl);
      const uint32_t a = G.adj[e0 + (int64_t)off];
      const int32_t v = (int32_t)(a & kVertexMask);
      bu ^= a >> 31;
      ++top;
      if (lane == 0) {
        pw[v] = kVisited | bu;
        stk[top] = v;
      }
      __threadfence_block();
      u = v;
    }
  }
  __syncthreads();
}

// Kruskal on random edge weights, as Boruvka rounds: each tree of the forest
// takes its lightest outgoing edge (weight, then position in the edge list:
// a strict order, so the result is the unique minimum spanning forest, the
// one Kruskal's algorithm builds) and hooks onto the tree across it; when
// two trees take the same edge, the larger root hooks.  q[v] = parent | parity
// << 31 (a union-find whose parity is v's state relative to its parent),
// flattened after every round so that every vertex points at its root;
// pw[r] collects root r's lightest edge, d[r] its hook.
__device__ __forceinline__ uint32_t kruskal_weight(uint64_t salt, uint32_t u, uint32_t v) {
  return (uint32_t)(mix64(salt ^ ((uint64_t)u << 32 | v)) >> 32);
}

template <int NT>
__device__ __forceinline__ void wg_tree_kruskal(const DevGraph& G, const SweepArgs& A, uint64_t t,
                                                uint64_t* pw, int32_t* q, int32_t* d,
                                                WgShared<NT>& sh) {
  const int tid = threadIdx.x;
  const int32_t n = G.n;
  const uint64_t salt = tree_salt(A.seed, t);
  constexpr uint32_t kPar = 0x80000000u, kPtr = 0x7FFFFFFFu;
  for (int32_t v = tid; v < n; v += NT) q[v] = v;
  __syncthreads();
  for (int round = 0; round < 64; ++round) {
    for (int32_t v = tid; v < n; v += NT) pw[v] = ~0ull;
    if (tid == 0) sh.tail = 0;
    __syncthreads();
    for (int64_t e = tid; e < G.m; e += NT) {
      const uint2 uv = G.edges[e];
      const uint32_t u = uv.x, v = uv.y & kVertexMask;
      const uint32_t ru = (uint32_t)q[u] & kPtr, rv = (uint32_t)q[v] & kPtr;
      if (ru == rv) continue;
      const uint64_t key = (uint64_t)kruskal_weight(salt, u, v) << 32 | (uint64_t)e;
      if (pw[ru] > key) amin64(pw + ru, key);
      if (pw[rv] > key) amin64(pw + rv, key);
    }
    __syncthreads();
    // decide every hook before any is made (q and pw stay unchanged here)
    for (int32_t r = tid; r < n; r += NT) {
      int32_t h = -1;
      const uint64_t key = pw[r];
      if (((uint32_t)q[r] & kPtr) == (uint32_t)r && key != ~0ull) {
        const uint2 uv = G.edges[key & 0xFFFFFFFFull];
        const uint32_t u = uv.x, v = uv.y & kVertexMask;
        const uint32_t qu = (uint32_t)q[u], qv = (uint32_t)q[v];
        const uint32_t other = (qu & kPtr) == (uint32_t)r ? (qv & kPtr) : (qu & kPtr);
        // parity(r -> other) = parity(u) ^ parity(v) ^ [edge negative]
        const uint32_t par = ((qu ^ qv) >> 31) ^ (uv.y >> 31);
        if (pw[other] != key || (uint32_t)r > other) h = (int32_t)(other | par << 31);
      }
      d[r] = h;
    }
    __syncthreads();
    uint32_t hooked = 0;
    for (int32_t r = tid; r < n; r += NT)
      if (d[r] != -1) {
        q[r] = d[r];
        hooked = 1;
      }
    if (hooked) sh.tail = 1;
    __syncthreads();
    if (sh.tail == 0) break;
    // pointer jumping with parities until every vertex points at its root
    while (true) {
      __syncthreads();
      if (tid == 0) sh.tail = 0;
      __syncthreads();
      uint32_t moved = 0;
      for (int32_t v = tid; v < n; v += NT) {
        const uint32_t qv = (uint32_t)q[v];
        const uint32_t p = qv & kPtr;
        const uint32_t qp = (uint32_t)q[p];
        if ((qp & kPtr) != p) {
          q[v] = (int32_t)((qp & kPtr) | ((qv ^ qp) & kPar));
          moved = 1;
        }
      }
      if (moved) sh.tail = 1;
      __syncthreads();
      if (sh.tail == 0) break;
    }
  }
  for (int32_t v = tid; v < n; v += NT) pw[v] = (uint64_t)((uint32_t)q[v] >> 31);
  __syncthreads();
}

// Tree t with the chosen sampler (paths 1 and 2 of the single-graph sweep);
// SMP is the family the kernel is built for (kSamplerRdfs also runs the
// hybrid, which takes BFS or randomized DFS per tree).
template <int NT, int SMP>
__device__ __forceinline__ void wg_tree_sampled(const DevGraph& G, const SweepArgs& A, uint64_t t,
                                                uint64_t* pw, int32_t* q, int32_t* d,
                                                WgShared<NT>& sh) {
  if constexpr (SMP == kSamplerBfs) {
    wg_tree<NT>(G, A, t, pw, q, sh);
  } else if constexpr (SMP == kSamplerKruskal) {
    wg_tree_kruskal<NT>(G, A, t, pw, q, d, sh);
    wg_finish<NT>(G, A, t, pw, sh);
  } else {
    if (A.sampler == kSamplerHybrid && !hybrid_coin(tree_salt(A.seed, t))) {
      wg_tree<NT>(G, A, t, pw, q, sh);
      return;
    }
    wg_tree_rdfs<NT>(G, A, t, pw, q, sh);
    wg_finish<NT>(G, A, t, pw, sh);
  }
}

}  // namespace wg
}  // namespace fi
