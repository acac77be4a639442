// The graphBpp sweep (Alg. alg-index): per tree, a level-synchronous BFS with
// the min-key parent rule and fused state propagation, the exact frustration
// count, the canonical-state key, and the cloud insert.
//
// Two kernel families compute identical results:
//   k_sweep_wg   - here: one workgroup per tree; the tree words and the BFS
//                  queue live in LDS (small graphs) or in a per-workgroup
//                  slice of the workspace.  Trees are spread over workgroups,
//                  so one launch runs thousands of trees with no grid barrier.
//   k_sweep_grid - sweep_grid.hip: the whole grid works on a few trees at a
//                  time (persistent cooperative kernel), for graphs far
//                  beyond one workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {

namespace {

__device__ __forceinline__ uint64_t amin64(uint64_t* p, uint64_t v) {
  return atomicMin((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void aor64(uint64_t* p, uint64_t v) {
  atomicOr((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void set_err(const DevGraph& G, uint64_t bit) {
  atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)bit);
}

// ================================================================ workgroup per tree

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
    if (rp[v + 1] > rp[v]) amin64(pw + G.comp[v], root_candidate(vhash20(km, v), v));
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
    pw[r] = tree_word(0, vhash20(km, r), r, 0);
  }
  for (int32_t v = tid; v < n; v += NT)
    if (rp[v + 1] == rp[v]) pw[v] = tree_word(0, vhash20(km, v), v, 0);
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
        base = tree_word(L + 1, vhash20(km, u), u, (uint32_t)(pw[u] & 1));
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

template <int NT, bool IN_LDS>
__global__ void __launch_bounds__(NT) k_sweep_wg(DevGraph G, SweepArgs A) {
  __shared__ WgShared<NT> sh;
  extern __shared__ uint64_t dyn[];
  uint64_t* pw;
  int32_t* q;
  if (IN_LDS) {
    pw = dyn;
    q = (int32_t*)(dyn + G.n);
  } else {
    char* slot = (char*)A.pw + (size_t)blockIdx.x * A.slot_stride;
    pw = (uint64_t*)slot;
    q = (int32_t*)(slot + 8 * (size_t)G.n);
  }
  for (uint64_t t = A.t0 + blockIdx.x; t < A.t1; t += gridDim.x) wg_tree<NT>(G, A, t, pw, q, sh);
}

size_t wg_lds_bytes(int32_t n) { return 12 * (size_t)n; }

template <int NT>
hipError_t launch_wg(fi_graph* g, const SweepArgs& a, int path, hipStream_t s) {
  const uint64_t ntrees = a.t1 - a.t0;
  const DevGraph& G = g->dg;
  int grid = g->sched.grid;
  if (path == 1) {
    const size_t lds = wg_lds_bytes(G.n);
    hipError_t ea = hipFuncSetAttribute((const void*)k_sweep_wg<NT, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_wg<NT, true>, NT, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    if (grid <= 0) grid = per_cu * g->cu_count;
    grid = (int)std::min<uint64_t>((uint64_t)grid, ntrees);
    hipLaunchKernelGGL((k_sweep_wg<NT, true>), dim3(grid), dim3(NT), lds, s, G, a);
  } else {
    SweepArgs b = a;
    b.pw = (uint64_t*)(g->ws + g->L.slots);
    b.slot_stride = g->L.slot_stride;
    if (grid <= 0) grid = 8 * g->cu_count;
    grid = (int)std::min<uint64_t>(std::min<uint64_t>((uint64_t)grid, ntrees), g->L.nslots);
    hipLaunchKernelGGL((k_sweep_wg<NT, false>), dim3(grid), dim3(NT), 0, s, G, b);
  }
  return hipGetLastError();
}

int pick_path(fi_graph* g) {
  if (g->sched.path != 0) return g->sched.path;
  const int32_t n = g->dg.n;
  if (wg_lds_bytes(n) + 32768 <= (size_t)g->max_shared) return 1;
  if (n <= 200000 && g->L.nslots > 0) return 2;
  return 3;
}

}  // namespace

hipError_t launch_sweep(fi_graph* g, const SweepArgs& a, hipStream_t s) {
  if (a.t1 <= a.t0) return hipSuccess;
  const int path = pick_path(g);
  const int nt = g->sched.block;
  void* tok = nullptr;
  if (prof_begin(g, s, &tok)) return hipErrorUnknown;
  hipError_t e;
  if (path == 3) {
    e = launch_grid(g, a, s);
  } else {
    e = nt == 1024 ? launch_wg<1024>(g, a, path, s) : nt == 512 ? launch_wg<512>(g, a, path, s)
                                                                 : launch_wg<256>(g, a, path, s);
  }
  prof_end(g, s, tok, 0);
  return e;
}

}  // namespace fi

using namespace fi;

extern "C" {

int fi_sweep_range(fi_graph* g, int64_t t0, int64_t t1, uint64_t seed, uint64_t* d_tree_switches,
                   void* stream) {
  if (!g || g->is_batch || t0 < 0 || t1 < t0) return FI_EINVAL;
  if (t1 > ((int64_t)1 << 32)) return FI_ERANGE;
  if (t1 == t0) return FI_OK;
  SweepArgs a{};
  a.seed = seed;
  a.t0 = (uint64_t)t0;
  a.t1 = (uint64_t)t1;
  a.tree_switches = d_tree_switches;
  a.bits_out = nullptr;
  a.insert = 1;
  return launch_sweep(g, a, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_sweep(fi_graph* g, int64_t K, uint64_t seed, void* stream) {
  return fi_sweep_range(g, 0, K, seed, nullptr, stream);
}

int fi_tree_state(fi_graph* g, uint64_t seed, int64_t t, uint64_t* d_bits_out,
                  uint64_t* d_switches_out, void* stream) {
  if (!g || g->is_batch || t < 0 || !d_bits_out) return FI_EINVAL;
  if (t >= ((int64_t)1 << 32)) return FI_ERANGE;
  SweepArgs a{};
  a.seed = seed;
  a.t0 = (uint64_t)t;
  a.t1 = (uint64_t)t + 1;
  a.tree_switches = d_switches_out;
  a.bits_out = d_bits_out;
  a.insert = 0;
  return launch_sweep(g, a, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
