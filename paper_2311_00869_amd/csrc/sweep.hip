// The graphBpp sweep (Alg. alg-index): per tree, a level-synchronous BFS with
// the min-key parent rule and fused state propagation, the exact frustration
// count, the canonical-state key, and the cloud insert.
//
// Three kernel families compute identical results:
//   k_sweep_wg   - here: one workgroup per tree; the tree words and the BFS
//                  queue live in LDS (small graphs) or in a per-workgroup
//                  slice of the workspace.  Trees are spread over workgroups,
//                  so one launch runs thousands of trees with no grid barrier.
//   k_sweep_grid - sweep_grid.hip: the whole grid works on a few trees at a
//                  time (persistent cooperative kernel), for graphs far
//                  beyond one workgroup.
//   k_sweep_multi - sweep_multi.hip: the whole grid sweeps 64 or 128 trees
//                  at once with one bit per tree in the fields of each
//                  vertex's record.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

#include "fi_wg.h"

namespace fi {

namespace {

using wg::WgShared;
using wg::wg_tree_sampled;

// SMP: the sampler family the kernel is built for (BFS, Kruskal, or the
// randomized DFS with the hybrid), so that each sampler's code is compiled
// and register-allocated on its own.
template <int NT, bool IN_LDS, int SMP>
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
  int32_t* d = q + G.n;  // Kruskal's hooks (its LDS and slots have room)
  for (uint64_t t = A.t0 + blockIdx.x; t < A.t1; t += gridDim.x)
    wg_tree_sampled<NT, SMP>(G, A, t, pw, q, d, sh);
}

// tree words and queue; Kruskal also keeps a hook per vertex
size_t wg_lds_bytes(int32_t n, int sampler = kSamplerBfs) {
  return (sampler == kSamplerKruskal ? 16 : 12) * (size_t)n;
}

template <int NT, int SMP>
hipError_t launch_wg_smp(fi_graph* g, const SweepArgs& a, int path, hipStream_t s) {
  const uint64_t ntrees = a.t1 - a.t0;
  const DevGraph& G = g->dg;
  int grid = g->sched.grid;
  if (path == 1) {
    const size_t lds = wg_lds_bytes(G.n, a.sampler);
    hipError_t ea = hipFuncSetAttribute((const void*)k_sweep_wg<NT, true, SMP>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_wg<NT, true, SMP>, NT, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    // at most six resident workgroups per CU: on a 1,000-vertex graph every
    // sampler ran a quarter slower at eight (the limit its registers allow)
    if (per_cu > 6) per_cu = 6;
    if (grid <= 0) grid = per_cu * g->cu_count;
    grid = (int)std::min<uint64_t>((uint64_t)grid, ntrees);
    hipLaunchKernelGGL((k_sweep_wg<NT, true, SMP>), dim3(grid), dim3(NT), lds, s, G, a);
  } else {
    SweepArgs b = a;
    b.pw = (uint64_t*)(g->ws + g->L.slots);
    b.slot_stride = g->L.slot_stride;
    if (grid <= 0) grid = 8 * g->cu_count;
    grid = (int)std::min<uint64_t>(std::min<uint64_t>((uint64_t)grid, ntrees), g->L.nslots);
    hipLaunchKernelGGL((k_sweep_wg<NT, false, SMP>), dim3(grid), dim3(NT), 0, s, G, b);
  }
  return hipGetLastError();
}

template <int NT>
hipError_t launch_wg(fi_graph* g, const SweepArgs& a, int path, hipStream_t s) {
  if (a.sampler == kSamplerKruskal) return launch_wg_smp<NT, kSamplerKruskal>(g, a, path, s);
  if (a.sampler == kSamplerRdfs || a.sampler == kSamplerHybrid)
    return launch_wg_smp<NT, kSamplerRdfs>(g, a, path, s);
  return launch_wg_smp<NT, kSamplerBfs>(g, a, path, s);
}

int pick_path(fi_graph* g) {
  const int32_t n = g->dg.n;
  const bool fits = wg_lds_bytes(n, g->sampler) + 32768 <= (size_t)g->max_shared;
  if (g->sampler != kSamplerBfs) {
    // the other samplers run one tree per workgroup only
    if (g->sched.path == 1 && fits) return 1;
    if (g->sched.path == 2 && g->L.nslots > 0) return 2;
    if (fits) return 1;
    return g->L.nslots > 0 ? 2 : 0;
  }
  if (g->sched.path != 0) return g->sched.path;
  if (fits) return 1;
  // one tree per workgroup costs about m per tree, while 128 trees per pass
  // (on a grid sized to the graph) cost about their BFS depth: past n + m/2 of
  // about 135,000 the pass wins (measured at average degrees 4, 10 and 16)
  if ((int64_t)n + g->dg.m / 2 <= 135000 && g->L.nslots > 0) return 2;
  return 5;
}

// threads per workgroup of the automatic schedule's one-tree-per-workgroup
// paths (measured up to 3 times apart).  Path 2: 256 for sparse graphs
// (average degree up to 10), else 1,024.  Path 1: the tree's LDS bounds the
// workgroups a CU holds, so the fewer fit, the wider each one (BFS and
// Kruskal; the randomized DFS keeps most waves idle and takes 256).
int auto_block(fi_graph* g, int path) {
  if (path == 2) return g->dg.m <= 5 * (int64_t)g->dg.n ? 256 : 1024;
  if (path != 1 || g->sampler == kSamplerRdfs || g->sampler == kSamplerHybrid) return 256;
  const size_t lds = wg_lds_bytes(g->dg.n, g->sampler);
  return lds <= 24576 ? 256 : lds <= 65536 ? 512 : 1024;
}

}  // namespace

hipError_t launch_sweep(fi_graph* g, const SweepArgs& a, hipStream_t s) {
  if (a.t1 <= a.t0) return hipSuccess;
  int path = pick_path(g);
  if (path == 0) return hipErrorInvalidValue;  // a sampler other than BFS above 1M vertices
  // the multi-tree path keeps no per-tree state words to hand out; it alone
  // gathers the cloud statistics
  if ((path == 4 || path == 5) && a.bits_out) path = 3;
  if (a.vminus || a.eswitch) path = path == 5 ? 5 : 4;  // (BFS only: checked by the caller)
  const int nt = g->sched.path == 0 ? auto_block(g, path) : g->sched.block;
  void* tok = nullptr;
  if (prof_begin(g, s, &tok)) return hipErrorUnknown;
  hipError_t e;
  if (path == 4 || path == 5) {
    e = launch_multi(g, a, path == 5 ? 2 : 1, s);
  } else if (path == 3) {
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

namespace {
SweepArgs base_args(fi_graph* g, uint64_t seed) {
  SweepArgs a{};
  a.seed = seed;
  a.sampler = g->sampler;
  a.cptr = (const int32_t*)(g->ws + g->L.cptr);
  return a;
}
}  // namespace

extern "C" {

int fi_sweep_range(fi_graph* g, int64_t t0, int64_t t1, uint64_t seed, uint64_t* d_tree_switches,
                   void* stream) {
  if (!g || g->is_batch || t0 < 0 || t1 < t0) return FI_EINVAL;
  if (t1 > ((int64_t)1 << 32)) return FI_ERANGE;
  if (t1 == t0) return FI_OK;
  SweepArgs a = base_args(g, seed);
  a.t0 = (uint64_t)t0;
  a.t1 = (uint64_t)t1;
  a.tree_switches = d_tree_switches;
  a.bits_out = nullptr;
  a.insert = 1;
  return launch_sweep(g, a, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_sweep_stats(fi_graph* g, int64_t t0, int64_t t1, uint64_t seed, uint64_t* d_vertex_minus,
                   uint64_t* d_edge_switched, void* stream) {
  if (!g || g->is_batch || t0 < 0 || t1 < t0 || (!d_vertex_minus && !d_edge_switched) ||
      g->sampler != kSamplerBfs)
    return FI_EINVAL;
  if (t1 > ((int64_t)1 << 32)) return FI_ERANGE;
  if (t1 == t0) return FI_OK;
  SweepArgs a = base_args(g, seed);
  a.t0 = (uint64_t)t0;
  a.t1 = (uint64_t)t1;
  a.insert = 1;
  a.vminus = d_vertex_minus;
  a.eswitch = d_edge_switched;
  return launch_sweep(g, a, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_set_sampler(fi_graph* g, int32_t sampler) {
  if (!g || g->is_batch || sampler < kSamplerBfs || sampler > kSamplerKruskal) return FI_EINVAL;
  if (sampler != kSamplerBfs && g->L.nslots == 0) {
    // one tree per workgroup needs the tree in LDS or in a workspace slot
    const size_t lds = (sampler == kSamplerKruskal ? 16 : 12) * (size_t)g->dg.n;
    if (lds + 32768 > (size_t)g->max_shared) return FI_ERANGE;
  }
  g->sampler = sampler;
  return FI_OK;
}

int fi_get_sampler(fi_graph* g, int32_t* out) {
  if (!g || g->is_batch || !out) return FI_EINVAL;
  *out = g->sampler;
  return FI_OK;
}

int fi_sweep(fi_graph* g, int64_t K, uint64_t seed, void* stream) {
  return fi_sweep_range(g, 0, K, seed, nullptr, stream);
}

int fi_tree_state(fi_graph* g, uint64_t seed, int64_t t, uint64_t* d_bits_out,
                  uint64_t* d_switches_out, void* stream) {
  if (!g || g->is_batch || t < 0 || !d_bits_out) return FI_EINVAL;
  if (t >= ((int64_t)1 << 32)) return FI_ERANGE;
  SweepArgs a = base_args(g, seed);
  a.t0 = (uint64_t)t;
  a.t1 = (uint64_t)t + 1;
  a.tree_switches = d_switches_out;
  a.bits_out = d_bits_out;
  a.insert = 0;
  return launch_sweep(g, a, (hipStream_t)stream) == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
