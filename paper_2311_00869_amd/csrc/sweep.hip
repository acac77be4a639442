// The graphBpp sweep (Alg. alg-index): per tree, a level-synchronous BFS with
// the min-key parent rule and fused state propagation, the exact frustration
// count, the canonical-state key, and the cloud insert.
//
// Two kernel families compute identical results:
//   k_sweep_wg   - one workgroup per tree; the tree words and the BFS queue
//                  live in LDS (small graphs) or in a per-workgroup slice of
//                  the workspace.  Trees are spread over workgroups, so one
//                  launch runs thousands of trees with no grid barrier.
//   k_sweep_grid - the whole grid per tree (persistent cooperative kernel):
//                  frontier work is handed out in units by a ticket counter
//                  (light chunks of vertices, and fixed-size edge ranges of
//                  high-degree vertices), levels are separated by a grid
//                  barrier.  For graphs far beyond one workgroup.
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

// ================================================================ whole grid per tree

constexpr int kHeavyUnit = 4096;  // edges per work unit of a high-degree vertex

template <int NT>
struct GridShared {
  int off[NT];
  int start[NT];
  uint64_t base[NT];
  int scan[NT / 64 + 1];
  uint64_t red[NT / 64];
  uint32_t unit;
  int2 heavy;
};

// Discovered vertex v goes to the light list, or (degree above `heavy`) to
// the heavy list with its first work-unit index.
__device__ __forceinline__ void append_next(bool found, int32_t v, const DevGraph& G,
                                            const SweepArgs& A, int32_t* ql, int2* qh,
                                            uint64_t* ring_next) {
  int dv = 0;
  if (found) dv = G.row_ptr[v + 1] - G.row_ptr[v];
  const bool heavy = found && dv > A.heavy;
  wave_append(found && !heavy, v, ql, (uint32_t*)ring_next);
  if (heavy) {
    const uint64_t units = (uint64_t)((dv + kHeavyUnit - 1) / kHeavyUnit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring_next + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// Expand frontier edges [e0, e1) of a single vertex whose next-level word
// (bit still to be xored with the edge sign) is `base`.
template <int NT>
__device__ __forceinline__ void expand_range(const DevGraph& G, const SweepArgs& A, int64_t e0,
                                             int64_t e1, uint64_t base, int32_t* ql, int2* qh,
                                             uint64_t* ring_next) {
  for (int64_t e = e0 + threadIdx.x; e - threadIdx.x < e1; e += NT) {
    bool found = false;
    int32_t v = 0;
    if (e < e1) {
      const uint32_t a = G.adj[e];
      v = (int32_t)(a & kVertexMask);
      const uint64_t nw = base ^ (uint64_t)(a >> 31);
      if (!((A.vis[v >> 6] >> (v & 63)) & 1) && A.pw[v] > nw)
        found = amin64(A.pw + v, nw) == kUnvisited;
    }
    append_next(found, v, G, A, ql, qh, ring_next);
  }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_sweep_grid(DevGraph G, SweepArgs A) {
  __shared__ GridShared<NT> sh;
  const int tid = threadIdx.x, lane = lane_id();
  const uint32_t nblocks = gridDim.x;
  const int64_t gtid = blockIdx.x * (int64_t)NT + tid;
  const int64_t gstride = (int64_t)nblocks * NT;
  const int64_t gwave = gtid >> 6, nwaves = gstride >> 6;
  const int32_t n = G.n;
  const int32_t* rp = G.row_ptr;
  uint64_t* ring = G.ctl + C_RING;
  uint64_t* acc = G.ctl + C_ACC;

  for (uint64_t t = A.t0; t < A.t1; ++t) {
    const KeyMix km = key_mix(tree_salt(A.seed, t));
    // ---- P0: reset, and per-component minimum keys
    for (int64_t v = gtid; v < n; v += gstride) A.pw[v] = kUnvisited;
    for (int64_t i = gtid; i < G.nwords; i += gstride) {
      A.vis[i] = 0;
      A.st[i] = 0;
    }
    if (blockIdx.x == 0 && tid < 8) ring[tid] = 0;
    {
      // contiguous word ranges per wave; one atomic per run of equal anchors
      const int64_t per = (G.nwords + nwaves - 1) / nwaves;
      const int64_t w0 = gwave * per, w1 = min<int64_t>(G.nwords, w0 + per);
      int32_t cur = -1;
      uint64_t cmin = kUnvisited;
      for (int64_t i = w0; i < w1; ++i) {
        const int32_t wc = G.word_comp[i];
        if (wc == -2) continue;
        const uint64_t wm = G.word_mask[i];
        const int32_t v = (int32_t)(i * 64 + lane);
        const bool has = (wm >> lane) & 1;
        const uint64_t key = has ? root_candidate(vhash20(km, v), v) : kUnvisited;
        if (wc >= 0) {
          const uint64_t mn = wave_min_u64(key);
          if (wc != cur) {
            if (cur >= 0 && lane == 0) amin64(A.rootkey + cur, cmin);
            cur = wc;
            cmin = mn;
          } else {
            cmin = mn < cmin ? mn : cmin;
          }
        } else if (has) {
          amin64(A.rootkey + G.comp[v], key);
        }
      }
      if (cur >= 0 && lane == 0) amin64(A.rootkey + cur, cmin);
    }
    grid_barrier(G.ctl, nblocks);

    // ---- P1: roots of the components with an edge form level 0
    for (int64_t c = gtid; c - tid < A.nanch; c += gstride) {
      bool ok = c < A.nanch;
      int32_t r = 0;
      if (ok) {
        const int32_t a = G.anchors[c];
        const uint64_t k = A.rootkey[a];
        A.rootkey[a] = kUnvisited;
        r = (int32_t)word_vertex(k);
        A.pw[r] = tree_word(0, vhash20(km, r), r, 0);
      }
      append_next(ok, r, G, A, A.ql[0], A.qh[0], ring);
    }
    grid_barrier(G.ctl, nblocks);

    // ---- P2: levels
    for (uint32_t L = 0;; ++L) {
      uint64_t* cur = ring + 4 * (L & 3);
      uint64_t* nxt = ring + 4 * ((L + 1) & 3);
      if (blockIdx.x == 0 && tid < 4) ring[4 * ((L + 2) & 3) + tid] = 0;
      const uint32_t nl = (uint32_t)load_agent(cur);
      const uint64_t hp = load_agent(cur + 1);
      const uint32_t nh = (uint32_t)(hp >> 32), hunits = (uint32_t)hp;
      if (nl == 0 && nh == 0) break;
      if (L + 1 > kMaxLevel) {
        if (gtid == 0) set_err(G, E_DEPTH);
        break;
      }
      const int32_t* ql_cur = A.ql[L & 1];
      const int2* qh_cur = A.qh[L & 1];
      int32_t* ql_nxt = A.ql[(L + 1) & 1];
      int2* qh_nxt = A.qh[(L + 1) & 1];
      const uint32_t nchunks = (nl + NT - 1) / NT;
      const uint32_t U = nchunks + hunits;
      while (true) {
        if (tid == 0) sh.unit = atomicAdd((uint32_t*)(cur + 2), 1u);
        __syncthreads();
        const uint32_t k = sh.unit;
        if (k >= U) break;
        if (k < nchunks) {
          // light chunk: NT frontier vertices, edges balanced by a block scan
          const uint32_t i = k * NT + tid;
          int d = 0, st = 0;
          uint64_t base = 0;
          if (i < nl) {
            const int32_t u = ql_cur[i];
            st = rp[u];
            d = rp[u + 1] - st;
            const uint32_t b = (uint32_t)(A.pw[u] & 1);
            base = tree_word(L + 1, vhash20(km, u), u, b);
            aor64(A.vis + (u >> 6), 1ull << (u & 63));
            if (b) aor64(A.st + (u >> 6), 1ull << (u & 63));
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
              const int kk = upper_index(sh.off, NT, j);
              const uint32_t a = G.adj[sh.start[kk] + (j - sh.off[kk])];
              v = (int32_t)(a & kVertexMask);
              const uint64_t nw = sh.base[kk] ^ (uint64_t)(a >> 31);
              if (!((A.vis[v >> 6] >> (v & 63)) & 1) && A.pw[v] > nw)
                found = amin64(A.pw + v, nw) == kUnvisited;
            }
            append_next(found, v, G, A, ql_nxt, qh_nxt, nxt);
          }
        } else {
          // heavy unit: kHeavyUnit edges of one high-degree vertex
          const uint32_t hk = k - nchunks;
          if (tid == 0) {
            int lo = 0, hi = (int)nh;
            while (hi - lo > 1) {
              int mid = (lo + hi) >> 1;
              if ((uint32_t)qh_cur[mid].y <= hk) lo = mid; else hi = mid;
            }
            sh.heavy = qh_cur[lo];
          }
          __syncthreads();
          const int32_t u = sh.heavy.x;
          const uint32_t part = hk - (uint32_t)sh.heavy.y;
          const uint32_t b = (uint32_t)(A.pw[u] & 1);
          if (part == 0 && tid == 0) {
            aor64(A.vis + (u >> 6), 1ull << (u & 63));
            if (b) aor64(A.st + (u >> 6), 1ull << (u & 63));
          }
          const int64_t e0 = rp[u] + (int64_t)part * kHeavyUnit;
          const int64_t e1 = min<int64_t>(rp[u + 1], e0 + kHeavyUnit);
          expand_range<NT>(G, A, e0, e1, tree_word(L + 1, vhash20(km, u), u, b), ql_nxt, qh_nxt,
                           nxt);
        }
        __syncthreads();
      }
      grid_barrier(G.ctl, nblocks);
    }

    // ---- P3: canonical words, key terms and the exact count
    uint64_t khi = 0, klo = 0, S = 0;
    for (int64_t i = gwave; i < G.nwords; i += nwaves) {
      uint64_t W = A.st[i];
      const int32_t wc = G.word_comp[i];
      if (wc >= 0) {
        if ((A.st[wc >> 6] >> (wc & 63)) & 1) W ^= G.word_mask[i];
      } else if (wc == -1) {
        const int64_t v = i * 64 + lane;
        uint32_t bit = (uint32_t)(W >> lane) & 1u;
        if (v < n && ((G.word_mask[i] >> lane) & 1)) {
          const int32_t a = G.comp[v];
          bit ^= (uint32_t)(A.st[a >> 6] >> (a & 63)) & 1u;
        }
        W = __ballot(bit);
      }
      if (lane == 0) {
        key_terms((uint64_t)i, W, khi, klo);
        if (A.bits_out) A.bits_out[i] = W;
      }
    }
    for (int64_t e = gtid; e < G.m; e += gstride) {
      const uint2 uv = G.edges[e];
      const uint32_t v = uv.y & kVertexMask;
      const uint32_t bu = (uint32_t)(A.st[uv.x >> 6] >> (uv.x & 63)) & 1u;
      const uint32_t bv = (uint32_t)(A.st[v >> 6] >> (v & 63)) & 1u;
      S += (uv.y >> 31) ^ bu ^ bv;
    }
    khi = block_sum_u64<NT>(khi, sh.red);
    klo = block_sum_u64<NT>(klo, sh.red);
    S = block_sum_u64<NT>(S, sh.red);
    if (tid == 0) {
      if (S) atomicAdd((unsigned long long*)acc, (unsigned long long)S);
      if (khi) atomicAdd((unsigned long long*)(acc + 1), (unsigned long long)khi);
      if (klo) atomicAdd((unsigned long long*)(acc + 2), (unsigned long long)klo);
    }
    grid_barrier(G.ctl, nblocks);

    // ---- P4: one thread inserts the tree
    if (gtid == 0) {
      const uint64_t s0 = load_agent(acc), h0 = load_agent(acc + 1), l0 = load_agent(acc + 2);
      acc[0] = 0;
      acc[1] = 0;
      acc[2] = 0;
      if (A.insert) cloud_insert(G, h0, l0, s0, t);
      if (A.tree_switches) A.tree_switches[t - A.t0] = s0;
    }
  }
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

template <int NT>
hipError_t launch_grid(fi_graph* g, const SweepArgs& a0, hipStream_t s) {
  SweepArgs a = a0;
  const Layout& L = g->L;
  a.pw = (uint64_t*)(g->ws + L.pw);
  a.ql[0] = (int32_t*)(g->ws + L.q0);
  a.ql[1] = (int32_t*)(g->ws + L.q1);
  a.qh[0] = (int2*)(g->ws + L.qh0);
  a.qh[1] = (int2*)(g->ws + L.qh1);
  a.vis = (uint64_t*)(g->ws + L.vis);
  a.st = (uint64_t*)(g->ws + L.st);
  a.rootkey = (uint64_t*)(g->ws + L.rootkey);
  a.heavy = g->sched.heavy;
  a.nanch = g->nanch;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_grid<NT>, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int maxg = per_cu * g->cu_count;
  int grid = g->sched.grid > 0 ? std::min(g->sched.grid, maxg) : std::min(maxg, 2 * g->cu_count);
  DevGraph G = g->dg;
  void* args[] = {(void*)&G, (void*)&a};
  e = hipLaunchCooperativeKernel((const void*)k_sweep_grid<NT>, dim3(grid), dim3(NT), args, 0, s);
  if (e != hipSuccess) return e;
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
    e = nt == 1024 ? launch_grid<1024>(g, a, s) : nt == 512 ? launch_grid<512>(g, a, s)
                                                             : launch_grid<256>(g, a, s);
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
