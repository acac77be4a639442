// Many independent graphs of uneven size swept together (Alg. alg-index per
// graph).  The graphs are validated, packed and split into components in one
// pass each over the concatenated arrays (every element finds its graph by a
// binary search over the offsets); each keeps its own vertex ids, its own
// small cloud and its own minimum.  Sweeping hands out work items
// (graph, tree), largest graph first, to persistent workgroups that each run
// one whole tree (the same routine as the single-graph sweep): graphs small
// enough keep their tree state in LDS, the others in a workspace slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "fi_internal.h"
#include "fi_prims.h"
#include "fi_wg.h"
#include "fi_multi.h"

namespace fi {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kCtlPerGraph = 32;       // err, best, distinct count, trees; own 256-byte line
constexpr int32_t kMaxBatchN = 1000000;
constexpr int kLdsMaxN = 6144;         // graphs up to this size keep their tree in LDS
// item tickets of the two size classes, each on its own 128-byte line of the
// batch control block
constexpr int kTicket0 = C_UNIT;
constexpr int kTicket1 = C_UNIT + 16;

inline int grid_for(int64_t work, int block, int cap = 65536) {
  int64_t g = (work + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

struct BatchGraph {
  int32_t n, nwords;
  int64_t nnz, m;
  int64_t vo, no, me, ro;  // first vertex, CSR entry, edge, row_ptr slot
  int32_t ncomp, cs;       // components with an edge; first one's slot among all graphs'
};

constexpr int kRootRows = 64;  // components whose roots one pass of the multi-tree sweep finds

struct BatchLayout {
  size_t meta, offs, row_ptr, adj, edges, comp, ustart, eoff, tiles, gctl, clouds, ctl, small, large,
      slots;
  size_t slot_stride, nslots;
  // multi-tree sweep: component index per vertex, graphs largest first, and
  // per-workgroup slices (four words per vertex, an unfinished bitmap, root
  // minima of kRootRows components)
  size_t cidx, order, mslots, mslot_stride, nmslots;
  size_t total;
};

struct BatchInfo {
  int32_t G;
  int64_t n_total, nnz_total, m_total;
  int64_t cap;
  uint64_t tsize;
  int32_t n_max_small, n_max_large;
  int32_t n_small, n_large;
  int per_cu[3][2];  // [block 256/512/1024][in LDS, in workspace]
  int mt_per_cu[3];  // multi-tree sweep, per block size
  int32_t n_max;
  BatchLayout L;
};

BatchLayout batch_layout(int32_t G, int64_t n_total, int64_t nnz_total, int32_t n_max_large,
                         int32_t n_max, uint64_t tsize) {
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t g = (size_t)G, n = (size_t)n_total, nnz = (size_t)nnz_total, m = nnz / 2;
  L.meta = take(sizeof(BatchGraph) * g);
  L.offs = take(8 * 4 * (g + 1));  // vo, no, me, ro
  L.row_ptr = take(4 * (n + g));
  L.adj = take(4 * nnz);
  L.edges = take(8 * m);
  L.comp = take(4 * n);
  L.ustart = take(4 * (n + 64));
  L.eoff = take(4 * (n + 64));
  L.tiles = take(4 * (n / 1024 + 2));
  L.gctl = take(8 * kCtlPerGraph * g);
  L.clouds = take(sizeof(CloudSlot) * tsize * g);
  L.ctl = take(8 * C_WORDS);
  L.small = take(4 * g);
  L.large = take(4 * g);
  L.slot_stride = align_up(12 * (size_t)std::max(n_max_large, 1));
  L.nslots = n_max_large > 0
                 ? std::min<size_t>(2048, std::max<size_t>(64, ((size_t)8 << 30) / L.slot_stride))
                 : 0;
  L.slots = take(L.slot_stride * L.nslots);
  L.cidx = take(4 * n);
  L.order = take(4 * g);
  const size_t nm = (size_t)std::max(n_max, 1);
  L.mslot_stride = align_up(32 * nm + 8 * (nm / 64 + 2) + 8 * 64 * (size_t)kRootRows);
  L.nmslots = std::min<size_t>(2048, std::max<size_t>(64, ((size_t)8 << 30) / L.mslot_stride));
  L.mslots = take(L.mslot_stride * L.nmslots);
  L.total = off;
  return L;
}

// Largest i in [0, len) with off[i] <= x.
__device__ __forceinline__ int32_t which(const int64_t* off, int32_t len, int64_t x) {
  int32_t lo = 0, hi = len;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int32_t row_in(const int32_t* rp, int32_t n, int64_t e) {
  int32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)rp[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// row_ptr entries: starts at 0, ends at the graph's nnz, never decreases
__global__ void k_b_rowptr(const int32_t* rp, const BatchGraph* meta, const int64_t* ro, int32_t G,
                           int64_t total, uint64_t* ctl) {
  bool bad = false;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(ro, G, r);
    const BatchGraph b = meta[g];
    const int64_t local = r - b.ro;
    const int32_t x = rp[r];
    if (local == 0 && x != 0) bad = true;
    if (local == b.n && (int64_t)x != b.nnz) bad = true;
    if (local > 0 && x < rp[r - 1]) bad = true;
  }
  if (bad) atomicOr((unsigned long long*)(ctl + C_FLAGS), (unsigned long long)V_ROWPTR);
}

__global__ void k_b_entries(const int32_t* rp, const int32_t* col, const int8_t* sign,
                            const BatchGraph* meta, const int64_t* no, int32_t G, int64_t total,
                            uint64_t* ctl) {
  uint32_t f = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(no, G, e);
    const BatchGraph b = meta[g];
    const int32_t* rpg = rp + b.ro;
    const int32_t* cg = col + b.no;
    const int8_t* sg = sign + b.no;
    const int64_t le = e - b.no;
    const int32_t u = row_in(rpg, b.n, le);
    const int32_t v = cg[le];
    const int s = sg[le];
    if (v < 0 || v >= b.n) { f |= V_RANGE; continue; }
    if (s != 1 && s != -1) f |= V_SIGN;
    if (v == u) f |= V_SELF;
    if (le + 1 < (int64_t)rpg[u + 1]) {
      const int32_t c2 = cg[le + 1];
      if (c2 == v) f |= V_DUP;
      else if (c2 < v) f |= V_UNSORTED;
    }
    int64_t lo = rpg[v], hi = rpg[v + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (cg[mid] < u) lo = mid + 1; else hi = mid;
    }
    if (lo >= rpg[v + 1] || cg[lo] != u || sg[lo] != s) f |= V_ASYM;
  }
  if (f) atomicOr((unsigned long long*)(ctl + C_FLAGS), (unsigned long long)f);
}

// per vertex: first entry above the diagonal (global entry index) and count
__global__ void k_b_upper(const int32_t* rp, const int32_t* col, const BatchGraph* meta,
                          const int64_t* vo, int32_t G, int64_t n_total, int32_t* ustart,
                          int32_t* ucnt) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n_total;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(vo, G, v);
    const BatchGraph b = meta[g];
    const int32_t u = (int32_t)(v - b.vo);
    const int32_t* rpg = rp + b.ro;
    const int32_t* cg = col + b.no;
    int32_t lo = rpg[u], hi = rpg[u + 1];
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      if (cg[mid] <= u) lo = mid + 1; else hi = mid;
    }
    ustart[v] = (int32_t)(b.no + lo);
    ucnt[v] = rpg[u + 1] - lo;
  }
}

__global__ void k_b_pack(const int32_t* rp, const int32_t* col, const int8_t* sign,
                         const BatchGraph* meta, const int64_t* no, int32_t G, int64_t total,
                         const int32_t* ustart, const int32_t* eoff, uint32_t* adj, uint2* edges,
                         int32_t* rp_out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(no, G, e);
    const BatchGraph b = meta[g];
    const int32_t* rpg = rp + b.ro;
    const int64_t le = e - b.no;
    const int32_t u = row_in(rpg, b.n, le);
    const uint32_t v = (uint32_t)col[e];
    const uint32_t a = v | ((sign[e] < 0 ? 1u : 0u) << 31);
    adj[e] = a;
    if ((int32_t)v > u) {
      const int64_t gv = b.vo + u;
      edges[eoff[gv] + (e - ustart[gv])] = make_uint2((uint32_t)u, a);
    }
  }
  (void)rp_out;
}

__global__ void k_b_copy_rp(const int32_t* rp, int32_t* out, int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = rp[i];
}

// Union-find over global vertex ids (graph offset + local id); graphs are
// disjoint, so every component lies inside one graph.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t p = load_agent_i32(parent + x);
  while (p != x) {
    x = p;
    p = load_agent_i32(parent + x);
  }
  return x;
}

__global__ void k_b_uf_init(int32_t* parent, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = (int32_t)v;
}

__global__ void k_b_uf_hook(const uint2* edges, const BatchGraph* meta, const int64_t* me, int32_t G,
                            int64_t m_total, int32_t* parent) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m_total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(me, G, e);
    const int64_t base = meta[g].vo;
    const int32_t u = (int32_t)(base + edges[e].x);
    const int32_t v = (int32_t)(base + (edges[e].y & kVertexMask));
    while (true) {
      const int32_t ru = uf_find(parent, u), rv = uf_find(parent, v);
      if (ru == rv) break;
      const int32_t lo = min(ru, rv), hi = max(ru, rv);
      if (atomicCAS(parent + hi, hi, lo) == hi) break;
    }
  }
}

// final: graph-local anchor (smallest local id of the component)
__global__ void k_b_uf_local(int32_t* parent, const BatchGraph* meta, const int64_t* vo, int32_t G,
                             int64_t n, int32_t* comp) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(vo, G, v);
    comp[v] = uf_find(parent, (int32_t)v) - (int32_t)meta[g].vo;
  }
}

__global__ void k_b_reset(CloudSlot* clouds, int64_t nslots, uint64_t* gctl, int32_t G,
                          uint64_t* ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nslots;
       i += (int64_t)gridDim.x * blockDim.x) {
    CloudSlot s;
    s.tag = kEmpty;
    s.khi_min = ~0ull; s.khi_max = 0;
    s.s_min = ~0ull; s.s_max = 0;
    s.freq = 0; s.first = ~0ull; s.pad = 0;
    clouds[i] = s;
  }
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G;
       g += (int64_t)gridDim.x * blockDim.x) {
    uint64_t* c = gctl + g * kCtlPerGraph;
    c[C_ERR] = 0;
    c[C_BEST] = ~0ull;
    c[C_COUNT] = 0;
    c[C_TREES] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[C_ERR] = 0;
    ctl[kTicket0] = 0;
    ctl[kTicket1] = 0;
  }
}

__global__ void k_b_finish(const uint64_t* gctl, int32_t G, uint64_t* min_out, uint64_t* distinct,
                           uint64_t* ctl) {
  uint64_t err = 0;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t* c = gctl + g * kCtlPerGraph;
    const uint64_t best = c[C_BEST];
    min_out[2 * g] = best >> 32;
    min_out[2 * g + 1] = best & 0xFFFFFFFFull;
    if (distinct) distinct[g] = c[C_COUNT];
    err |= c[C_ERR];
  }
  if (err) atomicOr((unsigned long long*)(ctl + C_ERR), (unsigned long long)err);
}

struct BatchArgs {
  const BatchGraph* meta;
  const int32_t* row_ptr;
  const uint32_t* adj;
  const uint2* edges;
  const int32_t* comp;
  CloudSlot* clouds;
  uint64_t* gctl;
  uint64_t* ticket;     // next work item of this size class
  const int32_t* order; // graph ids of this size class, largest first
  int64_t nitems;       // graphs in the class * trees per graph
  int64_t trees;
  uint64_t seed;
  uint64_t tsize;
  uint64_t cap;
  char* slots;
  size_t slot_stride;
};

template <int NT, bool IN_LDS>
__global__ void __launch_bounds__(NT) k_batch_wg(BatchArgs B) {
  __shared__ wg::WgShared<NT> sh;
  __shared__ int64_t s_item;
  extern __shared__ uint64_t dyn[];
  while (true) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long*)B.ticket, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= B.nitems) break;
    const int32_t gi = B.order[item / B.trees];
    const uint64_t t = (uint64_t)(item % B.trees);
    const BatchGraph b = B.meta[gi];
    DevGraph G{};
    G.n = b.n;
    G.nwords = b.nwords;
    G.nnz = b.nnz;
    G.m = b.m;
    G.row_ptr = B.row_ptr + b.ro;
    G.adj = B.adj + b.no;
    G.edges = B.edges + b.me;
    G.comp = B.comp + b.vo;
    G.cloud = B.clouds + (size_t)gi * B.tsize;
    G.cloud_mask = B.tsize - 1;
    G.cloud_cap = B.cap;
    G.ctl = B.gctl + (size_t)gi * kCtlPerGraph;
    SweepArgs A{};
    A.seed = B.seed;
    A.t0 = 0;
    A.t1 = (uint64_t)B.trees;
    A.insert = 1;
    uint64_t* pw;
    int32_t* q;
    if (IN_LDS) {
      pw = dyn;
      q = (int32_t*)(dyn + b.n);
    } else {
      char* slot = B.slots + (size_t)blockIdx.x * B.slot_stride;
      pw = (uint64_t*)slot;
      q = (int32_t*)(slot + 8 * (size_t)b.n);
    }
    wg::wg_tree<NT>(G, A, t, pw, q, sh);
  }
}

inline int nt_index(int nt) { return nt == 1024 ? 2 : nt == 512 ? 1 : 0; }

// Done once at create, so a sweep only launches kernels: the LDS size of the
// in-LDS class and the resident workgroups per CU of both classes.
template <int NT>
hipError_t batch_occupancy(BatchInfo* bi) {
  const int k = nt_index(NT);
  const size_t bytes = 12 * (size_t)bi->n_max_small;
  hipError_t e = hipFuncSetAttribute((const void*)k_batch_wg<NT, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bi->per_cu[k][0], k_batch_wg<NT, true>, NT, bytes);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&bi->per_cu[k][1], k_batch_wg<NT, false>, NT, 0);
}

template <int NT>
void launch_class(fi_graph* h, const BatchArgs& a, bool lds, hipStream_t s) {
  const BatchInfo* bi = (const BatchInfo*)h->batch;
  int64_t grid = (int64_t)std::max(1, bi->per_cu[nt_index(NT)][lds ? 0 : 1]) * h->cu_count;
  if (h->sched.grid > 0) grid = std::min<int64_t>(grid, h->sched.grid);
  if (!lds) grid = std::min<int64_t>(grid, (int64_t)bi->L.nslots);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, a.nitems));
  if (lds)
    hipLaunchKernelGGL((k_batch_wg<NT, true>), dim3((int)grid), dim3(NT), 12 * (size_t)bi->n_max_small,
                       s, a);
  else
    hipLaunchKernelGGL((k_batch_wg<NT, false>), dim3((int)grid), dim3(NT), 0, s, a);
}


// Anchors (each component's smallest vertex with an edge), global ids.
__global__ void k_b_anchors(const int32_t* rp, const BatchGraph* meta, const int64_t* vo, int32_t G,
                            int64_t n_total, const int32_t* comp, int32_t* list, uint32_t* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n_total; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    bool is = false;
    if (v < n_total) {
      const int32_t g = which(vo, G, v);
      const BatchGraph b = meta[g];
      const int32_t u = (int32_t)(v - b.vo);
      is = rp[b.ro + u + 1] > rp[b.ro + u] && comp[v] == u;
    }
    wave_append(is, (int32_t)v, list, count);
  }
}

__global__ void k_b_cidx_none(int32_t* cidx, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    cidx[v] = -1;
}

__global__ void k_b_scatter_slot(const int32_t* anchors, int64_t count, int32_t* slot) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    slot[anchors[i]] = (int32_t)i;
}

// Component index of every vertex within its graph (-1 without an edge).
__global__ void k_b_cidx(const int32_t* rp, const BatchGraph* meta, const int64_t* vo, int32_t G,
                         int64_t n_total, const int32_t* comp, const int32_t* slot, int32_t* cidx) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n_total;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = which(vo, G, v);
    const BatchGraph b = meta[g];
    const int32_t u = (int32_t)(v - b.vo);
    cidx[v] = rp[b.ro + u + 1] > rp[b.ro + u] ? slot[b.vo + comp[v]] - b.cs : -1;
  }
}

// The root-minima tables of every slice start at "none".
__global__ void k_b_mt_tables(char* slots, size_t stride, size_t nslots, size_t table_off) {
  const int64_t per = 64 * kRootRows;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)nslots * per;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t* t = (uint64_t*)(slots + (size_t)(i / per) * stride + table_off);
    t[i % per] = kUnvisited;
  }
}

struct BatchMArgs {
  const BatchGraph* meta;
  const int32_t* row_ptr;
  const uint32_t* adj;
  const uint2* edges;
  const int32_t* comp;
  const int32_t* cidx;
  CloudSlot* clouds;
  uint64_t* gctl;
  const int32_t* order;  // all graphs, largest first
  uint64_t* ticket;
  int32_t G, groups;      // graphs; groups of 64 trees per graph
  int64_t trees;
  uint64_t seed;
  uint64_t tsize, cap;
  char* slots;
  size_t slot_stride;
  int32_t n_max;
};

// Multi-tree sweep of a batch: one workgroup per (graph, group of up to 64
// trees), largest graph first, drawn by persistent workgroups.  Within a
// workgroup the levels are pulls over every vertex not yet visited by all
// trees (rows of up to 64 edges: the wave pulls the unfinished vertices of
// one 64-vertex word; longer rows: one per wave), separated by workgroup
// barriers.
template <int NT>
__global__ void __launch_bounds__(NT) k_batch_multi(BatchMArgs B) {
  constexpr int NW = NT / 64;
  constexpr int kPlanes = 8;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  __shared__ int64_t s_item;
  __shared__ int s_any[2];  // some vertex reached, by level parity
  __shared__ uint64_t s_acc[3][64];
  __shared__ mt::TW<1> s_pw[NW][4 * 64];  // per wave: short rows' wanted trees and outcomes, edge states
  __shared__ uint64_t s_pe[NW][65];       // per wave: where the short rows' edges start a row
  char* slot = B.slots + (size_t)blockIdx.x * B.slot_stride;
  const size_t nm = (size_t)B.n_max;
  // vertex records of one word per field, then the unfinished-vertex bitmap
  mt::MState S;
  S.nbw[0] = (uint64_t*)slot;
  S.stw = S.nbw[0] + 1;
  S.nbw[1] = S.nbw[0] + 2;
  S.vis = S.nbw[0] + 3;
  S.unf = S.nbw[0] + mt::kRecFields * nm;
  S.cand = nullptr;
  S.stc = nullptr;
  uint64_t* table = S.unf + (nm / 64 + 2);
  const int64_t nitems = (int64_t)B.G * B.groups;

  while (true) {
    if (tid == 0) s_item = (int64_t)atomicAdd((unsigned long long*)B.ticket, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= nitems) break;
    const int32_t gi = B.order[item / B.groups];
    const int64_t tb = (item % B.groups) * 64;
    const BatchGraph b = B.meta[gi];
    DevGraph G{};
    G.n = b.n;
    G.nwords = b.nwords;
    G.nnz = b.nnz;
    G.m = b.m;
    G.row_ptr = B.row_ptr + b.ro;
    G.adj = B.adj + b.no;
    G.edges = B.edges + b.me;
    G.comp = B.comp + b.vo;
    G.cloud = B.clouds + (size_t)gi * B.tsize;
    G.cloud_mask = B.tsize - 1;
    G.cloud_cap = B.cap;
    G.ctl = B.gctl + (size_t)gi * kCtlPerGraph;
    const int32_t n = b.n, nw = b.nwords;
    const int32_t* rp = G.row_ptr;
    const int32_t* cix = B.cidx + b.vo;
    const int nvalid = (int)min<int64_t>(64, B.trees - tb);
    const uint64_t valid = nvalid == 64 ? ~0ull : ((1ull << nvalid) - 1);
    const bool vlane = lane < nvalid;
    const KeyMix km = key_mix(tree_salt(B.seed, (uint64_t)(tb + lane)));

    // ---- reset
    for (int32_t v = tid; v < mt::kRecFields * n; v += NT) S.nbw[0][v] = 0;
    for (int32_t w = wave; w < nw; w += NW) {
      const int32_t v = w * 64 + lane;
      const uint64_t m = __ballot(v < n && rp[v + 1] > rp[v]);
      if (lane == 0) S.unf[w] = m;
    }
    __syncthreads();

    // ---- roots, kRootRows components per pass: each wave scans a range of
    // vertices keeping per-lane minima by component, then one wave per
    // component writes its roots
    for (int32_t r0 = 0; r0 < b.ncomp; r0 += kRootRows) {
      const int32_t rows = min(kRootRows, b.ncomp - r0);
      const int32_t chunk = (n + NW - 1) / NW;
      const int32_t v0 = wave * chunk, v1 = min(n, v0 + chunk);
      int32_t cur = -1;
      uint64_t best = kUnvisited;
      for (int32_t c = v0; c < v1; c += 64) {
        const int32_t vv = c + lane;
        const int32_t ci = vv < v1 ? cix[vv] : -1;
        const uint32_t hm = fmix32((uint32_t)vv);
        const int cnt = min(64, v1 - c);
        for (int j = 0; j < cnt; ++j) {
          const int32_t cj = __builtin_amdgcn_readlane(ci, j);
          if (cj < r0 || cj >= r0 + rows) continue;
          if (cj != cur) {
            if (cur >= 0 && vlane && best != kUnvisited)
              mt::amin64(table + (size_t)(cur - r0) * 64 + lane, best);
            cur = cj;
            best = kUnvisited;
          }
          const uint64_t k = root_candidate(vkey_of(km, (uint32_t)__builtin_amdgcn_readlane((int)hm, j)),
                                            (uint32_t)(c + j));
          best = k < best ? k : best;
        }
      }
      if (cur >= 0 && vlane && best != kUnvisited)
        mt::amin64(table + (size_t)(cur - r0) * 64 + lane, best);
      __syncthreads();
      for (int32_t row = wave; row < rows; row += NW) {
        uint64_t* tr = table + (size_t)row * 64;
        const uint64_t bk = vlane ? tr[lane] : kUnvisited;
        if (vlane) tr[lane] = kUnvisited;
        const bool ok = vlane && bk != kUnvisited;
        const uint32_t r = (uint32_t)word_vertex(bk);
        uint64_t rem = __ballot(ok);
        while (rem) {
          const int j = __builtin_ctzll(rem);
          const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)r, j);
          const uint64_t msk = __ballot(ok && r == r1);
          rem &= ~msk;
          if (lane == 0) {
            mt::stw_<1>(S.nbw[0], r1, mt::TW<1>{{msk}});
            mt::stw_<1>(S.vis, r1, mt::TW<1>{{msk}});
            if (msk == valid) mt::aand64(S.unf + (r1 >> 6), ~(1ull << (r1 & 63)));
          }
        }
      }
      __syncthreads();
    }

    // ---- levels
    if (tid == 0) {
      s_any[0] = 0;
      s_any[1] = 0;
    }
    for (uint32_t L = 1;; ++L) {
      const int pp = (int)((L - 1) & 1), p = (int)(L & 1);
      __syncthreads();
      // the other parity's flag was last read before the barrier above
      if (tid == 0) s_any[pp] = 0;
      uint64_t cnt = 0, deg = 0, fin = 0;
      for (int32_t w = wave; w < nw; w += NW) {
        const uint64_t bits = S.unf[w];
        if (!bits) continue;
        const int32_t v = w * 64 + lane;
        const int d = ((bits >> lane) & 1) ? rp[v + 1] - rp[v] : 0;
        const uint64_t small = __ballot(((bits >> lane) & 1) && d <= 64);
        const int ne = (int)__popcll(small);
        if (ne) {
          const int src = mt::select_lane(small, lane < ne ? lane : 0);
          const int32_t vk = __shfl(v, src);
          mt::pull_small_w<1, 64>(G, S, vk, ne, pp, p, mt::TW<1>{{valid}}, &km, false, s_pw[wave],
                                  s_pe[wave], cnt, deg, fin);
        }
        uint64_t big = bits & ~small;
        while (big) {
          const int j = __builtin_ctzll(big);
          big &= big - 1;
          const int32_t vj = w * 64 + j;
          const mt::TW<1> want = mt::uni_w(mt::and_not(mt::TW<1>{{valid}}, mt::ldw<1>(S.vis, vj)));
          uint64_t best = kUnvisited;
          if (want.w[0]) mt::pull_edges_w<1>(G.adj, S.nbw[pp], S.stw, rp[vj], rp[vj + 1], want, &km, &best);
          mt::settle_w<1>(S, vj, mt::ldw<1>(S.vis, vj), mt::ldw<1>(S.stw, vj), rp[vj + 1] - rp[vj], &best,
                          p, mt::TW<1>{{valid}}, cnt, deg, fin);
        }
      }
      if (lane == 0 && cnt) s_any[p] = 1;
      __syncthreads();
      if (!s_any[p]) break;
    }

    // ---- counts and canonical keys of the trees of the item
    if (tid < 192) (&s_acc[0][0])[tid] = 0;
    __syncthreads();
    {
      uint64_t c[kPlanes];
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) c[q] = 0;
      uint64_t myS = 0;
      int it = 0;
      auto flush = [&]() {
        for (int t = 0; t < 64; ++t) {
          uint32_t tot = 0;
#pragma unroll
          for (int q = 0; q < kPlanes; ++q) tot += (uint32_t)__popcll(__ballot((c[q] >> t) & 1)) << q;
          if (lane == t) myS += tot;
        }
#pragma unroll
        for (int q = 0; q < kPlanes; ++q) c[q] = 0;
      };
      for (int64_t e0 = 0; e0 < G.m; e0 += NT) {
        const int64_t e = e0 + tid;
        uint64_t x = 0;
        if (e < G.m) {
          const uint2 uv = G.edges[e];
          x = mt::ldw<1>(S.stw, uv.x).w[0] ^ mt::ldw<1>(S.stw, uv.y & kVertexMask).w[0];
          if (uv.y >> 31) x = ~x;
        }
#pragma unroll
        for (int q = 0; q < kPlanes; ++q) {
          const uint64_t carry = c[q] & x;
          c[q] ^= x;
          x = carry;
        }
        if (++it == 255) {
          flush();
          it = 0;
        }
      }
      flush();
      uint64_t khi = 0, klo = 0;
      for (int32_t i = wave; i < nw; i += NW) {
        const int32_t v = i * 64 + lane;
        uint64_t cs = 0;
        if (v < n) cs = mt::ldw<1>(S.stw, v).w[0] ^ mt::ldw<1>(S.stw, G.comp[v]).w[0];
        key_terms((uint64_t)i, mt::transpose64(cs), khi, klo);
      }
      atomicAdd((unsigned long long*)&s_acc[0][lane], (unsigned long long)myS);
      atomicAdd((unsigned long long*)&s_acc[1][lane], (unsigned long long)khi);
      atomicAdd((unsigned long long*)&s_acc[2][lane], (unsigned long long)klo);
    }
    __syncthreads();
    if (tid < nvalid) cloud_insert(G, s_acc[1][tid], s_acc[2][tid], s_acc[0][tid], (uint64_t)(tb + tid));
    __syncthreads();
  }
}

template <int NT>
hipError_t batch_mt_occupancy(BatchInfo* bi) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&bi->mt_per_cu[nt_index(NT)], k_batch_multi<NT>,
                                                      NT, 0);
}

template <int NT>
void launch_mt_batch(fi_graph* h, const BatchMArgs& a, hipStream_t s) {
  const BatchInfo* bi = (const BatchInfo*)h->batch;
  int64_t grid = (int64_t)std::max(1, bi->mt_per_cu[nt_index(NT)]) * h->cu_count;
  if (h->sched.grid > 0) grid = std::min<int64_t>(grid, h->sched.grid);
  grid = std::min<int64_t>(grid, (int64_t)bi->L.nmslots);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, (int64_t)a.G * a.groups));
  hipLaunchKernelGGL((k_batch_multi<NT>), dim3((int)grid), dim3(NT), 0, s, a);
}

bool host_offsets_ok(int32_t G, const int64_t* vo, const int64_t* no, int32_t* n_max) {
  if (G < 1 || !vo || !no || vo[0] != 0 || no[0] != 0) return false;
  *n_max = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t n = vo[g + 1] - vo[g], nnz = no[g + 1] - no[g];
    if (n < 0 || nnz < 0 || (nnz & 1) || n > kMaxBatchN) return false;
    *n_max = std::max(*n_max, (int32_t)n);
  }
  return vo[G] + G < ((int64_t)1 << 31) && no[G] < ((int64_t)1 << 31);
}

}  // namespace

void batch_info_free(void* p) { delete (BatchInfo*)p; }

}  // namespace fi

using namespace fi;

extern "C" {

int fi_batch_workspace_size(int32_t G, const int64_t* h_vertex_offsets,
                            const int64_t* h_nnz_offsets, int64_t cloud_capacity_per_graph,
                            size_t* out_bytes) {
  int32_t n_max = 0;
  if (!out_bytes || cloud_capacity_per_graph < 1 ||
      !host_offsets_ok(G, h_vertex_offsets, h_nnz_offsets, &n_max))
    return FI_EINVAL;
  int32_t n_max_large = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int32_t n = (int32_t)(h_vertex_offsets[g + 1] - h_vertex_offsets[g]);
    if (n > kLdsMaxN) n_max_large = std::max(n_max_large, n);
  }
  *out_bytes = batch_layout(G, h_vertex_offsets[G], h_nnz_offsets[G], n_max_large, n_max,
                            table_size_for(cloud_capacity_per_graph)).total;
  return FI_OK;
}

int fi_batch_create(int32_t G, const int64_t* h_vertex_offsets, const int64_t* h_nnz_offsets,
                    const int32_t* d_row_ptr, const int32_t* d_col, const int8_t* d_sign,
                    int64_t cloud_capacity_per_graph, void* d_workspace, size_t ws_bytes,
                    void* stream, fi_graph** out) {
  if (!out) return FI_EINVAL;
  *out = nullptr;
  int32_t n_max = 0;
  if (cloud_capacity_per_graph < 1 || !host_offsets_ok(G, h_vertex_offsets, h_nnz_offsets, &n_max))
    return FI_EINVAL;
  const int64_t n_total = h_vertex_offsets[G], nnz_total = h_nnz_offsets[G];
  if (!d_row_ptr || (nnz_total > 0 && (!d_col || !d_sign))) return FI_EINVAL;
  // host metadata and the two size classes, largest graph first
  std::vector<BatchGraph> meta(G);
  std::vector<int64_t> offs(4 * ((size_t)G + 1));
  int64_t me = 0;
  int32_t n_max_small = 0, n_max_large = 0;
  std::vector<int32_t> small, large;
  for (int32_t g = 0; g < G; ++g) {
    BatchGraph& b = meta[g];
    b.n = (int32_t)(h_vertex_offsets[g + 1] - h_vertex_offsets[g]);
    b.nwords = (b.n + 63) / 64;
    b.nnz = h_nnz_offsets[g + 1] - h_nnz_offsets[g];
    b.m = b.nnz / 2;
    b.vo = h_vertex_offsets[g];
    b.no = h_nnz_offsets[g];
    b.me = me;
    b.ro = h_vertex_offsets[g] + g;
    me += b.m;
    if (b.n <= kLdsMaxN) {
      small.push_back(g);
      n_max_small = std::max(n_max_small, b.n);
    } else {
      large.push_back(g);
      n_max_large = std::max(n_max_large, b.n);
    }
  }
  for (int32_t g = 0; g <= G; ++g) {
    offs[g] = g < G ? meta[g].vo : n_total;
    offs[(G + 1) + g] = g < G ? meta[g].no : nnz_total;
    offs[2 * (G + 1) + g] = g < G ? meta[g].me : me;
    offs[3 * (G + 1) + g] = g < G ? meta[g].ro : n_total + G;
  }
  auto by_size = [&](int32_t a, int32_t b) {
    return meta[a].nnz != meta[b].nnz ? meta[a].nnz > meta[b].nnz : a < b;
  };
  std::sort(small.begin(), small.end(), by_size);
  std::sort(large.begin(), large.end(), by_size);
  const uint64_t tsize = table_size_for(cloud_capacity_per_graph);
  BatchLayout L = batch_layout(G, n_total, nnz_total, n_max_large, n_max, tsize);
  if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace % kAlign)) return FI_EWORKSPACE;

  fi_graph* h = new (std::nothrow) fi_graph();
  BatchInfo* bi = new (std::nothrow) BatchInfo();
  if (!h || !bi) {
    delete h;
    delete bi;
    return FI_EINVAL;
  }
  h->is_batch = true;
  h->batch = bi;
  auto fail = [&](int code) {
    fi_graph_destroy(h);
    return code;
  };
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_workspace;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&h->max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return fail(FI_EDEVICE);
  bi->G = G;
  bi->n_total = n_total;
  bi->nnz_total = nnz_total;
  bi->m_total = me;
  bi->cap = cloud_capacity_per_graph;
  bi->tsize = tsize;
  bi->n_max_small = n_max_small;
  bi->n_max_large = n_max_large;
  bi->n_small = (int32_t)small.size();
  bi->n_large = (int32_t)large.size();
  bi->L = L;
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  h->sched = fi_schedule{0, 256, 0, 512, 1};
  h->dg.ctl = (uint64_t*)(ws + L.ctl);
  h->prof_events = prof_events_new();
  if (!h->prof_events) return fail(FI_EINVAL);

  BatchGraph* d_meta = (BatchGraph*)(ws + L.meta);
  int64_t* d_offs = (int64_t*)(ws + L.offs);
  const int64_t *d_vo = d_offs, *d_no = d_offs + (G + 1), *d_me = d_offs + 2 * (G + 1),
                *d_ro = d_offs + 3 * (G + 1);
  uint64_t* ctl = h->dg.ctl;
  const int B = 256;
  std::vector<uint64_t> zeros(C_WORDS, 0);
  if (hipMemcpyAsync(d_meta, meta.data(), sizeof(BatchGraph) * G, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(d_offs, offs.data(), 8 * offs.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ctl, zeros.data(), 8 * C_WORDS, hipMemcpyHostToDevice, s) != hipSuccess ||
      (small.size() && hipMemcpyAsync(ws + L.small, small.data(), 4 * small.size(),
                                      hipMemcpyHostToDevice, s) != hipSuccess) ||
      (large.size() && hipMemcpyAsync(ws + L.large, large.data(), 4 * large.size(),
                                      hipMemcpyHostToDevice, s) != hipSuccess))
    return fail(FI_EDEVICE);
  // row offsets first: the entry checks index columns through them
  hipLaunchKernelGGL(k_b_rowptr, dim3(grid_for(n_total + G, B)), dim3(B), 0, s, d_row_ptr, d_meta,
                     d_ro, G, n_total + G, ctl);
  uint64_t flags = 0;
  if (hipMemcpyAsync(&flags, ctl + C_FLAGS, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FI_EDEVICE);
  if (flags & V_ROWPTR) return fail(FI_EINVAL);
  if (nnz_total > 0)
    hipLaunchKernelGGL(k_b_entries, dim3(grid_for(nnz_total, B, 16384)), dim3(B), 0, s, d_row_ptr,
                       d_col, d_sign, d_meta, d_no, G, nnz_total, ctl);
  if (hipMemcpyAsync(&flags, ctl + C_FLAGS, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FI_EDEVICE);
  if (flags & V_RANGE) return fail(FI_EINVAL);
  if (flags & V_SIGN) return fail(FI_ESIGN);
  if (flags & V_SELF) return fail(FI_ESELFLOOP);
  if (flags & V_DUP) return fail(FI_EDUP);
  if (flags & V_UNSORTED) return fail(FI_EUNSORTED);
  if (flags & V_ASYM) return fail(FI_EASYM);

  int32_t* rp = (int32_t*)(ws + L.row_ptr);
  int32_t* ustart = (int32_t*)(ws + L.ustart);
  int32_t* eoff = (int32_t*)(ws + L.eoff);
  hipLaunchKernelGGL(k_b_copy_rp, dim3(grid_for(n_total + G, B)), dim3(B), 0, s, d_row_ptr, rp,
                     n_total + G);
  if (n_total > 0) {
    hipLaunchKernelGGL(k_b_upper, dim3(grid_for(n_total, B)), dim3(B), 0, s, d_row_ptr, d_col, d_meta,
                       d_vo, G, n_total, ustart, eoff);
    // exclusive scan of the per-vertex upper counts (graphs in order, so each
    // graph's edges are contiguous from its edge offset)
    std::vector<int32_t> cnt(n_total);
    if (hipMemcpyAsync(cnt.data(), eoff, 4 * n_total, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(FI_EDEVICE);
    int64_t acc = 0;
    for (int64_t v = 0; v < n_total; ++v) {
      const int32_t c = cnt[v];
      cnt[v] = (int32_t)acc;
      acc += c;
    }
    if (acc != me) return fail(FI_EASYM);
    if (hipMemcpyAsync(eoff, cnt.data(), 4 * n_total, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(FI_EDEVICE);
  }
  if (nnz_total > 0)
    hipLaunchKernelGGL(k_b_pack, dim3(grid_for(nnz_total, B, 16384)), dim3(B), 0, s, d_row_ptr, d_col,
                       d_sign, d_meta, d_no, G, nnz_total, ustart, eoff, (uint32_t*)(ws + L.adj),
                       (uint2*)(ws + L.edges), rp);
  if (n_total > 0) {
    int32_t* parent = (int32_t*)(ws + L.ustart);  // free again after packing
    hipLaunchKernelGGL(k_b_uf_init, dim3(grid_for(n_total, B)), dim3(B), 0, s, parent, n_total);
    if (me > 0)
      hipLaunchKernelGGL(k_b_uf_hook, dim3(grid_for(me, B, 16384)), dim3(B), 0, s,
                         (const uint2*)(ws + L.edges), d_meta, d_me, G, me, parent);
    hipLaunchKernelGGL(k_b_uf_local, dim3(grid_for(n_total, B)), dim3(B), 0, s, parent, d_meta, d_vo,
                       G, n_total, (int32_t*)(ws + L.comp));
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return fail(FI_EDEVICE);

  // multi-tree sweep: every graph's components numbered in id order of their
  // anchors (component index per vertex), graphs largest first, root tables
  {
    std::vector<int32_t> anchors;
    if (n_total > 0) {
      int32_t* alist = (int32_t*)(ws + L.ustart);  // free again after union-find
      uint64_t zero = 0, count = 0;
      if (hipMemcpyAsync(ctl + C_NANCH, &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(FI_EDEVICE);
      hipLaunchKernelGGL(k_b_anchors, dim3(grid_for(n_total, B)), dim3(B), 0, s, rp, d_meta, d_vo, G,
                         n_total, (const int32_t*)(ws + L.comp), alist, (uint32_t*)(ctl + C_NANCH));
      if (hipMemcpyAsync(&count, ctl + C_NANCH, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(FI_EDEVICE);
      anchors.resize(count);
      if (count && (hipMemcpyAsync(anchors.data(), alist, 4 * count, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess))
        return fail(FI_EDEVICE);
      std::sort(anchors.begin(), anchors.end());
    }
    for (int32_t g = 0; g < G; ++g) {
      const auto lo = std::lower_bound(anchors.begin(), anchors.end(), (int32_t)meta[g].vo);
      const auto hi = std::lower_bound(anchors.begin(), anchors.end(), (int32_t)(meta[g].vo + meta[g].n));
      meta[g].cs = (int32_t)(lo - anchors.begin());
      meta[g].ncomp = (int32_t)(hi - lo);
    }
    std::vector<int32_t> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), by_size);
    if (hipMemcpyAsync(d_meta, meta.data(), sizeof(BatchGraph) * G, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ws + L.order, order.data(), 4 * (size_t)G, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(FI_EDEVICE);
    if (!anchors.empty()) {
      int32_t* sorted = (int32_t*)(ws + L.eoff);  // free after packing
      int32_t* slot = (int32_t*)(ws + L.ustart);
      if (hipMemcpyAsync(sorted, anchors.data(), 4 * anchors.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(FI_EDEVICE);
      hipLaunchKernelGGL(k_b_scatter_slot, dim3(grid_for((int64_t)anchors.size(), B)), dim3(B), 0, s, sorted,
                         (int64_t)anchors.size(), slot);
      hipLaunchKernelGGL(k_b_cidx, dim3(grid_for(n_total, B)), dim3(B), 0, s, rp, d_meta, d_vo, G, n_total,
                         (const int32_t*)(ws + L.comp), (const int32_t*)slot, (int32_t*)(ws + L.cidx));
    } else if (n_total > 0) {
      hipLaunchKernelGGL(k_b_cidx_none, dim3(grid_for(n_total, B)), dim3(B), 0, s, (int32_t*)(ws + L.cidx),
                         n_total);
    }
    const size_t nm = (size_t)std::max(n_max, 1);
    hipLaunchKernelGGL(k_b_mt_tables, dim3(grid_for((int64_t)L.nmslots * 64 * kRootRows, B)), dim3(B), 0, s,
                       ws + L.mslots, L.mslot_stride, L.nmslots, 32 * nm + 8 * (nm / 64 + 2));
    bi->n_max = n_max;
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return fail(FI_EDEVICE);
  if (batch_occupancy<256>(bi) != hipSuccess || batch_occupancy<512>(bi) != hipSuccess ||
      batch_occupancy<1024>(bi) != hipSuccess || batch_mt_occupancy<256>(bi) != hipSuccess ||
      batch_mt_occupancy<512>(bi) != hipSuccess || batch_mt_occupancy<1024>(bi) != hipSuccess)
    return fail(FI_EDEVICE);
  *out = h;
  return FI_OK;
}

int fi_batch_sweep(fi_graph* h, int64_t trees_per_graph, uint64_t seed, uint64_t* d_min_per_graph,
                   uint64_t* d_distinct_per_graph, void* stream) {
  if (!h || !h->is_batch || trees_per_graph < 1 || !d_min_per_graph) return FI_EINVAL;
  if (trees_per_graph >= ((int64_t)1 << 32)) return FI_ERANGE;
  BatchInfo* bi = (BatchInfo*)h->batch;
  const BatchLayout& L = bi->L;
  hipStream_t s = (hipStream_t)stream;
  char* ws = h->ws;
  uint64_t* ctl = h->dg.ctl;
  BatchArgs a{};
  a.meta = (const BatchGraph*)(ws + L.meta);
  a.row_ptr = (const int32_t*)(ws + L.row_ptr);
  a.adj = (const uint32_t*)(ws + L.adj);
  a.edges = (const uint2*)(ws + L.edges);
  a.comp = (const int32_t*)(ws + L.comp);
  a.clouds = (CloudSlot*)(ws + L.clouds);
  a.gctl = (uint64_t*)(ws + L.gctl);
  a.trees = trees_per_graph;
  a.seed = seed;
  a.tsize = bi->tsize;
  a.cap = (uint64_t)bi->cap;
  a.slots = ws + L.slots;
  a.slot_stride = L.slot_stride;
  const int nt = h->sched.block;
  // clouds, per-graph minima and counters, error bits and both tickets
  hipLaunchKernelGGL(k_b_reset, dim3(grid_for((int64_t)bi->tsize * bi->G, 256)), dim3(256), 0, s,
                     (CloudSlot*)(ws + L.clouds), (int64_t)bi->tsize * bi->G, (uint64_t*)(ws + L.gctl),
                     bi->G, ctl);
  hipError_t e = hipGetLastError();
  // 64 trees of a graph per workgroup pass, unless a per-tree schedule is
  // asked for or there are too few trees per graph to share a pass
  const bool multi = h->sched.path == 4 || (h->sched.path == 0 && trees_per_graph >= 16);
  if (multi && e == hipSuccess) {
    BatchMArgs m{};
    m.meta = a.meta;
    m.row_ptr = a.row_ptr;
    m.adj = a.adj;
    m.edges = a.edges;
    m.comp = a.comp;
    m.cidx = (const int32_t*)(ws + L.cidx);
    m.clouds = a.clouds;
    m.gctl = a.gctl;
    m.order = (const int32_t*)(ws + L.order);
    m.ticket = ctl + kTicket0;
    m.G = bi->G;
    m.groups = (int32_t)((trees_per_graph + 63) / 64);
    m.trees = trees_per_graph;
    m.seed = seed;
    m.tsize = bi->tsize;
    m.cap = (uint64_t)bi->cap;
    m.slots = ws + L.mslots;
    m.slot_stride = L.mslot_stride;
    m.n_max = bi->n_max;
    void* tok = nullptr;
    if (prof_begin(h, s, &tok)) return FI_EDEVICE;
    if (nt == 1024) launch_mt_batch<1024>(h, m, s);
    else if (nt == 512) launch_mt_batch<512>(h, m, s);
    else launch_mt_batch<256>(h, m, s);
    e = hipGetLastError();
    prof_end(h, s, tok, 0);
  }
  for (int cls = 0; cls < 2 && e == hipSuccess && !multi; ++cls) {
    const bool lds = cls == 0;
    a.order = (const int32_t*)(ws + (lds ? L.small : L.large));
    a.nitems = (int64_t)(lds ? bi->n_small : bi->n_large) * trees_per_graph;
    a.ticket = ctl + (lds ? kTicket0 : kTicket1);
    if (a.nitems == 0) continue;
    void* tok = nullptr;
    if (prof_begin(h, s, &tok)) return FI_EDEVICE;
    if (nt == 1024) launch_class<1024>(h, a, lds, s);
    else if (nt == 512) launch_class<512>(h, a, lds, s);
    else launch_class<256>(h, a, lds, s);
    e = hipGetLastError();
    prof_end(h, s, tok, 0);
  }
  if (e != hipSuccess) return FI_EDEVICE;
  hipLaunchKernelGGL(k_b_finish, dim3(grid_for(bi->G, 256)), dim3(256), 0, s,
                     (const uint64_t*)(ws + L.gctl), bi->G, d_min_per_graph, d_distinct_per_graph, ctl);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_batch_cloud_read(fi_graph* h, int32_t graph, fi_cloud_entry* h_out, int64_t cap,
                        int64_t* written, void* stream) {
  if (!h || !h->is_batch || cap < 0 || (cap > 0 && !h_out)) return FI_EINVAL;
  auto* bi = (BatchInfo*)h->batch;
  if (graph < 0 || graph >= bi->G) return FI_EINVAL;
  const int e = fi_graph_status(h, stream);
  if (e) return e;
  const CloudSlot* table = (const CloudSlot*)(h->ws + bi->L.clouds) + (size_t)graph * bi->tsize;
  return read_cloud_table(table, bi->tsize, h_out, cap, written, (hipStream_t)stream);
}

}  // extern "C"
