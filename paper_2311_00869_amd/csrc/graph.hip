// Graph upload, validation, connected components, the cloud table and its
// readout, the exact frustration counter over given states, schedules,
// profiling and error strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline int grid_for(int64_t work, int block, int cap = 65536) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ------------------------------------------------------------ validation
// Row of CSR entry e: the largest u < n with row_ptr[u] <= e.
__device__ __forceinline__ int32_t row_of(const int32_t* rp, int32_t n, int64_t e) {
  int32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    int32_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)rp[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_check_rowptr(const int32_t* rp, int32_t n, int64_t nnz, uint64_t* ctl) {
  uint32_t bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (rp[i + 1] < rp[i]) bad = 1;
    if (i == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) bad = 1;
  }
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || nnz != 0)) bad = 1;
  if (bad) atomicOr((unsigned long long*)(ctl + C_FLAGS), (unsigned long long)V_ROWPTR);
}

__global__ void k_check_entries(const int32_t* rp, const int32_t* col, const int8_t* sign,
                                int32_t n, int64_t nnz, uint64_t* ctl) {
  uint32_t f = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = row_of(rp, n, e);
    int32_t v = col[e];
    int s = sign[e];
    if (v < 0 || v >= n) { f |= V_RANGE; continue; }
    if (s != 1 && s != -1) f |= V_SIGN;
    if (v == u) f |= V_SELF;
    if (e + 1 < (int64_t)rp[u + 1]) {
      int32_t c2 = col[e + 1];
      if (c2 == v) f |= V_DUP;
      else if (c2 < v) f |= V_UNSORTED;
    }
    // the reverse entry v -> u, by binary search in v's (sorted) row
    int64_t lo = rp[v], hi = rp[v + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (col[mid] < u) lo = mid + 1; else hi = mid;
    }
    if (lo >= rp[v + 1] || col[lo] != u || sign[lo] != s) f |= V_ASYM;
  }
  if (f) atomicOr((unsigned long long*)(ctl + C_FLAGS), (unsigned long long)f);
}

// ------------------------------------------------------------ packing
// Per row: first entry with column > u, and the number of such entries.
__global__ void k_row_upper(const int32_t* rp, const int32_t* col, int32_t n, int32_t* upper_start,
                            int32_t* upper_cnt) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = rp[u], hi = rp[u + 1];
    while (lo < hi) {
      int32_t mid = lo + ((hi - lo) >> 1);
      if (col[mid] <= (int32_t)u) lo = mid + 1; else hi = mid;
    }
    upper_start[u] = lo;
    upper_cnt[u] = rp[u + 1] - lo;
  }
}

// Exclusive scan, three passes of 1024-element tiles.
constexpr int kScanBlock = 256;
constexpr int kScanTile = 1024;

__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(int32_t* a, int64_t len, int32_t* tile_sums) {
  __shared__ int s_tmp[kScanBlock / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < len ? a[base + k] : 0;
    sum += v[k];
  }
  int total;
  int pre = block_exclusive_scan<kScanBlock>(sum, total, s_tmp);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < len) a[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int32_t* sums, int64_t ntiles, int32_t* total_out) {
  __shared__ int s_tmp[kScanBlock / 64 + 1];
  int carry = 0;
  for (int64_t c = 0; c < ntiles; c += kScanBlock) {
    int64_t i = c + threadIdx.x;
    int x = i < ntiles ? sums[i] : 0;
    int total;
    int pre = block_exclusive_scan<kScanBlock>(x, total, s_tmp);
    if (i < ntiles) sums[i] = pre + carry;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int32_t* a, int64_t len, const int32_t* tile_sums) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] += tile_sums[i / kScanTile];
}

__global__ void k_pack(const int32_t* rp, const int32_t* col, const int8_t* sign, int32_t n,
                       int64_t nnz, const int32_t* upper_start, const int32_t* edge_off,
                       uint32_t* adj, uint2* edges) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = row_of(rp, n, e);
    uint32_t v = (uint32_t)col[e];
    uint32_t neg = sign[e] < 0 ? 1u : 0u;
    uint32_t a = v | (neg << 31);
    adj[e] = a;
    if ((int32_t)v > u) edges[edge_off[u] + (e - upper_start[u])] = make_uint2((uint32_t)u, a);
  }
}

// The counting edge list: every edge once, from the endpoint of lower rank
// (degree, then id) to the one of higher rank, in row order.  A count streams
// the lower-ranked endpoint and gathers the other, so the gathers land on
// high-degree vertices, whose words the caches hold.  One wave per row; with
// out null it writes each row's entry count to cnt, else the entries at
// off[v].
__global__ void k_orient(const int32_t* rp, const uint32_t* adj, int32_t n, const int32_t* off,
                         int32_t* cnt, uint2* out) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
    int32_t k = 0;
    for (int32_t c = b; c < e; c += 64) {
      const int32_t i = c + lane;
      bool take = false;
      uint32_t a = 0;
      if (i < e) {
        a = adj[i];
        const int32_t u = (int32_t)(a & kVertexMask);
        const int32_t du = rp[u + 1] - rp[u];
        take = du > dv || (du == dv && u > (int32_t)v);
      }
      const uint64_t m = __ballot(take);
      if (out && take) out[off[v] + k + (int32_t)lanes_below(m)] = make_uint2((uint32_t)v, a);
      k += (int32_t)__popcll(m);
    }
    if (!out && lane == 0) cnt[v] = k;
  }
}

__global__ void k_copy_i32(const int32_t* src, int32_t* dst, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------------------ components
// Lock-free union-find: every edge hooks the larger of its two roots under the
// smaller, so each component's final root is its smallest vertex id.  Parent
// reads use agent-scope atomic loads so a retry always sees fresh pointers.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t p = load_agent_i32(parent + x);
  while (p != x) {
    x = p;
    p = load_agent_i32(parent + x);
  }
  return x;
}

__global__ void k_uf_init(int32_t* parent, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = (int32_t)v;
}

__global__ void k_uf_hook(const uint2* edges, int64_t m, int32_t* parent) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = (int32_t)edges[e].x;
    int32_t v = (int32_t)(edges[e].y & kVertexMask);
    while (true) {
      int32_t ru = uf_find(parent, u), rv = uf_find(parent, v);
      if (ru == rv) break;
      int32_t lo = min(ru, rv), hi = max(ru, rv);
      int32_t old = atomicCAS(parent + hi, hi, lo);
      if (old == hi) break;
    }
  }
}

__global__ void k_uf_compress(int32_t* parent, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = uf_find(parent, (int32_t)v);
}

// One wave per 64-vertex word: which vertices have edges, the smallest anchor
// among them (the word's "main" component, -2 if none) and which of them
// belong to it.  Also lists anchors of components with an edge and counts
// components and isolated vertices.
__global__ void k_word_info(const int32_t* rp, const int32_t* comp, int32_t n, int32_t nwords,
                            int32_t* word_comp, uint64_t* word_mask, uint64_t* word_main,
                            int32_t* anchors, uint64_t* ctl) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t ncomp = 0, niso = 0;
  for (int64_t i = wave; i < nwords; i += nwaves) {
    int64_t v = i * 64 + lane;
    bool valid = v < n;
    bool has_edge = valid && rp[v + 1] > rp[v];
    int32_t c = has_edge ? comp[v] : INT32_MAX;
    int32_t cmin = wave_min_i32(c);
    uint64_t mask = __ballot(has_edge);
    uint64_t main = __ballot(has_edge && c == cmin);
    if (lane == 0) {
      word_mask[i] = mask;
      word_main[i] = main;
      word_comp[i] = mask == 0 ? -2 : cmin;
    }
    bool is_anchor = has_edge && comp[v] == (int32_t)v;
    if (valid && comp[v] == (int32_t)v) ncomp++;
    if (valid && !has_edge) niso++;
    wave_append(is_anchor, (int32_t)v, anchors, (uint32_t*)(ctl + C_NANCH));
  }
  uint64_t a = wave_sum_u64(ncomp), b = wave_sum_u64(niso);
  if (lane == 0) {
    if (a) atomicAdd((unsigned long long*)(ctl + C_NCOMP), (unsigned long long)a);
    if (b) atomicAdd((unsigned long long*)(ctl + C_NISO), (unsigned long long)b);
  }
}

// Component vertex lists for the multi-tree path: slot of each anchor,
// vertices per slot, then every vertex with an edge placed in its slot's range.
__global__ void k_aslot(const int32_t* anchors, int32_t nanch, int32_t* aslot) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nanch;
       i += (int64_t)gridDim.x * blockDim.x)
    aslot[anchors[i]] = (int32_t)i;
}

// Slot of vertex v's component (-1 without an edge).  Whole waves of one
// component (the common case of a giant component) take one atomic.
__device__ __forceinline__ int32_t comp_slot(const int32_t* rp, const int32_t* comp,
                                             const int32_t* aslot, int64_t v, int32_t n) {
  return v < n && rp[v + 1] > rp[v] ? aslot[comp[v]] : -1;
}

__global__ void k_ccount(const int32_t* rp, const int32_t* comp, const int32_t* aslot, int32_t n,
                         int32_t* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    const int32_t sl = comp_slot(rp, comp, aslot, v, n);
    const uint64_t mask = __ballot(sl >= 0);
    if (!mask) continue;
    const int32_t s0 = __shfl(sl, __ffsll((unsigned long long)mask) - 1);
    if (__ballot(sl >= 0 && sl != s0) == 0) {
      if (lanes_below(mask) == 0 && sl >= 0) atomicAdd(count + s0, (int)__popcll(mask));
    } else if (sl >= 0) {
      atomicAdd(count + sl, 1);
    }
  }
}

__global__ void k_cfill(const int32_t* rp, const int32_t* comp, const int32_t* aslot,
                        const int32_t* cptr, int32_t n, int32_t* fill, int32_t* cverts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    const int32_t sl = comp_slot(rp, comp, aslot, v, n);
    const uint64_t mask = __ballot(sl >= 0);
    if (!mask) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    const int32_t s0 = __shfl(sl, leader);
    if (__ballot(sl >= 0 && sl != s0) == 0) {
      int32_t base = 0;
      if (lane_id() == leader) base = atomicAdd(fill + s0, (int)__popcll(mask));
      base = __shfl(base, leader);
      if (sl >= 0) cverts[cptr[s0] + base + (int32_t)lanes_below(mask)] = (int32_t)v;
    } else if (sl >= 0) {
      cverts[cptr[sl] + atomicAdd(fill + sl, 1)] = (int32_t)v;
    }
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t len, int32_t val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void k_fill_u64(uint64_t* p, int64_t len, uint64_t val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void k_cloud_reset(CloudSlot* t, int64_t size, uint64_t* ctl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < size;
       i += (int64_t)gridDim.x * blockDim.x) {
    CloudSlot s;
    s.tag = kEmpty;
    s.khi_min = ~0ull; s.khi_max = 0;
    s.s_min = ~0ull; s.s_max = 0;
    s.freq = 0; s.first = ~0ull; s.pad = 0;
    t[i] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[C_ERR] = 0;
    ctl[C_BEST] = ~0ull;
    ctl[C_COUNT] = 0;
    ctl[C_TREES] = 0;
  }
}

// Merge saved cloud entries (5 words each) as if their trees had been swept.
__global__ void k_cloud_load(DevGraph G, const uint64_t* e, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t khi = e[5 * i], klo = e[5 * i + 1], freq = e[5 * i + 2], S = e[5 * i + 3],
             first = e[5 * i + 4];
    if (klo == kEmpty) {
      atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_COLLISION);
      continue;
    }
    uint64_t idx = klo & G.cloud_mask;
    bool done = false;
    for (uint64_t probe = 0; probe <= G.cloud_mask && !done; ++probe) {
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
        atomicAdd((unsigned long long*)&s->freq, (unsigned long long)freq);
        atomicMin((unsigned long long*)&s->first, (unsigned long long)first);
        atomicAdd((unsigned long long*)(G.ctl + C_TREES), (unsigned long long)freq);
        atomicMin((unsigned long long*)(G.ctl + C_BEST), (unsigned long long)((S << 32) | first));
        done = true;
      }
      idx = (idx + 1) & G.cloud_mask;
    }
    if (!done) atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_CAPACITY);
  }
}

// ------------------------------------------------------------ exact count
// Frustrated edges of up to 64 states in one pass over the edge list.  st[v]
// holds vertex v's state in every state of the group (bit b = state b,
// set = -1).  Each lane takes one edge at a time: x = st[u] ^ st[v] ^ (all
// ones for a negative edge) has bit b set when the edge is frustrated in
// state b, and goes into 8 bit-sliced counter planes (a ripple-carry add of
// one bit per state).  Every 255 edges the planes are read out by ballots
// into per-state totals, lane b keeping state b's, and one LDS atomic per
// wave and one global atomic per block and state finish the sum.
constexpr int kCountBlock = 256;
constexpr int kCountPlanes = 8;
constexpr int kCountEdges = 4;
// T: uint32_t for up to 32 states (a 4-byte word per vertex, half the
// gathered bytes), uint64_t for up to 64.
template <typename T>
__global__ void __launch_bounds__(kCountBlock) k_count(const uint2* edges, int64_t m, const T* st,
                                                     int nstates, uint64_t* counts) {
  __shared__ uint64_t s_acc[64];
  const int lane = lane_id();
  if (threadIdx.x < 64) s_acc[threadIdx.x] = 0;
  __syncthreads();
  const T smask = nstates >= (int)(8 * sizeof(T)) ? (T)~(T)0 : (T)(((T)1 << nstates) - 1);
  T c[kCountPlanes];
#pragma unroll
  for (int p = 0; p < kCountPlanes; ++p) c[p] = 0;
  uint64_t mine = 0;
  int it = 0;
  auto flush = [&]() {
    for (int b = 0; b < nstates; ++b) {
      uint32_t tot = 0;
#pragma unroll
      for (int p = 0; p < kCountPlanes; ++p)
        tot += (uint32_t)__popcll(__ballot((c[p] >> b) & 1)) << p;
      if (lane == b) mine += tot;
    }
#pragma unroll
    for (int p = 0; p < kCountPlanes; ++p) c[p] = 0;
  };
  // kCountEdges edges per lane at a time keep that many gather chains in
  // flight (past the end a lane reads vertex 0 and adds nothing); the loop
  // bound is uniform over the block, so every wave reaches each flush
  for (int64_t e0 = (int64_t)blockIdx.x * kCountBlock * kCountEdges; e0 < m;
       e0 += (int64_t)gridDim.x * kCountBlock * kCountEdges) {
    uint2 uv[kCountEdges];
#pragma unroll
    for (int k = 0; k < kCountEdges; ++k) {
      const int64_t e = e0 + (int64_t)k * kCountBlock + threadIdx.x;
      uv[k] = e < m ? edges[e] : make_uint2(0u, 0u);
    }
    T su[kCountEdges], sv[kCountEdges];
#pragma unroll
    for (int k = 0; k < kCountEdges; ++k) {
      su[k] = st[uv[k].x];
      sv[k] = st[uv[k].y & kVertexMask];
    }
#pragma unroll
    for (int k = 0; k < kCountEdges; ++k) {
      const int64_t e = e0 + (int64_t)k * kCountBlock + threadIdx.x;
      const T neg = (uv[k].y >> 31) ? (T)~(T)0 : (T)0;
      T x = e < m ? (T)((su[k] ^ sv[k] ^ neg) & smask) : (T)0;
#pragma unroll
      for (int p = 0; p < kCountPlanes; ++p) {
        const T carry = c[p] & x;
        c[p] ^= x;
        x = carry;
      }
    }
    it += kCountEdges;
    if (it + kCountEdges > 255) {
      flush();
      it = 0;
    }
  }
  flush();
  if (mine) atomicAdd((unsigned long long*)&s_acc[lane], (unsigned long long)mine);
  __syncthreads();
  if (threadIdx.x < nstates && s_acc[threadIdx.x])
    atomicAdd((unsigned long long*)(counts + threadIdx.x), (unsigned long long)s_acc[threadIdx.x]);
}

// States given as bitmaps (state b: words bits[b * nwords + i], vertex v is
// bit v % 64 of word v / 64) turned into one word per vertex: bit b of st[v]
// is v's bit in state b, for b < nstates (<= 8 sizeof(T)).  The 64 lanes of
// a wave share each bitmap word, so every word is read once.
template <typename T>
__global__ void k_states_by_vertex(const uint64_t* bits, int32_t nwords, int32_t n, int nstates,
                                   T* st) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = v >> 6;
    const int sh = (int)(v & 63);
    T w = 0;
    for (int b = 0; b < nstates; ++b) w |= (T)((bits[(size_t)b * nwords + i] >> sh) & 1ull) << b;
    st[v] = w;
  }
}

int err_from_bits(uint64_t bits) {
  if (bits & E_DEPTH) return FI_EDEPTH;
  if (bits & E_COLLISION) return FI_ECOLLISION;
  if (bits & E_CAPACITY) return FI_ECAPACITY;
  return FI_OK;
}

struct ProfEvent {
  hipEvent_t a, b;
  int kernel;
};

}  // namespace

int read_cloud_table(const CloudSlot* d_table, uint64_t tsize, fi_cloud_entry* h_out, int64_t cap,
                     int64_t* written, hipStream_t s) {
  std::vector<CloudSlot> table(tsize);
  if (hipMemcpyAsync(table.data(), d_table, sizeof(CloudSlot) * tsize, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FI_EDEVICE;
  std::vector<fi_cloud_entry> rows;
  for (const CloudSlot& c : table) {
    if (c.tag == kEmpty) continue;
    if (c.khi_min != c.khi_max || c.s_min != c.s_max) return FI_ECOLLISION;
    rows.push_back(fi_cloud_entry{c.khi_min, c.tag, c.freq, c.s_min, c.first});
  }
  std::sort(rows.begin(), rows.end(), [](const fi_cloud_entry& a, const fi_cloud_entry& b) {
    return a.key_hi != b.key_hi ? a.key_hi < b.key_hi : a.key_lo < b.key_lo;
  });
  const int64_t k = std::min<int64_t>(cap, (int64_t)rows.size());
  if (k > 0) std::memcpy(h_out, rows.data(), sizeof(fi_cloud_entry) * k);
  if (written) *written = (int64_t)rows.size();
  return FI_OK;
}

uint64_t table_size_for(int64_t cloud_capacity) {
  uint64_t want = (uint64_t)std::max<int64_t>(cloud_capacity, 1) * 2;
  uint64_t s = 64;
  while (s < want) s <<= 1;
  return s;
}

// root-finding chunks of components up to kRootWide vertices (see
// build_components)
constexpr int32_t kRootChunkSmall = 256;
constexpr int32_t kRootWide = 2097152;

Layout make_layout(int32_t n, int64_t nnz, int64_t cloud_capacity, uint64_t table_size) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t nn = (size_t)n, m = (size_t)nnz / 2, nw = ((size_t)n + 63) / 64;
  L.row_ptr = take(4 * (nn + 1));
  L.adj = take(4 * (size_t)nnz);
  L.edges = take(8 * m);
  L.cedges = take(8 * m);
  L.comp = take(4 * nn);
  L.word_comp = take(4 * nw);
  L.word_mask = take(8 * nw);
  L.word_main = take(8 * nw);
  L.anchors = take(4 * nn);
  L.tmp = take(4 * (nn / kScanTile + 2));
  L.cloud = take(sizeof(CloudSlot) * table_size);
  L.ctl = take(8 * C_WORDS);
  // two int32 arrays of n + 64 at create; cloud staging; R <= 64 rounded states
  L.scratch = take(std::max<size_t>(8 * (nn + 64), 8 * (size_t)kGraphLMaxR * nw));
  L.gl = take(8 * (size_t)kGraphLBlocks * kGraphLMaxR);
  // whole-grid path
  const size_t S = kGridSlots;
  L.hcap = (size_t)nnz / 32 + 1;
  L.gpstride = (nn + 31) / 32 * 32;
  L.gwstride = (nw + 31) / 32 * 32;
  L.gpw = take(8 * S * L.gpstride);
  L.gql = take(4 * S * 2 * (nn + 64));
  L.gqh = take(8 * S * 2 * (L.hcap + 64));
  L.gfb = take(8 * 3 * S * L.gwstride); // three frontier bitmaps per slot
  L.gvis = take(8 * S * L.gwstride);    // visited, per slot
  L.gsb = take(8 * S * L.gwstride);     // state bits, per slot
  L.grootkey = take(8 * S * L.gpstride);
  L.gctl = take(8 * S * kGridCtlWords);
  L.gbar = take(8 * S * kGridBarWords);
  // per-workgroup tree scratch (a tree word and a queue entry per vertex)
  L.slot_stride = align_up(16 * nn);  // tree words, queue, and Kruskal's hooks
  L.nslots = 0;
  if (n > 0 && n <= 1000000) {
    size_t budget = (size_t)8 << 30;
    L.nslots = std::min<size_t>(2048, std::max<size_t>(1, budget / L.slot_stride));
  }
  L.slots = take(L.slot_stride * L.nslots);
  // multi-tree path (the lists, bitmaps, control and barrier words are the
  // whole-grid path's, which never runs at the same time)
  L.mrec = take(64 * nn);  // a record per vertex: four fields of up to two 8-byte tree words
  L.mhcap = (size_t)nnz / kMSplit + 1;
  L.mhslot = take(8 * 128 * L.mhcap);
  // reached bitmaps over the two levels' list entries: light, then split rows
  L.mreach = take(8 * (4 * ((nn + 64) / 64 + 2) + 2 * (L.mhcap / 64 + 2)));
  L.aslot = take(4 * nn);
  L.cverts = take(4 * nn);
  L.ccount = take(4 * (nn / 2 + 1));
  L.cptr = take(4 * (nn / 2 + 2));
  L.mtcap = nn / 2 + nn / kRootChunkSmall + 2;
  L.mtasks = take(16 * L.mtcap);
  L.nbigcap = nn / kBigComp + 1;
  L.rootbig = take(8 * 128 * L.nbigcap);
  L.swtile = take(16 * ((size_t)switch_tiles((int64_t)m) + 1));
  L.glheavy = take(4 * ((size_t)nnz / kGLHeavy + 2));
  L.glfirst = take(4 * ((size_t)nnz / kGLHeavy + 3));
  L.glicap = (size_t)nnz / kGLChunk + (size_t)nnz / kGLHeavy + 2;
  L.glitems = take(8 * L.glicap);
  L.glpart = take(4 * (size_t)kGraphLMaxR * L.glicap);
  L.glctl = take(64);
  L.cent = take(2 * nn);
  L.oroot = take(8 * (size_t)kOrderMax);
  L.okey = take(8 * (size_t)kOrderMax);
  L.operm = take(4 * (size_t)kOrderMax);
  L.total = off;
  return L;
}

// The multi-tree path's component lists and root-finding tasks: every
// component with an edge gets one task if it has at most kBigComp vertices,
// else one task per chunk of its vertices and a row of big-component minima.
// A task is one wave's serial scan, and every task of a component ends in
// the same 64 W minima: components up to kRootWide vertices take chunks of
// kRootChunkSmall (more waves on the scan), larger ones kRootChunk (fewer
// atomic minima on those words).  Also resets the split-row and big-component
// minima.
int build_components(fi_graph* g, hipStream_t s) {
  const Layout& L = g->L;
  char* ws = g->ws;
  const DevGraph& G = g->dg;
  const int32_t n = G.n;
  const int B = 256;
  uint64_t nanch64 = 0;
  if (hipMemcpyAsync(&nanch64, G.ctl + C_NANCH, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FI_EDEVICE;
  const int32_t nanch = (int32_t)nanch64;
  int32_t* aslot = (int32_t*)(ws + L.aslot);
  int32_t* count = (int32_t*)(ws + L.ccount);
  g->gl_main_slot = -1;
  g->main_begin = g->main_end = 0;
  g->main_big = -1;
  int32_t* cptr = (int32_t*)(ws + L.cptr);
  std::vector<int32_t> cnt(nanch), ptr(nanch + 1, 0);
  std::vector<int4> tasks;
  int32_t nbig = 0;
  if (nanch > 0) {
    hipLaunchKernelGGL(k_aslot, dim3(grid_for(nanch, B)), dim3(B), 0, s, G.anchors, nanch, aslot);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nanch, B)), dim3(B), 0, s, count, (int64_t)nanch, 0);
    hipLaunchKernelGGL(k_ccount, dim3(grid_for(n, B)), dim3(B), 0, s, G.row_ptr, G.comp, aslot, n,
                       count);
    if (hipMemcpyAsync(cnt.data(), count, 4 * (size_t)nanch, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FI_EDEVICE;
    for (int32_t i = 0; i < nanch; ++i) {
      const bool main = g->gl_main_slot < 0 || cnt[i] > cnt[g->gl_main_slot];
      if (main) g->gl_main_slot = i;
      ptr[i + 1] = ptr[i] + cnt[i];
      if (main) {
        g->main_begin = ptr[i];
        g->main_end = ptr[i + 1];
        g->main_big = cnt[i] <= kBigComp ? -1 : nbig;
      }
      if (cnt[i] <= kBigComp) {
        tasks.push_back(make_int4(ptr[i], ptr[i + 1], -1, 0));
      } else {
        const int32_t chunk = cnt[i] <= kRootWide ? kRootChunkSmall : kRootChunk;
        for (int32_t b = ptr[i]; b < ptr[i + 1]; b += chunk)
          tasks.push_back(make_int4(b, std::min(ptr[i + 1], b + chunk), nbig, 0));
        ++nbig;
      }
    }
    if (tasks.size() > L.mtcap || (size_t)nbig > L.nbigcap) return FI_EDEVICE;
    if (hipMemcpyAsync(cptr, ptr.data(), 4 * ptr.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ws + L.mtasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess)
      return FI_EDEVICE;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nanch, B)), dim3(B), 0, s, count, (int64_t)nanch, 0);
    hipLaunchKernelGGL(k_cfill, dim3(grid_for(n, B)), dim3(B), 0, s, G.row_ptr, G.comp, aslot, cptr,
                       n, count, (int32_t*)(ws + L.cverts));
  }
  // every row of 128 minima (two tree words of 64 trees each)
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(128 * (int64_t)L.mhcap, B)), dim3(B), 0, s,
                     (uint64_t*)(ws + L.mhslot), 128 * (int64_t)L.mhcap, kUnvisited);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(128 * (int64_t)L.nbigcap, B)), dim3(B), 0, s,
                     (uint64_t*)(ws + L.rootbig), 128 * (int64_t)L.nbigcap, kUnvisited);
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return FI_EDEVICE;
  g->mtasks = (int32_t)tasks.size();
  g->mnbig = nbig;
  return FI_OK;
}

}  // namespace fi

using namespace fi;

// ============================================================ C ABI

extern "C" {

const char* fi_strerror(int code) {
  switch (code) {
    case FI_OK: return "ok";
    case FI_EINVAL: return "invalid argument or malformed CSR";
    case FI_EASYM: return "CSR is not symmetric (missing reverse entry or sign mismatch)";
    case FI_ESELFLOOP: return "self-loop";
    case FI_EDUP: return "duplicate edge";
    case FI_ESIGN: return "sign not +1/-1";
    case FI_ERANGE: return "size or tree index out of range";
    case FI_EUNSORTED: return "row columns not increasing";
    case FI_ECAPACITY: return "frustration cloud capacity exceeded";
    case FI_EDEVICE: return "HIP runtime error";
    case FI_EDEPTH: return "BFS tree deeper than the level field holds (2^31 - 2 levels)";
    case FI_ECOLLISION: return "state key collision";
    case FI_EWORKSPACE: return "workspace missing, too small or misaligned";
    case FI_EORDER: return "bounded-cloud merge out of tree order";
    default: return "unknown error";
  }
}

int fi_graph_workspace_size(int32_t n, int64_t nnz, int64_t cloud_capacity, size_t* out_bytes) {
  if (!out_bytes || n < 0 || nnz < 0 || cloud_capacity < 0) return FI_EINVAL;
  if (nnz >= ((int64_t)1 << 31)) return FI_ERANGE;
  *out_bytes = make_layout(n, nnz, cloud_capacity, table_size_for(cloud_capacity)).total;
  return FI_OK;
}

#define FI_HIP(call)                              \
  do {                                            \
    if ((call) != hipSuccess) return FI_EDEVICE;  \
  } while (0)

int fi_graph_create(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                    const int8_t* d_sign, int64_t cloud_capacity, void* d_workspace,
                    size_t ws_bytes, void* stream, fi_graph** out) {
  if (!out) return FI_EINVAL;
  *out = nullptr;
  if (n < 0 || nnz < 0 || cloud_capacity < 0) return FI_EINVAL;
  if (nnz >= ((int64_t)1 << 31)) return FI_ERANGE;
  if (!d_row_ptr || (nnz > 0 && (!d_col || !d_sign))) return FI_EINVAL;
  if (nnz % 2) return FI_EASYM;
  const uint64_t tsize = table_size_for(cloud_capacity);
  Layout L = make_layout(n, nnz, cloud_capacity, tsize);
  if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace % kAlign)) return FI_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_workspace;

  fi_graph* g = new (std::nothrow) fi_graph();
  if (!g) return FI_EINVAL;
  g->L = L;
  g->ws = ws;
  g->ws_bytes = ws_bytes;
  g->cloud_capacity = cloud_capacity;
  g->table_size = tsize;
  int dev = 0;
  FI_HIP(hipGetDevice(&dev));
  FI_HIP(hipDeviceGetAttribute(&g->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
  FI_HIP(hipDeviceGetAttribute(&g->max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  g->sched = fi_schedule{0, 256, 0, 512, 4};

  DevGraph& G = g->dg;
  G.n = n;
  G.nwords = (n + 63) / 64;
  G.nnz = nnz;
  G.m = nnz / 2;
  G.row_ptr = (const int32_t*)(ws + L.row_ptr);
  G.adj = (const uint32_t*)(ws + L.adj);
  G.edges = (const uint2*)(ws + L.edges);
  G.cedges = (const uint2*)(ws + L.cedges);
  G.comp = (const int32_t*)(ws + L.comp);
  G.word_comp = (const int32_t*)(ws + L.word_comp);
  G.word_mask = (const uint64_t*)(ws + L.word_mask);
  G.word_main = (const uint64_t*)(ws + L.word_main);
  G.anchors = (const int32_t*)(ws + L.anchors);
  G.cloud = (CloudSlot*)(ws + L.cloud);
  G.cloud_mask = tsize - 1;
  G.cloud_cap = (uint64_t)cloud_capacity;
  G.ctl = (uint64_t*)(ws + L.ctl);

  const int B = 256;
  uint64_t* ctl = G.ctl;
  auto fail = [&](int code) {
    delete g;
    return code;
  };
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(B), 0, s, ctl, (int64_t)C_WORDS, 0ull);
  hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(n, B)), dim3(B), 0, s, d_row_ptr, n, nnz, ctl);
  uint64_t flags = 0;
  if (hipMemcpyAsync(&flags, ctl + C_FLAGS, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FI_EDEVICE);
  if (flags & V_ROWPTR) return fail(FI_EINVAL);
  if (nnz > 0)
    hipLaunchKernelGGL(k_check_entries, dim3(grid_for(nnz, B, 16384)), dim3(B), 0, s, d_row_ptr,
                       d_col, d_sign, n, nnz, ctl);
  if (hipMemcpyAsync(&flags, ctl + C_FLAGS, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FI_EDEVICE);
  if (flags & V_RANGE) return fail(FI_EINVAL);
  if (flags & V_SIGN) return fail(FI_ESIGN);
  if (flags & V_SELF) return fail(FI_ESELFLOOP);
  if (flags & V_DUP) return fail(FI_EDUP);
  if (flags & V_UNSORTED) return fail(FI_EUNSORTED);
  if (flags & V_ASYM) return fail(FI_EASYM);

  // packed adjacency and the upper-triangle edge list
  int32_t* upper_start = (int32_t*)(ws + L.scratch);
  int32_t* edge_off = upper_start + (n + 64);
  int32_t* tile_sums = (int32_t*)(ws + L.tmp);
  hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n + 1, B)), dim3(B), 0, s, d_row_ptr,
                     (int32_t*)G.row_ptr, (int64_t)n + 1);
  if (n > 0) {
    hipLaunchKernelGGL(k_row_upper, dim3(grid_for(n, B)), dim3(B), 0, s, d_row_ptr, d_col, n,
                       upper_start, edge_off);
    int64_t ntiles = ((int64_t)n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, edge_off,
                       (int64_t)n, tile_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, tile_sums, ntiles,
                       tile_sums + ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n, B)), dim3(B), 0, s, edge_off, (int64_t)n,
                       tile_sums);
  }
  if (nnz > 0)
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nnz, B, 16384)), dim3(B), 0, s, d_row_ptr, d_col,
                       d_sign, n, nnz, upper_start, edge_off, (uint32_t*)G.adj, (uint2*)G.edges);
  // the counting edge list (row counts, their scan, then the entries)
  if (nnz > 0) {
    const int gw = grid_for((int64_t)n * 64, B, 16384);
    hipLaunchKernelGGL(k_orient, dim3(gw), dim3(B), 0, s, G.row_ptr, G.adj, n, (const int32_t*)nullptr,
                       edge_off, (uint2*)nullptr);
    int64_t ntiles = ((int64_t)n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, edge_off,
                       (int64_t)n, tile_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, tile_sums, ntiles,
                       tile_sums + ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n, B)), dim3(B), 0, s, edge_off, (int64_t)n,
                       tile_sums);
    hipLaunchKernelGGL(k_orient, dim3(gw), dim3(B), 0, s, G.row_ptr, G.adj, n,
                       (const int32_t*)edge_off, (int32_t*)nullptr, (uint2*)G.cedges);
  }
  // components
  if (n > 0) {
    int32_t* comp = (int32_t*)G.comp;
    hipLaunchKernelGGL(k_uf_init, dim3(grid_for(n, B)), dim3(B), 0, s, comp, n);
    if (G.m > 0)
      hipLaunchKernelGGL(k_uf_hook, dim3(grid_for(G.m, B, 16384)), dim3(B), 0, s, G.edges, G.m, comp);
    hipLaunchKernelGGL(k_uf_compress, dim3(grid_for(n, B)), dim3(B), 0, s, comp, n);
    hipLaunchKernelGGL(k_word_info, dim3(grid_for((int64_t)G.nwords * 64, B)), dim3(B), 0, s,
                       G.row_ptr, G.comp, n, G.nwords, (int32_t*)G.word_comp,
                       (uint64_t*)G.word_mask, (uint64_t*)G.word_main, (int32_t*)G.anchors, ctl);
    const int64_t nroot = (int64_t)L.gpstride * kGridSlots;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nroot, B)), dim3(B), 0, s,
                       (uint64_t*)(ws + L.grootkey), nroot, kUnvisited);
  }
  if (build_components(g, s) != FI_OK) return fail(FI_EDEVICE);
  if (centrality_setup(g, s) != FI_OK) return fail(FI_EDEVICE);
  if (graphl_setup(g, s) != hipSuccess) return fail(FI_EDEVICE);
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(B), 0, s, (uint64_t*)(ws + L.gbar),
                     (int64_t)kGridSlots * kGridBarWords, 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(B), 0, s, (uint64_t*)(ws + L.gctl),
                     (int64_t)kGridSlots * kGridCtlWords, 0ull);
  hipLaunchKernelGGL(k_cloud_reset, dim3(grid_for((int64_t)tsize, B)), dim3(B), 0, s, G.cloud,
                     (int64_t)tsize, ctl);
  uint64_t info[3] = {0, 0, 0};
  if (hipMemcpyAsync(info, ctl + C_NCOMP, 24, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FI_EDEVICE);
  if (hipGetLastError() != hipSuccess) return fail(FI_EDEVICE);
  g->ncomp = (int32_t)info[0];
  g->nisolated = (int32_t)info[1];
  g->nanch = (int32_t)info[2];
  g->prof = false;
  g->prof_ms[0] = g->prof_ms[1] = 0;
  g->prof_n[0] = g->prof_n[1] = 0;
  g->prof_events = new std::vector<ProfEvent>();
  g->plog = nullptr;
  g->pcap = 0;
  g->is_batch = false;
  g->batch = nullptr;
  *out = g;
  return FI_OK;
}

}  // extern "C"

namespace fi {
void* prof_events_new() { return new (std::nothrow) std::vector<ProfEvent>(); }
}  // namespace fi

extern "C" {

void fi_graph_destroy(fi_graph* g) {
  if (!g) return;
  auto* ev = (std::vector<ProfEvent>*)g->prof_events;
  if (ev) {
    for (auto& e : *ev) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    delete ev;
  }
  if (g->batch) batch_info_free(g->batch);
  delete g;
}

int fi_graph_info(fi_graph* g, int32_t* out_components, int32_t* out_isolated) {
  if (!g || g->is_batch) return FI_EINVAL;
  if (out_components) *out_components = g->ncomp;
  if (out_isolated) *out_isolated = g->nisolated;
  return FI_OK;
}

int fi_graph_status(fi_graph* g, void* stream) {
  if (!g) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t bits = 0;
  FI_HIP(hipMemcpyAsync(&bits, g->dg.ctl + C_ERR, 8, hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  return err_from_bits(bits);
}

int fi_min_frustration(fi_graph* g, uint64_t* out_switches, uint64_t* out_first_tree,
                       void* stream) {
  if (!g || g->is_batch) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t w[4];
  FI_HIP(hipMemcpyAsync(w, g->dg.ctl, 32, hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  int e = err_from_bits(w[C_ERR]);
  if (e) return e;
  if (w[C_TREES] == 0) return FI_EINVAL;
  if (out_switches) *out_switches = w[C_BEST] >> 32;
  if (out_first_tree) *out_first_tree = w[C_BEST] & 0xFFFFFFFFull;
  return FI_OK;
}

int fi_cloud_size(fi_graph* g, int64_t* out, void* stream) {
  if (!g || !out || g->is_batch) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t c = 0;
  FI_HIP(hipMemcpyAsync(&c, g->dg.ctl + C_COUNT, 8, hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  *out = (int64_t)c;
  return FI_OK;
}

int fi_cloud_read(fi_graph* g, fi_cloud_entry* h_out, int64_t cap, int64_t* written, void* stream) {
  if (!g || g->is_batch || cap < 0 || (cap > 0 && !h_out)) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t bits = 0;
  FI_HIP(hipMemcpyAsync(&bits, g->dg.ctl + C_ERR, 8, hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  int e = err_from_bits(bits);
  if (e) return e;
  return read_cloud_table(g->dg.cloud, g->table_size, h_out, cap, written, s);
}

int fi_cloud_reset(fi_graph* g, void* stream) {
  if (!g || g->is_batch) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_cloud_reset, dim3(grid_for((int64_t)g->table_size, 256)), dim3(256), 0, s,
                     g->dg.cloud, (int64_t)g->table_size, g->dg.ctl);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_cloud_load(fi_graph* g, const fi_cloud_entry* h_entries, int64_t count, void* stream) {
  if (!g || g->is_batch || count < 0 || (count > 0 && !h_entries)) return FI_EINVAL;
  if (count == 0) return FI_OK;
  hipStream_t s = (hipStream_t)stream;
  // stage through the tree-word scratch, in chunks that fit it
  uint64_t* stage = (uint64_t*)(g->ws + g->L.scratch);
  int64_t per = std::max<int64_t>(1, (int64_t)g->dg.n / 5);
  std::vector<uint64_t> buf;
  for (int64_t c0 = 0; c0 < count; c0 += per) {
    int64_t k = std::min(per, count - c0);
    buf.resize(5 * k);
    for (int64_t i = 0; i < k; ++i) {
      const fi_cloud_entry& e = h_entries[c0 + i];
      buf[5 * i] = e.key_hi; buf[5 * i + 1] = e.key_lo; buf[5 * i + 2] = e.freq;
      buf[5 * i + 3] = e.switches; buf[5 * i + 4] = e.first_tree;
    }
    FI_HIP(hipMemcpyAsync(stage, buf.data(), 8 * buf.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_cloud_load, dim3(grid_for(k, 256)), dim3(256), 0, s, g->dg, stage, k);
    FI_HIP(hipStreamSynchronize(s));
  }
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_count(fi_graph* g, const uint64_t* d_bits, int32_t B, uint64_t* d_counts, void* stream) {
  if (!g || g->is_batch || B < 0 || (B > 0 && (!d_bits || !d_counts))) return FI_EINVAL;
  if (B == 0) return FI_OK;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(B, 256)), dim3(256), 0, s, d_counts, (int64_t)B, 0ull);
  // groups of 64 states: transposed to one word per vertex (4 bytes for up
  // to 32 states, else 8) in the scratch region (8 (n + 64) bytes), then one
  // pass over the edge list per group
  void* st = g->ws + g->L.scratch;
  const int32_t n = g->dg.n;
  for (int32_t b0 = 0; b0 < B && n > 0; b0 += 64) {
    const int nb = std::min<int32_t>(64, B - b0);
    const uint64_t* bits = d_bits + (size_t)b0 * g->dg.nwords;
    if (nb <= 32)
      hipLaunchKernelGGL(k_states_by_vertex<uint32_t>, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s,
                         bits, g->dg.nwords, n, nb, (uint32_t*)st);
    else
      hipLaunchKernelGGL(k_states_by_vertex<uint64_t>, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s,
                         bits, g->dg.nwords, n, nb, (uint64_t*)st);
    hipError_t e = launch_count(g->dg, st, nb, d_counts + b0, s);
    if (e != hipSuccess) return FI_EDEVICE;
  }
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_set_schedule(fi_graph* g, const fi_schedule* sc) {
  if (!g || !sc) return FI_EINVAL;
  if (sc->path < 0 || sc->path > 5 || (g->is_batch && sc->path == 5)) return FI_EINVAL;
  if (sc->block != 256 && sc->block != 512 && sc->block != 1024) return FI_EINVAL;
  if (sc->grid < 0 || sc->heavy < 32 || sc->batch < 1 || sc->batch > kGridSlots) return FI_EINVAL;
  if (sc->grid > 16 * 4096) return FI_EINVAL;
  if (sc->path == 1 && (size_t)g->dg.n * 12 + 32768 > (size_t)g->max_shared) return FI_EINVAL;
  if (sc->path == 2 && g->L.nslots == 0) return FI_EINVAL;
  g->sched = *sc;
  return FI_OK;
}

int fi_get_schedule(fi_graph* g, fi_schedule* out) {
  if (!g || !out) return FI_EINVAL;
  *out = g->sched;
  return FI_OK;
}

int fi_prof_enable(fi_graph* g, int on) {
  if (!g) return FI_EINVAL;
  auto* ev = (std::vector<ProfEvent>*)g->prof_events;
  for (auto& e : *ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  ev->clear();
  g->prof = on != 0;
  g->prof_ms[0] = g->prof_ms[1] = 0;
  g->prof_n[0] = g->prof_n[1] = 0;
  return FI_OK;
}

int fi_prof_phases(fi_graph* g, uint64_t* d_log, int64_t cap) {
  if (!g || g->is_batch || cap < 0 || (d_log && cap < 4)) return FI_EINVAL;
  g->plog = d_log;
  g->pcap = d_log ? cap : 0;
  return FI_OK;
}

int fi_prof_read(fi_graph* g, int kernel, double* out_ms, int64_t* out_launches) {
  if (!g || kernel < 0 || kernel > 1) return FI_EINVAL;
  auto* ev = (std::vector<ProfEvent>*)g->prof_events;
  for (auto& e : *ev) {
    FI_HIP(hipEventSynchronize(e.b));
    float ms = 0;
    FI_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    g->prof_ms[e.kernel] += ms;
    g->prof_n[e.kernel] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  ev->clear();
  if (out_ms) *out_ms = g->prof_ms[kernel];
  if (out_launches) *out_launches = g->prof_n[kernel];
  return FI_OK;
}

}  // extern "C"

namespace fi {

// Events around one launch, when profiling is on.
int prof_begin(fi_graph* g, hipStream_t s, void** token) {
  *token = nullptr;
  if (!g->prof) return 0;
  auto* pe = new ProfEvent();
  if (hipEventCreate(&pe->a) != hipSuccess || hipEventCreate(&pe->b) != hipSuccess) {
    delete pe;
    return -1;
  }
  (void)hipEventRecord(pe->a, s);
  *token = pe;
  return 0;
}

void prof_end(fi_graph* g, hipStream_t s, void* token, int kernel) {
  if (!token) return;
  auto* pe = (ProfEvent*)token;
  pe->kernel = kernel;
  (void)hipEventRecord(pe->b, s);
  ((std::vector<ProfEvent>*)g->prof_events)->push_back(*pe);
  delete pe;
}

hipError_t launch_count(const DevGraph& dg, const void* st, int32_t nstates, uint64_t* counts,
                        hipStream_t s) {
  if (dg.m == 0 || nstates <= 0) return hipSuccess;
  // a few rounds of kCountEdges edges per lane (64M edges: 16 per lane)
  const int gx = grid_for((dg.m + kCountEdges - 1) / kCountEdges, kCountBlock, 4096);
  if (nstates <= 32)
    hipLaunchKernelGGL(k_count<uint32_t>, dim3(gx), dim3(kCountBlock), 0, s, dg.cedges, dg.m,
                       (const uint32_t*)st, (int)nstates, counts);
  else
    hipLaunchKernelGGL(k_count<uint64_t>, dim3(gx), dim3(kCountBlock), 0, s, dg.cedges, dg.m,
                       (const uint64_t*)st, (int)nstates, counts);
  return hipGetLastError();
}

}  // namespace fi
