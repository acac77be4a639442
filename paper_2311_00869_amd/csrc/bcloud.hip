// Memory-bound frustration cloud (Alg. alg-scale, appendix "Scaling graphBpp
// for large signed graphs"): at most F_max states, the best ones by (switch
// count S, first tree), each with its count over every tree swept.
//
// A sweep runs in chunks of consecutive trees.  Each chunk is swept into the
// graph's own cloud (the staging table, exact for the chunk), and merged
// here in tree order:
//   gather  - each staged state already held adds its count; the others
//             become candidates (S, first tree of the chunk);
//   sort    - one workgroup sorts the candidates by (S, first) in LDS;
//   merge   - held entries (kept sorted) and candidates take their places in
//             the merged order by binary search; places >= F_max are dropped;
//   index   - the key -> place hash index is rebuilt for the new entries.
// Merging chunk by chunk in tree order gives the result of Alg. alg-scale
// tree by tree: after every chunk the table holds the F_max best distinct
// states seen so far, and a state once dropped is beaten by F_max states
// that stay ahead of it for good, so it can never return; every state held
// at the end was held since its first tree and has its full count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "fi_internal.h"
#include "frustration.h"

namespace fi {
namespace {

struct BEntry {
  uint64_t klo, khi, S, freq, first;
  uint64_t pad[3];
};
struct HSlot {
  uint64_t tag;  // key_lo of the entry, or kEmpty
  uint64_t pos;  // its place in the sorted entries
};

// control words
enum : int { B_NB = 0, B_NC = 1, B_ERR = 2, B_TREES = 3, B_DROP = 4, B_NB2 = 5, B_WORDS = 32 };
enum : uint64_t { BE_COLLISION = 1, BE_ORDER = 2, BE_OVERFLOW = 4, BE_CAPACITY = 8, BE_DEPTH = 16 };

constexpr int kSortMax = 8192;   // candidates per merge (sorted in LDS)
constexpr int kSortBlock = 1024;
constexpr int kBlock = 256;
constexpr size_t kAlign = 256;

struct BLayout {
  size_t e, e2, h, c, c2, ctl, total;
};

uint64_t hash_size_for(int64_t fmax) {
  uint64_t h = 64;
  while (h < 2 * (uint64_t)fmax) h <<= 1;
  return h;
}

BLayout bc_layout(int64_t fmax, int64_t staging, uint64_t hsize) {
  BLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += (bytes + kAlign - 1) / kAlign * kAlign;
    return at;
  };
  L.e = take(sizeof(BEntry) * fmax);
  L.e2 = take(sizeof(BEntry) * fmax);
  L.h = take(sizeof(HSlot) * hsize);
  L.c = take(sizeof(BEntry) * staging);
  L.c2 = take(sizeof(BEntry) * staging);
  L.ctl = take(8 * B_WORDS);
  L.total = off;
  return L;
}

struct BView {
  BEntry* e;
  BEntry* e2;
  HSlot* h;
  BEntry* c;
  BEntry* c2;
  uint64_t* ctl;
  uint64_t hmask;
  int64_t fmax;
  int64_t staging;
};

__device__ __forceinline__ uint64_t rank_of(uint64_t S, uint64_t first) { return (S << 32) | first; }

int grid_for(int64_t work, int block, int cap = 4096) {
  int64_t g = (work + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

__global__ void k_bc_init(BView b, uint64_t hsize) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)hsize;
       i += (int64_t)gridDim.x * blockDim.x)
    b.h[i].tag = kEmpty;
  if (blockIdx.x == 0 && threadIdx.x < B_WORDS) b.ctl[threadIdx.x] = 0;
}

// Staged states of one chunk (trees t0 .. t1-1): count the held ones, list
// the others as candidates.  The staging table's sticky errors carry over.
__global__ void k_bc_gather(const CloudSlot* cloud, uint64_t tsize, const uint64_t* gctl, BView b,
                            uint64_t t0, uint64_t t1) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint64_t ge = gctl[C_ERR], be = 0;
    if (ge & E_CAPACITY) be |= BE_CAPACITY;
    if (ge & E_DEPTH) be |= BE_DEPTH;
    if (ge & E_COLLISION) be |= BE_COLLISION;
    if (be) atomicOr((unsigned long long*)(b.ctl + B_ERR), (unsigned long long)be);
  }
  uint64_t trees = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)tsize;
       i += (int64_t)gridDim.x * blockDim.x) {
    const CloudSlot s = cloud[i];
    if (s.tag == kEmpty) continue;
    trees += s.freq;
    if (s.khi_min != s.khi_max || s.s_min != s.s_max) {
      atomicOr((unsigned long long*)(b.ctl + B_ERR), (unsigned long long)BE_COLLISION);
      continue;
    }
    if (s.first < t0 || s.first >= t1) {
      atomicOr((unsigned long long*)(b.ctl + B_ERR), (unsigned long long)BE_ORDER);
      continue;
    }
    int64_t found = -1;
    uint64_t at = s.tag & b.hmask;
    for (uint64_t probe = 0; probe <= b.hmask; ++probe) {
      const uint64_t tag = b.h[at].tag;
      if (tag == kEmpty) break;
      if (tag == s.tag) {
        found = (int64_t)b.h[at].pos;
        break;
      }
      at = (at + 1) & b.hmask;
    }
    if (found >= 0) {
      // tags are unique within the staging table: one writer per entry
      BEntry* e = b.e + found;
      if (e->khi != s.khi_min || e->S != s.s_min)
        atomicOr((unsigned long long*)(b.ctl + B_ERR), (unsigned long long)BE_COLLISION);
      else
        e->freq += s.freq;
      continue;
    }
    const uint64_t j = atomicAdd((unsigned long long*)(b.ctl + B_NC), 1ull);
    if ((int64_t)j >= b.staging) {
      atomicOr((unsigned long long*)(b.ctl + B_ERR), (unsigned long long)BE_OVERFLOW);
      continue;
    }
    BEntry c{};
    c.klo = s.tag;
    c.khi = s.khi_min;
    c.S = s.s_min;
    c.freq = s.freq;
    c.first = s.first;
    b.c[j] = c;
  }
  if (trees) atomicAdd((unsigned long long*)(b.ctl + B_TREES), (unsigned long long)trees);
}

// One workgroup: bitonic sort of the candidates by (S, first) in LDS.  The
// keys are distinct (a first tree belongs to one state) and S < 2^31, so
// the padding key ~0 sorts after all of them.
__global__ void __launch_bounds__(kSortBlock) k_bc_sort(BView b) {
  __shared__ uint64_t key[kSortMax];
  __shared__ uint16_t idx[kSortMax];
  const int nc = (int)min<uint64_t>(b.ctl[B_NC], (uint64_t)b.staging);
  int P = 1;
  while (P < nc) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    key[i] = i < nc ? rank_of(b.c[i].S, b.c[i].first) : ~0ull;
    idx[i] = (uint16_t)i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = key[i], c = key[l];
          if ((a > c) == up) {
            key[i] = c;
            key[l] = a;
            const uint16_t t = idx[i];
            idx[i] = idx[l];
            idx[l] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int r = threadIdx.x; r < nc; r += blockDim.x) b.c2[r] = b.c[idx[r]];
}

// Number of held entries (sorted, nb of them) whose rank is below r.
__device__ __forceinline__ int64_t held_below(const BEntry* e, int64_t nb, uint64_t r) {
  int64_t lo = 0, hi = nb;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rank_of(e[mid].S, e[mid].first) < r) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merge the held entries and the sorted candidates; keep the first F_max.
__global__ void k_bc_merge(BView b) {
  const int64_t nb = (int64_t)b.ctl[B_NB];
  const int64_t nc = (int64_t)min<uint64_t>(b.ctl[B_NC], (uint64_t)b.staging);
  uint64_t dropped = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb + nc;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t pos;
    const BEntry* src;
    if (i < nb) {
      src = b.e + i;
      pos = i + held_below(b.c2, nc, rank_of(src->S, src->first));
    } else {
      src = b.c2 + (i - nb);
      pos = (i - nb) + held_below(b.e, nb, rank_of(src->S, src->first));
    }
    if (pos < b.fmax) b.e2[pos] = *src;
    else ++dropped;
  }
  if (dropped) atomicAdd((unsigned long long*)(b.ctl + B_DROP), (unsigned long long)dropped);
  if (blockIdx.x == 0 && threadIdx.x == 0) b.ctl[B_NB2] = (uint64_t)min(b.fmax, nb + nc);
}

__global__ void k_bc_clear_copy(BView b, uint64_t hsize) {
  const int64_t nb2 = (int64_t)b.ctl[B_NB2];
  const int64_t n = max((int64_t)hsize, nb2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < (int64_t)hsize) b.h[i].tag = kEmpty;
    if (i < nb2) b.e[i] = b.e2[i];
  }
}

__global__ void k_bc_index(BView b) {
  const int64_t nb2 = (int64_t)b.ctl[B_NB2];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb2;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t tag = b.e[i].klo;
    uint64_t at = tag & b.hmask;
    for (uint64_t probe = 0; probe <= b.hmask; ++probe) {
      const uint64_t old = atomicCAS((unsigned long long*)&b.h[at].tag, (unsigned long long)kEmpty,
                                     (unsigned long long)tag);
      if (old == kEmpty) {
        b.h[at].pos = (uint64_t)i;
        break;
      }
      at = (at + 1) & b.hmask;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.ctl[B_NB] = (uint64_t)nb2;
    b.ctl[B_NC] = 0;
  }
}

int err_from_bcloud(uint64_t bits) {
  if (bits & BE_DEPTH) return FI_EDEPTH;
  if (bits & BE_COLLISION) return FI_ECOLLISION;
  if (bits & BE_ORDER) return FI_EORDER;
  if (bits & (BE_CAPACITY | BE_OVERFLOW)) return FI_ECAPACITY;
  return FI_OK;
}

}  // namespace
}  // namespace fi

using namespace fi;

struct fi_bcloud {
  char* ws;
  size_t ws_bytes;
  int64_t fmax, staging;
  uint64_t hsize;
  BLayout L;
  int64_t next_t;  // first tree of the next merge, -1 before the first
  BView view() const {
    BView b;
    b.e = (BEntry*)(ws + L.e);
    b.e2 = (BEntry*)(ws + L.e2);
    b.h = (HSlot*)(ws + L.h);
    b.c = (BEntry*)(ws + L.c);
    b.c2 = (BEntry*)(ws + L.c2);
    b.ctl = (uint64_t*)(ws + L.ctl);
    b.hmask = hsize - 1;
    b.fmax = fmax;
    b.staging = staging;
    return b;
  }
};

#define FI_HIP(call)                              \
  do {                                            \
    if ((call) != hipSuccess) return FI_EDEVICE;  \
  } while (0)

extern "C" {

int fi_bcloud_workspace_size(int64_t f_max, int64_t staging, size_t* out_bytes) {
  if (!out_bytes || f_max < 1 || f_max > ((int64_t)1 << 31) || staging < 1 || staging > kSortMax)
    return FI_EINVAL;
  *out_bytes = bc_layout(f_max, staging, hash_size_for(f_max)).total;
  return FI_OK;
}

int fi_bcloud_fmax_for(size_t cap_bytes, int64_t staging, int64_t* out_fmax) {
  if (!out_fmax || staging < 1 || staging > kSortMax) return FI_EINVAL;
  if (bc_layout(1, staging, hash_size_for(1)).total > cap_bytes) return FI_EWORKSPACE;
  int64_t lo = 1, hi = (int64_t)1 << 31;
  while (lo < hi) {  // largest F_max whose workspace fits
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (bc_layout(mid, staging, hash_size_for(mid)).total <= cap_bytes) lo = mid;
    else hi = mid - 1;
  }
  *out_fmax = lo;
  return FI_OK;
}

int fi_bcloud_create(int64_t f_max, int64_t staging, void* d_workspace, size_t ws_bytes,
                     void* stream, fi_bcloud** out) {
  if (!out) return FI_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = fi_bcloud_workspace_size(f_max, staging, &need);
  if (rc) return rc;
  if (!d_workspace || ws_bytes < need || ((uintptr_t)d_workspace % kAlign)) return FI_EWORKSPACE;
  fi_bcloud* c = new (std::nothrow) fi_bcloud();
  if (!c) return FI_EINVAL;
  c->ws = (char*)d_workspace;
  c->ws_bytes = ws_bytes;
  c->fmax = f_max;
  c->staging = staging;
  c->hsize = hash_size_for(f_max);
  c->L = bc_layout(f_max, staging, c->hsize);
  c->next_t = -1;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_bc_init, dim3(grid_for((int64_t)c->hsize, kBlock)), dim3(kBlock), 0, s,
                     c->view(), c->hsize);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    delete c;
    return FI_EDEVICE;
  }
  *out = c;
  return FI_OK;
}

void fi_bcloud_destroy(fi_bcloud* c) { delete c; }

int fi_bcloud_reset(fi_bcloud* c, void* stream) {
  if (!c) return FI_EINVAL;
  hipLaunchKernelGGL(k_bc_init, dim3(grid_for((int64_t)c->hsize, kBlock)), dim3(kBlock), 0,
                     (hipStream_t)stream, c->view(), c->hsize);
  c->next_t = -1;
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_bcloud_merge(fi_graph* g, fi_bcloud* c, int64_t t0, int64_t t1, void* stream) {
  if (!g || !c || g->is_batch || t0 < 0 || t1 < t0 || t1 > ((int64_t)1 << 32)) return FI_EINVAL;
  if (g->cloud_capacity > c->staging) return FI_EINVAL;
  if (c->next_t >= 0 && t0 != c->next_t) return FI_EORDER;
  hipStream_t s = (hipStream_t)stream;
  const BView b = c->view();
  hipLaunchKernelGGL(k_bc_gather, dim3(grid_for((int64_t)g->table_size, kBlock)), dim3(kBlock), 0,
                     s, g->dg.cloud, g->table_size, g->dg.ctl, b, (uint64_t)t0, (uint64_t)t1);
  hipLaunchKernelGGL(k_bc_sort, dim3(1), dim3(kSortBlock), 0, s, b);
  hipLaunchKernelGGL(k_bc_merge, dim3(grid_for(c->fmax + c->staging, kBlock)), dim3(kBlock), 0, s,
                     b);
  hipLaunchKernelGGL(k_bc_clear_copy, dim3(grid_for((int64_t)c->hsize, kBlock)), dim3(kBlock), 0,
                     s, b, c->hsize);
  hipLaunchKernelGGL(k_bc_index, dim3(grid_for(c->fmax, kBlock)), dim3(kBlock), 0, s, b);
  if (hipGetLastError() != hipSuccess) return FI_EDEVICE;
  int rc = fi_cloud_reset(g, stream);
  if (rc) return rc;
  c->next_t = t1;
  return FI_OK;
}

int fi_sweep_bounded(fi_graph* g, fi_bcloud* c, int64_t t0, int64_t t1, uint64_t seed,
                     int64_t chunk, void* stream) {
  if (!g || !c || g->is_batch || t0 < 0 || t1 < t0) return FI_EINVAL;
  if (t1 > ((int64_t)1 << 32)) return FI_ERANGE;
  const int64_t most = std::min<int64_t>(g->cloud_capacity, c->staging);
  if (chunk <= 0) chunk = most;
  if (chunk > most || chunk < 1) return FI_EINVAL;
  if (c->next_t >= 0 && t0 != c->next_t) return FI_EORDER;
  int rc = fi_cloud_reset(g, stream);
  if (rc) return rc;
  for (int64_t a = t0; a < t1; a += chunk) {
    const int64_t e = std::min(t1, a + chunk);
    rc = fi_sweep_range(g, a, e, seed, nullptr, stream);
    if (rc) return rc;
    rc = fi_bcloud_merge(g, c, a, e, stream);
    if (rc) return rc;
  }
  return FI_OK;
}

int fi_bcloud_size(fi_bcloud* c, int64_t* out, void* stream) {
  if (!c || !out) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t w[B_WORDS];
  FI_HIP(hipMemcpyAsync(w, c->ws + c->L.ctl, sizeof(w), hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  *out = (int64_t)w[B_NB];
  return err_from_bcloud(w[B_ERR]);
}

int fi_bcloud_stats(fi_bcloud* c, int64_t* out_trees, int64_t* out_dropped, void* stream) {
  if (!c) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t w[B_WORDS];
  FI_HIP(hipMemcpyAsync(w, c->ws + c->L.ctl, sizeof(w), hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  if (out_trees) *out_trees = (int64_t)w[B_TREES];
  if (out_dropped) *out_dropped = (int64_t)w[B_DROP];
  return err_from_bcloud(w[B_ERR]);
}

int fi_bcloud_min(fi_bcloud* c, uint64_t* out_switches, uint64_t* out_first_tree, void* stream) {
  if (!c) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t w[B_WORDS];
  BEntry e0{};
  FI_HIP(hipMemcpyAsync(w, c->ws + c->L.ctl, sizeof(w), hipMemcpyDeviceToHost, s));
  FI_HIP(hipMemcpyAsync(&e0, c->ws + c->L.e, sizeof(e0), hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  int rc = err_from_bcloud(w[B_ERR]);
  if (rc) return rc;
  if (w[B_NB] == 0) return FI_EINVAL;
  if (out_switches) *out_switches = e0.S;
  if (out_first_tree) *out_first_tree = e0.first;
  return FI_OK;
}

int fi_bcloud_read(fi_bcloud* c, fi_cloud_entry* h_out, int64_t cap, int64_t* written,
                   void* stream) {
  if (!c || cap < 0 || (cap > 0 && !h_out)) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t w[B_WORDS];
  FI_HIP(hipMemcpyAsync(w, c->ws + c->L.ctl, sizeof(w), hipMemcpyDeviceToHost, s));
  FI_HIP(hipStreamSynchronize(s));
  int rc = err_from_bcloud(w[B_ERR]);
  if (rc) return rc;
  const int64_t nb = (int64_t)w[B_NB];
  std::vector<BEntry> e(nb);
  if (nb > 0) {
    FI_HIP(hipMemcpyAsync(e.data(), c->ws + c->L.e, sizeof(BEntry) * nb, hipMemcpyDeviceToHost, s));
    FI_HIP(hipStreamSynchronize(s));
  }
  std::vector<fi_cloud_entry> rows;
  rows.reserve(nb);
  for (const BEntry& x : e) rows.push_back(fi_cloud_entry{x.khi, x.klo, x.freq, x.S, x.first});
  std::sort(rows.begin(), rows.end(), [](const fi_cloud_entry& a, const fi_cloud_entry& b) {
    return a.key_hi != b.key_hi ? a.key_hi < b.key_hi : a.key_lo < b.key_lo;
  });
  const int64_t k = std::min<int64_t>(cap, nb);
  if (k > 0) std::memcpy(h_out, rows.data(), sizeof(fi_cloud_entry) * k);
  if (written) *written = nb;
  return FI_OK;
}

}  // extern "C"
