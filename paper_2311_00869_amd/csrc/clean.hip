// Input cleaning (Section "Implementation": duplicates, inconsistencies,
// self-loops and invalid signs are eliminated) of a raw signed edge list into
// the symmetric sorted CSR that fi_graph_create takes.
//
//   keys     - each entry becomes one 64-bit key min(u,v) << 33 | max(u,v)
//              << 1 | [sign = -1]; invalid entries and self-loops get ~0;
//   sort     - radix sort of the keys (a library primitive);
//   mark     - an entry keeps its pair if it is the pair's first entry and
//              the pair does not occur with both signs (two binary searches
//              in the sorted keys); duplicates and inconsistent pairs are
//              counted;
//   directed - each kept pair emits (u, v) and (v, u) keys, the rest ~0;
//   sort     - the directed keys, rows ascending and columns within rows;
//   csr      - columns and signs from the keys, row offsets by binary search.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <mutex>

#include "fi_internal.h"
#include "fi_prims.h"
#include "frustration.h"

namespace fi {
namespace {

constexpr int kBlock = 256;
constexpr size_t kAlign = 256;

enum : int { CL_INVALID = 0, CL_LOOPS = 1, CL_DUPS = 2, CL_INCONS = 3, CL_KEPT = 4, CL_WORDS = 8 };

struct CleanLayout {
  size_t keys, keys2, dk, dk2, temp, ctl, total;
  size_t temp_bytes;
};

size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int grid_for(int64_t work, int cap = 16384) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + kBlock - 1) / kBlock, cap));
}

bool clean_layout(int64_t E, CleanLayout& L) {
  size_t t1 = 0, t2 = 0;
  uint64_t* nk = nullptr;
  if (rocprim::radix_sort_keys(nullptr, t1, nk, nk, (size_t)std::max<int64_t>(E, 1)) != hipSuccess ||
      rocprim::radix_sort_keys(nullptr, t2, nk, nk, (size_t)std::max<int64_t>(2 * E, 1)) != hipSuccess)
    return false;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t at = off;
    off += al(std::max<size_t>(b, 1));
    return at;
  };
  L.keys = take(8 * (size_t)E);
  L.keys2 = take(8 * (size_t)E);
  L.dk = take(16 * (size_t)E);
  L.dk2 = take(16 * (size_t)E);
  L.temp_bytes = std::max(t1, t2);
  L.temp = take(L.temp_bytes);
  L.ctl = take(8 * CL_WORDS);
  L.total = off;
  return true;
}

__global__ void k_cl_keys(int32_t n, int64_t E, const int32_t* src, const int32_t* dst,
                          const int32_t* sign, uint64_t* keys, uint64_t* ctl) {
  __shared__ uint64_t s_red[kBlock / 64];
  uint64_t bad = 0, loops = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = src[i], v = dst[i], s = sign[i];
    uint64_t k = ~0ull;
    if (u < 0 || u >= n || v < 0 || v >= n || (s != 1 && s != -1)) {
      ++bad;
    } else if (u == v) {
      ++loops;
    } else {
      const uint64_t a = (uint64_t)min(u, v), b = (uint64_t)max(u, v);
      k = a << 33 | b << 1 | (uint64_t)(s < 0);
    }
    keys[i] = k;
  }
  bad = block_sum_u64<kBlock>(bad, s_red);
  loops = block_sum_u64<kBlock>(loops, s_red);
  if (threadIdx.x == 0) {
    if (bad) atomicAdd((unsigned long long*)(ctl + CL_INVALID), (unsigned long long)bad);
    if (loops) atomicAdd((unsigned long long*)(ctl + CL_LOOPS), (unsigned long long)loops);
  }
}

__device__ __forceinline__ bool has_key(const uint64_t* a, int64_t len, uint64_t k) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && a[lo] == k;
}

// Sorted keys: keep the first entry of every pair met with one sign only;
// emit both directions of the kept pairs.
__global__ void k_cl_mark(int64_t E, const uint64_t* keys, uint64_t* dk, uint64_t* ctl) {
  __shared__ uint64_t s_red[kBlock / 64];
  uint64_t dups = 0, incons = 0, kept = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    uint64_t d0 = ~0ull, d1 = ~0ull;
    if (k != ~0ull) {
      const uint64_t pair = k >> 1;
      const bool first = i == 0 || (keys[i - 1] >> 1) != pair;
      const bool both = has_key(keys, E, pair << 1) && has_key(keys, E, pair << 1 | 1);
      if (both) {
        incons += first;
      } else if (first) {
        ++kept;
        const uint64_t a = pair >> 32, b = pair & 0x7FFFFFFFull, neg = k & 1;
        d0 = a << 33 | b << 1 | neg;
        d1 = b << 33 | a << 1 | neg;
      } else {
        ++dups;
      }
    }
    dk[2 * i] = d0;
    dk[2 * i + 1] = d1;
  }
  dups = block_sum_u64<kBlock>(dups, s_red);
  incons = block_sum_u64<kBlock>(incons, s_red);
  kept = block_sum_u64<kBlock>(kept, s_red);
  if (threadIdx.x == 0) {
    if (dups) atomicAdd((unsigned long long*)(ctl + CL_DUPS), (unsigned long long)dups);
    if (incons) atomicAdd((unsigned long long*)(ctl + CL_INCONS), (unsigned long long)incons);
    if (kept) atomicAdd((unsigned long long*)(ctl + CL_KEPT), (unsigned long long)kept);
  }
}

__global__ void k_cl_csr(int32_t n, const uint64_t* dk, const uint64_t* ctl, int32_t* row_ptr,
                         int32_t* col, int8_t* sign) {
  const int64_t nnz = 2 * (int64_t)ctl[CL_KEPT];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = dk[j];
    col[j] = (int32_t)((k >> 1) & 0x7FFFFFFFull);
    sign[j] = (k & 1) ? (int8_t)-1 : (int8_t)1;
  }
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = (uint64_t)r << 33;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (dk[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[r] = (int32_t)lo;
  }
}

__global__ void k_cl_zero(uint64_t* p, int len) {
  if (threadIdx.x < len) p[threadIdx.x] = 0;
}

// The cleaning steps on a workspace laid out by clean_layout(E) at ws
// (256-byte aligned, at least L.total bytes).  Blocks; returns an FI_ code.
int clean_into(int32_t n, int64_t E, const int32_t* d_src, const int32_t* d_dst,
               const int32_t* d_sign, char* ws, const CleanLayout& L, int32_t* d_row_ptr,
               int32_t* d_col, int8_t* d_sign_out, int64_t* h_counts, hipStream_t s) {
  uint64_t* keys = (uint64_t*)(ws + L.keys);
  uint64_t* keys2 = (uint64_t*)(ws + L.keys2);
  uint64_t* dk = (uint64_t*)(ws + L.dk);
  uint64_t* dk2 = (uint64_t*)(ws + L.dk2);
  uint64_t* ctl = (uint64_t*)(ws + L.ctl);
  size_t temp = L.temp_bytes;
  hipLaunchKernelGGL(k_cl_zero, dim3(1), dim3(64), 0, s, ctl, CL_WORDS);
  if (E > 0) {
    hipLaunchKernelGGL(k_cl_keys, dim3(grid_for(E)), dim3(kBlock), 0, s, n, E, d_src, d_dst, d_sign,
                       keys, ctl);
    if (rocprim::radix_sort_keys(ws + L.temp, temp, keys, keys2, (size_t)E, 0, 64, s) != hipSuccess)
      return FI_EDEVICE;
    hipLaunchKernelGGL(k_cl_mark, dim3(grid_for(E)), dim3(kBlock), 0, s, E, keys2, dk, ctl);
    temp = L.temp_bytes;
    if (rocprim::radix_sort_keys(ws + L.temp, temp, dk, dk2, (size_t)(2 * E), 0, 64, s) !=
        hipSuccess)
      return FI_EDEVICE;
  }
  hipLaunchKernelGGL(k_cl_csr, dim3(grid_for(std::max<int64_t>(2 * E, (int64_t)n + 1))),
                     dim3(kBlock), 0, s, n, E > 0 ? dk2 : dk, ctl, d_row_ptr, d_col, d_sign_out);
  if (hipGetLastError() != hipSuccess) return FI_EDEVICE;
  uint64_t c[CL_WORDS];
  if (hipMemcpyAsync(c, ctl, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FI_EDEVICE;
  h_counts[0] = (int64_t)c[CL_KEPT];
  h_counts[1] = (int64_t)c[CL_INVALID];
  h_counts[2] = (int64_t)c[CL_LOOPS];
  h_counts[3] = (int64_t)c[CL_DUPS];
  h_counts[4] = (int64_t)c[CL_INCONS];
  return FI_OK;
}

// ------------------------------------------------------------ no allocation
// Workspace of fi_clean_no_alloc: a file-scope device array, one per GPU,
// held until the process ends.  Host code never passes `scratch` itself to
// a kernel or a copy (on the host that name is not a device address): the
// device address comes from hipGetSymbolAddress, taken once per device.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`, or nullptr if its address is unavailable.
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace fi

using namespace fi;

extern "C" {

int fi_clean_workspace_size(int32_t n, int64_t E, size_t* out_bytes) {
  if (!out_bytes || n < 0 || E < 0) return FI_EINVAL;
  if (2 * E >= ((int64_t)1 << 31)) return FI_ERANGE;
  CleanLayout L;
  if (!clean_layout(E, L)) return FI_EDEVICE;
  *out_bytes = L.total;
  return FI_OK;
}

int fi_clean(int32_t n, int64_t E, const int32_t* d_src, const int32_t* d_dst, const int32_t* d_sign,
             void* d_workspace, size_t ws_bytes, int32_t* d_row_ptr, int32_t* d_col,
             int8_t* d_sign_out, int64_t* h_counts, void* stream) {
  if (n < 0 || E < 0 || !d_row_ptr || !h_counts || (E > 0 && (!d_src || !d_dst || !d_sign ||
                                                               !d_col || !d_sign_out)))
    return FI_EINVAL;
  if (2 * E >= ((int64_t)1 << 31)) return FI_ERANGE;
  CleanLayout L;
  if (!clean_layout(E, L)) return FI_EDEVICE;
  if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace % kAlign)) return FI_EWORKSPACE;
  return clean_into(n, E, d_src, d_dst, d_sign, (char*)d_workspace, L, d_row_ptr, d_col, d_sign_out,
                    h_counts, (hipStream_t)stream);
}

int fi_clean_no_alloc(int32_t n, int64_t E, const int32_t* d_src, const int32_t* d_dst,
                      const int32_t* d_sign, int32_t* d_row_ptr, int32_t* d_col, int8_t* d_sign_out,
                      int64_t* h_counts, void* stream) {
  if (n < 0 || E < 0 || !d_row_ptr || !h_counts || (E > 0 && (!d_src || !d_dst || !d_sign ||
                                                               !d_col || !d_sign_out)))
    return FI_EINVAL;
  if (E > FI_CLEAN_NO_ALLOC_MAX_ENTRIES) return FI_ERANGE;
  CleanLayout L;
  if (!clean_layout(E, L)) return FI_EDEVICE;
  if (L.total > kNoAllocBytes) return FI_ERANGE;
  char* ws = (char*)scratch_on_current_device();
  if (!ws) return FI_EDEVICE;
  return clean_into(n, E, d_src, d_dst, d_sign, ws, L, d_row_ptr, d_col, d_sign_out, h_counts,
                    (hipStream_t)stream);
}

}  // extern "C"
