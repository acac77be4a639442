// Measurement aid, not a step of the method: the gathers of one dense pull
// level of the multi-tree sweep with nothing else around them.  Entry e of
// idx names a 64-byte vertex record; the kernel reads that record's first 32
// bytes as two 16-byte loads (the pull reads the level's tree bits and the
// state bits of every neighbour the same way) and keeps nothing.  Run over a
// graph's adjacency in CSR order, it gives the time the memory system needs
// for one level's neighbour gathers; run over uniform random indices, the
// random-access ceiling of 32-byte reads from a table of that size.
#include <hip/hip_runtime.h>

#include "fi_internal.h"
#include "frustration.h"

namespace fi {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;       // independent gathers in flight per lane
constexpr int64_t kProbeMaxGrid = 8192;

__global__ void __launch_bounds__(kProbeBlock)
    k_probe_gather(const uint32_t* __restrict__ idx, int64_t count, const uint4* __restrict__ rec,
                   uint32_t last, uint32_t* sink) {
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  int64_t e = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  uint32_t acc = 0;
  for (; e + (kProbeUnroll - 1) * stride < count; e += kProbeUnroll * stride) {
    uint32_t u[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) u[k] = min(idx[e + k * stride] & kVertexMask, last);
    uint4 a[kProbeUnroll], b[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) {
      a[k] = rec[(size_t)u[k] * 4];
      b[k] = rec[(size_t)u[k] * 4 + 1];
    }
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) acc ^= a[k].x ^ a[k].w ^ b[k].y ^ b[k].z;
  }
  for (; e < count; e += stride) {
    const uint32_t u = min(idx[e] & kVertexMask, last);
    const uint4 a = rec[(size_t)u * 4], b = rec[(size_t)u * 4 + 1];
    acc ^= a.x ^ a.w ^ b.y ^ b.z;
  }
  // the loads must not be dropped; the store is taken with probability 2^-32
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

}  // namespace
}  // namespace fi

extern "C" {

int fi_probe_gather(const uint32_t* d_idx, int64_t count, const void* d_records, int64_t n_records,
                    uint32_t* d_sink, void* stream) {
  if (count < 0 || n_records < 1 || n_records > ((int64_t)1 << 31) || !d_sink ||
      (count > 0 && (!d_idx || !d_records)))
    return FI_EINVAL;
  if (count == 0) return FI_OK;
  const int64_t blocks = std::min<int64_t>((count + fi::kProbeBlock - 1) / fi::kProbeBlock,
                                           fi::kProbeMaxGrid);
  hipLaunchKernelGGL(fi::k_probe_gather, dim3((unsigned)blocks), dim3(fi::kProbeBlock), 0,
                     (hipStream_t)stream, d_idx, count, (const uint4*)d_records,
                     (uint32_t)(n_records - 1), d_sink);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
