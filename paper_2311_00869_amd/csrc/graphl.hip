// graphL (Section "graphL: optimization formulation"): the relaxed loss of
// Eq. eq-loss_imbalance_new, its gradient, the descent update of
// Alg. alg-gradient and the final rounding plus exact count, for R restarts
// stored as the columns of Gamma[n][R].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {

namespace {

constexpr int kGLBlock = 256;

// lanes per edge / row: the smallest power of two >= R (R <= 64)
__host__ __device__ __forceinline__ int lanes_for(int R) {
  int p = 1;
  while (p < R) p <<= 1;
  return p;
}

// Loss partials: block b, restart r -> part[b * 64 + r].  Edge terms
// (1 - e G_u G_v) / 2 are formed in float32 and accumulated in float64; the
// assignment of edges to threads and the reduction tree are fixed, so the
// result is bit-reproducible.
__global__ void __launch_bounds__(kGLBlock) k_gl_forward(const uint2* edges, int64_t m,
                                                         const float* gamma, int R, double* part) {
  __shared__ double s_acc[kGLBlock];
  const int P = lanes_for(R);
  const int sub = threadIdx.x % P;       // restart handled by this lane
  const int grp = threadIdx.x / P;       // edge slot within the block
  const int gpb = kGLBlock / P;          // edges per block per step
  double acc = 0.0;
  if (sub < R) {
    for (int64_t e = (int64_t)blockIdx.x * gpb + grp; e < m; e += (int64_t)gridDim.x * gpb) {
      const uint2 uv = edges[e];
      const uint32_t v = uv.y & kVertexMask;
      const float sg = (uv.y >> 31) ? -1.0f : 1.0f;
      const float gu = gamma[(size_t)uv.x * R + sub];
      const float gv = gamma[(size_t)v * R + sub];
      const float term = (1.0f - sg * gu * gv) * 0.5f;
      acc += (double)term;
    }
  }
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  // fold the edge slots of each restart: fixed pairwise tree over grp
  for (int stride = gpb / 2; stride > 0; stride >>= 1) {
    if (grp < stride) s_acc[threadIdx.x] += s_acc[threadIdx.x + stride * P];
    __syncthreads();
  }
  if (grp == 0 && sub < R) part[(size_t)blockIdx.x * kGraphLMaxR + sub] = s_acc[threadIdx.x];
}

__global__ void k_gl_forward_final(const double* part, int nblocks, int R, double* loss) {
  const int r = threadIdx.x;
  if (r >= R) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kGraphLMaxR + r];
  loss[r] = s;
}

// Row gather: g[i][r] = -1/2 * w_r * sum over the row of e_ij G[j][r]
// (float32 accumulation along the row, in CSR order).  With `alpha` != 0
// the kernel writes the descent update G - alpha * g instead of g.
__global__ void __launch_bounds__(kGLBlock) k_gl_rows(const int32_t* rp, const uint32_t* adj,
                                                      int32_t n, const float* gamma, int R,
                                                      const double* w, float alpha, int update,
                                                      float* out) {
  const int P = lanes_for(R);
  const int sub = threadIdx.x % P;
  const int grp = threadIdx.x / P;
  const int gpb = kGLBlock / P;
  if (sub >= R) return;
  const float wr = w ? (float)w[sub] : 1.0f;
  for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
    float acc = 0.0f;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const uint32_t a = adj[e];
      const float gj = gamma[(size_t)(a & kVertexMask) * R + sub];
      acc += (a >> 31) ? -gj : gj;
    }
    const float g = -0.5f * acc * wr;
    const size_t o = (size_t)i * R + sub;
    out[o] = update ? gamma[o] - alpha * g : g;
  }
}

// theta = +1 where Gamma >= 0, else -1; bit set = -1.  One wave per
// (64-vertex word, restart).
__global__ void k_gl_round(const float* gamma, int32_t n, int32_t nwords, int R, uint64_t* bits) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t total = (int64_t)nwords * R;
  for (int64_t k = wave; k < total; k += nwaves) {
    const int r = (int)(k / nwords);
    const int64_t i = k - (int64_t)r * nwords;
    const int64_t v = i * 64 + lane;
    bool neg = false;
    if (v < n) neg = !(gamma[(size_t)v * R + r] >= 0.0f);
    const uint64_t W = __ballot(neg);
    if (lane == 0) bits[(size_t)r * nwords + i] = W;
  }
}

__global__ void k_zero_u64(uint64_t* p, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int rows_grid(int32_t n, int R) {
  const int gpb = kGLBlock / lanes_for(R);
  int64_t g = ((int64_t)n + gpb - 1) / gpb;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

}  // namespace fi

using namespace fi;

extern "C" {

int fi_graphl_forward(fi_graph* g, const float* d_gamma, int32_t R, double* d_loss, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || !d_loss || (g->dg.n > 0 && !d_gamma))
    return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)(g->ws + g->L.gl);
  hipLaunchKernelGGL(k_gl_forward, dim3(kGraphLBlocks), dim3(kGLBlock), 0, s, g->dg.edges,
                     g->dg.m, d_gamma, (int)R, part);
  hipLaunchKernelGGL(k_gl_forward_final, dim3(1), dim3(64), 0, s, part, kGraphLBlocks, (int)R,
                     d_loss);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_graphl_backward(fi_graph* g, const float* d_gamma, int32_t R, const double* d_grad_loss,
                       float* d_grad_gamma, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR) return FI_EINVAL;
  if (g->dg.n == 0) return FI_OK;
  if (!d_gamma || !d_grad_gamma) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_gl_rows, dim3(rows_grid(g->dg.n, R)), dim3(kGLBlock), 0, s, g->dg.row_ptr,
                     g->dg.adj, g->dg.n, d_gamma, (int)R, d_grad_loss, 0.0f, 0, d_grad_gamma);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_graphl_step(fi_graph* g, const float* d_gamma_in, int32_t R, float alpha,
                   float* d_gamma_out, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR) return FI_EINVAL;
  if (g->dg.n == 0) return FI_OK;
  if (!d_gamma_in || !d_gamma_out || d_gamma_in == d_gamma_out) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_gl_rows, dim3(rows_grid(g->dg.n, R)), dim3(kGLBlock), 0, s, g->dg.row_ptr,
                     g->dg.adj, g->dg.n, d_gamma_in, (int)R, (const double*)nullptr, alpha, 1,
                     d_gamma_out);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_round_count(fi_graph* g, const float* d_gamma, int32_t R, uint64_t* d_counts,
                   uint64_t* d_bits_out, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || !d_counts) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, d_counts, (int64_t)R);
  if (g->dg.n == 0) return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
  if (!d_gamma) return FI_EINVAL;
  // rounded states go to the caller's buffer, or to the tree-word scratch
  // (R * ceil(n/64) words <= 8n bytes for R <= 64)
  uint64_t* bits = d_bits_out ? d_bits_out : (uint64_t*)(g->ws + g->L.scratch);
  const int64_t waves = (int64_t)g->dg.nwords * R;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((waves * 64 + 255) / 256, 65536));
  hipLaunchKernelGGL(k_gl_round, dim3(grid), dim3(256), 0, s, d_gamma, g->dg.n, g->dg.nwords,
                     (int)R, bits);
  void* tok = nullptr;
  if (prof_begin(g, s, &tok)) return FI_EDEVICE;
  hipError_t e = launch_count(g->dg, bits, R, d_counts, s);
  prof_end(g, s, tok, 1);
  return e == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
