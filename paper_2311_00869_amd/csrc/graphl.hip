// graphL (Section "graphL: optimization formulation"): the relaxed loss of
// Eq. eq-loss_imbalance_new, its gradient, the descent update of
// Alg. alg-gradient and the final rounding plus exact count, for R restarts
// stored as the columns of Gamma[n][R].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

// No multiply-add contraction in this file: every kernel that computes an
// update rounds the same operations the same way, so the fused small-graph
// descent, the per-step kernels and their vector variants agree bit for bit.
#pragma clang fp contract(off)

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

// Row gathers: g[i][r] = -1/2 * w_r * sum over the row of e_ij G[j][r].
// With `update` the kernels write the descent update G - alpha * g instead.
// Rows of up to kGLHeavy entries: one row per group of lanes, float32
// accumulation in CSR order.  Longer rows (power-law hubs): one row per
// workgroup, the groups striding over the row and their partial sums added
// in group order.  Either way every row's summation order is fixed, so the
// result is bit-reproducible.
//
// Overflow policy of the descent (graphs whose hubs make the update grow by
// up to (1 + alpha * lambda_max / 2) per step).  The update never mixes
// connected components, and components grow at very different rates (a hub
// component by many orders of magnitude more than a two-vertex one), so
// each (component, restart) pair keeps its own power-of-two scale: when the
// pair's largest |G| reached 2^shift after the previous step, this step
// reads the pair's entries scaled by 2^-shift and adds shift to its log2
// scale.  Scaling by a power of two is exact in floating point, so each
// component's stored iterates are the plain descent's times 2^-scale, bit
// for bit, unless an entry falls 2^-149 below its own component's largest.
// Vertices without edges never change and keep scale 0.
struct RowArgs {
  const double* w;          // gradient weights per restart, or null (1)
  float alpha;
  int update;
  // descent with scaling (all null for a plain step or gradient)
  const int32_t* comp;      // anchor of each vertex's component
  const int32_t* aslot;     // component slot of each anchor
  const uint32_t* max_in;   // [C][R] float bits of max |G_in|
  uint32_t* max_out;        // [C][R] max |G_out| (atomic max)
  uint32_t* max_clear;      // [C][R] the buffer the step after next fills
  int32_t* exps;            // [C][R] log2 scales
  int64_t ncr;              // C * R
  int32_t main_slot;        // the largest component: its maxima are combined per block
  int shift;                // rescale threshold and step, log2
};

__device__ __forceinline__ float pair_scale(const RowArgs& A, int32_t c, int R, int sub) {
  if (c < 0) return 1.0f;
  const uint32_t thresh = (uint32_t)(127 + A.shift) << 23;  // 2^shift
  return A.max_in[(size_t)c * R + sub] >= thresh ? __uint_as_float((uint32_t)(127 - A.shift) << 23)
                                                 : 1.0f;
}

// After a row's output v of restart `sub`: its component's maximum and, on
// the component's anchor row, the scale.
__device__ __forceinline__ void note_row(const RowArgs& A, int64_t i, int32_t c, int R, int sub,
                                         float sc, float v, float& mx_main) {
  if (c < 0) return;
  const float a = fabsf(v);
  if (c == A.main_slot) mx_main = fmaxf(mx_main, a);
  else atomicMax((unsigned int*)&A.max_out[(size_t)c * R + sub], __float_as_uint(a));
  if (A.comp[i] == i && sc != 1.0f) A.exps[(size_t)c * R + sub] += A.shift;
}

__device__ __forceinline__ void block_max_main(const RowArgs& A, float mx, float* s_mx, int P,
                                               int R, int sub, int grp, int gpb, bool active) {
  s_mx[threadIdx.x] = mx;
  __syncthreads();
  if (grp == 0 && active && A.main_slot >= 0) {
    float m = 0.0f;
    for (int g = 0; g < gpb; ++g) m = fmaxf(m, s_mx[g * P + sub]);
    if (m > 0.0f)
      atomicMax((unsigned int*)&A.max_out[(size_t)A.main_slot * R + sub], __float_as_uint(m));
  }
}

__device__ __forceinline__ int32_t row_slot(const RowArgs& A, int64_t i, int64_t e0, int64_t e1) {
  return e1 > e0 ? A.aslot[A.comp[i]] : -1;
}

// Sum of e_ij * G[j][sub] * sc over entries e0, e0 + step, ... < e1, added
// in that order.  Eight entries are loaded before their gathers so that
// eight gathers are in flight per lane.
__device__ __forceinline__ float row_sum(const uint32_t* adj, int64_t e0, int64_t e1, int step,
                                         const float* gamma, int R, int sub, float sc) {
  float acc = 0.0f;
  int64_t e = e0;
  for (; e + 7 * (int64_t)step < e1; e += 8 * (int64_t)step) {
    uint32_t a[8];
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = adj[e + k * step];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = gamma[(size_t)(a[k] & kVertexMask) * R + sub] * sc;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += (a[k] >> 31) ? -x[k] : x[k];
  }
  for (; e < e1; e += step) {
    const uint32_t a = adj[e];
    const float gj = gamma[(size_t)(a & kVertexMask) * R + sub] * sc;
    acc += (a >> 31) ? -gj : gj;
  }
  return acc;
}

__global__ void __launch_bounds__(kGLBlock) k_gl_rows(const int32_t* rp, const uint32_t* adj,
                                                      int32_t n, const float* gamma, int R,
                                                      RowArgs A, float* out) {
  __shared__ float s_mx[kGLBlock];
  const int P = lanes_for(R);
  const int sub = threadIdx.x % P;
  const int grp = threadIdx.x / P;
  const int gpb = kGLBlock / P;
  const bool active = sub < R;
  const bool scaled = A.max_in != nullptr;
  const float wr = (A.w && active) ? (float)A.w[sub] : 1.0f;
  if (scaled)
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < A.ncr;
         k += (int64_t)gridDim.x * blockDim.x)
      A.max_clear[k] = 0;
  float mx_main = 0.0f;
  if (active) {
    for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
      const int64_t e0 = rp[i], e1 = rp[i + 1];
      if (e1 - e0 > kGLHeavy) continue;
      const int32_t c = scaled ? row_slot(A, i, e0, e1) : -1;
      const float sc = scaled ? pair_scale(A, c, R, sub) : 1.0f;
      const float acc = row_sum(adj, e0, e1, 1, gamma, R, sub, sc);
      const float g = -0.5f * acc * wr;
      const size_t o = (size_t)i * R + sub;
      const float v = A.update ? gamma[o] * sc - A.alpha * g : g;
      out[o] = v;
      if (scaled) note_row(A, i, c, R, sub, sc, v, mx_main);
    }
  }
  if (scaled) block_max_main(A, mx_main, s_mx, P, R, sub, grp, gpb, active);
}

// The same for R divisible by 4: each lane owns four consecutive restarts and
// gathers them as one 16-byte load, so a wave covers 64 / (R / 4) rows per
// load instead of 64 / R and keeps that many more row gathers in flight.
// Every restart's sum runs over the row in the same order as in k_gl_rows,
// so the results are the same bit for bit.
__global__ void __launch_bounds__(kGLBlock) k_gl_rows4(const int32_t* rp, const uint32_t* adj,
                                                       int32_t n, const float* gamma, int R,
                                                       RowArgs A, float* out) {
  __shared__ float s_mx[kGLBlock][4];
  const int RV = R / 4;
  const int P = lanes_for(RV);
  const int sub = threadIdx.x % P;
  const int grp = threadIdx.x / P;
  const int gpb = kGLBlock / P;
  const bool active = sub < RV;
  const bool scaled = A.max_in != nullptr;
  const int r0 = 4 * sub;
  float wr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) wr[k] = (A.w && active) ? (float)A.w[r0 + k] : 1.0f;
  if (scaled)
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < A.ncr;
         k += (int64_t)gridDim.x * blockDim.x)
      A.max_clear[k] = 0;
  float mx_main[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (active) {
    for (int64_t i = (int64_t)blockIdx.x * gpb + grp; i < n; i += (int64_t)gridDim.x * gpb) {
      const int64_t e0 = rp[i], e1 = rp[i + 1];
      if (e1 - e0 > kGLHeavy) continue;
      const int32_t c = scaled ? row_slot(A, i, e0, e1) : -1;
      float sc[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) sc[k] = scaled ? pair_scale(A, c, R, r0 + k) : 1.0f;
      float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      int64_t e = e0;
      for (; e + 7 < e1; e += 8) {
        uint32_t a[8];
        float4 x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = adj[e + j];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          x[j] = *reinterpret_cast<const float4*>(gamma + (size_t)(a[j] & kVertexMask) * R + r0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ng = (a[j] >> 31) != 0;
          const float x0 = x[j].x * sc[0], x1 = x[j].y * sc[1], x2 = x[j].z * sc[2],
                      x3 = x[j].w * sc[3];
          acc[0] += ng ? -x0 : x0;
          acc[1] += ng ? -x1 : x1;
          acc[2] += ng ? -x2 : x2;
          acc[3] += ng ? -x3 : x3;
        }
      }
      for (; e < e1; ++e) {
        const uint32_t a = adj[e];
        const float4 x = *reinterpret_cast<const float4*>(gamma + (size_t)(a & kVertexMask) * R + r0);
        const bool ng = (a >> 31) != 0;
        const float x0 = x.x * sc[0], x1 = x.y * sc[1], x2 = x.z * sc[2], x3 = x.w * sc[3];
        acc[0] += ng ? -x0 : x0;
        acc[1] += ng ? -x1 : x1;
        acc[2] += ng ? -x2 : x2;
        acc[3] += ng ? -x3 : x3;
      }
      const size_t o = (size_t)i * R + r0;
      const float4 self = *reinterpret_cast<const float4*>(gamma + o);
      const float sv[4] = {self.x, self.y, self.z, self.w};
      float v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float g = -0.5f * acc[k] * wr[k];
        v[k] = A.update ? sv[k] * sc[k] - A.alpha * g : g;
      }
      *reinterpret_cast<float4*>(out + o) = make_float4(v[0], v[1], v[2], v[3]);
      if (scaled)
#pragma unroll
        for (int k = 0; k < 4; ++k) note_row(A, i, c, R, r0 + k, sc[k], v[k], mx_main[k]);
    }
  }
  if (scaled) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_mx[threadIdx.x][k] = mx_main[k];
    __syncthreads();
    if (grp == 0 && active && A.main_slot >= 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float m = 0.0f;
        for (int g = 0; g < gpb; ++g) m = fmaxf(m, s_mx[g * P + sub][k]);
        if (m > 0.0f)
          atomicMax((unsigned int*)&A.max_out[(size_t)A.main_slot * R + r0 + k],
                    __float_as_uint(m));
      }
    }
  }
}

// Heavy rows (more than kGLHeavy entries) are cut into items of up to
// kGLChunk entries spread over workgroups.  An item's groups stride over its
// entries and their sums are added in group order into part[item][r]; a row
// then adds its items in order.  Items of one row are consecutive.
__global__ void __launch_bounds__(kGLBlock) k_gl_chunks(const int32_t* rp, const uint32_t* adj,
                                                        const int32_t* list, const int2* items,
                                                        const uint32_t* ctl, const float* gamma,
                                                        int R, RowArgs A, float* part) {
  __shared__ float s_part[kGLBlock];
  const int P = lanes_for(R);
  const int sub = threadIdx.x % P;
  const int grp = threadIdx.x / P;
  const int gpb = kGLBlock / P;
  const bool active = sub < R;
  const bool scaled = A.max_in != nullptr;
  const uint32_t nitems = ctl[1];
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 hc = items[it];
    const int64_t i = list[hc.x];
    const int64_t r0 = rp[i], r1 = rp[i + 1];
    const int64_t e0 = r0 + (int64_t)hc.y * kGLChunk;
    const int64_t e1 = min(r1, e0 + kGLChunk);
    float acc = 0.0f;
    if (active) {
      const int32_t c = scaled ? row_slot(A, i, r0, r1) : -1;
      const float sc = scaled ? pair_scale(A, c, R, sub) : 1.0f;
      acc = row_sum(adj, e0 + grp, e1, gpb, gamma, R, sub, sc);
    }
    s_part[threadIdx.x] = acc;
    __syncthreads();
    if (grp == 0 && active) {
      float tot = 0.0f;
      for (int g = 0; g < gpb; ++g) tot += s_part[g * P + sub];
      part[(size_t)it * kGraphLMaxR + sub] = tot;
    }
    __syncthreads();
  }
}

// One group of lanes per heavy row: its items in order, then the update.
__global__ void __launch_bounds__(kGLBlock) k_gl_combine(const int32_t* rp, const int32_t* list,
                                                         const int32_t* first, const uint32_t* ctl,
                                                         const float* part, const float* gamma,
                                                         int R, RowArgs A, float* out) {
  __shared__ float s_mx[kGLBlock];
  const int P = lanes_for(R);
  const int sub = threadIdx.x % P;
  const int grp = threadIdx.x / P;
  const int gpb = kGLBlock / P;
  const bool active = sub < R;
  const bool scaled = A.max_in != nullptr;
  const float wr = (A.w && active) ? (float)A.w[sub] : 1.0f;
  const uint32_t cnt = ctl[0];
  float mx_main = 0.0f;
  if (active) {
    for (int64_t h = (int64_t)blockIdx.x * gpb + grp; h < cnt; h += (int64_t)gridDim.x * gpb) {
      const int64_t i = list[h];
      const int32_t c = scaled ? row_slot(A, i, rp[i], rp[i + 1]) : -1;
      const float sc = scaled ? pair_scale(A, c, R, sub) : 1.0f;
      float tot = 0.0f;
      for (int32_t it = first[h]; it < first[h + 1]; ++it) tot += part[(size_t)it * kGraphLMaxR + sub];
      const float g = -0.5f * tot * wr;
      const size_t o = (size_t)i * R + sub;
      const float v = A.update ? gamma[o] * sc - A.alpha * g : g;
      out[o] = v;
      if (scaled) note_row(A, i, c, R, sub, sc, v, mx_main);
    }
  }
  if (scaled) block_max_main(A, mx_main, s_mx, P, R, sub, grp, gpb, active);
}

// Items of the heavy rows (one workgroup): first[h] = the first item of
// heavy row h, first[count] = ctl[1] = the number of items.
__global__ void __launch_bounds__(1024) k_gl_plan(const int32_t* rp, const int32_t* list,
                                                  uint32_t* ctl, int32_t* first, int2* items) {
  __shared__ int s_scan[1024 / 64 + 1];
  const int64_t cnt = ctl[0];
  const int64_t per = (cnt + 1023) / 1024;
  const int64_t h0 = (int64_t)threadIdx.x * per, h1 = min(cnt, h0 + per);
  int mine = 0;
  for (int64_t h = h0; h < h1; ++h) {
    const int64_t i = list[h];
    mine += (int)((rp[i + 1] - rp[i] + kGLChunk - 1) / kGLChunk);
  }
  int total = 0;
  int at = block_exclusive_scan<1024>(mine, total, s_scan);
  for (int64_t h = h0; h < h1; ++h) {
    const int64_t i = list[h];
    const int nch = (int)((rp[i + 1] - rp[i] + kGLChunk - 1) / kGLChunk);
    first[h] = at;
    for (int c = 0; c < nch; ++c) items[at + c] = make_int2((int)h, c);
    at += nch;
  }
  if (threadIdx.x == 0) {
    first[cnt] = total;
    ctl[1] = (uint32_t)total;
  }
}

// The whole descent on a small graph without long rows: one workgroup per
// restart, Gamma's column in LDS (ping-pong), and the per-component maxima
// and scales of the overflow policy in LDS too, so the steps run with no
// launch between them.  Same rows, same order, same operations as the
// per-step kernels.  LDS: 8n (Gamma) + 4n (component slots) + 16 C bytes,
// plus the CSR itself (4(n+1) + 4 nnz) when it fits, so that a step touches
// no global memory.
constexpr int kSmallDescentN = 4096;
constexpr int kSmallRows = kSmallDescentN / 1024;  // rows per thread of the fused descent
constexpr int kHeldEntries = 8;  // leading entries of each row kept in registers
constexpr size_t kSmallDescentLds = 128 * 1024;

template <bool CSR_IN_LDS>
__global__ void __launch_bounds__(1024) k_gl_descend_small(const int32_t* rp_g,
                                                           const uint32_t* adj_g,
                                                           const int32_t* comp,
                                                           const int32_t* aslot, int32_t n,
                                                           int32_t ncomp, int R, float alpha,
                                                           int64_t steps, int shift, float* gamma,
                                                           int32_t* exps) {
  extern __shared__ uint32_t sm[];
  float* G0 = (float*)sm;
  float* G1 = G0 + n;
  int32_t* cs = (int32_t*)(G1 + n);
  uint32_t* mx = (uint32_t*)(cs + n);  // [3][ncomp]
  int32_t* ex = (int32_t*)(mx + 3 * ncomp);
  const int32_t* rp = rp_g;
  const uint32_t* adj = adj_g;
  if (CSR_IN_LDS) {
    int32_t* rp_l = ex + ncomp;
    uint32_t* adj_l = (uint32_t*)(rp_l + n + 1);
    const int32_t nnz = rp_g[n];
    for (int32_t i = threadIdx.x; i <= n; i += blockDim.x) rp_l[i] = rp_g[i];
    for (int32_t e = threadIdx.x; e < nnz; e += blockDim.x) adj_l[e] = adj_g[e];
    rp = rp_l;
    adj = adj_l;
    __syncthreads();
  }
  const int r = blockIdx.x;
  const uint32_t thresh = (uint32_t)(127 + shift) << 23;
  const float down = __uint_as_float((uint32_t)(127 - shift) << 23);
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    G0[i] = gamma[(size_t)i * R + r];
    cs[i] = rp[i + 1] > rp[i] ? aslot[comp[i]] : -1;
  }
  for (int32_t c = threadIdx.x; c < 3 * ncomp; c += blockDim.x) mx[c] = 0;
  for (int32_t c = threadIdx.x; c < ncomp; c += blockDim.x) ex[c] = 0;
  __syncthreads();
  float* gin = G0;
  float* gout = G1;
  // each thread's rows (at most kSmallRows of them, n <= kSmallRows * 1024)
  // keep their bounds, component slot and anchor flag in registers
  // and the first kHeldEntries entries of each row
  int32_t rb[kSmallRows], re[kSmallRows], rc[kSmallRows];
  bool ra[kSmallRows];
  uint32_t held[kSmallRows][kHeldEntries];
#pragma unroll
  for (int q = 0; q < kSmallRows; ++q) {
    const int32_t i = q * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    const bool in = i < n;
    rb[q] = in ? rp[i] : 0;
    re[q] = in ? rp[i + 1] : 0;
    rc[q] = in ? cs[i] : -1;
    ra[q] = in && comp[i] == i;
#pragma unroll
    for (int t = 0; t < kHeldEntries; ++t) held[q][t] = rb[q] + t < re[q] ? adj[rb[q] + t] : 0u;
  }
  int k3 = 0;  // step mod 3: which maxima buffer is read, written, cleared
  for (int64_t k = 0; k < steps; ++k) {
    const uint32_t* min_ = mx + k3 * ncomp;
    uint32_t* mout = mx + (k3 == 2 ? 0 : k3 + 1) * ncomp;
    uint32_t* mclr = mx + (k3 == 0 ? 2 : k3 - 1) * ncomp;
#pragma unroll
    for (int q = 0; q < kSmallRows; ++q) {
      if (q * (int32_t)blockDim.x >= n) break;
      const int32_t i = q * (int32_t)blockDim.x + (int32_t)threadIdx.x;
      const int32_t c = rc[q];
      float v = 0.0f;
      if (i < n) {
        const float sc = (c >= 0 && min_[c] >= thresh) ? down : 1.0f;
        float acc = 0.0f;
        // the held entries' loads all in flight, then four at a time; the
        // sum keeps the row's order
        const int32_t e1 = re[q];
        float xh[kHeldEntries];
#pragma unroll
        for (int t = 0; t < kHeldEntries; ++t) xh[t] = gin[held[q][t] & kVertexMask];
#pragma unroll
        for (int t = 0; t < kHeldEntries; ++t) {
          if (rb[q] + t < e1) {
            const float gt = xh[t] * sc;
            acc += (held[q][t] >> 31) ? -gt : gt;
          }
        }
        int32_t e = rb[q] + kHeldEntries;
        for (; e + 3 < e1; e += 4) {
          const uint32_t a0 = adj[e], a1 = adj[e + 1], a2 = adj[e + 2], a3 = adj[e + 3];
          const float x0 = gin[a0 & kVertexMask], x1 = gin[a1 & kVertexMask];
          const float x2 = gin[a2 & kVertexMask], x3 = gin[a3 & kVertexMask];
          const float g0 = x0 * sc, g1 = x1 * sc, g2 = x2 * sc, g3 = x3 * sc;
          acc += (a0 >> 31) ? -g0 : g0;
          acc += (a1 >> 31) ? -g1 : g1;
          acc += (a2 >> 31) ? -g2 : g2;
          acc += (a3 >> 31) ? -g3 : g3;
        }
        for (; e < e1; ++e) {
          const uint32_t a = adj[e];
          const float gj = gin[a & kVertexMask] * sc;
          acc += (a >> 31) ? -gj : gj;
        }
        const float g = -0.5f * acc * 1.0f;
        v = gin[i] * sc - alpha * g;
        gout[i] = v;
        if (sc != 1.0f && ra[q]) ex[c] += shift;
      }
      // the component maxima: one atomic per wave when its lanes share one
      // component (the maximum does not depend on the order)
      uint32_t m = c >= 0 ? __float_as_uint(fabsf(v)) : 0u;
      const int32_t c0 = __builtin_amdgcn_readfirstlane(c);
      if (__ballot(c != c0) == 0) {
        m = wave_max_u32(m);
        if (c0 >= 0 && (threadIdx.x & 63) == 0) atomicMax(mout + c0, m);
      } else if (c >= 0) {
        atomicMax(mout + c, m);
      }
    }
    k3 = k3 == 2 ? 0 : k3 + 1;
    for (int32_t c = threadIdx.x; c < ncomp; c += blockDim.x) mclr[c] = 0;
    __syncthreads();
    float* t = gin;
    gin = gout;
    gout = t;
  }
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) gamma[(size_t)i * R + r] = gin[i];
  for (int32_t c = threadIdx.x; c < ncomp; c += blockDim.x) exps[(size_t)c * R + r] = ex[c];
}

// Per-vertex log2 scales of a descent: out[i][r] = the scale of (component
// of i, r), 0 for vertices without edges.
__global__ void k_gl_scales(const int32_t* rp, const int32_t* comp, const int32_t* aslot,
                            int32_t n, const int32_t* exps, int R, int32_t* out) {
  const int64_t total = (int64_t)n * R;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / R;
    const int r = (int)(k - i * R);
    out[k] = rp[i + 1] > rp[i] ? exps[(size_t)aslot[comp[i]] * R + r] : 0;
  }
}

// Rows longer than kGLHeavy, in any order (each is summed on its own).
__global__ void k_gl_heavy_list(const int32_t* rp, int32_t n, int32_t* list, uint32_t* count) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = b + threadIdx.x;
    const bool heavy = i < n && rp[i + 1] - rp[i] > kGLHeavy;
    wave_append(heavy, (int32_t)i, list, count);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t len, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// theta = +1 where Gamma >= 0, else -1 (NaN: -1), as one word per vertex:
// bit r of st[v] is set when restart r rounds v to -1 (T: uint32_t for up to
// 32 restarts, else uint64_t).  When R divides 64 a wave reads 64
// consecutive floats of Gamma (64 / R whole vertices) and one ballot gives
// all their words, so Gamma streams through once, coalesced; otherwise each
// thread reads its own vertex's R floats.
template <typename T>
__global__ void k_gl_round(const float* gamma, int32_t n, int R, T* st) {
  const int lane = lane_id();
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  if (64 % R == 0) {
    const int64_t total = (int64_t)n * R;
    const int per = 64 / R;
    const uint64_t rmask = R == 64 ? ~0ull : ((1ull << R) - 1);
    // wave-uniform chunks of 64 elements (vertex-major, restart-minor)
    for (int64_t e0 = (tid >> 6) << 6; e0 < total; e0 += (nthr >> 6) << 6) {
      const int64_t e = e0 + lane;
      const bool neg = e < total && !(gamma[e] >= 0.0f);
      const uint64_t W = __ballot(neg);
      const int64_t v = e0 / R + lane;
      if (lane < per && v < n) st[v] = (T)((W >> (lane * R)) & rmask);
    }
  } else {
    for (int64_t v = tid; v < n; v += nthr) {
      uint64_t w = 0;
      for (int r = 0; r < R; ++r) w |= (uint64_t)!(gamma[(size_t)v * R + r] >= 0.0f) << r;
      st[v] = (T)w;
    }
  }
}

// Bit i of the low 16 bits of x moved to bit 4 i.
__device__ __forceinline__ uint64_t spread4(uint64_t x) {
  x &= 0xFFFFull;
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

// The same rounding for R a multiple of 4 that divides 64, Gamma 16-byte
// aligned: lane l of a wave reads floats 4 l .. 4 l + 3 of a 256-float chunk
// (256 / R whole vertices, R / 4 lanes each), one ballot per float of the
// four gives (vertex, restart) bits, and lane j < 256 / R interleaves vertex
// j's bits from them into its word.  Each wave takes two chunks per step, so
// two 16-byte loads per lane are in flight.
template <typename T>
__global__ void k_gl_round4(const float4* gamma4, int32_t n, int R, T* st) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t total4 = (int64_t)n * R / 4;
  const int q = R / 4;       // lanes per vertex
  const int per = 64 / q;    // vertices per chunk
  const uint64_t qmask = q == 16 ? 0xFFFFull : ((1ull << q) - 1);
  for (int64_t c0 = wave * 128; c0 < total4; c0 += nwaves * 128) {
    float4 x[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = c0 + 64 * h + lane;
      x[h] = i < total4 ? gamma4[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t b0 = __ballot(!(x[h].x >= 0.0f)), b1 = __ballot(!(x[h].y >= 0.0f));
      const uint64_t b2 = __ballot(!(x[h].z >= 0.0f)), b3 = __ballot(!(x[h].w >= 0.0f));
      const int64_t v = (c0 + 64 * h) / q + lane;
      if (lane < per && v < n) {
        const int sh = lane * q;
        const uint64_t w = spread4((b0 >> sh) & qmask) | (spread4((b1 >> sh) & qmask) << 1) |
                           (spread4((b2 >> sh) & qmask) << 2) | (spread4((b3 >> sh) & qmask) << 3);
        st[v] = (T)w;
      }
    }
  }
}

// The rounded states as bitmaps, restart by restart: bits[r * nwords + i],
// vertex v is bit v % 64 of word v / 64 (set = -1).  One wave per word: each
// lane reads its vertex's word once, R ballots transpose the 64 x R bits.
template <typename T>
__global__ void k_gl_unpack(const T* st, int32_t n, int32_t nwords, int R, uint64_t* bits) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < nwords; i += nwaves) {
    const int64_t v = i * 64 + lane;
    const uint64_t x = v < n ? (uint64_t)st[v] : 0ull;
    uint64_t mine = 0;
    for (int r = 0; r < R; ++r) {
      const uint64_t W = __ballot((x >> r) & 1);
      if (lane == r) mine = W;
    }
    if (lane < R) bits[(size_t)lane * nwords + i] = mine;
  }
}

__global__ void k_zero_u64(uint64_t* p, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

int grid_for_gl(int64_t work, int block) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + block - 1) / block, 65536));
}

int rows_grid(int32_t n, int R) {
  const int gpb = kGLBlock / lanes_for(R);
  int64_t g = ((int64_t)n + gpb - 1) / gpb;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// graphL control words in the workspace: heavy rows, their items
uint32_t* gl_ctl(fi_graph* g) { return (uint32_t*)(g->ws + g->L.glctl); }

// Descent scales in the caller's buffer: exponents, then three max buffers,
// each [C][R] 32-bit words (C = components with an edge, at least 1).
size_t aux_part(const fi_graph* g, int R) {
  const size_t c = (size_t)std::max<int32_t>(g->nanch, 1);
  return (4 * c * (size_t)R + 255) / 256 * 256;
}

hipError_t launch_rows(fi_graph* g, const float* gin, int R, const RowArgs& A, float* out,
                       hipStream_t s) {
  const Layout& L = g->L;
  int32_t* list = (int32_t*)(g->ws + L.glheavy);
  int32_t* first = (int32_t*)(g->ws + L.glfirst);
  int2* items = (int2*)(g->ws + L.glitems);
  float* part = (float*)(g->ws + L.glpart);
  uint32_t* ctl = gl_ctl(g);
  if (R % 4 == 0 && (uintptr_t)gin % 16 == 0 && (uintptr_t)out % 16 == 0)
    hipLaunchKernelGGL(k_gl_rows4, dim3(rows_grid(g->dg.n, R / 4)), dim3(kGLBlock), 0, s,
                       g->dg.row_ptr, g->dg.adj, g->dg.n, gin, R, A, out);
  else
    hipLaunchKernelGGL(k_gl_rows, dim3(rows_grid(g->dg.n, R)), dim3(kGLBlock), 0, s,
                       g->dg.row_ptr, g->dg.adj, g->dg.n, gin, R, A, out);
  if (g->gl_nheavy == 0) return hipGetLastError();
  const int cgrid = (int)std::min<int64_t>((int64_t)L.glicap, 8192);
  hipLaunchKernelGGL(k_gl_chunks, dim3(cgrid), dim3(kGLBlock), 0, s, g->dg.row_ptr, g->dg.adj, list,
                     items, ctl, gin, R, A, part);
  const int64_t hcap = g->dg.nnz / kGLHeavy + 1;
  const int hgrid = (int)std::max<int64_t>(1, std::min<int64_t>(hcap / (kGLBlock / lanes_for(R)) + 1,
                                                                4096));
  hipLaunchKernelGGL(k_gl_combine, dim3(hgrid), dim3(kGLBlock), 0, s, g->dg.row_ptr, list, first,
                     ctl, part, gin, R, A, out);
  return hipGetLastError();
}

}  // namespace

// At graph upload: the rows longer than kGLHeavy and their items (blocks).
hipError_t graphl_setup(fi_graph* g, hipStream_t s) {
  const Layout& L = g->L;
  int32_t* list = (int32_t*)(g->ws + L.glheavy);
  int32_t* first = (int32_t*)(g->ws + L.glfirst);
  int2* items = (int2*)(g->ws + L.glitems);
  uint32_t* ctl = gl_ctl(g);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ctl, (int64_t)2, 0u);
  if (g->dg.n > 0) {
    const int grid =
        (int)std::max<int64_t>(1, std::min<int64_t>(((int64_t)g->dg.n + 255) / 256, 16384));
    hipLaunchKernelGGL(k_gl_heavy_list, dim3(grid), dim3(256), 0, s, g->dg.row_ptr, g->dg.n, list,
                       ctl);
    hipLaunchKernelGGL(k_gl_plan, dim3(1), dim3(1024), 0, s, g->dg.row_ptr, list, ctl, first, items);
  }
  uint32_t cnt[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(cnt, ctl, sizeof(cnt), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  g->gl_nheavy = (int32_t)cnt[0];
  return e == hipSuccess ? hipGetLastError() : e;
}

}  // namespace fi

using namespace fi;

#define FI_HIP(call)                              \
  do {                                            \
    if ((call) != hipSuccess) return FI_EDEVICE;  \
  } while (0)

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
  RowArgs A{};
  A.w = d_grad_loss;
  A.update = 0;
  return launch_rows(g, d_gamma, R, A, d_grad_gamma, (hipStream_t)stream) == hipSuccess ? FI_OK
                                                                                        : FI_EDEVICE;
}

int fi_graphl_step(fi_graph* g, const float* d_gamma_in, int32_t R, float alpha,
                   float* d_gamma_out, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR) return FI_EINVAL;
  if (g->dg.n == 0) return FI_OK;
  if (!d_gamma_in || !d_gamma_out || d_gamma_in == d_gamma_out) return FI_EINVAL;
  RowArgs A{};
  A.alpha = alpha;
  A.update = 1;
  return launch_rows(g, d_gamma_in, R, A, d_gamma_out, (hipStream_t)stream) == hipSuccess
             ? FI_OK
             : FI_EDEVICE;
}

int fi_graphl_aux_size(fi_graph* g, int32_t R, size_t* out_bytes) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || !out_bytes) return FI_EINVAL;
  *out_bytes = 4 * aux_part(g, R);
  return FI_OK;
}

int fi_graphl_descend(fi_graph* g, float* d_gamma, float* d_work, int32_t R, float alpha,
                      int64_t steps, int32_t rescale_log2, void* d_aux, size_t aux_bytes,
                      void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || steps < 0) return FI_EINVAL;
  if (rescale_log2 == 0) rescale_log2 = 64;
  if (rescale_log2 < 1 || rescale_log2 > 100) return FI_EINVAL;
  const size_t part = aux_part(g, R);
  if (!d_aux || aux_bytes < 4 * part || ((uintptr_t)d_aux % 256)) return FI_EWORKSPACE;
  if (g->dg.n > 0 && (!d_gamma || !d_work || d_gamma == d_work)) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* aux = (char*)d_aux;
  // exponents and all three max buffers start at zero
  hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, s, (uint32_t*)aux,
                     (int64_t)(part), 0u);
  if (g->dg.n == 0 || steps == 0) return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
  const int32_t ncomp = std::max<int32_t>(g->nanch, 1);
  const size_t lds = 12 * (size_t)g->dg.n + 16 * (size_t)ncomp;
  const size_t lds_csr = lds + 4 * ((size_t)g->dg.n + 1) + 4 * (size_t)g->dg.nnz;
  if (g->dg.n <= kSmallDescentN && g->gl_nheavy == 0 && lds <= kSmallDescentLds) {
    const int32_t* aslot = (const int32_t*)(g->ws + g->L.aslot);
    if (lds_csr <= kSmallDescentLds) {
      FI_HIP(hipFuncSetAttribute((const void*)k_gl_descend_small<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_csr));
      hipLaunchKernelGGL(k_gl_descend_small<true>, dim3(R), dim3(1024), lds_csr, s, g->dg.row_ptr,
                         g->dg.adj, g->dg.comp, aslot, g->dg.n, ncomp, (int)R, alpha, steps,
                         (int)rescale_log2, d_gamma, (int32_t*)aux);
    } else {
      FI_HIP(hipFuncSetAttribute((const void*)k_gl_descend_small<false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(k_gl_descend_small<false>, dim3(R), dim3(1024), lds, s, g->dg.row_ptr,
                         g->dg.adj, g->dg.comp, aslot, g->dg.n, ncomp, (int)R, alpha, steps,
                         (int)rescale_log2, d_gamma, (int32_t*)aux);
    }
    return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
  }
  float* buf[2] = {d_gamma, d_work};
  for (int64_t k = 0; k < steps; ++k) {
    RowArgs A{};
    A.alpha = alpha;
    A.update = 1;
    A.comp = g->dg.comp;
    A.aslot = (const int32_t*)(g->ws + g->L.aslot);
    A.exps = (int32_t*)aux;
    A.max_in = (const uint32_t*)(aux + (1 + k % 3) * part);
    A.max_out = (uint32_t*)(aux + (1 + (k + 1) % 3) * part);
    A.max_clear = (uint32_t*)(aux + (1 + (k + 2) % 3) * part);
    A.ncr = (int64_t)std::max<int32_t>(g->nanch, 1) * R;
    A.main_slot = g->gl_main_slot;
    A.shift = rescale_log2;
    if (launch_rows(g, buf[k & 1], R, A, buf[(k + 1) & 1], s) != hipSuccess) return FI_EDEVICE;
  }
  if (steps & 1)
    FI_HIP(hipMemcpyAsync(d_gamma, d_work, sizeof(float) * (size_t)g->dg.n * R,
                          hipMemcpyDeviceToDevice, s));
  return FI_OK;
}

int fi_graphl_scales(fi_graph* g, const void* d_aux, int32_t R, int32_t* d_out, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || !d_aux || (g->dg.n > 0 && !d_out))
    return FI_EINVAL;
  if (g->dg.n == 0) return FI_OK;
  const int64_t total = (int64_t)g->dg.n * R;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(k_gl_scales, dim3(grid), dim3(256), 0, (hipStream_t)stream, g->dg.row_ptr,
                     g->dg.comp, (const int32_t*)(g->ws + g->L.aslot), g->dg.n,
                     (const int32_t*)d_aux, (int)R, d_out);
  return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
}

int fi_round_count(fi_graph* g, const float* d_gamma, int32_t R, uint64_t* d_counts,
                   uint64_t* d_bits_out, void* stream) {
  if (!g || g->is_batch || R < 1 || R > kGraphLMaxR || !d_counts) return FI_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, d_counts, (int64_t)R);
  if (g->dg.n == 0) return hipGetLastError() == hipSuccess ? FI_OK : FI_EDEVICE;
  if (!d_gamma) return FI_EINVAL;
  void* tok = nullptr;
  if (prof_begin(g, s, &tok)) return FI_EDEVICE;
  // rounded states, one word per vertex (4 bytes for up to 32 restarts, else
  // 8), in the scratch region (8 (n + 64) bytes)
  void* st = g->ws + g->L.scratch;
  const int64_t work = 64 % R == 0 ? (int64_t)g->dg.n * R : (int64_t)g->dg.n;
  const int ugrid = (int)std::max<int64_t>(1, std::min<int64_t>((g->dg.nwords + 3) / 4, 65536));
  // 16-byte reads when each vertex's R floats fill whole float4s
  const bool wide = R % 4 == 0 && 64 % R == 0 && ((uintptr_t)d_gamma & 15) == 0;
  const int wgrid = grid_for_gl(((int64_t)g->dg.n * R / 4 + 127) / 128 * 64, 256);
  if (R <= 32) {
    if (wide)
      hipLaunchKernelGGL(k_gl_round4<uint32_t>, dim3(wgrid), dim3(256), 0, s, (const float4*)d_gamma,
                         g->dg.n, (int)R, (uint32_t*)st);
    else
      hipLaunchKernelGGL(k_gl_round<uint32_t>, dim3(grid_for_gl(work, 256)), dim3(256), 0, s, d_gamma,
                         g->dg.n, (int)R, (uint32_t*)st);
    if (d_bits_out)
      hipLaunchKernelGGL(k_gl_unpack<uint32_t>, dim3(ugrid), dim3(256), 0, s, (const uint32_t*)st,
                         g->dg.n, g->dg.nwords, (int)R, d_bits_out);
  } else {
    if (wide)
      hipLaunchKernelGGL(k_gl_round4<uint64_t>, dim3(wgrid), dim3(256), 0, s, (const float4*)d_gamma,
                         g->dg.n, (int)R, (uint64_t*)st);
    else
      hipLaunchKernelGGL(k_gl_round<uint64_t>, dim3(grid_for_gl(work, 256)), dim3(256), 0, s, d_gamma,
                         g->dg.n, (int)R, (uint64_t*)st);
    if (d_bits_out)
      hipLaunchKernelGGL(k_gl_unpack<uint64_t>, dim3(ugrid), dim3(256), 0, s, (const uint64_t*)st,
                         g->dg.n, g->dg.nwords, (int)R, d_bits_out);
  }
  hipError_t e = launch_count(g->dg, st, R, d_counts, s);
  prof_end(g, s, tok, 1);
  return e == hipSuccess ? FI_OK : FI_EDEVICE;
}

}  // extern "C"
