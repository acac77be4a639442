// Whole-grid sweep for large graphs: a persistent cooperative kernel split
// into `batch` independent sub-grids.  Sub-grid s is the set of workgroups b
// with b % batch == s; workgroups are dealt to the XCDs round-robin, so with
// eight sub-grids each one runs on one XCD and its tree's bitmaps stay in
// that XCD's L2.  Sub-grid s sweeps trees t0 + s, t0 + s + batch, ... one at
// a time, with barriers among its own workgroups only.
//
// One tree is a level-synchronous BFS; each level picks its direction from
// the frontier's edge count:
//   top-down  - the frontier list is handed out in units (chunks of light
//               vertices, fixed edge ranges of heavy ones); every edge to an
//               unseen vertex applies an atomic minimum to its tree word, and
//               the thread that first reaches a vertex appends it to the next
//               list (staged in LDS) and sets its next-frontier bit.
//   bottom-up - a wave takes a 64-vertex word, concatenates the rows of its
//               unvisited vertices and walks them with all lanes, folding
//               every neighbour found in the frontier bitmap into that
//               vertex's minimum in LDS.  The wave owns the word: tree words
//               are plain stores, bitmap words atomic ORs.  Bottom-up levels
//               keep the frontier as a bitmap only; turning back to top-down
//               first compacts it into lists.
// Both directions produce the same words: the parent is the exact minimum
// key over previous-level neighbours whichever way it is found.
//
// Words that workgroups update with atomics are never written with plain
// stores while those atomics can run (a partly written cache line written
// back whole from one XCD's L2 would undo another XCD's atomic), so per-slot
// arrays are padded to 256 bytes and shared bitmap words are only OR-ed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {

namespace {

constexpr int kMaxSlots = kGridSlots;
constexpr int kHeavyUnit = 4096;    // edges per work unit of a heavy vertex
constexpr int kStage = 2048;        // LDS staging entries for next-level lists
constexpr int kBUWordsPerWave = 4;  // bottom-up words per wave per unit
constexpr int kWordCost = 16;       // bottom-up cost of one word, in edge visits
constexpr int kTDCost = 4;          // top-down cost of one frontier edge
constexpr int kGroup = kBarGroup;   // workgroups per barrier group

// control words of slot s: gctl + s * kSlotWords
//   [r * 8 + k], r = level % 4: k = 0 light count, 1 heavy (count << 32 |
//   units), 2 vertices reached, 3 their degree sum
//   [32 + 8 r]: work ticket of level slot r
//   [64 .. 66]: switches, key_hi, key_lo accumulators
constexpr int kSlotWords = kGridCtlWords;
// barrier words of slot s: bar + s * kBarWords: [0] generation, [16] root,
// [32 + 16 g] group g
constexpr int kBarWords = kGridBarWords;

struct GridArgs {
  uint64_t seed, t0, t1;
  uint64_t* tree_switches;
  uint64_t* bits_out;
  int insert;
  int batch;        // sub-grids, one tree in flight each
  int heavy;        // top-down: degree above which a vertex is split into units
  int nanch;
  int64_t hcap;     // heavy list capacity
  int64_t pstride;  // per-slot stride of pw / rootkey (n rounded up to 32)
  int64_t wstride;  // per-slot stride of each bitmap (nwords rounded up to 32)
  uint64_t* pw;     // [kMaxSlots][pstride]
  int32_t* ql;      // [kMaxSlots][2][n + 64]
  int2* qh;         // [kMaxSlots][2][hcap + 64]
  uint64_t* fb;     // [kMaxSlots][3][wstride]
  uint64_t* vis;    // [kMaxSlots][wstride]
  uint64_t* sb;     // [kMaxSlots][wstride]
  uint64_t* rootkey;// [kMaxSlots][pstride]
  uint64_t* gctl;   // [kMaxSlots][kSlotWords]
  uint64_t* bar;    // [kMaxSlots][kBarWords]
};

template <int NT>
struct GS {
  int off[NT];
  int start[NT];
  uint64_t base[NT];
  int scan[NT / 64 + 1];
  uint64_t red[NT / 64];
  int32_t q[kStage];
  uint32_t qn;
  uint32_t unit;
  int2 heavy;
  uint64_t cnt, deg;
  // level plan
  int mode, prev, active;           // mode: 1 top-down, 2 bottom-up
  uint32_t nl, nh, hunits, units;
  uint64_t vdeg;                    // degree sum of the vertices seen so far
  // bottom-up, per wave: the rows of its word
  int bu_off[NT];
  int bu_start[NT];
  uint64_t bu_best[NT];
};

__device__ __forceinline__ uint64_t amin64(uint64_t* p, uint64_t v) {
  return atomicMin((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void aor64(uint64_t* p, uint64_t v) {
  atomicOr((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void aadd64(uint64_t* p, uint64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ uint32_t bit_at(const uint64_t* words, uint32_t v) {
  return (uint32_t)(words[v >> 6] >> (v & 63)) & 1u;
}

// Barrier among the `nb` workgroups of one sub-grid (local ranks 0..nb-1).
__device__ __forceinline__ void sub_sync(uint64_t* bar, uint32_t rank, uint32_t nb) {
  group_sync(bar, rank, nb);
}

// Move the LDS staging list into a global list (one reservation per block).
template <int NT>
__device__ __forceinline__ void stage_flush(GS<NT>& sh, int32_t* list, uint64_t* ring) {
  __syncthreads();
  const uint32_t k = sh.qn;
  if (k) {
    if (threadIdx.x == 0) sh.unit = atomicAdd((uint32_t*)ring, k);  // reuse as base
    __syncthreads();
    const uint32_t base = sh.unit;
    for (uint32_t i = threadIdx.x; i < k; i += NT) list[base + i] = sh.q[i];
    __syncthreads();
    if (threadIdx.x == 0) sh.qn = 0;
  }
  __syncthreads();
}

// Listed vertices go to the light list (staged) or, above the heavy degree,
// to the heavy list with their first unit index.
template <int NT>
__device__ __forceinline__ void list_vertex(bool in, int32_t v, int dv, const GridArgs& A, GS<NT>& sh,
                                            int2* qh, uint64_t* ring) {
  const bool heavy = in && dv > A.heavy;
  const bool light = in && !heavy;
  const uint64_t mask = __ballot(light);
  if (mask) {
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&sh.qn, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (light) sh.q[base + lanes_below(mask)] = v;
  }
  if (heavy) {
    const uint64_t units = (uint64_t)((dv + kHeavyUnit - 1) / kHeavyUnit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// Newly reached vertices and their degree sum, into the block totals.
template <int NT>
__device__ __forceinline__ void count_reached(bool found, int dv, GS<NT>& sh) {
  const uint64_t c = __popcll(__ballot(found));
  const uint64_t d = wave_sum_u64(found ? (uint64_t)dv : 0ull);
  if (lane_id() == 0 && c) {
    atomicAdd((unsigned long long*)&sh.cnt, (unsigned long long)c);
    atomicAdd((unsigned long long*)&sh.deg, (unsigned long long)d);
  }
}

// Direction and unit count of this level (thread 0).  With `refresh` only
// the list sizes and units are re-read, after a compaction.
template <int NT>
__device__ void plan_level(GS<NT>& sh, const uint64_t* ctl, int64_t nnz, int32_t nw, uint32_t L,
                           bool refresh) {
  const uint64_t* ring = ctl + (L & 3) * 8;
  sh.nl = (uint32_t)load_agent(ring);
  const uint64_t hp = load_agent(ring + 1);
  sh.nh = (uint32_t)(hp >> 32);
  sh.hunits = (uint32_t)hp;
  if (!refresh) {
    const uint64_t nf = load_agent(ring + 2);
    const uint64_t mf = load_agent(ring + 3);
    sh.active = nf > 0;
    sh.mode = 0;
    if (nf > 0) {
      sh.vdeg += mf;
      // top-down pays per frontier edge (random atomics); bottom-up pays for
      // every word plus the rows of the unvisited vertices
      const uint64_t unvisited = (uint64_t)nnz - min<uint64_t>(sh.vdeg, (uint64_t)nnz);
      sh.mode = (uint64_t)kTDCost * mf > unvisited + (uint64_t)kWordCost * nw ? 2 : 1;
    }
  }
  constexpr uint32_t WPU = kBUWordsPerWave * (NT / 64);
  sh.units = sh.mode == 1 ? (sh.nl + NT - 1) / NT + sh.hunits
           : sh.mode == 2 ? (uint32_t)((nw + WPU - 1) / WPU) : 0u;
}

template <int NT>
__global__ void __launch_bounds__(NT, 4) k_sweep_grid(DevGraph G, GridArgs A) {
  __shared__ GS<NT> sh;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const uint32_t B = (uint32_t)A.batch;
  const int s = (int)(blockIdx.x % B);                       // sub-grid / slot
  const uint32_t rank = blockIdx.x / B;                      // rank within the sub-grid
  const uint32_t nb = (gridDim.x - s + B - 1) / B;           // sub-grid size
  const int64_t stid = (int64_t)rank * NT + tid;
  const int64_t sstride = (int64_t)nb * NT;
  const int64_t swave = stid >> 6, nswaves = sstride >> 6;
  const int32_t n = G.n;
  const int32_t nw = G.nwords;
  const int32_t* rp = G.row_ptr;
  const size_t ws = (size_t)A.wstride;

  uint64_t* pw = A.pw + (size_t)s * A.pstride;
  uint64_t* rootkey = A.rootkey + (size_t)s * A.pstride;
  uint64_t* fbuf = A.fb + (size_t)s * 3 * ws;
  uint64_t* vis = A.vis + (size_t)s * ws;
  uint64_t* sbs = A.sb + (size_t)s * ws;
  uint64_t* ctl = A.gctl + (size_t)s * kSlotWords;
  uint64_t* bar = A.bar + (size_t)s * kBarWords;
  const size_t lstride = (size_t)n + 64, hstride = (size_t)A.hcap + 64;
  int32_t* qlb = A.ql + (size_t)s * 2 * lstride;
  int2* qhb = A.qh + (size_t)s * 2 * hstride;

  for (uint64_t t = A.t0 + s; t < A.t1; t += B) {
    const KeyMix km = key_mix(tree_salt(A.seed, t));

    // ---- P0: reset tree words and bitmaps, per-component minimum keys
    for (int64_t v = stid; v < n; v += sstride) pw[v] = kUnvisited;
    for (int64_t i = stid; i < nw; i += sstride) {
      vis[i] = 0;
      sbs[i] = 0;
      fbuf[i] = 0;
      fbuf[ws + i] = 0;
      fbuf[2 * ws + i] = 0;
    }
    if (rank == 0) {
      for (int i = tid; i < kSlotWords; i += NT) ctl[i] = 0;
    }
    if (tid == 0) {
      sh.prev = 0;
      sh.vdeg = 0;
      sh.qn = 0;
    }
    {
      // contiguous word ranges per wave; one atomic per run of words with
      // the same main component, one per vertex of another component
      const int64_t per = (nw + nswaves - 1) / nswaves;
      const int64_t w0 = swave * per, w1 = min<int64_t>(nw, w0 + per);
      int32_t cur = -1;
      uint64_t cmin = kUnvisited;
      for (int64_t i = w0; i < w1; ++i) {
        const int32_t wc = G.word_comp[i];
        if (wc == -2) continue;
        const uint64_t main = G.word_main[i];
        const uint64_t minor = G.word_mask[i] & ~main;
        const int32_t v = (int32_t)(i * 64 + lane);
        if (wc != cur) {
          if (cur >= 0 && lane == 0) amin64(rootkey + cur, cmin);
          cur = wc;
          cmin = kUnvisited;
        }
        const uint64_t cand = root_candidate(vkey(km, v), v);
        const uint64_t mn = wave_min_u64(((main >> lane) & 1) ? cand : kUnvisited);
        cmin = mn < cmin ? mn : cmin;
        if ((minor >> lane) & 1) amin64(rootkey + G.comp[v], cand);
      }
      if (cur >= 0 && lane == 0) amin64(rootkey + cur, cmin);
    }
    sub_sync(bar, rank, nb);

    // ---- P1: the roots form level 0 (lists and frontier bits)
    {
      uint64_t* ring0 = ctl;
      if (tid == 0) {
        sh.cnt = 0;
        sh.deg = 0;
      }
      __syncthreads();
      for (int64_t c0 = (int64_t)rank * NT; c0 < A.nanch; c0 += sstride) {
        const int64_t c = c0 + tid;
        const bool ok = c < A.nanch;
        int32_t r = 0;
        int dr = 0;
        if (ok) {
          const int32_t a = G.anchors[c];
          const uint64_t k = rootkey[a];
          rootkey[a] = kUnvisited;
          r = (int32_t)word_vertex(k);
          dr = rp[r + 1] - rp[r];
          pw[r] = tree_word(0, vkey(km, r), 0);
          aor64(fbuf + (r >> 6), 1ull << (r & 63));
        }
        list_vertex<NT>(ok, r, dr, A, sh, qhb, ring0);
        count_reached<NT>(ok, dr, sh);
        __syncthreads();
        if (sh.qn > kStage - NT) stage_flush<NT>(sh, qlb, ring0);
      }
      stage_flush<NT>(sh, qlb, ring0);
      if (tid == 0 && sh.cnt) {
        aadd64(ring0 + 2, sh.cnt);
        aadd64(ring0 + 3, sh.deg);
      }
    }
    sub_sync(bar, rank, nb);

    // ---- P2: levels
    for (uint32_t L = 0;; ++L) {
      uint64_t* fb = fbuf + (size_t)(L % 3) * ws;
      uint64_t* nbm = fbuf + (size_t)((L + 1) % 3) * ws;
      uint64_t* zb = fbuf + (size_t)((L + 2) % 3) * ws;
      uint64_t* ring = ctl + (L & 3) * 8;
      uint64_t* ring_next = ctl + ((L + 1) & 3) * 8;
      int32_t* ql = qlb + (size_t)(L & 1) * lstride;
      int2* qh = qhb + (size_t)(L & 1) * hstride;
      int32_t* ql_next = qlb + (size_t)((L + 1) & 1) * lstride;
      int2* qh_next = qhb + (size_t)((L + 1) & 1) * hstride;
      if (tid == 0) plan_level<NT>(sh, ctl, G.nnz, nw, L, false);
      __syncthreads();
      if (!sh.active) break;
      if (L + 1 > kMaxLevel) {
        if (stid == 0) atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_DEPTH);
        break;
      }
      // the bitmap and the counters two levels ahead start from zero
      for (int64_t i = stid; i < nw; i += sstride) zb[i] = 0;
      if (rank == 0 && tid < 8) {
        ctl[((L + 2) & 3) * 8 + tid] = 0;
        if (tid == 0) ctl[32 + 8 * ((L + 2) & 3)] = 0;
      }
      if (sh.mode == 2 && sh.prev == 1) {
        // bottom-up after top-down: the frontier's state bits become final
        // only now (its words were minimised by atomics last level)
        const int64_t cnt = (int64_t)sh.nl + sh.nh;
        for (int64_t i = stid; i < cnt; i += sstride) {
          const int32_t u = i < sh.nl ? ql[i] : qh[i - sh.nl].x;
          if (pw[u] & 1) aor64(sbs + (u >> 6), 1ull << (u & 63));
        }
        sub_sync(bar, rank, nb);
      } else if (sh.mode == 1 && sh.prev == 2) {
        // top-down after bottom-up: list the frontier bitmap
        for (int64_t c0 = (int64_t)rank * (NT / 64); c0 < nw; c0 += (int64_t)nb * (NT / 64)) {
          const int64_t w = c0 + wave;
          const uint64_t bits = w < nw ? fb[w] : 0ull;
          const bool in = (bits >> lane) & 1;
          const int32_t v = (int32_t)(w * 64 + lane);
          const int dv = in ? rp[v + 1] - rp[v] : 0;
          list_vertex<NT>(in, v, dv, A, sh, qh, ring);
          __syncthreads();
          if (sh.qn > kStage - NT) stage_flush<NT>(sh, ql, ring);
        }
        stage_flush<NT>(sh, ql, ring);
        sub_sync(bar, rank, nb);
        if (tid == 0) plan_level<NT>(sh, ctl, G.nnz, nw, L, true);
        __syncthreads();
      }

      // units: rank r first takes unit r; only when there are more units
      // than workgroups do they draw further ones from the ticket
      const uint32_t U = sh.units;
      uint64_t* ticket = ctl + 32 + 8 * (L & 3);
      bool first = true;
      while (true) {
        if (tid == 0) {
          sh.unit = first ? rank : (U > nb ? nb + atomicAdd((uint32_t*)ticket, 1u) : U);
          sh.cnt = 0;
          sh.deg = 0;
        }
        first = false;
        __syncthreads();
        const uint32_t k = sh.unit;
        if (k >= U) break;

        if (sh.mode == 1) {
          // ---------------- top-down unit
          const uint32_t nchunks = (sh.nl + NT - 1) / NT;
          int64_t e0 = 0;
          uint64_t hbase = 0;
          int total = 0;
          if (k < nchunks) {
            const uint32_t i = k * NT + tid;
            int d = 0, st = 0;
            uint64_t base = 0;
            if (i < sh.nl) {
              const int32_t u = ql[i];
              st = rp[u];
              d = rp[u + 1] - st;
              const uint32_t b = (uint32_t)(pw[u] & 1);
              base = tree_word(L + 1, vkey(km, u), b);
              aor64(vis + (u >> 6), 1ull << (u & 63));
              if (b) aor64(sbs + (u >> 6), 1ull << (u & 63));
            }
            const int off = block_exclusive_scan<NT>(d, total, sh.scan);
            sh.off[tid] = off;
            sh.start[tid] = st;
            sh.base[tid] = base;
            __syncthreads();
          } else {
            const uint32_t hk = k - nchunks;
            if (tid == 0) {
              int lo = 0, hi = (int)sh.nh;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((uint32_t)qh[mid].y <= hk) lo = mid; else hi = mid;
              }
              sh.heavy = qh[lo];
            }
            __syncthreads();
            const int32_t u = sh.heavy.x;
            const uint32_t part = hk - (uint32_t)sh.heavy.y;
            const uint32_t b = (uint32_t)(pw[u] & 1);
            if (part == 0 && tid == 0) {
              aor64(vis + (u >> 6), 1ull << (u & 63));
              if (b) aor64(sbs + (u >> 6), 1ull << (u & 63));
            }
            e0 = rp[u] + (int64_t)part * kHeavyUnit;
            const int64_t e1 = min<int64_t>(rp[u + 1], e0 + kHeavyUnit);
            hbase = tree_word(L + 1, vkey(km, u), b);
            total = (int)(e1 - e0);
          }
          for (int j0 = 0; j0 < total; j0 += NT) {
            const int j = j0 + tid;
            bool found = false;
            int32_t v = 0;
            int dv = 0;
            if (j < total) {
              uint32_t a;
              uint64_t nwd;
              if (k < nchunks) {
                const int kk = upper_index(sh.off, NT, j);
                a = G.adj[sh.start[kk] + (j - sh.off[kk])];
                nwd = sh.base[kk];
              } else {
                a = G.adj[e0 + j];
                nwd = hbase;
              }
              v = (int32_t)(a & kVertexMask);
              nwd ^= (uint64_t)(a >> 31);
              const uint64_t seen = vis[v >> 6] | fb[v >> 6];
              if (!((seen >> (v & 63)) & 1) && pw[v] > nwd) {
                found = amin64(pw + v, nwd) == kUnvisited;
                if (found) {
                  dv = rp[v + 1] - rp[v];
                  aor64(nbm + (v >> 6), 1ull << (v & 63));
                }
              }
            }
            list_vertex<NT>(found, v, dv, A, sh, qh_next, ring_next);
            count_reached<NT>(found, dv, sh);
            __syncthreads();
            if (sh.qn > kStage - NT) stage_flush<NT>(sh, ql_next, ring_next);
          }
          stage_flush<NT>(sh, ql_next, ring_next);
        } else {
          // ---------------- bottom-up unit: kBUWordsPerWave words per wave
          constexpr int WPU = kBUWordsPerWave * (NT / 64);
          const int64_t wbeg = (int64_t)k * WPU;
          int* wo = sh.bu_off + wave * 64;
          int* wb = sh.bu_start + wave * 64;
          uint64_t* wbest = sh.bu_best + wave * 64;
          for (int it = 0; it < kBUWordsPerWave; ++it) {
            const int64_t w = wbeg + (int64_t)it * (NT / 64) + wave;
            if (w >= nw) continue;
            const uint64_t fbw = fb[w];
            const uint64_t vw = vis[w] | fbw;
            if (lane == 0 && fbw) aor64(vis + w, fbw);
            const uint64_t un = G.word_mask[w] & ~vw;
            if (un == 0) continue;
            const bool mine = (un >> lane) & 1;
            const int32_t v = (int32_t)(w * 64 + lane);
            int rb = 0, dv = 0;
            if (mine) {
              rb = rp[v];
              dv = rp[v + 1] - rb;
            }
            int inc = dv;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
              const int y = __shfl_up(inc, d);
              if (lane >= d) inc += y;
            }
            const int total = __shfl(inc, 63);
            wo[lane] = inc - dv;
            wb[lane] = rb;
            wbest[lane] = kUnvisited;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int j0 = 0; j0 < total; j0 += 4 * 64) {
              uint32_t a[4];
              int kk[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int j = j0 + q * 64 + lane;
                kk[q] = -1;
                a[q] = 0;
                if (j < total) {
                  kk[q] = upper_index(wo, 64, j);
                  a[q] = G.adj[wb[kk[q]] + (j - wo[kk[q]])];
                }
              }
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                if (kk[q] < 0) continue;
                const uint32_t u = a[q] & kVertexMask;
                if (bit_at(fb, u)) {
                  const uint64_t c = root_candidate(vkey(km, u), u) | (a[q] >> 31);
                  atomicMin((unsigned long long*)(wbest + kk[q]), (unsigned long long)c);
                }
              }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const uint64_t best = mine ? wbest[lane] : kUnvisited;
            const bool found = best != kUnvisited;
            uint32_t b = 0;
            if (found) {
              const uint32_t u = word_vertex(best);
              b = bit_at(sbs, u) ^ (uint32_t)(best & 1);
              pw[v] = tree_word(L + 1, (uint32_t)(best >> 32), b);
            }
            const uint64_t nbits = __ballot(found);
            const uint64_t bbits = __ballot(found && b);
            if (lane == 0 && nbits) {
              aor64(nbm + w, nbits);
              if (bbits) aor64(sbs + w, bbits);
            }
            count_reached<NT>(found, dv, sh);
          }
          __syncthreads();
        }
        if (tid == 0 && sh.cnt) {
          aadd64(ring_next + 2, sh.cnt);
          aadd64(ring_next + 3, sh.deg);
        }
        __syncthreads();
      }
      if (tid == 0) sh.prev = sh.mode;
      sub_sync(bar, rank, nb);
    }

    // ---- P3: canonical words, key terms and the exact count
    {
      uint64_t khi = 0, klo = 0, S = 0;
      for (int64_t i = swave; i < nw; i += nswaves) {
        const int32_t wc = G.word_comp[i];
        uint64_t W = sbs[i];
        if (wc >= 0) {
          const uint64_t main = G.word_main[i];
          const uint64_t minor = G.word_mask[i] & ~main;
          if (bit_at(sbs, (uint32_t)wc)) W ^= main;
          if (minor) {
            const int32_t a = ((minor >> lane) & 1) ? G.comp[i * 64 + lane] : -1;
            W ^= __ballot(a >= 0 && bit_at(sbs, (uint32_t)a));
          }
        }
        if (lane == 0) {
          key_terms((uint64_t)i, W, khi, klo);
          if (A.bits_out) A.bits_out[i] = W;
        }
      }
      for (int64_t e0 = stid; e0 < G.m; e0 += 4 * sstride) {
        uint2 uv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = e0 + q * sstride;
          uv[q] = e < G.m ? G.edges[e] : make_uint2(0u, 0u);  // (0, 0) is never frustrated
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          S += (uv[q].y >> 31) ^ bit_at(sbs, uv[q].x) ^ bit_at(sbs, uv[q].y & kVertexMask);
      }
      S = block_sum_u64<NT>(S, sh.red);
      khi = block_sum_u64<NT>(khi, sh.red);
      klo = block_sum_u64<NT>(klo, sh.red);
      if (tid == 0) {
        if (S) aadd64(ctl + 64, S);
        if (khi) aadd64(ctl + 65, khi);
        if (klo) aadd64(ctl + 66, klo);
      }
    }
    sub_sync(bar, rank, nb);

    // ---- P4: insert the tree
    if (rank == 0 && tid == 0) {
      const uint64_t s0 = load_agent(ctl + 64), h0 = load_agent(ctl + 65), l0 = load_agent(ctl + 66);
      if (A.insert) cloud_insert(G, h0, l0, s0, t);
      if (A.tree_switches) A.tree_switches[t - A.t0] = s0;
    }
    // the next tree clears the control words; finish reading them first
    sub_sync(bar, rank, nb);
  }
}

template <int NT>
hipError_t launch_nt(fi_graph* g, const GridArgs& a, hipStream_t s) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_grid<NT>, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int maxg = per_cu * g->cu_count;
  int grid = g->sched.grid > 0 ? std::min(g->sched.grid, maxg) : std::min(maxg, 2 * g->cu_count);
  grid = std::max(grid, a.batch);
  if (grid > maxg || (grid + a.batch - 1) / a.batch > kGroup * 512) return hipErrorInvalidConfiguration;
  DevGraph G = g->dg;
  GridArgs A = a;
  void* args[] = {(void*)&G, (void*)&A};
  e = hipLaunchCooperativeKernel((const void*)k_sweep_grid<NT>, dim3(grid), dim3(NT), args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid(fi_graph* g, const SweepArgs& sa, hipStream_t s) {
  const Layout& L = g->L;
  GridArgs a{};
  a.seed = sa.seed;
  a.t0 = sa.t0;
  a.t1 = sa.t1;
  a.tree_switches = sa.tree_switches;
  a.bits_out = sa.bits_out;
  a.insert = sa.insert;
  // never more sub-grids than trees, so every sub-grid has work
  a.batch = (int)std::max<uint64_t>(1, std::min<uint64_t>(std::min(g->sched.batch, kMaxSlots),
                                                          sa.t1 - sa.t0));
  a.heavy = g->sched.heavy;
  a.nanch = g->nanch;
  a.hcap = (int64_t)L.hcap;
  a.pstride = (int64_t)L.gpstride;
  a.wstride = (int64_t)L.gwstride;
  a.pw = (uint64_t*)(g->ws + L.gpw);
  a.ql = (int32_t*)(g->ws + L.gql);
  a.qh = (int2*)(g->ws + L.gqh);
  a.fb = (uint64_t*)(g->ws + L.gfb);
  a.vis = (uint64_t*)(g->ws + L.gvis);
  a.sb = (uint64_t*)(g->ws + L.gsb);
  a.rootkey = (uint64_t*)(g->ws + L.grootkey);
  a.gctl = (uint64_t*)(g->ws + L.gctl);
  a.bar = (uint64_t*)(g->ws + L.gbar);
  const int nt = g->sched.block;
  return nt == 1024 ? launch_nt<1024>(g, a, s) : nt == 512 ? launch_nt<512>(g, a, s)
                                                           : launch_nt<256>(g, a, s);
}

}  // namespace fi
