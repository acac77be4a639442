// Multi-tree sweep for large graphs: the trees of Alg. alg-index taken 64 at
// a time, one bit per tree in every per-vertex word (bit t is tree t0 + t and
// lane t of every wavefront).
//
// Each vertex has a 32-byte record: the trees in which it was discovered at
// the last even and the last odd level, its state bits, and the trees that
// have visited it.  One BFS level then serves all 64 trees with one pass over
// the rows involved:
//   push - while the frontier is small, its rows mark as candidates every
//          neighbour still unvisited in a tree where the frontier vertex was
//          just discovered;
//   pull - a wave takes a candidate (or, on large frontiers, every vertex not
//          yet visited by all trees) and walks its row; lane t keeps the
//          minimum key over the neighbours discovered at the previous level
//          of tree t, which is exactly the single-tree parent rule, and the
//          state bit that comes with it.  Rows longer than kMSplit are cut
//          into parts whose minima meet through atomic minima.
// A neighbour's discovery word may still carry bits from two levels back;
// such a tree has already visited every neighbour of that vertex, so the
// bit never survives the mask of unvisited trees and the words need no
// clearing between levels.
// After the BFS, bit-sliced counters over the edge list give every tree's
// frustrated-edge count, 64x64 bit transposes of the state words give its
// canonical key, and the 64 trees enter the cloud.
//
// Memory discipline across XCDs: within one phase a word is either written
// with plain stores by its single owner or updated with atomics, never both.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {

namespace {

constexpr int kStageM = 2048;      // LDS staging entries for light list appends
constexpr int kPushCost = 2;       // push while kPushCost * frontier edges < unfinished edges
constexpr int kPullPerWave = 4;    // light pull vertices per wave per unit
constexpr int kPlanes = 8;         // bit-sliced counter planes (flushed every 255 edges)

// Per-vertex record: discovered at the last even / odd level, state bits,
// visited.
struct __align__(32) MRec {
  uint64_t nb[2];
  uint64_t st;
  uint64_t vis;
};

// Control words; each group sits on its own 128-byte line.  r = level mod 4.
//   F(r): frontier lists of the level: light count, heavy (count << 32 |
//         units), vertices reached, their degree sum
//   P(r): pull lists of the level: light count, heavy (count << 32 | units)
//   TP(r), TQ(r): work tickets of the list / push phase and the pull phase
//   UNF: degree sum of vertices not yet visited by every tree
//   ACC + 4 t: tree t's switches, key_hi, key_lo
__host__ __device__ constexpr int cF(int r) { return 16 * r; }
__host__ __device__ constexpr int cP(int r) { return 64 + 16 * r; }
__host__ __device__ constexpr int cTP(int r) { return 128 + 16 * r; }
__host__ __device__ constexpr int cTQ(int r) { return 192 + 16 * r; }
constexpr int cUNF = 256;
constexpr int cACC = 512;
constexpr int kMCtlWords = 768;
static_assert(kMCtlWords <= kGridSlots * kGridCtlWords, "control block");

struct MArgs {
  uint64_t seed, t0, t1;
  uint64_t* tree_switches;
  int insert;
  int32_t ntasks, nbig;
  MRec* rec;
  uint64_t* unf;        // [nwords] vertices with an edge not yet visited by every tree
  uint64_t* cand;       // [nwords] push candidates of the level
  int32_t* fl;          // [2][lstride] frontier light lists (by level parity)
  int2* fh;             // [2][hstride] frontier heavy lists (vertex, first unit)
  int32_t* pl;          // [lstride] pull light list
  int2* ph;             // [hstride] pull heavy list; entry h owns hslot row h
  int64_t lstride, hstride;
  uint64_t* hslot;      // [rows][64] partial minima of split rows
  const int4* tasks;    // root tasks: (begin, end) in cverts, big slot or -1
  const int32_t* cverts;
  uint64_t* rootbig;    // [big components][64]
  uint64_t* ctl;
  uint64_t* bar;
};

template <int NT>
struct MS {
  int off[NT];
  int start[NT];
  uint64_t base[NT];
  int scan[NT / 64 + 1];
  int32_t q[kStageM];
  uint32_t qn;
  uint32_t unit;
  int hidx;
  int2 heavy;
  uint64_t cnt, deg, fin;
  int mode, active;
  uint32_t nl, nh, hunits;
  uint64_t hbest[64];
  uint64_t tacc[3][64];
};

__device__ __forceinline__ uint64_t amin64(uint64_t* p, uint64_t v) {
  return atomicMin((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ uint64_t aor64(uint64_t* p, uint64_t v) {
  return atomicOr((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void aand64(uint64_t* p, uint64_t v) {
  atomicAnd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void aadd64(uint64_t* p, uint64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int j) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, j);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// Move the LDS staging list into a global list (one reservation per block).
template <int NT>
__device__ __forceinline__ void mflush(MS<NT>& sh, int32_t* list, uint64_t* ring) {
  __syncthreads();
  const uint32_t k = sh.qn;
  if (k) {
    if (threadIdx.x == 0) sh.unit = atomicAdd((uint32_t*)ring, k);
    __syncthreads();
    const uint32_t base = sh.unit;
    for (uint32_t i = threadIdx.x; i < k; i += NT) list[base + i] = sh.q[i];
    __syncthreads();
    if (threadIdx.x == 0) sh.qn = 0;
  }
  __syncthreads();
}

// Lanes with `in` list vertex v of degree dv: light ones into the LDS
// staging list, split rows straight into the heavy list with their units.
template <int NT>
__device__ __forceinline__ void mlist(bool in, int32_t v, int dv, MS<NT>& sh, int2* qh,
                                      uint64_t* ring) {
  const bool heavy = in && dv > kMSplit;
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
    const uint64_t units = (uint64_t)((dv + kMSplit - 1) / kMSplit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// The same straight into the global lists (no staging).
__device__ __forceinline__ void mlist_global(bool in, int32_t v, int dv, int32_t* ql, int2* qh,
                                             uint64_t* ring) {
  const bool heavy = in && dv > kMSplit;
  wave_append(in && !heavy, v, ql, (uint32_t*)ring);
  if (heavy) {
    const uint64_t units = (uint64_t)((dv + kMSplit - 1) / kMSplit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// Lane t: minimum over the edges [e0, e1) of the candidate key (hash, id,
// state bit) of every neighbour discovered at the previous level of tree t
// (parity pp) in a tree of `want`.
__device__ __forceinline__ uint64_t pull_edges(const uint32_t* adj, const MRec* rec, int64_t e0,
                                               int64_t e1, int pp, uint64_t want, KeyMix km,
                                               uint64_t best) {
  const int lane = lane_id();
  for (int64_t c = e0; c < e1; c += 64) {
    const int64_t e = c + lane;
    uint32_t a = 0;
    uint64_t F = 0, S = 0;
    if (e < e1) {
      a = adj[e];
      const MRec* ru = rec + (a & kVertexMask);
      F = ru->nb[pp] & want;
      if (F) S = ru->st;
    }
    uint64_t hits = __ballot(F != 0);
    while (hits) {
      const int j = __builtin_ctzll(hits);
      hits &= hits - 1;
      const uint32_t aj = __builtin_amdgcn_readlane(a, j);
      const uint64_t Fj = readlane64(F, j);
      const uint64_t Sj = readlane64(S, j);
      if ((Fj >> lane) & 1) {
        const uint32_t uj = aj & kVertexMask;
        const uint64_t bit = ((Sj >> lane) & 1) ^ (uint64_t)(aj >> 31);
        const uint64_t c2 = ((uint64_t)vhash20(km, uj) << 33) | ((uint64_t)uj << 1) | bit;
        best = c2 < best ? c2 : best;
      }
    }
  }
  return best;
}

// Lane t: the minimum root candidate of tree t over cverts[b, e).
__device__ __forceinline__ uint64_t comp_min(const int32_t* cverts, int32_t b, int32_t e, KeyMix km) {
  const int lane = lane_id();
  uint64_t best = kUnvisited;
  for (int32_t c = b; c < e; c += 64) {
    const int32_t i = c + lane;
    const int32_t mine = i < e ? cverts[i] : 0;
    const int cnt = min(64, e - c);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t v = (uint32_t)__builtin_amdgcn_readlane(mine, j);
      const uint64_t k = root_candidate(vhash20(km, v), v);
      best = k < best ? k : best;
    }
  }
  return best;
}

// Roots of one component (the wave owns it): lanes are grouped by root
// vertex; each root's record gets the trees it roots, and it enters the
// level-0 lists.  cnt / deg gather the wave's roots and their degrees, fin
// (in the lanes that wrote a root) the degrees of vertices already visited
// by every tree.
__device__ __forceinline__ void set_roots(uint64_t best, bool vlane, uint64_t valid, const MArgs& A,
                                          const int32_t* rp, uint64_t& cnt, uint64_t& deg,
                                          uint64_t& fin) {
  const int lane = lane_id();
  const bool ok = vlane && best != kUnvisited;
  const uint32_t r = (uint32_t)word_vertex(best);
  uint64_t rem = __ballot(ok);
  bool leader = false;
  uint64_t mine = 0;
  while (rem) {
    const int j = __builtin_ctzll(rem);
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)r, j);
    const uint64_t m = __ballot(ok && r == r0);
    rem &= ~m;
    if (lane == j) {
      leader = true;
      mine = m;
    }
  }
  int dv = 0;
  if (leader) {
    dv = rp[r + 1] - rp[r];
    A.rec[r].nb[0] = mine;
    A.rec[r].vis = mine;
    if (mine == valid) {
      aand64(A.unf + (r >> 6), ~(1ull << (r & 63)));
      fin += (uint64_t)dv;
    }
  }
  mlist_global(leader, (int32_t)r, dv, A.fl, A.fh, A.ctl + cF(0));
  cnt += (uint64_t)__popcll(__ballot(leader));
  deg += wave_sum_u64(leader ? (uint64_t)dv : 0ull);
}

// Write back a vertex whose trees of this level are decided (one lane; newb
// / stb are the trees that reached it and their state bits) and clear its
// candidate bit; fin gathers the degree of a vertex every tree has now
// visited.
__device__ __forceinline__ void finish_vertex(const MArgs& A, int32_t v, uint64_t vis, uint64_t st,
                                              uint64_t newb, uint64_t stb, int p, uint64_t valid,
                                              bool push_mode, int dv, uint64_t& fin) {
  MRec* r = A.rec + v;
  const uint64_t bit = 1ull << (v & 63);
  if (newb) {
    r->vis = vis | newb;
    r->nb[p] = newb;
    if (stb) r->st = st | stb;
    if ((vis | newb) == valid) {
      aand64(A.unf + (v >> 6), ~bit);
      fin += (uint64_t)dv;
    }
  }
  if (push_mode) aand64(A.cand + (v >> 6), ~bit);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_sweep_multi(DevGraph G, MArgs A) {
  __shared__ MS<NT> sh;
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const uint32_t rank = blockIdx.x, nb = gridDim.x;
  const int64_t stid = (int64_t)rank * NT + tid, sstride = (int64_t)nb * NT;
  const int64_t gwave = stid >> 6, nwaves = sstride >> 6;
  const int32_t n = G.n, nw = G.nwords;
  const int32_t* rp = G.row_ptr;
  uint64_t* ctl = A.ctl;

  for (uint64_t tb = A.t0; tb < A.t1; tb += 64) {
    const int nvalid = (int)min<uint64_t>(64, A.t1 - tb);
    const uint64_t valid = nvalid == 64 ? ~0ull : ((1ull << nvalid) - 1);
    const bool vlane = lane < nvalid;
    const KeyMix km = key_mix(tree_salt(A.seed, tb + lane));

    // ---- reset: records, bitmaps, control words
    for (int64_t v = stid; v < n; v += sstride) {
      MRec z;
      z.nb[0] = 0;
      z.nb[1] = 0;
      z.st = 0;
      z.vis = 0;
      A.rec[v] = z;
    }
    for (int64_t i = stid; i < nw; i += sstride) {
      A.unf[i] = G.word_mask[i];
      A.cand[i] = 0;
    }
    if (rank == 0)
      for (int i = tid; i < kMCtlWords; i += NT) ctl[i] = i == cUNF ? (uint64_t)G.nnz : 0ull;
    if (tid == 0) sh.qn = 0;
    group_sync(A.bar, rank, nb);

    // ---- roots: the minimum key of every component, per tree
    {
      uint64_t cnt = 0, deg = 0, fin = 0;
      for (int64_t k = gwave; k < A.ntasks; k += nwaves) {
        const int4 tk = A.tasks[k];
        const uint64_t best = comp_min(A.cverts, tk.x, tk.y, km);
        if (tk.z < 0)
          set_roots(best, vlane, valid, A, rp, cnt, deg, fin);
        else if (vlane && best != kUnvisited)
          amin64(A.rootbig + (size_t)tk.z * 64 + lane, best);
      }
      group_sync(A.bar, rank, nb);
      for (int64_t b = gwave; b < A.nbig; b += nwaves) {
        uint64_t* rb = A.rootbig + (size_t)b * 64;
        const uint64_t best = vlane ? rb[lane] : kUnvisited;
        if (vlane) rb[lane] = kUnvisited;
        set_roots(best, vlane, valid, A, rp, cnt, deg, fin);
      }
      fin = wave_sum_u64(fin);
      if (lane == 0) {
        if (cnt) {
          aadd64(ctl + cF(0) + 2, cnt);
          aadd64(ctl + cF(0) + 3, deg);
        }
        if (fin) aadd64(ctl + cUNF, (uint64_t)0 - fin);
      }
    }
    group_sync(A.bar, rank, nb);

    // ---- levels
    for (uint32_t L = 1;; ++L) {
      const int pp = (int)((L - 1) & 1), p = (int)(L & 1);
      uint64_t* rfp = ctl + cF((L - 1) & 3);
      uint64_t* rf = ctl + cF(L & 3);
      uint64_t* rpl = ctl + cP(L & 3);
      const int32_t* flp = A.fl + (size_t)pp * A.lstride;
      const int2* fhp = A.fh + (size_t)pp * A.hstride;
      int32_t* fln = A.fl + (size_t)p * A.lstride;
      int2* fhn = A.fh + (size_t)p * A.hstride;
      if (tid == 0) {
        sh.nl = (uint32_t)load_agent(rfp);
        const uint64_t hp = load_agent(rfp + 1);
        sh.nh = (uint32_t)(hp >> 32);
        sh.hunits = (uint32_t)hp;
        const uint64_t reached = load_agent(rfp + 2), fdeg = load_agent(rfp + 3);
        const uint64_t unf = load_agent(ctl + cUNF);
        sh.active = reached > 0;
        sh.mode = (uint64_t)kPushCost * fdeg < unf ? 1 : 2;
      }
      __syncthreads();
      if (!sh.active) break;
      if (L > (uint32_t)kMaxLevel) {
        if (stid == 0) atomicOr((unsigned long long*)(G.ctl + C_ERR), (unsigned long long)E_DEPTH);
        break;
      }
      const bool push = sh.mode == 1;
      // counters and tickets of level L + 1 start from zero
      if (rank == 0 && tid < 4) {
        const int r = (int)((L + 1) & 3);
        ctl[cF(r) + tid] = 0;
        if (tid < 2) ctl[cP(r) + tid] = 0;
        if (tid == 0) {
          ctl[cTP(r)] = 0;
          ctl[cTQ(r)] = 0;
        }
      }

      // ---- phase 1: the pull lists
      if (push) {
        const uint32_t nchunks = (sh.nl + NT - 1) / NT;
        const uint32_t U = nchunks + sh.hunits;
        uint64_t* ticket = ctl + cTP(L & 3);
        bool firstu = true;
        while (true) {
          if (tid == 0) sh.unit = firstu ? rank : (U > nb ? nb + atomicAdd((uint32_t*)ticket, 1u) : U);
          firstu = false;
          __syncthreads();
          const uint32_t k = sh.unit;
          if (k >= U) break;
          int total = 0;
          int64_t e0 = 0;
          uint64_t hbits = 0;
          if (k < nchunks) {
            const uint32_t i = k * NT + tid;
            int d = 0, st = 0;
            uint64_t bits = 0;
            if (i < sh.nl) {
              const int32_t u = flp[i];
              st = rp[u];
              d = rp[u + 1] - st;
              bits = A.rec[u].nb[pp] & valid;
            }
            const int off = block_exclusive_scan<NT>(d, total, sh.scan);
            sh.off[tid] = off;
            sh.start[tid] = st;
            sh.base[tid] = bits;
            __syncthreads();
          } else {
            const uint32_t hk = k - nchunks;
            if (tid == 0) {
              int lo = 0, hi = (int)sh.nh;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((uint32_t)fhp[mid].y <= hk) lo = mid; else hi = mid;
              }
              sh.heavy = fhp[lo];
            }
            __syncthreads();
            const int32_t u = sh.heavy.x;
            const uint32_t part = hk - (uint32_t)sh.heavy.y;
            e0 = rp[u] + (int64_t)part * kMSplit;
            const int64_t e1 = min<int64_t>(rp[u + 1], e0 + kMSplit);
            hbits = A.rec[u].nb[pp] & valid;
            total = (int)(e1 - e0);
          }
          for (int j0 = 0; j0 < total; j0 += NT) {
            const int j = j0 + tid;
            bool first = false;
            int32_t v = 0;
            int dv = 0;
            if (j < total) {
              uint32_t a;
              uint64_t bits;
              if (k < nchunks) {
                const int kk = upper_index(sh.off, NT, j);
                a = G.adj[sh.start[kk] + (j - sh.off[kk])];
                bits = sh.base[kk];
              } else {
                a = G.adj[e0 + j];
                bits = hbits;
              }
              v = (int32_t)(a & kVertexMask);
              if (bits & ~A.rec[v].vis) {
                const uint64_t bit = 1ull << (v & 63);
                if (!(aor64(A.cand + (v >> 6), bit) & bit)) {
                  first = true;
                  dv = rp[v + 1] - rp[v];
                }
              }
            }
            mlist<NT>(first, v, dv, sh, A.ph, rpl);
            __syncthreads();
            if (sh.qn > kStageM - NT) mflush<NT>(sh, A.pl, rpl);
          }
          __syncthreads();
        }
      } else {
        // every vertex some tree has not visited yet
        for (int64_t c0 = (int64_t)rank * NW; c0 < nw; c0 += (int64_t)nb * NW) {
          const int64_t w = c0 + wave;
          const uint64_t bits = w < nw ? A.unf[w] : 0ull;
          const bool in = (bits >> lane) & 1;
          const int32_t v = (int32_t)(w * 64 + lane);
          const int dv = in ? rp[v + 1] - rp[v] : 0;
          mlist<NT>(in, v, dv, sh, A.ph, rpl);
          __syncthreads();
          if (sh.qn > kStageM - NT) mflush<NT>(sh, A.pl, rpl);
        }
      }
      mflush<NT>(sh, A.pl, rpl);
      group_sync(A.bar, rank, nb);

      // ---- phase 2: pull
      if (tid == 0) {
        sh.nl = (uint32_t)load_agent(rpl);
        const uint64_t hp = load_agent(rpl + 1);
        sh.nh = (uint32_t)(hp >> 32);
        sh.hunits = (uint32_t)hp;
        sh.cnt = 0;
        sh.deg = 0;
        sh.fin = 0;
      }
      __syncthreads();
      {
        constexpr uint32_t VPU = kPullPerWave * NW;
        const uint32_t nchunks = (sh.nl + VPU - 1) / VPU;
        const uint32_t U = nchunks + sh.hunits;
        uint64_t* ticket = ctl + cTQ(L & 3);
        bool firstu = true;
        while (true) {
          if (tid == 0) sh.unit = firstu ? rank : (U > nb ? nb + atomicAdd((uint32_t*)ticket, 1u) : U);
          firstu = false;
          __syncthreads();
          const uint32_t k = sh.unit;
          if (k >= U) break;
          if (k < nchunks) {
            uint64_t fin = 0;
            for (int it = 0; it < kPullPerWave; ++it) {
              const uint32_t i = k * VPU + (uint32_t)(it * NW + wave);
              if (i >= sh.nl) break;
              const int32_t v = A.pl[i];
              const uint64_t vis = A.rec[v].vis, st = A.rec[v].st;
              const uint64_t want = valid & ~vis;
              const int dv = rp[v + 1] - rp[v];
              uint64_t best = kUnvisited;
              if (want) best = pull_edges(G.adj, A.rec, rp[v], rp[v + 1], pp, want, km, best);
              const bool found = best != kUnvisited;
              const uint64_t newb = __ballot(found);
              const uint64_t stb = __ballot(found && (best & 1));
              if (lane == 0) {
                finish_vertex(A, v, vis, st, newb, stb, p, valid, push, dv, fin);
                if (newb) {
                  sh.q[atomicAdd(&sh.qn, 1u)] = v;
                  atomicAdd((unsigned long long*)&sh.cnt, 1ull);
                  atomicAdd((unsigned long long*)&sh.deg, (unsigned long long)dv);
                }
              }
            }
            if (lane == 0 && fin) atomicAdd((unsigned long long*)&sh.fin, (unsigned long long)fin);
          } else {
            // one part of a split row: the block's waves share its edges
            const uint32_t hk = k - nchunks;
            if (tid == 0) {
              int lo = 0, hi = (int)sh.nh;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((uint32_t)A.ph[mid].y <= hk) lo = mid; else hi = mid;
              }
              sh.hidx = lo;
              sh.heavy = A.ph[lo];
            }
            if (tid < 64) sh.hbest[tid] = kUnvisited;
            __syncthreads();
            const int32_t v = sh.heavy.x;
            const uint32_t part = hk - (uint32_t)sh.heavy.y;
            const int64_t e0 = rp[v] + (int64_t)part * kMSplit;
            const int64_t e1 = min<int64_t>(rp[v + 1], e0 + kMSplit);
            const uint64_t want = valid & ~A.rec[v].vis;
            const int64_t seg = ((e1 - e0 + NW - 1) / NW + 63) / 64 * 64;
            const int64_t s0 = min<int64_t>(e1, e0 + (int64_t)wave * seg);
            const int64_t s1 = min<int64_t>(e1, s0 + seg);
            uint64_t best = kUnvisited;
            if (want && s0 < s1) best = pull_edges(G.adj, A.rec, s0, s1, pp, want, km, best);
            if (best != kUnvisited) atomicMin((unsigned long long*)&sh.hbest[lane], (unsigned long long)best);
            __syncthreads();
            if (tid < 64 && sh.hbest[tid] != kUnvisited)
              amin64(A.hslot + (size_t)sh.hidx * 64 + tid, sh.hbest[tid]);
          }
          __syncthreads();
          if (sh.qn > kStageM - VPU) mflush<NT>(sh, fln, rf);
        }
        mflush<NT>(sh, fln, rf);
        if (tid == 0) {
          if (sh.cnt) {
            aadd64(rf + 2, sh.cnt);
            aadd64(rf + 3, sh.deg);
          }
          if (sh.fin) aadd64(ctl + cUNF, (uint64_t)0 - sh.fin);
        }
      }
      const uint32_t nheavy = sh.nh;
      group_sync(A.bar, rank, nb);

      // ---- phase 3: split rows take their minima
      if (nheavy > 0) {
        uint64_t cnt = 0, deg = 0, fin = 0;
        for (int64_t h = gwave; h < (int64_t)nheavy; h += nwaves) {
          const int32_t v = A.ph[h].x;
          uint64_t* hs = A.hslot + (size_t)h * 64;
          const uint64_t best = hs[lane];
          if (best != kUnvisited) hs[lane] = kUnvisited;
          const bool found = best != kUnvisited;
          const uint64_t newb = __ballot(found);
          const uint64_t stb = __ballot(found && (best & 1));
          const int dv = rp[v + 1] - rp[v];
          if (lane == 0) {
            const uint64_t vis = A.rec[v].vis, st = A.rec[v].st;
            finish_vertex(A, v, vis, st, newb, stb, p, valid, push, dv, fin);
          }
          mlist_global(lane == 0 && newb != 0, v, dv, fln, fhn, rf);
          if (newb) {
            cnt += 1;
            deg += (uint64_t)dv;
          }
        }
        if (lane == 0) {
          if (cnt) {
            aadd64(rf + 2, cnt);
            aadd64(rf + 3, deg);
          }
          if (fin) aadd64(ctl + cUNF, (uint64_t)0 - fin);
        }
        group_sync(A.bar, rank, nb);
      }
    }

    // ---- counts and canonical keys of the 64 trees
    {
      if (tid < 192) (&sh.tacc[0][0])[tid] = 0;
      __syncthreads();
      uint64_t c[kPlanes];
#pragma unroll
      for (int b = 0; b < kPlanes; ++b) c[b] = 0;
      uint64_t myS = 0;
      int it = 0;
      auto flush = [&]() {
        for (int t = 0; t < 64; ++t) {
          uint32_t tot = 0;
#pragma unroll
          for (int b = 0; b < kPlanes; ++b)
            tot += (uint32_t)__popcll(__ballot((c[b] >> t) & 1)) << b;
          if (lane == t) myS += tot;
        }
#pragma unroll
        for (int b = 0; b < kPlanes; ++b) c[b] = 0;
      };
      // frustrated iff the edge is negative xor the endpoint states differ
      for (int64_t e0 = (int64_t)rank * NT; e0 < G.m; e0 += sstride) {
        const int64_t e = e0 + tid;
        uint64_t x = 0;
        if (e < G.m) {
          const uint2 uv = G.edges[e];
          x = A.rec[uv.x].st ^ A.rec[uv.y & kVertexMask].st;
          if (uv.y >> 31) x = ~x;
        }
#pragma unroll
        for (int b = 0; b < kPlanes; ++b) {
          const uint64_t carry = c[b] & x;
          c[b] ^= x;
          x = carry;
        }
        if (++it == 255) {
          flush();
          it = 0;
        }
      }
      flush();
      // canonical words: state relative to the component's anchor
      uint64_t khi = 0, klo = 0;
      for (int64_t i = gwave; i < nw; i += nwaves) {
        const int64_t v = i * 64 + lane;
        uint64_t cs = 0;
        if (v < n) cs = A.rec[v].st ^ A.rec[G.comp[v]].st;
        uint64_t W = 0;
        for (int t = 0; t < 64; ++t) {
          const uint64_t b = __ballot((cs >> t) & 1);
          if (lane == t) W = b;
        }
        key_terms((uint64_t)i, W, khi, klo);
      }
      atomicAdd((unsigned long long*)&sh.tacc[0][lane], (unsigned long long)myS);
      atomicAdd((unsigned long long*)&sh.tacc[1][lane], (unsigned long long)khi);
      atomicAdd((unsigned long long*)&sh.tacc[2][lane], (unsigned long long)klo);
      __syncthreads();
      if (tid < 64) {
        aadd64(ctl + cACC + 4 * tid, sh.tacc[0][tid]);
        aadd64(ctl + cACC + 4 * tid + 1, sh.tacc[1][tid]);
        aadd64(ctl + cACC + 4 * tid + 2, sh.tacc[2][tid]);
      }
    }
    group_sync(A.bar, rank, nb);

    // ---- the 64 trees enter the cloud
    if (rank == 0 && tid < nvalid) {
      const uint64_t S = load_agent(ctl + cACC + 4 * tid);
      const uint64_t hi = load_agent(ctl + cACC + 4 * tid + 1);
      const uint64_t lo = load_agent(ctl + cACC + 4 * tid + 2);
      if (A.insert) cloud_insert(G, hi, lo, S, tb + tid);
      if (A.tree_switches) A.tree_switches[tb + tid - A.t0] = S;
    }
    // the next pass clears the control words; finish reading them first
    group_sync(A.bar, rank, nb);
  }
}

template <int NT>
hipError_t launch_mt(fi_graph* g, const MArgs& a, hipStream_t s) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_multi<NT>, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int maxg = per_cu * g->cu_count;
  int grid = g->sched.grid > 0 ? std::min(g->sched.grid, maxg) : maxg;
  if (grid > kBarGroup * 512) grid = kBarGroup * 512;
  DevGraph G = g->dg;
  MArgs A = a;
  void* args[] = {(void*)&G, (void*)&A};
  e = hipLaunchCooperativeKernel((const void*)k_sweep_multi<NT>, dim3(grid), dim3(NT), args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_multi(fi_graph* g, const SweepArgs& sa, hipStream_t s) {
  const Layout& L = g->L;
  char* ws = g->ws;
  MArgs a{};
  a.seed = sa.seed;
  a.t0 = sa.t0;
  a.t1 = sa.t1;
  a.tree_switches = sa.tree_switches;
  a.insert = sa.insert;
  a.ntasks = g->mtasks;
  a.nbig = g->mnbig;
  a.rec = (MRec*)(ws + L.mrec);
  a.unf = (uint64_t*)(ws + L.gvis);
  a.cand = (uint64_t*)(ws + L.gsb);
  a.lstride = (int64_t)g->dg.n + 64;
  a.hstride = (int64_t)L.hcap + 64;
  a.fl = (int32_t*)(ws + L.gql);
  a.pl = a.fl + 2 * a.lstride;
  a.fh = (int2*)(ws + L.gqh);
  a.ph = a.fh + 2 * a.hstride;
  a.hslot = (uint64_t*)(ws + L.mhslot);
  a.tasks = (const int4*)(ws + L.mtasks);
  a.cverts = (const int32_t*)(ws + L.cverts);
  a.rootbig = (uint64_t*)(ws + L.rootbig);
  a.ctl = (uint64_t*)(ws + L.gctl);
  a.bar = (uint64_t*)(ws + L.gbar);
  const int nt = g->sched.block;
  return nt == 1024 ? launch_mt<1024>(g, a, s) : nt == 512 ? launch_mt<512>(g, a, s)
                                                           : launch_mt<256>(g, a, s);
}

}  // namespace fi
