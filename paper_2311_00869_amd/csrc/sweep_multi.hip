// Multi-tree sweep for large graphs: the trees of Alg. alg-index taken 64 W
// at a time (W = 1 or 2 words per vertex), one bit per tree in every
// per-vertex word (word w, bit t is tree t0 + 64 w + t, carried by lane t of
// every wavefront).  A vertex's W words are adjacent, so gathering them costs
// one cache line whatever W is: the pass time grows far less than its tree
// count, and W = 2 sweeps more trees per second.
//
// Per vertex: the trees that discovered it at the last even and at the last
// odd level, its state bits, and the trees that have visited it.  One BFS
// level then serves all 64 W trees with one pass over the rows involved:
//   push - while the frontier is small, its rows mark as candidates every
//          neighbour still unvisited in a tree where the frontier vertex was
//          just discovered;
//   pull - a wave takes 64 entries of the candidate list (or, on large
//          frontiers, of the list of every vertex not yet visited by all
//          trees) and walks their rows, several short rows per 64-edge round;
//          for each vertex lane t keeps the minimum key over the neighbours
//          discovered at the previous level of tree t, which is exactly the
//          single-tree parent rule, and the state bit that comes with it.
//          Rows longer than kMSplit are cut into parts whose minima meet
//          through atomic minima.
// The frontier of a level is its pull list together with a bitmap of the
// entries some tree reached.
// A neighbour's discovery word may still carry bits from two levels back;
// such a tree has already visited every neighbour of that vertex, so the
// bit never survives the mask of unvisited trees and the words need no
// clearing between levels.
// After the BFS, bit-sliced counters over the edge list give every tree's
// frustrated-edge count, 64x64 bit transposes of the state words give its
// canonical key, and the pass's trees enter the cloud.
//
// Memory discipline across XCDs: within one phase a word is either written
// with plain stores by its single owner or updated with atomics, never both.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fi_internal.h"
#include "fi_prims.h"
#include "fi_multi.h"

namespace fi {

namespace {

using namespace mt;

constexpr int kStageM = 2048;      // LDS staging entries for list appends
// Small-row staging entries: each flush is one global reservation, so
// 1,024-thread workgroups (one per CU) stage three times as many; smaller
// workgroups keep kStageM and two workgroups per CU.
template <int NT>
constexpr int stage_small() { return NT >= 1024 ? 3 * kStageM : kStageM; }
constexpr int kPushCost = 32;      // push while kPushCost * frontier edges < unfinished edges
constexpr int kSmall = 32;         // rows up to this many edges are pulled 64 vertices per wave
static_assert(stage_small<1024>() / (kSmall + 1) <= kStageM, "sparse listing: medium rows");
constexpr int kMedChunk = 4;       // medium frontier rows per push unit (at most 8,192 edges)
constexpr int kPlanes = 8;         // bit-sliced counter planes (flushed before 255 edges)
constexpr int kCountBatch = 4;     // edges per lane in flight in the count

// Per-vertex state: one record of four W-word fields per vertex (the trees
// that discovered the vertex at the last even level, its state bits, the
// trees that discovered it at the last odd level, the trees that have
// visited it; 64 bytes at W = 2).  A pull gathers, for every neighbour, the
// previous parity's discovery words and the state words from one record.

// A copy of a per-lane index that the compiler cannot move: addresses derived
// from it are formed where they are used instead of at kernel entry, so they
// do not stay live (and spill) across the pass and level loops.
__device__ __forceinline__ int64_t fresh_index(int64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)((uint64_t)x >> 32);
  asm volatile("v_mov_b32 %0, %0" : "+v"(lo));
  asm volatile("v_mov_b32 %0, %0" : "+v"(hi));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Control words; each group sits on its own 128-byte line.  r = level mod 4.
//   F(r): the level's pull lists and frontier: small-row count, heavy
//         (count << 32 | units), vertices reached, their degree sum,
//         medium-row count
//   TP(r), TQ(r), TM(r): work tickets of the push phase, of the split-row
//         parts and of the medium rows
//   UNF: degree sum of vertices not yet visited by every tree
//   ACC + 4 t: tree t's switches, key_hi, key_lo (t < 64 W)
__host__ __device__ constexpr int cF(int r) { return 16 * r; }
__host__ __device__ constexpr int cTP(int r) { return 128 + 16 * r; }
__host__ __device__ constexpr int cTQ(int r) { return 192 + 16 * r; }
__host__ __device__ constexpr int cTM(int r) { return 384 + 16 * r; }
constexpr int cUNF = 256;
constexpr int cACC = 512;
constexpr int kMCtlWords = 1024;  // ACC holds 4 words for each of up to 128 trees
static_assert(kMCtlWords <= kGridSlots * kGridCtlWords, "control block");

struct MArgs {
  uint64_t seed, t0, t1;
  // the launch's trees in pass order (null: t0, t0 + 1, ...), and with them
  // each tree's root candidate in the component of big-component row
  // main_big, at oroot[tree - t0] (null: searched by the root tasks)
  const uint32_t* perm;
  const uint64_t* oroot;
  int32_t main_big;
  // phase log (null: off): plog[0] counts records; record i is
  // plog[2 + 2 i] = phase << 32 | level and plog[3 + 2 i] = the constant-rate
  // real-time counter (100 MHz), taken by workgroup 0 after each grid barrier
  uint64_t* plog;
  int64_t pcap;
  uint64_t* tree_switches;
  uint64_t* vminus;      // [n] statistics, or null
  uint64_t* eswitch;     // [m] statistics, or null
  int insert;
  int32_t ntasks, nbig;
  MState S;              // per-vertex words and bitmaps of the pass
  int32_t* pl;          // [2][lstride] pull lists of rows up to kSmall (by level parity)
  int32_t* pm;          // [2][lstride] pull lists of rows up to kMSplit
  int2* ph;             // [2][hstride] split rows (vertex, first unit); entry h owns hslot row h
  uint64_t* rl;         // [2][rlstride] entries of pl some tree reached
  uint64_t* rm;         // [2][rlstride] entries of pm some tree reached
  uint64_t* rh;         // [2][rhstride] entries of ph some tree reached
  int64_t lstride, hstride, rlstride, rhstride;
  uint64_t* hslot;      // [rows][64 W] partial minima of split rows
  const int4* tasks;    // root tasks: (begin, end) in cverts, big slot or -1
  const int32_t* cverts;
  uint64_t* rootbig;    // [big components][64 W]
  uint64_t* ctl;
  uint64_t* bar;
};

template <int NT, int W>
struct MS {
  int off[NT];
  int start[NT];
  uint64_t base[NT * W];
  int scan[NT / 64 + 1];
  int32_t q[stage_small<NT>()];  // staging: small rows
  int32_t q2[kStageM];  // staging: medium rows
  uint32_t qn, qn2;
  uint32_t bnext;       // next small-row batch of the block
  uint32_t mnext;       // next medium row of the block
  uint32_t unit;
  int hidx;
  int2 heavy;
  uint64_t cnt, deg, fin;
  int mode, active, sparse;
  uint32_t nl, nm, nh, hunits;
  uint64_t hbest[64 * W];
  uint64_t tacc[3][64 * W];
  TW<W> pw[NT / 64][4 * 64];  // per wave: small rows' wanted trees and outcomes, edge states
  uint64_t pe[NT / 64][kSmall + 1];  // per wave: where the small rows' edges start a row
};

// Move the LDS staging list into a global list (one reservation per block).
template <int NT, class SH>
__device__ __forceinline__ void mflush1(SH& sh, int32_t* q, uint32_t* qn, int32_t* list,
                                        uint64_t* counter) {
  __syncthreads();
  const uint32_t k = *qn;
  if (k) {
    if (threadIdx.x == 0) sh.unit = atomicAdd((uint32_t*)counter, k);
    __syncthreads();
    const uint32_t base = sh.unit;
    for (uint32_t i = threadIdx.x; i < k; i += NT) list[base + i] = q[i];
    __syncthreads();
    if (threadIdx.x == 0) *qn = 0;
  }
  __syncthreads();
}
// both staging lists into the level's small and medium lists
template <int NT, class SH>
__device__ __forceinline__ void mflush(SH& sh, int32_t* ls, int32_t* lm, uint64_t* ring) {
  mflush1<NT>(sh, sh.q, &sh.qn, ls, ring);
  mflush1<NT>(sh, sh.q2, &sh.qn2, lm, ring + 4);
}

// Lanes with `in` list vertex v of degree dv: small and medium rows into
// their LDS staging lists, split rows straight into the heavy list with
// their units.
__device__ __forceinline__ void stage(bool pred, int32_t v, int32_t* q, uint32_t* qn) {
  const uint64_t mask = __ballot(pred);
  if (mask) {
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(qn, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) q[base + lanes_below(mask)] = v;
  }
}
template <class SH>
__device__ __forceinline__ void mlist(bool in, int32_t v, int dv, SH& sh, int2* qh,
                                      uint64_t* ring) {
  const bool heavy = in && dv > kMSplit;
  stage(in && dv <= kSmall, v, sh.q, &sh.qn);
  stage(in && dv > kSmall && !heavy, v, sh.q2, &sh.qn2);
  if (heavy) {
    const uint64_t units = (uint64_t)((dv + kMSplit - 1) / kMSplit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// The same straight into the global lists (no staging).
__device__ __forceinline__ void mlist_global(bool in, int32_t v, int dv, int32_t* ql, int32_t* qm,
                                             int2* qh, uint64_t* ring) {
  const bool heavy = in && dv > kMSplit;
  wave_append(in && dv <= kSmall, v, ql, (uint32_t*)ring);
  wave_append(in && dv > kSmall && !heavy, v, qm, (uint32_t*)(ring + 4));
  if (heavy) {
    const uint64_t units = (uint64_t)((dv + kMSplit - 1) / kMSplit);
    const uint64_t old = atomicAdd((unsigned long long*)(ring + 1),
                                   (unsigned long long)((1ull << 32) | units));
    qh[old >> 32] = make_int2(v, (int)(old & 0xFFFFFFFFull));
  }
}

// Phases of a pass, as logged (fi_prof_phases).
enum : uint32_t {
  kPhReset = 1, kPhRoots = 2, kPhBigRoots = 3, kPhLists = 4, kPhPull = 5, kPhSplit = 6,
  kPhCountKey = 7, kPhInsert = 8
};
__device__ __forceinline__ void log_phase(const MArgs& A, uint32_t rank, uint32_t phase,
                                          uint32_t level) {
  if (A.plog && rank == 0 && threadIdx.x == 0) {
    const uint64_t i = atomicAdd((unsigned long long*)A.plog, 1ull);
    if ((int64_t)(2 + 2 * i + 1) < A.pcap) {
      // formed here: as constants hoisted to kernel entry they would be spilled
      uint32_t hi = phase, lo = level;
      asm volatile("" : "+v"(hi), "+v"(lo));
      A.plog[2 + 2 * i] = ((uint64_t)hi << 32) | lo;
      A.plog[3 + 2 * i] = __builtin_amdgcn_s_memrealtime();
    }
  }
}

// Root vertex r0 of the trees in `mine`: its records, the level-0 lists
// (once; through the block's LDS staging when sh is given, else straight to
// the global lists), and the wave's counters (fin in lane 0: the degree of a
// root already visited by every tree).
template <int W, class SH>
__device__ __forceinline__ void put_root(uint32_t r0, const TW<W>& mine, const TW<W>& valid,
                                         const MArgs& A, const int32_t* rp, uint64_t& cnt,
                                         uint64_t& deg, uint64_t& fin, SH* sh) {
  const int lane = lane_id();
  const int dv = rp[r0 + 1] - rp[r0];
  const bool full = eq_w(mine, valid);
  if (lane == 0) {
    stw_<W>(A.S.nbw[0], r0, mine);
    stw_<W>(A.S.vis, r0, mine);
    if (full) {
      aand64(A.S.unf + (r0 >> 6), ~(1ull << (r0 & 63)));
      put_final<W>(A.S, r0, TW<W>{});  // a root's state is +1 in its trees
      fin += (uint64_t)dv;
    }
  }
  if constexpr (std::is_void_v<SH>) mlist_global(lane == 0, (int32_t)r0, dv, A.pl, A.pm, A.ph, A.ctl + cF(0));
  else mlist(lane == 0, (int32_t)r0, dv, *sh, A.ph, A.ctl + cF(0));
  cnt += 1;
  deg += (uint64_t)dv;
}

// Roots of one component (the wave owns it): each distinct root vertex, over
// all W words, gets the trees it roots in its records and enters the level-0
// lists once.
template <int W, class SH>
__device__ __forceinline__ void set_roots(const uint64_t* best, const bool* vlane,
                                          const TW<W>& valid, const MArgs& A, const int32_t* rp,
                                          uint64_t& cnt, uint64_t& deg, uint64_t& fin, SH* sh) {
  bool ok[W];
  uint32_t r[W];
  uint64_t rem[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    ok[w] = vlane[w] && best[w] != kUnvisited;
    r[w] = (uint32_t)word_vertex(best[w]);
    rem[w] = __ballot(ok[w]);
  }
  while (true) {
    int ww = -1;
#pragma unroll
    for (int w = W - 1; w >= 0; --w)
      if (rem[w]) ww = w;
    if (ww < 0) break;
    uint32_t r0 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
      if (w == ww) r0 = (uint32_t)__builtin_amdgcn_readlane((int)r[w], __builtin_ctzll(rem[w]));
    TW<W> mine;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      mine.w[w] = __ballot(ok[w] && r[w] == r0);
      rem[w] &= ~mine.w[w];
    }
    put_root<W>(r0, mine, valid, A, rp, cnt, deg, fin, sh);
  }
}

// Roots of big components, one wave per (component, tree): the wave of tree t
// takes t's root vertex if no tree before t has the same root.
template <int W>
__device__ __forceinline__ void big_root(const uint64_t* rb, int t, const bool* vlane,
                                         const TW<W>& valid, const MArgs& A, const int32_t* rp,
                                         uint64_t& cnt, uint64_t& deg, uint64_t& fin) {
  uint64_t best[W];
  uint32_t r[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    best[w] = vlane[w] ? rb[64 * w + lane_id()] : kUnvisited;
    r[w] = (uint32_t)word_vertex(best[w]);
  }
  uint32_t rt = 0;
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (w == t / 64) rt = (uint32_t)__builtin_amdgcn_readlane((int)r[w], t % 64);
  TW<W> mine;
  int first = -1;
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    mine.w[w] = __ballot(vlane[w] && best[w] != kUnvisited && r[w] == rt);
    if (mine.w[w]) first = 64 * w + __builtin_ctzll(mine.w[w]);
  }
  if (first == t) put_root<W, void>(rt, mine, valid, A, rp, cnt, deg, fin, nullptr);
}

template <int NT, bool STATS, int W>
__global__ void __launch_bounds__(NT) k_sweep_multi(DevGraph G, MArgs A) {
  __shared__ MS<NT, W> sh;
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const uint32_t rank = blockIdx.x, nb = gridDim.x;
  const int64_t stid = (int64_t)rank * NT + tid, sstride = (int64_t)nb * NT;
  const int64_t gwave = stid >> 6, nwaves = sstride >> 6;
  const int32_t n = G.n, nw = G.nwords;
  const int32_t* rp = G.row_ptr;
  uint64_t* ctl = A.ctl;

  log_phase(A, rank, 0, 0);  // launch start
  const uint64_t ntrees = A.t1 - A.t0;
  // the tree carried by slot i of the launch
  auto tree_of = [&](uint64_t i) -> uint64_t { return A.perm ? (uint64_t)A.perm[i] : A.t0 + i; };
  for (uint64_t sb = 0; sb < ntrees; sb += 64 * W) {
    const int nvalid = (int)min<uint64_t>(64 * W, ntrees - sb);
    TW<W> valid;
    bool vlane[W];
    KeyMix km[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int nv = nvalid - 64 * w;
      valid.w[w] = nv >= 64 ? ~0ull : nv > 0 ? ((1ull << nv) - 1) : 0ull;
      vlane[w] = lane < nv;
      km[w] = key_mix(tree_salt(A.seed, vlane[w] ? tree_of(sb + 64 * w + lane) : A.t0));
    }

    // ---- reset: records, bitmaps, control words
    const int64_t ptid = fresh_index(stid);
    for (int64_t v = ptid; v < (int64_t)n * W * kRecFields; v += sstride) A.S.nbw[0][v] = 0;
    for (int64_t i = ptid; i < nw; i += sstride) {
      A.S.unf[i] = G.word_mask[i];
      A.S.cand[i] = 0;
    }
    // big components' root minima (read by several waves each, so cleared
    // here); the main component's come found already when oroot is given
    for (int64_t i = ptid; i < (int64_t)A.nbig * 64 * W; i += sstride) {
      uint64_t r = kUnvisited;
      if (A.oroot && i / (64 * W) == A.main_big) {
        const int t = (int)(i % (64 * W));
        if (t < nvalid) r = A.oroot[tree_of(sb + t) - A.t0];
      }
      A.rootbig[i] = r;
    }
    if (rank == 0)
      for (int i = tid; i < kMCtlWords; i += NT) ctl[i] = i == cUNF ? (uint64_t)G.nnz : 0ull;
    if (tid == 0) {
      sh.qn = 0;
      sh.qn2 = 0;
    }
    group_sync(A.bar, rank, nb);
    log_phase(A, rank, kPhReset, 0);

    // ---- roots: the minimum key of every component, per tree; they form
    // the lists of level 0, all reached
    {
      uint64_t cnt = 0, deg = 0, fin = 0;
      // a round of one task per wave, then the block's staged level-0 list
      // entries go out with one reservation (at most 64 W roots per wave fit
      // the staging lists); the loop bound is uniform over the block
      for (int64_t k0 = (int64_t)rank * NW; k0 < A.ntasks; k0 += nwaves) {
        const int64_t k = k0 + wave;
        const int4 tk = k < A.ntasks ? A.tasks[k] : make_int4(0, 0, -2, 0);
        if (k < A.ntasks && !(A.oroot && tk.z == A.main_big)) {
          uint64_t best[W];
          comp_min_w<W>(A.cverts, tk.x, tk.y, km, best);
          if (tk.z < 0) {
            set_roots<W>(best, vlane, valid, A, rp, cnt, deg, fin, &sh);
          } else {
#pragma unroll
            for (int w = 0; w < W; ++w)
              if (vlane[w] && best[w] != kUnvisited)
                amin64(A.rootbig + (size_t)tk.z * 64 * W + 64 * w + lane, best[w]);
          }
        }
        mflush<NT>(sh, A.pl, A.pm, A.ctl + cF(0));
      }
      group_sync(A.bar, rank, nb);
      log_phase(A, rank, kPhRoots, 0);
      for (int64_t it = gwave; it < (int64_t)A.nbig * 64 * W; it += nwaves) {
        const int t = (int)(it % (64 * W));
        if (t < nvalid)
          big_root<W>(A.rootbig + (size_t)(it / (64 * W)) * 64 * W, t, vlane, valid, A, rp, cnt, deg,
                      fin);
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
    log_phase(A, rank, kPhBigRoots, 0);

    // ---- levels
    for (uint32_t L = 1;; ++L) {
      const int pp = (int)((L - 1) & 1), p = (int)(L & 1);
      uint64_t* rfp = ctl + cF((L - 1) & 3);
      uint64_t* rf = ctl + cF(L & 3);
      // lists and frontier of level L-1
      const int32_t* plp = A.pl + (size_t)pp * A.lstride;
      const int32_t* pmp = A.pm + (size_t)pp * A.lstride;
      const int2* php = A.ph + (size_t)pp * A.hstride;
      const uint64_t* rlp = A.rl + (size_t)pp * A.rlstride;
      const uint64_t* rmp = A.rm + (size_t)pp * A.rlstride;
      const uint64_t* rhp = A.rh + (size_t)pp * A.rhstride;
      // lists of level L
      int32_t* pln = A.pl + (size_t)p * A.lstride;
      int32_t* pmn = A.pm + (size_t)p * A.lstride;
      int2* phn = A.ph + (size_t)p * A.hstride;
      uint64_t* rln = A.rl + (size_t)p * A.rlstride;
      uint64_t* rmn = A.rm + (size_t)p * A.rlstride;
      uint64_t* rhn = A.rh + (size_t)p * A.rhstride;
      const bool all_reached = L == 1;  // level 0 lists only roots
      if (tid == 0) {
        sh.nl = (uint32_t)load_agent(rfp);
        sh.nm = (uint32_t)load_agent(rfp + 4);
        const uint64_t hp = load_agent(rfp + 1);
        sh.nh = (uint32_t)(hp >> 32);
        sh.hunits = (uint32_t)hp;
        const uint64_t reached = load_agent(rfp + 2), fdeg = load_agent(rfp + 3);
        const uint64_t unf = load_agent(ctl + cUNF);
        sh.active = reached > 0;
        sh.mode = (uint64_t)kPushCost * fdeg < unf ? 1 : 2;
        // every unfinished vertex has an edge, so unf bounds their number
        sh.sparse = unf <= (uint64_t)stage_small<NT>();
      }
      __syncthreads();
      if (!uni(sh.active)) break;
      const bool push = uni(sh.mode) == 1;
      // counters and tickets of level L + 1 start from zero
      if (rank == 0 && tid < 8) {
        const int r = (int)((L + 1) & 3);
        ctl[cF(r) + tid] = 0;
        if (tid == 0) {
          ctl[cTP(r)] = 0;
          ctl[cTQ(r)] = 0;
          ctl[cTM(r)] = 0;
        }
      }
      // medium and split rows set their reached bits with atomics
      const int64_t ltid = fresh_index(stid);
      for (int64_t i = ltid; i < A.rlstride; i += sstride) rmn[i] = 0;
      for (int64_t i = ltid; i < A.rhstride; i += sstride) rhn[i] = 0;

      // ---- phase 1: the pull lists of level L
      if (push) {
        // the rows of the frontier mark their unvisited neighbours
        // units: chunks of NT small rows, chunks of kMedChunk medium rows,
        // then the parts of split rows
        const uint32_t nlp = uni(sh.nl), nmp = uni(sh.nm);
        const uint32_t nsc = (nlp + NT - 1) / NT;
        const uint32_t nchunks = nsc + (nmp + kMedChunk - 1) / kMedChunk;
        const uint32_t U = nchunks + uni(sh.hunits);
        uint64_t* ticket = ctl + cTP(L & 3);
        bool firstu = true;
        while (true) {
          if (tid == 0) sh.unit = firstu ? rank : (U > nb ? nb + atomicAdd((uint32_t*)ticket, 1u) : U);
          firstu = false;
          __syncthreads();
          const uint32_t k = uni(sh.unit);
          if (k >= U) break;
          int total = 0;
          int64_t e0 = 0;
          TW<W> hbits{};
          if (k < nchunks) {
            int d = 0, st = 0;
            TW<W> bits{};
            int32_t u = -1;
            if (k < nsc) {
              const uint32_t i = k * NT + tid;
              if (i < nlp && (all_reached || ((rlp[i >> 6] >> (i & 63)) & 1))) u = plp[i];
            } else if (tid < kMedChunk) {
              const uint32_t i = (k - nsc) * kMedChunk + tid;
              if (i < nmp && (all_reached || ((rmp[i >> 6] >> (i & 63)) & 1))) u = pmp[i];
            }
            if (u >= 0) {
              st = rp[u];
              d = rp[u + 1] - st;
              const TW<W> nbu = ldw<W>(A.S.nbw[pp], u);
#pragma unroll
              for (int w = 0; w < W; ++w) bits.w[w] = nbu.w[w] & valid.w[w];
            }
            const int off = block_exclusive_scan<NT>(d, total, sh.scan);
            sh.off[tid] = off;
            sh.start[tid] = st;
#pragma unroll
            for (int w = 0; w < W; ++w) sh.base[tid * W + w] = bits.w[w];
            __syncthreads();
            total = uni(total);
          } else {
            const uint32_t hk = k - nchunks;
            if (tid == 0) {
              int lo = 0, hi = (int)sh.nh;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((uint32_t)php[mid].y <= hk) lo = mid; else hi = mid;
              }
              sh.hidx = lo;
              sh.heavy = php[lo];
            }
            __syncthreads();
            const int hidx = uni(sh.hidx);
            if (all_reached || ((rhp[hidx >> 6] >> (hidx & 63)) & 1)) {
              const int32_t u = uni(sh.heavy.x);
              const uint32_t part = hk - (uint32_t)uni(sh.heavy.y);
              e0 = rp[u] + (int64_t)part * kMSplit;
              const int64_t e1 = min<int64_t>(rp[u + 1], e0 + kMSplit);
              const TW<W> nbu = ldw<W>(A.S.nbw[pp], u);
#pragma unroll
              for (int w = 0; w < W; ++w) hbits.w[w] = nbu.w[w] & valid.w[w];
              total = (int)(e1 - e0);
            }
          }
          for (int j0 = 0; j0 < total; j0 += NT) {
            const int j = j0 + tid;
            bool first = false;
            int32_t v = 0;
            int dv = 0;
            if (j < total) {
              uint32_t a;
              TW<W> bits;
              if (k < nchunks) {
                const int kk = upper_index(sh.off, NT, j);
                a = G.adj[sh.start[kk] + (j - sh.off[kk])];
#pragma unroll
                for (int w = 0; w < W; ++w) bits.w[w] = sh.base[kk * W + w];
              } else {
                a = G.adj[e0 + j];
                bits = hbits;
              }
              v = (int32_t)(a & kVertexMask);
              if (any_w(and_not(bits, ldw<W>(A.S.vis, v)))) {
                const uint64_t bit = 1ull << (v & 63);
                if (!(aor64(A.S.cand + (v >> 6), bit) & bit)) {
                  first = true;
                  dv = rp[v + 1] - rp[v];
                }
              }
            }
            mlist(first, v, dv, sh, phn, rf);
            __syncthreads();
            if (sh.qn > stage_small<NT>() - NT || sh.qn2 > kStageM - NT)
              mflush<NT>(sh, pln, pmn, rf);
          }
          __syncthreads();
        }
      } else if (uni(sh.sparse)) {
        // every vertex some tree has not visited yet, when they are at most as
        // many as a workgroup's small-row staging holds (medium rows, of more
        // than kSmall edges, are then fewer than its medium-row staging holds),
        // so that no workgroup's staging can overflow: each wave reads 64
        // bitmap words at once and lists the vertices of the nonzero ones,
        // with no barrier between words
        const int64_t wstep = (int64_t)nb * NW;
        for (int64_t x0 = (int64_t)rank * NW + wave; x0 < nw; x0 += 64 * wstep) {
          const int64_t x = x0 + (int64_t)lane * wstep;
          const uint64_t bx = x < nw ? A.S.unf[x] : 0ull;
          uint64_t nz = __ballot(bx != 0ull);
          while (nz) {
            const int k = __builtin_ctzll(nz);
            nz &= nz - 1;
            const uint64_t bits = readlane64(bx, k);
            const int64_t vx = (x0 + (int64_t)k * wstep) * 64 + lane;
            const bool in = (bits >> lane) & 1;
            mlist(in, (int32_t)vx, in ? rp[vx + 1] - rp[vx] : 0, sh, phn, rf);
          }
        }
      } else {
        // every vertex some tree has not visited yet; the bitmap word and the
        // row offsets of a wave's next word are read while its current word's
        // vertices are listed (nothing writes the bitmap in this phase)
        const int64_t wstep = (int64_t)nb * NW;
        int64_t w = (int64_t)rank * NW + wave;
        auto fetch = [&](int64_t x, uint64_t& bx, int32_t& lo, int32_t& hi) {
          const int64_t vx = x * 64 + lane;
          const bool ok = x < nw && vx < n;
          bx = x < nw ? A.S.unf[x] : 0ull;
          lo = ok ? rp[vx] : 0;
          hi = ok ? rp[vx + 1] : 0;
        };
        uint64_t bits;
        int32_t r0, r1;
        fetch(w, bits, r0, r1);
        for (int64_t c0 = (int64_t)rank * NW; c0 < nw; c0 += wstep) {
          uint64_t bn;
          int32_t q0, q1;
          fetch(w + wstep, bn, q0, q1);
          const bool in = (bits >> lane) & 1;
          const int32_t v = (int32_t)(w * 64 + lane);
          mlist(in, v, in ? r1 - r0 : 0, sh, phn, rf);
          __syncthreads();
          if (sh.qn > stage_small<NT>() - NT || sh.qn2 > kStageM - NT)
            mflush<NT>(sh, pln, pmn, rf);
          w += wstep;
          bits = bn;
          r0 = q0;
          r1 = q1;
        }
      }
      mflush<NT>(sh, pln, pmn, rf);
      group_sync(A.bar, rank, nb);
      log_phase(A, rank, kPhLists, L);

      // ---- phase 2: pull
      if (tid == 0) {
        sh.nl = (uint32_t)load_agent(rf);
        sh.nm = (uint32_t)load_agent(rf + 4);
        const uint64_t hp = load_agent(rf + 1);
        sh.nh = (uint32_t)(hp >> 32);
        sh.hunits = (uint32_t)hp;
        sh.cnt = 0;
        sh.deg = 0;
        sh.fin = 0;
        sh.bnext = 0;
        sh.mnext = 0;
      }
      __syncthreads();
      {
        uint64_t cnt = 0, deg = 0, fin = 0;
        // small rows: 64 list entries per wave, whole bitmap words; block b
        // owns batches b, b + nb, ... and its waves draw them one at a time
        const int64_t nl = (int64_t)uni(sh.nl);
        while (true) {
          uint32_t i = 0;
          if (lane == 0) i = atomicAdd(&sh.bnext, 1u);
          const int64_t b = (int64_t)rank + (int64_t)uni((int)i) * nb;
          if (b * 64 >= nl) break;
          const int ne = (int)min<int64_t>(64, nl - b * 64);
          const uint64_t r =
              pull_small_w<W, kSmall>(G, A.S, b * 64 + lane < nl ? pln[b * 64 + lane] : 0, ne, pp,
                                      p, valid, km, push, sh.pw[wave], sh.pe[wave], cnt, deg, fin);
          if (lane == 0) rln[b] = r;
        }
        // medium rows: block b owns rows b, b + nb, ...; its waves draw them
        // one at a time and walk each with all lanes
        {
          const uint32_t nm = uni(sh.nm);
          while (true) {
            uint32_t c = 0;
            if (lane == 0) c = atomicAdd(&sh.mnext, 1u);
            const int64_t i = (int64_t)rank + (int64_t)uni((int)c) * nb;
            if (i >= (int64_t)nm) break;
            const int32_t v = pmn[i];
            const int64_t e0 = rp[v], e1 = rp[v + 1];
            const TW<W> want = uni_w(and_not(valid, ldw<W>(A.S.vis, v)));  // v is the wave's
            uint64_t best[W];
#pragma unroll
            for (int w = 0; w < W; ++w) best[w] = kUnvisited;
            if (any_w(want)) pull_edges_w<W>(G.adj, A.S.nbw[pp], A.S.stw, e0, e1, want, km, best);
            TW<W> mnew, mstb;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              mnew.w[w] = __ballot(best[w] != kUnvisited);
              mstb.w[w] = __ballot(best[w] != kUnvisited && (best[w] & 1));
            }
            const int dq = (int)(e1 - e0);
            if (any_w(mnew)) {
              const TW<W> visq = ldw<W>(A.S.vis, v), stq = ldw<W>(A.S.stw, v);
              const TW<W> nv = or_w(visq, mnew);
              const bool full = eq_w(nv, valid);
              if (lane == 0) {
                stw_<W>(A.S.vis, v, nv);
                stw_<W>(A.S.nbw[p], v, mnew);
                if (any_w(mstb)) stw_<W>(A.S.stw, v, or_w(stq, mstb));
                if (full) {
                  aand64(A.S.unf + (v >> 6), ~(1ull << (v & 63)));
                  put_final<W>(A.S, v, or_w(stq, mstb));
                }
                aor64(rmn + (i >> 6), 1ull << (i & 63));
              }
              cnt += 1;
              deg += (uint64_t)dq;
              if (full) fin += (uint64_t)dq;
            }
            if (push && lane == 0) aand64(A.S.cand + (v >> 6), ~(1ull << (v & 63)));
          }
        }
        if (lane == 0 && cnt) {
          atomicAdd((unsigned long long*)&sh.cnt, (unsigned long long)cnt);
          atomicAdd((unsigned long long*)&sh.deg, (unsigned long long)deg);
        }
        if (lane == 0 && fin) atomicAdd((unsigned long long*)&sh.fin, (unsigned long long)fin);
        // parts of split rows: the block's waves share each part's edges
        const uint32_t U = uni(sh.hunits);
        uint64_t* ticket = ctl + cTQ(L & 3);
        bool firstu = true;
        while (true) {
          __syncthreads();
          if (tid == 0) sh.unit = firstu ? rank : (U > nb ? nb + atomicAdd((uint32_t*)ticket, 1u) : U);
          firstu = false;
          __syncthreads();
          const uint32_t hk = uni(sh.unit);
          if (hk >= U) break;
          if (tid == 0) {
            int lo = 0, hi = (int)sh.nh;
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if ((uint32_t)phn[mid].y <= hk) lo = mid; else hi = mid;
            }
            sh.hidx = lo;
            sh.heavy = phn[lo];
          }
          if (tid < 64 * W) sh.hbest[tid] = kUnvisited;
          __syncthreads();
          const int32_t v = uni(sh.heavy.x);
          const uint32_t part = hk - (uint32_t)uni(sh.heavy.y);
          const int64_t e0 = rp[v] + (int64_t)part * kMSplit;
          const int64_t e1 = min<int64_t>(rp[v + 1], e0 + kMSplit);
          const TW<W> want = uni_w(and_not(valid, ldw<W>(A.S.vis, v)));  // v is the block's
          const int64_t seg = ((e1 - e0 + NW - 1) / NW + 63) / 64 * 64;
          const int64_t s0 = min<int64_t>(e1, e0 + (int64_t)wave * seg);
          const int64_t s1 = min<int64_t>(e1, s0 + seg);
          uint64_t best[W];
#pragma unroll
          for (int w = 0; w < W; ++w) best[w] = kUnvisited;
          if (any_w(want) && s0 < s1)
            pull_edges_w<W>(G.adj, A.S.nbw[pp], A.S.stw, s0, s1, want, km, best);
#pragma unroll
          for (int w = 0; w < W; ++w)
            if (best[w] != kUnvisited)
              atomicMin((unsigned long long*)&sh.hbest[64 * w + lane], (unsigned long long)best[w]);
          __syncthreads();
          if (tid < 64 * W && sh.hbest[tid] != kUnvisited)
            amin64(A.hslot + (size_t)sh.hidx * 64 * W + tid, sh.hbest[tid]);
        }
        __syncthreads();
        if (tid == 0) {
          if (sh.cnt) {
            aadd64(rf + 2, sh.cnt);
            aadd64(rf + 3, sh.deg);
          }
          if (sh.fin) aadd64(ctl + cUNF, (uint64_t)0 - sh.fin);
        }
      }
      const uint32_t nheavy = uni(sh.nh);
      group_sync(A.bar, rank, nb);
      log_phase(A, rank, kPhPull, L);

      // ---- phase 3: split rows take their minima (one wave per row)
      if (nheavy > 0) {
        uint64_t cnt = 0, deg = 0, fin = 0;
        for (int64_t h = gwave; h < (int64_t)nheavy; h += nwaves) {
          const int32_t v = phn[h].x;
          uint64_t* hs = A.hslot + (size_t)h * 64 * W;
          uint64_t best[W];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            best[w] = hs[64 * w + lane];
            if (best[w] != kUnvisited) hs[64 * w + lane] = kUnvisited;
          }
          const TW<W> vis = ldw<W>(A.S.vis, v), st = ldw<W>(A.S.stw, v);
          const int dv = rp[v + 1] - rp[v];
          if (settle_w<W>(A.S, v, vis, st, dv, best, p, valid, cnt, deg, fin) && lane == 0)
            aor64(rhn + (h >> 6), 1ull << (h & 63));
          if (push && lane == 0) aand64(A.S.cand + (v >> 6), ~(1ull << (v & 63)));
        }
        if (lane == 0) {
          if (cnt) {
            aadd64(rf + 2, cnt);
            aadd64(rf + 3, deg);
          }
          if (fin) aadd64(ctl + cUNF, (uint64_t)0 - fin);
        }
        group_sync(A.bar, rank, nb);
        log_phase(A, rank, kPhSplit, L);
      }
    }

    // ---- counts and canonical keys of the 64 W trees
    {
      for (int i = tid; i < 3 * 64 * W; i += NT) (&sh.tacc[0][0])[i] = 0;
      __syncthreads();
      uint64_t myS[W];
#pragma unroll
      for (int w = 0; w < W; ++w) myS[w] = 0;
      {
        uint64_t c[W][kPlanes];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int b = 0; b < kPlanes; ++b) c[w][b] = 0;
        int it = 0;
        auto flush = [&]() {
#pragma unroll
          for (int w = 0; w < W; ++w) {
            for (int t = 0; t < 64; ++t) {
              uint32_t tot = 0;
#pragma unroll
              for (int b = 0; b < kPlanes; ++b)
                tot += (uint32_t)__popcll(__ballot((c[w][b] >> t) & 1)) << b;
              if (lane == t) myS[w] += tot;
            }
#pragma unroll
            for (int b = 0; b < kPlanes; ++b) c[w][b] = 0;
          }
        };
        // frustrated iff the edge is negative xor the endpoint states differ;
        // kCountBatch edges per lane at a time keep that many gather chains in
        // flight (past the end a lane reads vertex 0 and adds nothing).  The
        // per-edge statistics follow the edge list's order; the plain count
        // takes the counting list, whose gathers land on high-degree vertices
        const uint2* ce = STATS ? G.edges : G.cedges;
        for (int64_t e0 = (int64_t)rank * NT * kCountBatch; e0 < G.m;
             e0 += sstride * kCountBatch) {
          uint2 uv[kCountBatch];
#pragma unroll
          for (int k = 0; k < kCountBatch; ++k) {
            const int64_t e = e0 + (int64_t)k * NT + tid;
            uv[k] = e < G.m ? ce[e] : make_uint2(0u, 0u);
          }
          TW<W> su[kCountBatch], sv[kCountBatch];
#pragma unroll
          for (int k = 0; k < kCountBatch; ++k) {
            su[k] = get_final<W>(A.S.stc, uv[k].x);
            sv[k] = get_final<W>(A.S.stc, uv[k].y & kVertexMask);
          }
#pragma unroll
          for (int k = 0; k < kCountBatch; ++k) {
            const int64_t e = e0 + (int64_t)k * NT + tid;
            TW<W> x{};
            if (e < G.m) {
              const uint64_t neg = (uv[k].y >> 31) ? ~0ull : 0ull;
#pragma unroll
              for (int w = 0; w < W; ++w) x.w[w] = su[k].w[w] ^ sv[k].w[w] ^ neg;
              // one owner per edge word in every pass
              if constexpr (STATS) {
                if (A.eswitch) {
                  uint64_t c1 = 0;
#pragma unroll
                  for (int w = 0; w < W; ++w) c1 += (uint64_t)__popcll(x.w[w] & valid.w[w]);
                  A.eswitch[e] += c1;
                }
              }
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
              uint64_t xw = x.w[w];
#pragma unroll
              for (int b = 0; b < kPlanes; ++b) {
                const uint64_t carry = c[w][b] & xw;
                c[w][b] ^= xw;
                xw = carry;
              }
            }
          }
          it += kCountBatch;
          if (it + kCountBatch > 255) {
            flush();
            it = 0;
          }
        }
        flush();
      }
      // canonical words: state relative to the component's anchor
      uint64_t khi[W], klo[W];
#pragma unroll
      for (int w = 0; w < W; ++w) khi[w] = klo[w] = 0;
      for (int64_t i = gwave; i < nw; i += nwaves) {
        const int64_t v = i * 64 + lane;
        TW<W> cs{};
        if (v < n) {
          // an isolated vertex is its own anchor (its copy is never written)
          const TW<W> a = get_final<W>(A.S.stc, v), b = get_final<W>(A.S.stc, G.comp[v]);
#pragma unroll
          for (int w = 0; w < W; ++w) cs.w[w] = a.w[w] ^ b.w[w];
        }
        if constexpr (STATS) {
          if (A.vminus && v < n) {
            uint64_t k = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) k += (uint64_t)__popcll(cs.w[w] & valid.w[w]);
            A.vminus[v] += k;
          }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) key_terms((uint64_t)i, transpose64(cs.w[w]), khi[w], klo[w]);
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        atomicAdd((unsigned long long*)&sh.tacc[0][64 * w + lane], (unsigned long long)myS[w]);
        atomicAdd((unsigned long long*)&sh.tacc[1][64 * w + lane], (unsigned long long)khi[w]);
        atomicAdd((unsigned long long*)&sh.tacc[2][64 * w + lane], (unsigned long long)klo[w]);
      }
      __syncthreads();
      for (int t = tid; t < 64 * W; t += NT) {
        aadd64(ctl + cACC + 4 * t, sh.tacc[0][t]);
        aadd64(ctl + cACC + 4 * t + 1, sh.tacc[1][t]);
        aadd64(ctl + cACC + 4 * t + 2, sh.tacc[2][t]);
      }
    }
    group_sync(A.bar, rank, nb);
    log_phase(A, rank, kPhCountKey, 0);

    // ---- the trees of the pass enter the cloud
    if (rank == 0 && tid < nvalid) {
      const uint64_t S = load_agent(ctl + cACC + 4 * tid);
      const uint64_t hi = load_agent(ctl + cACC + 4 * tid + 1);
      const uint64_t lo = load_agent(ctl + cACC + 4 * tid + 2);
      const uint64_t t = tree_of(sb + tid);
      if (A.insert) cloud_insert(G, hi, lo, S, t);
      if (A.tree_switches) A.tree_switches[t - A.t0] = S;
    }
    // the next pass clears the control words; finish reading them first
    group_sync(A.bar, rank, nb);
    log_phase(A, rank, kPhInsert, 0);
  }
}

template <int NT, bool STATS, int W>
hipError_t launch_mt(fi_graph* g, const MArgs& a, hipStream_t s) {
  int per_cu = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_multi<NT, STATS, W>, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int maxg = per_cu * g->cu_count;
  // by default one workgroup per 16,384 of n + m/2, a multiple of 8 (the
  // XCDs), at least 64: on graphs of 10^5 vertices most of a level is its grid
  // barriers, and 64 workgroups ran 1.5 to 1.7 times faster than 256
  const int64_t work = (int64_t)g->dg.n + g->dg.m / 2;
  const int auto_grid = (int)std::max<int64_t>(64, std::min<int64_t>(maxg, work / 16384) & ~7);
  int grid = std::min(g->sched.grid > 0 ? g->sched.grid : auto_grid, maxg);
  if (grid > kBarGroup * 512) grid = kBarGroup * 512;
  DevGraph G = g->dg;
  MArgs A = a;
  void* args[] = {(void*)&G, (void*)&A};
  e = hipLaunchCooperativeKernel((const void*)k_sweep_multi<NT, STATS, W>, dim3(grid), dim3(NT),
                                 args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <bool STATS, int W>
hipError_t launch_mt_block(fi_graph* g, const MArgs& a, hipStream_t s) {
  // the automatic schedule runs full 1,024-thread workgroups
  const int nt = g->sched.path == 0 ? 1024 : g->sched.block;
  return nt == 1024 ? launch_mt<1024, STATS, W>(g, a, s)
         : nt == 512 ? launch_mt<512, STATS, W>(g, a, s)
                     : launch_mt<256, STATS, W>(g, a, s);
}

}  // namespace

// words: tree words per vertex (1: 64 trees per pass, 2: 128)
hipError_t launch_multi(fi_graph* g, const SweepArgs& sa, int words, hipStream_t s) {
  const Layout& L = g->L;
  char* ws = g->ws;
  MArgs a{};
  a.seed = sa.seed;
  a.t0 = sa.t0;
  a.t1 = sa.t1;
  a.tree_switches = sa.tree_switches;
  a.vminus = sa.vminus;
  a.eswitch = sa.eswitch;
  a.insert = sa.insert;
  a.ntasks = g->mtasks;
  a.nbig = g->mnbig;
  // one record of kRecFields fields of `words` words per vertex
  a.S.nbw[0] = (uint64_t*)(ws + L.mrec);
  a.S.stw = a.S.nbw[0] + words;
  a.S.nbw[1] = a.S.nbw[0] + 2 * words;
  a.S.vis = a.S.nbw[0] + 3 * words;
  a.S.unf = (uint64_t*)(ws + L.gvis);
  a.S.cand = (uint64_t*)(ws + L.gsb);
  // the final-state copy sits in the whole-grid path's tree words (8 words a
  // vertex per slot, never in use at the same time)
  a.S.stc = (uint64_t*)(ws + L.gpw);
  a.lstride = (int64_t)g->dg.n + 64;
  a.hstride = (int64_t)L.hcap + 64;
  a.rlstride = a.lstride / 64 + 2;
  a.rhstride = (int64_t)L.mhcap / 64 + 2;
  a.pl = (int32_t*)(ws + L.gql);
  a.pm = a.pl + 2 * a.lstride;
  a.ph = (int2*)(ws + L.gqh);
  a.rl = (uint64_t*)(ws + L.mreach);
  a.rm = a.rl + 2 * a.rlstride;
  a.rh = a.rm + 2 * a.rlstride;
  a.hslot = (uint64_t*)(ws + L.mhslot);
  a.tasks = (const int4*)(ws + L.mtasks);
  a.cverts = (const int32_t*)(ws + L.cverts);
  a.rootbig = (uint64_t*)(ws + L.rootbig);
  a.ctl = (uint64_t*)(ws + L.gctl);
  a.bar = (uint64_t*)(ws + L.gbar);
  a.perm = nullptr;
  a.oroot = nullptr;
  a.main_big = g->main_big;
  a.plog = g->plog;
  a.pcap = g->pcap;
  const bool stats = a.vminus || a.eswitch;
  auto run = [&](const MArgs& m) {
    if (words == 2)
      return stats ? launch_mt_block<true, 2>(g, m, s) : launch_mt_block<false, 2>(g, m, s);
    return stats ? launch_mt_block<true, 1>(g, m, s) : launch_mt_block<false, 1>(g, m, s);
  };
  // more than one pass: trees in blocks of up to kOrderMax, each taken in
  // the order of order_trees (same results, fewer steps per pass)
  if (!g->cent || sa.t1 - sa.t0 <= (uint64_t)(64 * words)) return run(a);
  for (uint64_t b0 = sa.t0; b0 < sa.t1; b0 += kOrderMax) {
    const uint64_t b1 = std::min<uint64_t>(sa.t1, b0 + kOrderMax);
    hipError_t e = order_trees(g, sa.seed, b0, (uint32_t)(b1 - b0), s);
    if (e != hipSuccess) return e;
    MArgs m = a;
    m.t0 = b0;
    m.t1 = b1;
    m.perm = (const uint32_t*)(ws + L.operm);
    m.oroot = (const uint64_t*)(ws + L.oroot);
    m.tree_switches = sa.tree_switches ? sa.tree_switches + (b0 - sa.t0) : nullptr;
    e = run(m);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fi
