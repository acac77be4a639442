// Device helpers of the multi-tree sweep: 64 W trees per pass, one bit per
// tree in the W-word fields of each vertex's record, lane t of a wavefront
// carrying trees t, 64 + t, ...  Shared by the whole-grid sweep of one large
// graph (sweep_multi.hip, W = 1 or 2) and the workgroup-per-graph sweep of
// batches (batch.hip, W = 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fi_internal.h"
#include "fi_prims.h"

namespace fi {
namespace mt {

// Per-vertex state of one pass: the trees that discovered the vertex at the
// last even / odd level, its state bits and the trees that have visited it
// (the fields of the vertex records, below); the vertices with an edge not yet
// visited by every tree, and the push candidates of the level (n/64 words
// each).
struct MState {
  uint64_t* nbw[2];
  uint64_t* stw;
  uint64_t* vis;
  uint64_t* unf;
  uint64_t* cand;
  // final states, W words per vertex side by side, written when the vertex
  // is visited by every tree (null: not kept)
  uint64_t* stc;
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

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Lane t's bit of a wave-uniform mask, taken as the execution mask.
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// A neighbour's candidate in the trees it reaches: its key in the high half,
// so that the unsigned order is the key's (the neighbours of one vertex have
// distinct keys).  While a chunk of 64 edges is walked, the low half holds
// kPending | the neighbour's lane in the chunk; once the chunk is walked, the
// minimum's low half becomes the state it hands down (0 or 1).  No candidate
// equals kUnvisited.
constexpr uint32_t kPending = 0x40;

// best = min(best, key << 32 | lo) for a key that no other candidate of best's
// vertex and tree shares: comparing the high halves alone suffices, and a key
// equal to kUnvisited's high half replaces it.
__device__ __forceinline__ void take_min(uint64_t& best, uint32_t key, uint32_t lo) {
  if (key <= (uint32_t)(best >> 32)) best = ((uint64_t)key << 32) | lo;
}

// One hit edge j of a row walk (the neighbour's key hash Hj, the candidate's
// low half lo): every lane computes its tree's key and keeps it as in
// take_min if its tree is in the edge's tree mask (word w of F held by lane
// j).  The mask only selects, so the execution mask never changes inside a
// walk.
template <int W, class TWW>
__device__ __forceinline__ void walk_edge(uint64_t* best, const TWW& F, int j, uint32_t Hj,
                                          uint32_t lo, const KeyMix* km) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t key = vkey_of(km[w], Hj);
    const bool take = lane_bit(readlane64(F.w[w], j)) & (key <= (uint32_t)(best[w] >> 32));
    best[w] = take ? (((uint64_t)key << 32) | lo) : best[w];
  }
}

// A value every lane holds alike (a scalar), copied into a vector register
// once, so that several selects under different execution masks share it.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t s) {
  uint32_t v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// 64 x 64 bit transpose across a wavefront: lane l holds row l on entry,
// and on return lane t holds the word whose bit l is bit t of row l.  Six
// stages, each swapping the off-diagonal blocks of size s = 32, 16, ..., 1
// with the partner lane l ^ s (mask: the bit positions c with c & s == 0).
__device__ __forceinline__ uint64_t transpose64(uint64_t x) {
  const int lane = lane_id();
  const uint64_t kMask[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                             0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = 32 >> k;
    const uint64_t m = kMask[k];
    const uint32_t ylo = (uint32_t)__shfl_xor((int)(uint32_t)x, s);
    const uint32_t yhi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), s);
    const uint64_t y = ((uint64_t)yhi << 32) | ylo;
    x = (lane & s) ? ((x & ~m) | ((y & ~m) >> s)) : ((x & m) | ((y & m) << s));
  }
  return x;
}

// Bits 0 .. j of a 64-bit mask (0 <= j <= 63).
__device__ __forceinline__ uint64_t bits_upto(int j) {
  return j >= 63 ? ~0ull : ((2ull << j) - 1);
}

// Lane t's state along edge j of the chunk: bit t of S_j (a lane-varying j).
__device__ __forceinline__ bool edge_state(uint64_t S, int j) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)S, j);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(S >> 32), j);
  const int t = lane_id();
  return ((t < 32 ? lo >> t : hi >> (t - 32)) & 1u) != 0;
}

// Wave-wide OR of a 64-bit value, returned to every lane.
__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
  return ((uint64_t)wave_or_u32((uint32_t)(x >> 32)) << 32) | wave_or_u32((uint32_t)x);
}

// Lane k < ne (ne = popcount of mask) gets the lane index of the k-th set
// bit of mask.
__device__ __forceinline__ int select_lane(uint64_t mask, int k) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const uint64_t below = (lo + step >= 64) ? mask : (mask & ((1ull << (lo + step)) - 1));
    if ((int)__popcll(below) <= k) lo += step;
  }
  return lo;
}

// ------------------------------------------------------------ W words per vertex
// Passes of 64 W trees.  Word w, bit t of a field is
// tree 64 w + t, and lane t of a wavefront carries trees t, 64 + t, ...  The
// four fields of a vertex (discoveries at even levels, states, discoveries at
// odd levels, visits) form one record of 4 W words, field f of vertex v at
// words 4 W v + f W .. + W - 1; MState's pointers point at field f of vertex 0.
// A gather of a neighbour's discoveries and states then touches one record,
// and a pass of 64 W trees moves about as many lines as a pass of 64.
constexpr int kRecFields = 4;

template <int W>
struct TW {
  uint64_t w[W];
};

template <int W>
__device__ __forceinline__ TW<W> ldw(const uint64_t* a, int64_t v) {
  TW<W> r;
  if constexpr (W == 1) {
    r.w[0] = a[kRecFields * v];
  } else {
    static_assert(W % 2 == 0, "one word or an even number of words per vertex");
#pragma unroll
    for (int k = 0; k < W; k += 2) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(a + kRecFields * W * v + k);
      r.w[k] = x.x;
      r.w[k + 1] = x.y;
    }
  }
  return r;
}

template <int W>
__device__ __forceinline__ void stw_(uint64_t* a, int64_t v, const TW<W>& x) {
  if constexpr (W == 1) {
    a[kRecFields * v] = x.w[0];
  } else {
#pragma unroll
    for (int k = 0; k < W; k += 2)
      *reinterpret_cast<ulonglong2*>(a + kRecFields * W * v + k) = make_ulonglong2(x.w[k], x.w[k + 1]);
  }
}

// The final-state copy of vertex v (W words at W v).
template <int W>
__device__ __forceinline__ void put_final(const MState& A, int64_t v, const TW<W>& st) {
  if (!A.stc) return;
  if constexpr (W == 1) {
    A.stc[v] = st.w[0];
  } else {
#pragma unroll
    for (int k = 0; k < W; k += 2)
      *reinterpret_cast<ulonglong2*>(A.stc + W * v + k) = make_ulonglong2(st.w[k], st.w[k + 1]);
  }
}

template <int W>
__device__ __forceinline__ TW<W> get_final(const uint64_t* stc, int64_t v) {
  TW<W> r;
  if constexpr (W == 1) {
    r.w[0] = stc[v];
  } else {
#pragma unroll
    for (int k = 0; k < W; k += 2) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(stc + W * v + k);
      r.w[k] = x.x;
      r.w[k + 1] = x.y;
    }
  }
  return r;
}

// A value every lane holds alike, moved to scalar registers.
template <int W>
__device__ __forceinline__ TW<W> uni_w(const TW<W>& x) {
  TW<W> r;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x.w[w]);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x.w[w] >> 32));
    r.w[w] = ((uint64_t)hi << 32) | lo;
  }
  return r;
}

template <int W>
__device__ __forceinline__ bool any_w(const TW<W>& x) {
  uint64_t o = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) o |= x.w[w];
  return o != 0;
}

template <int W>
__device__ __forceinline__ bool eq_w(const TW<W>& a, const TW<W>& b) {
  bool e = true;
#pragma unroll
  for (int w = 0; w < W; ++w) e = e && a.w[w] == b.w[w];
  return e;
}

template <int W>
__device__ __forceinline__ TW<W> and_not(const TW<W>& a, const TW<W>& b) {
  TW<W> r;
#pragma unroll
  for (int w = 0; w < W; ++w) r.w[w] = a.w[w] & ~b.w[w];
  return r;
}

template <int W>
__device__ __forceinline__ TW<W> or_w(const TW<W>& a, const TW<W>& b) {
  TW<W> r;
#pragma unroll
  for (int w = 0; w < W; ++w) r.w[w] = a.w[w] | b.w[w];
  return r;
}

// Lane t, word w: minimum over the edges [e0, e1) of the candidate of every
// neighbour discovered at the previous level of tree 64 w + t in a tree of
// `want`, folded into best[w].  The edges go in chunks of 64 through a
// two-stage pipeline, as in pull_small_w: a chunk's records and the next
// chunk's adjacency are in flight while the chunk before is walked; lanes
// past e1 read entry e0 and vertex 0.
template <int W>
__device__ __forceinline__ void pull_edges_w(const uint32_t* adj, const uint64_t* nbw,
                                             const uint64_t* stw, int64_t e0, int64_t e1,
                                             const TW<W>& want, const KeyMix* km, uint64_t* best) {
  if (e0 >= e1) return;
  const int lane = lane_id();
  uint32_t an = adj[e0 + lane < e1 ? e0 + lane : e0];
  uint32_t un = e0 + lane < e1 ? (an & kVertexMask) : 0u;
  uint64_t gn = (an >> 31) ? ~0ull : 0ull;
  TW<W> nb = ldw<W>(nbw, un);
  TW<W> st = ldw<W>(stw, un);  // the same record
  an = adj[e0 + 64 + lane < e1 ? e0 + 64 + lane : e0];
  for (int64_t c = e0; c < e1; c += 64) {
    const uint32_t H = fmix32(un);
    TW<W> F{}, S{};
    bool hit = false;
    if (c + lane < e1) {
#pragma unroll
      for (int w = 0; w < W; ++w) F.w[w] = nb.w[w] & want.w[w];
      hit = any_w(F);
#pragma unroll
      for (int w = 0; w < W; ++w) S.w[w] = st.w[w] ^ gn;
    }
    // the next chunk's records, then the adjacency of the chunk after it
    un = c + 64 + lane < e1 ? (an & kVertexMask) : 0u;
    gn = (an >> 31) ? ~0ull : 0ull;
    nb = ldw<W>(nbw, un);
    st = ldw<W>(stw, un);
    an = adj[c + 128 + lane < e1 ? c + 128 + lane : e0];
    uint64_t hits = __ballot(hit);
    if (!hits) continue;
    while (hits) {
      const int j = __builtin_ctzll(hits);
      hits &= hits - 1;
      const uint32_t Hj = __builtin_amdgcn_readlane(H, j);
      const uint32_t lo = to_vgpr(kPending | (uint32_t)j);
      walk_edge<W>(best, F, j, Hj, lo, km);
    }
    // minima found in this chunk take their state
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const bool pend = best[w] != kUnvisited && (best[w] & kPending);
      if (__ballot(pend)) {
        const bool st = edge_state(S.w[w], (int)(best[w] & 63));
        if (pend) best[w] = (best[w] & ~0xFFFFFFFFull) | (uint64_t)st;
      }
    }
  }
}

// Lane t, word w: the minimum root candidate of tree 64 w + t over
// cverts[b, e).
template <int W>
__device__ __forceinline__ void comp_min_w(const int32_t* cverts, int32_t b, int32_t e,
                                           const KeyMix* km, uint64_t* best) {
  const int lane = lane_id();
  // two running minima (even and odd vertices of each 64) keep two compare
  // chains in flight; the keys of distinct vertices never tie
  uint64_t alt[W];
#pragma unroll
  for (int w = 0; w < W; ++w) best[w] = alt[w] = kUnvisited;
  for (int32_t c = b; c < e; c += 64) {
    const int32_t i = c + lane;
    const int32_t mine = i < e ? cverts[i] : 0;
    const int cnt = min(64, e - c);
    const uint32_t hm = fmix32((uint32_t)mine);
    int j = 0;
    for (; j + 1 < cnt; j += 2) {
      const uint32_t v0 = (uint32_t)__builtin_amdgcn_readlane(mine, j);
      const uint32_t h0 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j);
      const uint32_t v1 = (uint32_t)__builtin_amdgcn_readlane(mine, j + 1);
      const uint32_t h1 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j + 1);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        take_min(best[w], vkey_of(km[w], h0), (uint32_t)root_candidate(0, v0));
        take_min(alt[w], vkey_of(km[w], h1), (uint32_t)root_candidate(0, v1));
      }
    }
    if (j < cnt) {
      const uint32_t v0 = (uint32_t)__builtin_amdgcn_readlane(mine, j);
      const uint32_t h0 = (uint32_t)__builtin_amdgcn_readlane((int)hm, j);
#pragma unroll
      for (int w = 0; w < W; ++w) take_min(best[w], vkey_of(km[w], h0), (uint32_t)root_candidate(0, v0));
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) best[w] = alt[w] < best[w] ? alt[w] : best[w];
}

// The write-back of vertex v once its trees of this level are decided.
template <int W>
__device__ __forceinline__ bool settle_w(const MState& A, int32_t v, const TW<W>& vis,
                                         const TW<W>& st, int dv, const uint64_t* best, int p,
                                         const TW<W>& valid, uint64_t& cnt, uint64_t& deg,
                                         uint64_t& fin) {
  TW<W> newb, stb;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    newb.w[w] = __ballot(best[w] != kUnvisited);
    stb.w[w] = __ballot(best[w] != kUnvisited && (best[w] & 1));
  }
  if (!any_w(newb)) return false;
  const TW<W> nv = or_w(vis, newb);
  const bool full = eq_w(nv, valid);
  if (lane_id() == 0) {
    stw_<W>(A.vis, v, nv);
    stw_<W>(A.nbw[p], v, newb);
    if (any_w(stb)) stw_<W>(A.stw, v, or_w(st, stb));
    if (full) {
      aand64(A.unf + (v >> 6), ~(1ull << (v & 63)));
      put_final<W>(A, v, or_w(st, stb));
    }
  }
  if (full) fin += (uint64_t)dv;
  cnt += 1;
  deg += (uint64_t)dv;
  return true;
}

// One wave pulls ne <= 64 vertices (lane k < ne holds vertex v; every row has
// between 1 and DMAX edges) and returns the entries some tree reached.
// The rows are walked in chunks of as many whole rows as fit in 64 lanes, in
// a two-stage pipeline: while the edges of one chunk are walked, the next
// chunk's records are in flight (its adjacency was read while this chunk's
// records arrived).  lw is the wave's LDS scratch of 4 x 64 entries: each
// row's wanted trees, its newly reached trees and their states, and the
// states each edge of the current chunk hands down.  ends is the wave's LDS
// bitmap of DMAX + 1 words (rows have at most DMAX edges, so the 64 rows hold
// at most 64 DMAX edges): bit e is set when an edge e > 0 of the concatenated
// rows starts a row.
template <int W, int DMAX>
__device__ __forceinline__ uint64_t pull_small_w(const DevGraph& G, const MState& A, int32_t v,
                                                 int ne, int pp, int p, const TW<W>& valid,
                                                 const KeyMix* km, bool push, TW<W>* lw,
                                                 uint64_t* ends, uint64_t& cnt, uint64_t& deg,
                                                 uint64_t& fin) {
  static_assert(DMAX >= 1 && DMAX <= 64, "rows of at most 64 edges");
  const int lane = lane_id();
  const bool ok = lane < ne;
  int s = 0, d = 0;
  TW<W> want{};
  if (ok) {
    s = G.row_ptr[v];
    d = G.row_ptr[v + 1] - s;
    want = and_not(valid, ldw<W>(A.vis, v));
  }
  lw[lane] = want;
  lw[64 + lane] = TW<W>{};
  lw[128 + lane] = TW<W>{};
  if (lane <= DMAX) ends[lane] = 0;
  if (DMAX == 64 && lane == 0) ends[64] = 0;
  const int inc = wave_incl_sum_i32(d);
  const int excl = inc - d;
  const int all = __builtin_amdgcn_readlane(inc, 63);
  __builtin_amdgcn_wave_barrier();
  // rows are never empty (a vertex without edges is its own tree's root), so
  // the row ends inc are distinct; the last one starts no row
  if (ok && inc < all) atomicOr((unsigned long long*)&ends[inc >> 6], 1ull << (inc & 63));
  const int sx = s - excl;  // edge e of the concatenation is entry sx + e of its row's vertex
  __builtin_amdgcn_wave_barrier();
  // the chunk that starts at row k0: lane i < total takes its edge i, of row kj
  struct Chunk {
    int k0, k1, total, kj;
    int64_t pos;
    uint64_t starts;  // bit i: edge i of the chunk starts a row
  };
  auto chunk_at = [&](int k0) {
    Chunk c;
    const int eb = __builtin_amdgcn_readlane(excl, k0);
    const int q = eb >> 6, sh = eb & 63;
    const uint64_t w0 = ends[q], w1 = ends[q + 1];
    const bool inr = ok && lane >= k0 && inc - eb <= 64;
    const uint64_t fit = __ballot(inr);
    c.k1 = k0 + (int)__popcll(fit);
    c.total = __builtin_amdgcn_readlane(inc, c.k1 - 1) - eb;
    const uint64_t win =
        readlane64(sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0, 0);
    const uint64_t starts = 1ull | (c.total >= 64 ? win : win & ((1ull << c.total) - 1));
    const int r = (int)__popcll(starts & bits_upto(lane));
    c.kj = k0 + r - 1;
    c.k0 = k0;
    c.starts = starts;
    c.pos = (int64_t)__shfl(sx, c.kj) + eb + lane;
    return c;
  };
  // c0: the chunk being walked; c1: its records are in flight; the adjacency
  // of the chunk after c1 is in flight.  Every lane issues every load (lanes
  // without an edge read entry 0 and vertex 0), so the wait counts are the
  // same on every path through the loop.
  Chunk c0 = chunk_at(0);
  uint32_t an = G.adj[lane < c0.total ? c0.pos : 0];
  uint32_t un = lane < c0.total ? (an & kVertexMask) : 0u;
  uint64_t gn = (an >> 31) ? ~0ull : 0ull;
  TW<W> nb = ldw<W>(A.nbw[pp], un);
  TW<W> su = ldw<W>(A.stw, un);  // the same record
  bool m1 = c0.k1 < ne;
  Chunk c1 = m1 ? chunk_at(c0.k1) : c0;
  an = G.adj[m1 && lane < c1.total ? c1.pos : 0];
  int k0 = 0;
  while (k0 < ne) {
    // c0's edges
    const uint32_t H = fmix32(un);
    TW<W> F{}, S{};
    bool hit = false;
    if (lane < c0.total) {
      const TW<W> wk = lw[c0.kj];
#pragma unroll
      for (int w = 0; w < W; ++w) F.w[w] = nb.w[w] & wk.w[w];
      hit = any_w(F);
#pragma unroll
      for (int w = 0; w < W; ++w) S.w[w] = su.w[w] ^ gn;
    }
    lw[192 + lane] = S;  // the states each edge hands down, read back per row
    const int kr0 = c0.k0;
    const int k1 = c0.k1;
    const uint64_t starts = c0.starts;
    // c1's records
    un = m1 && lane < c1.total ? (an & kVertexMask) : 0u;
    gn = (an >> 31) ? ~0ull : 0ull;
    nb = ldw<W>(A.nbw[pp], un);
    su = ldw<W>(A.stw, un);
    // the adjacency of the chunk after c1
    const bool m2 = m1 && c1.k1 < ne;
    const Chunk c2 = m2 ? chunk_at(c1.k1) : c1;
    an = G.adj[m2 && lane < c2.total ? c2.pos : 0];
    c0 = c1;
    c1 = c2;
    m1 = m2;
    uint64_t hits = __ballot(hit);
    uint64_t best[W];
#pragma unroll
    for (int w = 0; w < W; ++w) best[w] = kUnvisited;
    int cur = -1;
    auto keep = [&]() {
      TW<W> nbits, sbits;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const bool has = best[w] != kUnvisited;
        nbits.w[w] = __ballot(has);
        // the minimum's edge lies in this chunk (rows are never split)
        const bool st = (lw[192 + (int)(best[w] & 63)].w[w] >> lane) & 1;
        sbits.w[w] = __ballot(has && st);
      }
      if (lane == 0) {
        lw[64 + cur] = nbits;
        lw[128 + cur] = sbits;
      }
    };
    // row by row: the hits of the row holding the first remaining hit (rows
    // are runs of edges between the chunk's row starts), then its outcome
    while (hits) {
      const int j0 = __builtin_ctzll(hits);
      const uint64_t later = starts & ~bits_upto(j0);
      const uint64_t in_row = (later ? (later & (0 - later)) - 1 : ~0ull) & ~(bits_upto(j0) >> 1);
      uint64_t rh = hits & in_row;
      hits &= ~in_row;
      cur = kr0 + (int)__popcll(starts & bits_upto(j0)) - 1;
      if (W > 1 && (rh & (rh - 1)) == 0) {
        // one edge of the row hits: its trees are the row's new trees and
        // their states are the ones it hands down, no key to compare (with
        // one tree word the general walk is as short, and the batch kernel,
        // which pulls one word, ran 2 % slower with this branch)
        TW<W> nbits, sbits;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          nbits.w[w] = readlane64(F.w[w], j0);
          sbits.w[w] = nbits.w[w] & readlane64(S.w[w], j0);
        }
        if (lane == 0) {
          lw[64 + cur] = nbits;
          lw[128 + cur] = sbits;
        }
        continue;
      }
#pragma unroll
      for (int w = 0; w < W; ++w) best[w] = kUnvisited;
      while (rh) {
        const int jj = __builtin_ctzll(rh);
        rh &= rh - 1;
        const uint32_t Hj = __builtin_amdgcn_readlane(H, jj);
        const uint32_t lo = to_vgpr(kPending | (uint32_t)jj);
        walk_edge<W>(best, F, jj, Hj, lo, km);
      }
      keep();
    }
    k0 = k1;
  }
  __builtin_amdgcn_wave_barrier();
  TW<W> mnew{}, mstb{}, vis{}, st{};
  if (ok) {
    mnew = lw[64 + lane];
    mstb = lw[128 + lane];
  }
  const bool got = ok && any_w(mnew);
  if (got) {
    vis = ldw<W>(A.vis, v);
    st = ldw<W>(A.stw, v);
  }
  const TW<W> nv = or_w(vis, mnew);
  const bool full = got && eq_w(nv, valid);
  if (got) {
    stw_<W>(A.vis, v, nv);
    stw_<W>(A.nbw[p], v, mnew);
    if (any_w(mstb)) stw_<W>(A.stw, v, or_w(st, mstb));
    if (full) {
      aand64(A.unf + (v >> 6), ~(1ull << (v & 63)));
      put_final<W>(A, v, or_w(st, mstb));
    }
  }
  if (ok && push) aand64(A.cand + (v >> 6), ~(1ull << (v & 63)));
  const uint64_t reached = __ballot(got);
  cnt += (uint64_t)__popcll(reached);
  deg += wave_sum_u64(got ? (uint64_t)d : 0ull);
  fin += wave_sum_u64(full ? (uint64_t)d : 0ull);
  return reached;
}

}  // namespace mt
}  // namespace fi
