// Internal declarations of libfrustration: device helpers, the workspace
// layout and the host-side handle.  Everything here is the HIP path's own;
// nothing is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "frustration.h"

struct fi_graph;

namespace fi {

// ----------------------------------------------------------------- mixers
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): a Weyl sequence with
// increment 0x9E3779B97F4A7C15 read through a 64-bit finalizer.  `mix64(x)`
// is the value returned when the generator's state before the call is x.
constexpr uint64_t kWeyl = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += kWeyl;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// MurmurHash3's 32-bit finalizer (Appleby, public domain).
__host__ __device__ __forceinline__ constexpr uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Tree t of a sweep seeded with s: salt = output t of SplitMix64 seeded s.
__host__ __device__ __forceinline__ uint64_t tree_salt(uint64_t seed, uint64_t t) {
  return mix64(seed + t * kWeyl);
}

// Per-tree vertex key: (fmix32(u) xor x) * m mod 2^32, with x the salt's low
// word and m its high word forced odd.  A bijection of the 32-bit id, so no
// two vertices share a key; fmix32(u) does not depend on the tree, so it is
// computed once for all trees that need it.
struct KeyMix {
  uint32_t x, m;
};
__host__ __device__ __forceinline__ KeyMix key_mix(uint64_t salt) {
  return KeyMix{(uint32_t)salt, (uint32_t)(salt >> 32) | 1u};
}
__device__ __forceinline__ uint32_t vkey_of(KeyMix k, uint32_t h) { return (h ^ k.x) * k.m; }
__device__ __forceinline__ uint32_t vkey(KeyMix k, uint32_t u) { return vkey_of(k, fmix32(u)); }

// ----------------------------------------------------------------- tree words
// One 64-bit word per vertex carries the BFS level (31 bits), the parent's
// key (32 bits) and the vertex's state bit (1 = state -1):
//   level << 33 | key << 1 | bit.
// Unsigned order is (level, parent key), so an atomic minimum keeps the
// earliest level and, within it, the minimum-key parent; words of earlier
// levels are never overwritten.  All ones = not reached yet.  A BFS level is
// below n < 2^31, so every depth fits below that sentinel (a spanning forest
// of any graph, Definition def-FundamentalCycle and its corollary).
constexpr uint64_t kUnvisited = ~0ull;
constexpr uint32_t kMaxLevel = 0x7FFFFFFEu;

__device__ __forceinline__ uint64_t tree_word(uint32_t level, uint32_t key, uint32_t bit) {
  return ((uint64_t)level << 33) | ((uint64_t)key << 1) | bit;
}
// Candidate word used to pick a component's root or a parent while its id
// is still needed: key, then id, then a spare low bit.
__device__ __forceinline__ uint64_t root_candidate(uint32_t key, uint32_t u) {
  return ((uint64_t)key << 32) | ((uint64_t)u << 1);
}
__device__ __forceinline__ uint32_t word_vertex(uint64_t w) {
  return (uint32_t)(w >> 1) & 0x7FFFFFFFu;
}

// Packed adjacency entry: neighbour id in the low 31 bits, bit 31 set for a
// negative edge.
constexpr uint32_t kVertexMask = 0x7FFFFFFFu;

// ----------------------------------------------------------------- state keys
// 128-bit key of a canonical state, as two independent sums mod 2^64 of
// mix64(mix64(i + K) ^ W_i) over the state's 64-bit words W_i.
constexpr uint64_t kKeyHi = 0x243F6A8885A308D3ull;  // pi, hex digits 1-16
constexpr uint64_t kKeyLo = 0x13198A2E03707344ull;  // pi, hex digits 17-32

__device__ __forceinline__ void key_terms(uint64_t i, uint64_t w, uint64_t& hi, uint64_t& lo) {
  hi += mix64(mix64(i + kKeyHi) ^ w);
  lo += mix64(mix64(i + kKeyLo) ^ w);
}

// ----------------------------------------------------------------- cloud
// Open addressing on key_lo (linear probing).  Every field is updated with a
// commutative atomic, so the table contents never depend on insertion order;
// readout checks that each slot saw one key_hi and one switch count.
struct CloudSlot {
  uint64_t tag;        // key_lo, or kEmpty
  uint64_t khi_min, khi_max;
  uint64_t s_min, s_max;
  uint64_t freq;
  uint64_t first;      // smallest tree index
  uint64_t pad;
};
constexpr uint64_t kEmpty = ~0ull;

// ----------------------------------------------------------------- control
// uint64 words of the per-graph control block.
enum : int {
  C_ERR = 0,        // sticky error bits (E_*)
  C_BEST = 1,       // min over trees of (switches << 32 | tree)
  C_COUNT = 2,      // occupied cloud slots
  C_TREES = 3,      // trees inserted
  C_NCOMP = 4,      // components (create)
  C_NISO = 5,       // isolated vertices (create)
  C_NANCH = 6,      // anchors of non-trivial components (create)
  C_FLAGS = 7,      // validation flags (create)
  C_BAR = 16,       // grid barrier: arrivals (own 128-byte line)
  C_GEN = 32,       // grid barrier: generation (own line)
  C_ACC = 48,       // tree accumulators: switches, key_hi, key_lo
  C_RING = 64,      // per-level frontier counters, 4 slots x 4 words
  C_UNIT = 96,      // per-block work-unit ticket broadcast (unused on host)
  C_WORDS = 128
};
enum : uint64_t { E_CAPACITY = 1, E_DEPTH = 2, E_COLLISION = 4 };

// validation flags set by the create kernels
enum : uint32_t {
  V_ROWPTR = 1, V_RANGE = 2, V_SIGN = 4, V_SELF = 8, V_DUP = 16, V_UNSORTED = 32, V_ASYM = 64
};

// ----------------------------------------------------------------- device view
struct DevGraph {
  int32_t n;
  int32_t nwords;       // ceil(n / 64)
  int64_t nnz;
  int64_t m;            // undirected edges
  const int32_t* row_ptr;   // [n+1]
  const uint32_t* adj;      // [nnz] packed neighbour | neg << 31
  const uint2* edges;       // [m] (u, v | neg << 31), u < v
  const uint2* cedges;      // [m] (v, u | neg << 31): each edge once, in the row of its
                            // endpoint of lower rank (degree, then id), rows in order
  const int32_t* comp;      // [n] anchor (smallest id) of the component
  const int32_t* word_comp; // [nwords] smallest anchor among the word's vertices
                            // with an edge ("main" component), -2 if none
  const uint64_t* word_mask;// [nwords] vertices of the word with an edge
  const uint64_t* word_main;// [nwords] those of them in the main component
  const int32_t* anchors;   // [C] anchors of components with an edge
  CloudSlot* cloud;
  uint64_t cloud_mask;      // table size - 1
  uint64_t cloud_cap;       // user capacity (distinct states)
  uint64_t* ctl;            // [C_WORDS]
};

// Per-call sweep arguments.
struct SweepArgs {
  uint64_t seed;
  uint64_t t0, t1;
  uint64_t* tree_switches;  // [t1 - t0] or null
  uint64_t* bits_out;       // canonical words of the single tree, or null
  int insert;               // 0: compute only, leave the cloud alone
  // cloud statistics (multi-tree path only): per vertex, trees whose canonical
  // state puts it at -1; per upper-triangle edge, trees that switch it
  uint64_t* vminus;
  uint64_t* eswitch;
  int sampler;              // kSampler*: the tree sampler (paths 1 and 2)
  const int32_t* cptr;      // component offsets (randomized DFS stacks)
  // one-workgroup-per-tree scratch in workspace memory: [slots][slot_stride bytes]
  uint64_t* pw;
  size_t slot_stride;
};

// tree samplers (Section "Tree-Sampling techniques for graphBpp")
enum : int { kSamplerBfs = 0, kSamplerRdfs = 1, kSamplerHybrid = 2, kSamplerKruskal = 3 };

// ----------------------------------------------------------------- layout
constexpr int kGridSlots = 8;  // trees in flight on the whole-grid path (max)
constexpr int kGridCtlWords = 128;          // control words per tree slot
constexpr int kGridBarWords = 32 + 16 * 512;  // barrier words per tree slot

struct Layout {
  size_t row_ptr, adj, edges, cedges, comp, word_comp, word_mask, word_main, anchors, tmp, cloud, ctl;
  size_t scratch;      // create temporaries, cloud staging, rounded graphL states
  size_t gl;           // graphL loss partials
  // whole-grid path: kGridSlots trees in flight
  size_t gpw, gql, gqh, gfb, gvis, gsb, grootkey, gctl, gbar;
  size_t hcap;         // heavy-list entries per list
  size_t gpstride;     // per-slot vertex stride (n rounded up to 32)
  size_t gwstride;     // per-slot bitmap stride (words rounded up to 32)
  size_t slots;        // one-workgroup-per-tree scratch in workspace memory
  size_t nslots, slot_stride;
  // multi-tree path: 32-byte per-vertex records, split-row partial minima,
  // vertices listed by component, and root-finding tasks
  size_t mrec, mhslot, mhcap, mreach, aslot, cverts, ccount, cptr, mtasks, mtcap, rootbig, nbigcap;
  size_t swtile;       // switch lists: per-tile counts and offsets (8 bytes each)
  size_t glheavy;      // graphL: rows longer than kGLHeavy
  size_t glfirst;      // graphL: first item of each of those rows, and the item count
  size_t glitems;      // graphL: items (heavy row, chunk)
  size_t glicap;       // graphL: item capacity
  size_t glpart;       // graphL: [items][64] partial sums
  size_t glctl;        // graphL: heavy-row and item counts
  // tree order of the multi-tree path: per-vertex sums of BFS distances to
  // the highest-degree vertices, and per block of trees their main-component
  // root candidates, sort keys and order
  size_t cent, oroot, okey, operm;
  size_t total;
};

// trees ordered per block of the multi-tree sweep (a power of two)
constexpr int kOrderMax = 16384;

// multi-tree path constants shared by create and the kernel
constexpr int kMSplit = 2048;     // rows longer than this are split into units of this many edges
constexpr int kBigComp = 1024;    // components larger than this find their roots in chunks
constexpr int kRootChunk = 1024;  // vertices per root-finding task of a big component

Layout make_layout(int32_t n, int64_t nnz, int64_t cloud_capacity, uint64_t table_size);
int64_t switch_tiles(int64_t m);  // tiles of the switch-list compaction over m edges
uint64_t table_size_for(int64_t cloud_capacity);
// a cloud table (tsize slots of device memory) to host entries sorted by key
// (blocks); FI_ECOLLISION if a slot met two key_hi or two switch counts
int read_cloud_table(const CloudSlot* d_table, uint64_t tsize, fi_cloud_entry* h_out, int64_t cap,
                     int64_t* written, hipStream_t s);

constexpr int kGraphLMaxR = 64;
constexpr int kGraphLBlocks = 1024;
constexpr int kGLHeavy = 256;   // graphL rows longer than this are cut into items
constexpr int kGLChunk = 4096;  // CSR entries per item of a long graphL row

// profiling events around one launch (no-ops unless profiling is on)
void batch_info_free(void* p);
void* prof_events_new();
int prof_begin(fi_graph* g, hipStream_t s, void** token);
void prof_end(fi_graph* g, hipStream_t s, void* token, int kernel);

// launchers implemented in the .hip files
hipError_t launch_sweep(fi_graph* g, const SweepArgs& a, hipStream_t s);
hipError_t launch_grid(fi_graph* g, const SweepArgs& a, hipStream_t s);
hipError_t launch_multi(fi_graph* g, const SweepArgs& a, int words, hipStream_t s);
// exact count of up to 64 states given as one word per vertex (bit b = the
// vertex's state in state b, set = -1; uint32 words for up to 32 states,
// else uint64): counts[b] += frustrated edges
hipError_t launch_count(const DevGraph& dg, const void* st, int32_t nstates, uint64_t* counts,
                        hipStream_t s);
hipError_t graphl_setup(fi_graph* g, hipStream_t s);
// distance sums to the highest-degree vertices, for the multi-tree path's
// tree order (blocks; sets g->cent)
int centrality_setup(fi_graph* g, hipStream_t s);
// order of trees t0 .. t0 + count - 1 (count <= kOrderMax) for the
// multi-tree path: perm in the workspace, and each tree's main-component
// root candidate at oroot[tree - t0]
hipError_t order_trees(fi_graph* g, uint64_t seed, uint64_t t0, uint32_t count, hipStream_t s);

}  // namespace fi

// ----------------------------------------------------------------- host handle
struct fi_graph {
  fi::DevGraph dg;
  fi::Layout L;
  char* ws;
  size_t ws_bytes;
  int64_t cloud_capacity;
  uint64_t table_size;
  int32_t ncomp, nisolated, nanch;
  int32_t mtasks, mnbig;  // multi-tree path: root-finding tasks, big components
  int32_t gl_nheavy;      // graphL rows longer than kGLHeavy (their items are planned at upload)
  int32_t sampler;        // kSampler*
  int32_t gl_main_slot;   // slot of the component with the most vertices (-1: none)
  int32_t main_begin, main_end;  // its vertices in cverts
  int32_t main_big;       // its row of big-component root minima (-1: not a big component)
  bool cent;              // distance sums for the tree order are in the workspace
  uint64_t* plog;         // phase log of the multi-tree kernel (null: off)
  int64_t pcap;           // its length in words
  fi_schedule sched;
  int cu_count;
  int max_shared;
  // profiling
  bool prof;
  double prof_ms[2];
  int64_t prof_n[2];
  void* prof_events;  // std::vector of pending (start, stop, kernel)
  // batch mode
  bool is_batch;
  void* batch;        // fi::BatchInfo*
};
