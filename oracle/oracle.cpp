// CPU oracle for the graphBpp spanning-tree sweep.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the HIP path is checked against.  Only the tests, the smoke
// check and the benchmark's CPU-baseline leg load it.  It shares no code,
// header, table or constant generator with the library under
// paper_2311_00869_amd/csrc; every formula below is written out again from
// the paper and from the published definitions of the two integer mixers.
//
// What it follows (Shebaro & Tesic, "Scaling Frustration Index and
// Corresponding Balanced State Discovery for Real Signed Graphs"):
//   * Alg. alg-index (graphBpp, the outer loop): per sampled tree, balance the graph,
//     count the sign differences, turn the balanced state into a key, and
//     insert-or-increment it in the frustration cloud; return min S.
//   * Alg. alg-balance (graphB+ balancing): for every non-tree edge, flip it
//     when its fundamental cycle is negative.  Implemented literally by
//     walking the tree path between the edge's endpoints.
//   * Section "graphBpp: scaling the graph balancing": the balanced state is
//     turned into the string "src->tgt: sign" over the sorted edge tuples,
//     joined by "|"; the cloud is a std::map keyed by that state.
//   * Definition def-FundamentalCycle and its corollary: there are
//     |E|-|V|+1 fundamental cycles per connected component.
//   * Theorem t:HararyCut: a balanced graph is 2-colourable with negative
//     edges exactly across the two colour classes.
//
// Readings where the paper leaves a choice open (listed in the design notes):
//   * Tree sampler: BFS by default.  Each tree t of a sweep with seed s gets a
//     salt from the SplitMix64 stream seeded with s; every vertex u gets a
//     32-bit key, a bijection of u (see vertex_key).  The root of each
//     connected component is its minimum-key vertex, and the parent of every
//     other vertex is its minimum-key neighbour on the previous BFS level.
//     Disconnected graphs get a spanning forest.  The other samplers
//     (randomized DFS, the RDFS-BFS hybrid, Kruskal on random weights) take
//     their randomness from the same salt; see build_sampled_tree.
//   * Vertex state s (+1/-1): root +1, child = parent * sign(tree edge).
//   * Cloud key: the canonical vertex state (each component flipped so that
//     its smallest vertex is +1), which determines the balanced graph one to
//     one (Theorem t:HararyCut, item 4), hashed to 128 bits.
//
// Parity pins for every function here live in tests/test_oracle_*.py.

#include <cstdint>
#include <cstring>
#include <map>
#include <queue>
#include <set>
#include <string>
#include <tuple>
#include <vector>
#include <algorithm>

namespace {

// ---------------------------------------------------------------- mixers
// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the state advances by the golden-ratio
// increment, and the output is the state passed through a 64-bit finalizer.
const uint64_t kGolden = 0x9E3779B97F4A7C15ull;

uint64_t splitmix_output(uint64_t state_before_step) {
    uint64_t z = state_before_step + kGolden;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// MurmurHash3 32-bit finalizer (Appleby, public domain).
uint32_t murmur_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Salt of tree t: output number t (counting from 0) of the SplitMix64
// stream seeded with the sweep seed.
uint64_t tree_salt(uint64_t seed, int64_t t) {
    uint64_t state = seed;
    // state after t steps, written as a product so large t stays cheap
    state += (uint64_t)t * kGolden;
    return splitmix_output(state);
}

// Vertex key of u in the tree with the given salt: the MurmurHash3
// finalizer of u, xor the salt's low word, times the salt's high word forced
// odd, mod 2^32.  Each step is invertible, so distinct vertices never share
// a key and "the minimum-key vertex" is always one vertex.
uint64_t vertex_key(uint64_t salt, int32_t u) {
    const uint32_t x = (uint32_t)(salt & 0xFFFFFFFFull);
    const uint32_t m = (uint32_t)(salt >> 32) | 1u;
    return (uint64_t)((murmur_fmix32((uint32_t)u) ^ x) * m);
}

// 128-bit key of a canonical state given as 64-bit words (vertex v is bit
// v%64 of word v/64): for each half, the sum mod 2^64 over words i of
// splitmix(splitmix(i + K) ^ W_i), with K = 0x243F6A8885A308D3 for the high
// half and 0x13198A2E03707344 for the low half (hex digits of pi).
void state_hash(const std::vector<uint64_t>& words, uint64_t& hi, uint64_t& lo) {
    const uint64_t k_hi = 0x243F6A8885A308D3ull, k_lo = 0x13198A2E03707344ull;
    hi = 0; lo = 0;
    for (size_t i = 0; i < words.size(); ++i) {
        hi += splitmix_output(splitmix_output((uint64_t)i + k_hi) ^ words[i]);
        lo += splitmix_output(splitmix_output((uint64_t)i + k_lo) ^ words[i]);
    }
}

// ---------------------------------------------------------------- graph view
struct Graph {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* col;
    const int8_t* sign;
    int64_t begin(int32_t v) const { return row_ptr[v]; }
    int64_t end(int32_t v) const { return row_ptr[v + 1]; }
};

// CSR entry of edge (u, v) by binary search in u's sorted row; -1 if absent.
int64_t find_entry(const Graph& g, int32_t u, int32_t v) {
    const int32_t* first = g.col + g.begin(u);
    const int32_t* last = g.col + g.end(u);
    const int32_t* it = std::lower_bound(first, last, v);
    if (it == last || *it != v) return -1;
    return it - g.col;
}

// Sign of edge (u, v); 0 if absent.
int edge_sign(const Graph& g, int32_t u, int32_t v) {
    int64_t e = find_entry(g, u, v);
    return e < 0 ? 0 : g.sign[e];
}

// Connected components by plain BFS; label = smallest vertex id in the
// component (vertices are scanned in increasing id, so the first unlabelled
// vertex met is the component's smallest).
int32_t label_components(const Graph& g, std::vector<int32_t>& comp) {
    comp.assign(g.n, -1);
    int32_t count = 0;
    std::queue<int32_t> q;
    for (int32_t s = 0; s < g.n; ++s) {
        if (comp[s] >= 0) continue;
        ++count;
        comp[s] = s;
        q.push(s);
        while (!q.empty()) {
            int32_t u = q.front(); q.pop();
            for (int64_t e = g.begin(u); e < g.end(u); ++e) {
                int32_t v = g.col[e];
                if (comp[v] < 0) { comp[v] = s; q.push(v); }
            }
        }
    }
    return count;
}

struct Tree {
    std::vector<int32_t> level, parent;  // parent -1 at roots
    std::vector<int8_t> parent_sign;     // sign of the tree edge to the parent
    std::vector<int8_t> state;           // +1 / -1
    std::vector<int32_t> order;          // BFS order
};

// The sampled BFS spanning forest of tree t (root = min key per component,
// parent = min-key neighbour on the previous level) and its propagated state.
void build_tree(const Graph& g, const std::vector<int32_t>& comp, uint64_t seed, int64_t t,
                Tree& T) {
    const uint64_t salt = tree_salt(seed, t);
    const int32_t n = g.n;
    // roots: argmin of the key within each component
    std::vector<uint64_t> best(n, UINT64_MAX);
    std::vector<int32_t> argbest(n, -1);
    for (int32_t v = 0; v < n; ++v) {
        uint64_t k = vertex_key(salt, v);
        if (k < best[comp[v]]) { best[comp[v]] = k; argbest[comp[v]] = v; }
    }
    T.level.assign(n, -1);
    T.parent.assign(n, -1);
    T.parent_sign.assign(n, 1);
    T.state.assign(n, 0);
    T.order.clear();
    std::queue<int32_t> q;
    for (int32_t c = 0; c < n; ++c) {
        if (argbest[c] < 0) continue;
        int32_t r = argbest[c];
        T.level[r] = 0;
        q.push(r);
    }
    // multi-source BFS for the levels
    while (!q.empty()) {
        int32_t u = q.front(); q.pop();
        T.order.push_back(u);
        for (int64_t e = g.begin(u); e < g.end(u); ++e) {
            int32_t v = g.col[e];
            if (T.level[v] < 0) { T.level[v] = T.level[u] + 1; q.push(v); }
        }
    }
    // parent: linear scan for the min-key neighbour one level up
    for (int32_t v = 0; v < n; ++v) {
        if (T.level[v] <= 0) continue;
        uint64_t bk = UINT64_MAX;
        for (int64_t e = g.begin(v); e < g.end(v); ++e) {
            int32_t u = g.col[e];
            if (T.level[u] != T.level[v] - 1) continue;
            uint64_t k = vertex_key(salt, u);
            if (k < bk) { bk = k; T.parent[v] = u; T.parent_sign[v] = g.sign[e]; }
        }
    }
    // state: root +1, child = parent * sign(parent, child), in BFS order
    for (int32_t v : T.order) {
        if (T.parent[v] < 0) T.state[v] = 1;
        else T.state[v] = (int8_t)(T.state[T.parent[v]] * T.parent_sign[v]);
    }
}

// ---------------------------------------------------------------- other samplers
// Section "Tree-Sampling techniques for graphBpp" and Alg. alg-hybrid, made
// reproducible like BFS: all randomness comes from tree t's salt.
enum { SAMPLER_BFS = 0, SAMPLER_RDFS = 1, SAMPLER_HYBRID = 2, SAMPLER_KRUSKAL = 3 };

// Alg. alg-hybrid's fair coin (0 or 1): the top bit of the
// SplitMix64 finalizer applied to the tree's salt (0: BFS, 1: RDFS).
int hybrid_coin(uint64_t salt) { return (int)(splitmix_output(salt) >> 63); }

// Minimum-key vertex of every component (indexed by the component label).
std::vector<int32_t> min_key_roots(const Graph& g, const std::vector<int32_t>& comp, uint64_t salt) {
    std::vector<uint64_t> best(g.n, UINT64_MAX);
    std::vector<int32_t> arg(g.n, -1);
    for (int32_t v = 0; v < g.n; ++v) {
        uint64_t k = vertex_key(salt, v);
        if (k < best[comp[v]]) { best[comp[v]] = k; arg[comp[v]] = v; }
    }
    return arg;
}

void reset_tree(int32_t n, Tree& T) {
    T.level.assign(n, -1);
    T.parent.assign(n, -1);
    T.parent_sign.assign(n, 1);
    T.state.assign(n, 0);
    T.order.clear();
}

// Randomized DFS: the shuffled adjacency of the paper's RDFS is the order of
// the neighbours' keys, so from the current vertex the search moves to its
// unvisited neighbour of smallest key and backtracks when there is none.
// One search per component from its minimum-key vertex; states propagate
// along the discovery edges.
void build_rdfs(const Graph& g, const std::vector<int32_t>& comp, uint64_t salt, Tree& T) {
    reset_tree(g.n, T);
    std::vector<int32_t> root = min_key_roots(g, comp, salt);
    std::vector<int32_t> stack;
    for (int32_t c = 0; c < g.n; ++c) {
        if (root[c] < 0) continue;
        int32_t r = root[c];
        T.level[r] = 0;
        T.state[r] = 1;
        T.order.push_back(r);
        stack.assign(1, r);
        while (!stack.empty()) {
            int32_t u = stack.back();
            int32_t pick = -1;
            int8_t psign = 1;
            uint64_t pk = UINT64_MAX;
            for (int64_t e = g.begin(u); e < g.end(u); ++e) {
                int32_t v = g.col[e];
                if (T.level[v] >= 0) continue;
                uint64_t k = vertex_key(salt, v);
                if (k < pk) { pk = k; pick = v; psign = g.sign[e]; }
            }
            if (pick < 0) { stack.pop_back(); continue; }
            T.parent[pick] = u;
            T.parent_sign[pick] = psign;
            T.level[pick] = T.level[u] + 1;
            T.state[pick] = (int8_t)(T.state[u] * psign);
            T.order.push_back(pick);
            stack.push_back(pick);
        }
    }
}

// Random weight of the undirected edge (u, v), u < v, in tree t: the high
// half of the SplitMix64 finalizer of salt xor (u << 32 | v).
uint32_t kruskal_weight(uint64_t salt, int32_t u, int32_t v) {
    return (uint32_t)(splitmix_output(salt ^ ((uint64_t)(uint32_t)u << 32 | (uint32_t)v)) >> 32);
}

// Kruskal's algorithm on random edge weights: edges in increasing order of
// (weight, position in the sorted (u, v) edge list), each kept when it joins
// two trees of the forest.  The order is total, so the forest is the unique
// minimum spanning forest.  Each tree is then rooted at its smallest vertex
// and walked breadth-first along its edges for levels and states.
void build_kruskal(const Graph& g, const std::vector<int32_t>& comp, uint64_t salt, Tree& T) {
    reset_tree(g.n, T);
    struct E { uint64_t key; int32_t u, v; int8_t s; };
    std::vector<E> edges;
    uint64_t idx = 0;
    for (int32_t u = 0; u < g.n; ++u)
        for (int64_t e = g.begin(u); e < g.end(u); ++e)
            if (u < g.col[e]) {
                uint64_t w = kruskal_weight(salt, u, g.col[e]);
                edges.push_back({w << 32 | idx, u, g.col[e], g.sign[e]});
                ++idx;
            }
    std::sort(edges.begin(), edges.end(), [](const E& a, const E& b) { return a.key < b.key; });
    std::vector<int32_t> uf(g.n);
    for (int32_t v = 0; v < g.n; ++v) uf[v] = v;
    auto find = [&](int32_t x) {
        while (uf[x] != x) { uf[x] = uf[uf[x]]; x = uf[x]; }
        return x;
    };
    std::vector<std::vector<std::pair<int32_t, int8_t>>> tadj(g.n);
    for (const E& e : edges) {
        int32_t a = find(e.u), b = find(e.v);
        if (a == b) continue;
        uf[a] = b;
        tadj[e.u].push_back({e.v, e.s});
        tadj[e.v].push_back({e.u, e.s});
    }
    std::queue<int32_t> q;
    for (int32_t r = 0; r < g.n; ++r) {
        if (comp[r] != r) continue;
        T.level[r] = 0;
        T.state[r] = 1;
        q.push(r);
        while (!q.empty()) {
            int32_t u = q.front(); q.pop();
            T.order.push_back(u);
            for (auto& [v, sg] : tadj[u]) {
                if (T.level[v] >= 0) continue;
                T.level[v] = T.level[u] + 1;
                T.parent[v] = u;
                T.parent_sign[v] = sg;
                T.state[v] = (int8_t)(T.state[u] * sg);
                q.push(v);
            }
        }
    }
}

// Tree t with the chosen sampler.
void build_sampled_tree(const Graph& g, const std::vector<int32_t>& comp, uint64_t seed, int64_t t,
                        int sampler, Tree& T) {
    const uint64_t salt = tree_salt(seed, t);
    if (sampler == SAMPLER_HYBRID) sampler = hybrid_coin(salt) ? SAMPLER_RDFS : SAMPLER_BFS;
    if (sampler == SAMPLER_RDFS) build_rdfs(g, comp, salt, T);
    else if (sampler == SAMPLER_KRUSKAL) build_kruskal(g, comp, salt, T);
    else build_tree(g, comp, seed, t, T);
}

bool is_tree_edge(const Tree& T, int32_t u, int32_t v) {
    return T.parent[v] == u || T.parent[u] == v;
}

// Alg. alg-balance, literally: for each non-tree edge e = (u, v), take the
// product of the signs around the fundamental cycle (the tree path u..v plus
// e); if it is negative, flip e.  flip is indexed by CSR entry and set in
// both directions.  Returns the number of flipped (undirected) edges.
int64_t balance_by_cycles(const Graph& g, const Tree& T, std::vector<int8_t>& flip) {
    flip.assign(g.row_ptr[g.n], 0);
    int64_t flips = 0;
    for (int32_t u = 0; u < g.n; ++u) {
        for (int64_t e = g.begin(u); e < g.end(u); ++e) {
            int32_t v = g.col[e];
            if (v < u) continue;  // each undirected edge once
            if (is_tree_edge(T, u, v)) continue;
            int prod = g.sign[e];
            int32_t x = u, y = v;
            while (T.level[x] > T.level[y]) { prod *= T.parent_sign[x]; x = T.parent[x]; }
            while (T.level[y] > T.level[x]) { prod *= T.parent_sign[y]; y = T.parent[y]; }
            while (x != y) {
                prod *= T.parent_sign[x]; x = T.parent[x];
                prod *= T.parent_sign[y]; y = T.parent[y];
            }
            if (prod < 0) {
                ++flips;
                flip[e] = 1;
                flip[find_entry(g, v, u)] = 1;
            }
        }
    }
    return flips;
}

// Independent checks of one balanced state (Theorem t:HararyCut and the
// corollary on fundamental cycles).  Returns 0 or a negative check id.
int cross_check(const Graph& g, const std::vector<int32_t>& comp, int32_t ncomp, const Tree& T,
                const std::vector<int8_t>& flip) {
    // (i) the flips are exactly the edges frustrated under the propagated
    //     state, and no tree edge is flipped
    int64_t nontree = 0;
    for (int32_t u = 0; u < g.n; ++u)
        for (int64_t e = g.begin(u); e < g.end(u); ++e) {
            int32_t v = g.col[e];
            bool frustrated = g.sign[e] * T.state[u] * T.state[v] < 0;
            if ((bool)flip[e] != frustrated) return -101;
            if (is_tree_edge(T, u, v)) { if (flip[e]) return -102; }
            else if (u < v) ++nontree;
        }
    // (ii) the balanced graph is 2-colourable with its negative edges across
    std::vector<int8_t> colour(g.n, 0);
    std::queue<int32_t> q;
    for (int32_t s = 0; s < g.n; ++s) {
        if (colour[s]) continue;
        colour[s] = 1; q.push(s);
        while (!q.empty()) {
            int32_t u = q.front(); q.pop();
            for (int64_t e = g.begin(u); e < g.end(u); ++e) {
                int32_t v = g.col[e];
                int sp = flip[e] ? -g.sign[e] : g.sign[e];
                int want = colour[u] * sp;
                if (!colour[v]) { colour[v] = (int8_t)want; q.push(v); }
                else if (colour[v] != want) return -103;
            }
        }
    }
    // (iii) |E| - |V| + c non-tree edges
    int64_t m = g.row_ptr[g.n] / 2;
    if (nontree != m - g.n + ncomp) return -104;
    (void)comp;
    return 0;
}

// Canonical state: every component flipped so that its smallest vertex is +1;
// bit v of the word array is set where the canonical state is -1.
std::vector<uint64_t> canonical_words(int32_t n, const std::vector<int32_t>& comp,
                                      const std::vector<int8_t>& state) {
    std::vector<uint64_t> w((n + 63) / 64, 0);
    for (int32_t v = 0; v < n; ++v) {
        bool minus = state[v] != state[comp[v]];
        if (minus) w[v / 64] |= 1ull << (v % 64);
    }
    return w;
}

// The paper's string form of a balanced graph: sorted (src, tgt, sign)
// tuples with src < tgt, each written "src->tgt: sign", joined by "|".
std::string paper_state_string(const Graph& g, const std::vector<int8_t>& flip) {
    std::set<std::tuple<int32_t, int32_t, int>> tuples;
    for (int32_t u = 0; u < g.n; ++u)
        for (int64_t e = g.begin(u); e < g.end(u); ++e)
            if (u < g.col[e]) tuples.insert({u, g.col[e], flip[e] ? -g.sign[e] : g.sign[e]});
    std::string s;
    bool first = true;
    for (auto& tp : tuples) {
        if (!first) s += "|";
        first = false;
        s += std::to_string(std::get<0>(tp)) + "->" + std::to_string(std::get<1>(tp)) + ": " +
             std::to_string(std::get<2>(tp));
    }
    return s;
}

struct CloudValue {
    uint64_t freq = 0, switches = 0, first_tree = 0;
};

}  // namespace

extern "C" {

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_EASYM = -2,
    ORC_ESELFLOOP = -3,
    ORC_EDUP = -4,
    ORC_ESIGN = -5,
    ORC_ERANGE = -6,
    ORC_EUNSORTED = -7,
    ORC_ECOLLISION = -20,
    ORC_ESTATE = -21,
    ORC_ESTRING = -22,
    ORC_ECAP = -23,
};

// Input contract of the sweep: a simple undirected signed graph in symmetric
// CSR with sorted rows ("duplicates, inconsistencies, self-loops and invalid
// signs" removed, Section "Implementation").  Checks are made in this order
// and the first failure is returned.
int orc_validate(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                 const int8_t* sign) {
    if (n < 0 || nnz < 0) return ORC_EINVAL;
    if (nnz >= (int64_t)1 << 31) return ORC_ERANGE;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return ORC_EINVAL;
    for (int64_t e = 0; e < nnz; ++e)
        if (col[e] < 0 || col[e] >= n) return ORC_EINVAL;
    for (int64_t e = 0; e < nnz; ++e)
        if (sign[e] != 1 && sign[e] != -1) return ORC_ESIGN;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col[e] == v) return ORC_ESELFLOOP;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v] + 1; e < row_ptr[v + 1]; ++e)
            if (col[e] == col[e - 1]) return ORC_EDUP;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v] + 1; e < row_ptr[v + 1]; ++e)
            if (col[e] < col[e - 1]) return ORC_EUNSORTED;
    Graph g{n, row_ptr, col, sign};
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (edge_sign(g, col[e], u) != sign[e]) return ORC_EASYM;
    return ORC_OK;
}

// comp_out[v] = smallest vertex id of v's component.  Returns the number of
// components.
int32_t orc_components(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* comp_out) {
    Graph g{n, row_ptr, col, nullptr};
    std::vector<int32_t> comp;
    int32_t c = label_components(g, comp);
    std::memcpy(comp_out, comp.data(), sizeof(int32_t) * n);
    return c;
}

uint64_t orc_tree_salt(uint64_t seed, int64_t t) { return tree_salt(seed, t); }
uint64_t orc_vertex_key(uint64_t salt, int32_t u) { return vertex_key(salt, u); }

// Keys of vertices 0 .. n-1 in trees t0 .. t1-1 of the sweep with this
// seed, tree by tree: out[(t - t0) * n + u].
void orc_vertex_keys(uint64_t seed, int64_t t0, int64_t t1, int32_t n, uint32_t* out) {
    for (int64_t t = t0; t < t1; ++t) {
        const uint64_t salt = tree_salt(seed, t);
        for (int32_t u = 0; u < n; ++u) out[(t - t0) * n + u] = (uint32_t)vertex_key(salt, u);
    }
}

// Tree t of the sweep with this seed: level, parent (-1 at roots), parent
// edge sign, and the propagated +1/-1 state.
int orc_tree(int32_t n, const int32_t* row_ptr, const int32_t* col, const int8_t* sign,
             uint64_t seed, int64_t t, int sampler, int32_t* level_out, int32_t* parent_out,
             int8_t* state_out) {
    if (sampler < SAMPLER_BFS || sampler > SAMPLER_KRUSKAL) return ORC_EINVAL;
    Graph g{n, row_ptr, col, sign};
    std::vector<int32_t> comp;
    label_components(g, comp);
    Tree T;
    build_sampled_tree(g, comp, seed, t, sampler, T);
    for (int32_t v = 0; v < n; ++v) {
        level_out[v] = T.level[v];
        parent_out[v] = T.parent[v];
        state_out[v] = T.state[v];
    }
    return ORC_OK;
}

// Alg. alg-balance for a given tree (parent array, -1 at roots; levels).
// flip_out is per CSR entry.  Returns the number of flipped edges.
int64_t orc_balance(int32_t n, const int32_t* row_ptr, const int32_t* col, const int8_t* sign,
                    const int32_t* level, const int32_t* parent, int8_t* flip_out) {
    Graph g{n, row_ptr, col, sign};
    Tree T;
    T.level.assign(level, level + n);
    T.parent.assign(parent, parent + n);
    T.parent_sign.assign(n, 1);
    for (int32_t v = 0; v < n; ++v)
        if (parent[v] >= 0) T.parent_sign[v] = (int8_t)edge_sign(g, parent[v], v);
    std::vector<int8_t> flip;
    int64_t s = balance_by_cycles(g, T, flip);
    std::memcpy(flip_out, flip.data(), flip.size());
    return s;
}

// Number of frustrated undirected edges under a +1/-1 vertex state: edges
// with sign(u,v) * s_u * s_v = -1.
int64_t orc_count(int32_t n, const int32_t* row_ptr, const int32_t* col, const int8_t* sign,
                  const int8_t* state) {
    int64_t c = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (u < col[e] && sign[e] * state[u] * state[col[e]] < 0) ++c;
    return c;
}

// Canonical words of a +1/-1 state (component anchors forced to +1).
void orc_canonical(int32_t n, const int32_t* row_ptr, const int32_t* col, const int8_t* state,
                   uint64_t* words_out) {
    Graph g{n, row_ptr, col, nullptr};
    std::vector<int32_t> comp;
    label_components(g, comp);
    std::vector<int8_t> st(state, state + n);
    auto w = canonical_words(n, comp, st);
    std::memcpy(words_out, w.data(), w.size() * sizeof(uint64_t));
}

void orc_hash128(int64_t nwords, const uint64_t* words, uint64_t* out2) {
    std::vector<uint64_t> w(words, words + nwords);
    state_hash(w, out2[0], out2[1]);
}

uint64_t orc_splitmix(uint64_t x) { return splitmix_output(x); }
int orc_hybrid_coin(uint64_t salt) { return hybrid_coin(salt); }
uint32_t orc_kruskal_weight(uint64_t salt, int32_t u, int32_t v) { return kruskal_weight(salt, u, v); }
uint32_t orc_fmix32(uint32_t x) { return murmur_fmix32(x); }

// One graphBpp sweep over trees t0 .. t1-1 (Alg. alg-index) with the given
// tree sampler (0 BFS, 1 randomized DFS, 2 the RDFS-BFS hybrid, 3 Kruskal on
// random weights).
//   flags bit 0: run the independent cross-checks on every tree;
//   flags bit 1: also key a second cloud by the paper's string form and
//                check that string keys and state keys pair up one to one.
// Outputs (any may be null):
//   tree_out[3*(t-t0) + {0,1,2}] = switches, key_hi, key_lo of tree t;
//   cloud_out[5*i + {0..4}] = key_hi, key_lo, freq, switches, first_tree of
//   entry i, entries sorted by (key_hi, key_lo); at most cloud_cap entries;
//   *cloud_size = number of distinct states;
//   best_out[0..1] = minimum switches and the first tree reaching it.
int orc_sweep(int32_t n, const int32_t* row_ptr, const int32_t* col, const int8_t* sign,
              uint64_t seed, int64_t t0, int64_t t1, int flags, uint64_t* tree_out,
              uint64_t* cloud_out, int64_t cloud_cap, int64_t* cloud_size, uint64_t* best_out,
              int sampler) {
    if (sampler < SAMPLER_BFS || sampler > SAMPLER_KRUSKAL) return ORC_EINVAL;
    Graph g{n, row_ptr, col, sign};
    std::vector<int32_t> comp;
    int32_t ncomp = label_components(g, comp);
    std::map<std::vector<uint64_t>, CloudValue> cloud;       // exact state -> value
    std::map<std::string, CloudValue> string_cloud;          // the paper's keys
    std::map<std::string, std::vector<uint64_t>> string_to_state;
    uint64_t best_s = UINT64_MAX, best_t = 0;
    Tree T;
    std::vector<int8_t> flip;
    for (int64_t t = t0; t < t1; ++t) {
        build_sampled_tree(g, comp, seed, t, sampler, T);
        int64_t s = balance_by_cycles(g, T, flip);  // s = number of sign differences
        if (flags & 1) {
            int rc = cross_check(g, comp, ncomp, T, flip);
            if (rc) return rc;
        }
        std::vector<uint64_t> key = canonical_words(n, comp, T.state);
        uint64_t hi, lo;
        state_hash(key, hi, lo);
        if (tree_out) {
            tree_out[3 * (t - t0) + 0] = (uint64_t)s;
            tree_out[3 * (t - t0) + 1] = hi;
            tree_out[3 * (t - t0) + 2] = lo;
        }
        auto it = cloud.find(key);
        if (it == cloud.end()) {  // new balanced state: S = s, C = 1
            CloudValue cv;
            cv.freq = 1; cv.switches = (uint64_t)s; cv.first_tree = (uint64_t)t;
            cloud.emplace(key, cv);
        } else {                  // seen before: C++
            it->second.freq += 1;
            if (it->second.switches != (uint64_t)s) return ORC_ESTATE;
        }
        if (flags & 2) {
            std::string b = paper_state_string(g, flip);
            auto sit = string_to_state.find(b);
            if (sit == string_to_state.end()) string_to_state.emplace(b, key);
            else if (sit->second != key) return ORC_ESTRING;
            auto& sv = string_cloud[b];
            if (sv.freq == 0) { sv.switches = (uint64_t)s; sv.first_tree = (uint64_t)t; }
            sv.freq += 1;
        }
        if ((uint64_t)s < best_s) { best_s = (uint64_t)s; best_t = (uint64_t)t; }
    }
    if ((flags & 2) && string_cloud.size() != cloud.size()) return ORC_ESTRING;
    // readout sorted by the 128-bit key; two exact states may not share a key
    std::vector<std::tuple<uint64_t, uint64_t, CloudValue>> rows;
    for (auto& kv : cloud) {
        uint64_t hi, lo;
        state_hash(kv.first, hi, lo);
        rows.emplace_back(hi, lo, kv.second);
    }
    std::sort(rows.begin(), rows.end(), [](const auto& a, const auto& b) {
        return std::make_pair(std::get<0>(a), std::get<1>(a)) <
               std::make_pair(std::get<0>(b), std::get<1>(b));
    });
    for (size_t i = 1; i < rows.size(); ++i)
        if (std::get<0>(rows[i]) == std::get<0>(rows[i - 1]) &&
            std::get<1>(rows[i]) == std::get<1>(rows[i - 1]))
            return ORC_ECOLLISION;
    if (cloud_size) *cloud_size = (int64_t)rows.size();
    if (cloud_out) {
        if ((int64_t)rows.size() > cloud_cap) return ORC_ECAP;
        for (size_t i = 0; i < rows.size(); ++i) {
            cloud_out[5 * i + 0] = std::get<0>(rows[i]);
            cloud_out[5 * i + 1] = std::get<1>(rows[i]);
            cloud_out[5 * i + 2] = std::get<2>(rows[i]).freq;
            cloud_out[5 * i + 3] = std::get<2>(rows[i]).switches;
            cloud_out[5 * i + 4] = std::get<2>(rows[i]).first_tree;
        }
    }
    if (best_out) { best_out[0] = best_s; best_out[1] = best_t; }
    return ORC_OK;
}

}  // extern "C"
