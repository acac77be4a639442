/*
 * frustration.h - C ABI of the MI355X graphBpp sweep and graphL library
 * (libfrustration.so).
 *
 * The operations follow Shebaro & Tesic, "Scaling Frustration Index and
 * Corresponding Balanced State Discovery for Real Signed Graphs":
 *   - graphBpp, Alg. alg-index: sample k spanning trees of a signed graph,
 *     balance the graph on each tree (Alg. alg-balance), count the edge sign
 *     switches s, key the balanced state, and keep the frustration cloud
 *     B:(C, S) (Eq. eq-cloud); the approximate frustration index is
 *     min_i S(i) (Eq. eq-obj);
 *   - graphL, Eq. eq-loss_imbalance_new, its gradient and Alg. alg-gradient:
 *     relaxed vertex signs Gamma, loss sum over edges (1 - e_ij G_i G_j)/2,
 *     plain gradient descent, rounding at zero and an exact frustration count.
 *
 * Tree sampler (the paper's best, BFS, Section "Tree-Sampling techniques"),
 * made reproducible: tree t of a sweep with seed s takes as salt output t of
 * the SplitMix64 stream seeded with s; vertex u gets the 32-bit key
 * (fmix32(u) xor salt_lo) * (salt_hi | 1) mod 2^32 (fmix32: the MurmurHash3
 * finalizer), a bijection of u, so keys never tie.  The root of every connected
 * component is its minimum-key vertex, and the parent of every other vertex
 * is its minimum-key neighbour one BFS level closer to the root.  Vertex
 * states: root +1, child = parent * sign(tree edge); by Theorem t:HararyCut
 * this state frustrates exactly the edges Alg. alg-balance flips.  The cloud
 * key of a state is a 128-bit hash of its canonical form (each component
 * flipped so that its smallest vertex id is +1).
 *
 * Conventions
 *   - Every function returns FI_OK (0) or a negative FI_E* code.
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     current device); h_* and out_* are host pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on it unless marked "blocks".
 *   - The library never allocates device memory.  The caller allocates one
 *     workspace per graph (size from fi_graph_workspace_size), keeps it alive
 *     until fi_graph_destroy, and frees it afterwards.  Input CSR buffers are
 *     read only during fi_graph_create (the workspace keeps what it needs).
 *   - Errors found by kernels (a full cloud, a key collision) are sticky
 *     on the handle and returned by the next blocking call
 *     (fi_graph_status, fi_min_frustration, fi_cloud_read).
 *   - Every spanning forest is reachable: BFS trees of any depth (a path
 *     graph, a long grid) run on every schedule.
 *   - Results depend only on (graph, seed, tree indices), never on the
 *     schedule, the stream or how a tree range is split into calls.
 */
#ifndef FRUSTRATION_H
#define FRUSTRATION_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FI_OK = 0,
  FI_EINVAL = -1,      /* bad argument, row_ptr not 0..nnz non-decreasing, col out of range */
  FI_EASYM = -2,       /* an entry u->v without v->u of the same sign (an inconsistency) */
  FI_ESELFLOOP = -3,   /* an entry v->v */
  FI_EDUP = -4,        /* a repeated column in a row */
  FI_ESIGN = -5,       /* a sign other than +1 / -1 */
  FI_ERANGE = -6,      /* n or nnz >= 2^31, or a tree index >= 2^32 */
  FI_EUNSORTED = -7,   /* a row whose columns are not increasing */
  FI_ECAPACITY = -8,   /* more distinct balanced states than the cloud capacity */
  FI_EDEVICE = -9,     /* a HIP runtime call failed */
  FI_EDEPTH = -10,     /* a BFS tree deeper than 2^31 - 2 levels (cannot occur: depth < n) */
  FI_ECOLLISION = -11, /* two different states met under one 64-bit key half */
  FI_EWORKSPACE = -12, /* workspace missing, too small or misaligned (256 B) */
  FI_EORDER = -13      /* a bounded-cloud merge whose trees do not follow the last one's */
};

/* Opaque handle: views of the caller's workspace plus host-side settings. */
typedef struct fi_graph fi_graph;

/* One frustration-cloud entry (Eq. eq-cloud): key of the balanced state B,
 * its frequency C, its switch count S, and the first tree that produced it. */
typedef struct {
  uint64_t key_hi, key_lo;
  uint64_t freq;
  uint64_t switches;
  uint64_t first_tree;
} fi_cloud_entry;

/* ---------------------------------------------------------------- input cleaning */

/* Bytes of device workspace for fi_clean of E raw entries.  FI_ERANGE if
 * 2E >= 2^31. */
int fi_clean_workspace_size(int32_t n, int64_t E, size_t* out_bytes);

/* The paper's input cleaning (Section "Implementation": duplicates,
 * inconsistencies, self-loops and invalid signs are eliminated) on the GPU,
 * producing the symmetric sorted CSR that fi_graph_create takes.  Raw entry
 * i is (d_src[i], d_dst[i], d_sign[i]), int32 each, in any order and either
 * direction.  An entry with an endpoint outside 0 .. n-1 or a sign other
 * than +1 / -1 is invalid and dropped; self-loops are dropped; a vertex pair
 * met with one sign keeps one edge (the other entries are duplicates); a
 * pair met with both signs is inconsistent and dropped.  Outputs: d_row_ptr
 * int32[n+1], d_col int32 and d_sign_out int8 with room for 2E entries (the
 * first row_ptr[n] are written, rows sorted), and h_counts int64[5] (host) =
 * kept edges, invalid entries, self-loops, duplicate entries, inconsistent
 * pairs.  Blocks. */
int fi_clean(int32_t n, int64_t E, const int32_t* d_src, const int32_t* d_dst, const int32_t* d_sign,
             void* d_workspace, size_t ws_bytes, int32_t* d_row_ptr, int32_t* d_col,
             int8_t* d_sign_out, int64_t* h_counts, void* stream);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc, or that hold no workspace for cleaning):
 * fi_clean without a workspace argument.  The workspace is a 64 MiB device
 * array inside the library, one per GPU, held until the process ends; it
 * takes up to FI_CLEAN_NO_ALLOC_MAX_ENTRIES raw entries (FI_ERANGE beyond).
 * Outputs, counts and errors are those of fi_clean.  No device memory is
 * allocated or freed.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  Blocks. */
#define FI_CLEAN_NO_ALLOC_MAX_ENTRIES 1000000
int fi_clean_no_alloc(int32_t n, int64_t E, const int32_t* d_src, const int32_t* d_dst,
                      const int32_t* d_sign, int32_t* d_row_ptr, int32_t* d_col,
                      int8_t* d_sign_out, int64_t* h_counts, void* stream);

/* ---------------------------------------------------------------- graph */

/* Bytes of device workspace for a graph with n vertices, nnz CSR entries
 * (2 per undirected edge) and a cloud of up to cloud_capacity distinct
 * states.  Pure host arithmetic. */
int fi_graph_workspace_size(int32_t n, int64_t nnz, int64_t cloud_capacity, size_t* out_bytes);

/* Upload and validate a signed graph (blocks).
 * Input: symmetric CSR of a simple undirected signed graph - d_row_ptr
 * int32[n+1] (0 .. nnz, non-decreasing), d_col int32[nnz] (strictly
 * increasing within each row), d_sign int8[nnz] in {+1, -1}, each edge
 * present in both directions with one sign.  The paper's input cleaning
 * (Section "Implementation": duplicates, inconsistencies, self-loops,
 * invalid signs) is not done here: such inputs are rejected, and when an
 * input has several defects the first of FI_ERANGE, FI_EINVAL, FI_ESIGN,
 * FI_ESELFLOOP, FI_EDUP, FI_EUNSORTED, FI_EASYM is returned.  Builds, inside d_workspace (>= fi_graph_workspace_size bytes,
 * 256-byte aligned): the packed adjacency, the upper-triangle edge list,
 * connected components with their anchors (smallest vertex id), and an
 * empty cloud.  On success *out owns host memory only; release it with
 * fi_graph_destroy. */
int fi_graph_create(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                    const int8_t* d_sign, int64_t cloud_capacity, void* d_workspace,
                    size_t ws_bytes, void* stream, fi_graph** out);

/* Release the handle (host memory).  Does not touch the workspace. */
void fi_graph_destroy(fi_graph* g);

/* Number of connected components, and the number of isolated vertices. */
int fi_graph_info(fi_graph* g, int32_t* out_components, int32_t* out_isolated);

/* Blocks until the stream is idle; returns the sticky kernel error, if any. */
int fi_graph_status(fi_graph* g, void* stream);

/* ---------------------------------------------------------------- sweep */

/* Alg. alg-index over trees t = 0 .. K-1: for each tree, build the BFS
 * spanning forest, propagate states, count the frustrated edges (the
 * switches s of Alg. alg-balance), hash the canonical state and
 * insert-or-increment it in the cloud (new: C = 1, S = s; seen: C++).
 * Accumulates into the current cloud; asynchronous. */
int fi_sweep(fi_graph* g, int64_t K, uint64_t seed, void* stream);

/* The same for trees t0 .. t1-1 (0 <= t0 <= t1 <= 2^32), so that a sweep can
 * be split, resumed or sharded with identical results.  If d_tree_switches is
 * not NULL it receives uint64[t1 - t0], the switch count of each tree. */
int fi_sweep_range(fi_graph* g, int64_t t0, int64_t t1, uint64_t seed,
                   uint64_t* d_tree_switches, void* stream);

/* Eq. eq-obj: Fr = min_i S(i) over every tree inserted since the last reset,
 * and the smallest tree index reaching it (blocks).  FI_EINVAL if empty. */
int fi_min_frustration(fi_graph* g, uint64_t* out_switches, uint64_t* out_first_tree,
                       void* stream);

/* Number of distinct states in the cloud (blocks). */
int fi_cloud_size(fi_graph* g, int64_t* out, void* stream);

/* Copy the cloud to host memory, sorted by (key_hi, key_lo) (blocks).
 * Writes min(size, cap) entries and sets *written to the cloud size.
 * FI_ECOLLISION if two different states shared a key half or one key met
 * two switch counts. */
int fi_cloud_read(fi_graph* g, fi_cloud_entry* h_out, int64_t cap, int64_t* written,
                  void* stream);

/* Empty the cloud and the running minimum; clears the sticky error. */
int fi_cloud_reset(fi_graph* g, void* stream);

/* Re-insert saved entries (a checkpoint from fi_cloud_read) so that a sweep
 * can resume: entries are merged as if their trees had been swept (freq
 * added, first tree kept at the minimum).  h_entries is host memory. */
int fi_cloud_load(fi_graph* g, const fi_cloud_entry* h_entries, int64_t count, void* stream);

/* The canonical state of tree t: n bits as uint64[ceil(n/64)] (vertex v is
 * bit v%64 of word v/64; set = -1), written to d_bits_out.  Also returns the
 * tree's switch count in *d_switches_out if not NULL (device pointer). */
int fi_tree_state(fi_graph* g, uint64_t seed, int64_t t, uint64_t* d_bits_out,
                  uint64_t* d_switches_out, void* stream);

/* Exact frustration count (the switch count of Alg. alg-index, the number
 * of edges whose sign disagrees with the state): for B states given as bitmaps d_bits
 * uint64[B][ceil(n/64)] (set bit = vertex state -1), d_counts[b] = number of
 * undirected edges (u, v) with sign(u,v) * s_u * s_v = -1.  Groups of 64
 * states are transposed to one word per vertex and counted in one pass over
 * the edge list.  Uses the graph's workspace: calls on one handle must not
 * overlap. */
int fi_count(fi_graph* g, const uint64_t* d_bits, int32_t B, uint64_t* d_counts, void* stream);

/* ---------------------------------------------------------------- graphL */

/* Eq. eq-loss_imbalance_new for R restarts at once: d_gamma float32[n][R]
 * (restart r is column r), d_loss float64[R] with
 * L_r = sum over undirected edges (1 - e_ij G_ir G_jr) / 2.
 * Each edge term is formed in float32 and summed in float64 in a fixed order
 * (deterministic).  1 <= R <= 64. */
int fi_graphl_forward(fi_graph* g, const float* d_gamma, int32_t R, double* d_loss, void* stream);

/* Gradient of sum_r w_r L_r: d_grad_gamma[i][r] = -1/2 * w_r * sum over
 * neighbours j of e_ij G_jr, with w = d_grad_loss float64[R] (NULL = all 1).
 * One gather per CSR row, no atomics. */
int fi_graphl_backward(fi_graph* g, const float* d_gamma, int32_t R, const double* d_grad_loss,
                       float* d_grad_gamma, void* stream);

/* One step of Alg. alg-gradient's update loop for all restarts:
 * d_gamma_out = d_gamma_in - alpha * dL/dGamma (buffers must not overlap). */
int fi_graphl_step(fi_graph* g, const float* d_gamma_in, int32_t R, float alpha,
                   float* d_gamma_out, void* stream);

/* Bytes of the caller's buffer that fi_graphl_descend keeps its scales in,
 * for R restarts: 16 B per (component with an edge, restart). */
int fi_graphl_aux_size(fi_graph* g, int32_t R, size_t* out_bytes);

/* Alg. alg-gradient's update loop, `steps` steps for all restarts, with an
 * overflow policy for large graphs.  Each step multiplies Gamma by
 * (I + alpha/2 * A_signed), which grows by up to (1 + alpha * lambda_max / 2)
 * per step; power-law hubs make lambda_max large enough to overflow float32
 * in a few hundred steps, while small components barely grow.  Every
 * (connected component, restart) pair keeps its own power-of-two scale:
 * whenever the pair's largest |Gamma| reached 2^rescale_log2 (0 = 64;
 * 1 .. 100) after a step, the next step reads the pair scaled by
 * 2^-rescale_log2 and adds rescale_log2 to its log2 scale.  The true
 * iterate is d_gamma[i][r] * 2^scale(i, r) (fi_graphl_scales); scaling by a
 * power of two is exact, so the stored iterates are the plain descent's bit
 * for bit up to that factor (unless an entry falls 2^-149 below its own
 * component's largest), and the rounded states of the final loop are
 * unchanged.  d_gamma float32[n][R] holds Gamma_0 on entry and the result
 * on return; d_work is a buffer of the same size (no overlap); d_aux
 * (fi_graphl_aux_size bytes, 256-byte aligned) receives the scales and is
 * overwritten by each call.  Rows of more than 1,024 entries are summed by a
 * whole workgroup in a fixed order; results are deterministic.  Kernels and
 * one device copy only. */
int fi_graphl_descend(fi_graph* g, float* d_gamma, float* d_work, int32_t R, float alpha,
                      int64_t steps, int32_t rescale_log2, void* d_aux, size_t aux_bytes,
                      void* stream);

/* The log2 scale of every vertex and restart after fi_graphl_descend:
 * d_out int32[n][R] (0 for vertices without edges). */
int fi_graphl_scales(fi_graph* g, const void* d_aux, int32_t R, int32_t* d_out, void* stream);

/* Alg. alg-gradient's final loop: theta = +1 where Gamma >= 0 else -1, then
 * the exact frustration count of every restart: d_counts uint64[R].
 * d_bits_out (uint64[R][ceil(n/64)], set = -1) receives the rounded states
 * if not NULL.  Gamma is read once; all R restarts are counted in one pass
 * over the edge list.  Uses the graph's workspace: calls on one handle must
 * not overlap. */
int fi_round_count(fi_graph* g, const float* d_gamma, int32_t R, uint64_t* d_counts,
                   uint64_t* d_bits_out, void* stream);

/* ---------------------------------------------------------------- batches */

/* Many independent graphs swept together (Alg. alg-index per graph), for
 * batches of small and medium graphs of uneven size.
 * The graphs are concatenated: graph i has vertices
 * h_vertex_offsets[i] .. h_vertex_offsets[i+1]-1 (G+1 host int64 offsets
 * starting at 0) and CSR entries h_nnz_offsets[i] .. h_nnz_offsets[i+1]-1;
 * d_row_ptr int32[total_n + G] holds each graph's own row_ptr (starting at 0)
 * back to back, and d_col holds graph-local column ids.  Each graph must
 * satisfy the fi_graph_create contract on its own, have at most 1,000,000
 * vertices, and is swept with its own vertex ids, exactly as if it had been
 * uploaded alone.  Every graph keeps its own cloud of up to
 * cloud_capacity_per_graph states.  The workspace (fi_batch_workspace_size
 * bytes, 256-byte aligned, owned by the caller) must outlive the handle; the
 * input arrays may be freed once fi_batch_create returns.  Errors: FI_EINVAL
 * for bad offsets, sizes or row_ptr, the fi_graph_create codes for a graph
 * that breaks the contract, FI_EWORKSPACE for a short workspace.  The handle
 * serves fi_batch_sweep, fi_graph_status, fi_set_schedule (block and grid
 * only), fi_get_schedule, fi_prof_enable / fi_prof_read and
 * fi_graph_destroy; the single-graph calls return FI_EINVAL on it. */
int fi_batch_workspace_size(int32_t G, const int64_t* h_vertex_offsets, const int64_t* h_nnz_offsets,
                            int64_t cloud_capacity_per_graph, size_t* out_bytes);
int fi_batch_create(int32_t G, const int64_t* h_vertex_offsets, const int64_t* h_nnz_offsets,
                    const int32_t* d_row_ptr, const int32_t* d_col, const int8_t* d_sign,
                    int64_t cloud_capacity_per_graph, void* d_workspace, size_t ws_bytes,
                    void* stream, fi_graph** out);

/* Trees t = 0 .. trees_per_graph-1 of every graph (all graphs use `seed`):
 * one launch per size class, work items (graph, tree) ordered largest graph
 * first and drawn by persistent workgroups.  Each call starts from empty
 * clouds.  Outputs, device memory: d_min_per_graph uint64[G][2] =
 * (minimum switches, first tree reaching it), d_distinct_per_graph (may be
 * NULL) uint64[G] = distinct balanced states among the graph's trees.
 * Launches kernels only (no host synchronisation, memset or allocation), so
 * it may be recorded into a HIP graph on `stream`. */
int fi_batch_sweep(fi_graph* b, int64_t trees_per_graph, uint64_t seed, uint64_t* d_min_per_graph,
                   uint64_t* d_distinct_per_graph, void* stream);

/* The cloud of graph `graph` (0 .. G-1) of a batch after fi_batch_sweep
 * (Eq. eq-cloud per graph): copied to host memory sorted by (key_hi,
 * key_lo), as fi_cloud_read does for a single graph; first_tree counts the
 * graph's own trees from 0.  Blocks; returns the batch's sticky error, if
 * any, or FI_ECOLLISION. */
int fi_batch_cloud_read(fi_graph* b, int32_t graph, fi_cloud_entry* h_out, int64_t cap,
                        int64_t* written, void* stream);

/* ---------------------------------------------------------------- tree samplers */

/* The spanning-tree sampler of the sweep (Section "Tree-Sampling techniques
 * for graphBpp"), made reproducible like BFS: every random choice comes from
 * tree t's salt.
 *   0  BFS (default): the min-key rule above.
 *   1  randomized DFS: from each component's minimum-key vertex, move to the
 *      unvisited neighbour of smallest key (the shuffled adjacency order),
 *      back up when there is none.
 *   2  the RDFS-BFS hybrid of Alg. alg-hybrid: per tree a uniformly
 *      distributed 0/1 (the top bit of the SplitMix64 finalizer of the salt)
 *      picks BFS (0) or randomized DFS (1).
 *   3  Kruskal on random weights: edge (u, v), u < v, weighs the high half
 *      of the SplitMix64 finalizer of salt xor (u << 32 | v); ties go to the
 *      earlier edge of the sorted edge list; the tree is the unique minimum
 *      spanning forest (computed here by Boruvka rounds).
 * Samplers other than BFS run one tree per workgroup (schedule paths 1 and
 * 2, whatever fi_set_schedule chose), so they need the tree in LDS (n up to
 * about 8,000 for Kruskal, 10,000 for DFS) or a workspace slot (n <= 10^6):
 * FI_ERANGE otherwise.  fi_sweep_stats takes BFS only (FI_EINVAL). */
int fi_set_sampler(fi_graph* g, int32_t sampler);
int fi_get_sampler(fi_graph* g, int32_t* out);

/* ---------------------------------------------------------------- switch lists and statistics */

/* The upper-triangle edge list: d_uv_out int32[2m] receives (u, v) with
 * u < v for every undirected edge, in increasing (u, v) order.  Edge e of
 * fi_sweep_stats and the order of fi_switch_list refer to this list. */
int fi_edge_list(fi_graph* g, int32_t* d_uv_out, void* stream);

/* The balanced state Sigma' as the list of edges to switch (the paper's
 * concluding remarks: the method yields the edges to switch).  For a state
 * d_bits (n bits as uint64[ceil(n/64)], vertex v is bit v%64 of word v/64,
 * set = -1), every undirected edge (u, v) with sign(u, v) * s_u * s_v = -1:
 * for a tree's state (fi_tree_state) these are exactly the edges
 * Alg. alg-balance switches, for a rounded graphL state (fi_round_count)
 * the edges Alg. alg-gradient flips.  Writes the first min(count, cap)
 * pairs (u, v), u < v, in edge-list order to d_uv_out int32[2 cap] and the
 * count to *d_count (device uint64).  Uses the graph's workspace: calls on
 * one handle must not overlap. */
int fi_switch_list(fi_graph* g, const uint64_t* d_bits, int32_t* d_uv_out, int64_t cap,
                   uint64_t* d_count, void* stream);

/* Cloud statistics over trees t0 .. t1-1, each tree counted once, so each
 * state of the cloud weighs its count C (the frequencies the frustration
 * cloud keeps for consensus features, Section "The graphL Proof of Concept"):
 * d_vertex_minus uint64[n] (may be NULL) gets, added to what it holds, the
 * number of trees whose canonical state (each component's smallest vertex
 * at +1) puts v at -1; d_edge_switched uint64[m] (may be NULL) gets the
 * number of trees whose balanced state switches edge e (fi_edge_list
 * order).  The trees also enter the cloud, as with fi_sweep_range.  Runs on
 * the multi-tree schedule whatever fi_set_schedule chose (results are the
 * same on every schedule). */
int fi_sweep_stats(fi_graph* g, int64_t t0, int64_t t1, uint64_t seed, uint64_t* d_vertex_minus,
                   uint64_t* d_edge_switched, void* stream);

/* ---------------------------------------------------------------- memory-bound cloud */

/* Alg. alg-scale (appendix, scaling graphBpp for large signed graphs): a
 * frustration cloud of at most F_max states that keeps the best ones.
 * Readings of the printed algorithm, which is garbled: the state replaced
 * when the cloud is full is the worst one (largest S, and among equal S the
 * one whose first tree is latest), not the argmin printed; a repeat of a
 * held state always counts (C is the count through all k trees); below
 * F_max every new state is kept; a new state replaces the worst only if its
 * S is strictly smaller.  The result is the F_max best distinct states by
 * (S, first tree), each with its count over every tree swept, and
 * Fr = min S is the same as with an unbounded cloud.
 *
 * The table lives in a caller-owned workspace (fi_bcloud_workspace_size
 * bytes, 256-byte aligned, kept until fi_bcloud_destroy) of about 160 B per
 * entry.  Trees are swept in chunks into a graph's own cloud, which serves
 * as the staging table, and merged here in tree order; `staging` (1 ..
 * 8192) bounds the distinct states one merge takes, so a graph merged into
 * this cloud needs cloud_capacity <= staging. */
typedef struct fi_bcloud fi_bcloud;

/* Bytes of workspace for F_max entries (1 .. 2^31) and `staging` candidates
 * per merge.  Pure host arithmetic. */
int fi_bcloud_workspace_size(int64_t f_max, int64_t staging, size_t* out_bytes);

/* The largest F_max whose workspace fits in cap_bytes (the step of Alg.
 * alg-scale that sizes the bounded cloud from a memory cap, with the device
 * memory the caller grants as the cap).  FI_EWORKSPACE if not even one entry fits.  Pure host arithmetic. */
int fi_bcloud_fmax_for(size_t cap_bytes, int64_t staging, int64_t* out_fmax);

/* Empty table in d_workspace (blocks).  *out owns host memory only. */
int fi_bcloud_create(int64_t f_max, int64_t staging, void* d_workspace, size_t ws_bytes,
                     void* stream, fi_bcloud** out);
void fi_bcloud_destroy(fi_bcloud* c);

/* Empty the table, its counters and its sticky error; the next merge may
 * start at any tree. */
int fi_bcloud_reset(fi_bcloud* c, void* stream);

/* Merge the states in g's cloud, which must hold exactly trees t0 .. t1-1
 * (swept with fi_sweep_range after an empty cloud), into c, then empty g's
 * cloud.  t0 must equal the previous merge's t1 (FI_EORDER otherwise; a
 * staged state whose first tree lies outside [t0, t1) sets the sticky
 * FI_EORDER).  FI_EINVAL if g's cloud_capacity exceeds c's staging.  A
 * sticky error of g's cloud (capacity, depth, collision) moves into c.
 * Kernels only. */
int fi_bcloud_merge(fi_graph* g, fi_bcloud* c, int64_t t0, int64_t t1, void* stream);

/* Alg. alg-scale over trees t0 .. t1-1: empties g's cloud, then sweeps and
 * merges chunks of `chunk` trees (0: min(cloud_capacity, staging); larger
 * is FI_EINVAL).  Results do not depend on the chunk size or schedule. */
int fi_sweep_bounded(fi_graph* g, fi_bcloud* c, int64_t t0, int64_t t1, uint64_t seed,
                     int64_t chunk, void* stream);

/* Entries held (blocks); returns the sticky error, if any. */
int fi_bcloud_size(fi_bcloud* c, int64_t* out, void* stream);

/* Copy the entries to host memory sorted by (key_hi, key_lo) (blocks);
 * writes min(size, cap) and sets *written to the size. */
int fi_bcloud_read(fi_bcloud* c, fi_cloud_entry* h_out, int64_t cap, int64_t* written,
                   void* stream);

/* Fr = min S over the trees merged and the first tree reaching it (blocks);
 * FI_EINVAL if empty. */
int fi_bcloud_min(fi_bcloud* c, uint64_t* out_switches, uint64_t* out_first_tree, void* stream);

/* Trees merged since the last reset, and the entries dropped (states
 * replaced or turned away, once per merge that dropped them) (blocks). */
int fi_bcloud_stats(fi_bcloud* c, int64_t* out_trees, int64_t* out_dropped, void* stream);

/* ---------------------------------------------------------------- schedule */

/* How a sweep is laid on the GPU.  Every schedule gives bit-identical
 * results; fi_set_schedule only changes speed.  path: 0 = automatic (path 1
 * when the tree fits LDS, 2 while n + m/2 <= 135,000 with m undirected
 * edges, else 5; the block is then chosen from the graph's size and the
 * sampler, the block field is ignored, and a grid of 0 is sized to the
 * graph), 1 = one workgroup per tree with the tree state in LDS
 * (n <= 12,000), 2 = one workgroup per tree with the tree state in workspace memory
 * (n <= 1,000,000), 3 = the whole grid on a few trees at a time
 * (persistent cooperative kernel, any n), 4 = the whole grid on 64 trees
 * at once with one bit per tree in each field of a per-vertex record
 * (cooperative, any n; fi_tree_state falls back to path 3), 5 = the same
 * with 128 trees at once (two-word fields; a vertex's record is one 64-byte
 * line, so a pass moves about as many lines as a pass of 64; not for batch
 * handles).  block: threads per workgroup (256, 512 or 1024); grid:
 * workgroups (0 = default; on paths 4 and 5 one per 16,384 of n + m/2, a
 * multiple of 8, at least 64, at most what can be resident); heavy: degree above
 * which a top-down frontier vertex is expanded by several workgroups
 * (path 3, >= 32); batch: trees in flight on path 3 (1 .. 8). */
typedef struct {
  int32_t path;
  int32_t block;
  int32_t grid;
  int32_t heavy;
  int32_t batch;
} fi_schedule;

int fi_set_schedule(fi_graph* g, const fi_schedule* s);
int fi_get_schedule(fi_graph* g, fi_schedule* out);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of the sweep kernel (0) and of the exact count (1; in
 * fi_round_count the rounding and the count).  Enable, run,
 * then read: fi_prof_read blocks and returns the summed milliseconds and the
 * number of launches since the last enable. */
int fi_prof_enable(fi_graph* g, int on);
int fi_prof_read(fi_graph* g, int kernel, double* out_ms, int64_t* out_launches);

/* Phase log of the multi-tree sweep (paths 4 and 5), for profiling: while
 * d_log (device, uint64[cap], cap >= 4) is set, workgroup 0 of every
 * launch appends after each grid-wide barrier a record (phase << 32 |
 * BFS level, time): d_log[0] counts the records (the caller zeroes it),
 * record i sits at d_log[2 + 2 i] and d_log[3 + 2 i], records past cap are
 * dropped, and time is the GPU's constant-rate real-time counter (100 MHz).
 * Phases: 0 launch start, 1 reset, 2 root search, 3 big-component roots,
 * 4 lists of a level, 5 pull of a level, 6 split rows of a level, 7 counts
 * and keys, 8 cloud insert.  NULL turns the log off. */
int fi_prof_phases(fi_graph* g, uint64_t* d_log, int64_t cap);

/* Measurement aid, not part of the method: the neighbour gathers of one
 * dense pull level of the multi-tree sweep, alone.  For every e < count,
 * reads the first 32 bytes (two 16-byte loads) of the 64-byte record
 * min(d_idx[e] & 0x7FFFFFFF, n_records - 1) of d_records (device,
 * 64 * n_records bytes, 16-byte aligned) and discards them; d_sink (device,
 * one uint32) is written only with probability 2^-32, so that the loads are
 * kept.  With a graph's adjacency (col, in CSR order) as d_idx it times what
 * the memory system needs for one level's gathers; with uniform random
 * indices, the random-access ceiling of such reads.  FI_EINVAL for count < 0,
 * n_records outside 1 .. 2^31 or a missing pointer. */
int fi_probe_gather(const uint32_t* d_idx, int64_t count, const void* d_records, int64_t n_records,
                    uint32_t* d_sink, void* stream);

const char* fi_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* FRUSTRATION_H */
