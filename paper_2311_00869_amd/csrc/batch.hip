// Many independent graphs in one launch (placeholder entry points until the
// batched sweep lands).
#include <hip/hip_runtime.h>

#include "fi_internal.h"

extern "C" {

int fi_batch_workspace_size(int32_t G, const int64_t* h_vertex_offsets,
                            const int64_t* h_nnz_offsets, size_t* out_bytes) {
  (void)G; (void)h_vertex_offsets; (void)h_nnz_offsets; (void)out_bytes;
  return FI_EINVAL;
}

int fi_batch_create(int32_t G, const int64_t* h_vertex_offsets, const int64_t* h_nnz_offsets,
                    const int32_t* d_row_ptr, const int32_t* d_col, const int8_t* d_sign,
                    void* d_workspace, size_t ws_bytes, void* stream, fi_graph** out) {
  (void)G; (void)h_vertex_offsets; (void)h_nnz_offsets; (void)d_row_ptr; (void)d_col;
  (void)d_sign; (void)d_workspace; (void)ws_bytes; (void)stream;
  if (out) *out = nullptr;
  return FI_EINVAL;
}

int fi_batch_sweep(fi_graph* b, int64_t trees_per_graph, uint64_t seed, uint64_t* d_min_per_graph,
                   uint64_t* d_distinct_per_graph, void* stream) {
  (void)b; (void)trees_per_graph; (void)seed; (void)d_min_per_graph; (void)d_distinct_per_graph;
  (void)stream;
  return FI_EINVAL;
}

}  // extern "C"
