// Internal interface of the filter passes (filter.hip), shared by the
// single-graph entry point and the batch (batch.hip).
#pragma once

#include <vector>

#include "common.h"

namespace gift {

constexpr int kMaxTerms = 64;

// One graph's caller-side input and output (rows are the graph's cells).
struct GraphIO {
  const void *x_in;
  int64_t ld_in;
  void *y_out;
  int64_t ld_out;
  const uint8_t *fixed;  // may be NULL
  int64_t num_cells;
};

// One graph of a launch, for one sigma: its CSR (graph-local row and column
// indices), the normalised values of that sigma, where its rows start in the
// launch's signal buffers, and its I/O.
struct GraphDev {
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *diag;
  int64_t row_off;
  GraphIO io;
};

struct PlanGroup {
  double sigma;
  int32_t kmax;
  const void *val, *diag;  // single graph: this sigma's values
  const GraphDev *graphs;  // batch: device table [num_graphs] for this sigma
};

// Everything a filter launch sequence needs apart from its buffers.
struct FilterPlan {
  int32_t storage = GIFT_F32;
  int32_t tile_class = 0;
  int64_t R = 0;          // rows of all graphs
  int64_t nnz = 0;        // stored entries of all graphs
  int64_t cell_rows = 0;  // cell rows of all graphs
  int64_t nnz_cells = 0;  // entries in cell rows
  // Tiles of every pass and of the last pass (cell rows only); tile_graph
  // gives each tile's graph in a batch (NULL for a single graph).
  const TileDesc *tiles = nullptr;
  const int32_t *tile_graph = nullptr;
  int64_t num_tiles = 0;
  const TileDesc *final_tiles = nullptr;
  const int32_t *final_tile_graph = nullptr;
  int64_t num_final_tiles = 0;
  std::vector<PlanGroup> groups;  // ascending sigma
  GraphDev one{};                 // single graph (val/diag taken from the group)
  const gift_term *terms = nullptr;
  int32_t num_terms = 0;
  int32_t in_dtype = GIFT_F32, out_dtype = GIFT_F32;
  bool profile = true;  // bracket passes with profiler events
};

// Signal buffers of one column chunk: [R][C] storage-type rows.
struct ChunkBuffers {
  void *x0 = nullptr, *ping = nullptr, *pong = nullptr;
  void *saved[kMaxTerms] = {};  // NULL for the term the last pass forms
};

// Widest supported chunk (16, 8, 4, 2, 1) not above `remaining`.
int chunk_width(int remaining);
// Validates the terms against graph `g` and groups them by sigma.
gift_status plan_groups(const gift_graph *g, const gift_term *terms, int32_t nt,
                        std::vector<PlanGroup> *out);
// Device bytes of one chunk's buffers.
size_t chunk_buffer_bytes(const FilterPlan &pl, int C);
// Carves one chunk's buffers out of `base` and returns the bytes they take
// (with base == NULL only the size is meaningful).
size_t carve_chunk_buffers(const FilterPlan &pl, int C, unsigned char *base, ChunkBuffers *bf);
// Enqueues the prep and every pass of columns [col0, col0 + C) on `st`.
// Allocates nothing, so it can be captured into a HIP graph.
gift_status enqueue_filter_chunk(const FilterPlan &pl, const ChunkBuffers &bf, int C,
                                 int32_t col0, hipStream_t st);

}  // namespace gift
