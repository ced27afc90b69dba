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
// launch's signal buffers, and its I/O.  deg and the tile range (the graph's
// tiles in the launch's all-rows tile list) serve the centring of 16-bit
// signals.
struct GraphDev {
  const int32_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *diag;
  int64_t row_off;
  GraphIO io;
  const double *deg;
  int32_t tile_lo, tile_hi;
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
  // 16-bit storage: the iterates hold x - c v_sigma (v_sigma = sqrt(d + sigma),
  // the eigenvector of A~_sigma with eigenvalue 1), c per graph, group and
  // column; the final combine adds c v_sigma back.
  bool centre = false;
  int64_t num_graphs = 1;
  // Block b works on tile b itself (the tile lists are already laid out so
  // that block b's XCD, b mod 8, owns the tile) instead of xcd_remap(b).
  bool identity_map = false;
  // With identity_map, the centring sums run over each graph's contiguous
  // tiles in this all-rows list (tile_lo/tile_hi index it).
  const TileDesc *centre_tiles = nullptr;
  const int32_t *centre_tile_graph = nullptr;
  int64_t num_centre_tiles = 0;
};

// Signal buffers of one column chunk: [R][C] storage-type rows.
struct ChunkBuffers {
  void *x0 = nullptr, *ping = nullptr, *pong = nullptr;
  void *saved[kMaxTerms] = {};  // NULL for the term the last pass forms
  double *centre_part = nullptr;  // [tiles][C + groups] partial sums (centring)
  double *centre = nullptr;       // [graphs][groups][C] multipliers c (centring)
};

// Whether filters of this storage type centre their signal (16-bit types).
inline bool centred_storage(int32_t storage) {
  return storage == GIFT_BF16 || storage == GIFT_F16;
}

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

// Pinned host staging for small uploads: a ring of buffers, each reused only
// after the copy that last read it has run.
class PinnedRing {
 public:
  PinnedRing() = default;
  PinnedRing(const PinnedRing &) = delete;
  PinnedRing &operator=(const PinnedRing &) = delete;
  ~PinnedRing();
  // A pinned buffer of at least `bytes` (waits for the slot's previous copy).
  gift_status acquire(size_t bytes, void **p);
  // The buffer from the last acquire is read by work enqueued on `st` so far.
  gift_status release(hipStream_t st);

 private:
  static constexpr int kSlots = 4;
  void *buf_[kSlots] = {};
  size_t cap_[kSlots] = {};
  hipEvent_t ev_[kSlots] = {};
  int next_ = 0, cur_ = -1;
};

// Enqueues the filter of n graphs, each with its own I/O, as one uncaptured
// launch sequence on `st`: every pass is one launch over the tiles of all
// graphs (tile class 0, widest column chunks: the arithmetic of filtering
// each graph alone).  Device scratch comes from the stream-ordered cache, the
// per-graph table goes through `ring`.
gift_status enqueue_dynamic_batch(const gift_graph *const *graphs, const GraphIO *ios, int32_t n,
                                  const gift_term *terms, int32_t nt, int32_t num_cols,
                                  int32_t in_dt, int32_t out_dt, hipStream_t st,
                                  PinnedRing &ring);
// Device bytes enqueue_dynamic_batch takes from the cache for these graphs.
size_t dynamic_batch_bytes(const gift_graph *const *graphs, int32_t n, int32_t storage,
                           int32_t num_terms, int32_t num_cols);

}  // namespace gift
