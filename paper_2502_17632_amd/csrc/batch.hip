// Batched filter: many resident graphs (designs) filtered with the same terms
// and column count by one launch sequence.  Every pass covers the tiles of
// all graphs in one launch; each tile names its graph, whose CSR, normalised
// values, I/O and row offset in the batch's signal buffers come from a small
// device table (filter.hip).  The sequence for the chosen schedule is
// captured once into a HIP graph and replayed by every run; a run only
// uploads the table with the caller's I/O pointers and launches the graph.
//
// Schedules differ in the tile class (entries per tile and the long-row
// split), in the column chunk width (one pass sequence per chunk: wide
// chunks gather longer signal rows, narrow ones re-read the structure but
// stage products in LDS) and in the tile layout: chunks of consecutive tiles
// dealt round-robin to the XCDs, or every graph on one XCD so that the
// signal rows its tiles gather stay in that XCD's L2.  The autotuner captures every candidate, times its
// replays and keeps the fastest; the choice is cached per shape class.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "common.h"
#include "devutil.h"
#include "filter.h"

namespace gift {
namespace {

struct ConcatSrc {
  const TileDesc *src;
  int64_t count;
  int64_t out_off;
  int64_t graph;
};

// out[out_off + i] = src[i], out_graph[out_off + i] = graph for every source
// (blockIdx.x) and i < count; blockIdx.y strides over a source's tiles.
__global__ __launch_bounds__(kBlock) void k_concat_tiles(const ConcatSrc *srcs, TileDesc *out,
                                                         int32_t *out_graph) {
  const ConcatSrc s = gload(srcs, blockIdx.x);
  const gptr<int32_t> og = to_global(out_graph);
  for (int64_t i = static_cast<int64_t>(blockIdx.y) * kBlock + threadIdx.x; i < s.count;
       i += static_cast<int64_t>(gridDim.y) * kBlock) {
    gstore(out, s.out_off + i, gload(s.src, i));
    og[s.out_off + i] = static_cast<int32_t>(s.graph);
  }
}

constexpr int kSlots = 4;  // pinned staging slots for the I/O table

struct Candidate {
  int32_t tile_class;
  int32_t chunk;   // widest column chunk
  int32_t affine;  // 1: XCD-affine tile layout, 0: chunks dealt round-robin
};

// out[p] = src[perm[p]] (and its graph) for perm[p] >= 0, else an empty tile
// of graph `pad_graph` (rows [0, 0), entries [0, 0)).
__global__ void k_permute_tiles(const int32_t *perm, int64_t n, const TileDesc *src,
                                const int32_t *src_graph, int32_t pad_graph, TileDesc *out,
                                int32_t *out_graph) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t q = perm[p];
  gstore(out, p, q >= 0 ? gload(src, q) : TileDesc{0, 0, 0, 0});
  out_graph[p] = q >= 0 ? src_graph[q] : pad_graph;
}

// Column chunks of `num_cols` columns with chunks at most `widest` wide.
std::vector<int> chunk_list(int num_cols, int widest) {
  std::vector<int> out;
  for (int c0 = 0; c0 < num_cols;) {
    const int C = chunk_width(std::min(widest, num_cols - c0));
    out.push_back(C);
    c0 += C;
  }
  return out;
}

using TuneKey = std::tuple<int, int, int, int, int, int, int>;
struct TuneCache {
  std::mutex m;
  std::map<TuneKey, Candidate> best;
};
TuneCache &tune_cache() {
  static TuneCache *c = new TuneCache();
  return *c;
}

int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

}  // namespace
}  // namespace gift

using namespace gift;

struct gift_batch {
  int device = 0;
  hipStream_t home = nullptr;     // stream the batch's memory is ordered on
  hipStream_t capture = nullptr;  // owned, used for stream capture only
  std::vector<const gift_graph *> graphs;
  std::vector<gift_term> terms;
  int32_t num_cols = 0, in_dtype = GIFT_F32, out_dtype = GIFT_F32, storage = GIFT_F32;
  FilterPlan plan;  // tiles/tile class of the chosen schedule
  std::vector<int> chunks;
  int64_t R = 0, nnz = 0, cells = 0, nnz_cells = 0;
  // concatenated tiles of every class: all rows, and cell rows only
  TileDesc *tiles[kTileClasses] = {};
  int32_t *tile_graph[kTileClasses] = {};
  int64_t num_tiles[kTileClasses] = {};
  TileDesc *ftiles[kTileClasses] = {};
  int32_t *ftile_graph[kTileClasses] = {};
  int64_t num_ftiles[kTileClasses] = {};
  // the same tiles laid out per XCD (XCD-affine schedule): every graph is
  // given to one XCD and block b (on XCD b mod 8) takes tile b; short XCD
  // lists are padded with empty tiles
  TileDesc *atiles[kTileClasses] = {};
  int32_t *atile_graph[kTileClasses] = {};
  int64_t num_atiles[kTileClasses] = {};
  TileDesc *aftiles[kTileClasses] = {};
  int32_t *aftile_graph[kTileClasses] = {};
  int64_t num_aftiles[kTileClasses] = {};
  // graph table [groups][graphs]
  std::vector<GraphDev> table;
  GraphDev *table_dev = nullptr;
  GraphDev *staging[kSlots] = {};
  hipEvent_t slot_done[kSlots] = {};
  int slot = 0;
  unsigned char *buffers = nullptr;
  size_t buffer_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t last_run = nullptr;
  gift_batch_info info{};
};

namespace gift {
namespace {

void free_batch(gift_batch *b) {
  if (b->last_run) (void)hipEventSynchronize(b->last_run);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (int s = 0; s < kSlots; ++s) {
    if (b->slot_done[s]) {
      (void)hipEventSynchronize(b->slot_done[s]);
      (void)hipEventDestroy(b->slot_done[s]);
    }
    if (b->staging[s]) (void)hipHostFree(b->staging[s]);
  }
  for (int c = 0; c < kTileClasses; ++c) {
    dev_free(b->tiles[c], b->home);
    dev_free(b->tile_graph[c], b->home);
    dev_free(b->ftiles[c], b->home);
    dev_free(b->ftile_graph[c], b->home);
    dev_free(b->atiles[c], b->home);
    dev_free(b->atile_graph[c], b->home);
    dev_free(b->aftiles[c], b->home);
    dev_free(b->aftile_graph[c], b->home);
  }
  dev_free(b->table_dev, b->home);
  dev_free(b->buffers, b->home);
  if (b->last_run) (void)hipEventDestroy(b->last_run);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

// Concatenates `count(g)` leading tiles of every graph's class-c list.
gift_status concat_tiles(gift_batch *b, int c, bool cells_only, TileDesc **out,
                         int32_t **out_graph, int64_t *total) {
  std::vector<ConcatSrc> src;
  int64_t off = 0;
  int64_t most = 0;
  for (size_t g = 0; g < b->graphs.size(); ++g) {
    const gift_graph *gr = b->graphs[g];
    const int64_t n = cells_only ? gr->num_tiles_cells[c] : gr->num_tiles[c];
    if (n == 0) continue;
    src.push_back(ConcatSrc{gr->tiles[c], n, off, static_cast<int64_t>(g)});
    off += n;
    most = std::max(most, n);
  }
  *total = off;
  if (off >= (int64_t(1) << 31) - 1)
    return set_error(GIFT_EUNSUPPORTED, "batch has %lld tiles (limit 2^31 - 1)",
                     static_cast<long long>(off));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(out), sizeof(TileDesc) * (off + 1), b->home,
                     "batch tiles"));
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(out_graph), sizeof(int32_t) * (off + 1),
                     b->home, "batch tile graphs"));
  if (src.empty()) return GIFT_OK;
  Scratch sc(b->home);
  ConcatSrc *dsrc = nullptr;
  GIFT_TRY(sc.get(&dsrc, src.size(), "tile sources"));
  GIFT_HIP(hipMemcpyAsync(dsrc, src.data(), sizeof(ConcatSrc) * src.size(),
                          hipMemcpyHostToDevice, b->home));
  const unsigned gy = static_cast<unsigned>(std::min<int64_t>((most + kBlock - 1) / kBlock, 64));
  k_concat_tiles<<<dim3(static_cast<unsigned>(src.size()), gy), kBlock, 0, b->home>>>(
      dsrc, *out, *out_graph);
  GIFT_TRY(check_launch("k_concat_tiles"));
  // `src` must outlive the copy: wait for it before the vector goes away
  GIFT_HIP(hipStreamSynchronize(b->home));
  return GIFT_OK;
}

// The XCD-affine layout of class c: every graph goes to one XCD (largest
// graphs first, each to the XCD with the least work so far), so the signal
// rows a graph's tiles gather stay in that XCD's L2 while they run.  List
// position i * 8 + k holds the i-th tile of XCD k (block b runs on XCD
// b mod 8); shorter XCD lists are padded with empty tiles.  Built for the
// all-rows list and for the cell-rows list of the last pass.
gift_status affine_lists(gift_batch *b, int c) {
  const size_t ng = b->graphs.size();
  std::vector<int64_t> wgt(ng);
  std::vector<size_t> order(ng);
  int32_t pad_graph = -1;
  for (size_t g = 0; g < ng; ++g) {
    wgt[g] = b->graphs[g]->nnz + b->graphs[g]->num_rows;
    order[g] = g;
    if (pad_graph < 0 && b->graphs[g]->num_rows > 0) pad_graph = static_cast<int32_t>(g);
  }
  if (pad_graph < 0) return GIFT_OK;  // no rows at all: no launches
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return wgt[x] > wgt[y]; });
  std::vector<int64_t> load(kXcds, 0);
  std::vector<uint32_t> xcd_of(ng, 0);
  for (size_t g : order) {
    uint32_t k = 0;
    for (uint32_t j = 1; j < kXcds; ++j)
      if (load[j] < load[k]) k = j;
    xcd_of[g] = k;
    load[k] += wgt[g];
  }
  for (int cells_only = 0; cells_only <= 1; ++cells_only) {
    std::vector<std::vector<int32_t>> lists(kXcds);
    int64_t off = 0;
    for (size_t g = 0; g < ng; ++g) {
      const int64_t n = cells_only ? b->graphs[g]->num_tiles_cells[c] : b->graphs[g]->num_tiles[c];
      for (int64_t i = 0; i < n; ++i) lists[xcd_of[g]].push_back(static_cast<int32_t>(off + i));
      off += n;
    }
    size_t longest = 0;
    for (const auto &l : lists) longest = std::max(longest, l.size());
    const int64_t nout = static_cast<int64_t>(longest) * kXcds;
    if (nout >= (int64_t(1) << 31) - 1)
      return set_error(GIFT_EUNSUPPORTED, "batch has too many tiles for the XCD-affine layout");
    std::vector<int32_t> perm(static_cast<size_t>(nout), -1);
    for (uint32_t k = 0; k < kXcds; ++k)
      for (size_t i = 0; i < lists[k].size(); ++i) perm[i * kXcds + k] = lists[k][i];
    TileDesc **out = cells_only ? &b->aftiles[c] : &b->atiles[c];
    int32_t **out_graph = cells_only ? &b->aftile_graph[c] : &b->atile_graph[c];
    GIFT_TRY(dev_alloc(reinterpret_cast<void **>(out), sizeof(TileDesc) * (nout + 1), b->home,
                       "batch XCD-affine tiles"));
    GIFT_TRY(dev_alloc(reinterpret_cast<void **>(out_graph), sizeof(int32_t) * (nout + 1),
                       b->home, "batch XCD-affine tile graphs"));
    (cells_only ? b->num_aftiles[c] : b->num_atiles[c]) = nout;
    if (nout == 0) continue;
    Scratch sc(b->home);
    int32_t *dperm = nullptr;
    GIFT_TRY(sc.get(&dperm, perm.size(), "tile permutation"));
    GIFT_HIP(hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * perm.size(),
                            hipMemcpyHostToDevice, b->home));
    k_permute_tiles<<<grid_for(nout), kBlock, 0, b->home>>>(
        dperm, nout, cells_only ? b->ftiles[c] : b->tiles[c],
        cells_only ? b->ftile_graph[c] : b->tile_graph[c], pad_graph, *out, *out_graph);
    GIFT_TRY(check_launch("k_permute_tiles"));
    // `perm` must outlive the copy
    GIFT_HIP(hipStreamSynchronize(b->home));
  }
  return GIFT_OK;
}

void use_schedule(gift_batch *b, const Candidate &cand) {
  FilterPlan &pl = b->plan;
  const int c = cand.tile_class;
  pl.tile_class = c;
  pl.identity_map = cand.affine != 0;
  if (cand.affine) {
    pl.tiles = b->atiles[c];
    pl.tile_graph = b->atile_graph[c];
    pl.num_tiles = b->num_atiles[c];
    pl.final_tiles = b->aftiles[c];
    pl.final_tile_graph = b->aftile_graph[c];
    pl.num_final_tiles = b->num_aftiles[c];
    pl.centre_tiles = b->tiles[c];
    pl.centre_tile_graph = b->tile_graph[c];
    pl.num_centre_tiles = b->num_tiles[c];
  } else {
    pl.tiles = b->tiles[c];
    pl.tile_graph = b->tile_graph[c];
    pl.num_tiles = b->num_tiles[c];
    pl.final_tiles = b->ftiles[c];
    pl.final_tile_graph = b->ftile_graph[c];
    pl.num_final_tiles = b->num_ftiles[c];
    pl.centre_tiles = nullptr;
    pl.centre_tile_graph = nullptr;
    pl.num_centre_tiles = 0;
  }
  b->chunks = chunk_list(b->num_cols, cand.chunk);
  // each graph's tiles in the all-rows list of this class (the table is
  // uploaded with the next run)
  const size_t ng = b->graphs.size();
  int64_t t = 0;
  for (size_t g = 0; g < ng; ++g) {
    const int64_t n = b->graphs[g]->num_tiles[c];
    for (size_t k = 0; k < b->table.size() / ng; ++k) {
      b->table[k * ng + g].tile_lo = static_cast<int32_t>(t);
      b->table[k * ng + g].tile_hi = static_cast<int32_t>(t + n);
    }
    t += n;
  }
}

// Buffers for the widest chunk of any schedule: the centring partial sums
// grow with the tile count, so size them for the class with the most tiles.
size_t buffers_for(const gift_batch *b, int widest) {
  FilterPlan pl = b->plan;
  pl.centre_tiles = nullptr;
  pl.num_tiles = std::max(b->num_tiles[0], b->num_tiles[1]);
  return chunk_buffer_bytes(pl, chunk_width(std::min(widest, b->num_cols)));
}

// Enqueues the whole filter (every column chunk) of the current schedule.
gift_status enqueue_all(gift_batch *b, hipStream_t st) {
  int32_t col0 = 0;
  for (int C : b->chunks) {
    ChunkBuffers bf;
    carve_chunk_buffers(b->plan, C, b->buffers, &bf);
    GIFT_TRY(enqueue_filter_chunk(b->plan, bf, C, col0, st));
    col0 += C;
  }
  return GIFT_OK;
}

// Captures the current schedule into b->graph / b->exec (replacing them).
gift_status capture(gift_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  GIFT_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  gift_status s = enqueue_all(b, b->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture, &g);
  if (s != GIFT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess)
    return set_error(GIFT_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  b->graph = g;
  GIFT_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return GIFT_OK;
}

// Uploads the graph table with the given I/O through a pinned staging slot.
gift_status upload_table(gift_batch *b, const gift_batch_io *io, hipStream_t st) {
  const int s = b->slot;
  b->slot = (b->slot + 1) % kSlots;
  GIFT_HIP(hipEventSynchronize(b->slot_done[s]));
  GraphDev *h = b->staging[s];
  const size_t ng = b->graphs.size();
  for (size_t i = 0; i < b->table.size(); ++i) {
    h[i] = b->table[i];
    const gift_batch_io &o = io[i % ng];
    h[i].io.x_in = o.x_in;
    h[i].io.ld_in = o.ld_in;
    h[i].io.y_out = o.y_out;
    h[i].io.ld_out = o.ld_out;
    h[i].io.fixed = o.fixed_mask;
  }
  GIFT_HIP(hipMemcpyAsync(b->table_dev, h, sizeof(GraphDev) * b->table.size(),
                          hipMemcpyHostToDevice, st));
  GIFT_HIP(hipEventRecord(b->slot_done[s], st));
  return GIFT_OK;
}

// Times `reps` replays of the captured graph (milliseconds per replay).
gift_status time_replays(gift_batch *b, int reps, double *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GIFT_HIP(hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(GIFT_EDEVICE, "hipEventCreate: %s", hipGetErrorString(er));
  }
  hipError_t e = hipGraphLaunch(b->exec, b->home);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, b->home);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, b->home);
  if (e == hipSuccess) e = hipEventRecord(e1, b->home);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_error(GIFT_EDEVICE, "timing replays: %s", hipGetErrorString(e));
  *ms = static_cast<double>(t) / reps;
  return GIFT_OK;
}

gift_status alloc_buffers(gift_batch *b, size_t bytes) {
  dev_free(b->buffers, b->home);
  b->buffers = nullptr;
  b->buffer_bytes = 0;
  GIFT_TRY(dev_alloc(reinterpret_cast<void **>(&b->buffers), bytes, b->home,
                     "batch signal buffers"));
  b->buffer_bytes = bytes;
  return GIFT_OK;
}

// Times every candidate on scratch inputs (zeros) and returns the fastest.
gift_status autotune(gift_batch *b, Candidate *best) {
  std::vector<Candidate> cands;
  const int w0 = chunk_width(b->num_cols);
  for (int a = 0; a <= 1; ++a)
    for (int c = 0; c < kTileClasses; ++c)
      for (int w = w0; w >= 1 && w * 2 >= w0; w /= 2) cands.push_back(Candidate{c, w, a});
  if (cands.size() > GIFT_BATCH_MAX_CANDIDATES) cands.resize(GIFT_BATCH_MAX_CANDIDATES);

  const size_t ng = b->graphs.size();
  const size_t ein = b->in_dtype == GIFT_F64 ? 8 : 4, eout = b->out_dtype == GIFT_F64 ? 8 : 4;
  Scratch sc(b->home);
  unsigned char *xin = nullptr, *yout = nullptr;
  GIFT_TRY(sc.get(&xin, ein * b->num_cols * static_cast<size_t>(b->cells), "tuning input"));
  GIFT_TRY(sc.get(&yout, eout * b->num_cols * static_cast<size_t>(b->cells), "tuning output"));
  GIFT_HIP(hipMemsetAsync(xin, 0, ein * b->num_cols * static_cast<size_t>(b->cells), b->home));
  std::vector<gift_batch_io> io(ng);
  int64_t off = 0;
  for (size_t g = 0; g < ng; ++g) {
    io[g] = gift_batch_io{xin + ein * b->num_cols * off, b->num_cols,
                          yout + eout * b->num_cols * off, b->num_cols, nullptr};
    off += b->graphs[g]->num_cells;
  }
  GIFT_TRY(upload_table(b, io.data(), b->home));
  GIFT_TRY(alloc_buffers(b, buffers_for(b, w0)));
  double best_ms = 0;
  b->info.num_candidates = static_cast<int32_t>(cands.size());
  for (size_t i = 0; i < cands.size(); ++i) {
    use_schedule(b, cands[i]);
    GIFT_TRY(upload_table(b, io.data(), b->home));
    GIFT_TRY(capture(b));
    double ms = 0;
    GIFT_TRY(time_replays(b, 3, &ms));
    b->info.cand_tile_class[i] = cands[i].tile_class;
    b->info.cand_chunk_cols[i] = cands[i].chunk;
    b->info.cand_xcd_affine[i] = cands[i].affine;
    b->info.cand_ms[i] = ms;
    if (i == 0 || ms < best_ms) {
      best_ms = ms;
      *best = cands[i];
    }
  }
  b->info.tuned_ms = best_ms;
  return GIFT_OK;
}

}  // namespace

PinnedRing::~PinnedRing() {
  for (int i = 0; i < kSlots; ++i) {
    if (ev_[i]) {
      (void)hipEventSynchronize(ev_[i]);
      (void)hipEventDestroy(ev_[i]);
    }
    if (buf_[i]) (void)hipHostFree(buf_[i]);
  }
}

gift_status PinnedRing::acquire(size_t bytes, void **p) {
  const int s = next_;
  next_ = (next_ + 1) % kSlots;
  if (!ev_[s]) GIFT_HIP(hipEventCreateWithFlags(&ev_[s], hipEventDisableTiming));
  GIFT_HIP(hipEventSynchronize(ev_[s]));
  if (cap_[s] < bytes) {
    if (buf_[s]) (void)hipHostFree(buf_[s]);
    buf_[s] = nullptr;
    cap_[s] = 0;
    const size_t want = bytes < 65536 ? 65536 : bytes * 2;
    GIFT_HIP(hipHostMalloc(&buf_[s], want));
    cap_[s] = want;
  }
  cur_ = s;
  *p = buf_[s];
  return GIFT_OK;
}

gift_status PinnedRing::release(hipStream_t st) {
  if (cur_ < 0) return GIFT_OK;
  GIFT_HIP(hipEventRecord(ev_[cur_], st));
  cur_ = -1;
  return GIFT_OK;
}

size_t dynamic_batch_bytes(const gift_graph *const *graphs, int32_t n, int32_t storage,
                           int32_t num_terms, int32_t num_cols) {
  FilterPlan pl;
  pl.storage = storage;
  int64_t tiles = 0;
  for (int32_t g = 0; g < n; ++g) {
    pl.R += graphs[g]->num_rows;
    tiles += graphs[g]->num_tiles[0] + graphs[g]->num_tiles_cells[0];
  }
  // every term but one may keep a saved iterate
  const size_t rb = dtype_size(storage) * static_cast<size_t>(chunk_width(num_cols)) *
                    static_cast<size_t>(pl.R);
  // centring partial sums and multipliers (16-bit storage)
  const size_t C = static_cast<size_t>(chunk_width(num_cols));
  const size_t centre =
      centred_storage(storage)
          ? sizeof(double) * ((static_cast<size_t>(tiles) + 1) * (C + num_terms) +
                              static_cast<size_t>(n) * num_terms * C) + 512
          : 0;
  return (3 + static_cast<size_t>(num_terms)) * (rb + 256) +
         static_cast<size_t>(tiles) * (sizeof(TileDesc) + 4) +
         static_cast<size_t>(n) * (kMaxTerms * sizeof(GraphDev) + 2 * sizeof(ConcatSrc)) + 4096 +
         centre;
}

gift_status enqueue_dynamic_batch(const gift_graph *const *graphs, const GraphIO *ios, int32_t n,
                                  const gift_term *terms, int32_t nt, int32_t num_cols,
                                  int32_t in_dt, int32_t out_dt, hipStream_t st,
                                  PinnedRing &ring) {
  if (n < 1) return GIFT_OK;
  std::vector<std::vector<PlanGroup>> per(n);
  for (int32_t g = 0; g < n; ++g) GIFT_TRY(plan_groups(graphs[g], terms, nt, &per[g]));
  const size_t ngr = per[0].size();
  constexpr int c = 0;
  std::vector<GraphDev> table(ngr * n);
  std::vector<ConcatSrc> sa, sf;
  FilterPlan pl;
  pl.storage = graphs[0]->storage;
  int64_t most_a = 0, most_f = 0;
  for (int32_t g = 0; g < n; ++g) {
    const gift_graph *gr = graphs[g];
    if (gr->storage != pl.storage)
      return set_error(GIFT_EINVAL, "graph %d: storage differs from graph 0", g);
    GraphIO io = ios[g];
    io.num_cells = gr->num_cells;
    const int32_t tlo = static_cast<int32_t>(pl.num_tiles);
    const int32_t thi = static_cast<int32_t>(pl.num_tiles + gr->num_tiles[c]);
    for (size_t k = 0; k < ngr; ++k)
      table[k * n + g] = GraphDev{gr->row_ptr, gr->col, per[g][k].val, per[g][k].diag, pl.R, io,
                                  gr->deg, tlo, thi};
    if (gr->num_tiles[c] > 0) {
      sa.push_back(ConcatSrc{gr->tiles[c], gr->num_tiles[c], pl.num_tiles, g});
      pl.num_tiles += gr->num_tiles[c];
      most_a = std::max(most_a, gr->num_tiles[c]);
    }
    if (gr->num_tiles_cells[c] > 0) {
      sf.push_back(ConcatSrc{gr->tiles[c], gr->num_tiles_cells[c], pl.num_final_tiles, g});
      pl.num_final_tiles += gr->num_tiles_cells[c];
      most_f = std::max(most_f, gr->num_tiles_cells[c]);
    }
    pl.R += gr->num_rows;
    pl.nnz += gr->nnz;
    pl.cell_rows += gr->num_cells;
    pl.nnz_cells += gr->nnz_cells;
  }
  if (pl.num_tiles == 0) return GIFT_OK;
  if (pl.num_tiles >= (int64_t(1) << 31) - 1)
    return set_error(GIFT_EUNSUPPORTED, "batch has %lld tiles (limit 2^31 - 1)",
                     static_cast<long long>(pl.num_tiles));

  const size_t tb = sizeof(GraphDev) * table.size();
  const size_t ab = sizeof(ConcatSrc) * sa.size(), fb = sizeof(ConcatSrc) * sf.size();
  void *h = nullptr;
  GIFT_TRY(ring.acquire(tb + ab + fb, &h));
  unsigned char *hb = static_cast<unsigned char *>(h);
  std::memcpy(hb, table.data(), tb);
  std::memcpy(hb + tb, sa.data(), ab);
  if (fb) std::memcpy(hb + tb + ab, sf.data(), fb);
  Scratch sc(st);
  unsigned char *up = nullptr;
  GIFT_TRY(sc.get(&up, tb + ab + fb, "batch table"));
  GIFT_HIP(hipMemcpyAsync(up, hb, tb + ab + fb, hipMemcpyHostToDevice, st));
  GIFT_TRY(ring.release(st));
  const GraphDev *dtable = reinterpret_cast<const GraphDev *>(up);
  TileDesc *ta = nullptr, *tf = nullptr;
  int32_t *ga = nullptr, *gf = nullptr;
  GIFT_TRY(sc.get(&ta, pl.num_tiles, "batch tiles"));
  GIFT_TRY(sc.get(&ga, pl.num_tiles, "batch tile graphs"));
  GIFT_TRY(sc.get(&tf, pl.num_final_tiles + 1, "batch final tiles"));
  GIFT_TRY(sc.get(&gf, pl.num_final_tiles + 1, "batch final tile graphs"));
  auto gy = [](int64_t most) {
    return static_cast<unsigned>(std::min<int64_t>((most + kBlock - 1) / kBlock, 64));
  };
  const dim3 grid_a(static_cast<unsigned>(sa.size()), gy(most_a));
  k_concat_tiles<<<grid_a, kBlock, 0, st>>>(reinterpret_cast<const ConcatSrc *>(up + tb), ta, ga);
  GIFT_TRY(check_launch("k_concat_tiles"));
  if (!sf.empty()) {
    const dim3 grid_f(static_cast<unsigned>(sf.size()), gy(most_f));
    k_concat_tiles<<<grid_f, kBlock, 0, st>>>(reinterpret_cast<const ConcatSrc *>(up + tb + ab),
                                              tf, gf);
    GIFT_TRY(check_launch("k_concat_tiles"));
  }

  pl.tile_class = c;
  pl.tiles = ta;
  pl.tile_graph = ga;
  pl.final_tiles = tf;
  pl.final_tile_graph = gf;
  pl.centre = centred_storage(pl.storage);
  pl.num_graphs = n;
  pl.groups = per[0];
  for (size_t k = 0; k < ngr; ++k) pl.groups[k].graphs = dtable + k * n;
  pl.terms = terms;
  pl.num_terms = nt;
  pl.in_dtype = in_dt;
  pl.out_dtype = out_dt;
  pl.profile = false;
  const int widest = chunk_width(num_cols);
  unsigned char *buf = nullptr;
  GIFT_TRY(sc.get(&buf, chunk_buffer_bytes(pl, widest), "batch signal buffers"));
  for (int32_t col0 = 0; col0 < num_cols;) {
    const int C = chunk_width(num_cols - col0);
    ChunkBuffers bf;
    carve_chunk_buffers(pl, C, buf, &bf);
    GIFT_TRY(enqueue_filter_chunk(pl, bf, C, col0, st));
    col0 += C;
  }
  return GIFT_OK;
}

}  // namespace gift

extern "C" gift_status gift_batch_create(const gift_graph *const *graphs, int32_t num_graphs,
                                         const gift_term *terms, int32_t num_terms,
                                         int32_t num_cols, int32_t in_dtype, int32_t out_dtype,
                                         int32_t tune, void *stream, gift_batch **out) {
  clear_error();
  if (!out) return set_error(GIFT_EINVAL, "gift_batch_create: out is NULL");
  *out = nullptr;
  if (!graphs || !terms) return set_error(GIFT_EINVAL, "gift_batch_create: NULL graphs or terms");
  if (num_graphs < 1) return set_error(GIFT_EINVAL, "num_graphs %d < 1", num_graphs);
  if (num_terms < 1 || num_terms > kMaxTerms)
    return set_error(GIFT_EINVAL, "num_terms %d not in [1, 64]", num_terms);
  if (num_cols < 1) return set_error(GIFT_EINVAL, "num_cols %d < 1", num_cols);
  if (in_dtype != GIFT_F32 && in_dtype != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "in_dtype must be F32 or F64");
  if (out_dtype != GIFT_F32 && out_dtype != GIFT_F64)
    return set_error(GIFT_EUNSUPPORTED, "out_dtype must be F32 or F64");
  if (tune < 0 || tune > 3) return set_error(GIFT_EINVAL, "tune %d not in [0, 3]", tune);
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (!graphs[g]) return set_error(GIFT_EINVAL, "graph %d is NULL", g);
    if (graphs[g]->storage != graphs[0]->storage)
      return set_error(GIFT_EINVAL, "graph %d: storage differs from graph 0", g);
    if (graphs[g]->device != dev)
      return set_error(GIFT_EINVAL, "graph %d lives on device %d, current device is %d", g,
                       graphs[g]->device, dev);
  }

  gift_batch *b = new (std::nothrow) gift_batch();
  if (!b) return set_error(GIFT_ENOMEM, "gift_batch_create: host allocation");
  b->device = dev;
  b->home = static_cast<hipStream_t>(stream);
  b->graphs.assign(graphs, graphs + num_graphs);
  b->terms.assign(terms, terms + num_terms);
  b->num_cols = num_cols;
  b->in_dtype = in_dtype;
  b->out_dtype = out_dtype;
  b->storage = graphs[0]->storage;
  auto fail = [&](gift_status s) {
    std::string msg = gift_last_error();
    free_batch(b);
    set_error(s, "%s", msg.c_str());
    return s;
  };

  // groups (sigma, k_max) and every graph's values for them
  std::vector<std::vector<PlanGroup>> per(num_graphs);
  for (int32_t g = 0; g < num_graphs; ++g) {
    gift_status s = plan_groups(graphs[g], b->terms.data(), num_terms, &per[g]);
    if (s != GIFT_OK) return fail(s);
  }
  const size_t ngr = per[0].size();
  int64_t row_off = 0;
  b->table.resize(ngr * num_graphs);
  for (int32_t g = 0; g < num_graphs; ++g) {
    const gift_graph *gr = graphs[g];
    for (size_t k = 0; k < ngr; ++k)
      b->table[k * num_graphs + g] =
          GraphDev{gr->row_ptr, gr->col, per[g][k].val, per[g][k].diag, row_off,
                   GraphIO{nullptr, num_cols, nullptr, num_cols, nullptr, gr->num_cells},
                   gr->deg, 0, 0};
    row_off += gr->num_rows;
    b->nnz += gr->nnz;
    b->cells += gr->num_cells;
    b->nnz_cells += gr->nnz_cells;
  }
  b->R = row_off;

  if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
    b->capture = nullptr;
    set_error(GIFT_EDEVICE, "hipStreamCreateWithFlags failed");
    return fail(GIFT_EDEVICE);
  }
  for (int s = 0; s < kSlots; ++s) {
    if (hipHostMalloc(reinterpret_cast<void **>(&b->staging[s]),
                      sizeof(GraphDev) * b->table.size()) != hipSuccess) {
      b->staging[s] = nullptr;
      set_error(GIFT_ENOMEM, "hipHostMalloc of the I/O staging table failed");
      return fail(GIFT_ENOMEM);
    }
    if (hipEventCreateWithFlags(&b->slot_done[s], hipEventDisableTiming) != hipSuccess) {
      b->slot_done[s] = nullptr;
      set_error(GIFT_EDEVICE, "hipEventCreate failed");
      return fail(GIFT_EDEVICE);
    }
  }
  if (hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming) != hipSuccess) {
    b->last_run = nullptr;
    set_error(GIFT_EDEVICE, "hipEventCreate failed");
    return fail(GIFT_EDEVICE);
  }
  gift_status s = dev_alloc(reinterpret_cast<void **>(&b->table_dev),
                            sizeof(GraphDev) * b->table.size(), b->home, "batch graph table");
  if (s != GIFT_OK) return fail(s);
  for (int c = 0; c < kTileClasses; ++c) {
    s = concat_tiles(b, c, false, &b->tiles[c], &b->tile_graph[c], &b->num_tiles[c]);
    if (s == GIFT_OK)
      s = concat_tiles(b, c, true, &b->ftiles[c], &b->ftile_graph[c], &b->num_ftiles[c]);
    if (s == GIFT_OK) s = affine_lists(b, c);
    if (s != GIFT_OK) return fail(s);
  }

  FilterPlan &pl = b->plan;
  pl.storage = b->storage;
  pl.centre = centred_storage(b->storage);
  pl.num_graphs = num_graphs;
  pl.R = b->R;
  pl.nnz = b->nnz;
  pl.cell_rows = b->cells;
  pl.nnz_cells = b->nnz_cells;
  pl.groups = per[0];
  for (size_t k = 0; k < ngr; ++k) pl.groups[k].graphs = b->table_dev + k * num_graphs;
  pl.terms = b->terms.data();
  pl.num_terms = num_terms;
  pl.in_dtype = in_dtype;
  pl.out_dtype = out_dtype;
  pl.profile = false;

  // schedule: default, cached or tuned
  Candidate best{0, chunk_width(num_cols), tune == 3 ? 1 : 0};
  const TuneKey key{dev, b->storage, num_cols, num_terms, log2_bucket(b->nnz),
                    log2_bucket(b->R), log2_bucket(num_graphs)};
  b->info.tuned = 0;
  if (tune == 1) {
    std::lock_guard<std::mutex> lk(tune_cache().m);
    auto it = tune_cache().best.find(key);
    if (it != tune_cache().best.end()) {
      best = it->second;
      b->info.tuned = 2;
    }
  }
  if (tune == 2 || (tune == 1 && b->info.tuned == 0)) {
    if (b->cells > 0) {
      s = autotune(b, &best);
      if (s != GIFT_OK) return fail(s);
    }
    b->info.tuned = 1;
    std::lock_guard<std::mutex> lk(tune_cache().m);
    tune_cache().best[key] = best;
  }
  use_schedule(b, best);
  s = alloc_buffers(b, buffers_for(b, best.chunk));
  if (s == GIFT_OK) s = capture(b);
  if (s != GIFT_OK) return fail(s);

  // the staging copies above read pageable host vectors: finish them here
  if (hipStreamSynchronize(b->home) != hipSuccess) {
    set_error(GIFT_EDEVICE, "hipStreamSynchronize failed");
    return fail(GIFT_EDEVICE);
  }
  gift_batch_info &in = b->info;
  in.num_graphs = num_graphs;
  in.tile_class = best.tile_class;
  in.chunk_cols = best.chunk;
  in.xcd_affine = best.affine;
  in.num_rows = b->R;
  in.nnz = b->nnz;
  in.num_tiles = b->num_tiles[best.tile_class];
  in.device_bytes = static_cast<int64_t>(b->buffer_bytes + sizeof(GraphDev) * b->table.size());
  for (int c = 0; c < kTileClasses; ++c)
    in.device_bytes += static_cast<int64_t>(
        (sizeof(TileDesc) + 4) *
        (b->num_tiles[c] + b->num_ftiles[c] + b->num_atiles[c] + b->num_aftiles[c] + 4));
  *out = b;
  return GIFT_OK;
}

extern "C" gift_status gift_batch_run(gift_batch *b, const gift_batch_io *io, void *stream) {
  clear_error();
  if (!b || !io) return set_error(GIFT_EINVAL, "gift_batch_run: NULL batch or io");
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  if (dev != b->device)
    return set_error(GIFT_EINVAL, "batch lives on device %d, current device is %d", b->device, dev);
  for (size_t g = 0; g < b->graphs.size(); ++g) {
    const gift_batch_io &o = io[g];
    if (b->graphs[g]->num_cells == 0) continue;
    if (!o.x_in || !o.y_out) return set_error(GIFT_EINVAL, "io[%zu]: NULL x_in or y_out", g);
    if (o.ld_in < b->num_cols || o.ld_out < b->num_cols)
      return set_error(GIFT_EINVAL, "io[%zu]: leading dimension smaller than num_cols", g);
  }
  if (b->cells == 0) return GIFT_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the table and the signal buffers are shared by every run: order this run
  // after the previous one, which may have been enqueued on another stream
  GIFT_HIP(hipStreamWaitEvent(st, b->last_run, 0));
  GIFT_TRY(upload_table(b, io, st));
  GIFT_HIP(hipGraphLaunch(b->exec, st));
  GIFT_HIP(hipEventRecord(b->last_run, st));
  return GIFT_OK;
}

extern "C" gift_status gift_batch_get_info(const gift_batch *b, gift_batch_info *info) {
  clear_error();
  if (!b || !info) return set_error(GIFT_EINVAL, "gift_batch_get_info: NULL argument");
  *info = b->info;
  return GIFT_OK;
}

extern "C" gift_status gift_batch_destroy(gift_batch *b) {
  clear_error();
  if (!b) return GIFT_OK;
  free_batch(b);
  return GIFT_OK;
}
