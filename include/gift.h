/*
 * gift.h -- C ABI of the GiFt graph-filter placement library (AMD MI355X,
 * gfx950).
 *
 * GiFt ("The Power of Graph Signal Processing for Chip Placement
 * Acceleration", ICCAD'24) computes an initial cell placement by low-pass
 * filtering the cells' location signal on the circuit graph:
 *
 *     g' = sum_t alpha_t  A~_{sigma_t}^{k_t}  g                (eq. proposed_filter)
 *     A~_sigma = (D + sigma I)^-1/2 (A + sigma I) (D + sigma I)^-1/2
 *                                                             (eq. A_formulation)
 *
 * where A is the weighted adjacency of the netlist under the clique net model
 * (Section 3.2, the paragraph after Algorithm 1) and D its degree matrix
 * (Section 2.1).  The library has two steps:
 *
 *   gift_build_graph       netlist -> resident normalised graph
 *   gift_filter_placement  graph + signal -> filtered signal
 *
 * plus batched filtering of many graphs in one launch sequence and a
 * request-serving engine.
 *
 * Conventions for every entry point:
 *   - Every function returns a gift_status and never aborts or throws.  On an
 *     error gift_last_error() (per host thread) describes it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is ordered on it.  Functions that must read sizes back
 *     (gift_build_graph) synchronise that stream before returning; the others
 *     only enqueue work.
 *   - Caller-owned buffers stay caller-owned.  Device pointers must point to
 *     memory of the current HIP device.  Matrices are row-major with a
 *     leading dimension given in elements.
 *   - Objects created by the library (graphs, batches, servers) are owned by
 *     the caller's handle and released only by the matching destroy call.
 *   - Sizes are limited to fewer than 2^31 rows and 2^31 stored entries per
 *     graph; larger inputs return GIFT_EUNSUPPORTED.
 */
#ifndef GIFT_H
#define GIFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GIFT_ABI_VERSION 3

typedef enum {
  GIFT_OK = 0,
  GIFT_EINVAL = 1,       /* bad argument, malformed netlist, unknown sigma   */
  GIFT_ENOMEM = 2,       /* a device or host allocation failed               */
  GIFT_EDEVICE = 3,      /* a HIP runtime call failed (message kept)         */
  GIFT_EUNSUPPORTED = 4, /* valid but unsupported combination or size       */
  GIFT_EBUSY = 5         /* object in use (e.g. server still has work)       */
} gift_status;

/* Element types of stored values and of signals. */
typedef enum {
  GIFT_F32 = 0,
  GIFT_F64 = 1,
  GIFT_BF16 = 2, /* bfloat16, round-to-nearest-even when stored            */
  GIFT_F16 = 3   /* IEEE half, round-to-nearest-even when stored           */
} gift_dtype;

/* Weight a net of M distinct cells adds to each pair of its cells. */
typedef enum {
  GIFT_W_INV_M1 = 0,    /* 1/(M-1): every cell of a clique gets degree 1     */
  GIFT_W_TWO_OVER_M = 1 /* 2/M: the net weight of Section 2.2 (eq. wire_eq)  */
} gift_weight_model;

typedef enum { GIFT_MEM_HOST = 0, GIFT_MEM_DEVICE = 1 } gift_mem_space;

typedef struct gift_graph gift_graph;

/*
 * Netlist and graph options for gift_build_graph.
 *
 *   num_cells       N >= 0 cells (movable and fixed), rows 0..N-1 of every
 *                   signal.
 *   num_nets        E >= 0 nets.
 *   net_ptr         int64[E+1], net_ptr[0] = 0, non-decreasing: the pins of
 *                   net e are pin_cell[net_ptr[e] .. net_ptr[e+1]).
 *   pin_cell        int32[net_ptr[E]], each in [0, N).
 *   mem_space       where net_ptr and pin_cell live (GIFT_MEM_HOST or
 *                   GIFT_MEM_DEVICE).  They are read during the call only.
 *   weight_model    gift_weight_model.
 *   star_threshold  T >= 0.  A net with more than T distinct cells (T > 0) is
 *                   expanded as a star: one virtual node joined to each of its
 *                   cells with weight M*w(M) (the Laplacian of the star with
 *                   the virtual node eliminated is exactly the clique's).
 *                   T = 0 expands every net as a clique.  Virtual nodes are
 *                   rows N..N+V-1 in ascending order of their net's median
 *                   cell (the distinct cell at index M/2 of the net's
 *                   ascending list), ties in ascending net id, so that
 *                   neighbouring virtual rows join neighbouring cells; they
 *                   are internal and never appear in a signal handed to or
 *                   returned by the library.
 *   storage         gift_dtype of the normalised off-diagonal values and of
 *                   the filter's internal signal iterates.  F32, BF16 and F16
 *                   accumulate in float32; F64 accumulates in float64.
 *   num_sigmas      number of self-loop weights to prepare (>= 1).
 *   sigmas          host double[num_sigmas], each >= 0: the sigma values the
 *                   filter may use.  More can be added with
 *                   gift_graph_add_sigma.
 *   num_pins        the number of entries of pin_cell, or -1.  The pin count
 *                   is net_ptr[num_nets]; when num_pins >= 0 the call fails
 *                   with GIFT_EINVAL unless the two agree, before anything
 *                   reads a pin.  For a device netlist the library reads
 *                   net_ptr[num_nets] back itself, so the caller need not
 *                   (and need not wait for the stream to do so).  -1: the
 *                   caller vouches that pin_cell holds net_ptr[num_nets]
 *                   entries.
 *
 * Netlist semantics: repeated pins of one net count once; a net with fewer
 * than two distinct cells adds nothing; weights of different nets on the same
 * pair add up.  The degree d_i = sum_j w_ij excludes the self-loop.
 */
typedef struct {
  int64_t num_cells;
  int64_t num_nets;
  const int64_t *net_ptr;
  const int32_t *pin_cell;
  int32_t mem_space;
  int32_t weight_model;
  int64_t star_threshold;
  int32_t storage;
  int32_t num_sigmas;
  const double *sigmas;
  int64_t num_pins;
} gift_graph_desc;

/* One filter term alpha * A~_sigma^order (Section 3.2.1, eq. proposed_filter).
 * order >= 1, sigma >= 0 and prepared in the graph. */
typedef struct {
  double sigma;
  int32_t order;
  int32_t reserved; /* must be 0 */
  double alpha;
} gift_term;

typedef struct {
  int64_t num_cells;      /* N */
  int64_t num_virtual;    /* V: star nodes */
  int64_t num_rows;       /* R = N + V */
  int64_t nnz;            /* stored off-diagonal entries of A */
  int64_t bytes_resident; /* device bytes held by the graph */
  int32_t storage;        /* gift_dtype */
  int32_t num_sigmas;     /* prepared self-loop weights */
} gift_graph_info;

/*
 * gift_build_graph -- netlist -> resident graph (clique net model, Section
 * 3.2; degrees and Laplacian, Section 2.1; normalisation, eq. A_formulation).
 *
 * Builds the canonical CSR of A (rows ascending, columns ascending within a
 * row, parallel edges summed in ascending net id in float64, no diagonal),
 * the float64 degrees (summed in ascending column), and for every sigma the
 * normalised values a_ij = (w_ij s_i) s_j and diagonal (sigma s_i) s_i with
 * s_i = 1/sqrt(d_i + sigma) (s_i = 0 when d_i + sigma = 0), rounded once to
 * the storage type.  The structure, weights and degrees are deterministic.
 * The call synchronises `stream` while it reads sizes back and returns with
 * the last kernels (merge, normalisation) still enqueued on `stream`: work on
 * `stream` may use the graph at once; work on another stream must first wait
 * for `stream` (synchronise it, or wait on an event recorded on it).
 * Errors: GIFT_EINVAL for a malformed netlist (pin out of
 * range, net_ptr not starting at 0 or decreasing), negative sizes, sigma < 0,
 * num_sigmas < 1 or bad enums; GIFT_ENOMEM; GIFT_EDEVICE.  On error *out is
 * NULL and nothing is leaked.
 */
gift_status gift_build_graph(const gift_graph_desc *desc, void *stream, gift_graph **out);

/*
 * A caller-supplied weighted graph for gift_graph_import_csr: the undirected
 * weighted graph that Section 2.1 defines (A = {w_ij}, D = diag(sum_j w_ij))
 * and that Algorithm 1 takes as its input, as a canonical CSR.
 *
 *   num_rows   R >= 0 nodes.  Every node is a cell: row i of A is row i of
 *              every signal (there are no star rows).
 *   nnz        stored entries (off-diagonal weights), < 2^31 - 1.
 *   row_ptr    int64[R+1]: row_ptr[0] = 0, non-decreasing, row_ptr[R] = nnz.
 *   col        int32[nnz]: the columns of row i are col[row_ptr[i] ..
 *              row_ptr[i+1]), strictly ascending, in [0, R) and never i (the
 *              self-loop is sigma, added by eq. A_formulation).
 *   w          double[nnz]: w_ij, finite and >= 0.
 *   mem_space  where the three arrays live (GIFT_MEM_HOST or
 *              GIFT_MEM_DEVICE); they are read during the call only.
 *   storage, num_sigmas, sigmas   as in gift_graph_desc.
 *
 * The graph is used as given: symmetry w_ij = w_ji is the caller's (the
 * method assumes an undirected graph; the definitions below do not need it).
 */
typedef struct {
  int64_t num_rows;
  int64_t nnz;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *w;
  int32_t mem_space;
  int32_t storage;
  int32_t num_sigmas;
  int32_t reserved; /* must be 0 */
  const double *sigmas;
} gift_csr_desc;

/*
 * gift_graph_import_csr -- caller-supplied weighted graph -> resident graph
 * (Section 2.1; Algorithm 1, input; normalisation, eq. A_formulation).
 *
 * The result is what gift_build_graph produces from a netlist: the CSR of A
 * (copied), float64 degrees d_i = sum_j w_ij summed in ascending column, the
 * SpMM row tiles, and for every sigma the normalised values
 * a_ij = (w_ij s_i) s_j and diagonal (sigma s_i) s_i with s_i = 1/sqrt(d_i +
 * sigma) (0 when d_i + sigma = 0), rounded once to the storage type.  Every
 * other entry point takes the graph like a built one (gift_evaluate_placement
 * reports hpwl only when given a netlist).  The CSR is checked on the device;
 * the call synchronises `stream` to read the result of the check and returns
 * with the normalisation still enqueued on `stream`, as gift_build_graph does.
 * Errors: GIFT_EINVAL (NULL pointers, negative sizes, a malformed CSR as
 * described above, bad enums or sigmas), GIFT_EUNSUPPORTED (2^31 - 1 rows or
 * entries or more), GIFT_ENOMEM, GIFT_EDEVICE.  On error *out is NULL and
 * nothing is leaked.
 */
gift_status gift_graph_import_csr(const gift_csr_desc *desc, void *stream, gift_graph **out);

/*
 * gift_filter_placement -- g' = sum_t alpha_t A~_{sigma_t}^{k_t} g
 * (eq. proposed_filter; Section 3.2.2 for the role of the result).
 *
 *   terms, num_terms  host array of filter terms, num_terms in [1, 64].
 *   x_in              device, N x num_cols, leading dimension ld_in >=
 *                     num_cols, element type in_dtype (F32 or F64).
 *   y_out             device, N x num_cols, ld_out >= num_cols, out_dtype
 *                     (F32 or F64).  Must not overlap x_in.
 *   fixed_mask        device uint8[N] or NULL.  Rows with a non-zero mask are
 *                     copied from x_in to y_out (fixed cells keep their
 *                     position, Section 4.1); NULL returns the raw filter for
 *                     every row.
 *
 * Powers are formed by repeated sparse products per distinct sigma; virtual
 * rows start at the mean of their net's cells.  The terms are combined in
 * float64 in the given order and rounded once to out_dtype.  Asynchronous on
 * `stream`; device scratch comes from the library's stream-ordered cache
 * (see gift_memory_stats).  Errors: GIFT_EINVAL (NULL pointers, sizes, order < 1, a sigma
 * not prepared), GIFT_EUNSUPPORTED (dtype), GIFT_ENOMEM, GIFT_EDEVICE.
 */
gift_status gift_filter_placement(const gift_graph *graph, const gift_term *terms,
                                  int32_t num_terms, const void *x_in, int32_t num_cols,
                                  int64_t ld_in, int32_t in_dtype, void *y_out,
                                  int64_t ld_out, int32_t out_dtype,
                                  const uint8_t *fixed_mask, void *stream);

/*
 * gift_filter_placement_noalloc -- gift_filter_placement for callers that
 * cannot allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, the same
 * kernels and so bit-identical results; it calls no hipMalloc, hipFree or
 * other allocating routine.  Its signal buffers (x0, two ping-pong iterates
 * and one saved iterate per distinct stored term, each R x the widest column
 * chunk of 16, 8, 4, 2 or 1 columns in the storage type, rounded to 256
 * bytes) live in a static 128 MiB device array that each GPU the library runs
 * on holds until the process ends; inputs needing more fail with
 * GIFT_EUNSUPPORTED and a message giving the size.  (F32, 2 columns and the
 * five orders 1, 2, 4, 8, 16: 7 buffers of 8 bytes per row, up to about 2.3M
 * rows.)  Every call on a GPU shares that GPU's array, so calls that overlap
 * on one GPU (different streams or host threads without ordering) race and
 * must be serialised by the caller; nothing in the array needs to start at
 * zero.  Not timed by the library's profiler.  Errors as in
 * gift_filter_placement, plus GIFT_EUNSUPPORTED for the size limit.
 */
gift_status gift_filter_placement_noalloc(const gift_graph *graph, const gift_term *terms,
                                          int32_t num_terms, const void *x_in,
                                          int32_t num_cols, int64_t ld_in, int32_t in_dtype,
                                          void *y_out, int64_t ld_out, int32_t out_dtype,
                                          const uint8_t *fixed_mask, void *stream);

/*
 * gift_filter_exact -- the exact filter the paper's filter approximates
 * (Section 3.2.2: eq. incremental, eq. derivative, eq. spectral):
 *
 *     g' = (I + L~_sigma)^-1 g,   L~_sigma = I - A~_sigma,
 *
 * i.e. the solution of (2 I - A~_sigma) g' = g over all graph rows (star
 * rows start from the mean of their cells, as in the filter; only cell rows
 * are returned).  Solved per column by conjugate gradients from g' = 0 until
 * ||r|| <= tol ||g|| or max_iter iterations; each iteration is one SpMM pass
 * (the filter's kernel) and float64 dot products.  The matrix has
 * eigenvalues in [1, 3), so a few dozen iterations reach 1e-12.
 *
 *   sigma       a self-loop weight prepared in the graph.
 *   x_in, y_out, fixed_mask, dtypes: as in gift_filter_placement.
 *   tol         relative residual (> 0); max_iter >= 1.
 *   iterations  (nullable) iterations of the slowest column chunk.
 *
 * The graph must use F32 or F64 storage (GIFT_EUNSUPPORTED otherwise): the
 * iterates are kept in the storage type.  Synchronises `stream` (the host
 * checks convergence).  Errors as in gift_filter_placement.
 */
gift_status gift_filter_exact(const gift_graph *graph, double sigma, const void *x_in,
                              int32_t num_cols, int64_t ld_in, int32_t in_dtype, void *y_out,
                              int64_t ld_out, int32_t out_dtype, const uint8_t *fixed_mask,
                              double tol, int64_t max_iter, int64_t *iterations, void *stream);

/* Prepare one more self-loop weight (sigma >= 0).  No-op if already there.
 * Asynchronous on `stream`, like the tail of gift_build_graph. */
gift_status gift_graph_add_sigma(gift_graph *graph, double sigma, void *stream);

gift_status gift_graph_get_info(const gift_graph *graph, gift_graph_info *info);

/* Row-tile schedule gift_filter_placement uses for this graph: 0 (default:
 * tiles of up to 2048 entries / 512 rows, rows longer than 256 entries
 * alone) or 1 (1024 / 256, 128).  Both give results within rounding of each
 * other; the choice only changes speed (and the order of float32 sums). */
gift_status gift_graph_set_tile_class(gift_graph *graph, int32_t tile_class);

/*
 * Copy the graph to host memory (for inspection and tests).  Any pointer may
 * be NULL.  row_ptr: int64[R+1]; col: int32[nnz]; w: double[nnz] (A's
 * weights); deg: double[R].  Synchronises `stream`.
 */
gift_status gift_graph_export(const gift_graph *graph, int64_t *row_ptr, int32_t *col,
                              double *w, double *deg, void *stream);

/*
 * Copy the normalised values for one prepared sigma to host memory, widened
 * to double: val[nnz] in CSR order and diag[R].  Synchronises `stream`.
 */
gift_status gift_graph_export_normalised(const gift_graph *graph, double sigma, double *val,
                                         double *diag, void *stream);

/*
 * Release the graph.  Its device memory is returned in stream order on
 * `stream`: every use of the graph must be ordered before this point on
 * `stream` (same stream, or an event the stream waits on).
 */
gift_status gift_destroy_graph(gift_graph *graph, void *stream);

/*
 * gift_evaluate_placement -- placement metrics of a signal g (num_cols
 * columns, e.g. x and y) on a resident graph, in float64, per column:
 *
 *   smoothness[q]  S(g_q) = sum over edges w_ij (g_i - g_j)^2: the smoothness
 *                  of Section 2.1 (eq. smoothness), whose sum over the x and y
 *                  columns is the weighted quadratic wirelength of Section 2.2
 *                  (eq. wire_eq).  Star nodes count at the mean of their cells,
 *                  which gives exactly the clique model's value, so S does not
 *                  depend on the star threshold (up to rounding).
 *   norm2[q]       sum_i g_i^2.
 *   rayleigh[q]    S / norm2, the Rayleigh quotient of eq. smoothness_ray
 *                  (0 for a zero column).
 *   hpwl[q]        sum over nets of (max - min) of g over the net's pins: the
 *                  half-perimeter wirelength the paper evaluates placements
 *                  with.  Needs the netlist: net_ptr int64[num_nets + 1] and
 *                  pin_cell int32[num_pins] in device memory (offsets are
 *                  clamped to [0, num_pins); pins outside [0, N) are skipped).
 *
 *   x        device, N x num_cols (num_cols in [1, 128]), leading dimension
 *            ld, dtype F32 or F64.
 *   Any of smoothness / norm2 / rayleigh / hpwl may be NULL (host
 *   double[num_cols]);
 *   with hpwl NULL the netlist is not read.
 *
 * Sums are formed in a fixed order (deterministic).  Synchronises `stream`.
 * Errors: GIFT_EINVAL, GIFT_EUNSUPPORTED (dtype), GIFT_ENOMEM, GIFT_EDEVICE.
 */
gift_status gift_evaluate_placement(const gift_graph *graph, const void *x, int32_t num_cols,
                                    int64_t ld, int32_t dtype, const int64_t *net_ptr,
                                    const int32_t *pin_cell, int64_t num_nets, int64_t num_pins,
                                    double *smoothness, double *norm2, double *rayleigh,
                                    double *hpwl, void *stream);

/*
 * gift_eigen_placement -- the eigenvector placement that Section 3.3.1
 * analyses as the ideal low-pass filter (eq. ideal_filter): the placement
 * [u_2, u_3], the eigenvectors of the second and third smallest eigenvalues
 * of the graph Laplacian L = D - A (Section 2.1) of the clique net model.
 *
 * The graph's star nets are eliminated exactly (a star row at the mean of its
 * cells turns the star into its clique), so the result does not depend on
 * the star threshold.  Each connected component adds a zero eigenvalue, so
 * the eigenvectors are those of the largest component (most cells; ties: the
 * component with the smallest cell index) with its constant vector projected
 * out; cells outside it get 0.  Each vector has unit norm and its
 * largest-magnitude entry (first such row) positive.  Computed by
 * Chebyshev-filtered subspace iteration on a block of 4 vectors in float64
 * until both residuals ||L u - lambda u|| are at most tol * b (b = 2 max
 * degree >= lambda_max) or max_iter iterations.  The component labels are
 * found on the device (smallest row index of each component).
 *
 *   tol, max_iter  relative residual (> 0) and iteration cap (>= 1).
 *   seed           start block (a hash of seed, row and column).
 *   y_out          device float64 N x 2, leading dimension ld_out >= 2:
 *                  u_2 in column 0, u_3 in column 1.
 *   labels         device int32[num_rows] or NULL: every row's component
 *                  label (cells and star rows).
 *   result         host: eigenvalues, residuals, iterations, component.
 *
 * Synchronises `stream` (the host drives the iteration).  Errors: GIFT_EINVAL
 * (NULL pointers, bad tol / max_iter / ld_out, fewer than 6 cells in the
 * largest component), GIFT_EUNSUPPORTED (components not settled),
 * GIFT_ENOMEM, GIFT_EDEVICE.  Not converging within max_iter is not an error:
 * result->converged is 0.
 */
typedef struct {
  double lambda[2];         /* lambda_2, lambda_3 */
  double residual[2];       /* ||L u - lambda u|| of the unit eigenvectors */
  double spectral_bound;    /* b = 2 max degree, the scale of tol */
  int64_t component_label;  /* smallest cell index of the component used */
  int64_t component_cells;  /* cells in that component */
  int32_t iterations;       /* filtered subspace iterations */
  int32_t sweeps;           /* sweeps of the component labelling */
  int32_t converged;        /* 1 if both residuals <= tol * spectral_bound */
  int32_t reserved;
} gift_eigen_result;

gift_status gift_eigen_placement(const gift_graph *graph, double tol, int32_t max_iter,
                                 uint64_t seed, double *y_out, int64_t ld_out, int32_t *labels,
                                 gift_eigen_result *result, void *stream);

/*
 * gift_bin_density -- bin density of a placement (Section 2.2,
 * eq. density_eq): the region [xl, xh] x [yl, yh] is cut into nbx x nby equal
 * bins and
 *
 *     rho_b = sum_v l_x(v, b) l_y(v, b),
 *
 * the overlap area of bin b with each object's rectangle (width w_v, height
 * h_v, centred at the object's position).  Shows how much a placement (e.g.
 * the filtered one) overlaps, the over-smoothing the paper's multi-order
 * filter is designed to limit.
 *
 *   x          device, num_objects x ld (ld >= 2): columns 0 and 1 are the
 *              x and y centres, dtype F32 or F64.
 *   widths, heights   device float64[num_objects], or NULL to use w0 / h0.
 *   density    device float64[nby][nbx] (row-major, bin (i, j) at
 *              [j * nbx + i]), overwritten.
 *
 * Overlaps are summed exactly in 64-bit fixed point (2^-40 of a bin's area),
 * so the result is deterministic.  Objects with a non-finite position or a
 * size <= 0 are skipped.  Asynchronous on `stream`.  Errors: GIFT_EINVAL
 * (sizes, region, NULL buffers), GIFT_EUNSUPPORTED (dtype), GIFT_ENOMEM,
 * GIFT_EDEVICE.
 */
gift_status gift_bin_density(const void *x, int64_t num_objects, int64_t ld, int32_t dtype,
                             const double *widths, const double *heights, double w0,
                             double h0, double xl, double yl, double xh, double yh,
                             int32_t nbx, int32_t nby, double *density, void *stream);

/*
 * gift_density_overflow -- overflow of a bin-density map (the density of
 * Section 2.2, eq. density_eq, as placers track it): the area by which bins
 * exceed `target` times their own area, over the total object area,
 *
 *     sum_b max(0, rho_b - target * A_b) / total_area,
 *     A_b = ((xh - xl) / nbx) ((yh - yl) / nby).
 *
 *   density      device float64[nby][nbx] as gift_bin_density writes it.
 *   target       allowed fraction of a bin's area (finite).
 *   total_area   total object area (> 0).
 *   overflow     host double: the result.
 *
 * Summed in fixed ranges and then in range order (deterministic).
 * Synchronises `stream`.  Errors: GIFT_EINVAL (NULL buffers, grid, region,
 * total_area), GIFT_ENOMEM, GIFT_EDEVICE.
 */
gift_status gift_density_overflow(const double *density, int32_t nbx, int32_t nby, double xl,
                                  double yl, double xh, double yh, double target,
                                  double total_area, double *overflow, void *stream);

/* ------------------------------------------------------------------------
 * Batched filtering: many resident graphs (designs of any sizes) filtered
 * with the same terms and column count by one launch sequence, captured
 * once into a HIP graph and replayed.  A batch is block-diagonal: every
 * graph's result is the same as when filtered alone (the graphs share no
 * rows, and each row is computed by the same arithmetic).
 * ----------------------------------------------------------------------*/

typedef struct gift_batch gift_batch;

/* One graph's input and output for gift_batch_run (device pointers,
 * row-major N_g x num_cols, leading dimensions in elements, same meaning as
 * in gift_filter_placement). */
typedef struct {
  const void *x_in;          /* in_dtype [N_g][ld_in]                      */
  int64_t ld_in;             /* >= num_cols                                */
  void *y_out;               /* out_dtype [N_g][ld_out], not overlapping   */
  int64_t ld_out;            /* >= num_cols                                */
  const uint8_t *fixed_mask; /* uint8[N_g] or NULL                         */
} gift_batch_io;

#define GIFT_BATCH_MAX_CANDIDATES 8

/* The schedule a batch runs and how it was chosen. */
typedef struct {
  int32_t num_graphs;
  int32_t tile_class;   /* 0: row tiles of up to 2048 entries / 512 rows, rows
                           longer than 256 entries alone; 1: 1024 / 256, 128 */
  int32_t chunk_cols;   /* widest column chunk (one pass sequence per chunk)  */
  int32_t tuned;        /* 0 default, 1 timed at creation, 2 from the cache  */
  int64_t num_rows;     /* rows of all graphs (cells and star nodes)         */
  int64_t nnz;          /* stored off-diagonal entries of all graphs         */
  int64_t num_tiles;    /* tiles per SpMM pass                               */
  int64_t device_bytes; /* device memory held by the batch itself           */
  double tuned_ms;      /* replay time of the chosen schedule when timed     */
  int32_t num_candidates;
  int32_t xcd_affine;   /* 1: every graph's tiles run on one XCD (its L2 keeps the
                           graph's signal rows); 0: chunks of consecutive tiles
                           dealt round-robin to the XCDs                      */
  int32_t cand_tile_class[GIFT_BATCH_MAX_CANDIDATES];
  int32_t cand_chunk_cols[GIFT_BATCH_MAX_CANDIDATES];
  double cand_ms[GIFT_BATCH_MAX_CANDIDATES]; /* replay time of each candidate */
  int32_t cand_xcd_affine[GIFT_BATCH_MAX_CANDIDATES];
} gift_batch_info;

/*
 * gift_batch_create -- plan, tune and capture the filter of num_graphs graphs
 * (eq. proposed_filter applied to each graph's own signal).
 *
 *   graphs      host array of num_graphs >= 1 graphs on the current device,
 *               all with the same storage type and with every sigma of
 *               `terms` prepared.  The batch reads their device memory at
 *               every run: they must outlive it and must not change.
 *   terms       as in gift_filter_placement (copied).
 *   num_cols    columns of every graph's signal (>= 1).
 *   in_dtype, out_dtype   F32 or F64.
 *   tune        0: default schedule (tile class 0, widest column chunk,
 *               chunks of tiles dealt round-robin to the XCDs);
 *               1: time every candidate schedule on zero inputs unless a
 *               batch of the same shape class was tuned before in this
 *               process, and keep the fastest; 2: always time; 3: the
 *               default schedule with the XCD-affine tile layout (every
 *               graph's tiles on one XCD).  Candidates: tile class 0 or 1,
 *               the widest chunk or half of it, either layout.  Every
 *               schedule computes each row with the same arithmetic as
 *               filtering its graph alone with that tile class.
 *   stream      orders the batch's device memory and the tuning runs; the
 *               call synchronises it before returning.
 *
 * Every SpMM pass of every graph and column chunk is one launch over the
 * tiles of all graphs; the whole sequence is captured into a HIP graph (on an
 * internal stream of default priority) that gift_batch_run replays.  The
 * batch owns its signal buffers (rows of all graphs x the chunk width, see
 * device_bytes).  Errors: GIFT_EINVAL (NULL pointers, sizes, mixed storage or
 * devices, a sigma not prepared, bad tune), GIFT_EUNSUPPORTED (dtype, more
 * than 2^31 - 1 tiles), GIFT_ENOMEM, GIFT_EDEVICE.  On error *out is NULL.
 */
gift_status gift_batch_create(const gift_graph *const *graphs, int32_t num_graphs,
                              const gift_term *terms, int32_t num_terms, int32_t num_cols,
                              int32_t in_dtype, int32_t out_dtype, int32_t tune, void *stream,
                              gift_batch **out);

/*
 * gift_batch_run -- filter every graph of the batch: uploads the per-graph
 * I/O pointers (io: host array of num_graphs entries, read during the call
 * only; they may change from run to run) and replays the captured graph on
 * `stream`.  Asynchronous.  Runs of one batch share its buffers: each run
 * waits (on the device) for the previous run of the batch, whatever stream
 * it was enqueued on.  Errors: GIFT_EINVAL (NULL
 * pointers, leading dimension < num_cols, wrong device), GIFT_EDEVICE.
 */
gift_status gift_batch_run(gift_batch *batch, const gift_batch_io *io, void *stream);

gift_status gift_batch_get_info(const gift_batch *batch, gift_batch_info *info);

/* Waits for the batch's last run, then releases it.  The graphs are not
 * touched. */
gift_status gift_batch_destroy(gift_batch *batch);

/* ------------------------------------------------------------------------
 * Request serving: filter requests for many designs with graphs kept
 * resident, admission by a device-memory budget and continuous batching.
 * ----------------------------------------------------------------------*/

typedef struct gift_server gift_server;

/* Server options.  Every request uses the same filter (terms), column count
 * and data types. */
typedef struct {
  int64_t hbm_budget_bytes; /* device memory for resident graphs, builds and
                               filter work (>= 1 MiB)                        */
  int32_t max_inflight;     /* requests admitted at once (>= 1)              */
  int32_t num_streams;      /* filter streams, default priority (1..16)      */
  int32_t num_builders;     /* build threads, one stream each (1..16)        */
  int32_t max_batch;        /* requests per launch sequence (>= 1)           */
  int64_t max_batch_rows;   /* graph rows per launch; a larger request runs
                               alone (>= 1)                                  */
  int32_t storage;          /* gift_dtype of the graphs built               */
  int32_t weight_model;     /* gift_weight_model                            */
  int64_t star_threshold;   /* as in gift_graph_desc                        */
  int32_t num_cols;         /* signal columns of every request (>= 1)       */
  int32_t in_dtype;         /* F32 or F64                                   */
  int32_t out_dtype;        /* F32 or F64                                   */
  int32_t num_terms;        /* 1..64                                        */
  const gift_term *terms;   /* copied                                       */
} gift_server_config;

/* One filter request.  The netlist (host memory) is read only if the design's
 * graph is not resident; it must stay valid until gift_server_wait returns
 * for the request.  The signals are device buffers as in
 * gift_filter_placement, N x num_cols with leading dimensions. */
typedef struct {
  uint64_t design_id; /* key of the resident graph: equal ids must name
                         equal netlists                                     */
  int64_t num_cells;
  int64_t num_nets;
  const int64_t *net_ptr;    /* host int64[num_nets + 1]                     */
  const int32_t *pin_cell;   /* host int32[net_ptr[num_nets]]               */
  const void *x_in;          /* device, in_dtype [num_cells][ld_in]         */
  int64_t ld_in;
  void *y_out;               /* device, out_dtype [num_cells][ld_out]       */
  int64_t ld_out;
  const uint8_t *fixed_mask; /* device uint8[num_cells] or NULL             */
} gift_request;

typedef struct {
  int32_t status;     /* gift_status of the request                        */
  int32_t built;      /* 1 if this request built its design's graph        */
  double latency_ms;  /* submit -> result complete on the device           */
  double queue_ms;    /* submit -> admitted                                */
  double service_ms;  /* admitted -> complete                              */
} gift_request_result;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t builds, evictions;
  int64_t batches;          /* launch sequences                              */
  int64_t batched_requests; /* requests over all launch sequences           */
  int64_t resident_graphs, resident_bytes;
  int64_t reserved_bytes, peak_reserved_bytes; /* budget accounting         */
  double p50_ms, p99_ms, mean_ms, max_ms;      /* latency of completed ones */
  double elapsed_s;         /* first submit -> last completion              */
} gift_server_stats;

/*
 * gift_server_create -- start a server on the current device: a dispatcher
 * thread and num_builders build threads.
 *
 * A submitted request is admitted when fewer than max_inflight requests are
 * admitted and its memory fits the budget: filter buffers, plus, if its
 * design is not resident, a bound on the graph and on the build's scratch
 * computed from the pin counts.  To make room the server evicts resident
 * graphs that no admitted request uses, least recently used first; a request
 * that does not fit yet waits without blocking later ones that do, and one
 * that can never fit fails with GIFT_ENOMEM.  A missing graph is built on a
 * builder's stream (eq. A_formulation) and stays resident.  Requests whose
 * graphs are resident are grouped by size (rows within a factor of two, at
 * most max_batch requests and max_batch_rows rows) and filtered
 * (eq. proposed_filter) by one launch sequence on the least loaded filter
 * stream; each result is computed with the same arithmetic as
 * gift_filter_placement on that graph alone.  Requests that arrive while
 * others run join later launches, so their work overlaps on the device.
 * Errors: GIFT_EINVAL (bad options), GIFT_EUNSUPPORTED, GIFT_EDEVICE.
 */
gift_status gift_server_create(const gift_server_config *config, gift_server **out);

/* Queue one request; *ticket identifies it.  Every ticket must be waited for
 * (gift_server_wait releases it).  Errors: GIFT_EINVAL, GIFT_EBUSY (server
 * stopping). */
gift_status gift_server_submit(gift_server *server, const gift_request *request,
                               uint64_t *ticket);

/* Wait until the request is complete on the device (timeout_s < 0: no
 * limit).  Returns the request's status (GIFT_EBUSY if the timeout expired;
 * the ticket stays valid then) and fills *result (may be NULL). */
gift_status gift_server_wait(gift_server *server, uint64_t ticket, double timeout_s,
                             gift_request_result *result);

/* Counters and latency percentiles of the requests completed since the last
 * reset; reset != 0 starts a new window. */
gift_status gift_server_get_stats(gift_server *server, int32_t reset, gift_server_stats *out);

/* Finish every submitted request, stop the threads and release every
 * resident graph. */
gift_status gift_server_destroy(gift_server *server);

/* ------------------------------------------------------------------------
 * Kernel timing (for benchmarks).
 * ----------------------------------------------------------------------*/

/* Kernel classes timed by the library's event profiler. */
typedef enum {
  GIFT_PROF_SPMM = 0,       /* an SpMM pass that stores its iterate          */
  GIFT_PROF_SPMM_FINAL = 1, /* the last SpMM pass with the fused combine     */
  GIFT_PROF_BUILD = 2,      /* one whole gift_build_graph call (all kernels) */
  GIFT_PROF_NUM_CLASSES = 3
} gift_prof_class;

/*
 * Enable (on != 0) or disable the event profiler for the calling process.
 * While enabled, the library records a pair of HIP events on the launch
 * stream around every launch of the timed classes, at the cost of two event
 * records per launch.  Enabling clears earlier records.
 */
gift_status gift_profile_enable(int32_t on);

/*
 * Pause (paused != 0) or resume the enabled profiler without waiting for or
 * clearing its records: while paused no events are recorded, so launches run
 * as with the profiler off.  A caller can time a sample of its launches this
 * way without paying the events on every launch.  Enabling or disabling
 * resumes.
 */
gift_status gift_profile_pause(int32_t paused);

/*
 * Totals since the last enable/collect for one class: number of launches,
 * summed and per-launch maximum device duration (milliseconds, from the
 * event pairs) and the summed algorithmic bytes of the launches.  An SpMM
 * pass counts row_ptr, col and values of the rows it covers, their diagonal,
 * every signal row read once and the rows it writes (the final pass: the saved
 * iterates it reads and the output); the build class reports 0 bytes.  Waits
 * for the recorded events; clears that class's records.  Any pointer may be
 * NULL.
 */
gift_status gift_profile_collect(int32_t prof_class, int64_t *launches, double *total_ms,
                                 double *max_ms, double *bytes);

/* ------------------------------------------------------------------------
 * Misc.
 * ----------------------------------------------------------------------*/

/*
 * The caller's device allocator, for callers that keep device memory under
 * their own allocator and budget (e.g. a framework's caching allocator).
 *
 *   alloc(bytes, device, stream, ctx)   returns `bytes` of device memory on
 *        `device` (the current device during the call) for work ordered on
 *        `stream` (a hipStream_t as void*), aligned to at least 256 bytes,
 *        or NULL on failure (the library then returns GIFT_ENOMEM).
 *   free(ptr, bytes, device, stream, ctx)   releases a block alloc returned.
 *        Stream-ordered: every use of the block is enqueued on `stream`
 *        before this point (or ordered before it by an event), so the block
 *        may be reused at once by later work on `stream`; reuse on another
 *        stream must first wait for `stream` (synchronise it or wait on an
 *        event recorded on it).
 *   ctx  passed back unchanged.
 *
 * Both callbacks may be called from any host thread (the serving engine's
 * threads included) and must be thread-safe; they must not call back into
 * the library.
 */
typedef struct {
  void *(*alloc)(size_t bytes, int32_t device, void *stream, void *ctx);
  void (*free)(void *ptr, size_t bytes, int32_t device, void *stream, void *ctx);
  void *ctx;
} gift_allocator;

/*
 * gift_set_allocator -- every device allocation the library makes from now
 * on (graphs, build and filter scratch, batches, servers, evaluators) comes
 * from `allocator` (copied) instead of the library's caching allocator; NULL
 * switches back to the cache.  A block is always returned to the allocator
 * that provided it, so the switch may happen at any time.  Pinned host
 * memory (a few small readback and staging slots per device) stays the
 * library's own.  Errors: GIFT_EINVAL when alloc or free is NULL.
 */
gift_status gift_set_allocator(const gift_allocator *allocator);

/*
 * Device memory held by the library's caching allocator (every block it
 * obtained from the runtime, cached or in use) and the device memory in use
 * by graphs, batches and in-flight calls (from the cache or from the
 * caller's allocator).  Blocks freed on a stream are reused only for
 * that stream, so the cache never needs a device synchronisation to reuse.
 */
gift_status gift_memory_stats(int64_t *bytes_held, int64_t *bytes_in_use);

/* Return every cached (unused) block to the runtime.  Synchronises the
 * device first.  Memory in use is not affected. */
gift_status gift_release_cached_memory(void);

const char *gift_status_string(gift_status status);

/* Description of the last error raised on the calling host thread ("" if
 * none).  The pointer is valid until the next library call on that thread. */
const char *gift_last_error(void);

/* Library and ABI version: returns GIFT_ABI_VERSION. */
int32_t gift_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GIFT_H */
