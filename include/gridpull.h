/*
 * gridpull.h -- C ABI of the MI355X (gfx950) GridPull pull-step library.
 *
 * GridPull (Chen, Liu, Han, ICCV 2023) fits a signed distance field D stored
 * on the vertices of a uniform grid to a point cloud S, with no neural
 * network.  One optimisation iteration samples queries q near the points,
 * interpolates D trilinearly (Sec. 3, Eq. 1 / Eq. 3), pulls each query along
 * the normalised field gradient, p = q - f(q) grad f(q) / |grad f(q)|, and
 * minimises (Eq. 8)
 *
 *     L = L_Pull + alpha L_TV + beta L_Surface + gamma L_grad
 *
 * with L_Pull = |p - NN(q)| (Eq. 4), the per-vertex total variation L_TV over
 * six axis neighbours (Eq. 5), L_Surface = |f(s)| at the surface point
 * s = NN(q) (Eq. 6) and L_grad = 1 - cos(grad f(q), grad f(s)) (Eq. 7).
 * Pulling is restricted to the cells within M1 cells of a cell holding a
 * point, TV to the cells within M2 (Sec. 3, band paragraphs); only the
 * vertices of those cells are optimised.  The optimiser is Adam with the
 * learning rate multiplied by a decay factor every fixed number of
 * iterations (Sec. 4, "Details").
 *
 * Conventions (every entry point):
 *  - A grid has R_x x R_y x R_z cells and (R+1) vertices per axis over the
 *    box [lo, hi]; h_a = (hi_a - lo_a) / R_a.  Vertex (i,j,k) sits at
 *    lo + (i,j,k) h.  Linear ids are x-major: vertex (i*(R_y+1)+j)*(R_z+1)+k,
 *    cell (cx*R_y+cy)*R_z+cz.
 *  - Cell location is done in double: u_a = ((double)x_a - lo_a) * inv_h_a with
 *    inv_h_a = R_a / (hi_a - lo_a); the cell is floor(u) clamped to R-1 (a
 *    point on hi lies in the last cell); a position is inside iff
 *    0 <= u_a <= R_a on every axis.  A query is valid iff it is inside and its
 *    cell is in the M1 band; invalid queries carry no loss and no gradient.
 *  - Coordinates are structure-of-arrays float32 (x[], y[], z[]).
 *  - Pointers documented "device" are device memory owned by the caller; the
 *    library never frees them.  Pointers documented "host" are host memory.
 *  - The context owns its internal structures (brick directory, masks, point
 *    buckets, scratch) and frees them in gp_destroy.
 *  - Work is enqueued on the context's stream and is asynchronous unless the
 *    entry point says it synchronises.  Device-detected failures (a
 *    non-finite loss) raise a device flag that the next synchronising call
 *    (gp_sync, gp_build_band) reports.
 *  - No exceptions cross the ABI.  Every call returns a gp_status;
 *    gp_last_error gives a message for the last failure.  A context is not
 *    thread safe.
 *  - Several shapes can share one context ("batched"): each has its own grid
 *    and slices of the point and query arrays, and each kernel launch covers
 *    all shapes.  A single shape is n_shapes = 1.
 *
 * Field layout ("slots"): values of the optimised vertices are stored in
 * bricks of B x B x B vertices (B = gp_build_band's brick: 4, 8 or 16); the
 * brick holding vertex (i,j,k) is (i/B, j/B, k/B) and the vertex's slot is
 * brick*B^3 + ((i%B)*B + j%B)*B + k%B (for B = 8: brick*512 +
 * ((i&7)*8+(j&7))*8+(k&7)).
 * Only bricks that hold an optimised vertex exist.  Slots of different
 * shapes are disjoint, in shape order.  The field, its gradient and the Adam
 * moments are caller-owned float32 device arrays of n_slots entries in this
 * layout; gp_export_layout maps slots to vertex ids.
 */
#ifndef GRIDPULL_H
#define GRIDPULL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_ctx_s* gp_ctx;

typedef enum {
    GP_OK = 0,
    GP_ERR_ARG = 1,       /* null pointer, bad size or dimension, unsupported option */
    GP_ERR_DOMAIN = 2,    /* a point lies outside its shape's [lo, hi]              */
    GP_ERR_CAPACITY = 3,  /* a size exceeds what the library can index             */
    GP_ERR_OOM = 4,       /* device allocation failed                               */
    GP_ERR_DEVICE = 5,    /* a HIP runtime call failed                              */
    GP_ERR_STATE = 6,     /* call out of order (e.g. before gp_build_band)          */
    GP_ERR_NUMERIC = 7    /* a loss came out non-finite                             */
} gp_status;

/* One shape of a batch (host memory).  Sec. 3: grid G of R^3 cells over the
 * space occupied by the point cloud; here R may differ per axis. */
typedef struct {
    int32_t dims[3];              /* cells per axis, each >= 1                      */
    double lo[3], hi[3];          /* domain box, hi > lo on every axis              */
    int64_t point_off, point_cnt; /* this shape's points: [point_off, +point_cnt)   */
    int64_t query_off, query_cnt; /* this shape's queries: [query_off, +query_cnt)  */
} gp_shape;

/* Balance weights of Eq. 8 (the paper uses alpha = beta = 1, gamma = 0.005). */
typedef struct {
    float alpha, beta, gamma;
} gp_weights;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
gp_status gp_create(gp_ctx* out, int device, void* hip_stream);

/* Free the context and everything it owns.  NULL is ignored. */
void gp_destroy(gp_ctx ctx);

/* Message of the last failure on this context ("" if none).  The string is
 * owned by the context and valid until the next call on it. */
const char* gp_last_error(gp_ctx ctx);

/* Change the stream later calls enqueue on. */
gp_status gp_set_stream(gp_ctx ctx, void* hip_stream);

/* Wait for the context's stream, then report any device-side flag
 * (GP_ERR_NUMERIC for a non-finite loss since the last gp_sync). */
gp_status gp_sync(gp_ctx ctx);

/*
 * Build the bands and indices of every shape (Sec. 3: uniform grid for query
 * localisation, the M1 band for pulling, the M2 band for TV; the spatial
 * index over the points that replaces the paper's KD-tree).
 *   base cells  = cells holding at least one point (location rule above);
 *   M1 band     = cells within Chebyshev distance m1 of a base cell (clipped);
 *   M2 band     = same with m2;
 *   optimised vertices = corners of M1- or M2-band cells;
 *   TV vertices = corners of M2-band cells.
 * shapes:   host [n_shapes]; point and query slices must lie inside the arrays
 *           later passed and must not overlap between shapes.
 * px,py,pz: device float32 points of all shapes; the context keeps a sorted
 *           copy, so the arrays may be freed afterwards.
 * m1, m2:   band half-widths in cells, 0 <= m <= 1024; a width of at least
 *           the largest dims - 1 covers the whole grid ("all grids").
 * brick:    brick edge in vertices: 4, 8 or 16 (else GP_ERR_ARG).  The field
 *           layout is brick-major: slot = brick * brick^3 + local vertex, the
 *           local vertex x-major inside the brick.  Smaller bricks pad a thin
 *           band less, larger ones put more of a cell's corners in one brick;
 *           the TV kernels' wave layout exists for 8 only (other sizes take
 *           the block layout whatever gp_set_tv_layout asks).
 * n_slots_out, n_active_vertices_out: host; the field length and the number
 *           of optimised vertices over all shapes.
 * Synchronises.  May be called again to rebuild (previous state is dropped).
 * Errors: GP_ERR_ARG (null pointers, n_shapes < 1, dims < 1, hi <= lo,
 * m out of range), GP_ERR_DOMAIN (a point outside its shape's box),
 * GP_ERR_CAPACITY (more than 2^30 slots or brick directory entries, or
 * more than 2^31 points), GP_ERR_OOM.
 */
gp_status gp_build_band(gp_ctx ctx, const gp_shape* shapes, int32_t n_shapes,
                        const float* px, const float* py, const float* pz,
                        int32_t m1, int32_t m2, int32_t brick,
                        int64_t* n_slots_out, int64_t* n_active_vertices_out);

/*
 * Nearest surface point of every query (NN(q) of Eq. 4), within the query's
 * own shape: nn_out[k] = argmin_j d2(q_k, s_j) with
 * d2 = ((dx*dx + dy*dy) + dz*dz), dx = (double)q_x - (double)s_x in double
 * without fused multiply-add; ties go to the lowest point index.  The index
 * is relative to the shape's point_off.  Defined for every query, also those
 * outside the band or the domain.
 * qx,qy,qz: device float32 [n_queries]; n_queries must equal the end of the
 *           last shape's query slice.  nn_out: device int32 [n_queries].
 * Errors: GP_ERR_STATE before gp_build_band, GP_ERR_ARG.
 */
gp_status gp_nn_query(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                      int64_t n_queries, int32_t* nn_out);

/*
 * Shape of the nearest-neighbour search (the same exact result for any
 * values; only the speed changes).  The queries of a 1024-query tile are
 * sorted along a Morton curve of their cells and cut into groups of at most
 * 64 whose cells span fewer than group_span cells on every axis; a group's
 * lanes scan the group's cell box grown by first_shell cells together, and
 * the queries that box does not settle continue alone.  tile_parts blocks
 * share a tile (each sorts it and takes 1/tile_parts of the groups), which
 * gives small batches more blocks.  With skip_empty, every column of cells
 * to be scanned is first cut to its first and last cell holding a point (a
 * bitmap of one bit per cell), which saves range lookups where points are
 * sparse.  Without morton_sort the groups are cut along the queries' own
 * order (enough when the caller's order is already spatially coherent).
 *
 * The search runs on a grid of its own per shape (the index that replaces
 * the paper's KD-tree): the shape's box in cells 2^k band cells wide, k in
 * [0, 3] the integer nearest to log2(cell_points / m) / 2, m the mean number
 * of points per band cell holding a point (points on a surface fill a cell
 * twice as wide four times as densely), so that sparse points do not leave
 * most scanned cells empty at a fine band resolution.  "Cells" above are
 * cells of this grid.
 */
typedef struct {
    int32_t group_span;    /* [1, 64], default 8 */
    int32_t first_shell;   /* [0, 4], default 1 */
    int32_t tile_parts;    /* 1, 2 or 4, default 1 */
    int32_t skip_empty;    /* 0 or 1, default 0 */
    int32_t morton_sort;   /* 0 or 1, default 1 */
    int32_t cell_points;   /* [1, 65536], default 8 */
} gp_nn_params;

/*
 * Set / read the context's search shape (host struct; it survives
 * gp_build_band).  A new cell_points rebuilds the search grids of a built
 * context (synchronises); if that rebuild fails, the context needs
 * gp_build_band again (other calls report GP_ERR_STATE).  Errors: GP_ERR_ARG
 * (null pointer, a field out of range), GP_ERR_OOM, GP_ERR_CAPACITY.
 */
gp_status gp_set_nn_params(gp_ctx ctx, const gp_nn_params* params);
gp_status gp_get_nn_params(gp_ctx ctx, gp_nn_params* params);

/*
 * The search grid of shape `shape` (the index that stands in for the KD-tree
 * of Sec. 3, query sampling paragraph): dims_out (host [3]) its cells per
 * axis, level_out (host, may be NULL) its k (cells 2^k band cells wide).
 * Errors: GP_ERR_STATE before gp_build_band, GP_ERR_ARG (shape out of range,
 * null dims_out).
 */
gp_status gp_get_nn_grid(gp_ctx ctx, int32_t shape, int32_t* dims_out, int32_t* level_out);

/*
 * Autotuner of the search grid and shape, timing gp_nn_query's kernel on the
 * given queries at the current setting, then:
 *  1. the search grids of cell_points 4, 16, 64, ... times the current value
 *     (each factor of 4 moves every shape's k by one) while each is the
 *     fastest so far, else 1/4, 1/16, ... of it likewise (each grid rebuilt;
 *     a value that gives grids already timed ends its direction);
 *  2. on the fastest grid, group_span in {4, 6, 8, 12, 16, 24, 32} x
 *     first_shell in {0, 1, 2}, then tile_parts in {1, 2, 4} at the best of
 *     those (and, if that changes tile_parts, the span x shell grid again);
 *  3. the other skip_empty setting, then the other morton_sort setting.
 * Each candidate runs once and then reps times between HIP events on the
 * context's stream (its time: the smallest of the repeats; one whose first
 * run takes 4 times the best so far is not repeated).  Keeps the fastest in
 * the context (with its search grids) and leaves nn_out holding the nearest
 * neighbours (as gp_nn_query).  The current setting stays unless another is
 * at least 2% faster.
 * Arguments as gp_nn_query; reps in [1, 100]; chosen_out (host, may be NULL)
 * receives the choice and best_ms_out (host, may be NULL) its time in ms
 * (-1 with no queries).  Synchronises; not for use under stream capture.
 * Errors: as gp_nn_query, GP_ERR_ARG for reps, GP_ERR_DEVICE, GP_ERR_OOM.
 */
gp_status gp_autotune_nn(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                         int64_t n_queries, int32_t* nn_out, int32_t reps,
                         gp_nn_params* chosen_out, float* best_ms_out);

/*
 * Thread layout of the TV kernels (Eq. 5 and its gradient; the same
 * arithmetic either way): 1 = one block per brick, one thread per vertex;
 * 2 = one wave per brick, one lane per column of eight vertices; 0 (the
 * default) = by band size: the forward uses 2 from 2048 bricks on, the
 * backward from 16384.  Sets the two thresholds of gp_grad_params (1: both
 * INT64_MAX, 2: both 0, 0: the defaults).  The setting belongs to the context.
 * Errors: GP_ERR_ARG (layout not 0, 1 or 2).
 */
gp_status gp_set_tv_layout(gp_ctx ctx, int32_t layout);

/*
 * Settings of the gradient pass (derivative of Eq. 4-7 scattered to the
 * field) and of the TV kernels (Eq. 5); every value gives the same
 * arithmetic, only the speed changes (and, through the order of float
 * atomics between blocks, the last bits of the gradient).
 *   window_cap:         LDS accumulators of a query block, in vertices:
 *                       2048, 4096 (default) or 6144 (8 bytes each, in rows
 *                       of 16 consecutive slots: 16, 32 or 48 KB, plus 4 KB
 *                       of line map, per 256-query block; the largest leaves
 *                       fewer blocks per CU).  A block touching more 16-slot
 *                       lines than there are rows takes them in turns;
 *   window_max_passes:  [1, 64], default 16: a block whose box of query and
 *                       nearest-point cells needs more slabs (whole x layers
 *                       of at most 2048 lines) adds its contributions
 *                       straight to the gradient with global atomics;
 *   tv_forward_wave_from, tv_backward_wave_from: >= 0; from this many
 *                       bricks on, the TV forward (backward) takes one wave
 *                       per brick, below it one block (defaults 2048, 16384).
 * The settings belong to the context and survive gp_build_band.
 * Errors: GP_ERR_ARG (null pointer, a field out of range).
 */
typedef struct {
    int32_t window_cap;
    int32_t window_max_passes;
    int64_t tv_forward_wave_from;
    int64_t tv_backward_wave_from;
} gp_grad_params;

gp_status gp_set_grad_params(gp_ctx ctx, const gp_grad_params* params);
gp_status gp_get_grad_params(gp_ctx ctx, gp_grad_params* params);

/*
 * Autotuner of gp_grad_params (the passes that evaluate Eq. 4-8 and scatter
 * their derivative) on the caller's queries, nearest points and field
 * (arguments as gp_pull_forward_backward): times the fused query pass
 * for window_cap in {2048, 4096, 6144} x window_max_passes in {4, 16, 64},
 * then the TV forward and the TV backward in each layout at the band's size
 * (the faster one moves its threshold to the band's brick count, so that
 * bands at least as large take the wave layout, or just above it).  Each
 * candidate runs once and then reps times between HIP events on the
 * context's stream (its time: the smallest of the repeats).  The current
 * setting stays unless another is at least 2% faster.  Leaves the gradient
 * and loss arrays of the caller untouched (it runs on the context's
 * scratch), and invalidates the context's last forward (gp_forward_token).
 * reps in [1, 100]; chosen_out (host, may be NULL) receives the settings,
 * best_ms_out (host [3], may be NULL) the chosen query pass, TV forward and
 * TV backward times in ms (-1 for a part with nothing to time; the TV layouts
 * are timed for 8^3 bricks only, the other sizes having the block layout
 * alone).
 * Synchronises; not for use under stream capture.
 * Errors: GP_ERR_STATE before gp_build_band, GP_ERR_ARG (null pointers,
 * n_queries not the end of the last shape's query slice, reps),
 * GP_ERR_DEVICE.
 */
gp_status gp_autotune_grad(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                           int64_t n_queries, const float* field, gp_weights w, int32_t reps,
                           gp_grad_params* chosen_out, float* best_ms_out);

/*
 * Draw one iteration's queries (Sec. 3: Gaussian around randomly chosen
 * surface points, resampled every iteration).  For shape s with J points and
 * Q queries, query k uses source point P[(floor(k*J/Q) + o) mod J] where P is
 * the library's spatially sorted point order and o is a per-iteration random
 * offset, so every point is used floor(Q/J) or ceil(Q/J) times; the offset is
 * sigma_j * z with z from Philox4x32-10 (counter (k mod 2^32, k >> 32,
 * iteration, s), key (seed mod 2^32, seed >> 32)) and the Box-Muller
 * transform of U = ((x >> 8) + 1/2) 2^-24: z0, z1 = sqrt(-2 ln U0)
 * (cos, sin)(2 pi U1), z2 = sqrt(-2 ln U2) cos(2 pi U3).
 * sigma:  device float32 per point (indexed like the points) or NULL to use
 *         sigma_const for every point.
 * qx,qy,qz: device float32 outputs [total queries].
 * src_out: device int32 [total queries] or NULL; receives the source point
 *         index (relative to point_off).
 * iteration < 0 uses the context's device-resident iteration counter plus
 * one (the t of the next gp_step), for replayed graphs.
 */
gp_status gp_sample_queries(gp_ctx ctx, uint64_t seed, int32_t iteration,
                            const float* sigma, float sigma_const,
                            float* qx, float* qy, float* qz, int32_t* src_out);

/*
 * Forward pass of Eq. 8 for every shape.
 * qx,qy,qz,nn: device [n_queries] (nn as returned by gp_nn_query).
 * field:    device float32 [n_slots].
 * loss_out: device double [n_shapes][5] = {L, L_Pull, L_TV, L_Surface, L_grad}
 *           where L_Pull, L_Surface and L_grad are means over the shape's
 *           valid queries (0 if none) and L_TV is the mean of
 *           tau_i = sqrt(sum over the six neighbours j that are TV vertices of
 *           (D_i - D_j)^2) over the TV vertices; L = L_Pull + alpha L_TV +
 *           beta L_Surface + gamma L_grad.
 * n_valid_out: device int64 [n_shapes], the valid-query counts.
 * A normalised gradient with |grad f| < 1e-12 is taken as 0 (then
 * L_grad = 1 for that query).  The context keeps the valid counts and the
 * per-vertex tau for the next gp_pull_backward.
 */
gp_status gp_pull_forward(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                          const int32_t* nn, int64_t n_queries, const float* field,
                          gp_weights w, double* loss_out, int64_t* n_valid_out);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the loss of
 * gp_pull_forward, same arguments and same loss_out / n_valid_out, with no
 * allocation at all.  It neither allocates nor uses the context's scratch:
 * its partial sums live in a static device array of 8 MiB per GPU, held
 * until the process ends, and it leaves the context's forward state (what a
 * gp_pull_backward reuses, and gp_forward_token) as it was.  It stores no
 * per-vertex tau, so no backward follows it.  Calls that overlap on one GPU
 * (several contexts or threads on one device) share that array and race.
 * Errors: as gp_pull_forward, and GP_ERR_CAPACITY when the band needs more
 * scratch than 8 MiB (8 * (4 * tiles + bricks + 161 * shapes) + 4 * shapes
 * bytes, with tiles = ceil(queries / 1024) per shape).
 */
gp_status gp_pull_forward_static(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                                 const int32_t* nn, int64_t n_queries, const float* field,
                                 gp_weights w, double* loss_out, int64_t* n_valid_out);

/*
 * Token of the last forward (gp_pull_forward or gp_pull_forward_backward) on
 * this context, or 0 if there is none or it is no longer usable: a later call
 * of this library that writes its query, nearest-point or field array
 * (gp_sample_queries, gp_nn_query, gp_autotune_nn, gp_step, gp_init_sphere,
 * gp_gather_vertices) or rebuilds the band makes it 0.  Take it right after
 * the forward and hand it to the gp_pull_backward that differentiates it.
 * Writes the caller makes itself (a copy into the field) are not seen.
 */
uint64_t gp_forward_token(gp_ctx ctx);

/*
 * Backward pass: grad[slot] += sum_s dloss[s] * dL_s / dD[slot] for every
 * optimised vertex, with the L of gp_pull_forward, through trilinear
 * interpolation, the analytic gradient and its normalisation (derivative 0
 * where |grad f| < 1e-12 and where the residual p - s is 0; d|f_s| = sign f_s).
 * It reuses the valid counts and tau of the forward it differentiates, so it
 * must name that forward: forward_token is gp_forward_token() taken after
 * it, and qx, qy, qz, nn, field are the arrays it read.  GP_ERR_STATE if the
 * token is 0 or not the current one (another forward ran since, or one of
 * those arrays was written by the library), or if the arrays differ.
 * dloss: device double [n_shapes] upstream scale (1 for plain optimisation).
 * grad:  device float32 [n_slots], accumulated into.
 */
gp_status gp_pull_backward(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                           const int32_t* nn, int64_t n_queries, const float* field,
                           gp_weights w, const double* dloss, float* grad, uint64_t forward_token);

/*
 * Forward and backward in one pass over the queries (Eq. 4-8 and their
 * derivative): the same loss_out / n_valid_out as gp_pull_forward and the same
 * accumulation grad[slot] += sum_s dloss[s] * dL_s / dD[slot] as
 * gp_pull_backward, with each query evaluated once.  dloss must be known
 * before the call (the training iteration passes 1).  Leaves the context
 * state of a gp_pull_forward, so a gp_pull_backward may follow.
 * Arguments and errors as for gp_pull_forward and gp_pull_backward.
 */
gp_status gp_pull_forward_backward(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                                   const int32_t* nn, int64_t n_queries, const float* field,
                                   gp_weights w, const double* dloss, double* loss_out,
                                   int64_t* n_valid_out, float* grad);

/*
 * Normal supervision (Sec. 4, normals paragraph: with ground-truth normals,
 * the gradient of the field at the surface points is supervised by them).
 * Reading: L_N = (1/Q_v) sum over valid queries of (1 - gh_s . n_s), with
 * s = NN(q), gh_s = grad f(s) / |grad f(s)| (below 1e-12 the term is 1 with
 * zero gradient), Q_v and validity as for gp_pull_forward.  A separate term:
 * the caller adds weight * L_N to the objective of gp_pull_forward.
 * qx,qy,qz,nn,field: as gp_pull_backward.
 * nx,ny,nz: device float unit normals, indexed like the points of
 *          gp_build_band (global index point_off + j).
 * weight:  the term's weight; dloss: device [n_shapes] upstream scale or NULL
 *          (1).
 * term_out: device double [n_shapes], L_N of each shape (unweighted).
 * grad:    device float [n_slots] or NULL; receives += weight * dloss *
 *          dL_N/dD (float atomics: the order of the additions varies).
 * The first call on a context allocates its scratch.
 * Errors: GP_ERR_STATE, GP_ERR_ARG.
 */
gp_status gp_pull_normals(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                          const int32_t* nn, int64_t n_queries, const float* field,
                          const float* nx, const float* ny, const float* nz, float weight,
                          const double* dloss, double* term_out, float* grad);

/*
 * One Adam step (Kingma and Ba, 2015) on the optimised vertices at iteration
 * t, learning rate lr0 * decay^floor((t-1)/decay_every) (Sec. 4: decay 0.3
 * every 400 iterations); then grad is set to 0 on every slot.  Slots that are
 * not optimised vertices keep their field value.
 * t >= 1: that iteration.  t = 0: the context's device-resident iteration
 *   counter plus one (so a captured graph of a whole iteration replays the
 *   schedule correctly).  Either way the counter is left at the step's t;
 *   gp_build_band resets it to 0.
 * field, grad, m, v: device float32 [n_slots] (m, v start at 0).
 * Errors: GP_ERR_ARG for t < 0, decay_every < 1, beta outside [0, 1), eps < 0.
 */
gp_status gp_step(gp_ctx ctx, float* field, float* grad, float* m, float* v, int32_t t,
                  float lr0, float decay, int32_t decay_every,
                  float beta1, float beta2, float eps);

/* ---- per-kernel timing ---------------------------------------------------- */

/* enable != 0: bracket every kernel this context launches with HIP events on
 * its stream (not allowed while the stream is being captured into a graph). */
gp_status gp_timing_enable(gp_ctx ctx, int enable);

/* Synchronise, then write one line "kernel_name launches total_ms" per kernel
 * launched since the last report into buf (host, NUL-terminated, truncated to
 * buf_size), and start a new period.  GP_ERR_CAPACITY if buf is too small. */
gp_status gp_timing_report(gp_ctx ctx, char* buf, int64_t buf_size);

/* ---- layout helpers (not on the per-iteration path) ------------------- */

/* host [n_shapes + 1]: slot_begin[s] is the first slot of shape s,
 * slot_begin[n_shapes] = n_slots. */
gp_status gp_shape_slots(gp_ctx ctx, int64_t* slot_begin);

/* vertex_id_of_slot: device int64 [n_slots], the vertex id within the slot's
 * shape, -1 for slots past the grid's last vertex.  slot_flags: device
 * uint8 [n_slots] or NULL; bit 1 = optimised vertex, 2 = TV vertex,
 * 4 = the cell whose lowest corner is this vertex is in the M1 band,
 * 8 = ... in the M2 band, 16 = ... holds a point. */
gp_status gp_export_layout(gp_ctx ctx, int64_t* vertex_id_of_slot, uint8_t* slot_flags);

/* Sorted linear ids, (cx*Ry + cy)*Rz + cz, of the M1-band cells of one shape
 * (Sec. 3: the cells near the surface where queries are pulled; a query is
 * valid iff its cell is one of them).  cell_ids: device int64 [capacity];
 * *n_out (host) receives the number of cells.  When it exceeds capacity
 * nothing is written and GP_ERR_CAPACITY is returned with *n_out set, so a
 * call with capacity 0 asks for the size.  Synchronises with the context's
 * stream; allocates temporary device memory (not for the hot loop).
 * Errors: GP_ERR_ARG for a shape out of range or a null n_out. */
gp_status gp_export_active_cells(gp_ctx ctx, int32_t shape, int64_t* cell_ids, int64_t capacity,
                                 int64_t* n_out);

/*
 * Mesh of the zero level set of `field` over the cells of one shape whose
 * eight corners are optimised vertices (the surface extracted after the
 * optimisation: Sec. 3, last paragraph, cells not optimised are skipped;
 * Sec. 4 "Details", marching cubes).  A corner is inside where f < 0.
 * method 0, marching cubes: a cell's triangles follow from which of its
 * corners are inside (corner (a, b, c) at index 4a + 2b + c), by one rule:
 * on each face, walked counter-clockwise from outside, every run of inside
 * corners is cut off by a segment from the edge where the walk leaves it to
 * the edge where it entered (diagonal inside corners of a face are cut off
 * separately, the same from both cells of the face: no cracks); the
 * segments close into loops from the lowest crossed edge (edges along axis
 * d numbered 4d + 2u + v by the other two coordinates), each loop fanned
 * from its first edge.  At most 5 triangles per cell.
 * method 1, marching tetrahedra: each cell is cut into six tetrahedra along
 * its main diagonal, (0, A, B, 7) for the corner paths 0 -> A -> B -> 7,
 * which neighbouring cells cut alike; one corner against three gives one
 * triangle, two and two give two.
 * Either way each triangle corner is p + f_p / (f_p - f_q) (q - p) on an edge
 * from its inside end p to its outside end q, in double (vertex positions
 * lo + i * (hi - lo) / R), rounded to float at the end.
 * field:   device float [n_slots] (the slot layout of gp_build_band).
 * tri_xyz: device float [capacity][3][3], the corners' x, y, z.
 * tri_key: device int64 [capacity], cell_id * 16 + the triangle's number in
 *          its cell (method 1: tetrahedron * 2 + triangle; cell_id x-major),
 *          ascending; the triangles follow it.
 * n_out:   host; the number of triangles.  With capacity 0 (outputs may be
 *          NULL) only the count is returned.
 * Synchronises; allocates temporary device memory (about 40 bytes per
 * triangle plus 8 per slot of the shape).
 * Errors: GP_ERR_STATE before gp_build_band, GP_ERR_ARG (also a method
 * other than 0 or 1), GP_ERR_CAPACITY (capacity below the count; n_out is
 * set), GP_ERR_OOM.
 */
gp_status gp_extract_surface(gp_ctx ctx, int32_t shape, const float* field, float* tri_xyz, int64_t* tri_key,
                             int64_t capacity, int64_t* n_out, int32_t method);

/* field[slot] = dense[dense_off(s) + vertex id] for every slot (0 where the
 * slot has no vertex), where dense is the concatenation, in shape order, of
 * each shape's (R+1)^3 vertex values in x-major order.  Device arrays. */
gp_status gp_gather_vertices(gp_ctx ctx, const float* dense, float* field);

/* dense[dense_off(s) + vertex id] = field[slot] for every optimised vertex;
 * other entries are left as they are.  Device arrays. */
gp_status gp_scatter_vertices(gp_ctx ctx, const float* field, float* dense);

/* Geometric initialisation (Sec. 3): field = |x_v - centre_s| - radius_s at
 * every slot with a vertex.  centre: host double [n_shapes][3];
 * radius: host double [n_shapes]. */
gp_status gp_init_sphere(gp_ctx ctx, const double* centre, const double* radius, float* field);

#ifdef __cplusplus
}
#endif

#endif /* GRIDPULL_H */
