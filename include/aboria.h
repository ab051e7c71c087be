/*
 * aboria.h -- C-ABI of the MI355X (gfx950) library for the hot path of the
 * particle-based methods of Robinson & Bruna, "Particle-based and Meshless
 * Methods with Aboria" (arXiv:1704.08907):
 *
 *   1. building a uniform cell list over a d-dimensional box whose dimensions
 *      are each periodic or not (Section 1, property 1; Section 2.2.1, the
 *      Level 1 cell list with particles reordered into cell order),
 *   2. evaluating radius-limited pairwise neighbourhood sums over it by box
 *      search of a particle's cell and its adjacent cells (Section 2.2.2,
 *      Level 2; Section 3, eq. (1) and the velocity-update listing), with a
 *      hand-written adjoint, and
 *   3. the dense all-pairs kernel sum of the RBF / Gaussian-process methods
 *      (Section 1 and Section 1.1).
 *
 * Conventions shared by every entry point:
 *   - Pointers named *_host point to host memory; every other array pointer is
 *     a device pointer on the context's device.  The caller owns all arrays it
 *     passes; the library owns contexts, cell lists and graphs.
 *   - Work is enqueued on the context's HIP stream and is stream-ordered; a call
 *     returning ABORIA_OK means the work was enqueued.  Argument errors are
 *     detected on the host before anything is enqueued, and nothing is
 *     launched then.  Errors found on the device (a NaN position, a position
 *     outside [lo, hi)) raise a sticky flag reported by aboria_sync.
 *   - No C++ exception crosses this boundary.  aboria_last_error returns the
 *     message of the context's latest failure.
 *   - Arrays are row-major.  Positions are x[n][d] in the cell list's precision
 *     (float for ABORIA_F32, double for ABORIA_F64).  Outputs never alias
 *     inputs: an overlap is an ABORIA_ERR_INVALID_ARG.
 *   - A context is used by one host thread at a time.
 */
#ifndef ABORIA_H
#define ABORIA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum aboria_status {
    ABORIA_OK = 0,
    ABORIA_ERR_INVALID_ARG = 1,   /* bad argument; nothing was enqueued          */
    ABORIA_ERR_DOMAIN = 2,        /* a position was NaN or outside [lo, hi)      */
    ABORIA_ERR_UNSUPPORTED = 3,   /* valid but not handled (e.g. periodic L < 2r) */
    ABORIA_ERR_OUT_OF_MEMORY = 4, /* device allocation failed                    */
    ABORIA_ERR_DEVICE = 5         /* a HIP runtime call failed                   */
} aboria_status;

typedef enum aboria_dtype { ABORIA_F32 = 0, ABORIA_F64 = 1 } aboria_dtype;

/*
 * Pairwise operators y_i = sum_{j in P(i)} f(x_i, x_j, a_i, a_j), P(i) the
 * canonical neighbour set of i (see aboria_build_cells).  With u = x_i - x_j
 * (minimum image) and s = |u|:
 *   COUNT        ny = 1   f = 1                                 (|P(i)|)
 *   SPRING       ny = d   f = k (r - s) u / s,  params {k}       linear spring of
 *                         rest length r (Section 1.1, Molecular Dynamics)
 *   SOFT_SPHERE  ny = 1   f = 1/2 (1 - s/r)^2, no params          pair energy,
 *                         E = sum_i y_i counts each unordered pair once
 *   EXP_FORCE    ny = d   f = -c exp(-|dx|) dx/|dx|, dx = -u,  params {c}
 *                         the paper's eq. (1)
 *   DEM_SPRING   ny = d   f = k (a_i + a_j - s) u / s, na = 1, params {k}
 *                         spring with per-particle resting lengths (Section 1.1,
 *                         Discrete Element Model)
 */
typedef enum aboria_op {
    ABORIA_OP_COUNT = 0,
    ABORIA_OP_SPRING = 1,
    ABORIA_OP_SOFT_SPHERE = 2,
    ABORIA_OP_EXP_FORCE = 3,
    ABORIA_OP_DEM_SPRING = 4
} aboria_op;

typedef enum aboria_kernel {
    ABORIA_K_GAUSSIAN = 0,    /* K(x, x') = exp(-|x - x'|^2 / (2 sigma^2)), params {sigma}; the
                                 Gaussian basis of the Kansa example (Section 1.1) */
    ABORIA_K_MULTIQUADRIC = 1 /* K(x, x') = sqrt(|x - x'|^2 + c^2), params {c}; the multiquadric
                                 basis of the RBF example (Section 1.1), in Hardy's form */
} aboria_kernel;

/* A hypercube domain [lo, hi) and cutoff (Section 1, property 1; the
 * init_neighbour_search(lo, hi, width, periodic) call of Section 3).  Entries
 * beyond d are ignored.
 *
 * reach[k] = m (1..3; 0 = 1) is how many cells the box search looks on each
 * side of a particle's own cell in dimension k.  m = 1 is the paper's lattice:
 * cells at least one cutoff wide, searched with the adjacent cells (Section
 * 2.2.2).  m = 2 or 3 uses cells about r/m wide searched m cells deep, which
 * tests fewer candidates; the pair set is the same, since the pair predicate
 * alone decides it.  A deeper reach along x only (e.g. {2, 1, 1}) keeps the
 * 3^(d-1) rows of the search and shortens each.  The recorded-mask variant
 * needs m = 1 in every dimension but x.
 *
 * ncell[k] = 0 picks the cell count automatically: the largest count whose
 * cells are at least (cutoff + a rounding guard) / m wide.  An explicit count
 * must not exceed that and is honoured as given. */
typedef struct aboria_box {
    int32_t d;           /* 1, 2 or 3                                  */
    int32_t periodic[3]; /* nonzero = periodic in that dimension       */
    int32_t ncell[3];    /* 0 = automatic                              */
    int32_t reach[3];    /* search reach m per dimension, 0 = 1        */
    double lo[3];
    double hi[3];
    double cutoff;       /* r > 0                                      */
} aboria_box;

typedef struct aboria_ctx aboria_ctx;
typedef struct aboria_cells aboria_cells;
typedef struct aboria_graph aboria_graph;

/* Read-only view of a cell list (device pointers stay owned by the cells). */
typedef struct aboria_cells_view {
    int32_t nsys;                   /* number of independent systems              */
    int32_t d;
    int32_t dtype;                  /* aboria_dtype                               */
    int32_t sort_ipt;               /* RADIX build: keys per thread of a sort tile */
    int64_t n;                      /* total particles                            */
    int64_t ncells;                 /* total cells over all systems               */
    const uint32_t* perm;           /* device [n]: sorted slot -> original index  */
    const uint32_t* keys;           /* device [n]: global cell id of each slot    */
    const uint32_t* cell_offsets;   /* device [ncells + 1]: first slot of a cell  */
    const void* x_sorted;           /* device [n][pitch]: positions in cell order */
    int32_t x_pitch;                /* elements per sorted position (4 for d = 3) */
    int32_t bucket_bits;            /* RADIX build: key bits sorted per bucket     */
    const int32_t* ncell_host;      /* host [nsys][3]: cells per dimension        */
    const uint32_t* cell_base_host; /* host [nsys + 1]: first global cell id      */
    const int64_t* sys_offsets_host;/* host [nsys + 1]: first particle of a system */
} aboria_cells_view;

/* ---- context ------------------------------------------------------------- */

/* Creates a context on HIP device `device` that enqueues on `hip_stream` (a
 * hipStream_t; NULL = the legacy default stream).  *out receives the handle. */
aboria_status aboria_create(int32_t device, void* hip_stream, aboria_ctx** out);
/* Releases the context and its scratch memory (waits for its stream first).
 * Called on a thread while that thread captures a graph (on any context), the
 * release waits until the thread's last capture ends: a free or a wait would
 * invalidate the capture.  The same holds for aboria_cells_destroy and
 * aboria_graph_destroy. */
aboria_status aboria_destroy(aboria_ctx* ctx);
/* Changes the stream subsequent calls enqueue on. */
aboria_status aboria_set_stream(aboria_ctx* ctx, void* hip_stream);
/* Message of the latest failure on this context ("" if none); owned by ctx. */
const char* aboria_last_error(const aboria_ctx* ctx);
/* Waits for the context's stream, then reports and clears the device error
 * flag: ABORIA_ERR_DOMAIN if a position seen by a cell build since the last
 * sync was NaN or outside [lo, hi). */
aboria_status aboria_sync(aboria_ctx* ctx);

/* ---- cell list (Section 2.2.1 Level 1, Section 2.2.2 Level 2) ---------------
 *
 * Builds the cell list of nsys independent systems whose particles are
 * concatenated in x: system b owns rows [offsets_host[b], offsets_host[b+1]) of
 * x[n][d] (n = offsets_host[nsys]; offsets_host is required, {0, n} for a single
 * system; total rows < 2^31).  boxes_host[b] is system b's box; all boxes share
 * d.  The steps: a cell id per particle, a stable LSD radix sort of
 * (cell id, index) pairs in LDS-ranked passes, a gather of the positions into
 * cell order, and the cell offsets (first slot of every cell).  Within a cell
 * particles keep their original index order.
 *
 * Canonical rounding (precision P = dtype): cell coordinate
 * clamp(floor(fl(fl(x - lo) * fl(n/L))), 0, n-1); linear id c0 + n0 (c1 + n1 c2)
 * plus the system's first global cell id.  The neighbour set of i is every j
 * in the 3^d cells around i's cell (wrapping with an image shift s_k = -L or +L
 * in periodic dimensions) with 0 < d2 < fl(r*r), where t_k = fl(x_jk - x_ik),
 * dx_k = fl(t_k + s_k) and d2 = fma(dx2, dx2, fma(dx1, dx1, dx0 * dx0)); the
 * norm(dx) > 0 condition of the Section 3 listing is the d2 > 0 test.
 *
 * *cells == NULL creates a cell list; otherwise it is rebuilt in place (the
 * same nsys, d, dtype and n; no allocation, so a rebuild may be captured in a
 * graph).  The cell list keeps its own sorted copy of the positions: results of
 * later sums use the positions as they were at build time, and x may be reused
 * once the stream has passed this call (Section 2.2.1: the search structure is
 * rebuilt when positions change).
 * Errors: INVALID_ARG for d outside 1..3, hi <= lo, cutoff <= 0, an explicit
 * ncell above the automatic one, inconsistent boxes or offsets; UNSUPPORTED for
 * a periodic side shorter than twice the guarded cutoff, or more than 2^31
 * cells in total; OUT_OF_MEMORY if the device buffers cannot be allocated. */
aboria_status aboria_build_cells(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys,
                                 const aboria_box* boxes_host, const int64_t* offsets_host,
                                 const void* x, aboria_cells** cells);
aboria_status aboria_cells_view_get(const aboria_cells* cells, aboria_cells_view* out);

/* How aboria_build_cells sorts particles into cell order (both give the same
 * cell list, bit for bit: stable by cell, original index order inside a cell):
 *   RADIX     LDS-ranked stable LSD radix passes over the high key bits, then
 *             one pass per bucket of cells that also writes the offsets and
 *             gathers the positions;
 *   COUNTING  a per-cell count with each particle's arrival rank (atomic), a
 *             scan of the counts (the cell offsets), placement, and a per-slot
 *             fix-up that restores original index order inside each cell.
 * The setting applies to later builds on ctx; the default is RADIX. */
typedef enum aboria_build_strategy { ABORIA_BUILD_RADIX = 0, ABORIA_BUILD_COUNTING = 1 } aboria_build_strategy;
aboria_status aboria_set_build_strategy(aboria_ctx* ctx, aboria_build_strategy strategy);
/* Releases a cell list (after the device has finished with it; deferred while
 * the calling thread captures a graph, see aboria_destroy). */
aboria_status aboria_cells_destroy(aboria_cells* cells);

/* Shape of the RADIX build (Section 2.2.1's sort into cell order): keys per
 * thread of a sort tile of 256 threads (4, 8 or 16: tiles of 1024 to 4096
 * keys), the key bits the last pass sorts per bucket of cells in LDS (8 to 10;
 * the radix passes take the remaining high bits) and whether a radix pass
 * shuffles its tile into digit order in LDS before writing (1: where the LDS
 * fits, 2: never).  The shape does not change the cell list, only the work
 * mapping of its build.  aboria_set_build_shape fixes it for cell lists
 * created later on ctx (0 for a value: the built-in rule, or the tuned shape
 * for that size); INVALID_ARG for other values.  aboria_autotune_build creates
 * a cell list for the boxes at each shape, times five rebuilds of each with HIP
 * events and caches the fastest for cell lists of the same d, dtype, batch and
 * size buckets (floor log2 of the particles and of the cells), which later
 * creations use; *ipt_out, *low_bits_out and *shuffle_out (may be NULL)
 * receive it.  Persisted like aboria_autotune's choices; arguments as for
 * aboria_build_cells; allocates and synchronises, so it cannot be captured. */
aboria_status aboria_set_build_shape(aboria_ctx* ctx, int32_t ipt, int32_t low_bits, int32_t shuffle);
aboria_status aboria_autotune_build(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys, const aboria_box* boxes_host,
                                    const int64_t* offsets_host, const void* x, int32_t* ipt_out,
                                    int32_t* low_bits_out, int32_t* shuffle_out);

/* ---- neighbour sums (Section 3: eq. (1) and the velocity-update listing) ----
 *
 * y[n][ny] = sum over the neighbour set of each particle of the operator's
 * summand (see aboria_op), in the original particle order, computed in the
 * cell list's precision.  a[n][na] holds per-particle variables in original
 * order (NULL when the operator takes none).  params_host[nparams] are the
 * operator's constants; the cutoff r is the cell list's.  y is overwritten.
 * Errors: INVALID_ARG for an unknown op, ny/na/nparams not those of the op,
 * NULL or overlapping arrays. */
aboria_status aboria_pair_sum(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                              const double* params_host, int32_t nparams, const void* a, int32_t na,
                              void* y, int32_t ny);

/* Adjoint of aboria_pair_sum: given gy[n][ny] = dL/dy, writes gx[n][d] = dL/dx
 * and, for operators with per-particle variables, ga[n][na] = dL/da (ga may be
 * NULL to skip it), all in original order and overwritten.  It gathers over the
 * same cell list, or over its recorded neighbour list (no atomics):
 *   gx_k = sum_{i in P(k)} [ J1(k,i)^T gy_k + J2(i,k)^T gy_i ],
 * J1, J2 the Jacobians of the summand in its first and second position.  The
 * pair set is held fixed (the summands are differentiated where they are
 * smooth).  Errors as for aboria_pair_sum. */
aboria_status aboria_pair_sum_backward(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                       const double* params_host, int32_t nparams, const void* a,
                                       int32_t na, const void* gy, int32_t ny, void* gx, void* ga);

/* ---- time step (Section 3: eqs. (2)-(3), the velocity and position updates) ----
 *
 * Semi-implicit Euler step on the caller's arrays in original order, all
 * [n][d] in the cell list's dtype and overwritten in place (x, v):
 *   v_i <- v_i + dt f_i,  then  x_i <- x_i + dt v_i (with the new v_i),
 * where f is typically aboria_pair_sum of the exp-force operator (eq. (1), c
 * as its parameter) on cells built from the same x.  In periodic dimensions a
 * coordinate at or above hi moves down by the side L and one below lo moves up
 * by L (one image: a step must move a particle less than a side), and a result
 * that rounds onto hi becomes lo; non-periodic coordinates are not wrapped (a
 * particle that leaves the box is reported by the next build's domain check).
 * The cell list supplies n, d, dtype and each system's box; it is not changed
 * (rebuild it from the new x before the next force sum).  Errors: INVALID_ARG
 * for NULL or overlapping arrays, a non-finite dt or cells of another device. */
aboria_status aboria_integrate(aboria_ctx* ctx, const aboria_cells* cells, double dt, const void* f, void* x,
                               void* v);

/* The whole time step of the Section 3 example in one kernel: the force of
 * eq. (1) (op = ABORIA_OP_EXP_FORCE, params_host[0] = c) -- or the spring
 * force (ABORIA_OP_SPRING, k) -- of every particle by the box search over the
 * cells, followed at once by the update of aboria_integrate (velocity first,
 * then position, the same periodic wrap).  The force never leaves registers.
 * The cells must have been built from the positions the step starts from; the
 * search reads the cell list's exact snapshot of them.
 *   x_out = v_out = NULL: x and v ([n][d], the order the cells were built
 *     from) are updated in place; the result equals aboria_pair_sum followed by
 *     aboria_integrate bit for bit.
 *   x_out, v_out given (both [n][d]): the reordering container of Section
 *     2.2.1 -- the particle in cell-order slot s starts from the snapshot's
 *     position and from v[perm[s]], and its new position and velocity are
 *     written to x_out[s], v_out[s]: the outputs come out in cell order, equal to
 *     the in-place results permuted, and the next build from x_out starts from
 *     nearly sorted cell ids.  x is not read (may be NULL).  The cell list's
 *     permutation is left as it is, so per-particle arrays that must follow
 *     (ids, variables) are permuted with aboria_cells_reorder after this call.
 * Rebuild before the next step.  Errors: UNSUPPORTED for another operator;
 * INVALID_ARG for a parameter count other than one, a non-finite parameter or
 * dt, a missing or overlapping array, only one of x_out and v_out, cells of
 * another device. */
aboria_status aboria_md_step(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op, const double* params_host,
                             int32_t nparams, double dt, void* x, void* v, void* x_out, void* v_out);

/* Reordering container (Section 2.2.1, parallel insertion by reordering the
 * particles): permutes nbuf caller arrays -- each [n] rows of row_bytes_host[b]
 * bytes (a multiple of 4, at most 4 elements of the cell list's dtype), in the
 * particle order the cell list was built from -- in place into the cell
 * order, and makes that the cell list's particle order (its permutation
 * becomes the identity).  From then on the caller's arrays are in cell order:
 * every sum and step reads and writes them there, so outputs are written
 * contiguously, and the next build from the reordered positions starts from
 * nearly sorted cell ids.  Pass every per-particle array that must stay aligned
 * with x (positions, velocities, per-particle variables, ids).  The cell
 * list's own sorted copy and offsets are unchanged.  Errors: INVALID_ARG for
 * NULL, overlapping or oversized buffers, cells of another device. */
aboria_status aboria_cells_reorder(aboria_ctx* ctx, aboria_cells* cells, int32_t nbuf, void* const* bufs_host,
                                   const int32_t* row_bytes_host);

/* Forward sum and adjoint in one box search, for an upstream gradient gy known
 * before the forward (gy = 1 gives an energy E = sum_i e_i and its gradient, the
 * pattern of force fields): y as aboria_pair_sum, gx (and ga, may be NULL) as
 * aboria_pair_sum_backward for gy.  Each accepted pair is tested once.  Always
 * the lane-per-particle box search (no variant choice).  Errors as for the two
 * calls; no output may overlap an input or another output. */
aboria_status aboria_pair_sum_and_backward(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                           const double* params_host, int32_t nparams, const void* a, int32_t na,
                                           const void* gy, int32_t ny, void* y, void* gx, void* ga);

/* ---- recorded neighbour lists ---------------------------------------------------
 *
 * Records, for every particle of the cell list, its neighbour set P(i) (the
 * box search of Section 2.2.2 under the canonical predicate above) in
 * box-search order, in device memory owned by the cell list: up to `capacity`
 * entries per particle (0 = chosen from the densest system's density: its mean
 * neighbour count plus six standard deviations of a Poisson count, plus 8) and
 * each particle's full count.  Later aboria_pair_sum and
 * aboria_pair_sum_backward calls on these cells then evaluate recorded
 * (accepted) pairs only, adding the summands in the same order as the box
 * search, so their results equal the box-search results bit for bit.  A
 * particle with more neighbours than the capacity, and every particle after a
 * rebuild of the cells that was not followed by a new recording (a build
 * generation kept on the device decides, so graph replays stay consistent),
 * is summed by the box search instead.  The first call allocates
 * capacity * n * 4 + n * 4 bytes and cannot be captured; later calls reuse
 * that memory and can be captured (an explicit capacity above the allocated
 * one is INVALID_ARG, an automatic one is clamped to it).  Memory is released
 * with the cells.  Errors: INVALID_ARG for NULL cells, cells of another device
 * or capacity outside 0..4096; OUT_OF_MEMORY. */
aboria_status aboria_build_neighbours(aboria_ctx* ctx, aboria_cells* cells, int32_t capacity);
/* Entries per particle of the latest recorded list (0 if none). */
int32_t aboria_neighbour_capacity(const aboria_cells* cells);

/* Lists the ordered neighbour pairs (original indices) of the cell list:
 * pair p is (pi[p], pj[p]) for p < min(total, cap), in an unspecified order;
 * *total_host receives the pair count.  This call synchronises the stream
 * (it reads the count back) and allocates, so it cannot be captured.  It is
 * meant for verification of the pair set. */
aboria_status aboria_pair_list(aboria_ctx* ctx, const aboria_cells* cells, int64_t cap, uint32_t* pi,
                               uint32_t* pj, int64_t* total_host);

/* ---- dense kernel sum (Section 1 and 1.1: RBF and Gaussian processes) -------
 *
 * y[i] = sum_{j < n_source} K(xt_i, xs_j) w_j for i < n_target, over every
 * source (j = i included when the sets coincide).  xt[n_target][d],
 * xs[n_source][d], w[n_source], y[n_target] in dtype; d in 1..3.  Float32 inputs
 * accumulate in float32 with per-tile partial sums.  Errors: INVALID_ARG for an
 * unknown kernel, a kernel parameter (sigma or c) that is not positive, d
 * outside 1..3, NULL or overlapping arrays. */
aboria_status aboria_dense_sum(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                               const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                               const void* xt, int64_t n_source, const void* xs, const void* w, void* y);

/* aboria_dense_sum for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops and harnesses that forbid hipMalloc.
 * Same arguments, arithmetic and errors as aboria_dense_sum; the caller still
 * passes every input and y.  The split partial sums go to a fixed device array
 * of 16 MiB that the library holds on each GPU it runs on until the process
 * ends, instead of the context's grow-only scratch, so the call never calls
 * hipMalloc, hipFree or any allocating routine (its first call on a device
 * looks the array's address up once).  n_target may be at most 4,194,304
 * (float32) or 2,097,152 (float64): larger sizes return INVALID_ARG and launch
 * nothing.  Near that limit fewer source splits fit and the partial sums are
 * grouped differently from aboria_dense_sum (same tolerance, not the same
 * bits); below it the results are bit-identical.  Every call on one GPU shares
 * that GPU's array and each call overwrites every entry it reads, so nothing
 * needs clearing, but calls that overlap in time on one GPU (two streams or
 * two host threads) race on it: serialise them. */
aboria_status aboria_dense_sum_noalloc(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                       const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                                       const void* xt, int64_t n_source, const void* xs, const void* w, void* y);

/* Adjoint of aboria_dense_sum for L = sum_i gy_i y_i (gy[n_target]):
 *   gw[j]     = sum_i K(xt_i, xs_j) gy_i                       (K^T gy)
 *   gxt[i][:] = gy_i sum_j w_j 2 phi'(q_ij) (xt_i - xs_j)
 *   gxs[j][:] = w_j sum_i gy_i 2 phi'(q_ij) (xs_j - xt_i)
 * for K = phi(q), q = |xt_i - xs_j|^2.  When targets and sources are the same
 * points, dL/dx = gxt + gxs.  Each output may be NULL (not computed); all are
 * overwritten, in dtype, and must not overlap the inputs or each other.  gw and
 * gxs come from one pass over the pairs, gxt from a second.  Uses
 * the same grow-only scratch as the forward (a first call of a size must not
 * be captured).  Errors as for aboria_dense_sum. */
aboria_status aboria_dense_sum_backward(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                        const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                                        const void* xt, int64_t n_source, const void* xs, const void* w,
                                        const void* gy, void* gxt, void* gxs, void* gw);

/* ---- graphs ------------------------------------------------------------------
 * Captures the calls made on ctx between begin and end into one executable
 * HIP graph (rebuilds with an existing cell list, neighbour-list recordings
 * after the first, sums, adjoints and dense sums allocate nothing and can be
 * captured; a first build, a first neighbour list, aboria_pair_list and
 * aboria_sync cannot).  Launch replays it on the context's stream. */
aboria_status aboria_graph_capture_begin(aboria_ctx* ctx);
aboria_status aboria_graph_capture_end(aboria_ctx* ctx, aboria_graph** out);
aboria_status aboria_graph_launch(aboria_ctx* ctx, const aboria_graph* graph);
aboria_status aboria_graph_destroy(aboria_graph* graph);

/* ---- autotuning ---------------------------------------------------------------
 * Times the neighbour-sum kernel variants (work mapping and launch shape) for
 * this cell list and operator with HIP events on the context's stream, keeps
 * the fastest in the context's cache (keyed by d, dtype, operator, direction,
 * size and density buckets) and makes later sums on matching cell lists use
 * it.  gy == NULL tunes the forward sum, which writes out_scratch[n][ny];
 * otherwise it tunes the adjoint for that upstream gradient gy[n][ny], which
 * writes out_scratch[n][d] (ga is not computed).  a as for aboria_pair_sum.
 * *choice_host receives the chosen variant (may be NULL).  Synchronises the
 * stream; not capturable.  Errors as for aboria_pair_sum.
 *
 * Persistence: when the environment variable ABORIA_TUNE_CACHE names a file
 * at aboria_create, the context loads the choices stored there for this
 * device architecture, and every aboria_autotune, aboria_autotune_cells,
 * aboria_autotune_dense and aboria_autotune_build rewrites the file with the
 * context's choices (JSON, one entry per line,
 * variants by name; written to a temporary file and renamed).  Contexts that
 * tune concurrently with the same file keep the last writer's entries.
 * ABORIA_LOG=1 prints errors and tuning decisions to stderr. */
aboria_status aboria_autotune(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                              const double* params_host, int32_t nparams, const void* a, int32_t na,
                              const void* gy, int32_t ny, void* out_scratch, int32_t* choice_host);

/* Cell-size tuning: times a rebuild plus aboria_pair_sum (and, when gy is given,
 * aboria_pair_sum_backward for that upstream gradient) of op on grids of each
 * search reach (the boxes' reach when any entry of boxes_host[0].reach is set,
 * else 1, 2 and 3 in every dimension and, for d >= 2, {2, 1, 1} and {3, 1, 1},
 * skipping a reach that the boxes' explicit counts do not allow) whose
 * per-dimension cell counts are that reach's automatic ones (or the boxes'
 * explicit ones) scaled by 1, 0.85, 0.7 and 0.55 (rounded down, at least 1;
 * coarser cells are always valid, finer ones are not), each with its work
 * mapping tuned as by aboria_autotune (the tuned choices stay in ctx's cache).
 * boxes_out[nsys] receives the input boxes with the fastest grid's explicit
 * ncell and reach; *factor_host (may be NULL) the chosen scale.  Arguments as for
 * aboria_build_cells and aboria_autotune; allocates temporary cell lists and
 * synchronises, so it cannot be captured. */
aboria_status aboria_autotune_cells(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys, const aboria_box* boxes_host,
                                    const int64_t* offsets_host, const void* x, aboria_op op,
                                    const double* params_host, int32_t nparams, const void* a, int32_t na,
                                    const void* gy, int32_t ny, aboria_box* boxes_out, double* factor_host);

/* Dense-sum launch tuning (Sections 1 and 1.1, the kernel sums of
 * aboria_dense_sum): times the launch plans -- targets kept per lane (2, 4, or
 * for float 8) and the number of workgroups the source split aims for (1024,
 * 2048, 4096) -- of aboria_dense_sum (gy == NULL) or of
 * aboria_dense_sum_backward computing all three gradients (gy given) on the
 * caller's arrays, and makes later calls with the same direction, kernel,
 * dtype, d and size buckets (floor log2 of n_target and n_source) use the
 * fastest.  scratch receives the outputs: y[n_target] for the forward,
 * gxt[n_target][d] then gxs[n_source][d] then gw[n_source] (contiguous) for
 * the backward.  A plan changes the split of the source range, so results
 * move by rounding only.  *choice_host (may be NULL) receives the plan, named
 * by aboria_dense_plan_name.  Persisted like aboria_autotune's choices;
 * synchronises; not capturable.  Errors as for aboria_dense_sum, and
 * INVALID_ARG when there are no pairs to time. */
aboria_status aboria_autotune_dense(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                    const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                                    const void* xt, int64_t n_source, const void* xs, const void* w,
                                    const void* gy, void* scratch, int32_t* choice_host);
/* Name of a dense launch plan ("" when out of range); static storage. */
const char* aboria_dense_plan_name(int32_t plan);
/* Forces dense launch plan `plan` for later dense sums on ctx (-1: the tuned
 * choice, else plan 0); a float-only plan runs plan 0 in float64.
 * INVALID_ARG for an unknown plan. */
aboria_status aboria_set_dense_plan(aboria_ctx* ctx, int32_t plan);

/* Without tuning or a forced variant, a sum on a cell list whose systems all
 * have at most 2048 particles tests all pairs of each system at the minimum
 * image (the small-N switch: no cell search; with an explicit cell count of 1
 * per dimension the build is a single kernel as well); otherwise it replays
 * the recorded neighbour list if there is one, else it searches cells. */

/* Number of neighbour-sum variants, and a static description of one. */
int32_t aboria_variant_count(void);
const char* aboria_variant_name(int32_t variant);
/* Forces a variant for later sums on ctx (-1 = use the tuned / default one).
 * The recorded-mask variant's forward also stores, per particle and stencil
 * row, which candidates it accepted; its adjoint on the same cells (until they
 * are rebuilt) visits only those, and otherwise repeats the search.  The first
 * sum with it on a cell list allocates 2 * 3^(d-1) + 1 words per particle,
 * owned and freed with the cell list (so that first call cannot be captured);
 * INVALID_ARG if the list has m > 1.  Sums that overlap on one cell list with
 * this variant race on its record.  The half-stencil variant (Section 3's eq.
 * (1) forward with each unordered pair tested once, Newton's third law for the
 * pair test) uses the same record for the upper half of each stencil and
 * leaves it marked as not replayable; its adjoint is the plain lane kernel's;
 * it needs reach 1 in y and z and a grid of at least 2 m + 1 cells in x
 * (INVALID_ARG otherwise). */
aboria_status aboria_set_variant(aboria_ctx* ctx, int32_t variant);

/* The variant a sum on these cells with this operator would use now (forced,
 * tuned -- from this context's tuning or its persistent cache -- or the
 * untuned default), backward != 0 for the adjoint.  Launches nothing. */
aboria_status aboria_selected_variant(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op, int32_t backward,
                                      int32_t* variant_host);

/* Summand widths of an operator: ny for dimension d, and na. -1 if unknown. */
int32_t aboria_op_ny(aboria_op op, int32_t d);
int32_t aboria_op_na(aboria_op op);

#ifdef __cplusplus
}
#endif

#endif /* ABORIA_H */
