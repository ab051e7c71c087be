/*
 * oracle.c -- plain, slow CPU reference for the cell-list neighbour operators
 * and the dense kernel sum of Robinson & Bruna, "Particle-based and Meshless
 * Methods with Aboria" (arXiv:1704.08907).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * What it computes (paper citations by section / equation / listing):
 *   - The problem instance (Section 1): N points in a d-dimensional hypercube
 *     [lo, hi), each dimension periodic or not; operators defined only by the
 *     positions and per-particle variables.
 *   - The cell list (Section 2.2.1, "Aboria Level 1"): a square lattice of
 *     hypercube cells of width at least the cutoff (the worked example sets the
 *     width to r_cut, Section 3), each holding zero or more particles.  This
 *     file builds it twice: as cell ids + a stable counting sort (cell order,
 *     original index order inside a cell), and as the serial-insertion
 *     head/next linked list that Section 2.2.1 mentions as the second design.
 *   - The box search (Section 2.2.2, "Aboria Level 2"): candidates of particle
 *     i are the particles in i's cell and the adjacent cells.  A grid may also
 *     use cells narrower than the cutoff (reading R1 with reach m > 1); the
 *     search then takes every cell up to m cells away in each dimension.  The
 *     accepted pairs do not depend on the grid: the predicate R3 alone decides.
 *   - The radius-limited sum (Section 3, eq. (1) and the velocity-update
 *     listing): y_i = sum over j with 0 < |dx_ij| < r of f_ij, with dx_ij the
 *     shortest (minimum-image) vector r_j - r_i.  The norm(dx) > 0 condition
 *     of the listing excludes j = i and coincident points.
 *   - The dense global kernel sum of the RBF / Gaussian-process methods
 *     (Section 1 and Section 1.1): y_i = sum_j K(x_i, x_j) w_j over all j.
 *   - One time step of the Section 3 molecular-dynamics example: the
 *     velocity-update listing v_i += c sum_j (-exp(-|dx|) dx/|dx|) (eq. (1) in
 *     eq. (2)), then the position-update listing x_i += v_i (eq. (3)), with the
 *     step dt = 1 of the paper kept as a parameter.
 *
 * Readings the paper leaves open (each listed in the design notes):
 *   R1 cell count per dimension: n = floor(m L/r), then decreased while n > 1
 *      and L/n < (r + 16 u (|lo| + L)) / m, u the unit roundoff of the input
 *      precision, so that rounding in the cell assignment can never put the two
 *      points of a pair more than m cells apart.  m >= 1 is the search reach,
 *      given per dimension; m = 1 is the paper's lattice (cells at least one
 *      cutoff wide, searched with the adjacent cells).  An explicit count may
 *      not exceed this n.
 *   R2 cell of a coordinate: clamp(floor(fl(fl(x - lo) * fl(n / L))), 0, n-1);
 *      linear id = c0 + n0 (c1 + n1 c2); x == hi, x < lo or NaN is a domain
 *      error.
 *   R3 pair predicate, evaluated in the input precision P with this exact
 *      operation order: t_k = fl(x_jk - x_ik); dx_k = fl(t_k + s_k) with
 *      s_k in {-L, 0, +L} the periodic image shift; d2 = fma chain
 *      fma(dx2, dx2, fma(dx1, dx1, dx0*dx0)); pair iff 0 < d2 < fl(r*r).
 *   R4 summands are then evaluated in float64 from the P-rounded data.
 *   R5 operators: spring F_i = sum k (r - s) u/s with u = x_i - x_j; soft
 *      sphere e_i = 1/2 sum (1 - s/r)^2; the paper's eq. (1) force
 *      y_i = sum -c exp(-s) dx/s; a spring with per-particle resting lengths
 *      y_i = sum k (a_i + a_j - s) u/s (the DEM example of Section 1.1).
 *   R6 what a result is compared against.  Each output row gets two scales:
 *      S = the sum over the row's summands of their max-norm (the absolute-sum
 *      scale of a relative tolerance), and D = the sum over the row's summands
 *      of max_k sum_q |d f_k / d q| base_q, the summand's condition with respect
 *      to the quantities an evaluation in precision P forms by rounding: each
 *      displacement coordinate u_m (base |raw_m| + |u_m|, raw_m = x_jm - x_im
 *      the difference reading R3 rounds before the periodic shift is added),
 *      each coordinate of the upstream gradients a pair combines (gy_i - gy_j
 *      or gy_i + gy_j, base |gy_im| + |gy_jm|) and the per-particle variables
 *      (a_i + a_j, base |a_i| + |a_j|).  Each of these carries a rounding of
 *      at most u_P base_q, and the distance and the functions of it a few u_P
 *      relative (a perturbation of |u|), so a correct P evaluation differs
 *      from the exact summand by a few u_P D plus a few u_P |f|.  A row i
 *      passes at tolerance tol when |y_i - y*_i|_inf <= tol S_i + 16 u_P D_i;
 *      16 u_P is the same allowance the cell-count guard of R1 gives the
 *      rounding of a coordinate.  Near the cutoff k (r - s) -> 0 while its
 *      rounding does not; across a periodic face the displacement inherits the
 *      rounding of a coordinate up to L; and an adjoint summand g w_perp +
 *      gpar w_par with g ~ k r/s at a close pair amplifies the rounding of w
 *      by g: the D term carries exactly these, the S term everything else.
 *      The partial derivatives are forward differences of the float64 summand
 *      with the step 2^-20 base_q.
 *   R8 the multiquadric basis of the Section 1.1 RBF example, whose formula the
 *      paper does not print: Hardy's K(x, x') = sqrt(|x - x'|^2 + c^2), c > 0.
 *   R7 the periodic domain of the time step: after x += dt v, a coordinate at
 *      or above hi moves down by L, one below lo moves up by L (one image: a
 *      step moves a particle less than a box side), and a result that rounds
 *      onto hi becomes lo, so positions stay in the half-open box [lo, hi).
 *      Non-periodic coordinates are not wrapped.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID 1
#define OR_ERR_DOMAIN 2
#define OR_ERR_UNSUPPORTED 3
#define OR_ERR_NOMEM 4

#define OR_F32 0
#define OR_F64 1

#define OR_OP_COUNT 0
#define OR_OP_SPRING 1
#define OR_OP_SOFT_SPHERE 2
#define OR_OP_EXP_FORCE 3
#define OR_OP_DEM_SPRING 4

#define OR_ROUTE_BRUTE 0
#define OR_ROUTE_CELLS 1

typedef struct or_grid {
    int32_t d;
    int32_t dtype;
    int32_t periodic[3];
    int32_t n[3];
    double lo[3];
    double hi[3];
    double L[3];
    double inv_w[3];
    double r;
    double r2;
    int64_t ncells;
    int32_t reach[3]; /* m of reading R1 per dimension: cells searched on each side */
    int32_t pad;
} or_grid;

/* Round a double to the working precision P. */
static double to_p(int dtype, double v) { return dtype == OR_F32 ? (double)(float)v : v; }

static double unit_roundoff(int dtype) { return dtype == OR_F32 ? ldexp(1.0, -24) : ldexp(1.0, -53); }

/* ------------------------------------------------------------------------ */
/* Cell grid: readings R1 and R2 above.                                      */
/* ------------------------------------------------------------------------ */

int or_grid_init(or_grid* g, int32_t d, int32_t dtype, const double* lo, const double* hi,
                 const int32_t* periodic, double r, const int32_t* ncell_req, const int32_t* reach) {
    memset(g, 0, sizeof(*g));
    if (d < 1 || d > 3 || (dtype != OR_F32 && dtype != OR_F64)) return OR_ERR_INVALID;
    for (int k = 0; k < 3; ++k) {
        int32_t m = (reach && k < d) ? reach[k] : 1;
        if (m == 0) m = 1;
        if (m < 1 || m > 16) return OR_ERR_INVALID;
        g->reach[k] = m;
    }
    g->d = d;
    g->dtype = dtype;
    g->r = to_p(dtype, r);
    if (!(g->r > 0.0) || isinf(g->r)) return OR_ERR_INVALID;
    if (dtype == OR_F32) {
        float rf = (float)g->r;
        g->r2 = (double)(rf * rf);
    } else {
        g->r2 = g->r * g->r;
    }
    double u = unit_roundoff(dtype);
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
        g->n[k] = 1;
        g->inv_w[k] = 0.0;
    }
    for (int k = 0; k < d; ++k) {
        g->lo[k] = to_p(dtype, lo[k]);
        g->hi[k] = to_p(dtype, hi[k]);
        g->periodic[k] = periodic ? (periodic[k] != 0) : 0;
        if (!isfinite(g->lo[k]) || !isfinite(g->hi[k]) || !(g->hi[k] > g->lo[k])) return OR_ERR_INVALID;
        if (dtype == OR_F32)
            g->L[k] = (double)((float)g->hi[k] - (float)g->lo[k]);
        else
            g->L[k] = g->hi[k] - g->lo[k];
        double guard = g->r + 16.0 * u * (fabs(g->lo[k]) + g->L[k]);
        double q = floor((double)g->reach[k] * g->L[k] / g->r);
        int64_t nmax = q < 1.0 ? 1 : (q > 2147483647.0 ? 2147483647 : (int64_t)q);
        while (nmax > 1 && g->L[k] / (double)nmax < guard / (double)g->reach[k]) --nmax;
        int64_t nk = nmax;
        if (ncell_req && ncell_req[k] > 0) {
            if (ncell_req[k] > nmax) return OR_ERR_INVALID; /* cells narrower than the guard */
            nk = ncell_req[k];
        }
        /* a periodic dimension must hold at most one image of a point within r */
        if (g->periodic[k] && g->L[k] < 2.0 * guard) return OR_ERR_UNSUPPORTED;
        g->n[k] = (int32_t)nk;
        g->inv_w[k] = to_p(dtype, (double)nk / g->L[k]);
        total *= nk;
        if (total > 2147483647LL) return OR_ERR_UNSUPPORTED;
    }
    g->ncells = total;
    return OR_OK;
}

/* Cell coordinate of one P-rounded coordinate value; sets *bad on a domain error. */
static int32_t cell_coord(const or_grid* g, int k, double xk, int* bad) {
    if (!(xk >= g->lo[k]) || !(xk < g->hi[k])) *bad = 1;
    double q;
    if (g->dtype == OR_F32) {
        float t = (float)xk - (float)g->lo[k];
        q = (double)(t * (float)g->inv_w[k]);
    } else {
        double t = xk - g->lo[k];
        q = t * g->inv_w[k];
    }
    double f = floor(q);
    if (!(f >= 0.0)) return 0; /* negative or NaN */
    if (f > (double)(g->n[k] - 1)) return g->n[k] - 1;
    return (int32_t)f;
}

static uint32_t linear_id(const or_grid* g, const int32_t* c) {
    uint32_t id = (uint32_t)c[0];
    if (g->d > 1) id += (uint32_t)g->n[0] * (uint32_t)c[1];
    if (g->d > 2) id += (uint32_t)g->n[0] * (uint32_t)g->n[1] * (uint32_t)c[2];
    return id;
}

/* ids[i] = linear cell id of point i.  Returns OR_ERR_DOMAIN (ids still filled, clamped) on bad points. */
int or_cell_ids(const or_grid* g, int64_t n, const double* x, uint32_t* ids) {
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c[3] = {0, 0, 0};
        for (int k = 0; k < g->d; ++k) c[k] = cell_coord(g, k, x[i * g->d + k], &bad);
        ids[i] = linear_id(g, c);
    }
    return bad ? OR_ERR_DOMAIN : OR_OK;
}

/* Stable counting sort by cell id: perm[s] = original index of the s-th point in
 * cell order (original index order inside a cell); off[c] = number of points in
 * cells < c, for c = 0..ncells. */
int or_sort_cells(const or_grid* g, int64_t n, const uint32_t* ids, uint32_t* perm, uint32_t* off) {
    int64_t nc = g->ncells;
    int64_t* cnt = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    if (!cnt) return OR_ERR_NOMEM;
    for (int64_t i = 0; i < n; ++i) cnt[ids[i] + 1] += 1;
    for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    for (int64_t c = 0; c <= nc; ++c) off[c] = (uint32_t)cnt[c];
    for (int64_t i = 0; i < n; ++i) perm[cnt[ids[i]]++] = (uint32_t)i;
    free(cnt);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Pair predicate, reading R3.                                               */
/* ------------------------------------------------------------------------ */

static int pair_pred(const or_grid* g, const double* xi, const double* xj, const double* s) {
    if (g->dtype == OR_F32) {
        float dx[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < g->d; ++k) {
            float t = (float)xj[k] - (float)xi[k];
            dx[k] = t + (float)s[k];
        }
        float d2 = dx[0] * dx[0];
        if (g->d > 1) d2 = fmaf(dx[1], dx[1], d2);
        if (g->d > 2) d2 = fmaf(dx[2], dx[2], d2);
        return d2 > 0.0f && d2 < (float)g->r2;
    } else {
        double dx[3] = {0., 0., 0.};
        for (int k = 0; k < g->d; ++k) {
            double t = xj[k] - xi[k];
            dx[k] = t + s[k];
        }
        double d2 = dx[0] * dx[0];
        if (g->d > 1) d2 = fma(dx[1], dx[1], d2);
        if (g->d > 2) d2 = fma(dx[2], dx[2], d2);
        return d2 > 0.0 && d2 < g->r2;
    }
}

/* Minimum-image shift for the brute-force route: in each periodic dimension the
 * s in {0, -L, +L} (first one on ties) that minimises |fl(fl(x_j - x_i) + s)|. */
static void min_image_shift(const or_grid* g, const double* xi, const double* xj, double* s) {
    for (int k = 0; k < 3; ++k) s[k] = 0.0;
    for (int k = 0; k < g->d; ++k) {
        if (!g->periodic[k]) continue;
        const double cand[3] = {0.0, -g->L[k], g->L[k]};
        double best = INFINITY;
        for (int m = 0; m < 3; ++m) {
            double v;
            if (g->dtype == OR_F32) {
                float t = (float)xj[k] - (float)xi[k];
                v = fabs((double)(t + (float)cand[m]));
            } else {
                double t = xj[k] - xi[k];
                v = fabs(t + cand[m]);
            }
            if (v < best) {
                best = v;
                s[k] = cand[m];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour enumeration over the two routes.                                */
/* ------------------------------------------------------------------------ */

typedef void (*visit_fn)(void* ctx, int64_t i, int64_t j, const double* shift);

typedef struct {
    int32_t* head;
    int32_t* next;
} linked_cells;

/* Serial insertion into a head/next list, inserting from the last point to the
 * first so that a cell's list is traversed in increasing original index. */
static int build_linked(const or_grid* g, int64_t n, const double* x, linked_cells* lc) {
    lc->head = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->ncells);
    lc->next = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!lc->head || !lc->next) return OR_ERR_NOMEM;
    for (int64_t c = 0; c < g->ncells; ++c) lc->head[c] = -1;
    int bad = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        int32_t c[3] = {0, 0, 0};
        for (int k = 0; k < g->d; ++k) c[k] = cell_coord(g, k, x[i * g->d + k], &bad);
        uint32_t id = linear_id(g, c);
        lc->next[i] = lc->head[id];
        lc->head[id] = (int32_t)i;
    }
    return bad ? OR_ERR_DOMAIN : OR_OK;
}

static void free_linked(linked_cells* lc) {
    free(lc->head);
    free(lc->next);
}

/* Box search for point i: its cell and every cell up to m_k = reach[k] cells
 * away in dimension k (prod_k (2 m_k + 1) offsets; m = 1 in every dimension is
 * the paper's 3^d stencil).  A
 * periodic dimension wraps, and the wrap becomes the image shift of the
 * neighbour cell; a non-periodic dimension drops offsets outside the grid.  An
 * offset that would need a second wrap is dropped too: that image lies at
 * least one period L >= 2r from the first, so it can hold no pair. */
static void visit_cells(const or_grid* g, const linked_cells* lc, const double* x, int64_t i,
                        visit_fn fn, void* ctx) {
    int bad = 0;
    int32_t c[3] = {0, 0, 0};
    for (int k = 0; k < g->d; ++k) c[k] = cell_coord(g, k, x[i * g->d + k], &bad);
    int nstencil = 1;
    for (int k = 0; k < g->d; ++k) nstencil *= 2 * g->reach[k] + 1;
    for (int m = 0; m < nstencil; ++m) {
        int32_t cn[3] = {0, 0, 0};
        double s[3] = {0.0, 0.0, 0.0};
        int rest = m, skip = 0;
        for (int k = 0; k < g->d; ++k) {
            const int side = 2 * g->reach[k] + 1;
            int o = rest % side - g->reach[k];
            rest /= side;
            int32_t v = c[k] + o;
            if (v < 0) {
                if (!g->periodic[k]) { skip = 1; break; }
                v += g->n[k];
                s[k] = -g->L[k];
            } else if (v >= g->n[k]) {
                if (!g->periodic[k]) { skip = 1; break; }
                v -= g->n[k];
                s[k] = g->L[k];
            }
            if (v < 0 || v >= g->n[k]) { skip = 1; break; }
            cn[k] = v;
        }
        if (skip) continue;
        uint32_t id = linear_id(g, cn);
        for (int32_t j = lc->head[id]; j >= 0; j = lc->next[j]) {
            if (pair_pred(g, x + i * g->d, x + (int64_t)j * g->d, s)) fn(ctx, i, j, s);
        }
    }
}

static void visit_brute(const or_grid* g, int64_t n, const double* x, int64_t i, visit_fn fn, void* ctx) {
    for (int64_t j = 0; j < n; ++j) {
        double s[3];
        min_image_shift(g, x + i * g->d, x + j * g->d, s);
        if (pair_pred(g, x + i * g->d, x + j * g->d, s)) fn(ctx, i, j, s);
    }
}

/* Visit the accepted neighbours of each requested row by the chosen route.
 * With nthreads > 1 the rows are split into nthreads contiguous blocks, one
 * POSIX thread each; ctxs[t] is thread t's own context (row_begin and fn only
 * ever see the context of the thread that runs the row), so the threads share
 * nothing they write.  Every row is computed exactly as in one thread. */
typedef struct {
    const or_grid* g;
    int route;
    int64_t n;
    const double* x;
    const int64_t* rows;
    const linked_cells* lc;
    visit_fn fn;
    void (*row_begin)(void*, int64_t, int64_t);
    void* ctx;
    int64_t r0, r1;
} rows_job;

static void* rows_worker(void* vjob) {
    rows_job* J = (rows_job*)vjob;
    for (int64_t r = J->r0; r < J->r1; ++r) {
        int64_t i = J->rows ? J->rows[r] : r;
        if (i < 0 || i >= J->n) continue;
        if (J->row_begin) J->row_begin(J->ctx, r, i);
        if (J->route == OR_ROUTE_CELLS)
            visit_cells(J->g, J->lc, J->x, i, J->fn, J->ctx);
        else
            visit_brute(J->g, J->n, J->x, i, J->fn, J->ctx);
    }
    return NULL;
}

#define OR_MAX_THREADS 256

static int for_rows(const or_grid* g, int route, int64_t n, const double* x, int64_t nrows,
                    const int64_t* rows, visit_fn fn, void (*row_begin)(void*, int64_t, int64_t), void** ctxs,
                    int nthreads) {
    linked_cells lc = {0, 0};
    int st = OR_OK;
    if (route == OR_ROUTE_CELLS) {
        st = build_linked(g, n, x, &lc);
        if (st == OR_ERR_NOMEM) { free_linked(&lc); return st; }
    }
    int64_t m = rows ? nrows : n;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > OR_MAX_THREADS) nthreads = OR_MAX_THREADS;
    if ((int64_t)nthreads > m) nthreads = m > 0 ? (int)m : 1;
    rows_job jobs[OR_MAX_THREADS];
    pthread_t tid[OR_MAX_THREADS];
    int started[OR_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        rows_job J = {g, route, n, x, rows, &lc, fn, row_begin, ctxs[t], m * t / nthreads, m * (t + 1) / nthreads};
        jobs[t] = J;
        started[t] = 0;
    }
    for (int t = 1; t < nthreads; ++t) started[t] = pthread_create(&tid[t], NULL, rows_worker, &jobs[t]) == 0;
    rows_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) {
        if (started[t])
            pthread_join(tid[t], NULL);
        else
            rows_worker(&jobs[t]); /* no thread available: run the block here */
    }
    if (route == OR_ROUTE_CELLS) free_linked(&lc);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Pair lists.                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t count, cap;
    uint32_t* pi;
    uint32_t* pj;
} pair_list_ctx;

static void add_pair(void* vctx, int64_t i, int64_t j, const double* s) {
    (void)s;
    pair_list_ctx* c = (pair_list_ctx*)vctx;
    if (c->count < c->cap) {
        c->pi[c->count] = (uint32_t)i;
        c->pj[c->count] = (uint32_t)j;
    }
    c->count += 1;
}

/* All ordered pairs (i, j) by the chosen route; returns the pair count (which
 * may exceed cap: only the first cap are stored), or -1 on an allocation failure. */
int64_t or_pairs(const or_grid* g, int32_t route, int64_t n, const double* x, int64_t cap, uint32_t* pi,
                 uint32_t* pj) {
    pair_list_ctx c = {0, cap, pi, pj};
    void* ctxs[1] = {&c};
    int st = for_rows(g, route, n, x, 0, NULL, add_pair, NULL, ctxs, 1);
    if (st == OR_ERR_NOMEM) return -1;
    return c.count;
}

/* ------------------------------------------------------------------------ */
/* Operators (reading R5), summed in float64 (reading R4).                    */
/* ------------------------------------------------------------------------ */

int32_t or_op_ny(int32_t op, int32_t d) {
    switch (op) {
        case OR_OP_COUNT: return 1;
        case OR_OP_SPRING: return d;
        case OR_OP_SOFT_SPHERE: return 1;
        case OR_OP_EXP_FORCE: return d;
        case OR_OP_DEM_SPRING: return d;
        default: return -1;
    }
}

int32_t or_op_na(int32_t op) { return op == OR_OP_DEM_SPRING ? 1 : 0; }

/* u = x_i - x_j - shift in float64 (x_j + shift is the image of j nearest i). */
static double pair_u(const or_grid* g, const double* xi, const double* xj, const double* s, double* u) {
    double s2 = 0.0;
    for (int k = 0; k < 3; ++k) u[k] = 0.0;
    for (int k = 0; k < g->d; ++k) {
        u[k] = (xi[k] - xj[k]) - s[k];
        s2 += u[k] * u[k];
    }
    return sqrt(s2);
}

/* Radial profile g(s) of the vector operators f = g(s) u, and its derivative. */
static double radial_g(int op, const double* prm, double r, double s, double ai, double aj, double* dg) {
    switch (op) {
        case OR_OP_SPRING: {
            double k = prm[0];
            *dg = -k * r / (s * s);
            return k * (r - s) / s;
        }
        case OR_OP_EXP_FORCE: {
            /* eq. (1): f_ij = -c exp(-|dx|) dx/|dx| with dx = -u, i.e. g = c exp(-s)/s */
            double c = prm[0];
            double e = exp(-s);
            *dg = -c * e * (s + 1.0) / (s * s);
            return c * e / s;
        }
        case OR_OP_DEM_SPRING: {
            double k = prm[0];
            double rest = ai + aj;
            *dg = -k * rest / (s * s);
            return k * (rest - s) / s;
        }
        default:
            *dg = 0.0;
            return 0.0;
    }
}

/* Forward summand of one ordered pair, u = x_i - (x_j + shift), in float64. */
static void fwd_term(const or_grid* g, int op, const double* prm, const double* u, double ai, double aj,
                     double* t) {
    double s2 = 0.0;
    for (int k = 0; k < g->d; ++k) s2 += u[k] * u[k];
    double dist = sqrt(s2);
    switch (op) {
        case OR_OP_COUNT:
            t[0] = 1.0;
            break;
        case OR_OP_SOFT_SPHERE: {
            double v = 1.0 - dist / g->r;
            t[0] = 0.5 * v * v;
            break;
        }
        default: {
            double dg;
            double gv = radial_g(op, prm, g->r, dist, ai, aj, &dg);
            for (int k = 0; k < g->d; ++k) t[k] = gv * u[k];
            break;
        }
    }
}

/* Relative forward-difference step of the condition D of reading R6. */
#define OR_COND_EPS 0x1p-20

/* raw = x_j - x_i (the difference reading R3 rounds before the shift). */
static void pair_raw(const or_grid* g, const double* xi, const double* xj, double* raw) {
    for (int k = 0; k < 3; ++k) raw[k] = 0.0;
    for (int k = 0; k < g->d; ++k) raw[k] = xj[k] - xi[k];
}

typedef struct {
    const or_grid* g;
    int op;
    const double* prm;
    const double* x;
    const double* a;
    int ny;
    double* y;      /* [rows][ny] */
    double* scale;  /* [rows] or NULL */
    double* cond;   /* [rows] or NULL */
    double* yrow;
    double* srow;
    double* crow;
} sum_ctx;

static void sum_begin(void* vctx, int64_t r, int64_t i) {
    (void)i;
    sum_ctx* c = (sum_ctx*)vctx;
    c->yrow = c->y + r * c->ny;
    c->srow = c->scale ? c->scale + r : NULL;
    c->crow = c->cond ? c->cond + r : NULL;
    for (int m = 0; m < c->ny; ++m) c->yrow[m] = 0.0;
    if (c->srow) *c->srow = 0.0;
    if (c->crow) *c->crow = 0.0;
}

static void sum_pair(void* vctx, int64_t i, int64_t j, const double* s) {
    sum_ctx* c = (sum_ctx*)vctx;
    const or_grid* g = c->g;
    double u[3], t[3] = {0, 0, 0};
    pair_u(g, c->x + i * g->d, c->x + j * g->d, s, u);
    double ai = c->a ? c->a[i] : 0.0, aj = c->a ? c->a[j] : 0.0;
    fwd_term(g, c->op, c->prm, u, ai, aj, t);
    for (int k = 0; k < c->ny; ++k) c->yrow[k] += t[k];
    if (c->srow) {
        double mx = 0.0;
        for (int k = 0; k < c->ny; ++k)
            if (fabs(t[k]) > mx) mx = fabs(t[k]);
        *c->srow += mx;
    }
    if (c->crow) {
        /* D: sum over the formed quantities q of |df/dq| base_q, max over outputs:
         * the displacement coordinates (base |raw_m| + |u_m|) and the sum of the
         * per-particle variables (base |a_i| + |a_j|) */
        double raw[3], acc[3] = {0, 0, 0};
        pair_raw(g, c->x + i * g->d, c->x + j * g->d, raw);
        for (int m = 0; m < g->d; ++m) {
            double base = fabs(raw[m]) + fabs(u[m]);
            double up[3] = {u[0], u[1], u[2]}, tp[3] = {0, 0, 0};
            up[m] += OR_COND_EPS * base;
            fwd_term(g, c->op, c->prm, up, ai, aj, tp);
            for (int k = 0; k < c->ny; ++k) acc[k] += fabs(tp[k] - t[k]) / OR_COND_EPS;
        }
        if (c->a) {
            double tp[3] = {0, 0, 0};
            fwd_term(g, c->op, c->prm, u, ai + OR_COND_EPS * (fabs(ai) + fabs(aj)), aj, tp);
            for (int k = 0; k < c->ny; ++k) acc[k] += fabs(tp[k] - t[k]) / OR_COND_EPS;
        }
        double mx = 0.0;
        for (int k = 0; k < c->ny; ++k)
            if (acc[k] > mx) mx = acc[k];
        *c->crow += mx;
    }
}

/* y[row][ny] = sum over the accepted neighbours of the requested rows (all rows
 * if rows == NULL).  scale[row] = S and cond[row] = D of reading R6; either may
 * be NULL, and with both NULL nothing beyond the plain sum is computed.  a is
 * [n] or NULL.  nthreads >= 1 threads split the rows. */
int or_pair_sum(const or_grid* g, int32_t route, int32_t op, const double* prm, int64_t n, const double* x,
                const double* a, int64_t nrows, const int64_t* rows, double* y, double* scale, double* cond,
                int32_t nthreads) {
    int ny = or_op_ny(op, g->d);
    if (ny < 0) return OR_ERR_INVALID;
    if (or_op_na(op) && !a) return OR_ERR_INVALID;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > OR_MAX_THREADS) nthreads = OR_MAX_THREADS;
    sum_ctx c[OR_MAX_THREADS];
    void* ctxs[OR_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        sum_ctx ct = {g, op, prm, x, a, ny, y, scale, cond, NULL, NULL, NULL};
        c[t] = ct;
        ctxs[t] = &c[t];
    }
    int st = for_rows(g, route, n, x, nrows, rows, sum_pair, sum_begin, ctxs, nthreads);
    return st == OR_ERR_NOMEM ? st : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: gradient of L = sum_i gy_i . y_i with respect to x (and a).      */
/* For f(x_a, x_b) = g(s) u_ab the Jacobian in x_a is g I + (g'/s) u u^T and  */
/* the Jacobian in x_b is its negative, so over the symmetric pair set        */
/*   gx_k = sum_i [ g w + (g'/s)(u_ki . w) u_ki ],  w = gy_k - gy_i.          */
/* For the soft sphere e_a = 1/2 sum_b phi(s_ab), phi = (1 - s/r)^2:          */
/*   gx_k = sum_i 1/2 (gy_k + gy_i) phi'(s) u_ki/s.                           */
/* For the per-particle resting length: ga_k = sum_i k (gy_k - gy_i).u_ki/s.  */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_grid* g;
    int op;
    const double* prm;
    const double* x;
    const double* a;
    const double* gy;
    int ny;
    double *gx, *ga, *sx, *cx, *sa, *ca;             /* outputs, [rows][d] / [rows] */
    double *gxrow, *garow, *sxrow, *cxrow, *sarow, *carow;
} bwd_ctx;

static void bwd_begin(void* vctx, int64_t r, int64_t i) {
    (void)i;
    bwd_ctx* c = (bwd_ctx*)vctx;
    c->gxrow = c->gx + r * c->g->d;
    c->garow = c->ga ? c->ga + r : NULL;
    c->sxrow = c->sx ? c->sx + r : NULL;
    c->cxrow = c->cx ? c->cx + r : NULL;
    c->sarow = c->sa ? c->sa + r : NULL;
    c->carow = c->ca ? c->ca + r : NULL;
    for (int k = 0; k < c->g->d; ++k) c->gxrow[k] = 0.0;
    if (c->garow) *c->garow = 0.0;
    if (c->sxrow) *c->sxrow = 0.0;
    if (c->cxrow) *c->cxrow = 0.0;
    if (c->sarow) *c->sarow = 0.0;
    if (c->carow) *c->carow = 0.0;
}

/* Adjoint contribution of the ordered pair (k, i), u = x_k - (x_i + shift). */
static void bwd_term(const or_grid* g, int op, const double* prm, const double* u, double ak, double ai,
                     const double* gyk, const double* gyi, double* gx, double* ga) {
    int d = g->d;
    double s2 = 0.0;
    for (int m = 0; m < d; ++m) s2 += u[m] * u[m];
    double dist = sqrt(s2);
    for (int m = 0; m < 3; ++m) gx[m] = 0.0;
    *ga = 0.0;
    if (op == OR_OP_COUNT) return;
    if (op == OR_OP_SOFT_SPHERE) {
        double dphi = -(2.0 / g->r) * (1.0 - dist / g->r);
        double coef = 0.5 * (gyk[0] + gyi[0]) * dphi / dist;
        for (int m = 0; m < d; ++m) gx[m] = coef * u[m];
        return;
    }
    double dg;
    double gv = radial_g(op, prm, g->r, dist, ak, ai, &dg);
    double w[3] = {0, 0, 0};
    double uw = 0.0;
    for (int m = 0; m < d; ++m) {
        w[m] = gyk[m] - gyi[m];
        uw += u[m] * w[m];
    }
    for (int m = 0; m < d; ++m) gx[m] = gv * w[m] + (dg / dist) * uw * u[m];
    if (op == OR_OP_DEM_SPRING) *ga = prm[0] * uw / dist;
}

static void bwd_pair(void* vctx, int64_t k, int64_t i, const double* s) {
    bwd_ctx* c = (bwd_ctx*)vctx;
    const or_grid* g = c->g;
    int d = g->d;
    double u[3], t[3], ta;
    pair_u(g, c->x + k * d, c->x + i * d, s, u);
    const double* gyk = c->gy + k * c->ny;
    const double* gyi = c->gy + i * c->ny;
    double ak = c->a ? c->a[k] : 0.0, ai = c->a ? c->a[i] : 0.0;
    bwd_term(g, c->op, c->prm, u, ak, ai, gyk, gyi, t, &ta);
    for (int m = 0; m < d; ++m) c->gxrow[m] += t[m];
    if (c->garow) *c->garow += ta;
    if (c->sxrow) {
        double mx = 0.0;
        for (int m = 0; m < d; ++m)
            if (fabs(t[m]) > mx) mx = fabs(t[m]);
        *c->sxrow += mx;
    }
    if (c->sarow) *c->sarow += fabs(ta);
    if (c->cxrow || c->carow) {
        /* D over the displacement coordinates, the coordinates of the upstream
         * gradients the pair combines (base |gy_k,m| + |gy_i,m|: gy_k - gy_i or
         * gy_k + gy_i is formed in P) and the per-particle variables */
        double raw[3], acc[3] = {0, 0, 0}, acca = 0.0;
        double tp[3], tap;
        pair_raw(g, c->x + k * d, c->x + i * d, raw);
        for (int m = 0; m < d; ++m) {
            double base = fabs(raw[m]) + fabs(u[m]);
            double up[3] = {u[0], u[1], u[2]};
            up[m] += OR_COND_EPS * base;
            bwd_term(g, c->op, c->prm, up, ak, ai, gyk, gyi, tp, &tap);
            for (int q = 0; q < d; ++q) acc[q] += fabs(tp[q] - t[q]) / OR_COND_EPS;
            acca += fabs(tap - ta) / OR_COND_EPS;
        }
        for (int m = 0; m < c->ny; ++m) {
            double gp[3] = {0, 0, 0};
            for (int q = 0; q < c->ny; ++q) gp[q] = gyk[q];
            gp[m] += OR_COND_EPS * (fabs(gyk[m]) + fabs(gyi[m]));
            bwd_term(g, c->op, c->prm, u, ak, ai, gp, gyi, tp, &tap);
            for (int q = 0; q < d; ++q) acc[q] += fabs(tp[q] - t[q]) / OR_COND_EPS;
            acca += fabs(tap - ta) / OR_COND_EPS;
        }
        if (c->a) {
            bwd_term(g, c->op, c->prm, u, ak + OR_COND_EPS * (fabs(ak) + fabs(ai)), ai, gyk, gyi, tp, &tap);
            for (int q = 0; q < d; ++q) acc[q] += fabs(tp[q] - t[q]) / OR_COND_EPS;
            acca += fabs(tap - ta) / OR_COND_EPS;
        }
        if (c->cxrow) {
            double mx = 0.0;
            for (int q = 0; q < d; ++q)
                if (acc[q] > mx) mx = acc[q];
            *c->cxrow += mx;
        }
        if (c->carow) *c->carow += acca;
    }
}

/* gx[row][d], ga[row] (DEM spring only, else may be NULL); S and D of reading
 * R6 for gx (scale_x, cond_x) and ga (scale_a, cond_a), each may be NULL.  gy
 * is [n][ny] in original order.  nthreads >= 1 threads split the rows. */
int or_pair_sum_backward(const or_grid* g, int32_t route, int32_t op, const double* prm, int64_t n,
                         const double* x, const double* a, const double* gy, int64_t nrows, const int64_t* rows,
                         double* gx, double* ga, double* scale_x, double* cond_x, double* scale_a, double* cond_a,
                         int32_t nthreads) {
    int ny = or_op_ny(op, g->d);
    if (ny < 0) return OR_ERR_INVALID;
    if (or_op_na(op) && !a) return OR_ERR_INVALID;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > OR_MAX_THREADS) nthreads = OR_MAX_THREADS;
    bwd_ctx c[OR_MAX_THREADS];
    void* ctxs[OR_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        bwd_ctx ct = {g, op, prm, x, a, gy, ny, gx, ga, scale_x, cond_x, scale_a, cond_a,
                      NULL, NULL, NULL, NULL, NULL, NULL};
        c[t] = ct;
        ctxs[t] = &c[t];
    }
    int st = for_rows(g, route, n, x, nrows, rows, bwd_pair, bwd_begin, ctxs, nthreads);
    return st == OR_ERR_NOMEM ? st : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local central finite differences of L = sum_i gy_i . y_i.                 */
/* The pairs of point k are taken at the unperturbed positions (canonical     */
/* predicate), then L's dependence on coordinate (k, m) -- or on a_k -- is    */
/* evaluated in float64 at +h and -h:                                          */
/*   L_k = sum_{i in P(k)} [ gy_k . f(x_k, x_i) + gy_i . f(x_i, x_k) ].        */
/* coords[q] < n*d selects x[k][m] with q = k*d + m; coords[q] >= n*d selects  */
/* a[coords[q] - n*d].                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t count, cap;
    int64_t* j;
    double* s;
} nb_list;

static void nb_add(void* vctx, int64_t i, int64_t j, const double* s) {
    (void)i;
    nb_list* L = (nb_list*)vctx;
    if (L->count < L->cap) {
        L->j[L->count] = j;
        for (int k = 0; k < 3; ++k) L->s[L->count * 3 + k] = s[k];
    }
    L->count += 1;
}

/* one ordered-pair summand f(x_a, x_b) with u = xa - xb - s (float64) dotted with gya */
static double pair_term_dot(const or_grid* g, int op, const double* prm, const double* xa, const double* xb,
                            const double* s, double aa, double ab, const double* gya) {
    double u[3];
    double dist = pair_u(g, xa, xb, s, u);
    if (op == OR_OP_COUNT) return gya[0];
    if (op == OR_OP_SOFT_SPHERE) {
        double v = 1.0 - dist / g->r;
        return gya[0] * 0.5 * v * v;
    }
    double dg;
    double gv = radial_g(op, prm, g->r, dist, aa, ab, &dg);
    double acc = 0.0;
    for (int m = 0; m < g->d; ++m) acc += gya[m] * gv * u[m];
    return acc;
}

int or_fd_grad(const or_grid* g, int32_t op, const double* prm, int64_t n, const double* x, const double* a,
               const double* gy, int64_t ncoord, const int64_t* coords, double h, double* out) {
    int d = g->d;
    int ny = or_op_ny(op, d);
    if (ny < 0) return OR_ERR_INVALID;
    linked_cells lc = {0, 0};
    if (build_linked(g, n, x, &lc) == OR_ERR_NOMEM) { free_linked(&lc); return OR_ERR_NOMEM; }
    nb_list nb = {0, 0, NULL, NULL};
    nb.cap = 4096;
    nb.j = (int64_t*)malloc(sizeof(int64_t) * nb.cap);
    nb.s = (double*)malloc(sizeof(double) * 3 * nb.cap);
    int st = OR_OK;
    for (int64_t q = 0; q < ncoord && st == OR_OK; ++q) {
        int64_t c = coords[q];
        int is_a = c >= n * d;
        int64_t k = is_a ? c - n * d : c / d;
        int m = is_a ? -1 : (int)(c % d);
        nb.count = 0;
        visit_cells(g, &lc, x, k, nb_add, &nb);
        if (nb.count > nb.cap) { st = OR_ERR_NOMEM; break; }
        double val[2];
        for (int side = 0; side < 2; ++side) {
            double xk[3] = {0, 0, 0};
            for (int t = 0; t < d; ++t) xk[t] = x[k * d + t];
            double ak = a ? a[k] : 0.0;
            double delta = side == 0 ? h : -h;
            if (is_a) ak += delta; else xk[m] += delta;
            double acc = 0.0;
            for (int64_t p = 0; p < nb.count; ++p) {
                int64_t i = nb.j[p];
                const double* s = nb.s + p * 3;
                double ai = a ? a[i] : 0.0;
                double sneg[3] = {-s[0], -s[1], -s[2]};
                acc += pair_term_dot(g, op, prm, xk, x + i * d, s, ak, ai, gy + k * ny);
                acc += pair_term_dot(g, op, prm, x + i * d, xk, sneg, ai, ak, gy + i * ny);
            }
            val[side] = acc;
        }
        out[q] = (val[0] - val[1]) / (2.0 * h);
    }
    free(nb.j);
    free(nb.s);
    free_linked(&lc);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Dense Gaussian kernel sum (Section 1 / 1.1, RBF and Gaussian processes):  */
/*   y_i = sum_j exp(-|x_i - x_j|^2 / (2 sigma^2)) w_j over every source j,   */
/* j = i included; float64 from the given (P-rounded) inputs.  scale[row] =   */
/* sum_j |K_ij w_j|.                                                          */
/* ------------------------------------------------------------------------ */

int or_dense_gauss(int32_t d, int64_t nt, const double* xt, int64_t ns, const double* xs, const double* w,
                   double sigma, int64_t nrows, const int64_t* rows, double* y, double* scale) {
    if (d < 1 || d > 3 || !(sigma > 0.0)) return OR_ERR_INVALID;
    double inv = 1.0 / (2.0 * sigma * sigma);
    int64_t m = rows ? nrows : nt;
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        double acc = 0.0, sc = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = xt[i * d + k] - xs[j * d + k];
                d2 += t * t;
            }
            double term = exp(-d2 * inv) * w[j];
            acc += term;
            sc += fabs(term);
        }
        y[r] = acc;
        if (scale) scale[r] = sc;
    }
    return OR_OK;
}

/* Number of ordered pairs that the float64 predicate 0 < |u| < r would classify
 * differently from the canonical predicate in precision P (informational). */
int64_t or_tie_band(const or_grid* g, int64_t n, const double* x) {
    linked_cells lc = {0, 0};
    if (build_linked(g, n, x, &lc) == OR_ERR_NOMEM) { free_linked(&lc); return -1; }
    int64_t diff = 0;
    int d = g->d;
    for (int64_t i = 0; i < n; ++i) {
        int bad = 0;
        int32_t c[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) c[k] = cell_coord(g, k, x[i * d + k], &bad);
        int nst = 1;
        for (int k = 0; k < d; ++k) nst *= 3;
        for (int mm = 0; mm < nst; ++mm) {
            int32_t cn[3] = {0, 0, 0};
            double s[3] = {0, 0, 0};
            int rest = mm, skip = 0;
            for (int k = 0; k < d; ++k) {
                int o = rest % 3 - 1;
                rest /= 3;
                int32_t v = c[k] + o;
                if (v < 0) { if (!g->periodic[k]) { skip = 1; break; } v += g->n[k]; s[k] = -g->L[k]; }
                else if (v >= g->n[k]) { if (!g->periodic[k]) { skip = 1; break; } v -= g->n[k]; s[k] = g->L[k]; }
                cn[k] = v;
            }
            if (skip) continue;
            for (int32_t j = lc.head[linear_id(g, cn)]; j >= 0; j = lc.next[j]) {
                double u[3];
                double dist = pair_u(g, x + i * d, x + (int64_t)j * d, s, u);
                int p64 = dist > 0.0 && dist < g->r;
                int pp = pair_pred(g, x + i * d, x + (int64_t)j * d, s);
                if (p64 != pp) ++diff;
            }
        }
    }
    free_linked(&lc);
    return diff;
}

/* ------------------------------------------------------------------------ */
/* One step of the Section 3 example (eqs. (1)-(3) and the two update        */
/* listings), in the paper's order: S_i = sum_j -exp(-|dx_ij|) dx_ij/|dx_ij| */
/* over the box search (the force of eq. (1) without its constant), then     */
/* v_i += dt (c S_i), then x_i += dt v_i with the new velocity, then the     */
/* periodic wrap of reading R7.  x and v are [n][d], overwritten; x must hold */
/* P-rounded positions inside the box.  scale_v and cond_v (each may be NULL) */
/* are S and D of reading R6 for the velocity change dt c S_i.               */
/* ------------------------------------------------------------------------ */

int or_md_step(const or_grid* g, int32_t route, double c, double dt, int64_t n, double* x, double* v,
               double* scale_v, double* cond_v) {
    int d = g->d;
    double one[4] = {1.0, 0.0, 0.0, 0.0};
    size_t nn = (size_t)(n > 0 ? n : 1);
    double* S = (double*)calloc(nn * (size_t)d, sizeof(double));
    double* sc = (double*)calloc(nn, sizeof(double));
    double* cd = (double*)calloc(nn, sizeof(double));
    if (!S || !sc || !cd) { free(S); free(sc); free(cd); return OR_ERR_NOMEM; }
    int st = or_pair_sum(g, route, OR_OP_EXP_FORCE, one, n, x, NULL, 0, NULL, S, sc, cd, 1);
    if (st != OR_OK) { free(S); free(sc); free(cd); return st; }
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) {
            double vk = v[i * d + k] + dt * (c * S[i * d + k]);
            double xk = x[i * d + k] + dt * vk;
            if (g->periodic[k]) {
                if (xk >= g->hi[k]) xk -= g->L[k];
                else if (xk < g->lo[k]) xk += g->L[k];
                if (xk >= g->hi[k]) xk = g->lo[k];
            }
            v[i * d + k] = vk;
            x[i * d + k] = xk;
        }
        if (scale_v) scale_v[i] = fabs(dt * c) * sc[i];
        if (cond_v) cond_v[i] = fabs(dt * c) * cd[i];
    }
    free(S);
    free(sc);
    free(cd);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense kernel sums with a choice of radial kernel (Section 1.1: Gaussian   */
/* basis of the Kansa example, multiquadric basis of the RBF example, read   */
/* as R8), and their adjoint.  K(a, b) = phi(|a - b|^2):                      */
/*   Gaussian      phi(q) = exp(-q / (2 s^2)),   prm = s (sigma)              */
/*   multiquadric  phi(q) = sqrt(q + c^2),       prm = c                      */
/* y_i = sum_j K(xt_i, xs_j) w_j over every source (j = i included).  For     */
/* L = sum_i gy_i y_i:                                                         */
/*   dL/dw_j   = sum_i K(xt_i, xs_j) gy_i                                      */
/*   dL/dxt_i  = gy_i sum_j w_j 2 phi'(q_ij) (xt_i - xs_j)                     */
/*   dL/dxs_j  = w_j sum_i gy_i 2 phi'(q_ij) (xs_j - xt_i)                     */
/* (the gradient of phi(|a - b|^2) in a is 2 phi'(q)(a - b), and in b its     */
/* negative).  All in float64 from the given inputs; the scales are the sums */
/* of the summands' magnitudes.                                               */
/* ------------------------------------------------------------------------ */

#define OR_K_GAUSSIAN 0
#define OR_K_MULTIQUADRIC 1

static double kern_phi(int kind, double prm, double q) {
    return kind == OR_K_GAUSSIAN ? exp(-q / (2.0 * prm * prm)) : sqrt(q + prm * prm);
}

/* 2 phi'(q) */
static double kern_2dphi(int kind, double prm, double q) {
    return kind == OR_K_GAUSSIAN ? -exp(-q / (2.0 * prm * prm)) / (prm * prm) : 1.0 / sqrt(q + prm * prm);
}

static int kern_ok(int kind, double prm) {
    return (kind == OR_K_GAUSSIAN || kind == OR_K_MULTIQUADRIC) && prm > 0.0 && isfinite(prm);
}

static double sqdist(int d, const double* a, const double* b) {
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        q += t * t;
    }
    return q;
}

int or_dense_sum(int32_t kind, double prm, int32_t d, int64_t nt, const double* xt, int64_t ns, const double* xs,
                 const double* w, double* y, double* scale) {
    if (d < 1 || d > 3 || !kern_ok(kind, prm)) return OR_ERR_INVALID;
    for (int64_t i = 0; i < nt; ++i) {
        double acc = 0.0, sc = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double term = kern_phi(kind, prm, sqdist(d, xt + i * d, xs + j * d)) * w[j];
            acc += term;
            sc += fabs(term);
        }
        y[i] = acc;
        if (scale) scale[i] = sc;
    }
    return OR_OK;
}

/* gxt[nt][d], gxs[ns][d], gw[ns] (each may be NULL); sxt[nt], sxs[ns], sgw[ns]
 * their error scales (may be NULL). */
int or_dense_backward(int32_t kind, double prm, int32_t d, int64_t nt, const double* xt, int64_t ns,
                      const double* xs, const double* w, const double* gy, double* gxt, double* gxs, double* gw,
                      double* sxt, double* sxs, double* sgw) {
    if (d < 1 || d > 3 || !kern_ok(kind, prm)) return OR_ERR_INVALID;
    if (gxt) {
        for (int64_t i = 0; i < nt; ++i) {
            double acc[3] = {0, 0, 0}, sc = 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                double h = kern_2dphi(kind, prm, sqdist(d, xt + i * d, xs + j * d)) * w[j];
                double mx = 0.0;
                for (int k = 0; k < d; ++k) {
                    double dk = xt[i * d + k] - xs[j * d + k];
                    acc[k] += h * dk;
                    if (fabs(h * dk) > mx) mx = fabs(h * dk);
                }
                sc += mx;
            }
            for (int k = 0; k < d; ++k) gxt[i * d + k] = gy[i] * acc[k];
            if (sxt) sxt[i] = fabs(gy[i]) * sc;
        }
    }
    if (gxs || gw) {
        for (int64_t j = 0; j < ns; ++j) {
            double acc[3] = {0, 0, 0}, sc = 0.0, aw = 0.0, sw = 0.0;
            for (int64_t i = 0; i < nt; ++i) {
                double q = sqdist(d, xt + i * d, xs + j * d);
                double h = kern_2dphi(kind, prm, q) * gy[i];
                double mx = 0.0;
                for (int k = 0; k < d; ++k) {
                    double dk = xs[j * d + k] - xt[i * d + k];
                    acc[k] += h * dk;
                    if (fabs(h * dk) > mx) mx = fabs(h * dk);
                }
                sc += mx;
                double kt = kern_phi(kind, prm, q) * gy[i];
                aw += kt;
                sw += fabs(kt);
            }
            if (gxs) for (int k = 0; k < d; ++k) gxs[j * d + k] = w[j] * acc[k];
            if (sxs) sxs[j] = fabs(w[j]) * sc;
            if (gw) gw[j] = aw;
            if (sgw) sgw[j] = sw;
        }
    }
    return OR_OK;
}
