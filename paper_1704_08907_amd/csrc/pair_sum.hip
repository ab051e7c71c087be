// Radius-limited neighbour sums over the cell list: the Level 2 box search of
// Section 2.2.2 (a particle's cell and its adjacent cells) evaluating the
// summand of a sum(j, 0 < |dx| < r, f) operator (Section 3, eq. (1) and the
// velocity-update listing), its adjoint, and a pair listing for verification.
//
// Work mapping: one lane per particle in cell order, so the lanes of a wave
// share home cells and therefore candidate cells (their loads hit the same
// cache lines).  The 3^d neighbour cells are walked as 3^(d-1) rows, each row
// a contiguous slot range [off[first cell], off[last cell + 1]) of up to three
// cells along x (split where a periodic wrap changes the image shift).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.hpp"

namespace aboria {

constexpr int kPairBlock = 256;

// ---------------------------------------------------------------------------
// precision-specific primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return ::rsqrt(x); }
__device__ __forceinline__ float exp_neg_t(float s) { return __builtin_amdgcn_exp2f(-s * 1.4426950408889634f); }
__device__ __forceinline__ double exp_neg_t(double s) { return ::exp(-s); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// operators: forward summand and the adjoint contribution of one ordered pair
// (i = the lane's particle, j = its neighbour; dx = x_j + shift - x_i = -u)
// ---------------------------------------------------------------------------

template <typename T>
struct OpArgs {
    T p0;  // k (spring, DEM spring) or c (exp force)
};

template <int OP, int D>
struct OpShape {
    static constexpr int NY = (OP == ABORIA_OP_COUNT || OP == ABORIA_OP_SOFT_SPHERE) ? 1 : D;
    static constexpr int NA = OP == ABORIA_OP_DEM_SPRING ? 1 : 0;
};

template <typename T, int D, int OP>
struct PairOp {
    static constexpr int NY = OpShape<OP, D>::NY;

    // acc += f(x_i, x_j, a_i, a_j)
    __device__ __forceinline__ static void fwd(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj, T* acc) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            acc[0] += T(1);
        } else if constexpr (OP == ABORIA_OP_SPRING) {
            // k (r - s) u / s = (k r / s - k) u,  u = -dx
            const T rinv = rsqrt_t(d2);
            const T g = fma_t(q.p0 * r, rinv, -q.p0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T s = d2 * rsqrt_t(d2);
            const T v = fma_t(-s, T(1) / r, T(1));
            acc[0] = fma_t(T(0.5) * v, v, acc[0]);
        } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
            // eq. (1): -c exp(-|dx|) dx / |dx|
            const T rinv = rsqrt_t(d2);
            const T s = d2 * rinv;
            const T g = q.p0 * exp_neg_t(s) * rinv;
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        } else {  // DEM spring: k (a_i + a_j - s) u / s
            const T rinv = rsqrt_t(d2);
            const T g = fma_t(q.p0 * (ai + aj), rinv, -q.p0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        }
    }

    // gx += J1(i,j)^T gy_i + J2(j,i)^T gy_j ; ga += d/da_i of the same.
    // For f = g(s) u:  gx += g w + (g'/s)(u.w) u with w = gy_i - gy_j, and
    // (u.w) u = (dx.w) dx.  For the soft sphere: gx += 1/2 (gy_i + gy_j)
    // phi'(s) u/s with phi'(s) = -(2/r)(1 - s/r).
    __device__ __forceinline__ static void bwd(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj,
                                               const T* gyi, const T* gyj, T* gx, T* ga) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            return;
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T rinv = rsqrt_t(d2);
            const T s = d2 * rinv;
            const T inv_r = T(1) / r;
            const T coef = (gyi[0] + gyj[0]) * inv_r * fma_t(-s, inv_r, T(1)) * rinv;
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(coef, dx[k], gx[k]);
        } else {
            const T rinv = rsqrt_t(d2);
            const T rinv3 = rinv * rinv * rinv;
            T w[D];
            T dw = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                w[k] = gyi[k] - gyj[k];
                dw = fma_t(dx[k], w[k], dw);
            }
            T g, gps;  // g(s) and g'(s)/s
            if constexpr (OP == ABORIA_OP_SPRING) {
                g = fma_t(q.p0 * r, rinv, -q.p0);
                gps = -q.p0 * r * rinv3;
            } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
                const T s = d2 * rinv;
                const T ce = q.p0 * exp_neg_t(s);
                g = ce * rinv;
                gps = -ce * (s + T(1)) * rinv3;
            } else {
                const T A = ai + aj;
                g = fma_t(q.p0 * A, rinv, -q.p0);
                gps = -q.p0 * A * rinv3;
                // d/da_i: k (gy_i - gy_j).u / s = -k (w.dx) / s
                ga[0] = fma_t(-q.p0 * dw, rinv, ga[0]);
            }
            const T h = gps * dw;
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(g, w[k], fma_t(h, dx[k], gx[k]));
        }
    }
};

// ---------------------------------------------------------------------------
// the neighbour loop
// ---------------------------------------------------------------------------

// Calls visit(j, dx, d2) for every neighbour j of the point xi (cell order
// slot), dx = fl(fl(x_j - x_i) + shift) per dimension and d2 the fma chain,
// accepted iff 0 < d2 < r2.
template <typename T, int D, typename Visit>
__device__ __forceinline__ void neighbour_loop(const SysParams<T>& P, const T* __restrict__ xs,
                                               const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                               Visit&& visit) {
    constexpr int PITCH = Pitch<D>::value;
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T t = xi[k] - P.lo[k];
        const T q = t * P.inv_w[k];
        const T f = floor(q);
        c[k] = !(f >= T(0)) ? 0 : (f > T(P.n[k] - 1) ? P.n[k] - 1 : (int32_t)f);
    }
    // pieces of the x extent [c0-1, c0+1]: contiguous runs with one image shift
    const int32_t nx = P.n[0];
    int np = 0;
    int32_t plo[3], phi[3];
    T psh[3];
    if (nx >= 3) {
        plo[0] = c[0] > 0 ? c[0] - 1 : 0;
        phi[0] = c[0] < nx - 1 ? c[0] + 1 : nx - 1;
        psh[0] = T(0);
        np = 1;
        if (P.periodic[0]) {
            if (c[0] == 0) { plo[np] = phi[np] = nx - 1; psh[np] = -P.L[0]; ++np; }
            if (c[0] == nx - 1) { plo[np] = phi[np] = 0; psh[np] = P.L[0]; ++np; }
        }
    } else {
        for (int o = -1; o <= 1; ++o) {
            int32_t v = c[0] + o;
            T s = T(0);
            if (v < 0) { if (!P.periodic[0]) continue; v += nx; s = -P.L[0]; }
            else if (v >= nx) { if (!P.periodic[0]) continue; v -= nx; s = P.L[0]; }
            plo[np] = phi[np] = v;
            psh[np] = s;
            ++np;
        }
    }
    constexpr int NROWS = D == 1 ? 1 : (D == 2 ? 3 : 9);
    for (int rr = 0; rr < NROWS; ++rr) {
        T sh[3] = {T(0), T(0), T(0)};
        uint32_t row = 0;
        bool skip = false;
        if constexpr (D >= 2) {
            int32_t v = c[1] + (rr % 3) - 1;
            if (v < 0) { if (!P.periodic[1]) skip = true; v += P.n[1]; sh[1] = -P.L[1]; }
            else if (v >= P.n[1]) { if (!P.periodic[1]) skip = true; v -= P.n[1]; sh[1] = P.L[1]; }
            row = (uint32_t)v;
        }
        if constexpr (D >= 3) {
            int32_t v = c[2] + (rr / 3) - 1;
            if (v < 0) { if (!P.periodic[2]) skip = true; v += P.n[2]; sh[2] = -P.L[2]; }
            else if (v >= P.n[2]) { if (!P.periodic[2]) skip = true; v -= P.n[2]; sh[2] = P.L[2]; }
            row += (uint32_t)P.n[1] * (uint32_t)v;
        }
        if (skip) continue;
        const uint32_t rowbase = P.cell_base + (uint32_t)nx * row;
        for (int p = 0; p < np; ++p) {
            const uint32_t j0 = off[rowbase + plo[p]];
            const uint32_t j1 = min(off[rowbase + phi[p] + 1], n);
            sh[0] = psh[p];
            for (uint32_t j = j0; j < j1; ++j) {
                const VecN<T, PITCH> xj = reinterpret_cast<const VecN<T, PITCH>*>(xs)[j];
                T dx[D];
#pragma unroll
                for (int k = 0; k < D; ++k) dx[k] = (xj.v[k] - xi[k]) + sh[k];
                T d2 = dx[0] * dx[0];
                if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
                if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
                if (d2 > T(0) && d2 < P.r2) visit(j, dx, d2);
            }
        }
    }
}

__device__ __forceinline__ int find_system_slot(const uint32_t* __restrict__ first, int nsys, uint32_t i) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T, int D>
__device__ __forceinline__ void load_point(const T* __restrict__ xs, uint32_t s, T* xi) {
    constexpr int PITCH = Pitch<D>::value;
    const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[s];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = v.v[k];
}

// Forward: y[perm[s]] = sum over the neighbours of slot s.
template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(kPairBlock) void k_pair_fwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ perm, uint32_t n,
                                                         const SysParams<T>* __restrict__ sp,
                                                         const uint32_t* __restrict__ sys_part, int nsys,
                                                         const T* __restrict__ a_s, OpArgs<T> q,
                                                         T* __restrict__ y) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int b = BATCH ? find_system_slot(sys_part, nsys, s) : 0;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    const T r = P.r;
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    });
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
}

// Adjoint: gx[perm[s]] (and ga) gathered over the neighbours of slot s, with
// gy_s the upstream gradient already in cell order.
template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(kPairBlock) void k_pair_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ perm, uint32_t n,
                                                         const SysParams<T>* __restrict__ sp,
                                                         const uint32_t* __restrict__ sys_part, int nsys,
                                                         const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                         OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int b = BATCH ? find_system_slot(sys_part, nsys, s) : 0;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) gyi[k] = gy_s[(size_t)s * NY + k];
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        T gyj[NY];
#pragma unroll
        for (int k = 0; k < NY; ++k) gyj[k] = gy_s[(size_t)j * NY + k];
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    });
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

// Pair listing: count per slot, then fill at the scanned offsets.
template <typename T, int D, bool BATCH, bool FILL>
__global__ __launch_bounds__(kPairBlock) void k_pair_list(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                          const uint32_t* __restrict__ perm, uint32_t n,
                                                          const SysParams<T>* __restrict__ sp,
                                                          const uint32_t* __restrict__ sys_part, int nsys,
                                                          uint32_t* __restrict__ counts,
                                                          const uint32_t* __restrict__ starts, uint64_t cap,
                                                          uint32_t* __restrict__ pi, uint32_t* __restrict__ pj) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int b = BATCH ? find_system_slot(sys_part, nsys, s) : 0;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    uint32_t cnt = 0;
    const uint64_t base = FILL ? (uint64_t)starts[s] : 0;
    const uint32_t me = FILL ? perm[s] : 0u;
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T*, T) {
        if (FILL) {
            const uint64_t at = base + cnt;
            if (at < cap) {
                pi[at] = me;
                pj[at] = perm[j];
            }
        }
        ++cnt;
    });
    if (!FILL) counts[s] = cnt;
}

// dst[s][w] = src[perm[s]][w]
template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ src, const uint32_t* __restrict__ perm,
                                                     uint32_t n, int w, T* __restrict__ dst) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n * (uint32_t)w) return;
    const uint32_t s = t / w, k = t - s * w;
    dst[t] = src[(size_t)perm[s] * w + k];
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------

namespace {

template <typename T>
aboria_status gather(aboria_ctx* ctx, const aboria_cells* c, const void* src, int w, void* dst) {
    const uint64_t total = (uint64_t)c->n * (uint64_t)w;
    if (total == 0) return ABORIA_OK;
    hipLaunchKernelGGL(k_gather_rows<T>, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, ctx->stream,
                       (const T*)src, c->perm, (uint32_t)c->n, w, (T*)dst);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D, int OP>
aboria_status launch_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int block) {
    const uint32_t n = (uint32_t)c->n;
    if (n == 0) return ABORIA_OK;
    const dim3 grid((n + block - 1) / block);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_pair_fwd<T, D, OP, false>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs, c->off,
                           c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, y);
    else
        hipLaunchKernelGGL((k_pair_fwd<T, D, OP, true>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs, c->off,
                           c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, y);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D, int OP>
aboria_status launch_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                         T* gx, T* ga, int block) {
    const uint32_t n = (uint32_t)c->n;
    if (n == 0) return ABORIA_OK;
    const dim3 grid((n + block - 1) / block);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_pair_bwd<T, D, OP, false>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs, c->off,
                           c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga);
    else
        hipLaunchKernelGGL((k_pair_bwd<T, D, OP, true>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs, c->off,
                           c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D>
aboria_status fwd_op(aboria_ctx* ctx, const aboria_cells* c, int op, const OpArgs<T>& q, const T* a_s, T* y,
                     int block) {
    switch (op) {
        case ABORIA_OP_COUNT: return launch_fwd<T, D, ABORIA_OP_COUNT>(ctx, c, q, a_s, y, block);
        case ABORIA_OP_SPRING: return launch_fwd<T, D, ABORIA_OP_SPRING>(ctx, c, q, a_s, y, block);
        case ABORIA_OP_SOFT_SPHERE: return launch_fwd<T, D, ABORIA_OP_SOFT_SPHERE>(ctx, c, q, a_s, y, block);
        case ABORIA_OP_EXP_FORCE: return launch_fwd<T, D, ABORIA_OP_EXP_FORCE>(ctx, c, q, a_s, y, block);
        default: return launch_fwd<T, D, ABORIA_OP_DEM_SPRING>(ctx, c, q, a_s, y, block);
    }
}

template <typename T, int D>
aboria_status bwd_op(aboria_ctx* ctx, const aboria_cells* c, int op, const OpArgs<T>& q, const T* a_s,
                     const T* gy_s, T* gx, T* ga, int block) {
    switch (op) {
        case ABORIA_OP_COUNT: return launch_bwd<T, D, ABORIA_OP_COUNT>(ctx, c, q, a_s, gy_s, gx, ga, block);
        case ABORIA_OP_SPRING: return launch_bwd<T, D, ABORIA_OP_SPRING>(ctx, c, q, a_s, gy_s, gx, ga, block);
        case ABORIA_OP_SOFT_SPHERE:
            return launch_bwd<T, D, ABORIA_OP_SOFT_SPHERE>(ctx, c, q, a_s, gy_s, gx, ga, block);
        case ABORIA_OP_EXP_FORCE: return launch_bwd<T, D, ABORIA_OP_EXP_FORCE>(ctx, c, q, a_s, gy_s, gx, ga, block);
        default: return launch_bwd<T, D, ABORIA_OP_DEM_SPRING>(ctx, c, q, a_s, gy_s, gx, ga, block);
    }
}

aboria_status validate(aboria_ctx* ctx, const aboria_cells* c, int op, const double* params, int32_t nparams,
                       const void* a, int32_t na, int32_t ny) {
    if (!c) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (c->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells belong to another device");
    const int32_t eny = op_ny(op, c->d), ena = op_na(op), enp = op_nparams(op);
    if (eny < 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown operator");
    if (ny != eny) return fail(ctx, ABORIA_ERR_INVALID_ARG, "ny does not match the operator");
    if (na != ena) return fail(ctx, ABORIA_ERR_INVALID_ARG, "na does not match the operator");
    if (nparams != enp || (enp > 0 && !params)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "wrong number of params");
    if (ena > 0 && c->n > 0 && !a) return fail(ctx, ABORIA_ERR_INVALID_ARG, "operator needs per-particle variables");
    return ABORIA_OK;
}

int block_of_variant(int32_t v) {
    static const int blocks[] = {256, 128, 64};
    return blocks[v < 0 || v > 2 ? 0 : v];
}

}  // namespace

int32_t variant_count() { return 3; }

const char* variant_name(int32_t v) {
    switch (v) {
        case 0: return "lane-per-particle, x-row runs, 256-thread workgroups";
        case 1: return "lane-per-particle, x-row runs, 128-thread workgroups";
        case 2: return "lane-per-particle, x-row runs, 64-thread workgroups";
        default: return "";
    }
}

aboria_status pair_sum_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, void* y, int32_t ny, int32_t variant) {
    aboria_status st = validate(ctx, c, op, params, nparams, a, na, ny);
    if (st != ABORIA_OK) return st;
    if (c->n > 0 && !y) return fail(ctx, ABORIA_ERR_INVALID_ARG, "y is NULL");
    const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
    if (overlaps(y, tsz * ny * c->n, a, tsz * na * c->n))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "y overlaps a");
    const int block = block_of_variant(variant);
    if (c->dtype == ABORIA_F32) {
        OpArgs<float> q{nparams > 0 ? (float)params[0] : 0.f};
        const float* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<float>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const float*)c->work;
        }
        switch (c->d) {
            case 1: return fwd_op<float, 1>(ctx, c, op, q, a_s, (float*)y, block);
            case 2: return fwd_op<float, 2>(ctx, c, op, q, a_s, (float*)y, block);
            default: return fwd_op<float, 3>(ctx, c, op, q, a_s, (float*)y, block);
        }
    } else {
        OpArgs<double> q{nparams > 0 ? params[0] : 0.0};
        const double* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<double>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const double*)c->work;
        }
        switch (c->d) {
            case 1: return fwd_op<double, 1>(ctx, c, op, q, a_s, (double*)y, block);
            case 2: return fwd_op<double, 2>(ctx, c, op, q, a_s, (double*)y, block);
            default: return fwd_op<double, 3>(ctx, c, op, q, a_s, (double*)y, block);
        }
    }
}

namespace {

aboria_status pair_bwd_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, const void* gy, int32_t ny, void* gx,
                            void* ga, int32_t variant) {
    aboria_status st = validate(ctx, c, op, params, nparams, a, na, ny);
    if (st != ABORIA_OK) return st;
    if (c->n > 0 && (!gy || !gx)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "gy and gx are required");
    const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
    const size_t nb = (size_t)c->n;
    if (overlaps(gx, tsz * c->d * nb, gy, tsz * ny * nb) || overlaps(gx, tsz * c->d * nb, a, tsz * na * nb) ||
        overlaps(ga, tsz * na * nb, gy, tsz * ny * nb) || overlaps(ga, tsz * na * nb, a, tsz * na * nb) ||
        overlaps(ga, tsz * na * nb, gx, tsz * c->d * nb))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "outputs overlap inputs");
    const int block = block_of_variant(variant);
    if (c->dtype == ABORIA_F32) {
        OpArgs<float> q{nparams > 0 ? (float)params[0] : 0.f};
        const float* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<float>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const float*)c->work;
        }
        if ((st = gather<float>(ctx, c, gy, ny, c->work2)) != ABORIA_OK) return st;
        const float* g_s = (const float*)c->work2;
        switch (c->d) {
            case 1: return bwd_op<float, 1>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, block);
            case 2: return bwd_op<float, 2>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, block);
            default: return bwd_op<float, 3>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, block);
        }
    } else {
        OpArgs<double> q{nparams > 0 ? params[0] : 0.0};
        const double* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<double>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const double*)c->work;
        }
        if ((st = gather<double>(ctx, c, gy, ny, c->work2)) != ABORIA_OK) return st;
        const double* g_s = (const double*)c->work2;
        switch (c->d) {
            case 1: return bwd_op<double, 1>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, block);
            case 2: return bwd_op<double, 2>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, block);
            default: return bwd_op<double, 3>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, block);
        }
    }
}

template <typename T, int D>
aboria_status list_pairs(aboria_ctx* ctx, const aboria_cells* c, int64_t cap, uint32_t* pi, uint32_t* pj,
                         int64_t* total) {
    const uint32_t n = (uint32_t)c->n;
    *total = 0;
    if (n == 0) return ABORIA_OK;
    uint32_t* counts = nullptr;
    uint32_t* bsum = nullptr;
    uint32_t* h_last = nullptr;
    const int64_t nb = std::max<int64_t>(scan_block_count(n), 1);
    auto cleanup = [&]() {
        if (counts) (void)hipFree(counts);
        if (bsum) (void)hipFree(bsum);
        if (h_last) (void)hipHostFree(h_last);
    };
    if (hipMalloc((void**)&counts, sizeof(uint32_t) * (size_t)n * 2) != hipSuccess ||
        hipMalloc((void**)&bsum, sizeof(uint32_t) * (size_t)nb) != hipSuccess ||
        hipHostMalloc((void**)&h_last, sizeof(uint32_t) * 2, hipHostMallocDefault) != hipSuccess) {
        cleanup();
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "pair list scratch allocation failed");
    }
    uint32_t* starts = counts + n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + kPairBlock - 1) / kPairBlock);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_pair_list<T, D, false, false>), grid, dim3(kPairBlock), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, counts, starts,
                           (uint64_t)0, pi, pj);
    else
        hipLaunchKernelGGL((k_pair_list<T, D, true, false>), grid, dim3(kPairBlock), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, counts, starts,
                           (uint64_t)0, pi, pj);
    aboria_status st = scan_exclusive_u32(ctx, counts, starts, n, bsum, nb);
    if (st == ABORIA_OK) st = scan_finish_u32(ctx, starts, n, bsum);
    if (st != ABORIA_OK) { cleanup(); return st; }
    hipError_t e = hipMemcpyAsync(h_last, starts + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h_last + 1, counts + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && cap > 0 && pi && pj) {
        if (c->nsys == 1)
            hipLaunchKernelGGL((k_pair_list<T, D, false, true>), grid, dim3(kPairBlock), 0, ctx->stream,
                               (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, counts, starts,
                               (uint64_t)cap, pi, pj);
        else
            hipLaunchKernelGGL((k_pair_list<T, D, true, true>), grid, dim3(kPairBlock), 0, ctx->stream,
                               (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, counts, starts,
                               (uint64_t)cap, pi, pj);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) { cleanup(); return hip_fail(ctx, e, "pair list"); }
    *total = (int64_t)h_last[0] + (int64_t)h_last[1];
    cleanup();
    return ABORIA_OK;
}

}  // namespace

}  // namespace aboria

using namespace aboria;

extern "C" aboria_status aboria_pair_sum(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                         const double* params_host, int32_t nparams, const void* a, int32_t na,
                                         void* y, int32_t ny) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        const int32_t v = cells ? pick_variant(ctx, cells, op) : 0;
        return pair_sum_impl(ctx, cells, op, params_host, nparams, a, na, y, ny, v);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in pair_sum");
    }
}

extern "C" aboria_status aboria_pair_sum_backward(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                                  const double* params_host, int32_t nparams, const void* a,
                                                  int32_t na, const void* gy, int32_t ny, void* gx, void* ga) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        const int32_t v = cells ? pick_variant(ctx, cells, op) : 0;
        return pair_bwd_impl(ctx, cells, op, params_host, nparams, a, na, gy, ny, gx, ga, v);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in pair_sum_backward");
    }
}

extern "C" aboria_status aboria_pair_list(aboria_ctx* ctx, const aboria_cells* c, int64_t cap, uint32_t* pi,
                                          uint32_t* pj, int64_t* total_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!c || !total_host || cap < 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "bad pair_list arguments");
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "pair_list cannot be captured");
    if (cap > 0 && (!pi || !pj)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "pi and pj are required when cap > 0");
    try {
        if (c->dtype == ABORIA_F32) {
            switch (c->d) {
                case 1: return list_pairs<float, 1>(ctx, c, cap, pi, pj, total_host);
                case 2: return list_pairs<float, 2>(ctx, c, cap, pi, pj, total_host);
                default: return list_pairs<float, 3>(ctx, c, cap, pi, pj, total_host);
            }
        } else {
            switch (c->d) {
                case 1: return list_pairs<double, 1>(ctx, c, cap, pi, pj, total_host);
                case 2: return list_pairs<double, 2>(ctx, c, cap, pi, pj, total_host);
                default: return list_pairs<double, 3>(ctx, c, cap, pi, pj, total_host);
            }
        }
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in pair_list");
    }
}
