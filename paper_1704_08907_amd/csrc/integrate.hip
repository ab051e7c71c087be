// Time step of the Section 3 molecular-dynamics example: the semi-implicit
// Euler update of eqs. (2)-(3) (velocity first, then the position with the new
// velocity), applied to the caller's arrays after the force sum (eq. (1), the
// exp-force operator) of the same positions.  A periodic coordinate is wrapped
// back into [lo, hi) by one image; one that rounds onto hi becomes lo.
//
// Three entry points: aboria_integrate applies the update to a force array the
// caller computed; aboria_md_step computes the force by the box search and
// applies the update in the same kernel (the force never leaves registers);
// aboria_cells_reorder permutes the caller's per-particle arrays into the cell
// list's order and makes that the cell list's particle order, so that later
// sums and steps read and write them in cell order, coalesced (the reordering
// container of Section 2.2.1).
#include <hip/hip_runtime.h>

#include <cmath>

#include "pair_common.hpp"

namespace aboria {

namespace {

// The Euler update of one coordinate with its force component fk (eqs. (2)-(3)):
// shared by k_integrate and the fused step, so the two agree bit for bit.
template <typename T>
__device__ __forceinline__ void euler_update(const SysParams<T>& P, int k, T fk, T dt, T& xk, T& vk) {
    vk = vk + dt * fk;
    xk = xk + dt * vk;
    if (P.periodic[k]) {
        if (xk >= P.hi[k]) xk = xk - P.L[k];
        else if (xk < P.lo[k]) xk = xk + P.L[k];
        if (xk >= P.hi[k]) xk = P.lo[k];
    }
}

template <typename T, int D, bool BATCH>
__global__ __launch_bounds__(256) void k_integrate(T* __restrict__ x, T* __restrict__ v, const T* __restrict__ f,
                                                   uint32_t n, const SysParams<T>* __restrict__ sp,
                                                   const uint32_t* __restrict__ sys_part, int nsys, T dt) {
    const uint32_t first = blockIdx.x * blockDim.x;
    const uint32_t i = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, i);
    if (i >= n) return;
    const SysParams<T>& P = sp[b];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const size_t e = (size_t)i * D + k;
        T xk = x[e], vk = v[e];
        euler_update<T>(P, k, f[e], dt, xk, vk);
        v[e] = vk;
        x[e] = xk;
    }
}

// The force of every particle by the box search (the lane-per-particle row
// search, summands in its order, rows through the wave's LDS window), then
// the particle's Euler update as the epilogue.  In place (SORTED = false): x[o], v[o] with o = perm[s]; the
// search reads the cell-ordered snapshot xs, never x, so updating x in place
// is safe.  SORTED: the particle in slot s starts from xs[s] (the exact copy of
// its position) and v[perm[s]], and its new position and velocity go to
// x_out[s], v_out[s], so the outputs come out in cell order and only v is
// gathered.
template <typename T, int D, int OP, bool BATCH, bool OFF32, bool SORTED>
__global__ __launch_bounds__(256) void k_md_step(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ perm, uint32_t n,
                                                 const SysParams<T>* __restrict__ sp,
                                                 const uint32_t* __restrict__ sys_part, int nsys, OpArgs<T> q, T dt,
                                                 T* __restrict__ x, T* __restrict__ v, T* __restrict__ x_out,
                                                 T* __restrict__ v_out) {
    using Op = PairOp<T, D, OP>;
    static_assert(Op::NY == D, "the step needs a force operator");
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    T acc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t, const T* dx, T d2, bool) { Op::fwd(q, r, dx, d2, T(0), T(0), acc); };
    neighbour_loop_staged<T, D, OFF32>(P, xs, off, n, xi, visit);
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const size_t e = (size_t)o * D + k;
        T xk = SORTED ? xi[k] : x[e], vk = v[e];
        euler_update<T>(P, k, acc[k], dt, xk, vk);
        const size_t w = SORTED ? (size_t)s * D + k : e;
        (SORTED ? v_out : v)[w] = vk;
        (SORTED ? x_out : x)[w] = xk;
    }
}

// dst row s = src row perm[s], rows of w 32-bit words.
__global__ __launch_bounds__(256) void k_permute_words(const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ perm, uint32_t n, uint32_t w,
                                                       uint32_t* __restrict__ dst) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t p = perm[s];
    for (uint32_t k = 0; k < w; ++k) dst[(size_t)s * w + k] = src[(size_t)p * w + k];
}

__global__ __launch_bounds__(256) void k_iota(uint32_t* __restrict__ p, uint32_t n) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) p[s] = s;
}

template <typename T, int D, int OP, bool SORTED>
void launch_md_step(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, double dt, void* x, void* v,
                    void* x_out, void* v_out) {
    const uint32_t n = (uint32_t)c->n;
    const dim3 grid((n + 255) / 256);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
#define MD(B, O)                                                                                                 \
    hipLaunchKernelGGL((k_md_step<T, D, OP, B, O, SORTED>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,     \
                       c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, q, (T)dt, (T*)x, (T*)v, (T*)x_out,      \
                       (T*)v_out)
    const bool o32 = off32_rows<T>(n);
    if (c->nsys == 1) {
        if (o32) MD(false, true); else MD(false, false);
    } else {
        if (o32) MD(true, true); else MD(true, false);
    }
#undef MD
}

template <typename T, int D>
aboria_status dispatch_md_step(aboria_ctx* ctx, const aboria_cells* c, int32_t op, double prm, double dt, void* x,
                               void* v, void* x_out, void* v_out) {
    OpArgs<T> q;
    q.p0 = (T)prm;
    const bool sorted = x_out != nullptr;
    if (op == ABORIA_OP_SPRING) {
        if (sorted) launch_md_step<T, D, ABORIA_OP_SPRING, true>(ctx, c, q, dt, x, v, x_out, v_out);
        else launch_md_step<T, D, ABORIA_OP_SPRING, false>(ctx, c, q, dt, x, v, x_out, v_out);
    } else {
        if (sorted) launch_md_step<T, D, ABORIA_OP_EXP_FORCE, true>(ctx, c, q, dt, x, v, x_out, v_out);
        else launch_md_step<T, D, ABORIA_OP_EXP_FORCE, false>(ctx, c, q, dt, x, v, x_out, v_out);
    }
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D>
void launch_integrate(aboria_ctx* ctx, const aboria_cells* c, double dt, const void* f, void* x, void* v) {
    const uint32_t n = (uint32_t)c->n;
    const dim3 grid((n + 255) / 256);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_integrate<T, D, false>), grid, dim3(256), 0, ctx->stream, (T*)x, (T*)v, (const T*)f, n,
                           sp, c->sys_part_dev, c->nsys, (T)dt);
    else
        hipLaunchKernelGGL((k_integrate<T, D, true>), grid, dim3(256), 0, ctx->stream, (T*)x, (T*)v, (const T*)f, n,
                           sp, c->sys_part_dev, c->nsys, (T)dt);
}

}  // namespace

}  // namespace aboria

using namespace aboria;

extern "C" aboria_status aboria_integrate(aboria_ctx* ctx, const aboria_cells* c, double dt, const void* f, void* x,
                                          void* v) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!c) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (c->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells belong to another device");
    if (!std::isfinite(dt)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "dt must be finite");
    if (c->n == 0) return ABORIA_OK;
    if (!f || !x || !v) return fail(ctx, ABORIA_ERR_INVALID_ARG, "f, x and v are required");
    const size_t bytes = (size_t)c->n * (size_t)c->d * (c->dtype == ABORIA_F32 ? 4 : 8);
    if (overlaps(x, bytes, v, bytes) || overlaps(f, bytes, x, bytes) || overlaps(f, bytes, v, bytes))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "f, x and v must not overlap");
    try {
        if (c->dtype == ABORIA_F32) {
            switch (c->d) {
                case 1: launch_integrate<float, 1>(ctx, c, dt, f, x, v); break;
                case 2: launch_integrate<float, 2>(ctx, c, dt, f, x, v); break;
                default: launch_integrate<float, 3>(ctx, c, dt, f, x, v); break;
            }
        } else {
            switch (c->d) {
                case 1: launch_integrate<double, 1>(ctx, c, dt, f, x, v); break;
                case 2: launch_integrate<double, 2>(ctx, c, dt, f, x, v); break;
                default: launch_integrate<double, 3>(ctx, c, dt, f, x, v); break;
            }
        }
        ABORIA_HIP(ctx, hipGetLastError());
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in integrate");
    }
}

extern "C" aboria_status aboria_md_step(aboria_ctx* ctx, const aboria_cells* c, aboria_op op,
                                        const double* params_host, int32_t nparams, double dt, void* x, void* v,
                                        void* x_out, void* v_out) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!c) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (c->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells belong to another device");
    if (op != ABORIA_OP_EXP_FORCE && op != ABORIA_OP_SPRING)
        return fail(ctx, ABORIA_ERR_UNSUPPORTED, "the fused step takes the eq. (1) force or the spring force");
    if (nparams != 1 || !params_host || !std::isfinite(params_host[0]))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "the force takes one finite parameter");
    if (!std::isfinite(dt)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "dt must be finite");
    if ((x_out == nullptr) != (v_out == nullptr))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "x_out and v_out go together");
    if (c->n == 0) return ABORIA_OK;
    const bool sorted = x_out != nullptr;
    if (!v || (!sorted && !x)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "x and v are required");
    const size_t bytes = (size_t)c->n * (size_t)c->d * (c->dtype == ABORIA_F32 ? 4 : 8);
    if (!sorted && overlaps(x, bytes, v, bytes)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "x and v must not overlap");
    if (sorted && (overlaps(x_out, bytes, v_out, bytes) || overlaps(x_out, bytes, v, bytes) ||
                   overlaps(v_out, bytes, v, bytes) || (x && (overlaps(x_out, bytes, x, bytes) ||
                                                              overlaps(v_out, bytes, x, bytes)))))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "x_out and v_out must not overlap each other or the inputs");
    try {
        if (c->dtype == ABORIA_F32) {
            switch (c->d) {
                case 1: return dispatch_md_step<float, 1>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
                case 2: return dispatch_md_step<float, 2>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
                default: return dispatch_md_step<float, 3>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
            }
        }
        switch (c->d) {
            case 1: return dispatch_md_step<double, 1>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
            case 2: return dispatch_md_step<double, 2>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
            default: return dispatch_md_step<double, 3>(ctx, c, op, params_host[0], dt, x, v, x_out, v_out);
        }
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in md_step");
    }
}

extern "C" aboria_status aboria_cells_reorder(aboria_ctx* ctx, aboria_cells* c, int32_t nbuf, void* const* bufs_host,
                                              const int32_t* row_bytes_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!c) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (c->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells belong to another device");
    if (nbuf < 0 || (nbuf > 0 && (!bufs_host || !row_bytes_host)))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "buffer list is NULL");
    const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
    const size_t cap = 4 * tsz;  // the cell list's work buffer holds 4 elements per particle
    for (int32_t b = 0; b < nbuf; ++b) {
        const int32_t rb = row_bytes_host[b];
        if (!bufs_host[b] || rb <= 0 || rb % 4 != 0 || (size_t)rb > cap)
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "each buffer needs rows of 4 to " + std::to_string(cap) +
                                                         " bytes, a multiple of 4");
        for (int32_t b2 = 0; b2 < b; ++b2)
            if (overlaps(bufs_host[b], (size_t)rb * c->n, bufs_host[b2], (size_t)row_bytes_host[b2] * c->n))
                return fail(ctx, ABORIA_ERR_INVALID_ARG, "buffers overlap");
    }
    const uint32_t n = (uint32_t)c->n;
    if (n == 0) return ABORIA_OK;
    try {
        const dim3 grid((n + 255) / 256);
        for (int32_t b = 0; b < nbuf; ++b) {
            const uint32_t w = (uint32_t)row_bytes_host[b] / 4;
            hipLaunchKernelGGL(k_permute_words, grid, dim3(256), 0, ctx->stream, (const uint32_t*)bufs_host[b],
                               c->perm, n, w, (uint32_t*)c->work);
            ABORIA_HIP(ctx, hipGetLastError());
            ABORIA_HIP(ctx, hipMemcpyAsync(bufs_host[b], c->work, (size_t)w * 4 * n, hipMemcpyDeviceToDevice,
                                           ctx->stream));
        }
        // the caller's order is now the cell order: sums write their outputs in it
        hipLaunchKernelGGL(k_iota, grid, dim3(256), 0, ctx->stream, c->perm, n);
        ABORIA_HIP(ctx, hipGetLastError());
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in cells_reorder");
    }
}
