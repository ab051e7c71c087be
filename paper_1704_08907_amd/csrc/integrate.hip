// Time step of the Section 3 molecular-dynamics example: the semi-implicit
// Euler update of eqs. (2)-(3) (velocity first, then the position with the new
// velocity), applied to the caller's original-order arrays after the force sum
// (eq. (1), the exp-force operator) of the same positions.  A periodic
// coordinate is wrapped back into [lo, hi) by one image; one that rounds onto
// hi becomes lo.  One lane per particle; every array access is coalesced.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pair_common.hpp"

namespace aboria {

namespace {

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
        const T vk = v[e] + dt * f[e];
        T xk = x[e] + dt * vk;
        if (P.periodic[k]) {
            if (xk >= P.hi[k]) xk = xk - P.L[k];
            else if (xk < P.lo[k]) xk = xk + P.L[k];
            if (xk >= P.hi[k]) xk = P.lo[k];
        }
        v[e] = vk;
        x[e] = xk;
    }
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
