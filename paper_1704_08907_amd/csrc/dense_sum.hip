// Dense kernel sum of the RBF / Gaussian-process methods (Section 1 and the
// RBF and Kansa examples of Section 1.1): y_i = sum_j K(x_i, x_j) w_j over all
// sources, here with the Gaussian kernel K = exp(-|x_i - x_j|^2 / (2 sigma^2)).
//
// Each thread keeps TI targets in registers; the workgroup streams tiles of
// 256 sources (position and weight, 16 or 32 bytes each) through LDS, and every
// lane reads each source with one broadcast LDS load.  Coordinates are
// pre-scaled by sqrt(c) so that the squared scaled distance is directly the
// argument of one exp2 (float) or exp (double).  The source range is split over
// a second grid dimension so that the launch fills all compute units; the split
// partial sums are added in a fixed order by a second kernel, and inside a
// split every tile's sum is formed separately before it is added (pairwise
// accumulation keeps the float32 error well below the tile length times u).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace aboria {

constexpr int kDenseBlock = 256;
constexpr int kDenseTile = 256;

__device__ __forceinline__ float kexp(float a) { return __builtin_amdgcn_exp2f(-a); }
__device__ __forceinline__ double kexp(double a) { return ::exp(-a); }
__device__ __forceinline__ float kfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double kfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int D, int TI>
__global__ __launch_bounds__(kDenseBlock) void k_dense_gauss(const T* __restrict__ xt, uint32_t nt,
                                                             const T* __restrict__ xs, const T* __restrict__ w,
                                                             uint32_t ns, T sc, uint32_t jchunk,
                                                             T* __restrict__ ypart) {
    __shared__ VecN<T, 4> tile[kDenseTile];
    const uint32_t tb = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t split = blockIdx.y;
    T xi[TI][D];
    T acc[TI];
#pragma unroll
    for (int q = 0; q < TI; ++q) {
        const uint32_t t = tb * (kDenseBlock * TI) + q * kDenseBlock + threadIdx.x;
        const uint32_t tc = t < nt ? t : nt - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) xi[q][k] = xt[(size_t)tc * D + k] * sc;
        acc[q] = T(0);
    }
    const uint32_t jbeg = split * jchunk;
    const uint32_t jend = min(ns, jbeg + jchunk);
    for (uint32_t j0 = jbeg; j0 < jend; j0 += kDenseTile) {
        __syncthreads();
        {
            const uint32_t j = j0 + threadIdx.x;
            VecN<T, 4> v;
            v.v[0] = v.v[1] = v.v[2] = v.v[3] = T(0);
            if (j < jend) {
#pragma unroll
                for (int k = 0; k < D; ++k) v.v[k] = xs[(size_t)j * D + k] * sc;
                v.v[3] = w[j];
            }
            tile[threadIdx.x] = v;
        }
        __syncthreads();
        T part[TI];
#pragma unroll
        for (int q = 0; q < TI; ++q) part[q] = T(0);
#pragma unroll 4
        for (int jj = 0; jj < kDenseTile; ++jj) {
            const VecN<T, 4> p = tile[jj];
#pragma unroll
            for (int q = 0; q < TI; ++q) {
                const T d0 = xi[q][0] - p.v[0];
                T d2 = d0 * d0;
                if constexpr (D >= 2) {
                    const T d1 = xi[q][1] - p.v[1];
                    d2 = kfma(d1, d1, d2);
                }
                if constexpr (D >= 3) {
                    const T dz = xi[q][2] - p.v[2];
                    d2 = kfma(dz, dz, d2);
                }
                part[q] = kfma(kexp(d2), p.v[3], part[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < TI; ++q) acc[q] += part[q];
    }
#pragma unroll
    for (int q = 0; q < TI; ++q) {
        const uint32_t t = tb * (kDenseBlock * TI) + q * kDenseBlock + threadIdx.x;
        if (t < nt) ypart[(size_t)split * nt + t] = acc[q];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_reduce(const T* __restrict__ ypart, uint32_t nt, uint32_t nsplit,
                                                      T* __restrict__ y) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
    T s = T(0);
    for (uint32_t k = 0; k < nsplit; ++k) s += ypart[(size_t)k * nt + t];
    y[t] = s;
}

namespace {

constexpr int kTargetsPerThread = 4;

template <typename T, int D>
aboria_status launch_dense(aboria_ctx* ctx, uint32_t nt, const void* xt, uint32_t ns, const void* xs, const void* w,
                           double sigma, void* y) {
    const uint32_t per_block = kDenseBlock * kTargetsPerThread;
    const uint32_t tblocks = (nt + per_block - 1) / per_block;
    const uint32_t ntiles = std::max<uint32_t>((ns + kDenseTile - 1) / kDenseTile, 1);
    // enough workgroups to fill 256 CUs several times over
    uint32_t nsplit = std::max<uint32_t>(1, (2048 + tblocks - 1) / tblocks);
    nsplit = std::min(nsplit, ntiles);
    const uint32_t tiles_per_split = (ntiles + nsplit - 1) / nsplit;
    nsplit = (ntiles + tiles_per_split - 1) / tiles_per_split;
    const uint32_t jchunk = tiles_per_split * kDenseTile;
    const size_t need = sizeof(T) * (size_t)nsplit * nt;
    if (ctx->scratch_bytes < need) {
        if (ctx->capturing)
            return fail(ctx, ABORIA_ERR_UNSUPPORTED, "dense scratch must be sized by an uncaptured call first");
        if (ctx->scratch) {
            ABORIA_HIP(ctx, hipStreamSynchronize(ctx->stream));
            (void)hipFree(ctx->scratch);
            ctx->scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        if (hipMalloc(&ctx->scratch, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "dense scratch allocation failed");
        }
        ctx->scratch_bytes = need;
    }
    // float: exp2(-c d^2) with c = log2(e) / (2 sigma^2); double: exp(-d^2 / (2 sigma^2))
    const double c = (sizeof(T) == 4 ? 1.4426950408889634 : 1.0) / (2.0 * sigma * sigma);
    const T sc = (T)std::sqrt(c);
    hipLaunchKernelGGL((k_dense_gauss<T, D, kTargetsPerThread>), dim3(tblocks, nsplit), dim3(kDenseBlock), 0,
                       ctx->stream, (const T*)xt, nt, (const T*)xs, (const T*)w, ns, sc, jchunk, (T*)ctx->scratch);
    hipLaunchKernelGGL(k_dense_reduce<T>, dim3((nt + 255) / 256), dim3(256), 0, ctx->stream,
                       (const T*)ctx->scratch, nt, nsplit, (T*)y);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

}  // namespace

}  // namespace aboria

using namespace aboria;

extern "C" aboria_status aboria_dense_sum(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                          const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                                          const void* xt, int64_t n_source, const void* xs, const void* w, void* y) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        if (kernel != ABORIA_K_GAUSSIAN) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown kernel");
        if (dtype != ABORIA_F32 && dtype != ABORIA_F64) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown dtype");
        if (nparams != 1 || !params_host) return fail(ctx, ABORIA_ERR_INVALID_ARG, "the Gaussian kernel takes {sigma}");
        const double sigma = params_host[0];
        if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "sigma must be positive");
        if (d < 1 || d > 3) return fail(ctx, ABORIA_ERR_INVALID_ARG, "d must be 1, 2 or 3");
        if (n_target < 0 || n_source < 0 || n_target >= ((int64_t)1 << 31) || n_source >= ((int64_t)1 << 31))
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "sizes must lie in [0, 2^31)");
        if (n_target == 0) return ABORIA_OK;
        if (!xt || !y || (n_source > 0 && (!xs || !w))) return fail(ctx, ABORIA_ERR_INVALID_ARG, "NULL array");
        const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
        const size_t ny = tsz * (size_t)n_target;
        if (overlaps(y, ny, xt, tsz * d * (size_t)n_target) || overlaps(y, ny, xs, tsz * d * (size_t)n_source) ||
            overlaps(y, ny, w, tsz * (size_t)n_source))
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "y overlaps an input");
        const uint32_t nt = (uint32_t)n_target, ns = (uint32_t)n_source;
        if (dtype == ABORIA_F32) {
            switch (d) {
                case 1: return launch_dense<float, 1>(ctx, nt, xt, ns, xs, w, sigma, y);
                case 2: return launch_dense<float, 2>(ctx, nt, xt, ns, xs, w, sigma, y);
                default: return launch_dense<float, 3>(ctx, nt, xt, ns, xs, w, sigma, y);
            }
        } else {
            switch (d) {
                case 1: return launch_dense<double, 1>(ctx, nt, xt, ns, xs, w, sigma, y);
                case 2: return launch_dense<double, 2>(ctx, nt, xt, ns, xs, w, sigma, y);
                default: return launch_dense<double, 3>(ctx, nt, xt, ns, xs, w, sigma, y);
            }
        }
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in dense_sum");
    }
}
