// Dense kernel sums of the RBF / Gaussian-process methods (Section 1 and the
// RBF and Kansa examples of Section 1.1): y_i = sum_j K(x_i, x_j) w_j over all
// sources, for the radial kernels K = phi(|x_i - x_j|^2) of those examples:
// the Gaussian exp(-q / (2 sigma^2)) and the multiquadric sqrt(q + c^2); and
// the adjoint of the sum: dL/dw = K^T gy (the same sum with targets and
// sources exchanged) and the position gradients sum_j w_j 2 phi'(q) (a - b).
//
// Each thread keeps TI targets in registers; the workgroup streams tiles of
// 256 sources (position and weight, 16 or 32 bytes each) through LDS, and every
// lane reads each source with one broadcast LDS load.  Gaussian coordinates are
// pre-scaled by sqrt(c) so that the squared scaled distance is directly the
// argument of one exp2 (float) or exp (double).  The source range is split over
// a second grid dimension so that the launch fills all compute units; the split
// partial sums are added in a fixed order by a second kernel (which also
// applies the gradient's per-row factor), and inside a split every tile's sum
// is formed separately before it is added (pairwise accumulation keeps the
// float32 error well below the tile length times u).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"

namespace aboria {

constexpr int kDenseBlock = 256;
constexpr int kDenseTile = 256;

// Scratch of aboria_dense_sum_noalloc: its split partial sums live in this
// file-scope device array (each GPU holds its own copy until the process ends)
// instead of the context's grow-only buffer.  Host code never passes the
// array's name to a kernel: in host code it is only a stand-in, and the device
// address of each GPU's copy comes from hipGetSymbolAddress (noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

__device__ __forceinline__ float kexp(float a) { return __builtin_amdgcn_exp2f(-a); }
__device__ __forceinline__ double kexp(double a) { return ::exp(-a); }
__device__ __forceinline__ float kfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double kfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float ksqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double ksqrt(double a) { return ::sqrt(a); }
__device__ __forceinline__ float krsqrt(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ double krsqrt(double a) { return ::rsqrt(a); }

// phi of the kernel on its working coordinates (value) and the factor of the
// gradient summand w_j * slope * (a - b) (the constant 2 phi' / slope is
// applied by the reduction): Gaussian value = slope = exp(-q') on coordinates
// scaled by sqrt(c); multiquadric value = sqrt(q + c^2) and slope =
// 1/sqrt(q + c^2), each one transcendental instruction, so a pass needing both
// computes the value exactly as the forward does.
template <typename T, int KERN>
struct Radial {
    __device__ __forceinline__ static T value(T q, T c2) {
        if constexpr (KERN == ABORIA_K_GAUSSIAN) return kexp(q);
        else return ksqrt(q + c2);
    }
    __device__ __forceinline__ static T slope(T q, T c2) {
        if constexpr (KERN == ABORIA_K_GAUSSIAN) return kexp(q);
        else return krsqrt(q + c2);
    }
};

// What a pass sums per target t over the split's sources j:
//   kSum:     part[split][t]      = sum of K w
//   kGrad:    part[split][t][k]   = sum of w * slope * (xt_t - xs_j)_k
//   kSumGrad: part[split][t][0]   = sum of K w and part[split][t][1 + k] the kGrad sum
//             (one pass for two sums with the same targets, sources and weights:
//             the adjoint's K^T gy and source-position gradient)
enum DenseMode { kSum = 0, kGrad = 1, kSumGrad = 2 };

template <int MODE, int D>
constexpr int dense_out() { return MODE == kSum ? 1 : (MODE == kGrad ? D : D + 1); }

template <typename T, int D, int TI, int KERN, int MODE>
__global__ __launch_bounds__(kDenseBlock) void k_dense(const T* __restrict__ xt, uint32_t nt,
                                                       const T* __restrict__ xs, const T* __restrict__ w,
                                                       uint32_t ns, T sc, T c2, uint32_t jchunk,
                                                       T* __restrict__ ypart) {
    constexpr int OUT = dense_out<MODE, D>();
    __shared__ VecN<T, 4> tile[kDenseTile];
    const uint32_t tb = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t split = blockIdx.y;
    T xi[TI][D];
    T acc[TI][OUT];
#pragma unroll
    for (int q = 0; q < TI; ++q) {
        const uint32_t t = tb * (kDenseBlock * TI) + q * kDenseBlock + threadIdx.x;
        const uint32_t tc = t < nt ? t : nt - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) xi[q][k] = xt[(size_t)tc * D + k] * sc;
#pragma unroll
        for (int k = 0; k < OUT; ++k) acc[q][k] = T(0);
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
        T part[TI][OUT];
#pragma unroll
        for (int q = 0; q < TI; ++q)
#pragma unroll
            for (int k = 0; k < OUT; ++k) part[q][k] = T(0);
#pragma unroll 4
        for (int jj = 0; jj < kDenseTile; ++jj) {
            const VecN<T, 4> p = tile[jj];
#pragma unroll
            for (int q = 0; q < TI; ++q) {
                T dk[D];
#pragma unroll
                for (int k = 0; k < D; ++k) dk[k] = xi[q][k] - p.v[k];
                T d2 = dk[0] * dk[0];
                if constexpr (D >= 2) d2 = kfma(dk[1], dk[1], d2);
                if constexpr (D >= 3) d2 = kfma(dk[2], dk[2], d2);
                if constexpr (MODE == kSum) {
                    part[q][0] = kfma(Radial<T, KERN>::value(d2, c2), p.v[3], part[q][0]);
                } else {
                    constexpr int G = MODE == kSumGrad ? 1 : 0;  // first gradient component
                    T slope;
                    if constexpr (MODE == kSumGrad && KERN == ABORIA_K_MULTIQUADRIC) {
                        const T a = d2 + c2;
                        slope = krsqrt(a);
                        part[q][0] = kfma(ksqrt(a), p.v[3], part[q][0]);
                    } else {
                        slope = Radial<T, KERN>::slope(d2, c2);
                        if constexpr (MODE == kSumGrad)  // the Gaussian's value is its slope
                            part[q][0] = kfma(Radial<T, KERN>::value(d2, c2), p.v[3], part[q][0]);
                    }
                    const T h = slope * p.v[3];
#pragma unroll
                    for (int k = 0; k < D; ++k) part[q][G + k] = kfma(h, dk[k], part[q][G + k]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < TI; ++q)
#pragma unroll
            for (int k = 0; k < OUT; ++k) acc[q][k] += part[q][k];
    }
#pragma unroll
    for (int q = 0; q < TI; ++q) {
        const uint32_t t = tb * (kDenseBlock * TI) + q * kDenseBlock + threadIdx.x;
        if (t < nt)
#pragma unroll
            for (int k = 0; k < OUT; ++k) ypart[((size_t)split * nt + t) * OUT + k] = acc[q][k];
    }
}

// y[t][k] = sum over splits (in split order); with mult, y[t][k] = (mult[t] * C) * sum.
template <typename T, int OUT>
__global__ __launch_bounds__(256) void k_dense_reduce(const T* __restrict__ ypart, uint32_t nt, uint32_t nsplit,
                                                      const T* __restrict__ mult, T C, T* __restrict__ y) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
#pragma unroll
    for (int k = 0; k < OUT; ++k) {
        T s = T(0);
        for (uint32_t q = 0; q < nsplit; ++q) s += ypart[((size_t)q * nt + t) * OUT + k];
        y[(size_t)t * OUT + k] = mult ? (mult[t] * C) * s : s;
    }
}

// The kSumGrad partials: y[t] = sum of component 0, g[t][k] = (mult[t] * C) * sum of
// component 1 + k, each over the splits in split order.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_dense_reduce2(const T* __restrict__ ypart, uint32_t nt, uint32_t nsplit,
                                                       const T* __restrict__ mult, T C, T* __restrict__ y,
                                                       T* __restrict__ g) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        T s = T(0);
        for (uint32_t q = 0; q < nsplit; ++q) s += ypart[((size_t)q * nt + t) * (D + 1) + k];
        if (k == 0) y[t] = s;
        else g[(size_t)t * D + k - 1] = (mult[t] * C) * s;
    }
}

namespace {

// Launch shapes of the dense sum: targets kept per lane and the number of
// workgroups the source split aims for (the split count is that over the
// target blocks, at most one per source tile).  Plan 0 is the untuned default;
// eight targets per lane are float only (float64 would hold twice the
// registers).  aboria_autotune_dense times them.
struct DensePlan {
    int32_t ti;
    int32_t wg;
    const char* name;
};
constexpr DensePlan kDensePlans[] = {
    {4, 2048, "4 targets per lane, 2048 workgroups"}, {2, 2048, "2 targets per lane, 2048 workgroups"},
    {8, 2048, "8 targets per lane, 2048 workgroups"}, {4, 4096, "4 targets per lane, 4096 workgroups"},
    {8, 4096, "8 targets per lane, 4096 workgroups"}, {2, 1024, "2 targets per lane, 1024 workgroups"},
    {4, 1024, "4 targets per lane, 1024 workgroups"}, {8, 1024, "8 targets per lane, 1024 workgroups"},
};
constexpr int32_t kNumDensePlans = sizeof(kDensePlans) / sizeof(kDensePlans[0]);

bool dense_plan_ok(int32_t p, int dtype) {
    return p >= 0 && p < kNumDensePlans && (dtype == ABORIA_F32 || kDensePlans[p].ti <= 4);
}

// Tuning key: direction, kernel, dtype, d and the size buckets (floor log2) of
// the targets and sources.
uint64_t dense_key(bool backward, int kernel, int dtype, int d, int64_t nt, int64_t ns) {
    uint64_t k = backward ? 1u : 0u;
    k = k * 4 + (uint64_t)kernel;
    k = k * 4 + (uint64_t)dtype;
    k = k * 4 + (uint64_t)d;
    k = k * 64 + (uint64_t)std::floor(std::log2((double)nt + 1.0));
    k = k * 64 + (uint64_t)std::floor(std::log2((double)ns + 1.0));
    return k;
}

// The plan a call uses: the tuner's current trial, else the cached choice for
// its key, else plan 0.
int32_t dense_plan_for(const aboria_ctx* ctx, uint64_t key, int dtype) {
    if (ctx->dense_plan_forced >= 0) return ctx->dense_plan_forced;
    for (const auto& kv : ctx->dense_cache) {
        if (kv.first != key) continue;
        for (int32_t p = 0; p < kNumDensePlans; ++p)
            if (kDensePlans[p].ti == kv.second.ti && kDensePlans[p].wg == kv.second.wg && dense_plan_ok(p, dtype))
                return p;
    }
    return 0;
}

// Kernel constants: Gaussian prm = sigma, multiquadric prm = c.
struct KernelPlan {
    double sc;   // coordinate scale
    double c2;   // multiquadric c^2
    double C;    // gradient constant: 2 phi'(q) (a - b) = C * slope * (scaled a - scaled b)
};

template <typename T>
KernelPlan plan_kernel(int kernel, double prm) {
    KernelPlan k{1.0, 0.0, 1.0};
    if (kernel == ABORIA_K_GAUSSIAN) {
        // float: exp2(-c d^2) with c = log2(e) / (2 sigma^2); double: exp(-d^2 / (2 sigma^2))
        const double c = (sizeof(T) == 4 ? 1.4426950408889634 : 1.0) / (2.0 * prm * prm);
        k.sc = std::sqrt(c);
        k.C = -1.0 / (prm * prm * (double)(T)k.sc);  // 2 phi' = -phi / sigma^2, and d = d' / sc
    } else {
        k.c2 = prm * prm;
    }
    return k;
}

aboria_status ensure_scratch(aboria_ctx* ctx, size_t need) {
    if (ctx->scratch_bytes >= need) return ABORIA_OK;
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
    return ABORIA_OK;
}

// Device address of this GPU's copy of the no-allocation scratch array, looked
// up once per device with that device current and kept for the process.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

aboria_status noalloc_scratch(aboria_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(ctx, ABORIA_ERR_UNSUPPORTED, "device index beyond the no-allocation scratch table");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[ctx->device]) {
        int cur = 0;
        ABORIA_HIP(ctx, hipGetDevice(&cur));
        if (cur != ctx->device) ABORIA_HIP(ctx, hipSetDevice(ctx->device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != ctx->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(ctx, ABORIA_ERR_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                                    hipGetErrorString(e));
        }
        g_noalloc_ptr[ctx->device] = ptr;
    }
    *out = g_noalloc_ptr[ctx->device];
    return ABORIA_OK;
}

// kSum: out = sum_j K(xt_i, xs_j) w_j; kGrad: out = mult_i * C * sum_j w_j slope (xt_i - xs_j);
// kSumGrad: out = the kSum sum and out2 = the kGrad sum, from one pass.  The split
// partials go to the context's grow-only scratch, or, when part is given, to the
// part_cap bytes at part (fewer splits when they would not fit; an error when even
// one split's partials do not).  Every partial entry the reduction reads is
// written by k_dense, so the scratch needs no clearing.
template <typename T, int D, int KERN, int MODE>
aboria_status launch_dense(aboria_ctx* ctx, uint32_t nt, const void* xt, uint32_t ns, const void* xs, const void* w,
                           const KernelPlan& kp, const void* mult, void* out, void* out2, void* part,
                           size_t part_cap, int32_t plan) {
    constexpr int OUT = dense_out<MODE, D>();
    const DensePlan& pl = kDensePlans[dense_plan_ok(plan, sizeof(T) == 4 ? ABORIA_F32 : ABORIA_F64) ? plan : 0];
    const uint32_t per_block = kDenseBlock * (uint32_t)pl.ti;
    const uint32_t tblocks = (nt + per_block - 1) / per_block;
    const uint32_t ntiles = std::max<uint32_t>((ns + kDenseTile - 1) / kDenseTile, 1);
    // enough workgroups to fill 256 CUs several times over
    uint32_t nsplit = std::max<uint32_t>(1, ((uint32_t)pl.wg + tblocks - 1) / tblocks);
    nsplit = std::min(nsplit, ntiles);
    const size_t split_bytes = sizeof(T) * (size_t)nt * OUT;
    if (part) {
        const size_t fit = part_cap / split_bytes;
        if (fit == 0)
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "n_target too large for the no-allocation scratch (" +
                                                         std::to_string(part_cap / (sizeof(T) * OUT)) +
                                                         " targets at most)");
        nsplit = (uint32_t)std::min<size_t>(nsplit, fit);
    }
    const uint32_t tiles_per_split = (ntiles + nsplit - 1) / nsplit;
    nsplit = (ntiles + tiles_per_split - 1) / tiles_per_split;
    const uint32_t jchunk = tiles_per_split * kDenseTile;
    if (!part) {
        aboria_status st = ensure_scratch(ctx, split_bytes * nsplit);
        if (st != ABORIA_OK) return st;
        part = ctx->scratch;
    }
#define ABORIA_DENSE_LAUNCH(TI)                                                                            \
    hipLaunchKernelGGL((k_dense<T, D, TI, KERN, MODE>), dim3(tblocks, nsplit), dim3(kDenseBlock), 0, ctx->stream, \
                       (const T*)xt, nt, (const T*)xs, (const T*)w, ns, (T)kp.sc, (T)kp.c2, jchunk, (T*)part)
    if (pl.ti == 2) {
        ABORIA_DENSE_LAUNCH(2);
    } else if (pl.ti == 8) {
        if constexpr (sizeof(T) == 4) ABORIA_DENSE_LAUNCH(8);
    } else {
        ABORIA_DENSE_LAUNCH(4);
    }
#undef ABORIA_DENSE_LAUNCH
    if constexpr (MODE == kSumGrad)
        hipLaunchKernelGGL((k_dense_reduce2<T, D>), dim3((nt + 255) / 256), dim3(256), 0, ctx->stream,
                           (const T*)part, nt, nsplit, (const T*)mult, (T)kp.C, (T*)out, (T*)out2);
    else
        hipLaunchKernelGGL((k_dense_reduce<T, OUT>), dim3((nt + 255) / 256), dim3(256), 0, ctx->stream,
                           (const T*)part, nt, nsplit, (const T*)mult, (T)kp.C, (T*)out);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D, int MODE>
aboria_status launch_kernel(aboria_ctx* ctx, int kernel, uint32_t nt, const void* xt, uint32_t ns, const void* xs,
                            const void* w, double prm, const void* mult, void* out, void* out2, void* part,
                            size_t part_cap, int32_t plan) {
    const KernelPlan kp = plan_kernel<T>(kernel, prm);
    if (kernel == ABORIA_K_GAUSSIAN)
        return launch_dense<T, D, ABORIA_K_GAUSSIAN, MODE>(ctx, nt, xt, ns, xs, w, kp, mult, out, out2, part,
                                                            part_cap, plan);
    return launch_dense<T, D, ABORIA_K_MULTIQUADRIC, MODE>(ctx, nt, xt, ns, xs, w, kp, mult, out, out2, part,
                                                            part_cap, plan);
}

template <int MODE>
aboria_status dispatch(aboria_ctx* ctx, int dtype, int d, int kernel, uint32_t nt, const void* xt, uint32_t ns,
                       const void* xs, const void* w, double prm, const void* mult, void* out,
                       void* out2 = nullptr, void* part = nullptr, size_t part_cap = 0, int32_t plan = 0) {
    if (dtype == ABORIA_F32) {
        switch (d) {
            case 1:
                return launch_kernel<float, 1, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                     part_cap, plan);
            case 2:
                return launch_kernel<float, 2, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                     part_cap, plan);
            default:
                return launch_kernel<float, 3, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                     part_cap, plan);
        }
    }
    switch (d) {
        case 1:
            return launch_kernel<double, 1, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                  part_cap, plan);
        case 2:
            return launch_kernel<double, 2, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                  part_cap, plan);
        default:
            return launch_kernel<double, 3, MODE>(ctx, kernel, nt, xt, ns, xs, w, prm, mult, out, out2, part,
                                                  part_cap, plan);
    }
}

aboria_status check_common(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel, const double* params_host,
                           int32_t nparams, int32_t d, int64_t n_target, int64_t n_source) {
    if (kernel != ABORIA_K_GAUSSIAN && kernel != ABORIA_K_MULTIQUADRIC)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown kernel");
    if (dtype != ABORIA_F32 && dtype != ABORIA_F64) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown dtype");
    if (nparams != 1 || !params_host) return fail(ctx, ABORIA_ERR_INVALID_ARG, "the kernel takes one parameter");
    const double prm = params_host[0];
    if (!(prm > 0.0) || !std::isfinite(prm))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "the kernel parameter (sigma or c) must be positive");
    if (d < 1 || d > 3) return fail(ctx, ABORIA_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (n_target < 0 || n_source < 0 || n_target >= ((int64_t)1 << 31) || n_source >= ((int64_t)1 << 31))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "sizes must lie in [0, 2^31)");
    return ABORIA_OK;
}

}  // namespace

}  // namespace aboria

using namespace aboria;

namespace {

// The forward's argument checks, shared by the two entry points.
aboria_status check_dense_sum(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel, const double* params_host,
                              int32_t nparams, int32_t d, int64_t n_target, const void* xt, int64_t n_source,
                              const void* xs, const void* w, void* y) {
    aboria_status st = check_common(ctx, dtype, kernel, params_host, nparams, d, n_target, n_source);
    if (st != ABORIA_OK) return st;
    if (n_target == 0) return ABORIA_OK;
    if (!xt || !y || (n_source > 0 && (!xs || !w))) return fail(ctx, ABORIA_ERR_INVALID_ARG, "NULL array");
    const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
    const size_t ny = tsz * (size_t)n_target;
    if (overlaps(y, ny, xt, tsz * d * (size_t)n_target) || overlaps(y, ny, xs, tsz * d * (size_t)n_source) ||
        overlaps(y, ny, w, tsz * (size_t)n_source))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "y overlaps an input");
    return ABORIA_OK;
}

}  // namespace

extern "C" aboria_status aboria_dense_sum(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                          const double* params_host, int32_t nparams, int32_t d, int64_t n_target,
                                          const void* xt, int64_t n_source, const void* xs, const void* w, void* y) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        aboria_status st =
            check_dense_sum(ctx, dtype, kernel, params_host, nparams, d, n_target, xt, n_source, xs, w, y);
        if (st != ABORIA_OK || n_target == 0) return st;
        const int32_t plan = dense_plan_for(ctx, dense_key(false, kernel, dtype, d, n_target, n_source), dtype);
        return dispatch<kSum>(ctx, dtype, d, kernel, (uint32_t)n_target, xt, (uint32_t)n_source, xs, w,
                              params_host[0], nullptr, y, nullptr, nullptr, 0, plan);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in dense_sum");
    }
}

extern "C" aboria_status aboria_dense_sum_noalloc(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                                  const double* params_host, int32_t nparams, int32_t d,
                                                  int64_t n_target, const void* xt, int64_t n_source,
                                                  const void* xs, const void* w, void* y) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        aboria_status st =
            check_dense_sum(ctx, dtype, kernel, params_host, nparams, d, n_target, xt, n_source, xs, w, y);
        if (st != ABORIA_OK || n_target == 0) return st;
        const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
        if ((size_t)n_target * tsz > kNoAllocScratchBytes)
            return fail(ctx, ABORIA_ERR_INVALID_ARG,
                        "n_target too large for the no-allocation scratch (" +
                            std::to_string(kNoAllocScratchBytes / tsz) + " targets at most)");
        void* part = nullptr;
        if ((st = noalloc_scratch(ctx, &part)) != ABORIA_OK) return st;
        const int32_t plan = dense_plan_for(ctx, dense_key(false, kernel, dtype, d, n_target, n_source), dtype);
        return dispatch<kSum>(ctx, dtype, d, kernel, (uint32_t)n_target, xt, (uint32_t)n_source, xs, w,
                              params_host[0], nullptr, y, nullptr, part, kNoAllocScratchBytes, plan);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in dense_sum_noalloc");
    }
}

extern "C" aboria_status aboria_dense_sum_backward(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                                   const double* params_host, int32_t nparams, int32_t d,
                                                   int64_t n_target, const void* xt, int64_t n_source,
                                                   const void* xs, const void* w, const void* gy, void* gxt,
                                                   void* gxs, void* gw) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        aboria_status st = check_common(ctx, dtype, kernel, params_host, nparams, d, n_target, n_source);
        if (st != ABORIA_OK) return st;
        if (n_target == 0 || n_source == 0) {
            // no pairs: every requested gradient is zero (a fill kernel, so the call stays capturable)
            const int64_t words = dtype == ABORIA_F32 ? 1 : 2;
            if (gxt && n_target > 0 && (st = fill_u32(ctx, (uint32_t*)gxt, 0u, words * d * n_target)) != ABORIA_OK)
                return st;
            if (gxs && n_source > 0 && (st = fill_u32(ctx, (uint32_t*)gxs, 0u, words * d * n_source)) != ABORIA_OK)
                return st;
            if (gw && n_source > 0 && (st = fill_u32(ctx, (uint32_t*)gw, 0u, words * n_source)) != ABORIA_OK)
                return st;
            return ABORIA_OK;
        }
        if (!xt || !xs || !w || !gy) return fail(ctx, ABORIA_ERR_INVALID_ARG, "NULL input array");
        const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
        const size_t nt = (size_t)n_target, ns = (size_t)n_source;
        struct Span { const void* p; size_t bytes; };
        const Span ins[] = {{xt, tsz * d * nt}, {xs, tsz * d * ns}, {w, tsz * ns}, {gy, tsz * nt}};
        const Span outs[] = {{gxt, tsz * d * nt}, {gxs, tsz * d * ns}, {gw, tsz * ns}};
        for (const Span& o : outs) {
            if (!o.p) continue;
            for (const Span& i : ins)
                if (overlaps(o.p, o.bytes, i.p, i.bytes))
                    return fail(ctx, ABORIA_ERR_INVALID_ARG, "an output overlaps an input");
            for (const Span& o2 : outs)
                if (&o2 != &o && o2.p && overlaps(o.p, o.bytes, o2.p, o2.bytes))
                    return fail(ctx, ABORIA_ERR_INVALID_ARG, "outputs overlap");
        }
        const double prm = params_host[0];
        const uint32_t t32 = (uint32_t)n_target, s32 = (uint32_t)n_source;
        const int32_t plan = dense_plan_for(ctx, dense_key(true, kernel, dtype, d, n_target, n_source), dtype);
        // dL/dw = K^T gy (the forward sum over the targets, seen from the sources) and the
        // source-position gradient sum over the same pairs with the same weights gy: one
        // pass when both are requested
        if (gw && gxs) {
            if ((st = dispatch<kSumGrad>(ctx, dtype, d, kernel, s32, xs, t32, xt, gy, prm, w, gw, gxs, nullptr, 0,
                                         plan)) != ABORIA_OK)
                return st;
        } else if (gw) {
            if ((st = dispatch<kSum>(ctx, dtype, d, kernel, s32, xs, t32, xt, gy, prm, nullptr, gw, nullptr, nullptr,
                                     0, plan)) != ABORIA_OK)
                return st;
        } else if (gxs) {
            if ((st = dispatch<kGrad>(ctx, dtype, d, kernel, s32, xs, t32, xt, gy, prm, w, gxs, nullptr, nullptr, 0,
                                      plan)) != ABORIA_OK)
                return st;
        }
        if (gxt && (st = dispatch<kGrad>(ctx, dtype, d, kernel, t32, xt, s32, xs, w, prm, gy, gxt, nullptr, nullptr,
                                         0, plan)) != ABORIA_OK)
            return st;
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in dense_sum_backward");
    }
}

extern "C" aboria_status aboria_set_dense_plan(aboria_ctx* ctx, int32_t plan) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (plan < -1 || plan >= kNumDensePlans) return fail(ctx, ABORIA_ERR_INVALID_ARG, "no such dense plan");
    ctx->dense_plan_forced = plan;
    return ABORIA_OK;
}

extern "C" const char* aboria_dense_plan_name(int32_t plan) {
    return plan >= 0 && plan < kNumDensePlans ? kDensePlans[plan].name : "";
}

extern "C" aboria_status aboria_autotune_dense(aboria_ctx* ctx, aboria_dtype dtype, aboria_kernel kernel,
                                               const double* params_host, int32_t nparams, int32_t d,
                                               int64_t n_target, const void* xt, int64_t n_source, const void* xs,
                                               const void* w, const void* gy, void* scratch, int32_t* choice_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "autotune cannot be captured");
    try {
        aboria_status st = check_common(ctx, dtype, kernel, params_host, nparams, d, n_target, n_source);
        if (st != ABORIA_OK) return st;
        if (n_target == 0 || n_source == 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "nothing to time: no pairs");
        if (!xt || !xs || !w || !scratch) return fail(ctx, ABORIA_ERR_INVALID_ARG, "NULL array");
        const bool backward = gy != nullptr;
        const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
        char* sc = static_cast<char*>(scratch);
        void* gxt = sc;
        void* gxs = sc + tsz * (size_t)d * (size_t)n_target;
        void* gw = sc + tsz * (size_t)d * (size_t)(n_target + n_source);
        auto run = [&]() {
            return backward ? aboria_dense_sum_backward(ctx, dtype, kernel, params_host, nparams, d, n_target, xt,
                                                        n_source, xs, w, gy, gxt, gxs, gw)
                            : aboria_dense_sum(ctx, dtype, kernel, params_host, nparams, d, n_target, xt, n_source,
                                               xs, w, scratch);
        };
        ABORIA_HIP(ctx, hipSetDevice(ctx->device));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return hip_fail(ctx, hipGetLastError(), "hipEventCreate");
        }
        double best_ms = INFINITY;
        int32_t best = 0;
        const int32_t forced_before = ctx->dense_plan_forced;
        for (int32_t p = 0; p < kNumDensePlans && st == ABORIA_OK; ++p) {
            if (!dense_plan_ok(p, dtype)) continue;
            ctx->dense_plan_forced = p;
            if ((st = run()) != ABORIA_OK) break;  // warm-up
            (void)hipEventRecord(e0, ctx->stream);
            for (int rep = 0; rep < 3 && st == ABORIA_OK; ++rep) st = run();
            (void)hipEventRecord(e1, ctx->stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = hip_fail(ctx, hipGetLastError(), "timing a dense plan");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            log_msg("autotune_dense: %s %.4f ms", kDensePlans[p].name, ms / 3.0);
            if (ms < best_ms) {
                best_ms = ms;
                best = p;
            }
        }
        ctx->dense_plan_forced = forced_before;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != ABORIA_OK) return st;
        const uint64_t key = dense_key(backward, kernel, dtype, d, n_target, n_source);
        const aboria_ctx::DenseChoice ch{kDensePlans[best].ti, kDensePlans[best].wg};
        bool found = false;
        for (auto& kv : ctx->dense_cache)
            if (kv.first == key) {
                kv.second = ch;
                found = true;
            }
        if (!found) ctx->dense_cache.emplace_back(key, ch);
        tune_cache_save(ctx);
        log_msg("autotune_dense: %s chosen", kDensePlans[best].name);
        if (choice_host) *choice_host = best;
        return ABORIA_OK;
    } catch (...) {
        ctx->dense_plan_forced = -1;
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in autotune_dense");
    }
}
