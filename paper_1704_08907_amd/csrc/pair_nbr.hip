// Recorded neighbour lists: one box search per build that keeps each
// particle's accepted neighbours, so that the forward sums and the adjoints
// that follow on the same cell list evaluate accepted pairs only instead of
// repeating the pair test on every candidate of the 3^d cells (about 6.7
// candidates per accepted pair at 30 neighbours in 3-d).
//
// Layout: entry k of slot s at nbr[k * n + s] (a wave reads 64 consecutive
// words per entry), the neighbour's slot with kNbrShift set when the search
// reached it through an image shift, in box-search order, so a replayed sum
// adds its summands in the same order as the search kernels.  nbr_count[s] is
// the slot's full neighbour count; a slot with more neighbours than the list
// holds is summed by the box search when replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pair_common.hpp"

namespace aboria {

namespace {

constexpr uint32_t kMaxNbrCap = 4096;

template <typename T, int D, bool BATCH>
__global__ __launch_bounds__(256) void k_nbr_build(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                   uint32_t n, const SysParams<T>* __restrict__ sp,
                                                   const uint32_t* __restrict__ sys_part, int nsys,
                                                   uint32_t* __restrict__ nbr, uint32_t* __restrict__ nbr_count,
                                                   uint32_t cap, uint32_t* __restrict__ gen) {
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    if (s == 0) gen[1] = gen[0];  // the list now belongs to the latest build
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    uint32_t cnt = 0;
    uint32_t* p = nbr + s;
    const size_t stride = (size_t)n;
    auto visit = [&](uint32_t j, const T*, T, bool shifted) {
        if (cnt < cap) {
            *p = j | (shifted ? kNbrShift : 0u);
            p += stride;
        }
        ++cnt;
    };
    neighbour_loop<T, D>(P, xs, off, n, xi, visit);
    nbr_count[s] = cnt;
}

template <typename T, int D>
void launch_build_nbr(aboria_ctx* ctx, aboria_cells* c) {
    const uint32_t n = (uint32_t)c->n;
    const dim3 grid((n + 255) / 256);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_nbr_build<T, D, false>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs, c->off, n,
                           sp, c->sys_part_dev, c->nsys, c->nbr, c->nbr_count, c->nbr_cap, c->gen);
    else
        hipLaunchKernelGGL((k_nbr_build<T, D, true>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs, c->off, n,
                           sp, c->sys_part_dev, c->nsys, c->nbr, c->nbr_count, c->nbr_cap, c->gen);
}

// Entries per particle from the densest system: the mean neighbour count mu
// of a uniform system (its density times the volume of the cutoff ball) plus
// six standard deviations of a Poisson count and a margin.
uint32_t auto_capacity(const aboria_cells* c) {
    double mu = 0.0;
    for (int32_t b = 0; b < c->nsys; ++b) {
        const aboria_box& bx = c->boxes[(size_t)b];
        const double nb = (double)(c->sys_off[(size_t)b + 1] - c->sys_off[(size_t)b]);
        double vol = 1.0;
        for (int k = 0; k < c->d; ++k) vol *= bx.hi[k] - bx.lo[k];
        const double r = bx.cutoff;
        const double ball = c->d == 1 ? 2.0 * r : (c->d == 2 ? M_PI * r * r : 4.0 / 3.0 * M_PI * r * r * r);
        if (vol > 0.0) mu = std::max(mu, nb / vol * ball);
    }
    const double want = std::ceil(mu + 6.0 * std::sqrt(mu) + 8.0);
    uint32_t cap = (uint32_t)std::min<double>(want, (double)kMaxNbrCap);
    cap = (cap + 7u) & ~7u;
    return std::max<uint32_t>(cap, 8u);
}

}  // namespace

}  // namespace aboria

using namespace aboria;

extern "C" aboria_status aboria_build_neighbours(aboria_ctx* ctx, aboria_cells* c, int32_t capacity) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!c) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (c->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells belong to another device");
    if (capacity < 0 || capacity > (int32_t)kMaxNbrCap)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "capacity must be in 0..4096");
    try {
        uint32_t cap = capacity > 0 ? (uint32_t)capacity : auto_capacity(c);
        if (c->nbr_count) {
            // the buffers are fixed once allocated (graphs may hold them)
            if (cap > (uint32_t)c->nbr_alloc) {
                if (capacity > 0)
                    return fail(ctx, ABORIA_ERR_INVALID_ARG,
                                "capacity exceeds the one the list of these cells was allocated with");
                cap = (uint32_t)c->nbr_alloc;
            }
        } else {
            if (ctx->capturing)
                return fail(ctx, ABORIA_ERR_UNSUPPORTED, "a first neighbour list allocates and cannot be captured");
            ABORIA_HIP(ctx, hipSetDevice(ctx->device));
            const size_t nn = (size_t)std::max<int64_t>(c->n, 1);
            if (hipMalloc((void**)&c->nbr, sizeof(uint32_t) * nn * cap) != hipSuccess ||
                hipMalloc((void**)&c->nbr_count, sizeof(uint32_t) * nn) != hipSuccess) {
                (void)hipGetLastError();
                if (c->nbr) (void)hipFree(c->nbr);
                if (c->nbr_count) (void)hipFree(c->nbr_count);
                c->nbr = c->nbr_count = nullptr;
                return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "device allocation for the neighbour list failed");
            }
            c->nbr_alloc = cap;
        }
        c->nbr_cap = cap;
        if (c->n > 0) {
            if (c->dtype == ABORIA_F32) {
                switch (c->d) {
                    case 1: launch_build_nbr<float, 1>(ctx, c); break;
                    case 2: launch_build_nbr<float, 2>(ctx, c); break;
                    default: launch_build_nbr<float, 3>(ctx, c); break;
                }
            } else {
                switch (c->d) {
                    case 1: launch_build_nbr<double, 1>(ctx, c); break;
                    case 2: launch_build_nbr<double, 2>(ctx, c); break;
                    default: launch_build_nbr<double, 3>(ctx, c); break;
                }
            }
            ABORIA_HIP(ctx, hipGetLastError());
        }
        c->nbr_recorded = true;
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in build_neighbours");
    }
}

extern "C" int32_t aboria_neighbour_capacity(const aboria_cells* c) {
    return (c && c->nbr_recorded) ? (int32_t)c->nbr_cap : 0;
}
