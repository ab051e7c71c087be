// Radius-limited neighbour sums over the cell list: host dispatch, argument
// validation and the C-ABI entry points of the forward, the adjoint and the
// pair listing.  The kernels live in pair_lane_*.hip, pair_mask.hip,
// pair_flat_*.hip, pair_nbr*.hip and pair_allpairs.hip (see pair_common.hpp for
// the shared device code).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "pair_common.hpp"

namespace aboria {

constexpr int kPairBlock = 256;

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
    auto visit = [&](uint32_t j, const T*, T, bool) {
        if (FILL) {
            const uint64_t at = base + cnt;
            if (at < cap) {
                pi[at] = me;
                pj[at] = perm[j];
            }
        }
        ++cnt;
    };
    neighbour_loop<T, D>(P, xs, off, n, xi, visit);
    if (!FILL) counts[s] = cnt;
}

// dst[s][:] = src[perm[s]][:] for rows of W elements (W <= 4), written with a
// row pitch of WP elements (3-wide rows are padded to 4, zero-filled, so that
// the sums load a row with one vector load): one thread per row.
template <typename T, int W, int WP>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ src, const uint32_t* __restrict__ perm,
                                                     uint32_t n, T* __restrict__ dst) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t p = perm[s];
    VecN<T, WP> v;
#pragma unroll
    for (int k = 0; k < WP; ++k) v.v[k] = k < W ? src[(size_t)p * W + k] : T(0);
    reinterpret_cast<VecN<T, WP>*>(dst)[s] = v;
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------

namespace {

template <typename T>
aboria_status gather(aboria_ctx* ctx, const aboria_cells* c, const void* src, int w, void* dst) {
    const uint32_t n = (uint32_t)c->n;
    if (n == 0 || w == 0) return ABORIA_OK;
    const dim3 grid((n + 255) / 256);
    const T* s = (const T*)src;
    T* d = (T*)dst;
    switch (w) {
        case 1: hipLaunchKernelGGL((k_gather_rows<T, 1, 1>), grid, dim3(256), 0, ctx->stream, s, c->perm, n, d); break;
        case 2: hipLaunchKernelGGL((k_gather_rows<T, 2, 2>), grid, dim3(256), 0, ctx->stream, s, c->perm, n, d); break;
        case 3: hipLaunchKernelGGL((k_gather_rows<T, 3, 4>), grid, dim3(256), 0, ctx->stream, s, c->perm, n, d); break;
        default: hipLaunchKernelGGL((k_gather_rows<T, 4, 4>), grid, dim3(256), 0, ctx->stream, s, c->perm, n, d); break;
    }
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

// Work-mapping variants of the neighbour sums.
struct Variant {
    int kind;   // 0 = lane per particle, 2 = recorded neighbour list, 3 = all pairs,
                // 5 = flattened pruned search, 6 = lane per particle with recorded
                // accepted-pair masks, 7 = half stencil (forward; the adjoint is kind 0's)
    int block;  // threads per workgroup
    const char* name;
};

const Variant kVariants[] = {
    {0, 256, "lane per particle, 256-thread workgroups, adjoint evaluated on every candidate"},
    {2, 256, "lane per particle over the recorded neighbour list (accepted pairs only)"},
    {3, 256, "lane per particle over all particles of its system (minimum image; small systems)"},
    {5, 256, "lane per particle, flattened box search over pruned slot ranges listed in LDS"},
    {6, 256, "lane per particle, forward records accepted-pair bit masks per stencil row, adjoint replays them"},
    {7, 256, "lane per particle, half stencil: each pair tested once, the partner reads the recorded bit"},
};

// Modes of the flattened kernel (pair_flat.hpp).
constexpr int kFlatModeFwd = 0, kFlatModeBwd = 1, kFlatModeFused = 2;

// Largest system the all-pairs variant accepts (its lanes test every particle of their system).
constexpr int64_t kAllPairsMaxSystem = 16384;

// Largest search reach over the systems of a cell list in dimension k.
int32_t max_reach(const aboria_cells* c, int k) {
    int32_t m = 1;
    for (const aboria_box& b : c->boxes)
        if (k < b.d) m = std::max<int32_t>(m, b.reach[k] == 0 ? 1 : b.reach[k]);
    return m;
}

// Reach 1 in every dimension but x: the search has the 3^(d-1) rows of the
// paper's stencil (each row may span more, narrower cells along x).
bool rows_reach1(const aboria_cells* c) { return max_reach(c, 1) == 1 && max_reach(c, 2) == 1; }

// Variants with their own box-search loops, written for the 3^d stencil: the
// mask variant for its rows, the others for every cell of it.
// Every system's grid at least 2 m + 1 cells wide in x (m its x reach): each x
// offset of a stencil row is then one distinct cell.
bool wide_x(const aboria_cells* c) {
    for (int32_t b = 0; b < c->nsys; ++b) {
        const int32_t m = c->boxes[(size_t)b].reach[0] == 0 ? 1 : c->boxes[(size_t)b].reach[0];
        if (c->ncell_host[(size_t)b * 3] < 2 * m + 1) return false;
    }
    return true;
}

bool reach_ok(const Variant& v, const aboria_cells* c) {
    if (v.kind == 6) return rows_reach1(c);
    if (v.kind == 7) return rows_reach1(c) && wide_x(c);
    return true;
}

int64_t largest_system(const aboria_cells* c) {
    int64_t m = 0;
    for (int32_t b = 0; b < c->nsys; ++b) m = std::max<int64_t>(m, c->sys_off[(size_t)b + 1] - c->sys_off[(size_t)b]);
    return m;
}
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <typename T, int D, int OP, bool BATCH>
void launch_fwd_variant(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y,
                        const Variant& v) {
    if (v.kind == 6) launch_mask_fwd<T, D, OP, BATCH>(ctx, c, q, a_s, y);
    else if (v.kind == 7) launch_half_fwd<T, D, OP, BATCH>(ctx, c, q, a_s, y);
    else if (v.kind == 5) launch_flat<T, D, OP, BATCH, kFlatModeFwd>(ctx, c, q, a_s, nullptr, y, nullptr, nullptr);
    else if (v.kind == 3) launch_all_fwd<T, D, OP, BATCH>(ctx, c, q, a_s, y);
    else if (v.kind == 2) launch_nbr_fwd<T, D, OP, BATCH>(ctx, c, q, a_s, y);
    else launch_lane_fwd<T, D, OP, BATCH>(ctx, c, q, a_s, y, v.block);
}

template <typename T, int D, int OP, bool BATCH>
void launch_bwd_variant(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                        T* gx, T* ga, const Variant& v) {
    if (v.kind == 6) launch_mask_bwd<T, D, OP, BATCH>(ctx, c, q, a_s, gy_s, gx, ga);
    else if (v.kind == 5) launch_flat<T, D, OP, BATCH, kFlatModeBwd>(ctx, c, q, a_s, gy_s, nullptr, gx, ga);
    else if (v.kind == 3) launch_all_bwd<T, D, OP, BATCH>(ctx, c, q, a_s, gy_s, gx, ga);
    else if (v.kind == 2) launch_nbr_bwd<T, D, OP, BATCH>(ctx, c, q, a_s, gy_s, gx, ga);
    else launch_lane_bwd<T, D, OP, BATCH>(ctx, c, q, a_s, gy_s, gx, ga, v.block);
}

const Variant& variant_of(int variant) { return kVariants[(variant < 0 || variant >= kNumVariants) ? 0 : variant]; }

template <typename T, int D, int OP>
aboria_status launch_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int variant) {
    if (c->n == 0) return ABORIA_OK;
    if (c->nsys == 1) launch_fwd_variant<T, D, OP, false>(ctx, c, q, a_s, y, variant_of(variant));
    else launch_fwd_variant<T, D, OP, true>(ctx, c, q, a_s, y, variant_of(variant));
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D, int OP>
aboria_status launch_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                         T* gx, T* ga, int variant) {
    if (c->n == 0) return ABORIA_OK;
    if (c->nsys == 1) launch_bwd_variant<T, D, OP, false>(ctx, c, q, a_s, gy_s, gx, ga, variant_of(variant));
    else launch_bwd_variant<T, D, OP, true>(ctx, c, q, a_s, gy_s, gx, ga, variant_of(variant));
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D>
aboria_status fwd_op(aboria_ctx* ctx, const aboria_cells* c, int op, const OpArgs<T>& q, const T* a_s, T* y,
                     int variant) {
    switch (op) {
        case ABORIA_OP_COUNT: return launch_fwd<T, D, ABORIA_OP_COUNT>(ctx, c, q, a_s, y, variant);
        case ABORIA_OP_SPRING: return launch_fwd<T, D, ABORIA_OP_SPRING>(ctx, c, q, a_s, y, variant);
        case ABORIA_OP_SOFT_SPHERE: return launch_fwd<T, D, ABORIA_OP_SOFT_SPHERE>(ctx, c, q, a_s, y, variant);
        case ABORIA_OP_EXP_FORCE: return launch_fwd<T, D, ABORIA_OP_EXP_FORCE>(ctx, c, q, a_s, y, variant);
        default: return launch_fwd<T, D, ABORIA_OP_DEM_SPRING>(ctx, c, q, a_s, y, variant);
    }
}

template <typename T, int D>
aboria_status bwd_op(aboria_ctx* ctx, const aboria_cells* c, int op, const OpArgs<T>& q, const T* a_s,
                     const T* gy_s, T* gx, T* ga, int variant) {
    switch (op) {
        case ABORIA_OP_COUNT: return launch_bwd<T, D, ABORIA_OP_COUNT>(ctx, c, q, a_s, gy_s, gx, ga, variant);
        case ABORIA_OP_SPRING: return launch_bwd<T, D, ABORIA_OP_SPRING>(ctx, c, q, a_s, gy_s, gx, ga, variant);
        case ABORIA_OP_SOFT_SPHERE:
            return launch_bwd<T, D, ABORIA_OP_SOFT_SPHERE>(ctx, c, q, a_s, gy_s, gx, ga, variant);
        case ABORIA_OP_EXP_FORCE:
            return launch_bwd<T, D, ABORIA_OP_EXP_FORCE>(ctx, c, q, a_s, gy_s, gx, ga, variant);
        default: return launch_bwd<T, D, ABORIA_OP_DEM_SPRING>(ctx, c, q, a_s, gy_s, gx, ga, variant);
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

// Allocates the accepted-pair masks of a cell list on first use (status zeroed,
// so nothing counts as recorded until a recording forward runs).
aboria_status ensure_masks(aboria_ctx* ctx, const aboria_cells* cc) {
    aboria_cells* c = const_cast<aboria_cells*>(cc);
    if (c->masks || c->n == 0) return ABORIA_OK;
    if (ctx->capturing)
        return fail(ctx, ABORIA_ERR_UNSUPPORTED, "the mask variant allocates on first use and cannot be captured then");
    const size_t rows = c->d == 1 ? 1 : (c->d == 2 ? 3 : 9);
    const size_t nn = (size_t)c->n;
    if (hipMalloc((void**)&c->masks, sizeof(uint32_t) * 2 * rows * nn) != hipSuccess ||
        hipMalloc((void**)&c->mask_status, sizeof(uint32_t) * nn) != hipSuccess) {
        (void)hipGetLastError();
        if (c->masks) (void)hipFree(c->masks);
        if (c->mask_status) (void)hipFree(c->mask_status);
        c->masks = c->mask_status = nullptr;
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "device allocation for the pair masks failed");
    }
    return fill_u32(ctx, c->mask_status, 0u, (int64_t)nn);
}

aboria_status check_variant(aboria_ctx* ctx, const aboria_cells* c, int variant) {
    if (variant_needs_list(variant) && !c->nbr_recorded)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "the variant needs a neighbour list recorded on these cells");
    if (variant_of(variant).kind == 3 && largest_system(c) > kAllPairsMaxSystem)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "the all-pairs variant takes systems of at most 16384 particles");
    if (!reach_ok(variant_of(variant), c))
        return fail(ctx, ABORIA_ERR_INVALID_ARG,
                    variant_of(variant).kind == 7
                        ? "the variant needs reach 1 in every dimension but x and at least 2 m + 1 cells in x"
                        : "the variant needs reach 1 in every dimension but x");
    if (variant_of(variant).kind == 6 || variant_of(variant).kind == 7) return ensure_masks(ctx, c);
    return ABORIA_OK;
}

}  // namespace

int32_t variant_count() { return kNumVariants; }

const char* variant_name(int32_t v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : ""; }

bool variant_needs_list(int32_t v) { return v >= 0 && v < kNumVariants && kVariants[v].kind == 2; }

bool variant_worth_timing(int32_t v, const aboria_cells* c, bool backward) {
    (void)c;
    if (v < 0 || v >= kNumVariants) return false;
    // the mask-recording pair pays only across a forward and its adjoint, which the
    // tuner times separately: callers select it for both calls
    if (kVariants[v].kind == 6) return false;
    // the half stencil's adjoint is variant 0's
    if (kVariants[v].kind == 7 && backward) return false;
    return true;
}

bool variant_usable(int32_t v, const aboria_cells* c) {
    if (v < 0 || v >= kNumVariants) return false;
    if (!reach_ok(kVariants[v], c)) return false;
    if (kVariants[v].kind == 2) return c->nbr_recorded;
    if (kVariants[v].kind == 3) return largest_system(c) <= kAllPairsMaxSystem;
    return true;
}

int32_t list_variant() {
    for (int32_t v = 0; v < kNumVariants; ++v)
        if (kVariants[v].kind == 2) return v;
    return 0;
}

// Largest system for which an untuned sum tests all pairs instead of searching
// cells (the small-N switch; the autotuner decides for tuned cell lists).
constexpr int64_t kAllPairsDefaultMax = 2048;

int32_t flat_variant() {
    for (int32_t v = 0; v < kNumVariants; ++v)
        if (kVariants[v].kind == 5) return v;
    return 0;
}

int32_t default_variant(const aboria_cells* c) {
    if (largest_system(c) <= kAllPairsDefaultMax)
        for (int32_t v = 0; v < kNumVariants; ++v)
            if (kVariants[v].kind == 3) return v;
    if (c->nbr_recorded) return list_variant();
    // rows of the 3^d stencil (any x reach): the row search; deeper rows: the flattened search
    return rows_reach1(c) ? 0 : flat_variant();
}

aboria_status pair_sum_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, void* y, int32_t ny, int32_t variant) {
    aboria_status st = validate(ctx, c, op, params, nparams, a, na, ny);
    if (st != ABORIA_OK) return st;
    if ((st = check_variant(ctx, c, variant)) != ABORIA_OK) return st;
    if (c->n > 0 && !y) return fail(ctx, ABORIA_ERR_INVALID_ARG, "y is NULL");
    const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
    if (overlaps(y, tsz * ny * c->n, a, tsz * na * c->n))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "y overlaps a");
    if (c->dtype == ABORIA_F32) {
        OpArgs<float> q{nparams > 0 ? (float)params[0] : 0.f};
        const float* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<float>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const float*)c->work;
        }
        switch (c->d) {
            case 1: return fwd_op<float, 1>(ctx, c, op, q, a_s, (float*)y, variant);
            case 2: return fwd_op<float, 2>(ctx, c, op, q, a_s, (float*)y, variant);
            default: return fwd_op<float, 3>(ctx, c, op, q, a_s, (float*)y, variant);
        }
    } else {
        OpArgs<double> q{nparams > 0 ? params[0] : 0.0};
        const double* a_s = nullptr;
        if (na > 0) {
            if ((st = gather<double>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
            a_s = (const double*)c->work;
        }
        switch (c->d) {
            case 1: return fwd_op<double, 1>(ctx, c, op, q, a_s, (double*)y, variant);
            case 2: return fwd_op<double, 2>(ctx, c, op, q, a_s, (double*)y, variant);
            default: return fwd_op<double, 3>(ctx, c, op, q, a_s, (double*)y, variant);
        }
    }
}

aboria_status pair_bwd_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, const void* gy, int32_t ny, void* gx,
                            void* ga, int32_t variant) {
    aboria_status st = validate(ctx, c, op, params, nparams, a, na, ny);
    if (st != ABORIA_OK) return st;
    if ((st = check_variant(ctx, c, variant)) != ABORIA_OK) return st;
    if (c->n > 0 && (!gy || !gx)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "gy and gx are required");
    const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
    const size_t nb = (size_t)c->n;
    if (overlaps(gx, tsz * c->d * nb, gy, tsz * ny * nb) || overlaps(gx, tsz * c->d * nb, a, tsz * na * nb) ||
        overlaps(ga, tsz * na * nb, gy, tsz * ny * nb) || overlaps(ga, tsz * na * nb, a, tsz * na * nb) ||
        overlaps(ga, tsz * na * nb, gx, tsz * c->d * nb))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "outputs overlap inputs");
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
            case 1: return bwd_op<float, 1>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, variant);
            case 2: return bwd_op<float, 2>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, variant);
            default: return bwd_op<float, 3>(ctx, c, op, q, a_s, g_s, (float*)gx, (float*)ga, variant);
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
            case 1: return bwd_op<double, 1>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, variant);
            case 2: return bwd_op<double, 2>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, variant);
            default: return bwd_op<double, 3>(ctx, c, op, q, a_s, g_s, (double*)gx, (double*)ga, variant);
        }
    }
}

namespace {

template <typename T, int D>
aboria_status fused_op(aboria_ctx* ctx, const aboria_cells* c, int op, const OpArgs<T>& q, const T* a_s,
                       const T* gy_s, T* y, T* gx, T* ga, bool flat) {
    if (c->n == 0) return ABORIA_OK;
    const bool batch = c->nsys > 1;
#define F(OPC)                                                                                      \
    if (flat && batch) launch_flat<T, D, OPC, true, kFlatModeFused>(ctx, c, q, a_s, gy_s, y, gx, ga);   \
    else if (flat) launch_flat<T, D, OPC, false, kFlatModeFused>(ctx, c, q, a_s, gy_s, y, gx, ga);      \
    else if (batch) launch_lane_fused<T, D, OPC, true>(ctx, c, q, a_s, gy_s, y, gx, ga);                \
    else launch_lane_fused<T, D, OPC, false>(ctx, c, q, a_s, gy_s, y, gx, ga);
    switch (op) {
        case ABORIA_OP_COUNT: F(ABORIA_OP_COUNT) break;
        case ABORIA_OP_SPRING: F(ABORIA_OP_SPRING) break;
        case ABORIA_OP_SOFT_SPHERE: F(ABORIA_OP_SOFT_SPHERE) break;
        case ABORIA_OP_EXP_FORCE: F(ABORIA_OP_EXP_FORCE) break;
        default: F(ABORIA_OP_DEM_SPRING) break;
    }
#undef F
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T>
aboria_status fused_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params, int32_t nparams,
                         const void* a, int32_t na, const void* gy, int32_t ny, void* y, void* gx, void* ga,
                         bool flat) {
    OpArgs<T> q{nparams > 0 ? (T)params[0] : T(0)};
    aboria_status st;
    const T* a_s = nullptr;
    if (na > 0) {
        if ((st = gather<T>(ctx, c, a, na, c->work)) != ABORIA_OK) return st;
        a_s = (const T*)c->work;
    }
    if ((st = gather<T>(ctx, c, gy, ny, c->work2)) != ABORIA_OK) return st;
    const T* g_s = (const T*)c->work2;
    switch (c->d) {
        case 1: return fused_op<T, 1>(ctx, c, op, q, a_s, g_s, (T*)y, (T*)gx, (T*)ga, flat);
        case 2: return fused_op<T, 2>(ctx, c, op, q, a_s, g_s, (T*)y, (T*)gx, (T*)ga, flat);
        default: return fused_op<T, 3>(ctx, c, op, q, a_s, g_s, (T*)y, (T*)gx, (T*)ga, flat);
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
        const int32_t v = cells ? pick_variant(ctx, cells, op, false) : 0;
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
        const int32_t v = cells ? pick_variant(ctx, cells, op, true) : 0;
        return pair_bwd_impl(ctx, cells, op, params_host, nparams, a, na, gy, ny, gx, ga, v);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in pair_sum_backward");
    }
}

extern "C" aboria_status aboria_pair_sum_and_backward(aboria_ctx* ctx, const aboria_cells* c, aboria_op op,
                                                      const double* params_host, int32_t nparams, const void* a,
                                                      int32_t na, const void* gy, int32_t ny, void* y, void* gx,
                                                      void* ga) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        aboria_status st = validate(ctx, c, op, params_host, nparams, a, na, ny);
        if (st != ABORIA_OK) return st;
        if (c->n > 0 && (!gy || !y || !gx)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "gy, y and gx are required");
        const size_t tsz = c->dtype == ABORIA_F32 ? 4 : 8;
        const size_t nb = (size_t)c->n;
        struct Span { const void* p; size_t bytes; };
        const Span ins[] = {{a, tsz * na * nb}, {gy, tsz * ny * nb}};
        const Span outs[] = {{y, tsz * ny * nb}, {gx, tsz * c->d * nb}, {ga, tsz * na * nb}};
        for (const Span& o : outs) {
            if (!o.p) continue;
            for (const Span& i : ins)
                if (overlaps(o.p, o.bytes, i.p, i.bytes))
                    return fail(ctx, ABORIA_ERR_INVALID_ARG, "outputs overlap inputs");
            for (const Span& o2 : outs)
                if (&o2 != &o && o2.p && overlaps(o.p, o.bytes, o2.p, o2.bytes))
                    return fail(ctx, ABORIA_ERR_INVALID_ARG, "outputs overlap");
        }
        // one box search for both: the flattened one when the forward would use it
        const bool flat = variant_of(pick_variant(ctx, c, op, false)).kind == 5;
        return c->dtype == ABORIA_F32
                   ? fused_impl<float>(ctx, c, op, params_host, nparams, a, na, gy, ny, y, gx, ga, flat)
                   : fused_impl<double>(ctx, c, op, params_host, nparams, a, na, gy, ny, y, gx, ga, flat);
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in pair_sum_and_backward");
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
