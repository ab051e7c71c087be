// Autotuner for the neighbour-sum launch: times every work-mapping variant on
// the caller's cell list with HIP events on the context's stream and caches the
// fastest per (d, dtype, operator, direction, size bucket, density bucket,
// batch, neighbour list recorded).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace aboria {

uint64_t tune_key(const aboria_cells* c, int32_t op, bool backward) {
    const int64_t n = std::max<int64_t>(c->n, 1);
    const int size_bucket = (int)std::floor(std::log2((double)n));
    const double per_cell = (double)c->n / (double)std::max<int64_t>(c->ncells, 1);
    const int dens_bucket = (int)std::floor(2.0 * std::log2(per_cell + 1.0));
    uint64_t k = (uint64_t)c->d;
    k = k * 4 + (uint64_t)c->dtype;
    k = k * 16 + (uint64_t)op;
    k = k * 64 + (uint64_t)size_bucket;
    k = k * 64 + (uint64_t)std::min(dens_bucket, 63);
    k = k * 2 + (uint64_t)(c->nsys > 1);
    k = k * 2 + (uint64_t)backward;
    k = k * 2 + (uint64_t)c->nbr_recorded;
    return k;
}

int32_t pick_variant(aboria_ctx* ctx, const aboria_cells* c, int32_t op, bool backward) {
    if (ctx->variant_forced >= 0) return ctx->variant_forced;
    const uint64_t key = tune_key(c, op, backward);
    for (const auto& kv : ctx->tune_cache)
        if (kv.first == key) return kv.second;
    // untuned: all pairs for small systems, else the recorded list when there is one
    return default_variant(c);
}

}  // namespace aboria

using namespace aboria;

extern "C" int32_t aboria_variant_count(void) { return variant_count(); }

extern "C" const char* aboria_variant_name(int32_t v) { return variant_name(v); }

extern "C" aboria_status aboria_set_variant(aboria_ctx* ctx, int32_t v) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (v < -1 || v >= variant_count()) return fail(ctx, ABORIA_ERR_INVALID_ARG, "no such variant");
    ctx->variant_forced = v;
    return ABORIA_OK;
}

extern "C" aboria_status aboria_autotune(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                         const double* params_host, int32_t nparams, const void* a, int32_t na,
                                         const void* gy, int32_t ny, void* out_scratch, int32_t* choice_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!cells) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells is NULL");
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "autotune cannot be captured");
    try {
        ABORIA_HIP(ctx, hipSetDevice(ctx->device));
        hipEvent_t e0, e1;
        ABORIA_HIP(ctx, hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(ctx, ABORIA_ERR_DEVICE, "hipEventCreate failed");
        }
        const int reps = 5;
        int32_t best = 0;
        float best_ms = INFINITY;
        aboria_status st = ABORIA_OK;
        const bool backward = gy != nullptr;
        auto run = [&](int32_t v) {
            return backward ? pair_bwd_impl(ctx, cells, op, params_host, nparams, a, na, gy, ny, out_scratch,
                                            nullptr, v)
                            : pair_sum_impl(ctx, cells, op, params_host, nparams, a, na, out_scratch, ny, v);
        };
        for (int32_t v = 0; v < variant_count() && st == ABORIA_OK; ++v) {
            if (!variant_usable(v, cells)) continue;
            if (!variant_worth_timing(v, cells)) continue;
            st = run(v);  // warm-up
            if (st != ABORIA_OK) break;
            std::vector<float> times;
            for (int r = 0; r < reps && st == ABORIA_OK; ++r) {
                if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = ABORIA_ERR_DEVICE; break; }
                st = run(v);
                if (st != ABORIA_OK) break;
                if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = ABORIA_ERR_DEVICE;
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                times.push_back(ms);
            }
            if (st != ABORIA_OK) break;
            std::sort(times.begin(), times.end());
            const float med = times[times.size() / 2];
            if (med < best_ms) {
                best_ms = med;
                best = v;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != ABORIA_OK) {
            if (ctx->last_error.empty()) ctx->last_error = "autotune: a trial failed";
            return st;
        }
        const uint64_t key = tune_key(cells, op, backward);
        bool found = false;
        for (auto& kv : ctx->tune_cache)
            if (kv.first == key) { kv.second = best; found = true; }
        if (!found) ctx->tune_cache.emplace_back(key, best);
        if (choice_host) *choice_host = best;
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in autotune");
    }
}
