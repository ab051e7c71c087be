// Autotuner for the neighbour-sum launch: times every work-mapping variant on
// the caller's cell list with HIP events on the context's stream and caches the
// fastest per (d, dtype, operator, direction, size bucket, density bucket,
// batch, neighbour list recorded, search reach); and the cell-size tuner, which
// times rebuild + sums over search reaches and cell counts.  With the
// environment variable ABORIA_TUNE_CACHE naming a file, both caches persist:
// the file is read when a context is created and rewritten after every tuning
// call.  It is JSON with one entry per line, variants stored by name (so a
// library whose variant numbering differs skips what it does not know) and
// the whole file tied to the device architecture it was measured on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
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
    int32_t reach[3] = {1, 1, 1};
    for (const aboria_box& b : c->boxes)
        for (int q = 0; q < b.d; ++q) reach[q] = std::max<int32_t>(reach[q], b.reach[q] == 0 ? 1 : b.reach[q]);
    k = k * 32 + (uint64_t)((reach[0] - 1) + 3 * (reach[1] - 1) + 9 * (reach[2] - 1));
    return k;
}

void tune_cache_load(aboria_ctx* ctx) {
    if (ctx->cache_path.empty()) return;
    FILE* f = std::fopen(ctx->cache_path.c_str(), "r");
    if (!f) return;
    char line[1024];
    bool arch_ok = false;
    int nv = 0, nc = 0, nd = 0, nb = 0;
    while (std::fgets(line, sizeof line, f)) {
        const char* a = std::strstr(line, "\"arch\": \"");
        if (a) {
            a += 9;
            const char* e = std::strchr(a, '"');
            arch_ok = e && std::string(a, e) == ctx->arch;
            continue;
        }
        if (!arch_ok) continue;
        unsigned long long key = 0;
        char name[512];
        int m0, m1, m2;
        double factor;
        if (std::sscanf(line, " {\"key\": %llu, \"variant\": \"%511[^\"]\"}", &key, name) == 2) {
            for (int32_t v = 0; v < variant_count(); ++v)
                if (std::strcmp(variant_name(v), name) == 0) {
                    ctx->tune_cache.emplace_back((uint64_t)key, v);
                    ++nv;
                }
        } else if (std::sscanf(line, " {\"key\": %llu, \"reach\": [%d, %d, %d], \"factor\": %lf}", &key, &m0, &m1,
                               &m2, &factor) == 5) {
            aboria_ctx::CellsChoice ch{{m0, m1, m2}, factor};
            ctx->cells_cache.emplace_back((uint64_t)key, ch);
            ++nc;
        } else if (std::sscanf(line, " {\"key\": %llu, \"dense_plan\": [%d, %d]}", &key, &m0, &m1) == 3) {
            ctx->dense_cache.emplace_back((uint64_t)key, aboria_ctx::DenseChoice{m0, m1});
            ++nd;
        } else if (std::sscanf(line, " {\"key\": %llu, \"build\": [%d, %d, %d]}", &key, &m0, &m1, &m2) == 4) {
            ctx->build_cache.emplace_back((uint64_t)key, aboria_ctx::BuildShape{m0, m1, m2});
            ++nb;
        }
    }
    std::fclose(f);
    log_msg("tune cache %s: %d variant, %d cell-size, %d dense and %d build entries for %s", ctx->cache_path.c_str(),
            nv, nc, nd, nb, ctx->arch.c_str());
}

void tune_cache_save(aboria_ctx* ctx) {
    if (ctx->cache_path.empty()) return;
    const std::string tmp = ctx->cache_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) {
        log_msg("tune cache %s: cannot write", ctx->cache_path.c_str());
        return;
    }
    std::fprintf(f, "{\"format\": 1,\n\"arch\": \"%s\",\n\"variants\": [\n", ctx->arch.c_str());
    for (size_t i = 0; i < ctx->tune_cache.size(); ++i)
        std::fprintf(f, "{\"key\": %" PRIu64 ", \"variant\": \"%s\"}%s\n", ctx->tune_cache[i].first,
                     variant_name(ctx->tune_cache[i].second), i + 1 < ctx->tune_cache.size() ? "," : "");
    std::fprintf(f, "],\n\"cells\": [\n");
    for (size_t i = 0; i < ctx->cells_cache.size(); ++i) {
        const aboria_ctx::CellsChoice& ch = ctx->cells_cache[i].second;
        std::fprintf(f, "{\"key\": %" PRIu64 ", \"reach\": [%d, %d, %d], \"factor\": %.17g}%s\n",
                     ctx->cells_cache[i].first, ch.reach[0], ch.reach[1], ch.reach[2], ch.factor,
                     i + 1 < ctx->cells_cache.size() ? "," : "");
    }
    std::fprintf(f, "],\n\"dense\": [\n");
    for (size_t i = 0; i < ctx->dense_cache.size(); ++i)
        std::fprintf(f, "{\"key\": %" PRIu64 ", \"dense_plan\": [%d, %d]}%s\n", ctx->dense_cache[i].first,
                     ctx->dense_cache[i].second.ti, ctx->dense_cache[i].second.wg,
                     i + 1 < ctx->dense_cache.size() ? "," : "");
    std::fprintf(f, "],\n\"build\": [\n");
    for (size_t i = 0; i < ctx->build_cache.size(); ++i)
        std::fprintf(f, "{\"key\": %" PRIu64 ", \"build\": [%d, %d, %d]}%s\n", ctx->build_cache[i].first,
                     ctx->build_cache[i].second.ipt, ctx->build_cache[i].second.low_bits,
                     ctx->build_cache[i].second.shuffle, i + 1 < ctx->build_cache.size() ? "," : "");
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), ctx->cache_path.c_str()) != 0)
        log_msg("tune cache %s: cannot replace", ctx->cache_path.c_str());
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
            if (!variant_worth_timing(v, cells, gy != nullptr)) continue;
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
        log_msg("autotune %s (op %d, n %" PRId64 "): %s, %.4f ms", backward ? "adjoint" : "forward", (int)op,
                cells->n, variant_name(best), (double)best_ms);
        tune_cache_save(ctx);
        if (choice_host) *choice_host = best;
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in autotune");
    }
}

extern "C" aboria_status aboria_autotune_cells(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys,
                                               const aboria_box* boxes_host, const int64_t* offsets_host,
                                               const void* x, aboria_op op, const double* params_host,
                                               int32_t nparams, const void* a, int32_t na, const void* gy,
                                               int32_t ny, aboria_box* boxes_out, double* factor_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "autotune cannot be captured");
    if (nsys < 1 || !boxes_host || !offsets_host || !boxes_out)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "need nsys >= 1, boxes, offsets and boxes_out");
    if (dtype != ABORIA_F32 && dtype != ABORIA_F64) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown dtype");
    const int32_t d = boxes_host[0].d;
    if (d < 1 || d > 3) return fail(ctx, ABORIA_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (op_ny(op, d) != ny) return fail(ctx, ABORIA_ERR_INVALID_ARG, "ny does not match the operator");
    try {
        // cache key: (d, dtype, operator, adjoint timed, batch, caller's reach, size
        // bucket of the total, density bucket of the mean particles per cutoff cube)
        const int64_t ntot = offsets_host[nsys];
        double dens = 0.0;
        for (int32_t b = 0; b < nsys; ++b) {
            double vol = 1.0;
            for (int k = 0; k < d; ++k) vol *= (boxes_host[b].hi[k] - boxes_host[b].lo[k]) / boxes_host[b].cutoff;
            dens += (double)(offsets_host[b + 1] - offsets_host[b]) / std::max(vol, 1e-300);
        }
        dens /= nsys;
        uint64_t ckey = (uint64_t)d;
        ckey = ckey * 4 + (uint64_t)dtype;
        ckey = ckey * 16 + (uint64_t)op;
        ckey = ckey * 2 + (uint64_t)(gy != nullptr);
        ckey = ckey * 2 + (uint64_t)(nsys > 1);
        for (int k = 0; k < 3; ++k) ckey = ckey * 8 + (uint64_t)std::min<int32_t>(7, std::max(0, boxes_host[0].reach[k]));
        ckey = ckey * 64 + (uint64_t)std::floor(std::log2((double)std::max<int64_t>(ntot, 1)));
        ckey = ckey * 64 + (uint64_t)std::min(63.0, std::max(0.0, std::floor(2.0 * std::log2(dens + 1.0))));
        for (const auto& kv : ctx->cells_cache) {
            if (kv.first != ckey) continue;
            // a cached choice: the grid of that reach, coarsened by the factor
            for (int32_t b = 0; b < nsys; ++b) {
                aboria_box bx = boxes_host[b];
                for (int k = 0; k < 3; ++k) bx.reach[k] = kv.second.reach[k];
                int32_t base[3];
                aboria_status st = grid_counts(ctx, dtype, bx, base);
                if (st != ABORIA_OK) return st;
                for (int k = 0; k < 3; ++k)
                    bx.ncell[k] = k < d ? std::max<int32_t>(1, (int32_t)std::floor(kv.second.factor * base[k])) : 0;
                boxes_out[b] = bx;
            }
            if (factor_host) *factor_host = kv.second.factor;
            log_msg("autotune_cells: cached reach {%d, %d, %d}, factor %.2f", kv.second.reach[0], kv.second.reach[1],
                    kv.second.reach[2], kv.second.factor);
            return ABORIA_OK;
        }
        // reaches to try: the caller's, or, when the boxes leave it to the library,
        // 1, 2 and 3 in every dimension and (d >= 2) 2 and 3 along x only
        struct Reach {
            int32_t m[3];
        };
        std::vector<Reach> reaches;
        const int32_t* r0 = boxes_host[0].reach;
        if (r0[0] != 0 || r0[1] != 0 || r0[2] != 0) {
            reaches.push_back({{r0[0], r0[1], r0[2]}});
        } else {
            for (int32_t m = 1; m <= kMaxReach; ++m) reaches.push_back({{m, m, m}});
            if (d >= 2)
                for (int32_t m = 2; m <= kMaxReach; ++m) reaches.push_back({{m, 1, 1}});
        }
        const int64_t n = offsets_host[nsys];
        const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
        ABORIA_HIP(ctx, hipSetDevice(ctx->device));
        void* y = nullptr;
        void* gx = nullptr;
        const size_t nn = (size_t)std::max<int64_t>(n, 1);
        if (hipMalloc(&y, tsz * nn * (size_t)std::max(ny, 1)) != hipSuccess ||
            hipMalloc(&gx, tsz * nn * (size_t)d) != hipSuccess) {
            (void)hipGetLastError();
            if (y) (void)hipFree(y);
            return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "autotune scratch allocation failed");
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        aboria_status st = ABORIA_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = ABORIA_ERR_DEVICE;
        const double factors[] = {1.0, 0.85, 0.7, 0.55};
        double best_ms = INFINITY, best_f = 1.0;
        std::vector<aboria_box> trial(boxes_host, boxes_host + nsys), best_boxes(trial);
        for (const Reach& R : reaches) {
            // the grid every trial of this reach coarsens: the automatic (or given explicit) counts
            std::vector<int32_t> base((size_t)nsys * 3, 1);
            for (int32_t b = 0; b < nsys && st == ABORIA_OK; ++b) {
                aboria_box bx = boxes_host[b];
                for (int k = 0; k < 3; ++k) bx.reach[k] = R.m[k];
                st = grid_counts(ctx, dtype, bx, &base[(size_t)b * 3]);
            }
            if (st != ABORIA_OK && reaches.size() > 1) {  // explicit counts too fine for this reach
                st = ABORIA_OK;
                ctx->last_error.clear();
                continue;
            }
            std::vector<int32_t> last;
            for (double f : factors) {
                if (st != ABORIA_OK) break;
                std::vector<int32_t> counts(base.size());
                for (size_t i = 0; i < base.size(); ++i)
                    counts[i] = std::max<int32_t>(1, (int32_t)std::floor(f * base[i]));
                if (counts == last) continue;  // the same grid as the previous factor
                last = counts;
                for (int32_t b = 0; b < nsys; ++b) {
                    for (int k = 0; k < 3; ++k) trial[(size_t)b].reach[k] = R.m[k];
                    for (int k = 0; k < 3; ++k) trial[(size_t)b].ncell[k] = k < d ? counts[(size_t)b * 3 + k] : 0;
                }
                aboria_cells* cells = nullptr;
                if ((st = aboria_build_cells(ctx, dtype, nsys, trial.data(), offsets_host, x, &cells)) != ABORIA_OK)
                    break;
                st = aboria_autotune(ctx, cells, op, params_host, nparams, a, na, nullptr, ny, y, nullptr);
                if (st == ABORIA_OK && gy)
                    st = aboria_autotune(ctx, cells, op, params_host, nparams, a, na, gy, ny, gx, nullptr);
                const int reps = 3;
                if (st == ABORIA_OK && hipEventRecord(e0, ctx->stream) != hipSuccess) st = ABORIA_ERR_DEVICE;
                for (int r = 0; r < reps && st == ABORIA_OK; ++r) {
                    st = aboria_build_cells(ctx, dtype, nsys, trial.data(), offsets_host, x, &cells);
                    if (st == ABORIA_OK) st = aboria_pair_sum(ctx, cells, op, params_host, nparams, a, na, y, ny);
                    if (st == ABORIA_OK && gy)
                        st = aboria_pair_sum_backward(ctx, cells, op, params_host, nparams, a, na, gy, ny, gx,
                                                      nullptr);
                }
                float ms = 0.f;
                if (st == ABORIA_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                                        hipEventSynchronize(e1) != hipSuccess ||
                                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = ABORIA_ERR_DEVICE;
                (void)hipStreamSynchronize(ctx->stream);
                (void)aboria_cells_destroy(cells);
                if (st == ABORIA_OK && ms / reps < best_ms) {
                    best_ms = ms / reps;
                    best_f = f;
                    best_boxes = trial;
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(y);
        (void)hipFree(gx);
        if (st != ABORIA_OK) {
            if (ctx->last_error.empty()) ctx->last_error = "autotune_cells: a trial failed";
            return st;
        }
        for (int32_t b = 0; b < nsys; ++b) boxes_out[b] = best_boxes[(size_t)b];
        if (factor_host) *factor_host = best_f;
        aboria_ctx::CellsChoice ch{{best_boxes[0].reach[0], best_boxes[0].reach[1], best_boxes[0].reach[2]}, best_f};
        bool found = false;
        for (auto& kv : ctx->cells_cache)
            if (kv.first == ckey) { kv.second = ch; found = true; }
        if (!found) ctx->cells_cache.emplace_back(ckey, ch);
        log_msg("autotune_cells: reach {%d, %d, %d}, factor %.2f, %.4f ms", ch.reach[0], ch.reach[1], ch.reach[2],
                best_f, best_ms);
        tune_cache_save(ctx);
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in autotune_cells");
    }
}

extern "C" aboria_status aboria_selected_variant(aboria_ctx* ctx, const aboria_cells* cells, aboria_op op,
                                                 int32_t backward, int32_t* variant_host) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (!cells || !variant_host) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells and variant_host are required");
    if (op_ny(op, cells->d) < 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown operator");
    *variant_host = pick_variant(ctx, cells, op, backward != 0);
    return ABORIA_OK;
}
