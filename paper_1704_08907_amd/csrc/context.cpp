// Context, error state, device-flag synchronisation and HIP graph capture of
// the C-ABI.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace aboria {

int log_level() {
    static const int level = [] {
        const char* v = std::getenv("ABORIA_LOG");
        return v ? std::atoi(v) : 0;
    }();
    return level;
}

void log_msg(const char* fmt, ...) {
    if (log_level() < 1) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("aboria: ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

aboria_status fail(aboria_ctx* ctx, aboria_status code, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    log_msg("error %d: %s", (int)code, msg.c_str());
    return code;
}

aboria_status hip_fail(aboria_ctx* ctx, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (ctx) ctx->last_error = m;
    log_msg("HIP error: %s", m.c_str());
    return e == hipErrorOutOfMemory ? ABORIA_ERR_OUT_OF_MEMORY : ABORIA_ERR_DEVICE;
}

int32_t op_ny(int32_t op, int32_t d) {
    switch (op) {
        case ABORIA_OP_COUNT: return 1;
        case ABORIA_OP_SPRING: return d;
        case ABORIA_OP_SOFT_SPHERE: return 1;
        case ABORIA_OP_EXP_FORCE: return d;
        case ABORIA_OP_DEM_SPRING: return d;
        default: return -1;
    }
}

int32_t op_na(int32_t op) {
    switch (op) {
        case ABORIA_OP_COUNT:
        case ABORIA_OP_SPRING:
        case ABORIA_OP_SOFT_SPHERE:
        case ABORIA_OP_EXP_FORCE: return 0;
        case ABORIA_OP_DEM_SPRING: return 1;
        default: return -1;
    }
}

int32_t op_nparams(int32_t op) {
    switch (op) {
        case ABORIA_OP_COUNT: return 0;
        case ABORIA_OP_SPRING: return 1;
        case ABORIA_OP_SOFT_SPHERE: return 0;
        case ABORIA_OP_EXP_FORCE: return 1;
        case ABORIA_OP_DEM_SPRING: return 1;
        default: return -1;
    }
}

namespace {
thread_local int t_capture_depth = 0;
thread_local std::vector<std::pair<void (*)(void*), void*>> t_deferred;
}  // namespace

bool capture_active_on_thread() { return t_capture_depth > 0; }

void release_or_defer(void (*fn)(void*), void* obj) {
    if (t_capture_depth > 0) t_deferred.emplace_back(fn, obj);
    else fn(obj);
}

// Runs the releases queued while this thread captured (after its last capture ended).
static void run_deferred_releases() {
    if (t_capture_depth > 0) return;
    std::vector<std::pair<void (*)(void*), void*>> todo;
    todo.swap(t_deferred);
    for (auto& r : todo) r.first(r.second);
}

}  // namespace aboria

using namespace aboria;

struct aboria_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t device = 0;
};

extern "C" aboria_status aboria_create(int32_t device, void* hip_stream, aboria_ctx** out) {
    if (!out) return ABORIA_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ABORIA_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return ABORIA_ERR_DEVICE;
    aboria_ctx* ctx = new (std::nothrow) aboria_ctx();
    if (!ctx) return ABORIA_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void**)&ctx->d_flag, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_flag, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        if (ctx->d_flag) (void)hipFree(ctx->d_flag);
        delete ctx;
        return ABORIA_ERR_OUT_OF_MEMORY;
    }
    *ctx->h_flag = 0;
    if (fill_u32(ctx, ctx->d_flag, 0u, 1) != ABORIA_OK || hipStreamSynchronize(ctx->stream) != hipSuccess) {
        (void)hipFree(ctx->d_flag);
        (void)hipHostFree(ctx->h_flag);
        delete ctx;
        return ABORIA_ERR_DEVICE;
    }
    try {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->arch = prop.gcnArchName;
        const char* path = std::getenv("ABORIA_TUNE_CACHE");
        if (path && *path) {
            ctx->cache_path = path;
            tune_cache_load(ctx);
        }
    } catch (...) {
        // a context works without its persistent cache
    }
    *out = ctx;
    return ABORIA_OK;
}

static void release_ctx(void* p) {
    aboria_ctx* ctx = static_cast<aboria_ctx*>(p);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->d_flag) (void)hipFree(ctx->d_flag);
    if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    delete ctx;
}

extern "C" aboria_status aboria_destroy(aboria_ctx* ctx) {
    if (!ctx) return ABORIA_OK;
    aboria::release_or_defer(release_ctx, ctx);
    return ABORIA_OK;
}

extern "C" aboria_status aboria_set_stream(aboria_ctx* ctx, void* hip_stream) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "cannot change stream during a capture");
    ctx->stream = (hipStream_t)hip_stream;
    return ABORIA_OK;
}

extern "C" const char* aboria_last_error(const aboria_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

extern "C" aboria_status aboria_sync(aboria_ctx* ctx) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "aboria_sync cannot be captured");
    ABORIA_HIP(ctx, hipSetDevice(ctx->device));
    ABORIA_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    ABORIA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const uint32_t flag = *ctx->h_flag;
    if (flag) {
        aboria_status s = fill_u32(ctx, ctx->d_flag, 0u, 1);
        if (s != ABORIA_OK) return s;
        ABORIA_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return fail(ctx, ABORIA_ERR_DOMAIN, "a position was NaN or outside [lo, hi)");
    }
    return ABORIA_OK;
}

extern "C" aboria_status aboria_graph_capture_begin(aboria_ctx* ctx) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_INVALID_ARG, "capture already in progress");
    if (ctx->stream == nullptr) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "capture needs a non-default stream");
    ABORIA_HIP(ctx, hipSetDevice(ctx->device));
    ABORIA_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    ++aboria::t_capture_depth;
    return ABORIA_OK;
}

extern "C" aboria_status aboria_graph_capture_end(aboria_ctx* ctx, aboria_graph** out) {
    if (!ctx || !out) return ABORIA_ERR_INVALID_ARG;
    if (!ctx->capturing) return fail(ctx, ABORIA_ERR_INVALID_ARG, "no capture in progress");
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
    if (aboria::t_capture_depth > 0) --aboria::t_capture_depth;
    aboria::run_deferred_releases();
    ABORIA_HIP(ctx, ec);
    aboria_graph* gr = new (std::nothrow) aboria_graph();
    if (!gr) {
        (void)hipGraphDestroy(g);
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    gr->graph = g;
    gr->device = ctx->device;
    hipError_t e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete gr;
        return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    *out = gr;
    return ABORIA_OK;
}

extern "C" aboria_status aboria_graph_launch(aboria_ctx* ctx, const aboria_graph* graph) {
    if (!ctx || !graph) return ABORIA_ERR_INVALID_ARG;
    if (graph->device != ctx->device) return fail(ctx, ABORIA_ERR_INVALID_ARG, "graph belongs to another device");
    ABORIA_HIP(ctx, hipGraphLaunch(graph->exec, ctx->stream));
    return ABORIA_OK;
}

static void release_graph(void* p) {
    aboria_graph* graph = static_cast<aboria_graph*>(p);
    (void)hipSetDevice(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

extern "C" aboria_status aboria_graph_destroy(aboria_graph* graph) {
    if (!graph) return ABORIA_OK;
    aboria::release_or_defer(release_graph, graph);
    return ABORIA_OK;
}

extern "C" aboria_status aboria_set_build_strategy(aboria_ctx* ctx, aboria_build_strategy strategy) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (strategy != ABORIA_BUILD_RADIX && strategy != ABORIA_BUILD_COUNTING)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown build strategy");
    ctx->build_strategy = strategy;
    return ABORIA_OK;
}

extern "C" int32_t aboria_op_ny(aboria_op op, int32_t d) {
    if (d < 1 || d > 3) return -1;
    return op_ny(op, d);
}

extern "C" int32_t aboria_op_na(aboria_op op) { return op_na(op); }
