// Internal definitions shared by the HIP sources of the library (not part of
// the C-ABI).  Everything here is written for gfx950: wave64, 256 compute
// units in 8 XCDs, LDS per workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/aboria.h"
#include "generation.hpp"

namespace aboria {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;

// Per-system cell-grid parameters in the working precision T, uploaded once per
// build.  The rounded values follow the canonical rules of aboria_build_cells.
template <typename T>
struct SysParams {
    T lo[3];
    T hi[3];
    T L[3];
    T inv_w[3];
    T r;
    T r2;
    // pruning bound of the flattened search: a cell whose gap from a point,
    // (max(gap in cell units - slack, 0) * w_lo) summed in squares over the
    // dimensions, reaches prune_r2 holds no pair of that point
    T w_lo[3];     // cell width, rounded down
    T slack[3];    // rounding margin of a gap, in cell units
    T prune_r2;    // (r + rounding margin of the predicate)^2, rounded up
    int32_t n[3];
    int32_t periodic[3];
    int32_t reach[3];    // cells searched on each side of a point's own cell, per dimension
    uint32_t cell_base;  // first global cell id of the system
    uint32_t part_base;  // first sorted slot (= first row) of the system
    uint32_t part_end;   // one past its last slot
};

// Largest search reach a grid may use (cells at least r / kMaxReach wide).
constexpr int kMaxReach = 3;

// Aligned small vector so that one global load fetches a whole point.
template <typename T, int N>
struct alignas(sizeof(T) * N) VecN {
    T v[N];
};

// Elements stored per particle in the cell-ordered position array: 3-d points
// are padded to 4 so that one 16-byte (float) or 32-byte (double) load fetches
// a point.
template <int D>
struct Pitch {
    static constexpr int value = D == 3 ? 4 : D;
};

// Maps a hardware workgroup index to a logical tile so that consecutive tiles
// land on the same XCD (the dispatcher deals workgroups round-robin over the 8
// XCDs, each with its own L2): XCD x gets the contiguous tile range
// [x * per, (x + 1) * per).  Neighbouring tiles of a cell-ordered array then
// share an L2.  Valid for any grid size; the tail that does not divide evenly
// keeps the identity mapping.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nblocks) {
    uint32_t per = nblocks / kNumXcd;
    uint32_t full = per * kNumXcd;
    if (bid >= full) return bid;
    return (bid % kNumXcd) * per + bid / kNumXcd;
}

// Bit mask of lanes below the calling lane within the wave.
__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

struct Status {
    aboria_status code = ABORIA_OK;
    std::string msg;
};

}  // namespace aboria

// Context and cell-list objects behind the opaque handles of the C-ABI.
struct aboria_ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    uint32_t* d_flag = nullptr;      // device error flag (bit 0: domain error)
    uint32_t* h_flag = nullptr;      // pinned host copy
    bool capturing = false;
    void* scratch = nullptr;         // grow-only scratch for dense partial sums
    size_t scratch_bytes = 0;
    int32_t variant_forced = -1;
    int32_t build_strategy = ABORIA_BUILD_RADIX;
    int32_t lds_per_block = 0;       // device limit on LDS per workgroup (queried on first use)
    std::vector<std::pair<uint64_t, int32_t>> tune_cache;  // (key, variant)
    // cell-size tuner results: key -> search reach per dimension and cell-count factor
    struct CellsChoice {
        int32_t reach[3];
        double factor;
    };
    std::vector<std::pair<uint64_t, CellsChoice>> cells_cache;
    // dense-sum tuner results: key -> targets per lane and workgroup target of the launch
    struct DenseChoice {
        int32_t ti;
        int32_t wg;
    };
    std::vector<std::pair<uint64_t, DenseChoice>> dense_cache;
    int32_t dense_plan_forced = -1;  // the dense tuner's current trial (-1: none)
    // radix build shape: keys per thread of a sort tile (4, 8, 16) and the key bits
    // the bucket pass sorts (8 to 10); 0 = the built-in rule
    struct BuildShape {
        int32_t ipt;
        int32_t low_bits;
        int32_t shuffle;  // the scatter's LDS shuffle: 0 = rule, 1 = where it fits, 2 = never
    };
    std::vector<std::pair<uint64_t, BuildShape>> build_cache;
    BuildShape build_forced{0, 0, 0};
    std::string arch;        // the device's architecture name (keys the persistent cache)
    std::string cache_path;  // ABORIA_TUNE_CACHE at creation ("" = no persistent cache)
};

struct aboria_cells {
    int32_t device = 0;
    int32_t dtype = 0;
    int32_t d = 0;
    int32_t nsys = 0;
    int32_t pitch = 0;
    int64_t n = 0;
    int64_t ncells = 0;
    std::vector<aboria_box> boxes;
    std::vector<int64_t> sys_off;       // [nsys + 1]
    std::vector<int32_t> ncell_host;    // [nsys * 3]
    std::vector<uint32_t> cell_base;    // [nsys + 1]
    std::vector<unsigned char> params_host;  // SysParams<T>[nsys] as uploaded
    void* params_dev = nullptr;
    uint32_t* sys_part_dev = nullptr;   // [nsys + 1] first slot of each system
    uint32_t* cell_base_dev = nullptr;  // [nsys + 1] first global cell id of each system
    uint32_t* keys = nullptr;           // [n] final sorted keys
    uint32_t* perm = nullptr;           // [n] final permutation
    uint32_t* keys_alt = nullptr;       // [n] radix ping-pong buffers
    uint32_t* perm_alt = nullptr;
    uint32_t* off = nullptr;            // [ncells + 1]
    void* xs = nullptr;                 // [n][pitch] positions in cell order
    void* work = nullptr;               // [n][4] gathered per-particle inputs
    void* work2 = nullptr;              // [n][4]
    uint32_t* hist = nullptr;           // radix histograms / scans
    uint32_t* block_sums = nullptr;
    int32_t key_bits = 0;
    int32_t passes = 0;
    int32_t digit_bits = 0;
    int32_t low_bits = 0;      // bits sorted by the per-bucket pass
    int32_t sort_ipt = 16;     // keys per thread of a sort tile (tile = 256 * sort_ipt keys)
    int32_t shuffle_pref = 0;  // radix scatter's LDS shuffle: 0 = rule, 1 = where it fits, 2 = never
    int64_t ntiles = 0;
    int64_t hist_len = 0;
    int64_t nblock_sums = 0;
    // device [2]: generation of the latest build, generation the recorded
    // neighbour list belongs to (the list is used only while they agree)
    uint32_t* gen = nullptr;
    // recorded neighbour list (aboria_build_neighbours)
    uint32_t* nbr = nullptr;        // [nbr_cap][n] slot of each accepted neighbour, box-search order
    uint32_t* nbr_count = nullptr;  // [n] neighbours of each slot (may exceed nbr_cap)
    int64_t nbr_alloc = 0;          // entries per slot allocated in nbr (fixed once allocated)
    uint32_t nbr_cap = 0;           // entries per slot of the latest recording
    bool nbr_recorded = false;      // a list has been recorded on these cells
    // accepted-pair bit masks of the recording forward (pair_mask.hip), allocated on first use
    uint32_t* masks = nullptr;        // [2 * rows][n] two words per stencil row of each slot
    uint32_t* mask_status = nullptr;  // [n] generation the slot's masks belong to (0: none)
};

namespace aboria {

// Diagnostics on stderr, enabled by the environment variable ABORIA_LOG (an
// integer; 0 or unset: silent, 1: errors and tuning decisions).
int log_level();
void log_msg(const char* fmt, ...);

// Releases (hipFree, synchronisation) are not allowed on a thread while it
// captures a stream: such a call would invalidate the capture.  A release
// requested then (a cell list, a context or a graph, e.g. from a garbage
// collector) is queued and runs when the thread's last capture ends.
bool capture_active_on_thread();
void release_or_defer(void (*fn)(void*), void* obj);

// The persistent tuning cache (ABORIA_TUNE_CACHE): loaded when a context is
// created, written after every tuning call.
void tune_cache_load(aboria_ctx* ctx);
void tune_cache_save(aboria_ctx* ctx);

// Error helpers used by the host code (sets ctx->last_error).
aboria_status fail(aboria_ctx* ctx, aboria_status code, const std::string& msg);
aboria_status hip_fail(aboria_ctx* ctx, hipError_t e, const char* what);

#define ABORIA_HIP(ctx, call)                                        \
    do {                                                             \
        hipError_t _e = (call);                                      \
        if (_e != hipSuccess) return ::aboria::hip_fail((ctx), _e, #call); \
    } while (0)

// Host launch helpers implemented in the .hip files.
aboria_status scan_exclusive_u32(aboria_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t len,
                                 uint32_t* block_sums, int64_t nblock_sums);
aboria_status scan_finish_u32(aboria_ctx* ctx, uint32_t* out, int64_t len, const uint32_t* block_sums);
int64_t scan_block_count(int64_t len);
aboria_status fill_u32(aboria_ctx* ctx, uint32_t* p, uint32_t v, int64_t len);

// True if [a, a+na) and [b, b+nb) overlap (byte ranges).
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// Cells per dimension of a box under the cell-count rule (or its explicit
// counts); fails like aboria_build_cells on an invalid box.
aboria_status grid_counts(aboria_ctx* ctx, int dtype, const aboria_box& b, int32_t n[3]);

int32_t op_ny(int32_t op, int32_t d);
int32_t op_na(int32_t op);
int32_t op_nparams(int32_t op);

// Neighbour-sum variants (work mappings) selectable by the autotuner.
int32_t variant_count();
const char* variant_name(int32_t v);
bool variant_needs_list(int32_t v);  // replays a recorded neighbour list
bool variant_usable(int32_t v, const aboria_cells* c);  // its requirements hold for these cells
bool variant_worth_timing(int32_t v, const aboria_cells* c, bool backward);  // the tuner times it on these cells
int32_t list_variant();              // the variant that replays the list
int32_t default_variant(const aboria_cells* c);  // the variant of an untuned sum
int32_t pick_variant(aboria_ctx* ctx, const aboria_cells* cells, int32_t op, bool backward);
uint64_t tune_key(const aboria_cells* cells, int32_t op, bool backward);

aboria_status pair_sum_impl(aboria_ctx* ctx, const aboria_cells* cells, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, void* y, int32_t ny, int32_t variant);
aboria_status pair_bwd_impl(aboria_ctx* ctx, const aboria_cells* cells, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, const void* gy, int32_t ny, void* gx,
                            void* ga, int32_t variant);

}  // namespace aboria
