// Cell-list construction: the Level 1 search structure of Section 2.2.1 in its
// parallel-insertion form (the particles are reordered into cell order).
//
//   k_cell_ids       per particle: global cell id under the canonical rounding
//                    (k_cell_ids_hist: per sort tile, with the first radix
//                    pass's digit histogram)
//   k_radix_hist     per sort tile: digit histogram in LDS (later passes)
//   k_scan_local,    device-wide exclusive scan of the digit-major
//   k_scan_top       (digit, tile) counts
//   k_radix_scatter  stable in-tile ranks from wave ballots, then scatter
//                    (these three run once per radix pass over the high key
//                    bits, stably grouping particles by bucket of cells)
//   k_bucket_finalize  the last radix pass, one workgroup per bucket: low-digit
//                    histogram in LDS -> the bucket's cell offsets, stable
//                    placement, and the gather of the positions into cell order
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

#include "common.hpp"

namespace aboria {

constexpr int kBlock = 256;
// A sort tile is kBlock * IPT keys, IPT = 16, 8 or 4 chosen per cell list by
// sort_ipt_for.
constexpr int kScanIpt = 4;
constexpr int kScanTile = kBlock * kScanIpt;  // 1024 values per scan block
constexpr int kMaxDigitBits = 10;
// Scan blocks whose totals a radix pass's consumers prefix-sum themselves in LDS
// (one value per block of kScanTile histogram entries); a longer histogram keeps
// the separate top-level scan.
constexpr int kTopInline = 4 * 256;

// ---------------------------------------------------------------------------
// a1: cell ids
// ---------------------------------------------------------------------------

// System owning row i: the last b with first[b] <= i (empty systems skipped).
__device__ __forceinline__ int find_system(const uint32_t* __restrict__ first, int nsys, uint32_t i) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Global cell id of particle i under the canonical rounding (reading R2);
// *bad is set for a coordinate outside [lo, hi) or NaN (clamped into the grid).
template <typename T, int D>
__device__ __forceinline__ uint32_t cell_key(const SysParams<T>& P, const T* __restrict__ x, uint32_t i,
                                             bool* bad) {
    uint32_t id = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T xk = x[(size_t)i * D + k];
        *bad |= !(xk >= P.lo[k]) || !(xk < P.hi[k]);
        T t = xk - P.lo[k];  // contraction is off: two separately rounded operations
        T q = t * P.inv_w[k];
        T f = floor(q);
        int32_t c;
        if (!(f >= T(0))) c = 0;  // negative or NaN
        else if (f > T(P.n[k] - 1)) c = P.n[k] - 1;
        else c = (int32_t)f;
        id += mul * (uint32_t)c;
        mul *= (uint32_t)P.n[k];
    }
    return P.cell_base + id;
}

// With counts != nullptr it also takes the particle's arrival rank in its cell
// (an atomic increment of the cell's count; the order of arrival is not
// deterministic, the counting build restores the index order afterwards).
template <typename T, int D, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_cell_ids(const T* __restrict__ x, uint32_t n,
                                                     const SysParams<T>* __restrict__ sp,
                                                     const uint32_t* __restrict__ sys_part, int nsys,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ flag,
                                                     uint32_t* __restrict__ counts, uint32_t* __restrict__ ranks,
                                                     uint32_t* __restrict__ gen) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    // a new build generation: a neighbour list recorded for an older one is stale
    if (i == 0) gen[0] = next_generation(gen[0]);
    int b = 0;
    if (BATCH) {
        // the workgroup's rows are contiguous: one binary search for its first
        // row, then each lane steps forward over the (few) systems it spans
        __shared__ int s_first;
        if (threadIdx.x == 0) s_first = find_system(sys_part, nsys, blockIdx.x * kBlock);
        __syncthreads();
        b = s_first;
        while (b + 1 < nsys && sys_part[b + 1] <= i) ++b;
    }
    if (i >= n) return;
    bool bad = false;
    const uint32_t key = cell_key<T, D>(sp[b], x, i, &bad);
    if (bad) atomicOr(flag, 1u);
    keys[i] = key;
    if (counts) ranks[i] = atomicAdd(&counts[key], 1u);
}

// k_cell_ids fused with the digit histogram of the first radix pass: one
// workgroup per sort tile of kBlock * IPT particles (the tiles of
// k_radix_scatter) writes the tile's keys and hist[digit * ntiles + tile] for
// the digit (key >> shift) & (2^bits - 1), as k_radix_hist would from them.
// Threads of a k_cell_ids_hist workgroup for sort tiles of kBlock * IPT keys:
// two keys per thread (at most 1024 threads), so a CU holds four times the
// waves a sort pass would and the position loads' latency is hidden.
template <int IPT>
struct IdsThreads {
    static constexpr int value = kBlock * IPT / 2 > 1024 ? 1024 : kBlock * IPT / 2;
};

template <typename T, int D, bool BATCH, int IPT>
__global__ __launch_bounds__(IdsThreads<IPT>::value) void k_cell_ids_hist(const T* __restrict__ x, uint32_t n,
                                                          const SysParams<T>* __restrict__ sp,
                                                          const uint32_t* __restrict__ sys_part, int nsys,
                                                          uint32_t* __restrict__ keys, uint32_t* __restrict__ flag,
                                                          uint32_t* __restrict__ gen, int shift, int bits,
                                                          uint32_t* __restrict__ hist, uint32_t ntiles) {
    constexpr int NT = IdsThreads<IPT>::value;
    constexpr int KPT = kBlock * IPT / NT;
    extern __shared__ uint32_t lds[];
    const uint32_t radix = 1u << bits, mask = radix - 1u;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
    const uint32_t base = tile * (kBlock * IPT);
    if (tile == 0 && threadIdx.x == 0) gen[0] = next_generation(gen[0]);
    for (uint32_t d = threadIdx.x; d < radix; d += NT) lds[d] = 0;
    int b = 0;
    if (BATCH) {
        __shared__ int s_first;
        if (threadIdx.x == 0) s_first = find_system(sys_part, nsys, base);
        __syncthreads();
        b = s_first;
    }
    __syncthreads();
    bool bad = false;
    uint32_t key[KPT];
    // all keys first (their position loads in flight together), then the histogram
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        key[k] = 0u;
        if (i < n) {
            if (BATCH)
                while (b + 1 < nsys && sys_part[b + 1] <= i) ++b;
            key[k] = cell_key<T, D>(sp[b], x, i, &bad);
            keys[i] = key[k];
        }
    }
#pragma unroll
    for (int k = 0; k < KPT; ++k)
        if (base + k * NT + threadIdx.x < n) atomicAdd(&lds[(key[k] >> shift) & mask], 1u);
    if (bad) atomicOr(flag, 1u);
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < radix; d += NT) hist[(size_t)d * ntiles + tile] = lds[d];
}

// One cell per system (an explicit cell count of 1 in every dimension, the
// layout of the all-pairs sums of small systems): the stable cell order is the
// input order, so one kernel writes the identity permutation, the systems'
// cell ids, the positions and the offsets (the system offsets) in place of the
// sort.  Threads up to nsys also write the offsets, so the grid covers
// max(n, nsys + 1).
template <typename T, int D, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_single_cells(const T* __restrict__ x, uint32_t n,
                                                         const SysParams<T>* __restrict__ sp,
                                                         const uint32_t* __restrict__ sys_part, int nsys,
                                                         T* __restrict__ xs, uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ perm, uint32_t* __restrict__ off,
                                                         uint32_t* __restrict__ flag, uint32_t* __restrict__ gen) {
    constexpr int PITCH = Pitch<D>::value;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) gen[0] = next_generation(gen[0]);
    if (i <= (uint32_t)nsys) off[i] = sys_part[i];
    int b = 0;
    if (BATCH) {
        __shared__ int s_first;
        if (threadIdx.x == 0) s_first = find_system(sys_part, nsys, min(blockIdx.x * kBlock, n > 0 ? n - 1 : 0u));
        __syncthreads();
        b = s_first;
        while (b + 1 < nsys && sys_part[b + 1] <= i) ++b;
    }
    if (i >= n) return;
    const SysParams<T>& P = sp[b];
    VecN<T, PITCH> v;
#pragma unroll
    for (int k = 0; k < PITCH; ++k) v.v[k] = T(0);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T xk = x[(size_t)i * D + k];
        bad |= !(xk >= P.lo[k]) || !(xk < P.hi[k]);
        v.v[k] = xk;
    }
    if (bad) atomicOr(flag, 1u);
    reinterpret_cast<VecN<T, PITCH>*>(xs)[i] = v;
    keys[i] = P.cell_base;
    perm[i] = i;
}

// ---------------------------------------------------------------------------
// counting build: place by (cell offset + arrival rank), then restore the
// original index order inside each cell
// ---------------------------------------------------------------------------

// perm_tmp[off[key] + rank] = i and key_tmp of that slot = key; off is the
// local scan of the counts plus its block prefix.
__global__ __launch_bounds__(kBlock) void k_count_place(const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ ranks, uint32_t n,
                                                        const uint32_t* __restrict__ off_local,
                                                        const uint32_t* __restrict__ block_sums,
                                                        uint32_t* __restrict__ perm_tmp,
                                                        uint32_t* __restrict__ key_tmp) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys[i];
    const uint32_t slot = off_local[k] + block_sums[k / kScanTile] + ranks[i];
    if (slot < n) {  // always true for consistent counts; keeps bad ones in bounds
        perm_tmp[slot] = i;
        key_tmp[slot] = k;
    }
}

// Completes the cell offsets: off[c] += block prefix, and off[ncells] = n.
__global__ __launch_bounds__(kBlock) void k_count_offsets(uint32_t* __restrict__ off, uint32_t ncells, uint32_t n,
                                                          const uint32_t* __restrict__ block_sums) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c < ncells) off[c] += block_sums[c / kScanTile];
    else if (c == ncells) off[c] = n;
}

// Slot s of cell c holds element i = perm_tmp[s]; its final slot is
// off[c] + #{t in cell c : perm_tmp[t] < i}, i.e. the cell's elements in
// original index order.  Writes the final key, permutation and position.
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_count_finalize(const uint32_t* __restrict__ perm_tmp,
                                                           const uint32_t* __restrict__ key_tmp, uint32_t n,
                                                           const uint32_t* __restrict__ off, uint32_t ncells,
                                                           const T* __restrict__ x, T* __restrict__ xs,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ perm_out) {
    constexpr int PITCH = Pitch<D>::value;
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const uint32_t c = min(key_tmp[s], ncells - 1u);
    const uint32_t i = perm_tmp[s];
    const uint32_t b0 = off[c], b1 = min(off[c + 1], n);
    uint32_t rank = 0;
    for (uint32_t t = b0; t < b1; ++t) rank += perm_tmp[t] < i ? 1u : 0u;
    const uint32_t dest = min(b0 + rank, n - 1u);
    const uint32_t p = min(i, n - 1u);
    keys_out[dest] = c;
    perm_out[dest] = p;
    VecN<T, PITCH> v;
#pragma unroll
    for (int k = 0; k < PITCH; ++k) v.v[k] = k < D ? x[(size_t)p * D + k] : T(0);
    reinterpret_cast<VecN<T, PITCH>*>(xs)[dest] = v;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan (two kernels; the consumer adds the block prefix)
// ---------------------------------------------------------------------------

// Exclusive scan of one value per thread across the 256-thread block; returns
// the block total through *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t q = 0; q < w; ++q) pre += wsum[q];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return pre + incl - v;
}

// block_exclusive_scan for a workgroup of NW waves (wsum holds NW entries).
template <int NW>
__device__ __forceinline__ uint32_t block_exclusive_scan_w(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, all = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        pre += (uint32_t)q < w ? wsum[q] : 0u;
        all += wsum[q];
    }
    *total = all;
    __syncthreads();
    return pre + incl - v;
}

// out[p] = sum of in[q] for q < p within p's kScanTile-block; block_sums[b] = block
// total.  Where in and out are 16-byte aligned a thread's four values move as
// one 16-byte load and store.
__global__ __launch_bounds__(kBlock) void k_scan_local(const uint32_t* in, uint32_t* out,
                                                       uint32_t len, uint32_t* __restrict__ block_sums) {
    static_assert(kScanIpt == 4, "one uint4 per thread");
    __shared__ uint32_t wsum[4];
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanIpt;
    uint32_t v[kScanIpt];
    const bool aligned = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
    const bool whole = aligned && base + kScanIpt <= len;
    if (whole) {
        const uint4 q = *reinterpret_cast<const uint4*>(in + base);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanIpt; ++k) v[k] = base + k < len ? in[base + k] : 0u;
    }
    const uint32_t tot = v[0] + v[1] + v[2] + v[3];
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(tot, wsum, &total);
    const uint32_t e[kScanIpt] = {ex, ex + v[0], ex + v[0] + v[1], ex + v[0] + v[1] + v[2]};
    if (whole) {
        *reinterpret_cast<uint4*>(out + base) = make_uint4(e[0], e[1], e[2], e[3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanIpt; ++k)
            if (base + k < len) out[base + k] = e[k];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// In-place exclusive scan of the block totals by one workgroup (any length).
__global__ __launch_bounds__(kBlock) void k_scan_top(uint32_t* __restrict__ bs, uint32_t nb) {
    __shared__ uint32_t wsum[4];
    uint32_t carry = 0;
    for (uint32_t chunk = 0; chunk < nb; chunk += kScanTile) {
        const uint32_t base = chunk + threadIdx.x * kScanIpt;
        uint32_t v[kScanIpt];
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < kScanIpt; ++k) {
            uint32_t idx = base + k;
            v[k] = idx < nb ? bs[idx] : 0u;
            tot += v[k];
        }
        uint32_t total;
        uint32_t ex = carry + block_exclusive_scan(tot, wsum, &total);
#pragma unroll
        for (int k = 0; k < kScanIpt; ++k) {
            uint32_t idx = base + k;
            if (idx < nb) bs[idx] = ex;
            ex += v[k];
        }
        carry += total;
    }
}

// out[p] += block_sums[p / kScanTile]: completes a scan for consumers that need it whole.
__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t* __restrict__ out, uint32_t len,
                                                     const uint32_t* __restrict__ bs) {
    uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p < len) out[p] += bs[p / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint32_t len) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < len) p[i] = v;
}

int64_t scan_block_count(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

aboria_status scan_exclusive_u32(aboria_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t len,
                                 uint32_t* block_sums, int64_t nblock_sums) {
    if (len <= 0) return ABORIA_OK;
    int64_t nb = scan_block_count(len);
    if (nb > nblock_sums) return fail(ctx, ABORIA_ERR_INVALID_ARG, "scan: block-sum buffer too small");
    hipLaunchKernelGGL(k_scan_local, dim3((uint32_t)nb), dim3(kBlock), 0, ctx->stream, in, out, (uint32_t)len,
                       block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, ctx->stream, block_sums, (uint32_t)nb);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

// The first level of scan_exclusive_u32 only: out holds each kScanTile-block's
// exclusive scan and block_sums the blocks' raw totals.
aboria_status scan_local_u32(aboria_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t len, uint32_t* block_sums,
                             int64_t nblock_sums) {
    if (len <= 0) return ABORIA_OK;
    int64_t nb = scan_block_count(len);
    if (nb > nblock_sums) return fail(ctx, ABORIA_ERR_INVALID_ARG, "scan: block-sum buffer too small");
    hipLaunchKernelGGL(k_scan_local, dim3((uint32_t)nb), dim3(kBlock), 0, ctx->stream, in, out, (uint32_t)len,
                       block_sums);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

aboria_status scan_finish_u32(aboria_ctx* ctx, uint32_t* out, int64_t len, const uint32_t* block_sums) {
    if (len <= 0) return ABORIA_OK;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)((len + kBlock - 1) / kBlock)), dim3(kBlock), 0, ctx->stream, out,
                       (uint32_t)len, block_sums);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

aboria_status fill_u32(aboria_ctx* ctx, uint32_t* p, uint32_t v, int64_t len) {
    if (len <= 0) return ABORIA_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)((len + kBlock - 1) / kBlock)), dim3(kBlock), 0, ctx->stream, p, v,
                       (uint32_t)len);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

// ---------------------------------------------------------------------------
// a2: LSD radix sort of (cell id, index) pairs
// ---------------------------------------------------------------------------

// hist[digit * ntiles + tile] = number of keys of the tile with that digit.
template <int IPT>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys, uint32_t n, int shift,
                                                       int bits, uint32_t* __restrict__ hist, uint32_t ntiles) {
    extern __shared__ uint32_t lds[];
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (uint32_t d = threadIdx.x; d < radix; d += kBlock) lds[d] = 0;
    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
    const uint32_t base = tile * (kBlock * IPT);
#pragma unroll 4
    for (int k = 0; k < IPT; ++k) {
        uint32_t idx = base + k * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&lds[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < radix; d += kBlock) hist[(size_t)d * ntiles + tile] = lds[d];
}

// Stable scatter of one tile of kBlock * IPT keys.  Wave w owns keys
// [w * 64 IPT, (w + 1) * 64 IPT) of the tile and walks them in IPT steps of 64
// consecutive keys.  Lanes holding the
// same digit find each other with one ballot per digit bit; a lane's rank is
// the number of such lanes below it plus the wave's running count for the
// digit (kept in LDS, updated by the lowest such lane).  After all waves are
// done the per-wave counts become per-wave offsets, and the tile is shuffled
// into digit order in LDS, so that keys and indices leave in one contiguous
// run per digit instead of one scattered 4-byte store per lane.  The position
// rows ride along as a payload (FIRST: read from the caller's x in original
// order; later passes: from the previous pass's payload), so that the bucket
// pass reads them in order instead of gathering them by index.
template <typename T, int D, bool FIRST, bool SHUFFLE, bool PAYLOAD, int IPT>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          const T* __restrict__ x,
                                                          const VecN<T, Pitch<D>::value>* __restrict__ pay_in,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out,
                                                          VecN<T, Pitch<D>::value>* __restrict__ pay_out, uint32_t n,
                                                          int shift, int bits, const uint32_t* __restrict__ hist_scan,
                                                          const uint32_t* __restrict__ block_sums, uint32_t ntiles,
                                                          int top_done, uint32_t* __restrict__ top_out) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr int kSortTile = kBlock * IPT;
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_top[kTopInline];  // exclusive prefix of the scan blocks' totals
    const uint32_t radix = 1u << bits, mask = radix - 1;
    uint32_t* cnt = lds;                 // [4][radix] per-wave counts, then per-wave offsets
    uint32_t* gbase = lds + 4 * radix;   // [radix] first global slot of the tile's keys of a digit
    uint32_t* tstart = lds + 5 * radix;  // [radix] first tile slot of a digit
    uint32_t* sk = lds + 6 * radix;      // [kSortTile] keys in digit order
    uint32_t* sv = sk + kSortTile;       // [kSortTile] indices in digit order
    // [kSortTile] position rows in digit order (SHUFFLE and PAYLOAD)
    VecN<T, PITCH>* srow = reinterpret_cast<VecN<T, PITCH>*>(sv + kSortTile);
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD's L2
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t tbase = tile * kSortTile;
    const uint32_t wbase = tbase + w * (kWave * IPT);
    uint32_t key[IPT], val[IPT], loc[IPT];
    // the tile's key and index loads first, so they are in flight together and
    // with the histogram reads below
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
        const uint32_t idx = wbase + s * kWave + lane;
        const bool valid = idx < n;
        key[s] = valid ? keys_in[idx] : 0u;
        val[s] = valid ? (FIRST ? idx : vals_in[idx]) : 0u;
    }
    if (!top_done) {
        // the top level of the histogram scan: every tile prefix-sums the scan
        // blocks' totals itself (tile 0 also stores them for the bucket pass)
        const uint32_t nb = (radix * ntiles + kScanTile - 1) / kScanTile;
        uint32_t v[kTopInline / kBlock], tot = 0;
#pragma unroll
        for (int q = 0; q < kTopInline / kBlock; ++q) {
            const uint32_t b = threadIdx.x * (kTopInline / kBlock) + q;
            v[q] = b < nb ? block_sums[b] : 0u;
            tot += v[q];
        }
        uint32_t total;
        uint32_t ex = block_exclusive_scan(tot, s_wsum, &total);
#pragma unroll
        for (int q = 0; q < kTopInline / kBlock; ++q) {
            const uint32_t b = threadIdx.x * (kTopInline / kBlock) + q;
            if (b < nb) {
                s_top[b] = ex;
                if (tile == 0) top_out[b] = ex;
            }
            ex += v[q];
        }
        __syncthreads();
    }
    for (uint32_t d = threadIdx.x; d < radix; d += kBlock) {
        cnt[d] = 0;
        cnt[radix + d] = 0;
        cnt[2 * radix + d] = 0;
        cnt[3 * radix + d] = 0;
        size_t p = (size_t)d * ntiles + tile;
        gbase[d] = hist_scan[p] + (top_done ? block_sums[p / kScanTile] : s_top[p / kScanTile]);
    }
    __syncthreads();
    uint32_t* wc = cnt + w * radix;
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
        const uint32_t idx = wbase + s * kWave + lane;
        const bool valid = idx < n;
        const uint32_t k = key[s];
        const uint32_t dg = (k >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t c = valid ? wc[dg] : 0u;
        if (valid && below == 0) wc[dg] = c + (uint32_t)__popcll(peers);
        loc[s] = c + below;
    }
    __syncthreads();
    {   // per digit: offsets of the waves, and the tile's exclusive scan over digits
        constexpr uint32_t kMaxPer = (1u << kMaxDigitBits) / kBlock;
        const uint32_t per = radix >= (uint32_t)kBlock ? radix / kBlock : 1u;
        const uint32_t d0 = threadIdx.x * per;
        uint32_t tot[kMaxPer > 0 ? kMaxPer : 1];
        uint32_t sum = 0;
        for (uint32_t q = 0; q < per; ++q) {
            tot[q] = 0;
            const uint32_t d = d0 + q;
            if (d < radix) {
                const uint32_t a0 = cnt[d], a1 = cnt[radix + d], a2 = cnt[2 * radix + d], a3 = cnt[3 * radix + d];
                cnt[d] = 0;
                cnt[radix + d] = a0;
                cnt[2 * radix + d] = a0 + a1;
                cnt[3 * radix + d] = a0 + a1 + a2;
                tot[q] = a0 + a1 + a2 + a3;
                sum += tot[q];
            }
        }
        uint32_t total;
        uint32_t ex = block_exclusive_scan(sum, s_wsum, &total);
        for (uint32_t q = 0; q < per; ++q) {
            const uint32_t d = d0 + q;
            if (d < radix) {
                tstart[d] = ex;
                ex += tot[q];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < IPT; ++s) {
        const uint32_t idx = wbase + s * kWave + lane;
        if (idx < n) {
            const uint32_t dg = (key[s] >> shift) & mask;
            const uint32_t off_d = wc[dg] + loc[s];
            const uint32_t tl = tstart[dg] + off_d;
            const uint32_t pos = gbase[dg] + off_d;
            if (tl < (uint32_t)kSortTile && pos < n) {  // always true for a consistent histogram
                if (SHUFFLE) {
                    sk[tl] = key[s];
                    sv[tl] = val[s];
                } else {
                    keys_out[pos] = key[s];
                    vals_out[pos] = val[s];
                }
                if (PAYLOAD) {
                    VecN<T, PITCH> row;
                    if (FIRST) {
#pragma unroll
                        for (int k = 0; k < PITCH; ++k) row.v[k] = k < D ? x[(size_t)idx * D + k] : T(0);
                    } else {
                        row = pay_in[idx];
                    }
                    if (SHUFFLE) srow[tl] = row;  // leaves with its key, in digit order
                    else pay_out[pos] = row;
                }
            }
        }
    }
    if (!SHUFFLE) return;
    __syncthreads();
    const uint32_t count = min((uint32_t)kSortTile, n - tbase);
    for (uint32_t i = threadIdx.x; i < count; i += kBlock) {
        const uint32_t k = sk[i];
        const uint32_t dg = (k >> shift) & mask;
        const uint32_t pos = gbase[dg] + (i - tstart[dg]);
        if (pos < n) {  // always true for a consistent histogram; keeps a bad one in bounds
            keys_out[pos] = k;
            vals_out[pos] = sv[i];
            if (PAYLOAD) pay_out[pos] = srow[i];
        }
    }
}

// ---------------------------------------------------------------------------
// last radix pass fused with a3 + a4: per bucket of 2^lb consecutive cells
// ---------------------------------------------------------------------------

// The input is sorted (stably) by key >> lb, so bucket b -- the cells
// [b << lb, (b + 1) << lb) -- is one contiguous range of it, in original index
// order.  One workgroup per bucket: it histograms the low digit of its keys in
// LDS, writes the offsets of its cells (bucket start + exclusive scan), and
// places its elements stably, chunk by chunk, with the same wave-ballot ranks
// as k_radix_scatter, writing the sorted key, the permutation and the position
// gathered from the original array.  Buckets cover cells 0..ncells inclusive,
// so off[ncells] = n is written too.
// When exactly one radix pass sorted the high bits, its scanned digit-major
// histogram (hist_scan + block_sums, ntiles tiles) gives each bucket's start
// directly; otherwise (hist_scan == nullptr) the bounds are found by binary
// search of the high parts.
// Threads of a bucket workgroup: eight waves for sort tiles of 2048 keys or
// more (two workgroups fit a CU's LDS, so sixteen waves hide the bucket's
// loads), four below.
template <int IPT>
struct BucketThreads {
    static constexpr int value = IPT >= 8 ? 512 : 256;
};

template <typename T, int D, int IPT, bool STAGE>
__global__ __launch_bounds__(BucketThreads<IPT>::value) void k_bucket_finalize(const uint32_t* __restrict__ keys_in,
                                                            const uint32_t* __restrict__ vals_in, uint32_t n,
                                                            int lb, uint32_t ncells, const T* __restrict__ x,
                                                            T* __restrict__ xs, uint32_t* __restrict__ keys_out,
                                                            uint32_t* __restrict__ perm_out,
                                                            uint32_t* __restrict__ off,
                                                            const uint32_t* __restrict__ hist_scan,
                                                            const uint32_t* __restrict__ block_sums, uint32_t ntiles,
                                                            uint32_t ndigits,
                                                            const VecN<T, Pitch<D>::value>* __restrict__ pay) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr int kSortTile = kBlock * IPT;
    constexpr int NT = BucketThreads<IPT>::value;
    constexpr int NW = NT / kWave;
    constexpr int KPT = kSortTile / NT;  // keys of a chunk per thread
    extern __shared__ uint32_t lds[];
    const uint32_t R = 1u << lb, mask = R - 1u;
    uint32_t* hist = lds;              // [R]
    uint32_t* base = lds + R;          // [R] running destination base per digit
    uint32_t* cnt = lds + 2 * R;       // [NW][R] per-wave counts of the current chunk
    __shared__ uint32_t s_range[2];
    __shared__ uint32_t s_wsum[NW];
    const uint32_t bucket = blockIdx.x;
    const uint32_t cell0 = bucket << lb;
    if (threadIdx.x < 2) {
        // first index whose high part is >= bucket + threadIdx.x
        const uint32_t target = bucket + threadIdx.x;
        uint32_t lo;
        if (hist_scan) {
            if (target >= ndigits) {
                lo = n;
            } else {
                const size_t p = (size_t)target * ntiles;
                lo = hist_scan[p] + block_sums[p / kScanTile];
            }
        } else {
            lo = 0;
            uint32_t hi = n;
            while (lo < hi) {
                const uint32_t mid = lo + ((hi - lo) >> 1);
                if ((keys_in[mid] >> lb) < target) lo = mid + 1; else hi = mid;
            }
        }
        s_range[threadIdx.x] = lo;
    }
    __syncthreads();
    const uint32_t b0 = s_range[0], b1 = s_range[1];
    // exclusive scan of hist into base and the offsets of the bucket's cells: each
    // thread owns a run of R/NT digits (R >= NT) or one
    auto scan_hist = [&]() {
        const uint32_t per = R >= (uint32_t)NT ? R / NT : 1u;
        const uint32_t d0 = threadIdx.x * per;
        uint32_t tot = 0;
        if (d0 < R)
            for (uint32_t k = 0; k < per; ++k) tot += hist[d0 + k];
        uint32_t total;
        uint32_t ex = block_exclusive_scan_w<NW>(tot, s_wsum, &total);
        if (d0 < R) {
            for (uint32_t k = 0; k < per; ++k) {
                const uint32_t c = cell0 + d0 + k;
                base[d0 + k] = ex;
                if (c <= ncells) off[c] = b0 + ex;
                ex += hist[d0 + k];
            }
        }
    };
    // A nonempty bucket that fits one chunk takes its histogram from the chunk's
    // per-wave rank counts below; a larger (or empty) one counts its keys first.
    const bool single = b1 > b0 && b1 - b0 <= (uint32_t)kSortTile;
    if (!single) {
        for (uint32_t d = threadIdx.x; d < R; d += NT) hist[d] = 0;
        __syncthreads();
        for (uint32_t i = b0 + threadIdx.x; i < b1; i += NT) atomicAdd(&hist[keys_in[i] & mask], 1u);
        __syncthreads();
        scan_hist();
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t* wc = cnt + w * R;
    const uint64_t lt = lanemask_lt();
    for (uint32_t chunk = b0; chunk < b1; chunk += kSortTile) {
        for (uint32_t d = threadIdx.x; d < R; d += NT) {
#pragma unroll
            for (int q = 0; q < NW; ++q) cnt[q * R + d] = 0;
        }
        __syncthreads();
        const uint32_t wbase = chunk + w * (kWave * KPT);
        uint32_t key[KPT], val[KPT], loc[KPT];
        VecN<T, PITCH> row[KPT];
        // every load of the chunk first, so they are in flight together
#pragma unroll
        for (int st = 0; st < KPT; ++st) {
            const uint32_t idx = wbase + st * kWave + lane;
            const bool valid = idx < b1;
            key[st] = valid ? keys_in[idx] : 0u;
            val[st] = valid ? (vals_in ? vals_in[idx] : idx) : 0u;
            if (pay && valid) row[st] = pay[idx];  // the row travelled with its key through the radix passes
        }
#pragma unroll
        for (int st = 0; st < KPT; ++st) {
            const uint32_t idx = wbase + st * kWave + lane;
            const bool valid = idx < b1;
            const uint32_t k = key[st];
            const uint32_t dg = k & mask;
            uint64_t peers = __ballot(valid);
            for (int bb = 0; bb < lb; ++bb) {
                const bool bit = (dg >> bb) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            const uint32_t c = valid ? wc[dg] : 0u;
            if (valid && below == 0) wc[dg] = c + (uint32_t)__popcll(peers);
            loc[st] = c + below;
        }
        __syncthreads();
        if (single) {
            for (uint32_t d = threadIdx.x; d < R; d += NT) {
                uint32_t h = 0;
#pragma unroll
                for (int q = 0; q < NW; ++q) h += cnt[q * R + d];
                hist[d] = h;
            }
            __syncthreads();
            scan_hist();
            __syncthreads();
        }
        for (uint32_t d = threadIdx.x; d < R; d += NT) {
            // the waves' first destinations of digit d, in wave (= index) order
            uint32_t run = base[d];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint32_t a = cnt[q * R + d];
                cnt[q * R + d] = run;
                run += a;
            }
            base[d] = run;
        }
        __syncthreads();
        if (STAGE && single) {
            // sorted order assembled in LDS, then written as contiguous runs (scattered
            // stores into the bucket's range left partly written lines behind)
            uint32_t* sk = lds + (2 + NW) * R;  // after hist, base and the NW per-wave counts
            uint32_t* sv = sk + kSortTile;
            VecN<T, PITCH>* srow = reinterpret_cast<VecN<T, PITCH>*>(sv + kSortTile);
#pragma unroll
            for (int st = 0; st < KPT; ++st) {
                const uint32_t idx = wbase + st * kWave + lane;
                if (idx < b1) {
                    const uint32_t rel = wc[key[st] & mask] + loc[st];
                    if (rel < (uint32_t)kSortTile) {  // always true for a consistent histogram
                        sk[rel] = key[st];
                        sv[rel] = min(val[st], n - 1u);
                        srow[rel] = row[st];
                    }
                }
            }
            __syncthreads();
            const uint32_t count = b1 - b0;
            for (uint32_t i = threadIdx.x; i < count; i += NT) {
                if (b0 + i < n) {
                    keys_out[b0 + i] = sk[i];
                    perm_out[b0 + i] = sv[i];
                    reinterpret_cast<VecN<T, PITCH>*>(xs)[b0 + i] = srow[i];
                }
            }
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int st = 0; st < KPT; ++st) {
            const uint32_t idx = wbase + st * kWave + lane;
            if (idx < b1) {
                const uint32_t dest = b0 + wc[key[st] & mask] + loc[st];
                if (dest < n) {  // always true for a consistent histogram; keeps a bad one in bounds
                    keys_out[dest] = key[st];
                    const uint32_t p = min(val[st], n - 1u);
                    perm_out[dest] = p;
                    VecN<T, PITCH> v;
                    if (pay) {
                        v = row[st];
                    } else {
#pragma unroll
                        for (int k = 0; k < PITCH; ++k) v.v[k] = k < D ? x[(size_t)p * D + k] : T(0);
                    }
                    reinterpret_cast<VecN<T, PITCH>*>(xs)[dest] = v;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

struct GridPlan {
    int32_t n[3] = {1, 1, 1};
    int32_t reach[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, L[3] = {0, 0, 0}, inv_w[3] = {0, 0, 0};
    double w_lo[3] = {0, 0, 0}, slack[3] = {0, 0, 0};
    double r = 0, r2 = 0, prune_r2 = 0;
    int64_t ncells = 1;
};

double round_to(int dtype, double v) { return dtype == ABORIA_F32 ? (double)(float)v : v; }

// Cell grid of one box: the largest per-dimension count whose cells are at
// least (cutoff + a guard of 16 unit roundoffs of the coordinate magnitude) /
// m wide, m the dimension's reach, so that rounding in the cell assignment
// cannot put the points of a pair more than m cells apart.  Also the pruning bound of the
// flattened search (SysParams): the margins cover the rounding of both cell
// assignments (2 u |q| each, |q| <= n + 1 cell units), of an image shift
// (n u) and of the gap itself (u reach), with room to spare, and the pair
// predicate accepting a distance slightly above r (its differences round by
// u L, its sum of squares by a few u).
aboria_status plan_grid(aboria_ctx* ctx, int dtype, const aboria_box& b, GridPlan* g) {
    const double u = dtype == ABORIA_F32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
    for (int k = 0; k < 3; ++k) {
        g->reach[k] = k < b.d && b.reach[k] != 0 ? b.reach[k] : 1;
        if (g->reach[k] < 1 || g->reach[k] > kMaxReach)
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "reach must be 0 to 3 in every dimension");
    }
    g->r = round_to(dtype, b.cutoff);
    if (!(g->r > 0.0) || std::isinf(g->r)) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cutoff must be positive and finite");
    if (dtype == ABORIA_F32) {
        float rf = (float)g->r;
        g->r2 = (double)(rf * rf);
    } else {
        g->r2 = g->r * g->r;
    }
    int64_t total = 1;
    double Lmax = 0.0;
    for (int k = 0; k < b.d; ++k) {
        g->lo[k] = round_to(dtype, b.lo[k]);
        g->hi[k] = round_to(dtype, b.hi[k]);
        if (!std::isfinite(g->lo[k]) || !std::isfinite(g->hi[k]) || !(g->hi[k] > g->lo[k]))
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "box needs finite lo < hi in every dimension");
        g->L[k] = dtype == ABORIA_F32 ? (double)((float)g->hi[k] - (float)g->lo[k]) : g->hi[k] - g->lo[k];
        const double guard = g->r + 16.0 * u * (std::fabs(g->lo[k]) + g->L[k]);
        const double m = (double)g->reach[k];
        const double q = std::floor(m * g->L[k] / g->r);
        int64_t nmax = q < 1.0 ? 1 : (q > 2147483647.0 ? 2147483647 : (int64_t)q);
        while (nmax > 1 && g->L[k] / (double)nmax < guard / m) --nmax;
        int64_t nk = nmax;
        if (b.ncell[k] > 0) {
            if (b.ncell[k] > nmax)
                return fail(ctx, ABORIA_ERR_INVALID_ARG, "explicit ncell gives cells narrower than the guarded cutoff / reach");
            nk = b.ncell[k];
        }
        if (b.periodic[k] && g->L[k] < 2.0 * guard)
            return fail(ctx, ABORIA_ERR_UNSUPPORTED, "periodic side shorter than twice the guarded cutoff");
        g->n[k] = (int32_t)nk;
        g->inv_w[k] = round_to(dtype, (double)nk / g->L[k]);
        g->w_lo[k] = g->L[k] / (double)nk * (1.0 - 16.0 * u);
        g->slack[k] = 16.0 * u * ((double)nk + m + 2.0);
        Lmax = std::max(Lmax, g->L[k] + std::fabs(g->lo[k]));
        total *= nk;
        if (total > 2147483647LL) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "more than 2^31 cells");
    }
    const double rp = g->r * (1.0 + 16.0 * u) + 16.0 * u * (Lmax + 3.0 * g->r);
    g->prune_r2 = rp * rp * (1.0 + 64.0 * u);
    g->ncells = total;
    return ABORIA_OK;
}

template <typename T>
void fill_params(const std::vector<GridPlan>& plans, const std::vector<aboria_box>& boxes,
                 const std::vector<uint32_t>& cell_base, const std::vector<int64_t>& off,
                 std::vector<unsigned char>* out) {
    const size_t nsys = plans.size();
    out->assign(nsys * sizeof(SysParams<T>), 0);
    SysParams<T>* sp = reinterpret_cast<SysParams<T>*>(out->data());
    for (size_t b = 0; b < nsys; ++b) {
        SysParams<T> p;
        std::memset(&p, 0, sizeof(p));
        for (int k = 0; k < 3; ++k) {
            p.lo[k] = (T)plans[b].lo[k];
            p.hi[k] = (T)plans[b].hi[k];
            p.L[k] = (T)plans[b].L[k];
            p.inv_w[k] = (T)plans[b].inv_w[k];
            p.n[k] = plans[b].n[k];
            p.periodic[k] = k < boxes[b].d ? (boxes[b].periodic[k] != 0) : 0;
        }
        p.r = (T)plans[b].r;
        p.r2 = (T)plans[b].r2;
        // rounded the safe way: the width down, the slack and the threshold up
        for (int k = 0; k < 3; ++k) {
            p.w_lo[k] = (T)(plans[b].w_lo[k] * (1.0 - 4.0 * std::numeric_limits<T>::epsilon()));
            p.slack[k] = (T)(plans[b].slack[k] * (1.0 + 4.0 * std::numeric_limits<T>::epsilon()));
        }
        p.prune_r2 = (T)(plans[b].prune_r2 * (1.0 + 4.0 * std::numeric_limits<T>::epsilon()));
        for (int k = 0; k < 3; ++k) p.reach[k] = plans[b].reach[k];
        p.cell_base = cell_base[b];
        p.part_base = (uint32_t)off[b];
        p.part_end = (uint32_t)off[b + 1];
        std::memcpy(&sp[b], &p, sizeof(p));
    }
}

void free_cells_buffers(aboria_cells* c) {
    void* ptrs[] = {c->params_dev, c->sys_part_dev, c->cell_base_dev, c->keys, c->perm, c->keys_alt,
                    c->perm_alt, c->off, c->xs, c->work, c->work2, c->hist, c->block_sums,
                    c->nbr, c->nbr_count, c->gen, c->masks, c->mask_status};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    c->params_dev = nullptr;
    c->sys_part_dev = c->cell_base_dev = c->keys = c->perm = c->keys_alt = c->perm_alt = c->off = nullptr;
    c->hist = c->block_sums = nullptr;
    c->xs = c->work = c->work2 = nullptr;
    c->nbr = c->nbr_count = c->gen = nullptr;
    c->masks = c->mask_status = nullptr;
    c->nbr_alloc = 0;
    c->nbr_recorded = false;
}

template <typename T, int D>
aboria_status launch_build_counting(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    const uint32_t n = (uint32_t)c->n;
    const uint32_t nc = (uint32_t)c->ncells;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    hipStream_t st = ctx->stream;
    // keys_alt = keys in original order, perm_alt = arrival ranks, the work
    // buffers hold the placed (index, key); counts are made and scanned in off
    uint32_t* counts = c->off;
    uint32_t* perm_tmp = reinterpret_cast<uint32_t*>(c->work);
    uint32_t* key_tmp = reinterpret_cast<uint32_t*>(c->work2);
    aboria_status s = fill_u32(ctx, counts, 0u, (int64_t)nc + 1);
    if (s != ABORIA_OK) return s;
    if (n > 0) {
        const dim3 grid((n + kBlock - 1) / kBlock);
        if (c->nsys == 1)
            hipLaunchKernelGGL((k_cell_ids<T, D, false>), grid, dim3(kBlock), 0, st, (const T*)x, n, sp,
                               c->sys_part_dev, c->nsys, c->keys_alt, ctx->d_flag, counts, c->perm_alt, c->gen);
        else
            hipLaunchKernelGGL((k_cell_ids<T, D, true>), grid, dim3(kBlock), 0, st, (const T*)x, n, sp,
                               c->sys_part_dev, c->nsys, c->keys_alt, ctx->d_flag, counts, c->perm_alt, c->gen);
    }
    s = scan_exclusive_u32(ctx, counts, counts, nc, c->block_sums, c->nblock_sums);
    if (s != ABORIA_OK) return s;
    if (n > 0) {
        const dim3 grid((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_count_place, grid, dim3(kBlock), 0, st, c->keys_alt, c->perm_alt, n, counts,
                           c->block_sums, perm_tmp, key_tmp);
    }
    hipLaunchKernelGGL(k_count_offsets, dim3((nc + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, c->off, nc, n,
                       c->block_sums);
    if (n > 0) {
        const dim3 grid((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_count_finalize<T, D>), grid, dim3(kBlock), 0, st, perm_tmp, key_tmp, n, c->off, nc,
                           (const T*)x, (T*)c->xs, c->keys, c->perm);
    }
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

// Keys per thread of a sort tile for n keys: the largest of 16, 8, 4 that
// still gives at least 512 tiles (2 per CU; the scatter and bucket passes are
// latency-bound with fewer), else 4.  Measured on MI355X: a 2^20 cube builds
// in the same time with 4096- or 2048-key tiles but 25 % faster with 2048 on
// cells of half the width; 2^18 particles build 22 % faster with 1024-key
// tiles; 5.8 M particles in 512 systems are fastest with 4096.
// Key of the radix build-shape cache: d, dtype, batch and the size buckets
// (floor log2) of the particles and the cells.
uint64_t build_key(int32_t d, int32_t dtype, bool batch, int64_t n, int64_t ncells) {
    uint64_t k = (uint64_t)d;
    k = k * 4 + (uint64_t)dtype;
    k = k * 2 + (uint64_t)batch;
    k = k * 64 + (uint64_t)std::floor(std::log2((double)n + 1.0));
    k = k * 64 + (uint64_t)std::floor(std::log2((double)ncells + 1.0));
    return k;
}

int sort_ipt_for(int64_t n) {
    if (n >= (int64_t)512 * kBlock * 16) return 16;
    if (n >= (int64_t)512 * kBlock * 8) return 8;
    return 4;
}

template <typename T, int D, int IPT>
aboria_status launch_build_radix_ipt(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    constexpr int kSortTile = kBlock * IPT;
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    hipStream_t st = ctx->stream;
    // passes over the high bits [lb, key_bits) end in the *_alt buffers; the
    // bucket pass then writes keys / perm
    uint32_t* k0 = (c->passes % 2 == 1) ? c->keys : c->keys_alt;
    uint32_t* kin = k0;
    uint32_t* vin = nullptr;
    const uint32_t* top_scanned = c->block_sums;  // exclusive prefixes of the last pass's scan-block totals
    using Row = VecN<T, Pitch<D>::value>;
    const Row* pay = nullptr;  // position rows in the order of kin (after a radix pass)
    if (n > 0) {
        const uint32_t ntiles = (uint32_t)c->ntiles;
        const uint32_t radix = 1u << c->digit_bits;
        if (c->passes > 0) {  // cell ids with the first pass's digit histogram
            const int shift0 = c->low_bits;
            if (c->nsys == 1)
                hipLaunchKernelGGL((k_cell_ids_hist<T, D, false, IPT>), dim3(ntiles), dim3(IdsThreads<IPT>::value),
                                   radix * sizeof(uint32_t), st, (const T*)x, n, sp, c->sys_part_dev, c->nsys, k0,
                                   ctx->d_flag, c->gen, shift0, c->digit_bits, c->hist, ntiles);
            else
                hipLaunchKernelGGL((k_cell_ids_hist<T, D, true, IPT>), dim3(ntiles), dim3(IdsThreads<IPT>::value),
                                   radix * sizeof(uint32_t), st, (const T*)x, n, sp, c->sys_part_dev, c->nsys, k0,
                                   ctx->d_flag, c->gen, shift0, c->digit_bits, c->hist, ntiles);
        } else {
            const dim3 grid((n + kBlock - 1) / kBlock);
            if (c->nsys == 1)
                hipLaunchKernelGGL((k_cell_ids<T, D, false>), grid, dim3(kBlock), 0, st, (const T*)x, n, sp,
                                   c->sys_part_dev, c->nsys, k0, ctx->d_flag, nullptr, nullptr, c->gen);
            else
                hipLaunchKernelGGL((k_cell_ids<T, D, true>), grid, dim3(kBlock), 0, st, (const T*)x, n, sp,
                                   c->sys_part_dev, c->nsys, k0, ctx->d_flag, nullptr, nullptr, c->gen);
        }
        uint32_t* kout = (k0 == c->keys) ? c->keys_alt : c->keys;
        uint32_t* vout = (k0 == c->keys) ? c->perm_alt : c->perm;
        // Two choices, from measurements on MI355X (2^20 particles in one cube vs 512 systems
        // of up to 65536): shuffling a tile into digit order in LDS (keys, indices and carried
        // rows) makes its writes contiguous but needs tens of KB of LDS (72 KB for 2048 float
        // rows), which pays while the tiles do not outnumber the CUs much (it slowed 1411
        // tiles), and must fit the device's LDS per workgroup; carrying the position rows through the pass turns the
        // bucket pass's random gather into a sequential read, which pays when a system's
        // positions do not fit in L2 (a 12 MB cube: 58 -> 38 us), while the gather of a
        // 0.8 MB system already hits L2 and the payload only adds traffic.
        if (ctx->lds_per_block == 0) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess)
                v = 65536;
            ctx->lds_per_block = v;
        }
        int64_t largest = 0;
        for (int32_t b = 0; b < c->nsys; ++b)
            largest = std::max<int64_t>(largest, c->sys_off[(size_t)b + 1] - c->sys_off[(size_t)b]);
        const bool payload = (uint64_t)largest * D * sizeof(T) > (2u << 20);
        // position rows follow the keys through the passes, ping-ponging between the work buffers
        Row* pout = reinterpret_cast<Row*>(c->work);
        const size_t lds_bytes = (6 * (size_t)radix + 2 * (size_t)kSortTile) * sizeof(uint32_t) +
                                 (payload ? (size_t)kSortTile * sizeof(Row) : 0);
        const bool fits = lds_bytes + (kTopInline + 4) * sizeof(uint32_t) <= (size_t)ctx->lds_per_block;
        const bool shuffle = fits && (c->shuffle_pref == 1 || (c->shuffle_pref == 0 && ntiles <= 512));
        for (int p = 0; p < c->passes; ++p) {
            const int shift = c->low_bits + p * c->digit_bits;
            if (p > 0)  // the first pass's histogram came with the cell ids
                hipLaunchKernelGGL(k_radix_hist<IPT>, dim3(ntiles), dim3(kBlock), radix * sizeof(uint32_t), st, kin,
                                   n, shift, c->digit_bits, c->hist, ntiles);
            const int64_t hl = (int64_t)radix * ntiles;
            const int top_done = scan_block_count(hl) > kTopInline ? 1 : 0;
            aboria_status s = top_done ? scan_exclusive_u32(ctx, c->hist, c->hist, hl, c->block_sums, c->nblock_sums)
                                       : scan_local_u32(ctx, c->hist, c->hist, hl, c->block_sums, c->nblock_sums);
            if (s != ABORIA_OK) return s;
            top_scanned = top_done ? c->block_sums : c->block_sums + c->nblock_sums;
            const int pm = (shuffle ? 1 : 0) | (payload ? 2 : 0);
            const size_t lds_sel = shuffle ? lds_bytes : 6 * (size_t)radix * sizeof(uint32_t);
#define LS(F, SH, PL)                                                                                          \
    hipLaunchKernelGGL((k_radix_scatter<T, D, F, SH, PL, IPT>), dim3(ntiles), dim3(kBlock), lds_sel, st, kin, vin, \
                       (const T*)x, (const Row*)pay, kout, vout, pout, n, shift, c->digit_bits, c->hist,       \
                       c->block_sums, ntiles, top_done, c->block_sums + c->nblock_sums)
            if (p == 0) {
                switch (pm) {
                    case 0: LS(true, false, false); break;
                    case 1: LS(true, true, false); break;
                    case 2: LS(true, false, true); break;
                    default: LS(true, true, true); break;
                }
            } else {
                switch (pm) {
                    case 0: LS(false, false, false); break;
                    case 1: LS(false, true, false); break;
                    case 2: LS(false, false, true); break;
                    default: LS(false, true, true); break;
                }
            }
#undef LS
            std::swap(kin, kout);
            vin = vout;
            vout = (vout == c->perm) ? c->perm_alt : c->perm;
            pay = payload ? pout : nullptr;
            pout = reinterpret_cast<Row*>(pout == reinterpret_cast<Row*>(c->work) ? c->work2 : c->work);
        }
    }
    const uint32_t R = 1u << c->low_bits;
    const uint32_t nbuckets = (uint32_t)(((uint64_t)c->ncells + 1 + R - 1) / R);
    const bool direct = c->passes == 1 && n > 0;
    // Single-chunk buckets assemble their output in LDS when the rows travelled with the
    // keys and the staging area stays small (float rows, tiles of at most 2048 keys).
    constexpr bool kStageable = IPT <= 8 && sizeof(VecN<T, Pitch<D>::value>) <= 16;
    const bool stage = kStageable && pay != nullptr;
    const size_t stage_bytes = (size_t)kSortTile * (2 * sizeof(uint32_t) + sizeof(VecN<T, Pitch<D>::value>));
    constexpr int kBucketThreads = BucketThreads<IPT>::value;
    const size_t cnt_bytes = (2 + kBucketThreads / kWave) * (size_t)R * sizeof(uint32_t);
    if (stage)
        hipLaunchKernelGGL((k_bucket_finalize<T, D, IPT, kStageable>), dim3(nbuckets), dim3(kBucketThreads),
                           cnt_bytes + stage_bytes, st, kin, vin, n, c->low_bits, (uint32_t)c->ncells,
                           (const T*)x, (T*)c->xs, c->keys, c->perm, c->off, direct ? c->hist : nullptr,
                           top_scanned, (uint32_t)c->ntiles, 1u << c->digit_bits, pay);
    else
        hipLaunchKernelGGL((k_bucket_finalize<T, D, IPT, false>), dim3(nbuckets), dim3(kBucketThreads), cnt_bytes,
                           st, kin, vin, n, c->low_bits, (uint32_t)c->ncells, (const T*)x, (T*)c->xs, c->keys,
                           c->perm, c->off, direct ? c->hist : nullptr, top_scanned, (uint32_t)c->ntiles,
                           1u << c->digit_bits, pay);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D>
aboria_status launch_build_radix(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    switch (c->sort_ipt) {
        case 16: return launch_build_radix_ipt<T, D, 16>(ctx, c, x);
        case 8: return launch_build_radix_ipt<T, D, 8>(ctx, c, x);
        default: return launch_build_radix_ipt<T, D, 4>(ctx, c, x);
    }
}

template <typename T, int D>
aboria_status launch_build_single(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    const uint32_t n = (uint32_t)c->n;
    const uint32_t work = std::max<uint32_t>(n, (uint32_t)c->nsys + 1u);
    const dim3 grid((work + kBlock - 1) / kBlock);
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (c->nsys == 1)
        hipLaunchKernelGGL((k_single_cells<T, D, false>), grid, dim3(kBlock), 0, ctx->stream, (const T*)x, n, sp,
                           c->sys_part_dev, c->nsys, (T*)c->xs, c->keys, c->perm, c->off, ctx->d_flag, c->gen);
    else
        hipLaunchKernelGGL((k_single_cells<T, D, true>), grid, dim3(kBlock), 0, ctx->stream, (const T*)x, n, sp,
                           c->sys_part_dev, c->nsys, (T*)c->xs, c->keys, c->perm, c->off, ctx->d_flag, c->gen);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D>
aboria_status launch_build(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    if (c->ncells == c->nsys) return launch_build_single<T, D>(ctx, c, x);  // one cell per system: no sort
    return ctx->build_strategy == ABORIA_BUILD_RADIX ? launch_build_radix<T, D>(ctx, c, x)
                                                     : launch_build_counting<T, D>(ctx, c, x);
}

template <typename T>
aboria_status dispatch_build(aboria_ctx* ctx, aboria_cells* c, const void* x) {
    switch (c->d) {
        case 1: return launch_build<T, 1>(ctx, c, x);
        case 2: return launch_build<T, 2>(ctx, c, x);
        default: return launch_build<T, 3>(ctx, c, x);
    }
}

}  // namespace

aboria_status grid_counts(aboria_ctx* ctx, int dtype, const aboria_box& b, int32_t n[3]) {
    GridPlan g;
    aboria_status s = plan_grid(ctx, dtype, b, &g);
    for (int k = 0; k < 3; ++k) n[k] = g.n[k];
    return s;
}

}  // namespace aboria

using namespace aboria;

extern "C" aboria_status aboria_build_cells(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys,
                                            const aboria_box* boxes_host, const int64_t* offsets_host,
                                            const void* x, aboria_cells** cells) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    try {
        if (!cells) return fail(ctx, ABORIA_ERR_INVALID_ARG, "cells out-pointer is NULL");
        if (dtype != ABORIA_F32 && dtype != ABORIA_F64) return fail(ctx, ABORIA_ERR_INVALID_ARG, "unknown dtype");
        if (nsys < 1 || !boxes_host || !offsets_host)
            return fail(ctx, ABORIA_ERR_INVALID_ARG, "need nsys >= 1, boxes and offsets");
        const int32_t d = boxes_host[0].d;
        if (d < 1 || d > 3) return fail(ctx, ABORIA_ERR_INVALID_ARG, "d must be 1, 2 or 3");
        if (offsets_host[0] != 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "offsets must start at 0");
        for (int32_t b = 0; b < nsys; ++b) {
            if (boxes_host[b].d != d) return fail(ctx, ABORIA_ERR_INVALID_ARG, "all boxes must share d");
            if (offsets_host[b + 1] < offsets_host[b]) return fail(ctx, ABORIA_ERR_INVALID_ARG, "offsets must not decrease");
        }
        const int64_t n = offsets_host[nsys];
        if (n >= (int64_t)1 << 31) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "at most 2^31 - 1 particles");
        if (n > 0 && !x) return fail(ctx, ABORIA_ERR_INVALID_ARG, "x is NULL");
        std::vector<GridPlan> plans((size_t)nsys);
        std::vector<uint32_t> cell_base((size_t)nsys + 1, 0);
        int64_t total_cells = 0;
        for (int32_t b = 0; b < nsys; ++b) {
            aboria_status s = plan_grid(ctx, dtype, boxes_host[b], &plans[b]);
            if (s != ABORIA_OK) return s;
            cell_base[b] = (uint32_t)total_cells;
            total_cells += plans[b].ncells;
            if (total_cells > 2147483647LL) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "more than 2^31 cells in total");
        }
        cell_base[nsys] = (uint32_t)total_cells;
        std::vector<aboria_box> boxes(boxes_host, boxes_host + nsys);
        std::vector<int64_t> off(offsets_host, offsets_host + nsys + 1);
        std::vector<unsigned char> params;
        if (dtype == ABORIA_F32) fill_params<float>(plans, boxes, cell_base, off, &params);
        else fill_params<double>(plans, boxes, cell_base, off, &params);

        aboria_cells* c = *cells;
        const bool create = c == nullptr;
        if (!create) {
            if (c->nsys != nsys || c->d != d || c->dtype != dtype || c->n != n)
                return fail(ctx, ABORIA_ERR_INVALID_ARG, "rebuild must keep nsys, d, dtype and n");
            if (c->ncells != total_cells || c->sys_off != off)
                return fail(ctx, ABORIA_ERR_INVALID_ARG, "rebuild must keep the cell counts and system offsets");
        }
        if (create) {
            if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "a first build allocates and cannot be captured");
            ABORIA_HIP(ctx, hipSetDevice(ctx->device));
            c = new (std::nothrow) aboria_cells();
            if (!c) return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host allocation failed");
            c->device = ctx->device;
            c->dtype = dtype;
            c->d = d;
            c->nsys = nsys;
            c->n = n;
            c->ncells = total_cells;
            c->pitch = d == 3 ? 4 : d;
            c->sys_off = off;
            int32_t bits = 1;
            while (bits < 32 && ((int64_t)1 << bits) < total_cells) ++bits;
            c->key_bits = bits;
            // the bucket pass sorts the low bits (8 to 10 of them); LDS-ranked
            // radix passes of at most 10 bits sort the rest first
            c->low_bits = std::min(bits, std::max(8, std::min(bits - kMaxDigitBits, kMaxDigitBits)));
            c->sort_ipt = sort_ipt_for(n);
            // a forced shape, else the tuned one for this size, replaces the rule
            aboria_ctx::BuildShape shape = ctx->build_forced;
            if (shape.ipt == 0 && shape.low_bits == 0 && shape.shuffle == 0) {
                const uint64_t bkey = build_key(d, dtype, nsys > 1, n, total_cells);
                for (const auto& kv : ctx->build_cache)
                    if (kv.first == bkey) shape = kv.second;
            }
            if (shape.ipt == 4 || shape.ipt == 8 || shape.ipt == 16) c->sort_ipt = shape.ipt;
            if (shape.low_bits >= 8 && shape.low_bits <= kMaxDigitBits) c->low_bits = std::min(bits, shape.low_bits);
            if (shape.shuffle == 1 || shape.shuffle == 2) c->shuffle_pref = shape.shuffle;
            const int high = bits - c->low_bits;
            c->passes = (high + kMaxDigitBits - 1) / kMaxDigitBits;
            c->digit_bits = c->passes > 0 ? (high + c->passes - 1) / c->passes : 1;
            c->ntiles = (n + (int64_t)kBlock * c->sort_ipt - 1) / ((int64_t)kBlock * c->sort_ipt);
            c->hist_len = ((int64_t)1 << c->digit_bits) * std::max<int64_t>(c->ntiles, 1);
            c->nblock_sums = std::max<int64_t>(std::max(scan_block_count(c->hist_len),
                                                        scan_block_count(total_cells + 1)), 1);
            const size_t tsz = dtype == ABORIA_F32 ? 4 : 8;
            const size_t nn = (size_t)std::max<int64_t>(n, 1);
            struct Alloc { void** p; size_t bytes; } allocs[] = {
                {&c->params_dev, params.size()},
                {(void**)&c->sys_part_dev, sizeof(uint32_t) * ((size_t)nsys + 1)},
                {(void**)&c->cell_base_dev, sizeof(uint32_t) * ((size_t)nsys + 1)},
                {(void**)&c->keys, sizeof(uint32_t) * nn},
                {(void**)&c->perm, sizeof(uint32_t) * nn},
                {(void**)&c->keys_alt, sizeof(uint32_t) * nn},
                {(void**)&c->perm_alt, sizeof(uint32_t) * nn},
                {(void**)&c->off, sizeof(uint32_t) * ((size_t)total_cells + 1)},
                {&c->xs, tsz * (size_t)c->pitch * nn},
                {&c->work, tsz * 4 * nn},
                {&c->work2, tsz * 4 * nn},
                {(void**)&c->hist, sizeof(uint32_t) * (size_t)c->hist_len},
                // raw block totals, then (second half) the radix pass's scanned copy
                {(void**)&c->block_sums, sizeof(uint32_t) * 2 * (size_t)c->nblock_sums},
                {(void**)&c->gen, sizeof(uint32_t) * 2},
            };
            for (auto& a : allocs) {
                if (hipMalloc(a.p, a.bytes) != hipSuccess) {
                    (void)hipGetLastError();
                    free_cells_buffers(c);
                    delete c;
                    return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "device allocation for the cell list failed");
                }
            }
            std::vector<uint32_t> part((size_t)nsys + 1);
            for (int32_t b = 0; b <= nsys; ++b) part[b] = (uint32_t)off[b];
            const uint32_t gen0[2] = {kGenNone, kGenNeverListed};  // build generation, generation of the recorded list
            hipError_t e = hipMemcpyAsync(c->sys_part_dev, part.data(), part.size() * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->gen, gen0, sizeof(gen0), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) {
                free_cells_buffers(c);
                delete c;
                return hip_fail(ctx, e, "upload of system offsets");
            }
        }
        if (create || c->params_host != params) {
            if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "changing boxes inside a graph capture");
            hipError_t e = hipMemcpyAsync(c->params_dev, params.data(), params.size(), hipMemcpyHostToDevice,
                                          ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->cell_base_dev, cell_base.data(), cell_base.size() * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) {
                if (create) { free_cells_buffers(c); delete c; }
                return hip_fail(ctx, e, "upload of box parameters");
            }
            c->params_host = params;
            c->boxes = boxes;
            c->cell_base = cell_base;
            c->ncell_host.assign((size_t)nsys * 3, 1);
            for (int32_t b = 0; b < nsys; ++b)
                for (int k = 0; k < 3; ++k) c->ncell_host[(size_t)b * 3 + k] = plans[b].n[k];
        }
        aboria_status s = dtype == ABORIA_F32 ? dispatch_build<float>(ctx, c, x) : dispatch_build<double>(ctx, c, x);
        if (s != ABORIA_OK) {
            if (create) { free_cells_buffers(c); delete c; }
            return s;
        }
        *cells = c;
        return ABORIA_OK;
    } catch (...) {
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception during build");
    }
}

extern "C" aboria_status aboria_cells_view_get(const aboria_cells* c, aboria_cells_view* out) {
    if (!c || !out) return ABORIA_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    out->nsys = c->nsys;
    out->d = c->d;
    out->dtype = c->dtype;
    out->n = c->n;
    out->ncells = c->ncells;
    out->perm = c->perm;
    out->keys = c->keys;
    out->cell_offsets = c->off;
    out->x_sorted = c->xs;
    out->x_pitch = c->pitch;
    out->sort_ipt = c->sort_ipt;
    out->bucket_bits = c->low_bits;
    out->ncell_host = c->ncell_host.data();
    out->cell_base_host = c->cell_base.data();
    out->sys_offsets_host = c->sys_off.data();
    return ABORIA_OK;
}

static void release_cells(void* p) {
    aboria_cells* c = static_cast<aboria_cells*>(p);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_cells_buffers(c);
    delete c;
}

extern "C" aboria_status aboria_cells_destroy(aboria_cells* c) {
    if (!c) return ABORIA_OK;
    aboria::release_or_defer(release_cells, c);
    return ABORIA_OK;
}

extern "C" aboria_status aboria_set_build_shape(aboria_ctx* ctx, int32_t ipt, int32_t low_bits, int32_t shuffle) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ipt != 0 && ipt != 4 && ipt != 8 && ipt != 16)
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "keys per thread must be 0, 4, 8 or 16");
    if (low_bits != 0 && (low_bits < 8 || low_bits > kMaxDigitBits))
        return fail(ctx, ABORIA_ERR_INVALID_ARG, "bucket bits must be 0 or 8 to 10");
    if (shuffle < 0 || shuffle > 2) return fail(ctx, ABORIA_ERR_INVALID_ARG, "shuffle must be 0, 1 or 2");
    ctx->build_forced = aboria_ctx::BuildShape{ipt, low_bits, shuffle};
    return ABORIA_OK;
}

extern "C" aboria_status aboria_autotune_build(aboria_ctx* ctx, aboria_dtype dtype, int32_t nsys,
                                               const aboria_box* boxes_host, const int64_t* offsets_host,
                                               const void* x, int32_t* ipt_out, int32_t* low_bits_out,
                                               int32_t* shuffle_out) {
    if (!ctx) return ABORIA_ERR_INVALID_ARG;
    if (ctx->capturing) return fail(ctx, ABORIA_ERR_UNSUPPORTED, "autotune cannot be captured");
    if (nsys < 1 || !boxes_host || !offsets_host) return fail(ctx, ABORIA_ERR_INVALID_ARG, "need boxes and offsets");
    const aboria_ctx::BuildShape forced_before = ctx->build_forced;
    const int32_t strategy_before = ctx->build_strategy;
    try {
        ABORIA_HIP(ctx, hipSetDevice(ctx->device));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return hip_fail(ctx, hipGetLastError(), "hipEventCreate");
        }
        ctx->build_strategy = ABORIA_BUILD_RADIX;
        aboria_status st = ABORIA_OK;
        double best_ms = INFINITY;
        aboria_ctx::BuildShape best{0, 0, 0};
        int64_t ncells = 0, n = offsets_host[nsys];
        const int32_t ipts[] = {4, 8, 16};
        const int32_t lows[] = {8, 9, 10};
        int32_t last_bits = -1;
        for (int32_t ipt : ipts) {
            for (int32_t lb : lows) for (int32_t sh = 1; sh <= 2; ++sh) {
                if (st != ABORIA_OK) break;
                ctx->build_forced = aboria_ctx::BuildShape{ipt, lb, sh};
                aboria_cells* c = nullptr;
                st = aboria_build_cells(ctx, dtype, nsys, boxes_host, offsets_host, x, &c);
                if (st != ABORIA_OK) break;
                ncells = c->ncells;
                if (c->low_bits != lb && lb != lows[0]) {  // fewer key bits than lb: a smaller lb's shape
                    (void)aboria_cells_destroy(c);
                    continue;
                }
                last_bits = c->key_bits;
                (void)hipEventRecord(e0, ctx->stream);
                for (int rep = 0; rep < 5 && st == ABORIA_OK; ++rep)
                    st = aboria_build_cells(ctx, dtype, nsys, boxes_host, offsets_host, x, &c);
                (void)hipEventRecord(e1, ctx->stream);
                if (hipEventSynchronize(e1) != hipSuccess) st = hip_fail(ctx, hipGetLastError(), "timing a build");
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                (void)aboria_cells_destroy(c);
                if (st != ABORIA_OK) break;
                log_msg("autotune_build: %d keys per thread, %d bucket bits, shuffle %s: %.4f ms", ipt, lb,
                        sh == 1 ? "on" : "off", ms / 5.0);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = aboria_ctx::BuildShape{ipt, lb, sh};
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->build_forced = forced_before;
        ctx->build_strategy = strategy_before;
        if (st != ABORIA_OK) return st;
        if (best.ipt == 0) return fail(ctx, ABORIA_ERR_INVALID_ARG, "no build shape could be timed");
        const uint64_t key = build_key(boxes_host[0].d, dtype, nsys > 1, n, ncells);
        bool found = false;
        for (auto& kv : ctx->build_cache)
            if (kv.first == key) {
                kv.second = best;
                found = true;
            }
        if (!found) ctx->build_cache.emplace_back(key, best);
        tune_cache_save(ctx);
        log_msg("autotune_build: %d keys per thread, %d bucket bits, shuffle %s chosen (%d key bits)", best.ipt,
                best.low_bits, best.shuffle == 1 ? "on" : "off", last_bits);
        if (ipt_out) *ipt_out = best.ipt;
        if (low_bits_out) *low_bits_out = best.low_bits;
        if (shuffle_out) *shuffle_out = best.shuffle;
        return ABORIA_OK;
    } catch (...) {
        ctx->build_forced = forced_before;
        ctx->build_strategy = strategy_before;
        return fail(ctx, ABORIA_ERR_OUT_OF_MEMORY, "host exception in autotune_build");
    }
}
