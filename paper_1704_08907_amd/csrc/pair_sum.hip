// Radius-limited neighbour sums over the cell list: the Level 2 box search of
// Section 2.2.2 (a particle's cell and its adjacent cells) evaluating the
// summand of a sum(j, 0 < |dx| < r, f) operator (Section 3, eq. (1) and the
// velocity-update listing), its adjoint, and a pair listing for verification.
//
// Work mapping: one lane per particle in cell order, so the lanes of a wave
// share home cells and therefore candidate cells (their loads hit the same
// cache lines).  The 3^d neighbour cells are walked as 3^(d-1) rows, each row
// a contiguous slot range [off[first cell], off[last cell + 1]) of up to three
// cells along x (split where a periodic wrap changes the image shift).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "common.hpp"

namespace aboria {

constexpr int kPairBlock = 256;

// ---------------------------------------------------------------------------
// precision-specific primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return ::rsqrt(x); }
__device__ __forceinline__ float exp_neg_t(float s) { return __builtin_amdgcn_exp2f(-s * 1.4426950408889634f); }
__device__ __forceinline__ double exp_neg_t(double s) { return ::exp(-s); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// operators: forward summand and the adjoint contribution of one ordered pair
// (i = the lane's particle, j = its neighbour; dx = x_j + shift - x_i = -u)
// ---------------------------------------------------------------------------

template <typename T>
struct OpArgs {
    T p0;  // k (spring, DEM spring) or c (exp force)
};

template <int OP, int D>
struct OpShape {
    static constexpr int NY = (OP == ABORIA_OP_COUNT || OP == ABORIA_OP_SOFT_SPHERE) ? 1 : D;
    static constexpr int NA = OP == ABORIA_OP_DEM_SPRING ? 1 : 0;
};

template <typename T, int D, int OP>
struct PairOp {
    static constexpr int NY = OpShape<OP, D>::NY;

    // acc += f(x_i, x_j, a_i, a_j)
    __device__ __forceinline__ static void fwd(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj, T* acc) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            acc[0] += T(1);
        } else if constexpr (OP == ABORIA_OP_SPRING) {
            // k (r - s) u / s = (k r / s - k) u,  u = -dx
            const T rinv = rsqrt_t(d2);
            const T g = fma_t(q.p0 * r, rinv, -q.p0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T s = d2 * rsqrt_t(d2);
            const T v = fma_t(-s, T(1) / r, T(1));
            acc[0] = fma_t(T(0.5) * v, v, acc[0]);
        } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
            // eq. (1): -c exp(-|dx|) dx / |dx|
            const T rinv = rsqrt_t(d2);
            const T s = d2 * rinv;
            const T g = q.p0 * exp_neg_t(s) * rinv;
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        } else {  // DEM spring: k (a_i + a_j - s) u / s
            const T rinv = rsqrt_t(d2);
            const T g = fma_t(q.p0 * (ai + aj), rinv, -q.p0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        }
    }

    // Branchless forms: every lane evaluates the summand and keeps it only if
    // ok (a select, never a multiply, so the inf/NaN a rejected or sentinel
    // candidate produces cannot leak into the sums).
    __device__ __forceinline__ static void fwd_masked(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj, bool ok,
                                                      T* acc) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            acc[0] += ok ? T(1) : T(0);
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T s = d2 * rsqrt_t(d2);
            const T v = fma_t(-s, T(1) / r, T(1));
            const T term = T(0.5) * v * v;
            acc[0] += ok ? term : T(0);
        } else {
            const T rinv = rsqrt_t(d2);
            T g;
            if constexpr (OP == ABORIA_OP_SPRING) {
                g = fma_t(q.p0 * r, rinv, -q.p0);
            } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
                g = q.p0 * exp_neg_t(d2 * rinv) * rinv;
            } else {
                g = fma_t(q.p0 * (ai + aj), rinv, -q.p0);
            }
            g = ok ? g : T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[k] = fma_t(-g, dx[k], acc[k]);
        }
    }

    __device__ __forceinline__ static void bwd_masked(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj,
                                                      const T* gyi, const T* gyj, bool ok, T* gx, T* ga) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            return;
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T rinv = rsqrt_t(d2);
            const T s = d2 * rinv;
            const T inv_r = T(1) / r;
            T coef = (gyi[0] + gyj[0]) * inv_r * fma_t(-s, inv_r, T(1)) * rinv;
            coef = ok ? coef : T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(coef, dx[k], gx[k]);
        } else {
            const T rinv = rsqrt_t(d2);
            const T rinv3 = rinv * rinv * rinv;
            T w[D];
            T dw = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                w[k] = gyi[k] - gyj[k];
                dw = fma_t(dx[k], w[k], dw);
            }
            T g, gps;
            if constexpr (OP == ABORIA_OP_SPRING) {
                g = fma_t(q.p0 * r, rinv, -q.p0);
                gps = -q.p0 * r * rinv3;
            } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
                const T s = d2 * rinv;
                const T ce = q.p0 * exp_neg_t(s);
                g = ce * rinv;
                gps = -ce * (s + T(1)) * rinv3;
            } else {
                const T A = ai + aj;
                g = fma_t(q.p0 * A, rinv, -q.p0);
                gps = -q.p0 * A * rinv3;
                const T ta = -q.p0 * dw * rinv;
                ga[0] += ok ? ta : T(0);
            }
            g = ok ? g : T(0);
            const T h = ok ? gps * dw : T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(g, w[k], fma_t(h, dx[k], gx[k]));
        }
    }

    // gx += J1(i,j)^T gy_i + J2(j,i)^T gy_j ; ga += d/da_i of the same.
    // For f = g(s) u:  gx += g w + (g'/s)(u.w) u with w = gy_i - gy_j, and
    // (u.w) u = (dx.w) dx.  For the soft sphere: gx += 1/2 (gy_i + gy_j)
    // phi'(s) u/s with phi'(s) = -(2/r)(1 - s/r).
    __device__ __forceinline__ static void bwd(const OpArgs<T>& q, T r, const T* dx, T d2, T ai, T aj,
                                               const T* gyi, const T* gyj, T* gx, T* ga) {
        if constexpr (OP == ABORIA_OP_COUNT) {
            return;
        } else if constexpr (OP == ABORIA_OP_SOFT_SPHERE) {
            const T rinv = rsqrt_t(d2);
            const T s = d2 * rinv;
            const T inv_r = T(1) / r;
            const T coef = (gyi[0] + gyj[0]) * inv_r * fma_t(-s, inv_r, T(1)) * rinv;
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(coef, dx[k], gx[k]);
        } else {
            const T rinv = rsqrt_t(d2);
            const T rinv3 = rinv * rinv * rinv;
            T w[D];
            T dw = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                w[k] = gyi[k] - gyj[k];
                dw = fma_t(dx[k], w[k], dw);
            }
            T g, gps;  // g(s) and g'(s)/s
            if constexpr (OP == ABORIA_OP_SPRING) {
                g = fma_t(q.p0 * r, rinv, -q.p0);
                gps = -q.p0 * r * rinv3;
            } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
                const T s = d2 * rinv;
                const T ce = q.p0 * exp_neg_t(s);
                g = ce * rinv;
                gps = -ce * (s + T(1)) * rinv3;
            } else {
                const T A = ai + aj;
                g = fma_t(q.p0 * A, rinv, -q.p0);
                gps = -q.p0 * A * rinv3;
                // d/da_i: k (gy_i - gy_j).u / s = -k (w.dx) / s
                ga[0] = fma_t(-q.p0 * dw, rinv, ga[0]);
            }
            const T h = gps * dw;
#pragma unroll
            for (int k = 0; k < D; ++k) gx[k] = fma_t(g, w[k], fma_t(h, dx[k], gx[k]));
        }
    }
};

// ---------------------------------------------------------------------------
// the neighbour loop
// ---------------------------------------------------------------------------

// Calls visit(j, dx, d2) for every neighbour j of the point xi (cell order
// slot), dx = fl(fl(x_j - x_i) + shift) per dimension and d2 the fma chain,
// accepted iff 0 < d2 < r2.
template <typename T, int D, typename Visit>
__device__ __forceinline__ void neighbour_loop(const SysParams<T>& P, const T* __restrict__ xs,
                                               const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                               Visit&& visit) {
    constexpr int PITCH = Pitch<D>::value;
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T t = xi[k] - P.lo[k];
        const T q = t * P.inv_w[k];
        const T f = floor(q);
        c[k] = !(f >= T(0)) ? 0 : (f > T(P.n[k] - 1) ? P.n[k] - 1 : (int32_t)f);
    }
    // pieces of the x extent [c0-1, c0+1]: contiguous runs with one image shift
    const int32_t nx = P.n[0];
    int np = 0;
    int32_t plo[3], phi[3];
    T psh[3];
    if (nx >= 3) {
        plo[0] = c[0] > 0 ? c[0] - 1 : 0;
        phi[0] = c[0] < nx - 1 ? c[0] + 1 : nx - 1;
        psh[0] = T(0);
        np = 1;
        if (P.periodic[0]) {
            if (c[0] == 0) { plo[np] = phi[np] = nx - 1; psh[np] = -P.L[0]; ++np; }
            if (c[0] == nx - 1) { plo[np] = phi[np] = 0; psh[np] = P.L[0]; ++np; }
        }
    } else {
        for (int o = -1; o <= 1; ++o) {
            int32_t v = c[0] + o;
            T s = T(0);
            if (v < 0) { if (!P.periodic[0]) continue; v += nx; s = -P.L[0]; }
            else if (v >= nx) { if (!P.periodic[0]) continue; v -= nx; s = P.L[0]; }
            plo[np] = phi[np] = v;
            psh[np] = s;
            ++np;
        }
    }
    constexpr int NROWS = D == 1 ? 1 : (D == 2 ? 3 : 9);
    for (int rr = 0; rr < NROWS; ++rr) {
        T sh[3] = {T(0), T(0), T(0)};
        uint32_t row = 0;
        bool skip = false;
        if constexpr (D >= 2) {
            int32_t v = c[1] + (rr % 3) - 1;
            if (v < 0) { if (!P.periodic[1]) skip = true; v += P.n[1]; sh[1] = -P.L[1]; }
            else if (v >= P.n[1]) { if (!P.periodic[1]) skip = true; v -= P.n[1]; sh[1] = P.L[1]; }
            row = (uint32_t)v;
        }
        if constexpr (D >= 3) {
            int32_t v = c[2] + (rr / 3) - 1;
            if (v < 0) { if (!P.periodic[2]) skip = true; v += P.n[2]; sh[2] = -P.L[2]; }
            else if (v >= P.n[2]) { if (!P.periodic[2]) skip = true; v -= P.n[2]; sh[2] = P.L[2]; }
            row += (uint32_t)P.n[1] * (uint32_t)v;
        }
        if (skip) continue;
        const uint32_t rowbase = P.cell_base + (uint32_t)nx * row;
        for (int p = 0; p < np; ++p) {
            const uint32_t j0 = off[rowbase + plo[p]];
            const uint32_t j1 = min(off[rowbase + phi[p] + 1], n);
            sh[0] = psh[p];
            for (uint32_t j = j0; j < j1; ++j) {
                const VecN<T, PITCH> xj = reinterpret_cast<const VecN<T, PITCH>*>(xs)[j];
                T dx[D];
#pragma unroll
                for (int k = 0; k < D; ++k) dx[k] = (xj.v[k] - xi[k]) + sh[k];
                T d2 = dx[0] * dx[0];
                if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
                if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
                if (d2 > T(0) && d2 < P.r2) visit(j, dx, d2);
            }
        }
    }
}

__device__ __forceinline__ int find_system_slot(const uint32_t* __restrict__ first, int nsys, uint32_t i) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T, int D>
__device__ __forceinline__ void load_point(const T* __restrict__ xs, uint32_t s, T* xi) {
    constexpr int PITCH = Pitch<D>::value;
    const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[s];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = v.v[k];
}

// Forward: y[perm[s]] = sum over the neighbours of slot s.
template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(kPairBlock) void k_pair_fwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ perm, uint32_t n,
                                                         const SysParams<T>* __restrict__ sp,
                                                         const uint32_t* __restrict__ sys_part, int nsys,
                                                         const T* __restrict__ a_s, OpArgs<T> q,
                                                         T* __restrict__ y) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int b = BATCH ? find_system_slot(sys_part, nsys, s) : 0;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    const T r = P.r;
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    });
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
}

// Adjoint: gx[perm[s]] (and ga) gathered over the neighbours of slot s, with
// gy_s the upstream gradient already in cell order.
template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(kPairBlock) void k_pair_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ perm, uint32_t n,
                                                         const SysParams<T>* __restrict__ sp,
                                                         const uint32_t* __restrict__ sys_part, int nsys,
                                                         const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                         OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int b = BATCH ? find_system_slot(sys_part, nsys, s) : 0;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) gyi[k] = gy_s[(size_t)s * NY + k];
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        T gyj[NY];
#pragma unroll
        for (int k = 0; k < NY; ++k) gyj[k] = gy_s[(size_t)j * NY + k];
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    });
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

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
    neighbour_loop<T, D>(P, xs, off, n, xi, [&](uint32_t j, const T*, T) {
        if (FILL) {
            const uint64_t at = base + cnt;
            if (at < cap) {
                pi[at] = me;
                pj[at] = perm[j];
            }
        }
        ++cnt;
    });
    if (!FILL) counts[s] = cnt;
}

// dst[s][w] = src[perm[s]][w]
template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ src, const uint32_t* __restrict__ perm,
                                                     uint32_t n, int w, T* __restrict__ dst) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n * (uint32_t)w) return;
    const uint32_t s = t / w, k = t - s * w;
    dst[t] = src[(size_t)perm[s] * w + k];
}

// ---------------------------------------------------------------------------
// cell-group work mapping
//
// A group of 16 lanes owns one home cell.  The candidates of the cell (its
// 3^d neighbour cells, as up to 3^(d-1) x-rows of at most three pieces each)
// form one flattened list; lane l of the group takes entries l, l+16, l+32, ...
// walking a cursor over the group's piece table in LDS.  Each candidate is
// loaded once into registers and tested against every home particle of the
// current pass (up to IMAX, held in registers in all 16 lanes), so one load
// feeds IMAX pair tests.  Home slots beyond the cell's particles, and list
// entries beyond its candidates, hold far-away sentinel points whose squared
// distance overflows to +inf and is rejected by the predicate, so the
// unrolled i-loop needs no per-lane guard; the loop bounds are wave-uniform
// maxima over the wave's four groups.  At the end each home particle's sums
// are reduced across the 16 lanes with a xor butterfly and written to its
// original index.
// ---------------------------------------------------------------------------

constexpr int kGroup = 16;

template <typename T>
struct Far;
template <>
struct Far<float> {
    __device__ static constexpr float home() { return 1e30f; }
    __device__ static constexpr float cand() { return -1e30f; }
};
template <>
struct Far<double> {
    __device__ static constexpr double home() { return 1e300; }
    __device__ static constexpr double cand() { return -1e300; }
};

__device__ __forceinline__ uint32_t wave_max_of_groups(uint32_t v) {
    // v is uniform within each 16-lane group; lanes 0, 16, 32, 48 lead the groups
    uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

__device__ __forceinline__ int find_system_cell(const uint32_t* __restrict__ cell_base, int nsys, uint32_t c) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cell_base[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) v += __shfl_xor(v, m, kGroup);
    return v;
}

// Shift of one dimension from its 2-bit code: 0 -> -L, 1 -> 0, 2 -> +L.
template <typename T>
__device__ __forceinline__ T shift_of(uint32_t code, int k, T L) {
    const uint32_t m = (code >> (2 * k)) & 3u;
    return m == 0u ? -L : (m == 2u ? L : T(0));
}

template <typename T, int D, int OP, bool BATCH, bool BWD, int IMAX, int BLOCK, int ROUNDS>
__global__ __launch_bounds__(BLOCK) void k_pair_cells(
    const T* __restrict__ xs, const uint32_t* __restrict__ off, const uint32_t* __restrict__ perm, uint32_t n,
    uint32_t nwork, const SysParams<T>* __restrict__ sp, const uint32_t* __restrict__ cell_base, int nsys,
    const T* __restrict__ a_s, const T* __restrict__ gy_s, OpArgs<T> q, T* __restrict__ out,
    T* __restrict__ out_a) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr int NY = OpShape<OP, D>::NY;
    constexpr bool HAS_A = OpShape<OP, D>::NA > 0;
    constexpr int NROWS = D == 1 ? 1 : (D == 2 ? 3 : 9);
    constexpr int NPIECE = 3 * NROWS;
    constexpr int GPB = BLOCK / kGroup;
    constexpr int TILE = GPB * ROUNDS;  // cells per workgroup
    static_assert(TILE <= BLOCK, "one thread ranks one cell of the tile");
    constexpr uint32_t kCenter = D == 1 ? 1u : (D == 2 ? 5u : 21u);  // every dimension unshifted
    using Op = PairOp<T, D, OP>;

    __shared__ uint32_t s_start[GPB][NPIECE];
    __shared__ uint32_t s_cum[GPB][NPIECE + 1];
    __shared__ uint32_t s_code[GPB][NPIECE];
    __shared__ uint32_t s_key[TILE];
    __shared__ uint32_t s_order[TILE];

    const int g = threadIdx.x / kGroup;
    const int l = threadIdx.x % kGroup;
    const uint32_t tile_base = xcd_tile(blockIdx.x, gridDim.x) * TILE;

    // Rank the tile's cells by (stencil wraps, occupancy) so that the four
    // groups of a wave get cells of equal occupancy and equal wrap status.
    if (ROUNDS > 1) {
        if (threadIdx.x < TILE) {
            const uint32_t cell = tile_base + threadIdx.x;
            uint32_t key = 0xFFFFFFFFu;
            if (cell < nwork) {
                const int bb = BATCH ? find_system_cell(cell_base, nsys, cell) : 0;
                const SysParams<T>& Pb = sp[bb];
                uint32_t rest = cell - Pb.cell_base;
                bool wraps = false;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const uint32_t ck = rest % (uint32_t)Pb.n[k];
                    rest /= (uint32_t)Pb.n[k];
                    wraps |= Pb.periodic[k] && (ck == 0u || ck + 1u >= (uint32_t)Pb.n[k]);
                }
                key = ((uint32_t)wraps << 16) | min(off[cell + 1] - off[cell], 0xFFFFu);
            }
            s_key[threadIdx.x] = key;
        }
        __syncthreads();
        if (threadIdx.x < TILE) {
            const uint32_t me = s_key[threadIdx.x];
            uint32_t rank = 0;
            for (int u = 0; u < TILE; ++u) {
                const uint32_t ku = s_key[u];
                rank += (ku < me || (ku == me && u < (int)threadIdx.x)) ? 1u : 0u;
            }
            s_order[rank] = threadIdx.x;
        }
        __syncthreads();
    }

    for (int round = 0; round < ROUNDS; ++round) {
        const uint32_t slot_in_tile = (uint32_t)(round * GPB + g);
        const uint32_t gid = tile_base + (ROUNDS > 1 ? s_order[slot_in_tile] : slot_in_tile);
        const bool has_cell = gid < nwork;
        const uint32_t cell = has_cell ? gid : 0u;
        const int b = (BATCH && has_cell) ? find_system_cell(cell_base, nsys, cell) : 0;
        const SysParams<T> P = sp[b];
        const uint32_t local = cell - P.cell_base;
        int32_t c[3] = {0, 0, 0};
        {
            uint32_t rest = local;
            c[0] = (int32_t)(rest % (uint32_t)P.n[0]);
            rest /= (uint32_t)P.n[0];
            if (D >= 2) { c[1] = (int32_t)(rest % (uint32_t)P.n[1]); rest /= (uint32_t)P.n[1]; }
            if (D >= 3) c[2] = (int32_t)rest;
        }
        const uint32_t hbeg = has_cell ? off[cell] : 0u;
        const uint32_t nhome = has_cell ? off[cell + 1] - hbeg : 0u;

        // piece table: lane l < NROWS fills the three x-pieces of row l
        if (l < NROWS) {
            int32_t row = 0;
            uint32_t ycode = 0;
            bool skip = !has_cell;
            if (D >= 2) {
                int32_t v = c[1] + (l % 3) - 1, m = 1;
                if (v < 0) { if (!P.periodic[1]) skip = true; v += P.n[1]; m = 0; }
                else if (v >= P.n[1]) { if (!P.periodic[1]) skip = true; v -= P.n[1]; m = 2; }
                row = v;
                ycode |= (uint32_t)m << 2;
            }
            if (D >= 3) {
                int32_t v = c[2] + (l / 3) - 1, m = 1;
                if (v < 0) { if (!P.periodic[2]) skip = true; v += P.n[2]; m = 0; }
                else if (v >= P.n[2]) { if (!P.periodic[2]) skip = true; v -= P.n[2]; m = 2; }
                row += P.n[1] * v;
                ycode |= (uint32_t)m << 4;
            }
            const int32_t nx = P.n[0];
            const uint32_t rowbase = P.cell_base + (uint32_t)nx * (uint32_t)row;
            int32_t lo_[3] = {0, 0, 0}, hi_[3] = {-1, -1, -1};
            uint32_t xm[3] = {1, 1, 1};
            if (!skip) {
                if (nx >= 3) {
                    lo_[0] = c[0] > 0 ? c[0] - 1 : 0;
                    hi_[0] = c[0] < nx - 1 ? c[0] + 1 : nx - 1;
                    if (P.periodic[0] && c[0] == 0) { lo_[1] = hi_[1] = nx - 1; xm[1] = 0; }
                    if (P.periodic[0] && c[0] == nx - 1) { lo_[2] = hi_[2] = 0; xm[2] = 2; }
                } else {
                    for (int o = -1; o <= 1; ++o) {
                        int32_t v = c[0] + o;
                        uint32_t m = 1;
                        if (v < 0) { if (!P.periodic[0]) continue; v += nx; m = 0; }
                        else if (v >= nx) { if (!P.periodic[0]) continue; v -= nx; m = 2; }
                        lo_[o + 1] = hi_[o + 1] = v;
                        xm[o + 1] = m;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int p = 3 * l + k;
                uint32_t st = 0, len = 0;
                if (hi_[k] >= lo_[k]) {
                    st = off[rowbase + lo_[k]];
                    len = min(off[rowbase + hi_[k] + 1], n) - st;
                }
                s_start[g][p] = st;
                s_cum[g][p + 1] = len;
                s_code[g][p] = ycode | xm[k];
            }
        }
        __syncthreads();
        if (l == 0) {
            uint32_t acc = 0;
            s_cum[g][0] = 0;
            for (int p = 0; p < NPIECE; ++p) {
                acc += s_cum[g][p + 1];
                s_cum[g][p + 1] = acc;
            }
        }
        __syncthreads();

        const uint32_t M = s_cum[g][NPIECE];
        bool shifted = false;
        for (int p = 0; p < NPIECE; ++p) shifted |= (s_code[g][p] != kCenter) && (s_cum[g][p + 1] > s_cum[g][p]);
        const bool wave_shift = __ballot(shifted) != 0ull;
        const uint32_t Mw = wave_max_of_groups(M);
        const uint32_t passes_w = wave_max_of_groups((nhome + IMAX - 1) / IMAX);
        const T r = P.r;
        const T r2 = P.r2;

        for (uint32_t pass = 0; pass < passes_w; ++pass) {
            const uint32_t first = pass * IMAX;
            const uint32_t nq = nhome > first ? min(nhome - first, (uint32_t)IMAX) : 0u;
            const uint32_t nq_w = wave_max_of_groups(nq);
            T xi[IMAX][D];
            T gyi[IMAX][NY];
            T ai[IMAX];
            T acc[IMAX][BWD ? D : NY];
            T acc_a[IMAX];
#pragma unroll
            for (int qq = 0; qq < IMAX; ++qq) {
                const bool live = (uint32_t)qq < nq;
                const uint32_t s = hbeg + first + qq;
                if (live) {
                    const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[s];
#pragma unroll
                    for (int k = 0; k < D; ++k) xi[qq][k] = v.v[k];
                } else {
#pragma unroll
                    for (int k = 0; k < D; ++k) xi[qq][k] = Far<T>::home();
                }
#pragma unroll
                for (int k = 0; k < NY; ++k) gyi[qq][k] = (BWD && live) ? gy_s[(size_t)s * NY + k] : T(0);
                ai[qq] = (HAS_A && live) ? a_s[s] : T(0);
#pragma unroll
                for (int k = 0; k < (BWD ? D : NY); ++k) acc[qq][k] = T(0);
                acc_a[qq] = T(0);
            }

            auto body = [&](auto shift_tag) {
                constexpr bool SHIFT = decltype(shift_tag)::value;
                int p = 0;
                for (uint32_t t0 = 0; t0 < Mw; t0 += kGroup) {
                    const uint32_t t = t0 + (uint32_t)l;
                    T xj[D], sh[D], aj = T(0), gyj[NY];
#pragma unroll
                    for (int k = 0; k < NY; ++k) gyj[k] = T(0);
                    if (t < M) {
                        while (t >= s_cum[g][p + 1]) ++p;
                        const uint32_t slot = s_start[g][p] + (t - s_cum[g][p]);
                        const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[slot];
#pragma unroll
                        for (int k = 0; k < D; ++k) xj[k] = v.v[k];
                        if (SHIFT) {
                            const uint32_t code = s_code[g][p];
#pragma unroll
                            for (int k = 0; k < D; ++k) sh[k] = shift_of<T>(code, k, P.L[k]);
                        }
                        if (HAS_A) aj = a_s[slot];
                        if (BWD) {
#pragma unroll
                            for (int k = 0; k < NY; ++k) gyj[k] = gy_s[(size_t)slot * NY + k];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < D; ++k) { xj[k] = Far<T>::cand(); sh[k] = T(0); }
                    }
#pragma unroll
                    for (int qq = 0; qq < IMAX; ++qq) {
                        if ((uint32_t)qq < nq_w) {
                            T dx[D];
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                dx[k] = xj[k] - xi[qq][k];
                                if (SHIFT) dx[k] = dx[k] + sh[k];
                            }
                            T d2 = dx[0] * dx[0];
                            if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
                            if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
                            const bool ok = d2 > T(0) && d2 < r2;
                            if constexpr (BWD) {
                                Op::bwd_masked(q, r, dx, d2, ai[qq], aj, gyi[qq], gyj, ok, acc[qq], &acc_a[qq]);
                            } else {
                                Op::fwd_masked(q, r, dx, d2, ai[qq], aj, ok, acc[qq]);
                            }
                        }
                    }
                }
            };
            if (wave_shift) body(std::true_type{});
            else body(std::false_type{});

            // reduce over the group and write the pass's home particles
#pragma unroll
            for (int qq = 0; qq < IMAX; ++qq) {
                if ((uint32_t)qq < nq_w) {
#pragma unroll
                    for (int k = 0; k < (BWD ? D : NY); ++k) acc[qq][k] = group_sum(acc[qq][k]);
                    if (BWD && HAS_A) acc_a[qq] = group_sum(acc_a[qq]);
                    if ((uint32_t)l == (uint32_t)qq && (uint32_t)qq < nq) {
                        const uint32_t o = perm[hbeg + first + qq];
                        constexpr int W = BWD ? D : NY;
#pragma unroll
                        for (int k = 0; k < W; ++k) out[(size_t)o * W + k] = acc[qq][k];
                        if (BWD && HAS_A && out_a) out_a[o] = acc_a[qq];
                    }
                }
            }
        }
        __syncthreads();  // the piece tables are rewritten by the next round
    }
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------

namespace {

template <typename T>
aboria_status gather(aboria_ctx* ctx, const aboria_cells* c, const void* src, int w, void* dst) {
    const uint64_t total = (uint64_t)c->n * (uint64_t)w;
    if (total == 0) return ABORIA_OK;
    hipLaunchKernelGGL(k_gather_rows<T>, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, ctx->stream,
                       (const T*)src, c->perm, (uint32_t)c->n, w, (T*)dst);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

// Work-mapping variants of the neighbour sums.
struct Variant {
    int kind;    // 0 = cell group, 1 = lane per particle
    int imax;    // home particles per pass (cell group)
    int block;   // threads per workgroup
    int rounds;  // cell-group rounds per workgroup (tile = block/16 * rounds cells)
    const char* name;
};

const Variant kVariants[] = {
    {0, 8, 128, 8, "cell group of 16 lanes, 8 home particles per pass, 64-cell tiles ranked by occupancy"},
    {0, 16, 128, 8, "cell group of 16 lanes, 16 home particles per pass, 64-cell tiles ranked by occupancy"},
    {0, 8, 128, 1, "cell group of 16 lanes, 8 home particles per pass, cells in natural order"},
    {1, 0, 256, 0, "lane per particle, x-row runs, 256-thread workgroups"},
    {1, 0, 128, 0, "lane per particle, x-row runs, 128-thread workgroups"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <typename T, int D, int OP, bool BATCH, bool BWD, int IMAX, int BLOCK, int ROUNDS>
void launch_cells(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* out,
                  T* out_a) {
    constexpr int TILE = BLOCK / kGroup * ROUNDS;
    const uint32_t nwork = (uint32_t)c->ncells;
    const dim3 grid((nwork + TILE - 1) / TILE);
    hipLaunchKernelGGL((k_pair_cells<T, D, OP, BATCH, BWD, IMAX, BLOCK, ROUNDS>), grid, dim3(BLOCK), 0, ctx->stream,
                       (const T*)c->xs, c->off, c->perm, (uint32_t)c->n, nwork,
                       reinterpret_cast<const SysParams<T>*>(c->params_dev), c->cell_base_dev, c->nsys, a_s, gy_s, q,
                       out, out_a);
}

template <typename T, int D, int OP, bool BATCH, bool BWD>
void launch_variant(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* out,
                    T* out_a, int variant) {
    const Variant& v = kVariants[(variant < 0 || variant >= kNumVariants) ? 0 : variant];
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (v.kind == 0) {
        if (v.imax == 16) launch_cells<T, D, OP, BATCH, BWD, 16, 128, 8>(ctx, c, q, a_s, gy_s, out, out_a);
        else if (v.rounds == 1) launch_cells<T, D, OP, BATCH, BWD, 8, 128, 1>(ctx, c, q, a_s, gy_s, out, out_a);
        else launch_cells<T, D, OP, BATCH, BWD, 8, 128, 8>(ctx, c, q, a_s, gy_s, out, out_a);
        return;
    }
    const dim3 grid((n + v.block - 1) / v.block);
    if constexpr (BWD)
        hipLaunchKernelGGL((k_pair_bwd<T, D, OP, BATCH>), grid, dim3(v.block), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, out, out_a);
    else
        hipLaunchKernelGGL((k_pair_fwd<T, D, OP, BATCH>), grid, dim3(v.block), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, out);
}

template <typename T, int D, int OP>
aboria_status launch_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int variant) {
    if (c->n == 0) return ABORIA_OK;
    if (c->nsys == 1) launch_variant<T, D, OP, false, false>(ctx, c, q, a_s, nullptr, y, nullptr, variant);
    else launch_variant<T, D, OP, true, false>(ctx, c, q, a_s, nullptr, y, nullptr, variant);
    ABORIA_HIP(ctx, hipGetLastError());
    return ABORIA_OK;
}

template <typename T, int D, int OP>
aboria_status launch_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                         T* gx, T* ga, int variant) {
    if (c->n == 0) return ABORIA_OK;
    if (c->nsys == 1) launch_variant<T, D, OP, false, true>(ctx, c, q, a_s, gy_s, gx, ga, variant);
    else launch_variant<T, D, OP, true, true>(ctx, c, q, a_s, gy_s, gx, ga, variant);
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

}  // namespace

int32_t variant_count() { return kNumVariants; }

const char* variant_name(int32_t v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : ""; }

aboria_status pair_sum_impl(aboria_ctx* ctx, const aboria_cells* c, int32_t op, const double* params,
                            int32_t nparams, const void* a, int32_t na, void* y, int32_t ny, int32_t variant) {
    aboria_status st = validate(ctx, c, op, params, nparams, a, na, ny);
    if (st != ABORIA_OK) return st;
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
