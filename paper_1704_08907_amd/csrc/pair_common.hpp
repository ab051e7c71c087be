// Shared device code of the neighbour-sum kernels: precision primitives, the
// operator functors (forward summand and adjoint contribution of one ordered
// pair) and the per-particle box-search loop.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"

namespace aboria {

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

    // The radial profile of the vector operators f = g(s) u at one pair, as the
    // two factors of its Jacobian J = g I + (g'/s) u u^T: g across u and
    // gpar = g + s g' along u.  Spring and DEM spring: gpar = -k; eq. (1)
    // force: gpar = -c e^{-s}.  rinv = 1/s.
    __device__ __forceinline__ static void radial_parts(const OpArgs<T>& q, T r, T d2, T rinv, T ai, T aj, T& g,
                                                        T& gpar) {
        if constexpr (OP == ABORIA_OP_SPRING) {
            g = fma_t(q.p0 * r, rinv, -q.p0);
            gpar = -q.p0;
        } else if constexpr (OP == ABORIA_OP_EXP_FORCE) {
            const T ce = q.p0 * exp_neg_t(d2 * rinv);
            g = ce * rinv;
            gpar = -ce;
        } else {
            g = fma_t(q.p0 * (ai + aj), rinv, -q.p0);
            gpar = -q.p0;
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
            // as bwd(); every factor is zeroed on a rejected candidate, whose
            // d2 may be 0 (rinv = inf), before it meets a finite w
            const T rinv = rsqrt_t(d2);
            T w[D];
            T dw = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                w[k] = gyi[k] - gyj[k];
                dw = fma_t(dx[k], w[k], dw);
            }
            T g, gpar;
            radial_parts(q, r, d2, rinv, ai, aj, g, gpar);
            if constexpr (OP == ABORIA_OP_DEM_SPRING) {
                const T ta = -q.p0 * dw * rinv;
                ga[0] += ok ? ta : T(0);
            }
            if constexpr (D == 1) {
                gx[0] = fma_t(ok ? gpar : T(0), w[0], gx[0]);
            } else {
                const T c = ok ? dw * (rinv * rinv) : T(0);
                g = ok ? g : T(0);
                const T pc = gpar * c;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const T wperp = fma_t(-c, dx[k], w[k]);
                    gx[k] = fma_t(g, wperp, fma_t(pc, dx[k], gx[k]));
                }
            }
        }
    }

    // gx += J1(i,j)^T gy_i + J2(j,i)^T gy_j ; ga += d/da_i of the same.
    // For f = g(s) u the pair adds J w with w = gy_i - gy_j.  Splitting w into
    // its parts along and across u, w_par = ((dx.w)/s^2) dx and w_perp = w -
    // w_par, gives J w = g w_perp + gpar w_par: no two O(g) products cancel
    // (written as g w + (g'/s)(u.w) u, the spring's two terms are each about
    // k r/s along u and leave -k, so float32 rounding of them would grow as
    // r/s).  For the soft sphere: gx += 1/2 (gy_i + gy_j) phi'(s) u/s with
    // phi'(s) = -(2/r)(1 - s/r).
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
            T w[D];
            T dw = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                w[k] = gyi[k] - gyj[k];
                dw = fma_t(dx[k], w[k], dw);
            }
            T g, gpar;
            radial_parts(q, r, d2, rinv, ai, aj, g, gpar);
            if constexpr (OP == ABORIA_OP_DEM_SPRING) {
                // d/da_i: k (gy_i - gy_j).u / s = -k (w.dx) / s
                ga[0] = fma_t(-q.p0 * dw, rinv, ga[0]);
            }
            if constexpr (D == 1) {
                // one dimension: w is all along u, exactly (no rounded projection
                // whose residue g, large at small s, would multiply)
                gx[0] = fma_t(gpar, w[0], gx[0]);
            } else {
                const T c = dw * (rinv * rinv);  // w_par = c dx
                const T pc = gpar * c;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const T wperp = fma_t(-c, dx[k], w[k]);
                    gx[k] = fma_t(g, wperp, fma_t(pc, dx[k], gx[k]));
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// the per-particle box search
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_system_slot(const uint32_t* __restrict__ first, int nsys, uint32_t i) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// System of row i for a workgroup whose rows start at block_first and are
// contiguous: one binary search per workgroup, then a short forward step per
// lane.  Every thread of the workgroup must call it (it synchronises).
template <bool BATCH>
__device__ __forceinline__ int system_of_row(const uint32_t* __restrict__ sys_part, int nsys, uint32_t block_first,
                                             uint32_t i) {
    if (!BATCH) return 0;
    __shared__ int s_first;
    if (threadIdx.x == 0) s_first = find_system_slot(sys_part, nsys, block_first);
    __syncthreads();
    int b = s_first;
    while (b + 1 < nsys && sys_part[b + 1] <= i) ++b;
    return b;
}

// Rows of the upstream gradient in cell order: 3-wide rows are padded to 4 so
// that one 16-byte (float) or 32-byte (double) load fetches a row.
template <int NY>
struct GyPitch {
    static constexpr int value = NY == 3 ? 4 : NY;
};

// Element j of an array of N-element rows.  OFF32: the byte offset j * row size
// fits in 32 bits (the launcher checks it), so the load takes a scalar base and
// a 32-bit lane offset and its address costs one full-rate add.
template <typename T, int N, bool OFF32>
__device__ __forceinline__ VecN<T, N> load_row(const T* __restrict__ base, uint32_t j) {
    if constexpr (OFF32)
        return *reinterpret_cast<const VecN<T, N>*>(reinterpret_cast<const char*>(base) +
                                                   (uint32_t)(j * (uint32_t)sizeof(VecN<T, N>)));
    else
        return reinterpret_cast<const VecN<T, N>*>(base)[j];
}

// Row j + k with k a small constant: with 32-bit offsets the address is the
// row-j address plus k rows, which the load takes as an immediate offset
// (row j + k lies below the same 32-bit bound, so the two addresses agree).
template <typename T, int N, bool OFF32>
__device__ __forceinline__ VecN<T, N> load_row_at(const T* __restrict__ base, uint32_t j, uint32_t k) {
    if constexpr (OFF32)
        return *reinterpret_cast<const VecN<T, N>*>(reinterpret_cast<const char*>(base) +
                                                   (size_t)(uint32_t)(j * (uint32_t)sizeof(VecN<T, N>)) +
                                                   (size_t)k * sizeof(VecN<T, N>));
    else
        return reinterpret_cast<const VecN<T, N>*>(base)[j + k];
}

// Marks the first N elements of a loaded row as used at this point (an empty
// asm statement, no instruction).  A load whose only other use sits inside a
// branch would otherwise be sunk into that branch and issued only there; held
// here, it is issued where it is written and overlaps the work before it.
template <int N, typename T>
__device__ __forceinline__ void keep_issued(const T* v) {
#pragma unroll
    for (int k = 0; k < N; ++k) asm volatile("" ::"v"(v[k]));
}

// True when every per-particle row the sums load (at most 4 elements of T)
// lies below a 32-bit byte offset, so the kernels may use 32-bit offsets.
template <typename T>
inline bool off32_rows(uint64_t n) {
    return n * 4 * sizeof(T) <= 0xFFFFFFFFull;
}

template <typename T, int NY, bool OFF32 = false>
__device__ __forceinline__ void load_gy(const T* __restrict__ gy_s, uint32_t j, T* out) {
    const VecN<T, GyPitch<NY>::value> v = load_row<T, GyPitch<NY>::value, OFF32>(gy_s, j);
#pragma unroll
    for (int k = 0; k < NY; ++k) out[k] = v.v[k];
}

template <typename T, int D>
__device__ __forceinline__ void load_point(const T* __restrict__ xs, uint32_t s, T* xi) {
    constexpr int PITCH = Pitch<D>::value;
    const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[s];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = v.v[k];
}

// Pair test of one candidate: dx_k = fl(fl(x_jk - x_ik) + s_k) (the shift add
// only when SHIFT), d2 by the fixed fma chain; returns 0 < d2 < r2.
template <typename T, int D, bool SHIFT>
__device__ __forceinline__ bool pair_test(const T* xj, const T* xi, const T* sh, T r2, T* dx, T* d2out) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
        dx[k] = xj[k] - xi[k];
        if (SHIFT) dx[k] = dx[k] + sh[k];
    }
    T d2 = dx[0] * dx[0];
    if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
    if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
    *d2out = d2;
    return d2 > T(0) && d2 < r2;
}

// LDS windows of the lane-per-particle kernels.  The lanes of a wave are 64
// consecutive particles in cell order, so for one stencil row their main runs
// (the cells up to m away along x) overlap almost entirely, and in slot space
// their union is one range: from the first lane's run start to the last lane's
// run end (also when the wave spans the end of one x-row and the start of the
// next, which are adjacent slots).  When every lane's run lies in that range
// and it has at most kWindow slots, the wave copies it once into a window of
// its own with coalesced loads and the lanes read their candidates from LDS.
constexpr int kBlockWaves = 4;  // waves of a 256-thread workgroup
constexpr int kWindow = 128;    // slots of a wave's LDS window

// Bytes of one window: kWindow position rows and, with G > 0, as many rows of G
// elements.
template <typename T, int D, int G>
struct WindowBytes {
    static constexpr uint32_t value =
        (uint32_t)kWindow *
        (uint32_t)(sizeof(VecN<T, Pitch<D>::value>) + (G > 0 ? sizeof(VecN<T, (G > 0 ? G : 1)>) : 0));
};

// Copies slots [lo, lo + cnt) of xs (and, with G > 0, of ys, G elements a row,
// after the kWindow position rows) into the wave's window wb; rank and nact
// number the wave's running lanes.  1 <= cnt <= kWindow.
template <typename T, int D, int G>
__device__ __forceinline__ void stage_window(const T* __restrict__ xs, const T* __restrict__ ys, char* wb, uint32_t lo,
                                             uint32_t cnt, uint32_t rank, uint32_t nact) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr uint32_t RB = (uint32_t)sizeof(VecN<T, PITCH>);
    // two slots per lane first, both loads in flight together (a full wave
    // covers the window with them), then any rest
    using Row = VecN<T, PITCH>;
    const char* const src = reinterpret_cast<const char*>(xs) + (size_t)lo * RB;
    const uint32_t t1 = rank + nact;
    const Row ra = *reinterpret_cast<const Row*>(src + (size_t)min(rank, cnt - 1u) * RB);
    const Row rb = *reinterpret_cast<const Row*>(src + (size_t)min(t1, cnt - 1u) * RB);
    keep_issued<PITCH>(ra.v);
    keep_issued<PITCH>(rb.v);
    if (rank < cnt) *reinterpret_cast<Row*>(wb + rank * RB) = ra;
    if (t1 < cnt) *reinterpret_cast<Row*>(wb + t1 * RB) = rb;
    for (uint32_t t = t1 + nact; t < cnt; t += nact)
        *reinterpret_cast<Row*>(wb + t * RB) = *reinterpret_cast<const Row*>(src + (size_t)t * RB);
    if constexpr (G > 0) {
        using RowG = VecN<T, (G > 0 ? G : 1)>;
        constexpr uint32_t RG = (uint32_t)sizeof(RowG);
        const char* const sg = reinterpret_cast<const char*>(ys) + (size_t)lo * RG;
        char* const wg = wb + (uint32_t)kWindow * RB;
        const RowG ga = *reinterpret_cast<const RowG*>(sg + (size_t)min(rank, cnt - 1u) * RG);
        const RowG gb = *reinterpret_cast<const RowG*>(sg + (size_t)min(t1, cnt - 1u) * RG);
        keep_issued<G>(ga.v);
        keep_issued<G>(gb.v);
        if (rank < cnt) *reinterpret_cast<RowG*>(wg + rank * RG) = ga;
        if (t1 < cnt) *reinterpret_cast<RowG*>(wg + t1 * RG) = gb;
        for (uint32_t t = t1 + nact; t < cnt; t += nact)
            *reinterpret_cast<RowG*>(wg + t * RG) = *reinterpret_cast<const RowG*>(sg + (size_t)t * RG);
    }
    // the wave's own LDS operations complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The window of a staged row as the scans read it: slot j's position row at
// wb + (j - lo) * RB, its aux row after the kWindow position rows.
struct WinRef {
    const char* wb;
    uint32_t lo;
};

// One contiguous slot range [j0, j1) of candidates with one image shift:
// visit(j, dx, d2, shifted) for the accepted ones, shifted = the lane's shift
// is nonzero in some dimension.  Two candidates are loaded per iteration so
// their loads overlap.  With NAUX > 0 the candidates' rows of aux (NAUX
// elements, padded as gradient rows) are loaded with their positions and
// passed as a fifth argument, so an accepted pair never waits for them.
template <typename T, int D, bool SHIFT, bool OFF32, int NAUX = 0, bool WIN = false, typename Visit>
__device__ __forceinline__ void scan_range(const T* __restrict__ xs, uint32_t j0, uint32_t j1, const T* xi,
                                           const T* sh, T r2, bool shifted, Visit& visit,
                                           const T* __restrict__ aux = nullptr, WinRef w = WinRef{nullptr, 0u}) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr int AP = NAUX > 0 ? GyPitch<NAUX>::value : 1;
    constexpr uint32_t RB = (uint32_t)sizeof(VecN<T, PITCH>), RA = (uint32_t)sizeof(VecN<T, AP>);
    // slot j's rows: from HBM, or with WIN from the window (j inside it)
    auto ldx = [&](uint32_t jj, uint32_t k) {
        if constexpr (WIN) return *reinterpret_cast<const VecN<T, PITCH>*>(w.wb + (jj - w.lo + k) * RB);
        else return load_row_at<T, PITCH, OFF32>(xs, jj, k);
    };
    auto lda = [&](uint32_t jj, uint32_t k) {
        if constexpr (WIN)
            return *reinterpret_cast<const VecN<T, AP>*>(w.wb + (uint32_t)kWindow * RB + (jj - w.lo + k) * RA);
        else return load_row_at<T, AP, OFF32>(aux, jj, k);
    };
    auto call = [&](uint32_t jj, const T* dx, T d2, const VecN<T, AP>& av) {
        if constexpr (NAUX > 0) visit(jj, dx, d2, shifted, av.v);
        else visit(jj, dx, d2, shifted);
    };
    uint32_t j = j0;
    for (; j + 1 < j1; j += 2) {
        const VecN<T, PITCH> a = ldx(j, 0u);
        const VecN<T, PITCH> b = ldx(j, 1u);
        VecN<T, AP> aa{}, ab{};
        if constexpr (NAUX > 0) {
            aa = lda(j, 0u);
            ab = lda(j, 1u);
        }
        T dx[D], d2;
        if (pair_test<T, D, SHIFT>(a.v, xi, sh, r2, dx, &d2)) call(j, dx, d2, aa);
        if (pair_test<T, D, SHIFT>(b.v, xi, sh, r2, dx, &d2)) call(j + 1, dx, d2, ab);
    }
    if (j < j1) {
        const VecN<T, PITCH> a = ldx(j, 0u);
        VecN<T, AP> aa{};
        if constexpr (NAUX > 0) aa = lda(j, 0u);
        T dx[D], d2;
        if (pair_test<T, D, SHIFT>(a.v, xi, sh, r2, dx, &d2)) call(j, dx, d2, aa);
    }
}

// Operators whose adjoint summand (a d-vector update with a reciprocal square
// root and a dozen multiply-adds) costs several pair tests: their adjoint runs
// the deferred scan.  The soft sphere's scalar summand and the count do not.
template <int OP>
constexpr bool kDeferAdjoint = OP == ABORIA_OP_SPRING || OP == ABORIA_OP_EXP_FORCE || OP == ABORIA_OP_DEM_SPRING;

// scan_range in two passes per chunk of up to 32 candidates, for summands that
// cost much more than the pair test (the adjoint): the first pass tests every
// candidate and keeps a bit per accepted one; the second pops the bits in
// increasing order, reloads that candidate's position and aux row (the
// neighbour's gradient row), recomputes its dx and d2 exactly as the test did
// and calls visit(j, dx, d2, shifted, aux_j).  In SIMD the summand then runs
// as many times per chunk as the busiest lane has accepted pairs, instead of
// once per candidate that any lane of the wave accepts.  The pairs and their
// order are those of scan_range, so the sums are bit for bit the same.
template <typename T, int D, bool SHIFT, bool OFF32, int NAUX, bool WIN = false, typename Visit>
__device__ __forceinline__ void scan_range_deferred(const T* __restrict__ xs, const T* __restrict__ aux,
                                                    uint32_t j0, uint32_t j1, const T* xi, const T* sh, T r2,
                                                    bool shifted, Visit& visit, WinRef w = WinRef{nullptr, 0u}) {
    constexpr int PITCH = Pitch<D>::value;
    constexpr int AP = GyPitch<NAUX>::value;
    constexpr uint32_t RB = (uint32_t)sizeof(VecN<T, PITCH>), RA = (uint32_t)sizeof(VecN<T, AP>);
    auto ldx = [&](uint32_t jj, uint32_t k) {
        if constexpr (WIN) return *reinterpret_cast<const VecN<T, PITCH>*>(w.wb + (jj - w.lo + k) * RB);
        else return load_row_at<T, PITCH, OFF32>(xs, jj, k);
    };
    for (uint32_t c0 = j0; c0 < j1; c0 += 32u) {
        const uint32_t c1 = min(c0 + 32u, j1);
        // each test's bit is shifted in from the bottom (the first candidate ends
        // highest), then one bit reversal puts candidate c0 + k at bit k
        uint32_t mask = 0u;
        uint32_t j = c0;
        for (; j + 1 < c1; j += 2) {
            const VecN<T, PITCH> a = ldx(j, 0u);
            const VecN<T, PITCH> b = ldx(j, 1u);
            T dx[D], d2;
            mask = (mask << 1) | (pair_test<T, D, SHIFT>(a.v, xi, sh, r2, dx, &d2) ? 1u : 0u);
            mask = (mask << 1) | (pair_test<T, D, SHIFT>(b.v, xi, sh, r2, dx, &d2) ? 1u : 0u);
        }
        if (j < c1) {
            const VecN<T, PITCH> a = ldx(j, 0u);
            T dx[D], d2;
            mask = (mask << 1) | (pair_test<T, D, SHIFT>(a.v, xi, sh, r2, dx, &d2) ? 1u : 0u);
        }
        mask = __builtin_bitreverse32(mask) >> (32u - (c1 - c0));
        // the chunk's bit k is slot c0 + k; with WIN its window rows are at fixed
        // offsets from those of bit 0, formed once per chunk
        const char* const pxw = WIN ? w.wb + (c0 - w.lo) * RB : nullptr;
        const char* const paw = WIN ? w.wb + (uint32_t)kWindow * RB + (c0 - w.lo) * RA : nullptr;
        auto ldxk = [&](uint32_t k) {
            if constexpr (WIN) return *reinterpret_cast<const VecN<T, PITCH>*>(pxw + k * RB);
            else return load_row<T, PITCH, OFF32>(xs, c0 + k);
        };
        auto ldak = [&](uint32_t k) {
            if constexpr (WIN) return *reinterpret_cast<const VecN<T, AP>*>(paw + k * RA);
            else return load_row<T, AP, OFF32>(aux, c0 + k);
        };
        // two accepted pairs per iteration, so their four loads overlap
        while (mask != 0u) {
            const uint32_t ka = (uint32_t)__builtin_ctz(mask);
            mask &= mask - 1u;
            const bool vb = mask != 0u;
            const uint32_t kb = vb ? (uint32_t)__builtin_ctz(mask) : ka;
            mask &= mask - 1u;
            const uint32_t ja = c0 + ka, jb = c0 + kb;
            const VecN<T, PITCH> a = ldxk(ka);
            const VecN<T, AP> ava = ldak(ka);
            const VecN<T, PITCH> b = ldxk(kb);
            const VecN<T, AP> avb = ldak(kb);
            T dx[D], d2;
            (void)pair_test<T, D, SHIFT>(a.v, xi, sh, r2, dx, &d2);
            visit(ja, dx, d2, shifted, ava.v);
            keep_issued<D>(b.v);
            keep_issued<NAUX>(avb.v);
            if (vb) {
                (void)pair_test<T, D, SHIFT>(b.v, xi, sh, r2, dx, &d2);
                visit(jb, dx, d2, shifted, avb.v);
            }
        }
    }
}

// Cell coordinate of xi in dimension k by the arithmetic of the cell assignment
// (so it is the cell the build put the particle in), and the position inside
// that cell in cell units, fr = q - c (exact: c = floor(q)).
template <typename T>
__device__ __forceinline__ int32_t cell_coord(const SysParams<T>& P, int k, T xk, T* fr) {
    const T t = xk - P.lo[k];
    const T q = t * P.inv_w[k];
    const T f = floor(q);
    const int32_t c = !(f >= T(0)) ? 0 : (f > T(P.n[k] - 1) ? P.n[k] - 1 : (int32_t)f);
    *fr = q - T(c);
    return c;
}

// Cell v = c + o of a dimension of n cells, wrapped once when periodic (the
// wrap becomes the image shift); false when the offset leaves a non-periodic
// grid or would need a second wrap (an image one more period away lies at
// least L >= 2r further, so it holds no pair).
template <typename T>
__device__ __forceinline__ bool wrap_cell(int32_t v, int32_t n, int32_t periodic, T L, int32_t* out, T* shift) {
    T s = T(0);
    if (v < 0) {
        if (!periodic) return false;
        v += n;
        s = -L;
    } else if (v >= n) {
        if (!periodic) return false;
        v -= n;
        s = L;
    }
    if (v < 0 || v >= n) return false;
    *out = v;
    *shift = s;
    return true;
}

// Box search of the point xi (a particle of the cell list, Section 2.2.2): its
// cell and every cell up to m_k = P.reach[k] cells away in dimension k (m = 1:
// the adjacent cells), walked as (2 m_y + 1)(2 m_z + 1) x-rows in (z, y)
// order.  On a grid at least 2 m_x + 1 cells wide a row is one contiguous run
// of up to 2 m_x + 1 cells clipped to the grid, then, when periodic, the
// wrapped remainder with its image shift (only one side can wrap); on a
// narrower grid each offset is its own piece, in offset order.  A piece whose shift is zero on every active
// lane of the wave runs the loop without the shift additions (adding zero is
// exact, so both loops give the canonical dx).  flat_loop visits the accepted
// neighbours in this same order.
template <typename T, int D, bool OFF32, int NAUX, typename Visit, bool STAGE = false>
__device__ __forceinline__ void neighbour_loop_aux(const SysParams<T>& P, const T* __restrict__ xs,
                                                   const T* __restrict__ aux, const uint32_t* __restrict__ off,
                                                   uint32_t n, const T* xi, Visit&& visit) {
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T fr;
        c[k] = cell_coord(P, k, xi[k], &fr);
    }
    const int32_t M = P.reach[0];
    const int32_t nx = P.n[0];
    const bool wide = nx >= 2 * M + 1;
    const int32_t a0 = max(c[0] - M, 0), b0 = min(c[0] + M, nx - 1);
    int32_t a1 = 0, b1 = -1;
    T s1 = T(0);
    if (P.periodic[0]) {
        if (c[0] - M < 0) { a1 = c[0] - M + nx; b1 = nx - 1; s1 = -P.L[0]; }
        else if (c[0] + M >= nx) { a1 = 0; b1 = c[0] + M - nx; s1 = P.L[0]; }
    }
    const T r2 = P.r2;
    // the candidates [j0, j1), from HBM or (WIN) from the window w
    auto piece_j = [&](auto win_tag, uint32_t j0, uint32_t j1, const T* sh, WinRef w) {
        constexpr bool WIN = decltype(win_tag)::value;
        bool lane_shift = false;
#pragma unroll
        for (int k = 0; k < D; ++k) lane_shift |= sh[k] != T(0);
        if constexpr (NAUX > 0) {
            if (__ballot(lane_shift) != 0ull)
                scan_range_deferred<T, D, true, OFF32, NAUX, WIN>(xs, aux, j0, j1, xi, sh, r2, lane_shift, visit, w);
            else
                scan_range_deferred<T, D, false, OFF32, NAUX, WIN>(xs, aux, j0, j1, xi, sh, r2, false, visit, w);
        } else {
            if (__ballot(lane_shift) != 0ull)
                scan_range<T, D, true, OFF32, 0, WIN>(xs, j0, j1, xi, sh, r2, lane_shift, visit, nullptr, w);
            else
                scan_range<T, D, false, OFF32, 0, WIN>(xs, j0, j1, xi, sh, r2, false, visit, nullptr, w);
        }
    };
    auto piece = [&](uint32_t ca, uint32_t cb, const T* sh) {
        piece_j(std::integral_constant<bool, false>(), off[ca], min(off[cb + 1], n), sh, WinRef{nullptr, 0u});
    };
    if constexpr (STAGE && OFF32) {
        // Every grid of the wave at least 2 m + 1 cells wide, one reach in y and z
        // for all its lanes, workgroups of at most kBlockWaves waves: each row's
        // main runs are read through the wave's LDS window when they fit in it.
        const int32_t zl = D >= 3 ? P.reach[2] : 0, yl = D >= 2 ? P.reach[1] : 0;
        const int32_t zr = __builtin_amdgcn_readfirstlane(zl), yr = __builtin_amdgcn_readfirstlane(yl);
        if (__ballot(!wide || zl != zr || yl != yr) == 0ull && blockDim.x <= 64u * kBlockWaves) {
            constexpr int G = NAUX > 0 ? GyPitch<NAUX>::value : 0;
            __shared__ VecN<T, 4> win[kBlockWaves][WindowBytes<T, D, G>::value / sizeof(VecN<T, 4>)];
            char* const wb = reinterpret_cast<char*>(&win[threadIdx.x >> 6][0]);
            const uint64_t act = __ballot(true);
            const uint32_t nact = (uint32_t)__popcll(act);
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
#pragma unroll 1
            for (int32_t dz = -zr; dz <= zr; ++dz) {
#pragma unroll 1
                for (int32_t dy = -yr; dy <= yr; ++dy) {
                    int32_t cz = 0, cy = 0;
                    T sz = T(0), sy = T(0);
                    const bool ez = D < 3 || wrap_cell(c[2] + dz, P.n[2], P.periodic[2], P.L[2], &cz, &sz);
                    const bool ey = D < 2 || wrap_cell(c[1] + dy, P.n[1], P.periodic[1], P.L[1], &cy, &sy);
                    const bool ex = ez && ey;
                    uint32_t rowbase = 0, jm0 = 0, jm1 = 0;
                    if (ex) {
                        rowbase = P.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)P.n[1] * (uint32_t)cz);
                        jm0 = off[rowbase + a0];
                        jm1 = max(min(off[rowbase + b0 + 1], n), jm0);
                    }
                    const bool has = jm1 > jm0;
                    const uint64_t hb = __ballot(has);
                    bool staged = false;
                    uint32_t lo = 0;
                    if (hb != 0ull) {
                        lo = __builtin_amdgcn_readlane(jm0, __builtin_ctzll(hb));
                        const uint32_t hi = __builtin_amdgcn_readlane(jm1, 63 - __builtin_clzll(hb));
                        const bool inside = !has || (jm0 >= lo && jm1 <= hi);
                        // all inside: the first lane's run gives lo < hi
                        staged = __ballot(!inside) == 0ull && hi - lo <= (uint32_t)kWindow;
                        if (staged) stage_window<T, D, G>(xs, aux, wb, lo, hi - lo, rank, nact);
                    }
                    if (ex) {
                        T sh[3] = {T(0), sy, sz};
                        if (staged) piece_j(std::integral_constant<bool, true>(), jm0, jm1, sh, WinRef{wb, lo});
                        else piece_j(std::integral_constant<bool, false>(), jm0, jm1, sh, WinRef{nullptr, 0u});
                        if (b1 >= a1) {
                            sh[0] = s1;
                            piece(rowbase + a1, rowbase + b1, sh);
                        }
                    }
                }
            }
            return;
        }
    }
    const int32_t zr = D >= 3 ? P.reach[2] : 0, yr = D >= 2 ? P.reach[1] : 0;
    for (int32_t dz = -zr; dz <= zr; ++dz) {
        int32_t cz = 0;
        T sz = T(0);
        if (D >= 3 && !wrap_cell(c[2] + dz, P.n[2], P.periodic[2], P.L[2], &cz, &sz)) continue;
        for (int32_t dy = -yr; dy <= yr; ++dy) {
            int32_t cy = 0;
            T sy = T(0);
            if (D >= 2 && !wrap_cell(c[1] + dy, P.n[1], P.periodic[1], P.L[1], &cy, &sy)) continue;
            const uint32_t rowbase = P.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)P.n[1] * (uint32_t)cz);
            T sh[3] = {T(0), sy, sz};
            if (wide) {
                piece(rowbase + a0, rowbase + b0, sh);
                if (b1 >= a1) {
                    sh[0] = s1;
                    piece(rowbase + a1, rowbase + b1, sh);
                }
            } else {
                for (int32_t o = -M; o <= M; ++o) {
                    int32_t cx;
                    if (!wrap_cell(c[0] + o, nx, P.periodic[0], P.L[0], &cx, &sh[0])) continue;
                    piece(rowbase + cx, rowbase + cx, sh);
                }
            }
        }
    }
}

// neighbour_loop_aux with each row's main runs read through the wave's LDS
// window where they fit (same pairs, same order, same sums).
template <typename T, int D, bool OFF32, int NAUX, typename Visit>
__device__ __forceinline__ void neighbour_loop_aux_staged(const SysParams<T>& P, const T* __restrict__ xs,
                                                          const T* __restrict__ aux,
                                                          const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                                          Visit&& visit) {
    neighbour_loop_aux<T, D, OFF32, NAUX, Visit, true>(P, xs, aux, off, n, xi, visit);
}

// The box search without prefetched per-candidate rows: visit(j, dx, d2, shifted).
template <typename T, int D, bool OFF32 = false, typename Visit>
__device__ __forceinline__ void neighbour_loop(const SysParams<T>& P, const T* __restrict__ xs,
                                               const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                               Visit&& visit) {
    neighbour_loop_aux<T, D, OFF32, 0>(P, xs, nullptr, off, n, xi, visit);
}

// neighbour_loop with each row's main runs read through the wave's LDS window.
template <typename T, int D, bool OFF32 = false, typename Visit>
__device__ __forceinline__ void neighbour_loop_staged(const SysParams<T>& P, const T* __restrict__ xs,
                                                      const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                                      Visit&& visit) {
    neighbour_loop_aux<T, D, OFF32, 0, Visit, true>(P, xs, nullptr, off, n, xi, visit);
}

// ---------------------------------------------------------------------------
// flattened box search with per-lane pruning
// ---------------------------------------------------------------------------

// Per-lane slot ranges of the flattened search, in LDS: entry k of lane t at
// [k][t] (consecutive lanes in consecutive banks).  code packs the image shift
// of the range, two bits per dimension (0: none, 1: -L, 2: +L).
template <int CAP, int BLOCK>
struct FlatRanges {
    uint2 range[CAP][BLOCK];
    uint8_t code[CAP][BLOCK];
};

template <typename T, int D>
__device__ __forceinline__ void decode_shift(const SysParams<T>& P, uint32_t code, T* sh) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t b = (code >> (2 * k)) & 3u;
        sh[k] = b == 1u ? -P.L[k] : (b == 2u ? P.L[k] : T(0));
    }
}

// Lower bound of the length between the point and any point of the cell `o`
// cells away in one dimension, squared.  g = o - fr (o > 0) or fr - o - 1
// (o < 0) is the gap in cell units; the slack and the rounded-down cell width
// cover the rounding of the cell assignment of both points and of the image
// shift, so a cell this bound prunes can hold no pair the predicate accepts.
template <typename T>
__device__ __forceinline__ T gap2(const SysParams<T>& P, int k, int32_t o, T fr) {
    const T g = o > 0 ? T(o) - fr : (o < 0 ? fr - T(o) - T(1) : T(0));
    const T gl = max(g - P.slack[k], T(0)) * P.w_lo[k];
    return gl * gl;
}

// The box search of neighbour_loop, flattened per lane.  Each lane first lists
// the slot ranges of its (row, piece) sequence in LDS, dropping every row and
// every cell at the ends of a row that the pruning bound (gap2, threshold
// P.prune_r2) shows to be out of reach, and empty ranges; then it walks the
// listed ranges as one sequence, one candidate per iteration, so the wave
// runs as many iterations as its busiest lane has candidates instead of the
// sum over rows of the longest row.  A lane lists at most CAP ranges per
// round; rounds repeat while a lane of the wave has rows left.  The accepted
// neighbours and their order are those of neighbour_loop (pruning removes only
// candidates the predicate rejects).  A lane uses its own LDS column only, so
// no barrier is needed and lanes past the end may simply not call it.  t_self
// is the lane's own slot (< n), the target of loads issued past its last
// candidate.
template <typename T, int D, int CAP, int BLOCK, bool OFF32, typename Visit>
__device__ __forceinline__ void flat_loop(const SysParams<T>& P, const T* __restrict__ xs,
                                          const uint32_t* __restrict__ off, uint32_t n, const T* xi,
                                          uint32_t t_self, FlatRanges<CAP, BLOCK>& fr_lds, Visit&& visit) {
    constexpr int PITCH = Pitch<D>::value;
    const uint32_t t = threadIdx.x;
    int32_t c[3] = {0, 0, 0};
    T fr[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) c[k] = cell_coord(P, k, xi[k], &fr[k]);
    const int32_t M = P.reach[0];
    const int32_t nx = P.n[0];
    const bool wide = nx >= 2 * M + 1;
    const T pr2 = P.prune_r2;
    // squared x gaps of the offsets -t and +t, t = 1..3 (+inf past the reach)
    T gxn[kMaxReach], gxp[kMaxReach];
#pragma unroll
    for (int q = 0; q < kMaxReach; ++q) {
        const bool in = q < M;
        gxn[q] = in ? gap2(P, 0, -(q + 1), fr[0]) : T(INFINITY);
        gxp[q] = in ? gap2(P, 0, q + 1, fr[0]) : T(INFINITY);
    }
    // ranges a row can add: one run and one wrapped run, or one per offset
    const int pmax = wide ? (P.periodic[0] ? 2 : 1) : 2 * M + 1;
    const int32_t zr = D >= 3 ? P.reach[2] : 0, yr = D >= 2 ? P.reach[1] : 0;
    int32_t dy = -yr, dz = -zr;
    bool rows_left = true;
    const T r2 = P.r2;
    while (__ballot(rows_left) != 0ull) {
        // ---- list up to CAP ranges ----
        int kd = 0;
        bool any_shift = false;
        auto put = [&](uint32_t ca, uint32_t cb, uint32_t code) {
            const uint32_t j0 = off[ca];
            const uint32_t j1 = min(off[cb + 1], n);
            if (j1 > j0) {
                fr_lds.range[kd][t] = make_uint2(j0, j1);
                fr_lds.code[kd][t] = (uint8_t)code;
                any_shift |= code != 0u;
                ++kd;
            }
        };
        while (rows_left && kd + pmax <= CAP) {
            const int32_t ry = dy, rz = dz;
            if (++dy > yr) {
                dy = -yr;
                if (++dz > zr) rows_left = false;
            }
            const T g2 = (D >= 2 ? gap2(P, 1, ry, fr[1]) : T(0)) + (D >= 3 ? gap2(P, 2, rz, fr[2]) : T(0));
            if (!(g2 < pr2)) continue;
            int32_t cz = 0, cy = 0;
            T sz = T(0), sy = T(0);
            if (D >= 3 && !wrap_cell(c[2] + rz, P.n[2], P.periodic[2], P.L[2], &cz, &sz)) continue;
            if (D >= 2 && !wrap_cell(c[1] + ry, P.n[1], P.periodic[1], P.L[1], &cy, &sy)) continue;
            const uint32_t yz = (sy < T(0) ? 1u : (sy > T(0) ? 2u : 0u)) << 2 |
                                (sz < T(0) ? 1u : (sz > T(0) ? 2u : 0u)) << 4;
            // offsets lo..hi of the row that the bound keeps (the bound grows with |o|)
            int32_t lo = 0, hi = 0;
#pragma unroll
            for (int q = 0; q < kMaxReach; ++q) {
                lo -= (gxn[q] + g2 < pr2) ? 1 : 0;
                hi += (gxp[q] + g2 < pr2) ? 1 : 0;
            }
            const uint32_t rowbase = P.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)P.n[1] * (uint32_t)cz);
            if (wide) {
                put(rowbase + max(c[0] + lo, 0), rowbase + min(c[0] + hi, nx - 1), yz);
                if (P.periodic[0]) {
                    if (c[0] + lo < 0) put(rowbase + (c[0] + lo + nx), rowbase + (nx - 1), yz | 1u);
                    else if (c[0] + hi >= nx) put(rowbase, rowbase + (c[0] + hi - nx), yz | 2u);
                }
            } else {
                for (int32_t o = lo; o <= hi; ++o) {
                    int32_t cx;
                    T sx;
                    if (!wrap_cell(c[0] + o, nx, P.periodic[0], P.L[0], &cx, &sx)) continue;
                    put(rowbase + cx, rowbase + cx, yz | (sx < T(0) ? 1u : (sx > T(0) ? 2u : 0u)));
                }
            }
        }
        // ---- walk the listed ranges as one sequence ----
        // Two candidate registers, A and B, alternate: one is tested while the
        // other's load is in flight.  Every step reads the range the cursor
        // takes next from LDS, so a range change uses a value read one step
        // earlier, and issues its load unconditionally (a lane past its last
        // candidate reloads its own row); the loop leaves only when no lane of
        // the wave has candidates left.
        auto walk = [&](auto shift_tag) {
            constexpr bool SHIFT = decltype(shift_tag)::value;
            uint32_t kr = 0u;  // index of the next range to take
            uint2 ndp = fr_lds.range[0][t];
            uint32_t ndc = SHIFT ? (uint32_t)fr_lds.code[0][t] : 0u;
            uint32_t j = 0u, e = 0u;
            bool alive = true;
            T cs[3] = {T(0), T(0), T(0)};  // shift of the cursor's range
            // the slot of the lane's next candidate (its own slot once it has none)
            auto step = [&]() -> uint32_t {
                ++j;
                if (j >= e) {
                    if (kr < (uint32_t)kd) {
                        j = ndp.x;
                        e = ndp.y;
                        if (SHIFT) decode_shift<T, D>(P, ndc, cs);
                        ++kr;
                    } else {
                        alive = false;
                    }
                }
                const uint32_t kn = min(kr, (uint32_t)(CAP - 1));
                ndp = fr_lds.range[kn][t];
                if (SHIFT) ndc = fr_lds.code[kn][t];
                return alive ? j : t_self;
            };
            // evaluated on every lane (an idle lane tests its own row, which the
            // predicate rejects) so that the wait for the row is never skipped
            auto test = [&](const VecN<T, PITCH>& xj, uint32_t jj, const T* sh, bool valid) {
                T dx[D], d2;
                const bool acc = pair_test<T, D, SHIFT>(xj.v, xi, sh, r2, dx, &d2);
                if (acc & valid) {
                    bool shifted = false;
                    if (SHIFT) {
#pragma unroll
                        for (int k = 0; k < D; ++k) shifted |= sh[k] != T(0);
                    }
                    visit(jj, dx, d2, shifted);
                }
            };
            T sa[3], sb[3];
            uint32_t ja = step();
            bool va = alive;
#pragma unroll
            for (int k = 0; k < 3; ++k) sa[k] = cs[k];
            VecN<T, PITCH> A = load_row<T, PITCH, OFF32>(xs, ja);
            for (;;) {
                const uint32_t jb = step();
                const bool vb = alive;
#pragma unroll
                for (int k = 0; k < 3; ++k) sb[k] = cs[k];
                const VecN<T, PITCH> B = load_row<T, PITCH, OFF32>(xs, jb);
                test(A, ja, sa, va);
                if (__ballot(vb) == 0ull) break;
                ja = step();
                va = alive;
#pragma unroll
                for (int k = 0; k < 3; ++k) sa[k] = cs[k];
                A = load_row<T, PITCH, OFF32>(xs, ja);
                test(B, jb, sb, vb);
                if (__ballot(va) == 0ull) break;
            }
        };
        if (__ballot(any_shift) != 0ull) walk(std::integral_constant<bool, true>());
        else walk(std::integral_constant<bool, false>());
    }
}

// ---------------------------------------------------------------------------
// all pairs of a small system (the brute-force fallback for small N)
// ---------------------------------------------------------------------------

// visit(j, dx, d2, shifted) for every slot j in [j0, j1) that is a neighbour of
// xi, testing each particle once at its minimum image: in each periodic
// dimension s_k = -L if t_k > L/2, +L if t_k < -L/2, else 0, with t_k =
// fl(x_jk - x_ik).  For a neighbour this is the shift the box search uses (the
// side is at least twice the guarded cutoff, so only one image can be within
// r), so the pair set and each pair's dx are those of the box search; a
// non-neighbour is rejected at every image because its nearest one is.
// The slots visited are j0, j0 + step, j0 + 2 step, ... below j1 (a group of
// lanes splits one particle's slots this way).
template <typename T, int D, typename Visit>
__device__ __forceinline__ void allpairs_loop(const SysParams<T>& P, const T* __restrict__ xs, uint32_t j0,
                                              uint32_t j1, uint32_t step, const T* xi, Visit& visit) {
    constexpr int PITCH = Pitch<D>::value;
    const VecN<T, PITCH>* __restrict__ xv = reinterpret_cast<const VecN<T, PITCH>*>(xs);
    T h[D], L[D];
    bool per[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        L[k] = P.L[k];
        h[k] = T(0.5) * L[k];
        per[k] = P.periodic[k] != 0;
    }
    const T r2 = P.r2;
    auto one = [&](uint32_t j, const VecN<T, PITCH>& a) {
        T dx[D];
        bool shifted = false;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const T t = a.v[k] - xi[k];
            const T sk = !per[k] ? T(0) : (t > h[k] ? -L[k] : (t < -h[k] ? L[k] : T(0)));
            shifted |= sk != T(0);
            dx[k] = t + sk;
        }
        T d2 = dx[0] * dx[0];
        if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
        if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
        if (d2 > T(0) && d2 < r2) visit(j, dx, d2, shifted);
    };
    uint32_t j = j0;
    for (; j + step < j1; j += 2 * step) {
        const VecN<T, PITCH> a = xv[j];
        const VecN<T, PITCH> b = xv[j + step];
        one(j, a);
        one(j + step, b);
    }
    if (j < j1) one(j, xv[j]);
}

// Sum of v over the G lanes of a group (G a power of two dividing the wave) by a
// fixed xor butterfly, so the result does not depend on timing.
template <int G, typename T>
__device__ __forceinline__ T group_reduce(T v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

// ---------------------------------------------------------------------------
// recorded neighbour lists
// ---------------------------------------------------------------------------

// An entry of a recorded list: the neighbour's slot, with the top bit set when
// the box search reached it through a nonzero image shift.
constexpr uint32_t kNbrShift = 0x80000000u;
constexpr uint32_t kNbrSlot = 0x7FFFFFFFu;

// Displacement and squared distance of a recorded pair, bit for bit those of
// the box search: dx_k = fl(t_k + s_k) with t_k = fl(x_jk - x_ik).  For a
// flagged entry s_k is recovered as the minimum image of t_k in each periodic
// dimension: an accepted pair has |dx_k| < r, and the periodic side is at
// least twice the guarded cutoff, so exactly one of -L, 0, +L brings t_k
// within L/2, and it is the shift the search used.
template <typename T, int D>
__device__ __forceinline__ T replay_pair(const SysParams<T>& P, const T* xj, const T* xi, bool shifted, T* dx) {
#pragma unroll
    for (int k = 0; k < D; ++k) dx[k] = xj[k] - xi[k];
    if (shifted) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const T L = P.L[k];
            const T h = T(0.5) * L;
            const T sk = !P.periodic[k] ? T(0) : (dx[k] > h ? -L : (dx[k] < -h ? L : T(0)));
            dx[k] = dx[k] + sk;
        }
    }
    T d2 = dx[0] * dx[0];
    if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
    if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
    return d2;
}

// Calls visit(j, dx, d2) for the recorded neighbours of slot s in recorded
// order.  Entry k of slot s is at nbr[k * n + s], so the lanes of a wave read
// consecutive words.  Two entries per iteration keep two position loads in
// flight.
template <typename T, int D, typename Visit>
__device__ __forceinline__ void replay_list(const SysParams<T>& P, const T* __restrict__ xs,
                                            const uint32_t* __restrict__ nbr, uint32_t n, uint32_t s, uint32_t cnt,
                                            const T* xi, Visit& visit) {
    constexpr int PITCH = Pitch<D>::value;
    const VecN<T, PITCH>* __restrict__ xv = reinterpret_cast<const VecN<T, PITCH>*>(xs);
    const uint32_t* p = nbr + s;
    const size_t stride = (size_t)n;
    uint32_t k = 0;
    for (; k + 1 < cnt; k += 2) {
        const uint32_t e0 = p[0];
        const uint32_t e1 = p[stride];
        p += 2 * stride;
        const VecN<T, PITCH> a = xv[e0 & kNbrSlot];
        const VecN<T, PITCH> b = xv[e1 & kNbrSlot];
        T dx[D];
        T d2 = replay_pair<T, D>(P, a.v, xi, (e0 & kNbrShift) != 0u, dx);
        visit(e0 & kNbrSlot, dx, d2);
        d2 = replay_pair<T, D>(P, b.v, xi, (e1 & kNbrShift) != 0u, dx);
        visit(e1 & kNbrSlot, dx, d2);
    }
    if (k < cnt) {
        const uint32_t e0 = p[0];
        const VecN<T, PITCH> a = xv[e0 & kNbrSlot];
        T dx[D];
        const T d2 = replay_pair<T, D>(P, a.v, xi, (e0 & kNbrShift) != 0u, dx);
        visit(e0 & kNbrSlot, dx, d2);
    }
}

// ---------------------------------------------------------------------------
// helpers of the cell-group mapping
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


// ---------------------------------------------------------------------------
// launchers (one translation unit each, explicitly instantiated)
// ---------------------------------------------------------------------------

// Lane-per-particle forward.
template <typename T, int D, int OP, bool BATCH>
void launch_lane_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int block);

// Lane-per-particle adjoint.
template <typename T, int D, int OP, bool BATCH>
void launch_lane_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga, int block);

// Forward / adjoint over the cell list's recorded neighbour list (a particle
// with more neighbours than the list holds is summed by the box search).
template <typename T, int D, int OP, bool BATCH>
void launch_nbr_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y);
template <typename T, int D, int OP, bool BATCH>
void launch_nbr_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                    T* ga);

// Forward and adjoint (for an upstream gradient known in advance) in one box search.
template <typename T, int D, int OP, bool BATCH>
void launch_lane_fused(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                       T* y, T* gx, T* ga);
template <typename T, int D, int OP, bool BATCH>
void launch_mask_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y);
template <typename T, int D, int OP, bool BATCH>
void launch_half_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y);
template <typename T, int D, int OP, bool BATCH>
void launch_mask_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga);
template <typename T, int D, int OP, bool BATCH, int MODE>
void launch_flat(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* y,
                 T* gx, T* ga);

// Forward / adjoint over every particle of the lane's system (minimum image).
template <typename T, int D, int OP, bool BATCH>
void launch_all_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y);
template <typename T, int D, int OP, bool BATCH>
void launch_all_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                    T* ga);

#define ABORIA_FOR_EACH_PAIR_INSTANCE(X)                                                            \
    X(float, 1, 0, false) X(float, 1, 1, false) X(float, 1, 2, false)                     \
    X(float, 1, 3, false) X(float, 1, 4, false) X(float, 2, 0, false)                     \
    X(float, 2, 1, false) X(float, 2, 2, false) X(float, 2, 3, false)                     \
    X(float, 2, 4, false) X(float, 3, 0, false) X(float, 3, 1, false)                     \
    X(float, 3, 2, false) X(float, 3, 3, false) X(float, 3, 4, false)                     \
    X(float, 1, 0, true) X(float, 1, 1, true) X(float, 1, 2, true)                        \
    X(float, 1, 3, true) X(float, 1, 4, true) X(float, 2, 0, true)                        \
    X(float, 2, 1, true) X(float, 2, 2, true) X(float, 2, 3, true)                        \
    X(float, 2, 4, true) X(float, 3, 0, true) X(float, 3, 1, true)                        \
    X(float, 3, 2, true) X(float, 3, 3, true) X(float, 3, 4, true)                        \
    X(double, 1, 0, false) X(double, 1, 1, false) X(double, 1, 2, false)                  \
    X(double, 1, 3, false) X(double, 1, 4, false) X(double, 2, 0, false)                  \
    X(double, 2, 1, false) X(double, 2, 2, false) X(double, 2, 3, false)                  \
    X(double, 2, 4, false) X(double, 3, 0, false) X(double, 3, 1, false)                  \
    X(double, 3, 2, false) X(double, 3, 3, false) X(double, 3, 4, false)                  \
    X(double, 1, 0, true) X(double, 1, 1, true) X(double, 1, 2, true)                     \
    X(double, 1, 3, true) X(double, 1, 4, true) X(double, 2, 0, true)                     \
    X(double, 2, 1, true) X(double, 2, 2, true) X(double, 2, 3, true)                     \
    X(double, 2, 4, true) X(double, 3, 0, true) X(double, 3, 1, true)                     \
    X(double, 3, 2, true) X(double, 3, 3, true) X(double, 3, 4, true)

}  // namespace aboria
