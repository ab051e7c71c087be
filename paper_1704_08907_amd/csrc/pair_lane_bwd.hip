// Lane-per-particle neighbour-sum adjoint (gather form: no atomics, no stored
// pair list between calls).
//
// The compacting kernel runs in two phases per particle.  Phase 1 scans the
// box-search candidates with the cheap pair test and appends each accepted
// neighbour's slot to the lane's list in LDS (entry k of lane t at
// [k * BLOCK + t], so a wave's appends hit 64 different banks); the top bit
// marks a pair that needed an image shift.  Phase 2 walks the list and
// evaluates the adjoint summand only for accepted pairs, instead of for every
// candidate of a wave in which any lane accepted.  A flagged pair's shift is
// recomputed per periodic dimension as the minimum image of fl(x_j - x_i):
// for an accepted pair it is the stencil's shift, because the periodic side is
// at least twice the guarded cutoff.  A full list is drained early, so any
// number of neighbours is handled.
#include "pair_common.hpp"

namespace aboria {

template <typename T, int D, int OP, bool BATCH, bool OFF32>
__global__ __launch_bounds__(256) void k_lane_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                  const uint32_t* __restrict__ perm, uint32_t n,
                                                  const SysParams<T>* __restrict__ sp,
                                                  const uint32_t* __restrict__ sys_part, int nsys,
                                                  const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                  OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
    load_gy<T, NY, OFF32>(gy_s, s, gyi);
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    if constexpr (kDeferAdjoint<OP>) {
        // accepted pairs first, then their summands (the neighbour's gradient row is
        // loaded with its position)
        auto visit = [&](uint32_t j, const T* dx, T d2, bool, const T* gyj) {
            const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
        };
        neighbour_loop_aux<T, D, OFF32, NY>(P, xs, gy_s, off, n, xi, visit);
    } else {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
            T gyj[NY];
            load_gy<T, NY, OFF32>(gy_s, j, gyj);
            Op::bwd(q, r, dx, d2, ai, T(0), gyi, gyj, accx, acca);
        };
        neighbour_loop<T, D, OFF32>(P, xs, off, n, xi, visit);
    }
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

// Forward and adjoint in one box search (the upstream gradient is known before
// the forward): each accepted pair adds its forward summand to y_i and its
// adjoint contribution to gx_i (and ga_i), in the order of the separate kernels.
template <typename T, int D, int OP, bool BATCH, bool OFF32>
__global__ __launch_bounds__(256) void k_lane_fused(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                    const uint32_t* __restrict__ perm, uint32_t n,
                                                    const SysParams<T>* __restrict__ sp,
                                                    const uint32_t* __restrict__ sys_part, int nsys,
                                                    const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                    OpArgs<T> q, T* __restrict__ y, T* __restrict__ gx,
                                                    T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
    load_gy<T, NY, OFF32>(gy_s, s, gyi);
    T acc[NY], accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    if constexpr (kDeferAdjoint<OP>) {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool, const T* gyj) {
            const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
            Op::fwd(q, r, dx, d2, ai, aj, acc);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
        };
        neighbour_loop_aux<T, D, OFF32, NY>(P, xs, gy_s, off, n, xi, visit);
    } else {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
            T gyj[NY];
            load_gy<T, NY, OFF32>(gy_s, j, gyj);
            Op::fwd(q, r, dx, d2, ai, T(0), acc);
            Op::bwd(q, r, dx, d2, ai, T(0), gyi, gyj, accx, acca);
        };
        neighbour_loop<T, D, OFF32>(P, xs, off, n, xi, visit);
    }
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

template <typename T, int D, int OP, bool BATCH>
void launch_lane_fused(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                       T* y, T* gx, T* ga) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + 255) / 256);
    if (off32_rows<T>(n))
        hipLaunchKernelGGL((k_lane_fused<T, D, OP, BATCH, true>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, y, gx, ga);
    else
        hipLaunchKernelGGL((k_lane_fused<T, D, OP, BATCH, false>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, y, gx, ga);
}

template <typename T, int D, int OP, bool BATCH, int BLOCK, int CAP>
__global__ __launch_bounds__(BLOCK) void k_lane_bwd_compact(
    const T* __restrict__ xs, const uint32_t* __restrict__ off, const uint32_t* __restrict__ perm, uint32_t n,
    const SysParams<T>* __restrict__ sp, const uint32_t* __restrict__ sys_part, int nsys, const T* __restrict__ a_s,
    const T* __restrict__ gy_s, OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int PITCH = Pitch<D>::value;
    constexpr uint32_t kShiftBit = 0x80000000u;
    __shared__ uint32_t list[CAP * BLOCK];
    const uint32_t tid = threadIdx.x;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
    const uint32_t s = first + tid;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
    load_gy<T, NY>(gy_s, s, gyi);
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    uint32_t cnt = 0;

    auto drain = [&]() {
        for (uint32_t k = 0; k < cnt; ++k) {
            const uint32_t e = list[k * BLOCK + tid];
            const uint32_t j = e & ~kShiftBit;
            const VecN<T, PITCH> v = reinterpret_cast<const VecN<T, PITCH>*>(xs)[j];
            T dx[D];
#pragma unroll
            for (int m = 0; m < D; ++m) dx[m] = v.v[m] - xi[m];
            if (e & kShiftBit) {
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    if (P.periodic[m]) {
                        const T half = T(0.5) * P.L[m];
                        const T sm = dx[m] > half ? -P.L[m] : (dx[m] < -half ? P.L[m] : T(0));
                        dx[m] = dx[m] + sm;
                    }
                }
            }
            T d2 = dx[0] * dx[0];
            if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
            if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
            const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
            T gyj[NY];
            load_gy<T, NY>(gy_s, j, gyj);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
        }
        cnt = 0;
    };
    auto visit = [&](uint32_t j, const T*, T, bool shifted) {
        list[cnt * BLOCK + tid] = j | (shifted ? kShiftBit : 0u);
        if (++cnt == (uint32_t)CAP) drain();
    };
    neighbour_loop<T, D>(P, xs, off, n, xi, visit);
    drain();
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

// Wave-queue adjoint.  The box-search loop runs wave-uniformly over each
// stencil piece (lanes past their own piece length are masked), and every
// accepted pair is appended -- with its canonical dx, its neighbour slot and
// its owner lane -- to the wave's ring of 128 entries in LDS at the position
// ballot + mbcnt give it.  As soon as 64 entries are queued, the 64 lanes take
// one entry each and evaluate the adjoint summand at full width, adding it
// into the owner's accumulator in LDS.  The adds of one wave go to its own
// accumulators in queue order, so the result does not depend on scheduling.
template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(256) void k_lane_bwd_queue(
    const T* __restrict__ xs, const uint32_t* __restrict__ off, const uint32_t* __restrict__ perm, uint32_t n,
    const SysParams<T>* __restrict__ sp, const uint32_t* __restrict__ sys_part, int nsys, const T* __restrict__ a_s,
    const T* __restrict__ gy_s, OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr bool HAS_A = OpShape<OP, D>::NA > 0;
    constexpr int PITCH = Pitch<D>::value;
    constexpr int WAVES = 4;
    constexpr uint32_t QCAP = 128;
    __shared__ T q_dx[WAVES][D][QCAP];
    __shared__ uint32_t q_j[WAVES][QCAP];
    __shared__ uint32_t q_own[WAVES][QCAP];
    __shared__ T s_gyi[WAVES][NY][kWave];
    __shared__ T s_ai[WAVES][kWave];
    __shared__ T s_acc[WAVES][D + 1][kWave];

    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
    const bool live = s < n;
    const uint32_t sc = live ? s : 0u;
    const int b = system_of_row<BATCH>(sys_part, nsys, s - threadIdx.x, sc);
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, sc, xi);
    {
        T g[NY];
        load_gy<T, NY>(gy_s, sc, g);
#pragma unroll
        for (int k = 0; k < NY; ++k) s_gyi[w][k][lane] = live ? g[k] : T(0);
    }
    s_ai[w][lane] = (HAS_A && live) ? a_s[sc] : T(0);
#pragma unroll
    for (int k = 0; k <= D; ++k) s_acc[w][k][lane] = T(0);
    const T r = P.r;
    const T r2 = P.r2;

    // the wave's queue: entries [head, tail) of the ring, head and tail uniform
    uint32_t head = 0, tail = 0;
    auto drain = [&](uint32_t count) {  // evaluate `count` (<= 64) queued entries
        if (lane < count) {
            const uint32_t e = (head + lane) % QCAP;
            T dx[D];
#pragma unroll
            for (int k = 0; k < D; ++k) dx[k] = q_dx[w][k][e];
            const uint32_t j = q_j[w][e];
            const uint32_t own = q_own[w][e];
            T d2 = dx[0] * dx[0];
            if constexpr (D >= 2) d2 = fma_t(dx[1], dx[1], d2);
            if constexpr (D >= 3) d2 = fma_t(dx[2], dx[2], d2);
            T gyi[NY], gyj[NY];
            load_gy<T, NY>(gy_s, j, gyj);
#pragma unroll
            for (int k = 0; k < NY; ++k) gyi[k] = s_gyi[w][k][own];
            const T ai = s_ai[w][own];
            const T aj = HAS_A ? a_s[j] : T(0);
            T c[D], ca[1] = {T(0)};
#pragma unroll
            for (int k = 0; k < D; ++k) c[k] = T(0);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, c, ca);
#pragma unroll
            for (int k = 0; k < D; ++k) atomicAdd(&s_acc[w][k][own], c[k]);
            if (HAS_A) atomicAdd(&s_acc[w][D][own], ca[0]);
        }
        head += count;
    };

    // box search, wave-uniform over the (row, x-piece) slots
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T t = xi[k] - P.lo[k];
        const T qq = t * P.inv_w[k];
        const T f = floor(qq);
        c[k] = !(f >= T(0)) ? 0 : (f > T(P.n[k] - 1) ? P.n[k] - 1 : (int32_t)f);
    }
    const int32_t nx = P.n[0];
    int32_t plo[3] = {0, 0, 0}, phi[3] = {-1, -1, -1};
    T psh[3] = {T(0), T(0), T(0)};
    if (nx >= 3) {
        plo[0] = c[0] > 0 ? c[0] - 1 : 0;
        phi[0] = c[0] < nx - 1 ? c[0] + 1 : nx - 1;
        if (P.periodic[0] && c[0] == 0) { plo[1] = phi[1] = nx - 1; psh[1] = -P.L[0]; }
        if (P.periodic[0] && c[0] == nx - 1) { plo[2] = phi[2] = 0; psh[2] = P.L[0]; }
    } else {
        for (int o = -1; o <= 1; ++o) {
            int32_t v = c[0] + o;
            T sv = T(0);
            if (v < 0) { if (!P.periodic[0]) continue; v += nx; sv = -P.L[0]; }
            else if (v >= nx) { if (!P.periodic[0]) continue; v -= nx; sv = P.L[0]; }
            plo[o + 1] = phi[o + 1] = v;
            psh[o + 1] = sv;
        }
    }
    constexpr int NROWS = D == 1 ? 1 : (D == 2 ? 3 : 9);
    const VecN<T, PITCH>* __restrict__ xv = reinterpret_cast<const VecN<T, PITCH>*>(xs);
    for (int rr = 0; rr < NROWS; ++rr) {
        T sh[3] = {T(0), T(0), T(0)};
        uint32_t row = 0;
        bool skip = !live;
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
        const uint32_t rowbase = P.cell_base + (uint32_t)nx * row;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            uint32_t j0 = 0, len = 0;
            if (!skip && phi[p] >= plo[p]) {
                j0 = off[rowbase + plo[p]];
                len = min(off[rowbase + phi[p] + 1], n) - j0;
            }
            sh[0] = psh[p];
            bool lane_shift = false;
#pragma unroll
            for (int k = 0; k < D; ++k) lane_shift |= sh[k] != T(0);
            const bool any_shift = __ballot(lane_shift) != 0ull;
            uint32_t tmax = len;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) tmax = max(tmax, (uint32_t)__shfl_xor((int)tmax, m, 64));
            for (uint32_t t = 0; t < tmax; ++t) {
                bool ok = false;
                T dx[D], d2;
                uint32_t j = j0 + t;
                if (t < len) {
                    const VecN<T, PITCH> v = xv[j];
                    ok = any_shift ? pair_test<T, D, true>(v.v, xi, sh, r2, dx, &d2)
                                   : pair_test<T, D, false>(v.v, xi, sh, r2, dx, &d2);
                }
                const uint64_t mask = __ballot(ok);
                if (ok) {
                    const uint32_t pos = (tail + (uint32_t)__popcll(mask & lanemask_lt())) % QCAP;
#pragma unroll
                    for (int k = 0; k < D; ++k) q_dx[w][k][pos] = dx[k];
                    q_j[w][pos] = j;
                    q_own[w][pos] = lane;
                }
                tail += (uint32_t)__popcll(mask);
                if (tail - head >= kWave) drain(kWave);
            }
        }
    }
    drain(tail - head);
    if (live) {
        const uint32_t o = perm[s];
#pragma unroll
        for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = s_acc[w][k][lane];
        if (HAS_A && ga) ga[o] = s_acc[w][D][lane];
    }
}

template <typename T, int D, int OP, bool BATCH>
void launch_lane_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga, int block, bool compact) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (compact && block == 512) {  // the wave queue (workgroups of 256)
        hipLaunchKernelGGL((k_lane_bwd_queue<T, D, OP, BATCH>), dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga);
    } else if (compact && block == 128) {
        hipLaunchKernelGGL((k_lane_bwd_compact<T, D, OP, BATCH, 128, 64>), dim3((n + 127) / 128), dim3(128), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    } else if (compact) {
        hipLaunchKernelGGL((k_lane_bwd_compact<T, D, OP, BATCH, 256, 48>), dim3((n + 255) / 256), dim3(256), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    } else if (off32_rows<T>(n)) {
        hipLaunchKernelGGL((k_lane_bwd<T, D, OP, BATCH, true>), dim3((n + block - 1) / block), dim3(block), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    } else {
        hipLaunchKernelGGL((k_lane_bwd<T, D, OP, BATCH, false>), dim3((n + block - 1) / block), dim3(block), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    }
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                          \
    template void launch_lane_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*,   \
                                                   const T*, T*, T*, int, bool);                                   \
    template void launch_lane_fused<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, \
                                                     const T*, T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
