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

template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(256) void k_lane_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
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
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        T gyj[NY];
#pragma unroll
        for (int k = 0; k < NY; ++k) gyj[k] = gy_s[(size_t)j * NY + k];
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    };
    neighbour_loop<T, D>(P, xs, off, n, xi, visit);
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
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
    const uint32_t s = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + tid;
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
#pragma unroll
            for (int m = 0; m < NY; ++m) gyj[m] = gy_s[(size_t)j * NY + m];
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

template <typename T, int D, int OP, bool BATCH>
void launch_lane_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga, int block, bool compact) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (compact && block == 128) {
        hipLaunchKernelGGL((k_lane_bwd_compact<T, D, OP, BATCH, 128, 64>), dim3((n + 127) / 128), dim3(128), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    } else if (compact) {
        hipLaunchKernelGGL((k_lane_bwd_compact<T, D, OP, BATCH, 256, 48>), dim3((n + 255) / 256), dim3(256), 0,
                           ctx->stream, (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s,
                           q, gx, ga);
    } else {
        hipLaunchKernelGGL((k_lane_bwd<T, D, OP, BATCH>), dim3((n + block - 1) / block), dim3(block), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga);
    }
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                        \
    template void launch_lane_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, \
                                                   const T*, T*, T*, int, bool);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
