// Lane-per-particle neighbour-sum adjoint (gather form: no atomics, no stored
// pair list between calls).
//
// The row-search adjoint defers the summands of vector operators: it tests up
// to 32 candidates into a per-lane bit mask, then pops the bits, reloads each
// accepted pair's position and gradient row, recomputes its displacement
// exactly and evaluates the summand, so a wave runs the summand as often as
// its busiest lane has pairs instead of for every candidate that any lane
// accepted.  The pairs and their order are those of the box search.
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
        neighbour_loop_aux_staged<T, D, OFF32, NY>(P, xs, gy_s, off, n, xi, visit);
    } else {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
            T gyj[NY];
            load_gy<T, NY, OFF32>(gy_s, j, gyj);
            Op::bwd(q, r, dx, d2, ai, T(0), gyi, gyj, accx, acca);
        };
        neighbour_loop_staged<T, D, OFF32>(P, xs, off, n, xi, visit);
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
        neighbour_loop_aux_staged<T, D, OFF32, NY>(P, xs, gy_s, off, n, xi, visit);
    } else {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
            T gyj[NY];
            load_gy<T, NY, OFF32>(gy_s, j, gyj);
            Op::fwd(q, r, dx, d2, ai, T(0), acc);
            Op::bwd(q, r, dx, d2, ai, T(0), gyi, gyj, accx, acca);
        };
        neighbour_loop_staged<T, D, OFF32>(P, xs, off, n, xi, visit);
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

template <typename T, int D, int OP, bool BATCH>
void launch_lane_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga, int block) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    if (off32_rows<T>(n)) {
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
                                                   const T*, T*, T*, int);                                   \
    template void launch_lane_fused<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, \
                                                     const T*, T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
