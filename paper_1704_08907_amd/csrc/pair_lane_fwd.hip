// Lane-per-particle neighbour-sum forward: one lane per particle in cell
// order, so the lanes of a wave share home cells and therefore candidate
// cells, and their candidate loads hit the same cache lines.
#include "pair_common.hpp"

namespace aboria {

template <typename T, int D, int OP, bool BATCH, bool OFF32>
__global__ __launch_bounds__(256) void k_lane_fwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                  const uint32_t* __restrict__ perm, uint32_t n,
                                                  const SysParams<T>* __restrict__ sp,
                                                  const uint32_t* __restrict__ sys_part, int nsys,
                                                  const T* __restrict__ a_s, OpArgs<T> q, T* __restrict__ y) {
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
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    };
    neighbour_loop_staged<T, D, OFF32>(P, xs, off, n, xi, visit);
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
}

template <typename T, int D, int OP, bool BATCH>
void launch_lane_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int block) {
    const uint32_t n = (uint32_t)c->n;
    const dim3 grid((n + block - 1) / block);
    if (off32_rows<T>(n))
        hipLaunchKernelGGL((k_lane_fwd<T, D, OP, BATCH, true>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, reinterpret_cast<const SysParams<T>*>(c->params_dev), c->sys_part_dev,
                           c->nsys, a_s, q, y);
    else
        hipLaunchKernelGGL((k_lane_fwd<T, D, OP, BATCH, false>), grid, dim3(block), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, reinterpret_cast<const SysParams<T>*>(c->params_dev), c->sys_part_dev,
                           c->nsys, a_s, q, y);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                   \
    template void launch_lane_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, \
                                                   const T*, T*, int);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
