// Lane-per-particle neighbour sums whose candidates are staged in LDS: for
// each stencil row a wave copies the span of cell-ordered positions its lanes
// will test into its own 8 KB LDS region with coalesced loads, and the lanes
// read their candidates from there.  In the plain lane kernels every lane
// issues its own 16-byte load per candidate, which keeps the texture
// addressing unit about as busy as the vector ALUs; here the global side is one
// coalesced pass per row and wave, and lanes of one home cell read the same
// LDS entries.  Same candidates, order and arithmetic as the plain kernels, so
// the results are identical.
#include "pair_common.hpp"

namespace aboria {

template <typename T, int D>
struct StageCap {
    static constexpr int value = 8192 / (int)sizeof(VecN<T, Pitch<D>::value>);
};

template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(256) void k_stage_fwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                   const SysParams<T>* __restrict__ sp,
                                                   const uint32_t* __restrict__ sys_part, int nsys,
                                                   const T* __restrict__ a_s, OpArgs<T> q, T* __restrict__ y) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int CAP = StageCap<T, D>::value;
    __shared__ VecN<T, Pitch<D>::value> stage[256 / kWave][CAP];
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const bool live = s < n;
    const uint32_t sc = live ? s : n - 1;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, sc);
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, sc, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[sc] : T(0);
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? load_row<T, 1, true>(a_s, j).v[0] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    };
    neighbour_loop_staged<T, D, CAP>(P, xs, off, n, xi, live, stage[threadIdx.x / kWave], visit);
    if (!live) return;
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
}

template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(256) void k_stage_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                   const SysParams<T>* __restrict__ sp,
                                                   const uint32_t* __restrict__ sys_part, int nsys,
                                                   const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                   OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int CAP = StageCap<T, D>::value;
    __shared__ VecN<T, Pitch<D>::value> stage[256 / kWave][CAP];
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const bool live = s < n;
    const uint32_t sc = live ? s : n - 1;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, sc);
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, sc, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[sc] : T(0);
    T gyi[NY];
    load_gy<T, NY, true>(gy_s, sc, gyi);
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? load_row<T, 1, true>(a_s, j).v[0] : T(0);
        T gyj[NY];
        load_gy<T, NY, true>(gy_s, j, gyj);
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    };
    neighbour_loop_staged<T, D, CAP>(P, xs, off, n, xi, live, stage[threadIdx.x / kWave], visit);
    if (!live) return;
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

template <typename T, int D, int OP, bool BATCH>
void launch_stage_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y) {
    const uint32_t n = (uint32_t)c->n;
    hipLaunchKernelGGL((k_stage_fwd<T, D, OP, BATCH>), dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       (const T*)c->xs, c->off, c->perm, n, reinterpret_cast<const SysParams<T>*>(c->params_dev),
                       c->sys_part_dev, c->nsys, a_s, q, y);
}

template <typename T, int D, int OP, bool BATCH>
void launch_stage_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                      T* ga) {
    const uint32_t n = (uint32_t)c->n;
    hipLaunchKernelGGL((k_stage_bwd<T, D, OP, BATCH>), dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       (const T*)c->xs, c->off, c->perm, n, reinterpret_cast<const SysParams<T>*>(c->params_dev),
                       c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                                   \
    template void launch_stage_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, T*); \
    template void launch_stage_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*,      \
                                                    const T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
