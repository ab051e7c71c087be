// Lane-per-particle neighbour sums over the flattened, pruned box search
// (flat_loop): forward, adjoint, and both in one pass.  One kernel template;
// the three modes are instantiated in their own translation units.
#pragma once

#include "pair_common.hpp"

namespace aboria {

constexpr int kFlatBlock = 256;
constexpr int kFlatCap = 8;  // ranges a lane lists per round (>= 2 kMaxReach + 1)

enum FlatMode { kFlatFwd = 0, kFlatBwd = 1, kFlatFused = 2 };

template <typename T, int D, int OP, bool BATCH, bool OFF32, int MODE>
__global__ __launch_bounds__(kFlatBlock) void k_flat(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ perm, uint32_t n,
                                                     const SysParams<T>* __restrict__ sp,
                                                     const uint32_t* __restrict__ sys_part, int nsys,
                                                     const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                     OpArgs<T> q, T* __restrict__ y, T* __restrict__ gx,
                                                     T* __restrict__ ga) {
    static_assert(kFlatCap >= 2 * kMaxReach + 1, "a row of a narrow grid must fit one round");
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr bool FWD = MODE != kFlatBwd, BWD = MODE != kFlatFwd;
    __shared__ FlatRanges<kFlatCap, kFlatBlock> ranges;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    T gyi[NY];
    if (BWD) load_gy<T, NY, OFF32>(gy_s, s, gyi);
    T acc[NY], accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
        if (FWD) Op::fwd(q, r, dx, d2, ai, aj, acc);
        if (BWD) {
            T gyj[NY];
            load_gy<T, NY, OFF32>(gy_s, j, gyj);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
        }
    };
    flat_loop<T, D, kFlatCap, kFlatBlock, OFF32>(P, xs, off, n, xi, s, ranges, visit);
    const uint32_t o = perm[s];
    if (FWD) {
#pragma unroll
        for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
    }
    if (BWD) {
#pragma unroll
        for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
        if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
    }
}

template <typename T, int D, int OP, bool BATCH, int MODE>
void launch_flat(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* y,
                 T* gx, T* ga) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + kFlatBlock - 1) / kFlatBlock);
    if (off32_rows<T>(n))
        hipLaunchKernelGGL((k_flat<T, D, OP, BATCH, true, MODE>), grid, dim3(kFlatBlock), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, y, gx, ga);
    else
        hipLaunchKernelGGL((k_flat<T, D, OP, BATCH, false, MODE>), grid, dim3(kFlatBlock), 0, ctx->stream,
                           (const T*)c->xs, c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, y, gx, ga);
}

}  // namespace aboria
