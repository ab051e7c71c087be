// Neighbour-sum adjoint over a recorded neighbour list (gather form, no
// atomics): one lane per particle k in cell order adds, for each recorded
// neighbour i, J1(k,i)^T gy_k + J2(i,k)^T gy_i, evaluated on accepted pairs
// only.  Order and arithmetic are those of the box-search adjoint.  A particle
// whose list overflowed, or every particle when the list belongs to an older
// build, is summed by the box search.
#include "pair_common.hpp"

namespace aboria {

template <typename T, int D, int OP, bool BATCH>
__global__ __launch_bounds__(256) void k_nbr_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ perm, uint32_t n,
                                                 const SysParams<T>* __restrict__ sp,
                                                 const uint32_t* __restrict__ sys_part, int nsys,
                                                 const uint32_t* __restrict__ nbr,
                                                 const uint32_t* __restrict__ nbr_count, uint32_t cap,
                                                 const uint32_t* __restrict__ gen, const T* __restrict__ a_s,
                                                 const T* __restrict__ gy_s, OpArgs<T> q, T* __restrict__ gx,
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
    load_gy<T, NY>(gy_s, s, gyi);
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    auto pair = [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        T gyj[NY];
        load_gy<T, NY>(gy_s, j, gyj);
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    };
    const uint32_t cnt = nbr_count[s];
    if (gen[0] == gen[1] && cnt <= cap) {
        replay_list<T, D>(P, xs, nbr, n, s, cnt, xi, pair);
    } else {
        auto visit = [&](uint32_t j, const T* dx, T d2, bool) { pair(j, dx, d2); };
        neighbour_loop<T, D>(P, xs, off, n, xi, visit);
    }
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

template <typename T, int D, int OP, bool BATCH>
void launch_nbr_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                    T* ga) {
    const uint32_t n = (uint32_t)c->n;
    hipLaunchKernelGGL((k_nbr_bwd<T, D, OP, BATCH>), dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       (const T*)c->xs, c->off, c->perm, n, reinterpret_cast<const SysParams<T>*>(c->params_dev),
                       c->sys_part_dev, c->nsys, c->nbr, c->nbr_count, c->nbr_cap, c->gen, a_s, gy_s, q, gx, ga);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                         \
    template void launch_nbr_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, \
                                                  const T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
