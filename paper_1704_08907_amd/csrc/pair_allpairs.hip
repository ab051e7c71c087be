// Neighbour sums of small systems by testing all pairs of a system (the
// brute-force fallback that Section 3 notes the GROMACS search uses for small
// N): a group of lanes per particle in cell order walks every slot of its
// own system at the minimum image.  The pair set and each pair's displacement
// are those of the box search; each lane adds its summands in slot order and
// the group combines them by a fixed butterfly.  Meant for systems whose size makes the N^2 tests cheaper than a
// cell list (the dispatcher caps the system size).
#include "pair_common.hpp"

namespace aboria {

// G lanes per particle (G in {1, 4, 16, 64}, chosen so that the launch has
// tens of thousands of lanes even for a few hundred particles): lane l of a
// group takes slots l, l + G, ... of the system; the group's partial sums are
// combined by a fixed butterfly and its first lane writes the result.
template <typename T, int D, int OP, bool BATCH, int G>
__global__ __launch_bounds__(256) void k_all_fwd(const T* __restrict__ xs, const uint32_t* __restrict__ perm,
                                                 uint32_t n, const SysParams<T>* __restrict__ sp,
                                                 const uint32_t* __restrict__ sys_part, int nsys,
                                                 const T* __restrict__ a_s, OpArgs<T> q, T* __restrict__ y) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x / G);
    const uint32_t s = first + threadIdx.x / G;
    const uint32_t lane = threadIdx.x % G;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s < n ? s : n - 1);
    const bool live = s < n;
    const uint32_t sc = live ? s : n - 1;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, sc, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[sc] : T(0);
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    };
    if (live) allpairs_loop<T, D>(P, xs, P.part_base + lane, P.part_end, G, xi, visit);
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = group_reduce<G>(acc[k]);
    if (!live || lane != 0) return;
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
}

template <typename T, int D, int OP, bool BATCH, int G>
__global__ __launch_bounds__(256) void k_all_bwd(const T* __restrict__ xs, const uint32_t* __restrict__ perm,
                                                 uint32_t n, const SysParams<T>* __restrict__ sp,
                                                 const uint32_t* __restrict__ sys_part, int nsys,
                                                 const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                 OpArgs<T> q, T* __restrict__ gx, T* __restrict__ ga) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x / G);
    const uint32_t s = first + threadIdx.x / G;
    const uint32_t lane = threadIdx.x % G;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s < n ? s : n - 1);
    const bool live = s < n;
    const uint32_t sc = live ? s : n - 1;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, sc, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[sc] : T(0);
    T gyi[NY];
    load_gy<T, NY>(gy_s, sc, gyi);
    T accx[D], acca[1] = {T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = T(0);
    const T r = P.r;
    auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
        const T aj = OpShape<OP, D>::NA ? a_s[j] : T(0);
        T gyj[NY];
        load_gy<T, NY>(gy_s, j, gyj);
        Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
    };
    if (live) allpairs_loop<T, D>(P, xs, P.part_base + lane, P.part_end, G, xi, visit);
#pragma unroll
    for (int k = 0; k < D; ++k) accx[k] = group_reduce<G>(accx[k]);
    if (OpShape<OP, D>::NA) acca[0] = group_reduce<G>(acca[0]);
    if (!live || lane != 0) return;
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
    if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
}

// Lanes per particle: enough groups for about 64K lanes in flight, at most a wave.
inline int all_group(uint32_t n) {
    const uint64_t want = 65536;
    if ((uint64_t)n * 16 < want) return 64;
    if ((uint64_t)n * 4 < want) return 16;
    if ((uint64_t)n < want) return 4;
    return 1;
}

template <typename T, int D, int OP, bool BATCH>
void launch_all_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const int G = all_group(n);
    const dim3 grid((uint32_t)(((uint64_t)n * G + 255) / 256));
#define L(GG) hipLaunchKernelGGL((k_all_fwd<T, D, OP, BATCH, GG>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs, \
                                 c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, y)
    switch (G) {
        case 64: L(64); break;
        case 16: L(16); break;
        case 4: L(4); break;
        default: L(1); break;
    }
#undef L
}

template <typename T, int D, int OP, bool BATCH>
void launch_all_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                    T* ga) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const int G = all_group(n);
    const dim3 grid((uint32_t)(((uint64_t)n * G + 255) / 256));
#define L(GG) hipLaunchKernelGGL((k_all_bwd<T, D, OP, BATCH, GG>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs, \
                                 c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, gx, ga)
    switch (G) {
        case 64: L(64); break;
        case 16: L(16); break;
        case 4: L(4); break;
        default: L(1); break;
    }
#undef L
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                                 \
    template void launch_all_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, T*); \
    template void launch_all_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*,      \
                                                  const T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
