// Cell-group neighbour-sum kernel (device code shared by the forward and
// adjoint translation units).
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
#pragma once

#include "pair_common.hpp"

namespace aboria {

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
                if (BWD && live) load_gy<T, NY>(gy_s, s, gyi[qq]);
                else
                    for (int k = 0; k < NY; ++k) gyi[qq][k] = T(0);
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
                            load_gy<T, NY>(gy_s, slot, gyj);
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


template <typename T, int D, int OP, bool BATCH, bool BWD, int ROUNDS>
void launch_cells_impl(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s,
                       T* out, T* out_a) {
    constexpr int BLOCK = 128;
    constexpr int TILE = BLOCK / kGroup * ROUNDS;
    const uint32_t nwork = (uint32_t)c->ncells;
    const dim3 grid((nwork + TILE - 1) / TILE);
    hipLaunchKernelGGL((k_pair_cells<T, D, OP, BATCH, BWD, 8, BLOCK, ROUNDS>), grid, dim3(BLOCK), 0, ctx->stream,
                       (const T*)c->xs, c->off, c->perm, (uint32_t)c->n, nwork,
                       reinterpret_cast<const SysParams<T>*>(c->params_dev), c->cell_base_dev, c->nsys, a_s, gy_s, q,
                       out, out_a);
}

}  // namespace aboria
