// Lane-per-particle neighbour sums whose forward records, for every stencil
// row of a particle, one bit per candidate it accepted, and whose adjoint
// replays those bits instead of testing every candidate again.
//
// The row search with reach 1 in y and z visits the 3^(d-1) rows of the 3^d
// stencil, each the run of up to 2 m + 1 neighbouring cells in x (m the x
// reach) plus, at a periodic wrap, the wrapped remainder.  The candidates of
// row r, concatenated in visiting order, number at most kMaskBits; bit k of the
// row's mask word pair (masks[(2r) n + s], masks[(2r + 1) n + s] for slot s) is
// set when the k-th is a neighbour.
// The rows advance in lockstep across a wave, so each word is stored as one
// contiguous 256-byte run.  status[s] = the build generation the masks were
// recorded for, or 0 when a row of the particle held more than kMaskBits
// candidates; the adjoint replays a particle only when its status matches the
// current generation, and otherwise tests its candidates again (the row
// search, in the same order), so a stale or overflowing record only costs time.
//
// Replayed pairs are visited in box-search order with dx and d2 recomputed by
// the same pair test, so forward and adjoint equal the plain lane kernels' bit
// for bit.  Both read each row's main run through a per-wave LDS window
// (staged_rows): the wave copies the slots its lanes' runs span once, with
// coalesced loads, instead of every lane gathering its candidates or pairs
// from HBM.  The half-stencil forward below uses the same record layout for
// the upper half of each stencil.
#include "pair_common.hpp"

namespace aboria {

constexpr int kMaskBits = 64;  // candidates per stencil row a record covers

// Walks the stencil rows of xi that exist, in the visiting order of the box
// search with reach 1 in y and z: begin(row), then piece(j0, j1, sh) for each
// run of slots [j0, j1) of the row with its image shift sh (the cells up to m
// away in x as one run plus the wrapped remainder at a periodic boundary, or,
// on a grid narrower than 2 m + 1 cells, one run per offset), then end(row).
// Rows are numbered (dz + 1) * 3^(d-2) + (dy + 1) in visiting order, so skipped
// rows keep their numbers.
template <typename T, int D, typename Begin, typename Piece, typename End>
__device__ __forceinline__ void for_each_piece(const SysParams<T>& P, const uint32_t* __restrict__ off, uint32_t n,
                                               const T* xi, Begin&& begin, Piece&& piece, End&& end) {
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
    const int32_t zr = D >= 3 ? 1 : 0, yr = D >= 2 ? 1 : 0;
    // the row and offset loops stay rolled: unrolled, the compiler hoists work
    // across rows and the kernels hold 8 to 9 more registers per lane
#pragma unroll 1
    for (int32_t dz = -zr; dz <= zr; ++dz) {
        int32_t cz = 0;
        T sz = T(0);
        if (D >= 3 && !wrap_cell(c[2] + dz, P.n[2], P.periodic[2], P.L[2], &cz, &sz)) continue;
#pragma unroll 1
        for (int32_t dy = -yr; dy <= yr; ++dy) {
            int32_t cy = 0;
            T sy = T(0);
            if (D >= 2 && !wrap_cell(c[1] + dy, P.n[1], P.periodic[1], P.L[1], &cy, &sy)) continue;
            const int row = (dz + zr) * (2 * yr + 1) + (dy + yr);
            const uint32_t rowbase = P.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)P.n[1] * (uint32_t)cz);
            T sh[3] = {T(0), sy, sz};
            begin(row);
            auto run = [&](uint32_t ca, uint32_t cb) { piece(off[ca], min(off[cb + 1], n), sh); };
            if (wide) {
                run(rowbase + a0, rowbase + b0);
                if (b1 >= a1) {
                    sh[0] = s1;
                    run(rowbase + a1, rowbase + b1);
                }
            } else {
#pragma unroll 1
                for (int32_t o = -M; o <= M; ++o) {
                    int32_t cx;
                    if (!wrap_cell(c[0] + o, nx, P.periodic[0], P.L[0], &cx, &sh[0])) continue;
                    run(rowbase + cx, rowbase + cx);
                }
            }
            end(row);
        }
    }
}

// The walk of for_each_piece on grids at least 2 m + 1 cells wide, with each
// row's main run (the cells up to m away in x, clipped to the grid) read from
// the wave's LDS window wb when the runs of all its lanes fit in it: lo is the
// first lane's run start and hi the last lane's run end; if every lane's run
// lies in [lo, hi) and hi - lo <= kWindow, the lanes copy those slots with
// coalesced loads and win(j0, j1, sh, wb, lo) scans the run from LDS (with
// G > 0 the rows of a second array ys, G elements each, are copied too and
// follow the first array's kWindow rows in the window).  The
// wrapped remainder, and the runs of rows that do not fit, go to piece(j0, j1,
// sh) as in for_each_piece.  Rows, pieces and slot ranges are those of
// for_each_piece in the same order, so sums and records are identical.  All
// lanes of the wave that are still running take part in every row (no lane
// skips ahead), so the copy and the window reads stay in step.
template <typename T, int D, int G, typename Begin, typename Piece, typename End, typename Win>
__device__ __forceinline__ void staged_rows(const SysParams<T>& P, const uint32_t* __restrict__ off, uint32_t n,
                                            const T* xi, const T* __restrict__ xs, const T* __restrict__ ys,
                                            char* wb, Begin&& begin, Piece&& piece, End&& end, Win&& win) {
    const uint64_t act = __ballot(true);
    const uint32_t nact = (uint32_t)__popcll(act);
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T fr;
        c[k] = cell_coord(P, k, xi[k], &fr);
    }
    const int32_t M = P.reach[0];
    const int32_t nx = P.n[0];
    const int32_t a0 = max(c[0] - M, 0), b0 = min(c[0] + M, nx - 1);
    int32_t a1 = 0, b1 = -1;
    T s1 = T(0);
    if (P.periodic[0]) {
        if (c[0] - M < 0) { a1 = c[0] - M + nx; b1 = nx - 1; s1 = -P.L[0]; }
        else if (c[0] + M >= nx) { a1 = 0; b1 = c[0] + M - nx; s1 = P.L[0]; }
    }
    const int32_t zr = D >= 3 ? 1 : 0, yr = D >= 2 ? 1 : 0;
#pragma unroll 1
    for (int32_t dz = -zr; dz <= zr; ++dz) {
#pragma unroll 1
        for (int32_t dy = -yr; dy <= yr; ++dy) {
            int32_t cz = 0, cy = 0;
            T sz = T(0), sy = T(0);
            const bool ez = D < 3 || wrap_cell(c[2] + dz, P.n[2], P.periodic[2], P.L[2], &cz, &sz);
            const bool ey = D < 2 || wrap_cell(c[1] + dy, P.n[1], P.periodic[1], P.L[1], &cy, &sy);
            const bool ex = ez && ey;
            const int row = (dz + zr) * (2 * yr + 1) + (dy + yr);
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
                if (staged) stage_window<T, D, G>(xs, ys, wb, lo, hi - lo, rank, nact);
            }
            if (ex) {
                begin(row);
                T sh[3] = {T(0), sy, sz};
                if (staged) win(jm0, jm1, sh, wb, lo);
                else piece(jm0, jm1, sh);
                if (b1 >= a1) {
                    sh[0] = s1;
                    piece(off[rowbase + a1], min(off[rowbase + b1 + 1], n), sh);
                }
                end(row);
            }
        }
    }
}

// MODE 0: forward sum + record.  MODE 1: adjoint from the record (gy_s gathered
// into cell order, rows padded as gradient rows).
template <typename T, int D, int OP, bool BATCH, bool OFF32, int MODE>
__global__ __launch_bounds__(256) void k_lane_mask(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                   const SysParams<T>* __restrict__ sp,
                                                   const uint32_t* __restrict__ sys_part, int nsys,
                                                   const T* __restrict__ a_s, const T* __restrict__ gy_s,
                                                   OpArgs<T> q, T* __restrict__ y, T* __restrict__ gx,
                                                   T* __restrict__ ga, uint32_t* __restrict__ masks,
                                                   uint32_t* __restrict__ status, const uint32_t* __restrict__ gen) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int PITCH = Pitch<D>::value;
    constexpr int GP = GyPitch<NY>::value;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    const T r = P.r, r2 = P.r2;
    if constexpr (MODE == 0) {
        T acc[NY];
#pragma unroll
        for (int k = 0; k < NY; ++k) acc[k] = T(0);
        bool overflow = false;
        auto visit = [&](uint32_t j, const T* dx, T d2) {
            const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
            Op::fwd(q, r, dx, d2, ai, aj, acc);
        };
        // candidates [ja, jb): the summand of each accepted one, and its bit shifted
        // into rec from the bottom (the row's first candidate ends highest; the
        // record is bit-reversed when the row is done)
        auto scan = [&](auto shift_tag, uint32_t ja, uint32_t jb, const T* sh, uint64_t& rec) {
            constexpr bool SHIFT = decltype(shift_tag)::value;
            uint32_t j = ja;
            // float: four candidates per iteration keep four loads in flight (the
            // float64 kernel, with twice the registers per row, stays at two).
            // With 32-bit row offsets the loop runs on the first candidate's byte
            // offset, the other three loads take immediate offsets from the same
            // address, and the four bits enter the record as two 32-bit halves.
            if constexpr (sizeof(T) == 4 && OFF32) {
                constexpr uint32_t RB = (uint32_t)sizeof(VecN<T, PITCH>);
                const char* const xrow = reinterpret_cast<const char*>(xs);
                const uint32_t oend = jb * RB;
                const uint32_t olast = oend >= 3u * RB ? oend - 3u * RB : 0u;
                uint32_t o = ja * RB;
                uint32_t lo = (uint32_t)rec, hi = (uint32_t)(rec >> 32);
                for (; o < olast; o += 4u * RB) {
                    const char* const pj = xrow + (size_t)o;
                    const VecN<T, PITCH> xa = *reinterpret_cast<const VecN<T, PITCH>*>(pj);
                    const VecN<T, PITCH> xb = *reinterpret_cast<const VecN<T, PITCH>*>(pj + RB);
                    const VecN<T, PITCH> xc = *reinterpret_cast<const VecN<T, PITCH>*>(pj + 2u * RB);
                    const VecN<T, PITCH> xd = *reinterpret_cast<const VecN<T, PITCH>*>(pj + 3u * RB);
                    const uint32_t jj = o / RB;
                    // the record moves up four places first; each accepted candidate
                    // then sets its bit inside the branch that adds its summand
                    hi = (hi << 4) | (lo >> 28);
                    lo <<= 4;
                    T dx[D], d2;
                    if (pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2)) {
                        visit(jj, dx, d2);
                        lo |= 8u;
                    }
                    if (pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2)) {
                        visit(jj + 1, dx, d2);
                        lo |= 4u;
                    }
                    if (pair_test<T, D, SHIFT>(xc.v, xi, sh, r2, dx, &d2)) {
                        visit(jj + 2, dx, d2);
                        lo |= 2u;
                    }
                    if (pair_test<T, D, SHIFT>(xd.v, xi, sh, r2, dx, &d2)) {
                        visit(jj + 3, dx, d2);
                        lo |= 1u;
                    }
                }
                rec = ((uint64_t)hi << 32) | lo;
                j = o / RB;
            }
            for (; sizeof(T) == 4 && !OFF32 && j + 3 < jb; j += 4) {
                const VecN<T, PITCH> xa = load_row<T, PITCH, OFF32>(xs, j);
                const VecN<T, PITCH> xb = load_row<T, PITCH, OFF32>(xs, j + 1);
                const VecN<T, PITCH> xc = load_row<T, PITCH, OFF32>(xs, j + 2);
                const VecN<T, PITCH> xd = load_row<T, PITCH, OFF32>(xs, j + 3);
                T dx[D], d2;
                const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                if (oa) visit(j, dx, d2);
                const bool ob = pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2);
                if (ob) visit(j + 1, dx, d2);
                const bool oc = pair_test<T, D, SHIFT>(xc.v, xi, sh, r2, dx, &d2);
                if (oc) visit(j + 2, dx, d2);
                const bool od = pair_test<T, D, SHIFT>(xd.v, xi, sh, r2, dx, &d2);
                if (od) visit(j + 3, dx, d2);
                rec = (rec << 4) | (oa ? 8u : 0u) | (ob ? 4u : 0u) | (oc ? 2u : 0u) | (od ? 1u : 0u);
            }
            for (; j + 1 < jb; j += 2) {
                const VecN<T, PITCH> xa = load_row<T, PITCH, OFF32>(xs, j);
                const VecN<T, PITCH> xb = load_row_at<T, PITCH, OFF32>(xs, j, 1);
                T dx[D], d2;
                const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                if (oa) visit(j, dx, d2);
                const bool ob = pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2);
                if (ob) visit(j + 1, dx, d2);
                rec = (rec << 2) | (oa ? 2u : 0u) | (ob ? 1u : 0u);
            }
            if (j < jb) {
                const VecN<T, PITCH> xa = load_row<T, PITCH, OFF32>(xs, j);
                T dx[D], d2;
                const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                if (oa) visit(j, dx, d2);
                rec = (rec << 1) | (oa ? 1u : 0u);
            }
        };
        // candidates [ja, jb) as scan takes them, read from the wave's LDS window
        // that holds slots [lo, lo + kWindow) (byte offsets from the window start).
        // An empty run may lie outside the window (its offsets would wrap), so it
        // returns at once.
        auto scan_window = [&](auto shift_tag, uint32_t ja, uint32_t jb, const T* sh, uint64_t& rec,
                               const char* wb, uint32_t lo) {
            constexpr bool SHIFT = decltype(shift_tag)::value;
            constexpr uint32_t RB = (uint32_t)sizeof(VecN<T, PITCH>);
            if (jb <= ja) return;
            const uint32_t oend = (jb - lo) * RB;
            const uint32_t olast = oend >= 3u * RB ? oend - 3u * RB : 0u;
            uint32_t o = (ja - lo) * RB;
            uint32_t rlo = (uint32_t)rec, rhi = (uint32_t)(rec >> 32);
            for (; o < olast; o += 4u * RB) {
                const char* const pj = wb + o;
                const VecN<T, PITCH> xa = *reinterpret_cast<const VecN<T, PITCH>*>(pj);
                const VecN<T, PITCH> xb = *reinterpret_cast<const VecN<T, PITCH>*>(pj + RB);
                const VecN<T, PITCH> xc = *reinterpret_cast<const VecN<T, PITCH>*>(pj + 2u * RB);
                const VecN<T, PITCH> xd = *reinterpret_cast<const VecN<T, PITCH>*>(pj + 3u * RB);
                const uint32_t jj = lo + o / RB;
                // the record moves up four places first; each accepted candidate then
                // sets its bit inside the branch that adds its summand
                rhi = (rhi << 4) | (rlo >> 28);
                rlo <<= 4;
                T dx[D], d2;
                if (pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2)) {
                    visit(jj, dx, d2);
                    rlo |= 8u;
                }
                if (pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2)) {
                    visit(jj + 1, dx, d2);
                    rlo |= 4u;
                }
                if (pair_test<T, D, SHIFT>(xc.v, xi, sh, r2, dx, &d2)) {
                    visit(jj + 2, dx, d2);
                    rlo |= 2u;
                }
                if (pair_test<T, D, SHIFT>(xd.v, xi, sh, r2, dx, &d2)) {
                    visit(jj + 3, dx, d2);
                    rlo |= 1u;
                }
            }
            rec = ((uint64_t)rhi << 32) | rlo;
            for (; o + RB < oend; o += 2u * RB) {
                const VecN<T, PITCH> xa = *reinterpret_cast<const VecN<T, PITCH>*>(wb + o);
                const VecN<T, PITCH> xb = *reinterpret_cast<const VecN<T, PITCH>*>(wb + o + RB);
                const uint32_t jj = lo + o / RB;
                T dx[D], d2;
                const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                if (oa) visit(jj, dx, d2);
                const bool ob = pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2);
                if (ob) visit(jj + 1, dx, d2);
                rec = (rec << 2) | (oa ? 2u : 0u) | (ob ? 1u : 0u);
            }
            if (o < oend) {
                const VecN<T, PITCH> xa = *reinterpret_cast<const VecN<T, PITCH>*>(wb + o);
                T dx[D], d2;
                const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                if (oa) visit(lo + o / RB, dx, d2);
                rec = (rec << 1) | (oa ? 1u : 0u);
            }
        };
        uint64_t rec = 0;  // the current row's bits, most recent lowest
        uint32_t pos = 0;  // candidates of the current row so far
        auto begin_row = [&](int) {
            rec = 0;
            pos = 0;
        };
        auto piece = [&](uint32_t j0, uint32_t j1, const T* sh) {
            bool lane_shift = false;
#pragma unroll
            for (int k = 0; k < D; ++k) lane_shift |= sh[k] != T(0);
            j1 = max(j1, j0);
            if (__ballot(lane_shift) != 0ull) scan(std::integral_constant<bool, true>(), j0, j1, sh, rec);
            else scan(std::integral_constant<bool, false>(), j0, j1, sh, rec);
            pos += j1 - j0;
        };
        auto end_row = [&](int row) {
            overflow |= pos > (uint32_t)kMaskBits;
            // c <= 64 bits shifted in put row position k at bit c - 1 - k;
            // reversed and shifted down by 64 - c it lands at bit k
            const uint32_t c = min(pos, (uint32_t)kMaskBits);
            const uint64_t rev = ((uint64_t)__builtin_bitreverse32((uint32_t)rec) << 32) |
                                 __builtin_bitreverse32((uint32_t)(rec >> 32));
            const uint64_t m = c == 0u ? 0ull : rev >> (64u - c);
            masks[(size_t)(2 * row) * n + s] = (uint32_t)m;
            masks[(size_t)(2 * row + 1) * n + s] = (uint32_t)(m >> 32);
        };
        if constexpr (sizeof(T) == 4 && OFF32) {
            if (__ballot(P.n[0] < 2 * P.reach[0] + 1) == 0ull) {
                // Every grid of the wave is at least 2 m + 1 cells wide: each row's main
                // runs are staged in LDS (below); otherwise the plain walk.
                __shared__ VecN<T, PITCH> win[kBlockWaves][kWindow];
                auto win_piece = [&](uint32_t j0, uint32_t j1, const T* sh, const char* wb, uint32_t lo) {
                    j1 = max(j1, j0);
                    if (__ballot(sh[1] != T(0) || sh[2] != T(0)) != 0ull)
                        scan_window(std::integral_constant<bool, true>(), j0, j1, sh, rec, wb, lo);
                    else
                        scan_window(std::integral_constant<bool, false>(), j0, j1, sh, rec, wb, lo);
                    pos += j1 - j0;
                };
                staged_rows<T, D, 0>(P, off, n, xi, xs, nullptr, reinterpret_cast<char*>(&win[threadIdx.x >> 6][0]),
                                     begin_row, piece, end_row, win_piece);
            } else {
                for_each_piece<T, D>(P, off, n, xi, begin_row, piece, end_row);
            }
        } else {
            for_each_piece<T, D>(P, off, n, xi, begin_row, piece, end_row);
        }
        status[s] = overflow ? kGenNone : gen[0];
        const uint32_t o = perm[s];
#pragma unroll
        for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k];
    } else {
        T gyi[NY];
        load_gy<T, NY, OFF32>(gy_s, s, gyi);
        T accx[D], acca[1] = {T(0)};
#pragma unroll
        for (int k = 0; k < D; ++k) accx[k] = T(0);
        auto pair = [&](uint32_t j, const T* dx, T d2, const T* gyj) {
            const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
            Op::bwd(q, r, dx, d2, ai, aj, gyi, gyj, accx, acca);
        };
        // the accepted pairs of one piece, bits64 bit k = its k-th slot from j0: popped
        // three per iteration (their loads overlap), each 32-bit half of the piece's
        // record in turn (one-word bit operations), from HBM or, with WIN, from the
        // wave's LDS window, whose xs rows for slots [lo, lo + kWindow) are followed
        // by the gy rows of the same slots
        auto replay_s = [&](auto win_tag, auto shift_tag, uint32_t j0, uint64_t bits64, const T* sh, const char* wb,
                            uint32_t lo) {
            constexpr bool WIN = decltype(win_tag)::value;
            constexpr bool SHIFT = decltype(shift_tag)::value;
            constexpr uint32_t RBX = (uint32_t)sizeof(VecN<T, PITCH>), RBG = (uint32_t)sizeof(VecN<T, GP>);
#pragma unroll 1
            for (uint32_t h = 0; h < 2u; ++h) {
                uint32_t bits = h ? (uint32_t)(bits64 >> 32) : (uint32_t)bits64;
                const uint32_t base = j0 + 32u * h;
                // rows of the half's bit k: slot base + k, at window row base - lo + k
                // (the window addresses of bit 0 formed once per half)
                const char* const px = wb + (base - lo) * RBX;
                const char* const pg = wb + (uint32_t)kWindow * RBX + (base - lo) * RBG;
                auto ldx = [&](uint32_t k) {
                    if constexpr (WIN) return *reinterpret_cast<const VecN<T, PITCH>*>(px + k * RBX);
                    else return load_row<T, PITCH, OFF32>(xs, base + k);
                };
                auto ldg = [&](uint32_t k) {
                    if constexpr (WIN) return *reinterpret_cast<const VecN<T, GP>*>(pg + k * RBG);
                    else return load_row<T, GP, OFF32>(gy_s, base + k);
                };
                while (bits != 0u) {
                    const uint32_t ka = (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1u;
                    const bool vb = bits != 0u;
                    const uint32_t kb = vb ? (uint32_t)__builtin_ctz(bits) : ka;
                    bits &= bits - 1u;
                    const bool vc = bits != 0u;
                    const uint32_t kc = vc ? (uint32_t)__builtin_ctz(bits) : ka;
                    bits &= bits - 1u;
                    const VecN<T, PITCH> xa = ldx(ka);
                    const VecN<T, GP> ga_ = ldg(ka);
                    const VecN<T, PITCH> xb = ldx(kb);
                    const VecN<T, GP> gb_ = ldg(kb);
                    const VecN<T, PITCH> xc = ldx(kc);
                    const VecN<T, GP> gc_ = ldg(kc);
                    T dx[D], d2;
                    (void)pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
                    pair(base + ka, dx, d2, ga_.v);
                    keep_issued<D>(xb.v);
                    keep_issued<NY>(gb_.v);
                    keep_issued<D>(xc.v);
                    keep_issued<NY>(gc_.v);
                    if (vb) {
                        (void)pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2);
                        pair(base + kb, dx, d2, gb_.v);
                    }
                    if (vc) {
                        (void)pair_test<T, D, SHIFT>(xc.v, xi, sh, r2, dx, &d2);
                        pair(base + kc, dx, d2, gc_.v);
                    }
                }
            }
        };
        // the image shift's adds only where some lane of the wave needs them
        auto replay = [&](auto win_tag, uint32_t j0, uint64_t bits64, const T* sh, const char* wb, uint32_t lo) {
            bool lane_shift = false;
#pragma unroll
            for (int k = 0; k < D; ++k) lane_shift |= sh[k] != T(0);
            if (__ballot(lane_shift) != 0ull)
                replay_s(win_tag, std::integral_constant<bool, true>(), j0, bits64, sh, wb, lo);
            else
                replay_s(win_tag, std::integral_constant<bool, false>(), j0, bits64, sh, wb, lo);
        };
        if (status[s] == gen[0]) {
            uint64_t m = 0;    // the current row's record
            uint32_t pos = 0;  // row position of the next piece's first candidate
            auto begin_row = [&](int row) {
                m = (uint64_t)masks[(size_t)(2 * row) * n + s] | ((uint64_t)masks[(size_t)(2 * row + 1) * n + s] << 32);
                pos = 0;
            };
            // the record's bits of the piece [j0, j1) (a piece past 64 candidates keeps none)
            auto piece_bits = [&](uint32_t j0, uint32_t j1) {
                const uint32_t len = j1 > j0 ? j1 - j0 : 0u;
                uint64_t bits = pos < 64u ? m >> pos : 0ull;
                if (len < 64u) bits &= (1ull << len) - 1ull;
                pos += len;
                return bits;
            };
            auto piece = [&](uint32_t j0, uint32_t j1, const T* sh) {
                const uint64_t bits = piece_bits(j0, j1);
                replay(std::integral_constant<bool, false>(), j0, bits, sh, nullptr, 0u);
            };
            auto end_row = [&](int) {};
            if constexpr (sizeof(T) == 4 && OFF32) {
                if (__ballot(P.n[0] < 2 * P.reach[0] + 1) == 0ull) {
                    // as in the forward: each row's main runs from the wave's LDS window
                    // (positions, then the gy rows)
                    constexpr int kWinRows = kWindow * (int)(sizeof(VecN<T, PITCH>) + sizeof(VecN<T, GP>)) /
                                             (int)sizeof(VecN<T, 4>);
                    __shared__ VecN<T, 4> win[kBlockWaves][kWinRows];
                    staged_rows<T, D, GP>(P, off, n, xi, xs, gy_s, reinterpret_cast<char*>(&win[threadIdx.x >> 6][0]),
                                          begin_row, piece, end_row,
                                          [&](uint32_t j0, uint32_t j1, const T* sh, const char* wb, uint32_t lo) {
                                              const uint64_t bits = piece_bits(j0, j1);
                                              replay(std::integral_constant<bool, true>(), j0, bits, sh, wb, lo);
                                          });
                } else {
                    for_each_piece<T, D>(P, off, n, xi, begin_row, piece, end_row);
                }
            } else {
                for_each_piece<T, D>(P, off, n, xi, begin_row, piece, end_row);
            }
        } else {
            // no record: the plain row search (not its deferred form, whose
            // registers would lower the replay's occupancy)
            auto visit = [&](uint32_t j, const T* dx, T d2, bool) {
                const VecN<T, GP> gj = load_row<T, GP, OFF32>(gy_s, j);
                pair(j, dx, d2, gj.v);
            };
            neighbour_loop<T, D, OFF32>(P, xs, off, n, xi, visit);
        }
        const uint32_t o = perm[s];
#pragma unroll
        for (int k = 0; k < D; ++k) gx[(size_t)o * D + k] = accx[k];
        if (OpShape<OP, D>::NA && ga) ga[o] = acca[0];
    }
}

// ---------------------------------------------------------------------------
// Half stencil (Newton's third law for the pair test).  The pair test is
// symmetric bit for bit: a partner's dx is fl(x_i - x_j) + s = -(fl(x_j - x_i)
// + (-s)), so d2 and the decision are the same from both ends.  Each unordered
// pair is therefore tested once:
//   k_half_upper  lane i tests the upper half of its stencil -- the rows with
//                 dz > 0, or dz = 0 and dy > 0, and the part of its own row
//                 ahead of it (its own cell's later slots and the cells after
//                 it along x, including a forward wrap) -- adds those summands
//                 into a partial sum (cell order) and records the rows' bits as
//                 the recording forward does (a row over kMaskBits candidates
//                 records all ones);
//   k_half_mirror lane j walks the lower half cell by cell; for each
//                 candidate i it reads the bit that i's upper row holds at
//                 j's position (computed from i's cell), and for a set bit
//                 (or a position beyond the record) runs the pair test and the
//                 summand in j's frame, exactly as the full-stencil forward
//                 would; then adds the partial sum.
// The summands are those of the full-stencil kernels; the sum runs lower half
// first, then the partial, so it differs from them by rounding order only.
// Requires reach 1 in y and z and a grid at least 2 m + 1 cells wide in x.
// The records it leaves are not full-stencil records (status none).
template <typename T, int D, int OP, bool BATCH, bool OFF32>
__global__ __launch_bounds__(256) void k_half_upper(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                    uint32_t n, const SysParams<T>* __restrict__ sp,
                                                    const uint32_t* __restrict__ sys_part, int nsys,
                                                    const T* __restrict__ a_s, OpArgs<T> q, T* __restrict__ yh,
                                                    uint32_t* __restrict__ masks, uint32_t* __restrict__ status) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int PITCH = Pitch<D>::value;
    constexpr int NR = D == 1 ? 1 : (D == 2 ? 3 : 9);
    constexpr int C = NR / 2;  // the particle's own row
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xi[D];
    load_point<T, D>(xs, s, xi);
    const T ai = OpShape<OP, D>::NA ? a_s[s] : T(0);
    const T r = P.r, r2 = P.r2;
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    auto visit = [&](uint32_t j, const T* dx, T d2) {
        const T aj = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, j).v[0] : T(0);
        Op::fwd(q, r, dx, d2, ai, aj, acc);
    };
    // candidates [ja, jb) as the recording forward scans them: two per iteration,
    // each bit shifted into rec from the bottom
    auto scan_s = [&](auto shift_tag, uint32_t ja, uint32_t jb, const T* sh, uint64_t& rec) {
        constexpr bool SHIFT = decltype(shift_tag)::value;
        uint32_t j = ja;
        for (; j + 1 < jb; j += 2) {
            const VecN<T, PITCH> xa = load_row<T, PITCH, OFF32>(xs, j);
            const VecN<T, PITCH> xb = load_row_at<T, PITCH, OFF32>(xs, j, 1);
            T dx[D], d2;
            const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
            if (oa) visit(j, dx, d2);
            const bool ob = pair_test<T, D, SHIFT>(xb.v, xi, sh, r2, dx, &d2);
            if (ob) visit(j + 1, dx, d2);
            rec = (rec << 2) | (oa ? 2u : 0u) | (ob ? 1u : 0u);
        }
        if (j < jb) {
            const VecN<T, PITCH> xa = load_row<T, PITCH, OFF32>(xs, j);
            T dx[D], d2;
            const bool oa = pair_test<T, D, SHIFT>(xa.v, xi, sh, r2, dx, &d2);
            if (oa) visit(j, dx, d2);
            rec = (rec << 1) | (oa ? 1u : 0u);
        }
    };
    auto scan = [&](uint32_t ja, uint32_t jb, const T* sh, uint64_t& rec) {
        bool lane_shift = false;
#pragma unroll
        for (int k = 0; k < D; ++k) lane_shift |= sh[k] != T(0);
        // the image shift's adds only where some lane of the wave needs them
        if (__ballot(lane_shift) != 0ull) scan_s(std::integral_constant<bool, true>(), ja, jb, sh, rec);
        else scan_s(std::integral_constant<bool, false>(), ja, jb, sh, rec);
    };
    uint64_t rec = 0;
    uint32_t pos = 0;
    int cur = 0;
    for_each_piece<T, D>(
        P, off, n, xi,
        [&](int row) {
            rec = 0;
            pos = 0;
            cur = row;
        },
        [&](uint32_t j0, uint32_t j1, const T* sh) {
            if (cur < C) return;
            j1 = max(j1, j0);
            const uint32_t len = j1 - j0;
            if (cur == C) {
                if (sh[0] == T(0)) {  // the main run: its slots after s are ahead
                    scan(min(max(s + 1u, j0), j1), j1, sh, rec);
                    pos += len;
                    return;
                }
                if (sh[0] < T(0)) {  // a backward wrap: all behind (zeros keep the positions)
                    rec = len >= 64u ? 0ull : (rec << len);
                    pos += len;
                    return;
                }
            }
            scan(j0, j1, sh, rec);
            pos += len;
        },
        [&](int row) {
            if (row < C) return;
            uint64_t m;
            if (pos > (uint32_t)kMaskBits) {
                m = ~0ull;  // positions past the record: the mirror pass tests every candidate
            } else {
                const uint64_t rev = ((uint64_t)__builtin_bitreverse32((uint32_t)rec) << 32) |
                                     __builtin_bitreverse32((uint32_t)(rec >> 32));
                m = pos == 0u ? 0ull : rev >> (64u - pos);
            }
            masks[(size_t)(2 * row) * n + s] = (uint32_t)m;
            masks[(size_t)(2 * row + 1) * n + s] = (uint32_t)(m >> 32);
        });
    status[s] = kGenNone;  // not a full-stencil record: a replaying adjoint tests instead
#pragma unroll
    for (int k = 0; k < NY; ++k) yh[(size_t)s * 4 + k] = acc[k];
}

template <typename T, int D, int OP, bool BATCH, bool OFF32>
__global__ __launch_bounds__(256) void k_half_mirror(const T* __restrict__ xs, const uint32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ perm, uint32_t n,
                                                     const SysParams<T>* __restrict__ sp,
                                                     const uint32_t* __restrict__ sys_part, int nsys,
                                                     const T* __restrict__ a_s, OpArgs<T> q,
                                                     const T* __restrict__ yh, const uint32_t* __restrict__ masks,
                                                     T* __restrict__ y) {
    using Op = PairOp<T, D, OP>;
    constexpr int NY = Op::NY;
    constexpr int PITCH = Pitch<D>::value;
    constexpr int NR = D == 1 ? 1 : (D == 2 ? 3 : 9);
    constexpr int C = NR / 2;
    const uint32_t first = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
    const uint32_t s = first + threadIdx.x;
    const int b = system_of_row<BATCH>(sys_part, nsys, first, s);
    if (s >= n) return;
    const SysParams<T> P = sp[b];
    T xj[D];
    load_point<T, D>(xs, s, xj);
    const T aj = OpShape<OP, D>::NA ? a_s[s] : T(0);
    const T r = P.r, r2 = P.r2;
    T acc[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) acc[k] = T(0);
    int32_t c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T fr;
        c[k] = cell_coord(P, k, xj[k], &fr);
    }
    const int32_t M = P.reach[0];
    const int32_t nx = P.n[0];
    const int32_t zr = D >= 3 ? 1 : 0, yr = D >= 2 ? 1 : 0;
    // this particle's own x-row: the row of every partner's upper stencil row that reaches it
    const uint32_t rb_own = P.cell_base + (uint32_t)nx * ((uint32_t)c[1] + (uint32_t)P.n[1] * (uint32_t)c[2]);
#pragma unroll 1
    for (int32_t dz = -zr; dz <= 0; ++dz) {
        int32_t cz = 0;
        T sz = T(0);
        if (D >= 3 && !wrap_cell(c[2] + dz, P.n[2], P.periodic[2], P.L[2], &cz, &sz)) continue;
#pragma unroll 1
        for (int32_t dy = -yr; dy <= yr; ++dy) {
            const int row = (dz + zr) * (2 * yr + 1) + (dy + yr);
            if (row > C) break;  // the upper half belongs to k_half_upper
            int32_t cy = 0;
            T sy = T(0);
            if (D >= 2 && !wrap_cell(c[1] + dy, P.n[1], P.periodic[1], P.L[1], &cy, &sy)) continue;
            const int hr = NR - 1 - row;  // the partners' row that covers this particle's x-row
            const uint32_t rb = P.cell_base + (uint32_t)nx * ((uint32_t)cy + (uint32_t)P.n[1] * (uint32_t)cz);
            const int32_t o_end = row == C ? 0 : M;
#pragma unroll 1
            for (int32_t o = -M; o <= o_end; ++o) {
                int32_t cx;
                T sx = T(0);
                if (!wrap_cell(c[0] + o, nx, P.periodic[0], P.L[0], &cx, &sx)) continue;
                const uint32_t i0 = off[rb + cx];
                uint32_t i1 = min(off[rb + cx + 1], n);
                if (row == C && o == 0) i1 = min(i1, s);  // own cell: the slots before s
                if (i1 <= i0) continue;
                // position of this particle in the row hr of a partner in cell cx: that
                // row's main run starts at cell max(cx - M, 0) of the own x-row, its
                // wrapped remainder (if any) follows it
                const int32_t a0 = max(cx - M, 0), b0 = min(cx + M, nx - 1);
                uint32_t pos;
                if (c[0] >= a0 && c[0] <= b0) {
                    pos = s - off[rb_own + a0];
                } else {
                    const int32_t a1 = cx - M < 0 ? cx - M + nx : 0;
                    pos = (min(off[rb_own + b0 + 1], n) - off[rb_own + a0]) + (s - off[rb_own + a1]);
                }
                const T sh[3] = {sx, sy, sz};
                const size_t wrow = (size_t)(2 * hr + (pos >= 32u ? 1 : 0)) * n;
                const uint32_t bit = pos & 31u;
                auto pair = [&](uint32_t i) {
                    const VecN<T, PITCH> xi = load_row<T, PITCH, OFF32>(xs, i);
                    T dx[D], d2;
                    if (pair_test<T, D, true>(xi.v, xj, sh, r2, dx, &d2)) {
                        const T ai = OpShape<OP, D>::NA ? load_row<T, 1, OFF32>(a_s, i).v[0] : T(0);
                        Op::fwd(q, r, dx, d2, aj, ai, acc);
                    }
                };
                const bool all = pos >= (uint32_t)kMaskBits;  // past the record: test every candidate
                uint32_t i = i0;
                for (; i + 1 < i1; i += 2) {  // two partners' bits per iteration, their loads together
                    const uint32_t wa = all ? 1u : masks[wrow + i] >> bit;
                    const uint32_t wb = all ? 1u : masks[wrow + i + 1] >> bit;
                    if (wa & 1u) pair(i);
                    if (wb & 1u) pair(i + 1);
                }
                if (i < i1 && (all || ((masks[wrow + i] >> bit) & 1u))) pair(i);
            }
        }
    }
    const uint32_t o = perm[s];
#pragma unroll
    for (int k = 0; k < NY; ++k) y[(size_t)o * NY + k] = acc[k] + yh[(size_t)s * 4 + k];
}

template <typename T, int D, int OP, bool BATCH>
void launch_half_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + 255) / 256);
    T* yh = reinterpret_cast<T*>(c->work2);  // [n][4] partial sums in cell order
    if (off32_rows<T>(n)) {
        hipLaunchKernelGGL((k_half_upper<T, D, OP, BATCH, true>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, n, sp, c->sys_part_dev, c->nsys, a_s, q, yh, c->masks, c->mask_status);
        hipLaunchKernelGGL((k_half_mirror<T, D, OP, BATCH, true>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, (const T*)yh, c->masks, y);
    } else {
        hipLaunchKernelGGL((k_half_upper<T, D, OP, BATCH, false>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, n, sp, c->sys_part_dev, c->nsys, a_s, q, yh, c->masks, c->mask_status);
        hipLaunchKernelGGL((k_half_mirror<T, D, OP, BATCH, false>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, q, (const T*)yh, c->masks, y);
    }
}

template <typename T, int D, int OP, bool BATCH>
void launch_mask_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + 255) / 256);
    if (off32_rows<T>(n))
        hipLaunchKernelGGL((k_lane_mask<T, D, OP, BATCH, true, 0>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, nullptr, q, y, nullptr, nullptr,
                           c->masks, c->mask_status, c->gen);
    else
        hipLaunchKernelGGL((k_lane_mask<T, D, OP, BATCH, false, 0>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, nullptr, q, y, nullptr, nullptr,
                           c->masks, c->mask_status, c->gen);
}

template <typename T, int D, int OP, bool BATCH>
void launch_mask_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                     T* ga) {
    const uint32_t n = (uint32_t)c->n;
    const SysParams<T>* sp = reinterpret_cast<const SysParams<T>*>(c->params_dev);
    const dim3 grid((n + 255) / 256);
    if (off32_rows<T>(n))
        hipLaunchKernelGGL((k_lane_mask<T, D, OP, BATCH, true, 1>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, nullptr, gx, ga,
                           c->masks, c->mask_status, c->gen);
    else
        hipLaunchKernelGGL((k_lane_mask<T, D, OP, BATCH, false, 1>), grid, dim3(256), 0, ctx->stream, (const T*)c->xs,
                           c->off, c->perm, n, sp, c->sys_part_dev, c->nsys, a_s, gy_s, q, nullptr, gx, ga,
                           c->masks, c->mask_status, c->gen);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                          \
    template void launch_mask_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&,        \
                                                   const T*, T*);                                             \
    template void launch_half_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&,        \
                                                   const T*, T*);                                             \
    template void launch_mask_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&,        \
                                                   const T*, const T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
