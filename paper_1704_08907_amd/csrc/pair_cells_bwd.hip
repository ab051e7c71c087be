// Cell-group neighbour-sum adjoint (instantiations).
#include "pair_cells.hpp"

namespace aboria {

template <typename T, int D, int OP, bool BATCH>
void launch_cells_bwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, const T* gy_s, T* gx,
                      T* ga, int rounds) {
    if (rounds > 1) launch_cells_impl<T, D, OP, BATCH, true, 8>(ctx, c, q, a_s, gy_s, gx, ga);
    else launch_cells_impl<T, D, OP, BATCH, true, 1>(ctx, c, q, a_s, gy_s, gx, ga);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                         \
    template void launch_cells_bwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, const T*, \
                                                    const T*, T*, T*, int);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
