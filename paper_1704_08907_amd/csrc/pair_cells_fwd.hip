// Cell-group neighbour-sum forward (instantiations).
#include "pair_cells.hpp"

namespace aboria {

template <typename T, int D, int OP, bool BATCH>
void launch_cells_fwd(aboria_ctx* ctx, const aboria_cells* c, const OpArgs<T>& q, const T* a_s, T* y, int rounds) {
    if (rounds > 1) launch_cells_impl<T, D, OP, BATCH, false, 8>(ctx, c, q, a_s, nullptr, y, nullptr);
    else launch_cells_impl<T, D, OP, BATCH, false, 1>(ctx, c, q, a_s, nullptr, y, nullptr);
}

#define ABORIA_INST(T, D, OP, BATCH)                                                                    \
    template void launch_cells_fwd<T, D, OP, BATCH>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, \
                                                    const T*, T*, int);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
