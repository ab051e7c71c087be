// Instances of the flattened-search neighbour-sum kernel: mode fused.
#include "pair_flat.hpp"

namespace aboria {

#define ABORIA_INST(T, D, OP, BATCH)                                                                          \
    template void launch_flat<T, D, OP, BATCH, kFlatFused>(aboria_ctx*, const aboria_cells*, const OpArgs<T>&, \
                                                          const T*, const T*, T*, T*, T*);
ABORIA_FOR_EACH_PAIR_INSTANCE(ABORIA_INST)
#undef ABORIA_INST

}  // namespace aboria
