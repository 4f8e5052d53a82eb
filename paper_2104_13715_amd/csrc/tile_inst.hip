// Instantiates the tiled kernels for one kernel size (DIA_INST_M, set by the build).
#include "tile_impl.h"
#include "hess_impl.h"

#ifndef DIA_INST_M
#error "DIA_INST_M must be defined"
#endif

namespace dia {
template struct TileOps<DIA_INST_M>;
template struct HessOps<DIA_INST_M>;
}  // namespace dia
