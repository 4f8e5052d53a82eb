// Per-kernel-size entry points of the tiled kernels.  Each kernel size is compiled in
// its own translation unit (tile_inst.hip with DIA_INST_M), tile_dispatch.cpp switches.
#pragma once

#include "dia_common.h"

namespace dia {

// Kernel sizes with every tile-shape variant compiled (the others have the default only).
template <int M>
struct HasVariants {
    static constexpr bool value = (M == 9 || M == 17 || M == 19 || M == 25);
};

// Column strips of variant 6 (two thread sets of one row): whole waves mostly full (2 waves at
// m = 9, 5 at m = 17 ... 25), tiles narrow enough that a small image still has a few hundred.
template <int M>
struct ShortStrips {
    static constexpr int value = M == 9 ? 7 : (M == 17 ? 9 : (M == 19 ? 8 : (M == 25 ? 6 : 8)));
};

// Variant v -> the Geo parameter for kernel size M: forward rows per thread requested (0 = automatic;
// variant 3 asks for 4), variant 4 two thread sets of one row, variant 5 the narrow shape with one
// row, variant 6 two thread sets of ShortStrips<M> strips, variants 7 and 8 one row with the kernel
// rows split over two halves of the threads, ShortStrips<M> strips or the narrow shape's.
template <int M>
constexpr int variant_rbv(int v) {
    return v == 1 ? 1
         : v == 2 ? 2
         : v == 3 ? 4
         : v == 4 ? 17
         : v == 5 ? 9
         : v == 6 ? 32 + ShortStrips<M>::value
         : v == 7 ? 64 + ShortStrips<M>::value
         : v == 8 ? 64 + ((64 / M) > 1 ? (64 / M) : 1)
         : 0;
}

template <int M>
struct TileOps {
    static hipError_t launch(int mode, int grid, const TileArgs& a, hipStream_t s, int v);
    static hipError_t launch_batched(int grid, const BatchedArgs& b, hipStream_t s, int v);
    static int occupancy(int v, bool batched);
};

#define DIA_FOR_EACH_M(X) \
    X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) \
    X(27) X(29) X(31) X(33) X(35) X(37) X(39) X(41) X(43) X(45) X(47) X(49)

}  // namespace dia
