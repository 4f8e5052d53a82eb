// Dispatch of the tiled kernels over the kernel size, and their tile geometry.
#include "tile_ops.h"
#include "hess_impl.h"

namespace dia {

#define X(MM) extern template struct TileOps<MM>;
DIA_FOR_EACH_M(X)
#undef X
#define X(MM) extern template struct HessOps<MM>;
DIA_FOR_EACH_M(X)
#undef X

template <int M>
static int variant_rb_m(int v) {
    if (v < 0 || v >= kNumVariants) return 0;
    if (v > 0 && !HasVariants<M>::value) return 0;
    switch (v) {
        case 0: return Geo<M, 0>::RB;
        case 1: return Geo<M, 1>::RB;
        case 2: return Geo<M, 2>::RB;
        case 3: return Geo<M, 4>::RB;
        case 4: return Geo<M, 17>::RB;
        case 6: return Geo<M, variant_rbv<M>(6)>::RB;
        case 7: return Geo<M, variant_rbv<M>(7)>::RB;
        case 8: return Geo<M, variant_rbv<M>(8)>::RB;
        default: return Geo<M, 9>::RB;
    }
}

// tile height and width of a compiled variant
template <int M>
static void variant_dims_m(int v, int* ty, int* tx) {
    switch (v) {
        case 0: *ty = Geo<M, 0>::TY, *tx = Geo<M, 0>::TX; break;
        case 1: *ty = Geo<M, 1>::TY, *tx = Geo<M, 1>::TX; break;
        case 2: *ty = Geo<M, 2>::TY, *tx = Geo<M, 2>::TX; break;
        case 3: *ty = Geo<M, 4>::TY, *tx = Geo<M, 4>::TX; break;
        case 4: *ty = Geo<M, 17>::TY, *tx = Geo<M, 17>::TX; break;
        case 6: *ty = Geo<M, variant_rbv<M>(6)>::TY, *tx = Geo<M, variant_rbv<M>(6)>::TX; break;
        case 7: *ty = Geo<M, variant_rbv<M>(7)>::TY, *tx = Geo<M, variant_rbv<M>(7)>::TX; break;
        case 8: *ty = Geo<M, variant_rbv<M>(8)>::TY, *tx = Geo<M, variant_rbv<M>(8)>::TX; break;
        default: *ty = Geo<M, 9>::TY, *tx = Geo<M, 9>::TX; break;
    }
}

int tile_variant_rb(int m, int variant) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return variant_rb_m<MM>(variant);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 0;
    }
}

int tile_dims(int m, int variant, int* ty, int* tx) {
    const int rb = tile_variant_rb(m, variant);
    if (rb == 0) return -1;
    switch (m) {
#define X(MM)                                   \
    case MM:                                    \
        variant_dims_m<MM>(variant, ty, tx);    \
        break;
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return -1;
    }
    return 0;
}

template <int M>
static int variant_sets_m(int v) {
    if (tile_variant_rb(M, v) == 0) return 0;
    switch (v) {
        case 0: return Geo<M, 0>::TS;
        case 1: return Geo<M, 1>::TS;
        case 2: return Geo<M, 2>::TS;
        case 3: return Geo<M, 4>::TS;
        case 4: return Geo<M, 17>::TS;
        case 6: return Geo<M, variant_rbv<M>(6)>::TS;
        case 7: return Geo<M, variant_rbv<M>(7)>::TS;
        case 8: return Geo<M, variant_rbv<M>(8)>::TS;
        default: return Geo<M, 9>::TS;
    }
}

int tile_variant_sets(int m, int variant) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return variant_sets_m<MM>(variant);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 0;
    }
}

template <int M>
static int variant_threads_m(int v) {
    if (tile_variant_rb(M, v) == 0) return 0;
    switch (v) {
        case 0: return Geo<M, 0>::NT;
        case 1: return Geo<M, 1>::NT;
        case 2: return Geo<M, 2>::NT;
        case 3: return Geo<M, 4>::NT;
        case 4: return Geo<M, 17>::NT;
        case 6: return Geo<M, variant_rbv<M>(6)>::NT;
        case 7: return Geo<M, variant_rbv<M>(7)>::NT;
        case 8: return Geo<M, variant_rbv<M>(8)>::NT;
        default: return Geo<M, 9>::NT;
    }
}

int tile_variant_threads(int m, int variant) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return variant_threads_m<MM>(variant);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 0;
    }
}

int tile_grid_tiles(int m, int rows, int cols, int variant) {
    int ty = 0, tx = 0;
    if (tile_dims(m, variant, &ty, &tx) != 0) return -1;
    const int Hv = rows - m + 1, Wv = cols - m + 1;
    return ((Hv + ty - 1) / ty) * ((Wv + tx - 1) / tx);
}

int tile_max_blocks_per_cu(int m, int variant, bool batched) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return TileOps<MM>::occupancy(variant, batched);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 1;
    }
}

hipError_t launch_tile(int mode, int m, int grid, const TileArgs& a, hipStream_t s, int variant) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return TileOps<MM>::launch(mode, grid, a, s, variant);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

int hess_pair_blocks(int m) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return HessOps<MM>::pair_blocks();
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 0;
    }
}

int hess_splits(int m, int rows, int cols) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return HessOps<MM>::splits(rows, cols);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 0;
    }
}

hipError_t launch_hess(int m, const HessArgs& a, hipStream_t s) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return HessOps<MM>::launch(a, s);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_batched_eval(int m, int grid, const BatchedArgs& b, hipStream_t s, int variant) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return TileOps<MM>::launch_batched(grid, b, s, variant);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace dia
