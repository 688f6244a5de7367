// Backward raster instantiated for the MLP shape (16, 32, 2) and 8x8 tiles.
#include "raster_bwd_impl.hpp"

namespace soup {

void launch_raster_bwd_k16_32_2_t8(const BwdArgs& a, bool logp, hipStream_t s) {
    launch_bwd_t<8, MlpShape<16, 32, 2>>(a, logp, s);
}

}  // namespace soup
