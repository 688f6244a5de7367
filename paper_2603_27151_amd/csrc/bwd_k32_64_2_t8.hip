// Backward raster instantiated for the MLP shape (32, 64, 2) and 8x8 tiles.
#include "raster_bwd_impl.hpp"

namespace soup {

void launch_raster_bwd_k32_64_2_t8(const BwdArgs& a, bool logp, hipStream_t s) {
    launch_bwd_t<8, MlpShape<32, 64, 2>>(a, logp, s);
}

}  // namespace soup
