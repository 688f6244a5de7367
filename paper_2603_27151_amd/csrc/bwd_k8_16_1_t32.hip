// Backward raster instantiated for the MLP shape (8, 16, 1) and 32x32 tiles.
#include "raster_bwd_impl.hpp"

namespace soup {

void launch_raster_bwd_k8_16_1_t32(const BwdArgs& a, bool logp, hipStream_t s) {
    launch_bwd_t<32, MlpShape<8, 16, 1>>(a, logp, s);
}

}  // namespace soup
