// Backward raster instantiated for the MLP shape (32, 64, 2) and 16x16 tiles.
#include "raster_bwd_impl.hpp"

namespace soup {

void launch_raster_bwd_k32_64_2_t16(const BwdArgs& a, bool logp, hipStream_t s) {
    launch_bwd_t<16, MlpShape<32, 64, 2>>(a, logp, s);
}

}  // namespace soup
