// Forward raster instantiated for the MLP shape (8, 16, 1) and 32x32 tiles.
#include "raster_fwd_impl.hpp"

namespace soup {

void launch_raster_fwd_k8_16_1_t32(const RasterArgs& a, hipStream_t s) { launch_fwd_t<32, MlpShape<8, 16, 1>>(a, s); }
int raster_fwd_per_cu_k8_16_1_t32(int region) { return fwd_blocks_per_cu<32, MlpShape<8, 16, 1>>(region); }

}  // namespace soup
