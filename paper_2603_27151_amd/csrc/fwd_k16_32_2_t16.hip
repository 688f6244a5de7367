// Forward raster instantiated for the MLP shape (16, 32, 2) and 16x16 tiles.
#include "raster_fwd_impl.hpp"

namespace soup {

void launch_raster_fwd_k16_32_2_t16(const RasterArgs& a, hipStream_t s) { launch_fwd_t<16, MlpShape<16, 32, 2>>(a, s); }
int raster_fwd_per_cu_k16_32_2_t16(int region) { return fwd_blocks_per_cu<16, MlpShape<16, 32, 2>>(region); }

}  // namespace soup
