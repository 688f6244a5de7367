// Forward raster instantiated for the MLP shape (32, 64, 2) and 16x16 tiles.
#include "raster_fwd_impl.hpp"

namespace soup {

void launch_raster_fwd_k32_64_2_t16(const RasterArgs& a, hipStream_t s) { launch_fwd_t<16, MlpShape<32, 64, 2>>(a, s); }
int raster_fwd_per_cu_k32_64_2_t16(int region) { return fwd_blocks_per_cu<16, MlpShape<32, 64, 2>>(region); }

}  // namespace soup
