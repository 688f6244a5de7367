// Forward raster instantiated for the paper form (opacity texture only) and 16x16 tiles.
#include "raster_fwd_impl.hpp"

namespace soup {

void launch_raster_fwd_paper_t16(const RasterArgs& a, hipStream_t s) { launch_fwd_t<16, PaperTex>(a, s); }
int raster_fwd_per_cu_paper_t16(int region) { return fwd_blocks_per_cu<16, PaperTex>(region); }

}  // namespace soup
