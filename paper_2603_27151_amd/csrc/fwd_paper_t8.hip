// Forward raster instantiated for the paper form (opacity texture only) and 8x8 tiles.
#include "raster_fwd_impl.hpp"

namespace soup {

void launch_raster_fwd_paper_t8(const RasterArgs& a, hipStream_t s) { launch_fwd_t<8, PaperTex>(a, s); }
int raster_fwd_per_cu_paper_t8(int region) { return fwd_blocks_per_cu<8, PaperTex>(region); }

}  // namespace soup
