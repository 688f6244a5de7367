// Forward raster dispatch over the compiled MLP shapes and tile sizes (the
// kernel is in raster_fwd_impl.hpp, instantiated once per shape and tile in
// fwd_*.hip so that the units compile in parallel).
#include "internal.hpp"

namespace soup {

void launch_raster_fwd_k8_16_1_t8(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k8_16_1_t16(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k8_16_1_t32(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k16_32_2_t8(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k16_32_2_t16(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k16_32_2_t32(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k32_64_2_t8(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k32_64_2_t16(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_k32_64_2_t32(const RasterArgs& a, hipStream_t s);

void launch_raster_fwd_paper_t8(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_paper_t16(const RasterArgs& a, hipStream_t s);
void launch_raster_fwd_paper_t32(const RasterArgs& a, hipStream_t s);
int raster_fwd_per_cu_paper_t8(int region);
int raster_fwd_per_cu_paper_t16(int region);
int raster_fwd_per_cu_paper_t32(int region);

int raster_fwd_per_cu_k8_16_1_t8(int region);
int raster_fwd_per_cu_k8_16_1_t16(int region);
int raster_fwd_per_cu_k8_16_1_t32(int region);
int raster_fwd_per_cu_k16_32_2_t8(int region);
int raster_fwd_per_cu_k16_32_2_t16(int region);
int raster_fwd_per_cu_k16_32_2_t32(int region);
int raster_fwd_per_cu_k32_64_2_t8(int region);
int raster_fwd_per_cu_k32_64_2_t16(int region);
int raster_fwd_per_cu_k32_64_2_t32(int region);

void launch_raster_fwd(const RasterArgs& a, int tile, MlpKind k, hipStream_t s) {
    switch (k) {
        case MlpKind::k8_16_1:
            if (tile == 8) launch_raster_fwd_k8_16_1_t8(a, s);
            else if (tile == 32) launch_raster_fwd_k8_16_1_t32(a, s);
            else launch_raster_fwd_k8_16_1_t16(a, s);
            break;
        case MlpKind::k16_32_2:
            if (tile == 8) launch_raster_fwd_k16_32_2_t8(a, s);
            else if (tile == 32) launch_raster_fwd_k16_32_2_t32(a, s);
            else launch_raster_fwd_k16_32_2_t16(a, s);
            break;
        case MlpKind::k32_64_2:
            if (tile == 8) launch_raster_fwd_k32_64_2_t8(a, s);
            else if (tile == 32) launch_raster_fwd_k32_64_2_t32(a, s);
            else launch_raster_fwd_k32_64_2_t16(a, s);
            break;
        case MlpKind::kPaper:
            if (tile == 8) launch_raster_fwd_paper_t8(a, s);
            else if (tile == 32) launch_raster_fwd_paper_t32(a, s);
            else launch_raster_fwd_paper_t16(a, s);
            break;
        default: break;
    }
}

// Resident single-wave workgroups per CU of the forward for this shape, tile and region side.
int raster_fwd_blocks_per_cu(int tile, MlpKind k, int region) {
    switch (k) {
        case MlpKind::k8_16_1:
            return tile == 8 ? raster_fwd_per_cu_k8_16_1_t8(region) : tile == 32 ? raster_fwd_per_cu_k8_16_1_t32(region) : raster_fwd_per_cu_k8_16_1_t16(region);
        case MlpKind::k16_32_2:
            return tile == 8 ? raster_fwd_per_cu_k16_32_2_t8(region) : tile == 32 ? raster_fwd_per_cu_k16_32_2_t32(region) : raster_fwd_per_cu_k16_32_2_t16(region);
        case MlpKind::k32_64_2:
            return tile == 8 ? raster_fwd_per_cu_k32_64_2_t8(region) : tile == 32 ? raster_fwd_per_cu_k32_64_2_t32(region) : raster_fwd_per_cu_k32_64_2_t16(region);
        case MlpKind::kPaper:
            return tile == 8 ? raster_fwd_per_cu_paper_t8(region) : tile == 32 ? raster_fwd_per_cu_paper_t32(region) : raster_fwd_per_cu_paper_t16(region);
        default: return 1;
    }
}

}  // namespace soup
