// Four-step variants: the paper's synthesis rule 2 (Section IV-D) with the
// splits of Section V-D eq. (7)-(8) plus N2 = 2048 alternatives, and the same
// decomposition for lengths beyond one LDS-resident transform (rule 3's
// multi-level case): N = N1 x 16384 up to 2^20, the second stage's N1-point
// DFTs (N1 <= 64) done in registers with two-level twiddles, and the tiled
// splits N1 x N2 with N1, N2 in {256, 512, 1024} (tile.hpp).  Without a tuning entry a length takes its
// first split listed here.
#include "kernels.hpp"
#include "tile.hpp"

namespace stockfft {

namespace {
using Sub4096 = Shape<4096, 16, 1, 4, 16, 16, 16>;
using Sub2048 = Shape<2048, 16, 1, 4, 16, 16, 8>;
using Sub16384 = ShapeX<2, false, 4, 16384, 32, 1, 4, 16, 16, 16, 4>;
constexpr const char* kSub16384 = "n16384_e32_c2_b1_p4_r16.16.16.4";
// Tiled splits (tile.hpp): one 64-lane transform per tile column.
using Tile256 = ShapeX<1, 1, 1, 256, 4, 1, 4, 4, 4, 4, 4>;
using Tile512 = ShapeX<1, 1, 1, 512, 8, 1, 4, 8, 8, 8>;
using Tile1024 = ShapeX<1, 1, 1, 1024, 16, 1, 4, 16, 16, 4>;
// Stage-1 shapes with a two-round exchange (half the LDS per transform, two
// workgroups per CU): 32 lanes per transform.
using Tile512c = ShapeX<2, 1, 4, 512, 16, 1, 4, 8, 8, 8>;
using Tile1024c = ShapeX<2, 0, 4, 1024, 32, 1, 4, 16, 16, 4>;
}  // namespace

const FourStepVariant* four_step_variants(int* count) {
  static const FourStepVariant table[] = {
    {"fs8192_2x4096", 8192, 2, 4096, "n4096_e16_b1_p4_r16.16.16", Sub4096::TW_ELEMS,
     &launch_four_step_columns<Sub4096, 2>, &launch_four_step_combine<2, 4096, false>, false},
    {"fs8192_4x2048", 8192, 4, 2048, "n2048_e16_b1_p4_r16.16.8", Sub2048::TW_ELEMS,
     &launch_four_step_columns<Sub2048, 4>, &launch_four_step_combine<4, 2048, false>, false},
    {"fs16384_4x4096", 16384, 4, 4096, "n4096_e16_b1_p4_r16.16.16", Sub4096::TW_ELEMS,
     &launch_four_step_columns<Sub4096, 4>, &launch_four_step_combine<4, 4096, false>, false},
    {"fs16384_8x2048", 16384, 8, 2048, "n2048_e16_b1_p4_r16.16.8", Sub2048::TW_ELEMS,
     &launch_four_step_columns<Sub2048, 8>, &launch_four_step_combine<8, 2048, false>, false},
    {"fs32768_2x16384", 32768, 2, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 2>, &launch_four_step_combine<2, 16384, true>, true},
    {"fs65536_4x16384", 65536, 4, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 4>, &launch_four_step_combine<4, 16384, true>, true},
    {"fs131072_tile256x512", 131072, 256, 512, "n512_e8_b4_p4_r8.8.8", Tile512::TW_ELEMS,
     &launch_tile_columns<Tile512c, 256, 16>, &launch_tile_rows<Tile256, 512, 16>, true,
     "n256_e4_b4_p4_r4.4.4.4"},
    {"fs131072_8x16384", 131072, 8, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 8>, &launch_four_step_combine<8, 16384, true>, true},
    {"fs262144_tile512x512_c2", 262144, 512, 512, "n512_e8_b4_p4_r8.8.8", Tile512::TW_ELEMS,
     &launch_tile_columns<Tile512c, 512, 16>, &launch_tile_rows<Tile512, 512, 16>, true, nullptr},
    {"fs262144_tile512x512", 262144, 512, 512, "n512_e8_b4_p4_r8.8.8", Tile512::TW_ELEMS,
     &launch_tile_columns<Tile512, 512, 16>, &launch_tile_rows<Tile512, 512, 16>, true, nullptr},
    {"fs262144_16x16384", 262144, 16, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 16>, &launch_four_step_combine<16, 16384, true>, true},
    {"fs524288_tile1024x512", 524288, 1024, 512, "n512_e8_b4_p4_r8.8.8", Tile512::TW_ELEMS,
     &launch_tile_columns<Tile512c, 1024, 16>, &launch_tile_rows<Tile1024, 512, 8>, true,
     "n1024_e16_b1_p4_r16.16.4"},
    {"fs524288_32x16384", 524288, 32, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 32>, &launch_four_step_combine<32, 16384, true>, true},
    {"fs1048576_tile1024x1024", 1048576, 1024, 1024, "n1024_e16_b1_p4_r16.16.4",
     Tile1024::TW_ELEMS, &launch_tile_columns<Tile1024, 1024, 16>, &launch_tile_rows<Tile1024, 1024, 8>, true,
     nullptr},
    {"fs1048576_tile1024x1024_c2", 1048576, 1024, 1024, "n1024_e16_b1_p4_r16.16.4",
     Tile1024::TW_ELEMS, &launch_tile_columns<Tile1024c, 1024, 16>, &launch_tile_rows<Tile1024, 1024, 8>, true,
     nullptr},
    {"fs1048576_64x16384", 1048576, 64, 16384, kSub16384, Sub16384::TW_ELEMS,
     &launch_four_step_columns<Sub16384, 64>, &launch_four_step_combine<64, 16384, true>, true},
    {"fs65536_tile256x256", 65536, 256, 256, "n256_e4_b4_p4_r4.4.4.4", Tile256::TW_ELEMS,
     &launch_tile_columns<Tile256, 256, 16>, &launch_tile_rows<Tile256, 256, 16>, true, nullptr},
  };
  *count = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace stockfft
