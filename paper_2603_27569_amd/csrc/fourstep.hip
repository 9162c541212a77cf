// Four-step variants (the paper's synthesis rule 2, Section IV-D, with the
// splits of Section V-D eq. (7)-(8) plus N2 = 2048 alternatives).
#include "kernels.hpp"

namespace stockfft {

namespace {
using Sub4096 = Shape<4096, 16, 1, 4, 16, 16, 16>;
using Sub2048 = Shape<2048, 16, 1, 4, 16, 16, 8>;
}  // namespace

const FourStepVariant* four_step_variants(int* count) {
  static const FourStepVariant table[] = {
    {"fs8192_2x4096", 8192, 2, 4096, "n4096_e16_b1_p4_r16.16.16", Sub4096::TW_ELEMS,
     &launch_four_step_columns<Sub4096, 2>, &launch_four_step_combine<2, 4096>},
    {"fs8192_4x2048", 8192, 4, 2048, "n2048_e16_b1_p4_r16.16.8", Sub2048::TW_ELEMS,
     &launch_four_step_columns<Sub2048, 4>, &launch_four_step_combine<4, 2048>},
    {"fs16384_4x4096", 16384, 4, 4096, "n4096_e16_b1_p4_r16.16.16", Sub4096::TW_ELEMS,
     &launch_four_step_columns<Sub4096, 4>, &launch_four_step_combine<4, 4096>},
    {"fs16384_8x2048", 16384, 8, 2048, "n2048_e16_b1_p4_r16.16.8", Sub2048::TW_ELEMS,
     &launch_four_step_columns<Sub2048, 8>, &launch_four_step_combine<8, 2048>},
  };
  *count = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace stockfft
