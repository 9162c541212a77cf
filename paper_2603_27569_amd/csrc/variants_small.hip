// Single-pass shapes for N = 256 .. 2048 (several transforms per workgroup
// at the small sizes).  Names: n<N>_e<values per lane>_b<transforms per
// workgroup>_p<pad log2, 0 = none>_r<radices>.
#include "variant_maker.hpp"

using stockfft::PairedTwiddles;
using stockfft::Shape;
using stockfft::ShapeX;
using stockfft::make_variant;

STOCKFFT_VARIANT_GROUP(variants_small,
  make_variant<Shape<256, 4, 4, 4, 4, 4, 4, 4>>("n256_e4_b4_p4_r4.4.4.4"),
  make_variant<PairedTwiddles<Shape<256, 4, 4, 4, 4, 4, 4, 4>>>("n256_e4_b4_p4_r4.4.4.4_pt"),
  make_variant<Shape<256, 8, 8, 4, 8, 8, 4>>("n256_e8_b8_p4_r8.8.4"),
  make_variant<PairedTwiddles<Shape<256, 8, 8, 4, 8, 8, 4>>>("n256_e8_b8_p4_r8.8.4_pt"),
  make_variant<Shape<256, 16, 16, 4, 16, 16>>("n256_e16_b16_p4_r16.16"),
  make_variant<PairedTwiddles<Shape<256, 16, 16, 4, 16, 16>>>("n256_e16_b16_p4_r16.16_pt"),
  make_variant<Shape<256, 16, 4, 4, 16, 16>>("n256_e16_b4_p4_r16.16"),
  make_variant<PairedTwiddles<Shape<256, 16, 4, 4, 16, 16>>>("n256_e16_b4_p4_r16.16_pt"),
  make_variant<Shape<512, 4, 2, 4, 4, 4, 4, 4, 2>>("n512_e4_b2_p4_r4.4.4.4.2"),
  make_variant<PairedTwiddles<Shape<512, 4, 2, 4, 4, 4, 4, 4, 2>>>("n512_e4_b2_p4_r4.4.4.4.2_pt"),
  make_variant<Shape<512, 8, 4, 4, 8, 8, 8>>("n512_e8_b4_p4_r8.8.8"),
  make_variant<PairedTwiddles<Shape<512, 8, 4, 4, 8, 8, 8>>>("n512_e8_b4_p4_r8.8.8_pt"),
  make_variant<Shape<512, 16, 8, 4, 16, 16, 2>>("n512_e16_b8_p4_r16.16.2"),
  make_variant<Shape<512, 16, 2, 4, 16, 16, 2>>("n512_e16_b2_p4_r16.16.2"),
  make_variant<PairedTwiddles<Shape<512, 16, 2, 4, 16, 16, 2>>>("n512_e16_b2_p4_r16.16.2_pt"),
  make_variant<Shape<1024, 4, 1, 4, 4, 4, 4, 4, 4>>("n1024_e4_b1_p4_r4.4.4.4.4"),
  make_variant<PairedTwiddles<Shape<1024, 4, 1, 4, 4, 4, 4, 4, 4>>>("n1024_e4_b1_p4_r4.4.4.4.4_pt"),
  make_variant<Shape<1024, 8, 2, 4, 8, 8, 8, 2>>("n1024_e8_b2_p4_r8.8.8.2"),
  make_variant<PairedTwiddles<Shape<1024, 8, 2, 4, 8, 8, 8, 2>>>("n1024_e8_b2_p4_r8.8.8.2_pt"),
  make_variant<Shape<1024, 16, 4, 4, 16, 16, 4>>("n1024_e16_b4_p4_r16.16.4"),
  make_variant<PairedTwiddles<Shape<1024, 16, 4, 4, 16, 16, 4>>>("n1024_e16_b4_p4_r16.16.4_pt"),
  make_variant<Shape<1024, 16, 1, 4, 16, 16, 4>>("n1024_e16_b1_p4_r16.16.4"),
  make_variant<PairedTwiddles<Shape<1024, 16, 1, 4, 16, 16, 4>>>("n1024_e16_b1_p4_r16.16.4_pt"),
  make_variant<Shape<2048, 4, 1, 4, 4, 4, 4, 4, 4, 2>>("n2048_e4_b1_p4_r4.4.4.4.4.2"),
  make_variant<Shape<2048, 8, 1, 4, 8, 8, 8, 4>>("n2048_e8_b1_p4_r8.8.8.4"),
  make_variant<PairedTwiddles<Shape<2048, 8, 1, 4, 8, 8, 8, 4>>>("n2048_e8_b1_p4_r8.8.8.4_pt"),
  make_variant<Shape<2048, 16, 2, 4, 16, 16, 8>>("n2048_e16_b2_p4_r16.16.8"),
  make_variant<PairedTwiddles<Shape<2048, 16, 2, 4, 16, 16, 8>>>("n2048_e16_b2_p4_r16.16.8_pt"),
  make_variant<Shape<2048, 16, 1, 4, 16, 16, 8>>("n2048_e16_b1_p4_r16.16.8"),
  make_variant<PairedTwiddles<Shape<2048, 16, 1, 4, 16, 16, 8>>>("n2048_e16_b1_p4_r16.16.8_pt"),
  // Two-round exchanges (half the LDS), one wave per transform, at most 128
  // VGPRs: occupancy set by the registers rather than by the LDS.
  make_variant<ShapeX<2, false, 4, 2048, 32, 1, 4, 16, 16, 8>>("n2048_e32_c2_b1_p4_r16.16.8"),
  make_variant<PairedTwiddles<ShapeX<2, false, 4, 2048, 32, 1, 4, 16, 16, 8>>>("n2048_e32_c2_b1_p4_r16.16.8_pt"),
  make_variant<ShapeX<2, false, 4, 2048, 32, 2, 4, 16, 16, 8>>("n2048_e32_c2_b2_p4_r16.16.8"),
  make_variant<PairedTwiddles<ShapeX<2, false, 4, 2048, 32, 2, 4, 16, 16, 8>>>("n2048_e32_c2_b2_p4_r16.16.8_pt"))
