// Single-pass shapes for N = 8192 and 16384.  gfx950's 160 KiB LDS holds a
// whole 16384-point complex64 transform (128 KiB + pad), so these sizes need
// no device-memory exchange at all; the four-step path is kept beside them.
#include "variant_maker.hpp"

using stockfft::PairedTwiddles;
using stockfft::Shape;
using stockfft::ShapeX;
using stockfft::make_variant;

STOCKFFT_VARIANT_GROUP(variants_large,
  make_variant<Shape<8192, 8, 1, 4, 8, 8, 8, 8, 2>>("n8192_e8_b1_p4_r8.8.8.8.2"),
  make_variant<PairedTwiddles<Shape<8192, 8, 1, 4, 8, 8, 8, 8, 2>>>("n8192_e8_b1_p4_r8.8.8.8.2_pt"),
  make_variant<Shape<8192, 16, 1, 4, 16, 16, 16, 2>>("n8192_e16_b1_p4_r16.16.16.2"),
  make_variant<PairedTwiddles<Shape<8192, 16, 1, 4, 16, 16, 16, 2>>>("n8192_e16_b1_p4_r16.16.16.2_pt"),
  make_variant<Shape<8192, 32, 1, 4, 16, 16, 16, 2>>("n8192_e32_b1_p4_r16.16.16.2"),
  make_variant<PairedTwiddles<Shape<8192, 32, 1, 4, 16, 16, 16, 2>>>("n8192_e32_b1_p4_r16.16.16.2_pt"),
  make_variant<Shape<16384, 16, 1, 4, 16, 16, 16, 4>>("n16384_e16_b1_p4_r16.16.16.4"),
  make_variant<PairedTwiddles<Shape<16384, 16, 1, 4, 16, 16, 16, 4>>>("n16384_e16_b1_p4_r16.16.16.4_pt"),
  make_variant<Shape<16384, 32, 1, 4, 16, 16, 16, 4>>("n16384_e32_b1_p4_r16.16.16.4"),
  make_variant<PairedTwiddles<Shape<16384, 32, 1, 4, 16, 16, 16, 4>>>("n16384_e32_b1_p4_r16.16.16.4_pt"),
  // Two-round exchanges: half the LDS, two (16384) or four (8192) workgroups per CU.
  make_variant<ShapeX<2, false, 4, 16384, 32, 1, 4, 16, 16, 16, 4>>("n16384_e32_c2_b1_p4_r16.16.16.4"),
  make_variant<PairedTwiddles<ShapeX<2, false, 4, 16384, 32, 1, 4, 16, 16, 16, 4>>>("n16384_e32_c2_b1_p4_r16.16.16.4_pt"),
  make_variant<ShapeX<2, false, 4, 8192, 32, 1, 4, 16, 16, 16, 2>>("n8192_e32_c2_b1_p4_r16.16.16.2"),
  make_variant<PairedTwiddles<ShapeX<2, false, 4, 8192, 32, 1, 4, 16, 16, 16, 2>>>("n8192_e32_c2_b1_p4_r16.16.16.2_pt"),
  // Four-round exchanges (a quarter of the LDS): radix 8 before the last
  // pass, so that every exchange splits into four rounds.
  make_variant<ShapeX<4, false, 4, 16384, 32, 1, 4, 8, 8, 8, 8, 4>>("n16384_e32_c4_b1_p4_r8.8.8.8.4"),
  make_variant<ShapeX<4, false, 4, 8192, 32, 1, 4, 8, 8, 8, 16>>("n8192_e32_c4_b1_p4_r8.8.8.16"),
  // Sixteen values per lane with two-round exchanges: radix 8 leaves two
  // butterflies per lane per pass, so each round takes one, and the body fits
  // 64 VGPRs; two 1024-lane workgroups (32 waves) then share a CU.
  make_variant<ShapeX<2, false, 8, 16384, 16, 1, 4, 8, 8, 8, 8, 4>>("n16384_e16_c2_b1_p4_r8.8.8.8.4"),
  make_variant<PairedTwiddles<ShapeX<2, false, 8, 16384, 16, 1, 4, 8, 8, 8, 8, 4>>>("n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"))
