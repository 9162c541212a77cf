// Single-pass shapes for N = 4096: the paper's radix-4 (1024 lanes) and
// radix-8 (512 lanes) designs, the radix-16 re-derivation for gfx950's
// larger register file, and the LDS-layout ablation (no pad / 1 in 16 / 1 in 32).
#include "variant_maker.hpp"

using stockfft::DoubleBuffered;
using stockfft::PairedLanes;
using stockfft::PairedTwiddles;
using stockfft::Shape;
using stockfft::ShapeX;
using stockfft::Streamed;
using stockfft::WaveExchange;
using stockfft::make_variant;

STOCKFFT_VARIANT_GROUP(variants_4096,
  make_variant<Shape<4096, 4, 1, 4, 4, 4, 4, 4, 4, 4>>("n4096_e4_b1_p4_r4.4.4.4.4.4"),
  make_variant<Shape<4096, 8, 1, 4, 8, 8, 8, 8>>("n4096_e8_b1_p4_r8.8.8.8"),
  make_variant<PairedTwiddles<Shape<4096, 8, 1, 4, 8, 8, 8, 8>>>("n4096_e8_b1_p4_r8.8.8.8_pt"),
  make_variant<Shape<4096, 16, 1, 4, 16, 16, 16>>("n4096_e16_b1_p4_r16.16.16"),
  make_variant<Shape<4096, 16, 1, 0, 16, 16, 16>>("n4096_e16_b1_p0_r16.16.16"),
  make_variant<Shape<4096, 16, 1, 5, 16, 16, 16>>("n4096_e16_b1_p5_r16.16.16"),
  make_variant<Shape<4096, 16, 1, -1, 16, 16, 16>>("n4096_e16_b1_px_r16.16.16"),
  // Every pass's twiddles loaded with the input (measured slower at 4096 x 256
  // than one pass ahead: the extra loads delay the input's arrival).
  make_variant<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>("n4096_e16_b1_px_r16.16.16_tall"),
  make_variant<DoubleBuffered<Shape<4096, 16, 1, 5, 16, 16, 16>>>("n4096_e16_b1_p5_r16.16.16_db"),
  make_variant<DoubleBuffered<Shape<4096, 16, 1, -1, 16, 16, 16>>>("n4096_e16_b1_px_r16.16.16_db"),
  // Paired twiddle tables (_pt): half the twiddle load instructions.
  make_variant<DoubleBuffered<PairedTwiddles<Shape<4096, 16, 1, -1, 16, 16, 16>>>>("n4096_e16_b1_px_r16.16.16_db_pt"),
  // Paired twiddles loaded with the input (_tall): the load phase waits on
  // HBM anyway, and sixteen more 16-byte loads no longer delay it.
  make_variant<DoubleBuffered<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>>>("n4096_e16_b1_px_r16.16.16_db_pt_tall"),
  make_variant<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, 4, 8, 8, 8, 8>>>("n4096_e8_b1_p4_r8.8.8.8_pt_tall"),
  // Radix-8 exchanges with the XOR swizzle: no bank conflicts (the padded
  // layout has about one conflict cycle per LDS cycle), for 17% more VALU
  // work on the addresses; the two measure within 1% of each other.
  make_variant<PairedTwiddles<Shape<4096, 8, 1, -1, 8, 8, 8, 8>>>("n4096_e8_b1_px_r8.8.8.8_pt"),
  make_variant<PairedTwiddles<Shape<4096, 16, 1, -1, 16, 16, 16>>>("n4096_e16_b1_px_r16.16.16_pt"),
  make_variant<PairedTwiddles<Shape<4096, 16, 1, 5, 16, 16, 16>>>("n4096_e16_b1_p5_r16.16.16_pt"),
  make_variant<PairedTwiddles<Shape<4096, 32, 1, 4, 16, 16, 16>>>("n4096_e32_b1_p4_r16.16.16_pt"),
  // Paired lanes: 16-byte (FP32) and 8-byte (16-bit) row accesses.  They
  // tie the 4- and 8-byte forms here and lost at the other lengths measured
  // (lane-strided accesses once a lane owns more than two butterflies).
  make_variant<PairedLanes<PairedTwiddles<Shape<4096, 32, 1, 4, 16, 16, 16>>>>("n4096_e32_b1_p4_r16.16.16_pt_pl"),
  make_variant<PairedTwiddles<ShapeX<2, false, 4, 4096, 32, 1, 4, 16, 16, 16>>>("n4096_e32_c2_b1_p4_r16.16.16_pt"),
  make_variant<PairedLanes<PairedTwiddles<ShapeX<2, false, 4, 4096, 32, 1, 4, 16, 16, 16>>>>("n4096_e32_c2_b1_p4_r16.16.16_pt_pl"),
  make_variant<Shape<4096, 32, 1, 4, 16, 16, 16>>("n4096_e32_b1_p4_r16.16.16"),
  make_variant<Shape<4096, 32, 2, 4, 16, 16, 16>>("n4096_e32_b2_p4_r16.16.16"),
  // Two-round exchanges: half the LDS (17 KiB), so occupancy is set by the
  // registers (at most 128: four waves per SIMD) rather than by the LDS.
  make_variant<ShapeX<2, false, 4, 4096, 32, 1, 4, 16, 16, 16>>("n4096_e32_c2_b1_p4_r16.16.16"),
  // Persistent streaming forms (k workgroups per CU loop over the rows, the
  // next row's loads in flight during the current row's passes), for
  // batches of several rows per CU.
  // Names end in _st<workgroups per CU>d<rows in flight ahead>.
  make_variant<Streamed<DoubleBuffered<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>>, 2, 1>>(
      "n4096_e16_b1_px_r16.16.16_db_pt_tall_st2d1"),
  make_variant<Streamed<DoubleBuffered<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>>, 2, 2>>(
      "n4096_e16_b1_px_r16.16.16_db_pt_tall_st2d2"),
  make_variant<Streamed<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, 4, 8, 8, 8, 8>>, 1, 3>>(
      "n4096_e8_b1_p4_r8.8.8.8_pt_tall_st1d3"),
  make_variant<Streamed<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, 4, 8, 8, 8, 8>>, 2, 2>>(
      "n4096_e8_b1_p4_r8.8.8.8_pt_tall_st2d2"),
  // One persistent workgroup per CU, one row ahead: at 257-1024 rows each
  // loops over two to four rows, so the fused kernel's second transform
  // overlaps the next row's loads.
  make_variant<Streamed<DoubleBuffered<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 16, 16, 16>>>, 1, 1>>(
      "n4096_e16_b1_px_r16.16.16_db_pt_tall_st1d1"),
  make_variant<Streamed<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, 4, 8, 8, 8, 8>>, 1, 1>>(
      "n4096_e8_b1_p4_r8.8.8.8_pt_tall_st1d1"),
  // In-wave exchanges after passes 0 and 2 (8 x 8 transposes by cross-lane
  // moves), the LDS only between passes 1 and 2: one barrier per transform.
  // _wx1: one group per lane (8-byte accesses in 64-byte runs); _wx2: two
  // adjacent groups per lane (16-byte accesses in whole 128-byte lines).
  make_variant<WaveExchange<PairedTwiddles<ShapeX<1, 2, 1, 4096, 8, 1, -1, 8, 8, 8, 8>>, 1>>(
      "n4096_e8_b1_px_r8.8.8.8_pt_wx1"),
  make_variant<WaveExchange<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 8, 8, 8, 8>>, 2>>(
      "n4096_e16_b1_px_r8.8.8.8_pt_wx2"),
  make_variant<WaveExchange<ShapeX<1, 2, 1, 4096, 8, 1, -1, 8, 8, 8, 8>, 1>>(
      "n4096_e8_b1_px_r8.8.8.8_wx1"),
  // Two members of each group per lane (_wm2): 8-byte accesses covering whole
  // 128-byte lines, transposes by permlane swaps only.
  make_variant<WaveExchange<PairedTwiddles<ShapeX<1, 2, 1, 4096, 16, 1, -1, 8, 8, 8, 8>>, 1, 2>>(
      "n4096_e16_b1_px_r8.8.8.8_pt_wm2"))
