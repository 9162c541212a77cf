// Tiled four-step for N = N1 x N2 with N1, N2 in {256, 512, 1024}: both
// stages read and write whole cache-line segments.
//
// The decomposition is that of eq. (3), n = n1 + N1 n2 and k = k2 + N2 k1:
//   stage 1: Y[k2][n1] = sum_{n2} x[n1 + N1 n2] W_N2^{n2 k2}   (N2-point DFTs over n2)
//   stage 2: X[k2 + N2 k1] = sum_{n1} W_N1^{n1 k1} W_N^{n1 k2} Y[k2][n1].
// A workgroup runs TILE transforms side by side.  In stage 1 they are TILE
// adjacent n1, so for every n2 the workgroup reads TILE consecutive elements
// of x (one 128-byte segment for TILE = 16) and writes Y[k2][n1 .. n1 +
// TILE - 1] the same way; the workspace holds Y row by row in k2.  In stage 2
// they are TILE adjacent k2: each reads its contiguous workspace row, applies
// W_N^{n1 k2} (two-level table, as for the N1 x 16384 split) and runs the
// N1-point DFT; the results go through LDS once more so that the stores of
// X[k2 .. k2 + TILE - 1 + N2 k1] are again whole segments.  Each transform
// uses the single-pass body (run_passes) on its own slice of LDS; the slices
// are an odd number of 8-byte slots apart so that the TILE transforms'
// accesses to the same position fall on different banks.  Input loads and
// output stores carry the streaming hint (each segment is touched by one
// workgroup once); the workspace keeps ordinary accesses.  TILE = 8 halves
// the LDS (two workgroups per CU at L = 1024); the two tiles that share each
// 128-byte segment are then put on the same XCD (same L2).
#pragma once

#include "kernels.hpp"

namespace stockfft {

template <class S>
constexpr int tile_stride() {
  return S::LDS_ELEMS | 1;
}

// Tile of workgroup b: the G = 16 / TILE tiles of one 128-byte segment go to
// blocks 8 (G i + r) + x (x: the XCD of the block under round-robin
// dispatch), tile G (8 i + x) + r.  The grid is rounded up to 8 G blocks;
// blocks past the last tile return.
template <int TILE>
__device__ __forceinline__ int64_t tile_of_block(int64_t b) {
  constexpr int G = 16 / TILE;
  if constexpr (G == 1) return b;
  const int64_t x = b % kXcds, q = b / kXcds;
  return G * (kXcds * (q / G) + x) + q % G;
}

// Stage 1: S is the N2-point shape.
template <class S, int N1, int TILE, bool INV>
__global__ __launch_bounds__(TILE * S::T, S::WPE) void k_tile_columns(const c32* x, c32* y,
                                                                     const c32* tw, int64_t rows) {
  static_assert(S::TPB == 1 && N1 % 16 == 0 && 16 % TILE == 0, "tile shape");
  static_assert(!paired_lanes<S>::value, "tiled stages use the plain lane order");
  constexpr int L = N1;
  constexpr int64_t N = (int64_t)N1 * S::N;
  constexpr int tiles = N1 / TILE;
  __shared__ alignas(16) c32 lds[TILE * tile_stride<S>()];
  const int64_t g = tile_of_block<TILE>(blockIdx.x);
  const int64_t row = g / tiles;
  if (row >= rows) return;  // whole workgroup, before any barrier
  const int tile = (int)(g - row * tiles);
  const int tid = threadIdx.x;
  const int s = tid % TILE;  // adjacent lanes: adjacent n1
  const int t = tid / TILE;
  const int n1 = tile * TILE + s;
  const c32* src = x + row * N + n1;
  c32 a[S::E];
#pragma unroll
  for (int m = 0; m < S::E; ++m) a[m] = load_stream(src + (int64_t)(t + m * S::T) * L);
  run_passes<S, INV>(a, lds + s * tile_stride<S>(), tw, t);
  // The store addresses are formed only now (an opaque copy of the lane
  // index), not held in registers through the passes.
  int tl = t;
  asm volatile("" : "+v"(tl));
  c32* dst = y + row * N + n1 + (int64_t)tl * L;
#pragma unroll
  for (int m = 0; m < S::E; ++m) dst[(int64_t)m * S::T * L] = a[m];  // Y[k2][n1], k2 = t + m T
}

// Stage 2: S is the N1-point shape; tw its table, tw4 the two-level W_N table.
template <class S, int N2, int TILE, bool INV>
__global__ __launch_bounds__(TILE * S::T, S::WPE) void k_tile_rows(const c32* y, c32* out,
                                                                  const c32* tw,
                                                                  const c32* __restrict__ tw4,
                                                                  int64_t rows) {
  constexpr int L = S::N;  // N1: the length of a workspace row
  constexpr int64_t N = (int64_t)L * N2;
  constexpr int tiles = N2 / TILE;
  constexpr int SL = half_log2(N);
  static_assert(N2 % 16 == 0 && 16 % TILE == 0, "tile shape");
  static_assert(!paired_lanes<S>::value, "tiled stages use the plain lane order");
  static_assert(S::C == 1, "the closing transpose holds whole transforms in LDS");
  __shared__ alignas(16) c32 lds[TILE * tile_stride<S>()];
  const int64_t g = tile_of_block<TILE>(blockIdx.x);
  const int64_t row = g / tiles;
  if (row >= rows) return;  // whole workgroup, before any barrier
  const int tile = (int)(g - row * tiles);
  const int tid = threadIdx.x;
  const int s = tid / S::T;  // adjacent lanes: adjacent n1 of one row
  const int t = tid - s * S::T;
  const int k2 = tile * TILE + s;
  const c32* src = y + row * N + (int64_t)k2 * L;
  const c32* lo = tw4;
  const c32* hi = tw4 + (1 << SL);
  c32 a[S::E];
#pragma unroll
  for (int m = 0; m < S::E; ++m) {
    const int n1 = t + m * S::T;
    const int e = n1 * k2;  // < N
    a[m] = ctw<INV>(src[n1], cmul(hi[e >> SL], lo[e & ((1 << SL) - 1)]));
  }
  c32* mine = lds + s * tile_stride<S>();
  run_passes<S, INV>(a, mine, tw, t);
  __syncthreads();  // every wave is past its last exchange reads
#pragma unroll
  for (int m = 0; m < S::E; ++m) mine[t + m * S::T] = a[m];  // X[k2 + N2 k1], k1 = t + m T
  __syncthreads();
  const int s2 = tid % TILE;  // adjacent lanes: adjacent k2
  const int t2 = tid / TILE;
  const c32* col = lds + s2 * tile_stride<S>();
  c32* dst = out + row * N + tile * TILE + s2;
#pragma unroll
  for (int m = 0; m < S::E; ++m) {
    const int k1 = t2 + m * S::T;
    store_stream(dst + (int64_t)k1 * N2, col[k1]);
  }
}

// Grid of one launch over `rows` rows: every tile, rounded up to 8 G blocks.
template <int TILE>
inline int64_t tile_grid(int64_t rows, int tiles) {
  const int64_t q = 8 * (16 / TILE);
  return (rows * tiles + q - 1) / q * q;
}

template <int TILES>
inline int64_t tile_rows_per_launch() {
  const int64_t per = max_groups_per_launch() / TILES;
  return per > 0 ? per : 1;
}

template <class S, int N1, int TILE>
hipError_t launch_tile_columns(const void* x, void* y, const void* tw, int64_t batch, bool inverse,
                               hipStream_t s) {
  constexpr int tiles = N1 / TILE;
  constexpr int64_t N = (int64_t)N1 * S::N;
  const int64_t rows_per_launch = tile_rows_per_launch<tiles>();
  for (int64_t r0 = 0; r0 < batch; r0 += rows_per_launch) {
    const int64_t rows = batch - r0 < rows_per_launch ? batch - r0 : rows_per_launch;
    const c32* xp = static_cast<const c32*>(x) + r0 * N;
    c32* yp = static_cast<c32*>(y) + r0 * N;
    const c32* twp = static_cast<const c32*>(tw);
    const dim3 grid((unsigned)tile_grid<TILE>(rows, tiles)), block(TILE * S::T);
    if (inverse)
      k_tile_columns<S, N1, TILE, true><<<grid, block, 0, s>>>(xp, yp, twp, rows);
    else
      k_tile_columns<S, N1, TILE, false><<<grid, block, 0, s>>>(xp, yp, twp, rows);
  }
  return hipGetLastError();
}

// tw is the stage-1 (N2-point) table; when N1 != N2 the N1-point table follows
// the two-level table and W_N1 in tw4.
template <class S, int N2, int TILE>
hipError_t launch_tile_rows(const void* y, void* out, const void* tw, const void* tw4,
                            int64_t batch, bool inverse, hipStream_t s) {
  constexpr int tiles = N2 / TILE;
  constexpr int64_t N = (int64_t)S::N * N2;
  constexpr int SL = half_log2(N);
  constexpr int64_t own_off = S::N == N2 ? -1 : (int64_t(1) << SL) + (N >> SL) + S::N;
  const int64_t rows_per_launch = tile_rows_per_launch<tiles>();
  for (int64_t r0 = 0; r0 < batch; r0 += rows_per_launch) {
    const int64_t rows = batch - r0 < rows_per_launch ? batch - r0 : rows_per_launch;
    const c32* yp = static_cast<const c32*>(y) + r0 * N;
    c32* op = static_cast<c32*>(out) + r0 * N;
    const c32* tw4p = static_cast<const c32*>(tw4);
    const c32* twp = own_off < 0 ? static_cast<const c32*>(tw) : tw4p + own_off;
    const dim3 grid((unsigned)tile_grid<TILE>(rows, tiles)), block(TILE * S::T);
    if (inverse)
      k_tile_rows<S, N2, TILE, true><<<grid, block, 0, s>>>(yp, op, twp, tw4p, rows);
    else
      k_tile_rows<S, N2, TILE, false><<<grid, block, 0, s>>>(yp, op, twp, tw4p, rows);
  }
  return hipGetLastError();
}

}  // namespace stockfft
