// Twiddle tables, built on the host: every root exp(-2 pi i m / L) is
// evaluated in FP64 from the exactly reduced exponent m < L and rounded once
// to FP32 (round to nearest).  Host-only code with no HIP dependency, so the
// builders can also be compiled and checked by a plain C++ compiler.
#pragma once

#include <stdint.h>

#include <cmath>
#include <vector>

namespace stockfft {

inline int ilog2_i64(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

// exp(-2 pi i m / L) for 0 <= m < L, evaluated in FP64 and rounded once to FP32.
inline void root_f32(int64_t m, int64_t L, float* re, float* im) {
  const double a = -2.0 * M_PI * (double)m / (double)L;
  *re = (float)std::cos(a);
  *im = (float)std::sin(a);
}

// Per-pass tables of a Stockham plan with radices R_0 .. R_{npass-1}, for
// pass p >= 1 with Ns = R_0 ... R_{p-1} and W = W_{Ns R_p}, appended pass
// after pass (interleaved re, im):
//   plain   entry [r - 1][k] = W^{k r}, r in [1, R_p), k in [0, Ns);
//   paired  for passes with R_p >= 4, entry [q][k][h] = W^{k (2q + 1 + h)},
//           q in [0, R_p / 2), h in {0, 1}, k in [0, Ns), zero where
//           2q + 1 + h = R_p; radix-2 passes as plain.
inline void stockham_twiddles(const int* radix, int npass, bool paired, std::vector<float>& out) {
  out.clear();
  if (npass < 1) return;
  int64_t ns = radix[0];
  auto put = [&](int64_t m, int64_t L) {
    float re, im;
    root_f32(m, L, &re, &im);
    out.push_back(re);
    out.push_back(im);
  };
  for (int p = 1; p < npass; ++p) {
    const int R = radix[p];
    const int64_t L = ns * R;
    if (paired && R >= 4) {
      for (int q = 0; q < R / 2; ++q)
        for (int64_t k = 0; k < ns; ++k)
          for (int h = 0; h < 2; ++h) {
            const int r = 2 * q + 1 + h;
            if (r < R) {
              put(k * r, L);
            } else {
              out.push_back(0.0f);
              out.push_back(0.0f);
            }
          }
    } else {
      for (int r = 1; r < R; ++r)
        for (int64_t k = 0; k < ns; ++k) put(k * r, L);
    }
    ns *= R;
  }
}

// Four-step second-stage table for N = N1 N2.  Full layout: entry
// [n1 - 1][k2] = W_N^{n1 k2}, n1 in [1, N1), k2 in [0, N2).  Two-level layout
// (large N): lo[j] = W_N^j for j < 2^s, hi[j] = W_N^{j 2^s} for j < N / 2^s
// (s = floor(log2 N / 2)), so W_N^m = hi[m >> s] lo[m mod 2^s]; then W_N1^j
// for j < N1.  The caller appends any further table.
inline void four_step_twiddles(int64_t n1, int64_t n2, bool two_level, std::vector<float>& out) {
  out.clear();
  const int64_t N = n1 * n2;
  auto put = [&](int64_t m, int64_t L) {
    float re, im;
    root_f32(m, L, &re, &im);
    out.push_back(re);
    out.push_back(im);
  };
  if (!two_level) {
    for (int64_t i = 1; i < n1; ++i)
      for (int64_t k2 = 0; k2 < n2; ++k2) put(i * k2, N);
    return;
  }
  const int s = ilog2_i64(N) / 2;
  for (int64_t j = 0; j < (int64_t(1) << s); ++j) put(j, N);
  for (int64_t j = 0; j < (N >> s); ++j) put(j << s, N);
  for (int64_t j = 0; j < n1; ++j) put(j, n1);
}

}  // namespace stockfft
