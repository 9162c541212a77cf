// Builds SingleVariant table entries from Stockham shapes.
#pragma once

#include "kernels.hpp"
#include "wavex.hpp"

namespace stockfft {

template <class S>
SingleVariant make_variant(const char* name) {
  SingleVariant v{};
  v.name = name;
  v.n = S::N;
  v.e = S::E;
  v.t = S::T;
  v.tpb = S::TPB;
  v.padlog = S::PADLOG;
  v.npass = S::P;
  for (int i = 0; i < S::P; ++i) v.radix[i] = S::radix(i);
  v.chunks = S::C;
  v.double_buffered = double_buffered<S>::value;
  v.twiddle_schedule = S::PF;
  v.paired_twiddles = paired_twiddles<S>::value;
  v.paired_lanes = paired_lanes<S>::value;
  v.streamed = streamed<S>::value;
  v.threads = S::THREADS;
  v.lds_bytes = S::TPB * S::LDS_ELEMS * (int)sizeof(c32);
  v.tw_elems = S::TW_ELEMS;
  v.wave_exchange = wave_exchange<S>::value;
  v.wave_members = wave_members<S>::value;
  if constexpr (wave_exchange<S>::value > 0) {
    // The plain transform (either storage) and both fused kernels.
    v.launch = &launch_wx<S, IoF32>;
    v.fused = &launch_spectral_energy_wx<S>;
    v.filter = &launch_matched_filter_wx<S>;
    v.launch_f16 = &launch_wx<S, IoF16>;
    v.launch_bf16 = &launch_wx<S, IoBF16>;
    v.kernel = reinterpret_cast<const void*>(&k_stockham_wx<S, false, IoF32>);
    return v;
  } else if constexpr (streamed<S>::value > 0) {
    // Persistent shapes run the plain transform (either storage) and the
    // fused forward -> weight -> adjoint kernel.
    v.launch = &launch_stream<S, IoF32>;
    v.launch_f16 = &launch_stream<S, IoF16>;
    v.launch_bf16 = &launch_stream<S, IoBF16>;
    v.fused = &launch_spectral_energy_stream<S>;
    v.kernel = reinterpret_cast<const void*>(&k_stockham_stream<S, false, IoF32>);
    return v;
  } else {
    v.launch = &launch_single<S>;
    if constexpr (round_trip_layout<S>()) {
      v.fused = &launch_spectral_energy<S>;
      v.filter = &launch_matched_filter<S>;
    }
    v.launch_f16 = &launch_single_io<S, IoF16>;
    v.launch_bf16 = &launch_single_io<S, IoBF16>;
    v.kernel = reinterpret_cast<const void*>(&k_stockham<S, false>);
  }
  return v;
}

}  // namespace stockfft

// Each size group exports its entries through one accessor.
#define STOCKFFT_VARIANT_GROUP(FN, ...)                                   \
  namespace stockfft {                                                    \
  const SingleVariant* FN(int* count) {                                   \
    static const SingleVariant table[] = {__VA_ARGS__};                   \
    *count = (int)(sizeof(table) / sizeof(table[0]));                     \
    return table;                                                         \
  }                                                                       \
  }
