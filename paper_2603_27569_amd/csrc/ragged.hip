// Ragged batches: placeholder entry points (implementation pending).
#include "../../include/stockfft.h"

extern "C" int fft_plan_ragged(fft_ragged_plan_t* plan, const int64_t*, int64_t, int) {
  if (plan) *plan = nullptr;
  return FFT_UNSUPPORTED;
}
extern "C" int fft_exec_ragged(fft_ragged_plan_t, const void*, void*, void*) { return FFT_UNSUPPORTED; }
extern "C" int fft_exec_ragged_plain(fft_ragged_plan_t, const void* const*, void* const*, void*) {
  return FFT_UNSUPPORTED;
}
extern "C" int fft_destroy_ragged(fft_ragged_plan_t) { return FFT_SUCCESS; }
