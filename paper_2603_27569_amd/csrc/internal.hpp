// Helpers shared by the host-side translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "variants.hpp"

namespace stockfft {

extern thread_local int g_last_hip_error;

// Records e as the thread's last HIP error; returns the matching status.
int hip_fail(hipError_t e);

const SingleVariant* find_single(const char* name);
const SingleVariant* tuned_variant(int64_t n, int64_t batch);
const SingleVariant* tuned_filter_variant(int64_t n, int64_t batch);
void tuned_choice(int64_t n, int64_t batch, bool single_only, const SingleVariant** sv,
                  const FourStepVariant** fs);
bool valid_size(int64_t n);         // any plan length
bool valid_single_size(int64_t n);  // lengths with a single-pass kernel (and ragged batches)
int ilog2(int64_t n);
void build_stockham_twiddles(const SingleVariant& v, std::vector<float>& out);
// Matrix-core DFT stages with 16-bit storage (mma.hip): N = 16^P RL for
// N = 512 ... 16384, on the twiddle table of the variant mma_table_variant(n)
// (radix 16 throughout, then RL).
bool mma_supported(int64_t n);
const char* mma_table_variant(int64_t n);
hipError_t launch_mma_f16(int64_t n, const void* in, void* out, const void* tw, int64_t batch,
                          bool inverse, hipStream_t s);
hipError_t launch_mma_bf16(int64_t n, const void* in, void* out, const void* tw, int64_t batch,
                           bool inverse, hipStream_t s);
int upload(const std::vector<float>& host, void** dev);
int check_device(int* dev);
bool ranges_partially_overlap(const void* a, const void* b, size_t bytes);
bool aligned8(const void* p);

void register_handle(const void* p);
bool unregister_handle(const void* p);
bool live_handle(const void* p);

// Makes `dev` current for the lifetime of the guard when it is not already.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;

 private:
  int prev_ = 0;
  bool switched_ = false;
};

}  // namespace stockfft
