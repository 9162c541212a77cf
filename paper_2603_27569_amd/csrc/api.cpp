// C ABI of the library: planning, twiddle tables, execution, tuning and
// introspection.  Declarations and argument contracts: include/stockfft.h.
#include "../../include/stockfft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.hpp"
#include "json_lite.hpp"
#include "twiddles.hpp"
#include "variants.hpp"

namespace stockfft {
const SingleVariant* variants_small(int* count);
const SingleVariant* variants_4096(int* count);
const SingleVariant* variants_large(int* count);
}  // namespace stockfft

using namespace stockfft;

namespace stockfft {

thread_local int g_last_hip_error = 0;

namespace {
std::atomic<int64_t> g_max_groups{kDefaultMaxGroupsPerLaunch};
}
int64_t max_groups_per_launch() { return g_max_groups.load(std::memory_order_relaxed); }

namespace {
constexpr int kMaxDevices = 64;
std::atomic<int> g_cus[kMaxDevices];  // 0 = not queried yet
}  // namespace

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 1;
  if (dev < kMaxDevices) {
    const int c = g_cus[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 1;
  if (dev < kMaxDevices) g_cus[dev].store(cus, std::memory_order_relaxed);
  return cus;
}
void set_max_groups_per_launch(int64_t g) { g_max_groups.store(g, std::memory_order_relaxed); }

int hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return FFT_ALLOC_FAILED;
  return FFT_HIP_ERROR;
}

const std::vector<const SingleVariant*>& single_variants() {
  static const std::vector<const SingleVariant*> all = [] {
    std::vector<const SingleVariant*> v;
    for (auto fn : {variants_small, variants_4096, variants_large}) {
      int c = 0;
      const SingleVariant* t = fn(&c);
      for (int i = 0; i < c; ++i) v.push_back(&t[i]);
    }
    return v;
  }();
  return all;
}

const SingleVariant* find_single(const char* name) {
  if (!name) return nullptr;
  for (const SingleVariant* v : single_variants())
    if (std::strcmp(v->name, name) == 0) return v;
  return nullptr;
}

int num_four_step() {
  int c = 0;
  four_step_variants(&c);
  return c;
}

const FourStepVariant& four_step_at(int i) {
  int c = 0;
  return four_step_variants(&c)[i];
}

const FourStepVariant* find_four_step(const char* name) {
  if (!name) return nullptr;
  for (int i = 0; i < num_four_step(); ++i)
    if (std::strcmp(four_step_at(i).name, name) == 0) return &four_step_at(i);
  return nullptr;
}

bool valid_size(int64_t n) { return n >= 256 && n <= kMaxN && (n & (n - 1)) == 0; }
bool valid_single_size(int64_t n) { return valid_size(n) && n <= kMaxSinglePassN; }

int ilog2(int64_t n) { return ilog2_i64(n); }

void build_stockham_twiddles(const SingleVariant& v, std::vector<float>& out) {
  stockham_twiddles(v.radix, v.npass, v.paired_twiddles, out);
}

// The four-step table, plus (tiled splits with N1 != N2) the second stage's
// N1-point single-pass table appended.
void build_four_step_twiddles(const FourStepVariant& f, std::vector<float>& out) {
  four_step_twiddles(f.n1, f.n2, f.two_level, out);
  if (f.two_level && f.sub2_name) {
    std::vector<float> sub2;
    build_stockham_twiddles(*find_single(f.sub2_name), sub2);
    out.insert(out.end(), sub2.begin(), sub2.end());
  }
}

int upload(const std::vector<float>& host, void** dev) {
  *dev = nullptr;
  if (host.empty()) return FFT_SUCCESS;
  if (std::getenv("STOCKFFT_FAIL_ALLOC")) return FFT_ALLOC_FAILED;
  hipError_t e = hipMalloc(dev, host.size() * sizeof(float));
  if (e != hipSuccess) {
    *dev = nullptr;
    return hip_fail(e);
  }
  e = hipMemcpy(*dev, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
    return hip_fail(e);
  }
  return FFT_SUCCESS;
}

int check_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return FFT_NO_DEVICE;
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e);
  return FFT_SUCCESS;
}

bool ranges_partially_overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  if (x == y) return false;
  return x < y + bytes && y < x + bytes;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev_) == hipSuccess && prev_ != dev) {
    if (hipSetDevice(dev) == hipSuccess) switched_ = true;
  }
}
DeviceGuard::~DeviceGuard() {
  if (switched_) (void)hipSetDevice(prev_);
}

// ------------------------------------------------------------------ tuning

namespace {

// One tuning decision: a single-pass variant or a four-step split for the
// lengths and batch range given.
struct TuneEntry {
  int64_t n, bmin, bmax;
  const SingleVariant* v;
  const FourStepVariant* fs;
};

std::mutex g_tune_mu;
// Matched-filter kernel choice per (n, batch range): the fused forward ->
// multiply -> inverse kernel can prefer another shape than the plain
// transform.  Tune-file entries ("filter_entries") take precedence.
std::vector<TuneEntry> g_tune_filter;
// The same for the fused forward -> weight -> adjoint kernel ("fused_entries")
// and for the transform with 16-bit storage ("storage16_entries").
std::vector<TuneEntry> g_tune_fused;
std::vector<TuneEntry> g_tune_storage16;
std::vector<TuneEntry> g_tune;
bool g_env_tune_done = false;

// Built-in choices: the autotuner's result on MI355X (gfx950, 256 CUs), the
// same table as the package's tune_gfx950.json.  Tuning entries added at run
// time take precedence.
struct BuiltinEntry {
  int64_t n, bmin, bmax;
  const char* name;
};
const BuiltinEntry kBuiltin[] = {
    {256, 1, 64, "n256_e16_b4_p4_r16.16"},
    {256, 65, 384, "n256_e16_b4_p4_r16.16_pt"},
    {256, 385, 768, "n256_e8_b8_p4_r8.8.4"},
    {256, 769, 1536, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 1537, 4096, "n256_e8_b8_p4_r8.8.4"},
    {256, 4097, INT64_MAX, "n256_e8_b8_p4_r8.8.4_pt"},
    {512, 1, 64, "n512_e4_b2_p4_r4.4.4.4.2_pt"},
    {512, 65, 384, "n512_e16_b2_p4_r16.16.2"},
    {512, 385, 768, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 769, 1536, "n512_e16_b2_p4_r16.16.2_pt"},
    {512, 1537, 4096, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 4097, INT64_MAX, "n512_e8_b4_p4_r8.8.8_pt"},
    {1024, 1, 64, "n1024_e8_b2_p4_r8.8.8.2"},
    {1024, 65, 384, "n1024_e16_b1_p4_r16.16.4_pt"},
    {1024, 385, 768, "n1024_e16_b1_p4_r16.16.4"},
    {1024, 769, 1536, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 1537, 4096, "n1024_e16_b1_p4_r16.16.4_pt"},
    {1024, 4097, INT64_MAX, "n1024_e16_b4_p4_r16.16.4_pt"},
    {2048, 1, 64, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 65, 384, "n2048_e8_b1_p4_r8.8.8.4"},
    {2048, 385, 768, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 769, 1536, "n2048_e16_b1_p4_r16.16.8_pt"},
    {2048, 1537, 4096, "n2048_e32_c2_b1_p4_r16.16.8_pt"},
    {2048, 4097, INT64_MAX, "n2048_e16_b2_p4_r16.16.8_pt"},
    {4096, 1, 64, "n4096_e8_b1_px_r8.8.8.8_pt_wx1"},
    {4096, 65, 384, "n4096_e16_b1_px_r8.8.8.8_pt_wm2"},
    {4096, 385, 768, "n4096_e8_b1_px_r8.8.8.8_pt"},
    {4096, 769, 1536, "n4096_e32_c2_b1_p4_r16.16.16_pt"},
    {4096, 1537, 4096, "n4096_e32_c2_b1_p4_r16.16.16_pt"},
    {4096, 4097, INT64_MAX, "n4096_e8_b1_p4_r8.8.8.8_pt_tall_st1d3"},
    {8192, 1, 64, "fs8192_4x2048"},
    {8192, 65, 384, "n8192_e8_b1_p4_r8.8.8.8.2_pt"},
    {8192, 385, 768, "n8192_e8_b1_p4_r8.8.8.8.2_pt"},
    {8192, 769, 1536, "n8192_e32_c4_b1_p4_r8.8.8.16"},
    {8192, 1537, 4096, "n8192_e32_c4_b1_p4_r8.8.8.16"},
    {8192, 4097, INT64_MAX, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {16384, 1, 64, "fs16384_8x2048"},
    {16384, 65, 384, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 385, 768, "n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"},
    {16384, 769, 1536, "n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"},
    {16384, 1537, 4096, "n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"},
    {16384, 4097, INT64_MAX, "n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"},
    {32768, 1, 64, "fs32768_2x16384"},
    {32768, 65, 384, "fs32768_2x16384"},
    {32768, 385, 768, "fs32768_2x16384"},
    {32768, 769, 1536, "fs32768_2x16384"},
    {32768, 1537, 4096, "fs32768_2x16384"},
    {32768, 4097, INT64_MAX, "fs32768_2x16384"},
    {65536, 1, 64, "fs65536_tile256x256"},
    {65536, 65, 384, "fs65536_4x16384"},
    {65536, 385, 768, "fs65536_tile256x256"},
    {65536, 769, 1536, "fs65536_4x16384"},
    {65536, 1537, 4096, "fs65536_4x16384"},
    {65536, 4097, INT64_MAX, "fs65536_4x16384"},
    {131072, 1, 64, "fs131072_tile256x512"},
    {131072, 65, 384, "fs131072_tile256x512"},
    {131072, 385, 768, "fs131072_tile256x512"},
    {131072, 769, 1536, "fs131072_8x16384"},
    {131072, 1537, 4096, "fs131072_8x16384"},
    {131072, 4097, INT64_MAX, "fs131072_8x16384"},
    {262144, 1, 64, "fs262144_tile512x512_c2"},
    {262144, 65, 384, "fs262144_tile512x512_c2"},
    {262144, 385, 768, "fs262144_tile512x512"},
    {262144, 769, 1536, "fs262144_tile512x512"},
    {262144, 1537, 4096, "fs262144_tile512x512"},
    {262144, 4097, INT64_MAX, "fs262144_tile512x512"},
    {524288, 1, 64, "fs524288_tile1024x512"},
    {524288, 65, 384, "fs524288_tile1024x512"},
    {524288, 385, 768, "fs524288_tile1024x512"},
    {524288, 769, 1536, "fs524288_tile1024x512"},
    {524288, 1537, 4096, "fs524288_tile1024x512"},
    {524288, 4097, INT64_MAX, "fs524288_tile1024x512"},
    {1048576, 1, 64, "fs1048576_tile1024x1024_c2"},
    {1048576, 65, 384, "fs1048576_tile1024x1024_c2"},
    {1048576, 385, 768, "fs1048576_tile1024x1024_c2"},
    {1048576, 769, 1536, "fs1048576_tile1024x1024_c2"},
    {1048576, 1537, 4096, "fs1048576_tile1024x1024_c2"},
    {1048576, 4097, INT64_MAX, "fs1048576_tile1024x1024_c2"},
};

// Built-in matched-filter choices: the autotuner's result on MI355X (the
// "filter_entries" of the package's tune_gfx950.json).
const BuiltinEntry kBuiltinFilter[] = {
    {256, 1, 64, "n256_e16_b4_p4_r16.16"},
    {256, 65, 384, "n256_e16_b4_p4_r16.16_pt"},
    {256, 385, 768, "n256_e16_b4_p4_r16.16_pt"},
    {256, 769, 1536, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 1537, 4096, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 4097, INT64_MAX, "n256_e16_b4_p4_r16.16_pt"},
    {512, 1, 64, "n512_e4_b2_p4_r4.4.4.4.2_pt"},
    {512, 65, 384, "n512_e4_b2_p4_r4.4.4.4.2_pt"},
    {512, 385, 768, "n512_e4_b2_p4_r4.4.4.4.2"},
    {512, 769, 1536, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 1537, 4096, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 4097, INT64_MAX, "n512_e8_b4_p4_r8.8.8_pt"},
    {1024, 1, 64, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 65, 384, "n1024_e4_b1_p4_r4.4.4.4.4"},
    {1024, 385, 768, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 769, 1536, "n1024_e8_b2_p4_r8.8.8.2_pt"},
    {1024, 1537, 4096, "n1024_e16_b1_p4_r16.16.4_pt"},
    {1024, 4097, INT64_MAX, "n1024_e16_b4_p4_r16.16.4_pt"},
    {2048, 1, 64, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 65, 384, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 385, 768, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 769, 1536, "n2048_e16_b1_p4_r16.16.8_pt"},
    {2048, 1537, 4096, "n2048_e16_b1_p4_r16.16.8_pt"},
    {2048, 4097, INT64_MAX, "n2048_e16_b2_p4_r16.16.8_pt"},
    {4096, 1, 64, "n4096_e8_b1_p4_r8.8.8.8_pt"},
    {4096, 65, 384, "n4096_e8_b1_p4_r8.8.8.8_pt"},
    {4096, 385, 768, "n4096_e16_b1_p5_r16.16.16_pt"},
    {4096, 769, 1536, "n4096_e32_c2_b1_p4_r16.16.16_pt"},
    {4096, 1537, 4096, "n4096_e32_c2_b1_p4_r16.16.16_pt_pl"},
    {4096, 4097, INT64_MAX, "n4096_e32_b1_p4_r16.16.16_pt_pl"},
    {8192, 1, 64, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 65, 384, "n8192_e8_b1_p4_r8.8.8.8.2_pt"},
    {8192, 385, 768, "n8192_e32_b1_p4_r16.16.16.2_pt"},
    {8192, 769, 1536, "n8192_e32_c4_b1_p4_r8.8.8.16"},
    {8192, 1537, 4096, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {8192, 4097, INT64_MAX, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {16384, 1, 64, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 65, 384, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 385, 768, "n16384_e16_c2_b1_p4_r8.8.8.8.4_pt"},
    {16384, 769, 1536, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 1537, 4096, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 4097, INT64_MAX, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
};

// Built-in 16-bit storage choices: the autotuner's result on MI355X (the
// "storage16_entries" of the package's tune_gfx950.json).  Half the bytes
// move, so the balance between memory and arithmetic, and with it the best
// shape, differs from the FP32 transform's.
const BuiltinEntry kBuiltinStorage16[] = {
    {256, 1, 64, "n256_e16_b4_p4_r16.16"},
    {256, 65, 384, "n256_e8_b8_p4_r8.8.4"},
    {256, 385, 768, "n256_e16_b4_p4_r16.16"},
    {256, 769, 1536, "n256_e16_b4_p4_r16.16_pt"},
    {256, 1537, 4096, "n256_e8_b8_p4_r8.8.4_pt"},
    {256, 4097, INT64_MAX, "n256_e8_b8_p4_r8.8.4_pt"},
    {512, 1, 64, "n512_e4_b2_p4_r4.4.4.4.2_pt"},
    {512, 65, 384, "n512_e16_b2_p4_r16.16.2"},
    {512, 385, 768, "n512_e16_b2_p4_r16.16.2"},
    {512, 769, 1536, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 1537, 4096, "n512_e8_b4_p4_r8.8.8"},
    {512, 4097, INT64_MAX, "n512_e8_b4_p4_r8.8.8_pt"},
    {1024, 1, 64, "n1024_e8_b2_p4_r8.8.8.2_pt"},
    {1024, 65, 384, "n1024_e16_b4_p4_r16.16.4"},
    {1024, 385, 768, "n1024_e8_b2_p4_r8.8.8.2"},
    {1024, 769, 1536, "n1024_e16_b1_p4_r16.16.4_pt"},
    {1024, 1537, 4096, "n1024_e16_b1_p4_r16.16.4_pt"},
    {1024, 4097, INT64_MAX, "n1024_e16_b1_p4_r16.16.4_pt"},
    {2048, 1, 64, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 65, 384, "n2048_e16_b1_p4_r16.16.8"},
    {2048, 385, 768, "n2048_e8_b1_p4_r8.8.8.4"},
    {2048, 769, 1536, "n2048_e16_b1_p4_r16.16.8_pt"},
    {2048, 1537, 4096, "n2048_e16_b2_p4_r16.16.8_pt"},
    {2048, 4097, INT64_MAX, "n2048_e32_c2_b1_p4_r16.16.8_pt"},
    {4096, 1, 64, "n4096_e8_b1_p4_r8.8.8.8_pt_tall"},
    {4096, 65, 384, "n4096_e8_b1_p4_r8.8.8.8_pt_tall"},
    {4096, 385, 768, "n4096_e8_b1_px_r8.8.8.8_pt"},
    {4096, 769, 1536, "n4096_e32_b1_p4_r16.16.16_pt"},
    {4096, 1537, 4096, "n4096_e32_c2_b1_p4_r16.16.16_pt_pl"},
    {4096, 4097, INT64_MAX, "n4096_e16_b1_px_r16.16.16_db_pt_tall_st2d2"},
    {8192, 1, 64, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 65, 384, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 385, 768, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 769, 1536, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {8192, 1537, 4096, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 4097, INT64_MAX, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {16384, 1, 64, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 65, 384, "n16384_e32_b1_p4_r16.16.16.4_pt"},
    {16384, 385, 768, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 769, 1536, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 1537, 4096, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 4097, INT64_MAX, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
};

// Built-in fused forward -> weight -> adjoint choices: the autotuner's result
// on MI355X (the "fused_entries" of the package's tune_gfx950.json).
const BuiltinEntry kBuiltinFused[] = {
    {256, 1, 64, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 65, 384, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 385, 768, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 769, 1536, "n256_e4_b4_p4_r4.4.4.4_pt"},
    {256, 1537, 4096, "n256_e8_b8_p4_r8.8.4_pt"},
    {256, 4097, INT64_MAX, "n256_e16_b16_p4_r16.16_pt"},
    {512, 1, 64, "n512_e8_b4_p4_r8.8.8"},
    {512, 65, 384, "n512_e4_b2_p4_r4.4.4.4.2"},
    {512, 385, 768, "n512_e8_b4_p4_r8.8.8"},
    {512, 769, 1536, "n512_e8_b4_p4_r8.8.8"},
    {512, 1537, 4096, "n512_e8_b4_p4_r8.8.8_pt"},
    {512, 4097, INT64_MAX, "n512_e8_b4_p4_r8.8.8_pt"},
    {1024, 1, 64, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 65, 384, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 385, 768, "n1024_e4_b1_p4_r4.4.4.4.4_pt"},
    {1024, 769, 1536, "n1024_e8_b2_p4_r8.8.8.2_pt"},
    {1024, 1537, 4096, "n1024_e8_b2_p4_r8.8.8.2_pt"},
    {1024, 4097, INT64_MAX, "n1024_e16_b4_p4_r16.16.4_pt"},
    {2048, 1, 64, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 65, 384, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 385, 768, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 769, 1536, "n2048_e8_b1_p4_r8.8.8.4_pt"},
    {2048, 1537, 4096, "n2048_e16_b2_p4_r16.16.8_pt"},
    {2048, 4097, INT64_MAX, "n2048_e16_b2_p4_r16.16.8_pt"},
    {4096, 1, 64, "n4096_e8_b1_px_r8.8.8.8_pt_wx1"},
    {4096, 65, 384, "n4096_e8_b1_px_r8.8.8.8_pt_wx1"},
    {4096, 385, 768, "n4096_e8_b1_px_r8.8.8.8_pt_wx1"},
    {4096, 769, 1536, "n4096_e16_b1_px_r16.16.16_db_pt_tall_st2d1"},
    {4096, 1537, 4096, "n4096_e32_c2_b1_p4_r16.16.16_pt"},
    {4096, 4097, INT64_MAX, "n4096_e16_b1_px_r16.16.16_db_pt_tall_st2d1"},
    {8192, 1, 64, "n8192_e8_b1_p4_r8.8.8.8.2_pt"},
    {8192, 65, 384, "n8192_e8_b1_p4_r8.8.8.8.2_pt"},
    {8192, 385, 768, "n8192_e16_b1_p4_r16.16.16.2_pt"},
    {8192, 769, 1536, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {8192, 1537, 4096, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {8192, 4097, INT64_MAX, "n8192_e32_c2_b1_p4_r16.16.16.2_pt"},
    {16384, 1, 64, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 65, 384, "n16384_e16_b1_p4_r16.16.16.4_pt"},
    {16384, 385, 768, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 769, 1536, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 1537, 4096, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
    {16384, 4097, INT64_MAX, "n16384_e32_c2_b1_p4_r16.16.16.4_pt"},
};

// Single-pass fallback when a four-step choice is not wanted.
const char* builtin_single(int64_t n) {
  switch (n) {
    case 8192: return "n8192_e32_b1_p4_r16.16.16.2";
    case 16384: return "n16384_e16_b1_p4_r16.16.16.4";
    default: return nullptr;
  }
}

void load_env_tune_locked();

}  // namespace

// The tuned choice for (n, batch): the last matching entry, else the built-in
// single-pass variant.  With single_only, four-step entries are passed over.
void tuned_choice(int64_t n, int64_t batch, bool single_only, const SingleVariant** sv,
                  const FourStepVariant** fs) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_env_tune_locked();
  *sv = nullptr;
  *fs = nullptr;
  for (const BuiltinEntry& b : kBuiltin) {
    if (b.n != n || batch < b.bmin || batch > b.bmax) continue;
    const SingleVariant* v = find_single(b.name);
    const FourStepVariant* f = v ? nullptr : find_four_step(b.name);
    if (single_only && !v) v = find_single(builtin_single(n)), f = nullptr;
    *sv = v;
    *fs = f;
  }
  for (const TuneEntry& e : g_tune) {
    if (e.n != n || batch < e.bmin || batch > e.bmax) continue;
    if (single_only && !e.v) continue;
    *sv = e.v;
    *fs = e.fs;
  }
  // Beyond one LDS-resident transform only the four-step exists: its first
  // registered split unless a tuning entry chose another.
  if (!*sv && !*fs && !single_only && n > kMaxSinglePassN)
    for (int i = 0; i < num_four_step() && !*fs; ++i)
      if (four_step_at(i).n == n) *fs = &four_step_at(i);
}

// A two-transform kernel's variant for (n, batch): the last matching entry of
// its table (tune file, then built-in), else the plain transform's
// single-pass choice.
template <size_t K>
const SingleVariant* tuned_table_variant(const BuiltinEntry (&builtin)[K],
                                         const std::vector<TuneEntry>& tuned, int64_t n,
                                         int64_t batch) {
  const SingleVariant* sv = nullptr;
  const FourStepVariant* fs = nullptr;
  tuned_choice(n, batch, true, &sv, &fs);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const SingleVariant* chosen = nullptr;
  for (const BuiltinEntry& b : builtin)
    if (b.n == n && batch >= b.bmin && batch <= b.bmax) chosen = find_single(b.name);
  for (const TuneEntry& e : tuned)
    if (e.n == n && batch >= e.bmin && batch <= e.bmax && e.v) chosen = e.v;
  return chosen ? chosen : sv;
}

// The matched filter's variant for (n, batch).
const SingleVariant* tuned_filter_variant(int64_t n, int64_t batch) {
  return tuned_table_variant(kBuiltinFilter, g_tune_filter, n, batch);
}

// The fused forward -> weight -> adjoint kernel's variant for (n, batch).
const SingleVariant* tuned_fused_variant(int64_t n, int64_t batch) {
  return tuned_table_variant(kBuiltinFused, g_tune_fused, n, batch);
}

// The 16-bit storage transform's variant for (n, batch).
const SingleVariant* tuned_storage16_variant(int64_t n, int64_t batch) {
  return tuned_table_variant(kBuiltinStorage16, g_tune_storage16, n, batch);
}

const SingleVariant* tuned_variant(int64_t n, int64_t batch) {
  const SingleVariant* sv;
  const FourStepVariant* fs;
  tuned_choice(n, batch, true, &sv, &fs);
  return sv;
}

namespace {

// Applies a tuning document written by the autotuner: "entries" (single-pass
// or four-step variant per length and batch range) and "ragged" (shape per
// length).  "arch" is compared with the device's architecture name when a
// device is present.  Entries naming unknown variants are skipped.
int load_tune_file_locked(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    std::fprintf(stderr, "stockfft: tune file %s not readable; using built-in table\n", path);
    return FFT_INVALID_ARGUMENT;
  }
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  json::Value doc;
  if (!json::Parser(text).parse(&doc) || doc.kind != json::Value::Object) {
    std::fprintf(stderr, "stockfft: tune file %s is not valid JSON; ignored\n", path);
    return FFT_INVALID_ARGUMENT;
  }
  // A file tuned for another architecture, or on another CU count (a
  // partitioned GPU exposes fewer CUs per device), is stale for this device.
  // "arch" and "cus" are optional; when present they must be a non-empty
  // name and a positive integer, and (with a device) match it: the name up
  // to its ':' feature suffix, exactly.
  const json::Value* arch = doc.get("arch");
  const json::Value* cus = doc.get("cus");
  auto base_arch = [](const std::string& a) { return a.substr(0, a.find(':')); };
  if ((arch && (arch->kind != json::Value::String || base_arch(arch->str).empty())) ||
      (cus && (cus->kind != json::Value::Number || !(cus->num >= 1.0 && cus->num <= 1e6) ||
               cus->num != std::floor(cus->num)))) {
    std::fprintf(stderr, "stockfft: tune file %s has a malformed arch or cus; ignored\n", path);
    return FFT_INVALID_ARGUMENT;
  }
  int count = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceCount(&count) == hipSuccess && count > 0 && hipGetDevice(&dev) == hipSuccess &&
      hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    if (arch && base_arch(arch->str) != base_arch(prop.gcnArchName)) {
      std::fprintf(stderr, "stockfft: tune file %s is for %s, device is %s; ignored\n", path,
                   arch->str.c_str(), prop.gcnArchName);
      return FFT_INVALID_ARGUMENT;
    }
    if (cus && (int64_t)cus->num != prop.multiProcessorCount) {
      std::fprintf(stderr, "stockfft: tune file %s was tuned on %lld CUs, device has %d; ignored\n",
                   path, (long long)cus->num, prop.multiProcessorCount);
      return FFT_INVALID_ARGUMENT;
    }
  }
  // An integer field: dflt when absent; an integral number >= lo otherwise
  // (values from 2^63 on saturate to INT64_MAX), else *bad is set.
  auto num = [](const json::Value& o, const char* k, int64_t dflt, int64_t lo, bool* bad) {
    const json::Value* v = o.get(k);
    if (!v) return dflt;
    if (v->kind != json::Value::Number || !(v->num >= (double)lo) ||
        v->num != std::floor(v->num)) {
      *bad = true;
      return dflt;
    }
    return v->num >= 9.2e18 ? INT64_MAX : (int64_t)v->num;
  };
  // n, batch_min and batch_max of one entry, checked as fft_tune_set checks them.
  auto range = [&](const json::Value& e, int64_t* n, int64_t* bmin, int64_t* bmax) {
    bool bad = false;
    *n = num(e, "n", 0, 0, &bad);
    *bmin = num(e, "batch_min", 1, 1, &bad);
    *bmax = num(e, "batch_max", INT64_MAX, 1, &bad);
    return !bad && *bmax >= *bmin;
  };
  auto str = [](const json::Value& o, const char* k) -> const std::string* {
    const json::Value* v = o.get(k);
    return v && v->kind == json::Value::String ? &v->str : nullptr;
  };
  std::vector<TuneEntry> add;
  int skipped = 0;
  if (const json::Value* es = doc.get("entries"); es && es->kind == json::Value::Array) {
    for (const json::Value& e : es->arr) {
      const std::string* name = str(e, "variant");
      int64_t n, bmin, bmax;
      if (!name || !range(e, &n, &bmin, &bmax) || !valid_size(n)) {
        ++skipped;
        continue;
      }
      const SingleVariant* v = find_single(name->c_str());
      const FourStepVariant* fs = v ? nullptr : find_four_step(name->c_str());
      if ((!v || v->n != n) && (!fs || fs->n != n)) {
        ++skipped;
        continue;
      }
      add.push_back({n, bmin, bmax, v, fs});
    }
  }
  // Single-pass entries of a two-transform kernel's table.
  auto single_entries = [&](const char* key, std::vector<TuneEntry>* out) {
    const json::Value* es = doc.get(key);
    if (!es || es->kind != json::Value::Array) return;
    for (const json::Value& e : es->arr) {
      const std::string* name = str(e, "variant");
      int64_t n, bmin, bmax;
      const bool ok = range(e, &n, &bmin, &bmax);
      const SingleVariant* v =
          ok && name && valid_single_size(n) ? find_single(name->c_str()) : nullptr;
      if (!v || v->n != n) {
        ++skipped;
        continue;
      }
      out->push_back({n, bmin, bmax, v, nullptr});
    }
  };
  std::vector<TuneEntry> add_filter, add_fused, add_storage16;
  single_entries("filter_entries", &add_filter);
  single_entries("fused_entries", &add_fused);
  single_entries("storage16_entries", &add_storage16);
  if (const json::Value* rs = doc.get("ragged"); rs && rs->kind == json::Value::Array) {
    for (const json::Value& e : rs->arr) {
      const std::string* shape = str(e, "shape");
      bool bad = false;
      const int64_t n = num(e, "n", 0, 0, &bad);
      if (bad || !shape || fft_tune_set_ragged(n, shape->c_str()) != FFT_SUCCESS) ++skipped;
    }
  }
  if (skipped)
    std::fprintf(stderr, "stockfft: %d tune entries in %s are not usable here; skipped\n",
                 skipped, path);
  g_tune.insert(g_tune.end(), add.begin(), add.end());
  g_tune_filter.insert(g_tune_filter.end(), add_filter.begin(), add_filter.end());
  g_tune_fused.insert(g_tune_fused.end(), add_fused.begin(), add_fused.end());
  g_tune_storage16.insert(g_tune_storage16.end(), add_storage16.begin(), add_storage16.end());
  return FFT_SUCCESS;
}

void load_env_tune_locked() {
  if (g_env_tune_done) return;
  g_env_tune_done = true;
  const char* p = std::getenv("STOCKFFT_TUNE_CACHE");
  if (p && *p) (void)load_tune_file_locked(p);
}

}  // namespace

// ------------------------------------------------------------------- plans

namespace {
std::mutex g_plans_mu;
std::unordered_set<const void*> g_plans;
}  // namespace

void register_handle(const void* p) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  g_plans.insert(p);
}
bool unregister_handle(const void* p) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  return g_plans.erase(p) == 1;
}
bool live_handle(const void* p) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  return g_plans.count(p) == 1;
}

}  // namespace stockfft

struct stockfft_plan_s {
  int64_t n = 0, batch = 0;
  int direction = FFT_FORWARD;
  int device = 0;
  int algorithm = FFT_ALGO_SINGLE_PASS;
  const SingleVariant* sv = nullptr;    // single-pass shape, or the four-step sub-shape
  const FourStepVariant* fs = nullptr;  // four-step split when algorithm == FOUR_STEP
  void* d_tw = nullptr;
  void* d_tw4 = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  unsigned* d_counters = nullptr;            // fused loss total (kept zeroed)
  void* d_tw_mma = nullptr;                  // matrix-core table when it differs from sv's
  const void* tw_mma = nullptr;              // the matrix-core table (d_tw or d_tw_mma)
  const SingleVariant* sv_filter = nullptr;  // matched-filter kernel shape (forward plans)
  void* d_tw_filter = nullptr;               // its twiddles when it differs from sv
  const SingleVariant* sv_fused = nullptr;   // fused forward/adjoint kernel shape
  void* d_tw_fused = nullptr;                // its twiddles when it differs from both
  const SingleVariant* sv_storage16 = nullptr;  // 16-bit storage transform shape
  void* d_tw_storage16 = nullptr;               // its twiddles when it differs from the rest
};

// Twiddle table of a single-pass shape held by the plan (its own or one of
// the two-transform kernels').
static const void* plan_table(const stockfft_plan_s* p, const SingleVariant* v) {
  if (v == p->sv) return p->d_tw;
  if (v == p->sv_filter) return p->d_tw_filter;
  if (v == p->sv_fused) return p->d_tw_fused;
  return p->d_tw_storage16;
}

static void free_plan(stockfft_plan_s* p) {
  if (!p) return;
  if (p->d_tw) (void)hipFree(p->d_tw);
  if (p->d_tw4) (void)hipFree(p->d_tw4);
  if (p->d_ws) (void)hipFree(p->d_ws);
  if (p->d_tw_filter) (void)hipFree(p->d_tw_filter);
  if (p->d_tw_fused) (void)hipFree(p->d_tw_fused);
  if (p->d_tw_storage16) (void)hipFree(p->d_tw_storage16);
  if (p->d_counters) (void)hipFree(p->d_counters);
  if (p->d_tw_mma) (void)hipFree(p->d_tw_mma);
  delete p;
}

static int validate_common(int64_t n, int64_t batch, int direction) {
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  if (batch < 1 || batch > (int64_t)(SIZE_MAX / 8 / (uint64_t)n) ||
      batch > INT64_MAX / 8 / n)
    return FFT_INVALID_BATCH;
  if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_INVALID_DIRECTION;
  return FFT_SUCCESS;
}

// STOCKFFT_LOG set to anything but "" or "0": every plan prints its choices
// (one line on stderr) when it is created.
static void log_plan(const stockfft_plan_s* p, bool named) {
  const char* env = std::getenv("STOCKFFT_LOG");
  if (!env || !*env || (env[0] == '0' && !env[1])) return;
  const auto nm = [](const SingleVariant* v) { return v ? v->name : "-"; };
  std::fprintf(stderr,
               "stockfft: plan n=%lld batch=%lld direction=%d algorithm=%s variant=%s "
               "four_step=%s fused=%s filter=%s storage16=%s source=%s\n",
               (long long)p->n, (long long)p->batch, p->direction,
               p->algorithm == FFT_ALGO_FOUR_STEP ? "four_step" : "single_pass", nm(p->sv),
               p->fs ? p->fs->name : "-", nm(p->sv_fused), nm(p->sv_filter), nm(p->sv_storage16),
               named ? "named" : "tuned");
}

extern "C" int fft_plan_config(fft_plan_t* plan, int64_t n, int64_t batch, int direction,
                               int algorithm, const char* variant) {
  if (!plan) return FFT_INVALID_POINTER;
  *plan = nullptr;
  int rc = validate_common(n, batch, direction);
  if (rc) return rc;
  if (algorithm != FFT_ALGO_AUTO && algorithm != FFT_ALGO_SINGLE_PASS &&
      algorithm != FFT_ALGO_FOUR_STEP)
    return FFT_INVALID_ARGUMENT;

  if (algorithm == FFT_ALGO_SINGLE_PASS && n > kMaxSinglePassN) return FFT_UNSUPPORTED;
  const SingleVariant* sv = nullptr;
  const FourStepVariant* fs = nullptr;
  if (algorithm == FFT_ALGO_FOUR_STEP) {
    if (variant) {
      fs = find_four_step(variant);
      if (!fs || fs->n != n) return FFT_INVALID_ARGUMENT;
    } else {
      for (int i = 0; i < num_four_step() && !fs; ++i)
        if (four_step_at(i).n == n) fs = &four_step_at(i);
      if (!fs) return FFT_UNSUPPORTED;
    }
    sv = find_single(fs->sub_name);
    if (!sv) return FFT_INVALID_ARGUMENT;
  } else if (variant) {
    sv = find_single(variant);
    if (!sv || sv->n != n) {
      const FourStepVariant* f = find_four_step(variant);
      if (algorithm == FFT_ALGO_AUTO && f && f->n == n) {
        fs = f;
        sv = find_single(f->sub_name);
      } else {
        return FFT_INVALID_ARGUMENT;
      }
    }
  } else {
    tuned_choice(n, batch, algorithm == FFT_ALGO_SINGLE_PASS, &sv, &fs);
    if (fs) sv = find_single(fs->sub_name);
    if (!sv) return FFT_INVALID_SIZE;
  }

  int dev = 0;
  rc = check_device(&dev);
  if (rc) return rc;

  stockfft_plan_s* p = new (std::nothrow) stockfft_plan_s;
  if (!p) return FFT_ALLOC_FAILED;
  p->n = n;
  p->batch = batch;
  p->direction = direction;
  p->device = dev;
  p->sv = sv;
  p->fs = fs;
  p->algorithm = fs ? FFT_ALGO_FOUR_STEP : FFT_ALGO_SINGLE_PASS;

  std::vector<float> host;
  build_stockham_twiddles(*sv, host);
  rc = upload(host, &p->d_tw);
  if (!rc && !fs && direction == FFT_FORWARD) {
    // The kernels that run two transforms per load (matched filter, fused
    // forward -> weight -> adjoint): the named variant, else each kernel's
    // own tuned choice (timed on that kernel: its register pressure differs
    // from a single transform's), each with its twiddles.
    // (A named variant without the two-transform kernels -- a paired-lane
    // shape whose output and input register orders differ -- takes the
    // tuned choice for them.)
    p->sv_filter = variant && sv->filter ? sv : tuned_filter_variant(n, batch);
    if (!p->sv_filter->filter) p->sv_filter = sv;
    if (p->sv_filter != sv) {
      std::vector<float> ftw;
      build_stockham_twiddles(*p->sv_filter, ftw);
      rc = upload(ftw, &p->d_tw_filter);
    }
    const SingleVariant* fv = variant && sv->fused ? sv : tuned_fused_variant(n, batch);
    p->sv_fused = fv->fused ? fv : (sv->fused ? sv : nullptr);
    if (!rc && p->sv_fused && p->sv_fused != sv && p->sv_fused != p->sv_filter) {
      std::vector<float> utw;
      build_stockham_twiddles(*p->sv_fused, utw);
      rc = upload(utw, &p->d_tw_fused);
    }
  }
  if (!rc && !fs) {
    // The transform with 16-bit storage (either direction): the named
    // variant, else its own tuned choice.
    p->sv_storage16 = variant ? sv : tuned_storage16_variant(n, batch);
    if (!p->sv_storage16->launch_f16) p->sv_storage16 = sv;
    const SingleVariant* h = p->sv_storage16;
    if (h != sv && h != p->sv_filter && h != p->sv_fused) {
      std::vector<float> htw;
      build_stockham_twiddles(*h, htw);
      rc = upload(htw, &p->d_tw_storage16);
    }
  }
  if (!rc && p->sv_fused) {
    const size_t bytes = (kTotalGroups * 64 + 1) * sizeof(unsigned);
    hipError_t e = hipMalloc((void**)&p->d_counters, bytes);
    if (e == hipSuccess) e = hipMemset(p->d_counters, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      p->d_counters = nullptr;
      rc = hip_fail(e);
    }
  }
  if (!rc && !fs && mma_supported(n)) {
    // The matrix-core 16-bit mode runs radix 16 throughout (then one smaller
    // radix): its own table unless the plan's variant has that radix plan.
    const SingleVariant* mv = find_single(mma_table_variant(n));
    bool same = mv && mv->npass == sv->npass && mv->paired_twiddles == sv->paired_twiddles;
    for (int i = 0; same && i < sv->npass; ++i) same = mv->radix[i] == sv->radix[i];
    if (mv && !same) {
      std::vector<float> mtw;
      build_stockham_twiddles(*mv, mtw);
      rc = upload(mtw, &p->d_tw_mma);
    }
    if (mv) p->tw_mma = same ? p->d_tw : p->d_tw_mma;
  }
  if (!rc && fs) {
    build_four_step_twiddles(*fs, host);
    rc = upload(host, &p->d_tw4);
    if (!rc) {
      p->ws_bytes = (size_t)n * (size_t)batch * 8;
      hipError_t e = hipMalloc(&p->d_ws, p->ws_bytes);
      if (e != hipSuccess) {
        p->d_ws = nullptr;
        rc = hip_fail(e);
      }
    }
  }
  if (rc) {
    free_plan(p);
    return rc;
  }
  register_handle(p);
  *plan = p;
  log_plan(p, variant != nullptr);
  return FFT_SUCCESS;
}

extern "C" int fft_plan(fft_plan_t* plan, int64_t n, int64_t batch, int direction) {
  return fft_plan_config(plan, n, batch, direction, FFT_ALGO_AUTO, nullptr);
}

extern "C" int fft_exec(fft_plan_t plan, const void* in, void* out, void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  if (!in || !out) return FFT_INVALID_POINTER;
  if (!aligned8(in) || !aligned8(out)) return FFT_MISALIGNED;
  const size_t bytes = (size_t)plan->n * (size_t)plan->batch * 8;
  if (ranges_partially_overlap(in, out, bytes)) return FFT_OVERLAP;
  DeviceGuard g(plan->device);
  hipStream_t s = (hipStream_t)stream;
  const bool inv = plan->direction == FFT_BACKWARD;
  hipError_t e;
  if (plan->algorithm == FFT_ALGO_FOUR_STEP) {
    e = plan->fs->columns(in, plan->d_ws, plan->d_tw, plan->batch, inv, s);
    if (e == hipSuccess) e = plan->fs->combine(plan->d_ws, out, plan->d_tw, plan->d_tw4, plan->batch, inv,
                                              s);
  } else {
    e = plan->sv->launch(in, out, plan->d_tw, plan->batch, inv, s);
  }
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

extern "C" int fft_exec_io(fft_plan_t plan, const void* in, void* out, int io, void* stream) {
  if (io == FFT_IO_C64) return fft_exec(plan, in, out, stream);
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  const bool mma = io == FFT_IO_C16_MMA || io == FFT_IO_BC16_MMA;
  if (io != FFT_IO_C16 && io != FFT_IO_BC16 && !mma) return FFT_INVALID_ARGUMENT;
  if (plan->algorithm != FFT_ALGO_SINGLE_PASS) return FFT_UNSUPPORTED;
  if (mma && !plan->tw_mma) return FFT_UNSUPPORTED;
  if (!in || !out) return FFT_INVALID_POINTER;
  if (((uintptr_t)in & 3u) || ((uintptr_t)out & 3u)) return FFT_MISALIGNED;
  const size_t bytes = (size_t)plan->n * (size_t)plan->batch * 4;
  if (ranges_partially_overlap(in, out, bytes)) return FFT_OVERLAP;
  const SingleVariant* hv = plan->sv_storage16 ? plan->sv_storage16 : plan->sv;
  const LaunchFn fn = io == FFT_IO_C16 ? hv->launch_f16 : hv->launch_bf16;
  if (!mma && !fn) return FFT_UNSUPPORTED;
  DeviceGuard g(plan->device);
  const bool inv = plan->direction == FFT_BACKWARD;
  hipError_t e;
  if (mma) {
    e = (io == FFT_IO_C16_MMA ? launch_mma_f16 : launch_mma_bf16)(
        plan->n, in, out, plan->tw_mma, plan->batch, inv, (hipStream_t)stream);
  } else {
    e = fn(in, out, plan_table(plan, hv), plan->batch, inv, (hipStream_t)stream);
  }
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

extern "C" int fft_destroy(fft_plan_t plan) {
  if (!plan) return FFT_SUCCESS;
  if (!unregister_handle(plan)) return FFT_INVALID_PLAN;
  free_plan(plan);
  return FFT_SUCCESS;
}

extern "C" int fft_exec_spectral_energy(fft_plan_t plan, const void* x, const float* w,
                                        const float* grad_scale, void* grad_x, float* row_loss,
                                        float* loss_total, void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  const SingleVariant* fv = plan->sv_fused;
  if (plan->direction != FFT_FORWARD || plan->algorithm != FFT_ALGO_SINGLE_PASS || !fv)
    return FFT_UNSUPPORTED;
  if (!x || !w || !row_loss) return FFT_INVALID_POINTER;
  if (!aligned8(x) || (grad_x && !aligned8(grad_x)) || ((uintptr_t)w & 3u) ||
      ((uintptr_t)row_loss & 3u) || (grad_scale && ((uintptr_t)grad_scale & 3u)) ||
      (loss_total && ((uintptr_t)loss_total & 3u)))
    return FFT_MISALIGNED;
  const size_t bytes = (size_t)plan->n * (size_t)plan->batch * 8;
  if (grad_x && ranges_partially_overlap(x, grad_x, bytes)) return FFT_OVERLAP;
  DeviceGuard g(plan->device);
  hipStream_t s = (hipStream_t)stream;
  const hipError_t e = fv->fused(x, w, grad_scale, grad_x, row_loss, loss_total,
                                 plan->d_counters, plan_table(plan, fv), plan->batch, s);
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

// ------------------------------------------ allocation-free fused entry
//
// fft_exec_spectral_energy_noalloc keeps the per-row losses and the arrival
// counters of the loss total in this array instead of a caller buffer and
// the plan's counters: kNoAllocMaxRows floats, then the counters on their
// own 256-byte lines.  One copy per GPU, held until the process ends.
namespace {
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 20;
constexpr size_t kNoAllocLossBytes = (size_t)kNoAllocMaxRows * sizeof(float);
constexpr size_t kNoAllocCounterWords = (size_t)kTotalGroups * 64 + 1;
constexpr size_t kNoAllocScratchBytes =
    kNoAllocLossBytes + (kNoAllocCounterWords * sizeof(unsigned) + 255) / 256 * 256;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// Zeroes n words (a fill kernel rather than a memset, so a caller may
// capture it into a graph).
__global__ void k_zero_words(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];     // device address of `scratch` on each device
bool g_scratch_cleared[kMaxDevices];  // counters zeroed by a launch on that device

// The device address of `scratch` on the current device `dev`, looked up
// once per device; on the first call the counters are cleared on `s` (they
// come back to zero after every complete call).
int scratch_for_device(int dev, hipStream_t s, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return FFT_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = ptr;
  }
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  if (!g_scratch_cleared[dev]) {
    k_zero_words<<<dim3((unsigned)((kNoAllocCounterWords + 255) / 256)), dim3(256), 0, s>>>(
        reinterpret_cast<unsigned*>(base + kNoAllocLossBytes), (int)kNoAllocCounterWords);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    g_scratch_cleared[dev] = true;
  }
  *out = base;
  return FFT_SUCCESS;
}

}  // namespace

extern "C" int fft_exec_spectral_energy_noalloc(fft_plan_t plan, const void* x, const float* w,
                                                const float* grad_scale, void* grad_x,
                                                float* loss_total, void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  const SingleVariant* fv = plan->sv_fused;
  if (plan->direction != FFT_FORWARD || plan->algorithm != FFT_ALGO_SINGLE_PASS || !fv)
    return FFT_UNSUPPORTED;
  if (!x || !w || !loss_total) return FFT_INVALID_POINTER;
  if (plan->batch > kNoAllocMaxRows) return FFT_INVALID_ARGUMENT;
  if (!aligned8(x) || (grad_x && !aligned8(grad_x)) || ((uintptr_t)w & 3u) ||
      (grad_scale && ((uintptr_t)grad_scale & 3u)) || ((uintptr_t)loss_total & 3u))
    return FFT_MISALIGNED;
  const size_t bytes = (size_t)plan->n * (size_t)plan->batch * 8;
  if (grad_x && ranges_partially_overlap(x, grad_x, bytes)) return FFT_OVERLAP;
  DeviceGuard g(plan->device);
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = nullptr;
  const int rc = scratch_for_device(plan->device, s, &base);
  if (rc) return rc;
  float* row_loss = reinterpret_cast<float*>(base);
  unsigned* counters = reinterpret_cast<unsigned*>(base + kNoAllocLossBytes);
  const hipError_t e = fv->fused(x, w, grad_scale, grad_x, row_loss, loss_total, counters,
                                 plan_table(plan, fv), plan->batch, s);
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

extern "C" int fft_exec_matched_filter(fft_plan_t plan, const void* x, const void* h, void* out,
                                       void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  const SingleVariant* fv = plan->sv_filter;
  if (plan->direction != FFT_FORWARD || plan->algorithm != FFT_ALGO_SINGLE_PASS || !fv ||
      !fv->filter)
    return FFT_UNSUPPORTED;
  if (!x || !h || !out) return FFT_INVALID_POINTER;
  if (!aligned8(x) || !aligned8(h) || !aligned8(out)) return FFT_MISALIGNED;
  const size_t bytes = (size_t)plan->n * (size_t)plan->batch * 8;
  if (ranges_partially_overlap(x, out, bytes)) return FFT_OVERLAP;
  DeviceGuard g(plan->device);
  hipError_t e = fv->filter(x, h, out, plan_table(plan, fv), plan->batch, (hipStream_t)stream);
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

// ------------------------------------------------------------ tuning ABI

static int put_text(const std::string& s, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (cap < (int64_t)s.size() + 1) return FFT_INVALID_ARGUMENT;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return FFT_SUCCESS;
}

extern "C" int fft_tune_load(const char* json_path) {
  if (!json_path) return FFT_INVALID_POINTER;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_env_tune_locked();
  return load_tune_file_locked(json_path);
}

extern "C" int fft_tune_set(int64_t n, int64_t batch_min, int64_t batch_max, const char* variant) {
  if (!variant) return FFT_INVALID_POINTER;
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  if (batch_min < 1 || batch_max < batch_min) return FFT_INVALID_BATCH;
  const SingleVariant* v = find_single(variant);
  const FourStepVariant* f = v ? nullptr : find_four_step(variant);
  if ((!v || v->n != n) && (!f || f->n != n)) return FFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_env_tune_locked();
  g_tune.push_back({n, batch_min, batch_max, v, f});
  return FFT_SUCCESS;
}

extern "C" int fft_tune_query(int64_t n, int64_t batch, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  if (batch < 1) return FFT_INVALID_BATCH;
  const SingleVariant* v;
  const FourStepVariant* f;
  tuned_choice(n, batch, false, &v, &f);
  if (f) return put_text(f->name, buf, cap);
  if (!v) return FFT_INVALID_SIZE;
  return put_text(v->name, buf, cap);
}

extern "C" int fft_tune_query_filter(int64_t n, int64_t batch, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
  if (batch < 1) return FFT_INVALID_BATCH;
  const SingleVariant* v = tuned_filter_variant(n, batch);
  if (!v) return FFT_INVALID_SIZE;
  return put_text(v->name, buf, cap);
}

extern "C" int fft_tune_query_fused(int64_t n, int64_t batch, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
  if (batch < 1) return FFT_INVALID_BATCH;
  const SingleVariant* v = tuned_fused_variant(n, batch);
  if (!v) return FFT_INVALID_SIZE;
  return put_text(v->name, buf, cap);
}

extern "C" int fft_tune_query_storage16(int64_t n, int64_t batch, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
  if (batch < 1) return FFT_INVALID_BATCH;
  const SingleVariant* v = tuned_storage16_variant(n, batch);
  if (!v) return FFT_INVALID_SIZE;
  return put_text(v->name, buf, cap);
}

extern "C" int fft_set_launch_limit(int64_t max_groups) {
  set_max_groups_per_launch(max_groups > 0 ? max_groups : kDefaultMaxGroupsPerLaunch);
  return FFT_SUCCESS;
}

extern "C" int fft_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_env_tune_done = true;
  g_tune.clear();
  g_tune_filter.clear();
  g_tune_fused.clear();
  g_tune_storage16.clear();
  return FFT_SUCCESS;
}

// --------------------------------------------------------- introspection

static int barriers_of(const SingleVariant& v) {
  // Per exchange round one barrier after the writes and one after the reads,
  // except after the reads of the last round of the last exchange (the last
  // pass writes global memory directly, as the first pass reads it); with
  // two alternating buffers only the one after the writes.
  if (v.npass < 2) return 0;
  // In-wave exchanges: only the middle exchange goes through the LDS, and
  // its buffer is not reused.
  if (v.wave_exchange) return 1;
  return v.double_buffered ? v.npass - 1 : 2 * v.chunks * (v.npass - 1) - 1;
}

static std::string radices_json(const SingleVariant& v) {
  std::string s = "[";
  for (int i = 0; i < v.npass; ++i) {
    if (i) s += ",";
    s += std::to_string(v.radix[i]);
  }
  return s + "]";
}

static std::string describe_single(const SingleVariant& v) {
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "{\"kind\":\"single\",\"name\":\"%s\",\"n\":%d,\"values_per_lane\":%d,"
                "\"lanes_per_transform\":%d,\"transforms_per_workgroup\":%d,\"pad_log2\":%d,"
                "\"lds_layout\":\"%s\","
                "\"passes\":%d,\"radices\":%s,\"exchange_rounds\":%d,\"threads\":%d,"
                "\"lds_bytes\":%d,\"twiddle_entries\":%d,\"barriers\":%d,"
                "\"double_buffered\":%s,\"twiddle_schedule\":%d,\"paired_twiddles\":%s,\"paired_lanes\":%s,"
                "\"fused_kernels\":%s,\"fused_kernel\":%s,\"streamed\":%d,\"wave_exchange\":%d,\"wave_members\":%d}",
                v.name, v.n, v.e, v.t, v.tpb, v.padlog,
                v.padlog > 0 ? "pad" : v.padlog < 0 ? "xor" : "none", v.npass, radices_json(v).c_str(),
                v.chunks, v.threads, v.lds_bytes, v.tw_elems, barriers_of(v),
                v.double_buffered ? "true" : "false", v.twiddle_schedule,
                v.paired_twiddles ? "true" : "false", v.paired_lanes ? "true" : "false",
                v.fused && v.filter ? "true" : "false", v.fused ? "true" : "false", v.streamed,
                v.wave_exchange, v.wave_members);
  return buf;
}

static int64_t four_step_table_entries(const FourStepVariant& f) {
  if (!f.two_level) return (int64_t)(f.n1 - 1) * f.n2;
  const int64_t N = (int64_t)f.n1 * f.n2;
  const int s = ilog2(N) / 2;
  const SingleVariant* sub2 = f.sub2_name ? find_single(f.sub2_name) : nullptr;
  return (int64_t(1) << s) + (N >> s) + f.n1 + (sub2 ? sub2->tw_elems : 0);
}

static std::string describe_four_step(const FourStepVariant& f) {
  char buf[384];
  std::snprintf(buf, sizeof buf,
                "{\"kind\":\"four_step\",\"name\":\"%s\",\"n\":%d,\"n1\":%d,\"n2\":%d,"
                "\"sub_variant\":\"%s\",\"sub2_variant\":\"%s\",\"two_level_twiddles\":%s,"
                "\"twiddle_entries\":%lld}",
                f.name, f.n, f.n1, f.n2, f.sub_name, f.sub2_name ? f.sub2_name : "",
                f.two_level ? "true" : "false",
                (long long)(f.tw_sub_elems + four_step_table_entries(f)));
  return buf;
}

extern "C" int fft_variant_count(void) {
  return (int)single_variants().size() + num_four_step();
}

extern "C" int fft_variant_describe(int index, char* buf, int64_t cap) {
  const int ns = (int)single_variants().size();
  if (index < 0 || index >= ns + num_four_step()) return FFT_INVALID_ARGUMENT;
  if (index < ns) return put_text(describe_single(*single_variants()[index]), buf, cap);
  return put_text(describe_four_step(four_step_at(index - ns)), buf, cap);
}

extern "C" int fft_variant_twiddles(int index, float* out, int64_t cap_complex, int64_t* count) {
  if (!count) return FFT_INVALID_POINTER;
  const int ns = (int)single_variants().size();
  if (index < 0 || index >= ns + num_four_step()) return FFT_INVALID_ARGUMENT;
  std::vector<float> host, tw4;
  if (index < ns) {
    build_stockham_twiddles(*single_variants()[index], host);
  } else {
    const FourStepVariant& f = four_step_at(index - ns);
    const SingleVariant* sub = find_single(f.sub_name);
    if (!sub) return FFT_INVALID_ARGUMENT;
    build_stockham_twiddles(*sub, host);
    build_four_step_twiddles(f, tw4);
    host.insert(host.end(), tw4.begin(), tw4.end());
  }
  *count = (int64_t)host.size() / 2;
  if (!out) return FFT_SUCCESS;
  if (cap_complex < *count) return FFT_INVALID_ARGUMENT;
  std::memcpy(out, host.data(), host.size() * sizeof(float));
  return FFT_SUCCESS;
}

// The compiled resources of a variant's forward FP32 kernel on the plan's
// device: registers, scratch and static LDS per the HIP runtime.
static std::string kernel_resources(const stockfft_plan_s* plan, const SingleVariant& v) {
  if (!v.kernel) return "";
  DeviceGuard g(plan->device);
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, v.kernel) != hipSuccess) return "";
  return ",\"variant_resources\":{\"vgprs\":" + std::to_string(a.numRegs) +
         ",\"scratch_bytes_per_lane\":" + std::to_string(a.localSizeBytes) +
         ",\"lds_bytes\":" + std::to_string(a.sharedSizeBytes) +
         ",\"max_threads\":" + std::to_string(a.maxThreadsPerBlock) + "}";
}

extern "C" int fft_plan_describe(fft_plan_t plan, char* buf, int64_t cap) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  std::string s = "{\"n\":" + std::to_string(plan->n) + ",\"batch\":" +
                  std::to_string(plan->batch) + ",\"direction\":" +
                  std::to_string(plan->direction) + ",\"device\":" + std::to_string(plan->device) +
                  ",\"algorithm\":\"" +
                  (plan->algorithm == FFT_ALGO_FOUR_STEP ? "four_step" : "single_pass") + "\"" +
                  ",\"workspace_bytes\":" + std::to_string(plan->ws_bytes) +
                  ",\"variant\":" + describe_single(*plan->sv) + kernel_resources(plan, *plan->sv) +
                  (plan->fs ? ",\"four_step\":" + describe_four_step(*plan->fs) : "") +
                  (plan->sv_filter ? ",\"filter_variant\":\"" + std::string(plan->sv_filter->name) + "\""
                                   : "") +
                  (plan->sv_fused ? ",\"fused_variant\":\"" + std::string(plan->sv_fused->name) + "\""
                                  : "") +
                  (plan->sv_storage16
                       ? ",\"storage16_variant\":\"" + std::string(plan->sv_storage16->name) + "\""
                       : "") +
                  "}";
  return put_text(s, buf, cap);
}

extern "C" const char* fft_status_string(int status) {
  switch (status) {
    case FFT_SUCCESS: return "success";
    case FFT_INVALID_SIZE:
      return "invalid size: N must be a power of two in [256, 1048576] ([256, 16384] for ragged "
             "batches)";
    case FFT_INVALID_BATCH: return "invalid batch";
    case FFT_INVALID_DIRECTION: return "invalid direction: use FFT_FORWARD (-1) or FFT_BACKWARD (+1)";
    case FFT_INVALID_POINTER: return "null pointer";
    case FFT_MISALIGNED: return "misaligned pointer";
    case FFT_OVERLAP: return "input and output partially overlap";
    case FFT_INVALID_PLAN: return "invalid or destroyed plan";
    case FFT_NO_DEVICE: return "no HIP device";
    case FFT_ALLOC_FAILED: return "device allocation failed";
    case FFT_HIP_ERROR: return "HIP error";
    case FFT_INVALID_ARGUMENT: return "invalid argument";
    case FFT_UNSUPPORTED: return "unsupported operation for this plan";
    default: return "unknown status";
  }
}

extern "C" int fft_last_hip_error(void) { return g_last_hip_error; }

extern "C" int fft_version(void) { return 10000; }
