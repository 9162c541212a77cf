// Ragged batches: transforms of different power-of-two lengths, packed one
// after another, run by one persistent kernel launched from a hipGraph.
//
// Every persistent workgroup has 1024 lanes and the LDS of the largest shape
// (a whole 16384-point transform plus pad).  Work is cut into tasks of one
// size class each; a task is as many transforms of that size as one
// workgroup holds under the shape chosen for the size (the radix / lanes per
// transform / LDS tile picked by the autotuner).  Tasks are ordered longest
// transform first and taken from a device queue counter, so the big
// transforms start early and the small ones fill the tail.  The counter
// resets itself: the last workgroup to leave clears it, so the graph holds a
// single kernel node and no memset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/stockfft.h"
#include "internal.hpp"
#include "kernels.hpp"

namespace stockfft {
namespace {

constexpr int kRaggedThreads = 1024;

// Candidate shapes per size class, all with 1024 lanes per workgroup.
// Radix-16 passes (16 values per lane, 16384 / N transforms per task):
using G256 = Shape<256, 16, 64, 4, 16, 16>;
using G512 = Shape<512, 16, 32, 4, 16, 16, 2>;
using G1024 = Shape<1024, 16, 16, 4, 16, 16, 4>;
using G2048 = Shape<2048, 16, 8, 4, 16, 16, 8>;
using G4096 = Shape<4096, 16, 4, 4, 16, 16, 16>;
using G8192 = Shape<8192, 16, 2, 4, 16, 16, 16, 2>;
using G16384 = Shape<16384, 16, 1, 4, 16, 16, 16, 4>;
// Radix-8 passes (8 values per lane, twice the lanes per transform):
using H256 = Shape<256, 8, 32, 4, 8, 8, 4>;
using H512 = Shape<512, 8, 16, 4, 8, 8, 8>;
using H1024 = Shape<1024, 8, 8, 4, 8, 8, 8, 2>;
using H2048 = Shape<2048, 8, 4, 4, 8, 8, 8, 4>;
using H4096 = Shape<4096, 8, 2, 4, 8, 8, 8, 8>;
using H8192 = Shape<8192, 8, 1, 4, 8, 8, 8, 8, 2>;

constexpr int kNumShapes = 13;
constexpr int kLdsElems = G16384::LDS_ELEMS;

struct ShapeInfo {
  const char* name;
  int n, e, tpb, npass;
  int radix[kMaxPasses];
};

template <class S>
constexpr ShapeInfo info(const char* name) {
  ShapeInfo s{name, S::N, S::E, S::TPB, S::P, {}};
  for (int i = 0; i < S::P; ++i) s.radix[i] = S::radix(i);
  return s;
}

const ShapeInfo kShapes[kNumShapes] = {
    info<G256>("ragged_n256_e16"),   info<G512>("ragged_n512_e16"),
    info<G1024>("ragged_n1024_e16"), info<G2048>("ragged_n2048_e16"),
    info<G4096>("ragged_n4096_e16"), info<G8192>("ragged_n8192_e16"),
    info<G16384>("ragged_n16384_e16"), info<H256>("ragged_n256_e8"),
    info<H512>("ragged_n512_e8"),    info<H1024>("ragged_n1024_e8"),
    info<H2048>("ragged_n2048_e8"),  info<H4096>("ragged_n4096_e8"),
    info<H8192>("ragged_n8192_e8"),
};

struct Task {
  int32_t shape;  // index into kShapes
  int32_t count;  // transforms in this task (<= the shape's TPB)
  int64_t first;  // index of the first transform's offset in item_off
};

struct Queue {
  int next;  // next task to hand out
  int done;  // workgroups that have left
};

struct RaggedArgs {
  const c32* in;
  c32* out;
  const Task* tasks;
  const int64_t* item_off;
  Queue* queue;
  int ntasks;
  const c32* tw[kNumShapes];
};

// One task body per shape, kept out of line: inlined together into the one
// dispatching kernel, the thirteen bodies' register arrays would no longer
// be promoted to VGPRs.
template <class S, bool INV>
__device__ __noinline__ void run_task(const c32* in, c32* out, const int64_t* item_off,
                                      int64_t first, int count, c32* lds_all, const c32* tw) {
  static_assert(S::THREADS == kRaggedThreads, "ragged shapes use 1024 lanes");
  static_assert(S::TPB * S::LDS_ELEMS <= kLdsElems, "shape exceeds the persistent LDS");
  const int tid = threadIdx.x;
  const int slot = tid / S::T;
  const int t = tid - slot * S::T;
  const bool live = slot < count;
  const int64_t off = live ? item_off[first + slot] : 0;
  c32* lds = lds_all + slot * S::LDS_ELEMS;
  c32 a[S::E];
  global_load_row<S>(a, in + off, t, live);
  run_passes<S, INV>(a, lds, tw, t);
  global_store_row<S>(a, out + off, t, live);
}

template <bool INV>
__global__ __launch_bounds__(kRaggedThreads) void k_ragged(RaggedArgs A) {
  __shared__ c32 lds_all[kLdsElems];
  __shared__ int s_task;
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(&A.queue->next, 1);
    __syncthreads();
    const int task = s_task;
    __syncthreads();  // every lane has read s_task before lane 0 rewrites it
    if (task >= A.ntasks) break;
    const Task tk = A.tasks[task];
    switch (tk.shape) {
      case 0: run_task<G256, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[0]); break;
      case 1: run_task<G512, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[1]); break;
      case 2: run_task<G1024, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[2]); break;
      case 3: run_task<G2048, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[3]); break;
      case 4: run_task<G4096, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[4]); break;
      case 5: run_task<G8192, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[5]); break;
      case 6: run_task<G16384, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[6]); break;
      case 7: run_task<H256, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[7]); break;
      case 8: run_task<H512, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[8]); break;
      case 9: run_task<H1024, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[9]); break;
      case 10: run_task<H2048, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[10]); break;
      case 11: run_task<H4096, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[11]); break;
      default: run_task<H8192, INV>(A.in, A.out, A.item_off, tk.first, tk.count, lds_all, A.tw[12]); break;
    }
    __syncthreads();  // the task's last LDS reads are done before the next task writes
  }
  // Every workgroup took exactly one out-of-range ticket before arriving
  // here, so when the last one arrives nobody touches the counter again in
  // this launch: it resets both counters for the next launch.
  if (threadIdx.x == 0) {
    __threadfence();
    const int d = atomicAdd(&A.queue->done, 1);
    if (d == (int)gridDim.x - 1) {
      atomicExch(&A.queue->next, 0);
      atomicExch(&A.queue->done, 0);
    }
  }
}

int shape_index(const char* name) {
  for (int i = 0; i < kNumShapes; ++i)
    if (std::strcmp(kShapes[i].name, name) == 0) return i;
  return -1;
}

// Built-in per-size shape: the autotuner's choice on MI355X (radix-8 lanes for
// N <= 8192, radix-16 for 16384, the only shape that fits).
int builtin_shape(int64_t n) { return n == 16384 ? 6 : 7 + ilog2(n) - 8; }

std::mutex g_rtune_mu;
int g_rtune[7] = {-1, -1, -1, -1, -1, -1, -1};

}  // namespace
}  // namespace stockfft

using namespace stockfft;

struct stockfft_ragged_s {
  int direction = FFT_FORWARD;
  int device = 0;
  int64_t count = 0;
  int64_t total = 0;  // sum of sizes (elements)
  int ntasks = 0;
  int grid = 0;
  int shape_of_class[7] = {};
  int64_t class_count[7] = {};
  Task* d_tasks = nullptr;
  int64_t* d_off = nullptr;
  Queue* d_queue = nullptr;
  void* d_tw[kNumShapes] = {};
  RaggedArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  fft_plan_t plain[7] = {};
};

static void free_ragged(stockfft_ragged_s* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_tasks) (void)hipFree(p->d_tasks);
  if (p->d_off) (void)hipFree(p->d_off);
  if (p->d_queue) (void)hipFree(p->d_queue);
  for (void* t : p->d_tw)
    if (t) (void)hipFree(t);
  for (fft_plan_t q : p->plain)
    if (q) (void)fft_destroy(q);
  delete p;
}

static SingleVariant as_variant(const ShapeInfo& s) {
  SingleVariant v{};
  v.name = s.name;
  v.n = s.n;
  v.npass = s.npass;
  for (int i = 0; i < s.npass; ++i) v.radix[i] = s.radix[i];
  return v;
}

extern "C" int fft_plan_ragged(fft_ragged_plan_t* plan, const int64_t* sizes, int64_t count,
                               int direction) {
  if (!plan) return FFT_INVALID_POINTER;
  *plan = nullptr;
  if (!sizes) return FFT_INVALID_POINTER;
  if (count < 1 || count > (int64_t)1 << 30) return FFT_INVALID_BATCH;
  if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_INVALID_DIRECTION;
  int64_t total = 0;
  for (int64_t i = 0; i < count; ++i) {
    if (!valid_size(sizes[i])) return FFT_INVALID_SIZE;
    total += sizes[i];
  }
  int dev = 0;
  int rc = check_device(&dev);
  if (rc) return rc;

  stockfft_ragged_s* p = new (std::nothrow) stockfft_ragged_s;
  if (!p) return FFT_ALLOC_FAILED;
  p->direction = direction;
  p->device = dev;
  p->count = count;
  p->total = total;
  {
    std::lock_guard<std::mutex> lk(g_rtune_mu);
    for (int c = 0; c < 7; ++c)
      p->shape_of_class[c] = g_rtune[c] >= 0 ? g_rtune[c] : builtin_shape(int64_t(256) << c);
  }

  // Offsets in the packed buffer, grouped by size class, largest class first
  // (longest processing time first), draw order inside a class.
  std::vector<int64_t> offs(count);
  {
    int64_t o = 0;
    for (int64_t i = 0; i < count; ++i) {
      offs[i] = o;
      o += sizes[i];
    }
  }
  std::vector<int64_t> item_off;
  std::vector<Task> tasks;
  item_off.reserve(count);
  for (int c = 6; c >= 0; --c) {
    const int64_t n = int64_t(256) << c;
    const int shape = p->shape_of_class[c];
    const int tpb = kShapes[shape].tpb;
    const int64_t first = (int64_t)item_off.size();
    for (int64_t i = 0; i < count; ++i)
      if (sizes[i] == n) item_off.push_back(offs[i]);
    const int64_t k = (int64_t)item_off.size() - first;
    p->class_count[c] = k;
    for (int64_t j = 0; j < k; j += tpb)
      tasks.push_back(Task{shape, (int32_t)std::min<int64_t>(tpb, k - j), first + j});
  }
  p->ntasks = (int)tasks.size();

  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    free_ragged(p);
    return hip_fail(e);
  }
  p->grid = std::max(1, std::min(cus, p->ntasks));

  std::vector<float> tw;
  for (int s = 0; s < kNumShapes && !rc; ++s) {
    bool used = false;
    for (int c = 0; c < 7; ++c) used |= p->shape_of_class[c] == s;
    if (!used) continue;
    SingleVariant v = as_variant(kShapes[s]);
    build_stockham_twiddles(v, tw);
    rc = upload(tw, &p->d_tw[s]);
  }
  if (!rc) {
    e = hipMalloc((void**)&p->d_tasks, tasks.size() * sizeof(Task));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tasks, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_off, item_off.size() * sizeof(int64_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_off, item_off.data(), item_off.size() * sizeof(int64_t),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_queue, sizeof(Queue));
    if (e == hipSuccess) e = hipMemset(p->d_queue, 0, sizeof(Queue));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e);
  }
  // Per-size plain plans for the comparison entry point.
  for (int c = 0; c < 7 && !rc; ++c)
    if (p->class_count[c] > 0)
      rc = fft_plan(&p->plain[c], int64_t(256) << c, p->class_count[c], direction);
  if (rc) {
    free_ragged(p);
    return rc;
  }
  p->args.tasks = p->d_tasks;
  p->args.item_off = p->d_off;
  p->args.queue = p->d_queue;
  p->args.ntasks = p->ntasks;
  for (int s = 0; s < kNumShapes; ++s) p->args.tw[s] = static_cast<const c32*>(p->d_tw[s]);
  register_handle(p);
  *plan = p;
  return FFT_SUCCESS;
}

// Kernel-node parameters of the persistent launch; argv[0] must point at the
// plan's RaggedArgs (the graph copies the argument values when it is set).
static hipKernelNodeParams ragged_node_params(stockfft_ragged_s* p, void** argv) {
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = p->direction == FFT_BACKWARD ? reinterpret_cast<void*>(&k_ragged<true>)
                                         : reinterpret_cast<void*>(&k_ragged<false>);
  kp.gridDim = dim3((unsigned)p->grid);
  kp.blockDim = dim3(kRaggedThreads);
  kp.sharedMemBytes = 0;
  argv[0] = &p->args;
  kp.kernelParams = argv;
  kp.extra = nullptr;
  return kp;
}

extern "C" int fft_exec_ragged(fft_ragged_plan_t plan, const void* in, void* out, void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  if (!in || !out) return FFT_INVALID_POINTER;
  if (!aligned8(in) || !aligned8(out)) return FFT_MISALIGNED;
  if (ranges_partially_overlap(in, out, (size_t)plan->total * 8)) return FFT_OVERLAP;
  DeviceGuard g(plan->device);
  const bool changed = plan->args.in != in || plan->args.out != out;
  plan->args.in = static_cast<const c32*>(in);
  plan->args.out = static_cast<c32*>(out);
  void* argv[1];
  hipKernelNodeParams kp = ragged_node_params(plan, argv);
  hipError_t e = hipSuccess;
  if (!plan->exec) {
    e = hipGraphCreate(&plan->graph, 0);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&plan->node, plan->graph, nullptr, 0, &kp);
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  } else if (changed) {
    e = hipGraphExecKernelNodeSetParams(plan->exec, plan->node, &kp);
  }
  if (e == hipSuccess) e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  return e == hipSuccess ? FFT_SUCCESS : hip_fail(e);
}

extern "C" int fft_exec_ragged_plain(fft_ragged_plan_t plan, const void* const* in_by_size,
                                     void* const* out_by_size, void* stream) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  if (!in_by_size || !out_by_size) return FFT_INVALID_POINTER;
  for (int c = 0; c < 7; ++c) {
    if (plan->class_count[c] == 0) continue;
    if (!in_by_size[c] || !out_by_size[c]) return FFT_INVALID_POINTER;
  }
  for (int c = 6; c >= 0; --c) {
    if (plan->class_count[c] == 0) continue;
    const int rc = fft_exec(plan->plain[c], in_by_size[c], out_by_size[c], stream);
    if (rc) return rc;
  }
  return FFT_SUCCESS;
}

extern "C" int fft_destroy_ragged(fft_ragged_plan_t plan) {
  if (!plan) return FFT_SUCCESS;
  if (!unregister_handle(plan)) return FFT_INVALID_PLAN;
  free_ragged(plan);
  return FFT_SUCCESS;
}

extern "C" int fft_tune_set_ragged(int64_t n, const char* shape) {
  if (!shape) return FFT_INVALID_POINTER;
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  const int s = shape_index(shape);
  if (s < 0 || kShapes[s].n != n) return FFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(g_rtune_mu);
  g_rtune[ilog2(n) - 8] = s;
  return FFT_SUCCESS;
}

extern "C" int fft_tune_query_ragged(int64_t n, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  int s;
  {
    std::lock_guard<std::mutex> lk(g_rtune_mu);
    s = g_rtune[ilog2(n) - 8];
  }
  if (s < 0) s = builtin_shape(n);
  const size_t len = std::strlen(kShapes[s].name);
  if (cap < (int64_t)len + 1) return FFT_INVALID_ARGUMENT;
  std::memcpy(buf, kShapes[s].name, len + 1);
  return FFT_SUCCESS;
}

extern "C" int fft_ragged_shapes(int64_t n, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_size(n)) return FFT_INVALID_SIZE;
  std::string s;
  for (int i = 0; i < kNumShapes; ++i)
    if (kShapes[i].n == n) {
      if (!s.empty()) s += ",";
      s += kShapes[i].name;
    }
  if (cap < (int64_t)s.size() + 1) return FFT_INVALID_ARGUMENT;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return FFT_SUCCESS;
}

extern "C" int fft_tune_clear_ragged(void) {
  std::lock_guard<std::mutex> lk(g_rtune_mu);
  for (int& v : g_rtune) v = -1;
  return FFT_SUCCESS;
}
