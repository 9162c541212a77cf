// Ragged batches: transforms of different power-of-two lengths, packed one
// after another, run by one persistent kernel.
//
// Two persistent workgroups of 512 lanes per CU (at most 128 VGPRs and a
// 68 KiB exchange tile each) work through a list of tasks; a task is as many
// transforms of one length as the workgroup holds under the shape chosen for
// that length (values per lane, exchange rounds, radix order; picked by the
// autotuner): 4096 to 16384 elements, costed by their measured durations.  The plan
// deals the tasks out on the host with Graham's longest-processing-time list
// schedule, costing each task by its shape's measured duration, and stores
// every workgroup's tasks contiguously, longest length first, with the start
// of each length in a small per-workgroup table; the kernel needs no device
// atomic or queue.
//
// A workgroup runs its tasks one after another; the second workgroup on the
// CU overlaps its loads and stores with this one's arithmetic (measured
// faster on MI355X than one software-pipelined workgroup per CU holding two
// tasks in registers).  The next task's descriptor and row offsets are
// loaded while the current one computes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "../../include/stockfft.h"
#include "internal.hpp"
#include "kernels.hpp"

namespace stockfft {
namespace {

constexpr int kRaggedThreads = 512;
constexpr int kClasses = 7;  // lengths 256 << c, c = 0..6

// Two candidate shapes per length, all 512 lanes, at most 128 VGPRs (two
// workgroups per CU) and at most an 8192-element (+ pad) exchange tile.
// A: 32 values per lane, two-round exchanges, 16384 elements per task (for
// 256: 8 values per lane, radix 8 8 4, 4096 elements per task -- 64 tasks of
// 8 lanes at 32 values needed more than 128 VGPRs and spilled).
// B: 16 values per lane, whole-tile exchanges, 8192 elements per task (for
// 16384, B is the radix-16 order of the A shape).
using A256 = ShapeX<1, false, 4, 256, 8, 16, 4, 8, 8, 4>;
using A512 = ShapeX<2, false, 4, 512, 32, 32, 4, 16, 16, 2>;
using A1024 = ShapeX<2, false, 4, 1024, 32, 16, 4, 16, 16, 4>;
using A2048 = ShapeX<2, false, 4, 2048, 32, 8, 4, 16, 16, 8>;
using A4096 = ShapeX<2, false, 4, 4096, 32, 4, 4, 16, 16, 16>;
using A8192 = ShapeX<2, false, 4, 8192, 32, 2, 4, 16, 16, 16, 2>;
using A16384 = ShapeX<2, false, 4, 16384, 32, 1, 4, 8, 16, 16, 8>;
using B256 = ShapeX<1, false, 4, 256, 16, 32, 4, 16, 16>;
using B512 = ShapeX<1, false, 4, 512, 16, 16, 4, 16, 16, 2>;
using B1024 = ShapeX<1, false, 4, 1024, 16, 8, 4, 16, 16, 4>;
using B2048 = ShapeX<1, false, 4, 2048, 16, 4, 4, 16, 16, 8>;
using B4096 = ShapeX<1, false, 4, 4096, 16, 2, 4, 16, 16, 16>;
using B8192 = ShapeX<1, false, 4, 8192, 16, 1, 4, 16, 16, 16, 2>;
using B16384 = ShapeX<2, false, 4, 16384, 32, 1, 4, 16, 16, 16, 4>;

constexpr int kNumShapes = 2 * kClasses;  // shape 2c + alt
constexpr int kLdsElems = B8192::LDS_ELEMS;

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
    info<A256>("ragged_n256_e8"),          info<B256>("ragged_n256_e16"),
    info<A512>("ragged_n512_e32c2"),       info<B512>("ragged_n512_e16"),
    info<A1024>("ragged_n1024_e32c2"),     info<B1024>("ragged_n1024_e16"),
    info<A2048>("ragged_n2048_e32c2"),     info<B2048>("ragged_n2048_e16"),
    info<A4096>("ragged_n4096_e32c2"),     info<B4096>("ragged_n4096_e16"),
    info<A8192>("ragged_n8192_e32c2"),     info<B8192>("ragged_n8192_e16"),
    info<A16384>("ragged_n16384_e32c2_r8"), info<B16384>("ragged_n16384_e32c2_r16"),
};

// Duration of one full task of each shape in microseconds on an MI355X: a
// batch of one length and shape, 4096 full tasks over 512 workgroups (two per
// CU, every CU busy), kernel time x 512 / 4096.  The list schedule uses them
// as task costs; only their ratios matter to it.
constexpr float kShapeTaskUs[kNumShapes] = {
    7.38f, 13.76f,   // 256
    29.60f, 14.43f,  // 512
    29.07f, 14.09f,  // 1024
    28.39f, 14.41f,  // 2048
    28.27f, 14.77f,  // 4096
    31.17f, 16.07f,  // 8192
    31.26f, 31.47f,  // 16384
};

struct Task {
  int64_t first;  // index of the task's first transform offset in item_off
  int32_t count;  // transforms in this task (<= the shape's TPB)
  int32_t cls;    // length class: the transforms have length 256 << cls
};

struct RaggedArgs {
  const c32* in;
  c32* out;
  const Task* tasks;
  const int64_t* item_off;
  // Workgroup w runs tasks [r[0], r[7]) of the list, r = wg_cls + 8w; its
  // tasks of length 256 << c are [r[6 - c], r[7 - c]).
  const int* wg_cls;
  int alt[kClasses];        // shape chosen for length 256 << c (0 = A, 1 = B)
  const c32* tw[kClasses];  // twiddle table of the chosen shape
};

// Runs this workgroup's tasks [pos, end) of one length one after another (no
// prefetch of rows; a second resident workgroup overlaps its loads instead).
// The next task's descriptor and row offsets are loaded while the current
// task computes, so only a workgroup's first task of a length waits on them.
template <class S, bool INV>
__device__ __forceinline__ void run_class_serial(int pos, int end, const RaggedArgs& A,
                                                 c32* lds_all, const c32* tw) {
  static_assert(S::THREADS == kRaggedThreads, "ragged shapes use 512 lanes");
  static_assert(S::TPB * S::LDS_ELEMS <= kLdsElems, "shape exceeds the exchange tile");
  if (pos >= end) return;
  const int tid = threadIdx.x;
  const int slot = tid / S::T;
  const int t = tid - slot * S::T;
  Task tc = A.tasks[pos];
  int64_t off = slot < tc.count ? A.item_off[tc.first + slot] : 0;
  for (;;) {
    const bool live = slot < tc.count;
    c32 a[S::E];
    // A dead slot (off = 0) reads the buffer's first N elements, which exist:
    // a length class has a task only if an item of that length does.
    global_load_row<S>(a, A.in + off, t);
    const bool more = pos + 1 < end;
    Task tn = tc;
    int64_t off_n = 0;
    if (more) {
      tn = A.tasks[pos + 1];
      if (slot < tn.count) off_n = A.item_off[tn.first + slot];
    }
    // The table pointer and the lane index are made opaque inside the loop so
    // that the compiler does not hoist every pass's twiddle loads and LDS
    // addresses out of it (they would then all stay live across tasks).
    const c32* twl = tw;
    int tl = t;
    asm volatile("" : "+s"(twl), "+v"(tl));
    run_passes<S, INV>(a, lds_all + slot * S::LDS_ELEMS, twl, tl);
    global_store_row<S>(a, A.out + off, t, live);
    __syncthreads();  // the task's last exchange reads are done before the next task writes
    if (!more) return;
    ++pos;
    tc = tn;
    off = off_n;
  }
}

template <class SA, class SB, bool INV>
__device__ __forceinline__ void run_length_serial(int c, const int* r, const RaggedArgs& A,
                                                  c32* lds_all) {
  if (A.alt[c] == 0)
    run_class_serial<SA, INV>(r[6 - c], r[7 - c], A, lds_all, A.tw[c]);
  else
    run_class_serial<SB, INV>(r[6 - c], r[7 - c], A, lds_all, A.tw[c]);
}

template <bool INV>
__global__ __launch_bounds__(kRaggedThreads, 4) void k_ragged(RaggedArgs A) {
  __shared__ alignas(16) c32 lds_all[kLdsElems];
  int r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = A.wg_cls[8 * blockIdx.x + i];
  run_length_serial<A16384, B16384, INV>(6, r, A, lds_all);
  run_length_serial<A8192, B8192, INV>(5, r, A, lds_all);
  run_length_serial<A4096, B4096, INV>(4, r, A, lds_all);
  run_length_serial<A2048, B2048, INV>(3, r, A, lds_all);
  run_length_serial<A1024, B1024, INV>(2, r, A, lds_all);
  run_length_serial<A512, B512, INV>(1, r, A, lds_all);
  run_length_serial<A256, B256, INV>(0, r, A, lds_all);
}

int shape_index(const char* name) {
  for (int i = 0; i < kNumShapes; ++i)
    if (std::strcmp(kShapes[i].name, name) == 0) return i;
  return -1;
}

// Built-in per-length shape: the autotuner's choice on MI355X (the package's
// tune_gfx950.json).
constexpr int kBuiltinShape[kClasses] = {1, 2, 4, 6, 8, 11, 13};
int builtin_shape(int64_t n) { return kBuiltinShape[ilog2(n) - 8]; }

std::mutex g_rtune_mu;
int g_rtune[kClasses] = {-1, -1, -1, -1, -1, -1, -1};

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
  int shape_of_class[kClasses] = {};
  int64_t class_count[7] = {};
  Task* d_tasks = nullptr;
  int64_t* d_off = nullptr;
  int* d_wg = nullptr;
  void* d_tw[kClasses] = {};
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
  if (p->d_wg) (void)hipFree(p->d_wg);
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
    if (!valid_single_size(sizes[i])) return FFT_INVALID_SIZE;
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
      tasks.push_back(Task{first + j, (int32_t)std::min<int64_t>(tpb, k - j), c});
    p->args.alt[c] = shape & 1;
  }
  p->ntasks = (int)tasks.size();

  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    free_ragged(p);
    return hip_fail(e);
  }
  p->grid = std::max(1, std::min(2 * cus, p->ntasks));  // two workgroups per CU

  // List schedule (Graham's longest-processing-time rule): tasks, longest
  // length first, each go to the workgroup with the least work so far.  A
  // task costs its shape's measured duration, scaled down for a partly
  // filled task: half of it (the loads and stores) is taken as proportional to
  // the live transforms, the other half (the arithmetic of every slot) not.
  // Each workgroup's tasks are then laid out contiguously, still longest
  // length first.
  std::vector<int> owner(tasks.size());
  {
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int w = 0; w < p->grid; ++w) heap.push(Load{0, w});
    std::vector<double> cost(tasks.size());
    std::vector<size_t> order(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i) {
      const Task& tk = tasks[i];
      const int shape = p->shape_of_class[tk.cls];
      const double fill = double(tk.count) / kShapes[shape].tpb;
      cost[i] = kShapeTaskUs[shape] * (0.5 + 0.5 * fill);
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    for (size_t i : order) {
      Load l = heap.top();
      heap.pop();
      owner[i] = l.second;
      heap.push(Load{l.first + cost[i], l.second});
    }
  }
  std::vector<int> wg_begin(p->grid + 1, 0);
  for (int w : owner) ++wg_begin[w + 1];
  for (int w = 0; w < p->grid; ++w) wg_begin[w + 1] += wg_begin[w];
  {
    std::vector<int> fill(wg_begin.begin(), wg_begin.end() - 1);
    std::vector<Task> listed(tasks.size());
    for (size_t i = 0; i < tasks.size(); ++i) listed[fill[owner[i]]++] = tasks[i];
    tasks.swap(listed);
  }
  // Per workgroup: where each length's tasks begin in its slice, then its end.
  std::vector<int> wg_cls(8 * (size_t)p->grid);
  for (int w = 0; w < p->grid; ++w) {
    int q = wg_begin[w];
    for (int k = 0; k < kClasses; ++k) {
      wg_cls[8 * w + k] = q;
      while (q < wg_begin[w + 1] && tasks[q].cls == 6 - k) ++q;
    }
    wg_cls[8 * w + 7] = q;
  }

  std::vector<float> tw;
  for (int c = 0; c < kClasses && !rc; ++c) {
    if (p->class_count[c] == 0) continue;
    SingleVariant v = as_variant(kShapes[p->shape_of_class[c]]);
    build_stockham_twiddles(v, tw);
    rc = upload(tw, &p->d_tw[c]);
  }
  if (!rc) {
    e = hipMalloc((void**)&p->d_tasks, tasks.size() * sizeof(Task));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tasks, tasks.data(), tasks.size() * sizeof(Task), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_off, item_off.size() * sizeof(int64_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_off, item_off.data(), item_off.size() * sizeof(int64_t),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_wg, wg_cls.size() * sizeof(int));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_wg, wg_cls.data(), wg_cls.size() * sizeof(int),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e);
  }
  // Per-size plain plans for the comparison entry point.
  for (int c = 0; c < kClasses && !rc; ++c)
    if (p->class_count[c] > 0)
      rc = fft_plan(&p->plain[c], int64_t(256) << c, p->class_count[c], direction);
  if (rc) {
    free_ragged(p);
    return rc;
  }
  p->args.tasks = p->d_tasks;
  p->args.item_off = p->d_off;
  p->args.wg_cls = p->d_wg;

  for (int c = 0; c < kClasses; ++c) p->args.tw[c] = static_cast<const c32*>(p->d_tw[c]);
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

static int check_ragged_exec(fft_ragged_plan_t plan, const void* in, void* out) {
  if (!plan || !live_handle(plan)) return FFT_INVALID_PLAN;
  if (!in || !out) return FFT_INVALID_POINTER;
  if (!aligned8(in) || !aligned8(out)) return FFT_MISALIGNED;
  if (ranges_partially_overlap(in, out, (size_t)plan->total * 8)) return FFT_OVERLAP;
  return FFT_SUCCESS;
}

extern "C" int fft_exec_ragged(fft_ragged_plan_t plan, const void* in, void* out, void* stream) {
  const int rc = check_ragged_exec(plan, in, out);
  if (rc) return rc;
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

extern "C" int fft_exec_ragged_direct(fft_ragged_plan_t plan, const void* in, void* out,
                                      void* stream) {
  const int rc = check_ragged_exec(plan, in, out);
  if (rc) return rc;
  DeviceGuard g(plan->device);
  RaggedArgs args = plan->args;
  args.in = static_cast<const c32*>(in);
  args.out = static_cast<c32*>(out);
  void* argv[1] = {&args};
  const void* fn = plan->direction == FFT_BACKWARD ? reinterpret_cast<const void*>(&k_ragged<true>)
                                                   : reinterpret_cast<const void*>(&k_ragged<false>);
  const hipError_t e = hipLaunchKernel(fn, dim3((unsigned)plan->grid), dim3(kRaggedThreads), argv,
                                       0, (hipStream_t)stream);
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
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
  const int s = shape_index(shape);
  if (s < 0 || kShapes[s].n != n) return FFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(g_rtune_mu);
  g_rtune[ilog2(n) - 8] = s;
  return FFT_SUCCESS;
}

extern "C" int fft_tune_query_ragged(int64_t n, char* buf, int64_t cap) {
  if (!buf) return FFT_INVALID_POINTER;
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
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
  if (!valid_single_size(n)) return FFT_INVALID_SIZE;
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
