// Ragged batches: transforms of different power-of-two lengths, packed one
// after another, run by one persistent kernel launched from a hipGraph.
//
// One persistent workgroup of 512 lanes per CU works through a queue of
// tasks; a task is as many transforms of one length as the workgroup holds
// under the shape chosen for that length (radix, lanes per transform and
// exchange tile, picked by the autotuner), 8192 or 16384 elements.  Tasks are
// grouped by length, longest first (longest processing time first), and
// handed out by one device counter.
//
// The workgroup is software-pipelined: it takes its next ticket and issues the
// global loads of that task into a second register set before it computes
// the current one, so a CU keeps loading while it computes.  That needs the
// register file (about 250 VGPRs per lane, one workgroup per CU) instead of a
// second resident workgroup.  The queue code is one pipelined loop per
// length, in queue order: tickets only grow, so a workgroup carries its
// ticket from one length's loop to the next and never returns.
//
// The counter resets itself: the last workgroup to leave clears it, so the
// graph holds a single kernel node and no memset.
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

constexpr int kRaggedThreads = 512;
constexpr int kClasses = 7;  // lengths 256 << c, c = 0..6

// Two candidate shapes per length, all 512 lanes with at most an 8192-element
// (+ pad) exchange tile.  A: 32 values per lane, two-round exchanges, 16384
// elements per task.  B: 16 values per lane, whole-tile exchanges, 8192
// elements per task (for 16384, B is the radix-16 order of the A shape).
using A256 = ShapeX<2, false, 2, 256, 32, 64, 4, 16, 16>;
using A512 = ShapeX<2, false, 2, 512, 32, 32, 4, 16, 16, 2>;
using A1024 = ShapeX<2, false, 2, 1024, 32, 16, 4, 16, 16, 4>;
using A2048 = ShapeX<2, false, 2, 2048, 32, 8, 4, 16, 16, 8>;
using A4096 = ShapeX<2, false, 2, 4096, 32, 4, 4, 16, 16, 16>;
using A8192 = ShapeX<2, false, 2, 8192, 32, 2, 4, 16, 16, 16, 2>;
using A16384 = ShapeX<2, false, 2, 16384, 32, 1, 4, 8, 16, 16, 8>;
using B256 = ShapeX<1, true, 2, 256, 16, 32, 4, 16, 16>;
using B512 = ShapeX<1, true, 2, 512, 16, 16, 4, 16, 16, 2>;
using B1024 = ShapeX<1, true, 2, 1024, 16, 8, 4, 16, 16, 4>;
using B2048 = ShapeX<1, true, 2, 2048, 16, 4, 4, 16, 16, 8>;
using B4096 = ShapeX<1, true, 2, 4096, 16, 2, 4, 16, 16, 16>;
using B8192 = ShapeX<1, true, 2, 8192, 16, 1, 4, 16, 16, 16, 2>;
using B16384 = ShapeX<2, false, 2, 16384, 32, 1, 4, 16, 16, 16, 4>;

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
    info<A256>("ragged_n256_e32c2"),       info<B256>("ragged_n256_e16"),
    info<A512>("ragged_n512_e32c2"),       info<B512>("ragged_n512_e16"),
    info<A1024>("ragged_n1024_e32c2"),     info<B1024>("ragged_n1024_e16"),
    info<A2048>("ragged_n2048_e32c2"),     info<B2048>("ragged_n2048_e16"),
    info<A4096>("ragged_n4096_e32c2"),     info<B4096>("ragged_n4096_e16"),
    info<A8192>("ragged_n8192_e32c2"),     info<B8192>("ragged_n8192_e16"),
    info<A16384>("ragged_n16384_e32c2_r8"), info<B16384>("ragged_n16384_e32c2_r16"),
};

struct Task {
  int64_t first;  // index of the task's first transform offset in item_off
  int32_t count;  // transforms in this task (<= the shape's TPB)
  int32_t pad;
};

struct Queue {
  int next;  // next ticket to hand out
  int done;  // workgroups that have left
};

struct RaggedArgs {
  const c32* in;
  c32* out;
  const Task* tasks;
  const int64_t* item_off;
  Queue* queue;
  int ntasks;
  int end[kClasses];      // one past the last ticket of length 256 << c
  int alt[kClasses];      // shape chosen for length 256 << c (0 = A, 1 = B)
  const c32* tw[kClasses];  // twiddle table of the chosen shape
};

__device__ __forceinline__ int take_ticket(Queue* q, int* s_ticket) {
  if (threadIdx.x == 0) *s_ticket = atomicAdd(&q->next, 1);
  __syncthreads();
  const int v = *s_ticket;
  __syncthreads();  // every lane has read it before lane 0 overwrites it
  return v;
}

// Issues the global loads of task tk's rows into b (the shape's load pattern).
template <class S>
__device__ __forceinline__ void fetch(c32 (&b)[S::E], const RaggedArgs& A, const Task& tk) {
  const int tid = threadIdx.x;
  const int slot = tid / S::T;
  const int t = tid - slot * S::T;
  const bool live = slot < tk.count;
  const int64_t off = live ? A.item_off[tk.first + slot] : 0;
  global_load_row<S>(b, A.in + off, t, live);
}

template <class S, bool INV>
__device__ __forceinline__ void compute_store(c32 (&a)[S::E], const RaggedArgs& A, const Task& tk,
                                              c32* lds_all, const c32* tw) {
  // An optimization barrier: keeps the table loads inside the task loop
  // (hoisted out of it they would stay live across every task).
  asm volatile("" : "+s"(tw));
  const int tid = threadIdx.x;
  const int slot = tid / S::T;
  const int t = tid - slot * S::T;
  const bool live = slot < tk.count;
  const int64_t off = live ? A.item_off[tk.first + slot] : 0;
  run_passes<S, INV>(a, lds_all + slot * S::LDS_ELEMS, tw, t);
  global_store_row<S>(a, A.out + off, t, live);
}

// Processes tickets below `end` (all of one length) with shape S, loading
// task i+1 while computing task i.  Returns the first ticket at or past end.
template <class S, bool INV>
__device__ __forceinline__ int run_class(int ticket, int end, const RaggedArgs& A, c32* lds_all,
                                         int* s_ticket, const c32* tw) {
  static_assert(S::THREADS == kRaggedThreads, "ragged shapes use 512 lanes");
  static_assert(S::TPB * S::LDS_ELEMS <= kLdsElems, "shape exceeds the exchange tile");
  if (ticket >= end) return ticket;
  Task tc = A.tasks[ticket];
  c32 b[S::E];
  fetch<S>(b, A, tc);
  for (;;) {
    c32 a[S::E];
#pragma unroll
    for (int m = 0; m < S::E; ++m) a[m] = b[m];
    const int nxt = take_ticket(A.queue, s_ticket);
    Task tn = tc;
    if (nxt < end) {
      tn = A.tasks[nxt];
      fetch<S>(b, A, tn);
    }
    compute_store<S, INV>(a, A, tc, lds_all, tw);
    if (nxt >= end) return nxt;
    tc = tn;
  }
}

template <class SA, class SB, bool INV>
__device__ __forceinline__ int run_length(int c, int ticket, const RaggedArgs& A, c32* lds_all,
                                          int* s_ticket) {
  if (A.alt[c] == 0) return run_class<SA, INV>(ticket, A.end[c], A, lds_all, s_ticket, A.tw[c]);
  return run_class<SB, INV>(ticket, A.end[c], A, lds_all, s_ticket, A.tw[c]);
}

template <bool INV>
__global__ __launch_bounds__(kRaggedThreads, 2) void k_ragged(RaggedArgs A) {
  __shared__ c32 lds_all[kLdsElems];
  __shared__ int s_ticket;
  int ticket = take_ticket(A.queue, &s_ticket);
  ticket = run_length<A16384, B16384, INV>(6, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A8192, B8192, INV>(5, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A4096, B4096, INV>(4, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A2048, B2048, INV>(3, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A1024, B1024, INV>(2, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A512, B512, INV>(1, ticket, A, lds_all, &s_ticket);
  ticket = run_length<A256, B256, INV>(0, ticket, A, lds_all, &s_ticket);
  // Every workgroup leaves holding exactly one ticket at or past ntasks, so
  // when the last one arrives nobody touches the counter again in this
  // launch: it resets both counters for the next launch.
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

// Built-in per-length shape: the autotuner's choice on MI355X (the package's
// tune_gfx950.json).
constexpr int kBuiltinShape[kClasses] = {0, 3, 4, 7, 8, 11, 12};
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
  Queue* d_queue = nullptr;
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
      tasks.push_back(Task{first + j, (int32_t)std::min<int64_t>(tpb, k - j), 0});
    p->args.end[c] = (int)tasks.size();
    p->args.alt[c] = shape & 1;
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
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_queue, sizeof(Queue));
    if (e == hipSuccess) e = hipMemset(p->d_queue, 0, sizeof(Queue));
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
  p->args.queue = p->d_queue;
  p->args.ntasks = p->ntasks;
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
