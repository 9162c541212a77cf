// Ragged batches: transforms of different power-of-two lengths, packed one
// after another, run by one persistent kernel launched from a hipGraph.
//
// One persistent workgroup of 512 lanes per CU works through a list of
// tasks; a task is as many transforms of one length as the workgroup holds
// under the shape chosen for that length (radix, lanes per transform and
// exchange tile, picked by the autotuner): 8192 or 16384 elements, so tasks
// cost about the same.  The plan deals the tasks out on the host with
// Graham's longest-processing-time list schedule (longest length first, each
// task to the least-loaded workgroup) and stores every workgroup's tasks
// contiguously, so a workgroup knows its next task without any device
// atomic or queue.
//
// For shapes with 16 values per lane the workgroup is software-pipelined: it
// issues the global loads of its next task into a second register set before
// it computes the current one, so a CU keeps loading while it computes (that
// needs the register file, about 250 VGPRs per lane, instead of a second
// resident workgroup).  Because vector memory counters retire in order on
// CDNA, nothing inside a task may wait on a global load issued after that
// prefetch: the twiddles of every pass but the last are staged in LDS once
// per length, and the last pass's twiddles are loaded into registers before
// the prefetch is issued.  Shapes with 32 values per lane have no registers
// left for a second task and run their tasks one after another.  The code is
// one loop per length, longest first; a workgroup carries its list position
// from one length's loop to the next and never returns to an earlier one.
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
using B256 = ShapeX<1, false, 2, 256, 16, 32, 4, 16, 16>;
using B512 = ShapeX<1, false, 2, 512, 16, 16, 4, 16, 16, 2>;
using B1024 = ShapeX<1, false, 2, 1024, 16, 8, 4, 16, 16, 4>;
using B2048 = ShapeX<1, false, 2, 2048, 16, 4, 4, 16, 16, 8>;
using B4096 = ShapeX<1, false, 2, 4096, 16, 2, 4, 16, 16, 16>;
using B8192 = ShapeX<1, false, 2, 8192, 16, 1, 4, 16, 16, 16, 2>;
using B16384 = ShapeX<2, false, 2, 16384, 32, 1, 4, 16, 16, 16, 4>;

constexpr int kNumShapes = 2 * kClasses;  // shape 2c + alt
constexpr int kLdsElems = B8192::LDS_ELEMS;
// Staged twiddles: the entries of every pass but the last, largest over shapes.
constexpr int kTabElems = 4080;

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
  int32_t cls;    // length class: the transforms have length 256 << cls
};

struct RaggedArgs {
  const c32* in;
  c32* out;
  const Task* tasks;
  const int64_t* item_off;
  const int* wg_begin;      // workgroup w runs tasks [wg_begin[w], wg_begin[w + 1])
  int alt[kClasses];        // shape chosen for length 256 << c (0 = A, 1 = B)
  const c32* tw[kClasses];  // twiddle table of the chosen shape
};

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

// Processes this workgroup's consecutive tasks of length class c, from
// position pos of its list (which ends at end), with shape S; loads task i+1
// while computing task i.  Returns the position of its first task of a
// later class (or end).
template <class S, bool INV>
__device__ __forceinline__ int run_class(int c, int pos, int end, const RaggedArgs& A,
                                         c32* lds_all, c32* tab, const c32* tw) {
  static_assert(S::THREADS == kRaggedThreads, "ragged shapes use 512 lanes");
  static_assert(S::TPB * S::LDS_ELEMS <= kLdsElems, "shape exceeds the exchange tile");
  static_assert(S::tw_off(S::P - 1) <= kTabElems, "staged twiddles exceed their LDS region");
  if (pos >= end || A.tasks[pos].cls != c) return pos;
  const int tid = threadIdx.x;
  const int slot = tid / S::T;
  const int t = tid - slot * S::T;
  if constexpr (S::E > 16) {
    // 32 values per lane leave no registers for a second task: no pipelining,
    // and so no ordering constraint on the twiddle loads, which come from
    // the global table one butterfly at a time.
    for (;;) {
      const Task tc = A.tasks[pos];
      c32 a[S::E];
      fetch<S>(a, A, tc);
      const bool live = slot < tc.count;
      const int64_t off = live ? A.item_off[tc.first + slot] : 0;
      run_passes<S, INV>(a, lds_all + slot * S::LDS_ELEMS, tw, t);
      global_store_row<S>(a, A.out + off, t, live);
      __syncthreads();  // the task's last exchange reads are done before the next task writes
      ++pos;
      if (pos >= end || A.tasks[pos].cls != c) return pos;
    }
  } else {
    // Stage the twiddles of passes 1 .. P-2 (the previous class's are no
    // longer read).
    __syncthreads();
    for (int i = tid; i < S::tw_off(S::P - 1); i += kRaggedThreads) tab[i] = tw[i];
    __syncthreads();
    Task tc = A.tasks[pos];
    c32 b[S::E];
    fetch<S>(b, A, tc);
    for (;;) {
      c32 a[S::E];
#pragma unroll
      for (int m = 0; m < S::E; ++m) a[m] = b[m];
      c32 wl[S::TW_REGS];
      load_twiddles<S, S::P - 1>(wl, tw, t);  // issued before the prefetch
      __builtin_amdgcn_sched_barrier(0);     // and kept before it
      const int nxt = pos + 1;
      const bool more = nxt < end && A.tasks[nxt].cls == c;
      Task tn = tc;
      if (more) {
        tn = A.tasks[nxt];
        fetch<S>(b, A, tn);
      }
      const bool live = slot < tc.count;
      const int64_t off = live ? A.item_off[tc.first + slot] : 0;
      run_passes_tiered_from<S, 0, INV>(a, wl, lds_all + slot * S::LDS_ELEMS, tab, t);
      global_store_row<S>(a, A.out + off, t, live);
      __syncthreads();  // the task's last exchange reads are done before the next task writes
      if (!more) return nxt;
      pos = nxt;
      tc = tn;
    }
  }
}

template <class SA, class SB, bool INV>
__device__ __forceinline__ int run_length(int c, int pos, int end, const RaggedArgs& A,
                                          c32* lds_all, c32* tab) {
  if (A.alt[c] == 0) return run_class<SA, INV>(c, pos, end, A, lds_all, tab, A.tw[c]);
  return run_class<SB, INV>(c, pos, end, A, lds_all, tab, A.tw[c]);
}

template <bool INV>
__global__ __launch_bounds__(kRaggedThreads, 2) void k_ragged(RaggedArgs A) {
  __shared__ c32 lds_all[kLdsElems];
  __shared__ c32 tab[kTabElems];
  const int end = A.wg_begin[blockIdx.x + 1];
  int pos = A.wg_begin[blockIdx.x];
  pos = run_length<A16384, B16384, INV>(6, pos, end, A, lds_all, tab);
  pos = run_length<A8192, B8192, INV>(5, pos, end, A, lds_all, tab);
  pos = run_length<A4096, B4096, INV>(4, pos, end, A, lds_all, tab);
  pos = run_length<A2048, B2048, INV>(3, pos, end, A, lds_all, tab);
  pos = run_length<A1024, B1024, INV>(2, pos, end, A, lds_all, tab);
  pos = run_length<A512, B512, INV>(1, pos, end, A, lds_all, tab);
  pos = run_length<A256, B256, INV>(0, pos, end, A, lds_all, tab);
}

int shape_index(const char* name) {
  for (int i = 0; i < kNumShapes; ++i)
    if (std::strcmp(kShapes[i].name, name) == 0) return i;
  return -1;
}

// Built-in per-length shape: the autotuner's choice on MI355X (the package's
// tune_gfx950.json).
constexpr int kBuiltinShape[kClasses] = {1, 3, 4, 6, 8, 11, 12};
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
  p->grid = std::max(1, std::min(cus, p->ntasks));

  // List schedule (Graham's longest-processing-time rule): tasks, longest
  // length first, each go to the workgroup with the least work so far.  A
  // task's cost counts its memory traffic (live transforms) and its
  // arithmetic (every slot computes, live or not).  Each workgroup's tasks are
  // then laid out contiguously, still longest length first.
  std::vector<int> owner(tasks.size());
  {
    using Load = std::pair<int64_t, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int w = 0; w < p->grid; ++w) heap.push(Load{0, w});
    for (size_t i = 0; i < tasks.size(); ++i) {
      const Task& tk = tasks[i];
      const int64_t n = int64_t(256) << tk.cls;
      const int64_t cost = n * (int64_t(16) * tk.count +
                                int64_t(kShapes[p->shape_of_class[tk.cls]].tpb) * ilog2(n));
      Load l = heap.top();
      heap.pop();
      owner[i] = l.second;
      heap.push(Load{l.first + cost, l.second});
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
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_wg, wg_begin.size() * sizeof(int));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_wg, wg_begin.data(), wg_begin.size() * sizeof(int),
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
  p->args.wg_begin = p->d_wg;
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
