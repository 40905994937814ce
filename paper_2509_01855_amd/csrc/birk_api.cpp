// C-ABI entry points of libbirk: plan management, products, preconditioner, FastAX and
// the right-preconditioned GMRES solve with double-precision iterative refinement.
//
// Solve (arXiv 2509.01855, eq:Newton-ivp, eq:rightPx2, Algorithm 2, FastLinSol box):
// every outer step forms the true residual r = beta - A chi in double (FastAX in
// double), stops when ||r|| <= rtol ||beta|| per instance, and otherwise runs one
// right-preconditioned GMRES cycle on A d = r / ||r|| in the Krylov precision
// (double for BIRK_F64 plans, float for BIRK_F32_REFINE_F64 plans), then chi += ||r|| d.
// With a double Krylov precision this is restarted GMRES whose restarts use the true
// residual; with float it is mixed-precision iterative refinement.  The Arnoldi
// process uses classical Gram-Schmidt with one re-orthogonalisation (CGS2); dot
// products and norms accumulate in double; the Hessenberg least-squares problem is
// solved with Givens rotations on the host, one small device-to-host copy per
// iteration.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "birk_internal.h"

using namespace birk;

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
inline int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

constexpr int64_t kMaxN = int64_t(1) << 22;       // any N
constexpr int64_t kMaxNPow2 = int64_t(1) << 23;   // N a power of two
constexpr int64_t kMaxTotal = int64_t(1) << 31;
constexpr int kMaxPrecondNx = 12;

static void drop_graphs(birk_plan* p) {
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
  for (auto& g : p->kgraphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->kgraphs.clear();
}

void free_plan(birk_plan* p) {
  if (!p) return;
  drop_graphs(p);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  for (int k = 0; k < birk_plan::kExtraStreams; ++k) {
    if (p->ev_join[k]) (void)hipEventDestroy(p->ev_join[k]);
    if (p->xstream[k]) (void)hipStreamDestroy(p->xstream[k]);
  }
  for (auto& in : p->inst)
    if (in.w) (void)hipFree(in.w);
  for (void* q : p->allocs) if (q) (void)hipFree(q);
  for (void* q : p->work) if (q) (void)hipFree(q);
  for (void* q : p->tmp_vec) if (q) (void)hipFree(q);
  if (p->partials) (void)hipFree(p->partials);
  if (p->scan) (void)hipFree(p->scan);
  if (p->jsw) (void)hipFree(p->jsw);
  if (p->krylov_Q) (void)hipFree(p->krylov_Q);
  if (p->krylov_vec) (void)hipFree(p->krylov_vec);
  if (p->newton_buf) (void)hipFree(p->newton_buf);
  if (p->kkt_buf) (void)hipFree(p->kkt_buf);
  if (p->krylov_dots) (void)hipFree(p->krylov_dots);
  if (p->krylov_part) (void)hipFree(p->krylov_part);
  if (p->krylov_coef) (void)hipFree(p->krylov_coef);
  if (p->krylov_gm) (void)hipFree(p->krylov_gm);
  if (p->krylov_prm) (void)hipFree(p->krylov_prm);
  if (p->krylov_stage) (void)hipHostFree(p->krylov_stage);
  if (p->flag) (void)hipFree(p->flag);
  delete p;
}

birk_status dev_err(hipError_t e) { return e == hipErrorOutOfMemory ? BIRK_ERR_NOMEM : BIRK_ERR_DEVICE; }

__global__ void k_extract_weights(const double* __restrict__ v, double* __restrict__ w, int64_t Nn) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < Nn) w[k] = v[k];
}

__global__ void k_set_unit(double* __restrict__ v, int64_t idx) { v[idx] = 1.0; }

}  // namespace

// ---- fixed product workspace of birk_apply_noalloc
// One array per device, held from the library's first use on that device to the end of
// the process.  Host code never uses the array's name as an address: every device needs
// its own copy's address, resolved once per device by noalloc_base (with that device
// current) and kept in noalloc_ptr.
constexpr size_t kNoallocBytes = size_t(128) << 20;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

std::mutex noalloc_mu;
void* noalloc_ptr[kNoallocMaxDevices] = {};

// Address of this device's array; the caller has made `dev` the current device.
hipError_t noalloc_base(int dev, void** base) {
  *base = nullptr;
  if (dev < 0 || dev >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    noalloc_ptr[dev] = ptr;
  }
  *base = noalloc_ptr[dev];
  return hipSuccess;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the product workspace of a plan inside the fixed array: the complex work
// buffers (two for power-of-two groups only, three when the general path runs) and the
// c^_0 partials, each 256-byte aligned.
size_t noalloc_need(const birk_plan* p, int* nbuf) {
  *nbuf = (p->gen[0].host.empty() && p->gen[1].host.empty()) ? 2 : 3;
  return (size_t)*nbuf * align256((size_t)std::max<int64_t>(p->total_work, 1) * sizeof(double2)) +
         align256((size_t)std::max<int64_t>(p->total_part, 1) * sizeof(double));
}

}  // namespace

extern "C" {

const char* birk_status_string(birk_status s) {
  switch (s) {
    case BIRK_OK: return "BIRK_OK: success";
    case BIRK_ERR_ARG: return "BIRK_ERR_ARG: invalid argument (null pointer, bad enum or overlap)";
    case BIRK_ERR_SIZE: return "BIRK_ERR_SIZE: size out of range (batch < 1, N_n < 3, n_x < 1 or too large)";
    case BIRK_ERR_DEVICE: return "BIRK_ERR_DEVICE: a HIP runtime call failed";
    case BIRK_ERR_NOMEM: return "BIRK_ERR_NOMEM: device allocation failed";
    case BIRK_ERR_SINGULAR: return "BIRK_ERR_SINGULAR: I - w_k J_k / 2 is singular at some node";
    case BIRK_ERR_NOCONV: return "BIRK_ERR_NOCONV: iteration limit reached before the tolerance";
    case BIRK_ERR_BREAKDOWN: return "BIRK_ERR_BREAKDOWN: Krylov breakdown without convergence";
    case BIRK_ERR_NONFINITE: return "BIRK_ERR_NONFINITE: NaN or Inf met during the solve";
    case BIRK_ERR_UNSUPPORTED: return "BIRK_ERR_UNSUPPORTED: request not implemented by this build";
  }
  return "unknown birk_status";
}

void birk_solve_opts_default(birk_solve_opts* o) {
  if (!o) return;
  o->method = 0;
  o->restart = 30;
  o->max_iter = 300;
  o->rtol = 1e-10;
  o->use_precond = 1;
  o->use_x0 = 0;
  o->max_refine = 8;
  o->inner_rtol = 1e-5;
}

int64_t birk_plan_length(const birk_plan* p) { return p ? p->total_len : 0; }

birk_status birk_plan_tune(birk_plan* p, char* report, int64_t report_len) {
  if (!p || (report && report_len <= 0)) return BIRK_ERR_ARG;
  std::string text;
  DeviceGuard g(p->device);
  drop_graphs(p);  // recorded with the previous schedule
  hipError_t e = tune_fast(p, p->stream, &text);
  if (e == hipSuccess && !p->gen[1].host.empty()) e = tune_general(p, p->stream, &text);
  if (report) {
    const size_t n = std::min<size_t>(text.size(), (size_t)report_len - 1);
    std::memcpy(report, text.data(), n);
    report[n] = '\0';
  }
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

birk_status birk_plan_create(birk_plan** out, int32_t batch, const int64_t* n_nodes_host,
                             const int32_t* n_x_host, birk_precision prec, void* hip_stream) {
  if (!out) return BIRK_ERR_ARG;
  *out = nullptr;
  if (!n_nodes_host || !n_x_host) return BIRK_ERR_ARG;
  if (prec != BIRK_F64 && prec != BIRK_F32 && prec != BIRK_F32_REFINE_F64 && prec != BIRK_DF32)
    return BIRK_ERR_ARG;
  if (batch < 1) return BIRK_ERR_SIZE;
  int64_t total = 0;
  for (int i = 0; i < batch; ++i) {
    const int64_t Nn = n_nodes_host[i];
    const int nx = n_x_host[i];
    if (Nn < 3 || nx < 1) return BIRK_ERR_SIZE;
    const int64_t N = Nn - 1;
    if (N > (is_pow2(N) ? kMaxNPow2 : kMaxN)) return BIRK_ERR_SIZE;
    total += Nn * nx;
    if (total > kMaxTotal) return BIRK_ERR_SIZE;
  }
  birk_plan* p = new (std::nothrow) birk_plan();
  if (!p) return BIRK_ERR_NOMEM;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return BIRK_ERR_DEVICE;
  }
  p->stream = (hipStream_t)hip_stream;
  p->prec = prec;
  {
    // BIRK_FAST=0 routes power-of-two sizes through the general FFT path (testing aid)
    const char* f = std::getenv("BIRK_FAST");
    p->use_fast = (f && f[0] == '0') ? 0 : 1;
    // tuning of the three-pass kernels: LDS budget per workgroup (KB) for double and
    // float, and which side of 2N = L1 L2 is the longer one
    const char* l64 = std::getenv("BIRK_FAST_LDS_KB_F64");
    const char* l32 = std::getenv("BIRK_FAST_LDS_KB_F32");
    const char* sp = std::getenv("BIRK_FAST_SPLIT");
    if (l64) p->fast_kn.lds_kb[0] = std::max(16, std::min(160, std::atoi(l64)));
    if (l32) p->fast_kn.lds_kb[1] = std::max(16, std::min(160, std::atoi(l32)));
    if (sp) p->fast_kn.split = std::atoi(sp) ? 1 : 0;
    const char* tb = std::getenv("BIRK_FAST_TB");
    if (tb) p->fast_kn.tb = std::max(0, std::min(14, std::atoi(tb))) & ~1;
    const char* bt = std::getenv("BIRK_FAST_B_THREADS");
    if (bt) p->fast_kn.b_threads = std::atoi(bt) <= 256 ? 256 : 512;
    const char* xc = std::getenv("BIRK_FAST_XCD");
    if (xc) p->fast_kn.xcd = std::atoi(xc) ? 1 : 0;
    const char* b2 = std::getenv("BIRK_FAST_B2");
    if (b2) p->fast_kn.b2 = std::atoi(b2) ? 1 : 0;
    // four-column tiles in passes A and C measured faster for 8-byte reals (double and
    // double-float), eight-column ones for float
    p->fast_kn.narrow = prec == BIRK_F32 || prec == BIRK_F32_REFINE_F64 ? 0 : 1;
    const char* nw = std::getenv("BIRK_FAST_NARROW");
    if (nw) p->fast_kn.narrow = std::atoi(nw) ? 1 : 0;
    const char* b3 = std::getenv("BIRK_FAST_B3");
    if (b3) p->fast_kn.b3 = std::atoi(b3) ? 1 : 0;
    const char* st = std::getenv("BIRK_FAST_STREAMS");
    if (st) p->fast_kn.streams = std::max(1, std::min(1 + birk_plan::kExtraStreams, std::atoi(st)));
  }
  p->inst.resize(batch);
  int64_t off = 0, joff = 0, jcoff = 0, soff = 0, jswoff = 0;
  for (int i = 0; i < batch; ++i) {
    Instance& in = p->inst[i];
    in.Nn = n_nodes_host[i];
    in.N = in.Nn - 1;
    in.nx = n_x_host[i];
    in.off = off;
    in.joff = joff;
    in.jcoff = jcoff;
    in.scan_off = soff;
    off += in.Nn * in.nx;
    joff += in.Nn * in.nx * in.nx;
    jcoff += (int64_t)in.nx * in.nx;
    soff += pinv_scratch(in.Nn, in.nx) + (int64_t)in.nx * ((in.Nn + 1023) / 1024) + 64;
    in.jsw_off = jswoff;
    jswoff += pinv_jsw_size(in.Nn, in.nx);
  }
  p->total_len = off;
  p->total_jnode = joff;
  p->total_jconst = jcoff;
  p->total_scan = soff;
  p->total_jsw = jswoff;
  // product schedule: three-pass groups and the general-path pair sets
  plan_products(p);
  const int64_t woff = std::max<int64_t>(p->total_work, 1), poff = p->total_part;

  hipError_t e = hipSuccess;
  for (int b = 0; b < 3 && e == hipSuccess; ++b) e = hipMalloc(&p->work[b], woff * sizeof(double2));
  for (int b = 0; b < 4 && e == hipSuccess; ++b) e = hipMalloc(&p->tmp_vec[b], off * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->partials, std::max<int64_t>(poff, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->scan, std::max<int64_t>(soff, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->jsw, std::max<int64_t>(jswoff, 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->flag, sizeof(int));
  // extra streams (default priority) for the multi-stream schedule of the three-pass groups
  if (e == hipSuccess && !p->fgroups.empty()) {
    e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    for (int k = 0; k < birk_plan::kExtraStreams && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&p->xstream[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming);
    }
  }
  for (int i = 0; i < batch && e == hipSuccess; ++i) e = hipMalloc(&p->inst[i].w, p->inst[i].Nn * sizeof(double));
  if (e == hipSuccess) e = build_tables(p);
  // CC weights: w = B^aT e_N (the last row of B^a), instance by instance on component 0
  if (e == hipSuccess) {
    double* v = (double*)p->tmp_vec[0];
    double* o = (double*)p->tmp_vec[1];
    e = hipMemsetAsync(v, 0, off * sizeof(double), p->stream);
    for (int i = 0; i < batch && e == hipSuccess; ++i) {
      hipLaunchKernelGGL(k_set_unit, dim3(1), dim3(1), 0, p->stream, v, p->inst[i].off + p->inst[i].N);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = apply_product<double>(p, v, o, 1, p->stream);
    for (int i = 0; i < batch && e == hipSuccess; ++i) {
      const Instance& in = p->inst[i];
      hipLaunchKernelGGL(k_extract_weights, dim3((unsigned)((in.Nn + 255) / 256)), dim3(256), 0, p->stream,
                         o + in.off, in.w, in.Nn);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  }
  if (e == hipSuccess) e = plan_bform(p);
  if (e == hipSuccess) e = plan_instances(p);
  if (e == hipSuccess) e = plan_solve(p);
  if (e == hipSuccess) e = plan_kkt(p);
  if (e != hipSuccess) {
    free_plan(p);
    return dev_err(e);
  }
  // set-up of birk_apply_noalloc on this device (its first call retries if this fails)
  {
    void* base = nullptr;
    (void)noalloc_base(p->device, &base);
  }
  *out = p;
  return BIRK_OK;
}

birk_status birk_plan_destroy(birk_plan* p) {
  if (!p) return BIRK_OK;
  DeviceGuard g(p->device);
  (void)hipStreamSynchronize(p->stream);
  free_plan(p);
  return BIRK_OK;
}

birk_status birk_weights(birk_plan* p, int32_t inst, double* w_host) {
  if (!p || !w_host) return BIRK_ERR_ARG;
  if (inst < 0 || inst >= (int32_t)p->inst.size()) return BIRK_ERR_SIZE;
  DeviceGuard g(p->device);
  const Instance& in = p->inst[inst];
  hipError_t e = hipMemcpyAsync(w_host, in.w, in.Nn * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

static hipError_t launch_product(birk_plan* p, const void* v, void* out, int transpose) {
  switch (p->prec) {
    case BIRK_F64:
      return apply_product<double>(p, (const double*)v, (double*)out, transpose, p->stream);
    case BIRK_DF32:
      return apply_product<df32>(p, (const df32*)v, (df32*)out, transpose, p->stream);
    default:
      return apply_product<float>(p, (const float*)v, (float*)out, transpose, p->stream);
  }
}

constexpr size_t kMaxGraphs = 8;

// Graph mode: the first use of a (direction, v, out) triple runs eagerly (and sets any
// kernel attributes), the second records the launches into a graph and replays it,
// later uses replay it.  At most kMaxGraphs triples; the least recently used goes.
static hipError_t graph_product(birk_plan* p, const void* v, void* out, int transpose) {
  const uint64_t now = ++p->graph_clock;
  for (auto& g : p->graphs) {
    if (g.transpose != transpose || g.v != v || g.out != out) continue;
    g.used = now;
    if (!g.exec) {
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      e = launch_product(p, v, out, transpose);
      const hipError_t e2 = hipStreamEndCapture(p->stream, &graph);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        g.exec = nullptr;
        return e;
      }
    }
    return hipGraphLaunch(g.exec, p->stream);
  }
  if (p->graphs.size() >= kMaxGraphs) {
    auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                [](const birk_plan::GraphSlot& a, const birk_plan::GraphSlot& b) {
                                  return a.used < b.used;
                                });
    if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
    p->graphs.erase(lru);
  }
  p->graphs.push_back({transpose, v, out, nullptr, now});
  return launch_product(p, v, out, transpose);
}

static birk_status product(birk_plan* p, const void* v, void* out, int transpose) {
  if (!p || !v || !out || v == out) return BIRK_ERR_ARG;
  DeviceGuard g(p->device);
  const hipError_t e = p->use_graphs ? graph_product(p, v, out, transpose) : launch_product(p, v, out, transpose);
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

birk_status birk_plan_set_graphs(birk_plan* p, int32_t enable) {
  if (!p || (enable != 0 && enable != 1)) return BIRK_ERR_ARG;
  if (enable && !p->stream) return BIRK_ERR_UNSUPPORTED;  // the legacy null stream cannot be captured
  DeviceGuard g(p->device);
  (void)hipStreamSynchronize(p->stream);
  drop_graphs(p);
  p->use_graphs = enable;
  return BIRK_OK;
}

birk_status birk_apply(birk_plan* p, const void* v, void* out) { return product(p, v, out, 0); }
birk_status birk_apply_T(birk_plan* p, const void* g, void* out) { return product(p, g, out, 1); }

// birk_apply / birk_apply_T with the product kernels' work buffers and partial sums in
// the device's fixed array instead of the plan's own buffers: no allocation, no graph.
// Every kernel writes each workspace element before it reads it, so nothing needs
// clearing between calls.
birk_status birk_apply_noalloc(birk_plan* p, const void* v, void* out, int32_t transpose) {
  if (!p || !v || !out || v == out || (transpose != 0 && transpose != 1)) return BIRK_ERR_ARG;
  int nbuf = 0;
  const size_t need = noalloc_need(p, &nbuf);
  if (need > kNoallocBytes) return BIRK_ERR_SIZE;
  DeviceGuard g(p->device);
  void* base = nullptr;
  if (noalloc_base(p->device, &base) != hipSuccess) return BIRK_ERR_DEVICE;
  const size_t buf = align256((size_t)std::max<int64_t>(p->total_work, 1) * sizeof(double2));
  void* saved_work[3] = {p->work[0], p->work[1], p->work[2]};
  double* saved_part = p->partials;
  unsigned char* b = (unsigned char*)base;
  for (int k = 0; k < 3; ++k) p->work[k] = k < nbuf ? (void*)(b + k * buf) : nullptr;
  p->partials = (double*)(b + nbuf * buf);
  const hipError_t e = launch_product(p, v, out, transpose);
  for (int k = 0; k < 3; ++k) p->work[k] = saved_work[k];
  p->partials = saved_part;
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

// b-form products (eq:xN=Birka+b): the B^a product and a per-component rank-one
// correction on the plan's stream.
birk_status birk_apply_b(birk_plan* p, const void* v, void* out) {
  const birk_status st = product(p, v, out, 0);
  if (st != BIRK_OK) return st;
  DeviceGuard g(p->device);
  hipError_t e;
  switch (p->prec) {
    case BIRK_F64: e = bform_correct<double>(p, (double*)out, p->stream); break;
    case BIRK_DF32: e = bform_correct<df32>(p, (df32*)out, p->stream); break;
    default: e = bform_correct<float>(p, (float*)out, p->stream); break;
  }
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

birk_status birk_apply_bT(birk_plan* p, const void* gv, void* out) {
  if (!p || !gv || !out || gv == out) return BIRK_ERR_ARG;
  hipError_t e;
  {
    DeviceGuard g(p->device);
    switch (p->prec) {
      case BIRK_F64: e = bform_sums<double>(p, (const double*)gv, p->stream); break;
      case BIRK_DF32: e = bform_sums<df32>(p, (const df32*)gv, p->stream); break;
      default: e = bform_sums<float>(p, (const float*)gv, p->stream); break;
    }
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
  }
  const birk_status st = product(p, gv, out, 1);
  if (st != BIRK_OK) return st;
  DeviceGuard g(p->device);
  switch (p->prec) {
    case BIRK_F64: e = bform_correct_T<double>(p, (double*)out, p->stream); break;
    case BIRK_DF32: e = bform_correct_T<df32>(p, (df32*)out, p->stream); break;
    default: e = bform_correct_T<float>(p, (float*)out, p->stream); break;
  }
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

birk_status birk_endpoint(birk_plan* p, const double* xa, const void* v, double* xb) {
  if (!p || !xa || !v || !xb) return BIRK_ERR_ARG;
  DeviceGuard g(p->device);
  hipError_t e;
  switch (p->prec) {
    case BIRK_F64: e = endpoint<double>(p, xa, (const double*)v, xb, p->stream); break;
    case BIRK_DF32: e = endpoint<df32>(p, xa, (const df32*)v, xb, p->stream); break;
    default: e = endpoint<float>(p, xa, (const float*)v, xb, p->stream); break;
  }
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

static bool nx_ok_for_precond(const birk_plan* p) {
  for (const auto& in : p->inst)
    if (in.nx > kMaxPrecondNx) return false;
  return true;
}

birk_status birk_precond(birk_plan* p, birk_jac_kind jk, const double* J, const void* y, void* out,
                         int32_t inverse) {
  if (!p || !J || !y || !out || y == out) return BIRK_ERR_ARG;
  if (jk != BIRK_J_CONSTANT && jk != BIRK_J_PER_NODE) return BIRK_ERR_ARG;
  if (inverse != 0 && inverse != 1 && inverse != 2) return BIRK_ERR_ARG;
  if (p->prec == BIRK_DF32) return BIRK_ERR_UNSUPPORTED;
  if (inverse && !nx_ok_for_precond(p)) return BIRK_ERR_UNSUPPORTED;
  if (inverse == 2 && p->prec != BIRK_F64) return BIRK_ERR_UNSUPPORTED;
  DeviceGuard g(p->device);
  hipError_t e;
  if (inverse == 2) {
    e = precond_inverse_t(p, jk, J, (const double*)y, (double*)out, p->bt_scr, p->stream);
    return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
  }
  if (inverse) {
    e = precond_prepare(p, jk, J, p->prec == BIRK_F64 ? 0 : 1, p->stream, kPrepLarge);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
  }
  if (p->prec == BIRK_F64) {
    e = inverse ? precond_inverse<double>(p, jk, J, (const double*)y, (double*)out, nullptr, p->stream, nullptr, 0)
                : precond_forward<double>(p, jk, J, (const double*)y, (double*)out, p->stream);
  } else {
    e = inverse ? precond_inverse<float>(p, jk, J, (const float*)y, (float*)out, nullptr, p->stream, nullptr, 0)
                : precond_forward<float>(p, jk, J, (const float*)y, (float*)out, p->stream);
  }
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

// A x = x - B^a (J x) in double; uses tmp_vec[2], tmp_vec[3].
static hipError_t fast_ax_f64(birk_plan* p, int jk, const double* J, const double* x, double* t_out) {
  double* y = (double*)p->tmp_vec[2];
  hipError_t e = jac_times<double>(p, jk, J, x, y, p->stream);
  if (e == hipSuccess) e = apply_product<double>(p, y, t_out, 0, p->stream);
  return e;
}

birk_status birk_fast_ax(birk_plan* p, birk_jac_kind jk, const double* J, const double* x, double* out) {
  if (!p || !J || !x || !out || x == out) return BIRK_ERR_ARG;
  if (jk != BIRK_J_CONSTANT && jk != BIRK_J_PER_NODE) return BIRK_ERR_ARG;
  DeviceGuard g(p->device);
  double* t = (double*)p->tmp_vec[3];
  hipError_t e = fast_ax_f64(p, jk, J, x, t);
  if (e == hipSuccess) kry::sub<double>(x, t, out, p->total_len, p->stream);
  e = (e == hipSuccess) ? hipGetLastError() : e;
  return e == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

}  // extern "C"

// ------------------------------------------------------------------ GMRES
namespace {

constexpr int kDotsStride = kKryMaxDots + 1;

struct InstState {
  double bnorm = 0.0;
  double rnorm = 0.0;
  int status = BIRK_OK;
  int inner = 0;
  int outer = 0;
  bool done = false;
  bool breakdown_last = false;
};

// Pinned host staging of the Krylov driver: [dots: B x 2 x kDotsStride doubles][flag: one
// double slot][coefficients: B x kDotsStride doubles][counts: B ints], the last two laid
// out like krylov_coef on the device so one copy uploads both.
size_t stage_bytes(size_t B) { return (B * 3 * kDotsStride + 1) * sizeof(double) + B * sizeof(int); }
double* stage_dots(birk_plan* p) { return (double*)p->krylov_stage; }
int* stage_flag(birk_plan* p) { return (int*)(stage_dots(p) + p->inst.size() * 2 * kDotsStride); }
double* stage_coef(birk_plan* p) { return stage_dots(p) + p->inst.size() * 2 * kDotsStride + 1; }
int* stage_cnt(birk_plan* p) { return (int*)(stage_coef(p) + p->inst.size() * kDotsStride); }

hipError_t ensure_krylov(birk_plan* p, int m, size_t esize) {
  hipError_t e = hipSuccess;
  const size_t B = p->inst.size();
  if (!p->krylov_dots) e = hipMalloc(&p->krylov_dots, B * 2 * kDotsStride * sizeof(double));
  if (e == hipSuccess && !p->krylov_part)
    e = hipMalloc(&p->krylov_part, (size_t)std::max(p->seg.ntiles, 1) * kDotsStride * sizeof(double));
  if (e == hipSuccess && !p->krylov_coef) {
    e = hipMalloc(&p->krylov_coef, B * kDotsStride * sizeof(double) + B * sizeof(int));
    if (e == hipSuccess) p->krylov_cnt = (int*)(p->krylov_coef + B * kDotsStride);
  }
  if (e == hipSuccess && !p->krylov_stage) e = hipHostMalloc(&p->krylov_stage, stage_bytes(B), hipHostMallocDefault);
  if (e == hipSuccess && !p->krylov_gm) e = hipMalloc(&p->krylov_gm, B * kGmStride * sizeof(double));
  if (e == hipSuccess && !p->krylov_prm) e = hipMalloc(&p->krylov_prm, 6 * B * sizeof(double));
  if (e != hipSuccess) return e;
  if (p->krylov_Q && p->krylov_m >= m) return hipSuccess;
  // recorded Arnoldi chunks hold the old buffers' addresses
  for (auto& g : p->kgraphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->kgraphs.clear();
  if (p->krylov_Q) (void)hipFree(p->krylov_Q);
  if (p->krylov_vec) (void)hipFree(p->krylov_vec);
  p->krylov_Q = p->krylov_vec = nullptr;
  // sized for double so that one allocation serves either Krylov precision
  (void)esize;
  // Q: m + 1 basis vectors; Z: m preconditioned vectors z_j = P^{-1} q_j (kept so the
  // update chi += P^{-1} Q y = Z y needs no further preconditioner application); double
  // plans also keep Y: the m vectors J z_j, so that J chi follows by the same combination
  const int nvec = (p->prec == BIRK_F64 ? 3 : 2) * m + 1;
  e = hipMalloc(&p->krylov_Q, (size_t)nvec * p->total_len * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->krylov_vec, (size_t)4 * p->total_len * sizeof(double));
  if (e == hipSuccess) p->krylov_m = m;
  return e;
}

// Per-instance ||v_i||^2 for a double vector (one segmented launch); results into host array.
hipError_t seg_norms(birk_plan* p, const double* v, std::vector<double>& out) {
  const int B = (int)p->inst.size();
  kry::sdots<double>(p, nullptr, 0, v, p->krylov_dots, 2 * kDotsStride, p->stream);
  const double* h = stage_dots(p);
  hipError_t e = hipMemcpyAsync(stage_dots(p), p->krylov_dots, (size_t)B * 2 * kDotsStride * sizeof(double),
                                hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  out.resize(B);
  for (int i = 0; i < B; ++i) {
    const double v = h[(size_t)i * 2 * kDotsStride + kKryMaxDots];
    // NaN must survive: std::max(0.0, NaN) would return 0
    out[i] = std::isfinite(v) ? std::sqrt(v > 0.0 ? v : 0.0) : std::numeric_limits<double>::quiet_NaN();
  }
  return e;
}

// One Arnoldi step j of every instance (stopped instances are carried along; the device
// state ignores their columns): z = P^{-1} q_j and y = J z (or y = J q_j without the
// preconditioner), t = B^a y, u = z - t, CGS2 against q_0..q_j, q_{j+1} = u / ||u||, and
// the device update of the Hessenberg column, rotations and g.
template <typename TK>
static hipError_t arnoldi_step(birk_plan* p, int jk, const double* J, int j, int m, int use_precond, bool keep_jz,
                               int cached) {
  const int64_t n = p->total_len;
  hipStream_t s = p->stream;
  TK* Q = (TK*)p->krylov_Q;
  TK* Z = Q + (size_t)(m + 1) * n;
  TK* u = (TK*)p->krylov_vec;
  TK* y = keep_jz ? Z + (size_t)m * n + (size_t)j * n : u + n;
  TK* t = u + 2 * n;
  const TK* qj = Q + (size_t)j * n;
  TK* z = Z + (size_t)j * n;
  const TK* uz = qj;
  hipError_t e;
  if (use_precond) {
    e = precond_inverse<TK>(p, jk, J, qj, z, y, s, p->flag, cached);
    uz = z;
  } else {
    e = jac_times<TK>(p, jk, J, qj, y, s);
  }
  if (e == hipSuccess) e = apply_product<TK>(p, y, t, 0, s);
  if (e != hipSuccess) return e;
  double* d1 = p->krylov_dots;
  double* d2 = d1 + kDotsStride;
  const int64_t ds = 2 * kDotsStride;
  kry::sub_sdots<TK>(p, Q, j + 1, uz, t, u, d1, ds, s);
  kry::saxpys_dots<TK>(p, Q, j + 1, d1, ds, u, d2, ds, s);
  kry::saxpys<TK>(p, Q, j + 1, d2, ds, u, d2, s);
  kry::snormalize<TK>(p, u, d2 + kKryMaxDots, ds, Q + (size_t)(j + 1) * n, s);
  kry::gm_column(p, j, p->krylov_dots, ds, p->krylov_gm, s);
  return hipGetLastError();
}

constexpr size_t kMaxKryGraphs = 48;

// Arnoldi steps [j0, j0 + k) on the plan's stream: launched eagerly, or in graph mode
// from a HIP graph recorded the first time this (precision, steps, Jacobian) chunk runs.
template <typename TK>
static hipError_t arnoldi_chunk(birk_plan* p, int jk, const double* J, int j0, int k, int m, int use_precond,
                                bool keep_jz, int cached) {
  if (!p->use_graphs) {
    for (int j = j0; j < j0 + k; ++j) {
      const hipError_t e = arnoldi_step<TK>(p, jk, J, j, m, use_precond, keep_jz, cached);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int prec = sizeof(TK) == 8 ? 0 : 1;
  for (const auto& g : p->kgraphs)
    if (g.prec == prec && g.j0 == j0 && g.k == k && g.m == m && g.J == J && g.jk == jk &&
        g.use_precond == use_precond && g.keep_jz == (int)keep_jz && g.cached == cached)
      return hipGraphLaunch(g.exec, p->stream);
  if (p->kgraphs.size() >= kMaxKryGraphs) {
    for (auto& g : p->kgraphs) (void)hipGraphExecDestroy(g.exec);
    p->kgraphs.clear();
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  for (int j = j0; j < j0 + k && e == hipSuccess; ++j)
    e = arnoldi_step<TK>(p, jk, J, j, m, use_precond, keep_jz, cached);
  const hipError_t e2 = hipStreamEndCapture(p->stream, &graph);
  if (e == hipSuccess) e = e2;
  birk_plan::KryGraph kg{prec, j0, k, m, J, jk, use_precond, (int)keep_jz, cached, nullptr};
  if (e == hipSuccess) e = hipGraphInstantiate(&kg.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  p->kgraphs.push_back(kg);
  return hipGraphLaunch(kg.exec, p->stream);
}

// One right-preconditioned GMRES cycle in precision TK on A d = r / ||r||, for every
// instance not yet done; chi += ||r|| d.  r: the current residual (double).  jchi
// (double plans, else null): J chi, updated alongside chi from the kept J z_j.  The
// Hessenberg columns, rotations and the small least-squares solve run on the device; the
// host reads the per-instance running flags after each of the first three steps, then
// (plans shorter than 2^20 elements) after chunks of 2, then 4 steps.
template <typename TK>
birk_status gmres_cycle(birk_plan* p, int jk, const double* J, const double* r, double* chi, double* jchi,
                        std::vector<InstState>& st, const std::vector<double>& tol_inner, int m, int use_precond,
                        int& budget, int& pinv_state) {
  const int B = (int)p->inst.size();
  const int64_t n = p->total_len;
  hipStream_t s = p->stream;
  TK* Q = (TK*)p->krylov_Q;
  TK* Z = Q + (size_t)(m + 1) * n;
  TK* Yb = jchi ? Z + (size_t)m * n : nullptr;  // J z_j, j < m
  hipError_t e = hipSuccess;

  std::vector<char> active(B, 0);
  for (int i = 0; i < B; ++i) active[i] = !st[i].done;
  // q_0 = r / ||r|| (zero for inactive instances), and the device state (active,
  // tolerance, ||r||); the pinned staging is rewritten only after the synchronisations
  // that follow these copies
  {
    double* sc = stage_coef(p);
    double* prm = sc + B;
    for (int i = 0; i < B; ++i) {
      sc[i] = active[i] && st[i].rnorm > 0 ? 1.0 / st[i].rnorm : 0.0;
      prm[3 * i] = active[i] ? 1.0 : 0.0;
      prm[3 * i + 1] = tol_inner[i];
      prm[3 * i + 2] = st[i].rnorm;
    }
    e = hipMemcpyAsync(p->krylov_coef, sc, B * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p->krylov_prm, prm, 3 * B * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
    kry::sscale_conv<double, TK>(p, r, Q, p->krylov_coef, s);
    kry::gm_init(p, p->krylov_prm, p->krylov_gm, s);
  }
  double* flags = stage_dots(p);
  int j = 0, checks = 0;
  bool flag_checked = !use_precond;
  // the first three chunks are single steps (most solves here converge within them, and a
  // step past convergence of a large batch costs more than a host read); small plans,
  // whose steps are short, then read the flags every 2, then 4 steps
  const bool small = n < (int64_t(1) << 20);
  while (j < m && budget > 0) {
    const int want = (!small || checks < 3) ? 1 : checks < 4 ? 2 : 4;
    const int k = std::min(want, std::min(m - j, budget));
    // the first P^{-1} of the solve forms K_k on the fly; per-node H_k are cached (one
    // preparation pass, outside any recorded chunk) before the second
    if (use_precond && pinv_state == 1) {
      if (precond_prepare(p, jk, J, sizeof(TK) == 4 ? 1 : 0, s, kPrepCache) != hipSuccess) return BIRK_ERR_DEVICE;
      pinv_state = 2;
    }
    e = arnoldi_chunk<TK>(p, jk, J, j, k, m, use_precond, Yb != nullptr, pinv_state == 2 ? 1 : 0);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
    if (pinv_state == 0) pinv_state = 1;
    j += k;
    budget -= k;
    ++checks;
    kry::gm_running(p, p->krylov_gm, p->krylov_prm + 3 * B, s);
    e = hipMemcpyAsync(flags, p->krylov_prm + 3 * B, B * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !flag_checked) e = hipMemcpyAsync(stage_flag(p), p->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
    if (!flag_checked) {
      flag_checked = true;
      if (*stage_flag(p)) {
        for (int i = 0; i < B; ++i) st[i].status = BIRK_ERR_SINGULAR;
        return BIRK_ERR_SINGULAR;
      }
    }
    bool any = false;
    for (int i = 0; i < B; ++i) any = any || flags[i] != 0.0;
    if (!any) break;
  }
  // y = R^{-1} g and chi += ||r|| Z y (Z = Q without preconditioning) on the device
  kry::gm_solve(p, p->krylov_gm, p->krylov_coef, kDotsStride, p->krylov_cnt, p->krylov_prm + 3 * B, s);
  const TK* basis = use_precond ? Z : Q;
  kry::scombine<TK>(p, basis, p->krylov_coef, kDotsStride, p->krylov_cnt, chi, s);
  // J chi += ||r|| J Z y (J Q y without preconditioning) from the kept J z_j
  if (Yb) kry::scombine<TK>(p, Yb, p->krylov_coef, kDotsStride, p->krylov_cnt, jchi, s);
  e = hipMemcpyAsync(flags, p->krylov_prm + 3 * B, 3 * B * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return BIRK_ERR_DEVICE;
  for (int i = 0; i < B; ++i) {
    if (!active[i]) continue;
    st[i].inner += (int)flags[3 * i + 1];
    const int stat = (int)flags[3 * i + 2];
    if (stat != 0) st[i].status = stat;
  }
  return BIRK_OK;
}

}  // namespace

extern "C" birk_status birk_krylov_solve(birk_plan* p, birk_jac_kind jk, const double* J, const double* beta, double* chi,
                              const birk_solve_opts* opts_in, birk_solve_info* info) {
  if (!p || !J || !beta || !chi || beta == chi) return BIRK_ERR_ARG;
  if (jk != BIRK_J_CONSTANT && jk != BIRK_J_PER_NODE) return BIRK_ERR_ARG;
  birk_solve_opts o;
  birk_solve_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (o.method == 1) {
    // MINRES on the symmetric form [[I, A^T], [A, 0]] [chi; lambda] = [0; beta]: A is square
    // and invertible, so its chi part solves A chi = beta
    if (o.max_iter < 1 || !(o.rtol > 0.0)) return BIRK_ERR_ARG;
    if (p->prec != BIRK_F64) return BIRK_ERR_UNSUPPORTED;
    if (o.use_precond && !nx_ok_for_precond(p)) return BIRK_ERR_UNSUPPORTED;
    DeviceGuard g(p->device);
    birk_solve_opts k = o;
    k.use_x0 = 0;
    if (o.use_x0) return BIRK_ERR_UNSUPPORTED;
    return kkt_solve(p, jk, J, nullptr, nullptr, beta, chi, nullptr, &k, info);
  }
  if (o.method != 0) return BIRK_ERR_ARG;
  if (o.restart < 1 || o.restart > kKryMaxDots - 1 || o.max_iter < 1 || !(o.rtol > 0.0)) return BIRK_ERR_ARG;
  if (p->prec == BIRK_F32 || p->prec == BIRK_DF32) return BIRK_ERR_UNSUPPORTED;
  if (o.use_precond && !nx_ok_for_precond(p)) return BIRK_ERR_UNSUPPORTED;
  const bool mixed = p->prec == BIRK_F32_REFINE_F64;
  if (mixed && (!(o.inner_rtol > 0.0) || o.max_refine < 1)) return BIRK_ERR_ARG;
  DeviceGuard g(p->device);
  const int B = (int)p->inst.size();
  const int64_t n = p->total_len;
  hipStream_t s = p->stream;
  hipError_t e = ensure_krylov(p, o.restart, mixed ? sizeof(float) : sizeof(double));
  if (e != hipSuccess) return dev_err(e);
  if (hipMemsetAsync(p->flag, 0, sizeof(int), s) != hipSuccess) return BIRK_ERR_DEVICE;
  // P^{-1} applications so far: 0, 1, or 2 = several (per-node H_k cached).  Mixed plans
  // cache the float H_k at once: their staged double J reads cost more than a float table.
  int pinv_state = mixed ? 2 : 0;
  if (o.use_precond && precond_prepare(p, jk, J, mixed ? 1 : 0, s, mixed ? kPrepLarge | kPrepCache : kPrepLarge) !=
                           hipSuccess)
    return BIRK_ERR_DEVICE;
  if (!o.use_x0 && hipMemsetAsync(chi, 0, n * sizeof(double), s) != hipSuccess) return BIRK_ERR_DEVICE;

  std::vector<InstState> st(B);
  std::vector<double> nb;
  if (seg_norms(p, beta, nb) != hipSuccess) return BIRK_ERR_DEVICE;
  for (int i = 0; i < B; ++i) st[i].bnorm = nb[i];

  int budget = o.max_iter;
  const int max_outer = mixed ? o.max_refine + 1 : o.max_iter + 1;
  birk_status result = BIRK_OK;
  double* r = (double*)p->tmp_vec[0];
  double* t = (double*)p->tmp_vec[1];
  // double plans carry J chi (tmp_vec[2]) alongside chi, updated from the kept J z_j, so
  // the true residual needs no Jacobian product; mixed plans form J chi from chi in double
  double* jchi = mixed ? nullptr : (double*)p->tmp_vec[2];
  if (jchi) {
    e = o.use_x0 ? jac_times<double>(p, jk, J, chi, jchi, s) : hipMemsetAsync(jchi, 0, n * sizeof(double), s);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
  }
  for (int outer = 0;; ++outer) {
    // true residual r = beta - A chi = beta - chi + B^a (J chi) in double (chi = 0 on the
    // first step without x0: r = beta, whose norms are known)
    const double* rcur = r;
    std::vector<double> rn;
    if (outer == 0 && !o.use_x0) {
      rcur = beta;
      rn = nb;
    } else {
      e = jchi ? apply_product<double>(p, jchi, t, 0, s) : fast_ax_f64(p, jk, J, chi, t);
      if (e != hipSuccess) return BIRK_ERR_DEVICE;
      kry::residual(beta, chi, t, r, n, s);
      if (seg_norms(p, r, rn) != hipSuccess) return BIRK_ERR_DEVICE;
    }
    bool all_done = true;
    for (int i = 0; i < B; ++i) {
      st[i].rnorm = rn[i];
      if (st[i].done) continue;
      if (!std::isfinite(rn[i])) {
        st[i].status = BIRK_ERR_NONFINITE;
        st[i].done = true;
        continue;
      }
      if (rn[i] <= o.rtol * st[i].bnorm) {
        st[i].status = BIRK_OK;
        st[i].done = true;
        continue;
      }
      if (st[i].status == BIRK_ERR_BREAKDOWN && st[i].breakdown_last) {
        st[i].done = true;
        continue;
      }
      all_done = false;
    }
    if (all_done) break;
    if (outer >= max_outer || budget <= 0) {
      for (int i = 0; i < B; ++i)
        if (!st[i].done) {
          st[i].status = BIRK_ERR_NOCONV;
          st[i].done = true;
        }
      break;
    }
    std::vector<double> tol(B, 0.0);
    for (int i = 0; i < B; ++i) {
      if (st[i].done) continue;
      const double need = 0.5 * o.rtol * st[i].bnorm / st[i].rnorm;
      tol[i] = mixed ? std::max(o.inner_rtol, need) : need;
      st[i].outer += 1;
      st[i].breakdown_last = st[i].status == BIRK_ERR_BREAKDOWN;
      if (st[i].status == BIRK_ERR_BREAKDOWN) st[i].status = BIRK_OK;
    }
    birk_status cs = mixed ? gmres_cycle<float>(p, jk, J, rcur, chi, nullptr, st, tol, o.restart, o.use_precond, budget,
                                                pinv_state)
                           : gmres_cycle<double>(p, jk, J, rcur, chi, jchi, st, tol, o.restart, o.use_precond, budget,
                                                 pinv_state);
    if (cs == BIRK_ERR_SINGULAR || cs == BIRK_ERR_DEVICE) {
      result = cs;
      for (int i = 0; i < B; ++i) st[i].done = true;
      break;
    }
    for (int i = 0; i < B; ++i)
      if (st[i].status == BIRK_ERR_NONFINITE) st[i].done = true;
  }
  for (int i = 0; i < B; ++i) {
    if (result == BIRK_OK && st[i].status != BIRK_OK) result = (birk_status)st[i].status;
    if (info) {
      if (info->status) info->status[i] = st[i].status;
      if (info->inner_iters) info->inner_iters[i] = st[i].inner;
      if (info->outer_iters) info->outer_iters[i] = st[i].outer;
      if (info->rel_resid_fp64) info->rel_resid_fp64[i] = st[i].bnorm > 0 ? st[i].rnorm / st[i].bnorm : st[i].rnorm;
    }
  }
  if (result == BIRK_ERR_SINGULAR && info && info->status)
    for (int i = 0; i < B; ++i) info->status[i] = BIRK_ERR_SINGULAR;
  return result;
}

// ------------------------------------------------------------------ the KKT form
extern "C" birk_status birk_kkt_solve(birk_plan* p, birk_jac_kind jk, const double* J, const double* h,
                                      const double* f, const double* g, double* chi, double* lam,
                                      const birk_solve_opts* opts_in, birk_solve_info* info) {
  if (!p || !J || !g || !chi) return BIRK_ERR_ARG;
  if (jk != BIRK_J_CONSTANT && jk != BIRK_J_PER_NODE) return BIRK_ERR_ARG;
  const void* in[] = {J, h, f, g};
  for (const void* a : in)
    if (a && (a == chi || a == lam)) return BIRK_ERR_ARG;
  if (lam && lam == chi) return BIRK_ERR_ARG;
  birk_solve_opts o;
  birk_solve_opts_default(&o);
  o.method = 1;
  if (opts_in) o = *opts_in;
  if (o.max_iter < 1 || !(o.rtol > 0.0) || (o.use_x0 != 0 && o.use_x0 != 1)) return BIRK_ERR_ARG;
  if (o.use_x0 && !lam) return BIRK_ERR_ARG;
  if (p->prec != BIRK_F64) return BIRK_ERR_UNSUPPORTED;
  if (o.use_precond && !nx_ok_for_precond(p)) return BIRK_ERR_UNSUPPORTED;
  DeviceGuard gd(p->device);
  return kkt_solve(p, jk, J, h, f, g, chi, lam, &o, info);
}

// ------------------------------------------------------------------ Newton on the IVP
namespace {

constexpr double kArmijo = 1e-4;
constexpr double kMinStep = 1.0 / 4096.0;

// Newton workspace: F, G, Gt, D, Xt, beta (total_len each), the per-node Jacobians, and
// per-instance step lengths, beta scales and combination counts.
hipError_t ensure_newton(birk_plan* p) {
  if (p->newton_buf) return hipSuccess;
  const size_t B = p->inst.size();
  const size_t bytes = (6 * (size_t)p->total_len + (size_t)p->total_jnode + 2 * B) * sizeof(double) + B * sizeof(int);
  return hipMalloc(&p->newton_buf, bytes);
}

struct NewtonBufs {
  double *F, *G, *Gt, *D, *Xt, *beta, *J, *lam, *alpha;
  int* cnt;
};

NewtonBufs newton_bufs(birk_plan* p) {
  NewtonBufs b;
  const int64_t n = p->total_len;
  double* q = (double*)p->newton_buf;
  b.F = q;
  b.G = q + n;
  b.Gt = q + 2 * n;
  b.D = q + 3 * n;
  b.Xt = q + 4 * n;
  b.beta = q + 5 * n;
  b.J = q + 6 * n;
  b.lam = b.J + p->total_jnode;
  b.alpha = b.lam + p->inst.size();
  b.cnt = (int*)(b.alpha + p->inst.size());
  return b;
}

birk_status eval_model(birk_plan* p, const birk_ivp_model& m, const double* X, double* F, double* J) {
  if (m.kind == BIRK_MODEL_TWO_BODY)
    return two_body(p, m.mu, m.scale, X, F, J, p->stream) == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
  return m.fn(m.ctx, X, F, J, (void*)p->stream);
}

// G = X - x^a b - B^a F(X), then the per-instance norms ||G|| and ||X||.
birk_status newton_residual(birk_plan* p, const birk_ivp_model& m, const double* xa, const double* X, double* F,
                            double* G, std::vector<double>& gn, std::vector<double>& xn) {
  birk_status st = eval_model(p, m, X, F, nullptr);
  if (st != BIRK_OK) return st;
  if (apply_product<double>(p, F, G, 0, p->stream) != hipSuccess) return BIRK_ERR_DEVICE;
  if (ivp_residual(p, xa, X, G, p->stream) != hipSuccess) return BIRK_ERR_DEVICE;
  if (seg_norms(p, G, gn) != hipSuccess || seg_norms(p, X, xn) != hipSuccess) return BIRK_ERR_DEVICE;
  return BIRK_OK;
}

hipError_t upload(double* dst, const std::vector<double>& h, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s);
  return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

}  // namespace

extern "C" {

void birk_newton_opts_default(birk_newton_opts* o) {
  if (!o) return;
  o->max_newton = 30;
  o->tol = 1e-13;
  o->line_search = 1;
  birk_solve_opts_default(&o->linear);
}

birk_status birk_two_body(birk_plan* p, double mu, double scale, const double* X, double* F, double* J) {
  if (!p || !X || (!F && !J) || X == F || X == J || (F && F == J)) return BIRK_ERR_ARG;
  for (const auto& in : p->inst)
    if (in.nx != 6) return BIRK_ERR_UNSUPPORTED;
  DeviceGuard g(p->device);
  return two_body(p, mu, scale, X, F, J, p->stream) == hipSuccess ? BIRK_OK : BIRK_ERR_DEVICE;
}

birk_status birk_newton_ivp(birk_plan* p, const birk_ivp_model* model, const double* xa, double* X,
                            const birk_newton_opts* opts_in, birk_newton_info* info) {
  if (!p || !model || !xa || !X) return BIRK_ERR_ARG;
  if (model->kind == BIRK_MODEL_TWO_BODY) {
    for (const auto& in : p->inst)
      if (in.nx != 6) return BIRK_ERR_UNSUPPORTED;
  } else if (model->kind != BIRK_MODEL_CALLBACK || !model->fn) {
    return BIRK_ERR_ARG;
  }
  birk_newton_opts o;
  birk_newton_opts_default(&o);
  if (opts_in) o = *opts_in;
  if (o.max_newton < 1 || !(o.tol > 0.0) || (o.line_search != 0 && o.line_search != 1)) return BIRK_ERR_ARG;
  if (o.linear.method != 0 || o.linear.restart < 1 || o.linear.restart > kKryMaxDots - 1 || o.linear.max_iter < 1 ||
      !(o.linear.rtol > 0.0))
    return o.linear.method == 1 ? BIRK_ERR_UNSUPPORTED : BIRK_ERR_ARG;
  if (p->prec == BIRK_F32_REFINE_F64 && (!(o.linear.inner_rtol > 0.0) || o.linear.max_refine < 1)) return BIRK_ERR_ARG;
  if (p->prec == BIRK_F32 || p->prec == BIRK_DF32) return BIRK_ERR_UNSUPPORTED;
  if (o.linear.use_precond && !nx_ok_for_precond(p)) return BIRK_ERR_UNSUPPORTED;
  DeviceGuard g(p->device);
  const int B = (int)p->inst.size();
  hipStream_t s = p->stream;
  hipError_t e = ensure_newton(p);
  if (e == hipSuccess) e = ensure_krylov(p, o.linear.restart, sizeof(double));
  if (e != hipSuccess) return dev_err(e);
  NewtonBufs b = newton_bufs(p);
  std::vector<int> status(B, BIRK_OK), iters(B, 0), lin(B, 0);
  std::vector<bool> done(B, false);
  std::vector<double> gn, xn, gtn, xtn;
  birk_status result = newton_residual(p, *model, xa, X, b.F, b.G, gn, xn);
  birk_solve_opts lo = o.linear;
  lo.use_x0 = 0;
  std::vector<int32_t> lst(B), lin_it(B);
  birk_solve_info li{lst.data(), lin_it.data(), nullptr, nullptr};
  for (int it = 0; result == BIRK_OK; ++it) {
    bool all_done = true;
    for (int i = 0; i < B; ++i) {
      if (done[i]) continue;
      if (!std::isfinite(gn[i])) {
        status[i] = BIRK_ERR_NONFINITE;
        done[i] = true;
      } else if (gn[i] <= o.tol * xn[i]) {
        done[i] = true;
      } else if (it == o.max_newton) {
        status[i] = BIRK_ERR_NOCONV;
        done[i] = true;
      } else {
        all_done = false;
      }
    }
    if (all_done) break;
    // Newton system [I - B^a df(X)] D = -G for the instances still running (zero
    // right-hand side, hence D = 0, for the others)
    result = eval_model(p, *model, X, b.F, b.J);
    if (result != BIRK_OK) break;
    std::vector<double> alpha(B);
    for (int i = 0; i < B; ++i) alpha[i] = done[i] ? 0.0 : -1.0;
    if (upload(b.alpha, alpha, s) != hipSuccess) {
      result = BIRK_ERR_DEVICE;
      break;
    }
    kry::sscale_conv<double, double>(p, b.G, b.beta, b.alpha, s);
    std::fill(lst.begin(), lst.end(), BIRK_OK);
    std::fill(lin_it.begin(), lin_it.end(), 0);
    const birk_status ls = birk_krylov_solve(p, BIRK_J_PER_NODE, b.J, b.beta, b.D, &lo, &li);
    if (ls != BIRK_OK && ls != BIRK_ERR_NOCONV && ls != BIRK_ERR_BREAKDOWN && ls != BIRK_ERR_NONFINITE) {
      result = ls;
      break;
    }
    for (int i = 0; i < B; ++i) {
      if (done[i]) continue;
      lin[i] += lin_it[i];
      iters[i] = it + 1;
      // an inexact step (NOCONV, BREAKDOWN) is still tried; a non-finite one is not
      if (lst[i] == BIRK_ERR_NONFINITE) {
        status[i] = BIRK_ERR_NONFINITE;
        done[i] = true;
      }
    }
    // backtracking: X_t = X + lam_i D per instance; accepted steps keep their length while
    // other instances go on halving; a failed instance keeps X (lam = 0)
    std::vector<double> lam(B);
    std::vector<int> pending(B, 0);
    for (int i = 0; i < B; ++i) {
      lam[i] = done[i] ? 0.0 : 1.0;
      pending[i] = done[i] ? 0 : 1;
    }
    for (;;) {
      // lam_i = 0 takes instance i out of the update (its D may not be finite)
      std::vector<int> cnt(B);
      for (int i = 0; i < B; ++i) cnt[i] = lam[i] > 0.0 ? 1 : 0;
      e = hipMemcpyAsync(b.cnt, cnt.data(), B * sizeof(int), hipMemcpyHostToDevice, s);
      if (e != hipSuccess || upload(b.lam, lam, s) != hipSuccess) {
        result = BIRK_ERR_DEVICE;
        break;
      }
      if (hipMemcpyAsync(b.Xt, X, p->total_len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
        result = BIRK_ERR_DEVICE;
        break;
      }
      kry::scombine<double>(p, b.D, b.lam, 1, b.cnt, b.Xt, s);
      result = newton_residual(p, *model, xa, b.Xt, b.F, b.Gt, gtn, xtn);
      if (result != BIRK_OK) break;
      bool again = false;
      for (int i = 0; i < B; ++i) {
        if (!pending[i]) continue;
        const bool ok = gtn[i] <= (1.0 - kArmijo * lam[i]) * gn[i] || gtn[i] <= o.tol * xtn[i];
        if (ok || !o.line_search) {
          pending[i] = 0;
          continue;
        }
        lam[i] *= 0.5;
        if (lam[i] < kMinStep) {
          lam[i] = 0.0;
          pending[i] = 0;
          status[i] = BIRK_ERR_NOCONV;
          done[i] = true;
        }
        again = true;   // X_t must be formed again with the new lengths
      }
      if (!again) break;
    }
    if (result != BIRK_OK) break;
    if (hipMemcpyAsync(X, b.Xt, p->total_len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
      result = BIRK_ERR_DEVICE;
      break;
    }
    std::swap(b.G, b.Gt);
    for (int i = 0; i < B; ++i) {
      if (lam[i] > 0.0 || !done[i]) {
        gn[i] = gtn[i];
        xn[i] = xtn[i];
      }
    }
  }
  if (result == BIRK_OK && hipStreamSynchronize(s) != hipSuccess) result = BIRK_ERR_DEVICE;
  for (int i = 0; i < B; ++i) {
    if (result == BIRK_OK && status[i] != BIRK_OK) result = (birk_status)status[i];
    if (info) {
      if (info->status) info->status[i] = status[i];
      if (info->newton_iters) info->newton_iters[i] = iters[i];
      if (info->linear_iters) info->linear_iters[i] = lin[i];
      if (info->rel_resid) info->rel_resid[i] = (i < (int)gn.size() && xn[i] > 0.0) ? gn[i] / xn[i] : gn.empty() ? -1.0 : gn[i];
    }
  }
  return result;
}

}  // extern "C"
