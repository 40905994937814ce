// b-form products and the endpoint row (arXiv 2509.01855, eq:xN=Birka+b, eq:Prob-PNa).
//
// The b-form basis is anchored at tau = +1 instead of -1 with the same derivative
// conditions (eq:birk-conditions), so B_j^b = B_j^a - B_j^a(1) and B^b = B^a - 1 w_B^T,
// w_B the last row of B^a (the Clenshaw-Curtis weights).  Every operation here is a
// per-component rank-one correction of a B^a product, or a weighted sum:
//
//   B^b v   = B^a v - 1 (B^a v)_N        ((B^a v)_N = w_B^T v, already in the product)
//   B^bT g  = B^aT g - w_B (1^T g)
//   x^b     = x^a + w_B^T v              (the endpoint row of eq:Prob-PNa)
//
// All three are bandwidth-bound passes over the vector.  Sums over a component are
// taken in double by a fixed tile split (per-tile partials, then the tiles in order),
// so results do not depend on scheduling.

#include "birk_internal.h"

namespace birk {
namespace {

constexpr int kThreads = 256;
constexpr int kElemsPerTile = 2048;   // elements summed by one reduction workgroup (at least)
constexpr unsigned kMaxGridY = 65535;

__host__ __device__ inline int comp_tiles(int64_t Nn) {
  const int64_t t = (Nn + kElemsPerTile - 1) / kElemsPerTile;
  return (int)(t < 1 ? 1 : (t > kCompTiles ? kCompTiles : t));
}

// Sum of a over the workgroup (256 threads, four waves of 64); the result is valid in
// thread 0.  Fixed order: wave tree, then the four wave sums pairwise.
__device__ inline double block_sum(double a, double* sh) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

template <typename T>
__device__ inline double ld(const T& x) {
  return (double)x;
}
template <typename T>
__device__ inline T st(double d) {
  return T(d);
}

// part[c.part + t] = sum over tile t of component c of x (WEIGHTED = 0) or of w_k x_k
// (WEIGHTED = 1).  grid = (max tiles, min(ncomp, 65535)); tiles past a component's own
// count return at once.  Each thread keeps four accumulators over strides of 256 nodes
// (fixed order), then the workgroup adds them as a tree.
template <typename T, int WEIGHTED>
__global__ __launch_bounds__(kThreads) void k_comp_reduce(const CompDesc* __restrict__ cd, int64_t ncomp,
                                                          const T* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[kThreads / 64];
  for (int64_t c = blockIdx.y; c < ncomp; c += gridDim.y) {
    const CompDesc d = cd[c];
    const int nt = comp_tiles(d.Nn);
    if ((int)blockIdx.x >= nt) continue;   // uniform over the workgroup
    const int64_t chunk = (d.Nn + nt - 1) / nt;
    const int64_t b = (int64_t)blockIdx.x * chunk;
    const int64_t e = b + chunk < d.Nn ? b + chunk : d.Nn;
    const T* xc = x + d.off;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t k = b + threadIdx.x;
    for (; k + 3 * kThreads < e; k += 4 * kThreads) {
      const double x0 = ld(xc[k]), x1 = ld(xc[k + kThreads]);
      const double x2 = ld(xc[k + 2 * kThreads]), x3 = ld(xc[k + 3 * kThreads]);
      if (WEIGHTED) {
        a0 += d.w[k] * x0;
        a1 += d.w[k + kThreads] * x1;
        a2 += d.w[k + 2 * kThreads] * x2;
        a3 += d.w[k + 3 * kThreads] * x3;
      } else {
        a0 += x0;
        a1 += x1;
        a2 += x2;
        a3 += x3;
      }
    }
    for (; k < e; k += kThreads) a0 += WEIGHTED ? d.w[k] * ld(xc[k]) : ld(xc[k]);
    const double s = block_sum((a0 + a1) + (a2 + a3), sh);
    if (threadIdx.x == 0) part[d.part + blockIdx.x] = s;
  }
}

// Totals of the tile partials, one wave per component (lane l adds tiles l, l + 64, ...
// in order, then a shuffle tree).  MODE 0: val[c] = total; MODE 1: xb[c] = xa[c] + total
// (xa may be xb).
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_comp_total(const CompDesc* __restrict__ cd, int64_t ncomp,
                                                         const double* __restrict__ part, double* val,
                                                         const double* xa) {
  const int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (c >= ncomp) return;   // whole waves leave together
  const int lane = threadIdx.x & 63;
  const CompDesc d = cd[c];
  const int nt = comp_tiles(d.Nn);
  double a = 0.0;
  for (int t = lane; t < nt; t += 64) a += part[d.part + t];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  if (lane == 0) val[c] = MODE == 0 ? a : xa[c] + a;
}

// val[c] = x[c][N]: the last node of every component (one thread per component).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_last_node(const CompDesc* __restrict__ cd, int64_t ncomp,
                                                        const T* __restrict__ x, double* __restrict__ val) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= ncomp) return;
  const CompDesc d = cd[c];
  val[c] = ld(x[d.off + d.Nn - 1]);
}

// x[c][k] -= val[c] for every node (MODE 0), or x[c][k] -= w_k val[c] (MODE 1).
// grid = (tiles over the longest component, min(ncomp, 65535)).
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_comp_correct(const CompDesc* __restrict__ cd, int64_t ncomp,
                                                           const double* __restrict__ val, T* __restrict__ x) {
  for (int64_t c = blockIdx.y; c < ncomp; c += gridDim.y) {
    const CompDesc d = cd[c];
    const double s = val[c];
    T* xc = x + d.off;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < d.Nn; k += (int64_t)gridDim.x * kThreads) {
      const double corr = MODE == 0 ? s : d.w[k] * s;
      xc[k] = st<T>(ld(xc[k]) - corr);
    }
  }
}

inline dim3 comp_grid(const birk_plan* p, unsigned gx) {
  return dim3(gx, (unsigned)std::min<int64_t>(p->ncomp, kMaxGridY));
}

// Tiles of the elementwise correction: about eight elements per thread on the longest
// component, at most 1024 workgroups per component.
inline unsigned correct_tiles(const birk_plan* p) {
  const int64_t t = (p->max_nn + kThreads * 8 - 1) / (kThreads * 8);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(t, 1024));
}

inline unsigned reduce_tiles(const birk_plan* p) { return (unsigned)comp_tiles(p->max_nn); }

inline unsigned per_comp_blocks(const birk_plan* p) { return (unsigned)((p->ncomp + kThreads - 1) / kThreads); }

inline unsigned per_comp_waves(const birk_plan* p) {
  return (unsigned)((p->ncomp + kThreads / 64 - 1) / (kThreads / 64));
}

}  // namespace

hipError_t plan_bform(birk_plan* p) {
  std::vector<CompDesc> h;
  h.reserve(p->inst.size());
  int64_t max_nn = 0, npart = 0;
  for (const Instance& in : p->inst) {
    for (int r = 0; r < in.nx; ++r) {
      h.push_back({in.off + r * in.Nn, in.Nn, in.w, npart});
      npart += comp_tiles(in.Nn);
    }
    max_nn = std::max(max_nn, in.Nn);
  }
  p->ncomp = (int64_t)h.size();
  p->max_nn = max_nn;
  void* cd = nullptr;
  hipError_t e = hipMalloc(&cd, h.size() * sizeof(CompDesc));
  if (e != hipSuccess) return e;
  p->allocs.push_back(cd);
  p->comps = (CompDesc*)cd;
  void* part = nullptr;
  e = hipMalloc(&part, (size_t)(npart + p->ncomp) * sizeof(double));
  if (e != hipSuccess) return e;
  p->allocs.push_back(part);
  p->comp_val = (double*)part;
  p->comp_part = p->comp_val + p->ncomp;
  e = hipMemcpyAsync(cd, h.data(), h.size() * sizeof(CompDesc), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return e;
}

template <typename T>
hipError_t bform_correct(birk_plan* p, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_last_node<T>), dim3(per_comp_blocks(p)), dim3(kThreads), 0, s, p->comps, p->ncomp,
                     (const T*)out, p->comp_val);
  hipLaunchKernelGGL((k_comp_correct<T, 0>), comp_grid(p, correct_tiles(p)), dim3(kThreads), 0, s, p->comps,
                     p->ncomp, (const double*)p->comp_val, out);
  return hipGetLastError();
}

template <typename T>
hipError_t bform_sums(birk_plan* p, const T* g, hipStream_t s) {
  hipLaunchKernelGGL((k_comp_reduce<T, 0>), comp_grid(p, reduce_tiles(p)), dim3(kThreads), 0, s, p->comps,
                     p->ncomp, g, p->comp_part);
  hipLaunchKernelGGL(k_comp_total<0>, dim3(per_comp_waves(p)), dim3(kThreads), 0, s, p->comps, p->ncomp,
                     (const double*)p->comp_part, p->comp_val, (const double*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t bform_correct_T(birk_plan* p, T* out, hipStream_t s) {
  hipLaunchKernelGGL((k_comp_correct<T, 1>), comp_grid(p, correct_tiles(p)), dim3(kThreads), 0, s, p->comps,
                     p->ncomp, (const double*)p->comp_val, out);
  return hipGetLastError();
}

template <typename T>
hipError_t endpoint(birk_plan* p, const double* xa, const T* v, double* xb, hipStream_t s) {
  hipLaunchKernelGGL((k_comp_reduce<T, 1>), comp_grid(p, reduce_tiles(p)), dim3(kThreads), 0, s, p->comps,
                     p->ncomp, v, p->comp_part);
  hipLaunchKernelGGL(k_comp_total<1>, dim3(per_comp_waves(p)), dim3(kThreads), 0, s, p->comps, p->ncomp,
                     (const double*)p->comp_part, xb, xa);
  return hipGetLastError();
}

#define BIRK_BFORM_INST(T)                                                              \
  template hipError_t bform_correct<T>(birk_plan*, T*, hipStream_t);                    \
  template hipError_t bform_sums<T>(birk_plan*, const T*, hipStream_t);                 \
  template hipError_t bform_correct_T<T>(birk_plan*, T*, hipStream_t);                  \
  template hipError_t endpoint<T>(birk_plan*, const double*, const T*, double*, hipStream_t);
BIRK_BFORM_INST(double)
BIRK_BFORM_INST(float)
BIRK_BFORM_INST(df32)
#undef BIRK_BFORM_INST

}  // namespace birk
