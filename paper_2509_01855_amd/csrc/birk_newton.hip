// Kernels of the Newton solve of the nonlinear IVP (arXiv 2509.01855, eq:X-V=nonlin,
// eq:Newton-ivp): the two-body right-hand side with its per-node Jacobian, and the
// residual G = X - x^a b - B^a F once the product B^a F is in G.
//
// Two-body model, state x = (r, v): dx/dtau = s (v, -mu r / |r|^3) with
// df/dx = s [[0, I], [mu (3 r r^T / |r|^2 - I) / |r|^3, 0]].  Both are one pass over the
// nodes: 48 bytes read and 48 (F) + 288 (J) bytes written per node.

#include "birk_internal.h"

namespace birk {
namespace {

constexpr int kThreads = 256;
constexpr unsigned kMaxGridY = 65535;

// grid = (tiles over the longest instance, min(batch, 65535)); per node k of instance i.
__global__ __launch_bounds__(kThreads) void k_two_body(const InstDesc* __restrict__ idesc, int64_t ninst,
                                                       double mu, double scale, const double* __restrict__ X,
                                                       double* __restrict__ F, double* __restrict__ J) {
  for (int64_t i = blockIdx.y; i < ninst; i += gridDim.y) {
    const InstDesc d = idesc[i];
    const int64_t Nn = d.Nn;
    const double* x = X + d.off;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < Nn; k += (int64_t)gridDim.x * kThreads) {
      const double r0 = x[k], r1 = x[Nn + k], r2 = x[2 * Nn + k];
      const double rr = r0 * r0 + r1 * r1 + r2 * r2;
      const double inv_r = 1.0 / sqrt(rr);
      const double inv_r3 = inv_r * inv_r * inv_r;
      const double g = -scale * mu * inv_r3;   // acceleration factor
      if (F) {
        double* f = F + d.off;
        f[k] = scale * x[3 * Nn + k];
        f[Nn + k] = scale * x[4 * Nn + k];
        f[2 * Nn + k] = scale * x[5 * Nn + k];
        f[3 * Nn + k] = g * r0;
        f[4 * Nn + k] = g * r1;
        f[5 * Nn + k] = g * r2;
      }
      if (J) {
        double* j = J + d.joff;
        const double r[3] = {r0, r1, r2};
        const double c3 = 3.0 * scale * mu * inv_r3 / rr;
        const double c1 = scale * mu * inv_r3;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            double val = 0.0;
            if (a < 3) {
              val = (b == a + 3) ? scale : 0.0;
            } else if (b < 3) {
              val = c3 * r[a - 3] * r[b] - (a - 3 == b ? c1 : 0.0);
            }
            j[(int64_t)(a * 6 + b) * Nn + k] = val;
          }
        }
      }
    }
  }
}

// G[c][k] = X[c][k] - xa[c] - G[c][k] for every component c (G holds B^a F on entry).
__global__ __launch_bounds__(kThreads) void k_ivp_residual(const CompDesc* __restrict__ cd, int64_t ncomp,
                                                           const double* __restrict__ xa,
                                                           const double* __restrict__ X, double* __restrict__ G) {
  for (int64_t c = blockIdx.y; c < ncomp; c += gridDim.y) {
    const CompDesc d = cd[c];
    const double a = xa[c];
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < d.Nn; k += (int64_t)gridDim.x * kThreads)
      G[d.off + k] = X[d.off + k] - a - G[d.off + k];
  }
}

inline unsigned node_tiles(const birk_plan* p) {
  const int64_t t = (p->max_nn + kThreads * 4 - 1) / (kThreads * 4);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(t, 2048));
}

}  // namespace

hipError_t plan_instances(birk_plan* p) {
  std::vector<InstDesc> h;
  h.reserve(p->inst.size());
  for (const Instance& in : p->inst)
    h.push_back({in.off, in.Nn, in.joff, (int64_t)in.nx, in.jcoff, in.scan_off, in.w});
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, h.size() * sizeof(InstDesc));
  if (e != hipSuccess) return e;
  p->allocs.push_back(d);
  p->idesc = (InstDesc*)d;
  e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(InstDesc), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  return e;
}

hipError_t two_body(birk_plan* p, double mu, double scale, const double* X, double* F, double* J, hipStream_t s) {
  const int64_t ninst = (int64_t)p->inst.size();
  hipLaunchKernelGGL(k_two_body, dim3(node_tiles(p), (unsigned)std::min<int64_t>(ninst, kMaxGridY)), dim3(kThreads),
                     0, s, p->idesc, ninst, mu, scale, X, F, J);
  return hipGetLastError();
}

hipError_t ivp_residual(birk_plan* p, const double* xa, const double* X, double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_ivp_residual, dim3(node_tiles(p), (unsigned)std::min<int64_t>(p->ncomp, kMaxGridY)),
                     dim3(kThreads), 0, s, p->comps, p->ncomp, xa, X, G);
  return hipGetLastError();
}

}  // namespace birk
