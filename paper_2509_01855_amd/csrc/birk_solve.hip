// Jacobian products, the Birkhoff preconditioner and the Krylov BLAS-1 kernels (gfx950).
//
// Preconditioner (arXiv 2509.01855, "Development of a Special Birkhoff-Centric
// Preconditioner"): P = I - B~^a J with B~^a lower triangular, w_j below the diagonal
// and w_j / 2 on it (w = CC weights).
//
//   P y:      y - B~^a (J y); B~^a u is an exclusive prefix sum of w u plus w u / 2
//             (FastBccV).  Three kernels: block sums, a scan of the block sums, and
//             the block-local scan.  Sums are carried in double.
//   P^{-1} y: exact block forward substitution (FastPinvY box, with its running-sum
//             update read as forward substitution):
//                 xi_k = K_k^{-1} (y_k + S_k),  K_k = I - w_k J_k / 2,
//                 S_{k+1} = S_k + w_k J_k xi_k.
//             As an affine map of the carried sum, S_{k+1} = G_k S_k + h_k with
//             G_k = I + w_k J_k K_k^{-1} and h_k = w_k J_k K_k^{-1} y_k.  The chain is
//             evaluated as a hierarchical scan of affine maps: chunks of kChunk nodes
//             (one thread each) are reduced to (A, b) with S_out = A S_in + b, then
//             groups of kFan aggregates per level up to a single sequential top, then
//             start states are pushed back down and each chunk is replayed from its
//             start state, emitting xi_k and J_k xi_k (the latter feeds FastAX).
//             All arithmetic in double; y, xi and J xi are stored in the plan type.

#include <hip/hip_runtime.h>

#include <cmath>

#include "birk_internal.h"

namespace birk {

constexpr int kChunk = 16;
constexpr int kFan = 16;

// ------------------------------------------------------------------ J x per node
template <typename T>
__global__ void k_jac_times(const double* __restrict__ J, int per_node, const T* __restrict__ x,
                            T* __restrict__ y, int nx, int64_t Nn) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nn) return;
  for (int r = 0; r < nx; ++r) {
    double acc = 0.0;
    for (int c = 0; c < nx; ++c) {
      const double j = per_node ? J[((int64_t)(r * nx + c)) * Nn + k] : J[r * nx + c];
      acc += j * (double)x[(int64_t)c * Nn + k];
    }
    y[(int64_t)r * Nn + k] = (T)acc;
  }
}

template <typename T>
hipError_t jac_times(birk_plan* p, int jac_kind, const double* J, const T* x, T* y, hipStream_t s) {
  for (const Instance& in : p->inst) {
    const double* Ji = J + (jac_kind == BIRK_J_PER_NODE ? in.joff : in.jcoff);
    hipLaunchKernelGGL(k_jac_times<T>, dim3((unsigned)((in.Nn + 255) / 256)), dim3(256), 0, s, Ji,
                       jac_kind == BIRK_J_PER_NODE ? 1 : 0, x + in.off, y + in.off, in.nx, in.Nn);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ P y (forward)
constexpr int kScanItems = 4;
constexpr int kScanBlock = 256 * kScanItems;

template <typename T>
__device__ __forceinline__ double wju(const double* __restrict__ J, int per_node, const T* __restrict__ y,
                                      const double* __restrict__ w, int r, int nx, int64_t Nn, int64_t k) {
  double acc = 0.0;
  for (int c = 0; c < nx; ++c) {
    const double j = per_node ? J[((int64_t)(r * nx + c)) * Nn + k] : J[r * nx + c];
    acc += j * (double)y[(int64_t)c * Nn + k];
  }
  return w[k] * acc;
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// grid = (blocks over nodes, nx)
template <typename T>
__global__ __launch_bounds__(256) void k_pfwd_sums(const double* __restrict__ J, int per_node,
                                                   const T* __restrict__ y, const double* __restrict__ w,
                                                   int nx, int64_t Nn, double* __restrict__ part) {
  __shared__ double sh[256];
  const int r = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  double acc = 0.0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + threadIdx.x * kScanItems + i;
    if (k < Nn) acc += wju<T>(J, per_node, y, w, r, nx, Nn, k);
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = s;
}

__global__ void k_pfwd_scanparts(double* __restrict__ part, int nblk, int nx) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nx) return;
  double run = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double v = part[(int64_t)r * nblk + b];
    part[(int64_t)r * nblk + b] = run;
    run += v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pfwd_final(const double* __restrict__ J, int per_node,
                                                    const T* __restrict__ y, const double* __restrict__ w,
                                                    int nx, int64_t Nn, const double* __restrict__ part,
                                                    T* __restrict__ out) {
  __shared__ double sh[256];
  const int r = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  double u[kScanItems];
  double tsum = 0.0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + threadIdx.x * kScanItems + i;
    u[i] = (k < Nn) ? wju<T>(J, per_node, y, w, r, nx, Nn, k) : 0.0;
    tsum += u[i];
  }
  // exclusive scan of the per-thread sums (Hillis-Steele in LDS)
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int st = 1; st < 256; st <<= 1) {
    const double v = threadIdx.x >= st ? sh[threadIdx.x - st] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  double run = part[(int64_t)r * gridDim.x + blockIdx.x] + sh[threadIdx.x] - tsum;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + threadIdx.x * kScanItems + i;
    if (k < Nn) {
      const double bt = run + 0.5 * u[i];
      out[(int64_t)r * Nn + k] = (T)((double)y[(int64_t)r * Nn + k] - bt);
    }
    run += u[i];
  }
}

template <typename T>
hipError_t precond_forward(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           hipStream_t s) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const Instance& in : p->inst) {
    const double* Ji = J + (pn ? in.joff : in.jcoff);
    const int nblk = (int)((in.Nn + kScanBlock - 1) / kScanBlock);
    double* part = p->scan + in.scan_off;  // nx * nblk doubles (fits: scan scratch is larger)
    hipLaunchKernelGGL(k_pfwd_sums<T>, dim3(nblk, in.nx), dim3(256), 0, s, Ji, pn, y + in.off, in.w,
                       in.nx, in.Nn, part);
    hipLaunchKernelGGL(k_pfwd_scanparts, dim3(1), dim3(64), 0, s, part, nblk, in.nx);
    hipLaunchKernelGGL(k_pfwd_final<T>, dim3(nblk, in.nx), dim3(256), 0, s, Ji, pn, y + in.off, in.w,
                       in.nx, in.Nn, part, out + in.off);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ P^{-1} y (inverse)

// Unpivoted LU of K = I - (w/2) Jk in place, with reciprocal pivots.  K is strongly
// diagonally dominant on the configurations of interest (w_k <= ~pi/N).  A pivot that
// is non-finite, or not above 1e-13 times the scale 1 + |w/2| max|J_k| of K, marks K as
// numerically singular in *flag.
template <int NX>
__device__ __forceinline__ void lu_kmat(double (&K)[NX][NX], double (&rp)[NX], int* flag, double scale) {
#pragma unroll
  for (int p = 0; p < NX; ++p) {
    const double piv = K[p][p];
    if (flag && (!(fabs(piv) > 1e-13 * scale) || !isfinite(piv))) atomicOr(flag, 1);
    rp[p] = 1.0 / piv;
#pragma unroll
    for (int i = p + 1; i < NX; ++i) {
      const double f = K[i][p] * rp[p];
      K[i][p] = f;
#pragma unroll
      for (int j = p + 1; j < NX; ++j) K[i][j] -= f * K[p][j];
    }
  }
}

template <int NX>
__device__ __forceinline__ void lu_solve(const double (&K)[NX][NX], const double (&rp)[NX], double (&x)[NX]) {
#pragma unroll
  for (int i = 1; i < NX; ++i) {
#pragma unroll
    for (int j = 0; j < i; ++j) x[i] -= K[i][j] * x[j];
  }
#pragma unroll
  for (int i = NX - 1; i >= 0; --i) {
#pragma unroll
    for (int j = i + 1; j < NX; ++j) x[i] -= K[i][j] * x[j];
    x[i] *= rp[i];
  }
}

template <int NX>
__device__ __forceinline__ void load_jk(const double* __restrict__ J, int per_node, int64_t Nn, int64_t k,
                                        double (&Jk)[NX][NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) Jk[r][c] = per_node ? J[((int64_t)(r * NX + c)) * Nn + k] : J[r * NX + c];
}

template <int NX>
__device__ __forceinline__ void form_k(const double (&Jk)[NX][NX], double wk, double (&K)[NX][NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) K[r][c] = (r == c ? 1.0 : 0.0) - 0.5 * wk * Jk[r][c];
}

// ---- level-0 layout ----
// Chunks of kChunk consecutive nodes are reduced by one thread each.  Chunk c is child
// i = c % kFan of level-1 group g = c / kFan.  Level-0 threads are laid out so that the
// 64 lanes of a wave hold 64 consecutive groups g and the wave index within a block of
// kFan waves is the child index i:  thread tau -> block B = tau / (64 kFan),
// i = (tau / 64) % kFan, lane l = tau % 64, g = 64 B + l, c = kFan g + i.
// Every per-chunk array (swizzled Jacobians, aggregates, start states) is stored as
// [B][i][field][l], so each access of a wave is 64 consecutive doubles.
__device__ __forceinline__ int64_t swz(int64_t B, int i, int field, int nfield, int l) {
  return (((B * kFan + i) * nfield) + field) * 64 + l;
}

// Swizzle per-node data for the level-0 kernels: field e < nx^2 is J entry e at the node
// (per-node Jacobians only), the last field is w_k.  Node k -> chunk c = k / kChunk,
// j = k % kChunk; g = c / kFan, i = c % kFan; B = g / 64, l = g % 64; stored at
// jsw[(((B kFan + i) kChunk + j) E + e) 64 + l] with E = fields.  Nodes past N_n are zero
// (identity maps).  One workgroup per (B, i, e): for each of the 64 lanes l it reads the
// kChunk consecutive nodes of chunk (64 B + l) kFan + i, and writes kChunk rows of 64
// consecutive lanes, transposing through LDS.
template <typename JT>
__global__ __launch_bounds__(256) void k_swizzle_nodes(const double* __restrict__ J, int per_node,
                                                       const double* __restrict__ w, int nx, int64_t Nn,
                                                       JT* __restrict__ jsw) {
  __shared__ double tile[64][kChunk + 1];
  const int E = per_node ? nx * nx + 1 : 1;
  const int e = blockIdx.y;
  const int i = blockIdx.x % kFan;
  const int64_t B = blockIdx.x / kFan;
  const double* src = (e == E - 1) ? w : J + (int64_t)e * Nn;
  for (int t = threadIdx.x; t < 64 * kChunk; t += blockDim.x) {
    const int l = t / kChunk, j = t % kChunk;
    const int64_t k = (((B * 64 + l) * kFan + i) * kChunk) + j;
    tile[l][j] = (k < Nn) ? src[k] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * kChunk; t += blockDim.x) {
    const int l = t & 63, j = t >> 6;
    jsw[((((B * kFan + i) * kChunk) + j) * E + e) * 64 + l] = (JT)tile[l][j];
  }
}

template <int NX, typename JT>
__device__ __forceinline__ void load_jk_sw(const JT* __restrict__ jsw, const double* __restrict__ Jc,
                                           int per_node, int64_t slot, double (&Jk)[NX][NX], double& wk) {
  // slot = ((B kFan + i) kChunk + j); per-node: fields 0..NX^2-1 then w; constant: w only
  const int E = per_node ? NX * NX + 1 : 1;
  const JT* base = jsw + slot * E * 64;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int q = 0; q < NX; ++q) Jk[r][q] = per_node ? (double)base[(r * NX + q) * 64 + l] : Jc[r * NX + q];
  wk = (double)base[(E - 1) * 64 + l];
}

// Level-0 up-sweep: each thread reduces one chunk of kChunk nodes to (A, b) with
// S_out = A S_in + b.
template <int NX, typename T>
__global__ __launch_bounds__(256) void k_pinv_up0(const T* __restrict__ jsw, const double* __restrict__ Jc,
                                                  int per_node, int64_t Nn, const T* __restrict__ y,
                                                  int64_t nchunks, double* __restrict__ agg, int* flag) {
  const int64_t tau = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t B = tau / (64 * kFan);
  const int i = (int)((tau >> 6) % kFan);
  const int l = (int)(tau & 63);
  const int64_t g = B * 64 + l;
  const int64_t c = g * kFan + i;
  if (c >= nchunks) return;
  constexpr int F = NX * NX + NX;
  double A[NX][NX], b[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    b[r] = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) A[r][q] = (r == q) ? 1.0 : 0.0;
  }
  const int64_t k0 = c * kChunk;
  const int jn = (int)min((int64_t)kChunk, Nn - k0);
  for (int j = 0; j < jn; ++j) {
    const int64_t k = k0 + j;
    double Jk[NX][NX], K[NX][NX], rp[NX], wk;
    load_jk_sw<NX, T>(jsw, Jc, per_node, (B * kFan + i) * kChunk + j, Jk, wk);
    double x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) x[r] = (double)y[(int64_t)r * Nn + k];
    form_k<NX>(Jk, wk, K);
    double jmax = 0.0;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int q = 0; q < NX; ++q) jmax = fmax(jmax, fabs(Jk[r][q]));
    lu_kmat<NX>(K, rp, flag, 1.0 + 0.5 * fabs(wk) * jmax);
    // b <- b + wk Jk K^{-1} (b + y_k)
#pragma unroll
    for (int r = 0; r < NX; ++r) x[r] += b[r];
    lu_solve<NX>(K, rp, x);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += Jk[r][q] * x[q];
      b[r] += wk * acc;
    }
    // A <- A + wk Jk K^{-1} A, column by column
#pragma unroll
    for (int col = 0; col < NX; ++col) {
      double xc[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) xc[r] = A[r][col];
      lu_solve<NX>(K, rp, xc);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) acc += Jk[r][q] * xc[q];
        A[r][col] += wk * acc;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int q = 0; q < NX; ++q) agg[swz(B, i, r * NX + q, F, l)] = A[r][q];
#pragma unroll
  for (int r = 0; r < NX; ++r) agg[swz(B, i, NX * NX + r, F, l)] = b[r];
}

// Level 0 -> 1 up-sweep: thread per group g combines its kFan chunk aggregates, stored
// swizzled, into a plain-layout level-1 aggregate.
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_up_sw(const double* __restrict__ child, int64_t nchild,
                                                    double* __restrict__ parent, int64_t nparent) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nparent) return;
  constexpr int F = NX * NX + NX;
  const int64_t B = g >> 6;
  const int l = (int)(g & 63);
  double A[NX][NX], b[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    b[r] = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) A[r][q] = (r == q) ? 1.0 : 0.0;
  }
  const int nc = (int)min((int64_t)kFan, nchild - g * kFan);
  for (int i = 0; i < nc; ++i) {
    double a[F];
#pragma unroll
    for (int f = 0; f < F; ++f) a[f] = child[swz(B, i, f, F, l)];
    double nb[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = a[NX * NX + r];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * b[q];
      nb[r] = acc;
    }
#pragma unroll
    for (int col = 0; col < NX; ++col) {
      double ncol[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * A[q][col];
        ncol[r] = acc;
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) A[r][col] = ncol[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) b[r] = nb[r];
  }
  double* o = parent + g * F;
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int q = 0; q < NX; ++q) o[r * NX + q] = A[r][q];
#pragma unroll
  for (int r = 0; r < NX; ++r) o[NX * NX + r] = b[r];
}

// Level 1 -> 0 down-sweep: group g pushes its start state through its chunks, writing
// swizzled chunk start states.
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_down_sw(const double* __restrict__ child, int64_t nchild,
                                                      const double* __restrict__ pstate, int64_t nparent,
                                                      double* __restrict__ cstate) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nparent) return;
  constexpr int F = NX * NX + NX;
  const int64_t B = g >> 6;
  const int l = (int)(g & 63);
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = pstate[g * NX + r];
  const int nc = (int)min((int64_t)kFan, nchild - g * kFan);
  for (int i = 0; i < nc; ++i) {
#pragma unroll
    for (int r = 0; r < NX; ++r) cstate[swz(B, i, r, NX, l)] = s[r];
    double ns[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = child[swz(B, i, NX * NX + r, F, l)];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += child[swz(B, i, r * NX + q, F, l)] * s[q];
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] = ns[r];
  }
}

// Up-sweep one level: thread per parent combines up to kFan child aggregates in order.
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_up(const double* __restrict__ child, int64_t nchild,
                                                 double* __restrict__ parent, int64_t nparent) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nparent) return;
  constexpr int S = NX * NX + NX;
  double A[NX][NX], b[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    b[r] = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) A[r][q] = (r == q) ? 1.0 : 0.0;
  }
  const int64_t c0 = g * kFan, c1 = min(c0 + (int64_t)kFan, nchild);
  for (int64_t c = c0; c < c1; ++c) {
    const double* a = child + c * S;
    // (A, b) <- (Ac A, Ac b + bc)
    double nb[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = a[NX * NX + r];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * b[q];
      nb[r] = acc;
    }
#pragma unroll
    for (int col = 0; col < NX; ++col) {
      double nc[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * A[q][col];
        nc[r] = acc;
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) A[r][col] = nc[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) b[r] = nb[r];
  }
  double* o = parent + g * S;
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int q = 0; q < NX; ++q) o[r * NX + q] = A[r][q];
#pragma unroll
  for (int r = 0; r < NX; ++r) o[NX * NX + r] = b[r];
}

// Top: one thread walks the top-level aggregates from S = 0, writing start states.
template <int NX>
__global__ void k_pinv_top(const double* __restrict__ agg, int64_t n, double* __restrict__ state) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  constexpr int S = NX * NX + NX;
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double* a = agg + i * S;
#pragma unroll
    for (int r = 0; r < NX; ++r) state[i * NX + r] = s[r];
    double ns[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = a[NX * NX + r];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * s[q];
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] = ns[r];
  }
}

// Single group (at most kFan chunks): walk the swizzled level-0 aggregates of group 0
// from S = 0 and write their swizzled start states.
template <int NX>
__global__ void k_pinv_top1(const double* __restrict__ agg, int64_t n, double* __restrict__ state) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  constexpr int F = NX * NX + NX;
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = 0.0;
  for (int i = 0; i < (int)n; ++i) {
#pragma unroll
    for (int r = 0; r < NX; ++r) state[swz(0, i, r, NX, 0)] = s[r];
    double ns[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = agg[swz(0, i, NX * NX + r, F, 0)];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += agg[swz(0, i, r * NX + q, F, 0)] * s[q];
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] = ns[r];
  }
}

// Down-sweep one level: thread per parent pushes its start state through its children.
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_down(const double* __restrict__ child, int64_t nchild,
                                                   const double* __restrict__ pstate, int64_t nparent,
                                                   double* __restrict__ cstate) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nparent) return;
  constexpr int S = NX * NX + NX;
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = pstate[g * NX + r];
  const int64_t c0 = g * kFan, c1 = min(c0 + (int64_t)kFan, nchild);
  for (int64_t c = c0; c < c1; ++c) {
    const double* a = child + c * S;
#pragma unroll
    for (int r = 0; r < NX; ++r) cstate[c * NX + r] = s[r];
    double ns[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = a[NX * NX + r];
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += a[r * NX + q] * s[q];
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] = ns[r];
  }
}

// Replay each chunk from its start state (same thread layout as k_pinv_up0): xi_k and
// (J xi)_k.
template <int NX, typename T>
__global__ __launch_bounds__(256) void k_pinv_final(const T* __restrict__ jsw, const double* __restrict__ Jc,
                                                    int per_node, int64_t Nn, const T* __restrict__ y,
                                                    int64_t nchunks, const double* __restrict__ state,
                                                    T* __restrict__ out, T* __restrict__ jout) {
  const int64_t tau = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t B = tau / (64 * kFan);
  const int i = (int)((tau >> 6) % kFan);
  const int l = (int)(tau & 63);
  const int64_t g = B * 64 + l;
  const int64_t c = g * kFan + i;
  if (c >= nchunks) return;
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = state[swz(B, i, r, NX, l)];
  const int64_t k0 = c * kChunk;
  const int jn = (int)min((int64_t)kChunk, Nn - k0);
  for (int j = 0; j < jn; ++j) {
    const int64_t k = k0 + j;
    double Jk[NX][NX], K[NX][NX], rp[NX], wk;
    load_jk_sw<NX, T>(jsw, Jc, per_node, (B * kFan + i) * kChunk + j, Jk, wk);
    double x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) x[r] = s[r] + (double)y[(int64_t)r * Nn + k];
    form_k<NX>(Jk, wk, K);
    lu_kmat<NX>(K, rp, nullptr, 1.0);
    lu_solve<NX>(K, rp, x);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += Jk[r][q] * x[q];
      s[r] += wk * acc;
      out[(int64_t)r * Nn + k] = (T)x[r];
      if (jout) jout[(int64_t)r * Nn + k] = (T)acc;
    }
  }
}

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Level sizes of the scan for one instance: cnt[0] chunks, then groups of kFan.
static int pinv_levels(int64_t Nn, int64_t* cnt) {
  int L = 0;
  cnt[0] = (Nn + kChunk - 1) / kChunk;
  while (cnt[L] > kFan && L < 15) {
    cnt[L + 1] = (cnt[L] + kFan - 1) / kFan;
    ++L;
  }
  return L;
}

// Level-0 threads (and swizzled slots) are allocated in blocks of 64 groups.
static int64_t pinv_blocks0(int64_t nchunks) {
  const int64_t groups = (nchunks + kFan - 1) / kFan;
  return (groups + 63) / 64;
}

int64_t pinv_jsw_size(int64_t Nn, int nx) {
  int64_t cnt[16];
  pinv_levels(Nn, cnt);
  return pinv_blocks0(cnt[0]) * 64 * kFan * kChunk * ((int64_t)nx * nx + 1);
}

hipError_t precond_prepare(birk_plan* p, int jac_kind, const double* J, int single, hipStream_t s) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const Instance& in : p->inst) {
    int64_t cnt[16];
    pinv_levels(in.Nn, cnt);
    const int64_t nslots = pinv_blocks0(cnt[0]) * kFan * kChunk;
    const int E = pn ? in.nx * in.nx + 1 : 1;
    const double* Ji = J + (pn ? in.joff : in.jcoff);
    const dim3 grid((unsigned)(pinv_blocks0(cnt[0]) * kFan), E);
    (void)nslots;
    if (single)
      hipLaunchKernelGGL(k_swizzle_nodes<float>, grid, dim3(256), 0, s, Ji, pn, in.w, in.nx, in.Nn,
                         (float*)p->jsw + in.jsw_off);
    else
      hipLaunchKernelGGL(k_swizzle_nodes<double>, grid, dim3(256), 0, s, Ji, pn, in.w, in.nx, in.Nn,
                         p->jsw + in.jsw_off);
  }
  return hipGetLastError();
}

template <int NX, typename T>
static void pinv_instance(birk_plan* p, const Instance& in, const double* Ji, int pn, const T* y, T* out,
                          T* jout, int* flag, hipStream_t s) {
  constexpr int S = NX * NX + NX;
  int64_t cnt[16];
  const int L = pinv_levels(in.Nn, cnt);
  // scratch: for each level l: agg[cnt[l] * S], then state[cnt[l] * NX]; level 0 swizzled
  const int64_t nb0 = pinv_blocks0(cnt[0]);
  double* base = p->scan + in.scan_off;
  double* agg[16];
  double* st[16];
  for (int l = 0; l <= L; ++l) {
    const int64_t slots = (l == 0) ? nb0 * 64 * kFan : cnt[l];
    agg[l] = base;
    base += slots * S;
    st[l] = base;
    base += slots * NX;
  }
  // per-node data in the plan's storage type (float copies for float products)
  const T* jsw = (const T*)p->jsw + in.jsw_off;
  const int64_t thr0 = nb0 * 64 * kFan;
  hipLaunchKernelGGL((k_pinv_up0<NX, T>), dim3(nblocks(thr0, 256)), dim3(256), 0, s, jsw, Ji, pn, in.Nn, y, cnt[0],
                     agg[0], flag);
  if (L == 0) {
    // a single group of at most kFan chunks: walk it from zero in one thread
    hipLaunchKernelGGL((k_pinv_top1<NX>), dim3(1), dim3(64), 0, s, agg[0], cnt[0], st[0]);
  } else {
    hipLaunchKernelGGL((k_pinv_up_sw<NX>), dim3(nblocks(cnt[1], 256)), dim3(256), 0, s, agg[0], cnt[0], agg[1],
                       cnt[1]);
    for (int l = 1; l < L; ++l)
      hipLaunchKernelGGL((k_pinv_up<NX>), dim3(nblocks(cnt[l + 1], 256)), dim3(256), 0, s, agg[l], cnt[l],
                         agg[l + 1], cnt[l + 1]);
    hipLaunchKernelGGL((k_pinv_top<NX>), dim3(1), dim3(64), 0, s, agg[L], cnt[L], st[L]);
    for (int l = L - 1; l >= 1; --l)
      hipLaunchKernelGGL((k_pinv_down<NX>), dim3(nblocks(cnt[l + 1], 256)), dim3(256), 0, s, agg[l], cnt[l],
                         st[l + 1], cnt[l + 1], st[l]);
    hipLaunchKernelGGL((k_pinv_down_sw<NX>), dim3(nblocks(cnt[1], 256)), dim3(256), 0, s, agg[0], cnt[0], st[1],
                       cnt[1], st[0]);
  }
  hipLaunchKernelGGL((k_pinv_final<NX, T>), dim3(nblocks(thr0, 256)), dim3(256), 0, s, jsw, Ji, pn, in.Nn, y,
                     cnt[0], st[0], out, jout);
}

// Scratch (doubles) the inverse scan needs for one instance (level 0 in whole blocks).
int64_t pinv_scratch(int64_t Nn, int nx) {
  const int64_t S = (int64_t)nx * nx + 2 * nx;
  int64_t cnt[16];
  const int L = pinv_levels(Nn, cnt);
  int64_t tot = pinv_blocks0(cnt[0]) * 64 * kFan * S;
  for (int l = 1; l <= L; ++l) tot += cnt[l] * S;
  return tot;
}

template <typename T>
hipError_t precond_inverse(birk_plan* p, int jac_kind, const double* J, const T* y, T* out, T* jout,
                           hipStream_t s, int* flag) {
  // the per-node data must have been swizzled for this J by precond_prepare
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const Instance& in : p->inst) {
    const double* Ji = J + (pn ? in.joff : in.jcoff);
    const T* yi = y + in.off;
    T* oi = out + in.off;
    T* ji = jout ? jout + in.off : nullptr;
    switch (in.nx) {
#define BIRK_PINV_CASE(n) \
  case n:                 \
    pinv_instance<n, T>(p, in, Ji, pn, yi, oi, ji, flag, s); \
    break;
      BIRK_PINV_CASE(1)
      BIRK_PINV_CASE(2)
      BIRK_PINV_CASE(3)
      BIRK_PINV_CASE(4)
      BIRK_PINV_CASE(5)
      BIRK_PINV_CASE(6)
      BIRK_PINV_CASE(7)
      BIRK_PINV_CASE(8)
      BIRK_PINV_CASE(9)
      BIRK_PINV_CASE(10)
      BIRK_PINV_CASE(11)
      BIRK_PINV_CASE(12)
#undef BIRK_PINV_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template hipError_t jac_times<double>(birk_plan*, int, const double*, const double*, double*, hipStream_t);
template hipError_t jac_times<float>(birk_plan*, int, const double*, const float*, float*, hipStream_t);
template hipError_t precond_forward<double>(birk_plan*, int, const double*, const double*, double*, hipStream_t);
template hipError_t precond_forward<float>(birk_plan*, int, const double*, const float*, float*, hipStream_t);
template hipError_t precond_inverse<double>(birk_plan*, int, const double*, const double*, double*, double*,
                                            hipStream_t, int*);
template hipError_t precond_inverse<float>(birk_plan*, int, const double*, const float*, float*, float*,
                                           hipStream_t, int*);

// ------------------------------------------------------------------ Krylov BLAS-1
// Dot products of u with up to kMaxDots basis vectors plus ||u||^2, accumulated in
// double.  part[block][nq + 1]; k_reduce_parts then sums blocks in a fixed order.
constexpr int kMaxDots = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_dots(const T* __restrict__ Q, int64_t ld, int nq,
                                              const T* __restrict__ u, int64_t n, double* __restrict__ part) {
  double acc[kMaxDots + 1];
#pragma unroll
  for (int i = 0; i <= kMaxDots; ++i) acc[i] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double ue = (double)u[e];
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nq) acc[i] += (double)Q[(int64_t)i * ld + e] * ue;
    acc[kMaxDots] += ue * ue;
  }
  __shared__ double sh[256];
#pragma unroll
  for (int i = 0; i <= kMaxDots; ++i) {
    if (i < nq || i == kMaxDots) {
      const double s = block_sum256(acc[i], sh);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + i] = s;
    }
  }
}

// One block per needed output (index blockIdx.x < nq, or the norm slot kMaxDots for the
// last block): strided partial sums, then a fixed-order tree; deterministic.
__global__ __launch_bounds__(256) void k_reduce_parts(const double* __restrict__ part, int nblk, int nq,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  const int i = (blockIdx.x < (unsigned)nq) ? (int)blockIdx.x : kMaxDots;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)b * (kMaxDots + 1) + i];
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) out[i] = t;
}

// u -= sum_i h[i] Q_i ; optionally part <- block sums of ||u||^2
template <typename T>
__global__ __launch_bounds__(256) void k_axpys(const T* __restrict__ Q, int64_t ld, int nq,
                                               const double* __restrict__ h, T* __restrict__ u, int64_t n,
                                               double* __restrict__ part) {
  __shared__ double hs[kMaxDots];
  if (threadIdx.x < kMaxDots) hs[threadIdx.x] = threadIdx.x < nq ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double nrm = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double ue = (double)u[e];
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nq) ue -= hs[i] * (double)Q[(int64_t)i * ld + e];
    const T us = (T)ue;
    u[e] = us;
    nrm += (double)us * (double)us;
  }
  if (part) {
    __shared__ double sh[256];
    const double s = block_sum256(nrm, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + kMaxDots] = s;
  }
}

// q = u / sqrt(nrm2[0])
template <typename T>
__global__ void k_normalize(const T* __restrict__ u, const double* __restrict__ nrm2, T* __restrict__ q,
                            int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double inv = 1.0 / sqrt(nrm2[0]);
  q[e] = (T)((double)u[e] * inv);
}

// y = alpha * x (type conversion allowed)
template <typename TI, typename TO>
__global__ void k_scale_conv(const TI* __restrict__ x, TO* __restrict__ y, double alpha, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  y[e] = (TO)(alpha * (double)x[e]);
}

// z = a - b  (FastAX step 3)
template <typename T>
__global__ void k_sub(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ z, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  z[e] = a[e] - b[e];
}

// r = beta - (x - t) = beta - x + t, in double
__global__ void k_residual(const double* __restrict__ beta, const double* __restrict__ x,
                           const double* __restrict__ t, double* __restrict__ r, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  r[e] = beta[e] - x[e] + t[e];
}

// x += (double) d
template <typename T>
__global__ void k_add_to(double* __restrict__ x, const T* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  x[e] += (double)d[e];
}

// u = sum_i c_i Q_i with c on the host side passed through a small device array
template <typename T>
__global__ __launch_bounds__(256) void k_combine(const T* __restrict__ Q, int64_t ld, int nq,
                                                 const double* __restrict__ c, T* __restrict__ u, int64_t n) {
  __shared__ double cs[kMaxDots];
  if (threadIdx.x < kMaxDots) cs[threadIdx.x] = threadIdx.x < nq ? c[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nq) acc += cs[i] * (double)Q[(int64_t)i * ld + e];
    u[e] = (T)acc;
  }
}

// Host-side launch helpers used by the GMRES driver.
namespace kry {

static inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

template <typename T>
void dots(const T* Q, int64_t ld, int nq, const T* u, int64_t n, double* part, double* out, hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_dots<T>, dim3(g), dim3(256), 0, s, Q, ld, nq, u, n, part);
  hipLaunchKernelGGL(k_reduce_parts, dim3(nq + 1), dim3(256), 0, s, part, (int)g, nq, out);
}

template <typename T>
void axpys(const T* Q, int64_t ld, int nq, const double* h, T* u, int64_t n, double* part, double* nrm_out,
           hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_axpys<T>, dim3(g), dim3(256), 0, s, Q, ld, nq, h, u, n, part);
  if (part) hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, part, (int)g, 0, nrm_out);
}

template <typename T>
void normalize(const T* u, const double* nrm2, T* q, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, u, nrm2, q, n);
}

template <typename TI, typename TO>
void scale_conv(const TI* x, TO* y, double alpha, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_scale_conv<TI, TO>), dim3(nblocks(n, 256)), dim3(256), 0, s, x, y, alpha, n);
}

template <typename T>
void sub(const T* a, const T* b, T* z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, a, b, z, n);
}

void residual(const double* beta, const double* x, const double* t, double* r, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, s, beta, x, t, r, n);
}

template <typename T>
void add_to(double* x, const T* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_to<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, x, d, n);
}

template <typename T>
void combine(const T* Q, int64_t ld, int nq, const double* c, T* u, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_combine<T>, dim3(grid_for(n)), dim3(256), 0, s, Q, ld, nq, c, u, n);
}

template void dots<double>(const double*, int64_t, int, const double*, int64_t, double*, double*, hipStream_t);
template void dots<float>(const float*, int64_t, int, const float*, int64_t, double*, double*, hipStream_t);
template void axpys<double>(const double*, int64_t, int, const double*, double*, int64_t, double*, double*,
                            hipStream_t);
template void axpys<float>(const float*, int64_t, int, const double*, float*, int64_t, double*, double*,
                           hipStream_t);
template void normalize<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void normalize<float>(const float*, const double*, float*, int64_t, hipStream_t);
template void scale_conv<double, double>(const double*, double*, double, int64_t, hipStream_t);
template void scale_conv<double, float>(const double*, float*, double, int64_t, hipStream_t);
template void scale_conv<float, double>(const float*, double*, double, int64_t, hipStream_t);
template void scale_conv<float, float>(const float*, float*, double, int64_t, hipStream_t);
template void sub<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void sub<float>(const float*, const float*, float*, int64_t, hipStream_t);
template void add_to<double>(double*, const double*, int64_t, hipStream_t);
template void add_to<float>(double*, const float*, int64_t, hipStream_t);
template void combine<double>(const double*, int64_t, int, const double*, double*, int64_t, hipStream_t);
template void combine<float>(const float*, int64_t, int, const double*, float*, int64_t, hipStream_t);

}  // namespace kry
}  // namespace birk
