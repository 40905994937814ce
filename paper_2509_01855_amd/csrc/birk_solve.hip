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
//             evaluated as a scan of affine maps S_out = A S_in + b.  n_x <= 8: each
//             thread holds whole maps; a DPP scan across waves, tile aggregates and
//             tile start states (three launches), each node's K_k formed from J and
//             w_k and factored where it is used.  Larger n_x: chunks of kChunk nodes
//             worked by sixteen-lane groups, groups of kFan aggregates per level up to a
//             sequential top, start states pushed back down.  Either way each chunk is
//             replayed from its start state, emitting xi_k and J_k xi_k (the latter
//             feeds FastAX).  All arithmetic in double; y, xi and J xi are stored in the
//             plan type.

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "birk_internal.h"

namespace birk {

constexpr int kChunk = 16;
constexpr int kFan = 16;

// Lane P of each row of sixteen lanes, broadcast across its row (DPP row_newbcast: a VALU
// move, in place of an LDS permute), for a double.
template <int P>
__device__ __forceinline__ double row_bcast(double v) {
  const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)x, (int)(unsigned)x, 0x150 + P, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(x >> 32), (int)(unsigned)(x >> 32), 0x150 + P, 0xF, 0xF,
                                             false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// f(std::integral_constant<int, P>) for P = B .. E - 1, in order (compile-time lane indices).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
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

// P y = y - B~^a (J y) per component r: an exclusive prefix sum of u_k = w_k (J_k y_k)_r
// plus half the node's own term (B~^a: w_j below the diagonal, w_k / 2 on it).  Three
// launches: block sums over tiles of kScanBlock nodes, an exclusive scan of the block sums
// (one workgroup per component), and the final pass, which scans inside the tile.  Global
// accesses are coalesced (node k = tile base + i * 256 + thread); the final pass moves u
// through LDS to scan it in node order.  Double plans with n_x <= 16 form u once for all
// components (k_pfwd_sums_all, u kept in out); otherwise each component's passes rebuild
// their u_r from J and y.

// One workgroup per tile of kScanBlock nodes of one component of one instance, over the
// whole batch: tile = (instance, component * ntiles + tile index); the tile sums of
// (instance i, component r) sit at scan[scan_off(i) + r * ntiles(i) + tile].
__device__ __forceinline__ int pfwd_ntiles(int64_t Nn) { return (int)((Nn + kScanBlock - 1) / kScanBlock); }

template <typename T>
__global__ __launch_bounds__(256) void k_pfwd_sums(const int2* __restrict__ tiles, const InstDesc* __restrict__ idesc,
                                                   const double* __restrict__ J, int per_node,
                                                   const T* __restrict__ y, double* __restrict__ scan) {
  __shared__ double sh[256];
  const int2 t = tiles[blockIdx.x];
  const InstDesc d = idesc[t.x];
  const int nt = pfwd_ntiles(d.Nn);
  const int r = t.y / nt, b = t.y - r * nt;
  const double* Ji = J + (per_node ? d.joff : d.jcoff);
  const T* yi = y + d.off;
  const int64_t base = (int64_t)b * kScanBlock;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    if (k < d.Nn) acc += wju<T>(Ji, per_node, yi, d.w, r, (int)d.nx, d.Nn, k);
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) scan[d.scan_off + t.y] = s;
}

// Inclusive scan of v over the 256 threads of the workgroup (Hillis-Steele in LDS).
__device__ __forceinline__ double block_scan256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = 1; st < 256; st <<= 1) {
    const double a = threadIdx.x >= st ? sh[threadIdx.x - st] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += a;
    __syncthreads();
  }
  const double r = sh[threadIdx.x];
  __syncthreads();
  return r;
}

// Exclusive scan of the tile sums of one (instance, component) per workgroup, in chunks
// of 256.
__global__ __launch_bounds__(256) void k_pfwd_scanparts(const int2* __restrict__ pairs,
                                                        const InstDesc* __restrict__ idesc,
                                                        double* __restrict__ scan) {
  __shared__ double sh[256];
  __shared__ double total;
  const int2 q = pairs[blockIdx.x];
  const InstDesc d = idesc[q.x];
  const int nblk = pfwd_ntiles(d.Nn);
  double* pr = scan + d.scan_off + (int64_t)q.y * nblk;
  double carry = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 256) {
    const int b = b0 + (int)threadIdx.x;
    const double v = b < nblk ? pr[b] : 0.0;
    const double incl = block_scan256(v, sh);
    if (b < nblk) pr[b] = carry + incl - v;
    if (threadIdx.x == 255) total = incl;
    __syncthreads();
    carry += total;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pfwd_final(const int2* __restrict__ tiles, const InstDesc* __restrict__ idesc,
                                                    const double* __restrict__ J, int per_node,
                                                    const T* __restrict__ y, const double* __restrict__ scan,
                                                    T* __restrict__ out) {
  __shared__ double su[kScanBlock];
  __shared__ double sh[256];
  const int2 t = tiles[blockIdx.x];
  const InstDesc d = idesc[t.x];
  const int nt = pfwd_ntiles(d.Nn);
  const int r = t.y / nt, b = t.y - r * nt;
  const double* Ji = J + (per_node ? d.joff : d.jcoff);
  const T* yi = y + d.off;
  const int64_t base = (int64_t)b * kScanBlock;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    su[i * 256 + threadIdx.x] = (k < d.Nn) ? wju<T>(Ji, per_node, yi, d.w, r, (int)d.nx, d.Nn, k) : 0.0;
  }
  __syncthreads();
  // thread t scans nodes base + kScanItems t + j, j < kScanItems, in order
  double u[kScanItems];
  double tsum = 0.0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    u[j] = su[threadIdx.x * kScanItems + j];
    tsum += u[j];
  }
  double run = scan[d.scan_off + t.y] + block_scan256(tsum, sh) - tsum;
  // each thread rewrites only the entries it read itself
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    su[threadIdx.x * kScanItems + j] = run + 0.5 * u[j];
    run += u[j];
  }
  __syncthreads();
  T* oi = out + d.off + (int64_t)r * d.Nn;
  const T* yr = yi + (int64_t)r * d.Nn;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    if (k < d.Nn) oi[k] = (T)((double)yr[k] - su[i * 256 + threadIdx.x]);
  }
}

// Double plans with n_x <= 16: one workgroup per tile forms u_k = w_k J_k y_k for all
// components (J and y read once), stores u in out (which does not overlap y) and sums it
// per component; the final pass of component r then reads u_r back instead of J and all
// of y.  Tile = (instance, tile); the sums go where k_pfwd_sums puts them.  NXC > 0: every
// instance has n_x = NXC, so the loops unroll completely and a node's J and y loads issue
// together.
template <int MAXNX, int NXC = 0>
__global__ __launch_bounds__(256) void k_pfwd_sums_all(const int2* __restrict__ tiles,
                                                       const InstDesc* __restrict__ idesc,
                                                       const double* __restrict__ J, int per_node,
                                                       const double* __restrict__ y, double* __restrict__ u,
                                                       double* __restrict__ scan) {
  __shared__ double sh[4][MAXNX];
  const int2 t = tiles[blockIdx.x];
  const InstDesc d = idesc[t.x];
  const int nt = pfwd_ntiles(d.Nn), b = t.y, nx = NXC > 0 ? NXC : (int)d.nx;
  const int64_t Nn = d.Nn;
  const double* Ji = J + (per_node ? d.joff : d.jcoff);
  const double* yi = y + d.off;
  double* ui = u + d.off;
  const int64_t base = (int64_t)b * kScanBlock;
  double acc[MAXNX];
#pragma unroll
  for (int r = 0; r < MAXNX; ++r) acc[r] = 0.0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    if (k >= Nn) break;
    double yv[MAXNX];
#pragma unroll
    for (int c = 0; c < MAXNX; ++c) yv[c] = c < nx ? yi[(int64_t)c * Nn + k] : 0.0;
    const double wk = d.w[k];
#pragma unroll
    for (int r = 0; r < MAXNX; ++r) {
      if (r >= nx) break;
      double a = 0.0;
#pragma unroll
      for (int c = 0; c < MAXNX; ++c) {
        if (c >= nx) break;
        a += (per_node ? Ji[(int64_t)(r * nx + c) * Nn + k] : Ji[r * nx + c]) * yv[c];
      }
      a *= wk;
      ui[(int64_t)r * Nn + k] = a;
      acc[r] += a;
    }
  }
  const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
#pragma unroll
  for (int r = 0; r < MAXNX; ++r) {
    if (r >= nx) break;
    double v = acc[r];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (l == 0) sh[w][r] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nx) {
    const int r = (int)threadIdx.x;
    scan[d.scan_off + (int64_t)r * nt + b] = ((sh[0][r] + sh[1][r]) + sh[2][r]) + sh[3][r];
  }
}

// Final pass of component r from u_r held in out (in place: a workgroup reads its tile of
// u_r before it writes the same elements of out).
__global__ __launch_bounds__(256) void k_pfwd_final_u(const int2* __restrict__ tiles, const InstDesc* __restrict__ idesc,
                                                      const double* __restrict__ y, const double* __restrict__ scan,
                                                      double* __restrict__ out) {
  __shared__ double su[kScanBlock];
  __shared__ double sh[256];
  const int2 t = tiles[blockIdx.x];
  const InstDesc d = idesc[t.x];
  const int nt = pfwd_ntiles(d.Nn);
  const int r = t.y / nt, b = t.y - r * nt;
  const int64_t base = (int64_t)b * kScanBlock;
  double* oi = out + d.off + (int64_t)r * d.Nn;
  const double* yr = y + d.off + (int64_t)r * d.Nn;
  double yv[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    su[i * 256 + threadIdx.x] = (k < d.Nn) ? oi[k] : 0.0;
    yv[i] = (k < d.Nn) ? yr[k] : 0.0;
  }
  __syncthreads();
  // thread t scans nodes base + kScanItems t + j, j < kScanItems, in order
  double uu[kScanItems];
  double tsum = 0.0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    uu[j] = su[threadIdx.x * kScanItems + j];
    tsum += uu[j];
  }
  double run = scan[d.scan_off + t.y] + block_scan256(tsum, sh) - tsum;
  // each thread rewrites only the entries it read itself
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    su[threadIdx.x * kScanItems + j] = run + 0.5 * uu[j];
    run += uu[j];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i * 256 + threadIdx.x;
    if (k < d.Nn) oi[k] = yv[i] - su[i * 256 + threadIdx.x];
  }
}

template <typename T>
hipError_t precond_forward(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           hipStream_t s) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  if constexpr (std::is_same<T, double>::value) {
    if (p->pfwd_maxnx <= 16) {
      static constexpr decltype(&k_pfwd_sums_all<8>) kUniform[9] = {
          nullptr,
          k_pfwd_sums_all<1, 1>,
          k_pfwd_sums_all<2, 2>,
          k_pfwd_sums_all<3, 3>,
          k_pfwd_sums_all<4, 4>,
          k_pfwd_sums_all<5, 5>,
          k_pfwd_sums_all<6, 6>,
          k_pfwd_sums_all<7, 7>,
          k_pfwd_sums_all<8, 8>};
      auto f = (p->pfwd_unx >= 1 && p->pfwd_unx <= 8) ? kUniform[p->pfwd_unx]
               : p->pfwd_maxnx <= 4                   ? k_pfwd_sums_all<4>
               : p->pfwd_maxnx <= 8                   ? k_pfwd_sums_all<8>
                                                      : k_pfwd_sums_all<16>;
      hipLaunchKernelGGL(f, dim3(p->pfwd_nbtiles), dim3(256), 0, s, p->pfwd_btiles, p->idesc, J, pn, y, out, p->scan);
      hipLaunchKernelGGL(k_pfwd_scanparts, dim3(p->pfwd_npairs), dim3(256), 0, s, p->pfwd_pairs, p->idesc, p->scan);
      hipLaunchKernelGGL(k_pfwd_final_u, dim3(p->pfwd_ntiles), dim3(256), 0, s, p->pfwd_tiles, p->idesc, y,
                         (const double*)p->scan, out);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL(k_pfwd_sums<T>, dim3(p->pfwd_ntiles), dim3(256), 0, s, p->pfwd_tiles, p->idesc, J, pn, y,
                     p->scan);
  hipLaunchKernelGGL(k_pfwd_scanparts, dim3(p->pfwd_npairs), dim3(256), 0, s, p->pfwd_pairs, p->idesc, p->scan);
  hipLaunchKernelGGL(k_pfwd_final<T>, dim3(p->pfwd_ntiles), dim3(256), 0, s, p->pfwd_tiles, p->idesc, J, pn, y,
                     (const double*)p->scan, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ P^{-1} y (inverse)

// 1 / x from the hardware estimate and two Newton steps (within an ulp of the quotient;
// several times cheaper than a division).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

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
    rp[p] = recip(piv);
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

// ---- hierarchical path (n_x > kWaveNx): level-0 layout ----
// Chunks of kChunk consecutive nodes are the level-0 slots (each worked by a group of
// sixteen lanes).  Chunk c is child i = c % kFan of level-1 group g = c / kFan.  Slot
// indices tau are laid out so that the
// 64 slots of a block of 64 hold 64 consecutive groups g and the index of that block
// within kFan of them is the child index i:  slot tau -> block B = tau / (64 kFan),
// i = (tau / 64) % kFan, lane l = tau % 64, g = 64 B + l, c = kFan g + i.
// Every per-chunk array (swizzled Jacobians, aggregates, start states) is stored as
// [B][i][field][l]: neighbouring slots hold neighbouring values of a field.
//
// Batching: the instances of one n_x form a PinvClass; every phase below is one launch
// over all of them, each block reading its instance from a (k, block) tile and the
// instance's sizes and scratch offsets from a PinvDesc.
__device__ __forceinline__ int64_t swz(int64_t B, int i, int field, int nfield, int l) {
  return (((B * kFan + i) * nfield) + field) * 64 + l;
}

// Per-node tables of the level-0 kernels: node k -> chunk c = k / kChunk, j = k % kChunk;
// g = c / kFan, i = c % kFan; B = g / 64, l = g % 64; slot sigma = (B kFan + i) 64 + l.
// Node j of slot sigma keeps row-major H_k (NX^2 values) then w_k in a record of
// hrec<NX>() values (a multiple of four, so that the rows start 16-byte aligned for
// doubles with NX even and for floats with NX a multiple of four) at
// jsw[(sigma kChunk + j) hrec].  A lane holding row r of a chunk's state reads the NX
// contiguous values of row r of H_k; the sixteen lanes of a chunk read one record.
template <int NX>
__host__ __device__ constexpr int hrec() { return (NX * NX + 1 + 3) & ~3; }

// Row r of H_k (NX values at p) into registers; 16-byte loads where every row is 16-byte
// aligned (records are multiples of four values).
template <int NX, typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ p, double (&h)[NX]) {
  if constexpr (sizeof(T) == 8 && (NX % 2) == 0) {
    typedef double v2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int q = 0; q < NX; q += 2) {
      const v2 v = *reinterpret_cast<const v2*>(p + q);
      h[q] = v.x;
      h[q + 1] = v.y;
    }
  } else if constexpr (sizeof(T) == 4 && (NX % 4) == 0) {
    typedef float v4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < NX; q += 4) {
      const v4 v = *reinterpret_cast<const v4*>(p + q);
      h[q] = v.x;
      h[q + 1] = v.y;
      h[q + 2] = v.z;
      h[q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NX; ++q) h[q] = (double)p[q];
  }
}

// Per node, H_k = w_k J_k K_k^{-1} with K_k = I - w_k J_k / 2 (J_k commutes with K_k^{-1}).
// Everything the scan needs follows from H_k:  K_k^{-1} = I + H_k / 2, so for
// u = y_k + S_k
//     xi_k = u + H_k u / 2,   J_k xi_k = H_k u / w_k,   S_{k+1} = S_k + H_k u,
// and the affine map of the node is S -> (I + H_k) S + H_k y_k.  H_k and w_k go to the
// node's record (J, per node or constant, and w are read where they are).
// Sixteen lanes per chunk: lane r < NX holds row r of [K_k | w_k J_k] and Gauss-Jordan
// elimination without pivoting, the pivot row broadcast across the sixteen lanes, turns
// it into [I | K_k^{-1} w_k J_k]; its pivots are those of the unpivoted LU, and one that
// is non-finite or not above 1e-13 (1 + |w_k / 2| max |J_k|) sets *flag.  A chunk's 16
// nodes are taken in turn; the four chunks of a wave are neighbours in the slot layout.
// grid = (tile (k, block of 256 level-0 threads), 16 groups of 16 chunks).
template <int NX, typename JT>
__global__ __launch_bounds__(256) void k_make_h_rows(JT* __restrict__ jsw, const double* __restrict__ J,
                                                    int per_node, const PinvDesc* __restrict__ pd,
                                                    const int2* __restrict__ tiles, int* flag) {
  static_assert(NX <= 16, "one row per lane of a 16-lane group");
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t tau = (int64_t)t.y * 256 + blockIdx.y * 16 + (threadIdx.x >> 4);
  const int r = (int)(threadIdx.x & 15);
  const int64_t B = tau / (64 * kFan);
  const int i = (int)((tau >> 6) % kFan);
  const int l = (int)(tau & 63);
  const int64_t c = (B * 64 + l) * kFan + i;
  if (c >= d.cnt[0]) return;  // the whole group leaves together
  constexpr int E = hrec<NX>();
  const double* Jc = J + d.jcoff;
  const double* Jn = J + d.joff;
  JT* js = jsw + d.jsw_off + (((B * kFan + i) * 64 + l) * kChunk) * E;
  const int jn = (int)min((int64_t)kChunk, d.Nn - c * kChunk);
  const bool act = r < NX;
  const int rr = act ? r : 0;
#pragma unroll 1
  for (int j = 0; j < jn; ++j) {
    JT* base = js + (int64_t)j * E;
    const int64_t k = c * kChunk + j;
    const double wk = d.w[k];
    double Kr[NX], Xr[NX];
    double jm = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const double jv = act ? (per_node ? Jn[(int64_t)(rr * NX + q) * d.Nn + k] : Jc[rr * NX + q]) : 0.0;
      jm = fmax(jm, fabs(jv));
      Xr[q] = wk * jv;
      Kr[q] = (r == q ? 1.0 : 0.0) - 0.5 * wk * jv;
    }
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) jm = fmax(jm, __shfl_xor(jm, o, 16));
    const double scale = 1.0 + 0.5 * fabs(wk) * jm;
    static_for<0, NX>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      double pk[NX], px[NX];
#pragma unroll
      for (int q = p; q < NX; ++q) pk[q] = row_bcast<p>(Kr[q]);
#pragma unroll
      for (int q = 0; q < NX; ++q) px[q] = row_bcast<p>(Xr[q]);
      const double piv = pk[p];
      if (r == 0 && flag && (!(fabs(piv) > 1e-13 * scale) || !isfinite(piv))) atomicOr(flag, 1);
      const double rp = recip(piv);
      if (r == p) {
#pragma unroll
        for (int q = p + 1; q < NX; ++q) Kr[q] *= rp;
#pragma unroll
        for (int q = 0; q < NX; ++q) Xr[q] *= rp;
      } else {
        const double f = Kr[p] * rp;
#pragma unroll
        for (int q = p + 1; q < NX; ++q) Kr[q] -= f * pk[q];
#pragma unroll
        for (int q = 0; q < NX; ++q) Xr[q] -= f * px[q];
      }
    });
    if (act) {
#pragma unroll
      for (int q = 0; q < NX; ++q) base[r * NX + q] = (JT)Xr[q];
    }
    if (r == 0) base[NX * NX] = (JT)wk;
  }
}

// Level-0 up-sweep: each chunk of kChunk nodes is reduced to (A, b) with
// S_out = A S_in + b by the node maps S -> (I + H_k) S + H_k y_k, sixteen lanes per chunk
// with lane r < NX holding row r of A and b: from A = I, b = 0 each node takes
//     A <- A + H_k A,   b <- b + H_k (b + y_k),
// row r of H_k read contiguously from the node's record and the rows of A and of
// b + y_k broadcast across the sixteen lanes (DPP row_newbcast).
// grid = (tile (k, block of 256 level-0 threads), 16 groups of 16 chunks).
template <int NX, typename T>
__global__ __launch_bounds__(256) void k_pinv_up0(const T* __restrict__ jsw, const T* __restrict__ y,
                                                  const PinvDesc* __restrict__ pd, const int2* __restrict__ tiles,
                                                  double* __restrict__ scan) {
  static_assert(NX <= 16, "one row per lane of a 16-lane group");
  constexpr int E = hrec<NX>();
  constexpr int F = NX * NX + NX;
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t tau = (int64_t)t.y * 256 + blockIdx.y * 16 + (threadIdx.x >> 4);
  const int r = (int)(threadIdx.x & 15);
  const int64_t B = tau / (64 * kFan);
  const int i = (int)((tau >> 6) % kFan);
  const int l = (int)(tau & 63);
  const int64_t ch = (B * 64 + l) * kFan + i;
  if (ch >= d.cnt[0]) return;  // the whole group leaves together
  const bool act = r < NX;
  const int rr = act ? r : 0;
  const int64_t Nn = d.Nn;
  const T* hs = jsw + d.jsw_off + (((B * kFan + i) * 64 + l) * kChunk) * E + rr * NX;
  const T* yi = y + d.off + (int64_t)rr * Nn;
  double a[NX], b = 0.0;
#pragma unroll
  for (int c = 0; c < NX; ++c) a[c] = (act && c == r) ? 1.0 : 0.0;
  const int64_t k0 = ch * kChunk;
  const int jn = (int)min((int64_t)kChunk, Nn - k0);
  double yv[kChunk];  // the chunk's run of y for component r, loaded together
#pragma unroll
  for (int j = 0; j < kChunk; ++j) yv[j] = (act && j < jn) ? (double)yi[k0 + j] : 0.0;
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    if (j >= jn) break;
    double h[NX];
    load_row<NX, T>(hs + (int64_t)j * E, h);  // lanes r >= NX read row 0 (in bounds), unused
    const double u = b + yv[j];
    double na[NX], nb = b;
#pragma unroll
    for (int c = 0; c < NX; ++c) na[c] = a[c];
    static_for<0, NX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      nb += h[q] * row_bcast<q>(u);
#pragma unroll
      for (int c = 0; c < NX; ++c) na[c] += h[q] * row_bcast<q>(a[c]);
    });
#pragma unroll
    for (int c = 0; c < NX; ++c) a[c] = na[c];
    b = nb;
  }
  if (act) {
    double* agg = scan + d.agg[0];
#pragma unroll
    for (int c = 0; c < NX; ++c) agg[swz(B, i, r * NX + c, F, l)] = a[c];
    agg[swz(B, i, NX * NX + r, F, l)] = b;
  }
}

// (A, b) <- (a_A A, a_A b + a_b) for the NX x NX + NX fields of aggregate a (field f at
// a[f * fs]).
template <int NX>
__device__ __forceinline__ void compose(const double* __restrict__ a, int64_t fs, double (&A)[NX][NX],
                                        double (&b)[NX]) {
  double nb[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    double acc = a[(NX * NX + r) * fs];
#pragma unroll
    for (int q = 0; q < NX; ++q) acc += a[(r * NX + q) * fs] * b[q];
    nb[r] = acc;
  }
#pragma unroll
  for (int col = 0; col < NX; ++col) {
    double ncol[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += a[(r * NX + q) * fs] * A[q][col];
      ncol[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) A[r][col] = ncol[r];
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) b[r] = nb[r];
}

// s <- a_A s + a_b
template <int NX>
__device__ __forceinline__ void advance(const double* __restrict__ a, int64_t fs, double (&s)[NX]) {
  double ns[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    double acc = a[(NX * NX + r) * fs];
#pragma unroll
    for (int q = 0; q < NX; ++q) acc += a[(r * NX + q) * fs] * s[q];
    ns[r] = acc;
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = ns[r];
}

// Upper levels of the hierarchical scan, sixteen lanes per parent (lane r < NX holds row
// r of a map or component r of a state; rows and states broadcast with DPP row_newbcast).
// Child aggregate i of parent g: level 0 in the slot layout (field f at stride 64), upper
// levels plain (F consecutive fields).  grid = (tile (k, block of 256 parents), 16 groups
// of 16 parents).
template <int NX>
__device__ __forceinline__ const double* child_agg(const double* __restrict__ child, int lv, int64_t g, int i,
                                                   int64_t& fs) {
  constexpr int F = NX * NX + NX;
  if (lv == 0) {
    fs = 64;
    return child + swz(g >> 6, i, 0, F, (int)(g & 63));
  }
  fs = 1;
  return child + (g * kFan + i) * F;
}

// Up-sweep level lv -> lv + 1: each parent composes its kFan child aggregates in order,
// (A, b) <- (a_A A, a_A b + a_b).
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_up(double* __restrict__ scan, const PinvDesc* __restrict__ pd,
                                                 const int2* __restrict__ tiles, int lv) {
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t g = (int64_t)t.y * 256 + blockIdx.y * 16 + (threadIdx.x >> 4);
  if (g >= d.cnt[lv + 1]) return;  // the whole group leaves together
  const int r = (int)(threadIdx.x & 15);
  const bool act = r < NX;
  const int rr = act ? r : 0;
  constexpr int F = NX * NX + NX;
  const double* child = scan + d.agg[lv];
  double a[NX], b = 0.0;
#pragma unroll
  for (int c = 0; c < NX; ++c) a[c] = (act && c == r) ? 1.0 : 0.0;
  const int nc = (int)min((int64_t)kFan, d.cnt[lv] - g * kFan);
#pragma unroll 1
  for (int i = 0; i < nc; ++i) {
    int64_t fs;
    const double* ca = child_agg<NX>(child, lv, g, i, fs);
    double row[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) row[q] = ca[(rr * NX + q) * fs];
    double na[NX], nb = ca[(NX * NX + rr) * fs];
#pragma unroll
    for (int c = 0; c < NX; ++c) na[c] = 0.0;
    static_for<0, NX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      nb += row[q] * row_bcast<q>(b);
#pragma unroll
      for (int c = 0; c < NX; ++c) na[c] += row[q] * row_bcast<q>(a[c]);
    });
#pragma unroll
    for (int c = 0; c < NX; ++c) a[c] = na[c];
    b = nb;
  }
  if (act) {
    double* o = scan + d.agg[lv + 1] + g * F;
#pragma unroll
    for (int c = 0; c < NX; ++c) o[r * NX + c] = a[c];
    o[NX * NX + r] = b;
  }
}

// Top: sixteen lanes per instance (one workgroup of 64 threads, the first row working)
// walk the top-level aggregates from S = 0 and write their start states (level 0 in the
// slot layout when the instance has a single group).
template <int NX>
__global__ void k_pinv_top(double* __restrict__ scan, const PinvDesc* __restrict__ pd) {
  if (threadIdx.x >= 16) return;
  const int r = (int)threadIdx.x;
  const bool act = r < NX;
  const int rr = act ? r : 0;
  const PinvDesc& d = pd[blockIdx.x];
  constexpr int F = NX * NX + NX;
  const int L = d.L;
  const double* agg = scan + d.agg[L];
  double* state = scan + d.st[L];
  double s = 0.0;
  for (int64_t i = 0; i < d.cnt[L]; ++i) {
    const double* ca = (L == 0) ? agg + swz(0, (int)i, 0, F, 0) : agg + i * F;
    const int64_t fs = (L == 0) ? 64 : 1;
    if (act) {
      if (L == 0) state[swz(0, (int)i, r, NX, 0)] = s;
      else state[i * NX + r] = s;
    }
    double ns = ca[(NX * NX + rr) * fs];
    static_for<0, NX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      ns += ca[(rr * NX + q) * fs] * row_bcast<q>(s);
    });
    s = ns;
  }
}

// Down-sweep level lv + 1 -> lv: each parent pushes its start state through its children
// (level 0 written in the slot layout).
template <int NX>
__global__ __launch_bounds__(256) void k_pinv_down(double* __restrict__ scan, const PinvDesc* __restrict__ pd,
                                                   const int2* __restrict__ tiles, int lv) {
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t g = (int64_t)t.y * 256 + blockIdx.y * 16 + (threadIdx.x >> 4);
  if (g >= d.cnt[lv + 1]) return;  // the whole group leaves together
  const int r = (int)(threadIdx.x & 15);
  const bool act = r < NX;
  const int rr = act ? r : 0;
  const double* child = scan + d.agg[lv];
  double* cstate = scan + d.st[lv];
  double s = act ? scan[d.st[lv + 1] + g * NX + r] : 0.0;
  const int nc = (int)min((int64_t)kFan, d.cnt[lv] - g * kFan);
#pragma unroll 1
  for (int i = 0; i < nc; ++i) {
    if (act) {
      if (lv == 0) cstate[swz(g >> 6, i, r, NX, (int)(g & 63))] = s;
      else cstate[(g * kFan + i) * NX + r] = s;
    }
    int64_t fs;
    const double* ca = child_agg<NX>(child, lv, g, i, fs);
    double row[NX];
#pragma unroll
    for (int q = 0; q < NX; ++q) row[q] = ca[(rr * NX + q) * fs];
    double ns = ca[(NX * NX + rr) * fs];
    static_for<0, NX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      ns += row[q] * row_bcast<q>(s);
    });
    s = ns;
  }
}

// ---- wave-scan path (n_x <= kWaveNx) ----
// A tile is kTileThreads threads of kTC consecutive nodes each: thread t of tile g owns
// chunk c = g kTileThreads + t, nodes k = c kTC + j (j < kTC), so the lanes of a wave
// hold consecutive chunks in node order.  Per-node fields (the n_x^2 entries of H_k, then
// w_k) are stored as [g][j][e][t]: each access of a wave is 64 consecutive values.
// Three launches per class:
//   reduce  each thread composes its chunk's node maps; a DPP scan across the wave and a
//           4-lane scan of the wave totals give every chunk the map from the start of its
//           tile through its last node (stored), the last of them the tile aggregate;
//   tiles   one workgroup per instance scans the tile aggregates into tile start states;
//   apply   each chunk advances its tile's start state by the stored map of the chunk
//           before it and replays its nodes (no scan, few registers).
// Nodes past N_n carry H = 0 (identity maps) and are neither read from y nor written.
constexpr int kWaveNx = 8;
constexpr int kTileThreads = 256;
constexpr int kTC = 4;
constexpr int64_t kTileNodes = (int64_t)kTileThreads * kTC;
// Where the scan kernels take K_k from: formed from one J per instance (uniform), formed
// from per-node J staged through LDS, or H_k = w_k J_k K_k^{-1} laid out once per J by
// precond_prepare (k_tmake_h) and read coalesced, for solves that apply P^{-1} repeatedly.
constexpr int kFlyConst = 0, kFlyPerNode = 1, kCachedH = 2;

template <int NX>
struct Aff {
  double A[NX][NX];
  double b[NX];
};

template <int NX>
__device__ __forceinline__ void aff_identity(Aff<NX>& m) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    m.b[r] = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) m.A[r][q] = (r == q) ? 1.0 : 0.0;
  }
}

// s <- m(s) = A s + b
template <int NX>
__device__ __forceinline__ void aff_apply(const Aff<NX>& m, double (&s)[NX]) {
  double ns[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    double acc = m.b[r];
#pragma unroll
    for (int q = 0; q < NX; ++q) acc += m.A[r][q] * s[q];
    ns[r] = acc;
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = ns[r];
}

// v of the lane that DPP control CTRL selects, in the rows that ROWMASK enables
// (row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143); a lane with no
// source keeps its own v.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
  const int lo = (int)(unsigned)x, hi = (int)(unsigned)(x >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)rhi << 32) | (unsigned)(unsigned)rlo);
}

// Where take: m <- m o e, e = the map of the source lane (applied first):
// (A_m A_e, A_m b_e + b_m).  e arrives one row at a time.
template <int NX, int CTRL, int ROWMASK>
__device__ __forceinline__ void scan_step(Aff<NX>& m, bool take) {
  double nA[NX][NX], nb[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    nb[r] = m.b[r];
#pragma unroll
    for (int c = 0; c < NX; ++c) nA[r][c] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < NX; ++q) {
    double er[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) er[c] = dpp_f64<CTRL, ROWMASK>(m.A[q][c]);
    const double eb = dpp_f64<CTRL, ROWMASK>(m.b[q]);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      const double a = m.A[r][q];
#pragma unroll
      for (int c = 0; c < NX; ++c) nA[r][c] += a * er[c];
      nb[r] += a * eb;
    }
  }
  if (take) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      m.b[r] = nb[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) m.A[r][c] = nA[r][c];
    }
  }
}

// Inclusive scan of the lanes' maps in lane order: lane l ends with m_l o ... o m_0.
// Rows of 16 lanes scan by row_shr 1, 2, 4, 8; row_bcast:15 then row_bcast:31 carry the
// totals of the earlier rows.
template <int NX>
__device__ __forceinline__ void wave_scan(Aff<NX>& m) {
  const int l = (int)(threadIdx.x & 63), lr = l & 15;
  scan_step<NX, 0x111, 0xF>(m, lr >= 1);
  scan_step<NX, 0x112, 0xF>(m, lr >= 2);
  scan_step<NX, 0x114, 0xF>(m, lr >= 4);
  scan_step<NX, 0x118, 0xF>(m, lr >= 8);
  scan_step<NX, 0x142, 0xA>(m, ((l >> 4) & 1) != 0);
  scan_step<NX, 0x143, 0xC>(m, l >= 32);
}

// K_k = I - (w_k / 2) J_k of node k, factored in place by lu_kmat (pivot check into *flag
// when flag is set); entry (r, q) of J_k at Jp[(r NX + q) js] (per node in global memory:
// Jp = J + k, js = N_n; staged in LDS: js = 64; one J for the instance: js = 1).  With u
// given, also ju = J_k u (J is read once, for both).  TRJ: the same with J_k^T in place
// of J_k (K_k^T = I - (w_k / 2) J_k^T, ju = J_k^T u).
template <int NX, bool TRJ, typename P>
__device__ __forceinline__ void node_lu(P Jp, int64_t js, double wk, double (&K)[NX][NX], double (&rp)[NX],
                                        int* flag, const double* u, double* ju) {
  double jmax = 0.0;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const double jv = Jp[(int64_t)(TRJ ? q * NX + r : r * NX + q) * js];
      if (flag) jmax = fmax(jmax, fabs(jv));
      if (u) acc += jv * u[q];
      K[r][q] = (r == q ? 1.0 : 0.0) - 0.5 * wk * jv;
    }
    if (u) ju[r] = acc;
  }
  lu_kmat<NX>(K, rp, flag, 1.0 + 0.5 * fabs(wk) * jmax);
}

// Per-node J staged through LDS: the kTC nodes of a chunk are consecutive, so a lane's
// direct reads of J would be 32 bytes apart across the wave.  Instead each of kTC rounds
// stages 64 consecutive nodes of the wave's 4 * 64 (J entry e of node 64 j + l at
// lds[e * 64 + l], coalesced global reads), and the 16 lanes whose chunks lie in them
// (lanes 16 j .. 16 j + 15) then work their nodes from LDS.
// BACK: scan positions run from the last node down (position p is node N_n - 1 - p).
// The loads of a round go to registers first (fetch_j), so that the next round's loads
// can be in flight while the current round is worked; put_j then writes them to LDS.
template <int NX, bool BACK>
__device__ __forceinline__ void fetch_j(double (&v)[NX * NX], const double* __restrict__ Jn, int64_t Nn, int64_t kl) {
  const int64_t k = BACK ? Nn - 1 - kl : kl;
#pragma unroll
  for (int e = 0; e < NX * NX; ++e) v[e] = (kl < Nn) ? Jn[(int64_t)e * Nn + k] : 0.0;
}
template <int NX>
__device__ __forceinline__ void put_j(double* __restrict__ jw, const double (&v)[NX * NX], int l) {
#pragma unroll
  for (int e = 0; e < NX * NX; ++e) jw[e * 64 + l] = v[e];
}

// The map of one chunk, composed node by node from A = I, b = 0.  Node k takes
// S -> S + w_k J_k K_k^{-1} (y_k + S); since w_k J_k = 2 (I - K_k), that is
// S -> C_k S + (C_k - I) y_k with C_k = 2 K_k^{-1} - I, so with x = K_k^{-1} v
//     A <- C_k A:  each column a of A becomes a + 2 (K_k^{-1} a - a),
//     b <- C_k b + (C_k - I) y_k = b + 2 (K_k^{-1} u - u),  u = b + y_k,
// which needs only the factors of K_k (no J_k and no H_k kept).  BACK (P^{-T}, backward
// substitution with P^T from the last node, T the sum of the later x): node k takes
// T -> T + K_k^{-T} (y_k + w_k J_k^T T) = C'_k T + K_k^{-T} y_k with C'_k = 2 K_k^{-T} - I,
// so A as above with K_k^T, and b <- K_k^{-T} (2 b + y_k) - b.  Positions p = k0 + j run
// over the nodes (node p, or N_n - 1 - p with BACK); positions past N_n are identity maps.
template <int NX, bool BACK, typename P, typename T>
__device__ __forceinline__ void chunk_map(P Jp, int64_t jstep, int64_t js, const double* __restrict__ w,
                                          const T* __restrict__ yi, int64_t Nn, int64_t k0, Aff<NX>& m, int* flag) {
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int64_t pos = k0 + j;
    if (pos >= Nn) break;
    const int64_t k = BACK ? Nn - 1 - pos : pos;
    const double wk = w[k];
    double K[NX][NX], rp[NX];
    node_lu<NX, BACK>(Jp + j * jstep, js, wk, K, rp, flag, nullptr, nullptr);
    double u[NX], x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      const double yv = (double)yi[(int64_t)r * Nn + k];
      u[r] = BACK ? 2.0 * m.b[r] + yv : m.b[r] + yv;
      x[r] = u[r];
    }
    lu_solve<NX>(K, rp, x);
#pragma unroll
    for (int r = 0; r < NX; ++r) m.b[r] = BACK ? x[r] - m.b[r] : m.b[r] + 2.0 * (x[r] - u[r]);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
#pragma unroll
      for (int r = 0; r < NX; ++r) x[r] = m.A[r][c];
      lu_solve<NX>(K, rp, x);
#pragma unroll
      for (int r = 0; r < NX; ++r) m.A[r][c] += 2.0 * (x[r] - m.A[r][c]);
    }
  }
}

// Replay of a chunk from state s (FastPinvY box): per node u = y_k + S,
// xi_k = K_k^{-1} u, (J xi)_k = K_k^{-1} (J_k u) (J_k commutes with K_k^{-1}),
// S <- S + w_k (J xi)_k.  BACK (P^{-T}, from the last node): x_k = K_k^{-T} (y_k +
// w_k J_k^T T), T <- T + x_k; ji is not written.
// LOUT (J_k staged in LDS, one column of 64-strided entries per node): xi_k and (J xi)_k
// go to entries 0..NX-1 and NX..2NX-1 of the node's own column, whose J_k has been read
// by then, and the caller stores them coalesced after the round.
template <int NX, bool BACK, bool LOUT = false, typename P, typename T>
__device__ __forceinline__ void chunk_replay(P Jp, int64_t jstep, int64_t js, const double* __restrict__ w,
                                             const T* __restrict__ yi, T* __restrict__ oi, T* __restrict__ ji,
                                             int64_t Nn, int64_t k0, double (&s)[NX]) {
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int64_t pos = k0 + j;
    if (pos >= Nn) break;
    const int64_t k = BACK ? Nn - 1 - pos : pos;
    const double wk = w[k];
    double u[NX], ju[NX], K[NX][NX], rp[NX];
    if constexpr (BACK) {
      node_lu<NX, true>(Jp + j * jstep, js, wk, K, rp, nullptr, s, ju);
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = (double)yi[(int64_t)r * Nn + k] + wk * ju[r];
      lu_solve<NX>(K, rp, u);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        s[r] += u[r];
        if constexpr (LOUT) Jp[j * jstep + (int64_t)r * js] = u[r];
        else oi[(int64_t)r * Nn + k] = (T)u[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = s[r] + (double)yi[(int64_t)r * Nn + k];
      node_lu<NX, false>(Jp + j * jstep, js, wk, K, rp, nullptr, u, ju);
      lu_solve<NX>(K, rp, u);
      lu_solve<NX>(K, rp, ju);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        s[r] += wk * ju[r];
        if constexpr (LOUT) {
          Jp[j * jstep + (int64_t)r * js] = u[r];
          Jp[j * jstep + (int64_t)(NX + r) * js] = ju[r];
        } else {
          oi[(int64_t)r * Nn + k] = (T)u[r];
          if (ji) ji[(int64_t)r * Nn + k] = (T)ju[r];
        }
      }
    }
  }
}

// The same replay from LDS-staged J_k for a whole wave, in round j of the staging
// (positions kw + 64 j + c, c < 64, of which lane c read y and w coalesced into yc, wc):
// lanes 16 j .. 16 j + 15 (act) replay their chunks, the node at column
// c = 4 (l mod 16) + jj taking y and w from lane c by a shuffle, which every lane of the
// wave executes; the other lanes run the same instructions on column 0 and change
// nothing.  Outputs as with LOUT.
template <int NX, bool BACK>
__device__ __forceinline__ void chunk_replay_wave(double* __restrict__ jcol, bool act, const double (&yc)[NX],
                                                  double wc, int64_t Nn, int64_t k0, double (&s)[NX]) {
  const int l = (int)(threadIdx.x & 63);
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int src = 4 * (l & 15) + j;
    double yv[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) yv[r] = __shfl(yc[r], src, 64);
    const double wk = __shfl(wc, src, 64);
    const bool live = act && k0 + j < Nn;
    double* Jp = jcol + j;
    double u[NX], ju[NX], K[NX][NX], rp[NX];
    if constexpr (BACK) {
      node_lu<NX, true>(Jp, int64_t(64), wk, K, rp, nullptr, s, ju);
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = yv[r] + wk * ju[r];
      lu_solve<NX>(K, rp, u);
      if (live) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          s[r] += u[r];
          Jp[r * 64] = u[r];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = s[r] + yv[r];
      node_lu<NX, false>(Jp, int64_t(64), wk, K, rp, nullptr, u, ju);
      lu_solve<NX>(K, rp, u);
      lu_solve<NX>(K, rp, ju);
      if (live) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          s[r] += wk * ju[r];
          Jp[r * 64] = u[r];
          Jp[(NX + r) * 64] = ju[r];
        }
      }
    }
  }
}

// The map of one chunk: node k takes S -> (I + H_k) S + H_k y_k, so from A = I, b = 0 the
// first node gives (I + H, H y) and each further node A <- A + H A, b <- b + H (b + y).
// hs points at the thread's slot of field 0, node 0 of its tile.
// y of node j of the chunk, component r, at yb[r ystride + j] (global: yb = y + k0,
// ystride = N_n; staged in LDS: the tile's y component-major).
template <int NX, typename T>
__device__ __forceinline__ void chunk_map_h(const T* __restrict__ hs, const T* __restrict__ yb, int64_t ystride,
                                          int64_t Nn, int64_t k0, Aff<NX>& m) {
  constexpr int E = NX * NX + 1;
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int64_t k = k0 + j;
    const T* base = hs + (int64_t)j * E * kTileThreads;
    double H[NX][NX], yv[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int q = 0; q < NX; ++q) H[r][q] = (double)base[(r * NX + q) * kTileThreads];
#pragma unroll
    for (int r = 0; r < NX; ++r) yv[r] = (k < Nn) ? (double)yb[(int64_t)r * ystride + j] : 0.0;
    if (j == 0) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) {
          m.A[r][q] = H[r][q] + ((r == q) ? 1.0 : 0.0);
          acc += H[r][q] * yv[q];
        }
        m.b[r] = acc;
      }
    } else {
      double u[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = m.b[r] + yv[r];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) acc += H[r][q] * u[q];
        m.b[r] += acc;
      }
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        double t[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < NX; ++q) acc += H[r][q] * m.A[q][c];
          t[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < NX; ++r) m.A[r][c] += t[r];
      }
    }
  }
}

// Backward (P^{-T}) counterparts reading the same cached tables: position p is node
// k = N_n - 1 - p, whose H_k sits in its own tile slot (tile k / kTileNodes, thread
// (k / kTC) mod kTileThreads, node k mod kTC); G_k = H_k^T.  Node map (K_k^{-T} = I + G/2
// and w_k J_k^T K_k^{-T} = G): T -> (I + G) T + (I + G / 2) y_k, so A <- A + G A and
// b <- b + y_k + G (b + y_k / 2); replay x_k = y_k + G (T + y_k / 2), T <- T + x_k.
template <typename T>
__device__ __forceinline__ const T* node_slot(const T* __restrict__ tab, int64_t k, int E) {
  return tab + (k / kTileNodes) * kTC * E * kTileThreads + (k % kTC) * E * kTileThreads + (k / kTC) % kTileThreads;
}

// yp: y of the chunk's positions, component r of position k0 + j at yp[r kTileNodes + j]
// (the tile's y staged in LDS in position order).
template <int NX, typename T>
__device__ __forceinline__ void chunk_map_ht(const T* __restrict__ tab, const T* __restrict__ yp, int64_t Nn,
                                             int64_t k0, Aff<NX>& m) {
  constexpr int E = NX * NX + 1;
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int64_t pos = k0 + j;
    if (pos >= Nn) break;
    const int64_t k = Nn - 1 - pos;
    const T* base = node_slot<T>(tab, k, E);
    double G[NX][NX], yv[NX], u[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int q = 0; q < NX; ++q) G[r][q] = (double)base[(q * NX + r) * kTileThreads];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      yv[r] = (double)yp[r * kTileNodes + j];
      u[r] = m.b[r] + 0.5 * yv[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += G[r][q] * u[q];
      m.b[r] += yv[r] + acc;
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double t[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) acc += G[r][q] * m.A[q][c];
        t[r] = acc;
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) m.A[r][c] += t[r];
    }
  }
}

// yp as in chunk_map_ht; x_k replaces y_k there (the caller stores the tile).
template <int NX, typename T>
__device__ __forceinline__ void chunk_replay_ht(const T* __restrict__ tab, T* __restrict__ yp, int64_t Nn, int64_t k0,
                                                double (&s)[NX]) {
  constexpr int E = NX * NX + 1;
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int64_t pos = k0 + j;
    if (pos >= Nn) break;
    const int64_t k = Nn - 1 - pos;
    const T* base = node_slot<T>(tab, k, E);
    double yv[NX], u[NX], x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      yv[r] = (double)yp[r * kTileNodes + j];
      u[r] = s[r] + 0.5 * yv[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) acc += (double)base[(q * NX + r) * kTileThreads] * u[q];
      x[r] = yv[r] + acc;
      yp[r * kTileNodes + j] = (T)x[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] += x[r];
  }
}

template <int NX>
__device__ __forceinline__ void aff_store(double* __restrict__ o, const Aff<NX>& m) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
#pragma unroll
    for (int q = 0; q < NX; ++q) o[r * NX + q] = m.A[r][q];
    o[NX * NX + r] = m.b[r];
  }
}

template <int NX>
__device__ __forceinline__ void aff_load(const double* __restrict__ o, Aff<NX>& m) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
#pragma unroll
    for (int q = 0; q < NX; ++q) m.A[r][q] = o[r * NX + q];
    m.b[r] = o[NX * NX + r];
  }
}

// H_k and w_k of every node in the tile layout, straight from J (per node or constant)
// and the weights: K = I - (w_k / 2) J_k by unpivoted LU (pivot check as lu_kmat), then
// H_k = K^{-1} (w_k J_k) column by column.  Slots of nodes past N_n are zeroed.  Each
// of the kTC rounds of the workgroup takes kTileThreads consecutive nodes (coalesced
// reads of J and w) and writes each node to its chunk's slot.  tile = (k, g).
template <int NX, typename JT>
__global__ __launch_bounds__(kTileThreads, 2) void k_tmake_h(JT* __restrict__ jsw, const double* __restrict__ J,
                                                            int per_node, const PinvDesc* __restrict__ pd,
                                                            const int2* __restrict__ tiles, int* flag) {
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t g = t.y;
  constexpr int E = NX * NX + 1;
  const int64_t Nn = d.Nn;
  JT* tb = jsw + d.jsw_off + g * kTC * E * kTileThreads;
  const double* Jn = J + d.joff;
  const double* Jc = J + d.jcoff;
#pragma unroll 1
  for (int j = 0; j < kTC; ++j) {
    const int i = j * kTileThreads + (int)threadIdx.x;  // node within the tile
    const int64_t k = g * kTileNodes + i;
    JT* base = tb + (int64_t)(i % kTC) * E * kTileThreads + i / kTC;
    if (k >= Nn) {
#pragma unroll
      for (int e = 0; e < E; ++e) base[e * kTileThreads] = (JT)0;
      continue;
    }
    const double wk = d.w[k];
    double Jk[NX][NX], K[NX][NX], rp[NX];
    double jmax = 0.0;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        const double jv = per_node ? Jn[(int64_t)(r * NX + q) * Nn + k] : Jc[r * NX + q];
        Jk[r][q] = jv;
        jmax = fmax(jmax, fabs(jv));
        K[r][q] = (r == q ? 1.0 : 0.0) - 0.5 * wk * jv;
      }
    lu_kmat<NX>(K, rp, flag, 1.0 + 0.5 * fabs(wk) * jmax);
#pragma unroll
    for (int cc = 0; cc < NX; ++cc) {
      double x[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) x[r] = wk * Jk[r][cc];
      lu_solve<NX>(K, rp, x);
#pragma unroll
      for (int r = 0; r < NX; ++r) base[(r * NX + cc) * kTileThreads] = (JT)x[r];
    }
    base[(E - 1) * kTileThreads] = (JT)wk;
  }
}

// A tile's y in position order (node k = tb + i, or N_n - 1 - tb - i with BACK) into
// buf[r kTileNodes + i], coalesced; zeros past the instance.  And the store of buf back
// to out in the same order.
template <int NX, bool BACK, typename T>
__device__ __forceinline__ void stage_tile(T* __restrict__ buf, const T* __restrict__ yi, int64_t Nn, int64_t tb) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
#pragma unroll
    for (int q = 0; q < kTC; ++q) {
      const int i = (int)threadIdx.x + q * kTileThreads;
      const int64_t pos = tb + i;
      buf[r * kTileNodes + i] = pos < Nn ? yi[(int64_t)r * Nn + (BACK ? Nn - 1 - pos : pos)] : T(0);
    }
  }
}
template <int NX, bool BACK, typename T>
__device__ __forceinline__ void store_tile(const T* __restrict__ buf, T* __restrict__ oi, int64_t Nn, int64_t tb) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
#pragma unroll
    for (int q = 0; q < kTC; ++q) {
      const int i = (int)threadIdx.x + q * kTileThreads;
      const int64_t pos = tb + i;
      if (pos < Nn) oi[(int64_t)r * Nn + (BACK ? Nn - 1 - pos : pos)] = buf[r * kTileNodes + i];
    }
  }
}

// Tile maps: each chunk's map composed from its node maps, scanned across the wave by
// DPP, then composed with the maps of the tile's earlier waves (a 4-lane scan of the wave
// totals gives their prefixes), so chunk t holds the map of nodes 0 .. 4t + 3 of its tile.
// These inclusive maps are stored as [g][field][t] (scan[tmap + g F 256 + f 256 + t]) and
// the last one is the tile aggregate, stored field-major (scan[tagg + f ntile + g]) so
// that the one-workgroup tile scan reads it coalesced.  tile = (k, g).
template <int NX, int MODE, bool BACK, typename T>
__global__ __launch_bounds__(kTileThreads, 2) void k_tscan_reduce(const double* __restrict__ J, const T* __restrict__ jsw,
                                                             const T* __restrict__ y,
                                                             const PinvDesc* __restrict__ pd,
                                                             const int2* __restrict__ tiles,
                                                             double* __restrict__ scan, int* flag) {
  constexpr int F = NX * NX + NX;
  constexpr int NW = kTileThreads / 64;
  __shared__ double tot[NW][F];
  __shared__ double jl[MODE == kFlyPerNode ? NW * 64 * NX * NX : 1];
  __shared__ T yl[MODE == kCachedH ? NX * kTileNodes : 1];
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t g = t.y;
  const int64_t k0 = (g * kTileThreads + threadIdx.x) * kTC;
  const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
  double* cm = scan + d.tmap + g * F * kTileThreads + threadIdx.x;
  {
    Aff<NX> m;
    aff_identity<NX>(m);
    if constexpr (MODE == kFlyPerNode) {
      double* jw = jl + w * 64 * NX * NX;
      const int64_t kw = g * kTileNodes + (int64_t)w * 64 * kTC;
      double pre[NX * NX];
      fetch_j<NX, BACK>(pre, J + d.joff, d.Nn, kw + l);
      for (int j = 0; j < kTC; ++j) {
        put_j<NX>(jw, pre, l);
        __syncthreads();
        if (j + 1 < kTC) fetch_j<NX, BACK>(pre, J + d.joff, d.Nn, kw + 64 * (j + 1) + l);
        if ((l >> 4) == j)
          chunk_map<NX, BACK>(jw + (4 * l - 64 * j), int64_t(1), int64_t(64), d.w, y + d.off, d.Nn, k0, m, flag);
        __syncthreads();
      }
    } else if constexpr (MODE == kFlyConst) {
      chunk_map<NX, BACK>(J + d.jcoff, int64_t(0), int64_t(1), d.w, y + d.off, d.Nn, k0, m, flag);
    } else {
      // the tile's y staged coalesced through LDS (component-major, position order)
      stage_tile<NX, BACK, T>(yl, y + d.off, d.Nn, g * kTileNodes);
      __syncthreads();
      if constexpr (BACK) {
        chunk_map_ht<NX, T>(jsw + d.jsw_off, yl + (int)threadIdx.x * kTC, d.Nn, k0, m);
      } else {
        constexpr int E = NX * NX + 1;
        chunk_map_h<NX, T>(jsw + d.jsw_off + g * kTC * E * kTileThreads + threadIdx.x, yl + (int)threadIdx.x * kTC,
                           int64_t(kTileNodes), d.Nn, k0, m);
      }
    }
    wave_scan<NX>(m);
    if (l == 63) aff_store<NX>(&tot[w][0], m);
#pragma unroll
    for (int f = 0; f < F; ++f) cm[f * kTileThreads] = (f < NX * NX) ? m.A[f / NX][f % NX] : m.b[f - NX * NX];
  }
  __syncthreads();
  if (w == 0) {
    // lanes 1..NW-1 of wave 0 turn the wave totals into the maps of waves 0..l-1; within
    // the wave every lane reads tot before any lane writes it
    Aff<NX> p;
    if (l >= 1 && l < NW)
      aff_load<NX>(&tot[l - 1][0], p);
    else
      aff_identity<NX>(p);
    scan_step<NX, 0x111, 0xF>(p, l >= 2);
    scan_step<NX, 0x112, 0xF>(p, l >= 3);
    if (l >= 1 && l < NW) aff_store<NX>(&tot[l][0], p);
  }
  __syncthreads();
  if (w > 0) {
    // the wave's maps, stored above, <- map o (map of the earlier waves); row r of the
    // product needs row r of the map only
    Aff<NX> q;
    aff_load<NX>(&tot[w][0], q);
    double last[F];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double a[NX];
#pragma unroll
      for (int c = 0; c < NX; ++c) a[c] = cm[(r * NX + c) * kTileThreads];
      double nb = cm[(NX * NX + r) * kTileThreads];
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        nb += a[c] * q.b[c];
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < NX; ++u) v += a[u] * q.A[u][c];
        cm[(r * NX + c) * kTileThreads] = v;
        last[r * NX + c] = v;
      }
      cm[(NX * NX + r) * kTileThreads] = nb;
      last[NX * NX + r] = nb;
    }
    if (threadIdx.x == kTileThreads - 1) {
#pragma unroll
      for (int f = 0; f < F; ++f) scan[d.tagg + f * d.ntile + g] = last[f];
    }
  }
}


// Tile start states of one instance (S = 0 before node 0), one workgroup of
// tiles_threads<NX>() per instance: thread t composes the aggregates of tiles
// [t q, t q + q), the maps are scanned across the workgroup, and each thread then walks
// its tiles from its start state.  Aggregates and start states are field-major
// ([field][tile]), so a wave's loads and stores touch a few cache lines rather than one
// per lane: the whole scan runs on one CU, whose request rate bounds it.  512 threads
// (fewer tiles per thread) where a thread's map fits two waves per SIMD, 256 above
// n_x = 6.
template <int NX>
constexpr int tiles_threads() { return NX <= 6 ? 512 : 256; }

template <int NX>
__global__ __launch_bounds__(tiles_threads<NX>()) void k_tscan_tiles(double* __restrict__ scan,
                                                                     const PinvDesc* __restrict__ pd) {
  constexpr int F = NX * NX + NX;
  constexpr int NT = tiles_threads<NX>();
  __shared__ double tot[NT / 64][F];
  const PinvDesc& d = pd[blockIdx.x];
  const int64_t nt = d.ntile;
  const int64_t q = (nt + NT - 1) / NT;
  const int64_t i0 = (int64_t)threadIdx.x * q;
  const int64_t i1 = min(nt, i0 + q);
  const double* agg = scan + d.tagg;
  Aff<NX> m;
  aff_identity<NX>(m);
  for (int64_t i = i0; i < i1; ++i) compose<NX>(agg + i, nt, m.A, m.b);
  wave_scan<NX>(m);
  const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
  if (l == 63) aff_store<NX>(&tot[w][0], m);
  __syncthreads();
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = 0.0;
  for (int v = 0; v < w; ++v) advance<NX>(&tot[v][0], 1, s);
  double x[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) x[r] = s[r];
  aff_apply<NX>(m, x);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    const double up = __shfl_up(x[r], 1);
    s[r] = (l == 0) ? s[r] : up;
  }
  double* st = scan + d.tst;
  for (int64_t i = i0; i < i1; ++i) {
#pragma unroll
    for (int r = 0; r < NX; ++r) st[r * nt + i] = s[r];
    advance<NX>(agg + i, nt, s);
  }
}

// Replay of one tile: chunk t starts from the tile start state advanced by the inclusive
// map of chunk t - 1 (k_tscan_reduce), then replays its nodes (chunk_replay); K_k is
// formed and factored here again from J_k and w_k.  tile = (k, g).
template <int NX, int MODE, bool BACK, typename T>
__global__ __launch_bounds__(kTileThreads) void k_tscan_apply(const double* __restrict__ J, const T* __restrict__ jsw,
                                                            const T* __restrict__ y,
                                                            const PinvDesc* __restrict__ pd,
                                                            const int2* __restrict__ tiles,
                                                            const double* __restrict__ scan, T* __restrict__ out,
                                                            T* __restrict__ jout) {
  constexpr int F = NX * NX + NX;
  constexpr int NW = kTileThreads / 64;
  __shared__ double jl[MODE == kFlyPerNode ? NW * 64 * NX * NX : 1];
  // cached H, forward: the tile's y (component-major, node i of the tile at io[r][i]) and
  // then its xi, so that both move coalesced
  __shared__ T io[MODE == kCachedH ? NX * kTileNodes : 1];
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t g = t.y;
  const int64_t Nn = d.Nn;
  const int64_t k0 = (g * kTileThreads + threadIdx.x) * kTC;
  double s[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) s[r] = scan[d.tst + r * d.ntile + g];
  if (threadIdx.x > 0 && k0 < Nn) {
    const double* cm = scan + d.tmap + g * F * kTileThreads + (threadIdx.x - 1);
    double ns[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double acc = cm[(NX * NX + r) * kTileThreads];
#pragma unroll
      for (int c = 0; c < NX; ++c) acc += cm[(r * NX + c) * kTileThreads] * s[c];
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) s[r] = ns[r];
  }
  const T* yi = y + d.off;
  T* oi = out + d.off;
  T* ji = jout ? jout + d.off : nullptr;
  if constexpr (MODE == kFlyPerNode) {
    // every thread takes part in the staging rounds (no early exit before the barriers)
    const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    double* jw = jl + w * 64 * NX * NX;
    const int64_t kw = g * kTileNodes + (int64_t)w * 64 * kTC;
    double pre[NX * NX];
    fetch_j<NX, BACK>(pre, J + d.joff, Nn, kw + l);
    // the round's outputs come back through the LDS columns (xi in entries 0..NX-1, J xi in
    // NX..2NX-1) and are stored coalesced, lane l taking node kw + 64 j + l; each lane then
    // writes only its own column in the next put_j, so no barrier is needed between
    // (n_x >= 2) y and w are read coalesced with the staged J, one round ahead, and handed
    // to the replaying lanes by shuffles (chunk_replay_wave)
    constexpr bool kLout = 2 * NX <= NX * NX;
    double ypre[NX], wpre = 0.0;
    if constexpr (kLout) {
      const int64_t pos = kw + l;
      const int64_t k = BACK ? Nn - 1 - pos : pos;
#pragma unroll
      for (int r = 0; r < NX; ++r) ypre[r] = pos < Nn ? (double)yi[(int64_t)r * Nn + k] : 0.0;
      wpre = pos < Nn ? d.w[k] : 0.0;
    }
    for (int j = 0; j < kTC; ++j) {
      put_j<NX>(jw, pre, l);
      double ycur[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) ycur[r] = kLout ? ypre[r] : 0.0;
      const double wcur = wpre;
      __syncthreads();
      if (j + 1 < kTC) {
        fetch_j<NX, BACK>(pre, J + d.joff, Nn, kw + 64 * (j + 1) + l);
        if constexpr (kLout) {
          const int64_t pos = kw + 64 * (j + 1) + l;
          const int64_t k = BACK ? Nn - 1 - pos : pos;
#pragma unroll
          for (int r = 0; r < NX; ++r) ypre[r] = pos < Nn ? (double)yi[(int64_t)r * Nn + k] : 0.0;
          wpre = pos < Nn ? d.w[k] : 0.0;
        }
      }
      const bool act = (l >> 4) == j;
      if constexpr (kLout) {
        chunk_replay_wave<NX, BACK>(jw + (act ? 4 * l - 64 * j : 0), act, ycur, wcur, Nn, k0, s);
      } else if (act) {
        chunk_replay<NX, BACK>(jw + (4 * l - 64 * j), int64_t(1), int64_t(64), d.w, yi, oi, ji, Nn, k0, s);
      }
      __syncthreads();
      if constexpr (kLout) {
        const int64_t pos = kw + 64 * j + l;
        if (pos < Nn) {
          const int64_t k = BACK ? Nn - 1 - pos : pos;
#pragma unroll
          for (int r = 0; r < NX; ++r) oi[(int64_t)r * Nn + k] = (T)jw[r * 64 + l];
          if (!BACK && ji) {
#pragma unroll
            for (int r = 0; r < NX; ++r) ji[(int64_t)r * Nn + k] = (T)jw[(NX + r) * 64 + l];
          }
        }
      }
    }
  } else if constexpr (MODE == kFlyConst) {
    chunk_replay<NX, BACK>(J + d.jcoff, int64_t(0), int64_t(1), d.w, yi, oi, ji, Nn, k0, s);
  } else {
    // H_k from precond_prepare: v = H_k u, xi_k = u + v / 2, (J xi)_k = v / w_k, S <- S + v
    const int64_t tb = g * kTileNodes;  // first position of the tile
    stage_tile<NX, BACK, T>(io, yi, Nn, tb);
    __syncthreads();
    if constexpr (BACK) {
      chunk_replay_ht<NX, T>(jsw + d.jsw_off, io + (int)threadIdx.x * kTC, Nn, k0, s);
      __syncthreads();
      store_tile<NX, true, T>(io, oi, Nn, tb);
      return;
    }
    constexpr int E = NX * NX + 1;
    const T* hs = jsw + d.jsw_off + g * kTC * E * kTileThreads + threadIdx.x;
    const int i0 = (int)threadIdx.x * kTC;
#pragma unroll 1
    for (int j = 0; j < kTC; ++j) {
      const int64_t k = k0 + j;
      if (k >= Nn) break;
      const T* base = hs + (int64_t)j * E * kTileThreads;
      const double inv_w = 1.0 / (double)base[(E - 1) * kTileThreads];
      double u[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) u[r] = s[r] + (double)io[r * kTileNodes + i0 + j];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) v += (double)base[(r * NX + q) * kTileThreads] * u[q];
        s[r] += v;
        io[r * kTileNodes + i0 + j] = (T)(u[r] + 0.5 * v);
        if (ji) ji[(int64_t)r * Nn + k] = (T)(v * inv_w);
      }
    }
    __syncthreads();
    store_tile<NX, false, T>(io, oi, Nn, tb);
  }
}

// Replay for n_x > 8, sixteen lanes per chunk: lane r < NX carries component r of the
// state; per node u_r = y_r + S_r, v_r = (H_k u)_r with u gathered across the group,
// xi_r = u_r + v_r / 2, (J xi)_r = v_r / w_k, S_r <- S_r + v_r, from the chunk's level-0
// start state.  grid = (tile (k, block of 256 level-0 threads), 16 groups of 16 chunks).
template <int NX, typename T>
__global__ __launch_bounds__(256) void k_pinv_final_lanes(const T* __restrict__ jsw, const T* __restrict__ y,
                                                          const PinvDesc* __restrict__ pd,
                                                          const int2* __restrict__ tiles,
                                                          const double* __restrict__ scan, T* __restrict__ out,
                                                          T* __restrict__ jout) {
  static_assert(NX <= 16, "one state component per lane of a 16-lane group");
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t tau = (int64_t)t.y * 256 + blockIdx.y * 16 + (threadIdx.x >> 4);
  const int r = (int)(threadIdx.x & 15);
  const int64_t B = tau / (64 * kFan);
  const int i = (int)((tau >> 6) % kFan);
  const int l = (int)(tau & 63);
  const int64_t c = (B * 64 + l) * kFan + i;
  if (c >= d.cnt[0]) return;  // the whole group leaves together
  constexpr int E = hrec<NX>();
  const int64_t Nn = d.Nn;
  const bool act = r < NX;
  const int rr = act ? r : 0;
  const T* js = jsw + d.jsw_off + (((B * kFan + i) * 64 + l) * kChunk) * E;
  const T* yi = y + d.off;
  T* oi = out + d.off;
  T* ji = jout ? jout + d.off : nullptr;
  double s = act ? scan[d.st[0] + swz(B, i, rr, NX, l)] : 0.0;
  const int64_t k0 = c * kChunk;
  const int jn = (int)min((int64_t)kChunk, Nn - k0);
  // the chunk's kChunk values of y (one 128-byte run per component) are loaded together,
  // and its outputs kept in registers and stored together at the end, so that each run
  // is read and written back to back; row r of H_k and w_k of the next node are loaded
  // while the current node is replayed (the replay itself waits on the carried state)
  const T* yr = yi + (int64_t)rr * Nn + k0;
  double yv[kChunk], xo[kChunk], jo[kChunk];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) yv[j] = (act && j < jn) ? (double)yr[j] : 0.0;
  double hn[NX], wn = 1.0;
  auto fetch = [&](int j) {
    const T* base = js + (int64_t)j * E;
    load_row<NX, T>(base + rr * NX, hn);
    if (!act) {
#pragma unroll
      for (int q = 0; q < NX; ++q) hn[q] = 0.0;
    }
    wn = (double)base[NX * NX];
  };
  if (jn > 0) fetch(0);
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    if (j < jn) {
      double h[NX];
#pragma unroll
      for (int q = 0; q < NX; ++q) h[q] = hn[q];
      const double wk = wn;
      const double u = s + yv[j];
      if (j + 1 < jn) fetch(j + 1);
      double v = 0.0;
      static_for<0, NX>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        v += h[q] * row_bcast<q>(u);
      });
      s += v;
      xo[j] = u + 0.5 * v;
      jo[j] = v * recip(wk);
    }
  }
  if (act) {
    T* orow = oi + (int64_t)r * Nn + k0;
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (j < jn) orow[j] = (T)xo[j];
    if (ji) {
      T* jrow = ji + (int64_t)r * Nn + k0;
#pragma unroll
      for (int j = 0; j < kChunk; ++j)
        if (j < jn) jrow[j] = (T)jo[j];
    }
  }
}

// y_k = J_k x_k per node for every instance of a class.  tile = (k, block of 256 nodes).
template <int NX, typename T>
__global__ __launch_bounds__(256) void k_jac_class(const double* __restrict__ J, int per_node,
                                                   const T* __restrict__ x, T* __restrict__ y,
                                                   const PinvDesc* __restrict__ pd, const int2* __restrict__ tiles) {
  const int2 t = tiles[blockIdx.x];
  const PinvDesc& d = pd[t.x];
  const int64_t k = (int64_t)t.y * blockDim.x + threadIdx.x;
  const int64_t Nn = d.Nn;
  if (k >= Nn) return;
  const T* xi = x + d.off;
  T* yi = y + d.off;
  double xv[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) xv[c] = (double)xi[(int64_t)c * Nn + k];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double j = per_node ? J[d.joff + ((int64_t)(r * NX + c)) * Nn + k] : J[d.jcoff + r * NX + c];
      acc += j * xv[c];
    }
    yi[(int64_t)r * Nn + k] = (T)acc;
  }
}

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Level sizes of the scan for one instance: cnt[0] chunks, then groups of kFan.
static int pinv_levels(int64_t Nn, int64_t* cnt) {
  int L = 0;
  cnt[0] = (Nn + kChunk - 1) / kChunk;
  while (cnt[L] > kFan && L < kPinvMaxLevels - 1) {
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

static int64_t pinv_tiles(int64_t Nn) { return (Nn + kTileNodes - 1) / kTileNodes; }

int64_t pinv_jsw_size(int64_t Nn, int nx) {
  if (nx <= kWaveNx) return pinv_tiles(Nn) * kTileNodes * ((int64_t)nx * nx + 1);
  int64_t cnt[kPinvMaxLevels];
  pinv_levels(Nn, cnt);
  return pinv_blocks0(cnt[0]) * 64 * kFan * kChunk * (((int64_t)nx * nx + 4) & ~int64_t(3));  // hrec<nx>()
}

// Scratch (doubles) the inverse scan needs for one instance (level 0 in whole blocks).
int64_t pinv_scratch(int64_t Nn, int nx) {
  const int64_t S = (int64_t)nx * nx + 2 * nx;
  if (nx <= kWaveNx) return pinv_tiles(Nn) * (S + ((int64_t)nx * nx + nx) * kTileThreads);
  int64_t cnt[kPinvMaxLevels];
  const int L = pinv_levels(Nn, cnt);
  int64_t tot = pinv_blocks0(cnt[0]) * 64 * kFan * S;
  for (int l = 1; l <= L; ++l) tot += cnt[l] * S;
  return tot;
}

static hipError_t upload_tiles(birk_plan* p, const std::vector<int2>& v, int2** dst) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(v.size(), 1) * sizeof(int2));
  if (e != hipSuccess) return e;
  p->allocs.push_back(d);
  *dst = (int2*)d;
  if (v.empty()) return hipSuccess;
  return hipMemcpy(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice);
}

hipError_t plan_solve(birk_plan* p) {
  hipError_t e = hipSuccess;
  {
    // P y work lists: every tile of every component of every instance, and every
    // (instance, component) scan
    std::vector<int2> tl, pr;
    for (int i = 0; i < (int)p->inst.size(); ++i) {
      const Instance& in = p->inst[i];
      const int nt = (int)((in.Nn + kScanBlock - 1) / kScanBlock);
      for (int r = 0; r < in.nx; ++r) {
        pr.push_back(make_int2(i, r));
        for (int b = 0; b < nt; ++b) tl.push_back(make_int2(i, r * nt + b));
      }
    }
    if ((e = upload_tiles(p, tl, &p->pfwd_tiles)) != hipSuccess) return e;
    p->pfwd_ntiles = (int)tl.size();
    if ((e = upload_tiles(p, pr, &p->pfwd_pairs)) != hipSuccess) return e;
    p->pfwd_npairs = (int)pr.size();
    std::vector<int2> bt;
    p->pfwd_maxnx = 0;
    p->pfwd_unx = p->inst.empty() ? 0 : (int)p->inst[0].nx;
    for (int i = 0; i < (int)p->inst.size(); ++i) {
      const Instance& in = p->inst[i];
      const int nt = (int)((in.Nn + kScanBlock - 1) / kScanBlock);
      for (int b = 0; b < nt; ++b) bt.push_back(make_int2(i, b));
      p->pfwd_maxnx = std::max(p->pfwd_maxnx, (int)in.nx);
      if ((int)in.nx != p->pfwd_unx) p->pfwd_unx = 0;
    }
    if ((e = upload_tiles(p, bt, &p->pfwd_btiles)) != hipSuccess) return e;
    p->pfwd_nbtiles = (int)bt.size();
  }
  p->pclass.clear();
  for (int nx = 1; nx <= 12; ++nx) {
    PinvClass pc;
    pc.nx = nx;
    for (const Instance& in : p->inst) {
      if (in.nx != nx) continue;
      PinvDesc d;
      d.Nn = in.Nn;
      d.off = in.off;
      d.joff = in.joff;
      d.jcoff = in.jcoff;
      d.jsw_off = in.jsw_off;
      d.w = in.w;
      const int64_t S = (int64_t)nx * nx + nx;
      int64_t base = in.scan_off;
      if (nx <= kWaveNx) {
        // scratch: tile aggregates, tile start states, inclusive chunk maps per tile
        d.ntile = pinv_tiles(in.Nn);
        d.tagg = base;
        d.tst = base + d.ntile * S;
        d.tmap = d.tst + d.ntile * nx;
        pc.host.push_back(d);
        continue;
      }
      d.L = pinv_levels(in.Nn, d.cnt);
      d.nb0 = (int)pinv_blocks0(d.cnt[0]);
      // scratch: for each level l: agg[slots * S] then state[slots * NX]; level 0 swizzled
      for (int l = 0; l <= d.L; ++l) {
        const int64_t slots = (l == 0) ? (int64_t)d.nb0 * 64 * kFan : d.cnt[l];
        d.agg[l] = base;
        base += slots * S;
        d.st[l] = base;
        base += slots * nx;
      }
      pc.host.push_back(d);
      pc.Lmax = std::max(pc.Lmax, d.L);
    }
    if (pc.host.empty()) continue;
    pc.ninst = (int)pc.host.size();
    std::vector<int2> t0, tn, tt, tup[kPinvMaxLevels];
    for (int k = 0; k < pc.ninst; ++k) {
      const PinvDesc& d = pc.host[k];
      if (nx <= kWaveNx) {
        for (int64_t g = 0; g < d.ntile; ++g) tt.push_back(make_int2(k, (int)g));
        for (unsigned b = 0; b < nblocks(d.Nn, 256); ++b) tn.push_back(make_int2(k, (int)b));
        continue;
      }
      const int64_t thr0 = (int64_t)d.nb0 * 64 * kFan;
      for (unsigned b = 0; b < nblocks(thr0, 256); ++b) t0.push_back(make_int2(k, (int)b));
      for (unsigned b = 0; b < nblocks(d.Nn, 256); ++b) tn.push_back(make_int2(k, (int)b));
      for (int l = 0; l < d.L; ++l) {
        for (unsigned b = 0; b < nblocks(d.cnt[l + 1], 256); ++b) tup[l].push_back(make_int2(k, (int)b));
      }
    }
    void* dd = nullptr;
    if ((e = hipMalloc(&dd, pc.host.size() * sizeof(PinvDesc))) != hipSuccess) return e;
    p->allocs.push_back(dd);
    pc.dev = (PinvDesc*)dd;
    if ((e = hipMemcpy(dd, pc.host.data(), pc.host.size() * sizeof(PinvDesc), hipMemcpyHostToDevice)) != hipSuccess)
      return e;
    if ((e = upload_tiles(p, t0, &pc.t_node0)) != hipSuccess) return e;
    pc.n_node0 = (int)t0.size();
    if ((e = upload_tiles(p, tn, &pc.t_nodes)) != hipSuccess) return e;
    pc.n_nodes = (int)tn.size();
    if ((e = upload_tiles(p, tt, &pc.t_tile)) != hipSuccess) return e;
    pc.n_tile = (int)tt.size();
    for (int l = 0; l < pc.Lmax; ++l) {
      if ((e = upload_tiles(p, tup[l], &pc.t_up[l])) != hipSuccess) return e;
      pc.n_up[l] = (int)tup[l].size();
    }
    p->pclass.push_back(std::move(pc));
  }
  // Krylov segmentation
  {
    const int B = (int)p->inst.size();
    std::vector<int2> tiles, ranges(B);
    std::vector<int64_t> ioff(B), ilen(B);
    for (int i = 0; i < B; ++i) {
      const Instance& in = p->inst[i];
      ioff[i] = in.off;
      ilen[i] = in.Nn * in.nx;
      ranges[i].x = (int)tiles.size();
      for (int64_t c = 0; c * kSegChunk < ilen[i]; ++c) tiles.push_back(make_int2(i, (int)c));
      ranges[i].y = (int)tiles.size();
    }
    SegSet& sg = p->seg;
    sg.ntiles = (int)tiles.size();
    if ((e = upload_tiles(p, tiles, &sg.tiles)) != hipSuccess) return e;
    if ((e = upload_tiles(p, ranges, &sg.ranges)) != hipSuccess) return e;
    void* d1 = nullptr;
    void* d2 = nullptr;
    if ((e = hipMalloc(&d1, B * sizeof(int64_t))) != hipSuccess) return e;
    p->allocs.push_back(d1);
    if ((e = hipMalloc(&d2, B * sizeof(int64_t))) != hipSuccess) return e;
    p->allocs.push_back(d2);
    sg.ioff = (int64_t*)d1;
    sg.ilen = (int64_t*)d2;
    if ((e = hipMemcpy(d1, ioff.data(), B * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(d2, ilen.data(), B * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NX, typename JT>
static void make_h_class(birk_plan* p, const PinvClass& pc, const double* J, int pn, int what, hipStream_t s) {
  if constexpr (NX <= kWaveNx) {
    // per-node J applied repeatedly: H_k cached in the tile layout; otherwise the scan
    // kernels form K_k from J and w_k themselves
    if (pn && (what & kPrepCache))
      hipLaunchKernelGGL((k_tmake_h<NX, JT>), dim3(pc.n_tile), dim3(kTileThreads), 0, s, (JT*)p->jsw, J, pn, pc.dev,
                         pc.t_tile, p->flag);
  } else {
    if (!(what & kPrepLarge) || pc.n_node0 == 0) return;
    hipLaunchKernelGGL((k_make_h_rows<NX, JT>), dim3(pc.n_node0, 16), dim3(256), 0, s, (JT*)p->jsw, J, pn, pc.dev,
                       pc.t_node0, p->flag);
  }
}

#define BIRK_NX_SWITCH(nx, CALL)                                       \
  switch (nx) {                                                        \
    case 1: { constexpr int NXC = 1; CALL; } break;                    \
    case 2: { constexpr int NXC = 2; CALL; } break;                    \
    case 3: { constexpr int NXC = 3; CALL; } break;                    \
    case 4: { constexpr int NXC = 4; CALL; } break;                    \
    case 5: { constexpr int NXC = 5; CALL; } break;                    \
    case 6: { constexpr int NXC = 6; CALL; } break;                    \
    case 7: { constexpr int NXC = 7; CALL; } break;                    \
    case 8: { constexpr int NXC = 8; CALL; } break;                    \
    case 9: { constexpr int NXC = 9; CALL; } break;                    \
    case 10: { constexpr int NXC = 10; CALL; } break;                  \
    case 11: { constexpr int NXC = 11; CALL; } break;                  \
    case 12: { constexpr int NXC = 12; CALL; } break;                  \
    default: return hipErrorInvalidValue;                              \
  }

// Per-Jacobian preparation of the scan: n_x > kWaveNx lay J and w out in the level-0
// slots and replace the J fields by H_k (k_make_h_rows), which their scan kernels read.
// n_x <= kWaveNx with per-node J and kPrepCache (a solve, before its second application)
// cache H_k in the tile layout (k_tmake_h: one pass that turns the later applications'
// staged J reads and per-node factorisations into coalesced H_k reads); otherwise they
// need nothing.  what: kPrepLarge, kPrepCache or both.
hipError_t precond_prepare(birk_plan* p, int jac_kind, const double* J, int single, hipStream_t s, int what) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const PinvClass& pc : p->pclass) {
    if (single) {
      BIRK_NX_SWITCH(pc.nx, (make_h_class<NXC, float>(p, pc, J, pn, what, s)))
    } else {
      BIRK_NX_SWITCH(pc.nx, (make_h_class<NXC, double>(p, pc, J, pn, what, s)))
    }
  }
  return hipGetLastError();
}

template <int NX, typename T>
static void pinv_class(birk_plan* p, const PinvClass& pc, const double* J, int pn, int cached, const T* y, T* out,
                       T* jout, hipStream_t s) {
  const T* jsw = (const T*)p->jsw;
  double* scan = p->scan;
  if constexpr (NX <= kWaveNx) {
    const dim3 grid(pc.n_tile), block(kTileThreads);
    if (!pn) {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kFlyConst, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan,
                         p->flag);
    } else if (cached) {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kCachedH, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan,
                         p->flag);
    } else {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kFlyPerNode, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan,
                         p->flag);
    }
    hipLaunchKernelGGL((k_tscan_tiles<NX>), dim3(pc.ninst), dim3(tiles_threads<NX>()), 0, s, scan, pc.dev);
    if (!pn) {
      hipLaunchKernelGGL((k_tscan_apply<NX, kFlyConst, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan, out,
                         jout);
    } else if (cached) {
      hipLaunchKernelGGL((k_tscan_apply<NX, kCachedH, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan, out,
                         jout);
    } else {
      hipLaunchKernelGGL((k_tscan_apply<NX, kFlyPerNode, false, T>), grid, block, 0, s, J, jsw, y, pc.dev, pc.t_tile, scan,
                         out, jout);
    }
  } else {
    (void)J;
    (void)pn;
    (void)cached;
    hipLaunchKernelGGL((k_pinv_up0<NX, T>), dim3(pc.n_node0, 16), dim3(256), 0, s, jsw, y, pc.dev, pc.t_node0, scan);
    for (int l = 0; l < pc.Lmax; ++l)
      hipLaunchKernelGGL((k_pinv_up<NX>), dim3(pc.n_up[l], 16), dim3(256), 0, s, scan, pc.dev, pc.t_up[l], l);
    hipLaunchKernelGGL((k_pinv_top<NX>), dim3(pc.ninst), dim3(64), 0, s, scan, pc.dev);
    for (int l = pc.Lmax - 1; l >= 0; --l)
      hipLaunchKernelGGL((k_pinv_down<NX>), dim3(pc.n_up[l], 16), dim3(256), 0, s, scan, pc.dev, pc.t_up[l], l);
    hipLaunchKernelGGL((k_pinv_final_lanes<NX, T>), dim3(pc.n_node0, 16), dim3(256), 0, s, jsw, y, pc.dev,
                       pc.t_node0, scan, out, jout);
  }
}

template <int NX, typename T>
static void jac_class(const PinvClass& pc, const double* J, int pn, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL((k_jac_class<NX, T>), dim3(pc.n_nodes), dim3(256), 0, s, J, pn, x, y, pc.dev, pc.t_nodes);
}


template <typename T>
hipError_t precond_inverse(birk_plan* p, int jac_kind, const double* J, const T* y, T* out, T* jout,
                           hipStream_t s, int* flag, int cached) {
  // n_x <= 8: K_k formed from J and factored inside the scan kernels (pivot checks into
  // the plan's flag), or, per-node J with cached = 1, the H_k that precond_prepare laid
  // out with kPrepCache; larger n_x read the H_k that precond_prepare laid out for this
  // J with kPrepLarge (checking the pivots there)
  (void)flag;
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const PinvClass& pc : p->pclass) {
    BIRK_NX_SWITCH(pc.nx, (pinv_class<NXC, T>(p, pc, J, pn, cached, y, out, jout, s)))
  }
  return hipGetLastError();
}

// P^{-T} y for the classes with n_x <= kWaveNx: the same three launches run backwards over
// the nodes with K_k^T (double only; the classes above are left to the caller).
template <int NX>
static void pinv_t_class(birk_plan* p, const PinvClass& pc, const double* J, int pn, int cached, const double* y,
                         double* out, hipStream_t s) {
  if constexpr (NX <= kWaveNx) {
    const dim3 grid(pc.n_tile), block(kTileThreads);
    const double* jsw = (const double*)p->jsw;
    if (pn && cached) {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kCachedH, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, p->flag);
    } else if (pn) {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kFlyPerNode, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, p->flag);
    } else {
      hipLaunchKernelGGL((k_tscan_reduce<NX, kFlyConst, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, p->flag);
    }
    hipLaunchKernelGGL((k_tscan_tiles<NX>), dim3(pc.ninst), dim3(tiles_threads<NX>()), 0, s, p->scan, pc.dev);
    if (pn && cached) {
      hipLaunchKernelGGL((k_tscan_apply<NX, kCachedH, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, out, nullptr);
    } else if (pn) {
      hipLaunchKernelGGL((k_tscan_apply<NX, kFlyPerNode, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, out, nullptr);
    } else {
      hipLaunchKernelGGL((k_tscan_apply<NX, kFlyConst, true, double>), grid, block, 0, s, J, jsw, y, pc.dev,
                         pc.t_tile, p->scan, out, nullptr);
    }
  } else {
    (void)p, (void)pc, (void)J, (void)pn, (void)cached, (void)y, (void)out, (void)s;
  }
}

hipError_t precond_inverse_t_wave(birk_plan* p, int jac_kind, const double* J, const double* y, double* out,
                                  hipStream_t s, int cached) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const PinvClass& pc : p->pclass) {
    if (pc.nx > kWaveNx) continue;
    BIRK_NX_SWITCH(pc.nx, (pinv_t_class<NXC>(p, pc, J, pn, cached, y, out, s)))
  }
  return hipGetLastError();
}

template <typename T>
hipError_t jac_times(birk_plan* p, int jac_kind, const double* J, const T* x, T* y, hipStream_t s) {
  const int pn = jac_kind == BIRK_J_PER_NODE ? 1 : 0;
  for (const PinvClass& pc : p->pclass) {
    BIRK_NX_SWITCH(pc.nx, (jac_class<NXC, T>(pc, J, pn, x, y, s)))
  }
  return hipGetLastError();
}

#undef BIRK_NX_SWITCH

template hipError_t jac_times<double>(birk_plan*, int, const double*, const double*, double*, hipStream_t);
template hipError_t jac_times<float>(birk_plan*, int, const double*, const float*, float*, hipStream_t);
template hipError_t precond_forward<double>(birk_plan*, int, const double*, const double*, double*, hipStream_t);
template hipError_t precond_forward<float>(birk_plan*, int, const double*, const float*, float*, hipStream_t);
template hipError_t precond_inverse<double>(birk_plan*, int, const double*, const double*, double*, double*,
                                            hipStream_t, int*, int);
template hipError_t precond_inverse<float>(birk_plan*, int, const double*, const float*, float*, float*,
                                           hipStream_t, int*, int);

// ------------------------------------------------------------------ Krylov BLAS-1
// Krylov BLAS-1: at most kMaxDots basis vectors per call, reductions in double.
constexpr int kMaxDots = 32;

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


// ---- segmented forms: one launch over every instance of the batch ----
// A tile is kSegChunk consecutive elements of one instance; partial results go to
// part[tile][kMaxDots + 1] and are summed per instance over its tile range in a fixed
// order.

// MAXQ >= nq bounds the per-thread accumulators (registers) at compile time.  SUB = 1
// first forms u = a - b (in T, as k_sub does) and stores it, in the same pass.
template <typename T, int MAXQ, int SUB>
__global__ __launch_bounds__(256) void k_sdots(const T* __restrict__ Q, int64_t ld, int nq, const T* u_in,
                                               const T* __restrict__ a, const T* __restrict__ b, T* u_out,
                                               SegSet sg, double* __restrict__ part) {
  const int2 t = sg.tiles[blockIdx.x];
  const int64_t base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk;
  const int64_t end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]);
  double acc[MAXQ], nrm = 0.0;
#pragma unroll
  for (int i = 0; i < MAXQ; ++i) acc[i] = 0.0;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    double ue;
    if (SUB) {
      const T d = a[e] - b[e];
      u_out[e] = d;
      ue = (double)d;
    } else {
      ue = (double)u_in[e];
    }
#pragma unroll
    for (int i = 0; i < MAXQ; ++i)
      if (i < nq) acc[i] += (double)Q[(int64_t)i * ld + e] * ue;
    nrm += ue * ue;
  }
  __shared__ double sh[256];
#pragma unroll
  for (int i = 0; i < MAXQ; ++i) {
    if (i < nq) {
      const double v = block_sum256(acc[i], sh);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + i] = v;
    }
  }
  const double v = block_sum256(nrm, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + kMaxDots] = v;
}

// Smallest accumulator bound of the Krylov kernels that covers nq basis vectors.
#define BIRK_MAXQ_SWITCH(nq, CALL)                         \
  if ((nq) <= 2) { constexpr int MQ = 2; CALL; }           \
  else if ((nq) <= 8) { constexpr int MQ = 8; CALL; }      \
  else { constexpr int MQ = kMaxDots; CALL; }

// grid = (nq + 1, instances): block (x, i) sums output x (x == nq: the norm slot) of
// instance i over its tiles into out[i * ostride + slot].
__global__ __launch_bounds__(256) void k_sreduce(const double* __restrict__ part, SegSet sg, int nq,
                                                 double* __restrict__ out, int64_t ostride) {
  __shared__ double sh[256];
  const int i = blockIdx.y;
  const int slot = (blockIdx.x < (unsigned)nq) ? (int)blockIdx.x : kMaxDots;
  const int2 r = sg.ranges[i];
  double s = 0.0;
  for (int b = r.x + threadIdx.x; b < r.y; b += blockDim.x) s += part[(int64_t)b * (kMaxDots + 1) + slot];
  const double tot = block_sum256(s, sh);
  if (threadIdx.x == 0) out[(int64_t)i * ostride + slot] = tot;
}

// u -= sum_k h[i][k] Q_k on instance i's tiles; part <- tile sums of ||u||^2 when asked,
// and with DOTS also of Q_k . u (the updated u), the first half of the next Gram-Schmidt
// pass fused into this one.
template <typename T, bool DOTS, int MAXQ>
__global__ __launch_bounds__(256) void k_saxpys(const T* __restrict__ Q, int64_t ld, int nq,
                                                const double* __restrict__ h, int64_t hstride, T* __restrict__ u,
                                                SegSet sg, double* __restrict__ part) {
  const int2 t = sg.tiles[blockIdx.x];
  __shared__ double hs[kMaxDots];
  if (threadIdx.x < kMaxDots) hs[threadIdx.x] = (int)threadIdx.x < nq ? h[(int64_t)t.x * hstride + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk;
  const int64_t end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]);
  constexpr int ND = DOTS ? MAXQ : 1;
  double acc[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) acc[i] = 0.0;
  double nrm = 0.0;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    double ue = (double)u[e];
    double qv[ND];
#pragma unroll
    for (int i = 0; i < MAXQ; ++i)
      if (i < nq) {
        const double q = (double)Q[(int64_t)i * ld + e];
        if constexpr (DOTS) qv[i] = q;
        ue -= hs[i] * q;
      }
    const T us = (T)ue;
    u[e] = us;
    const double un = (double)us;
    nrm += un * un;
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < MAXQ; ++i)
        if (i < nq) acc[i] += qv[i] * un;
    }
  }
  if (part) {
    __shared__ double sh[256];
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < MAXQ; ++i) {
        if (i < nq) {
          const double v = block_sum256(acc[i], sh);
          if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + i] = v;
        }
      }
    }
    const double v = block_sum256(nrm, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (kMaxDots + 1) + kMaxDots] = v;
  }
}

// q = u / sqrt(nrm2[i]) on instance i's tiles; a zero or non-finite norm writes zeros
// (the instance has stopped; its later basis vectors are never combined).
template <typename T>
__global__ __launch_bounds__(256) void k_snormalize(const T* __restrict__ u, const double* __restrict__ nrm2,
                                                    int64_t stride, T* __restrict__ q, SegSet sg) {
  const int2 t = sg.tiles[blockIdx.x];
  const double n2 = nrm2[(int64_t)t.x * stride];
  const double inv = (n2 > 0.0 && isfinite(n2)) ? 1.0 / sqrt(n2) : 0.0;
  const int64_t base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk;
  const int64_t end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]);
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) q[e] = (T)(inv == 0.0 ? 0.0 : (double)u[e] * inv);
}

// y = alpha[i] x on instance i's tiles
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_sscale_conv(const TI* __restrict__ x, TO* __restrict__ y,
                                                     const double* __restrict__ alpha, SegSet sg) {
  const int2 t = sg.tiles[blockIdx.x];
  const double a = alpha[t.x];
  const int64_t base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk;
  const int64_t end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]);
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) y[e] = (TO)(a == 0.0 ? 0.0 : a * (double)x[e]);
}

// x += sum_{k < cnt[i]} c[i][k] Q_k on instance i's tiles (x double, sum in double)
template <typename T>
__global__ __launch_bounds__(256) void k_scombine(const T* __restrict__ Q, int64_t ld, const double* __restrict__ c,
                                                  int64_t cstride, const int* __restrict__ cnt,
                                                  double* __restrict__ x, SegSet sg) {
  const int2 t = sg.tiles[blockIdx.x];
  const int nq = cnt[t.x];
  __shared__ double cs[kMaxDots];
  if (threadIdx.x < kMaxDots) cs[threadIdx.x] = (int)threadIdx.x < nq ? c[(int64_t)t.x * cstride + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk;
  const int64_t end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]);
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nq) acc += cs[i] * (double)Q[(int64_t)i * ld + e];
    x[e] += acc;
  }
}

// ---- GMRES scalars on the device: per instance the rotated Hessenberg columns R, the
// right-hand side g of the small least-squares problem, the Givens rotations, and
// (running, columns kept, iterations, status, tolerance, ||r||); one thread per instance.
__global__ void k_gm_init(const double* __restrict__ prm, double* __restrict__ st, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kGmStride;
  for (int k = 0; k < kGmLd; ++k) s[kGmG + k] = 0.0;
  s[kGmG] = 1.0;
  s[kGmMisc + GM_RUN] = prm[3 * i];
  s[kGmMisc + GM_ACTIVE] = prm[3 * i];
  s[kGmMisc + GM_JEND] = 0.0;
  s[kGmMisc + GM_INNER] = 0.0;
  s[kGmMisc + GM_STATUS] = 0.0;
  s[kGmMisc + GM_TOL] = prm[3 * i + 1];
  s[kGmMisc + GM_RNORM] = prm[3 * i + 2];
}

// Arnoldi column j of every running instance from the CGS2 dot products (d1 + d2 = the
// coefficients, the norm slot of d2 = ||u||^2): earlier rotations, a new rotation that
// annihilates h_{j+1,j}, the update of g; the instance stops when |g_{j+1}| <= tol, on a
// lucky breakdown, on breakdown (no column kept) or on a non-finite value.
__global__ void k_gm_column(int j, const double* __restrict__ dots, int64_t dstride, double* __restrict__ st,
                            int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kGmStride;
  double* misc = s + kGmMisc;
  if (misc[GM_RUN] == 0.0) return;
  misc[GM_INNER] += 1.0;
  const double* d1 = dots + (int64_t)i * dstride;
  const double* d2 = d1 + kGmLd;
  double* col = s + kGmR + (int64_t)j * kGmLd;
  double* cs = s + kGmCs;
  double* sn = s + kGmSn;
  double* g = s + kGmG;
  const double hn2 = d2[kMaxDots];
  const double hn = isfinite(hn2) ? sqrt(hn2 > 0.0 ? hn2 : 0.0) : NAN;
  bool finite = isfinite(hn);
  for (int k = 0; k <= j; ++k) {
    col[k] = d1[k] + d2[k];
    finite = finite && isfinite(col[k]);
  }
  if (!finite) {
    misc[GM_STATUS] = (double)BIRK_ERR_NONFINITE;
    misc[GM_RUN] = 0.0;
    misc[GM_JEND] = (double)j;
    return;
  }
  double below = hn;
  for (int k = 0; k < j; ++k) {
    const double a = cs[k] * col[k] + sn[k] * col[k + 1];
    col[k + 1] = -sn[k] * col[k] + cs[k] * col[k + 1];
    col[k] = a;
  }
  const double den = hypot(col[j], below);
  if (den == 0.0) {
    misc[GM_STATUS] = (double)BIRK_ERR_BREAKDOWN;
    misc[GM_RUN] = 0.0;
    misc[GM_JEND] = (double)j;
    return;
  }
  cs[j] = col[j] / den;
  sn[j] = below / den;
  col[j] = den;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  misc[GM_JEND] = (double)(j + 1);
  const bool lucky = hn <= 1e-14 * den;
  if (fabs(g[j + 1]) <= misc[GM_TOL] || lucky) misc[GM_RUN] = 0.0;
}

// End of a cycle: y = R^{-1} g on the kept columns, coefficients ||r|| y and their count
// for the combination chi += sum_k c_k z_k; (running, iterations, status) per instance
// into flags[3 i ...] for the host.
__global__ void k_gm_solve(double* __restrict__ st, double* __restrict__ coef, int64_t cstride, int* __restrict__ cnt,
                           double* __restrict__ flags, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kGmStride;
  const double* misc = s + kGmMisc;
  double* c = coef + (int64_t)i * cstride;
  const int k = misc[GM_ACTIVE] != 0.0 ? (int)misc[GM_JEND] : 0;
  const double* R = s + kGmR;
  const double* g = s + kGmG;
  double y[kMaxDots];
  for (int a = k - 1; a >= 0; --a) {
    double acc = g[a];
    for (int b = a + 1; b < k; ++b) acc -= R[(int64_t)b * kGmLd + a] * y[b];
    y[a] = acc / R[(int64_t)a * kGmLd + a];
  }
  for (int a = 0; a < k; ++a) c[a] = y[a] * misc[GM_RNORM];
  cnt[i] = k;
  flags[3 * i] = misc[GM_RUN];
  flags[3 * i + 1] = misc[GM_INNER];
  flags[3 * i + 2] = misc[GM_STATUS];
}

// running flag per instance into flags[i] (read by the host between chunks)
__global__ void k_gm_running(const double* __restrict__ st, double* __restrict__ flags, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  flags[i] = st[(int64_t)i * kGmStride + kGmMisc + GM_RUN];
}

// Host-side launch helpers used by the GMRES driver.
namespace kry {

template <typename T>
void sub(const T* a, const T* b, T* z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub<T>, dim3(nblocks(n, 256)), dim3(256), 0, s, a, b, z, n);
}

void residual(const double* beta, const double* x, const double* t, double* r, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, s, beta, x, t, r, n);
}


template <typename T>
void sdots(const birk_plan* p, const T* Q, int nq, const T* u, double* out, int64_t ostride, hipStream_t s) {
  const SegSet& sg = p->seg;
  BIRK_MAXQ_SWITCH(nq, hipLaunchKernelGGL((k_sdots<T, MQ, 0>), dim3(sg.ntiles), dim3(256), 0, s, Q, p->total_len, nq,
                                           u, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, sg, p->krylov_part))
  hipLaunchKernelGGL(k_sreduce, dim3(nq + 1, (unsigned)p->inst.size()), dim3(256), 0, s, p->krylov_part, sg, nq, out,
                     ostride);
}

template <typename T>
void sub_sdots(const birk_plan* p, const T* Q, int nq, const T* a, const T* b, T* u, double* out, int64_t ostride,
               hipStream_t s) {
  const SegSet& sg = p->seg;
  BIRK_MAXQ_SWITCH(nq, hipLaunchKernelGGL((k_sdots<T, MQ, 1>), dim3(sg.ntiles), dim3(256), 0, s, Q, p->total_len, nq,
                                           (const T*)nullptr, a, b, u, sg, p->krylov_part))
  hipLaunchKernelGGL(k_sreduce, dim3(nq + 1, (unsigned)p->inst.size()), dim3(256), 0, s, p->krylov_part, sg, nq, out,
                     ostride);
}

template <typename T>
void saxpys(const birk_plan* p, const T* Q, int nq, const double* h, int64_t hstride, T* u, double* nrm_out,
            hipStream_t s) {
  const SegSet& sg = p->seg;
  BIRK_MAXQ_SWITCH(nq, hipLaunchKernelGGL((k_saxpys<T, false, MQ>), dim3(sg.ntiles), dim3(256), 0, s, Q,
                                           p->total_len, nq, h, hstride, u, sg, nrm_out ? p->krylov_part : nullptr))
  if (nrm_out)
    hipLaunchKernelGGL(k_sreduce, dim3(1, (unsigned)p->inst.size()), dim3(256), 0, s, p->krylov_part, sg, 0, nrm_out,
                       hstride);
}

template <typename T>
void saxpys_dots(const birk_plan* p, const T* Q, int nq, const double* h, int64_t hstride, T* u, double* out,
                 int64_t ostride, hipStream_t s) {
  const SegSet& sg = p->seg;
  BIRK_MAXQ_SWITCH(nq, hipLaunchKernelGGL((k_saxpys<T, true, MQ>), dim3(sg.ntiles), dim3(256), 0, s, Q,
                                           p->total_len, nq, h, hstride, u, sg, p->krylov_part))
  hipLaunchKernelGGL(k_sreduce, dim3(nq + 1, (unsigned)p->inst.size()), dim3(256), 0, s, p->krylov_part, sg, nq, out,
                     ostride);
}

template <typename T>
void snormalize(const birk_plan* p, const T* u, const double* nrm2, int64_t stride, T* q, hipStream_t s) {
  hipLaunchKernelGGL(k_snormalize<T>, dim3(p->seg.ntiles), dim3(256), 0, s, u, nrm2, stride, q, p->seg);
}

template <typename TI, typename TO>
void sscale_conv(const birk_plan* p, const TI* x, TO* y, const double* alpha, hipStream_t s) {
  hipLaunchKernelGGL((k_sscale_conv<TI, TO>), dim3(p->seg.ntiles), dim3(256), 0, s, x, y, alpha, p->seg);
}

template <typename T>
void scombine(const birk_plan* p, const T* Q, const double* c, int64_t cstride, const int* cnt, double* x,
              hipStream_t s) {
  hipLaunchKernelGGL(k_scombine<T>, dim3(p->seg.ntiles), dim3(256), 0, s, Q, p->total_len, c, cstride, cnt, x,
                     p->seg);
}

void gm_init(const birk_plan* p, const double* prm, double* st, hipStream_t s) {
  const int B = (int)p->inst.size();
  hipLaunchKernelGGL(k_gm_init, dim3(nblocks(B, 64)), dim3(64), 0, s, prm, st, B);
}
void gm_column(const birk_plan* p, int j, const double* dots, int64_t dstride, double* st, hipStream_t s) {
  const int B = (int)p->inst.size();
  hipLaunchKernelGGL(k_gm_column, dim3(nblocks(B, 64)), dim3(64), 0, s, j, dots, dstride, st, B);
}
void gm_solve(const birk_plan* p, double* st, double* coef, int64_t cstride, int* cnt, double* flags, hipStream_t s) {
  const int B = (int)p->inst.size();
  hipLaunchKernelGGL(k_gm_solve, dim3(nblocks(B, 64)), dim3(64), 0, s, st, coef, cstride, cnt, flags, B);
}
void gm_running(const birk_plan* p, const double* st, double* flags, hipStream_t s) {
  const int B = (int)p->inst.size();
  hipLaunchKernelGGL(k_gm_running, dim3(nblocks(B, 64)), dim3(64), 0, s, st, flags, B);
}

template void sdots<double>(const birk_plan*, const double*, int, const double*, double*, int64_t, hipStream_t);
template void sdots<float>(const birk_plan*, const float*, int, const float*, double*, int64_t, hipStream_t);
template void sub_sdots<double>(const birk_plan*, const double*, int, const double*, const double*, double*, double*,
                                int64_t, hipStream_t);
template void sub_sdots<float>(const birk_plan*, const float*, int, const float*, const float*, float*, double*,
                               int64_t, hipStream_t);
template void saxpys_dots<double>(const birk_plan*, const double*, int, const double*, int64_t, double*, double*,
                                  int64_t, hipStream_t);
template void saxpys_dots<float>(const birk_plan*, const float*, int, const double*, int64_t, float*, double*,
                                 int64_t, hipStream_t);
template void saxpys<double>(const birk_plan*, const double*, int, const double*, int64_t, double*, double*,
                             hipStream_t);
template void saxpys<float>(const birk_plan*, const float*, int, const double*, int64_t, float*, double*,
                            hipStream_t);
template void snormalize<double>(const birk_plan*, const double*, const double*, int64_t, double*, hipStream_t);
template void snormalize<float>(const birk_plan*, const float*, const double*, int64_t, float*, hipStream_t);
template void sscale_conv<double, double>(const birk_plan*, const double*, double*, const double*, hipStream_t);
template void sscale_conv<double, float>(const birk_plan*, const double*, float*, const double*, hipStream_t);
template void scombine<double>(const birk_plan*, const double*, const double*, int64_t, const int*, double*,
                               hipStream_t);
template void scombine<float>(const birk_plan*, const float*, const double*, int64_t, const int*, double*,
                              hipStream_t);

template void sub<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void sub<float>(const float*, const float*, float*, int64_t, hipStream_t);
}  // namespace kry
}  // namespace birk
