// The symmetric saddle-point (KKT) form of the collocated system and its MINRES solve.
//
// The paper counts matrix-free KKT solves per SQP step (Table 1, orbit-transfer results)
// without writing the system down.  Here: the equality-constrained quadratic model
//     min 1/2 (chi - chi_r)^T H (chi - chi_r)  s.t.  A chi = g,   A = I - (I (x) B^a) J
// (eq:Newton-ivp), H = diag(h) > 0, whose optimality conditions are
//     K [chi; lambda] = [f; g],   K = [[H, A^T], [A, 0]],   f = H chi_r,
// symmetric and indefinite.  MINRES (Paige-Saunders) with the symmetric positive definite
// block preconditioner M = blockdiag(H, P H^{-1} P^T), P = I - B~^a J the Birkhoff
// preconditioner (B~^a section) standing in for A in the Schur complement A H^{-1} A^T:
//     M^{-1} [r1; r2] = [r1 / h; P^{-T} (h * P^{-1} r2)].
//
// P^{-T}: P^T is block upper triangular in node order; row j of P^T x = y reads
//     (I - w_j J_j^T / 2) x_j - w_j J_j^T T_j = y_j,   T_j = sum_{k>j} x_k,
// i.e. with G_j = H_j^T, H_j = w_j (I - w_j J_j / 2)^{-1} J_j (the matrix of the forward
// substitution),
//     x_j = y_j + G_j (y_j / 2 + T_j),   T_{j-1} = T_j + x_j
//         = (I + G_j) T_j + (I + G_j / 2) y_j,
// an affine recurrence run from the last node down.  It is evaluated as a scan of affine
// maps: each thread composes the maps of a chunk of kBtChunk consecutive nodes, a
// one-wave block combines its 64 chunk maps into a block map, one wave per instance
// carries the state across the blocks from the last one down, and each block replays
// its chunks from their entry states.  H_j is formed from J in every pass (no stored
// preparation).  All arithmetic in double.
//
// MINRES keeps its scalar recurrences (the Lanczos coefficients, the Givens rotations and
// the step lengths) per instance in device memory, updated by one-thread-per-instance
// kernels between the vector passes, so an iteration enqueues no host work; the host
// reads the per-instance states once per chunk of iterations to test convergence.

#include <hip/hip_runtime.h>

#include <cmath>

#include "birk_internal.h"

namespace birk {
namespace kkt {

constexpr int kBtChunk = 16;
constexpr int kBtThreads = 64;
constexpr int64_t kBtNodes = (int64_t)kBtChunk * kBtThreads;

// ------------------------------------------------------------------ per-node matrices
template <int NX>
__device__ __forceinline__ void node_jac(const BtDesc& d, const double* __restrict__ J, int per_node, int64_t k,
                                         double (&Jk)[NX][NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c)
      Jk[r][c] = per_node ? J[d.joff + (int64_t)(r * NX + c) * d.Nn + k] : J[d.jcoff + r * NX + c];
}

// G_k = H_k^T, H_k = w_k K^{-1} J_k, K = I - (w_k / 2) J_k (unpivoted LU: K is strongly
// diagonally dominant for w_k <= ~pi/N; the solve's forward preparation checks pivots).
template <int NX>
__device__ __forceinline__ void node_g(const double (&Jk)[NX][NX], double wk, double (&G)[NX][NX]) {
  double K[NX][NX], rp[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) K[r][c] = (r == c ? 1.0 : 0.0) - 0.5 * wk * Jk[r][c];
#pragma unroll
  for (int p = 0; p < NX; ++p) {
    rp[p] = 1.0 / K[p][p];
#pragma unroll
    for (int i = p + 1; i < NX; ++i) {
      const double f = K[i][p] * rp[p];
      K[i][p] = f;
#pragma unroll
      for (int j = p + 1; j < NX; ++j) K[i][j] -= f * K[p][j];
    }
  }
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    double x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) x[r] = wk * Jk[r][c];
#pragma unroll
    for (int i = 1; i < NX; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) x[i] -= K[i][j] * x[j];
#pragma unroll
    for (int i = NX - 1; i >= 0; --i) {
#pragma unroll
      for (int j = i + 1; j < NX; ++j) x[i] -= K[i][j] * x[j];
      x[i] *= rp[i];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) G[c][r] = x[r];   // column c of H is row c of G
  }
}

// ------------------------------------------------------------------ P^{-T}: chunk maps
// Map of the chunk [k0, k1): T_out = A T_in + c, with T_in the state after node k1 - 1
// and T_out the state after node k0 (i.e. T_{k0 - 1}); the nodes are applied from the
// last one down, each as T -> (I + G_k) T + (I + G_k / 2) y_k.
template <int NX>
__device__ __forceinline__ void chunk_map(const BtDesc& d, const double* __restrict__ J, int per_node,
                                          const double* __restrict__ y, int64_t k0, int64_t k1,
                                          double (&A)[NX][NX], double (&c)[NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    c[r] = 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) A[r][q] = (r == q) ? 1.0 : 0.0;
  }
  for (int64_t k = k1 - 1; k >= k0; --k) {
    double Jk[NX][NX], G[NX][NX], yk[NX];
    node_jac<NX>(d, J, per_node, k, Jk);
    node_g<NX>(Jk, d.w[k], G);
#pragma unroll
    for (int r = 0; r < NX; ++r) yk[r] = y[d.off + (int64_t)r * d.Nn + k];
    double An[NX][NX], cn[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double s = c[r], dy = yk[r];
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        s += G[r][q] * c[q];
        dy += 0.5 * G[r][q] * yk[q];
      }
      cn[r] = s + dy;
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        double a = A[r][q];
#pragma unroll
        for (int m = 0; m < NX; ++m) a += G[r][m] * A[m][q];
        An[r][q] = a;
      }
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      c[r] = cn[r];
#pragma unroll
      for (int q = 0; q < NX; ++q) A[r][q] = An[r][q];
    }
  }
}

template <int NX>
constexpr int map_len() { return NX * NX + NX; }

// tile = (descriptor, block): chunk maps of the block's 64 threads combined into the block
// map (thread t holds nodes [k0 + 16 t, k0 + 16 t + 16); the block map is
// map_0 o map_1 o ... o map_63, thread 63 applied first).
template <int NX>
__global__ __launch_bounds__(kBtThreads) void k_bt_reduce(const double* __restrict__ J, int per_node,
                                                          const double* __restrict__ y, double* __restrict__ scr,
                                                          const BtDesc* __restrict__ dd,
                                                          const int2* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);   // [64][map_len]
  constexpr int ML = map_len<NX>();
  const int2 tile = tiles[blockIdx.x];
  const BtDesc& d = dd[tile.x];
  const int t = (int)threadIdx.x;
  const int64_t k0 = (int64_t)tile.y * kBtNodes + (int64_t)t * kBtChunk;
  const int64_t k1 = min(k0 + kBtChunk, d.Nn);
  double A[NX][NX], c[NX];
  chunk_map<NX>(d, J, per_node, y, k0, k1 > k0 ? k1 : k0, A, c);
  double* mine = sm + t * ML;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
#pragma unroll
    for (int q = 0; q < NX; ++q) mine[r * NX + q] = A[r][q];
    mine[NX * NX + r] = c[r];
  }
  __syncthreads();
  for (int s = 1; s < kBtThreads; s <<= 1) {
    if ((t & (2 * s - 1)) == 0) {
      // (A_t, c_t) o (A_{t+s}, c_{t+s}) = (A_t A_{t+s}, A_t c_{t+s} + c_t)
      const double* hi = sm + (t + s) * ML;
      double An[NX][NX], cn[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double cc = mine[NX * NX + r];
#pragma unroll
        for (int q = 0; q < NX; ++q) {
          double a = 0.0;
#pragma unroll
          for (int m = 0; m < NX; ++m) a += mine[r * NX + m] * hi[m * NX + q];
          An[r][q] = a;
          cc += mine[r * NX + q] * hi[NX * NX + q];
        }
        cn[r] = cc;
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) {
#pragma unroll
        for (int q = 0; q < NX; ++q) mine[r * NX + q] = An[r][q];
        mine[NX * NX + r] = cn[r];
      }
    }
    __syncthreads();
  }
  double* out = scr + d.soff + (int64_t)tile.y * ML;
  for (int e = t; e < ML; e += kBtThreads) out[e] = sm[e];
}

// One wave per instance: entry states of the blocks, from the last block down
// (T = 0 after node N); lane r < NX holds component r of the state.
template <int NX>
__global__ __launch_bounds__(kBtThreads) void k_bt_top(double* __restrict__ scr, const BtDesc* __restrict__ dd) {
  constexpr int ML = map_len<NX>();
  const BtDesc& d = dd[blockIdx.x];
  const int lane = (int)threadIdx.x;
  const double* maps = scr + d.soff;
  double* tin = scr + d.soff + d.nblk * ML;
  double T = 0.0;
  for (int64_t b = d.nblk - 1; b >= 0; --b) {
    if (lane < NX) tin[b * NX + lane] = T;
    const double* m = maps + b * ML;
    double s = lane < NX ? m[NX * NX + lane] : 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const double tq = __shfl(T, q, 64);
      if (lane < NX) s += m[lane * NX + q] * tq;
    }
    T = s;
  }
}

// tile = (descriptor, block): entry state of every chunk from the block's entry state,
// then each chunk replayed from its last node down: x_k = y_k + G_k (y_k / 2 + T),
// T += x_k.
template <int NX>
__global__ __launch_bounds__(kBtThreads) void k_bt_apply(const double* __restrict__ J, int per_node,
                                                         const double* __restrict__ y, double* __restrict__ x,
                                                         const double* __restrict__ scr,
                                                         const BtDesc* __restrict__ dd,
                                                         const int2* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);   // [64][map_len], then [64][NX] entry states
  constexpr int ML = map_len<NX>();
  const int2 tile = tiles[blockIdx.x];
  const BtDesc& d = dd[tile.x];
  const int t = (int)threadIdx.x;
  const int64_t k0 = (int64_t)tile.y * kBtNodes + (int64_t)t * kBtChunk;
  const int64_t k1 = min(k0 + kBtChunk, d.Nn);
  {
    double A[NX][NX], c[NX];
    chunk_map<NX>(d, J, per_node, y, k0, k1 > k0 ? k1 : k0, A, c);
    double* mine = sm + t * ML;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
#pragma unroll
      for (int q = 0; q < NX; ++q) mine[r * NX + q] = A[r][q];
      mine[NX * NX + r] = c[r];
    }
  }
  double* tst = sm + kBtThreads * ML;
  __syncthreads();
  // entry states: thread 63 enters with the block's state; thread s - 1 with map_s(T_s)
  double T = t < NX ? scr[d.soff + d.nblk * ML + (int64_t)tile.y * NX + t] : 0.0;
  for (int s = kBtThreads - 1; s >= 0; --s) {
    if (t < NX) tst[s * NX + t] = T;
    if (s == 0) break;
    const double* m = sm + s * ML;
    double v = t < NX ? m[NX * NX + t] : 0.0;
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      const double tq = __shfl(T, q, 64);
      if (t < NX) v += m[t * NX + q] * tq;
    }
    T = v;
  }
  __syncthreads();
  double Tv[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) Tv[r] = tst[t * NX + r];
  for (int64_t k = k1 - 1; k >= k0; --k) {
    double Jk[NX][NX], G[NX][NX], yk[NX], u[NX];
    node_jac<NX>(d, J, per_node, k, Jk);
    node_g<NX>(Jk, d.w[k], G);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      yk[r] = y[d.off + (int64_t)r * d.Nn + k];
      u[r] = 0.5 * yk[r] + Tv[r];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double v = yk[r];
#pragma unroll
      for (int q = 0; q < NX; ++q) v += G[r][q] * u[q];
      x[d.off + (int64_t)r * d.Nn + k] = v;
      Tv[r] += v;
    }
  }
}

// ------------------------------------------------------------------ J^T x per node
template <int NX>
__global__ __launch_bounds__(256) void k_jac_t(const double* __restrict__ J, int per_node,
                                               const double* __restrict__ x, double* __restrict__ yv,
                                               const BtDesc* __restrict__ dd, const int2* __restrict__ tiles) {
  const int2 tile = tiles[blockIdx.x];
  const BtDesc& d = dd[tile.x];
  const int64_t k = (int64_t)tile.y * 256 + threadIdx.x;
  if (k >= d.Nn) return;
  double xv[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) xv[r] = x[d.off + (int64_t)r * d.Nn + k];
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      const double j = per_node ? J[d.joff + (int64_t)(r * NX + c) * d.Nn + k] : J[d.jcoff + r * NX + c];
      acc += j * xv[r];
    }
    yv[d.off + (int64_t)c * d.Nn + k] = acc;
  }
}

// ------------------------------------------------------------------ segmented vector passes
// The KKT vectors are pairs [top (n); bottom (n)]; a launch covers both halves: block b
// of 2 ntiles works half b / ntiles on the plan's segment tile b % ntiles.
struct Seg {
  const int2* tiles;
  const int64_t* ioff;
  const int64_t* ilen;
  int ntiles;
  int64_t n;
};

__device__ __forceinline__ void seg_range(const Seg& sg, int blk, int* inst, int64_t* base, int64_t* end) {
  const int half = blk >= sg.ntiles;
  const int2 t = sg.tiles[blk - half * sg.ntiles];
  *inst = t.x;
  *base = sg.ioff[t.x] + (int64_t)t.y * kSegChunk + half * sg.n;
  *end = sg.ioff[t.x] + min((int64_t)(t.y + 1) * kSegChunk, sg.ilen[t.x]) + half * sg.n;
}

__device__ __forceinline__ double wave_block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

// Per-instance state of MINRES (doubles, kSt per instance).
enum {
  S_BETA1, S_BETA, S_OLDB, S_ALPHA, S_DBAR, S_EPS, S_PHIBAR, S_CS, S_SN, S_ACTIVE, S_SV, S_C1, S_C2, S_AV,
  S_A1, S_A2, S_PHI, S_THR, S_ITERS, S_IT0, kSt
};

// z = a[i] x + b[i] y (+ c[i] z when ADDZ) on both halves; DOT: per-tile partial of q . z
// (x and z may be the same vector.)  ia / ib / ic: state slot of the coefficient, -1 for
// 1 (a) or 0 (b, c); a negative slot - 2 - k takes minus the coefficient in slot k.
template <bool ADDZ, bool DOT>
__global__ __launch_bounds__(256) void k_kv_lin(const double* x, const double* __restrict__ yv, double* z,
                                                const double* __restrict__ st, int ia, int ib, int ic,
                                                const double* __restrict__ q, double* __restrict__ part, Seg sg) {
  int inst;
  int64_t base, end;
  seg_range(sg, blockIdx.x, &inst, &base, &end);
  const double* s = st + (int64_t)inst * kSt;
  auto coef = [s](int slot, double dflt) { return slot >= 0 ? s[slot] : slot <= -2 ? -s[-2 - slot] : dflt; };
  const double a = coef(ia, 1.0), b = coef(ib, 0.0), c = coef(ic, 0.0);
  double acc = 0.0;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    double v = a * x[e];
    if (yv) v += b * yv[e];
    if (ADDZ) v += c * z[e];
    z[e] = v;
    if (DOT) acc += q[e] * v;
  }
  if (DOT) {
    __shared__ double sh[4];
    const double tot = wave_block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
  }
}

// per-tile partial of a . b over both halves
__global__ __launch_bounds__(256) void k_kv_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                double* __restrict__ part, Seg sg) {
  int inst;
  int64_t base, end;
  seg_range(sg, blockIdx.x, &inst, &base, &end);
  double acc = 0.0;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) acc += a[e] * b[e];
  __shared__ double sh[4];
  const double tot = wave_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[i] = sum of instance i's partials (both halves, tiles in order)
__global__ __launch_bounds__(64) void k_kv_reduce(const double* __restrict__ part, const int2* __restrict__ ranges,
                                                  int ntiles, double* __restrict__ out) {
  const int i = blockIdx.x;
  const int2 r = ranges[i];
  double s = 0.0;
  for (int b = r.x + (int)threadIdx.x; b < r.y; b += 64) s += part[b] + part[ntiles + b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) out[i] = s;
}

// ------------------------------------------------------------------ KKT operator pieces
// top = h * u + l - t (t = J^T B^aT l), bottom = u - s (s = B^a J u); h == null: H = I
__global__ __launch_bounds__(256) void k_kkt_combine(const double* __restrict__ u, const double* __restrict__ l,
                                                     const double* __restrict__ t, const double* __restrict__ s,
                                                     const double* __restrict__ h, double* __restrict__ top,
                                                     double* __restrict__ bot, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double hu = h ? h[e] * u[e] : u[e];
  top[e] = hu + l[e] - t[e];
  bot[e] = u[e] - s[e];
}

// z = a / h (or a), z = h * a (or a)
__global__ __launch_bounds__(256) void k_hscale(const double* __restrict__ a, const double* __restrict__ h,
                                                double* __restrict__ z, int64_t n, int divide) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  z[e] = h ? (divide ? a[e] / h[e] : a[e] * h[e]) : a[e];
}

// r = b - k (the true residual), both halves at once (length 2n)
__global__ __launch_bounds__(256) void k_sub2(const double* __restrict__ b, const double* __restrict__ k,
                                              double* __restrict__ r, int64_t n2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2) return;
  r[e] = b[e] - k[e];
}

// ------------------------------------------------------------------ MINRES scalar recurrences
// Cycle start: beta1 = sqrt(r1 . M^{-1} r1) from dot; thr = tol[i] beta1.
__global__ void k_mr_init(double* __restrict__ st, const double* __restrict__ dot, const double* __restrict__ tol,
                          const int* __restrict__ run, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kSt;
  const double b2 = dot[i];
  const double b = (b2 > 0.0 && isfinite(b2)) ? sqrt(b2) : 0.0;
  for (int k = 0; k < kSt; ++k) s[k] = 0.0;
  s[S_BETA1] = b;
  s[S_BETA] = b;
  s[S_PHIBAR] = b;
  s[S_CS] = -1.0;
  s[S_THR] = tol[i] * b;
  s[S_ACTIVE] = (run[i] && b > 0.0) ? 1.0 : 0.0;
  s[S_IT0] = 1.0;
}

// Before an iteration: v = y / beta, and the coefficient of r1 in y = K v - (beta / oldb) r1.
__global__ void k_mr_pre(double* __restrict__ st, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kSt;
  const bool on = s[S_ACTIVE] != 0.0;
  s[S_SV] = on ? 1.0 / s[S_BETA] : 0.0;
  s[S_C1] = (on && s[S_IT0] == 0.0) ? s[S_BETA] / s[S_OLDB] : 0.0;
}

// alpha = v . y; coefficient of r2 in y -= (alpha / beta) r2.
__global__ void k_mr_alpha(double* __restrict__ st, const double* __restrict__ dot, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kSt;
  const bool on = s[S_ACTIVE] != 0.0;
  s[S_ALPHA] = on ? dot[i] : 0.0;
  s[S_C2] = on ? dot[i] / s[S_BETA] : 0.0;
}

// beta_{k+1} = sqrt(r2 . M^{-1} r2), the new Givens rotation, the step phi and the
// coefficients of w_k = (v - eps_{k-1} w_{k-2} - delta w_{k-1}) / gamma; stop when
// |phibar| <= thr, on breakdown, or on a non-finite value.
__global__ void k_mr_givens(double* __restrict__ st, const double* __restrict__ dot, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  double* s = st + (int64_t)i * kSt;
  if (s[S_ACTIVE] == 0.0) {
    s[S_PHI] = s[S_AV] = s[S_A1] = s[S_A2] = 0.0;
    return;
  }
  const double b2 = dot[i];
  const double beta = (b2 > 0.0 && isfinite(b2)) ? sqrt(b2) : (b2 == 0.0 ? 0.0 : NAN);
  const double oldeps = s[S_EPS];
  const double cs = s[S_CS], sn = s[S_SN], dbar = s[S_DBAR], alpha = s[S_ALPHA];
  const double delta = cs * dbar + sn * alpha;
  const double gbar = sn * dbar - cs * alpha;
  const double gamma = hypot(gbar, beta);
  s[S_OLDB] = s[S_BETA];
  s[S_BETA] = beta;
  s[S_EPS] = sn * beta;
  s[S_DBAR] = -cs * beta;
  s[S_IT0] = 0.0;
  s[S_ITERS] += 1.0;
  if (!(gamma > 0.0) || !isfinite(gamma)) {
    s[S_PHI] = s[S_AV] = s[S_A1] = s[S_A2] = 0.0;
    s[S_ACTIVE] = 0.0;
    if (!isfinite(gamma) || !isfinite(beta)) s[S_PHIBAR] = NAN;
    return;
  }
  const double cn = gbar / gamma, snn = beta / gamma;
  const double phi = cn * s[S_PHIBAR];
  s[S_PHIBAR] = snn * s[S_PHIBAR];
  s[S_CS] = cn;
  s[S_SN] = snn;
  s[S_PHI] = phi;
  s[S_AV] = 1.0 / gamma;
  s[S_A1] = -oldeps / gamma;
  s[S_A2] = -delta / gamma;
  if (fabs(s[S_PHIBAR]) <= s[S_THR] || beta == 0.0) s[S_ACTIVE] = 0.0;
}

// w_new = av v + a1 w1 + a2 w2 (into w1's buffer), x += phi w_new
__global__ __launch_bounds__(256) void k_mr_update(const double* __restrict__ v, double* __restrict__ w1,
                                                   const double* __restrict__ w2, double* __restrict__ x,
                                                   const double* __restrict__ st, Seg sg) {
  int inst;
  int64_t base, end;
  seg_range(sg, blockIdx.x, &inst, &base, &end);
  const double* s = st + (int64_t)inst * kSt;
  const double av = s[S_AV], a1 = s[S_A1], a2 = s[S_A2], phi = s[S_PHI];
  if (phi == 0.0 && av == 0.0) return;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    const double wn = av * v[e] + a1 * w1[e] + a2 * w2[e];
    w1[e] = wn;
    x[e] += phi * wn;
  }
}

// ------------------------------------------------------------------ host side
template <int NX>
static void bt_class(const BtClass& bc, const double* J, int per_node, const double* y, double* x, double* scr,
                     hipStream_t s) {
  constexpr int ML = map_len<NX>();
  constexpr int lds_r = kBtThreads * ML * (int)sizeof(double);
  constexpr int lds_a = lds_r + kBtThreads * NX * (int)sizeof(double);
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_bt_reduce<NX>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_a);
    (void)hipFuncSetAttribute((const void*)k_bt_apply<NX>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_a);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(k_bt_reduce<NX>, dim3(bc.nblk), dim3(kBtThreads), lds_r, s, J, per_node, y, scr, bc.dev,
                     bc.tiles);
  hipLaunchKernelGGL(k_bt_top<NX>, dim3(bc.ninst), dim3(kBtThreads), 0, s, scr, bc.dev);
  hipLaunchKernelGGL(k_bt_apply<NX>, dim3(bc.nblk), dim3(kBtThreads), lds_a, s, J, per_node, y, x, scr, bc.dev,
                     bc.tiles);
}

template <int NX>
static void jt_class(const BtClass& bc, const double* J, int per_node, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_jac_t<NX>, dim3(bc.nnode), dim3(256), 0, s, J, per_node, x, y, bc.dev, bc.ntiles256);
}

#define BIRK_NX_SWITCH(nx, CALL)                                      \
  switch (nx) {                                                       \
    case 1: { constexpr int NX = 1; CALL; } break;                    \
    case 2: { constexpr int NX = 2; CALL; } break;                    \
    case 3: { constexpr int NX = 3; CALL; } break;                    \
    case 4: { constexpr int NX = 4; CALL; } break;                    \
    case 5: { constexpr int NX = 5; CALL; } break;                    \
    case 6: { constexpr int NX = 6; CALL; } break;                    \
    case 7: { constexpr int NX = 7; CALL; } break;                    \
    case 8: { constexpr int NX = 8; CALL; } break;                    \
    case 9: { constexpr int NX = 9; CALL; } break;                    \
    case 10: { constexpr int NX = 10; CALL; } break;                  \
    case 11: { constexpr int NX = 11; CALL; } break;                  \
    default: { constexpr int NX = 12; CALL; } break;                  \
  }

}  // namespace kkt

using namespace kkt;

hipError_t plan_kkt(birk_plan* p) {
  // classes by n_x; descriptors, block and node tile lists; scan scratch offsets
  // (the KKT preconditioner covers n_x <= 12; instances with more states get no class)
  std::vector<std::vector<int>> by(13);
  for (int i = 0; i < (int)p->inst.size(); ++i)
    if (p->inst[i].nx <= 12) by[p->inst[i].nx].push_back(i);
  int64_t soff = 0;
  hipError_t e = hipSuccess;
  for (int nx = 1; nx <= 12 && e == hipSuccess; ++nx) {
    if (by[nx].empty()) continue;
    BtClass bc;
    bc.nx = nx;
    bc.ninst = (int)by[nx].size();
    std::vector<BtDesc> h;
    std::vector<int2> tb, tn;
    for (int k = 0; k < bc.ninst; ++k) {
      const Instance& in = p->inst[by[nx][k]];
      BtDesc d;
      d.Nn = in.Nn;
      d.off = in.off;
      d.joff = in.joff;
      d.jcoff = in.jcoff;
      d.w = in.w;
      d.nblk = (in.Nn + kBtNodes - 1) / kBtNodes;
      d.soff = soff;
      soff += d.nblk * (int64_t)(nx * nx + nx) + d.nblk * nx;
      for (int64_t b = 0; b < d.nblk; ++b) tb.push_back(make_int2(k, (int)b));
      for (int64_t b = 0; b < (in.Nn + 255) / 256; ++b) tn.push_back(make_int2(k, (int)b));
      h.push_back(d);
    }
    bc.nblk = (int)tb.size();
    bc.nnode = (int)tn.size();
    e = hipMalloc((void**)&bc.dev, h.size() * sizeof(BtDesc));
    if (e == hipSuccess) p->allocs.push_back(bc.dev);
    if (e == hipSuccess) e = hipMemcpy(bc.dev, h.data(), h.size() * sizeof(BtDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&bc.tiles, tb.size() * sizeof(int2));
    if (e == hipSuccess) p->allocs.push_back(bc.tiles);
    if (e == hipSuccess) e = hipMemcpy(bc.tiles, tb.data(), tb.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&bc.ntiles256, tn.size() * sizeof(int2));
    if (e == hipSuccess) p->allocs.push_back(bc.ntiles256);
    if (e == hipSuccess) e = hipMemcpy(bc.ntiles256, tn.data(), tn.size() * sizeof(int2), hipMemcpyHostToDevice);
    p->btclass.push_back(bc);
  }
  p->total_bt = std::max<int64_t>(soff, 1);
  if (e == hipSuccess) e = hipMalloc((void**)&p->bt_scr, p->total_bt * sizeof(double));
  if (e == hipSuccess) p->allocs.push_back(p->bt_scr);
  return e;
}

hipError_t precond_inverse_t(birk_plan* p, int jac_kind, const double* J, const double* y, double* x, double* scr,
                             hipStream_t s, int cached) {
  // n_x <= 8: the backward wave scan of birk_solve.hip; larger n_x: the chunked scan here
  hipError_t e = precond_inverse_t_wave(p, jac_kind, J, y, x, s, cached);
  if (e != hipSuccess) return e;
  for (const BtClass& bc : p->btclass) {
    if (bc.nx <= 8) continue;
    BIRK_NX_SWITCH(bc.nx, (bt_class<NX>(bc, J, jac_kind == BIRK_J_PER_NODE, y, x, scr, s)))
  }
  return hipGetLastError();
}

hipError_t jac_t_times(birk_plan* p, int jac_kind, const double* J, const double* x, double* y, hipStream_t s) {
  for (const BtClass& bc : p->btclass) {
    BIRK_NX_SWITCH(bc.nx, (jt_class<NX>(bc, J, jac_kind == BIRK_J_PER_NODE, x, y, s)))
  }
  return hipGetLastError();
}

#undef BIRK_NX_SWITCH

// ------------------------------------------------------------------ the MINRES driver
namespace {

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

struct KktBufs {
  double *x, *v, *y, *r1, *r2, *w, *w1, *rhs, *tmp;   // pair vectors (2n each)
  double *st, *part, *dot, *tol;
  int* run;
};

Seg make_seg(const birk_plan* p) {
  Seg sg;
  sg.tiles = p->seg.tiles;
  sg.ioff = p->seg.ioff;
  sg.ilen = p->seg.ilen;
  sg.ntiles = p->seg.ntiles;
  sg.n = p->total_len;
  return sg;
}

}  // namespace

hipError_t ensure_kkt(birk_plan* p) {
  if (p->kkt_buf) return hipSuccess;
  const size_t n = (size_t)p->total_len, B = p->inst.size();
  const size_t nt = 2 * (size_t)std::max(p->seg.ntiles, 1);
  const size_t doubles = 9 * 2 * n + B * kSt + nt + 2 * B;
  hipError_t e = hipMalloc(&p->kkt_buf, doubles * sizeof(double) + B * sizeof(int));
  return e;
}

static KktBufs kkt_bufs(birk_plan* p) {
  const int64_t n2 = 2 * p->total_len;
  const size_t B = p->inst.size();
  const size_t nt = 2 * (size_t)std::max(p->seg.ntiles, 1);
  double* q = (double*)p->kkt_buf;
  KktBufs b;
  double** vecs[] = {&b.x, &b.v, &b.y, &b.r1, &b.r2, &b.w, &b.w1, &b.rhs, &b.tmp};
  for (double** v : vecs) {
    *v = q;
    q += n2;
  }
  b.st = q;
  q += B * kSt;
  b.part = q;
  q += nt;
  b.dot = q;
  q += B;
  b.tol = q;
  q += B;
  b.run = (int*)q;
  return b;
}

// K [u; l] -> [top; bottom] (pair vectors); uses tmp_vec[0..3]
static hipError_t kkt_apply(birk_plan* p, int jk, const double* J, const double* h, const double* z, double* out,
                            hipStream_t s) {
  const int64_t n = p->total_len;
  const double* u = z;
  const double* l = z + n;
  double* t0 = (double*)p->tmp_vec[0];
  double* t1 = (double*)p->tmp_vec[1];
  double* t2 = (double*)p->tmp_vec[2];
  double* t3 = (double*)p->tmp_vec[3];
  hipError_t e = jac_times<double>(p, jk, J, u, t0, s);                 // J u
  if (e == hipSuccess) e = apply_product<double>(p, t0, t1, 0, s);       // B^a J u
  if (e == hipSuccess) e = apply_product<double>(p, l, t2, 1, s);        // B^aT l
  if (e == hipSuccess) e = jac_t_times(p, jk, J, t2, t3, s);             // J^T B^aT l
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kkt_combine, dim3(nb256(n)), dim3(256), 0, s, u, l, t3, t1, h, out, out + n, n);
  return hipGetLastError();
}

// M^{-1} [r1; r2] = [r1 / h; P^{-T}(h * P^{-1} r2)] (P^{-1} prepared for J)
static hipError_t kkt_prec(birk_plan* p, int jk, const double* J, const double* h, const double* r, double* z,
                           double* scr, int use_precond, int cached, hipStream_t s) {
  const int64_t n = p->total_len;
  if (!use_precond) return hipMemcpyAsync(z, r, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s);
  hipLaunchKernelGGL(k_hscale, dim3(nb256(n)), dim3(256), 0, s, r, h, z, n, 1);
  double* t0 = (double*)p->tmp_vec[0];
  hipError_t e = precond_inverse<double>(p, jk, J, r + n, t0, nullptr, s, nullptr, cached);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hscale, dim3(nb256(n)), dim3(256), 0, s, t0, h, t0, n, 0);
  return precond_inverse_t(p, jk, J, t0, z + n, scr, s, cached);
}

// MINRES on the KKT system for every instance of the batch (arguments checked by the
// caller): restarted on the true residual [f; g] - K [chi; lambda] in double until
// ||r|| <= rtol ||[f; g]|| per instance; each cycle runs MINRES on K d = r (the
// correction accumulates into the iterate) to a preconditioned-residual tolerance.
birk_status kkt_solve(birk_plan* p, int jk, const double* J, const double* h, const double* f, const double* g,
                      double* chi, double* lam, const birk_solve_opts* o, birk_solve_info* info) {
  const int B = (int)p->inst.size();
  const int64_t n = p->total_len;
  hipStream_t s = p->stream;
  hipError_t e = ensure_kkt(p);
  if (e == hipSuccess) e = (p->krylov_part ? hipSuccess : hipMalloc(&p->krylov_part, sizeof(double)));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? BIRK_ERR_NOMEM : BIRK_ERR_DEVICE;
  KktBufs b = kkt_bufs(p);
  const Seg sg = make_seg(p);
  const unsigned nt2 = 2u * (unsigned)sg.ntiles;
  const unsigned ib = (unsigned)((B + 63) / 64);
  // rhs = [f; g]; x = [chi; lam] (zero unless use_x0)
  if (f) e = hipMemcpyAsync(b.rhs, f, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  else e = hipMemsetAsync(b.rhs, 0, n * sizeof(double), s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.rhs + n, g, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && o->use_x0) {
    e = hipMemcpyAsync(b.x, chi, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b.x + n, lam, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  } else if (e == hipSuccess) {
    e = hipMemsetAsync(b.x, 0, 2 * n * sizeof(double), s);
  }
  if (e == hipSuccess && o->use_precond) e = precond_prepare(p, jk, J, 0, s, kPrepLarge);
  if (e != hipSuccess) return BIRK_ERR_DEVICE;
  // the first preconditioner application forms K_k on the fly; per-node H_k are cached
  // before the second
  int napp = 0;
  auto prec = [&](const double* r, double* z) -> hipError_t {
    if (o->use_precond && napp == 1) {
      const hipError_t ee = precond_prepare(p, jk, J, 0, s, kPrepCache);
      if (ee != hipSuccess) return ee;
    }
    const int cached = napp >= 1 ? 1 : 0;
    ++napp;
    return kkt_prec(p, jk, J, h, r, z, p->bt_scr, o->use_precond, cached, s);
  };
  std::vector<double> hst((size_t)B * kSt), bn(B), rn(B), tolv(B);
  std::vector<int> run(B, 1), status(B, BIRK_OK), inner(B, 0), outer(B, 0);
  std::vector<char> done(B, 0);
  auto norms = [&](const double* vec, std::vector<double>& out) -> hipError_t {
    hipLaunchKernelGGL(k_kv_dot, dim3(nt2), dim3(256), 0, s, vec, vec, b.part, sg);
    hipLaunchKernelGGL(k_kv_reduce, dim3(B), dim3(64), 0, s, b.part, p->seg.ranges, sg.ntiles, b.dot);
    hipError_t ee = hipMemcpyAsync(hst.data(), b.dot, B * sizeof(double), hipMemcpyDeviceToHost, s);
    if (ee == hipSuccess) ee = hipStreamSynchronize(s);
    for (int i = 0; i < B; ++i) out[i] = std::isfinite(hst[i]) ? std::sqrt(std::max(hst[i], 0.0)) : NAN;
    return ee;
  };
  if (norms(b.rhs, bn) != hipSuccess) return BIRK_ERR_DEVICE;
  int budget = o->max_iter;
  // iterations between host reads of the convergence state: 2, 2, 4, then 8 per cycle
  // (the preconditioned counts are small, and an iteration past convergence costs a
  // whole operator and preconditioner application)
  constexpr int kChunkIts = 8;
  birk_status result = BIRK_OK;
  for (int cycle = 0;; ++cycle) {
    // true residual r = rhs - K x in double
    e = kkt_apply(p, jk, J, h, b.x, b.tmp, s);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
    hipLaunchKernelGGL(k_sub2, dim3(nb256(2 * n)), dim3(256), 0, s, b.rhs, b.tmp, b.r1, 2 * n);
    if (norms(b.r1, rn) != hipSuccess) return BIRK_ERR_DEVICE;
    bool all = true;
    for (int i = 0; i < B; ++i) {
      run[i] = 0;
      if (done[i]) continue;
      if (!std::isfinite(rn[i])) {
        status[i] = BIRK_ERR_NONFINITE;
        done[i] = 1;
      } else if (rn[i] <= o->rtol * bn[i]) {
        status[i] = BIRK_OK;
        done[i] = 1;
      } else if (budget <= 0 || cycle > o->max_iter) {
        status[i] = BIRK_ERR_NOCONV;
        done[i] = 1;
      } else {
        run[i] = 1;
        all = false;
        outer[i] += 1;
        tolv[i] = std::min(0.5, 0.1 * o->rtol * bn[i] / rn[i]);
      }
    }
    if (all) break;
    // cycle start: r2 = r1, y = M^{-1} r1, beta1; w = w2 = 0
    e = hipMemcpyAsync(b.r2, b.r1, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(b.w, 0, 2 * n * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(b.w1, 0, 2 * n * sizeof(double), s);
    if (e == hipSuccess) e = hipMemcpyAsync(b.tol, tolv.data(), B * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b.run, run.data(), B * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = prec(b.r1, b.y);
    if (e != hipSuccess) return BIRK_ERR_DEVICE;
    hipLaunchKernelGGL(k_kv_dot, dim3(nt2), dim3(256), 0, s, b.r1, b.y, b.part, sg);
    hipLaunchKernelGGL(k_kv_reduce, dim3(B), dim3(64), 0, s, b.part, p->seg.ranges, sg.ntiles, b.dot);
    hipLaunchKernelGGL(k_mr_init, dim3(ib), dim3(64), 0, s, b.st, b.dot, b.tol, b.run, B);
    // w: w_{k-1}, w1: w_{k-2}
    double *r1 = b.r1, *r2 = b.r2, *y = b.y, *w = b.w, *w1 = b.w1;
    bool cycle_done = false;
    int chunk_no = 0;
    while (!cycle_done && budget > 0) {
      const int want = chunk_no < 2 ? 2 : chunk_no < 3 ? 4 : kChunkIts;
      ++chunk_no;
      const int its = std::min(want, budget);
      for (int k = 0; k < its; ++k) {
        hipLaunchKernelGGL(k_mr_pre, dim3(ib), dim3(64), 0, s, b.st, B);
        // v = y / beta
        hipLaunchKernelGGL((k_kv_lin<false, false>), dim3(nt2), dim3(256), 0, s, y, (const double*)nullptr, b.v,
                           b.st, (int)S_SV, -1, -1, (const double*)nullptr, (double*)nullptr, sg);
        // y = K v - (beta / oldb) r1; alpha = v . y
        if (kkt_apply(p, jk, J, h, b.v, y, s) != hipSuccess) return BIRK_ERR_DEVICE;
        hipLaunchKernelGGL((k_kv_lin<false, true>), dim3(nt2), dim3(256), 0, s, y, r1, y, b.st, -1, -2 - S_C1, -1,
                           b.v, b.part, sg);
        hipLaunchKernelGGL(k_kv_reduce, dim3(B), dim3(64), 0, s, b.part, p->seg.ranges, sg.ntiles, b.dot);
        hipLaunchKernelGGL(k_mr_alpha, dim3(ib), dim3(64), 0, s, b.st, b.dot, B);
        // y -= (alpha / beta) r2; then r1 <- r2, r2 <- y
        hipLaunchKernelGGL((k_kv_lin<false, false>), dim3(nt2), dim3(256), 0, s, y, r2, y, b.st, -1, -2 - S_C2, -1,
                           (const double*)nullptr, (double*)nullptr, sg);
        double* t = r1;
        r1 = r2;
        r2 = y;
        y = t;
        // y = M^{-1} r2; beta = sqrt(r2 . y)
        if (prec(r2, y) != hipSuccess) return BIRK_ERR_DEVICE;
        hipLaunchKernelGGL(k_kv_dot, dim3(nt2), dim3(256), 0, s, r2, y, b.part, sg);
        hipLaunchKernelGGL(k_kv_reduce, dim3(B), dim3(64), 0, s, b.part, p->seg.ranges, sg.ntiles, b.dot);
        hipLaunchKernelGGL(k_mr_givens, dim3(ib), dim3(64), 0, s, b.st, b.dot, B);
        // w_new = (v - eps w1 - delta w2) / gamma into w1's buffer; x += phi w_new
        hipLaunchKernelGGL(k_mr_update, dim3(nt2), dim3(256), 0, s, b.v, w1, w, b.x, b.st, sg);
        double* wn = w1;
        w1 = w;
        w = wn;
      }
      budget -= its;
      e = hipMemcpyAsync(hst.data(), b.st, hst.size() * sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return BIRK_ERR_DEVICE;
      cycle_done = true;
      for (int i = 0; i < B; ++i)
        if (run[i] && hst[(size_t)i * kSt + S_ACTIVE] != 0.0) cycle_done = false;
    }
    for (int i = 0; i < B; ++i) {
      if (!run[i]) continue;
      inner[i] += (int)hst[(size_t)i * kSt + S_ITERS];
      if (!std::isfinite(hst[(size_t)i * kSt + S_PHIBAR])) {
        status[i] = BIRK_ERR_NONFINITE;
        done[i] = 1;
      }
    }
  }
  e = hipMemcpyAsync(chi, b.x, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && lam) e = hipMemcpyAsync(lam, b.x + n, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return BIRK_ERR_DEVICE;
  for (int i = 0; i < B; ++i) {
    if (result == BIRK_OK && status[i] != BIRK_OK) result = (birk_status)status[i];
    if (info) {
      if (info->status) info->status[i] = status[i];
      if (info->inner_iters) info->inner_iters[i] = inner[i];
      if (info->outer_iters) info->outer_iters[i] = outer[i];
      if (info->rel_resid_fp64) info->rel_resid_fp64[i] = bn[i] > 0 ? rn[i] / bn[i] : rn[i];
    }
  }
  return result;
}

}  // namespace birk
