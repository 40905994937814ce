// Fast Birkhoff products B^a v and B^aT g on the CGL grid (gfx950): the general path,
// for any N, batched over every pair of components of every instance of a plan.
//
// FastBV (arXiv 2509.01855, FastBV box) applies Fastv2a, the integration recurrence
// with the T_{N+1} alias (eq:c_k=bydef, eq:chatk=) and Fasta2v.  Writing C for the
// DCT-I of eq:vm=DCT-1, R for index reversal, E = diag(1/2, 1, ..., 1, 1/2) and
// S = diag((-1)^k), Fastv2a is E (2/N) C R and Fasta2v is R C E^{-1}.  Because
// C R = S C and R C = C S, the reversals become sign flips in coefficient space:
//
//     B^a  = (2/N) C [E^{-1} S M S E] C          (M: a -> c^, the recurrence)
//     B^aT = (2/N) E C [S M^T S] C E^{-1}        (C^T = E C E^{-1})
//
// so both products are DCT-I, a three-point coefficient stencil, DCT-I.
//
// The DCT-I of a length-(N+1) vector x is half the DFT of its even extension of
// length L = 2N.  Two real vectors are packed into one complex sequence (the DFT of a
// real even sequence is real, so real and imaginary parts separate).  L a power of
// two: radix-4/2 Stockham FFTs in LDS, four-step above the LDS limit.  Any other L:
// Bluestein's chirp-z identity with a power-of-two FFT of length M >= N + L = 3N.  Only
// the N + 1 outputs k = 0..N are needed, so the lags k - n of the convolution lie in
// [-(L - 1), N]: the filter holds lags 0..N at the start and -1..-(L - 1) at the end of
// the circular buffer, which do not meet once M >= N + L.
//
// Batching: the pairs of all instances of one kind (plain power of two, or Bluestein)
// form a PairSet.  Each phase of the product (pack, FFT passes, filter, stencil, c^_0,
// unpack) is ONE launch over the whole set, whatever the mix of sizes: the grid is a
// list of (pair, block) tiles built at plan creation, and every block reads its pair's
// sizes, offsets and tables from a descriptor.  A product of a batch of uneven
// instances is therefore a fixed number of launches (at most 14 per set).

#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "birk_fft.h"
#include "birk_internal.h"

namespace birk {

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  cplx<T> r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  cplx<T> r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}

template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  cplx<T> r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}

// One radix-R (R = 2 or 4) Stockham autosort stage over `count` contiguous transforms
// of length 2^logL held in LDS.  Ns = 2^logNs is the length of the sub-transforms
// already formed.  All reads of the stage complete before any write (in place).
template <typename T, int R, int NB>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int logL, int count, int logNs,
                                               const cplx<T>* __restrict__ tw, int inverse) {
  constexpr int logR = (R == 4) ? 2 : 1;
  const int logNb = logL - logR;
  const int nb = 1 << logNb;  // butterflies per transform
  const int total = count << logNb;
  const int Ns = 1 << logNs;
  const int tshift = kLdsMaxLog - (logNs + logR);
  cplx<T> v[NB][R];
  int dst[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * blockDim.x;
    dst[i] = -1;
    if (b < total) {
      const int t = b >> logNb;
      const int j = b & (nb - 1);
      const cplx<T>* base = buf + (t << logL);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = base[j + r * nb];
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cplx<T> w = tw[(jm * r) << tshift];
        if (inverse) w.y = -w.y;
        v[i][r] = cmul<T>(v[i][r], w);
      }
      if (R == 2) {
        cplx<T> a = v[i][0], c = v[i][1];
        v[i][0] = cadd<T>(a, c);
        v[i][1] = csub<T>(a, c);
      } else {
        cplx<T> t0 = cadd<T>(v[i][0], v[i][2]);
        cplx<T> t1 = csub<T>(v[i][0], v[i][2]);
        cplx<T> t2 = cadd<T>(v[i][1], v[i][3]);
        cplx<T> d = csub<T>(v[i][1], v[i][3]);
        // forward: multiply by -i; inverse: by +i
        cplx<T> t3 = inverse ? mk<T>(-d.y, d.x) : mk<T>(d.y, -d.x);
        v[i][0] = cadd<T>(t0, t2);
        v[i][2] = csub<T>(t0, t2);
        v[i][1] = cadd<T>(t1, t3);
        v[i][3] = csub<T>(t1, t3);
      }
      dst[i] = (t << logL) + ((j >> logNs) << (logNs + logR)) + jm;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (dst[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

// `count` in-place FFTs of length 2^logL in LDS (count << logL <= 4 * NB * blockDim.x).
template <typename T, int NB>
__device__ void lds_fft(cplx<T>* buf, int logL, int count, const cplx<T>* __restrict__ tw,
                        int inverse) {
  int logNs = 0;
  if (logL & 1) {
    stockham_stage<T, 2, 2 * NB>(buf, logL, count, 0, tw, inverse);
    logNs = 1;
  }
  for (; logNs < logL; logNs += 2) stockham_stage<T, 4, NB>(buf, logL, count, logNs, tw, inverse);
}


// Whole transforms of length M = 2^logM <= kLdsMax: tile = (first pair, count); the
// pairs of a tile have the same M and adjacent work slots.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_lds(cplx<T>* __restrict__ data, const PairDesc* __restrict__ pd,
                                                        const int2* __restrict__ tiles,
                                                        const cplx<T>* __restrict__ tw, int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int logM = d.logM;
  const int n = tile.y << logM;
  cplx<T>* g = data + d.work;
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = g[e];
  __syncthreads();
  lds_fft<T, 4>(buf, logM, tile.y, tw, inverse);
  for (int e = threadIdx.x; e < n; e += blockDim.x) g[e] = buf[e];
}

template <typename T>
__device__ __forceinline__ cplx<T> tw4(const cplx<T>* __restrict__ hi, const cplx<T>* __restrict__ lo,
                                       int shift, int64_t t, int inverse) {
  cplx<T> w = cmul<T>(hi[t >> shift], lo[t & ((1 << shift) - 1)]);
  if (inverse) w.y = -w.y;
  return w;
}

// Four-step, pass 1: columns n2 of x[M2 n1 + n2], FFT over n1 (length M1), twiddle
// W_M^(n2 k1), store tmp[k1 M2 + n2].  tile = (pair, column block of W).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft4_cols(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ tmp,
                                                          const PairDesc* __restrict__ pd,
                                                          const int2* __restrict__ tiles,
                                                          const cplx<T>* __restrict__ tw, int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  constexpr int pi = prec_index<T>();
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int logM1 = d.logM1, logM2 = d.logM2;
  const int M1 = 1 << logM1;
  const int logW = min(kLdsMaxLog - logM1, logM2);
  const int W = 1 << logW;
  const int c0 = tile.y << logW;
  const cplx<T>* xs = x + d.work;
  cplx<T>* ts = tmp + d.work;
  const cplx<T>* thi = (const cplx<T>*)d.thi[pi];
  const cplx<T>* tlo = (const cplx<T>*)d.tlo[pi];
  const int n = M1 << logW;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int w = e & (W - 1), n1 = e >> logW;
    buf[(w << logM1) + n1] = xs[((int64_t)n1 << logM2) + c0 + w];
  }
  __syncthreads();
  lds_fft<T, 4>(buf, logM1, W, tw, inverse);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int w = e & (W - 1), k1 = e >> logW;
    const int64_t t = (int64_t)(c0 + w) * k1;
    ts[((int64_t)k1 << logM2) + c0 + w] = cmul<T>(buf[(w << logM1) + k1], tw4<T>(thi, tlo, d.tw_shift, t, inverse));
  }
}

// Four-step, pass 2: rows k1 of tmp, FFT over n2 (length M2), store X[k1 + M1 k2].
// tile = (pair, row block of W).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft4_rows(const cplx<T>* __restrict__ tmp, cplx<T>* __restrict__ x,
                                                          const PairDesc* __restrict__ pd,
                                                          const int2* __restrict__ tiles,
                                                          const cplx<T>* __restrict__ tw, int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int logM1 = d.logM1, logM2 = d.logM2;
  const int M2 = 1 << logM2;
  const int logW = min(kLdsMaxLog - logM2, logM1);
  const int W = 1 << logW;
  const int r0 = tile.y << logW;
  const cplx<T>* ts = tmp + d.work + ((int64_t)r0 << logM2);
  cplx<T>* xs = x + d.work;
  const int n = M2 << logW;
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = ts[e];
  __syncthreads();
  lds_fft<T, 4>(buf, logM2, W, tw, inverse);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int w = e & (W - 1), k2 = e >> logW;
    xs[r0 + w + ((int64_t)k2 << logM1)] = buf[(w << logM2) + k2];
  }
}

// FFTs of length M over every pair of the set, in place in `data` (tmp: four-step
// intermediate).
template <typename T>
static hipError_t fft_set(const birk_plan* p, const PairSet& ps, cplx<T>* data, cplx<T>* tmp, int inverse,
                          hipStream_t s) {
  const cplx<T>* tw = (const cplx<T>*)p->lds_tw[prec_index<T>()];
  if (ps.n_lds > 0)
    hipLaunchKernelGGL(k_fft_lds<T>, dim3(ps.n_lds), dim3(kFftThreads), 0, s, data, ps.dev, ps.tiles_lds, tw,
                       inverse);
  if (ps.n_c4 > 0) {
    hipLaunchKernelGGL(k_fft4_cols<T>, dim3(ps.n_c4), dim3(kFftThreads), 0, s, data, tmp, ps.dev, ps.tiles_c4, tw,
                       inverse);
    hipLaunchKernelGGL(k_fft4_rows<T>, dim3(ps.n_r4), dim3(kFftThreads), 0, s, tmp, data, ps.dev, ps.tiles_r4, tw,
                       inverse);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- DCT-I plumbing

// Pack components (2p, 2p+1) into the even extension of length L = M, optionally
// doubling the end points (the E^{-1} pre-factor of the transpose).  tile = (pair, block
// over M).
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T* __restrict__ x, cplx<T>* __restrict__ z,
                                              const PairDesc* __restrict__ pd, const int2* __restrict__ tiles,
                                              int ends2) {
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int64_t n = (int64_t)tile.y * blockDim.x + threadIdx.x;
  if (n >= d.M) return;
  cplx<T> val = mk<T>(T(0), T(0));
  if (n < d.L) {
    const int64_t N = d.N;
    const int64_t k = n <= N ? n : d.L - n;
    const T* xa = x + d.src;
    T a = xa[k];
    T b = d.has2 ? xa[d.Nn + k] : T(0);
    if (ends2 && (k == 0 || k == N)) {
      a = a + a;
      b = b + b;
    }
    val = mk<T>(a, b);
  }
  z[d.work + n] = val;
}

// DFT value Y_k (k in [0, N]) of the even extension from the FFT output.
template <typename T>
__device__ __forceinline__ cplx<T> dft_value(const cplx<T>* __restrict__ z, const cplx<T>* __restrict__ chirp,
                                             int64_t k) {
  cplx<T> v = z[k];
  return chirp ? cmul<T>(v, chirp[k]) : v;
}

// Forward mid stage.  From Y = DFT(even ext of v) (so C v = Y/2), form the Chebyshev
// coefficients a_k = (-1)^k e_k Y_k / N (Fastv2a), the integrated coefficients c^_k
// (eq:c_k=bydef with the alias of eq:chatk=), and d_k = (-1)^k c^_k / e_k, the input of
// Fasta2v's DCT.  Writes d into the packed even extension for the second transform,
// except d_0, which needs c^_0, a reduction over all k; partial sums of
//     c^_0 = (1/N) [ e_0 Y_0 + Y_1 / 4 - sum_{k>=2} e_k Y_k / (k^2 - 1) ]
// go to the pair's partials (double, two per block).  tile = (pair, block over N_n).
template <typename T>
__global__ __launch_bounds__(256) void k_mid_fwd(const cplx<T>* __restrict__ z, cplx<T>* __restrict__ z2,
                                                 const PairDesc* __restrict__ pd, const int2* __restrict__ tiles,
                                                 double* __restrict__ part, int compact) {
  constexpr int pi = prec_index<T>();
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int64_t N = d.N, L = d.L, M = d.M;
  // compact: z holds Y_k (chirp applied) and d_k, k <= N, goes to z2 as is
  const cplx<T>* chirp = compact ? nullptr : (const cplx<T>*)d.chirp[pi];
  const cplx<T>* zz = z + d.work;
  cplx<T>* z2p = z2 + d.work;
  const int64_t k = (int64_t)tile.y * blockDim.x + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (k <= N) {
    const T invN = T(1) / T(N);
    cplx<T> Yk = dft_value<T>(zz, chirp, k);
    const T ek = (k == 0 || k == N) ? T(0.5) : T(1);
    {
      double c;
      if (k == 0) c = 0.5;
      else if (k == 1) c = 0.25;
      else c = -(k == N ? 0.5 : 1.0) / ((double)k * (double)k - 1.0);
      s0 = c * (double)Yk.x;
      s1 = c * (double)Yk.y;
    }
    if (k >= 1) {
      // (-1)^k c^_k = -lo_k e_{k-1} Y_{k-1}/N - hi_k e_{k+1} Y_{k+1}/N - [k = N-1] Y_N / (4 N (N+1))
      const T lo = (k == 1) ? T(1) : T(1) / (T(2) * T(k));
      const T em1 = (k - 1 == 0) ? T(0.5) : T(1);
      cplx<T> Ym = dft_value<T>(zz, chirp, k - 1);
      T rx = -lo * em1 * Ym.x;
      T ry = -lo * em1 * Ym.y;
      if (k < N) {
        const T hi = -T(1) / (T(2) * T(k));
        const T ep1 = (k + 1 == N) ? T(0.5) : T(1);
        cplx<T> Yp = dft_value<T>(zz, chirp, k + 1);
        rx -= hi * ep1 * Yp.x;
        ry -= hi * ep1 * Yp.y;
      }
      if (k == N - 1) {
        cplx<T> YN = dft_value<T>(zz, chirp, N);
        const T f = T(1) / (T(4) * T(N + 1));
        rx -= f * YN.x;
        ry -= f * YN.y;
      }
      const T sc = invN / ek;
      cplx<T> dv = mk<T>(rx * sc, ry * sc);
      z2p[k] = chirp ? cmul<T>(dv, chirp[k]) : dv;
      if (k < N && !compact) {
        const int64_t m = L - k;
        z2p[m] = chirp ? cmul<T>(dv, chirp[m]) : dv;
      }
    }
  }
  // zero fill of the Bluestein padding [L, M)
  if (!compact)
    for (int64_t m = L + k; m < M; m += (int64_t)d.nblk * blockDim.x) z2p[m] = mk<T>(T(0), T(0));
  // block reduction of the c^_0 partials, fixed order
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      r0[threadIdx.x] += r0[threadIdx.x + st];
      r1[threadIdx.x] += r1[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[d.part + 2 * tile.y + 0] = r0[0];
    part[d.part + 2 * tile.y + 1] = r1[0];
  }
}

// d_0 = 2 c^_0 from the partials: one block per pair, fixed-order tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_c0(const double* __restrict__ part, cplx<T>* __restrict__ z2,
                                            const PairDesc* __restrict__ pd) {
  const PairDesc& d = pd[blockIdx.x];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < d.nblk; i += blockDim.x) {
    a += part[d.part + 2 * i + 0];
    b += part[d.part + 2 * i + 1];
  }
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      ra[threadIdx.x] += ra[threadIdx.x + st];
      rb[threadIdx.x] += rb[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double s = 2.0 / (double)d.N;
    // the Bluestein chirp is 1 at index 0, so no pre-multiplication is needed here
    z2[d.work] = mk<T>((T)(ra[0] * s), (T)(rb[0] * s));
  }
}

// Transpose mid stage.  p = C E^{-1} g = Y / 2; q = S M^T S p, i.e.
//   q_0 = p_0 - p_1,   q_1 = (p_0 - p_2) / 4,
//   q_j = -p_0/(j^2-1) + p_{j-1} (1/(2(j-1)) - [j = N]/(2(N+1))) - [j < N] p_{j+1}/(2(j+1)).
template <typename T>
__global__ __launch_bounds__(256) void k_mid_tr(const cplx<T>* __restrict__ z, cplx<T>* __restrict__ z2,
                                                const PairDesc* __restrict__ pd, const int2* __restrict__ tiles,
                                                int compact) {
  constexpr int pi = prec_index<T>();
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int64_t N = d.N, L = d.L, M = d.M;
  const cplx<T>* chirp = compact ? nullptr : (const cplx<T>*)d.chirp[pi];
  const cplx<T>* zz = z + d.work;
  cplx<T>* z2p = z2 + d.work;
  const int64_t j = (int64_t)tile.y * blockDim.x + threadIdx.x;
  if (j <= N) {
    cplx<T> p0 = dft_value<T>(zz, chirp, 0);
    p0.x *= T(0.5);
    p0.y *= T(0.5);
    cplx<T> q;
    if (j == 0) {
      cplx<T> p1 = dft_value<T>(zz, chirp, 1);
      q = mk<T>(p0.x - T(0.5) * p1.x, p0.y - T(0.5) * p1.y);
    } else if (j == 1) {
      cplx<T> p2 = dft_value<T>(zz, chirp, 2);
      q = mk<T>(T(0.25) * (p0.x - T(0.5) * p2.x), T(0.25) * (p0.y - T(0.5) * p2.y));
    } else {
      const T jj = T(j);
      const T c0 = -T(1) / (jj * jj - T(1));
      T cm = T(1) / (T(2) * (jj - T(1)));
      if (j == N) cm -= T(1) / (T(2) * T(N + 1));
      cplx<T> pm = dft_value<T>(zz, chirp, j - 1);
      T qx = c0 * p0.x + cm * T(0.5) * pm.x;
      T qy = c0 * p0.y + cm * T(0.5) * pm.y;
      if (j < N) {
        const T cp = -T(1) / (T(2) * (jj + T(1)));
        cplx<T> pp = dft_value<T>(zz, chirp, j + 1);
        qx += cp * T(0.5) * pp.x;
        qy += cp * T(0.5) * pp.y;
      }
      q = mk<T>(qx, qy);
    }
    z2p[j] = chirp ? cmul<T>(q, chirp[j]) : q;
    if (j >= 1 && j < N && !compact) z2p[L - j] = chirp ? cmul<T>(q, chirp[L - j]) : q;
  }
  if (!compact)
    for (int64_t m = L + j; m < M; m += (int64_t)d.nblk * blockDim.x) z2p[m] = mk<T>(T(0), T(0));
}

// Final stage: out_j = scale_j * Y_j for j in [0, N], unpacking the pair.
// forward: scale = 1/2; transpose: scale = e_j / N.  tile = (pair, block over N_n).
template <typename T>
__global__ __launch_bounds__(256) void k_final(const cplx<T>* __restrict__ z, T* __restrict__ out,
                                               const PairDesc* __restrict__ pd, const int2* __restrict__ tiles,
                                               int transpose, int compact) {
  constexpr int pi = prec_index<T>();
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  const int64_t N = d.N;
  const int64_t j = (int64_t)tile.y * blockDim.x + threadIdx.x;
  if (j > N) return;
  const cplx<T> Y = dft_value<T>(z + d.work, compact ? nullptr : (const cplx<T>*)d.chirp[pi], j);
  T sc;
  if (transpose) sc = ((j == 0 || j == N) ? T(0.5) : T(1)) / T(N);
  else sc = T(0.5);
  T* o = out + d.src;
  o[j] = Y.x * sc;
  if (d.has2) o[d.Nn + j] = Y.y * sc;
}

// Product over a set with L = 2N a power of two: pack, FFT (= DCT-I, unnormalised), stencil
// and c^_0, FFT, unpack.
template <typename T>
static hipError_t product_set(birk_plan* p, const PairSet& ps, const T* v, T* out, int transpose, hipStream_t s) {
  if (ps.host.empty()) return hipSuccess;
  cplx<T>* z = (cplx<T>*)p->work[0];
  cplx<T>* z2 = (cplx<T>*)p->work[1];
  cplx<T>* tmp = (cplx<T>*)p->work[2];
  hipLaunchKernelGGL(k_pack<T>, dim3(ps.n_m), dim3(256), 0, s, v, z, ps.dev, ps.tiles_m, transpose);
  hipError_t e = fft_set<T>(p, ps, z, tmp, 0, s);
  if (e != hipSuccess) return e;
  if (!transpose) {
    hipLaunchKernelGGL(k_mid_fwd<T>, dim3(ps.n_n), dim3(256), 0, s, z, z2, ps.dev, ps.tiles_n, p->partials, 0);
    hipLaunchKernelGGL(k_c0<T>, dim3((unsigned)ps.host.size()), dim3(256), 0, s, p->partials, z2, ps.dev);
  } else {
    hipLaunchKernelGGL(k_mid_tr<T>, dim3(ps.n_n), dim3(256), 0, s, z, z2, ps.dev, ps.tiles_n, 0);
  }
  e = fft_set<T>(p, ps, z2, tmp, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final<T>, dim3(ps.n_n), dim3(256), 0, s, z2, out, ps.dev, ps.tiles_n, transpose, 0);
  return hipGetLastError();
}

// ----------------------------------------------------------------- fused Bluestein path
// For 2N not a power of two each DCT-I is a Bluestein convolution of the chirped even
// extension (length L = 2N, padded to M).  The fused path runs it in three passes over M
// (two-step FFTs above the LDS limit, one kernel below it) instead of pack, FFT, filter,
// inverse FFT as separate passes:
//   columns:  even extension x chirp, column FFTs (length M1), twiddle    -> tmp
//   rows:     row FFTs (M2), x filter spectrum, inverse row FFTs, inverse twiddle
//   icolumns: inverse column FFTs, x chirp, only the N + 1 outputs Y_k are stored.
// The inverse two-step transform takes its factors in the reverse order of the forward
// one, so the rows pass sees the forward spectrum of a row, multiplies it by the filter,
// and transforms it straight back.  Inputs: the pair's two components (first DCT,
// optionally with doubled end points) or the compact stencil output d_k (second DCT);
// outputs Y_k, k <= N, with the chirp applied.

// Padded Bluestein input at position n: (even extension of the source) x chirp_n.
template <typename T>
__device__ __forceinline__ cplx<T> blu_in(const PairDesc& d, const T* __restrict__ x, const cplx<T>* __restrict__ dz,
                                         int src_x, int ends2, const cplx<T>* __restrict__ chirp, int64_t n) {
  if (n >= d.L) return mk<T>(T(0), T(0));
  const int64_t k = n <= d.N ? n : d.L - n;
  cplx<T> v;
  if (src_x) {
    const T* xa = x + d.src;
    T a = xa[k];
    T b = d.has2 ? xa[d.Nn + k] : T(0);
    if (ends2 && (k == 0 || k == d.N)) {
      a = a + a;
      b = b + b;
    }
    v = mk<T>(a, b);
  } else {
    v = dz[d.work + k];
  }
  return cmul<T>(v, chirp[n]);
}

// ---- fused Bluestein passes on the compile-time FFTs of birk_fft.h ----
// A block of kBluThreads threads transforms kLdsMax points: kLdsMax / 2^LOGL transforms
// of length 2^LOGL in the split layout of fast::fft_ct (transform t: real parts in row
// 2t, imaginary parts in row 2t + 1, rows padded_ld(2^LOGL) reals apart).  A pair's
// length is known only at run time, so each kernel switches to the body compiled for
// it.  The inverse transform is conj(FFT(conj(.))), unnormalised (the filter spectrum
// carries 1/M).
constexpr int kBluThreads = kLdsMax / fast::kPPT;

__host__ __device__ constexpr int blu_lds_reals(int logL) {
  return 2 * (kLdsMax >> logL) * fast::padded_ld(1 << logL);
}
constexpr int blu_lds_reals_max() {
  int m = 0;
  for (int l = 3; l <= kLdsMaxLog; ++l) m = blu_lds_reals(l) > m ? blu_lds_reals(l) : m;
  return m;
}
constexpr int kBluLdsReals = blu_lds_reals_max();

template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
  return mk<T>(a.x, -a.y);
}

template <typename T, int LOGL>
__device__ __forceinline__ void sput(T* sm, int t, int n, cplx<T> v) {
  constexpr int LD = fast::padded_ld(1 << LOGL);
  sm[2 * t * LD + fast::pad(n)] = v.x;
  sm[(2 * t + 1) * LD + fast::pad(n)] = v.y;
}

template <typename T, int LOGL>
__device__ __forceinline__ cplx<T> sget(const T* sm, int t, int n) {
  constexpr int LD = fast::padded_ld(1 << LOGL);
  return mk<T>(sm[2 * t * LD + fast::pad(n)], sm[(2 * t + 1) * LD + fast::pad(n)]);
}

#define BIRK_LOG_SWITCH(val, LO, CALL)                                         \
  switch (val) {                                                               \
    case 3: if constexpr (3 >= LO) { constexpr int LG = 3; CALL; } break;      \
    case 4: if constexpr (4 >= LO) { constexpr int LG = 4; CALL; } break;      \
    case 5: if constexpr (5 >= LO) { constexpr int LG = 5; CALL; } break;      \
    case 6: if constexpr (6 >= LO) { constexpr int LG = 6; CALL; } break;      \
    case 7: { constexpr int LG = 7; CALL; } break;                             \
    case 8: { constexpr int LG = 8; CALL; } break;                             \
    case 9: { constexpr int LG = 9; CALL; } break;                             \
    case 10: { constexpr int LG = 10; CALL; } break;                           \
    case 11: { constexpr int LG = 11; CALL; } break;                           \
    case 12: { constexpr int LG = 12; CALL; } break;                           \
    default: break;                                                            \
  }

// Whole convolutions of length M = 2^LOGM <= kLdsMax, kLdsMax / M pairs per block (the
// tile's pairs share M; the remaining transforms of the block run on zeros).
template <typename T, int LOGM>
__device__ __forceinline__ void blu_lds_body(const T* __restrict__ x, const cplx<T>* __restrict__ dz,
                                             cplx<T>* __restrict__ Y, const PairDesc* __restrict__ pd, int2 tile,
                                             const cplx<T>* __restrict__ tw, int src_x, int ends2, T* sm) {
  constexpr int pi = prec_index<T>();
  constexpr int M = 1 << LOGM;
  constexpr int COUNT = kLdsMax >> LOGM;
  constexpr int PER = kLdsMax / kBluThreads;
  // the inputs, the filter spectra and the chirp of the outputs are read in one batch
  cplx<T> v[PER], fv[PER], cv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int t = e >> LOGM, n = e & (M - 1);
    v[i] = fv[i] = cv[i] = mk<T>(T(0), T(0));
    if (t < tile.y) {
      const PairDesc& d = pd[tile.x + t];
      const cplx<T>* chirp = (const cplx<T>*)d.chirp[pi];
      v[i] = blu_in<T>(d, x, dz, src_x, ends2, chirp, n);
      fv[i] = ((const cplx<T>*)d.filt[pi])[n];
      if (n <= d.N) cv[i] = chirp[n];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    sput<T, LOGM>(sm, e >> LOGM, e & (M - 1), v[i]);
  }
  __syncthreads();
  fast::fft_ct<T, LOGM, COUNT>(sm, tw);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int t = e >> LOGM, k = e & (M - 1);
    if (t < tile.y) sput<T, LOGM>(sm, t, k, cconj<T>(cmul<T>(sget<T, LOGM>(sm, t, k), fv[i])));
  }
  __syncthreads();
  fast::fft_ct<T, LOGM, COUNT>(sm, tw);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int t = e >> LOGM, k = e & (M - 1);
    if (t < tile.y) {
      const PairDesc& d = pd[tile.x + t];
      if (k <= d.N) Y[d.work + k] = cmul<T>(cconj<T>(sget<T, LOGM>(sm, t, k)), cv[i]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBluThreads) void k_blu_lds(const T* __restrict__ x, const cplx<T>* __restrict__ dz,
                                                        cplx<T>* __restrict__ Y, const PairDesc* __restrict__ pd,
                                                        const int2* __restrict__ tiles, const cplx<T>* __restrict__ tw,
                                                        int src_x, int ends2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int2 tile = tiles[blockIdx.x];
  BIRK_LOG_SWITCH(pd[tile.x].logM, 3, (blu_lds_body<T, LG>(x, dz, Y, pd, tile, tw, src_x, ends2, sm)))
}

// Columns pass: n = M2 n1 + n2; the W = kLdsMax / M1 columns [c0, c0 + W) of the padded
// input, FFT over n1, twiddle W_M^(n2 k1), tmp[k1 M2 + n2].  tile = (pair, column block).
template <typename T, int LOGM1>
__device__ __forceinline__ void blu_cols_body(const T* __restrict__ x, const cplx<T>* __restrict__ dz,
                                              cplx<T>* __restrict__ tmp, const PairDesc& d, int ty,
                                              const cplx<T>* __restrict__ tw, int src_x, int ends2, T* sm) {
  constexpr int pi = prec_index<T>();
  constexpr int LOGW = kLdsMaxLog - LOGM1;
  constexpr int W = 1 << LOGW;
  const int logM2 = d.logM2;
  const int c0 = ty << LOGW;
  const cplx<T>* chirp = (const cplx<T>*)d.chirp[pi];
  const cplx<T>* thi = (const cplx<T>*)d.thi[pi];
  const cplx<T>* tlo = (const cplx<T>*)d.tlo[pi];
  cplx<T>* ts = tmp + d.work;
  if constexpr (std::is_floating_point<T>::value) {
    // double and float: a thread's outputs k1 = k1_0 + i s (s = blockDim / W) share the
    // column n2, so their twiddles W_M^(n2 k1) are W_M^(n2 k1_0) times powers of W_M^(n2 s):
    // two reads of the double table issued with the inputs, the powers formed in double
    // (at most seven rounded products per twiddle)
    constexpr int PER = kLdsMax / kBluThreads;
    constexpr int S = kBluThreads >> LOGW;
    const int w = (int)threadIdx.x & (W - 1), k10 = (int)threadIdx.x >> LOGW;
    const int n2 = c0 + w;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int n1 = k10 + i * S;
      sput<T, LOGM1>(sm, w, n1, blu_in<T>(d, x, dz, src_x, ends2, chirp, ((int64_t)n1 << logM2) + n2));
    }
    const cplx<double>* thd = (const cplx<double>*)d.thi[0];
    const cplx<double>* tld = (const cplx<double>*)d.tlo[0];
    cplx<double> wv = tw4<double>(thd, tld, d.tw_shift, (int64_t)n2 * k10, 0);
    const cplx<double> ws = tw4<double>(thd, tld, d.tw_shift, (int64_t)n2 * S, 0);
    __syncthreads();
    fast::fft_ct<T, LOGM1, W>(sm, tw);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k1 = k10 + i * S;
      ts[((int64_t)k1 << logM2) + n2] = cmul<T>(sget<T, LOGM1>(sm, w, k1), mk<T>((T)wv.x, (T)wv.y));
      wv = cmul<double>(wv, ws);
    }
  } else {
    for (int e = threadIdx.x; e < kLdsMax; e += kBluThreads) {
      const int w = e & (W - 1), n1 = e >> LOGW;
      sput<T, LOGM1>(sm, w, n1, blu_in<T>(d, x, dz, src_x, ends2, chirp, ((int64_t)n1 << logM2) + c0 + w));
    }
    __syncthreads();
    fast::fft_ct<T, LOGM1, W>(sm, tw);
    for (int e = threadIdx.x; e < kLdsMax; e += kBluThreads) {
      const int w = e & (W - 1), k1 = e >> LOGW;
      const int64_t t = (int64_t)(c0 + w) * k1;
      ts[((int64_t)k1 << logM2) + c0 + w] = cmul<T>(sget<T, LOGM1>(sm, w, k1), tw4<T>(thi, tlo, d.tw_shift, t, 0));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBluThreads) void k_blu_cols(const T* __restrict__ x, const cplx<T>* __restrict__ dz,
                                                         cplx<T>* __restrict__ tmp, const PairDesc* __restrict__ pd,
                                                         const int2* __restrict__ tiles,
                                                         const cplx<T>* __restrict__ tw, int src_x, int ends2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  BIRK_LOG_SWITCH(d.logM1, 7, (blu_cols_body<T, LG>(x, dz, tmp, d, tile.y, tw, src_x, ends2, sm)))
}

// Rows pass: the W = kLdsMax / M2 rows k1 in [r0, r0 + W) of tmp; FFT over n2 (frequency
// k2 of k = k1 + M1 k2), times the filter spectrum (stored in this order), inverse FFT
// back to n2, times W_M^(-n2 k1), in place.  tile = (pair, row block).
template <typename T, int LOGM2>
__device__ __forceinline__ void blu_rows_body(cplx<T>* __restrict__ tmp, const PairDesc& d, int ty,
                                              const cplx<T>* __restrict__ tw, T* sm) {
  constexpr int pi = prec_index<T>();
  constexpr int M2 = 1 << LOGM2;
  constexpr int LOGW = kLdsMaxLog - LOGM2;
  constexpr int W = 1 << LOGW;
  const int r0 = ty << LOGW;
  cplx<T>* ts = tmp + d.work + ((int64_t)r0 << LOGM2);
  const cplx<T>* filt = (const cplx<T>*)d.filt[pi] + ((int64_t)r0 << LOGM2);
  constexpr int PER = kLdsMax / kBluThreads;
  // the tile and its filter spectrum are read in one batch
  cplx<T> v[PER], fv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    v[i] = ts[e];
    fv[i] = filt[e];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    sput<T, LOGM2>(sm, e >> LOGM2, e & (M2 - 1), v[i]);
  }
  __syncthreads();
  fast::fft_ct<T, LOGM2, W>(sm, tw);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int w = e >> LOGM2, k2 = e & (M2 - 1);
    sput<T, LOGM2>(sm, w, k2, cconj<T>(cmul<T>(sget<T, LOGM2>(sm, w, k2), fv[i])));
  }
  __syncthreads();
  const cplx<T>* thi = (const cplx<T>*)d.thi[pi];
  const cplx<T>* tlo = (const cplx<T>*)d.tlo[pi];
  if constexpr (std::is_floating_point<T>::value && LOGM2 <= 9) {
    // double and float, rows of at most blockDim points: a thread's elements share n2 and
    // step through rows w = w_0 + i s, so their twiddles W_M^(-n2 (r0 + w)) are powers of
    // one step times a base (double table, read before the second transform; powers in
    // double)
    constexpr int S = kBluThreads >> LOGM2;
    const int n2 = (int)threadIdx.x & (M2 - 1), w0 = (int)threadIdx.x >> LOGM2;
    const cplx<double>* thd = (const cplx<double>*)d.thi[0];
    const cplx<double>* tld = (const cplx<double>*)d.tlo[0];
    cplx<double> wv = tw4<double>(thd, tld, d.tw_shift, (int64_t)n2 * (r0 + w0), 1);
    const cplx<double> ws = tw4<double>(thd, tld, d.tw_shift, (int64_t)n2 * S, 1);
    fast::fft_ct<T, LOGM2, W>(sm, tw);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int w = w0 + i * S;
      ts[(w << LOGM2) + n2] = cmul<T>(cconj<T>(sget<T, LOGM2>(sm, w, n2)), mk<T>((T)wv.x, (T)wv.y));
      wv = cmul<double>(wv, ws);
    }
  } else {
    fast::fft_ct<T, LOGM2, W>(sm, tw);
    for (int e = threadIdx.x; e < kLdsMax; e += kBluThreads) {
      const int w = e >> LOGM2, n2 = e & (M2 - 1);
      ts[e] = cmul<T>(cconj<T>(sget<T, LOGM2>(sm, w, n2)), tw4<T>(thi, tlo, d.tw_shift, (int64_t)n2 * (r0 + w), 1));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBluThreads) void k_blu_rows(cplx<T>* __restrict__ tmp, const PairDesc* __restrict__ pd,
                                                         const int2* __restrict__ tiles,
                                                         const cplx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  BIRK_LOG_SWITCH(d.logM2, 6, (blu_rows_body<T, LG>(tmp, d, tile.y, tw, sm)))
}

// Inverse columns pass: columns n2 in [c0, c0 + W) of tmp[k1 M2 + n2], inverse FFT over
// k1 -> n1, output index n = M2 n1 + n2; Y_n = value x chirp_n for n <= N.
// tile = (pair, column block).
template <typename T, int LOGM1>
__device__ __forceinline__ void blu_icols_body(const cplx<T>* __restrict__ tmp, cplx<T>* __restrict__ Y,
                                               const PairDesc& d, int ty, const cplx<T>* __restrict__ tw, T* sm) {
  constexpr int pi = prec_index<T>();
  constexpr int LOGW = kLdsMaxLog - LOGM1;
  constexpr int W = 1 << LOGW;
  const int logM2 = d.logM2;
  const int c0 = ty << LOGW;
  const cplx<T>* ts = tmp + d.work;
  const cplx<T>* chirp = (const cplx<T>*)d.chirp[pi];
  constexpr int PER = kLdsMax / kBluThreads;
  // the tile and the chirp of its outputs n = M2 n1 + n2 <= N are read in one batch
  cplx<T> v[PER], cv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int w = e & (W - 1), k = e >> LOGW;
    const int64_t idx = ((int64_t)k << logM2) + c0 + w;
    v[i] = ts[idx];
    cv[i] = idx <= d.N ? chirp[idx] : mk<T>(T(0), T(0));
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    sput<T, LOGM1>(sm, e & (W - 1), e >> LOGW, cconj<T>(v[i]));
  }
  __syncthreads();
  fast::fft_ct<T, LOGM1, W>(sm, tw);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = (int)threadIdx.x + i * kBluThreads;
    const int w = e & (W - 1), n1 = e >> LOGW;
    const int64_t idx = ((int64_t)n1 << logM2) + c0 + w;
    if (idx <= d.N) Y[d.work + idx] = cmul<T>(cconj<T>(sget<T, LOGM1>(sm, w, n1)), cv[i]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBluThreads) void k_blu_icols(const cplx<T>* __restrict__ tmp, cplx<T>* __restrict__ Y,
                                                          const PairDesc* __restrict__ pd,
                                                          const int2* __restrict__ tiles,
                                                          const cplx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int2 tile = tiles[blockIdx.x];
  const PairDesc& d = pd[tile.x];
  BIRK_LOG_SWITCH(d.logM1, 7, (blu_icols_body<T, LG>(tmp, Y, d, tile.y, tw, sm)))
}

#undef BIRK_LOG_SWITCH

// One DCT-I (= 2 C) of every pair of a Bluestein set by the fused passes; Y receives
// Y_k, k <= N, at each pair's work offset.
template <typename T>
static hipError_t dct_blu(birk_plan* p, const PairSet& ps, const T* x, const cplx<T>* dz, cplx<T>* Y, int src_x,
                          int ends2, hipStream_t s) {
  const cplx<T>* tw = (const cplx<T>*)p->lds_tw[prec_index<T>()];
  cplx<T>* tmp = (cplx<T>*)p->work[0];
  const size_t lds = (size_t)kBluLdsReals * sizeof(T);
  static const bool attr = [] {  // above the default dynamic LDS limit in double
    constexpr int b = (int)(kBluLdsReals * sizeof(T));
    (void)hipFuncSetAttribute((const void*)k_blu_lds<T>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)k_blu_cols<T>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)k_blu_rows<T>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)k_blu_icols<T>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    return true;
  }();
  (void)attr;
  if (ps.n_lds > 0)
    hipLaunchKernelGGL(k_blu_lds<T>, dim3(ps.n_lds), dim3(kBluThreads), lds, s, x, dz, Y, ps.dev, ps.tiles_lds, tw,
                       src_x, ends2);
  if (ps.n_c4 > 0) {
    hipLaunchKernelGGL(k_blu_cols<T>, dim3(ps.n_c4), dim3(kBluThreads), lds, s, x, dz, tmp, ps.dev, ps.tiles_c4, tw,
                       src_x, ends2);
    hipLaunchKernelGGL(k_blu_rows<T>, dim3(ps.n_r4), dim3(kBluThreads), lds, s, tmp, ps.dev, ps.tiles_r4, tw);
    hipLaunchKernelGGL(k_blu_icols<T>, dim3(ps.n_c4), dim3(kBluThreads), lds, s, tmp, Y, ps.dev, ps.tiles_c4, tw);
  }
  return hipGetLastError();
}

// Product over a Bluestein set: DCT (fused) -> stencil and c^_0 -> DCT (fused) -> unpack.
template <typename T>
static hipError_t product_blu(birk_plan* p, const PairSet& ps, const T* v, T* out, int transpose, hipStream_t s) {
  if (ps.host.empty()) return hipSuccess;
  cplx<T>* Y = (cplx<T>*)p->work[1];
  cplx<T>* dz = (cplx<T>*)p->work[2];
  hipError_t e = dct_blu<T>(p, ps, v, nullptr, Y, 1, transpose, s);
  if (e != hipSuccess) return e;
  if (!transpose) {
    hipLaunchKernelGGL(k_mid_fwd<T>, dim3(ps.n_n), dim3(256), 0, s, Y, dz, ps.dev, ps.tiles_n, p->partials, 1);
    hipLaunchKernelGGL(k_c0<T>, dim3((unsigned)ps.host.size()), dim3(256), 0, s, p->partials, dz, ps.dev);
  } else {
    hipLaunchKernelGGL(k_mid_tr<T>, dim3(ps.n_n), dim3(256), 0, s, Y, dz, ps.dev, ps.tiles_n, 1);
  }
  e = dct_blu<T>(p, ps, nullptr, dz, Y, 0, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final<T>, dim3(ps.n_n), dim3(256), 0, s, Y, out, ps.dev, ps.tiles_n, transpose, 1);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_product(birk_plan* p, const T* v, T* out, int transpose, hipStream_t s) {
  for (const FastGroup& g : p->fgroups) {
    hipError_t e = fast_product<T>(p, g, v, out, transpose, s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = product_set<T>(p, p->gen[0], v, out, transpose, s);
  if (e == hipSuccess) e = product_blu<T>(p, p->gen[1], v, out, transpose, s);
  return e;
}

template hipError_t apply_product<double>(birk_plan*, const double*, double*, int, hipStream_t);
template hipError_t apply_product<float>(birk_plan*, const float*, float*, int, hipStream_t);
template hipError_t apply_product<df32>(birk_plan*, const df32*, df32*, int, hipStream_t);

// ----------------------------------------------------------------- tables

// exp(-i pi num / den) in double.  The angle is reduced exactly in integers and folded
// into [0, pi/4] before the library sin/cos, so each entry is correctly rounded to
// within about one ulp.
static void expi_pi(int64_t num, int64_t den, double* c, double* s) {
  // theta = pi * m / den with m in [0, 2 den); work with numerators over 4 den so that
  // the octant boundaries are integers.
  int64_t m = num % (2 * den);
  if (m < 0) m += 2 * den;
  int64_t q = 4 * m;            // theta = pi * q / (4 den), q in [0, 8 den)
  const int64_t D = 4 * den;    // pi  <-> D
  double sgn_c = 1.0, sgn_s = 1.0;
  if (q >= D) { q -= D; sgn_c = -sgn_c; sgn_s = -sgn_s; }          // theta - pi
  bool swap = false;
  if (2 * q > D) { q = D - q; sgn_c = -sgn_c; }                     // pi - theta
  if (4 * q > D) { q = D / 2 - q; swap = true; }                    // pi/2 - theta (D even)
  const double th = M_PI * (double)q / (double)D;
  double cs = std::cos(th), sn = std::sin(th);
  if (q == 0) { cs = 1.0; sn = 0.0; }
  if (swap) { const double t = cs; cs = sn; sn = t; }
  *c = sgn_c * cs;
  *s = -(sgn_s * sn);
}

static hipError_t upload_raw(birk_plan* p, const void* h, size_t bytes, void** d) {
  *d = nullptr;
  hipError_t e = hipMalloc(d, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) return e;
  p->allocs.push_back(*d);
  return hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice);
}

template <typename T>
static hipError_t upload_cplx(birk_plan* p, const std::vector<double>& re, const std::vector<double>& im,
                              const void** dptr) {
  const size_t n = re.size();
  std::vector<cplx<T>> h(n);
  for (size_t i = 0; i < n; ++i) h[i] = mk<T>((T)re[i], (T)im[i]);
  void* d = nullptr;
  hipError_t e = upload_raw(p, h.data(), n * sizeof(cplx<T>), &d);
  *dptr = d;
  return e;
}

// One table in all three precisions.
static hipError_t upload_all(birk_plan* p, const std::vector<double>& re, const std::vector<double>& im,
                             const void** dst) {
  hipError_t e = upload_cplx<double>(p, re, im, &dst[0]);
  if (e == hipSuccess) e = upload_cplx<float>(p, re, im, &dst[1]);
  if (e == hipSuccess) e = upload_cplx<df32>(p, re, im, &dst[2]);
  return e;
}

// Bluestein filter b_m = conj(chirp_|lag|) on the circular buffer of length M: lags
// 0..N at m = lag, lags -1..-(L - 1) at m = M + lag, zero between.
template <typename T>
__global__ void k_build_filter(cplx<T>* __restrict__ b, const cplx<T>* __restrict__ chirp, int64_t L,
                               int64_t M) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  cplx<T> v = mk<T>(T(0), T(0));
  if (m <= L / 2) {
    v = chirp[m];
    v.y = -v.y;
  } else if (M - m < L) {
    v = chirp[M - m];
    v.y = -v.y;
  }
  b[m] = v;
}

// dst = s src; with logM1 > 0 in the order of the two-step rows pass: dst[k1 M2 + k2] =
// s src[k1 + M1 k2] (frequency k = k1 + M1 k2), so each row reads its filter contiguously.
template <typename T>
__global__ void k_scale_to(const cplx<double>* __restrict__ src, cplx<T>* __restrict__ dst, int64_t M,
                           double s, int logM1, int logM2) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int64_t from = m;
  if (logM1 > 0) from = (m >> logM2) + ((m & ((int64_t(1) << logM2) - 1)) << logM1);
  dst[m] = mk<T>((T)(src[from].x * s), (T)(src[from].y * s));
}

// Filter spectrum moved from the rows-pass order of the split (a1, a2) of M to that of
// (b1, b2): dst[k1 M2' + k2] = src at the position of frequency k1 + M1' k2 in the old order.
template <typename T>
__global__ void k_relayout(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst, int64_t M, int a1, int a2,
                           int b1, int b2) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int64_t q = (m >> b2) + ((m & ((int64_t(1) << b2) - 1)) << b1);     // frequency
  const int64_t from = ((q & ((int64_t(1) << a1) - 1)) << a2) + (q >> a1);  // its old position
  dst[m] = src[from];
}

static int ilog2_ceil(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

static PairDesc make_pair(int64_t src, int64_t Nn, int has2, const int* split) {
  PairDesc d;
  d.src = src;
  d.Nn = Nn;
  d.N = Nn - 1;
  d.L = 2 * d.N;
  const bool pow2 = (d.L & (d.L - 1)) == 0;
  d.M = pow2 ? d.L : (int64_t(1) << ilog2_ceil(d.N + d.L));
  d.logM = ilog2_ceil(d.M);
  if (d.logM > kLdsMaxLog) {
    d.logM1 = (split && split[d.logM] > 0) ? split[d.logM] : (d.logM + 1) / 2;
    d.logM2 = d.logM - d.logM1;
  }
  d.tw_shift = (d.logM + 1) / 2;
  d.has2 = has2;
  d.nblk = (int)((Nn + 255) / 256);
  return d;
}

// Sort the pairs by M (so that pairs of one LDS-sized M are adjacent), then give each
// its work slot and partials.
static void layout_set(PairSet& ps, int64_t& woff, int64_t& poff) {
  std::stable_sort(ps.host.begin(), ps.host.end(),
                   [](const PairDesc& a, const PairDesc& b) { return a.M < b.M; });
  ps.work = 0;
  ps.parts = 0;
  for (PairDesc& d : ps.host) {
    d.work = woff;
    woff += d.M;
    ps.work += d.M;
    d.part = poff;
    poff += 2 * (int64_t)d.nblk;
    ps.parts += 2 * (int64_t)d.nblk;
  }
}

void plan_products(birk_plan* p) {
  p->fgroups.clear();
  p->gen[0] = PairSet();
  p->gen[1] = PairSet();
  int64_t woff = 0, poff = 0;
  const int B = (int)p->inst.size();
  for (int i = 0; i < B;) {
    const Instance& in = p->inst[i];
    if (p->use_fast && fast_eligible(in.N)) {
      FastGroup g;
      g.Nn = in.Nn;
      g.N = in.N;
      g.off = in.off;
      g.kn = p->fast_kn;
      int j = i;
      while (j < B && p->inst[j].N == in.N) g.nc += p->inst[j++].nx;
      int64_t fw = 0, fp = 0;
      fast_sizes(p, g.N, g.nc, &fw, &fp);
      g.work_off = woff;
      g.part_off = poff;
      woff += fw;
      poff += fp;
      p->fgroups.push_back(g);
      i = j;
      continue;
    }
    const int np = (in.nx + 1) / 2;
    for (int q = 0; q < np; ++q) {
      PairDesc d = make_pair(in.off + 2 * (int64_t)q * in.Nn, in.Nn, 2 * q + 1 < in.nx, p->blu_split);
      p->gen[(d.L == d.M) ? 0 : 1].host.push_back(d);
    }
    ++i;
  }
  layout_set(p->gen[0], woff, poff);
  layout_set(p->gen[1], woff, poff);
  p->total_work = woff;
  p->total_part = poff;
}

// Tile lists of a set (see PairSet), uploaded with the descriptors.
static hipError_t finalize_set(birk_plan* p, PairSet& ps) {
  std::vector<int2> tm, tn, tl, tc, tr;
  const int np = (int)ps.host.size();
  for (int q = 0; q < np; ++q) {
    const PairDesc& d = ps.host[q];
    for (int64_t b = 0; b < (d.M + 255) / 256; ++b) tm.push_back(make_int2(q, (int)b));
    for (int b = 0; b < d.nblk; ++b) tn.push_back(make_int2(q, b));
    if (d.logM > kLdsMaxLog) {
      const int logW1 = std::min(kLdsMaxLog - d.logM1, d.logM2);
      const int logW2 = std::min(kLdsMaxLog - d.logM2, d.logM1);
      for (int b = 0; b < (1 << (d.logM2 - logW1)); ++b) tc.push_back(make_int2(q, b));
      for (int b = 0; b < (1 << (d.logM1 - logW2)); ++b) tr.push_back(make_int2(q, b));
    }
  }
  for (int q = 0; q < np;) {
    const PairDesc& d = ps.host[q];
    if (d.logM > kLdsMaxLog) {
      ++q;
      continue;
    }
    const int per = kLdsMax >> d.logM;
    int cnt = 1;
    while (q + cnt < np && cnt < per && ps.host[q + cnt].M == d.M && ps.host[q + cnt].work == d.work + cnt * d.M)
      ++cnt;
    tl.push_back(make_int2(q, cnt));
    q += cnt;
  }
  ps.n_m = (int)tm.size();
  ps.n_n = (int)tn.size();
  ps.n_lds = (int)tl.size();
  ps.n_c4 = (int)tc.size();
  ps.n_r4 = (int)tr.size();
  void* d = nullptr;
  hipError_t e = upload_raw(p, ps.host.data(), ps.host.size() * sizeof(PairDesc), &d);
  ps.dev = (PairDesc*)d;
  auto up = [&](const std::vector<int2>& v, int2** dst) {
    void* x = nullptr;
    if (e == hipSuccess) e = upload_raw(p, v.data(), v.size() * sizeof(int2), &x);
    *dst = (int2*)x;
  };
  up(tm, &ps.tiles_m);
  up(tn, &ps.tiles_n);
  up(tl, &ps.tiles_lds);
  up(tc, &ps.tiles_c4);
  up(tr, &ps.tiles_r4);
  return e;
}

// ----------------------------------------------------------------- general-path tuner
// Bluestein pairs with M above the LDS limit run their two-step FFTs with M = M1 M2; the
// default M1 = 2^ceil(log2(M) / 2).  For each such size (2^logM) the tuner times the plan's
// product with every split the compile-time kernels support (7 <= log2 M1 <= 12,
// 6 <= log2 M2 <= 12), one size at a time with the others fixed, and keeps the fastest
// (the current choice stays unless another is more than 2 % faster).  A change of split
// moves the filter spectra of that size into the new rows-pass order and rebuilds the
// four-step tile lists; the products change only in rounding order.

// Split (log2 M1) of every pair of size 2^logM in the Bluestein set: descriptors,
// filter tables (each distinct filter once) and the cols / rows tile lists.
static hipError_t set_blu_split(birk_plan* p, int logM, int logM1, hipStream_t s) {
  PairSet& ps = p->gen[1];
  hipError_t e = hipSuccess;
  std::vector<const void*> moved;
  cplx<double>* tmp = (cplx<double>*)p->work[0];
  for (PairDesc& d : ps.host) {
    if (d.logM != logM || d.logM1 == logM1) continue;
    const int a1 = d.logM1, a2 = d.logM2, b1 = logM1, b2 = logM - logM1;
    if (std::find(moved.begin(), moved.end(), d.filt[0]) == moved.end()) {
      moved.push_back(d.filt[0]);
      const dim3 grid((unsigned)((d.M + 255) / 256));
      // through work[0] (free between products), one precision at a time
      hipLaunchKernelGGL(k_relayout<double>, grid, dim3(256), 0, s, (const cplx<double>*)d.filt[0], tmp, d.M, a1, a2,
                         b1, b2);
      e = hipMemcpyAsync((void*)d.filt[0], tmp, d.M * sizeof(cplx<double>), hipMemcpyDeviceToDevice, s);
      hipLaunchKernelGGL(k_relayout<float>, grid, dim3(256), 0, s, (const cplx<float>*)d.filt[1], (cplx<float>*)tmp,
                         d.M, a1, a2, b1, b2);
      if (e == hipSuccess) e = hipMemcpyAsync((void*)d.filt[1], tmp, d.M * sizeof(cplx<float>), hipMemcpyDeviceToDevice, s);
      hipLaunchKernelGGL(k_relayout<df32>, grid, dim3(256), 0, s, (const cplx<df32>*)d.filt[2], (cplx<df32>*)tmp,
                         d.M, a1, a2, b1, b2);
      if (e == hipSuccess) e = hipMemcpyAsync((void*)d.filt[2], tmp, d.M * sizeof(cplx<df32>), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
    d.logM1 = b1;
    d.logM2 = b2;
  }
  p->blu_split[logM] = logM1;
  // descriptors in place; cols / rows tile lists rebuilt (their lengths depend on the split)
  e = hipMemcpyAsync(ps.dev, ps.host.data(), ps.host.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
  std::vector<int2> tc, tr;
  for (int q = 0; q < (int)ps.host.size(); ++q) {
    const PairDesc& d = ps.host[q];
    if (d.logM <= kLdsMaxLog) continue;
    const int logW1 = std::min(kLdsMaxLog - d.logM1, d.logM2);
    const int logW2 = std::min(kLdsMaxLog - d.logM2, d.logM1);
    for (int b = 0; b < (1 << (d.logM2 - logW1)); ++b) tc.push_back(make_int2(q, b));
    for (int b = 0; b < (1 << (d.logM1 - logW2)); ++b) tr.push_back(make_int2(q, b));
  }
  auto replace = [&](const std::vector<int2>& v, int2** dst, int* cnt) {
    if (e != hipSuccess) return;
    if (*dst) {
      e = hipStreamSynchronize(s);
      auto it = std::find(p->allocs.begin(), p->allocs.end(), (void*)*dst);
      if (it != p->allocs.end()) p->allocs.erase(it);
      if (e == hipSuccess) e = hipFree(*dst);
    }
    void* x = nullptr;
    if (e == hipSuccess) e = upload_raw(p, v.data(), v.size() * sizeof(int2), &x);
    *dst = (int2*)x;
    *cnt = (int)v.size();
  };
  replace(tc, &ps.tiles_c4, &ps.n_c4);
  replace(tr, &ps.tiles_r4, &ps.n_r4);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

template <typename T>
static hipError_t tune_general_t(birk_plan* p, hipStream_t s, std::string* report) {
  std::vector<int> sizes;
  for (const PairDesc& d : p->gen[1].host)
    if (d.logM > kLdsMaxLog && std::find(sizes.begin(), sizes.end(), d.logM) == sizes.end()) sizes.push_back(d.logM);
  if (sizes.empty()) {
    *report += "general path: no Bluestein sizes above the LDS limit\n";
    return hipSuccess;
  }
  T* in[2] = {(T*)p->tmp_vec[0], (T*)p->tmp_vec[2]};
  T* out[2] = {(T*)p->tmp_vec[1], (T*)p->tmp_vec[3]};
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(in[b], 0, (size_t)p->total_len * sizeof(T), s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto time_product = [&](float* ms) -> hipError_t {
    hipError_t r = apply_product<T>(p, in[0], out[0], 0, s);
    float best = 0.0f;
    for (int round = 0; round < 2 && r == hipSuccess; ++round) {
      r = hipEventRecord(e0, s);
      for (int k = 0; k < 3 && r == hipSuccess; ++k) r = apply_product<T>(p, in[k & 1], out[k & 1], 0, s);
      if (r == hipSuccess) r = hipEventRecord(e1, s);
      if (r == hipSuccess) r = hipEventSynchronize(e1);
      float t = 0.0f;
      if (r == hipSuccess) r = hipEventElapsedTime(&t, e0, e1);
      if (round == 0 || t < best) best = t;
    }
    *ms = best / 3.0f;
    return r;
  };
  std::sort(sizes.begin(), sizes.end());
  char line[160];
  for (int logM : sizes) {
    if (e != hipSuccess) break;
    int cur = 0;
    for (const PairDesc& d : p->gen[1].host)
      if (d.logM == logM) cur = d.logM1;
    float best_ms = 0.0f;
    if ((e = time_product(&best_ms)) != hipSuccess) break;
    snprintf(line, sizeof line, "general path M=2^%d: [M1 2^%d] %.1f us;", logM, cur, 1000.0 * best_ms);
    *report += line;
    int best = cur;
    const int lo = std::max(7, logM - kLdsMaxLog), hi = std::min(kLdsMaxLog, logM - 6);
    for (int l1 = lo; l1 <= hi && e == hipSuccess; ++l1) {
      if (l1 == cur) continue;
      if ((e = set_blu_split(p, logM, l1, s)) != hipSuccess) break;
      float ms = 0.0f;
      if ((e = time_product(&ms)) != hipSuccess) break;
      snprintf(line, sizeof line, " [M1 2^%d] %.1f us;", l1, 1000.0 * ms);
      *report += line;
      if (ms < best_ms * (1.0f - 0.02f)) {
        best_ms = ms;
        best = l1;
      }
    }
    if (e == hipSuccess) e = set_blu_split(p, logM, best, s);
    snprintf(line, sizeof line, " chosen [M1 2^%d]\n", best);
    *report += line;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

hipError_t tune_general(birk_plan* p, hipStream_t s, std::string* report) {
  if (p->prec == BIRK_F64) return tune_general_t<double>(p, s, report);
  if (p->prec == BIRK_DF32) return tune_general_t<df32>(p, s, report);
  return tune_general_t<float>(p, s, report);
}

hipError_t build_tables(birk_plan* p) {
  hipError_t e;
  {
    std::vector<double> re(kLdsMax), im(kLdsMax);
    for (int t = 0; t < kLdsMax; ++t) expi_pi(2 * (int64_t)t, kLdsMax, &re[t], &im[t]);
    if ((e = upload_all(p, re, im, p->lds_tw)) != hipSuccess) return e;
  }
  // four-step twiddles, one set per transform length
  std::map<int64_t, TwiddleSet> twsets;
  auto twiddles = [&](int64_t M, TwiddleSet* out) -> hipError_t {
    auto it = twsets.find(M);
    if (it != twsets.end()) {
      *out = it->second;
      return hipSuccess;
    }
    TwiddleSet ts;
    const int logM = ilog2_ceil(M);
    ts.shift = (logM + 1) / 2;
    const int64_t nlo = (int64_t)1 << ts.shift, nhi = M >> ts.shift;
    std::vector<double> re(nlo), im(nlo);
    for (int64_t t = 0; t < nlo; ++t) expi_pi(2 * t, M, &re[t], &im[t]);
    hipError_t err = upload_all(p, re, im, ts.lo);
    re.assign(nhi, 0.0);
    im.assign(nhi, 0.0);
    for (int64_t t = 0; t < nhi; ++t) expi_pi(2 * (t << ts.shift), M, &re[t], &im[t]);
    if (err == hipSuccess) err = upload_all(p, re, im, ts.hi);
    twsets[M] = ts;
    *out = ts;
    return err;
  };
  for (FastGroup& g : p->fgroups)
    if ((e = twiddles(2 * g.N, &g.tw)) != hipSuccess) return e;
  for (int k = 0; k < 2; ++k)
    for (PairDesc& d : p->gen[k].host)
      if (d.logM > kLdsMaxLog) {
        TwiddleSet ts;
        if ((e = twiddles(d.M, &ts)) != hipSuccess) return e;
        for (int pi = 0; pi < kNumPrec; ++pi) {
          d.thi[pi] = ts.hi[pi];
          d.tlo[pi] = ts.lo[pi];
        }
      }
  // Bluestein chirp and filter spectrum, one per distinct L
  struct Blue {
    const void* chirp[kNumPrec];
    const void* filt[kNumPrec];
  };
  std::map<int64_t, Blue> blue;
  PairSet fs;  // one pair per distinct L: the filter FFTs
  for (const PairDesc& d : p->gen[1].host) {
    if (blue.count(d.L)) continue;
    Blue b{};
    std::vector<double> re(d.L), im(d.L);
    for (int64_t n = 0; n < d.L; ++n) {
      const int64_t m = (int64_t)(((__int128)n * n) % (2 * d.L));
      expi_pi(m, d.L, &re[n], &im[n]);
    }
    if ((e = upload_all(p, re, im, b.chirp)) != hipSuccess) return e;
    blue[d.L] = b;
    PairDesc f = d;
    fs.host.push_back(f);
  }
  if (!fs.host.empty()) {
    int64_t woff = 0, poff = 0;
    layout_set(fs, woff, poff);  // filter slots from the start of work[0] / work[2]
    for (PairDesc& f : fs.host) {
      if (f.logM > kLdsMaxLog) {
        TwiddleSet ts;
        if ((e = twiddles(f.M, &ts)) != hipSuccess) return e;
        for (int pi = 0; pi < kNumPrec; ++pi) {
          f.thi[pi] = ts.hi[pi];
          f.tlo[pi] = ts.lo[pi];
        }
      }
      cplx<double>* bw = (cplx<double>*)p->work[0] + f.work;
      hipLaunchKernelGGL(k_build_filter<double>, dim3((unsigned)((f.M + 255) / 256)), dim3(256), 0, p->stream, bw,
                         (const cplx<double>*)blue[f.L].chirp[0], f.L, f.M);
    }
    if ((e = finalize_set(p, fs)) != hipSuccess) return e;
    e = fft_set<double>(p, fs, (cplx<double>*)p->work[0], (cplx<double>*)p->work[2], 0, p->stream);
    if (e != hipSuccess) return e;
    for (const PairDesc& f : fs.host) {
      Blue& b = blue[f.L];
      const cplx<double>* bw = (const cplx<double>*)p->work[0] + f.work;
      const double s = 1.0 / (double)f.M;
      const dim3 grid((unsigned)((f.M + 255) / 256));
      void* d0 = nullptr;
      void* d1 = nullptr;
      void* d2 = nullptr;
      if ((e = hipMalloc(&d0, f.M * sizeof(cplx<double>))) != hipSuccess) return e;
      p->allocs.push_back(d0);
      if ((e = hipMalloc(&d1, f.M * sizeof(cplx<float>))) != hipSuccess) return e;
      p->allocs.push_back(d1);
      if ((e = hipMalloc(&d2, f.M * sizeof(cplx<df32>))) != hipSuccess) return e;
      p->allocs.push_back(d2);
      const int l1 = f.logM > kLdsMaxLog ? f.logM1 : 0;  // two-step rows pass order
      const int l2 = f.logM2;
      hipLaunchKernelGGL(k_scale_to<double>, grid, dim3(256), 0, p->stream, bw, (cplx<double>*)d0, f.M, s, l1, l2);
      hipLaunchKernelGGL(k_scale_to<float>, grid, dim3(256), 0, p->stream, bw, (cplx<float>*)d1, f.M, s, l1, l2);
      hipLaunchKernelGGL(k_scale_to<df32>, grid, dim3(256), 0, p->stream, bw, (cplx<df32>*)d2, f.M, s, l1, l2);
      b.filt[0] = d0;
      b.filt[1] = d1;
      b.filt[2] = d2;
    }
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return e;
    for (PairDesc& d : p->gen[1].host) {
      const Blue& b = blue[d.L];
      for (int pi = 0; pi < kNumPrec; ++pi) {
        d.chirp[pi] = b.chirp[pi];
        d.filt[pi] = b.filt[pi];
      }
    }
  }
  for (int k = 0; k < 2; ++k)
    if (!p->gen[k].host.empty() && (e = finalize_set(p, p->gen[k])) != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace birk
