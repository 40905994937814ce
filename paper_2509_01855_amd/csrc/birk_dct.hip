// Fast Birkhoff products B^a v and B^aT g on the CGL grid (gfx950).
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
// Bluestein's chirp-z identity with a power-of-two FFT of length M >= 2L - 1.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

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
__device__ __forceinline__ cplx<T> mk(T x, T y) {
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

// Whole transforms of length M = 2^logM <= kLdsMax, several per block when short.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_lds(cplx<T>* __restrict__ data, int logM,
                                                        int count, const cplx<T>* __restrict__ tw,
                                                        int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  const int per = kLdsMax >> logM;
  const int t0 = blockIdx.x * per;
  const int cnt = min(per, count - t0);
  if (cnt <= 0) return;
  const int n = cnt << logM;
  cplx<T>* g = data + ((int64_t)t0 << logM);
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = g[e];
  __syncthreads();
  lds_fft<T, 4>(buf, logM, cnt, tw, inverse);
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
// W_M^(n2 k1), store tmp[k1 M2 + n2].  grid = (M2 / W, count).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft4_cols(const cplx<T>* __restrict__ x,
                                                          cplx<T>* __restrict__ tmp, int logM1,
                                                          int logM2, const cplx<T>* __restrict__ tw,
                                                          const cplx<T>* __restrict__ thi,
                                                          const cplx<T>* __restrict__ tlo,
                                                          int tshift, int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  const int M1 = 1 << logM1, M2 = 1 << logM2;
  const int logW = min(kLdsMaxLog - logM1, logM2);
  const int W = 1 << logW;
  const int c0 = blockIdx.x << logW;
  const int64_t M = (int64_t)M1 << logM2;
  const cplx<T>* xs = x + (int64_t)blockIdx.y * M;
  cplx<T>* ts = tmp + (int64_t)blockIdx.y * M;
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
    ts[((int64_t)k1 << logM2) + c0 + w] = cmul<T>(buf[(w << logM1) + k1], tw4<T>(thi, tlo, tshift, t, inverse));
  }
}

// Four-step, pass 2: rows k1 of tmp, FFT over n2 (length M2), store X[k1 + M1 k2].
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft4_rows(const cplx<T>* __restrict__ tmp,
                                                          cplx<T>* __restrict__ x, int logM1,
                                                          int logM2, const cplx<T>* __restrict__ tw,
                                                          int inverse) {
  __shared__ cplx<T> buf[kLdsMax];
  const int M2 = 1 << logM2;
  const int logW = min(kLdsMaxLog - logM2, logM1);
  const int W = 1 << logW;
  const int r0 = blockIdx.x << logW;
  const int64_t M = (int64_t)M2 << logM1;
  const cplx<T>* ts = tmp + (int64_t)blockIdx.y * M + ((int64_t)r0 << logM2);
  cplx<T>* xs = x + (int64_t)blockIdx.y * M;
  const int n = M2 << logW;
  for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = ts[e];
  __syncthreads();
  lds_fft<T, 4>(buf, logM2, W, tw, inverse);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int w = e & (W - 1), k2 = e >> logW;
    xs[r0 + w + ((int64_t)k2 << logM1)] = buf[(w << logM2) + k2];
  }
}

template <typename T>
hipError_t fft_batched(const birk_plan* p, const Instance& in, cplx<T>* data, cplx<T>* tmp,
                       int count, int inverse, hipStream_t s) {
  const int pi = std::is_same<T, double>::value ? 0 : 1;
  const cplx<T>* tw = (const cplx<T>*)p->lds_tw[pi];
  if (in.logM <= kLdsMaxLog) {
    const int per = kLdsMax >> in.logM;
    const int blocks = (count + per - 1) / per;
    hipLaunchKernelGGL(k_fft_lds<T>, dim3(blocks), dim3(kFftThreads), 0, s, data, in.logM, count,
                       tw, inverse);
  } else {
    const int logW1 = std::min(kLdsMaxLog - in.logM1, in.logM2);
    const int logW2 = std::min(kLdsMaxLog - in.logM2, in.logM1);
    hipLaunchKernelGGL(k_fft4_cols<T>, dim3(1 << (in.logM2 - logW1), count), dim3(kFftThreads), 0,
                       s, data, tmp, in.logM1, in.logM2, tw, (const cplx<T>*)in.tab[pi].tw4_hi,
                       (const cplx<T>*)in.tab[pi].tw4_lo, in.tw4_shift, inverse);
    hipLaunchKernelGGL(k_fft4_rows<T>, dim3(1 << (in.logM1 - logW2), count), dim3(kFftThreads), 0,
                       s, tmp, data, in.logM1, in.logM2, tw, inverse);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- DCT-I plumbing

// Pack pairs of real vectors (components 2p, 2p+1) into the even extension of length L,
// optionally scaling the end points by `endscale` (2 for the E^{-1} pre-factor of the
// transpose) and multiplying by the Bluestein chirp; zero-fill [L, M).
template <typename T>
__global__ void k_pack(const T* __restrict__ x, int nx, int64_t Nn, cplx<T>* __restrict__ z,
                       int64_t L, int64_t M, const cplx<T>* __restrict__ chirp, T endscale) {
  const int pidx = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= M) return;
  cplx<T> val = mk<T>(T(0), T(0));
  if (n < L) {
    const int64_t N = Nn - 1;
    const int64_t k = n <= N ? n : L - n;
    const int c0 = 2 * pidx, c1 = 2 * pidx + 1;
    T a = x[(int64_t)c0 * Nn + k];
    T b = c1 < nx ? x[(int64_t)c1 * Nn + k] : T(0);
    if (k == 0 || k == N) {
      a *= endscale;
      b *= endscale;
    }
    val = mk<T>(a, b);
    if (chirp) val = cmul<T>(val, chirp[n]);
  }
  z[(int64_t)pidx * M + n] = val;
}

template <typename T>
__global__ void k_pointwise(cplx<T>* __restrict__ z, const cplx<T>* __restrict__ f, int64_t M) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= M) return;
  cplx<T>* zz = z + (int64_t)blockIdx.y * M;
  zz[n] = cmul<T>(zz[n], f[n]);
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
// go to `part` (double, per block, two per pair).
template <typename T>
__global__ void k_mid_fwd(const cplx<T>* __restrict__ z, cplx<T>* __restrict__ z2, int64_t N,
                          int64_t L, int64_t M, const cplx<T>* __restrict__ chirp,
                          double* __restrict__ part) {
  const int pidx = blockIdx.y;
  const cplx<T>* zz = z + (int64_t)pidx * M;
  cplx<T>* z2p = z2 + (int64_t)pidx * M;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
      cplx<T> d = mk<T>(rx * sc, ry * sc);
      cplx<T> o = chirp ? cmul<T>(d, chirp[k]) : d;
      z2p[k] = o;
      if (k < N) {
        const int64_t m = L - k;
        z2p[m] = chirp ? cmul<T>(d, chirp[m]) : d;
      }
    }
  }
  // zero fill of the Bluestein padding [L, M)
  for (int64_t m = L + k; m < M; m += (int64_t)gridDim.x * blockDim.x) z2p[m] = mk<T>(T(0), T(0));
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
    part[((int64_t)pidx * gridDim.x + blockIdx.x) * 2 + 0] = r0[0];
    part[((int64_t)pidx * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
  }
}

// d_0 = 2 c^_0 from the partials: one block per pair, fixed-order tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_c0(const double* __restrict__ part, int nblk, cplx<T>* __restrict__ z2,
                                            int64_t N, int64_t M) {
  const int pidx = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    a += part[((int64_t)pidx * nblk + i) * 2 + 0];
    b += part[((int64_t)pidx * nblk + i) * 2 + 1];
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
    const double s = 2.0 / (double)N;
    z2[(int64_t)pidx * M] = mk<T>((T)(ra[0] * s), (T)(rb[0] * s));
  }
}

// Transpose mid stage.  p = C E^{-1} g = Y / 2; q = S M^T S p, i.e.
//   q_0 = p_0 - p_1,   q_1 = (p_0 - p_2) / 4,
//   q_j = -p_0/(j^2-1) + p_{j-1} (1/(2(j-1)) - [j = N]/(2(N+1))) - [j < N] p_{j+1}/(2(j+1)).
template <typename T>
__global__ void k_mid_tr(const cplx<T>* __restrict__ z, cplx<T>* __restrict__ z2, int64_t N,
                         int64_t L, int64_t M, const cplx<T>* __restrict__ chirp) {
  const int pidx = blockIdx.y;
  const cplx<T>* zz = z + (int64_t)pidx * M;
  cplx<T>* z2p = z2 + (int64_t)pidx * M;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    if (j >= 1 && j < N) z2p[L - j] = chirp ? cmul<T>(q, chirp[L - j]) : q;
  }
  for (int64_t m = L + j; m < M; m += (int64_t)gridDim.x * blockDim.x) z2p[m] = mk<T>(T(0), T(0));
}

// Final stage: out_j = scale_j * Y_j for j in [0, N], unpacking the pair.
// forward: scale = 1/2; transpose: scale = e_j / N.
template <typename T>
__global__ void k_final(const cplx<T>* __restrict__ z, T* __restrict__ out, int nx, int64_t Nn,
                        int64_t M, const cplx<T>* __restrict__ chirp, int transpose) {
  const int pidx = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = Nn - 1;
  if (j > N) return;
  cplx<T> Y = dft_value<T>(z + (int64_t)pidx * M, chirp, j);
  T sc;
  if (transpose) sc = ((j == 0 || j == N) ? T(0.5) : T(1)) / T(N);
  else sc = T(0.5);
  const int c0 = 2 * pidx, c1 = 2 * pidx + 1;
  out[(int64_t)c0 * Nn + j] = Y.x * sc;
  if (c1 < nx) out[(int64_t)c1 * Nn + j] = Y.y * sc;
}

template <typename T>
static hipError_t dct_transform(birk_plan* p, const Instance& in, cplx<T>* z, cplx<T>* tmp,
                                hipStream_t s) {
  const int pi = std::is_same<T, double>::value ? 0 : 1;
  hipError_t e = fft_batched<T>(p, in, z, tmp, in.npairs, 0, s);
  if (e != hipSuccess) return e;
  if (in.method == DCT_BLUESTEIN) {
    const int64_t M = in.M;
    hipLaunchKernelGGL(k_pointwise<T>, dim3((unsigned)((M + 255) / 256), in.npairs), dim3(256), 0, s,
                       z, (const cplx<T>*)in.tab[pi].filt, M);
    e = fft_batched<T>(p, in, z, tmp, in.npairs, 1, s);
  }
  return e;
}

template <typename T>
hipError_t apply_product(birk_plan* p, const T* v, T* out, int transpose, hipStream_t s) {
  const int pi = std::is_same<T, double>::value ? 0 : 1;
  for (const Instance& in : p->inst) {
    if (p->use_fast && fast_eligible(in)) {
      hipError_t e = fast_product<T>(p, in, v, out, transpose, s);
      if (e != hipSuccess) return e;
      continue;
    }
    cplx<T>* z = (cplx<T>*)p->work[0] + in.work_off;
    cplx<T>* z2 = (cplx<T>*)p->work[1] + in.work_off;
    cplx<T>* tmp = (cplx<T>*)p->work[2] + in.work_off;
    const cplx<T>* chirp = in.method == DCT_BLUESTEIN ? (const cplx<T>*)in.tab[pi].chirp : nullptr;
    const int64_t M = in.M;
    const T* vi = v + in.off;
    T* oi = out + in.off;
    hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)((M + 255) / 256), in.npairs), dim3(256), 0, s, vi,
                       in.nx, in.Nn, z, in.L, M, chirp, transpose ? T(2) : T(1));
    hipError_t e = dct_transform<T>(p, in, z, tmp, s);
    if (e != hipSuccess) return e;
    const int nblk = in.nblk_mid;
    if (!transpose) {
      double* part = p->partials + in.part_off;
      hipLaunchKernelGGL(k_mid_fwd<T>, dim3(nblk, in.npairs), dim3(256), 0, s, z, z2, in.N, in.L, M,
                         chirp, part);
      hipLaunchKernelGGL(k_c0<T>, dim3(in.npairs), dim3(256), 0, s, part, nblk, z2, in.N, M);
    } else {
      hipLaunchKernelGGL(k_mid_tr<T>, dim3(nblk, in.npairs), dim3(256), 0, s, z, z2, in.N, in.L, M,
                         chirp);
    }
    e = dct_transform<T>(p, in, z2, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final<T>, dim3(nblk, in.npairs), dim3(256), 0, s, z2, oi, in.nx, in.Nn, M,
                       chirp, transpose);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t apply_product<double>(birk_plan*, const double*, double*, int, hipStream_t);
template hipError_t apply_product<float>(birk_plan*, const float*, float*, int, hipStream_t);
template hipError_t fft_batched<double>(const birk_plan*, const Instance&, cplx<double>*, cplx<double>*,
                                        int, int, hipStream_t);
template hipError_t fft_batched<float>(const birk_plan*, const Instance&, cplx<float>*, cplx<float>*,
                                       int, int, hipStream_t);

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

template <typename T>
static hipError_t upload_cplx(const std::vector<double>& re, const std::vector<double>& im, void** dptr) {
  const size_t n = re.size();
  std::vector<T> h(2 * n);
  for (size_t i = 0; i < n; ++i) {
    h[2 * i] = (T)re[i];
    h[2 * i + 1] = (T)im[i];
  }
  hipError_t e = hipMalloc(dptr, 2 * n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dptr, h.data(), 2 * n * sizeof(T), hipMemcpyHostToDevice);
}

static hipError_t upload_both(birk_plan* p, Instance* in, int which, const std::vector<double>& re,
                              const std::vector<double>& im) {
  // which: 0 chirp, 2 tw4_hi, 3 tw4_lo
  for (int pi = 0; pi < 2; ++pi) {
    void** dst = which == 0 ? &in->tab[pi].chirp : (which == 2 ? &in->tab[pi].tw4_hi : &in->tab[pi].tw4_lo);
    hipError_t e = pi == 0 ? upload_cplx<double>(re, im, dst) : upload_cplx<float>(re, im, dst);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
__global__ void k_build_filter(cplx<T>* __restrict__ b, const cplx<T>* __restrict__ chirp, int64_t L,
                               int64_t M) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  cplx<T> v = mk<T>(T(0), T(0));
  if (m < L) {
    v = chirp[m];
    v.y = -v.y;
  } else if (M - m < L) {
    v = chirp[M - m];
    v.y = -v.y;
  }
  b[m] = v;
}

template <typename T>
__global__ void k_scale_to(const cplx<double>* __restrict__ src, cplx<T>* __restrict__ dst, int64_t M,
                           double s) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  dst[m] = mk<T>((T)(src[m].x * s), (T)(src[m].y * s));
}

hipError_t build_tables(birk_plan* p) {
  hipError_t e;
  {
    std::vector<double> re(kLdsMax), im(kLdsMax);
    for (int t = 0; t < kLdsMax; ++t) expi_pi(2 * (int64_t)t, kLdsMax, &re[t], &im[t]);
    for (int pi = 0; pi < 2; ++pi) {
      e = pi == 0 ? upload_cplx<double>(re, im, &p->lds_tw[0]) : upload_cplx<float>(re, im, &p->lds_tw[1]);
      if (e != hipSuccess) return e;
    }
  }
  for (Instance& in : p->inst) {
    if (in.logM > kLdsMaxLog || fast_eligible(in)) {
      const int sh = in.tw4_shift;
      const int64_t nlo = (int64_t)1 << sh, nhi = in.M >> sh;
      std::vector<double> re(nlo), im(nlo);
      for (int64_t t = 0; t < nlo; ++t) expi_pi(2 * t, in.M, &re[t], &im[t]);
      if ((e = upload_both(p, &in, 3, re, im)) != hipSuccess) return e;
      re.assign(nhi, 0.0);
      im.assign(nhi, 0.0);
      for (int64_t t = 0; t < nhi; ++t) expi_pi(2 * (t << sh), in.M, &re[t], &im[t]);
      if ((e = upload_both(p, &in, 2, re, im)) != hipSuccess) return e;
    }
    if (in.method == DCT_BLUESTEIN) {
      // chi_n = exp(-i pi n^2 / L), n in [0, L)
      std::vector<double> re(in.L), im(in.L);
      for (int64_t n = 0; n < in.L; ++n) {
        const int64_t m = (int64_t)(((__int128)n * n) % (2 * in.L));
        expi_pi(m, in.L, &re[n], &im[n]);
      }
      if ((e = upload_both(p, &in, 0, re, im)) != hipSuccess) return e;
      // filter spectrum FFT_M(b) / M in double on the device, then rounded for float
      cplx<double>* b = (cplx<double>*)p->work[0] + in.work_off;
      cplx<double>* tmp = (cplx<double>*)p->work[2] + in.work_off;
      hipLaunchKernelGGL(k_build_filter<double>, dim3((unsigned)((in.M + 255) / 256)), dim3(256), 0,
                         p->stream, b, (const cplx<double>*)in.tab[0].chirp, in.L, in.M);
      if ((e = fft_batched<double>(p, in, b, tmp, 1, 0, p->stream)) != hipSuccess) return e;
      if ((e = hipMalloc(&in.tab[0].filt, in.M * sizeof(cplx<double>))) != hipSuccess) return e;
      if ((e = hipMalloc(&in.tab[1].filt, in.M * sizeof(cplx<float>))) != hipSuccess) return e;
      const double s = 1.0 / (double)in.M;
      hipLaunchKernelGGL(k_scale_to<double>, dim3((unsigned)((in.M + 255) / 256)), dim3(256), 0,
                         p->stream, b, (cplx<double>*)in.tab[0].filt, in.M, s);
      hipLaunchKernelGGL(k_scale_to<float>, dim3((unsigned)((in.M + 255) / 256)), dim3(256), 0,
                         p->stream, b, (cplx<float>*)in.tab[1].filt, in.M, s);
      if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace birk
