// Three-pass fused Birkhoff products for N a power of two (gfx950).
//
// A DCT-I of length N + 1 (eq:vm=DCT-1) is half the length-2N DFT of the even extension
// z of its input.  With 2N = L1 L2, the four-step factorisation n = L2 n1 + n2,
// k = k1 + L1 k2 of that DFT inherits the symmetry of z:
//   * every column n2 (z[L2 n1 + n2] over n1) is real, and column L2 - n2 is column n2
//     reversed, so only columns 0..L2/2 are transformed -- two real columns per complex
//     FFT of length L1 -- and only outputs k1 = 0..L1/2 are kept;
//   * after the twiddle W_2N^(n2 k1), each row k1 is Hermitian in n2 (the output is
//     real), so a row is rebuilt from its half and two rows share one complex FFT of
//     length L2; rows L1 - k1 are mirror images and are never formed.
// Both DCT-I of FastBV (B^a = (2/N) C [E^{-1} S M S E] C, see birk_dct.hip) use this
// scheme, the second with the transposed factorisation (stride L1 first), so that the
// rows produced by the first DCT are exactly the columns the second one needs:
//
//   pass A: columns of DCT 1                       x        -> G  [k1][n2]
//   pass B: rows of DCT 1, the coefficient stencil          G -> G2 [r][q1]
//           (eq:c_k=bydef with the alias of eq:chatk=), columns of DCT 2
//   pass C: rows of DCT 2, plus the constant c^_0 term      G2 -> out
//
// The stencil couples coefficient k with k +- 1, i.e. row k1 with rows k1 +- 1, so a
// pass-B workgroup that owns rows [t0, t0 + TB) also transforms the two neighbouring
// rows (halo).  c^_0 (a reduction over all coefficients) only adds a constant to every
// output (T_0 = 1), so pass B emits partial sums and pass C adds the total.  Three
// round trips through memory per product: read x, write G, read G, write G2, read G2,
// write out.  FFTs are radix-4/2 Stockham in LDS on split real/imaginary rows.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "birk_fft.h"
#include "birk_internal.h"

namespace birk {

namespace fast {

// Twiddles of the radix-8 stages of one FFT length, per thread: a thread's butterfly
// index within its transform depends only on threadIdx (not on which transforms a
// chunk holds), so W^(jm), W^(2 jm), W^(4 jm) of every stage with Ns > 1 are read from
// the table once per kernel and kept in registers; the other powers are products of
// these.  Entry k belongs to the radix-8 stage at logNs = r + 3 k, r = logL mod 3 (3
// when logL mod 3 = 0); for 9 <= logL <= 12 there are at most three such stages.
template <typename T>
struct TwCache {
  cplx<T> w[3][3];
};

__device__ __forceinline__ int tw_base(int logL) {
  const int rem = logL % 3;
  return rem ? rem : 3;
}

template <typename T>
__device__ __forceinline__ void load_twcache(TwCache<T>& c, int logL, const cplx<T>* __restrict__ tw) {
  const int base = tw_base(logL);
#pragma unroll
  for (int k = 0; k < 3; ++k) load_tw_stage<T>(c.w[k], logL, base + 3 * k, tw);
}

// One radix-R Stockham stage on `count` split-complex transforms: transform t has its
// real part in row (first + 2t) and imaginary part in row (first + 2t + 1) of a
// row-major array with `ld` reals per (padded) row.  Each thread owns kPPT / R
// butterflies; all reads of the stage precede all writes.  Radix 2 and 4 occur only as
// the first stage (Ns = 1, no twiddles); radix-8 stages take the thread's cached
// twiddles w = (W^jm, W^2jm, W^4jm) of W = W_(8 Ns).
template <typename T, int R>
__device__ __forceinline__ void split_stage(T* buf, int first, int ld, int logL, int count, int logNs,
                                            const cplx<T> (&w)[3]) {
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  constexpr int NB = kPPT / R;
  const int logNb = logL - logR;
  const int nb = 1 << logNb;
  const int total = count << logNb;
  const int Ns = 1 << logNs;
  T vr[NB][R], vi[NB][R];
  int dst[NB], tt[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * blockDim.x;
    dst[i] = -1;
    tt[i] = 0;
    if (b < total) {
      const int t = b >> logNb;
      const int j = b & (nb - 1);
      const T* re = buf + (first + 2 * t) * ld;
      const T* im = re + ld;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[i][r] = re[pad(j + r * nb)];
        vi[i][r] = im[pad(j + r * nb)];
      }
      const int jm = j & (Ns - 1);
      if constexpr (R == 8) {
        if (jm != 0) {
          const cplx<T> w1 = w[0], w2 = w[1], w4 = w[2];
          const cplx<T> w3 = cmul<T>(w2, w1);
          const cplx<T> w5 = cmul<T>(w4, w1), w6 = cmul<T>(w4, w2), w7 = cmul<T>(w4, w3);
          cmul_inplace<T>(vr[i][1], vi[i][1], w1.x, w1.y);
          cmul_inplace<T>(vr[i][2], vi[i][2], w2.x, w2.y);
          cmul_inplace<T>(vr[i][3], vi[i][3], w3.x, w3.y);
          cmul_inplace<T>(vr[i][4], vi[i][4], w4.x, w4.y);
          cmul_inplace<T>(vr[i][5], vi[i][5], w5.x, w5.y);
          cmul_inplace<T>(vr[i][6], vi[i][6], w6.x, w6.y);
          cmul_inplace<T>(vr[i][7], vi[i][7], w7.x, w7.y);
        }
      }
      dft_reg<T, R>(vr[i], vi[i]);
      dst[i] = ((j >> logNs) << (logNs + logR)) + jm;
      tt[i] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (dst[i] >= 0) {
      T* re = buf + (first + 2 * tt[i]) * ld;
      T* im = re + ld;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        re[pad(dst[i] + r * Ns)] = vr[i][r];
        im[pad(dst[i] + r * Ns)] = vi[i][r];
      }
    }
  }
  __syncthreads();
}

// `count` transforms of length 2^logL (9 <= logL <= 12) that fit kPPT * blockDim.x
// complex points: a first stage of radix 2, 4 or 8 (logL mod 3 = 1, 2, 0; Ns = 1, no
// twiddles), then radix-8 stages with the cached twiddles.
template <typename T>
__device__ __forceinline__ void split_fft_chunk(T* buf, int first, int ld, int logL, int count,
                                                const TwCache<T>& tc) {
  const int rem = logL % 3;
  if (rem == 1) split_stage<T, 2>(buf, first, ld, logL, count, 0, tc.w[0]);
  else if (rem == 2) split_stage<T, 4>(buf, first, ld, logL, count, 0, tc.w[0]);
  else split_stage<T, 8>(buf, first, ld, logL, count, 0, tc.w[0]);
  const int base = tw_base(logL);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int logNs = base + 3 * k;
    if (logNs < logL) split_stage<T, 8>(buf, first, ld, logL, count, logNs, tc.w[k]);
  }
}

// The same with the twiddles of each stage read from the table just before it (fewer
// registers than a TwCache held through the kernel).
template <typename T>
__device__ __forceinline__ void split_fft_chunk_tab(T* buf, int first, int ld, int logL, int count,
                                                    const cplx<T>* __restrict__ tw) {
  const int rem = logL % 3;
  cplx<T> w[3];
  if (rem == 1) split_stage<T, 2>(buf, first, ld, logL, count, 0, w);
  else if (rem == 2) split_stage<T, 4>(buf, first, ld, logL, count, 0, w);
  else split_stage<T, 8>(buf, first, ld, logL, count, 0, w);
  const int base = tw_base(logL);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int logNs = base + 3 * k;
    if (logNs < logL) {
      load_tw_stage<T>(w, logL, logNs, tw);
      split_stage<T, 8>(buf, first, ld, logL, count, logNs, w);
    }
  }
}

// Any number of transforms, in chunks of whole transforms.
template <typename T>
__device__ __forceinline__ void split_fft(T* buf, int first, int ld, int logL, int count, const TwCache<T>& tc) {
  const int per = max(1, (kPPT * (int)blockDim.x) >> logL);
#pragma nounroll
  for (int t0 = 0; t0 < count; t0 += per)
    split_fft_chunk<T>(buf, first + 2 * t0, ld, logL, min(per, count - t0), tc);
}

// Tile of a one-dimensional grid of nt tiles per component and nc components, mapped
// so that each XCD (workgroups are dealt to the 8 XCDs round robin) runs a contiguous
// range of tiles: neighbouring tiles, which share cache lines at their edges, then
// meet in one L2.
__device__ __forceinline__ void xcd_tile(int nt, int nc, int xcd_order, int& comp, int& tile) {
  if (!xcd_order) {
    comp = (int)blockIdx.x / nt;
    tile = (int)blockIdx.x - comp * nt;
    return;
  }
  const int total = nt * nc;
  const int lid = (int)blockIdx.x;
  const int xcd = lid & 7, idx = lid >> 3;
  const int q = total >> 3, r = total & 7;
  const int L = xcd * q + min(xcd, r) + idx;
  comp = L / nt;
  tile = L - comp * nt;
}

// Separate the DFTs of two real sequences a, b from F = DFT(a + i b):
//   Fa[k] = (F[k] + conj F[-k]) / 2,  Fb[k] = (F[k] - conj F[-k]) / (2i)
template <typename T>
__device__ __forceinline__ cplx<T> separate(T fr, T fi, T mr, T mi, int second) {
  const T h = T(0.5);
  return second ? mk<T>(h * (fi + mi), h * (mr - fr)) : mk<T>(h * (fr + mr), h * (fi - mi));
}

// Sum over the block for any blockDim.x that is a multiple of 64 (<= 1024): wavefront
// butterfly with shuffles, then the per-wave sums in a fixed order.  Every thread gets
// the total.  `red` needs blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int nw = (int)(blockDim.x >> 6);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += red[i];
  __syncthreads();
  return r;
}

// Global-memory phases process kUnroll elements per thread per batch: all loads of a
// batch are issued before any of them is consumed, so each thread keeps several
// requests in flight instead of one.
constexpr int kUnroll = 8;
constexpr int kUnrollB = 4;  // pass B keeps four complex values per element in flight

// ---------------------------------------------------------------- pass A
// Columns n2 in [c0, c0 + W) of the even extension of x (optionally with both end
// points doubled: the E^{-1} pre-factor of the transpose), FFT over n1, keep k1 <= L1/2,
// twiddle W_2N^(n2 k1), store G[k1][n2] for n2 <= L2/2.  W is a power of two.
template <typename T>
__global__ __launch_bounds__(512) void k_fastA(const T* __restrict__ x, int64_t Nn, int logL1, int logL2, int logW,
                                               cplx<T>* __restrict__ G, int64_t gcomp, int64_t sg,
                                               const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ thi,
                                               const cplx<T>* __restrict__ tlo, int tsh, int ends2, int nt, int nc,
                                               int xcd_order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* A = reinterpret_cast<T*>(smem_raw);
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  TwCache<T> tc;
  load_twcache<T>(tc, logL1, tw);
  const T* xc = x + (int64_t)comp * Nn;
  const int N = (int)(Nn - 1), N2 = 2 * N;
  const int L1 = 1 << logL1, L2 = 1 << logL2;
  const int W = 1 << logW;
  const int c0 = tile * W;
  const int ld1 = padded_ld(L1);
  const int n = W << logL1;
  for (int base = threadIdx.x; base < n; base += kUnroll * blockDim.x) {
    T val[kUnroll];
    int dst[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = base + u * blockDim.x;
      dst[u] = -1;
      if (e < n) {
        const int w = e & (W - 1), n1 = e >> logW;
        const int m = (n1 << logL2) + c0 + w;
        const int idx = m <= N ? m : N2 - m;
        val[u] = xc[idx];
        if (ends2 && (idx == 0 || idx == N)) val[u] *= T(2);
        dst[u] = w * ld1 + pad(n1);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (dst[u] >= 0) A[dst[u]] = val[u];
  }
  __syncthreads();
  split_fft_chunk<T>(A, 0, ld1, logL1, W / 2, tc);
  const int half1 = L1 / 2;
  cplx<T>* Gc = G + (int64_t)comp * gcomp;
  const int nout = (half1 + 1) << logW;
  const int tmask = (1 << tsh) - 1;
  for (int base = threadIdx.x; base < nout; base += kUnroll * blockDim.x) {
    cplx<T> wh[kUnroll], wl[kUnroll], v[kUnroll];
    int gi[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = base + u * blockDim.x;
      gi[u] = -1;
      const int w = e & (W - 1), k1 = e >> logW;
      const int n2 = c0 + w;
      if (e < nout && n2 <= L2 / 2) {
        const int t = n2 * k1;
        wh[u] = thi[t >> tsh];
        wl[u] = tlo[t & tmask];
        const T* re = A + (w & ~1) * ld1;
        const T* im = re + ld1;
        const int km = (L1 - k1) & (L1 - 1);
        v[u] = separate<T>(re[pad(k1)], im[pad(k1)], re[pad(km)], im[pad(km)], w & 1);
        gi[u] = k1 * (int)sg + n2;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (gi[u] >= 0) Gc[gi[u]] = cmul<T>(v[u], cmul<T>(wh[u], wl[u]));
  }
}

// ---------------------------------------------------------------- pass B
// Source of the Hermitian row that reproduces Y_ext[k1 + L1 m] (m in [0, L2)) for any
// k1 in [-1, L1): rows 0..L1/2 are stored; row -1 is row 1 read backwards (conjugate
// input); rows above L1/2 are mirrors of row L1 - k1 read backwards with a shift of one
// (conjugate input times W_L2^n2).  mode: 0 plain, 1 conjugate, 2 conjugate + twiddle.
__device__ __forceinline__ int hrow_src(int k1, int L1, int* mode) {
  if (k1 < 0) {
    *mode = 1;
    return 1;
  }
  if (k1 <= L1 / 2) {
    *mode = 0;
    return k1;
  }
  *mode = 2;
  return L1 - k1;
}

// Forward stencil (FastBV step 2 with the reversals folded into signs):
//   d_k = (-1)^k c^_k / e_k with c^ from eq:c_k=bydef and eq:chatk= applied to the
//   Chebyshev coefficients a_k = (-1)^k e_k Y_k / N; d_0 is deferred (c^_0 term).
//   invN = 1/N, inv4N1 = 1/(4 (N + 1)).
template <typename T>
__device__ __forceinline__ T stencil_fwd(int k, int N, T Ym, T Yp, T invN, T inv4N1) {
  if (k == 0) return T(0);
  const T i2k = T(1) / T(2 * k);
  const T lo = (k == 1) ? T(1) : i2k;
  const T em1 = (k == 1) ? T(0.5) : T(1);
  T r = -lo * em1 * Ym;
  if (k < N) {
    const T ep1 = (k + 1 == N) ? T(0.5) : T(1);
    r += ep1 * Yp * i2k;
  }
  if (k == N - 1) r -= Yp * inv4N1;
  const T sc = (k == N) ? T(2) : T(1);
  return r * invN * sc;
}

// Transpose stencil: q = S M^T S p with p = Y / 2 (see birk_dct.hip, k_mid_tr).
//   inv2N1 = 1/(2 (N + 1)).
template <typename T>
__device__ __forceinline__ T stencil_tr(int j, int N, T Ym, T Yp, T p0, T inv2N1) {
  const T h = T(0.5);
  if (j == 0) return p0 - h * Yp;
  if (j == 1) return T(0.25) * (p0 - h * Yp);
  const T jj = T(j);
  T cm = T(1) / (T(2) * (jj - T(1)));
  if (j == N) cm -= inv2N1;
  T q = -p0 / ((jj - T(1)) * (jj + T(1))) + cm * h * Ym;
  if (j < N) q -= h * Yp / (T(2) * (jj + T(1)));
  return q;
}

// c^_0 = (1/N) [ e_0 Y_0 + Y_1 / 4 - sum_{k >= 2} e_k Y_k / (k^2 - 1) ]
__device__ __forceinline__ double c0_coef(int k, int N) {
  if (k == 0) return 0.5;
  if (k == 1) return 0.25;
  const double ek = (k == N) ? 0.5 : 1.0;
  return -ek / (((double)k - 1.0) * ((double)k + 1.0));
}

template <typename T, int TB, int TRANS>
__global__ __launch_bounds__(512) void k_fastB(const cplx<T>* __restrict__ G, int64_t gcomp, int64_t sg,
                                               cplx<T>* __restrict__ G2, int64_t g2comp, int64_t sg2, int64_t N64,
                                               int logL1, int logL2, const cplx<T>* __restrict__ tw,
                                               const cplx<T>* __restrict__ thi, const cplx<T>* __restrict__ tlo,
                                               int tsh, double* __restrict__ part, int nt, int nc,
                                               int xcd_order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Y = reinterpret_cast<T*>(smem_raw);  // (TB + 2) real rows of L2
  __shared__ double red[16];
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  TwCache<T> tc;
  load_twcache<T>(tc, logL2, tw);
  const int N = (int)N64;
  const int L1 = 1 << logL1, L2 = 1 << logL2;
  const int half2 = L2 / 2;
  const int t0 = tile * TB;
  const int ld2 = padded_ld(L2);
  const int sgi = (int)sg;
  const cplx<T>* Gc = G + (int64_t)comp * gcomp;
  constexpr int NR = TB + 2;
  // rows rho = 0..TB+1 <-> k1 = t0 - 1 + rho; pairs (2i, 2i+1) share one complex FFT
  const int hp1 = half2 + 1;
  const int nin = (NR / 2) * hp1;
  const int twsh = kLdsMaxLog - logL2;
  for (int base = threadIdx.x; base < nin; base += kUnrollB * blockDim.x) {
    cplx<T> ra[kUnrollB], rb[kUnrollB], wa[kUnrollB], wb[kUnrollB];
    int ma[kUnrollB], mb[kUnrollB], pr_[kUnrollB], n2_[kUnrollB];
#pragma unroll
    for (int u = 0; u < kUnrollB; ++u) {
      const int e = base + u * blockDim.x;
      pr_[u] = -1;
      if (e < nin) {
        const int pr = e / hp1, n2 = e - pr * hp1;
        const int sa = hrow_src(t0 - 1 + 2 * pr, L1, &ma[u]);
        const int sb = hrow_src(t0 + 2 * pr, L1, &mb[u]);
        ra[u] = Gc[sa * sgi + n2];
        rb[u] = Gc[sb * sgi + n2];
        wa[u] = tw[(ma[u] == 2 ? n2 : 0) << twsh];
        wb[u] = tw[(mb[u] == 2 ? n2 : 0) << twsh];
        pr_[u] = pr;
        n2_[u] = n2;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnrollB; ++u) {
      if (pr_[u] < 0) continue;
      cplx<T> a = ra[u], b = rb[u];
      if (ma[u]) a = conjg<T>(a);
      if (ma[u] == 2) a = cmul<T>(a, wa[u]);
      if (mb[u]) b = conjg<T>(b);
      if (mb[u] == 2) b = cmul<T>(b, wb[u]);
      const int n2 = n2_[u];
      T* re = Y + (2 * pr_[u]) * ld2;
      T* im = re + ld2;
      re[pad(n2)] = a.x - b.y;
      im[pad(n2)] = a.y + b.x;
      if (n2 > 0 && n2 < half2) {
        re[pad(L2 - n2)] = a.x + b.y;
        im[pad(L2 - n2)] = b.x - a.y;
      }
    }
  }
  T p0 = T(0);
  if (TRANS) {
    // Y_0 of the first DCT is the sum of row 0 of the Hermitian G: p_0 = Y_0 / 2
    double acc = 0.0;
    for (int n2 = threadIdx.x; n2 <= half2; n2 += blockDim.x)
      acc += (double)Gc[n2].x * ((n2 == 0 || n2 == half2) ? 1.0 : 2.0);
    p0 = (T)(0.5 * block_sum(acc, red));
  }
  __syncthreads();
  split_fft<T>(Y, 0, ld2, logL2, NR / 2, tc);
  // stencil, one thread per m (owns column m of the tile: no cross-thread hazard)
  double c0acc = 0.0;
  const int N2 = 2 * N;
  const T invN = T(1) / T(N), inv4N1 = T(1) / T(4 * (int64_t)N + 4), inv2N1 = T(1) / T(2 * (int64_t)N + 2);
  for (int m = threadIdx.x; m < L2; m += blockDim.x) {
    T yv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) yv[r] = Y[r * ld2 + pad(m)];
#pragma unroll
    for (int r = 1; r <= TB; ++r) {
      const int k1 = t0 - 1 + r;
      const int K = k1 + L1 * m;
      const bool lowhalf = K <= N;
      const int k = lowhalf ? K : N2 - K;
      const T Ym = lowhalf ? yv[r - 1] : yv[r + 1];
      const T Yp = lowhalf ? yv[r + 1] : yv[r - 1];
      T d;
      if (TRANS) {
        d = stencil_tr<T>(k, N, Ym, Yp, p0, inv2N1);
      } else {
        d = stencil_fwd<T>(k, N, Ym, Yp, invN, inv4N1);
        if (k1 <= L1 / 2 && ((k1 != 0 && k1 != L1 / 2) || lowhalf)) c0acc += c0_coef(k, N) * (double)yv[r];
      }
      Y[r * ld2 + pad(m)] = d;
    }
  }
  if (!TRANS) {
    const double tot = block_sum(c0acc, red);
    if (threadIdx.x == 0) part[(int64_t)comp * nt + tile] = tot;
  }
  __syncthreads();
  // columns of the second DCT: d rows (1 + 2i, 2 + 2i) as one complex FFT each
  split_fft<T>(Y, 1, ld2, logL2, TB / 2, tc);
  cplx<T>* G2c = G2 + (int64_t)comp * g2comp;
  const int nout = hp1 * TB;
  const int tmask = (1 << tsh) - 1;
  const int sg2i = (int)sg2;
  for (int base = threadIdx.x; base < nout; base += kUnrollB * blockDim.x) {
    cplx<T> wh[kUnrollB], wl[kUnrollB], v[kUnrollB];
    int gi[kUnrollB];
#pragma unroll
    for (int u = 0; u < kUnrollB; ++u) {
      const int e = base + u * blockDim.x;
      gi[u] = -1;
      const int rl = e / hp1, q = e - rl * hp1;
      const int r = t0 + rl;
      if (e < nout && r <= L1 / 2) {
        const int t = r * q;
        wh[u] = thi[t >> tsh];
        wl[u] = tlo[t & tmask];
        const T* re = Y + (1 + (rl & ~1)) * ld2;
        const T* im = re + ld2;
        const int qm = (L2 - q) & (L2 - 1);
        v[u] = separate<T>(re[pad(q)], im[pad(q)], re[pad(qm)], im[pad(qm)], rl & 1);
        gi[u] = r * sg2i + q;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnrollB; ++u)
      if (gi[u] >= 0) G2c[gi[u]] = cmul<T>(v[u], cmul<T>(wh[u], wl[u]));
  }
}

// Pass B for rows of L2 = 2^LOGL2 (512..2048) points, blockDim = L2 / 8, TB = 2 or 4
// rows per tile.  One LDS buffer holds one complex row transform at a time: the pairs
// of DCT-1 rows (t0 - 1 + 2p, t0 + 2p), p = 0..TB/2, are transformed one after the other
// and each thread keeps its eight outputs m = tid + i blockDim of every row in
// registers, so the stencil of rows t0..t0+TB-1 runs in registers; the pairs
// d(t0 + 2q) + i d(t0 + 2q + 1) then go back through the buffer for the column transforms
// of DCT 2.  The small LDS footprint (one row pair) lets several workgroups share a CU,
// which hides the latency of the load / transform / store phases.
template <typename T, int TRANS, int LOGL2, int TB>
__global__ __launch_bounds__(1 << (LOGL2 - 3)) void k_fastB2(
    const cplx<T>* __restrict__ G, int64_t gcomp, int64_t sg, cplx<T>* __restrict__ G2, int64_t g2comp, int64_t sg2,
    int64_t N64, int logL1, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ thi,
    const cplx<T>* __restrict__ tlo, int tsh, double* __restrict__ part, int nt, int nc, int xcd_order) {
  constexpr int L2 = 1 << LOGL2;
  constexpr int NTHR = L2 / kPPT;
  constexpr int half2 = L2 / 2, hp1 = half2 + 1;
  constexpr int ld2 = padded_ld(L2);
  constexpr int twsh = kLdsMaxLog - LOGL2;
  constexpr int NP = TB / 2 + 1;  // DCT-1 row pairs (TB rows and the two halo rows)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Yre = reinterpret_cast<T*>(smem_raw);  // one complex row: real part, imaginary part
  T* Yim = Yre + ld2;
  __shared__ double red[16];
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  const int N = (int)N64;
  const int L1 = 1 << logL1;
  const int t0 = TB * tile;
  const int sgi = (int)sg;
  const cplx<T>* Gc = G + (int64_t)comp * gcomp;
  T p0 = T(0);
  if (TRANS) {
    // Y_0 of the first DCT is the sum of row 0 of the Hermitian G: p_0 = Y_0 / 2
    double acc = 0.0;
    for (int n2 = threadIdx.x; n2 <= half2; n2 += NTHR)
      acc += (double)Gc[n2].x * ((n2 == 0 || n2 == half2) ? 1.0 : 2.0);
    p0 = (T)(0.5 * block_sum(acc, red));
  }
  // DCT-1 rows: y[rho][i] = row t0 - 1 + rho at m = tid + i NTHR, rho = 0..TB+1.  The
  // loads of row pair pp + 1 are issued before the FFT of pair pp, so that they are in
  // flight while it runs.
  T y[2 * NP][kPPT];
  constexpr int per = (hp1 + NTHR - 1) / NTHR;  // half-row elements per thread (5)
  cplx<T> na[per], nb[per];
  int nma, nmb;
  {
    const int sa = hrow_src(t0 - 1, L1, &nma);
    const int sb = hrow_src(t0, L1, &nmb);
#pragma unroll
    for (int u = 0; u < per; ++u) {
      const int n2 = (int)threadIdx.x + u * NTHR;
      if (n2 < hp1) {
        na[u] = Gc[sa * sgi + n2];
        nb[u] = Gc[sb * sgi + n2];
      }
    }
  }
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    const int ma = nma, mb = nmb;
#pragma unroll
    for (int u = 0; u < per; ++u) {
      const int n2 = (int)threadIdx.x + u * NTHR;
      if (n2 < hp1) {
        cplx<T> a = na[u], b = nb[u];
        if (ma) a = conjg<T>(a);
        if (ma == 2) a = cmul<T>(a, tw[n2 << twsh]);
        if (mb) b = conjg<T>(b);
        if (mb == 2) b = cmul<T>(b, tw[n2 << twsh]);
        Yre[pad(n2)] = a.x - b.y;
        Yim[pad(n2)] = a.y + b.x;
        if (n2 > 0 && n2 < half2) {
          Yre[pad(L2 - n2)] = a.x + b.y;
          Yim[pad(L2 - n2)] = b.x - a.y;
        }
      }
    }
    if (pp + 1 < NP) {
      const int sa = hrow_src(t0 + 1 + 2 * pp, L1, &nma);
      const int sb = hrow_src(t0 + 2 + 2 * pp, L1, &nmb);
#pragma unroll
      for (int u = 0; u < per; ++u) {
        const int n2 = (int)threadIdx.x + u * NTHR;
        if (n2 < hp1) {
          na[u] = Gc[sa * sgi + n2];
          nb[u] = Gc[sb * sgi + n2];
        }
      }
    }
    __syncthreads();
    fft_ct<T, LOGL2, 1>(Yre, tw);
#pragma unroll
    for (int i = 0; i < kPPT; ++i) {
      const int m = (int)threadIdx.x + i * NTHR;
      y[2 * pp][i] = Yre[pad(m)];
      y[2 * pp + 1][i] = Yim[pad(m)];
    }
    __syncthreads();
  }
  // stencil of rows t0 + rl (rho = rl + 1, neighbours rho - 1 and rho + 1)
  double c0acc = 0.0;
  const int N2 = 2 * N;
  const T invN = T(1) / T(N), inv4N1 = T(1) / T(4 * (int64_t)N + 4), inv2N1 = T(1) / T(2 * (int64_t)N + 2);
  T dv[TB][kPPT];
#pragma unroll
  for (int i = 0; i < kPPT; ++i) {
    const int m = (int)threadIdx.x + i * NTHR;
#pragma unroll
    for (int rl = 0; rl < TB; ++rl) {
      const int k1 = t0 + rl;
      const T ylo = y[rl][i];      // row k1 - 1
      const T ymid = y[rl + 1][i]; // row k1
      const T yhi = y[rl + 2][i];  // row k1 + 1
      const int K = k1 + L1 * m;
      const bool lowhalf = K <= N;
      const int k = lowhalf ? K : N2 - K;
      const T Ym = lowhalf ? ylo : yhi;
      const T Yp = lowhalf ? yhi : ylo;
      if (TRANS) {
        dv[rl][i] = stencil_tr<T>(k, N, Ym, Yp, p0, inv2N1);
      } else {
        dv[rl][i] = stencil_fwd<T>(k, N, Ym, Yp, invN, inv4N1);
        if (k1 <= L1 / 2 && ((k1 != 0 && k1 != L1 / 2) || lowhalf)) c0acc += c0_coef(k, N) * (double)ymid;
      }
    }
  }
  if (!TRANS) {
    const double tot = block_sum(c0acc, red);
    if (threadIdx.x == 0) part[(int64_t)comp * nt + tile] = tot;
  }
  cplx<T>* G2c = G2 + (int64_t)comp * g2comp;
  const int tmask = (1 << tsh) - 1;
  const int sg2i = (int)sg2;
  // column transforms of DCT 2 on d(t0 + 2q) + i d(t0 + 2q + 1)
#pragma unroll
  for (int qq = 0; qq < TB / 2; ++qq) {
#pragma unroll
    for (int i = 0; i < kPPT; ++i) {
      const int m = (int)threadIdx.x + i * NTHR;
      Yre[pad(m)] = dv[2 * qq][i];
      Yim[pad(m)] = dv[2 * qq + 1][i];
    }
    __syncthreads();
    fft_ct<T, LOGL2, 1>(Yre, tw);
#pragma unroll
    for (int rl = 0; rl < 2; ++rl) {
      const int r = t0 + 2 * qq + rl;
      if (r > L1 / 2) continue;
      constexpr int per = (hp1 + NTHR - 1) / NTHR;
#pragma unroll
      for (int u = 0; u < per; ++u) {
        const int q = (int)threadIdx.x + u * NTHR;
        if (q < hp1) {
          const int t = r * q;
          const cplx<T> w = cmul<T>(thi[t >> tsh], tlo[t & tmask]);
          const int qm = (L2 - q) & (L2 - 1);
          const cplx<T> v = separate<T>(Yre[pad(q)], Yim[pad(q)], Yre[pad(qm)], Yim[pad(qm)], rl);
          G2c[r * sg2i + q] = cmul<T>(v, w);
        }
      }
    }
    __syncthreads();
  }
}

// Reciprocal of a positive integer-valued x: the hardware estimate refined by two Newton
// steps in double (within an ulp of 1/x, several times cheaper than a division); a plain
// division for the other storage types.
template <typename T>
__device__ __forceinline__ T recip_int(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ double recip_int<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// stencil_fwd and stencil_tr with one or two reciprocals per element in place of their
// divisions (same formulas).
template <typename T>
__device__ __forceinline__ T stencil_fwd_r(int k, int N, T Ym, T Yp, T invN, T inv4N1) {
  if (k == 0) return T(0);
  const T i2k = recip_int<T>(T(2 * k));
  const T lo = (k == 1) ? T(1) : i2k;
  const T em1 = (k == 1) ? T(0.5) : T(1);
  T r = -lo * em1 * Ym;
  if (k < N) {
    const T ep1 = (k + 1 == N) ? T(0.5) : T(1);
    r += ep1 * Yp * i2k;
  }
  if (k == N - 1) r -= Yp * inv4N1;
  const T sc = (k == N) ? T(2) : T(1);
  return r * invN * sc;
}

template <typename T>
__device__ __forceinline__ T stencil_tr_r(int j, int N, T Ym, T Yp, T p0, T inv2N1) {
  const T h = T(0.5);
  if (j == 0) return p0 - h * Yp;
  if (j == 1) return T(0.25) * (p0 - h * Yp);
  const T rm = recip_int<T>(T(j - 1)), rp = recip_int<T>(T(j + 1));
  T cm = h * rm;
  if (j == N) cm -= inv2N1;
  T q = -p0 * rm * rp + cm * h * Ym;
  if (j < N) q -= T(0.25) * Yp * rp;
  return q;
}

// Pass B for rows of L2 = 2^LOGL2 (512..2048) points, TB rows per tile (2 or 4), blockDim
// = L2 / 8, with the row transforms kept in registers at both ends (fft_regs): each thread
// builds its eight elements m = tid + i blockDim of a Hermitian row pair straight from G
// (the elements above L2/2 from their mirror images, so each G value is read by two
// threads), runs the first butterflies in registers, and receives its outputs
// m = tid + i blockDim of the last stage in registers, which is the layout the stencil and
// the second DCT's column transform use.  Only the stages in between, and the mirror
// reads of the final separation, go through LDS.
//
// The stencil of rows k1, k1 + 1 reads Y of rows k1 - 1 .. k1 + 2 at the same m.
// * Forward: d_k = +-(Y_{k+1} - Y_{k-1}) / (2 k N) for every k in [1, N - 2], so by
//   linearity one FFT of the row differences G(k1 + 1) - G(k1 - 1), G(k1 + 2) - G(k1)
//   gives the stencil of both rows.  The three other coefficients lie in the first tile:
//   d_0 = 0, and d_N, d_{N-1} need Y_{N-2}, Y_{N-1}, Y_N, which are element L2/2 of rows
//   2, 1, 0, i.e. alternating sums over those rows (block reductions).  c^_0 makes the
//   integral vanish at the first node, where every T_k is 1 after the sign folding:
//   c^_0 = -(d_1 + ... + d_{N-1} + d_N / 2) with d_N as stored (already doubled), so the
//   partial sums add the stencil outputs (each k once: rows 1..L1/2 - 1 in full, rows 0
//   and L1/2 for K <= N) and are scaled by N, the form pass C divides out.
// * Transpose (Y_{k-1} and Y_{k+1} weighted differently): the tile's rows are swept in
//   pairs with a rolling window: DCT-1 row pair (t0 + 2q + 1, t0 + 2q + 2) joins the pair
//   before it, the stencil of rows t0 + 2q, t0 + 2q + 1 follows, then their DCT-2 column
//   transform and store; so TB rows cost TB/2 + 1 DCT-1 and TB/2 DCT-2 transforms.
template <typename T, int TRANS, int LOGL2, int TB>
__global__ __launch_bounds__(1 << (LOGL2 - 3)) void k_fastB3(
    const cplx<T>* __restrict__ G, int64_t gcomp, int64_t sg, cplx<T>* __restrict__ G2, int64_t g2comp, int64_t sg2,
    int64_t N64, int logL1, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ thi,
    const cplx<T>* __restrict__ tlo, int tsh, const cplx<double>* __restrict__ thd,
    const cplx<double>* __restrict__ tld, double* __restrict__ part, int nt, int nc, int xcd_order) {
  constexpr int L2 = 1 << LOGL2;
  constexpr int NTHR = L2 / kPPT;
  constexpr int half2 = L2 / 2, hp1 = half2 + 1;
  constexpr int ld2 = padded_ld(L2);
  constexpr int twsh = kLdsMaxLog - LOGL2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Yre = reinterpret_cast<T*>(smem_raw);  // one complex row: real part, imaginary part
  T* Yim = Yre + ld2;
  __shared__ double red[16];
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  const int N = (int)N64;
  const int L1 = 1 << logL1;
  const int t0 = TB * tile;
  const int sgi = (int)sg;
  const int t = (int)threadIdx.x;
  const cplx<T>* Gc = G + (int64_t)comp * gcomp;
  cplx<T>* G2c = G2 + (int64_t)comp * g2comp;
  const int tmask = (1 << tsh) - 1;
  const int sg2i = (int)sg2;
  const int N2 = 2 * N;
  const T invN = T(1) / T(N), inv4N1 = T(1) / T(4 * (int64_t)N + 4), inv2N1 = T(1) / T(2 * (int64_t)N + 2);
  // a + i b of two Hermitian rows at element m (values aa, bb of the stored half)
  auto pack = [&](int m, T ax, T ay, T bx, T by, T& vr, T& vi) {
    if (m <= half2) {
      vr = ax - by;
      vi = ay + bx;
    } else {
      vr = ax + by;
      vi = bx - ay;
    }
  };
  // column transform of DCT 2 on d(k1) + i d(k1 + 1); the separation needs the mirror
  // element L2 - q, held by another thread, so the outputs go through LDS once
  auto dct2_store = [&](int k1, T (&dr)[kPPT], T (&di)[kPPT]) {
    // double and float: the twiddles W_2N^(r qq), qq = t + u NTHR, of row r are W_2N^(r t)
    // times powers of W_2N^(r NTHR); the four reads of the double table are issued before
    // the transform and the powers are formed in double
    constexpr bool kStep = std::is_floating_point<T>::value;
    cplx<double> wb[2], wst[2];
    if constexpr (kStep) {
#pragma unroll
      for (int rl = 0; rl < 2; ++rl) {
        const int r = k1 + rl, ta = r * t, tb = r * NTHR;
        wb[rl] = cmul<double>(thd[ta >> tsh], tld[ta & tmask]);
        wst[rl] = cmul<double>(thd[tb >> tsh], tld[tb & tmask]);
      }
    }
    fft_regs<T, LOGL2>(Yre, dr, di, tw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPPT; ++i) {
      const int m = t + i * NTHR;
      Yre[pad(m)] = dr[i];
      Yim[pad(m)] = di[i];
    }
    __syncthreads();
    constexpr int per = (hp1 + NTHR - 1) / NTHR;  // 5
#pragma unroll
    for (int u = 0; u < per; ++u) {
      const int qq = t + u * NTHR;
      if (qq < hp1) {
        const int qm = (L2 - qq) & (L2 - 1);
        const T mr = Yre[pad(qm)], mi = Yim[pad(qm)];
#pragma unroll
        for (int rl = 0; rl < 2; ++rl) {
          const int r = k1 + rl;
          if (r > L1 / 2) continue;
          const int tt = r * qq;
          const cplx<T> w = kStep ? mk<T>((T)wb[rl].x, (T)wb[rl].y) : cmul<T>(thi[tt >> tsh], tlo[tt & tmask]);
          const cplx<T> v = separate<T>(dr[u], di[u], mr, mi, rl);
          G2c[r * sg2i + qq] = cmul<T>(v, w);
        }
      }
      if constexpr (kStep) {
#pragma unroll
        for (int rl = 0; rl < 2; ++rl) wb[rl] = cmul<double>(wb[rl], wst[rl]);
      }
    }
  };
  if constexpr (!TRANS) {
    double c0acc = 0.0;
#pragma unroll
    for (int q = 0; q < TB / 2; ++q) {
      const int k1 = t0 + 2 * q;
      const bool first = k1 == 0;
      // DCT-1 transform of the row differences; rows k1 - 1 .. k1 + 2 read in two halves
      // of four elements (as many loads in flight as one row pair of eight); the first
      // tile also sums rows 0, 1, 2 with alternating signs ((-1)^m = (-1)^t)
      T dr[kPPT], di[kPPT];
      double alt[3] = {0.0, 0.0, 0.0};
      {
        int mo[4];
        const cplx<T>* g[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) g[r] = Gc + (int64_t)hrow_src(k1 - 1 + r, L1, &mo[r]) * sgi;
#pragma unroll
        for (int h = 0; h < kPPT; h += 4) {
          cplx<T> x[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = t + (h + u) * NTHR;
            const int gi = m <= half2 ? m : L2 - m;
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r][u] = g[r][gi];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = t + (h + u) * NTHR;
            const int gi = m <= half2 ? m : L2 - m;
            cplx<T> y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              y[r] = x[r][u];
              if (mo[r]) y[r] = conjg<T>(y[r]);
              if (mo[r] == 2) y[r] = cmul<T>(y[r], tw[gi << twsh]);
            }
            if (first) {
#pragma unroll
              for (int r = 0; r < 3; ++r) alt[r] += (double)y[r + 1].x;
            }
            pack(m, y[2].x - y[0].x, y[2].y - y[0].y, y[3].x - y[1].x, y[3].y - y[1].y, dr[h + u], di[h + u]);
          }
        }
      }
      fft_regs<T, LOGL2>(Yre, dr, di, tw);
      T yN = T(0), yN1 = T(0), yN2 = T(0);  // Y_N, Y_{N-1}, Y_{N-2}
      if (first) {
        const double sgn = (t & 1) ? -1.0 : 1.0;
        yN = (T)block_sum(sgn * alt[0], red);
        yN1 = (T)block_sum(sgn * alt[1], red);
        yN2 = (T)block_sum(sgn * alt[2], red);
      }
      // stencil of rows k1 (dr) and k1 + 1 (di), in place; K = k1 + rl + L1 m <= N exactly
      // when m < L2 / 2, i.e. for the thread's elements i < 4, except K = N (row 0, m = L2/2)
#pragma unroll
      for (int i = 0; i < kPPT; ++i) {
        const int m = t + i * NTHR;
#pragma unroll
        for (int rl = 0; rl < 2; ++rl) {
          const int kr = k1 + rl;
          const int K = kr + L1 * m;
          const int k = i < 4 ? K : N2 - K;
          const T D = rl ? di[i] : dr[i];
          T d = (i < 4 ? D : -D) * recip_int<T>(T(2 * k)) * invN;
          double wc = (kr < L1 / 2 || (kr == L1 / 2 && i < 4)) ? 1.0 : 0.0;  // weight in c^_0
          if (first && i == 0 && rl == 0 && t == 0) d = T(0);  // k = 0
          if (first && i >= 4 && rl == 0) wc = 0.0;  // row 0 above K = N mirrors its lower half
          if (first && i == 4 && t == 0) {
            if (rl == 0) {  // k = N
              d = stencil_fwd_r<T>(N, N, yN1, T(0), invN, inv4N1);
              wc = 0.5;
            } else {  // k = N - 1
              d = stencil_fwd_r<T>(N - 1, N, yN2, yN, invN, inv4N1);
            }
          }
          c0acc -= wc * (double)d;
          if (rl == 0) dr[i] = d;
          else di[i] = d;
        }
      }
      dct2_store(k1, dr, di);
    }
    const double tot = block_sum(c0acc, red);
    if (t == 0) part[(int64_t)comp * nt + tile] = tot * (double)N;
  } else {
    // p0 = (row 0 summed over n2) / 2: its reads are issued before the first row pair's,
    // and its block sum follows that pair's transform
    double p0acc = 0.0;
#pragma unroll
    for (int u = 0; u < (hp1 + NTHR - 1) / NTHR; ++u) {
      const int n2 = t + u * NTHR;
      if (n2 <= half2) p0acc += (double)Gc[n2].x * ((n2 == 0 || n2 == half2) ? 1.0 : 2.0);
    }
    // one DCT-1 row pair (k1a, k1a + 1) into registers: element m = t + i NTHR
    auto dct1_pair = [&](int k1a, T (&vr)[kPPT], T (&vi)[kPPT]) {
      int ma, mb;
      const int sa = hrow_src(k1a, L1, &ma);
      const int sb = hrow_src(k1a + 1, L1, &mb);
      const cplx<T>* ga = Gc + (int64_t)sa * sgi;
      const cplx<T>* gb = Gc + (int64_t)sb * sgi;
      cplx<T> a[kPPT], b[kPPT];
#pragma unroll
      for (int i = 0; i < kPPT; ++i) {
        const int m = t + i * NTHR;
        const int gi = m <= half2 ? m : L2 - m;
        a[i] = ga[gi];
        b[i] = gb[gi];
      }
#pragma unroll
      for (int i = 0; i < kPPT; ++i) {
        const int m = t + i * NTHR;
        const int gi = m <= half2 ? m : L2 - m;
        cplx<T> aa = a[i], bb = b[i];
        if (ma) aa = conjg<T>(aa);
        if (ma == 2) aa = cmul<T>(aa, tw[gi << twsh]);
        if (mb) bb = conjg<T>(bb);
        if (mb == 2) bb = cmul<T>(bb, tw[gi << twsh]);
        pack(m, aa.x, aa.y, bb.x, bb.y, vr[i], vi[i]);
      }
      fft_regs<T, LOGL2>(Yre, vr, vi, tw);
    };
    // window: rows k1 - 1, k1 (pa*) and k1 + 1, k1 + 2 (pb*) around the pair k1 = t0 + 2q
    T par[kPPT], pai[kPPT];
    dct1_pair(t0 - 1, par, pai);
    const T p0 = (T)(0.5 * block_sum(p0acc, red));
#pragma unroll
    for (int q = 0; q < TB / 2; ++q) {
      const int k1 = t0 + 2 * q;
      T pbr[kPPT], pbi[kPPT];
      dct1_pair(k1 + 1, pbr, pbi);
      // stencil of rows k1 and k1 + 1; rows k1 - 1, k1, k1 + 1, k1 + 2 = par, pai, pbr, pbi
      T dr[kPPT], di[kPPT];
      if (t0 >= 2) {
        // rows k1 >= 2: every coefficient index k = K or 2N - K lies in [2, N - 2], and
        // K <= N exactly when m < L2 / 2, i.e. for the thread's elements i < 4; there
        // stencil_tr is -p0 / (j^2 - 1) + (Ym / (j - 1) - Yp / (j + 1)) / 4
#pragma unroll
        for (int i = 0; i < kPPT; ++i) {
          const int m = t + i * NTHR;
#pragma unroll
          for (int rl = 0; rl < 2; ++rl) {
            const int K = k1 + rl + L1 * m;
            const int k = i < 4 ? K : N2 - K;
            const T ylo = rl ? pai[i] : par[i];
            const T yhi = rl ? pbi[i] : pbr[i];
            const T Ym = i < 4 ? ylo : yhi;
            const T Yp = i < 4 ? yhi : ylo;
            const T rm = recip_int<T>(T(k - 1)), rp = recip_int<T>(T(k + 1));
            const T d = -p0 * rm * rp + T(0.25) * (Ym * rm - Yp * rp);
            if (rl == 0) dr[i] = d;
            else di[i] = d;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < kPPT; ++i) {
          const int m = t + i * NTHR;
#pragma unroll
          for (int rl = 0; rl < 2; ++rl) {
            const int K = k1 + rl + L1 * m;
            const T ylo = rl ? pai[i] : par[i];
            const T yhi = rl ? pbi[i] : pbr[i];
            const bool lowhalf = K <= N;
            const int k = lowhalf ? K : N2 - K;
            const T d = stencil_tr_r<T>(k, N, lowhalf ? ylo : yhi, lowhalf ? yhi : ylo, p0, inv2N1);
            if (rl == 0) dr[i] = d;
            else di[i] = d;
          }
        }
      }
      dct2_store(k1, dr, di);
#pragma unroll
      for (int i = 0; i < kPPT; ++i) {
        par[i] = pbr[i];
        pai[i] = pbi[i];
      }
    }
  }
}

// ---------------------------------------------------------------- pass C
// Rows q1 in [c0, c0 + W) of the second DCT (Hermitian in r, rebuilt from r <= L1/2),
// two per complex FFT of length L1, written to the natural output positions
// j = q1 + L2 q2 and, for 0 < q1 < L2/2, the mirrored j = (L2 - q1) + L2 q2.
template <typename T, int TRANS>
__global__ __launch_bounds__(512) void k_fastC(const cplx<T>* __restrict__ G2, int64_t g2comp, int64_t sg2,
                                               T* __restrict__ out, int64_t Nn, int logL1, int logL2, int logW,
                                               const cplx<T>* __restrict__ tw, const double* __restrict__ part,
                                               int ntB, int nt, int nc, int xcd_order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* U = reinterpret_cast<T*>(smem_raw);  // W real rows of L1
  __shared__ double red[16];
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  TwCache<T> tc;
  load_twcache<T>(tc, logL1, tw);
  const int L1 = 1 << logL1, L2 = 1 << logL2;
  const int half1 = L1 / 2, half2 = L2 / 2;
  const int N = (int)(Nn - 1);
  const int W = 1 << logW;
  const int c0 = tile * W;
  const int ld1 = padded_ld(L1);
  const int sg2i = (int)sg2;
  T c0hat = T(0);
  if (!TRANS) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < ntB; i += blockDim.x) acc += part[(int64_t)comp * ntB + i];
    c0hat = (T)(block_sum(acc, red) / (double)N);
  }
  const cplx<T>* G2c = G2 + (int64_t)comp * g2comp;
  const int hp1 = half1 + 1;
  const int np = W / 2;
  const int nin = np * hp1;
  for (int base = threadIdx.x; base < nin; base += kUnroll * blockDim.x) {
    cplx<T> ra[kUnroll], rb[kUnroll];
    int pr_[kUnroll], r_[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = base + u * blockDim.x;
      pr_[u] = -1;
      if (e < nin) {
        // G2 row r holds q = 0..L2/2 contiguously: the W columns of this tile are one
        // contiguous segment per row
        const int r = e / np, pr = e - r * np;
        const int qa = c0 + 2 * pr, qb = qa + 1;
        ra[u] = qa <= half2 ? G2c[r * sg2i + qa] : mk<T>(T(0), T(0));
        rb[u] = qb <= half2 ? G2c[r * sg2i + qb] : mk<T>(T(0), T(0));
        pr_[u] = pr;
        r_[u] = r;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (pr_[u] < 0) continue;
      const int r = r_[u];
      T* re = U + (2 * pr_[u]) * ld1;
      T* im = re + ld1;
      re[pad(r)] = ra[u].x - rb[u].y;
      im[pad(r)] = ra[u].y + rb[u].x;
      if (r > 0 && r < half1) {
        re[pad(L1 - r)] = ra[u].x + rb[u].y;
        im[pad(L1 - r)] = rb[u].x - ra[u].y;
      }
    }
  }
  __syncthreads();
  split_fft_chunk<T>(U, 0, ld1, logL1, W / 2, tc);
  T* oc = out + (int64_t)comp * Nn;
  const T invN = T(1) / T(N);
  const int nout = W * hp1;
  for (int e = threadIdx.x; e < nout; e += blockDim.x) {
    const int w = e & (W - 1), q2 = e >> logW;
    const int q1 = c0 + w;
    if (q1 > half2) continue;
    const T* row = U + w * ld1;
    if (q2 < half1 || (q1 == 0 && q2 == half1)) {
      const int j = q1 + L2 * q2;
      const T u = row[pad(q2)];
      T o;
      if (TRANS) o = ((j == 0 || j == N) ? T(0.5) : T(1)) * u * invN;
      else o = T(0.5) * u + c0hat;
      oc[j] = o;
    }
    if (q1 > 0 && q1 < half2 && q2 < half1) {
      const int j = (L2 - q1) + L2 * q2;
      const T u = row[pad(L1 - 1 - q2)];
      T o;
      if (TRANS) o = u * invN;
      else o = T(0.5) * u + c0hat;
      oc[j] = o;
    }
  }
}

// ---- passes A and C at fixed lengths (L1 = 2^LOGL1, W = 2^LOGW columns per tile,
// blockDim = W L1 / 16: one radix-8 butterfly per thread per stage) ----
// Pass A: every thread issues all of its loads (PER values) at once, and its NO outputs
// are one unrolled batch (their twiddle reads in flight together).
template <typename T, int LOGL1, int LOGW>
__global__ __launch_bounds__((1 << LOGW) << (LOGL1 - 4)) void k_fastA2(
    const T* __restrict__ x, int64_t Nn, int logL2, cplx<T>* __restrict__ G, int64_t gcomp, int64_t sg,
    const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ thi, const cplx<T>* __restrict__ tlo, int tsh,
    const cplx<double>* __restrict__ thd, const cplx<double>* __restrict__ tld, int ends2, int nt, int nc, int xcd_order) {
  constexpr int L1 = 1 << LOGL1, W = 1 << LOGW;
  constexpr int NTHR = W * L1 / 16;
  constexpr int LD = padded_ld(L1);
  constexpr int NIN = W * L1;
  constexpr int PER = NIN / NTHR;  // 16 values per thread
  constexpr int half1 = L1 / 2;
  constexpr int NOUT = (half1 + 1) * W;
  constexpr int NO = (NOUT + NTHR - 1) / NTHR;  // outputs per thread (the last one for few threads)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* A = reinterpret_cast<T*>(smem_raw);
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  const T* xc = x + (int64_t)comp * Nn;
  const int N = (int)(Nn - 1), N2 = 2 * N;
  const int c0 = tile * W;
  const int t = (int)threadIdx.x;
  T val[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * NTHR;
    const int w = e & (W - 1), n1 = e >> LOGW;
    const int m = (n1 << logL2) + c0 + w;
    const int idx = m <= N ? m : N2 - m;
    val[u] = xc[idx];
    if (ends2 && (idx == 0 || idx == N)) val[u] *= T(2);
  }
  const int L2h = (1 << logL2) / 2;
  const int tmask = (1 << tsh) - 1;
  // double and float: the thread's outputs share n2 and step through k1 = k1_0 + u NTHR / W,
  // so their twiddles W_2N^(n2 k1) are a base times powers of one step (four reads of the
  // double table, issued with the inputs; the powers formed in double)
  constexpr bool kStep = std::is_floating_point<T>::value;
  constexpr int S = NTHR / W;
  const int n2t = c0 + (t & (W - 1)), k10 = t >> LOGW;
  cplx<double> wv, ws;
  if constexpr (kStep) {
    const int ta = n2t * k10, tb = n2t * S;
    wv = cmul<double>(thd[ta >> tsh], tld[ta & tmask]);
    ws = cmul<double>(thd[tb >> tsh], tld[tb & tmask]);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * NTHR;
    const int w = e & (W - 1), n1 = e >> LOGW;
    A[w * LD + pad(n1)] = val[u];
  }
  __syncthreads();
  fft_ct<T, LOGL1, W / 2>(A, tw);
  cplx<T>* Gc = G + (int64_t)comp * gcomp;
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int e = t + u * NTHR;
    const int w = e & (W - 1), k1 = e >> LOGW;
    const int n2 = c0 + w;
    if (e < NOUT && n2 <= L2h) {
      const T* re = A + (w & ~1) * LD;
      const int km = (L1 - k1) & (L1 - 1);
      const cplx<T> tws = kStep ? mk<T>((T)wv.x, (T)wv.y) : cmul<T>(thi[(n2 * k1) >> tsh], tlo[(n2 * k1) & tmask]);
      Gc[k1 * (int)sg + n2] =
          cmul<T>(separate<T>(re[pad(k1)], re[LD + pad(k1)], re[pad(km)], re[LD + pad(km)], w & 1), tws);
    }
    if constexpr (kStep) wv = cmul<double>(wv, ws);
  }
}

template <typename T, int TRANS, int LOGL1, int LOGW>
__global__ __launch_bounds__((1 << LOGW) << (LOGL1 - 4)) void k_fastC2(
    const cplx<T>* __restrict__ G2, int64_t g2comp, int64_t sg2, T* __restrict__ out, int64_t Nn, int logL2,
    const cplx<T>* __restrict__ tw, const double* __restrict__ part, int ntB, int nt, int nc, int xcd_order) {
  constexpr int L1 = 1 << LOGL1, W = 1 << LOGW;
  constexpr int NTHR = W * L1 / 16;
  constexpr int LD = padded_ld(L1);
  constexpr int half1 = L1 / 2, hp1 = half1 + 1;
  constexpr int NP = W / 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* U = reinterpret_cast<T*>(smem_raw);  // W real rows of L1
  __shared__ double red[16];
  int comp, tile;
  xcd_tile(nt, nc, xcd_order, comp, tile);
  const int L2 = 1 << logL2;
  const int half2 = L2 / 2;
  const int N = (int)(Nn - 1);
  const int c0 = tile * W;
  const int sg2i = (int)sg2;
  // all G2 loads of the thread at once (the last one for few threads), then the c^_0
  // total, whose reads and block sum overlap their latency
  const cplx<T>* G2c = G2 + (int64_t)comp * g2comp;
  constexpr int NIN = NP * hp1;
  constexpr int NI = (NIN + NTHR - 1) / NTHR;
  const int t = (int)threadIdx.x;
  cplx<T> ra[NI], rb[NI];
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int e = t + u * NTHR;
    ra[u] = rb[u] = mk<T>(T(0), T(0));
    if (e < NIN) {
      // G2 row r holds q = 0..L2/2 contiguously: the W columns of this tile are one
      // contiguous segment per row
      const int r = e / NP, pr = e - r * NP;
      const int qa = c0 + 2 * pr, qb = qa + 1;
      if (qa <= half2) ra[u] = G2c[r * sg2i + qa];
      if (qb <= half2) rb[u] = G2c[r * sg2i + qb];
    }
  }
  T c0hat = T(0);
  if (!TRANS) {
    double acc = 0.0;
    for (int i = t; i < ntB; i += NTHR) acc += part[(int64_t)comp * ntB + i];
    c0hat = (T)(block_sum(acc, red) / (double)N);
  }
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int e = t + u * NTHR;
    if (e >= NIN) continue;
    const int r = e / NP, pr = e - r * NP;
    T* re = U + (2 * pr) * LD;
    T* im = re + LD;
    re[pad(r)] = ra[u].x - rb[u].y;
    im[pad(r)] = ra[u].y + rb[u].x;
    if (r > 0 && r < half1) {
      re[pad(L1 - r)] = ra[u].x + rb[u].y;
      im[pad(L1 - r)] = rb[u].x - ra[u].y;
    }
  }
  __syncthreads();
  fft_ct<T, LOGL1, NP>(U, tw);
  T* oc = out + (int64_t)comp * Nn;
  const T invN = T(1) / T(N);
  constexpr int NOUT = W * hp1;
  for (int e = threadIdx.x; e < NOUT; e += NTHR) {
    const int w = e & (W - 1), q2 = e >> LOGW;
    const int q1 = c0 + w;
    if (q1 > half2) continue;
    const T* row = U + w * LD;
    if (q2 < half1 || (q1 == 0 && q2 == half1)) {
      const int j = q1 + L2 * q2;
      const T u = row[pad(q2)];
      T o;
      if (TRANS) o = ((j == 0 || j == N) ? T(0.5) : T(1)) * u * invN;
      else o = T(0.5) * u + c0hat;
      oc[j] = o;
    }
    if (q1 > 0 && q1 < half2 && q2 < half1) {
      const int j = (L2 - q1) + L2 * q2;
      const T u = row[pad(L1 - 1 - q2)];
      T o;
      if (TRANS) o = u * invN;
      else o = T(0.5) * u + c0hat;
      oc[j] = o;
    }
  }
}

}  // namespace fast

// ---------------------------------------------------------------- host side

// Shape of the fast path for one transform size and precision (chosen at plan creation).
bool fast_eligible(int64_t N) {
  if (N < 512 || (N & (N - 1)) != 0) return false;
  int s = 0;
  while ((int64_t(1) << s) < 2 * N) ++s;
  return s <= 2 * kLdsMaxLog;
}

template <typename T>
static void fast_shape(const FastKnobs& kn, int64_t N, int& logL1, int& logL2, int& WA, int& TB, int& WC) {
  int s = 0;
  while ((int64_t(1) << s) < 2 * N) ++s;
  if (kn.split == 0) {
    logL2 = (s + 1) / 2;  // rows of the first DCT (pass B) are the longer side
    logL1 = s - logL2;
  } else {
    logL1 = (s + 1) / 2;
    logL2 = s - logL1;
  }
  const int kb = kn.lds_kb[sizeof(T) == 8 ? 0 : 1];
  const int budget = (int)((int64_t)kb * 1024 / sizeof(T));  // reals of LDS per workgroup
  const int L1 = 1 << logL1, L2 = 1 << logL2;
  WA = std::max(2, std::min(16, budget / fast::padded_ld(L1)));
  while (WA & (WA - 1)) WA &= WA - 1;  // power of two
  WC = WA;
  const int rows = std::max(4, std::min(16, budget / fast::padded_ld(L2)));
  TB = kn.tb > 0 ? kn.tb : std::max(2, (rows - 2) & ~1);
  // the halo rows of a pass-B tile must stay inside [-1, L1)
  while (TB > 2 && TB > L1 / 2 - 2) TB -= 2;
  while (TB > 2 && (int64_t)(TB + 2) * fast::padded_ld(L2) * (int64_t)sizeof(T) > 160 * 1024) TB -= 2;
  // Passes A and C: one split_fft chunk per workgroup (W L1 / 2 <= 512 kPPT points), which
  // keeps tiles small and workgroups many.  Pass B: larger tiles amortise the two halo
  // rows; its split_fft works through the rows in chunks.
  const int maxpts = 512 * fast::kPPT;
  while (WA > 2 && WA * L1 / 2 > maxpts) WA /= 2;
  while (WC > 2 && WC * L1 / 2 > maxpts) WC /= 2;
}

// Pass B takes the register kernel when its rows are 512..2048 points long, with 2 or 4
// rows per tile.
static bool use_b2(const FastKnobs& kn, int logL2) { return kn.b2 && logL2 >= 9 && logL2 <= 11; }
static int b2_rows(const FastKnobs& kn) { return kn.tb == 4 ? 4 : 2; }

// Pass-B tiles per component (rows 0..L1/2 in tiles of TB, or of 2 or 4 for the register
// kernels).
template <typename T>
static int fast_tiles_b(const FastKnobs& kn, int64_t N) {
  int logL1, logL2, WA, TB, WC;
  fast_shape<T>(kn, N, logL1, logL2, WA, TB, WC);
  const int rows = (1 << logL1) / 2 + 1;
  const int tb = use_b2(kn, logL2) ? b2_rows(kn) : TB;
  return (rows + tb - 1) / tb;
}

// Passes A and C take the compile-time-length kernels for L1 = 2^8..2^11 (tiles of 8
// columns, 4 at 2^11); returns log2 of the tile width, or 0 for the general kernels.
static int fixed_logw(const FastKnobs& kn, int logL1) {
  if (!kn.b2 || logL1 < 8 || logL1 > 11) return 0;
  if (kn.narrow && (logL1 == 9 || logL1 == 10)) return 2;
  return logL1 == 11 ? 2 : 3;
}

static int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Threads per workgroup: one per kPPT complex points of the largest split_fft call.
static int threads_for(int complex_points) {
  int t = (complex_points + fast::kPPT - 1) / fast::kPPT;
  t = (t + 63) / 64 * 64;
  return std::max(64, std::min(512, t));
}

template <typename F>
static void lds_attr(F f, int bytes) {
  (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T, int TB, int TRANS>
static void launch_B(int xcd, int nt, int nc, int thr, int lds, hipStream_t s, const cplx<T>* G, int64_t gcomp, int64_t sg,
                     cplx<T>* G2, int64_t g2comp, int64_t sg2, int64_t N, int logL1, int logL2, const cplx<T>* tw,
                     const cplx<T>* thi, const cplx<T>* tlo, int tsh, double* part) {
  auto f = fast::k_fastB<T, TB, TRANS>;
  lds_attr(f, lds);
  hipLaunchKernelGGL(f, dim3(nt * nc), dim3(thr), lds, s, G, gcomp, sg, G2, g2comp, sg2, N, logL1, logL2, tw, thi,
                     tlo, tsh, part, nt, nc, xcd);
}

// The three passes for the components of g (a whole group or a contiguous part of one).
template <typename T>
static hipError_t fast_passes(birk_plan* p, const FastGroup& g, const T* v, T* out, int transpose, hipStream_t s) {
  constexpr int pi = prec_index<T>();
  int logL1, logL2, WA, TB, WC;
  const FastKnobs& kn = g.kn;
  fast_shape<T>(kn, g.N, logL1, logL2, WA, TB, WC);
  const int L1 = 1 << logL1, L2 = 1 << logL2;
  const int ld1 = fast::padded_ld(L1), ld2 = fast::padded_ld(L2);
  const int64_t sg = L2 / 2 + 1, sg2 = L2 / 2 + 1;  // G [k1][n2] and G2 [r][q]: rows of L2/2 + 1
  const int64_t gcomp = (int64_t)(L1 / 2 + 1) * sg, g2comp = (int64_t)(L1 / 2 + 1) * sg2;
  cplx<T>* G = (cplx<T>*)p->work[0] + g.work_off;
  cplx<T>* G2 = (cplx<T>*)p->work[1] + g.work_off;
  double* part = p->partials + g.part_off;
  const cplx<T>* tw = (const cplx<T>*)p->lds_tw[pi];
  const cplx<T>* thi = (const cplx<T>*)g.tw.hi[pi];
  const cplx<T>* tlo = (const cplx<T>*)g.tw.lo[pi];
  const int tsh = g.tw.shift;
  const cplx<double>* thd = (const cplx<double>*)g.tw.hi[0];
  const cplx<double>* tld = (const cplx<double>*)g.tw.lo[0];
  const int nc = g.nc;
  const int lw = fixed_logw(kn, logL1);
  if (lw > 0) {
    // compile-time lengths: one tile of W = 2^lw columns per workgroup
    const int W = 1 << lw;
    const int ntA = (L2 / 2 + 1 + W - 1) / W;
    const int lds = W * ld1 * (int)sizeof(T);
    auto f = fast::k_fastA2<T, 10, 3>;
    switch (logL1) {
      case 8: f = fast::k_fastA2<T, 8, 3>; break;
      case 9: f = lw == 2 ? fast::k_fastA2<T, 9, 2> : fast::k_fastA2<T, 9, 3>; break;
      case 10: f = lw == 2 ? fast::k_fastA2<T, 10, 2> : fast::k_fastA2<T, 10, 3>; break;
      default: f = fast::k_fastA2<T, 11, 2>; break;
    }
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntA * nc), dim3(W * L1 / 16), lds, s, v + g.off, g.Nn, logL2, G, gcomp, sg, tw, thi,
                       tlo, tsh, thd, tld, transpose ? 1 : 0, ntA, nc, kn.xcd);
  } else {
    const int ntA = (L2 / 2 + 1 + WA - 1) / WA;
    const int lds = WA * ld1 * (int)sizeof(T);
    auto f = fast::k_fastA<T>;
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntA * nc), dim3(threads_for(WA * L1 / 2)), lds, s, v + g.off, g.Nn, logL1, logL2,
                       ilog2i(WA), G, gcomp, sg, tw, thi, tlo, tsh, transpose ? 1 : 0, ntA, nc, kn.xcd);
  }
  const int ntB = fast_tiles_b<T>(kn, g.N);
  if (use_b2(kn, logL2) && kn.b3) {
    const int lds = 2 * ld2 * (int)sizeof(T);
    const int thr = L2 / fast::kPPT;
    const int tb4 = b2_rows(kn) == 4;
    auto f = fast::k_fastB3<T, 0, 11, 2>;
    switch ((logL2 * 2 + (transpose ? 1 : 0)) * 2 + tb4) {
      case 36: f = fast::k_fastB3<T, 0, 9, 2>; break;
      case 37: f = fast::k_fastB3<T, 0, 9, 4>; break;
      case 38: f = fast::k_fastB3<T, 1, 9, 2>; break;
      case 39: f = fast::k_fastB3<T, 1, 9, 4>; break;
      case 40: f = fast::k_fastB3<T, 0, 10, 2>; break;
      case 41: f = fast::k_fastB3<T, 0, 10, 4>; break;
      case 42: f = fast::k_fastB3<T, 1, 10, 2>; break;
      case 43: f = fast::k_fastB3<T, 1, 10, 4>; break;
      case 44: f = fast::k_fastB3<T, 0, 11, 2>; break;
      case 45: f = fast::k_fastB3<T, 0, 11, 4>; break;
      case 46: f = fast::k_fastB3<T, 1, 11, 2>; break;
      default: f = fast::k_fastB3<T, 1, 11, 4>; break;
    }
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntB * nc), dim3(thr), lds, s, G, gcomp, sg, G2, g2comp, sg2, g.N, logL1, tw, thi, tlo,
                       tsh, thd, tld, part, ntB, nc, kn.xcd);
  } else if (use_b2(kn, logL2)) {
    const int lds = 2 * ld2 * (int)sizeof(T);
    const int thr = L2 / fast::kPPT;
    auto f = fast::k_fastB2<T, 0, 11, 2>;
    const int tb4 = b2_rows(kn) == 4;
    switch ((logL2 * 2 + (transpose ? 1 : 0)) * 2 + tb4) {
      case 36: f = fast::k_fastB2<T, 0, 9, 2>; break;
      case 37: f = fast::k_fastB2<T, 0, 9, 4>; break;
      case 38: f = fast::k_fastB2<T, 1, 9, 2>; break;
      case 39: f = fast::k_fastB2<T, 1, 9, 4>; break;
      case 40: f = fast::k_fastB2<T, 0, 10, 2>; break;
      case 41: f = fast::k_fastB2<T, 0, 10, 4>; break;
      case 42: f = fast::k_fastB2<T, 1, 10, 2>; break;
      case 43: f = fast::k_fastB2<T, 1, 10, 4>; break;
      case 44: f = fast::k_fastB2<T, 0, 11, 2>; break;
      case 45: f = fast::k_fastB2<T, 0, 11, 4>; break;
      case 46: f = fast::k_fastB2<T, 1, 11, 2>; break;
      default: f = fast::k_fastB2<T, 1, 11, 4>; break;
    }
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntB * nc), dim3(thr), lds, s, G, gcomp, sg, G2, g2comp, sg2, g.N, logL1, tw, thi, tlo,
                       tsh, part, ntB, nc, kn.xcd);
  } else {
    const int lds = (TB + 2) * ld2 * (int)sizeof(T);
    const int thr = std::min(threads_for((TB + 2) * L2 / 2), kn.b_threads);
#define BIRK_LB(tb)                                                                                                \
  case tb:                                                                                                         \
    if (transpose)                                                                                                 \
      launch_B<T, tb, 1>(kn.xcd, ntB, nc, thr, lds, s, G, gcomp, sg, G2, g2comp, sg2, g.N, logL1, logL2, tw, thi, tlo, tsh, \
                         part);                                                                                    \
    else                                                                                                           \
      launch_B<T, tb, 0>(kn.xcd, ntB, nc, thr, lds, s, G, gcomp, sg, G2, g2comp, sg2, g.N, logL1, logL2, tw, thi, tlo, tsh, \
                         part);                                                                                    \
    break;
    switch (TB) {
      BIRK_LB(2)
      BIRK_LB(4)
      BIRK_LB(6)
      BIRK_LB(8)
      BIRK_LB(10)
      BIRK_LB(12)
      BIRK_LB(14)
      default:
        return hipErrorInvalidValue;
    }
#undef BIRK_LB
  }
  if (lw > 0) {
    const int W = 1 << lw;
    const int ntC = (L2 / 2 + 1 + W - 1) / W;
    const int lds = W * ld1 * (int)sizeof(T);
    T* o = out + g.off;
    auto f = fast::k_fastC2<T, 0, 10, 3>;
    switch (logL1 * 2 + (transpose ? 1 : 0)) {
      case 16: f = fast::k_fastC2<T, 0, 8, 3>; break;
      case 17: f = fast::k_fastC2<T, 1, 8, 3>; break;
      case 18: f = lw == 2 ? fast::k_fastC2<T, 0, 9, 2> : fast::k_fastC2<T, 0, 9, 3>; break;
      case 19: f = lw == 2 ? fast::k_fastC2<T, 1, 9, 2> : fast::k_fastC2<T, 1, 9, 3>; break;
      case 20: f = lw == 2 ? fast::k_fastC2<T, 0, 10, 2> : fast::k_fastC2<T, 0, 10, 3>; break;
      case 21: f = lw == 2 ? fast::k_fastC2<T, 1, 10, 2> : fast::k_fastC2<T, 1, 10, 3>; break;
      case 22: f = fast::k_fastC2<T, 0, 11, 2>; break;
      default: f = fast::k_fastC2<T, 1, 11, 2>; break;
    }
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntC * nc), dim3(W * L1 / 16), lds, s, G2, g2comp, sg2, o, g.Nn, logL2, tw, part, ntB,
                       ntC, nc, kn.xcd);
  } else {
    const int ntC = (L2 / 2 + 1 + WC - 1) / WC;
    const int lds = WC * ld1 * (int)sizeof(T);
    const int thr = threads_for(WC * L1 / 2);
    T* o = out + g.off;
    auto f = transpose ? fast::k_fastC<T, 1> : fast::k_fastC<T, 0>;
    lds_attr(f, lds);
    hipLaunchKernelGGL(f, dim3(ntC * nc), dim3(thr), lds, s, G2, g2comp, sg2, o, g.Nn, logL1, logL2, ilog2i(WC), tw,
                       part, ntB, ntC, nc, kn.xcd);
  }
  return hipGetLastError();
}

// Tile schedules the autotuner tries for a group: the defaults first, then both splits of
// 2N = L1 L2, two or four rows per pass-B tile, both tile orders, one to three streams,
// and, where L1 is 2^9 or 2^10, tiles of four or eight columns in passes A and C.
static int log_l1(const FastKnobs& kn, int64_t N) {
  int s = 0;
  while ((int64_t(1) << s) < 2 * N) ++s;
  return kn.split == 0 ? s - (s + 1) / 2 : (s + 1) / 2;
}

static std::vector<FastKnobs> tune_candidates(const FastKnobs& base, int64_t N) {
  std::vector<FastKnobs> c{base};
  for (int split = 0; split < 2; ++split)
    for (int tb = 2; tb <= 4; tb += 2)
      for (int xcd = 0; xcd < 2; ++xcd)
        for (int st = 1; st <= 3; ++st)
          for (int nw = 0; nw < 2; ++nw) {
            FastKnobs k = base;
            k.split = split;
            k.tb = tb;
            k.xcd = xcd;
            k.streams = st;
            k.narrow = nw;
            FastKnobs k0 = k;
            k0.narrow = 0;
            const int l1 = log_l1(k, N);
            if (nw && fixed_logw(k, l1) == fixed_logw(k0, l1)) continue;   // no effect at this size
            if (k.split != base.split || k.tb != base.tb || k.xcd != base.xcd || k.streams != base.streams ||
                k.narrow != base.narrow)
              c.push_back(k);
          }
  return c;
}

// A group's product.  With kn.streams = S > 1 the components are split into S contiguous
// parts, part k > 0 on the plan's extra stream k - 1 (forked from and joined back into the
// caller's stream by events), so that when one part's pass runs out of tiles another's
// keeps the CUs busy.  Each component's kernels, tiles and partial sums are those of the
// one-stream schedule.
template <typename T>
hipError_t fast_product(birk_plan* p, const FastGroup& g, const T* v, T* out, int transpose, hipStream_t s) {
  const int S = std::min(std::min(g.kn.streams, g.nc), 1 + birk_plan::kExtraStreams);
  if (S < 2 || !p->xstream[0]) return fast_passes<T>(p, g, v, out, transpose, s);
  int logL1, logL2, WA, TB, WC;
  fast_shape<T>(g.kn, g.N, logL1, logL2, WA, TB, WC);
  const int64_t gcomp = (int64_t)((1 << logL1) / 2 + 1) * ((1 << logL2) / 2 + 1);
  const int64_t ntB = fast_tiles_b<T>(g.kn, g.N);
  hipError_t e = hipEventRecord(p->ev_fork, s);
  int c0 = 0;
  for (int k = 0; k < S && e == hipSuccess; ++k) {
    const int c1 = (int)((int64_t)g.nc * (k + 1) / S);
    FastGroup part = g;
    part.nc = c1 - c0;
    part.off = g.off + (int64_t)c0 * g.Nn;
    part.work_off = g.work_off + (int64_t)c0 * gcomp;
    part.part_off = g.part_off + (int64_t)c0 * ntB;
    if (k == 0) {
      e = fast_passes<T>(p, part, v, out, transpose, s);
    } else {
      hipStream_t x = p->xstream[k - 1];
      e = hipStreamWaitEvent(x, p->ev_fork, 0);
      if (e == hipSuccess) e = fast_passes<T>(p, part, v, out, transpose, x);
      if (e == hipSuccess) e = hipEventRecord(p->ev_join[k - 1], x);
    }
    c0 = c1;
  }
  for (int k = 1; k < S && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, p->ev_join[k - 1], 0);
  return e;
}

// Work (complex elements per buffer) and partials (doubles) of the fast path for nc
// components of length N + 1, for any of the storage types and any schedule the
// autotuner may choose.
void fast_sizes(const birk_plan* p, int64_t N, int nc, int64_t* work, int64_t* part) {
  int64_t w = 0, ntB = 0;
  for (const FastKnobs& kn : tune_candidates(p->fast_kn, N)) {
    int l1, l2, wa, tb, wc;
    fast_shape<double>(kn, N, l1, l2, wa, tb, wc);
    w = std::max(w, (int64_t)nc * ((int64_t(1) << l1) / 2 + 1) * ((int64_t(1) << l2) / 2 + 1));
    ntB = std::max(ntB, (int64_t)std::max(fast_tiles_b<float>(kn, N),
                                          std::max(fast_tiles_b<double>(kn, N), fast_tiles_b<df32>(kn, N))));
  }
  *work = w;
  *part = (int64_t)nc * ntB;
}

// Autotuner: per group, B^a over every candidate schedule on the plan's scratch vectors,
// alternating two input/output pairs; each candidate runs once to warm up and then
// kTuneReps times between HIP events, in kTuneRounds interleaved rounds, and keeps its
// best round.  The default schedule (first candidate) stays unless another is faster by
// more than kTuneMargin, so that timing noise does not flip the choice between
// near-equal schedules.
constexpr int kTuneReps = 4;
constexpr int kTuneRounds = 2;
constexpr float kTuneMargin = 0.02f;

template <typename T>
static hipError_t tune_groups(birk_plan* p, hipStream_t s, std::string* report) {
  T* in[2] = {(T*)p->tmp_vec[0], (T*)p->tmp_vec[2]};
  T* out[2] = {(T*)p->tmp_vec[1], (T*)p->tmp_vec[3]};
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(in[b], 0, (size_t)p->total_len * sizeof(T), s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  char line[160];
  for (FastGroup& g : p->fgroups) {
    if (e != hipSuccess) break;
    const std::vector<FastKnobs> cand = tune_candidates(p->fast_kn, g.N);
    std::vector<float> best_of(cand.size(), 0.0f);
    for (int round = 0; round < kTuneRounds && e == hipSuccess; ++round) {
      for (size_t ci = 0; ci < cand.size() && e == hipSuccess; ++ci) {
        g.kn = cand[ci];
        if ((e = fast_product<T>(p, g, in[0], out[0], 0, s)) != hipSuccess) break;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
        for (int r = 0; r < kTuneReps && e == hipSuccess; ++r) e = fast_product<T>(p, g, in[r & 1], out[r & 1], 0, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= kTuneReps;
        if (round == 0 || ms < best_of[ci]) best_of[ci] = ms;
      }
    }
    if (e != hipSuccess) break;
    snprintf(line, sizeof line, "N=%lld x %d:", (long long)g.N, g.nc);
    *report += line;
    size_t best = 0;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      snprintf(line, sizeof line, " [split %d, tb %d, xcd %d, streams %d, narrow %d] %.1f us;", cand[ci].split,
               cand[ci].tb, cand[ci].xcd, cand[ci].streams, cand[ci].narrow, 1000.0 * best_of[ci]);
      *report += line;
      if (best_of[ci] < best_of[best] * (1.0f - kTuneMargin)) best = ci;
    }
    g.kn = cand[best];
    snprintf(line, sizeof line, " chosen [split %d, tb %d, xcd %d, streams %d, narrow %d]\n", g.kn.split, g.kn.tb,
             g.kn.xcd, g.kn.streams, g.kn.narrow);
    *report += line;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

hipError_t tune_fast(birk_plan* p, hipStream_t s, std::string* report) {
  if (p->fgroups.empty()) {
    *report += "no power-of-two groups to tune\n";
    return hipSuccess;
  }
  if (p->prec == BIRK_F64) return tune_groups<double>(p, s, report);
  if (p->prec == BIRK_DF32) return tune_groups<df32>(p, s, report);
  return tune_groups<float>(p, s, report);  // float storage, with or without refinement
}

template hipError_t fast_product<double>(birk_plan*, const FastGroup&, const double*, double*, int, hipStream_t);
template hipError_t fast_product<float>(birk_plan*, const FastGroup&, const float*, float*, int, hipStream_t);
template hipError_t fast_product<df32>(birk_plan*, const FastGroup&, const df32*, df32*, int, hipStream_t);

}  // namespace birk
