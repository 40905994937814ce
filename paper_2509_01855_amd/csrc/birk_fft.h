// Radix-8 Stockham FFTs in LDS on split real/imaginary rows, shared by the three-pass
// power-of-two product (birk_fast.hip) and the fused Bluestein passes (birk_dct.hip).
//
// Twiddles come from one table of W_4096^j = exp(-2 pi i j / 4096), j < 4096 (2^kLdsMaxLog
// entries): W_L^m = tw[m << (kLdsMaxLog - log2 L)].

#pragma once

#include <hip/hip_runtime.h>

#include "birk_internal.h"

namespace birk {
namespace fast {

template <typename T>
__device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return fast::mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T>
__device__ __forceinline__ cplx<T> conjg(cplx<T> a) {
  return fast::mk<T>(a.x, -a.y);
}

// ---- in-register DFTs of length 2, 4, 8 (forward, W_R = exp(-2 pi i / R)) ----
// vr/vi hold the R inputs in natural order and receive the R outputs in natural order.
template <typename T>
__device__ __forceinline__ void dft4(T& ar, T& ai, T& br, T& bi, T& cr, T& ci, T& dr, T& di) {
  const T t0r = ar + cr, t0i = ai + ci, t1r = ar - cr, t1i = ai - ci;
  const T t2r = br + dr, t2i = bi + di, ur = br - dr, ui = bi - di;
  // (b - d) * (-i) = (ui, -ur)
  ar = t0r + t2r;
  ai = t0i + t2i;
  cr = t0r - t2r;
  ci = t0i - t2i;
  br = t1r + ui;
  bi = t1i - ur;
  dr = t1r - ui;
  di = t1i + ur;
}

template <typename T>
__device__ __forceinline__ void cmul_inplace(T& r, T& i, T wr, T wi) {
  const T a = r * wr - i * wi;
  i = r * wi + i * wr;
  r = a;
}

template <typename T, int R>
__device__ __forceinline__ void dft_reg(T (&vr)[R], T (&vi)[R]) {
  if constexpr (R == 2) {
    const T ar = vr[0], ai = vi[0];
    vr[0] = ar + vr[1];
    vi[0] = ai + vi[1];
    vr[1] = ar - vr[1];
    vi[1] = ai - vi[1];
  } else if constexpr (R == 4) {
    dft4<T>(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
  } else {
    static_assert(R == 8, "radix 2, 4 or 8");
    // n = q + 2p, k = s + 4t: two DFT4 over p, twiddle W8^(q s), DFT2 over q
    dft4<T>(vr[0], vi[0], vr[2], vi[2], vr[4], vi[4], vr[6], vi[6]);
    dft4<T>(vr[1], vi[1], vr[3], vi[3], vr[5], vi[5], vr[7], vi[7]);
    const T h = T(0.70710678118654752440);  // sqrt(1/2)
    // q = 1 row, s = 1..3: W8^1 = (h, -h), W8^2 = (0, -1), W8^3 = (-h, -h)
    cmul_inplace<T>(vr[3], vi[3], h, -h);
    { const T a = vr[5]; vr[5] = vi[5]; vi[5] = -a; }
    cmul_inplace<T>(vr[7], vi[7], -h, -h);
    T outr[8], outi[8];
#pragma unroll
    for (int sI = 0; sI < 4; ++sI) {
      const T a0r = vr[2 * sI], a0i = vi[2 * sI], a1r = vr[2 * sI + 1], a1i = vi[2 * sI + 1];
      outr[sI] = a0r + a1r;
      outi[sI] = a0i + a1i;
      outr[sI + 4] = a0r - a1r;
      outi[sI + 4] = a0i - a1i;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      vr[i] = outr[i];
      vi[i] = outi[i];
    }
  }
}

// LDS rows are padded with one element after every 16 (and rows are an odd number of
// elements apart) so that the strided accesses of the early Stockham stages and the
// column-tile loads spread over the 64 LDS banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_ld(int L) { return L + (L >> 4) + 1; }

// Complex points per thread in the LDS FFTs: one radix-8 butterfly per thread per stage.
constexpr int kPPT = 8;

// W^(jm), W^(2 jm), W^(4 jm) of the thread's butterfly in the radix-8 stage at logNs.
template <typename T>
__device__ __forceinline__ void load_tw_stage(cplx<T> (&w)[3], int logL, int logNs, const cplx<T>* __restrict__ tw) {
  const int j = threadIdx.x & ((1 << (logL - 3)) - 1);
  const int jm = logNs < logL ? (j & ((1 << logNs) - 1)) : 0;
  if (jm != 0) {
    const int tshift = kLdsMaxLog - (logNs + 3);
    w[0] = tw[jm << tshift];
    w[1] = tw[(2 * jm) << tshift];
    w[2] = tw[(4 * jm) << tshift];
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) w[q] = fast::mk<T>(T(1), T(0));
  }
}

// ---- fixed-length transforms: COUNT transforms of length 2^LOGL, blockDim = COUNT 2^LOGL / 8 ----
// Transform t has its real part in row 2t and its imaginary part in row 2t + 1 of a
// split array with padded rows of padded_ld(2^LOGL) reals.  With the length known at
// compile time every LDS address of a butterfly is the padded position of its first
// element plus a constant: pad(j + r s) = pad(j) + r s + (r s) / 16 for s a power of two
// (s divides 16 or 16 divides s), so a thread needs one address register per butterfly
// and the element offsets become instruction immediates.
template <typename T, int LOGL, int LOGNS, int R, int COUNT>
__device__ __forceinline__ void stage_ct(T* __restrict__ buf, const cplx<T> (&w)[3]) {
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  constexpr int NB = kPPT / R;             // butterflies per thread
  constexpr int LOGNBF = LOGL - logR;
  constexpr int NBF = 1 << LOGNBF;         // butterflies per transform
  constexpr int NTHR = COUNT << (LOGL - 3);  // threads (blockDim)
  constexpr int NS = 1 << LOGNS;
  constexpr int LD = padded_ld(1 << LOGL);
  T vr[NB][R], vi[NB][R];
  int pd[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = (int)threadIdx.x + i * NTHR;
    const int t = b >> LOGNBF;
    const int j = b & (NBF - 1);
    const int rowoff = 2 * t * LD;
    const int pj = rowoff + j + (j >> 4);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int off = r * NBF + ((r * NBF) >> 4);
      vr[i][r] = buf[pj + off];
      vi[i][r] = buf[pj + LD + off];
    }
    const int jm = j & (NS - 1);
    if constexpr (R == 8 && LOGNS > 0) {
      if (jm != 0) {
        const cplx<T> w1 = w[0], w2 = w[1], w4 = w[2];
        const cplx<T> w3 = fast::cmul<T>(w2, w1);
        const cplx<T> w5 = fast::cmul<T>(w4, w1), w6 = fast::cmul<T>(w4, w2), w7 = fast::cmul<T>(w4, w3);
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
    const int dst = ((j >> LOGNS) << (LOGNS + logR)) + jm;
    pd[i] = rowoff + dst + (dst >> 4);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int off = r * NS + ((r * NS) >> 4);
      buf[pd[i] + off] = vr[i][r];
      buf[pd[i] + LD + off] = vi[i][r];
    }
  }
  __syncthreads();
}

template <typename T, int LOGL, int COUNT, int K>
__device__ __forceinline__ void stages8_ct(T* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  constexpr int BASE = (LOGL % 3) ? (LOGL % 3) : 3;
  constexpr int LOGNS = BASE + 3 * K;
  if constexpr (LOGNS < LOGL) {
    cplx<T> w[3];
    load_tw_stage<T>(w, LOGL, LOGNS, tw);
    stage_ct<T, LOGL, LOGNS, 8, COUNT>(buf, w);
    stages8_ct<T, LOGL, COUNT, K + 1>(buf, tw);
  }
}

// COUNT in-place transforms of length 2^LOGL (see stage_ct for the layout).
template <typename T, int LOGL, int COUNT>
__device__ __forceinline__ void fft_ct(T* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  cplx<T> w[3];
  if constexpr (LOGL % 3 == 1) stage_ct<T, LOGL, 0, 2, COUNT>(buf, w);
  else if constexpr (LOGL % 3 == 2) stage_ct<T, LOGL, 0, 4, COUNT>(buf, w);
  else stage_ct<T, LOGL, 0, 8, COUNT>(buf, w);
  stages8_ct<T, LOGL, COUNT, 0>(buf, tw);
}

// ---- one transform of length 2^LOGL per workgroup (blockDim = 2^LOGL / 8) whose input
// and output live in registers: v[i] is element m = threadIdx.x + NT i (NT = 2^LOGL / 8)
// both before and after.  The first stage (radix 2^(LOGL mod 3), or 8; no twiddles) reads
// its butterfly inputs straight from the registers, and the last radix-8 stage (Ns = NT)
// leaves butterfly t's outputs exactly at m = t + NT r, so only the stages in between
// pass through the LDS rows (two fewer LDS round trips than fft_ct).
template <typename T, int LOGL>
__device__ __forceinline__ void stage_first_regs(T* __restrict__ buf, const T (&vr)[kPPT], const T (&vi)[kPPT]) {
  constexpr int R = (LOGL % 3 == 1) ? 2 : (LOGL % 3 == 2) ? 4 : 8;
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  constexpr int NB = kPPT / R;
  constexpr int NT = 1 << (LOGL - 3);
  constexpr int LD = padded_ld(1 << LOGL);
  T xr[NB][R], xi[NB][R];
#pragma unroll
  for (int ib = 0; ib < NB; ++ib) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xr[ib][r] = vr[ib + NB * r];   // butterfly b = t + NT ib takes b + (L / R) r = t + NT (ib + NB r)
      xi[ib][r] = vi[ib + NB * r];
    }
    dft_reg<T, R>(xr[ib], xi[ib]);
  }
  __syncthreads();  // earlier readers of buf are done
#pragma unroll
  for (int ib = 0; ib < NB; ++ib) {
    const int dst = ((int)threadIdx.x + NT * ib) << logR;   // Ns = 1: outputs at R b + r
    const int pd = dst + (dst >> 4);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      buf[pd + r] = xr[ib][r];
      buf[LD + pd + r] = xi[ib][r];
    }
  }
  __syncthreads();
}

template <typename T, int LOGL, int K>
__device__ __forceinline__ void stages8_mid(T* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  constexpr int BASE = (LOGL % 3) ? (LOGL % 3) : 3;
  constexpr int LOGNS = BASE + 3 * K;
  if constexpr (LOGNS < LOGL - 3) {
    cplx<T> w[3];
    load_tw_stage<T>(w, LOGL, LOGNS, tw);
    stage_ct<T, LOGL, LOGNS, 8, 1>(buf, w);
    stages8_mid<T, LOGL, K + 1>(buf, tw);
  }
}

template <typename T, int LOGL>
__device__ __forceinline__ void stage_last_regs(const T* __restrict__ buf, T (&vr)[kPPT], T (&vi)[kPPT],
                                                const cplx<T>* __restrict__ tw) {
  constexpr int NT = 1 << (LOGL - 3);
  constexpr int LD = padded_ld(1 << LOGL);
  const int t = (int)threadIdx.x;
  const int pj = t + (t >> 4);
#pragma unroll
  for (int r = 0; r < kPPT; ++r) {
    const int off = r * NT + ((r * NT) >> 4);
    vr[r] = buf[pj + off];
    vi[r] = buf[LD + pj + off];
  }
  if (t != 0) {   // butterfly j = t of the stage at Ns = NT: twiddles W_(8 NT)^(t r)
    cplx<T> w[3];
    load_tw_stage<T>(w, LOGL, LOGL - 3, tw);
    const cplx<T> w1 = w[0], w2 = w[1], w4 = w[2];
    const cplx<T> w3 = fast::cmul<T>(w2, w1);
    const cplx<T> w5 = fast::cmul<T>(w4, w1), w6 = fast::cmul<T>(w4, w2), w7 = fast::cmul<T>(w4, w3);
    cmul_inplace<T>(vr[1], vi[1], w1.x, w1.y);
    cmul_inplace<T>(vr[2], vi[2], w2.x, w2.y);
    cmul_inplace<T>(vr[3], vi[3], w3.x, w3.y);
    cmul_inplace<T>(vr[4], vi[4], w4.x, w4.y);
    cmul_inplace<T>(vr[5], vi[5], w5.x, w5.y);
    cmul_inplace<T>(vr[6], vi[6], w6.x, w6.y);
    cmul_inplace<T>(vr[7], vi[7], w7.x, w7.y);
  }
  dft_reg<T, 8>(vr, vi);
}

// The whole transform; buf is one split complex row (real part, then imaginary part).
template <typename T, int LOGL>
__device__ __forceinline__ void fft_regs(T* __restrict__ buf, T (&vr)[kPPT], T (&vi)[kPPT],
                                         const cplx<T>* __restrict__ tw) {
  stage_first_regs<T, LOGL>(buf, vr, vi);
  stages8_mid<T, LOGL, 0>(buf, tw);
  stage_last_regs<T, LOGL>(buf, vr, vi, tw);
}

}  // namespace fast
}  // namespace birk
