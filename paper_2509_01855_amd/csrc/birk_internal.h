// Internal declarations shared by the HIP translation units of libbirk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "birk.h"

namespace birk {

// Longest transform a single workgroup performs in LDS (complex elements).
constexpr int kLdsMaxLog = 12;
constexpr int kLdsMax = 1 << kLdsMaxLog;
constexpr int kFftThreads = 256;

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <typename T> using cplx = typename C2<T>::type;

enum DctMethod { DCT_POW2 = 0, DCT_BLUESTEIN = 1 };

// Device tables of one precision for one instance.
struct DctTables {
  void* chirp = nullptr;   // Bluestein: chi_n = exp(-i pi n^2 / L), n in [0, L)
  void* filt = nullptr;    // Bluestein: FFT_M of conj(chi) wrapped, times 1/M
  void* tw4_hi = nullptr;  // four-step twiddles W_M^(t) = hi[t >> s] * lo[t & (2^s - 1)]
  void* tw4_lo = nullptr;
};

struct Instance {
  int64_t Nn = 0, N = 0;
  int nx = 0, npairs = 0;
  int64_t off = 0;      // vector offset (elements)
  int64_t joff = 0;     // per-node Jacobian offset (elements)
  int64_t jcoff = 0;    // constant Jacobian offset (elements)
  int method = DCT_POW2;
  int64_t L = 0;        // 2N: length of the even extension
  int64_t M = 0;        // FFT length (L for pow2, pow2 >= 2L - 1 for Bluestein)
  int logM = 0;
  int logM1 = 0, logM2 = 0;  // four-step split (logM1 + logM2 = logM) when M > kLdsMax
  int tw4_shift = 0;
  int64_t work_off = 0; // offset into the complex work buffers (elements)
  int64_t part_off = 0; // offset into the reduction partials (doubles)
  int nblk_mid = 0;     // blocks of the mid kernel per pair
  int64_t scan_off = 0; // offset into the preconditioner scan scratch (doubles)
  int64_t jsw_off = 0;  // offset into the swizzled per-node Jacobian buffer (doubles)
  double* w = nullptr;  // CC weights on the device [Nn]
  DctTables tab[2];     // [0] double, [1] float
};

struct ScanLevel {
  int64_t items = 0;    // number of aggregates at this level (per instance)
};

}  // namespace birk

struct birk_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  birk_precision prec = BIRK_F64;
  std::vector<birk::Instance> inst;
  int64_t total_len = 0;
  int64_t total_jnode = 0;
  int64_t total_jconst = 0;
  int64_t total_work = 0;     // complex elements per work buffer
  int64_t total_part = 0;
  int64_t total_scan = 0;
  void* work[3] = {nullptr, nullptr, nullptr};   // complex work buffers sized for double
  double* partials = nullptr;
  double* scan = nullptr;     // preconditioner scan scratch
  double* jsw = nullptr;      // per-node Jacobians and weights in the scan's thread layout
  int64_t total_jsw = 0;
  void* lds_tw[2] = {nullptr, nullptr};          // exp(-2 pi i t / kLdsMax), t < kLdsMax
  void* tmp_vec[4] = {nullptr, nullptr, nullptr, nullptr};  // vectors of total_len doubles
  // Krylov workspace, allocated by the first solve that needs it.
  int krylov_m = 0;
  void* krylov_Q = nullptr;   // (m + 1) vectors of the Krylov precision
  void* krylov_vec = nullptr; // 4 vectors of the Krylov precision
  double* krylov_dots = nullptr;  // [batch][2][kKryMaxDots + 1]
  double* krylov_part = nullptr;  // reduction partials
  int* flag = nullptr;            // device flag: singular pivot seen
  int use_fast = 1;               // power-of-two N takes the three-pass path
  int fast_lds_kb[2] = {128, 64};  // LDS budget per workgroup of the three-pass kernels [double, float]
  int fast_ppt = 8;               // complex points per thread in the three-pass FFTs (8 or 16)
  int fast_split = 0;             // 0: rows of the first DCT are the longer side (L2 >= L1); 1: L1 >= L2
};

namespace birk {

// ---- transforms (birk_dct.hip) ----
template <typename T>
hipError_t fft_batched(const birk_plan* p, const Instance& in, cplx<T>* data, cplx<T>* tmp,
                       int count, int inverse, hipStream_t s);

template <typename T>
hipError_t apply_product(birk_plan* p, const T* v, T* out, int transpose, hipStream_t s);

hipError_t build_tables(birk_plan* p);

// ---- power-of-two three-pass path (birk_fast.hip) ----
bool fast_eligible(const Instance& in);
template <typename T>
hipError_t fast_product(birk_plan* p, const Instance& in, const T* v, T* out, int transpose, hipStream_t s);
void fast_sizes(const birk_plan* p, const Instance& in, int64_t* work, int64_t* part);

// ---- preconditioner, Jacobian products and Krylov kernels (birk_solve.hip) ----
template <typename T>
hipError_t jac_times(birk_plan* p, int jac_kind, const double* J, const T* x, T* y,
                     hipStream_t s);
template <typename T>
hipError_t precond_forward(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           hipStream_t s);
template <typename T>
hipError_t precond_inverse(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           T* jout, hipStream_t s, int* flag);
int64_t pinv_scratch(int64_t Nn, int nx);
int64_t pinv_jsw_size(int64_t Nn, int nx);
// Lay out per-node J (or, for constant J, the weights) for the inverse scan; must precede
// precond_inverse whenever J changes.
// single = 1 lays the data out in float (for precond_inverse<float>), else in double.
hipError_t precond_prepare(birk_plan* p, int jac_kind, const double* J, int single, hipStream_t s);

// Krylov BLAS-1 launchers (birk_solve.hip).  Reductions accumulate in double.
constexpr int kKryMaxDots = 32;
namespace kry {
template <typename T>
void dots(const T* Q, int64_t ld, int nq, const T* u, int64_t n, double* part, double* out, hipStream_t s);
template <typename T>
void axpys(const T* Q, int64_t ld, int nq, const double* h, T* u, int64_t n, double* part, double* nrm_out,
           hipStream_t s);
template <typename T>
void normalize(const T* u, const double* nrm2, T* q, int64_t n, hipStream_t s);
template <typename TI, typename TO>
void scale_conv(const TI* x, TO* y, double alpha, int64_t n, hipStream_t s);
template <typename T>
void sub(const T* a, const T* b, T* z, int64_t n, hipStream_t s);
void residual(const double* beta, const double* x, const double* t, double* r, int64_t n, hipStream_t s);
template <typename T>
void add_to(double* x, const T* d, int64_t n, hipStream_t s);
template <typename T>
void combine(const T* Q, int64_t ld, int nq, const double* c, T* u, int64_t n, hipStream_t s);
}  // namespace kry

}  // namespace birk
