// Internal declarations shared by the HIP translation units of libbirk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

#include "birk.h"
#include "birk_df32.h"

namespace birk {

// Longest transform a single workgroup performs in LDS (complex elements).
constexpr int kLdsMaxLog = 12;
constexpr int kLdsMax = 1 << kLdsMaxLog;
constexpr int kFftThreads = 256;

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <> struct C2<df32> { using type = df32c; };
template <typename T> using cplx = typename C2<T>::type;

// Index of a storage type in the per-precision table arrays: 0 double, 1 float,
// 2 double-float.
template <typename T>
constexpr int prec_index() {
  return std::is_same<T, double>::value ? 0 : std::is_same<T, float>::value ? 1 : 2;
}
constexpr int kNumPrec = 3;

// Per-instance data of the preconditioner and the solve.
struct Instance {
  int64_t Nn = 0, N = 0;
  int nx = 0;
  int64_t off = 0;      // vector offset (elements)
  int64_t joff = 0;     // per-node Jacobian offset (elements)
  int64_t jcoff = 0;    // constant Jacobian offset (elements)
  int64_t scan_off = 0; // offset into the preconditioner scan scratch (doubles)
  int64_t jsw_off = 0;  // offset into the swizzled per-node Jacobian buffer (doubles)
  double* w = nullptr;  // CC weights on the device [Nn]
};

// Four-step twiddles W_M^t = hi[t >> shift] * lo[t & (2^shift - 1)], one array pair per
// precision, shared by every transform of length M in the plan.
struct TwiddleSet {
  const void* hi[kNumPrec] = {nullptr, nullptr, nullptr};
  const void* lo[kNumPrec] = {nullptr, nullptr, nullptr};
  int shift = 0;
};

// Three-pass power-of-two product (birk_fast.hip): a run of consecutive instances with
// the same N, whose nc components are then contiguous with stride N_n.
struct FastGroup {
  int64_t Nn = 0, N = 0;
  int nc = 0;
  int64_t off = 0;       // vector offset of the first component
  int64_t work_off = 0;  // complex elements into work[0], work[1]
  int64_t part_off = 0;  // doubles into partials
  TwiddleSet tw;         // M = 2N
};

// General product path (birk_dct.hip): one pair of components (2p, 2p + 1) of one
// instance.  Plain old data, copied to the device; kernels index it by pair.
struct PairDesc {
  int64_t src = 0;       // vector offset of component 2p
  int64_t Nn = 0, N = 0, L = 0, M = 0;
  int64_t work = 0;      // complex offset of this pair's M-long slot in work[0..2]
  int64_t part = 0;      // offset of the pair's c^_0 partials (2 per block)
  int logM = 0, logM1 = 0, logM2 = 0, tw_shift = 0;
  int has2 = 0;          // component 2p + 1 exists
  int nblk = 0;          // 256-wide blocks over [0, N_n)
  const void* chirp[kNumPrec] = {nullptr, nullptr, nullptr};  // Bluestein chirp, or null (L = M)
  const void* filt[kNumPrec] = {nullptr, nullptr, nullptr};   // Bluestein filter spectrum / M
  const void* thi[kNumPrec] = {nullptr, nullptr, nullptr};    // four-step twiddles (M > kLdsMax)
  const void* tlo[kNumPrec] = {nullptr, nullptr, nullptr};
};

// Work lists of the general path.  Each launch of a phase covers every pair of every
// size: its grid is a list of tiles (pair, block) read from the device.
struct PairSet {
  std::vector<PairDesc> host;
  PairDesc* dev = nullptr;
  int2* tiles_m = nullptr;    // (pair, block of 256 over [0, M))
  int2* tiles_n = nullptr;    // (pair, block of 256 over [0, N_n))
  int2* tiles_lds = nullptr;  // (first pair, count): whole transforms of M <= kLdsMax
  int2* tiles_c4 = nullptr;   // (pair, column block) of the four-step first pass
  int2* tiles_r4 = nullptr;   // (pair, row block) of the four-step second pass
  int n_m = 0, n_n = 0, n_lds = 0, n_c4 = 0, n_r4 = 0;
  int64_t work = 0;           // complex elements needed per work buffer
  int64_t parts = 0;          // doubles of partials needed
};

}  // namespace birk

struct birk_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  birk_precision prec = BIRK_F64;
  std::vector<birk::Instance> inst;
  std::vector<birk::FastGroup> fgroups;
  birk::PairSet gen[2];           // general-path pairs: [0] 2N a power of two, [1] Bluestein
  std::vector<void*> allocs;      // device tables owned by the plan
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
  const void* lds_tw[birk::kNumPrec] = {nullptr, nullptr, nullptr};  // exp(-2 pi i t / kLdsMax)
  void* tmp_vec[4] = {nullptr, nullptr, nullptr, nullptr};  // vectors of total_len doubles
  // Krylov workspace, allocated by the first solve that needs it.
  int krylov_m = 0;
  void* krylov_Q = nullptr;   // (2m + 1) vectors of the Krylov precision (Q and Z)
  void* krylov_vec = nullptr; // 4 vectors of the Krylov precision
  double* krylov_dots = nullptr;  // [batch][2][kKryMaxDots + 1]
  double* krylov_part = nullptr;  // reduction partials
  int* flag = nullptr;            // device flag: singular pivot seen
  int use_fast = 1;               // power-of-two N takes the three-pass path
  int fast_lds_kb[2] = {128, 64};  // LDS budget per workgroup of the three-pass kernels [8-byte, 4-byte reals]
  int fast_ppt = 8;               // complex points per thread in the three-pass FFTs (8 or 16)
  int fast_split = 0;             // 0: rows of the first DCT are the longer side (L2 >= L1); 1: L1 >= L2
};

namespace birk {

// ---- products (birk_dct.hip) ----
template <typename T>
hipError_t apply_product(birk_plan* p, const T* v, T* out, int transpose, hipStream_t s);

// Lay out the general-path pairs and the fast groups of a plan, with their table needs;
// called once at plan creation, before any allocation of work buffers.
void plan_products(birk_plan* p);
// Allocate and fill every transform table and work list (after the work buffers exist).
hipError_t build_tables(birk_plan* p);

// ---- power-of-two three-pass path (birk_fast.hip) ----
bool fast_eligible(int64_t N);
template <typename T>
hipError_t fast_product(birk_plan* p, const FastGroup& g, const T* v, T* out, int transpose, hipStream_t s);
void fast_sizes(const birk_plan* p, int64_t N, int nc, int64_t* work, int64_t* part);

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
