// Internal declarations shared by the HIP translation units of libbirk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <string>
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

// One component of one instance, for the per-component corrections of the b-form
// products and the endpoint row (birk_bform.hip).
struct CompDesc {
  int64_t off;       // vector offset of the component
  int64_t Nn;        // its node count
  const double* w;   // CC weights of its instance
  int64_t part;      // offset of its reduction partials
};
constexpr int kCompTiles = 256;  // most reduction tiles per component

// One instance, for the node-wise model kernels of the Newton solve (birk_newton.hip).
struct InstDesc {
  int64_t off;       // vector offset
  int64_t Nn;        // node count
  int64_t joff;      // per-node Jacobian offset
  int64_t nx;        // state count
  int64_t jcoff;     // constant Jacobian offset
  int64_t scan_off;  // offset into the preconditioner scan scratch
  const double* w;   // CC weights
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
// Tile schedule of the three-pass kernels (environment defaults, or the autotuner's
// choice per group of same-length components).
struct FastKnobs {
  int lds_kb[2] = {128, 64};  // LDS budget per workgroup of the runtime-length kernels [8-byte, 4-byte reals]
  int split = 0;              // 0: rows of the first DCT are the longer side (L2 >= L1); 1: L1 >= L2
  int tb = 0;                 // rows per pass-B tile (0: from the LDS budget; 2 or 4 in the register kernel)
  int b_threads = 512;        // workgroup size cap of the runtime-length pass B
  int xcd = 1;                // XCD-aware tile order
  int b2 = 1;                 // compile-time-length kernels where they apply
  int streams = 1;            // 2 or 3: the components run in that many parts on as many
                              // streams, so that one part's next pass fills another's tail
  int narrow = 0;             // 1: passes A and C of L1 = 2^9, 2^10 in tiles of 4 columns (else 8);
                              // plans of 8-byte reals start with 1
  int b3 = 1;                 // two-row pass B with the row transforms register-resident at both ends
};

struct FastGroup {
  int64_t Nn = 0, N = 0;
  int nc = 0;
  int64_t off = 0;       // vector offset of the first component
  int64_t work_off = 0;  // complex elements into work[0], work[1]
  int64_t part_off = 0;  // doubles into partials
  TwiddleSet tw;         // M = 2N
  FastKnobs kn;          // tile schedule of this group
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

// Inverse-preconditioner scan of one instance (birk_solve.hip): level sizes and the
// offsets of its aggregates and start states in the plan's scan scratch.
constexpr int kPinvMaxLevels = 8;
struct PinvDesc {
  int64_t Nn = 0, off = 0, joff = 0, jcoff = 0, jsw_off = 0;
  const double* w = nullptr;            // CC weights
  int64_t cnt[kPinvMaxLevels] = {};     // cnt[0] chunks of kChunk nodes, then groups of kFan
  int64_t agg[kPinvMaxLevels] = {};     // aggregate offsets (doubles) per level
  int64_t st[kPinvMaxLevels] = {};      // start-state offsets (doubles) per level
  int L = 0;                            // top level
  int nb0 = 0;                          // level-0 blocks of 64 groups
  // wave-scan path (n_x <= kWaveNx): tiles of kTileNodes nodes
  int64_t ntile = 0;                    // tiles of the instance
  int64_t tagg = 0, tst = 0;            // tile aggregates and start states, [field][tile] (doubles)
  int64_t tmap = 0;                     // inclusive chunk maps, [tile][field][thread] (doubles)
};

// Instances with one state count n_x: each scan phase is one launch over all of them.
struct PinvClass {
  int nx = 0;
  int ninst = 0;
  int Lmax = 0;
  std::vector<PinvDesc> host;
  PinvDesc* dev = nullptr;
  int2* t_node0 = nullptr;                   // (k, block) over level-0 threads
  int n_node0 = 0;
  int2* t_up[kPinvMaxLevels] = {};           // (k, block) over cnt[l + 1] parents of level l
  int n_up[kPinvMaxLevels] = {};
  int2* t_nodes = nullptr;                   // (k, block of 256 nodes): J x
  int n_nodes = 0;
  int2* t_tile = nullptr;                    // (k, tile) of the wave-scan path
  int n_tile = 0;
};

// Backward scan of P^{-T} (birk_kkt.hip): one instance of one n_x class.
struct BtDesc {
  int64_t Nn, off, joff, jcoff;
  int64_t nblk;        // blocks of 1024 nodes
  int64_t soff;        // offset of its block maps and entry states in the scan scratch (doubles)
  const double* w;     // CC weights
};
struct BtClass {
  int nx = 0, ninst = 0;
  int nblk = 0;        // (instance, block) tiles over all instances
  int nnode = 0;       // (instance, block of 256 nodes) tiles
  BtDesc* dev = nullptr;
  int2* tiles = nullptr;
  int2* ntiles256 = nullptr;
};

// Krylov vector segmentation: tiles of kSegChunk elements, each inside one instance.
constexpr int kSegChunk = 2048;
struct SegSet {
  int2* tiles = nullptr;    // (instance, chunk)
  int ntiles = 0;
  int2* ranges = nullptr;   // per instance [first tile, end tile)
  int64_t* ioff = nullptr;  // per instance vector offset
  int64_t* ilen = nullptr;  // per instance length n_x N_n
};

}  // namespace birk

struct birk_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  birk_precision prec = BIRK_F64;
  std::vector<birk::Instance> inst;
  std::vector<birk::FastGroup> fgroups;
  birk::PairSet gen[2];           // general-path pairs: [0] 2N a power of two, [1] Bluestein
  std::vector<birk::PinvClass> pclass;  // preconditioner scan schedule, one class per n_x
  birk::SegSet seg;               // Krylov segmentation of the batch
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
  double* krylov_part = nullptr;  // reduction partials [tiles][kKryMaxDots + 1]
  double* krylov_coef = nullptr;  // per instance: scale factors / combination coefficients,
                                  // followed by the counts krylov_cnt (one upload for both)
  int* krylov_cnt = nullptr;      // per instance: number of combined basis vectors
  double* krylov_gm = nullptr;    // device-side GMRES state, kGmStride doubles per instance
  double* krylov_prm = nullptr;   // per instance (active, tolerance, ||r||), then 3 flags
  void* krylov_stage = nullptr;   // pinned host staging: dots, singular flag, coefficients + counts
  int* flag = nullptr;            // device flag: singular pivot seen
  birk::CompDesc* comps = nullptr;  // component table (device), one entry per component
  int64_t ncomp = 0;
  int64_t max_nn = 0;               // longest component
  birk::InstDesc* idesc = nullptr;  // instance table (device)
  int2* pfwd_tiles = nullptr;       // P y tiles: (instance, component * tiles + tile)
  int pfwd_ntiles = 0;
  int2* pfwd_pairs = nullptr;       // P y scans: (instance, component)
  int pfwd_npairs = 0;
  int2* pfwd_btiles = nullptr;      // P y, all components at once: (instance, tile)
  int pfwd_nbtiles = 0;
  int pfwd_maxnx = 0;               // largest n_x of the plan
  int pfwd_unx = 0;                 // the n_x every instance shares, else 0
  void* newton_buf = nullptr;       // Newton workspace, allocated by the first Newton solve
  std::vector<birk::BtClass> btclass;  // P^{-T} scan schedule, one class per n_x
  int64_t total_bt = 0;             // doubles of P^{-T} scan scratch
  double* bt_scr = nullptr;         // P^{-T} scan scratch (block maps and entry states)
  void* kkt_buf = nullptr;          // KKT / MINRES workspace, allocated by the first KKT solve
  double* comp_val = nullptr;       // one double per component (last node, or a total)
  double* comp_part = nullptr;      // per-component reduction partials (CompDesc::part)
  int use_fast = 1;               // power-of-two N takes the three-pass path
  int blu_split[40] = {};         // log2 M1 of the Bluestein two-step FFTs per log2 M (0: default)
  birk::FastKnobs fast_kn;        // default tile schedule of the three-pass groups
  // HIP graphs of the products (birk_plan_set_graphs), per (direction, input, output)
  struct GraphSlot {
    int transpose;
    const void* v;
    void* out;
    hipGraphExec_t exec;  // null until the second use of the triple
    uint64_t used;
  };
  int use_graphs = 0;
  std::vector<GraphSlot> graphs;
  // HIP graphs of GMRES chunks (graph mode): Arnoldi steps [j0, j0 + k) for one precision,
  // restart length, Jacobian pointer and kind, preconditioner setting and J z storage
  struct KryGraph {
    int prec, j0, k, m;
    const double* J;
    int jk, use_precond, keep_jz, cached;
    hipGraphExec_t exec;
  };
  std::vector<KryGraph> kgraphs;
  uint64_t graph_clock = 0;
  // extra streams and their fork / join events of the multi-stream three-pass schedule
  static constexpr int kExtraStreams = 2;
  hipStream_t xstream[kExtraStreams] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kExtraStreams] = {nullptr, nullptr};
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
// Autotuner of the three-pass groups (birk_plan_tune); appends a summary to *report.
hipError_t tune_fast(birk_plan* p, hipStream_t s, std::string* report);
// Autotuner of the general path: the two-step split of each Bluestein size (birk_dct.hip).
hipError_t tune_general(birk_plan* p, hipStream_t s, std::string* report);

// ---- b-form corrections and the endpoint row (birk_bform.hip) ----
// Build the component table and its partial-sum scratch (after the weights exist).
hipError_t plan_bform(birk_plan* p);
// out[c][k] -= out[c][N] for every component c (B^a v -> B^b v).
template <typename T>
hipError_t bform_correct(birk_plan* p, T* out, hipStream_t s);
// Partial sums of every component of g, kept for bform_correct_T.
template <typename T>
hipError_t bform_sums(birk_plan* p, const T* g, hipStream_t s);
// out[c][k] -= w_k (1^T g_c) from the sums of bform_sums (B^aT g -> B^bT g).
template <typename T>
hipError_t bform_correct_T(birk_plan* p, T* out, hipStream_t s);
// xb[c] = xa[c] + w^T v_c.
template <typename T>
hipError_t endpoint(birk_plan* p, const double* xa, const T* v, double* xb, hipStream_t s);

// ---- Newton solve of the nonlinear IVP (birk_newton.hip) ----
hipError_t plan_instances(birk_plan* p);
// Two-body right-hand side F and per-node Jacobian J (either may be null), n_x = 6.
hipError_t two_body(birk_plan* p, double mu, double scale, const double* X, double* F, double* J, hipStream_t s);
// G = X - xa - G per component (G holds B^a F on entry).
hipError_t ivp_residual(birk_plan* p, const double* xa, const double* X, double* G, hipStream_t s);

// ---- preconditioner, Jacobian products and Krylov kernels (birk_solve.hip) ----
template <typename T>
hipError_t jac_times(birk_plan* p, int jac_kind, const double* J, const T* x, T* y,
                     hipStream_t s);
template <typename T>
hipError_t precond_forward(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           hipStream_t s);
// cached = 1: per-node H_k laid out by precond_prepare(..., kPrepCache) for this J.
template <typename T>
hipError_t precond_inverse(birk_plan* p, int jac_kind, const double* J, const T* y, T* out,
                           T* jout, hipStream_t s, int* flag, int cached);
// P^{-T} y for the instances with n_x <= 8 (backward wave scan, double); the instances
// with larger n_x are left untouched (birk_kkt.hip covers them).  cached = 1: per-node
// H_k laid out by precond_prepare(..., kPrepCache) in double for this J (read transposed).
hipError_t precond_inverse_t_wave(birk_plan* p, int jac_kind, const double* J, const double* y, double* out,
                                  hipStream_t s, int cached);
int64_t pinv_scratch(int64_t Nn, int nx);
int64_t pinv_jsw_size(int64_t Nn, int nx);
// Build the per-n_x scan classes and the Krylov segmentation (after scan_off, jsw_off
// and the weights exist); allocations are recorded in p->allocs.
hipError_t plan_solve(birk_plan* p);
// Per-J preparation of the inverse scan; must precede precond_inverse whenever J changes.
// kPrepLarge: n_x > 8 lay H_k out in the level-0 slots (always needed there).
// kPrepCache: n_x <= 8 with per-node J lay H_k out in the tile layout, read by
// precond_inverse with cached = 1 (worth it from the second application with one J).
// single = 1 lays the data out in float (for precond_inverse<float>), else in double.
constexpr int kPrepLarge = 1, kPrepCache = 2;
hipError_t precond_prepare(birk_plan* p, int jac_kind, const double* J, int single, hipStream_t s,
                           int what);

// Krylov BLAS-1 launchers (birk_solve.hip).  Reductions accumulate in double.
constexpr int kKryMaxDots = 32;
// Device-side GMRES state per instance (doubles): rotated Hessenberg columns R
// (column-major, kGmLd rows per column), g, cos, sin, then the scalars of GM_*.
constexpr int kGmLd = kKryMaxDots + 1;
constexpr int kGmR = 0;
constexpr int kGmG = kGmLd * kKryMaxDots;
constexpr int kGmCs = kGmG + kGmLd;
constexpr int kGmSn = kGmCs + kKryMaxDots;
constexpr int kGmMisc = kGmSn + kKryMaxDots;
enum { GM_RUN, GM_ACTIVE, GM_JEND, GM_INNER, GM_STATUS, GM_TOL, GM_RNORM, kGmMiscLen };
constexpr int kGmStride = kGmMisc + kGmMiscLen + 1;
namespace kry {
template <typename T>
void sub(const T* a, const T* b, T* z, int64_t n, hipStream_t s);
void residual(const double* beta, const double* x, const double* t, double* r, int64_t n, hipStream_t s);
// Segmented forms over every instance of the batch at once (ld = plan length; per
// instance i results at out + i * ostride).
template <typename T>
void sdots(const birk_plan* p, const T* Q, int nq, const T* u, double* out, int64_t ostride, hipStream_t s);
// u = a - b, then the dots of sdots, in one pass
template <typename T>
void sub_sdots(const birk_plan* p, const T* Q, int nq, const T* a, const T* b, T* u, double* out, int64_t ostride,
               hipStream_t s);
template <typename T>
void saxpys(const birk_plan* p, const T* Q, int nq, const double* h, int64_t hstride, T* u, double* nrm_out,
            hipStream_t s);
// u -= sum_k h_k Q_k, then out = (Q_k . u for k < nq, ||u||^2 in the norm slot): the
// update and the next Gram-Schmidt dot products in one pass
template <typename T>
void saxpys_dots(const birk_plan* p, const T* Q, int nq, const double* h, int64_t hstride, T* u, double* out,
                 int64_t ostride, hipStream_t s);
template <typename T>
void snormalize(const birk_plan* p, const T* u, const double* nrm2, int64_t stride, T* q, hipStream_t s);
template <typename TI, typename TO>
void sscale_conv(const birk_plan* p, const TI* x, TO* y, const double* alpha, hipStream_t s);
// x += sum_{k < cnt[i]} c[i][k] Q_k (x double, the sum in double)
template <typename T>
void scombine(const birk_plan* p, const T* Q, const double* c, int64_t cstride, const int* cnt, double* x,
              hipStream_t s);
// device-side GMRES scalars: prm = (active, tolerance, ||r||) per instance
void gm_init(const birk_plan* p, const double* prm, double* st, hipStream_t s);
void gm_column(const birk_plan* p, int j, const double* dots, int64_t dstride, double* st, hipStream_t s);
void gm_solve(const birk_plan* p, double* st, double* coef, int64_t cstride, int* cnt, double* flags, hipStream_t s);
void gm_running(const birk_plan* p, const double* st, double* flags, hipStream_t s);
}  // namespace kry

// ---- the KKT form and MINRES (birk_kkt.hip) ----
// Build the P^{-T} scan classes (after the weights exist).
hipError_t plan_kkt(birk_plan* p);
// x = P^{-T} y in double (scr: the plan's KKT scan scratch).  cached = 1: the per-node
// H_k tables of precond_prepare(..., kPrepCache) (double) hold this J.
hipError_t precond_inverse_t(birk_plan* p, int jac_kind, const double* J, const double* y, double* x, double* scr,
                             hipStream_t s, int cached = 0);
// y_k = J_k^T x_k per node, double.
hipError_t jac_t_times(birk_plan* p, int jac_kind, const double* J, const double* x, double* y, hipStream_t s);
// MINRES on [[H, A^T], [A, 0]] [chi; lambda] = [f; g] (h or f null: identity, zero).
birk_status kkt_solve(birk_plan* p, int jac_kind, const double* J, const double* h, const double* f,
                      const double* g, double* chi, double* lam, const birk_solve_opts* o, birk_solve_info* info);

}  // namespace birk
