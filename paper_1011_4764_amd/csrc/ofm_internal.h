// Internal declarations of the OFM library: device descriptors, handles and
// kernel launchers.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "ofm.h"

// extra block vectors beyond s_j in the fragment eigensolver (6 with the
// default filter degrees below measured best of 4..16 on the amorphous
// workload in both forms)
#ifndef OFM_GUARD_VECTORS
#define OFM_GUARD_VECTORS 6
#endif

namespace ofm {

// ---------------------------------------------------------------------------
// device-side fragment descriptor (plain old data, copied to HBM once)
// ---------------------------------------------------------------------------
// Face bits: which faces of the box lie on the global grid's walls.  The
// fragment operator has a wall at every face; the whole-system operator only
// at global-grid faces.
enum : int { FACE_XLO = 1, FACE_XHI = 2, FACE_YLO = 4, FACE_YHI = 8,
             FACE_ZLO = 16, FACE_ZHI = 32 };

struct FragDev {
  int lo[3], dims[3];     // box (global indices, x y z)
  int dlo[3], ddims[3];   // box grown by 2 per side, clipped to the grid
  int n_states;           // s_j
  int bw;                 // eigensolver block width b_j (s_j + guard, <= n_j)
  int npts;               // n_j
  int ld;                 // leading dimension of box vectors (n_j rounded up)
  int ndil;               // points of the dilated box
  int ldd;                // leading dimension of dilated-box vectors
  int gfaces;             // FACE_* bits of global-wall faces
  int small_off;          // offset of this fragment's b_j x b_j matrices
  int th_off;             // offset of this fragment's b_j Ritz values
  int rt_begin, rt_count; // range of this fragment's point chunks (rotation)
  long long v_off;        // offset of V restricted to the box (n_j values)
  long long x_off;        // offset of the b_j block vectors (b_j * ld)
  long long hphi_off;     // offset of the s_j dilated-box vectors (s_j * ldd)
  long long basis_off;    // offset of the fragment's states in the basis
  double vmax;            // max of V over the box (filter upper bound)
};

// one task of the grouped pair contraction: both blocks of the pair (j, n),
// j <= n, over Omega' = box_j ^ dil(box_n), the support of the H block:
//   H_jn = Phi_j^T (H Phi_n)  over Omega',
//   S_jn = Phi_j^T Phi_n      over Omega = box_j ^ box_n (inside Omega').
// Phi_j lives on box_j, Phi_n on box_n, H Phi_n on dil(box_n), x fastest.
struct PairTask {
  long long a_off;          // Phi_j, first state (state arena)
  long long b_off;          // Phi_n, first state (state arena)
  long long h_off;          // H Phi_n, first state (H phi arena)
  long long c_off;          // offset of both ma x mb row-major blocks
  int a_org[3];             // Omega' corner in box_j coordinates
  int b_org[3];             // Omega' corner in box_n coordinates (may be < 0)
  int h_org[3];             // Omega' corner in dil(box_n) coordinates
  int om[3];                // Omega' dims
  int s_lo[3], s_hi[3];     // Omega in Omega' coordinates, [s_lo, s_hi)
  int a_nx, a_nxy;          // box_j: points per row, per plane
  int b_nx, b_nxy;          // box_n
  int h_nx, h_nxy;          // dil(box_n)
  int lda, ldb, ldh;        // vector strides
  int ma, mb;               // s_j, s_n
  int sym;                  // diagonal block: symmetrise on write
  int has_s;                // Omega is not empty (else S_jn = 0)
  int ident;                // mixed form: S_jj = I (solver-orthonormalised)
  int frag;                 // j
};

// per-fragment Chebyshev filter state (device)
struct FilterState {
  double lower;   // lower end of the damped interval (largest block Ritz value)
  double upper;   // upper bound of the spectrum
  double scale;   // point normalised to 1 (smallest Ritz value)
  double worst;   // largest residual over the wanted states
  int lock;       // leading Ritz vectors already converged (not filtered)
  int pad;
};

struct KernelStat {
  long long launches = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
};

}  // namespace ofm

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct ofm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ofm_precision precision = OFM_FP64;
  std::string err;
  bool profiling = false;
  std::map<std::string, ofm::KernelStat> stats;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  struct Pending {
    std::string fam;
    hipEvent_t a, b;
    double bytes, flops;
    int launches;
  };
  std::vector<Pending> pending;
  double t_solve = 0, t_elem = 0, t_global = 0;
  void* blas = nullptr;    // rocblas_handle, created lazily
  int live = 0;            // fragment / matrix handles made with this context
  std::map<long long, int> tuned;  // stencil variant per (precision, plane class)
  std::map<int, int> pair_tuned;   // pair-kernel variant per (precision, tile class)
  int pair_variant = -1;           // pinned pair-kernel variant, -1: autotune
  int n_cu = 256;
};

struct ofm_frags {
  ofm_ctx* ctx = nullptr;
  ofm_grid grid{};
  int n_frag = 0;
  int guard = OFM_GUARD_VECTORS;
  std::vector<ofm::FragDev> host;      // descriptors (host copy)
  std::vector<int> pair_j, pair_n;     // pair list j <= n
  std::vector<long long> block_off;    // packed block offsets
  long long n_values = 0;              // sum over pairs of s_j * s_n
  long long n_basis = 0, total_points = 0;
  long long v_total = 0, x_total = 0, hphi_total = 0;
  int small_total = 0;
  int max_bw = 0, max_plane = 0, max_states = 0;
  ofm::FragDev* d_frag = nullptr;
  double* d_v = nullptr;       // V restricted to boxes (FP64): whole H
  float* d_v32 = nullptr;      // same, FP32 (mixed form)
  double* d_vf = nullptr;      // potential of the fragment Hamiltonians
  float* d_vf32 = nullptr;     // (aliases d_v / d_v32 unless own wells set)
  bool own_wells = false;
  void* d_x = nullptr;         // block vectors (T)
  void* d_p = nullptr;         // filter work vectors (T)
  void* d_hx = nullptr;        // H times block vectors (T)
  void* d_hphi = nullptr;      // whole-system H phi on dilated boxes (T)
  // tile lists: (fragment, vector < b_j), (fragment, state < s_j) and
  // (fragment, 256-point chunk)
  int2* d_tiles[3] = {nullptr, nullptr, nullptr};   // per stencil variant
  int n_tiles[3] = {0, 0, 0};
  // FP32: (fragment, vector) tiles of the boxes the on-chip filter takes,
  // and the strip tiles of the remaining boxes per variant
  int2* d_ftiles = nullptr;
  int n_ftiles = 0;
  int2* d_tiles_nr[3] = {nullptr, nullptr, nullptr};
  int n_tiles_nr[3] = {0, 0, 0};
  // multi-step kernel: (fragment, vector) tiles of the boxes it takes, with
  // the on-chip filter off [0] or on [1] (then it takes none of those), per
  // launch class (points per thread and workgroup size, multistep_class: one
  // launch per class, so a small plane does not run on a workgroup sized
  // for the largest), and the strip tiles of the remaining boxes per stencil
  // variant
  int2* d_vt[2][5] = {{nullptr, nullptr, nullptr, nullptr, nullptr},
                      {nullptr, nullptr, nullptr, nullptr, nullptr}};
  int n_vt[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
  int n_vt_all[2] = {0, 0};
  // width classes of the Gram and rotation kernels: one launch per class,
  // so a narrow block does not run with the registers of the widest one
  int* d_gfl[4] = {nullptr, nullptr, nullptr, nullptr};   // fragments with
  int n_gfl[4] = {0, 0, 0, 0};                            // ceil(bw/16) = 1..4
  int* d_rtl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int n_rtl[5] = {0, 0, 0, 0, 0};   // chunk indices, bw <= 16/24/32/48/64
  int2* d_tiles_rest[2][3] = {{nullptr, nullptr, nullptr},
                              {nullptr, nullptr, nullptr}};
  int n_tiles_rest[2][3] = {{0, 0, 0}, {0, 0, 0}};
  int variant = -1;            // stencil variant in use (-1: not chosen)
  int2* d_stiles = nullptr;
  int n_stiles = 0;
  int2* d_rtiles = nullptr;
  int n_rtiles = 0;
  int th_total = 0;
  // eigensolver work buffers
  double* d_G = nullptr;       // split-K Gram partials (16 per fragment)
  double* d_Q = nullptr;       // b_j x b_j rotation per fragment
  double* d_theta = nullptr;   // Ritz values (th_off indexing)
  double* d_res = nullptr;     // residual norms (th_off indexing)
  double* d_res_partial = nullptr;  // per rotation chunk, 64 entries
  ofm::FilterState* d_fs = nullptr;
  int* d_active = nullptr;
  int* d_iters = nullptr;
  unsigned char* d_conv = nullptr;
  int* d_flags = nullptr;
  int* d_nactive = nullptr;
  void* d_coef = nullptr;    // Chebyshev step coefficients (solve_impl)
  size_t coef_bytes = 0;
  std::vector<double> eps_host;  // sum_j s_j, valid when have_states
  bool have_states = false;
  // per fragment: 1 when its states come from ofm_solve_fragments (FP64
  // CholQR-orthonormal), 0 when imported with ofm_set_states
  std::vector<char> solver_states;
  // per fragment after a solve: bit 0 the CholQR Gram needed the shifted
  // Cholesky factorisation, bit 1 that one lost a pivot too
  std::vector<int> solve_flags;
  // tasks of the grouped pair contraction (planned once, longest first)
  std::vector<ofm::PairTask> pair_tasks;
};

struct ofm_mats {
  ofm_ctx* ctx = nullptr;
  const ofm_frags* frags = nullptr;
  long long n_values = 0, n_basis = 0;
  std::vector<int> pair_j, pair_n;
  std::vector<long long> block_off;
  std::vector<int> states;            // s_j per fragment
  std::vector<long long> basis_off;   // per fragment
  double* d_H = nullptr;
  double* d_S = nullptr;
};

// ---------------------------------------------------------------------------
// helpers shared by the host files
// ---------------------------------------------------------------------------
// Serialises HIP stream capture with rocBLAS / rocSOLVER calls across host
// threads (contexts driven from several threads at once): a capture in one
// thread (the fragment sweep's graph) and a call in another that touches the
// legacy stream (rocBLAS's hipBLASLt back end does, on first use) make that
// call fail, and hipBLASLt ends the process on the error.  A capture holds
// this lock exclusively, every rocBLAS / rocSOLVER call shared (calls of
// different threads still overlap); none is taken inside another.
namespace ofm {

std::shared_mutex& capture_lock();

struct Error {
  ofm_status code;
  std::string msg;
};

#define OFM_HIP(call)                                                       \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      throw ::ofm::Error{OFM_E_DEVICE, std::string(#call) + ": " +          \
                                           hipGetErrorString(e_)};          \
  } while (0)

#define OFM_REQUIRE(cond, code, msg)                                        \
  do {                                                                      \
    if (!(cond)) throw ::ofm::Error{code, msg};                             \
  } while (0)

template <typename T>
T* dev_alloc(size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess)
    throw Error{OFM_E_NOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) +
                                 " bytes failed"};
  return static_cast<T*>(p);
}

inline void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

// device buffer freed with its scope
template <typename T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) { p = dev_alloc<T>(n); }
  ~DevBuf() { dev_free(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// timed-launch bracket (no-op unless profiling is on)
struct Timed {
  ofm_ctx* c;
  std::string fam;
  double bytes, flops;
  int launches;
  hipEvent_t a = nullptr, b = nullptr;
  // `n` launches of the family happen between construction and destruction
  Timed(ofm_ctx* ctx, const char* family, double by, double fl, int n = 1);
  ~Timed();
};
void collect_stats(ofm_ctx* c);

// geometry planner (planner.cpp)
void plan_fragments(ofm_frags* f, const ofm_grid& g, int n_frag,
                    const ofm_fragment_desc* fr, int guard);
void plan_pairs(ofm_frags* f, const double* atom_xyz,
                const long long* frag_atom_ptr, const int* frag_atom_idx,
                double d_cut);
std::vector<PairTask> plan_pair_tasks(const ofm_frags* f);

// global solve (global_solve.cpp)
void global_solve(ofm_ctx* c, const ofm_mats* m, double s_thresh, double e_lo,
                  double e_hi, int* n_kept, int* n_eig, double* E, double* C,
                  double* s_min, const unsigned char* keep = nullptr);
void homo_energies(const ofm_mats* m, double* e);
// dense symmetric eigensolver (tridiag.hip): eigenvalues of the n x n
// symmetric A (full storage, column-major, leading dimension n; destroyed)
// in ascending order into w; with Z != nullptr the orthonormal eigenvectors
// into Z (n x n, leading dimension n).  info (device) is 0 on success.
// c (may be null) receives the "tridiag" kernel statistics.
void dense_eigh(ofm_ctx* c, hipStream_t s, void* blas_handle, int n, double* A,
                double* w, double* Z, int* info);
// the same on host arrays, on the context's stream
void dense_eigh_host(ofm_ctx* c, int n, const double* A, double* w, double* Z);
void destroy_blas(ofm_ctx* c);
// the matrix-element stage on a planned task list: sets the tasks' ident
// flags from the fragments' state origin, uploads the list to d_tasks
// (device, n_tasks entries), fills H and S (n_values doubles each, device)
// and launches the contraction kernels on the context stream; with
// may_tune, a kernel variant not yet chosen for this (precision, tile
// class) is chosen by timing each variant once (this synchronises)
void run_pair_elements(ofm_ctx* c, ofm_frags* f, PairTask* d_tasks, double* H,
                       double* S, bool may_tune);
// per-device scratch of the allocation-free entry point (noalloc.hip):
// resolved once per device at context creation
void noalloc_init(int device);

// kernel launchers (kernels.hip)
namespace k {
void restrict_potential(hipStream_t s, const double* V, const ofm_grid& g,
                        const ofm_frags* f);
void fragment_wells(hipStream_t s, const ofm_frags* f, const double* xyz,
                    const double* Z, const long long* ptr, const int* idx,
                    double sigma, double r_cut);
template <typename T>
void init_random(hipStream_t s, const ofm_frags* f, T* X,
                 unsigned long long seed);
constexpr int NVARIANT = 3;   // stencil variants (points per thread)
int stencil_ppt(int elem_bytes, int variant);
// strip tiles of the fragments with keep[j] (every fragment without keep)
std::vector<int2> stencil_tiles(const ofm_frags* f, int elem_bytes,
                                int variant, int nvec_only, int only,
                                const std::vector<char>* keep = nullptr);
// two or three Chebyshev steps per launch for boxes whose plane fits one
// workgroup
// launch classes of the multi-step kernel (ofm_frags::d_vt holds one tile
// list per class)
constexpr int NMSCLS = 5;
// launch class (1..NMSCLS) of the multi-step kernel for a box (0: not taken)
int multistep_class(int elem_bytes, const FragDev& d);
bool multistep_eligible(int elem_bytes, const FragDev& d);
template <typename T>
void apply_hm(ofm_ctx* c, const ofm_frags* f, T* IN, T* PV, const int2* tiles,
              int ntiles, int cls, int ns, const int* active, int step,
              const FilterState* fs, const void* coef, int cdeg,
              double alg_bytes, double flops);
// Chebyshev step coefficients of every fragment for steps 1..degree from
// the filter intervals in f->d_fs: `degree` records of 5 values of T per
// fragment (step_coef_bytes each), read by the filter kernels (mode 1)
template <typename T>
void step_coefs_table(hipStream_t s, const ofm_frags* f, int degree,
                      void* table);
inline size_t step_coef_bytes(int elem_bytes) { return 5 * (size_t)elem_bytes; }
// whole Chebyshev filter with the vector on chip (FP32, boxes <= 32^3)
bool resident_eligible(int elem_bytes, const FragDev& d);
void filter_resident(ofm_ctx* c, const ofm_frags* f, float* X,
                     const int2* tiles, int ntiles, const int* active,
                     const FilterState* fs, const void* coef, int degree,
                     double alg_bytes, double flops);
template <typename T>
void apply_h(ofm_ctx* c, const ofm_frags* f, const T* in, const T* prev,
             T* out, const int2* tiles, int ntiles, int variant,
             const int* active, int step, const FilterState* fs,
             const void* coef, int cdeg, int mode, long long base_override,
             double alg_bytes, double flops, hipEvent_t ev0 = nullptr,
             hipEvent_t ev1 = nullptr);
template <typename T>
void gram(ofm_ctx* c, const ofm_frags* f, const T* A, const T* B, double* G,
          const int* active, double bytes, double flops);
void gram_x3(ofm_ctx* c, const ofm_frags* f, const float* A, const float* B,
             double* G, const int* active, double bytes, double flops);
void cholinv(hipStream_t s, const ofm_frags* f, const double* G, double* Q,
             const int* active, int* flags);
void rr_eig(hipStream_t s, const ofm_frags* f, const double* G, double* Q,
            double* theta, const int* active, int pre);
template <typename T>
void rotate(ofm_ctx* c, const ofm_frags* f, T* X, T* HX, const double* Q,
            const double* theta, double* res_partial, const int* active,
            int upper, double bytes, double flops);
void finalize_iter(hipStream_t s, const ofm_frags* f, const double* theta,
                   const double* res_partial, FilterState* fs, int* active,
                   int* iters, unsigned char* conv, double tol, int* n_active,
                   double* res);
template <typename T>
void gauge(hipStream_t s, const ofm_frags* f, T* X);
template <typename T>
void whole_h(ofm_ctx* c, const ofm_frags* f, const T* X, T* HPHI,
             int only_frag);
// both blocks of every task of the list (the mixed form leaves the diagonal
// S blocks of imported states, tasks with sym and ident == 0, to
// pair_elements_f64_on_f32)
// variant (autotuned, same bits): 0 loads a chunk and then multiplies it,
// 1 keeps the next chunk's loads in flight during the products
constexpr int NPAIRVARIANT = 2;
template <typename T>
void pair_elements(ofm_ctx* c, const ofm_frags* f, const PairTask* tasks,
                   int n_tasks, const T* phi, const T* hphi, double* H,
                   double* S, double flops, double bytes, int variant);
// mixed form: the diagonal S blocks of imported states (tasks with sym and
// ident == 0 of the same list) with FP64 MFMA products on the FP32
// operands
void pair_elements_f64_on_f32(ofm_ctx* c, const ofm_frags* f,
                              const PairTask* tasks, int n_tasks,
                              const float* phi, const float* hphi, double* H,
                              double* S);
// zero n doubles (a kernel, not hipMemsetAsync: safe under stream capture)
void fill_zero(hipStream_t s, double* p, long long n);
template <typename T>
void convert(hipStream_t s, const double* in, T* out, long long n);
template <typename T>
void convert_back(hipStream_t s, const T* in, double* out, long long n);
constexpr int GCH = 16;   // split-K chunks per fragment of the Gram kernel
constexpr int RCH = 256;  // points per rotation chunk
// width class of the rotation kernel for a block of bw vectors (0..4:
// registers sized for 16, 24, 32, 48, 64 vectors)
inline int rotate_class(int bw) {
  return bw <= 16 ? 0 : bw <= 24 ? 1 : bw <= 32 ? 2 : bw <= 48 ? 3 : 4;
}
constexpr int SMAX = 64;  // largest block width
}  // namespace k

}  // namespace ofm
