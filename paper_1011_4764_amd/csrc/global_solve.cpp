// Generalised eigenproblem sum_mn (H - E S) C = 0 in the fragment basis
// (method Eq. 2), FP64 on the GPU by thresholded canonical
// orthogonalisation:
//   S = U diag(s) U^T            (dense_eigh: own tridiagonal reduction,
//                                 rocSOLVER stedc and ormtr)
//   K = { k : s_k >= s_thresh }  (directions of S below the threshold are
//                                 linearly dependent combinations of
//                                 overlapping fragment states and are dropped)
//   X = U_K diag(s_K^-1/2)       (own kernel)
//   H' = X^T H X                 (two rocBLAS dgemm)
//   H' = Y diag(E) Y^T           (dense_eigh; rocSOLVER sterf without
//                                 vectors), C = X Y
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ofm_internal.h"

using namespace ofm;

namespace {

#define OFM_BLAS(call)                                                      \
  do {                                                                      \
    std::shared_lock<std::shared_mutex> lk_(ofm::capture_lock());           \
    rocblas_status s_ = (call);                                             \
    if (s_ != rocblas_status_success)                                       \
      throw Error{OFM_E_DEVICE, std::string(#call) + " failed: " +          \
                                    rocblas_status_to_string(s_)};          \
  } while (0)

// scatter the packed upper blocks (and their transposes) into dense N x N;
// sel maps a basis function to its row in the (possibly restricted) pencil,
// -1 for a function left out
__global__ void k_assemble(const int* __restrict__ pj, const int* __restrict__ pn,
                           const long long* __restrict__ boff,
                           const int* __restrict__ st,
                           const long long* __restrict__ bas,
                           const long long* __restrict__ sel, int npair,
                           const double* __restrict__ Hb,
                           const double* __restrict__ Sb, double* __restrict__ H,
                           double* __restrict__ S, long long N) {
  const int p = blockIdx.x;
  if (p >= npair) return;
  const int j = pj[p], n = pn[p];
  const int sj = st[j], sn = st[n];
  const long long r0 = bas[j], c0 = bas[n];
  for (int e = threadIdx.x; e < sj * sn; e += blockDim.x) {
    const int i = e / sn, m = e % sn;
    const long long r = sel[r0 + i], c = sel[c0 + m];
    if (r < 0 || c < 0) continue;
    const double h = Hb[boff[p] + e], s = Sb[boff[p] + e];
    // symmetric: column-major and row-major storage coincide
    H[r * N + c] = h;
    S[r * N + c] = s;
    H[c * N + r] = h;
    S[c * N + r] = s;
  }
}

// out[i] = v[idx[i]]
__global__ void k_gather(const double* __restrict__ v,
                         const long long* __restrict__ idx, int n,
                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v[idx[i]];
}

// X[:, k] = U[:, first + k] / sqrt(s[first + k])   (column-major N x K)
__global__ void k_scale_cols(const double* __restrict__ U,
                             const double* __restrict__ s, double* __restrict__ X,
                             long long N, int first, int K) {
  const long long total = N * (long long)K;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long col = e / N, row = e % N;
    X[e] = U[(first + col) * N + row] / sqrt(s[first + col]);
  }
}

// A = (A + A^T) / 2 for the K x K product X^T H X, whose two triangles
// differ by rounding
__global__ void k_symmetrize(double* __restrict__ A, int K) {
  const long long total = (long long)K * K;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % K), c = (int)(e / K);
    if (r < c) {
      const double m = 0.5 * (A[e] + A[c + (long long)r * K]);
      A[e] = m;
      A[c + (long long)r * K] = m;
    }
  }
}

rocblas_handle blas(ofm_ctx* c) {
  if (!c->blas) {
    rocblas_handle h;
    OFM_BLAS(rocblas_create_handle(&h));
    c->blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(c->blas);
  OFM_BLAS(rocblas_set_stream(h, c->stream));
  return h;
}

}  // namespace

namespace ofm {

void destroy_blas(ofm_ctx* c) {
  if (c && c->blas) {
    std::shared_lock<std::shared_mutex> lk(capture_lock());
    (void)rocblas_destroy_handle(static_cast<rocblas_handle>(c->blas));
    c->blas = nullptr;
  }
}

void homo_energies(const ofm_mats* m, double* e) {
  ofm_ctx* c = m->ctx;
  const int nf = (int)m->states.size();
  // offset of the last diagonal element of every diagonal block
  std::vector<long long> idx(nf, -1);
  for (size_t p = 0; p < m->pair_j.size(); ++p)
    if (m->pair_j[p] == m->pair_n[p]) {
      const int j = m->pair_j[p];
      const long long sj = m->states[j];
      idx[j] = m->block_off[p] + (sj - 1) * sj + (sj - 1);
    }
  for (int j = 0; j < nf; ++j)
    OFM_REQUIRE(idx[j] >= 0, OFM_E_STATE, "a fragment has no diagonal block");
  hipStream_t st = c->stream;
  DevBuf<long long> di(nf);
  DevBuf<double> out(nf);
  OFM_HIP(hipMemcpyAsync(di.p, idx.data(), sizeof(long long) * nf,
                         hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_gather, dim3((nf + 255) / 256), dim3(256), 0, st,
                     m->d_H, di.p, nf, out.p);
  OFM_HIP(hipGetLastError());
  OFM_HIP(hipMemcpyAsync(e, out.p, sizeof(double) * nf, hipMemcpyDeviceToHost,
                         st));
  OFM_HIP(hipStreamSynchronize(st));
}

void dense_eigh_host(ofm_ctx* c, int n, const double* A, double* w,
                     double* Z) {
  hipStream_t st = c->stream;
  rocblas_handle h = blas(c);
  const long long nn = (long long)n * n;
  DevBuf<double> Ad(nn), wd(n), Zd(Z ? nn : 1);
  DevBuf<int> info(1);
  OFM_HIP(hipMemcpyAsync(Ad.p, A, sizeof(double) * nn, hipMemcpyHostToDevice,
                         st));
  dense_eigh(c, st, h, n, Ad.p, wd.p, Z ? Zd.p : nullptr, info.p);
  int info_h = 0;
  OFM_HIP(hipMemcpyAsync(&info_h, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  OFM_HIP(hipMemcpyAsync(w, wd.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (Z)
    OFM_HIP(hipMemcpyAsync(Z, Zd.p, sizeof(double) * nn, hipMemcpyDeviceToHost,
                           st));
  OFM_HIP(hipStreamSynchronize(st));
  OFM_REQUIRE(info_h == 0, OFM_E_DEVICE, "the tridiagonal eigensolver did not converge");
}

void global_solve(ofm_ctx* c, const ofm_mats* m, double s_thresh, double e_lo,
                  double e_hi, int* n_kept, int* n_eig, double* E, double* C,
                  double* s_min, const unsigned char* keep) {
  // rows of the pencil: every basis function, or the kept ones in order
  std::vector<long long> selh(m->n_basis);
  long long N = 0;
  for (long long i = 0; i < m->n_basis; ++i)
    selh[i] = (!keep || keep[i]) ? N++ : -1;
  OFM_REQUIRE(N >= 1, OFM_E_INVALID, "no basis function is kept");
  OFM_REQUIRE(N <= 200000, OFM_E_INVALID,
              "basis size outside the dense solver's range");
  hipStream_t st = c->stream;
  rocblas_handle h = blas(c);
  const int np = (int)m->pair_j.size();
  const int nf = (int)m->states.size();
  DevBuf<double> H(N * N), S(N * N), U(N * N), s(N);
  DevBuf<int> pj(np), pn(np), sts(nf), info(1);
  DevBuf<long long> boff(np), bas(nf), sel(m->n_basis);
  OFM_HIP(hipMemcpyAsync(sel.p, selh.data(), sizeof(long long) * m->n_basis,
                         hipMemcpyHostToDevice, st));
  OFM_HIP(hipMemsetAsync(H.p, 0, sizeof(double) * N * N, st));
  OFM_HIP(hipMemsetAsync(S.p, 0, sizeof(double) * N * N, st));
  OFM_HIP(hipMemcpyAsync(pj.p, m->pair_j.data(), sizeof(int) * np,
                         hipMemcpyHostToDevice, st));
  OFM_HIP(hipMemcpyAsync(pn.p, m->pair_n.data(), sizeof(int) * np,
                         hipMemcpyHostToDevice, st));
  OFM_HIP(hipMemcpyAsync(boff.p, m->block_off.data(), sizeof(long long) * np,
                         hipMemcpyHostToDevice, st));
  OFM_HIP(hipMemcpyAsync(sts.p, m->states.data(), sizeof(int) * nf,
                         hipMemcpyHostToDevice, st));
  OFM_HIP(hipMemcpyAsync(bas.p, m->basis_off.data(), sizeof(long long) * nf,
                         hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_assemble, dim3(np), dim3(256), 0, st, pj.p, pn.p,
                     boff.p, sts.p, bas.p, sel.p, np, m->d_H, m->d_S, H.p, S.p,
                     N);
  OFM_HIP(hipGetLastError());
  // eig(S), ascending
  dense_eigh(c, st, h, (int)N, S.p, s.p, U.p, info.p);
  std::vector<double> sh(N);
  int info_h = 0;
  OFM_HIP(hipMemcpyAsync(sh.data(), s.p, sizeof(double) * N,
                         hipMemcpyDeviceToHost, st));
  OFM_HIP(hipMemcpyAsync(&info_h, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  OFM_HIP(hipStreamSynchronize(st));
  OFM_REQUIRE(info_h == 0, OFM_E_DEVICE, "eig(S) did not converge");
  long long first = 0;
  while (first < N && !(sh[first] >= s_thresh)) ++first;
  const int K = (int)(N - first);
  if (n_kept) *n_kept = K;
  if (K == 0) {
    *n_eig = 0;
    throw Error{OFM_E_SINGULAR, "every eigenvalue of S is below the threshold"};
  }
  if (s_min) *s_min = sh[first];
  DevBuf<double> X(N * (long long)K), T1(N * (long long)K), Hp((long long)K * K),
      E_d(K);
  hipLaunchKernelGGL(k_scale_cols, dim3(1024), dim3(256), 0, st, U.p, s.p, X.p,
                     N, (int)first, K);
  OFM_HIP(hipGetLastError());
  const double one = 1.0, zero = 0.0;
  // T1 = H X  (N x K), H' = X^T T1  (K x K)
  OFM_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none,
                         (rocblas_int)N, K, (rocblas_int)N, &one, H.p,
                         (rocblas_int)N, X.p, (rocblas_int)N, &zero, T1.p,
                         (rocblas_int)N));
  OFM_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none,
                         K, K, (rocblas_int)N, &one, X.p, (rocblas_int)N, T1.p,
                         (rocblas_int)N, &zero, Hp.p, K));
  hipLaunchKernelGGL(k_symmetrize, dim3(1024), dim3(256), 0, st, Hp.p, K);
  OFM_HIP(hipGetLastError());
  // the eigenvectors of H' replace U (no longer needed) when asked for
  double* Y = C ? U.p : nullptr;
  dense_eigh(c, st, h, K, Hp.p, E_d.p, Y, info.p);
  std::vector<double> Eh(K);
  OFM_HIP(hipMemcpyAsync(Eh.data(), E_d.p, sizeof(double) * K,
                         hipMemcpyDeviceToHost, st));
  OFM_HIP(hipMemcpyAsync(&info_h, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  OFM_HIP(hipStreamSynchronize(st));
  OFM_REQUIRE(info_h == 0, OFM_E_DEVICE, "eig(H') did not converge");
  int lo = 0;
  while (lo < K && !(Eh[lo] >= e_lo)) ++lo;
  int hi = lo;
  while (hi < K && Eh[hi] <= e_hi) ++hi;
  const int ne = hi - lo;
  *n_eig = ne;
  for (int i = 0; i < ne; ++i) E[i] = Eh[lo + i];
  if (C && ne > 0) {
    // C = X Y[:, lo:hi]   (N x ne, column-major, stride N)
    DevBuf<double> Cd(N * (long long)ne);
    OFM_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none,
                           (rocblas_int)N, ne, K, &one, X.p, (rocblas_int)N,
                           Y + (long long)lo * K, K, &zero, Cd.p,
                           (rocblas_int)N));
    OFM_HIP(hipMemcpyAsync(C, Cd.p, sizeof(double) * N * ne,
                           hipMemcpyDeviceToHost, st));
    OFM_HIP(hipStreamSynchronize(st));
  }
}

}  // namespace ofm
