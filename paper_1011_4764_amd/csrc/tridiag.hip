// Dense symmetric eigensolver of the global solve.
//
// Householder reduction to tridiagonal form, T = Q^T A Q with
// Q = H_0 H_1 ... H_{n-2}, H_i = I - tau_i v_i v_i^T, in the blocked form of
// Golub & Van Loan (Sec. 8.3.1, with the panel factorisation of LAPACK's
// latrd).  The output follows the LAPACK lower-storage convention (D the
// diagonal, E the subdiagonal, v_i in A(i+2:n, i) with its unit leading
// element implicit at A(i+1, i), which holds E(i) on return, and tau_i), so
// rocSOLVER's divide and conquer (stedc) takes T directly; the eigenvalues
// alone come from multisection on the Sturm count, and Q is applied to the
// tridiagonal eigenvectors in blocks of reflectors (both below).
//
// Shape on the GPU: the matrix is kept in full symmetric storage (both
// triangles) with the leading dimension padded to 64 rows, so the product
// with the trailing matrix is a column-parallel, coalesced matrix-vector
// product that streams each column once.  Each column takes two launches
// and no workgroup ever waits for another: k_mv forms y = A22 v and the
// panel projections W^T v, V^T v (one dot product per wave), every wave
// rebuilding the reflector from the previous launch's partial norms; k_fin,
// row-parallel, forms w (its correction -tau/2 (w.v) v from
// w.v = tau (y.v - 2 u1.u2)), stores v and w, and applies the panel's
// reflectors to the next column.  After a panel of NB columns one GEMM
// applies A22 -= V W^T + W V^T.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

#include "ofm_internal.h"

namespace ofm {
namespace {

#ifndef OFM_TD_NB
#define OFM_TD_NB 32
#endif
constexpr int NB = OFM_TD_NB;   // panel width (a multiple of 4, at most 64)

// one DPP step on both halves of a double
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf,
                                             true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the wave, the same value (and the same rounding) in every lane:
// quad swaps and row rotations by DPP, then the four rows' sums in order
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);   // row_ror:4
  v += dpp_d<0x128>(v);   // row_ror:8
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// sum over a workgroup of NW waves, returned to every thread
template <int NW>
__device__ double block_sum(double v, double* red) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  for (int k = 0; k < NW; ++k) s += red[k];
  return s;
}

constexpr int FR = 256;   // rows per workgroup of the row-parallel kernels

// Start of the panel at column p (already updated by every earlier panel):
// partial sums of A(r, p)^2 over rows r >= p+2, one per FR rows from p+1.
__global__ __launch_bounds__(FR) void k_pstart(const double* A, long long lda,
                                               int n, int p, double* part) {
  __shared__ double red[FR / 64];
  const int r = p + 1 + blockIdx.x * FR + threadIdx.x;
  double x = 0;
  if (r >= p + 2 && r < n) x = A[r + (long long)p * lda];
  const double s = block_sum<FR / 64>(x * x, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

constexpr int MV = 256;   // threads of k_mv (one wave per dot product)
constexpr int MU = 4;     // double2 loads in flight per lane in k_mv

// Column i = p + il: c = A(i:n, i) holds the column with every earlier
// reflector applied; v(i+1) = 1, v(r) = scale c(r) for r >= i+2.  Waves
// 0..L-1 form y(k) = A22(:, k) . v, waves L..L+il-1 u1 = W(i+1:n, 0:il)^T v,
// the next il waves u2 = V(i+1:n, 0:il)^T v, each as x(i+1) + scale
// sum_{r>=i+2} x(r) c(r), so that the loads do not wait for the reflector.
// Each wave then sums the np partial norms of c(i+2:n) and builds the
// reflector (beta, tau, scale = 1/(c(i+1) - beta)); pm gets each
// workgroup's share of y . v.
// Storage: lda and ldw even and at least n rounded up to even, rows n.. of
// A and W zero, so every column is read as 16-byte pairs from the even row
// rb = (i+1) & ~1 (the pair holding row i+1 is formed by lane 0 alone).
__global__ __launch_bounds__(MV) void k_mv(
    const double* A, long long lda, int n, int p, int il, const double* W,
    long long ldw, const double* part, int np, double* D, double* E,
    double* tau, double* sc, double* y, double* u, double* pm) {
  __shared__ double red[MV / 64];
  const int i = p + il;
  const int L = n - i - 1;
  const double* c = A + (long long)i * lda;   // indexed by row
  const int wave = blockIdx.x * (MV / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // the reflector's inputs, loaded with the columns; every wave sums the
  // partial norms itself (same order everywhere, so every wave of every
  // workgroup gets the same value)
  double ss = 0;
  for (int k = lane; k < np; k += 64) ss += part[k];
  const double alpha = c[i + 1], cii = c[i];
  double s1 = 0, sr = 0, cy = 0;   // x(i+1), sum_{r>=i+2} x(r) c(r), c(ycol)
  int ycol = -1;
  if (wave < L + 2 * il) {
    const double* col;
    if (wave < L) {
      ycol = i + 1 + wave;
      col = A + (long long)ycol * lda;
      cy = c[ycol];
    } else if (wave < L + il) {
      col = W + (long long)(wave - L) * ldw;
    } else {
      col = A + (long long)(p + wave - L - il) * lda;
    }
    const int rb = (i + 1) & ~1;
    const int npair = (n - rb + 1) >> 1;
    const double2* a2 = reinterpret_cast<const double2*>(col + rb);
    const double2* c2 = reinterpret_cast<const double2*>(c + rb);
    if (lane == 0) {   // pair 0: rows rb, rb+1, one of them is i+1
      const double2 a = a2[0], cc = c2[0];
      if (rb == i + 1) {
        s1 = a.x;
        sr = a.y * cc.y;
      } else {
        s1 = a.y;
      }
    }
    double acc[MU];
#pragma unroll
    for (int q = 0; q < MU; ++q) acc[q] = 0;
    int k = 1 + lane;
    for (; k + 64 * (MU - 1) < npair; k += 64 * MU) {
      double2 a[MU], cc[MU];
#pragma unroll
      for (int q = 0; q < MU; ++q) {
        a[q] = a2[k + 64 * q];
        cc[q] = c2[k + 64 * q];
      }
#pragma unroll
      for (int q = 0; q < MU; ++q) acc[q] += a[q].x * cc[q].x + a[q].y * cc[q].y;
    }
    for (; k < npair; k += 64) {
      const double2 a = a2[k], cc = c2[k];
      acc[0] += a.x * cc.x + a.y * cc.y;
    }
#pragma unroll
    for (int q = 0; q < MU; ++q) sr += acc[q];
    s1 = wave_sum_d(s1);
    sr = wave_sum_d(sr);
  }
  const double xn2 = wave_sum_d(ss);
  double t = 0, beta = alpha, scale = 1;
  if (xn2 > 0) {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D[i] = cii;
    E[i] = beta;
    tau[i] = t;
    sc[i] = scale;
  }
  double yv = 0;
  if (wave < L + 2 * il && lane == 0) {
    const double sv = s1 + scale * sr;
    if (ycol >= 0) {
      y[wave] = sv;
      yv = sv * (ycol == i + 1 ? 1.0 : scale * cy);
    } else {
      u[wave - L] = sv;   // u1 at u[0:il], u2 at u[il:2il]
    }
  }
  const double bs = block_sum<MV / 64>(yv, red);
  if (threadIdx.x == 0) pm[blockIdx.x] = bs;
}

constexpr int FROWS = 64;   // rows per workgroup of k_fin (4 waves)
constexpr int PMU = 8;      // partial sums in flight per lane in k_fin

// Column i = p + il, rows r = i+1..n-1, FROWS per workgroup; wave g sums
// the panel terms q = g, g+4, ... < il for its workgroup's rows:
//   v(r) = scale c(r) (v(i+1) = 1), stored over c in A(:, i);
//   w(r) = tau (y(r) - V(r,:) u1 - W(r,:) u2) + alpha v(r), stored as
//          column il of W, with alpha = -tau/2 (w~ . v) and
//          w~ . v = tau (y . v - 2 u1 . u2);
//   next column (when the panel has one): c'(r) = A(r, i+1)
//          - sum_{q<=il} (V(r,q) W(i+1,q) + W(r,q) V(i+1,q)) in place, and
//          the workgroup's partial sum of c'(r)^2 over r >= i+3.
// The pivot row's w(i+1) is formed by every wave (and stored as such).
// Every load is issued before the first barrier.
__global__ __launch_bounds__(256) void k_fin(
    double* A, long long lda, int n, int p, int il, int nb_panel, double* W,
    long long ldw, const double* tau, const double* sc, const double* y,
    const double* u, const double* pm, int gm, double* part) {
  __shared__ double sw[4][64], scn[4][64];
  const int i = p + il, piv = i + 1;
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool next = il + 1 < nb_panel;
  const int r = piv + blockIdx.x * FROWS + lane;
  const int rc = r < n ? r : n - 1;
  double* cv = A + (long long)i * lda;
  double* cn = A + (long long)(next ? i + 1 : i) * lda;
  const double cvr = cv[rc], cnr = cn[rc], yr = y[rc - piv], y0 = y[0];
  const double t = tau[i], scale = sc[i];
  double pacc[PMU];
#pragma unroll
  for (int q = 0; q < PMU; ++q) pacc[q] = 0;
  int k = lane;
  for (; k + 64 * (PMU - 1) < gm; k += 64 * PMU) {
#pragma unroll
    for (int q = 0; q < PMU; ++q) pacc[q] += pm[k + 64 * q];
  }
  for (; k < gm; k += 64) pacc[0] += pm[k];
  const bool lq = lane < il;
  const int lqc = lq ? lane : 0;
  const double u1l = u[lqc], u2l = u[il + lqc];
  const double pvl = A[piv + (long long)(p + lqc) * lda];
  const double pwl = W[piv + (long long)lqc * ldw];
  double aw = 0, ac = 0;
#pragma unroll
  for (int sl = 0; sl < NB / 4; ++sl) {
    const int q = g + 4 * sl;
    const bool ok = q < il;
    const int qc = ok ? q : 0;
    const double vq = A[rc + (long long)(p + qc) * lda];
    const double wq = W[rc + (long long)qc * ldw];
    const double wpq = W[piv + (long long)qc * ldw];
    const double vpq = A[piv + (long long)(p + qc) * lda];
    const double u1 = ok ? u[qc] : 0.0, u2 = ok ? u[il + qc] : 0.0;
    const double m = ok ? 1.0 : 0.0;
    aw += vq * u1 + wq * u2;
    ac += m * (vq * wpq + wq * vpq);
  }
  double ps = 0;
#pragma unroll
  for (int q = 0; q < PMU; ++q) ps += pacc[q];
  const double yv = wave_sum_d(ps);
  const double uu = wave_sum_d(lq ? u1l * u2l : 0.0);
  const double alpha = -0.5 * t * (t * (yv - 2.0 * uu));
  const double wp = t * (y0 - wave_sum_d(lq ? pvl * u1l + pwl * u2l : 0.0)) + alpha;
  sw[g][lane] = aw;
  scn[g][lane] = ac;
  __syncthreads();
  double ssq = 0;
  if (g == 0 && r < n) {
    const double sumw = (sw[0][lane] + sw[1][lane]) + (sw[2][lane] + sw[3][lane]);
    const double vr = r == piv ? 1.0 : scale * cvr;
    const double wr = r == piv ? wp : t * (yr - sumw) + alpha * vr;
    cv[r] = vr;
    W[r + (long long)il * ldw] = wr;
    if (next) {
      const double sumc =
          (scn[0][lane] + scn[1][lane]) + (scn[2][lane] + scn[3][lane]);
      const double cr = cnr - sumc - (vr * wp + wr);   // q = il: V(piv, il) = 1
      cn[r] = cr;
      if (r >= i + 3) ssq = cr * cr;
    }
  }
  if (next && g == 0) {   // only wave 0 holds rows
    const double bs = wave_sum_d(ssq);
    if (lane == 0) part[blockIdx.x] = bs;
  }
}

// 1/d from the hardware reciprocal and two Newton steps (about 1 ulp; |d|
// is at least pivmin, a normal number)
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Sturm count of T - x I: the number of negative pivots of its LDL^T
// factorisation, pivots of magnitude below pivmin replaced by -pivmin (the
// safeguard of LAPACK's stebz).  The quotient uses a reciprocal of about
// 1 ulp, so the count is that of T with entries perturbed by a few ulps.
__device__ __forceinline__ int sturm_count(int n, const double* __restrict__ D,
                                           const double* __restrict__ E2,
                                           double x, double pivmin) {
  double d = D[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  int cnt = d < 0;
#pragma unroll 8
  for (int j = 1; j < n; ++j) {
    d = (D[j] - x) - E2[j - 1] * rcp_nr(d);
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0;
  }
  return cnt;
}

// E2 = E^2 and the Gershgorin bounds of T: gb = {min, max, max E^2}
__global__ void k_tri_prep(int n, const double* __restrict__ D,
                           const double* __restrict__ E, double* __restrict__ E2,
                           double* __restrict__ gb) {
  __shared__ double rl[4], ru[4], re[4];
  double gl = INFINITY, gu = -INFINITY, em = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double el = j > 0 ? fabs(E[j - 1]) : 0.0;
    const double er = j + 1 < n ? fabs(E[j]) : 0.0;
    gl = fmin(gl, D[j] - (el + er));
    gu = fmax(gu, D[j] + (el + er));
    if (j + 1 < n) {
      E2[j] = E[j] * E[j];
      em = fmax(em, E2[j]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o));
    gu = fmax(gu, __shfl_xor(gu, o));
    em = fmax(em, __shfl_xor(em, o));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rl[w] = gl;
    ru[w] = gu;
    re[w] = em;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      gl = fmin(gl, rl[k]);
      gu = fmax(gu, ru[k]);
      em = fmax(em, re[k]);
    }
    gl = fmin(gl, rl[0]);
    gu = fmax(gu, ru[0]);
    em = fmax(em, re[0]);
    gb[0] = gl;
    gb[1] = gu;
    gb[2] = em;
  }
}

// Eigenvalue k of T by multisection on the Sturm count, one wave per
// eigenvalue: each step the 64 lanes count at 64 interior points of the
// bracket [lo, hi) (count(lo) <= k < count(hi)) and the bracket shrinks 65
// fold, down to a width of 4 eps ||T||.
__global__ __launch_bounds__(256) void k_msect(int n, const double* __restrict__ D,
                                               const double* __restrict__ E2,
                                               const double* __restrict__ gb,
                                               double* __restrict__ w) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  const double eps = 2.220446049250313e-16;
  const double safmin = 2.2250738585072014e-308;
  const double pivmin = safmin * fmax(1.0, gb[2]);
  const double tnorm = fmax(fabs(gb[0]), fabs(gb[1]));
  const double atol = 4.0 * eps * tnorm;
  double lo = gb[0] - atol - pivmin, hi = gb[1] + atol + pivmin;
  for (int it = 0; it < 40 && hi - lo > atol; ++it) {
    const double x = lo + (hi - lo) * ((lane + 1) / 65.0);
    const int cnt = sturm_count(n, D, E2, x, pivmin);
    const unsigned long long above = __ballot(cnt > k);
    const double xprev = __shfl_up(x, 1);
    const int first = above ? __ffsll((long long)above) - 1 : 64;
    const double nlo = first == 0 ? lo : __shfl(first == 64 ? x : xprev, first == 64 ? 63 : first);
    const double nhi = first == 64 ? hi : __shfl(x, first);
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[k] = 0.5 * (lo + hi);
}

// B = A with leading dimension ldb >= n, rows n..ldb-1 zero
__global__ void k_pad_copy(const double* __restrict__ A, int n,
                           double* __restrict__ B, long long ldb) {
  const long long total = ldb * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % ldb, cidx = e / ldb;
    B[e] = r < n ? A[r + cidx * (long long)n] : 0.0;
  }
}

// Z1 = [V W], Z2 = [W V] over rows s0..n-1 (V = A(s0:n, p:p+b)), m = n-s0
__global__ void k_pack(const double* A, long long lda, const double* W,
                       long long ldw, int n, int p, int b, int s0, double* Z1,
                       double* Z2) {
  const int m = n - s0;
  const long long total = (long long)m * b;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), q = (int)(e / m);
    const double vv = A[(s0 + r) + (long long)(p + q) * lda];
    const double ww = W[(s0 + r) + q * ldw];
    Z1[r + (long long)q * m] = vv;
    Z1[r + (long long)(q + b) * m] = ww;
    Z2[r + (long long)q * m] = ww;
    Z2[r + (long long)(q + b) * m] = vv;
  }
}

// after the panel: A(i+1, i) = E(i); the last panel records D(n-1)
__global__ void k_restore(double* A, long long lda, int n, int p, int b,
                          const double* E, double* D) {
  const int q = threadIdx.x;
  if (q < b) A[(p + q + 1) + (long long)(p + q) * lda] = E[p + q];
  if (q == 0 && p + b == n - 1)
    D[n - 1] = A[(n - 1) + (long long)(n - 1) * lda];
}

__global__ void k_zero_u32(unsigned int* x) { *x = 0; }

constexpr int QB = 128;   // reflectors per block when Q is applied

// Vb (m x nb, leading dimension m) = the reflectors j0 .. j0+nb-1 as
// explicit columns over rows j0+1 .. n-1: zero above the unit element, 1 at
// row i+1, A(r, i) below it; a reflector with tau = 0 (the identity) is a
// zero column.
__global__ void k_build_v(const double* __restrict__ A, long long lda, int n,
                          int j0, int nb, const double* __restrict__ tau,
                          double* __restrict__ Vb) {
  const int m = n - 1 - j0;
  const long long total = (long long)m * nb;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), q = (int)(e / m);
    const int row = j0 + 1 + r, i = j0 + q;
    double v = 0.0;
    if (tau[i] != 0.0)
      v = row < i + 1 ? 0.0 : (row == i + 1 ? 1.0 : A[row + (long long)i * lda]);
    Vb[e] = v;
  }
}

// T^{-1} of the block's compact WY form H_j0 ... H_j0+nb-1 = I - V T V^T:
// diag(1 / tau) + the strict upper triangle of G = V^T V (Joffrain et al.,
// "Accumulating Householder transformations, revisited", the UT transform);
// an identity reflector (tau = 0, zero column) takes 1 on the diagonal.
__global__ void k_build_tinv(const double* __restrict__ G, int nb,
                             const double* __restrict__ tau, int j0,
                             double* __restrict__ Ti) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb * nb;
       e += gridDim.x * blockDim.x) {
    const int i = e % nb, j = e / nb;   // column-major (i, j)
    const double t = tau[j0 + i];
    Ti[e] = i < j ? G[e] : (i == j ? (t != 0.0 ? 1.0 / t : 1.0) : 0.0);
  }
}


#define OFM_BLAS_TD(call)                                                   \
  do {                                                                      \
    rocblas_status s_ = (call);                                             \
    if (s_ != rocblas_status_success)                                       \
      throw Error{OFM_E_DEVICE, std::string(#call) + " failed: " +          \
                                    rocblas_status_to_string(s_)};          \
  } while (0)

// Reduction of the n x n symmetric A (full storage, n >= 2, lda even and
// >= n rounded up to even, rows n..lda-1 zero) to tridiagonal form; D (n),
// E (n-1), tau (n-1) on the device.
void sytrd_lower(hipStream_t s, rocblas_handle h, int n, double* A,
                 long long lda, double* D, double* E, double* tau) {
  const long long ldw = lda;
  const int max_gm = (n + 2 * NB + MV / 64 - 1) / (MV / 64);
  const int max_part = (n + FROWS - 1) / FROWS + 1;
  DevBuf<double> W((size_t)ldw * NB), y(n), u(2 * NB), sc(n), pm(max_gm),
      part(max_part);
  DevBuf<double> Z1((size_t)n * 2 * NB), Z2((size_t)n * 2 * NB);
  OFM_HIP(hipMemsetAsync(W.p, 0, sizeof(double) * ldw * NB, s));
  const double one = 1.0, mone = -1.0;
  for (int p = 0; p < n - 1; p += NB) {
    const int b = std::min(NB, n - 1 - p);
    int np = (n - p - 1 + FR - 1) / FR;
    hipLaunchKernelGGL(k_pstart, dim3(np), dim3(FR), 0, s, A, lda, n, p,
                       part.p);
    OFM_HIP(hipGetLastError());
    for (int il = 0; il < b; ++il) {
      const int L = n - (p + il) - 1;
      const int gm = (L + 2 * il + MV / 64 - 1) / (MV / 64);
      const int gf = (L + FROWS - 1) / FROWS;
      hipLaunchKernelGGL(k_mv, dim3(gm), dim3(MV), 0, s, A, lda, n, p, il,
                         W.p, ldw, part.p, np, D, E, tau, sc.p, y.p, u.p,
                         pm.p);
      OFM_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_fin, dim3(gf), dim3(256), 0, s, A, lda, n, p, il,
                         b, W.p, ldw, tau, sc.p, y.p, u.p, pm.p, gm, part.p);
      OFM_HIP(hipGetLastError());
      np = gf;
    }
    const int s0 = p + b, m = n - s0;
    hipLaunchKernelGGL(k_pack, dim3(std::min(1024, (m * b + 255) / 256)),
                       dim3(256), 0, s, A, lda, W.p, ldw, n, p, b, s0, Z1.p,
                       Z2.p);
    OFM_HIP(hipGetLastError());
    // A22 -= [V W] [W V]^T, both triangles
    OFM_BLAS_TD(rocblas_dgemm(h, rocblas_operation_none,
                              rocblas_operation_transpose, m, m, 2 * b, &mone,
                              Z1.p, m, Z2.p, m, &one,
                              A + s0 + (long long)s0 * lda, (int)lda));
    hipLaunchKernelGGL(k_restore, dim3(1), dim3(64), 0, s, A, lda, n, p, b,
                       E, D);
    OFM_HIP(hipGetLastError());
  }
  // the scratch buffers are freed on return
  OFM_HIP(hipStreamSynchronize(s));
}

// Z = Q Z for the Q of sytrd_lower (n x n Z, leading dimension ldz), in
// blocks of QB reflectors from the last block to the first: per block,
// W = V^T Z(j0+1:n, :), W <- T W (a triangular solve with T^{-1}),
// Z(j0+1:n, :) -= V W, all as rocBLAS GEMM / TRSM.
void apply_q(hipStream_t s, rocblas_handle h, int n, const double* A,
             long long lda, const double* tau, double* Z, int ldz) {
  if (n < 2) return;
  DevBuf<double> Vb((size_t)n * QB), G((size_t)QB * QB), Ti((size_t)QB * QB),
      W((size_t)QB * n);
  const double one = 1.0, zero = 0.0, mone = -1.0;
  const int nref = n - 1;
  for (int j0 = (nref - 1) / QB * QB; j0 >= 0; j0 -= QB) {
    const int nb = std::min(QB, nref - j0);
    const int m = n - 1 - j0;
    hipLaunchKernelGGL(k_build_v, dim3(std::min(2048, (m * nb + 255) / 256)),
                       dim3(256), 0, s, A, lda, n, j0, nb, tau, Vb.p);
    OFM_HIP(hipGetLastError());
    OFM_BLAS_TD(rocblas_dgemm(h, rocblas_operation_transpose,
                              rocblas_operation_none, nb, nb, m, &one, Vb.p, m,
                              Vb.p, m, &zero, G.p, nb));
    hipLaunchKernelGGL(k_build_tinv, dim3((nb * nb + 255) / 256), dim3(256), 0,
                       s, G.p, nb, tau, j0, Ti.p);
    OFM_HIP(hipGetLastError());
    double* Zs = Z + (j0 + 1);
    OFM_BLAS_TD(rocblas_dgemm(h, rocblas_operation_transpose,
                              rocblas_operation_none, nb, n, m, &one, Vb.p, m,
                              Zs, ldz, &zero, W.p, nb));
    OFM_BLAS_TD(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_upper,
                              rocblas_operation_none,
                              rocblas_diagonal_non_unit, nb, n, &one, Ti.p, nb,
                              W.p, nb));
    OFM_BLAS_TD(rocblas_dgemm(h, rocblas_operation_none,
                              rocblas_operation_none, m, n, nb, &mone, Vb.p, m,
                              W.p, nb, &one, Zs, ldz));
  }
  OFM_HIP(hipStreamSynchronize(s));
}

}  // namespace

void dense_eigh(ofm_ctx* c, hipStream_t s, void* blas_handle, int n, double* A,
                double* w, double* Z, int* info) {
  OFM_REQUIRE(n >= 1, OFM_E_INVALID, "empty matrix");
  rocblas_handle h = static_cast<rocblas_handle>(blas_handle);
  if (n == 1) {
    OFM_HIP(hipMemcpyAsync(w, A, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (Z) {
      const double one = 1.0;
      OFM_HIP(hipMemcpyAsync(Z, &one, sizeof(double), hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<unsigned int*>(info));
    OFM_HIP(hipGetLastError());
    OFM_HIP(hipStreamSynchronize(s));
    return;
  }
  // padded copy: leading dimension a multiple of 64 doubles, pad rows zero
  const long long ldp = ((long long)n + 63) / 64 * 64;
  DevBuf<double> Ap((size_t)ldp * n), E(n), tau(n);
  hipLaunchKernelGGL(k_pad_copy, dim3(2048), dim3(256), 0, s, A, n, Ap.p, ldp);
  OFM_HIP(hipGetLastError());
  {
    // the reduction streams the trailing matrix once per column (k_mv):
    // sum over columns of 8 L (L + 2 il) bytes, L = n - i - 1
    double bytes = 0;
    for (int i = 0; i + 1 < n; ++i) {
      const double L = n - i - 1;
      bytes += 8.0 * L * (L + 2.0 * (i % NB));
    }
    Timed tm(c, "tridiag", bytes, bytes / 4.0);
    sytrd_lower(s, h, n, Ap.p, ldp, w, E.p, tau.p);
  }
  if (!Z) {
    DevBuf<double> D(n), E2(n), gb(3);
    OFM_HIP(hipMemcpyAsync(D.p, w, sizeof(double) * n, hipMemcpyDeviceToDevice,
                           s));
    hipLaunchKernelGGL(k_tri_prep, dim3(1), dim3(256), 0, s, n, D.p, E.p, E2.p,
                       gb.p);
    OFM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_msect, dim3((n + 3) / 4), dim3(256), 0, s, n, D.p,
                       E2.p, gb.p, w);
    OFM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<unsigned int*>(info));
    OFM_HIP(hipGetLastError());
    OFM_HIP(hipStreamSynchronize(s));
    return;
  }
  // eigenvectors of T, then Z = Q Z
  OFM_BLAS_TD(rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, w, E.p, Z, n,
                               info));
  apply_q(s, h, n, Ap.p, ldp, tau.p, Z, n);
}

}  // namespace ofm
