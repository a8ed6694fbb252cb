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
// triangles) with the leading dimension padded to 64 rows.  Each column
// takes two launches and no workgroup ever waits for another.  The first
// forms y = A22 v and the panel projections W^T v, V^T v, rebuilding the
// reflector from the previous launch's partial norms: for large trailing
// matrices k_mvt reads the lower triangle once in tiles (half the bytes)
// and leaves per-tile partial sums, for small ones k_mv streams whole
// columns, one dot product per wave.  k_fin, row-parallel, completes y,
// forms w (its correction -tau/2 (w.v) v from w.v = tau (y.v - 2 u1.u2)),
// stores v and w, and applies the panel's reflectors to the next column.
// After a panel of NB columns one GEMM applies A22 -= V W^T + W V^T to both
// triangles.
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
constexpr int MU = 4;     // 16-byte pairs per lane and round in col_dot

// One wave: s1 = x(i+1) and sr = sum_{r>=i+2} x(r) c(r) for the column x
// (rows i+1..n-1), read as 16-byte pairs from the even row rb = (i+1) & ~1
// (pair 0 holds row i+1; lane 0 forms its terms); wave-uniform sums.  The
// loads are unconditional (indices clamped, the excess selected away), MU
// pairs per lane and round, so that a column of up to 128 MU rows and the
// caller's earlier loads take one round trip to memory.
__device__ __forceinline__ void col_dot(const double* col, const double* c,
                                        int i, int n, int lane, double& s1,
                                        double& sr) {
  const int rb = (i + 1) & ~1;
  const int npair = (n - rb + 1) >> 1;   // >= 1
  const double2* a2 = reinterpret_cast<const double2*>(col + rb);
  const double2* c2 = reinterpret_cast<const double2*>(c + rb);
  const double2 a0 = a2[0], c0 = c2[0];
  double acc[MU];
#pragma unroll
  for (int q = 0; q < MU; ++q) acc[q] = 0;
  for (int k = 1 + lane; k < npair; k += 64 * MU) {
    double2 a[MU], cc[MU];
#pragma unroll
    for (int q = 0; q < MU; ++q) {
      const int kq = k + 64 * q;
      const int kc = kq < npair ? kq : npair - 1;
      a[q] = a2[kc];
      cc[q] = c2[kc];
    }
#pragma unroll
    for (int q = 0; q < MU; ++q) {
      const double t = a[q].x * cc[q].x + a[q].y * cc[q].y;
      acc[q] += k + 64 * q < npair ? t : 0.0;
    }
  }
  s1 = 0;
  sr = 0;
  if (lane == 0) {   // pair 0: rows rb, rb+1, one of them is i+1
    if (rb == i + 1) {
      s1 = a0.x;
      sr = a0.y * c0.y;
    } else {
      s1 = a0.y;
    }
  }
#pragma unroll
  for (int q = 0; q < MU; ++q) sr += acc[q];
  s1 = wave_sum_d(s1);
  sr = wave_sum_d(sr);
}

// The reflector of column i from alpha = c(i+1) and the squared norm xn2 of
// c(i+2:n): beta = -sign(alpha) sqrt(alpha^2 + xn2), tau = (beta - alpha) /
// beta, scale = 1 / (alpha - beta); the identity (tau = 0) when xn2 = 0.
__device__ __forceinline__ void reflector(double alpha, double xn2,
                                          double& beta, double& t,
                                          double& scale) {
  t = 0;
  beta = alpha;
  scale = 1;
  if (xn2 > 0) {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
}

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
  const double p0 = part[lane < np ? lane : np - 1];   // np >= 1
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
    col_dot(col, c, i, n, lane, s1, sr);
  }
  double ss = lane < np ? p0 : 0.0;
  for (int k = lane + 64; k < np; k += 64) ss += part[k];   // np > 64: rare
  double t, beta, scale;
  reflector(alpha, wave_sum_d(ss), beta, t, scale);
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

// Large trailing matrices: the product with A22 from its lower triangle
// alone, half the bytes of k_mv.
constexpr int TR = 256;      // rows per tile (two 16-byte pairs per lane)
constexpr int TC = 32;       // columns per tile (8 per wave)
constexpr int LTILE = 2048;  // trailing sizes from which k_mvt replaces k_mv

// Tiles of A22 = A(k0:n, k0:n), k0 = i+1: tile row rb covers rows
// rbase + rb TR .. (rbase = k0 & ~1, so that rows are read as aligned
// pairs), tile column cb columns k0 + cb TC ..; tile row rb holds the tiles
// that reach the diagonal or lie below it, cb < tile_cols(rb).
__host__ __device__ inline int tile_cols(int rb, int rbase, int k0, int ncb) {
  const int c = (rbase + (rb + 1) * TR - 1 - k0) / TC + 1;
  return c < ncb ? c : ncb;
}

// Column i = p + il, k0 = i+1, x(r) = c(r) for r >= i+2 (zero elsewhere).
// Workgroups 0..ntiles-1 each take one lower tile and form, from its
// elements A(r, k) with r >= k (each stored element read once):
//   P[rb][k - k0]       = sum_{r >= k, r in tile} A(r, k) x(r)   (8 columns
//                         per wave, all TR rows),
//   P[nrb + cb][r - k0] = sum_{k < r, k in tile} A(r, k) x(k)    (the
//                         symmetric half, summed over the 4 waves),
//   pq[tile]            = the tile's share of x^T A22 x;
// so (A22 x)(r) is the sum of the slots that exist for r (k_fin adds them
// up), and y = A22 v = A(:, k0) + scale A22 x since v = e_{k0} + scale x.
// Workgroups ntiles.. form u1 = W(i+1:n, 0:il)^T v and u2 =
// V(i+1:n, 0:il)^T v (one wave each) and build the reflector; the first of
// them stores D, E, tau, scale and A(i+1, i+1) (as y[0]).
// Storage as for k_mv; P holds nrb + ncb slots of leading dimension ldp >= L.
__global__ __launch_bounds__(256) void k_mvt(
    const double* A, long long lda, int n, int p, int il, const double* W,
    long long ldw, const double* part, int np, double* D, double* E,
    double* tau, double* sc, double* y, double* u, int ntiles, int nrb,
    int ncb, double* P, long long ldp, double* pq) {
  __shared__ double red[4][TR];
  __shared__ double qs[4];
  const int i = p + il, k0 = i + 1;
  const double* c = A + (long long)i * lda;   // indexed by row
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if ((int)blockIdx.x >= ntiles) {
    const int uw = ((int)blockIdx.x - ntiles) * 4 + w;
    const double p0 = part[lane < np ? lane : np - 1];   // np >= 1
    const double alpha = c[k0], cii = c[i];
    double s1 = 0, sr = 0;
    if (uw < 2 * il) {
      const double* col = uw < il ? W + (long long)uw * ldw
                                  : A + (long long)(p + uw - il) * lda;
      col_dot(col, c, i, n, lane, s1, sr);
    }
    double ss = lane < np ? p0 : 0.0;
    for (int k = lane + 64; k < np; k += 64) ss += part[k];   // np > 64
    double t, beta, scale;
    reflector(alpha, wave_sum_d(ss), beta, t, scale);
    if ((int)blockIdx.x == ntiles && threadIdx.x == 0) {
      D[i] = cii;
      E[i] = beta;
      tau[i] = t;
      sc[i] = scale;
      y[0] = A[k0 + (long long)k0 * lda];   // k_fin updates it in place
    }
    if (uw < 2 * il && lane == 0) u[uw] = s1 + scale * sr;
    return;
  }
  const int rbase = k0 & ~1;
  int tl = blockIdx.x, rb = 0;
  for (;; ++rb) {   // ends: blockIdx.x < the sum of tile_cols over rb < nrb
    const int cnt = tile_cols(rb, rbase, k0, ncb);
    if (tl < cnt) break;
    tl -= cnt;
  }
  const int cb = tl;
  constexpr int TRP = TR / 128;   // pairs per lane
  const int npair = (n + 1) >> 1;
  const double2* c2 = reinterpret_cast<const double2*>(c);
  int pr[TRP];
  double2 xr[TRP];
#pragma unroll
  for (int h = 0; h < TRP; ++h) {
    pr[h] = (rbase >> 1) + rb * (TR / 2) + lane + 64 * h;
    const int r0 = 2 * pr[h];
    double2 x = c2[pr[h] < npair ? pr[h] : npair - 1];
    x.x = (r0 < n && r0 >= k0 + 1) ? x.x : 0.0;
    x.y = (r0 + 1 < n && r0 + 1 >= k0 + 1) ? x.y : 0.0;
    xr[h] = x;
  }
  double2 rowp[TRP];
#pragma unroll
  for (int h = 0; h < TRP; ++h) rowp[h] = make_double2(0.0, 0.0);
  const int kb = k0 + cb * TC + w * 8;
  double2 a[8][TRP];
  double xk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kc = kb + j;
    const int kcc = kc < n ? kc : n - 1;
    const double2* a2 = reinterpret_cast<const double2*>(A + (long long)kcc * lda);
#pragma unroll
    for (int h = 0; h < TRP; ++h) a[j][h] = a2[pr[h] < npair ? pr[h] : npair - 1];
    xk[j] = (kc < n && kc >= k0 + 1) ? c[kcc] : 0.0;
  }
  double q = 0, mine = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kc = kb + j;
    double s = 0;
#pragma unroll
    for (int h = 0; h < TRP; ++h) {
      const int r0 = 2 * pr[h];
      const double ax = r0 >= kc ? a[j][h].x : 0.0;
      const double ay = r0 + 1 >= kc ? a[j][h].y : 0.0;
      s += ax * xr[h].x + ay * xr[h].y;
      rowp[h].x += (r0 > kc ? a[j][h].x : 0.0) * xk[j];
      rowp[h].y += (r0 + 1 > kc ? a[j][h].y : 0.0) * xk[j];
    }
    const double sj = wave_sum_d(s);
    q += sj * xk[j];
    if (lane == j) mine = sj;
  }
  if (lane < 8 && kb + lane < n) P[(long long)rb * ldp + (kb + lane - k0)] = mine;
#pragma unroll
  for (int h = 0; h < TRP; ++h) {
    red[w][2 * (lane + 64 * h)] = rowp[h].x;
    red[w][2 * (lane + 64 * h) + 1] = rowp[h].y;
  }
  __syncthreads();
  double qr = 0;
  for (int rr = threadIdx.x; rr < TR; rr += 256) {
    const double s = (red[0][rr] + red[1][rr]) + (red[2][rr] + red[3][rr]);
    const int r = rbase + rb * TR + rr;
    if (r >= k0 && r < n) {
      P[(long long)(nrb + cb) * ldp + (r - k0)] = s;
      qr += (r >= k0 + 1 ? c[r] : 0.0) * s;
    }
  }
  const double qrs = wave_sum_d(qr);
  if (lane == 0) qs[w] = qrs + q;
  __syncthreads();
  if (threadIdx.x == 0) pq[blockIdx.x] = (qs[0] + qs[1]) + (qs[2] + qs[3]);
}

// Tiles of the product at trailing size L = n - k0 (host side).
inline int tile_count(int n, int k0, int& nrb, int& ncb) {
  const int rbase = k0 & ~1;
  nrb = (n - rbase + TR - 1) / TR;
  ncb = (n - k0 + TC - 1) / TC;
  int t = 0;
  for (int rb = 0; rb < nrb; ++rb) t += tile_cols(rb, rbase, k0, ncb);
  return t;
}

constexpr int FROWS = 64;   // rows per workgroup of k_fin (one per lane)
constexpr int PMU = 4;      // partial sums per lane and round in k_fin
constexpr int SU = 24;      // slot loads per lane and round in k_fin (tiled)

// waves per workgroup of k_fin: 4 on k_mv's output; 8 on k_mvt's, whose
// slot sums add several times the loads (4 and 16 measured slower there)
__host__ __device__ constexpr int fin_waves(bool tiled) { return tiled ? 8 : 4; }

// Column i = p + il, rows r = i+1..n-1, FROWS per workgroup of FW waves;
// wave g sums the panel terms q = g, g+FW, ... < il for its workgroup's
// rows:
//   v(r) = scale c(r) (v(i+1) = 1), stored over c in A(:, i);
//   w(r) = tau (y(r) - V(r,:) u1 - W(r,:) u2) + alpha v(r), stored as
//          column il of W, with alpha = -tau/2 (w~ . v) and
//          w~ . v = tau (y . v - 2 u1 . u2);
//   next column (when the panel has one): c'(r) = A(r, i+1)
//          - sum_{q<=il} (V(r,q) W(i+1,q) + W(r,q) V(i+1,q)) in place, and
//          the workgroup's partial sum of c'(r)^2 over r >= i+3.
// y comes from k_mv (tiled = false: y complete, pm the shares of y . v) or
// from k_mvt (tiled: y(r) = A(r, i+1) + scale (A22 x)(r), wave g adding the
// slots g, g+FW, ... of P that exist for row r; pm the shares of
// x^T A22 x, and y . v = A(i+1, i+1) + 2 scale (A22 x)(i+1)
// + scale^2 x^T A22 x).
// The kernel is bound by the latency of its loads (at most n/64
// workgroups): the FW waves split every sum (the pm shares too) and issue
// all their loads (addresses clamped, so none is conditional) before the
// first wait; wave 0 combines the sums after the barrier and forms the
// pivot row's w(i+1) and the rows.
template <bool tiled, int FW = fin_waves(tiled)>
__global__ __launch_bounds__(64 * FW) void k_fin(
    double* A, long long lda, int n, int p, int il, int nb_panel, double* W,
    long long ldw, const double* tau, const double* sc, const double* y,
    const double* u, const double* pm, int gm, double* part, const double* P,
    long long ldp, int nrb, int ncb) {
  __shared__ double sw[FW][64], scn[FW][64], sy[tiled ? FW : 1][64], sp[2][FW];
  const int i = p + il, piv = i + 1;
  const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool next = il + 1 < nb_panel;
  const int r = piv + blockIdx.x * FROWS + lane;
  const int rc = r < n ? r : n - 1;
  double* cv = A + (long long)i * lda;
  double* cn = A + (long long)(next ? i + 1 : i) * lda;
  const double cvr = cv[rc], cnr = cn[rc];
  const double yr0 = tiled ? A[rc + (long long)piv * lda] : y[rc - piv];
  const double t = tau[i], scale = sc[i];
  const double y00 = y[0];   // A(i+1, i+1) when tiled (row piv of cn changes)
  const bool lq = lane < il;
  const int lqc = lq ? lane : 0;
  const double u1l = u[lqc], u2l = u[il + lqc];
  const double pvl = A[piv + (long long)(p + lqc) * lda];
  const double pwl = W[piv + (long long)lqc * ldw];
  // panel terms of this wave
  constexpr int QW = (NB + FW - 1) / FW;
  double vq[QW], wq[QW], wpq[QW], vpq[QW];
#pragma unroll
  for (int sl = 0; sl < QW; ++sl) {
    const int q = g + FW * sl;
    const int qc = q < il ? q : 0;
    vq[sl] = A[rc + (long long)(p + qc) * lda];
    wq[sl] = W[rc + (long long)qc * ldw];
    wpq[sl] = W[piv + (long long)qc * ldw];
    vpq[sl] = A[piv + (long long)(p + qc) * lda];
  }
  // this wave's share of the pm partial sums and (tiled) of the slots: the
  // first round of each is loaded before anything is summed, the rest (more
  // than 64 FW PMU shares or FW SU slots) in further rounds
  double vp[PMU];
#pragma unroll
  for (int q = 0; q < PMU; ++q) {
    const int k = g * 64 + lane + 64 * FW * q;
    const double x = pm[k < gm ? k : gm - 1];
    vp[q] = k < gm ? x : 0.0;
  }
  double ya = 0, y0a = 0;
  int rbase = 0, cbr = 0, nrow = 0;
  const int ns = nrb + ncb;
  auto slot = [&](int sq) {
    const bool ex = sq < ns && (sq < nrb ? cbr < tile_cols(sq, rbase, piv, ncb)
                                         : sq - nrb < nrow);
    const double x = P[(long long)(sq < ns ? sq : ns - 1) * ldp + (rc - piv)];
    return ex ? x : 0.0;
  };
  if constexpr (tiled) {
    rbase = piv & ~1;
    cbr = (rc - piv) / TC;
    nrow = tile_cols((rc - rbase) / TR, rbase, piv, ncb);
    double v[SU];
#pragma unroll
    for (int q = 0; q < SU; ++q) v[q] = slot(g + FW * q);
    // (A22 x)(i+1): the column slots alone (no element lies left of i+1)
    const int k = g * 64 + lane;
    const double x0 = P[(long long)(k < nrb ? k : nrb - 1) * ldp];
    y0a = k < nrb ? x0 : 0.0;
#pragma unroll
    for (int q = 0; q < SU; ++q) ya += v[q];
    for (int sl = g + FW * SU; sl < ns; sl += FW * SU) {
#pragma unroll
      for (int q = 0; q < SU; ++q) v[q] = slot(sl + FW * q);
#pragma unroll
      for (int q = 0; q < SU; ++q) ya += v[q];
    }
    for (int k1 = k + 64 * FW; k1 < nrb; k1 += 64 * FW) y0a += P[(long long)k1 * ldp];
  }
  double ps = 0;
#pragma unroll
  for (int q = 0; q < PMU; ++q) ps += vp[q];
  for (int k0 = g * 64 + lane + 64 * FW * PMU; k0 < gm; k0 += 64 * FW * PMU) {
#pragma unroll
    for (int q = 0; q < PMU; ++q) {
      const int k = k0 + 64 * FW * q;
      const double x = pm[k < gm ? k : gm - 1];
      vp[q] = k < gm ? x : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PMU; ++q) ps += vp[q];
  }
  double aw = 0, ac = 0;
#pragma unroll
  for (int sl = 0; sl < QW; ++sl) {
    const int q = g + FW * sl;
    const bool ok = q < il;
    const double u1 = ok ? u[q] : 0.0, u2 = ok ? u[il + q] : 0.0;
    const double m = ok ? 1.0 : 0.0;
    aw += vq[sl] * u1 + wq[sl] * u2;
    ac += m * (vq[sl] * wpq[sl] + wq[sl] * vpq[sl]);
  }
  sw[g][lane] = aw;
  scn[g][lane] = ac;
  if constexpr (tiled) sy[g][lane] = ya;
  const double psw = wave_sum_d(ps);
  const double y0w = tiled ? wave_sum_d(y0a) : 0.0;
  if (lane == 0) {
    sp[0][g] = psw;
    sp[1][g] = y0w;
  }
  __syncthreads();
  if (g != 0) return;   // wave 0 holds the rows
  double yv = 0, x0 = 0, sumw = 0, sumc = 0, sya = 0;
#pragma unroll
  for (int k = 0; k < FW; ++k) {
    yv += sp[0][k];
    x0 += sp[1][k];
    sumw += sw[k][lane];
    sumc += scn[k][lane];
    if constexpr (tiled) sya += sy[k][lane];
  }
  double y0 = y00;
  if constexpr (tiled) {
    yv = y00 + 2.0 * scale * x0 + scale * scale * yv;
    y0 = y00 + scale * x0;
  }
  const double uu = wave_sum_d(lq ? u1l * u2l : 0.0);
  const double alpha = -0.5 * t * (t * (yv - 2.0 * uu));
  const double wp = t * (y0 - wave_sum_d(lq ? pvl * u1l + pwl * u2l : 0.0)) + alpha;
  double ssq = 0;
  if (r < n) {
    const double yr = tiled ? yr0 + scale * sya : yr0;
    const double vr = r == piv ? 1.0 : scale * cvr;
    const double wr = r == piv ? wp : t * (yr - sumw) + alpha * vr;
    cv[r] = vr;
    W[r + (long long)il * ldw] = wr;
    if (next) {
      const double cr = cnr - sumc - (vr * wp + wr);   // q = il: V(piv, il) = 1
      cn[r] = cr;
      if (r >= i + 3) ssq = cr * cr;
    }
  }
  if (next) {
    const double bs = wave_sum_d(ssq);
    if (lane == 0) part[blockIdx.x] = bs;
  }
}

// Sturm count of T - x I: the number of negative pivots of its LDL^T
// factorisation, pivots of magnitude below pivmin replaced by -pivmin (the
// safeguard of LAPACK's stebz).  Every operation of the recurrence is
// correctly rounded (IEEE division, no contraction is possible), which makes
// the count a monotone function of x (Demmel, Dhillon and Ren, 1995): each
// wave brackets its own eigenvalue, and only a monotone count guarantees
// that the independently found eigenvalues come out ascending and none is
// counted twice or missed.  (A hardware reciprocal with one Newton step was
// ~2x faster per count but is not monotone in x.)
__device__ __forceinline__ int sturm_count(int n, const double* __restrict__ D,
                                           const double* __restrict__ E2,
                                           double x, double pivmin) {
  double d = D[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  int cnt = d < 0;
#pragma unroll 8
  for (int j = 1; j < n; ++j) {
    d = (D[j] - x) - E2[j - 1] / d;
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

// Starting bracket of the multisection: the Gershgorin interval of T
// widened by atol + pivmin (gb = {min, max, max E^2} from k_tri_prep).
__device__ __forceinline__ void msect_bracket(const double* __restrict__ gb,
                                              double& lo, double& hi,
                                              double& atol, double& pivmin) {
  const double eps = 2.220446049250313e-16;
  const double safmin = 2.2250738585072014e-308;
  pivmin = safmin * fmax(1.0, gb[2]);
  const double tnorm = fmax(fabs(gb[0]), fabs(gb[1]));
  atol = 4.0 * eps * tnorm;
  lo = gb[0] - atol - pivmin;
  hi = gb[1] + atol + pivmin;
}

constexpr int MG = 4096;   // points of the shared starting grid (64 x 64)

// Sturm counts at MG points spread evenly over the starting bracket, one
// per thread: every eigenvalue's multisection starts from the two grid
// points around it, which replaces its first two 65-fold steps.
__global__ __launch_bounds__(256) void k_msect_grid(
    int n, const double* __restrict__ D, const double* __restrict__ E2,
    const double* __restrict__ gb, double* __restrict__ gx,
    int* __restrict__ gc) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= MG) return;
  double lo, hi, atol, pivmin;
  msect_bracket(gb, lo, hi, atol, pivmin);
  const double x = lo + (hi - lo) * ((g + 1) / (MG + 1.0));
  gx[g] = x;
  gc[g] = sturm_count(n, D, E2, x, pivmin);
}

// Eigenvalue k of T by multisection on the Sturm count, one wave per
// eigenvalue: each step the 64 lanes count at 64 interior points of the
// bracket [lo, hi) (count(lo) <= k < count(hi)) and the bracket shrinks 65
// fold, down to a width of 4 eps ||T||.  The first bracket comes from the
// grid of k_msect_grid: with m grid points of count <= k (the counts grow
// along the grid), [x_{m-1}, x_m); it is taken only where the stored counts
// confirm count(lo) <= k < count(hi), else the whole starting bracket.
__global__ __launch_bounds__(256) void k_msect(int n, const double* __restrict__ D,
                                               const double* __restrict__ E2,
                                               const double* __restrict__ gb,
                                               const double* __restrict__ gx,
                                               const int* __restrict__ gc,
                                               double* __restrict__ w) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  double lo, hi, atol, pivmin;
  msect_bracket(gb, lo, hi, atol, pivmin);
  {
    // last point of each 64-point block, then the block holding the step
    const int B = __popcll(__ballot(gc[64 * lane + 63] <= k));
    int m = 64 * B;
    if (B < 64) m += __popcll(__ballot(gc[64 * B + lane] <= k));
    const bool okl = m == 0 || gc[m - 1] <= k;
    const bool okh = m == MG || gc[m] > k;
    if (okl && okh) {
      if (m > 0) lo = gx[m - 1];
      if (m < MG) hi = gx[m];
    }
  }
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
    std::shared_lock<std::shared_mutex> lk_(ofm::capture_lock());           \
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
  // tiled product (k_mvt) for the columns with L >= LTILE: partial-sum slots
  // of leading dimension n and one x^T A22 x share per tile
  int max_tiles = 0, max_slots = 0;
  for (int k0 = 1; n - k0 >= LTILE; ++k0) {
    int nrb, ncb;
    max_tiles = std::max(max_tiles, tile_count(n, k0, nrb, ncb));
    max_slots = std::max(max_slots, nrb + ncb);
  }
  const long long ldP = n;
  DevBuf<double> W((size_t)ldw * NB), y(n), u(2 * NB), sc(n),
      pm(std::max(max_gm, max_tiles)), part(max_part),
      P((size_t)ldP * std::max(max_slots, 1));
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
      const int gf = (L + FROWS - 1) / FROWS;
      int gm, nrb = 0, ncb = 0;
      if (L >= LTILE) {
        gm = tile_count(n, p + il + 1, nrb, ncb);
        const int gu = std::max(1, (2 * il + 3) / 4);
        hipLaunchKernelGGL(k_mvt, dim3(gm + gu), dim3(256), 0, s, A, lda, n,
                           p, il, W.p, ldw, part.p, np, D, E, tau, sc.p, y.p,
                           u.p, gm, nrb, ncb, P.p, ldP, pm.p);
      } else {
        gm = (L + 2 * il + MV / 64 - 1) / (MV / 64);
        hipLaunchKernelGGL(k_mv, dim3(gm), dim3(MV), 0, s, A, lda, n, p, il,
                           W.p, ldw, part.p, np, D, E, tau, sc.p, y.p, u.p,
                           pm.p);
      }
      OFM_HIP(hipGetLastError());
      hipLaunchKernelGGL(nrb > 0 ? k_fin<true> : k_fin<false>, dim3(gf),
                         dim3(64 * fin_waves(nrb > 0)), 0, s, A, lda, n, p, il, b, W.p, ldw, tau,
                         sc.p, y.p, u.p, pm.p, gm, part.p, P.p, ldP, nrb, ncb);
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
    // the reduction streams the trailing matrix once per column, its lower
    // triangle (k_mvt, L >= LTILE) or both triangles (k_mv), and the panel's
    // 2 il columns: 8 (L (L + 1) / 2 + 2 il L) or 8 L (L + 2 il) bytes,
    // L = n - i - 1
    double bytes = 0;
    for (int i = 0; i + 1 < n; ++i) {
      const double L = n - i - 1;
      const double il = i % NB;
      bytes += L >= LTILE ? 8.0 * (L * (L + 1) / 2 + 2.0 * il * L)
                          : 8.0 * L * (L + 2.0 * il);
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
    DevBuf<double> gx(MG);
    DevBuf<int> gc(MG);
    hipLaunchKernelGGL(k_msect_grid, dim3(MG / 256), dim3(256), 0, s, n, D.p,
                       E2.p, gb.p, gx.p, gc.p);
    OFM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_msect, dim3((n + 3) / 4), dim3(256), 0, s, n, D.p,
                       E2.p, gb.p, gx.p, gc.p, w);
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
