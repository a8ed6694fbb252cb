// HIP kernels of the OFM hot path for gfx950 (MI355X, CDNA4); the fragment
// Hamiltonian stencil k_apply_h lives in stencil.hip.
//
//  * k_gram         G = A^T B per fragment over its box points, FP64 MFMA
//                   (16x16x4) with split-K partials summed in fixed order.
//  * k_cholinv      Cholesky of a Gram matrix and the inverse of its factor
//                   (CholQR), one workgroup per fragment, FP64 in LDS.
//  * k_rr_eig       cyclic two-sided Jacobi on the projected matrix (Rayleigh-
//                   Ritz), one workgroup per fragment, FP64 in LDS.
//  * k_rotate       X <- X Q (and HX <- HX Q with fused residual norms).
//  * k_whole_h      H|phi> with the whole-system H on the dilated box.
//  * k_pair         grouped pair contraction: H_jn and S_jn of a pair over
//                   the box overlaps, FP64 MFMA, one workgroup per pair
//                   (k_pair_x3: split-BF16 x3 MFMA, mixed form).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "kdev.h"
#include "ofm_internal.h"

namespace ofm {
namespace k {

// ---------------------------------------------------------------------------
// potential restricted to every box
// ---------------------------------------------------------------------------
__global__ void k_restrict(const FragDev* __restrict__ F, int nf,
                           const double* __restrict__ V, int nx, int ny,
                           double* __restrict__ out, float* __restrict__ out32) {
  const int j = blockIdx.y;
  if (j >= nf) return;
  const FragDev f = F[j];
  for (int p = blockIdx.x * WG + threadIdx.x; p < f.npts;
       p += gridDim.x * WG) {
    const int x = p % f.dims[0];
    const int y = (p / f.dims[0]) % f.dims[1];
    const int z = p / (f.dims[0] * f.dims[1]);
    const long long g = (long long)(f.lo[0] + x) +
                        (long long)nx * ((f.lo[1] + y) + (long long)ny *
                                                             (f.lo[2] + z));
    const double v = V[g];
    out[f.v_off + p] = v;
    out32[f.v_off + p] = (float)v;
  }
}

void restrict_potential(hipStream_t s, const double* V, const ofm_grid& g,
                        const ofm_frags* f) {
  int maxp = 0;
  for (auto& d : f->host) maxp = std::max(maxp, d.npts);
  dim3 grid((maxp + WG - 1) / WG, f->n_frag);
  hipLaunchKernelGGL(k_restrict, grid, dim3(WG), 0, s, f->d_frag, f->n_frag,
                     V, g.nx, g.ny, f->d_v, f->d_v32);
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// own-atoms fragment potential: wells of the fragment's atoms on its box
// ---------------------------------------------------------------------------
__global__ void k_wells(const FragDev* __restrict__ F, int nf,
                        const double* __restrict__ xyz,
                        const double* __restrict__ Z,
                        const long long* __restrict__ ptr,
                        const int* __restrict__ idx, double ox, double oy,
                        double oz, double h, double inv2s2, double rc2,
                        double* __restrict__ out, float* __restrict__ out32) {
  const int j = blockIdx.y;
  if (j >= nf) return;
  const FragDev f = F[j];
  const long long a0 = ptr[j], a1 = ptr[j + 1];
  for (int p = blockIdx.x * WG + threadIdx.x; p < f.npts;
       p += gridDim.x * WG) {
    const int x = p % f.dims[0];
    const int y = (p / f.dims[0]) % f.dims[1];
    const int z = p / (f.dims[0] * f.dims[1]);
    const double rx = ox + (f.lo[0] + x) * h, ry = oy + (f.lo[1] + y) * h,
                 rz = oz + (f.lo[2] + z) * h;
    double v = 0;
    for (long long a = a0; a < a1; ++a) {
      const int at = idx[a];
      const double dx = rx - xyz[3 * at], dy = ry - xyz[3 * at + 1],
                   dz = rz - xyz[3 * at + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2) v -= Z[at] * exp(-r2 * inv2s2);
    }
    out[f.v_off + p] = v;
    out32[f.v_off + p] = (float)v;
  }
}

void fragment_wells(hipStream_t s, const ofm_frags* f, const double* xyz,
                    const double* Z, const long long* ptr, const int* idx,
                    double sigma, double r_cut) {
  int maxp = 0;
  for (auto& d : f->host) maxp = std::max(maxp, d.npts);
  dim3 grid((maxp + WG - 1) / WG, f->n_frag);
  hipLaunchKernelGGL(k_wells, grid, dim3(WG), 0, s, f->d_frag, f->n_frag, xyz,
                     Z, ptr, idx, f->grid.origin[0], f->grid.origin[1],
                     f->grid.origin[2], f->grid.h, 1.0 / (2.0 * sigma * sigma),
                     r_cut * r_cut, f->d_vf, f->d_vf32);
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// seeded start vectors: splitmix64 of (seed, fragment, vector, point)
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_init_random(const FragDev* __restrict__ F,
                              const int2* __restrict__ rt, int nrt,
                              T* __restrict__ X, unsigned long long seed) {
  const int t = blockIdx.x;
  if (t >= nrt) return;
  const int j = rt[t].x;
  const FragDev f = F[j];
  const int p = rt[t].y * RCH + threadIdx.x;
  if (p >= f.npts) return;
  for (int v = 0; v < f.bw; ++v) {
    unsigned long long key = seed * 0x100000001B3ULL ^
                             ((unsigned long long)j << 40) ^
                             ((unsigned long long)v << 26) ^
                             (unsigned long long)p;
    const unsigned long long r = splitmix64(key);
    const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
    X[f.x_off + (long long)v * f.ld + p] = (T)(2.0 * u - 1.0);
  }
}

template <typename T>
void init_random(hipStream_t s, const ofm_frags* f, T* X,
                 unsigned long long seed) {
  hipLaunchKernelGGL(k_init_random<T>, dim3(f->n_rtiles), dim3(RCH), 0, s,
                     f->d_frag, f->d_rtiles, f->n_rtiles, X, seed);
  OFM_HIP(hipGetLastError());
}
template void init_random<double>(hipStream_t, const ofm_frags*, double*,
                                  unsigned long long);
template void init_random<float>(hipStream_t, const ofm_frags*, float*,
                                 unsigned long long);


// ---------------------------------------------------------------------------
// Gram products G = A^T B per fragment (FP64 MFMA 16x16x4)
// ---------------------------------------------------------------------------
// MFMA operand placement: lane l = r + 16 g supplies A[r][g] and B[g][r]; the
// K index is free to permute, so lane (r, g) feeds four consecutive points
// of vector r from one 32-byte load.  Accumulator: item i of lane l holds
// row l/16 + 4 i, column l % 16.
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ void load4(const T* p, double* o) {
  if constexpr (sizeof(T) == 8) {
    const d4 v = *reinterpret_cast<const d4*>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = *reinterpret_cast<const f4*>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
}

// One workgroup per (fragment, contraction chunk).  Every wave computes all
// 16x16 tiles of the block (NT x NT tiles, the upper ones only when A == B)
// over its own interleaved share of the chunk, so each row segment is
// loaded once; the four waves' tiles are then summed in LDS in wave order.
template <typename T, int NT, bool SYM>
__global__ __launch_bounds__(WG) void k_gram(
    const FragDev* __restrict__ F, const int* __restrict__ flist, int nf,
    const T* __restrict__ A, const T* __restrict__ B,
    double* __restrict__ partial, const int* __restrict__ active) {
  constexpr int NTILE = SYM ? NT * (NT + 1) / 2 : NT * NT;
  const int fi = blockIdx.x / GCH, ch = blockIdx.x % GCH;
  if (fi >= nf) return;
  const int j = flist[fi];   // a fragment of this launch's width class
  if (active && !active[j]) return;
  const FragDev& fr = F[j];
  const int bw = fr.bw;
  int cs = (fr.ld + GCH - 1) / GCH;
  cs = (cs + 31) / 32 * 32;
  const int kb = ch * cs;
  const int ke = min(kb + cs, fr.ld);
  double* out = partial + (long long)fr.small_off * GCH + (long long)ch * bw * bw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const T* pa[NT];
  const T* pb[NT];
  bool va[NT], vb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int row = t * 16 + r;
    va[t] = row < bw;
    pa[t] = A + fr.x_off + (long long)(va[t] ? row : 0) * fr.ld;
    vb[t] = va[t];
    pb[t] = B + fr.x_off + (long long)(vb[t] ? row : 0) * fr.ld;
  }
  d4 acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) acc[t] = d4{0, 0, 0, 0};
  // kb and ke are multiples of 16: every lane of a wave runs the same trip
  // count (an MFMA reads all lanes' operands)
  for (int k = kb + 16 * wave + 4 * g; k < ke; k += 64) {
    double a[NT][4], b[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      a[t][0] = a[t][1] = a[t][2] = a[t][3] = 0;
      if (va[t]) load4(pa[t] + k, a[t]);
      if constexpr (!SYM) {
        b[t][0] = b[t][1] = b[t][2] = b[t][3] = 0;
        if (vb[t]) load4(pb[t] + k, b[t]);
      }
    }
    int tile = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
      for (int tj = SYM ? ti : 0; tj < NT; ++tj, ++tile)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[tile] = mfma_f64(a[ti][u], SYM ? a[tj][u] : b[tj][u], acc[tile]);
  }
  // sum the waves' tiles in wave order
  __shared__ double red[NTILE * 4 * 64];
  for (int w = 1; w < WG / 64; ++w) {
    if (wave == w)
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[(t * 4 + i) * 64 + lane] = acc[t][i];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[t][i] += red[(t * 4 + i) * 64 + lane];
    __syncthreads();
  }
  if (wave != 0) return;
  int tile = 0;
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = SYM ? ti : 0; tj < NT; ++tj, ++tile)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = ti * 16 + g + 4 * i, col = tj * 16 + r;
        if (row < bw && col < bw) out[row * bw + col] = acc[tile][i];
      }
}

template <typename T>
void gram(ofm_ctx* c, const ofm_frags* f, const T* A, const T* B, double* G,
          const int* active, double bytes, double flops) {
  int nl = 0;
  for (int cl = 0; cl < 4; ++cl) nl += f->n_gfl[cl] > 0;
  Timed tm(c, "gram", bytes, flops, nl);
  const bool sym = A == B;
  // one launch per width class (16-state tiles per block side)
#define GRAM(NT)                                                             \
  if (sym)                                                                   \
    hipLaunchKernelGGL((k_gram<T, NT, true>), dim3(n * GCH), dim3(WG), 0,    \
                       c->stream, f->d_frag, fl, n, A, B, G, active);        \
  else                                                                       \
    hipLaunchKernelGGL((k_gram<T, NT, false>), dim3(n * GCH), dim3(WG), 0,   \
                       c->stream, f->d_frag, fl, n, A, B, G, active)
  for (int cl = 0; cl < 4; ++cl) {
    const int n = f->n_gfl[cl];
    const int* fl = f->d_gfl[cl];
    if (n == 0) continue;
    if (cl == 0) GRAM(1);
    else if (cl == 1) GRAM(2);
    else if (cl == 2) GRAM(3);
    else GRAM(4);
  }
#undef GRAM
  OFM_HIP(hipGetLastError());
}
template void gram<double>(ofm_ctx*, const ofm_frags*, const double*,
                           const double*, double*, const int*, double, double);
template void gram<float>(ofm_ctx*, const ofm_frags*, const float*,
                          const float*, double*, const int*, double, double);

// ---------------------------------------------------------------------------
// mixed forms: 3-term split products on MFMA (16x16x32) with FP32
// accumulation, a b ~ a_hi b_hi + (a_hi b_lo + a_lo b_hi) s:
//  * BF16 x3: a_hi = bf16(a), a_lo = bf16(a - a_hi), s = 1; the dropped
//    a_lo b_lo term is ~2^-16 |a b|;
//  * FP16 x3: a_hi = f16(a), a_lo = f16((a - a_hi) 2^11), s = 2^-11 (the
//    scaled low part stays in FP16's normal range wherever a_hi does, and
//    below it a_lo carries what the subnormal a_hi loses); the dropped term
//    is ~2^-22 |a b|.  Box vectors are unit-norm states or H times them, so
//    every operand lies far inside FP16's range (|a| <= ~40).
// a_hi b_hi and the two cross products go to separate FP32 accumulators,
// which are added into FP64 sums (cross scaled by s) every few hundred
// points: the FP32 error stays that of a short sum, the long sums are
// FP64.  The separate cross accumulator matters in the BF16 form too: with
// the cross products added into the a_hi b_hi accumulator over four
// products, the element error measured 8.5e-5 of max|H| on the tiny chain
// against 5.6e-7 (the small cross terms lose their low bits when an MFMA
// adds them to a large accumulator).
// Operand placement as for the FP64 kernels, 8 consecutive points per lane;
// accumulator item i of lane l holds row 4 (l/16) + i, column l % 16.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

template <int MODE>   // 0: split-BF16 x3, 1: scaled split-FP16 x3
struct Split3;

template <>
struct Split3<0> {
  typedef bf8v V;
  static constexpr double kCross = 1.0;
  static __device__ __forceinline__ void split(const float* v, V& hi, V& lo) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const __bf16 h = (__bf16)v[t];
      hi[t] = h;
      lo[t] = (__bf16)(v[t] - (float)h);
    }
  }
  static __device__ __forceinline__ f4v mma(const V& a, const V& b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Split3<1> {
  typedef h8v V;
  static constexpr double kCross = 1.0 / 2048.0;
  static __device__ __forceinline__ void split(const float* v, V& hi, V& lo) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const _Float16 h = (_Float16)v[t];
      hi[t] = h;
      lo[t] = (_Float16)((v[t] - (float)h) * 2048.0f);
    }
  }
  static __device__ __forceinline__ f4v mma(const V& a, const V& b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// acc_hh += a_hi b_hi, acc_x += a_hi b_lo + a_lo b_hi
template <int MODE>
__device__ __forceinline__ void mma3(const typename Split3<MODE>::V& ah,
                                     const typename Split3<MODE>::V& al,
                                     const typename Split3<MODE>::V& bh,
                                     const typename Split3<MODE>::V& bl,
                                     f4v& hh, f4v& x) {
  hh = Split3<MODE>::mma(ah, bh, hh);
  x = Split3<MODE>::mma(ah, bl, x);
  x = Split3<MODE>::mma(al, bh, x);
}

__device__ __forceinline__ void load8(const float* p, float* o) {
  const f4v u = *reinterpret_cast<const f4v*>(p);
  const f4v w = *reinterpret_cast<const f4v*>(p + 4);
  o[0] = u[0]; o[1] = u[1]; o[2] = u[2]; o[3] = u[3];
  o[4] = w[0]; o[5] = w[1]; o[6] = w[2]; o[7] = w[3];
}

// points per FP64 flush of the Gram kernel's FP32 sums (per wave and tile)
constexpr int GRAM_FLUSH_PTS = 256;

template <int MODE>
__global__ __launch_bounds__(WG) void k_gram_x3(
    const FragDev* __restrict__ F, int nf, const float* __restrict__ A,
    const float* __restrict__ B, double* __restrict__ partial,
    const int* __restrict__ active) {
  using SP = Split3<MODE>;
  const int j = blockIdx.x / GCH, ch = blockIdx.x % GCH;
  if (j >= nf) return;
  if (active && !active[j]) return;
  const FragDev& fr = F[j];
  const int bw = fr.bw;
  const int nt = (bw + 15) / 16;
  int cs = (fr.ld + GCH - 1) / GCH;
  cs = (cs + 31) / 32 * 32;
  const int kb = ch * cs;
  const int ke = min(kb + cs, fr.ld);
  double* out = partial + (long long)fr.small_off * GCH + (long long)ch * bw * bw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  int tile = 0;
  for (int ti = 0; ti < nt; ++ti) {
    for (int tj = 0; tj < nt; ++tj, ++tile) {
      if ((tile & 3) != wave) continue;
      const int ra = ti * 16 + r, rb = tj * 16 + r;
      const bool va = ra < bw, vb = rb < bw;
      const float* pa = A + fr.x_off + (long long)(va ? ra : 0) * fr.ld;
      const float* pb = B + fr.x_off + (long long)(vb ? rb : 0) * fr.ld;
      f4v hh = {0, 0, 0, 0}, x = {0, 0, 0, 0};
      double tot[4] = {0, 0, 0, 0};
      int since = 0;
      // kb and ke are multiples of 32: uniform trip count across the wave
      for (int k = kb + 8 * g; k < ke; k += 32) {
        float a[8] = {0, 0, 0, 0, 0, 0, 0, 0}, b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (va) load8(pa + k, a);
        if (vb) load8(pb + k, b);
        typename SP::V ah, al, bh, bl;
        SP::split(a, ah, al);
        SP::split(b, bh, bl);
        mma3<MODE>(ah, al, bh, bl, hh, x);
        if (++since == GRAM_FLUSH_PTS / 32) {
          since = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) tot[i] += (double)hh[i] + SP::kCross * (double)x[i];
          hh = x = f4v{0, 0, 0, 0};
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        tot[i] += (double)hh[i] + SP::kCross * (double)x[i];
        const int row = ti * 16 + 4 * g + i, col = tj * 16 + r;
        if (row < bw && col < bw) out[row * bw + col] = tot[i];
      }
    }
  }
}

void gram_x3(ofm_ctx* c, const ofm_frags* f, const float* A, const float* B,
             double* G, const int* active, double bytes, double flops) {
  Timed tm(c, "gram", bytes, flops);
  if (c->precision == OFM_MIXED_FP16X3)
    hipLaunchKernelGGL(k_gram_x3<1>, dim3(f->n_frag * GCH), dim3(WG), 0,
                       c->stream, f->d_frag, f->n_frag, A, B, G, active);
  else
    hipLaunchKernelGGL(k_gram_x3<0>, dim3(f->n_frag * GCH), dim3(WG), 0,
                       c->stream, f->d_frag, f->n_frag, A, B, G, active);
  OFM_HIP(hipGetLastError());
}

// sum the split-K partials of fragment fr into a symmetric LDS matrix
__device__ void load_sym(const FragDev& fr, const double* __restrict__ partial,
                         double* M, int ldm, int symmetric) {
  const int bw = fr.bw;
  const double* base = partial + (long long)fr.small_off * GCH;
  for (int e = threadIdx.x; e < bw * bw; e += blockDim.x) {
    const int i = e / bw, jj = e % bw;
    if (symmetric && jj < i) continue;
    double s = 0;
    for (int ch = 0; ch < GCH; ++ch) s += base[(long long)ch * bw * bw + e];
    M[i * ldm + jj] = s;
    if (symmetric) M[jj * ldm + i] = s;
  }
  __syncthreads();
  if (!symmetric) {   // symmetrise (A + A^T)/2
    for (int e = threadIdx.x; e < bw * bw; e += blockDim.x) {
      const int i = e / bw, jj = e % bw;
      if (jj <= i) continue;
      const double m = 0.5 * (M[i * ldm + jj] + M[jj * ldm + i]);
      M[i * ldm + jj] = m;
      M[jj * ldm + i] = m;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// CholQR factor: G = R^T R (after unit-diagonal scaling), Q = R^-1
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(WG) void k_cholinv(
    const FragDev* __restrict__ F, int nf, const double* __restrict__ partial,
    double* __restrict__ Q, const int* __restrict__ active,
    int* __restrict__ flags, int ld) {
  const int j = blockIdx.x;
  if (j >= nf) return;
  if (active && !active[j]) return;
  const FragDev& fr = F[j];
  const int bw = fr.bw;
  // two n x n matrices of row pitch ld = (largest block width) + 1, sized at
  // launch
  extern __shared__ double ch_lds[];
  double* M = ch_lds;
  double* R = M + (ld - 1) * ld;
  __shared__ double dsc[SMAX];
  __shared__ int fail;
  load_sym(fr, partial, M, ld, 1);
  // unit-diagonal scaling (column norms of X)
  for (int i = threadIdx.x; i < bw; i += WG) {
    const double d = M[i * ld + i];
    dsc[i] = d > 0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < bw * bw; e += WG) {
    const int i = e / bw, jj = e % bw;
    R[i * ld + jj] = M[i * ld + jj] * dsc[i] * dsc[jj];
  }
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 1) {
      // shifted Cholesky: G + 1e-12 * bw * I (scaled matrix has unit diagonal)
      for (int e = threadIdx.x; e < bw * bw; e += WG) {
        const int i = e / bw, jj = e % bw;
        R[i * ld + jj] = M[i * ld + jj] * dsc[i] * dsc[jj] +
                          (i == jj ? 1e-12 * bw : 0.0);
      }
      if (threadIdx.x == 0) fail = 0;
      __syncthreads();
    }
    for (int k = 0; k < bw; ++k) {
      if (threadIdx.x == 0) {
        const double d = R[k * ld + k];
        if (!(d > 1e-300)) fail = 1;
        R[k * ld + k] = sqrt(d > 1e-300 ? d : 1e-300);
      }
      __syncthreads();
      const double piv = R[k * ld + k];
      for (int jj = k + 1 + threadIdx.x; jj < bw; jj += WG)
        R[k * ld + jj] /= piv;
      __syncthreads();
      const int m = bw - k - 1;
      for (int e = threadIdx.x; e < m * m; e += WG) {
        const int a = k + 1 + e / m, b = k + 1 + e % m;
        if (b >= a) R[a * ld + b] -= R[k * ld + a] * R[k * ld + b];
      }
      __syncthreads();
    }
    // every thread takes the outcome into a register, and all of them have
    // taken it before thread 0 may reset `fail` for the shifted attempt
    const int failed = fail;
    __syncthreads();
    if (!failed) break;
    // bit 0: the shifted factorisation was needed; bit 1: it lost a pivot
    // as well (the block is numerically rank deficient)
    if (threadIdx.x == 0 && flags) atomicOr(&flags[j], attempt == 0 ? 1 : 2);
  }
  // inverse of the upper-triangular factor, one column per thread
  double* Qj = Q + fr.small_off;
  for (int col = threadIdx.x; col < bw; col += WG) {
    // back substitution for column col of R^-1: entries row <= col
    double x[SMAX];
    for (int row = col; row >= 0; --row) {
      double s = (row == col) ? 1.0 : 0.0;
      for (int kk = row + 1; kk <= col; ++kk) s -= R[row * ld + kk] * x[kk];
      x[row] = s / R[row * ld + row];
    }
    for (int row = 0; row < bw; ++row)
      Qj[row * bw + col] = row <= col ? x[row] * dsc[row] : 0.0;
  }
}

void cholinv(hipStream_t s, const ofm_frags* f, const double* G, double* Q,
             const int* active, int* flags) {
  const int ld = f->max_bw + 1;
  hipLaunchKernelGGL(k_cholinv, dim3(f->n_frag), dim3(WG),
                     2 * (size_t)f->max_bw * ld * sizeof(double), s,
                     f->d_frag, f->n_frag, G, Q, active, flags, ld);
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz: cyclic two-sided Jacobi on the symmetric projected matrix
// ---------------------------------------------------------------------------
// With `pre`, Q holds on entry the inverse R^-1 of the last Cholesky factor
// of X^T X (the second CholQR pass, not applied to X): the projected matrix
// becomes R^-T (X^T H X) R^-1 and the rotation returned is R^-1 Y, so the
// second orthonormalisation and the Rayleigh-Ritz rotation cost one pass.
constexpr int RRW = WG;   // threads per fragment
__global__ __launch_bounds__(RRW) void k_rr_eig(
    const FragDev* __restrict__ F, int nf, const double* __restrict__ partial,
    double* __restrict__ Q, double* __restrict__ theta,
    const int* __restrict__ active, int pre, int ld) {
  const int j = blockIdx.x;
  if (j >= nf) return;
  if (active && !active[j]) return;
  const FragDev& fr = F[j];
  const int n = fr.bw;
  // three n x n matrices of row pitch ld = (largest block width) + 1, sized
  // at launch so that a 40-wide block does not reserve room for 64 (four
  // fragments per CU instead of one)
  extern __shared__ double rr_lds[];
  const int nmax = ld - 1;
  double* A = rr_lds;
  double* U = A + nmax * ld;
  double* Pm = U + nmax * ld;
  __shared__ double cs[SMAX / 2], sn[SMAX / 2];
  __shared__ int pp[SMAX / 2], qq[SMAX / 2];
  __shared__ double red[RRW / 64];
  __shared__ double offn, totn;
  load_sym(fr, partial, A, ld, 0);
  if (pre) {
    const double* Qj0 = Q + fr.small_off;
    for (int e = threadIdx.x; e < n * n; e += RRW)
      Pm[(e / n) * ld + e % n] = Qj0[e];
    __syncthreads();
    // U = A P, then A = P^T U (symmetrised)
    for (int e = threadIdx.x; e < n * n; e += RRW) {
      const int r = e / n, c = e % n;
      double acc = 0;
      for (int k = 0; k < n; ++k) acc += A[r * ld + k] * Pm[k * ld + c];
      U[r * ld + c] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += RRW) {
      const int r = e / n, c = e % n;
      double acc = 0;
      for (int k = 0; k < n; ++k) acc += Pm[k * ld + r] * U[k * ld + c];
      A[r * ld + c] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += RRW) {
      const int r = e / n, c = e % n;
      if (c > r) {
        const double m = 0.5 * (A[r * ld + c] + A[c * ld + r]);
        A[r * ld + c] = m;
        A[c * ld + r] = m;
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * n; e += RRW)
    U[(e / n) * ld + e % n] = (e / n == e % n) ? 1.0 : 0.0;
  const int n2 = n + (n & 1);       // round-robin over an even count
  const int npair = n2 / 2;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal and total Frobenius norms
    double so = 0, st = 0;
    for (int e = threadIdx.x; e < n * n; e += RRW) {
      const double a = A[(e / n) * ld + e % n];
      st += a * a;
      if (e / n != e % n) so += a * a;
    }
    for (int o = 32; o > 0; o >>= 1) {
      so += __shfl_xor(so, o);
      st += __shfl_xor(st, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = so;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < RRW / 64; ++w) t += red[w];
      offn = t;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = st;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < RRW / 64; ++w) t += red[w];
      totn = t;
    }
    __syncthreads();
    if (!(offn > 1e-32 * totn) || n == 1) break;
    for (int round = 0; round < n2 - 1; ++round) {
      if (threadIdx.x < npair) {
        const int i = threadIdx.x;
        auto pos = [&](int m) { return m == 0 ? 0 : 1 + (m - 1 + round) % (n2 - 1); };
        int p = pos(i), q = pos(n2 - 1 - i);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1, s = 0;
        if (q < n) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double app = A[p * ld + p], aqq = A[q * ld + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0 ? 1.0 : -1.0) /
                             (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[i] = p; qq[i] = q; cs[i] = c; sn[i] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = threadIdx.x; e < npair * n; e += RRW) {
        const int i = e / n, m = e % n;
        const int p = pp[i], q = qq[i];
        if (q >= n || sn[i] == 0.0) continue;
        const double c = cs[i], s = sn[i];
        const double ap = A[p * ld + m], aq = A[q * ld + m];
        A[p * ld + m] = c * ap - s * aq;
        A[q * ld + m] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, U <- U J
      for (int e = threadIdx.x; e < npair * n; e += RRW) {
        const int i = e / n, m = e % n;
        const int p = pp[i], q = qq[i];
        if (q >= n || sn[i] == 0.0) continue;
        const double c = cs[i], s = sn[i];
        const double ap = A[m * ld + p], aq = A[m * ld + q];
        A[m * ld + p] = c * ap - s * aq;
        A[m * ld + q] = s * ap + c * aq;
        const double up = U[m * ld + p], uq = U[m * ld + q];
        U[m * ld + p] = c * up - s * uq;
        U[m * ld + q] = s * up + c * uq;
      }
      __syncthreads();
    }
  }
  // ascending order (stable by index), Q[k][rank] = U[k][i]
  double* Qj = Q + fr.small_off;
  for (int i = threadIdx.x; i < n; i += RRW) {
    const double d = A[i * ld + i];
    int rank = 0;
    for (int m = 0; m < n; ++m) {
      const double dm = A[m * ld + m];
      rank += (dm < d) || (dm == d && m < i);
    }
    theta[fr.th_off + rank] = d;
    if (pre) {
      for (int k2 = 0; k2 < n; ++k2) {
        double acc = 0;
        for (int mm = 0; mm < n; ++mm) acc += Pm[k2 * ld + mm] * U[mm * ld + i];
        Qj[k2 * n + rank] = acc;
      }
    } else {
      for (int k2 = 0; k2 < n; ++k2) Qj[k2 * n + rank] = U[k2 * ld + i];
    }
  }
}

void rr_eig(hipStream_t s, const ofm_frags* f, const double* G, double* Q,
            double* theta, const int* active, int pre) {
  const int ld = f->max_bw + 1;
  hipLaunchKernelGGL(k_rr_eig, dim3(f->n_frag), dim3(RRW),
                     3 * (size_t)f->max_bw * ld * sizeof(double), s, f->d_frag,
                     f->n_frag, G, Q, theta, active, pre, ld);
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// rotation X <- X Q (and HX <- HX Q with residual partial sums)
// ---------------------------------------------------------------------------
// Sum of v over a wave: butterflies inside each 16-lane row (DPP quad
// permutations and row rotations), then the four row sums.  Every lane of
// the wave must be active.
__device__ __forceinline__ float wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1,
                                                  0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e,
                                                  0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124,
                                                  0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128,
                                                  0xf, 0xf, true));
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 32)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

// One thread per point of a 256-point chunk.  Q sits in LDS transposed and
// zero-padded to BMAX x BMAX (column i of Q is a contiguous row), so a
// thread reads four coefficients per LDS load; the products accumulate in
// the storage type over k in ascending order.  With `upper` (a triangular
// CholQR factor) only k <= i contributes.  The squared residuals
// |HX'_i - theta_i X'_i|^2 of the stored values are summed per wave in FP32
// (a convergence test needs only a few digits) and per chunk in FP64.  The
// block is streamed once (non-temporal loads and stores: ~1% faster than
// cached access on the alkane workload).
template <typename T, int BMAX, bool WITH_HX>
__global__ __launch_bounds__(RCH) void k_rotate(
    const FragDev* __restrict__ F, const int2* __restrict__ rt,
    const int* __restrict__ tlist, int nt, T* __restrict__ X,
    T* __restrict__ HX, const double* __restrict__ Q,
    const double* __restrict__ theta, double* __restrict__ res_partial,
    const int* __restrict__ active, int upper) {
  static_assert(BMAX % 4 == 0, "BMAX must be a multiple of 4");
  if ((int)blockIdx.x >= nt) return;
  const int t = tlist[blockIdx.x];   // a chunk of this launch's width class
  const int j = rt[t].x;
  if (active && !active[j]) return;
  const FragDev& fr = F[j];
  const int bw = fr.bw;
  __shared__ __align__(16) T qt[BMAX * BMAX];
  __shared__ double th[BMAX];
  __shared__ float red[RCH / 64][BMAX];
  const double* Qj = Q + fr.small_off;
  for (int e = threadIdx.x; e < BMAX * BMAX; e += RCH) {
    const int i = e / BMAX, k = e % BMAX;
    qt[e] = (i < bw && k < bw && (!upper || k <= i)) ? (T)Qj[k * bw + i]
                                                    : T(0);
  }
  if (WITH_HX)
    for (int i = threadIdx.x; i < bw; i += RCH) th[i] = theta[fr.th_off + i];
  __syncthreads();
  const int p = rt[t].y * RCH + threadIdx.x;
  const bool ok = p < fr.npts;
  T* xp = X + fr.x_off + (ok ? p : 0);
  T x[BMAX], hx[BMAX];
#pragma unroll
  for (int k = 0; k < BMAX; ++k) {
    x[k] = (ok && k < bw) ? __builtin_nontemporal_load(&xp[(long long)k * fr.ld])
                          : T(0);
  }
  T* hp = nullptr;
  if (WITH_HX) {
    hp = HX + fr.x_off + (ok ? p : 0);
#pragma unroll
    for (int k = 0; k < BMAX; ++k)
      hx[k] = (ok && k < bw)
                  ? __builtin_nontemporal_load(&hp[(long long)k * fr.ld])
                  : T(0);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < bw; ++i) {
    T a = 0, h = 0;
    const T* qi = qt + i * BMAX;
#pragma unroll
    for (int k = 0; k < BMAX; k += 4) {
      if (k < bw && (!upper || k <= i)) {
        T q4[4];
        if constexpr (sizeof(T) == 4) {
          typedef float f4 __attribute__((ext_vector_type(4)));
          const f4 v = *reinterpret_cast<const f4*>(qi + k);
          q4[0] = v[0]; q4[1] = v[1]; q4[2] = v[2]; q4[3] = v[3];
        } else {
          const d4 v = *reinterpret_cast<const d4*>(qi + k);
          q4[0] = v[0]; q4[1] = v[1]; q4[2] = v[2]; q4[3] = v[3];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a = fma(x[k + u], q4[u], a);
          if (WITH_HX) h = fma(hx[k + u], q4[u], h);
        }
      }
    }
    if (ok) __builtin_nontemporal_store(a, &xp[(long long)i * fr.ld]);
    if (WITH_HX) {
      if (ok) __builtin_nontemporal_store(h, &hp[(long long)i * fr.ld]);
      const double r = ok ? (double)h - th[i] * (double)a : 0.0;
      const float ws = wave_sum((float)(r * r));
      if (lane == 0) red[wave][i] = ws;
    }
  }
  if (WITH_HX) {
    __syncthreads();
    for (int i = threadIdx.x; i < bw; i += RCH) {
      double s = 0;
      for (int w = 0; w < RCH / 64; ++w) s += red[w][i];
      res_partial[(long long)t * SMAX + i] = s;
    }
  }
}

template <typename T>
void rotate(ofm_ctx* c, const ofm_frags* f, T* X, T* HX, const double* Q,
            const double* theta, double* res_partial, const int* active,
            int upper, double bytes, double flops) {
  int nl = 0;
  for (int cl = 0; cl < 5; ++cl) nl += f->n_rtl[cl] > 0;
  Timed tm(c, "rotate", bytes, flops, nl);
  // one launch per width class (rotate_class)
  // the X-only form (CholQR) holds half the registers of the X and HX form
  // (a split of the Rayleigh-Ritz rotation into an X launch and an HX launch
  // that reads the rotated X back ran 7% slower than the fused form)
#define ROT(BM)                                                              \
  do {                                                                       \
    if (HX)                                                                  \
      hipLaunchKernelGGL((k_rotate<T, BM, true>), dim3(n), dim3(RCH), 0,     \
                         c->stream, f->d_frag, f->d_rtiles, f->d_rtl[cl], n, \
                         X, HX, Q, theta, res_partial, active, upper);       \
    else                                                                     \
      hipLaunchKernelGGL((k_rotate<T, BM, false>), dim3(n), dim3(RCH), 0,    \
                         c->stream, f->d_frag, f->d_rtiles, f->d_rtl[cl], n, \
                         X, HX, Q, theta, res_partial, active, upper);       \
  } while (0)
  for (int cl = 0; cl < 5; ++cl) {
    const int n = f->n_rtl[cl];
    if (n == 0) continue;
    if (cl == 0) ROT(16);
    else if (cl == 1) ROT(24);
    else if (cl == 2) ROT(32);
    else if (cl == 3) ROT(48);
    else ROT(64);
  }
#undef ROT
  OFM_HIP(hipGetLastError());
}
template void rotate<double>(ofm_ctx*, const ofm_frags*, double*, double*,
                             const double*, const double*, double*,
                             const int*, int, double, double);
template void rotate<float>(ofm_ctx*, const ofm_frags*, float*, float*,
                            const double*, const double*, double*,
                            const int*, int, double, double);

// ---------------------------------------------------------------------------
// end of an outer iteration: residual norms, convergence, filter bounds
// ---------------------------------------------------------------------------
// one workgroup per fragment: residual norms (chunk partials summed in a
// fixed order), convergence, locking of the converged leading Ritz vectors
// (the filter skips them) and the next filter interval
__global__ __launch_bounds__(WG) void k_finalize(
    const FragDev* __restrict__ F, int nf, const double* __restrict__ theta,
    const double* __restrict__ res_partial, FilterState* __restrict__ fs,
    int* __restrict__ active, int* __restrict__ iters,
    unsigned char* __restrict__ conv, double tol, int* __restrict__ n_active,
    double* __restrict__ res, double upper_kin) {
  const int j = blockIdx.x;
  if (j >= nf) return;
  if (!active[j]) return;
  const FragDev& fr = F[j];
  const int bw = fr.bw;
  constexpr int PARTS = 16;
  __shared__ double part[SMAX][PARTS];
  __shared__ double rn[SMAX];
  for (int e = threadIdx.x; e < bw * PARTS; e += WG) {
    const int i = e / PARTS, q = e % PARTS;
    double s = 0;
    for (int t = fr.rt_begin + q; t < fr.rt_begin + fr.rt_count; t += PARTS)
      s += res_partial[(long long)t * SMAX + i];
    part[i][q] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < bw; i += WG) {
    double s = 0;
    for (int q = 0; q < PARTS; ++q) s += part[i][q];
    rn[i] = sqrt(s);
    res[fr.th_off + i] = rn[i];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double worst = 0;
  int lock = 0;
  bool prefix = true;
  for (int i = 0; i < fr.n_states; ++i) {
    worst = fmax(worst, rn[i]);
    if (prefix && rn[i] <= tol)
      lock = i + 1;
    else
      prefix = false;
  }
  iters[j] += 1;
  FilterState st;
  st.upper = upper_kin + fmax(fr.vmax, 0.0);
  st.lower = theta[fr.th_off + bw - 1];
  st.scale = theta[fr.th_off];
  st.worst = worst;
  st.lock = lock;
  st.pad = 0;
  fs[j] = st;
  if (worst <= tol || bw == fr.npts) {
    active[j] = 0;
    conv[j] = 1;
  } else {
    atomicAdd(n_active, 1);
  }
}

void finalize_iter(hipStream_t s, const ofm_frags* f, const double* theta,
                   const double* res_partial, FilterState* fs, int* active,
                   int* iters, unsigned char* conv, double tol, int* n_active,
                   double* res) {
  const double h = f->grid.h;
  hipLaunchKernelGGL(k_finalize, dim3(f->n_frag), dim3(WG), 0, s, f->d_frag,
                     f->n_frag, theta, res_partial, fs, active, iters, conv,
                     tol, n_active, res, 8.0 / (h * h));
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// sign gauge: the largest-|.| component of every state is positive
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(WG) void k_gauge(const FragDev* __restrict__ F,
                                             const int2* __restrict__ st,
                                             int nst, T* __restrict__ X) {
  const int t = blockIdx.x;
  if (t >= nst) return;
  const FragDev& fr = F[st[t].x];
  T* x = X + fr.x_off + (long long)st[t].y * fr.ld;
  double best = -1;
  int bi = 0x7fffffff;
  for (int p = threadIdx.x; p < fr.npts; p += WG) {
    const double a = fabs((double)x[p]);
    if (a > best) { best = a; bi = p; }
  }
  __shared__ double sb[WG];
  __shared__ int si[WG];
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double b2 = sb[threadIdx.x + o];
      const int i2 = si[threadIdx.x + o];
      if (b2 > sb[threadIdx.x] || (b2 == sb[threadIdx.x] && i2 < si[threadIdx.x])) {
        sb[threadIdx.x] = b2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const bool flip = x[si[0]] < T(0);
  __syncthreads();
  if (flip)
    for (int p = threadIdx.x; p < fr.npts; p += WG) x[p] = -x[p];
}

template <typename T>
void gauge(hipStream_t s, const ofm_frags* f, T* X) {
  hipLaunchKernelGGL(k_gauge<T>, dim3(f->n_stiles), dim3(WG), 0, s, f->d_frag,
                     f->d_stiles, f->n_stiles, X);
  OFM_HIP(hipGetLastError());
}
template void gauge<double>(hipStream_t, const ofm_frags*, double*);
template void gauge<float>(hipStream_t, const ofm_frags*, float*);

// ---------------------------------------------------------------------------
// H|phi> with the whole-system H on the dilated box
// ---------------------------------------------------------------------------
// phi is zero outside box_j; walls (with the odd second ghost) only where the
// point lies on a global-grid face.  V enters only inside the box.
template <typename T>
__global__ __launch_bounds__(WG) void k_whole_h(
    const FragDev* __restrict__ F, const int2* __restrict__ st, int nst,
    const T* __restrict__ Vj, const T* __restrict__ X, T* __restrict__ HP,
    double nh, int gnx, int gny, int gnz, int only_frag) {
  const int t = blockIdx.y;
  if (t >= nst) return;
  const int j = st[t].x, i = st[t].y;
  if (only_frag >= 0 && j != only_frag) return;
  const FragDev& fr = F[j];
  const T* x = X + fr.x_off + (long long)i * fr.ld;
  T* out = HP + fr.hphi_off + (long long)i * fr.ldd;
  const int bx = fr.dims[0], by = fr.dims[1], bz = fr.dims[2];
  const int ox = fr.lo[0] - fr.dlo[0], oy = fr.lo[1] - fr.dlo[1],
            oz = fr.lo[2] - fr.dlo[2];
  for (int p = blockIdx.x * WG + threadIdx.x; p < fr.ndil;
       p += gridDim.x * WG) {
    const int dx = p % fr.ddims[0];
    const int dy = (p / fr.ddims[0]) % fr.ddims[1];
    const int dz = p / (fr.ddims[0] * fr.ddims[1]);
    const int x0 = dx - ox, y0 = dy - oy, z0 = dz - oz;  // box-local
    auto at = [&](int xx, int yy, int zz) -> double {
      if (xx < 0 || yy < 0 || zz < 0 || xx >= bx || yy >= by || zz >= bz)
        return 0.0;
      return (double)x[xx + bx * (yy + by * zz)];
    };
    const double c = at(x0, y0, z0);
    double lap = W0 * 3.0 * c +
                 W1 * (at(x0 - 1, y0, z0) + at(x0 + 1, y0, z0) +
                       at(x0, y0 - 1, z0) + at(x0, y0 + 1, z0) +
                       at(x0, y0, z0 - 1) + at(x0, y0, z0 + 1)) +
                 W2 * (at(x0 - 2, y0, z0) + at(x0 + 2, y0, z0) +
                       at(x0, y0 - 2, z0) + at(x0, y0 + 2, z0) +
                       at(x0, y0, z0 - 2) + at(x0, y0, z0 + 2));
    const int gx = fr.dlo[0] + dx, gy = fr.dlo[1] + dy, gz = fr.dlo[2] + dz;
    const int nfaces = (gx == 0) + (gx == gnx - 1) + (gy == 0) +
                       (gy == gny - 1) + (gz == 0) + (gz == gnz - 1);
    lap -= W2 * nfaces * c;
    double v = 0;
    if (x0 >= 0 && y0 >= 0 && z0 >= 0 && x0 < bx && y0 < by && z0 < bz)
      v = (double)Vj[fr.v_off + x0 + bx * (y0 + by * z0)];
    out[p] = (T)(nh * lap + v * c);
  }
}

template <typename T>
void whole_h(ofm_ctx* c, const ofm_frags* f, const T* X, T* HPHI,
             int only_frag) {
  const T* Vj;
  if constexpr (sizeof(T) == 8)
    Vj = (const T*)f->d_v;
  else
    Vj = (const T*)f->d_v32;
  int maxd = 0;
  for (auto& d : f->host) maxd = std::max(maxd, d.ndil);
  dim3 grid(std::min((maxd + WG - 1) / WG, 32), f->n_stiles);
  const double h = f->grid.h;
  hipLaunchKernelGGL(k_whole_h<T>, grid, dim3(WG), 0, c->stream, f->d_frag,
                     f->d_stiles, f->n_stiles, Vj, X, HPHI, -0.5 / (h * h),
                     f->grid.nx, f->grid.ny, f->grid.nz, only_frag);
  OFM_HIP(hipGetLastError());
}
template void whole_h<double>(ofm_ctx*, const ofm_frags*, const double*,
                              double*, int);
template void whole_h<float>(ofm_ctx*, const ofm_frags*, const float*, float*,
                             int);

// ---------------------------------------------------------------------------
// grouped pair contraction: one workgroup per pair, its H and S blocks
// together
// ---------------------------------------------------------------------------
// Omega' (the support of the H block, with Omega, the support of S, inside
// it) is walked in groups of G consecutive points along x, every row of
// Omega' padded to whole groups.  Lane (r, g) of a wave feeds state r of
// each 16-state tile with the G points of group g of the wave's current
// chunk of four groups, loaded from global memory straight into MFMA
// operands (no LDS staging and no barrier in the loop); the states of
// fragment j are loaded once for both blocks.  Work split over the four
// waves of a workgroup:
//  * blocks of at most 32 x 32 states (KSPLIT): every wave computes all
//    tiles of both blocks over every fourth chunk; the four waves' sums are
//    added in LDS in wave order;
//  * wider blocks: wave w computes row tile w of both blocks over every
//    chunk.
// Every sum is formed in a fixed order: the results do not depend on
// scheduling.
struct GroupPos {   // a lane's group inside Omega'
  int q;            // linear group index (x groups fastest, then y, then z)
  int xg, y, z;
};

__device__ __forceinline__ void group_init(GroupPos& p, int q, int gx, int oy) {
  p.q = q;
  p.xg = q % gx;
  const int row = q / gx;
  p.y = row % oy;
  p.z = row / oy;
}

// advance by `step` groups, i.e. drow = step / gx whole rows and
// dx = step % gx groups
__device__ __forceinline__ void group_step(GroupPos& p, int step, int dx,
                                           int drow, int gx, int oy) {
  p.q += step;
  p.xg += dx;
  p.y += drow;
  if (p.xg >= gx) {
    p.xg -= gx;
    ++p.y;
  }
  while (p.y >= oy) {
    p.y -= oy;
    ++p.z;
  }
}

__device__ __forceinline__ long long box_off(const int* org, int nx, int nxy,
                                             int x, int y, int z) {
  return (long long)(org[0] + x) + (long long)nx * (org[1] + y) +
         (long long)nxy * (org[2] + z);
}

// 16-byte vectors at the element type's own alignment: a whole group of a
// row is loaded with dwordx4 loads wherever it starts
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

// o[u] = p[off + u] for lo <= u < hi, 0 elsewhere (u < G); a whole group
// (lo = 0, hi = G) is read with 16-byte loads, a partial one (row ends, the
// edge of Omega) element by element, so nothing outside [lo, hi) is read
template <int G, typename TI, typename TO>
__device__ __forceinline__ void load_range(const TI* __restrict__ p,
                                           long long off, int lo, int hi,
                                           TO* o) {
  constexpr int VW = 16 / sizeof(TI);   // elements per 16-byte load
  static_assert(G % VW == 0, "a group is whole 16-byte loads");
  if (lo == 0 && hi == G) {
#pragma unroll
    for (int u = 0; u < G; u += VW) {
      if constexpr (sizeof(TI) == 8) {
        const d2u v = *reinterpret_cast<const d2u*>(p + off + u);
        o[u] = (TO)v[0];
        o[u + 1] = (TO)v[1];
      } else {
        const f4u v = *reinterpret_cast<const f4u*>(p + off + u);
        o[u] = (TO)v[0];
        o[u + 1] = (TO)v[1];
        o[u + 2] = (TO)v[2];
        o[u + 3] = (TO)v[3];
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < G; ++u)
      o[u] = (u >= lo && u < hi) ? (TO)p[off + u] : TO(0);
  }
}

// where a lane's group meets Omega (the S block's support): [slo, shi)
__device__ __forceinline__ void s_range(const PairTask& tk, const GroupPos& p,
                                        int x0, int nv, bool doS, int& slo,
                                        int& shi) {
  slo = shi = 0;
  if (doS && nv > 0 && p.y >= tk.s_lo[1] && p.y < tk.s_hi[1] &&
      p.z >= tk.s_lo[2] && p.z < tk.s_hi[2]) {
    slo = max(tk.s_lo[0] - x0, 0);
    shi = min(tk.s_hi[0] - x0, nv);
  }
}

// LDS: the cross-wave sums (KSPLIT) and then both blocks as dense
// RM x RM matrices (row stride RM + 1), H first
template <int NTA, int NTB, bool KSPLIT>
struct PairLds {
  static constexpr int RM = 16 * NTB, LD = RM + 1;
  static constexpr int RED = KSPLIT ? 2 * NTA * NTB * 256 : 0;
  static constexpr int OUT = 2 * RM * LD;
  static constexpr int SIZE = RED > OUT ? RED : OUT;
};

// write both blocks from the LDS matrices (diagonal blocks symmetrised);
// with s_ident the S block is the identity
template <int RM>
__device__ __forceinline__ void pair_write(const PairTask& tk,
                                           const double* sh, bool wH,
                                           bool wS, bool s_ident,
                                           double* __restrict__ Hout,
                                           double* __restrict__ Sout) {
  constexpr int LD = RM + 1;
  const int ma = tk.ma, mb = tk.mb;
  double* CH = Hout + tk.c_off;
  double* CS = Sout + tk.c_off;
  const double* sS = sh + RM * LD;
  for (int e = threadIdx.x; e < ma * mb; e += WG) {
    const int i = e / mb, m = e % mb;
    if (wH) {
      double v = sh[i * LD + m];
      if (tk.sym) v = 0.5 * (v + sh[m * LD + i]);
      CH[e] = v;
    }
    if (s_ident) {
      CS[e] = i == m ? 1.0 : 0.0;
    } else if (wS) {
      double v = sS[i * LD + m];
      if (tk.sym) v = 0.5 * (v + sS[m * LD + i]);
      CS[e] = v;
    }
  }
}

// FP64 MFMA 16x16x4, G = 4 points per lane group.  TI is the storage type of
// the operands (FP32 operands are widened, so products and sums are FP64).
// With s_only, only the S blocks of diagonal tasks of imported states
// (sym, ident == 0) are computed and every other task returns at once.
template <int NTA, int NTB, bool KSPLIT, typename TI, bool PF>
__global__ __launch_bounds__(WG) void k_pair(
    const PairTask* __restrict__ tasks, int ntask, const TI* __restrict__ X,
    const TI* __restrict__ HP, double* __restrict__ Hout,
    double* __restrict__ Sout, int s_only) {
  constexpr int G = 4;
  using L = PairLds<NTA, NTB, KSPLIT>;
  __shared__ double sh[L::SIZE];
  const int ti = blockIdx.x;
  if (ti >= ntask) return;
  const PairTask& tk = tasks[ti];
  if (s_only && !(tk.sym && !tk.ident)) return;
  const bool doH = !s_only;
  const bool doS = tk.has_s != 0;
  const int ma = tk.ma, mb = tk.mb;
  const int ox = tk.om[0], oy = tk.om[1], oz = tk.om[2];
  const int gx = (ox + G - 1) / G;
  const int ngrp = gx * oy * oz;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ta0 = KSPLIT ? 0 : wave;           // first row tile of the wave
  const bool wave_on = KSPLIT || 16 * wave < ma;
  const TI* pa[NTA];
  bool va[NTA];
#pragma unroll
  for (int t = 0; t < NTA; ++t) {
    const int row = 16 * (ta0 + t) + r;
    va[t] = row < ma;
    pa[t] = X + tk.a_off + (long long)(va[t] ? row : 0) * tk.lda;
  }
  const TI* pb[NTB];
  const TI* ph[NTB];
  bool vb[NTB];
#pragma unroll
  for (int t = 0; t < NTB; ++t) {
    const int row = 16 * t + r;
    vb[t] = row < mb;
    pb[t] = X + tk.b_off + (long long)(vb[t] ? row : 0) * tk.ldb;
    ph[t] = HP + tk.h_off + (long long)(vb[t] ? row : 0) * tk.ldh;
  }
  d4 accH[NTA][NTB], accS[NTA][NTB];
#pragma unroll
  for (int a = 0; a < NTA; ++a)
#pragma unroll
    for (int b = 0; b < NTB; ++b) accH[a][b] = accS[a][b] = d4{0, 0, 0, 0};
  const int step = KSPLIT ? 16 : 4;   // groups per iteration of one wave
  const int first = KSPLIT ? 4 * wave : 0;
  GroupPos pos;
  group_init(pos, first + g, gx, oy);
  const int dx = step % gx, drow = step / gx;
  // the operands of a lane's group (zeros outside Omega' / Omega)
  auto fetch = [&](const GroupPos& p, double (&A)[NTA][G],
                   double (&BH)[NTB][G], double (&BS)[NTB][G]) {
    const int x0 = G * p.xg;
    const int nv = p.q < ngrp ? min(G, ox - x0) : 0;
    const long long oa = box_off(tk.a_org, tk.a_nx, tk.a_nxy, x0, p.y, p.z);
    const long long oh = box_off(tk.h_org, tk.h_nx, tk.h_nxy, x0, p.y, p.z);
    const long long ob = box_off(tk.b_org, tk.b_nx, tk.b_nxy, x0, p.y, p.z);
    int slo, shi;
    s_range(tk, p, x0, nv, doS, slo, shi);
#pragma unroll
    for (int t = 0; t < NTA; ++t)
      load_range<G>(pa[t], oa, 0, va[t] ? nv : 0, A[t]);
#pragma unroll
    for (int t = 0; t < NTB; ++t) {
      load_range<G>(ph[t], oh, 0, (doH && vb[t]) ? nv : 0, BH[t]);
      load_range<G>(pb[t], ob, slo, vb[t] ? shi : 0, BS[t]);
    }
  };
  double a[NTA][G], bh[NTB][G], bs[NTB][G];
  if (PF && wave_on && first < ngrp) fetch(pos, a, bh, bs);
  if (wave_on)
    for (int c0 = first; c0 < ngrp; c0 += step) {   // wave-uniform
      // PF (software pipeline): the next chunk's loads are in flight while
      // this chunk's products run; otherwise a chunk is loaded, then used
      const bool more = PF && c0 + step < ngrp;      // wave-uniform
      GroupPos nxt = pos;
      group_step(nxt, step, dx, drow, gx, oy);
      double a2[NTA][G], bh2[NTB][G], bs2[NTB][G];
      if (!PF) fetch(pos, a, bh, bs);
      if (more) fetch(nxt, a2, bh2, bs2);
#pragma unroll
      for (int ta = 0; ta < NTA; ++ta) {
        if (16 * (ta0 + ta) >= ma) continue;   // wave-uniform
#pragma unroll
        for (int tb = 0; tb < NTB; ++tb) {
          if (16 * tb >= mb) continue;
#pragma unroll
          for (int u = 0; u < G; ++u) {
            if (doH) accH[ta][tb] = mfma_f64(a[ta][u], bh[tb][u], accH[ta][tb]);
            if (doS) accS[ta][tb] = mfma_f64(a[ta][u], bs[tb][u], accS[ta][tb]);
          }
        }
      }
      if (more) {
#pragma unroll
        for (int t = 0; t < NTA; ++t)
#pragma unroll
          for (int u = 0; u < G; ++u) a[t][u] = a2[t][u];
#pragma unroll
        for (int t = 0; t < NTB; ++t)
#pragma unroll
          for (int u = 0; u < G; ++u) {
            bh[t][u] = bh2[t][u];
            bs[t][u] = bs2[t][u];
          }
      }
      pos = nxt;
    }
  if constexpr (KSPLIT) {
    // the four waves' sums, in wave order
    for (int w = 1; w < WG / 64; ++w) {
      if (wave == w)
#pragma unroll
        for (int a = 0; a < NTA; ++a)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              sh[(((0 * NTA + a) * NTB + b) * 4 + i) * 64 + lane] = accH[a][b][i];
              sh[(((1 * NTA + a) * NTB + b) * 4 + i) * 64 + lane] = accS[a][b][i];
            }
      __syncthreads();
      if (wave == 0)
#pragma unroll
        for (int a = 0; a < NTA; ++a)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              accH[a][b][i] += sh[(((0 * NTA + a) * NTB + b) * 4 + i) * 64 + lane];
              accS[a][b][i] += sh[(((1 * NTA + a) * NTB + b) * 4 + i) * 64 + lane];
            }
      __syncthreads();
    }
  }
  // accumulator item i of lane (r, g): row g + 4 i, column r of the tile
  if (KSPLIT ? wave == 0 : wave_on) {
#pragma unroll
    for (int a = 0; a < NTA; ++a)
#pragma unroll
      for (int b = 0; b < NTB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * (ta0 + a) + g + 4 * i, col = 16 * b + r;
          if (row < ma && col < mb) {
            sh[row * L::LD + col] = accH[a][b][i];
            sh[L::RM * L::LD + row * L::LD + col] = accS[a][b][i];
          }
        }
  }
  __syncthreads();
  pair_write<L::RM>(tk, sh, doH, doS, false, Hout, Sout);
}

// mixed forms: split x3 MFMA 16x16x32 on the FP32 operands (MODE as in
// Split3), G = 8 points per lane group, the FP32 sums (a_hi b_hi and the
// cross terms apart) flushed into FP64 every PAIR_FLUSH iterations of a wave
// (128 points of Omega' per wave at most).  Diagonal S blocks: the identity
// for the solver's FP64-orthonormalised states (ident); for imported states
// k_pair<.., float> (s_only) computes them.
constexpr int PAIR_FLUSH = 4;

template <int NTA, int NTB, bool KSPLIT, int MODE, bool PF>
__global__ __launch_bounds__(WG) void k_pair_x3(
    const PairTask* __restrict__ tasks, int ntask,
    const float* __restrict__ X, const float* __restrict__ HP,
    double* __restrict__ Hout, double* __restrict__ Sout) {
  constexpr int G = 8;
  using L = PairLds<NTA, NTB, KSPLIT>;
  __shared__ double sh[L::SIZE];
  const int ti = blockIdx.x;
  if (ti >= ntask) return;
  const PairTask& tk = tasks[ti];
  const bool s_ident = tk.sym && tk.ident;
  const bool doS = tk.has_s && !tk.sym;   // diagonal S: identity or s_only
  const int ma = tk.ma, mb = tk.mb;
  const int ox = tk.om[0], oy = tk.om[1], oz = tk.om[2];
  const int gx = (ox + G - 1) / G;
  const int ngrp = gx * oy * oz;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ta0 = KSPLIT ? 0 : wave;
  const bool wave_on = KSPLIT || 16 * wave < ma;
  const float* pa[NTA];
  bool va[NTA];
#pragma unroll
  for (int t = 0; t < NTA; ++t) {
    const int row = 16 * (ta0 + t) + r;
    va[t] = row < ma;
    pa[t] = X + tk.a_off + (long long)(va[t] ? row : 0) * tk.lda;
  }
  const float* pb[NTB];
  const float* ph[NTB];
  bool vb[NTB];
#pragma unroll
  for (int t = 0; t < NTB; ++t) {
    const int row = 16 * t + r;
    vb[t] = row < mb;
    pb[t] = X + tk.b_off + (long long)(vb[t] ? row : 0) * tk.ldb;
    ph[t] = HP + tk.h_off + (long long)(vb[t] ? row : 0) * tk.ldh;
  }
  using SP = Split3<MODE>;
  f4v accH[NTA][NTB], accS[NTA][NTB], crH[NTA][NTB], crS[NTA][NTB];
  double totH[NTA][NTB][4], totS[NTA][NTB][4];
#pragma unroll
  for (int a = 0; a < NTA; ++a)
#pragma unroll
    for (int b = 0; b < NTB; ++b) {
      accH[a][b] = accS[a][b] = crH[a][b] = crS[a][b] = f4v{0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 4; ++i) totH[a][b][i] = totS[a][b][i] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < NTA; ++a)
#pragma unroll
      for (int b = 0; b < NTB; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          totH[a][b][i] += (double)accH[a][b][i] + SP::kCross * (double)crH[a][b][i];
          totS[a][b][i] += (double)accS[a][b][i] + SP::kCross * (double)crS[a][b][i];
        }
        accH[a][b] = accS[a][b] = crH[a][b] = crS[a][b] = f4v{0, 0, 0, 0};
      }
  };
  const int step = KSPLIT ? 16 : 4;
  const int first = KSPLIT ? 4 * wave : 0;
  GroupPos pos;
  group_init(pos, first + g, gx, oy);
  const int dx = step % gx, drow = step / gx;
  // the operands of a lane's group (zeros outside Omega' / Omega)
  auto fetch = [&](const GroupPos& p, float (&A)[NTA][G], float (&BH)[NTB][G],
                   float (&BS)[NTB][G]) {
    const int x0 = G * p.xg;
    const int nv = p.q < ngrp ? min(G, ox - x0) : 0;
    const long long oa = box_off(tk.a_org, tk.a_nx, tk.a_nxy, x0, p.y, p.z);
    const long long oh = box_off(tk.h_org, tk.h_nx, tk.h_nxy, x0, p.y, p.z);
    const long long ob = box_off(tk.b_org, tk.b_nx, tk.b_nxy, x0, p.y, p.z);
    int slo, shi;
    s_range(tk, p, x0, nv, doS, slo, shi);
#pragma unroll
    for (int t = 0; t < NTA; ++t)
      load_range<G>(pa[t], oa, 0, va[t] ? nv : 0, A[t]);
#pragma unroll
    for (int t = 0; t < NTB; ++t) {
      load_range<G>(ph[t], oh, 0, vb[t] ? nv : 0, BH[t]);
      load_range<G>(pb[t], ob, slo, vb[t] ? shi : 0, BS[t]);
    }
  };
  int since = 0;
  float fa[NTA][G], fh[NTB][G], fs[NTB][G];
  if (PF && wave_on && first < ngrp) fetch(pos, fa, fh, fs);
  if (wave_on)
    for (int c0 = first; c0 < ngrp; c0 += step) {   // wave-uniform
      // PF (software pipeline): the next chunk's loads are in flight while
      // this chunk's products run; otherwise a chunk is loaded, then used
      const bool more = PF && c0 + step < ngrp;      // wave-uniform
      GroupPos nxt = pos;
      group_step(nxt, step, dx, drow, gx, oy);
      float fa2[NTA][G], fh2[NTB][G], fs2[NTB][G];
      if (!PF) fetch(pos, fa, fh, fs);
      if (more) fetch(nxt, fa2, fh2, fs2);
      typename SP::V ah[NTA], al[NTA];
#pragma unroll
      for (int t = 0; t < NTA; ++t) SP::split(fa[t], ah[t], al[t]);
#pragma unroll
      for (int tb = 0; tb < NTB; ++tb) {
        if (16 * tb >= mb) continue;   // wave-uniform
        typename SP::V bh, bl, sh8, sl8;
        SP::split(fh[tb], bh, bl);
        if (doS) SP::split(fs[tb], sh8, sl8);
#pragma unroll
        for (int ta = 0; ta < NTA; ++ta) {
          if (16 * (ta0 + ta) >= ma) continue;
          mma3<MODE>(ah[ta], al[ta], bh, bl, accH[ta][tb], crH[ta][tb]);
          if (doS)
            mma3<MODE>(ah[ta], al[ta], sh8, sl8, accS[ta][tb], crS[ta][tb]);
        }
      }
      if (++since == PAIR_FLUSH) {
        since = 0;
        flush();
      }
      if (more) {
#pragma unroll
        for (int t = 0; t < NTA; ++t)
#pragma unroll
          for (int u = 0; u < G; ++u) fa[t][u] = fa2[t][u];
#pragma unroll
        for (int t = 0; t < NTB; ++t)
#pragma unroll
          for (int u = 0; u < G; ++u) {
            fh[t][u] = fh2[t][u];
            fs[t][u] = fs2[t][u];
          }
      }
      pos = nxt;
    }
  flush();
  if constexpr (KSPLIT) {
    for (int w = 1; w < WG / 64; ++w) {
      if (wave == w)
#pragma unroll
        for (int a = 0; a < NTA; ++a)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              sh[(((0 * NTA + a) * NTB + b) * 4 + i) * 64 + lane] = totH[a][b][i];
              sh[(((1 * NTA + a) * NTB + b) * 4 + i) * 64 + lane] = totS[a][b][i];
            }
      __syncthreads();
      if (wave == 0)
#pragma unroll
        for (int a = 0; a < NTA; ++a)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              totH[a][b][i] += sh[(((0 * NTA + a) * NTB + b) * 4 + i) * 64 + lane];
              totS[a][b][i] += sh[(((1 * NTA + a) * NTB + b) * 4 + i) * 64 + lane];
            }
      __syncthreads();
    }
  }
  // accumulator item i of lane (r, g): row 4 g + i, column r of the tile
  if (KSPLIT ? wave == 0 : wave_on) {
#pragma unroll
    for (int a = 0; a < NTA; ++a)
#pragma unroll
      for (int b = 0; b < NTB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * (ta0 + a) + 4 * g + i, col = 16 * b + r;
          if (row < ma && col < mb) {
            sh[row * L::LD + col] = totH[a][b][i];
            sh[L::RM * L::LD + row * L::LD + col] = totS[a][b][i];
          }
        }
  }
  __syncthreads();
  pair_write<L::RM>(tk, sh, true, doS, s_ident, Hout, Sout);
}

template <typename T>
void pair_elements(ofm_ctx* c, const ofm_frags* f, const PairTask* tasks,
                   int n_tasks, const T* phi, const T* hphi, double* H,
                   double* S, double flops, double bytes, int variant) {
  if (n_tasks <= 0) return;
  Timed tm(c, "elements", bytes, flops);
  const int nt = (f->max_states + 15) / 16;
  const bool fp16 = c->precision == OFM_MIXED_FP16X3;
#define PAIR1(A, B, K, PF)                                                   \
  do {                                                                       \
    if constexpr (sizeof(T) == 8)                                            \
      hipLaunchKernelGGL((k_pair<A, B, K, double, PF>), dim3(n_tasks),       \
                         dim3(WG), 0, c->stream, tasks, n_tasks,             \
                         (const double*)phi, (const double*)hphi, H, S, 0);  \
    else if (fp16)                                                           \
      hipLaunchKernelGGL((k_pair_x3<A, B, K, 1, PF>), dim3(n_tasks),         \
                         dim3(WG), 0, c->stream, tasks, n_tasks,             \
                         (const float*)phi, (const float*)hphi, H, S);       \
    else                                                                     \
      hipLaunchKernelGGL((k_pair_x3<A, B, K, 0, PF>), dim3(n_tasks),         \
                         dim3(WG), 0, c->stream, tasks, n_tasks,             \
                         (const float*)phi, (const float*)hphi, H, S);       \
  } while (0)
#define PAIR(A, B, K)                                                        \
  do {                                                                       \
    if (variant == 1) PAIR1(A, B, K, true);                                  \
    else PAIR1(A, B, K, false);                                              \
  } while (0)
  if (nt <= 1) PAIR(1, 1, true);
  else if (nt == 2) PAIR(2, 2, true);
  else if (nt == 3) PAIR(1, 3, false);
  else PAIR(1, 4, false);
#undef PAIR
#undef PAIR1
  OFM_HIP(hipGetLastError());
}

void pair_elements_f64_on_f32(ofm_ctx* c, const ofm_frags* f,
                              const PairTask* tasks, int n_tasks,
                              const float* phi, const float* hphi, double* H,
                              double* S) {
  if (n_tasks <= 0) return;
  const int nt = (f->max_states + 15) / 16;
#define PAIRF(A, B, K)                                                       \
  hipLaunchKernelGGL((k_pair<A, B, K, float, true>), dim3(n_tasks), dim3(WG), \
                     0, c->stream, tasks, n_tasks, phi, hphi, H, S, 1)
  if (nt <= 1) PAIRF(1, 1, true);
  else if (nt == 2) PAIRF(2, 2, true);
  else if (nt == 3) PAIRF(1, 3, false);
  else PAIRF(1, 4, false);
#undef PAIRF
  OFM_HIP(hipGetLastError());
}
template void pair_elements<double>(ofm_ctx*, const ofm_frags*,
                                    const PairTask*, int, const double*,
                                    const double*, double*, double*, double,
                                    double, int);
template void pair_elements<float>(ofm_ctx*, const ofm_frags*, const PairTask*,
                                   int, const float*, const float*, double*,
                                   double*, double, double, int);


__global__ void k_fill_zero(double* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < n;
       i += (long long)gridDim.x * WG)
    p[i] = 0.0;
}

void fill_zero(hipStream_t s, double* p, long long n) {
  if (n <= 0) return;
  const int nb = (int)std::min<long long>((n + WG - 1) / WG, 8192);
  hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(WG), 0, s, p, n);
  OFM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// conversions and copies between the FP64 host layout and the arenas
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_convert(const double* __restrict__ in, T* __restrict__ out,
                          long long n) {
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < n;
       i += (long long)gridDim.x * WG)
    out[i] = (T)in[i];
}
template <typename T>
__global__ void k_convert_back(const T* __restrict__ in,
                               double* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)WG + threadIdx.x; i < n;
       i += (long long)gridDim.x * WG)
    out[i] = (double)in[i];
}
template <typename T>
void convert(hipStream_t s, const double* in, T* out, long long n) {
  const int nb = (int)std::min<long long>((n + WG - 1) / WG, 4096);
  hipLaunchKernelGGL(k_convert<T>, dim3(std::max(nb, 1)), dim3(WG), 0, s, in,
                     out, n);
  OFM_HIP(hipGetLastError());
}
template <typename T>
void convert_back(hipStream_t s, const T* in, double* out, long long n) {
  const int nb = (int)std::min<long long>((n + WG - 1) / WG, 4096);
  hipLaunchKernelGGL(k_convert_back<T>, dim3(std::max(nb, 1)), dim3(WG), 0, s,
                     in, out, n);
  OFM_HIP(hipGetLastError());
}
template void convert<double>(hipStream_t, const double*, double*, long long);
template void convert<float>(hipStream_t, const double*, float*, long long);
template void convert_back<double>(hipStream_t, const double*, double*,
                                   long long);
template void convert_back<float>(hipStream_t, const float*, double*,
                                  long long);

}  // namespace k
}  // namespace ofm
