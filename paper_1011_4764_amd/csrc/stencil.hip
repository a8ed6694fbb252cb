// Fragment Hamiltonian stencil for gfx950 (MI355X, CDNA4): H_j = -1/2 Lap
// + V_j on a box with image-ghost Dirichlet walls (4th-order central
// differences), and the scaled three-term Chebyshev step built on it.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>
#include <vector>

#include "kdev.h"
#include "ofm_internal.h"

namespace ofm {
namespace k {

// ---------------------------------------------------------------------------
// fragment Hamiltonian / Chebyshev step
// ---------------------------------------------------------------------------
// mode 0: out = H_j in
// mode 1: step k of the scaled Chebyshev filter on [lower, upper] normalised
//         at `scale`:  Y_1 = (s1/e)(H - c) Y_0,
//         Y_k = (2 s_k/e)(H - c) Y_{k-1} - s_{k-1} s_k Y_{k-2},
//         e = (upper-lower)/2, c = (upper+lower)/2, s1 = e/(scale-c),
//         s_k = 1/(2/s1 - s_{k-1}).
// `prev` and `out` may alias (each point of `out` depends on `prev` at the
// same point only); `in` must not alias either.
// One workgroup handles a strip of SP = 256 PPT consecutive points of the
// xy plane of one (fragment, vector) and marches along z.  Its LDS window is
// the strip plus two rows on each side (the y neighbours); when the whole
// plane fits in one strip there is no halo at all.  The +-1, +-2 z
// neighbours of the strip's own points ride in a 5-deep register queue; V
// and the previous Chebyshev vector are prefetched one plane ahead.  All
// strips of a vector compute the same arithmetic per point, so every PPT
// variant gives bit-identical results.
constexpr int HALO_NX_MAX = 128;   // boxes may span at most 128 points in x

// Per-step coefficients of out = a1 s1 + a2 s2 + (alpha u + gamma) c
// + beta pn, where c is the point's value, s1 / s2 the sums of its +-1 /
// +-2 neighbours along the three axes, u = nh (3 W0 - W2 nfaces) + V its
// diagonal (nh = -1/(2 h^2); each box face the point touches adds the odd
// image of the second ghost) and pn the point's value two steps back.
// mode 0 (out = H_j y): a1 = nh W1, a2 = nh W2, alpha = 1, gamma = beta = 0.
// mode 1, Chebyshev step k: out = alpha H y_{k-1} + gamma y_{k-1}
// + beta y_{k-2}, so a1 = alpha nh W1 and a2 = alpha nh W2.  A degenerate
// interval gives the identity.
template <typename T>
struct StepCoef {
  T a1, a2, alpha, gamma, beta;
};

// a value every lane of the wave holds alike, moved to scalar registers
// (the coefficients of a step are the same for the whole workgroup; kept in
// vector registers they would take 20 of them for two FP64 steps)
__device__ __forceinline__ float wave_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double wave_uniform(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ StepCoef<T> wave_uniform(const StepCoef<T>& k) {
  return {wave_uniform(k.a1), wave_uniform(k.a2), wave_uniform(k.alpha),
          wave_uniform(k.gamma), wave_uniform(k.beta)};
}

// mode 0 (out = H_j y)
template <typename T>
__device__ __forceinline__ StepCoef<T> h_coefs(double nh) {
  StepCoef<T> k;
  k.a1 = (T)(nh * W1); k.a2 = (T)(nh * W2);
  k.alpha = 1; k.gamma = 0; k.beta = 0;
  return k;
}

// Chebyshev step coefficients of every fragment for steps 1..degree (mode
// 1), one row of `degree` records per fragment, from the filter interval the
// last Rayleigh-Ritz step left in fs.  The recurrence s_k = 1/(2/s1 -
// s_{k-1}) runs once per fragment here instead of once per thread and step
// in the filter kernels, which read their step's record with a scalar load.
template <typename T>
__global__ __launch_bounds__(64) void k_step_coefs(
    const FilterState* __restrict__ fs, int nf, int degree, double nh,
    StepCoef<T>* __restrict__ coef) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= nf) return;
  const FilterState st = fs[j];
  StepCoef<T>* out = coef + (long long)j * degree;
  const double e = 0.5 * (st.upper - st.lower);
  if (!(e > 1e-12 * fabs(st.upper))) {   // degenerate interval: identity
    for (int k = 0; k < degree; ++k) {
      StepCoef<T> c;
      c.a1 = 0; c.a2 = 0; c.alpha = 0; c.gamma = 1; c.beta = 0;
      out[k] = c;
    }
    return;
  }
  const double c = 0.5 * (st.upper + st.lower);
  const double s1 = e / (st.scale - c);
  const double tau = 2.0 / s1;
  double sp = s1, sc = s1;
  for (int step = 1; step <= degree; ++step) {
    if (step >= 2) {
      sp = sc;
      sc = 1.0 / (tau - sp);
    }
    const double a = (step == 1 ? sc : 2.0 * sc) / e;
    StepCoef<T> k;
    k.a1 = (T)(a * nh * W1);
    k.a2 = (T)(a * nh * W2);
    k.alpha = (T)a;
    k.gamma = (T)(-c * a);
    k.beta = (T)(step == 1 ? 0.0 : -sp * sc);
    out[step - 1] = k;
  }
}

// diagonal of H_j at a point touching `nfaces` box faces with potential v
template <typename T>
__device__ __forceinline__ T point_diag(T nh, int nfaces, T v) {
  const T dg = fma(-(T)W2, T(nfaces), (T)W0 * T(3));
  return fma(nh, dg, v);
}

// One output point.  Every stencil kernel evaluates points through this
// function with explicit fused multiply-adds, so they all produce the same
// bits.
template <typename T>
__device__ __forceinline__ T stencil_point(T c, T s1, T s2, T u, T pn,
                                           const StepCoef<T>& k) {
  const T d = fma(k.alpha, u, k.gamma);
  return fma(k.a1, s1, fma(k.a2, s2, fma(d, c, k.beta * pn)));
}

template <typename T, int PPT>
__global__ __launch_bounds__(WG) void k_apply_h(
    const FragDev* __restrict__ F, const int2* __restrict__ tiles, int ntiles,
    int nblk_pad, const T* __restrict__ Vj, const T* __restrict__ in,
    const T* prev, T* out, const FilterState* __restrict__ fs,
    const StepCoef<T>* __restrict__ coef, int cdeg,
    const int* __restrict__ active, int step, int mode, double nh,
    long long base_override) {
  constexpr int SP = PPT * WG;
  constexpr int LW = SP + 4 * HALO_NX_MAX;
  const int t = xcd_tile(blockIdx.x, nblk_pad);
  if (t >= ntiles) return;
  const int j = tiles[t].x;
  const int v = tiles[t].y >> 16, strip = tiles[t].y & 0xffff;
  if (active && !active[j]) return;
  // converged leading Ritz vectors are locked: the filter leaves them as they
  // are (they stay in the orthogonalisation and the Rayleigh-Ritz step)
  if (mode == 1 && v < fs[j].lock) return;
  const FragDev& fr = F[j];
  const int nx = fr.dims[0], ny = fr.dims[1], nz = fr.dims[2];
  const int plane = nx * ny;
  const int p0 = strip * SP;
  const int p1 = min(p0 + SP, plane);
  const int h0 = max(p0 - 2 * nx, 0), h1 = min(p1 + 2 * nx, plane);
  const int nlo = p0 - h0, nhi = h1 - p1;
  const long long base =
      (base_override >= 0 ? base_override : fr.x_off) + (long long)v * fr.ld;
  const T* __restrict__ src = in + base;
  const T* pv = prev + base;
  T* dst = out + base;
  const T* __restrict__ vv = Vj + fr.v_off;

  const StepCoef<T> kc =
      mode == 0 ? h_coefs<T>(nh)
                : wave_uniform(coef[(long long)j * cdeg + step - 1]);
  const bool use_prev = (mode == 1 && step > 1);

  __shared__ T lds[2][LW];
  const int tid = threadIdx.x;
  int px[PPT], py[PPT], pp[PPT];
  bool ok[PPT];
  T q0[PPT], q1[PPT], q2[PPT], q3[PPT], q4[PPT], vn[PPT], pn[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int p = p0 + tid + k * WG;
    ok[k] = p < p1;
    pp[k] = ok[k] ? p : p0;
    px[k] = pp[k] % nx;
    py[k] = pp[k] / nx;
    q0[k] = 0;
    q1[k] = 0;
    q2[k] = ok[k] ? src[pp[k]] : T(0);
    q3[k] = (ok[k] && nz > 1) ? src[plane + pp[k]] : T(0);
    q4[k] = (ok[k] && nz > 2) ? src[2 * plane + pp[k]] : T(0);
    vn[k] = ok[k] ? vv[pp[k]] : T(0);
    pn[k] = (ok[k] && use_prev) ? pv[pp[k]] : T(0);
  }
  // halo slots (2 rows on each side of the strip): nlo + nhi <= 4 nx <= 2 WG
  int hq[2];
  bool hok[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int hidx = tid + u * WG;
    if (hidx < nlo) {
      hq[u] = h0 + hidx;
      hok[u] = true;
    } else if (hidx - nlo < nhi) {
      hq[u] = p1 + (hidx - nlo);
      hok[u] = true;
    } else {
      hq[u] = h0;
      hok[u] = false;
    }
  }
  const T tnh = (T)nh;
  for (int z = 0; z < nz; ++z) {
    const int zoff = z * plane;
    T nxt[PPT], vnx[PPT], pnx[PPT], hv[2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      nxt[k] = (ok[k] && z + 3 < nz) ? src[zoff + 3 * plane + pp[k]] : T(0);
      vnx[k] = (ok[k] && z + 1 < nz) ? vv[zoff + plane + pp[k]] : T(0);
      pnx[k] = (ok[k] && use_prev && z + 1 < nz)
                   ? __builtin_nontemporal_load(&pv[zoff + plane + pp[k]])
                   : T(0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) hv[u] = hok[u] ? src[zoff + hq[u]] : T(0);
    T* L = lds[z & 1];
#pragma unroll
    for (int k = 0; k < PPT; ++k)
      if (ok[k]) L[pp[k] - h0] = q2[k];
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (hok[u]) L[hq[u] - h0] = hv[u];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (!ok[k]) continue;
      const int li = pp[k] - h0, x = px[k], y = py[k];
      const T c = q2[k];
      const T xm1 = x >= 1 ? L[li - 1] : T(0);
      const T xm2 = x >= 2 ? L[li - 2] : T(0);
      const T xp1 = x + 1 < nx ? L[li + 1] : T(0);
      const T xp2 = x + 2 < nx ? L[li + 2] : T(0);
      const T ym1 = y >= 1 ? L[li - nx] : T(0);
      const T ym2 = y >= 2 ? L[li - 2 * nx] : T(0);
      const T yp1 = y + 1 < ny ? L[li + nx] : T(0);
      const T yp2 = y + 2 < ny ? L[li + 2 * nx] : T(0);
      // walls at every box face: odd image of the second ghost
      const int nfaces = (x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1) +
                         (z == 0) + (z == nz - 1);
      const T s1 = (xm1 + xp1) + (ym1 + yp1) + (q1[k] + q3[k]);
      const T s2 = (xm2 + xp2) + (ym2 + yp2) + (q0[k] + q4[k]);
      const T o = stencil_point<T>(c, s1, s2, point_diag<T>(tnh, nfaces, vn[k]),
                                   pn[k], kc);
      __builtin_nontemporal_store(o, &dst[zoff + pp[k]]);
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      q0[k] = q1[k];
      q1[k] = q2[k];
      q2[k] = q3[k];
      q3[k] = q4[k];
      q4[k] = nxt[k];
      vn[k] = vnx[k];
      pn[k] = pnx[k];
    }
  }
}

// ---------------------------------------------------------------------------
// NS Chebyshev steps per launch (boxes whose xy plane fits one workgroup)
// ---------------------------------------------------------------------------
// One workgroup per (fragment, vector) owns the whole box and marches along
// z.  At iteration t, stage s = 1..NS computes y_{k+s-1} at plane
// t - 2(s-1) from the outputs of stage s-1: their z neighbours ride in a
// register window of four planes plus the plane stage s-1 produced this
// iteration, their x/y neighbours come from LDS (the input plane t for
// stage 1, a ring of the last three planes of stage s-1 otherwise), and the
// point two steps back is the oldest plane of stage s-2's window (the y_{k-2}
// stream for stage 1).  HBM sees y_{k-1} and y_{k-2} read once and only the
// last two iterates written, per NS steps: 4 passes instead of 3 NS.  An
// iterate goes to the buffer of its parity (IN holds y_{k-1}, PV y_{k-2}),
// after each point's last read there, exactly as single-step launches leave
// it.  Points are evaluated by stencil_point in the same order as k_apply_h,
// so the results are bit-identical to NS single-step launches.  NS = 1
// (FP32) is the Rayleigh-Ritz product PV <- H_j IN over every vector
// (locked ones included), bit-identical to k_apply_h in mode 0.
#ifndef OFM_H2_THREADS
#define OFM_H2_THREADS 512
#endif
constexpr int H2T = OFM_H2_THREADS;   // threads of a multi-step workgroup
// Planes of 1025..2048 points run with 2 points per thread on 3 H2T / 2
// (up to 1536 points) or 2 H2T threads in FP64 and with 3..4 points per
// thread on H2T threads in FP32 (which also takes planes of 2049..3072
// points, 3 per thread on 2 H2T threads): on the amorphous workload (boxes of 24..40
// points per axis) the FP64 fragment stage measured 1386 against 1440 ms
// with the wide workgroups and the FP32 one 519 against 585 ms with the
// narrow ones; the 3 H2T / 2 class then took it from 1035 to 938 ms.
constexpr bool wide_wg(int elem_bytes) { return elem_bytes == 8; }

// LDS planes of the multi-step kernel: rows of nx + 2 values whose first two
// are zero, between two zero rows above and two below the box, so every +-1,
// +-2 neighbour beyond a face reads 0 without a test; hm_cap is the padded
// plane a launch of SP plane points holds (5/4 of SP: a 32 x 32 plane pads
// to 1224 of 1280; eight planes of NS = 3 fit the 160 KB of LDS of a CU)
constexpr int hm_padded(int nx, int ny) { return (ny + 4) * (nx + 2); }
// Global accesses of the multi-step kernel go through buffer resources
// sized to the vector (or to nothing), whose range check makes a load past
// the end return 0 and drops such a store: planes beyond the box, y_{k-2}
// on the first step of a filter and lanes past the plane need no branch and
// no select.  aux 2 marks an access non-temporal.
typedef unsigned int hm_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t hm_rsrc(const void* p,
                                                          unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes,
                                           0x00020000);
}
template <int AUX>
__device__ __forceinline__ double hm_load(__amdgpu_buffer_rsrc_t r, double,
                                          unsigned off) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ float hm_load(__amdgpu_buffer_rsrc_t r, float,
                                         unsigned off) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ void hm_store(double v, __amdgpu_buffer_rsrc_t r,
                                         unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(hm_u2, v), r, off,
                                        0, AUX);
}
template <int AUX>
__device__ __forceinline__ void hm_store(float v, __amdgpu_buffer_rsrc_t r,
                                         unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r,
                                        off, 0, AUX);
}
// byte offset that every buffer of the kernel rejects (boxes hold far fewer
// than 2^30 bytes per vector; plane offsets added to it stay below 2^32)
constexpr unsigned HM_OOB = 0x40000000u;
constexpr int hm_cap(int sp, int elem_bytes) {
  return sp + sp / 4 < 163840 / (8 * elem_bytes)
             ? sp + sp / 4
             : 163840 / (8 * elem_bytes);
}
// waves per SIMD the compiler must leave room for: the FP64 three-step
// form on 512 threads with 2 points each is held to 128 registers so that
// two of its workgroups share a CU (their LDS planes fit 160 KB together):
// 2.4% off the amorphous FP64 fragment stage
template <typename T, int PPT, int NS, int NT>
constexpr int hm_waves_per_eu() {
  return (sizeof(T) == 8 && NS == 3 && PPT == 2 && NT == 512) ? 4 : 1;
}

template <typename T, int PPT, int NS, int NT>
__global__ __launch_bounds__(NT) __attribute__((
    amdgpu_waves_per_eu(hm_waves_per_eu<T, PPT, NS, NT>()))) void k_apply_hm(
    const FragDev* __restrict__ F, const int2* __restrict__ tiles, int ntiles,
    int nblk_pad, const T* __restrict__ Vj, T* IN, T* PV,
    const FilterState* __restrict__ fs, const StepCoef<T>* __restrict__ coef,
    int cdeg, const int* __restrict__ active, int step, double nh) {
  static_assert(NS >= 1 && NS <= 3, "H y, or two or three steps per launch");
  constexpr int SP = PPT * NT;
  constexpr int CAP = hm_cap(SP, sizeof(T));
  // V at the planes of the NS stages: a register window of planes
  // t - 2(NS-1) .. t, or (FP64, three steps, 512 or 1024 threads, where the
  // window would not fit the 128 registers of the occupancy these launches
  // keep) V(t) alone with the other stages' planes read again from L2 at
  // every plane.  At 768 threads (three waves per SIMD, up to 168
  // registers) the window fits, and that class ran 1.2x faster per point
  // than the 1024-thread one with the reloads.
  constexpr bool VRELOAD = NS == 3 && sizeof(T) == 8 && NT % 512 == 0;
  constexpr int NV = VRELOAD ? 1 : 2 * (NS - 1) + 1;
  const int t0 = xcd_tile(blockIdx.x, nblk_pad);
  if (t0 >= ntiles) return;
  const int j = tiles[t0].x, v = tiles[t0].y;
  if (active && !active[j]) return;
  // the filter leaves locked Ritz vectors as they are
  if (NS > 1 && v < fs[j].lock) return;
  const FragDev& fr = F[j];
  const int nx = fr.dims[0], ny = fr.dims[1], nz = fr.dims[2];
  const int plane = nx * ny;
  // the host launches only boxes that fit
  if (plane > SP || hm_padded(nx, ny) > CAP) return;
  const int px = nx + 2;   // LDS row pitch
  const long long base = fr.x_off + (long long)v * fr.ld;
  T* in = IN + base;
  T* pv = PV + base;
  const T* __restrict__ vv = Vj + fr.v_off;
  const unsigned vbytes = (unsigned)fr.npts * sizeof(T);
  const unsigned pbytes = (unsigned)plane * sizeof(T);
  const __amdgpu_buffer_rsrc_t r_in = hm_rsrc(in, vbytes);
  const __amdgpu_buffer_rsrc_t r_pv = hm_rsrc(pv, vbytes);
  const __amdgpu_buffer_rsrc_t r_v = hm_rsrc(vv, vbytes);
  StepCoef<T> kc[NS];
  if constexpr (NS == 1) {
    kc[0] = h_coefs<T>(nh);
  } else {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      kc[s] = wave_uniform(coef[(long long)j * cdeg + step + s - 1]);
  }
  const bool use_prev = NS > 1 && step > 1;
  // y_{k-2} does not exist on the first step of a filter: every load of it
  // is out of range and returns 0
  const __amdgpu_buffer_rsrc_t r_q = hm_rsrc(pv, use_prev ? vbytes : 0u);
  const T tnh = (T)nh;
  // y_{k-1}, plane t (double-buffered); stage outputs, last three planes
  // (no stage output is read back when NS = 1)
  __shared__ T L0[2][CAP];
  __shared__ T R[NS > 1 ? NS - 1 : 1][NS > 1 ? 3 : 1][NS > 1 ? CAP : 1];
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * CAP; i += NT) (&L0[0][0])[i] = T(0);
  for (int i = tid; i < (NS - 1) * 3 * CAP; i += NT) (&R[0][0][0])[i] = T(0);
  __syncthreads();   // the zeros land before any interior write
  int pp[PPT];
  int lf[PPT];   // LDS index of the point | (box faces it touches in x, y) << 20
  unsigned po[PPT];   // byte offset of the point in a plane (HM_OOB: none)
  bool wl[PPT];       // the wave holds a point of the plane in slot k
  bool ok[PPT];
  T W[NS][4][PPT];   // stage s outputs at planes n_s-4..n_s-1, n_s = t-2(s-1)
                     // (stage 0: the input y_{k-1} at planes t-2..t+1)
  T nw0[PPT];        // input plane t+2
  T vq[NV][PPT];     // V at planes t-2(NS-1) .. t (t alone with VRELOAD)
  T q[PPT];          // y_{k-2} at plane t
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int p = tid + k * NT;
    ok[k] = p < plane;
    pp[k] = ok[k] ? p : 0;   // lanes past the plane work on point 0 and
                             // store nothing
    const int x = pp[k] % nx, y = pp[k] / nx;
    lf[k] = ((y + 2) * px + x + 2) |
            (((x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1)) << 20);
    po[k] = ok[k] ? (unsigned)pp[k] * sizeof(T) : HM_OOB;
    wl[k] = __builtin_amdgcn_readfirstlane((tid & ~63) + k * NT < plane);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) W[s][i][k] = 0;
    W[0][2][k] = hm_load<0>(r_in, T(), po[k]);
    W[0][3][k] = hm_load<0>(r_in, T(), po[k] + pbytes);
    nw0[k] = hm_load<0>(r_in, T(), po[k] + 2 * pbytes);
#pragma unroll
    for (int i = 0; i < NV - 1; ++i) vq[i][k] = 0;
    vq[NV - 1][k] = hm_load<0>(r_v, T(), po[k]);
    q[k] = hm_load<0>(r_q, T(), po[k]);
  }
  // the point's LDS index; LDS writes of lanes past the plane go to element
  // 0, a pad that no point reads (the first two elements of the top zero
  // row), so every lane computes and writes and no branch hides a store
  auto li_of = [&](int k) { return lf[k] & 0xfffff; };
  auto wi_of = [&](int k) { return ok[k] ? (lf[k] & 0xfffff) : 0; };
  // One z plane.  Loads are issued for every lane at clamped addresses and
  // the unwanted values replaced by 0, and in the steady state (every stage
  // on a plane of the box) no branch depends on the plane, so the wait for
  // a plane's loads does not also wait for the stores issued after them.
  auto iter = [&](int t, auto steady_c) {
    constexpr bool STEADY = decltype(steady_c)::value;
    T an[PPT], vn[PPT], qn[PPT];
    T vs[NS][PPT];   // VRELOAD: V at stage s's plane t - 2(s-1), s >= 2
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      // the input and y_{k-2} streams are read once (non-temporal, leaving
      // L2 to V_j, which the box's other vectors read again); planes past
      // the box (and before it) read 0
      if (VRELOAD)
#pragma unroll
        for (int s = 2; s <= NS; ++s)
          vs[s - 1][k] =
              hm_load<0>(r_v, T(), po[k] + (unsigned)(t - 2 * (s - 1)) * pbytes);
      an[k] = hm_load<2>(r_in, T(), po[k] + (unsigned)(t + 3) * pbytes);
      vn[k] = hm_load<0>(r_v, T(), po[k] + (unsigned)(t + 1) * pbytes);
      qn[k] = hm_load<2>(r_q, T(), po[k] + (unsigned)(t + 1) * pbytes);
      if (STEADY || t < nz) L0[t & 1][wi_of(k)] = W[0][2][k];
    }
    __syncthreads();
    T nw[NS + 1][PPT];   // nw[s]: stage s output at plane n_s
#pragma unroll
    for (int k = 0; k < PPT; ++k) nw[0][k] = nw0[k];
#pragma unroll
    for (int s = 1; s <= NS; ++s) {
      const int z = t - 2 * (s - 1);
      const bool live = STEADY || (z >= 0 && z < nz);
      const T* L = s == 1 ? L0[t & 1] : R[s >= 2 ? s - 2 : 0][live ? z % 3 : 0];
      const int nfz = (z == 0) + (z == nz - 1);
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        nw[s][k] = 0;
        if (!live) continue;
        // waves with no point of the plane in this slot skip the arithmetic
        // (a scalar branch); their stores below go out of range and their
        // LDS writes to the dead pad element.  Their value is a sum of this
        // plane's inputs, so that no load is needed only inside the branch
        // (a load sunk into it would make the wait counts path-dependent,
        // and every plane would then wait for the stores issued after its
        // loads).
        const T vz = (VRELOAD && s >= 2) ? vs[s - 1][k]
                                         : vq[VRELOAD ? 0 : NV - 1 - 2 * (s - 1)][k];
        T o = W[s - 1][2][k] + (vz + q[k]);
        if (wl[k]) {
          const int c0 = li_of(k);
          const T xm1 = L[c0 - 1], xm2 = L[c0 - 2];
          const T xp1 = L[c0 + 1], xp2 = L[c0 + 2];
          const T ym1 = L[c0 - px], ym2 = L[c0 - 2 * px];
          const T yp1 = L[c0 + px], yp2 = L[c0 + 2 * px];
          const T s1 = (xm1 + xp1) + (ym1 + yp1) + (W[s - 1][1][k] + W[s - 1][3][k]);
          const T s2 = (xm2 + xp2) + (ym2 + yp2) + (W[s - 1][0][k] + nw[s - 1][k]);
          const T pn = s == 1 ? q[k] : W[s >= 2 ? s - 2 : 0][0][k];
          o = stencil_point<T>(
              W[s - 1][2][k], s1, s2,
              point_diag<T>(tnh, (lf[k] >> 20) + nfz, vz), pn,
              kc[s - 1]);
        }
        if (s >= NS - 1)   // the last two iterates go to HBM
          hm_store<2>(o, (s % 2 == 0) ? r_in : r_pv,
                      po[k] + (unsigned)z * pbytes);
        if (NS > 1 && s <= NS - 1) R[s - 1][z % 3][wi_of(k)] = o;
        nw[s][k] = o;
      }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        W[s][0][k] = W[s][1][k];
        W[s][1][k] = W[s][2][k];
        W[s][2][k] = W[s][3][k];
        W[s][3][k] = nw[s][k];
      }
      nw0[k] = an[k];
#pragma unroll
      for (int i = 0; i < NV - 1; ++i) vq[i][k] = vq[i + 1][k];
      vq[NV - 1][k] = vn[k];
      q[k] = qn[k];
    }
  };
  // planes [s_lo, s_hi) are steady: every stage lies inside the box; the
  // three loops keep the steady one free of the edge tests
  const int t_end = nz + 2 * (NS - 1);
  const int s_lo = min(2 * (NS - 1), nz), s_hi = nz;
  int t = 0;
  for (; t < s_lo; ++t) iter(t, std::integral_constant<bool, false>{});
  for (; t < s_hi; ++t) iter(t, std::integral_constant<bool, true>{});
  for (; t < t_end; ++t) iter(t, std::integral_constant<bool, false>{});
}

// boxes the multi-step kernel takes: planes that fit one of its launch
// classes (a box runs in the launch of its own class of points per thread, so
// only the large planes pay the larger register windows; on the amorphous
// workload FP64 planes of 1025..1600 points ran 6% faster overall in
// multi-step classes than in one-step strips)
bool multistep_eligible(int elem_bytes, const FragDev& d) {
  return multistep_class(elem_bytes, d) > 0;
}

// launch class of the multi-step kernel for a box (0: not taken): the first
// whose plane (SP points) and padded LDS plane (hm_cap) hold the box's.  The
// classes hold planes of up to cl H2T points, cl = 1..4, as (points per
// thread, threads) 1: (1, H2T), 2: (2, H2T), and with wide workgroups
// 3: (2, 3 H2T / 2) and 4: (2, 2 H2T), else 3: (3, H2T) and 4: (4, H2T);
// FP32 adds class 5, planes of up to 6 H2T points as (3, 2 H2T)
int multistep_class(int elem_bytes, const FragDev& d) {
  const int plane = d.dims[0] * d.dims[1];
  const int padded = hm_padded(d.dims[0], d.dims[1]);
  const int ncls = wide_wg(elem_bytes) ? 4 : 5;
  for (int cl = 1; cl <= ncls; ++cl) {
    const int sp = cl == 5 ? 6 * H2T : cl * H2T;
    if (plane <= sp && padded <= hm_cap(sp, elem_bytes)) return cl;
  }
  return 0;
}



template <typename T>
void apply_hm(ofm_ctx* c, const ofm_frags* f, T* IN, T* PV, const int2* tiles,
              int ntiles, int cls, int ns, const int* active, int step,
              const FilterState* fs, const void* coef, int cdeg,
              double alg_bytes, double flops) {
  const T* Vj;
  if constexpr (sizeof(T) == 8)
    Vj = (const T*)f->d_vf;
  else
    Vj = (const T*)f->d_vf32;
  const double nh = -0.5 / (f->grid.h * f->grid.h);
  const int nblk = pad8(ntiles);
  // the H X launches (ns = 1) are booked with the other H X launches
  Timed tm(c, ns == 1 ? "stencil" : "multistep", alg_bytes, flops);
  hipStream_t stream = f->ctx->stream;
#define LAUNCHM(PP, NSS, NTT)                                                \
  hipLaunchKernelGGL((k_apply_hm<T, PP, NSS, NTT>), dim3(nblk), dim3(NTT), 0, \
                     stream, f->d_frag, tiles, ntiles, nblk, Vj, IN, PV, fs, \
                     (const StepCoef<T>*)coef, cdeg, active, step, nh)
#define LAUNCHP(PP, NTT)                                                     \
  do {                                                                       \
    if (ns == 3) LAUNCHM(PP, 3, NTT);                                        \
    else if (ns == 2) LAUNCHM(PP, 2, NTT);                                   \
    else if constexpr (sizeof(T) == 4) LAUNCHM(PP, 1, NTT);                  \
    else OFM_REQUIRE(false, OFM_E_INVALID, "H X form is FP32 only");         \
  } while (0)
  // the classes of multistep_class
  OFM_REQUIRE(cls >= 1 && cls <= (wide_wg(sizeof(T)) ? 4 : 5), OFM_E_INVALID,
              "unknown multi-step launch class");
  if (cls == 1) {
    LAUNCHP(1, H2T);
  } else if (cls == 2) {
    LAUNCHP(2, H2T);
  } else if constexpr (wide_wg(sizeof(T))) {
    if (cls == 3) LAUNCHP(2, 3 * H2T / 2);
    else LAUNCHP(2, 2 * H2T);
  } else {
    if (cls == 3) LAUNCHP(3, H2T);
    else if (cls == 4) LAUNCHP(4, H2T);
    else LAUNCHP(3, 2 * H2T);
  }
#undef LAUNCHP
#undef LAUNCHM
  OFM_HIP(hipGetLastError());
}
template void apply_hm<double>(ofm_ctx*, const ofm_frags*, double*, double*,
                               const int2*, int, int, int, const int*, int,
                               const FilterState*, const void*, int, double,
                               double);
template void apply_hm<float>(ofm_ctx*, const ofm_frags*, float*, float*,
                              const int2*, int, int, int, const int*, int,
                              const FilterState*, const void*, int, double,
                              double);

// ---------------------------------------------------------------------------
// whole Chebyshev filter with the vector resident on chip (FP32 boxes of at
// most 32 x 32 x 32 points)
// ---------------------------------------------------------------------------
// One workgroup of 1024 threads per (fragment, vector) runs every filter
// step.  y_{k-1} of the whole box sits in LDS in a zero-padded layout (two
// zero columns between rows, two zero rows between planes, zero planes
// beyond the box), so every +-1, +-2 neighbour beyond a box face reads 0
// without a test.  Thread (x, y) owns the z column at that plane point and
// keeps y_{k-2} and the point diagonals u of its column in registers.  After
// each step's barrier a thread swaps its own column: LDS takes y_k, the
// registers take y_{k-1}.  HBM is touched once per filter (read y_0 and V,
// write y_d) instead of once per step.  Points are evaluated by
// stencil_point exactly as in the strip kernel, so the filtered vectors are
// bit-identical to `degree` strip launches.
constexpr int RN = 32;
constexpr int RX = RN + 2;          // LDS row pitch
constexpr int RPL = RX * (RN + 2);  // LDS plane pitch
constexpr int RLDS = RN * RPL + 2 * RX;

// LDS index of box point (x, y, z)
__device__ __forceinline__ int rl(int x, int y, int z) {
  return z * RPL + (y + 2) * RX + (x + 2);
}

// one filter step over the own column; FULLZ: the box spans all RN planes
template <bool FULLZ>
__device__ __forceinline__ void resident_step(float (&old)[RN],
                                              const float (&u)[RN], float* L,
                                              int a0, bool own, int nz,
                                              const StepCoef<float>& kc) {
  // 5-deep window of the own column of y_{k-1}, streamed from LDS (planes
  // beyond the box are zero)
  float q0 = 0.f, q1 = 0.f;
  float q2 = L[a0], q3 = L[a0 + RPL], q4 = L[a0 + 2 * RPL];
#pragma unroll
  for (int z = 0; z < RN; ++z) {
    if (FULLZ || z < nz) {
      const int a = a0 + z * RPL;
      const float nxt = z + 3 < RN ? L[a0 + (z + 3 < RN ? z + 3 : 0) * RPL]
                                   : 0.f;
      const float s1 = (L[a - 1] + L[a + 1]) + (L[a - RX] + L[a + RX]) +
                       (q1 + q3);
      const float s2 = (L[a - 2] + L[a + 2]) +
                       (L[a - 2 * RX] + L[a + 2 * RX]) + (q0 + q4);
      old[z] = stencil_point<float>(q2, s1, s2, u[z], old[z], kc);
      q0 = q1;
      q1 = q2;
      q2 = q3;
      q3 = q4;
      q4 = nxt;
    }
  }
  __syncthreads();   // every read of y_{k-1} in LDS is done
  if (own) {
#pragma unroll
    for (int z = 0; z < RN; ++z)
      if (FULLZ || z < nz) {
        const float prev = L[a0 + z * RPL];
        L[a0 + z * RPL] = old[z];
        old[z] = prev;
      }
  }
  __syncthreads();
}

template <bool FULLZ>
__device__ __forceinline__ void resident_filter(float* L, float (&old)[RN],
                                                const float (&u)[RN], int a0,
                                                bool own, int nz,
                                                const StepCoef<float>* coef,
                                                int degree) {
  for (int step = 1; step <= degree; ++step) {
    const StepCoef<float> kc = wave_uniform(coef[step - 1]);
    int nzs = nz;
    asm volatile("" : "+s"(nzs));   // keep per-plane tests inside the step
    resident_step<FULLZ>(old, u, L, a0, own, nzs, kc);
  }
}

__global__ __launch_bounds__(RN * RN) void k_filter_resident(
    const FragDev* __restrict__ F, const int2* __restrict__ tiles, int ntiles,
    int nblk_pad, const float* __restrict__ Vj, float* X,
    const FilterState* __restrict__ fs,
    const StepCoef<float>* __restrict__ coef, const int* __restrict__ active,
    int degree, double nh) {
  const int t = xcd_tile(blockIdx.x, nblk_pad);
  if (t >= ntiles) return;
  const int j = tiles[t].x, v = tiles[t].y;
  if (active && !active[j]) return;
  if (v < fs[j].lock) return;   // locked Ritz vectors are left as they are
  const FragDev& fr = F[j];
  const int nx = fr.dims[0], ny = fr.dims[1], nz = fr.dims[2];
  const int plane = nx * ny;
  const int tid = threadIdx.x;
  const int x = tid % RN, y = tid / RN;
  const bool own = x < nx && y < ny;
  const int p = own ? x + nx * y : 0;
  float* col = X + fr.x_off + (long long)v * fr.ld + p;
  const float* vc = Vj + fr.v_off + p;
  __shared__ float L[RLDS];
  for (int i = tid; i < RLDS; i += RN * RN) L[i] = 0.f;
  __syncthreads();
  const int a0 = rl(x, y, 0);
  const int nfxy = (x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1);
  const float tnh = (float)nh;
  float old[RN], u[RN];   // y_{k-2} (zero before the first step), diagonals
#pragma unroll
  for (int z = 0; z < RN; ++z) {
    old[z] = 0.f;
    u[z] = 0.f;
    if (own && z < nz) {
      u[z] = point_diag<float>(tnh, nfxy + (z == 0) + (z == nz - 1),
                               vc[z * plane]);
      L[a0 + z * RPL] = col[z * plane];
    }
  }
  __syncthreads();
  const StepCoef<float>* cj = coef + (long long)j * degree;
  if (nz == RN)
    resident_filter<true>(L, old, u, a0, own, nz, cj, degree);
  else
    resident_filter<false>(L, old, u, a0, own, nz, cj, degree);
#pragma unroll
  for (int z = 0; z < RN; ++z)
    if (own && z < nz)
      __builtin_nontemporal_store(L[a0 + z * RPL], &col[z * plane]);
}

bool resident_eligible(int elem_bytes, const FragDev& d) {
  return elem_bytes == 4 && d.dims[0] <= RN && d.dims[1] <= RN &&
         d.dims[2] <= RN;
}

void filter_resident(ofm_ctx* c, const ofm_frags* f, float* X,
                     const int2* tiles, int ntiles, const int* active,
                     const FilterState* fs, const void* coef, int degree,
                     double alg_bytes, double flops) {
  const int nblk = pad8(ntiles);
  Timed tm(c, "filter", alg_bytes, flops);
  hipLaunchKernelGGL(k_filter_resident, dim3(nblk), dim3(RN * RN), 0,
                     f->ctx->stream, f->d_frag, tiles, ntiles, nblk,
                     (const float*)f->d_vf32, X, fs,
                     (const StepCoef<float>*)coef, active, degree,
                     -0.5 / (f->grid.h * f->grid.h));
  OFM_HIP(hipGetLastError());
}

// PPT of stencil variant i for storage type T
int stencil_ppt(int elem_bytes, int variant) {
  static const int p64[NVARIANT] = {1, 2, 4};
  static const int p32[NVARIANT] = {2, 4, 8};
  return elem_bytes == 8 ? p64[variant] : p32[variant];
}

// tiles (fragment, vector << 16 | strip) of one stencil variant for the
// vectors v < nvec(j) of every fragment (or of fragment `only` alone)
std::vector<int2> stencil_tiles(const ofm_frags* f, int elem_bytes,
                                int variant, int nvec_only, int only,
                                const std::vector<char>* keep) {
  const int sp = stencil_ppt(elem_bytes, variant) * WG;
  std::vector<int2> t;
  for (int j = 0; j < f->n_frag; ++j) {
    if (only >= 0 && j != only) continue;
    const FragDev& d = f->host[j];
    if (keep && !(*keep)[j]) continue;
    const int ns = (d.dims[0] * d.dims[1] + sp - 1) / sp;
    const int nv = nvec_only > 0 ? nvec_only : d.bw;
    for (int v = 0; v < nv; ++v)
      for (int s = 0; s < ns; ++s) t.push_back(make_int2(j, (v << 16) | s));
  }
  return t;
}

template <typename T>
void apply_h(ofm_ctx* c, const ofm_frags* f, const T* in, const T* prev,
             T* out, const int2* tiles, int ntiles, int variant,
             const int* active, int step, const FilterState* fs,
             const void* coef, int cdeg, int mode, long long base_override,
             double alg_bytes, double flops, hipEvent_t ev0, hipEvent_t ev1) {
  const T* Vj;   // potential of the fragment Hamiltonians
  if constexpr (sizeof(T) == 8)
    Vj = (const T*)f->d_vf;
  else
    Vj = (const T*)f->d_vf32;
  const double nh = -0.5 / (f->grid.h * f->grid.h);
  const int nblk = pad8(ntiles);
  Timed tm(c, "stencil", alg_bytes, flops);
  hipStream_t stream = f->ctx->stream;
  if (ev0) OFM_HIP(hipEventRecord(ev0, stream));
  const int ppt = stencil_ppt(sizeof(T), variant);
#define LAUNCH(P)                                                            \
  hipLaunchKernelGGL((k_apply_h<T, P>), dim3(nblk), dim3(WG), 0, stream,     \
                     f->d_frag, tiles, ntiles, nblk, Vj, in, prev, out, fs,  \
                     (const StepCoef<T>*)coef, cdeg, active, step, mode, nh, \
                     base_override)
  if (ppt == 1) LAUNCH(1);
  else if (ppt == 2) LAUNCH(2);
  else if (ppt == 4) LAUNCH(4);
  else LAUNCH(8);
#undef LAUNCH
  if (ev1) OFM_HIP(hipEventRecord(ev1, stream));
  OFM_HIP(hipGetLastError());
}
template void apply_h<double>(ofm_ctx*, const ofm_frags*, const double*,
                              const double*, double*, const int2*, int, int,
                              const int*, int, const FilterState*,
                              const void*, int, int, long long, double,
                              double, hipEvent_t, hipEvent_t);
template void apply_h<float>(ofm_ctx*, const ofm_frags*, const float*,
                             const float*, float*, const int2*, int, int,
                             const int*, int, const FilterState*, const void*,
                             int, int, long long, double, double, hipEvent_t,
                             hipEvent_t);

template <typename T>
void step_coefs_table(hipStream_t s, const ofm_frags* f, int degree,
                      void* table) {
  hipLaunchKernelGGL(k_step_coefs<T>, dim3((f->n_frag + 63) / 64), dim3(64),
                     0, s, f->d_fs, f->n_frag, degree,
                     -0.5 / (f->grid.h * f->grid.h), (StepCoef<T>*)table);
  OFM_HIP(hipGetLastError());
}
template void step_coefs_table<double>(hipStream_t, const ofm_frags*, int,
                                       void*);
template void step_coefs_table<float>(hipStream_t, const ofm_frags*, int,
                                      void*);

}  // namespace k
}  // namespace ofm
