// Fragment Hamiltonian stencil for gfx950 (MI355X, CDNA4): H_j = -1/2 Lap
// + V_j on a box with image-ghost Dirichlet walls (4th-order central
// differences), and the scaled three-term Chebyshev step built on it.
#include <hip/hip_runtime.h>

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

// Coefficients (alpha, gamma, beta) of Chebyshev step `step`:
// out = alpha H y_{k-1} + gamma y_{k-1} + beta y_{k-2}.  A degenerate
// interval gives the identity.
template <typename T>
__device__ __forceinline__ void cheb_coefs(const FilterState& st, int step,
                                           T& alpha, T& gamma, T& beta) {
  const double e = 0.5 * (st.upper - st.lower);
  if (!(e > 1e-12 * fabs(st.upper))) {
    alpha = 0; gamma = 1; beta = 0;
    return;
  }
  const double c = 0.5 * (st.upper + st.lower);
  const double s1 = e / (st.scale - c);
  double sp = s1, sc = s1;
  const double tau = 2.0 / s1;
  for (int k = 2; k <= step; ++k) {
    sp = sc;
    sc = 1.0 / (tau - sp);
  }
  const double a = (step == 1 ? sc : 2.0 * sc) / e;
  alpha = (T)a;
  gamma = (T)(-c * a);
  beta = (T)(step == 1 ? 0.0 : -sp * sc);
}

// One output point: H_j y at a point whose value is c, from its +-1 and +-2
// neighbours along each axis (0 beyond the box faces) and the number of box
// faces it touches (each adds the odd image of the second ghost), then the
// Chebyshev update (mode 1) or H_j y itself (mode 0).  Every stencil kernel
// evaluates points through this function with explicit fused multiply-adds,
// so they all produce the same bits.
template <typename T>
__device__ __forceinline__ T stencil_point(T c, T s1, T s2, int nfaces, T v,
                                           T pn, T nh, T alpha, T gamma,
                                           T beta, int mode) {
  const T dg = fma(-(T)W2, T(nfaces), (T)W0 * T(3));
  const T lap = fma((T)W1, s1, fma((T)W2, s2, dg * c));
  const T hval = fma(nh, lap, v * c);
  return mode == 0 ? hval : fma(alpha, hval, fma(gamma, c, beta * pn));
}

template <typename T, int PPT>
__global__ __launch_bounds__(WG) void k_apply_h(
    const FragDev* __restrict__ F, const int2* __restrict__ tiles, int ntiles,
    int nblk_pad, const T* __restrict__ Vj, const T* __restrict__ in,
    const T* prev, T* out, const FilterState* __restrict__ fs,
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

  T alpha = 1, gamma = 0, beta = 0;
  if (mode == 1) cheb_coefs<T>(fs[j], step, alpha, gamma, beta);
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
      const T o = stencil_point<T>(c, s1, s2, nfaces, vn[k], pn[k], tnh,
                                   alpha, gamma, beta, mode);
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
// whole Chebyshev filter with the vector resident on chip (FP32 boxes of at
// most 32 x 32 x 32 points)
// ---------------------------------------------------------------------------
// One workgroup of 1024 threads per (fragment, vector) runs every filter
// step: y_{k-1} of the whole box (128 KB) sits in LDS, thread (x, y) owns
// the z column at that plane point and keeps y_{k-2} and V_j of its column
// in registers.  After each step's barrier a thread swaps
// its own column: LDS takes y_k, the registers take y_{k-1}.  HBM is touched
// once per filter (read y_0 and V, write y_d) instead of once per step.
// Points are evaluated by stencil_point in the same order as the strip
// kernel, so the filtered vectors are bit-identical to `degree` strip
// launches.
constexpr int RN = 32;
constexpr int RP = RN * RN;        // LDS plane pitch
constexpr int RPAD = 2 * RN + 2;   // LDS pad below and above the box: every
                                   // neighbour address stays in the array
#ifndef OFM_RZG
#define OFM_RZG 1
#endif
constexpr int RZG = OFM_RZG;       // planes per scheduling group

__device__ __forceinline__ void resident_step(
    float (&old)[RN], float* L, int li0, bool own, int nz, int nfxy,
    bool xm1ok, bool xm2ok, bool xp1ok, bool xp2ok, bool ym1ok, bool ym2ok,
    bool yp1ok, bool yp2ok, const float (&vr)[RN], float nh, float alpha,
    float gamma, float beta) {
  // Neighbour values are loaded unconditionally (all addresses lie inside
  // the padded array) and selected to 0 beyond the box faces; lanes outside
  // the box and planes z >= nz compute values nobody reads (the planes
  // beyond the box are only ever selected away), so the whole step is one
  // straight-line block.
  // 5-deep window of the own column of y_{k-1}, streamed from LDS
  float q0 = 0.f, q1 = 0.f;
  const float r3 = L[li0 + RP], r4 = L[li0 + 2 * RP];
  float q2 = L[li0];
  float q3 = nz > 1 ? r3 : 0.f;
  float q4 = nz > 2 ? r4 : 0.f;
#pragma unroll
  for (int z = 0; z < RN; ++z) {
    {
      const int li = li0 + z * RP;
      float nxt = 0.f;
      if (z + 3 < RN) {
        const float r = L[li0 + (z + 3 < RN ? z + 3 : 0) * RP];
        nxt = z + 3 < nz ? r : 0.f;
      }
      const float rxm1 = L[li - 1], rxm2 = L[li - 2];
      const float rxp1 = L[li + 1], rxp2 = L[li + 2];
      const float rym1 = L[li - RN], rym2 = L[li - 2 * RN];
      const float ryp1 = L[li + RN], ryp2 = L[li + 2 * RN];
      const float xm1 = xm1ok ? rxm1 : 0.f, xm2 = xm2ok ? rxm2 : 0.f;
      const float xp1 = xp1ok ? rxp1 : 0.f, xp2 = xp2ok ? rxp2 : 0.f;
      const float ym1 = ym1ok ? rym1 : 0.f, ym2 = ym2ok ? rym2 : 0.f;
      const float yp1 = yp1ok ? ryp1 : 0.f, yp2 = yp2ok ? ryp2 : 0.f;
      const int nfaces = nfxy + (z == 0) + (z == nz - 1);
      const float s1 = (xm1 + xp1) + (ym1 + yp1) + (q1 + q3);
      const float s2 = (xm2 + xp2) + (ym2 + yp2) + (q0 + q4);
      old[z] = stencil_point<float>(q2, s1, s2, nfaces, vr[z], old[z], nh,
                                    alpha, gamma, beta, 1);
      q0 = q1;
      q1 = q2;
      q2 = q3;
      q3 = q4;
      q4 = nxt;
    }
    // keep the scheduler from hoisting loads of later planes (registers)
    if ((z & (RZG - 1)) == RZG - 1) __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();   // every read of y_{k-1} in LDS is done
#pragma unroll
  for (int z = 0; z < RN; ++z) {
      const float prev = L[li0 + z * RP];
      L[li0 + z * RP] = old[z];
      old[z] = prev;
    }
  __syncthreads();
}

__global__ __launch_bounds__(RP) void k_filter_resident(
    const FragDev* __restrict__ F, const int2* __restrict__ tiles, int ntiles,
    int nblk_pad, const float* __restrict__ Vj, float* X,
    const FilterState* __restrict__ fs, const int* __restrict__ active,
    int degree, double nh) {
  const int t = xcd_tile(blockIdx.x, nblk_pad);
  if (t >= ntiles) return;
  const int j = tiles[t].x, v = tiles[t].y;
  if (active && !active[j]) return;
  const FilterState st = fs[j];
  if (v < st.lock) return;   // locked Ritz vectors are left as they are
  const FragDev& fr = F[j];
  const int nx = fr.dims[0], ny = fr.dims[1], nz = fr.dims[2];
  const int plane = nx * ny;
  const int tid = threadIdx.x;
  const int x = tid % RN, y = tid / RN;
  const bool own = x < nx && y < ny;
  const int p = own ? x + nx * y : 0;
  float* col = X + fr.x_off + (long long)v * fr.ld + p;
  const float* vc = Vj + fr.v_off + p;
  __shared__ float Lbuf[RPAD + RN * RP + RPAD];
  float* L = Lbuf + RPAD;
  const int li0 = y * RN + x;
  float old[RN], vr[RN];   // y_{k-2} (zero before the first step), V_j
#pragma unroll
  for (int z = 0; z < RN; ++z) {
    old[z] = 0.f;
    vr[z] = (own && z < nz) ? vc[z * plane] : 0.f;
    if (own && z < nz) L[li0 + z * RP] = col[z * plane];
  }
  __syncthreads();
  const int nfxy = (x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1);
  const bool xm1ok = x >= 1, xm2ok = x >= 2, xp1ok = x + 1 < nx,
             xp2ok = x + 2 < nx;
  const bool ym1ok = y >= 1, ym2ok = y >= 2, yp1ok = y + 1 < ny,
             yp2ok = y + 2 < ny;
  const float tnh = (float)nh;
  for (int step = 1; step <= degree; ++step) {
    float al, ga, be;
    cheb_coefs<float>(st, step, al, ga, be);
    // the per-plane tests on nz are recomputed inside each step rather than
    // hoisted out of the step loop as 32 lane masks (register pressure)
    int nzs = nz;
    asm volatile("" : "+s"(nzs));
    resident_step(old, L, li0, own, nzs, nfxy, xm1ok, xm2ok, xp1ok, xp2ok,
                  ym1ok, ym2ok, yp1ok, yp2ok, vr, tnh, al, ga, be);
  }
#pragma unroll
  for (int z = 0; z < RN; ++z)
    if (own && z < nz)
      __builtin_nontemporal_store(L[li0 + z * RP], &col[z * plane]);
}

bool resident_eligible(int elem_bytes, const FragDev& d) {
  return elem_bytes == 4 && d.dims[0] <= RN && d.dims[1] <= RN &&
         d.dims[2] <= RN;
}

void filter_resident(ofm_ctx* c, const ofm_frags* f, float* X,
                     const int2* tiles, int ntiles, const int* active,
                     const FilterState* fs, int degree, double alg_bytes,
                     double flops) {
  const int nblk = pad8(ntiles);
  Timed tm(c, "filter", alg_bytes, flops);
  hipLaunchKernelGGL(k_filter_resident, dim3(nblk), dim3(RP), 0,
                     f->ctx->stream, f->d_frag, tiles, ntiles, nblk,
                     (const float*)f->d_vf32, X, fs, active, degree,
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
                                bool skip_resident) {
  const int sp = stencil_ppt(elem_bytes, variant) * WG;
  std::vector<int2> t;
  for (int j = 0; j < f->n_frag; ++j) {
    if (only >= 0 && j != only) continue;
    const FragDev& d = f->host[j];
    if (skip_resident && resident_eligible(elem_bytes, d)) continue;
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
             const int* active, int step, const FilterState* fs, int mode,
             long long base_override, double alg_bytes, double flops,
             hipEvent_t ev0, hipEvent_t ev1) {
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
                     active, step, mode, nh, base_override)
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
                              const int*, int, const FilterState*, int,
                              long long, double, double, hipEvent_t,
                              hipEvent_t);
template void apply_h<float>(ofm_ctx*, const ofm_frags*, const float*,
                             const float*, float*, const int2*, int, int,
                             const int*, int, const FilterState*, int,
                             long long, double, double, hipEvent_t,
                             hipEvent_t);

}  // namespace k
}  // namespace ofm
