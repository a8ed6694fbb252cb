// C ABI of the OFM library: argument checking, device arenas and the host
// loop of the batched fragment eigensolver.
//
// Fragment eigensolver (method Sec. II: every fragment Hamiltonian is
// diagonalised for its lowest states; Sec. III-B: the lowest s_j states form
// the basis).  All fragments advance together through one batched
// Chebyshev-filtered block subspace iteration:
//   X <- p_d(H_j) X          (degree-d scaled Chebyshev filter damping
//                             [theta_b, lambda_max], every fragment at once)
//   X <- X R1^-1; R2 from X^T X  (CholQR2, FP64 Cholesky of the Gram
//                                 matrices; R2 is not applied separately)
//   HX <- H_j X; G = R2^-T X^T HX R2^-1 = Y Theta Y^T  (Rayleigh-Ritz, FP64
//                                 Jacobi)
//   X <- X R2^-1 Y, HX <- HX R2^-1 Y, r_i = ||HX_i - theta_i X_i||
// until every wanted residual is below tol; a converged fragment drops out
// of all later launches.  The Chebyshev filter plays the role of the
// preconditioner of a block-Davidson correction step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "ofm_internal.h"

using namespace ofm;

std::shared_mutex& ofm::capture_lock() {
  static std::shared_mutex m;
  return m;
}

namespace {

const char* kVersion = "ofm-mi355x 0.1 (gfx950)";
thread_local std::string g_create_err;

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void set_err(ofm_ctx* c, const std::string& m) {
  if (c)
    c->err = m;
  else
    g_create_err = m;
}

template <typename F>
ofm_status guarded(ofm_ctx* c, F&& fn) {
  try {
    if (c) c->err.clear();
    return fn();
  } catch (const Error& e) {
    set_err(c, e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_err(c, "host allocation failed");
    return OFM_E_NOMEM;
  } catch (const std::exception& e) {
    set_err(c, e.what());
    return OFM_E_INVALID;
  }
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

void use_device(ofm_ctx* c) { OFM_HIP(hipSetDevice(c->device)); }

size_t wsize(const ofm_ctx* c) { return c->precision == OFM_FP64 ? 8 : 4; }

}  // namespace

// --------------------------------------------------------------------------
// timing brackets
// --------------------------------------------------------------------------
namespace ofm {
Timed::Timed(ofm_ctx* ctx, const char* family, double by, double fl, int n)
    : c(ctx), fam(family), bytes(by), flops(fl), launches(n) {
  if (!c || !c->profiling) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, c->stream);
}
Timed::~Timed() {
  if (!a) return;
  (void)hipEventRecord(b, c->stream);
  c->pending.push_back({fam, a, b, bytes, flops, launches});
}
void collect_stats(ofm_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& s = c->stats[p.fam];
      s.launches += p.launches;
      s.ms += ms;
      s.bytes += p.bytes;
      s.flops += p.flops;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->pending.clear();
}
}  // namespace ofm

// --------------------------------------------------------------------------
// V statistics per box: max (filter bound) and finiteness
// --------------------------------------------------------------------------
namespace {

__global__ void k_vstats(FragDev* F, int nf, const double* __restrict__ Vj,
                         int* bad) {
  const int j = blockIdx.x;
  if (j >= nf) return;
  const FragDev& fr = F[j];
  double m = -INFINITY;
  int b = 0;
  for (int p = threadIdx.x; p < fr.npts; p += 256) {
    const double v = Vj[fr.v_off + p];
    if (!isfinite(v)) b = 1;
    m = fmax(m, v);
  }
  __shared__ double sm[256];
  __shared__ int sb;
  if (threadIdx.x == 0) sb = 0;
  sm[threadIdx.x] = m;
  __syncthreads();
  if (b) atomicOr(&sb, 1);
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    F[j].vmax = sm[0];
    if (sb) atomicOr(bad, 1);
  }
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
T* arena(void* p) {
  return static_cast<T*>(p);
}

void free_frags(ofm_frags* f) {
  if (f->own_wells) {
    dev_free(f->d_vf);
    dev_free(f->d_vf32);
  }
  void* ptrs[] = {f->d_frag, f->d_v, f->d_v32, f->d_x, f->d_p, f->d_hx,
                  f->d_hphi, f->d_tiles[0], f->d_tiles[1], f->d_tiles[2],
                  f->d_ftiles, f->d_tiles_nr[0], f->d_tiles_nr[1],
                  f->d_tiles_nr[2], f->d_vt[0][0], f->d_vt[0][1],
                  f->d_vt[0][2], f->d_vt[0][3], f->d_vt[0][4], f->d_vt[1][0],
                  f->d_vt[1][1], f->d_vt[1][2], f->d_vt[1][3], f->d_vt[1][4],
                  f->d_tiles_rest[0][0], f->d_tiles_rest[0][1],
                  f->d_tiles_rest[0][2], f->d_tiles_rest[1][0],
                  f->d_tiles_rest[1][1], f->d_tiles_rest[1][2],
                  f->d_stiles, f->d_rtiles, f->d_G,
                  f->d_gfl[0], f->d_gfl[1], f->d_gfl[2], f->d_gfl[3],
                  f->d_rtl[0], f->d_rtl[1], f->d_rtl[2], f->d_rtl[3],
                  f->d_rtl[4],
                  f->d_Q, f->d_theta, f->d_res, f->d_res_partial, f->d_fs,
                  f->d_active, f->d_iters, f->d_conv, f->d_flags,
                  f->d_nactive, f->d_coef};
  for (void* p : ptrs) dev_free(p);
}

// ---------------------------------------------------------------------------
// the batched eigensolver
// ---------------------------------------------------------------------------
// Steps per launch of the multi-step filter kernel for an even degree:
// (3, n3) then (2, n2) with n3 even, so the filtered block ends in X.
static std::vector<std::pair<int, int>> multistep_plan(int degree,
                                                       int max_steps) {
  const int n3 = max_steps >= 3 ? 2 * (degree / 6) : 0;
  return {{3, n3}, {2, (degree - 3 * n3) / 2}};
}

// Three steps per launch is the default in both forms.  Measured on the
// amorphous workload (fragment stage): FP32 363 ms against 403 with two (and
// 382 with four, a form since dropped); FP64 1136 against 1217 with two,
// once the three-step form of the 1024-thread class stopped spilling
// registers (V read again from L2 instead of a five-plane register window).

struct SolveCfg {
  double tol;
  int max_iter, degree;
  unsigned long long seed;
  bool autotune;
  bool use_graph;
  bool resident;
  int fused;   // 0 or 1: one step per launch, else the most steps per launch
};

template <typename T>
ofm_status solve_impl(ofm_ctx* c, ofm_frags* f, const SolveCfg& cfg,
                      double* eps, int* iters, unsigned char* converged) {
  hipStream_t s = c->stream;
  const int nf = f->n_frag;
  T* X = arena<T>(f->d_x);
  T* P = arena<T>(f->d_p);
  T* HX = arena<T>(f->d_hx);
  const double w = sizeof(T);
  OFM_HIP(hipMemsetAsync(f->d_iters, 0, sizeof(int) * nf, s));
  OFM_HIP(hipMemsetAsync(f->d_conv, 0, nf, s));
  OFM_HIP(hipMemsetAsync(f->d_flags, 0, sizeof(int) * nf, s));
  hipLaunchKernelGGL(k_fill_int, dim3((nf + 255) / 256), dim3(256), 0, s,
                     f->d_active, nf, 1);
  OFM_HIP(hipGetLastError());
  k::init_random<T>(s, f, X, cfg.seed);

  // Chebyshev step coefficients, refreshed from the filter intervals at the
  // start of every outer iteration (the captured sweep reads this buffer)
  const size_t coef_need = (size_t)nf * cfg.degree * k::step_coef_bytes(sizeof(T));
  if (f->coef_bytes < coef_need) {
    dev_free(f->d_coef);
    f->d_coef = nullptr;
    f->coef_bytes = 0;
    f->d_coef = dev_alloc<char>(coef_need);
    f->coef_bytes = coef_need;
  }
  std::vector<int> act(nf, 1);
  std::vector<FilterState> fsh(nf);
  hipGraphExec_t sweep_exec = nullptr;
  struct GraphGuard {
    hipGraphExec_t* e;
    ~GraphGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
    }
  } graph_guard{&sweep_exec};
  // stencil variant of the strip launches: cached per (precision, largest
  // plane), else timed on the strips of the first filter sweep (steps 2..7
  // cycle through the variants; every variant computes identical values, so
  // tuning never changes results)
  const long long key = (long long)sizeof(T) * 1000000000LL + f->max_plane;
  int var = f->variant;
  bool tuning = false;
  if (var < 0) {
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
      var = it->second;
    } else {
      var = 1;
      tuning = cfg.autotune && cfg.degree >= 8;
    }
  }
  hipEvent_t tev[6][2] = {};
  if (tuning)
    for (auto& e : tev) {
      OFM_HIP(hipEventCreate(&e[0]));
      OFM_HIP(hipEventCreate(&e[1]));
    }
  // algorithmic bytes / flops of one pass over the active fragments
  auto sums = [&](double& nb, double& npt, double& nb2) {
    nb = npt = nb2 = 0;
    for (int j = 0; j < nf; ++j)
      if (act[j]) {
        const auto& d = f->host[j];
        nb += (double)d.npts * d.bw;
        npt += d.npts;
        nb2 += (double)d.npts * d.bw * d.bw;
      }
  };
  // CholQR2: the first factor is applied to X; the second one (R2^-1, left
  // in d_Q) is folded into the Rayleigh-Ritz rotation
  auto cholqr = [&]() {
    double nb, npt, nb2;
    sums(nb, npt, nb2);
    k::gram<T>(c, f, X, X, f->d_G, f->d_active, nb * w, nb2 * 2.0 * 0.5);
    k::cholinv(s, f, f->d_G, f->d_Q, f->d_active, f->d_flags);
    k::rotate<T>(c, f, X, nullptr, f->d_Q, nullptr, nullptr, f->d_active, 1,
                 2 * nb * w, nb2 * 2.0 * 0.5);
    k::gram<T>(c, f, X, X, f->d_G, f->d_active, nb * w, nb2 * 2.0 * 0.5);
    k::cholinv(s, f, f->d_G, f->d_Q, f->d_active, f->d_flags);
  };
  // H X over every vector of the active fragments.  FP32: boxes of the
  // multi-step classes march along z one plane per workgroup (one stage),
  // the others run in strips; both evaluate a point with the same
  // arithmetic, so the split does not change a bit (amorphous workload:
  // 1.27 against ~2.2 ms per H X; in FP64 the strips were faster, 2.56
  // against 3.03 ms, the 2048-point planes holding one workgroup per CU)
  const bool hx_ms = sizeof(T) == 4 && cfg.fused >= 2 && f->n_vt_all[0] > 0;
  auto apply_plain = [&]() {
    double cb[k::NMSCLS] = {}, cp[k::NMSCLS] = {}, rb = 0, rp = 0;
    for (int j = 0; j < nf; ++j)
      if (act[j]) {
        const FragDev& d = f->host[j];
        const int cls = hx_ms ? k::multistep_class((int)w, d) : 0;
        (cls > 0 ? cb[cls - 1] : rb) += (double)d.npts * d.bw;
        (cls > 0 ? cp[cls - 1] : rp) += d.npts;
      }
    if (hx_ms)
      for (int cl = 0; cl < k::NMSCLS; ++cl)
        if (f->n_vt[0][cl] > 0)
          k::apply_hm<T>(c, f, X, HX, f->d_vt[0][cl], f->n_vt[0][cl], cl + 1,
                         1, f->d_active, 1, nullptr, nullptr, 0,
                         (2 * cb[cl] + cp[cl]) * w, 28.0 * cb[cl]);
    int2* const* tl = hx_ms ? f->d_tiles_rest[0] : f->d_tiles;
    const int* tn = hx_ms ? f->n_tiles_rest[0] : f->n_tiles;
    if (tn[var] > 0)
      k::apply_h<T>(c, f, X, X, HX, tl[var], tn[var], var, f->d_active, 0,
                    f->d_fs, nullptr, 0, 0, -1, (2 * rb + rp) * w, 28.0 * rb);
  };
  int n_active = nf;
  auto rayleigh_ritz = [&]() {
    double nb, npt, nb2;
    sums(nb, npt, nb2);
    if constexpr (sizeof(T) == 8)
      k::gram<T>(c, f, X, HX, f->d_G, f->d_active, 2 * nb * w, nb2 * 2.0);
    else   // mixed form: Rayleigh-Ritz product as split-BF16 x3 on MFMA
      k::gram_x3(c, f, X, HX, f->d_G, f->d_active, 2 * nb * w, nb2 * 2.0);
    k::rr_eig(s, f, f->d_G, f->d_Q, f->d_theta, f->d_active, 1);
    k::rotate<T>(c, f, X, HX, f->d_Q, f->d_theta, f->d_res_partial,
                 f->d_active, 0, 4 * nb * w, nb2 * 4.0);
    OFM_HIP(hipMemsetAsync(f->d_nactive, 0, sizeof(int), s));
    k::finalize_iter(s, f, f->d_theta, f->d_res_partial, f->d_fs, f->d_active,
                     f->d_iters, f->d_conv, cfg.tol, f->d_nactive, f->d_res);
    OFM_HIP(hipMemcpyAsync(&n_active, f->d_nactive, sizeof(int),
                           hipMemcpyDeviceToHost, s));
    OFM_HIP(hipMemcpyAsync(act.data(), f->d_active, sizeof(int) * nf,
                           hipMemcpyDeviceToHost, s));
    OFM_HIP(hipMemcpyAsync(fsh.data(), f->d_fs, sizeof(FilterState) * nf,
                           hipMemcpyDeviceToHost, s));
    OFM_HIP(hipStreamSynchronize(s));
    collect_stats(c);
  };

  cholqr();
  apply_plain();
  rayleigh_ritz();
  // mixed form: boxes of at most 32^3 run the whole filter on chip; boxes
  // whose plane fits the multi-step kernel run two steps per launch; the
  // rest one step per launch in strips
  const bool res = sizeof(T) == 4 && cfg.resident && f->n_ftiles > 0;
  const int vset = res ? 1 : 0;
  const bool have_ms = cfg.fused >= 2 && f->n_vt_all[vset] > 0;
  int2* const* strip_tiles = have_ms ? f->d_tiles_rest[vset]
                             : res ? f->d_tiles_nr : f->d_tiles;
  const int* strip_n = have_ms ? f->n_tiles_rest[vset]
                       : res ? f->n_tiles_nr : f->n_tiles;
  // the variant only changes the strip launches, so the autotuning sweep
  // times those (boxes of the multi-step classes keep their launches)
  if (strip_n[var] == 0) tuning = false;   // nothing to tune
  for (int it = 1; it < cfg.max_iter && n_active > 0; ++it) {
    k::step_coefs_table<T>(s, f, cfg.degree, f->d_coef);
    // filter work: unlocked vectors of the active fragments, per class
    double snb = 0, snpt = 0, mnb = 0, mnpt = 0, rnb = 0, rnpt = 0;
    double cnb[k::NMSCLS] = {}, cnpt[k::NMSCLS] = {};
    for (int j = 0; j < nf; ++j)
      if (act[j] && fsh[j].lock < f->host[j].bw) {
        const FragDev& d = f->host[j];
        const double u = (double)d.npts * (d.bw - fsh[j].lock);
        const int cls = k::multistep_class((int)w, d);
        if (res && k::resident_eligible((int)w, d)) {
          rnb += u;
          rnpt += d.npts;
        } else if (have_ms && cls > 0) {
          mnb += u;
          mnpt += d.npts;
          cnb[cls - 1] += u;
          cnpt[cls - 1] += d.npts;
        } else {
          snb += u;
          snpt += d.npts;
        }
      }
    if (res && rnb > 0) {
      // HBM: y_0 read and y_d written per vector, V_j once per fragment
      // (its 24 vector workgroups share it through L2), once per filter
      if constexpr (sizeof(T) == 4)
        k::filter_resident(c, f, X, f->d_ftiles, f->n_ftiles, f->d_active,
                           f->d_fs, f->d_coef, cfg.degree,
                           (2 * rnb + rnpt) * w, 32.0 * rnb * cfg.degree);
    }
    auto sweep = [&](bool timed_each) {
      if (have_ms) {
        // y_{k-1}, y_{k-2} read (no y_{k-2} on the first launch), the last
        // two iterates written, V_j once per box; a three-step launch leaves
        // its last iterate in the other buffer, so they come in pairs and
        // the filtered block ends in X
        // each class follows its own plan (the classes hold different
        // fragments, so their launches are independent)
        for (int cl = 0; cl < k::NMSCLS; ++cl) {
          if (f->n_vt[vset][cl] == 0) continue;
          T* in = X;
          T* pv = P;
          int step = 1;
          for (const auto& [ns, count] : multistep_plan(cfg.degree, cfg.fused))
            for (int i = 0; i < count; ++i) {
              const double by =
                  (step == 1 ? 3 * cnb[cl] : 4 * cnb[cl]) * w + cnpt[cl] * w;
              k::apply_hm<T>(timed_each ? c : nullptr, f, in, pv,
                             f->d_vt[vset][cl], f->n_vt[vset][cl], cl + 1, ns,
                             f->d_active, step, f->d_fs, f->d_coef,
                             cfg.degree, by, 32.0 * cnb[cl] * ns);
              if (ns % 2) std::swap(in, pv);
              step += ns;
            }
        }
      }
      if (strip_n[var] == 0) return;
      for (int step = 1; step <= cfg.degree; ++step) {
        const bool odd = step & 1;
        const T* in = odd ? X : P;
        const T* prev = odd ? P : X;
        T* out = odd ? P : X;
        const double by = (step == 1 ? 2 * snb : 3 * snb) * w + snpt * w;
        int sv = var;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tuning && step >= 2 && step < 8) {
          sv = (step - 2) % k::NVARIANT;
          e0 = tev[step - 2][0];
          e1 = tev[step - 2][1];
        }
        k::apply_h<T>(timed_each ? c : nullptr, f, in, prev, out,
                      strip_tiles[sv], strip_n[sv], sv, f->d_active, step,
                      f->d_fs, f->d_coef, cfg.degree, 1, -1, by, 32.0 * snb,
                      e0, e1);
      }
    };
    if (!have_ms && strip_n[var] == 0) {
      // every box took the on-chip filter
    } else if (tuning || !cfg.use_graph) {
      sweep(true);
    } else {
      // the sweep is static (tiles, buffers and step coefficients fixed;
      // the active flags, locks and intervals are read from device memory),
      // so it is captured once and replayed every outer iteration
      if (!sweep_exec) {
        std::unique_lock<std::shared_mutex> lk(capture_lock());
        hipGraph_t g = nullptr;
        OFM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
          sweep(false);
        } catch (...) {
          (void)hipStreamEndCapture(s, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        OFM_HIP(hipStreamEndCapture(s, &g));
        const hipError_t ie = hipGraphInstantiate(&sweep_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        OFM_HIP(ie);
      }
      // one event pair brackets the replayed sweep: it is booked under the
      // kernel family that carries its work (a mix of both, "sweep")
      double by = 0;
      int launches = 0;
      if (have_ms) {
        for (int cl = 0; cl < k::NMSCLS; ++cl) {
          if (f->n_vt[vset][cl] == 0) continue;
          int steps_l = 0;
          for (const auto& [ns, count] : multistep_plan(cfg.degree, cfg.fused)) {
            (void)ns;
            steps_l += count;
          }
          launches += steps_l;
          by += (3 * cnb[cl] + cnpt[cl]) * w +
                (steps_l - 1) * (4 * cnb[cl] + cnpt[cl]) * w;
        }
      }
      if (strip_n[var] > 0) {
        launches += cfg.degree;
        for (int step = 1; step <= cfg.degree; ++step)
          by += (step == 1 ? 2 * snb : 3 * snb) * w + snpt * w;
      }
      const char* fam = !have_ms ? "stencil"
                        : strip_n[var] == 0 ? "multistep" : "sweep";
      Timed tm(c, fam, by, 32.0 * (mnb + snb) * cfg.degree, launches);
      OFM_HIP(hipGraphLaunch(sweep_exec, s));
    }
    cholqr();
    apply_plain();
    rayleigh_ritz();
    if (tuning) {
      double tsum[k::NVARIANT] = {0, 0, 0};
      for (int i = 0; i < 6; ++i) {
        float ms = 0;
        OFM_HIP(hipEventElapsedTime(&ms, tev[i][0], tev[i][1]));
        tsum[i % k::NVARIANT] += ms;
      }
      int best = 0;
      for (int v = 1; v < k::NVARIANT; ++v)
        if (tsum[v] < tsum[best]) best = v;
      var = best;
      c->tuned[key] = best;
      tuning = false;
      for (auto& e : tev) {
        (void)hipEventDestroy(e[0]);
        (void)hipEventDestroy(e[1]);
      }
    }
  }
  f->variant = var;
  // states: the lowest s_j Ritz vectors, sign gauge, whole-system H phi
  k::gauge<T>(s, f, X);
  k::whole_h<T>(c, f, X, arena<T>(f->d_hphi), -1);
  std::vector<double> theta(f->th_total);
  std::vector<int> it_h(nf);
  std::vector<unsigned char> cv(nf);
  f->solve_flags.assign(nf, 0);
  OFM_HIP(hipMemcpyAsync(theta.data(), f->d_theta, sizeof(double) * theta.size(),
                         hipMemcpyDeviceToHost, s));
  OFM_HIP(hipMemcpyAsync(it_h.data(), f->d_iters, sizeof(int) * nf,
                         hipMemcpyDeviceToHost, s));
  OFM_HIP(hipMemcpyAsync(cv.data(), f->d_conv, nf, hipMemcpyDeviceToHost, s));
  OFM_HIP(hipMemcpyAsync(f->solve_flags.data(), f->d_flags, sizeof(int) * nf,
                         hipMemcpyDeviceToHost, s));
  OFM_HIP(hipStreamSynchronize(s));
  collect_stats(c);
  f->eps_host.assign(f->n_basis, 0.0);
  bool all = true;
  int n_rank = 0;
  for (int j = 0; j < nf; ++j) {
    const auto& d = f->host[j];
    for (int i = 0; i < d.n_states; ++i)
      f->eps_host[d.basis_off + i] = theta[d.th_off + i];
    // a block that stayed rank deficient after the shifted factorisation
    // cannot be trusted to be orthonormal: not converged
    if (f->solve_flags[j] & 2) {
      cv[j] = 0;
      ++n_rank;
    }
    all = all && cv[j];
    f->solver_states[j] = 1;
  }
  if (eps) std::memcpy(eps, f->eps_host.data(), sizeof(double) * f->n_basis);
  if (iters) std::memcpy(iters, it_h.data(), sizeof(int) * nf);
  if (converged) std::memcpy(converged, cv.data(), nf);
  f->have_states = true;
  if (!all) {
    c->err = "eigensolver reached max_iter before every fragment converged";
    if (n_rank)
      c->err += "; " + std::to_string(n_rank) +
                " fragment(s) kept a rank-deficient block after the shifted "
                "Cholesky factorisation (ofm_solve_flags bit 1)";
    return OFM_E_NOCONV;
  }
  return OFM_OK;
}

}  // namespace

void ofm::run_pair_elements(ofm_ctx* c, ofm_frags* f, PairTask* d_tasks,
                            double* H, double* S, bool may_tune) {
  hipStream_t s = c->stream;
  const bool mixed = c->precision != OFM_FP64;
  // mixed form: the diagonal S block of solver-orthonormalised states is the
  // identity; imported states get theirs from FP64 products
  bool any_imported = false;
  for (auto& t : f->pair_tasks)
    if (t.sym) {
      t.ident = mixed && f->solver_states[t.frag] ? 1 : 0;
      any_imported = any_imported || (mixed && !t.ident);
    }
  const int nt = (int)f->pair_tasks.size();
  if (nt > 0)
    OFM_HIP(hipMemcpyAsync(d_tasks, f->pair_tasks.data(),
                           sizeof(PairTask) * nt, hipMemcpyHostToDevice, s));
  // blocks without a task (S of halo-only pairs) stay zero
  k::fill_zero(s, H, f->n_values);
  k::fill_zero(s, S, f->n_values);
  // algorithmic bytes of the pair-centric contraction: every pair reads the
  // states of j and H|phi> of n over Omega' and the states of n over Omega
  // once (each fragment's data is read once per pair that touches it), plus
  // both blocks; flops 2 s_j s_n per point of each block's support
  const double w = (double)wsize(c);
  double flops = 0, bytes = 2.0 * 8.0 * f->n_values;
  for (auto& t : f->pair_tasks) {
    const double K1 = (double)t.om[0] * t.om[1] * t.om[2];
    const double K0 = t.has_s ? (double)(t.s_hi[0] - t.s_lo[0]) *
                                    (t.s_hi[1] - t.s_lo[1]) *
                                    (t.s_hi[2] - t.s_lo[2])
                              : 0.0;
    const bool s_done = !(mixed && t.sym);   // mixed: S_jj set or separate
    flops += 2.0 * t.ma * t.mb * (K1 + (s_done ? K0 : 0.0));
    bytes += ((double)(t.ma + t.mb) * K1 + (s_done ? t.mb * K0 : 0.0)) * w;
  }
  auto launch = [&](int variant) {
    if (!mixed)
      k::pair_elements<double>(c, f, d_tasks, nt, arena<double>(f->d_x),
                               arena<double>(f->d_hphi), H, S, flops, bytes,
                               variant);
    else
      k::pair_elements<float>(c, f, d_tasks, nt, arena<float>(f->d_x),
                              arena<float>(f->d_hphi), H, S, flops, bytes,
                              variant);
  };
  // kernel variant: pinned, cached per (precision, tile class), or timed
  // once here (every variant writes every block with the same bits, so the
  // last timed run leaves the result)
  const int key = (int)c->precision * 16 + (f->max_states + 15) / 16;
  int variant = c->pair_variant;
  bool done = false;
  if (variant < 0) {
    auto it = c->pair_tuned.find(key);
    if (it != c->pair_tuned.end()) {
      variant = it->second;
    } else if (may_tune) {
      hipEvent_t e[k::NPAIRVARIANT][2];
      for (auto& ev : e) {
        OFM_HIP(hipEventCreate(&ev[0]));
        OFM_HIP(hipEventCreate(&ev[1]));
      }
      float best_ms = 0;
      int best = 0;
      try {
        for (int v = 0; v < k::NPAIRVARIANT; ++v) {
          OFM_HIP(hipEventRecord(e[v][0], s));
          launch(v);
          OFM_HIP(hipEventRecord(e[v][1], s));
        }
        for (int v = 0; v < k::NPAIRVARIANT; ++v) {
          OFM_HIP(hipEventSynchronize(e[v][1]));
          float ms = 0;
          OFM_HIP(hipEventElapsedTime(&ms, e[v][0], e[v][1]));
          if (v == 0 || ms < best_ms) {
            best_ms = ms;
            best = v;
          }
        }
      } catch (...) {
        for (auto& ev : e) {
          (void)hipEventDestroy(ev[0]);
          (void)hipEventDestroy(ev[1]);
        }
        throw;
      }
      for (auto& ev : e) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
      }
      c->pair_tuned[key] = best;
      variant = best;
      done = true;
    } else {
      variant = 1;
    }
  }
  if (!done) launch(variant);
  if (mixed) {
    if (any_imported)
      k::pair_elements_f64_on_f32(c, f, d_tasks, nt, arena<float>(f->d_x),
                                  arena<float>(f->d_hphi), H, S);
  }
}

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* ofm_version(void) { return kVersion; }

ofm_status ofm_create(ofm_ctx** out, int device, void* hip_stream,
                      ofm_precision precision) {
  if (!out) return OFM_E_INVALID;
  *out = nullptr;
  if (precision != OFM_FP64 && precision != OFM_MIXED_BF16X3 &&
      precision != OFM_MIXED_FP16X3) {
    g_create_err = "unknown precision form";
    return OFM_E_INVALID;
  }
  return guarded(nullptr, [&]() -> ofm_status {
    int n = 0;
    OFM_HIP(hipGetDeviceCount(&n));
    OFM_REQUIRE(device >= 0 && device < n, OFM_E_INVALID,
                "device index out of range");
    auto* c = new ofm_ctx;
    c->device = device;
    c->precision = precision;
    try {
      OFM_HIP(hipSetDevice(device));
      if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
      } else {
        OFM_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
      }
      hipDeviceProp_t prop;
      OFM_HIP(hipGetDeviceProperties(&prop, device));
      c->n_cu = prop.multiProcessorCount;
      // device address of the allocation-free entry point's scratch array
      noalloc_init(device);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return OFM_OK;
  });
}

ofm_status ofm_destroy(ofm_ctx* c) {
  if (!c) return OFM_E_INVALID;
  if (c->live > 0) {
    c->err = "destroy every fragment and matrix handle before the context";
    return OFM_E_STATE;
  }
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  collect_stats(c);
  ofm::destroy_blas(c);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return OFM_OK;
}

const char* ofm_last_error(const ofm_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

ofm_status ofm_build_fragments(ofm_ctx* c, const ofm_grid* grid,
                               const double* V, int n_frag,
                               const ofm_fragment_desc* frags,
                               const double* atom_xyz,
                               const long long* frag_atom_ptr,
                               const int* frag_atom_idx, double d_cut,
                               ofm_frags** out) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(grid && V && frags && out, OFM_E_INVALID,
                "grid, V, frags and out are required");
    *out = nullptr;
    use_device(c);
    auto* f = new ofm_frags;
    f->ctx = c;
    try {
      plan_fragments(f, *grid, n_frag, frags, OFM_GUARD_VECTORS);
      plan_pairs(f, atom_xyz, frag_atom_ptr, frag_atom_idx, d_cut);
      f->solver_states.assign(n_frag, 0);
      f->solve_flags.assign(n_frag, 0);
      f->pair_tasks = plan_pair_tasks(f);
      // tile lists
      std::vector<int2> stiles, rtiles;
      int th = 0;
      for (int j = 0; j < n_frag; ++j) {
        auto& d = f->host[j];
        d.th_off = th;
        th += d.bw;
        for (int i = 0; i < d.n_states; ++i) stiles.push_back(make_int2(j, i));
        d.rt_begin = (int)rtiles.size();
        d.rt_count = (d.npts + k::RCH - 1) / k::RCH;
        for (int ch = 0; ch < d.rt_count; ++ch) rtiles.push_back(make_int2(j, ch));
      }
      f->th_total = th;
      f->n_stiles = (int)stiles.size();
      f->n_rtiles = (int)rtiles.size();
      hipStream_t s = c->stream;
      const size_t w = wsize(c);
      f->d_frag = dev_alloc<FragDev>(n_frag);
      // fragment classes: on-chip filter (FP32, <= 32^3), multi-step,
      // strips; the tile lists below cover each combination a solve uses
      std::vector<char> nres(n_frag), rest0(n_frag), rest1(n_frag);
      for (int j = 0; j < n_frag; ++j) {
        const FragDev& d = f->host[j];
        const bool r = k::resident_eligible((int)w, d);
        const bool m = k::multistep_eligible((int)w, d);
        nres[j] = !r;
        rest0[j] = !m;
        rest1[j] = !r && !m;
      }
      auto upload = [&](const std::vector<int2>& tv, int2*& dst, int& n) {
        n = (int)tv.size();
        dst = dev_alloc<int2>(tv.size());
        if (!tv.empty())
          OFM_HIP(hipMemcpyAsync(dst, tv.data(), sizeof(int2) * tv.size(),
                                 hipMemcpyHostToDevice, s));
        OFM_HIP(hipStreamSynchronize(s));
      };
      for (int v = 0; v < k::NVARIANT; ++v) {
        upload(k::stencil_tiles(f, (int)w, v, 0, -1), f->d_tiles[v],
               f->n_tiles[v]);
        upload(k::stencil_tiles(f, (int)w, v, 0, -1, &nres), f->d_tiles_nr[v],
               f->n_tiles_nr[v]);
        upload(k::stencil_tiles(f, (int)w, v, 0, -1, &rest0),
               f->d_tiles_rest[0][v], f->n_tiles_rest[0][v]);
        upload(k::stencil_tiles(f, (int)w, v, 0, -1, &rest1),
               f->d_tiles_rest[1][v], f->n_tiles_rest[1][v]);
      }
      for (int set = 0; set < 2; ++set) {
        std::vector<int2> vt[k::NMSCLS];
        for (int j = 0; j < n_frag; ++j) {
          const FragDev& d = f->host[j];
          if (set == 1 && k::resident_eligible((int)w, d)) continue;
          const int cls = k::multistep_class((int)w, d);
          if (cls == 0) continue;
          for (int v = 0; v < d.bw; ++v) vt[cls - 1].push_back(make_int2(j, v));
        }
        f->n_vt_all[set] = 0;
        for (int cl = 0; cl < k::NMSCLS; ++cl) {
          upload(vt[cl], f->d_vt[set][cl], f->n_vt[set][cl]);
          f->n_vt_all[set] += f->n_vt[set][cl];
        }
      }
      {
        std::vector<int2> ft;
        for (int j = 0; j < n_frag; ++j)
          if (k::resident_eligible((int)w, f->host[j]))
            for (int v = 0; v < f->host[j].bw; ++v) ft.push_back(make_int2(j, v));
        f->n_ftiles = (int)ft.size();
        f->d_ftiles = dev_alloc<int2>(ft.size());
        if (!ft.empty())
          OFM_HIP(hipMemcpyAsync(f->d_ftiles, ft.data(), sizeof(int2) * ft.size(),
                                 hipMemcpyHostToDevice, s));
        OFM_HIP(hipStreamSynchronize(s));
      }
      {
        auto upload_int = [&](const std::vector<int>& v, int*& dst, int& n) {
          n = (int)v.size();
          dst = dev_alloc<int>(v.size());
          if (!v.empty())
            OFM_HIP(hipMemcpyAsync(dst, v.data(), sizeof(int) * v.size(),
                                   hipMemcpyHostToDevice, s));
          OFM_HIP(hipStreamSynchronize(s));
        };
        std::vector<int> gl[4], rl[5];
        for (int j = 0; j < n_frag; ++j) {
          const FragDev& d = f->host[j];
          gl[(d.bw + 15) / 16 - 1].push_back(j);
          for (int ch = 0; ch < d.rt_count; ++ch)
            rl[k::rotate_class(d.bw)].push_back(d.rt_begin + ch);
        }
        for (int cl = 0; cl < 4; ++cl) upload_int(gl[cl], f->d_gfl[cl], f->n_gfl[cl]);
        for (int cl = 0; cl < 5; ++cl) upload_int(rl[cl], f->d_rtl[cl], f->n_rtl[cl]);
      }
      f->d_stiles = dev_alloc<int2>(stiles.size());
      f->d_rtiles = dev_alloc<int2>(rtiles.size());
      f->d_v = dev_alloc<double>(f->v_total);
      f->d_v32 = dev_alloc<float>(f->v_total);
      f->d_vf = f->d_v;
      f->d_vf32 = f->d_v32;
      f->d_x = dev_alloc<char>(f->x_total * w);
      f->d_p = dev_alloc<char>(f->x_total * w);
      f->d_hx = dev_alloc<char>(f->x_total * w);
      f->d_hphi = dev_alloc<char>(f->hphi_total * w);
      f->d_G = dev_alloc<double>((size_t)f->small_total * k::GCH);
      f->d_Q = dev_alloc<double>(f->small_total);
      f->d_theta = dev_alloc<double>(th);
      f->d_res = dev_alloc<double>(th);
      f->d_res_partial = dev_alloc<double>((size_t)f->n_rtiles * k::SMAX);
      f->d_fs = dev_alloc<FilterState>(n_frag);
      f->d_active = dev_alloc<int>(n_frag);
      f->d_iters = dev_alloc<int>(n_frag);
      f->d_conv = dev_alloc<unsigned char>(n_frag);
      f->d_flags = dev_alloc<int>(n_frag);
      f->d_nactive = dev_alloc<int>(4);
      OFM_HIP(hipMemsetAsync(f->d_x, 0, f->x_total * w, s));
      OFM_HIP(hipMemsetAsync(f->d_p, 0, f->x_total * w, s));
      OFM_HIP(hipMemsetAsync(f->d_hx, 0, f->x_total * w, s));
      OFM_HIP(hipMemsetAsync(f->d_hphi, 0, f->hphi_total * w, s));
      OFM_HIP(hipMemsetAsync(f->d_theta, 0, sizeof(double) * th, s));
      OFM_HIP(hipMemcpyAsync(f->d_frag, f->host.data(),
                             sizeof(FragDev) * n_frag, hipMemcpyHostToDevice, s));
      OFM_HIP(hipMemcpyAsync(f->d_stiles, stiles.data(),
                             sizeof(int2) * stiles.size(), hipMemcpyHostToDevice, s));
      OFM_HIP(hipMemcpyAsync(f->d_rtiles, rtiles.data(),
                             sizeof(int2) * rtiles.size(), hipMemcpyHostToDevice, s));
      // potential: copy to the device if needed, restrict to the boxes
      const long long nv = (long long)grid->nx * grid->ny * grid->nz;
      const double* dV = V;
      double* tmp = nullptr;
      if (!is_device_ptr(V)) {
        tmp = dev_alloc<double>(nv);
        OFM_HIP(hipMemcpyAsync(tmp, V, sizeof(double) * nv,
                               hipMemcpyHostToDevice, s));
        dV = tmp;
      }
      int* bad = dev_alloc<int>(1);
      OFM_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
      k::restrict_potential(s, dV, *grid, f);
      hipLaunchKernelGGL(k_vstats, dim3(n_frag), dim3(256), 0, s, f->d_frag,
                         n_frag, f->d_v, bad);
      OFM_HIP(hipGetLastError());
      int bad_h = 0;
      OFM_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
      std::vector<FragDev> back(n_frag);
      OFM_HIP(hipMemcpyAsync(back.data(), f->d_frag, sizeof(FragDev) * n_frag,
                             hipMemcpyDeviceToHost, s));
      OFM_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < n_frag; ++j) f->host[j].vmax = back[j].vmax;
      dev_free(bad);
      dev_free(tmp);
      OFM_REQUIRE(!bad_h, OFM_E_INVALID,
                  "V holds a NaN or Inf inside a fragment box");
    } catch (...) {
      free_frags(f);
      delete f;
      throw;
    }
    c->live += 1;
    *out = f;
    return OFM_OK;
  });
}

ofm_status ofm_frags_destroy(ofm_frags* f) {
  if (!f) return OFM_E_INVALID;
  if (f->ctx) {
    (void)hipSetDevice(f->ctx->device);
    (void)hipStreamSynchronize(f->ctx->stream);
    f->ctx->live -= 1;
  }
  free_frags(f);
  delete f;
  return OFM_OK;
}

ofm_status ofm_frags_info(const ofm_frags* f, long long* n_basis,
                          long long* n_pairs, long long* total_points) {
  if (!f) return OFM_E_INVALID;
  if (n_basis) *n_basis = f->n_basis;
  if (n_pairs) *n_pairs = (long long)f->pair_j.size();
  if (total_points) *total_points = f->total_points;
  return OFM_OK;
}

ofm_status ofm_fragment_geometry(const ofm_frags* f, int j, int lo[3],
                                 int dims[3], int dlo[3], int ddims[3],
                                 int* n_states) {
  if (!f || j < 0 || j >= f->n_frag) return OFM_E_INVALID;
  const FragDev& d = f->host[j];
  for (int a = 0; a < 3; ++a) {
    if (lo) lo[a] = d.lo[a];
    if (dims) dims[a] = d.dims[a];
    if (dlo) dlo[a] = d.dlo[a];
    if (ddims) ddims[a] = d.ddims[a];
  }
  if (n_states) *n_states = d.n_states;
  return OFM_OK;
}

ofm_status ofm_pairs(const ofm_frags* f, int* pair_j, int* pair_n,
                     long long* block_off) {
  if (!f) return OFM_E_INVALID;
  const size_t n = f->pair_j.size();
  if (pair_j) std::memcpy(pair_j, f->pair_j.data(), sizeof(int) * n);
  if (pair_n) std::memcpy(pair_n, f->pair_n.data(), sizeof(int) * n);
  if (block_off) std::memcpy(block_off, f->block_off.data(), sizeof(long long) * n);
  return OFM_OK;
}

ofm_status ofm_solve_fragments(ofm_ctx* c, ofm_frags* f,
                               const ofm_solve_opts* opts, double* eps,
                               int* iters, unsigned char* converged) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(f && f->ctx == c, OFM_E_INVALID,
                "fragments were built with another context");
    use_device(c);
    SolveCfg cfg;
    const bool fp64 = c->precision == OFM_FP64;
    cfg.tol = (opts && opts->tol > 0) ? opts->tol : (fp64 ? 1e-10 : 2e-5);
    cfg.max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 60;
    // default filter degree: multiples of 6 (every multi-step launch takes
    // three steps); with 6 guard vectors the fastest of 30..54 on the
    // amorphous workload, FP64 at tol 1e-10 and the mixed form at 2e-5
    cfg.degree = (opts && opts->degree > 0) ? opts->degree : (fp64 ? 42 : 36);
    cfg.degree += cfg.degree & 1;   // even: the filtered block ends in X
    cfg.seed = opts ? opts->seed : 0;
    cfg.autotune = !opts || opts->autotune >= 0;
    cfg.use_graph = !opts || opts->use_graph >= 0;
    cfg.resident = !opts || opts->resident >= 0;
    cfg.fused = !opts || opts->fused == 0 ? 3
                : opts->fused < 0 ? 0 : std::min(opts->fused, 3);
    OFM_REQUIRE(!opts || opts->guard == 0 || opts->guard == f->guard,
                OFM_E_INVALID,
                "guard vectors are fixed when the fragments are built");
    const double t0 = now_ms();
    ofm_status st = fp64 ? solve_impl<double>(c, f, cfg, eps, iters, converged)
                         : solve_impl<float>(c, f, cfg, eps, iters, converged);
    c->t_solve = now_ms() - t0;
    return st;
  });
}

ofm_status ofm_solve_flags(const ofm_frags* f, int* flags) {
  if (!f || !flags) return OFM_E_INVALID;
  for (int j = 0; j < f->n_frag; ++j)
    flags[j] = j < (int)f->solve_flags.size() ? f->solve_flags[j] : 0;
  return OFM_OK;
}

ofm_status ofm_get_states(const ofm_frags* f, int j, double* phi,
                          double* eps) {
  if (!f || j < 0 || j >= f->n_frag) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(f->have_states, OFM_E_STATE, "no states yet");
    use_device(c);
    const FragDev& d = f->host[j];
    if (phi) {
      const size_t w = wsize(c);
      std::vector<char> buf((size_t)d.n_states * d.npts * w);
      OFM_HIP(hipMemcpy2DAsync(buf.data(), d.npts * w,
                               (char*)f->d_x + d.x_off * w, (size_t)d.ld * w,
                               d.npts * w, d.n_states, hipMemcpyDeviceToHost,
                               c->stream));
      OFM_HIP(hipStreamSynchronize(c->stream));
      const size_t n = (size_t)d.n_states * d.npts;
      if (w == 8)
        std::memcpy(phi, buf.data(), n * 8);
      else
        for (size_t i = 0; i < n; ++i) phi[i] = ((const float*)buf.data())[i];
    }
    if (eps)
      for (int i = 0; i < d.n_states; ++i) eps[i] = f->eps_host[d.basis_off + i];
    return OFM_OK;
  });
}

ofm_status ofm_set_states(ofm_frags* f, int j, const double* phi,
                          const double* eps) {
  if (!f || j < 0 || j >= f->n_frag || !phi) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    use_device(c);
    const FragDev& d = f->host[j];
    const size_t w = wsize(c);
    const size_t n = (size_t)d.n_states * d.npts;
    std::vector<char> buf(n * w);
    if (w == 8)
      std::memcpy(buf.data(), phi, n * 8);
    else
      for (size_t i = 0; i < n; ++i) ((float*)buf.data())[i] = (float)phi[i];
    OFM_HIP(hipMemcpy2DAsync((char*)f->d_x + d.x_off * w, (size_t)d.ld * w,
                             buf.data(), d.npts * w, d.npts * w, d.n_states,
                             hipMemcpyHostToDevice, c->stream));
    if (c->precision == OFM_FP64)
      k::whole_h<double>(c, f, arena<double>(f->d_x), arena<double>(f->d_hphi), j);
    else
      k::whole_h<float>(c, f, arena<float>(f->d_x), arena<float>(f->d_hphi), j);
    OFM_HIP(hipStreamSynchronize(c->stream));
    if (f->eps_host.size() != (size_t)f->n_basis) f->eps_host.assign(f->n_basis, 0.0);
    for (int i = 0; i < d.n_states; ++i)
      f->eps_host[d.basis_off + i] = eps ? eps[i] : 0.0;
    f->solver_states[j] = 0;
    f->have_states = true;
    return OFM_OK;
  });
}

ofm_status ofm_get_hphi(const ofm_frags* f, int j, double* hphi) {
  if (!f || j < 0 || j >= f->n_frag || !hphi) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(f->have_states, OFM_E_STATE, "no states yet");
    use_device(c);
    const FragDev& d = f->host[j];
    const size_t w = wsize(c);
    std::vector<char> buf((size_t)d.n_states * d.ndil * w);
    OFM_HIP(hipMemcpy2DAsync(buf.data(), d.ndil * w,
                             (char*)f->d_hphi + d.hphi_off * w, (size_t)d.ldd * w,
                             d.ndil * w, d.n_states, hipMemcpyDeviceToHost,
                             c->stream));
    OFM_HIP(hipStreamSynchronize(c->stream));
    const size_t n = (size_t)d.n_states * d.ndil;
    if (w == 8)
      std::memcpy(hphi, buf.data(), n * 8);
    else
      for (size_t i = 0; i < n; ++i) hphi[i] = ((const float*)buf.data())[i];
    return OFM_OK;
  });
}

ofm_status ofm_apply_fragment_h(ofm_ctx* c, ofm_frags* f, int j, int nvec,
                                const double* x, double* y) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(f && f->ctx == c && j >= 0 && j < f->n_frag && x && y,
                OFM_E_INVALID, "bad arguments");
    // the stencil's tiles carry the vector index in 15 bits
    OFM_REQUIRE(nvec >= 1 && nvec <= OFM_MAX_APPLY_VECTORS, OFM_E_INVALID,
                "nvec must be in [1, 32767]");
    use_device(c);
    const FragDev& d = f->host[j];
    const size_t w = wsize(c);
    const size_t n = (size_t)nvec * d.ld;
    char* din = dev_alloc<char>(n * w);
    char* dout = dev_alloc<char>(n * w);
    int2* dt = nullptr;
    try {
      std::vector<char> buf((size_t)nvec * d.npts * w);
      for (size_t i = 0; i < (size_t)nvec * d.npts; ++i) {
        if (w == 8)
          ((double*)buf.data())[i] = x[i];
        else
          ((float*)buf.data())[i] = (float)x[i];
      }
      const int var = f->variant >= 0 ? f->variant : 1;
      std::vector<int2> t = k::stencil_tiles(f, (int)w, var, nvec, j);
      OFM_HIP(hipMemsetAsync(din, 0, n * w, c->stream));
      OFM_HIP(hipMemcpy2DAsync(din, (size_t)d.ld * w, buf.data(), d.npts * w,
                               d.npts * w, nvec, hipMemcpyHostToDevice, c->stream));
      dt = dev_alloc<int2>(t.size());
      OFM_HIP(hipMemcpyAsync(dt, t.data(), sizeof(int2) * t.size(),
                             hipMemcpyHostToDevice, c->stream));
      // nvec may exceed b_j: the descriptor's ld is used, tiles list v < nvec
      if (w == 8)
        k::apply_h<double>(c, f, (const double*)din, (const double*)din,
                           (double*)dout, dt, (int)t.size(), var, nullptr, 0,
                           nullptr, nullptr, 0, 0, 0, 0, 0);
      else
        k::apply_h<float>(c, f, (const float*)din, (const float*)din,
                          (float*)dout, dt, (int)t.size(), var, nullptr, 0,
                          nullptr, nullptr, 0, 0, 0, 0, 0);
      OFM_HIP(hipMemcpy2DAsync(buf.data(), d.npts * w, dout, (size_t)d.ld * w,
                               d.npts * w, nvec, hipMemcpyDeviceToHost, c->stream));
      OFM_HIP(hipStreamSynchronize(c->stream));
      collect_stats(c);
      for (size_t i = 0; i < (size_t)nvec * d.npts; ++i)
        y[i] = w == 8 ? ((double*)buf.data())[i] : ((float*)buf.data())[i];
    } catch (...) {
      dev_free(din);
      dev_free(dout);
      dev_free(dt);
      throw;
    }
    dev_free(din);
    dev_free(dout);
    dev_free(dt);
    return OFM_OK;
  });
}

ofm_status ofm_set_fragment_wells(ofm_frags* f, int n_atoms,
                                  const double* atom_xyz, const double* Z,
                                  double sigma, double r_cut,
                                  const long long* frag_atom_ptr,
                                  const int* frag_atom_idx) {
  if (!f) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(n_atoms >= 1 && atom_xyz && Z && frag_atom_ptr && frag_atom_idx,
                OFM_E_INVALID, "atoms, depths and fragment lists are required");
    OFM_REQUIRE(std::isfinite(sigma) && sigma > 0 && std::isfinite(r_cut) &&
                    r_cut > 0, OFM_E_INVALID, "sigma and r_cut must be > 0");
    for (long long a = 0; a < 3LL * n_atoms; ++a)
      OFM_REQUIRE(std::isfinite(atom_xyz[a]), OFM_E_INVALID,
                  "non-finite atom coordinate");
    for (int a = 0; a < n_atoms; ++a)
      OFM_REQUIRE(std::isfinite(Z[a]), OFM_E_INVALID, "non-finite well depth");
    const int nf = f->n_frag;
    OFM_REQUIRE(frag_atom_ptr[0] == 0, OFM_E_INVALID, "frag_atom_ptr[0] != 0");
    for (int j = 0; j < nf; ++j)
      OFM_REQUIRE(frag_atom_ptr[j + 1] >= frag_atom_ptr[j], OFM_E_INVALID,
                  "frag_atom_ptr must be non-decreasing");
    const long long nnz = frag_atom_ptr[nf];
    for (long long a = 0; a < nnz; ++a)
      OFM_REQUIRE(frag_atom_idx[a] >= 0 && frag_atom_idx[a] < n_atoms,
                  OFM_E_INVALID, "atom index out of range");
    use_device(c);
    hipStream_t s = c->stream;
    if (!f->own_wells) {
      f->d_vf = dev_alloc<double>(f->v_total);
      f->d_vf32 = dev_alloc<float>(f->v_total);
      f->own_wells = true;
    }
    double* dxyz = dev_alloc<double>(3LL * n_atoms);
    double* dZ = dev_alloc<double>(n_atoms);
    long long* dptr = dev_alloc<long long>(nf + 1);
    int* didx = dev_alloc<int>(nnz);
    int* bad = dev_alloc<int>(1);
    try {
      OFM_HIP(hipMemcpyAsync(dxyz, atom_xyz, sizeof(double) * 3 * n_atoms,
                             hipMemcpyHostToDevice, s));
      OFM_HIP(hipMemcpyAsync(dZ, Z, sizeof(double) * n_atoms,
                             hipMemcpyHostToDevice, s));
      OFM_HIP(hipMemcpyAsync(dptr, frag_atom_ptr, sizeof(long long) * (nf + 1),
                             hipMemcpyHostToDevice, s));
      if (nnz)
        OFM_HIP(hipMemcpyAsync(didx, frag_atom_idx, sizeof(int) * nnz,
                               hipMemcpyHostToDevice, s));
      k::fragment_wells(s, f, dxyz, dZ, dptr, didx, sigma, r_cut);
      // the filter's spectral bound follows the fragment potential
      OFM_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_vstats, dim3(nf), dim3(256), 0, s, f->d_frag, nf,
                         f->d_vf, bad);
      OFM_HIP(hipGetLastError());
      std::vector<FragDev> back(nf);
      OFM_HIP(hipMemcpyAsync(back.data(), f->d_frag, sizeof(FragDev) * nf,
                             hipMemcpyDeviceToHost, s));
      OFM_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < nf; ++j) f->host[j].vmax = back[j].vmax;
    } catch (...) {
      dev_free(dxyz); dev_free(dZ); dev_free(dptr); dev_free(didx); dev_free(bad);
      throw;
    }
    dev_free(dxyz); dev_free(dZ); dev_free(dptr); dev_free(didx); dev_free(bad);
    return OFM_OK;
  });
}

ofm_status ofm_set_pair_variant(ofm_ctx* c, int variant) {
  if (!c || variant < -1 || variant >= k::NPAIRVARIANT) return OFM_E_INVALID;
  c->pair_variant = variant;
  return OFM_OK;
}

ofm_status ofm_set_stencil_variant(ofm_frags* f, int variant) {
  if (!f || variant < -1 || variant >= k::NVARIANT) return OFM_E_INVALID;
  f->variant = variant;
  return OFM_OK;
}

ofm_status ofm_matrix_elements(ofm_ctx* c, ofm_frags* f, ofm_mats** out) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(f && f->ctx == c && out, OFM_E_INVALID, "bad arguments");
    OFM_REQUIRE(f->have_states, OFM_E_STATE,
                "matrix elements need fragment states (solve or set_states)");
    *out = nullptr;
    use_device(c);
    const double t0 = now_ms();
    auto* m = new ofm_mats;
    m->ctx = c;
    m->frags = f;
    m->n_values = f->n_values;
    m->n_basis = f->n_basis;
    m->pair_j = f->pair_j;
    m->pair_n = f->pair_n;
    m->block_off = f->block_off;
    for (auto& d : f->host) {
      m->states.push_back(d.n_states);
      m->basis_off.push_back(d.basis_off);
    }
    PairTask* dt = nullptr;
    try {
      m->d_H = dev_alloc<double>(f->n_values);
      m->d_S = dev_alloc<double>(f->n_values);
      dt = dev_alloc<PairTask>(f->pair_tasks.size());
      run_pair_elements(c, f, dt, m->d_H, m->d_S, true);
      OFM_HIP(hipStreamSynchronize(c->stream));
      collect_stats(c);
    } catch (...) {
      dev_free(dt);
      dev_free(m->d_H);
      dev_free(m->d_S);
      delete m;
      throw;
    }
    dev_free(dt);
    c->t_elem = now_ms() - t0;
    c->live += 1;
    *out = m;
    return OFM_OK;
  });
}

ofm_status ofm_mats_info(const ofm_mats* m, long long* n_values) {
  if (!m) return OFM_E_INVALID;
  if (n_values) *n_values = m->n_values;
  return OFM_OK;
}

ofm_status ofm_mats_copy(const ofm_mats* m, double* H_blocks,
                         double* S_blocks) {
  if (!m) return OFM_E_INVALID;
  ofm_ctx* c = m->ctx;
  return guarded(c, [&]() -> ofm_status {
    use_device(c);
    if (H_blocks)
      OFM_HIP(hipMemcpyAsync(H_blocks, m->d_H, sizeof(double) * m->n_values,
                             hipMemcpyDeviceToHost, c->stream));
    if (S_blocks)
      OFM_HIP(hipMemcpyAsync(S_blocks, m->d_S, sizeof(double) * m->n_values,
                             hipMemcpyDeviceToHost, c->stream));
    OFM_HIP(hipStreamSynchronize(c->stream));
    return OFM_OK;
  });
}

ofm_status ofm_mats_destroy(ofm_mats* m) {
  if (!m) return OFM_E_INVALID;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  m->ctx->live -= 1;
  dev_free(m->d_H);
  dev_free(m->d_S);
  delete m;
  return OFM_OK;
}

ofm_status ofm_solve_global(ofm_ctx* c, const ofm_mats* m, double s_thresh,
                            double e_lo, double e_hi, int* n_kept, int* n_eig,
                            double* E, double* C, double* s_min) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(m && m->ctx == c && n_eig && E, OFM_E_INVALID, "bad arguments");
    OFM_REQUIRE(std::isfinite(s_thresh) && s_thresh >= 0, OFM_E_INVALID,
                "s_thresh must be finite and >= 0");
    use_device(c);
    const double t0 = now_ms();
    global_solve(c, m, s_thresh, e_lo, e_hi, n_kept, n_eig, E, C, s_min);
    c->t_global = now_ms() - t0;
    return OFM_OK;
  });
}

ofm_status ofm_solve_global_subset(ofm_ctx* c, const ofm_mats* m,
                                   const unsigned char* keep, double s_thresh,
                                   double e_lo, double e_hi, int* n_kept,
                                   int* n_eig, double* E, double* C,
                                   double* s_min) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(m && m->ctx == c && n_eig && E, OFM_E_INVALID, "bad arguments");
    OFM_REQUIRE(std::isfinite(s_thresh) && s_thresh >= 0, OFM_E_INVALID,
                "s_thresh must be finite and >= 0");
    use_device(c);
    const double t0 = now_ms();
    global_solve(c, m, s_thresh, e_lo, e_hi, n_kept, n_eig, E, C, s_min, keep);
    c->t_global = now_ms() - t0;
    return OFM_OK;
  });
}

ofm_status ofm_select_homo(const ofm_frags* f, int n_max, double gap_min,
                           unsigned char* keep) {
  if (!f) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(keep && n_max >= 1, OFM_E_INVALID,
                "keep is required and n_max must be >= 1");
    OFM_REQUIRE(std::isfinite(gap_min), OFM_E_INVALID, "gap_min must be finite");
    OFM_REQUIRE(f->have_states && (long long)f->eps_host.size() == f->n_basis,
                OFM_E_STATE, "no states yet");
    for (int j = 0; j < f->n_frag; ++j) {
      const FragDev& d = f->host[j];
      const double* e = f->eps_host.data() + d.basis_off;
      const int s = d.n_states;
      int n = std::min(n_max, s);
      if (gap_min > 0)
        for (int k = s - 1; k > std::max(s - n_max, 0); --k)
          if (e[k] - e[k - 1] >= gap_min) {
            n = s - k;
            break;
          }
      for (int i = 0; i < s; ++i) keep[d.basis_off + i] = i >= s - n ? 1 : 0;
    }
    return OFM_OK;
  });
}

ofm_status ofm_select_band(const ofm_frags* f, double e_lo, double e_hi,
                           unsigned char* keep) {
  if (!f) return OFM_E_INVALID;
  ofm_ctx* c = f->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(keep && std::isfinite(e_lo) && std::isfinite(e_hi),
                OFM_E_INVALID, "keep is required and the bounds must be finite");
    OFM_REQUIRE(f->have_states && (long long)f->eps_host.size() == f->n_basis,
                OFM_E_STATE, "no states yet");
    for (long long i = 0; i < f->n_basis; ++i) {
      const double e = f->eps_host[i];
      keep[i] = (e >= e_lo && e <= e_hi) ? 1 : 0;
    }
    return OFM_OK;
  });
}

ofm_status ofm_solve_global_window(ofm_ctx* c, const ofm_mats* m,
                                   double s_thresh, double e_lo, double e_hi,
                                   double margin0, double margin_step,
                                   int max_rounds, double tol, int* n_eig,
                                   double* E, double* margin, long long* n_sel,
                                   int* n_kept) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(m && m->ctx == c && n_eig && E, OFM_E_INVALID, "bad arguments");
    OFM_REQUIRE(std::isfinite(s_thresh) && s_thresh >= 0, OFM_E_INVALID,
                "s_thresh must be finite and >= 0");
    OFM_REQUIRE(std::isfinite(e_lo) && std::isfinite(e_hi) && e_hi >= e_lo,
                OFM_E_INVALID, "the window must be finite with e_hi >= e_lo");
    OFM_REQUIRE(std::isfinite(margin0) && margin0 >= 0 &&
                    std::isfinite(margin_step) && margin_step > 0,
                OFM_E_INVALID, "margin0 must be >= 0 and margin_step > 0");
    OFM_REQUIRE(max_rounds >= 2 && std::isfinite(tol) && tol >= 0,
                OFM_E_INVALID, "max_rounds must be >= 2 and tol >= 0");
    const ofm_frags* f = m->frags;
    OFM_REQUIRE(f->have_states && (long long)f->eps_host.size() == f->n_basis,
                OFM_E_STATE, "no fragment eigenvalues");
    use_device(c);
    const double t0 = now_ms();
    std::vector<unsigned char> keep(f->n_basis);
    std::vector<double> cur(f->n_basis), prev;
    bool have_prev = false, conv = false;
    long long last = -1;
    int ne = 0;
    for (int r = 0; r < max_rounds && !conv; ++r) {
      const double d = margin0 + r * margin_step;
      long long cnt = 0;
      for (long long i = 0; i < f->n_basis; ++i) {
        const double e = f->eps_host[i];
        keep[i] = (e >= e_lo - d && e <= e_hi + d) ? 1 : 0;
        cnt += keep[i];
      }
      // a band that adds nothing to the last one solved gives nothing new
      if (cnt == 0 || cnt == last) continue;
      int kept = 0;
      global_solve(c, m, s_thresh, e_lo, e_hi, &kept, &ne, cur.data(), nullptr,
                   nullptr, keep.data());
      if (cnt == f->n_basis) {   // the whole basis: the full solve
        conv = true;
      } else if (have_prev && (int)prev.size() == ne) {
        double dmax = 0;
        for (int i = 0; i < ne; ++i) dmax = std::max(dmax, std::fabs(cur[i] - prev[i]));
        conv = dmax <= tol;
      }
      prev.assign(cur.begin(), cur.begin() + ne);
      have_prev = true;
      last = cnt;
      if (margin) *margin = d;
      if (n_sel) *n_sel = cnt;
      if (n_kept) *n_kept = kept;
    }
    ne = have_prev ? (int)prev.size() : 0;
    *n_eig = ne;
    for (int i = 0; i < ne; ++i) E[i] = prev[i];
    c->t_global = now_ms() - t0;
    if (!conv) {
      c->err = "the window's eigenvalues did not settle within max_rounds";
      return OFM_E_NOCONV;
    }
    return OFM_OK;
  });
}

ofm_status ofm_dense_eigh(ofm_ctx* c, int n, const double* A, double* w,
                          double* Z) {
  if (!c) return OFM_E_INVALID;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(A && w, OFM_E_INVALID, "A and w are required");
    OFM_REQUIRE(n >= 1 && n <= 65536, OFM_E_INVALID,
                "n outside the dense solver's range [1, 65536]");
    const long long nn = (long long)n * n;
    for (long long e = 0; e < nn; ++e)
      OFM_REQUIRE(std::isfinite(A[e]), OFM_E_INVALID, "A has a NaN or Inf");
    use_device(c);
    dense_eigh_host(c, n, A, w, Z);
    return OFM_OK;
  });
}

ofm_status ofm_homo_energies(const ofm_mats* m, double* e) {
  if (!m) return OFM_E_INVALID;
  ofm_ctx* c = m->ctx;
  return guarded(c, [&]() -> ofm_status {
    OFM_REQUIRE(e, OFM_E_INVALID, "e is required");
    use_device(c);
    homo_energies(m, e);
    return OFM_OK;
  });
}

ofm_status ofm_homo_lumo_gap(const double* E, int n, double e_ref,
                             double gap_min, int* n_occ, double* e_homo,
                             double* e_lumo) {
  if (n < 0 || (n > 0 && !E) || !n_occ || !e_homo || !e_lumo ||
      !std::isfinite(e_ref) || !(gap_min >= 0) || !std::isfinite(gap_min))
    return OFM_E_INVALID;
  for (int k = 0; k + 1 < n; ++k)
    if (!(E[k + 1] >= E[k])) return OFM_E_INVALID;
  *n_occ = -1;
  *e_homo = *e_lumo = std::nan("");
  int k = 0;
  while (k < n && !(E[k] >= e_ref)) ++k;
  for (; k + 1 < n; ++k)
    if (E[k + 1] - E[k] >= gap_min) {
      *n_occ = k + 1;
      *e_homo = E[k];
      *e_lumo = E[k + 1];
      break;
    }
  return OFM_OK;
}

ofm_status ofm_set_profiling(ofm_ctx* c, int on) {
  if (!c) return OFM_E_INVALID;
  c->profiling = on != 0;
  return OFM_OK;
}

ofm_status ofm_kernel_stats(ofm_ctx* c, const char* family,
                            long long* launches, double* total_ms,
                            double* alg_bytes, double* flops) {
  if (!c || !family) return OFM_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  collect_stats(c);
  auto it = c->stats.find(family);
  KernelStat s;
  if (it != c->stats.end()) s = it->second;
  if (launches) *launches = s.launches;
  if (total_ms) *total_ms = s.ms;
  if (alg_bytes) *alg_bytes = s.bytes;
  if (flops) *flops = s.flops;
  return OFM_OK;
}

ofm_status ofm_reset_stats(ofm_ctx* c) {
  if (!c) return OFM_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  collect_stats(c);
  c->stats.clear();
  return OFM_OK;
}

ofm_status ofm_stage_times(const ofm_ctx* c, double* solve_ms,
                           double* elements_ms, double* global_ms) {
  if (!c) return OFM_E_INVALID;
  if (solve_ms) *solve_ms = c->t_solve;
  if (elements_ms) *elements_ms = c->t_elem;
  if (global_ms) *global_ms = c->t_global;
  return OFM_OK;
}

}  // extern "C"
