// Host-side geometry planner: validates the fragment boxes, lays out the
// device arenas (64-bit offsets) and enumerates the fragment pairs whose
// matrix elements can be non-zero.
//
// Pair set (method Sec. II: only pairs of fragments that are close enough
// are evaluated; Sec. III-C: closeness by a distance cutoff).  With a
// 5-point-per-axis stencil, <phi^(j)|H|phi^(n)> and <phi^(j)|phi^(n)> vanish
// exactly unless box_j grown by 2 points meets box_n, so that test gives the
// exact pair set; the optional atom-distance cutoff prunes it further.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "ofm_internal.h"

namespace ofm {

static constexpr int REACH = 2;

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

void plan_fragments(ofm_frags* f, const ofm_grid& g, int n_frag,
                    const ofm_fragment_desc* fr, int guard) {
  OFM_REQUIRE(g.nx >= 1 && g.ny >= 1 && g.nz >= 1, OFM_E_INVALID,
              "grid dimensions must be >= 1");
  OFM_REQUIRE(std::isfinite(g.h) && g.h > 0, OFM_E_INVALID,
              "grid spacing must be finite and > 0");
  OFM_REQUIRE(n_frag >= 1 && fr != nullptr, OFM_E_INVALID,
              "need at least one fragment");
  const int N[3] = {g.nx, g.ny, g.nz};
  f->grid = g;
  f->n_frag = n_frag;
  f->guard = guard;
  f->host.resize(n_frag);
  long long v_off = 0, x_off = 0, h_off = 0, basis = 0;
  int small = 0;
  f->max_bw = f->max_plane = f->max_states = 0;
  for (int j = 0; j < n_frag; ++j) {
    FragDev d{};
    long long npts = 1;
    for (int a = 0; a < 3; ++a) {
      const int lo = fr[j].lo[a], dm = fr[j].dims[a];
      OFM_REQUIRE(dm >= 1 && lo >= 0 && (long long)lo + dm <= N[a],
                  OFM_E_INVALID,
                  "fragment " + std::to_string(j) + " box outside the grid");
      d.lo[a] = lo;
      d.dims[a] = dm;
      d.dlo[a] = std::max(lo - REACH, 0);
      d.ddims[a] = std::min(lo + dm + REACH, N[a]) - d.dlo[a];
      npts *= dm;
    }
    OFM_REQUIRE(npts <= (1LL << 24), OFM_E_INVALID,
                "fragment " + std::to_string(j) + " box too large");
    OFM_REQUIRE((long long)d.dims[0] * d.dims[1] <= (1 << 22), OFM_E_INVALID,
                "fragment " + std::to_string(j) + ": xy plane too large");
    OFM_REQUIRE(d.dims[0] <= 128, OFM_E_INVALID,
                "fragment " + std::to_string(j) +
                    ": a box may span at most 128 points along x");
    const int s = fr[j].n_states;
    OFM_REQUIRE(s >= 1 && s <= npts, OFM_E_INVALID,
                "fragment " + std::to_string(j) +
                    ": n_states must be in [1, box points]");
    OFM_REQUIRE(s <= 64, OFM_E_INVALID,
                "fragment " + std::to_string(j) +
                    ": at most 64 states per fragment are supported");
    d.n_states = s;
    d.npts = (int)npts;
    d.bw = (int)std::min<long long>(s + guard, std::min<long long>(npts, 64));
    d.ld = round_up(d.npts, 32);
    d.ndil = d.ddims[0] * d.ddims[1] * d.ddims[2];
    d.ldd = round_up(d.ndil, 32);
    d.gfaces = (d.lo[0] == 0 ? FACE_XLO : 0) |
               (d.lo[0] + d.dims[0] == N[0] ? FACE_XHI : 0) |
               (d.lo[1] == 0 ? FACE_YLO : 0) |
               (d.lo[1] + d.dims[1] == N[1] ? FACE_YHI : 0) |
               (d.lo[2] == 0 ? FACE_ZLO : 0) |
               (d.lo[2] + d.dims[2] == N[2] ? FACE_ZHI : 0);
    d.small_off = small;
    d.v_off = v_off;
    d.x_off = x_off;
    d.hphi_off = h_off;
    d.basis_off = basis;
    small += d.bw * d.bw;
    v_off += d.npts;
    x_off += (long long)d.bw * d.ld;
    h_off += (long long)s * d.ldd;
    basis += s;
    f->max_bw = std::max(f->max_bw, d.bw);
    f->max_plane = std::max(f->max_plane, d.dims[0] * d.dims[1]);
    f->max_states = std::max(f->max_states, s);
    f->host[j] = d;
  }
  f->v_total = v_off;
  f->x_total = x_off;
  f->hphi_total = h_off;
  f->small_total = small;
  f->n_basis = basis;
  f->total_points = v_off;
}

// minimum atom-atom distance between two fragments (brute force over their
// atom lists)
static double min_atom_distance(const double* xyz, const long long* ptr,
                                const int* idx, int j, int n) {
  double best = INFINITY;
  for (long long a = ptr[j]; a < ptr[j + 1]; ++a) {
    const double* p = xyz + 3LL * idx[a];
    for (long long b = ptr[n]; b < ptr[n + 1]; ++b) {
      const double* q = xyz + 3LL * idx[b];
      const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
      best = std::min(best, dx * dx + dy * dy + dz * dz);
    }
  }
  return std::sqrt(best);
}

void plan_pairs(ofm_frags* f, const double* atom_xyz,
                const long long* frag_atom_ptr, const int* frag_atom_idx,
                double d_cut) {
  const int nf = f->n_frag;
  const auto& H = f->host;
  // sort-and-sweep along x: after sorting by lower x, box k can reach box j
  // only while lo_x(k) < hi_x(j) + REACH
  std::vector<int> order(nf);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return H[a].lo[0] != H[b].lo[0] ? H[a].lo[0] < H[b].lo[0] : a < b;
  });
  std::vector<std::pair<int, int>> pairs;
  pairs.reserve((size_t)nf * 16);
  for (int j = 0; j < nf; ++j) pairs.emplace_back(j, j);
  for (int ii = 0; ii < nf; ++ii) {
    const FragDev& a = H[order[ii]];
    const int ahi = a.lo[0] + a.dims[0];
    for (int kk = ii + 1; kk < nf; ++kk) {
      const FragDev& b = H[order[kk]];
      if (b.lo[0] >= ahi + REACH) break;
      bool near = true;
      for (int ax = 1; ax < 3 && near; ++ax)
        near = (a.lo[ax] - REACH < b.lo[ax] + b.dims[ax]) &&
               (b.lo[ax] < a.lo[ax] + a.dims[ax] + REACH);
      if (!near) continue;
      int j = order[ii], n = order[kk];
      if (j > n) std::swap(j, n);
      if (d_cut > 0 && atom_xyz && frag_atom_ptr && frag_atom_idx &&
          min_atom_distance(atom_xyz, frag_atom_ptr, frag_atom_idx, j, n) >=
              d_cut)
        continue;
      pairs.emplace_back(j, n);
    }
  }
  std::sort(pairs.begin(), pairs.end());
  f->pair_j.resize(pairs.size());
  f->pair_n.resize(pairs.size());
  f->block_off.resize(pairs.size());
  long long off = 0;
  for (size_t p = 0; p < pairs.size(); ++p) {
    f->pair_j[p] = pairs[p].first;
    f->pair_n[p] = pairs[p].second;
    f->block_off[p] = off;
    off += (long long)H[pairs[p].first].n_states * H[pairs[p].second].n_states;
  }
  f->n_values = off;
}

// intersection of [alo, alo+ad) and [blo, blo+bd) per axis; false if empty
static bool intersect(const int* alo, const int* ad, const int* blo,
                      const int* bd, int* lo, int* dims) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = std::max(alo[a], blo[a]);
    const int hi = std::min(alo[a] + ad[a], blo[a] + bd[a]);
    dims[a] = hi - lo[a];
    if (dims[a] <= 0) return false;
  }
  return true;
}

std::vector<PairTask> plan_pair_tasks(const ofm_frags* f) {
  std::vector<PairTask> tasks;
  tasks.reserve(f->pair_j.size());
  for (size_t p = 0; p < f->pair_j.size(); ++p) {
    const FragDev& a = f->host[f->pair_j[p]];
    const FragDev& b = f->host[f->pair_n[p]];
    int lo[3], dm[3], slo[3], sdm[3];
    // Omega' = box_j ^ dil(box_n) is never empty for a pair of the list
    if (!intersect(a.lo, a.dims, b.dlo, b.ddims, lo, dm)) continue;
    PairTask t{};
    t.a_off = a.x_off;
    t.b_off = b.x_off;
    t.h_off = b.hphi_off;
    t.c_off = f->block_off[p];
    t.has_s = intersect(a.lo, a.dims, b.lo, b.dims, slo, sdm) ? 1 : 0;
    for (int ax = 0; ax < 3; ++ax) {
      t.a_org[ax] = lo[ax] - a.lo[ax];
      t.b_org[ax] = lo[ax] - b.lo[ax];
      t.h_org[ax] = lo[ax] - b.dlo[ax];
      t.om[ax] = dm[ax];
      t.s_lo[ax] = t.has_s ? slo[ax] - lo[ax] : 0;
      t.s_hi[ax] = t.has_s ? slo[ax] + sdm[ax] - lo[ax] : 0;
    }
    t.a_nx = a.dims[0];
    t.a_nxy = a.dims[0] * a.dims[1];
    t.b_nx = b.dims[0];
    t.b_nxy = b.dims[0] * b.dims[1];
    t.h_nx = b.ddims[0];
    t.h_nxy = b.ddims[0] * b.ddims[1];
    t.lda = a.ld;
    t.ldb = b.ld;
    t.ldh = b.ldd;
    t.ma = a.n_states;
    t.mb = b.n_states;
    t.sym = f->pair_j[p] == f->pair_n[p];
    t.frag = f->pair_j[p];
    tasks.push_back(t);
  }
  // longest contraction first: better load balance across workgroups
  std::stable_sort(tasks.begin(), tasks.end(),
                   [](const PairTask& x, const PairTask& y) {
                     const long long kx = (long long)x.om[0] * x.om[1] *
                                          x.om[2] * x.ma * x.mb;
                     const long long ky = (long long)y.om[0] * y.om[1] *
                                          y.om[2] * y.ma * y.mb;
                     return kx > ky;
                   });
  return tasks;
}

}  // namespace ofm
