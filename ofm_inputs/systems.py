"""Seeded synthetic systems: geometry, grid, potential samples and fragment boxes.

Conventions (Hartree atomic units: Ha, bohr):

* Grid point (ix, iy, iz) sits at ``origin + (ix, iy, iz) * h``.  Arrays that
  live on the grid are stored x-fastest, i.e. numpy shape ``(nz, ny, nx)`` and
  linear index ``ix + nx * (iy + ny * iz)``.
* The potential is a sum of Gaussian wells, ``V(r) = sum_a -Z_a exp(-|r-R_a|^2
  / (2 sigma^2))``, each well truncated at ``|r-R_a| < r_cut`` (8 bohr = 10
  sigma, where a well has fallen below 2e-22 of its depth).  It stands in for
  the whole-system potential that the paper takes as input (Sec. II).
* A fragment is a cuboid box of grid points, ``lo`` (x, y, z) and ``dims``
  (x, y, z) in global grid indices, plus the number of its lowest states that
  enter the basis (Sec. II: a molecule embedded in a cuboid box; Sec. III-B:
  the lowest states of each fragment).  ``frag_atom_ptr``/``frag_atom_idx``
  list the atoms of each fragment in CSR form.

Every random quantity is drawn from ``numpy.random.default_rng(seed)`` in a
fixed order, so a (config, seed) pair always gives the same system.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIGMA = 0.8     # Gaussian well width (bohr)
R_CUT = 8.0     # well truncation radius (bohr)
Z_C, Z_H, Z_S = 1.0, 0.5, 1.5   # well depths (Ha) by element

TETRA = math.radians(109.47122063449069)   # tetrahedral angle


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    h: float
    origin: np.ndarray = field(default_factory=lambda: np.zeros(3))

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)

    @property
    def npoints(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class System:
    name: str
    grid: Grid
    atoms: np.ndarray          # (n_atoms, 3) float64, bohr
    Z: np.ndarray              # (n_atoms,) float64, well depth (Ha)
    frag_lo: np.ndarray        # (n_frag, 3) int32, (x, y, z)
    frag_dims: np.ndarray      # (n_frag, 3) int32, (x, y, z)
    frag_states: np.ndarray    # (n_frag,) int32
    frag_atom_ptr: np.ndarray  # (n_frag + 1,) int64
    frag_atom_idx: np.ndarray  # (nnz,) int32
    sigma: float = SIGMA
    r_cut: float = R_CUT
    seed: int = 0
    notes: str = ""
    _V: np.ndarray | None = None

    @property
    def n_frag(self) -> int:
        return int(self.frag_lo.shape[0])

    @property
    def n_basis(self) -> int:
        return int(self.frag_states.sum())

    def potential(self) -> np.ndarray:
        """V sampled on the grid, shape (nz, ny, nx), float64 (cached)."""
        if self._V is None:
            self._V = sample_wells(self.grid, self.atoms, self.Z,
                                   self.sigma, self.r_cut)
        return self._V

    def with_potential(self, V: np.ndarray) -> "System":
        """Copy of the system with an explicit potential array (e.g. V = 0)."""
        s = System(**{k: getattr(self, k) for k in self.__dataclass_fields__
                      if k != "_V"})
        s._V = np.ascontiguousarray(V, dtype=np.float64).reshape(
            self.grid.shape_zyx)
        return s


def sample_wells(grid: Grid, atoms, Z, sigma=SIGMA, r_cut=R_CUT) -> np.ndarray:
    """Sum of truncated Gaussian wells sampled at the grid points."""
    V = np.zeros(grid.shape_zyx, dtype=np.float64)
    h = grid.h
    n = np.array([grid.nx, grid.ny, grid.nz])
    inv2s2 = 1.0 / (2.0 * sigma * sigma)
    rc2 = r_cut * r_cut
    for a in range(atoms.shape[0]):
        rel = (atoms[a] - grid.origin) / h
        lo = np.maximum(np.ceil(rel - r_cut / h).astype(np.int64), 0)
        hi = np.minimum(np.floor(rel + r_cut / h).astype(np.int64), n - 1)
        if np.any(hi < lo):
            continue
        dx = grid.origin[0] + np.arange(lo[0], hi[0] + 1) * h - atoms[a, 0]
        dy = grid.origin[1] + np.arange(lo[1], hi[1] + 1) * h - atoms[a, 1]
        dz = grid.origin[2] + np.arange(lo[2], hi[2] + 1) * h - atoms[a, 2]
        r2 = (dz * dz)[:, None, None] + (dy * dy)[None, :, None] \
            + (dx * dx)[None, None, :]
        w = np.where(r2 < rc2, np.exp(-r2 * inv2s2), 0.0)
        V[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] -= Z[a] * w
    return V


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------

def _unit(v):
    return v / np.linalg.norm(v)


def _place(a, b, c, bond, angle, dihedral):
    """Position d with |cd| = bond, angle(b,c,d) = angle, dihedral(a,b,c,d)."""
    bc = _unit(c - b)
    nrm = np.cross(b - a, bc)
    ln = np.linalg.norm(nrm)
    if ln < 1e-12:  # collinear a,b,c: pick any perpendicular
        nrm = np.cross(bc, [1.0, 0.0, 0.0])
        if np.linalg.norm(nrm) < 1e-6:
            nrm = np.cross(bc, [0.0, 1.0, 0.0])
        ln = np.linalg.norm(nrm)
    nrm = nrm / ln
    m = np.cross(nrm, bc)
    return (c - bond * math.cos(angle) * bc
            + bond * math.sin(angle) * math.cos(dihedral) * m
            + bond * math.sin(angle) * math.sin(dihedral) * nrm)


def _alkane_hydrogens(C, bond_ch=2.1):
    """Two tetrahedral H per interior carbon, three per chain-end carbon.

    Returns (positions (nH,3), owner carbon index (nH,))."""
    nC = C.shape[0]
    hs, own = [], []
    half = 0.5 * TETRA
    for k in range(nC):
        if 0 < k < nC - 1:
            a, c = C[k - 1], C[k + 1]
            u = _unit(2.0 * C[k] - a - c)
            nn = _unit(np.cross(a - C[k], c - C[k]))
            for sgn in (1.0, -1.0):
                hs.append(C[k] + bond_ch * (math.cos(half) * u
                                            + sgn * math.sin(half) * nn))
                own.append(k)
        else:
            nb = C[1] if k == 0 else C[nC - 2]
            nb2 = C[2] if k == 0 else C[nC - 3]
            d = _unit(C[k] - nb)
            e1 = nb2 - nb
            e1 = _unit(e1 - np.dot(e1, d) * d)
            e2 = np.cross(d, e1)
            beta = math.pi - TETRA
            for i in range(3):
                phi = math.pi / 3.0 + 2.0 * math.pi * i / 3.0
                hs.append(C[k] + bond_ch * (math.cos(beta) * d + math.sin(beta)
                                            * (math.cos(phi) * e1
                                               + math.sin(phi) * e2)))
                own.append(k)
    return np.array(hs), np.array(own, dtype=np.int64)


def _csr(lists):
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    idx = (np.concatenate([np.asarray(x, dtype=np.int32) for x in lists])
           if lists else np.zeros(0, np.int32))
    return ptr, idx.astype(np.int32)


def _box_around(centre, dims, grid: Grid):
    """Lower corner of a box of ``dims`` points centred on ``centre``
    (bohr), snapped to the grid and clipped to lie inside it."""
    n = np.array([grid.nx, grid.ny, grid.nz])
    dims = np.asarray(dims)
    rel = (np.asarray(centre) - grid.origin) / grid.h
    lo = np.rint(rel - 0.5 * (dims - 1)).astype(np.int64)
    return np.clip(lo, 0, n - dims).astype(np.int32)


def _grid_around(atoms, h, margin):
    lo = atoms.min(axis=0) - margin
    ext = atoms.max(axis=0) + margin - lo
    n = np.ceil(ext / h).astype(int) + 1
    return Grid(int(n[0]), int(n[1]), int(n[2]), h, lo.astype(np.float64))


def _windows(n_sites, n_windows):
    """Index windows of consecutive sites with 50% overlap: stride
    n_sites/(n_windows+1), width two strides."""
    stride = n_sites / (n_windows + 1)
    out = []
    for k in range(n_windows):
        a = int(math.ceil(k * stride - 1e-9))
        b = int(math.ceil((k + 2) * stride - 1e-9))
        out.append(np.arange(a, min(b, n_sites)))
    return out


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def tiny_chain(seed: int = 0, frag_width: int = 12, n_states: int = 6,
               offsets=(0, 6, 12)) -> System:
    """Tiny plain OFM: 24x12x12 grid (h = 0.5), six Z = 1 wells on a straight
    chain along x (spacing 2 bohr, jitter U(-0.2, 0.2) per coordinate), three
    12^3 fragments at x offsets 0, 6, 12 with the six lowest states each."""
    g = Grid(24, 12, 12, 0.5, np.zeros(3))
    centre = 0.5 * g.h * np.array([g.nx - 1, g.ny - 1, g.nz - 1])
    atoms = np.array([centre + np.array([(k - 2.5) * 2.0, 0.0, 0.0])
                      for k in range(6)])
    rng = np.random.default_rng(seed)
    atoms = atoms + rng.uniform(-0.2, 0.2, size=(6, 3))
    Z = np.full(6, Z_C)
    lo = np.array([[o, 0, 0] for o in offsets], dtype=np.int32)
    dims = np.array([[frag_width, g.ny, g.nz]] * len(offsets), dtype=np.int32)
    lists = []
    for f in range(len(offsets)):
        x0 = g.origin[0] + lo[f, 0] * g.h
        x1 = x0 + (dims[f, 0] - 1) * g.h
        lists.append(np.nonzero((atoms[:, 0] >= x0) & (atoms[:, 0] <= x1))[0])
    ptr, idx = _csr(lists)
    return System("tiny_chain", g, atoms, Z, lo, dims,
                  np.full(len(offsets), n_states, np.int32), ptr, idx,
                  seed=seed,
                  notes="6-well straight chain, 24x12x12 grid, 3 fragments")


def alkane_chain(seed: int = 0, n_carbon: int = 666, n_frag: int = 256,
                 box: int = 32, n_states: int = 16, h: float = 0.5) -> System:
    """Alkane-like chain C_nH_(2n+2) (2000 atoms at n = 666): C-C 2.9 bohr,
    C-C-C 109.47 deg, dihedrals U[0, 2 pi) (not self-avoiding), C-H 2.1 bohr
    tetrahedral.  Grid = atom bounding box + 8 bohr margin.  Fragments are
    50%-overlap windows of consecutive carbons (with their hydrogens), each in
    a ``box``^3 box centred on the window's carbon centroid."""
    rng = np.random.default_rng(seed)
    bond = 2.9
    C = np.zeros((n_carbon, 3))
    C[1] = [bond, 0.0, 0.0]
    C[2] = C[1] + bond * np.array([-math.cos(TETRA), math.sin(TETRA), 0.0])
    dih = rng.uniform(0.0, 2.0 * math.pi, size=n_carbon)
    for k in range(3, n_carbon):
        C[k] = _place(C[k - 3], C[k - 2], C[k - 1], bond, TETRA, dih[k])
    H, own = _alkane_hydrogens(C)
    atoms = np.vstack([C, H])
    Z = np.concatenate([np.full(n_carbon, Z_C), np.full(H.shape[0], Z_H)])
    g = _grid_around(atoms, h, R_CUT)
    wins = _windows(n_carbon, n_frag)
    lo, lists = [], []
    for w in wins:
        lo.append(_box_around(C[w].mean(axis=0), (box, box, box), g))
        hidx = n_carbon + np.nonzero(np.isin(own, w))[0]
        lists.append(np.concatenate([w, hidx]))
    ptr, idx = _csr(lists)
    return System("alkane_chain", g, atoms, Z, np.array(lo, np.int32),
                  np.full((n_frag, 3), box, np.int32),
                  np.full(n_frag, n_states, np.int32), ptr, idx, seed=seed,
                  notes=f"C{n_carbon}H{H.shape[0]} random-dihedral chain")


def _saw_chain(rng, n, bond, placed, lo_b, hi_b, start_lo, start_hi,
               min_dist=3.0, tries=60):
    """Self-avoiding tetrahedral backbone: a new site is rejected when it is
    closer than ``min_dist`` to any earlier non-bonded site (``placed`` holds
    the sites of earlier chains) or leaves the box [lo_b, hi_b]^3."""
    from scipy.spatial import cKDTree
    for _restart in range(200):
        P = np.zeros((n, 3))
        P[0] = rng.uniform(start_lo, start_hi, size=3)
        d = _unit(rng.normal(size=3))
        P[1] = P[0] + bond * d
        tmp = _unit(np.cross(d, rng.normal(size=3)))
        P[2] = P[1] + bond * (-math.cos(TETRA) * d + math.sin(TETRA) * tmp)
        if np.any(P[1:3] < lo_b) or np.any(P[1:3] > hi_b):
            continue
        tree = cKDTree(placed) if len(placed) else None
        ok = True
        for k in range(3, n):
            good = False
            for _t in range(tries):
                q = _place(P[k - 3], P[k - 2], P[k - 1], bond, TETRA,
                           rng.uniform(0.0, 2.0 * math.pi))
                if np.any(q < lo_b) or np.any(q > hi_b):
                    continue
                if k - 2 > 0 and np.min(np.linalg.norm(
                        P[:k - 1] - q, axis=1)) < min_dist:
                    continue
                if tree is not None and tree.query(q)[0] < min_dist:
                    continue
                good = True
                break
            if not good:
                ok = False
                break
            P[k] = q
        if ok:
            return P
    raise RuntimeError("self-avoiding walk failed to place a chain")


def amorphous_polymer(seed: int = 0, n_chains: int = 20, n_carbon: int = 166,
                      n_frag: int = 1024, edge_range=(24, 40),
                      state_range=(8, 32), box_bohr: float = 120.0,
                      h: float = 0.5) -> System:
    """Amorphous alkane-like polymer: ``n_chains`` self-avoiding chains of
    C_nH_(2n+2) (10,000 atoms at 20 x 166 carbons) started uniformly in
    [16, 104]^3 bohr and confined to [8, 112]^3 inside a 120^3 bohr cell
    (240^3 grid at h = 0.5).  ``n_frag`` 50%-overlap windows are spread over
    the chains as evenly as possible; box edges are drawn per axis from
    U{edge_range} and state counts from U{state_range}."""
    rng = np.random.default_rng(seed)
    bond = 2.9
    chains, placed = [], np.zeros((0, 3))
    for _c in range(n_chains):
        P = _saw_chain(rng, n_carbon, bond, placed, 8.0, box_bohr - 8.0,
                       16.0, box_bohr - 16.0)
        chains.append(P)
        placed = np.vstack([placed, P])
    atoms_c, atoms_h, owners = [], [], []
    for ci, P in enumerate(chains):
        H, own = _alkane_hydrogens(P)
        atoms_c.append(P)
        atoms_h.append(H)
        owners.append(own)
    nC = n_chains * n_carbon
    C_all = np.vstack(atoms_c)
    H_all = np.vstack(atoms_h)
    atoms = np.vstack([C_all, H_all])
    Z = np.concatenate([np.full(nC, Z_C), np.full(H_all.shape[0], Z_H)])
    n = int(round(box_bohr / h))
    g = Grid(n, n, n, h, np.zeros(3))
    per = [n_frag // n_chains + (1 if c < n_frag % n_chains else 0)
           for c in range(n_chains)]
    lo, dims, lists = [], [], []
    h_off = nC
    for ci, P in enumerate(chains):
        nH_c = atoms_h[ci].shape[0]
        for w in _windows(n_carbon, per[ci]):
            d = rng.integers(edge_range[0], edge_range[1] + 1, size=3)
            dims.append(d)
            lo.append(_box_around(P[w].mean(axis=0), d, g))
            hidx = h_off + np.nonzero(np.isin(owners[ci], w))[0]
            lists.append(np.concatenate([ci * n_carbon + w, hidx]))
        h_off += nH_c
    states = rng.integers(state_range[0], state_range[1] + 1, size=n_frag)
    ptr, idx = _csr(lists)
    return System("amorphous_polymer", g, atoms, Z, np.array(lo, np.int32),
                  np.array(dims, np.int32), states.astype(np.int32), ptr, idx,
                  seed=seed,
                  notes=f"{n_chains} self-avoiding C{n_carbon} chains")


def _thiophene_chain(rng, n_rings, placed, lo_b, hi_b, start_lo, start_hi,
                     side=2.7, link=2.7, bond_ch=2.05, min_dist=4.0,
                     tries=60):
    """Chain of planar 5-rings (S + 4 C as a regular pentagon) linked
    alpha-alpha and alternating anti; the ring direction follows a
    self-avoiding walk.  Returns (atoms (7*n_rings, 3), elements, ring
    centres)."""
    from scipy.spatial import cKDTree
    # pentagon in its own frame: S at the apex, alpha carbons next to S
    R = side / (2.0 * math.sin(math.pi / 5.0))
    ang = [math.pi / 2.0 + 2.0 * math.pi * k / 5.0 for k in range(5)]
    pent = np.array([[R * math.cos(a), R * math.sin(a)] for a in ang])
    # order: 0 S, 1 C_alpha, 2 C_beta, 3 C_beta, 4 C_alpha
    ca1, ca2 = pent[1], pent[4]
    axis = _unit(ca2 - ca1)
    for _restart in range(200):
        atoms, elems, centres = [], [], []
        pos = rng.uniform(start_lo, start_hi, size=3)
        d = _unit(rng.normal(size=3))
        up = _unit(np.cross(d, rng.normal(size=3)))
        ok = True
        tree = cKDTree(placed) if len(placed) else None
        prev_end = None
        for r in range(n_rings):
            good = False
            for _t in range(tries):
                if r == 0:
                    dn, un = d, up
                else:
                    # persistent direction first, any direction when stuck
                    spread = 0.45 if _t < tries // 3 else 3.0
                    dn = _unit(d + spread * rng.normal(size=3))
                    un = _unit(np.cross(dn, np.cross(up, dn)))
                    if not np.all(np.isfinite(un)):
                        continue
                    un = -un  # anti alternation
                vn = np.cross(dn, un)
                # map local (axis, perp) onto (dn, un) in the ring plane
                perp = np.array([-axis[1], axis[0]])
                start = pos if prev_end is None else prev_end + link * dn
                origin = start - (ca1 @ axis) * dn - (ca1 @ perp) * un
                loc = [origin + (p @ axis) * dn + (p @ perp) * un
                       for p in pent]
                loc = np.array(loc)
                cen = loc.mean(axis=0)
                hb = []
                for bi in (2, 3):
                    out = _unit(loc[bi] - cen)
                    hb.append(loc[bi] + bond_ch * out)
                ring = np.vstack([loc, np.array(hb)])
                if np.any(ring < lo_b) or np.any(ring > hi_b):
                    continue
                if centres and len(centres) > 1:
                    dc = np.linalg.norm(np.array(centres[:-1]) - cen, axis=1)
                    if np.min(dc) < min_dist:
                        continue
                if tree is not None and tree.query(cen)[0] < min_dist:
                    continue
                good = True
                break
            if not good:
                ok = False
                break
            atoms.append(ring)
            elems += ["S", "C", "C", "C", "C", "H", "H"]
            centres.append(cen)
            prev_end = ring[4]
            d, up = dn, un
            _ = vn
        if ok:
            return np.vstack(atoms), elems, np.array(centres)
    raise RuntimeError("thiophene walk failed to place a chain")


def thiophene_polymer(seed: int = 0, n_chains: int = 64, n_rings: int = 66,
                      edge_range=(32, 48), n_states: int = 24,
                      h: float = 0.5) -> System:
    """Polythiophene-like amorphous system: ``n_chains`` chains of
    ``n_rings`` 5-rings (S + 4 C, side 2.7 bohr, alpha-alpha links 2.7 bohr,
    two H on the beta carbons at 2.05 bohr: 7 atoms per ring, 29,568 atoms at
    64 x 66) in a cubic cell at the amorphous polymer's atom density.
    Fragments are overlapping trimers (three consecutive rings, stride one:
    64 x 64 = 4096), cubic boxes with edges from U{edge_range}, ``n_states``
    states each."""
    rng = np.random.default_rng(seed)
    n_atoms = n_chains * n_rings * 7
    density = 10000.0 / 120.0 ** 3
    L = (n_atoms / density) ** (1.0 / 3.0)
    n = int(round(L / h))
    L = n * h
    g = Grid(n, n, n, h, np.zeros(3))
    atoms, elems, centres_all = [], [], []
    placed = np.zeros((0, 3))
    for _c in range(n_chains):
        A, E, cen = _thiophene_chain(rng, n_rings, placed, 8.0, L - 8.0,
                                     16.0, L - 16.0)
        atoms.append(A)
        elems += E
        centres_all.append(cen)
        placed = np.vstack([placed, cen])
    atoms = np.vstack(atoms)
    zmap = {"S": Z_S, "C": Z_C, "H": Z_H}
    Z = np.array([zmap[e] for e in elems])
    lo, dims, lists = [], [], []
    for ci in range(n_chains):
        base = ci * n_rings * 7
        for r in range(n_rings - 2):
            idx = base + np.arange(7 * r, 7 * (r + 3))
            e = int(rng.integers(edge_range[0], edge_range[1] + 1))
            d = (e, e, e)
            dims.append(d)
            lo.append(_box_around(atoms[idx].mean(axis=0), d, g))
            lists.append(idx)
    ptr, idx = _csr(lists)
    nf = len(lo)
    return System("thiophene_polymer", g, atoms, Z, np.array(lo, np.int32),
                  np.array(dims, np.int32), np.full(nf, n_states, np.int32),
                  ptr, idx, seed=seed,
                  notes=f"{n_chains} chains x {n_rings} thiophene-like rings")


def box_system(shape_xyz, h, frag_lo, frag_dims, frag_states, atoms=None,
               Z=None, V=None, name="custom", seed=0) -> System:
    """A hand-specified system for tests: explicit grid, boxes and either
    atoms (wells) or an explicit potential array ``V`` (shape (nz, ny, nx))."""
    g = Grid(int(shape_xyz[0]), int(shape_xyz[1]), int(shape_xyz[2]), float(h),
             np.zeros(3))
    atoms = np.zeros((0, 3)) if atoms is None else np.asarray(atoms, float)
    Z = np.zeros(atoms.shape[0]) if Z is None else np.asarray(Z, float)
    nf = len(frag_lo)
    ptr, idx = _csr([np.zeros(0, np.int32)] * nf)
    s = System(name, g, atoms, Z, np.asarray(frag_lo, np.int32).reshape(nf, 3),
               np.asarray(frag_dims, np.int32).reshape(nf, 3),
               np.asarray(frag_states, np.int32).reshape(nf), ptr, idx,
               seed=seed)
    if V is not None:
        s = s.with_potential(V)
    return s


CONFIGS = {
    "tiny": tiny_chain,            # 24x12x12, 3 fragments, FP64 and mixed
    "alkane": alkane_chain,        # 2000 atoms, 256 fragments of 32^3
    "amorphous": amorphous_polymer,  # 10,000 atoms, 1024 uneven fragments
    "thiophene": thiophene_polymer,  # 29,568 atoms, 4096 trimer fragments
}


def make_system(name: str, seed: int = 0, **kw) -> System:
    return CONFIGS[name](seed=seed, **kw)
