"""Plain FP64 CPU oracle for the OFM hot path (test infrastructure only).

What the method computes, and where the paper defines it:

* The single-particle Hamiltonian H = -1/2 Laplacian + V (Eq. 1, atomic
  units), here discretised on a uniform real-space grid with the standard
  4th-order central second difference, and V a given array on that grid.
* Fragments are cuboid boxes (Sec. II); fragment j contributes the lowest
  s_j eigenstates of its own Hamiltonian (Sec. III-B: the lowest states of
  each fragment form the basis; Sec. II: each fragment is diagonalised).
* H|phi> is taken with the Hamiltonian of the *whole* system, not the
  fragment's (Sec. II).
* The outputs are H_{ij,mn} = <phi_i^(j)|H|phi_m^(n)> and S_{ij,mn} =
  <phi_i^(j)|phi_m^(n)> for fragment pairs that are close enough (Sec. II,
  Sec. III-C), and the generalised eigenproblem sum_mn (H - E S) C = 0
  (Eq. 2).

Readings taken where the paper is silent (each restated in the design notes):

* Walls: a box of N points along an axis has Dirichlet walls one spacing
  outside it, psi(-1) = psi(N) = 0; the second ghosts of the 5-point stencil
  are odd images, psi(-2) = -psi(0) and psi(N+1) = -psi(N-1).  The same rule
  holds for the global grid and for every fragment box.  With it the 1-D
  operator is diagonalised by the sine transform (closed-form spectrum).
* The fragment Hamiltonian is the global V restricted to the box, with walls
  at the box faces.
* Inner products are plain l2 sums over grid points; states have sum phi^2 = 1.
* The pair set is exact for the stencil: {j, n} is kept iff box_j dilated by
  the stencil reach (2 points) intersects box_n.  Outside that set every
  H and S element is exactly zero.
* Eigenvector gauge: the component of largest magnitude is positive (lowest
  linear index on ties).
* Global solve: S = U s U^T, directions with s < tau (1e-6) are dropped,
  X = U_K s_K^(-1/2), E = eig(X^T H X).

Parity pins for every function live in tests/test_oracle_*.py.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "REACH", "D2_COEFFS", "gaussian_potential", "d2_line", "kinetic_box",
    "hamiltonian_box", "fragment_states", "canonical_sign", "dilated_box",
    "apply_whole_H", "pair_list", "pair_blocks", "assemble", "global_solve",
    "full_grid_eigs", "line_spectrum", "box_spectrum", "OracleResult",
    "run", "window_below_cutoff", "own_wells", "select_top",
    "select_by_gap", "subset", "homo_energies", "homo_lumo_gap",
    "select_band", "window_by_band",
]

#: stencil reach (points) of the 4th-order central second difference
REACH = 2
#: 4th-order central second-difference weights for offsets -2..2 (times 1/h^2)
D2_COEFFS = (-1.0 / 12.0, 4.0 / 3.0, -5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0)


# --------------------------------------------------------------------------
# potential (input check only: the method takes V as given, Sec. II)
# --------------------------------------------------------------------------

def gaussian_potential(shape_xyz, h, origin, atoms, Z, sigma=0.8,
                       r_cut=None):
    """V(r_i) = sum_a -Z_a exp(-|r_i - R_a|^2 / (2 sigma^2)) at every grid
    point r_i = origin + i*h, optionally truncated at |r - R| < r_cut.
    Evaluated point-by-point against every atom (no local boxes)."""
    nx, ny, nz = shape_xyz
    x = origin[0] + h * np.arange(nx)
    y = origin[1] + h * np.arange(ny)
    z = origin[2] + h * np.arange(nz)
    Zg, Yg, Xg = np.meshgrid(z, y, x, indexing="ij")
    V = np.zeros((nz, ny, nx))
    for a in range(len(Z)):
        r2 = (Xg - atoms[a, 0]) ** 2 + (Yg - atoms[a, 1]) ** 2 \
            + (Zg - atoms[a, 2]) ** 2
        term = -Z[a] * np.exp(-r2 / (2.0 * sigma ** 2))
        if r_cut is not None:
            term[r2 >= r_cut ** 2] = 0.0
        V += term
    return V


# --------------------------------------------------------------------------
# finite-difference kinetic operator (Eq. 1 kinetic term, discretised)
# --------------------------------------------------------------------------

def d2_line(N, h, start=0, n=None):
    """Second-difference matrix of a line of N points with Dirichlet walls
    (odd-image second ghosts), restricted to rows/cols [start, start+n).

    Row i gets w_o / h^2 at column i+o for o in -2..2; a column that falls on
    a wall (-1 or N) is zero; column -2 maps to -psi(0) and N+1 to
    -psi(N-1)."""
    if n is None:
        n = N - start
    rows, cols, vals = [], [], []
    for i in range(N):
        for o, w in zip(range(-2, 3), D2_COEFFS):
            j = i + o
            if 0 <= j < N:
                rows.append(i); cols.append(j); vals.append(w)
            elif j == -2:
                rows.append(i); cols.append(0); vals.append(-w)
            elif j == N + 1:
                rows.append(i); cols.append(N - 1); vals.append(-w)
    A = sp.coo_matrix((np.array(vals) / h ** 2, (rows, cols)),
                      shape=(N, N)).tocsr()
    return A[start:start + n, start:start + n]


def kinetic_box(grid_xyz, lo, dims, h):
    """T = -1/2 (D2x + D2y + D2z) on the sub-box [lo, lo+dims) of a grid of
    shape grid_xyz (walls at that grid's faces), x-fastest ordering."""
    Ax = d2_line(grid_xyz[0], h, lo[0], dims[0])
    Ay = d2_line(grid_xyz[1], h, lo[1], dims[1])
    Az = d2_line(grid_xyz[2], h, lo[2], dims[2])
    Ix, Iy, Iz = (sp.identity(d, format="csr") for d in dims)
    lap = sp.kron(Iz, sp.kron(Iy, Ax)) + sp.kron(Iz, sp.kron(Ay, Ix)) \
        + sp.kron(Az, sp.kron(Iy, Ix))
    return (-0.5 * lap).tocsr()


def _slice(V, lo, dims):
    return V[lo[2]:lo[2] + dims[2], lo[1]:lo[1] + dims[1],
             lo[0]:lo[0] + dims[0]]


def hamiltonian_box(V, h, lo, dims, walls="box", Vbox=None):
    """Sparse H restricted to a box.  walls="box": the fragment Hamiltonian
    (walls at the box faces, V restricted to the box, or the box potential
    ``Vbox`` (dims[2], dims[1], dims[0]) when given).  walls="global": the
    rows/columns of the whole-system Hamiltonian that fall in the box."""
    nz, ny, nx = V.shape
    lo = tuple(int(v) for v in lo)
    dims = tuple(int(v) for v in dims)
    if walls == "box":
        T = kinetic_box(dims, (0, 0, 0), dims, h)
    else:
        T = kinetic_box((nx, ny, nz), lo, dims, h)
    vb = _slice(V, lo, dims) if Vbox is None else np.asarray(Vbox)
    return (T + sp.diags(vb.ravel())).tocsr()


def own_wells(h, origin, lo, dims, atoms, Z, members, sigma=0.8, r_cut=8.0):
    """Potential of a fragment's own atoms on its box: the wells of the atoms
    listed in ``members`` only (the fragment Hamiltonian built from the
    fragment's own atoms, as the paper builds it from the fragment's own
    charge density, Sec. II)."""
    members = np.asarray(members, dtype=np.int64)
    box_origin = np.asarray(origin, float) + h * np.asarray(lo, float)
    return gaussian_potential(tuple(int(d) for d in dims), h, box_origin,
                              np.asarray(atoms)[members],
                              np.asarray(Z)[members], sigma, r_cut)


def canonical_sign(phi):
    """Flip each column so its largest-|.| entry (first on ties) is > 0."""
    phi = np.array(phi, copy=True)
    for k in range(phi.shape[1]):
        i = int(np.argmax(np.abs(phi[:, k])))
        if phi[i, k] < 0:
            phi[:, k] = -phi[:, k]
    return phi


def fragment_states(V, h, lo, dims, s, dense_max=14000, Vbox=None):
    """Lowest s eigenpairs of the fragment Hamiltonian: dense symmetric
    eigensolver for boxes up to dense_max points, ARPACK (smallest
    algebraic, tol 1e-12) above that.  Returns (eps (s,), phi (n_j, s)).
    ``Vbox`` replaces the global V on the box (own-atoms fragment)."""
    H = hamiltonian_box(V, h, lo, dims, walls="box", Vbox=Vbox)
    n = H.shape[0]
    if n <= dense_max:
        w, U = sla.eigh(H.toarray(), subset_by_index=[0, s - 1],
                        driver="evr")
    else:
        rng = np.random.default_rng(12345)
        w, U = spla.eigsh(H, k=s, which="SA", tol=1e-12,
                          v0=rng.standard_normal(n), ncv=max(2 * s + 1, 40))
        order = np.argsort(w)
        w, U = w[order], U[:, order]
    return w, canonical_sign(U)


# --------------------------------------------------------------------------
# whole-system H on the dilated box (Sec. II)
# --------------------------------------------------------------------------

def dilated_box(lo, dims, grid_xyz, reach=REACH):
    """Box grown by ``reach`` points per side, clipped to the grid."""
    lo = np.asarray(lo, dtype=np.int64)
    hi = lo + np.asarray(dims, dtype=np.int64)
    dlo = np.maximum(lo - reach, 0)
    dhi = np.minimum(hi + reach, np.asarray(grid_xyz, dtype=np.int64))
    return dlo, dhi - dlo


def _embed(phi, lo, dims, dlo, ddims):
    """Zero-extend columns of phi (box [lo, lo+dims)) onto box [dlo, ...)."""
    s = phi.shape[1]
    out = np.zeros((ddims[2], ddims[1], ddims[0], s))
    off = np.asarray(lo) - np.asarray(dlo)
    out[off[2]:off[2] + dims[2], off[1]:off[1] + dims[1],
        off[0]:off[0] + dims[0], :] = phi.reshape(dims[2], dims[1], dims[0], s)
    return out.reshape(-1, s)


def apply_whole_H(V, h, lo, dims, phi):
    """H_whole @ phi for states supported on box [lo, lo+dims), evaluated on
    the dilated box (the only points where the product can be non-zero).
    Returns (dlo, ddims, Hphi (n_dilated, s))."""
    nz, ny, nx = V.shape
    dlo, ddims = dilated_box(lo, dims, (nx, ny, nz))
    Hd = hamiltonian_box(V, h, dlo, ddims, walls="global")
    return dlo, ddims, Hd @ _embed(phi, lo, dims, dlo, ddims)


# --------------------------------------------------------------------------
# pair set and matrix elements (Sec. II)
# --------------------------------------------------------------------------

def pair_list(frag_lo, frag_dims, reach=REACH, d_cut=None, atoms=None,
              frag_atom_ptr=None, frag_atom_idx=None):
    """All pairs j <= n (diagonal included) whose boxes come within the
    stencil reach of each other, in lexicographic (j, n) order.

    With d_cut > 0 (Sec. III-C), an off-diagonal pair is kept only if the
    closest two atoms of the two fragments are less than d_cut apart."""
    lo = np.asarray(frag_lo, dtype=np.int64)
    hi = lo + np.asarray(frag_dims, dtype=np.int64)   # exclusive
    nf = lo.shape[0]
    out = []
    for j in range(nf):
        ok = np.all((lo[j] - reach < hi[j:]) & (lo[j:] < hi[j] + reach),
                    axis=1)
        for n in np.nonzero(ok)[0]:
            out.append((j, j + int(n)))
    if d_cut is not None and d_cut > 0:
        def members(f):
            return np.asarray(frag_atom_idx[frag_atom_ptr[f]:
                                            frag_atom_ptr[f + 1]])
        kept = []
        for (j, n) in out:
            if j == n:
                kept.append((j, n))
                continue
            a, b = atoms[members(j)], atoms[members(n)]
            if len(a) and len(b):
                d = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1))
                if d.min() < d_cut:
                    kept.append((j, n))
        out = kept
    return out


def _intersect(alo, adims, blo, bdims):
    lo = np.maximum(np.asarray(alo), np.asarray(blo))
    hi = np.minimum(np.asarray(alo) + np.asarray(adims),
                    np.asarray(blo) + np.asarray(bdims))
    return lo, np.maximum(hi - lo, 0)


def _restrict(arr, alo, adims, lo, dims):
    """Rows of arr (box [alo, alo+adims), x-fastest) that lie in [lo, ...)."""
    s = arr.shape[1]
    a = arr.reshape(adims[2], adims[1], adims[0], s)
    o = np.asarray(lo) - np.asarray(alo)
    return a[o[2]:o[2] + dims[2], o[1]:o[1] + dims[1],
             o[0]:o[0] + dims[0], :].reshape(-1, s)


def pair_blocks(j, n, frag_lo, frag_dims, phi, hphi, hphi_box):
    """(S_jn, H_jn, H_nj^T) for one pair.

    S_jn = Phi_j^T Phi_n summed over box_j & box_n.
    H_jn = Phi_j^T (H Phi_n) summed over box_j & dil(box_n).
    The second ordering (H Phi_j)^T Phi_n is returned for the symmetry check.
    """
    lo_j, d_j = frag_lo[j], frag_dims[j]
    lo_n, d_n = frag_lo[n], frag_dims[n]
    olo, od = _intersect(lo_j, d_j, lo_n, d_n)
    sj, sn = phi[j].shape[1], phi[n].shape[1]
    if np.all(od > 0):
        S = _restrict(phi[j], lo_j, d_j, olo, od).T @ \
            _restrict(phi[n], lo_n, d_n, olo, od)
    else:
        S = np.zeros((sj, sn))
    dlo_n, dd_n = hphi_box[n]
    hlo, hd = _intersect(lo_j, d_j, dlo_n, dd_n)
    if np.all(hd > 0):
        H = _restrict(phi[j], lo_j, d_j, hlo, hd).T @ \
            _restrict(hphi[n], dlo_n, dd_n, hlo, hd)
    else:
        H = np.zeros((sj, sn))
    dlo_j, dd_j = hphi_box[j]
    glo, gd = _intersect(dlo_j, dd_j, lo_n, d_n)
    if np.all(gd > 0):
        H2 = _restrict(hphi[j], dlo_j, dd_j, glo, gd).T @ \
            _restrict(phi[n], lo_n, d_n, glo, gd)
    else:
        H2 = np.zeros((sj, sn))
    return S, H, H2


def assemble(n_states, pairs, blocks):
    """Dense symmetric H, S (basis ordered fragment by fragment) from the
    upper blocks j <= n; diagonal blocks symmetrised as (A + A^T)/2."""
    off = np.concatenate([[0], np.cumsum(n_states)])
    N = int(off[-1])
    H = np.zeros((N, N))
    S = np.zeros((N, N))
    for (j, n), (Sb, Hb) in zip(pairs, blocks):
        a, b = slice(off[j], off[j + 1]), slice(off[n], off[n + 1])
        if j == n:
            H[a, a] = 0.5 * (Hb + Hb.T)
            S[a, a] = 0.5 * (Sb + Sb.T)
        else:
            H[a, b] = Hb
            H[b, a] = Hb.T
            S[a, b] = Sb
            S[b, a] = Sb.T
    return H, S


# --------------------------------------------------------------------------
# generalised eigenproblem (Eq. 2)
# --------------------------------------------------------------------------

def global_solve(H, S, tau=1e-6, e_lo=-np.inf, e_hi=np.inf,
                 want_vectors=False):
    """Thresholded canonical orthogonalisation: S = U diag(s) U^T, keep
    s >= tau, X = U_K s_K^(-1/2), eigenpairs of X^T H X.  Returns a dict
    with all eigenvalues E (ascending), the window selection, the kept count
    and the smallest kept s."""
    s, U = np.linalg.eigh(S)
    keep = s >= tau
    if not np.any(keep):
        raise np.linalg.LinAlgError("every eigenvalue of S is below tau")
    X = U[:, keep] / np.sqrt(s[keep])
    Hp = X.T @ H @ X
    Hp = 0.5 * (Hp + Hp.T)
    if want_vectors:
        E, Y = np.linalg.eigh(Hp)
        C = X @ Y
    else:
        E = np.linalg.eigvalsh(Hp)
        C = None
    sel = (E >= e_lo) & (E <= e_hi)
    return {"E": E, "window": E[sel], "n_kept": int(keep.sum()),
            "s_min_kept": float(s[keep].min()), "s": s,
            "C": None if C is None else C[:, sel]}


# --------------------------------------------------------------------------
# basis selection near the top of the occupied fragment states and the
# HOMO-LUMO gap of the whole system (Sec. III-B)
# --------------------------------------------------------------------------
# The fragment states computed for fragment j, eps_j[0] <= ... <= eps_j[s-1],
# play the role of its occupied states; the last one is its HOMO.

def select_top(eps, n_top):
    """Keep mask over the basis (fragment by fragment): the n_top highest
    computed states of every fragment (all of them where s_j <= n_top)."""
    keep = []
    for e in eps:
        s = len(e)
        keep.append(np.arange(s) >= s - min(n_top, s))
    return np.concatenate(keep)


def select_by_gap(eps, gap_min, n_max):
    """Keep mask: for each fragment, walk down from its HOMO and cut at the
    first substantial gap, eps_j[k] - eps_j[k-1] >= gap_min, keeping the
    states k..s-1; with no such gap among the top n_max states keep those
    n_max (the paper's rule: cut where the fragment levels have a gap)."""
    keep = []
    for e in eps:
        s = len(e)
        n = min(n_max, s)
        for k in range(s - 1, max(s - n_max, 0), -1):
            if e[k] - e[k - 1] >= gap_min:
                n = s - k
                break
        keep.append(np.arange(s) >= s - n)
    return np.concatenate(keep)


def subset(H, S, keep):
    """The pencil restricted to the kept basis functions (principal
    submatrices)."""
    idx = np.flatnonzero(keep)
    return H[np.ix_(idx, idx)], S[np.ix_(idx, idx)]


def select_band(eps, e_lo, e_hi):
    """Keep mask over the basis (fragment by fragment) of the states whose
    fragment eigenvalue lies in [e_lo, e_hi], bounds included.  With the
    restricted pencil (subset) this is the windowed solve of a basis too
    large for the whole pencil (Sec. II: the generalised eigenproblem of the
    fragment basis; Sec. III-D: its cost grows as the cube of the basis)."""
    e = np.concatenate([np.asarray(x, float) for x in eps])
    return (e >= e_lo) & (e <= e_hi)


def window_by_band(H, S, eps, e_lo, e_hi, tau=1e-6, margin0=0.1,
                   margin_step=0.1, max_rounds=6, tol=1e-8):
    """Eigenvalues of the thresholded pencil in [e_lo, e_hi] on the basis
    functions within a margin of the window.  The margin grows by
    margin_step from margin0 (max_rounds margins at most); a margin whose
    band holds no more functions than the last one solved is skipped.  The
    result is converged when two successive solved bands give the same
    number of window eigenvalues, equal within tol, or when a band holds the
    whole basis (then it is the full solve).  Returns (E, converged, margin
    of the last solved band, number of basis functions in it)."""
    n_all = sum(len(x) for x in eps)
    prev = None
    last = -1
    out = (np.zeros(0), False, margin0, 0)
    for r in range(max_rounds):
        d = margin0 + r * margin_step
        keep = select_band(eps, e_lo - d, e_hi + d)
        n = int(keep.sum())
        if n == 0 or n == last:
            continue
        Hs, Ss = subset(H, S, keep)
        E = global_solve(Hs, Ss, tau, e_lo, e_hi)["window"]
        conv = n == n_all or (
            prev is not None and len(prev) == len(E) and
            (len(E) == 0 or np.abs(E - prev).max() <= tol))
        out = (E, conv, d, n)
        if conv:
            break
        prev, last = E, n
    return out


def homo_energies(H, n_states):
    """e_j = <HOMO_j|H|HOMO_j> with the whole-system H, from the diagonal of
    each fragment's diagonal block (the HOMO is its last basis state)."""
    off = np.concatenate([[0], np.cumsum(n_states)])
    return np.array([H[off[j + 1] - 1, off[j + 1] - 1]
                     for j in range(len(n_states))])


def homo_lumo_gap(E, e_ref, gap_min):
    """First gap in the spectrum E above e_ref: scanning upward from the
    first eigenvalue at or above e_ref, the first spacing
    E[k+1] - E[k] >= gap_min; the states up to k are occupied.  Returns
    (n_occ, E_homo, E_lumo), or (-1, nan, nan) when there is no such gap."""
    E = np.sort(np.asarray(E, dtype=float))
    start = int(np.searchsorted(E, e_ref, side="left"))
    for k in range(max(start, 0), len(E) - 1):
        if E[k + 1] - E[k] >= gap_min:
            return k + 1, float(E[k]), float(E[k + 1])
    return -1, math.nan, math.nan


# --------------------------------------------------------------------------
# brute force and closed forms
# --------------------------------------------------------------------------

def full_grid_eigs(V, h, k):
    """Lowest k eigenvalues of the whole-grid Hamiltonian (dense: tiny grids
    only)."""
    nz, ny, nx = V.shape
    H = hamiltonian_box(V, h, (0, 0, 0), (nx, ny, nz), walls="box")
    return sla.eigh(H.toarray(), eigvals_only=True, subset_by_index=[0, k - 1])


def line_spectrum(N, h):
    """Eigenvalues of -1/2 D2 on N points with the wall rule above:
    (15 - 16 cos t + cos 2t) / (12 h^2), t = k pi / (N + 1), k = 1..N."""
    t = np.arange(1, N + 1) * math.pi / (N + 1)
    return (15.0 - 16.0 * np.cos(t) + np.cos(2.0 * t)) / (12.0 * h * h)


def box_spectrum(dims, h, k=None):
    """Sorted eigenvalues of T on a box (sums of the three line spectra)."""
    ex, ey, ez = (line_spectrum(d, h) for d in dims)
    e = (ez[:, None, None] + ey[None, :, None] + ex[None, None, :]).ravel()
    e.sort()
    return e if k is None else e[:k]


# --------------------------------------------------------------------------
# the whole path
# --------------------------------------------------------------------------

@dataclass
class OracleResult:
    eps: list            # per fragment (s_j,)
    phi: list            # per fragment (n_j, s_j)
    hphi: list           # per fragment (n_dil_j, s_j)
    hphi_box: list       # per fragment (dlo, ddims)
    pairs: list          # [(j, n)] j <= n
    S_blocks: list
    H_blocks: list
    H_other: list        # (H Phi_j)^T Phi_n ordering
    H: np.ndarray | None = None
    S: np.ndarray | None = None
    solve: dict | None = None


def window_below_cutoff(eps):
    """Energy window used for the tiny configurations: every OFM eigenvalue
    below the lowest basis cutoff min_j eps_j[s_j - 1]."""
    return -np.inf, float(min(e[-1] for e in eps))


def run(V, h, frag_lo, frag_dims, frag_states, tau=1e-6, window=None,
        states=None, fragments=None, solve=True, d_cut=None, atoms=None,
        frag_atom_ptr=None, frag_atom_idx=None, own=None):
    """Fragment states -> whole-H products -> pair blocks -> global solve.

    ``d_cut`` and the atom lists prune the pair set by atom distance.
    ``own = (origin, Z, sigma, r_cut)`` builds every fragment Hamiltonian
    from the wells of the fragment's own atoms (H|phi> keeps the global V).
    ``states`` may supply (eps, phi) per fragment to skip the eigensolves.
    ``fragments`` restricts the eigensolves / products to a subset (the
    blocks and the global solve then need every fragment they touch)."""
    nz, ny, nx = V.shape
    nf = len(frag_states)
    frag_lo = np.asarray(frag_lo)
    frag_dims = np.asarray(frag_dims)
    todo = range(nf) if fragments is None else fragments
    eps, phi, hphi, hbox = [None] * nf, [None] * nf, [None] * nf, [None] * nf
    for j in todo:
        if states is not None:
            eps[j], phi[j] = states[0][j], states[1][j]
        else:
            vb = None
            if own is not None:   # (origin, Z, sigma, r_cut): own-atoms wells
                o_origin, o_Z, o_sigma, o_rc = own
                vb = own_wells(h, o_origin, frag_lo[j], frag_dims[j], atoms,
                               o_Z, frag_atom_idx[frag_atom_ptr[j]:
                                                  frag_atom_ptr[j + 1]],
                               o_sigma, o_rc)
            eps[j], phi[j] = fragment_states(V, h, frag_lo[j], frag_dims[j],
                                             int(frag_states[j]), Vbox=vb)
        dlo, dd, hp = apply_whole_H(V, h, frag_lo[j], frag_dims[j], phi[j])
        hphi[j], hbox[j] = hp, (dlo, dd)
    pairs = [p for p in pair_list(frag_lo, frag_dims, d_cut=d_cut,
                                  atoms=atoms, frag_atom_ptr=frag_atom_ptr,
                                  frag_atom_idx=frag_atom_idx)
             if phi[p[0]] is not None and phi[p[1]] is not None]
    Sb, Hb, H2 = [], [], []
    for (j, n) in pairs:
        S_, H_, H2_ = pair_blocks(j, n, frag_lo, frag_dims, phi, hphi, hbox)
        Sb.append(S_); Hb.append(H_); H2.append(H2_)
    res = OracleResult(eps, phi, hphi, hbox, pairs, Sb, Hb, H2)
    if solve and fragments is None:
        res.H, res.S = assemble(frag_states, pairs, list(zip(Sb, Hb)))
        if window is None:
            window = window_below_cutoff(eps)
        res.solve = global_solve(res.H, res.S, tau, window[0], window[1])
    return res
