"""Pins of the oracle's fragment states, whole-system H|phi>, pair blocks and
generalised eigenproblem against brute force, closed forms and the
variational principle (Sec. III-B)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from ofm_inputs import box_system, tiny_chain


# ---------------------------------------------------------------- fragments

def test_fragment_states_residual_orthonormal(tiny0, tiny0_oracle):
    s, r = tiny0, tiny0_oracle
    V = s.potential()
    for j in range(s.n_frag):
        H = O.hamiltonian_box(V, s.grid.h, s.frag_lo[j], s.frag_dims[j])
        phi, eps = r.phi[j], r.eps[j]
        assert np.abs(H @ phi - phi * eps).max() < 1e-12
        assert np.abs(phi.T @ phi - np.eye(phi.shape[1])).max() < 1e-13
        assert np.all(np.diff(eps) > 0)
        # gauge: largest component positive
        idx = np.argmax(np.abs(phi), axis=0)
        assert np.all(phi[idx, np.arange(phi.shape[1])] > 0)


def test_fragment_states_v0_closed_form():
    dims = (7, 6, 5)
    V = np.zeros((9, 8, 10))
    eps, phi = O.fragment_states(V, 0.5, (1, 1, 2), dims, 8)
    assert np.allclose(eps, O.box_spectrum(dims, 0.5, 8), atol=1e-12)


def test_arpack_matches_dense():
    rng = np.random.default_rng(7)
    V = -np.abs(rng.standard_normal((16, 16, 16)))
    e1, p1 = O.fragment_states(V, 0.5, (0, 0, 0), (16, 16, 16), 6,
                               dense_max=10 ** 9)
    e2, p2 = O.fragment_states(V, 0.5, (0, 0, 0), (16, 16, 16), 6,
                               dense_max=0)
    assert np.abs(e1 - e2).max() < 1e-12
    # same subspace (gauge-free): projector difference
    assert np.abs(p1 @ p1.T - p2 @ p2.T).max() < 1e-9


# ---------------------------------------------------------------- H|phi>

def _global_sparse(V, h):
    nz, ny, nx = V.shape
    return O.hamiltonian_box(V, h, (0, 0, 0), (nx, ny, nz), walls="box")


def _zero_extend(phi, lo, dims, shape_zyx):
    out = np.zeros(shape_zyx + (phi.shape[1],))
    out[lo[2]:lo[2] + dims[2], lo[1]:lo[1] + dims[1],
        lo[0]:lo[0] + dims[0]] = phi.reshape(dims[2], dims[1], dims[0], -1)
    return out.reshape(-1, phi.shape[1])


def test_hphi_brute_force(tiny0, tiny0_oracle):
    """H_whole @ (zero-extended phi) on the whole grid: equal to the oracle's
    dilated-box product inside the dilated box and exactly zero outside."""
    s, r = tiny0, tiny0_oracle
    V = s.potential()
    Hg = _global_sparse(V, s.grid.h)
    for j in range(s.n_frag):
        B = _zero_extend(r.phi[j], s.frag_lo[j], s.frag_dims[j], V.shape)
        full = (Hg @ B).reshape(V.shape + (-1,))
        dlo, dd = r.hphi_box[j]
        inside = np.zeros(V.shape, bool)
        inside[dlo[2]:dlo[2] + dd[2], dlo[1]:dlo[1] + dd[1],
               dlo[0]:dlo[0] + dd[0]] = True
        got = full[inside]
        ref = r.hphi[j].reshape(dd[2], dd[1], dd[0], -1).reshape(-1, got.shape[1])
        assert np.abs(got - ref).max() < 1e-13
        assert np.array_equal(full[~inside], np.zeros_like(full[~inside]))


def test_hphi_in_box_identity():
    """Inside its own box, H_whole phi = phi eps + D phi where D adds
    +1/(24 h^2) per box face that is not a grid face (the fragment operator
    has the wall term there, the whole-system operator does not)."""
    rng = np.random.default_rng(11)
    V = -np.abs(rng.standard_normal((10, 11, 12)))
    lo, dims, h = (3, 0, 2), (6, 7, 8), 0.5
    eps, phi = O.fragment_states(V, h, lo, dims, 4)
    dlo, dd, hp = O.apply_whole_H(V, h, lo, dims, phi)
    off = np.array(lo) - dlo
    inbox = hp.reshape(dd[2], dd[1], dd[0], -1)[
        off[2]:off[2] + dims[2], off[1]:off[1] + dims[1],
        off[0]:off[0] + dims[0]].reshape(-1, 4)
    cnt = np.zeros((dims[2], dims[1], dims[0]))
    cnt[:, :, 0] += 1
    cnt[:, :, -1] += 1          # x: 3..8 of 12, both faces interior
    cnt[:, -1, :] += 1          # y: 0..6 of 11, lower face is the grid wall
    cnt[0, :, :] += 1           # z: 2..9 of 10, upper face is the grid wall
    D = cnt.ravel() / (24 * h * h)
    assert np.abs(inbox - (phi * eps + D[:, None] * phi)).max() < 1e-12


# ---------------------------------------------------------------- blocks

def test_blocks_brute_force(tiny0, tiny0_oracle):
    """S = B^T B and H = B^T H_whole B with B the zero-extended states of all
    fragments, against the oracle's pair-by-pair assembly."""
    s, r = tiny0, tiny0_oracle
    V = s.potential()
    B = np.hstack([_zero_extend(r.phi[j], s.frag_lo[j], s.frag_dims[j],
                                V.shape) for j in range(s.n_frag)])
    S_ref = B.T @ B
    H_ref = B.T @ (_global_sparse(V, s.grid.h) @ B)
    assert np.abs(r.S - S_ref).max() < 1e-13
    assert np.abs(r.H - 0.5 * (H_ref + H_ref.T)).max() < 1e-13
    assert np.abs(H_ref - H_ref.T).max() < 1e-12


def test_blocks_invariants(tiny0, tiny0_oracle):
    s, r = tiny0, tiny0_oracle
    # both orderings of H agree
    for Hb, H2 in zip(r.H_blocks, r.H_other):
        assert np.abs(Hb - H2).max() < 1e-13
    assert np.abs(np.diag(r.S) - 1).max() < 1e-13
    assert np.abs(r.S).max() <= 1 + 1e-13
    assert np.linalg.eigvalsh(r.S).min() > -1e-13
    # the touching pair (0, 2) (boxes 0..11 and 12..23) has S = 0, H != 0
    k = r.pairs.index((0, 2))
    assert np.array_equal(r.S_blocks[k], np.zeros((6, 6)))
    assert np.abs(r.H_blocks[k]).max() > 1e-3
    # H_jj = diag(eps) + Phi^T D Phi, D = +1/(24 h^2) per interior face
    h = s.grid.h
    for j in range(s.n_frag):
        d = s.frag_dims[j]
        cnt = np.zeros((d[2], d[1], d[0]))
        if s.frag_lo[j, 0] > 0:
            cnt[:, :, 0] += 1
        if s.frag_lo[j, 0] + d[0] < s.grid.nx:
            cnt[:, :, -1] += 1
        D = cnt.ravel() / (24 * h * h)
        closed = np.diag(r.eps[j]) + r.phi[j].T @ (D[:, None] * r.phi[j])
        kk = r.pairs.index((j, j))
        assert np.abs(r.H_blocks[kk] - closed).max() < 1e-12


def test_pair_set_exact():
    """Random boxes on a small grid: every pair left out of the pair list
    has exactly zero S and H blocks (brute force over the whole grid), and
    boxes at distance <= 2 along one axis are always listed."""
    rng = np.random.default_rng(5)
    shape = (20, 14, 12)
    V = -np.abs(rng.standard_normal(shape[::-1]))
    nf = 9
    dims = rng.integers(3, 7, size=(nf, 3))
    lo = np.array([[rng.integers(0, shape[a] - dims[f, a] + 1)
                    for a in range(3)] for f in range(nf)])
    # boxes 7 and 8 sit beside box 6 along x with the same y,z range, their
    # nearest points 2 and 3 spacings away from box 6's last x plane
    lo[6, 0] = 0
    lo[7] = [dims[6, 0] + 1, lo[6, 1], lo[6, 2]]
    lo[8] = [dims[6, 0] + 2, lo[6, 1], lo[6, 2]]
    dims[7, 1:] = dims[6, 1:]
    dims[8, 1:] = dims[6, 1:]
    states = [np.linalg.qr(rng.standard_normal((int(np.prod(d)), 2)))[0]
              for d in dims]
    pairs = set(O.pair_list(lo, dims))
    assert (6, 7) in pairs and (6, 8) not in pairs
    Hg = _global_sparse(V, 0.5)
    B = [_zero_extend(states[f], lo[f], dims[f], V.shape) for f in range(nf)]
    HB = [Hg @ b for b in B]
    for j in range(nf):
        for n in range(j, nf):
            if (j, n) in pairs:
                continue
            assert np.array_equal(B[j].T @ B[n], np.zeros((2, 2)))
            assert np.array_equal(B[j].T @ HB[n], np.zeros((2, 2)))
    assert np.abs(B[6].T @ HB[7]).max() > 0


# ---------------------------------------------------------------- global

def test_global_matches_cholesky_pencil(tiny0_oracle):
    """Nothing is dropped on the tiny case, so the thresholded canonical
    orthogonalisation must equal LAPACK's Cholesky-based generalised
    solver."""
    r = tiny0_oracle
    assert r.solve["n_kept"] == 18
    ref = sla.eigh(r.H, r.S, eigvals_only=True)
    assert np.abs(r.solve["E"] - ref).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_poincare_bound(seed):
    """Variational principle (Sec. III-B): the k-th OFM eigenvalue is never
    below the k-th eigenvalue of the whole-grid Hamiltonian."""
    s = tiny_chain(seed)
    V = s.potential()
    r = O.run(V, s.grid.h, s.frag_lo, s.frag_dims, s.frag_states)
    E = r.solve["E"]
    full = O.full_grid_eigs(V, s.grid.h, len(E))
    assert np.all(E - full >= -1e-12)


def test_nested_bases_monotone():
    """Adding states to every fragment never raises any OFM eigenvalue."""
    s = tiny_chain(0)
    V = s.potential()
    prev = None
    for ns in (3, 5, 6, 8):
        r = O.run(V, s.grid.h, s.frag_lo, s.frag_dims,
                  np.full(3, ns, np.int32))
        E = r.solve["E"]
        if prev is not None:
            assert np.all(E[:len(prev)] <= prev + 1e-12)
        prev = E


def test_whole_grid_fragment_is_exact():
    s = tiny_chain(0)
    V = s.potential()
    r = O.run(V, 0.5, [[0, 0, 0]], [[24, 12, 12]], [6])
    full = O.full_grid_eigs(V, 0.5, 6)
    assert np.abs(r.solve["E"] - full).max() < 1e-12
    # with V = 0 this is the closed-form box spectrum
    r0 = O.run(np.zeros_like(V), 0.5, [[0, 0, 0]], [[24, 12, 12]], [6])
    assert np.abs(r0.solve["E"] - O.box_spectrum((24, 12, 12), 0.5, 6)).max() \
        < 1e-12


def test_duplicate_fragment_drops_its_directions(tiny0_oracle):
    s = tiny_chain(0)
    V = s.potential()
    lo = np.vstack([s.frag_lo, s.frag_lo[1:2]])
    dims = np.vstack([s.frag_dims, s.frag_dims[1:2]])
    st = np.concatenate([s.frag_states, [6]])
    r = O.run(V, 0.5, lo, dims, st)
    assert r.solve["n_kept"] == 18
    assert np.abs(r.solve["E"] - tiny0_oracle.solve["E"]).max() < 1e-10


def test_error_shrinks_with_fragment_width():
    """Three fragments covering the 24-point chain axis: wider boxes (more
    overlap) bring the OFM eigenvalues down toward the whole-grid ones; at
    full width they coincide."""
    s = tiny_chain(0)
    V = s.potential()
    full = O.full_grid_eigs(V, 0.5, 4)
    errs = []
    for w in (8, 12, 16, 20, 24):
        offs = [0, (24 - w) // 2, 24 - w]
        r = O.run(V, 0.5, [[o, 0, 0] for o in offs], [[w, 12, 12]] * 3,
                  [6, 6, 6])
        errs.append(np.abs(r.solve["E"][:4] - full).max())
    assert errs[-1] < 1e-12
    for a, b in zip(errs, errs[1:]):
        assert b <= a * 1.1 + 1e-12


def test_distance_cutoff_pairs(tiny0):
    """Atom-distance pruning (Sec. III-C): on the tiny chain the end
    fragments' closest atoms are one chain spacing (about 2 bohr) apart, so a
    1.5 bohr cutoff drops exactly the pair (0, 2), a 3 bohr cutoff keeps
    everything; brute-force distances decide the same."""
    s = tiny0
    full = O.pair_list(s.frag_lo, s.frag_dims)
    kw = dict(atoms=s.atoms, frag_atom_ptr=s.frag_atom_ptr,
              frag_atom_idx=s.frag_atom_idx)
    assert O.pair_list(s.frag_lo, s.frag_dims, d_cut=3.0, **kw) == full
    cut = O.pair_list(s.frag_lo, s.frag_dims, d_cut=1.5, **kw)
    assert set(full) - set(cut) == {(0, 2)}
    a0 = s.atoms[s.frag_atom_idx[s.frag_atom_ptr[0]:s.frag_atom_ptr[1]]]
    a2 = s.atoms[s.frag_atom_idx[s.frag_atom_ptr[2]:s.frag_atom_ptr[3]]]
    dmin = min(np.linalg.norm(p - q) for p in a0 for q in a2)
    assert 1.5 < dmin < 3.0
    # the pruned pencil is the full one with the (0, 2) blocks zeroed
    r = O.run(s.potential(), 0.5, s.frag_lo, s.frag_dims, s.frag_states,
              d_cut=1.5, **kw)
    assert r.pairs == cut
    ref = O.run(s.potential(), 0.5, s.frag_lo, s.frag_dims, s.frag_states)
    H0 = ref.H.copy()
    H0[0:6, 12:18] = 0.0
    H0[12:18, 0:6] = 0.0
    assert np.array_equal(r.H, H0)
    assert np.array_equal(r.S, ref.S)      # the (0, 2) overlap is zero anyway
    assert np.abs(r.solve["E"] - ref.solve["E"]).max() > 1e-3


def test_own_atoms_fragments(tiny0):
    """Fragment Hamiltonians built from each fragment's own wells: a fragment
    that owns every atom and spans the whole grid sees exactly the global V;
    the OFM pencil built on own-atoms states is still a Galerkin projection
    of the whole-grid H (variational bound), and its H blocks still use the
    global V (brute force)."""
    s = tiny0
    V = s.potential()
    allm = np.arange(len(s.Z))
    Vw = O.own_wells(0.5, s.grid.origin, (0, 0, 0), (24, 12, 12), s.atoms,
                     s.Z, allm)
    assert np.abs(Vw - V).max() < 1e-15
    own = (s.grid.origin, s.Z, 0.8, 8.0)
    kw = dict(atoms=s.atoms, frag_atom_ptr=s.frag_atom_ptr,
              frag_atom_idx=s.frag_atom_idx, own=own)
    r = O.run(V, 0.5, s.frag_lo, s.frag_dims, s.frag_states, **kw)
    full = O.full_grid_eigs(V, 0.5, len(r.solve["E"]))
    assert np.all(r.solve["E"] - full >= -1e-12)
    ref = O.run(V, 0.5, s.frag_lo, s.frag_dims, s.frag_states)
    assert np.abs(np.concatenate(r.eps) - np.concatenate(ref.eps)).max() > 1e-3
    # blocks: B^T H_whole B with the own-atoms states
    Hg = O.hamiltonian_box(V, 0.5, (0, 0, 0), (24, 12, 12))
    B = []
    for j in range(3):
        z = np.zeros((12, 12, 24, 6))
        lo, d = s.frag_lo[j], s.frag_dims[j]
        z[:, :, lo[0]:lo[0] + d[0]] = r.phi[j].reshape(d[2], d[1], d[0], 6)
        B.append(z.reshape(-1, 6))
    B = np.hstack(B)
    Hb = B.T @ (Hg @ B)
    assert np.abs(r.H - 0.5 * (Hb + Hb.T)).max() < 1e-12


# ------------------------------------------------ energy window (reading)

def test_window_below_cutoff_worked_example():
    """Hand-worked window of the tiny configurations: the upper bound is the
    lowest basis cutoff, i.e. the minimum over fragments of each fragment's
    highest kept eigenvalue, and the bound is inclusive.  The fragment
    spectra are chosen so that the maximum over fragments, the minimum of
    the lowest eigenvalues, the last fragment's cutoff or an exclusive bound
    would each select a different set."""
    eps = [np.array([-1.0, -0.5, 0.30]),     # cutoff 0.30
           np.array([-0.8, 0.10]),           # cutoff 0.10  <- the minimum
           np.array([-0.9, -0.2, 0.05, 0.70])]   # cutoff 0.70 (last one)
    lo, hi = O.window_below_cutoff(eps)
    assert lo == -np.inf and hi == 0.10
    # the pencil's eigenvalues: one sits exactly on the cutoff
    E = np.array([-0.95, -0.4, 0.0, 0.10, 0.2, 0.5])
    sel = E[(E >= lo) & (E <= hi)]
    assert sel.tolist() == [-0.95, -0.4, 0.0, 0.10]   # inclusive bound
    # the alternatives a wrong rule would give, to show the example
    # separates them
    assert max(e[-1] for e in eps) == 0.70
    assert min(e[0] for e in eps) == -1.0
    assert eps[-1][-1] == 0.70
    assert E[E < hi].tolist() == [-0.95, -0.4, 0.0]
    # on an oracle run, the window returned is exactly the eigenvalues up to
    # the cutoff, through the same selection
    H = np.diag(E)
    S = np.eye(len(E))
    g = O.global_solve(H, S, 1e-6, lo, hi)
    assert g["window"].tolist() == [-0.95, -0.4, 0.0, 0.10]


# ------------------------------------------- basis near the HOMO (Sec. III-B)

def test_select_top_and_by_gap_worked_examples():
    """Hand-worked masks: the top-n rule and the cut at the first
    substantial gap below each fragment's HOMO."""
    eps = [np.array([-3.0, -2.0, -1.0]), np.array([-5.0, -4.0])]
    assert O.select_top(eps, 2).tolist() == [False, True, True, True, True]
    assert O.select_top(eps, 1).tolist() == [False, False, True, False, True]
    e = [np.array([-3.0, -2.9, -1.0, -0.95])]
    # walking down: 0.05 (no gap), then 1.9 >= 0.5: keep the top two
    assert O.select_by_gap(e, 0.5, 4).tolist() == [False, False, True, True]
    # no gap within the top three: keep three
    assert O.select_by_gap(e, 5.0, 3).tolist() == [False, True, True, True]
    # the gap lies deeper than n_max allows: keep n_max
    assert O.select_by_gap(e, 0.5, 1).tolist() == [False, False, False, True]


def test_homo_lumo_gap_worked_examples():
    E = [-5.0, -4.9, -4.8, -2.0, -1.9]
    assert O.homo_lumo_gap(E, -4.95, 0.5) == (3, -4.8, -2.0)
    # the scan starts at the first level at or above e_ref: above -1.95
    # only -1.9 remains, so there is no gap
    n, lo, hi = O.homo_lumo_gap(E, -1.95, 0.05)
    assert n == -1 and np.isnan(lo) and np.isnan(hi)
    assert O.homo_lumo_gap(E, -10.0, 0.05) == (1, -5.0, -4.9)


def test_homo_energies_and_subset_pencil_brute_force(tiny0, tiny0_oracle):
    """e_j equals the HOMO's expectation value with the whole-grid H (brute
    force on the zero-extended state), and the pencil restricted to a
    selected basis equals the projection of the whole-grid H and identity
    onto those states."""
    s, r = tiny0, tiny0_oracle
    V = s.potential()
    Hg = O.hamiltonian_box(V, 0.5, (0, 0, 0), (24, 12, 12))
    cols = []
    for j in range(3):
        z = np.zeros((12, 12, 24, 6))
        lo, d = s.frag_lo[j], s.frag_dims[j]
        z[:, :, lo[0]:lo[0] + d[0]] = r.phi[j].reshape(d[2], d[1], d[0], 6)
        cols.append(z.reshape(-1, 6))
    B = np.hstack(cols)
    e = O.homo_energies(r.H, s.frag_states)
    for j in range(3):
        b = cols[j][:, -1]
        assert abs(e[j] - b @ (Hg @ b)) < 1e-12
    keep = O.select_top(r.eps, 3)
    Hs, Ss = O.subset(r.H, r.S, keep)
    Bs = B[:, keep]
    assert np.abs(Ss - Bs.T @ Bs).max() < 1e-12
    Hb = Bs.T @ (Hg @ Bs)
    assert np.abs(Hs - 0.5 * (Hb + Hb.T)).max() < 1e-12
    # keeping everything gives the full pencil
    Ha, Sa = O.subset(r.H, r.S, np.ones(len(keep), bool))
    assert np.array_equal(Ha, r.H) and np.array_equal(Sa, r.S)
    # the subset pencil solved directly (Cholesky) agrees with the
    # thresholded solve when nothing is dropped
    g = O.global_solve(Hs, Ss, 1e-6)
    assert g["n_kept"] == int(keep.sum())
    ref = sla.eigh(Hs, Ss, eigvals_only=True)
    assert np.abs(g["E"] - ref).max() < 1e-10


# ------------------------------------- windowed solve of a large basis (f1)

def test_select_band_worked_example():
    """Hand-worked band masks: inclusive bounds, fragment by fragment."""
    eps = [np.array([-1.0, -0.5, 0.2]), np.array([-0.7, 0.0])]
    assert O.select_band(eps, -0.7, 0.0).tolist() == \
        [False, True, False, True, True]
    assert O.select_band(eps, -0.69, -0.01).tolist() == \
        [False, True, False, False, False]
    assert not O.select_band(eps, 1.0, 2.0).any()


def test_window_by_band_exact_when_band_covers_basis(tiny0, tiny0_oracle):
    """A margin that takes every fragment state gives the whole pencil, so
    the windowed solve equals the full thresholded solve exactly."""
    r = tiny0_oracle
    e_all = np.concatenate(r.eps)
    lo, hi = -0.2, 0.3
    full = O.global_solve(r.H, r.S, 1e-6, lo, hi)["window"]
    d = float(e_all.max() - e_all.min()) + 1.0
    E, conv, mg, nsel = O.window_by_band(r.H, r.S, r.eps, lo, hi,
                                        margin0=d, margin_step=0.5,
                                        max_rounds=2)
    assert conv and nsel == len(e_all)
    assert np.array_equal(E, full)


def test_window_by_band_upper_bounds_at_bottom(tiny0, tiny0_oracle):
    """At the bottom of the spectrum the band pencil is a principal
    sub-pencil with S positive definite (nothing dropped), so by Cauchy
    interlacing its k-th eigenvalue is at least the whole pencil's k-th, and
    the bound tightens as the margin grows; the largest margin reproduces
    the whole pencil."""
    r = tiny0_oracle
    full = O.global_solve(r.H, r.S, 1e-6)
    assert full["n_kept"] == r.S.shape[0]
    E_all = full["E"]
    lo, hi = E_all[0] - 1e-9, E_all[0] + 0.05
    prev_err = np.inf
    for d in (0.0, 0.2, 0.5, 1.0, 3.0):
        keep = O.select_band(r.eps, -np.inf, hi + d)
        Hs, Ss = O.subset(r.H, r.S, keep)
        g = O.global_solve(Hs, Ss, 1e-6)
        k = min(3, len(g["E"]))
        assert np.all(g["E"][:k] >= E_all[:k] - 1e-12)
        err = float(np.abs(g["E"][:k] - E_all[:k]).max())
        assert err <= prev_err + 1e-12
        prev_err = err
    assert prev_err < 1e-12
