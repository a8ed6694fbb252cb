"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Tolerances: fragment and window eigenvalues 1e-8 Ha
(FP64), matrix elements 1e-10 relative to max|H| (FP64)."""
import numpy as np
import pytest

import oracle as O
from ofm_inputs import box_system, tiny_chain

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1011_4764_amd")


def _say(*a):
    print("[gpu-test]", *a, flush=True)


def _build(ctx, s, V=None):
    V = s.potential() if V is None else V
    return P.ofm_build_fragments(
        ctx, (s.grid.nx, s.grid.ny, s.grid.nz), s.grid.h, V, s.frag_lo,
        s.frag_dims, s.frag_states, origin=s.grid.origin)


@pytest.fixture(scope="module")
def ctx():
    c = P.ofm_create(0, None, P.OFM_FP64)
    yield c
    c.close()


# ------------------------------------------------------------------ stencil

@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("dims", [(12, 12, 12), (7, 5, 9), (48, 40, 3),
                                  (1, 1, 6), (33, 31, 2), (64, 64, 2),
                                  (128, 3, 4), (5, 300, 3)])
def test_fragment_stencil(ctx, dims, variant):
    """H_j x on random vectors vs the oracle's sparse fragment operator:
    ragged boxes, planes from 1 to 4096 points split into strips with halo
    rows, 1-point axes, the widest allowed x extent; every stencil variant."""
    _say("stencil", dims, "variant", variant)
    rng = np.random.default_rng(sum(dims))
    shape = (dims[0] + 3, dims[1] + 2, dims[2] + 1)
    V = rng.standard_normal(shape[::-1])
    lo = (2, 1, 0)
    s = box_system(shape, 0.45, [lo], [dims], [1], V=V)
    f = _build(ctx, s)
    P.ofm_set_stencil_variant(f, variant)
    n = int(np.prod(dims))
    x = rng.standard_normal((3, n))
    y = P.ofm_apply_fragment_h(ctx, f, 0, x)
    H = O.hamiltonian_box(V, 0.45, lo, dims, walls="box")
    ref = (H @ x.T).T
    err = np.abs(y - ref).max() / np.abs(ref).max()
    _say("  rel err", err)
    assert err < 1e-13


# ------------------------------------------------------------------ H|phi>

def test_whole_h_with_imported_states(ctx, tiny0, tiny0_oracle):
    s, r = tiny0, tiny0_oracle
    _say("whole-system H phi, tiny")
    f = _build(ctx, s)
    for j in range(s.n_frag):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    for j in range(s.n_frag):
        lo, dims, dlo, dd, ns = f.geometry(j)
        assert tuple(dlo) == tuple(r.hphi_box[j][0])
        assert tuple(dd) == tuple(r.hphi_box[j][1])
        got = P.ofm_get_hphi(f, j)
        ref = r.hphi[j].T
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max() * 10


# ------------------------------------------------------------------ elements

def _oracle_blocks(r, pj, pn):
    idx = {p: k for k, p in enumerate(r.pairs)}
    Hs, Ss = [], []
    for j, n in zip(pj, pn):
        k = idx[(int(j), int(n))]
        Hb = r.H_blocks[k]
        Sb = r.S_blocks[k]
        if j == n:
            Hb = 0.5 * (Hb + Hb.T)
            Sb = 0.5 * (Sb + Sb.T)
        Hs.append(Hb.ravel())
        Ss.append(Sb.ravel())
    return np.concatenate(Hs), np.concatenate(Ss)


def test_elements_imported_states_tiny(ctx, tiny0, tiny0_oracle):
    s, r = tiny0, tiny0_oracle
    _say("elements, tiny, imported oracle states")
    f = _build(ctx, s)
    for j in range(s.n_frag):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    pj, pn, off = f.pairs()
    assert [(int(a), int(b)) for a, b in zip(pj, pn)] == r.pairs
    m = P.ofm_matrix_elements(ctx, f)
    H, S = P.ofm_mats_copy(m)
    Hr, Sr = _oracle_blocks(r, pj, pn)
    scale = np.abs(Hr).max()
    assert np.abs(H - Hr).max() / scale < 1e-10
    assert np.abs(S - Sr).max() < 1e-10
    # global solve on the same blocks
    g = P.ofm_solve_global(ctx, m, 1e-6)
    ref = O.global_solve(r.H, r.S, 1e-6)
    assert g["n_kept"] == ref["n_kept"]
    assert np.abs(g["E"] - ref["E"]).max() < 1e-10


@pytest.mark.parametrize("srange", [(1, 9), (14, 41)])
def test_elements_random_boxes(ctx, srange):
    """Uneven boxes with halo-only pairs, ragged overlaps and differing state
    counts (1 to 9 MFMA tiles per block); oracle states imported so the
    comparison is gauge-free."""
    _say("elements, random uneven boxes, states", srange)
    rng = np.random.default_rng(21)
    shape = (30, 22, 18)
    V = -np.abs(rng.standard_normal(shape[::-1]))
    nf = 7
    dims = rng.integers(5, 12, size=(nf, 3))
    lo = np.array([[rng.integers(0, shape[a] - dims[f_, a] + 1)
                    for a in range(3)] for f_ in range(nf)])
    states = rng.integers(srange[0], srange[1], size=nf)
    r = O.run(V, 0.5, lo, dims, states, solve=False)
    s = box_system(shape, 0.5, lo, dims, states, V=V)
    f = _build(ctx, s)
    for j in range(nf):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    herr = []
    for j in range(nf):
        e, phi = P.ofm_get_states(f, j)
        assert np.abs(phi - r.phi[j].T).max() == 0.0
        herr.append(np.abs(P.ofm_get_hphi(f, j) - r.hphi[j].T).max())
    _say("  hphi errors per fragment", herr)
    assert max(herr) < 1e-12
    pj, pn, off = f.pairs()
    assert [(int(a), int(b)) for a, b in zip(pj, pn)] == r.pairs
    m = P.ofm_matrix_elements(ctx, f)
    H, S = P.ofm_mats_copy(m)
    Hr, Sr = _oracle_blocks(r, pj, pn)
    _say("  S err", np.abs(S - Sr).max(), "H err", np.abs(H - Hr).max())
    assert np.abs(S - Sr).max() < 1e-10
    assert np.abs(H - Hr).max() / np.abs(Hr).max() < 1e-10


# ------------------------------------------------------------------ eigensolver

def _subspace_gap(A, B):
    """Largest principal-angle sine between column spaces (orthonormal)."""
    sv = np.linalg.svd(A.T @ B, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - sv.min() ** 2)))


def test_fragment_eigenpairs_tiny(ctx, tiny0, tiny0_oracle):
    s, r = tiny0, tiny0_oracle
    _say("eigensolver, tiny")
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    _say("  iters", it, "status", st)
    assert st == 0 and cv.all()
    ref = np.concatenate(r.eps)
    assert np.abs(eps - ref).max() < 1e-8
    for j in range(s.n_frag):
        e, phi = P.ofm_get_states(f, j)
        assert np.abs(phi @ phi.T - np.eye(len(e))).max() < 1e-12
        assert _subspace_gap(phi.T, r.phi[j]) < 1e-7
        # gauge: largest component positive
        idx = np.argmax(np.abs(phi), axis=1)
        assert np.all(phi[np.arange(len(e)), idx] > 0)


def test_end_to_end_tiny_window(ctx, tiny0, tiny0_oracle):
    """Full path on the tiny chain: fragment states, elements, global solve;
    window eigenvalues (below the lowest basis cutoff) within 1e-8 Ha."""
    s, r = tiny0, tiny0_oracle
    _say("end to end, tiny")
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    m = P.ofm_matrix_elements(ctx, f)
    lo, hi = O.window_below_cutoff(r.eps)
    g = P.ofm_solve_global(ctx, m, 1e-6, -1e30, hi)
    ref = r.solve["window"]
    _say("  window", len(g["E"]), "vs", len(ref))
    assert len(g["E"]) == len(ref)
    assert np.abs(g["E"] - ref).max() < 1e-8


@pytest.mark.parametrize("seed", [1, 2])
def test_end_to_end_tiny_seeds(ctx, seed):
    s = tiny_chain(seed)
    _say("end to end, tiny seed", seed)
    V = s.potential()
    r = O.run(V, s.grid.h, s.frag_lo, s.frag_dims, s.frag_states)
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    assert np.abs(eps - np.concatenate(r.eps)).max() < 1e-8
    m = P.ofm_matrix_elements(ctx, f)
    g = P.ofm_solve_global(ctx, m, 1e-6, -1e30, O.window_below_cutoff(r.eps)[1])
    assert np.abs(g["E"] - r.solve["window"]).max() < 1e-8


def test_v0_box_closed_form(ctx):
    """V = 0: fragment eigenvalues equal the closed-form box spectrum
    (degenerate levels: eigenvalues only)."""
    _say("V=0 closed form")
    dims = (10, 9, 8)
    V = np.zeros((8, 9, 10))
    s = box_system((10, 9, 8), 0.5, [(0, 0, 0)], [dims], [5], V=V)
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    assert np.abs(eps - O.box_spectrum(dims, 0.5, 5)).max() < 1e-9


# ------------------------------------------------------------------ errors

def test_error_paths(ctx, tiny0):
    s = tiny0
    _say("error paths")
    with pytest.raises(P.OfmError) as e:
        P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, s.potential(),
                              [[20, 0, 0]], [[12, 12, 12]], [6])
    assert e.value.status == P.OFM_E_INVALID
    Vbad = s.potential().copy()
    Vbad[3, 3, 3] = np.nan
    with pytest.raises(P.OfmError) as e:
        P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, Vbad, s.frag_lo,
                              s.frag_dims, s.frag_states)
    assert e.value.status == P.OFM_E_INVALID
    f = _build(ctx, s)
    with pytest.raises(P.OfmError) as e:
        P.ofm_matrix_elements(ctx, f)
    assert e.value.status == P.OFM_E_STATE
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f, max_iter=1)
    assert st == P.OFM_E_NOCONV and not cv.all()


def test_apply_rejects_too_many_vectors(ctx, tiny0):
    """nvec above OFM_MAX_APPLY_VECTORS (the stencil's tiles carry the vector
    index in 15 bits) is rejected before any device work; the buffers are
    never read, so a one-element buffer suffices."""
    import ctypes as C
    _say("apply: nvec bound")
    f = _build(ctx, tiny0)
    one = np.zeros(1)
    dp = one.ctypes.data_as(C.POINTER(C.c_double))
    for nvec in (P.OFM_MAX_APPLY_VECTORS + 1, 1 << 20, 0, -1):
        st = P.lib().ofm_apply_fragment_h(ctx.handle, f.handle, 0, nvec, dp, dp)
        assert st == P.OFM_E_INVALID, nvec
    # the context stays usable
    x = np.random.default_rng(0).standard_normal((2, 12 ** 3))
    y = P.ofm_apply_fragment_h(ctx, f, 0, x)
    H = O.hamiltonian_box(tiny0.potential(), 0.5, tiny0.frag_lo[0],
                          tiny0.frag_dims[0])
    assert np.abs(y - (H @ x.T).T).max() < 1e-12 * np.abs(y).max()


def test_shifted_cholesky_flagged_and_converges(ctx, tiny0):
    """A filter of degree 128 on small boxes (8^3, 4 states, block of 12)
    makes the filtered block numerically rank deficient, so the CholQR
    Cholesky loses a pivot and the shifted factorisation takes over (a CPU
    model of the solver flags 15 of 16 such boxes and converges on all).
    The solve reports it per fragment in ofm_solve_flags (bit 0), no block
    stays rank deficient (bit 1), and every fragment converges to the
    oracle's eigenvalues.  A default solve afterwards clears the flags."""
    _say("shifted Cholesky path, degree 128")
    V = tiny0.potential()
    lo = [(2 * k, 2, 2) for k in range(8)]
    dims = [(8, 8, 8)] * 8
    st = [4] * 8
    s = box_system((24, 12, 12), 0.5, lo, dims, st, V=V)
    f = _build(ctx, s)
    assert (P.ofm_solve_flags(f) == 0).all()
    status, eps, it, cv = P.ofm_solve_fragments(ctx, f, degree=128)
    fl = P.ofm_solve_flags(f)
    _say("  flags", fl.tolist(), "iterations", it.tolist())
    assert status == 0 and cv.all()
    assert (fl & 1).any()
    assert not (fl & 2).any()
    for j in range(8):
        e_o, _ = O.fragment_states(V, 0.5, lo[j], dims[j], 4)
        assert np.abs(eps[4 * j:4 * j + 4] - e_o).max() < 1e-8
    status, eps2, it, cv = P.ofm_solve_fragments(ctx, f)
    assert status == 0 and cv.all()
    assert np.abs(eps2 - eps).max() < 1e-8
    fl2 = P.ofm_solve_flags(f)
    _say("  flags at the default degree", fl2.tolist())
    assert not (fl2 & 2).any()


# ------------------------------------------------------------------ global solve

def _run_path(ctx, lo, dims, st, V, h=0.5):
    s = box_system((V.shape[2], V.shape[1], V.shape[0]), h, lo, dims, st, V=V)
    f = _build(ctx, s)
    r = O.run(V, h, lo, dims, st, solve=False)
    for j in range(len(st)):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    return f, r


def test_global_duplicate_fragment_drops_directions(ctx, tiny0):
    """A duplicated fragment makes S exactly singular in s_j directions: the
    GPU keeps the same count as the oracle and the same eigenvalues."""
    _say("global solve, duplicated fragment")
    s = tiny0
    V = s.potential()
    lo = np.vstack([s.frag_lo, s.frag_lo[1:2]])
    dims = np.vstack([s.frag_dims, s.frag_dims[1:2]])
    st = np.concatenate([s.frag_states, [6]])
    f, r = _run_path(ctx, lo, dims, st, V)
    m = P.ofm_matrix_elements(ctx, f)
    H, S = P.ofm_mats_copy(m)
    Hd, Sd = P.unpack_blocks(f, H, S)
    ref = O.global_solve(Hd, Sd, 1e-6)
    g = P.ofm_solve_global(ctx, m, 1e-6)
    _say("  kept", g["n_kept"], "oracle", ref["n_kept"])
    assert g["n_kept"] == ref["n_kept"] == 18
    assert np.abs(g["E"] - ref["E"]).max() < 1e-8
    assert abs(g["s_min"] - ref["s_min_kept"]) < 1e-10


def test_global_direct_path_and_vectors(ctx, tiny0, tiny0_oracle):
    """Nothing is dropped on the tiny case, so thresholds 1e-6 and 0 agree;
    the returned coefficients solve H c = E S c with c^T S c = 1."""
    _say("global solve, thresholds and vectors")
    s, r = tiny0, tiny0_oracle
    f = _build(ctx, s)
    for j in range(s.n_frag):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    m = P.ofm_matrix_elements(ctx, f)
    g1 = P.ofm_solve_global(ctx, m, 1e-6, want_vectors=True)
    g0 = P.ofm_solve_global(ctx, m, 0.0)
    assert np.abs(g1["E"] - g0["E"]).max() < 1e-10
    H, S = P.ofm_mats_copy(m)
    Hd, Sd = P.unpack_blocks(f, H, S)
    Cm = g1["C"]
    res = Hd @ Cm - (Sd @ Cm) * g1["E"]
    assert np.abs(res).max() < 1e-9
    assert np.abs(np.diag(Cm.T @ Sd @ Cm) - 1).max() < 1e-10


def test_graph_replay_and_variants_bit_identical(ctx):
    """The HIP-graph replay of the filter sweep, one-by-one launches and every
    stencil variant compute the same values bit for bit (uneven boxes, two
    strips per plane for the smaller variants)."""
    _say("graph replay / stencil variants")
    rng = np.random.default_rng(8)
    shape = (40, 36, 20)
    V = -np.abs(rng.standard_normal(shape[::-1]))
    lo = [(0, 0, 0), (14, 10, 4), (20, 16, 6)]
    dims = [(22, 20, 12), (19, 24, 14), (20, 20, 14)]
    st = [5, 7, 4]
    s = box_system(shape, 0.5, lo, dims, st, V=V)
    outs = []
    for use_graph, variant in [(0, -1), (-1, 0), (0, 1), (-1, 2)]:
        f = _build(ctx, s)
        if variant >= 0:
            P.ofm_set_stencil_variant(f, variant)
        stt, eps, it, cv = P.ofm_solve_fragments(ctx, f, use_graph=use_graph)
        assert stt == 0
        outs.append((eps, [P.ofm_get_states(f, j)[1] for j in range(3)]))
        f.close()
    for eps, phis in outs[1:]:
        assert np.array_equal(eps, outs[0][0])
        for a, b in zip(phis, outs[0][1]):
            assert np.array_equal(a, b)
    ref = O.run(V, 0.5, lo, dims, st, solve=False)
    assert np.abs(outs[0][0] - np.concatenate(ref.eps)).max() < 1e-8


@pytest.mark.parametrize("d_cut", [1.5, 3.0])
def test_distance_cutoff_end_to_end(ctx, tiny0, d_cut):
    """The planner's atom-distance pruning gives the oracle's pair list, and
    the pruned basis gives the oracle's pruned window eigenvalues."""
    s = tiny0
    _say("d_cut", d_cut)
    kw = dict(atoms=s.atoms, frag_atom_ptr=s.frag_atom_ptr,
              frag_atom_idx=s.frag_atom_idx)
    r = O.run(s.potential(), 0.5, s.frag_lo, s.frag_dims, s.frag_states,
              d_cut=d_cut, **kw)
    f = P.ofm_build_fragments(
        ctx, (24, 12, 12), 0.5, s.potential(), s.frag_lo, s.frag_dims,
        s.frag_states, atom_xyz=s.atoms, frag_atom_ptr=s.frag_atom_ptr,
        frag_atom_idx=s.frag_atom_idx, d_cut=d_cut)
    pj, pn, off = f.pairs()
    assert [(int(a), int(b)) for a, b in zip(pj, pn)] == r.pairs
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    m = P.ofm_matrix_elements(ctx, f)
    g = P.ofm_solve_global(ctx, m, 1e-6, -1e30,
                           O.window_below_cutoff(r.eps)[1])
    assert np.abs(g["E"] - r.solve["window"]).max() < 1e-8


def test_own_atoms_end_to_end(ctx, tiny0):
    """Fragment Hamiltonians built from each fragment's own wells: the
    fragment eigenpairs, the blocks (whole-system V in H|phi>) and the
    window eigenvalues match the oracle run with the same own-atoms
    fragments."""
    s = tiny0
    V = s.potential()
    own = (s.grid.origin, s.Z, 0.8, 8.0)
    r = O.run(V, 0.5, s.frag_lo, s.frag_dims, s.frag_states, atoms=s.atoms,
              frag_atom_ptr=s.frag_atom_ptr, frag_atom_idx=s.frag_atom_idx,
              own=own)
    f = P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, V, s.frag_lo,
                              s.frag_dims, s.frag_states, origin=s.grid.origin)
    P.ofm_set_fragment_wells(f, s.atoms, s.Z, s.frag_atom_ptr,
                             s.frag_atom_idx, sigma=0.8, r_cut=8.0)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0 and cv.all()
    err = np.abs(eps - np.concatenate(r.eps)).max()
    _say("own-atoms eps err", err)
    assert err < 1e-8
    m = P.ofm_matrix_elements(ctx, f)
    g = P.ofm_solve_global(ctx, m, 1e-6, -1e30,
                           O.window_below_cutoff(r.eps)[1])
    assert np.abs(g["E"] - r.solve["window"]).max() < 1e-8
    m.close()
    # with the oracle's states imported (gauge-free), H|phi> still uses the
    # whole-system V: blocks match the oracle's to 1e-10
    for j in range(s.n_frag):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    pj, pn, off = f.pairs()
    m = P.ofm_matrix_elements(ctx, f)
    H, S = P.ofm_mats_copy(m)
    Hr, Sr = _oracle_blocks(r, pj, pn)
    assert np.abs(H - Hr).max() < 1e-10 * np.abs(Hr).max()
    assert np.abs(S - Sr).max() < 1e-10
    m.close()
    f.close()


def test_own_atoms_whole_grid_is_global_v(ctx, tiny0):
    """One fragment spanning the grid that owns every atom sees exactly the
    global V: its eigenpairs equal those of the global-V fragment."""
    s = tiny0
    V = s.potential()
    lo = np.zeros((1, 3), np.int64)
    dims = np.array([[24, 12, 12]])
    nst = np.array([8])
    out = []
    for own in (False, True):
        f = P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, V, lo, dims, nst,
                                  origin=s.grid.origin)
        if own:
            P.ofm_set_fragment_wells(f, s.atoms, s.Z, [0, len(s.Z)],
                                     np.arange(len(s.Z)))
        st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
        assert st == 0
        out.append(eps)
        f.close()
    assert np.abs(out[0] - out[1]).max() < 1e-10


def test_own_atoms_invalid(ctx, tiny0):
    s = tiny0
    f = P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, s.potential(),
                              s.frag_lo, s.frag_dims, s.frag_states)
    bad = np.array(s.frag_atom_idx, copy=True)
    bad[0] = len(s.Z)
    with pytest.raises(P.OfmError, match="OFM_E_INVALID"):
        P.ofm_set_fragment_wells(f, s.atoms, s.Z, s.frag_atom_ptr, bad)
    with pytest.raises(P.OfmError, match="OFM_E_INVALID"):
        P.ofm_set_fragment_wells(f, s.atoms, s.Z, s.frag_atom_ptr,
                                 s.frag_atom_idx, sigma=0.0)
    f.close()


# ------------------------------------------- basis near the HOMO (Sec. III-B)

@pytest.mark.parametrize("rule", ["top3", "gap"])
def test_homo_basis_subset(ctx, tiny0, tiny0_oracle, rule):
    """Keep masks from the GPU's fragment eigenvalues equal the oracle's;
    with the oracle's states imported, the HOMO energies match to 1e-12 of
    max|H| and the subset pencil's eigenvalues to 1e-10; the gap above the
    HOMO energies is the oracle's."""
    s, r = tiny0, tiny0_oracle
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    if rule == "top3":
        keep = P.ofm_select_homo(f, 3)
        ref_keep = O.select_top(r.eps, 3)
    else:
        gap = 0.05
        keep = P.ofm_select_homo(f, 6, gap)
        ref_keep = O.select_by_gap(r.eps, gap, 6)
    _say("keep", rule, int(keep.sum()), "of", keep.size)
    assert np.array_equal(keep, ref_keep)
    for j in range(s.n_frag):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    m = P.ofm_matrix_elements(ctx, f)
    e = P.ofm_homo_energies(m)
    e_ref = O.homo_energies(r.H, s.frag_states)
    assert np.abs(e - e_ref).max() < 1e-12 * np.abs(r.H).max()
    g = P.ofm_solve_global_subset(ctx, m, keep, 1e-6)
    Hs, Ss = O.subset(r.H, r.S, ref_keep)
    ref = O.global_solve(Hs, Ss, 1e-6)
    assert g["n_kept"] == ref["n_kept"]
    assert np.abs(g["E"] - ref["E"]).max() < 1e-10
    got_gap = P.ofm_homo_lumo_gap(g["E"], float(e.max()), 0.02)
    ref_gap = O.homo_lumo_gap(ref["E"], float(e_ref.max()), 0.02)
    _say("gap", got_gap, ref_gap)
    assert got_gap[0] == ref_gap[0]
    if ref_gap[0] >= 0:
        assert abs(got_gap[1] - ref_gap[1]) < 1e-10
        assert abs(got_gap[2] - ref_gap[2]) < 1e-10
    # keeping everything is the plain solve
    ga = P.ofm_solve_global_subset(ctx, m, np.ones(keep.size, bool), 1e-6)
    gb = P.ofm_solve_global(ctx, m, 1e-6)
    assert np.array_equal(ga["E"], gb["E"])
    m.close()
    f.close()


def test_homo_subset_errors(ctx, tiny0):
    s = tiny0
    f = _build(ctx, s)
    with pytest.raises(P.OfmError, match="OFM_E_STATE"):
        P.ofm_select_homo(f, 3)           # no states yet
    P.ofm_solve_fragments(ctx, f)
    with pytest.raises(P.OfmError, match="OFM_E_INVALID"):
        P.ofm_select_homo(f, 0)
    m = P.ofm_matrix_elements(ctx, f)
    with pytest.raises(P.OfmError, match="OFM_E_INVALID"):
        P.ofm_solve_global_subset(ctx, m, np.zeros(f.n_basis, bool))
    m.close()
    f.close()


def test_widest_block_end_to_end(ctx):
    """The widest supported block (58 states + 6 guard vectors = 64: 4x4
    Gram tiles, 64-wide rotations, 64x64 Jacobi, 4x4 pair tiles) on two
    overlapping ragged boxes: eigenvalues within 1e-8 Ha and the window of
    the global solve within 1e-8 Ha of the oracle."""
    rng = np.random.default_rng(64)
    shape = (17, 11, 12)
    V = -np.abs(rng.standard_normal(shape[::-1])) * 0.5
    lo = [(0, 0, 0), (6, 1, 1)]
    dims = [(11, 10, 11), (11, 10, 10)]
    states = [58, 58]
    s = box_system(shape, 0.5, lo, dims, states, V=V)
    r = O.run(V, 0.5, lo, dims, states)
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    _say("widest block: iterations", it, "status", st)
    assert st == 0 and cv.all()
    err = np.abs(eps - np.concatenate(r.eps)).max()
    _say("  eps err", err)
    assert err < 1e-8
    m = P.ofm_matrix_elements(ctx, f)
    g = P.ofm_solve_global(ctx, m, 1e-6, -1e30, O.window_below_cutoff(r.eps)[1])
    assert len(g["E"]) == len(r.solve["window"])
    assert np.abs(g["E"] - r.solve["window"]).max() < 1e-8
    m.close()
    f.close()


@pytest.mark.parametrize("case", ["tiny", "wide", "split"])
def test_multistep_bit_identical(ctx, tiny0, case):
    """Three (the default) or two filter steps per launch give the same bits
    as one step per launch (eigenvalues, iteration counts, states), graph on
    and off; planes of 144 to 2208 points: every FP64 launch class of the
    multi-step kernel (144, 900, 1200 and 1800 points) beside a plane over
    its limit of 2048 points (strips) in one sweep."""
    if case == "tiny":
        s = tiny0
    elif case == "split":
        rng = np.random.default_rng(8)
        shape = (60, 52, 12)
        V = -np.abs(rng.standard_normal(shape[::-1])) * 0.3
        s = box_system(shape, 0.5,
                       [(0, 0, 0), (30, 20, 0), (10, 8, 4), (20, 20, 7),
                        (0, 4, 8)],
                       [(48, 46, 3), (12, 12, 12), (40, 30, 4), (30, 30, 4),
                        (45, 40, 4)],
                       [4, 5, 4, 3, 4], V=V)
    else:
        rng = np.random.default_rng(7)
        shape = (40, 34, 14)
        V = -np.abs(rng.standard_normal(shape[::-1])) * 0.3
        s = box_system(shape, 0.5, [(0, 0, 0), (16, 17, 1)],
                       [(32, 32, 10), (20, 15, 12)], [5, 4], V=V)
    out = []
    for fused, graph in ((0, 0), (-1, 0), (0, -1), (2, 0), (2, -1)):
        _say("fused", fused, "graph", graph, case)
        f = _build(ctx, s)
        st, eps, it, cv = P.ofm_solve_fragments(ctx, f, fused=fused,
                                                use_graph=graph)
        assert st == 0 and cv.all()
        out.append((eps, it, [P.ofm_get_states(f, j)[1]
                              for j in range(s.n_frag)]))
        f.close()
    for eps, it, phis in out[1:]:
        assert np.array_equal(eps, out[0][0])
        assert np.array_equal(it, out[0][1])
        for a, b in zip(phis, out[0][2]):
            assert np.array_equal(a, b)
    if case != "tiny":
        r = O.run(s.potential(), 0.5, s.frag_lo, s.frag_dims, s.frag_states,
                  solve=False)
        assert np.abs(out[0][0] - np.concatenate(r.eps)).max() < 1e-8


def test_more_error_paths(ctx, tiny0):
    """Rejected inputs and states: every one returns its status, and the
    context stays usable afterwards."""
    s = tiny0
    V = s.potential()
    bad = [
        ([[0, 0, 0]], [[12, 12, 12]], [65]),     # more than 64 states
        ([[0, 0, 0]], [[12, 12, 12]], [0]),      # no states
        ([[0, 0, 0]], [[2, 2, 2]], [9]),         # more states than points
        ([[0, 0, 0]], [[0, 12, 12]], [1]),       # empty box
    ]
    for lo, dims, st in bad:
        with pytest.raises(P.OfmError) as e:
            P.ofm_build_fragments(ctx, (24, 12, 12), 0.5, V, lo, dims, st)
        assert e.value.status == P.OFM_E_INVALID
    big = np.zeros((4, 4, 130))
    with pytest.raises(P.OfmError) as e:            # x extent above 128
        P.ofm_build_fragments(ctx, (130, 4, 4), 0.5, big, [[0, 0, 0]],
                              [[130, 4, 4]], [1])
    assert e.value.status == P.OFM_E_INVALID
    f = _build(ctx, s)
    # the context refuses to go away while its fragments live
    assert P.lib().ofm_destroy(ctx.handle) == P.OFM_E_STATE
    with pytest.raises(P.OfmError) as e:
        P.ofm_get_states(f, 0)                      # no states yet
    assert e.value.status == P.OFM_E_STATE
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    with pytest.raises(P.OfmError) as e:
        P.ofm_get_states(f, s.n_frag)               # fragment out of range
    assert e.value.status == P.OFM_E_INVALID
    m = P.ofm_matrix_elements(ctx, f)
    with pytest.raises(P.OfmError) as e:            # nothing reaches tau
        P.ofm_solve_global(ctx, m, 1e30)
    assert e.value.status == P.OFM_E_SINGULAR
    g = P.ofm_solve_global(ctx, m, 1e-6)            # still usable
    assert len(g["E"]) == s.n_basis
    m.close()
    f.close()


def test_two_contexts_in_flight_bit_identical(tiny0):
    """Two contexts on two streams driven from two host threads at once (the
    bench's throughput mode): every step returns the serial run's fragment
    eigenvalues, blocks and global eigenvalues bit for bit."""
    import threading
    _say("two contexts in flight")
    s = tiny0

    def run(cx):
        f = _build(cx, s)
        st, eps, it, cv = P.ofm_solve_fragments(cx, f)
        m = P.ofm_matrix_elements(cx, f)
        H, S = P.ofm_mats_copy(m)
        E = P.ofm_solve_global(cx, m, 1e-6)["E"]
        m.close()
        f.close()
        return eps, H, S, E

    c0 = P.ofm_create(0, None, P.OFM_FP64)
    ref = run(c0)
    c1 = P.ofm_create(0, None, P.OFM_FP64)
    out, err = [None] * 6, []

    def worker(cx, first):
        try:
            for k in range(first, 6, 2):
                out[k] = run(cx)
        except Exception as e:
            err.append(e)

    th = [threading.Thread(target=worker, args=(cx, i))
          for i, cx in enumerate((c0, c1))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    c1.close()
    c0.close()
    assert not err, err
    for o in out:
        for a, b in zip(o, ref):
            assert np.array_equal(a, b)


def test_new_contexts_while_another_thread_captures(tiny0):
    """Contexts created and driven in one thread (each with a fresh rocBLAS
    handle, whose first calls initialise its back end) while another thread
    solves fragment sets over and over (each solve captures its sweep as a
    HIP graph): the library serialises captures with BLAS calls, so both
    threads finish and every global solve returns the serial eigenvalues."""
    import threading
    _say("new contexts while another thread captures")
    s = tiny0

    def whole(cx):
        f = _build(cx, s)
        P.ofm_solve_fragments(cx, f)
        m = P.ofm_matrix_elements(cx, f)
        E = P.ofm_solve_global(cx, m, 1e-6)["E"]
        m.close()
        f.close()
        return E

    c0 = P.ofm_create(0, None, P.OFM_FP64)
    ref = whole(c0)
    out, err = [], []

    def capturer():
        try:
            for _ in range(6):
                f = _build(c0, s)
                P.ofm_solve_fragments(c0, f)
                f.close()
        except Exception as e:
            err.append(e)

    def creator():
        try:
            for _ in range(4):
                cx = P.ofm_create(0, None, P.OFM_FP64)
                out.append(whole(cx))
                cx.close()
        except Exception as e:
            err.append(e)

    th = [threading.Thread(target=capturer), threading.Thread(target=creator)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    c0.close()
    assert not err, err
    assert len(out) == 4
    for E in out:
        assert np.array_equal(E, ref)

def test_pair_variants_bit_identical(ctx):
    """Both variants of the pair-contraction kernels (a chunk loaded, then
    multiplied; or the next chunk's loads in flight during the products) give
    the same blocks bit for bit, on uneven boxes with halo-only pairs and
    blocks up to 40 states wide (both work splits of the kernels)."""
    rng = np.random.default_rng(31)
    shape = (30, 22, 18)
    V = -np.abs(rng.standard_normal(shape[::-1]))
    dims = rng.integers(5, 12, size=(7, 3))
    lo = np.array([[rng.integers(0, shape[a] - dims[f_, a] + 1)
                    for a in range(3)] for f_ in range(7)])
    for st in (rng.integers(1, 9, size=7), rng.integers(14, 41, size=7)):
        s = box_system(shape, 0.5, lo, dims, st, V=V)
        f = _build(ctx, s)
        r = O.run(V, 0.5, lo, dims, st, solve=False)
        for j in range(7):
            P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
        out = []
        for v in (0, 1):
            P.ofm_set_pair_variant(ctx, v)
            m = P.ofm_matrix_elements(ctx, f)
            out.append(P.ofm_mats_copy(m))
            m.close()
        P.ofm_set_pair_variant(ctx, -1)
        _say("pair variants, max states", int(st.max()))
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1])
        f.close()


def test_band_selection_and_windowed_solve(ctx, tiny0, tiny0_oracle):
    """The band mask equals the oracle's on the solver's fragment
    eigenvalues; the windowed solve equals the oracle's windowed solve of
    the same (GPU) blocks, round by round the same margin, and a band that
    covers the basis reproduces the full solve."""
    _say("band selection and windowed solve")
    s = tiny0
    f = _build(ctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
    assert st == 0
    boff = np.concatenate([[0], np.cumsum(s.frag_states)])
    eps_list = [eps[boff[j]:boff[j + 1]] for j in range(s.n_frag)]
    for lo, hi in ((-0.3, 0.4), (0.1, 0.6), (5.0, 6.0)):
        assert np.array_equal(P.ofm_select_band(f, lo, hi),
                              O.select_band(eps_list, lo, hi))
    m = P.ofm_matrix_elements(ctx, f)
    Hb, Sb = P.ofm_mats_copy(m)
    H, S = P.unpack_blocks(f, Hb, Sb)
    lo, hi = -0.3, 0.25
    ref = O.window_by_band(H, S, eps_list, lo, hi, margin0=0.05,
                           margin_step=0.1, max_rounds=8, tol=1e-9)
    got = P.ofm_solve_global_window(ctx, m, lo, hi, margin0=0.05,
                                    margin_step=0.1, max_rounds=8, tol=1e-9)
    _say(f"  windowed: {len(got['E'])} eigenvalues, margin {got['margin']}, "
         f"{got['n_sel']} functions; oracle margin {ref[2]}, {ref[3]}")
    assert got["status"] == (0 if ref[1] else P.OFM_E_NOCONV)
    assert abs(got["margin"] - ref[2]) < 1e-12 and got["n_sel"] == ref[3]
    assert len(got["E"]) == len(ref[0])
    assert np.abs(got["E"] - ref[0]).max() < 1e-8
    full = P.ofm_solve_global(ctx, m, 1e-6, lo, hi)["E"]
    wide = P.ofm_solve_global_window(ctx, m, lo, hi, margin0=10.0,
                                     margin_step=1.0, max_rounds=2)
    assert wide["status"] == 0 and wide["n_sel"] == s.n_basis
    assert np.abs(wide["E"] - full).max() < 1e-12
    with pytest.raises(P.OfmError):
        P.ofm_solve_global_window(ctx, m, hi, lo)
    with pytest.raises(P.OfmError):
        P.ofm_solve_global_window(ctx, m, lo, hi, margin_step=0.0)
    m.close()
    f.close()
