"""GPU parity of the mixed forms (FP32 vectors and stencil, split-BF16 x3 or
scaled split-FP16 x3 MFMA contractions, FP64 Cholesky / small eigensolves /
global solve; every test runs in both forms) against
the FP64 oracle: eigenvalues within 1e-5 Ha, matrix elements within 1e-6
relative to max|H|; diagonal S blocks exactly the identity for the solver's
states, computed from the states for imported ones."""
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


@pytest.fixture(scope="module", params=["bf16x3", "fp16x3"])
def mctx(request):
    c = P.ofm_create(0, None, request.param)
    yield c
    c.close()


def test_mixed_stencil(mctx):
    _say("mixed stencil")
    rng = np.random.default_rng(3)
    dims = (13, 11, 9)
    shape = (16, 12, 10)
    V = -np.abs(rng.standard_normal(shape[::-1]))
    s = box_system(shape, 0.5, [(1, 1, 0)], [dims], [1], V=V)
    f = _build(mctx, s)
    x = rng.standard_normal((2, int(np.prod(dims))))
    y = P.ofm_apply_fragment_h(mctx, f, 0, x)
    ref = (O.hamiltonian_box(V, 0.5, (1, 1, 0), dims) @ x.T).T
    err = np.abs(y - ref).max() / np.abs(ref).max()
    _say("  rel err", err)
    assert err < 2e-6


def _blocks(r, pj, pn):
    idx = {p: k for k, p in enumerate(r.pairs)}
    Hs, Ss, diag = [], [], []
    for j, n in zip(pj, pn):
        k = idx[(int(j), int(n))]
        Hb, Sb = r.H_blocks[k], r.S_blocks[k]
        if j == n:
            Hb = 0.5 * (Hb + Hb.T)
            Sb = 0.5 * (Sb + Sb.T)
        Hs.append(Hb.ravel())
        Ss.append(Sb.ravel())
        diag.append(np.full(Sb.size, j == n))
    return np.concatenate(Hs), np.concatenate(Ss), np.concatenate(diag)


@pytest.mark.parametrize("case", ["tiny", "random", "random_wide"])
def test_mixed_elements_imported_states(mctx, case):
    _say("mixed elements", case)
    if case == "tiny":
        s = tiny_chain(0)
        V = s.potential()
        lo, dims, st = s.frag_lo, s.frag_dims, s.frag_states
        shape = (s.grid.nx, s.grid.ny, s.grid.nz)
    else:
        rng = np.random.default_rng(21)
        shape = (30, 22, 18)
        V = -np.abs(rng.standard_normal(shape[::-1]))
        dims = rng.integers(5, 12, size=(7, 3))
        lo = np.array([[rng.integers(0, shape[a] - dims[f_, a] + 1)
                        for a in range(3)] for f_ in range(7)])
        st = rng.integers(1, 9, size=7) if case == "random" else \
            rng.integers(14, 41, size=7)
    r = O.run(V, 0.5, lo, dims, st, solve=False)
    s = box_system(shape, 0.5, lo, dims, st, V=V)
    f = _build(mctx, s)
    for j in range(len(st)):
        P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
    pj, pn, off = f.pairs()
    m = P.ofm_matrix_elements(mctx, f)
    H, S = P.ofm_mats_copy(m)
    Hr, Sr, dg = _blocks(r, pj, pn)
    eh = np.abs(H - Hr).max() / np.abs(Hr).max()
    es = np.abs(S - Sr)[~dg].max() if (~dg).any() else 0.0
    _say("  H rel", eh, "S offdiag", es)
    assert eh < 1e-6
    assert es < 1e-6
    # imported states: the diagonal S blocks are computed from the states
    # (FP64 products on their FP32 values), within FP32 rounding of the
    # oracle's Phi_j^T Phi_j = I
    ed = np.abs(S - Sr)[dg].max()
    _say("  S diagonal blocks", ed)
    assert ed < 1e-6


def test_mixed_diag_s_of_non_orthonormal_imports(mctx, tiny0):
    """Imported states are used as given: in the mixed form a fragment whose
    states were imported gets S_jj = Phi_j^T Phi_j (FP64 products on its
    FP32-stored states), not the identity the solver's FP64-orthonormalised
    states receive.  Non-orthonormal imports (oracle states mixed by a
    random non-orthogonal matrix) are checked against the brute-force Gram
    matrix of the same FP32-rounded states; off-diagonal and H blocks keep
    the mixed bound.  After a solve the diagonal S blocks are I again."""
    _say("mixed: diagonal S of non-orthonormal imports")
    s = tiny0
    V = s.potential()
    r = O.run(V, 0.5, s.frag_lo, s.frag_dims, s.frag_states, solve=False)
    rng = np.random.default_rng(17)
    mix = [np.eye(6) + 0.3 * rng.standard_normal((6, 6)) for _ in range(3)]
    phi = [r.phi[j] @ mix[j] for j in range(3)]
    f = _build(mctx, s)
    for j in range(3):
        P.ofm_set_states(f, j, phi[j].T)
    pj, pn, off = f.pairs()
    m = P.ofm_matrix_elements(mctx, f)
    H, S = P.ofm_mats_copy(m)
    m.close()
    hp = {}
    for j in range(3):
        dlo, dd, h_ = O.apply_whole_H(V, 0.5, s.frag_lo[j], s.frag_dims[j],
                                      phi[j])
        hp[j] = (h_, (dlo, dd))
    hmax = np.abs(H).max()   # the bound is relative to max|H_ij|
    for p in range(len(pj)):
        j, n = int(pj[p]), int(pn[p])
        Sb, Hb, _ = O.pair_blocks(j, n, s.frag_lo, s.frag_dims, phi,
                                  {k: hp[k][0] for k in hp},
                                  {k: hp[k][1] for k in hp})
        gS = S[off[p]:off[p] + 36].reshape(6, 6)
        gH = H[off[p]:off[p] + 36].reshape(6, 6)
        if j == n:
            Hb = 0.5 * (Hb + Hb.T)
            p32 = phi[j].astype(np.float32).astype(np.float64)
            ref = p32.T @ p32
            es = np.abs(gS - ref).max() / np.abs(ref).max()
            _say(f"  S_{j}{j} vs Gram of the FP32 states: {es:.2e}")
            assert es < 1e-12
            assert np.abs(gS - np.eye(6)).max() > 0.1   # not the identity
        else:
            es = np.abs(gS - Sb).max() / max(np.abs(Sb).max(), 1e-300)
            assert es < 1e-6
        eh = np.abs(gH - Hb).max() / hmax
        _say(f"  block ({j},{n}): H {eh:.2e} of max|H|")
        assert eh < 1e-6
    st, eps, it, cv = P.ofm_solve_fragments(mctx, f)
    assert st == 0
    m = P.ofm_matrix_elements(mctx, f)
    H, S = P.ofm_mats_copy(m)
    m.close()
    for p in range(len(pj)):
        if pj[p] == pn[p]:
            assert np.array_equal(S[off[p]:off[p] + 36].reshape(6, 6),
                                  np.eye(6))
    f.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mixed_end_to_end_tiny(mctx, seed):
    s = tiny_chain(seed)
    _say("mixed end to end, tiny seed", seed)
    V = s.potential()
    r = O.run(V, s.grid.h, s.frag_lo, s.frag_dims, s.frag_states)
    f = _build(mctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(mctx, f)
    _say("  status", st, "iters", it)
    assert st == 0
    assert np.abs(eps - np.concatenate(r.eps)).max() < 1e-5
    m = P.ofm_matrix_elements(mctx, f)
    g = P.ofm_solve_global(mctx, m, 1e-6, -1e30,
                           O.window_below_cutoff(r.eps)[1])
    err = np.abs(g["E"] - r.solve["window"]).max()
    _say("  window", len(g["E"]), "max err", err)
    assert len(g["E"]) == len(r.solve["window"])
    assert err < 1e-5


def _wells_system(seed):
    """Uneven boxes: three of at most 32 points per axis (one with a full
    32-point z column) take the on-chip filter, one 36 points wide in x
    takes the per-step launches."""
    rng = np.random.default_rng(seed)
    shape = (48, 20, 34)
    h = 0.5
    zz, yy, xx = np.meshgrid(*[np.arange(n) * h for n in shape[::-1]],
                             indexing="ij")
    V = np.zeros(shape[::-1])
    for _ in range(8):
        c = rng.uniform(0, 1, 3) * np.array(shape) * h
        V -= np.exp(-((xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2)
                    / (2 * 0.8 ** 2))
    lo = [(0, 0, 0), (10, 4, 4), (30, 2, 1), (40, 12, 20)]
    dims = [(12, 12, 12), (36, 10, 10), (8, 8, 32), (5, 7, 3)]
    return box_system(shape, h, lo, dims, [6, 4, 5, 2], V=V)


def test_multistep_plane_classes_bit_identical(mctx):
    """FP32 boxes in all five plane classes of the multi-step kernel (1 to 4
    points per thread of a 512-thread workgroup: planes of 480, 900, 1280
    and 1920 points; 3 points per thread of a 1024-thread workgroup: 2100
    points), on-chip filter off: three steps per launch (the
    default) and two, one launch per class, give the same bits as
    one step per launch, graph on and off, and the eigenvalues match the
    oracle's."""
    rng = np.random.default_rng(12)
    shape = (52, 44, 8)
    V = -np.abs(rng.standard_normal(shape[::-1])) * 0.3
    lo = [(0, 0, 0), (10, 8, 1), (4, 6, 2), (2, 2, 3), (1, 1, 4)]
    dims = [(24, 20, 5), (30, 30, 5), (40, 32, 4), (48, 40, 3), (50, 42, 3)]
    st = [3, 4, 3, 4, 3]
    s = box_system(shape, 0.5, lo, dims, st, V=V)
    out = []
    for fused, graph in ((0, 0), (-1, 0), (0, -1), (2, 0), (2, -1)):
        _say("plane classes: fused", fused, "graph", graph)
        f = _build(mctx, s)
        status, eps, it, cv = P.ofm_solve_fragments(
            mctx, f, fused=fused, use_graph=graph, resident=-1)
        assert status == 0 and cv.all()
        out.append((eps, it, [P.ofm_get_states(f, j)[1] for j in range(5)]))
        f.close()
    for eps, it, phis in out[1:]:
        assert np.array_equal(eps, out[0][0])
        assert np.array_equal(it, out[0][1])
        for a, b in zip(phis, out[0][2]):
            assert np.array_equal(a, b)
    r = O.run(V, 0.5, lo, dims, st, solve=False)
    err = np.abs(out[0][0] - np.concatenate(r.eps)).max()
    _say(f"  eps vs oracle {err:.2e} Ha")
    assert err < 1e-5


@pytest.mark.parametrize("seed", [0, 1])
def test_resident_filter_bit_identical(mctx, seed):
    """The on-chip whole-filter kernel and the multi-step kernel (two or
    three steps per launch) give the same bits as the one-step strip
    launches: eigenvalues, iteration counts and states."""
    s = _wells_system(seed)
    out = []
    for res, graph, fused in ((0, 0, 0), (-1, 0, 0), (-1, -1, 0),
                              (-1, 0, -1), (0, 0, -1), (-1, 0, 3)):
        _say("resident", res, "graph", graph, "fused", fused, "seed", seed)
        f = _build(mctx, s)
        st, eps, it, cv = P.ofm_solve_fragments(mctx, f, resident=res,
                                                use_graph=graph, fused=fused)
        assert st == 0 and cv.all()
        phis = [P.ofm_get_states(f, j)[1] for j in range(s.n_frag)]
        out.append((eps, it, phis))
        f.close()
    for eps, it, phis in out[1:]:
        assert np.array_equal(eps, out[0][0])
        assert np.array_equal(it, out[0][1])
        for a, b in zip(phis, out[0][2]):
            assert np.array_equal(a, b)
    # and the eigenvalues agree with the oracle's to the mixed tolerance
    r = O.run(s.potential(), s.grid.h, s.frag_lo, s.frag_dims, s.frag_states,
              solve=False)
    err = np.abs(out[0][0] - np.concatenate(r.eps)).max()
    _say("  eps err vs oracle", err)
    assert err < 1e-5


def test_mixed_homo_basis_subset(mctx, tiny0, tiny0_oracle):
    """Mixed form: the top-2 HOMO basis gives the oracle's subset-pencil
    eigenvalues within 1e-5 Ha."""
    s, r = tiny0, tiny0_oracle
    f = _build(mctx, s)
    st, eps, it, cv = P.ofm_solve_fragments(mctx, f)
    assert st == 0
    keep = P.ofm_select_homo(f, 2)
    ref_keep = O.select_top(r.eps, 2)
    assert np.array_equal(keep, ref_keep)
    m = P.ofm_matrix_elements(mctx, f)
    g = P.ofm_solve_global_subset(mctx, m, keep, 1e-6)
    ref = O.global_solve(*O.subset(r.H, r.S, ref_keep), 1e-6)
    err = np.abs(g["E"] - ref["E"]).max()
    _say("mixed HOMO subset err", err)
    assert err < 1e-5
    m.close()
    f.close()

def test_pair_variants_bit_identical(mctx):
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
        f = _build(mctx, s)
        r = O.run(V, 0.5, lo, dims, st, solve=False)
        for j in range(7):
            P.ofm_set_states(f, j, r.phi[j].T, r.eps[j])
        out = []
        for v in (0, 1):
            P.ofm_set_pair_variant(mctx, v)
            m = P.ofm_matrix_elements(mctx, f)
            out.append(P.ofm_mats_copy(m))
            m.close()
        P.ofm_set_pair_variant(mctx, -1)
        _say("pair variants, max states", int(st.max()))
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1])
        f.close()
