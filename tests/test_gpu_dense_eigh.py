"""GPU parity of the dense FP64 symmetric eigensolver behind the global solve
(own Householder tridiagonal reduction in panels of 32 columns, rocSOLVER's
tridiagonal solvers): eigenvalues against LAPACK's (numpy) and closed forms,
eigenvectors through residual and orthonormality, on sizes that span one to
many panels with ragged tails, and on the degenerate cases of the reduction
(zero columns, diagonal and tridiagonal input, repeated and zero
eigenvalues).

Tolerance: a backward-stable reduction perturbs A by O(n eps ||A||_2), which
moves each eigenvalue by at most that much (Weyl); the tests allow
8 n eps ||A||_2, residuals ||A z - w z|| the same, and |Z^T Z - I| 8 n eps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1011_4764_amd")

EPS = np.finfo(np.float64).eps


def _say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = P.ofm_create(0, None, P.OFM_FP64)
    yield c
    c.close()


def _sym(rng, n):
    a = rng.standard_normal((n, n))
    return (a + a.T) / 2


def _check(A, w, Z, w_ref=None):
    n = A.shape[0]
    norm = max(np.abs(np.linalg.eigvalsh(A)).max() if w_ref is None
               else np.abs(w_ref).max(), 1e-300)
    tol = 8 * n * EPS * norm
    assert np.all(np.diff(w) >= 0), "eigenvalues not ascending"
    if w_ref is not None:
        err = np.abs(w - w_ref).max()
        _say(f"  n={n} max|dw|={err:.2e} tol={tol:.2e}")
        assert err <= tol
    if Z is not None:
        res = np.linalg.norm(A @ Z - Z * w, axis=0).max()
        orth = np.abs(Z.T @ Z - np.eye(n)).max()
        _say(f"  residual {res:.2e} orthonormality {orth:.2e}")
        assert res <= tol
        assert orth <= 8 * n * EPS


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 34, 64, 65, 97, 300, 1025,
                               2049, 2056, 2601])
def test_random_symmetric(ctx, n):
    """Random symmetric matrices: one panel, exact multiples of the panel
    width (n - 1 reflectors = 31, 63, 64, ...), ragged tails; from 2049 on
    the first columns (trailing size >= 2048) take the lower-triangle tiled
    product: one column (2049), eight (2056), and an odd size with ragged
    tiles on both edges (2601)."""
    _say("dense eigh random", n)
    rng = np.random.default_rng(1000 + n)
    A = _sym(rng, n)
    w_ref, Z_ref = np.linalg.eigh(A)
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, w_ref)
    w2, none = P.ofm_dense_eigh(ctx, A)
    assert none is None
    assert np.abs(w2 - w_ref).max() <= 8 * n * EPS * np.abs(w_ref).max()
    # well-separated eigenvalues have eigenvectors unique up to sign
    gaps = np.minimum(np.diff(w_ref, prepend=-np.inf), np.diff(w_ref, append=np.inf))
    sep = gaps > 1e-3 * np.abs(w_ref).max()
    ov = np.abs(np.sum(Z[:, sep] * Z_ref[:, sep], axis=0))
    if ov.size:
        assert ov.min() > 1 - 1e-8


def test_second_difference_closed_form(ctx):
    """Already tridiagonal input, the 1D second difference tridiag(-1, 2, -1):
    eigenvalues 2 - 2 cos(k pi / (n + 1)), k = 1..n."""
    n = 200
    _say("dense eigh second difference", n)
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    k = np.arange(1, n + 1)
    w_ref = np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, w_ref)


def test_diagonal_and_zero_columns(ctx):
    """Diagonal input (every reflector is the identity, tau = 0) and a matrix
    whose columns 5, 40 and 41 are zero below the diagonal block they start
    (xnorm = 0 in the middle of a panel and across a panel boundary)."""
    rng = np.random.default_rng(7)
    d = rng.standard_normal(70)
    _say("dense eigh diagonal")
    w, Z = P.ofm_dense_eigh(ctx, np.diag(d), want_vectors=True)
    _check(np.diag(d), w, Z, np.sort(d))
    A = _sym(rng, 90)
    for c in (5, 40, 41):
        A[c + 1:, c] = 0
        A[c, c + 1:] = 0
    _say("dense eigh zero columns")
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, np.linalg.eigvalsh(A))


def test_zero_columns_in_tiled_columns(ctx):
    """The same degenerate reflectors where the product runs over the lower
    triangle in tiles (trailing size >= 2048): zero columns below the
    diagonal at 3, 31 and 32 (tau = 0 inside and at the end of a panel) of
    a 2100 x 2100 matrix, and a diagonal 2100 x 2100 matrix (every column
    zero, every tile product zero)."""
    n = 2100
    rng = np.random.default_rng(2100)
    A = _sym(rng, n) / np.sqrt(n)
    for c in (3, 31, 32):
        A[c + 1:, c] = 0
        A[c, c + 1:] = 0
    _say("dense eigh zero columns, tiled", n)
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    w_ref = np.linalg.eigvalsh(A)
    tol = 8 * n * EPS * np.abs(w_ref).max()
    err = np.abs(w - w_ref).max()
    _say(f"  max|dw|={err:.2e} tol={tol:.2e}")
    assert err <= tol
    idx = np.linspace(0, n - 1, 16).astype(int)
    res = np.linalg.norm(A @ Z[:, idx] - Z[:, idx] * w[idx], axis=0).max()
    assert res <= tol
    assert np.abs(Z[:, idx].T @ Z - np.eye(n)[idx]).max() <= 8 * n * EPS
    d = rng.standard_normal(n)
    w, _ = P.ofm_dense_eigh(ctx, np.diag(d))
    assert np.abs(w - np.sort(d)).max() <= 8 * n * EPS * np.abs(d).max()


def test_degenerate_spectra(ctx):
    """Zero matrix, identity (one n-fold eigenvalue) and a rank-deficient
    overlap-like Gram matrix B B^T (half its eigenvalues are zero, the
    case the global solve's threshold exists for)."""
    _say("dense eigh zero / identity / rank deficient")
    w, Z = P.ofm_dense_eigh(ctx, np.zeros((40, 40)), want_vectors=True)
    assert np.all(w == 0)
    assert np.abs(Z.T @ Z - np.eye(40)).max() <= 8 * 40 * EPS
    w, Z = P.ofm_dense_eigh(ctx, np.eye(33), want_vectors=True)
    assert np.abs(w - 1).max() <= 8 * 33 * EPS
    _check(np.eye(33), w, Z)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((130, 65)) / np.sqrt(65)
    S = B @ B.T
    w, Z = P.ofm_dense_eigh(ctx, S, want_vectors=True)
    _check(S, w, Z, np.linalg.eigvalsh(S))
    assert np.abs(w[:65]).max() <= 8 * 130 * EPS * w[-1]


def _glued_wilkinson(m, copies, glue):
    """`copies` Wilkinson W_m^+ matrices (diagonal |k - (m-1)/2|, unit
    off-diagonal) glued by off-diagonal entries `glue`: its eigenvalues come
    in pairs and clusters closer than 1e-13."""
    d = np.abs(np.arange(m) - (m - 1) / 2.0)
    D = np.tile(d, copies)
    E = np.ones(m * copies - 1)
    E[m - 1::m] = glue
    return np.diag(D) + np.diag(E, 1) + np.diag(E, -1)


@pytest.mark.parametrize("glue", [1e-8, 1e-14])
def test_glued_wilkinson_clusters(ctx, glue):
    """Glued Wilkinson matrices (tight pairs and clusters of eigenvalues):
    every eigenvalue is bracketed independently on the Sturm count, so the
    count must be monotone in x for the results to come out ascending with
    none counted twice or missed.  Values against LAPACK within the bound,
    ascending, and the multiplicity of each cluster preserved."""
    A = _glued_wilkinson(21, 20, glue)
    n = A.shape[0]
    _say("dense eigh glued Wilkinson", n, "glue", glue)
    w_ref = np.linalg.eigvalsh(A)
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, w_ref)
    # cluster sizes agree (a doubly counted or missed eigenvalue changes one)
    tol = 8 * n * EPS * np.abs(w_ref).max()
    for c in np.unique(np.round(w_ref, 6)):
        assert np.count_nonzero(np.abs(w - c) < 5e-7) == \
            np.count_nonzero(np.abs(w_ref - c) < 5e-7)
    assert np.abs(w - w_ref).max() <= tol


def test_clustered_spectrum(ctx):
    """Many eigenvalues within a few ulps of each other in a random basis
    (three clusters of 60 plus spread values)."""
    n = 300
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([1.0 + 1e-15 * rng.standard_normal(60),
                          -2.0 + 1e-15 * rng.standard_normal(60),
                          0.25 + 1e-15 * rng.standard_normal(60),
                          rng.uniform(-3, 3, n - 180)])
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    _say("dense eigh clustered")
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, np.linalg.eigvalsh(A))


def test_wide_dynamic_range(ctx):
    """Eigenvalues spread over 1e-10 .. 1 in a random orthonormal basis:
    the small ones come out within the absolute bound set by ||A||."""
    n = 257
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(np.logspace(-10, 0, n))
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    _say("dense eigh dynamic range")
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    _check(A, w, Z, np.linalg.eigvalsh(A))


def test_largest_tested_size_sampled(ctx):
    """n = 4096, the alkane workload's basis size (128 panels), values
    against LAPACK, and residual and orthonormality of 16 sampled
    eigenpairs."""
    n = 4096
    rng = np.random.default_rng(4096)
    A = _sym(rng, n) / np.sqrt(n)
    _say("dense eigh", n)
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    w_ref = np.linalg.eigvalsh(A)
    tol = 8 * n * EPS * np.abs(w_ref).max()
    err = np.abs(w - w_ref).max()
    _say(f"  max|dw|={err:.2e} tol={tol:.2e}")
    assert err <= tol
    idx = np.linspace(0, n - 1, 16).astype(int)
    res = np.linalg.norm(A @ Z[:, idx] - Z[:, idx] * w[idx], axis=0).max()
    orth = np.abs(Z[:, idx].T @ Z - np.eye(n)[idx]).max()
    _say(f"  residual {res:.2e} orthonormality {orth:.2e}")
    assert res <= tol
    assert orth <= 8 * n * EPS
    w2, _ = P.ofm_dense_eigh(ctx, A)          # values only: bisection on T
    err2 = np.abs(w2 - w_ref).max()
    _say(f"  values only max|dw|={err2:.2e}")
    assert err2 <= tol


def test_two_slot_rounds_sampled(ctx):
    """n = 6000: the first columns' rows take 6000/256 + 6000/32 > 192 partial
    sums of the tiled product, more than one round of k_fin's slot loads;
    values (with and without vectors) against LAPACK and 16 sampled
    eigenpairs."""
    n = 6000
    rng = np.random.default_rng(6000)
    A = _sym(rng, n) / np.sqrt(n)
    _say("dense eigh", n)
    w, Z = P.ofm_dense_eigh(ctx, A, want_vectors=True)
    w_ref = np.linalg.eigvalsh(A)
    tol = 8 * n * EPS * np.abs(w_ref).max()
    err = np.abs(w - w_ref).max()
    _say(f"  max|dw|={err:.2e} tol={tol:.2e}")
    assert err <= tol
    idx = np.linspace(0, n - 1, 16).astype(int)
    res = np.linalg.norm(A @ Z[:, idx] - Z[:, idx] * w[idx], axis=0).max()
    assert res <= tol
    assert np.abs(Z[:, idx].T @ Z - np.eye(n)[idx]).max() <= 8 * n * EPS
    w2, _ = P.ofm_dense_eigh(ctx, A)
    assert np.abs(w2 - w_ref).max() <= tol


def test_dense_eigh_errors(ctx):
    _say("dense eigh errors")
    with pytest.raises(ValueError):
        P.ofm_dense_eigh(ctx, np.zeros((3, 4)))
    with pytest.raises(P.OfmError) as e:
        P.ofm_dense_eigh(ctx, np.zeros((0, 0)))
    assert e.value.status == P.OFM_E_INVALID
    for bad in (np.nan, np.inf):
        A = np.eye(5)
        A[3, 1] = A[1, 3] = bad
        with pytest.raises(P.OfmError) as e:
            P.ofm_dense_eigh(ctx, A)
        assert e.value.status == P.OFM_E_INVALID
    w, _ = P.ofm_dense_eigh(ctx, np.eye(5))   # the context is still usable
    assert np.allclose(w, 1.0)
