"""Pins of the oracle's finite-difference Hamiltonian against facts fixed by
the mathematics: exactness on low-degree polynomials, sine-mode
eigenvectors with the closed-form spectrum, O(h^4) convergence to the
continuum particle in a box, and symmetry."""
import math

import numpy as np
import pytest

import oracle as O


def _grid_fn(dims, h, f):
    x = h * np.arange(dims[0])
    y = h * np.arange(dims[1])
    z = h * np.arange(dims[2])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return f(X, Y, Z)


def test_polynomial_exactness_interior():
    """A 4th-order central second difference is exact on polynomials of
    degree <= 5.  At points at least two from every face (no ghost used),
    T f = -1/2 Laplacian f exactly, per axis and mixed."""
    dims, h = (9, 8, 7), 0.37
    T = O.kinetic_box(dims, (0, 0, 0), dims, h)
    f = _grid_fn(dims, h, lambda X, Y, Z: X ** 5 - 2 * X ** 2 * Y ** 3
                 + 3 * Y * Z ** 4 + Z ** 2 + 1.5)
    lap = _grid_fn(dims, h, lambda X, Y, Z: 20 * X ** 3 - 4 * Y ** 3
                   - 12 * X ** 2 * Y + 36 * Y * Z ** 2 + 2)
    out = (T @ f.ravel()).reshape(dims[::-1])
    inner = (slice(2, -2),) * 3
    assert np.allclose(out[inner], -0.5 * lap[inner], rtol=1e-9, atol=1e-8)


def test_line_spectrum_closed_form():
    """With walls one spacing outside and odd-image second ghosts, sin(pi k
    (i+1)/(N+1)) is an exact eigenvector of the 1-D operator with eigenvalue
    (15 - 16 cos t + cos 2t)/(12 h^2), t = k pi/(N+1)."""
    for N in (1, 2, 3, 5, 12, 24):
        h = 0.5
        A = (-0.5 * O.d2_line(N, h)).toarray()
        ev = np.linalg.eigvalsh(A)
        t = np.arange(1, N + 1) * math.pi / (N + 1)
        closed = (15 - 16 * np.cos(t) + np.cos(2 * t)) / (12 * h * h)
        assert np.allclose(ev, np.sort(closed), rtol=1e-13, atol=1e-13)
        i = np.arange(N)
        for k in range(1, N + 1):
            v = np.sin(math.pi * k * (i + 1) / (N + 1))
            assert np.allclose(A @ v, closed[k - 1] * v, atol=1e-12)
    assert np.allclose(O.line_spectrum(12, 0.5)[0], 0.11679565, atol=1e-8)
    assert np.allclose(O.line_spectrum(24, 0.5)[0], 0.03158265, atol=1e-8)


def test_box_sine_modes_anisotropic():
    """Products of sine modes are eigenvectors of the 3-D box operator with
    the sum of the three line eigenvalues; an anisotropic box catches any
    mix-up of the axes."""
    dims, h = (5, 4, 3), 0.4
    T = O.kinetic_box(dims, (0, 0, 0), dims, h).toarray()
    ex, ey, ez = (O.line_spectrum(d, h) for d in dims)
    for (kx, ky, kz) in [(1, 1, 1), (2, 1, 3), (5, 4, 1), (3, 2, 2)]:
        v = _grid_fn(dims, 1.0, lambda X, Y, Z: np.sin(math.pi * kx * (X + 1) / 6)
                     * np.sin(math.pi * ky * (Y + 1) / 5)
                     * np.sin(math.pi * kz * (Z + 1) / 4)).ravel()
        lam = ex[kx - 1] + ey[ky - 1] + ez[kz - 1]
        assert np.allclose(T @ v, lam * v, atol=1e-11)
    assert np.allclose(np.linalg.eigvalsh(T), O.box_spectrum(dims, h),
                       rtol=1e-13)


def test_continuum_limit_fourth_order():
    """V = 0 ground state of an N^3-point box approaches the continuum
    3 pi^2 / (2 L^2), L = (N+1) h, with an error that falls ~16x when h
    halves at fixed L."""
    L = 6.5
    errs = []
    for N in (12, 25):
        h = L / (N + 1)
        e0 = O.box_spectrum((N, N, N), h, 1)[0]
        exact = 3 * math.pi ** 2 / (2 * L * L)
        errs.append(abs(e0 - exact) / exact)
    assert errs[0] < 1e-4
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_tiny_grid_v0_ground_state():
    """Whole 24x12x12 grid at h = 0.5 with V = 0: E0 = T(pi/25) + 2 T(pi/13)
    = 0.265174 Ha, within 1e-4 of the continuum value 0.265180."""
    V = np.zeros((12, 12, 24))
    e = O.full_grid_eigs(V, 0.5, 1)[0]
    closed = O.line_spectrum(24, 0.5)[0] + 2 * O.line_spectrum(12, 0.5)[0]
    assert e == pytest.approx(closed, abs=1e-12)
    assert e == pytest.approx(0.265174, abs=1e-6)
    cont = math.pi ** 2 / 2 * (1 / 12.5 ** 2 + 2 / 6.5 ** 2)
    assert abs(e - cont) / cont < 1e-4


def test_symmetry_and_global_restriction():
    """H is symmetric; the rows/cols of the whole-grid operator inside a box
    equal the kinetic sub-block taken from the whole-grid matrix."""
    rng = np.random.default_rng(3)
    V = rng.standard_normal((6, 7, 8))
    H = O.hamiltonian_box(V, 0.5, (0, 0, 0), (8, 7, 6), walls="box")
    x, y = rng.standard_normal((2, H.shape[0]))
    assert abs(x @ (H @ y) - (H @ x) @ y) <= 1e-13 * np.abs(H).max() * 50
    full = H.toarray().reshape(6, 7, 8, 6, 7, 8)
    sub = O.hamiltonian_box(V, 0.5, (2, 1, 3), (4, 5, 2), walls="global")
    ref = full[3:5, 1:6, 2:6, 3:5, 1:6, 2:6].reshape(40, 40)
    assert np.array_equal(sub.toarray(), ref)


def test_fragment_wall_correction():
    """A fragment operator differs from the whole-grid rows of the same box
    only on the diagonal, by -1/(24 h^2) per box face that is not a grid
    face."""
    rng = np.random.default_rng(4)
    V = rng.standard_normal((10, 10, 10))
    h, lo, dims = 0.5, (0, 3, 2), (5, 4, 8)
    Hf = O.hamiltonian_box(V, h, lo, dims, walls="box").toarray()
    Hg = O.hamiltonian_box(V, h, lo, dims, walls="global").toarray()
    diff = Hf - Hg
    assert np.array_equal(diff - np.diag(np.diag(diff)), np.zeros_like(diff))
    d = np.diag(diff).reshape(dims[2], dims[1], dims[0])
    cnt = np.zeros_like(d)
    cnt[:, :, -1] += 1   # x: 0..4, only the upper face (x = 5) is interior
    cnt[:, 0, :] += 1    # y: 3..6, both faces interior
    cnt[:, -1, :] += 1
    cnt[0, :, :] += 1    # z: 2..9, the upper face is the grid's own wall
    assert np.allclose(d, -cnt / (24 * h * h), atol=1e-14)
