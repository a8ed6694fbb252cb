"""Seeded input generators: determinism, shapes, and the potential pinned to
the oracle's own point-by-point evaluation."""
import json
import os

import numpy as np
import pytest

import oracle as O
from ofm_inputs import (alkane_chain, amorphous_polymer, box_system,
                        thiophene_polymer, tiny_chain)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inside(s):
    n = np.array([s.grid.nx, s.grid.ny, s.grid.nz])
    assert np.all(s.frag_lo >= 0)
    assert np.all(s.frag_lo + s.frag_dims <= n)
    assert np.all(s.frag_dims >= 1)
    assert np.all(s.frag_states >= 1)


def test_tiny_deterministic_and_shape():
    a, b, c = tiny_chain(0), tiny_chain(0), tiny_chain(1)
    assert np.array_equal(a.atoms, b.atoms)
    assert not np.array_equal(a.atoms, c.atoms)
    assert (a.grid.nx, a.grid.ny, a.grid.nz) == (24, 12, 12)
    assert a.potential().shape == (12, 12, 24)
    assert a.n_frag == 3 and a.n_basis == 18
    assert list(a.frag_lo[:, 0]) == [0, 6, 12]
    # jitter is within +-0.2 bohr of the straight chain
    ideal = 0.5 * 0.5 * np.array([23, 11, 11]) + \
        np.array([[(k - 2.5) * 2.0, 0, 0] for k in range(6)])
    assert np.abs(a.atoms - ideal).max() <= 0.2
    _inside(a)


def test_potential_matches_untruncated_sum(tiny0):
    """The generator truncates each well at 8 bohr; the oracle evaluates the
    full sum point by point.  The tails are below 2e-22 Ha."""
    s = tiny0
    Vo = O.gaussian_potential((s.grid.nx, s.grid.ny, s.grid.nz), s.grid.h,
                              s.grid.origin, s.atoms, s.Z, s.sigma, None)
    assert np.abs(Vo - s.potential()).max() <= 1e-15
    Vt = O.gaussian_potential((s.grid.nx, s.grid.ny, s.grid.nz), s.grid.h,
                              s.grid.origin, s.atoms, s.Z, s.sigma, 8.0)
    assert np.abs(Vt - s.potential()).max() <= 1e-15


def test_potential_single_well_value():
    """One well of depth Z at a grid point: V there is exactly -Z, and at a
    point d away it is -Z exp(-d^2 / (2 sigma^2))."""
    s = box_system((9, 9, 9), 0.5, [[0, 0, 0]], [[9, 9, 9]], [1],
                   atoms=[[2.0, 2.0, 2.0]], Z=[0.7])
    V = s.potential()
    assert V[4, 4, 4] == pytest.approx(-0.7, abs=1e-15)
    assert V[4, 4, 6] == pytest.approx(-0.7 * np.exp(-1.0 / (2 * 0.64)),
                                       rel=1e-14)


def test_alkane_chain_shape():
    s = alkane_chain(0)
    assert s.atoms.shape == (2000, 3)
    nC = int((s.Z == 1.0).sum())
    assert nC == 666 and int((s.Z == 0.5).sum()) == 1334
    assert s.n_frag == 256 and s.n_basis == 4096
    assert np.all(s.frag_dims == 32)
    _inside(s)
    # C-C bonds are 2.9 bohr and C-H bonds 2.1 bohr
    C = s.atoms[:nC]
    assert np.allclose(np.linalg.norm(np.diff(C, axis=0), axis=1), 2.9)
    # consecutive windows overlap by about half their carbons
    w0 = set(s.frag_atom_idx[s.frag_atom_ptr[0]:s.frag_atom_ptr[1]])
    w1 = set(s.frag_atom_idx[s.frag_atom_ptr[1]:s.frag_atom_ptr[2]])
    assert len(w0 & w1) > 0
    # the grid keeps an 8 bohr margin around every atom
    lo = s.grid.origin
    hi = lo + s.grid.h * (np.array([s.grid.nx, s.grid.ny, s.grid.nz]) - 1)
    assert np.all(s.atoms.min(0) - lo >= 8.0 - 1e-9)
    assert np.all(hi - s.atoms.max(0) >= 8.0 - 1e-9)


@pytest.mark.slow
def test_amorphous_polymer_shape():
    s = amorphous_polymer(0)
    assert s.atoms.shape == (10000, 3)
    assert s.n_frag == 1024
    assert (s.grid.nx, s.grid.ny, s.grid.nz) == (240, 240, 240)
    assert s.frag_dims.min() >= 24 and s.frag_dims.max() <= 40
    assert s.frag_states.min() >= 8 and s.frag_states.max() <= 32
    _inside(s)


def test_paper_basis_sizes():
    """Sec. IV / Sec. III counting: overlapping trimers of a chain of M
    monomers number M - 2, so 5 chains x 20 rings with 3 states per trimer
    give the paper's 270 basis functions, and 20 alkane chains x 20 monomers
    with 5 states per trimer give 1800."""
    with open(os.path.join(GOLDEN, "paper_basis_sizes.json")) as fh:
        g = json.load(fh)
    p3ht = g["p3ht"]
    s = thiophene_polymer(0, n_chains=p3ht["chains"], n_rings=p3ht["rings"],
                          n_states=p3ht["states_per_fragment"])
    assert s.n_frag == p3ht["chains"] * (p3ht["rings"] - 2)
    assert s.n_basis == p3ht["basis_size"]
    alk = g["alkane"]
    assert alk["chains"] * (alk["monomers"] - 2) * \
        alk["states_per_fragment"] == alk["basis_size"]
    _inside(s)
