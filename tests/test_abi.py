"""The C ABI library loads and exports every symbol the header declares
(no GPU call), and the host-side planner's checks need no device."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofm.h")
LIB = os.path.join(ROOT, "paper_1011_4764_amd", "libofm.so")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ofm_[a-z_0-9]+)\s*\(", txt)))


def test_header_matches_binding_list():
    from paper_1011_4764_amd.ofm import EXPORTS
    assert sorted(EXPORTS) == _declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofm.so not built")
def test_library_exports_every_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], check=True,
                         capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [s for s in _declared() if s not in syms]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofm.so not built")
def test_library_loads_without_gpu():
    import paper_1011_4764_amd as P
    L = P.lib()
    for name in _declared():
        assert hasattr(L, name)
    assert "gfx950" in P.ofm_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofm.so not built")
def test_homo_lumo_gap_host_matches_oracle():
    """ofm_homo_lumo_gap is host arithmetic in the library: it needs no GPU
    and gives the oracle's gap on seeded random spectra, including the
    no-gap and empty cases."""
    import numpy as np

    import oracle as O
    import paper_1011_4764_amd as P
    rng = np.random.default_rng(5)
    for trial in range(200):
        n = int(rng.integers(0, 40))
        E = np.sort(rng.normal(size=n) * rng.uniform(0.1, 3.0))
        e_ref = float(rng.normal())
        gmin = float(rng.uniform(0, 1.0))
        got = P.ofm_homo_lumo_gap(E, e_ref, gmin)
        ref = O.homo_lumo_gap(E, e_ref, gmin)
        assert got[0] == ref[0]
        if ref[0] >= 0:
            assert got[1:] == ref[1:]
        else:
            assert np.isnan(got[1]) and np.isnan(got[2])
    with pytest.raises(P.OfmError):
        P.ofm_homo_lumo_gap([1.0, 0.0], 0.0, 0.1)   # not ascending
    with pytest.raises(P.OfmError):
        P.ofm_homo_lumo_gap([0.0, 1.0], 0.0, -1.0)  # negative gap


@pytest.mark.skipif(not os.path.exists(LIB), reason="libofm.so not built")
def test_null_handles_rejected_without_a_gpu():
    """Every entry point that takes a context, fragment or matrix handle
    returns OFM_E_INVALID for a NULL handle (all other pointers NULL, sizes
    zero) before touching the device; ofm_homo_lumo_gap rejects NULL outputs
    and ofm_last_error(NULL) still returns text."""
    import ctypes as C

    import paper_1011_4764_amd as P
    L = P.lib()
    skip = {"ofm_create", "ofm_version", "ofm_last_error"}
    checked = 0
    for name in _declared():
        if name in skip:
            continue
        fn = getattr(L, name)
        args = []
        for t in fn.argtypes:
            if t in (C.c_int, C.c_longlong):
                args.append(t(0))
            elif t is C.c_double:
                args.append(t(0.0))
            else:
                args.append(None)
        assert fn(*args) == P.OFM_E_INVALID, name
        checked += 1
    assert checked == len(_declared()) - len(skip)
    assert isinstance(L.ofm_last_error(None), bytes)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it says so and exits with
    status 2 before touching a device."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""
