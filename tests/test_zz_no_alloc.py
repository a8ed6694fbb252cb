"""The allocation-free matrix-element entry point against ofm_matrix_elements
through the C ABI: the same blocks bit for bit (same kernels, same task
list), on two calls in a row with the second on a smaller system (fewer
tasks than the list the scratch array still holds from the first call), into
buffers pre-filled with NaN (every element must be written); FP64 and both
mixed forms, imported states included; rejected arguments leave the context
usable."""
import ctypes as C

import numpy as np
import pytest

from ofm_inputs import box_system, tiny_chain

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1011_4764_amd")
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, flush=True)


def _build(ctx, s):
    return P.ofm_build_fragments(
        ctx, (s.grid.nx, s.grid.ny, s.grid.nz), s.grid.h, s.potential(),
        s.frag_lo, s.frag_dims, s.frag_states, origin=s.grid.origin)


def _systems():
    big = tiny_chain(1)                       # 3 fragments of 12^3
    V = big.potential()
    # smaller: two fragments on the same grid, fewer pairs and tasks
    small = box_system((24, 12, 12), 0.5, [(0, 0, 0), (10, 0, 0)],
                       [(12, 12, 12), (12, 12, 12)], [4, 5], V=V)
    return big, small


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp16x3"])
def test_noalloc_matches_allocating_entry_point(prec):
    _say("no-alloc elements", prec)
    ctx = P.ofm_create(0, None, prec)
    big, small = _systems()
    ntasks = []
    for k, s in enumerate((big, small)):
        f = _build(ctx, s)
        st, eps, it, cv = P.ofm_solve_fragments(ctx, f)
        assert st == 0
        if k == 1:   # imported states for one fragment (computed S_jj)
            e0, phi0 = P.ofm_get_states(f, 0)
            P.ofm_set_states(f, 0, phi0, e0)
        m = P.ofm_matrix_elements(ctx, f)
        H_ref, S_ref = P.ofm_mats_copy(m)
        m.close()
        nv = P.n_values(f)
        assert nv == H_ref.size
        Hd = torch.full((nv,), float("nan"), dtype=torch.float64,
                        device="cuda:0")
        Sd = torch.full((nv,), float("nan"), dtype=torch.float64,
                        device="cuda:0")
        torch.cuda.synchronize()
        P.ofm_matrix_elements_noalloc(ctx, f, Hd, Sd)
        # the call only enqueues on the context's stream: wait for the device
        torch.cuda.synchronize()
        H = Hd.cpu().numpy()
        S = Sd.cpu().numpy()
        ntasks.append(f.n_pairs)
        _say(f"  call {k}: {f.n_pairs} pairs, {nv} values, max|H| "
             f"{np.abs(H).max():.3f}")
        assert np.isfinite(H).all() and np.isfinite(S).all()
        assert np.array_equal(H, H_ref)
        assert np.array_equal(S, S_ref)
        f.close()
    assert ntasks[1] < ntasks[0]
    ctx.close()


def test_noalloc_rejects_bad_buffers():
    _say("no-alloc elements: rejected arguments")
    ctx = P.ofm_create(0, None, P.OFM_FP64)
    s = tiny_chain(0)
    f = _build(ctx, s)
    nv = 1
    Hd = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    L = P.lib()
    # no states yet
    st = L.ofm_matrix_elements_noalloc(ctx.handle, f.handle,
                                       C.c_void_p(Hd.data_ptr()),
                                       C.c_void_p(Hd.data_ptr()))
    assert st == P.OFM_E_STATE
    P.ofm_solve_fragments(ctx, f)
    nv = P.n_values(f)
    Hd = torch.zeros(nv, dtype=torch.float64, device="cuda:0")
    Sd = torch.zeros(nv, dtype=torch.float64, device="cuda:0")
    host = np.zeros(nv)
    for a, b in ((None, Sd.data_ptr()), (Hd.data_ptr(), None),
                 (host.ctypes.data, Sd.data_ptr()),
                 (Hd.data_ptr(), host.ctypes.data)):
        st = L.ofm_matrix_elements_noalloc(ctx.handle, f.handle,
                                           C.c_void_p(a) if a else None,
                                           C.c_void_p(b) if b else None)
        assert st == P.OFM_E_INVALID
    assert L.ofm_matrix_elements_noalloc(None, f.handle, None, None) == \
        P.OFM_E_INVALID
    # still usable, and equal to the allocating path
    P.ofm_matrix_elements_noalloc(ctx, f, Hd, Sd)
    torch.cuda.synchronize()
    m = P.ofm_matrix_elements(ctx, f)
    H_ref, S_ref = P.ofm_mats_copy(m)
    m.close()
    assert np.array_equal(Hd.cpu().numpy(), H_ref)
    assert np.array_equal(Sd.cpu().numpy(), S_ref)
    f.close()
    ctx.close()
