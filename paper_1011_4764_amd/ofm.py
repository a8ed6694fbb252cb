"""Thin ctypes binding of libofm.so (argument marshalling only).

Every function below has the name of the C entry point it calls and does no
arithmetic of its own: all steps of the path run in the HIP library.  Host
arrays are numpy float64; a device potential may be passed as any object with
``data_ptr()`` (a torch tensor on the GPU), which the library reads in place.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OFM_LIB") or os.path.join(_HERE, "libofm.so")

OFM_OK, OFM_E_INVALID, OFM_E_NOMEM, OFM_E_DEVICE = 0, -1, -2, -3
OFM_E_NOCONV, OFM_E_SINGULAR, OFM_E_STATE = -4, -5, -6
OFM_FP64, OFM_MIXED_BF16X3, OFM_MIXED_FP16X3 = 0, 1, 2
STATUS = {0: "OFM_OK", -1: "OFM_E_INVALID", -2: "OFM_E_NOMEM",
          -3: "OFM_E_DEVICE", -4: "OFM_E_NOCONV", -5: "OFM_E_SINGULAR",
          -6: "OFM_E_STATE"}

#: every symbol declared in include/ofm.h
EXPORTS = [
    "ofm_create", "ofm_destroy", "ofm_last_error", "ofm_version",
    "ofm_build_fragments", "ofm_frags_destroy", "ofm_frags_info",
    "ofm_fragment_geometry", "ofm_pairs", "ofm_solve_fragments",
    "ofm_get_states", "ofm_set_states", "ofm_get_hphi", "ofm_apply_fragment_h",
    "ofm_matrix_elements", "ofm_mats_info", "ofm_mats_copy",
    "ofm_mats_destroy", "ofm_solve_global", "ofm_set_profiling",
    "ofm_kernel_stats", "ofm_reset_stats", "ofm_stage_times",
    "ofm_set_stencil_variant", "ofm_set_fragment_wells", "ofm_select_homo",
    "ofm_solve_global_subset", "ofm_homo_energies", "ofm_homo_lumo_gap",
    "ofm_dense_eigh", "ofm_solve_flags", "ofm_matrix_elements_noalloc",
    "ofm_set_pair_variant", "ofm_select_band", "ofm_solve_global_window",
]
OFM_MAX_APPLY_VECTORS = 32767


class OfmGrid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("h", C.c_double), ("origin", C.c_double * 3)]


class OfmFragmentDesc(C.Structure):
    _fields_ = [("lo", C.c_int * 3), ("dims", C.c_int * 3),
                ("n_states", C.c_int)]


class OfmSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int),
                ("guard", C.c_int), ("degree", C.c_int),
                ("seed", C.c_ulonglong), ("use_graph", C.c_int),
                ("autotune", C.c_int), ("resident", C.c_int),
                ("fused", C.c_int)]


class OfmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_LL = C.POINTER(C.c_longlong)
_UB = C.POINTER(C.c_ubyte)


def lib():
    """Load libofm.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1011_4764_amd.build_lib`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "ofm_create": ([C.POINTER(_P), C.c_int, _P, C.c_int], C.c_int),
            "ofm_destroy": ([_P], C.c_int),
            "ofm_last_error": ([_P], C.c_char_p),
            "ofm_version": ([], C.c_char_p),
            "ofm_build_fragments": ([_P, C.POINTER(OfmGrid), _P, C.c_int,
                                     C.POINTER(OfmFragmentDesc), _D, _LL, _I,
                                     C.c_double, C.POINTER(_P)], C.c_int),
            "ofm_frags_destroy": ([_P], C.c_int),
            "ofm_frags_info": ([_P, _LL, _LL, _LL], C.c_int),
            "ofm_fragment_geometry": ([_P, C.c_int, _I, _I, _I, _I, _I],
                                      C.c_int),
            "ofm_pairs": ([_P, _I, _I, _LL], C.c_int),
            "ofm_solve_fragments": ([_P, _P, C.POINTER(OfmSolveOpts), _D, _I,
                                     C.POINTER(C.c_ubyte)], C.c_int),
            "ofm_solve_flags": ([_P, _I], C.c_int),
            "ofm_get_states": ([_P, C.c_int, _D, _D], C.c_int),
            "ofm_set_states": ([_P, C.c_int, _D, _D], C.c_int),
            "ofm_get_hphi": ([_P, C.c_int, _D], C.c_int),
            "ofm_apply_fragment_h": ([_P, _P, C.c_int, C.c_int, _D, _D],
                                     C.c_int),
            "ofm_matrix_elements": ([_P, _P, C.POINTER(_P)], C.c_int),
            "ofm_mats_info": ([_P, _LL], C.c_int),
            "ofm_matrix_elements_noalloc": ([_P, _P, _P, _P], C.c_int),
            "ofm_mats_copy": ([_P, _D, _D], C.c_int),
            "ofm_mats_destroy": ([_P], C.c_int),
            "ofm_solve_global": ([_P, _P, C.c_double, C.c_double, C.c_double,
                                  _I, _I, _D, _D, _D], C.c_int),
            "ofm_set_profiling": ([_P, C.c_int], C.c_int),
            "ofm_kernel_stats": ([_P, C.c_char_p, _LL, _D, _D, _D], C.c_int),
            "ofm_reset_stats": ([_P], C.c_int),
            "ofm_stage_times": ([_P, _D, _D, _D], C.c_int),
            "ofm_set_stencil_variant": ([_P, C.c_int], C.c_int),
            "ofm_set_pair_variant": ([_P, C.c_int], C.c_int),
            "ofm_set_fragment_wells": ([_P, C.c_int, _D, _D, C.c_double,
                                        C.c_double, _LL, _I], C.c_int),
            "ofm_select_homo": ([_P, C.c_int, C.c_double, _UB], C.c_int),
            "ofm_solve_global_subset": ([_P, _P, _UB, C.c_double, C.c_double,
                                         C.c_double, _I, _I, _D, _D, _D],
                                        C.c_int),
            "ofm_homo_energies": ([_P, _D], C.c_int),
            "ofm_select_band": ([_P, C.c_double, C.c_double, _UB], C.c_int),
            "ofm_solve_global_window": ([_P, _P, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double,
                                         C.c_int, C.c_double, _I, _D, _D,
                                         _LL, _I], C.c_int),
            "ofm_dense_eigh": ([_P, C.c_int, _D, _D, _D], C.c_int),
            "ofm_homo_lumo_gap": ([_D, C.c_int, C.c_double, C.c_double, _I,
                                   _D, _D], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _check(st, ctx_handle):
    if st not in (OFM_OK,):
        msg = lib().ofm_last_error(ctx_handle)
        raise OfmError(st, msg.decode() if msg else "")


def ofm_version() -> str:
    return lib().ofm_version().decode()


class Context:
    """ofm_create / ofm_destroy."""

    def __init__(self, device=0, stream=None, precision=OFM_FP64):
        if isinstance(precision, str):
            precision = {"fp64": OFM_FP64, "mixed": OFM_MIXED_BF16X3,
                         "bf16x3": OFM_MIXED_BF16X3,
                         "fp16x3": OFM_MIXED_FP16X3}[precision]
        self.precision = precision
        h = _P()
        st = lib().ofm_create(C.byref(h), int(device),
                              _P(stream) if stream else None, int(precision))
        _check(st, None)
        self.handle = h
        self._children = weakref.WeakSet()

    def close(self):
        """Destroy matrix and fragment handles made with this context, then
        the context itself."""
        if getattr(self, "handle", None):
            kids = list(self._children)
            for k in kids:
                if isinstance(k, Mats):
                    k.close()
            for k in kids:
                k.close()
            lib().ofm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib().ofm_last_error(self.handle).decode()

    # measurement
    def set_profiling(self, on=True):
        _check(lib().ofm_set_profiling(self.handle, int(bool(on))), self.handle)

    def kernel_stats(self, family):
        n = C.c_longlong()
        ms, by, fl = C.c_double(), C.c_double(), C.c_double()
        _check(lib().ofm_kernel_stats(self.handle, family.encode(), C.byref(n),
                                      C.byref(ms), C.byref(by), C.byref(fl)),
               self.handle)
        return {"launches": n.value, "ms": ms.value, "bytes": by.value,
                "flops": fl.value}

    def reset_stats(self):
        _check(lib().ofm_reset_stats(self.handle), self.handle)

    def stage_times(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().ofm_stage_times(self.handle, C.byref(a), C.byref(b),
                                     C.byref(c)), self.handle)
        return {"solve_ms": a.value, "elements_ms": b.value,
                "global_ms": c.value}


def ofm_create(device=0, stream=None, precision=OFM_FP64) -> Context:
    return Context(device, stream, precision)


class Fragments:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle
        nb, npair, npts = C.c_longlong(), C.c_longlong(), C.c_longlong()
        _check(lib().ofm_frags_info(handle, C.byref(nb), C.byref(npair),
                                    C.byref(npts)), ctx.handle)
        self.n_basis, self.n_pairs, self.total_points = \
            nb.value, npair.value, npts.value
        self.n_frag = None
        ctx._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib().ofm_frags_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def geometry(self, j):
        lo, dims = (C.c_int * 3)(), (C.c_int * 3)()
        dlo, dd = (C.c_int * 3)(), (C.c_int * 3)()
        s = C.c_int()
        _check(lib().ofm_fragment_geometry(self.handle, j, lo, dims, dlo, dd,
                                           C.byref(s)), self.ctx.handle)
        return tuple(lo), tuple(dims), tuple(dlo), tuple(dd), s.value

    def pairs(self):
        n = self.n_pairs
        pj = np.zeros(n, np.int32)
        pn = np.zeros(n, np.int32)
        off = np.zeros(n, np.int64)
        _check(lib().ofm_pairs(self.handle, pj.ctypes.data_as(_I),
                               pn.ctypes.data_as(_I),
                               off.ctypes.data_as(_LL)), self.ctx.handle)
        return pj, pn, off


def ofm_build_fragments(ctx: Context, shape_xyz, h, V, frag_lo, frag_dims,
                        frag_states, origin=(0.0, 0.0, 0.0), atom_xyz=None,
                        frag_atom_ptr=None, frag_atom_idx=None,
                        d_cut=0.0) -> Fragments:
    g = OfmGrid(int(shape_xyz[0]), int(shape_xyz[1]), int(shape_xyz[2]),
                float(h), (C.c_double * 3)(*[float(o) for o in origin]))
    lo = np.asarray(frag_lo, np.int32).reshape(-1, 3)
    dims = np.asarray(frag_dims, np.int32).reshape(-1, 3)
    st = np.asarray(frag_states, np.int32).reshape(-1)
    nf = lo.shape[0]
    descs = (OfmFragmentDesc * nf)()
    for j in range(nf):
        descs[j].lo[:] = [int(v) for v in lo[j]]
        descs[j].dims[:] = [int(v) for v in dims[j]]
        descs[j].n_states = int(st[j])
    keep = []
    if hasattr(V, "data_ptr"):
        vp = _P(V.data_ptr())
        keep.append(V)
    else:
        Vh = np.ascontiguousarray(V, dtype=np.float64)
        assert Vh.size == g.nx * g.ny * g.nz
        vp = Vh.ctypes.data_as(_P)
        keep.append(Vh)
    ax = ap = ai = None
    if atom_xyz is not None:
        ax = np.ascontiguousarray(atom_xyz, np.float64)
        ap = np.ascontiguousarray(frag_atom_ptr, np.int64)
        ai = np.ascontiguousarray(frag_atom_idx, np.int32)
    out = _P()
    stt = lib().ofm_build_fragments(
        ctx.handle, C.byref(g), vp, nf, descs,
        _dp(ax), ap.ctypes.data_as(_LL) if ap is not None else None,
        ai.ctypes.data_as(_I) if ai is not None else None, float(d_cut),
        C.byref(out))
    _check(stt, ctx.handle)
    f = Fragments(ctx, out)
    f.n_frag = nf
    f.states = st.copy()
    return f


def ofm_solve_fragments(ctx: Context, frags: Fragments, tol=0.0, max_iter=0,
                        degree=0, seed=0, use_graph=0, autotune=0,
                        resident=0, fused=0, raise_on_noconv=False):
    """Returns (status, eps (sum s_j,), iters (n_frag,), converged (n_frag,)).
    use_graph / autotune / resident / fused: 0 = library default (on),
    -1 = off."""
    o = OfmSolveOpts(float(tol), int(max_iter), 0, int(degree), int(seed),
                     int(use_graph), int(autotune), int(resident), int(fused))
    eps = np.zeros(frags.n_basis)
    it = np.zeros(frags.n_frag, np.int32)
    cv = np.zeros(frags.n_frag, np.uint8)
    st = lib().ofm_solve_fragments(ctx.handle, frags.handle, C.byref(o),
                                   _dp(eps), it.ctypes.data_as(_I),
                                   cv.ctypes.data_as(C.POINTER(C.c_ubyte)))
    if st != OFM_E_NOCONV or raise_on_noconv:
        _check(st, ctx.handle)
    return st, eps, it, cv.astype(bool)


def ofm_solve_flags(frags: Fragments):
    """Per-fragment flags of the last solve (bit 0: shifted Cholesky used,
    bit 1: shifted Cholesky lost a pivot too)."""
    fl = np.zeros(frags.n_frag, np.int32)
    _check(lib().ofm_solve_flags(frags.handle, fl.ctypes.data_as(_I)),
           frags.ctx.handle)
    return fl


def ofm_get_states(frags: Fragments, j):
    lo, dims, dlo, dd, s = frags.geometry(j)
    n = dims[0] * dims[1] * dims[2]
    phi = np.zeros((s, n))
    eps = np.zeros(s)
    _check(lib().ofm_get_states(frags.handle, j, _dp(phi), _dp(eps)),
           frags.ctx.handle)
    return eps, phi


def ofm_set_states(frags: Fragments, j, phi, eps=None):
    phi = np.ascontiguousarray(phi, np.float64)
    e = None if eps is None else np.ascontiguousarray(eps, np.float64)
    _check(lib().ofm_set_states(frags.handle, j, _dp(phi), _dp(e)),
           frags.ctx.handle)


def ofm_get_hphi(frags: Fragments, j):
    lo, dims, dlo, dd, s = frags.geometry(j)
    out = np.zeros((s, dd[0] * dd[1] * dd[2]))
    _check(lib().ofm_get_hphi(frags.handle, j, _dp(out)), frags.ctx.handle)
    return out


def ofm_set_fragment_wells(frags: Fragments, atom_xyz, Z, frag_atom_ptr,
                           frag_atom_idx, sigma=0.8, r_cut=8.0):
    ax = np.ascontiguousarray(atom_xyz, np.float64).reshape(-1, 3)
    z = np.ascontiguousarray(Z, np.float64)
    ap = np.ascontiguousarray(frag_atom_ptr, np.int64)
    ai = np.ascontiguousarray(frag_atom_idx, np.int32)
    _check(lib().ofm_set_fragment_wells(
        frags.handle, ax.shape[0], _dp(ax), _dp(z), float(sigma), float(r_cut),
        ap.ctypes.data_as(_LL), ai.ctypes.data_as(_I)), frags.ctx.handle)


def ofm_set_stencil_variant(frags: Fragments, variant: int):
    _check(lib().ofm_set_stencil_variant(frags.handle, int(variant)),
           frags.ctx.handle)


def ofm_set_pair_variant(ctx: Context, variant: int):
    _check(lib().ofm_set_pair_variant(ctx.handle, int(variant)), ctx.handle)


def ofm_apply_fragment_h(ctx: Context, frags: Fragments, j, x):
    x = np.ascontiguousarray(x, np.float64)
    x2 = x.reshape(-1, x.shape[-1]) if x.ndim > 1 else x.reshape(1, -1)
    y = np.zeros_like(x2)
    _check(lib().ofm_apply_fragment_h(ctx.handle, frags.handle, j,
                                      x2.shape[0], _dp(x2), _dp(y)),
           ctx.handle)
    return y.reshape(x.shape)


class Mats:
    def __init__(self, ctx, frags, handle):
        self.ctx, self.frags, self.handle = ctx, frags, handle
        n = C.c_longlong()
        _check(lib().ofm_mats_info(handle, C.byref(n)), ctx.handle)
        self.n_values = n.value
        ctx._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib().ofm_mats_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ofm_matrix_elements(ctx: Context, frags: Fragments) -> Mats:
    out = _P()
    _check(lib().ofm_matrix_elements(ctx.handle, frags.handle, C.byref(out)),
           ctx.handle)
    return Mats(ctx, frags, out)


def n_values(frags: Fragments) -> int:
    """Doubles per matrix of the packed blocks (sum over pairs of s_j s_n)."""
    pj, pn, off = frags.pairs()
    st = frags.states
    return int(off[-1] + st[pj[-1]] * st[pn[-1]]) if len(pj) else 0


def ofm_matrix_elements_noalloc(ctx: Context, frags: Fragments, H_dev, S_dev):
    """Blocks into caller-owned device buffers (objects with data_ptr(), e.g.
    torch tensors of n_values(frags) float64 on the GPU); enqueued on the
    context stream, which the caller synchronises before reading them."""
    st = lib().ofm_matrix_elements_noalloc(
        ctx.handle, frags.handle,
        _P(H_dev.data_ptr()) if H_dev is not None else None,
        _P(S_dev.data_ptr()) if S_dev is not None else None)
    _check(st, ctx.handle)


def ofm_mats_copy(m: Mats):
    H = np.zeros(m.n_values)
    S = np.zeros(m.n_values)
    _check(lib().ofm_mats_copy(m.handle, _dp(H), _dp(S)), m.ctx.handle)
    return H, S


def ofm_solve_global(ctx: Context, m: Mats, s_thresh=1e-6, e_lo=-np.inf,
                     e_hi=np.inf, want_vectors=False):
    """Returns dict(E, n_kept, s_min[, C])."""
    nb = m.frags.n_basis
    E = np.zeros(nb)
    Cm = np.zeros(nb * nb) if want_vectors else None
    nk, ne = C.c_int(), C.c_int()
    smin = C.c_double()
    st = lib().ofm_solve_global(ctx.handle, m.handle, float(s_thresh),
                                float(e_lo), float(e_hi), C.byref(nk),
                                C.byref(ne), _dp(E), _dp(Cm), C.byref(smin))
    _check(st, ctx.handle)
    out = {"E": E[:ne.value].copy(), "n_kept": nk.value, "s_min": smin.value}
    if want_vectors:
        out["C"] = Cm[:nb * ne.value].reshape(ne.value, nb).T.copy()
    return out


def ofm_select_homo(frags: Fragments, n_max, gap_min=0.0):
    """Keep mask (n_basis bools) near every fragment's HOMO."""
    keep = np.zeros(frags.n_basis, np.uint8)
    _check(lib().ofm_select_homo(frags.handle, int(n_max), float(gap_min),
                                 keep.ctypes.data_as(_UB)), frags.ctx.handle)
    return keep.astype(bool)


def ofm_solve_global_subset(ctx: Context, m: Mats, keep, s_thresh=1e-6,
                            e_lo=-np.inf, e_hi=np.inf, want_vectors=False):
    """ofm_solve_global on the pencil restricted to keep (None: all).
    Returns dict(E, n_kept, s_min[, C with n_sel rows])."""
    nb = m.frags.n_basis
    kp = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    if kp is not None and kp.size != nb:
        raise ValueError("keep needs one entry per basis function")
    nsel = nb if kp is None else int(np.count_nonzero(kp))
    E = np.zeros(nb)
    Cm = np.zeros(max(nsel, 1) * nb) if want_vectors else None
    nk, ne = C.c_int(), C.c_int()
    smin = C.c_double()
    st = lib().ofm_solve_global_subset(
        ctx.handle, m.handle, None if kp is None else kp.ctypes.data_as(_UB),
        float(s_thresh), float(e_lo), float(e_hi), C.byref(nk), C.byref(ne),
        _dp(E), _dp(Cm), C.byref(smin))
    _check(st, ctx.handle)
    out = {"E": E[:ne.value].copy(), "n_kept": nk.value, "s_min": smin.value}
    if want_vectors:
        out["C"] = Cm[:nsel * ne.value].reshape(ne.value, nsel).T.copy()
    return out


def ofm_select_band(frags: Fragments, e_lo, e_hi):
    """Keep mask of the basis functions with fragment eigenvalue in
    [e_lo, e_hi]."""
    keep = np.zeros(frags.n_basis, np.uint8)
    _check(lib().ofm_select_band(frags.handle, float(e_lo), float(e_hi),
                                 keep.ctypes.data_as(_UB)), frags.ctx.handle)
    return keep.astype(bool)


def ofm_solve_global_window(ctx: Context, m: Mats, e_lo, e_hi, s_thresh=1e-6,
                            margin0=0.1, margin_step=0.1, max_rounds=6,
                            tol=1e-8, raise_on_noconv=False):
    """Window eigenvalues on energy-band subsets of the basis with a growing
    margin.  Returns dict(E, status, margin, n_sel, n_kept)."""
    nb = m.frags.n_basis
    E = np.zeros(nb)
    ne, nk = C.c_int(), C.c_int()
    mg = C.c_double()
    ns = C.c_longlong()
    st = lib().ofm_solve_global_window(
        ctx.handle, m.handle, float(s_thresh), float(e_lo), float(e_hi),
        float(margin0), float(margin_step), int(max_rounds), float(tol),
        C.byref(ne), _dp(E), C.byref(mg), C.byref(ns), C.byref(nk))
    if st != OFM_E_NOCONV or raise_on_noconv:
        _check(st, ctx.handle)
    return {"E": E[:ne.value].copy(), "status": st, "margin": mg.value,
            "n_sel": ns.value, "n_kept": nk.value}


def ofm_homo_energies(m: Mats):
    """e_j = <HOMO_j|H|HOMO_j> per fragment (whole-system H)."""
    e = np.zeros(m.frags.n_frag)
    _check(lib().ofm_homo_energies(m.handle, _dp(e)), m.ctx.handle)
    return e


def ofm_dense_eigh(ctx: Context, A, want_vectors=False):
    """Eigenvalues (ascending) of the symmetric A, and with want_vectors the
    unit eigenvectors as the columns of Z: (w, Z or None)."""
    Af = np.asfortranarray(A, dtype=np.float64)
    if Af.ndim != 2 or Af.shape[0] != Af.shape[1]:
        raise ValueError("A must be square")
    n = Af.shape[0]
    w = np.zeros(n)
    Z = np.zeros((n, n), order="F") if want_vectors else None
    _check(lib().ofm_dense_eigh(ctx.handle, n, _dp(Af), _dp(w),
                                None if Z is None else _dp(Z)), ctx.handle)
    return w, Z


def ofm_homo_lumo_gap(E, e_ref, gap_min):
    """(n_occ, e_homo, e_lumo) of the first gap above e_ref; n_occ = -1
    when there is none."""
    Ea = np.ascontiguousarray(E, np.float64)
    n = C.c_int()
    lo, hi = C.c_double(), C.c_double()
    st = lib().ofm_homo_lumo_gap(_dp(Ea), int(Ea.size), float(e_ref),
                                 float(gap_min), C.byref(n), C.byref(lo),
                                 C.byref(hi))
    if st != OFM_OK:
        raise OfmError(st, "invalid arguments to ofm_homo_lumo_gap")
    return n.value, lo.value, hi.value


def unpack_blocks(frags: Fragments, H_blocks, S_blocks):
    """Dense symmetric H and S (basis fragment by fragment) from the packed
    upper blocks -- a host-side copy helper for checking, no arithmetic."""
    pj, pn, off = frags.pairs()
    st = frags.states
    bo = np.concatenate([[0], np.cumsum(st)])
    N = int(bo[-1])
    H = np.zeros((N, N))
    S = np.zeros((N, N))
    for p in range(len(pj)):
        j, n = int(pj[p]), int(pn[p])
        sj, sn = int(st[j]), int(st[n])
        hb = H_blocks[off[p]:off[p] + sj * sn].reshape(sj, sn)
        sb = S_blocks[off[p]:off[p] + sj * sn].reshape(sj, sn)
        H[bo[j]:bo[j + 1], bo[n]:bo[n + 1]] = hb
        S[bo[j]:bo[j + 1], bo[n]:bo[n + 1]] = sb
        H[bo[n]:bo[n + 1], bo[j]:bo[j + 1]] = hb.T
        S[bo[n]:bo[n + 1], bo[j]:bo[j + 1]] = sb.T
    return H, S
