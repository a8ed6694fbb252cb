"""MI355X-native hot path of the overlapping fragments method (OFM).

The compute path is libofm.so (HIP for gfx950, C ABI in include/ofm.h); this
package holds the hipcc build script and a thin ctypes binding with the same
entry-point names.  Importing the package does not load the library; the
first call does, and raises if it has not been built.
"""
from .ofm import (  # noqa: F401
    EXPORTS, OFM_FP64, OFM_MIXED_BF16X3, OFM_MIXED_FP16X3, OFM_E_NOCONV, OFM_E_SINGULAR,
    OFM_E_INVALID, OFM_E_STATE, Context, Fragments, Mats, OfmError, lib,
    ofm_apply_fragment_h, ofm_build_fragments, ofm_create, ofm_get_hphi,
    ofm_get_states, ofm_matrix_elements, ofm_mats_copy, ofm_set_states, ofm_set_stencil_variant,
    ofm_set_fragment_wells, ofm_select_homo, ofm_solve_global_subset,
    ofm_homo_energies, ofm_homo_lumo_gap, ofm_dense_eigh, ofm_solve_flags,
    OFM_MAX_APPLY_VECTORS, ofm_matrix_elements_noalloc, n_values,
    ofm_set_pair_variant, ofm_select_band, ofm_solve_global_window,
    ofm_solve_fragments, ofm_solve_global, ofm_version, unpack_blocks,
)
