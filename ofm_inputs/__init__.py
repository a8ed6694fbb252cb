"""Seeded synthetic inputs for the overlapping-fragments method (OFM).

This package only *builds inputs*: atom positions and well depths, the
real-space grid, the potential sampled on that grid, and the cuboid fragment
boxes with their state counts.  It holds none of the method's arithmetic (no
kinetic operator, no eigensolver, no matrix elements), so that the CPU oracle
and the GPU path can both consume it without sharing any computation.

The systems follow the paper's test cases in shape only: disordered alkane-like
chains cut into overlapping windows of consecutive monomers (Sec. III) and
thiophene-like chains cut into overlapping trimers (Sec. IV).  The paper's
charge-patching potential is replaced by a sum of Gaussian wells, one per atom.
"""

from .systems import (  # noqa: F401
    Grid,
    System,
    CONFIGS,
    make_system,
    tiny_chain,
    alkane_chain,
    amorphous_polymer,
    thiophene_polymer,
    box_system,
)
