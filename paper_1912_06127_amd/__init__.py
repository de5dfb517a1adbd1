"""MI355X (gfx950) TDVP time evolution of matrix product states.

The compute path lives in the HIP library ``libtdvp.so`` (C ABI in
``include/tdvp.h``); this package only marshals arguments to it.
"""
from .api import (  # noqa: F401
    MPO, MPS, Context, SegmentOptions, Segments, TDVPError, TDVPOptions, apply_heff, apply_heff_adjoint, apply_heff_batched, apply_heff_u1, energy, env_update, env_update_adjoint, env_update_u1, expect, expect2,
    infidelity, norm2, overlap, segment_schedule, transition_expect, tdvp1_step, tdvp2_step, tdvp_hybrid_step, dmrg2_sweep,
)
from ._lib import lib_path, load  # noqa: F401
from . import fit  # noqa: F401

PAULI_X = [[0, 1], [1, 0]]
PAULI_Y = [[0, -1j], [1j, 0]]
PAULI_Z = [[1, 0], [0, -1]]
