"""MI355X (gfx950) laser-cluster molecular dynamics: the hot path of arXiv:1307.3711's model.

Python face of liblcmd.so.  See include/lcmd.h for the C ABI; this package only marshals
arguments and lends PyTorch device memory and streams to the library.
"""
from ._binding import (  # noqa: F401
    LC_MAX_Z, LC_REC, LC_DET_BINS, LC_DET_SLOTS, LC_FIELD_STATIC_MAX_BYTES, LcError, Simulation, Surrogate, field,
    LC_OK, LC_E_INVALID, LC_E_CAPACITY, LC_E_NONFINITE, LC_E_HIP, LC_E_STATE, LC_E_UNSUPPORTED,
    field_static, lib, make_cluster,
    make_config, make_tuning, pair_blocks_for, units,
    PRECISIONS, ENVELOPES, PHASES, OFI, POLARIZATIONS, BOUNDARIES,
    R_T, R_STEP, R_N, R_NION, R_NEL, R_KE_HALF, R_KE_BAR, R_PE, R_WL, R_WC, R_WSP, R_P, R_F, R_FABS,
    R_MEANZ, R_ABS_EV, R_DROPPED, R_EVENTS, R_ENV, R_KE_START, R_ZHIST,
)
