"""Host-side checks of the C ABI (no GPU call): the library loads and exports every entry
point include/lcmd.h declares, configurations are validated, the state size is consistent,
and the library's unit constants equal the oracle's independently written ones."""
import ctypes
import os
import re

import pytest

import paper_1307_3711_amd as lc
from paper_1307_3711_amd import _binding
from oracle import units
from workloads import small_ar, ar_20k, xe_200k
from workloads.species import SPECIES

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lcmd.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lc.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), f"liblcmd.so does not export {n}"


def test_version_and_error_strings():
    L = lc.lib()
    assert L.lc_version() == 6
    for code in [0, -1, -2, -3, -4, -5, -6]:
        assert L.lc_error_string(code)
    assert L.lc_error_string(0).decode() == "ok"


def test_units_match_oracle():
    """Constants of the two independent implementations (C++ host runtime vs oracle/units.py)."""
    for lam, inten in [(0.8, 1e16), (0.806, 8e15), (0.857, 5e16), (0.79, 4e15)]:
        u = lc.units(lam, inten)
        assert u["kappa"] == pytest.approx(units.kappa(lam), rel=1e-15)
        assert u["field_au"] == pytest.approx(units.field_au_per_a0(lam), rel=1e-14)
        assert u["rate_scale"] == pytest.approx(units.rate_scale(lam), rel=1e-14)
        assert u["a0"] == pytest.approx(units.a0_from_intensity(inten, lam), rel=1e-15)
        assert u["k_per_nm"] == pytest.approx(units.nm_to_norm(1.0, lam), rel=1e-15)
        assert u["mec2_ev"] == units.MEC2_EV


def _desc(c):
    return lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                           envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, n_cycles=c.laser.n_cycles)


def _bytes(cfg, cls):
    arr = (_binding.ClusterDesc * len(cls))(*cls)
    return lc.lib().lc_state_bytes(ctypes.byref(cfg), arr, len(cls))


def test_state_bytes_scales_with_capacity():
    c, run = small_ar()
    cfg = lc.make_config("fp64", max_splits=8)
    b1 = _bytes(cfg, [_desc(c)])
    assert b1 > 0
    c2 = _binding.ClusterDesc.from_buffer_copy(_desc(c))
    c2.capacity = 2 * c.capacity
    b2 = _bytes(cfg, [c2])
    # per-slot bytes: 10 FP64 arrays + double4 source + Z + detector flag + 8 splits x 4 FP64
    # partials + ionization flag, over a share of the capacity rounded up to 64 slots (plus a
    # 4-byte cluster index per 64 slots)
    per_slot = 10 * 8 + 32 + 1 + 1 + 8 * 4 * 8 + 4
    share = lambda cap: -(-cap // 64) * 64
    assert abs((b2 - b1) - per_slot * (share(2 * c.capacity) - share(c.capacity))) <= 64 * 256
    cfg32 = lc.make_config("fp32_acc64", max_splits=8)
    assert _bytes(cfg32, [_desc(c)]) < b1  # float4 sources instead of double4
    for mk in (ar_20k, xe_200k):
        cc, _ = mk()
        assert _bytes(cfg, [_desc(cc)]) > 0


@pytest.mark.parametrize("field,value", [("dt", 0.0), ("dt", -1.0), ("softening_nm", 0.0), ("lambda_um", 0.0),
                                         ("max_splits", 0), ("max_splits", 65), ("precision", 7),
                                         ("diag_every", -1), ("struct_size", 8), ("detector_r0", -1.0),
                                         ("detector_half_angle_deg", 90.0), ("detector_half_angle_deg", 0.0),
                                         ("boundary", 3), ("box_r0", 0.0), ("box_r0", -2.0), ("precision", 2),
                                         ("collisional", 2), ("ionize", 0)])
def test_invalid_config_rejected(field, value):
    c, run = small_ar()
    cfg = lc.make_config("fp64", detector_r0=9.0 if field.startswith("detector_half") else 0.0,
                         boundary="periodic" if field in ("box_r0", "precision") else "open",
                         collisional=field == "ionize")
    assert _bytes(cfg, [_desc(c)]) > 0
    setattr(cfg, field, value)
    assert _bytes(cfg, [_desc(c)]) == 0


@pytest.mark.parametrize("field,value", [("capacity", 100), ("z_max", 16), ("z_max", -1), ("r0_nm", 0.0),
                                         ("envelope", 9), ("n_ion", -1), ("fwhm_fs", 0.0), ("polarization", 2),
                                         ("polarization", -1), ("lotz_a", -1.0)])
def test_invalid_cluster_rejected(field, value):
    c, run = small_ar()
    d = _desc(c)
    if field == "fwhm_fs":
        d.envelope = 0
    setattr(d, field, value)
    assert _bytes(lc.make_config("fp64"), [d]) == 0


def test_plane_wave_needs_ionization_off():
    c, run = small_ar()
    d = _desc(c)
    d.phase = 1
    assert _bytes(lc.make_config("fp64", ionize=True), [d]) == 0
    assert _bytes(lc.make_config("fp64", ionize=False), [d]) > 0


def test_field_workspace_size():
    L = lc.lib()
    assert L.lc_field_workspace_bytes(0, 1000, None) > 1000 * 32
    bad = lc.make_tuning(R=3)
    assert L.lc_field_workspace_bytes(0, 1000, ctypes.byref(bad)) == 0
    assert L.lc_field_workspace_bytes(9, 1000, None) == 0


def test_pair_once_rows_in_state_bytes():
    """max_pair_blocks M adds 3 M FP32 rows per slot, slots rounded up to 512 per cluster plus
    one more 512-slot block (blocks of 192, 320 or 384 slots round a capacity past the next
    multiple of 512: capacity 1000 in blocks of 192 spans 1152 slots)."""
    c, run = small_ar()
    d = _desc(c)
    base = _bytes(lc.make_config("fp32_acc64", max_splits=8), [d])
    with_rows = _bytes(lc.make_config("fp32_acc64", max_splits=8, max_pair_blocks=10), [d])
    slots = -(-c.capacity // 512) * 512 + 512
    assert abs((with_rows - base) - 12 * 10 * slots) <= 256
    base64 = _bytes(lc.make_config("fp64", max_splits=8), [d])
    rows64 = _bytes(lc.make_config("fp64", max_splits=8, max_pair_blocks=10), [d])
    assert abs((rows64 - base64) - 24 * 10 * slots) <= 256                     # FP64 rows
    assert _bytes(lc.make_config("fp32_kahan", max_pair_blocks=10), [d]) == 0   # no Kahan variant
    assert _bytes(lc.make_config("fp32_acc64", max_pair_blocks=-1), [d]) == 0
    assert _bytes(lc.make_config("fp32_acc64", max_pair_blocks=40000), [d]) == 0


@pytest.mark.parametrize("R,WJ,ok", [(1, 1, True), (2, 1, True), (1, 2, True), (2, 2, True), (4, 2, True),
                                     (3, 3, True), (4, 4, True), (5, 5, True), (6, 6, True), (4, 1, False),
                                     (1, 4, False), (2, 4, False), (8, 1, False), (3, 1, False), (7, 7, False),
                                     (8, 8, False)])
def test_pair_once_field_workspace(R, WJ, ok):
    L = lc.lib()
    n = 1000
    t = lc.make_tuning(R=R, WJ=WJ, newton3=1)
    wb = L.lc_field_workspace_bytes(1, n, ctypes.byref(t))
    if not ok:
        assert wb == 0
        return
    B = 64 * R if (R == WJ and R >= 3) else (4 // WJ) * 64 * R   # square shapes: one target group
    nb = -(-n // B)
    assert wb >= nb * nb * 3 * B * 4 + n * 16
    square = R == WJ and R >= 3
    tg, waves = (1, WJ) if square else (4 // WJ, 4)
    lds64 = 8 * (waves * 4 * 136 + tg * 3 * B + (WJ - 1) * 3 * B)   # FP64 chunk copies + reductions
    wb64 = L.lc_field_workspace_bytes(0, n, ctypes.byref(t))
    if lds64 <= 65536:
        assert wb64 >= nb * nb * 3 * B * 8 + n * 32   # FP64 rows
    else:
        assert wb64 == 0                              # shape needs more LDS than a block may take
    assert L.lc_field_workspace_bytes(2, n, ctypes.byref(t)) == 0   # not for Kahan


# Pair-once shapes lc_set_tuning accepts: (R, WJ) with 4/WJ target groups of 64 R slots, and the
# square shapes R = WJ = 3..6 with one group of 64 R slots.
PAIR_SHAPES = [(1, 1), (2, 1), (1, 2), (2, 2), (4, 2), (3, 3), (4, 4), (5, 5), (6, 6)]


def _block_of(R, WJ):
    return 64 * R if (R == WJ and R >= 3) else (4 // WJ) * 64 * R


def test_pair_once_rows_stay_inside_each_share():
    """Host-only bound check of the pair-once partial rows (no GPU).  For every pair-once shape
    and every capacity 1..20000 (a cluster of an ensemble has its own share, so mixes reduce to
    single capacities), and rows per block M from just enough (ceil(capacity / 128), the
    binding's choice) to a few more: whenever the library accepts the shape for the capacity,
    the largest row element the kernel writes and the fold reads, from the documented indexing
    ((K M + m) 3 + d) B + l with K, m < nb, d < 3, l < B, lies inside the share of 3 M
    (capacity rounded up to 512, plus 512); and the library rejects the shape when nb exceeds M.
    Checked against the indexing written out here, not the library's own predicate."""
    import numpy as np
    L = lc.lib()
    out = (ctypes.c_int64 * 3)()
    caps = np.arange(1, 20001)
    shapes = 0
    for prec in (0, 1):
        for R, WJ in PAIR_SHAPES:
            B = _block_of(R, WJ)
            if L.lc_pair_rows_fit(prec, R, WJ, 1, 1, out) != 0:
                # shapes whose LDS does not fit in FP64 (R, WJ = 2, 1 and 6, 6) are not accepted at all
                assert prec == 0 and (R, WJ) in ((2, 1), (6, 6))
                continue
            shapes += 1
            for cap in caps:
                cap = int(cap)
                m_min = -(-cap // 128)
                for M in (m_min, m_min + 1, m_min + 7):
                    rc = L.lc_pair_rows_fit(prec, R, WJ, cap, M, out)
                    nb = -(-cap // B)
                    assert out[0] == B and out[1] == nb
                    if rc == 0:
                        last = (((nb - 1) * M + (nb - 1)) * 3 + 2) * B + (B - 1)
                        assert last < out[2], (prec, R, WJ, cap, M)
                        assert out[2] == 3 * M * ((cap + 511) // 512 * 512 + 512)
                    else:
                        assert rc == -1
                    if nb > M:
                        assert rc == -1
                    if nb <= M and nb * B <= (cap + 511) // 512 * 512:
                        assert rc == 0, (R, WJ, cap, M)  # the share always has room for these
    assert shapes == 2 * len(PAIR_SHAPES) - 2
    # invalid shapes and arguments
    for args in ((1, 3, 1, 100, 4), (1, 7, 7, 100, 4), (2, 4, 4, 100, 4), (1, 4, 4, 0, 4), (1, 4, 4, 100, 0)):
        assert L.lc_pair_rows_fit(*args, out) == -1
