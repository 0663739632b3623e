"""The allocation-free field entry point (lc_field_static: the workspace is the library's device
array, not a caller buffer) against lc_field with a caller-owned workspace, through the C ABI.

Both run the same kernels on the same inputs, so the results must be identical bit for bit.
Checked on two calls in a row for each precision and tiling, the second with a smaller input
(the array keeps the first call's contents, so anything the second call failed to reset would
show), and a request whose workspace exceeds the array is rejected before any launch.
"""
import numpy as np
import pytest

from oracle import units
from workloads import Cluster, initial_state

from _helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

EPS2 = units.nm_to_norm(0.1, 0.8) ** 2


def _xyzq(n, seed):
    import torch
    n_ion = max(1, n // 2)
    c = Cluster(species="Ar", r0_nm=4.0, n_ion=n_ion, capacity=2 * n_ion, z_init=1)
    st = initial_state(c, seed)
    x = units.nm_to_norm(st["x_nm"], 0.8)[:n]
    q = units.kappa(0.8) * (units.n_atoms(4.0, 2.4) / n_ion) * st["Z"][:n].astype(np.float64)
    q[: n_ion: 5] *= 2.0
    return torch.tensor(np.concatenate([x.T, q[None, :]], axis=0), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision,tiling,phi", [
    ("fp64", None, True),
    ("fp32_acc64", dict(R=4, WJ=4, newton3=1), False),
    ("fp32_acc64", dict(R=1, WJ=4, T=1024, S=8, scalar=1), True),
    ("fp64", dict(R=4, WJ=4, newton3=1), False),
    ("fp32_kahan", dict(R=2, WJ=2, T=256, S=3, persistent=1), True),
])
def test_static_field_equals_field_with_workspace(precision, tiling, phi):
    import torch
    import paper_1307_3711_amd as lc
    t = lc.make_tuning(**tiling) if tiling else None
    for n, seed in ((5003, 1), (1301, 2)):  # the second call is smaller
        xyzq = _xyzq(n, seed)
        E1, P1 = lc.field(xyzq, EPS2, precision=precision, want_phi=phi, tuning=t)
        E2, P2 = lc.field_static(xyzq, EPS2, precision=precision, want_phi=phi, tuning=t)
        torch.cuda.synchronize()
        print(f"{precision} {tiling} n={n}: max |dE| = {float((E1 - E2).abs().max()):.3e}", flush=True)
        assert torch.equal(E1, E2)
        if phi:
            assert torch.equal(P1, P2)
        assert bool(torch.isfinite(E2).all())


def test_static_field_rejects_oversized_requests():
    import ctypes
    import torch
    import paper_1307_3711_amd as lc
    t = lc.make_tuning(R=4, WJ=4, newton3=1)
    L = lc.lib()
    n = 60000  # pair-once rows: 12 B x 235 blocks x 60000 slots, far above the array
    assert L.lc_field_workspace_bytes(1, n, ctypes.byref(t)) > lc.LC_FIELD_STATIC_MAX_BYTES
    xyzq = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    with pytest.raises(lc.LcError):
        lc.field_static(xyzq, EPS2, precision="fp32_acc64", want_phi=False, tuning=t)
    # empty input: nothing to do
    E, P = lc.field_static(torch.zeros((4, 0), dtype=torch.float64, device="cuda"), EPS2)
    assert E.shape == (3, 0)
