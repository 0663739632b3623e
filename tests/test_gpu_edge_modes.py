"""Degenerate settings of the optional parts of the step, which must reduce exactly (bitwise)
to simpler runs of the same library: mixed boundaries that switch at or before the start are
open boundaries, ones that never switch are periodic boundaries; the collisional rate with
no electron inside the estimate's sphere adds nothing; detectors that no ion reaches count
nothing."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import units
from workloads import small_ar

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _state_of(run, c, steps=60, states=None, **kw):
    sim, st = gpu_run([c], run, "fp64", states=states, **kw)
    sim.step(steps)
    g = sim.particles(0)
    rec = sim.diagnostics(0)
    sim.close()
    return g, rec, st


@pytest.mark.parametrize("t_switch,equal_to", [(0.0, "open"), (-5.0, "open"), (math.inf, "periodic")])
def test_mixed_boundary_limits(t_switch, equal_to):
    c, run = small_ar()
    mixed = dataclasses.replace(run, boundary="mixed", box_r0=1.6, t_switch=t_switch)
    ref = dataclasses.replace(run, boundary=equal_to, box_r0=1.6)
    g1, r1, _ = _state_of(mixed, c)
    g2, r2, _ = _state_of(ref, c)
    for k in ("x", "u", "Z"):
        assert np.array_equal(g1[k], g2[k])
    assert np.array_equal(r1, r2)


def test_collisional_without_electrons_in_the_sphere():
    """Every electron placed beyond R0 (2 R0 out along its ion's direction): the estimate finds
    no electron, the collisional rate is zero, and the run equals the run without it."""
    c, run = small_ar()
    run = dataclasses.replace(run, collisional=True)
    from workloads import initial_state
    st = initial_state(c, run.seed)
    x = st["x_nm"].copy()
    ions = x[:c.n_ion]
    dirs = ions / np.maximum(np.linalg.norm(ions, axis=1), 1e-12)[:, None]
    x[c.n_ion:] = ions + 2.0 * c.r0_nm * dirs
    st = dict(st, x_nm=x)
    g1, r1, _ = _state_of(run, c, steps=30, states=[st])
    g2, r2, _ = _state_of(dataclasses.replace(run, collisional=False), c, steps=30, states=[st])
    assert np.min(np.linalg.norm(x[c.n_ion:], axis=1)) > c.r0_nm
    for k in ("x", "u", "Z"):
        assert np.array_equal(g1[k], g2[k])
    assert np.array_equal(r1, r2)


def test_detectors_nothing_arrives():
    """Detectors at 50 R0: in 60 steps no ion gets there, every count stays zero, and the run
    itself equals the run without detectors."""
    import paper_1307_3711_amd as lc
    from _helpers import descs
    from workloads import initial_state
    c, run = small_ar()
    st = initial_state(c, run.seed)
    out = []
    for det in (50.0, 0.0):
        cfg = lc.make_config("fp64", ionize=True, dt=run.dt, diag_every=run.diag_every, seed=run.seed,
                             detector_r0=det)
        sim = lc.Simulation(cfg, descs([c]))
        sim.init_from_host(0, st["x_nm"], st["u"], st["Z"])
        sim.start()
        sim.step(60)
        g = sim.particles(0)
        if det:
            counts, _ = sim.iedf(0)
            assert counts.sum() == 0
        out.append((g["x"].copy(), g["u"].copy(), g["Z"].copy()))
        sim.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
