"""GPU parity of the seeded initial placement (lc_init_generate; Sec. II random atoms inside R0,
lumped into ion macroparticles, each with z_init electrons at the spawn offset) against the
oracle's placement from the same Philox counters.

Tolerances (fixed before measuring): charges and slot order identical; positions within 16 ulp
of R0 (the device's cube root, sine and cosine against the host library's, a few ulp each);
a 200-step FP64 run started from the device placement matches the oracle started from its own
placement as the host-uploaded runs do (max |dx| / R0 <= 1e-9, energies 1e-10).
"""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, small_ar

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _sim(clusters, run, precision="fp64"):
    import paper_1307_3711_amd as lc
    from _helpers import descs
    cfg = lc.make_config(precision, ionize=run.ionize, dt=run.dt, softening_nm=run.softening_nm,
                         diag_every=run.diag_every, max_records=64, seed=run.seed)
    return lc.Simulation(cfg, descs(clusters))


@pytest.mark.parametrize("z_init", [0, 1, 3])
def test_placement_matches_oracle(z_init):
    clusters = [Cluster(species="Ar", r0_nm=2.5, n_ion=500, capacity=4500, z_init=z_init),
                Cluster(species="Xe", r0_nm=6.0, n_ion=1031, capacity=9000, z_init=z_init)]
    c, run = small_ar()
    sim = _sim(clusters, run)
    sim.init_generate(-1, z_init)
    for k, cl in enumerate(clusters):
        g = sim.particles(k)
        r0 = units.nm_to_norm(cl.r0_nm, 0.8)
        xo, Zo = oracle.init_cluster(run.seed, k, cl.n_ion, z_init, r0,
                                     units.nm_to_norm(cl.electron_offset_nm, 0.8))
        print(f"cluster {k} z_init {z_init}: n {g['n']} max |dx| / R0 = "
              f"{np.max(np.abs(g['x'] - xo)) / r0:.2e}", flush=True)
        assert g["n"] == cl.n_ion * (1 + z_init)
        assert np.array_equal(g["Z"], Zo)
        assert np.all(g["u"] == 0.0)
        assert np.max(np.abs(g["x"] - xo)) <= 16 * 2.0**-52 * r0
    sim.close()


def test_single_cluster_and_errors():
    import paper_1307_3711_amd as lc
    clusters = [Cluster(species="Ar", r0_nm=2.5, n_ion=100, capacity=250, z_init=1, z_max=2),
                Cluster(species="Ar", r0_nm=3.0, n_ion=64, capacity=128, z_init=1, z_max=2)]
    c, run = small_ar()
    sim = _sim(clusters, run)
    with pytest.raises(lc.LcError):
        sim.start()  # nothing placed yet
    with pytest.raises(lc.LcError):
        sim.init_generate(-1, 2)  # 100 (1 + 2) > 250
    with pytest.raises(lc.LcError):
        sim.init_generate(1, 3)  # above z_max
    with pytest.raises(lc.LcError):
        sim.init_generate(2, 1)  # no such cluster
    sim.init_generate(1, 1)
    with pytest.raises(lc.LcError):
        sim.start()  # cluster 0 still missing
    sim.init_generate(0, 1)
    sim.start()
    sim.step(3)  # the sin^2 envelope is still far too weak to ionize
    assert sim.particles(0)["n"] == 200 and sim.particles(1)["n"] == 128
    sim.close()


def test_run_from_device_placement_matches_oracle():
    c, run = small_ar()
    sim = _sim([c], run)
    sim.init_generate(0, c.z_init)
    sim.start()
    r0 = units.nm_to_norm(c.r0_nm, 0.8)
    xo, Zo = oracle.init_cluster(run.seed, 0, c.n_ion, c.z_init, r0, units.nm_to_norm(c.electron_offset_nm, 0.8))
    osim = oracle.Sim(oracle.make_params(c, run), c.capacity, xo, np.zeros_like(xo), Zo)
    osim.start()
    sim.step(200)
    rg = sim.diagnostics(0)
    ro = osim.run(200)
    g = sim.particles(0)
    assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges())
    dx = np.max(np.abs(g["x"] - osim.positions())) / r0
    print(f"device placement, 200 FP64 steps: max |dx| / R0 = {dx:.2e}, events {rg[-1][21]:.0f}", flush=True)
    assert dx <= 1e-9
    for col in (5, 6, 7, 8, 9, 10):
        scale = np.max(np.abs(ro[:, col])) + 1e-300
        assert np.max(np.abs(rg[:, col] - ro[:, col])) / scale <= 1e-10
    assert np.array_equal(rg[:, 21], ro[:, 21])
    sim.close()
