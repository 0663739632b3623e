"""GPU parity of the collisional ionization rate (Sec. II: nu_total = nu_ofi + nu_ci; Lotz rate
over the electron density and temperature of the cluster sphere) against the oracle.

Both sides draw the same Philox numbers and decide alpha < P in FP64, so the FP64 path must
produce the same ionization events.  Electrons hot enough to ionize by impact make the orbits
chaotic (rounding differences grow by orders of magnitude within the run), so states and
energy records are held, as for the long ensemble runs, within 100x the spread of
rounding-perturbed oracle runs (and within 1e-9 / 1e-10 where that spread is smaller).  The
case checks on the oracle that the collisional term changes the events, so it is exercised.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run, initial_state

from _helpers import gpu_available, gpu_run, oracle_spread

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_collisional_warm_cluster():
    """Small Ar cluster (500 Ar+ + 500 e-, R0 = 2.5 nm) whose electrons start with 30 eV in random
    directions, in a weak flat field (1e15 W/cm^2), 200 steps: collisions do most of the
    ionizing."""
    c = Cluster(species="Ar", r0_nm=2.5, n_ion=500, capacity=4500, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=1e15, envelope="flat"))
    run = Run(dt=0.05, ionize=True, collisional=True, diag_every=10, seed=4)
    st = initial_state(c, run.seed)
    rng = np.random.default_rng(8)
    v = rng.normal(size=(c.n_ion, 3))
    g = 1.0 + 30.0 / units.MEC2_EV
    v *= (np.sqrt(g * g - 1.0) / np.linalg.norm(v, axis=1))[:, None]
    st["u"] = st["u"].copy()
    st["u"][c.n_ion:] = v
    sim, _ = gpu_run([c], run, "fp64", states=[st])
    ref = oracle.Sim.from_workload(c, dataclasses.replace(run, collisional=False), st)
    ref.start()
    ref.run(200)
    sim.step(200)
    osim, ro, spread = oracle_spread(c, run, st, 0, 200)
    rg = sim.diagnostics(0)
    print(f"events: gpu {rg[-1][21]}, oracle {ro[-1][21]}, oracle without collisions {ref.counters[1]}", flush=True)
    assert ro[-1][21] > ref.counters[1] + 50
    g = sim.particles(0)
    assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges())
    assert np.array_equal(rg[:, 21], ro[:, 21]) and np.array_equal(rg[:, 24:41], ro[:, 24:41])
    r0n = units.nm_to_norm(c.r0_nm, 0.8)
    dx = np.max(np.abs(g["x"] - osim.positions())) / r0n
    du = np.max(np.abs(g["u"] - osim.momenta())) / np.max(np.abs(osim.momenta()))
    print(f"dx={dx:.2e} (spread {spread['dx']:.2e}) du={du:.2e} (spread {spread['du']:.2e})", flush=True)
    assert dx <= max(1e-9, 100 * spread["dx"]) and du <= max(1e-9, 100 * spread["du"])
    for col, sp in spread["cols"].items():
        sc = np.max(np.abs(ro[:, col])) + 1e-300
        err = np.max(np.abs(rg[:, col] - ro[:, col])) / sc
        assert err <= max(1e-10, 100 * sp), (col, err, sp)
    sim.close()
