"""The widened features inside multi-cluster launches (every per-cluster table indexed by the
cluster) and combined with each other, against one oracle run per cluster (FP64).

Detectors: each cluster's histogram equals its own oracle run's exactly.  Collisional
ionization: each cluster's ionization events equal its oracle run's (the estimate is per
cluster).  Circular polarization in a periodic cube: states within 1e-9 R0 of the oracle.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run, initial_state, small_ar

from _helpers import descs, gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_ensemble_detectors_per_cluster():
    """Two deuterium spheres of different size and placement exploding in one launch."""
    import paper_1307_3711_amd as lc
    cl = [Cluster(species="D", r0_nm=3.0, n_ion=800, capacity=1600, z_init=1,
                  laser=Laser(envelope="flat", intensity_wcm2=0.0)),
          Cluster(species="D", r0_nm=2.0, n_ion=300, capacity=600, z_init=1,
                  laser=Laser(envelope="flat", intensity_wcm2=0.0))]
    run = Run(dt=2.0, ionize=False, diag_every=0, softening_nm=0.01)
    states = []
    for i, c in enumerate(cl):
        st = initial_state(c, 9, i)
        n = c.n_ion
        states.append({"x_nm": st["x_nm"][:n], "u": st["u"][:n], "Z": st["Z"][:n], "n_ion": n})
    cfg = lc.make_config("fp64", ionize=False, dt=run.dt, softening_nm=run.softening_nm, diag_every=0,
                         detector_r0=9.0, detector_half_angle_deg=30.0)
    sim = lc.Simulation(cfg, descs(cl))
    for i, st in enumerate(states):
        sim.init_from_host(i, st["x_nm"], st["u"], st["Z"])
    sim.start()
    sim.step(3000)
    for i, c in enumerate(cl):
        osim = oracle.Sim.from_workload(c, run, states[i], cluster_index=i)
        osim.enable_detectors(9.0 * osim.r0_norm, 30.0)
        osim.start()
        osim.run(3000)
        g, _ = sim.iedf(i)
        o, _ = osim.iedf()
        print(f"cluster {i}: detected gpu {g[0].sum()} oracle {o[0].sum()}", flush=True)
        assert g[0].sum() == c.n_ion and np.array_equal(g, o)
    sim.close()


def test_ensemble_collisional_per_cluster():
    """Two warm argon clusters (30 eV electrons) of different size in one launch: the electron
    density and temperature are estimated per cluster."""
    cl = [Cluster(species="Ar", r0_nm=2.5, n_ion=500, capacity=4500, z_init=1, z_max=8,
                  laser=Laser(intensity_wcm2=1e15, envelope="flat")),
          Cluster(species="Ar", r0_nm=2.0, n_ion=250, capacity=2250, z_init=1, z_max=8,
                  laser=Laser(intensity_wcm2=1e15, envelope="flat"))]
    run = Run(dt=0.05, ionize=True, collisional=True, diag_every=10, seed=4)
    rng = np.random.default_rng(8)
    states = []
    for i, c in enumerate(cl):
        st = initial_state(c, run.seed, i)
        v = rng.normal(size=(c.n_ion, 3))
        g = 1.0 + 30.0 / units.MEC2_EV
        v *= (np.sqrt(g * g - 1.0) / np.linalg.norm(v, axis=1))[:, None]
        st["u"] = st["u"].copy()
        st["u"][c.n_ion:] = v
        states.append(st)
    sim, _ = gpu_run(cl, run, "fp64", states=states)
    sim.step(100)
    for i, c in enumerate(cl):
        osim = oracle.Sim.from_workload(c, run, states[i], cluster_index=i)
        osim.start()
        ro = osim.run(100)
        rg = sim.diagnostics(i)
        print(f"cluster {i}: events gpu {rg[-1][21]} oracle {ro[-1][21]}", flush=True)
        assert ro[-1][21] > 0
        assert np.array_equal(rg[:, 21], ro[:, 21]) and np.array_equal(sim.particles(i)["Z"], osim.charges())
    sim.close()


@pytest.mark.parametrize("tiling", [None, dict(R=4, WJ=4, newton3=1)])
def test_circular_in_periodic_cube(tiling):
    import paper_1307_3711_amd as lc
    c, run = small_ar()
    c = dataclasses.replace(c, laser=dataclasses.replace(c.laser, polarization="circular"))
    run = dataclasses.replace(run, boundary="periodic", box_r0=1.6)
    mpb = lc.pair_blocks_for([c.capacity]) if tiling else 0
    sim, states = gpu_run([c], run, "fp64", tuning=tiling, max_pair_blocks=mpb)
    osim = oracle.Sim.from_workload(c, run, states[0])
    osim.start()
    sim.step(200)
    osim.run(200)
    g = sim.particles(0)
    assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges())
    dx = np.max(np.abs(g["x"] - osim.positions())) / units.nm_to_norm(c.r0_nm, 0.8)
    print(f"circular + periodic {tiling}: max|dx|/R0 = {dx:.3e}", flush=True)
    assert dx <= 1e-9
    sim.close()


def test_adaptive_pass_choice_keeps_the_run_exact():
    """An autotuned ensemble run that checks, on real steps, whether the pair-once pass has
    become faster (the pass may change mid-run): every cluster takes exactly its steps and
    retires, the tiling log starts with the autotuner's choice and can only add the pair-once
    pass, and the exact discrete energy identity KE(n+1/2) - KE(-1/2) = W_L + W_C + spawn KE
    holds for every cluster (it holds for whatever field each step used)."""
    import paper_1307_3711_amd as lc
    from paper_1307_3711_amd.ensemble import run_ensemble
    from workloads import ensemble, initial_state
    from workloads.species import SPECIES
    cl = ensemble(24, seed=9, cap_lo=300, cap_hi=3000)
    steps = [1200 + 60 * i for i in range(len(cl))]
    descs = [lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                             envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max, n_steps=n)
             for c, n in zip(cl, steps)]
    states = [initial_state(c, 9, i) for i, c in enumerate(cl)]
    r = run_ensemble(descs, states, "fp32_acc64", seed=9, diag_every=50, graph_steps=10, probe_steps=40)
    print("tilings:", r["tunings"], flush=True)
    assert 1 <= len(r["tunings"]) <= 2 and r["tunings"][0]["at_step"] == 0
    if len(r["tunings"]) == 2:
        assert r["tunings"][1]["newton3"] == 1 and r["tunings"][0]["newton3"] == 0
    for i, cnt in enumerate(r["counters"]):
        assert cnt["steps"] == steps[i]
    rec = r["last"]
    ident = np.abs(rec[:, 5] - rec[:, 23] - (rec[:, 8] + rec[:, 9] + rec[:, 10]))
    scale = np.abs(rec[:, 8]) + np.abs(rec[:, 9]) + rec[:, 10] + np.abs(rec[:, 23])
    assert np.max(ident / scale) <= 1e-11
