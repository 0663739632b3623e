"""Degenerate clusters side by side in one ensemble, each against its own oracle run, in FP64
pairs and in FP32 pairs with FP64 accumulation (one-sided and pair-once passes): an empty
cluster (no macroparticle, explicit weight), a single neutral atom (weight 1: one real atom,
so its bound electrons stay resolved at this dt) that a strong flat field strips to Ar8+ and
so fills its capacity of 9 exactly, a cluster whose live count is exactly
one 64-slot group at the start, one whose live count is one past a group, and an ordinary
small cluster.  Placement on the device (lc_init_generate) against the oracle's own placement.

Bar: identical charge arrays, particle counts and ionization events (the laser-only rate
depends on charge and time only and both sides draw the same numbers); positions within
1e-9 R0 (FP64) or 1e-4 R0 (FP32 pairs, 12 steps); energy records within 1e-10 (FP64) or 1e-4
(FP32) of each column's scale; the empty cluster's records all zero."""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run

from _helpers import descs, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

LASER = Laser(intensity_wcm2=3e17, envelope="flat")
# (cluster, z_init, weight or None)
CASES = [
    (Cluster(species="Ar", r0_nm=1.5, n_ion=40, capacity=400, z_init=1, z_max=8, laser=LASER), 1, None),
    (Cluster(species="Ar", r0_nm=1.0, n_ion=0, capacity=64, z_init=1, z_max=8, laser=LASER), 1, 1.0),
    (Cluster(species="Ar", r0_nm=1.0, n_ion=1, capacity=9, z_init=0, z_max=8, laser=LASER), 0, 1.0),
    (Cluster(species="Ar", r0_nm=1.2, n_ion=32, capacity=640, z_init=1, z_max=8, laser=LASER), 1, None),
    (Cluster(species="Ar", r0_nm=1.2, n_ion=65, capacity=585, z_init=0, z_max=8, laser=LASER), 0, None),
]
STEPS = 12


@pytest.mark.parametrize("precision,pair_once", [("fp64", False), ("fp64", True), ("fp32_acc64", False),
                                                 ("fp32_acc64", True)])
def test_degenerate_clusters_against_oracle(precision, pair_once):
    import paper_1307_3711_amd as lc
    run = Run(dt=0.05, t0=1.2, ionize=True, diag_every=4, seed=5)
    clusters = [c for c, _, _ in CASES]
    mpb = lc.pair_blocks_for([c.capacity for c in clusters]) if pair_once else 0
    cfg = lc.make_config(precision, ionize=True, dt=run.dt, t0=run.t0, softening_nm=run.softening_nm,
                         diag_every=run.diag_every, max_records=16, max_splits=4, seed=run.seed,
                         max_pair_blocks=mpb)
    ds = descs(clusters)
    for d, (_, _, w) in zip(ds, CASES):
        if w is not None:
            d.weight = w
    sim = lc.Simulation(cfg, ds)
    if pair_once:
        sim.set_tuning(R=2, WJ=2, newton3=1)
    for k, (_, z0, _) in enumerate(CASES):
        sim.init_generate(k, z0)
    sim.start()
    print(f"{precision} pair_once={pair_once}: {STEPS} steps", flush=True)
    sim.step(STEPS)
    xtol, etol = (1e-9, 1e-10) if precision == "fp64" else (1e-4, 1e-4)
    for k, (c, z0, w) in enumerate(CASES):
        r0 = units.nm_to_norm(c.r0_nm, 0.8)
        delta = units.nm_to_norm(c.electron_offset_nm, 0.8)
        xo, Zo = oracle.init_cluster(run.seed, k, c.n_ion, z0, r0, delta)
        osim = oracle.Sim(oracle.make_params(c, run, cluster_index=k, weight=w), c.capacity, xo, np.zeros_like(xo), Zo)
        osim.start()
        ro = osim.run(STEPS)
        g = sim.particles(k)
        rg = sim.diagnostics(k)
        cnt = sim.counters(k)
        assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges()), k
        assert rg.shape == ro.shape and np.array_equal(rg[:, 21], ro[:, 21]), k
        assert np.array_equal(rg[:, 24:41], ro[:, 24:41]), k
        # every event spawns one electron (none dropped here); the last record is from step 8
        assert not np.any(ro[:, 20]) and cnt["events"] == osim.N - len(Zo) and cnt["steps"] == STEPS, (k, cnt)
        if osim.N:
            dx = np.max(np.abs(g["x"] - osim.positions())) / r0
            assert dx <= xtol, (k, dx)
        for col in [5, 6, 7, 8, 9, 10]:
            sc = np.max(np.abs(ro[:, col]))
            err = np.max(np.abs(rg[:, col] - ro[:, col]))
            assert err <= etol * sc, (k, col, err, sc)
        print(f"cluster {k}: N {len(Zo)} -> {osim.N}, events {cnt['events']}", flush=True)
    assert sim.particles(1)["n"] == 0 and not np.any(sim.diagnostics(1)[:, 5:11])
    assert sim.particles(2)["n"] == 9 and sim.particles(2)["Z"][0] == 8  # capacity reached exactly
    sim.close()
