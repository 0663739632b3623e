"""An ensemble of 16,500 small argon clusters (more ion blocks than one pass of the spawn-offset
scan covers, 16,384) placed on the device (lc_init_generate) and ionized by a strong flat
field for 12 FP64 steps.  Sampled clusters, in both passes of the scan and at its seam, against
the oracle run of the same cluster from its own placement: identical charges and particle
counts, positions within 1e-9 R0 (the tolerance of the other FP64 runs); every cluster conserves
charge (ion charges equal the electron count) and spawns exactly its ionization events."""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run

from _helpers import descs, gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_many_clusters_scan_passes_and_placement():
    import paper_1307_3711_amd as lc
    n_cl = 16500
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=2, capacity=64, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=3e17, envelope="flat"))
    run = Run(dt=0.05, t0=1.2, ionize=True, diag_every=4, seed=11)
    cfg = lc.make_config("fp64", ionize=True, dt=run.dt, t0=run.t0, softening_nm=run.softening_nm,
                         diag_every=run.diag_every, max_records=8, max_splits=1, seed=run.seed)
    sim = lc.Simulation(cfg, descs([c]) * n_cl)
    sim.init_generate(-1, 1)
    sim.start()
    print(f"{n_cl} clusters: 12 steps", flush=True)
    sim.step(12)
    r0 = units.nm_to_norm(c.r0_nm, 0.8)
    delta = units.nm_to_norm(c.electron_offset_nm, 0.8)
    events = 0
    for k in [0, 1, 777, 16382, 16383, 16384, 16385, 16499]:
        g = sim.particles(k)
        xo, Zo = oracle.init_cluster(run.seed, k, c.n_ion, 1, r0, delta)
        osim = oracle.Sim(oracle.make_params(c, run, cluster_index=k), c.capacity, xo, np.zeros_like(xo), Zo)
        osim.start()
        osim.run(12)
        assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges()), k
        assert np.max(np.abs(g["x"] - osim.positions())) <= 1e-9 * r0, k
        events += osim.N - 4
    ev_total = 0
    for k in range(0, n_cl, 97):
        cnt = sim.counters(k)
        g = sim.particles(k)
        Z = g["Z"].astype(np.int64)
        assert np.sum(Z[Z > 0]) == np.sum(Z < 0)  # charge conservation
        assert cnt["events"] == g["n"] - 4          # one spawned electron per event
        ev_total += cnt["events"]
    print(f"events in sampled clusters: {events} (oracle), {ev_total} over every 97th cluster", flush=True)
    assert events > 0 and ev_total > 0
    sim.close()


def test_spawn_order_with_the_scan_kernel():
    """One cluster of 1,100 ion blocks (281,600 neutral argon atoms, above the 1,024 blocks up to
    which each spawn block sums the earlier blocks' counts itself, so the one-workgroup scan sets
    the ranks): after one step in a strong flat field, the spawned electrons occupy the slots after
    the atoms in ascending order of their parent, each exactly the spawn offset from it (atoms are
    ~0.5 nm apart, far more than the 0.01 nm offset, so any misplaced rank shows), and no slot is
    used twice."""
    import paper_1307_3711_amd as lc
    n_ion = 1100 * 256
    c = Cluster(species="Ar", r0_nm=20.0, n_ion=n_ion, capacity=2 * n_ion, z_init=0, z_max=1,
                laser=Laser(intensity_wcm2=2e15, envelope="flat"))
    run = Run(dt=0.05, t0=1.5, ionize=True, diag_every=0, seed=5)
    cfg = lc.make_config("fp32_acc64", ionize=True, dt=run.dt, t0=run.t0, softening_nm=run.softening_nm,
                         diag_every=0, max_records=1, max_splits=1, seed=run.seed)
    sim = lc.Simulation(cfg, descs([c]))
    sim.init_generate(0, 0)
    sim.start()
    sim.step(1)
    g = sim.particles(0)
    Z = g["Z"]
    flagged = np.nonzero(Z[:n_ion] == 1)[0]
    ne = g["n"] - n_ion
    print(f"scan path: {ne} spawns of {n_ion} atoms", flush=True)
    assert 1000 < ne == flagged.size and np.all(Z[n_ion:] == -1)
    delta = units.nm_to_norm(c.electron_offset_nm, 0.8)
    dist = np.linalg.norm(g["x"][n_ion:] - g["x"][flagged], axis=1)
    assert np.max(np.abs(dist - delta)) <= 1e-9 * delta
    sim.close()
