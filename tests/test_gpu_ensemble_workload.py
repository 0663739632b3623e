"""The ensemble benchmark's configuration at its full size (256 uneven Ar/Xe clusters,
capacities 1k-16k, R0 2-10 nm, 1e15-1e17 W/cm^2, FWHM 20-100 fs, ionization on) in the
pair-once persistent pass the ensemble runner settles on, started at t = 150 (near the peak of
the shorter pulses, so clusters ionize) and stepped for real: the smallest and largest
clusters and two others against their own oracle runs from the same start.  Bar: identical
charges and particle counts; positions within 1e-9 R0 in FP64 pairs and 1e-4 R0 in FP32 pairs
after 3 steps."""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Run, ensemble, initial_state

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_ensemble_workload_sampled_against_oracle(precision):
    import paper_1307_3711_amd as lc
    cl = ensemble(256, seed=0)
    run = Run(dt=0.05, t0=150.0, ionize=True, diag_every=0, seed=0)
    states = [initial_state(c, run.seed, i) for i, c in enumerate(cl)]
    caps = [c.capacity for c in cl]
    tiling = dict(R=4, WJ=4, persistent=1, newton3=1)
    print(f"{precision}: 256 clusters, {sum(s['x_nm'].shape[0] for s in states)} macroparticles, 3 steps", flush=True)
    sim, _ = gpu_run(cl, run, precision, states=states, max_records=1, tuning=tiling,
                     max_pair_blocks=lc.pair_blocks_for(caps))
    sim.step(3)
    tol = 1e-9 if precision == "fp64" else 1e-4
    picks = sorted({int(np.argmin(caps)), int(np.argmax(caps)), 7, 200})
    events = 0
    for k in picks:
        c = cl[k]
        osim = oracle.Sim.from_workload(c, run, states[k], k)
        osim.start()
        osim.run(3)
        g = sim.particles(k)
        assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges()), k
        r0 = units.nm_to_norm(c.r0_nm, c.laser.lambda_um)
        dx = np.max(np.abs(g["x"] - osim.positions())) / r0
        print(f"cluster {k} ({c.species}, capacity {c.capacity}): N {osim.N}, max|dx|/R0 {dx:.2e}", flush=True)
        assert dx <= tol, (k, dx)
        events += osim.N - states[k]["x_nm"].shape[0]
    print(f"events in the sampled clusters: {events}", flush=True)
    sim.close()
