"""The particle-kernel benchmark's configuration at its full size (1024 argon clusters of 2048
Ar+ and 2048 electrons, capacity 8192 each, FP32 sources with one split, ionization in a flat
1e15 W/cm^2 field), stepped for real: sampled clusters against their own oracle runs from the
same start.  Bar as for the other FP32 runs: identical charges and particle counts (the
laser-only rate depends on charge and time only), positions within 1e-4 R0 after 3 steps."""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run, initial_state

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_particles_workload_sampled_against_oracle():
    nc = 1024
    c = Cluster(species="Ar", r0_nm=6.0, n_ion=2048, capacity=8192, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=1e15, envelope="flat"))
    run = Run(dt=0.05, t0=1.3, ionize=True, diag_every=0, seed=1)
    st = initial_state(c, 1, 0)
    print(f"{nc} clusters x {st['x_nm'].shape[0]} macroparticles: 3 steps", flush=True)
    sim, _ = gpu_run([c] * nc, run, "fp32_acc64", states=[st] * nc, max_records=1, max_splits=1,
                     tuning=dict(S=1))
    sim.step(3)
    r0 = units.nm_to_norm(c.r0_nm, c.laser.lambda_um)
    events = 0
    for k in (0, 511, 1023):
        osim = oracle.Sim.from_workload(c, run, st, k)
        osim.start()
        osim.run(3)
        g = sim.particles(k)
        assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges()), k
        dx = np.max(np.abs(g["x"] - osim.positions())) / r0
        print(f"cluster {k}: N {osim.N}, max|dx|/R0 {dx:.2e}", flush=True)
        assert dx <= 1e-4, (k, dx)
        events += osim.N - st["x_nm"].shape[0]
    assert events > 0
    sim.close()
