"""Seeded random runs stepped two ways, bitwise: one step per call (every step ends with its
schedule) against captured groups of steps (hipGraph replays; without ionization the schedule
is left out between steps of a group and the force launches do the step bookkeeping).  Random
cluster mixes with random retirement steps, precision, tiling, ionization, boundary mode
(open, periodic, or periodic switching to open inside the run), diagnostic interval and group
length.  Particles, diagnostic records and per-cluster counters must be identical."""
import numpy as np
import pytest

from workloads import Cluster, Laser, Run, initial_state

from _helpers import gpu_available, gpu_run

ONE_SIDED = [dict(R=2, WJ=2, T=256, S=3), dict(R=4, WJ=4, T=512, S=2), dict(R=1, WJ=4, T=128, S=5, persistent=1)]
PAIR_ONCE = [dict(R=4, WJ=4, newton3=1), dict(R=2, WJ=2, newton3=1, persistent=1), dict(R=3, WJ=3, newton3=1)]


def _case(k):
    rng = np.random.default_rng(7100 + k)
    precision = ["fp64", "fp32_acc64"][k % 2]
    tiling = (ONE_SIDED + PAIR_ONCE)[int(rng.integers(len(ONE_SIDED) + len(PAIR_ONCE)))]
    # the twelve cases take every combination of precision, ionization and boundary mode once
    ionize = (k // 2) % 2 == 1
    boundary = ["open", "periodic", "mixed"][k % 3]
    steps = int(rng.integers(60, 121))
    clusters, n_steps = [], []
    for _ in range(int(rng.integers(1, 6))):
        n_ion = int(rng.integers(1, 200))
        z_max = int(rng.integers(2, 9))
        laser = Laser(intensity_wcm2=float(10 ** rng.uniform(15, 17)),
                      envelope=["gauss_field", "sin2", "flat"][int(rng.integers(3))],
                      polarization=["linear_x", "circular"][int(rng.integers(2))])
        clusters.append(Cluster(species=["Ar", "Xe"][int(rng.integers(2))], r0_nm=float(rng.uniform(1.0, 2.5)),
                                n_ion=n_ion, capacity=n_ion * (1 + z_max) + int(rng.integers(0, 64)), z_init=1,
                                z_max=z_max, laser=laser))
        n_steps.append(int(rng.integers(steps // 3, steps + 20)))
    dt = 0.05
    t0 = float(rng.uniform(0.0, 40.0))
    run = Run(dt=dt, t0=t0, ionize=ionize, diag_every=int(rng.choice([3, 7, 10])), seed=int(rng.integers(1000)),
              boundary=boundary, t_switch=t0 + dt * float(rng.integers(10, steps)) if boundary == "mixed" else np.inf)
    graph = int(rng.choice([5, 16, 40]))
    return precision, tiling, run, clusters, n_steps, steps, graph


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("k", range(12))
def test_graph_groups_match_single_steps(k):
    import paper_1307_3711_amd as lc
    precision, tiling, run, clusters, n_steps, steps, graph = _case(k)
    print(f"case {k}: {precision} {tiling} ionize={run.ionize} {run.boundary} diag_every={run.diag_every} "
          f"graph={graph} steps={steps} n_steps={n_steps}", flush=True)
    states = [initial_state(c, run.seed, i) for i, c in enumerate(clusters)]
    mpb = lc.pair_blocks_for([c.capacity for c in clusters]) if tiling.get("newton3") else 0
    out = []
    for g in (0, graph):
        sim, _ = gpu_run(clusters, run, precision, states=states, max_records=64, n_steps_per_cluster=n_steps,
                         tuning=tiling, max_pair_blocks=mpb)
        if g:
            sim.set_graph(g)
        sim.step(steps)
        out.append([(sim.particles(i), sim.diagnostics(i), sim.counters(i)) for i in range(len(clusters))])
        sim.close()
    for i, ((p0, r0, c0), (p1, r1, c1)) in enumerate(zip(out[0], out[1])):
        assert p0["n"] == p1["n"] and c0 == c1, (i, c0, c1)
        for key in ("x", "u", "Z", "wl", "wc"):
            assert np.array_equal(p0[key], p1[key]), (i, key)
        assert np.array_equal(r0, r1), i
        assert c0["steps"] == min(steps, n_steps[i]), (i, c0)


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("k", [1, 2, 5, 6, 9, 10])
def test_checkpoint_mid_run_resumes_bitwise(k, tmp_path):
    """Six of the random runs (both precisions, with and without ionization, every boundary
    mode) with captured groups, saved part way (between groups or inside one, wherever the
    split falls) and resumed in a fresh handle: identical to the unbroken run."""
    import paper_1307_3711_amd as lc
    precision, tiling, run, clusters, n_steps, steps, graph = _case(k)
    split = steps // 2 + k
    print(f"case {k}: {precision} ionize={run.ionize} {run.boundary}: save at step {split} of {steps}", flush=True)
    states = [initial_state(c, run.seed, i) for i, c in enumerate(clusters)]
    mpb = lc.pair_blocks_for([c.capacity for c in clusters]) if tiling.get("newton3") else 0

    def make():
        sim, _ = gpu_run(clusters, run, precision, states=states, max_records=64, n_steps_per_cluster=n_steps,
                         tuning=tiling, max_pair_blocks=mpb)
        sim.set_graph(graph)
        return sim

    ref = make()
    ref.step(steps)
    a = make()
    a.step(split)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    a.close()
    b = make()
    b.load(path)
    assert b.step_index == split
    b.step(steps - split)
    for i in range(len(clusters)):
        p0, p1 = ref.particles(i), b.particles(i)
        for key in ("x", "u", "Z", "wl", "wc"):
            assert np.array_equal(p0[key], p1[key]), (i, key)
        assert np.array_equal(ref.diagnostics(i), b.diagnostics(i)) and ref.counters(i) == b.counters(i), i
    ref.close()
    b.close()


def test_graph_cases_cover_the_modes():
    cases = [_case(k) for k in range(12)]
    assert {c[0] for c in cases} == {"fp64", "fp32_acc64"}
    assert len({(c[0], c[2].ionize, c[2].boundary) for c in cases}) == 12
    assert any(c[2].ionize for c in cases) and any(not c[2].ionize for c in cases)
    assert any(c[1].get("newton3") for c in cases) and any(not c[1].get("newton3") for c in cases)
    # some cluster retires inside the run
    assert any(min(c[4]) < c[5] for c in cases)
