"""The profiling and tuning entry points on a live simulation.

lc_profile_steps is where the benchmark's per-kernel times come from: it must advance the
simulation exactly as lc_step does (bitwise: particles, records, counters, step index) and
count one launch per kernel group and step (the Coulomb pass of a diagnostic step, one-sided
with the potential, is booked under the diagnostics when the tiling is pair-once).
lc_time_particle_kernels returns positive times (zero for the ionization group when ionization
is off).  lc_autotune keeps a tiling whose field matches the default tiling's, appends its
choice to the cache file, and the run continues on it."""
import dataclasses
import json

import numpy as np
import pytest

from workloads import small_ar

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

STEPS = 13  # steps 0, 4, 8 and 12 are diagnostic steps (diag_every = 4)


def _sims(precision, pair_once, ionize=True, count=2):
    """count simulations of the small argon cluster from one initial state (t0 = 25, near the
    peak of the sin^2 envelope, so ions ionize within a few steps)."""
    import paper_1307_3711_amd as lc
    c, run = small_ar()
    run = dataclasses.replace(run, t0=25.0, diag_every=4, ionize=ionize)
    mpb = lc.pair_blocks_for([c.capacity]) if pair_once else 0
    tuning = dict(R=2, WJ=2, newton3=1) if pair_once else None
    sims, st = [], None
    for _ in range(count):
        sim, st = gpu_run([c], run, precision, states=st, max_records=16, tuning=tuning, max_pair_blocks=mpb)
        sims.append(sim)
    return sims


@pytest.mark.parametrize("precision,pair_once", [("fp64", False), ("fp64", True), ("fp32_acc64", False),
                                                 ("fp32_acc64", True)])
def test_profile_steps_advances_like_step(precision, pair_once):
    a, b = _sims(precision, pair_once)
    print(f"{precision} pair_once={pair_once}: {STEPS} steps each way", flush=True)
    a.step(STEPS)
    prof = b.profile_steps(STEPS)
    pa, pb = a.particles(0), b.particles(0)
    assert pa["n"] == pb["n"]
    for k in ("x", "u", "Z"):
        assert np.array_equal(pa[k], pb[k]), k
    ra, rb = a.diagnostics(0), b.diagnostics(0)
    assert ra.shape == rb.shape and ra.shape[0] == 4 and np.array_equal(ra, rb)
    assert a.counters(0) == b.counters(0) and a.step_index == b.step_index == STEPS
    assert a.counters(0)["events"] > 0  # the check and spawn kernels did work
    n_diag = ra.shape[0]
    assert prof["field"][1] == (STEPS - n_diag if pair_once else STEPS)
    assert prof["push"][1] == STEPS and prof["diag"][1] == n_diag and prof["ionize"][1] == STEPS
    assert all(ms > 0.0 for ms, n in prof.values())
    a.close()
    b.close()


@pytest.mark.parametrize("ionize", [True, False])
def test_time_particle_kernels(ionize):
    (a,) = _sims("fp32_acc64", True, ionize=ionize, count=1)
    a.step(3)
    t = a.time_particle_kernels(5)
    print(t, flush=True)
    assert t["push_ms"] > 0.0
    assert (t["ionize_ms"] > 0.0) if ionize else (t["ionize_ms"] == 0.0)
    a.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_acc64"])
def test_autotune_choice_and_cache(precision, tmp_path):
    a, b = _sims(precision, False)
    a.step(2)
    b.step(2)
    cache = tmp_path / "tune.jsonl"
    chosen = a.autotune(str(cache))
    print(precision, chosen, flush=True)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert [rec[k] for k in ("R", "WJ", "T", "S", "newton3")] == \
        [chosen[k] for k in ("R", "WJ", "T", "S", "newton3")]
    assert rec["rel_err_vs_default"] <= (1e-12 if precision == "fp64" else 1e-5)
    assert rec["candidates"] > 1 and a.tuning() == chosen
    # the tuner restores the state: the field on the chosen tiling matches the untuned run's
    Ea, Eb = a.field(0), b.field(0)
    s = np.linalg.norm(Eb)
    assert np.linalg.norm(Ea - Eb) <= (1e-12 if precision == "fp64" else 1e-5) * s
    # and the run goes on
    a.step(3)
    b.step(3)
    assert a.counters(0)["steps"] == b.counters(0)["steps"] == 5
    if precision == "fp64":
        dx = np.max(np.abs(a.particles(0)["x"] - b.particles(0)["x"]))
        assert dx <= 1e-12 * np.max(np.abs(b.particles(0)["x"]))
    a.close()
    b.close()
