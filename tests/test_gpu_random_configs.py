"""Seeded random configurations against the oracle: ensembles of one to four clusters with
random species, radius, ion count (edge counts 0, 1, 63, 64, 65 among them), initial charge,
charge cap, capacity slack, intensity, envelope, polarization and start time, each run in a
random precision, tiling (one-sided or pair-once, plain or persistent, LDS or scalar sources),
boundary mode and (FP64) tunnelling field and collisional rate, with device placement (lc_init_generate) against the oracle's own, for 10
steps with diagnostics every 2-5 steps.

Bar: identical particle counts, charge arrays, ionization events and charge histograms
(laser-only rates depend on charge and time only, and both sides draw the same numbers);
positions within 1e-9 R0 (FP64) or 1e-4 R0 (FP32 pairs); energy records within 1e-10 (FP64) or
1e-4 (FP32) of each column's scale.  FP64 cases keep the lumping of Eq.(1) (weights up to
hundreds of atoms per macroparticle).  FP32 cases set the weight to 0.5-1.5 atoms: an electron
inside the softening core (0.1 nm) of a macro-ion of charge Z w turns by about 0.34 (Z w)^(1/2)
radians per step (dt = 0.05 in 1/w), and with tens of atoms per macroparticle that is beyond the
leap-frog's stability limit of 2, where the FP32 rounding of the pair differences (about 200 u
of the bound pair's separation) grows by orders of magnitude within ten steps (the FP64 path's
1e-16 grows too, but stays far below its bar)."""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run

from _helpers import descs, gpu_available


ONE_SIDED = [{}, dict(R=1, WJ=1, T=64, S=1), dict(R=2, WJ=2, T=256, S=3), dict(R=4, WJ=4, T=512, S=2),
             dict(R=1, WJ=4, T=128, S=5, persistent=1), dict(R=2, WJ=1, T=1920, S=1, persistent=1)]
SCALAR = [dict(R=1, WJ=4, T=1024, S=7, scalar=1), dict(R=2, WJ=2, T=256, S=3, persistent=1, scalar=1)]
PAIR_ONCE = [dict(R=1, WJ=1, newton3=1), dict(R=2, WJ=1, newton3=1), dict(R=2, WJ=2, newton3=1, persistent=1),
             dict(R=4, WJ=2, newton3=1), dict(R=4, WJ=4, newton3=1), dict(R=3, WJ=3, newton3=1),
             dict(R=5, WJ=5, newton3=1)]
EDGE_IONS = [0, 1, 63, 64, 65]
STEPS = 10


def _case(k):
    rng = np.random.default_rng(9000 + k)
    precision = ["fp64", "fp32_acc64"][k % 2]
    # FP64 has no scalar-source path and no (2, 1) pair-once shape (its LDS would exceed 64 KB)
    tilings = ONE_SIDED + PAIR_ONCE + SCALAR if precision != "fp64" else \
        ONE_SIDED + [t for t in PAIR_ONCE if (t["R"], t["WJ"]) != (2, 1)]
    tiling = tilings[int(rng.integers(len(tilings)))]
    boundary = "periodic" if (precision == "fp64" and rng.random() < 0.3) else "open"
    clusters, weights, z0s = [], [], []
    for _ in range(int(rng.integers(1, 5))):
        species = ["Ar", "Xe"][int(rng.integers(2))]
        n_ion = int(rng.choice(EDGE_IONS)) if rng.random() < 0.3 else int(rng.integers(2, 400))
        z_max = int(rng.integers(2, 9))
        z0 = int(rng.integers(0, 2))
        cap = max(n_ion * (1 + z_max) + int(rng.integers(0, 100)), 1)
        laser = Laser(intensity_wcm2=float(10 ** rng.uniform(15, 17.5)),
                      envelope=["gauss_field", "sin2", "flat"][int(rng.integers(3))],
                      fwhm_fs=float(rng.uniform(10, 40)), n_cycles=float(rng.uniform(6, 14)),
                      polarization=["linear_x", "circular"][int(rng.integers(2))])
        clusters.append(Cluster(species=species, r0_nm=float(rng.uniform(1.0, 3.0)), n_ion=n_ion, capacity=cap,
                                z_init=z0, z_max=z_max, laser=laser))
        w32 = float(rng.uniform(0.5, 1.5))
        weights.append(w32 if precision != "fp64" else (1.0 if n_ion == 0 else None))
        z0s.append(z0)
    # FP64 cases also draw the local-field tunnelling rate and the collisional rate (both sides
    # take every ionization decision in FP64, so the events stay identical)
    ofi = "local" if (precision == "fp64" and rng.random() < 0.3) else "laser_only"
    collisional = bool(precision == "fp64" and rng.random() < 0.3)
    run = Run(dt=0.05, t0=float(rng.uniform(0.0, 60.0)), ionize=True, diag_every=int(rng.choice([2, 3, 5])),
              seed=int(rng.integers(1000)), boundary=boundary, ofi_field=ofi, collisional=collisional)
    return precision, tiling, run, clusters, weights, z0s


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("k", range(24))
def test_random_configuration_against_oracle(k):
    import paper_1307_3711_amd as lc
    precision, tiling, run, clusters, weights, z0s = _case(k)
    print(f"case {k}: {precision} {tiling} {run.boundary} {run.ofi_field} collisional={run.collisional} "
          f"t0={run.t0:.1f} diag_every={run.diag_every} "
          f"clusters {[(c.species, c.n_ion, c.capacity, c.z_init, c.z_max) for c in clusters]}", flush=True)
    pair_once = tiling.get("newton3", 0) == 1
    mpb = lc.pair_blocks_for([c.capacity for c in clusters]) if pair_once else 0
    cfg = lc.make_config(precision, ionize=True, dt=run.dt, t0=run.t0, softening_nm=run.softening_nm,
                         diag_every=run.diag_every, max_records=16, max_splits=8, seed=run.seed,
                         max_pair_blocks=mpb, boundary=run.boundary, box_r0=run.box_r0, ofi_field=run.ofi_field,
                         collisional=run.collisional)
    ds = descs(clusters)
    for d, w in zip(ds, weights):
        if w is not None:
            d.weight = w
    sim = lc.Simulation(cfg, ds)
    if tiling:
        sim.set_tuning(**tiling)
    for i, z0 in enumerate(z0s):
        sim.init_generate(i, z0)
    sim.start()
    sim.step(STEPS)
    xtol, etol = (1e-9, 1e-10) if precision == "fp64" else (1e-4, 1e-4)
    for i, (c, w, z0) in enumerate(zip(clusters, weights, z0s)):
        r0 = units.nm_to_norm(c.r0_nm, 0.8)
        delta = units.nm_to_norm(c.electron_offset_nm, 0.8)
        xo, Zo = oracle.init_cluster(run.seed, i, c.n_ion, z0, r0, delta)
        osim = oracle.Sim(oracle.make_params(c, run, cluster_index=i, weight=w), c.capacity, xo, np.zeros_like(xo),
                          Zo)
        osim.start()
        ro = osim.run(STEPS)
        g = sim.particles(i)
        rg = sim.diagnostics(i)
        cnt = sim.counters(i)
        assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges()), i
        assert rg.shape == ro.shape and np.array_equal(rg[:, 21], ro[:, 21]), i
        assert np.array_equal(rg[:, 24:41], ro[:, 24:41]), i
        assert cnt["steps"] == STEPS and cnt["events"] == osim.N - len(Zo), (i, cnt)
        dx = np.max(np.abs(g["x"] - osim.positions())) / r0 if osim.N else 0.0
        print(f"  cluster {i}: w {w}, N {len(Zo)} -> {osim.N}, events {cnt['events']}, dx {dx:.2e}", flush=True)
        assert dx <= xtol, (i, dx)
        for col in [5, 6, 7, 8, 9, 10]:
            sc = np.max(np.abs(ro[:, col]))
            err = np.max(np.abs(rg[:, col] - ro[:, col]))
            assert err <= etol * sc, (i, col, err, sc)
    sim.close()


def test_cases_cover_the_edges():
    """The seeded cases include both precisions, pair-once and one-sided passes, periodic
    boundaries, circular polarization and every edge ion count."""
    cases = [_case(k) for k in range(24)]
    assert {p for p, *_ in cases} == {"fp64", "fp32_acc64"}
    assert any(t.get("newton3") for _, t, *_ in cases) and any(not t.get("newton3") for _, t, *_ in cases)
    assert any(r.boundary == "periodic" for _, _, r, *_ in cases)
    assert any(r.ofi_field == "local" for _, _, r, *_ in cases) and any(r.collisional for _, _, r, *_ in cases)
    cl = [c for *_, cs, _, _ in cases for c in cs]
    assert any(c.laser.polarization == "circular" for c in cl)
    assert {c.n_ion for c in cl} >= set(EDGE_IONS), sorted({c.n_ion for c in cl} & set(EDGE_IONS))
