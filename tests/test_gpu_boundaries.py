"""GPU parity of the periodic and mixed boundaries (Sec. II: periodic cube around the cluster,
minimum image, re-entry through the opposite face; mixed = periodic before t_switch) against
the oracle.

The cube is made tight (1.6 R0, smaller than the cluster: the particles beyond its faces are
wrapped by the first push, and pairs more than 0.8 R0 apart interact through a periodic copy)
so that every part of the boundary handling acts within 200 steps.

Tolerances (fixed before measuring):
  FP64 runs: as for open boundaries, max |dx| / R0 <= 1e-9, max |du| <= 1e-9 max |u|, KE, PE,
        W_L, W_C within 1e-10 relative.
  FP32 pairs: the FP32 kernels take separations from positions on the cube's 32-bit grid
        (each coordinate moved by at most L 2^-33, the wrapped integer difference is the minimum
        image).  A single field pass on a fixed wrapped state is compared with the plain FP64
        minimum-image oracle on the same FP64 positions, away from half-box ties:
        |dE_i| <= 64 u S1_i + 4 (L 2^-32) S2_i, S2_i = sum_j |q_j| / (r_ij^2 + eps^2)^{3/2}
        (kernel arithmetic as for open boundaries, plus the quantization: a separation moves by
        at most sqrt(3) L 2^-32 and the pair term's derivative is below 2 / (r^2 + eps^2)^{3/2}).
        FP32 runs are not compared orbit by orbit: once FP32 force
        rounding has moved the positions (1e-5 R0), pairs near half the box are decided from
        different positions on the two sides, and the minimum-image force jumps there; they
        are checked for staying in the cube and for the exact discrete energy identity
        instead.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import units
from workloads import small_ar

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

U32 = 2.0**-24


def _oracle(c, run, state):
    sim = oracle.Sim.from_workload(c, run, state)
    sim.start()
    return sim


def _sums(x, q, eps2, L=None):
    """S1_i = sum_j |q_j| r_ij / (r_ij^2+eps^2)^{3/2}, S2_i = sum_j |q_j| / (r_ij^2+eps^2)^{3/2} and
    S3_i = sum_j |q_j| (|r_i|_inf + |r_j|_inf) / (r_ij^2+eps^2)^{3/2} (minimum image if L is given)."""
    d = x[:, None, :] - x[None, :, :]
    if L is not None:
        d -= L * np.rint(d / L)
    r2 = np.sum(d * d, axis=2)
    den = (r2 + eps2) ** 1.5
    a = np.abs(q)[None, :] / den
    np.fill_diagonal(a, 0.0)
    m = np.max(np.abs(x), axis=1)
    return np.sum(a * np.sqrt(r2), axis=1), np.sum(a, axis=1), np.sum(a * (m[:, None] + m[None, :]), axis=1)


def _fp32_bound(x, q, eps2, L=None):
    """Per-target bound on |E_fp32 - E_oracle| with the oracle on the unrounded FP64 inputs: 64 u S1
    for the FP32 arithmetic; the rounding of the inputs adds 4 (L 2^-32) S2 for grid records of a
    periodic pass (L given), 4 u S3 for FP32 coordinates of an open one."""
    s1, s2, s3 = _sums(x, q, eps2, L)
    extra = 4.0 * L * 2.0**-32 * s2 if L is not None else 4.0 * U32 * s3
    return 64.0 * U32 * s1 + extra, s1


def _case(boundary):
    c, run = small_ar()
    run = dataclasses.replace(run, boundary=boundary, box_r0=1.6, t_switch=5.0)
    return c, run


@pytest.mark.parametrize("boundary", ["periodic", "mixed"])
@pytest.mark.parametrize("tiling", [None, dict(R=4, WJ=4, newton3=1), dict(R=2, WJ=1, S=4)])
def test_boundaries_fp64_match_oracle(boundary, tiling):
    import paper_1307_3711_amd as lc
    c, run = _case(boundary)
    mpb = lc.pair_blocks_for([c.capacity]) if tiling and tiling.get("newton3") else 0
    sim, states = gpu_run([c], run, "fp64", tuning=tiling, max_pair_blocks=mpb)
    osim = _oracle(c, run, states[0])
    print(f"{boundary} fp64 {tiling}: 200 steps", flush=True)
    sim.step(200)
    rg = sim.diagnostics(0)
    ro = osim.run(200)
    r0n = units.nm_to_norm(c.r0_nm, 0.8)
    L = osim.p.box
    g = sim.particles(0)
    assert np.max(np.abs(states[0]["x_nm"])) * units.nm_to_norm(1.0, 0.8) > L / 2  # the first push wraps
    if boundary == "periodic":
        assert np.all(np.abs(g["x"]) <= L / 2)
    else:  # the switch to open boundaries changes the outcome
        other = _oracle(c, dataclasses.replace(run, boundary="periodic"), states[0])
        other.run(200)
        assert np.max(np.abs(other.positions() - osim.positions())) > 0.0
    assert g["n"] == osim.N and np.array_equal(g["Z"], osim.charges())
    dx = np.max(np.abs(g["x"] - osim.positions())) / r0n
    uo = osim.momenta()
    du = np.max(np.abs(g["u"] - uo)) / np.max(np.abs(uo))
    print(f"max|dx|/R0 = {dx:.3e}  max|du|/max|u| = {du:.3e}")
    assert dx <= 1e-9 and du <= 1e-9
    for col in [5, 6, 7, 8, 9, 10]:
        scale = np.max(np.abs(ro[:, col])) + 1e-300
        err = np.max(np.abs(rg[:, col] - ro[:, col])) / scale
        assert err <= 1e-10, f"record column {col}: {err:.3e}"
    sim.close()


@pytest.mark.parametrize("tiling", [None, dict(R=1, WJ=4, T=1024, S=8, scalar=1), dict(R=2, WJ=2, S=4),
                                    dict(R=4, WJ=4, newton3=1), dict(R=2, WJ=1, newton3=1)])
def test_periodic_field_fp32_matches_oracle(tiling):
    import paper_1307_3711_amd as lc
    c, run = _case("periodic")
    # a wrapped state with pairs at every separation up to half the box: 30 oracle steps
    from workloads import initial_state
    osim = _oracle(c, run, initial_state(c, run.seed))
    osim.run(30)
    kn = units.nm_to_norm(1.0, 0.8)
    state = {"x_nm": osim.positions() / kn, "u": osim.momenta(), "Z": osim.charges(), "n_ion": c.n_ion}
    mpb = lc.pair_blocks_for([c.capacity]) if tiling and tiling.get("newton3") else 0
    sim, _ = gpu_run([c], run, "fp32_acc64", states=[state], tuning=tiling, max_pair_blocks=mpb)
    g = sim.particles(0)
    Eg = sim.field(0)
    sim.close()
    x = g["x"]
    L = osim.p.box
    q = osim.p.kappa * osim.p.weight * g["Z"].astype(np.float64)
    Eo, _ = oracle.coulomb_field(x, q, osim.p.eps2, want_phi=False, box=L)
    d = x[:, None, :] - x[None, :, :]
    # no pair within 4 grid steps of half the box, where the grid could pick the other copy
    tie = np.abs(np.abs(d) - L / 2) / (L * 2.0**-32)
    assert tie.min() > 4
    bound, s1 = _fp32_bound(x, q, osim.p.eps2, L)
    err = np.max(np.abs(Eg - Eo) / s1[:, None])
    ratio = np.max(np.abs(Eg - Eo) / bound[:, None])
    print(f"fp32 periodic field {tiling}: max |dE| / S1 = {err / U32:.1f} u, {ratio:.3f} of the bound", flush=True)
    d -= L * np.rint(d / L)
    assert np.max(np.abs(x)) <= L / 2 and np.max(np.abs(d)) > 0.45 * L  # pairs reach half the box
    assert ratio <= 1.0


@pytest.mark.parametrize("boundary", ["periodic", "mixed"])
def test_boundaries_fp32_run_invariants(boundary):
    import paper_1307_3711_amd as lc
    c, run = _case(boundary)
    sim, _ = gpu_run([c], run, "fp32_acc64", tuning=dict(R=4, WJ=4, newton3=1),
                     max_pair_blocks=lc.pair_blocks_for([c.capacity]))
    sim.step(200)
    rec = sim.diagnostics(0)
    g = sim.particles(0)
    L = 1.6 * units.nm_to_norm(c.r0_nm, 0.8)
    if boundary == "periodic":
        assert np.all(np.abs(g["x"]) <= L / 2)
    assert np.sum(g["Z"].astype(np.int64)) == 0  # one electron per charge, spawns included
    ident = np.abs(rec[:, 5] - rec[:, 23] - (rec[:, 8] + rec[:, 9] + rec[:, 10]))
    scale = np.abs(rec[:, 8]) + np.abs(rec[:, 9]) + rec[:, 10] + np.abs(rec[:, 23])
    assert np.max(ident / scale) <= 1e-11
    sim.close()


def test_mixed_boundary_graph_replay_bitwise():
    """Captured groups of steps bake in the boundary mode: replays across the switch from
    periodic to open give bitwise the state of stepping one launch sequence at a time."""
    c, run = _case("mixed")
    out = []
    for graph in (0, 10):
        sim, _ = gpu_run([c], run, "fp64")
        if graph:
            sim.set_graph(graph)
        sim.step(200)
        g = sim.particles(0)
        out.append((g["x"].copy(), g["u"].copy(), g["Z"].copy(), sim.diagnostics(0).copy()))
        sim.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def _fp32_field_error(E, x, q, eps2, L=None):
    """max |E - E_oracle| / bound with the plain FP64 oracle on the unrounded positions (minimum
    image if L is given, away from half-box ties) and the bound of _fp32_bound."""
    Eo, _ = oracle.coulomb_field(x, q, eps2, want_phi=False, box=0.0 if L is None else L)
    if L is not None:
        d = x[:, None, :] - x[None, :, :]
        assert (np.abs(np.abs(d) - L / 2) / (L * 2.0**-32)).min() > 4
    bound, _ = _fp32_bound(x, q, eps2, L)
    return np.max(np.abs(E - Eo) / bound[:, None])


@pytest.mark.parametrize("tiling", [dict(R=4, WJ=4, newton3=1), dict(R=2, WJ=2, S=4),
                                    dict(R=1, WJ=4, T=1024, S=8, scalar=1)])
def test_mixed_fp32_records_across_the_switch(tiling):
    """FP32 source records change form at the switch (grid coordinates while periodic, plain
    coordinates afterwards; the push of a step writes them in the form of the next step's
    pass): the passes of the last periodic step (99, t = 4.95) and the first open one (100,
    t = 5) each against the oracle on the GPU's positions, within the bound of _fp32_bound."""
    import paper_1307_3711_amd as lc
    c, run = _case("mixed")
    mpb = lc.pair_blocks_for([c.capacity]) if tiling.get("newton3") else 0
    sim, states = gpu_run([c], run, "fp32_acc64", tuning=tiling, max_pair_blocks=mpb)
    op = _oracle(c, run, states[0]).p
    for steps, periodic in ((99, True), (1, False)):
        sim.step(steps)
        g = sim.particles(0)
        E = sim.field(0)
        q = op.kappa * op.weight * g["Z"].astype(np.float64)
        err = _fp32_field_error(E, g["x"], q, op.eps2, op.box if periodic else None)
        print(f"{tiling} step {99 if periodic else 100} ({'periodic' if periodic else 'open'}): "
              f"{err:.3f} of the bound", flush=True)
        assert err <= 1.0
    sim.close()


def test_half_box_tie_on_the_grid():
    """Two ions exactly half a box apart along x on the grid (2^30 grid steps either side of
    the centre).  The FP32 kernels take the wrapped difference of grid records, -2^31 grid steps
    whichever ion is the target, so each ion sees the other's copy on its +x side (r_i - r_j' =
    -L/2), in a single block (every pair evaluated from both ends) as in the pair-once kernel.
    The expected field of each ion is the FP64 oracle's with the other ion moved by 1e-6 L to the
    side that makes that copy the nearest; the two electrons (no tie) take the plain oracle."""
    import paper_1307_3711_amd as lc
    from workloads import Cluster, Laser, Run
    c = Cluster(species="Ar", r0_nm=2.5, n_ion=2, capacity=4, z_init=1, z_max=1,
                laser=Laser(intensity_wcm2=0.0, envelope="flat"), n_steps=10)
    run = Run(dt=0.05, ionize=False, boundary="periodic", box_r0=4.0, diag_every=0)
    kn = units.nm_to_norm(1.0, 0.8)
    L = run.box_r0 * units.nm_to_norm(c.r0_nm, 0.8)
    xg = 2.0**30 * (L / 2.0**32)  # on the grid
    x = np.array([[xg, 0, 0], [-xg, 0, 0], [0, 0.31 * L, 0], [0.1 * L, -0.2 * L, 0.1 * L]]) / kn
    state = {"x_nm": x, "u": np.zeros_like(x), "Z": np.array([1, 1, -1, -1], np.int8), "n_ion": 2}
    for tiling in (dict(R=4, WJ=4, newton3=1), dict(R=2, WJ=2, S=2)):
        mpb = lc.pair_blocks_for([c.capacity]) if tiling.get("newton3") else 0
        sim, _ = gpu_run([c], run, "fp32_acc64", states=[state], tuning=tiling, max_pair_blocks=mpb)
        g = sim.particles(0)
        E = sim.field(0)
        sim.close()
        op = _oracle(c, run, state).p
        q = op.kappa * op.weight * g["Z"].astype(np.float64)
        near = {}
        for side, dx in (("-L/2", -1e-6), ("+L/2", 1e-6)):
            xs = g["x"].copy()
            xs[1, 0] += dx * op.box  # ion 0 minus ion 1: just over or just under half the box
            near[side], _ = oracle.coulomb_field(xs, q, op.eps2, want_phi=False, box=op.box)
        scale = np.max(np.abs(near["-L/2"]))
        # ion 0 sees ion 1's copy at x0 + L/2, as when ion 0 - ion 1 is just over L/2 (first
        # nudge); ion 1 sees ion 0's copy at x1 + L/2, as when it is just under (second nudge)
        for ion, same, other in ((0, "-L/2", "+L/2"), (1, "+L/2", "-L/2")):
            assert np.max(np.abs(E[ion] - near[same][ion])) <= 1e-4 * scale, (tiling, ion)
            assert np.max(np.abs(E[ion] - near[other][ion])) > 1e-2 * scale
        Eo, _ = oracle.coulomb_field(g["x"], q, op.eps2, want_phi=False, box=op.box)
        d = g["x"][2:, None, :] - g["x"][None, :, :]
        assert (np.abs(np.abs(d) - op.box / 2) / (op.box * 2.0**-32)).min() > 4  # electrons: no tie
        bound, _ = _fp32_bound(g["x"], q, op.eps2, op.box)
        assert np.all(np.abs(E[2:] - Eo[2:]) <= bound[2:, None]), (tiling, E, Eo)
