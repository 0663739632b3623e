"""GPU parity of the periodic and mixed boundaries (Sec. II: periodic cube around the cluster,
minimum image, re-entry through the opposite face; mixed = periodic before t_switch) against
the oracle.

The cube is made tight (1.6 R0, smaller than the cluster: the particles beyond its faces are
wrapped by the first push, and pairs more than 0.8 R0 apart interact through a periodic copy)
so that every part of the boundary handling acts within 200 steps.

Tolerances (fixed before measuring):
  FP64 runs: as for open boundaries, max |dx| / R0 <= 1e-9, max |du| <= 1e-9 max |u|, KE, PE,
        W_L, W_C within 1e-10 relative.
  FP32 pairs: which periodic copy is nearest is an integer decided by floating point, and the
        FP32 kernels decide it from FP32 positions.  A single field pass on a fixed wrapped
        state is compared with the oracle taking the same decision (image32) on the kernel's
        FP32 operands: |dE| <= 64 u S1_i as for open boundaries.  FP32 runs are not compared
        orbit by orbit: once FP32 force rounding has moved the positions (1e-5 R0), pairs
        near half the box are decided from different positions on the two sides, and the
        minimum-image force jumps there; they are checked for staying in the cube and for the
        exact discrete energy identity instead.
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


def _oracle(c, run, state, image32=False):
    sim = oracle.Sim.from_workload(c, run, state)
    sim.p.image32 = 1 if image32 else 0
    sim.start()
    return sim


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
    xr = x.astype(np.float32).astype(np.float64)
    qr = q.astype(np.float32).astype(np.float64)
    eps2 = float(np.float32(osim.p.eps2))
    Eo, _ = oracle.coulomb_field(xr, qr, eps2, want_phi=False, box=float(np.float32(L)), image32=True)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.rint(d / L)
    r2 = np.sum(d * d, axis=2)
    t = np.abs(q)[None, :] * np.sqrt(r2) / (r2 + osim.p.eps2) ** 1.5
    np.fill_diagonal(t, 0.0)
    s1 = t.sum(axis=1)
    err = np.max(np.abs(Eg - Eo) / s1[:, None])
    print(f"fp32 periodic field {tiling}: max |dE| / S1 = {err:.3e} ({err / U32:.1f} u)", flush=True)
    assert np.max(np.abs(x)) <= L / 2 and np.max(np.abs(d)) > 0.45 * L  # pairs reach half the box
    assert err <= 64 * U32


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
