"""GPU parity of the Coulomb direct sum (lc_field) against the FP64 oracle.

Element by element on seeded cluster states spanning several LDS tiles, target blocks and a
ragged tail, for every precision and a range of tilings; then sampled targets of the full
20k-macroparticle argon state in the tiling the benchmark uses, and of a cluster of a million
macroparticles (pair-once rows beyond 32-bit offsets).

Tolerances (fixed before measuring):
  FP64: per target |dE| <= 1e-12 * S1_i and |dphi| <= 1e-12 * S0_i, where
        S1_i = sum_j |q_j| |r_ij| / (r_ij^2 + eps^2)^{3/2} and S0_i = sum_j |q_j| / (r_ij^2+eps^2)^{1/2}
        bound the magnitudes of the summed terms (rounding of a sum is relative to them);
  FP32 (+FP64 accumulation): compared with the oracle evaluated on the FP32-rounded inputs
        (the kernel's actual operands): |dE| <= 64 u S1_i with u = 2^-24 (per-term rounding of a
        few ulp plus FP32 summation within one LDS tile, which grows like sqrt(T) u);
  FP32 Kahan: |dE| <= 16 u S1_i.
  FP32 path against the oracle on the unrounded FP64 inputs (the field error a user of the FP32
        path sees): |dE_i| <= 64 u S1_i + 4 u S3_i, S3_i = sum_j |q_j| (|r_i|_inf + |r_j|_inf) /
        (r_ij^2 + eps^2)^{3/2} (rounding a coordinate to FP32 moves a separation by at most
        sqrt(3) u (|r_i|_inf + |r_j|_inf), the pair term's derivative is below 2 / (r^2+eps^2)^{3/2});
        the 99.9th percentile of the per-particle relative error |dE_i| / |E_i| <= 1e-3; the
        normwise error at most twice that of the oracle itself on the FP32-rounded inputs, which
        no kernel storing FP32 coordinates can go below (7.5e-6 on the small argon state,
        2.1e-5 on the 20k state).
"""
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, ar_20k, initial_state

from _helpers import gpu_available

pytestmark = pytest.mark.gpu

U32 = 2.0**-24


def _state(n, seed, r0=2.5):
    n_ion = max(1, n // 2)
    c = Cluster(species="Ar", r0_nm=r0, n_ion=n_ion, capacity=2 * n_ion, z_init=1)
    st = initial_state(c, seed)
    x = units.nm_to_norm(st["x_nm"], 0.8)[:n]
    Z = st["Z"][:n].astype(np.float64)
    w = units.n_atoms(r0, 2.4) / n_ion
    q = units.kappa(0.8) * w * Z
    # a few higher charge states, as after ionization
    q[: n_ion: 7] *= 3.0
    return x, q


def _scales(x, q, eps2, idx=None):
    idx = np.arange(x.shape[0]) if idx is None else idx
    s1 = np.zeros(len(idx))
    s0 = np.zeros(len(idx))
    for k, i in enumerate(idx):
        d = x[i] - x
        r2 = np.sum(d * d, axis=1) + eps2
        r = np.sqrt(r2 - eps2)
        m = np.ones(x.shape[0], bool)
        m[i] = False
        s1[k] = np.sum(np.abs(q[m]) * r[m] / r2[m] ** 1.5)
        s0[k] = np.sum(np.abs(q[m]) / np.sqrt(r2[m]))
    return s1, s0


def _gpu_field(x, q, eps2, precision, tuning=None, phi=True):
    import torch
    import paper_1307_3711_amd as lc
    xyzq = torch.tensor(np.concatenate([x.T, q[None, :]], axis=0), dtype=torch.float64, device="cuda")
    t = lc.make_tuning(**tuning) if tuning else None
    E, P = lc.field(xyzq, eps2, precision=precision, want_phi=phi, tuning=t)
    torch.cuda.synchronize()
    return E.cpu().numpy().T, (P.cpu().numpy() if phi else None)


EPS2 = units.nm_to_norm(0.1, 0.8) ** 2

TILINGS = [
    {},
    dict(R=1, WJ=1, T=64, S=1),
    dict(R=2, WJ=2, T=256, S=3),
    dict(R=4, WJ=4, T=512, S=2),
    dict(R=1, WJ=4, T=128, S=5, persistent=1),
    dict(R=2, WJ=1, T=1920, S=1, persistent=1),
    dict(R=1, WJ=4, T=1024, S=7, scalar=1),
    dict(R=2, WJ=2, T=256, S=3, persistent=1, scalar=1),
]


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("n", [1, 2, 3, 65, 257, 1000, 2053])
@pytest.mark.parametrize("ti", [0, 1, 2, 3, 4, 5])
def test_field_fp64_elementwise(n, ti):
    x, q = _state(n, n + 17)
    Eo, Po = oracle.coulomb_field(x, q, EPS2)
    Eg, Pg = _gpu_field(x, q, EPS2, "fp64", TILINGS[ti])
    s1, s0 = _scales(x, q, EPS2)
    print(f"fp64 n={n} tiling={TILINGS[ti]} maxrel={np.max(np.abs(Eg - Eo) / s1[:, None]):.3e}", flush=True)
    assert np.all(np.abs(Eg - Eo) <= 1e-12 * s1[:, None] + 1e-300)
    assert np.all(np.abs(Pg - Po) <= 1e-12 * s0 + 1e-300)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("precision,factor", [("fp32_acc64", 64.0), ("fp32_kahan", 16.0)])
@pytest.mark.parametrize("n", [2, 63, 1000, 2053])
@pytest.mark.parametrize("ti", [0, 1, 2, 3, 4, 6, 7])
def test_field_fp32_elementwise(precision, factor, n, ti):
    if precision == "fp32_kahan" and TILINGS[ti].get("R", 4) == 8:
        pytest.skip("no R=8 Kahan variant")
    x, q = _state(n, 3 * n + 1)
    xr = x.astype(np.float32).astype(np.float64)
    qr = q.astype(np.float32).astype(np.float64)
    Eo, Po = oracle.coulomb_field(xr, qr, float(np.float32(EPS2)))
    Eg, Pg = _gpu_field(x, q, EPS2, precision, TILINGS[ti])
    s1, s0 = _scales(xr, qr, EPS2)
    print(f"{precision} n={n} tiling={TILINGS[ti]} maxrel={np.max(np.abs(Eg - Eo) / s1[:, None]):.3e}", flush=True)
    assert np.all(np.abs(Eg - Eo) <= factor * U32 * s1[:, None] + 1e-300)
    assert np.all(np.abs(Pg - Po) <= factor * U32 * s0 + 1e-300)


N3_TILINGS = [
    dict(R=1, WJ=1, newton3=1),
    dict(R=2, WJ=1, newton3=1),
    dict(R=1, WJ=2, newton3=1),
    dict(R=2, WJ=2, newton3=1, persistent=1),
    dict(R=4, WJ=2, newton3=1),
    dict(R=4, WJ=4, newton3=1),
    dict(R=4, WJ=4, newton3=1, persistent=1),
    dict(R=3, WJ=3, newton3=1),
    dict(R=5, WJ=5, newton3=1),
    dict(R=6, WJ=6, newton3=1, persistent=1),
]


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("n", [1, 2, 63, 129, 1000, 2053])
@pytest.mark.parametrize("ti", range(len(N3_TILINGS)))
def test_field_pair_once_elementwise(n, ti):
    """Each unordered pair evaluated once and applied to both particles: same tolerance as the
    one-sided FP32 kernel (64 u S1 against the oracle on the FP32-rounded inputs).  The state
    has non-uniform ion charges and uniform electrons, so blocks and chunks of every charge
    pattern occur, and n spans one block, several blocks and ragged tails."""
    x, q = _state(n, 5 * n + 3)
    xr = x.astype(np.float32).astype(np.float64)
    qr = q.astype(np.float32).astype(np.float64)
    Eo, _ = oracle.coulomb_field(xr, qr, float(np.float32(EPS2)))
    Eg, _ = _gpu_field(x, q, EPS2, "fp32_acc64", N3_TILINGS[ti], phi=False)
    s1, _ = _scales(xr, qr, EPS2)
    print(f"pair-once n={n} tiling={N3_TILINGS[ti]} maxrel={np.max(np.abs(Eg - Eo) / s1[:, None]):.3e}", flush=True)
    assert np.all(np.abs(Eg - Eo) <= 64.0 * U32 * s1[:, None] + 1e-300)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("n", [1, 2, 63, 129, 1000, 2053])
@pytest.mark.parametrize("ti", [0, 2, 3, 5, 7, 8])
def test_field_pair_once_fp64_elementwise(n, ti):
    """FP64 pair-once kernel: each pair once in FP64, FP64 rows: same tolerance as the FP64
    one-sided kernel (1e-12 S1)."""
    x, q = _state(n, 7 * n + 5)
    Eo, _ = oracle.coulomb_field(x, q, EPS2)
    Eg, _ = _gpu_field(x, q, EPS2, "fp64", N3_TILINGS[ti], phi=False)
    s1, _ = _scales(x, q, EPS2)
    print(f"pair-once fp64 n={n} tiling={N3_TILINGS[ti]} maxrel={np.max(np.abs(Eg - Eo) / s1[:, None]):.3e}",
          flush=True)
    assert np.all(np.abs(Eg - Eo) <= 1e-12 * s1[:, None] + 1e-300)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_field_pair_once_rejects_potential():
    import torch
    import paper_1307_3711_amd as lc
    xyzq = torch.zeros((4, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(lc.LcError):
        lc.field(xyzq, EPS2, precision="fp32_acc64", want_phi=True, tuning=lc.make_tuning(R=4, WJ=4, newton3=1))
    with pytest.raises(lc.LcError):
        lc.field(xyzq, EPS2, precision="fp32_kahan", want_phi=False, tuning=lc.make_tuning(R=4, WJ=4, newton3=1))


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_field_empty_input():
    import torch
    import paper_1307_3711_amd as lc
    xyzq = torch.zeros((4, 0), dtype=torch.float64, device="cuda")
    E, P = lc.field(xyzq, EPS2)
    assert E.shape == (3, 0) and P.shape == (0,)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_field_rejects_bad_arguments():
    import torch
    import paper_1307_3711_amd as lc
    xyzq = torch.zeros((4, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(lc.LcError):
        lc.field(xyzq, 0.0)
    with pytest.raises(lc.LcError):
        lc.field(xyzq, EPS2, tuning=lc.make_tuning(R=3))


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("precision,tiling", [("fp64", dict(S=16)), ("fp32_acc64", dict(S=16)),
                                              ("fp32_acc64", dict(R=1, WJ=4, T=1024, S=16, scalar=1)),
                                              ("fp32_acc64", dict(R=4, WJ=4, newton3=1)),
                                              ("fp32_acc64", dict(R=5, WJ=5, newton3=1)),
                                              ("fp64", dict(R=2, WJ=2, newton3=1)),
                                              ("fp32_acc64", dict(R=2, WJ=2, newton3=1, persistent=1))])
def test_field_full_20k_sampled(precision, tiling):
    """The 20k-macroparticle argon state at full size (the benchmark's workload, including the
    scalar-source tiling the autotuner picks for it): sampled targets against the oracle
    evaluated target by target."""
    c, run = ar_20k()
    st = initial_state(c, run.seed)
    x = units.nm_to_norm(st["x_nm"], 0.8)
    w = units.n_atoms(c.r0_nm, 2.4) / c.n_ion
    q = units.kappa(0.8) * w * st["Z"].astype(np.float64)
    idx = np.unique(np.concatenate([np.arange(0, x.shape[0], 997), [0, 9999, 10000, x.shape[0] - 1]]))
    phi = not tiling.get("newton3", 0)
    Eg, Pg = _gpu_field(x, q, EPS2, precision, tiling, phi=phi)
    if precision == "fp64":
        Eo, Po = oracle.coulomb_field_at(x, q, EPS2, idx)
        tol = 1e-12
    else:
        xr = x.astype(np.float32).astype(np.float64)
        qr = q.astype(np.float32).astype(np.float64)
        Eo, Po = oracle.coulomb_field_at(xr, qr, float(np.float32(EPS2)), idx)
        tol = 64 * U32
    s1, s0 = _scales(x, q, EPS2, idx)
    assert np.all(np.abs(Eg[idx] - Eo) <= tol * s1[:, None])
    if phi:
        assert np.all(np.abs(Pg[idx] - Po) <= tol * s0)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("precision,tiling", [("fp32_acc64", None), ("fp32_acc64", dict(R=4, WJ=4, newton3=1)),
                                              ("fp32_acc64", dict(R=4, WJ=4, S=64, persistent=1)),
                                              ("fp64", dict(S=16)), ("fp64", dict(R=4, WJ=4, newton3=1))])
def test_field_one_million_sampled(precision, tiling):
    """One cluster of a million macroparticles (500k Ar+ + 500k e-, R0 = 30 nm, the density of
    the 20k state): 3907 blocks of 256 targets, 7.6M pair-once tiles whose rows (47 GB in FP32,
    94 GB in FP64) sit far beyond 32-bit element offsets.  Sampled targets (first and last
    slots, both sides of block and ion/electron boundaries) against the oracle target by
    target, at the bars of the 20k test."""
    n_ion = 500_000
    c = Cluster(species="Ar", r0_nm=30.0, n_ion=n_ion, capacity=2 * n_ion, z_init=1)
    st = initial_state(c, 3)
    x = units.nm_to_norm(st["x_nm"], 0.8)
    q = units.kappa(0.8) * (units.n_atoms(30.0, 2.4) / n_ion) * st["Z"].astype(np.float64)
    n = x.shape[0]
    idx = np.array([0, 1, 255, 256, 257, 65535, 65536, 262143, 262144, n_ion - 1, n_ion, n_ion + 1, 777_777,
                    n - 257, n - 256, n - 2, n - 1])
    print(f"{precision} {tiling}: n={n}", flush=True)
    Eg, _ = _gpu_field(x, q, EPS2, precision, tiling, phi=False)
    import torch
    torch.cuda.empty_cache()  # hand the workspace back before the next case
    if precision == "fp64":
        Eo, _ = oracle.coulomb_field_at(x, q, EPS2, idx, want_phi=False)
        tol = 1e-12
    else:
        xr = x.astype(np.float32).astype(np.float64)
        qr = q.astype(np.float32).astype(np.float64)
        Eo, _ = oracle.coulomb_field_at(xr, qr, float(np.float32(EPS2)), idx, want_phi=False)
        tol = 64 * U32
    s1, _ = _scales(x, q, EPS2, idx)
    err = np.max(np.abs(Eg[idx] - Eo) / s1[:, None])
    print(f"max error / S1 = {err:.2e}", flush=True)
    assert err <= tol
    assert np.all(np.isfinite(Eg))


def _s3(x, q, eps2, idx):
    m = np.max(np.abs(x), axis=1)
    out = np.zeros(len(idx))
    for k, i in enumerate(idx):
        d = x[i] - x
        r2 = np.sum(d * d, axis=1)
        t = np.abs(q) * (m[i] + m) / (r2 + eps2) ** 1.5
        t[i] = 0.0
        out[k] = np.sum(t)
    return out


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("workload", ["small_ar", "ar_20k"])
@pytest.mark.parametrize("tiling", [None, dict(R=4, WJ=4, newton3=1), dict(R=1, WJ=4, T=1024, S=16, scalar=1)])
def test_field_fp32_path_against_unrounded_oracle(workload, tiling):
    """The FP32 path's own field error: the GPU in FP32 pairs on the FP64 state against the FP64
    oracle on the same unrounded state (the small argon state in full, sampled targets of the 20k
    state), element by element within the derived bound, the 99.9th percentile of the relative
    error, and normwise against the floor that rounding the inputs to FP32 alone sets."""
    from workloads import small_ar
    c, run = small_ar() if workload == "small_ar" else ar_20k()
    st = initial_state(c, run.seed)
    x = units.nm_to_norm(st["x_nm"], 0.8)
    w = units.n_atoms(c.r0_nm, 2.4) / c.n_ion
    q = units.kappa(0.8) * w * st["Z"].astype(np.float64)
    n = x.shape[0]
    idx = np.arange(n) if n <= 2000 else np.unique(np.concatenate([np.arange(0, n, 331), [0, n // 2, n - 1]]))
    Eg, _ = _gpu_field(x, q, EPS2, "fp32_acc64", tiling, phi=False)
    Eo, _ = oracle.coulomb_field_at(x, q, EPS2, idx, want_phi=False)
    r32 = lambda v: v.astype(np.float32).astype(np.float64)
    Ef, _ = oracle.coulomb_field_at(r32(x), r32(q), float(np.float32(EPS2)), idx, want_phi=False)
    s1, _ = _scales(x, q, EPS2, idx)
    bound = 64 * U32 * s1 + 4 * U32 * _s3(x, q, EPS2, idx)
    d = Eg[idx] - Eo
    rel = np.linalg.norm(d, axis=1) / np.linalg.norm(Eo, axis=1)
    nw = np.linalg.norm(d) / np.linalg.norm(Eo)
    floor = np.linalg.norm(Ef - Eo) / np.linalg.norm(Eo)
    print(f"fp32 path {workload} {tiling}: normwise {nw:.3e} (floor {floor:.3e}), p99.9 {np.percentile(rel, 99.9):.3e}, "
          f"max {np.max(np.abs(d) / bound[:, None]):.3f} of the bound", flush=True)
    assert np.all(np.abs(d) <= bound[:, None])
    assert np.percentile(rel, 99.9) <= 1e-3
    assert nw <= 2.0 * floor
