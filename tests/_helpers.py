"""Test helpers: build matching GPU and oracle runs from one workload description."""
import numpy as np

import oracle
from oracle import units
from workloads import initial_state
from workloads.species import SPECIES


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def descs(clusters, weight=None):
    import paper_1307_3711_amd as lc
    out = []
    for c in clusters:
        out.append(lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                                   envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, n_cycles=c.laser.n_cycles,
                                   phase=c.laser.phase, weight=0.0 if weight is None else weight, z_max=c.z_max,
                                   electron_offset_nm=c.electron_offset_nm, n_steps=0,
                                   polarization=c.laser.polarization))
    return out


def gpu_run(clusters, run, precision="fp64", states=None, max_records=4096, weight=None, n_steps_per_cluster=None,
            max_splits=32, tuning=None, max_pair_blocks=0):
    """Create, initialise and start a GPU simulation of the given clusters (a tuning is set
    before the start, so the start's field pass already uses it)."""
    import paper_1307_3711_amd as lc
    lam = clusters[0].laser.lambda_um
    cfg = lc.make_config(precision, ionize=run.ionize, ofi_field=run.ofi_field, lambda_um=lam, dt=run.dt, t0=run.t0,
                         softening_nm=run.softening_nm, diag_every=run.diag_every, max_records=max_records,
                         max_splits=max_splits, seed=run.seed, max_pair_blocks=max_pair_blocks,
                         boundary=run.boundary, box_r0=run.box_r0, t_switch=run.t_switch,
                         collisional=run.collisional)
    ds = descs(clusters, weight)
    if n_steps_per_cluster is not None:
        for d, n in zip(ds, n_steps_per_cluster):
            d.n_steps = int(n)
    sim = lc.Simulation(cfg, ds)
    if tuning is not None:
        sim.set_tuning(**tuning)
    if states is None:
        states = [initial_state(c, run.seed, i) for i, c in enumerate(clusters)]
    for i, st in enumerate(states):
        sim.init_from_host(i, st["x_nm"], st["u"], st["Z"])
    sim.start()
    return sim, states


def oracle_run(cluster, run, state, cluster_index=0, weight=None):
    kw = {} if weight is None else {"weight": weight}
    sim = oracle.Sim.from_workload(cluster, run, state, cluster_index, **kw)
    sim.start()
    return sim


def field_scale(x, q, eps2):
    """S1_i = sum_{j != i} |q_j| |r_ij| / (r_ij^2 + eps^2)^{3/2}: the magnitude of the terms a
    field sum adds, against which its rounding is measured."""
    s1 = np.zeros(x.shape[0])
    for i in range(x.shape[0]):
        d = x[i] - x
        r2 = np.sum(d * d, axis=1)
        t = np.abs(q) * np.sqrt(r2) / (r2 + eps2) ** 1.5
        t[i] = 0.0
        s1[i] = np.sum(t)
    return s1


def norm_positions(state, lam=0.8):
    return units.nm_to_norm(np.asarray(state["x_nm"], np.float64), lam)


def oracle_spread(cluster, run, state, cluster_index, nsteps, cols=(5, 6, 7, 8, 9)):
    """Reference run plus rounding-level perturbed runs of the oracle (softening squared one
    ulp up and down, electrons reordered so every field sum is added in another order).

    The model is chaotic: electrons bound inside the softening core of their ion are only
    marginally resolved at dt = 0.05, so rounding differences grow by orders of magnitude
    within tens of steps.  The spread of these perturbed runs measures how far two correct
    FP64 implementations that round differently can drift apart.  Returns the reference
    Sim, its records, and the largest perturbed deviation in positions (relative to R0),
    momenta (relative to max |u|) and each record column (relative to its scale)."""
    r0n = units.nm_to_norm(cluster.r0_nm, cluster.laser.lambda_um)
    ref = oracle_run(cluster, run, state, cluster_index)
    rref = ref.run(nsteps)
    out = {"dx": 0.0, "du": 0.0, "cols": {c: 0.0 for c in cols}, "same_events": True}
    n = state["x_nm"].shape[0]
    ni = cluster.n_ion
    rng = np.random.default_rng(1234)
    perm = np.concatenate([np.arange(ni), ni + rng.permutation(n - ni)])
    variants = []
    for sgn in (1.0, -1.0):
        v = oracle.Sim.from_workload(cluster, run, state, cluster_index)
        v.p.eps2 = float(np.nextafter(v.p.eps2, sgn * np.inf))
        variants.append((v, None))
    st2 = {"x_nm": state["x_nm"][perm], "u": state["u"][perm], "Z": state["Z"][perm], "n_ion": ni}
    variants.append((oracle.Sim.from_workload(cluster, run, st2, cluster_index), perm))
    uscale = None
    for v, pm in variants:
        v.start()
        rv = v.run(nsteps)
        if v.N != ref.N or (pm is None and not np.array_equal(v.charges(), ref.charges())):
            out["same_events"] = False
            continue
        xv, uv = v.positions(), v.momenta()
        if pm is not None:
            if v.N != n:
                continue  # spawned electrons are ordered differently; positions not comparable
            inv = np.argsort(pm)
            xv, uv = xv[inv], uv[inv]
        uscale = max(np.max(np.abs(ref.momenta())), 1e-300)
        out["dx"] = max(out["dx"], float(np.max(np.abs(xv - ref.positions())) / r0n))
        out["du"] = max(out["du"], float(np.max(np.abs(uv - ref.momenta())) / uscale))
        for c in cols:
            sc = np.max(np.abs(rref[:, c])) + 1e-300
            out["cols"][c] = max(out["cols"][c], float(np.max(np.abs(rv[:, c] - rref[:, c])) / sc))
    return ref, rref, out
