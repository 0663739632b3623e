"""Ensembles of clusters in one launch sequence, and the surrogate's features and targets.

A run of many uneven clusters is one Simulation: every step enumerates the tiles of all live
clusters in one Coulomb-kernel launch, finished clusters retire on the device, and steps are
replayed from a captured hipGraph.  The surrogate maps the cluster and laser parameters of a
run to two outcomes of it (absorbed laser energy per atom and mean ion charge at the end).
"""
import time

import numpy as np
import torch

from ._binding import R_ABS_EV, R_MEANZ, Simulation, make_config, pair_blocks_for


def run_ensemble(descs, states, precision="fp32_acc64", dt=0.05, softening_nm=0.1, seed=0, diag_every=50,
                 graph_steps=50, autotune=True, max_steps=None, tiling=None, progress=None, lambda_um=0.8,
                 keep_particles=False, adapt=True, probe_steps=100):
    """Integrate every cluster until it retires.  descs: lc_cluster descriptions with n_steps
    set; states: initial particle arrays (x_nm, u, Z) per cluster.  Returns a dict with the
    last diagnostic record of each cluster, per-cluster counters and the timed wall clock (and
    each cluster's final particles with keep_particles).

    With autotune the tiling is chosen at the start.  Ionization grows the clusters from their
    initial counts towards capacity, which favours the pair-once pass (its row fold costs less
    against a larger pair count), so a run that starts on the one-sided pass checks, with
    adapt, whether the pair-once pass (R = WJ = 4, persistent) has become faster: a chunk of
    steps opens with two timed stretches of probe_steps real steps, one on each pass, and
    keeps the faster; after a loss the next check waits twice as many chunks (up to 8), after
    a win there are no more checks.  The probes advance the run like any other steps, so a
    check costs two synchronizations and a graph capture.  The choice follows measured times,
    so FP32 results of two runs may differ at rounding level where they chose differently."""
    # room for the pair-once kernel (blocks of 128 slots and up) where the precision allows it
    mpb = pair_blocks_for([d.capacity for d in descs], 128) if precision in ("fp32_acc64", "fp64") else 0
    cfg = make_config(precision, ionize=True, lambda_um=lambda_um, dt=dt, softening_nm=softening_nm,
                      diag_every=diag_every, max_records=4, max_splits=8, seed=seed, max_pair_blocks=mpb)
    sim = Simulation(cfg, descs)
    for i, st in enumerate(states):
        sim.init_from_host(i, st["x_nm"], st["u"], st["Z"])
    sim.start()
    tuned = None
    if tiling:
        sim.set_tuning(**tiling)
    elif autotune:
        tuned = sim.autotune()
    if graph_steps:
        sim.set_graph(graph_steps)
    total = max(int(d.n_steps) for d in descs)
    if max_steps is not None:
        total = min(total, int(max_steps))
    sim.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = max(graph_steps or 1, 1) * 20
    done = 0
    tunings = [dict(tuned, at_step=0)] if tuned else []
    other = None
    if adapt and tuned and mpb and not tuned["newton3"]:
        other = dict(R=4, WJ=4, newton3=1, persistent=1)
    wait, interval = 0, 1

    def timed(n):
        sim.stream.synchronize()
        t = time.perf_counter()
        sim.step(n)
        sim.stream.synchronize()
        return time.perf_counter() - t

    warm = max(graph_steps or 1, 1)  # the steps that capture a new graph stay out of the timing
    while done < total:
        k = min(chunk, total - done)
        if other is not None and wait > 0:
            wait -= 1
            sim.step(k)
        elif other is not None and k >= 2 * (probe_steps + warm):
            cur = sim.tuning()
            t_cur = timed(probe_steps)
            sim.set_tuning(**other)
            if graph_steps:
                sim.set_graph(graph_steps)
            sim.step(warm)
            t_other = timed(probe_steps)
            if t_other < t_cur:
                tunings.append(dict(sim.tuning(), at_step=done + probe_steps))
                other = None
            else:
                sim.set_tuning(**cur)
                if graph_steps:
                    sim.set_graph(graph_steps)
                interval = min(2 * interval, 8)
                wait = interval - 1
            sim.step(k - 2 * probe_steps - warm)
        else:
            sim.step(k)
        done += k
        if progress:
            sim.stream.synchronize()
            progress(done, total)
    sim.stream.synchronize()
    wall = time.perf_counter() - t0
    last = []
    counters = []
    parts = []
    for i in range(len(descs)):
        rec = sim.diagnostics(i)
        last.append(rec[-1] if rec.shape[0] else np.full(48, np.nan))
        counters.append(sim.counters(i))
        if keep_particles:
            parts.append(sim.particles(i))
    out = {"last": np.array(last), "counters": counters, "wall_s": wall, "steps": total, "tiling": sim.tuning(),
           "tunings": tunings,
           "pairs": float(sum(c["pairs"] for c in counters)),
           "cluster_steps": int(sum(c["steps"] for c in counters))}
    if keep_particles:
        out["particles"] = parts
    sim.close()
    return out


def features(r0_nm, n_atoms, intensity_wcm2, fwhm_fs):
    """Surrogate inputs: logs of cluster radius (nm), atom count (Eq.(1)), peak intensity
    (W/cm^2) and pulse FWHM (fs); rows of float32."""
    return np.stack([np.log(r0_nm), np.log(n_atoms), np.log(intensity_wcm2), np.log(fwhm_fs)],
                    axis=-1).astype(np.float32)


def targets(last_records):
    """Surrogate outputs from each cluster's last record: asinh of the absorbed laser energy per
    atom in eV (log(2 W) for W well above 1 eV, and continuous through the weakly driven runs
    whose net laser work ends near zero or below it) and the mean ion charge."""
    r = np.asarray(last_records)
    return np.stack([np.arcsinh(r[:, R_ABS_EV]), r[:, R_MEANZ]], axis=-1).astype(np.float32)
