"""Benchmark: whole time steps of one argon cluster of 20k macroparticles on one MI355X.

Workload (synthetic, seeded): Ar cluster, R0 = 8 nm, 10,000 Ar+ + 10,000 electrons at
0.01 nm, 1e16 W/cm^2 at 800 nm, 30 fs FWHM Gaussian (Eq.(3)), dt = 0.05/w, softening
0.1 nm, charges frozen so the count stays 20k.  A step is one pass of the whole path: laser
value, Coulomb direct sum, Boris push, diagnostics every 100 steps (the ionization check is
not launched because ionization is off in this workload).

Prints one JSON line: G pair-interactions/s of the FP32+FP64-accumulation path (value), the
FP64 path on the same steps, the error between them, the Coulomb kernel's roofline figures
from HIP events recorded around its launches, and the FP64 CPU oracle timed on a bounded
sample of the same workload on this host's cores.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 20.0          # N-body convention for one softened pair interaction
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (published)
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (published)
VALU_ISSUE_PER_S = 256 * 2.4e9  # wave64 VALU instructions per second: 4 SIMD16 per CU, 4 cycles each


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_sim(precision, c, run, st, graph, tiling=None, boundary="open"):
    import paper_1307_3711_amd as lc
    from workloads.species import SPECIES
    # room for the pair-once kernel (blocks of 128 slots and up) where the precision allows it
    mpb = lc.pair_blocks_for([c.capacity], 128) if precision in ("fp32_acc64", "fp64") else 0
    cfg = lc.make_config(precision, ionize=run.ionize, dt=run.dt, softening_nm=run.softening_nm,
                         diag_every=run.diag_every, max_records=256, max_splits=64, seed=run.seed,
                         max_pair_blocks=mpb, boundary=boundary, box_r0=run.box_r0)
    desc = lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                           envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max,
                           electron_offset_nm=c.electron_offset_nm)
    sim = lc.Simulation(cfg, [desc])
    sim.init_from_host(0, st["x_nm"], st["u"], st["Z"])
    sim.start()
    if tiling:
        sim.set_tuning(**tiling)
        tuned = sim.tuning()
    else:
        tuned = sim.autotune()
    if graph:
        sim.set_graph(graph)
    return sim, tuned


def kernel_code_digest(path):
    """sha256 of a source file's code: '//' comments, trailing blanks and empty lines removed,
    so that a record stays valid across comment edits and is voided by any code change."""
    import hashlib
    import re
    lines = []
    for line in open(path, encoding="utf-8"):
        line = re.sub(r"//.*", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def counter_record(tuned, n, precision="fp32_acc64", boundary="open"):
    """The committed rocprofv3 counter record (HBM bytes per launch, VALU instructions) of the
    Coulomb kernel this precision, boundary and tiling run, or None when the kernel code or the
    tiling has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_force_ar20k_counters.json")
    try:
        recs = json.load(open(path))["records"]
        digest = kernel_code_digest(os.path.join(ROOT, "paper_1307_3711_amd", "csrc", "force.hip"))
    except (OSError, KeyError, ValueError):
        return None
    for rec in recs:
        if rec.get("force_hip_code_sha256") != digest or rec["n_particles"] != n:
            continue
        if rec.get("precision", "fp32_acc64") != precision or rec.get("boundary", "open") != boundary:
            continue
        if all(tuned.get(k) == v for k, v in rec["tiling"].items()):
            return rec
    return None


def pair_evaluations(n, tuned):
    """Pair terms one field pass evaluates: n^2 one-sided; with the pair-once kernel each pair
    of different blocks once and the pairs inside a block (self pair included) one-sided."""
    if not tuned.get("newton3"):
        return float(n) * n
    R, WJ = tuned["R"], tuned["WJ"]
    B = 64 * R if (R == WJ and R >= 3) else (4 // WJ) * 64 * R   # square shapes: one target group
    sizes = [min(B, n - i) for i in range(0, n, B)]
    return (float(n) * n + sum(float(b) * b for b in sizes)) / 2.0


def timed_steps(sim, steps):
    import torch
    sim.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.stream.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _oracle_steps(c, run, st, k=None, target_s=10.0):
    """Start the oracle on the state, take one calibration step, then time k steps (k sized to
    about target_s when not given); returns (k, seconds, positions after the run)."""
    import oracle
    osim = oracle.Sim.from_workload(c, run, st)
    osim.start()
    t0 = time.perf_counter()
    osim.run(1)
    t1 = time.perf_counter() - t0
    if k is None:
        k = max(1, min(200, int(target_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    osim.run(k)
    return k, time.perf_counter() - t0, osim.positions()


def cpu_baseline(c, run, st, n, target_s=10.0):
    """The FP64 oracle, as it is (gcc -O2), on a bounded number of steps of the same workload;
    beside it, for context, the same source built with -O3 -march=native on this host (same
    arithmetic: contraction and fast math stay off, which the equal positions confirm)."""
    import tempfile
    import numpy as np
    import oracle
    k, dt, x = _oracle_steps(c, run, st, target_s=target_s)
    out = {"value": k * n * n / dt / 1e9, "unit": "Gpair/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{k} steps of the same 20k-macroparticle state after 1 calibration step "
                     f"(FP64, gcc -O2, {dt:.1f} s)", "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    try:
        with tempfile.TemporaryDirectory() as d:
            with oracle.library(oracle.build_native(os.path.join(d, "liblc_oracle_native.so"))):
                _, dtn, xn = _oracle_steps(c, run, st, k=k)
        out["native"] = {"value": k * n * n / dtn / 1e9, "flags": "-O3 -march=native",
                         "same_positions": bool(np.array_equal(x, xn)), "seconds": round(dtn, 2)}
    except (OSError, subprocess.CalledProcessError) as e:
        out["native"] = {"value": None, "error": str(e)[:200]}
    return out


def cpu_model():
    """The host CPU's model name with its family / model / stepping numbers (/proc/cpuinfo;
    a virtual machine may report only a short name), for the CPU-baseline record."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
            elif info:
                break
    except OSError:
        return None
    if "model name" not in info:
        return None
    ids = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return info["model name"] + (f" ({ids})" if ids else "")


def ensemble_inputs(n_clusters, seed, steps_scale=1.0, capacity_rule="random"):
    """Descriptions and initial states of one seeded ensemble of uneven Ar/Xe clusters."""
    import paper_1307_3711_amd as lc
    from workloads import ensemble, initial_state
    from workloads.species import SPECIES
    cl = ensemble(n_clusters, seed=seed, capacity_rule=capacity_rule)
    descs, states = [], []
    for i, c in enumerate(cl):
        d = lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                            envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max,
                            electron_offset_nm=c.electron_offset_nm, n_steps=max(1, int(c.n_steps * steps_scale)))
        descs.append(d)
        states.append(initial_state(c, seed, i))
    return cl, descs, states


def ensemble_cpu_baseline(cl, states, r32, n_sample=8, steps=3000):
    """The FP64 oracle on a stratified sample of the ensemble (every len/n_sample-th cluster
    by capacity, `steps` steps each, about 10-30 s of CPU work): its cost per step is a N^2,
    so its pair rate on the sample (N^2 counted at the start of every step, as the GPU counts),
    applied to the pair count the GPU run evaluated, gives the oracle's time for the whole run
    and its cluster-steps/s."""
    import oracle
    from workloads import Run
    order = sorted(range(len(cl)), key=lambda i: cl[i].capacity)
    pick = [order[(2 * k + 1) * len(order) // (2 * n_sample)] for k in range(n_sample)]
    run = Run(dt=0.05, ionize=True, diag_every=50, seed=0)
    pairs, secs = 0.0, 0.0
    for i in pick:
        osim = oracle.Sim.from_workload(cl[i], run, states[i], i)
        osim.start()
        t0 = time.perf_counter()
        for _ in range(steps):
            pairs += float(osim.N) ** 2
            osim.run(1)
        secs += time.perf_counter() - t0
    rate = pairs / secs
    cpu_wall = r32["pairs"] / rate
    return {"value": round(r32["cluster_steps"] / cpu_wall, 2), "unit": "cluster-steps/s", "cores": oracle.threads(),
            "kind": "oracle", "sample": f"{n_sample} clusters stratified by capacity x {steps} steps "
                                        f"({secs:.1f} s, {rate / 1e9:.2f} G pair/s), extrapolated to the run's "
                                        f"{r32['pairs']:.3g} pair interactions"}


def bench_ensemble(args):
    """256 uneven clusters (Ar/Xe, 1k-16k capacity, 2-10 nm, 1e15-1e17 W/cm^2, 20-100 fs),
    each run to t_end = 4 FWHM (or --steps), FP32+FP64acc vs the FP64 path on the same work."""
    import numpy as np
    from paper_1307_3711_amd.ensemble import run_ensemble
    cl, descs, states = ensemble_inputs(args.clusters, args.seed)
    max_steps = args.steps if args.steps_given else None
    log(f"ensemble: {len(cl)} clusters, capacity {sum(c.capacity for c in cl)}, "
        f"up to {max(c.n_steps for c in cl)} steps")
    r32 = run_ensemble(descs, states, "fp32_acc64", max_steps=max_steps, graph_steps=args.graph // 2 or 50,
                       progress=lambda d, t: log(f"  fp32 step {d}/{t}"))
    out = {"metric": "cluster-steps/s (FP32 pair math + FP64 accumulation), 256-cluster ensemble",
           "value": round(r32["cluster_steps"] / r32["wall_s"], 2), "unit": "cluster-steps/s", "n_gpus": 1,
           "steps": r32["steps"], "warmup": 0, "ms_per_step": round(r32["wall_s"] / r32["steps"] * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64acc",
           "data": "synthetic",
           "config": {"workload": f"{len(cl)} Ar/Xe clusters, capacity log-uniform 1k-16k, R0 2-10 nm, "
                                  "1e15-1e17 W/cm2, FWHM 20-100 fs, t_end = 4 FWHM, ionization on",
                      "seed": args.seed, "tiling": r32["tiling"], "tilings": r32["tunings"],
                      "total_capacity": int(sum(c.capacity for c in cl))},
           "gpairs_per_s": round(r32["pairs"] / r32["wall_s"] / 1e9, 2), "pairs": r32["pairs"],
           "wall_s": round(r32["wall_s"], 3)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = ensemble_cpu_baseline(cl, states, r32)
    if not args.no_fp64:
        r64 = run_ensemble(descs, states, "fp64", max_steps=max_steps, graph_steps=args.graph // 2 or 50,
                           progress=lambda d, t: log(f"  fp64 step {d}/{t}"))
        a32, a64 = r32["last"][:, 19], r64["last"][:, 19]
        z32, z64 = r32["last"][:, 18], r64["last"][:, 18]
        rel_a = np.abs(a32 - a64) / np.maximum(np.abs(a64), 1e-30)
        out["fp64"] = {"value": round(r64["cluster_steps"] / r64["wall_s"], 2), "unit": "cluster-steps/s",
                       "gpairs_per_s": round(r64["pairs"] / r64["wall_s"] / 1e9, 2), "wall_s": round(r64["wall_s"], 3)}
        out["error_vs_fp64"] = {"absorbed_eV_per_atom_rel_median": float(np.median(rel_a)),
                                "absorbed_eV_per_atom_rel_p90": float(np.quantile(rel_a, 0.9)),
                                "mean_charge_abs_median": float(np.median(np.abs(z32 - z64))),
                                "mean_charge_abs_max": float(np.max(np.abs(z32 - z64)))}
    print(json.dumps(out), flush=True)


PUSH_BYTES = 173     # per live particle: read x,u (48) Z (1) cluster id (4) W_L,W_C (16) field (24);
                     # write x,u (48) W_L,W_C (16) float4 source (16)
ION_BYTES = 9        # per ion: read Z (1), write + read the ionization flag (8)


def bench_scan(args):
    """Coulomb-kernel rate against N: argon clusters at the density of the 20k workload
    (R0 = 8 nm (N / 20000)^(1/3), Ar+ and e- pairs, charges frozen), one-sided scalar-source
    tiling and pair-once tiling in FP32 pairs with FP64 accumulation, and the one-sided tiling
    with Kahan-compensated FP32 sums, each timed with HIP events around its field passes."""
    import paper_1307_3711_amd as lc
    from workloads import Cluster, Laser, Run, initial_state
    from workloads.species import SPECIES
    sizes = [int(v) for v in args.sizes.split(",")]
    tilings = {"one_sided": dict(R=1, WJ=4, T=1024, S=16, scalar=1),
               "pair_once": dict(R=4, WJ=4, T=1024, S=16, scalar=1, newton3=1),
               "kahan_one_sided": dict(R=1, WJ=4, T=1024, S=16, scalar=1)}
    precisions = {"one_sided": "fp32_acc64", "pair_once": "fp32_acc64", "kahan_one_sided": "fp32_kahan"}
    res = []
    for n in sizes:
        r0 = 8.0 * (n / 20000.0) ** (1.0 / 3.0)
        c = Cluster(species="Ar", r0_nm=r0, n_ion=n // 2, capacity=n, z_init=1,
                    laser=Laser(intensity_wcm2=1e16, envelope="flat"))
        run = Run(dt=0.05, ionize=False, diag_every=0, seed=args.seed)
        st = initial_state(c, run.seed)
        row = {"n": n, "r0_nm": round(r0, 3)}
        for name, til in tilings.items():
            sim, _ = make_sim(precisions[name], c, run, st, 0, til)
            sim.profile_steps(max(20, args.reps))  # warm-up at steady clocks, same launches
            prof = sim.profile_steps(args.reps)
            ms, cnt = prof["field"]
            t = ms / max(cnt, 1) * 1e-3
            row[name] = {"us_per_pass": round(t * 1e6, 2), "interactions_per_s": float(n) * n / t}
            sim.close()
            log(f"scan n={n} {name}: {t * 1e6:.1f} us, {float(n) * n / t / 1e12:.3f}e12 interactions/s")
        res.append(row)
    big = res[-1]["pair_once"]["interactions_per_s"]
    out = {"metric": "Coulomb pass interactions/s against N (FP32 pair math + FP64 accumulation)",
           "value": round(big / 1e9, 1), "unit": "Gpair/s", "n_gpus": 1, "steps": args.reps, "warmup": 5,
           "ms_per_step": res[-1]["pair_once"]["us_per_pass"] / 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64acc", "data": "synthetic",
           "config": {"workload": "Ar clusters at the 20k workload's density, sizes " + args.sizes,
                      "tilings": tilings, "precisions": precisions},
           "scan": res}
    print(json.dumps(out), flush=True)


def bench_particles(args):
    """HBM probe of the particle-parallel kernels on >= 4M live macroparticles: 1024 Ar
    clusters of 2048 Ar+ + 2048 e- (capacity 8192 each), FP32 sources, one source split."""
    import numpy as np
    import paper_1307_3711_amd as lc
    from workloads import Cluster, Laser, initial_state
    from workloads.species import SPECIES
    nc = args.clusters if args.clusters != 256 else 1024
    c = Cluster(species="Ar", r0_nm=6.0, n_ion=2048, capacity=8192, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=1e15, envelope="flat"))
    cfg = lc.make_config("fp32_acc64", ionize=True, diag_every=0, max_records=1, max_splits=1, seed=1, t0=1.3,
                         detector_r0=9.0 if args.detectors else 0.0, collisional=args.collisional)
    d = lc.make_cluster(SPECIES["Ar"], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2, envelope="flat",
                        polarization=args.polarization)
    sim = lc.Simulation(cfg, [d] * nc)
    st = initial_state(c, 1, 0)
    for i in range(nc):
        sim.init_from_host(i, st["x_nm"], st["u"], st["Z"])
    sim.set_tuning(S=1)
    sim.start()
    n_live = nc * st["x_nm"].shape[0]
    t = sim.time_particle_kernels(5)
    t = sim.time_particle_kernels(args.reps)
    push_gbs = n_live * PUSH_BYTES / (t["push_ms"] * 1e-3) / 1e9
    ion_gbs = nc * c.n_ion * ION_BYTES / (t["ionize_ms"] * 1e-3) / 1e9
    out = {"metric": "HBM GB/s of the push and ionization kernels (>= 4M live macroparticles)",
           "value": round(push_gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.reps, "warmup": 5,
           "ms_per_step": round(t["push_ms"], 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{nc} Ar clusters x (2048 Ar+ + 2048 e-), capacity 8192, 1e15 W/cm2 flat, "
                                  f"{args.polarization} polarization" + (", detectors at 9 R0" if args.detectors else "")
                                  + (", collisional ionization" if args.collisional else ""),
                      "live_particles": n_live, "ions": nc * c.n_ion},
           "roofline": {"bound": "hbm", "achieved": round(push_gbs, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(push_gbs / 8000.0, 4), "traffic": None, "kernel": "k_push",
                        "bytes_per_particle": PUSH_BYTES},
           # the check is bound by VALU issue (Philox4x64-10 per ion), not by its few bytes per ion
           "ionize": {"ms": round(t["ionize_ms"], 5), "GB_per_s": round(ion_gbs, 1), "bytes_per_ion": ION_BYTES,
                      "frac_of_hbm_peak": round(ion_gbs / 8000.0, 4), "bound": "valu"}}
    print(json.dumps(out), flush=True)


def _xe_run(precision, c, run, st, steps, tiling=None):
    import numpy as np
    import torch
    import paper_1307_3711_amd as lc
    from workloads.species import SPECIES
    de = 100
    mpb = lc.pair_blocks_for([c.capacity], 256) if precision in ("fp32_acc64", "fp64") else 0
    cfg = lc.make_config(precision, ionize=True, dt=run.dt, softening_nm=run.softening_nm, diag_every=de,
                         max_records=steps // de + 2, max_splits=16, seed=run.seed, max_pair_blocks=mpb)
    d = lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                        envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max,
                        electron_offset_nm=c.electron_offset_nm)
    sim = lc.Simulation(cfg, [d])
    sim.init_from_host(0, st["x_nm"], st["u"], st["Z"])
    sim.start()
    tuned = sim.autotune() if tiling is None else (sim.set_tuning(**tiling) or sim.tuning())
    sim.set_graph(de)
    sim.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(1000, steps - done)
        sim.step(k)
        done += k
        sim.stream.synchronize()
        log(f"  {precision}: step {done}/{steps}, N = {sim.counters(0)['n']}")
    wall = time.perf_counter() - t0
    rec = sim.diagnostics(0)
    cnt = sim.counters(0)
    sim.close()
    return {"wall": wall, "rec": rec, "counters": cnt, "tiling": tuned}


def bench_xe(args):
    """Xe, R0 = 20 nm, capacity 200k macroparticles (22,222 Xe+ + 22,222 e- at the start, room
    for Xe8+), 5e16 W/cm^2, 100 fs FWHM Gaussian, ionization on, 10k steps: long-pulse
    throughput of the FP32+FP64acc path and its energy bookkeeping, with the FP64 path on the
    first --fp64-steps steps for the error statement."""
    import numpy as np
    from workloads import initial_state, xe_200k
    c, run = xe_200k()
    st = initial_state(c, run.seed)
    steps = args.steps if args.steps_given else c.n_steps
    r32 = _xe_run("fp32_acc64", c, run, st, steps)
    rec = r32["rec"]
    # discrete energy identity (exact up to rounding) and total-energy bookkeeping
    ident = np.abs(rec[:, 5] - rec[:, 23] - (rec[:, 8] + rec[:, 9] + rec[:, 10]))
    ident_rel = float(np.max(ident / (np.abs(rec[:, 8]) + np.abs(rec[:, 9]) + rec[:, 10] + np.abs(rec[:, 23]))))
    out = {"metric": "G pair-interactions/s (FP32 pair math + FP64 accumulation), Xe long pulse",
           "value": round(r32["counters"]["pairs"] / r32["wall"] / 1e9, 2), "unit": "Gpair/s", "n_gpus": 1,
           "steps": steps, "warmup": 0, "ms_per_step": round(r32["wall"] / steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64acc", "data": "synthetic",
           "config": {"workload": "Xe cluster R0=20nm, capacity 200k (22,222 Xe+ + 22,222 e- at start), 5e16 W/cm2, "
                                  "100 fs Gaussian, ionization to Xe8+, dt=0.05", "tiling": r32["tiling"]},
           "cluster_steps_per_s": round(steps / r32["wall"], 2), "pairs": r32["counters"]["pairs"],
           "final_macroparticles": r32["counters"]["n"], "ionization_events": r32["counters"]["events"],
           "mean_charge_end": float(rec[-1, 18]), "absorbed_eV_per_atom_end": float(rec[-1, 19]),
           "energy_identity_max_rel_residual": ident_rel,
           "records": {"t": rec[:, 0].tolist(), "N": rec[:, 2].tolist(), "mean_Z": rec[:, 18].tolist(),
                       "absorbed_eV_per_atom": rec[:, 19].tolist()}}
    if not args.no_cpu_baseline:
        # the FP64 oracle on 20 steps from the same start (44,444 macroparticles); its cost per
        # step is a N^2, so its pair rate gives its time for the run's pair count
        import oracle
        from oracle import units
        osim = oracle.Sim.from_workload(c, run, st)
        osim.start()
        n0 = float(osim.N)
        t0 = time.perf_counter()
        osim.run(20)
        dt = time.perf_counter() - t0
        rate = 20 * n0 * n0 / dt
        # one field pass each on synthetic states of 100k and 200k macroparticles (the oracle's
        # own placement in the same sphere, one electron per ion), sizes the run grows through;
        # the run's time on the oracle is then the sum over its steps of N^2 / rate(N), the rate
        # interpolated linearly in N between the three samples
        sizes, rates = [n0], [rate]
        r0n = units.nm_to_norm(c.r0_nm, c.laser.lambda_um)
        eps2 = units.nm_to_norm(run.softening_nm, c.laser.lambda_um) ** 2
        for m in (100_000, 200_000):
            xs, zs = oracle.init_cluster(seed=99, cluster_index=0, n_ion=m // 2, z_init=1, r0=r0n, delta=r0n * 1e-3)
            t1 = time.perf_counter()
            oracle.coulomb_field(xs, zs.astype(np.float64), eps2, want_phi=False)
            sizes.append(float(m))
            rates.append(float(m) * m / (time.perf_counter() - t1))
        nrec = rec[:, 2]
        steps_per_rec = np.diff(np.concatenate([[0.0], rec[:, 1]]))
        t_run = float(np.sum(steps_per_rec * nrec * nrec / np.interp(nrec, sizes, rates)))
        value = float(r32["counters"]["pairs"]) / t_run
        out["cpu_baseline"] = {"value": round(value / 1e9, 3), "unit": "Gpair/s", "cores": oracle.threads(),
                               "kind": "oracle", "cpu": cpu_model(),
                               "rates_by_size": {str(int(n)): round(r / 1e9, 3) for n, r in zip(sizes, rates)},
                               "sample": f"20 steps at the start ({int(n0)} macroparticles, {dt:.1f} s) and one "
                                         f"field pass each at 100k and 200k; the run's "
                                         f"{r32['counters']['pairs']:.3g} pair interactions at these rates "
                                         f"(extrapolated over the run's N(t) records): {t_run / 3600:.1f} h"}
    if not args.no_fp64:
        n64 = min(args.fp64_steps, steps)
        r64 = _xe_run("fp64", c, run, st, n64)
        k = r64["rec"].shape[0]
        a, b = rec[:k], r64["rec"]

        def rel(col):
            return float(np.max(np.abs(a[:, col] - b[:, col])) / max(np.max(np.abs(b[:, col])), 1e-300))

        out["fp64"] = {"steps": n64, "gpairs_per_s": round(r64["counters"]["pairs"] / r64["wall"] / 1e9, 2),
                       "ms_per_step": round(r64["wall"] / n64 * 1e3, 4)}
        out["error_vs_fp64"] = {"over_steps": n64, "rel_KE": rel(5), "rel_PE": rel(7), "rel_W_laser": rel(8),
                                "events_fp32": float(a[-1, 21]), "events_fp64": float(b[-1, 21]),
                                "max_abs_mean_charge": float(np.max(np.abs(a[:, 18] - b[:, 18])))}
    print(json.dumps(out), flush=True)


def bench_iedf(args):
    """The Sec. III anisotropy study on synthetic input: Ar cluster of R0 = 8.2 nm (5000 Ar+
    macro-ions + 5000 e-, capacity for Ar8+), 806 nm, 8e15 W/cm^2, 100 fs Gaussian, ionization
    on, detectors at 9 R0 on the polarization axis (x) and across it (y), 30 degree acceptance.
    Reports the run's throughput and the time-integrated ion energy distributions."""
    import numpy as np
    import torch
    import paper_1307_3711_amd as lc
    from workloads import ar_anisotropy, initial_state
    from workloads.species import SPECIES
    c, run = ar_anisotropy()
    steps = args.steps if args.steps_given else c.n_steps
    st = initial_state(c, run.seed)
    mpb = lc.pair_blocks_for([c.capacity], 256)
    cfg = lc.make_config("fp32_acc64", ionize=True, lambda_um=c.laser.lambda_um, dt=run.dt,
                         softening_nm=run.softening_nm, diag_every=run.diag_every,
                         max_records=steps // run.diag_every + 2, max_splits=16, seed=run.seed, max_pair_blocks=mpb,
                         detector_r0=9.0, detector_half_angle_deg=30.0)
    d = lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                        envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max,
                        electron_offset_nm=c.electron_offset_nm)
    sim = lc.Simulation(cfg, [d])
    sim.init_from_host(0, st["x_nm"], st["u"], st["Z"])
    sim.start()
    tuned = sim.autotune()
    sim.set_graph(run.diag_every)
    sim.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(5000, steps - done)
        sim.step(k)
        done += k
        sim.stream.synchronize()
        counts, _ = sim.iedf(0)
        log(f"  iedf: step {done}/{steps}, N = {sim.counters(0)['n']}, ions detected {counts[0].sum()}")
    wall = time.perf_counter() - t0
    counts, edges = sim.iedf(0)
    rec = sim.diagnostics(0)
    cnt = sim.counters(0)
    sim.close()
    centres = np.concatenate([[edges[0] / 2], np.sqrt(edges[:-1] * edges[1:]), [edges[-1]]])

    def summary(row):
        n = int(counts[row].sum())
        mean = float(np.sum(counts[row] * centres) / n) if n else None
        return {"ions": n, "mean_keV": None if mean is None else round(mean / 1e3, 3),
                "counts": counts[row].tolist()}

    along, perp = summary(1), summary(2)
    out = {"metric": "G pair-interactions/s (FP32 pair math + FP64 accumulation), Ar anisotropy run",
           "value": round(cnt["pairs"] / wall / 1e9, 2), "unit": "Gpair/s", "n_gpus": 1, "steps": steps,
           "warmup": 0, "ms_per_step": round(wall / steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32+fp64acc", "data": "synthetic",
           "config": {"workload": "Ar cluster R0=8.2nm (~40k atoms), 5000 Ar+ + 5000 e- (capacity 45k), 806 nm, "
                                  "8e15 W/cm2, 100 fs Gaussian, ionization to Ar8+, dt=0.05, detectors at 9 R0, "
                                  "30 deg", "tiling": tuned},
           "final_macroparticles": cnt["n"], "mean_charge_end": float(rec[-1, 18]),
           "t_end_fs": float(rec[-1, 0]) * c.laser.lambda_um * 1e-6 / (2 * math.pi * 299792458.0) * 1e15,
           "ions_detected": int(counts[0].sum()), "along_polarization": along, "perpendicular": perp,
           "mean_energy_ratio_along_over_perp": (round(along["mean_keV"] / perp["mean_keV"], 4)
                                                 if along["mean_keV"] and perp["mean_keV"] else None),
           "bin_edges_eV": edges.tolist()}
    print(json.dumps(out), flush=True)


def bench_paper_scaling(args):
    """The run behind the paper's timing figure (Sec. III, Fig. 7), on synthetic input: a
    deuterium cluster of radius 80 A, fully ionized at the start (D+ with its electron beside
    it), 3000 macroparticles, 5000 steps.  The figure's laser is not given; this takes the
    deuterium study's 5e16 W/cm^2 and 25 fs at 800 nm.  The paper prints no absolute times (the
    figure is not in the text; it states the hardware, a 6-core Xeon E5645 at 2.40 GHz, and
    the fitted laws, time ~ N^2 and ~ cores^-2).  Reports the wall time of the 5000 steps on
    the GPU (FP32 pairs with FP64 accumulation, and FP64), the FP64 oracle's time for the same
    steps on the host, and the GPU time per step over N = 1000 .. 24000 macroparticles with
    the fitted exponent."""
    import numpy as np
    import oracle
    from workloads import Cluster, Laser, Run, initial_state
    laser = Laser(lambda_um=0.8, intensity_wcm2=5e16, envelope="gauss_field", fwhm_fs=25.0)
    steps = args.steps if args.steps_given else 5000
    run = Run(dt=0.05, ionize=False, diag_every=1000, seed=args.seed)

    def case(n_macro):
        c = Cluster(species="D", r0_nm=8.0, n_ion=n_macro // 2, capacity=n_macro, z_init=1, z_max=1, laser=laser,
                    n_steps=steps)
        return c, initial_state(c, args.seed)

    c, st = case(3000)
    out = {"metric": "wall seconds, 5000 steps of the paper's 3000-macroparticle deuterium cluster (Fig. 7 run)",
           "unit": "s", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "fp32+fp64acc", "data": "synthetic",
           "config": {"workload": "D cluster, R0 = 8 nm, fully ionized (1500 D+ + 1500 e-), 5e16 W/cm2, 25 fs, "
                                  "800 nm, dt = 0.05"}}
    for prec in ("fp32_acc64", "fp64"):
        sim, tuned = make_sim(prec, c, run, st, args.graph)
        sim.step(args.warmup)
        wall = timed_steps(sim, steps)
        sim.close()
        log(f"paper scaling: {prec} {steps} steps in {wall:.3f} s ({tuned})")
        if prec == "fp32_acc64":
            out["value"] = round(wall, 4)
            out["ms_per_step"] = round(wall / steps * 1e3, 5)
            out["tiling"] = tuned
        else:
            out["fp64"] = {"value": round(wall, 4), "unit": "s", "tiling": tuned}
    if not args.no_cpu_baseline:
        osim = oracle.Sim.from_workload(c, run, st)
        osim.start()
        t0 = time.perf_counter()
        osim.run(steps)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(dt, 3), "unit": "s", "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"the same {steps} steps in FP64 (gcc -O2)"}
        log(f"paper scaling: oracle {dt:.2f} s on {oracle.threads()} threads")
    sweep = []
    for n in (1000, 3000, 6000, 12000, 24000):
        cn, stn = case(n)
        sim, _ = make_sim("fp64", cn, run, stn, args.graph)
        sim.step(args.warmup)
        k = 1000
        wall = timed_steps(sim, k)
        sim.close()
        sweep.append({"n_macro": n, "ms_per_step_fp64": round(wall / k * 1e3, 5)})
    ns = np.array([r["n_macro"] for r in sweep], dtype=float)
    ts = np.array([r["ms_per_step_fp64"] for r in sweep])
    out["n_sweep"] = sweep
    # exponent of time ~ N^p over the three largest sizes (small N is launch-bound on the GPU)
    out["n_exponent_fp64"] = round(float(np.polyfit(np.log(ns[-3:]), np.log(ts[-3:]), 1)[0]), 3)
    print(json.dumps(out), flush=True)


def bench_lumping(args):
    """The Sec. III lumping study on synthetic input: the D_8007 cluster (R0 from Eq.(1) with
    R_W = 1.70 A), 857 nm, 5e16 W/cm^2, 25 fs Gaussian, run as one ensemble of copies lumped
    into 40 .. 500 ion macroparticles (one electron each; deuterium is fully ionized), four
    independent random placements per lumping.  Reports per lumping the final mean ion energy
    (mean and standard deviation over the placements) and mean / maximum (the paper: about
    3/5), and the spread of the mean over the lumpings (the paper: 7 % for a 92 % change of
    N_atoms / N_macro)."""
    import numpy as np
    import paper_1307_3711_amd as lc
    from paper_1307_3711_amd.ensemble import run_ensemble
    from workloads import Cluster, Laser, initial_state
    from workloads.species import SPECIES
    lam = 0.857
    r0 = SPECIES["D"]["rw_angstrom"] * 8007 ** (1.0 / 3.0) / 10.0
    laser = Laser(lambda_um=lam, intensity_wcm2=5e16, envelope="gauss_field", fwhm_fs=25.0)
    counts = [40, 60, 80, 120, 160, 200, 300, 400, 500]
    copies = args.copies
    t_end_fs = 300.0
    dt, soft = args.dt, args.softening
    w_fs = 2.0 * math.pi * 299792458.0 / (lam * 1e-6) * 1e-15
    steps = args.steps if args.steps_given else int(math.ceil(t_end_fs * w_fs / dt))
    cl = [Cluster(species="D", r0_nm=r0, n_ion=n, capacity=2 * n, z_init=1, z_max=1, laser=laser, n_steps=steps)
          for n in counts for _ in range(copies)]
    descs = [lc.make_cluster(SPECIES["D"], c.r0_nm, c.n_ion, c.capacity, laser.intensity_wcm2, envelope=laser.envelope,
                             fwhm_fs=laser.fwhm_fs, z_max=1, n_steps=steps) for c in cl]
    states = [initial_state(c, args.seed, i) for i, c in enumerate(cl)]
    log(f"lumping: D_8007 (R0 = {r0:.3f} nm) at {counts} ion macroparticles x {copies} placements, {steps} steps")
    out = run_ensemble(descs, states, "fp64", dt=dt, softening_nm=soft, lambda_um=lam, seed=args.seed,
                       diag_every=1000, autotune=False, keep_particles=True)
    # angular frequency of an electron bound at rest inside the softening core of its ion of
    # charge w (w real deuterons per macro-ion): omega_b = (kappa w / eps^3)^(1/2) in units of the
    # laser frequency; the leap-frog is stable for omega_b dt < 2
    u = lc.units(lam)
    eps = soft * u["k_per_nm"]
    mass = SPECIES["D"]["mass_u"] * 931494102.42  # eV
    rows = []
    for k, n in enumerate(counts):
        means, ratios = [], []
        for parts in out["particles"][k * copies:(k + 1) * copies]:
            ion = parts["Z"] > 0
            u2 = np.sum(parts["u"][ion] ** 2, axis=1)
            ke = mass * u2 / (1.0 + np.sqrt(1.0 + u2))  # M (gamma - 1) c^2 per real ion, eV
            means.append(ke.mean() / 1e3)
            ratios.append(ke.mean() / ke.max())
        rows.append({"n_macro_ions": n, "n_atoms_per_macro": round(8007 / n, 2),
                     "omega_bound_dt": round(math.sqrt(u["kappa"] * (8007 / n) / eps ** 3) * dt, 3),
                     "mean_keV": round(float(np.mean(means)), 4), "mean_keV_std": round(float(np.std(means)), 4),
                     "mean_over_max": round(float(np.mean(ratios)), 4)})
    m = np.array([r["mean_keV"] for r in rows])
    res = {"metric": "cluster-steps/s (FP64), D_8007 lumping ensemble", "value": round(out["cluster_steps"] / out["wall_s"], 1),
           "unit": "cluster-steps/s", "n_gpus": 1, "steps": steps, "warmup": 0,
           "ms_per_step": round(out["wall_s"] / steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"D_8007 (R0 {r0:.3f} nm), 857 nm, 5e16 W/cm2, 25 fs Gaussian, {t_end_fs:.0f} fs, "
                                  f"lumped into {counts[0]}..{counts[-1]} ion macroparticles, {copies} placements each",
                      "dt": dt, "softening_nm": soft},
           "lumpings": rows,
           "mean_energy_spread": round(float((m.max() - m.min()) / m.mean()), 4),
           "mean_energy_40_vs_500": round(float(abs(rows[0]["mean_keV"] - rows[-1]["mean_keV"]) / rows[-1]["mean_keV"]), 4),
           "atoms_per_macro_change": round(1.0 - counts[0] / counts[-1], 4)}
    print(json.dumps(res), flush=True)


def _features_of(cl):
    from paper_1307_3711_amd.ensemble import features
    from workloads.species import SPECIES
    import numpy as np
    r0 = np.array([c.r0_nm for c in cl])
    na = np.array([(c.r0_nm * 10.0 / SPECIES[c.species]["rw_angstrom"]) ** 3 for c in cl])
    inten = np.array([c.laser.intensity_wcm2 for c in cl])
    fwhm = np.array([c.laser.fwhm_fs for c in cl])
    return features(r0, na, inten, fwhm)


def bench_surrogate(args):
    """Train the 4-64-64-2 surrogate on ensemble MD runs, time 1M-point inference, and score it
    on held-out clusters re-run by the MD (three extra seeds give the MD's own spread)."""
    import numpy as np
    import torch
    import paper_1307_3711_amd as lc
    from paper_1307_3711_amd.ensemble import run_ensemble, targets
    from workloads import initial_state, surrogate_inputs
    from workloads.species import SPECIES
    from workloads.surrogate import init_params, row_order

    Xl, Yl = [], []
    md_wall = md_runs = md_cs = 0
    if args.load_data:  # an earlier run's MD training set (and its MD rate), to try training settings
        d = np.load(args.load_data)
        Xl, Yl = [d["X"]], [d["Y"]]
        md_wall, md_runs, md_cs = float(d["md_wall"]), int(d["md_runs"]), float(d["md_cs"])
    for b in range(0 if args.load_data else args.batches):
        cl, descs, states = ensemble_inputs(256, b, capacity_rule=args.lumping)
        r = run_ensemble(descs, states, "fp32_acc64", seed=b, progress=lambda d, t: log(f"  batch {b}: {d}/{t}"))
        md_wall += r["wall_s"]
        md_runs += len(cl)
        md_cs += r["cluster_steps"]
        Xl.append(_features_of(cl))
        Yl.append(targets(r["last"]))
        log(f"surrogate data: batch {b} done in {r['wall_s']:.1f} s")
    X = np.concatenate(Xl)
    Y = np.concatenate(Yl)
    if args.save_data:
        np.savez(args.save_data, X=X, Y=Y, md_wall=md_wall, md_runs=md_runs, md_cs=md_cs)
    n = X.shape[0]
    perm = np.random.Generator(np.random.Philox(key=[0, 77])).permutation(n)
    n_tr = int(0.9 * n)
    tr, va = perm[:n_tr], perm[n_tr:]
    Xtr, Ytr = torch.from_numpy(X[tr]).cuda(), torch.from_numpy(Y[tr]).cuda()
    net = lc.Surrogate(init_params(0))
    net.fit_scaler(Xtr, Ytr)
    batch = 256
    rows = torch.from_numpy(row_order(n_tr, batch, args.train_steps, 1)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # piecewise-constant learning rate: lr, lr/3, lr/10, lr/30 over four equal phases (Adam
    # moments and step count carry across the calls)
    q = args.train_steps // 4
    losses = torch.cat([net.train(Xtr, Ytr, rows[k * q * batch:], batch, q, args.lr * f)
                        for k, f in enumerate((1.0, 1 / 3, 0.1, 1 / 30))])
    net.stream.synchronize()
    train_s = time.perf_counter() - t0
    pv = net.infer(torch.from_numpy(X[va]).cuda()).cpu().numpy()
    val_rmse = np.sqrt(np.mean((pv - Y[va]) ** 2, axis=0))

    # inference throughput on 1M query points
    q = surrogate_inputs(1_000_000, seed=100)
    na = (q[:, 0] * 10.0 / q[:, 1]) ** 3
    from paper_1307_3711_amd.ensemble import features
    Xq = torch.from_numpy(features(q[:, 0], na, q[:, 2], q[:, 3])).cuda()
    net.infer(Xq)
    net.stream.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        Yq = net.infer(Xq)
    net.stream.synchronize()
    inf_s = (time.perf_counter() - t0) / reps

    # held-out clusters (ensemble seed 200) re-run by the MD with 4 seeds
    cl, descs, _ = ensemble_inputs(64, 200, capacity_rule=args.lumping)
    ph = net.infer(torch.from_numpy(_features_of(cl)).cuda()).cpu().numpy()
    md = []
    for sd in (200, 201, 202, 203):
        states = [initial_state(c, sd, i) for i, c in enumerate(cl)]
        r = run_ensemble(descs, states, "fp32_acc64", seed=sd)
        md.append(targets(r["last"]))
    md = np.array(md)
    # the same held-out clusters lumped differently: capacities (hence ion macroparticle counts)
    # drawn again log-uniformly, physics unchanged; their spread is what the lumping alone does to
    # the MD's outcome, which the network's inputs cannot tell apart
    lump = []
    if args.lumping == "random":
        from dataclasses import replace as dc_replace
        for k in range(3):
            rng = np.random.Generator(np.random.Philox(key=[300 + k, 5]))
            cl2 = []
            for c in cl:
                cap = int(round(math.exp(rng.uniform(math.log(1000), math.log(16000)))))
                n_atoms = int(math.floor((c.r0_nm * 10.0 / SPECIES[c.species]["rw_angstrom"]) ** 3))
                cl2.append(dc_replace(c, capacity=cap, n_ion=max(1, min(cap // 9, n_atoms))))
            d2 = [lc.make_cluster(SPECIES[c.species], c.r0_nm, c.n_ion, c.capacity, c.laser.intensity_wcm2,
                                  envelope=c.laser.envelope, fwhm_fs=c.laser.fwhm_fs, z_max=c.z_max,
                                  electron_offset_nm=c.electron_offset_nm, n_steps=c.n_steps) for c in cl2]
            st2 = [initial_state(c, 200, i) for i, c in enumerate(cl2)]
            lump.append(targets(run_ensemble(d2, st2, "fp32_acc64", seed=200)["last"]))
    rmse_lump = (np.sqrt(np.mean((np.array(lump) - md[0][None]) ** 2, axis=(0, 1))) if lump else None)
    rmse_sur = np.sqrt(np.mean((ph - md[0]) ** 2, axis=0))
    rmse_md = np.sqrt(np.mean((md[1:] - md[0][None]) ** 2, axis=(0, 1)))
    med_sur = np.median(np.abs(ph - md[0]), axis=0)
    med_md = np.median(np.abs(md[1:] - md[0][None]), axis=(0, 1))
    # the method without the network: predicting the training mean
    rmse_mean = np.sqrt(np.mean((Y[tr].mean(axis=0)[None] - md[0]) ** 2, axis=0))
    md_runs_per_s = md_runs / md_wall
    out = {"metric": "surrogate points/s (BF16 MFMA 4-64-64-2) vs MD cluster runs/s", "value": round(1e6 / inf_s, 1),
           "unit": "points/s", "n_gpus": 1, "steps": args.train_steps, "warmup": 0,
           "ms_per_step": round(train_s / max(args.train_steps, 1) * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
           "config": {"workload": f"{md_runs} ensemble MD runs ({args.batches} x 256 clusters), 90/10 split, "
                                  "batch 256, Adam; 1M-point inference; 64 held-out clusters re-run by MD",
                      "lr": args.lr, "lumping": args.lumping},
           "md_runs_per_s": round(md_runs_per_s, 3), "md_cluster_steps_per_s": round(md_cs / md_wall, 1),
           "speedup_vs_md": round((1e6 / inf_s) / md_runs_per_s, 1), "train_s": round(train_s, 3),
           "final_train_loss": float(losses[-50:].mean().cpu()),
           "targets": "asinh(absorbed eV per atom), mean ion charge",
           "val_rmse": {"asinh_absorbed_eV": float(val_rmse[0]), "mean_charge": float(val_rmse[1])},
           "heldout_rmse_vs_md": {"asinh_absorbed_eV": float(rmse_sur[0]), "mean_charge": float(rmse_sur[1])},
           "md_seed_spread_rmse": {"asinh_absorbed_eV": float(rmse_md[0]), "mean_charge": float(rmse_md[1])},
           "heldout_median_abs_err": {"asinh_absorbed_eV": float(med_sur[0]), "mean_charge": float(med_sur[1])},
           "md_seed_spread_median_abs": {"asinh_absorbed_eV": float(med_md[0]), "mean_charge": float(med_md[1])},
           "train_mean_predictor_rmse": {"asinh_absorbed_eV": float(rmse_mean[0]), "mean_charge": float(rmse_mean[1])}}
    if rmse_lump is not None:
        out["md_lumping_spread_rmse"] = {"asinh_absorbed_eV": float(rmse_lump[0]), "mean_charge": float(rmse_lump[1])}
    print(json.dumps(out), flush=True)


PROFILE_STEPS = 400  # MD steps whose dispatches record their own events, after the timed window


def default_counts(workload, steps, warmup):
    """Timed and warmup steps when not given: for the Ar 20k workload a step is one diagnostic
    period, and 5 + 30 periods plus the profiled steps stay inside the workload's 4000 MD steps,
    so the default run also reaches the comparison with the oracle's records; other workloads
    count their own steps."""
    if steps is None:
        steps = 30 if workload == "ar20k" else 1000
    if warmup is None:
        warmup = 5 if workload == "ar20k" else 100
    return steps, warmup


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batches", type=int, default=16, help="surrogate: 256-cluster ensembles of training data")
    ap.add_argument("--train-steps", type=int, default=48000)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--lumping", default="radius", choices=["random", "radius"],
                    help="surrogate: capacity (lumping) drawn at random (the ensemble recipe) or fixed by R0")
    ap.add_argument("--save-data", default="", help="surrogate: write the MD training set (npz) here")
    ap.add_argument("--load-data", default="", help="surrogate: train on a saved MD training set instead")
    ap.add_argument("--fp64-steps", type=int, default=2000, help="xe200k: steps of the FP64 comparison run")
    ap.add_argument("--workload", default="ar20k", choices=["ar20k", "ensemble", "surrogate", "particles", "xe200k", "iedf",
                                                            "lumping",
                                                            "scan", "paper_scaling"])
    ap.add_argument("--sizes", default="20000,30000,40000,60000,100000",
                    help="particle counts of the scan workload")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--dt", type=float, default=0.05, help="lumping: time step (1/w)")
    ap.add_argument("--softening", type=float, default=0.4,
                    help="lumping: softening length (nm); 0.4 nm resolves the lumped electron-ion pairs")
    ap.add_argument("--copies", type=int, default=4, help="lumping: random placements per lumping")
    ap.add_argument("--clusters", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (ar20k: diagnostic periods of 100 MD steps, default 30; others: 1000)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before them (ar20k: periods, default 5; others: 100)")
    ap.add_argument("--profile-steps", type=int, default=PROFILE_STEPS)
    ap.add_argument("--graph", type=int, default=100)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-records", action="store_true",
                    help="ar20k: skip running both paths to step 4000 against the oracle's records")
    ap.add_argument("--tiling", default="", help="R,WJ,T,S,persistent[,scalar[,newton3]]: skip the autotuner")
    ap.add_argument("--tiling-fp64", default="", help="the same for the FP64 comparison run")
    ap.add_argument("--polarization", default="linear_x", choices=["linear_x", "circular"],
                    help="particles workload: laser polarization")
    ap.add_argument("--detectors", action="store_true", help="particles workload: ion detectors at 9 R0")
    ap.add_argument("--collisional", action="store_true",
                    help="particles workload: collisional ionization rate added to the tunnelling rate")
    ap.add_argument("--boundary", default="open", choices=["open", "periodic"],
                    help="ar20k: boundaries of the simulation box (periodic: cube of 20 R0)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB buffer 3 times (HBM counter calibration for rocprofv3)")
    args = ap.parse_args()
    args.steps_given = args.steps is not None
    args.steps, args.warmup = default_counts(args.workload, args.steps, args.warmup)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be at least 1 and --warmup at least 0", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}))
        return
    def parse_tiling(text):
        if not text:
            return None
        v = [int(x) for x in text.split(",")] + [0, 0]
        return dict(R=v[0], WJ=v[1], T=v[2], S=v[3], persistent=v[4], scalar=v[5], newton3=v[6])

    tiling = parse_tiling(args.tiling)
    tiling64 = parse_tiling(args.tiling_fp64)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "particles":
        return bench_particles(args)
    if args.workload == "scan":
        return bench_scan(args)
    if args.workload == "xe200k":
        return bench_xe(args)
    if args.workload == "iedf":
        return bench_iedf(args)
    if args.workload == "lumping":
        return bench_lumping(args)
    if args.workload == "paper_scaling":
        return bench_paper_scaling(args)

    import numpy as np
    import torch
    import paper_1307_3711_amd as lc
    from workloads import ar_20k, initial_state

    c, run = ar_20k()
    st = initial_state(c, run.seed)
    n = st["x_nm"].shape[0]
    pairs = float(n) * float(n)

    # One benchmark step is one diagnostic period: diag_every MD steps (one captured graph
    # replay) whose last one carries the diagnostic pass, so that the timed window of exactly
    # --steps steps holds the work the workload prescribes, diagnostics included, starting on a
    # period boundary after --warmup such steps.
    period = max(run.diag_every, 1)
    warmup_md = args.warmup * period
    steps_md = args.steps * period
    log(f"bench: {n} macroparticles, fp32_acc64, autotune")
    sim, tuned = make_sim("fp32_acc64", c, run, st, args.graph, tiling, args.boundary)
    log(f"bench: tiling {tuned}; warmup {args.warmup} x {period} MD steps")
    sim.step(warmup_md)
    sim.stream.synchronize()
    log(f"bench: timing {args.steps} x {period} MD steps")
    wall = timed_steps(sim, steps_md)
    log(f"bench: {wall:.3f} s; profiling {args.profile_steps} MD steps")
    prof = sim.profile_steps(args.profile_steps)
    rec32 = sim.diagnostics(0)
    force_ms, force_n = prof["field"]
    avg_force_s = force_ms / max(force_n, 1) * 1e-3
    achieved = FLOPS_PER_PAIR * pairs / avg_force_s / 1e12
    value = steps_md * pairs / wall / 1e9
    crec = counter_record(tuned, n, "fp32_acc64", args.boundary)
    evals = pair_evaluations(n, tuned)
    kname = "k_force_n3" if tuned.get("newton3") else "k_force_f32"
    out = {
        "metric": "G pair-interactions/s (FP32 pair math + FP64 accumulation), one Ar cluster",
        "value": round(value, 3), "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32+fp64acc", "data": "synthetic",
        "config": {"workload": "Ar cluster R0=8nm, 20k macroparticles (10k Ar+ + 10k e-), 1e16 W/cm2, "
                               "30 fs Gaussian, dt=0.05, softening 0.1 nm, charges frozen"
                               + ("" if args.boundary == "open" else f", {args.boundary} boundaries (cube of 20 R0)"),
                   "n_particles": n, "pairs_per_md_step": pairs, "tiling": tuned, "graph_steps": args.graph,
                   "diagnostic_every": period,
                   "step": f"one diagnostic period: {period} MD steps of dt=0.05/w, the last with the diagnostic pass",
                   "md_steps_per_step": period},
        "ms_per_md_step": round(wall / steps_md * 1e3, 5),
        "cluster_steps_per_s": round(steps_md / wall, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": crec["traffic_bytes_per_launch"] if crec else None,
                     "kernel": kname, "avg_launch_ms": round(avg_force_s * 1e3, 5),
                     "launches": force_n, "flops_per_pair": FLOPS_PER_PAIR,
                     "pair_interactions_per_launch": pairs, "pair_evaluations_per_launch": evals,
                     "valu_issue_frac": (round(crec["valu_wave_instructions"] / (crec["avg_duration_ns"] * 1e-9)
                                               / VALU_ISSUE_PER_S, 4) if crec else None)},
        "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items() if v[1]},
    }
    total_steps = warmup_md + steps_md + args.profile_steps
    if not args.no_fp64:
        log("bench: fp64 path on the same steps")
        sim64, tuned64 = make_sim("fp64", c, run, st, args.graph, tiling64, args.boundary)
        sim64.step(warmup_md)
        wall64 = timed_steps(sim64, steps_md)
        prof64 = sim64.profile_steps(args.profile_steps)
        rec64 = sim64.diagnostics(0)
        f64_ms, f64_n = prof64["field"]
        avg64_s = f64_ms / max(f64_n, 1) * 1e-3
        ach64 = FLOPS_PER_PAIR * pairs / avg64_s / 1e12
        crec64 = counter_record(tuned64, n, "fp64", args.boundary)
        p32 = sim.particles(0)
        p64 = sim64.particles(0)
        r0n = c.r0_nm * lc.units(0.8)["k_per_nm"]
        last32, last64 = rec32[-1], rec64[-1]

        def rel(col):
            return float(abs(last32[col] - last64[col]) / max(abs(last64[col]), 1e-300))

        out["fp64"] = {"value": round(steps_md * pairs / wall64 / 1e9, 3), "unit": "Gpair/s",
                       "ms_per_step": round(wall64 / args.steps * 1e3, 5),
                       "ms_per_md_step": round(wall64 / steps_md * 1e3, 5), "tiling": tuned64,
                       "roofline": {"bound": "alu", "achieved": round(ach64, 3), "peak": FP64_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(ach64 / FP64_PEAK_TFLOPS, 4),
                                    "traffic": crec64["traffic_bytes_per_launch"] if crec64 else None,
                                    "kernel": "k_force_n3" if tuned64.get("newton3") else "k_force_f64",
                                    "avg_launch_ms": round(avg64_s * 1e3, 5), "launches": f64_n,
                                    "pair_evaluations_per_launch": pair_evaluations(n, tuned64),
                                    "valu_issue_frac": (round(crec64["valu_wave_instructions"]
                                                              / (crec64["avg_duration_ns"] * 1e-9)
                                                              / VALU_ISSUE_PER_S, 4) if crec64 else None)}}
        out["error_vs_fp64"] = {"after_steps": total_steps, "t": float(last64[0]),
                                "max_dx_over_R0": float(np.max(np.abs(p32["x"] - p64["x"])) / r0n),
                                "median_dx_over_R0": float(np.median(np.linalg.norm(p32["x"] - p64["x"], axis=1)) / r0n),
                                "rel_KE": rel(lc.R_KE_HALF), "rel_PE": rel(lc.R_PE),
                                "rel_absorbed_eV_per_atom": rel(lc.R_ABS_EV)}
        # both runs to the workload's end (4000 steps), record by record against the FP64
        # oracle's records of the same run (tests/golden, written from the oracle alone)
        if c.n_steps >= total_steps and args.boundary == "open" and not args.no_oracle_records:
            log("bench: runs to the end, against the oracle's records")
            out["error_vs_fp64_oracle"] = {
                "fp32_acc64": oracle_record_errors(sim, c.n_steps - total_steps),
                "fp64": oracle_record_errors(sim64, c.n_steps - total_steps)}
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(c, run, st, n, target_s=13.0)
    print(json.dumps(out), flush=True)


def oracle_record_errors(sim, more_steps):
    """Step a 20k argon run to the workload's end and compare its diagnostic records with the
    FP64 oracle's (tests/golden/ar20k_oracle_records.json): the largest difference of KE, PE,
    laser and Coulomb work over the run, relative to the energy scale |KE|+|PE|+|W_L|+|W_C| of
    each record, and the absorbed energy per atom at the end, relative."""
    import numpy as np
    with open(os.path.join(ROOT, "tests", "golden", "ar20k_oracle_records.json")) as f:
        gold = json.load(f)
    cols = gold["columns"]
    g = np.array(gold["records"])
    sim.step(more_steps)
    r = sim.diagnostics(0)
    steps = list(r[:, 1])
    idx = [steps.index(s) for s in g[:, cols.index("step")]]
    r = r[idx]
    col = lambda name: g[:, cols.index(name)]
    scale = np.abs(col("KE_half")) + np.abs(col("PE")) + np.abs(col("W_laser")) + np.abs(col("W_coulomb"))
    out = {"records": len(idx), "last_step": int(r[-1, 1])}
    for name, c in (("KE", 5), ("PE", 7), ("W_laser", 8), ("W_coulomb", 9)):
        key = {"KE": "KE_half"}.get(name, name)
        out["max_rel_" + name] = float(np.max(np.abs(r[:, c] - col(key)) / scale))
    a_g, a_o = float(r[-1, 19]), float(col("absorbed_eV_per_atom")[-1])
    out["absorbed_eV_per_atom"] = {"gpu": a_g, "oracle": a_o, "rel": abs(a_g - a_o) / abs(a_o)}
    return out


if __name__ == "__main__":
    main()
