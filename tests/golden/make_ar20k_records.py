"""Writes ar20k_oracle_records.json: the FP64 oracle's diagnostic records of the 20k-macroparticle
argon workload (R0 = 8 nm, 10k Ar+ + 10k electrons, 1e16 W/cm^2, 30 fs Gaussian, dt = 0.05,
charges frozen, 4000 steps, one record every 100 steps).  Calls only the oracle and the seeded
workload generator; the GPU tests and the benchmark compare the GPU path's records with these.

Usage: python tests/golden/make_ar20k_records.py [--plain]   (about 10-20 minutes on 8 cores;
--plain uses the -O2 build instead of the -O3 -march=native build of the same source, whose
arithmetic is identical: contraction and fast math are off in both)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import ar_20k, initial_state  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ar20k_oracle_records.json")
COLS = {"t": 0, "step": 1, "N": 2, "KE_half": 5, "KE_bar": 6, "PE": 7, "W_laser": 8, "W_coulomb": 9,
        "p_x": 11, "p_y": 12, "p_z": 13, "F_x": 14, "F_y": 15, "F_z": 16, "F_abs": 17, "absorbed_eV_per_atom": 19,
        "envelope": 22}


def main():
    c, run = ar_20k()
    st = initial_state(c, run.seed)
    t0 = time.time()
    lib_path = None
    if "--plain" not in sys.argv:
        lib_path = oracle.build_native(os.path.join(os.path.dirname(oracle.__file__), "liblc_oracle_native.so"))
    import contextlib
    ctx = oracle.library(lib_path) if lib_path else contextlib.nullcontext()
    recs = []
    with ctx:
        sim = oracle.Sim.from_workload(c, run, st)
        sim.start()
        ke_start = sim.ke_start
        for k in range(0, c.n_steps, 100):
            r = sim.run(100)
            recs.extend(r.tolist())
            print(f"step {k + 100}/{c.n_steps}: {time.time() - t0:.0f} s", flush=True)
    out = {
        "_about": "FP64 oracle records of the 20k argon workload (Sec. II model; workloads.ar_20k, seed 0), "
                  "written by tests/golden/make_ar20k_records.py",
        "workload": "Ar R0=8nm, 10k Ar+ + 10k e-, 1e16 W/cm2, 30 fs Gaussian (Eq.(3) as printed), dt=0.05, "
                    "softening 0.1 nm, charges frozen, 4000 steps, record every 100 steps",
        "oracle_build": "gcc -O2 -fopenmp -ffp-contract=off" if lib_path is None else
                        "gcc -O3 -march=native -fopenmp -ffp-contract=off (same arithmetic as -O2)",
        "threads": oracle.threads(),
        "seconds": round(time.time() - t0, 1),
        "ke_start": ke_start,
        "columns": list(COLS),
        "records": [[r[i] for i in COLS.values()] for r in recs],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("wrote", OUT, len(recs), "records", flush=True)


if __name__ == "__main__":
    main()
