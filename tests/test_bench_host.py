"""Host logic of bench.py that needs no GPU: the one-GPU guard, the code digest that keeps a
rocprofv3 counter record tied to the Coulomb kernel's source, the record lookup, and the pair
count one field pass evaluates."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and not r.stdout.strip()


SRC = """// a kernel
__global__ void k(float* x) {  // one thread per element
  x[threadIdx.x] += 1.0f;
}
"""


def _fake_root(tmp_path, src, rec_digest_of=None, n=20000):
    d = tmp_path / "paper_1307_3711_amd" / "csrc"
    d.mkdir(parents=True)
    (d / "force.hip").write_text(src)
    (tmp_path / "profiles").mkdir()
    digest = bench.kernel_code_digest(str(d / "force.hip")) if rec_digest_of is None else rec_digest_of
    rec = {"force_hip_code_sha256": digest, "n_particles": n, "precision": "fp32_acc64", "boundary": "open",
           "tiling": {"R": 4, "WJ": 4, "newton3": 1}, "fetch_bytes": 1.0, "write_bytes": 2.0}
    (tmp_path / "profiles" / "k_force_ar20k_counters.json").write_text(json.dumps({"records": [rec]}))
    return d / "force.hip"


def test_code_digest_ignores_comments_and_blank_lines(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text(SRC)
    b.write_text("// another comment\n\n" + SRC.replace("// one thread per element", "// changed   ") + "\n\n")
    c.write_text(SRC.replace("1.0f", "2.0f"))
    assert bench.kernel_code_digest(str(a)) == bench.kernel_code_digest(str(b))
    assert bench.kernel_code_digest(str(a)) != bench.kernel_code_digest(str(c))


def test_counter_record_follows_the_kernel_source(tmp_path, monkeypatch):
    src = _fake_root(tmp_path, SRC)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tuned = {"R": 4, "WJ": 4, "T": 1024, "S": 1, "persistent": 0, "scalar": 0, "newton3": 1}
    rec = bench.counter_record(tuned, 20000)
    assert rec is not None and rec["write_bytes"] == 2.0
    # another tiling, size, precision or boundary has no record
    assert bench.counter_record(dict(tuned, R=2), 20000) is None
    assert bench.counter_record(tuned, 20001) is None
    assert bench.counter_record(tuned, 20000, precision="fp64") is None
    assert bench.counter_record(tuned, 20000, boundary="periodic") is None
    # a comment edit keeps the record, a code change voids it
    src.write_text("// note\n" + SRC)
    assert bench.counter_record(tuned, 20000) is not None
    src.write_text(SRC.replace("+=", "-="))
    assert bench.counter_record(tuned, 20000) is None


def test_counter_record_absent_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_record({"R": 4, "WJ": 4, "newton3": 1}, 20000) is None


@pytest.mark.parametrize("n", [1, 255, 256, 257, 20000])
def test_pair_evaluations(n):
    # one-sided: every ordered pair (self pairs included, they add zero)
    assert bench.pair_evaluations(n, {"newton3": 0}) == float(n) * n
    # pair-once, blocks of 256: pairs of different blocks once, pairs inside a block one-sided
    B = 256
    nb = -(-n // B)
    sizes = [min(B, n - k * B) for k in range(nb)]
    cross = sum(sizes[i] * sizes[j] for i in range(nb) for j in range(i + 1, nb))
    inside = sum(b * b for b in sizes)
    assert bench.pair_evaluations(n, {"newton3": 1, "R": 4, "WJ": 4}) == float(cross + inside)
    if n == 20000:
        assert bench.pair_evaluations(n, {"newton3": 1, "R": 4, "WJ": 4}) == 202556416.0


def test_step_counts_are_checked_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "0"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--steps" in r.stderr and not r.stdout.strip()


def test_default_ar20k_run_reaches_the_oracle_records():
    """A step of the Ar 20k benchmark is one diagnostic period; the default warmup, timed and
    profiled steps must end inside the workload's MD steps, where the runs continue to the
    workload's end against the oracle's records."""
    from workloads import ar_20k
    c, run = ar_20k()
    steps, warmup = bench.default_counts("ar20k", None, None)
    assert (steps + warmup) * run.diag_every + bench.PROFILE_STEPS <= c.n_steps
    assert bench.default_counts("ar20k", 20, 5) == (20, 5)
    assert bench.default_counts("ensemble", None, None) == (1000, 100)
