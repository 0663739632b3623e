"""Failure handling that a caller can force from the host: non-finite or mis-ordered initial
particles are rejected before anything reaches the device (LC_E_NONFINITE, LC_E_INVALID), and a
checkpoint that is truncated or belongs to another configuration is refused (LC_E_INVALID)
without touching the handle's state, which keeps stepping as before."""
import os
import tempfile

import numpy as np
import pytest

from workloads import Run, small_ar

from _helpers import gpu_available, gpu_run

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_rejected_inputs_and_checkpoints():
    import paper_1307_3711_amd as lc
    c, run = small_ar()
    sim, states = gpu_run([c], run, "fp64")
    st = states[0]
    x = st["x_nm"].copy()
    x[7, 1] = np.nan
    with pytest.raises(lc.LcError) as ei:
        sim.init_from_host(0, x, st["u"], st["Z"])
    assert ei.value.code == lc.LC_E_NONFINITE
    Z = st["Z"].copy()
    Z[c.n_ion + 3] = 2  # an ion charge in an electron slot
    with pytest.raises(lc.LcError) as ei:
        sim.init_from_host(0, st["x_nm"], st["u"], Z)
    assert ei.value.code == lc.LC_E_INVALID
    sim.step(10)
    with tempfile.TemporaryDirectory() as d:
        good = os.path.join(d, "ck.bin")
        sim.save(good)
        cut = os.path.join(d, "cut.bin")
        with open(good, "rb") as f:
            blob = f.read()
        with open(cut, "wb") as f:
            f.write(blob[: len(blob) // 2])
        with pytest.raises(lc.LcError) as ei:
            sim.load(cut)
        assert ei.value.code == lc.LC_E_INVALID
        other, _ = gpu_run([c], Run(dt=0.025, ionize=True, diag_every=10, seed=0), "fp64")
        with pytest.raises(lc.LcError) as ei:
            other.load(good)
        assert ei.value.code == lc.LC_E_INVALID
        other.close()
        # the refused loads left the handle as it was: it resumes bitwise from its own state
        sim2, _ = gpu_run([c], run, "fp64", states=states)
        sim2.load(good)
        sim.step(5)
        sim2.step(5)
        assert np.array_equal(sim.particles(0)["x"], sim2.particles(0)["x"])
        assert np.array_equal(sim.particles(0)["Z"], sim2.particles(0)["Z"])
        sim2.close()
    sim.close()
