"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times (block, chunk and re-sort cadence the autotuner picks on
the MI355X), against the FP64 oracle on what the oracle can afford:

  * cfg3, all 256 scenes (7.7 M particles) stepped together, one control
    step (25 substeps, replayed from a captured hipGraph as the benchmark
    runs it) with block 8, chunk 8192: sampled scenes (the first,
    the last, the largest, the smallest) against the oracle run on each
    alone (the scenes are independent), 1e-3 dx; every scene's state stays
    finite and inside its grid;
  * cfg4, the 1,048,576-particle heap on a 128^3 grid with 3 colliders,
    one control step (25 substeps, graph replay) with block 4, chunk 8192,
    re-sort every 10 (three sorts in the run): every particle against the
    oracle, 1e-3 dx.
"""
import numpy as np
import pytest

from gpu_util import announce
from paper_2302_04659_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2302_04659_amd import mpm as m
    m.lib()
    return m


def test_cfg3_full_batch_sampled_scenes(mpm, orc):
    batch = scenes.cfg3(n_ctrl=2)
    counts = np.array([sc.n for sc in batch])
    announce("full-size cfg3", len(batch), "scenes", int(counts.sum()), "particles")
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, 8)
    sim.set_option(mpm.OPT_CHUNK, 8192)
    sim.set_option(mpm.OPT_SORT_EVERY, 50)
    sim.set_option(mpm.OPT_GRAPH, 1)
    sim.set_colliders_ctrl(0)
    sim.step(25)
    assert sim.sync() == mpm.OK
    sample = sorted({0, len(batch) - 1, int(counts.argmax()), int(counts.argmin())})
    for s in sample:
        sc = batch[s]
        o = orc.Oracle(sc)
        o.set_colliders(sc.ctrl_poses[0], sc.ctrl_vels[0])
        o.step(25)
        x, v, C, F = sim.get_state(s)
        err = np.abs(x - o.x).max() / sc.dx
        print("cfg3 scene", s, "n", sc.n, "max |dx| / dx", err)
        assert err <= 1e-3
    x_all, *_ = sim.get_state(-1)
    assert np.all(np.isfinite(x_all))
    lo = np.repeat([sc.dx for sc in batch], counts)[:, None]
    assert np.all(x_all >= 0.0) and np.all(x_all <= 64 * lo)
    sim.close()


def test_cfg4_full_scene(mpm, orc):
    sc = scenes.cfg4(n_ctrl=2)
    announce("full-size cfg4", sc.n, "particles")
    sim = mpm.Sim([sc])
    sim.set_option(mpm.OPT_BLOCK, 4)
    sim.set_option(mpm.OPT_CHUNK, 8192)
    sim.set_option(mpm.OPT_SORT_EVERY, 10)
    sim.set_option(mpm.OPT_GRAPH, 1)
    sim.set_colliders_ctrl(0)
    sim.step(25)
    assert sim.sync() == mpm.OK
    o = orc.Oracle(sc)
    o.set_colliders(sc.ctrl_poses[0], sc.ctrl_vels[0])
    o.step(25)
    x, v, C, F = sim.get_state(0)
    err = np.abs(x - o.x).max() / sc.dx
    print("cfg4 max |dx| / dx after 25 substeps:", err, "rms", np.sqrt(((x - o.x) ** 2).sum(1).mean()) / sc.dx)
    assert err <= 1e-3
    sim.close()
