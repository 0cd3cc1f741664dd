"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times (block, chunk and re-sort cadence the autotuner picks on
the MI355X), against the FP64 oracle on what the oracle can afford:

  * cfg3, all 256 scenes (7.7 M particles) stepped together with block 8,
    chunk 8192, re-sort every 100 substeps, G2P fused with the next P2G:
      - positions after 100 substeps (four 25-substep control steps, each
        replayed from a captured hipGraph as the benchmark runs them) of
        sampled scenes (the first, the last, the largest, the smallest)
        against the oracle run on each alone (the scenes are independent),
        1e-3 dx; every scene's state stays finite and inside its grid;
      - the per-substep grid-momentum bar (1e-5) on 16 sampled scenes at
        substep 1 (a handed-in state with seeded C, F), at substep 25
        (the state the GPU reached, read back for the oracle), and for the
        P2G inside the fused launch (substep 2 of a two-substep call,
        against the oracle's P2G of the state separate launches reach after
        one substep from the same start);
  * cfg4, the 1,048,576-particle heap on a 128^3 grid with 3 colliders,
    block 4, chunk 8192, re-sort every 10, fused launches: every particle
    after 100 substeps (graph replay, ten sorts in the run) against the
    oracle, 1e-3 dx; grid momentum at substeps 1, 2 (fused) and 25.
"""
import numpy as np
import pytest

from gpu_util import announce, momentum_floor, random_state, rel_l2
from paper_2302_04659_amd import scenes

pytestmark = pytest.mark.gpu

CFG3_LAUNCH = dict(block=8, chunk=8192, sort_every=100, fuse=1)
CFG4_LAUNCH = dict(block=4, chunk=8192, sort_every=10, fuse=1)


@pytest.fixture(scope="module")
def mpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2302_04659_amd import mpm as m
    m.lib()
    return m


def _sim(mpm, batch, launch, graph=1, capture=0, fuse=None):
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, launch["block"])
    sim.set_option(mpm.OPT_CHUNK, launch["chunk"])
    sim.set_option(mpm.OPT_SORT_EVERY, launch["sort_every"])
    sim.set_option(mpm.OPT_FUSE, launch["fuse"] if fuse is None else fuse)
    sim.set_option(mpm.OPT_GRAPH, graph)
    sim.set_option(mpm.OPT_CAPTURE_GRID, capture)
    return sim


def _grid_momentum(sim, orc, batch, sample, states, what):
    worst = 0.0
    for s in sample:
        sc = batch[s]
        x, v, C, F = states[s]
        om, op = orc.Oracle(sc, x=x, v=v, C=C, F=F).p2g()
        gm, gp = sim.get_grid(s)
        assert rel_l2(gm, om) <= 1e-6, (what, s)
        worst = max(worst, rel_l2(gp, op, momentum_floor(sc, om.sum())))
    print(what, "worst grid momentum rel err", worst)
    assert worst <= 1e-5, (what, worst)


def _c18_at_1_and_25(mpm, orc, batch, sample, launch):
    states = {}
    xs, vs, Cs, Fs = [], [], [], []
    for s, sc in enumerate(batch):
        C, F = random_state(sc, 500 + s, c_scale=2.0, f_scale=0.05)
        xs.append(sc.x), vs.append(sc.v), Cs.append(C), Fs.append(F)
        if s in sample:
            states[s] = (sc.x, sc.v, C, F)
    start = [np.concatenate(a) for a in (xs, vs, Cs, Fs)]
    # the P2G inside the fused launch: substep 2 of a two-substep call, against the oracle's P2G
    # of the state separate launches reach after one substep
    ref = _sim(mpm, batch, launch, graph=0, fuse=0)
    ref.set_state(*start)
    ref.set_colliders_ctrl(0)
    ref.step(1)
    assert ref.sync() == mpm.OK
    after_one = {s: ref.get_state(s) for s in sample}
    ref.close()
    fused = _sim(mpm, batch, launch, graph=0, capture=1, fuse=1)
    fused.set_option(mpm.OPT_TIMING, 1)
    fused.set_state(*start)
    fused.set_colliders_ctrl(0)
    fused.timing(reset=True)
    fused.step(2)
    assert fused.sync() == mpm.OK
    assert fused.timing(reset=True)["g2p2g"][1] == 1
    _grid_momentum(fused, orc, batch, sample, after_one, "substep 2 (fused P2G)")
    fused.close()

    sim = _sim(mpm, batch, launch, graph=0, capture=1)
    sim.set_state(*start)
    sim.set_colliders_ctrl(0)
    sim.step(1)
    assert sim.sync() == mpm.OK
    _grid_momentum(sim, orc, batch, sample, states, "substep 1")
    sim.step(23)
    assert sim.sync() == mpm.OK
    states = {s: sim.get_state(s) for s in sample}
    sim.step(1)
    assert sim.sync() == mpm.OK
    _grid_momentum(sim, orc, batch, sample, states, "substep 25")
    sim.close()


def test_cfg3_full_batch_100_substeps(mpm, orc):
    batch = scenes.cfg3(n_ctrl=4)
    counts = np.array([sc.n for sc in batch])
    announce("full-size cfg3, 100 substeps", len(batch), "scenes", int(counts.sum()), "particles")
    sim = _sim(mpm, batch, CFG3_LAUNCH)
    sim.run_schedule(4)
    assert sim.sync() == mpm.OK
    sample = sorted({0, len(batch) - 1, int(counts.argmax()), int(counts.argmin())})
    for s in sample:
        sc = batch[s]
        o = orc.Oracle(sc)
        o.run_schedule(4)
        x, v, C, F = sim.get_state(s)
        err = np.abs(x - o.x).max() / sc.dx
        print("cfg3 scene", s, "n", sc.n, "max |dx| / dx after 100 substeps", err,
              "rms", np.sqrt(((x - o.x) ** 2).sum(1).mean()) / sc.dx)
        assert err <= 1e-3
    x_all, *_ = sim.get_state(-1)
    assert np.all(np.isfinite(x_all))
    lo = np.repeat([sc.dx for sc in batch], counts)[:, None]
    assert np.all(x_all >= 0.0) and np.all(x_all <= 64 * lo)
    sim.close()


def test_cfg3_full_batch_grid_momentum(mpm, orc):
    batch = scenes.cfg3(n_ctrl=2)
    counts = np.array([sc.n for sc in batch])
    announce("full-size cfg3, grid momentum", len(batch), "scenes", int(counts.sum()), "particles")
    sample = sorted(set(range(0, 256, 17)) | {int(counts.argmax())})
    _c18_at_1_and_25(mpm, orc, batch, sample, CFG3_LAUNCH)


def test_cfg4_full_scene_100_substeps(mpm, orc):
    sc = scenes.cfg4(n_ctrl=4)
    announce("full-size cfg4, 100 substeps", sc.n, "particles")
    sim = _sim(mpm, [sc], CFG4_LAUNCH)
    sim.run_schedule(4)
    assert sim.sync() == mpm.OK
    o = orc.Oracle(sc)
    o.run_schedule(4)
    x, v, C, F = sim.get_state(0)
    err = np.abs(x - o.x).max() / sc.dx
    print("cfg4 max |dx| / dx after 100 substeps:", err, "rms", np.sqrt(((x - o.x) ** 2).sum(1).mean()) / sc.dx)
    assert err <= 1e-3
    sim.close()


def test_cfg4_full_scene_grid_momentum(mpm, orc):
    sc = scenes.cfg4(n_ctrl=2)
    announce("full-size cfg4, grid momentum", sc.n, "particles")
    _c18_at_1_and_25(mpm, orc, [sc], [0], CFG4_LAUNCH)
