"""The fused G2P + next-substep P2G (MPM_OPT_FUSE) against the oracle and
against separate launches.

With the option on, between two re-sorts the library runs P2G, grid,
(G2P2G, grid) x (run - 1), G2P: the fused launch scatters each advanced
particle from registers into the fixed-point LDS tile, with its scale taken
from the state before the move (particles that change base cell or outgrow
the scale go straight into the grid).  Bars as in the other parity tests:
  * grid momentum of the fused P2G against the oracle's P2G of the state the
    preceding G2P produces: |p_gpu - p_orc|_2 / max(|p_orc|_2, sum m |g| dt) <= 1e-5
  * positions after two control steps: max |dx| <= 1e-3 dx against the oracle
"""
import numpy as np
import pytest

from gpu_util import announce, momentum_floor, random_state, rel_l2
from paper_2302_04659_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2302_04659_amd import mpm as m
    m.lib()
    return m


def _batch(which):
    if which == "cfg2":
        return [scenes.cfg2(n_ctrl=2)]
    return scenes.cfg3(n_scenes=16, n_ctrl=2)      # the first 16 scenes of the batched workload


def _configure(mpm, sim, block, chunk, wg, fuse):
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CHUNK, chunk)
    sim.set_option(mpm.OPT_WG, wg)
    sim.set_option(mpm.OPT_FUSE, fuse)


@pytest.mark.parametrize("which", ["cfg2", "cfg3x16"])
@pytest.mark.parametrize("block,chunk,wg", [(4, 512, 256), (4, 8192, 256), (8, 2048, 256), (8, 8192, 256),
                                            (8, 8192, 512), (4, 2048, 512)])
def test_fused_p2g_grid_momentum(mpm, orc, which, block, chunk, wg):
    """c18 for the P2G inside the fused launch: two substeps in one call put
    the second substep's P2G into the G2P2G kernel; its grid (captured before
    the grid update) is compared with the oracle's P2G of the state after one
    substep, which a run of separate launches from the same start writes back."""
    batch = _batch(which)
    announce("fused grid momentum", which, "B", block, "chunk", chunk, "wg", wg, "n", sum(sc.n for sc in batch))
    states = []
    for s, sc in enumerate(batch):
        C, F = random_state(sc, 170 + s, c_scale=2.0, f_scale=0.05)
        states.append((sc.x, sc.v, C, F))
    start = [np.concatenate([st[k] for st in states]) for k in range(4)]

    ref = mpm.Sim(batch)
    _configure(mpm, ref, block, chunk, wg, 0)
    ref.set_state(*start)
    ref.set_colliders_ctrl(0)
    ref.step(1)
    assert ref.sync() == mpm.OK
    after_one = [ref.get_state(s) for s in range(len(batch))]
    ref.close()

    sim = mpm.Sim(batch)
    _configure(mpm, sim, block, chunk, wg, 1)
    sim.set_option(mpm.OPT_CAPTURE_GRID, 1)
    sim.set_option(mpm.OPT_TIMING, 1)
    sim.set_state(*start)
    sim.set_colliders_ctrl(0)
    sim.timing(reset=True)
    sim.step(2)
    assert sim.sync() == mpm.OK
    kt = sim.timing(reset=True)
    assert kt["g2p2g"][1] == 1 and kt["p2g"][1] == 1 and kt["g2p"][1] == 1, kt
    worst = 0.0
    for s, sc in enumerate(batch):
        x, v, C, F = after_one[s]
        o = orc.Oracle(sc, x=x, v=v, C=C, F=F)
        om, op = o.p2g()
        gm, gp = sim.get_grid(s)
        assert rel_l2(gm, om) <= 1e-6, s
        worst = max(worst, rel_l2(gp, op, momentum_floor(sc, om.sum())))
    print(which, "fused P2G worst grid momentum rel err", worst)
    assert worst <= 1e-5
    sim.close()


@pytest.mark.parametrize("contact", [0, 2])
@pytest.mark.parametrize("block,chunk,wg", [(4, 1024, 256), (8, 8192, 512)])
def test_fused_matches_separate_launches(mpm, orc, contact, block, chunk, wg):
    """Two control steps fused and unfused (grid-node contact alone and with
    penalty contact): the same particles and collider wrenches to FP32
    reorder tolerance, both within the bar of the oracle; the fused run
    queues one P2G and one G2P per run of substeps between re-sorts."""
    batch = [scenes.small_scene(300 + s, n=1500 + 900 * s, res=32, model=scenes.HENCKY_VM, n_ctrl=2, dt=1e-4)
             for s in range(3)]
    announce("fused vs separate", "contact", contact, "B", block, "chunk", chunk, "wg", wg)
    out = []
    for fuse in (0, 1):
        sim = mpm.Sim(batch)
        _configure(mpm, sim, block, chunk, wg, fuse)
        sim.set_option(mpm.OPT_CONTACT, contact)
        sim.set_option(mpm.OPT_SORT_EVERY, 20)
        sim.set_option(mpm.OPT_TIMING, 1)
        sim.timing(reset=True)
        sim.run_schedule(2)
        assert sim.sync() == mpm.OK
        kt = sim.timing(reset=True)
        if fuse:
            # 50 substeps with a re-sort before substeps 0, 20 and 40: runs of 20, 5 | 15, 10 (one per call and sort)
            assert kt["p2g"][1] == 4 and kt["g2p"][1] == 4 and kt["g2p2g"][1] == 46, kt
        else:
            assert kt["g2p2g"][1] == 0 and kt["p2g"][1] == 50, kt
        out.append((sim.get_state(-1), sim.collider_wrenches()))
        sim.close()
    (s0, w0), (s1, w1) = out
    # the two summation orders differ by rounding, which the penalty springs amplify (measured up
    # to 1.0e-4 dx with penalty contact); the oracle bar below is the binding one
    assert np.abs(s0[0] - s1[0]).max() <= 3e-4 * batch[0].dx
    assert np.abs(s0[3] - s1[3]).max() <= 1e-3 * max(np.abs(s0[3]).max(), 1.0)
    assert np.abs(w0 - w1).max() <= 1e-3 * max(np.abs(w0).max(), 1e-12)
    off = np.cumsum([0] + [sc.n for sc in batch])
    for s, sc in enumerate(batch):
        o = orc.Oracle(sc, contact=contact)
        o.run_schedule(2)
        assert np.abs(s1[0][off[s]:off[s + 1]] - o.x).max() <= 1e-3 * sc.dx, s


@pytest.mark.parametrize("block", [4, 8])
def test_fused_drift_across_blocks(mpm, orc, block):
    """A run of 100 fused substeps with no re-sort while the material moves
    about two cells: particles leave their work item's tile (scattered
    straight into the grid) and reach grid blocks off the update list (the
    overflow lists, alternating by substep parity), against the oracle."""
    sc = scenes.small_scene(401, n=3000, res=32, model=scenes.HENCKY_VM, n_ctrl=4, dt=2e-4, speed=1.0)
    sc.v = (sc.v + np.array([1.5, -3.0, 2.0], np.float32)).astype(np.float32)
    announce("fused drift", "B", block, "n", sc.n)
    sim = mpm.Sim([sc])
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CHUNK, 512)
    sim.set_option(mpm.OPT_SORT_EVERY, 100)
    sim.set_option(mpm.OPT_GRAPH, 0)
    sim.set_state(sc.x, sc.v, np.zeros((sc.n, 3, 3), np.float32), np.tile(np.eye(3, dtype=np.float32), (sc.n, 1, 1)))
    o = orc.Oracle(sc, x=sc.x, v=sc.v)
    sim.run_schedule(4)
    o.run_schedule(4)
    assert sim.sync() == mpm.OK
    x, _, _, _ = sim.get_state(0)
    moved = np.abs(x - sc.x).max() / sc.dx
    err = np.abs(x - o.x).max() / sc.dx
    print("fused drift: moved", moved, "cells, max error / dx", err)
    assert moved >= 1.5
    assert err <= 1e-3
    sim.close()
