"""Two-way coupling read-out (Algorithm 1 accumulates the soft body's forces
on the rigid bodies for the rigid step): the impulse and angular impulse
each collider receives from grid-node contact, summed over the substeps,
through mpm_get_collider_wrenches, against the FP64 oracle's sums (which
are pinned by Newton's third law on the CPU).

Bars: per collider, |W_gpu - W_orc| <= 2e-3 |W_orc| + 1e-4 W_ref, W_ref the
largest wrench component of the batch (FP32 sums of thousands of node terms
in either order, and free-running states that differ at 1e-5 dx); with
gravity off and walls out of reach the material's momentum change on the
GPU is minus the colliders' summed impulse to 1e-3.
"""
from dataclasses import replace

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


def _batch(g=True):
    out = []
    for s in range(3):
        sc = scenes.small_scene(400 + s, n=1500 + 700 * s, res=32, model=s % 2, speed=0.6, omega=2.0 * s,
                                n_ctrl=2, dt=1e-4)
        out.append(sc if g else replace(sc, gravity=(0.0, 0.0, 0.0)))
    return out


@pytest.mark.parametrize("block,graph", [(4, 0), (8, 1)])
def test_collider_wrenches_match_oracle(mpm, orc, block, graph):
    batch = _batch()
    announce("collider wrenches", "B", block, "graph", graph, "scenes", len(batch))
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_GRAPH, graph)
    orcs = [orc.Oracle(sc, wrench=True) for sc in batch]
    for k in range(2):
        sim.set_colliders_ctrl(k)
        sim.step(25)
        assert sim.sync() == mpm.OK
        W = sim.collider_wrenches()
        ref = []
        for s, (sc, o) in enumerate(zip(batch, orcs)):
            o.set_colliders(sc.ctrl_poses[k], sc.ctrl_vels[k])
            o.step(25)
            ref.append(o.take_wrench())
        wref = max(np.abs(r).max() for r in ref)
        assert wref > 0.0, "no contact in the test scenes"
        for s, (sc, r) in enumerate(zip(batch, ref)):
            g = W[s, : sc.n_colliders].astype(np.float64)
            err = np.abs(g - r)
            bar = 2e-3 * np.abs(r).max(axis=1, keepdims=True) + 1e-4 * wref
            print("control step", k, "scene", s, "max err / bar", float((err / bar).max()))
            assert (err <= bar).all(), (k, s, g, r)
            assert not W[s, sc.n_colliders:].any()
    # the read resets the sums
    assert not sim.collider_wrenches().any()
    sim.close()


def test_material_momentum_change_is_minus_collider_impulse(mpm):
    """Newton's third law on the GPU path: gravity off, walls out of reach."""
    batch = _batch(g=False)
    announce("coupling momentum balance", len(batch))
    sim = mpm.Sim(batch)
    m = np.array([sc.rho * sc.particle_volume for sc in batch])

    def momentum():
        x, v, C, F = sim.get_state(-1)
        out, b = [], 0
        for s, sc in enumerate(batch):
            out.append(m[s] * v[b: b + sc.n].astype(np.float64).sum(0))
            b += sc.n
        return np.array(out)

    P0 = momentum()
    sim.collider_wrenches()
    sim.run_schedule(2)
    assert sim.sync() == mpm.OK
    J = sim.collider_wrenches().astype(np.float64)
    dP = momentum() - P0
    for s, sc in enumerate(batch):
        Js = J[s, : sc.n_colliders, :3].sum(0)
        print("scene", s, "dP", dP[s], "-J", -Js)
        assert np.abs(Js).max() > 0.0
        assert np.allclose(dP[s], -Js, rtol=0, atol=1e-3 * np.abs(Js).max())
    sim.close()


def test_autotune_leaves_wrenches(mpm):
    batch = _batch()
    announce("wrenches across autotune", len(batch))
    sim = mpm.Sim(batch)
    sim.set_colliders_ctrl(0)
    sim.step(25)
    assert sim.sync() == mpm.OK
    before = sim.collider_wrenches()
    sim.step(10)
    assert sim.sync() == mpm.OK
    mid = sim.collider_wrenches()      # the sums of these 10 substeps, then reset
    sim.autotune(5)
    assert sim.sync() == mpm.OK
    assert not sim.collider_wrenches().any(), "the autotuner's trial substeps leaked into the sums"
    assert np.abs(before).max() > 0.0 and np.abs(mid).max() > 0.0
    sim.close()


@pytest.mark.parametrize("model", [scenes.FLUID, scenes.HENCKY_VM])
def test_sdf_volume_collider_matches_oracle(mpm, orc, model):
    """A mesh collider as a sampled SDF volume (a synthetic beaker, sliding
    and slowly turning) catching material dropped into it: positions after
    four control steps against the oracle (1e-3 dx), and the beaker's
    wrenches per control step (same bar as the analytic colliders)."""
    sc = scenes.pour_scene(seed=3, n=5000, model=model)
    announce("sdf volume", "model", model, "n", sc.n)
    sim = mpm.Sim([sc])
    o = orc.Oracle(sc, wrench=True)
    wmax = 0.0
    for k in range(4):
        sim.set_colliders_ctrl(k)
        sim.step(25)
        o.set_colliders(sc.ctrl_poses[k], sc.ctrl_vels[k])
        o.step(25)
        assert sim.sync() == mpm.OK
        g = sim.collider_wrenches()[0, 0].astype(np.float64)
        r = o.take_wrench()[0]
        wmax = max(wmax, np.abs(r).max())
        assert (np.abs(g - r) <= 2e-3 * np.abs(r).max() + 1e-4 * wmax).all(), (k, g, r)
    x, _, _, _ = sim.get_state(0)
    err = np.abs(x - o.x).max() / sc.dx
    print("sdf volume model", model, "max |dx| / dx after 100 substeps", err, "wrench max", wmax)
    assert err <= 1e-3
    assert wmax > 0.0, "the material never touched the beaker"
    sim.close()


def _approach_scene(seed, model):
    """A box starting 2 mm off a blob's +x face, moving into it at 1 m/s."""
    sc = scenes.small_scene(500 + seed, n=3000, res=32, model=model, n_ctrl=2, dt=1e-4)
    box = scenes.ColliderShape(scenes.BOX, (0.08, 0.12, 0.12), friction=0.5)
    c0 = np.array([float(sc.x[:, 0].max()) + 0.08 + 0.002, 0.5, 0.5])
    vel = np.array([-1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    poses = np.zeros((2, 1, 7), np.float32)
    vels = np.zeros((2, 1, 6), np.float32)
    for k in range(2):
        poses[k, 0, :3] = c0 + vel[:3] * 25 * k * sc.dt
        poses[k, 0, 3] = 1.0
        vels[k, 0] = vel
    return replace(sc, colliders=[box], ctrl_poses=poses, ctrl_vels=vels)


@pytest.mark.parametrize("contact,graph", [(1, 0), (2, 1)])
def test_penalty_contact_matches_oracle(mpm, orc, contact, graph):
    """Particle penalty contact (alone, and with the grid-node projection):
    positions after two control steps (1e-3 dx) and the wrenches per control
    step against the oracle, a box pressing into Hencky and fluid blobs."""
    batch = [_approach_scene(0, scenes.HENCKY_VM), _approach_scene(1, scenes.FLUID)]
    announce("penalty contact", contact, "graph", graph)
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_CONTACT, contact)
    sim.set_option(mpm.OPT_GRAPH, graph)
    assert sim.get_option(mpm.OPT_CONTACT) == contact
    orcs = [orc.Oracle(sc, wrench=True, contact=contact) for sc in batch]
    wmax = 0.0
    for k in range(2):
        sim.set_colliders_ctrl(k)
        sim.step(25)
        assert sim.sync() == mpm.OK
        W = sim.collider_wrenches()
        for s, (sc, o) in enumerate(zip(batch, orcs)):
            o.set_colliders(sc.ctrl_poses[k], sc.ctrl_vels[k])
            o.step(25)
            r = o.take_wrench()[0]
            g = W[s, 0].astype(np.float64)
            wmax = max(wmax, np.abs(r).max())
            print("contact", contact, "step", k, "scene", s, "wrench gpu", g[:3], "oracle", r[:3])
            assert (np.abs(g - r) <= 2e-3 * np.abs(r).max() + 1e-4 * wmax).all(), (k, s, g, r)
    for s, (sc, o) in enumerate(zip(batch, orcs)):
        x, _, _, _ = sim.get_state(s)
        err = np.abs(x - o.x).max() / sc.dx
        print("contact", contact, "scene", s, "max |dx| / dx", err)
        assert err <= 1e-3
    assert wmax > 0.0, "the box never reached the blobs"
    with pytest.raises(mpm.MPMError):
        sim.set_option(mpm.OPT_CONTACT, 3)
    sim.close()


def test_particle_view_is_the_state(mpm):
    """The zero-copy position view (internal order) holds, scene by scene, the
    same positions as the creation-order read-out, after a control step with
    re-sorts."""
    import ctypes as ct
    batch = _batch()
    announce("particle view", len(batch))
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_SORT_EVERY, 7)
    sim.set_colliders_ctrl(0)
    sim.step(25)
    assert sim.sync() == mpm.OK
    px, py, pz, begin = sim.particle_view()
    assert begin[0] == 0 and begin[-1] == sum(sc.n for sc in batch)
    hip = ct.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_int]
    n = int(begin[-1])
    view = np.zeros((3, n), np.float32)
    for a, p in enumerate((px, py, pz)):
        assert hip.hipMemcpy(view[a].ctypes.data, p, 4 * n, 2) == 0    # device to host
    x_all, _, _, _ = sim.get_state(-1)
    off = 0
    for s, sc in enumerate(batch):
        mine = view[:, begin[s]: begin[s + 1]].T
        ref = x_all[off: off + sc.n]
        off += sc.n
        assert mine.shape == ref.shape
        order = lambda a: a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))]
        assert np.array_equal(order(mine), order(ref)), s
    sim.close()
