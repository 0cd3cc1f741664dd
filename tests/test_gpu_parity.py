"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (from the method's own tolerances):
  * grid momentum of one P2G from identical FP32 inputs:
      |p_gpu - p_orc|_2 / max(|p_orc|_2, sum m |g| dt) <= 1e-5
  * particle positions after 100 free-running substeps: max |dx| <= 1e-3 dx
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


def _teacher_scenes():
    return [
        ("small-nh", scenes.small_scene(1, n=3000, res=16, model=scenes.NEO_HOOKEAN)),
        ("small-hencky", scenes.small_scene(2, n=3000, res=16, model=scenes.HENCKY_VM)),
        ("small-fluid", scenes.small_scene(5, n=3000, res=16, model=scenes.FLUID)),
        ("cfg1b", scenes.cfg1b()),
        ("cfg2", scenes.cfg2()),
    ]


@pytest.mark.parametrize("name,idx", [(n, i) for i, (n, _) in enumerate(_teacher_scenes())])
@pytest.mark.parametrize("block", [4, 8])
def test_teacher_forced_p2g_and_substep(mpm, orc, name, idx, block):
    sc = _teacher_scenes()[idx][1]
    announce("teacher-forced", name, "B", block, "n", sc.n)
    C, F = random_state(sc, 10 + idx, c_scale=2.0, f_scale=0.05)
    sim = mpm.Sim([sc])
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CAPTURE_GRID, 1)
    sim.set_state(sc.x, sc.v, C, F)
    o = orc.Oracle(sc, x=sc.x, v=sc.v, C=C, F=F)
    if sc.n_colliders:
        sim.set_colliders_ctrl(0)
        o.set_colliders(sc.ctrl_poses[0], sc.ctrl_vels[0])
    sim.step(1)
    sim.sync()
    gm, gp = sim.get_grid(0)
    om, op = o.p2g()
    floor = momentum_floor(sc, om.sum())
    assert rel_l2(gm, om) <= 1e-6
    err_p = rel_l2(gp, op, floor)
    print(name, "grid momentum rel err", err_p)
    assert err_p <= 1e-5
    o.grid_op()
    o.g2p()
    x, v, Cg, Fg = sim.get_state(0)
    dx = sc.dx
    assert np.abs(x - o.x).max() <= 1e-4 * dx
    vs = max(np.abs(o.v).max(), 1e-3)
    assert np.abs(v - o.v).max() <= 1e-4 * vs
    assert np.abs(Fg - o.F).max() <= 1e-5
    cs = max(np.abs(o.C).max(), 1e-3)
    assert np.abs(Cg - o.C).max() <= 1e-3 * cs
    sim.close()


def _c18_batch(which):
    if which == "cfg2":
        return [scenes.cfg2(n_ctrl=2)]
    return scenes.cfg3(n_scenes=16, n_ctrl=2)      # the first 16 scenes of the batched workload


def _c18_check(sim, orc, batch, states, what):
    """Grid momentum of the last P2G of every scene against the oracle's P2G
    of the same particle state (c18 bar)."""
    worst = 0.0
    for s, sc in enumerate(batch):
        x, v, C, F = states[s]
        o = orc.Oracle(sc, x=x, v=v, C=C, F=F)
        om, op = o.p2g()
        gm, gp = sim.get_grid(s)
        assert rel_l2(gm, om) <= 1e-6, (what, s)
        err = rel_l2(gp, op, momentum_floor(sc, om.sum()))
        worst = max(worst, err)
    print(what, "worst grid momentum rel err", worst)
    assert worst <= 1e-5, (what, worst)


@pytest.mark.parametrize("which", ["cfg2", "cfg3x16"])
@pytest.mark.parametrize("block,chunk,wg", [(4, 512, 256), (4, 2048, 256), (4, 8192, 256), (8, 512, 256),
                                            (8, 2048, 256), (8, 8192, 256), (4, 2048, 512), (8, 8192, 512)])
def test_grid_momentum_every_launch_config(mpm, orc, which, block, chunk, wg):
    """The per-substep grid-momentum bar at every block edge and chunk size
    the autotuner can pick, with both workgroup sizes (the fixed-point scale of P2G depends on the
    work item's particle count): the first P2G after a re-sort, from a
    handed-in state (seeded C, F; scale bound from the sort), and the P2G of
    the next substep (scale bound from the G2P that wrote the state, which is
    read back for the oracle)."""
    batch = _c18_batch(which)
    announce("grid momentum", which, "B", block, "chunk", chunk, "wg", wg, "n", sum(sc.n for sc in batch))
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CHUNK, chunk)
    sim.set_option(mpm.OPT_WG, wg)
    sim.set_option(mpm.OPT_CAPTURE_GRID, 1)
    states = []
    for s, sc in enumerate(batch):
        C, F = random_state(sc, 70 + s, c_scale=2.0, f_scale=0.05)
        states.append((sc.x, sc.v, C, F))
    sim.set_state(np.concatenate([st[0] for st in states]), np.concatenate([st[1] for st in states]),
                  np.concatenate([st[2] for st in states]), np.concatenate([st[3] for st in states]))
    sim.set_colliders_ctrl(0)
    sim.step(1)
    assert sim.sync() == mpm.OK
    _c18_check(sim, orc, batch, states, "after sort")
    states = [sim.get_state(s) for s in range(len(batch))]
    sim.step(1)
    assert sim.sync() == mpm.OK
    _c18_check(sim, orc, batch, states, "bound from G2P")
    sim.close()


@pytest.mark.parametrize("name", ["cfg1", "cfg1b", "cfg2", "small-hencky", "small-sticky", "small-fluid"])
def test_free_running_100(mpm, orc, name):
    if name == "small-hencky":
        sc = scenes.small_scene(3, n=4000, res=32, model=scenes.HENCKY_VM, n_ctrl=4, dt=1e-4)
    elif name == "small-fluid":
        sc = scenes.small_scene(6, n=4000, res=32, model=scenes.FLUID, n_ctrl=4, dt=1e-4, omega=2.0)
    elif name == "small-sticky":
        sc = scenes.small_scene(4, n=4000, res=32, model=scenes.NEO_HOOKEAN, n_ctrl=4, dt=1e-4,
                                friction=float("inf"), omega=2.0)
    else:
        sc = scenes.WORKLOADS[name]()
    announce("free-running 100", name, "n", sc.n)
    sim = mpm.Sim([sc])
    o = orc.Oracle(sc)
    sim.run_schedule(4)
    o.run_schedule(4)
    st = sim.sync()
    assert st == mpm.OK
    x, v, C, F = sim.get_state(0)
    err = np.abs(x - o.x).max() / sc.dx
    print(name, "max position error / dx after 100 substeps:", err,
          "rms", np.sqrt(((x - o.x) ** 2).sum(1).mean()) / sc.dx)
    assert err <= 1e-3
    if name == "cfg1":      # ballistic closed form
        n = 100
        g = np.array(sc.gravity)
        x_exp = sc.x.astype(np.float64) + g * sc.dt ** 2 * n * (n + 1) / 2
        assert np.abs(x - x_exp).max() <= 1e-3 * sc.dx
        assert np.abs(F - np.eye(3)).max() <= 1e-5
    sim.close()


def _morton(x, y, z):
    out = 0
    for bit in range(10):
        out |= ((x >> bit) & 1) << (3 * bit) | ((y >> bit) & 1) << (3 * bit + 1) | ((z >> bit) & 1) << (3 * bit + 2)
    return out


@pytest.mark.parametrize("block", [4, 8])
def test_sort_order_is_valid(mpm, block):
    """Internal order right after a re-sort: a permutation, scene segments
    kept, Morton codes of the particles' blocks non-decreasing per scene.
    (Equal keys may come in any order; only the key sequence is unique.)"""
    batch = [scenes.small_scene(s, n=500 + 300 * s, res=32) for s in range(4)]
    announce("sort order", len(batch), "B", block)
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, block)
    x0 = np.concatenate([sc.x for sc in batch])
    v0 = np.concatenate([sc.v for sc in batch])
    n = x0.shape[0]
    sim.set_state(x0, v0, np.zeros((n, 3, 3)), np.tile(np.eye(3), (n, 1, 1)))
    sim.step(1)                      # the step starts with the re-sort
    sim.sync()
    pid = sim.order()
    assert np.array_equal(np.sort(pid), np.arange(sim.N))
    for s, sc in enumerate(batch):
        lo, hi = sim.offsets[s], sim.offsets[s + 1]
        seg = pid[lo:hi]
        assert seg.min() >= lo and seg.max() < hi
        base = np.clip(np.floor(x0[seg].astype(np.float64) * sc.res - 0.5).astype(int), 0, sc.res - 3)
        blk = base // block
        keys = np.array([_morton(*b) for b in blk])
        assert (np.diff(keys) >= 0).all()
    sim.close()


def test_batched_equals_single(mpm, orc):
    """Scenes in one batch evolve exactly as when simulated alone (to FP32
    reorder tolerance) and match the oracle; includes an empty scene."""
    batch = [scenes.small_scene(10 + s, n=800 * (s + 1), res=16 * (1 + s % 2)) for s in range(3)]
    empty = scenes.small_scene(99, n=1, res=16, colliders=False)
    empty.x = np.zeros((0, 3), np.float32)
    empty.v = np.zeros((0, 3), np.float32)
    batch.insert(1, empty)
    announce("batched", len(batch))
    sim = mpm.Sim(batch)
    sim.run_schedule(2)
    assert sim.sync() == mpm.OK
    for s, sc in enumerate(batch):
        if sc.n == 0:
            continue
        o = orc.Oracle(sc)
        o.run_schedule(2)
        x, _, _, _ = sim.get_state(s)
        assert np.abs(x - o.x).max() <= 1e-3 * sc.dx, s
    sim.close()


RAGGED_COUNTS = (1, 2, 63, 64, 65, 127, 129, 255, 257, 700)


@pytest.mark.parametrize("block,chunk", [(4, 64), (8, 96)])
@pytest.mark.parametrize("graph", [0, 1])
def test_ragged_items_match_oracle(mpm, orc, block, chunk, graph):
    """Work items of every awkward size: scenes of 1 to 700 particles, split
    into chunks of 64 or 96, give items that end inside a wave, on a wave
    boundary and inside a workgroup's last wave (the G2P batch loop, its LDS
    prefetch of the next batch and the tile staging all see partial waves),
    eager and graph-replayed, against the oracle after two control steps."""
    batch = [scenes.small_scene(200 + k, n=n, res=16, model=k % 2, n_ctrl=2) for k, n in enumerate(RAGGED_COUNTS)]
    announce("ragged items", "B", block, "chunk", chunk, "graph", graph, "counts", RAGGED_COUNTS)
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CHUNK, chunk)
    sim.set_option(mpm.OPT_GRAPH, graph)
    sim.run_schedule(2)
    assert sim.sync() == mpm.OK
    for s, sc in enumerate(batch):
        o = orc.Oracle(sc)
        o.run_schedule(2)
        x, _, _, _ = sim.get_state(s)
        err = np.abs(x - o.x).max() / sc.dx
        assert err <= 1e-3, (sc.n, err)
    sim.close()


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("block,chunk,sort_every", [(4, 1024, 25), (8, 512, 1), (8, 256, 25), (4, 256, 7)])
def test_launch_modes_match_oracle(mpm, orc, persistent, block, chunk, sort_every):
    """Every launch configuration (one cooperative launch or three launches
    per substep, block edge, chunk size, sort cadence) matches the oracle on
    a batch of uneven scenes."""
    batch = [scenes.small_scene(20 + s, n=600 * (1 + s), res=32, model=s % 2, n_ctrl=2, dt=1e-4) for s in range(3)]
    announce("modes", "persistent", persistent, "B", block, "chunk", chunk, "sort_every", sort_every)
    sim = mpm.Sim(batch)
    sim.set_option(mpm.OPT_PERSISTENT, persistent)
    sim.set_option(mpm.OPT_BLOCK, block)
    sim.set_option(mpm.OPT_CHUNK, chunk)
    sim.set_option(mpm.OPT_SORT_EVERY, sort_every)
    sim.run_schedule(2)
    assert sim.sync() == mpm.OK
    for s, sc in enumerate(batch):
        o = orc.Oracle(sc)
        o.run_schedule(2)
        x, v, _, _ = sim.get_state(s)
        assert np.abs(x - o.x).max() <= 1e-3 * sc.dx, (s, np.abs(x - o.x).max() / sc.dx)
    sim.close()


@pytest.mark.parametrize("contact", [0, 2])
def test_one_launch_substep_matches_three_launches(mpm, orc, contact):
    """The one-launch substep (MPM_OPT_PERSISTENT: one cooperative kernel,
    grid-wide barriers between P2G, grid update and G2P) queues exactly one
    kernel per substep and gives what the three launches give (to FP32
    reorder tolerance), with grid-node contact and with penalty contact too,
    and the collider wrench sums agree."""
    batch = [scenes.small_scene(90 + s, n=1500 + 700 * s, res=32, model=scenes.HENCKY_VM, n_ctrl=2, dt=1e-4)
             for s in range(3)]
    announce("one-launch substep, contact", contact)
    out = []
    for persistent in (0, 1):
        sim = mpm.Sim(batch)
        sim.set_option(mpm.OPT_CONTACT, contact)
        sim.set_option(mpm.OPT_FUSE, 0)   # the three launches of a substep on the other side
        sim.set_option(mpm.OPT_PERSISTENT, persistent)
        sim.set_option(mpm.OPT_TIMING, 1)
        sim.timing(reset=True)
        sim.run_schedule(2)
        assert sim.sync() == mpm.OK
        kt = sim.timing(reset=True)
        if persistent:
            assert kt["persistent"][1] == 50 and kt["p2g"][1] == 0 and kt["g2p"][1] == 0
        out.append((sim.get_state(-1), sim.collider_wrenches()))
        sim.close()
    (s0, w0), (s1, w1) = out
    assert np.abs(s0[0] - s1[0]).max() <= 1e-4 * batch[0].dx
    assert np.abs(w0 - w1).max() <= 1e-3 * max(np.abs(w0).max(), 1e-12)
    x1 = s1[0]
    off = np.cumsum([0] + [sc.n for sc in batch])
    for s, sc in enumerate(batch):
        o = orc.Oracle(sc, contact=contact)
        o.run_schedule(2)
        assert np.abs(x1[off[s]:off[s + 1]] - o.x).max() <= 1e-3 * sc.dx, s


def test_nonfinite_state_is_reported(mpm):
    """A non-finite state handed in is refused (host x / v: MPM_ERR_ARG) or
    reported by the next sync (C, F: MPM_ERR_NONFINITE), and a clean state
    clears the report; no substep runs on the broken state."""
    sc = scenes.small_scene(300, n=500, res=16)
    announce("non-finite state", sc.n)
    sim = mpm.Sim([sc])
    x, v, C, F = sim.get_state(-1)
    bad_x = x.copy()
    bad_x[11, 1] = np.nan
    with pytest.raises(mpm.MPMError) as e:
        sim.set_state(bad_x, v, C, F)
    assert e.value.status == mpm.ERR_ARG
    for which, val in (("C", np.nan), ("F", np.inf)):
        C2, F2 = C.copy(), F.copy()
        (C2 if which == "C" else F2)[7, 1, 2] = val
        sim.set_state(x, v, C2, F2)
        with pytest.raises(mpm.MPMError) as e:
            sim.sync()
        assert e.value.status == mpm.ERR_NONFINITE, which
    sim.set_state(x, v, C, F)
    assert sim.sync() == mpm.OK
    sim.close()


def test_graph_replays_match_eager(mpm, orc):
    """25-substep control steps replayed from captured hipGraphs (with eager
    work and host syncs between replays) match the eager path after every
    replay, and the oracle at the end."""
    batch = [scenes.small_scene(40 + s, n=1500 + 500 * s, res=32, model=scenes.HENCKY_VM, n_ctrl=6, dt=1e-4)
             for s in range(3)]
    announce("graph replays", len(batch))
    eager = mpm.Sim(batch)
    graph = mpm.Sim(batch)
    graph.set_option(mpm.OPT_GRAPH, 1)
    for k in range(6):
        for sim in (eager, graph):
            sim.set_colliders_ctrl(k)
            sim.step(25)
        assert graph.sync() == mpm.OK and eager.sync() == mpm.OK
        xe, ve, _, _ = eager.get_state(-1)
        xg, vg, _, _ = graph.get_state(-1)
        assert np.abs(xe - xg).max() <= 1e-4 * batch[0].dx, k
        if k == 2:
            # eager work between replays: a state round trip forces a re-sort
            x, v, C, F = graph.get_state(-1)
            graph.set_state(x, v, C, F)
            x, v, C, F = eager.get_state(-1)
            eager.set_state(x, v, C, F)
    for s, sc in enumerate(batch):
        o = orc.Oracle(sc)
        o.run_schedule(6)
        x, _, _, _ = graph.get_state(s)
        assert np.abs(x - o.x).max() <= 1e-3 * sc.dx
    eager.close()
    graph.close()


def test_autotune_keeps_state(mpm, tmp_path, monkeypatch):
    """The autotuner's trials (block edge x chunk x sort cadence x separate or
    fused launches, then the workgroup size) leave the particle state as it was; the tuning is cached
    for the process and in a file, so that a second process on the same
    kind of workload gets it without trials."""
    import json
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MPM_AUTOTUNE_CACHE", str(cache))
    batch = [scenes.small_scene(60 + s, n=3000, res=32, n_ctrl=2, dt=1e-4) for s in range(4)]
    announce("autotune", len(batch))
    sim = mpm.Sim(batch)
    sim.set_colliders_ctrl(0)
    sim.step(5)
    before = sim.get_state(-1)
    rep = sim.autotune(5)
    print(rep)
    r = json.loads(rep)
    assert not r["cached"]
    assert {t["wg"] for t in r["trials"]} == {256, 512}
    assert {t["fuse"] for t in r["trials"]} == {0, 1} and r["best"]["fuse"] in (0, 1)
    assert r["best"]["block"] in (4, 8) and r["best"]["chunk"] in (512, 2048, 8192) and r["best"]["wg"] in (256, 512)
    after = sim.get_state(-1)
    for a, b in zip(before, after):
        assert np.abs(a - b).max() <= 1e-6 * max(1.0, np.abs(a).max())
    assert sim.get_option(mpm.OPT_BLOCK) == r["best"]["block"]
    assert sim.get_option(mpm.OPT_WG) == r["best"]["wg"]
    assert sim.get_option(mpm.OPT_FUSE) == r["best"]["fuse"]
    rep2 = json.loads(sim.autotune(5))
    assert rep2["cached"] and rep2["best"] == r["best"]
    sim.step(10)
    assert sim.sync() == mpm.OK
    sim.close()
    assert cache.exists()
    code = ("import json, sys; sys.path.insert(0, %r); from paper_2302_04659_amd import mpm, scenes; "
            "b = [scenes.small_scene(60 + s, n=3000, res=32, n_ctrl=2, dt=1e-4) for s in range(4)]; "
            "sim = mpm.Sim(b); print(sim.autotune(5)); sim.close()" % (str(__import__("pathlib").Path(__file__).parents[1]),))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    r3 = json.loads(out.stdout.strip().splitlines()[-1])
    print(r3)
    assert r3["cached"] and r3["source"] == "file" and r3["best"] == r["best"]


def test_workgroup_sizes_match_oracle(mpm, orc):
    """Both workgroup sizes of the particle kernels (256 and 512 threads) on
    uneven items, against the oracle after two control steps."""
    batch = [scenes.small_scene(80 + s, n=700 * (1 + s), res=32, model=s % 2, n_ctrl=2, dt=1e-4) for s in range(3)]
    for nt in (256, 512):
        announce("workgroup size", nt)
        sim = mpm.Sim(batch)
        sim.set_option(mpm.OPT_WG, nt)
        sim.set_option(mpm.OPT_BLOCK, 8)
        sim.set_option(mpm.OPT_CHUNK, 512)
        sim.run_schedule(2)
        assert sim.sync() == mpm.OK
        for s, sc in enumerate(batch):
            o = orc.Oracle(sc)
            o.run_schedule(2)
            x, *_ = sim.get_state(s)
            assert np.abs(x - o.x).max() <= 1e-3 * sc.dx, (nt, s)
        sim.close()
