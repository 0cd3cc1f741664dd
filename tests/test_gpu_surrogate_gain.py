"""What the trained surrogate gains over having no network.

A small U-Net (half width) is trained on plain-MPM rollouts of seeded
slab-pushing scenes, handed to the library (mpm_surrogate_load) and run
through its control step (mpm_step_blocks, no fallback), then judged per
control step (25 substeps) against the FP64 oracle on held-out scenes:
every block starts from the oracle's state rounded to FP32, and the error is
the distance of each particle from the oracle's position after the block
(max and RMS, in grid cells).

At these speeds every predictor below stays inside the 2e-2 dx per-block
bar (particles move about 0.016 dx per block), so the bar itself shows no
gain.  The gain criteria are comparisons: the trained network's error (max
and RMS) is below that of
  * the method without the network (no velocity change predicted: the
    particles keep their velocities and move with the start field),
  * the gravity-only predictor (every node's velocity changes by 25 dt g),
  * the zero-update predictor (particles frozen for the block);
and its re-splat residual is below the untrained network's for every scene
and block, so at any gate threshold it falls back no more often.
"""
import numpy as np
import pytest

from gpu_util import announce
from paper_2302_04659_amd import scenes

pytestmark = pytest.mark.gpu

N_TRAIN, N_BLOCKS_TRAIN, STEPS = 8, 6, 300
N_EVAL, N_BLOCKS_EVAL = 2, 3


def test_trained_surrogate_beats_baselines(orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    from paper_2302_04659_amd import surrogate, unet
    announce("surrogate gain: train", N_TRAIN, "x", N_BLOCKS_TRAIN, "steps", STEPS)
    data = surrogate.RolloutData([scenes.cfg2(seed=s) for s in range(N_TRAIN)], n_blocks=N_BLOCKS_TRAIN)
    net = unet.UNet(cin=surrogate.CIN, cout=surrogate.COUT, width=2, seed=0)
    untrained = unet.UNet(cin=surrogate.CIN, cout=surrogate.COUT, width=2, seed=0)
    surrogate.train(net, data, steps=STEPS, batch=8, lr=1e-3, log_every=STEPS)
    del data
    announce("surrogate gain: evaluate", N_EVAL, "x", N_BLOCKS_EVAL)
    ev = [scenes.cfg2(seed=2000 + s) for s in range(N_EVAL)]
    orcs = [orc.Oracle(sc) for sc in ev]
    sim = surrogate.make_sim(ev)
    R = ev[0].res
    T = 25 * ev[0].dt
    with torch.cuda.stream(sim.torch_stream):
        g_pred = torch.zeros((N_EVAL, R, R, R, 4), dtype=torch.float32, device="cuda")
        g_pred[..., 1] = -9.8 * T / 0.2
        keep = torch.zeros((N_EVAL, R, R, R, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    blobs = {"trained": net.export_weights(), "untrained": untrained.export_weights()}
    err = {k: [] for k in ("trained", "no_network", "gravity", "zero")}
    res = {k: [] for k in ("trained", "untrained")}
    gs = surrogate.GridSurrogate(sim, net, chunk=N_EVAL)
    for b in range(N_BLOCKS_EVAL):
        start = []
        for o, sc in zip(orcs, ev):
            o.set_colliders(sc.ctrl_poses[b], sc.ctrl_vels[b])
            start.append([a.astype(np.float32).copy() for a in (o.x, o.v, o.C, o.F)])
        for o in orcs:
            o.step(25)
        for name in ("trained", "untrained", "no_network", "gravity"):
            for s in range(N_EVAL):
                sim.set_state(*start[s], scene=s)
            sim.set_colliders_ctrl(b)
            if name in blobs:
                sim.surrogate_load(blobs[name])
                sim.step_blocks(1, True, float("inf"))
                res[name].append(sim.surrogate_residuals().astype(np.float64))
            else:
                gs.block_with(g_pred if name == "gravity" else keep, fallback=False)
            torch.cuda.synchronize()
            assert sim.sync() >= 0
            if name in err:
                for s in range(N_EVAL):
                    x, *_ = sim.get_state(s)
                    e = np.linalg.norm(x - orcs[s].x, axis=1) / ev[s].dx
                    err[name].append((e.max(), np.sqrt((e ** 2).mean())))
        for s in range(N_EVAL):
            e = np.linalg.norm(start[s][0] - orcs[s].x, axis=1) / ev[s].dx
            err["zero"].append((e.max(), np.sqrt((e ** 2).mean())))
    summary = {k: (float(np.mean([a for a, _ in v])), float(np.mean([c for _, c in v]))) for k, v in err.items()}
    print("per-block error (mean of max, mean of rms) in dx:", summary)
    rt, ru = np.concatenate(res["trained"]), np.concatenate(res["untrained"])
    print("residual trained", rt, "untrained", ru)
    for name in err:
        assert max(a for a, _ in err[name]) <= 2e-2, name
    for base in ("no_network", "gravity", "zero"):
        assert summary["trained"][0] < summary[base][0], base
        assert summary["trained"][1] < summary[base][1], base
    assert np.all(rt < ru)
    sim.close()
