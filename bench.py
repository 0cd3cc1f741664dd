"""Throughput of the MLS-MPM substep on one MI355X.

A step is one control step of every scene of the workload: its collider
poses and velocities are handed over, then 25 substeps run (each a re-sort
when due, P2G, grid update and G2P with the return map), replayed from a
captured hipGraph by default.  The timed window therefore holds whole
control steps and the re-sorts that fall in them; the library's own
counters report how many substeps, graph replays, host launches and
re-sorts it actually queued.  Inputs are seeded synthetic scenes already
resident in HBM when the timed region starts.

Prints ONE JSON line: particle-substeps/s, the HBM roofline fraction of the
dominant kernel (its average duration measured with HIP events on the
library's stream over a second, host-launched window of the same length),
and the FP64 CPU oracle timed on a bounded sample of the same workload on
the host cores, single-threaded and on all cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic particle bytes per particle-substep touched by each kernel
# (FP32): P2G reads x, v, A (15 floats); G2P reads x, G (12 floats) and
# writes x, v, A, G (24 floats); the G2P fused with the next substep's P2G
# reads x, G and writes x, G (v and A stay in registers for the scatter).
# Grid bytes (16 B per active node and pass) are left out, so `achieved` is
# a lower bound.
ALG_BYTES = {"p2g": 60.0, "g2p": 144.0, "grid": 0.0, "sort": 0.0, "persistent": 204.0, "g2p2g": 96.0}
# Sources the substep kernels are compiled from: a traffic summary is valid
# only for the exact sources it was measured on.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2302_04659_amd", "csrc", f) for f in
                  ("mpm_kernels.hip", "mpm_device.hpp", "mpm_math.hpp", "mpm_kernels.hpp", "mpm_types.hpp")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def workload(name):
    from paper_2302_04659_amd import scenes
    if name == "cfg3":
        return scenes.cfg3(n_ctrl=64), ("cfg3: 256 independent slabs, 10k-60k particles each (log-uniform, seed 0), "
                                       "64^3 grid per scene, 1-2 box/capsule pushers on piecewise-linear trajectories, "
                                       "Hencky + von Mises (E 5e3, nu 0.3, yield 1e3), dt 5e-5")
    if name == "cfg4":
        return [scenes.cfg4(n_ctrl=64)], ("cfg4: 1,048,576-particle plasticine heap, 128^3 grid, 3 moving SDF colliders, "
                                          "dt 2.5e-5, re-sort every 10 substeps")
    if name == "cfg2":
        return [scenes.cfg2(n_ctrl=64)], "cfg2: 65,536-particle slab pushed by a box, 64^3 grid, dt 5e-5"
    raise SystemExit(f"unknown workload {name}")


def kernel_traffic(kernel, wl):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{wl}_traffic.txt")
    if not os.path.exists(path):
        return None
    src_hash = kernel_source_hash()
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def path_roofline(kt, value):
    """The whole substep path against HBM: its algorithmic particle bytes per
    particle-substep follow from the launch mix of the timed configuration
    (separate P2G + G2P: 204 B; fused runs of 25 substeps: P2G, 24 fused
    launches and G2P = 100.3 B), over the 8 TB/s peak."""
    substeps = kt["grid"][1] + kt["persistent"][1]
    if not substeps:
        return None
    b = sum(ALG_BYTES[k] * kt[k][1] for k in ALG_BYTES) / substeps
    peak = HBM_PEAK_GBS * 1e9 / b
    return {"alg_bytes_per_particle_substep": round(b, 2), "peak_particle_substeps_per_s": peak, "frac": value / peak}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene_list, n_scenes, substeps, n_scenes_1t, substeps_1t):
    """The FP64 oracle on the host cores: all cores on n_scenes x substeps,
    one thread on n_scenes_1t x substeps_1t (each scene set up with its
    first control step's collider poses; set-up not timed)."""
    import oracle
    oracle.build(force=False)
    all_cores = len(os.sched_getaffinity(0))

    def timed(count, steps, threads):
        oracle.set_threads(threads)
        sample = scene_list[:count]
        orcs = [oracle.Oracle(sc) for sc in sample]
        for o, sc in zip(orcs, sample):
            if sc.n_colliders:
                o.set_colliders(sc.ctrl_poses[0], sc.ctrl_vels[0])
        t0 = time.perf_counter()
        for o in orcs:
            o.step(steps)
        dt = time.perf_counter() - t0
        n = sum(sc.n for sc in sample)
        return n * steps / dt, f"{count} scenes of the workload ({n} particles) x {steps} substeps, FP64, {dt:.1f} s wall"

    v_all, s_all = timed(n_scenes, substeps, all_cores)
    v_one, s_one = timed(n_scenes_1t, substeps_1t, 1)
    oracle.set_threads(all_cores)
    return {"value": v_all, "unit": "particle-substeps/s", "cores": all_cores, "kind": "oracle",
            "sample": s_all, "cpu_model": cpu_model(),
            "single_thread": {"value": v_one, "cores": 1, "sample": s_one}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed control steps (25 substeps each)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed control steps before the window")
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--block", type=int, default=0, help="grid block edge (0 = library default / autotuned)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library defaults (block 4, chunk 2048, re-sort every 25) unless given")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: replay each 25-substep control step from a captured hipGraph (the default "
                         "production path), 0: launch every kernel from the host")
    ap.add_argument("--persistent", type=int, default=-1)
    ap.add_argument("--fuse", type=int, default=-1, help="1: G2P and the next P2G in one launch (library default 1)")
    ap.add_argument("--wg", type=int, default=0, help="threads per workgroup of the particle kernels (256, 512)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-scenes", type=int, default=64)
    ap.add_argument("--cpu-substeps", type=int, default=50)
    ap.add_argument("--cpu-scenes-1t", type=int, default=8)
    ap.add_argument("--cpu-substeps-1t", type=int, default=25)
    ap.add_argument("--train-steps", type=int, default=12000, help="surrogate: training steps")
    ap.add_argument("--train-seeds", type=int, default=2000, help="surrogate: cfg2 rollouts generated for training")
    ap.add_argument("--train-blocks", type=int, default=20, help="surrogate: control steps per training rollout")
    ap.add_argument("--eval-scenes", type=int, default=256, help="surrogate: held-out scenes timed")
    ap.add_argument("--error-scenes", type=int, default=16, help="surrogate: held-out scenes judged by the oracle")
    ap.add_argument("--error-blocks", type=int, default=2, help="surrogate: control steps judged per scene")
    ap.add_argument("--gate", type=float, default=1e-3, help="surrogate: residual threshold of the fallback")
    ap.add_argument("--no-surrogate", action="store_true", help="leave the surrogate section out of the default run")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, run a plain device-to-device copy of this many MiB three "
                         "times (the reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(scenes would shard across GPUs with no per-substep exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_04659_amd import mpm
    assert torch.cuda.is_available(), "needs the MI355X"
    torch.cuda.set_device(0)
    if args.workload == "cfg5":
        return bench_surrogate(args)

    scene_list, desc = workload(args.workload)
    sim = mpm.Sim(scene_list)
    N = sim.N
    if args.workload == "cfg4":
        sim.set_option(mpm.OPT_SORT_EVERY, 10)
    if args.block:
        sim.set_option(mpm.OPT_BLOCK, args.block)
    if args.chunk:
        sim.set_option(mpm.OPT_CHUNK, args.chunk)
    if args.sort_every:
        sim.set_option(mpm.OPT_SORT_EVERY, args.sort_every)
    if args.graph >= 0:
        sim.set_option(mpm.OPT_GRAPH, args.graph)
    if args.persistent >= 0:
        sim.set_option(mpm.OPT_PERSISTENT, args.persistent)
    if args.fuse >= 0:
        sim.set_option(mpm.OPT_FUSE, args.fuse)
    if args.wg:
        sim.set_option(mpm.OPT_WG, args.wg)
    tune = None
    if args.autotune and not (args.block or args.chunk or args.sort_every):
        tune = sim.autotune(10)
        if args.workload == "cfg4":
            sim.set_option(mpm.OPT_SORT_EVERY, 10)   # the workload fixes its re-sort cadence

    SUB = 25                      # substeps per control step (one step of the benchmark)
    n_ctrl_avail = max(scene_list[0].n_ctrl, 1)
    ctrl = [0]

    def run(n_steps):
        # one control step: hand over poses / velocities, then 25 substeps
        for _ in range(n_steps):
            sim.set_colliders_ctrl(ctrl[0] % n_ctrl_avail)
            ctrl[0] += 1
            sim.step(SUB)

    run(args.warmup)
    st = sim.sync()
    use_graph = sim.get_option(mpm.OPT_GRAPH) == 1
    # Timed region.  Per-kernel HIP events (library stream) bracket every
    # launch of a host-launched run; graph replays cannot be bracketed, so
    # the kernels are then timed over a second region of the same length.
    sim.set_option(mpm.OPT_TIMING, 0 if use_graph else 1)
    sim.timing(reset=True)
    sim.counters(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    window = sim.counters(reset=True)
    st = sim.sync()
    if use_graph:
        sim.set_option(mpm.OPT_TIMING, 1)
        sim.timing(reset=True)
        run(args.steps)
        sim.sync()
    kt = sim.timing(reset=True)
    sim.set_option(mpm.OPT_TIMING, 0)
    if st < 0:
        raise SystemExit(f"simulation reported status {st}")

    substeps = window["substeps"]
    assert substeps == SUB * args.steps, window
    value = N * substeps / elapsed
    per_launch = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    dom = max(("p2g", "g2p", "grid", "sort", "persistent", "g2p2g"), key=lambda k: kt[k][0])
    dom_ms = per_launch[dom]
    bytes_launch = ALG_BYTES[dom] * N
    achieved = bytes_launch / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else None
    window["sort_ms_per_launch"] = round(per_launch["sort"], 5)
    window["sort_share"] = window["sorts"] * per_launch["sort"] / (elapsed * 1e3)
    out = {
        "metric": "MPM particle-substeps/s at 1 GPU",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "scenes": len(scene_list), "particles": N, "substeps_per_step": SUB,
                   "block": sim.get_option(mpm.OPT_BLOCK), "chunk": sim.get_option(mpm.OPT_CHUNK),
                   "sort_every": sim.get_option(mpm.OPT_SORT_EVERY),
                   "wg": sim.get_option(mpm.OPT_WG), "fuse": sim.get_option(mpm.OPT_FUSE),
                   "graph": sim.get_option(mpm.OPT_GRAPH), "persistent": sim.get_option(mpm.OPT_PERSISTENT)},
        "window": window,
        "kernels_ms_per_launch": {k: round(v, 5) for k, v in per_launch.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": kernel_traffic(dom, args.workload)},
        "path_roofline": path_roofline(kt, value),
    }
    if tune:
        out["autotune"] = tune
    if args.copy_probe_mb:
        nb = args.copy_probe_mb << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy probe: 3 x {nb} bytes device-to-device", file=sys.stderr)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(scene_list, min(args.cpu_scenes, len(scene_list)), args.cpu_substeps,
                                           min(args.cpu_scenes_1t, len(scene_list)), args.cpu_substeps_1t)
    sim.close()
    if args.workload == "cfg3" and not args.no_surrogate and not args.no_cpu:
        torch.cuda.empty_cache()
        out["surrogate"] = surrogate_section(args)
    print(json.dumps(out), flush=True)


def unet_forward_flop(shape, cin: int = 8, cout: int = 4, width: int = 1) -> float:
    """Multiply-add FLOPs (2 per MAC) of one U-Net forward on a (D, H, W) grid."""
    from paper_2302_04659_amd.unet import LAYERS, TAPS
    D, H, W = shape
    level = {"e1": 1, "d1": 8, "e2": 8, "d2": 64, "e3": 64, "u2": 8, "c2": 8, "u1": 1, "c1": 1, "he": 1}
    flop = 0.0
    for name, kind, ci, co, _ in LAYERS:
        ci = cin if ci is None else ci // width
        co = cout if co is None else co // width
        vox = D * H * W / level[name[:2]]
        flop += 2.0 * vox * TAPS[kind] * ci * co
    return flop


def cpu_baseline_surrogate(ev, n_blocks):
    """CPU-baseline leg of the surrogate section: the FP64 oracle run on the
    held-out scenes for n_blocks control steps, timed; returns the timing and
    each block's start state (FP32) and end positions, against which the GPU
    runs are then measured (per-block error, each block from the oracle's
    state)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    orcs = [oracle.Oracle(sc) for sc in ev]
    starts, ends = [], []
    t = 0.0
    for b in range(n_blocks):
        st = []
        for o, sc in zip(orcs, ev):
            o.set_colliders(sc.ctrl_poses[b], sc.ctrl_vels[b])
            st.append([a.astype(np.float32).copy() for a in (o.x, o.v, o.C, o.F)])
        t0 = time.perf_counter()
        for o in orcs:
            o.step(25)
        t += time.perf_counter() - t0
        starts.append(st)
        ends.append([o.x.copy() for o in orcs])
    n = sum(sc.n for sc in ev)
    timing = {"value": n * 25 * n_blocks / t, "unit": "particle-substeps/s", "cores": oracle.threads(),
              "kind": "oracle", "sample": f"{len(ev)} held-out scenes ({n} particles) x {n_blocks} control steps "
                                          f"of 25 substeps, FP64, {t:.1f} s wall"}
    return timing, starts, ends


def surrogate_section(args):
    """The grid U-Net surrogate with its residual gate and plain-MPM fallback,
    through the library's own control step (mpm_surrogate_load +
    mpm_step_blocks), against plain batched MPM on held-out slab-pushing
    scenes: training on rollouts the MPM generates, the speedup over plain
    MPM at the residual gate and without it, the fallback fraction, and the
    per-block position error judged by the FP64 oracle (from the oracle's
    state at the start of every block) beside the predictors without a
    network."""
    import numpy as np
    import torch
    from paper_2302_04659_amd import mpm, scenes, surrogate, unet
    t_start = time.perf_counter()
    gate = args.gate
    train_scenes = [scenes.cfg2(seed=s, n_ctrl=args.train_blocks + 1) for s in range(args.train_seeds)]
    t0 = time.perf_counter()
    data = surrogate.RolloutData(train_scenes, n_blocks=args.train_blocks)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    train_shape = data.shape
    net = unet.UNet(cin=surrogate.CIN, cout=surrogate.COUT, width=1, seed=0)
    t0 = time.perf_counter()
    log = surrogate.train(net, data, steps=args.train_steps, batch=8, lr=1e-3, log_every=max(args.train_steps // 4, 1),
                          tail=0.25)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples = data.n_samples
    del data
    torch.cuda.empty_cache()
    blob = net.export_weights()

    n_blocks = 8                  # control steps timed per side (after one untimed)
    ev = [scenes.cfg2(seed=2000 + s, n_ctrl=n_blocks + 1) for s in range(args.eval_scenes)]
    plain = mpm.Sim(ev)
    plain.autotune(10)            # both sides run the tuned substep configuration
    tuned = {o: plain.get_option(o) for o in (mpm.OPT_BLOCK, mpm.OPT_CHUNK, mpm.OPT_SORT_EVERY)}

    def run(sim, use_surrogate, threshold):
        sim.set_colliders_ctrl(0)
        sim.step_blocks(1, use_surrogate, threshold)     # warm-up (graph capture, buffers)
        sim.sync()
        fb, res = 0, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(1, n_blocks + 1):
            sim.set_colliders_ctrl(b)
            fb += sim.step_blocks(1, use_surrogate, threshold)
            if use_surrogate:
                res.append(sim.surrogate_residuals())
        st = sim.sync()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n_blocks
        if st < 0:
            raise SystemExit(f"simulation reported status {st}")
        return t, fb / (n_blocks * len(ev)), (np.concatenate(res) if res else None)

    plain.set_option(mpm.OPT_GRAPH, 1)
    t_plain, _, _ = run(plain, False, 0.0)
    plain.close()
    out = {}
    for name, thr in (("gate", gate), ("no_fallback", float("inf"))):
        sim = mpm.Sim(ev)
        for o, v in tuned.items():
            sim.set_option(o, v)
        sim.set_option(mpm.OPT_GRAPH, 1)
        sim.surrogate_load(blob)
        out[name] = run(sim, True, thr)
        sim.close()
    t_sur, fb_frac, res = out["gate"]
    t_nofb = out["no_fallback"][0]

    # per-block error against the oracle on a subset of the held-out scenes
    sub = ev[: args.error_scenes]
    cpu, starts, ends = cpu_baseline_surrogate(sub, args.error_blocks)
    R, T = sub[0].res, 25 * sub[0].dt
    err = {k: [] for k in ("surrogate", "surrogate_gated", "no_network", "gravity_only", "zero_update")}
    sim = surrogate.make_sim(sub)
    for o, v in tuned.items():
        sim.set_option(o, v)
    sim.surrogate_load(blob)
    with torch.cuda.stream(sim.torch_stream):
        keep = torch.zeros((len(sub), R, R, R, 4), dtype=torch.float32, device="cuda")
        grav = torch.zeros_like(keep)
        grav[..., 1] = -9.8 * T / 0.2
    torch.cuda.synchronize()
    gs = surrogate.GridSurrogate(sim, net)
    for b in range(args.error_blocks):
        for name in err:
            for s in range(len(sub)):
                sim.set_state(*starts[b][s], scene=s)
            sim.set_colliders_ctrl(b)
            if name == "surrogate":
                sim.step_blocks(1, True, float("inf"))
            elif name == "surrogate_gated":
                sim.step_blocks(1, True, gate)
            elif name == "no_network":
                gs.block_with(keep, fallback=False)
            elif name == "gravity_only":
                gs.block_with(grav, fallback=False)
            torch.cuda.synchronize()
            if sim.sync() < 0:
                raise SystemExit("simulation error in the error run")
            for s, sc in enumerate(sub):
                x = starts[b][s][0] if name == "zero_update" else sim.get_state(s)[0]
                e = np.linalg.norm(x.astype(np.float64) - ends[b][s], axis=1) / sc.dx
                err[name].append((float(e.max()), float(np.sqrt((e ** 2).mean()))))
    sim.close()
    per_block = {k: {"max": max(a for a, _ in v), "rms": float(np.sqrt(np.mean([c * c for _, c in v])))}
                 for k, v in err.items()}
    # the network alone (the same kernels) on the training crop, batch = the timed scenes, event-timed
    D, H, W = train_shape
    with torch.cuda.stream(torch.cuda.Stream()):
        x = torch.zeros((len(ev), D, H, W, surrogate.CIN), dtype=torch.float32, device="cuda")
        y = torch.zeros((len(ev), D, H, W, surrogate.COUT), dtype=torch.float32, device="cuda")
        net.forward(x, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            net.forward(x, out=y)
        e1.record()
        torch.cuda.synchronize()
        t_net = e0.elapsed_time(e1) * 1e-3 / 3
    del x, y
    flop = unet_forward_flop(train_shape) * len(ev)
    return {
        "speedup_at_gate": t_plain / t_sur,
        "timed_control_steps": n_blocks,
        "gate": gate,
        "fallback_fraction_at_gate": fb_frac,
        "speedup_without_fallback": t_plain / t_nofb,
        "plain_ms_per_control_step": t_plain * 1e3,
        "surrogate_ms_per_control_step": t_sur * 1e3,
        "surrogate_no_fallback_ms_per_control_step": t_nofb * 1e3,
        "residual": {"median": float(np.median(res)), "p10": float(np.percentile(res, 10)),
                     "p90": float(np.percentile(res, 90)), "max": float(res.max())},
        "per_block_error_dx": per_block,
        "per_block_error_bar_dx": 2e-2,
        "error_sample": f"{len(sub)} held-out scenes x {args.error_blocks} control steps, each started from the "
                        f"oracle's state; max and RMS over particles of |x - x_oracle| / dx",
        "cpu_baseline": cpu,
        "workload": f"cfg5: grid U-Net (3 levels, 32/64/128, 3^3 convs) on a box around the material; trained "
                    f"{args.train_steps} steps (Adam, batch 8, lr 1e-3 falling linearly to 5e-5 over the last quarter, mass-weighted masked MSE) on {n_samples} samples = "
                    f"{args.train_seeds} cfg2 rollouts x {args.train_blocks} control steps made on the GPU; timed on "
                    f"{len(ev)} held-out cfg2 scenes (65,536 particles, 64^3 each), library control step "
                    f"(mpm_step_blocks), residual gate {gate}",
        "scenes": len(ev), "particles": int(sum(sc.n for sc in ev)), "train_crop": list(train_shape),
        "unet_forward": {"bound": "mfma", "achieved": flop / t_net / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": flop / t_net / 1e12 / 2500.0, "ms": t_net * 1e3,
                         "shape": [len(ev), D, H, W]},
        "train": {"steps": args.train_steps, "seconds": t_train, "data_seconds": t_data, "log": log},
        "substep_config": {"block": tuned[mpm.OPT_BLOCK], "chunk": tuned[mpm.OPT_CHUNK],
                           "sort_every": tuned[mpm.OPT_SORT_EVERY]},
        "wall_s": time.perf_counter() - t_start,
    }


def bench_surrogate(args):
    """cfg5 alone: one JSON line with the surrogate's speedup as the value."""
    sec = surrogate_section(args)
    out = {
        "metric": "surrogate+fallback speedup over plain batched MPM (one control step)",
        "value": sec["speedup_at_gate"],
        "unit": "x",
        "n_gpus": 1,
        "steps": sec["timed_control_steps"],
        "warmup": 1,
        "ms_per_step": sec["surrogate_ms_per_control_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": sec["workload"], "scenes": sec["scenes"], "particles": sec["particles"]},
        "surrogate": sec,
        "cpu_baseline": sec["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
