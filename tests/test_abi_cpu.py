"""Host-side checks that need no GPU: the C-ABI library loads and exports
every function the headers under include/ declare, and the seeded scene generators are
reproducible and shaped like the workloads they stand for."""
import os

import numpy as np
import pytest

from paper_2302_04659_amd import scenes


def test_library_exports_every_declared_symbol():
    from paper_2302_04659_amd import mpm
    if not os.path.exists(mpm.LIB_PATH):
        pytest.skip("libmpm_hip.so not built (run __graft_entry__.build())")
    L = mpm.lib()
    names = mpm.declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    from paper_2302_04659_amd import mpm
    if not os.path.exists(mpm.LIB_PATH):
        pytest.skip("libmpm_hip.so not built")
    L = mpm.lib()
    assert L.mpm_status_string(0) == b"ok"
    assert b"invalid" in L.mpm_status_string(-1)
    assert L.mpm_num_scenes(None) == 0


def test_struct_layout_matches_header():
    """ctypes mirrors of the C structs have the C sizes (x86-64 SysV)."""
    from paper_2302_04659_amd import mpm
    import ctypes as ct
    assert ct.sizeof(mpm.Material) == 24
    # int, 3 floats, 3 floats (28), pad to 8, pointer, 3 ints, float, 3 floats (68), pad to 8
    assert ct.sizeof(mpm.ColliderShape) == 72
    assert mpm.ColliderShape.sdf.offset == 32 and mpm.ColliderShape.sdf_origin.offset == 56
    # int, pad, 2 pointers, float, int, 2 floats, 3 floats, int, material(24), int, pad, pointer
    assert ct.sizeof(mpm.SceneDesc) == 4 + 4 + 8 + 8 + 4 + 4 + 8 + 12 + 4 + 24 + 4 + 4 + 8


def test_scene_generators_reproducible():
    a, b = scenes.cfg2(seed=5), scenes.cfg2(seed=5)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.ctrl_poses, b.ctrl_poses)
    c = scenes.cfg2(seed=6)
    assert not np.array_equal(a.x, c.x)


def test_workload_shapes():
    s1 = scenes.cfg1()
    assert s1.n == 8192 and s1.res == 32 and s1.x.dtype == np.float32
    # 16 particles in each of the 8^3 sub-cubes (stratified)
    cell = np.floor((s1.x.astype(np.float64) - [0.375, 3 / 32 + 0.1, 0.375]) / (0.25 / 8)).astype(int)
    _, counts = np.unique(cell, axis=0, return_counts=True)
    assert counts.min() == 16 and counts.max() == 16
    s2 = scenes.cfg2()
    assert s2.n == 65536 and s2.res == 64 and s2.n_colliders == 1
    counts = scenes.cfg3_counts()
    assert len(counts) == 256 and counts.min() >= 1e4 and counts.max() <= 6e4
    assert abs(counts.mean() - 27906) < 0.1 * 27906          # E[N] of log-uniform [1e4, 6e4]
    for sc in scenes.cfg3(n_scenes=8, n_ctrl=2):
        assert 1 <= sc.n_colliders <= 2
        lo = sc.x.min(0)
        assert lo[1] >= 3 * sc.dx - 1e-6                   # resting on the floor plane
        assert (sc.x.max(0) < 1 - 3 * sc.dx).all()


def test_cfg4_heap_shape():
    s = scenes.cfg4(n_ctrl=2)
    assert s.n == 1048576 and s.res == 128 and s.n_colliders == 3
    r = np.linalg.norm(s.x.astype(np.float64) - [0.5, 3 / 128, 0.5], axis=1)
    assert r.max() <= 0.311 and (s.x[:, 1] >= 3 / 128 - 1e-6).all()


def test_bin_scramble_multiplier_is_prime():
    """The sort places the r-th particle of a bin at r * M mod size (or r when
    M divides size): a bijection for every size exactly when M is prime."""
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2302_04659_amd", "csrc", "mpm_kernels.hip")).read()
    M = int(re.search(r"BIN_SCRAMBLE\s*=\s*(\d+)", src).group(1))
    assert M > 2 and all(M % d for d in range(2, int(M ** 0.5) + 1))
    for size in (1, 2, 3, 63, 64, 512, 4097, M, 2 * M):
        mul = M if size % M else 1
        assert len(set((r * mul) % size for r in range(size))) == size


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it exits with a message
    (before touching any device)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr), r.stdout + r.stderr


def test_traffic_summaries_match_current_kernel_sources():
    """The committed HBM-traffic summaries were taken on the kernel sources in
    the tree (else the benchmark reports their traffic as null), and each
    summary's byte total follows from its own counter readings and copy
    calibration."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for kernel, wl in [(k, w) for w in ("cfg3", "cfg4") for k in ("g2p2g", "g2p", "p2g", "grid")]:
        total = bench.kernel_traffic(kernel, wl)
        assert total is not None, f"{kernel} {wl}: summary missing or taken on other kernel sources"
        vals = {}
        for line in open(os.path.join(root, "profiles", f"{kernel}_{wl}_traffic.txt")):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = float(v.split("#")[0]) if k.strip() not in ("kernel", "workload",
                                                                             "kernel_source_sha256_16") else v
        rd = vals["fetch_size_kib_per_dispatch"] * 1024 / vals["copy_probe_fetch_factor"]
        wr = vals["write_size_kib_per_dispatch"] * 1024 / vals["copy_probe_write_factor"]
        assert abs(rd + wr - total) <= 1e-3 * total, (kernel, wl, rd + wr, total)
