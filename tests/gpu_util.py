"""Helpers shared by the GPU tests (no simulation arithmetic here)."""
import sys

import numpy as np


def announce(*what):
    """Name the case before any GPU work (so a failing run says which)."""
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, floor=0.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor, 1e-300))


def random_state(scene, seed, c_scale=2.0, f_scale=0.03):
    """Seeded FP32 (C, F) for teacher forcing."""
    rng = np.random.default_rng(seed)
    n = scene.n
    C = (c_scale * rng.normal(size=(n, 3, 3))).astype(np.float32)
    F = (np.eye(3) + f_scale * rng.normal(size=(n, 3, 3))).astype(np.float32)
    return C, F


def momentum_floor(scene, m_total):
    """max(|p|, sum m |g| dt): the floor of the grid-momentum error metric."""
    return m_total * float(np.linalg.norm(scene.gravity)) * scene.dt
