"""Seeded synthetic scenes for the soft-body substep (inputs only).

This module draws initial particle positions and velocities, material and
grid parameters, collider shapes and collider trajectories from a seed.  It
holds none of the simulation arithmetic: both the HIP path and the FP64 CPU
oracle read the same float32 arrays produced here, and each computes the
method on its own.

The scenes stand in for the paper's soft-body tasks (Pinch, Write, Fill and
the rest, Sec. 2.1 and App. C.5), whose assets are not available.  They use the
paper's parameter ranges (App. D.3, Table "tab:mpm_param": about 8 particles
per cell, Poisson ratio 0.3) and primitive box / capsule colliders (Sec. 3,
"Rigid-soft Coupling").  Collider poses and velocities are handed over once
per control step of 25 substeps (App. E.3: 25 physics steps per control step),
as Algorithm 1 copies rigid poses once per rigid step.

Workloads:

* ``cfg1``  8,192 particles, 16 per cell stratified, 0.25 m cube 0.1 m above
  the floor, 32^3 grid, dt 1e-4 s, neo-Hookean E 1e4, nu 0.3, rho 1e3.
* ``cfg1b`` the same cube with a seeded rotating + shearing + noisy velocity.
* ``cfg2``  65,536 particles in a 0.4 x 0.2 x 0.4 m slab, 64^3 grid,
  dt 5e-5 s, Hencky + von Mises (E 5e3, nu 0.3, yield 1e3), one box pusher.
* ``cfg3``  256 slabs of 10k-60k particles (log-uniform), 64^3 grids,
  1-2 box/capsule colliders on piecewise-linear trajectories.
* ``cfg4``  1,048,576 particles in a hemispherical heap, 128^3 grid,
  dt 2.5e-5 s, 2 boxes + 1 capsule moving inward.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

BOX = 0
CAPSULE = 1
SDF_VOLUME = 2     # sampled signed distance brick (a mesh collider), trilinear
NEO_HOOKEAN = 0
HENCKY_VM = 1
FLUID = 2          # weakly compressible fluid (Tait pressure, volume-only state)
SUBSTEPS_PER_CTRL = 25


@dataclass
class ColliderShape:
    type: int                       # BOX, CAPSULE or SDF_VOLUME
    half_extents: tuple = (0.0, 0.0, 0.0)   # box, body frame
    radius: float = 0.0             # capsule
    half_length: float = 0.0        # capsule, along body y
    friction: float = 0.5           # Coulomb coefficient; math.inf = sticky
    sdf: object = None              # SDF_VOLUME: float32 [nx][ny][nz] body-frame distances
    sdf_cell: float = 0.0           #   sample spacing (m)
    sdf_origin: tuple = (0.0, 0.0, 0.0)     # body-frame position of sample (0, 0, 0)


@dataclass
class Scene:
    name: str
    x: np.ndarray                   # (N, 3) float32, metres
    v: np.ndarray                   # (N, 3) float32, m/s
    res: int
    dx: float
    dt: float
    gravity: tuple
    bound: int
    model: int
    E: float
    nu: float
    rho: float
    yield_stress: float
    yield_form: int
    particle_volume: float
    colliders: List[ColliderShape] = field(default_factory=list)
    ctrl_poses: np.ndarray = None   # (n_ctrl, K, 7) float32: p xyz, q wxyz
    ctrl_vels: np.ndarray = None    # (n_ctrl, K, 6) float32: v xyz, omega xyz

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_colliders(self) -> int:
        return len(self.colliders)

    @property
    def n_ctrl(self) -> int:
        return 0 if self.ctrl_poses is None else int(self.ctrl_poses.shape[0])


def _yaw_quat(phi: float) -> np.ndarray:
    return np.array([math.cos(phi / 2), 0.0, math.sin(phi / 2), 0.0])


def _trajectory(p0: np.ndarray, q0: np.ndarray, vels: np.ndarray, dt: float):
    """Poses at control-step starts for piecewise-constant velocities.

    ``vels`` is (n_ctrl, 6).  Angular velocities of the generated scenes are
    zero, so the orientation stays ``q0``; the linear part is integrated in
    FP64 over each 25-substep segment, then rounded once to float32.
    """
    n_ctrl = vels.shape[0]
    poses = np.zeros((n_ctrl, 7))
    p = p0.astype(np.float64).copy()
    for k in range(n_ctrl):
        poses[k, :3] = p
        poses[k, 3:] = q0
        p = p + SUBSTEPS_PER_CTRL * dt * vels[k, :3]
    return poses


def _pack(poses_per_col, vels_per_col):
    P = np.stack(poses_per_col, axis=1).astype(np.float32)
    V = np.stack(vels_per_col, axis=1).astype(np.float32)
    return P, V


def cfg1(seed: int = 0, n_ctrl: int = 4) -> Scene:
    """0.25 m cube, 8 x 8 x 8 sub-cubes with 16 stratified points each."""
    rng = np.random.default_rng(seed)
    res, dx = 32, 1.0 / 32
    lo = np.array([0.375, 3 * dx + 0.1, 0.375])
    side, m = 0.25, 8
    h = side / m
    cells = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    pts = (cells[:, None, :] + rng.random((cells.shape[0], 16, 3))) * h + lo
    x = pts.reshape(-1, 3).astype(np.float32)
    v = np.zeros_like(x)
    return Scene("cfg1", x, v, res, dx, 1e-4, (0.0, -9.8, 0.0), 3, NEO_HOOKEAN, 1e4, 0.3, 1e3,
                 0.0, 0, side ** 3 / x.shape[0], [],
                 np.zeros((n_ctrl, 0, 7), np.float32), np.zeros((n_ctrl, 0, 6), np.float32))


def cfg1b(seed: int = 0, n_ctrl: int = 4) -> Scene:
    """cfg1 plus v = w x (x - c) + S (x - c) + 0.01 N(0, 1), |w| = 2, |S|_F = 1."""
    s = cfg1(seed, n_ctrl)
    rng = np.random.default_rng(seed + 7919)
    c = s.x.astype(np.float64).mean(0)
    w = rng.normal(size=3)
    w *= 2.0 / np.linalg.norm(w)
    S = rng.normal(size=(3, 3))
    S = 0.5 * (S + S.T)
    S /= np.linalg.norm(S)
    r = s.x.astype(np.float64) - c
    v = np.cross(w, r) + r @ S.T + 0.01 * rng.normal(size=r.shape)
    return replace(s, name="cfg1b", v=v.astype(np.float32))


def cfg2(seed: int = 0, n_ctrl: int = 20) -> Scene:
    """Plasticine slab pushed by one box moving at a seeded constant speed."""
    rng = np.random.default_rng(seed)
    res, dx = 64, 1.0 / 64
    n = 65536
    lo = np.array([0.3, 3 * dx, 0.3])
    size = np.array([0.4, 0.2, 0.4])
    x = (lo + rng.random((n, 3)) * size).astype(np.float32)
    v = np.zeros_like(x)
    he = (0.05, 0.15, 0.025)
    p0 = np.array([rng.uniform(0.4, 0.6), 3 * dx + 0.15, 0.7 + 0.025 - 0.5 * dx])
    speed = rng.uniform(0.05, 0.2)
    vel = np.tile(np.array([0.0, 0.0, -speed, 0.0, 0.0, 0.0]), (n_ctrl, 1))
    q0 = np.array([1.0, 0.0, 0.0, 0.0])
    P, V = _pack([_trajectory(p0, q0, vel, 5e-5)], [vel])
    return Scene("cfg2", x, v, res, dx, 5e-5, (0.0, -9.8, 0.0), 3, HENCKY_VM, 5e3, 0.3, 1e3,
                 1e3, 0, float(np.prod(size)) / n, [ColliderShape(BOX, he, friction=0.5)], P, V)


def _slab_scene(rng, n: int, name: str, n_ctrl: int) -> Scene:
    res, dx = 64, 1.0 / 64
    floor = 3 * dx
    vol = n / 8.0 * dx ** 3                           # 8 particles per cell
    h = rng.uniform(0.12, 0.2)
    aspect = rng.uniform(1.0, 2.0)
    area = vol / h
    lx = min(math.sqrt(area * aspect), 0.55)
    lz = area / lx
    size = np.array([lx, h, lz])
    centre = np.array([0.5, floor + h / 2, 0.5])
    x = (centre - size / 2 + rng.random((n, 3)) * size).astype(np.float32)
    v = np.zeros_like(x)
    n_col = 1 + int(rng.random() < 0.5)
    shapes, poses, vels = [], [], []
    theta0 = rng.uniform(0, 2 * math.pi)
    for k in range(n_col):
        theta = theta0 + k * math.pi + rng.uniform(-0.5, 0.5)
        d = np.array([math.cos(theta), 0.0, math.sin(theta)])
        reach = min((lx / 2) / max(abs(d[0]), 1e-9), (lz / 2) / max(abs(d[2]), 1e-9))
        if rng.random() < 0.5:
            he = (rng.uniform(0.03, 0.06), rng.uniform(0.08, 0.15), rng.uniform(0.015, 0.03))
            shape = ColliderShape(BOX, he, friction=0.5)
            thick, hy = he[2], he[1]
            phi = math.atan2(-d[0], -d[2])          # body +z faces the slab centre
            q0 = _yaw_quat(phi)
        else:
            r, hl = rng.uniform(0.02, 0.04), rng.uniform(0.05, 0.15)
            shape = ColliderShape(CAPSULE, (0.0, 0.0, 0.0), r, hl, friction=0.5)
            thick, hy = r, hl + r
            q0 = np.array([1.0, 0.0, 0.0, 0.0])
        p0 = centre + d * (reach + thick - 0.5 * dx)
        p0[1] = floor + hy + 0.01
        vel = np.zeros((n_ctrl, 6))
        for j in range(n_ctrl):                       # knots every 25 substeps
            yaw = rng.uniform(-math.pi / 6, math.pi / 6)
            c, s = math.cos(yaw), math.sin(yaw)
            dirn = np.array([c * -d[0] - s * -d[2], 0.0, s * -d[0] + c * -d[2]])
            vel[j, :3] = rng.uniform(0.05, 0.2) * dirn
        shapes.append(shape)
        poses.append(_trajectory(p0, q0, vel, 5e-5))
        vels.append(vel)
    P, V = _pack(poses, vels)
    return Scene(name, x, v, res, dx, 5e-5, (0.0, -9.8, 0.0), 3, HENCKY_VM, 5e3, 0.3, 1e3,
                 1e3, 0, float(np.prod(size)) / n, shapes, P, V)


def cfg3(seed: int = 0, n_scenes: int = 256, n_ctrl: int = 20) -> List[Scene]:
    """Batch of uneven slabs; particle counts log-uniform in [1e4, 6e4]."""
    rng = np.random.default_rng(seed)
    counts = np.rint(np.exp(rng.uniform(math.log(1e4), math.log(6e4), n_scenes))).astype(int)
    return [_slab_scene(np.random.default_rng([seed, e]), int(counts[e]), f"cfg3[{e}]", n_ctrl)
            for e in range(n_scenes)]


def cfg3_counts(seed: int = 0, n_scenes: int = 256) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(1e4), math.log(6e4), n_scenes))).astype(int)


def cfg4(seed: int = 0, n_ctrl: int = 40) -> Scene:
    """1,048,576 particles uniform in a hemisphere on the floor, 3 pushers."""
    rng = np.random.default_rng(seed)
    res, dx = 128, 1.0 / 128
    floor = 3 * dx
    n = 1048576
    vol = n / 8.0 * dx ** 3
    r = (3 * vol / (2 * math.pi)) ** (1 / 3)
    centre = np.array([0.5, floor, 0.5])
    out = np.empty((0, 3))
    while out.shape[0] < n:                           # rejection sampling
        c = rng.uniform(-1, 1, (2 * n, 3))
        c[:, 1] = np.abs(c[:, 1])
        c = c[np.einsum("ij,ij->i", c, c) <= 1.0]
        out = np.concatenate([out, c])
    x = (centre + r * out[:n]).astype(np.float32)
    v = np.zeros_like(x)
    shapes, poses, vels = [], [], []
    theta0 = rng.uniform(0, 2 * math.pi)
    for k in range(3):
        theta = theta0 + 2 * math.pi * k / 3 + rng.uniform(-0.3, 0.3)
        d = np.array([math.cos(theta), 0.0, math.sin(theta)])
        if k < 2:
            he = (rng.uniform(0.04, 0.08), rng.uniform(0.08, 0.12), rng.uniform(0.02, 0.03))
            shape = ColliderShape(BOX, he, friction=0.5)
            thick, hy = he[2], he[1]
            q0 = _yaw_quat(math.atan2(-d[0], -d[2]))
        else:
            rad, hl = rng.uniform(0.02, 0.04), rng.uniform(0.05, 0.1)
            shape = ColliderShape(CAPSULE, (0.0, 0.0, 0.0), rad, hl, friction=0.5)
            thick, hy = rad, hl + rad
            q0 = np.array([1.0, 0.0, 0.0, 0.0])
        yc = floor + hy + 0.01
        surf = math.sqrt(max(r * r - (yc - floor) ** 2, 0.0))
        p0 = centre + d * (surf + thick - 0.5 * dx)
        p0[1] = yc
        vel = np.tile(np.concatenate([-d * rng.uniform(0.05, 0.2), np.zeros(3)]), (n_ctrl, 1))
        shapes.append(shape)
        poses.append(_trajectory(p0, q0, vel, 2.5e-5))
        vels.append(vel)
    P, V = _pack(poses, vels)
    return Scene("cfg4", x, v, res, dx, 2.5e-5, (0.0, -9.8, 0.0), 3, HENCKY_VM, 5e3, 0.3, 1e3,
                 1e3, 0, vol / n, shapes, P, V)


def small_scene(seed: int, n: int = 256, res: int = 16, model: int = HENCKY_VM,
                colliders: bool = True, speed: float = 0.5, omega: float = 0.0,
                friction: float = 0.5, n_ctrl: int = 2, dt: float = 2e-4) -> Scene:
    """A small random blob with optional box + capsule colliders (test input)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / res
    lo, hi = 0.3, 0.7
    x = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    v = (0.3 * rng.normal(size=(n, 3))).astype(np.float32)
    shapes, poses, vels = [], [], []
    if colliders:
        for k, typ in enumerate((BOX, CAPSULE)):
            if typ == BOX:
                shape = ColliderShape(BOX, (0.08, 0.1, 0.05), friction=friction)
            else:
                shape = ColliderShape(CAPSULE, (0.0, 0.0, 0.0), 0.06, 0.08, friction=friction)
            p0 = np.array([0.5 + (0.12 if k == 0 else -0.12), 0.5, 0.5 + 0.05 * k])
            ax = rng.normal(size=3)
            ax /= np.linalg.norm(ax)
            ang = rng.uniform(0, math.pi)
            q0 = np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * ax])
            vel = np.zeros((n_ctrl, 6))
            for j in range(n_ctrl):
                vel[j, :3] = speed * rng.normal(size=3)
                vel[j, 3:] = omega * rng.normal(size=3)
            # orientation changes under omega are integrated by the simulators;
            # the control-step poses handed over here carry q0 unchanged
            shapes.append(shape)
            poses.append(_trajectory(p0, q0, vel, dt))
            vels.append(vel)
        P, V = _pack(poses, vels)
    else:
        P = np.zeros((n_ctrl, 0, 7), np.float32)
        V = np.zeros((n_ctrl, 0, 6), np.float32)
    return Scene(f"small[{seed}]", x, v, res, dx, dt, (0.0, -9.8, 0.0), 3, model, 1e4, 0.3, 1e3,
                 300.0 if model == HENCKY_VM else 0.0, 0, (hi - lo) ** 3 / n, shapes, P, V)


def beaker_sdf(radius: float, height: float, wall: float, cell: float, margin: int = 3):
    """A synthetic container mesh as a sampled SDF brick (stand-in for the
    paper's beakers and buckets, whose meshes are not available): an
    open-top cup along body y, outer radius `radius`, height `height`,
    wall and bottom thickness `wall`, centred on the origin.  The solid is
    the outer capped cylinder minus the inner cavity (a cylinder of radius
    radius - wall from the bottom's top face up through the opening); its
    distance is max(outer, -cavity), sampled every `cell` over a box
    `margin` cells larger than the cup.  Returns (samples float32
    [nx][ny][nz], origin)."""
    ext = np.array([radius, height / 2, radius]) + margin * cell
    n = np.ceil(2 * ext / cell).astype(int) + 1
    origin = -ext
    axes = [origin[a] + cell * np.arange(n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    rho = np.sqrt(X * X + Z * Z)

    def capped(r, y0, y1):
        # signed distance to the solid cylinder rho <= r, y0 <= y <= y1
        dr = rho - r
        dy = np.abs(Y - 0.5 * (y0 + y1)) - 0.5 * (y1 - y0)
        out = np.sqrt(np.maximum(dr, 0) ** 2 + np.maximum(dy, 0) ** 2)
        return out + np.minimum(np.maximum(dr, dy), 0.0)

    outer = capped(radius, -height / 2, height / 2)
    cavity = capped(radius - wall, -height / 2 + wall, height / 2 + 4 * cell)
    return np.maximum(outer, -cavity).astype(np.float32), tuple(float(o) for o in origin)


def pour_scene(seed: int = 0, n: int = 6000, res: int = 32, model: int = FLUID, dt: float = 1e-4,
               n_ctrl: int = 4) -> Scene:
    """Material dropped into a beaker (an SDF-volume collider), the beaker
    sliding and tilting slowly: a seeded stand-in for the Pour / Fill tasks."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / res
    floor = 3 * dx
    R, H, W = 0.16, 0.22, 0.03
    c0 = np.array([0.5, floor + H / 2 + 0.01, 0.5])
    # a column of material above the opening
    x = np.stack([rng.uniform(0.5 - 0.08, 0.5 + 0.08, n), rng.uniform(c0[1] + 0.02, c0[1] + 0.18, n),
                  rng.uniform(0.5 - 0.08, 0.5 + 0.08, n)], 1).astype(np.float32)
    v = np.zeros((n, 3), np.float32)
    v[:, 1] = -0.5
    sdf, origin = beaker_sdf(R, H, W, dx / 2)
    shape = ColliderShape(SDF_VOLUME, friction=0.3, sdf=sdf, sdf_cell=dx / 2, sdf_origin=origin)
    vel = np.zeros((n_ctrl, 6))
    for j in range(n_ctrl):
        vel[j, :3] = 0.05 * rng.normal(size=3)
        vel[j, 1] = 0.0
        vel[j, 3:] = [0.0, 0.0, 0.5 * rng.normal()]
    q0 = np.array([1.0, 0.0, 0.0, 0.0])
    P, V = _pack([_trajectory(c0, q0, vel, dt)], [vel])
    vol = 0.16 * 0.16 * 0.16 / n
    return Scene(f"pour[{seed}]", x, v, res, dx, dt, (0.0, -9.8, 0.0), 3, model, 1e4, 0.3, 1e3,
                 300.0 if model == HENCKY_VM else 0.0, 0, vol, [shape], P, V)


WORKLOADS = {"cfg1": cfg1, "cfg1b": cfg1b, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4}
