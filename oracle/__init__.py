"""FP64 CPU oracle for the MLS-MPM substep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it.
It shares no code with the HIP path; the only common input is the seeded
scene generator (``paper_2302_04659_amd.scenes``), which holds no
simulation arithmetic.

The arithmetic lives in ``mpm_oracle.c`` (plain C, FP64); this module is a
ctypes binding plus array marshalling.  Build it with ``build()`` (gcc,
``-O2 -fopenmp``).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpm_oracle.c")
LIB = os.path.join(HERE, "_mpm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Collider(ct.Structure):
    _fields_ = [("type", ct.c_int), ("half_extents", ct.c_double * 3), ("radius", ct.c_double),
                ("half_length", ct.c_double), ("friction", ct.c_double), ("pos", ct.c_double * 3),
                ("quat", ct.c_double * 4), ("vlin", ct.c_double * 3), ("omega", ct.c_double * 3),
                ("sdf", ct.POINTER(ct.c_double)), ("sdf_dims", ct.c_int * 3), ("sdf_cell", ct.c_double),
                ("sdf_origin", ct.c_double * 3)]


def set_collider_shape(col, c, keep):
    """Fill a Collider struct from a scene shape; keep holds the FP64 copy
    of a sampled SDF volume alive."""
    col.type = c.type
    col.half_extents[:] = [float(h) for h in c.half_extents]
    col.radius = c.radius
    col.half_length = c.half_length
    col.friction = c.friction
    col.quat[:] = [1.0, 0.0, 0.0, 0.0]
    if getattr(c, "sdf", None) is not None:
        a = np.ascontiguousarray(c.sdf, np.float64)
        keep.append(a)
        col.sdf = _dp(a)
        col.sdf_dims[:] = list(a.shape)
        col.sdf_cell = float(c.sdf_cell)
        col.sdf_origin[:] = [float(o) for o in c.sdf_origin]


class SceneC(ct.Structure):
    _fields_ = [("n", ct.c_int), ("x", ct.POINTER(ct.c_double)), ("v", ct.POINTER(ct.c_double)),
                ("C", ct.POINTER(ct.c_double)), ("F", ct.POINTER(ct.c_double)), ("res", ct.c_int),
                ("dx", ct.c_double), ("dt", ct.c_double), ("g", ct.c_double * 3), ("bound", ct.c_int),
                ("model", ct.c_int), ("E", ct.c_double), ("nu", ct.c_double), ("rho", ct.c_double),
                ("yield_stress", ct.c_double), ("yield_form", ct.c_int), ("p_vol", ct.c_double),
                ("n_col", ct.c_int), ("col", ct.POINTER(Collider)), ("wrench", ct.POINTER(ct.c_double)),
                ("contact", ct.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        dp = ct.POINTER(ct.c_double)
        sp = ct.POINTER(SceneC)
        L.orc_weights.argtypes = [ct.c_double, dp]
        L.orc_svd3.argtypes = [dp, dp, dp, dp]
        L.orc_svd3.restype = ct.c_int
        L.orc_stress.argtypes = [sp, dp, dp]
        L.orc_return_map.argtypes = [sp, dp]
        L.orc_return_map.restype = ct.c_int
        L.orc_sdf.argtypes = [ct.POINTER(Collider), dp, dp]
        L.orc_sdf.restype = ct.c_double
        L.orc_collide.argtypes = [ct.POINTER(Collider), dp, dp]
        L.orc_collide.restype = ct.c_int
        L.orc_affine.argtypes = [sp, dp]
        L.orc_p2g.argtypes = [sp, dp, dp]
        L.orc_p2g.restype = ct.c_int
        L.orc_grid_op.argtypes = [sp, dp, dp, dp]
        L.orc_g2p.argtypes = [sp, dp]
        L.orc_g2p.restype = ct.c_int
        L.orc_advance_colliders.argtypes = [sp]
        L.orc_sur_advance.argtypes = [sp, dp, dp, ct.c_int, ct.c_int]
        L.orc_sur_advance.restype = ct.c_int
        L.orc_step.argtypes = [sp, ct.c_int, dp, dp, dp]
        L.orc_step.restype = ct.c_int
        L.orc_threads.restype = ct.c_int
        L.orc_set_threads.argtypes = [ct.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


class OracleError(RuntimeError):
    pass


class Oracle:
    """One scene held in FP64.  State arrays are numpy views you may edit."""

    def __init__(self, scene, x=None, v=None, C=None, F=None, wrench: bool = False, contact: int = 0):
        n = scene.n
        self.scene = scene
        self.x = np.ascontiguousarray(scene.x if x is None else x, dtype=np.float64).reshape(n, 3).copy()
        self.v = np.ascontiguousarray(scene.v if v is None else v, dtype=np.float64).reshape(n, 3).copy()
        self.C = (np.zeros((n, 3, 3)) if C is None else np.asarray(C, np.float64).reshape(n, 3, 3)).copy()
        self.F = (np.tile(np.eye(3), (n, 1, 1)) if F is None else np.asarray(F, np.float64).reshape(n, 3, 3)).copy()
        self.res = scene.res
        nn = self.res ** 3
        self.gm = np.zeros(nn)
        self.gp = np.zeros((nn, 3))
        self.vg = np.zeros((nn, 3))
        self.cols = (Collider * max(scene.n_colliders, 1))()
        self._sdf_keep = []
        for k, c in enumerate(scene.colliders):
            set_collider_shape(self.cols[k], c, self._sdf_keep)
        # impulse (3) and angular impulse about the centre (3) received by each
        # collider, summed over the grid updates since the last take_wrench()
        self.wrench = np.zeros((max(scene.n_colliders, 1), 6)) if wrench else None
        self.contact = contact    # 0 grid-node projection, 1 particle penalty, 2 both
        self.s = SceneC()
        self._bind()

    def _bind(self):
        sc, s = self.scene, self.s
        s.n = sc.n
        s.x, s.v, s.C, s.F = _dp(self.x), _dp(self.v), _dp(self.C), _dp(self.F)
        s.res, s.dx, s.dt = sc.res, sc.dx, sc.dt
        s.g[:] = list(sc.gravity)
        s.bound, s.model = sc.bound, sc.model
        s.E, s.nu, s.rho = sc.E, sc.nu, sc.rho
        s.yield_stress, s.yield_form = sc.yield_stress, sc.yield_form
        s.p_vol = sc.particle_volume
        s.n_col = sc.n_colliders
        s.col = ct.cast(self.cols, ct.POINTER(Collider))
        s.wrench = _dp(self.wrench) if self.wrench is not None else ct.POINTER(ct.c_double)()
        s.contact = getattr(self, "contact", 0)

    # -- colliders ---------------------------------------------------------
    def set_colliders(self, poses, vels):
        poses = np.asarray(poses, np.float64).reshape(-1, 7)
        vels = np.asarray(vels, np.float64).reshape(-1, 6)
        for k in range(self.scene.n_colliders):
            self.cols[k].pos[:] = poses[k, :3].tolist()
            self.cols[k].quat[:] = poses[k, 3:].tolist()
            self.cols[k].vlin[:] = vels[k, :3].tolist()
            self.cols[k].omega[:] = vels[k, 3:].tolist()

    def take_wrench(self):
        """[n_colliders][6]: impulse on each collider and angular impulse
        about its centre since the last call (then zeroed)."""
        w = self.wrench[: self.scene.n_colliders].copy()
        self.wrench[:] = 0.0
        return w

    def collider_poses(self):
        return np.array([list(c.pos) + list(c.quat) for c in self.cols[: self.scene.n_colliders]]).reshape(-1, 7)

    # -- steps ---------------------------------------------------------------
    def p2g(self):
        e = lib().orc_p2g(ct.byref(self.s), _dp(self.gm), _dp(self.gp))
        if e:
            raise OracleError(f"p2g failed ({e}): particle stencil outside the grid")
        return self.gm.reshape((self.res,) * 3), self.gp.reshape((self.res,) * 3 + (3,))

    def grid_op(self):
        lib().orc_grid_op(ct.byref(self.s), _dp(self.gm), _dp(self.gp), _dp(self.vg))
        return self.vg.reshape((self.res,) * 3 + (3,))

    def g2p(self):
        e = lib().orc_g2p(ct.byref(self.s), _dp(self.vg))
        if e:
            raise OracleError(f"g2p failed ({e}): particle stencil outside the grid")

    def advance_colliders(self):
        lib().orc_advance_colliders(ct.byref(self.s))

    def step(self, n: int = 1):
        e = lib().orc_step(ct.byref(self.s), int(n), _dp(self.gm), _dp(self.gp), _dp(self.vg))
        if e:
            raise OracleError(f"step failed ({e}): particle stencil outside the grid")

    def sur_advance(self, vs, dv, n_sub: int = 25, mode: int = 1):
        """Surrogate control step from a grid prediction: vs, dv [res^3][3]
        (start P2G velocity, predicted change), particles advanced in place
        (mode 1: they take the predicted change; mode 0: the end field)."""
        vs = np.ascontiguousarray(vs, np.float64).reshape(-1, 3)
        dv = np.ascontiguousarray(dv, np.float64).reshape(-1, 3)
        assert vs.shape[0] == self.res ** 3 and dv.shape[0] == self.res ** 3
        e = lib().orc_sur_advance(ct.byref(self.s), _dp(vs), _dp(dv), int(n_sub), int(mode))
        if e:
            raise OracleError(f"sur_advance failed ({e}): particle stencil outside the grid")

    def affine(self):
        A = np.zeros((self.scene.n, 3, 3))
        lib().orc_affine(ct.byref(self.s), _dp(A))
        return A

    def run_schedule(self, n_ctrl: int, substeps: int = 25, ctrl0: int = 0):
        """Hand over the scene's control-step poses/velocities, step each block."""
        sc = self.scene
        for k in range(ctrl0, ctrl0 + n_ctrl):
            if sc.n_colliders:
                self.set_colliders(sc.ctrl_poses[k], sc.ctrl_vels[k])
            self.step(substeps)


# -- surrogate residual ------------------------------------------------------
# Reference velocity of the momentum term: the speed that carries a particle
# across the per-block error bar (2e-2 dx) in one control step.
SUR_ERR_BAR_DX = 2e-2


def sur_residual(scene, m_s, v_s, dm, dv, m_r, p_r, n_sub: int = 25):
    """Self-consistency residual of a surrogate control step, in FP64.

    m_s [res^3], v_s [res^3][3]: mass and P2G velocity at the start of the
    step; dm, dv: the predicted changes; m_r, p_r: a P2G of the particles the
    prediction advanced.  Over the nodes holding material before or after,
        r_m = sum |m_r - (m_s + dm)| / sum m_s,
        r_p = sum |p_r - (m_s + dm) (v_s + dv)|_1 / (sum m_s * u_ref),
    u_ref = SUR_ERR_BAR_DX dx / (n_sub dt); returns (max(r_m, r_p), r_m, r_p).
    """
    m_s = np.asarray(m_s, np.float64).reshape(-1)
    v_s = np.asarray(v_s, np.float64).reshape(-1, 3)
    dm = np.asarray(dm, np.float64).reshape(-1)
    dv = np.asarray(dv, np.float64).reshape(-1, 3)
    m_r = np.asarray(m_r, np.float64).reshape(-1)
    p_r = np.asarray(p_r, np.float64).reshape(-1, 3)
    sel = (m_s > 0) | (m_r > 0)
    m_pred = m_s + dm
    v_end = v_s + dv
    total = m_s.sum()
    if total <= 0:
        return 0.0, 0.0, 0.0
    u_ref = SUR_ERR_BAR_DX * scene.dx / (n_sub * scene.dt)
    r_m = np.abs(m_r - m_pred)[sel].sum() / total
    r_p = np.abs(p_r - m_pred[:, None] * v_end)[sel].sum() / (total * u_ref)
    return max(r_m, r_p), r_m, r_p


def p2g_velocity(m, p):
    """Grid velocity p / m of a P2G output (0 where the mass is 0)."""
    m = np.asarray(m, np.float64).reshape(-1)
    p = np.asarray(p, np.float64).reshape(-1, 3)
    v = np.zeros_like(p)
    nz = m > 0
    v[nz] = p[nz] / m[nz, None]
    return v


# -- single-matrix helpers (pinned by the tests) ----------------------------
def svd3(F):
    F = np.ascontiguousarray(F, np.float64).reshape(3, 3)
    U, S, V = np.zeros((3, 3)), np.zeros(3), np.zeros((3, 3))
    lib().orc_svd3(_dp(F), _dp(U), _dp(S), _dp(V))
    return U, S, V


def _scene_struct(scene):
    o = Oracle.__new__(Oracle)
    o.scene = scene
    n = 1
    o.x = np.zeros((n, 3)); o.v = np.zeros((n, 3)); o.C = np.zeros((n, 3, 3)); o.F = np.zeros((n, 3, 3))
    o.cols = (Collider * 1)()
    o.wrench = None
    o.s = SceneC()
    o._bind()
    return o


def stress(scene, F):
    o = _scene_struct(scene)
    F = np.ascontiguousarray(F, np.float64).reshape(3, 3)
    tau = np.zeros((3, 3))
    lib().orc_stress(ct.byref(o.s), _dp(F), _dp(tau))
    return tau


def return_map(scene, F):
    o = _scene_struct(scene)
    F = np.ascontiguousarray(F, np.float64).reshape(3, 3).copy()
    y = lib().orc_return_map(ct.byref(o.s), _dp(F))
    return F, bool(y)


def weights(f):
    w = np.zeros(3)
    lib().orc_weights(float(f), _dp(w))
    return w


def make_collider(shape, pose, vel=(0, 0, 0, 0, 0, 0)):
    c = Collider()
    c._keep = []     # the FP64 copy of a sampled SDF volume lives as long as the struct
    set_collider_shape(c, shape, c._keep)
    c.pos[:] = [float(p) for p in pose[:3]]
    c.quat[:] = [float(q) for q in pose[3:]]
    c.vlin[:] = [float(a) for a in vel[:3]]
    c.omega[:] = [float(a) for a in vel[3:]]
    return c


def sdf(collider, x):
    x = np.ascontiguousarray(x, np.float64).reshape(3)
    n = np.zeros(3)
    phi = lib().orc_sdf(ct.byref(collider), _dp(x), _dp(n))
    return phi, n


def collide(collider, xi, v):
    xi = np.ascontiguousarray(xi, np.float64).reshape(3)
    v = np.ascontiguousarray(v, np.float64).reshape(3).copy()
    hit = lib().orc_collide(ct.byref(collider), _dp(xi), _dp(v))
    return v, bool(hit)


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from here on (timing)."""
    lib().orc_set_threads(int(n))
