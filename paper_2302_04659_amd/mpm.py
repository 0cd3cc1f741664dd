"""Python binding of libmpm_hip.so (argument marshalling only).

Every step of the substep runs in the library's HIP kernels; this module
builds the C structs, passes host arrays or torch device pointers, and maps
status codes to exceptions.  The library must exist (``__graft_entry__.build``
or ``python -m paper_2302_04659_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
import re
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpm.h")

OK, WARN_CLAMPED, WARN_FALLBACK = 0, 1, 2
ERR_ARG, ERR_HIP, ERR_OOM, ERR_NONFINITE, ERR_STATE = -1, -2, -3, -4, -5
OPT_SORT_EVERY, OPT_BLOCK, OPT_CHUNK, OPT_PERSISTENT, OPT_GRAPH, OPT_CAPTURE_GRID, OPT_TIMING, OPT_CONTACT, OPT_WG, \
    OPT_FUSE = range(10)
K_SORT, K_P2G, K_GRID, K_G2P, K_PERSISTENT, K_G2P2G = range(6)
KERNEL_CLASSES = ("sort", "p2g", "grid", "g2p", "persistent", "g2p2g")
MAX_COLLIDERS = 4


class Material(ct.Structure):
    _fields_ = [("model", ct.c_int), ("E", ct.c_float), ("nu", ct.c_float), ("rho", ct.c_float),
                ("yield_stress", ct.c_float), ("yield_form", ct.c_int)]


class ColliderShape(ct.Structure):
    _fields_ = [("type", ct.c_int), ("half_extents", ct.c_float * 3), ("radius", ct.c_float),
                ("half_length", ct.c_float), ("friction", ct.c_float), ("sdf", ct.POINTER(ct.c_float)),
                ("sdf_dims", ct.c_int * 3), ("sdf_cell", ct.c_float), ("sdf_origin", ct.c_float * 3)]


class SceneDesc(ct.Structure):
    _fields_ = [("n_particles", ct.c_int), ("x", ct.POINTER(ct.c_float)), ("v", ct.POINTER(ct.c_float)),
                ("particle_volume", ct.c_float), ("res", ct.c_int), ("dx", ct.c_float), ("dt", ct.c_float),
                ("gravity", ct.c_float * 3), ("bound", ct.c_int), ("mat", Material), ("n_colliders", ct.c_int),
                ("colliders", ct.POINTER(ColliderShape))]


class MPMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libmpm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_04659_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, fp, ip = ct.c_void_p, ct.POINTER(ct.c_float), ct.POINTER(ct.c_int)
        L.mpm_create.argtypes = [ct.POINTER(SceneDesc), ct.c_int, vp, ct.POINTER(vp)]
        L.mpm_destroy.argtypes = [vp]
        L.mpm_set_colliders.argtypes = [vp, vp, vp, ct.c_int]
        L.mpm_get_collider_wrenches.argtypes = [vp, vp, ct.c_int]
        L.mpm_particle_view.argtypes = [vp, ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(ct.c_int)]
        L.mpm_step.argtypes = [vp, ct.c_int]
        L.mpm_sync.argtypes = [vp]
        L.mpm_get_particles.argtypes = [vp, ct.c_int, vp, vp, vp, ct.c_int]
        L.mpm_get_state.argtypes = [vp, ct.c_int, vp, vp, vp, vp, ct.c_int]
        L.mpm_set_state.argtypes = [vp, ct.c_int, vp, vp, vp, vp, ct.c_int]
        L.mpm_get_grid.argtypes = [vp, ct.c_int, vp, vp, ct.c_int]
        L.mpm_set_option.argtypes = [vp, ct.c_int, ct.c_int]
        L.mpm_get_option.argtypes = [vp, ct.c_int, ip]
        L.mpm_autotune.argtypes = [vp, ct.c_int, ct.c_char_p, ct.c_size_t]
        L.mpm_get_order.argtypes = [vp, vp]
        L.mpm_get_timing.argtypes = [vp, vp, vp, ct.c_int]
        L.mpm_get_counters.argtypes = [vp, vp, ct.c_int]
        L.mpm_set_scene_mask.argtypes = [vp, vp]
        L.mpm_sur_bbox.argtypes = [vp, vp]
        L.mpm_sur_features.argtypes = [vp, vp, ct.c_int, vp, vp, ct.c_int, ct.c_int, ct.c_int]
        L.mpm_sur_block.argtypes = [vp, vp, ct.c_int, vp, vp, ct.c_int, ct.c_int, ct.c_int, ct.c_float, ct.c_int, vp,
                                    vp]
        L.mpm_sur_targets.argtypes = [vp, vp, vp, vp, ct.c_int, vp]
        L.mpm_surrogate_load.argtypes = [vp, ct.c_char_p, ct.c_size_t]
        L.mpm_step_blocks.argtypes = [vp, ct.c_int, ct.c_int, ct.c_float, vp]
        L.mpm_surrogate_residuals.argtypes = [vp, vp]
        for name in ("mpm_num_scenes", "mpm_max_colliders"):
            getattr(L, name).argtypes = [vp]
        L.mpm_num_particles.argtypes = [vp, ct.c_int]
        L.mpm_res.argtypes = [vp, ct.c_int]
        L.mpm_status_string.argtypes = [ct.c_int]
        L.mpm_status_string.restype = ct.c_char_p
        L.mpm_last_error.argtypes = [vp]
        L.mpm_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def declared_functions() -> List[str]:
    """Names of the functions the headers under include/ declare."""
    names = set()
    for h in sorted(os.listdir(os.path.dirname(HEADER))):
        if h.endswith(".h"):
            txt = open(os.path.join(os.path.dirname(HEADER), h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names.update(re.findall(r"\b(mpm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def _ptr(a) -> Optional[int]:
    """Host numpy float32/int32 array or torch tensor -> raw address."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous, "array must be C-contiguous"
        return a.ctypes.data
    return a.data_ptr()   # torch tensor (device or host)


def _f32(a, shape) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.float32)
    return out.reshape(shape)


SUR_NO_FALLBACK = 1
SUR_SYNC = 2


class Sim:
    """A batch of MPM scenes living on the GPU (one mpm_ctx)."""

    def __init__(self, scene_list: Sequence, stream=None):
        self.L = lib()
        self.scenes = list(scene_list)
        n = len(self.scenes)
        self._keep = []
        descs = (SceneDesc * n)()
        for i, sc in enumerate(self.scenes):
            x = _f32(sc.x, (sc.n, 3))
            v = _f32(sc.v, (sc.n, 3))
            self._keep += [x, v]
            d = descs[i]
            d.n_particles = sc.n
            d.x = x.ctypes.data_as(ct.POINTER(ct.c_float))
            d.v = v.ctypes.data_as(ct.POINTER(ct.c_float))
            d.particle_volume = sc.particle_volume
            d.res, d.dx, d.dt = sc.res, sc.dx, sc.dt
            d.gravity[:] = list(sc.gravity)
            d.bound = sc.bound
            d.mat = Material(sc.model, sc.E, sc.nu, sc.rho, sc.yield_stress, sc.yield_form)
            d.n_colliders = sc.n_colliders
            if sc.n_colliders:
                cs = (ColliderShape * sc.n_colliders)()
                for k, c in enumerate(sc.colliders):
                    cs[k].type = c.type
                    cs[k].half_extents[:] = [float(h) for h in c.half_extents]
                    cs[k].radius, cs[k].half_length = c.radius, c.half_length
                    cs[k].friction = c.friction
                    if getattr(c, "sdf", None) is not None:       # sampled SDF volume
                        a = np.ascontiguousarray(c.sdf, np.float32)
                        self._keep.append(a)
                        cs[k].sdf = a.ctypes.data_as(ct.POINTER(ct.c_float))
                        cs[k].sdf_dims[:] = list(a.shape)
                        cs[k].sdf_cell = c.sdf_cell
                        cs[k].sdf_origin[:] = [float(o) for o in c.sdf_origin]
                self._keep.append(cs)
                d.colliders = ct.cast(cs, ct.POINTER(ColliderShape))
        h = ct.c_void_p()
        st = self.L.mpm_create(descs, n, ct.c_void_p(stream) if stream else None, ct.byref(h))
        if st != OK:
            raise MPMError(st, "mpm_create failed: " + self.L.mpm_status_string(st).decode())
        self.h = h
        self.stream = stream          # the caller's stream handle (None: the library's own stream)
        self._keep = []
        self.n_scenes = n
        self.N = int(self.L.mpm_num_particles(self.h, -1))
        self.max_col = int(self.L.mpm_max_colliders(self.h))
        self.offsets = np.cumsum([0] + [sc.n for sc in self.scenes])

    # ----------------------------------------------------------------- errors
    def _check(self, st: int, what: str, allow_warn: bool = True):
        if st == OK or (allow_warn and st > 0):
            return st
        raise MPMError(st, f"{what}: {self.L.mpm_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None):
            self.L.mpm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- calls
    def set_colliders(self, poses, vels, on_device: bool = False):
        """poses (n_scenes, max_col, 7), vels (n_scenes, max_col, 6)."""
        if on_device:
            return self._check(self.L.mpm_set_colliders(self.h, _ptr(poses), _ptr(vels), 1), "set_colliders")
        P = _f32(poses, (self.n_scenes, self.max_col, 7))
        V = _f32(vels, (self.n_scenes, self.max_col, 6))
        return self._check(self.L.mpm_set_colliders(self.h, P.ctypes.data, V.ctypes.data, 0), "set_colliders")

    def particle_view(self):
        """Device pointers (ints) of the x, y, z position arrays in internal
        order, and the per-scene slot ranges [n_scenes + 1]."""
        px, py, pz = ct.c_void_p(), ct.c_void_p(), ct.c_void_p()
        begin = (ct.c_int * (self.n_scenes + 1))()
        self._check(self.L.mpm_particle_view(self.h, ct.byref(px), ct.byref(py), ct.byref(pz), begin),
                    "particle_view")
        return px.value, py.value, pz.value, np.array(begin[:], np.int64)

    def collider_wrenches(self):
        """[n_scenes][max_colliders][6]: impulse and angular impulse (about
        each collider's centre) the colliders received since the last call."""
        out = np.zeros((self.n_scenes, max(self.max_col, 1), 6), np.float32)
        self._check(self.L.mpm_get_collider_wrenches(self.h, out.ctypes.data, 0), "get_collider_wrenches")
        return out[:, : self.max_col]

    def set_colliders_ctrl(self, k: int):
        """Hand over every scene's poses / velocities of control step k."""
        if self.max_col == 0:
            return
        P = np.zeros((self.n_scenes, self.max_col, 7), np.float32)
        V = np.zeros((self.n_scenes, self.max_col, 6), np.float32)
        P[:, :, 3] = 1.0
        for s, sc in enumerate(self.scenes):
            if sc.n_colliders:
                P[s, : sc.n_colliders] = sc.ctrl_poses[k]
                V[s, : sc.n_colliders] = sc.ctrl_vels[k]
        self.set_colliders(P, V)

    def step(self, n: int = 1):
        return self._check(self.L.mpm_step(self.h, int(n)), "step")

    def set_scene_mask(self, active=None):
        """Step only the scenes with active[s] != 0 (None: all scenes)."""
        if active is None:
            return self._check(self.L.mpm_set_scene_mask(self.h, None), "set_scene_mask")
        a = np.ascontiguousarray(np.asarray(active) != 0, dtype=np.int32).reshape(self.n_scenes)
        return self._check(self.L.mpm_set_scene_mask(self.h, a.ctypes.data), "set_scene_mask")

    # ----------------------------------------------------------------- grid surrogate (device tensors)
    def sur_bbox(self, box):
        """box [n_scenes, 6] int32 device tensor <- nodes the P2G stencils reach (lo, hi inclusive)."""
        return self._check(self.L.mpm_sur_bbox(self.h, _ptr(box)), "sur_bbox")

    def sur_features(self, feat, grid0, origin=None):
        """feat [n_scenes, D, H, W, cf] and grid0 [n_scenes, D, H, W, 4] FP32 device tensors on the
        per-scene boxes at `origin` ([n_scenes, 3] int32 device tensor), or on the whole grid
        (origin None, D = H = W = res)."""
        D, H, W = (int(d) for d in feat.shape[1:4])
        return self._check(self.L.mpm_sur_features(self.h, _ptr(feat), int(feat.shape[-1]), _ptr(grid0), _ptr(origin),
                                                   D, H, W), "sur_features")

    def sur_block(self, pred, grid0, threshold: float = 1e-3, fallback: bool = True, sync: bool = False,
                  residual=None, n_fallback=None, origin=None):
        flags = (0 if fallback else SUR_NO_FALLBACK) | (SUR_SYNC if sync else 0)
        D, H, W = (int(d) for d in pred.shape[1:4])
        return self._check(self.L.mpm_sur_block(self.h, _ptr(pred), int(pred.shape[-1]), _ptr(grid0), _ptr(origin),
                                                D, H, W, float(threshold), flags, _ptr(residual), _ptr(n_fallback)),
                           "sur_block")

    def sur_targets(self, g0, g1, target, mask):
        return self._check(self.L.mpm_sur_targets(self.h, _ptr(g0), _ptr(g1), _ptr(target), int(target.shape[-1]),
                                                  _ptr(mask)), "sur_targets")

    def surrogate_load(self, blob: bytes):
        """Hand the library a trained surrogate network (UNet.export_weights())."""
        self._check(self.L.mpm_surrogate_load(self.h, blob, len(blob)), "surrogate_load")

    def step_blocks(self, n_blocks: int = 1, use_surrogate: bool = True, threshold: float = 1e-3) -> int:
        """n_blocks control steps (25 substeps each), through the loaded surrogate
        with its residual gate when use_surrogate; returns the number of
        scene-blocks that fell back to the plain substeps."""
        fb = ct.c_int(0)
        self._check(self.L.mpm_step_blocks(self.h, int(n_blocks), int(bool(use_surrogate)), float(threshold),
                                           ct.byref(fb)), "step_blocks")
        return int(fb.value)

    def surrogate_residuals(self) -> np.ndarray:
        """Per-scene residuals of the last surrogate block of step_blocks."""
        r = np.zeros(self.n_scenes, np.float32)
        self._check(self.L.mpm_surrogate_residuals(self.h, r.ctypes.data), "surrogate_residuals")
        return r

    def sync(self):
        return self._check(self.L.mpm_sync(self.h), "sync")

    def run_schedule(self, n_ctrl: int, substeps: int = 25, ctrl0: int = 0):
        for k in range(ctrl0, ctrl0 + n_ctrl):
            self.set_colliders_ctrl(k)
            self.step(substeps)

    def _count(self, scene: int) -> int:
        return self.N if scene < 0 else int(self.offsets[scene + 1] - self.offsets[scene])

    def get_state(self, scene: int = -1):
        n = self._count(scene)
        x = np.zeros((n, 3), np.float32)
        v = np.zeros((n, 3), np.float32)
        C = np.zeros((n, 3, 3), np.float32)
        F = np.zeros((n, 3, 3), np.float32)
        self._check(self.L.mpm_get_state(self.h, scene, x.ctypes.data, v.ctypes.data, C.ctypes.data,
                                         F.ctypes.data, 0), "get_state")
        return x, v, C, F

    def get_particles(self, scene: int = -1, with_v: bool = True, with_F: bool = False):
        n = self._count(scene)
        x = np.zeros((n, 3), np.float32)
        v = np.zeros((n, 3), np.float32) if with_v else None
        F = np.zeros((n, 3, 3), np.float32) if with_F else None
        self._check(self.L.mpm_get_particles(self.h, scene, x.ctypes.data, _ptr(v), _ptr(F), 0), "get_particles")
        return x, v, F

    def get_particles_device(self, x, v=None, F=None, scene: int = -1):
        """Copy into torch device tensors (stream-ordered, no host round trip)."""
        return self._check(self.L.mpm_get_particles(self.h, scene, _ptr(x), _ptr(v), _ptr(F), 1),
                           "get_particles")

    def get_state_device(self, x, v, C, F, scene: int = -1):
        """Copy the state (creation order) into device tensors, stream-ordered."""
        return self._check(self.L.mpm_get_state(self.h, scene, _ptr(x), _ptr(v), _ptr(C), _ptr(F), 1), "get_state")

    def set_state_device(self, x, v, C, F, scene: int = -1):
        return self._check(self.L.mpm_set_state(self.h, scene, _ptr(x), _ptr(v), _ptr(C), _ptr(F), 1), "set_state")

    def set_state(self, x, v, C, F, scene: int = -1):
        n = self._count(scene)
        arrs = [_f32(x, (n, 3)), _f32(v, (n, 3)), _f32(C, (n, 3, 3)), _f32(F, (n, 3, 3))]
        return self._check(self.L.mpm_set_state(self.h, scene, *[a.ctypes.data for a in arrs], 0), "set_state")

    def get_grid(self, scene: int):
        r = int(self.L.mpm_res(self.h, scene))
        m = np.zeros((r, r, r), np.float32)
        p = np.zeros((r, r, r, 3), np.float32)
        self._check(self.L.mpm_get_grid(self.h, scene, m.ctypes.data, p.ctypes.data, 0), "get_grid")
        return m, p

    def set_option(self, opt: int, value: int):
        return self._check(self.L.mpm_set_option(self.h, opt, int(value)), "set_option", allow_warn=False)

    def get_option(self, opt: int) -> int:
        v = ct.c_int()
        self._check(self.L.mpm_get_option(self.h, opt, ct.byref(v)), "get_option")
        return v.value

    def order(self) -> np.ndarray:
        pid = np.zeros(self.N, np.int32)
        self._check(self.L.mpm_get_order(self.h, pid.ctypes.data), "get_order")
        return pid

    def timing(self, reset: bool = True):
        """{kernel class: (total ms, launches)} from the library's HIP events."""
        ms = np.zeros(len(KERNEL_CLASSES), np.float64)
        n = np.zeros(len(KERNEL_CLASSES), np.int64)
        self._check(self.L.mpm_get_timing(self.h, ms.ctypes.data, n.ctypes.data, int(reset)), "get_timing")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def counters(self, reset: bool = True):
        """Work queued since the last reset: substeps, graph launches, host-launched substeps, re-sorts."""
        c = np.zeros(4, np.int64)
        self._check(self.L.mpm_get_counters(self.h, c.ctypes.data, int(reset)), "get_counters")
        return {"substeps": int(c[0]), "graph_launches": int(c[1]), "host_substeps": int(c[2]), "sorts": int(c[3])}

    def autotune(self, substeps: int = 10) -> str:
        n = 1 << 15                # the report lists every trial (about 120 bytes each)
        buf = ct.create_string_buffer(n)
        self._check(self.L.mpm_autotune(self.h, int(substeps), buf, n), "autotune")
        return buf.value.decode()
