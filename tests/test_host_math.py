"""The HIP path's FP32 material routines (mpm_math.hpp, built for the host)
against the FP64 oracle on random deformation gradients: Hencky stress,
von Mises return map, neo-Hookean stress and the fluid update.

Hencky states near the identity that stay elastic take a series for the
spatial log strain (no eigen-decomposition); the rest the eigen path.  Both
are held to the oracle, and to each other where both apply.

Bars (relative Frobenius error against the oracle; FP32 arithmetic):
  * stresses: 2e-5; the fluid's stress follows J - 1, which an FP32
    determinant of unit-size entries carries with an absolute error of a few
    ulp of 1, so its bar adds K * 10 * 2^-23 (times sqrt(3), the Frobenius
    norm of I) to 2e-5 |tau|.  The Hencky stress comes from an FP32 eigen-decomposition
    of F^T F - I, whose smallest eigenvalues carry an absolute error of a few
    ulp of |F|^2, so the relative error grows as the strains shrink (measured
    worst: 1.1e-5 for principal log strains up to 0.1, 2.7e-6 up to 0.3);
  * projected deformation gradients: 2e-6 (their entries are O(1)).
"""
import ctypes as ct
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host_math.cpp")
LIB = os.path.join(HERE, "_host_math.so")


@pytest.fixture(scope="module")
def hostmath():
    cmd = ["/opt/rocm/bin/hipcc", "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", LIB + ".tmp",
           SRC]
    subprocess.run(cmd, check=True, capture_output=True, cwd="/tmp")
    os.replace(LIB + ".tmp", LIB)
    L = ct.CDLL(LIB)
    vp = ct.c_void_p
    L.host_material.argtypes = [vp, ct.c_int, ct.c_int, ct.c_int, ct.c_float, ct.c_float, ct.c_float, vp, vp, vp]
    L.host_hencky_paths.argtypes = [vp, ct.c_int, ct.c_int, ct.c_float, ct.c_float, ct.c_float, vp, vp, vp]
    return L


class _Mat:
    """Scene fields the oracle's material routines read."""

    def __init__(self, model, E=5e3, nu=0.3, sy=1e3, yield_form=0):
        self.model, self.E, self.nu, self.yield_stress, self.yield_form = model, E, nu, sy, yield_form
        self.x = np.zeros((1, 3), np.float32)
        self.v = np.zeros((1, 3), np.float32)
        self.res, self.dx, self.dt, self.gravity, self.bound = 16, 1 / 16, 1e-4, (0.0, 0.0, 0.0), 3
        self.rho, self.particle_volume = 1e3, 1e-6
        self.colliders = []
        self.n, self.n_colliders = 1, 0
        self.mu = E / (2 * (1 + nu))
        self.la = E * nu / ((1 + nu) * (1 - 2 * nu))
        self.yield_eps = sy / (2 * self.mu) * (np.sqrt(2 / 3) if yield_form else 1.0)


def _rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _random_F(rng, n, strain, rotate=True):
    """Stretches exp(+-strain) along random axes, then a random rotation
    (rotate = False: a pure stretch, F = Q diag Q^T, whose small strains FP32
    carries at full relative precision, as the state F - I of a particle
    that does not rotate)."""
    F = np.empty((n, 3, 3))
    for p in range(n):
        Q = _rot(rng)
        F[p] = (_rot(rng) if rotate else Q.T) @ np.diag(np.exp(rng.uniform(-strain, strain, 3))) @ Q
    return F.astype(np.float32)


def _host(L, F, model, plastic, m):
    n = F.shape[0]
    Fo = np.zeros_like(F)
    tau = np.zeros_like(F)
    bad = np.zeros(n, np.int32)
    L.host_material(F.ctypes.data, n, model, int(plastic), m.mu, m.la, m.yield_eps, Fo.ctypes.data, tau.ctypes.data,
                    bad.ctypes.data)
    return Fo.astype(np.float64), tau.astype(np.float64), bad


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("strain,rotate", [(0.003, False), (0.03, False), (0.1, True), (0.3, True)])
def test_hencky_stress(hostmath, orc, strain, rotate):
    """Small strains as pure stretches: with a rotation, F's FP32 entries of
    size 1 carry the strain only to a few ulp of 1, a relative error of
    ~1e-4 at strain 3e-3 for any FP32 method."""
    rng = np.random.default_rng(7)
    F = _random_F(rng, 400, strain, rotate)
    elastic = _Mat(1, sy=0.0)            # no yield: the stress of F itself
    Fo, tau, bad = _host(hostmath, F, 1, 0, elastic)
    assert not bad.any()
    worst = max(_rel(tau[p], orc.stress(elastic, F[p].astype(np.float64))) for p in range(len(F)))
    print("Hencky stress, strain", strain, "worst rel err", worst)
    assert worst <= 2e-5
    assert np.abs(Fo - F).max() <= 2e-6 * max(1.0, np.abs(F).max())


@pytest.mark.parametrize("strain", [0.3, 0.6])
def test_von_mises_return_map(hostmath, orc, strain):
    """Yield radius 0.26 in deviatoric log strain (E 5e3, nu 0.3, sy 1e3):
    principal strains up to 0.3 or 0.6 make a part or most of them yield."""
    rng = np.random.default_rng(17)
    F = _random_F(rng, 400, strain)
    plastic = _Mat(1)
    Fo, tau, bad = _host(hostmath, F, 1, 1, plastic)
    assert not bad.any()
    wf = wt = 0.0
    yielded = 0
    for p in range(len(F)):
        Fr, y = orc.return_map(plastic, F[p].astype(np.float64))
        yielded += y
        wf = max(wf, _rel(Fo[p], Fr))
        wt = max(wt, _rel(tau[p], orc.stress(plastic, Fr)))
    print("return map, strain", strain, ": yielded", yielded, "of", len(F), "worst F", wf, "worst tau", wt)
    assert yielded >= len(F) // 10
    assert wf <= 2e-6 and wt <= 2e-5


def test_neo_hookean_stress(hostmath, orc):
    rng = np.random.default_rng(8)
    F = _random_F(rng, 400, 0.3)
    m = _Mat(0, E=1e4)
    _, tau, bad = _host(hostmath, F, 0, 0, m)
    assert not bad.any()
    worst = max(_rel(tau[p], orc.stress(m, F[p].astype(np.float64))) for p in range(len(F)))
    print("neo-Hookean worst rel err", worst)
    assert worst <= 2e-5


def test_fluid_update(hostmath, orc):
    rng = np.random.default_rng(9)
    F = _random_F(rng, 400, 0.05)
    m = _Mat(2)
    Fo, tau, bad = _host(hostmath, F, 2, 0, m)
    assert not bad.any()
    # |d tau| <= 2e-5 |tau| + K * 10 ulp(1) * sqrt(3): J - 1 from an FP32 determinant
    K = m.la + 2 * m.mu / 3
    floor = K * 10 * 2.0 ** -23 * np.sqrt(3)
    wf = wt = 0.0
    for p in range(len(F)):
        F64 = F[p].astype(np.float64)
        Fr = np.cbrt(np.linalg.det(F64)) * np.eye(3)   # the fluid keeps only its volume change
        wf = max(wf, _rel(Fo[p], Fr))
        ref = orc.stress(m, Fr)
        wt = max(wt, float(np.linalg.norm(tau[p] - ref) / (2e-5 * np.linalg.norm(ref) + floor)))
    print("fluid: worst F", wf, "worst tau error / bar", wt)
    assert wf <= 2e-6 and wt <= 1.0


def test_hencky_series_and_eigen_paths(hostmath, orc):
    """States spread over the series' range and past it (principal log
    strains up to 0.2): the series takes exactly the states with
    |F F^T - I|_F <= 0.35 and det F > 1/2 that do not yield, and there its
    stress matches both the eigen path and the oracle; with plasticity it
    declines every state the oracle's return map projects."""
    rng = np.random.default_rng(23)
    F = _random_F(rng, 600, 0.2)
    n = len(F)
    for plastic, mat in ((0, _Mat(1, sy=0.0)), (1, _Mat(1, sy=300.0))):
        ts = np.zeros_like(F)
        te = np.zeros_like(F)
        applied = np.zeros(n, np.int32)
        hostmath.host_hencky_paths(F.ctypes.data, n, plastic, mat.mu, mat.la,
                                   mat.yield_eps if plastic else np.inf, ts.ctypes.data, te.ctypes.data,
                                   applied.ctypes.data)
        F64 = F.astype(np.float64)
        b = np.einsum("nij,nkj->nik", F64, F64) - np.eye(3)
        near = (np.linalg.norm(b.reshape(n, 9), axis=1) <= 0.35 - 1e-4) & (np.linalg.det(F64) > 0.5)
        far = np.linalg.norm(b.reshape(n, 9), axis=1) > 0.35 + 1e-4
        yielded = np.array([orc.return_map(mat, F64[p])[1] for p in range(n)]) if plastic else np.zeros(n, bool)
        assert not applied[far].any()
        assert applied[near & ~yielded].all()
        assert not applied[yielded].any()
        ws = max(_rel(ts[p], orc.stress(mat, F64[p])) for p in np.flatnonzero(applied))
        we = max(_rel(ts[p], te[p]) for p in np.flatnonzero(applied))
        print("plastic", plastic, "series took", int(applied.sum()), "of", n, "worst vs oracle", ws, "vs eigen", we)
        assert (0.2 * n if not plastic else 30) <= applied.sum() <= 0.9 * n
        assert ws <= 2e-5 and we <= 2e-5
