"""FP64 CPU oracle of the immersed-boundary lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its binding) never does. It shares no code with the HIP path.

The arithmetic lives in lbm_oracle.cpp (plain C++17, double precision,
OpenMP over z for lattice sweeps); this module only marshals numpy arrays
through ctypes. Conventions (see lbm_oracle.cpp): populations are
[27][nz][ny][nx] pre-collision values, D3Q27 index i = (cx+1) + 3(cy+1) +
9(cz+1); marker arrays are (3, n); frames are (nsteps, 18); bone poses are
(nsteps, nbones, 24).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

BC_PERIODIC, BC_VELOCITY, BC_OUTFLOW = 0, 1, 2
IB_DIRECT, IB_IMPLICIT = 0, 1
COLLIDE_BGK, COLLIDE_TRT = 0, 1
WALL_NO_SLIP, WALL_SLIP = 0, 1
TRT_MAGIC = 3.0 / 16.0


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-Wextra", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_lo", ctypes.c_int32), ("bc_hi", ctypes.c_int32), ("mdf_iters", ctypes.c_int32),
                ("tau", ctypes.c_double), ("ib_alpha", ctypes.c_double),
                ("bc_y", ctypes.c_int32 * 2), ("bc_z", ctypes.c_int32 * 2), ("ib_scheme", ctypes.c_int32),
                ("collision", ctypes.c_int32), ("trt_lambda", ctypes.c_double), ("wall_mode", ctypes.c_int32)]


class _Markers(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nbones", ctypes.c_int32),
                ("xrest", ctypes.c_void_p), ("bone", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("dv", ctypes.c_void_p), ("nrest", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.c_void_p
        L.or_abi_version.restype = ctypes.c_int
        L.or_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = None
        L.or_lattice.argtypes = [dp, dp]
        L.or_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.or_equilibrium_field.argtypes = [dp, dp, ctypes.c_int64, dp]
        L.or_phi.argtypes = [ctypes.c_double]
        L.or_phi.restype = ctypes.c_double
        L.or_frame_accel_static.argtypes = [dp, dp, dp]
        L.or_node_velocity.argtypes = [ctypes.c_double, dp, dp, dp, dp, dp, dp]
        L.or_collide_node.argtypes = [dp, dp, dp, dp, ctypes.c_double, dp, dp, dp]
        L.or_collide_node_trt.argtypes = [dp, dp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.or_skin.argtypes = [dp, dp, dp, dp]
        L.or_skin_normals.argtypes = [dp, dp, dp]
        L.or_skin_normals.restype = ctypes.c_int
        L.or_interpolate.argtypes = [dp, dp, ctypes.c_int, dp, ctypes.c_int, dp]
        L.or_spread.argtypes = [dp, dp, ctypes.c_int, dp, dp]
        L.or_macros.argtypes = [dp, dp, dp, dp, dp]
        L.or_run.argtypes = [dp, dp, dp, dp, dp, ctypes.c_int, dp, dp, dp, dp]
        L.or_run.restype = ctypes.c_int
        L.or_run_forced.argtypes = [dp, dp, dp, ctypes.c_int, dp]
        L.or_run_forced.restype = ctypes.c_int
        L.or_run_tangent.argtypes = [dp, dp, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp]
        L.or_run_tangent.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def params(nx, ny, nz, tau, bc_lo=BC_PERIODIC, bc_hi=BC_PERIODIC, mdf_iters=1, ib_alpha=1.0,
           bc_y=(BC_PERIODIC, BC_PERIODIC), bc_z=(BC_PERIODIC, BC_PERIODIC), ib_scheme=IB_DIRECT,
           collision=COLLIDE_BGK, trt_lambda=TRT_MAGIC, wall_mode=WALL_NO_SLIP) -> _Params:
    """Face conditions: x by bc_lo / bc_hi, y and z by the pairs bc_y, bc_z
    (low, high); an axis is periodic or open on both faces. ib_scheme
    IB_DIRECT: explicit direct forcing plus mdf_iters - 1 multi-direct-forcing
    passes; IB_IMPLICIT: the implicit velocity correction, mdf_iters
    conjugate-gradient steps. collision COLLIDE_BGK, or COLLIDE_TRT with
    Lambda = (tau - 1/2)(tau- - 1/2) = trt_lambda. wall_mode WALL_NO_SLIP, or
    WALL_SLIP (forcing along the marker normals only; needs the marker set's
    normals)."""
    return _Params(nx, ny, nz, bc_lo, bc_hi, mdf_iters, tau, ib_alpha, (ctypes.c_int32 * 2)(*bc_y),
                   (ctypes.c_int32 * 2)(*bc_z), ib_scheme, collision, trt_lambda, wall_mode)


def threads() -> int:
    """OpenMP threads the oracle's lattice sweeps use."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Use n OpenMP threads for later lattice sweeps."""
    lib().or_set_threads(int(n))


def lattice():
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    lib().or_lattice(_p(c), _p(w))
    return c, w


def equilibrium(rho: float, u) -> np.ndarray:
    u = _f64(u)
    out = np.zeros(27)
    lib().or_equilibrium(float(rho), _p(u), _p(out))
    return out


def equilibrium_field(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """rho (nz,ny,nx), u (3,nz,ny,nx) -> f (27,nz,ny,nx)."""
    rho = _f64(rho)
    u = _f64(u)
    out = np.zeros((27,) + rho.shape)
    lib().or_equilibrium_field(_p(rho), _p(u), rho.size, _p(out))
    return out


def phi(r: float) -> float:
    return lib().or_phi(float(r))


def frame_accel_static(frame, x) -> np.ndarray:
    fr = _f64(frame)
    x = _f64(x)
    out = np.zeros(3)
    lib().or_frame_accel_static(_p(fr), _p(x), _p(out))
    return out


def node_velocity(rho, m, g, frame, x):
    m, g, fr, x = _f64(m), _f64(g), _f64(frame), _f64(x)
    u = np.zeros(3)
    F = np.zeros(3)
    lib().or_node_velocity(float(rho), _p(m), _p(g), _p(fr), _p(x), _p(u), _p(F))
    return u, F


def collide_node(f, g, frame, x, tau, trt_lambda=None):
    """One node's collision: BGK, or TRT with Lambda = trt_lambda."""
    f, g, fr, x = _f64(f), _f64(g), _f64(frame), _f64(x)
    out = np.zeros(27)
    u = np.zeros(3)
    F = np.zeros(3)
    if trt_lambda is None:
        lib().or_collide_node(_p(f), _p(g), _p(fr), _p(x), float(tau), _p(out), _p(u), _p(F))
    else:
        lib().or_collide_node_trt(_p(f), _p(g), _p(fr), _p(x), float(tau), float(trt_lambda), _p(out), _p(u),
                                  _p(F))
    return out, u, F


def _markers(ms, keep):
    xr = _f64(ms.xrest)
    bone = np.ascontiguousarray(ms.bone, dtype=np.int32)
    wt = _f64(ms.weight)
    dv = _f64(ms.dv)
    nr = None if getattr(ms, "normals", None) is None else _f64(ms.normals)
    keep.extend([xr, bone, wt, dv, nr])
    return _Markers(xr.shape[1], int(ms.nbones), xr.ctypes.data, bone.ctypes.data, wt.ctypes.data, dv.ctypes.data,
                    None if nr is None else nr.ctypes.data)


def skin(ms, pose):
    keep = []
    m = _markers(ms, keep)
    pose = _f64(pose)
    X = np.zeros((3, ms.n))
    U = np.zeros((3, ms.n))
    lib().or_skin(ctypes.byref(m), _p(pose), _p(X), _p(U))
    return X, U


def skin_normals(ms, pose):
    """Skinned outward normals (3, n) of marker set ms at bone poses pose."""
    keep = []
    m = _markers(ms, keep)
    pose = _f64(pose)
    N = np.zeros((3, ms.n))
    if lib().or_skin_normals(ctypes.byref(m), _p(pose), _p(N)) != 0:
        raise OracleError("the marker set has no normals")
    return N


def interpolate(prm: _Params, field: np.ndarray, X: np.ndarray) -> np.ndarray:
    field = _f64(field)
    ncomp = field.shape[0] if field.ndim == 4 else 1
    X = _f64(X)
    out = np.zeros((ncomp, X.shape[1]))
    lib().or_interpolate(ctypes.byref(prm), _p(field), ncomp, _p(X), X.shape[1], _p(out))
    return out


def spread(prm: _Params, X: np.ndarray, Fdv: np.ndarray) -> np.ndarray:
    X = _f64(X)
    Fdv = _f64(Fdv)
    g = np.zeros((3, prm.nz, prm.ny, prm.nx))
    lib().or_spread(ctypes.byref(prm), _p(X), X.shape[1], _p(Fdv), _p(g))
    return g


def macros(prm: _Params, f: np.ndarray, frame) -> tuple:
    f = _f64(f)
    fr = _f64(frame)
    rho = np.zeros((prm.nz, prm.ny, prm.nx))
    u = np.zeros((3, prm.nz, prm.ny, prm.nx))
    lib().or_macros(ctypes.byref(prm), _p(f), _p(fr), _p(rho), _p(u))
    return rho, u


class OracleError(RuntimeError):
    pass


def run(prm: _Params, f: np.ndarray, frames: np.ndarray, markers=None, poses=None, nsteps=None):
    """Advance pre-collision populations f (27,nz,ny,nx) in place (a float64
    contiguous copy is made if needed and returned). Returns dict with f,
    wrench (nsteps, 8), X, U, F of the last step."""
    f = _f64(f)
    frames = _f64(frames)
    if nsteps is None:
        nsteps = frames.shape[0]
    assert frames.shape[0] >= nsteps
    keep = []
    mptr = None
    n = 0
    if markers is not None:
        m = _markers(markers, keep)
        mptr = ctypes.byref(m)
        n = markers.n
        poses = _f64(poses)
        assert poses.shape[0] >= nsteps and poses.shape[1] == markers.nbones
    wrench = np.zeros((nsteps, 8))
    X = np.zeros((3, n))
    U = np.zeros((3, n))
    F = np.zeros((3, n))
    rc = lib().or_run(ctypes.byref(prm), _p(f), mptr, _p(poses) if poses is not None else None, _p(frames),
                      int(nsteps), _p(wrench), _p(X) if n else None, _p(U) if n else None, _p(F) if n else None)
    if rc != 0:
        raise OracleError(f"oracle run failed with code {rc}")
    return {"f": f, "wrench": wrench, "X": X, "U": U, "F": F}


def run_forced(prm: _Params, f: np.ndarray, g: np.ndarray, nsteps: int, frame=None) -> np.ndarray:
    """nsteps steps of the fluid alone with a constant body-force density
    field g (3, nz, ny, nx) added at every node; returns the advanced f."""
    f = _f64(f)
    g = _f64(g)
    frames = _f64(np.repeat(np.asarray(frame if frame is not None else np.zeros(18), np.float64).reshape(1, 18),
                            nsteps, axis=0))
    rc = lib().or_run_forced(ctypes.byref(prm), _p(f), _p(frames), int(nsteps), _p(g))
    if rc != 0:
        raise OracleError(f"oracle run failed with code {rc}")
    return f


def run_tangent(prm: _Params, f: np.ndarray, frames: np.ndarray, markers, poses, poses_d, nsteps=None):
    """Forward-mode tangent of run() along a direction poses_d of the bone
    poses (initial populations and frames fixed), in dual-number arithmetic.
    f is advanced in place as by run(). Returns dict with f, f_d (d f), wrench
    and wrench_d (d wrench), each of the shape run() uses."""
    f = _f64(f)
    frames = _f64(frames)
    if nsteps is None:
        nsteps = frames.shape[0]
    keep = []
    m = _markers(markers, keep)
    poses = _f64(poses)
    poses_d = _f64(poses_d)
    assert poses.shape == poses_d.shape and poses.shape[0] >= nsteps and poses.shape[1] == markers.nbones
    f_d = np.zeros_like(f)
    wrench = np.zeros((nsteps, 8))
    wrench_d = np.zeros((nsteps, 8))
    rc = lib().or_run_tangent(ctypes.byref(prm), _p(f), _p(f_d), ctypes.byref(m), _p(poses), _p(poses_d), _p(frames),
                              int(nsteps), _p(wrench), _p(wrench_d))
    if rc != 0:
        raise OracleError(f"oracle tangent run failed with code {rc}")
    return {"f": f, "f_d": f_d, "wrench": wrench, "wrench_d": wrench_d}


def initial_populations(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    return equilibrium_field(rho, u)


def run_workload(w, nsteps=None, f0=None):
    """Run an inputs.Workload from its initial state f = f^eq(1, u0)."""
    prm = params(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, w.mdf_iters, w.ib_alpha, w.bc_y, w.bc_z, w.ib_scheme,
                 w.collision, w.trt_lambda, w.wall_mode)
    if f0 is None:
        f0 = equilibrium_field(np.ones((w.nz, w.ny, w.nx)), w.u0)
    return run(prm, f0, w.frames, w.markers, w.poses, nsteps or w.nsteps)
