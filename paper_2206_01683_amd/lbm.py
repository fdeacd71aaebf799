"""Python binding of the C interface in include/lbm_ib.h.

Argument marshalling only: every step of the method runs in the HIP library
(liblbmib.so, built in-tree by paper_2206_01683_amd.build). PyTorch supplies
device memory and the stream. There is no CPU fallback: if the library is
missing or no GPU is visible, constructing a Simulation raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmib.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "lbm_ib.h")

LBM_OK = 0
STATUS = {0: "LBM_OK", -1: "LBM_ERR_ARG", -2: "LBM_ERR_DEVICE", -3: "LBM_ERR_UNSTABLE",
          -4: "LBM_ERR_MARKER_RANGE", -5: "LBM_ERR_CAPACITY", -6: "LBM_ERR_UNSUPPORTED"}
BC_PERIODIC, BC_VELOCITY, BC_OUTFLOW = 0, 1, 2
OK, ERR_ARG, ERR_DEVICE, ERR_UNSTABLE, ERR_MARKER_RANGE, ERR_CAPACITY, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
STATIC_WORKSPACE_BYTES = 64 << 20  # LBM_STATIC_WORKSPACE_BYTES
IB_DIRECT, IB_IMPLICIT = 0, 1
COLLIDE_BGK, COLLIDE_TRT = 0, 1
LAYOUT_AUTO, LAYOUT_PLANES, LAYOUT_ROWS = 0, 1, 2
WALL_NO_SLIP, WALL_SLIP = 0, 1
TRT_MAGIC = 3.0 / 16.0


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_lo", ctypes.c_int32), ("bc_hi", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("max_markers", ctypes.c_int32), ("max_bones", ctypes.c_int32), ("mdf_iters", ctypes.c_int32),
                ("max_active_tiles", ctypes.c_int32), ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("with_adjoint", ctypes.c_int32), ("tau", ctypes.c_double), ("ib_alpha", ctypes.c_double),
                ("bc_y", ctypes.c_int32 * 2), ("bc_z", ctypes.c_int32 * 2), ("ib_scheme", ctypes.c_int32),
                ("collision", ctypes.c_int32), ("trt_lambda", ctypes.c_double), ("wall_mode", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("ib_workgroups", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double * 3) for name in ("acc", "omega", "alpha", "origin", "u_lo", "u_hi")]


class Markers(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nbones", ctypes.c_int32),
                ("xrest", ctypes.c_void_p), ("bone", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("dv", ctypes.c_void_p), ("X", ctypes.c_void_p), ("U", ctypes.c_void_p), ("F", ctypes.c_void_p),
                ("nrest", ctypes.c_void_p)]


class Env(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("m", Markers), ("poses", ctypes.c_void_p), ("frames", ctypes.c_void_p),
                ("wrench", ctypes.c_void_p), ("rotating", ctypes.c_int32)]


BATCH_PHASES, BATCH_PERSISTENT = 0, 1
BATCH_SHAPES = ((64, 8), (128, 4), (256, 2), (512, 1), (512, 0))  # (512, 0): linear cell order


class Swimmer(ctypes.Structure):
    _fields_ = [("nbones", ctypes.c_int32), ("free_yaw", ctypes.c_int32), ("link_length", ctypes.c_double),
                ("mass", ctypes.c_void_p), ("com", ctypes.c_void_p), ("inertia", ctypes.c_void_p),
                ("joints_rest", ctypes.c_void_p), ("fluid_ratio", ctypes.c_double), ("origin", ctypes.c_double * 3),
                ("added_mass", ctypes.c_double)]


class SwimmerState(ctypes.Structure):
    _fields_ = [("vel", ctypes.c_double * 2), ("acc", ctypes.c_double * 2), ("heading", ctypes.c_double),
                ("spin", ctypes.c_double), ("spin_prev", ctypes.c_double), ("ang_mom", ctypes.c_double),
                ("inertia", ctypes.c_double), ("pos", ctypes.c_double * 2)]


class LBMError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({strerror(code)})")


_lib = None


def lib():
    """Load liblbmib.so. Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        P = ctypes.POINTER(Params)
        L.lbm_population_bytes.argtypes = [P]
        L.lbm_population_bytes.restype = sz
        L.lbm_workspace_bytes.argtypes = [P]
        L.lbm_workspace_bytes.restype = sz
        L.lbm_population_strides.argtypes = [P, vp]
        L.lbm_init.argtypes = [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp, vp]
        L.lbm_init_static.argtypes = [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp]
        L.lbm_load_populations.argtypes = [vp, vp]
        L.lbm_read_populations.argtypes = [vp, vp]
        L.lbm_macros.argtypes = [vp, vp, vp, vp]
        L.lbm_ib_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp]
        L.lbm_body_forces.argtypes = [vp, vp, vp, vp]
        L.lbm_state_save.argtypes = [vp, vp]
        L.lbm_state_restore.argtypes = [vp, vp, ctypes.c_int64]
        L.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lbm_bind_populations.argtypes = [vp, vp, vp]
        L.lbm_swimmer_init.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp]
        L.lbm_swimmer_prepare.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lbm_swimmer_advance.argtypes = [vp, vp, vp, vp, vp]
        L.lbm_adjoint_ring_bytes.argtypes = [P, ctypes.c_int32]
        L.lbm_adjoint_ring_bytes.restype = sz
        L.lbm_adjoint_segment.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lbm_adjoint_sweep.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lbm_adjoint_record.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.lbm_check.argtypes = [vp]
        L.lbm_set_stream.argtypes = [vp, vp]
        L.lbm_profile_enable.argtypes = [vp, ctypes.c_int]
        L.lbm_profile_collect.argtypes = [vp, vp, vp, vp]
        L.lbm_batch_bytes.argtypes = [ctypes.c_int32]
        L.lbm_batch_bytes.restype = sz
        L.lbm_batch_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_int32, vp, vp]
        L.lbm_batch_run.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.lbm_batch_autotune.argtypes = [vp, ctypes.c_int32, vp]
        L.lbm_batch_set_shapes.argtypes = [vp, vp]
        L.lbm_batch_check.argtypes = [vp]
        L.lbm_batch_group_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.lbm_batch_group_bytes.restype = sz
        L.lbm_batch_set_groups.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp), vp]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        L.lbm_step_count.argtypes = [vp]
        L.lbm_step_count.restype = ctypes.c_int64
        L.lbm_strerror.argtypes = [ctypes.c_int]
        L.lbm_strerror.restype = ctypes.c_char_p
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        for name in ("lbm_init", "lbm_init_static", "lbm_population_strides", "lbm_load_populations",
                     "lbm_read_populations", "lbm_macros", "lbm_ib_step", "lbm_body_forces", "lbm_check",
                     "lbm_set_stream", "lbm_profile_enable",
                     "lbm_profile_collect", "lbm_state_save", "lbm_state_restore", "lbm_adjoint_step",
                     "lbm_bind_populations", "lbm_adjoint_segment", "lbm_adjoint_sweep", "lbm_adjoint_record",
                     "lbm_swimmer_init", "lbm_swimmer_prepare",
                     "lbm_swimmer_advance",
                     "lbm_batch_create", "lbm_batch_run", "lbm_batch_autotune",
                     "lbm_batch_set_shapes", "lbm_batch_set_groups", "lbm_batch_check"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().lbm_strerror(int(code)).decode()
    except Exception:
        return "?"


def _check(rc: int, what: str):
    if rc != LBM_OK:
        raise LBMError(rc, what)


def make_params(nx, ny, nz, tau, bc_lo=BC_PERIODIC, bc_hi=BC_PERIODIC, storage="f32", max_markers=0,
                max_bones=1, mdf_iters=1, ib_alpha=1.0, max_active_tiles=0, block=(0, 0), with_adjoint=False,
                bc_y=(BC_PERIODIC, BC_PERIODIC), bc_z=(BC_PERIODIC, BC_PERIODIC), ib_scheme=0, collision=0,
                trt_lambda=TRT_MAGIC, wall_mode=0, layout=LAYOUT_AUTO, ib_workgroups=0) -> Params:
    """ib_scheme: IB_DIRECT (direct forcing, mdf_iters passes) or IB_IMPLICIT
    (implicit velocity correction, mdf_iters conjugate-gradient steps).
    collision: COLLIDE_BGK or COLLIDE_TRT with Lambda = trt_lambda.
    wall_mode: WALL_NO_SLIP or WALL_SLIP (normal component only).
    layout: LAYOUT_AUTO, LAYOUT_PLANES or LAYOUT_ROWS (stored populations).
    ib_workgroups: workgroups running the IB phases beside the collide (0
    automatic); -1 runs them before the collide in launches of their own.
    block: collide block (bx, by); (bx, -1) is bx consecutive cells."""
    return Params(nx, ny, nz, bc_lo, bc_hi, STORAGE[storage] if isinstance(storage, str) else storage,
                  max_markers, max_bones, mdf_iters, max_active_tiles, block[0], block[1], 1 if with_adjoint else 0,
                  tau, ib_alpha, (ctypes.c_int32 * 2)(*bc_y), (ctypes.c_int32 * 2)(*bc_z), ib_scheme, collision,
                  trt_lambda, wall_mode, layout, ib_workgroups)


def frames_array(frames: np.ndarray) -> np.ndarray:
    """(nsteps, 18) float64, C-contiguous: the lbm_frame layout."""
    fr = np.ascontiguousarray(frames, dtype=np.float64)
    assert fr.ndim == 2 and fr.shape[1] == 18
    return fr


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class DeviceMarkers:
    """Marker arrays on the device in the lbm_markers layout (float32/int32)."""

    def __init__(self, ms, device="cuda"):
        dev = torch.device(device)
        self.n = int(ms.xrest.shape[1])
        self.nbones = int(ms.nbones)
        self.xrest = torch.as_tensor(np.ascontiguousarray(ms.xrest, np.float32), device=dev)
        self.bone = torch.as_tensor(np.ascontiguousarray(ms.bone, np.int32), device=dev)
        self.weight = torch.as_tensor(np.ascontiguousarray(ms.weight, np.float32), device=dev)
        self.dv = torch.as_tensor(np.ascontiguousarray(ms.dv, np.float32), device=dev)
        self.X = torch.zeros((3, self.n), dtype=torch.float32, device=dev)
        self.U = torch.zeros((3, self.n), dtype=torch.float32, device=dev)
        self.F = torch.zeros((3, self.n), dtype=torch.float32, device=dev)
        nr = getattr(ms, "normals", None)  # rest normals, needed by slip walls only
        self.nrest = None if nr is None else torch.as_tensor(np.ascontiguousarray(nr, np.float32), device=dev)

    def struct(self) -> Markers:
        return Markers(self.n, self.nbones, self.xrest.data_ptr(), self.bone.data_ptr(), self.weight.data_ptr(),
                       self.dv.data_ptr(), self.X.data_ptr(), self.U.data_ptr(), self.F.data_ptr(),
                       None if self.nrest is None else self.nrest.data_ptr())


class Simulation:
    """One lattice with its two population buffers and workspace (torch-owned).

    static_workspace=True creates the context with lbm_init_static: no
    workspace tensor; the library's per-device static workspace is used
    (shared by every such Simulation on the device, so only the latest one
    is usable)."""

    def __init__(self, nx, ny, nz, tau, bc_lo=BC_PERIODIC, bc_hi=BC_PERIODIC, storage="f32", max_markers=0,
                 max_bones=1, mdf_iters=1, ib_alpha=1.0, rho0=None, u0=None, device="cuda", block=(0, 0),
                 max_active_tiles=0, stream=None, with_adjoint=False, bc_y=(BC_PERIODIC, BC_PERIODIC),
                 bc_z=(BC_PERIODIC, BC_PERIODIC), ib_scheme=0, collision=0, trt_lambda=TRT_MAGIC, wall_mode=0,
                 static_workspace=False, layout=LAYOUT_AUTO, ib_workgroups=0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice Boltzmann library runs only on the GPU")
        L = lib()
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.params = make_params(nx, ny, nz, tau, bc_lo, bc_hi, storage, max_markers, max_bones, mdf_iters,
                                  ib_alpha, max_active_tiles, block, with_adjoint, bc_y, bc_z, ib_scheme,
                                  collision, trt_lambda, wall_mode, layout, ib_workgroups)
        pb = L.lbm_population_bytes(ctypes.byref(self.params))
        wb = L.lbm_workspace_bytes(ctypes.byref(self.params))
        if pb == 0 or wb == 0:
            raise LBMError(-1, "invalid parameters")
        self.population_bytes = pb
        self.workspace_bytes = wb
        st = (ctypes.c_int64 * 3)()
        _check(L.lbm_population_strides(ctypes.byref(self.params), st), "lbm_population_strides")
        self.pop_stride, self.row_stride, self.rows_layout = int(st[0]), int(st[1]), bool(st[2])
        self.fa = torch.empty(pb, dtype=torch.uint8, device=self.device)
        self.fb = torch.empty(pb, dtype=torch.uint8, device=self.device)
        self.static_workspace = bool(static_workspace)
        if self.static_workspace:
            self.ws = None
        else:
            self._ws_raw = torch.empty(wb + 256, dtype=torch.uint8, device=self.device)
            shift = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[shift:shift + wb]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        rho0_t = None if rho0 is None else self._dev_f32(rho0)
        u0_t = None if u0 is None else self._dev_f32(u0)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if self.static_workspace:
                _check(L.lbm_init_static(ctypes.byref(ctx), ctypes.byref(self.params), _ptr(self.fa),
                                         _ptr(self.fb), _ptr(rho0_t), _ptr(u0_t),
                                         ctypes.c_void_p(self.stream.cuda_stream)), "lbm_init_static")
            else:
                _check(L.lbm_init(ctypes.byref(ctx), ctypes.byref(self.params), _ptr(self.fa), _ptr(self.fb),
                                  _ptr(self.ws), _ptr(rho0_t), _ptr(u0_t), ctypes.c_void_p(self.stream.cuda_stream)),
                       "lbm_init")
        self.ctx = ctx
        self._keep = [rho0_t, u0_t]

    def _dev_f32(self, a) -> torch.Tensor:
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=torch.float32).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)

    @property
    def ncell(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz

    def load_populations(self, f):
        t = self._dev_f32(f)
        assert t.numel() == 27 * self.ncell
        _check(lib().lbm_load_populations(self.ctx, _ptr(t)), "lbm_load_populations")
        self._keep.append(t)

    def read_populations(self) -> torch.Tensor:
        out = torch.empty((27,) + self.shape, dtype=torch.float32, device=self.device)
        _check(lib().lbm_read_populations(self.ctx, _ptr(out)), "lbm_read_populations")
        return out

    def macros(self, frame=None):
        rho = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        fr = None
        if frame is not None:
            fr = frames_array(np.asarray(frame).reshape(1, 18))
        _check(lib().lbm_macros(self.ctx, None if fr is None else fr.ctypes.data_as(ctypes.c_void_p),
                                _ptr(rho), _ptr(u)), "lbm_macros")
        return rho, u

    def step(self, frames, markers: Optional[DeviceMarkers] = None, poses: Optional[torch.Tensor] = None,
             wrench: Optional[torch.Tensor] = None, nsteps: Optional[int] = None):
        fr = frames_array(frames)
        n = fr.shape[0] if nsteps is None else int(nsteps)
        assert fr.shape[0] >= n
        ms = None
        if markers is not None:
            ms = markers.struct()
            assert poses is not None and poses.dtype == torch.float32 and poses.is_contiguous()
            assert poses.shape[0] >= n and poses.shape[1] == markers.nbones and poses.shape[2] == 24
        if wrench is not None:
            assert wrench.dtype == torch.float32 and wrench.is_contiguous() and wrench.numel() >= 8 * n
        _check(lib().lbm_ib_step(self.ctx, None if ms is None else ctypes.byref(ms), _ptr(poses),
                                 fr.ctypes.data_as(ctypes.c_void_p), n, _ptr(wrench)), "lbm_ib_step")

    def body_forces(self, markers: DeviceMarkers, center) -> torch.Tensor:
        out = torch.empty((1 + markers.nbones, 8), dtype=torch.float32, device=self.device)
        c = np.ascontiguousarray(center, dtype=np.float64)
        ms = markers.struct()
        _check(lib().lbm_body_forces(self.ctx, ctypes.byref(ms), c.ctypes.data_as(ctypes.c_void_p), _ptr(out)),
               "lbm_body_forces")
        return out

    def profile(self, enable: bool = True):
        _check(lib().lbm_profile_enable(self.ctx, 1 if enable else 0), "lbm_profile_enable")

    def profile_collect(self):
        """(ib_ms_total, collide_ms_total, timed_steps) since the last collect."""
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().lbm_profile_collect(self.ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
               "lbm_profile_collect")
        return a.value, b.value, n.value

    def stored_view(self, state: torch.Tensor) -> torch.Tensor:
        """[27][nz][ny][nx] strided view of a float32 buffer in the stored
        population layout (a state, or an adjoint buffer of the same layout)."""
        nz, ny, nx = self.shape
        flat = state.view(torch.float32) if state.dtype != torch.float32 else state
        return flat.as_strided((27, nz, ny, nx), (self.pop_stride, ny * self.row_stride, self.row_stride, 1))

    def new_state(self) -> torch.Tensor:
        """An uninitialized buffer in the stored population layout."""
        return torch.empty(self.population_bytes, dtype=torch.uint8, device=self.device)

    def save_state(self, dst: torch.Tensor):
        _check(lib().lbm_state_save(self.ctx, _ptr(dst)), "lbm_state_save")

    def restore_state(self, src: torch.Tensor, step: int = 0):
        _check(lib().lbm_state_restore(self.ctx, _ptr(src), int(step)), "lbm_state_restore")

    def set_stream(self, stream: torch.cuda.Stream):
        """Enqueue all further work on `stream` (e.g. a graph-capture stream)."""
        _check(lib().lbm_set_stream(self.ctx, ctypes.c_void_p(stream.cuda_stream)), "lbm_set_stream")
        self.stream = stream

    def bind_populations(self, cur: torch.Tensor, nxt: torch.Tensor):
        """The next step reads `cur` and writes `nxt` (then ping-pong)."""
        for t in (cur, nxt):
            assert t.is_cuda and t.numel() * t.element_size() >= self.population_bytes
        _check(lib().lbm_bind_populations(self.ctx, _ptr(cur), _ptr(nxt)), "lbm_bind_populations")
        self._bound = (cur, nxt)

    def bind_own_buffers(self):
        """Return to the context's own two buffers; the state is not carried over."""
        self.bind_populations(self.fa, self.fb)

    def adjoint_step(self, state: torch.Tensor, markers: Optional[DeviceMarkers], pose: Optional[torch.Tensor],
                     frame, weights, lam_next: torch.Tensor, lam_prev: torch.Tensor,
                     pose_bar: Optional[torch.Tensor]):
        fr = frames_array(np.asarray(frame).reshape(1, 18))
        wts = np.ascontiguousarray(weights, dtype=np.float64).reshape(4)
        ms = None if markers is None else markers.struct()
        _check(lib().lbm_adjoint_step(self.ctx, _ptr(state), None if ms is None else ctypes.byref(ms), _ptr(pose),
                                      fr.ctypes.data_as(ctypes.c_void_p), wts.ctypes.data_as(ctypes.c_void_p),
                                      _ptr(lam_next), _ptr(lam_prev), _ptr(pose_bar)), "lbm_adjoint_step")

    def adjoint_ring(self, nseg: int) -> torch.Tensor:
        """Device buffer for the forward IB data of nseg steps (256-byte aligned)."""
        nb = lib().lbm_adjoint_ring_bytes(ctypes.byref(self.params), int(nseg))
        if nb == 0:
            raise LBMError(-1, "invalid adjoint ring size")
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        shift = (-raw.data_ptr()) % 256
        return raw[shift:shift + nb]

    def adjoint_segment(self, ckpt: torch.Tensor, ring, markers: Optional[DeviceMarkers],
                        poses: Optional[torch.Tensor], frames, weights, lam: torch.Tensor, lam_tmp: torch.Tensor,
                        pose_bar: Optional[torch.Tensor], ib_ring: torch.Tensor, sweep_only: bool = False):
        """Native reverse sweep over len(frames) steps from checkpoint ckpt
        (lbm_adjoint_segment): lam in = dJ/d(state after), out = dJ/d(ckpt).
        sweep_only: the segment was recorded by adjoint_record into ring and
        ib_ring (lbm_adjoint_sweep, no recompute)."""
        fr = frames_array(frames)
        nseg = fr.shape[0]
        assert len(ring) >= nseg - 1
        ptrs = (ctypes.c_void_p * max(1, nseg - 1))(*[t.data_ptr() for t in ring[:nseg - 1]] or [None])
        wts = np.ascontiguousarray(weights, dtype=np.float64).reshape(4)
        ms = None if markers is None else markers.struct()
        if markers is not None:
            assert poses.is_contiguous() and pose_bar.is_contiguous() and poses.shape[0] >= nseg
        fn = lib().lbm_adjoint_sweep if sweep_only else lib().lbm_adjoint_segment
        _check(fn(self.ctx, _ptr(ckpt), ptrs, nseg, None if ms is None else ctypes.byref(ms), _ptr(poses),
                  fr.ctypes.data_as(ctypes.c_void_p), wts.ctypes.data_as(ctypes.c_void_p), _ptr(lam), _ptr(lam_tmp),
                  _ptr(pose_bar), _ptr(ib_ring)), "lbm_adjoint_sweep" if sweep_only else "lbm_adjoint_segment")

    def adjoint_record(self, ckpt: torch.Tensor, ring, markers: Optional[DeviceMarkers],
                       poses: Optional[torch.Tensor], frames, ib_ring: torch.Tensor,
                       wrench: Optional[torch.Tensor] = None):
        """Forward over len(frames) steps from ckpt keeping every state
        (ring[t] = state after step t; len(ring) == nsteps, the last entry may
        be None) and every step's IB data in ib_ring (lbm_adjoint_record);
        wrench (nsteps, 8) receives the step wrenches."""
        fr = frames_array(frames)
        nseg = fr.shape[0]
        assert len(ring) == nseg
        ptrs = (ctypes.c_void_p * nseg)(*[None if t is None else t.data_ptr() for t in ring])
        ms = None if markers is None else markers.struct()
        if markers is not None:
            assert poses.is_contiguous() and poses.shape[0] >= nseg
        if wrench is not None:
            assert wrench.is_contiguous() and wrench.dtype == torch.float32 and wrench.shape[0] >= nseg
        _check(lib().lbm_adjoint_record(self.ctx, _ptr(ckpt), ptrs, nseg, None if ms is None else ctypes.byref(ms),
                                        _ptr(poses), fr.ctypes.data_as(ctypes.c_void_p), _ptr(ib_ring),
                                        _ptr(wrench)), "lbm_adjoint_record")

    def check(self) -> int:
        return lib().lbm_check(self.ctx)

    def step_count(self) -> int:
        return lib().lbm_step_count(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lib().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many workloads (inputs.Workload, each with markers) advanced together
    by the batched kernels; every environment owns a Simulation. Per-step
    poses, frames and wrenches live on the device for `nsteps` steps of a run
    (a run re-reads them from step 0). storage: one population format for
    every environment ("f32", "f16", "bf16") or a sequence, one per
    environment; the persistent driver takes "f32" and direct forcing only
    (the per-phase driver also takes the implicit correction, when every
    environment uses it)."""

    def __init__(self, workloads, nsteps, block=(128, 4), max_active_tiles=1024, device="cuda", keep_wrench=True,
                 storage="f32"):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice Boltzmann library runs only on the GPU")
        L = lib()
        self.device = torch.device(device)
        self.nsteps = int(nsteps)
        self.stream = torch.cuda.Stream(self.device)  # default priority
        self.sims, self.markers, self.poses, self.frames, self.wrench = [], [], [], [], []
        envs = (Env * len(workloads))()
        with torch.cuda.stream(self.stream):
            formats = [storage] * len(workloads) if isinstance(storage, str) else list(storage)
            assert len(formats) == len(workloads)
            for j, w in enumerate(workloads):
                ntiles = ((w.nx + 7) // 8) * ((w.ny + 7) // 8) * ((w.nz + 7) // 8)
                sim = Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=formats[j], max_markers=w.markers.n,
                                 max_bones=w.markers.nbones, mdf_iters=w.mdf_iters, ib_alpha=w.ib_alpha,
                                 u0=w.u0.astype(np.float32), device=self.device, block=block,
                                 max_active_tiles=min(ntiles, max_active_tiles), stream=self.stream,
                                 bc_y=w.bc_y, bc_z=w.bc_z, ib_scheme=w.ib_scheme, collision=w.collision,
                                 trt_lambda=w.trt_lambda, wall_mode=w.wall_mode)
                dm = DeviceMarkers(w.markers, self.device)
                poses = torch.as_tensor(np.ascontiguousarray(w.poses[:self.nsteps], np.float32), device=self.device)
                frames = torch.as_tensor(np.ascontiguousarray(w.frames[:self.nsteps], np.float64), device=self.device)
                wr = torch.zeros((self.nsteps, 8), dtype=torch.float32, device=self.device) if keep_wrench else None
                rot = bool(np.any(w.frames[:self.nsteps, 3:9] != 0.0))
                envs[j] = Env(sim.ctx.value, dm.struct(), poses.data_ptr(), frames.data_ptr(),
                              None if wr is None else wr.data_ptr(), 1 if rot else 0)
                self.sims.append(sim)
                self.markers.append(dm)
                self.poses.append(poses)
                self.frames.append(frames)
                self.wrench.append(wr)
            nb = L.lbm_batch_bytes(len(workloads))
            if nb == 0:
                raise LBMError(-1, "batch size")
            self._dev_raw = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            shift = (-self._dev_raw.data_ptr()) % 256
            self._dev = self._dev_raw[shift:shift + nb]
            b = ctypes.c_void_p()
            _check(L.lbm_batch_create(ctypes.byref(b), envs, len(workloads), _ptr(self._dev),
                                      ctypes.c_void_p(self.stream.cuda_stream)), "lbm_batch_create")
        self.batch = b
        self._envs = envs

    @property
    def ncell(self) -> int:
        return sum(s.ncell for s in self.sims)

    def run(self, nsteps=None, mode="persistent", graph=True):
        n = self.nsteps if nsteps is None else int(nsteps)
        assert n <= self.nsteps
        m = BATCH_PERSISTENT if mode == "persistent" else BATCH_PHASES
        _check(lib().lbm_batch_run(self.batch, n, m, 1 if graph else 0), "lbm_batch_run")

    def autotune(self, reps=5):
        shapes = np.zeros((len(self.sims), 2), dtype=np.int32)
        _check(lib().lbm_batch_autotune(self.batch, int(reps), shapes.ctypes.data_as(ctypes.c_void_p)),
               "lbm_batch_autotune")
        return shapes

    def set_shapes(self, shapes):
        a = np.ascontiguousarray(shapes, dtype=np.int32).reshape(len(self.sims), 2)
        _check(lib().lbm_batch_set_shapes(self.batch, a.ctypes.data_as(ctypes.c_void_p)), "lbm_batch_set_shapes")

    def set_groups(self, ngroups):
        """Run the per-phase driver as `ngroups` concurrent, cell-balanced
        groups, each on a stream of its own (default priority); 1 drops them."""
        L = lib()
        n = int(ngroups)
        if n == 1:
            _check(L.lbm_batch_set_groups(self.batch, 1, None, None), "lbm_batch_set_groups")
            self._groups = None
            return
        nb = L.lbm_batch_group_bytes(len(self.sims), n)
        if nb == 0:
            raise LBMError(-1, "group count")
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        shift = (-raw.data_ptr()) % 256
        streams = [torch.cuda.Stream(self.device) for _ in range(n)]  # default priority
        arr = (ctypes.c_void_p * n)(*[s.cuda_stream for s in streams])
        _check(L.lbm_batch_set_groups(self.batch, n, arr, ctypes.c_void_p(raw.data_ptr() + shift)),
               "lbm_batch_set_groups")
        self._groups = (raw, streams)

    def check(self) -> int:
        return lib().lbm_batch_check(self.batch)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "batch", None):
            lib().lbm_batch_destroy(self.batch)
            self.batch = None
        self._groups = None
        for s in getattr(self, "sims", []):
            s.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def header_functions(path: str = HEADER_PATH):
    """Names of the functions declared in the public header."""
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))
