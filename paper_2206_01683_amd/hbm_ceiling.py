"""Practical HBM ceiling on this device: the reference kernels of
libhbmceiling.so (include/hbm_ceiling.h) timed with HIP events on the stream
they run on.

    python -m paper_2206_01683_amd.hbm_ceiling            # all patterns, one JSON line
    python -m paper_2206_01683_amd.hbm_ceiling --only copy --mib 1024 --reps 3

The second form is the calibration run for HBM byte counters: profiled with
`rocprofv3 --pmc FETCH_SIZE` (then `WRITE_SIZE`), the counters read per copy
dispatch, divided by the bytes the copy must move (SIZE read, SIZE written),
give the factor that turns the same counters read on another kernel into
bytes.
"""
import argparse
import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbmceiling.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.hbm_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.hbm_read.argtypes = [vp, ctypes.c_size_t, vp, vp]
        L.hbm_pull27.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int32, vp]
        for f in (L.hbm_copy, L.hbm_read, L.hbm_pull27):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _time(fn, reps: int) -> float:
    """Average milliseconds of fn() over reps launches after two warm-ups."""
    for _ in range(2):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _ok(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with {rc}")


def measure(nx: int = 384, ny: int = 192, nz: int = 192, reps: int = 20) -> dict:
    """GB/s of a copy and a read of 27 nx ny nz floats (the bytes one collide
    reads and writes), and of the collide's pull-27 pattern in both layouts
    (216 B per cell moved)."""
    L = lib()
    cells = nx * ny * nz
    plane = (cells + 255) // 256 * 256 + 192  # the library's plane stride for these sizes
    n = 27 * plane
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.zeros(n, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nbytes = 27 * cells * 4
    pa, pb, ps_ = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(sink.data_ptr())
    out = {"workload": f"{nx}x{ny}x{nz}", "bytes_per_pass": 2 * nbytes}
    ms = _time(lambda: _ok(L.hbm_copy(pa, pb, nbytes, s), "hbm_copy"), reps)
    out["copy"] = {"us": round(ms * 1e3, 2), "GBps": round(2 * nbytes / ms / 1e6, 1)}
    ms = _time(lambda: _ok(L.hbm_read(pa, nbytes, ps_, s), "hbm_read"), reps)
    out["read"] = {"us": round(ms * 1e3, 2), "GBps": round(nbytes / ms / 1e6, 1)}
    for name, (ps, rs, cap) in (("pull27_rows", (nx, 27 * nx, 0)), ("pull27_planes", (plane, nx, 0)),
                                ("pull27_rows_3_blocks_per_cu", (nx, 27 * nx, 3))):
        ms = _time(lambda: _ok(L.hbm_pull27(pa, pb, nx, ny, nz, ps, rs, cap, s), "hbm_pull27"), reps)
        out[name] = {"us": round(ms * 1e3, 2), "GBps": round(2 * nbytes / ms / 1e6, 1)}
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    out["runtime_copy"] = {"us": round(ms * 1e3, 2), "GBps": round(2 * n * 4 / ms / 1e6, 1)}
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--only", choices=("copy",), default=None, help="only the copy, for counter calibration")
    ap.add_argument("--mib", type=int, default=1024, help="--only copy: bytes copied per dispatch, in MiB")
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if a.only == "copy":
        nbytes = a.mib * (1 << 20)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        ms = _time(lambda: _ok(lib().hbm_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                               nbytes, s), "hbm_copy"), a.reps)
        print(f"hbm_copy of {a.mib} MiB x {a.reps + 2} dispatches: {ms:.3f} ms per copy = "
              f"{2 * nbytes / ms / 1e6:.0f} GB/s read + write", flush=True)
        return
    print(json.dumps(measure(reps=a.reps)), flush=True)


if __name__ == "__main__":
    main()
