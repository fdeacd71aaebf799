"""Calibration run for HBM byte counters: a plain device-to-device copy of a
known size, repeated. Profiled with `rocprofv3 --pmc FETCH_SIZE` (then
`WRITE_SIZE`), the counters read per copy dispatch, divided by the bytes the
copy must move (SIZE read, SIZE written), give the factor that turns the same
counters read on another kernel into bytes. It also prints the copy's own
read + write bandwidth, a reference ceiling for streaming kernels.

    python -m paper_2206_01683_amd.hbm_copy [--mib 1024] [--reps 5]
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--mib", type=int, default=1024, help="bytes copied per dispatch, in MiB")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(a.reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / a.reps
    gbs = 2 * a.mib * (1 << 20) / (ms * 1e-3) / 1e9
    print(f"copied {a.mib} MiB x {a.reps}: read {a.mib} MiB and wrote {a.mib} MiB per dispatch, "
          f"{ms:.3f} ms per copy = {gbs:.0f} GB/s read + write", flush=True)


if __name__ == "__main__":
    main()
