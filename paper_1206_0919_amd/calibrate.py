"""Streaming-copy calibration: the plain copy kernel of libshasta.so moves a
buffer of known size, timed with HIP events on the library call's stream.

    python -m paper_1206_0919_amd.calibrate [--mib 1024] [--reps 10]

Gives the achievable HBM bandwidth (read + write bytes / time) and, run under
rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, the factor between the counters and
the bytes a kernel really moves.
"""
import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    import torch
    from paper_1206_0919_amd import binding as B
    n = args.mib << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    for _ in range(3):
        B.stream_copy(src, dst, n, st)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(args.reps):
        B.stream_copy(src, dst, n, st)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.reps
    assert torch.equal(src, dst)
    print(json.dumps({"copy_bytes_per_launch": n, "hbm_bytes_per_launch": 2 * n,
                      "avg_us": ms * 1000, "GBps": 2 * n / (ms * 1e-3) / 1e9,
                      "launches": args.reps + 3}))


if __name__ == "__main__":
    main()
