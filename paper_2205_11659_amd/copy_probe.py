"""Calibration probe for HBM byte counters: a plain device-to-device copy of
a known size (1 GiB), repeated.  Profiled with rocprofv3's FETCH_SIZE and
WRITE_SIZE counters, the ratio of the true bytes to what the counters report
for this copy kernel is the factor applied to the counters of the library's
own kernels.

    python3 paper_2205_11659_amd/copy_probe.py
"""
import torch

NBYTES = 1 << 30


def main(reps: int = 3) -> None:
    dev = torch.device("cuda:0")
    src = torch.ones(NBYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {NBYTES} bytes x {reps}", flush=True)


if __name__ == "__main__":
    main()
