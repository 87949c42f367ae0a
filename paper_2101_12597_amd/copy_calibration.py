"""A plain device-to-device copy of a known size, for calibrating HBM traffic counters.

  python3 -m paper_2101_12597_amd.copy_calibration [MiB]

copies MiB mebibytes (default 1024) once with torch's copy_ (one
__amd_rocclr_copyBuffer dispatch) after an untimed warm-up copy.  Run under
rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE), the counter of the second dispatch
divided by the bytes read (written) gives the factor that turns the counter into
bytes for the other kernels.
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)  # warm-up
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB", flush=True)


if __name__ == "__main__":
    main()
