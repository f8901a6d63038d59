"""Reference copy for scaling hardware traffic counters.

Copies a float64 buffer of known size on the GPU (one read and one write of `mib` MiB)
so that rocprofv3's FETCH_SIZE and WRITE_SIZE for that dispatch can be compared with
the exact byte count: the ratio is the factor applied to the solver kernel's counters.
Usage: python -m paper_2604_22625_amd.copyprobe [mib]
"""
import sys

import torch


def main(mib: int = 256) -> None:
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copyprobe: {mib} MiB read + {mib} MiB written per copy ({n * 8} bytes each way)", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 256)
