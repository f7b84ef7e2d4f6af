"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE / WRITE_SIZE) of rocprofv3: the counters read for
this copy are compared with the 2 x 512 MiB it must move.

Usage: python paper_2112_14064_amd/copy_probe.py
"""
import torch

NBYTES = 512 * 1024 * 1024


def main():
    a = torch.ones(NBYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {NBYTES} bytes 3 times")


if __name__ == "__main__":
    main()
