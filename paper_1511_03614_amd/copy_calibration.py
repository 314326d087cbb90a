"""Plain device-to-device copy of a known size (256 MiB, three times).

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) to calibrate
what those counters read per byte actually moved on this GPU; the factors scale
the counters of the tile kernel to HBM bytes.
"""
import torch

NBYTES = 256 * 1024 * 1024


def main():
    n = NBYTES // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied bytes per launch:", NBYTES)


if __name__ == "__main__":
    main()
