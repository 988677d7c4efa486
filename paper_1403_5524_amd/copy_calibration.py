"""Plain device copy of known size, for calibrating HBM byte counters.

Run under ``rocprofv3 --pmc FETCH_SIZE`` and again under ``--pmc WRITE_SIZE``:
each of the three copies reads and writes exactly 1 GiB, so the counters'
readings for ``__amd_rocclr_copyBuffer`` give the factor from counter units
to bytes moved.

    python -m paper_1403_5524_amd.copy_calibration
"""
import torch


def main():
    n = (1 << 30) // 8
    x = torch.empty(n, dtype=torch.float64, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copy_calibration: 3 copies of 1 GiB done", flush=True)


if __name__ == "__main__":
    main()
