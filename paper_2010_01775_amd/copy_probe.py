"""Copy kernel of known size, for calibrating HBM byte counters.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2010_01775_amd.copy_probe

copies a 1 GiB device buffer into another 8 times; each dispatch must read
and write 2^30 bytes, so FETCH_SIZE / WRITE_SIZE per dispatch divided by
2^30 gives the counters' scale factor.
"""
import torch


def main(nbytes: int = 1 << 30, reps: int = 8):
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x {reps}")


if __name__ == "__main__":
    main()
