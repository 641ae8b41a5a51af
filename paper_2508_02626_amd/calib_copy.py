"""Plain device-to-device copy of a known size (256 MiB, twice), used to
calibrate the HBM byte counters (FETCH_SIZE, WRITE_SIZE) read by rocprofv3:
factor = counter reading / bytes the copy must move."""
import torch

NBYTES = 256 << 20


def main():
    x = torch.ones(NBYTES // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes twice" % NBYTES)


if __name__ == "__main__":
    main()
