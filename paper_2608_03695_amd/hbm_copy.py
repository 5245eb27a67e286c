"""A plain 1 GiB device-to-device copy, run under rocprofv3 --pmc to calibrate the
FETCH_SIZE / WRITE_SIZE counters: each copy reads and writes exactly 2^30 bytes.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2608_03695_amd.hbm_copy
"""
import torch


def main():
    n = 1 << 28                      # 2^28 int32 = 1 GiB
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x", b.numel() * 4, "bytes", flush=True)


if __name__ == "__main__":
    main()
