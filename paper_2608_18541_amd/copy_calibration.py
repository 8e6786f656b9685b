"""Plain device-to-device copy of a known size (1 GiB, three times).

Run under ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` it gives
the counters' reading for a copy whose HBM traffic is known exactly (1 GiB
read and 1 GiB written per copy), which calibrates the same counters taken
on the spin-lattice kernels.
"""
import torch


def main() -> None:
    n = 256 << 20                      # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d bytes three times" % (4 * n))


if __name__ == "__main__":
    main()
