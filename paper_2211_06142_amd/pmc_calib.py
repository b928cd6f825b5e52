"""Calibration program for HBM traffic counters: one device-to-device copy of
a known size (256 MiB read, 256 MiB written), run under
  rocprofv3 --pmc FETCH_SIZE -- python paper_2211_06142_amd/pmc_calib.py
and again with WRITE_SIZE; the counters of the copy kernel divided by 262144
KiB give the factor that scales the counters of the DEM kernels to bytes."""
import torch


def main():
    n = 256 * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("pmc_calib: 3 copies of %d bytes" % (4 * n), flush=True)


if __name__ == "__main__":
    main()
