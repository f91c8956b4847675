"""Plain device-to-device copy of a known size, for calibrating the HBM byte
counters (FETCH_SIZE / WRITE_SIZE) that the sweep's traffic figure uses:
``rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2602_01330_amd.hbm_copy_probe``
copies exactly 1 GiB once (plus one warm-up copy of the same size)."""
import torch

N_BYTES = 1 << 30


def main():
    a = torch.ones(N_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {N_BYTES} bytes twice", flush=True)


if __name__ == "__main__":
    main()
