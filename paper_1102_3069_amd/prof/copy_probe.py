"""A plain device-to-device copy of a known size (default 1 GiB, three times),
used to calibrate the FETCH_SIZE / WRITE_SIZE counters: the counter values
of this copy divided into its true byte count give the scale factors."""
import sys, torch
nbytes = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30
n = nbytes // 4
a = torch.ones(n, device="cuda"); b = torch.empty_like(a)
torch.cuda.synchronize()
for _ in range(3):
    b.copy_(a)
torch.cuda.synchronize()
print("copied", nbytes, "bytes x3", flush=True)
