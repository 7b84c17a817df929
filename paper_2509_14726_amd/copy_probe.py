"""A plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE, WRITE_SIZE) that profiles report for the kernels of
this package: counter / known bytes = the scale applied to their readings."""
import sys

import torch

MIB = int(sys.argv[1]) if len(sys.argv) > 1 else 256
x = torch.ones(MIB * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
y = torch.empty_like(x)
torch.cuda.synchronize()
for _ in range(3):
    y.copy_(x)
torch.cuda.synchronize()
print(f"copied {MIB} MiB three times", flush=True)
