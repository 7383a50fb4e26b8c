"""Workload for the rocprofv3 counter runs: 3 fastqsl_q2d calls on the 256x256x128
cube with 1024x1024 seeds (as timed by bench.py), then one 1 GiB device copy whose
FETCH_SIZE / WRITE_SIZE calibrate the byte counters."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import torch  # noqa: E402

import paper_2208_12569_amd as fq  # noqa: E402
import synth  # noqa: E402

prec = fq.FQ_PREC_F64 if "--f64" in sys.argv else fq.FQ_PREC_F32X
w = synth.config_c2(0)
B = torch.from_numpy(w.field).cuda()
r = fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec))
for _ in range(3):
    r = fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec), ws=r["_ws"])
torch.cuda.synchronize()
x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
y = torch.empty_like(x)
y.copy_(x)
torch.cuda.synchronize()
print("prof_c2 done", flush=True)
