"""Workloads for rocprofv3 runs that bench.py does not make by itself.

    python -m paper_1410_3677_amd.profile_cases rows1024

rows1024: a plain 1 GiB copy (out = x * 1, which calibrates the HBM counters), then one
search of one synthetic segment of N = 150 000 samples (nfft = 2^19: rows of P = 1024
points in the second pass), 16 sky x 64 spindown templates, mixed precision, 256 templates
and 8 skies per batch, without graph capture.  It prints the plan and the candidate count.
"""
from __future__ import annotations

import sys


def rows1024() -> None:
    import numpy as np
    import torch  # before the library: one HIP runtime in the process

    import synth
    from paper_1410_3677_amd import fstat as F

    nel = (1 << 30) // 4
    xc = torch.ones(nel, dtype=torch.float32, device="cuda")
    yc = torch.empty_like(xc)
    torch.mul(xc, 1.0, out=yc)
    torch.cuda.synchronize()
    del xc, yc
    rng = np.random.default_rng(77)
    injs = synth.draw_injections(rng, 2, 12.0, 20.0)
    seg = synth.make_segment(150000, 2.0, 100.0, 1.0, 7150, injs)
    alpha, delta = synth.fibonacci_sky(16)
    fdot = synth.spindown_grid(64)

    def dev(v):
        return torch.as_tensor(v, dtype=torch.float64, device="cuda")

    plan = F.Plan([F.segment_to_device(seg)], precision=F.PREC_MIXED, threshold_2F=20.0,
                  candidate_capacity=1 << 22, templates_per_launch=256, skies_per_batch=8, use_graph=0)
    print(plan.info(), flush=True)
    plan.search_batch(0, dev(alpha), dev(delta), dev(fdot))
    torch.cuda.synchronize()
    print("candidates", plan.candidate_count(), flush=True)
    plan.destroy()


CASES = {"rows1024": rows1024}

if __name__ == "__main__":
    if len(sys.argv) != 2 or sys.argv[1] not in CASES:
        raise SystemExit(f"usage: python -m paper_1410_3677_amd.profile_cases {{{','.join(CASES)}}}")
    CASES[sys.argv[1]]()
