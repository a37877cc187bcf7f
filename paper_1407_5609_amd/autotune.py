"""Autotuner for the screen configurations.

Runs `cpmi_autotune` on synthetic problems of each (dimension, size) bucket:
float32 points with AUTO precision (the FP32 and the BF16 screen, tile edge
128 and 256) and int8 points (tile edge 128 and 256), and writes the choices
as the JSON tune cache that `cpmi_create` reads. The synthetic inputs are
N(0,1) float32 rows and {0,1,2} int8 rows drawn on the device; screen time
depends on the shape, not on the values, beyond the second-pass selection
that random rows keep small.

    python -m paper_1407_5609_amd.autotune [--out FILE] [--reps 3] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

FLOAT_DIMS = (64, 128, 256, 512)
FLOAT_ROWS = (4096, 16384, 65536, 262144)
INT8_DIMS = (4096,)
INT8_ROWS = (4096, 16384, 100000)


def main(argv=None):
    import torch

    import paper_1407_5609_amd as cp

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=cp.DEFAULT_TUNE_CACHE)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="small shapes only (a check of the tuner itself)")
    args = ap.parse_args(argv)

    ctx = cp.Context(0, tune_cache=None)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(14075609)
    frows = FLOAT_ROWS[:2] if args.quick else FLOAT_ROWS
    irows = INT8_ROWS[:1] if args.quick else INT8_ROWS
    shapes = [("f32", n, d) for d in FLOAT_DIMS for n in frows] + [("i8", n, d) for d in INT8_DIMS for n in irows]
    report = []
    for kind, n, d in shapes:
        if kind == "f32":
            X = torch.randn((n, d), generator=g, device="cuda:0", dtype=torch.float32)
        else:
            X = torch.randint(0, 3, (n, d), generator=g, device="cuda:0", dtype=torch.int8)
        t = time.perf_counter()
        r = ctx.autotune(X, "auto", reps=args.reps)
        r.update(kind=kind, n=n, d=d, seconds=round(time.perf_counter() - t, 2))
        report.append(r)
        print(json.dumps(r), flush=True)
        del X
    ctx.save_tune_cache(args.out)
    print("wrote", os.path.abspath(args.out), flush=True)
    return report


if __name__ == "__main__":
    sys.exit(0 if main() is not None else 1)
