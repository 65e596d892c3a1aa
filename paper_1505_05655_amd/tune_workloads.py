"""Autotune the correction plan for the synthetic single-scene workloads and
save the plan cache next to librc.so (or to --out).

    python paper_1505_05655_amd/tune_workloads.py --workloads 0 1 2 --effort 1

Each workload's seeded inputs are generated on the host, copied to the GPU,
its LUT is built, and rc_tune times the candidate launch shapes on those
buffers. rc_correct then finds the winning plan for any shape of the same
class (levels, detector and line magnitude, bands, vector width).
"""
import argparse
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
import paper_1505_05655_amd as rc  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--effort", type=int, default=1)
    ap.add_argument("--out", default=None, help="plan cache file (default: next to librc.so)")
    ap.add_argument("--fresh", action="store_true", help="start from an empty cache")
    args = ap.parse_args()
    if args.fresh:
        rc.rc_tune_clear()
    dev = torch.device("cuda:0")
    for w in args.workloads:
        s = gen.workload(w)
        dn = torch.from_numpy(s.dn().view(np.int16)).to(dev)
        lut = rc.lut_build(torch.from_numpy(s.coeffs()).to(dev), s.levels)
        out = torch.empty_like(dn)
        plan, us = rc.rc_tune(dn, lut, s.lines, s.detectors, s.bands, s.levels, out,
                              effort=args.effort)
        algo = 4 * s.pixels + s.bands * s.detectors * s.levels * 2
        print(json.dumps({"workload": s.name, "us": round(us, 1),
                          "gb_s": round(algo / (us * 1e-6) / 1e9, 1), "plan": plan.as_dict()}),
              flush=True)
        del dn, lut, out
        torch.cuda.empty_cache()
    n = rc.rc_tune_save(args.out)
    print(f"saved {n} plan(s) to {args.out or 'the default plan cache'}")


if __name__ == "__main__":
    main()
