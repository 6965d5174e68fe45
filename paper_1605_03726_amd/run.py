"""Runs a named workload on the GPU: the lattice is built and frozen, then
stepped for warm-up and measured events, and the counters of the measured
events are printed as one JSON line.  Nothing else runs in the process, which
makes it the program to put under a profiler:

    python -m paper_1605_03726_amd.run --workload cfg3 --warmup 10 --events 30

--copy-bytes N instead copies an N-byte device buffer --reps times (nothing
else), the reference for scaling memory-traffic counters.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--events", type=int, default=30)
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args(argv)

    import torch
    if args.copy_bytes:
        x = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        for _ in range(args.reps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "reps": args.reps}), flush=True)
        return 0

    from paper_1605_03726_amd import psc
    from psc_inputs import workload
    w = workload(args.workload)
    nv = int(w["dims"][0]) * int(w["dims"][1]) * int(w["dims"][2])
    placed = sum(c for _, c in w["place"]) + sum(c for _, c, _ in w.get("place_in", []))
    lat = psc.lattice_from_workload(w, max_molecules=min(nv, int(placed * 1.25) + 4096))
    lat.step(args.warmup)
    lat.sync()
    print("warm-up done", file=sys.stderr, flush=True)
    c0 = lat.counters()
    t0 = time.perf_counter()
    lat.step(args.events)
    lat.sync()
    dt = time.perf_counter() - t0
    c1 = lat.counters()
    out = {"workload": w["name"], "warmup": args.warmup, "events": args.events,
           "stage_launches": 16 * args.events, "wall_s": dt}
    for k in ("attempts", "hops", "collisions", "placement_failures"):
        out[k] = c1[k] - c0[k]
    lat.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
