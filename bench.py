"""Benchmark of the lattice walk on one MI355X.

One step = one diffusion event of the whole hot path (first-order pass, the 16
colour stages of the walk with collision reactions, re-binning, flag sweep)
over the workload's lattice.  Default workload: the 2^32-voxel MAPK-style
lattice (2048 x 2048 x 1024, 0.3 % occupancy, 10 species, 8 second-order and
10 first-order reactions), inputs resident in HBM before timing starts.

Prints one JSON line: hop attempts/s, the walk-stage kernel against the HBM
roofline (algorithmic bytes: 6 B per attempt + 8 B per hop), and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("psc_kernels.hip", "psc_core.h"):
        with open(os.path.join(ROOT, "paper_1605_03726_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload_name: str):
    """HBM bytes per walk-stage launch from the committed rocprofv3 counter
    summary, or None if absent or taken from a different kernel source."""
    path = os.path.join(PROFILE_DIR, "walk_stage_traffic_%s.txt" % workload_name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def pick_workload(name: str):
    from psc_inputs import workload
    if name == "cfg3":
        return workload("cfg3")
    if name == "cfg2":
        return workload("cfg2")
    if name == "cfg1":
        return workload("cfg1")
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(w: dict, events: int) -> dict:
    """the oracle (coloured-stage mode, single thread) on the first events of
    the same workload; setup excluded from the timing"""
    import oracle
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"])
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    t0 = time.perf_counter()
    o.run(events, oracle.MODE_C)
    dt = time.perf_counter() - t0
    att = o.state(with_occ=False)["attempts"]
    o.close()
    return {"value": att / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": "first %d events of %s (%d attempts, %.1f s)" % (events, w["name"], att, dt)}


def calibrate_copy(nbytes: int, reps: int):
    """plain device-to-device copies of a known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters"""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cfg3", choices=["cfg1", "cfg2", "cfg3"])
    ap.add_argument("--timing-steps", type=int, default=40)
    ap.add_argument("--cpu-events", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run N-byte device copies (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the walk of a "
              "single lattice is measured on one MI355X" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, 10)
        return

    import torch
    from paper_1605_03726_amd import psc

    w = pick_workload(args.workload)
    nv = int(w["dims"][0]) * int(w["dims"][1]) * int(w["dims"][2])
    placed = sum(c for _, c in w["place"])
    t_setup = time.perf_counter()
    lat = psc.lattice_from_workload(w, max_molecules=min(nv, int(placed * 1.25) + 4096))
    stream = torch.cuda.current_stream()
    lat.step(args.warmup)
    lat.sync()
    setup_s = time.perf_counter() - t_setup
    print("setup + warmup %.1f s" % setup_s, file=sys.stderr, flush=True)

    # ---- timed region: K events, HIP events on the launch stream ----
    c0 = lat.counters()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    c1 = lat.counters()
    attempts = c1["attempts"] - c0["attempts"]
    hops = c1["hops"] - c0["hops"]
    print("timed %d events: %.2f ms, %d attempts" % (args.steps, ms, attempts), file=sys.stderr,
          flush=True)

    # ---- per-kernel times of the dominant kernel (the walk stage) ----
    lat.set_kernel_timing(True)
    c2 = lat.counters()
    lat.step(args.timing_steps)
    kt = lat.kernel_times()
    c3 = lat.counters()
    lat.set_kernel_timing(False)
    t_att = c3["attempts"] - c2["attempts"]
    t_hop = c3["hops"] - c2["hops"]
    stage_launches = max(kt["stage_launches"], 1)
    stage_avg_ms = kt["stage_ms"] / stage_launches
    alg_bytes_per_launch = (6.0 * t_att + 8.0 * t_hop) / stage_launches
    achieved = alg_bytes_per_launch / (stage_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(w["name"])
    lat.close()

    result = {
        "metric": "molecule hop attempts/s",
        "value": attempts / (ms * 1e-3),
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w["name"], "voxels": nv, "molecules": placed,
                   "species": len(w["species"]), "reactions": len(w["reactions"]),
                   "step": "one diffusion event", "hop_fraction": hops / max(attempts, 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage (one colour stage of the walk)",
                     "avg_launch_ms": stage_avg_ms,
                     "algorithmic_bytes_per_launch": alg_bytes_per_launch},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_events)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
