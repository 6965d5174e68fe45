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

# Share of (voxel, direction) pairs whose neighbour lies in another 4x4x4
# brick of the default lattice layout (one 128-byte line per brick): a hop's
# source and target words then sit in different lines.  Counted over the
# stencils of section 2.1 (HCP) and its ABC-stacked form (FCC).
CROSS_BRICK_FRACTION = {"hcp": 11.0 / 32.0, "fcc": 45.0 / 128.0}


# the device code of the walk-stage kernel whose traffic the counter summary
# holds (its translation units and every header they include): a change to
# any of them makes the summary stale
KERNEL_SOURCES = ("psc_stage_hcp.hip", "psc_stage_fcc.hip", "psc_stage_impl.h", "psc_device.h",
                  "psc_core.h")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1605_03726_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload_name: str):
    """HBM bytes per walk-stage launch and per attempt from the committed
    rocprofv3 counter summary (averages over the timed events of the default
    command), or None if absent or taken from a different kernel source."""
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
        return {"per_dispatch": float(kv["traffic_bytes_per_dispatch"]),
                "per_attempt": float(kv["traffic_bytes_per_attempt"])}
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
    if name == "mapk_paper":
        return workload("mapk_paper")
    if name == "births":
        return workload("births")
    if name == "membrane":
        return dict(workload("membrane", dims=(256, 256, 256), seed=5, events=2000),
                    track_displacement=False, name="membrane_256x256x256")
    if name == "multiproduct":
        return dict(workload("multiproduct", dims=(256, 256, 256), seed=3, n_a=100000,
                             events=2000), track_displacement=False,
                    name="multiproduct_256x256x256")
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(w: dict, events: int) -> dict:
    """the oracle on one core over the first events of the same workload, in
    the coloured-stage order the GPU follows (the reported value) and in the
    paper's sequential order; setup excluded from the timing"""
    import oracle

    def timed(mode):
        o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                          boundary=oracle.REFLECT if w.get("boundary") == "walls"
                          else oracle.PERIODIC,
                          lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
        for _, D in w["species"]:
            o.add_species(D)
        for r, p, k in w["reactions"]:
            o.add_reaction(r, p, k)
        if w.get("compartments") is not None:
            o.set_compartments(w["compartments"])
        for s, c in w["place"]:
            o.place_uniform(s, c)
        for s, c, cc in w.get("place_in", []):
            o.place_uniform_in(s, c, cc)
        t0 = time.perf_counter()
        o.run(events, mode)
        dt = time.perf_counter() - t0
        att = o.state(with_occ=False)["attempts"]
        o.close()
        return att, dt

    att, dt = timed(oracle.MODE_C)
    att_s, dt_s = timed(oracle.MODE_S)
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"value": att / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": "first %d events of %s (%d attempts, %.1f s), coloured-stage order"
                      % (events, w["name"], att, dt),
            "sequential_order": {"value": att_s / dt_s, "attempts": att_s, "s": dt_s,
                                 "cores": 1,
                                 "kind": "oracle in the paper's order (species, then ascending "
                                         "id; Gillespie's method for first order)"},
            "host_cpus": os.cpu_count(), "host_cpus_usable": usable}


def ensemble_bench(n_members: int, events: int, plain_events: int, trial_events: int) -> dict:
    """Replicate ensemble: all members in batched launches (autotuned shape)
    for `events` events, against the plain form, every member alone (one
    lattice per launch sequence, the launches of psc_step) for `plain_events`
    events, scaled to `events` by the event count only."""
    import torch
    from paper_1605_03726_amd import psc
    from psc_inputs import ensemble_members

    ws = ensemble_members(n=n_members, events=events)
    t0 = time.perf_counter()
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    c0 = sum(l.counters()["attempts"] for l in lats)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ens.autotune(trial_events)
    torch.cuda.synchronize()
    ev0.record(stream)
    ens.step(events)
    ev1.record(stream)
    torch.cuda.synchronize()
    batched_s = ev0.elapsed_time(ev1) / 1e3
    ens.sync()
    attempts = sum(l.counters()["attempts"] for l in lats) - c0
    tuned = ens.tuned()
    ens.close()
    for l in lats:
        l.close()
    del lats

    # the plain form, measured on every member: its events only are timed
    # (model, placement and the freeze happen before)
    plain_measured_s = 0.0
    plain_attempts = 0
    for w in ws if plain_events > 0 else []:
        lat = psc.lattice_from_workload(w)
        lat.step(0)
        lat.sync()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.step(plain_events)
        b.record(stream)
        torch.cuda.synchronize()
        plain_measured_s += a.elapsed_time(b) / 1e3
        plain_attempts += lat.counters()["attempts"]
        lat.close()
    plain_s = plain_measured_s * events / plain_events if plain_events > 0 else None
    return {"members": n_members, "events": events, "edges": [32, 48, 64, 96, 128],
            "batched_s": batched_s, "attempts": attempts,
            "batched_attempts_per_s": attempts / batched_s,
            "plain_measured_s": plain_measured_s, "plain_measured_events": plain_events,
            "plain_measured_attempts_per_s": (plain_attempts / plain_measured_s
                                              if plain_events > 0 else None),
            "plain_s": plain_s, "speedup": plain_s / batched_s if plain_s else None,
            "tuned_launch": tuned, "setup_s": setup_s,
            "plain_form": "all %d members one after another, one lattice per launch sequence "
                          "(psc_step), %d events each, timed; scaled to %d events by the event "
                          "count" % (n_members, plain_events, events),
            "equal_accuracy": "members are bit-identical in both forms (tests)"}


def serving_bench(duration: float, rate: float, budget_gb: float, quantum: int,
                  drain_s: float, max_active: int) -> dict:
    """Poisson arrivals submitted in real time to the continuous-batching
    server for `duration` seconds; then at most `drain_s` more seconds for the
    backlog, after which every unfinished job is cancelled.  Latency =
    completion - submission, over the jobs done; the queue is sampled every
    second."""
    import threading

    import numpy as np
    from paper_1605_03726_amd import psc
    from psc_inputs import serving_jobs

    jobs = serving_jobs(rate=rate, duration=duration)
    srv = psc.Server(budget_bytes=int(budget_gb * (1 << 30)), quantum_events=quantum,
                     max_active=max_active)
    samples = []
    stop = threading.Event()
    t0 = time.perf_counter()

    def sampler():
        while not stop.is_set():
            st = srv.stats()
            samples.append([round(time.perf_counter() - t0, 2), st["queued"], st["active"],
                            st["done"], round(st["device_bytes_in_use"] / 2**30, 2)])
            stop.wait(1.0)

    th = threading.Thread(target=sampler, daemon=True)
    th.start()
    ids = []
    for w in jobs:
        dt = w["arrival"] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(srv.submit(w))
    deadline = t0 + duration + drain_s
    while time.perf_counter() < deadline:
        st = srv.stats()
        if st["done"] + st["failed"] >= len(ids):
            break
        time.sleep(0.2)
    t_cap = time.perf_counter() - t0
    at_cap = srv.stats()
    sts = [srv.poll(j) for j in ids]
    unfinished = [j for j, s in zip(ids, sts) if s["state"] in (psc.JOB_QUEUED, psc.JOB_RUNNING)]
    for j in unfinished:
        try:
            srv.cancel(j)
        except psc.PscError:
            pass  # finished meanwhile
    stop.set()
    th.join()
    final = [srv.wait(j) for j in ids]
    srv.close()
    done = [s for s in final if s["state"] == psc.JOB_DONE]
    lat = np.array([s["done_s"] - s["submit_s"] for s in done]) if done else np.zeros(1)
    t_last = max([s["done_s"] for s in done], default=t_cap)
    attempts = sum(s["attempts"] for s in done)
    work = [sum(c for _, c in w["place"]) * w["events"] for w in jobs]
    offered = sum(work) / duration
    left = sum(wk for wk, s in zip(work, final) if s["state"] != psc.JOB_DONE)
    return {"arrival_rate": rate, "arrival_window_s": duration, "drain_cap_s": drain_s,
            "jobs": len(jobs), "done": len(done),
            "cancelled_at_cap": sum(s["state"] == psc.JOB_CANCELLED for s in final),
            "failed": sum(s["state"] == psc.JOB_FAILED for s in final),
            "wall_s": t_last, "jobs_per_s": len(done) / t_last,
            "attempts_per_s": attempts / t_last,
            "offered_attempts_per_s_upper": offered,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "backlog_at_cap": {"t_s": round(t_cap, 2), "queued": at_cap["queued"],
                               "running": at_cap["active"],
                               "offered_attempts_left": left},
            "queue_depth": {"columns": ["t_s", "queued", "running", "done", "budget_gib_in_use"],
                            "samples": samples[::5]},
            "budget_gb": budget_gb, "quantum_events": quantum, "max_active": max_active,
            "peak_resident_jobs": at_cap["peak_active"], "batched_steps": at_cap["quanta"],
            "note": "offered load exceeds one GPU: latency includes queueing; jobs not done "
                    "by the cap are cancelled and counted in the backlog"}


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


def random_reference(n_words: int, n_access: int, reps: int) -> dict:
    """Reference times for scattered 2-byte accesses: torch's own gather
    (index_select), scatter (index_put_) and gather-then-scatter at the same
    positions, each over n_access uniformly random words of an n_words int16
    array, with fresh positions every repetition (no cache reuse between
    them); microseconds per call, event-timed.  Library kernels, not a
    ceiling: what a plain random probe of the same count costs on this
    memory system."""
    import torch
    x = torch.zeros(n_words, dtype=torch.int16, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(12345)
    idx = [torch.randint(0, n_words, (n_access,), device="cuda", generator=g) for _ in range(reps)]
    y = torch.empty(n_access, dtype=torch.int16, device="cuda")
    vals = torch.ones(n_access, dtype=torch.int16, device="cuda")

    def timed(fn):
        fn(idx[0])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in idx:
            fn(i)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1000.0 / len(idx)

    def gather(i):
        torch.index_select(x, 0, i, out=y)

    def scatter(i):
        x.index_put_((i,), vals)

    def both(i):
        torch.index_select(x, 0, i, out=y)
        x.index_put_((i,), y)

    out = {name + "_us": round(timed(fn), 2)
           for name, fn in (("gather", gather), ("scatter", scatter), ("gather_then_scatter", both))}
    del x, idx, y, vals
    torch.cuda.empty_cache()
    return out


def calibrate_random(n_words: int, n_access: int, reps: int):
    out = {"calibrate_random_words": n_words, "accesses": n_access, "reps": reps}
    out.update(random_reference(n_words, n_access, reps))
    for name in ("gather", "scatter", "gather_then_scatter"):
        out[name + "_accesses_per_s"] = n_access / (out[name + "_us"] * 1e-6)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cfg3",
                    choices=["cfg1", "cfg2", "cfg3", "mapk_paper", "multiproduct", "births",
                             "membrane"])
    ap.add_argument("--timing-steps", type=int, default=40,
                    help="events after the timed region whose launches are timed one by one")
    ap.add_argument("--graph", action="store_true",
                    help="replay each event's launches from a HIP graph (psc_set_graph_replay)")
    ap.add_argument("--walls", action="store_true",
                    help="close the workload's box by walls instead of wrapping it")
    ap.add_argument("--fcc", action="store_true",
                    help="the workload on the FCC lattice (nk rounded down to a multiple of 12)")
    ap.add_argument("--cpu-events", type=int, default=4,
                    help="events of the workload the CPU oracle runs (about 10-30 s of CPU work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-only", action="store_true")
    ap.add_argument("--ensemble-members", type=int, default=512)
    ap.add_argument("--ensemble-events", type=int, default=5000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--serving-window", type=float, default=60.0,
                    help="seconds of Poisson arrivals (200 jobs/s)")
    ap.add_argument("--serving-drain", type=float, default=15.0,
                    help="seconds after the arrivals before unfinished jobs are cancelled")
    ap.add_argument("--serving-max-active", type=int, default=1024)
    ap.add_argument("--plain-events", type=int, default=200,
                    help="events each ensemble member runs alone in the plain form")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run N-byte device copies (counter calibration)")
    ap.add_argument("--calibrate-random", type=int, default=0,
                    help="only time N scattered 2-byte gathers/scatters into a 2^32-word array")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU (got --gpus %d): one lattice's walk runs on one "
              "MI355X; replicates and jobs shard over GPUs without exchange" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, 10)
        return
    if args.calibrate_random:
        calibrate_random(1 << 32, args.calibrate_random, 50)
        return

    import torch
    from paper_1605_03726_amd import psc

    if args.serving_only:
        print(json.dumps(serving_bench(args.serving_window, 200.0, 200.0, 64, args.serving_drain,
                                       args.serving_max_active)))
        return
    if args.ensemble_only:
        print(json.dumps(ensemble_bench(args.ensemble_members, args.ensemble_events,
                                        args.plain_events, 3)))
        return

    w = pick_workload(args.workload)
    if args.fcc:
        # FCC boxes: i and j edges multiples of 8, k of 12
        ni, nj, nk = (int(x) for x in w["dims"])
        d8 = (8 * (ni // 8), 8 * (nj // 8), 12 * (nk // 12))
        w = dict(w, lattice="fcc", dims=d8,
                 name="%s_%dx%dx%d_fcc" % (w["name"].rsplit("_", 1)[0], *d8))
    if args.walls:
        w = dict(w, boundary="walls", name=w["name"] + "_walls")
    nv = int(w["dims"][0]) * int(w["dims"][1]) * int(w["dims"][2])
    placed = sum(c for _, c in w["place"]) + sum(c for _, c, _ in w.get("place_in", []))
    t_setup = time.perf_counter()
    lat = psc.lattice_from_workload(
        w, max_molecules=w.get("max_molecules", min(nv, int(placed * 1.25) + 4096)))
    if args.graph:
        lat.set_graph_replay(True)
    stream = torch.cuda.current_stream()
    lat.step(args.warmup)
    lat.sync()
    setup_s = time.perf_counter() - t_setup
    print("setup + warmup %.1f s" % setup_s, file=sys.stderr, flush=True)

    # ---- timed region: K events of plain launches, HIP events on the launch
    # stream before and after ----
    stages = 16  # colour stages per event on either lattice
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

    # ---- launch times, right after the timed region: every launch of the
    # next `timing_steps` events between HIP events on the launch stream (a
    # pass of its own, so that the event records do not perturb the timed
    # region) ----
    tsteps = max(args.timing_steps, 1)
    lat.set_kernel_timing(True)
    ct0 = lat.counters()
    lat.step(tsteps)
    lat.set_kernel_timing(False)
    kt = lat.kernel_times()
    ct1 = lat.counters()
    s_att = ct1["attempts"] - ct0["attempts"]
    s_hops = ct1["hops"] - ct0["hops"]

    # ---- the dominant kernel (the walk stage) against the HBM roofline:
    # algorithmic bytes of the timed region per stage launch over the
    # sampled launches' average time ----
    stage_avg_ms = kt["stage_ms"] / max(kt["stage_launches"], 1)
    launches = tsteps * stages
    t_att = s_att / launches
    alg_bytes_per_launch = (6.0 * s_att + 8.0 * s_hops) / launches
    achieved = alg_bytes_per_launch / (stage_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(w["name"])
    lat.close()
    # the same count of scattered 2-byte accesses in an array of the lattice's
    # size, done by torch's gather and scatter kernels alone: the target read
    # and the write to its line (gather then scatter), plus the source write
    # for the hops whose target lies in another 4x4x4 brick (another line)
    ref = random_reference(nv, max(int(round(t_att)), 1), 20)
    cross = CROSS_BRICK_FRACTION[w.get("lattice", "hcp")]
    ref_us = ref["gather_then_scatter_us"] + cross * ref["scatter_us"]

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
                   "boundary": w.get("boundary", "periodic"),
                   "lattice": w.get("lattice", "hcp"),
                   "species": len(w["species"]), "reactions": len(w["reactions"]),
                   "step": "one diffusion event", "hop_fraction": hops / max(attempts, 1),
                   "launch": "graph replay" if args.graph else "direct launches"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # HBM bytes per launch: the profile's bytes per attempt
                     # (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain
                     # copy) times this run's attempts per launch
                     "traffic": traffic["per_attempt"] * t_att if traffic else None,
                     "traffic_profiled_per_dispatch": traffic["per_dispatch"] if traffic else None,
                     "kernel": "k_stage (one colour stage of the walk)",
                     "avg_launch_ms": stage_avg_ms,
                     "timed_launches_sampled": kt["stage_launches"],
                     "algorithmic_bytes_per_launch": alg_bytes_per_launch,
                     "attempts_per_launch": t_att,
                     # measured HBM bytes per attempt (profile), the rate they
                     # imply at the live launch time, and the share of them the
                     # method needs
                     "traffic_per_attempt": traffic["per_attempt"] if traffic else None,
                     "traffic_gbs": (traffic["per_attempt"] * t_att
                                     / (stage_avg_ms * 1e-3) / 1e9 if traffic else None),
                     "useful_byte_fraction": (alg_bytes_per_launch / t_att
                                              / traffic["per_attempt"] if traffic else None),
                     },
        # beside the roofline, not part of it: the HBM rate a walk that
        # streamed the whole lattice (read and write 2 B per voxel per event)
        # would need for the measured event rate, and the time torch's own
        # gather and scatter take for the walk stage's scattered accesses
        "context": {
            "stream_equivalent_gbs": 4.0 * nv / (ms / args.steps * 1e-3) / 1e9,
            "random_access_reference": dict(
                ref, cross_line_fraction=cross, estimate_us=ref_us,
                walk_over_reference=stage_avg_ms * 1e3 / ref_us,
                kind="torch index_select / index_put_ of attempts_per_launch random "
                     "2-byte words in an array of the lattice's size, event-timed")},
    }
    if not args.no_ensemble:
        result["ensemble"] = ensemble_bench(args.ensemble_members, args.ensemble_events,
                                            args.plain_events, 3)
        print("ensemble: %.2f s batched, %s over plain" % (
            result["ensemble"]["batched_s"], result["ensemble"]["speedup"]), file=sys.stderr,
            flush=True)
    if not args.no_serving:
        result["serving"] = serving_bench(args.serving_window, 200.0, 200.0, 64,
                                          args.serving_drain, args.serving_max_active)
        print("serving: %d jobs, p50 %.2f s, p99 %.2f s" % (
            result["serving"]["done"], result["serving"]["latency_p50_s"],
            result["serving"]["latency_p99_s"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_events)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
