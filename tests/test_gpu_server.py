"""Serving loop on the GPU: jobs submitted while others run are admitted at
step boundaries as memory frees up, their work overlaps in the batched
steps, and every result equals the same job run alone (bit for bit; the
small ones also equal the CPU oracle).  Failure paths, forced from the host:
an invalid job and an oversize job fail with a status and leave the others
unchanged; a tiny memory budget makes jobs wait but changes no result."""
import time

import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import serving_jobs, workload

pytestmark = pytest.mark.gpu


def small_jobs(n, seed=3):
    js = serving_jobs(rate=50.0, duration=10.0, seed=seed, edge_range=(12, 40),
                      phi_range=(0.01, 0.06), event_range=(20, 120))
    return js[:n]


def alone(w):
    lat = psc.lattice_from_workload(w)
    lat.step(w["events"])
    return lat.read_state()


def oracle_state(w):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
                      lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    o.run(w["events"], oracle.MODE_C)
    return o.state()


def same(a, b):
    for key in ("occ", "id", "vox", "species"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
        assert a[key] == b[key], (key, a[key], b[key])
    assert a["time"] == b["time"]
    assert np.array_equal(a["fired"], b["fired"])


def cap_of(w):
    nv = int(np.prod(w["dims"]))
    return min(nv, max(1024, int(sum(c for _, c in w["place"]) * 1.5) + 1024))


def test_results_same_alone_and_in_the_mix():
    jobs = small_jobs(24)
    # every third job is closed by walls, every fourth is an FCC lattice
    jobs = [dict(w, boundary="walls") if i % 3 == 1 else w for i, w in enumerate(jobs)]
    jobs = [dict(w, lattice="fcc", dims=(8 * max(1, w["dims"][0] // 8), 8 * max(1, w["dims"][1] // 8),
                                       12 * max(1, w["dims"][2] // 12)))
            if i % 4 == 2 else w for i, w in enumerate(jobs)]
    srv = psc.Server(budget_bytes=8 << 30, quantum_events=16)
    ids = []
    for i, w in enumerate(jobs):
        ids.append(srv.submit(w, keep_state=True))
        if i % 6 == 5:
            time.sleep(0.05)  # later arrivals join running jobs at step boundaries
    states = []
    for jid in ids:
        st = srv.wait(jid)
        assert st["state"] == psc.JOB_DONE, st
    for w, jid in zip(jobs, ids):
        s = srv.read_state(jid, cap_of(w))
        same(s, alone(w))
        states.append(s)
    for w, s in list(zip(jobs, states))[:6]:
        same(s, oracle_state(w))
    stats = srv.stats()
    assert stats["done"] == len(jobs) and stats["quanta"] > 1
    # the jobs overlapped: fewer batched steps than the sum of their events
    assert stats["quanta"] * 16 < sum(w["events"] for w in jobs)
    srv.close()


def test_tiny_budget_serialises_without_changing_results():
    base = small_jobs(1, seed=8)[0]
    jobs = [dict(base, seed=base["seed"] + 100 * i, events=base["events"] + 7 * i)
            for i in range(5)]
    srv = psc.Server(budget_bytes=1, quantum_events=8)  # every job alone
    # a budget below any job: each is rejected at once
    jid = srv.submit(jobs[0], keep_state=True)
    assert srv.wait(jid)["state"] == psc.JOB_FAILED
    srv.close()
    sizes = [psc.Server.job_bytes(w) for w in jobs]
    # room for the largest job, never for two: the jobs run one after another
    budget = max(max(sizes), int(1.5 * min(sizes)))
    assert budget < 2 * min(sizes)
    srv = psc.Server(budget_bytes=budget, quantum_events=8)
    ids = [srv.submit(w) for w in jobs]
    for w, jid in zip(jobs, ids):
        st = srv.wait(jid)
        assert st["state"] == psc.JOB_DONE
        a = alone(w)
        assert (st["attempts"], st["hops"], st["collisions"], st["events_done"]) == (
            a["attempts"], a["hops"], a["collisions"], a["event"])
    assert srv.stats()["peak_active"] == 1
    srv.close()


def test_invalid_job_fails_alone():
    jobs = small_jobs(4, seed=11)
    bad = dict(jobs[0], dims=(6, 8, 8))                        # not a multiple of 4
    worse = dict(jobs[1], reactions=[((1, 9), (2,), 1e-18)])   # unknown species
    srv = psc.Server(budget_bytes=4 << 30, quantum_events=16)
    ids = [srv.submit(w, keep_state=True) for w in jobs]
    b1 = srv.submit(bad)
    b2 = srv.submit(worse)
    assert srv.wait(b1)["state"] == psc.JOB_FAILED and srv.wait(b1)["error"] == psc.PSC_EINVAL
    assert srv.wait(b2)["state"] == psc.JOB_FAILED
    for w, jid in zip(jobs, ids):
        assert srv.wait(jid)["state"] == psc.JOB_DONE
        same(srv.read_state(jid, cap_of(w)), alone(w))
    # the failed jobs returned what their admission charged, and so does
    # every kept job once released
    assert srv.stats()["device_bytes_in_use"] > 0
    for jid in ids:
        srv.release(jid)
    assert srv.stats()["device_bytes_in_use"] == 0
    srv.close()


def test_cancel_queued_and_running_jobs():
    base = small_jobs(1, seed=21)[0]
    long_job = dict(base, seed=77, events=2_000_000)      # would run for minutes
    j1 = dict(base, seed=78)
    j2 = dict(base, seed=79, events=base["events"] + 5)
    sizes = [psc.Server.job_bytes(w) for w in (long_job, j1, j2)]
    srv = psc.Server(budget_bytes=max(sizes) + min(sizes) // 2, quantum_events=8)
    lid = srv.submit(long_job)
    time.sleep(0.2)                                        # admitted and running alone
    assert srv.poll(lid)["state"] == psc.JOB_RUNNING
    i1 = srv.submit(j1)
    i2 = srv.submit(j2)
    assert srv.poll(i1)["state"] == psc.JOB_QUEUED
    srv.cancel(i1)                                         # leaves the queue at once
    assert srv.poll(i1)["state"] == psc.JOB_CANCELLED
    srv.cancel(lid)                                        # retired at the next step boundary
    assert srv.wait(lid)["state"] == psc.JOB_CANCELLED
    with pytest.raises(psc.PscError) as e:
        srv.cancel(lid)
    assert e.value.code == psc.PSC_ESTATE
    st = srv.wait(i2)                                      # the next one runs, unchanged
    assert st["state"] == psc.JOB_DONE
    a = alone(j2)
    assert (st["attempts"], st["hops"], st["collisions"], st["events_done"]) == (
        a["attempts"], a["hops"], a["collisions"], a["event"])
    stats = srv.stats()
    assert stats["cancelled"] == 2 and stats["done"] == 1
    assert stats["device_bytes_in_use"] == 0
    srv.close()


def test_server_started_with_default_options():
    w = small_jobs(1, seed=31)[0]
    srv = psc.Server(budget_bytes=1 << 30, defaults=True)
    st = srv.wait(srv.submit(w))
    a = alone(w)
    assert st["state"] == psc.JOB_DONE
    assert (st["attempts"], st["hops"], st["events_done"]) == (a["attempts"], a["hops"], a["event"])
    srv.close()
