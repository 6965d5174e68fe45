"""Ensembles on the GPU: every member advanced in the batched launches equals
the same lattice stepped alone and the CPU oracle, bit for bit; the launch
shape chosen by the autotuner and the way steps are split change nothing."""
import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import ensemble_members, workload

pytestmark = pytest.mark.gpu


def oracle_run(w, events):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
                      lattice=oracle.FCC if w.get("lattice") == "fcc" else oracle.HCP)
    for _, D in w["species"]:
        o.add_species(D)
    for r, p, k in w["reactions"]:
        o.add_reaction(r, p, k)
    for s, c in w["place"]:
        o.place_uniform(s, c)
    o.run(events, oracle.MODE_C)
    return o.state()


def same(g, o, disp):
    keys = ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ())
    for key in keys:
        assert np.array_equal(g[key], o[key]), key
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id"):
        assert g[key] == o[key], (key, g[key], o[key])
    assert g["time"] == o["time"]
    assert np.array_equal(g["fired"], o["fired"])


def mixed_members(n_rep=10, events=40):
    ws = ensemble_members(n=n_rep, events=events, edges=(16, 20, 24, 32), seed=9)
    ws.append(workload("small_reactive", seed=5, events=events))
    ws.append(workload("cfg2", dims=(32, 32, 32), events=events))
    ws.append(dict(workload("cfg1"), dims=(24, 16, 8), events=events, place=[(1, 60)]))
    # members closed by walls beside periodic ones
    ws.append(dict(workload("small_reactive", seed=6, events=events), boundary="walls"))
    ws.append(dict(ws[0], boundary="walls"))
    # collisions with more than two products
    ws.append(workload("multiproduct", seed=8, events=events))
    # FCC members beside HCP ones
    ws.append(dict(workload("small_reactive", seed=13, dims=(16, 16, 12), events=events),
                   lattice="fcc"))
    ws.append(dict(workload("cfg2", dims=(24, 24, 24), events=events), lattice="fcc",
                   boundary="walls"))
    return ws


def test_members_equal_alone_and_oracle():
    events = 40
    ws = mixed_members(events=events)
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    ens.step(events)
    ens.sync()
    for w, lat in zip(ws, lats):
        g = lat.read_state()
        alone = psc.lattice_from_workload(w)
        alone.step(events)
        a = alone.read_state()
        same(g, a, disp=w.get("track_displacement", False))
        same(g, oracle_run(w, events), disp=w.get("track_displacement", False))


def test_autotuned_and_split_steps_are_result_invariant():
    events = 60
    ws = mixed_members(n_rep=6, events=events)
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    ens.autotune(2)
    ens.step(45)
    tuned = ens.tuned()
    assert tuned["items_per_thread"] in (2, 4, 8) and tuned["ms_per_event"] > 0
    for _ in range(3):
        ens.step(5)
    ens.sync()
    for w, lat in zip(ws, lats):
        same(lat.read_state(), oracle_run(w, events), disp=w.get("track_displacement", False))


def test_member_rules():
    ws = mixed_members(n_rep=2, events=10)
    lats = [psc.lattice_from_workload(w) for w in ws]
    with pytest.raises(psc.PscError) as e:
        psc.Ensemble([lats[0], lats[0]])
    assert e.value.code == psc.PSC_EINVAL
    ens = psc.Ensemble(lats)
    with pytest.raises(psc.PscError) as e:
        lats[0].step(1)          # grouped lattices are stepped by their ensemble
    assert e.value.code == psc.PSC_ESTATE
    ens.step(6)
    ens.close()
    lats[0].step(4)              # released: steps alone again, continuing exactly
    same(lats[0].read_state(), oracle_run(ws[0], 10), disp=False)


def test_benchmark_ensemble_at_full_size_sampled():
    """The benchmark's ensemble at its full size (512 replicates, edges 32 to
    128, 1-10 % occupancy) launched as the benchmark launches it (batched,
    autotuned), for 50 events; the first member of every edge and the last
    member are compared with the oracle one by one."""
    ws = ensemble_members(n=512, events=50)
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    ens.autotune(3)
    ens.step(50)
    ens.sync()
    picks = {next(i for i, w in enumerate(ws) if w["dims"][0] == e) for e in (32, 48, 64, 96, 128)}
    for i in sorted(picks | {len(ws) - 1}):
        same(lats[i].read_state(), oracle_run(ws[i], 50), disp=False)


def test_ensemble_read_equals_the_members_read_back():
    ws = [workload("small_reactive", dims=(16, 12, 8), seed=70 + a, events=20) for a in range(3)]
    lats = [psc.lattice_from_workload(w) for w in ws]
    ens = psc.Ensemble(lats)
    ens.step(20)
    for i, lat in enumerate(lats):
        a, b = ens.read(i), lat.read_state()
        for key in ("occ", "id", "vox", "species", "dx", "dy", "dz", "fired"):
            assert np.array_equal(a[key], b[key]), key
        assert (a["event"], a["attempts"], a["next_id"]) == (b["event"], b["attempts"], b["next_id"])
    with pytest.raises(psc.PscError) as e:
        ens.read(3)
    assert e.value.code == psc.PSC_EINVAL
    ens.close()
