"""Graph replay of a single lattice's events (psc_set_graph_replay) on the
GPU: every replayed step equals the same steps launched one by one and the
CPU oracle, with the host's own synchronisations and read-backs between the
replays; events that need the separate first-order decision launch are
launched directly in between; a change of launch shape rebuilds the graph."""
import numpy as np
import pytest

import oracle
from paper_1605_03726_amd import psc
from psc_inputs import membrane, workload

pytestmark = pytest.mark.gpu


def build_oracle(w):
    o = oracle.Oracle(w["dims"], w["rv"], w["seed"],
                      boundary=oracle.REFLECT if w.get("boundary") == "walls" else oracle.PERIODIC,
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
    return o


def same(a, b, disp=True):
    for key in ("occ", "id", "vox", "species") + (("dx", "dy", "dz") if disp else ()):
        assert np.array_equal(a[key], b[key]), key
    for key in ("attempts", "hops", "collisions", "place_fail", "event", "next_id", "time"):
        assert a[key] == b[key], key
    assert np.array_equal(a["fired"], b["fired"])


@pytest.mark.parametrize("w", [
    workload("small_reactive", dims=(24, 16, 16), seed=5),
    workload("multiproduct", dims=(32, 32, 24), seed=6, n_a=3000),
    membrane(dims=(24, 24, 24), seed=8, lattice="fcc", boundary="walls"),
], ids=["small_reactive", "multiproduct", "membrane_fcc_walls"])
def test_replayed_events_equal_direct_launches_and_the_oracle(w):
    g = psc.lattice_from_workload(w)
    g.set_graph_replay(True)
    d = psc.lattice_from_workload(w)
    o = build_oracle(w)
    disp = w.get("track_displacement", False)
    for n in (1, 7, 20, 3):
        g.step(n)
        d.step(n)
        o.run(n, oracle.MODE_C)
        a = g.read_state()          # a synchronisation and eager work between replays
        same(a, d.read_state(), disp)
        same(a, o.state(), disp)
    g.set_launch(items_per_thread=1, stage_blocks=5)   # a new shape: the graph is rebuilt
    g.step(9)
    d.step(9)
    o.run(9, oracle.MODE_C)
    same(g.read_state(), o.state(), disp)
    same(d.read_state(), o.state(), disp)
    g.close()
    d.close()


def test_events_with_a_decision_launch_between_replays():
    # ~10 k first-order candidates per event: every event takes the separate
    # decision launch, launched directly among the replays
    w = workload("multiproduct", dims=(96, 96, 64), seed=9, n_a=40000)
    g = psc.lattice_from_workload(w)
    g.set_graph_replay(True)
    o = build_oracle(w)
    for n in (2, 10):
        g.step(n)
        o.run(n, oracle.MODE_C)
        same(g.read_state(), o.state())
    g.close()
