"""Workload descriptions (seeded, synthetic).

A workload is a plain dict:
  name, dims (ni, nj, nk), rv (voxel radius, m), seed,
  species: [(name, D m^2/s)]   -> species ids 1, 2, ... in this order
  reactions: [(reactant ids, product ids, k)]  k in 1/s or m^3/s
  place: [(species id, count)] uniform placements, in this order
  events: number of diffusion events, track_displacement: bool
  max_molecules (optional): the capacity a run of the workload needs

The five benchmark workloads follow the paper's workload shapes (HCP lattice,
homogeneous start, crowding by immobile voxels, a MAPK-style network); the
paper's own datasets are not used.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
RV = 4.4e-9          # voxel radius used by every benchmark workload
D1 = 1e-12           # 1 um^2/s
D05 = 0.5e-12


def cfg3_network() -> dict:
    with open(os.path.join(HERE, "cfg3_network.json")) as f:
        return json.load(f)


def _motif(kb: float = 0.1, kf: float = 1e-18):
    """A + B -> C (second order) and C -> A + B (first order): species ids
    assume A, B, C are registered as 1, 2, 3 (after any obstacle species the
    caller shifts them)."""
    return [((1, 2), (3,), kf), ((3,), (1, 2), kb)]


def cfg1(events: int = 1000) -> dict:
    n = 64 ** 3
    return dict(name="diffusion_64cubed", dims=(64, 64, 64), rv=RV, seed=1,
                species=[("A", D1)], reactions=[], place=[(1, int(0.01 * n))],
                events=events, track_displacement=True)


def cfg2(events: int = 10000, dims=(256, 256, 256)) -> dict:
    n = dims[0] * dims[1] * dims[2]
    # species: 1 obstacle (immobile), 2 A, 3 B, 4 C
    return dict(name="crowded_reaction_%dx%dx%d" % dims, dims=tuple(dims), rv=RV, seed=2,
                species=[("O", 0.0), ("A", D1), ("B", D05), ("C", D1)],
                reactions=[((2, 3), (4,), 1e-18), ((4,), (2, 3), 0.1)],
                place=[(1, int(0.30 * n)), (2, int(0.02 * n)), (3, int(0.02 * n))],
                events=events, track_displacement=False)


def cfg3(events: int = 2000, dims=(2048, 2048, 1024)) -> dict:
    net = cfg3_network()
    n = dims[0] * dims[1] * dims[2]
    total = int(0.003 * n)
    kinase = total * 4 // 6
    kk = (total - kinase) // 2
    pase = total - kinase - kk
    species = [(name, D) for name, D in zip(net["species"], net["D"])]
    reactions = [(tuple(x + 1 for x in r["reactants"]), tuple(x + 1 for x in r["products"]),
                  r["k"]) for r in net["reactions"]]
    # initial molecules: MAPK (K), MAPKK (KK) and phosphatase (P) in 4 : 1 : 1
    return dict(name="mapk_%dx%dx%d" % dims, dims=tuple(dims), rv=RV, seed=3,
                species=species, reactions=reactions,
                place=[(1, kinase), (4, kk), (5, pase)],
                events=events, track_displacement=False)


def ensemble_members(n: int = 512, events: int = 5000, base_seed: int = 4000,
                     edges=(32, 48, 64, 96, 128), seed: int = 44) -> list:
    """Independent replicates of the A + B <-> C motif with random cubic edge
    and occupancy (1 % .. 10 %, split A : B = 1 : 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        e = int(rng.choice(edges))
        phi = float(rng.uniform(0.01, 0.10))
        nv = e ** 3
        half = int(phi * nv) // 2
        out.append(dict(name="replicate_%d" % r, dims=(e, e, e), rv=RV, seed=base_seed + r,
                        species=[("A", D1), ("B", D05), ("C", D1)],
                        reactions=_motif(kb=1.0), place=[(1, half), (2, half)],
                        events=events, track_displacement=False))
    return out


def serving_jobs(rate: float = 200.0, duration: float = 60.0, seed: int = 55,
                 edge_range=(32, 256), phi_range=(0.005, 0.05),
                 event_range=(500, 20000)) -> list:
    """Poisson arrivals; per job a cubic lattice with edge log-uniform in
    edge_range (multiple of 4), occupancy uniform in phi_range, events
    log-uniform in event_range, motif A + B <-> C without obstacles."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        e = math.exp(rng.uniform(math.log(edge_range[0]), math.log(edge_range[1])))
        e = max(4, int(round(e / 4.0)) * 4)
        phi = float(rng.uniform(*phi_range))
        ev = int(round(math.exp(rng.uniform(math.log(event_range[0]),
                                            math.log(event_range[1])))))
        nv = e ** 3
        half = int(phi * nv) // 2
        jobs.append(dict(name="job_%d" % len(jobs), arrival=t, dims=(e, e, e), rv=RV,
                         seed=5000 + len(jobs),
                         species=[("A", D1), ("B", D05), ("C", D1)],
                         reactions=_motif(kb=0.1), place=[(1, half), (2, half)],
                         events=ev, track_displacement=False))
    return jobs


def small_reactive(dims=(16, 12, 8), seed: int = 7, events: int = 40) -> dict:
    """A compact test network that exercises every rule: obstacles, two
    mobile reactants of different D (so events alternate), 1- and 2-product
    collisions, first-order reactions with 0, 1, 2 and 3 products."""
    n = dims[0] * dims[1] * dims[2]
    return dict(name="small_reactive", dims=tuple(dims), rv=RV, seed=seed,
                species=[("O", 0.0), ("A", D1), ("B", D05), ("C", D1), ("D", 2 * D1)],
                reactions=[((2, 3), (4,), 1e-18),          # A + B -> C
                           ((2, 5), (3, 2), 2e-20),        # A + D -> B + A (swap-like)
                           ((4,), (2, 3), 2000.0),         # C -> A + B
                           ((5,), (), 500.0),              # D -> 0
                           ((3,), (5,), 300.0),            # B -> D
                           ((2,), (2, 5, 5), 400.0)],      # A -> A + D + D
                place=[(1, n // 10), (2, n // 20), (3, n // 20), (5, n // 40)],
                events=events, track_displacement=True)


def multiproduct(dims=(16, 12, 8), seed: int = 3, n_a: int = 0, events: int = 40,
                 boundary=None) -> dict:
    """Collisions with more than two products next to first-order decays, with
    a bounded population: A + B -> B + A + 2 C (p about 0.36),
    C + B -> D + B + E (p about 0.54), C -> 0, D -> 2 C, E -> 0; A and B at
    n_a each (default 1/12 of the voxels)."""
    nv = dims[0] * dims[1] * dims[2]
    n_a = n_a or nv // 12
    w = dict(name="multiproduct", dims=tuple(dims), rv=RV, seed=seed,
             species=[("A", D1), ("B", D05), ("C", 2 * D1), ("D", 0.0), ("E", D1)],
             reactions=[((1, 2), (2, 1, 3, 3), 2e-20),
                        ((3, 2), (4, 2, 5), 5e-20),
                        ((3,), (), 20000.0),
                        ((4,), (3, 3), 800.0),
                        ((5,), (), 800.0)],
             place=[(1, n_a), (2, n_a)], events=events, track_displacement=True)
    if boundary:
        w["boundary"] = boundary
    return w


AVOGADRO = 6.02214076e23


def per_nM_s(k: float) -> float:
    """second-order rate constant in 1/(nM s) -> m^3/s per molecule pair"""
    return k * 1e9 * 1e-3 / AVOGADRO


def mapk_paper(events: int = 450000, dims=(480, 480, 480), seed: int = 6,
               mapkk_nM: float = 50.0) -> dict:
    """The paper's MAPK model (its section 3.4): MAPK doubly phosphorylated by
    MAPKK and dephosphorylated by a phosphatase, 9 species, 12 reactions,
    D = 1 um^2/s, r_v = 10 nm, 480^3 voxels, MAPK 200 nM, MAPKK 50 nM, Pase
    50 nM.  Counts come from those concentrations over the simulated
    lattice's own volume (n_v 4 sqrt2 r^3 = 0.626 pL for 480^3; the paper's
    0.443 pL does not match its lattice).  30 s simulated = 450,000 events."""
    rv = 10e-9
    D = 1e-12
    nv = dims[0] * dims[1] * dims[2]
    volume_l = nv * 4.0 * math.sqrt(2.0) * rv ** 3 * 1e3
    def count(nM):
        return int(nM * 1e-9 * volume_l * AVOGADRO)
    k1, k2, k3 = per_nM_s(0.027), 1.3, 1.5
    k4, k5, k6 = per_nM_s(0.026), 1.73, 15.0
    names = ["MAPK", "pMAPK", "ppMAPK", "MAPKK", "Pase",
             "MAPK/MAPKK", "pMAPK/MAPKK", "ppMAPK/Pase", "pMAPK/Pase"]
    K, Kp, Kpp, KK, P, C1, C2, C3, C4 = range(1, 10)
    reactions = [
        ((K, KK), (C1,), k1), ((C1,), (K, KK), k2),
        ((Kp, KK), (C2,), k4), ((C2,), (Kp, KK), k5),
        ((Kpp, P), (C3,), k1), ((C3,), (Kpp, P), k2),
        ((Kp, P), (C4,), k4), ((C4,), (Kp, P), k5),
        ((C1,), (Kp, KK), k3), ((C2,), (Kpp, KK), k6),
        ((C3,), (Kp, P), k3), ((C4,), (K, P), k6),
    ]
    return dict(name="mapk_paper_%dx%dx%d" % dims, dims=tuple(dims), rv=rv, seed=seed,
                species=[(n, D) for n in names], reactions=reactions,
                place=[(K, count(200.0)), (KK, count(mapkk_nM)), (P, count(50.0))],
                events=events, track_displacement=False)


def births(dims=(128, 128, 128), seed: int = 8, n_a: int = 90000, n_b: int = 150000,
           events: int = 200) -> dict:
    """Birth-heavy: a fast first-order A -> A + C (about a fifth of the A
    fire per event) beside a collision A + B -> A + B + C that always fires
    (11 % occupancy): tens of thousands of newborns per event, C immobile."""
    return dict(name="births_%dx%dx%d" % tuple(dims), dims=tuple(dims), rv=RV, seed=seed,
                species=[("A", D1), ("B", D1), ("C", 0.0)],
                reactions=[((1,), (1, 3), 20000.0), ((1, 2), (1, 2, 3), 1e-15)],
                place=[(1, n_a), (2, n_b)], events=events, track_displacement=False,
                max_molecules=dims[0] * dims[1] * dims[2])


WORKLOADS = {
    "cfg1": cfg1,
    "cfg2": cfg2,
    "cfg3": cfg3,
    "small_reactive": small_reactive,
    "mapk_paper": mapk_paper,
    "multiproduct": multiproduct,
    "births": births,
}


def _membrane(**kw):
    from .compartments import membrane
    return membrane(**kw)


WORKLOADS["membrane"] = _membrane


def workload(name: str, **kw) -> dict:
    return WORKLOADS[name](**kw)
