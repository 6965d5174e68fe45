"""Workload descriptions (seeded, synthetic).

A workload is a plain dict:
  name, dims (ni, nj, nk), rv (voxel radius, m), seed,
  species: [(name, D m^2/s)]   -> species ids 1, 2, ... in this order
  reactions: [(reactant ids, product ids, k)]  k in 1/s or m^3/s
  place: [(species id, count)] uniform placements, in this order
  events: number of diffusion events, track_displacement: bool

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


WORKLOADS = {
    "cfg1": cfg1,
    "cfg2": cfg2,
    "cfg3": cfg3,
    "small_reactive": small_reactive,
}


def workload(name: str, **kw) -> dict:
    return WORKLOADS[name](**kw)
