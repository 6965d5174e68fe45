"""Writes cfg3_network.json: the 10-species MAPK-style dual-phosphorylation
network of the 2^32-voxel workload, with rate constants drawn once,
log-uniformly, from a fixed seed (bimolecular in [1e-19, 1e-17] m^3/s,
first-order in [0.1, 10] 1/s).  Run once; the JSON is committed."""
import json
import os

import numpy as np

SPECIES = ["K", "Kp", "Kpp", "KK", "P", "K.KK", "Kp.KK", "Kpp.P", "Kp.P", "Kpp.KK"]
# second-order reactions: (reactant, reactant) -> products, species indices
BIMOLECULAR = [
    ((0, 3), (5,)), ((1, 3), (6,)), ((2, 4), (7,)), ((1, 4), (8,)), ((2, 3), (9,)),
    ((0, 9), (5, 2)), ((1, 9), (6, 2)), ((1, 7), (8, 2)),
]
FIRST_ORDER = [
    (5, (0, 3)), (5, (1, 3)), (6, (1, 3)), (6, (2, 3)), (7, (2, 4)),
    (7, (1, 4)), (8, (1, 4)), (8, (0, 4)), (9, (2, 3)), (2, (1,)),
]


def main():
    rng = np.random.default_rng(1605_03726)
    k2 = 10.0 ** rng.uniform(-19.0, -17.0, size=len(BIMOLECULAR))
    k1 = 10.0 ** rng.uniform(-1.0, 1.0, size=len(FIRST_ORDER))
    net = {
        "species": SPECIES,
        "D": [1e-12] * len(SPECIES),
        "reactions": (
            [{"reactants": list(r), "products": list(p), "k": float(k)}
             for (r, p), k in zip(BIMOLECULAR, k2)]
            + [{"reactants": [r], "products": list(p), "k": float(k)}
               for (r, p), k in zip(FIRST_ORDER, k1)]),
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg3_network.json")
    with open(out, "w") as f:
        json.dump(net, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
