"""Random initial states for load_state (numpy RNG, not the method's Philox)."""
from __future__ import annotations

import numpy as np


def random_state(dims, counts, seed: int, id_gaps: bool = True, disp: bool = True,
                 event: int = 0, voxels=None) -> dict:
    """Occupancy plus a molecule table.

    counts: [(species id, number)], placed on distinct voxels drawn without
    replacement (or at the given `voxels`).  Ids are ascending, optionally
    with random gaps, and next_id leaves room above the largest id.
    """
    rng = np.random.default_rng(seed)
    nv = int(dims[0]) * int(dims[1]) * int(dims[2])
    total = sum(c for _, c in counts)
    if voxels is None:
        vox = rng.choice(nv, size=total, replace=False).astype(np.uint32)
    else:
        vox = np.asarray(voxels, np.uint32)
        assert len(vox) == total
    sp = np.concatenate([np.full(c, s, np.uint16) for s, c in counts]) if total else \
        np.zeros(0, np.uint16)
    order = rng.permutation(total)
    vox, sp = vox[order], sp[order]
    if id_gaps:
        ids = np.cumsum(rng.integers(1, 4, size=total)).astype(np.uint64) - 1
    else:
        ids = np.arange(total, dtype=np.uint64)
    ids = ids.astype(np.uint32)
    occ = np.zeros(nv, np.uint16)
    occ[vox] = sp
    if disp:
        d = rng.integers(-50, 51, size=(3, total)).astype(np.int32)
    else:
        d = np.zeros((3, total), np.int32)
    next_id = int(ids[-1]) + 1 + int(rng.integers(0, 5)) if total else 0
    return dict(occ=occ, id=ids, vox=vox, species=sp, dx=d[0], dy=d[1], dz=d[2],
                event=event, next_id=next_id)
