"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This package holds workload descriptions (lattice sizes, species, reaction
networks, molecule counts, seeds) and random initial states.  It contains none
of the method's arithmetic: no stencil, no random-number scheme of the method,
no reaction probabilities.  Both the GPU path and the CPU oracle consume what
it produces.
"""
from .workloads import (WORKLOADS, workload, ensemble_members, serving_jobs,  # noqa: F401
                        cfg3_network)
from .states import random_state  # noqa: F401
from .compartments import shell_map, sub_box_map, layered_map, membrane  # noqa: F401
