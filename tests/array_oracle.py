"""Oracle M for regular arrays of identical loops (a workloads Geometry with
its lattice shape), through ``oracle.inductance_matrix_lattice``, which
evaluates each distinct loop offset once.  tests/test_oracle_pins.py checks it
against the direct oracle.  Test infrastructure."""
import numpy as np

import oracle as O


def oracle_M_array(g) -> np.ndarray:
    return O.inductance_matrix_lattice(g.verts, g.seg_off, g.wire_a, int(g.nx), int(g.ny))
