"""Oracle M for regular arrays of identical loops, one oracle call per
distinct loop offset.

The Neumann double integral between two loops is unchanged when both loops
are translated together, so in an array of identical loops (same polygon,
same wire radius) M[k, l] depends only on the offset (ix_l - ix_k, iy_l -
iy_k).  Each distinct offset is evaluated by the oracle on a two-loop
geometry; the diagonal on a one-loop geometry.  This only reuses equal
values, it computes nothing the oracle does not; tests/test_oracle_pins.py
checks it against the direct oracle.  Test infrastructure.
"""
import numpy as np

import oracle as O


def oracle_M_array(g) -> np.ndarray:
    nx, ny = int(g.nx), int(g.ny)
    n = nx * ny
    so = np.asarray(g.seg_off)
    assert len(so) == n + 1
    assert np.all(np.asarray(g.wire_a) == g.wire_a[0])

    def verts(k):
        return g.verts[so[k]:so[k + 1]]

    cache = {}
    M = np.empty((n, n))
    for k in range(n):
        iyk, ixk = divmod(k, nx)
        for l in range(n):
            iyl, ixl = divmod(l, nx)
            key = (ixl - ixk, iyl - iyk)
            v = cache.get(key)
            if v is None:
                if k == l:
                    vk = verts(k)
                    v = O.inductance_matrix_fast(vk, np.array([0, len(vk)], dtype=np.int32),
                                                 np.array([g.wire_a[k]]))[0, 0]
                else:
                    vk, vl = verts(k), verts(l)
                    two = np.concatenate([vk, vl])
                    off = np.array([0, len(vk), len(vk) + len(vl)], dtype=np.int32)
                    v = O.inductance_matrix_fast(two, off, np.array([g.wire_a[k], g.wire_a[l]]))[0, 1]
                cache[key] = v
            M[k, l] = v
    return M
