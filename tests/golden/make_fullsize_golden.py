"""Writes the full-size expected values under tests/golden/ from the FP64 oracle.

Run from the repository root (about 10 minutes on 8 cores):
    python tests/golden/make_fullsize_golden.py [part ...]
with parts among: single_loop line8 array8x8 array32x32 ragged (default: all).

Only ``oracle`` and ``workloads`` are used; nothing here touches the HIP
library.  The field matrix G is evaluated by ``oracle.field_matrix`` on
blocks of points in worker processes (each block is the oracle's own call on
a subset of the points; the blocks are stacked in order).  Every value is
the magnitude-MSE loss of Eq. 1 and its gradient dL/dC by the adjoint of
Eq. 8-10 (the oracle's ``evaluate`` and ``grad_adjoint``), at the shapes and
seeded inputs of ``workloads``; the 8x1 line adds central differences of the
loss with h = 1e-3 pF, and the 32x32 array the first Adam steps on C.
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

_G_ARGS = None


def _g_block(rows):
    verts, seg_off, pts = _G_ARGS
    return O.field_matrix(verts, seg_off, pts[rows[0]:rows[1]])


def field_matrix_parallel(g, pts, workers=8, block=8192):
    """oracle.field_matrix over blocks of points, in order."""
    global _G_ARGS
    _G_ARGS = (g.verts, g.seg_off, pts)
    blocks = [(i, min(i + block, len(pts))) for i in range(0, len(pts), block)]
    if len(blocks) == 1:
        return _g_block(blocks[0])
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_g_block, blocks)
    return np.concatenate(parts, axis=0)


def operators(wl, lattice=True, general=False):
    g = wl.geom
    t0 = time.time()
    G = field_matrix_parallel(g, wl.pts)
    if general:
        M = O.inductance_matrix(g.verts, g.seg_off, g.wire_a)
    elif lattice:
        M = O.inductance_matrix_lattice(g.verts, g.seg_off, g.wire_a, g.nx, g.ny)
    else:
        M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    print(f"  {wl.name}: G {G.shape} and M in {time.time() - t0:.1f} s", flush=True)
    return G, M, Phi


def loss_grad(wl, G, M, Phi, configs):
    g = wl.geom
    C = wl.C[configs]
    L = O.evaluate(G, M, g.R, Phi, C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, g.R, Phi, C, wl.omega, wl.target)
    return [float(x) for x in L], [[float(x) for x in row] for row in gr]


def dump(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, indent=None, separators=(",", ":"))
        f.write("\n")
    print(f"  wrote {path} ({os.path.getsize(path)} bytes)", flush=True)


SOURCE = ("FP64 oracle (oracle.evaluate / oracle.grad_adjoint: loss of Eq. 1 on magnitudes, "
          "dL/dC by the adjoint of Eq. 8-10); regenerate with tests/golden/make_fullsize_golden.py")


def part_single_loop():
    wl = W.config1_single_loop(batch=64, grid=32)
    G, M, Phi = operators(wl, lattice=False, general=True)
    cfg = list(range(wl.B))
    L, gr = loss_grad(wl, G, M, Phi, cfg)
    dump("single_loop_full.json", dict(
        _source=SOURCE, workload="config1_single_loop(batch=64, grid=32)", configs=cfg,
        loss=L, grad=gr))


def part_line8():
    wl = W.config2_line8(batch=1024, grid=64)
    G, M, Phi = operators(wl, lattice=True)
    cfg = list(range(wl.B))
    L, gr = loss_grad(wl, G, M, Phi, cfg)
    fd_cfg = list(range(16))
    fd = O.grad_fd(G, M, wl.geom.R, Phi, wl.C[fd_cfg], wl.omega, wl.target, h=1e-15)
    dump("line_8x1_full.json", dict(
        _source=SOURCE + "; fd: central differences of the oracle loss, h = 1e-15 F",
        workload="config2_line8(batch=1024, grid=64)", configs=cfg, loss=L, grad=gr,
        fd_configs=fd_cfg, fd_h=1e-15, fd=[[float(x) for x in row] for row in fd]))


# configurations of the 8x8 batch (4,096 configurations, 21 frequencies,
# system s = 21 b + f): the first and last, and ones whose systems straddle
# the 32-system wave and 128-system workgroup blocks of the fused kernels
# (b = 6: s 126..146; b = 12: 252..272; b = 97: 2037..2057 around 2048; b = 195:
# 4095..4115 around 4096) and a few more spread over the batch
ARRAY8X8_CONFIGS = [0, 1, 6, 12, 97, 195, 512, 1023, 1024, 2047, 2048, 3000, 3071, 4000, 4094, 4095]


def part_array8x8():
    wl = W.config3_array8x8(batch=4096)
    G, M, Phi = operators(wl)
    L, gr = loss_grad(wl, G, M, Phi, ARRAY8X8_CONFIGS)
    out = dict(_source=SOURCE, workload="config3_array8x8(batch=4096)",
               configs=ARRAY8X8_CONFIGS, loss=L, grad=gr)
    # both observation planes (131,072 points)
    wl2 = W.config3_array8x8(batch=4096, two_planes=True)
    G2 = field_matrix_parallel(wl2.geom, wl2.pts)
    cfg2 = [0, 6, 2048, 4095]
    L2, gr2 = loss_grad(wl2, G2, M, Phi, cfg2)
    out["two_planes"] = dict(workload="config3_array8x8(batch=4096, two_planes=True)",
                             configs=cfg2, loss=L2, grad=gr2)
    dump("array_8x8_full.json", out)


ARRAY32_CONFIGS = [0, 5, 128, 255]
ADAM = dict(batch=2, grid=64, steps=3, lr=1e-13, beta1=0.9, beta2=0.999, eps=1e-8)


def part_array32x32():
    wl = W.config5_array32x32(batch=256)
    G, M, Phi = operators(wl)
    L, gr = loss_grad(wl, G, M, Phi, ARRAY32_CONFIGS)
    del G
    out = dict(_source=SOURCE, workload="config5_array32x32(batch=256)",
               configs=ARRAY32_CONFIGS, loss=L, grad=gr)
    # Adam on C (Sec. IV) for a few steps, at a reduced grid of the same array
    a = ADAM
    wr = W.config5_array32x32(batch=a["batch"], grid=a["grid"])
    Gr = field_matrix_parallel(wr.geom, wr.pts)
    C = wr.C.copy()
    m = np.zeros_like(C)
    v = np.zeros_like(C)
    Cs, Ls = [], []
    for t in range(1, a["steps"] + 1):
        Lt = O.evaluate(Gr, M, wr.geom.R, Phi, C, wr.omega, wr.target)[2]
        gt = O.grad_adjoint(Gr, M, wr.geom.R, Phi, C, wr.omega, wr.target)
        C, m, v = O.adam_step(C, gt, m, v, t, a["lr"], a["beta1"], a["beta2"], a["eps"])
        Ls.append([float(x) for x in Lt])
        Cs.append([[float(x) for x in row] for row in C])
    out["adam"] = dict(workload=f"config5_array32x32(batch={a['batch']}, grid={a['grid']})",
                       params=a, loss_before_step=Ls, C_after_step=Cs)
    dump("array_32x32_full.json", out)


def ragged_pick(count=64):
    """First instances of the ragged configuration with 16, 64, 144 and 256
    loops (full grids of 128..256 points a side); the generator's instance i
    does not depend on how many follow it."""
    wls = W.config4_instances(count)
    want = [16, 64, 144, 256]
    idx = []
    for n in want:
        for i, wl in enumerate(wls):
            if wl.geom.n == n and i not in idx:
                idx.append(i)
                break
    return idx, wls


def part_ragged():
    idx, wls = ragged_pick()
    inst = []
    for i in idx:
        wl = wls[i]
        G, M, Phi = operators(wl)
        L, gr = loss_grad(wl, G, M, Phi, [0])
        inst.append(dict(index=i, loops=wl.geom.n, points=wl.P, freqs=wl.F, loss=L[0],
                         grad=gr[0]))
    dump("ragged_full.json", dict(_source=SOURCE, workload="config4_instances(count=64)",
                                  instances=inst))


PARTS = dict(single_loop=part_single_loop, line8=part_line8, array8x8=part_array8x8,
             array32x32=part_array32x32, ragged=part_ragged)


def main(argv):
    names = argv or list(PARTS)
    for n in names:
        t0 = time.time()
        print(f"[{n}]", flush=True)
        PARTS[n]()
        print(f"[{n}] done in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
