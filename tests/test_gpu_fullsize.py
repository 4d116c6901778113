"""Full-size parity: the HIP path at the workloads' own shapes, in the launch
configuration the benchmark times, against stored FP64 oracle values
(tests/golden/*_full.json, written by tests/golden/make_fullsize_golden.py
from ``oracle`` and ``workloads`` only).

Per configuration: the loss (Eq. 1 on magnitudes) to a relative tolerance and
dL/dC (adjoint of Eq. 8-10) normwise, FP64 1e-9, FP32 1e-5, BF16X3 3e-3.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-9, 1: 1e-5, 2: 3e-3}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2503_18479_amd as pkg
    pkg.load_library()
    return torch.device("cuda:0")


def _plan(wl, dev, precisions=None):
    from paper_2503_18479_amd import Geometry, Plan
    plan = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), wl.bext_z,
                precisions=precisions)
    return (plan, torch.tensor(wl.C, device=dev), torch.tensor(wl.omega, device=dev),
            torch.tensor(wl.target, device=dev))


def _compare(tag, loss, grad, cfg, ref_loss, ref_grad, tol):
    l = loss.cpu().numpy()[cfg]
    g = grad.cpu().numpy()[cfg]
    rl = np.asarray(ref_loss)
    rg = np.asarray(ref_grad)
    el = np.abs(l - rl) / np.abs(rl)
    eg = np.linalg.norm(g - rg, axis=1) / np.linalg.norm(rg, axis=1)
    _say(f"[{tag}] loss err {el.max():.2e} grad err {eg.max():.2e} over {len(cfg)} configurations")
    assert el.max() < tol, (tag, int(np.argmax(el)))
    assert eg.max() < tol, (tag, int(np.argmax(eg)))


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_single_loop_full(dev, prec):
    """Single 64-gon loop, 32x32 points, the 64-value capacitance sweep."""
    gd = _golden("single_loop_full.json")
    wl = W.config1_single_loop(batch=64, grid=32)
    plan, C, om, T = _plan(wl, dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    _compare(f"c1 prec={prec}", loss, grad, gd["configs"], gd["loss"], gd["grad"], TOL[prec])


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_line8_full(dev, prec):
    """8x1 line, 64x64 points, batch 1,024: every configuration; the FP64
    gradient of the first 16 also against the oracle's central differences
    (h = 1e-3 pF, whose own truncation error is about 1e-7)."""
    gd = _golden("line_8x1_full.json")
    wl = W.config2_line8(batch=1024, grid=64)
    plan, C, om, T = _plan(wl, dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    _compare(f"c2 prec={prec}", loss, grad, gd["configs"], gd["loss"], gd["grad"], TOL[prec])
    if prec == 0:
        fc = gd["fd_configs"]
        g = grad.cpu().numpy()[fc]
        fd = np.asarray(gd["fd"])
        e = np.linalg.norm(g - fd, axis=1) / np.linalg.norm(fd, axis=1)
        _say(f"[c2] FP64 gradient vs oracle central differences: {e.max():.2e}")
        assert e.max() < 1e-6


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_array8x8_full(dev, prec):
    """8x8 array, 65,536 points, 21 frequencies, batch 4,096 (86,016 systems):
    16 configurations, among them the first and last and ones whose systems
    straddle the fused kernels' wave and workgroup blocks."""
    gd = _golden("array_8x8_full.json")
    wl = W.config3_array8x8(batch=4096)
    plan, C, om, T = _plan(wl, dev)
    _say(f"[c3] prec={prec}")
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    _compare(f"c3 prec={prec}", loss, grad, gd["configs"], gd["loss"], gd["grad"], TOL[prec])


@pytest.mark.parametrize("prec", [0, 2])
def test_array8x8_two_planes_full(dev, prec):
    """The same array at both observation planes (131,072 points)."""
    gd = _golden("array_8x8_full.json")["two_planes"]
    wl = W.config3_array8x8(batch=4096, two_planes=True)
    plan, C, om, T = _plan(wl, dev, precisions=["fp64", "bf16x3"])
    _say(f"[c3 two planes] prec={prec}")
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    _compare(f"c3x2 prec={prec}", loss, grad, gd["configs"], gd["loss"], gd["grad"], TOL[prec])


@pytest.fixture(scope="module")
def c5(dev):
    wl = W.config5_array32x32(batch=256)
    _say("[c5] assembling 32x32 / 262,144 points")
    plan, C, om, T = _plan(wl, dev)
    plan.reserve(wl.B, wl.F)
    return wl, plan, C, om, T


@pytest.mark.parametrize("prec,refined", [(0, False), (1, False), (2, False), (0, True), (2, True)])
def test_array32x32_full(dev, c5, prec, refined):
    """32x32 array (1,024 loops), 262,144 points, batch 256: four
    configurations in every precision, with the FP64 factor and with the FP32
    factor refined in FP64."""
    gd = _golden("array_32x32_full.json")
    wl, plan, C, om, T = c5
    plan.set_refinement(refined)
    _say(f"[c5] prec={prec} refined={refined}")
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    torch.cuda.synchronize()
    plan.set_refinement(False)
    assert int(st.abs().sum()) == 0
    _compare(f"c5 prec={prec} refined={refined}", loss, grad, gd["configs"], gd["loss"],
             gd["grad"], TOL[prec])


def test_array32x32_adam_steps(dev):
    """The first Adam steps on C (Sec. IV) for the 32x32 array at a reduced
    grid, FP64, against the oracle's own trajectory: the loss before every
    step (1e-9) and C after it.  Adam divides by sqrt(v) + eps, so an
    absolute gradient difference d moves C_k by up to lr d / (4 eps) where
    |g_k| is near eps (gradient components here span 0.5 eps to 4e8 eps):
    C is held to 1e-6 of the largest displacement, which a wrong step (of
    order lr) misses by far."""
    from paper_2503_18479_amd import adam_step
    gd = _golden("array_32x32_full.json")["adam"]
    a = gd["params"]
    wl = W.config5_array32x32(batch=a["batch"], grid=a["grid"])
    plan, C, om, T = _plan(wl, dev, precisions=["fp64"])
    C0 = wl.C.copy()
    m = torch.zeros_like(C)
    v = torch.zeros_like(C)
    t = torch.zeros((1,), dtype=torch.int32, device=dev)
    for k in range(a["steps"]):
        loss, grad, st = plan.loss_and_grad(C, om, T, precision=0)
        adam_step(C, grad, m, v, t, lr=a["lr"], betas=(a["beta1"], a["beta2"]), eps=a["eps"])
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        el = np.abs(loss.cpu().numpy() - gd["loss_before_step"][k]) / np.abs(gd["loss_before_step"][k])
        Cr = np.asarray(gd["C_after_step"][k])
        dC = np.abs(C.cpu().numpy() - Cr).max() / np.abs(Cr - C0).max()
        _say(f"[c5 adam] step {k + 1}: loss err {el.max():.2e}, C err / displacement {dC:.2e}")
        assert el.max() < 1e-9
        assert dC < 1e-6


@pytest.mark.parametrize("prec", [0, 2])
def test_ragged_instances_full(dev, prec):
    """Instances of the ragged configuration with 16, 64, 144 and 256 loops at
    their own grids (27k-59k points, 1-8 frequencies) in one
    cosim_loss_and_grad_many call together with the other instances of the
    same generator prefix up to the largest index used."""
    from paper_2503_18479_amd import loss_and_grad_many
    gd = _golden("ragged_full.json")
    idx = [i["index"] for i in gd["instances"]]
    wls = W.config4_instances(max(idx) + 1)
    plans, Cs, Os, Ts = [], [], [], []
    for wl in wls:
        plan, C, om, T = _plan(wl, dev, precisions=["fp64", "bf16x3"])
        plan.reserve(wl.B, wl.F)
        plans.append(plan); Cs.append(C); Os.append(om); Ts.append(T)
    _say(f"[ragged] prec={prec} {len(wls)} instances, checked {idx}")
    outs = loss_and_grad_many(plans, Cs, Os, Ts, precision=prec)
    torch.cuda.synchronize()
    for rec in gd["instances"]:
        loss, grad, st = outs[rec["index"]]
        assert wls[rec["index"]].geom.n == rec["loops"] and wls[rec["index"]].P == rec["points"]
        assert int(st.abs().sum()) == 0
        _compare(f"ragged {rec['index']} n={rec['loops']} prec={prec}", loss, grad, [0],
                 [rec["loss"]], [rec["grad"]], TOL[prec])
