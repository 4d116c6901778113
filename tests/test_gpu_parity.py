"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (normwise relative): FP64 1e-9, FP32 1e-5, BF16X3 3e-3 for B_z,
the loss and dL/dC.  The solve, G, M and Phi are FP64 in every mode and are
held to 1e-10 or tighter.
"""
import functools
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {0: 1e-9, 1: 1e-5, 2: 3e-3}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2503_18479_amd as pkg
    pkg.load_library()
    return torch.device("cuda:0")


def _nrel(a, b, axis=None):
    a = np.asarray(a); b = np.asarray(b)
    if axis is None:
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
    return np.linalg.norm(a - b, axis=axis) / np.linalg.norm(b, axis=axis)


class Case:
    """A workload with its oracle operators and a GPU plan."""

    def __init__(self, wl, dev, need_M_general=False, array_M=False):
        from paper_2503_18479_amd import Geometry, Plan
        self.wl = wl
        g = wl.geom
        self.G = O.field_matrix(g.verts, g.seg_off, wl.pts)
        if array_M:
            from array_oracle import oracle_M_array
            self.M = oracle_M_array(g)
        else:
            self.M = (O.inductance_matrix(g.verts, g.seg_off, g.wire_a) if need_M_general
                      else O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a))
        self.Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
        self.geom = Geometry.from_workload(g)
        self.pts = torch.tensor(wl.pts, device=dev)
        self.plan = Plan(self.geom, self.pts, wl.bext_z)
        self.C = torch.tensor(wl.C, device=dev)
        self.om = torch.tensor(wl.omega, device=dev)
        self.T = torch.tensor(wl.target, device=dev)

    def oracle_eval(self, C=None, mode=O.LOSS_MAG):
        C = self.wl.C if C is None else C
        return O.evaluate(self.G, self.M, self.wl.geom.R, self.Phi, C, self.wl.omega,
                          self.wl.target, mode)

    def oracle_grad(self, C=None, mode=O.LOSS_MAG):
        C = self.wl.C if C is None else C
        return O.grad_adjoint(self.G, self.M, self.wl.geom.R, self.Phi, C, self.wl.omega,
                              self.wl.target, mode)


@functools.lru_cache(maxsize=None)
def _case(name):
    dev = torch.device("cuda:0")
    if name == "n6":      # NP=32 (6 loops padded), 400 points: 7 tiles with a ragged last tile
        return Case(W.small_array(3, 2, batch=5, grid=20, n_freq=3, seed=1), dev)
    if name == "n25":     # NP=32
        return Case(W.small_array(5, 5, batch=4, grid=17, n_freq=2, seed=2), dev)
    if name == "n64":     # NP=64, 900 points (14 tiles + 4 rows)
        return Case(W.small_array(8, 8, batch=3, grid=30, n_freq=4, seed=3), dev)
    if name == "n6wide":  # many systems: several fused workgroups along S
        return Case(W.small_array(3, 2, batch=90, grid=9, n_freq=3, seed=4), dev)
    if name == "circle":  # config-1 geometry: non-parallel segment pairs
        wl = W.config1_single_loop(batch=16, grid=12)
        return Case(wl, dev, need_M_general=True)
    # more than 64 loops: pivoted LU and GEMM contractions
    if name == "n81":     # NP=128, 4,489 points: three adjoint P-chunks, ragged last
        return Case(W.small_array(9, 9, batch=3, grid=67, n_freq=2, seed=5), dev, array_M=True)
    if name == "n144":    # NP=192 (n not a multiple of 64)
        return Case(W.small_array(12, 12, batch=2, grid=12, n_freq=2, seed=6), dev, array_M=True)
    if name == "n256":    # NP=256, the largest size of the ragged configuration
        return Case(W.small_array(16, 16, batch=2, grid=16, n_freq=1, seed=7), dev, array_M=True)
    if name == "n81wide":  # NP=128 with 36 systems: several system blocks of the contraction
        return Case(W.small_array(9, 9, batch=12, grid=12, n_freq=3, seed=8), dev, array_M=True)
    raise KeyError(name)


CASES = ["n6", "n25", "n64", "n6wide", "circle"]


# ----------------------------------------------------------------- assembly

@pytest.mark.parametrize("name", CASES)
def test_assembly_G_M_phi(dev, name):
    _say(f"[assembly] case={name}")
    c = _case(name)
    G = c.plan.G().cpu().numpy()
    assert G.shape == c.G.shape
    assert _nrel(G, c.G) < 1e-12
    np.testing.assert_allclose(G, c.G, rtol=1e-10, atol=1e-14 * np.abs(c.G).max())
    M = c.plan.M()
    assert _nrel(M, c.M) < 1e-12
    np.testing.assert_allclose(np.diag(M), np.diag(c.M), rtol=1e-12)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=0)
    np.testing.assert_allclose(c.plan.phi(), c.Phi, rtol=1e-14, atol=0)


def test_assembly_polygon_on_axis(dev):
    """G on the axis of a regular polygon equals the closed form."""
    from paper_2503_18479_amd import Geometry, Plan
    g = W._pack([W.regular_polygon(0.05, 64)], 1e-3, 0.5, 1, 1, 0.0)
    z = np.array([0.0, 0.01, 0.02, -0.03, 0.1])
    pts = np.zeros((5, 3)); pts[:, 2] = z
    plan = Plan(Geometry.from_workload(g), torch.tensor(pts, device=dev))
    G = plan.G().cpu().numpy()[:, 0]
    ref = np.array([O.polygon_axis_bz(64, 0.05, zz) for zz in z])
    np.testing.assert_allclose(G, ref, rtol=1e-13)


# ----------------------------------------------------------------- solve

@pytest.mark.parametrize("name", CASES)
def test_solve_currents(dev, name):
    _say(f"[solve] case={name}")
    c = _case(name)
    I, st = c.plan.solve(c.C, c.om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir = O.currents(c.M, c.wl.geom.R, c.Phi, c.wl.C, c.wl.omega)
    err = _nrel(I.cpu().numpy(), Ir, axis=2)
    assert err.max() < 1e-11, err.max()


def test_solve_sparameter_route(dev):
    """GPU currents equal the paper's Eq. 3-7 wave formulation."""
    c = _case("n25")
    I, _ = c.plan.solve(c.C, c.om)
    Is = O.sform_currents(c.M, c.wl.geom.R, c.Phi, c.wl.C, c.wl.omega)
    assert _nrel(I.cpu().numpy(), Is) < 1e-11


def test_solve_resonance_single_loop(dev):
    """At C_r = 1/(w^2 L) the current is -j w Phi / R."""
    c = _case("circle")
    L = c.plan.M()[0, 0]
    w = 2 * np.pi * 128e6
    Cr = 1.0 / (w * w * L)
    C = torch.tensor([[Cr]], dtype=torch.float64, device=dev)
    I, st = c.plan.solve(C, torch.tensor([w], dtype=torch.float64, device=dev))
    ref = -1j * w * c.plan.phi()[0] / c.wl.geom.R[0]
    np.testing.assert_allclose(I.cpu().numpy()[0, 0, 0], ref, rtol=1e-10)


def test_solve_status_flags(dev):
    from paper_2503_18479_amd import SYS_BAD_INPUT, SYS_NEGATIVE_C
    c = _case("n6")
    C = c.C.clone()
    C[0, 2] = 0.0
    C[1, 0] = float("nan")
    C[2, 1] = -C[2, 1]
    I, st = c.plan.solve(C, c.om)
    st = st.cpu().numpy()
    Ih = I.cpu().numpy()
    assert np.all(st[0] & SYS_BAD_INPUT) and np.all(np.isnan(Ih[0]))
    assert np.all(st[1] & SYS_BAD_INPUT) and np.all(np.isnan(Ih[1]))
    assert np.all(st[2] == SYS_NEGATIVE_C) and np.all(np.isfinite(Ih[2]))
    assert np.all(st[3:] == 0)
    # the negative capacitance is solved, not rejected
    Ir = O.currents(c.M, c.wl.geom.R, c.Phi, C[2:3].cpu().numpy(), c.wl.omega)
    assert _nrel(Ih[2:3], Ir) < 1e-11


def test_empty_batch_is_noop(dev):
    c = _case("n6")
    C = torch.empty((0, c.plan.n), dtype=torch.float64, device=dev)
    I, st = c.plan.solve(C, c.om)
    assert I.shape == (0, c.om.shape[0], c.plan.n)
    loss, g, st = c.plan.loss_and_grad(C, c.om, c.T)
    assert loss.shape == (0,)


# ----------------------------------------------------------------- field

@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", ["n6", "n64", "circle"])
def test_field(dev, name, prec):
    _say(f"[field] case={name} prec={prec}")
    c = _case(name)
    I, _ = c.plan.solve(c.C, c.om)
    Bz = c.plan.field(I, prec).cpu().numpy()
    Br = O.field(c.G, I.cpu().numpy())
    err = _nrel(Bz, Br, axis=2)
    assert err.max() < TOL[prec], err.max()


# ----------------------------------------------------------------- fused loss and gradient

@pytest.mark.parametrize("mode", [O.LOSS_MAG, O.LOSS_COMPLEX])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", CASES)
def test_loss_and_grad(dev, name, prec, mode):
    _say(f"[loss_and_grad] case={name} prec={prec} mode={mode}")
    c = _case(name)
    loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, mode, prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = c.oracle_eval(mode=mode)[2]
    gr = c.oracle_grad(mode=mode)
    el = np.abs(loss.cpu().numpy() - Lr) / np.abs(Lr)
    eg = _nrel(grad.cpu().numpy(), gr, axis=1)
    assert el.max() < TOL[prec], ("loss", el.max())
    assert eg.max() < TOL[prec], ("grad", eg.max())


def test_loss_only_matches_loss_with_grad(dev):
    c = _case("n64")
    l1, _, _ = c.plan.loss_and_grad(c.C, c.om, c.T, precision=1, grad=False)
    l2, _, _ = c.plan.loss_and_grad(c.C, c.om, c.T, precision=1, grad=True)
    assert torch.equal(l1, l2)


def test_gradient_vs_central_differences(dev):
    """dL/dC against central differences of the GPU loss, h = 1e-3 pF."""
    c = _case("n6")
    C0 = c.C[:2].clone()
    _, g, _ = c.plan.loss_and_grad(C0, c.om, c.T, precision=0)
    g = g.cpu().numpy()
    h = 1e-15
    fd = np.zeros_like(g)
    for k in range(C0.shape[1]):
        Cp = C0.clone(); Cp[:, k] += h
        Cm = C0.clone(); Cm[:, k] -= h
        lp, _, _ = c.plan.loss_and_grad(Cp, c.om, c.T, precision=0, grad=False)
        lm, _, _ = c.plan.loss_and_grad(Cm, c.om, c.T, precision=0, grad=False)
        fd[:, k] = ((lp - lm) / (2 * h)).cpu().numpy()
    assert _nrel(g, fd, axis=1).max() < 1e-5


def test_deterministic_repeat(dev):
    c = _case("n64")
    a = c.plan.loss_and_grad(c.C, c.om, c.T, precision=1)
    b = c.plan.loss_and_grad(c.C, c.om, c.T, precision=1)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ----------------------------------------------------------------- autograd

def test_autograd_backward_matches_oracle(dev):
    from paper_2503_18479_amd import cosim_field
    c = _case("n25")
    C = c.C.clone().requires_grad_(True)
    Bz = cosim_field(C, c.plan, c.om, 0)
    L = ((Bz.abs() - c.T[None, None, :]) ** 2).mean(dim=(1, 2)).sum()
    L.backward()
    gr = c.oracle_grad()
    assert _nrel(C.grad.cpu().numpy(), gr, axis=1).max() < 1e-9


def test_autograd_gradcheck(dev):
    from paper_2503_18479_amd import cosim_field
    c = _case("n6")
    scale = 1e-12

    def f(Cp):
        return cosim_field(Cp * scale, c.plan, c.om, 0)

    Cp = (c.C[:2] / scale).clone().requires_grad_(True)
    assert torch.autograd.gradcheck(f, (Cp,), eps=1e-4, atol=1e-12, rtol=1e-4)


# ----------------------------------------------------------------- full-size sampled parity

def test_full_size_array8x8_operators(dev):
    """The 8x8 array at 65,536 points: M in full and G at sampled rows against
    the oracle (loss and gradient at this size: tests/test_gpu_fullsize.py)."""
    from paper_2503_18479_amd import Geometry, Plan
    wl = W.config3_array8x8(batch=1)
    g = wl.geom
    _say("[full] assembling 8x8 / 65536 points")
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    rng = np.random.default_rng(11)
    prow = np.sort(rng.choice(wl.P, 1024, replace=False))
    Gr = O.field_matrix(g.verts, g.seg_off, wl.pts[prow])
    Gd = plan.G()[torch.tensor(prow, device=dev)].cpu().numpy()
    assert _nrel(Gd, Gr) < 1e-12
    assert _nrel(plan.M(), O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)) < 1e-12


# ----------------------------------------------------------------- solver paths

def _custom_case(dev, R, C_override=None, seed=21):
    from paper_2503_18479_amd import Geometry, Plan
    wl = W.small_array(3, 2, batch=3, grid=11, n_freq=2, seed=seed)
    g = wl.geom
    g.R[:] = R
    if C_override is not None:
        C_override(wl)
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    return wl, G, M, Phi, plan


@pytest.mark.parametrize("prec", [0, 1])
def test_loss_and_grad_without_resistance_uses_pivoting(dev, prec):
    """R = 0: the unpivoted LDL^T path does not apply; results still match."""
    wl, G, M, Phi, plan = _custom_case(dev, 0.0)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
    Lr = O.evaluate(G, M, wl.geom.R, Phi, wl.C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, wl.geom.R, Phi, wl.C, wl.omega, wl.target)
    assert int(st.abs().sum()) == 0
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < TOL[prec]
    assert _nrel(grad.cpu().numpy(), gr, axis=1).max() < TOL[prec]


def test_loss_and_grad_small_pivot_falls_back(dev):
    """Tiny R with one loop tuned to its own resonance gives a tiny LDL^T pivot;
    that configuration is re-solved with pivoting, the others are not."""
    def tune(wl):
        g = wl.geom
        Mloc = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
        w = wl.omega[0]
        wl.C[0, 0] = 1.0 / (w * w * Mloc[0, 0])
    wl, G, M, Phi, plan = _custom_case(dev, 1e-6, tune)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=0)
    Lr = O.evaluate(G, M, wl.geom.R, Phi, wl.C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, wl.geom.R, Phi, wl.C, wl.omega, wl.target)
    assert int(st.abs().sum()) == 0
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < 1e-9
    assert _nrel(grad.cpu().numpy(), gr, axis=1).max() < 1e-9


# ----------------------------------------------------------------- tuning variants

@pytest.mark.parametrize("prec", [0, 1, 2])
def test_every_fused_variant_matches_oracle(dev, prec):
    c = _case("n64")
    _, nv = c.plan.variants(prec)
    assert nv >= 2
    Lr = c.oracle_eval()[2]
    gr = c.oracle_grad()
    try:
        for v in range(nv):
            _say(f"[variant] prec={prec} variant={v}")
            c.plan.set_variant(prec, v)
            loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, precision=prec)
            assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < TOL[prec], v
            assert _nrel(grad.cpu().numpy(), gr, axis=1).max() < TOL[prec], v
    finally:
        c.plan.set_variant(prec, 0)


def test_every_fused_variant_multi_tile_chunks(dev):
    """A batch large enough for the fused kernels' P-chunks to hold several
    64-row tiles (at small batches every tile is a chunk of its own): 8x8
    array at 1,600 points (25 tiles, split into one chunk or into chunks of
    13 and 12 tiles depending on the variant's workgroup size), batch 8,191
    x 4 frequencies (32,764 systems, the last system block ragged).  Every
    variant in every precision against the oracle on sampled configurations,
    among them both sides of the variants' system-block boundaries and the
    last configuration."""
    wl = W.small_array(8, 8, batch=8191, grid=40, n_freq=4, seed=9)
    c = Case(wl, dev)
    cfg = [0, 1, 7, 8, 31, 32, 63, 64, 2047, 4096, 8189, 8190]
    Lr = O.evaluate(c.G, c.M, wl.geom.R, c.Phi, wl.C[cfg], wl.omega, wl.target)[2]
    gr = O.grad_adjoint(c.G, c.M, wl.geom.R, c.Phi, wl.C[cfg], wl.omega, wl.target)
    for prec in (0, 1, 2):
        _, nv = c.plan.variants(prec)
        try:
            for v in range(nv):
                _say(f"[variant, multi-tile chunks] prec={prec} variant={v}")
                c.plan.set_variant(prec, v)
                loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, precision=prec)
                assert int(st.abs().sum()) == 0
                l = loss.cpu().numpy()[cfg]
                g = grad.cpu().numpy()[cfg]
                assert np.max(np.abs(l - Lr) / Lr) < TOL[prec], (prec, v)
                assert _nrel(g, gr, axis=1).max() < TOL[prec], (prec, v)
        finally:
            c.plan.set_variant(prec, 0)


def test_autotune_picks_a_variant(dev):
    c = _case("n64")
    chosen, ms = c.plan.autotune(c.C, c.om, c.T, precision=2, reps=1)
    assert 0 <= chosen < len(ms) and np.all(ms > 0)
    assert ms[chosen] == ms.min()
    loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, precision=2)
    assert np.max(np.abs(loss.cpu().numpy() - c.oracle_eval()[2]) / c.oracle_eval()[2]) < TOL[2]
    c.plan.set_variant(2, 0)


# ----------------------------------------------------------- driver: Adam and graphs
def test_adam_step_matches_oracle(dev):
    from paper_2503_18479_amd import adam_step
    rng = np.random.default_rng(31)
    C0 = rng.uniform(20e-12, 150e-12, size=(7, 9))
    grads = [rng.standard_normal(C0.shape) * 10.0 ** rng.uniform(-4, 1) for _ in range(5)]
    C = torch.tensor(C0, device=dev)
    m = torch.zeros_like(C); v = torch.zeros_like(C)
    t = torch.zeros((1,), dtype=torch.int32, device=dev)
    Co, mo, vo = C0.copy(), np.zeros_like(C0), np.zeros_like(C0)
    for k, g in enumerate(grads, start=1):
        _say(f"[adam] step {k}")
        adam_step(C, torch.tensor(g, device=dev), m, v, t, lr=1e-13)
        Co, mo, vo = O.adam_step(Co, g, mo, vo, k, lr=1e-13)
    torch.cuda.synchronize()
    assert int(t.item()) == len(grads)
    np.testing.assert_allclose(C.cpu().numpy(), Co, rtol=1e-14, atol=0)
    np.testing.assert_allclose(m.cpu().numpy(), mo, rtol=1e-14, atol=0)
    np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=1e-13, atol=0)


def test_optimize_follows_oracle_adam(dev):
    """Four Adam steps driven by cosim_loss_and_grad (FP64) against the oracle's
    loss, adjoint gradient and Adam step."""
    c = _case("n6")
    _say("[optimize] n6 fp64, 4 steps")
    C = c.C.clone()
    hist, st = c.plan.optimize(C, c.om, c.T, steps=4, lr=1e-13, precision=0)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    Co = c.wl.C.copy(); m = np.zeros_like(Co); v = np.zeros_like(Co)
    for k in range(1, 5):
        L = c.oracle_eval(Co)[2]
        assert _nrel(hist[k - 1].cpu().numpy(), L) < 1e-9, k
        g = c.oracle_grad(Co)
        Co, m, v = O.adam_step(Co, g, m, v, k, lr=1e-13)
    np.testing.assert_allclose(C.cpu().numpy(), Co, rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", [0, 2])
def test_loss_and_grad_graph_replays_match_eager(dev, prec):
    """cosim_loss_and_grad captured once in a HIP graph; each replay (with new C
    written in place and eager work in between) equals the eager call bit for bit."""
    c = _case("n64") if prec == 2 else _case("n6")
    B, F = c.C.shape[0], c.om.shape[0]
    c.plan.reserve(B, F)
    C = c.C.clone()
    outs = (torch.empty((B,), dtype=torch.float64, device=dev), torch.empty_like(C),
            torch.empty((B, F), dtype=torch.int32, device=dev))
    c.plan.loss_and_grad(C, c.om, c.T, precision=prec, out=outs)  # warm-up
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        c.plan.loss_and_grad(C, c.om, c.T, precision=prec, out=outs)
    for rep in range(3):
        _say(f"[graph] prec={prec} replay {rep}")
        C.copy_(c.C * (1.0 + 0.05 * rep))
        gr.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outs]
        loss, g, st = c.plan.loss_and_grad(C, c.om, c.T, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(got[0], loss) and torch.equal(got[1], g) and torch.equal(got[2], st)
        L = c.oracle_eval(C.cpu().numpy())[2]
        assert _nrel(got[0].cpu().numpy(), L) < TOL[prec]


def test_optimize_in_one_graph_equals_eager(dev):
    c = _case("n25")
    _say("[optimize] n25 bf16x3, graph vs eager")
    Ca, Cb = c.C.clone(), c.C.clone()
    ha, _ = c.plan.optimize(Ca, c.om, c.T, steps=5, precision=2, graph=False)
    hb, _ = c.plan.optimize(Cb, c.om, c.T, steps=5, precision=2, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(Ca, Cb) and torch.equal(ha, hb)
    assert not torch.equal(Ca, c.C)


# ------------------------------------------------- more than 64 loops (LU + GEMM path)
BIG = ["n81", "n144", "n256"]


@pytest.mark.parametrize("name", BIG)
def test_big_assembly_solve_and_field(dev, name):
    c = _case(name)
    _say(f"[big] {name}: n={c.wl.geom.n}")
    assert _nrel(c.plan.G().cpu().numpy(), c.G) < 1e-12
    assert _nrel(c.plan.M(), c.M) < 1e-12
    I, st = c.plan.solve(c.C, c.om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir = c.oracle_eval()[0]
    assert _nrel(I.cpu().numpy(), Ir) < 1e-10
    Br = O.field(c.G, Ir)
    for prec in (0, 1, 2):
        Bz = c.plan.field(I, prec)
        torch.cuda.synchronize()
        assert _nrel(Bz.cpu().numpy(), Br) < TOL[prec], prec


@pytest.mark.parametrize("mode", [O.LOSS_MAG, O.LOSS_COMPLEX])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", BIG)
def test_big_loss_and_grad(dev, name, prec, mode):
    c = _case(name)
    _say(f"[big] {name} prec={prec} mode={mode}")
    loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, loss_mode=mode, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = c.oracle_eval(mode=mode)[2]
    gr = c.oracle_grad(mode=mode)
    el = np.abs(loss.cpu().numpy() - Lr) / Lr
    eg = _nrel(grad.cpu().numpy(), gr, axis=1)
    _say(f"[big] {name} prec={prec} mode={mode}: loss {el.max():.2e} grad {eg.max():.2e}")
    assert el.max() < TOL[prec] and eg.max() < TOL[prec]


def test_big_several_system_blocks(dev):
    """81 loops with 36 systems, below the batch the GEMM passes take: the
    matrix-core contraction kernel runs three blocks of 16 systems (five of 8
    in FP64), each wave two loop steps with its operands loaded a phase ahead;
    loss, gradient and field in every precision against the oracle."""
    c = _case("n81wide")
    I, st = c.plan.solve(c.C, c.om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir = c.oracle_eval()[0]
    Br = O.field(c.G, Ir)
    ref = {mode: (c.oracle_eval(mode=mode)[2], c.oracle_grad(mode=mode))
           for mode in (O.LOSS_MAG, O.LOSS_COMPLEX)}
    for prec in (0, 1, 2):
        Bz = c.plan.field(I, prec)
        torch.cuda.synchronize()
        assert _nrel(Bz.cpu().numpy(), Br) < TOL[prec], prec
        for mode, (Lr, gr) in ref.items():
            loss, grad, st = c.plan.loss_and_grad(c.C, c.om, c.T, loss_mode=mode, precision=prec)
            torch.cuda.synchronize()
            assert int(st.abs().sum()) == 0
            el = np.abs(loss.cpu().numpy() - Lr) / Lr
            eg = _nrel(grad.cpu().numpy(), gr, axis=1)
            _say(f"[big] n81wide prec={prec} mode={mode}: loss {el.max():.2e} grad {eg.max():.2e}")
            assert el.max() < TOL[prec] and eg.max() < TOL[prec], (prec, mode)


def test_big_autograd_backward_matches_oracle(dev):
    from paper_2503_18479_amd import cosim_field
    c = _case("n81")
    C = c.C.clone().requires_grad_(True)
    Bz = cosim_field(C, c.plan, c.om, 0)
    T = c.T.to(torch.float64)
    L = ((Bz.abs() - T) ** 2).mean(dim=(1, 2))
    L.sum().backward()
    torch.cuda.synchronize()
    gr = c.oracle_grad()
    assert _nrel(C.grad.cpu().numpy(), gr) < 1e-9


def test_big_without_resistance_pivots(dev):
    """R = 0: the impedance has no positive Hermitian part; the pivoted LU of
    the large-loop path handles it like any other system."""
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wl = W.small_array(9, 9, batch=2, grid=9, n_freq=2, seed=22)
    g = wl.geom
    g.R[:] = 0.0
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = oracle_M_array(g)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = O.evaluate(G, M, g.R, Phi, wl.C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < 1e-9
    assert np.max(_nrel(grad.cpu().numpy(), gr, axis=1)) < 1e-9


def test_big_small_pivot_falls_back(dev):
    """Above 64 loops: tiny R with one loop tuned to its own resonance gives a
    tiny pivot in the blocked LDL^T; that system is re-factored with pivoting
    and every result still matches the oracle."""
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wl = W.small_array(9, 9, batch=3, grid=9, n_freq=2, seed=23)
    g = wl.geom
    g.R[:] = 1e-6
    M = oracle_M_array(g)
    w = wl.omega[0]
    wl.C[1, 0] = 1.0 / (w * w * M[0, 0])
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = O.evaluate(G, M, g.R, Phi, wl.C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < 1e-9
    assert np.max(_nrel(grad.cpu().numpy(), gr, axis=1)) < 1e-9
    I, st = plan.solve(C, om)
    torch.cuda.synchronize()
    Ir = O.evaluate(G, M, g.R, Phi, wl.C, wl.omega, wl.target)[0]
    assert _nrel(I.cpu().numpy(), Ir) < 1e-9


def test_big_bad_input_flags(dev):
    c = _case("n144")
    C = c.C.clone()
    C[1, 5] = 0.0
    C[0, 3] = -C[0, 3]
    loss, grad, st = c.plan.loss_and_grad(C, c.om, c.T, precision=0)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert np.all(st[1] & 1) and np.all(st[0] & 8) and not np.any(st[0] & 1)
    assert np.isnan(loss[1].item()) and np.isfinite(loss[0].item())


def test_full_size_array32x32_sampled(dev):
    """The 32x32 array (1,024 loops) at 262,144 points: M in full, G at
    sampled points, I for sampled configurations and B_z at sampled points
    against the oracle (loss and gradient at this size against stored oracle
    values: tests/test_gpu_fullsize.py)."""
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wl = W.config5_array32x32(batch=8)
    g = wl.geom
    _say("[c5] assembling 32x32 / 262144 points")
    pts = torch.tensor(wl.pts, device=dev)
    plan = Plan(Geometry.from_workload(g), pts, wl.bext_z, precisions=["fp64"])
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    _say("[c5] oracle M (1,024 loops)")
    Mr = oracle_M_array(g)
    assert _nrel(plan.M(), Mr) < 1e-12
    rng = np.random.default_rng(51)
    prow = np.sort(rng.choice(wl.P, 256, replace=False))
    Gr = O.field_matrix(g.verts, g.seg_off, wl.pts[prow])
    Gd = plan.G()[torch.tensor(prow, device=dev)].cpu().numpy()
    assert _nrel(Gd, Gr) < 1e-12
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    cs = [0, 5]
    _say("[c5] solve")
    I, st = plan.solve(C, om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir = O.currents(Mr, g.R, Phi, wl.C[cs], wl.omega)
    assert _nrel(I.cpu().numpy()[cs], Ir) < 1e-10
    _say("[c5] field")
    Bz = plan.field(I, 0)
    torch.cuda.synchronize()
    assert _nrel(Bz.cpu().numpy()[cs][:, :, prow], O.field(Gr, Ir)) < 1e-9


# ------------------------------------------------- ragged instances (one call, many plans)
def _ragged(dev, count=8, seed_stream=0):
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wls = W.config4_instances(count, grid_range=(10, 18), stream=seed_stream)
    inst = []
    for wl in wls:
        g = wl.geom
        plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z,
                    precisions=["fp64", "bf16x3"])
        inst.append(dict(wl=wl, plan=plan, G=O.field_matrix(g.verts, g.seg_off, wl.pts),
                         M=oracle_M_array(g), Phi=O.flux(g.verts, g.seg_off, wl.bext_z),
                         C=torch.tensor(wl.C, device=dev), om=torch.tensor(wl.omega, device=dev),
                         T=torch.tensor(wl.target, device=dev)))
    return inst


@pytest.mark.parametrize("prec", [0, 2])
def test_ragged_instances_match_oracle(dev, prec):
    from paper_2503_18479_amd import loss_and_grad_many
    inst = _ragged(dev)
    _say(f"[ragged] prec={prec} sizes={[(i['wl'].geom.n, i['wl'].P, i['wl'].F) for i in inst]}")
    outs = loss_and_grad_many([i["plan"] for i in inst], [i["C"] for i in inst],
                              [i["om"] for i in inst], [i["T"] for i in inst], precision=prec)
    torch.cuda.synchronize()
    for i, (loss, grad, st) in zip(inst, outs):
        wl = i["wl"]
        assert int(st.abs().sum()) == 0
        Lr = O.evaluate(i["G"], i["M"], wl.geom.R, i["Phi"], wl.C, wl.omega, wl.target)[2]
        gr = O.grad_adjoint(i["G"], i["M"], wl.geom.R, i["Phi"], wl.C, wl.omega, wl.target)
        assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < TOL[prec], wl.name
        assert np.max(_nrel(grad.cpu().numpy(), gr, axis=1)) < TOL[prec], wl.name
    # the same numbers as one call per plan
    for i, (loss, grad, st) in zip(inst, outs):
        l1, g1, s1 = i["plan"].loss_and_grad(i["C"], i["om"], i["T"], precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(l1, loss) and torch.equal(g1, grad) and torch.equal(s1, st)


def test_assembly_mask_refuses_missing_copies(dev):
    from paper_2503_18479_amd import CosimError, Geometry, Plan
    wl = W.small_array(3, 2, batch=2, grid=9, n_freq=2, seed=31)
    plan = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), wl.bext_z,
                precisions=["bf16x3"])
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, T, precision=2)
    torch.cuda.synchronize()
    assert torch.isfinite(loss).all()
    I, _ = plan.solve(C, om)
    assert torch.isfinite(plan.field(I, 2)).all()  # the bf16 copies serve the bf16 field
    for call in (lambda: plan.loss_and_grad(C, om, T, precision=0),
                 lambda: plan.loss_and_grad(C, om, T, precision=1),
                 lambda: plan.G(),
                 lambda: plan.field(I, 0),
                 lambda: plan.field(I, 1)):
        with pytest.raises(CosimError):
            call()


# ------------------------------------------- the other circuit variables (R, L, w), Eq. 13, projection

@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", ["n25", "n64", "circle", "n81"])
def test_parameter_gradients_match_oracle(dev, name, prec):
    """dL/dR, dL/dL (series inductance per loop) and dL/dw from
    cosim_loss_and_grad_params against the oracle's adjoint form (itself pinned
    to forward sensitivity and differences); dL/dC and the loss as in
    cosim_loss_and_grad."""
    c = _case(name)
    _say(f"[params] {name} prec={prec}")
    loss, gC, gR, gL, gw, st = c.plan.loss_and_grad_params(c.C, c.om, c.T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    g = c.wl.geom
    rR, rL, rw = O.grad_params_adjoint(c.G, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, c.wl.target)
    tol = TOL[prec]
    assert np.max(_nrel(gC.cpu().numpy(), c.oracle_grad(), axis=1)) < tol
    assert np.max(_nrel(gR.cpu().numpy(), rR, axis=1)) < tol
    assert np.max(_nrel(gL.cpu().numpy(), rL, axis=1)) < tol
    assert np.max(_nrel(gw.cpu().numpy(), rw, axis=1)) < tol
    l2, g2, _ = c.plan.loss_and_grad(c.C, c.om, c.T, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(l2, loss) and torch.equal(g2, gC)


def test_parameter_gradients_without_resistance(dev):
    """R = 0: the pivoted path (Gauss-Jordan record) supplies the adjoint."""
    wl, G, M, Phi, plan = _custom_case(dev, 0.0)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    loss, gC, gR, gL, gw, st = plan.loss_and_grad_params(C, om, T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    rR, rL, rw = O.grad_params_adjoint(G, M, wl.geom.R, Phi, wl.C, wl.omega, wl.target)
    # without resistance Z = jX (X real symmetric): I is real, mu imaginary, so
    # dL/dR = -2 Re(mu_k I_k) vanishes; compare on the scale |dL/dL| / w
    scale = np.abs(rL).max() / wl.omega.max()
    assert np.abs(rR).max() < 1e-12 * scale
    assert np.abs(gR.cpu().numpy() - rR).max() < 1e-9 * scale
    assert np.max(_nrel(gL.cpu().numpy(), rL, axis=1)) < 1e-9
    assert np.max(_nrel(gw.cpu().numpy(), rw, axis=1)) < 1e-9


@pytest.mark.parametrize("name", ["n25", "circle", "n81"])
def test_resonant_capacitance_matches_oracle(dev, name):
    c = _case(name)
    for coupled in (False, True):
        Cr = c.plan.resonant_capacitance(c.om, coupled)
        torch.cuda.synchronize()
        ref = np.stack([O.resonant_capacitance(c.M, w, coupled) for w in c.wl.omega])
        assert _nrel(Cr.cpu().numpy(), ref) < 1e-12


def test_tanh_projection_and_clip(dev):
    from paper_2503_18479_amd import tanh_projection, clip_
    th = np.linspace(-7, 7, 1001)
    C, dC = tanh_projection(torch.tensor(th, device=dev), 10e-12, 300e-12, derivative=True)
    rC, rdC = O.tanh_projection(th, 10e-12, 300e-12)
    assert _nrel(C.cpu().numpy(), rC) < 1e-15 and _nrel(dC.cpu().numpy(), rdC) < 1e-14
    x = torch.tensor(np.linspace(-1.0, 2.0, 301), device=dev)
    clip_(x, 0.0, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), np.clip(np.linspace(-1.0, 2.0, 301), 0.0, 1.0))


def test_multi_start_sweep_is_the_batch_of_single_starts(dev):
    """A batched multi-start sweep (many initial C in one batch, Sec. V-A) runs
    every start independently: each trajectory equals the one optimised alone,
    and Eq. 13's capacitance is a start like any other."""
    c = _case("circle")
    w = c.wl.omega
    Cr = c.plan.resonant_capacitance(c.om, coupled=False)[0]
    starts = torch.linspace(2e-12, 30e-12, 7, dtype=torch.float64, device=dev)[:, None]
    starts = torch.cat([starts, Cr[None, :]], dim=0).contiguous()
    T = c.T
    Cb = starts.clone()
    hb, _ = c.plan.optimize(Cb, c.om, T, steps=20, precision=0, lr=2e-13)
    for i in (0, 3, 7):
        Ci = starts[i:i + 1].clone()
        hi, _ = c.plan.optimize(Ci, c.om, T, steps=20, precision=0, lr=2e-13)
        torch.cuda.synchronize()
        assert _nrel(Ci.cpu().numpy(), Cb[i:i + 1].cpu().numpy()) < 1e-12
        assert _nrel(hi[:, 0].cpu().numpy(), hb[:, i].cpu().numpy()) < 1e-12


def test_parameter_gradients_on_a_fresh_plan_with_growing_batches(dev):
    """Regression: on a fresh plan the first cosim_loss_and_grad_params call
    grows the regular workspace after its own adjoint-solution workspace was
    allocated; the latter must survive that growth.  Two calls with growing
    batches, results against the oracle."""
    from paper_2503_18479_amd import Geometry, Plan
    wl = W.small_array(3, 3, batch=5, grid=7, n_freq=2, seed=31)
    g = wl.geom
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    om = torch.tensor(wl.omega, device=dev); T = torch.tensor(wl.target, device=dev)
    for nb in (1, 5):
        C = torch.tensor(wl.C[:nb], device=dev)
        loss, gC, gR, gL, gw, st = plan.loss_and_grad_params(C, om, T, precision=0)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        rR, rL, rw = O.grad_params_adjoint(G, M, g.R, Phi, wl.C[:nb], wl.omega, wl.target)
        assert np.max(_nrel(gR.cpu().numpy(), rR, axis=1)) < 1e-9
        assert np.max(_nrel(gL.cpu().numpy(), rL, axis=1)) < 1e-9
        assert np.max(_nrel(gw.cpu().numpy(), rw, axis=1)) < 1e-9


# ------------------------------------------- enhancement factor (Sec. IV-B)

@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", ["n25", "n64", "n81"])
def test_ratio_loss_and_grad_matches_oracle(dev, name, prec):
    """COSIM_LOSS_RATIO: beta = |bext + B_z| / |bext| against target factors,
    loss and dL/dC against the oracle (fused kernels and the GEMM path)."""
    c = _case(name)
    rng = np.random.default_rng(41)
    beta = rng.uniform(0.8, 1.6, c.wl.P)
    Tb = torch.tensor(beta, device=dev)
    loss, grad, st = c.plan.loss_and_grad(c.C, c.om, Tb, loss_mode=2, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    g = c.wl.geom
    Lr = O.evaluate(c.G, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, beta, O.LOSS_RATIO, c.wl.bext_z)[2]
    gr = O.grad_adjoint(c.G, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, beta, O.LOSS_RATIO, c.wl.bext_z)
    el = np.max(np.abs(loss.cpu().numpy() - Lr) / Lr)
    eg = np.max(_nrel(grad.cpu().numpy(), gr, axis=1))
    _say(f"[ratio] {name} prec={prec}: loss {el:.2e} grad {eg:.2e}")
    assert el < TOL[prec] and eg < TOL[prec]


def test_ratio_loss_needs_an_incident_field(dev):
    from paper_2503_18479_amd import Geometry, Plan, CosimError
    wl = W.small_array(2, 2, batch=1, grid=5, n_freq=1, seed=3)
    plan = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), 0.0)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    with pytest.raises(CosimError):
        plan.loss_and_grad(C, om, torch.ones(wl.P, dtype=torch.float64, device=dev), loss_mode=2)


# --------------------------------------- field components (Sec. I-B: B_x, B_y)

@functools.lru_cache(maxsize=None)
def _component_plan(name, comp):
    from paper_2503_18479_amd import Plan
    c = _case(name)
    g = c.wl.geom
    return Plan(c.geom, c.pts, c.wl.bext_z, component=comp), O.field_matrix(g.verts, g.seg_off, c.wl.pts, comp)


@pytest.mark.parametrize("comp", [0, 1])
@pytest.mark.parametrize("name", ["n25", "circle", "n81"])
def test_field_component_matches_oracle(dev, name, comp):
    """G of B_x / B_y, the field from the solved currents, and the loss and
    dL/dC on that component in every precision."""
    c = _case(name)
    plan, Gc = _component_plan(name, comp)
    _say(f"[component] {name} comp={comp}")
    assert _nrel(plan.G().cpu().numpy(), Gc) < 1e-12
    g = c.wl.geom
    I, st = plan.solve(c.C, c.om)
    B = plan.field(I).cpu().numpy()
    Ir = O.currents(c.M, g.R, c.Phi, c.wl.C, c.wl.omega)
    assert _nrel(B, O.field(Gc, Ir)) < 1e-10
    T = 0.7 * np.abs(O.field(Gc, Ir)).mean(axis=(0, 1))   # any magnitudes will do
    Tt = torch.tensor(T, device=dev)
    Lr = O.evaluate(Gc, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, T)[2]
    gr = O.grad_adjoint(Gc, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, T)
    for prec in (0, 1, 2):
        loss, grad, st = plan.loss_and_grad(c.C, c.om, Tt, precision=prec)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        el = np.max(np.abs(loss.cpu().numpy() - Lr) / Lr)
        eg = np.max(_nrel(grad.cpu().numpy(), gr, axis=1))
        _say(f"  prec={prec}: loss {el:.2e} grad {eg:.2e}")
        assert el < TOL[prec] and eg < TOL[prec]


def test_ratio_loss_needs_the_z_component(dev):
    from paper_2503_18479_amd import CosimError
    c = _case("n25")
    plan, _ = _component_plan("n25", 0)
    with pytest.raises(CosimError):
        plan.loss_and_grad(c.C, c.om, torch.ones_like(c.T), loss_mode=2)


# -------------------------------------------- drive port (Sec. IV-A, Eq. 4)

class DriveCase:
    """An array with an excitation coil as its last loop, driven through a
    50 ohm port with 1 W; the coil has no capacitor (C = +inf)."""

    def __init__(self, geom, pts, batch, freqs, bext, seed, dev, phase=0.4, array_M=False):
        from paper_2503_18479_amd import Geometry, Plan
        self.g = geom
        rng = np.random.default_rng([7, seed])
        n = geom.n
        self.n = n
        self.pts_h = pts
        self.omega = 2 * np.pi * np.asarray(freqs, float)
        C = rng.uniform(20e-12, 150e-12, (batch, n))
        C[:, -1] = np.inf
        self.C_h = C
        self.G = O.field_matrix(geom.verts, geom.seg_off, pts)
        self.M = O.inductance_matrix_fast(geom.verts, geom.seg_off, geom.wire_a)
        self.Phi = O.flux(geom.verts, geom.seg_off, bext)
        self.R = geom.R.copy(); self.R[-1] += 50.0
        self.emf = np.zeros(n, complex); self.emf[-1] = O.drive_emf(1.0, 50.0, phase)
        I = O.currents(self.M, self.R, self.Phi, C[:1], self.omega[:1], self.emf)
        self.T_h = 0.8 * np.abs(O.field(self.G, I))[0, 0] + 1e-7 * rng.uniform(size=len(pts))
        self.plan = Plan(Geometry.from_workload(geom), torch.tensor(pts, device=dev), bext)
        self.plan.set_drive([n - 1], power=1.0, phase=phase, z0=50.0)
        self.C = torch.tensor(C, device=dev)
        self.om = torch.tensor(self.omega, device=dev)
        self.T = torch.tensor(self.T_h, device=dev)

    def args(self):
        return self.G, self.M, self.R, self.Phi, self.C_h, self.omega, self.T_h


@functools.lru_cache(maxsize=None)
def _drive(name):
    dev = torch.device("cuda:0")
    if name == "drive1":   # single cell r = 30 mm and its coil (Sec. IV-A): NP = 32
        geom = W.with_drive_coil(W.single_circle(0.03, 64, 1e-3, 0.5), radius=0.0445, z=0.01)
        return DriveCase(geom, W.grid_points(13, 0.08, [-0.0224]), 6, [123.5e6, 128e6], 0.0, 1, dev)
    if name == "drive9":   # 3x3 array, coil and a uniform incident field together
        geom = W.with_drive_coil(W.square_array(3, 3, 0.03, 0.035, 16), radius=0.06, z=0.015)
        return DriveCase(geom, W.grid_points(15, 0.1, [0.01]), 4, [118e6, 128e6, 138e6], 1e-6, 2,
                         dev, phase=1.1)
    if name == "drive81":  # 9x9 array and a square coil: 82 loops, the large-loop path
        geom = W.with_drive_coil(W.square_array(9, 9, 0.03, 0.035, 32), radius=0.17, z=0.02,
                                 square=True)
        return DriveCase(geom, W.grid_points(40, 0.3, [0.01]), 3, [123.5e6, 128e6], 0.0, 3, dev)
    raise KeyError(name)


DRIVES = ["drive1", "drive9", "drive81"]


@pytest.mark.parametrize("name", DRIVES)
def test_drive_solve_matches_oracle(dev, name):
    d = _drive(name)
    _say(f"[drive solve] {name}")
    I, st = d.plan.solve(d.C, d.om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir = O.currents(d.M, d.R, d.Phi, d.C_h, d.omega, d.emf)
    assert np.max(_nrel(I.cpu().numpy(), Ir, axis=2)) < 1e-10


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", DRIVES)
def test_drive_loss_and_grad_matches_oracle(dev, name, prec):
    d = _drive(name)
    _say(f"[drive loss] {name} prec={prec}")
    loss, grad, st = d.plan.loss_and_grad(d.C, d.om, d.T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = O.evaluate(*d.args(), emf=d.emf)[2]
    gr = O.grad_adjoint(*d.args(), emf=d.emf)
    g = grad.cpu().numpy()
    assert np.all(g[:, -1] == 0.0)       # the coil has no capacitor
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < TOL[prec]
    assert np.max(_nrel(g, gr, axis=1)) < TOL[prec]


@pytest.mark.parametrize("name", DRIVES)
def test_drive_parameter_gradients_match_oracle(dev, name):
    d = _drive(name)
    _say(f"[drive params] {name}")
    loss, gC, gR, gL, gw, st = d.plan.loss_and_grad_params(d.C, d.om, d.T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    rR, rL, rw = O.grad_params_adjoint(*d.args(), emf=d.emf)
    assert np.max(_nrel(gR.cpu().numpy(), rR, axis=1)) < 1e-9
    assert np.max(_nrel(gL.cpu().numpy(), rL, axis=1)) < 1e-9
    assert np.max(_nrel(gw.cpu().numpy(), rw, axis=1)) < 1e-9


def test_drive_ports_replace_and_clear(dev):
    """set_drive replaces the port set; an empty set restores the plan."""
    from paper_2503_18479_amd import CosimError
    d = _drive("drive9")
    d.plan.set_drive([d.n - 1], power=4.0, phase=1.1)     # 4 W: twice the EMF
    I4, _ = d.plan.solve(d.C, d.om)
    d.plan.set_drive([])
    Ic, _ = d.plan.solve(d.C, d.om)
    d.plan.set_drive([d.n - 1], power=1.0, phase=1.1)     # back to the case's ports
    torch.cuda.synchronize()
    R0 = d.g.R.copy()
    Ir4 = O.currents(d.M, d.R, d.Phi, d.C_h, d.omega, 2.0 * d.emf)
    assert np.max(_nrel(I4.cpu().numpy(), Ir4, axis=2)) < 1e-10
    # without ports the coil has R = 0 and, with C = inf, no impedance but
    # j w L: the flux still drives it
    Ic_ref = O.currents(d.M, R0, d.Phi, d.C_h, d.omega)
    assert np.max(_nrel(Ic.cpu().numpy(), Ic_ref, axis=2)) < 1e-10
    with pytest.raises(CosimError):
        d.plan.set_drive([0, 0])
    with pytest.raises(CosimError):
        d.plan.set_drive([d.n])
    with pytest.raises(CosimError):
        d.plan.loss_and_grad(d.C, d.om, torch.ones_like(d.T), loss_mode=2)


# ----------------------- FP32 factorisation with FP64 iterative refinement

@functools.lru_cache(maxsize=None)
def _refined(name, max_iter=8, tol=0.0):
    from paper_2503_18479_amd import Plan
    c = _case(name)
    plan = Plan(c.geom, c.pts, c.wl.bext_z)
    plan.set_refinement(True, max_iter, tol)
    return plan


@pytest.mark.parametrize("name", BIG)
def test_refined_solve_matches_oracle(dev, name):
    c = _case(name)
    _say(f"[refined solve] {name}")
    I, st = _refined(name).solve(c.C, c.om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    assert np.max(_nrel(I.cpu().numpy(), c.oracle_eval()[0], axis=2)) < 1e-10


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", BIG)
def test_refined_loss_and_grad_matches_oracle(dev, name, prec):
    c = _case(name)
    _say(f"[refined loss] {name} prec={prec}")
    loss, grad, st = _refined(name).loss_and_grad(c.C, c.om, c.T, precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = c.oracle_eval()[2]
    el = np.max(np.abs(loss.cpu().numpy() - Lr) / Lr)
    eg = np.max(_nrel(grad.cpu().numpy(), c.oracle_grad(), axis=1))
    _say(f"  loss {el:.2e} grad {eg:.2e}")
    assert el < TOL[prec] and eg < TOL[prec]


def test_refined_parameter_gradients_match_oracle(dev):
    c = _case("n81")
    loss, gC, gR, gL, gw, st = _refined("n81").loss_and_grad_params(c.C, c.om, c.T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    g = c.wl.geom
    rR, rL, rw = O.grad_params_adjoint(c.G, c.M, g.R, c.Phi, c.wl.C, c.wl.omega, c.wl.target)
    for a, r in ((gC, c.oracle_grad()), (gR, rR), (gL, rL), (gw, rw)):
        assert np.max(_nrel(a.cpu().numpy(), r, axis=1)) < 1e-9


def test_refined_autograd_backward_matches_oracle(dev):
    from paper_2503_18479_amd import cosim_field
    c = _case("n81")
    C = c.C.clone().requires_grad_(True)
    Bz = cosim_field(C, _refined("n81"), c.om, 0)
    L = ((Bz.abs() - c.T.to(torch.float64)) ** 2).mean(dim=(1, 2))
    L.sum().backward()
    torch.cuda.synchronize()
    assert _nrel(C.grad.cpu().numpy(), c.oracle_grad()) < 1e-9


def test_refined_fallback_when_refinement_does_not_converge(dev):
    """A tolerance no system can meet sends every system to the pivoted FP64
    factorisation, forward and adjoint; results still match the oracle."""
    c = _case("n144")
    plan = _refined("n144", 1, 1e-300)
    I, st = plan.solve(c.C, c.om)
    loss, grad, st2 = plan.loss_and_grad(c.C, c.om, c.T, precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0 and int(st2.abs().sum()) == 0
    assert np.max(_nrel(I.cpu().numpy(), c.oracle_eval()[0], axis=2)) < 1e-10
    Lr = c.oracle_eval()[2]
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < 1e-9
    assert np.max(_nrel(grad.cpu().numpy(), c.oracle_grad(), axis=1)) < 1e-9


def test_refined_small_pivot_falls_back(dev):
    """Tiny R with one loop at its own resonance: that system's FP32 factor
    meets a tiny pivot and takes the FP64 fallback; the others refine."""
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wl = W.small_array(9, 9, batch=3, grid=9, n_freq=2, seed=23)
    g = wl.geom
    g.R[:] = 1e-6
    M = oracle_M_array(g)
    wl.C[1, 0] = 1.0 / (wl.omega[0] ** 2 * M[0, 0])
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    plan.set_refinement(True)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    loss, grad, st = plan.loss_and_grad(C, om, torch.tensor(wl.target, device=dev), precision=0)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = O.evaluate(G, M, g.R, Phi, wl.C, wl.omega, wl.target)[2]
    gr = O.grad_adjoint(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < 1e-9
    assert np.max(_nrel(grad.cpu().numpy(), gr, axis=1)) < 1e-9


def test_refinement_switch_keeps_captured_graphs_valid(dev):
    """cosim_plan_set_refinement keeps the workspace: a graph of
    cosim_loss_and_grad captured with the FP64 factor (81 loops) replays,
    after switching refinement on and running eager calls in that mode (the
    FP32 factor slots are added then), to the FP64-factor results bit for
    bit, and again after switching back; the refined calls match the oracle."""
    c = _case("n81")
    plan = c.plan
    plan.set_refinement(False)
    plan.reserve(c.C.shape[0], c.om.shape[0])
    loss = torch.empty((c.C.shape[0],), dtype=torch.float64, device=dev)
    grad = torch.empty_like(c.C)
    st = torch.empty((c.C.shape[0], c.om.shape[0]), dtype=torch.int32, device=dev)
    out = (loss, grad, st)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.loss_and_grad(c.C, c.om, c.T, precision=2, out=out)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.loss_and_grad(c.C, c.om, c.T, precision=2, out=out)
    torch.cuda.synchronize()
    ref = plan.loss_and_grad(c.C, c.om, c.T, precision=2)
    torch.cuda.synchronize()
    Lr = c.oracle_eval()[2]
    gr = c.oracle_grad()
    try:
        for refine in (True, False):
            plan.set_refinement(refine)
            l1, g1, s1 = plan.loss_and_grad(c.C, c.om, c.T, precision=2)
            torch.cuda.synchronize()
            assert int(s1.abs().sum()) == 0
            assert np.max(np.abs(l1.cpu().numpy() - Lr) / Lr) < TOL[2]
            assert _nrel(g1.cpu().numpy(), gr, axis=1).max() < TOL[2]
            loss.zero_(); grad.zero_(); st.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(loss, ref[0]) and torch.equal(grad, ref[1]) and torch.equal(st, ref[2]), refine
    finally:
        plan.set_refinement(False)
        del g


def test_refined_1024_loops(dev):
    """The 32x32 array's 1,024 loops (16 panels) with refinement, few
    configurations and points: currents, loss and dL/dC against the oracle."""
    from paper_2503_18479_amd import Geometry, Plan
    from array_oracle import oracle_M_array
    wl = W.config5_array32x32(batch=3, grid=24)
    g = wl.geom
    _say(f"[refined 1024] n={g.n} P={wl.P}")
    M = oracle_M_array(g)
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    plan.set_refinement(True)
    C = torch.tensor(wl.C, device=dev); om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    I, st = plan.solve(C, om)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Ir, _, Lr = O.evaluate(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    assert np.max(_nrel(I.cpu().numpy(), Ir, axis=2)) < 1e-10
    gr = O.grad_adjoint(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    for prec in (0, 2):
        loss, grad, st = plan.loss_and_grad(C, om, T, precision=prec)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        assert np.max(np.abs(loss.cpu().numpy() - Lr) / Lr) < TOL[prec]
        assert np.max(_nrel(grad.cpu().numpy(), gr, axis=1)) < TOL[prec]


# ------------------------------------------- ragged instances in a HIP graph

def test_ragged_graph_replay_matches_eager(dev):
    """cosim_loss_and_grad_many captured once (6, 25 and 81 loops: fused
    kernels, side streams and the GEMM path) and replayed three times, each
    after eager work with new capacitances; every replay equals the eager
    call bit for bit."""
    from paper_2503_18479_amd import (Geometry, Plan, loss_and_grad_many,
                                      capture_loss_and_grad_many)
    wls = [W.small_array(3, 2, batch=5, grid=20, n_freq=3, seed=31),
           W.small_array(5, 5, batch=4, grid=17, n_freq=2, seed=32),
           W.small_array(9, 9, batch=3, grid=40, n_freq=2, seed=33)]
    plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
             for w in wls]
    Cs = [torch.tensor(w.C, device=dev) for w in wls]
    Os = [torch.tensor(w.omega, device=dev) for w in wls]
    Ts = [torch.tensor(w.target, device=dev) for w in wls]
    for prec in (0, 2):
        gr, gouts = capture_loss_and_grad_many(plans, Cs, Os, Ts, precision=prec)
        for rep in range(3):
            for C in Cs:
                C.mul_(1.0 + 0.01 * (rep + 1))
            ref = loss_and_grad_many(plans, Cs, Os, Ts, precision=prec)
            torch.cuda.synchronize()
            gr.replay()
            torch.cuda.synchronize()
            for (l, g, s), (lr, g_r, sr) in zip(gouts, ref):
                assert torch.equal(l, lr) and torch.equal(g, g_r) and torch.equal(s, sr), (prec, rep)
        del gr


def test_many_call_reruns_match_fresh_calls(dev):
    """ManyCall checks its instances once; each run() after the capacitances
    are updated in place equals a fresh loss_and_grad_many call bit for bit,
    including the loss-only form."""
    from paper_2503_18479_amd import Geometry, Plan, ManyCall, loss_and_grad_many
    wls = [W.small_array(3, 2, batch=5, grid=20, n_freq=3, seed=41),
           W.small_array(5, 5, batch=4, grid=17, n_freq=2, seed=42),
           W.small_array(9, 9, batch=3, grid=40, n_freq=2, seed=43)]
    plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
             for w in wls]
    Cs = [torch.tensor(w.C, device=dev) for w in wls]
    Os = [torch.tensor(w.omega, device=dev) for w in wls]
    Ts = [torch.tensor(w.target, device=dev) for w in wls]
    for prec, grad in ((0, True), (2, True), (2, False)):
        call = ManyCall(plans, Cs, Os, Ts, precision=prec, grad=grad)
        for rep in range(2):
            for C in Cs:
                C.mul_(1.0 + 0.02 * (rep + 1))
            outs = call.run()
            ref = loss_and_grad_many(plans, Cs, Os, Ts, precision=prec, grad=grad)
            torch.cuda.synchronize()
            for (l, g, st), (lr, g_r, sr) in zip(outs, ref):
                assert torch.equal(l, lr) and torch.equal(st, sr), (prec, grad, rep)
                assert (g is None and g_r is None) or torch.equal(g, g_r), (prec, grad, rep)


def test_grouped_large_instances_match_single_calls(dev):
    """Instances above 64 loops of one size are factored and solved together
    by cosim_loss_and_grad_many: three of 81 loops (different batches,
    frequency counts and points), two of 144 and two small ones.  Every
    result equals the instance's own cosim_loss_and_grad call bit for bit,
    in three precisions.  Under stream capture the call runs the instances
    above 64 loops one by one (a capture of their grouped launches once
    crashed the HIP runtime, cause not found); graph replays of it equal the
    single calls too."""
    from paper_2503_18479_amd import (Geometry, Plan, loss_and_grad_many,
                                      capture_loss_and_grad_many)
    wls = [W.small_array(9, 9, batch=2, grid=30, n_freq=3, seed=41),
           W.small_array(9, 9, batch=1, grid=45, n_freq=1, seed=42),
           W.small_array(12, 12, batch=2, grid=20, n_freq=2, seed=43),
           W.small_array(3, 2, batch=3, grid=16, n_freq=2, seed=44),
           W.small_array(9, 9, batch=3, grid=24, n_freq=2, seed=45),
           W.small_array(12, 12, batch=1, grid=28, n_freq=3, seed=46),
           W.small_array(5, 5, batch=2, grid=18, n_freq=1, seed=47)]
    plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
             for w in wls]
    Cs = [torch.tensor(w.C, device=dev) for w in wls]
    Os = [torch.tensor(w.omega, device=dev) for w in wls]
    Ts = [torch.tensor(w.target, device=dev) for w in wls]
    for prec in (0, 1, 2):
        _say(f"[grouped] prec={prec}")
        many = loss_and_grad_many(plans, Cs, Os, Ts, precision=prec)
        torch.cuda.synchronize()
        for pl, C, o, T, (l, g, s) in zip(plans, Cs, Os, Ts, many):
            l1, g1, s1 = pl.loss_and_grad(C, o, T, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(l, l1) and torch.equal(g, g1) and torch.equal(s, s1), prec
            assert int(s.abs().sum()) == 0
    # the complex and enhancement-ratio losses, and loss-only calls, in BF16X3
    from paper_2503_18479_amd import LOSS_COMPLEX, LOSS_RATIO
    Rs = [1.0 + 0.5 * T / T.max() for T in Ts]
    for mode, tg in ((LOSS_COMPLEX, Ts), (LOSS_RATIO, Rs)):
        for grad in (True, False):
            _say(f"[grouped] mode={mode} grad={grad}")
            many = loss_and_grad_many(plans, Cs, Os, tg, loss_mode=mode, precision=2, grad=grad)
            torch.cuda.synchronize()
            for pl, C, o, T, (l, g, s) in zip(plans, Cs, Os, tg, many):
                l1, g1, s1 = pl.loss_and_grad(C, o, T, loss_mode=mode, precision=2, grad=grad)
                torch.cuda.synchronize()
                assert torch.equal(l, l1) and torch.equal(s, s1), (mode, grad)
                assert (g is None) == (not grad)
                if grad:
                    assert torch.equal(g, g1), mode
    gr, gouts = capture_loss_and_grad_many(plans, Cs, Os, Ts, precision=0)
    for rep in range(3):
        for C in Cs:
            C.mul_(1.0 + 0.02 * (rep + 1))
        ref = [pl.loss_and_grad(C, o, T, precision=0) for pl, C, o, T in zip(plans, Cs, Os, Ts)]
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        for (l, g, s), (l1, g1, s1) in zip(gouts, ref):
            assert torch.equal(l, l1) and torch.equal(g, g1) and torch.equal(s, s1), rep
    del gr


def test_grouped_small_instances_captured(dev):
    """Instances of 64 loops or fewer of one padded size share launches also
    under stream capture: nine instances of 16 to 64 loops (padded to 32 and
    64) with other instances beside them, captured once and replayed three
    times after eager work with new capacitances; every replay equals the
    instances' own calls bit for bit."""
    from paper_2503_18479_amd import Geometry, Plan, capture_loss_and_grad_many
    shapes = [(4, 4, 2, 20, 3), (5, 5, 1, 25, 2), (6, 6, 2, 18, 1), (7, 7, 1, 22, 4),
              (8, 8, 3, 16, 2), (4, 4, 1, 30, 1), (6, 6, 1, 24, 3), (8, 8, 1, 20, 2),
              (5, 6, 2, 19, 2), (9, 9, 1, 21, 2)]
    wls = [W.small_array(nx, ny, batch=b, grid=g, n_freq=f, seed=60 + i)
           for i, (nx, ny, b, g, f) in enumerate(shapes)]
    plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
             for w in wls]
    Cs = [torch.tensor(w.C, device=dev) for w in wls]
    Os = [torch.tensor(w.omega, device=dev) for w in wls]
    Ts = [torch.tensor(w.target, device=dev) for w in wls]
    for prec in (0, 2):
        _say(f"[captured groups] prec={prec}")
        gr, gouts = capture_loss_and_grad_many(plans, Cs, Os, Ts, precision=prec)
        for rep in range(3):
            for C in Cs:
                C.mul_(1.0 + 0.01 * (rep + 1))
            ref = [pl.loss_and_grad(C, o, T, precision=prec)
                   for pl, C, o, T in zip(plans, Cs, Os, Ts)]
            torch.cuda.synchronize()
            gr.replay()
            torch.cuda.synchronize()
            for (l, g, s), (l1, g1, s1) in zip(gouts, ref):
                assert torch.equal(l, l1) and torch.equal(g, g1) and torch.equal(s, s1), (prec, rep)
        del gr


@pytest.mark.gpu
def test_grouped_calls_on_two_streams(dev):
    """Two cosim_loss_and_grad_many calls enqueued back to back on two streams,
    each with grouped instances of the same padded size: they share the
    library's per-device group workspace, so the second call's grouped work
    must wait for the first call's.  Both equal the instances' own calls bit
    for bit, twice over."""
    from paper_2503_18479_amd import Geometry, Plan, loss_and_grad_many
    shapes = [(9, 9, 2, 30, 3), (9, 9, 1, 45, 1), (9, 9, 3, 24, 2)]
    sets = []
    for base in (61, 71):
        wls = [W.small_array(nx, ny, batch=b, grid=gd, n_freq=nf, seed=base + j)
               for j, (nx, ny, b, gd, nf) in enumerate(shapes)]
        plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
                 for w in wls]
        Cs = [torch.tensor(w.C, device=dev) for w in wls]
        Os = [torch.tensor(w.omega, device=dev) for w in wls]
        Ts = [torch.tensor(w.target, device=dev) for w in wls]
        ref = [pl.loss_and_grad(C, o, T, precision=2) for pl, C, o, T in zip(plans, Cs, Os, Ts)]
        sets.append((plans, Cs, Os, Ts, ref))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(2):
        _say(f"[two streams] rep={rep}")
        outs = []
        for (plans, Cs, Os, Ts, _), s in zip(sets, (s1, s2)):
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                outs.append(loss_and_grad_many(plans, Cs, Os, Ts, precision=2))
        torch.cuda.synchronize()
        for (_, _, _, _, ref), many in zip(sets, outs):
            for (l, g, st), (l1, g1, s1r) in zip(many, ref):
                assert torch.equal(l, l1) and torch.equal(g, g1) and torch.equal(st, s1r), rep
                assert int(st.abs().sum()) == 0


@pytest.mark.gpu
def test_grouped_small_instances_match_single_calls(dev):
    """Instances of 64 loops or fewer of one padded size are factored and
    solved together by cosim_loss_and_grad_many (their contractions stay per
    instance): two of 64 loops and one of 36 (padded to 64), two of 25 and
    one of 16 (padded to 32), one of 81 alone.  Every result equals the
    instance's own call bit for bit, for the magnitude, complex and
    enhancement-ratio losses, with and without the gradient, in three
    precisions."""
    from paper_2503_18479_amd import (Geometry, Plan, loss_and_grad_many, LOSS_MAG,
                                      LOSS_COMPLEX, LOSS_RATIO)
    wls = [W.small_array(8, 8, batch=2, grid=20, n_freq=3, seed=81),
           W.small_array(6, 6, batch=3, grid=18, n_freq=2, seed=82),
           W.small_array(5, 5, batch=1, grid=25, n_freq=1, seed=83),
           W.small_array(8, 8, batch=1, grid=33, n_freq=2, seed=84),
           W.small_array(4, 4, batch=4, grid=16, n_freq=3, seed=85),
           W.small_array(5, 5, batch=2, grid=12, n_freq=2, seed=86),
           W.small_array(9, 9, batch=1, grid=16, n_freq=1, seed=87)]
    plans = [Plan(Geometry.from_workload(w.geom), torch.tensor(w.pts, device=dev), w.bext_z)
             for w in wls]
    Cs = [torch.tensor(w.C, device=dev) for w in wls]
    Os = [torch.tensor(w.omega, device=dev) for w in wls]
    Ts = [torch.tensor(w.target, device=dev) for w in wls]
    # ratio targets: enhancement factors near 1
    Rs = [1.0 + 0.5 * torch.tensor(w.target, device=dev) / float(np.max(w.target)) for w in wls]
    for mode, tg in ((LOSS_MAG, Ts), (LOSS_COMPLEX, Ts), (LOSS_RATIO, Rs)):
        for prec in (0, 1, 2):
            for grad in (True, False):
                _say(f"[small groups] mode={mode} prec={prec} grad={grad}")
                many = loss_and_grad_many(plans, Cs, Os, tg, loss_mode=mode, precision=prec,
                                          grad=grad)
                torch.cuda.synchronize()
                for pl, C, o, T, (l, g, s) in zip(plans, Cs, Os, tg, many):
                    l1, g1, s1 = pl.loss_and_grad(C, o, T, loss_mode=mode, precision=prec,
                                                  grad=grad)
                    torch.cuda.synchronize()
                    assert torch.equal(l, l1) and torch.equal(s, s1), (mode, prec, grad)
                    assert (g is None) == (not grad)
                    if grad:
                        assert torch.equal(g, g1), (mode, prec)
                    assert int(s.abs().sum()) == 0


@pytest.mark.gpu
def test_reserved_plan_captures_smaller_batch(dev):
    """cosim_plan_reserve(B, F) covers every smaller batch: a batch of one
    system splits P into more chunks (64) than the reserved batch of 8,192
    systems does, and its first call, captured straight into a HIP graph,
    must allocate nothing (an allocation inside the capture fails it).
    Replays with new capacitances equal eager calls bit for bit."""
    from paper_2503_18479_amd import Geometry, Plan
    wl = W.small_array(5, 5, batch=1, grid=64, n_freq=1, seed=93)
    pl = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), wl.bext_z)
    pl.reserve(512, 16)
    C = torch.tensor(wl.C, device=dev)
    o = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    out = (torch.empty((1,), dtype=torch.float64, device=dev),
           torch.empty((1, wl.geom.n), dtype=torch.float64, device=dev),
           torch.empty((1, 1), dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    _say("[reserve] capture of a 1-system call after reserving 8,192 systems")
    with torch.cuda.graph(g, stream=side):
        pl.loss_and_grad(C, o, T, precision=2, out=out)
    for rep in range(3):
        C.mul_(1.0 + 0.03 * (rep + 1))
        g.replay()
        torch.cuda.synchronize()
        l1, g1, s1 = pl.loss_and_grad(C, o, T, precision=2)
        torch.cuda.synchronize()
        assert torch.equal(out[0], l1) and torch.equal(out[1], g1) and torch.equal(out[2], s1), rep
        assert int(s1.abs().sum()) == 0
    del g
