"""The matrix-core contraction kernel behind cosim_field (B = G I, Eq. 7) and
cosim_field_backward (r = G^T conj(g) / 2, then the adjoint solve of Eq. 8-10)
for every padded loop count, and the autograd path that replays the forward
factorisation, against the FP64 oracle.  (The kernel's loss path above 64
loops is covered by test_gpu_parity.py and test_gpu_fullsize.py.)"""
import functools
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


SHAPES = {  # name: (nx, ny, batch, grid, n_freq, seed); loops padded to 32, 64, 128, 192, 256
    "n6": (3, 2, 7, 13, 3, 71),        # 169 points: ragged last sub-tile, 21 systems (2 blocks)
    "n49": (7, 7, 3, 11, 2, 72),
    "n81": (9, 9, 5, 12, 4, 73),       # 20 systems (FP64: three blocks of 8)
    "n144": (12, 12, 2, 10, 3, 74),
    "n256": (16, 16, 1, 9, 2, 75),
}


@functools.lru_cache(maxsize=None)
def _case(name):
    from paper_2503_18479_amd import Geometry, Plan
    nx, ny, batch, grid, nf, seed = SHAPES[name]
    wl = W.small_array(nx, ny, batch=batch, grid=grid, n_freq=nf, seed=seed)
    g = wl.geom
    dev = torch.device("cuda:0")
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = O.inductance_matrix_lattice(g.verts, g.seg_off, g.wire_a, nx, ny)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    I = O.currents(M, g.R, Phi, wl.C, wl.omega)
    rng = np.random.default_rng([seed, 1])
    gB = (rng.standard_normal((wl.B, wl.F, wl.P)) + 1j * rng.standard_normal((wl.B, wl.F, wl.P)))
    return dict(wl=wl, G=G, M=M, Phi=Phi, plan=plan, I=I, gB=gB,
                C=torch.tensor(wl.C, device=dev), om=torch.tensor(wl.omega, device=dev))


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", list(SHAPES))
def test_field_matches_oracle(dev, name, prec):
    """B = G I from the oracle's currents, and with the incident field added."""
    c = _case(name)
    _say(f"[mfma field] {name} prec={prec}")
    I = torch.tensor(c["I"], device=dev)
    Br = O.field(c["G"], c["I"])
    Bz = c["plan"].field(I, prec).cpu().numpy()
    assert _nrel(Bz, Br, axis=2).max() < TOL[prec]
    bext = c["wl"].bext_z
    Bt = c["plan"].field(I, prec, add_incident=True).cpu().numpy()
    assert _nrel(Bt, Br + bext, axis=2).max() < TOL[prec]


@pytest.mark.parametrize("reuse", [False, True])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", list(SHAPES))
def test_field_backward_matches_oracle(dev, name, prec, reuse):
    """dL/dC of an upstream gradient g (PyTorch's 2 dL/d conj(B)) in every
    contraction precision, factorising again or replaying the solve's record."""
    c = _case(name)
    wl, plan = c["wl"], c["plan"]
    _say(f"[mfma vjp] {name} prec={prec} reuse={reuse}")
    I, st = plan.solve(c["C"], c["om"])
    gB = torch.tensor(c["gB"], device=dev)
    n0 = plan.factorisations()
    gC, st2 = plan.field_backward(c["C"], c["om"], I, gB, prec, reuse=reuse)
    torch.cuda.synchronize()
    assert plan.factorisations() == n0 + (0 if reuse else 1)
    assert int(st.abs().sum()) == 0 and int(st2.abs().sum()) == 0
    gr = O.backward_from_field_grad(c["G"], c["M"], wl.geom.R, wl.C, wl.omega, c["I"], c["gB"])
    assert _nrel(gC.cpu().numpy(), gr, axis=1).max() < TOL[prec]


def test_field_backward_reuse_needs_an_intact_record(dev):
    from paper_2503_18479_amd import CosimError
    c = _case("n49")
    plan = c["plan"]
    I, _ = plan.solve(c["C"], c["om"])
    gB = torch.tensor(c["gB"], device=dev)
    # a different shape
    with pytest.raises(CosimError):
        plan.field_backward(c["C"][:1].contiguous(), c["om"], I[:1].contiguous(),
                            gB[:1].contiguous(), 0, reuse=True)
    # a call that used the workspace in between
    T = torch.zeros((c["wl"].P,), dtype=torch.float64, device=dev)
    plan.loss_and_grad(c["C"], c["om"], T, precision=0)
    with pytest.raises(CosimError):
        plan.field_backward(c["C"], c["om"], I, gB, 0, reuse=True)
    # factorising again always works
    gC, _ = plan.field_backward(c["C"], c["om"], I, gB, 0, reuse=False)
    torch.cuda.synchronize()
    assert torch.isfinite(gC).all()


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("name", ["n6", "n81", "n144"])
def test_autograd_backward_replays_forward_factor(dev, name, prec):
    """CosimField: the backward factorises nothing (the forward's record is
    replayed) and matches the oracle; with another call on the plan between
    forward and backward it factorises again and still matches."""
    from paper_2503_18479_amd import cosim_field
    c = _case(name)
    wl, plan = c["wl"], c["plan"]
    T = torch.tensor(wl.target, device=dev)
    gr = O.grad_adjoint(c["G"], c["M"], wl.geom.R, c["Phi"], wl.C, wl.omega, wl.target)
    for interleave in (False, True):
        _say(f"[autograd] {name} prec={prec} interleave={interleave}")
        C = c["C"].clone().requires_grad_(True)
        Bz = cosim_field(C, plan, c["om"], prec)
        L = ((Bz.abs().to(torch.float64) - T) ** 2).mean(dim=(1, 2)).sum()
        if interleave:
            plan.loss_and_grad(c["C"], c["om"], T, precision=0)
        n0 = plan.factorisations()
        L.backward()
        torch.cuda.synchronize()
        assert plan.factorisations() == n0 + (1 if interleave else 0)
        assert _nrel(C.grad.cpu().numpy(), gr, axis=1).max() < TOL[prec]


@functools.lru_cache(maxsize=None)
def _batch_case(name):
    """Batches large enough for the two GEMM passes above 64 loops (at least
    128 systems; 64 in FP64), with ragged row and column blocks."""
    from paper_2503_18479_amd import Geometry, Plan
    nx, batch, grid, nf, seed = {"n81": (9, 70, 21, 2, 76), "n144": (12, 33, 15, 4, 77)}[name]
    wl = W.small_array(nx, nx, batch=batch, grid=grid, n_freq=nf, seed=seed)
    g = wl.geom
    dev = torch.device("cuda:0")
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = O.inductance_matrix_lattice(g.verts, g.seg_off, g.wire_a, nx, nx)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    return dict(wl=wl, G=G, M=M, Phi=Phi, plan=plan, C=torch.tensor(wl.C, device=dev),
                om=torch.tensor(wl.omega, device=dev), T=torch.tensor(wl.target, device=dev))


@pytest.mark.parametrize("mode", [O.LOSS_MAG, O.LOSS_COMPLEX])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("name", ["n81", "n144"])
def test_gemm_passes_loss_and_grad(dev, name, prec, mode):
    c = _batch_case(name)
    wl = c["wl"]
    _say(f"[gemm] {name} S={wl.B * wl.F} prec={prec} mode={mode}")
    loss, grad, st = c["plan"].loss_and_grad(c["C"], c["om"], c["T"], loss_mode=mode,
                                             precision=prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    Lr = O.evaluate(c["G"], c["M"], wl.geom.R, c["Phi"], wl.C, wl.omega, wl.target, mode)[2]
    gr = O.grad_adjoint(c["G"], c["M"], wl.geom.R, c["Phi"], wl.C, wl.omega, wl.target, mode)
    el = np.abs(loss.cpu().numpy() - Lr) / np.abs(Lr)
    eg = _nrel(grad.cpu().numpy(), gr, axis=1)
    _say(f"[gemm] {name} prec={prec} mode={mode}: loss {el.max():.2e} grad {eg.max():.2e}")
    assert el.max() < TOL[prec] and eg.max() < TOL[prec]
    # loss only: the same loss
    l2, _, _ = c["plan"].loss_and_grad(c["C"], c["om"], c["T"], loss_mode=mode, precision=prec,
                                       grad=False)
    torch.cuda.synchronize()
    assert torch.equal(l2, loss)
