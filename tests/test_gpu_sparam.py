"""GPU parity of the S-parameter pipeline (cosim_sp_*) against its FP64 oracle.

Every case compares the HIP path element by element with oracle/sparam_oracle
on the same seeded inputs: incident waves x, the combined field of every
component, the loss and the gradient with respect to every variable entry,
in FP64 (1e-9) and with FP32 contractions (1e-5); the RC preprocessing and its
chain rule; the quasi-static exports of the impedance model; a singular
system's status bits.
"""
import numpy as np
import pytest

import oracle as O
from oracle import sparam_oracle as SO
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {0: 1e-9, 1: 1e-5}


def _say(msg):
    print(msg, flush=True)


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


def _general(seed, B, F, n0, n1, P, ncomp, diag_only=False):
    """A general network: a non-reciprocal S0 of norm 0.8, random port fields,
    constant entries everywhere (also off the S_C11 diagonal), variable entries
    on and off the S_C11 diagonal, in S_C12 and in S_C21 / S_C22, one index pair
    repeated."""
    rng = np.random.default_rng(seed)
    N = n0 + n1
    S0 = rng.normal(size=(F, n0, n0)) + 1j * rng.normal(size=(F, n0, n0))
    S0 *= 0.8 / np.linalg.norm(S0, 2, axis=(1, 2))[:, None, None]
    fields = rng.normal(size=(F, P, ncomp, n0)) + 1j * rng.normal(size=(F, P, ncomp, n0))
    scc = 0.05 * (rng.normal(size=(F, N, N)) + 1j * rng.normal(size=(F, N, N)))
    ix, iy = list(range(n0)), list(range(n0))            # RC-like loads on the diagonal
    if not diag_only:
        ix += [0, n0 - 1, min(1, n0 - 1), n0, N - 1, 0]
        iy += [n0, n0 + n1 - 1, 0, 0, N - 1, n0]             # S_C12, S_C11 off-diagonal, S_C21, S_C22, repeat
    ix, iy = np.array(ix, np.int32), np.array(iy, np.int32)
    vals = 0.6 * np.exp(1j * rng.uniform(0, 2 * np.pi, (B, F, len(ix))))
    exc = (rng.normal(size=n1) + 1j * rng.normal(size=n1)) * np.sqrt(50.0)
    T = np.abs(rng.normal(size=P))
    return S0, fields, scc, ix, iy, vals, exc, T


def _plan(dev, S0, fields, scc, ix, iy, exc, prec=("fp64", "fp32")):
    from paper_2503_18479_amd import SParamPlan
    t = lambda a: torch.tensor(a, dtype=torch.complex128, device=dev)
    return SParamPlan(t(S0), t(fields), ix, iy, exc, sc_const=None if scc is None else t(scc),
                      precisions=prec)


CASES = {
    "n1": dict(seed=1, B=3, F=1, n0=1, n1=1, P=5, ncomp=1),
    "n5": dict(seed=2, B=2, F=2, n0=5, n1=2, P=37, ncomp=3),
    "n37": dict(seed=3, B=4, F=3, n0=37, n1=1, P=300, ncomp=3),
    "n64": dict(seed=4, B=3, F=2, n0=64, n1=2, P=2100, ncomp=1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_field_matches_oracle(dev, name):
    c = CASES[name]
    S0, fields, scc, ix, iy, vals, exc, T = _general(**c)
    _say(f"[sp] field {name}")
    pl = _plan(dev, S0, fields, scc, ix, iy, exc)
    x, Bc, st = pl.field(torch.tensor(vals, device=dev))
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    SC = SO.assemble_network(scc, vals, ix, iy)
    xr, Br = SO.combine(S0, fields, SC, c["n0"], exc)
    assert _nrel(x.cpu().numpy(), xr) < 1e-12
    assert _nrel(Bc.cpu().numpy(), Br) < 1e-12


@pytest.mark.parametrize("mode", [SO.LOSS_MAG, SO.LOSS_COMPLEX])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_loss_and_grad_matches_oracle(dev, name, prec, mode):
    c = CASES[name]
    S0, fields, scc, ix, iy, vals, exc, T = _general(**c)
    comp = c["ncomp"] - 1
    _say(f"[sp] loss/grad {name} prec={prec} mode={mode}")
    pl = _plan(dev, S0, fields, scc, ix, iy, exc)
    loss, g, st = pl.loss_and_grad(torch.tensor(vals, device=dev), torch.tensor(T, device=dev), comp,
                                   mode, prec)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    SC = SO.assemble_network(scc, vals, ix, iy)
    Lr = SO.loss(SO.combine(S0, fields, SC, c["n0"], exc)[1], T, comp, mode)
    gr = SO.grad_adjoint(S0, fields, SC, c["n0"], exc, ix, iy, T, comp, mode)
    el = np.max(np.abs(loss.cpu().numpy() - Lr) / Lr)
    eg = _nrel(g.cpu().numpy(), gr)
    _say(f"[sp] {name} prec={prec} mode={mode}: loss {el:.2e} grad {eg:.2e}")
    assert el < TOL[prec] and eg < TOL[prec]
    gd = g.cpu().numpy()
    assert np.all(gd[..., ix >= c["n0"]] == 0)   # S_C21 / S_C22 entries
    # loss only
    l2, g2, _ = pl.loss_and_grad(torch.tensor(vals, device=dev), torch.tensor(T, device=dev), comp,
                                 mode, prec, grad=False)
    assert g2 is None
    assert np.allclose(l2.cpu().numpy(), loss.cpu().numpy(), rtol=1e-14, atol=0)


def test_quasi_static_exports_reproduce_the_impedance_route(dev):
    """Fed with S0 = (jwM - Z0)(jwM + Z0)^-1 and the fields G (I - S0)/Z0 of the
    loop array, RC reflections on the S_C11 diagonal (cosim_sp_rc) and the EMF
    injection in S_C12, the GPU pipeline gives the impedance route's B_z and
    loss; the chain rule through cosim_sp_rc_backward and the injection gives its
    dL/dC."""
    from paper_2503_18479_amd import sp_rc, sp_rc_backward
    Z0 = 50.0
    wl = W.small_array(3, 3, 2, 6, n_freq=2, seed=5)
    g = wl.geom
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    n, F, P, B = M.shape[0], len(wl.omega), wl.P, wl.C.shape[0]
    S0 = np.zeros((F, n, n), complex)
    fields = np.zeros((F, P, 1, n), complex)
    for f, w in enumerate(wl.omega):
        Zs = 1j * w * M
        S0[f] = (Zs - Z0 * np.eye(n)) @ np.linalg.inv(Zs + Z0 * np.eye(n))
        fields[f, :, 0, :] = G @ (np.eye(n) - S0[f]) / Z0
    ix = np.concatenate([np.arange(n), np.arange(n)]).astype(np.int32)
    iy = np.concatenate([np.arange(n), np.full(n, n)]).astype(np.int32)
    pl = _plan(dev, S0, fields, None, ix, iy, np.array([1.0 + 0j]))
    Cd = torch.tensor(wl.C, device=dev)
    om = torch.tensor(wl.omega, device=dev)
    Rd = torch.tensor(g.R, device=dev)
    vals = torch.empty((B, F, 2 * n), dtype=torch.complex128, device=dev)
    sp_rc(Rd, Cd, om, Z0, out=vals)               # Gamma into the first n columns
    ZL = g.R[None, None, :] - 1j / (wl.omega[None, :, None] * wl.C[:, None, :])
    E = -1j * wl.omega[None, :, None] * Phi[None, None, :]
    q = Z0 * E / (ZL + Z0)
    vals[..., n:] = torch.tensor(q, device=dev)
    gam_r = SO.rc_reflection(g.R, wl.C, wl.omega, Z0)
    assert _nrel(vals[..., :n].cpu().numpy(), gam_r) < 1e-14
    T = torch.tensor(wl.target, device=dev)
    _, Bc, st = pl.field(vals)
    loss, gv, st2 = pl.loss_and_grad(vals, T, 0, 0, 0)
    gC_gam = sp_rc_backward(Rd, Cd, om, gv, Z0)    # the first n columns of the gradient
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0 and int(st2.abs().sum()) == 0
    I = O.currents(M, g.R, Phi, wl.C, wl.omega)
    Bz = O.field(G, I)
    assert _nrel(Bc.cpu().numpy()[..., 0], Bz) < 1e-10
    Lz = O.loss(Bz, wl.target)
    assert np.max(np.abs(loss.cpu().numpy() - Lz) / Lz) < 1e-9
    # chain rule: the RC reflections through the library, the injection here
    gq = gv.cpu().numpy()[..., n:]
    dq = -Z0 * E / (ZL + Z0) ** 2 * (1j / (wl.omega[None, :, None] * wl.C[:, None, :] ** 2))
    gC = gC_gam.cpu().numpy() + np.real(np.conj(gq) * dq).sum(axis=1)
    gz = O.grad_adjoint(G, M, g.R, Phi, wl.C, wl.omega, wl.target)
    assert _nrel(gC, gz) < 1e-8
    gr = SO.rc_grad_C(gv.cpu().numpy()[..., :n], g.R, wl.C, wl.omega, Z0)
    assert _nrel(gC_gam.cpu().numpy(), gr) < 1e-12


def test_singular_system_is_flagged_alone(dev):
    """S0 = I and S_C11 = I make A = I - S_C11 S0 = 0 for one configuration:
    that system is flagged singular with NaN outputs, the others are not."""
    n0, F, P = 3, 1, 8
    S0 = np.eye(n0)[None].astype(complex)
    rng = np.random.default_rng(7)
    fields = rng.normal(size=(F, P, 1, n0)) + 0j
    ix = np.arange(n0, dtype=np.int32)
    iy = np.arange(n0, dtype=np.int32)
    scc = np.zeros((F, n0 + 1, n0 + 1), complex)
    scc[:, :n0, n0] = 0.5
    vals = np.full((2, F, n0), 0.3 + 0j)
    vals[1] = 1.0
    pl = _plan(dev, S0, fields, scc, ix, iy, np.array([1.0 + 0j]))
    x, Bc, st = pl.field(torch.tensor(vals, device=dev))
    loss, g, st2 = pl.loss_and_grad(torch.tensor(vals, device=dev), torch.ones(P, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[0, 0] == 0 and (st[1, 0] & 2)
    assert np.all(np.isfinite(x.cpu().numpy()[0])) and np.all(np.isnan(x.cpu().numpy()[1]))
    assert np.isfinite(loss[0].item()) and np.isnan(loss[1].item())
    SC = SO.assemble_network(scc, vals[:1], ix, iy)
    xr, _ = SO.combine(S0, fields, SC, n0, np.array([1.0]))
    assert _nrel(x.cpu().numpy()[:1], xr) < 1e-12


def test_empty_batch_and_reuse(dev):
    S0, fields, scc, ix, iy, vals, exc, T = _general(seed=9, B=5, F=2, n0=6, n1=1, P=40, ncomp=2)
    pl = _plan(dev, S0, fields, scc, ix, iy, exc)
    z = torch.empty((0, 2, len(ix)), dtype=torch.complex128, device=dev)
    x, Bc, st = pl.field(z)
    assert x.shape[0] == 0
    # a large call, then a smaller one on the same workspace
    Tt = torch.tensor(T, device=dev)
    l5, g5, _ = pl.loss_and_grad(torch.tensor(vals, device=dev), Tt, 1, 0, 0)
    l2, g2, _ = pl.loss_and_grad(torch.tensor(vals[:2], device=dev), Tt, 1, 0, 0)
    torch.cuda.synchronize()
    # the GEMMs may take other kernels at another batch size: equal to rounding
    assert np.allclose(l5[:2].cpu().numpy(), l2.cpu().numpy(), rtol=1e-13, atol=0)
    assert _nrel(g5[:2].cpu().numpy(), g2.cpu().numpy()) < 1e-12


def test_full_size_8x8_shape_sampled(dev):
    """The launch configuration of the benchmark (64 ports, 65,536 points, 21
    frequencies, 4,096 configurations: 86,016 systems, several P-chunks):
    seeded random exports, RC reflections of the 8x8 workload's capacitances as
    the variable S_C11 diagonal; loss and gradient of sampled configurations
    against the oracle in FP64 and FP32."""
    from paper_2503_18479_amd import sp_rc
    wl = W.config3_array8x8(batch=4096)
    n0, F, P = 64, wl.F, wl.P
    rng = np.random.default_rng(11)
    S0 = rng.normal(size=(F, n0, n0)) + 1j * rng.normal(size=(F, n0, n0))
    S0 *= 0.8 / np.linalg.norm(S0, 2, axis=(1, 2))[:, None, None]
    _say("[sp] full-size exports")
    fields = (rng.standard_normal((F, P, 1, n0), dtype=np.float32)
              + 1j * rng.standard_normal((F, P, 1, n0), dtype=np.float32)).astype(np.complex128)
    scc = np.zeros((F, n0 + 1, n0 + 1), complex)
    scc[:, :n0, n0] = 0.1
    ix = np.arange(n0, dtype=np.int32)
    pl = _plan(dev, S0, fields, scc, ix, ix, np.array([np.sqrt(50.0) + 0j]))
    R = np.full(n0, 0.3)
    vals = torch.empty((wl.B, F, n0), dtype=torch.complex128, device=dev)
    sp_rc(torch.tensor(R, device=dev), torch.tensor(wl.C, device=dev), torch.tensor(wl.omega, device=dev),
          50.0, out=vals)
    T = np.abs(rng.normal(size=P)) * 0.05
    Tt = torch.tensor(T, device=dev)
    sel = [0, 1777, 4095]
    gam = SO.rc_reflection(R, wl.C[sel], wl.omega)
    SC = SO.assemble_network(scc, gam, ix, ix)
    Lr = SO.loss(SO.combine(S0, fields, SC, n0, np.array([np.sqrt(50.0)]))[1], T)
    gr = SO.grad_adjoint(S0, fields, SC, n0, np.array([np.sqrt(50.0)]), ix, ix, T)
    for prec in (0, 1):
        _say(f"[sp] full size prec={prec}")
        loss, g, st = pl.loss_and_grad(vals, Tt, 0, 0, prec)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        el = np.max(np.abs(loss.cpu().numpy()[sel] - Lr) / Lr)
        eg = _nrel(g.cpu().numpy()[sel], gr)
        _say(f"[sp] full size prec={prec}: loss {el:.2e} grad {eg:.2e}")
        assert el < TOL[prec] and eg < TOL[prec]
