"""Pins of the S-parameter pipeline oracle (CPU only).

The general pipeline (user-supplied S0 and port fields, S_C = S_C,const +
S_C,var, Eq. 6-7, the gradient of Eq. 8-10) is tied to the impedance route,
which tests/test_oracle_pins.py pins against closed forms and quadrature: fed
with the exports of the quasi-static model it must reproduce that route's
B_z, loss and dL/dC.  Its gradient is further checked by forward sensitivity,
central differences and closed forms.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle as O  # noqa: E402
from oracle import sparam_oracle as SO  # noqa: E402
import workloads as W  # noqa: E402

Z0 = 50.0


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _quasi_static(nx=3, ny=2, B=3, F=2, P=40, seed=0):
    """The impedance-route problem and its S-parameter exports: S0 of the
    structure j w M, the field per unit incident wave of port k with the other
    ports matched, G (I - S0) e_k / Z0, and the per-loop preprocessing output
    (Gamma_k of the RC load at S_C[k][k], the injected wave
    q_k = Z0 E_k / (Z_L,k + Z0) of the EMF E = -j w Phi at S_C[k][n0])."""
    wl = W.small_array(nx, ny, B, 8, n_freq=F, seed=seed)
    rng = np.random.default_rng(seed)
    pts = W.random_points(rng, P, 0.12, 0.005, 0.03)
    g = wl.geom
    G = O.field_matrix(g.verts, g.seg_off, pts)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    T = rng.uniform(0, 2e-7, P)
    n = M.shape[0]
    S0 = np.zeros((F, n, n), complex)
    fields = np.zeros((F, P, 1, n), complex)
    for f, w in enumerate(wl.omega):
        Zs = 1j * w * M
        S0[f] = (Zs - Z0 * np.eye(n)) @ np.linalg.inv(Zs + Z0 * np.eye(n))
        fields[f, :, 0, :] = G @ (np.eye(n) - S0[f]) / Z0
    gam = SO.rc_reflection(g.R, wl.C, wl.omega, Z0)                    # [B][F][n]
    ZL = g.R[None, None, :] - 1j / (wl.omega[None, :, None] * wl.C[:, None, :])
    E = -1j * wl.omega[None, :, None] * Phi[None, None, :]
    q = Z0 * E / (ZL + Z0)
    values = np.concatenate([gam, q], axis=2)                           # [B][F][2n]
    idx_x = np.concatenate([np.arange(n), np.arange(n)])
    idx_y = np.concatenate([np.arange(n), np.full(n, n)])
    sc_const = np.zeros((F, n + 1, n + 1), complex)
    return dict(G=G, M=M, R=g.R, Phi=Phi, C=wl.C, om=wl.omega, T=T, S0=S0, fields=fields,
                values=values, idx_x=idx_x, idx_y=idx_y, sc_const=sc_const, n=n, ZL=ZL, E=E)


@pytest.mark.parametrize("mode", [SO.LOSS_MAG, SO.LOSS_COMPLEX])
def test_pipeline_reproduces_the_impedance_route(mode):
    d = _quasi_static()
    n = d["n"]
    SC = SO.assemble_network(d["sc_const"], d["values"], d["idx_x"], d["idx_y"])
    x, Bc = SO.combine(d["S0"], d["fields"], SC, n, np.array([1.0]))
    I = O.currents(d["M"], d["R"], d["Phi"], d["C"], d["om"])
    Bz = O.field(d["G"], I)
    assert _rel(Bc[..., 0], Bz) < 1e-12
    # the incident waves are those of the oracle's own wave formulation
    S0 = d["S0"]
    Iw = np.einsum("fkl,bfl->bfk", np.eye(n)[None] - S0, x) / Z0
    assert _rel(Iw, I) < 1e-12
    L = SO.loss(Bc, d["T"], 0, mode)
    Lz = O.loss(Bz, d["T"], mode)
    assert np.max(np.abs(L - Lz) / Lz) < 1e-12
    # dL/dC through the pipeline's gradient and the chain rule of Eq. 2-3
    g = SO.grad_adjoint(d["S0"], d["fields"], SC, n, np.array([1.0]), d["idx_x"], d["idx_y"],
                        d["T"], 0, mode)
    dgam = SO.rc_reflection_dC(d["R"], d["C"], d["om"], Z0)
    w = d["om"][None, :, None]
    dq = -Z0 * d["E"] / (d["ZL"] + Z0) ** 2 * (1j / (w * d["C"][:, None, :] ** 2))
    gC = np.real(np.conj(g[..., :n]) * dgam + np.conj(g[..., n:]) * dq).sum(axis=1)
    gz = O.grad_adjoint(d["G"], d["M"], d["R"], d["Phi"], d["C"], d["om"], d["T"], mode)
    assert _rel(gC, gz) < 1e-10


def test_single_port_closed_form():
    rng = np.random.default_rng(1)
    F, P = 3, 5
    s0 = 0.9 * np.exp(1j * rng.uniform(0, 2 * np.pi, F))
    fields = rng.normal(size=(F, P, 3, 1)) + 1j * rng.normal(size=(F, P, 3, 1))
    vals = np.stack([0.7 * np.exp(1j * rng.uniform(0, 6, (2, F))),
                     0.5 * np.exp(1j * rng.uniform(0, 6, (2, F)))], axis=2)   # s11, s12
    SC = SO.assemble_network(np.zeros((F, 2, 2)), vals, [0, 0], [0, 1])
    exc = np.array([np.sqrt(50.0)])
    x, Bc = SO.combine(s0[:, None, None], fields, SC, 1, exc)
    xr = vals[..., 1] * exc[0] / (1.0 - vals[..., 0] * s0[None, :])
    np.testing.assert_allclose(x[..., 0], xr, rtol=1e-14)
    np.testing.assert_allclose(Bc, fields[None, :, :, :, 0] * xr[:, :, None, None], rtol=1e-13)


def _general(seed=2, B=2, F=2, n0=5, n1=2, P=7, ncomp=3):
    """A general network: non-reciprocal S0 of norm below 1, three field
    components, constant entries everywhere, variable entries on and off the
    S_C11 diagonal, in S_C12 and in S_C21 / S_C22 (which Eq. 6-7 never read)."""
    rng = np.random.default_rng(seed)
    N = n0 + n1
    S0 = rng.normal(size=(F, n0, n0)) + 1j * rng.normal(size=(F, n0, n0))
    S0 *= 0.6 / np.linalg.norm(S0, 2, axis=(1, 2))[:, None, None]
    fields = rng.normal(size=(F, P, ncomp, n0)) + 1j * rng.normal(size=(F, P, ncomp, n0))
    sc_const = 0.1 * (rng.normal(size=(F, N, N)) + 1j * rng.normal(size=(F, N, N)))
    idx_x = np.array([0, 1, 2, 3, 0, 4, 1, 5, 6, 2])
    idx_y = np.array([0, 1, 4, 1, 5, 6, 0, 0, 6, 4])   # (2, 4) twice: values add
    values = 0.3 * (rng.normal(size=(B, F, len(idx_x))) + 1j * rng.normal(size=(B, F, len(idx_x))))
    exc = np.array([1.2 - 0.4j, 0.3 + 0.9j])[:n1]
    T = rng.uniform(0, 1.5, P)
    return S0, fields, sc_const, values, idx_x, idx_y, n0, exc, T


@pytest.mark.parametrize("mode", [SO.LOSS_MAG, SO.LOSS_COMPLEX])
@pytest.mark.parametrize("comp", [0, 2])
def test_gradient_adjoint_sensitivity_fd(mode, comp):
    S0, fields, scc, vals, ix, iy, n0, exc, T = _general()
    SC = SO.assemble_network(scc, vals, ix, iy)
    ga = SO.grad_adjoint(S0, fields, SC, n0, exc, ix, iy, T, comp, mode)
    gs = SO.grad_forward_sensitivity(S0, fields, SC, n0, exc, ix, iy, T, comp, mode)
    assert _rel(ga, gs) < 1e-12
    gd = SO.grad_fd(S0, fields, scc, vals, ix, iy, n0, exc, T, comp, mode, h=1e-6)
    assert _rel(ga, gd) < 1e-6
    # entries in S_C21 / S_C22 have no effect on Eq. 6-7
    assert np.all(ga[..., ix >= n0] == 0)


def test_linear_in_the_drive():
    S0, fields, scc, vals, ix, iy, n0, exc, T = _general()
    SC = SO.assemble_network(scc, vals, ix, iy)
    _, B1 = SO.combine(S0, fields, SC, n0, exc)
    _, B2 = SO.combine(S0, fields, SC, n0, (2.0 - 1.0j) * exc)
    np.testing.assert_allclose(B2, (2.0 - 1.0j) * B1, rtol=1e-12, atol=1e-14)
    # superposition over the external ports
    _, Ba = SO.combine(S0, fields, SC, n0, np.array([exc[0], 0.0]))
    _, Bb = SO.combine(S0, fields, SC, n0, np.array([0.0, exc[1]]))
    np.testing.assert_allclose(Ba + Bb, B1, rtol=1e-12, atol=1e-14)


def test_rc_chain_rule_against_differences():
    rng = np.random.default_rng(4)
    n, F, B = 4, 2, 2
    S0 = 0.5 * (rng.normal(size=(F, n, n)) + 1j * rng.normal(size=(F, n, n))) / n
    fields = rng.normal(size=(F, 6, 1, n)) + 1j * rng.normal(size=(F, 6, 1, n))
    R = np.full(n, 0.3)
    C = rng.uniform(20e-12, 150e-12, (B, n))
    om = 2 * np.pi * np.array([120e6, 130e6])
    T = rng.uniform(0, 1, 6)
    scc = np.zeros((F, n + 1, n + 1), complex)
    scc[:, :n, n] = 0.4
    ix, iy = np.arange(n), np.arange(n)

    def L(Cv):
        SC = SO.assemble_network(scc, SO.rc_reflection(R, Cv, om), ix, iy)
        return SO.loss(SO.combine(S0, fields, SC, n, np.array([1.0]))[1], T)

    SC = SO.assemble_network(scc, SO.rc_reflection(R, C, om), ix, iy)
    g = SO.grad_adjoint(S0, fields, SC, n, np.array([1.0]), ix, iy, T)
    gC = SO.rc_grad_C(g, R, C, om)
    h = 1e-16
    for k in range(n):
        Cp, Cm = C.copy(), C.copy()
        Cp[:, k] += h
        Cm[:, k] -= h
        fd = (L(Cp) - L(Cm)) / (2 * h)
        np.testing.assert_allclose(gC[:, k], fd, rtol=1e-5)


def test_reflection_of_rc_loads():
    C = np.array([[1e-12, 50e-12, 1e-9]])
    om = np.array([2 * np.pi * 128e6])
    gam = SO.rc_reflection(np.full(3, 0.3), C, om)
    assert np.all(np.abs(gam) < 1.0)                     # lossy load: passive
    gam0 = SO.rc_reflection(np.zeros(3), C, om)
    np.testing.assert_allclose(np.abs(gam0), 1.0, rtol=1e-14)   # pure reactance
