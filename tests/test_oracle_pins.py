"""Pins of the FP64 oracle against closed forms, brute-force quadrature,
invariants and the paper's own S-parameter equations (Eq. 3-7).

Each test checks the oracle against something other than itself, so that a
dropped term, a wrong sign or index, or a transposed operand fails here.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ---------------------------------------------------------------- geometry

def test_vector_area_square_and_polygon():
    g = W.square_array(2, 2, 0.03, 0.035, 32)
    np.testing.assert_allclose(O.vector_area_z(g.verts, g.seg_off), 0.03 ** 2, rtol=1e-14)
    c = W.single_circle(0.05, 64)
    exact = 0.5 * 64 * 0.05 ** 2 * math.sin(2 * math.pi / 64)
    np.testing.assert_allclose(O.vector_area_z(c.verts, c.seg_off), exact, rtol=1e-14)
    # clockwise loop has negative area
    v = c.verts[::-1].copy()
    assert O.vector_area_z(v, c.seg_off)[0] < 0


# ---------------------------------------------------------------- G (T1-T3)

def test_T1_segment_closed_form_vs_quadrature():
    rng = np.random.default_rng(1)
    for _ in range(20):
        x1 = rng.uniform(-0.02, 0.02, 3); x2 = rng.uniform(-0.02, 0.02, 3)
        p = rng.uniform(-0.05, 0.05, (16, 3)); p[:, 2] += 0.03 * np.sign(p[:, 2] + 1e-9)
        cf = O.bz_segment(p, x1, x2)
        q = O.bz_segment_quadrature(p, x1, x2, order=48, panels=16)
        np.testing.assert_allclose(cf, q, rtol=1e-10, atol=1e-12 * np.abs(q).max())


def test_T1_sign_right_hand_rule():
    # current along +x at y=0; a point at y=-1 lies below: B_z < 0 there
    bz = O.bz_segment(np.array([0.0, -1.0, 0.0]), np.array([-1.0, 0, 0]), np.array([1.0, 0, 0]))
    assert bz < 0
    # infinite-wire limit mu0 I / (2 pi d)
    bz = O.bz_segment(np.array([0.0, 0.1, 0.0]), np.array([-1e4, 0, 0]), np.array([1e4, 0, 0]))
    np.testing.assert_allclose(bz, O.MU0 / (2 * math.pi * 0.1), rtol=1e-9)


@pytest.mark.parametrize("N", [3, 4, 7, 64])
@pytest.mark.parametrize("z", [0.0, 0.013, -0.04])
def test_T2_polygon_on_axis(N, z):
    g = W._pack([W.regular_polygon(0.05, N)], 1e-3, 0.5, 1, 1, 0.0)
    G = O.field_matrix(g.verts, g.seg_off, np.array([[0.0, 0.0, z]]))
    np.testing.assert_allclose(G[0, 0], O.polygon_axis_bz(N, 0.05, z), rtol=1e-13)


def test_T2_circle_limit():
    # O(1/N^2) approach to mu0 R^2 / (2 (R^2+z^2)^1.5)
    errs = []
    for N in (64, 128, 256):
        g = W._pack([W.regular_polygon(0.05, N)], 1e-3, 0.5, 1, 1, 0.0)
        G = O.field_matrix(g.verts, g.seg_off, np.array([[0.0, 0.0, 0.02]]))
        errs.append(abs(G[0, 0] / O.circle_axis_bz(0.05, 0.02) - 1))
    assert errs[0] < 6e-4
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_T3_square_on_axis_subdivided():
    s = 0.03
    for nseg in (4, 32):
        g = W.square_array(1, 1, s, 0.0, nseg)
        for z in (0.0, 0.01, 0.03):
            G = O.field_matrix(g.verts, g.seg_off, np.array([[0.0, 0.0, z]]))
            h = s / 2
            ref = 2 * O.MU0 * h * h / (math.pi * (h * h + z * z) * math.sqrt(2 * h * h + z * z))
            np.testing.assert_allclose(G[0, 0], ref, rtol=1e-13)


def test_G_translation_and_superposition():
    # a 2x1 array: loop 1's column equals loop 0's column at shifted points
    g = W.square_array(2, 1, 0.03, 0.035, 32)
    rng = np.random.default_rng(2)
    p = W.random_points(rng, 64, 0.2, 0.005, 0.04)
    G = O.field_matrix(g.verts, g.seg_off, p)
    shift = np.array([0.035, 0.0, 0.0])
    G0s = O.field_matrix(g.verts, g.seg_off, p - shift)
    np.testing.assert_allclose(G[:, 1], G0s[:, 0], rtol=1e-12, atol=1e-18)


# ---------------------------------------------------------------- M (T4-T7)

def _brute_neumann(x1, x2, y1, y2, a, order=40, panels=24):
    """2-D composite Gauss-Legendre of dl.dl'/sqrt(|r-r'|^2+a^2)."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    t = ((np.arange(panels)[:, None] + 0.5 * (xg[None, :] + 1)) / panels).ravel()
    w = np.tile(0.5 * wg / panels, panels)
    P = x1[None, :] + t[:, None] * (x2 - x1)[None, :]
    Q = y1[None, :] + t[:, None] * (y2 - y1)[None, :]
    d = P[:, None, :] - Q[None, :, :]
    ker = 1.0 / np.sqrt(np.sum(d * d, axis=-1) + a * a)
    return O.MU0_4PI * float(np.dot(x2 - x1, y2 - y1)) * float(w @ ker @ w)


def test_T4_parallel_and_general_pairs_vs_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(12):
        # parallel filaments with an offset, both orientations
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        x1 = rng.uniform(-0.01, 0.01, 3); x2 = x1 + 0.02 * u
        off = rng.normal(size=3); off -= off.dot(u) * u; off *= 0.01 / np.linalg.norm(off)
        y1 = x1 + off + rng.uniform(-0.01, 0.01) * u
        y2 = y1 + rng.choice([-1, 1]) * rng.uniform(0.005, 0.03) * u
        np.testing.assert_allclose(O.neumann_segments(x1, x2, y1, y2),
                                   _brute_neumann(x1, x2, y1, y2, 0.0), rtol=1e-10)
        # arbitrary angle, separated
        y1 = rng.uniform(-0.01, 0.01, 3) + np.array([0, 0, 0.015])
        y2 = y1 + rng.uniform(-0.02, 0.02, 3)
        np.testing.assert_allclose(O.neumann_segments(x1, x2, y1, y2),
                                   _brute_neumann(x1, x2, y1, y2, 0.0), rtol=1e-10)
        # arbitrary angle with the reduced kernel, sharing a vertex
        y1 = x2.copy(); y2 = x2 + 0.01 * rng.normal(size=3)
        np.testing.assert_allclose(O.neumann_segments(x1, x2, y1, y2, 2e-3),
                                   _brute_neumann(x1, x2, y1, y2, 2e-3, panels=64), rtol=1e-9)


def test_T4_perpendicular_is_zero_and_collinear_limit():
    z = O.neumann_segments([0, 0, 0], [1, 0, 0], [0.5, 0.2, 0], [0.5, 0.9, 0])
    assert z == 0.0
    # collinear, separated: the d->0 limit equals the brute-force integral
    x1, x2 = np.zeros(3), np.array([0.01, 0, 0])
    y1, y2 = np.array([0.015, 0, 0]), np.array([0.04, 0, 0])
    np.testing.assert_allclose(O.neumann_segments(x1, x2, y1, y2),
                               _brute_neumann(x1, x2, y1, y2, 0.0, panels=48), rtol=1e-10)
    # ... and the nearly-collinear formula approaches it
    y1b, y2b = y1 + [0, 1e-7, 0], y2 + [0, 1e-7, 0]
    np.testing.assert_allclose(O.neumann_segments(x1, x2, y1b, y2b),
                               O.neumann_segments(x1, x2, y1, y2), rtol=1e-8)


def test_T5_square_self_inductance_brute_force():
    s, a = 0.03, 1e-3
    g = W.square_array(1, 1, s, 0.0, 32)
    L = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)[0, 0]
    # brute force: 2-D quadrature of the reduced kernel around the whole loop
    xg, wg = np.polynomial.legendre.leggauss(16)
    panels = 96
    t = ((np.arange(panels)[:, None] + 0.5 * (xg[None, :] + 1)) / panels).ravel()
    w = np.tile(0.5 * wg / panels, panels) * s
    h = s / 2
    sides = [(np.array([-h, -h]), np.array([1.0, 0])), (np.array([h, -h]), np.array([0, 1.0])),
             (np.array([h, h]), np.array([-1.0, 0])), (np.array([-h, h]), np.array([0, -1.0]))]
    pts = np.concatenate([o[None, :] + s * t[:, None] * d[None, :] for o, d in sides])
    dirs = np.concatenate([np.repeat(d[None, :], t.size, 0) for _, d in sides])
    ww = np.tile(w, 4)
    diff = pts[:, None, :] - pts[None, :, :]
    ker = (dirs @ dirs.T) / np.sqrt(np.sum(diff * diff, -1) + a * a)
    brute = O.MU0_4PI * float(ww @ ker @ ww)
    np.testing.assert_allclose(L, brute, rtol=2e-9)
    with open(os.path.join(GOLDEN, "inductance.json")) as f:
        gold = json.load(f)
    np.testing.assert_allclose(L, gold["square_3cm_a1mm_self_H"], rtol=1e-12)


def test_T6_polygon_self_inductance_tends_to_maxwell_circle():
    R, a = 0.05, 1e-3
    ref = O.coaxial_circles_mutual(R, R, a)
    errs = []
    for N in (32, 64, 128):
        v = W.regular_polygon(R, N)
        b = np.roll(v, -1, 0)
        # rotational symmetry: every segment sees the same row sum
        L = N * sum(O.neumann_segments(v[0], b[0], v[t], b[t], a) for t in range(N))
        errs.append(abs(L / ref - 1))
    assert errs[1] < 1.2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    # the full matrix routine agrees with the symmetric row sum
    g = W.single_circle(R, 64, a)
    M = O.inductance_matrix(g.verts, g.seg_off, g.wire_a)
    v = W.regular_polygon(R, 64); b = np.roll(v, -1, 0)
    Lrow = 64 * sum(O.neumann_segments(v[0], b[0], v[t], b[t], a) for t in range(64))
    np.testing.assert_allclose(M[0, 0], Lrow, rtol=1e-11)
    # thin-wire asymptote mu0 R (ln(8R/a) - 2)
    np.testing.assert_allclose(ref, O.MU0 * R * (math.log(8 * R / a) - 2), rtol=2e-3)


def test_T7_reciprocity_and_flux_form():
    g = W.square_array(3, 2, 0.03, 0.035, 32)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    np.testing.assert_allclose(M, M.T, rtol=1e-12, atol=0)
    Ms = O.inductance_matrix(g.verts, g.seg_off, g.wire_a)
    np.testing.assert_allclose(M, Ms, rtol=1e-12)
    # flux of loop l's Biot-Savart field through the square of loop k (k != l)
    xg, wg = np.polynomial.legendre.leggauss(20)
    panels = 6
    t = ((np.arange(panels)[:, None] + 0.5 * (xg[None, :] + 1)) / panels).ravel() - 0.5
    w = np.tile(0.5 * wg / panels, panels) * 0.03
    for k, l in [(0, 1), (0, 4), (2, 3), (5, 0)]:
        c = g.loop(k)[:, :2].mean(axis=0)
        X, Y = np.meshgrid(c[0] + 0.03 * t, c[1] + 0.03 * t, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
        G = O.field_matrix(g.verts, g.seg_off, pts)
        flux = float(np.outer(w, w).ravel() @ G[:, l])
        np.testing.assert_allclose(flux, M[k, l], rtol=1e-7)
    # coplanar neighbours couple negatively
    assert M[0, 1] < 0


# ---------------------------------------------------------------- circuit (T8, T9)

def _small_problem(nx=3, ny=2, B=3, F=2, P=50, seed=0):
    wl = W.small_array(nx, ny, B, 8, n_freq=F, seed=seed)
    rng = np.random.default_rng(seed)
    pts = W.random_points(rng, P, 0.12, 0.005, 0.03)
    g = wl.geom
    G = O.field_matrix(g.verts, g.seg_off, pts)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    T = rng.uniform(0, 2e-7, P)
    return G, M, g.R, Phi, wl.C, wl.omega, T


def test_T8_single_loop_resonance():
    g = W.single_circle()
    M = O.inductance_matrix(g.verts, g.seg_off, g.wire_a)
    L = M[0, 0]
    w = 2 * math.pi * 128e6
    Cr = 1.0 / (w * w * L)
    Z = O.impedance(M, g.R, np.array([Cr]), w)
    assert abs(Z[0, 0].imag) < 1e-12 * abs(w * L)
    Phi = O.flux(g.verts, g.seg_off, 1e-6)
    I = O.currents(M, g.R, Phi, np.array([[Cr]]), np.array([w]))[0, 0, 0]
    np.testing.assert_allclose(I, -1j * w * Phi[0] / g.R[0], rtol=1e-12)
    # phase of I sweeps through pi across the resonance
    Cs = Cr * np.array([0.5, 0.9, 1.1, 2.0])
    Is = O.currents(M, g.R, Phi, Cs[:, None], np.array([w]))[:, 0, 0]
    ph = np.unwrap(np.angle(Is))
    assert abs(abs(ph[-1] - ph[0]) - math.pi) < 0.2
    # Lenz: with a large capacitance the loop current opposes the applied flux
    Ib = O.currents(M, g.R, Phi, np.array([[1e-6]]), np.array([w]))[0, 0, 0]
    assert Ib.real < 0


def test_T9_sparameter_route_equals_impedance_solve():
    G, M, R, Phi, C, om, T = _small_problem()
    Iz = O.currents(M, R, Phi, C, om)
    Is = O.sform_currents(M, R, Phi, C, om)
    assert _rel(Is, Iz) < 1e-12
    # and through Eq. 7 the fields agree
    assert _rel(O.field(G, Is), O.field(G, Iz)) < 1e-12


# ---------------------------------------------------------------- field, loss, gradient (T10-T12)

def test_T10_linearity_and_dot_product():
    G, M, R, Phi, C, om, T = _small_problem()
    I1 = O.currents(M, R, Phi, C, om)
    I2 = O.currents(M, R, 2.5 * Phi, C, om)
    np.testing.assert_allclose(I2, 2.5 * I1, rtol=1e-12)
    rng = np.random.default_rng(5)
    w = rng.normal(size=G.shape[0]) + 1j * rng.normal(size=G.shape[0])
    i = I1[0, 0]
    lhs = np.vdot(G.T @ np.conj(w), np.conj(i))
    rhs = np.vdot(np.conj(w), np.conj(G @ i))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_loss_weights_are_conjugate_derivative():
    rng = np.random.default_rng(3)
    B = rng.normal(size=(1, 2, 7)) + 1j * rng.normal(size=(1, 2, 7))
    T = rng.uniform(0, 1, 7)
    for mode in (O.LOSS_MAG, O.LOSS_COMPLEX):
        w = O.loss_weights(B, T, mode)
        h = 1e-7
        for idx in [(0, 0, 0), (0, 1, 4)]:
            e = np.zeros_like(B); e[idx] = h
            dre = (O.loss(B + e, T, mode) - O.loss(B - e, T, mode))[0] / (2 * h)
            dim = (O.loss(B + 1j * e, T, mode) - O.loss(B - 1j * e, T, mode))[0] / (2 * h)
            # dL/dB_re = 2 Re w, dL/dB_im = 2 Im w
            np.testing.assert_allclose([dre, dim], [2 * w[idx].real, 2 * w[idx].imag], rtol=1e-6)
    z = np.zeros((1, 1, 3), complex)
    assert np.all(O.loss_weights(z, np.ones(3)) == 0)


@pytest.mark.parametrize("mode", [O.LOSS_MAG, O.LOSS_COMPLEX])
def test_T11_adjoint_equals_forward_sensitivity_and_fd(mode):
    G, M, R, Phi, C, om, T = _small_problem(B=2, F=2)
    ga = O.grad_adjoint(G, M, R, Phi, C, om, T, mode)
    gf = O.grad_forward_sensitivity(G, M, R, Phi, C, om, T, mode)
    assert _rel(ga, gf) < 1e-12
    gd = O.grad_fd(G, M, R, Phi, C, om, T, h=1e-15, mode=mode)
    assert _rel(ga, gd) < 1e-6


def test_backward_from_field_grad_matches_loss_gradient():
    G, M, R, Phi, C, om, T = _small_problem(B=2, F=3)
    I = O.currents(M, R, Phi, C, om)
    Bz = O.field(G, I)
    gBz = 2 * O.loss_weights(Bz, T)
    np.testing.assert_allclose(O.backward_from_field_grad(G, M, R, C, om, I, gBz),
                               O.grad_adjoint(G, M, R, Phi, C, om, T), rtol=1e-12)


def test_T12_gram_identity_complex_mode():
    G, M, R, Phi, C, om, T = _small_problem(B=2, F=2, P=80)
    I = O.currents(M, R, Phi, C, om)
    L = O.loss(O.field(G, I), T, O.LOSS_COMPLEX)
    H = G.T @ G
    g = G.T @ T
    P = G.shape[0]
    for b in range(C.shape[0]):
        acc = 0.0
        for f in range(om.shape[0]):
            i = I[b, f]
            acc += (np.real(np.conj(i) @ H @ i) - 2 * np.real(g @ i) + T @ T) / P
        np.testing.assert_allclose(L[b], acc / om.shape[0], rtol=1e-10)


# ---------------------------------------------------------------- the optimiser on C
def test_adam_first_step_and_constant_gradient_closed_forms():
    """Step 1 of Adam moves every coordinate by lr * g / (|g| + eps) (both bias
    corrections are exact at t = 1), and under a constant gradient every later
    step does the same, so after t steps C = C0 - t * lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    C0 = rng.uniform(20e-12, 150e-12, size=(3, 5))
    g = rng.standard_normal((3, 5)) * 1e-2
    lr, eps = 1e-13, 1e-8
    C, m, v = O.adam_step(C0, g, np.zeros_like(C0), np.zeros_like(C0), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(C, C0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-26)
    for t in range(2, 8):
        C, m, v = O.adam_step(C, g, m, v, t, lr=lr, eps=eps)
    np.testing.assert_allclose(C, C0 - 7 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-25)


def test_adam_matches_torch_optimizer():
    """Independent implementation: torch.optim.Adam (CPU, float64) on the same
    gradient sequence follows the same trajectory."""
    import torch
    rng = np.random.default_rng(8)
    C0 = rng.uniform(20e-12, 150e-12, size=(4, 6))
    grads = [rng.standard_normal(C0.shape) * 10.0 ** rng.uniform(-3, 1) for _ in range(6)]
    p = torch.nn.Parameter(torch.tensor(C0))
    opt = torch.optim.Adam([p], lr=1e-13, betas=(0.9, 0.999), eps=1e-8)
    C, m, v = C0.copy(), np.zeros_like(C0), np.zeros_like(C0)
    for t, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g)
        opt.step()
        C, m, v = O.adam_step(C, g, m, v, t)
    np.testing.assert_allclose(C, p.detach().numpy(), rtol=1e-14, atol=0)


def test_array_inductance_by_offsets_equals_direct_oracle():
    """The offset-reuse builder used for large arrays in the GPU tests gives
    the direct oracle's M (rectangular array, so offsets are not symmetric)."""
    from array_oracle import oracle_M_array
    g = W.square_array(4, 3, 0.03, 0.035, 32, 1e-3, 0.3)
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    np.testing.assert_allclose(oracle_M_array(g), M, rtol=1e-13, atol=0)


# ------------------------------------------- the other circuit variables (R, L, w)

@pytest.mark.parametrize("mode", [O.LOSS_MAG, O.LOSS_COMPLEX])
def test_parameter_gradients_adjoint_sensitivity_fd(mode):
    """dL/dR, dL/dL (series inductance per loop) and dL/dw: the adjoint equals
    forward sensitivity through the solve, and both equal central differences."""
    G, M, R, Phi, C, om, T = _small_problem(B=2, F=2)
    a = O.grad_params_adjoint(G, M, R, Phi, C, om, T, mode)
    s = O.grad_params_forward_sensitivity(G, M, R, Phi, C, om, T, mode)
    d = O.grad_params_fd(G, M, R, Phi, C, om, T, mode)
    for x, y, z in zip(a, s, d):
        assert _rel(x, y) < 1e-12
        assert _rel(y, z) < 1e-6


def test_resonant_capacitance_eq13():
    """Eq. 13 makes the reactance vanish: for one loop Im Z(C_r) = 0; for the
    coupled array with equal currents in every loop Im (Z 1)_k = 0."""
    g = W.single_circle()
    M1 = O.inductance_matrix(g.verts, g.seg_off, g.wire_a)
    w = 2 * math.pi * 128e6
    Cr = O.resonant_capacitance(M1, w, coupled=False)
    assert abs(O.impedance(M1, g.R, Cr, w)[0, 0].imag) < 1e-12 * w * M1[0, 0]
    wl = W.small_array(3, 2, 1, 4, n_freq=1)
    M = O.inductance_matrix_fast(wl.geom.verts, wl.geom.seg_off, wl.geom.wire_a)
    Cr = O.resonant_capacitance(M, w, coupled=True)
    Z = O.impedance(M, wl.geom.R, Cr, w)
    assert np.max(np.abs((Z @ np.ones(len(Cr))).imag)) < 1e-10 * w * np.abs(M).max()
    Cs = O.resonant_capacitance(M, w, coupled=False)
    np.testing.assert_allclose(Cs, 1.0 / (w * w * np.diag(M)), rtol=1e-15)


def test_tanh_projection_range_and_derivative():
    th = np.linspace(-6, 6, 13)
    C, dC = O.tanh_projection(th, 10e-12, 300e-12)
    assert np.all(C > 10e-12) and np.all(C < 300e-12)
    np.testing.assert_allclose(O.tanh_projection(np.array([0.0]), 10e-12, 300e-12)[0], 155e-12, rtol=1e-15)
    h = 1e-6
    fd = (O.tanh_projection(th + h, 10e-12, 300e-12)[0] - O.tanh_projection(th - h, 10e-12, 300e-12)[0]) / (2 * h)
    # differences of values of order 1e-10 with step 1e-6 round at about 1e-20
    np.testing.assert_allclose(dC, fd, rtol=1e-7, atol=1e-9 * np.abs(dC).max())


# ------------------------------------------- enhancement factor (Sec. IV-B)

def test_ratio_loss_definition_cases():
    """beta = |bext + B| / |bext|: no scattered field gives beta = 1, a field that
    cancels the incident one gives beta = 0; the loss is the mean of
    (beta - T)^2."""
    bext = 1e-6
    T = np.array([0.5, 1.0, 2.0])
    z = np.zeros((1, 1, 3), complex)
    np.testing.assert_allclose(O.loss(z, T, O.LOSS_RATIO, bext), [np.mean((1 - T) ** 2)], rtol=1e-15)
    c = np.full((1, 1, 3), -bext + 0j)
    np.testing.assert_allclose(O.loss(c, T, O.LOSS_RATIO, bext), [np.mean(T ** 2)], rtol=1e-15)
    # doubled field, purely imaginary scattered field: beta = sqrt(1 + 1)
    q = np.full((1, 1, 3), 1j * bext)
    np.testing.assert_allclose(O.loss(q, T, O.LOSS_RATIO, bext), [np.mean((np.sqrt(2) - T) ** 2)],
                               rtol=1e-14)


def test_ratio_loss_weights_are_conjugate_derivative():
    rng = np.random.default_rng(8)
    bext = 1e-6
    B = (rng.normal(size=(1, 2, 7)) + 1j * rng.normal(size=(1, 2, 7))) * 4e-7
    T = rng.uniform(0.5, 2.0, 7)
    w = O.loss_weights(B, T, O.LOSS_RATIO, bext)
    h = 1e-13
    for idx in [(0, 0, 0), (0, 1, 4)]:
        e = np.zeros_like(B); e[idx] = h
        dre = (O.loss(B + e, T, O.LOSS_RATIO, bext) - O.loss(B - e, T, O.LOSS_RATIO, bext))[0] / (2 * h)
        dim = (O.loss(B + 1j * e, T, O.LOSS_RATIO, bext) - O.loss(B - 1j * e, T, O.LOSS_RATIO, bext))[0] / (2 * h)
        np.testing.assert_allclose([dre, dim], [2 * w[idx].real, 2 * w[idx].imag], rtol=1e-6)


def test_ratio_gradient_adjoint_sensitivity_fd():
    G, M, R, Phi, C, om, T = _small_problem(B=2, F=2)
    bext = 1e-6
    beta = np.linspace(0.8, 1.6, len(T))
    ga = O.grad_adjoint(G, M, R, Phi, C, om, beta, O.LOSS_RATIO, bext)
    gf = O.grad_forward_sensitivity(G, M, R, Phi, C, om, beta, O.LOSS_RATIO, bext)
    assert _rel(ga, gf) < 1e-12
    gd = O.grad_fd(G, M, R, Phi, C, om, beta, h=1e-15, mode=O.LOSS_RATIO, bext=bext)
    assert _rel(ga, gd) < 1e-5


# ------------------------------------------ field components (Sec. I-B: B_x, B_y, B_z)

@pytest.mark.parametrize("comp", [0, 1, 2])
def test_field_component_closed_form_vs_quadrature(comp):
    rng = np.random.default_rng(7 + comp)
    for _ in range(10):
        x1 = rng.uniform(-0.02, 0.02, 3); x2 = rng.uniform(-0.02, 0.02, 3)
        p = rng.uniform(-0.05, 0.05, (16, 3)); p[:, 2] += 0.03 * np.sign(p[:, 2] + 1e-9)
        cf = O.b_segment(p, x1, x2, comp)
        q = O.bz_segment_quadrature(p, x1, x2, order=48, panels=16, comp=comp)
        np.testing.assert_allclose(cf, q, rtol=1e-10, atol=1e-12 * np.abs(q).max())


def test_field_components_far_field_is_a_dipole():
    # a small planar loop far away: B = mu0/(4 pi r^3) (3 (m.rhat) rhat - m), m = I A z
    g = W.square_array(1, 1, 0.01, 0.0, 64)
    A = O.vector_area_z(g.verts, g.seg_off)[0]
    rng = np.random.default_rng(3)
    d = rng.normal(size=(12, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = 2.0 * d
    Gc = np.stack([O.field_matrix(g.verts, g.seg_off, pts, c)[:, 0] for c in range(3)], axis=1)
    m = np.array([0.0, 0.0, A])
    r = np.linalg.norm(pts, axis=1, keepdims=True)
    rh = pts / r
    dip = O.MU0_4PI * (3.0 * (rh @ m)[:, None] * rh - m[None, :]) / r ** 3
    # next multipole term is (size / r)^2 ~ 1e-5 smaller
    np.testing.assert_allclose(Gc, dip, atol=1e-4 * np.abs(dip).max())


def test_field_is_divergence_and_curl_free_off_the_wires():
    g = W.square_array(2, 1, 0.03, 0.035, 16)
    rng = np.random.default_rng(5)
    pts = np.column_stack([rng.uniform(-0.04, 0.04, 8), rng.uniform(-0.03, 0.03, 8),
                           rng.uniform(0.008, 0.02, 8)])
    h = 1e-6  # truncation ~ (h / distance)^2, rounding ~ eps distance / h

    def B(p):  # [P,3] field of loop 0 + 0.7 loop 1 (any current vector will do)
        return np.stack([O.field_matrix(g.verts, g.seg_off, p, c) @ np.array([1.0, 0.7])
                         for c in range(3)], axis=1)

    J = np.zeros((pts.shape[0], 3, 3))  # J[p, i, j] = dB_i / dx_j
    for j in range(3):
        e = np.zeros(3); e[j] = h
        J[:, :, j] = (B(pts + e) - B(pts - e)) / (2 * h)
    scale = np.abs(J).reshape(len(pts), -1).max(axis=1)   # per point
    div = J[:, 0, 0] + J[:, 1, 1] + J[:, 2, 2]
    curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)
    assert np.all(np.abs(div) < 1e-7 * scale)
    assert np.all(np.abs(curl).max(axis=1) < 1e-7 * scale)


def test_field_transverse_components_vanish_on_the_axis():
    c = W.single_circle(0.05, 64)
    pts = np.array([[0.0, 0.0, z] for z in (-0.03, 0.0, 0.01, 0.2)])
    bz = O.field_matrix(c.verts, c.seg_off, pts, 2)[:, 0]
    for comp in (0, 1):
        b = O.field_matrix(c.verts, c.seg_off, pts, comp)[:, 0]
        assert np.abs(b).max() < 1e-12 * np.abs(bz).max()


# ------------------------------------------------ drive port (Sec. IV-A, Eq. 4)

def _drive_setup(g, omega=123.5e6 * 2 * math.pi, seed=0, z0=50.0):
    M = O.inductance_matrix_fast(g.verts, g.seg_off, g.wire_a)
    n = g.n
    rng = np.random.default_rng(seed)
    C = rng.uniform(20e-12, 150e-12, (2, n))
    C[:, -1] = np.inf          # the coil has no capacitor
    R = g.R.copy(); R[-1] += z0  # the source impedance in series with the coil
    return M, R, C, np.array([omega])


def test_short_circuit_limit_of_a_missing_capacitor():
    g = W.with_drive_coil(W.single_circle(0.03, 64))
    M, R, C, om = _drive_setup(g)
    emf = np.array([0.0, O.drive_emf(1.0)])
    Phi = np.zeros(g.n)
    Cbig = C.copy(); Cbig[:, -1] = 1e30
    np.testing.assert_allclose(O.currents(M, R, Phi, C, om, emf),
                               O.currents(M, R, Phi, Cbig, om, emf), rtol=1e-13)


def test_drive_two_loop_closed_form():
    # coil d driven by E, loop 1 coupled through M12: Cramer's rule on the 2x2 system
    g = W.with_drive_coil(W.single_circle(0.03, 64))
    M, R, C, om = _drive_setup(g)
    w = om[0]
    E = O.drive_emf(1.0, 50.0, 0.3)
    Z11 = R[0] + 1j * w * M[0, 0] - 1j / (w * C[0, 0])
    Zdd = R[1] + 1j * w * M[1, 1]
    Zm = 1j * w * M[0, 1]
    det = Z11 * Zdd - Zm * Zm
    I = O.currents(M, R, np.zeros(2), C[:1], om, np.array([0.0, E]))[0, 0]
    np.testing.assert_allclose(I, [-Zm * E / det, Z11 * E / det], rtol=1e-13)
    np.testing.assert_allclose(abs(E), 2.0 * math.sqrt(50.0), rtol=1e-15)


def test_drive_power_balance():
    # sources deliver what the resistors dissipate: Re(I^H V) = sum R |I|^2
    g = W.with_drive_coil(W.square_array(3, 3, 0.03, 0.035, 16), radius=0.06, z=0.015)
    M, R, C, om = _drive_setup(g, seed=2)
    Phi = O.flux(g.verts, g.seg_off, 1e-6)
    emf = np.zeros(g.n, complex); emf[-1] = O.drive_emf(1.0, 50.0, 0.5)
    I = O.currents(M, R, Phi, C, om, emf)
    for b in range(C.shape[0]):
        V = O.excitation(Phi, om[0], emf)
        lhs = np.real(np.vdot(I[b, 0], V))
        rhs = np.sum(R * np.abs(I[b, 0]) ** 2)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("phase", [0.0, math.pi / 2])
def test_drive_port_matches_the_sparameter_pipeline(phase):
    """The same driven structure through Eq. 3-7: every loop is a port of the
    lossless structure j w M (S0 = (Zs - Z0)(Zs + Z0)^-1); the RC loads
    reflect with Gamma (Eq. 3); the coil's port is joined straight through to
    one external port (S_C12 = 1, S_C11 = 0 there) that sends sqrt(Z0 P)
    (Eq. 4).  Per-port fields with the other ports matched are G (1 - S0)/Z0,
    so Eq. 7 gives B = G I of the loop equations with the Thevenin EMF
    2 sqrt(Z0 P) and Z0 in series with the coil."""
    import oracle.sparam_oracle as SO
    z0, P = 50.0, 1.0
    g = W.with_drive_coil(W.square_array(2, 2, 0.03, 0.035, 16), radius=0.05, z=0.012)
    M, R, C, om = _drive_setup(g, seed=4, z0=z0)
    w = om[0]
    n0 = g.n
    pts = W.grid_points(4, 0.07, [0.01])
    Gm = O.field_matrix(g.verts, g.seg_off, pts)
    eye = np.eye(n0)
    Zs = 1j * w * M
    S0 = (Zs - z0 * eye) @ np.linalg.inv(Zs + z0 * eye)
    fields = (Gm @ (eye - S0) / z0)[None, :, None, :]          # [F][P][1][n0]
    N = n0 + 1
    SC = np.zeros((C.shape[0], 1, N, N), complex)
    gam = SO.rc_reflection(R[:-1], C[:, :-1], om, z0)           # [B][F][n0-1]
    for b in range(C.shape[0]):
        SC[b, 0, np.arange(n0 - 1), np.arange(n0 - 1)] = gam[b, 0]
        SC[b, 0, n0 - 1, n0] = 1.0
        SC[b, 0, n0, n0 - 1] = 1.0
    exc = np.array([math.sqrt(z0 * P) * complex(math.cos(phase), math.sin(phase))])
    x, Bc = SO.combine(S0[None], fields, SC, n0, exc)
    emf = np.zeros(n0, complex); emf[-1] = O.drive_emf(P, z0, phase)
    I = O.currents(M, R, np.zeros(n0), C, om, emf)
    np.testing.assert_allclose(Bc[..., 0], O.field(Gm, I), rtol=1e-10, atol=1e-12 * np.abs(Bc).max())
    np.testing.assert_allclose(np.einsum("ij,bfj->bfi", eye - S0, x) / z0, I, rtol=1e-10,
                               atol=1e-12 * np.abs(I).max())


def test_drive_gradients_adjoint_vs_differences():
    g = W.with_drive_coil(W.square_array(2, 1, 0.03, 0.035, 16), radius=0.045, z=0.015)
    M, R, C, om = _drive_setup(g, seed=6)
    pts = W.grid_points(5, 0.06, [0.01])
    G = O.field_matrix(g.verts, g.seg_off, pts)
    Phi = np.zeros(g.n)
    emf = np.zeros(g.n, complex); emf[-1] = O.drive_emf(1.0, 50.0, 0.2)
    I = O.currents(M, R, Phi, C, om, emf)
    T = 0.8 * np.abs(O.field(G, I))[0, 0]
    ga = O.grad_adjoint(G, M, R, Phi, C, om, T, emf=emf)
    gs = O.grad_forward_sensitivity(G, M, R, Phi, C, om, T, emf=emf)
    Cf = C.copy(); Cf[:, -1] = 1e30   # differences need a finite value; the limit is the same
    gd = O.grad_fd(G, M, R, Phi, Cf, om, T, h=1e-16, emf=emf)
    assert np.all(ga[:, -1] == 0.0)
    np.testing.assert_allclose(ga, gs, rtol=1e-9, atol=1e-12 * np.abs(ga).max())
    np.testing.assert_allclose(ga[:, :-1], gd[:, :-1], rtol=1e-5)
    pa = O.grad_params_adjoint(G, M, R, Phi, C, om, T, emf=emf)
    ps = O.grad_params_forward_sensitivity(G, M, R, Phi, C, om, T, emf=emf)
    pd = O.grad_params_fd(G, M, R, Phi, C, om, T, emf=emf)
    for a, s_, d in zip(pa, ps, pd):
        np.testing.assert_allclose(a, s_, rtol=1e-9, atol=1e-12 * np.abs(a).max())
        np.testing.assert_allclose(a, d, rtol=2e-5, atol=1e-6 * np.abs(a).max())
