"""FP64 CPU oracle for the capacitance -> B_z path and its gradient.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: the two meet only in the seeded input
generators of ``workloads``.

What is computed (paper: Sec. I-A names the quasi-static model "circuit model
combined with the Biot-Savart law"; Sec. II states the forward problem C -> B
and the MSE inverse problem, Eq. 1; Sec. III gives the RC load, Eq. 2, and the
S-parameter cosimulation, Eq. 3-7; Sec. IV-A gives the loop impedance, Eq. 11):

1. G[p,k]   field at point p per ampere in loop k (Biot-Savart, straight
            filaments, closed form of Hanson & Hirshman 2002); the z-component
            (normal to the structure) by default, x or y on request (Sec. I-B
            asks for all three Cartesian components).
2. M[k,l]   Neumann mutual inductance between loop filaments; the diagonal
            uses the reduced kernel 1/sqrt(|r-r'|^2 + a^2) with wire radius a.
3. Phi[k]   flux of the uniform incident field B_ext,z through loop k
            (z-component of the vector area, shoelace formula).
4. Z        R + j w M + 1/(j w C) per (configuration, frequency) (Eq. 2, 11).
5. I        Z I = emf - j w Phi   (Eq. 6 in impedance form; see
            ``sform_currents`` for the literal S-parameter route, which reaches
            the same I).  emf: source EMF of driven ports (Eq. 4 through
            ``drive_emf``); a loop without a capacitor has C = +inf.
6. B_z      G I               (Eq. 7, z-component of the superposition).
7. loss     mean over (f,p) of (|B_z| - T)^2 (Eq. 1 on magnitudes), or
            mean |B_z - T|^2 (complex mode).
8. dL/dC    by brute-force forward sensitivity (Eq. 8-10 specialised to
            dZ/dC_k), by the adjoint, and by central finite differences.
9. Adam     the optimiser the paper runs on C (Sec. IV), one step as defined
            by Kingma & Ba (bias-corrected first and second moments).
10. the other circuit variables of Fig. 2: dL/dR, dL/dL (a series
            inductance per loop) and dL/dw, by forward sensitivity, by the
            adjoint and by central differences; the resonance capacitance of
            Eq. 13; the bounded tanh projection of C and its derivative.

Everything is float64 / complex128 NumPy.  Pins: tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np
from scipy import integrate

# Vacuum permeability, CODATA 2018 value (N/A^2).
MU0 = 1.25663706212e-6
MU0_4PI = MU0 / (4.0 * math.pi)

LOSS_MAG = 0
LOSS_COMPLEX = 1
LOSS_RATIO = 2  # enhancement factor of the total field (Sec. IV-B); needs bext


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------

def segments(verts: np.ndarray, seg_off: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Start and end points of the closed polygon k."""
    v = np.asarray(verts[seg_off[k]:seg_off[k + 1]], dtype=np.float64)
    return v, np.roll(v, -1, axis=0)


def vector_area_z(verts: np.ndarray, seg_off: np.ndarray) -> np.ndarray:
    """z-component of each loop's vector area, 1/2 sum (x_i y_{i+1} - x_{i+1} y_i).

    For a uniform incident field along z the flux is exactly B_ext,z times this."""
    n = len(seg_off) - 1
    out = np.zeros(n)
    for k in range(n):
        a, b = segments(verts, seg_off, k)
        out[k] = 0.5 * float(np.sum(a[:, 0] * b[:, 1] - b[:, 0] * a[:, 1]))
    return out


# ---------------------------------------------------------------------------
# 1. Biot-Savart field matrix
# ---------------------------------------------------------------------------

def b_segment(p: np.ndarray, x1: np.ndarray, x2: np.ndarray, comp: int = 2) -> np.ndarray:
    """Cartesian component `comp` (0 x, 1 y, 2 z) of the field per ampere of the
    straight filament x1 -> x2 at points p [...,3].

    With a = x1 - p, b = x2 - p the field of a finite straight filament is
    mu0/(4 pi) * (a x b) (|a| + |b|) / (|a| |b| (|a| |b| + a.b)).
    Where a.b < 0 (p beside the filament) the factor 1/(|a||b| + a.b) is
    replaced by the equal (|a||b| - a.b)/|a x b|^2, which does not cancel."""
    a = x1 - p
    b = x2 - p
    la = np.sqrt(np.sum(a * a, axis=-1))
    lb = np.sqrt(np.sum(b * b, axis=-1))
    c = np.cross(a, b)
    cz = c[..., comp]
    dot = np.sum(a * b, axis=-1)
    ab = la * lb
    c2 = np.sum(c * c, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(dot >= 0, 1.0 / (ab + dot), (ab - dot) / c2)
    return MU0_4PI * cz * (la + lb) * inv / ab


def bz_segment(p: np.ndarray, x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """z-component of ``b_segment``."""
    return b_segment(p, x1, x2, 2)


def field_matrix(verts: np.ndarray, seg_off: np.ndarray, pts: np.ndarray,
                 comp: int = 2) -> np.ndarray:
    """G[p,k] = sum over the segments of loop k of b_segment (T/A), field
    component `comp` (0 x, 1 y, 2 z)."""
    n = len(seg_off) - 1
    G = np.zeros((pts.shape[0], n))
    for k in range(n):
        a, b = segments(verts, seg_off, k)
        for s in range(a.shape[0]):
            G[:, k] += b_segment(pts, a[s], b[s], comp)
    return G


def bz_segment_quadrature(p: np.ndarray, x1: np.ndarray, x2: np.ndarray,
                          order: int = 64, panels: int = 8, comp: int = 2) -> np.ndarray:
    """Same quantity by composite Gauss-Legendre quadrature of the
    Biot-Savart integrand (dl x r)/|r|^3 along the filament (a brute-force
    check of the closed form); component `comp` of dl x r."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    d = x2 - x1
    out = np.zeros(p.shape[:-1])
    for j in range(panels):
        t = (j + 0.5 * (xg + 1.0)) / panels
        w = 0.5 * wg / panels
        for ti, wi in zip(t, w):
            src = x1 + ti * d
            r = p - src
            r3 = np.sum(r * r, axis=-1) ** 1.5
            u, v = (comp + 1) % 3, (comp + 2) % 3
            out += wi * (d[u] * r[..., v] - d[v] * r[..., u]) / r3
    return MU0_4PI * out


# ---------------------------------------------------------------------------
# 2. Neumann inductance
# ---------------------------------------------------------------------------

def _parallel_F(u: float, d: float) -> float:
    """Double antiderivative of 1/sqrt(u^2+d^2); the d -> 0 limit drops the
    terms that cancel between the four corners (they are linear in |u|)."""
    if d == 0.0:
        return 0.0 if u == 0.0 else abs(u) * math.log(abs(u))
    return u * math.asinh(u / d) - math.sqrt(u * u + d * d)


def neumann_segments(x1, x2, y1, y2, a: float = 0.0) -> float:
    """(mu0/4pi) * integral over both filaments of dl.dl' / sqrt(|r-r'|^2 + a^2).

    Parallel (or anti-parallel) filaments: closed form (Grover).  Perpendicular
    filaments: exactly zero (dl.dl' = 0).  Otherwise: inner integral in closed
    form, outer integral by adaptive quadrature (QUADPACK)."""
    x1 = np.asarray(x1, float); x2 = np.asarray(x2, float)
    y1 = np.asarray(y1, float); y2 = np.asarray(y2, float)
    du = x2 - x1
    dv = y2 - y1
    L1 = float(np.linalg.norm(du))
    L2 = float(np.linalg.norm(dv))
    u = du / L1
    v = dv / L2
    cosang = float(np.dot(u, v))
    cross = np.cross(u, v)
    sinang = float(np.linalg.norm(cross))
    if sinang < 1e-12:
        # both on lines parallel to u; coordinates along u and perpendicular distance
        sgn = 1.0 if cosang > 0 else -1.0
        w = y1 - x1
        s_along = float(np.dot(w, u))
        perp = w - s_along * u
        d2 = float(np.dot(perp, perp)) + a * a
        d = math.sqrt(d2)
        if d < 1e-12 * max(L1, L2):
            d = 0.0
        # filament 2 spans [b1, b2] along u (in the direction of u)
        b1 = s_along
        b2 = s_along + sgn * L2
        lo2, hi2 = min(b1, b2), max(b1, b2)
        val = (_parallel_F(L1 - lo2, d) - _parallel_F(L1 - hi2, d)
               - _parallel_F(0.0 - lo2, d) + _parallel_F(0.0 - hi2, d))
        return MU0_4PI * sgn * val
    if abs(cosang) < 1e-12:
        return 0.0

    def inner(s):
        x = x1 + s * u
        w = x - y1
        t0 = float(np.dot(w, v))
        rho2 = float(np.dot(w, w)) - t0 * t0
        r = math.sqrt(max(rho2, 0.0) + a * a)
        if r == 0.0:
            r = 1e-300
        return math.asinh((L2 - t0) / r) + math.asinh(t0 / r)

    val, _ = integrate.quad(inner, 0.0, L1, epsabs=0.0, epsrel=1e-13, limit=400)
    return MU0_4PI * cosang * val


def inductance_matrix(verts, seg_off, wire_a) -> np.ndarray:
    """M[k,l]: exact Neumann integral between the filament axes for k != l;
    the reduced-kernel self term (offset a = wire radius) on the diagonal.
    Every entry is computed on its own (no mirroring), so M - M^T is a check."""
    n = len(seg_off) - 1
    M = np.zeros((n, n))
    for k in range(n):
        ak, bk = segments(verts, seg_off, k)
        for l in range(n):
            al, bl = segments(verts, seg_off, l)
            reg = float(wire_a[k]) if k == l else 0.0
            acc = 0.0
            for s in range(ak.shape[0]):
                for t in range(al.shape[0]):
                    acc += neumann_segments(ak[s], bk[s], al[t], bl[t], reg)
            M[k, l] = acc
    return M


def inductance_matrix_fast(verts, seg_off, wire_a) -> np.ndarray:
    """Same values for arrays of axis-aligned loops (every segment parallel or
    perpendicular to every other), vectorised over segment pairs with the
    same closed forms; falls back to ``inductance_matrix`` otherwise."""
    n = len(seg_off) - 1
    starts = [segments(verts, seg_off, k) for k in range(n)]
    allv = np.concatenate([a for a, _ in starts]); allw = np.concatenate([b for _, b in starts])
    d = allw - allv
    nz = np.count_nonzero(np.abs(d) > 1e-15 * np.max(np.abs(d)), axis=1)
    if np.any(nz != 1):
        return inductance_matrix(verts, seg_off, wire_a)
    M = np.zeros((n, n))
    for k in range(n):
        ak, bk = starts[k]
        for l in range(n):
            al, bl = starts[l]
            reg = float(wire_a[k]) if k == l else 0.0
            M[k, l] = _axis_aligned_block(ak, bk, al, bl, reg)
    return M


def inductance_matrix_lattice(verts, seg_off, wire_a, nx: int, ny: int) -> np.ndarray:
    """M of an nx-by-ny lattice of identical loops (loop k = iy*nx + ix, the
    same polygon translated, one wire radius), with the values of
    ``inductance_matrix_fast``: the Neumann integral between two loops is
    unchanged when both are translated together, so M[k, l] depends only on
    the lattice offset of l from k.  Each distinct offset is evaluated once
    on a two-loop geometry, the diagonal on a one-loop geometry; equal values
    are reused, nothing else differs."""
    n = nx * ny
    so = np.asarray(seg_off)
    wa = np.asarray(wire_a, dtype=np.float64)
    if len(so) != n + 1:
        raise ValueError("seg_off does not describe nx * ny loops")
    if np.any(wa != wa[0]):
        raise ValueError("a lattice needs one wire radius")

    def loop(k):
        return np.asarray(verts[so[k]:so[k + 1]], dtype=np.float64)

    cache = {}
    M = np.empty((n, n))
    for k in range(n):
        iyk, ixk = divmod(k, nx)
        for l in range(n):
            iyl, ixl = divmod(l, nx)
            key = (ixl - ixk, iyl - iyk)
            v = cache.get(key)
            if v is None:
                vk = loop(k)
                if k == l:
                    v = inductance_matrix_fast(vk, np.array([0, len(vk)], dtype=np.int32),
                                               wa[k:k + 1])[0, 0]
                else:
                    vl = loop(l)
                    two = np.concatenate([vk, vl])
                    off = np.array([0, len(vk), len(vk) + len(vl)], dtype=np.int32)
                    v = inductance_matrix_fast(two, off, np.array([wa[k], wa[l]]))[0, 1]
                cache[key] = v
            M[k, l] = v
    return M


def _axis_aligned_block(ak, bk, al, bl, a):
    du = bk - ak
    dv = bl - al
    axis_u = np.argmax(np.abs(du), axis=1)
    axis_v = np.argmax(np.abs(dv), axis=1)
    total = 0.0
    for ax in range(3):
        iu = np.nonzero(axis_u == ax)[0]
        iv = np.nonzero(axis_v == ax)[0]
        if iu.size == 0 or iv.size == 0:
            continue
        x1 = ak[iu][:, None, :]; x2 = bk[iu][:, None, :]
        y1 = al[iv][None, :, :]; y2 = bl[iv][None, :, :]
        lo1 = np.minimum(x1[..., ax], x2[..., ax]); hi1 = np.maximum(x1[..., ax], x2[..., ax])
        lo2 = np.minimum(y1[..., ax], y2[..., ax]); hi2 = np.maximum(y1[..., ax], y2[..., ax])
        sgn = np.sign(x2[..., ax] - x1[..., ax]) * np.sign(y2[..., ax] - y1[..., ax])
        others = [c for c in range(3) if c != ax]
        d2 = sum((x1[..., c] - y1[..., c]) ** 2 for c in others) + a * a
        dd = np.sqrt(d2)
        dd = np.where(dd < 1e-12 * (hi1 - lo1), 0.0, dd)

        def F(u):
            with np.errstate(divide="ignore", invalid="ignore"):
                par = u * np.arcsinh(u / np.where(dd > 0, dd, 1.0)) - np.sqrt(u * u + dd * dd)
                au = np.abs(u)
                lim = np.where(au > 0, au * np.log(np.where(au > 0, au, 1.0)), 0.0)
            return np.where(dd > 0, par, lim)

        val = F(hi1 - lo2) - F(hi1 - hi2) - F(lo1 - lo2) + F(lo1 - hi2)
        total += float(np.sum(sgn * val))
    return MU0_4PI * total


# ---------------------------------------------------------------------------
# 3.-6. excitation, impedance, currents, field
# ---------------------------------------------------------------------------

def flux(verts, seg_off, bext_z: float) -> np.ndarray:
    return bext_z * vector_area_z(verts, seg_off)


def impedance(M: np.ndarray, R: np.ndarray, C: np.ndarray, omega: float) -> np.ndarray:
    """Z = diag(R) + j w M + diag(1/(j w C)) for one configuration (Eq. 2, 11).
    The capacitor term is written -j/(w C) so that C = +inf (a loop without a
    series capacitor, e.g. a drive coil) gives the short-circuit limit 0."""
    Z = 1j * omega * M.astype(np.complex128)
    Z[np.diag_indices_from(Z)] += R - 1j / (omega * C)
    return Z


def drive_emf(power: float = 1.0, z0: float = 50.0, phase: float = 0.0) -> complex:
    """Source EMF of a port driven as in Eq. 4: the excitation sends the wave
    sqrt(Z0 P) toward the port through its characteristic impedance Z0; a
    source of internal impedance Z0 emitting that wave has the Thevenin EMF
    2 sqrt(Z0 P).  In the loop equations the port adds Z0 to the loop's
    series resistance and this EMF (times exp(j phase)) to its voltage."""
    return 2.0 * math.sqrt(z0 * power) * complex(math.cos(phase), math.sin(phase))


def excitation(Phi, omega: float, emf=None) -> np.ndarray:
    """Loop voltages V = emf - j w Phi: the EMF of the incident flux plus any
    source EMF in series with a loop (frequency independent)."""
    V = -1j * omega * np.asarray(Phi, dtype=np.complex128)
    if emf is not None:
        V = V + np.asarray(emf, dtype=np.complex128)
    return V


def currents(M, R, Phi, C, omega, emf=None) -> np.ndarray:
    """I[b,f,:] solving Z I = emf - j w Phi with LAPACK (zgesv) per system."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    out = np.zeros((C.shape[0], omega.shape[0], M.shape[0]), dtype=np.complex128)
    for b in range(C.shape[0]):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            out[b, f] = np.linalg.solve(Z, excitation(Phi, w, emf))
    return out


def field(G: np.ndarray, I: np.ndarray) -> np.ndarray:
    """B_z[b,f,p] = sum_k G[p,k] I[b,f,k] (Eq. 7, z-component)."""
    return np.einsum("pk,bfk->bfp", G, I)


# ---------------------------------------------------------------------------
# 7. loss
# ---------------------------------------------------------------------------

def loss(Bz: np.ndarray, T: np.ndarray, mode: int = LOSS_MAG, bext: float = 0.0) -> np.ndarray:
    """Per-configuration loss, mean over (f,p).  LOSS_RATIO: the enhancement
    factor of Sec. IV-B, beta = |H_with structure| / |H_reference|, here
    |bext + B_z| / |bext| (the reference is the incident field alone), against
    the targets T: mean of (beta - T)^2."""
    F, P = Bz.shape[1], Bz.shape[2]
    if mode == LOSS_RATIO:
        e = np.abs(bext + Bz) / abs(bext) - T[None, None, :]
        return np.sum(e * e, axis=(1, 2)) / (F * P)
    if mode == LOSS_MAG:
        e = np.abs(Bz) - T[None, None, :]
        return np.sum(e * e, axis=(1, 2)) / (F * P)
    e = Bz - T[None, None, :]
    return np.sum((e * np.conj(e)).real, axis=(1, 2)) / (F * P)


def loss_weights(Bz: np.ndarray, T: np.ndarray, mode: int = LOSS_MAG,
                 bext: float = 0.0) -> np.ndarray:
    """w = dL/d conj(B_z): the loss is real, so dL = 2 Re(sum conj(w) dB).
    Magnitude mode: w = (|B|-T) B/|B| / (F P), taken as 0 where B = 0.
    Ratio mode: with Bt = bext + B_z, d(|Bt|/|bext| - T)^2 / dconj(B_z) =
    (|Bt|/|bext| - T) Bt / (|bext| |Bt|), over (F P)."""
    F, P = Bz.shape[1], Bz.shape[2]
    if mode == LOSS_RATIO:
        Bt = bext + Bz
        mag = np.abs(Bt)
        with np.errstate(divide="ignore", invalid="ignore"):
            unit = np.where(mag > 0, Bt / np.where(mag > 0, mag, 1.0), 0.0)
        return (mag / abs(bext) - T[None, None, :]) * unit / abs(bext) / (F * P)
    if mode == LOSS_MAG:
        mag = np.abs(Bz)
        with np.errstate(divide="ignore", invalid="ignore"):
            unit = np.where(mag > 0, Bz / np.where(mag > 0, mag, 1.0), 0.0)
        return (mag - T[None, None, :]) * unit / (F * P)
    return (Bz - T[None, None, :]) / (F * P)


def evaluate(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, bext: float = 0.0, emf=None):
    I = currents(M, R, Phi, C, omega, emf)
    Bz = field(G, I)
    return I, Bz, loss(Bz, T, mode, bext)


# ---------------------------------------------------------------------------
# 8. gradient
# ---------------------------------------------------------------------------

def grad_forward_sensitivity(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, bext: float = 0.0,
                             emf=None) -> np.ndarray:
    """dL/dC by differentiating the solve column by column (Eq. 9 with
    dZ/dC_k = -e_k e_k^T / (j w C_k^2)):  dI/dC_k = Z^-1 e_k I_k / (j w C_k^2),
    dL/dC_k = 2 Re sum_{f,p} conj(w) (G dI/dC_k)."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    I = currents(M, R, Phi, C, omega, emf)
    W = loss_weights(field(G, I), T, mode, bext)
    n = M.shape[0]
    g = np.zeros(C.shape)
    for b in range(C.shape[0]):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            for k in range(n):
                e = np.zeros(n, dtype=np.complex128)
                e[k] = 1.0
                dI = np.linalg.solve(Z, e) * I[b, f, k] * (-1j / (w * C[b, k] ** 2))
                dB = G @ dI
                g[b, k] += 2.0 * float(np.real(np.sum(np.conj(W[b, f]) * dB)))
    return g


def grad_adjoint(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, bext: float = 0.0,
                 emf=None) -> np.ndarray:
    """dL/dC by the adjoint: r = G^T conj(w); Z^T mu = r;
    dL/dC_k = 2 Re sum_f mu_k I_k / (j w C_k^2)."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    I = currents(M, R, Phi, C, omega, emf)
    W = loss_weights(field(G, I), T, mode, bext)
    g = np.zeros(C.shape)
    for b in range(C.shape[0]):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            r = G.T @ np.conj(W[b, f])
            mu = np.linalg.solve(Z.T, r)
            g[b] += 2.0 * np.real(mu * I[b, f] * (-1j / (w * C[b] ** 2)))
    return g


def grad_fd(G, M, R, Phi, C, omega, T, h: float = 1e-15, mode: int = LOSS_MAG,
            bext: float = 0.0, emf=None) -> np.ndarray:
    """Central finite differences of the loss, step h farads."""
    C = np.atleast_2d(np.asarray(C, float))
    g = np.zeros(C.shape)
    for b in range(C.shape[0]):
        for k in range(C.shape[1]):
            cp = C[b:b + 1].copy(); cp[0, k] += h
            cm = C[b:b + 1].copy(); cm[0, k] -= h
            lp = evaluate(G, M, R, Phi, cp, omega, T, mode, bext, emf)[2][0]
            lm = evaluate(G, M, R, Phi, cm, omega, T, mode, bext, emf)[2][0]
            g[b, k] = (lp - lm) / (2 * h)
    return g


def grad_params_forward_sensitivity(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, bext: float = 0.0,
                                    emf=None):
    """Gradients of each configuration's loss with respect to the other circuit
    parameters of Eq. 11 (the variables of Fig. 2 besides C), by perturbing one
    parameter at a time through the solve (Eq. 9): dI = Z^-1 (dV - dZ I) with
    V = emf - j w Phi (emf does not depend on w), and dL = 2 Re sum_p conj(w_p) (G dI)_p.
      R_k:  dZ = e_k e_k^T;
      L_k (a series inductance added to loop k): dZ = j w e_k e_k^T;
      w_f:  dZ = j M - diag(1 / (j w^2 C)) and dV = -j Phi (G does not depend on w).
    Returns (dL/dR [B][n], dL/dL [B][n], dL/dw [B][F])."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    I = currents(M, R, Phi, C, omega, emf)
    W = loss_weights(field(G, I), T, mode, bext)
    B, n, F = C.shape[0], M.shape[0], omega.shape[0]
    gR = np.zeros((B, n))
    gL = np.zeros((B, n))
    gw = np.zeros((B, F))
    for b in range(B):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            i = I[b, f]

            def dL(dZ, dV):
                dI = np.linalg.solve(Z, dV - dZ @ i)
                return 2.0 * float(np.real(np.sum(np.conj(W[b, f]) * (G @ dI))))

            zero = np.zeros(n, dtype=np.complex128)
            for k in range(n):
                E = np.zeros((n, n), dtype=np.complex128)
                E[k, k] = 1.0
                gR[b, k] += dL(E, zero)
                gL[b, k] += dL(1j * w * E, zero)
            dZw = 1j * M + np.diag(1j / (w * w * C[b]))
            gw[b, f] = dL(dZw, -1j * Phi)
    return gR, gL, gw


def grad_params_adjoint(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, bext: float = 0.0,
                        emf=None):
    """The same gradients through the adjoint of each system: with
    Z mu = G^T conj(w) (Z is complex symmetric), dL = 2 Re(mu^T (dV - dZ I)):
      dL/dR_k = -2 Re(mu_k I_k),  dL/dL_k = 2 w Im(mu_k I_k),
      dL/dw = 2 Re(-j mu^T Phi - j mu^T M I + sum_k mu_k I_k / (j w^2 C_k))."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    I = currents(M, R, Phi, C, omega, emf)
    W = loss_weights(field(G, I), T, mode, bext)
    B, n, F = C.shape[0], M.shape[0], omega.shape[0]
    gR = np.zeros((B, n))
    gL = np.zeros((B, n))
    gw = np.zeros((B, F))
    for b in range(B):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            mu = np.linalg.solve(Z, G.T @ np.conj(W[b, f]))
            i = I[b, f]
            gR[b] += -2.0 * np.real(mu * i)
            gL[b] += 2.0 * w * np.imag(mu * i)
            t = -1j * (mu @ Phi) - 1j * (mu @ (M @ i)) + np.sum(mu * i * (-1j / (w * w * C[b])))
            gw[b, f] = 2.0 * np.real(t)
    return gR, gL, gw


def grad_params_fd(G, M, R, Phi, C, omega, T, mode: int = LOSS_MAG, hR: float = 1e-7,
                   hL: float = 1e-15, hw: float = 1.0, bext: float = 0.0, emf=None):
    """Central differences of the loss for the same parameters (steps in ohm,
    henry and rad/s); a series inductance L_k enters as M_kk + L_k."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(np.asarray(omega, float))
    B, n, F = C.shape[0], M.shape[0], omega.shape[0]
    gR = np.zeros((B, n))
    gL = np.zeros((B, n))
    gw = np.zeros((B, F))
    L0 = evaluate  # local alias

    def loss_of(Mv, Rv, om):
        return L0(G, Mv, Rv, Phi, C, om, T, mode, bext, emf)[2]

    for k in range(n):
        Rp, Rm = R.copy(), R.copy()
        Rp[k] += hR
        Rm[k] -= hR
        gR[:, k] = (loss_of(M, Rp, omega) - loss_of(M, Rm, omega)) / (2 * hR)
        Mp, Mm = M.copy(), M.copy()
        Mp[k, k] += hL
        Mm[k, k] -= hL
        gL[:, k] = (loss_of(Mp, R, omega) - loss_of(Mm, R, omega)) / (2 * hL)
    for f in range(F):
        op, om_ = omega.copy(), omega.copy()
        op[f] += hw
        om_[f] -= hw
        gw[:, f] = (loss_of(M, R, op) - loss_of(M, R, om_)) / (2 * hw)
    return gR, gL, gw


def resonant_capacitance(M, omega: float, coupled: bool = True) -> np.ndarray:
    """Eq. 13: C_r = 1 / (w^2 (L + M)).  L_k = M_kk; with `coupled`, M is the
    sum of the loop's mutual inductances to all others (every loop carrying the
    same current), otherwise 0 (the single-cell case of Sec. IV-A)."""
    Lk = np.diag(M) if not coupled else M.sum(axis=1)
    return 1.0 / (omega * omega * Lk)


def tanh_projection(theta, cmin: float, cmax: float):
    """The bounded projection discussed in Sec. V: C = cmin + (cmax - cmin)
    (1 + tanh(theta)) / 2, and dC/dtheta = (cmax - cmin) (1 - tanh^2) / 2."""
    t = np.tanh(theta)
    return cmin + 0.5 * (cmax - cmin) * (1.0 + t), 0.5 * (cmax - cmin) * (1.0 - t * t)


def backward_from_field_grad(G, M, R, C, omega, I, gBz) -> np.ndarray:
    """Real dL/dC given an upstream complex gradient gBz in PyTorch's
    convention (gBz = 2 dL/d conj(B_z)) for B_z = G I(C)."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    g = np.zeros(C.shape)
    for b in range(C.shape[0]):
        for f, w in enumerate(omega):
            Z = impedance(M, R, C[b], w)
            r = G.T @ np.conj(0.5 * gBz[b, f])
            mu = np.linalg.solve(Z.T, r)
            g[b] += 2.0 * np.real(mu * I[b, f] * (-1j / (w * C[b] ** 2)))
    return g


# ---------------------------------------------------------------------------
# Optimiser on C (Sec. IV: Adam on the capacitances)
# ---------------------------------------------------------------------------

def adam_step(C, g, m, v, t: int, lr: float = 1e-13, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """Step t (1-based) of Adam (Kingma & Ba 2015, Algorithm 1): moments
    m, v of g, their bias corrections m / (1 - beta1^t), v / (1 - beta2^t),
    and C - lr * mhat / (sqrt(vhat) + eps).  Returns new (C, m, v)."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return C - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# S-parameter route (Eq. 3-7), used as an independent check of the solve
# ---------------------------------------------------------------------------

def sform_currents(M, R, Phi, C, omega, Z0: float = 50.0) -> np.ndarray:
    """Loop currents reached through the paper's wave formulation.

    Each loop is a port loaded by the RC branch of Eq. 2 in series with the
    induced EMF E = -j w Phi.  The structure is the multiport with impedance
    matrix j w M, so its scattering matrix is S0 = (Zs - Z0)(Zs + Z0)^-1.
    The load reflection is Eq. 3 and the source injects Z0 E/(Z_L + Z0) into
    the incident wave (Eq. 4); Eq. 5-6 give V+ = (1 - Gamma S0)^-1 q and the
    port current is (V+ - V-)/Z0 = (1 - S0) V+ / Z0."""
    C = np.atleast_2d(C)
    omega = np.atleast_1d(omega)
    n = M.shape[0]
    out = np.zeros((C.shape[0], omega.shape[0], n), dtype=np.complex128)
    eye = np.eye(n)
    for b in range(C.shape[0]):
        for f, w in enumerate(omega):
            Zs = 1j * w * M
            S0 = (Zs - Z0 * eye) @ np.linalg.inv(Zs + Z0 * eye)
            ZL = R - 1j / (w * C[b])                        # Eq. 2
            gam = (ZL - Z0) / (ZL + Z0)                      # Eq. 3
            E = -1j * w * Phi
            q = Z0 * E / (ZL + Z0)
            A = eye - np.diag(gam) @ S0                      # A of Eq. 6
            vp = np.linalg.solve(A, q)
            vm = S0 @ vp                                     # Eq. 5
            out[b, f] = (vp - vm) / Z0
    return out


# ---------------------------------------------------------------------------
# textbook references used by the pins
# ---------------------------------------------------------------------------

def polygon_axis_bz(N: int, Rc: float, z: float, I: float = 1.0) -> float:
    """On-axis z-field of a regular N-gon of circumradius Rc carrying I."""
    s = Rc * math.sin(math.pi / N)
    h = Rc * math.cos(math.pi / N)
    return N * MU0 * I * s * h / (2.0 * math.pi * (h * h + z * z) * math.sqrt(Rc * Rc + z * z))


def circle_axis_bz(R: float, z: float, I: float = 1.0) -> float:
    return MU0 * I * R * R / (2.0 * (R * R + z * z) ** 1.5)


def coaxial_circles_mutual(R1: float, R2: float, d: float) -> float:
    """Maxwell's mutual inductance of two coaxial circles at axial distance d,
    complete elliptic integrals K, E (scipy uses parameter m = k^2)."""
    from scipy.special import ellipk, ellipe
    k2 = 4.0 * R1 * R2 / ((R1 + R2) ** 2 + d * d)
    k = math.sqrt(k2)
    return MU0 * math.sqrt(R1 * R2) * ((2.0 / k - k) * ellipk(k2) - (2.0 / k) * ellipe(k2))
