"""FP64 CPU oracle for the paper's S-parameter cosimulation pipeline.

TEST INFRASTRUCTURE ONLY.  Like ``cosim_oracle``, this module is the slow,
plain reference that the HIP library is checked against; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may use
it, and it shares no code with the HIP library.

What is computed (paper: Sec. III, Eq. 2-10, and the pipeline of Sec. III-A):

* The resonant structure has n0 ports, described per frequency by its
  scattering matrix S0 [n0][n0] and by the field each port radiates for a
  unit incident voltage wave with the other ports matched, B [P][ncomp][n0]
  (the paper's (n_points, 3, n0) export).
* The connecting network S_C [(n0+n1)][(n0+n1)] per (configuration,
  frequency) is S_C,const + S_C,var, where S_C,var is zero except at the
  user's (row, column) index pairs, which receive the values produced by a
  user-defined preprocessing step (Sec. III-A, steps 1-3).  Its blocks are
  S_C11 = S_C[:n0, :n0], S_C12 = S_C[:n0, n0:] (Fig. 1).
* Eq. 6: the ratio of incident waves at the structure to the outgoing waves
  of the n1 external ports is X = (I - S_C11 S0)^-1 S_C12.  The external
  ports are driven by the waves `exc` [n1] (for one port of power P behind
  the impedance Z'_exc that is sqrt(Z'_exc P), Eq. 4), so the incident waves
  are x = X exc.
* Eq. 7: the combined field is B_comb[p, c] = sum_k B[p, c, k] x_k.
* The loss is the mean over frequencies and points of (|B_comb[p, comp]| -
  T_p)^2 (magnitudes, as in Sec. IV) or |B_comb[p, comp] - T_p|^2.
* Gradients with respect to the variable entries v_e, reported as
  2 dL/dconj(v_e) (PyTorch's convention for complex leaves): by forward
  sensitivity of Eq. 8-10 one entry at a time, by the adjoint, and by central
  differences.
* The RC preprocessing of Eq. 2-3: Z_C = R - j/(w C), Gamma = (Z_C - Z0) /
  (Z_C + Z0), and dL/dC from the gradient with respect to Gamma.

Pins: tests/test_sparam_pins.py.
"""
from __future__ import annotations

import numpy as np

LOSS_MAG = 0
LOSS_COMPLEX = 1


def rc_reflection(R, C, omega, Z0: float = 50.0) -> np.ndarray:
    """Eq. 2 and Eq. 3 for each configuration, frequency and load:
    R [n], C [B][n], omega [F] -> Gamma [B][F][n]."""
    C = np.atleast_2d(C)
    w = np.atleast_1d(omega)[None, :, None]
    ZC = np.asarray(R)[None, None, :] - 1j / (w * C[:, None, :])
    return (ZC - Z0) / (ZC + Z0)


def rc_reflection_dC(R, C, omega, Z0: float = 50.0) -> np.ndarray:
    """dGamma/dC of Eq. 2-3: dGamma/dZ_C = 2 Z0 / (Z_C + Z0)^2 and
    dZ_C/dC = j / (w C^2); shape [B][F][n]."""
    C = np.atleast_2d(C)
    w = np.atleast_1d(omega)[None, :, None]
    Cb = C[:, None, :]
    ZC = np.asarray(R)[None, None, :] - 1j / (w * Cb)
    return 2.0 * Z0 / (ZC + Z0) ** 2 * (1j / (w * Cb * Cb))


def assemble_network(sc_const, values, idx_x, idx_y) -> np.ndarray:
    """S_C = S_C,var + S_C,const (Sec. III-A, steps 1-3).

    sc_const [F][N][N]; values [B][F][nvar]; idx_x, idx_y [nvar] (rows and
    columns of S_C,var; an index pair may repeat, its values then add).
    Returns S_C [B][F][N][N]."""
    sc_const = np.asarray(sc_const, dtype=np.complex128)
    values = np.asarray(values, dtype=np.complex128)
    B, F = values.shape[:2]
    N = sc_const.shape[-1]
    var = np.zeros((B, F, N, N), dtype=np.complex128)
    for e in range(len(idx_x)):
        var[:, :, idx_x[e], idx_y[e]] += values[:, :, e]
    return var + sc_const[None]


def combine(S0, fields, SC, n0: int, exc):
    """Eq. 6 and Eq. 7 for every (configuration, frequency).

    S0 [F][n0][n0]; fields [F][P][ncomp][n0]; SC [B][F][N][N]; exc [n1].
    Returns x [B][F][n0] (incident waves at the structure's ports) and
    B_comb [B][F][P][ncomp]."""
    S0 = np.asarray(S0, dtype=np.complex128)
    fields = np.asarray(fields, dtype=np.complex128)
    exc = np.asarray(exc, dtype=np.complex128)
    B, F = SC.shape[:2]
    P, ncomp = fields.shape[1:3]
    x = np.zeros((B, F, n0), dtype=np.complex128)
    Bc = np.zeros((B, F, P, ncomp), dtype=np.complex128)
    eye = np.eye(n0)
    for b in range(B):
        for f in range(F):
            S11 = SC[b, f, :n0, :n0]
            S12 = SC[b, f, :n0, n0:]
            A = eye - S11 @ S0[f]                      # A of Eq. 8
            X = np.linalg.solve(A, S12)                # Eq. 6
            x[b, f] = X @ exc
            Bc[b, f] = fields[f] @ x[b, f]             # Eq. 7
    return x, Bc


def loss(Bc, T, comp: int = 0, mode: int = LOSS_MAG) -> np.ndarray:
    """Per configuration: mean over (f, p) of (|B_comb| - T)^2 or |B_comb - T|^2
    on component `comp`."""
    v = Bc[..., comp]
    if mode == LOSS_MAG:
        e = (np.abs(v) - T[None, None, :]) ** 2
    else:
        e = np.abs(v - T[None, None, :]) ** 2
    return e.mean(axis=(1, 2))


def loss_weights(Bc, T, comp: int = 0, mode: int = LOSS_MAG) -> np.ndarray:
    """w = dL/dconj(B_comb) [B][F][P][ncomp]; zero off component `comp` and,
    in the magnitude mode, where |B| = 0."""
    F, P = Bc.shape[1], Bc.shape[2]
    v = Bc[..., comp]
    w = np.zeros_like(Bc)
    if mode == LOSS_MAG:
        a = np.abs(v)
        with np.errstate(invalid="ignore", divide="ignore"):
            wc = np.where(a > 0, (a - T[None, None, :]) * v / np.where(a > 0, a, 1.0), 0.0)
    else:
        wc = v - T[None, None, :]
    w[..., comp] = wc / (F * P)
    return w


def grad_forward_sensitivity(S0, fields, SC, n0, exc, idx_x, idx_y, T, comp=0,
                             mode=LOSS_MAG) -> np.ndarray:
    """2 dL/dconj(v_e) [B][F][nvar] by differentiating Eq. 6-7 with respect to
    one entry at a time (Eq. 8-10): with dS_C = E_(x_e, y_e),
    dx = A^-1 (dS_C11 S0 x + dS_C12 exc) and dB_comb = fields dx; then
    dL/dv_e = sum over (p, c) of conj(w) dB_comb, and the reported value is
    2 conj(dL/dv_e)."""
    S0 = np.asarray(S0, dtype=np.complex128)
    fields = np.asarray(fields, dtype=np.complex128)
    exc = np.asarray(exc, dtype=np.complex128)
    x, Bc = combine(S0, fields, SC, n0, exc)
    w = loss_weights(Bc, T, comp, mode)
    B, F = SC.shape[:2]
    nvar = len(idx_x)
    g = np.zeros((B, F, nvar), dtype=np.complex128)
    eye = np.eye(n0)
    for b in range(B):
        for f in range(F):
            A = eye - SC[b, f, :n0, :n0] @ S0[f]
            for e in range(nvar):
                r, c = idx_x[e], idx_y[e]
                if r >= n0:
                    continue  # S_C21 and S_C22 do not enter Eq. 6-7
                dS11 = np.zeros((n0, n0), dtype=np.complex128)
                dS12 = np.zeros((n0, len(exc)), dtype=np.complex128)
                if c < n0:
                    dS11[r, c] = 1.0
                else:
                    dS12[r, c - n0] = 1.0
                dx = np.linalg.solve(A, dS11 @ S0[f] @ x[b, f] + dS12 @ exc)  # Eq. 10
                dB = fields[f] @ dx
                dLdv = np.sum(np.conj(w[b, f]) * dB)
                g[b, f, e] = 2.0 * np.conj(dLdv)
    return g


def grad_adjoint(S0, fields, SC, n0, exc, idx_x, idx_y, T, comp=0, mode=LOSS_MAG) -> np.ndarray:
    """The same gradient through the adjoint: lam = A^-H (fields^H w) per
    system; 2 lam_x conj(exc_j) for an entry of S_C12 at (x, n0 + j),
    2 lam_x conj((S0 x)_y) for an entry of S_C11 at (x, y), 0 for S_C21 and
    S_C22."""
    S0 = np.asarray(S0, dtype=np.complex128)
    fields = np.asarray(fields, dtype=np.complex128)
    exc = np.asarray(exc, dtype=np.complex128)
    x, Bc = combine(S0, fields, SC, n0, exc)
    w = loss_weights(Bc, T, comp, mode)
    B, F = SC.shape[:2]
    nvar = len(idx_x)
    g = np.zeros((B, F, nvar), dtype=np.complex128)
    eye = np.eye(n0)
    for b in range(B):
        for f in range(F):
            A = eye - SC[b, f, :n0, :n0] @ S0[f]
            r = np.einsum("pck,pc->k", np.conj(fields[f]), w[b, f])
            lam = np.linalg.solve(A.conj().T, r)
            y = S0[f] @ x[b, f]
            for e in range(nvar):
                rr, cc = idx_x[e], idx_y[e]
                if rr >= n0:
                    continue
                if cc < n0:
                    g[b, f, e] = 2.0 * lam[rr] * np.conj(y[cc])
                else:
                    g[b, f, e] = 2.0 * lam[rr] * np.conj(exc[cc - n0])
    return g


def grad_fd(S0, fields, sc_const, values, idx_x, idx_y, n0, exc, T, comp=0, mode=LOSS_MAG,
            h: float = 1e-7) -> np.ndarray:
    """Central differences of the loss with respect to the real and imaginary
    part of every value; returns dL/dRe + j dL/dIm (= 2 dL/dconj(v))."""
    values = np.asarray(values, dtype=np.complex128)
    g = np.zeros_like(values)

    def L(vals):
        SC = assemble_network(sc_const, vals, idx_x, idx_y)
        return loss(combine(S0, fields, SC, n0, exc)[1], T, comp, mode)

    B, F, nvar = values.shape
    for f in range(F):
        for e in range(nvar):
            for part, unit in ((0, 1.0), (1, 1j)):
                d = np.zeros_like(values)
                d[:, f, e] = h * unit
                diff = (L(values + d) - L(values - d)) / (2 * h)
                if part == 0:
                    g[:, f, e] += diff
                else:
                    g[:, f, e] += 1j * diff
    return g


def rc_grad_C(g, R, C, omega, Z0: float = 50.0) -> np.ndarray:
    """dL/dC [B][n] from g = 2 dL/dconj(Gamma) [B][F][n] of the RC loads:
    dL/dC = sum over f of Re(conj(g) dGamma/dC) (Gamma is holomorphic in Z_C,
    and Z_C is a real-parameter function of C)."""
    return np.real(np.conj(g) * rc_reflection_dC(R, C, omega, Z0)).sum(axis=1)
