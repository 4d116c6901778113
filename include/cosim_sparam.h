/*
 * cosim_sparam.h -- C ABI of the S-parameter cosimulation pipeline of
 * "Differentiable Cosimulator for Electrically Reconfigurable Structures"
 * (arXiv 2503.18479), Sec. III and III-A, on MI355X (gfx950).
 *
 * A resonant structure with n0 ports is described per frequency by exports
 * of a full-wave simulation: its scattering matrix S0 and the field each port
 * produces for a unit incident voltage wave with the other ports matched
 * (the paper's (n_points, 3, n0) field tensor).  A connecting network S_C of
 * (n0 + n1) ports joins it to n1 external ports (Fig. 1); its blocks are
 * S_C11 = S_C[:n0, :n0] and S_C12 = S_C[:n0, n0:].  S_C = S_C,const + S_C,var,
 * where S_C,var is zero except at user-chosen (row, column) index pairs that
 * receive the values of a user-defined preprocessing step (Sec. III-A,
 * steps 1-3; an index pair may repeat, its values then add).
 *
 * Per configuration b and frequency f (system s = b F + f):
 *   A = I - S_C11 S0                               (Eq. 6, A of Eq. 8)
 *   x = A^-1 S_C12 exc                             (Eq. 6, incident waves at the
 *                                                   structure for the external
 *                                                   drive waves exc, Eq. 4)
 *   B_comb[p][c] = sum_k fields[p][c][k] x_k       (Eq. 7)
 *   L_b = mean over (f, p) of (|B_comb[p][comp]| - T_p)^2   (Eq. 1 on
 *         magnitudes; or |B_comb[p][comp] - T_p|^2 in the complex mode)
 *   gradient of L with respect to every variable value (Eq. 8-10), reported
 *   as 2 dL/dconj(v) (PyTorch's convention for complex leaves): for an entry of
 *   S_C12 at (r, n0 + j) it is 2 lam_r conj(exc_j), for an entry of S_C11 at
 *   (r, c) it is 2 lam_r conj((S0 x)_c), with A^H lam = fields^H w and
 *   w = dL/dconj(B_comb); entries in S_C21 and S_C22 do not enter Eq. 6-7 and
 *   get 0.
 * The RC preprocessing of Eq. 2-3 (Gamma = (Z_C - Z0)/(Z_C + Z0),
 * Z_C = R - j/(w C)) and its chain rule to dL/dC are provided as calls.
 *
 * Conventions are those of cosim.h: SI units, row-major arrays, complex
 * values interleaved (re, im) as torch.complex128 stores them, device
 * pointers with the suffix _d, host pointers otherwise, every call enqueued on
 * `stream` (a hipStream_t), argument errors reported before any device work
 * (cosim_last_error()), numerical trouble per system in status bits
 * (COSIM_SYS_SINGULAR: a zero pivot; COSIM_SYS_NONFINITE: a non-finite
 * result) with NaN outputs for that system.  The caller owns every buffer it
 * passes; a plan copies what it needs at creation and owns its device memory.
 * A plan is used by one host thread and one stream at a time.
 */
#ifndef COSIM_SPARAM_H
#define COSIM_SPARAM_H

#include <stdint.h>

#include "cosim.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { COSIM_SP_MAX_PORTS = 64, COSIM_SP_MAX_EXTERNAL = 8 };

typedef struct cosim_sp *cosim_sp_t;

/* Creates a plan and copies the exports to it (stream-ordered on `stream`).
 *   n0: 1..COSIM_SP_MAX_PORTS ports of the structure; n1: 1..COSIM_SP_MAX_EXTERNAL
 *   external ports; F >= 1 frequencies; P >= 1 points; ncomp 1..3 field components.
 *   S0_d       [F][n0][n0] complex128
 *   fields_d   [F][P][ncomp][n0] complex128
 *   sc_const_d [F][N][N] complex128, N = n0 + n1; NULL means zero
 *   idx_x, idx_y [nvar] host int32: row and column in S_C of each variable value,
 *              0 <= index < N; nvar may be 0
 *   exc        [n1] host complex128: drive waves of the external ports (for one
 *              port fed with power P behind Z'_exc, sqrt(Z'_exc P), Eq. 4)
 *   precisions bit mask (1 << COSIM_FP64) | (1 << COSIM_FP32): contraction
 *              precisions the plan keeps field copies for (COSIM_BF16X3 is not
 *              offered here: COSIM_EUNSUPPORTED)
 * Allocates the plan's device memory.  Errors: COSIM_EINVAL for shapes, indices or
 * pointers, COSIM_ENOMEM, COSIM_EDEVICE. */
int cosim_sp_create(int n0, int n1, int F, int P, int ncomp, const double *S0_d,
                    const double *fields_d, const double *sc_const_d, int nvar,
                    const int32_t *idx_x, const int32_t *idx_y, const double *exc,
                    int precisions, void *stream, cosim_sp_t *out);

/* Waits for the plan's work on its last stream and frees it.  NULL is accepted. */
int cosim_sp_destroy(cosim_sp_t plan);

/* Reserves the workspace for up to max_batch configurations (allocates; the
 * field and loss calls allocate on first use otherwise). */
int cosim_sp_reserve(cosim_sp_t plan, int max_batch);

/* Forward pipeline for B >= 0 configurations.
 *   values_d [B][F][nvar] complex128: the preprocessing output
 *   x_d      [B][F][n0] complex128 or NULL: incident waves at the structure
 *   field_d  [B][F][P][ncomp] complex128 or NULL: B_comb of Eq. 7 (FP64)
 *   status_d [B][F] int32 */
int cosim_sp_field(cosim_sp_t plan, int B, const double *values_d, double *x_d, double *field_d,
                   int32_t *status_d, void *stream);

/* Loss and gradient for B >= 0 configurations without materialising B_comb.
 *   T_d [P] target (magnitudes, or real targets in the complex mode);
 *   comp: field component of the loss (0..ncomp-1); loss_mode COSIM_LOSS_MAG or
 *   COSIM_LOSS_COMPLEX; precision COSIM_FP64 or COSIM_FP32 (of the two
 *   contractions; the solves and reductions are FP64), one the plan kept.
 *   loss_d [B]; grad_d [B][F][nvar] complex128 (2 dL/dconj(v)) or NULL;
 *   status_d [B][F]. */
int cosim_sp_loss_and_grad(cosim_sp_t plan, int B, const double *values_d, const double *T_d,
                           int comp, int loss_mode, int precision, double *loss_d, double *grad_d,
                           int32_t *status_d, void *stream);

/* RC preprocessing, Eq. 2 and Eq. 3, for B >= 0 configurations of n >= 1 loads:
 *   gamma[(b F + f) ld + k] = (Z_C - z0) / (Z_C + z0), Z_C = R_k - j / (w_f C_bk).
 *   R_d [n], C_d [B][n], omega_d [F], gamma_d complex128 with row stride ld >= n
 *   (complex elements), so that the reflections can fill the first n values of
 *   a [B][F][nvar] array. */
int cosim_sp_rc(int B, int F, int n, const double *R_d, const double *C_d, const double *omega_d,
                double z0, double *gamma_d, int ld, void *stream);

/* Chain rule of the RC preprocessing: from g = 2 dL/dconj(Gamma) (row stride ld,
 * as written by cosim_sp_loss_and_grad for the first n values),
 *   gC[b][k] = sum over f of Re(conj(g) dGamma/dC),
 *   dGamma/dC = 2 z0 / (Z_C + z0)^2 * j / (w C^2)  (summed in fixed order). */
int cosim_sp_rc_backward(int B, int F, int n, const double *R_d, const double *C_d,
                         const double *omega_d, double z0, const double *g_d, int ld, double *gC_d,
                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* COSIM_SPARAM_H */
