/*
 * cosim.h -- C ABI of the MI355X (gfx950) library for the capacitance -> B_z
 * map of reconfigurable resonant loop arrays and its gradient.
 *
 * The computed quantities follow the paper "Differentiable Cosimulator for
 * Electrically Reconfigurable Structures" (arXiv 2503.18479):
 *   - forward problem C -> B and the MSE inverse problem: Sec. II, Eq. 1;
 *   - RC load Z_C = R - j/(wC): Sec. III, Eq. 2; loop impedance
 *     Z = R + jwL - j/(wC) with L and mutual coupling M: Sec. IV-A, Eq. 11;
 *   - the quasi-static model "circuit model + Biot-Savart law": Sec. I-A;
 *   - the wave-ratio solve of Eq. 6 is used in its impedance form
 *     (R + jwM + 1/(jwC)) I = -jw Phi_ext, which reaches the same currents;
 *   - field superposition B = G I: Sec. III, Eq. 7 (z-component);
 *   - gradient through the solve, d(A^-1) = -A^-1 dA A^-1: Sec. III, Eq. 8-10.
 *
 * Conventions for every call:
 *   - Units are SI (m, F, ohm, rad/s, T).  Arrays are row-major.
 *   - Complex arrays are interleaved (re, im): complex128 = 2 doubles,
 *     complex64 = 2 floats, as torch.complex128 / torch.complex64 store them.
 *   - Pointers with the suffix _d are device pointers (HIP device memory of
 *     the device current when the plan was assembled); all others are host.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     of a call is enqueued on it; calls return without synchronising unless
 *     stated.
 *   - The caller owns every buffer it passes; the library never frees or
 *     keeps them past the call, and never writes to inputs.  The library owns
 *     the geometry and plan objects and the device memory inside a plan.
 *   - Return value: COSIM_OK (0) or a negative cosim_status.  Argument and
 *     shape errors are detected on the host before any device work is
 *     enqueued; cosim_last_error() then describes the problem.  Numerical
 *     trouble in one (configuration, frequency) system is not a call error:
 *     it sets bits in that system's status word and NaN outputs for it; the
 *     rest of the batch is unaffected.
 *   - Threading: geometry objects are immutable after creation and may be
 *     shared.  A plan may be used by one host thread and one stream at a time
 *     (its workspace is reused by every call).
 */
#ifndef COSIM_H
#define COSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum cosim_status {
    COSIM_OK = 0,
    COSIM_EINVAL = -1,       /* bad argument, shape or pointer */
    COSIM_ENOMEM = -2,       /* device or host allocation failed */
    COSIM_EDEVICE = -3,      /* a HIP runtime call failed */
    COSIM_EUNSUPPORTED = -4  /* valid request outside what this build implements */
};

/* Arithmetic used for the superposition B = G I and its adjoint G^T w.
 * Z, the solves, the loss reduction and the gradient are always FP64. */
enum cosim_precision {
    COSIM_FP64 = 0,   /* FP64 matrix cores (v_mfma_f64) */
    COSIM_FP32 = 1,   /* FP32 matrix cores, FP32 accumulation */
    COSIM_BF16X3 = 2  /* bf16 hi/lo split of both operands, 3 products, FP32 accumulation */
};

/* Masks of precisions for cosim_assemble_ex: bit (1 << precision). */
enum { COSIM_PREC_ALL = (1 << COSIM_FP64) | (1 << COSIM_FP32) | (1 << COSIM_BF16X3) };

/* Loss of Eq. 1 per configuration b, mean over frequencies f and points p:
 *   MAG:     L_b = 1/(F P) sum_{f,p} (|B_z| - T_p)^2   (magnitude targets)
 *   COMPLEX: L_b = 1/(F P) sum_{f,p} |B_z - T_p|^2                          */
enum cosim_loss {
    COSIM_LOSS_MAG = 0,      /* mean over (f, p) of (|B_z| - T_p)^2 (Eq. 1 on magnitudes) */
    COSIM_LOSS_COMPLEX = 1,  /* mean of |B_z - T_p|^2 */
    COSIM_LOSS_RATIO = 2     /* enhancement factor of Sec. IV-B: beta = |bext_z + B_z| / |bext_z|
                                (the total field over the incident one), mean of (beta - T_p)^2
                                with T_p the target factors; needs bext_z != 0 at assembly */
};

/* Per-system status bits written to status_d[b*F + f]. */
enum cosim_sys_status {
    COSIM_SYS_BAD_INPUT = 1,  /* C_k zero or NaN, or omega zero or not finite (outputs NaN);
                                 C_k = +INFINITY is a loop without a capacitor */
    COSIM_SYS_SINGULAR = 2,   /* zero pivot in the elimination (outputs NaN) */
    COSIM_SYS_NONFINITE = 4,  /* result not finite */
    COSIM_SYS_NEGATIVE_C = 8  /* some C_k < 0: accepted (the feasible set is unbounded), flagged */
};

typedef struct cosim_geom *cosim_geom_t;
typedef struct cosim_plan *cosim_plan_t;

/* Human-readable description of the last error on the calling thread. */
const char *cosim_last_error(void);

/* Library ABI version (currently 1). */
int cosim_version(void);

/* --------------------------------------------------------------------------
 * Geometry: n_loops closed polygonal wire loops, one tunable capacitor each.
 *   seg_off [n_loops+1] int32: loop k owns vertices seg_off[k]..seg_off[k+1]-1
 *                       (seg_off[0] = 0, each loop >= 3 vertices);
 *   verts   [V][3] double: vertices, V = seg_off[n_loops]; segment s of loop
 *                       k joins vertex s to s+1 and the last vertex back to
 *                       the first.  Positive loop current circulates in vertex
 *                       order (counter-clockwise seen from +z gives +B_z
 *                       inside the loop);
 *   wire_a  [n_loops] double > 0: wire radius (regularises the self term);
 *   R       [n_loops] double >= 0: series resistance of each loop's RC load
 *                       (Eq. 2).
 * All inputs are host memory and are copied.  Loops may not touch each other.
 * -------------------------------------------------------------------------- */
int cosim_geometry_create(int n_loops, const int32_t *seg_off, const double *verts,
                          const double *wire_a, const double *R, cosim_geom_t *out);
int cosim_geometry_destroy(cosim_geom_t g);
/* Loop count and total vertex count. */
int cosim_geometry_size(cosim_geom_t g, int *n_loops, int *n_verts);

/* --------------------------------------------------------------------------
 * Assembly (once per geometry and point set).  Runs on the current device:
 *   G[p][k]  z-field at point p per ampere in loop k (Biot-Savart law,
 *            closed form per straight segment), stored FP64 and rounded to
 *            FP32 and to bf16 hi/lo for the mixed-precision modes;
 *   M[k][l]  Neumann mutual inductance between loop axes (k != l); the
 *            diagonal uses the reduced kernel 1/sqrt(|r-r'|^2 + a_k^2)
 *            (thin-wire surface-current self inductance);
 *   Phi[k]   flux of the uniform incident field bext_z through loop k.
 * pts_d [P][3] double, device.  P >= 1.  Synchronises `stream` before return.
 * The plan keeps its own copies; pts_d may be freed afterwards.
 * -------------------------------------------------------------------------- */
int cosim_assemble(cosim_geom_t g, int P, const double *pts_d, double bext_z, void *stream,
                   cosim_plan_t *out);
/* The same, keeping only the copies of G that the precisions in the mask
 * `precisions` (bits 1 << COSIM_FP64 / FP32 / BF16X3, non-empty subset of
 * COSIM_PREC_ALL) need: 16, 8 and 8 bytes per entry of G (each precision keeps
 * G and its transpose).  Calls that read a missing copy return COSIM_EINVAL:
 * cosim_loss_and_grad, cosim_field, cosim_field_backward and
 * cosim_plan_autotune in a precision outside the mask, and cosim_plan_copy_G
 * without the FP64 bit.  For many plans at once (independent instances). */
int cosim_assemble_ex(cosim_geom_t g, int P, const double *pts_d, double bext_z, int precisions,
                      void *stream, cosim_plan_t *out);
/* The same with G holding another Cartesian component of the field
 * (Sec. I-B: all three components are available): component 0 = B_x,
 * 1 = B_y, 2 = B_z (what cosim_assemble_ex builds).  Everything below that
 * reads G (fields, losses, gradients) then works on that component; to
 * shape several components, use one plan per component with the same
 * geometry, points and excitation.  COSIM_LOSS_RATIO needs component 2.
 * Errors: those of cosim_assemble_ex; COSIM_EINVAL for a component outside 0..2. */
int cosim_assemble_component(cosim_geom_t g, int P, const double *pts_d, double bext_z,
                             int precisions, int component, void *stream, cosim_plan_t *out);
int cosim_plan_destroy(cosim_plan_t p);
/* Loops n, points P of a plan. */
int cosim_plan_size(cosim_plan_t p, int *n_loops, int *n_points);
/* Number of batches whose impedance matrices the plan's calls have
 * factorised so far (cosim_solve, cosim_loss_and_grad and its variants, one
 * per instance of cosim_loss_and_grad_many, cosim_field_backward with
 * reuse = 0); a cosim_field_backward that replays a record adds none. */
int cosim_plan_factorisations(cosim_plan_t p, long long *count);
/* Pre-allocate the workspace for batches up to max_batch configurations of
 * max_freq frequencies, so that later calls with B*F <= max_batch*max_freq
 * allocate nothing.  Calls that need more grow the workspace themselves. */
int cosim_plan_reserve(cosim_plan_t p, int max_batch, int max_freq);
/* Copies of the assembled operators, for inspection and testing.
 * G_d: device [P][n] double.  M: host [n][n] double.  phi: host [n] double. */
int cosim_plan_copy_G(cosim_plan_t p, double *G_d, void *stream);
int cosim_plan_copy_M(cosim_plan_t p, double *M);
int cosim_plan_copy_phi(cosim_plan_t p, double *phi);

/* --------------------------------------------------------------------------
 * Driven ports (Sec. III, Eq. 4; the excitation coil of Sec. IV-A).  A port
 * in series with loop loop[i] is fed by an excitation that sends the voltage
 * wave sqrt(z0 power[i]) exp(j phase[i]) toward it through the characteristic
 * impedance z0 (the paper takes 1 W and 50 ohm).  In the loop equations that
 * source is its Thevenin equivalent: z0 is added to the loop's series
 * resistance and the EMF E = 2 sqrt(z0 power[i]) exp(j phase[i]) to its
 * voltage, so every solve below becomes
 *     (diag(R + z0 [driven]) + j w M + diag(1/(j w C))) I = E - j w Phi.
 * E does not depend on w.  A driven coil without a capacitor passes
 * C = +INFINITY for its loop (the short-circuit limit; its gradient is 0).
 *   nport 0..n (0 removes all ports); loop [nport] host int32, distinct loops;
 *   power [nport] host double >= 0 (watts); phase [nport] host double
 *   (radians) or NULL for 0; z0 > 0 (ohms; ignored when nport = 0).
 * Replaces the previous port set.  Parameter gradients with respect to R
 * (cosim_loss_and_grad_params) are then taken with respect to the loop's
 * total series resistance.  Synchronises `stream`.  Errors: COSIM_EINVAL. */
int cosim_plan_set_drive(cosim_plan_t p, int nport, const int32_t *loop, const double *power,
                         const double *phase, double z0, void *stream);

/* --------------------------------------------------------------------------
 * FP32 factorisation with FP64 iterative refinement for plans of more than
 * 64 loops whose every series resistance is > 0 (the blocked LDL^T path; the
 * pivoted paths and plans of up to 64 loops stay FP64 and ignore this).
 * With enable != 0 every call that solves (cosim_solve, cosim_field_backward,
 * cosim_loss_and_grad and cosim_loss_and_grad_params, forward and adjoint)
 * factors Z in complex64 on FP32 matrix cores and refines each solution in
 * FP64: x = F^-1 b, then r = b - Z x with Z formed in FP64 from M, R, C and
 * w, x += F^-1 r, until the error left (estimated from the geometric
 * shrinking of the corrections) is at most tol |x| in the max norm.  A system
 * that is not done after max_iter steps (or whose FP32 pivot is small) gets
 * the pivoted FP64 factorisation instead, so results keep the accuracy of
 * the FP64 path whatever the conditioning.
 *   max_iter 1..64; tol in [0, 1): 0 chooses it from the precision of the
 *   call's contraction (FP64 1e-12, FP32 1e-9, BF16X3 1e-7; cosim_solve and
 *   cosim_field_backward 1e-12).
 * Changing the mode keeps the plan's workspace: enabling adds 8 NP^2 bytes
 * per reserved system for the FP32 factor at the next call that needs them
 * (or at cosim_plan_reserve), beside the buffers already there, so HIP graphs
 * captured before stay valid and replay the mode they were captured in.  The
 * call itself enqueues and allocates nothing.  Errors: COSIM_EINVAL. */
int cosim_plan_set_refinement(cosim_plan_t p, int enable, int max_iter, double tol);

/* --------------------------------------------------------------------------
 * Currents (Eq. 6 in impedance form).  For every configuration b < B and
 * frequency f < F solves
 *     (diag(R) + j w_f M + diag(1/(j w_f C_b))) I_{b,f} = E - j w_f Phi
 * (E: the EMF of driven ports, zero unless cosim_plan_set_drive set some;
 * C = +INFINITY is a loop without a capacitor) in FP64: up to 64 loops by a
 * complex-symmetric LDL^T on FP64 matrix cores (every R_k > 0) with pivoted
 * Gauss-Jordan elimination for systems with a small pivot, or pivoted
 * Gauss-Jordan throughout (some R_k = 0); above 64 loops by a blocked LDL^T
 * (or, with cosim_plan_set_refinement, its FP32 form refined in FP64) with
 * pivoted LU for systems with a small pivot, or pivoted LU throughout.
 * The factorisation is recorded in the plan's workspace, with the status of
 * every system, for cosim_field_backward with reuse != 0; the record lasts
 * until another call uses the workspace (cosim_loss_and_grad, _params,
 * _many, cosim_plan_autotune, cosim_field_backward with reuse = 0,
 * cosim_plan_set_drive, cosim_plan_set_refinement, or a larger cosim_solve).
 * Grows the workspace (allocates) when B*F systems need more room.
 *   C_d      [B][n] double, device (farads)
 *   omega_d  [F] double, device (rad/s)
 *   I_d      [B][F][n] complex128, device (output, amperes)
 *   status_d [B][F] int32, device (output, cosim_sys_status bits)
 * -------------------------------------------------------------------------- */
int cosim_solve(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                double *I_d, int32_t *status_d, void *stream);

/* Field superposition B_z[b][f][p] = sum_k G[p][k] I[b][f][k] (Eq. 7) on the
 * matrix cores in `precision` (the plan must hold that copy of G), plus the
 * incident field bext_z when add_incident != 0 (the total field of the
 * forward problem, Sec. II; z-component plans only).
 *   I_d  [B][F][n] complex128, device
 *   Bz_d [B][F][P] complex128 (precision FP64) or complex64 (FP32, BF16X3),
 *        device, output.
 * Allocates nothing.                                                          */
int cosim_field(cosim_plan_t p, int B, int F, const double *I_d, int precision, int add_incident,
                void *Bz_d, void *stream);

/* Vector-Jacobian product of C -> B_z (Eq. 8-10 through the adjoint solve).
 *   gBz_d  [B][F][P] complex128, device: upstream gradient in PyTorch's
 *          convention for a real loss L, gBz = dL/dRe(B) + j dL/dIm(B)
 *          (= 2 dL/d conj(B)); an added incident field does not change it;
 *   precision  arithmetic of the contraction r = G^T conj(gBz) / 2 on the
 *          matrix cores (the plan must hold that copy of G); the solve and
 *          the gradient are FP64;
 *   reuse  != 0: the adjoint solve Z^T mu = r replays the factor record of
 *          the plan's last cosim_solve (Z is complex symmetric, so the
 *          forward factorisation serves Z^T), which must be of the same B
 *          and F and still intact (see cosim_solve), else COSIM_EINVAL;
 *          C_d, omega_d and I_d must be that solve's.  0: Z is factorised
 *          again (and any record is lost);
 *   gC_d   [B][n] double, device, output: dL/dC;
 *   status_d [B][F] int32, device, output: the system status (with reuse,
 *          that of the recorded solve plus COSIM_SYS_NONFINITE if mu is not
 *          finite).
 * With reuse = 0 the workspace grows (allocates) when B*F systems need more
 * room. */
int cosim_field_backward(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                         const double *I_d, const double *gBz_d, int precision, int reuse,
                         double *gC_d, int32_t *status_d, void *stream);

/* Fused forward + loss + gradient (the optimisation step's evaluation).
 *   T_d      [P] double, device: target field magnitudes (tesla)
 *   loss_d   [B] double, device, output: L_b of `loss_mode`
 *   grad_d   [B][n] double, device, output: dL_b/dC_b (may be NULL: loss only)
 *   status_d [B][F] int32, device, output
 * B_z is formed in registers tile by tile and never written to memory; the
 * adjoint contraction G^T conj(w) shares each G tile with the forward
 * product.  Solves and reductions are FP64; `precision` selects the matrix
 * core arithmetic of the two contractions.  Deterministic: no atomics.
 * Once the workspace covers B*F systems (cosim_plan_reserve, or an earlier
 * call of that size) the call only enqueues kernels on `stream`: no
 * allocation, memset, copy or synchronisation, so it can be captured in a HIP
 * graph (phase timing, when switched on, adds event records). */
int cosim_loss_and_grad(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                        const double *T_d, int loss_mode, int precision, double *loss_d,
                        double *grad_d, int32_t *status_d, void *stream);

/* cosim_loss_and_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same results (bit for bit), but the call's
 * device buffers -- currents, factor records, partial sums and per-system
 * gradient terms -- live in a library-owned device array of
 * cosim_noalloc_scratch_bytes() bytes (64 MiB) per device instead of the
 * plan's workspace, so the call never allocates, frees or reserves memory
 * and leaves the plan's workspace untouched.  The array is taken on a
 * device's first call and held until the process ends.  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.  The array
 * keeps the last call's contents; nothing in it needs to start at zero.
 * Plans of at most 64 loops (else COSIM_EUNSUPPORTED).  A call whose
 * buffers do not fit -- about 16 NP^2 + 16 NP nchunk + 40 NP bytes per
 * system with NP = 32 or 64 the padded loop count and nchunk the P-chunks of
 * the fused contraction, i.e. several hundred 64-loop systems -- returns
 * COSIM_EINVAL naming the size.  No phase timing. */
int cosim_loss_and_grad_noalloc(cosim_plan_t p, int B, int F, const double *C_d,
                                const double *omega_d, const double *T_d, int loss_mode,
                                int precision, double *loss_d, double *grad_d, int32_t *status_d,
                                void *stream);
/* Bytes of the per-device array behind cosim_loss_and_grad_noalloc. */
size_t cosim_noalloc_scratch_bytes(void);

/* Loss, dL/dC and the gradients with respect to the other circuit variables of
 * Fig. 2 / Eq. 11, for the same call as cosim_loss_and_grad (which it runs):
 *   gR_d     [B][n] or NULL: dL_b/dR_k = -2 sum_f Re(mu_k I_k);
 *   gL_d     [B][n] or NULL: dL_b/dL_k of a series inductance added to loop k
 *            (Z_kk += j w L_k), 2 sum_f w Im(mu_k I_k);
 *   gomega_d [B][F] or NULL: dL_b/dw_f = 2 [Im(mu^T Phi) + Im(mu^T M I)
 *            + sum_k Im(mu_k I_k) / (w^2 C_k)] (V = E - j w Phi and Z both
 *            depend on w; G and the EMF E of driven ports do not);
 * with mu the adjoint solution of each system (Z mu = G^T conj(w), Eq. 8-10;
 * Z is complex symmetric).  gC_d is required (the adjoint always runs).
 * Allocates a [S][n] workspace for mu on first use at a new size.  Systems with
 * status bits get NaN terms, as in cosim_loss_and_grad. */
int cosim_loss_and_grad_params(cosim_plan_t plan, int B, int F, const double *C_d,
                               const double *omega_d, const double *T_d, int loss_mode,
                               int precision, double *loss_d, double *gC_d, double *gR_d,
                               double *gL_d, double *gomega_d, int32_t *status_d, void *stream);

/* Resonance capacitance of Eq. 13, C_r = 1 / (w^2 (L + M)), per frequency and
 * loop: Cr_d [F][n] from omega_d [F].  L_k = M_kk; coupled != 0 adds the loop's
 * mutual inductances to all others (the array resonance with equal currents),
 * coupled = 0 neglects them (the single-cell case of Sec. IV-A). */
int cosim_resonant_capacitance(cosim_plan_t plan, int F, const double *omega_d, int coupled,
                               double *Cr_d, void *stream);

/* Bounded projection of the capacitances (Sec. V): for count elements,
 * C = cmin + (cmax - cmin) (1 + tanh(theta)) / 2 and, if dC_d is not NULL,
 * dC/dtheta = (cmax - cmin) (1 - tanh^2(theta)) / 2 (the chain rule factor).
 * Requires cmin < cmax, both finite. */
int cosim_tanh_projection(int64_t count, const double *theta_d, double cmin, double cmax,
                          double *C_d, double *dC_d, void *stream);

/* Clipping in place to [lo, hi] (Sec. V: a wide range and clipping in place of a
 * bounded projection).  Requires lo <= hi. */
int cosim_clip(int64_t count, double *x_d, double lo, double hi, void *stream);

/* One Adam step on the capacitances, the optimiser the paper runs on C
 * (Sec. IV; learning rate 1e-13 F there), with the bias-corrected moments of
 * Kingma & Ba: with t the 1-based step and g = dL/dC,
 *   m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
 *   C <- C - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 *   count    number of elements (B*n for a batch of configurations); 0 is a no-op
 *   C_d      [count] double, device, updated in place
 *   grad_d   [count] double, device (e.g. grad_d of cosim_loss_and_grad)
 *   m_d, v_d [count] double, device: moments, zero before the first step,
 *            updated in place (caller-owned)
 *   step_d   [1] int32, device: steps taken so far (0 before the first step);
 *            read as t - 1 and advanced by one
 * Requires 0 <= beta1, beta2 < 1, finite lr and eps >= 0 (else COSIM_EINVAL).
 * Enqueues two kernels on `stream` and nothing else; together with a reserved
 * cosim_loss_and_grad it can be captured in one HIP graph and replayed for
 * any number of steps, since t is read from device memory. */
int cosim_adam_step(int count, double *C_d, const double *grad_d, double *m_d, double *v_d,
                    int32_t *step_d, double lr, double beta1, double beta2, double eps,
                    void *stream);

/* cosim_loss_and_grad over `count` independent instances (own geometry,
 * points, targets, batch and frequencies; e.g. unevenly sized arrays).  Host
 * arrays of `count` entries: plans[i] (each plan at most once), B[i], F[i],
 * and the device pointers of instance i with the meaning and shapes of
 * cosim_loss_and_grad (grad_d may be NULL for loss only, or hold NULL
 * entries).  Every instance is validated before anything is enqueued; an
 * error names the instance.  The instances run on 16 library-owned side
 * streams (default priority; the largest instances first, each to the stream
 * with the least work so far) that wait for `stream` and that `stream` waits
 * for when the call returns, so the work is ordered on `stream` as one
 * operation and can be captured with it.  Each plan's own workspace is used:
 * reserve every plan beforehand.
 * Outside stream capture, instances with every R_k > 0 (no refinement, no
 * phase timing) that share a padded loop count are factored and solved in
 * shared launches (up to 24 per launch for 64 loops or fewer, 32 above), and
 * their final sums run in one launch per group; their results equal their
 * own calls bit for bit.  Above 64 loops their factor records live in a
 * library-owned workspace per device, grown (after a device
 * synchronisation) when a call needs more, so the first such call, or a
 * larger one, allocates.  Calls on
 * one device may overlap (other streams, other host threads): the enqueueing
 * is serialised, and the side streams of a call that groups instances wait
 * for the previous such call to finish.  Under capture, instances of 64
 * loops or fewer are grouped as outside it; instances above 64 loops run on
 * their own and the shared workspace is not touched. */
int cosim_loss_and_grad_many(int count, const cosim_plan_t *plans, const int *B, const int *F,
                             const double *const *C_d, const double *const *omega_d,
                             const double *const *T_d, int loss_mode, int precision,
                             double *const *loss_d, double *const *grad_d,
                             int32_t *const *status_d, void *stream);

/* --------------------------------------------------------------------------
 * Tuning of the fused contraction (performance only; every variant computes
 * the same quantities to the precision's tolerance).  A variant fixes the
 * systems per wavefront and the field points per LDS tile.
 * cosim_plan_set_variant / cosim_plan_get_variant select or read the variant
 * used for `precision` (0 is the default; n_variants receives the count).
 * cosim_plan_autotune runs cosim_loss_and_grad reps times (after one warm-up)
 * with every variant on the given inputs, keeps the fastest for `precision`,
 * and writes the mean milliseconds per call of each variant to ms_out (host,
 * n_variants entries; may be NULL).  It allocates and frees its own scratch
 * and synchronises `stream`; it is a set-up call, not a hot one.
 * -------------------------------------------------------------------------- */
int cosim_plan_set_variant(cosim_plan_t p, int precision, int variant);
int cosim_plan_get_variant(cosim_plan_t p, int precision, int *variant, int *n_variants);
int cosim_plan_autotune(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                        const double *T_d, int loss_mode, int precision, int reps, void *stream,
                        double *ms_out);

/* --------------------------------------------------------------------------
 * Phase timing of cosim_loss_and_grad with HIP events on the call's stream
 * (for benchmarks and metrics; not a paper quantity).
 * cosim_plan_timing(p, max_records) creates event sets for the next
 * max_records calls of cosim_loss_and_grad (0 switches timing off and frees
 * them); each of those calls records its phase boundaries.
 * cosim_plan_timing_read waits for the recorded calls and writes, per call,
 * COSIM_PHASES durations in milliseconds to ms[record][phase]:
 *   0 forward solve, 1 fused contraction (B = G I, loss, G^T w),
 *   2 adjoint solve, 3 reductions.
 * *n_records receives the number of calls recorded; recording restarts at 0.
 * -------------------------------------------------------------------------- */
enum { COSIM_PHASES = 4 };
int cosim_plan_timing(cosim_plan_t p, int max_records);
int cosim_plan_timing_read(cosim_plan_t p, double *ms, int max_records, int *n_records);

#ifdef __cplusplus
}
#endif

#endif /* COSIM_H */
