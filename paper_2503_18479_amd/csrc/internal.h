// Internal declarations shared by the host entry points and the HIP kernels
// of libcosim.  Not part of the public ABI (see include/cosim.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "cosim.h"

namespace cosim {

// Vacuum permeability, CODATA 2018 (N/A^2), and mu0/(4 pi).
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kMu0Over4Pi = kMu0 / (4.0 * 3.14159265358979323846);

// Gauss-Legendre rule used for the outer integral of non-parallel segment
// pairs in the Neumann assembly (inner integral is closed form).
constexpr int kGLOrder = 16;

struct GLRule {
    double x[kGLOrder];  // nodes on [-1, 1]
    double w[kGLOrder];  // weights
};

// Loop excitation on the device, [3][n] doubles: the flux Phi_k of the
// uniform incident field, then Re and Im of a source EMF E_k in series with
// the loop (a driven port; zero elsewhere).  The loop voltage is
// V_k = E_k - j w Phi_k.
__device__ inline double2 loop_voltage(const double *exc, int n, int k, double w) {
    return make_double2(exc[n + k], exc[2 * n + k] - w * exc[k]);
}

// Matrix-core precision of the superposition (mirrors cosim_precision).
enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };

// Padded loop dimension used by the solver and the contraction kernels:
// 32 or 64 for the register-resident (fused) path (the bf16 matrix-core
// product needs K = 32), a multiple of 64 above.
constexpr int kMaxLoops = 64;       // largest loop count of the fused path
constexpr int kMaxLoopsBig = 1024;  // largest loop count of this build
inline int padded_loops(int n) {
    return n <= 32 ? 32 : (n + 63) / 64 * 64;
}
inline bool big_plan(int NP) { return NP > kMaxLoops; }
constexpr int kPTile = 64;          // rows of G per LDS tile in the fused kernels, and the
                                    // padding of P in every plan

// ---------------------------------------------------------------------------
// kernel launchers (implemented in the .hip files); all return hipError_t
// ---------------------------------------------------------------------------
// G of Cartesian component `comp` at P points into the non-null copies:
// [P_pad][NP] FP64 / FP32 / bf16 hi and lo, and the transposed [NP][P_pad]
// copies of each (rows p >= P and columns k >= n are zero).
hipError_t launch_assemble_G(int n, int NP, int P, int P_pad, int comp, const int32_t *seg_off_d,
                             const double *verts_d, const double *pts_d, double *G64,
                             float *G32, uint16_t *Ghi, uint16_t *Glo, double *GT64,
                             float *GT32, uint16_t *GThi, uint16_t *GTlo, hipStream_t st);

hipError_t launch_assemble_M(int n, const int32_t *seg_off_d, const double *verts_d,
                             const double *wire_a_d, const GLRule &gl, double *M_d,
                             hipStream_t st);

// Record of a factorisation, per system s, in one of two formats (fmt[s]):
//   kFmtLDL: strictly lower part of Z = L D L^T packed by columns inside the
//            system's NP*NP slot: L_ik (i > k) at L[s*NP*NP + ldl_col(NP, k) +
//            i - k - 1]; piv_val[s][k] = 1/d_k;
//   kFmtGJ : L[s][k][i] = multiplier of Gauss-Jordan step k for row i,
//            piv_row[s][k] = pivot row, piv_val[s][k] = pivot value.
struct GJFactor {
    double2 *L = nullptr;
    int *piv_row = nullptr;
    double2 *piv_val = nullptr;
    int *fmt = nullptr;
};
constexpr int kFmtLDL = 0, kFmtGJ = 1, kFmtNeedsPivot = 2;
// above 64 loops with refinement on: the FP32 record did not converge in the
// forward (or only in the adjoint) solve, so the system holds a pivoted FP64 record
constexpr int kFmtRefineFailed = 3, kFmtRefineFailedAdj = 4;
// first element of column k in the packed LDL^T record (columns of NP - 1 - k)
__host__ __device__ constexpr int ldl_col(int NP, int k) { return k * (2 * NP - k - 1) / 2; }
constexpr int kFlagPivot = 1 << 16;  // kernel-internal status bit, never returned

// LDL^T fast path (all R_k > 0): factorises, records and solves,
// I = Z^-1 (E - j w Phi) in I_d; marks systems that need pivoting
// (fmt = kFmtNeedsPivot, I_d left for it) for launch_solve_fallback.
hipError_t launch_ldl(int NP, int n, int S, int F, const double *M_d, const double *R_d,
                      const double *C_d, const double *omega_d, const double *phi_d, GJFactor fac,
                      double2 *I_d, int32_t *status_d, hipStream_t st);
// Pivoted Gauss-Jordan for the marked systems only (writes I and a kFmtGJ record).
hipError_t launch_solve_fallback(int NP, int n, int S, int F, const double *M_d,
                                 const double *R_d, const double *phi_d, const double *C_d,
                                 const double *omega_d, double2 *I_d, int32_t *status_d,
                                 GJFactor fac, hipStream_t st);
// Adjoint solve from the record and the per-system gradient terms.
// mu_d (optional, [S][n]): the adjoint solution itself.
hipError_t launch_replay_adjoint(int NP, int n, int S, int F, GJFactor fac, const double *C_d,
                                 const double *omega_d, double2 *I_d, const double2 *rpart_d,
                                 int nchunk, double rscale, double *gsys_d, double2 *mu_d,
                                 int32_t *status_d, hipStream_t st);

// Forward solve by pivoted Gauss-Jordan: Z I = E - j w Phi for S = B*F systems
// (s = b*F + f); records the elimination (kFmtGJ) in `fac` when fac.L is set.
hipError_t launch_solve_forward(int NP, int n, int S, int F, const double *M_d,
                                const double *R_d, const double *phi_d, const double *C_d,
                                const double *omega_d, double2 *I_d, int32_t *status_d,
                                GJFactor fac, hipStream_t st);

// Adjoint solve by a second pivoted Gauss-Jordan elimination of Z (used by the
// vector-Jacobian product, which has no recorded factorisation):
// Z mu = rscale * sum_c (rr_c - j ri_c); writes the per-system gradient term
// gsys[s][k] = 2 Re(mu_k I_k / (j w C_k^2)).  The system status is OR-ed into
// status_d when or_status, else assigned.
hipError_t launch_solve_adjoint(int NP, int n, int S, int F, const double *M_d,
                                const double *R_d, const double *C_d, const double *omega_d,
                                const double2 *I_d, const double2 *rpart_d, int nchunk,
                                double rscale, double *gsys_d, double2 *mu_d, int32_t *status_d,
                                bool or_status, hipStream_t st);

// Sum over frequencies (and chunks for the loss) per configuration.
hipError_t launch_reduce(int n, int B, int F, int nchunk, const double *gsys_d,
                         const double *lpart_d, double lscale, double *grad_d, double *loss_d,
                         hipStream_t st);

// Fused B = G I, loss epilogue, r = G^T conj(w) over a P-chunk grid.
struct FusedArgs {
    const void *G;        // [P_pad][NP] in the precision's storage type
    const void *Glo;      // bf16 lo part (BF16X3 only)
    const uint16_t *GThi, *GTlo;  // [NP][P_pad] transposed bf16 hi/lo (BF16X3 only)
    const double *T;      // [P] target
    int P, P_pad, rows_per_chunk, nchunk;
    const double2 *I;     // [S][n]
    int S, n;
    double2 *rpart;       // [nchunk][S][NP] (rr, ri); may be null when !grad
    double *lpart;        // [nchunk][S]
    double inc = 0.0;     // incident field added before the loss (COSIM_LOSS_RATIO)
};
hipError_t launch_fused(Prec prec, int NP, int variant, int loss_mode, bool grad,
                        const FusedArgs &a, hipStream_t st);
// Tuning variants of the fused kernel per precision, and the number of
// systems one workgroup of a variant covers.
hipError_t launch_adam(int count, double *C_d, const double *grad_d, double *m_d, double *v_d,
                       int32_t *step_d, double lr, double beta1, double beta2, double eps,
                       hipStream_t st);
int fused_variant_count(Prec prec);
int fused_systems_per_block(Prec prec, int NP, int variant);
// Workgroups of the variant's fused kernel that one compute unit holds at once.
int fused_blocks_per_cu(Prec prec, int NP, int variant);
// The fused contraction of several plans (64 loops or fewer, one precision,
// variant 0) in one launch: member m owns workgroups [first[m], first[m + 1])
// (the last up to the launch's total), bx[m] system blocks times its chunks.
constexpr int kFusedGroupMax = 24;
struct FusedGroup {
    int count;
    int first[kFusedGroupMax];
    int bx[kFusedGroupMax];
    FusedArgs in[kFusedGroupMax];
};
hipError_t launch_fused_group(Prec prec, int NP, int loss_mode, bool grad, const FusedGroup &g,
                              int blocks, hipStream_t st);

// ---- more than 64 loops: blocked LU with partial pivoting (solve_big.hip)
// and GEMM-based contractions (contract_big.hip).
// Right-hand side of launch_lu_solve.
enum BigRhs {
    kRhsExcitation = 0,  // E - j w Phi (loop_voltage), writes I
    kRhsPairs = 1,       // rpart[c][s][k] (rr, ri) FP64 pairs, writes gsys
    kRhsPlanarF32 = 2,   // R[c] NP x 2S FP32 planes, writes gsys
    kRhsPlanarF64 = 3    // R[c] NP x 2S FP64 planes, writes gsys
};
hipError_t launch_lu_big(int NP, int n, int S, int F, const double *M_d, const double *R_d,
                         const double *C_d, const double *omega_d, double2 *A_d, int *piv_d,
                         int32_t *status_d, hipStream_t st);
// Workspace of the blocked LDL^T above 64 loops (ldl: every R_k > 0).
struct BigFactor {
    bool ldl = false;
    int *fmt = nullptr;       // [S] kFmtLDL / kFmtNeedsPivot
    double *zmax = nullptr;   // [S] largest |re| + |im| of a diagonal entry of Z
    double2 *wt = nullptr;    // [S][64][NP] L21 of the current panel, column-major
    double2 *tinv = nullptr;  // [S][64][64] L11^-T of the current panel
};
// FP32 factorisation with FP64 iterative refinement (above 64 loops, every
// R_k > 0): the blocked LDL^T runs on a complex64 record A32 [S][NP][NP].
struct BigRefine {
    bool on = false;
    void *A32 = nullptr;  // float2 [S][NP][NP]
    int max_iter = 0;     // refinement steps before the FP64 fallback
    double tol = 0.0;     // estimated relative error at which a system is done
};
// Factor of the S systems: blocked LDL^T (in FP32 into rf.A32 when rf.on) with
// pivoted FP64 LU into A_d for the marked systems when bf.ldl, else pivoted
// LU throughout.
hipError_t big_factor(const BigFactor &bf, const BigRefine &rf, int NP, int n, int S, int F,
                      const double *M_d, const double *R_d, const double *C_d,
                      const double *omega_d, double2 *A_d, int *piv_d, int32_t *status_d,
                      hipStream_t st);
// Solves with the records big_factor left (arguments as launch_lu_solve): the
// FP64 records directly; with refinement, the FP32 records refined in FP64
// and FP64 fallbacks for the systems that do not converge.
hipError_t big_solve(const BigFactor &bf, const BigRefine &rf, int NP, int n, int S, int F,
                     const double *M_d, const double *R_d, const double *phi_d, const double *C_d,
                     const double *omega_d, double2 *A_d, int *piv_d, double2 *I_d, int rhs_kind,
                     const void *rhs_d, int nchunk, double rscale, double *gsys_d,
                     int32_t *status_d, hipStream_t st, double2 *mu_d = nullptr);
// Instances of one padded size above 64 loops factored and solved together,
// each system as it would be alone (GroupArgs travels by value in the kernel
// arguments; s0 numbers the systems instance after instance).
constexpr int kGroupMax = 32;
struct GroupInst {
    const double *M, *R, *phi, *C, *omega;
    double2 *I;        // [S][n] currents
    const void *rhs;   // adjoint sums, as for launch_lu_solve
    double *gsys;      // [S][n] adjoint gradient terms
    double2 *mu;       // [S][n] adjoint solutions or null
    int32_t *status;   // [S]
    int n, F, S, nchunk, s0;
    double rscale;
};
struct GroupArgs {
    int count;
    GroupInst in[kGroupMax];
};
// Plans of 64 loops or fewer with every R_k > 0, grouped the same way: each
// member keeps its own factor record (fac) and workspace; members are stored
// in order of their first system s0 within the group.
constexpr int kSmallGroupMax = 24;
static_assert(kSmallGroupMax <= kFusedGroupMax, "a small group's contractions fit one FusedGroup");
struct SmallInst {
    const double *M, *R, *phi, *C, *omega;
    double2 *I;            // [S][n] currents (z from the factorisation, then I)
    const double2 *rpart;  // [nchunk][S][NP] partial adjoint sums
    double *gsys;          // [S][n] adjoint gradient terms
    double2 *mu;           // [S][n] adjoint solutions or null
    int32_t *status;       // [S]
    GJFactor fac;
    int n, F, S, nchunk, s0;
    double rscale;
};
struct SmallGroup {
    int count;
    SmallInst in[kSmallGroupMax];
};
enum class SmallPhase { Factor, Fallback, Adjoint };
// The final sums (k_reduce) of a group's members in one launch; member i owns
// configurations [b0, b0 + B) of the launch.
struct ReduceInst {
    const double *gsys, *lpart;
    double *grad, *loss;
    double lscale;
    int n, B, F, nchunk, b0;
};
struct ReduceGroup {
    int count;
    ReduceInst in[kGroupMax];
};
hipError_t launch_reduce_group(const ReduceGroup &g, int Btot, hipStream_t st);
// One phase of the small-plan solver path (k_ldl with the forward solve, the
// pivoted fallback of marked systems, the adjoint replay) over a group's S systems.
hipError_t launch_small_group(int NP, const SmallGroup &g, int S, SmallPhase phase,
                              hipStream_t st);
// Blocked LDL^T (pivoted LU for marked systems) of the group's systems into A_d.
hipError_t big_group_factor(const BigFactor &bf, const GroupArgs &g, int NP, int S,
                            double2 *A_d, int *piv_d, hipStream_t st);
// Forward (kRhsExcitation, writes I) or adjoint solves of the group's systems.
hipError_t big_group_solve(const GroupArgs &g, int NP, int S, const double2 *A_d,
                           const int *piv_d, int rhs_kind, hipStream_t st);
hipError_t launch_lu_solve(int NP, int n, int S, int F, const double2 *A_d, const int *piv_d,
                           const double *phi_d, const double *C_d, const double *omega_d,
                           double2 *I_d, int rhs_kind, const void *rhs_d, int nchunk,
                           double rscale, double *gsys_d, int32_t *status_d, hipStream_t st,
                           double2 *mu_d = nullptr);
// ---- matrix-core contractions for any padded loop count (contract_mfma.hip):
// the loss path above 64 loops, the materialised field and its vector-Jacobian
// product for every plan.
enum MfmaMode {
    kMfmaLoss = 0,      // B = G I, loss partials per (chunk, system)
    kMfmaLossGrad = 1,  // and r = G^T w per (chunk, system)
    kMfmaField = 2,     // B = G I written to Bout
    kMfmaVjp = 3        // r = G^T g of the upstream gradient gB
};
// FP32 accumulation of r covers at most this many points per chunk.
constexpr int kMfmaRowsF32 = 2048;
struct MfmaArgs {
    const void *G = nullptr, *Glo = nullptr;    // [P_pad][NP] (Glo: bf16 lo part, BF16X3)
    const void *GT = nullptr, *GTlo = nullptr;  // [NP][P_pad] transposed copies
    const double2 *I = nullptr;                 // [S][n] currents (loss, field)
    const double2 *gB = nullptr;                // [S][P] upstream gradient (vjp)
    const double *T = nullptr;                  // [P] targets (loss)
    double inc = 0.0;                           // incident field of COSIM_LOSS_RATIO
    void *Bout = nullptr;  // [S][P] complex128 (FP64) or complex64 (field)
    int n = 0, NP = 0, P = 0, P_pad = 0, S = 0;
    int rows_per_chunk = 0, nchunk = 0, nsb = 0;  // chunks of points, system blocks
    double2 *rpart = nullptr;  // [nchunk][S][NP] (rr, ri) of r = G^T w
    double *lpart = nullptr;   // [nchunk][S] loss partial sums
};
struct MfmaShape {
    int waves = 1, nsb = 1, rows_per_chunk = 0, nchunk = 0;
};
// Systems per workgroup, and the launch shape for S systems.
int mfma_systems_per_block(Prec prec);
MfmaShape mfma_shape(Prec prec, int NP, int S, int P_pad, int cus);
hipError_t launch_mfma(Prec prec, int mode, int loss_mode, const MfmaArgs &a, int waves,
                       hipStream_t st);
// The loss (and gradient) contraction of several plans of one padded loop
// count in one launch (cosim_loss_and_grad_many): member m owns the
// workgroups [first[m], first[m + 1]), first[m] a multiple of 8 and the range
// at least its nchunk * nsb; all members launch with `waves` waves.
struct MfmaGroup {
    int count = 0;
    int first[kGroupMax] = {};
    MfmaArgs in[kGroupMax];
};
static_assert(sizeof(MfmaGroup) <= 4096 && sizeof(GroupArgs) <= 4096 &&
                  sizeof(SmallGroup) <= 4096 && sizeof(FusedGroup) <= 4096 &&
                  sizeof(ReduceGroup) <= 4096,
              "group descriptors go by value: kernel arguments are limited to 4 KB");
hipError_t launch_mfma_group(Prec prec, bool grad, int loss_mode, const MfmaGroup &g, int blocks,
                             int waves, hipStream_t st);

// ---- large batches above 64 loops: two GEMM passes (gemm_big.hip)
// One pass: C (M x N) = A B^T with A [M][lda] and B [N][ldb] K-contiguous.
struct GemmArgs {
    const void *A = nullptr, *Alo = nullptr;  // Alo / Blo: bf16 lo planes (BF16X3)
    const void *B = nullptr, *Blo = nullptr;
    int M = 0, N = 0, K = 0, lda = 0, ldb = 0;
    int kchunk = 0, nkc = 1;  // K in chunks (pass 2: one partial per chunk)
    // pass 1: loss per (row block, system), w planes [N][ldw] when W is set
    const double *T = nullptr;
    double inc = 0.0;
    int P = 0;
    void *W = nullptr, *Wlo = nullptr;
    int ldw = 0;
    double *lpart = nullptr;
    // pass 2: r per (chunk, system) as (rr, ri)
    double2 *rpart = nullptr;
    int S = 0, NP = 0;
};
struct GemmShape {
    int N = 0;           // columns (2 S padded to the column block)
    int row_blocks = 0;  // loss partials per system
    int kchunk = 0, nkc = 0;  // adjoint chunks of points: r partials per system
};
// The loss and gradient contractions of S systems by the two passes.
struct GemmLoss {
    const void *G, *Glo, *GT, *GTlo;  // the precision's copies of G
    const double2 *I;                 // [S][n]
    const double *T;
    double inc;
    int n, NP, P, P_pad, S;
    void *ws;         // gemm_ws_bytes: X^T and W^T planes
    double *lpart;    // [row_blocks][S]
    double2 *rpart;   // [nkc][S][NP]
};
bool gemm_path(Prec prec, int NP, int S);
GemmShape gemm_shape(Prec prec, int NP, int S, int P_pad);
size_t gemm_ws_bytes(int NP, int S, int P_pad);
hipError_t launch_gemm_loss(Prec prec, int loss_mode, bool grad, const GemmLoss &L,
                            hipStream_t st);

// ---- the other circuit variables and the helpers around C (params.hip)
// Per system from I and mu ([S][n]): the R and L terms to gRs, gLs ([S][n])
// and dL/dw to gw ([B][F]); then, if gR / gL is set, their sums over
// frequencies ([B][n]).
hipError_t launch_param_grads(int n, int B, int F, const double2 *I, const double2 *mu,
                              const double *C, const double *omega, const double *phi,
                              const double *M, double *gRs, double *gLs, double *gR, double *gL,
                              double *gw, hipStream_t st);
hipError_t launch_resonant_c(int n, int F, const double *M, const double *omega, int coupled,
                             double *Cr, hipStream_t st);
hipError_t launch_tanh_project(size_t count, const double *theta, double cmin, double cmax,
                               double *C, double *dC, hipStream_t st);
hipError_t launch_clip(size_t count, double *x, double lo, double hi, hipStream_t st);
// y = a x for count elements
hipError_t launch_scale(size_t count, double a, const double *x, double *y, hipStream_t st);

// ---- S-parameter pipeline (sparam.hip)
constexpr int kSpMaxPorts = 64;
// Device-side view of an S-parameter plan (all complex arrays complex128
// unless noted).
struct SpDev {
    int n0 = 0, n1 = 0, F = 0, P = 0, ncomp = 0, nvar = 0;
    double2 *S0 = nullptr;        // [F][n0][n0]
    double2 *K = nullptr;         // [F][n0][n0]  I - S_C11,const S0
    double2 *r0 = nullptr;        // [F][n0]      S_C12,const exc
    double2 *exc = nullptr;       // [n1]
    int *ix = nullptr, *iy = nullptr;  // [nvar] rows / columns of the variable entries
    double2 *fields64 = nullptr;  // [F][P][ncomp][n0]
    float2 *fields32 = nullptr;   // the same in complex64 (FP32 contractions)
};
// Workspace for B configurations (s = b F + f).
struct SpWork {
    int B = 0, rows = 0, nchunk = 0;  // P-chunk of the contractions
    double2 *X = nullptr;             // [S][n0] forward solution, FP64
    void *Xg = nullptr;               // [F][B][n0] GEMM operand (complex128 or complex64)
    void *Y = nullptr;                // [F][B][rows] B_comb, then conj(w), of one chunk
    void *Rp = nullptr;               // [nchunk][F][B][n0] conj(fields^H w) per chunk
    double *lpart = nullptr;          // [nchunk][F][B] loss partial sums
};
// The S-parameter pipeline's complex contractions run on rocBLAS; its handle.
hipError_t sp_blas_create(void **handle);
void sp_blas_destroy(void *handle);
hipError_t sp_prep(const SpDev &d, const double2 *sc_const, hipStream_t st);
hipError_t sp_set_lds_limit();
hipError_t sp_to_c64(size_t count, const double2 *a, float2 *b, hipStream_t st);
// Forward solves: X and Xg (prec 0: complex128, 1: complex64), status.
hipError_t sp_forward(const SpDev &d, int B, const double2 *values, double2 *X, void *Xg, int prec,
                      int32_t *status, hipStream_t st);
// B_comb of every component: out[b][f][p][c] from the complex128 Xg of sp_forward.
hipError_t sp_field(void *blas, const SpDev &d, int B, const double2 *Xg64, double2 *out,
                    hipStream_t st);
hipError_t sp_loss_and_grad(void *blas, const SpDev &d, const SpWork &w, int B,
                            const double2 *values, const double *T, int comp, int loss_mode, int prec,
                            double *loss, double2 *grad, int32_t *status, hipStream_t st);
hipError_t sp_rc(int B, int F, int n, const double *R, const double *C, const double *omega,
                 double z0, double2 *gam, int ld, hipStream_t st);
hipError_t sp_rc_backward(int B, int F, int n, const double *R, const double *C, const double *omega,
                          double z0, const double2 *g, int ld, double *gC, hipStream_t st);

// cosim_loss_and_grad with the call's device buffers (currents, factor
// records, partial sums, per-system gradient terms) carved from `scratch`
// (scratch_bytes long, 256-byte aligned) instead of the plan's workspace:
// allocates nothing.  Plans of 64 loops or fewer; COSIM_EINVAL when the call
// needs more than scratch_bytes.
int loss_and_grad_scratch(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                          const double *T_d, int loss_mode, int precision, double *loss_d,
                          double *grad_d, int32_t *status_d, void *stream, void *scratch,
                          size_t scratch_bytes);
// Sets the message cosim_last_error returns; returns code.
int set_error(int code, const char *msg);
// The plan's device, which must be the current one (else COSIM_EINVAL).
int plan_device(const cosim_plan *p, int *device);

}  // namespace cosim

// Library-owned objects behind the opaque handles.
struct cosim_geom {
    int n = 0, V = 0;
    std::vector<int32_t> seg_off;
    std::vector<double> verts, wire_a, R, area_z;
};

struct cosim_plan {
    int device = 0;
    int cus = 0;  // compute units of the device
    int n = 0, NP = 0, P = 0, P_pad = 0;
    double bext_z = 0.0;
    int component = 2;          // Cartesian component of the field that G holds (0 x, 1 y, 2 z)
    int n_drive = 0;            // loops with a source EMF (cosim_plan_set_drive)
    double *T_ratio = nullptr;  // [P] targets beta |bext_z| of the enhancement-factor loss
    std::vector<double> M_h, phi_h;
    std::vector<double> R_geom;  // series resistances of the geometry (without port impedances)
    std::vector<double> R_h;     // what R_d holds
    std::vector<double> exc_h;   // what phi_d holds: [3][n], see loop_voltage
    // operators (device)
    // [P_pad][NP] row-major per precision, and transposed [NP][P_pad] copies
    double *G64 = nullptr, *GT64 = nullptr;
    float *G32 = nullptr, *GT32 = nullptr;
    uint16_t *Ghi = nullptr, *Glo = nullptr;    // bf16 hi / lo
    uint16_t *GThi = nullptr, *GTlo = nullptr;
    double *M_d = nullptr, *R_d = nullptr;
    double *phi_d = nullptr;  // [3][n] loop excitation, see loop_voltage
    // workspace (device)
    size_t cap_systems = 0;
    size_t cap_parts = 0;  // (P-chunk, system) slots of the partial sums rpart
    size_t cap_lparts = 0; // (P-chunk, system) slots of the loss partial sums lpart
    void *gws = nullptr;   // above 64 loops, large batches: the GEMM passes' planes
    size_t cap_gws = 0;
    double2 *I_ws = nullptr;
    double2 *rpart = nullptr;
    double *lpart = nullptr;
    double *gsys = nullptr;
    cosim::GJFactor fac;  // recorded forward eliminations (loss_and_grad, solve)
    // the factor record of the last cosim_solve, while no other call has
    // overwritten the workspace: its B and F (rec_S = 0: none)
    int rec_B = 0, rec_F = 0;
    size_t rec_S = 0;
    int32_t *rec_status = nullptr;  // [cap_systems] status of that solve
    long long factorisations = 0;   // batches whose Z this plan has factorised
    // optional phase timing: (COSIM_PHASES + 1) events per recorded call
    std::vector<hipEvent_t> events;
    int timing_cap = 0, timing_used = 0;
    // more than 64 loops: the blocked LDL^T and refinement workspace
    double2 *bWt = nullptr;   // blocked LDL^T panel copy ([S][64][NP], see BigFactor)
    double2 *bTinv = nullptr; // blocked LDL^T L11^-T ([S][64][64])
    double *bZmax = nullptr;  // [S] largest diagonal |Z_kk| (blocked LDL^T)
    void *bA32 = nullptr;     // [S][NP][NP] complex64 records of the refined solves
    bool refine = false;      // FP32 factorisation + FP64 refinement (cosim_plan_set_refinement)
    int refine_iter = 0;
    double refine_tol = 0.0;  // 0: chosen per precision
    double2 *mu_ws = nullptr; // [S][n] adjoint solutions (gradients of R, L, w)
    double *gpar_ws = nullptr; // [2][S][n] per-system R and L terms
    size_t par_cap = 0;       // systems mu_ws / gpar_ws hold
    int prec_mask = 7;    // precisions whose copies of G were assembled (bit 1 << precision)
    bool ldl_ok = false;  // every R_k > 0: the LDL^T fast path applies
    int variant[3] = {0, 0, 0};  // fused-kernel variant per precision
};
