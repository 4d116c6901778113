// Batched FP64 complex solves for more than 64 loops (NP a multiple of 64, up
// to kMaxLoopsBig): Z I = -j w Phi (Eq. 6 in impedance form) and, Z being
// complex symmetric, the adjoint Z mu = r with the same factor.
//
// One workgroup per (configuration, frequency) system; Z and its factor live
// in HBM ([NP][NP] complex, row-major, per system).  Right-looking LU with
// partial pivoting in panels of kPW columns:
//   1. each panel column: arg-max of |re|+|im| below the diagonal (ties to the
//      lower row), the whole row swapped at once, multipliers scaled, the rest
//      of the panel updated (rank-1);
//   2. U12 = L11^-1 A12 (one thread per column);
//   3. A22 -= L21 U12 over 16x16 tiles staged in LDS.
// The result is P Z = L U with the swaps recorded in order; the solve kernel
// replays the swaps on the right-hand side and runs the two triangular solves
// in blocks of 16 rows (dot products against solved rows, then the 16x16
// diagonal block inside one wave).
#include "internal.h"

namespace cosim {

namespace {

constexpr int kPW = 16;   // panel width
constexpr int kTB = 256;  // threads per workgroup

__device__ inline double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc - l * u
__device__ inline double2 zfms(double2 acc, double2 l, double2 u) {
    return make_double2(fma(-l.x, u.x, fma(l.y, u.y, acc.x)), fma(-l.x, u.y, fma(-l.y, u.x, acc.y)));
}
// acc + l * u
__device__ inline double2 zfma(double2 acc, double2 l, double2 u) {
    return make_double2(fma(l.x, u.x, fma(-l.y, u.y, acc.x)), fma(l.x, u.y, fma(l.y, u.x, acc.y)));
}
__device__ inline double2 zinv(double2 a) {
    const double d = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * d, -a.y * d);
}

// Arg-max of (m, idx) over the workgroup, ties to the lower index; every
// thread returns with the result.  sm/si: 4-entry LDS scratch.
__device__ inline void block_amax(double &m, int &idx, double *sm, int *si) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double om = __shfl_xor(m, off);
        const int oi = __shfl_xor(idx, off);
        if (om > m || (om == m && oi < idx)) {
            m = om;
            idx = oi;
        }
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[wv] = m;
        si[wv] = idx;
    }
    __syncthreads();
    m = sm[0];
    idx = si[0];
#pragma unroll
    for (int w = 1; w < kTB / 64; ++w)
        if (sm[w] > m || (sm[w] == m && si[w] < idx)) {
            m = sm[w];
            idx = si[w];
        }
    __syncthreads();
}

__global__ __launch_bounds__(kTB) void k_lu_big(int n, int NP, int S, int F,
                                                const double *__restrict__ M,
                                                const double *__restrict__ Rv,
                                                const double *__restrict__ C,
                                                const double *__restrict__ omega,
                                                double2 *__restrict__ Aall, int *__restrict__ pivall,
                                                int32_t *__restrict__ status) {
    __shared__ double sm[kTB / 64];
    __shared__ int si[kTB / 64];
    __shared__ int sFlag;
    __shared__ double2 sU[kPW];
    __shared__ double2 sL11[kPW][kPW];
    __shared__ double2 sLt[16][kPW + 1];
    __shared__ double2 sUt[kPW][16 + 1];
    const int s = blockIdx.x;
    if (s >= S) return;  // whole workgroup
    const int tid = threadIdx.x;
    double2 *A = Aall + (size_t)s * NP * NP;
    int *piv = pivall + (size_t)s * NP;
    const int b = s / F, f = s - b * F;
    const double w = omega[f];
    const double *Cb = C + (size_t)b * n;
    if (tid == 0) sFlag = 0;
    __syncthreads();
    for (int k = tid; k < n; k += kTB) {
        const double c = Cb[k];
        if (!isfinite(c) || c == 0.0 || !isfinite(w) || w == 0.0) atomicOr(&sFlag, COSIM_SYS_BAD_INPUT);
        else if (c < 0.0) atomicOr(&sFlag, COSIM_SYS_NEGATIVE_C);
    }
    // Z = diag(R) + j w M + diag(1/(j w C)), identity padding
    for (size_t e = tid; e < (size_t)NP * NP; e += kTB) {
        const int i = (int)(e / NP), j = (int)(e - (size_t)i * NP);
        double zr = 0.0, zi = 0.0;
        if (i < n && j < n) {
            zi = w * M[(size_t)i * n + j];
            if (i == j) {
                zr = Rv[i];
                zi -= 1.0 / (w * Cb[i]);
            }
        } else if (i == j) {
            zr = 1.0;
        }
        A[e] = make_double2(zr, zi);
    }
    __syncthreads();

    for (int j0 = 0; j0 < NP; j0 += kPW) {
        // ---- 1. panel columns j0 .. j0 + kPW - 1
        for (int jj = 0; jj < kPW; ++jj) {
            const int j = j0 + jj;
            double m = -1.0;
            int idx = j;
            for (int i = j + tid; i < NP; i += kTB) {
                const double2 a = A[(size_t)i * NP + j];
                double mg = fabs(a.x) + fabs(a.y);
                if (!(mg == mg)) mg = __builtin_inf();
                if (mg > m) {
                    m = mg;
                    idx = i;
                }
            }
            block_amax(m, idx, sm, si);
            const int p = idx;
            if (tid == 0) piv[j] = p;
            if (p != j) {
                for (int c = tid; c < NP; c += kTB) {
                    const double2 t = A[(size_t)j * NP + c];
                    A[(size_t)j * NP + c] = A[(size_t)p * NP + c];
                    A[(size_t)p * NP + c] = t;
                }
            }
            __syncthreads();
            if (tid < kPW) sU[tid] = A[(size_t)j * NP + j0 + tid];
            __syncthreads();
            const double2 d = sU[jj];
            if (tid == 0 && !(d.x != 0.0 || d.y != 0.0)) atomicOr(&sFlag, COSIM_SYS_SINGULAR);
            const double2 inv = zinv(d);
            for (int i = j + 1 + tid; i < NP; i += kTB) {
                double2 *row = A + (size_t)i * NP + j0;
                const double2 l = zmul(row[jj], inv);
                row[jj] = l;
                for (int c = jj + 1; c < kPW; ++c) row[c] = zfms(row[c], l, sU[c]);
            }
            __syncthreads();
        }
        if (j0 + kPW >= NP) break;
        // ---- 2. U12 = L11^-1 A12
        for (int e = tid; e < kPW * kPW; e += kTB) {
            const int r = e / kPW, c = e - r * kPW;
            sL11[r][c] = A[(size_t)(j0 + r) * NP + j0 + c];
        }
        __syncthreads();
        for (int c = j0 + kPW + tid; c < NP; c += kTB) {
            double2 u[kPW];
#pragma unroll
            for (int r = 0; r < kPW; ++r) u[r] = A[(size_t)(j0 + r) * NP + c];
#pragma unroll
            for (int r = 1; r < kPW; ++r)
#pragma unroll
                for (int r2 = 0; r2 < r; ++r2) u[r] = zfms(u[r], sL11[r][r2], u[r2]);
#pragma unroll
            for (int r = 1; r < kPW; ++r) A[(size_t)(j0 + r) * NP + c] = u[r];
        }
        __syncthreads();
        // ---- 3. A22 -= L21 U12, tiles of 16 x 16
        const int base = j0 + kPW, nt = (NP - base) / 16;
        const int tr = tid >> 4, tc = tid & 15;
        for (int t = 0; t < nt * nt; ++t) {
            const int ti = t / nt, tj = t - ti * nt;
            const int r0 = base + 16 * ti, c0 = base + 16 * tj;
            sLt[tr][tc] = A[(size_t)(r0 + tr) * NP + j0 + tc];
            sUt[tr][tc] = A[(size_t)(j0 + tr) * NP + c0 + tc];
            __syncthreads();
            double2 acc = A[(size_t)(r0 + tr) * NP + c0 + tc];
#pragma unroll
            for (int k = 0; k < kPW; ++k) acc = zfms(acc, sLt[tr][k], sUt[k][tc]);
            A[(size_t)(r0 + tr) * NP + c0 + tc] = acc;
            __syncthreads();
        }
    }
    if (tid == 0) status[s] = sFlag;
}

// Adjoint right-hand side: rscale * conj(sum over chunks of (rr + j ri)).
// Forward: I[s][k]; adjoint: gsys[s][k] = 2 Re(mu_k I_k / (j w C_k^2)).
template <int RHS>
__global__ __launch_bounds__(kTB) void k_lu_solve(int n, int NP, int S, int F,
                                                  const double2 *__restrict__ Aall,
                                                  const int *__restrict__ pivall,
                                                  const double *__restrict__ phi,
                                                  const double *__restrict__ C,
                                                  const double *__restrict__ omega,
                                                  double2 *__restrict__ I, const void *rhs,
                                                  int nchunk, double rscale,
                                                  double *__restrict__ gsys,
                                                  int32_t *__restrict__ status) {
    __shared__ double2 sx[kMaxLoopsBig];
    __shared__ double2 st[16];
    __shared__ int sFlag;
    const int s = blockIdx.x;
    if (s >= S) return;
    const int tid = threadIdx.x;
    const double2 *A = Aall + (size_t)s * NP * NP;
    const int *piv = pivall + (size_t)s * NP;
    const int b = s / F, f = s - b * F;
    const double w = omega[f];
    for (int k = tid; k < NP; k += kTB) {
        double2 x = make_double2(0.0, 0.0);
        if (k < n) {
            if (RHS == kRhsExcitation) {
                x = make_double2(0.0, -w * phi[k]);
            } else {
                double rr = 0.0, ri = 0.0;
                for (int c = 0; c < nchunk; ++c) {
                    if (RHS == kRhsPairs) {
                        const double2 v = ((const double2 *)rhs)[((size_t)c * S + s) * NP + k];
                        rr += v.x;
                        ri += v.y;
                    } else if (RHS == kRhsPlanarF32) {
                        const float *R = (const float *)rhs + (size_t)c * NP * 2 * S;
                        rr += (double)R[(size_t)(2 * s) * NP + k];
                        ri += (double)R[(size_t)(2 * s + 1) * NP + k];
                    } else {
                        const double *R = (const double *)rhs + (size_t)c * NP * 2 * S;
                        rr += R[(size_t)(2 * s) * NP + k];
                        ri += R[(size_t)(2 * s + 1) * NP + k];
                    }
                }
                x = make_double2(rscale * rr, -rscale * ri);
            }
        }
        sx[k] = x;
    }
    if (tid == 0) sFlag = 0;
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < NP; ++j) {
            const int p = piv[j];
            if (p != j) {
                const double2 t = sx[j];
                sx[j] = sx[p];
                sx[p] = t;
            }
        }
    }
    __syncthreads();
    const int r = tid >> 4, q = tid & 15;
    // forward: L y = P b, L unit lower
    for (int r0 = 0; r0 < NP; r0 += 16) {
        double2 acc = make_double2(0.0, 0.0);
        const double2 *row = A + (size_t)(r0 + r) * NP;
        for (int j = q; j < r0; j += 16) acc = zfma(acc, row[j], sx[j]);
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off);
            acc.y += __shfl_xor(acc.y, off);
        }
        if (q == 0) st[r] = make_double2(sx[r0 + r].x - acc.x, sx[r0 + r].y - acc.y);
        __syncthreads();
        if (tid < 64) {
            const int l = tid & 15;
            double2 t = st[l];
            for (int k = 0; k < 15; ++k) {
                const double2 yk = make_double2(__shfl(t.x, k), __shfl(t.y, k));
                const double2 lk = l > k ? A[(size_t)(r0 + l) * NP + r0 + k] : make_double2(0.0, 0.0);
                t = zfms(t, lk, yk);
            }
            if (tid < 16) sx[r0 + l] = t;
        }
        __syncthreads();
    }
    // backward: U x = y
    for (int r0 = NP - 16; r0 >= 0; r0 -= 16) {
        double2 acc = make_double2(0.0, 0.0);
        const double2 *row = A + (size_t)(r0 + r) * NP;
        for (int j = r0 + 16 + q; j < NP; j += 16) acc = zfma(acc, row[j], sx[j]);
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off);
            acc.y += __shfl_xor(acc.y, off);
        }
        if (q == 0) st[r] = make_double2(sx[r0 + r].x - acc.x, sx[r0 + r].y - acc.y);
        __syncthreads();
        if (tid < 64) {
            const int l = tid & 15;
            double2 t = st[l];
            for (int k = 15; k >= 0; --k) {
                // lane k finishes x_k; the lanes of the rows above subtract its term
                if (l == k) t = zmul(t, zinv(A[(size_t)(r0 + k) * NP + r0 + k]));
                const double2 xk = make_double2(__shfl(t.x, k), __shfl(t.y, k));
                const double2 uk = l < k ? A[(size_t)(r0 + l) * NP + r0 + k] : make_double2(0.0, 0.0);
                t = zfms(t, uk, xk);
            }
            if (tid < 16) sx[r0 + l] = t;
        }
        __syncthreads();
    }
    const int flag = status[s];
    const bool bad = (flag & (COSIM_SYS_BAD_INPUT | COSIM_SYS_SINGULAR)) != 0;
    int oflag = 0;
    for (int k = tid; k < n; k += kTB) {
        double2 x = sx[k];
        if (bad) x = make_double2(__builtin_nan(""), __builtin_nan(""));
        if (RHS == kRhsExcitation) {
            I[(size_t)s * n + k] = x;
            if (!bad && !(isfinite(x.x) && isfinite(x.y))) oflag = COSIM_SYS_NONFINITE;
        } else {
            const double2 Ik = I[(size_t)s * n + k];
            const double ck = C[(size_t)b * n + k];
            const double g = 2.0 * (x.x * Ik.y + x.y * Ik.x) / (w * ck * ck);
            gsys[(size_t)s * n + k] = g;
            if (!bad && !isfinite(g)) oflag = COSIM_SYS_NONFINITE;
        }
    }
    if (oflag) atomicOr(&sFlag, oflag);
    __syncthreads();
    if (tid == 0 && sFlag) status[s] = flag | sFlag;
}

}  // namespace

hipError_t launch_lu_big(int NP, int n, int S, int F, const double *M_d, const double *R_d,
                         const double *C_d, const double *omega_d, double2 *A_d, int *piv_d,
                         int32_t *status_d, hipStream_t st) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lu_big, dim3(S), dim3(kTB), 0, st, n, NP, S, F, M_d, R_d, C_d, omega_d,
                       A_d, piv_d, status_d);
    return hipGetLastError();
}

hipError_t launch_lu_solve(int NP, int n, int S, int F, const double2 *A_d, const int *piv_d,
                           const double *phi_d, const double *C_d, const double *omega_d,
                           double2 *I_d, int rhs_kind, const void *rhs_d, int nchunk,
                           double rscale, double *gsys_d, int32_t *status_d, hipStream_t st) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig) return hipErrorInvalidValue;
    const dim3 grid(S), blk(kTB);
    switch (rhs_kind) {
        case kRhsExcitation:
            hipLaunchKernelGGL(k_lu_solve<kRhsExcitation>, grid, blk, 0, st, n, NP, S, F, A_d, piv_d,
                               phi_d, C_d, omega_d, I_d, rhs_d, nchunk, rscale, gsys_d, status_d);
            break;
        case kRhsPairs:
            hipLaunchKernelGGL(k_lu_solve<kRhsPairs>, grid, blk, 0, st, n, NP, S, F, A_d, piv_d,
                               phi_d, C_d, omega_d, I_d, rhs_d, nchunk, rscale, gsys_d, status_d);
            break;
        case kRhsPlanarF32:
            hipLaunchKernelGGL(k_lu_solve<kRhsPlanarF32>, grid, blk, 0, st, n, NP, S, F, A_d,
                               piv_d, phi_d, C_d, omega_d, I_d, rhs_d, nchunk, rscale, gsys_d,
                               status_d);
            break;
        case kRhsPlanarF64:
            hipLaunchKernelGGL(k_lu_solve<kRhsPlanarF64>, grid, blk, 0, st, n, NP, S, F, A_d,
                               piv_d, phi_d, C_d, omega_d, I_d, rhs_d, nchunk, rscale, gsys_d,
                               status_d);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cosim
