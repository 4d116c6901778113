// S-parameter cosimulation pipeline (Sec. III, Eq. 2-10; Sec. III-A):
// exports S0 and per-port fields of an n0-port structure, a connecting network
// S_C = S_C,const + S_C,var with n1 external ports, per (configuration,
// frequency) system s = b F + f:
//   A = I - S_C11 S0,  x = A^-1 S_C12 exc  (Eq. 6),  B_comb = fields x  (Eq. 7),
// the loss of Eq. 1 on one component, and its gradient with respect to the
// variable entries through A^H lam = fields^H w (Eq. 8-10).
//
// Kernels:
//   k_sp_prep   per frequency: K = I - S_C11,const S0 and r0 = S_C12,const exc
//               (the constant parts; the variable entries are applied per system);
//   k_sp_solve  one workgroup of four waves per system, the n0 x n0 matrix in
//               LDS (rows padded to a multiple of 16 plus 4 entries): A = K minus the variable rows of S_C11 S0, the
//               right-hand side r0 plus the variable entries of S_C12 exc, LU with
//               partial pivoting (largest |re| + |im|, ties to the lower row)
//               applied to the right-hand side as it goes, back substitution.
//               The adjoint form builds A^H and the right-hand side from the
//               contraction's partial sums, and ends with the gradient of every
//               variable entry;
//   rocBLAS complex GEMMs (per frequency, strided over frequencies, in P-chunks)
//               for B_comb = fields x and fields^H w, only on the rows of the
//               loss component;
//   k_sp_epilogue  loss terms and conj(w) in place of B_comb per chunk;
//   k_sp_reduce    fixed-order loss sums;
//   k_sp_rc, k_sp_rc_backward  the RC preprocessing of Eq. 2-3 and its chain rule.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "epilogue.h"
#include "internal.h"

namespace cosim {

namespace {

__device__ inline double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 zmulc(double2 a, double2 b) {  // a conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline double2 zfms(double2 acc, double2 l, double2 u) {  // acc - l u
    return make_double2(fma(-l.x, u.x, fma(l.y, u.y, acc.x)), fma(-l.x, u.y, fma(-l.y, u.x, acc.y)));
}
__device__ inline double2 zinv(double2 a) {
    const double d = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * d, -a.y * d);
}
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

// LDS row stride (complex entries) of the per-system matrix: a multiple of 16
// plus 4, so that the 16 lanes of one 16-byte access pass (4 rows x 4
// consecutive columns in the trailing update) fall on distinct banks
__host__ __device__ inline int sp_ld(int n0) { return (n0 + 15) / 16 * 16 + 4; }

template <int CTRL>
__device__ inline int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
// (magnitude, row) arg-max step with a DPP partner; ties to the lower row
template <int CTRL>
__device__ inline void amax_step(float &m, int &idx) {
    const float m2 = __int_as_float(dpp_i<CTRL>(__float_as_int(m)));
    const int i2 = dpp_i<CTRL>(idx);
    const bool take = (m2 > m) || (m2 == m && i2 < idx);
    m = take ? m2 : m;
    idx = take ? i2 : idx;
}
// arg-max over the wave: DPP inside each row of 16 lanes, shuffles across rows
__device__ inline int wave_amax(float m, int idx) {
    amax_step<0xB1>(m, idx);   // quad_perm [1,0,3,2]
    amax_step<0x4E>(m, idx);   // quad_perm [2,3,0,1]
    amax_step<0x141>(m, idx);  // row_half_mirror
    amax_step<0x140>(m, idx);  // row_mirror
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
        const float om = __shfl_xor(m, off);
        const int oi = __shfl_xor(idx, off);
        if (om > m || (om == m && oi < idx)) {
            m = om;
            idx = oi;
        }
    }
    return __builtin_amdgcn_readfirstlane(idx);
}
__device__ inline double rl(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ inline double2 rl2(double2 v, int src) { return make_double2(rl(v.x, src), rl(v.y, src)); }

// K[f] = I - S11c[f] S0[f], r0[f] = S12c[f] exc; grid (n0, F), 64 threads.
__global__ __launch_bounds__(64) void k_sp_prep(int n0, int n1, int F, const double2 *__restrict__ S0,
                                                const double2 *__restrict__ scc,
                                                const double2 *__restrict__ exc,
                                                double2 *__restrict__ K, double2 *__restrict__ r0) {
    const int i = blockIdx.x, f = blockIdx.y, lane = threadIdx.x;
    const int N = n0 + n1;
    const double2 *S0f = S0 + (size_t)f * n0 * n0;
    const double2 *Sc = scc ? scc + (size_t)f * N * N + (size_t)i * N : nullptr;
    for (int j = lane; j < n0; j += 64) {
        double2 acc = make_double2(0.0, 0.0);
        if (Sc)
            for (int k = 0; k < n0; ++k) {
                const double2 a = Sc[k], b = S0f[(size_t)k * n0 + j];
                acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
                acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
            }
        K[((size_t)f * n0 + i) * n0 + j] = make_double2((i == j ? 1.0 : 0.0) - acc.x, -acc.y);
    }
    if (lane == 0) {
        double2 acc = make_double2(0.0, 0.0);
        if (Sc)
            for (int j = 0; j < n1; ++j) {
                const double2 a = Sc[n0 + j], b = exc[j];
                acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
                acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
            }
        r0[(size_t)f * n0 + i] = acc;
    }
}

// One workgroup of four waves per system s = b F + f; the matrix in LDS (rows
// padded to sp_ld(n0) entries) and the right-hand side after it.  Elimination
// step k: every wave finds the pivot row itself (shuffles over column k), the
// row exchange runs over columns, the trailing update over (row, column
// quarter) with four threads per row, two workgroup barriers per step; wave 0
// then runs the back substitution and writes the outputs.
// ADJ = false: solves A x = S_C12 exc, writes X[s][n0] (FP64) and the GEMM
// operand Xg[f][b][n0] (PREC 0: complex128, 1: complex64).  ADJ = true:
// right-hand side r = rscale conj(sum over chunks of Rp[c][f][b][:]) (the chunks
// hold conj(fields^H w)), solves A^H lam = r and writes the gradient of every
// variable entry to grad[s][nvar].
template <bool ADJ, int PREC>
__global__ __launch_bounds__(256) void k_sp_solve(SpDev d, int B, const double2 *__restrict__ values,
                                                  double2 *__restrict__ X, void *Xg,
                                                  const void *Rp, int nchunk, double rscale,
                                                  double2 *__restrict__ grad,
                                                  int32_t *__restrict__ status) {
    extern __shared__ double2 sa[];
    const int n0 = d.n0, ld = sp_ld(n0), F = d.F, nvar = d.nvar;
    double2 *sx = sa + (size_t)n0 * ld;  // right-hand side, then solution
    const int s = blockIdx.x;
    const int b = s / F, f = s - b * F;
    const int tid = threadIdx.x, lane = tid & 63;
    const double2 *K = d.K + (size_t)f * n0 * n0;
    const double2 *S0f = d.S0 + (size_t)f * n0 * n0;
    const double2 *v = values + (size_t)s * nvar;
    __shared__ int s_ix[256], s_iy[256];
    __shared__ double2 s_v[256];
    // A = K - sum over variable S_C11 entries (r, c) of v e_r S0[c][:]
#pragma unroll 4
    for (int e = tid; e < n0 * n0; e += 256) {
        const int i = e / n0, j = e - i * n0;
        sa[i * ld + j] = K[e];
    }
    double2 x = make_double2(0.0, 0.0);  // thread i < n0: right-hand side entry i
    if (!ADJ && tid < n0) x = d.r0[(size_t)f * n0 + tid];
    // the variable entries, 256 at a time through LDS; thread j owns column j,
    // so repeated rows keep their order
    for (int e0 = 0; e0 < nvar; e0 += 256) {
        const int ne = min(256, nvar - e0);
        __syncthreads();
        if (tid < ne) {
            s_ix[tid] = d.ix[e0 + tid];
            s_iy[tid] = d.iy[e0 + tid];
            s_v[tid] = v[e0 + tid];
        }
        __syncthreads();
        if (tid < n0) {
            const int j = tid;
#pragma unroll 4
            for (int e = 0; e < ne; ++e) {
                const int r = s_ix[e], c = s_iy[e];
                if (r < n0 && c < n0) sa[r * ld + j] = zfms(sa[r * ld + j], s_v[e], S0f[(size_t)c * n0 + j]);
                if (!ADJ && r == j && c >= n0) {
                    const double2 t = zmul(s_v[e], d.exc[c - n0]);
                    x.x += t.x;
                    x.y += t.y;
                }
            }
        }
    }
    if (tid < n0) {
        const int i = tid;
        if (ADJ) {
            double sr = 0.0, si = 0.0;
#pragma unroll 8
            for (int c = 0; c < nchunk; ++c) {
                const size_t o = (((size_t)c * F + f) * B + b) * n0 + i;
                if (PREC == 0) {
                    const double2 t = ((const double2 *)Rp)[o];
                    sr += t.x;
                    si += t.y;
                } else {
                    const float2 t = ((const float2 *)Rp)[o];
                    sr += (double)t.x;
                    si += (double)t.y;
                }
            }
            x = make_double2(rscale * sr, -rscale * si);
        }
        sx[i] = x;
    }
    __syncthreads();
    if (ADJ) {
        // A -> A^H in place: thread i takes row i right of the diagonal and
        // column i below it (disjoint from every other thread's entries)
        if (tid < n0) {
            const int i = tid;
            sa[i * ld + i] = zconj(sa[i * ld + i]);
            for (int j = i + 1; j < n0; ++j) {
                const double2 t = sa[i * ld + j];
                sa[i * ld + j] = zconj(sa[j * ld + i]);
                sa[j * ld + i] = zconj(t);
            }
        }
        __syncthreads();
    }
    // LU with partial pivoting, right-hand side eliminated alongside
    int flag = 0;
    const int ur = tid >> 2, uq = tid & 3;  // update: row k + 1 + ur, columns = uq mod 4
    for (int k = 0; k < n0; ++k) {
        // pivot: largest |re| + |im| in column k (compared in FP32; a NaN wins)
        float mg = -1.0f;
        if (lane >= k && lane < n0) {
            const double2 a = sa[lane * ld + k];
            mg = (float)(fabs(a.x) + fabs(a.y));
            if (!(mg == mg)) mg = __builtin_inff();
        }
        const int p = wave_amax(mg, lane);
        __syncthreads();  // every wave has read column k
        if (p != k) {
            for (int j = tid; j < n0; j += 256) {
                const double2 t = sa[k * ld + j];
                sa[k * ld + j] = sa[p * ld + j];
                sa[p * ld + j] = t;
            }
            if (tid == 0) {
                const double2 t = sx[k];
                sx[k] = sx[p];
                sx[p] = t;
            }
        }
        __syncthreads();
        const double2 dk = sa[k * ld + k];
        if (!(dk.x != 0.0 || dk.y != 0.0)) flag |= COSIM_SYS_SINGULAR;
        const int i = k + 1 + ur;
        if (i < n0) {
            const double2 l = zmul(sa[i * ld + k], zinv(dk));
            if (uq == 0) sx[i] = zfms(sx[i], l, sx[k]);
            // this thread's columns j = k + 1 + uq + 4t, four at a time with every
            // load issued before the stores (the LDS round trips overlap)
            int j = k + 1 + uq;
            for (; j + 12 < n0; j += 16) {
                double2 a[4], u[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = sa[i * ld + j + 4 * t];
                    u[t] = sa[k * ld + j + 4 * t];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) sa[i * ld + j + 4 * t] = zfms(a[t], l, u[t]);
            }
            for (; j < n0; j += 4) sa[i * ld + j] = zfms(sa[i * ld + j], l, sa[k * ld + j]);
        }
        __syncthreads();
    }
    if (tid >= 64) return;  // wave 0 finishes alone (no barrier below)
    x = lane < n0 ? sx[lane] : make_double2(0.0, 0.0);
    for (int k = n0 - 1; k >= 0; --k) {
        const double2 xk = zmul(rl2(x, k), zinv(sa[k * ld + k]));
        if (lane == k) x = xk;
        if (lane < k) x = zfms(x, sa[lane * ld + k], xk);
    }
    const bool finite = isfinite(x.x) && isfinite(x.y);
    if (__ballot(lane < n0 && !finite) != 0) flag |= COSIM_SYS_NONFINITE;
    if (flag & COSIM_SYS_SINGULAR) x = make_double2(__builtin_nan(""), __builtin_nan(""));
    if (!ADJ) {
        if (lane == 0) status[s] = flag;
        if (lane < n0) {
            X[(size_t)s * n0 + lane] = x;
            const size_t o = ((size_t)f * B + b) * n0 + lane;
            if (PREC == 0) ((double2 *)Xg)[o] = x;
            else ((float2 *)Xg)[o] = make_float2((float)x.x, (float)x.y);
        }
        return;
    }
    // gradient: 2 lam_r conj(exc_j) for S_C12 entries (r, n0 + j), 2 lam_r
    // conj((S0 x)_c) for S_C11 entries (r, c), 0 for S_C21 / S_C22 entries
    if (lane == 0 && flag) status[s] |= flag;
    // y = S0 x once (lane c: row c, x broadcast from the forward solution)
    const double2 xs = lane < n0 ? X[(size_t)s * n0 + lane] : make_double2(0.0, 0.0);
    double2 y = make_double2(0.0, 0.0);
    if (lane < n0) {
        const double2 *row = S0f + (size_t)lane * n0;
#pragma unroll 8
        for (int k = 0; k < n0; ++k) {
            const double2 a = row[k], xk = rl2(xs, k);
            y.x = fma(a.x, xk.x, fma(-a.y, xk.y, y.x));
            y.y = fma(a.x, xk.y, fma(a.y, xk.x, y.y));
        }
    }
    // lane e % 64 forms entry e
    for (int e0 = 0; e0 < nvar; e0 += 64) {
        const int e = e0 + lane;
        const int r = e < nvar ? d.ix[e] : n0, c = e < nvar ? d.iy[e] : 0;
        // gathers from other lanes: every lane takes part in the shuffles
        const int rs = r < n0 ? r : 0, cs = c < n0 ? c : 0;
        const double2 lam = make_double2(__shfl(x.x, rs), __shfl(x.y, rs));
        const double2 yv = make_double2(__shfl(y.x, cs), __shfl(y.y, cs));
        if (e < nvar) {
            double2 g = make_double2(0.0, 0.0);
            if (r < n0) {
                const double2 gv = zmulc(lam, c >= n0 ? d.exc[c - n0] : yv);
                g = make_double2(2.0 * gv.x, 2.0 * gv.y);
            }
            grad[(size_t)s * nvar + e] = g;
        }
    }
}

// Loss terms of one P-chunk and conj(w) in place of B_comb; grid (B, F).
// Y[f][b][rows] (PREC 0 complex128, 1 complex64) holds B_comb of rows
// p0 .. p0 + nrows - 1 of the loss component; lpart[f][b] receives the chunk's
// sum of loss terms.
template <int PREC, int LOSS>
__global__ __launch_bounds__(256) void k_sp_epilogue(int B, int F, int rows, int p0, int nrows,
                                                     void *Y, const double *__restrict__ T,
                                                     double *__restrict__ lpart, bool grad) {
    __shared__ double red[4];
    const int b = blockIdx.x, f = blockIdx.y;
    const size_t base = ((size_t)f * B + b) * rows;
    double acc = 0.0;
    for (int p = threadIdx.x; p < nrows; p += 256) {
        if (PREC == 0) {
            double2 *y = (double2 *)Y + base + p;
            double vx = y->x, vy = y->y;
            acc += epilogue<LOSS>(vx, vy, T[p0 + p]);
            if (grad) *y = make_double2(vx, -vy);
        } else {
            float2 *y = (float2 *)Y + base + p;
            float vx = y->x, vy = y->y;
            acc += epilogue<LOSS>(vx, vy, (float)T[p0 + p]);
            if (grad) *y = make_float2(vx, -vy);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) lpart[(size_t)f * B + b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss[b] = lscale * sum over f, then chunks, of lpart[c][f][b]
__global__ void k_sp_reduce(int B, int F, int nchunk, const double *__restrict__ lpart, double lscale,
                            double *__restrict__ loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double acc = 0.0;
    for (int f = 0; f < F; ++f)
        for (int c = 0; c < nchunk; ++c) acc += lpart[((size_t)c * F + f) * B + b];
    loss[b] = lscale * acc;
}

// Eq. 2-3 per (b, f, k)
__global__ void k_sp_rc(int B, int F, int n, const double *__restrict__ R, const double *__restrict__ C,
                        const double *__restrict__ omega, double z0, double2 *__restrict__ gam, int ld) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)B * F * n) return;
    const int k = (int)(t % n);
    const size_t sf = t / n;
    const int f = (int)(sf % F), b = (int)(sf / F);
    const double zr = R[k], zi = -1.0 / (omega[f] * C[(size_t)b * n + k]);
    // (zr - z0 + j zi) / (zr + z0 + j zi)
    const double2 num = make_double2(zr - z0, zi), den = make_double2(zr + z0, zi);
    gam[sf * ld + k] = zmul(num, zinv(den));
}

// gC[b][k] = sum over f of Re(conj(g) dGamma/dC), dGamma/dC = 2 z0/(Z_C + z0)^2 j/(w C^2)
__global__ void k_sp_rc_backward(int B, int F, int n, const double *__restrict__ R,
                                 const double *__restrict__ C, const double *__restrict__ omega,
                                 double z0, const double2 *__restrict__ g, int ld,
                                 double *__restrict__ gC) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)B * n) return;
    const int k = (int)(t % n), b = (int)(t / n);
    const double c = C[t];
    double acc = 0.0;
    for (int f = 0; f < F; ++f) {
        const double w = omega[f];
        const double2 den = make_double2(R[k] + z0, -1.0 / (w * c));
        const double2 inv = zinv(den);
        const double2 inv2 = zmul(inv, inv);
        const double s = 2.0 * z0 / (w * c * c);
        const double2 dg = make_double2(-s * inv2.y, s * inv2.x);  // j s inv2
        const double2 gv = g[((size_t)b * F + f) * ld + k];
        acc += gv.x * dg.x + gv.y * dg.y;  // Re(conj(g) dg)
    }
    gC[t] = acc;
}

__global__ void k_sp_to_c64(size_t count, const double2 *__restrict__ a, float2 *__restrict__ b) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) b[t] = make_float2((float)a[t].x, (float)a[t].y);
}

hipError_t blas(rocblas_status r) { return r == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure; }

// C[f] (m x n, ldc) = op(A[f]) B[f] per frequency, column-major, complex
hipError_t cgemm(rocblas_handle h, int prec, rocblas_operation ta, int m, int n, int k, const void *A,
                 int lda, size_t sA, const void *Bm, int ldb, size_t sB, void *C, int ldc, size_t sC,
                 int batch) {
    if (prec == 0) {
        const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
        return blas(rocblas_zgemm_strided_batched(
            h, ta, rocblas_operation_none, m, n, k, &one, (const rocblas_double_complex *)A, lda,
            (rocblas_stride)sA, (const rocblas_double_complex *)Bm, ldb, (rocblas_stride)sB, &zero,
            (rocblas_double_complex *)C, ldc, (rocblas_stride)sC, batch));
    }
    const rocblas_float_complex one(1.0f, 0.0f), zero(0.0f, 0.0f);
    return blas(rocblas_cgemm_strided_batched(
        h, ta, rocblas_operation_none, m, n, k, &one, (const rocblas_float_complex *)A, lda,
        (rocblas_stride)sA, (const rocblas_float_complex *)Bm, ldb, (rocblas_stride)sB, &zero,
        (rocblas_float_complex *)C, ldc, (rocblas_stride)sC, batch));
}

size_t lds_bytes(int n0) { return ((size_t)n0 * sp_ld(n0) + 64) * sizeof(double2); }

template <bool ADJ, int PREC>
hipError_t launch_solve(const SpDev &d, int B, const double2 *values, double2 *X, void *Xg,
                        const void *Rp, int nchunk, double rscale, double2 *grad, int32_t *status,
                        hipStream_t st) {
    const int S = B * d.F;
    hipLaunchKernelGGL((k_sp_solve<ADJ, PREC>), dim3(S), dim3(256), lds_bytes(d.n0), st, d, B, values,
                       X, Xg, Rp, nchunk, rscale, grad, status);
    return hipGetLastError();
}

}  // namespace

hipError_t sp_blas_create(void **handle) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return hipErrorOutOfMemory;
    *handle = h;
    return hipSuccess;
}

void sp_blas_destroy(void *handle) {
    if (handle) (void)rocblas_destroy_handle((rocblas_handle)handle);
}

hipError_t sp_prep(const SpDev &d, const double2 *scc, hipStream_t st) {
    hipLaunchKernelGGL(k_sp_prep, dim3(d.n0, d.F), dim3(64), 0, st, d.n0, d.n1, d.F, d.S0, scc,
                       d.exc, d.K, d.r0);
    return hipGetLastError();
}

hipError_t sp_set_lds_limit() {
    const int bytes = (int)lds_bytes(kSpMaxPorts);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_sp_solve<false, 0>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)k_sp_solve<false, 1>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)k_sp_solve<true, 0>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess ||
        (e = hipFuncSetAttribute((const void *)k_sp_solve<true, 1>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    return hipSuccess;
}

hipError_t sp_forward(const SpDev &d, int B, const double2 *values, double2 *X, void *Xg, int prec,
                      int32_t *status, hipStream_t st) {
    return prec == 0 ? launch_solve<false, 0>(d, B, values, X, Xg, nullptr, 0, 0.0, nullptr, status, st)
                     : launch_solve<false, 1>(d, B, values, X, Xg, nullptr, 0, 0.0, nullptr, status, st);
}

hipError_t sp_field(void *handle, const SpDev &d, int B, const double2 *Xg64, double2 *out,
                    hipStream_t st) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidValue;
    const int m = d.P * d.ncomp;
    // out[b][f][p][c]: per frequency a (P ncomp) x B column-major block with ld F P ncomp
    return cgemm(h, 0, rocblas_operation_transpose, m, B, d.n0, d.fields64, d.n0,
                 (size_t)d.P * d.ncomp * d.n0, Xg64, d.n0, (size_t)B * d.n0, out, d.F * m, (size_t)m,
                 d.F);
}

hipError_t sp_loss_and_grad(void *handle, const SpDev &d, const SpWork &w, int B,
                            const double2 *values, const double *T, int comp, int loss_mode, int prec,
                            double *loss, double2 *grad, int32_t *status, hipStream_t st) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidValue;
    hipError_t e = sp_forward(d, B, values, w.X, w.Xg, prec, status, st);
    if (e != hipSuccess) return e;
    const void *fields = prec == 0 ? (const void *)d.fields64 : (const void *)d.fields32;
    const size_t esz = prec == 0 ? sizeof(double2) : sizeof(float2);
    const int lda = d.ncomp * d.n0;
    const size_t sA = (size_t)d.P * d.ncomp * d.n0;
    const bool want_grad = grad != nullptr;
    for (int c = 0; c < w.nchunk; ++c) {
        const int p0 = c * w.rows, nr = std::min(w.rows, d.P - p0);
        const char *A = (const char *)fields + ((size_t)p0 * d.ncomp + comp) * d.n0 * esz;
        // B_comb of the chunk: (nr x n0)(n0 x B) per frequency
        if ((e = cgemm(h, prec, rocblas_operation_transpose, nr, B, d.n0, A, lda, sA, w.Xg, d.n0,
                       (size_t)B * d.n0, w.Y, w.rows, (size_t)B * w.rows, d.F)) != hipSuccess)
            return e;
#define SP_EPI(PR, LS)                                                                         \
    hipLaunchKernelGGL((k_sp_epilogue<PR, LS>), dim3(B, d.F), dim3(256), 0, st, B, d.F, w.rows, \
                       p0, nr, w.Y, T, w.lpart + (size_t)c * d.F * B, want_grad)
        if (prec == 0) {
            if (loss_mode == COSIM_LOSS_MAG) SP_EPI(0, COSIM_LOSS_MAG);
            else SP_EPI(0, COSIM_LOSS_COMPLEX);
        } else {
            if (loss_mode == COSIM_LOSS_MAG) SP_EPI(1, COSIM_LOSS_MAG);
            else SP_EPI(1, COSIM_LOSS_COMPLEX);
        }
#undef SP_EPI
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (!want_grad) continue;
        // conj(fields^H w) of the chunk: (n0 x nr)(nr x B) per frequency
        char *Rc = (char *)w.Rp + (size_t)c * d.F * B * d.n0 * esz;
        if ((e = cgemm(h, prec, rocblas_operation_none, d.n0, B, nr, A, lda, sA, w.Y, w.rows,
                       (size_t)B * w.rows, Rc, d.n0, (size_t)B * d.n0, d.F)) != hipSuccess)
            return e;
    }
    const double scale = 1.0 / ((double)d.F * d.P);
    hipLaunchKernelGGL(k_sp_reduce, dim3((B + 255) / 256), dim3(256), 0, st, B, d.F, w.nchunk,
                       w.lpart, scale, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!want_grad) return hipSuccess;
    return prec == 0 ? launch_solve<true, 0>(d, B, values, w.X, nullptr, w.Rp, w.nchunk, scale, grad,
                                             status, st)
                     : launch_solve<true, 1>(d, B, values, w.X, nullptr, w.Rp, w.nchunk, scale, grad,
                                             status, st);
}

hipError_t sp_to_c64(size_t count, const double2 *a, float2 *b, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sp_to_c64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, a,
                       b);
    return hipGetLastError();
}

hipError_t sp_rc(int B, int F, int n, const double *R, const double *C, const double *omega,
                 double z0, double2 *gam, int ld, hipStream_t st) {
    const size_t t = (size_t)B * F * n;
    if (t == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sp_rc, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, B, F, n, R, C,
                       omega, z0, gam, ld);
    return hipGetLastError();
}

hipError_t sp_rc_backward(int B, int F, int n, const double *R, const double *C, const double *omega,
                          double z0, const double2 *g, int ld, double *gC, hipStream_t st) {
    const size_t t = (size_t)B * n;
    if (t == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sp_rc_backward, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, B, F, n,
                       R, C, omega, z0, g, ld, gC);
    return hipGetLastError();
}

}  // namespace cosim
