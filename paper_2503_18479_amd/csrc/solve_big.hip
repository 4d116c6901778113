// Batched FP64 complex solves for more than 64 loops (NP a multiple of 64, up
// to kMaxLoopsBig): Z I = E - j w Phi (Eq. 6 in impedance form) and, Z being
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
//
// When every R_k > 0 the impedance is complex symmetric with a positive
// definite real part, and Z = L D L^T needs no row exchanges (as for the
// smaller systems).  big_factor then runs a blocked LDL^T in panels of 64
// columns, the matrix in HBM and only its lower triangle maintained:
//   1. k_ldl_big_diag: the 64x64 diagonal block factored in LDS (one
//      workgroup per system), written back as L11, D and U11 = D L11^T, with
//      T = L11^-T for step 2;
//   2.-3. k_ldl_big_panel: V21 = A21 T on FP64 matrix cores, then
//      L21 = V21 D^-1 to the lower part, U12 = V21^T to the upper part, a
//      copy of L21 for step 4;
//   4. k_ldl_big_update: A22 -= L21 V21^T (= L21 D L21^T) on the tiles on and
//      below the diagonal, FP64 matrix cores.
// The upper triangle then holds U = D L^T, so with identity swaps the record
// is an LU factor and k_lu_solve serves both.  Systems whose smallest pivot is
// below 1e-5 of the largest |Z_kk| (or not finite), or whose input is invalid,
// are marked and re-factored by k_lu_big with pivoting.
//
// With refinement on, steps 1-4 run on a complex64 copy of Z (diagonal block
// still eliminated in FP64 in LDS; panel and trailing update on FP32 matrix
// cores, half the bytes and twice the peak of FP64), and k_solve_refined
// turns the FP32 factor F into FP64 solutions by iterative refinement:
// x = F^-1 b, then r = b - Z x in FP64 (Z formed on the fly from M, R, C and
// w; it is never stored in FP64) and x += F^-1 r until the next correction is
// predicted below tol |x|.  A system that does not converge is re-factored in
// FP64 with pivoting and solved again.
#include "internal.h"

namespace cosim {

namespace {

constexpr int kPW = 16;    // panel width
constexpr int kTB = 256;   // threads per workgroup
constexpr int kTS = 1024;  // threads per workgroup of the solves: one wave per row of a 16-row block

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

// Factor storage: complex128 (FP64 path) or complex64 (FP32 factor of the
// refined path); arithmetic outside the matrix cores is FP64 either way.
__device__ inline double2 ld2(double2 v) { return v; }
__device__ inline double2 ld2(float2 v) { return make_double2((double)v.x, (double)v.y); }
template <typename T2>
__device__ inline T2 st2(double2 v);
template <>
__device__ inline double2 st2<double2>(double2 v) {
    return v;
}
template <>
__device__ inline float2 st2<float2>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}
template <typename T2>
struct Scal;
template <>
struct Scal<double2> {
    typedef double type;
};
template <>
struct Scal<float2> {
    typedef float type;
};

// One 16x16x4 matrix-core step on FP64 or FP32 operands.  Operand lanes are
// laid out alike (A: row l % 16, k = l / 16; B: k = l / 16, column l % 16);
// accumulator element m of lane group g = l / 16 sits in row g + 4m (FP64)
// or 4g + m (FP32), column l % 16.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline f64x4 mfma4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
    typedef f64x4 type;
};
template <>
struct Acc4<float> {
    typedef f32x4 type;
};
template <typename T>
__device__ inline int acc_row(int g, int m) {
    return sizeof(T) == 8 ? g + 4 * m : 4 * g + m;
}

// One system's view of its instance: the operands of Z and of the right-hand
// side, and where its outputs go.  s is the system's index in its instance.
struct SysRef {
    int n, S, s;
    double w;
    const double *M, *R, *phi, *Cb;  // Cb: the capacitances of the system's configuration
    double2 *I;                      // the instance's [S][n] currents
    const void *rhs;                 // the instance's adjoint sums
    int nchunk;
    double rscale;
    double *gsys;
    double2 *mu;
    int32_t *status;  // the instance's [S] status
};

// The systems of one instance (grid index = system index).
struct OneInst {
    const double *M, *R, *phi, *C, *omega;
    double2 *I;
    const void *rhs;
    double *gsys;
    double2 *mu;
    int32_t *status;
    int n, F, S, nchunk;
    double rscale;
    __device__ SysRef ref(int g) const {
        const int b = g / F, f = g - b * F;
        return SysRef{n, S, g, omega[f], M, R, phi, C + (size_t)b * n, I, rhs, nchunk, rscale,
                      gsys, mu, status};
    }
};

// The systems of up to kGroupMax instances of one padded size, numbered
// instance after instance (GroupArgs, passed by value).
struct GroupSrc {
    GroupArgs g;
    __device__ SysRef ref(int gs) const {
        int j = 0;
        while (j + 1 < g.count && gs >= g.in[j + 1].s0) ++j;
        const GroupInst &e = g.in[j];
        const int s = gs - e.s0, b = s / e.F, f = s - b * e.F;
        return SysRef{e.n, e.S, s, e.omega[f], e.M, e.R, e.phi, e.C + (size_t)b * e.n, e.I, e.rhs,
                      e.nchunk, e.rscale, e.gsys, e.mu, e.status};
    }
};

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

template <class Src>
__global__ __launch_bounds__(kTB) void k_lu_big(int NP, int S, Src src,
                                                double2 *__restrict__ Aall, int *__restrict__ pivall,
                                                const int *__restrict__ only, int want) {
    __shared__ double sm[kTB / 64];
    __shared__ int si[kTB / 64];
    __shared__ int sFlag;
    __shared__ double2 sU[kPW];
    __shared__ double2 sL11[kPW][kPW];
    __shared__ double2 sLt[16][kPW + 1];
    __shared__ double2 sUt[kPW][16 + 1];
    const int s = blockIdx.x;
    if (s >= S) return;  // whole workgroup
    if (only && only[s] != want) return;  // re-factor marked systems only
    const int tid = threadIdx.x;
    double2 *A = Aall + (size_t)s * NP * NP;
    int *piv = pivall + (size_t)s * NP;
    const SysRef r = src.ref(s);
    const int n = r.n;
    const double w = r.w;
    const double *__restrict__ M = r.M;
    const double *__restrict__ Rv = r.R;
    const double *__restrict__ Cb = r.Cb;
    if (tid == 0) sFlag = 0;
    __syncthreads();
    for (int k = tid; k < n; k += kTB) {
        const double c = Cb[k];
        if (isnan(c) || c == 0.0 || !isfinite(w) || w == 0.0) atomicOr(&sFlag, COSIM_SYS_BAD_INPUT);
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
    if (tid == 0) r.status[r.s] = sFlag;
}

// Lower triangle of Z = diag(R) + j w M + diag(1/(j w C)) (identity padding),
// grid (S, NP/16): workgroup y writes rows 16y .. 16y + 15; the one with
// y = 0 also sets the input flags, fmt = kFmtLDL (kFmtNeedsPivot for invalid
// input) and the largest |re| + |im| of a diagonal entry.
template <typename T2, class Src>
__global__ __launch_bounds__(kTB) void k_big_assemble(int NP, int S, Src src,
                                                      T2 *__restrict__ Aall,
                                                      int *__restrict__ fmt,
                                                      double *__restrict__ zmax) {
    __shared__ double sm[kTB / 64];
    __shared__ int si[kTB / 64];
    __shared__ int sFlag;
    const int s = blockIdx.x;
    if (s >= S) return;  // whole workgroup
    const int tid = threadIdx.x;
    T2 *A = Aall + (size_t)s * NP * NP;
    const SysRef r = src.ref(s);
    const int n = r.n;
    const double w = r.w;
    const double *__restrict__ M = r.M;
    const double *__restrict__ Rv = r.R;
    const double *__restrict__ Cb = r.Cb;
    if (tid == 0) sFlag = 0;
    __syncthreads();
    double zm = 0.0;
    const bool first = blockIdx.y == 0;
    for (int k = tid; first && k < n; k += kTB) {
        const double c = Cb[k];
        if (isnan(c) || c == 0.0 || !isfinite(w) || w == 0.0) atomicOr(&sFlag, COSIM_SYS_BAD_INPUT);
        else if (c < 0.0) atomicOr(&sFlag, COSIM_SYS_NEGATIVE_C);
        zm = fmax(zm, fabs(Rv[k]) + fabs(w * M[(size_t)k * n + k] - 1.0 / (w * c)));
    }
    // row i, columns j <= i: lanes along j (coalesced), waves over rows
    for (int i = 16 * blockIdx.y + (tid >> 6); i < 16 * blockIdx.y + 16; i += kTB / 64) {
        for (int j = tid & 63; j <= i; j += 64) {
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
            A[(size_t)i * NP + j] = st2<T2>(make_double2(zr, zi));
        }
    }
    if (!first) return;  // whole workgroup
    int dummy = 0;
    block_amax(zm, dummy, sm, si);  // max over the workgroup (index unused)
    if (tid == 0) {
        r.status[r.s] = sFlag;
        fmt[s] = (sFlag & COSIM_SYS_BAD_INPUT) ? kFmtNeedsPivot : kFmtLDL;
        zmax[s] = zm;
    }
}

// Step 1 of the blocked LDL^T: the diagonal block at k0 (lower triangle in
// HBM) factored in LDS, V (= L D, unscaled) kept in place,
//   a_rc2 -= v_r v_c2 / d_c  for c < c2 <= r,
// in four sub-panels of 16 columns: column by column inside the sub-panel
// (each step touches at most 15 columns), then the rest of the block at once,
// 16 terms per entry with the thread's own row of the sub-panel in registers.
// Then X = L11^-1 of the unit lower L = V D^-1 in 16x16 blocks: the diagonal
// blocks column by column (64 independent substitutions of length 16), then
// X_ij = -X_ii sum_(j <= k < i) L_ik X_kj block by block, for i - j = 1, 2, 3
// (whole blocks at once, one entry per thread).
// Written back: L_rc = v_rc / d_c below the diagonal, d_c on it, U_cr = v_rc
// above it, identity swaps, and T = X^T = L11^-T ([64][64] per system) for
// step 2; a pivot below 1e-5 zmax marks the system.  The arithmetic is FP64
// for either storage type.
template <typename T2>
__global__ __launch_bounds__(kTB) void k_ldl_big_diag(int NP, int k0, int S,
                                                      T2 *__restrict__ Aall,
                                                      int *__restrict__ pivall,
                                                      int *__restrict__ fmt,
                                                      const double *__restrict__ zmax,
                                                      T2 *__restrict__ tinv) {
    __shared__ double2 sa[64][65];
    __shared__ double2 sx[64][65];
    const int s = blockIdx.x;
    if (s >= S) return;  // whole workgroup
    if (fmt[s] != kFmtLDL) return;  // invalid input: left to the pivoted LU
    const int tid = threadIdx.x;
    T2 *A = Aall + (size_t)s * NP * NP + (size_t)k0 * NP + k0;
    for (int e = tid; e < 64 * 64; e += kTB) {
        const int r = e >> 6, c = e & 63;
        sa[r][c] = c <= r ? ld2(A[(size_t)r * NP + c]) : make_double2(0.0, 0.0);
        sx[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int rr = tid >> 2, q = tid & 3;  // four threads per row
    __shared__ double2 sdi[64];          // D^-1
    __shared__ double2 sw[3][16][17];
    for (int c0 = 0; c0 < 64; c0 += 16) {
        const int ce = c0 + 15;  // last column of the sub-panel
        for (int c = c0; c < c0 + 16; ++c) {
            if (rr > c) {
                const double2 l = zmul(sa[rr][c], zinv(sa[c][c]));
                const int hi = min(rr, ce);
                for (int c2 = c + 1 + q; c2 <= hi; c2 += 4) sa[rr][c2] = zfms(sa[rr][c2], l, sa[c2][c]);
            }
            __syncthreads();
        }
        if (tid < 16) sdi[c0 + tid] = zinv(sa[c0 + tid][c0 + tid]);
        __syncthreads();
        if (c0 + 16 < 64 && rr >= c0 + 16) {
            double2 w[16];  // row rr of the sub-panel, scaled by D^-1
#pragma unroll
            for (int m = 0; m < 16; ++m) w[m] = zmul(sa[rr][c0 + m], sdi[c0 + m]);
            for (int c2 = c0 + 16 + q; c2 <= rr; c2 += 4) {
                double2 acc = sa[rr][c2];
#pragma unroll
                for (int m = 0; m < 16; ++m) acc = zfms(acc, w[m], sa[c2][c0 + m]);
                sa[rr][c2] = acc;
            }
        }
        __syncthreads();
    }
    // X = L^-1, L_rc = v_rc / d_c (sx holds the identity, so the blocks above
    // the diagonal stay zero)
    if (tid < 64) {  // diagonal block j, column k
        const int j = tid >> 4, k = tid & 15, b0 = 16 * j;
        double2 x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            double2 acc = make_double2(i == k ? 1.0 : 0.0, 0.0);
#pragma unroll
            for (int m = 0; m < i; ++m)
                if (m >= k) acc = zfms(acc, zmul(sa[b0 + i][b0 + m], sdi[b0 + m]), x[m]);
            x[i] = i < k ? make_double2(0.0, 0.0) : acc;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) sx[b0 + i][b0 + k] = x[i];
    }
    __syncthreads();
    for (int d = 1; d < 4; ++d) {
        const int npair = 4 - d;  // blocks (j + d, j), j < npair
        for (int e = tid; e < npair * 256; e += kTB) {  // W = sum_k L_ik X_kj
            const int j = e >> 8, r = (e >> 4) & 15, c = e & 15, i = j + d;
            double2 acc = make_double2(0.0, 0.0);
            for (int kb = j; kb < i; ++kb)
#pragma unroll 4
                for (int m = 0; m < 16; ++m)
                    acc = zfma(acc, zmul(sa[16 * i + r][16 * kb + m], sdi[16 * kb + m]),
                               sx[16 * kb + m][16 * j + c]);
            sw[j][r][c] = acc;
        }
        __syncthreads();
        for (int e = tid; e < npair * 256; e += kTB) {  // X_ij = -X_ii W
            const int j = e >> 8, r = (e >> 4) & 15, c = e & 15, i = j + d;
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
            for (int m = 0; m < 16; ++m) acc = zfms(acc, sx[16 * i + r][16 * i + m], sw[j][m][c]);
            sx[16 * i + r][16 * j + c] = acc;
        }
        __syncthreads();
    }
    T2 *T = tinv + (size_t)s * 64 * 64;
    for (int e = tid; e < 64 * 64; e += kTB) T[e] = st2<T2>(sx[e & 63][e >> 6]);  // T[k][c] = X[c][k]
    double dmin = __builtin_inf();
    for (int e = tid; e < 64 * 64; e += kTB) {
        const int r = e >> 6, c = e & 63;  // lower part and diagonal by rows
        if (c < r) A[(size_t)r * NP + c] = st2<T2>(zmul(sa[r][c], zinv(sa[c][c])));
        else if (c == r) {
            const double2 d = sa[r][r];
            A[(size_t)r * NP + r] = st2<T2>(d);
            const double ad = fabs(d.x) + fabs(d.y);
            dmin = ad == ad ? fmin(dmin, ad) : 0.0;  // a NaN pivot counts as zero
        }
        const int c2 = e >> 6, r2 = e & 63;  // upper part by rows: U_c2,r2 = v_r2,c2
        if (r2 > c2) A[(size_t)c2 * NP + r2] = st2<T2>(sa[r2][c2]);
    }
    if (tid < 64) pivall[(size_t)s * NP + k0 + tid] = k0 + tid;
    int dummy = 0;
    double neg = -dmin;  // min via the arg-max helper
    __shared__ double sm[kTB / 64];
    __shared__ int si[kTB / 64];
    block_amax(neg, dummy, sm, si);
    if (tid == 0 && !(-neg >= 1e-5 * zmax[s])) fmt[s] = kFmtNeedsPivot;
}

// Steps 2-3 for 64 rows i of the panel below the diagonal block, grid
// (S, m/64): V21 = A21 T (T = L11^-T from step 1) on FP64 matrix cores, then
// L21 = V21 D^-1 to the lower part, U12 = V21^T to the upper part and L21
// again as column-major [64][NP] rows of wt (the A operand of step 4).  The
// rows of A21 are staged in LDS (rows padded to 65 entries); each wave forms
// a 32x32 quarter as 2x2 blocks of 16x16 (the layout of k_ldl_big_update,
// with the contraction index k = 16 g + ks); V goes back through the same
// LDS tile so that every HBM write is a run of consecutive entries.
template <typename T2>
__global__ __launch_bounds__(kTB) void k_ldl_big_panel(int NP, int k0, int S,
                                                       const int *__restrict__ fmt,
                                                       T2 *__restrict__ Aall,
                                                       const T2 *__restrict__ tinv,
                                                       T2 *__restrict__ wt) {
    typedef typename Scal<T2>::type T;
    typedef typename Acc4<T>::type V4;
    __shared__ T2 sv[64][65];
    __shared__ double2 dinv[64];
    const int s = blockIdx.x;
    if (s >= S) return;  // whole workgroup
    if (fmt[s] != kFmtLDL) return;
    const int tid = threadIdx.x;
    T2 *A = Aall + (size_t)s * NP * NP;
    const int i0 = k0 + 64 + 64 * blockIdx.y;  // first row of this block
    if (tid < 64) dinv[tid] = zinv(ld2(A[(size_t)(k0 + tid) * NP + k0 + tid]));
    for (int e = tid; e < 64 * 64; e += kTB) {
        const int r = e >> 6, c = e & 63;
        sv[r][c] = A[(size_t)(i0 + r) * NP + k0 + c];
    }
    __syncthreads();
    const int lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wr = 32 * (wv >> 1), wc = 32 * (wv & 1);
    const T2 *Tm = tinv + (size_t)s * 64 * 64 + (size_t)(16 * g) * 64 + wc + r16;
    V4 Vr[2][2], Vi[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            Vr[bi][bj] = V4{0, 0, 0, 0};
            Vi[bi][bj] = V4{0, 0, 0, 0};
        }
    auto step = [&](int ks, const T2 (&t)[2]) {
        T2 a[2];
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2) a[b2] = sv[wr + 16 * b2 + r16][16 * g + ks];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                Vr[bi][bj] = mfma4(a[bi].x, t[bj].x, Vr[bi][bj]);
                Vr[bi][bj] = mfma4(-a[bi].y, t[bj].y, Vr[bi][bj]);
                Vi[bi][bj] = mfma4(a[bi].x, t[bj].y, Vi[bi][bj]);
                Vi[bi][bj] = mfma4(a[bi].y, t[bj].x, Vi[bi][bj]);
            }
    };
    if constexpr (sizeof(T) == 8) {
        // FP64: the T operands of two steps loaded one pair ahead into the
        // other of two register sets (unrolled: the sets alternate in place)
        T2 t0[2][2], t1[2][2];
        auto load = [&](int ks, T2 (&t)[2][2]) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) t[u][b2] = Tm[(ks + u) * 64 + 16 * b2];
        };
        load(0, t0);
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            load(ks + 2, t1);
            step(ks, t0[0]);
            step(ks + 1, t0[1]);
            if (ks + 4 < 16) load(ks + 4, t0);
            step(ks + 2, t1[0]);
            step(ks + 3, t1[1]);
        }
    } else {
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
            T2 t[2];
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) t[b2] = Tm[ks * 64 + 16 * b2];
            step(ks, t);
        }
    }
    __syncthreads();  // every wave is done reading A21
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                T2 v;
                v.x = Vr[bi][bj][m];
                v.y = Vi[bi][bj][m];
                sv[wr + 16 * bi + acc_row<T>(g, m)][wc + 16 * bj + r16] = v;
            }
    __syncthreads();
    T2 *W = wt + (size_t)s * 64 * NP;
    for (int e = tid; e < 64 * 64; e += kTB) {
        const int r = e >> 6, c = e & 63;
        A[(size_t)(i0 + r) * NP + k0 + c] = st2<T2>(zmul(ld2(sv[r][c]), dinv[c]));
        const int c2 = e >> 6, r2 = e & 63;  // transposed: consecutive threads along rows
        A[(size_t)(k0 + c2) * NP + i0 + r2] = sv[r2][c2];
        W[(size_t)c2 * NP + (i0 - k0 - 64) + r2] = st2<T2>(zmul(ld2(sv[r2][c2]), dinv[c2]));
    }
}

// Step 4: A22 -= L21 V21^T on the 64x64 tiles of the trailing matrix on or
// below the diagonal (a diagonal tile is updated in full; its part above the
// diagonal is never read), nt(nt+1)/2 = T tiles per system, tile
// t = ti(ti+1)/2 + tj.  One-dimensional grid of 8 ceil(S/8) T workgroups,
// mapped so that every tile of a system runs on one XCD and the tiles of a
// system are consecutive there (workgroups are dealt to the 8 XCDs round
// robin): workgroup id -> XCD x = id % 8, its k = id / 8-th workgroup on that
// XCD takes tile k % T of system 8 (k / T) + x.  The L21 and V21 panels of
// the few systems in flight on an XCD then stay in its L2 across their tiles.
// Each wave takes a 32x32 quarter as 2x2 FP64 MFMA blocks of 16x16 (real and
// imaginary accumulators; lane l holds column l%16, rows g + 4m, g = l/16).
// Panel column c enters as MFMA step ks = c % 16 of lane group g = c / 16 for
// both operands, so each lane's operand is one 16-byte load and the 16 lanes
// of a group read 256 consecutive bytes: the A operand from wt (rows of
// L21^T), the B operand from U12 (rows of V21^T).
template <typename T2>
__global__ __launch_bounds__(kTB) void k_ldl_big_update(int NP, int k0, int S,
                                                        const int *__restrict__ fmt,
                                                        T2 *__restrict__ Aall,
                                                        const T2 *__restrict__ wt, int T) {
    typedef typename Scal<T2>::type Ts;
    typedef typename Acc4<Ts>::type V4;
    const int kx = blockIdx.x >> 3;
    const int s = 8 * (kx / T) + (blockIdx.x & 7);
    if (s >= S) return;  // whole workgroup
    if (fmt[s] != kFmtLDL) return;
    const int t = kx % T;
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int base = k0 + 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wi = base + 64 * ti + 32 * (wv >> 1);  // first row of this wave's quarter
    const int wj = base + 64 * tj + 32 * (wv & 1);   // first column
    T2 *A = Aall + (size_t)s * NP * NP;
    // lane's operand streams: L21[wi + 16 bi + r16][16 g + ks] and V21[wj + 16 bj + r16][16 g + ks]
    const T2 *La = wt + (size_t)s * 64 * NP + (size_t)(16 * g) * NP + (wi - base) + r16;
    const T2 *Vb = A + (size_t)(k0 + 16 * g) * NP + wj + r16;
    V4 Cr[2][2], Ci[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            Cr[bi][bj] = V4{0, 0, 0, 0};
            Ci[bi][bj] = V4{0, 0, 0, 0};
        }
    // FP64: operands of two steps at a time, loaded one pair of steps ahead
    // into the other of two register sets (the loop is unrolled, so the sets
    // alternate without copies); the tile's current values are loaded before
    // the last pair of steps, so that the epilogue does not wait for them
    auto load = [&](int ks, T2 (&l)[2][2], T2 (&v)[2][2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                l[u][b2] = La[(size_t)(ks + u) * NP + 16 * b2];
                v[u][b2] = Vb[(size_t)(ks + u) * NP + 16 * b2];
            }
    };
    auto steps = [&](const T2 (&l)[2][2], const T2 (&v)[2][2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    // (lr + j li)(vr + j vi): re = lr vr - li vi, im = lr vi + li vr
                    Cr[bi][bj] = mfma4(l[u][bi].x, v[u][bj].x, Cr[bi][bj]);
                    Cr[bi][bj] = mfma4(-l[u][bi].y, v[u][bj].y, Cr[bi][bj]);
                    Ci[bi][bj] = mfma4(l[u][bi].x, v[u][bj].y, Ci[bi][bj]);
                    Ci[bi][bj] = mfma4(l[u][bi].y, v[u][bj].x, Ci[bi][bj]);
                }
    };
    auto cell = [&](int bi, int bj, int m) {
        return A + (size_t)(wi + 16 * bi + acc_row<Ts>(g, m)) * NP + wj + 16 * bj + r16;
    };
    if constexpr (sizeof(Ts) == 8) {
        T2 l0[2][2], v0[2][2], l1[2][2], v1[2][2], c[2][2][4];
        load(0, l0, v0);
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            load(ks + 2, l1, v1);
            steps(l0, v0);
            if (ks + 4 < 16) {
                load(ks + 4, l0, v0);
            } else {
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                        for (int m = 0; m < 4; ++m) c[bi][bj][m] = *cell(bi, bj, m);
            }
            steps(l1, v1);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    T2 a = c[bi][bj][m];
                    a.x -= Cr[bi][bj][m];
                    a.y -= Ci[bi][bj][m];
                    *cell(bi, bj, m) = a;
                }
    } else {
        // FP32: the operands of four steps loaded as they come, the tile read
        // in the epilogue (more resident waves do the hiding: the prefetching
        // form holds five instead of six and runs 3% slower)
#pragma unroll 4
        for (int ks = 0; ks < 16; ++ks) {
            T2 l[2], v[2];
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                l[b2] = La[(size_t)ks * NP + 16 * b2];
                v[b2] = Vb[(size_t)ks * NP + 16 * b2];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    Cr[bi][bj] = mfma4(l[bi].x, v[bj].x, Cr[bi][bj]);
                    Cr[bi][bj] = mfma4(-l[bi].y, v[bj].y, Cr[bi][bj]);
                    Ci[bi][bj] = mfma4(l[bi].x, v[bj].y, Ci[bi][bj]);
                    Ci[bi][bj] = mfma4(l[bi].y, v[bj].x, Ci[bi][bj]);
                }
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    T2 *cp = cell(bi, bj, m);
                    T2 a = *cp;
                    a.x -= Cr[bi][bj][m];
                    a.y -= Ci[bi][bj][m];
                    *cp = a;
                }
    }
}

// sum of row[j] x[j] over j = j0, j0 + 64, ... < j1 (one lane of the wave
// that owns the row).  Rows have at most kMaxLoopsBig = 16 x 64 entries, so a
// lane has at most 16, loaded in two batches of 8 issued at once: the solves
// walk their blocks of rows one after another and each block is
// latency-bound; a batch is what fits the 128 registers a lane has in a
// 1,024-thread workgroup without spilling.
static_assert(kMaxLoopsBig <= 16 * 64, "at most 16 entries of a row per lane");
// Entries past j1 are loaded from column 0 (always inside the row) and both
// factors replaced by zero, so that the loads need no branches.
template <typename T2>
__device__ inline double2 dot_run(const T2 *__restrict__ row, const double2 *x, int j0, int j1) {
    constexpr int D = 8;
    const double2 z = make_double2(0.0, 0.0);
    double2 a0 = z, a1 = z;
#pragma unroll 1
    for (int e0 = 0; e0 < 16 && j0 + 64 * e0 < j1; e0 += D) {
        T2 v[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
            const int j = j0 + 64 * (e0 + e);
            v[e] = row[j < j1 ? j : 0];
        }
#pragma unroll
        for (int e = 0; e < D; e += 2) {
            const int j = j0 + 64 * (e0 + e);
            const bool in0 = j < j1, in1 = j + 64 < j1;
            a0 = zfma(a0, in0 ? ld2(v[e]) : z, x[in0 ? j : 0]);
            a1 = zfma(a1, in1 ? ld2(v[e + 1]) : z, x[in1 ? j + 64 : 0]);
        }
    }
    return make_double2(a0.x + a1.x, a0.y + a1.y);
}

// The same for a real row (a row of M) against a complex vector, in two
// batches of 8 loads.
__device__ inline double2 dot_real_run(const double *__restrict__ row, const double2 *x, int j0,
                                       int j1) {
    double r0 = 0.0, i0 = 0.0;
#pragma unroll 1
    for (int e0 = 0; e0 < 16 && j0 + 64 * e0 < j1; e0 += 8) {
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = j0 + 64 * (e0 + e);
            v[e] = row[j < j1 ? j : 0];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = j0 + 64 * (e0 + e);
            const bool in = j < j1;
            const double m = in ? v[e] : 0.0;
            const double2 xv = x[in ? j : 0];
            r0 = fma(m, xv.x, r0);
            i0 = fma(m, xv.y, i0);
        }
    }
    return make_double2(r0, i0);
}

// Sum over the 64 lanes of a wave; every lane returns with it.
__device__ inline double2 wave_sum(double2 a) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a.x += __shfl_xor(a.x, off);
        a.y += __shfl_xor(a.y, off);
    }
    return a;
}

// Right-hand side of row k < n of system r: the loop voltage (forward) or
// rscale * conj(sum over chunks of (rr + j ri)) (adjoint).
template <int RHS>
__device__ inline double2 rhs_entry(int k, int NP, const SysRef &r) {
    if (RHS == kRhsExcitation) return loop_voltage(r.phi, r.n, k, r.w);
    const int S = r.S, s = r.s;
    const void *rhs = r.rhs;
    double rr = 0.0, ri = 0.0;
    for (int c = 0; c < r.nchunk; ++c) {
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
    return make_double2(r.rscale * rr, -r.rscale * ri);
}

// sx <- U^-1 L^-1 P sx for one system's LU record A (unit lower L below the
// diagonal, U on and above it; the row swaps piv first when PIV), the vector
// in LDS, the kTS threads of the workgroup taking part: blocks of 16 rows,
// dot products against the solved rows (wave r takes row r of the block and
// stages its diagonal-block entries in LDS), then the 16x16 diagonal block
// inside wave 0.  st: 16 entries, sd: 16 x 17 entries of LDS scratch.
//   The blocks follow one another, so each block's loads of its rows are
// latency on the critical path.  With PF (rows of at most 64 kPf entries),
// the next block's row entries (kPf per lane) and diagonal-block entries are
// loaded while the current block's diagonal part is solved.  Identity swaps
// (the records of the blocked LDL^T) are found by one vote and skipped.
constexpr int kPf = 4;
template <typename T2, bool PIV, bool PF>
__device__ __forceinline__ void lu_apply_inverse(const T2 *__restrict__ A, const int *__restrict__ piv, int NP,
                                 double2 *sx, double2 *st, double2 (*sd)[17]) {
    const int tid = threadIdx.x;
    if (PIV) {
        int moved = 0;
        for (int j = tid; j < NP; j += kTS) moved |= piv[j] != j;
        if (__syncthreads_or(moved)) {
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
        }
    }
    const int r = tid >> 6, q = tid & 63;
    const double2 z = make_double2(0.0, 0.0);
    // PF: entries j = j0 + 64 e (e < kPf) of row r0 + r inside [j0, j1)
    // (others from column 0, always inside the row, and zeroed when used),
    // and the diagonal-block entry of column r0 + (q & 15)
    T2 pf[kPf], pd;
    auto fetch = [&](int r0, int j0, int j1) {
        const T2 *row = A + (size_t)(r0 + r) * NP;
#pragma unroll
        for (int e = 0; e < kPf; ++e) {
            const int j = j0 + 64 * e;
            pf[e] = row[j < j1 ? j : 0];
        }
        pd = row[r0 + (q & 15)];
    };
    // row r0 + r against sx over [j0, j1) (PF: the prefetched entries)
    auto dot = [&](int r0, int j0, int j1) {
        double2 acc = z;
        if constexpr (PF) {
#pragma unroll
            for (int e = 0; e < kPf; ++e) {
                const int j = j0 + 64 * e;
                const bool in = j < j1;
                acc = zfma(acc, in ? ld2(pf[e]) : z, sx[in ? j : 0]);
            }
        } else {
            acc = dot_run(A + (size_t)(r0 + r) * NP, sx, j0, j1);
        }
        return wave_sum(acc);
    };
    auto diag_entry = [&](int r0) {
        if constexpr (PF)
            return ld2(pd);
        else
            return ld2(A[(size_t)(r0 + r) * NP + r0 + (q & 15)]);
    };
    // forward: L y = P b, L unit lower; block r0 uses columns [0, r0)
    if (PF) fetch(0, q, 0);
    for (int r0 = 0; r0 < NP; r0 += 16) {
        if (q < 16) sd[r][q] = diag_entry(r0);
        const double2 acc = dot(r0, q, r0);
        if (PF && r0 + 16 < NP) fetch(r0 + 16, q, r0 + 16);  // in flight across the diagonal block
        if (q == 0) st[r] = make_double2(sx[r0 + r].x - acc.x, sx[r0 + r].y - acc.y);
        __syncthreads();
        if (tid < 64) {
            const int l = tid & 15;
            double2 t = st[l];
#pragma unroll
            for (int k = 0; k < 15; ++k) {
                const double2 yk = make_double2(__shfl(t.x, k), __shfl(t.y, k));
                const double2 lk = l > k ? sd[l][k] : make_double2(0.0, 0.0);
                t = zfms(t, lk, yk);
            }
            if (tid < 16) sx[r0 + l] = t;
        }
        __syncthreads();
    }
    // backward: U x = y; block r0 uses columns [r0 + 16, NP)
    if (PF) fetch(NP - 16, NP + q, NP);
    for (int r0 = NP - 16; r0 >= 0; r0 -= 16) {
        if (q < 16) sd[r][q] = diag_entry(r0);
        const double2 acc = dot(r0, r0 + 16 + q, NP);
        if (PF && r0 >= 16) fetch(r0 - 16, r0 + q, NP);
        if (q == 0) st[r] = make_double2(sx[r0 + r].x - acc.x, sx[r0 + r].y - acc.y);
        __syncthreads();
        if (tid < 64) {
            const int l = tid & 15;
            double2 t = st[l];
#pragma unroll
            for (int k = 15; k >= 0; --k) {
                // lane k finishes x_k; the lanes of the rows above subtract its term
                if (l == k) t = zmul(t, zinv(sd[k][k]));
                const double2 xk = make_double2(__shfl(t.x, k), __shfl(t.y, k));
                const double2 uk = l < k ? sd[l][k] : make_double2(0.0, 0.0);
                t = zfms(t, uk, xk);
            }
            if (tid < 16) sx[r0 + l] = t;
        }
        __syncthreads();
    }
}

// Outputs of a solved system: forward I[s][k]; adjoint gsys[s][k] =
// 2 Re(mu_k I_k / (j w C_k^2)) (and mu when asked for); status bits.
template <int RHS>
__device__ __forceinline__ void write_solution(const SysRef &r, const double2 *sx, int *sFlag) {
    const int tid = threadIdx.x;
    const int n = r.n, s = r.s;
    const double w = r.w;
    const double *__restrict__ Cb = r.Cb;
    double2 *__restrict__ I = r.I;
    double *__restrict__ gsys = r.gsys;
    double2 *__restrict__ mu = r.mu;
    int32_t *__restrict__ status = r.status;
    const int flag = status[s];
    const bool bad = (flag & (COSIM_SYS_BAD_INPUT | COSIM_SYS_SINGULAR)) != 0;
    int oflag = 0;
    for (int k = tid; k < n; k += kTS) {
        double2 x = sx[k];
        if (bad) x = make_double2(__builtin_nan(""), __builtin_nan(""));
        if (RHS == kRhsExcitation) {
            I[(size_t)s * n + k] = x;
            if (!bad && !(isfinite(x.x) && isfinite(x.y))) oflag = COSIM_SYS_NONFINITE;
        } else {
            const double2 Ik = I[(size_t)s * n + k];
            const double ck = Cb[k];
            // 2 Re(mu I / (j w C^2)) = 2 Im(mu I) / (w C^2)
            const double g = 2.0 * (x.x * Ik.y + x.y * Ik.x) / (w * ck * ck);
            gsys[(size_t)s * n + k] = g;
            if (mu) mu[(size_t)s * n + k] = x;
            if (!bad && !isfinite(g)) oflag = COSIM_SYS_NONFINITE;
        }
    }
    if (oflag) atomicOr(sFlag, oflag);
    __syncthreads();
    if (tid == 0 && *sFlag) status[s] = flag | *sFlag;
}

// One workgroup per system (only those with only[s] == want when `only` is
// set): right-hand side, the two triangular solves with the FP64 record,
// outputs.
template <int RHS, class Src>
__global__ __launch_bounds__(kTS) void k_lu_solve(int NP, int S, Src src,
                                                  const double2 *__restrict__ Aall,
                                                  const int *__restrict__ pivall,
                                                  const int *__restrict__ only, int want) {
    __shared__ double2 sx[kMaxLoopsBig];
    __shared__ double2 st[16];
    __shared__ double2 sd[16][17];
    __shared__ int sFlag;
    const int s = blockIdx.x;
    if (s >= S) return;
    if (only && only[s] != want) return;
    const int tid = threadIdx.x;
    const SysRef r = src.ref(s);
    for (int k = tid; k < NP; k += kTS)
        sx[k] = k < r.n ? rhs_entry<RHS>(k, NP, r) : make_double2(0.0, 0.0);
    if (tid == 0) sFlag = 0;
    __syncthreads();
    if (NP <= 64 * kPf)  // uniform over the launch
        lu_apply_inverse<double2, true, true>(Aall + (size_t)s * NP * NP, pivall + (size_t)s * NP,
                                              NP, sx, st, sd);
    else
        lu_apply_inverse<double2, true, false>(Aall + (size_t)s * NP * NP, pivall + (size_t)s * NP,
                                               NP, sx, st, sd);
    write_solution<RHS>(r, sx, &sFlag);
}

// Largest of a and b over the kTS threads, NaN taken as +inf; every thread
// returns with both.  sm: 2 kTS/64 entries of LDS scratch.
__device__ inline void block_max2(double &a, double &b, double *sm) {
    if (!(a == a)) a = __builtin_inf();
    if (!(b == b)) b = __builtin_inf();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a = fmax(a, __shfl_xor(a, off));
        b = fmax(b, __shfl_xor(b, off));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[2 * wv] = a;
        sm[2 * wv + 1] = b;
    }
    __syncthreads();
    a = sm[0];
    b = sm[1];
#pragma unroll
    for (int v = 1; v < kTS / 64; ++v) {
        a = fmax(a, sm[2 * v]);
        b = fmax(b, sm[2 * v + 1]);
    }
    __syncthreads();
}

// Refined solve of the systems factored in FP32 (fmt kFmtLDL, record A32 of
// the blocked LDL^T): x = F^-1 b, then up to max_iter times
//   r = b - Z x   in FP64: (R_k - j/(w C_k)) x_k + j w (M x)_k, rows of M read
//                 by 16 threads each as in the triangular solves;
//   d = F^-1 r,   x += d.
// With d_0 = x_0 the corrections shrink geometrically by about
// |d_i| / |d_(i-1)|, so the error left after step i is estimated as
// |d_i|^2 / |d_(i-1)|; the system is done once that is at most tol |x| and
// |d_i| <= |d_(i-1)| / 2 (max norms).  A system that is not done after
// max_iter steps is marked fail_fmt, writes nothing and is left to the
// pivoted FP64 fallback.
template <int RHS>
__global__ __launch_bounds__(kTS) void k_solve_refined(int NP, int S, OneInst src,
                                                       const float2 *__restrict__ A32all,
                                                       int *__restrict__ fmt, int fail_fmt,
                                                       int max_iter, double tol) {
    __shared__ double2 sb[kMaxLoopsBig];
    __shared__ double2 sx[kMaxLoopsBig];
    __shared__ double2 sr[kMaxLoopsBig];
    __shared__ double2 st[16];
    __shared__ double2 sd[16][17];
    __shared__ double sm[2 * (kTS / 64)];
    __shared__ int sFlag;
    const int s = blockIdx.x;
    if (s >= S) return;
    if (fmt[s] != kFmtLDL) return;  // whole workgroup: handled by the FP64 record
    const int tid = threadIdx.x;
    const SysRef sys = src.ref(s);
    const int n = sys.n;
    const double w = sys.w;
    const double *__restrict__ M = sys.M;
    const double *__restrict__ Rv = sys.R;
    const double *__restrict__ Cb = sys.Cb;
    const float2 *A = A32all + (size_t)s * NP * NP;
    for (int k = tid; k < NP; k += kTS) {
        const double2 v = k < n ? rhs_entry<RHS>(k, NP, sys) : make_double2(0.0, 0.0);
        sb[k] = v;
        sr[k] = v;
    }
    if (tid == 0) sFlag = 0;
    __syncthreads();
    const int r = tid >> 6, q = tid & 63;  // wave r takes row r0 + r of each block
    bool done = false;
    double prev = 0.0;
    // step 0 solves for x_0 (d_0 = x_0); step i >= 1 for the correction d_i
    for (int it = 0; it <= max_iter; ++it) {
        lu_apply_inverse<float2, false, false>(A, nullptr, NP, sr, st, sd);
        double dm = 0.0, xm = 0.0;
        for (int k = tid; k < NP; k += kTS) {
            const double2 d = sr[k];
            double2 x = it == 0 ? make_double2(0.0, 0.0) : sx[k];
            x.x += d.x;
            x.y += d.y;
            sx[k] = x;
            dm = fmax(dm, fabs(d.x) + fabs(d.y));
            xm = fmax(xm, fabs(x.x) + fabs(x.y));
            if (!(d.x == d.x && d.y == d.y)) dm = __builtin_inf();
        }
        block_max2(dm, xm, sm);  // also orders the x updates before the residual
        if (it > 0) done = dm < __builtin_inf() && dm * dm <= tol * xm * prev && dm <= 0.5 * prev;
        prev = dm;
        if (done || it == max_iter) break;
        // r = b - Z x
        for (int r0 = 0; r0 < NP; r0 += 16) {
            const int i = r0 + r;
            double2 acc = make_double2(0.0, 0.0);
            if (i < n) acc = dot_real_run(M + (size_t)i * n, sx, q, n);
            acc = wave_sum(acc);
            if (q == 0) {
                double2 v = make_double2(0.0, 0.0);
                if (i < n) {
                    const double2 xi = sx[i], bi = sb[i];
                    const double zr = Rv[i], zi = -1.0 / (w * Cb[i]);
                    // b - z_ii x_i - j w (M x)_i
                    v.x = bi.x - (zr * xi.x - zi * xi.y) + w * acc.y;
                    v.y = bi.y - (zr * xi.y + zi * xi.x) - w * acc.x;
                }
                sr[i] = v;
            }
        }
        __syncthreads();
    }
    if (!done) {
        if (tid == 0) fmt[s] = fail_fmt;
        return;  // whole workgroup
    }
    write_solution<RHS>(sys, sx, &sFlag);
}

}  // namespace

namespace {

OneInst one_inst(int n, int F, int S, const double *M, const double *R, const double *phi,
                 const double *C, const double *omega, double2 *I, const void *rhs, int nchunk,
                 double rscale, double *gsys, double2 *mu, int32_t *status) {
    OneInst o;
    o.M = M;
    o.R = R;
    o.phi = phi;
    o.C = C;
    o.omega = omega;
    o.I = I;
    o.rhs = rhs;
    o.gsys = gsys;
    o.mu = mu;
    o.status = status;
    o.n = n;
    o.F = F;
    o.S = S;
    o.nchunk = nchunk;
    o.rscale = rscale;
    return o;
}

template <class Src>
hipError_t lu_big_launch(int NP, int S, const Src &src, double2 *A_d, int *piv_d,
                         const int *only, int want, hipStream_t st) {
    hipLaunchKernelGGL(k_lu_big<Src>, dim3(S), dim3(kTB), 0, st, NP, S, src, A_d, piv_d, only, want);
    return hipGetLastError();
}

// Blocked LDL^T of the systems marked kFmtLDL, in the storage type T2.
template <typename T2, class Src>
hipError_t blocked_ldl(const BigFactor &bf, int NP, int S, const Src &src, T2 *A_d, int *piv_d,
                       hipStream_t st) {
    T2 *wt = (T2 *)bf.wt, *tinv = (T2 *)bf.tinv;
    hipLaunchKernelGGL((k_big_assemble<T2, Src>), dim3(S, NP / 16), dim3(kTB), 0, st, NP, S, src,
                       A_d, bf.fmt, bf.zmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int k0 = 0; k0 < NP; k0 += 64) {
        hipLaunchKernelGGL(k_ldl_big_diag<T2>, dim3(S), dim3(kTB), 0, st, NP, k0, S, A_d, piv_d,
                           bf.fmt, bf.zmax, tinv);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int m = NP - k0 - 64;
        if (m == 0) break;
        hipLaunchKernelGGL(k_ldl_big_panel<T2>, dim3(S, m / 64), dim3(kTB), 0, st, NP, k0, S,
                           (const int *)bf.fmt, A_d, (const T2 *)tinv, wt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nt = m / 64, T = nt * (nt + 1) / 2;
        hipLaunchKernelGGL(k_ldl_big_update<T2>, dim3(8 * ((S + 7) / 8) * T), dim3(kTB), 0, st,
                           NP, k0, S, (const int *)bf.fmt, A_d, (const T2 *)wt, T);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class Src>
hipError_t lu_solve_any(int rhs_kind, int NP, int S, const Src &src, const double2 *A_d,
                        const int *piv_d, const int *only, int want, hipStream_t st) {
#define COSIM_LU_SOLVE(K)                                                                    \
    hipLaunchKernelGGL((k_lu_solve<K, Src>), dim3(S), dim3(kTS), 0, st, NP, S, src, A_d, piv_d, \
                       only, want);                                                          \
    break
    switch (rhs_kind) {
        case kRhsExcitation: COSIM_LU_SOLVE(kRhsExcitation);
        case kRhsPairs: COSIM_LU_SOLVE(kRhsPairs);
        case kRhsPlanarF32: COSIM_LU_SOLVE(kRhsPlanarF32);
        case kRhsPlanarF64: COSIM_LU_SOLVE(kRhsPlanarF64);
        default: return hipErrorInvalidValue;
    }
#undef COSIM_LU_SOLVE
    return hipGetLastError();
}

hipError_t refined_any(int rhs_kind, const BigRefine &rf, int NP, int S, const OneInst &src,
                       int *fmt, int fail_fmt, hipStream_t st) {
#define COSIM_REFINED(K)                                                                      \
    hipLaunchKernelGGL(k_solve_refined<K>, dim3(S), dim3(kTS), 0, st, NP, S, src,              \
                       (const float2 *)rf.A32, fmt, fail_fmt, rf.max_iter, rf.tol);           \
    break
    switch (rhs_kind) {
        case kRhsExcitation: COSIM_REFINED(kRhsExcitation);
        case kRhsPairs: COSIM_REFINED(kRhsPairs);
        case kRhsPlanarF32: COSIM_REFINED(kRhsPlanarF32);
        case kRhsPlanarF64: COSIM_REFINED(kRhsPlanarF64);
        default: return hipErrorInvalidValue;
    }
#undef COSIM_REFINED
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lu_big(int NP, int n, int S, int F, const double *M_d, const double *R_d,
                         const double *C_d, const double *omega_d, double2 *A_d, int *piv_d,
                         int32_t *status_d, hipStream_t st) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig) return hipErrorInvalidValue;
    const OneInst src = one_inst(n, F, S, M_d, R_d, nullptr, C_d, omega_d, nullptr, nullptr, 0,
                                 0.0, nullptr, nullptr, status_d);
    return lu_big_launch(NP, S, src, A_d, piv_d, nullptr, 0, st);
}

hipError_t big_factor(const BigFactor &bf, const BigRefine &rf, int NP, int n, int S, int F,
                      const double *M_d, const double *R_d, const double *C_d,
                      const double *omega_d, double2 *A_d, int *piv_d, int32_t *status_d,
                      hipStream_t st) {
    if (!bf.ldl) return launch_lu_big(NP, n, S, F, M_d, R_d, C_d, omega_d, A_d, piv_d, status_d, st);
    if (NP % 64 != 0 || NP > kMaxLoopsBig || !bf.fmt || !bf.zmax || !bf.wt || !bf.tinv)
        return hipErrorInvalidValue;
    if (rf.on && !rf.A32) return hipErrorInvalidValue;
    const OneInst src = one_inst(n, F, S, M_d, R_d, nullptr, C_d, omega_d, nullptr, nullptr, 0,
                                 0.0, nullptr, nullptr, status_d);
    hipError_t e = rf.on ? blocked_ldl<float2>(bf, NP, S, src, (float2 *)rf.A32, piv_d, st)
                         : blocked_ldl<double2>(bf, NP, S, src, A_d, piv_d, st);
    if (e != hipSuccess) return e;
    // pivoted FP64 LU (from a fresh Z) for the systems marked on the way
    return lu_big_launch(NP, S, src, A_d, piv_d, bf.fmt, kFmtNeedsPivot, st);
}

hipError_t big_solve(const BigFactor &bf, const BigRefine &rf, int NP, int n, int S, int F,
                     const double *M_d, const double *R_d, const double *phi_d, const double *C_d,
                     const double *omega_d, double2 *A_d, int *piv_d, double2 *I_d, int rhs_kind,
                     const void *rhs_d, int nchunk, double rscale, double *gsys_d,
                     int32_t *status_d, hipStream_t st, double2 *mu_d) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig) return hipErrorInvalidValue;
    const OneInst src = one_inst(n, F, S, M_d, R_d, phi_d, C_d, omega_d, I_d, rhs_d, nchunk,
                                 rscale, gsys_d, mu_d, status_d);
    if (!(bf.ldl && rf.on)) return lu_solve_any(rhs_kind, NP, S, src, A_d, piv_d, nullptr, 0, st);
    const bool fwd = rhs_kind == kRhsExcitation;
    const int fail = fwd ? kFmtRefineFailed : kFmtRefineFailedAdj;
    hipError_t e;
    // 1. the FP32 records, refined
    if ((e = refined_any(rhs_kind, rf, NP, S, src, bf.fmt, fail, st)) != hipSuccess) return e;
    // 2. systems that already hold an FP64 record
    const int have[2] = {kFmtNeedsPivot, kFmtRefineFailed};
    for (int h = 0; h < (fwd ? 1 : 2); ++h)
        if ((e = lu_solve_any(rhs_kind, NP, S, src, A_d, piv_d, bf.fmt, have[h], st)) != hipSuccess)
            return e;
    // 3. systems whose refinement did not converge just now: pivoted FP64
    // record from a fresh Z, then the FP64 solve
    if ((e = lu_big_launch(NP, S, src, A_d, piv_d, bf.fmt, fail, st)) != hipSuccess) return e;
    return lu_solve_any(rhs_kind, NP, S, src, A_d, piv_d, bf.fmt, fail, st);
}

hipError_t launch_lu_solve(int NP, int n, int S, int F, const double2 *A_d, const int *piv_d,
                           const double *phi_d, const double *C_d, const double *omega_d,
                           double2 *I_d, int rhs_kind, const void *rhs_d, int nchunk,
                           double rscale, double *gsys_d, int32_t *status_d, hipStream_t st,
                           double2 *mu_d) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig) return hipErrorInvalidValue;
    const OneInst src = one_inst(n, F, S, nullptr, nullptr, phi_d, C_d, omega_d, I_d, rhs_d,
                                 nchunk, rscale, gsys_d, mu_d, status_d);
    return lu_solve_any(rhs_kind, NP, S, src, A_d, piv_d, nullptr, 0, st);
}

hipError_t big_group_factor(const BigFactor &bf, const GroupArgs &g, int NP, int S,
                            double2 *A_d, int *piv_d, hipStream_t st) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig || g.count < 1 || g.count > kGroupMax || !bf.fmt ||
        !bf.zmax || !bf.wt || !bf.tinv)
        return hipErrorInvalidValue;
    const GroupSrc src{g};
    hipError_t e = blocked_ldl<double2>(bf, NP, S, src, A_d, piv_d, st);
    if (e != hipSuccess) return e;
    return lu_big_launch(NP, S, src, A_d, piv_d, bf.fmt, kFmtNeedsPivot, st);
}

hipError_t big_group_solve(const GroupArgs &g, int NP, int S, const double2 *A_d,
                           const int *piv_d, int rhs_kind, hipStream_t st) {
    if (NP % 64 != 0 || NP > kMaxLoopsBig || g.count < 1 || g.count > kGroupMax)
        return hipErrorInvalidValue;
    const GroupSrc src{g};
    return lu_solve_any(rhs_kind, NP, S, src, A_d, piv_d, nullptr, 0, st);
}

}  // namespace cosim
