// Batched FP64 complex solves of the loop impedance system (Eq. 6 in
// impedance form, Eq. 2 and 11 for Z) on gfx950.
//
// One workgroup per (configuration, frequency) system.  Z (NP x NP complex,
// NP = n padded to 16/32/64 with an identity block) lives in registers: thread
// (ti, tj) owns the 4x4 tile Z[4ti..4ti+3][4tj..4tj+3].  Gauss-Jordan
// elimination with partial pivoting (pivot = largest |re|+|im| among rows not
// yet used, rows are never swapped) eliminates column k from every other row,
// so the solution is read off at the end as x_k = b'_{p_k} / pivot_k with no
// back substitution.  Per step:
//   * the NT lanes owning column k (one column of tiles, always inside one
//     wave) find the pivot with a shuffle reduction and publish the
//     multipliers l_i = a_ik / a_pk through LDS (one block barrier);
//   * inside each wave the owner of the pivot row's tile publishes that tile
//     through LDS (wave-local, no barrier) and every thread applies the rank-1
//     update to its tile; tiles left of column k are skipped.
// The right-hand side is carried by the column of tiles holding column n-1.
// Z is complex symmetric (M symmetric, R and C diagonal), so the same routine
// serves the adjoint system Z^T mu = r.
#include <type_traits>

#include "internal.h"

namespace cosim {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 csub_mul(double2 acc, double2 a, double2 b) {
    // acc - a*b
    return make_double2(acc.x - (a.x * b.x - a.y * b.y), acc.y - (a.x * b.y + a.y * b.x));
}
__device__ inline double2 cinv(double2 a) {
    const double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
}

template <int NP>
struct GJShape {
    static constexpr int NT = NP / 4;
    static constexpr int NTHR = NT * NT;
    static constexpr int BLOCK = NTHR < 64 ? 64 : NTHR;
};

// ADJ = false: rhs = -j w Phi, writes I[s][k].
// ADJ = true : rhs = rscale * sum_c (rr - j ri) of rpart[c][s][:], writes
//              gsys[s][k] = 2 Re(mu_k I_k / (j w C_k^2)).
template <int NP, bool ADJ>
__global__ __launch_bounds__(GJShape<NP>::BLOCK) void k_gj(
    int n, int S, int F, const double *__restrict__ M, const double *__restrict__ Rv,
    const double *__restrict__ phi, const double *__restrict__ C,
    const double *__restrict__ omega, const double2 *__restrict__ Iin,
    const double2 *__restrict__ rpart, int nchunk, double rscale, double2 *__restrict__ Iout,
    double *__restrict__ gsys, int32_t *__restrict__ status, bool or_status) {
    constexpr int NT = GJShape<NP>::NT;
    constexpr int NTHR = GJShape<NP>::NTHR;
    const int s = blockIdx.x;
    const int t = threadIdx.x;
    const bool act = t < NTHR;
    const int ti = t % NT, tj = t / NT;
    const int b = s / F, f = s - b * F;

    __shared__ double2 sL[2][NP];
    __shared__ int sP[2];
    __shared__ double2 sPiv[NP];
    __shared__ int sKof[NP];
    __shared__ double2 sU[NT][4][4];
    __shared__ double2 sRhs[4];
    __shared__ int sFlag;

    if (t == 0) sFlag = 0;
    __syncthreads();

    const double w = omega[f];
    const double *Cb = C + (size_t)b * n;
    const int tb = (n - 1) >> 2;  // column of tiles that carries the rhs

    // ---- build the tile of Z and the rhs ---------------------------------
    double2 a[4][4];
    double2 rhs[4];
    if (act) {
        int flag = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * ti + r;
            double dre = 0.0, dim = 0.0;
            if (i < n) {
                const double c = Cb[i];
                if (tj == 0) {
                    if (!isfinite(c) || c == 0.0 || !isfinite(w) || w == 0.0) flag |= COSIM_SYS_BAD_INPUT;
                    else if (c < 0.0) flag |= COSIM_SYS_NEGATIVE_C;
                }
                dre = Rv[i];
                dim = -1.0 / (w * c);  // 1/(j w C) = -j/(w C)
            }
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const int j = 4 * tj + cc;
                double2 z = make_double2(0.0, 0.0);
                if (i < n && j < n) {
                    z.y = w * M[(size_t)i * n + j];
                    if (i == j) {
                        z.x += dre;
                        z.y += dim;
                    }
                } else if (i == j) {
                    z.x = 1.0;  // identity padding
                }
                a[r][cc] = z;
            }
            rhs[r] = make_double2(0.0, 0.0);
            if (tj == tb && i < n) {
                if (!ADJ) {
                    rhs[r] = make_double2(0.0, -w * phi[i]);
                } else {
                    double rr = 0.0, ri = 0.0;
                    for (int c = 0; c < nchunk; ++c) {
                        const double2 v = rpart[((size_t)c * S + s) * NP + i];
                        rr += v.x;
                        ri += v.y;
                    }
                    rhs[r] = make_double2(rscale * rr, -rscale * ri);
                }
            }
        }
        if (flag) atomicOr(&sFlag, flag);
    }

    // ---- elimination ------------------------------------------------------
    uint64_t used = 0;
    // one elimination step for column k = 4 kt + C; C is a compile-time
    // constant so that every access to the tile a[][] has a constant index
    auto step = [&](int kt, auto cconst) {
        constexpr int c = decltype(cconst)::value;
        const int k = 4 * kt + c;
        if (k >= n) return;  // uniform
        const int buf = k & 1;
        if (act && tj == kt) {
            double best = -1.0;
            int bi = 1 << 30;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * ti + r;
                if (i < n && !((used >> i) & 1ull)) {
                    double m = fabs(a[r][c].x) + fabs(a[r][c].y);
                    if (!(m == m)) m = __builtin_inf();  // NaN rows still yield a valid pivot index
                    if (m > best) {
                        best = m;
                        bi = i;
                    }
                }
            }
#pragma unroll
            for (int off = 1; off < NT; off <<= 1) {
                const double ob = __shfl_xor(best, off, NT);
                const int oi = __shfl_xor(bi, off, NT);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            // every column has an unused valid row, so bi < n; the clamp keeps
            // the index in range whatever the data
            const int p = bi < n ? bi : n - 1;
            const int pr = p & 3;
            // value select (no address select) of the pivot row's entry
            const double m0x = a[0][c].x, m0y = a[0][c].y, m1x = a[1][c].x, m1y = a[1][c].y;
            const double m2x = a[2][c].x, m2y = a[2][c].y, m3x = a[3][c].x, m3y = a[3][c].y;
            const double mx = pr == 0 ? m0x : (pr == 1 ? m1x : (pr == 2 ? m2x : m3x));
            const double my = pr == 0 ? m0y : (pr == 1 ? m1y : (pr == 2 ? m2y : m3y));
            double2 piv;
            piv.x = __shfl(mx, p >> 2, NT);
            piv.y = __shfl(my, p >> 2, NT);
            const bool sing = !(piv.x != 0.0 || piv.y != 0.0);
            const double2 inv = sing ? make_double2(0.0, 0.0) : cinv(piv);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * ti + r;
                sL[buf][i] = (i == p) ? make_double2(0.0, 0.0) : cmul(a[r][c], inv);
            }
            if (ti == 0) {
                sP[buf] = p;
                sPiv[k] = piv;
                sKof[p] = k;
                if (sing) atomicOr(&sFlag, COSIM_SYS_SINGULAR);
            }
        }
        __syncthreads();
        const int p = sP[buf];
        used |= 1ull << p;
        if (act && 4 * tj + 3 >= k) {
            const int pr = p & 3;
            if (ti == (p >> 2)) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) sU[tj][r][cc] = a[r][cc];
                if (tj == tb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sRhs[r] = rhs[r];
                }
            }
            // writer and readers of sU[tj] / sRhs are lanes of one wave
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            double2 u[4], l[4];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) u[cc] = sU[tj][pr][cc];
#pragma unroll
            for (int r = 0; r < 4; ++r) l[r] = sL[buf][4 * ti + r];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) a[r][cc] = csub_mul(a[r][cc], l[r], u[cc]);
            if (tj == tb) {
                const double2 ub = sRhs[pr];
#pragma unroll
                for (int r = 0; r < 4; ++r) rhs[r] = csub_mul(rhs[r], l[r], ub);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    };
    for (int kt = 0; 4 * kt < n; ++kt) {
        step(kt, std::integral_constant<int, 0>{});
        step(kt, std::integral_constant<int, 1>{});
        step(kt, std::integral_constant<int, 2>{});
        step(kt, std::integral_constant<int, 3>{});
    }
    __syncthreads();

    // ---- solution and outputs ---------------------------------------------
    const int flag0 = sFlag;
    const bool bad = (flag0 & (COSIM_SYS_BAD_INPUT | COSIM_SYS_SINGULAR)) != 0;
    int oflag = 0;
    if (act && tj == tb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * ti + r;
            if (i >= n) continue;
            const int k = sKof[i];
            double2 x = cmul(rhs[r], cinv(sPiv[k]));
            if (bad) x = make_double2(__builtin_nan(""), __builtin_nan(""));
            if (!ADJ) {
                Iout[(size_t)s * n + k] = x;
                if (!bad && !(isfinite(x.x) && isfinite(x.y))) oflag |= COSIM_SYS_NONFINITE;
            } else {
                const double2 Ik = Iin[(size_t)s * n + k];
                const double ck = Cb[k];
                // 2 Re(mu I / (j w C^2)) = 2 Im(mu I) / (w C^2)
                const double g = 2.0 * (x.x * Ik.y + x.y * Ik.x) / (w * ck * ck);
                gsys[(size_t)s * n + k] = g;
                if (!bad && !isfinite(g)) oflag |= COSIM_SYS_NONFINITE;
            }
        }
    }
    if (oflag) atomicOr(&sFlag, oflag);
    __syncthreads();
    if (t == 0) {
        if (or_status) status[s] |= sFlag;
        else status[s] = sFlag;
    }
}

__global__ __launch_bounds__(256) void k_reduce(int n, int B, int F, int nchunk,
                                                const double *__restrict__ gsys,
                                                const double *__restrict__ lpart, double lscale,
                                                double *__restrict__ grad,
                                                double *__restrict__ loss) {
    const int b = blockIdx.x;
    const int S = B * F;
    if (grad) {
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            double acc = 0.0;
            for (int f = 0; f < F; ++f) acc += gsys[((size_t)b * F + f) * n + k];
            grad[(size_t)b * n + k] = acc;
        }
    }
    if (threadIdx.x == 0 && loss) {
        double acc = 0.0;
        for (int f = 0; f < F; ++f)
            for (int c = 0; c < nchunk; ++c) acc += lpart[(size_t)c * S + (size_t)b * F + f];
        loss[b] = lscale * acc;
    }
}

template <bool ADJ>
hipError_t launch_gj(int NP, int n, int S, int F, const double *M, const double *R,
                     const double *phi, const double *C, const double *omega, const double2 *Iin,
                     const double2 *rpart, int nchunk, double rscale, double2 *Iout,
                     double *gsys, int32_t *status, bool or_status, hipStream_t st) {
    switch (NP) {
        case 16:
            hipLaunchKernelGGL((k_gj<16, ADJ>), dim3(S), dim3(GJShape<16>::BLOCK), 0, st, n, S,
                               F, M, R, phi, C, omega, Iin, rpart, nchunk, rscale, Iout, gsys,
                               status, or_status);
            break;
        case 32:
            hipLaunchKernelGGL((k_gj<32, ADJ>), dim3(S), dim3(GJShape<32>::BLOCK), 0, st, n, S,
                               F, M, R, phi, C, omega, Iin, rpart, nchunk, rscale, Iout, gsys,
                               status, or_status);
            break;
        case 64:
            hipLaunchKernelGGL((k_gj<64, ADJ>), dim3(S), dim3(GJShape<64>::BLOCK), 0, st, n, S,
                               F, M, R, phi, C, omega, Iin, rpart, nchunk, rscale, Iout, gsys,
                               status, or_status);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_solve_forward(int NP, int n, int S, int F, const double *M_d,
                                const double *R_d, const double *phi_d, const double *C_d,
                                const double *omega_d, double2 *I_d, int32_t *status_d,
                                hipStream_t st) {
    return launch_gj<false>(NP, n, S, F, M_d, R_d, phi_d, C_d, omega_d, nullptr, nullptr, 0, 0.0,
                            I_d, nullptr, status_d, false, st);
}

hipError_t launch_solve_adjoint(int NP, int n, int S, int F, const double *M_d,
                                const double *R_d, const double *C_d, const double *omega_d,
                                const double2 *I_d, const double2 *rpart_d, int nchunk,
                                double rscale, double *gsys_d, int32_t *status_d,
                                bool or_status, hipStream_t st) {
    return launch_gj<true>(NP, n, S, F, M_d, R_d, nullptr, C_d, omega_d, I_d, rpart_d, nchunk,
                           rscale, nullptr, gsys_d, status_d, or_status, st);
}

hipError_t launch_reduce(int n, int B, int F, int nchunk, const double *gsys_d,
                         const double *lpart_d, double lscale, double *grad_d, double *loss_d,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(B), dim3(64), 0, st, n, B, F, nchunk, gsys_d, lpart_d,
                       lscale, grad_d, loss_d);
    return hipGetLastError();
}

}  // namespace cosim
