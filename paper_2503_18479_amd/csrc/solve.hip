// Batched FP64 complex solves of the loop impedance system (Eq. 6 in
// impedance form, Eq. 2 and 11 for Z) on gfx950.
//
// One workgroup per (configuration, frequency) system.  Z (NP x NP complex,
// NP = n padded to 16/32/64 with an identity block) lives in registers: thread
// (ti, tj) owns the 4x4 tile Z[4ti..4ti+3][4tj..4tj+3]; the NT threads of a
// column of tiles (a "column group") are consecutive lanes of one wave.
// Gauss-Jordan elimination with partial pivoting (pivot = largest |re|+|im|
// among rows not yet used; rows are never swapped) eliminates each column from
// every other row, so the solution is read off at the end as
// x_k = b'_{p_k} / pivot_k with no back substitution.  Columns are processed
// in panels of 4 (see k_gj); the right-hand side is carried by the column
// group holding column n-1.  Z is complex symmetric (M symmetric, R and C
// diagonal), so the same routine serves the adjoint system Z^T mu = r.
#include <type_traits>

#include "internal.h"

namespace cosim {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cinv(double2 a) {
    const double d = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * d, -a.y * d);
}
// 1/a for a pivot known to be a normal, finite number away from zero or
// flagged afterwards: hardware reciprocal and two Newton steps (relative error
// at the level of the rounding of the result), no IEEE division sequence.
__device__ inline double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ inline double2 cinv_nr(double2 a) {
    const double d = rcp_nr(fma(a.x, a.x, a.y * a.y));
    return make_double2(a.x * d, -a.y * d);
}

template <int NP>
struct GJShape {
    static constexpr int NT = NP / 4;
    static constexpr int NTHR = NT * NT;
    static constexpr int BLOCK = NTHR < 64 ? 64 : NTHR;
};

// acc - l*u with explicit fused multiply-adds (4 per complex product)
__device__ inline double2 cfms(double2 acc, double2 l, double2 u) {
    double2 r;
    r.x = fma(-l.x, u.x, fma(l.y, u.y, acc.x));
    r.y = fma(-l.x, u.y, fma(-l.y, u.x, acc.y));
    return r;
}

template <int CTRL>
__device__ inline int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}

// (magnitude, row) arg-max step with a DPP partner; ties -> lower row
template <int CTRL>
__device__ inline void amax_step(float &m, int &idx) {
    const float m2 = __int_as_float(dpp_i<CTRL>(__float_as_int(m)));
    const int i2 = dpp_i<CTRL>(idx);
    const bool take = (m2 > m) || (m2 == m && i2 < idx);
    m = take ? m2 : m;
    idx = take ? i2 : idx;
}

// arg-max over the NT lanes of a column group (NT = 4, 8 or 16 consecutive
// lanes inside one DPP row); every lane of the group ends with the result
template <int NT>
__device__ inline void group_amax(float &m, int &idx) {
    amax_step<0xB1>(m, idx);                    // quad_perm [1,0,3,2]
    amax_step<0x4E>(m, idx);                    // quad_perm [2,3,0,1]
    if (NT >= 8) amax_step<0x141>(m, idx);      // row_half_mirror
    if (NT >= 16) amax_step<0x140>(m, idx);     // row_mirror
}

// value of a double held by lane `src` (wave-uniform index) for every lane
__device__ inline double readlane_d(double x, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}

// ADJ = false: rhs = E - j w Phi (loop_voltage), writes I[s][k].
// ADJ = true : rhs = rscale * sum_c (rr - j ri) of rpart[c][s][:], writes
//              gsys[s][k] = 2 Re(mu_k I_k / (j w C_k^2)).
//
// Blocked Gauss-Jordan, panels of 4 columns.  Panel kt is owned by the lane
// group tj == kt, which runs the four pivot steps on its own 4 columns
// (arg-max by DPP, pivot-row entries by readlane, no barrier) and
// publishes the multiplier columns l_c (c = 0..3) and pivot rows p_c through
// LDS.  After one block barrier every other column group applies the
// composite rank-4 update  a_ij -= sum_c l_c[i] u_cj  with
//   u_cj = a_{p_c j} - sum_{c' < c} l_{c'}[p_c] u_{c' j}
// (the pivot row of step c as it stands after steps c' < c), i.e. u = W a_p
// with W = (I + N)^-1, N[c][c'] = l_{c'}[p_c]; the panel group publishes W.
// Column groups left of the panel hold only eliminated columns and skip the
// update.
// One system s (block-uniform) of a plan with n loops, S systems, F
// frequencies; the kernels below call it for their own system index.
template <int NP, bool ADJ>
__device__ __forceinline__ void gj_system(
    int s, int n, int S, int F, const double *__restrict__ M, const double *__restrict__ Rv,
    const double *__restrict__ phi, const double *__restrict__ C,
    const double *__restrict__ omega, const double2 *__restrict__ Iin,
    const double2 *__restrict__ rpart, int nchunk, double rscale, double2 *__restrict__ Iout,
    double *__restrict__ gsys, int32_t *__restrict__ status, bool or_status,
    GJFactor fac, bool fallback_only) {
    constexpr int NT = GJShape<NP>::NT;
    constexpr int NTHR = GJShape<NP>::NTHR;
    // fallback launch: only systems the LDL^T fast path handed over
    if (fallback_only && fac.fmt[s] != kFmtNeedsPivot) return;  // uniform per block
    const int t = threadIdx.x;
    const bool act = t < NTHR;
    const int ti = t % NT, tj = t / NT;
    const int b = s / F, f = s - b * F;

    __shared__ double2 sL[2][4][NP];      // multiplier columns of a panel
    __shared__ int sP[2][4];              // pivot rows of a panel
    __shared__ double2 sPiv[NP];
    __shared__ int sKof[NP];
    __shared__ double2 sU[NT][4][4][4];   // [group][step c][row in tile][col in tile]
    __shared__ double2 sUu[NT][4][4];     // [group][step c][col in tile]: u_c of the group's columns
    __shared__ double2 sW[2][4][4];       // W = (I + N)^-1, N[c][c'] = l_c'[p_c] (c' < c)
    __shared__ double2 sRb[4][4];         // rhs tiles of the pivot-row owners
    __shared__ int sFlag;

    if (t == 0) sFlag = 0;
    __syncthreads();

    const double w = omega[f];
    const double *Cb = C + (size_t)b * n;
    const int tb = (n - 1) >> 2;  // column group that carries the rhs

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
                    if (isnan(c) || c == 0.0 || !isfinite(w) || w == 0.0) flag |= COSIM_SYS_BAD_INPUT;
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
                    rhs[r] = loop_voltage(phi, n, i, w);
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

    // ---- elimination, one panel of 4 columns per iteration ------------------
    uint64_t used = 0;
    for (int kt = 0; 4 * kt < n; ++kt) {
        const int buf = kt & 1;
        const int nc = min(4, n - 4 * kt);  // real columns in this panel
        // -- panel factorisation by the owning column group
        if (act && tj == kt) {
            // first lane of this column group (the group is the only active one here)
            const int gbase = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & 63));
            int pc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                pc[c] = 0;
                if (c >= nc) continue;  // uniform
                // pivot search on |re| + |im| rounded to float: any near-maximal
                // pivot is as good, and the float arg-max needs 2 DPP moves per round
                float best = -1.0f;
                int bi = 1 << 30;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * ti + r;
                    if (i < n && !((used >> i) & 1ull)) {
                        float m = (float)(fabs(a[r][c].x) + fabs(a[r][c].y));
                        if (!(m == m)) m = __builtin_inff();  // NaN rows still yield a pivot
                        if (m > best) {
                            best = m;
                            bi = i;
                        }
                    }
                }
                group_amax<NT>(best, bi);
                // the group's lanes agree on the pivot: make it wave-uniform; an unused
                // valid row always exists and the clamp keeps the index in range
                int p = __builtin_amdgcn_readfirstlane(bi);
                p = p < n ? p : n - 1;
                const int pr = p & 3;
                const int src = gbase + (p >> 2);  // lane holding row p
                auto rowsel = [&](int cc, bool im) {
                    const double v0 = im ? a[0][cc].y : a[0][cc].x, v1 = im ? a[1][cc].y : a[1][cc].x;
                    const double v2 = im ? a[2][cc].y : a[2][cc].x, v3 = im ? a[3][cc].y : a[3][cc].x;
                    return pr == 0 ? v0 : (pr == 1 ? v1 : (pr == 2 ? v2 : v3));
                };
                const double2 piv = make_double2(readlane_d(rowsel(c, false), src),
                                                 readlane_d(rowsel(c, true), src));
                const bool sing = !(piv.x != 0.0 || piv.y != 0.0);
                const double2 inv = sing ? make_double2(0.0, 0.0) : cinv(piv);
                double2 l[4];
                double2 *lcol = fac.L ? fac.L + ((size_t)s * NP + 4 * kt + c) * NP : nullptr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * ti + r;
                    l[r] = (i == p) ? make_double2(0.0, 0.0) : cmul(a[r][c], inv);
                    sL[buf][c][i] = l[r];
                    if (lcol) lcol[i] = l[r];
                }
                // remaining panel columns: a_ic' -= l_i a_pc'
#pragma unroll
                for (int c2 = c + 1; c2 < 4; ++c2) {
                    const double2 up = make_double2(readlane_d(rowsel(c2, false), src),
                                                    readlane_d(rowsel(c2, true), src));
#pragma unroll
                    for (int r = 0; r < 4; ++r) a[r][c2] = cfms(a[r][c2], l[r], up);
                }
                used |= 1ull << p;
                pc[c] = p;
                if (ti == 0) {
                    sPiv[4 * kt + c] = piv;
                    sKof[p] = 4 * kt + c;
                    if (sing) atomicOr(&sFlag, COSIM_SYS_SINGULAR);
                    if (fac.L) {
                        fac.piv_row[(size_t)s * NP + 4 * kt + c] = p;
                        fac.piv_val[(size_t)s * NP + 4 * kt + c] = piv;
                    }
                }
            }
            if (ti == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sP[buf][c] = pc[c];
            }
            // W = (I + N)^-1 (unit lower triangular) so that the pivot rows as
            // they stand at their own step are u = W a_p (a_p: rows before the panel)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (ti == 0) {
                double2 N[4][4], Wm[4][4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < 4; ++c2) {
                        N[c][c2] = (c2 < c && c < nc) ? sL[buf][c2][pc[c]] : make_double2(0.0, 0.0);
                        Wm[c][c2] = make_double2(c == c2 ? 1.0 : 0.0, 0.0);
                    }
#pragma unroll
                for (int c = 1; c < 4; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < c; ++c2) {
                        double2 v = make_double2(0.0, 0.0);
#pragma unroll
                        for (int c3 = c2; c3 < c; ++c3) v = cfms(v, N[c][c3], Wm[c3][c2]);
                        Wm[c][c2] = v;
                    }
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < 4; ++c2) sW[buf][c][c2] = Wm[c][c2];
            }
            if (nc < 4) {  // unused steps of a ragged last panel contribute nothing
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c >= nc)
#pragma unroll
                        for (int r = 0; r < 4; ++r) sL[buf][c][4 * ti + r] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        int pc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pc[c] = sP[buf][c];
        if (!(act && tj == kt)) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nc) used |= 1ull << pc[c];
        }
        const bool upd_tile = act && tj > kt;
        const bool upd_rhs = act && tj == tb;
        if (upd_tile || upd_rhs) {
            // pivot-row owners of this column group publish their tiles / rhs
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c < nc && ti == (pc[c] >> 2)) {
                    if (upd_tile) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int cc = 0; cc < 4; ++cc) sU[tj][c][r][cc] = a[r][cc];
                    }
                    if (upd_rhs) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) sRb[c][r] = rhs[r];
                    }
                }
            }
            // writers and readers are lanes of one wave
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (upd_tile) {
                // lane ti forms u[c][cc] for c = ti / 4, cc = ti % 4 (NT >= 16), or a
                // strided share of the 16 entries (NT < 16)
                for (int e = ti; e < 16; e += NT) {
                    const int c = e >> 2, cc = e & 3;
                    double2 v = make_double2(0.0, 0.0);
                    if (c < nc) {
                        for (int c2 = 0; c2 <= c; ++c2) {
                            const double2 wv = sW[buf][c][c2];
                            const double2 ap = sU[tj][c2][pc[c2] & 3][cc];
                            v.x = fma(wv.x, ap.x, fma(-wv.y, ap.y, v.x));
                            v.y = fma(wv.x, ap.y, fma(wv.y, ap.x, v.y));
                        }
                    }
                    sUu[tj][c][cc] = v;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c >= nc) continue;  // uniform
                    double2 lr[4], uc[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) lr[r] = sL[buf][c][4 * ti + r];
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) uc[cc] = sUu[tj][c][cc];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cc = 0; cc < 4; ++cc) a[r][cc] = cfms(a[r][cc], lr[r], uc[cc]);
                }
            }
            if (upd_rhs) {
                double2 bp[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) bp[c] = c < nc ? sRb[c][pc[c] & 3] : make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c >= nc) continue;  // uniform
                    double2 ub = make_double2(0.0, 0.0);
#pragma unroll
                    for (int c2 = 0; c2 <= c; ++c2) {
                        const double2 wv = sW[buf][c][c2];
                        ub.x = fma(wv.x, bp[c2].x, fma(-wv.y, bp[c2].y, ub.x));
                        ub.y = fma(wv.x, bp[c2].y, fma(wv.y, bp[c2].x, ub.y));
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) rhs[r] = cfms(rhs[r], sL[buf][c][4 * ti + r], ub);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
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
                if (Iout) Iout[(size_t)s * n + k] = x;  // the adjoint solution mu, on request
                if (!bad && !isfinite(g)) oflag |= COSIM_SYS_NONFINITE;
            }
        }
    }
    if (oflag) atomicOr(&sFlag, oflag);
    __syncthreads();
    if (t == 0) {
        if (or_status) status[s] |= sFlag;
        else status[s] = sFlag;
        if (fac.L) fac.fmt[s] = kFmtGJ;
    }
}

// One block per system.
template <int NP, bool ADJ>
__global__ __launch_bounds__(GJShape<NP>::BLOCK) void k_gj(
    int n, int S, int F, const double *__restrict__ M, const double *__restrict__ Rv,
    const double *__restrict__ phi, const double *__restrict__ C,
    const double *__restrict__ omega, const double2 *__restrict__ Iin,
    const double2 *__restrict__ rpart, int nchunk, double rscale, double2 *__restrict__ Iout,
    double *__restrict__ gsys, int32_t *__restrict__ status, bool or_status,
    GJFactor fac, bool fallback_only) {
    gj_system<NP, ADJ>(blockIdx.x, n, S, F, M, Rv, phi, C, omega, Iin, rpart, nchunk, rscale,
                       Iout, gsys, status, or_status, fac, fallback_only);
}

// Member of a group that holds global system sg (wave-uniform): members are
// stored in order of their first system s0.
__device__ __forceinline__ int group_member(const SmallGroup &g, int sg) {
    int i = 0;
    while (i + 1 < g.count && sg >= g.in[i + 1].s0) ++i;
    return i;
}

// The forward fallback of a group's systems: one block per system, only those
// the factorisation marked.
template <int NP>
__global__ __launch_bounds__(GJShape<NP>::BLOCK) void k_gj_group(SmallGroup g) {
    const int sg = blockIdx.x;
    const SmallInst &e = g.in[group_member(g, sg)];
    gj_system<NP, false>(sg - e.s0, e.n, e.S, e.F, e.M, e.R, e.phi, e.C, e.omega, nullptr, nullptr,
                         0, 0.0, e.I, nullptr, e.status, false, e.fac, true);
}

// Sum of a complex value over the 64 lanes of a wave (all lanes active):
// DPP butterflies inside each row of 16, then the four row sums.
template <int CTRL>
__device__ inline double dpp_sum_step(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
    return v + __hiloint2double(hi, lo);
}
__device__ inline double wave_sum(double v) {
    v = dpp_sum_step<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_sum_step<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_sum_step<0x141>(v);  // row_half_mirror
    v = dpp_sum_step<0x140>(v);  // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// One butterfly stage of a transposed reduction: lanes with `upper` keep the
// upper half of their values and send the lower half to the DPP partner,
// which does the opposite; each keeps the pair sum of its half.
template <int CTRL, int N>
__device__ inline void halve(const double (&v)[2 * N], double (&w)[N], bool upper) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double send = upper ? v[j] : v[j + N];
        const double keep = upper ? v[j + N] : v[j];
        w[j] = keep + dpp_d<CTRL>(send);
    }
}
// Sixteen wave sums at once: returns, in lane l, the sum over all 64 lanes
// of v[l & 15].  Within each row of 16 lanes the partners are 15 - i
// (row_mirror), the mirror inside each half row, then i ^ 2 and i ^ 1, so
// lane i keeps value index i; the four row results are then added across
// rows (lane ^ 16, lane ^ 32).
__device__ inline double wave_sum16(const double (&v)[16], int lane) {
    double w8[8], w4[4], w2[2], w1[1];
    halve<0x140, 8>(v, w8, (lane & 8) != 0);
    halve<0x141, 4>(w8, w4, (lane & 4) != 0);
    halve<0x4E, 2>(w4, w2, (lane & 2) != 0);
    halve<0xB1, 1>(w2, w1, (lane & 1) != 0);
    double t = w1[0];
    t += __shfl_xor(t, 16);
    t += __shfl_xor(t, 32);
    return t;
}

// Back substitution L^T x = z with the packed LDL^T record Ls of one system,
// one wave, lane i holding z_i on entry and x_i on return (0 beyond n).
// Columns go in blocks of U = 8, [k0, k1), from the bottom.  The terms with
// i >= k1 (x_i final) of the block's 8 columns are summed over the lanes
// through LDS: lane i stores its 8 products L_{i,k0+u} x_i as row i of red
// (rows padded to 9 entries, so 16 consecutive lanes hit distinct banks),
// lane l adds up column l % 8 over every 8th row starting at row l / 8, and
// three butterfly steps combine the 8 partial sums.  The terms inside the
// block use L's 8x8 diagonal block, transposed through LDS (tr) so that lane
// k0 + u holds row entries L_{k0+ii, k0+u}, and x_{k0+ii} broadcast from its
// lane as soon as it is final.  Each lane reads only its own row of L
// (entries L_{lane,k}, 0 unless k < lane < n).  red: NP x 9 double2, tr: 64
// (NP = 64) or 128 double2 of the wave's LDS.
constexpr int kBsU = 8;
template <int NP>
__device__ __forceinline__ void bs_load(double2 (&l)[kBsU], const double2 *__restrict__ Ls, int n,
                                        int lane, int k0) {
#pragma unroll
    for (int u = 0; u < kBsU; ++u) {
        const int k = k0 + u;
        l[u] = (lane > k && lane < n) ? Ls[ldl_col(NP, k) + lane - k - 1] : make_double2(0.0, 0.0);
    }
}
// One block [k1 - U, k1) from l (the lanes' row entries of its columns);
// then k1 -= U.  Two LDS exchanges: (1) every lane stores its products and
// the block's lanes their rows of the diagonal block; (2) lane l stores the
// sum of column l % 8 over rows l / 8, l / 8 + 8, ..., and the block's lanes
// read their transposed row entries; then each block lane adds up the 8
// partial sums of its own column.
template <int NP>
__device__ __forceinline__ void bs_block(double2 &x, int &k1, const double2 (&l)[kBsU], int lane,
                                         double2 *red, double2 *tr) {
    constexpr int U = kBsU, RS = U + 1;
    const int cu = lane & (U - 1), part = lane / U;  // column and first row this lane sums
    const int k0 = k1 - U;
    const int ub = (lane - k0) & (U - 1);  // column of the block lane k0 + ub owns
    const bool ext = lane >= k1, blk = lane >= k0 && lane < k1;
    const double2 xe = make_double2(ext ? x.x : 0.0, ext ? x.y : 0.0);
    // U x U partial sums: in the pad column of red when it has 64 rows
    auto psum = [&](int i) -> double2 & { return NP >= 64 ? red[i * RS + U] : tr[U * U + i]; };
    if (lane < NP) {
#pragma unroll
        for (int u = 0; u < U; ++u) red[lane * RS + u] = cmul(l[u], xe);
    }
    if (blk) {
#pragma unroll
        for (int u = 0; u < U; ++u) tr[ub * U + u] = l[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < NP / U; ++r) {
        const double2 t = red[(r * U + part) * RS + cu];
        acc.x += t.x;
        acc.y += t.y;
    }
    psum(part * U + cu) = acc;
    double2 t[U];
#pragma unroll
    for (int ii = 1; ii < U; ++ii) t[ii] = blk ? tr[ii * U + ub] : make_double2(0.0, 0.0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (blk) {
        double er = 0.0, ei = 0.0;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double2 e = psum(q * U + ub);
            er += e.x;
            ei += e.y;
        }
        x = make_double2(x.x - er, x.y - ei);
    }
#pragma unroll
    for (int ii = U - 1; ii >= 1; --ii) {
        const double2 xk = make_double2(readlane_d(x.x, k0 + ii), readlane_d(x.y, k0 + ii));
        x = cfms(x, t[ii], xk);  // t[ii] = 0 unless lane < k0 + ii in the block
    }
    // the next block's stores wait for this block's reads
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    k1 = k0;
}
// The columns left of the last whole block, one at a time by wave sums.
__device__ __forceinline__ double2 bs_tail(double2 x, int k1, const double2 *__restrict__ Ls,
                                           int NP, int n, int lane) {
    for (int k = k1 - 1; k >= 0; --k) {
        const double2 l = (lane > k && lane < n) ? Ls[ldl_col(NP, k) + lane - k - 1]
                                                 : make_double2(0.0, 0.0);
        const double pr = l.x * x.x - l.y * x.y;
        const double pi = l.x * x.y + l.y * x.x;
        const double sr = wave_sum(pr), si = wave_sum(pi);
        if (lane == k) x = make_double2(x.x - sr, x.y - si);
    }
    return x;
}
// Any n: loads run DEPTH (1 or 2) blocks ahead, from a ring of DEPTH + 1
// register sets that rotate without copies (the block loop is unrolled).
template <int NP, int DEPTH>
__device__ __forceinline__ double2 ldl_backward(double2 x, const double2 *__restrict__ Ls, int n,
                                                int lane, double2 *red, double2 *tr) {
    constexpr int U = kBsU;
    static_assert(DEPTH == 1 || DEPTH == 2, "one or two blocks ahead");
    int k1 = n;  // columns >= k1 are done
    double2 s0[U], s1[U], s2[U];
    if (n >= U) bs_load<NP>(s0, Ls, n, lane, n - U);
    if (DEPTH == 2 && n >= 2 * U) bs_load<NP>(s1, Ls, n, lane, n - 2 * U);
    auto step = [&](const double2(&l)[U], double2(&fill)[U]) {
        if (k1 - U >= DEPTH * U) bs_load<NP>(fill, Ls, n, lane, k1 - U - DEPTH * U);
        bs_block<NP>(x, k1, l, lane, red, tr);
    };
    while (k1 >= U) {
        if constexpr (DEPTH == 1) {
            step(s0, s1);
            if (k1 < U) break;
            step(s1, s0);
        } else {
            step(s0, s2);
            if (k1 < U) break;
            step(s1, s0);
            if (k1 < U) break;
            step(s2, s1);
        }
    }
    return bs_tail(x, k1, Ls, NP, n, lane);
}
// Complex-symmetric LDL^T factorisation without pivoting, Z = L D L^T.
// The Hermitian part of Z is diag(R) (j w M and 1/(j w C) are skew-Hermitian),
// so with every R_k > 0 each Schur complement keeps a positive-definite real
// part and no pivot can vanish; the elimination needs no row exchanges and
// touches only the lower triangle.
//
// One wave per system.  The lower triangle is held as NB(NB+1)/2 blocks of
// 16x16 (NB = NP/16), each as two FP64 matrix-core accumulators (real and
// imaginary part; lane l holds column l%16, rows g+4m, g = l/16, m = 0..3).
// Panels of 8 columns:
//   1. the lanes holding the panel's columns copy them to LDS;
//   2. lane r eliminates row r of the panel (diagonal block and below) column
//      by column, with the diagonal-block rows broadcast by readlane, giving
//      L and V = L D; their rows replace the panel's rows in LDS;
//   3. every lower block right of the panel takes the rank-8 update
//      A -= L21 V21^T as eight 16x16x4 FP64 MFMAs (complex = 4 real products
//      per 4 columns).
// Wider panels halve the LDS round trips and wave barriers per column, which
// with one wave per system are latency that the MFMAs do not hide.
// Columns left of the trailing part also receive updates; they are finished
// and never read again.  The factor is recorded (L by columns, D^-1) for
// k_forward and the adjoint, and the forward right-hand side b = E - j w Phi
// rides along: y = L^-1 b is formed panel by panel and z = D^-1 y is written
// to Z, so that k_forward only runs the backward substitution.  A system whose
// smallest pivot is below 1e-5 of its largest impedance diagonal (or is not
// finite) is marked for the pivoted fallback.
// The accumulators and the row state fit 256 registers, so two systems share
// a SIMD: one wave's panel elimination runs while the other's MFMAs do.
template <int NP>
__device__ __forceinline__ void ldl_system(
    int s, int n, int F, const double *__restrict__ M, const double *__restrict__ Rv,
    const double *__restrict__ C, const double *__restrict__ omega,
    const double *__restrict__ phi, GJFactor fac, double2 *__restrict__ Z,
    int32_t *__restrict__ status) {
    constexpr int NB = NP / 16;
    constexpr int NBLK = NB * (NB + 1) / 2;
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // per wave: panel rows (A, then L21) and V21 rows; a row holds 8 entries
    // padded to 9 (144 bytes), so that the row-per-lane accesses of 16
    // consecutive lanes fall on disjoint LDS banks
    constexpr int PW = 8;  // panel width
    __shared__ double2 sPan[4][NP][PW + 1];
    __shared__ double2 sV[4][NP][PW + 1];
    const int b = s / F, f = s - b * F;
    const double w = omega[f];
    const double *Cb = C + (size_t)b * n;
    const int g = lane >> 4, c16 = lane & 15;

    // ---- Z in accumulator layout: block (bi, bj) at index bi (bi + 1) / 2 + bj.
    // Loads use clamped indices and no branches, so they are all in flight at
    // once; out-of-range entries are replaced by the identity padding.
    double rdg[NB], cdg[NB];  // R_j, 1/(w C_j) of column j = 16 bj + c16
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
        const int j = min(16 * bj + c16, n - 1);
        rdg[bj] = Rv[j];
        cdg[bj] = Cb[j];
    }
    f64x4 Xr[NBLK], Xi[NBLK];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj <= bi; ++bj) {
            const int bx = bi * (bi + 1) / 2 + bj;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = 16 * bi + g + 4 * m, j = 16 * bj + c16;
                const double mij = M[(size_t)min(i, n - 1) * n + min(j, n - 1)];
                Xr[bx][m] = 0.0;
                Xi[bx][m] = (i < n && j < n) ? w * mij : 0.0;
            }
        }
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
        const double xc = 1.0 / (w * cdg[bj]);
        const int bx = bj * (bj + 1) / 2 + bj;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (g + 4 * m == c16) {  // diagonal entry i = j = 16 bj + c16
                const bool real = 16 * bj + c16 < n;
                Xr[bx][m] = real ? rdg[bj] : 1.0;
                Xi[bx][m] = real ? Xi[bx][m] - xc : 0.0;
            }
        }
    }
    // input flags and the largest |re|+|im| diagonal entry (lane k handles k)
    int flag = 0;
    float zdiag = 0.0f;
    if (lane < n) {
        const double c = Cb[lane];
        if (isnan(c) || c == 0.0 || !isfinite(w) || w == 0.0) flag = COSIM_SYS_BAD_INPUT;
        else if (c < 0.0) flag = COSIM_SYS_NEGATIVE_C;
        zdiag = (float)(fabs(Rv[lane]) + fabs(w * M[(size_t)lane * n + lane] - 1.0 / (w * c)));
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        flag |= __shfl_xor(flag, off);
        zdiag = fmaxf(zdiag, __shfl_xor(zdiag, off));
    }
    // right-hand side b = E - j w Phi (lane i holds b_i), turned into y = L^-1 b
    // column by column as L is formed
    double2 y = lane < n ? loop_voltage(phi, n, lane, w) : make_double2(0.0, 0.0);
    double2 dk = make_double2(1.0, 0.0);  // D_i of the lane's own column

    double2 (*pan)[PW + 1] = sPan[wv];
    double2 (*vv)[PW + 1] = sV[wv];
    double2 *Ls = fac.L + (size_t)s * NP * NP;  // packed columns, see ldl_col
#pragma unroll
    for (int bc = 0; bc < NB; ++bc) {
#pragma unroll
        for (int h = 0; h < 16 / PW; ++h) {
            const int k0 = 16 * bc + PW * h;  // first column of the panel
            if (k0 >= n) break;               // uniform
            // 1. panel columns -> LDS (rows >= k0 matter)
            if (c16 >= PW * h && c16 < PW * h + PW) {
                const int c = c16 - PW * h;
                // real parts, then imaginary parts: 8-byte stores straight from
                // the accumulators (the empty asm keeps the two halves from
                // being merged into 16-byte stores, which need register copies)
#pragma unroll
                for (int bi = bc; bi < NB; ++bi) {
                    const int bx = bi * (bi + 1) / 2 + bc;
#pragma unroll
                    for (int m = 0; m < 4; ++m) pan[16 * bi + g + 4 * m][c].x = Xr[bx][m];
                }
                asm volatile("" ::: "memory");
#pragma unroll
                for (int bi = bc; bi < NB; ++bi) {
                    const int bx = bi * (bi + 1) / 2 + bc;
#pragma unroll
                    for (int m = 0; m < 4; ++m) pan[16 * bi + g + 4 * m][c].y = Xi[bx][m];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // 2. lane r takes row r of the panel, column by column:
            //      V_rc = A_rc - sum_{j<c} L_rj V_cj,  D_c = V_cc,  L_rc = V_rc / D_c.
            //    Row c of V (entries j < c, stored by lane k0 + c in earlier
            //    columns) reaches every lane as broadcast LDS reads, D_c by
            //    readlane; V and L rows replace the panel rows in LDS as they
            //    are formed.  Rows above the panel end in the upper triangle or
            //    in eliminated columns, which are never read again, so every
            //    row is stored as it comes.
            const int r = lane, rr = min(r, NP - 1);
            double2 l[PW];
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                double2 v = pan[rr][c];
                double2 vc[PW];
#pragma unroll
                for (int j = 0; j < c; ++j) vc[j] = vv[k0 + c][j];
#pragma unroll
                for (int j = 0; j < c; ++j) v = cfms(v, l[j], vc[j]);
                const double2 d = make_double2(readlane_d(v.x, k0 + c), readlane_d(v.y, k0 + c));
                const double2 dinv = cinv_nr(d);
                l[c] = cmul(v, dinv);
                // L below the diagonal (rows of the diagonal block and below
                // it); the column's base is wave-uniform, so the store takes a
                // scalar base and the lane's constant offset
                double2 *col = Ls + (ldl_col(NP, k0 + c) - (k0 + c) - 1);
                if (r > k0 + c && r < NP) col[r] = l[c];
                if (r < NP) {
                    pan[r][c] = l[c];
                    vv[r][c] = v;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            // D_c = V_cc to the lane of column c
            if (r >= k0 && r < k0 + PW) dk = vv[r][r - k0];
            // forward substitution for the panel's columns: y_r -= L_rc y_c (r > k0 + c)
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                const double2 yc = make_double2(readlane_d(y.x, k0 + c), readlane_d(y.y, k0 + c));
                const double2 yn = cfms(y, l[c], yc);
                const bool below = r > k0 + c;
                y.x = below ? yn.x : y.x;  // componentwise: a select of the
                y.y = below ? yn.y : y.y;  // vector struct goes through memory
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // 3. rank-PW update of every lower block right of the panel, as
            // PW / 4 steps of four 16x16x4 FP64 MFMAs; the operands of a block
            // row are read from LDS just before its MFMAs.  The last panel of
            // a block column leaves that column fully eliminated, so its
            // blocks are skipped.
            const int bj0 = h == 16 / PW - 1 ? bc + 1 : bc;
#pragma unroll
            for (int bi = bj0; bi < NB; ++bi) {
                double2 La[PW / 4];  // A operand: row c16 of block bi, k = g + 4 q
#pragma unroll
                for (int q = 0; q < PW / 4; ++q) La[q] = pan[16 * bi + c16][g + 4 * q];
#pragma unroll
                for (int bj = bj0; bj <= bi; ++bj) {
                    const int bx = bi * (bi + 1) / 2 + bj;
#pragma unroll
                    for (int q = 0; q < PW / 4; ++q) {
                        const double2 Vb = vv[16 * bj + c16][g + 4 * q];  // B operand: column c16 of block bj
                        Xr[bx] = __builtin_amdgcn_mfma_f64_16x16x4f64(-La[q].x, Vb.x, Xr[bx], 0, 0, 0);
                        Xr[bx] = __builtin_amdgcn_mfma_f64_16x16x4f64(La[q].y, Vb.y, Xr[bx], 0, 0, 0);
                        Xi[bx] = __builtin_amdgcn_mfma_f64_16x16x4f64(-La[q].x, Vb.y, Xi[bx], 0, 0, 0);
                        Xi[bx] = __builtin_amdgcn_mfma_f64_16x16x4f64(-La[q].y, Vb.x, Xi[bx], 0, 0, 0);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    const double2 dl = cinv_nr(dk);  // the D^-1 the elimination used
    if (lane < NP) fac.piv_val[(size_t)s * NP + lane] = dl;  // D^-1 (1 on the padding)
    // smallest |re| + |im| pivot of the real columns
    double dmin = lane < n ? fabs(dk.x) + fabs(dk.y) : __builtin_inf();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) dmin = fmin(dmin, __shfl_xor(dmin, off));
    if (lane < n) Z[(size_t)s * n + lane] = cmul(y, dl);  // z = D^-1 L^-1 b
    if (lane == 0) {
        const bool pivot = (flag & COSIM_SYS_BAD_INPUT) || !(dmin >= 1e-5 * (double)zdiag);
        status[s] = flag;
        fac.fmt[s] = pivot ? kFmtNeedsPivot : kFmtLDL;
    }
}

// Forward solve of a system in the LDL^T format from the z the factorisation
// left in I: x = L^-T z, written over it (systems handed to the pivoted
// fallback are skipped; it writes their I).
template <int NP>
__device__ __forceinline__ void forward_system(int s, int n, GJFactor fac, double2 *__restrict__ I,
                                               int32_t *__restrict__ status) {
    __shared__ double2 sRed[4][NP * 9];
    __shared__ double2 sTr[4][NP >= 64 ? 64 : 128];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (__builtin_amdgcn_readfirstlane(fac.fmt[s]) != kFmtLDL) return;
    double2 x = lane < n ? I[(size_t)s * n + lane] : make_double2(0.0, 0.0);
    x = ldl_backward<NP, 2>(x, fac.L + (size_t)s * NP * NP, n, lane, sRed[wv], sTr[wv]);
    bool nonfinite = false;
    if (lane < n) {
        I[(size_t)s * n + lane] = x;
        nonfinite = !(isfinite(x.x) && isfinite(x.y));
    }
    if (__ballot(nonfinite) != 0 && lane == 0) status[s] |= COSIM_SYS_NONFINITE;
}

template <int NP>
__global__ __launch_bounds__(256) void k_forward(int n, int S, GJFactor fac,
                                                 double2 *__restrict__ I,
                                                 int32_t *__restrict__ status) {
    const int s = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (s >= S) return;
    forward_system<NP>(s, n, fac, I, status);
}

// One wave per system, four per block.
template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_ldl(
    int n, int S, int F, const double *__restrict__ M, const double *__restrict__ Rv,
    const double *__restrict__ C, const double *__restrict__ omega,
    const double *__restrict__ phi, GJFactor fac, double2 *__restrict__ Z,
    int32_t *__restrict__ status) {
    const int s = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (s >= S) return;  // whole wave; the block never synchronises
    ldl_system<NP>(s, n, F, M, Rv, C, omega, phi, fac, Z, status);
}

template <int NP>
__global__ __launch_bounds__(256) void k_forward_group(SmallGroup g, int S) {
    const int sg = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (sg >= S) return;
    const SmallInst &e = g.in[group_member(g, sg)];
    forward_system<NP>(sg - e.s0, e.n, e.fac, e.I, e.status);
}

// The same over the S systems of a group of plans (each wave resolves its own
// member, so the waves of a block may serve different plans).
template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_ldl_group(
    SmallGroup g, int S) {
    const int sg = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (sg >= S) return;
    const SmallInst &e = g.in[group_member(g, sg)];
    ldl_system<NP>(sg - e.s0, e.n, e.F, e.M, e.R, e.C, e.omega, e.phi, e.fac, e.I, e.status);
}

// Adjoint solve with a recorded factorisation, one wave per system, lane i
// holds component i; b = rscale * sum_c (rr - j ri) of rpart[c][s][:].
// Format kFmtLDL: y = L^-1 b by columns (readlane broadcast of y_k, one
// coalesced column load), z = D^-1 y, then L^T x = z (ldl_backward).
// Format kFmtGJ: replays the recorded Gauss-Jordan row operations
// b <- b - l_k b_{p_k}, then x_k = b_{p_k} / piv_k.
// Writes gsys[s][k] = 2 Re(mu_k I_k / (j w C_k^2)) and, if given, mu.
template <int NP>
__device__ __forceinline__ void replay_system(int s, int n, int S, int F, GJFactor fac,
                                              const double *__restrict__ C,
                                              const double *__restrict__ omega,
                                              const double2 *__restrict__ I,
                                              const double2 *__restrict__ rpart, int nchunk,
                                              double rscale, double *__restrict__ gsys,
                                              double2 *__restrict__ mu,
                                              int32_t *__restrict__ status) {
    __shared__ double2 sRed[4][NP * 9];  // per wave: the lane products of ldl_backward
    __shared__ double2 sTr[4][NP >= 64 ? 64 : 128];  // per wave: an 8x8 block of L, transposed
    const int lane = threadIdx.x & 63;
    const int fmt = __builtin_amdgcn_readfirstlane(fac.fmt[s]);
    const int b = s / F, f = s - b * F;
    const double w = omega[f];
    double2 x = make_double2(0.0, 0.0);
    if (lane < n) {
        double rr = 0.0, ri = 0.0;
#pragma unroll 8
        for (int c = 0; c < nchunk; ++c) {  // loads ahead, sums in chunk order
            const double2 v = rpart[((size_t)c * S + s) * NP + lane];
            rr += v.x;
            ri += v.y;
        }
        x = make_double2(rscale * rr, -rscale * ri);
    }
    const double2 *__restrict__ Ls = fac.L + (size_t)s * NP * NP;
    constexpr int U = 8;
    if (fmt == kFmtLDL) {
        // column k of L as lane i sees it: L_ik for k < i < n, else 0
        auto lcol = [&](int k) {
            return (lane > k && lane < n) ? Ls[ldl_col(NP, k) + lane - k - 1] : make_double2(0.0, 0.0);
        };
        // Columns are loaded in groups of U; the next group's loads are in
        // flight while the current group is applied (cur / nxt registers).
        double2 cur[U], nxt[U];
        auto load_group = [&](double2(&l)[U], int k0) {
#pragma unroll
            for (int u = 0; u < U; ++u) l[u] = lcol(k0 + u);
        };
        // forward: y_i -= L_ik y_k for i > k
        const int nfg = n / U;  // full groups
        if (nfg > 0) load_group(cur, 0);
        int k0 = 0;
        for (; k0 + U <= n; k0 += U) {
            if (k0 + 2 * U <= n) load_group(nxt, k0 + U);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double2 yk = make_double2(readlane_d(x.x, k0 + u), readlane_d(x.y, k0 + u));
                x = cfms(x, cur[u], yk);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = nxt[u];
        }
        for (; k0 < n; ++k0) {
            const double2 l = lcol(k0);
            const double2 yk = make_double2(readlane_d(x.x, k0), readlane_d(x.y, k0));
            x = cfms(x, l, yk);
        }
        if (lane < n) x = cmul(x, fac.piv_val[(size_t)s * NP + lane]);  // D^-1
        x = ldl_backward<NP, 1>(x, Ls, n, lane, sRed[threadIdx.x >> 6], sTr[threadIdx.x >> 6]);
    } else {
        const int *__restrict__ Ps = fac.piv_row + (size_t)s * NP;
        int k0 = 0;
        for (; k0 + U <= n; k0 += U) {
            double2 l[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                l[u] = lane < NP ? Ls[(size_t)(k0 + u) * NP + lane] : make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = Ps[k0 + u];
                const double2 bp = make_double2(readlane_d(x.x, p), readlane_d(x.y, p));
                x = cfms(x, l[u], bp);
            }
        }
        for (; k0 < n; ++k0) {
            const double2 l = lane < NP ? Ls[(size_t)k0 * NP + lane] : make_double2(0.0, 0.0);
            const int p = Ps[k0];
            const double2 bp = make_double2(readlane_d(x.x, p), readlane_d(x.y, p));
            x = cfms(x, l, bp);
        }
        const int pk = lane < n ? Ps[lane] : 0;
        const double2 bpk = make_double2(__shfl(x.x, pk), __shfl(x.y, pk));
        x = lane < n ? cmul(bpk, cinv(fac.piv_val[(size_t)s * NP + lane])) : make_double2(0.0, 0.0);
    }
    const int flag = status[s];
    const bool bad = (flag & (COSIM_SYS_BAD_INPUT | COSIM_SYS_SINGULAR)) != 0;
    bool nonfinite = false;
    if (lane < n) {
        if (bad) x = make_double2(__builtin_nan(""), __builtin_nan(""));
        const double2 Ik = I[(size_t)s * n + lane];
        const double ck = C[(size_t)b * n + lane];
        // 2 Re(mu I / (j w C^2)) = 2 Im(mu I) / (w C^2)
        const double g = 2.0 * (x.x * Ik.y + x.y * Ik.x) / (w * ck * ck);
        gsys[(size_t)s * n + lane] = g;
        if (mu) mu[(size_t)s * n + lane] = x;
        nonfinite = !bad && !isfinite(g);
    }
    if (__ballot(nonfinite) != 0 && lane == 0) status[s] = flag | COSIM_SYS_NONFINITE;
}

template <int NP>
__global__ __launch_bounds__(256) void k_replay_adjoint(int n, int S, int F, GJFactor fac,
                                                        const double *__restrict__ C,
                                                        const double *__restrict__ omega,
                                                        const double2 *__restrict__ I,
                                                        const double2 *__restrict__ rpart,
                                                        int nchunk, double rscale,
                                                        double *__restrict__ gsys,
                                                        double2 *__restrict__ mu,
                                                        int32_t *__restrict__ status) {
    const int s = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (s >= S) return;  // whole wave; no block-level synchronisation below
    replay_system<NP>(s, n, S, F, fac, C, omega, I, rpart, nchunk, rscale, gsys, mu, status);
}

template <int NP>
__global__ __launch_bounds__(256) void k_replay_adjoint_group(SmallGroup g, int S) {
    const int sg = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (sg >= S) return;
    const SmallInst &e = g.in[group_member(g, sg)];
    replay_system<NP>(sg - e.s0, e.n, e.S, e.F, e.fac, e.C, e.omega, e.I, e.rpart, e.nchunk,
                      e.rscale, e.gsys, e.mu, e.status);
}

// One 64-lane block per configuration b: dL/dC_b summed over frequencies per
// loop, and the loss over frequencies and P-chunks, each lane taking every
// 64th partial loss and the lanes combined by a fixed shuffle tree (both
// orders are fixed, so repeated calls agree bit for bit).
__device__ __forceinline__ void reduce_config(int b, int n, int B, int F, int nchunk,
                                              const double *__restrict__ gsys,
                                              const double *__restrict__ lpart, double lscale,
                                              double *__restrict__ grad,
                                              double *__restrict__ loss) {
    const int S = B * F;
    if (grad) {
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            double acc = 0.0;
            for (int f = 0; f < F; ++f) acc += gsys[((size_t)b * F + f) * n + k];
            grad[(size_t)b * n + k] = acc;
        }
    }
    if (loss) {
        const int m = F * nchunk;
        double acc = 0.0;
        for (int e = threadIdx.x; e < m; e += 64) {
            const int c = e / F, f = e - c * F;  // consecutive lanes: consecutive f
            acc += lpart[(size_t)c * S + (size_t)b * F + f];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (threadIdx.x == 0) loss[b] = lscale * acc;
    }
}

__global__ __launch_bounds__(64) void k_reduce(int n, int B, int F, int nchunk,
                                               const double *__restrict__ gsys,
                                               const double *__restrict__ lpart, double lscale,
                                               double *__restrict__ grad,
                                               double *__restrict__ loss) {
    reduce_config(blockIdx.x, n, B, F, nchunk, gsys, lpart, lscale, grad, loss);
}

__global__ __launch_bounds__(64) void k_reduce_group(ReduceGroup g) {
    const int bg = blockIdx.x;
    int i = 0;
    while (i + 1 < g.count && bg >= g.in[i + 1].b0) ++i;
    const ReduceInst &e = g.in[i];
    reduce_config(bg - e.b0, e.n, e.B, e.F, e.nchunk, e.gsys, e.lpart, e.lscale, e.grad, e.loss);
}

template <bool ADJ>
hipError_t launch_gj(int NP, int n, int S, int F, const double *M, const double *R,
                     const double *phi, const double *C, const double *omega, const double2 *Iin,
                     const double2 *rpart, int nchunk, double rscale, double2 *Iout,
                     double *gsys, int32_t *status, bool or_status, GJFactor fac,
                     bool fallback_only, hipStream_t st) {
    switch (NP) {
        case 32:
            hipLaunchKernelGGL((k_gj<32, ADJ>), dim3(S), dim3(GJShape<32>::BLOCK), 0, st, n, S,
                               F, M, R, phi, C, omega, Iin, rpart, nchunk, rscale, Iout, gsys,
                               status, or_status, fac, fallback_only);
            break;
        case 64:
            hipLaunchKernelGGL((k_gj<64, ADJ>), dim3(S), dim3(GJShape<64>::BLOCK), 0, st, n, S,
                               F, M, R, phi, C, omega, Iin, rpart, nchunk, rscale, Iout, gsys,
                               status, or_status, fac, fallback_only);
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
                                GJFactor fac, hipStream_t st) {
    return launch_gj<false>(NP, n, S, F, M_d, R_d, phi_d, C_d, omega_d, nullptr, nullptr, 0, 0.0,
                            I_d, nullptr, status_d, false, fac, false, st);
}

hipError_t launch_ldl(int NP, int n, int S, int F, const double *M_d, const double *R_d,
                      const double *C_d, const double *omega_d, const double *phi_d, GJFactor fac,
                      double2 *I_d, int32_t *status_d, hipStream_t st) {
    const dim3 grid((S + 3) / 4);
    switch (NP) {
        case 32:
            hipLaunchKernelGGL(k_ldl<32>, grid, dim3(256), 0, st, n, S, F, M_d, R_d, C_d, omega_d,
                               phi_d, fac, I_d, status_d);
            hipLaunchKernelGGL(k_forward<32>, grid, dim3(256), 0, st, n, S, fac, I_d, status_d);
            break;
        case 64:
            hipLaunchKernelGGL(k_ldl<64>, grid, dim3(256), 0, st, n, S, F, M_d, R_d, C_d, omega_d,
                               phi_d, fac, I_d, status_d);
            hipLaunchKernelGGL(k_forward<64>, grid, dim3(256), 0, st, n, S, fac, I_d, status_d);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_solve_fallback(int NP, int n, int S, int F, const double *M_d,
                                 const double *R_d, const double *phi_d, const double *C_d,
                                 const double *omega_d, double2 *I_d, int32_t *status_d,
                                 GJFactor fac, hipStream_t st) {
    return launch_gj<false>(NP, n, S, F, M_d, R_d, phi_d, C_d, omega_d, nullptr, nullptr, 0, 0.0,
                            I_d, nullptr, status_d, false, fac, true, st);
}

hipError_t launch_replay_adjoint(int NP, int n, int S, int F, GJFactor fac, const double *C_d,
                                 const double *omega_d, double2 *I_d, const double2 *rpart_d,
                                 int nchunk, double rscale, double *gsys_d, double2 *mu_d,
                                 int32_t *status_d, hipStream_t st) {
    const dim3 grid((S + 3) / 4);
    switch (NP) {
        case 32:
            hipLaunchKernelGGL(k_replay_adjoint<32>, grid, dim3(256), 0, st, n, S, F, fac, C_d,
                               omega_d, I_d, rpart_d, nchunk, rscale, gsys_d, mu_d, status_d);
            break;
        case 64:
            hipLaunchKernelGGL(k_replay_adjoint<64>, grid, dim3(256), 0, st, n, S, F, fac, C_d,
                               omega_d, I_d, rpart_d, nchunk, rscale, gsys_d, mu_d, status_d);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_solve_adjoint(int NP, int n, int S, int F, const double *M_d,
                                const double *R_d, const double *C_d, const double *omega_d,
                                const double2 *I_d, const double2 *rpart_d, int nchunk,
                                double rscale, double *gsys_d, double2 *mu_d, int32_t *status_d,
                                bool or_status, hipStream_t st) {
    return launch_gj<true>(NP, n, S, F, M_d, R_d, nullptr, C_d, omega_d, I_d, rpart_d, nchunk,
                           rscale, mu_d, gsys_d, status_d, or_status, GJFactor{}, false, st);
}

hipError_t launch_reduce(int n, int B, int F, int nchunk, const double *gsys_d,
                         const double *lpart_d, double lscale, double *grad_d, double *loss_d,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(B), dim3(64), 0, st, n, B, F, nchunk, gsys_d, lpart_d,
                       lscale, grad_d, loss_d);
    return hipGetLastError();
}

hipError_t launch_reduce_group(const ReduceGroup &g, int Btot, hipStream_t st) {
    if (Btot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_group, dim3(Btot), dim3(64), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_small_group(int NP, const SmallGroup &g, int S, SmallPhase phase,
                              hipStream_t st) {
    if (S <= 0) return hipSuccess;
    const dim3 wave_grid((S + 3) / 4);
#define COSIM_SMALL_GROUP(NPC)                                                                   \
    switch (phase) {                                                                             \
        case SmallPhase::Factor:                                                                 \
            hipLaunchKernelGGL(k_ldl_group<NPC>, wave_grid, dim3(256), 0, st, g, S);             \
            hipLaunchKernelGGL(k_forward_group<NPC>, wave_grid, dim3(256), 0, st, g, S);         \
            break;                                                                               \
        case SmallPhase::Fallback:                                                               \
            hipLaunchKernelGGL(k_gj_group<NPC>, dim3(S), dim3(GJShape<NPC>::BLOCK), 0, st, g);   \
            break;                                                                               \
        case SmallPhase::Adjoint:                                                                \
            hipLaunchKernelGGL(k_replay_adjoint_group<NPC>, wave_grid, dim3(256), 0, st, g, S);   \
            break;                                                                               \
    }
    switch (NP) {
        case 32:
            COSIM_SMALL_GROUP(32)
            break;
        case 64:
            COSIM_SMALL_GROUP(64)
            break;
        default:
            return hipErrorInvalidValue;
    }
#undef COSIM_SMALL_GROUP
    return hipGetLastError();
}

}  // namespace cosim
