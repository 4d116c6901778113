// Large batches above 64 loops: the superposition and its adjoint as two
// LDS-tiled matrix-core GEMM passes, both with K-contiguous operands.
//   pass 1  C = G X         rows = points, K = loops (G [P_pad][NP] as is,
//                           X^T [N][NP]: the currents as column planes);
//           epilogue: the loss of Eq. 1 per (row block, system) and, for the
//           gradient, w = dL/d conj(B) written as W^T [N][P_pad] planes;
//   pass 2  R = G^T W       rows = loops, K = points in chunks (G^T
//                           [NP][P_pad], W^T as written by pass 1): r of
//                           Eq. 8-10 per (chunk, system) for the adjoint solve.
// Columns come in groups of 32: the real parts of the currents of 16 systems,
// then their imaginary parts (so that a lane holds both parts of its system).
// When a workgroup of the fused kernel (contract_mfma.hip) would have to
// hold the currents of too few systems for G to be read only a few times,
// this pair reads G once per column block of BN = 64 to 128 columns instead.
//
// A workgroup (WM x WN waves) computes a BM x BN tile over K in steps of 32:
// each step's operands are loaded from memory into registers two steps ahead
// and stored to LDS while the step before is multiplied (two LDS buffers, two
// register sets, one barrier per step).  Each wave multiplies a (BM / WM) x (BN / WN) block with 16x16
// matrix-core tiles: BF16X3 (hi hi + hi lo + lo hi into FP32), FP32 or FP64,
// the same products as the fused kernel.  BF16X3 uses 256 x 128 tiles of 8
// waves (one workgroup per compute unit: fewer operand bytes per product),
// FP32 128 x 128 tiles of 4 waves (two workgroups per compute unit, one's
// barrier waits overlapping the other's products), FP64 (bound by its
// matrix-core rate) 128 x 64 tiles of 8 waves.
#include <algorithm>

#include "epilogue.h"
#include "internal.h"

namespace cosim {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32;  // K per step

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats as packed bf16 (RNE) high parts and the packed low parts of
// their remainders: hi = bf16(x), lo = bf16(x - hi).
__device__ inline void split_pair(float a, float b, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
    const float ha = __builtin_bit_cast(float, hi << 16);
    const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2));
}

// Operands of one 16x16 tile and one step of 32 K: 8 consecutive K per lane
// (lane group q = lane / 16 holds K entries 8q..8q+7).
struct GBF3 {
    static constexpr int ESZ = 2, PLANES = 2, BM = 256, BN = 128, WM = 4, WN = 2;
    typedef float Acc;
    typedef f32x4 V;
    struct Op {
        bf16x8 h, l;
    };
    __device__ static constexpr int row(int q, int m) { return 4 * q + m; }
    __device__ static Op lds(const char *hi, const char *lo) {
        return Op{__builtin_bit_cast(bf16x8, *(const u32x4 *)hi),
                  __builtin_bit_cast(bf16x8, *(const u32x4 *)lo)};
    }
    __device__ static V mma(const Op &a, const Op &b, V c) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
    }
};
template <typename T>
struct GScalar {
    static constexpr int ESZ = sizeof(T), PLANES = 1;
    static constexpr int BM = 128, BN = sizeof(T) == 4 ? 128 : 64;
    static constexpr int WM = sizeof(T) == 4 ? 2 : 4, WN = 2;
    typedef T Acc;
    typedef T V __attribute__((ext_vector_type(4)));
    struct Op {
        T v[8];
    };
    __device__ static constexpr int row(int q, int m) { return sizeof(T) == 4 ? 4 * q + m : q + 4 * m; }
    __device__ static Op lds(const char *p, const char *) {
        Op o;
#pragma unroll
        for (int j = 0; j < 8; j += 16 / (int)sizeof(T)) {
            const u32x4 u = *(const u32x4 *)(p + j * sizeof(T));
            const T *e = (const T *)&u;
#pragma unroll
            for (int i = 0; i < 16 / (int)sizeof(T); ++i) o.v[j + i] = e[i];
        }
        return o;
    }
    __device__ static V mma(const Op &a, const Op &b, V c) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (sizeof(T) == 4)
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[j], b.v[j], c, 0, 0, 0);
            else
                c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[j], b.v[j], c, 0, 0, 0);
        }
        return c;
    }
};
typedef GScalar<float> GF32;
typedef GScalar<double> GF64;

// LDS rows of one step: 32 K entries plus 16 bytes of padding
template <class Pol>
constexpr int row_bytes() {
    return kBK * Pol::ESZ + 16;
}
template <class Pol>
constexpr int stage_bytes() {
    return (Pol::BM + Pol::BN) * row_bytes<Pol>() * Pol::PLANES;
}

// EPI 0: pass 1 (loss; w planes when a.W is set).  EPI 1: pass 2 (r partials).
template <class Pol>
constexpr int threads() {
    return 64 * Pol::WM * Pol::WN;
}

template <class Pol, int EPI, int LOSS>
__global__ __launch_bounds__(threads<Pol>(), 2) void k_gemm(GemmArgs a) {
    typedef typename Pol::Acc Acc;
    typedef typename Pol::V V;
    typedef typename Pol::Op Op;
    constexpr int BM = Pol::BM, BN = Pol::BN, ESZ = Pol::ESZ, PL = Pol::PLANES;
    constexpr int WM = Pol::WM, WN = Pol::WN, NT = threads<Pol>();
    constexpr int TM = BM / WM, TN = BN / WN;  // wave block
    constexpr int TI = TM / 16, TJ = TN / 16;
    constexpr int RB = row_bytes<Pol>();
    constexpr int CPR = kBK * ESZ / 16;      // 16-byte pieces per row and plane
    constexpr int NA = BM * CPR * PL / NT, NB = BN * CPR * PL / NT;  // pieces per thread
    static_assert(BM * CPR * PL % NT == 0 && BN * CPR * PL % NT == 0, "whole pieces per thread");
    static_assert(TN % 32 == 0, "a wave holds whole column groups");
    extern __shared__ __attribute__((aligned(16))) char smem[];

    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave - wm * WN;
    const int r16 = lane & 15, q = lane >> 4;
    // work item: column blocks fastest, so that the column blocks of one row
    // block (which share its A tile) run side by side on one XCD
    const int nbn = a.N / BN, nbm = (a.M + BM - 1) / BM;
    const int Nw = nbn * nbm * a.nkc, b = (int)blockIdx.x;
    const int item = (Nw & 7) == 0 ? (b & 7) * (Nw >> 3) + (b >> 3) : b;
    const int bn = item % nbn, bm = (item / nbn) % nbm, kc = item / (nbn * nbm);
    const int row0 = bm * BM, col0 = bn * BN;
    const int k0 = kc * a.kchunk, k1 = min(a.K, k0 + a.kchunk);
    const int nsteps = (k1 - k0) / kBK;

    // global -> registers -> LDS staging of one step, two register sets
    auto fetch = [&](int kb, u32x4 (&ga)[NA], u32x4 (&gb)[NB]) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + NT * u;
            const int pl = e / (BM * CPR), rem = e - pl * (BM * CPR);
            const int r = rem / CPR, c = rem - r * CPR;
            // rows past M: the last row is read (in bounds, unconditionally, so
            // that no merge of register values waits on the load) and zeroed
            // when stored
            const int gr = min(row0 + r, a.M - 1);
            const char *src = (const char *)(pl ? a.Alo : a.A);
            ga[u] = *(const u32x4 *)(src + ((size_t)gr * a.lda + kb) * ESZ + 16 * c);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + NT * u;
            const int pl = e / (BN * CPR), rem = e - pl * (BN * CPR);
            const int r = rem / CPR, c = rem - r * CPR;
            const char *src = (const char *)(pl ? a.Blo : a.B);
            gb[u] = *(const u32x4 *)(src + ((size_t)(col0 + r) * a.ldb + kb) * ESZ + 16 * c);
        }
    };
    auto stash = [&](char *st, const u32x4 (&ga)[NA], const u32x4 (&gb)[NB]) {
        char *sa = st, *sb = st + BM * RB * PL;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int e = tid + NT * u;
            const int pl = e / (BM * CPR), rem = e - pl * (BM * CPR);
            const int r = rem / CPR, c = rem - r * CPR;
            *(u32x4 *)(sa + (pl * BM + r) * RB + 16 * c) =
                row0 + r < a.M ? ga[u] : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = tid + NT * u;
            const int pl = e / (BN * CPR), rem = e - pl * (BN * CPR);
            const int r = rem / CPR, c = rem - r * CPR;
            *(u32x4 *)(sb + (pl * BN + r) * RB + 16 * c) = gb[u];
        }
    };

    V acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = V{};
    auto compute = [&](const char *sa) {
        const char *sb = sa + BM * RB * PL;
        Op bo[TJ];
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int r = wn * TN + 16 * j + r16;
            bo[j] = Pol::lds(sb + r * RB + 8 * ESZ * q, sb + (BN + r) * RB + 8 * ESZ * q);
        }
#pragma unroll
        for (int i = 0; i < TI; ++i) {
            const int r = wm * TM + 16 * i + r16;
            const Op ao = Pol::lds(sa + r * RB + 8 * ESZ * q, sa + (BM + r) * RB + 8 * ESZ * q);
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = Pol::mma(ao, bo[j], acc[i][j]);
        }
    };

    // Steps in pairs over two LDS buffers; each step's operands are loaded two
    // steps ahead (register set 0 for even steps, 1 for odd), stored to LDS at
    // the end of the step before theirs, one barrier per step.  The loads are
    // unconditional (the step index clamped to the last step), so that each
    // register set is filled by its loads alone and no copy waits on them.
    constexpr int SB = stage_bytes<Pol>();
    const int last = nsteps > 0 ? nsteps - 1 : 0;
    u32x4 ga0[NA], gb0[NB], ga1[NA], gb1[NB];
    if (nsteps > 0) {
        fetch(k0, ga0, gb0);
        stash(smem, ga0, gb0);
        fetch(k0 + min(1, last) * kBK, ga1, gb1);
    }
    __syncthreads();
    // nsteps is even: K and every chunk of it are multiples of 64
    for (int s = 0; s < nsteps; s += 2) {
        fetch(k0 + min(s + 2, last) * kBK, ga0, gb0);
        compute(smem);
        stash(smem + SB, ga1, gb1);
        __syncthreads();
        fetch(k0 + min(s + 3, last) * kBK, ga1, gb1);
        compute(smem + SB);
        if (s + 2 < nsteps) stash(smem, ga0, gb0);
        __syncthreads();
    }

    // ---- epilogues.  Column group g of the wave (tiles 2g, 2g + 1) holds the
    // real and imaginary parts of systems sys0 + r16.
    constexpr int NG = TJ / 2;
    if constexpr (EPI == 0) {
        double lacc[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) lacc[g] = 0.0;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int cre = col0 + wn * TN + 32 * g + r16;  // column of the real part
                Acc wx[4], wy[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int p = row0 + wm * TM + 16 * i + Pol::row(q, m);
                    Acc x = acc[i][2 * g][m], y = acc[i][2 * g + 1][m];
                    // padded points: field = incident field, target |inc|: no residual
                    const Acc t = p < a.P ? (Acc)a.T[p] : (Acc)fabs(a.inc);
                    lacc[g] += epilogue<LOSS>(x, y, t, (Acc)a.inc);
                    wx[m] = x;
                    wy[m] = y;
                }
                // w planes: the lane's 4 rows are consecutive points (BF16X3,
                // FP32), so each plane gets one 8- or 16-byte store per lane
                const int pb4 = row0 + wm * TM + 16 * i + Pol::row(q, 0);
                if (!a.W || pb4 >= a.M) continue;
                if constexpr (ESZ == 2) {
                    unsigned hx[2], lx[2], hy[2], ly[2];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        split_pair(wx[2 * j], wx[2 * j + 1], hx[j], lx[j]);
                        split_pair(wy[2 * j], wy[2 * j + 1], hy[j], ly[j]);
                    }
                    uint16_t *wh = (uint16_t *)a.W, *wl = (uint16_t *)a.Wlo;
                    const size_t ox = (size_t)cre * a.ldw + pb4, oy = ox + (size_t)16 * a.ldw;
                    *(uint2 *)(wh + ox) = make_uint2(hx[0], hx[1]);
                    *(uint2 *)(wl + ox) = make_uint2(lx[0], lx[1]);
                    *(uint2 *)(wh + oy) = make_uint2(hy[0], hy[1]);
                    *(uint2 *)(wl + oy) = make_uint2(ly[0], ly[1]);
                } else if constexpr (ESZ == 4) {
                    float *wf = (float *)a.W;
                    const size_t ox = (size_t)cre * a.ldw + pb4, oy = ox + (size_t)16 * a.ldw;
                    *(float4 *)(wf + ox) = make_float4(wx[0], wx[1], wx[2], wx[3]);
                    *(float4 *)(wf + oy) = make_float4(wy[0], wy[1], wy[2], wy[3]);
                } else {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int p = row0 + wm * TM + 16 * i + Pol::row(q, m);
                        ((Acc *)a.W)[(size_t)cre * a.ldw + p] = wx[m];
                        ((Acc *)a.W)[(size_t)(cre + 16) * a.ldw + p] = wy[m];
                    }
                }
            }
        // loss of the row block per system: lane groups, then the 4 row waves
        double *red = (double *)smem;  // [wn][g][wm][16]
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            double v = lacc[g];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (q == 0) red[((wn * NG + g) * WM + wm) * 16 + r16] = v;
        }
        __syncthreads();
        for (int e = tid; e < WN * NG * 16; e += NT) {
            const int c16 = e & 15, wg = e >> 4;  // wg = wn * NG + g
            double v = 0.0;
            for (int r = 0; r < WM; ++r) v += red[(wg * WM + r) * 16 + c16];  // row waves in order
            const int s = (col0 + 32 * wg) / 2 + c16;
            if (s < a.S) a.lpart[(size_t)bm * a.S + s] = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int s = (col0 + wn * TN + 32 * g) / 2 + r16;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int k = row0 + wm * TM + 16 * i + Pol::row(q, m);
                    if (s < a.S && k < a.NP)
                        a.rpart[((size_t)kc * a.S + s) * a.NP + k] =
                            make_double2((double)acc[i][2 * g][m], (double)acc[i][2 * g + 1][m]);
                }
            }
    }
}

// X^T planes of the currents: row c of [N][NP] is the real (c % 32 < 16) or
// imaginary part of system 16 (c / 32) + c % 16; zero beyond S and n.
template <class Pol>
__global__ __launch_bounds__(256) void k_pack_xt(int n, int NP, int S, int N,
                                                 const double2 *__restrict__ I, void *X, void *Xlo) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)N * NP) return;
    const int c = (int)(e / NP), k = (int)(e - (size_t)c * NP);
    const int s = 16 * (c / 32) + c % 16;
    double v = 0.0;
    if (s < S && k < n) {
        const double2 z = I[(size_t)s * n + k];
        v = (c % 32) < 16 ? z.x : z.y;
    }
    if constexpr (Pol::ESZ == 2) {
        const float f = (float)v;
        const __bf16 h = (__bf16)f;
        ((uint16_t *)X)[e] = __builtin_bit_cast(uint16_t, h);
        ((uint16_t *)Xlo)[e] = __builtin_bit_cast(uint16_t, (__bf16)(f - (float)h));
    } else {
        ((typename Pol::Acc *)X)[e] = (typename Pol::Acc)v;
    }
}

template <class Pol, int EPI, int LOSS>
hipError_t go(const GemmArgs &a, hipStream_t st) {
    const int nbn = a.N / Pol::BN, nbm = (a.M + Pol::BM - 1) / Pol::BM;
    const unsigned blocks = (unsigned)(nbn * nbm * a.nkc);
    if (blocks == 0) return hipSuccess;
    // the kernel runs whole pairs of 32-deep steps
    if (a.K % (2 * kBK) != 0 || a.kchunk % (2 * kBK) != 0 || a.N % Pol::BN != 0)
        return hipErrorInvalidValue;
    // more dynamic LDS than the default limit: raised once per kernel
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_gemm<Pol, EPI, LOSS>, hipFuncAttributeMaxDynamicSharedMemorySize,
        2 * stage_bytes<Pol>());
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_gemm<Pol, EPI, LOSS>), dim3(blocks), dim3(threads<Pol>()), 2 * stage_bytes<Pol>(),
                       st, a);
    return hipGetLastError();
}

template <class Pol>
hipError_t go_pair(int loss_mode, bool grad, const GemmArgs &fw, const GemmArgs &ad,
                   const double2 *I, int n, hipStream_t st) {
    const size_t ne = (size_t)fw.N * fw.K;
    hipLaunchKernelGGL(k_pack_xt<Pol>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, n,
                       fw.K, fw.S, fw.N, I, (void *)fw.B, (void *)fw.Blo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (loss_mode) {
        case COSIM_LOSS_MAG: e = go<Pol, 0, COSIM_LOSS_MAG>(fw, st); break;
        case COSIM_LOSS_COMPLEX: e = go<Pol, 0, COSIM_LOSS_COMPLEX>(fw, st); break;
        case COSIM_LOSS_RATIO: e = go<Pol, 0, COSIM_LOSS_RATIO>(fw, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || !grad) return e;
    return go<Pol, 1, 0>(ad, st);
}

}  // namespace

GemmShape gemm_shape(Prec prec, int NP, int S, int P_pad) {
    GemmShape g;
    const int BM = prec == Prec::F64 ? GF64::BM : prec == Prec::F32 ? GF32::BM : GBF3::BM;
    const int BN = prec == Prec::F64 ? GF64::BN : prec == Prec::F32 ? GF32::BN : GBF3::BN;
    g.N = (2 * S + BN - 1) / BN * BN;
    g.row_blocks = (P_pad + BM - 1) / BM;
    // adjoint chunks of points: FP32 accumulation over at most kMfmaRowsF32
    // (BF16X3: four times that, its own rounding being far larger), FP64 over
    // enough to keep every compute unit busy with a few workgroups
    const int col_blocks = g.N / BN, k_blocks = (NP + BM - 1) / BM;
    int kchunk = prec == Prec::F32 ? kMfmaRowsF32 : prec == Prec::BF16X3 ? 4 * kMfmaRowsF32 : P_pad;
    if (prec == Prec::F64) {
        const int want = 512;
        int nk = std::max(1, want / std::max(1, col_blocks * k_blocks));
        kchunk = P_pad / nk;
    }
    kchunk = (kchunk + 2 * kBK - 1) / (2 * kBK) * (2 * kBK);  // whole pairs of steps
    kchunk = std::max(2 * kBK, std::min(kchunk, P_pad));
    g.kchunk = kchunk;
    g.nkc = (P_pad + kchunk - 1) / kchunk;
    return g;
}

bool gemm_path(Prec prec, int NP, int S) {
    // the fused kernel reads G once per block of 8 or 16 systems: with many
    // blocks and many loops the two passes read it far fewer times
    return NP > kMaxLoops && S >= (prec == Prec::F64 ? 64 : 128);
}

size_t gemm_ws_bytes(int NP, int S, int P_pad) {
    // the largest precision's X^T and W^T (FP64: 8 bytes; bf16 hi/lo: 4)
    const int N = (2 * S + 127) / 128 * 128;
    return ((size_t)N * NP + (size_t)N * P_pad) * sizeof(double) + 512;
}

hipError_t launch_gemm_loss(Prec prec, int loss_mode, bool grad, const GemmLoss &L,
                            hipStream_t st) {
    const GemmShape sh = gemm_shape(prec, L.NP, L.S, L.P_pad);
    const size_t esz = prec == Prec::F64 ? 8 : prec == Prec::F32 ? 4 : 2;
    const size_t nx = (size_t)sh.N * L.NP, nw = (size_t)sh.N * L.P_pad;
    char *ws = (char *)L.ws;
    char *X = ws, *Xlo = prec == Prec::BF16X3 ? X + nx * esz : nullptr;
    char *W = ws + ((nx * esz * (prec == Prec::BF16X3 ? 2 : 1) + 255) / 256) * 256;
    char *Wlo = prec == Prec::BF16X3 ? W + nw * esz : nullptr;
    GemmArgs fw;
    fw.A = L.G; fw.Alo = L.Glo; fw.B = X; fw.Blo = Xlo;
    fw.M = L.P_pad; fw.N = sh.N; fw.K = L.NP; fw.lda = L.NP; fw.ldb = L.NP;
    fw.kchunk = L.NP; fw.nkc = 1;
    fw.T = L.T; fw.inc = L.inc; fw.P = L.P;
    fw.W = grad ? W : nullptr; fw.Wlo = Wlo; fw.ldw = L.P_pad;
    fw.lpart = L.lpart; fw.S = L.S; fw.NP = L.NP;
    GemmArgs ad;
    ad.A = L.GT; ad.Alo = L.GTlo; ad.B = W; ad.Blo = Wlo;
    ad.M = L.NP; ad.N = sh.N; ad.K = L.P_pad; ad.lda = L.P_pad; ad.ldb = L.P_pad;
    ad.kchunk = sh.kchunk; ad.nkc = sh.nkc;
    ad.rpart = L.rpart; ad.S = L.S; ad.NP = L.NP;
    switch (prec) {
        case Prec::BF16X3: return go_pair<GBF3>(loss_mode, grad, fw, ad, L.I, L.n, st);
        case Prec::F32: return go_pair<GF32>(loss_mode, grad, fw, ad, L.I, L.n, st);
        case Prec::F64: return go_pair<GF64>(loss_mode, grad, fw, ad, L.I, L.n, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace cosim
