// Fused superposition + loss + adjoint contraction on gfx950 matrix cores.
//
// For every system s = (b, f) the forward product is B_z = G I (Eq. 7,
// z-component) and the loss of Eq. 1 needs, per field point, the residual
// weight w = dL/d conj(B); the gradient then needs r = G^T conj(w) (the
// adjoint right-hand side of Eq. 8-10).  Both are real-split contractions
// with the same G:
//     forward  [P x NP] . [NP x 2S]   (columns: Re I and Im I per system)
//     adjoint  [NP x P] . [P x 2S]
// One workgroup (4 waves) streams a P-chunk of G through LDS in 64-row tiles;
// each wave keeps I of its 16*NB systems as matrix-core B operands in
// registers for the whole chunk, computes B for a 16-row sub-tile with
// 16x16x4 MFMA (f32 or f64), turns it into w in registers, and feeds w
// straight back as the B operand of the adjoint MFMA: the accumulator layout
// of the forward product (register m of lane group q holds row row(q, m) of
// column lane%16) equals the operand layout of the adjoint product once the
// contraction index p is permuted to pi(4kk + q) = row(q, kk), so no data
// moves between the two.  B_z
// itself is never written.  The forward K index (loop k) is likewise permuted
// to sigma(4kk + q) = (NP/4) q + kk so that each lane reads NP/4 contiguous
// elements of a G row.  Partial r and loss per (chunk, system) go to memory
// and are summed in a fixed order by the solve/reduce kernels (no atomics).
//
// BF16X3: G = Gh + Gl and I = Ih + Il with bf16 hi/lo parts; the product is
// Gh Ih + Gh Il + Gl Ih accumulated in FP32 with 16x16x32 bf16 MFMA; w is split
// the same way for the adjoint.
#include <atomic>

#include "internal.h"
#include "epilogue.h"

namespace cosim {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Mma;
// row(g, m): row of the 16x16 accumulator held in register m by the lanes of
// group g = lane / 16 (the column is lane % 16).  Measured on gfx950:
// f32 16x16x4 keeps rows 4g..4g+3 per lane, f64 16x16x4 interleaves them
// (rows g, g+4, g+8, g+12).
template <>
struct Mma<float> {
    typedef f32x4 V;
    static __device__ inline V op(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ constexpr int row(int g, int m) { return 4 * g + m; }
};
template <>
struct Mma<double> {
    typedef f64x4 V;
    static __device__ inline V op(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ constexpr int row(int g, int m) { return g + 4 * m; }
};

template <typename T>
__device__ inline T tcast(double x) {
    return (T)x;
}

// One workgroup: system block bx (4 waves of 16 NB systems) of P-chunk `chunk`.
template <typename T, int NP, int NB, int LOSS, bool GRAD>
__device__ __forceinline__ void fused_block(const FusedArgs &a, int bx, int chunk) {
    typedef typename Mma<T>::V V;
    constexpr int KS = NP / 4;   // forward k-steps of 4
    constexpr int IB = NP / 16;  // 16-row blocks of the adjoint output
    constexpr int PT = kPTile;
    constexpr int LDR = NP + (sizeof(T) == 4 ? 4 : 2);  // padded LDS row
    __shared__ __attribute__((aligned(16))) T sG[PT * LDR];
    __shared__ T sT[PT];

    const T *__restrict__ G = (const T *)a.G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int sys0 = (bx * 4 + wave) * (16 * NB);
    const int pb = chunk * a.rows_per_chunk;
    const int pe = min(a.P_pad, pb + a.rows_per_chunk);

    // I as forward B operands: lane (r16, q), k-step kk holds I[sys][KS q + kk]
    T Ire[NB][KS], Iim[NB][KS];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int s = sys0 + 16 * b + r16;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int k = KS * q + kk;
            double2 v = make_double2(0.0, 0.0);
            if (s < a.S && k < a.n) v = a.I[(size_t)s * a.n + k];
            Ire[b][kk] = tcast<T>(v.x);
            Iim[b][kk] = tcast<T>(v.y);
        }
    }
    V racc[IB][NB][2];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            racc[ib][b][0] = V{};
            racc[ib][b][1] = V{};
        }
    double lacc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lacc[b] = 0.0;
    // FP32: the adjoint accumulators are flushed into FP64 after every 64-row
    // tile, so FP32 rounding accumulates over 64 rows only (the sum over P
    // cancels strongly: sum |G||w| reaches ~100 |G^T w| on the 8x8 array)
    constexpr bool FLUSH = sizeof(T) == 4;
    double r64[IB][NB][2][4];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int m = 0; m < 4; ++m) r64[ib][b][c][m] = 0.0;

    constexpr int E = 16 / sizeof(T);  // elements per 16-byte vector
    constexpr int NV = PT * NP / E;
    for (int p0 = pb; p0 < pe; p0 += PT) {
        __syncthreads();
        for (int v = threadIdx.x; v < NV; v += 256) {
            const int e0 = v * E;
            const int row = e0 / NP, col = e0 - row * NP;
            const uint4 val = *(const uint4 *)(G + (size_t)(p0 + row) * NP + col);
            *(uint4 *)(sG + row * LDR + col) = val;
        }
        if (threadIdx.x < PT) {
            const int p = p0 + threadIdx.x;
            // a padded row's field is the incident field alone: the target |inc|
            // makes its residual zero (inc = 0 outside the ratio mode)
            sT[threadIdx.x] = p < a.P ? tcast<T>(a.T[p]) : tcast<T>(fabs(a.inc));
        }
        __syncthreads();
#pragma unroll 1
        for (int sp = 0; sp < PT / 16; ++sp) {
            T af[KS];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) af[kk] = sG[(16 * sp + r16) * LDR + KS * q + kk];
            V br[NB], bi[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                br[b] = V{};
                bi[b] = V{};
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
                    br[b] = Mma<T>::op(af[kk], Ire[b][kk], br[b]);
                    bi[b] = Mma<T>::op(af[kk], Iim[b][kk], bi[b]);
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const T t = sT[16 * sp + Mma<T>::row(q, m)];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    T x = br[b][m], y = bi[b][m];
                    lacc[b] += epilogue<LOSS>(x, y, t, (T)a.inc);
                    br[b][m] = x;
                    bi[b][m] = y;
                }
            }
            if (GRAD) {
#pragma unroll
                for (int ib = 0; ib < IB; ++ib) {
                    T at[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        at[kk] = sG[(16 * sp + Mma<T>::row(q, kk)) * LDR + 16 * ib + r16];
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            racc[ib][b][0] = Mma<T>::op(at[kk], br[b][kk], racc[ib][b][0]);
                            racc[ib][b][1] = Mma<T>::op(at[kk], bi[b][kk], racc[ib][b][1]);
                        }
                }
            }
        }
        if (FLUSH && GRAD) {
#pragma unroll
            for (int ib = 0; ib < IB; ++ib)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
#pragma unroll
                        for (int m = 0; m < 4; ++m) r64[ib][b][c][m] += (double)racc[ib][b][c][m];
                        racc[ib][b][c] = V{};
                    }
        }
    }

    // ---- partial results of this chunk -------------------------------------
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int s = sys0 + 16 * b + r16;
        double v = lacc[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (s < a.S) {
            if (q == 0) a.lpart[(size_t)chunk * a.S + s] = v;
            if (GRAD) {
                double2 *dst = a.rpart + ((size_t)chunk * a.S + s) * NP;
#pragma unroll
                for (int ib = 0; ib < IB; ++ib)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        dst[16 * ib + Mma<T>::row(q, m)] =
                            FLUSH ? make_double2(r64[ib][b][0][m], r64[ib][b][1][m])
                                  : make_double2((double)racc[ib][b][0][m],
                                                 (double)racc[ib][b][1][m]);
            }
        }
    }
}

template <typename T, int NP, int NB, int LOSS, bool GRAD>
__global__ __launch_bounds__(256) void k_fused(FusedArgs a) {
    fused_block<T, NP, NB, LOSS, GRAD>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// BF16X3
// ---------------------------------------------------------------------------
__device__ inline f32x4 mma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// hi = RNE_bf16(x), lo = RNE_bf16(x - hi) (v_cvt_pk_bf16_f32 on gfx950)
__device__ inline void split2(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// split2 of two values at once, packed as they sit in an MFMA operand dword:
// one packed convert for the high parts, which are widened back from the
// packed dword itself (shift / mask), and one for the low parts.
__device__ inline void split2_pair(float a, float b, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
    const float ha = __builtin_bit_cast(float, hi << 16);
    const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2));
}

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Sub-tiles of 32 rows.  Forward: the 16-row halves of a sub-tile use K = 32
// (loop index; lane (r16, q) holds k = 8q..8q+7 of each 32-wide k-step).
// Adjoint: K = the sub-tile's 32 rows, taken from the two forward
// accumulators: lane (r16, q) supplies rows {4q..4q+3} of the first half and
// {16+4q..16+4q+3} of the second, i.e. pi(8q + j) = (j < 4 ? 4q + j :
// 16 + 4q + j - 4).  The adjoint A operand G^T[i][pi(8q + j)] is two 8-byte
// reads of the transposed tile held in LDS next to the row-major one.

// I of the wave's 16 NB systems as forward B operands (hi/lo), k-step kk:
// I[sys][32 kk + 8 q + j], j = 0..7.
template <int NP, int NB>
__device__ __forceinline__ void bf3_load_I(const FusedArgs &a, int sys0, int r16, int q,
                                           bf16x8 (&Ih)[NB][2][NP / 32],
                                           bf16x8 (&Il)[NB][2][NP / 32]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int s = sys0 + 16 * b + r16;
#pragma unroll
        for (int kk = 0; kk < NP / 32; ++kk) {
            // the block's 8 loads first (clamped, in bounds), then the splits,
            // so that the loads are in flight together
            double2 raw[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                raw[j] = a.I[(size_t)min(s, a.S - 1) * a.n + min(32 * kk + 8 * q + j, a.n - 1)];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * kk + 8 * q + j;
                const double2 v = s < a.S && k < a.n ? raw[j] : make_double2(0.0, 0.0);
                __bf16 h, l;
                split2((float)v.x, h, l);
                Ih[b][0][kk][j] = h;
                Il[b][0][kk][j] = l;
                split2((float)v.y, h, l);
                Ih[b][1][kk][j] = h;
                Il[b][1][kk][j] = l;
            }
        }
    }
}

// One PT-row tile of G (hi/lo, row-major with padded rows), of G^T (hi/lo,
// PT columns) and of T, moved global -> registers (fetch) -> LDS (stash) in
// 16-byte vectors by the 256 threads of the block.
template <int NP, int PT, bool GRAD>
struct Bf3Stage {
    static constexpr int NV = PT * NP / 8;
    static_assert(NV % 64 == 0, "tile must split evenly over whole waves");
    static constexpr int VPT = (NV + 255) / 256;
    static constexpr int LDR = NP + 8, LDT = PT + 8;
    u32x4 gh[VPT], gl[VPT], th[VPT], tl[VPT];
    // the target as loaded, converted at the stash so that the fetch does
    // not wait for its own loads; padded rows take |inc| (see k_fused)
    double t = 0.0;
    float tpad = 0.0f;
    bool pad = true;

    __device__ __forceinline__ void fetch(const FusedArgs &a, int p0) {
        const uint16_t *__restrict__ Gh = (const uint16_t *)a.G;
        const uint16_t *__restrict__ Gl = (const uint16_t *)a.Glo;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int e0 = (threadIdx.x + 256 * u) * 8;
            if (NV % 256 != 0 && e0 >= 8 * NV) continue;
            const int row = e0 / NP, col = e0 - row * NP;
            const size_t go = (size_t)(p0 + row) * NP + col;
            gh[u] = *(const u32x4 *)(Gh + go);
            gl[u] = *(const u32x4 *)(Gl + go);
            if (GRAD) {
                const int trow = e0 / PT, tcol = e0 - trow * PT;  // trow = loop index i
                const size_t to = (size_t)trow * a.P_pad + p0 + tcol;
                th[u] = *(const u32x4 *)(a.GThi + to);
                tl[u] = *(const u32x4 *)(a.GTlo + to);
            }
        }
        // every thread holds the target of row threadIdx.x % PT, so that the
        // store below needs no branch (equal values to equal addresses)
        const int p = p0 + (int)(threadIdx.x & (PT - 1));
        pad = p >= a.P;
        tpad = (float)fabs(a.inc);
        t = a.T[min(p, a.P - 1)];
    }
    __device__ __forceinline__ void stash(uint16_t *sH, uint16_t *sL, uint16_t *tH, uint16_t *tL,
                                          float *sT) const {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int e0 = (threadIdx.x + 256 * u) * 8;
            if (NV % 256 != 0 && e0 >= 8 * NV) continue;
            const int row = e0 / NP, col = e0 - row * NP;
            *(u32x4 *)(sH + row * LDR + col) = gh[u];
            *(u32x4 *)(sL + row * LDR + col) = gl[u];
            if (GRAD) {
                const int trow = e0 / PT, tcol = e0 - trow * PT;
                *(u32x4 *)(tH + trow * LDT + tcol) = th[u];
                *(u32x4 *)(tL + trow * LDT + tcol) = tl[u];
            }
        }
        sT[threadIdx.x & (PT - 1)] = pad ? tpad : (float)t;
    }
};

// Forward: B = G I for the 32 rows starting at row0 of the LDS tile, 16x16
// accumulators per 16-row half h and system group b.
template <int NP, int NB>
__device__ __forceinline__ void bf3_forward(const uint16_t *__restrict__ cH,
                                            const uint16_t *__restrict__ cL, int row0, int r16,
                                            int q, const bf16x8 (&Ih)[NB][2][NP / 32],
                                            const bf16x8 (&Il)[NB][2][NP / 32],
                                            f32x4 (&br)[2][NB], f32x4 (&bi)[2][NB]) {
    constexpr int KS = NP / 32, LDR = NP + 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = row0 + 16 * h + r16;
        bf16x8 ah[KS], al[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            ah[kk] = *(const bf16x8 *)(cH + row * LDR + 32 * kk + 8 * q);
            al[kk] = *(const bf16x8 *)(cL + row * LDR + 32 * kk + 8 * q);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            f32x4 xr = f32x4{}, xi = f32x4{};
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                xr = mma_bf16(al[kk], Ih[b][0][kk], xr);
                xr = mma_bf16(ah[kk], Il[b][0][kk], xr);
                xr = mma_bf16(ah[kk], Ih[b][0][kk], xr);
                xi = mma_bf16(al[kk], Ih[b][1][kk], xi);
                xi = mma_bf16(ah[kk], Il[b][1][kk], xi);
                xi = mma_bf16(ah[kk], Ih[b][1][kk], xi);
            }
            br[h][b] = xr;
            bi[h][b] = xi;
        }
    }
}

// Loss of the 32 rows starting at row0 (accumulated into lacc) and
// w = dL/d conj(B) as packed bf16 hi/lo adjoint B operands.
template <int NB, int LOSS>
__device__ __forceinline__ void bf3_epilogue(const float *__restrict__ sT, int row0, int q,
                                             const f32x4 (&br)[2][NB], const f32x4 (&bi)[2][NB],
                                             bf16x8 (&wrh)[NB], bf16x8 (&wrl)[NB],
                                             bf16x8 (&wih)[NB], bf16x8 (&wil)[NB],
                                             double (&lacc)[NB], float inc) {
    u32x4 rh[NB], rl[NB], ih[NB], il[NB];  // packed pairs of rows
    float lsub[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lsub[b] = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const f32x4 t4 = *(const f32x4 *)(sT + row0 + 16 * h + 4 * q);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            f32x4 x = br[h][b], y = bi[h][b];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                float xm = x[m], ym = y[m];
                lsub[b] += epilogue_f<LOSS>(xm, ym, t4[m], inc);
                x[m] = xm;
                y[m] = ym;
            }
#pragma unroll
            for (int mp = 0; mp < 2; ++mp) {
                unsigned hh, ll;
                split2_pair(x[2 * mp], x[2 * mp + 1], hh, ll);
                rh[b][2 * h + mp] = hh;
                rl[b][2 * h + mp] = ll;
                split2_pair(y[2 * mp], y[2 * mp + 1], hh, ll);
                ih[b][2 * h + mp] = hh;
                il[b][2 * h + mp] = ll;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        lacc[b] += (double)lsub[b];
        wrh[b] = __builtin_bit_cast(bf16x8, rh[b]);
        wrl[b] = __builtin_bit_cast(bf16x8, rl[b]);
        wih[b] = __builtin_bit_cast(bf16x8, ih[b]);
        wil[b] = __builtin_bit_cast(bf16x8, il[b]);
    }
}

// A operands of the adjoint for loop blocks ib0 .. ib0 + BATCH - 1:
// Gt[i = 16 ib + r16][p = pi(8q + j)] from the LDS tile.
template <int LDT, int BATCH>
__device__ __forceinline__ void bf3_adjoint_load(const uint16_t *__restrict__ ctH,
                                                 const uint16_t *__restrict__ ctL, int col0,
                                                 int r16, int q, int ib0, bf16x8 (&th)[BATCH],
                                                 bf16x8 (&tl)[BATCH]) {
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
        const int base = (16 * (ib0 + u) + r16) * LDT + col0 + 4 * q;
        const s16x4 h0 = *(const s16x4 *)(ctH + base), h1 = *(const s16x4 *)(ctH + base + 16);
        const s16x4 l0 = *(const s16x4 *)(ctL + base), l1 = *(const s16x4 *)(ctL + base + 16);
        th[u] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7));
        tl[u] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7));
    }
}

// Adjoint: racc += G^T w over the 32 rows starting at column col0 of the
// transposed LDS tile (row stride LDT).  BATCH blocks of 16 loops have their
// operands read from LDS together, before their products (BATCH > 1 trades
// registers for fewer exposed LDS latencies).  PRE: the first batch's
// operands were loaded by the caller (pth, ptl).
template <int NP, int NB, int LDT, int BATCH = 1, bool PRE = false>
__device__ __forceinline__ void bf3_adjoint(const uint16_t *__restrict__ ctH,
                                            const uint16_t *__restrict__ ctL, int col0, int r16,
                                            int q, const bf16x8 (&wrh)[NB],
                                            const bf16x8 (&wrl)[NB], const bf16x8 (&wih)[NB],
                                            const bf16x8 (&wil)[NB],
                                            f32x4 (&racc)[NP / 16][NB][2],
                                            const bf16x8 *pth = nullptr,
                                            const bf16x8 *ptl = nullptr) {
    static_assert((NP / 16) % BATCH == 0, "whole batches of loop blocks");
#pragma unroll
    for (int ib0 = 0; ib0 < NP / 16; ib0 += BATCH) {
        bf16x8 th[BATCH], tl[BATCH];
        if (PRE && ib0 == 0) {
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                th[u] = pth[u];
                tl[u] = ptl[u];
            }
        } else {
            bf3_adjoint_load<LDT, BATCH>(ctH, ctL, col0, r16, q, ib0, th, tl);
        }
        if constexpr (BATCH > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int ib = ib0 + u;
                racc[ib][b][0] = mma_bf16(tl[u], wrh[b], racc[ib][b][0]);
                racc[ib][b][0] = mma_bf16(th[u], wrl[b], racc[ib][b][0]);
                racc[ib][b][0] = mma_bf16(th[u], wrh[b], racc[ib][b][0]);
                racc[ib][b][1] = mma_bf16(tl[u], wih[b], racc[ib][b][1]);
                racc[ib][b][1] = mma_bf16(th[u], wil[b], racc[ib][b][1]);
                racc[ib][b][1] = mma_bf16(th[u], wih[b], racc[ib][b][1]);
            }
        if constexpr (BATCH > 1) __builtin_amdgcn_sched_barrier(0);
    }
}

// Per-chunk partial loss and adjoint right-hand side of the wave's systems.
template <int NP, int NB, bool GRAD>
__device__ __forceinline__ void bf3_store(const FusedArgs &a, int chunk, int sys0, int r16, int q,
                                          const double (&lacc)[NB],
                                          const f32x4 (&racc)[NP / 16][NB][2]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int s = sys0 + 16 * b + r16;
        double v = lacc[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (s < a.S) {
            if (q == 0) a.lpart[(size_t)chunk * a.S + s] = v;
            if (GRAD) {
                double2 *dst = a.rpart + ((size_t)chunk * a.S + s) * NP;
#pragma unroll
                for (int ib = 0; ib < NP / 16; ++ib)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        dst[16 * ib + 4 * q + m] = make_double2((double)racc[ib][b][0][m],
                                                                (double)racc[ib][b][1][m]);
            }
        }
    }
}

// Sub-tile by sub-tile: forward, epilogue, adjoint.
// DB: two LDS buffers, the next tile's global loads in flight in registers
// while the current tile is computed (one barrier per tile); otherwise one
// buffer, loaded between two barriers (half the LDS, so more blocks per CU).
template <int NP, int NB, int PT, bool DB, int LOSS, bool GRAD>
__device__ __forceinline__ void bf3_block(const FusedArgs &a, int bx, int chunk) {
    static_assert(NP % 32 == 0, "bf16x3 path needs NP multiple of 32");
    static_assert(kPTile % PT == 0, "tile rows must divide the 64-row padding of G");
    constexpr int IB = NP / 16;
    constexpr int LDR = NP + 8, LDT = PT + 8;
    constexpr int TSZ = PT * LDR, TTSZ = GRAD ? NP * LDT : 8;
    constexpr int NBUF = DB ? 2 : 1;
    __shared__ __attribute__((aligned(16))) uint16_t sH[NBUF][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t sL[NBUF][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tH[NBUF][TTSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tL[NBUF][TTSZ];
    __shared__ __attribute__((aligned(16))) float sTg[NBUF][PT];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int sys0 = (bx * 4 + wave) * (16 * NB);
    const int pb = chunk * a.rows_per_chunk;
    const int pe = min(a.P_pad, pb + a.rows_per_chunk);

    bf16x8 Ih[NB][2][NP / 32], Il[NB][2][NP / 32];
    bf3_load_I<NP, NB>(a, sys0, r16, q, Ih, Il);
    f32x4 racc[IB][NB][2];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int b = 0; b < NB; ++b) racc[ib][b][0] = racc[ib][b][1] = f32x4{};
    double lacc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lacc[b] = 0.0;

    Bf3Stage<NP, PT, GRAD> stg;
    if (DB) {
        if (pb < pe) {
            stg.fetch(a, pb);
            stg.stash(sH[0], sL[0], tH[0], tL[0], sTg[0]);
        }
        __syncthreads();
    }
    int cur = 0;
    for (int p0 = pb; p0 < pe; p0 += PT, cur ^= (DB ? 1 : 0)) {
        const bool more = p0 + PT < pe;
        if (DB) {
            if (more) stg.fetch(a, p0 + PT);  // loads in flight during the compute below
        } else {
            if (p0 != pb) __syncthreads();  // every wave is done with the previous tile
            stg.fetch(a, p0);
            stg.stash(sH[0], sL[0], tH[0], tL[0], sTg[0]);
            __syncthreads();
        }
#pragma unroll 1
        for (int sp = 0; sp < PT / 32; ++sp) {
            f32x4 br[2][NB], bi[2][NB];
            bf3_forward<NP, NB>(sH[cur], sL[cur], 32 * sp, r16, q, Ih, Il, br, bi);
            bf16x8 wrh[NB], wrl[NB], wih[NB], wil[NB];
            bf3_epilogue<NB, LOSS>(sTg[cur], 32 * sp, q, br, bi, wrh, wrl, wih, wil, lacc, (float)a.inc);
            if (GRAD) bf3_adjoint<NP, NB, LDT>(tH[cur], tL[cur], 32 * sp, r16, q, wrh, wrl, wih, wil, racc);
        }
        if (DB) {
            if (more) stg.stash(sH[cur ^ 1], sL[cur ^ 1], tH[cur ^ 1], tL[cur ^ 1], sTg[cur ^ 1]);
            __syncthreads();
        }
    }
    bf3_store<NP, NB, GRAD>(a, chunk, sys0, r16, q, lacc, racc);
}

template <int NP, int NB, int PT, bool DB, int LOSS, bool GRAD>
__global__ __launch_bounds__(256, 2) void k_fused_bf16x3(FusedArgs a) {
    bf3_block<NP, NB, PT, DB, LOSS, GRAD>(a, blockIdx.x, blockIdx.y);
}

// The default variant (0) of each precision over the members of a group of
// plans: workgroup b belongs to the member with first[m] <= b < first[m + 1]
// and is its workgroup b - first[m] in (system block, chunk) order, system
// blocks fastest.
template <typename T, int NP, int LOSS, bool GRAD>
__global__ __launch_bounds__(256) void k_fused_group(FusedGroup g) {
    const int b = blockIdx.x;
    int m = 0;
    while (m + 1 < g.count && b >= g.first[m + 1]) ++m;
    const int loc = b - g.first[m], bxn = g.bx[m];
    fused_block<T, NP, (sizeof(T) == 8 ? 1 : 2), LOSS, GRAD>(g.in[m], loc % bxn, loc / bxn);
}
template <int NP, int LOSS, bool GRAD>
__global__ __launch_bounds__(256, 2) void k_fused_bf16x3_group(FusedGroup g) {
    const int b = blockIdx.x;
    int m = 0;
    while (m + 1 < g.count && b >= g.first[m + 1]) ++m;
    const int loc = b - g.first[m], bxn = g.bx[m];
    bf3_block<NP, 2, 64, false, LOSS, GRAD>(g.in[m], loc % bxn, loc / bxn);
}

// Software-pipelined form: the forward MFMAs of sub-tile j+1 are issued in the
// same basic block as the epilogue (VALU) of sub-tile j, so the matrix cores
// and the vector ALUs of a wave work side by side; the adjoint of sub-tile j
// follows.  Tiles are double-buffered; crossing into tile t+1 costs two
// barriers (every wave done with the buffer tile t-1 used, then tile t+1
// visible), and tile t+2 is fetched into registers right after.  The last
// iteration's look-ahead forward reads a stale buffer and is discarded.
template <int NP, int NB, int PT, int LOSS, bool GRAD>
__global__ __launch_bounds__(256, 2) void k_fused_bf16x3_pipe(FusedArgs a) {
    static_assert(NP % 32 == 0, "bf16x3 path needs NP multiple of 32");
    static_assert(kPTile % PT == 0, "tile rows must divide the 64-row padding of G");
    constexpr int IB = NP / 16;
    constexpr int LDR = NP + 8, LDT = PT + 8;
    constexpr int TSZ = PT * LDR, TTSZ = GRAD ? NP * LDT : 8;
    constexpr int SPT = PT / 32;  // sub-tiles per tile
    __shared__ __attribute__((aligned(16))) uint16_t sH[2][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t sL[2][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tH[2][TTSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tL[2][TTSZ];
    __shared__ __attribute__((aligned(16))) float sTg[2][PT];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int sys0 = (blockIdx.x * 4 + wave) * (16 * NB);
    const int chunk = blockIdx.y;
    const int pb = chunk * a.rows_per_chunk;
    const int pe = min(a.P_pad, pb + a.rows_per_chunk);
    const int ntile = pe > pb ? (pe - pb) / PT : 0;

    bf16x8 Ih[NB][2][NP / 32], Il[NB][2][NP / 32];
    bf3_load_I<NP, NB>(a, sys0, r16, q, Ih, Il);
    f32x4 racc[IB][NB][2];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int b = 0; b < NB; ++b) racc[ib][b][0] = racc[ib][b][1] = f32x4{};
    double lacc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lacc[b] = 0.0;

    if (ntile > 0) {
        Bf3Stage<NP, PT, GRAD> stg;
        stg.fetch(a, pb);
        stg.stash(sH[0], sL[0], tH[0], tL[0], sTg[0]);
        __syncthreads();
        if (ntile > 1) stg.fetch(a, pb + PT);
        f32x4 br[2][NB], bi[2][NB];
        bf3_forward<NP, NB>(sH[0], sL[0], 0, r16, q, Ih, Il, br, bi);
        const int nsub = ntile * SPT;
#pragma unroll 1
        for (int j = 0; j < nsub; ++j) {
            const int t = j / SPT, s = j - t * SPT;
            const int t1 = (j + 1) / SPT, s1 = (j + 1) - t1 * SPT;
            if (s1 == 0 && t1 < ntile) {  // uniform over the block
                __syncthreads();
                stg.stash(sH[t1 & 1], sL[t1 & 1], tH[t1 & 1], tL[t1 & 1], sTg[t1 & 1]);
                __syncthreads();
                if (t1 + 1 < ntile) stg.fetch(a, pb + (t1 + 1) * PT);
            }
            f32x4 brn[2][NB], bin[2][NB];
            bf3_forward<NP, NB>(sH[t1 & 1], sL[t1 & 1], 32 * s1, r16, q, Ih, Il, brn, bin);
            bf16x8 wrh[NB], wrl[NB], wih[NB], wil[NB];
            bf3_epilogue<NB, LOSS>(sTg[t & 1], 32 * s, q, br, bi, wrh, wrl, wih, wil, lacc, (float)a.inc);
            if (GRAD) bf3_adjoint<NP, NB, LDT>(tH[t & 1], tL[t & 1], 32 * s, r16, q, wrh, wrl, wih, wil, racc);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    br[h][b] = brn[h][b];
                    bi[h][b] = bin[h][b];
                }
        }
    }
    bf3_store<NP, NB, GRAD>(a, chunk, sys0, r16, q, lacc, racc);
}

// Ping-pong form: eight waves in two groups of four, waves w and w + 4 on one
// SIMD.  A wave cannot run its own vector work beside its own matrix-core
// products, but the two waves of a SIMD can run side by side; so the work is
// cut into phases separated by workgroup barriers, and in every phase one
// group runs matrix-core work (the adjoint of sub-tile j - 1 and the forward
// product of sub-tile j) while the other runs the vector epilogue of its
// current sub-tile.  Group 1 runs one phase behind group 0 (OFF = 1), so
// the two waves of a SIMD swap roles at every barrier; with OFF = 0 both
// groups run in step (every wave of a SIMD in the same kind of phase), the
// form to compare against.
//   Tile t (32-row sub-tiles 2t and 2t + 1) sits in LDS buffer t & 1 and is
// read in phases 4t .. 4t + 4 + OFF.  The rows of G for tile u >= 2 are
// written to LDS by group 1 in phase 4u - 1 - OFF, those of G^T and the
// targets by group 0 in phase 4u - 1: each in that group's vector phase,
// after the last read of the tile the buffer held before and before the
// barrier that opens phase 4u.  Each group fetches its share of a tile into
// registers right after storing the previous one, four phases ahead.
// Barriers wait for LDS traffic only, so global loads stay in flight across
// them.  A wave raises its issue priority for its matrix-core phases, so that
// where both waves of a SIMD have an instruction ready the products go first
// (the other way round, the kernel runs 4% slower; with equal priorities 2%).
template <int NP, int PT, bool GRAD>
struct PpStage {
    static constexpr int NV = PT * NP / 8;  // 16-byte vectors per plane
    static constexpr int VPT = (NV + 255) / 256;
    static constexpr int LDR = NP + 8, LDT = PT + 8;
    u32x4 h[VPT], l[VPT];
    double t = 0.0;  // target as loaded (see Bf3Stage)
    float tpad = 0.0f;
    bool pad = true;

    // group 1: rows of G; group 0: columns of G^T and the targets
    __device__ __forceinline__ void fetch(const FusedArgs &a, int p0, int grp, int gtid) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int e0 = (gtid + 256 * u) * 8;
            if (NV % 256 != 0 && e0 >= 8 * NV) continue;
            if (grp) {
                const int row = e0 / NP, col = e0 - row * NP;
                const size_t go = (size_t)(p0 + row) * NP + col;
                h[u] = *(const u32x4 *)((const uint16_t *)a.G + go);
                l[u] = *(const u32x4 *)((const uint16_t *)a.Glo + go);
            } else if (GRAD) {
                const int trow = e0 / PT, tcol = e0 - trow * PT;
                const size_t to = (size_t)trow * a.P_pad + p0 + tcol;
                h[u] = *(const u32x4 *)(a.GThi + to);
                l[u] = *(const u32x4 *)(a.GTlo + to);
            }
        }
        if (!grp) {
            const int p = p0 + (gtid & (PT - 1));
            pad = p >= a.P;
            tpad = (float)fabs(a.inc);
            t = a.T[min(p, a.P - 1)];
        }
    }
    __device__ __forceinline__ void stash(uint16_t *sH, uint16_t *sL, uint16_t *tH, uint16_t *tL,
                                          float *sT, int grp, int gtid) const {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int e0 = (gtid + 256 * u) * 8;
            if (NV % 256 != 0 && e0 >= 8 * NV) continue;
            if (grp) {
                const int row = e0 / NP, col = e0 - row * NP;
                *(u32x4 *)(sH + row * LDR + col) = h[u];
                *(u32x4 *)(sL + row * LDR + col) = l[u];
            } else if (GRAD) {
                const int trow = e0 / PT, tcol = e0 - trow * PT;
                *(u32x4 *)(tH + trow * LDT + tcol) = h[u];
                *(u32x4 *)(tL + trow * LDT + tcol) = l[u];
            }
        }
        if (!grp) sT[gtid & (PT - 1)] = pad ? tpad : (float)t;
    }
};

// Barrier that waits for the wave's LDS operations only (global loads issued
// before it stay in flight).  The scheduling barriers keep the compiler from
// moving any instruction across it, so that each phase's matrix-core and
// vector work stays in its phase.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    __builtin_amdgcn_sched_barrier(0);
}
// The same with `issue` (LDS loads of data that an earlier barrier already
// published) placed after the release fence, so that they are in flight
// while the wave waits at the barrier.
template <typename F>
__device__ __forceinline__ void lds_barrier_then(F &&issue) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_sched_barrier(0);
    issue();
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    __builtin_amdgcn_sched_barrier(0);
}

// An empty use of a register value: the value has to be computed before
// this point, which keeps the compiler from sinking a phase's arithmetic past
// the barrier that ends the phase (scheduling barriers act inside one basic
// block only).
template <typename T>
__device__ __forceinline__ void keep(const T &v) {
    asm volatile("" ::"v"(v));
}

template <int NP, int NB, int OFF, int LOSS, bool GRAD>
__global__ __launch_bounds__(512, 1) void k_fused_bf16x3_pp(FusedArgs a) {
    static_assert(NP % 32 == 0, "bf16x3 path needs NP multiple of 32");
    constexpr int PT = 64, SPT = 2;  // tile rows, 32-row sub-tiles per tile
    static_assert(kPTile % PT == 0, "tile rows must divide the 64-row padding of G");
    constexpr int IB = NP / 16;
    constexpr int LDR = NP + 8, LDT = PT + 8;
    constexpr int TSZ = PT * LDR, TTSZ = GRAD ? NP * LDT : 8;
    __shared__ __attribute__((aligned(16))) uint16_t sH[2][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t sL[2][TSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tH[2][TTSZ];
    __shared__ __attribute__((aligned(16))) uint16_t tL[2][TTSZ];
    __shared__ __attribute__((aligned(16))) float sTg[2][PT];

    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = wave >> 2, gtid = tid & 255;
    const int sgrp = OFF ? grp : 0;  // phase lag of the group
    const int r16 = lane & 15, q = lane >> 4;
    const int sys0 = (blockIdx.x * 8 + wave) * (16 * NB);
    const int chunk = blockIdx.y;
    const int pb = chunk * a.rows_per_chunk;
    const int pe = min(a.P_pad, pb + a.rows_per_chunk);
    const int ntile = pe > pb ? (pe - pb) / PT : 0;
    const int nsub = ntile * SPT;

    bf16x8 Ih[NB][2][NP / 32], Il[NB][2][NP / 32];
    bf3_load_I<NP, NB>(a, sys0, r16, q, Ih, Il);
    f32x4 racc[IB][NB][2];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int b = 0; b < NB; ++b) racc[ib][b][0] = racc[ib][b][1] = f32x4{};
    double lacc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lacc[b] = 0.0;

    PpStage<NP, PT, GRAD> stg;
    for (int u = 0; u < min(ntile, 2); ++u) {
        stg.fetch(a, pb + u * PT, grp, gtid);
        stg.stash(sH[u], sL[u], tH[u], tL[u], sTg[u], grp, gtid);
    }
    __syncthreads();

    // Every wave runs (matrix-core phase j; barrier; vector phase j;
    // barrier) for j = 0 .. nsub; with OFF, group 1 enters one barrier late
    // and group 0 leaves one barrier late, so both pass the same barriers and
    // the global phase of a group's local phase k is k + sgrp (its lag).  The
    // first and last matrix-core phases are peeled, so that in the others the
    // adjoint of sub-tile j - 1 and the forward product of sub-tile j sit in
    // one block.
    f32x4 br[2][NB], bi[2][NB];
    bf16x8 wrh[NB], wrl[NB], wih[NB], wil[NB];
    // The first operand batch of adjoint(jj) is loaded during the barrier
    // that ends vector phase jj: its tile was published one matrix-core
    // phase earlier (forward(jj) read it), and its buffer is not stored again
    // before adjoint(jj) has run, so the loads wait for nothing and the
    // matrix-core phase starts on operands already in registers.
    bf16x8 pth[2], ptl[2];
    auto preload = [&](int jj) {
        const int bf = (jj / SPT) & 1;
        bf3_adjoint_load<LDT, 2>(tH[bf], tL[bf], 32 * (jj % SPT), r16, q, 0, pth, ptl);
    };
    auto adjoint = [&](int jj) {
        const int bf = (jj / SPT) & 1;
        bf3_adjoint<NP, NB, LDT, 2, true>(tH[bf], tL[bf], 32 * (jj % SPT), r16, q, wrh, wrl, wih,
                                          wil, racc, pth, ptl);
    };
    auto end_vector_phase = [&](int j) {
        if constexpr (GRAD)
            lds_barrier_then([&] { preload(j); });
        else
            lds_barrier();
    };
    auto forward = [&](int j) {
        const int bf = (j / SPT) & 1;
        bf3_forward<NP, NB>(sH[bf], sL[bf], 32 * (j % SPT), r16, q, Ih, Il, br, bi);
    };
    // Vector phase j (global phase 2j + 1 + sgrp): in every other one, those
    // with j + sgrp odd, the group stores its share of tile u = (j + 1 +
    // sgrp) / 2 in LDS (fetched four phases earlier) and then fetches its
    // share of tile u + 1 into the same registers (the scheduling barrier
    // keeps the loads after the stores, so that the registers are reused in
    // place rather than copied, a copy waiting for the loads); then the
    // epilogue of sub-tile j.
    auto vector_phase = [&](int j) {
        if ((j + sgrp) & 1) {
            const int u = (j + 1 + sgrp) >> 1;
            if (u >= 2 && u < ntile)
                stg.stash(sH[u & 1], sL[u & 1], tH[u & 1], tL[u & 1], sTg[u & 1], grp, gtid);
            __builtin_amdgcn_sched_barrier(0);
            if (u + 1 >= 2 && u + 1 < ntile) stg.fetch(a, pb + (u + 1) * PT, grp, gtid);
        }
        if (j < nsub) {
            const int bf = (j / SPT) & 1;
            bf3_epilogue<NB, LOSS>(sTg[bf], 32 * (j % SPT), q, br, bi, wrh, wrl, wih, wil, lacc,
                                   (float)a.inc);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                keep(wrh[b]);
                keep(wrl[b]);
                keep(wih[b]);
                keep(wil[b]);
                keep(lacc[b]);
            }

        }
    };
    auto keep_forward = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                keep(br[h][b]);
                keep(bi[h][b]);
            }
    };
    auto keep_adjoint = [&]() {
#pragma unroll
        for (int ib = 0; ib < IB; ++ib)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                keep(racc[ib][b][0]);
                keep(racc[ib][b][1]);
            }
    };
    if (OFF && grp) lds_barrier();
    if (nsub > 0) {
        __builtin_amdgcn_s_setprio(2);
        forward(0);
        keep_forward();
        __builtin_amdgcn_s_setprio(0);
        lds_barrier();
        vector_phase(0);
        end_vector_phase(0);
#pragma unroll 1
        for (int j = 1; j < nsub; ++j) {
            __builtin_amdgcn_s_setprio(2);
            if (GRAD) adjoint(j - 1);
            forward(j);
            if (GRAD) keep_adjoint();
            keep_forward();
            __builtin_amdgcn_s_setprio(0);
            lds_barrier();
            vector_phase(j);
            end_vector_phase(j);
        }
        if (GRAD) {
            adjoint(nsub - 1);
            keep_adjoint();
        }
    }
    lds_barrier();
    vector_phase(nsub);  // staging only: nothing is left to reduce
    lds_barrier();
    if (OFF && !grp) lds_barrier();
    bf3_store<NP, NB, GRAD>(a, chunk, sys0, r16, q, lacc, racc);
}

// Tuning variants of the fused kernels: systems per wave (16 * NB), rows per
// LDS tile (PT) and, for BF16X3, single or double LDS buffering.  Variant 0 is
// the default; cosim_plan_autotune picks per plan and precision.
struct Variant {
    int nb, pt;
    bool db;
    int pipe;  // 0: sub-tile by sub-tile, 1: look-ahead forward of the next sub-tile,
               // 2: ping-pong of two wave groups (eight waves, 32 NB systems per SIMD pair),
               // 3: the same eight-wave kernel with both groups in step
};
constexpr Variant kVarF64[] = {{1, 64, false, 0}, {2, 64, false, 0}};
constexpr Variant kVarF32[] = {{2, 64, false, 0}, {1, 64, false, 0}};
constexpr Variant kVarBF16[] = {{2, 64, false, 0}, {2, 32, false, 0}, {1, 64, false, 0},
                                {1, 32, false, 0}, {2, 64, true, 0},  {2, 32, true, 0},
                                {1, 64, true, 1},  {1, 32, true, 1},  {2, 32, true, 1},
                                {2, 64, true, 1}, {2, 64, true, 2}, {1, 64, true, 2},
                                {2, 64, true, 3}};
// the group kernels hard-wire variant 0 of each precision
static_assert(kVarF64[0].nb == 1 && kVarF32[0].nb == 2 && kVarBF16[0].nb == 2 &&
                  kVarBF16[0].pt == 64 && !kVarBF16[0].db && kVarBF16[0].pipe == 0,
              "k_fused_group / k_fused_bf16x3_group follow variant 0");

// With `occ` set, the resident-workgroup count per compute unit of the
// kernel is written there and nothing is launched.
template <typename K>
hipError_t occupancy_of(K kernel, int *occ, int threads = 256) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kernel, threads, 0);
}

template <typename T, int NP, int NB, int LOSS, bool GRAD>
hipError_t go_typed(const FusedArgs &a, hipStream_t st, int *occ) {
    if (occ) return occupancy_of(k_fused<T, NP, NB, LOSS, GRAD>, occ);
    const int per_block = 4 * 16 * NB;
    dim3 grid((a.S + per_block - 1) / per_block, a.nchunk);
    hipLaunchKernelGGL((k_fused<T, NP, NB, LOSS, GRAD>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int NP, int NB, int PT, bool DB, int PIPE, int LOSS, bool GRAD>
hipError_t go_bf16(const FusedArgs &a, hipStream_t st, int *occ) {
    if (occ) {
        if constexpr (PIPE >= 2) return occupancy_of(k_fused_bf16x3_pp<NP, NB, PIPE == 2, LOSS, GRAD>, occ, 512);
        else if constexpr (PIPE == 1) return occupancy_of(k_fused_bf16x3_pipe<NP, NB, PT, LOSS, GRAD>, occ);
        else return occupancy_of(k_fused_bf16x3<NP, NB, PT, DB, LOSS, GRAD>, occ);
    }
    const int per_block = (PIPE >= 2 ? 8 : 4) * 16 * NB;
    dim3 grid((a.S + per_block - 1) / per_block, a.nchunk);
    if constexpr (PIPE >= 2)
        hipLaunchKernelGGL((k_fused_bf16x3_pp<NP, NB, PIPE == 2, LOSS, GRAD>), grid, dim3(512), 0, st, a);
    else if constexpr (PIPE == 1)
        hipLaunchKernelGGL((k_fused_bf16x3_pipe<NP, NB, PT, LOSS, GRAD>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_fused_bf16x3<NP, NB, PT, DB, LOSS, GRAD>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int NP, int LOSS, bool GRAD>
hipError_t go_np(Prec prec, int variant, const FusedArgs &a, hipStream_t st, int *occ) {
    switch (prec) {
        case Prec::F64:
            switch (variant) {
                case 0: return go_typed<double, NP, 1, LOSS, GRAD>(a, st, occ);
                case 1: return go_typed<double, NP, 2, LOSS, GRAD>(a, st, occ);
            }
            break;
        case Prec::F32:
            switch (variant) {
                case 0: return go_typed<float, NP, 2, LOSS, GRAD>(a, st, occ);
                case 1: return go_typed<float, NP, 1, LOSS, GRAD>(a, st, occ);
            }
            break;
        case Prec::BF16X3:
            if constexpr (NP % 32 == 0) {
                switch (variant) {
#define COSIM_BF16_CASE(i)                                                               \
    case i:                                                                              \
        return go_bf16<NP, kVarBF16[i].nb, kVarBF16[i].pt, kVarBF16[i].db, kVarBF16[i].pipe, \
                       LOSS, GRAD>(a, st, occ);
                    COSIM_BF16_CASE(0)
                    COSIM_BF16_CASE(1)
                    COSIM_BF16_CASE(2)
                    COSIM_BF16_CASE(3)
                    COSIM_BF16_CASE(4)
                    COSIM_BF16_CASE(5)
                    COSIM_BF16_CASE(6)
                    COSIM_BF16_CASE(7)
                    COSIM_BF16_CASE(8)
                    COSIM_BF16_CASE(9)
                    COSIM_BF16_CASE(10)
                    COSIM_BF16_CASE(11)
                    COSIM_BF16_CASE(12)
#undef COSIM_BF16_CASE
                }
            }
            break;
    }
    return hipErrorInvalidValue;
}

template <int LOSS, bool GRAD>
hipError_t go_loss(Prec prec, int NP, int variant, const FusedArgs &a, hipStream_t st,
                   int *occ = nullptr) {
    switch (NP) {
        case 32: return go_np<32, LOSS, GRAD>(prec, variant, a, st, occ);
        case 64: return go_np<64, LOSS, GRAD>(prec, variant, a, st, occ);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int fused_variant_count(Prec prec) {
    switch (prec) {
        case Prec::F64: return (int)(sizeof(kVarF64) / sizeof(Variant));
        case Prec::F32: return (int)(sizeof(kVarF32) / sizeof(Variant));
        case Prec::BF16X3: return (int)(sizeof(kVarBF16) / sizeof(Variant));
    }
    return 1;
}

int fused_systems_per_block(Prec prec, int NP, int variant) {
    (void)NP;
    switch (prec) {
        case Prec::F64: return 64 * kVarF64[variant].nb;
        case Prec::F32: return 64 * kVarF32[variant].nb;
        case Prec::BF16X3: return (kVarBF16[variant].pipe >= 2 ? 128 : 64) * kVarBF16[variant].nb;
    }
    return 64;
}

int fused_blocks_per_cu(Prec prec, int NP, int variant) {
    // per (precision, NP 32 / 64, variant); the magnitude loss with gradient
    // stands for every loss mode (their register and LDS use agree)
    static std::atomic<int> cache[3][2][16];
    const int pi = (int)prec, ni = NP == 32 ? 0 : 1;
    if (pi < 0 || pi > 2 || (NP != 32 && NP != 64) || variant < 0 || variant >= 16) return 1;
    int v = cache[pi][ni][variant].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int occ = 0;
    if (go_loss<COSIM_LOSS_MAG, true>(prec, NP, variant, FusedArgs{}, nullptr, &occ) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    cache[pi][ni][variant].store(occ, std::memory_order_relaxed);
    return occ;
}

namespace {
template <int LOSS, bool GRAD>
hipError_t go_group(Prec prec, int NP, const FusedGroup &g, int blocks, hipStream_t st) {
#define COSIM_FUSED_GROUP(NPC)                                                                      \
    switch (prec) {                                                                                \
        case Prec::F64:                                                                            \
            hipLaunchKernelGGL((k_fused_group<double, NPC, LOSS, GRAD>), dim3(blocks), dim3(256),  \
                               0, st, g);                                                          \
            break;                                                                                 \
        case Prec::F32:                                                                            \
            hipLaunchKernelGGL((k_fused_group<float, NPC, LOSS, GRAD>), dim3(blocks), dim3(256),   \
                               0, st, g);                                                          \
            break;                                                                                 \
        case Prec::BF16X3:                                                                         \
            hipLaunchKernelGGL((k_fused_bf16x3_group<NPC, LOSS, GRAD>), dim3(blocks), dim3(256),   \
                               0, st, g);                                                          \
            break;                                                                                 \
    }
    switch (NP) {
        case 32:
            COSIM_FUSED_GROUP(32)
            break;
        case 64:
            COSIM_FUSED_GROUP(64)
            break;
        default:
            return hipErrorInvalidValue;
    }
#undef COSIM_FUSED_GROUP
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fused_group(Prec prec, int NP, int loss_mode, bool grad, const FusedGroup &g,
                              int blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    if (loss_mode == COSIM_LOSS_MAG)
        return grad ? go_group<COSIM_LOSS_MAG, true>(prec, NP, g, blocks, st)
                    : go_group<COSIM_LOSS_MAG, false>(prec, NP, g, blocks, st);
    if (loss_mode == COSIM_LOSS_RATIO)
        return grad ? go_group<COSIM_LOSS_RATIO, true>(prec, NP, g, blocks, st)
                    : go_group<COSIM_LOSS_RATIO, false>(prec, NP, g, blocks, st);
    return grad ? go_group<COSIM_LOSS_COMPLEX, true>(prec, NP, g, blocks, st)
                : go_group<COSIM_LOSS_COMPLEX, false>(prec, NP, g, blocks, st);
}

hipError_t launch_fused(Prec prec, int NP, int variant, int loss_mode, bool grad,
                        const FusedArgs &a, hipStream_t st) {
    if (variant < 0 || variant >= fused_variant_count(prec)) return hipErrorInvalidValue;
    if (loss_mode == COSIM_LOSS_MAG) {
        return grad ? go_loss<COSIM_LOSS_MAG, true>(prec, NP, variant, a, st)
                    : go_loss<COSIM_LOSS_MAG, false>(prec, NP, variant, a, st);
    }
    if (loss_mode == COSIM_LOSS_RATIO) {
        return grad ? go_loss<COSIM_LOSS_RATIO, true>(prec, NP, variant, a, st)
                    : go_loss<COSIM_LOSS_RATIO, false>(prec, NP, variant, a, st);
    }
    return grad ? go_loss<COSIM_LOSS_COMPLEX, true>(prec, NP, variant, a, st)
                : go_loss<COSIM_LOSS_COMPLEX, false>(prec, NP, variant, a, st);
}

}  // namespace cosim
