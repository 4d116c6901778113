// Matrix-core contractions of the field superposition for any padded loop
// count NP (a multiple of 32 up to 1,024), one kernel family for three uses:
//   loss (+ gradient)  B = G I (Eq. 7), the loss of Eq. 1 and w = dL/d conj(B)
//                      in registers, then r = G^T w (the adjoint right-hand
//                      side of Eq. 8-10) from the same tile of points; B is
//                      never written;
//   field              B = G I written out (cosim_field);
//   vector-Jacobian    r = G^T g of an upstream field gradient g
//                      (cosim_field_backward).
// All three are real-split: the columns of a workgroup are the real parts of
// the currents of its NS systems, then their imaginary parts.
//
// Work split.  A workgroup owns a block of NS systems and a chunk of field
// points, walked in sub-tiles of 32 points.  Its W waves split the loop index
// k: wave w owns a range of at most 2 (up to 512 loops) or 4 steps of 32
// loops, keeps the currents of that range as matrix-core B operands in
// registers for the whole chunk, and accumulates r for that range over the
// chunk.  Per sub-tile:
//   1. each wave multiplies its loop range: a partial B (32 points x 2 NS),
//      A operands G[p][k] read straight from memory (8 consecutive k per lane);
//   2. the partials meet in LDS and every thread sums one or more (point,
//      system) entries over the waves in a fixed order, applies the loss
//      epilogue and stores w transposed in LDS (8 consecutive points per lane
//      make the adjoint's B operand);
//   3. each wave multiplies G^T for its loop range (A operands from the
//      transposed copy of G, 8 consecutive points per lane) by w.
// At the end each wave writes its rows of r per (chunk, system) in FP64 and the
// workgroup its per-system loss; the solves sum the chunks in a fixed order.
// No atomics: results are deterministic.
//
// Precisions (one MFMA "step" covers 32 consecutive k, or 32 points in the
// adjoint; lane group q = lane / 16 holds entries 8q..8q+7 of the step):
//   BF16X3  one 16x16x32 bf16 product per step on hi/lo splits of both
//           operands, three products hi hi + hi lo + lo hi into FP32;
//   FP32    eight 16x16x4 f32 products per step (product j takes entry j);
//   FP64    eight 16x16x4 f64 products per step.
// FP32 accumulation of r runs over at most kMfmaRowsF32 points per chunk (the
// sum over points cancels strongly), FP64 over any number.
//
// Workgroups are numbered so that the system blocks of one chunk of points run
// on one XCD side by side and share the chunk's rows of G in its L2.
#include <algorithm>

#include "epilogue.h"
#include "internal.h"

namespace cosim {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kSub = 32;    // points per sub-tile
constexpr int kMaxKs = 4;   // 32-loop steps per wave

// Two floats as packed bf16 (RNE) high parts and the packed low parts of
// their remainders: hi = bf16(x), lo = bf16(x - hi).
__device__ inline void split_pair(float a, float b, unsigned &hi, unsigned &lo) {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
    const float ha = __builtin_bit_cast(float, hi << 16);
    const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2));
}

// ---------------------------------------------------------------- precisions
struct PolBF3 {
    static constexpr int NC = 2;  // 16-column tiles: NS = 16 systems
    typedef float Acc;
    typedef f32x4 V;
    struct Op {
        bf16x8 h, l;
    };
    // C/D layout of the 16x16 accumulator: register m of lane group q holds row
    __device__ static constexpr int row(int q, int m) { return 4 * q + m; }
    __device__ static Op load(const void *hi, const void *lo, size_t off) {
        Op o;
        o.h = __builtin_bit_cast(bf16x8, *(const u32x4 *)((const uint16_t *)hi + off));
        o.l = __builtin_bit_cast(bf16x8, *(const u32x4 *)((const uint16_t *)lo + off));
        return o;
    }
    __device__ static Op make(const double (&v)[8]) {
        u32x4 h, l;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            unsigned hh, ll;
            split_pair((float)v[2 * j], (float)v[2 * j + 1], hh, ll);
            h[j] = hh;
            l[j] = ll;
        }
        return Op{__builtin_bit_cast(bf16x8, h), __builtin_bit_cast(bf16x8, l)};
    }
    __device__ static V mma(const Op &a, const Op &b, V c) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
    }
    // w in LDS, transposed: [column][point] hi and lo planes, rows padded
    static constexpr int LDW = kSub + 8;
    static constexpr int WBYTES = 2 * 16 * NC * LDW * 2;
    __device__ static void wstore(char *wb, int col, int row, float x) {
        uint16_t *h = (uint16_t *)wb, *l = h + 16 * NC * LDW;
        const __bf16 hb = (__bf16)x;
        h[col * LDW + row] = __builtin_bit_cast(uint16_t, hb);
        l[col * LDW + row] = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)hb));
    }
    __device__ static Op wload(const char *wb, int col, int q) {
        const uint16_t *h = (const uint16_t *)wb, *l = h + 16 * NC * LDW;
        Op o;
        o.h = __builtin_bit_cast(bf16x8, *(const u32x4 *)(h + col * LDW + 8 * q));
        o.l = __builtin_bit_cast(bf16x8, *(const u32x4 *)(l + col * LDW + 8 * q));
        return o;
    }
};

template <typename T>
struct PolScalar {
    static constexpr int NC = sizeof(T) == 4 ? 2 : 1;  // NS = 16 (FP32) or 8 (FP64) systems
    typedef T Acc;
    typedef T V __attribute__((ext_vector_type(4)));
    struct Op {
        T v[8];
    };
    // f32 16x16x4: rows 4q..4q+3 per lane group; f64 16x16x4: rows q, q+4, q+8, q+12
    __device__ static constexpr int row(int q, int m) { return sizeof(T) == 4 ? 4 * q + m : q + 4 * m; }
    __device__ static Op load(const void *g, const void *, size_t off) {
        Op o;
        const T *p = (const T *)g + off;
        if constexpr (sizeof(T) == 4) {
            const f32x4 a = *(const f32x4 *)p, b = *(const f32x4 *)(p + 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                o.v[j] = a[j];
                o.v[4 + j] = b[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double2 d = *(const double2 *)(p + 2 * j);
                o.v[2 * j] = d.x;
                o.v[2 * j + 1] = d.y;
            }
        }
        return o;
    }
    __device__ static Op make(const double (&v)[8]) {
        Op o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o.v[j] = (T)v[j];
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
    static constexpr int LDW = kSub + (sizeof(T) == 4 ? 4 : 2);
    static constexpr int WBYTES = 16 * NC * LDW * (int)sizeof(T);
    __device__ static void wstore(char *wb, int col, int row, T x) { ((T *)wb)[col * LDW + row] = x; }
    __device__ static Op wload(const char *wb, int col, int q) {
        return load((const T *)wb + col * LDW + 8 * q, nullptr, 0);
    }
};
typedef PolScalar<float> PolF32;
typedef PolScalar<double> PolF64;

template <class Pol>
constexpr int red_stride() {
    return 16 * Pol::NC + (sizeof(typename Pol::Acc) == 4 ? 4 : 2);
}

// Dynamic LDS of a workgroup of W waves.
template <class Pol>
constexpr size_t lds_bytes(int W) {
    const size_t red = (size_t)W * kSub * red_stride<Pol>() * sizeof(typename Pol::Acc);
    const size_t main = red + Pol::WBYTES;
    const size_t fin = (size_t)64 * W * sizeof(double);
    return main > fin ? main : fin;
}

// Loop steps per wave: two for up to 512 loops (more waves per workgroup, and
// registers left to load each phase's operands one phase ahead), four above.
__host__ __device__ constexpr int mfma_steps(int NP) { return NP <= 512 ? 2 : kMaxKs; }

// The work of workgroup b of a launch for one set of arguments, with at most
// KS loop steps per wave.  With KS = 2 (and operands of at most 32 bytes per
// lane) the operands of G^T for the adjoint are loaded at the start of the
// sub-tile and those of G for the next sub-tile after its forward product,
// so that their loads are in flight across the barriers and the epilogue.
template <class Pol, int MODE, int LOSS, int KS>
__device__ __forceinline__ void mfma_block(const MfmaArgs &a, int b) {
    typedef typename Pol::Acc Acc;
    typedef typename Pol::V V;
    typedef typename Pol::Op Op;
    constexpr int NC = Pol::NC, NS = 8 * NC;
    constexpr int RS = red_stride<Pol>();
    constexpr bool FWD = MODE != kMfmaVjp;
    constexpr bool ADJ = MODE == kMfmaLossGrad || MODE == kMfmaVjp;
    constexpr bool LOSSM = MODE == kMfmaLoss || MODE == kMfmaLossGrad;
    extern __shared__ __attribute__((aligned(16))) char smem[];

    const int W = (int)(blockDim.x >> 6);
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r16 = lane & 15, q = lane >> 4;
    // (chunk, system block) of this workgroup: with the grid a multiple of 8,
    // consecutive work items go to one XCD (workgroup b runs on XCD b % 8)
    const int N = a.nchunk * a.nsb;
    const int item = (N & 7) == 0 ? (b & 7) * (N >> 3) + (b >> 3) : b;
    const int chunk = item / a.nsb, sb = item - chunk * a.nsb;
    const int s0 = sb * NS;
    const int pb = chunk * a.rows_per_chunk;
    const int pe = min(a.P_pad, pb + a.rows_per_chunk);
    // this wave's loop steps [kb, kb + ks) of 32 loops
    const int m = a.NP >> 5;
    const int kb = (wave * m) / W, ks = ((wave + 1) * m) / W - kb;
    const int NP = a.NP;

    Acc *red = (Acc *)smem;
    char *wbuf = smem + (size_t)W * kSub * RS * sizeof(Acc);

    // currents of the block as forward B operands: column c of tile t is
    // system s0 + c % NS, real part for c < NS, imaginary part after
    Op X[KS][NC];
    if constexpr (FWD) {
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const int col = 16 * t + r16;
            const int s = s0 + col % NS;
            const bool im = col >= NS;
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                double v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * (kb + kk) + 8 * q + j;
                    double2 c = make_double2(0.0, 0.0);
                    if (kk < ks && s < a.S && k < a.n) c = a.I[(size_t)s * a.n + k];
                    v[j] = im ? c.y : c.x;
                }
                X[kk][t] = Pol::make(v);
            }
        }
    }
    V racc[2 * KS][NC];
    if constexpr (ADJ) {
#pragma unroll
        for (int i = 0; i < 2 * KS; ++i)
#pragma unroll
            for (int t = 0; t < NC; ++t) racc[i][t] = V{};
    }
    double lacc = 0.0;
    const int nthr = 64 * W;

    constexpr bool PF = KS <= 2 && sizeof(Op) <= 32;
    Op ga[KS][2], gt[2 * KS];  // operands loaded ahead (PF)
    auto load_g = [&](int p, int kk, int h) {
        return Pol::load(a.G, a.Glo, (size_t)(p + 16 * h + r16) * NP + 32 * (kb + kk) + 8 * q);
    };
    auto load_gt = [&](int p, int kt) {
        return Pol::load(a.GT, a.GTlo, (size_t)(32 * kb + 16 * kt + r16) * a.P_pad + p + 8 * q);
    };
    auto prefetch_g = [&](int p) {
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
            if (kk < ks)
#pragma unroll
                for (int h = 0; h < 2; ++h) ga[kk][h] = load_g(p, kk, h);
    };
    if constexpr (PF && FWD)
        if (pb < pe) prefetch_g(pb);

    for (int p0 = pb; p0 < pe; p0 += kSub) {
        if constexpr (PF && ADJ) {
#pragma unroll
            for (int kt = 0; kt < 2 * KS; ++kt)
                if (kt < 2 * ks) gt[kt] = load_gt(p0, kt);
        }
        // 1. partial B of this wave's loop range
        if constexpr (FWD) {
            V facc[2][NC];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int t = 0; t < NC; ++t) facc[h][t] = V{};
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                if (kk < ks) {  // uniform over the wave
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const Op A = PF ? ga[kk][h] : load_g(p0, kk, h);
#pragma unroll
                        for (int t = 0; t < NC; ++t) facc[h][t] = Pol::mma(A, X[kk][t], facc[h][t]);
                    }
                }
            }
            if constexpr (PF)
                if (p0 + kSub < pe) prefetch_g(p0 + kSub);
            Acc *rw = red + (size_t)wave * kSub * RS;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int t = 0; t < NC; ++t)
#pragma unroll
                    for (int mm = 0; mm < 4; ++mm)
                        rw[(16 * h + Pol::row(q, mm)) * RS + 16 * t + r16] = facc[h][t][mm];
        }
        __syncthreads();  // partials visible; every wave is done with the last w
        // 2. sums over the waves, in wave order, and what each mode does with B
        if constexpr (LOSSM) {
            // entry e = (point e / NS, system e % NS): a thread always meets the
            // same system (nthr is a multiple of NS), so its loss sum is one system's
            for (int e = tid; e < kSub * NS; e += nthr) {
                const int r = e / NS, sys = e - r * NS;
                const int p = p0 + r;
                Acc x = 0, y = 0;
                for (int w = 0; w < W; ++w) {
                    x += red[((size_t)w * kSub + r) * RS + sys];
                    y += red[((size_t)w * kSub + r) * RS + NS + sys];
                }
                // a padded point's field is the incident field alone: the target
                // |inc| makes its residual zero (inc = 0 outside the ratio mode)
                const Acc tg = p < a.P ? (Acc)a.T[p] : (Acc)fabs(a.inc);
                lacc += epilogue<LOSS>(x, y, tg, (Acc)a.inc);
                if constexpr (ADJ) {
                    Pol::wstore(wbuf, sys, r, x);
                    Pol::wstore(wbuf, NS + sys, r, y);
                }
            }
        } else if constexpr (MODE == kMfmaField) {
            // entry e = (system e / 32, point e % 32): consecutive threads write
            // consecutive points of one system
            for (int e = tid; e < kSub * NS; e += nthr) {
                const int sys = e / kSub, r = e - sys * kSub;
                const int p = p0 + r, s = s0 + sys;
                Acc x = 0, y = 0;
                for (int w = 0; w < W; ++w) {
                    x += red[((size_t)w * kSub + r) * RS + sys];
                    y += red[((size_t)w * kSub + r) * RS + NS + sys];
                }
                x += (Acc)a.inc;  // the incident field, when asked for (else 0)
                if (p < a.P && s < a.S) {
                    if constexpr (sizeof(Acc) == 8)
                        ((double2 *)a.Bout)[(size_t)s * a.P + p] = make_double2(x, y);
                    else
                        ((float2 *)a.Bout)[(size_t)s * a.P + p] = make_float2(x, y);
                }
            }
        } else {  // vector-Jacobian product: w is the upstream gradient
            for (int e = tid; e < kSub * NS; e += nthr) {
                const int sys = e / kSub, r = e - sys * kSub;
                const int p = p0 + r, s = s0 + sys;
                double2 g = make_double2(0.0, 0.0);
                if (p < a.P && s < a.S) g = a.gB[(size_t)s * a.P + p];
                Pol::wstore(wbuf, sys, r, (Acc)g.x);
                Pol::wstore(wbuf, NS + sys, r, (Acc)g.y);
            }
        }
        if constexpr (ADJ) {
            __syncthreads();  // w visible
            // 3. r += G^T w for this wave's loops: 16 loops per tile
#pragma unroll
            for (int kt = 0; kt < 2 * KS; ++kt) {
                if (kt < 2 * ks) {
                    const Op A = PF ? gt[kt] : load_gt(p0, kt);
#pragma unroll
                    for (int t = 0; t < NC; ++t)
                        racc[kt][t] = Pol::mma(A, Pol::wload(wbuf, 16 * t + r16, q), racc[kt][t]);
                }
            }
        } else {
            __syncthreads();  // every thread is done with the partials
        }
    }

    // per-system loss of the chunk: the threads of one system in thread order
    if constexpr (LOSSM) {
        __syncthreads();
        double *lred = (double *)smem;
        lred[tid] = lacc;
        __syncthreads();
        if (tid < NS) {
            double v = 0.0;
            for (int j = tid; j < nthr; j += NS) v += lred[j];
            const int s = s0 + tid;
            if (s < a.S) a.lpart[(size_t)chunk * a.S + s] = v;
        }
    }
    // r of this wave's loops: (real, imaginary) column pair of each system
    if constexpr (ADJ) {
#pragma unroll
        for (int kt = 0; kt < 2 * KS; ++kt) {
            if (kt < 2 * ks) {
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) {
                    const int k = 32 * kb + 16 * kt + Pol::row(q, mm);
                    double re, im;
                    int sys;
                    if constexpr (NC == 2) {
                        re = (double)racc[kt][0][mm];
                        im = (double)racc[kt][1][mm];
                        sys = r16;
                    } else {  // columns 0..7 real, 8..15 imaginary parts of 8 systems
                        re = (double)racc[kt][0][mm];
                        im = __shfl_down(re, 8, 16);
                        sys = r16 < 8 ? r16 : NS;  // NS: no store
                    }
                    const int s = s0 + sys;
                    if (sys < NS && s < a.S)
                        a.rpart[((size_t)chunk * a.S + s) * NP + k] = make_double2(re, im);
                }
            }
        }
    }
}

template <class Pol, int MODE, int LOSS, int KS>
__global__ __launch_bounds__(512) void k_mfma(MfmaArgs a) {
    mfma_block<Pol, MODE, LOSS, KS>(a, (int)blockIdx.x);
}

// Several plans of one padded loop count in one launch: member m owns the
// workgroups [first[m], first[m + 1]) (the last up to the launch's total);
// first[m] is a multiple of 8, so that the member's XCD-aware order holds,
// and the workgroups past its own count exit at once.
template <class Pol, int MODE, int LOSS, int KS>
__global__ __launch_bounds__(512) void k_mfma_group(MfmaGroup g) {
    const int b = (int)blockIdx.x;
    int m = 0;
    while (m + 1 < g.count && b >= g.first[m + 1]) ++m;
    const int loc = b - g.first[m];
    if (loc >= g.in[m].nchunk * g.in[m].nsb) return;
    mfma_block<Pol, MODE, LOSS, KS>(g.in[m], loc);
}

// (the members of a group share their padded loop count)
template <class Pol, int MODE, int LOSS>
hipError_t go_group(const MfmaGroup &g, int blocks, int W, hipStream_t st) {
    if (mfma_steps(g.in[0].NP) == 2)
        hipLaunchKernelGGL((k_mfma_group<Pol, MODE, LOSS, 2>), dim3((unsigned)blocks),
                           dim3(64 * W), lds_bytes<Pol>(W), st, g);
    else
        hipLaunchKernelGGL((k_mfma_group<Pol, MODE, LOSS, kMaxKs>), dim3((unsigned)blocks),
                           dim3(64 * W), lds_bytes<Pol>(W), st, g);
    return hipGetLastError();
}

template <class Pol, int MODE, int LOSS>
hipError_t go(const MfmaArgs &a, int W, hipStream_t st) {
    const size_t lds = lds_bytes<Pol>(W);
    const unsigned blocks = (unsigned)a.nchunk * (unsigned)a.nsb;
    if (mfma_steps(a.NP) == 2)
        hipLaunchKernelGGL((k_mfma<Pol, MODE, LOSS, 2>), dim3(blocks), dim3(64 * W), lds, st, a);
    else
        hipLaunchKernelGGL((k_mfma<Pol, MODE, LOSS, kMaxKs>), dim3(blocks), dim3(64 * W), lds, st,
                           a);
    return hipGetLastError();
}

template <class Pol, int MODE>
hipError_t go_loss(int loss_mode, const MfmaArgs &a, int W, hipStream_t st) {
    switch (loss_mode) {
        case COSIM_LOSS_MAG: return go<Pol, MODE, COSIM_LOSS_MAG>(a, W, st);
        case COSIM_LOSS_COMPLEX: return go<Pol, MODE, COSIM_LOSS_COMPLEX>(a, W, st);
        case COSIM_LOSS_RATIO: return go<Pol, MODE, COSIM_LOSS_RATIO>(a, W, st);
    }
    return hipErrorInvalidValue;
}

template <class Pol>
hipError_t go_mode(int mode, int loss_mode, const MfmaArgs &a, int W, hipStream_t st) {
    switch (mode) {
        case kMfmaLoss: return go_loss<Pol, kMfmaLoss>(loss_mode, a, W, st);
        case kMfmaLossGrad: return go_loss<Pol, kMfmaLossGrad>(loss_mode, a, W, st);
        case kMfmaField: return go<Pol, kMfmaField, 0>(a, W, st);
        case kMfmaVjp: return go<Pol, kMfmaVjp, 0>(a, W, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int mfma_systems_per_block(Prec prec) { return prec == Prec::F64 ? 8 : 16; }

MfmaShape mfma_shape(Prec prec, int NP, int S, int P_pad, int cus) {
    MfmaShape sh;
    const int m = NP / 32;
    const int ks = mfma_steps(NP);
    sh.waves = (m + ks - 1) / ks;
    const int ns = mfma_systems_per_block(prec);
    sh.nsb = (S + ns - 1) / ns;
    // fewest chunks of points (whole sub-tiles) that give the launch at least
    // two workgroups per compute unit, within the accumulation limit of the
    // precision and down to 256 points per chunk
    const int subs = P_pad / kSub;
    const int maxrows = prec == Prec::F64 ? P_pad : kMfmaRowsF32;
    int per = std::max(1, std::min(subs, maxrows / kSub));  // sub-tiles per chunk
    const long long want = 2LL * std::max(1, cus);
    while (per > 8 && (long long)((subs + per - 1) / per) * sh.nsb < want) per = (per + 1) / 2;
    sh.rows_per_chunk = per * kSub;
    sh.nchunk = (subs + per - 1) / per;
    return sh;
}

hipError_t launch_mfma_group(Prec prec, bool grad, int loss_mode, const MfmaGroup &g, int blocks,
                             int waves, hipStream_t st) {
    if (blocks <= 0 || g.count <= 0) return hipSuccess;
    if (g.count > kGroupMax || waves < 1 || waves > 8) return hipErrorInvalidValue;
    for (int m = 0; m < g.count; ++m) {
        const MfmaArgs &a = g.in[m];
        if (a.NP % 32 != 0 || a.NP / 32 > mfma_steps(a.NP) * waves || a.NP != g.in[0].NP ||
            a.P_pad % kSub != 0 ||
            a.rows_per_chunk % kSub != 0 || g.first[m] % 8 != 0 ||
            (m + 1 < g.count ? g.first[m + 1] : blocks) - g.first[m] < a.nchunk * a.nsb)
            return hipErrorInvalidValue;
    }
#define COSIM_MFMA_GROUP(POL)                                                                   \
    switch (loss_mode) {                                                                        \
        case COSIM_LOSS_MAG:                                                                    \
            return grad ? go_group<POL, kMfmaLossGrad, COSIM_LOSS_MAG>(g, blocks, waves, st)    \
                        : go_group<POL, kMfmaLoss, COSIM_LOSS_MAG>(g, blocks, waves, st);       \
        case COSIM_LOSS_COMPLEX:                                                                \
            return grad ? go_group<POL, kMfmaLossGrad, COSIM_LOSS_COMPLEX>(g, blocks, waves, st) \
                        : go_group<POL, kMfmaLoss, COSIM_LOSS_COMPLEX>(g, blocks, waves, st);   \
        case COSIM_LOSS_RATIO:                                                                  \
            return grad ? go_group<POL, kMfmaLossGrad, COSIM_LOSS_RATIO>(g, blocks, waves, st)  \
                        : go_group<POL, kMfmaLoss, COSIM_LOSS_RATIO>(g, blocks, waves, st);     \
    }                                                                                           \
    return hipErrorInvalidValue;
    switch (prec) {
        case Prec::BF16X3: COSIM_MFMA_GROUP(PolBF3)
        case Prec::F32: COSIM_MFMA_GROUP(PolF32)
        case Prec::F64: COSIM_MFMA_GROUP(PolF64)
    }
#undef COSIM_MFMA_GROUP
    return hipErrorInvalidValue;
}

hipError_t launch_mfma(Prec prec, int mode, int loss_mode, const MfmaArgs &a, int waves,
                       hipStream_t st) {
    if (a.NP % 32 != 0 || a.NP / 32 > mfma_steps(a.NP) * waves || waves < 1 || waves > 8 ||
        a.P_pad % kSub != 0 || a.rows_per_chunk % kSub != 0)
        return hipErrorInvalidValue;
    if (a.nchunk <= 0 || a.nsb <= 0) return hipSuccess;
    switch (prec) {
        case Prec::BF16X3: return go_mode<PolBF3>(mode, loss_mode, a, waves, st);
        case Prec::F32: return go_mode<PolF32>(mode, loss_mode, a, waves, st);
        case Prec::F64: return go_mode<PolF64>(mode, loss_mode, a, waves, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace cosim
