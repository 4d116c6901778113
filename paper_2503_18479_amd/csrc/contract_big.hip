// Superposition, loss and adjoint contraction for more than 64 loops
// (Eq. 7, Eq. 1, and the right-hand side of Eq. 8-10).
//
// With many loops the currents of a workgroup's systems no longer fit the
// matrix-core operand registers of the fused kernels, so the two contractions
// run as plain GEMMs on the library (rocBLAS) with the loss epilogue between:
//   X  [2S][NP]        re / im planes of I (packed, zero padded), column-major
//                      NP x 2S for the GEMM;
//   Y  = G X           P_pad x 2S planes of B_z (GEMM, K = NP);
//   epilogue           loss partials per (P-chunk, system) and the planes of
//                      w = dL/d conj(B) in the adjoint's operand precision;
//   R_c = G_c^T W_c    per P-chunk c of kBigRows rows (K = rows of the chunk),
//                      NP x 2S planes, summed over chunks in FP64 by the solve.
// BF16X3 splits both operands into bf16 hi / lo and adds the three products
// hi hi + hi lo + lo hi into FP32, each contraction as one GEMM: the forward
// over K = 3 NP ((hi | hi | lo) rows of G against (hi; lo; hi) planes of I),
// the adjoint per chunk over K = 3 rows (the chunk's hi, hi, lo rows of G
// against (hi; lo; hi) rows of w).  G is stored [P_pad][NP] row-major, i.e.
// column-major NP x P_pad, so the FP64 / FP32 GEMMs read it in place.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "epilogue.h"
#include "internal.h"

namespace cosim {

namespace {

__device__ inline uint16_t bf16_bits(float x) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ inline float bf16_float(uint16_t h) {
    return __builtin_bit_cast(float, ((uint32_t)h) << 16);
}

// X[(2s + c) NP + k] = (Re, Im)_c of I[s][k], 0 for k >= n.
// PREC 0: double planes; 1: float; 2: bf16 planes of 3 NP rows, each plane
// (hi; lo; hi) of its values (the operand of the one-GEMM forward product).
template <int PREC>
__global__ __launch_bounds__(256) void k_pack_x(int n, int NP, int S,
                                                const double2 *__restrict__ I, void *X) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)S * NP) return;
    const int s = (int)(e / NP), k = (int)(e - (size_t)s * NP);
    const double2 v = k < n ? I[(size_t)s * n + k] : make_double2(0.0, 0.0);
    const size_t o0 = (size_t)(2 * s) * NP + k, o1 = o0 + NP;
    if (PREC == 0) {
        ((double *)X)[o0] = v.x;
        ((double *)X)[o1] = v.y;
    } else if (PREC == 1) {
        ((float *)X)[o0] = (float)v.x;
        ((float *)X)[o1] = (float)v.y;
    } else {
        const float re = (float)v.x, im = (float)v.y;
        const uint16_t hr = bf16_bits(re), hi = bf16_bits(im);
        uint16_t *pr = (uint16_t *)X + (size_t)(2 * s) * 3 * NP + k;  // plane 2s
        uint16_t *pi = pr + 3 * NP;                                   // plane 2s + 1
        pr[0] = hr;
        pr[NP] = bf16_bits(re - bf16_float(hr));
        pr[2 * NP] = hr;
        pi[0] = hi;
        pi[NP] = bf16_bits(im - bf16_float(hi));
        pi[2 * NP] = hi;
    }
}

// grid (S, chunks): rows [c*rows, (c+1)*rows) of system s.  Loss partial in
// FP64, summed in a fixed order; w planes written when GRAD.
template <int PREC, int LOSS, bool GRAD>
__global__ __launch_bounds__(256) void k_epilogue_big(int P, int P_pad, int S, int rows,
                                                      const void *Y, const double *__restrict__ T,
                                                      void *W,
                                                      double *__restrict__ lpart, double inc) {
    __shared__ double red[4];
    const int s = blockIdx.x, c = blockIdx.y;
    const int p0 = c * rows, p1 = min(P_pad, p0 + rows);
    const size_t o0 = (size_t)(2 * s) * P_pad, o1 = o0 + P_pad;
    double acc = 0.0;
    for (int p = p0 + (int)threadIdx.x; p < p1; p += 256) {
        if (PREC == 0) {
            double x = ((const double *)Y)[o0 + p], y = ((const double *)Y)[o1 + p];
            const double t = p < P ? T[p] : fabs(inc);  // padded rows: residual 0
            acc += epilogue<LOSS>(x, y, t, inc);
            if (GRAD) {
                ((double *)W)[o0 + p] = x;
                ((double *)W)[o1 + p] = y;
            }
        } else {
            float x = ((const float *)Y)[o0 + p], y = ((const float *)Y)[o1 + p];
            const float t = p < P ? (float)T[p] : (float)fabs(inc);
            acc += (double)epilogue_f<LOSS>(x, y, t, (float)inc);
            if (GRAD) {
                if (PREC == 1) {
                    ((float *)W)[o0 + p] = x;
                    ((float *)W)[o1 + p] = y;
                } else {  // chunk c, planes 2s and 2s + 1: 3 rows (hi; lo; hi) each
                    const uint16_t hx = bf16_bits(x), hy = bf16_bits(y);
                    const size_t w0 = ((size_t)c * 2 * S + 2 * s) * 3 * rows + (p - p0);
                    const size_t w1 = w0 + (size_t)3 * rows;
                    uint16_t *Wb = (uint16_t *)W;
                    Wb[w0] = hx;
                    Wb[w0 + rows] = bf16_bits(x - bf16_float(hx));
                    Wb[w0 + 2 * rows] = hx;
                    Wb[w1] = hy;
                    Wb[w1 + rows] = bf16_bits(y - bf16_float(hy));
                    Wb[w1 + 2 * rows] = hy;
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) lpart[(size_t)c * S + s] = (red[0] + red[1]) + (red[2] + red[3]);
}

// W[(2s + c) P_pad + p] = (Re, Im)_c of g[s][p] (FP64), 0 for p >= P: the
// upstream gradient of the materialised field as adjoint GEMM operand.
__global__ __launch_bounds__(256) void k_pack_w64(int P, int P_pad, int S,
                                                  const double2 *__restrict__ g,
                                                  double *__restrict__ W) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)S * P_pad) return;
    const int s = (int)(e / P_pad), p = (int)(e - (size_t)s * P_pad);
    const double2 v = p < P ? g[(size_t)s * P + p] : make_double2(0.0, 0.0);
    W[(size_t)(2 * s) * P_pad + p] = v.x;
    W[(size_t)(2 * s + 1) * P_pad + p] = v.y;
}

hipError_t blas_status(rocblas_status r) {
    return r == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// C (m x n, ldc) = beta C + op(A) B, column-major, in the precision's types.
hipError_t gemm(rocblas_handle h, Prec prec, rocblas_operation ta, int m, int nn, int k,
                const void *A, int lda, const void *B, int ldb, float beta, void *C, int ldc) {
    if (prec == Prec::F64) {
        const double a1 = 1.0, b1 = beta;
        return blas_status(rocblas_gemm_ex(h, ta, rocblas_operation_none, m, nn, k, &a1, A,
                                           rocblas_datatype_f64_r, lda, B, rocblas_datatype_f64_r,
                                           ldb, &b1, C, rocblas_datatype_f64_r, ldc, C,
                                           rocblas_datatype_f64_r, ldc, rocblas_datatype_f64_r,
                                           rocblas_gemm_algo_standard, 0, 0));
    }
    const float a1 = 1.0f, b1 = beta;
    const rocblas_datatype t = prec == Prec::F32 ? rocblas_datatype_f32_r : rocblas_datatype_bf16_r;
    return blas_status(rocblas_gemm_ex(h, ta, rocblas_operation_none, m, nn, k, &a1, A, t, lda, B,
                                       t, ldb, &b1, C, rocblas_datatype_f32_r, ldc, C,
                                       rocblas_datatype_f32_r, ldc, rocblas_datatype_f32_r,
                                       rocblas_gemm_algo_standard, 0, 0));
}

template <int PREC, int LOSS>
hipError_t launch_epi(bool grad, dim3 grid, hipStream_t st, int P, int P_pad, int S, int rows,
                      const void *Y, const double *T, void *W, double *lpart,
                      double inc) {
    if (grad)
        hipLaunchKernelGGL((k_epilogue_big<PREC, LOSS, true>), grid, dim3(256), 0, st, P, P_pad, S,
                           rows, Y, T, W, lpart, inc);
    else
        hipLaunchKernelGGL((k_epilogue_big<PREC, LOSS, false>), grid, dim3(256), 0, st, P, P_pad,
                           S, rows, Y, T, W, lpart, inc);
    return hipGetLastError();
}

}  // namespace

hipError_t big_blas_create(void **handle) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return hipErrorOutOfMemory;
    *handle = h;
    return hipSuccess;
}

void big_blas_destroy(void *handle) {
    if (handle) (void)rocblas_destroy_handle((rocblas_handle)handle);
}

// Forward GEMM, loss epilogue and (if grad) the chunked adjoint GEMMs.
// R receives nchunk blocks of NP x 2S planes (double for F64, float otherwise).
hipError_t big_contract(void *handle, Prec prec, int loss_mode, bool grad, const BigArgs &a,
                        hipStream_t st) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidValue;
    const int S = a.S, NP = a.NP, P_pad = a.P_pad;
    const size_t planes = (size_t)2 * S;
    // 1. X planes
    const size_t nx = (size_t)S * NP;
    const dim3 gx((unsigned)((nx + 255) / 256));
    switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL(k_pack_x<0>, gx, dim3(256), 0, st, a.n, NP, S, a.I, a.X);
            break;
        case Prec::F32:
            hipLaunchKernelGGL(k_pack_x<1>, gx, dim3(256), 0, st, a.n, NP, S, a.I, a.X);
            break;
        case Prec::BF16X3:
            hipLaunchKernelGGL(k_pack_x<2>, gx, dim3(256), 0, st, a.n, NP, S, a.I, a.X);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 2. Y = G X
    const rocblas_operation T_ = rocblas_operation_transpose;
    if (prec == Prec::BF16X3) {
        // (hi | hi | lo) rows of G times (hi; lo; hi) planes of I: Gh Ih + Gh Il + Gl Ih
        if ((e = gemm(h, prec, T_, P_pad, (int)planes, 3 * NP, a.G3, 3 * NP, a.X, 3 * NP, 0.0f,
                      a.Y, P_pad)))
            return e;
    } else {
        if ((e = gemm(h, prec, T_, P_pad, (int)planes, NP, a.G, NP, a.X, NP, 0.0f, a.Y, P_pad)))
            return e;
    }
    // 3. loss partials and w planes
    const dim3 ge(S, a.nchunk);
    const int pr = prec == Prec::F64 ? 0 : (prec == Prec::F32 ? 1 : 2);
#define COSIM_EPI(PR)                                                                          \
    (loss_mode == COSIM_LOSS_MAG                                                               \
         ? launch_epi<PR, COSIM_LOSS_MAG>(grad, ge, st, a.P, P_pad, S, a.rows, a.Y, a.T, a.W,  \
                                          a.lpart, a.inc)                                  \
     : loss_mode == COSIM_LOSS_RATIO                                                           \
         ? launch_epi<PR, COSIM_LOSS_RATIO>(grad, ge, st, a.P, P_pad, S, a.rows, a.Y, a.T,     \
                                            a.W, a.lpart, a.inc)                           \
         : launch_epi<PR, COSIM_LOSS_COMPLEX>(grad, ge, st, a.P, P_pad, S, a.rows, a.Y, a.T,   \
                                              a.W, a.lpart, a.inc))
    e = pr == 0 ? COSIM_EPI(0) : (pr == 1 ? COSIM_EPI(1) : COSIM_EPI(2));
#undef COSIM_EPI
    if (e != hipSuccess || !grad) return e;
    // 4. R_c = G_c^T W_c per chunk of rows
    return big_adjoint(handle, prec, a, st);
}

// One adjoint product over `nb` consecutive chunks of `rows` rows starting at
// row p0: C_c = A_c B_c for c < nb, with A_c = G rows [p0 + c rows, ...) (NP x
// rows, column-major), B_c the same rows of W (rows x 2S, ld P_pad), C_c the
// chunk's NP x 2S block of R; one strided-batched call.
hipError_t gemm_chunks(rocblas_handle h, Prec prec, int NP, int planes, int rows, int nb, int P_pad,
                       const char *A, size_t a_esz, const char *B, size_t b_esz, float beta, char *C,
                       size_t c_esz) {
    const rocblas_operation N_ = rocblas_operation_none;
    const rocblas_stride sa = (rocblas_stride)rows * NP, sb = rows, sc = (rocblas_stride)NP * planes;
    (void)a_esz;
    (void)b_esz;
    (void)c_esz;
    if (prec == Prec::F64) {
        const double a1 = 1.0, b1 = beta;
        return blas_status(rocblas_gemm_strided_batched_ex(
            h, N_, N_, NP, planes, rows, &a1, A, rocblas_datatype_f64_r, NP, sa, B,
            rocblas_datatype_f64_r, P_pad, sb, &b1, C, rocblas_datatype_f64_r, NP, sc, C,
            rocblas_datatype_f64_r, NP, sc, nb, rocblas_datatype_f64_r, rocblas_gemm_algo_standard,
            0, 0));
    }
    const float a1 = 1.0f, b1 = beta;
    const rocblas_datatype t = prec == Prec::F32 ? rocblas_datatype_f32_r : rocblas_datatype_bf16_r;
    return blas_status(rocblas_gemm_strided_batched_ex(
        h, N_, N_, NP, planes, rows, &a1, A, t, NP, sa, B, t, P_pad, sb, &b1, C,
        rocblas_datatype_f32_r, NP, sc, C, rocblas_datatype_f32_r, NP, sc, nb,
        rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0));
}

// Adjoint GEMMs only (W already holds the planes of w): the full chunks in one
// strided-batched call, a shorter last chunk in another.  BF16X3: the three
// products of a chunk are one GEMM over K = 3 rows ((hi, hi, lo) rows of G in
// GA3 against the (hi; lo; hi) w rows the epilogue wrote), whole chunks only.
hipError_t big_adjoint(void *handle, Prec prec, const BigArgs &a, hipStream_t st) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidValue;
    const int S = a.S, NP = a.NP, P_pad = a.P_pad;
    const int planes = 2 * S;
    const size_t esz = prec == Prec::F64 ? sizeof(double) : sizeof(float);
    const size_t gsz = prec == Prec::F64 ? sizeof(double) : sizeof(float);
    const int full = P_pad / a.rows;                   // whole chunks
    const int tail = P_pad - full * a.rows;            // rows of a last, shorter chunk
    if (prec == Prec::BF16X3) {
        if (tail != 0 || !a.GA3) return hipErrorInvalidValue;  // P_pad is whole chunks here
        const int K = 3 * a.rows;
        const float one = 1.0f, zero = 0.0f;
        const rocblas_operation N_ = rocblas_operation_none;
        return blas_status(rocblas_gemm_strided_batched_ex(
            h, N_, N_, NP, planes, K, &one, a.GA3, rocblas_datatype_bf16_r, NP,
            (rocblas_stride)K * NP, a.W, rocblas_datatype_bf16_r, K, (rocblas_stride)K * planes,
            &zero, a.R, rocblas_datatype_f32_r, NP, (rocblas_stride)NP * planes, a.R,
            rocblas_datatype_f32_r, NP, (rocblas_stride)NP * planes, full, rocblas_datatype_f32_r,
            rocblas_gemm_algo_standard, 0, 0));
    }
    hipError_t e = hipSuccess;
    for (int part = 0; part < 2; ++part) {
        const int nb = part == 0 ? full : (tail > 0 ? 1 : 0);
        const int rows = part == 0 ? a.rows : tail;
        if (nb == 0) continue;
        const size_t p0 = part == 0 ? 0 : (size_t)full * a.rows;
        char *R = (char *)a.R + (part == 0 ? 0 : (size_t)full * NP * planes * esz);
        const char *g = (const char *)a.G + p0 * NP * gsz;
        const char *w = (const char *)a.W + p0 * gsz;
        if ((e = gemm_chunks(h, prec, NP, planes, rows, nb, P_pad, g, gsz, w, gsz, 0.0f, R, esz))) return e;
    }
    return e;
}

hipError_t launch_pack_w64(int P, int P_pad, int S, const double2 *g_d, double *W_d,
                           hipStream_t st) {
    const size_t ne = (size_t)S * P_pad;
    hipLaunchKernelGGL(k_pack_w64, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, P, P_pad,
                       S, g_d, W_d);
    return hipGetLastError();
}

}  // namespace cosim
