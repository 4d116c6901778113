// Materialised superposition B_z = G I (Eq. 7) and the FP64 contraction
// G^T conj(g) used by the vector-Jacobian product.  These serve the autograd
// path (B_z handed to an arbitrary user loss); the optimisation step itself
// uses the fused kernels, which never write B_z.
#include "internal.h"

namespace cosim {

namespace {

__device__ inline uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline float bf16_round(float x) { return bf16_val(bf16_bits(x)); }

// grid (ceil(P/256), S): thread = point, I of system s staged in LDS.
template <int PREC>
__global__ __launch_bounds__(256) void k_field(int NP, int P, int S, int n,
                                               const double *__restrict__ G64,
                                               const double2 *__restrict__ I,
                                               void *__restrict__ Bz) {
    __shared__ double2 sI[kMaxLoopsBig];
    const int s = blockIdx.y;
    for (int k = threadIdx.x; k < n; k += blockDim.x) sI[k] = I[(size_t)s * n + k];
    __syncthreads();
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const double *g = G64 + (size_t)p * NP;
    if (PREC == 0) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < n; ++k) {
            re += g[k] * sI[k].x;
            im += g[k] * sI[k].y;
        }
        ((double2 *)Bz)[(size_t)s * P + p] = make_double2(re, im);
    } else if (PREC == 1) {
        float re = 0.f, im = 0.f;
        for (int k = 0; k < n; ++k) {
            const float gk = (float)g[k];
            re += gk * (float)sI[k].x;
            im += gk * (float)sI[k].y;
        }
        ((float2 *)Bz)[(size_t)s * P + p] = make_float2(re, im);
    } else {
        float re = 0.f, im = 0.f;
        for (int k = 0; k < n; ++k) {
            const float g32 = (float)g[k];
            const float gh = bf16_round(g32), gl = bf16_round(g32 - gh);
            const float xr = (float)sI[k].x, xi = (float)sI[k].y;
            const float rh = bf16_round(xr), rl = bf16_round(xr - rh);
            const float ih = bf16_round(xi), il = bf16_round(xi - ih);
            re += gl * rh + gh * rl + gh * rh;
            im += gl * ih + gh * il + gh * ih;
        }
        ((float2 *)Bz)[(size_t)s * P + p] = make_float2(re, im);
    }
}

// Block per system: thread t handles loop i = t % NP over the points
// p = t / NP, t / NP + 256 / NP, ...; the groups are summed in fixed order.
__global__ __launch_bounds__(256) void k_backward_contract(int NP, int P, int S, int n,
                                                           const double *__restrict__ G64,
                                                           const double2 *__restrict__ g,
                                                           double2 *__restrict__ rpart) {
    __shared__ double2 red[256];
    const int s = blockIdx.x;
    const int i = threadIdx.x % NP, grp = threadIdx.x / NP, ngrp = 256 / NP;
    double rr = 0.0, ri = 0.0;
    for (int p = grp; p < P; p += ngrp) {
        const double gi = G64[(size_t)p * NP + i];
        const double2 v = g[(size_t)s * P + p];
        rr += gi * v.x;
        ri += gi * v.y;
    }
    red[threadIdx.x] = make_double2(rr, ri);
    __syncthreads();
    if (threadIdx.x < NP) {
        double2 acc = make_double2(0.0, 0.0);
        for (int c = 0; c < ngrp; ++c) {
            acc.x += red[c * NP + threadIdx.x].x;
            acc.y += red[c * NP + threadIdx.x].y;
        }
        rpart[(size_t)s * NP + threadIdx.x] = acc;
    }
}

}  // namespace

hipError_t launch_field(Prec prec, int NP, int P, int S, int n, const double *G64,
                        const double2 *I_d, void *Bz_d, hipStream_t st) {
    dim3 grid((P + 255) / 256, S);
    switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL(k_field<0>, grid, dim3(256), 0, st, NP, P, S, n, G64, I_d, Bz_d);
            break;
        case Prec::F32:
            hipLaunchKernelGGL(k_field<1>, grid, dim3(256), 0, st, NP, P, S, n, G64, I_d, Bz_d);
            break;
        case Prec::BF16X3:
            hipLaunchKernelGGL(k_field<2>, grid, dim3(256), 0, st, NP, P, S, n, G64, I_d, Bz_d);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_field_backward_contract(int NP, int P, int S, int n, const double *G64,
                                          const double2 *gBz_d, double2 *rpart_d,
                                          hipStream_t st) {
    (void)n;
    hipLaunchKernelGGL(k_backward_contract, dim3(S), dim3(256), 0, st, NP, P, S, n, G64, gBz_d,
                       rpart_d);
    return hipGetLastError();
}

}  // namespace cosim
