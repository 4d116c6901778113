// The other circuit variables of the cosimulation (Fig. 2: R, L, C, w) and the
// helpers of the optimisation around C (Sec. IV-A, Sec. V):
//   k_param_sys    per system, from the currents I and the adjoint solution mu
//                  (Z mu = G^T conj(w); Z is complex symmetric, so
//                  dL = 2 Re(mu^T (dV - dZ I)) with V = E - j w Phi, E the
//                  source EMF of driven ports, independent of w):
//                    dL/dR_k = -2 Re(mu_k I_k)          (dZ = e_k e_k^T),
//                    dL/dL_k =  2 w Im(mu_k I_k)        (a series inductance
//                                                        added to loop k: dZ = j w e_k e_k^T),
//                    dL/dw   =  2 [Im(mu^T Phi) + Im(mu^T M I)
//                                  + sum_k Im(mu_k I_k) / (w^2 C_k)]
//                                                       (dZ = j M - diag(1/(j w^2 C)),
//                                                        dV = -j Phi);
//   k_param_reduce  fixed-order sums of the R and L terms over frequencies;
//   k_resonant_c    the resonance capacitance of Eq. 13, C_r = 1 / (w^2 (L + M));
//   k_tanh_project  the bounded projection C = cmin + (cmax - cmin)(1 + tanh t)/2
//                   and its derivative; k_clip clamps to a range.
#include "internal.h"

namespace cosim {

namespace {

// one 64-thread block per system s = b F + f
__global__ __launch_bounds__(64) void k_param_sys(int n, int S, int F, const double2 *__restrict__ I,
                                                  const double2 *__restrict__ mu,
                                                  const double *__restrict__ C,
                                                  const double *__restrict__ omega,
                                                  const double *__restrict__ phi,
                                                  const double *__restrict__ M,
                                                  double *__restrict__ gRs, double *__restrict__ gLs,
                                                  double *__restrict__ gw) {
    const int s = blockIdx.x, lane = threadIdx.x;
    const int b = s / F, f = s - b * F;
    const double w = omega[f];
    const double2 *Is = I + (size_t)s * n;
    const double2 *ms = mu + (size_t)s * n;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) {
        const double2 m = ms[k], i = Is[k];
        const double pr = m.x * i.x - m.y * i.y, pi = m.x * i.y + m.y * i.x;  // mu_k I_k
        gRs[(size_t)s * n + k] = -2.0 * pr;
        gLs[(size_t)s * n + k] = 2.0 * w * pi;
        // (M I)_k = sum_l M[l][k] I_l (M symmetric: lanes read consecutive k)
        double ar = 0.0, ai = 0.0;
#pragma unroll 8
        for (int l = 0; l < n; ++l) {
            const double mlk = M[(size_t)l * n + k];
            const double2 il = Is[l];
            ar = fma(mlk, il.x, ar);
            ai = fma(mlk, il.y, ai);
        }
        ar += phi[k];
        // Im(mu_k (Phi_k + (M I)_k)) + Im(mu_k I_k) / (w^2 C_k)
        acc += m.x * ai + m.y * ar + pi / (w * w * C[(size_t)b * n + k]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) gw[s] = 2.0 * acc;
}

// gR[b][k] = sum over f of gRs[b F + f][k]; gL likewise
__global__ void k_param_reduce(int n, int B, int F, const double *__restrict__ gRs,
                               const double *__restrict__ gLs, double *__restrict__ gR,
                               double *__restrict__ gL) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)B * n) return;
    const int k = (int)(t % n), b = (int)(t / n);
    double r = 0.0, l = 0.0;
    for (int f = 0; f < F; ++f) {
        const size_t o = ((size_t)b * F + f) * n + k;
        r += gRs[o];
        l += gLs[o];
    }
    if (gR) gR[t] = r;
    if (gL) gL[t] = l;
}

// Cr[f][k] = 1 / (w_f^2 L_k), L_k = M_kk or sum_l M_kl
__global__ void k_resonant_c(int n, int F, const double *__restrict__ M,
                             const double *__restrict__ omega, int coupled,
                             double *__restrict__ Cr) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)F * n) return;
    const int k = (int)(t % n), f = (int)(t / n);
    double L = M[(size_t)k * n + k];
    if (coupled) {
        L = 0.0;
        for (int l = 0; l < n; ++l) L += M[(size_t)k * n + l];
    }
    const double w = omega[f];
    Cr[t] = 1.0 / (w * w * L);
}

__global__ void k_tanh_project(size_t count, const double *__restrict__ theta, double cmin,
                               double cmax, double *__restrict__ C, double *__restrict__ dC) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double h = tanh(theta[t]);
    C[t] = cmin + 0.5 * (cmax - cmin) * (1.0 + h);
    if (dC) dC[t] = 0.5 * (cmax - cmin) * (1.0 - h * h);
}

__global__ void k_clip(size_t count, double *__restrict__ x, double lo, double hi) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    x[t] = fmin(fmax(x[t], lo), hi);
}

__global__ void k_scale(size_t count, double a, const double *__restrict__ x,
                        double *__restrict__ y) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) y[t] = a * x[t];
}

unsigned blocks(size_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

hipError_t launch_param_grads(int n, int B, int F, const double2 *I, const double2 *mu,
                              const double *C, const double *omega, const double *phi,
                              const double *M, double *gRs, double *gLs, double *gR, double *gL,
                              double *gw, hipStream_t st) {
    const int S = B * F;
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_param_sys, dim3(S), dim3(64), 0, st, n, S, F, I, mu, C, omega, phi, M,
                       gRs, gLs, gw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || (!gR && !gL)) return e;
    hipLaunchKernelGGL(k_param_reduce, dim3(blocks((size_t)B * n)), dim3(256), 0, st, n, B, F, gRs,
                       gLs, gR, gL);
    return hipGetLastError();
}

hipError_t launch_resonant_c(int n, int F, const double *M, const double *omega, int coupled,
                             double *Cr, hipStream_t st) {
    const size_t t = (size_t)F * n;
    if (t == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resonant_c, dim3(blocks(t)), dim3(256), 0, st, n, F, M, omega, coupled, Cr);
    return hipGetLastError();
}

hipError_t launch_tanh_project(size_t count, const double *theta, double cmin, double cmax,
                               double *C, double *dC, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tanh_project, dim3(blocks(count)), dim3(256), 0, st, count, theta, cmin,
                       cmax, C, dC);
    return hipGetLastError();
}

hipError_t launch_clip(size_t count, double *x, double lo, double hi, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clip, dim3(blocks(count)), dim3(256), 0, st, count, x, lo, hi);
    return hipGetLastError();
}

hipError_t launch_scale(size_t count, double a, const double *x, double *y, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(blocks(count)), dim3(256), 0, st, count, a, x, y);
    return hipGetLastError();
}

}  // namespace cosim
