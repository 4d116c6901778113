// Adam update of the tunable capacitances: the optimiser the paper runs on C
// (Sec. IV), with the bias-corrected moment estimates of Kingma & Ba (2015).
// The step count lives in device memory so that one captured graph of
// [cosim_loss_and_grad, cosim_adam_step] replays any number of steps.
#include "internal.h"

namespace cosim {

namespace {

// t = *step + 1 for every element; the counter itself is advanced by
// k_adam_count, the next launch on the same stream.
__global__ __launch_bounds__(256) void k_adam(int count, double *__restrict__ C,
                                              const double *__restrict__ g,
                                              double *__restrict__ m, double *__restrict__ v,
                                              const int32_t *__restrict__ step, double lr,
                                              double b1, double b2, double eps) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const double t = (double)(step[0] + 1);
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    C[i] -= (lr / c1) * mi / (sqrt(vi) / sqrt(c2) + eps);
}

__global__ void k_adam_count(int32_t *step) {
    if (threadIdx.x == 0) step[0] = step[0] + 1;
}

}  // namespace

hipError_t launch_adam(int count, double *C_d, const double *grad_d, double *m_d, double *v_d,
                       int32_t *step_d, double lr, double beta1, double beta2, double eps,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, st, count, C_d, grad_d,
                       m_d, v_d, step_d, lr, beta1, beta2, eps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adam_count, dim3(1), dim3(64), 0, st, step_d);
    return hipGetLastError();
}

}  // namespace cosim
