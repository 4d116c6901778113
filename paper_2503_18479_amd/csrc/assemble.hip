// One-time operator assembly on gfx950: the Biot-Savart field matrix G and
// the Neumann inductance matrix M.  Both are plain-ALU kernels (FP64 sqrt,
// division and asinh dominate); they run once per geometry and point set.
#include "internal.h"

namespace cosim {

namespace {

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ inline uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Cartesian component `comp` (0 x, 1 y, 2 z) of the field per ampere of the
// straight filament v1 -> v2 at point p.  With a = v1 - p, b = v2 - p:
//   mu0/(4pi) (a x b)_comp (|a|+|b|) / (|a||b| (|a||b| + a.b)).
// For a.b < 0 the last factor is evaluated as (|a||b| - a.b)/|a x b|^2, its
// equal that does not cancel beside the filament.
__device__ inline double b_filament(int comp, double ax, double ay, double az, double la,
                                    double bx, double by, double bz, double lb) {
    double cx = ay * bz - az * by;
    double cy = az * bx - ax * bz;
    double cz = ax * by - ay * bx;
    double dot = ax * bx + ay * by + az * bz;
    double ab = la * lb;
    double inv;
    if (dot >= 0.0) {
        inv = 1.0 / (ab + dot);
    } else {
        inv = (ab - dot) / (cx * cx + cy * cy + cz * cz);
    }
    const double cc = comp == 2 ? cz : comp == 1 ? cy : cx;
    return cc * (la + lb) * inv / ab;
}

// Block: 64 points x 4 waves.  Wave w evaluates loops w, w+4, ... for the 64
// points of its lanes (every lane of a wave walks the same vertices, so each
// vertex load is one cache line for the whole wave), one chunk of 64 loops at a time; each chunk of
// the block tile [64][64] is staged in LDS and written out row-major, so that
// a row segment of G is one contiguous store, and transposed, so that a
// column segment of each transposed copy is one too.  Copies the plan did not
// ask for are null and skipped.
constexpr int kGPts = 64;
constexpr int kGLoops = 64;

__global__ __launch_bounds__(256) void k_assemble_G(int n, int NP, int P, int P_pad, int comp,
                                                    const int32_t *__restrict__ seg_off,
                                                    const double *__restrict__ verts,
                                                    const double *__restrict__ pts,
                                                    double *__restrict__ G64,
                                                    float *__restrict__ G32,
                                                    uint16_t *__restrict__ Ghi,
                                                    uint16_t *__restrict__ Glo,
                                                    double *__restrict__ GT64,
                                                    float *__restrict__ GT32,
                                                    uint16_t *__restrict__ GThi,
                                                    uint16_t *__restrict__ GTlo) {
    __shared__ double tile[kGPts][kGLoops + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int p = blockIdx.x * kGPts + lane;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (p < P) {
        px = pts[3 * p + 0];
        py = pts[3 * p + 1];
        pz = pts[3 * p + 2];
    }
    const int prow0 = blockIdx.x * kGPts;
    for (int k0 = 0; k0 < NP; k0 += kGLoops) {
        const int kc = min(kGLoops, NP - k0);
        for (int kk = wave; kk < kc; kk += 4) {
            const int k = k0 + kk;
            double acc = 0.0;
            if (k < n && p < P) {
                const int v0 = seg_off[k], v1 = seg_off[k + 1];
                // first vertex relative to p; distances are shared by neighbouring segments
                double fx = verts[3 * v0 + 0] - px, fy = verts[3 * v0 + 1] - py,
                       fz = verts[3 * v0 + 2] - pz;
                double fl = sqrt(fx * fx + fy * fy + fz * fz);
                double ax = fx, ay = fy, az = fz, la = fl;
                for (int v = v0 + 1; v <= v1; ++v) {
                    double bx, by, bz, lb;
                    if (v < v1) {
                        bx = verts[3 * v + 0] - px;
                        by = verts[3 * v + 1] - py;
                        bz = verts[3 * v + 2] - pz;
                        lb = sqrt(bx * bx + by * by + bz * bz);
                    } else {  // closing segment back to the first vertex
                        bx = fx; by = fy; bz = fz; lb = fl;
                    }
                    acc += b_filament(comp, ax, ay, az, la, bx, by, bz, lb);
                    ax = bx; ay = by; az = bz; la = lb;
                }
                acc *= kMu0Over4Pi;
            }
            tile[lane][kk] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kGPts * kc; e += 256) {
            const int r = e / kc, kk = e - r * kc;
            const int pr = prow0 + r;
            if (pr >= P_pad) continue;
            const double g = tile[r][kk];
            const size_t o = (size_t)pr * NP + k0 + kk;
            const float g32 = (float)g;
            if (G64) G64[o] = g;  // copies the plan did not ask for are null
            if (G32) G32[o] = g32;
            if (Ghi) {
                const uint16_t hi = bf16_rne(g32);
                Ghi[o] = hi;
                Glo[o] = bf16_rne(g32 - bf16_to_f(hi));
            }
        }
        // transposed copies [NP][P_pad]: each loop's column is contiguous in p
        if (GT64 || GT32 || GThi) {
            for (int e = threadIdx.x; e < kGPts * kc; e += 256) {
                const int kk = e / kGPts, r = e - kk * kGPts;
                const int pr = prow0 + r;
                if (pr >= P_pad) continue;
                const double g = tile[r][kk];
                const float g32 = (float)g;
                const size_t o = (size_t)(k0 + kk) * P_pad + pr;
                if (GT64) GT64[o] = g;
                if (GT32) GT32[o] = g32;
                if (GThi) {
                    const uint16_t hi = bf16_rne(g32);
                    GThi[o] = hi;
                    GTlo[o] = bf16_rne(g32 - bf16_to_f(hi));
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Neumann mutual inductance of two straight filaments x1->x2, y1->y2 with the
// kernel 1/sqrt(|r - r'|^2 + a^2):
//   parallel:      Grover's closed form, four corner terms of
//                  F(u) = u asinh(u/d) - sqrt(u^2 + d^2); for d = 0 (collinear)
//                  F(u) = |u| ln|u| (the terms linear in |u| cancel);
//   perpendicular: exactly zero;
//   otherwise:     inner integral along y in closed form
//                  asinh((L2 - t0)/r) + asinh(t0/r), outer integral along x by
//                  composite Gauss-Legendre with panels scaled to the closest
//                  approach of the two filaments.
// ----------------------------------------------------------------------------
struct V3 {
    double x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline double dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }

__device__ inline double cornerF(double u, double d) {
    if (d > 0.0) return u * asinh(u / d) - sqrt(u * u + d * d);
    double au = fabs(u);
    return au > 0.0 ? au * log(au) : 0.0;
}

// distance from point c to the segment p0 + t*e, t in [0, L] (e unit)
__device__ inline double point_seg_dist(V3 c, V3 p0, V3 e, double L) {
    V3 w = sub(c, p0);
    double t = fmin(fmax(dot3(w, e), 0.0), L);
    V3 d = sub(w, scl(e, t));
    return sqrt(dot3(d, d));
}

__device__ double neumann_pair(V3 x1, V3 x2, V3 y1, V3 y2, double a, const GLRule &gl) {
    V3 du = sub(x2, x1), dv = sub(y2, y1);
    const double L1 = sqrt(dot3(du, du)), L2 = sqrt(dot3(dv, dv));
    const V3 u = scl(du, 1.0 / L1), v = scl(dv, 1.0 / L2);
    const double c = dot3(u, v);
    const V3 cr = {u.y * v.z - u.z * v.y, u.z * v.x - u.x * v.z, u.x * v.y - u.y * v.x};
    const double s2 = dot3(cr, cr);
    if (s2 < 1e-24) {
        const double sgn = c > 0.0 ? 1.0 : -1.0;
        const V3 w = sub(y1, x1);
        const double along = dot3(w, u);
        const V3 perp = sub(w, scl(u, along));
        double d = sqrt(dot3(perp, perp) + a * a);
        if (d < 1e-12 * fmax(L1, L2)) d = 0.0;
        const double b1 = along, b2 = along + sgn * L2;
        const double lo = fmin(b1, b2), hi = fmax(b1, b2);
        const double val = cornerF(L1 - lo, d) - cornerF(L1 - hi, d) - cornerF(-lo, d) +
                           cornerF(-hi, d);
        return kMu0Over4Pi * sgn * val;
    }
    if (fabs(c) < 1e-12) return 0.0;
    // closest approach (endpoint-to-segment distances bound it for separated
    // filaments) sets the panel count so that each panel spans ~1/4 of it
    double dmin = fmin(fmin(point_seg_dist(x1, y1, v, L2), point_seg_dist(x2, y1, v, L2)),
                       fmin(point_seg_dist(y1, x1, u, L1), point_seg_dist(y2, x1, u, L1)));
    const double reff = sqrt(dmin * dmin + a * a);
    int npan = 4;
    if (reff > 0.0) {
        const double want = ceil(4.0 * L1 / reff);
        npan = (int)fmin(fmax(want, 4.0), 64.0);
    } else {
        npan = 64;
    }
    const double h = L1 / npan;
    double acc = 0.0;
    for (int j = 0; j < npan; ++j) {
        const double mid = (j + 0.5) * h;
        for (int q = 0; q < kGLOrder; ++q) {
            const double s = mid + 0.5 * h * gl.x[q];
            const V3 x = add(x1, scl(u, s));
            const V3 w = sub(x, y1);
            const double t0 = dot3(w, v);
            const double rho2 = fmax(dot3(w, w) - t0 * t0, 0.0);
            double r = sqrt(rho2 + a * a);
            if (r == 0.0) r = 1e-300;
            acc += 0.5 * h * gl.w[q] * (asinh((L2 - t0) / r) + asinh(t0 / r));
        }
    }
    return kMu0Over4Pi * c * acc;
}

// One block per unordered loop pair (k <= l); threads stride over the
// segment pairs, then a fixed-order tree reduction (deterministic).
__global__ __launch_bounds__(256) void k_assemble_M(int n, const int32_t *__restrict__ seg_off,
                                                    const double *__restrict__ verts,
                                                    const double *__restrict__ wire_a, GLRule gl,
                                                    double *__restrict__ M) {
    __shared__ double red[256];
    // linear pair index -> (k, l), k <= l, row-major over the upper triangle
    const long long idx = blockIdx.x;
    int k = 0;
    long long rem = idx;
    while (rem >= n - k) {
        rem -= n - k;
        ++k;
    }
    const int l = k + (int)rem;
    const int ka = seg_off[k], kn = seg_off[k + 1] - ka;
    const int la = seg_off[l], ln = seg_off[l + 1] - la;
    const double a = (k == l) ? wire_a[k] : 0.0;
    double acc = 0.0;
    for (int e = threadIdx.x; e < kn * ln; e += blockDim.x) {
        const int s = e / ln, t = e - s * ln;
        const int s2 = (s + 1 == kn) ? 0 : s + 1;
        const int t2 = (t + 1 == ln) ? 0 : t + 1;
        const double *p = verts + 3 * (size_t)(ka + s);
        const double *p2 = verts + 3 * (size_t)(ka + s2);
        const double *q = verts + 3 * (size_t)(la + t);
        const double *q2 = verts + 3 * (size_t)(la + t2);
        acc += neumann_pair({p[0], p[1], p[2]}, {p2[0], p2[1], p2[2]}, {q[0], q[1], q[2]},
                            {q2[0], q2[1], q2[2]}, a, gl);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        M[(size_t)k * n + l] = red[0];
        M[(size_t)l * n + k] = red[0];
    }
}

}  // namespace

hipError_t launch_assemble_G(int n, int NP, int P, int P_pad, int comp, const int32_t *seg_off_d,
                             const double *verts_d, const double *pts_d, double *G64,
                             float *G32, uint16_t *Ghi, uint16_t *Glo, double *GT64,
                             float *GT32, uint16_t *GThi, uint16_t *GTlo, hipStream_t st) {
    const int blocks = (P_pad + kGPts - 1) / kGPts;
    hipLaunchKernelGGL(k_assemble_G, dim3(blocks), dim3(256), 0, st, n, NP, P, P_pad, comp, seg_off_d,
                       verts_d, pts_d, G64, G32, Ghi, Glo, GT64, GT32, GThi, GTlo);
    return hipGetLastError();
}

hipError_t launch_assemble_M(int n, const int32_t *seg_off_d, const double *verts_d,
                             const double *wire_a_d, const GLRule &gl, double *M_d,
                             hipStream_t st) {
    const long long pairs = (long long)n * (n + 1) / 2;
    hipLaunchKernelGGL(k_assemble_M, dim3((unsigned)pairs), dim3(256), 0, st, n, seg_off_d,
                       verts_d, wire_a_d, gl, M_d);
    return hipGetLastError();
}

}  // namespace cosim
