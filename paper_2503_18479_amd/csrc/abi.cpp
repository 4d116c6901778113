// Host side of the C ABI declared in include/cosim.h: argument validation,
// geometry and plan objects, device memory, and the launch sequence of each
// call.  Every argument check runs before any HIP call, so the error paths
// are exercised without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cosim_sparam.h"
#include "internal.h"

using namespace cosim;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(COSIM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on the
// Legendre polynomial P_m (three-term recurrence), starting from the
// asymptotic root estimate cos(pi (i + 3/4) / (m + 1/2)).
GLRule make_gl_rule() {
    GLRule r;
    const int m = kGLOrder;
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int j = 2; j <= m; ++j) {
                const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int j = 2; j <= m; ++j) {
            const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = m * (x * p1 - p0) / (x * x - 1.0);
        const double w = 2.0 / ((1.0 - x * x) * dp * dp);
        r.x[i] = -x;
        r.w[i] = w;
        r.x[m - 1 - i] = x;
        r.w[m - 1 - i] = w;
    }
    return r;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void plan_free_workspace(cosim_plan *p) {
    dfree(p->bWt);
    dfree(p->bZmax);
    dfree(p->bTinv);
    dfree(p->bA32);
    dfree(p->I_ws);
    dfree(p->rpart);
    dfree(p->lpart);
    dfree(p->gws);
    dfree(p->gsys);
    dfree(p->rec_status);
    dfree(p->fac.L);
    dfree(p->fac.piv_row);
    dfree(p->fac.piv_val);
    dfree(p->fac.fmt);
    p->cap_systems = 0;
    p->cap_parts = 0;
    p->cap_lparts = 0;
    p->cap_gws = 0;
    p->rec_S = 0;
}

// FP32 records with FP64 refinement when the plan asks for them and the
// blocked LDL^T applies.  The default tolerance follows the precision of the
// contraction that consumes the solution: well below its own error.
BigRefine big_refine_args(const cosim_plan *p, int precision) {
    BigRefine rf;
    rf.on = p->refine && p->ldl_ok && big_plan(p->NP);
    rf.A32 = p->bA32;
    rf.max_iter = p->refine_iter;
    rf.tol = p->refine_tol > 0.0            ? p->refine_tol
             : precision == COSIM_FP64      ? 1e-12
             : precision == COSIM_FP32      ? 1e-9
                                            : 1e-7;
    return rf;
}

// The blocked LDL^T above 64 loops when every R_k > 0, else pivoted LU.
BigFactor big_factor_args(const cosim_plan *p) {
    BigFactor bf;
    bf.ldl = p->ldl_ok;
    bf.fmt = p->fac.fmt;
    bf.zmax = p->bZmax;
    bf.wt = p->bWt;
    bf.tinv = p->bTinv;
    return bf;
}

int check_loss_mode(const cosim_plan *p, int loss_mode) {
    if (loss_mode != COSIM_LOSS_MAG && loss_mode != COSIM_LOSS_COMPLEX &&
        loss_mode != COSIM_LOSS_RATIO)
        return fail(COSIM_EINVAL, "unknown loss mode %d", loss_mode);
    if (loss_mode == COSIM_LOSS_RATIO) {
        if (!(p->bext_z != 0.0))
            return fail(COSIM_EINVAL, "the enhancement-factor loss needs a nonzero incident field "
                                      "(the plan was assembled with bext_z = 0)");
        if (p->component != 2)
            return fail(COSIM_EINVAL, "the enhancement-factor loss is defined on the z-component "
                                      "(the uniform incident field has no x or y part)");
        if (p->n_drive > 0)
            return fail(COSIM_EINVAL, "the enhancement-factor loss is defined against the uniform "
                                      "incident field; this plan has a driven port");
    }
    return COSIM_OK;
}

int check_device(const cosim_plan *p) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(COSIM_EINVAL, "current device %d differs from the plan's device %d", dev,
                    p->device);
    return COSIM_OK;
}

// Workspace for `systems` systems whose partial sums use `chunks` P-chunks
// (and at least `parts` (chunk, system) slots of r, `lparts` of the loss),
// with the GEMM passes' planes when a batch this large above 64 loops takes
// them.
int ensure_workspace(cosim_plan *p, size_t systems, int chunks, size_t parts = 0,
                     size_t lparts = 0) {
    parts = std::max(parts, systems * (size_t)chunks);
    lparts = std::max(lparts, parts);
    const size_t gneed = big_plan(p->NP) && gemm_path(Prec::F64, p->NP, (int)systems)
                             ? gemm_ws_bytes(p->NP, (int)systems, p->P_pad)
                             : 0;
    const bool need32 = big_plan(p->NP) && p->ldl_ok && p->refine;
    if (systems <= p->cap_systems && parts <= p->cap_parts && lparts <= p->cap_lparts &&
        gneed <= p->cap_gws) {
        if (need32 && !p->bA32) {
            // the FP32 factor slots alone, beside the workspace (nothing else
            // moves, so buffers that captured graphs use stay where they are)
            const size_t NP = (size_t)p->NP;
            if (hipMalloc(&p->bA32, p->cap_systems * NP * NP * sizeof(float2)) != hipSuccess) {
                p->bA32 = nullptr;
                (void)hipGetLastError();
                return fail(COSIM_ENOMEM, "FP32 factor workspace for %zu systems failed",
                            p->cap_systems);
            }
        }
        return COSIM_OK;
    }
    const size_t ns = std::max(systems, p->cap_systems);
    const size_t np_parts = std::max(parts, p->cap_parts);
    const size_t nl_parts = std::max(lparts, p->cap_lparts);
    const size_t ngws = std::max(gneed, p->cap_gws);
    plan_free_workspace(p);
    const size_t n = (size_t)p->n, NP = (size_t)p->NP;
    const bool big = big_plan(p->NP);
    if (big && p->ldl_ok &&
        (hipMalloc((void **)&p->bWt, ns * 64 * NP * sizeof(double2)) != hipSuccess ||
         hipMalloc((void **)&p->bZmax, ns * sizeof(double)) != hipSuccess ||
         hipMalloc((void **)&p->bTinv, ns * 64 * 64 * sizeof(double2)) != hipSuccess)) {
        plan_free_workspace(p);
        (void)hipGetLastError();
        return fail(COSIM_ENOMEM, "LDL^T panel workspace for %zu systems failed", ns);
    }
    if (need32 && hipMalloc(&p->bA32, ns * NP * NP * sizeof(float2)) != hipSuccess) {
        plan_free_workspace(p);
        (void)hipGetLastError();
        return fail(COSIM_ENOMEM, "FP32 factor workspace for %zu systems failed", ns);
    }
    if (hipMalloc((void **)&p->I_ws, ns * n * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&p->rpart, np_parts * NP * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&p->lpart, nl_parts * sizeof(double)) != hipSuccess ||
        (ngws > 0 && hipMalloc(&p->gws, ngws) != hipSuccess) ||
        hipMalloc((void **)&p->gsys, ns * n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&p->rec_status, ns * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&p->fac.L, ns * NP * NP * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&p->fac.piv_row, ns * NP * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&p->fac.piv_val, ns * NP * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&p->fac.fmt, ns * sizeof(int)) != hipSuccess) {
        plan_free_workspace(p);
        (void)hipGetLastError();
        return fail(COSIM_ENOMEM, "workspace allocation for %zu systems, %zu partial sums failed",
                    ns, np_parts);
    }
    p->cap_systems = ns;
    p->cap_parts = np_parts;
    p->cap_lparts = nl_parts;
    p->cap_gws = ngws;
    return COSIM_OK;
}

// P-chunk count of the fused kernels (at most one per 64-row tile, at most 64).
int choose_chunks(const cosim_plan *p, Prec prec, size_t S, int variant) {
    // The launch has bx x c workgroups of equal work (c P-chunks of the
    // systems' blocks) and the chip holds `slots` of them at once.  Take the
    // fewest chunks whose workgroups fill the last round of resident
    // workgroups to at least 95% (fewer chunks, fewer partial sums to write
    // and read back); if none does (small batches), the best fill.
    const size_t per_block = (size_t)fused_systems_per_block(prec, p->NP, variant);
    const size_t bx = (S + per_block - 1) / per_block;
    const int tiles = p->P_pad / kPTile;
    const int cmax = std::max(1, std::min(tiles, 64));
    const size_t slots =
        (size_t)std::max(1, p->cus) * (size_t)fused_blocks_per_cu(prec, p->NP, variant);
    int best = cmax;
    double best_fill = -1.0;
    for (int c = 1; c <= cmax; ++c) {
        const int tpc = (tiles + c - 1) / c;
        const int cc = (tiles + tpc - 1) / tpc;  // chunks the tiles actually form
        const size_t blocks = bx * (size_t)cc;
        const size_t rounds = (blocks + slots - 1) / slots;
        const double fill = (double)blocks / (double)(rounds * slots);
        if (fill >= 0.95) return cc;
        if (fill > best_fill) {
            best_fill = fill;
            best = cc;
        }
    }
    return best;
}

// chunks of whole 64-row tiles, every chunk non-empty; *tiles_per_chunk out
int chunks_for(const cosim_plan *p, Prec prec, size_t S, int variant, int *tiles_per_chunk = nullptr) {
    const int tiles = p->P_pad / kPTile;
    if (big_plan(p->NP)) {  // chunks of r of the contraction kernels
        if (tiles_per_chunk) *tiles_per_chunk = 0;
        if (gemm_path(prec, p->NP, (int)S)) return gemm_shape(prec, p->NP, (int)S, p->P_pad).nkc;
        return mfma_shape(prec, p->NP, (int)S, p->P_pad, p->cus).nchunk;
    }
    const int want = choose_chunks(p, prec, S, variant);
    const int tpc = (tiles + want - 1) / want;
    if (tiles_per_chunk) *tiles_per_chunk = tpc;
    return (tiles + tpc - 1) / tpc;
}

// Loss partial sums per system of the contraction (the chunks of r, except
// for the GEMM passes, which sum the loss per block of points).
int loss_chunks(const cosim_plan *p, Prec prec, size_t S, int nchunk) {
    if (big_plan(p->NP) && gemm_path(prec, p->NP, (int)S))
        return gemm_shape(prec, p->NP, (int)S, p->P_pad).row_blocks;
    return nchunk;
}

// Tuning variants of a plan: the fused kernels' for up to 64 loops, a single
// one (the GEMM path) above.
int plan_variants(const cosim_plan *p, Prec prec) {
    return big_plan(p->NP) ? 1 : fused_variant_count(prec);
}

// Operands of the matrix-core contraction kernel in `prec` for S systems.
MfmaArgs mfma_args(const cosim_plan *p, Prec prec, int S, const MfmaShape &sh) {
    MfmaArgs a;
    switch (prec) {
        case Prec::F64: a.G = p->G64; a.GT = p->GT64; break;
        case Prec::F32: a.G = p->G32; a.GT = p->GT32; break;
        case Prec::BF16X3:
            a.G = p->Ghi; a.Glo = p->Glo; a.GT = p->GThi; a.GTlo = p->GTlo;
            break;
    }
    a.n = p->n;
    a.NP = p->NP;
    a.P = p->P;
    a.P_pad = p->P_pad;
    a.S = S;
    a.rows_per_chunk = sh.rows_per_chunk;
    a.nchunk = sh.nchunk;
    a.nsb = sh.nsb;
    a.rpart = p->rpart;
    a.lpart = p->lpart;
    return a;
}

// The loss (and gradient) contraction above 64 loops of S systems into the
// plan's rpart / lpart: the GEMM passes for large batches, else the fused
// kernel.
hipError_t big_contract(cosim_plan *p, Prec prec, int loss_mode, bool grad, int S,
                        const double2 *I, const double *T, double inc, hipStream_t st) {
    if (gemm_path(prec, p->NP, S)) {
        GemmLoss L;
        const MfmaArgs m = mfma_args(p, prec, S, MfmaShape{});
        L.G = m.G; L.Glo = m.Glo; L.GT = m.GT; L.GTlo = m.GTlo;
        L.I = I; L.T = T; L.inc = inc;
        L.n = p->n; L.NP = p->NP; L.P = p->P; L.P_pad = p->P_pad; L.S = S;
        L.ws = p->gws; L.lpart = p->lpart; L.rpart = p->rpart;
        return launch_gemm_loss(prec, loss_mode, grad, L, st);
    }
    const MfmaShape sh = mfma_shape(prec, p->NP, S, p->P_pad, p->cus);
    MfmaArgs a = mfma_args(p, prec, S, sh);
    a.I = I;
    a.T = T;
    a.inc = inc;
    return launch_mfma(prec, grad ? kMfmaLossGrad : kMfmaLoss, loss_mode, a, sh.waves, st);
}

int check_batch(const cosim_plan *p, int B, int F) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (B < 0 || F < 0) return fail(COSIM_EINVAL, "negative batch (%d) or frequency count (%d)", B, F);
    if ((size_t)B * (size_t)F > (size_t)INT32_MAX)
        return fail(COSIM_EINVAL, "B*F = %lld exceeds the system limit", (long long)B * F);
    return COSIM_OK;
}

// Side streams of the multi-instance call, per device, created on first use
// and kept for the life of the process (default priority), with one event per
// stream to join back and one to fork from.
struct StreamPool {
    int device = -1;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
    std::vector<hipEvent_t> extra;  // ordering of grouped instances
    // One multi-instance call at a time enqueues on the pool (host side).
    std::mutex mu;
    // Recorded on the caller's stream at the end of every call that used the
    // group workspace; the next such call's side streams wait for it, so the
    // grouped work of calls on different streams never overlaps.
    hipEvent_t ws_free = nullptr;
    bool ws_used = false;
    // factor records of grouped instances, sized for the largest call so far
    double2 *gA = nullptr, *gWt = nullptr, *gTinv = nullptr;
    int *gPiv = nullptr, *gFmt = nullptr;
    double *gZmax = nullptr;
    size_t capA = 0, capWt = 0, capTinv = 0, capPiv = 0, capSys = 0;
};
constexpr int kPoolStreams = 16;

// At least `count` events in pool->extra.
int pool_events(StreamPool *pool, size_t count) {
    while (pool->extra.size() < count) {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(COSIM_EDEVICE, "creating events failed");
        }
        pool->extra.push_back(ev);
    }
    return COSIM_OK;
}

// Group workspace of at least the given sizes (elements).  Growing it waits
// for the device first: earlier calls may still be using the old buffers.
int pool_group_ws(StreamPool *pool, size_t nA, size_t nWt, size_t nTinv, size_t nPiv, size_t nSys) {
    if (nA <= pool->capA && nWt <= pool->capWt && nTinv <= pool->capTinv && nPiv <= pool->capPiv &&
        nSys <= pool->capSys)
        return COSIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    dfree(pool->gA);
    dfree(pool->gWt);
    dfree(pool->gTinv);
    dfree(pool->gPiv);
    dfree(pool->gFmt);
    dfree(pool->gZmax);
    pool->capA = pool->capWt = pool->capTinv = pool->capPiv = pool->capSys = 0;
    if (hipMalloc((void **)&pool->gA, nA * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&pool->gWt, nWt * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&pool->gTinv, nTinv * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&pool->gPiv, nPiv * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&pool->gFmt, nSys * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&pool->gZmax, nSys * sizeof(double)) != hipSuccess) {
        dfree(pool->gA);
        dfree(pool->gWt);
        dfree(pool->gTinv);
        dfree(pool->gPiv);
        dfree(pool->gFmt);
        dfree(pool->gZmax);
        (void)hipGetLastError();
        return fail(COSIM_ENOMEM, "group workspace allocation failed");
    }
    pool->capA = nA;
    pool->capWt = nWt;
    pool->capTinv = nTinv;
    pool->capPiv = nPiv;
    pool->capSys = nSys;
    return COSIM_OK;
}

int stream_pool(int device, StreamPool **out) {
    static std::mutex mu;
    static std::vector<StreamPool *> pools;
    std::lock_guard<std::mutex> lock(mu);
    for (StreamPool *p : pools)
        if (p->device == device) {
            *out = p;
            return COSIM_OK;
        }
    StreamPool *p = new (std::nothrow) StreamPool;
    if (!p) return fail(COSIM_ENOMEM, "host allocation failed");
    p->device = device;
    bool ok = hipEventCreateWithFlags(&p->start, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&p->ws_free, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kPoolStreams; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (st) p->streams.push_back(st);
        if (ev) p->done.push_back(ev);
    }
    if (!ok) {
        for (hipStream_t st : p->streams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : p->done) (void)hipEventDestroy(ev);
        if (p->start) (void)hipEventDestroy(p->start);
        if (p->ws_free) (void)hipEventDestroy(p->ws_free);
        delete p;
        (void)hipGetLastError();
        return fail(COSIM_EDEVICE, "creating the side streams failed");
    }
    pools.push_back(p);
    *out = p;
    return COSIM_OK;
}

// Prefixes the current error message with the index of a multi-instance call.
int fail_instance(int code, int i) {
    char msg[sizeof(g_err)];
    std::snprintf(msg, sizeof(msg), "%s", g_err);
    return fail(code, "instance %d: %s", i, msg);
}

int check_assembled(const cosim_plan *p, int precision) {
    if (!(p->prec_mask & (1 << precision)))
        return fail(COSIM_EINVAL, "the plan was assembled without precision %d (mask %d)", precision,
                    p->prec_mask);
    return COSIM_OK;
}

int check_prec(int precision) {
    if (precision < COSIM_FP64 || precision > COSIM_BF16X3)
        return fail(COSIM_EINVAL, "unknown precision %d", precision);
    return COSIM_OK;
}

}  // namespace

extern "C" {

const char *cosim_last_error(void) { return g_err; }

int cosim_version(void) { return 1; }

int cosim_geometry_create(int n_loops, const int32_t *seg_off, const double *verts,
                          const double *wire_a, const double *R, cosim_geom_t *out) {
    if (!out) return fail(COSIM_EINVAL, "out is null");
    *out = nullptr;
    if (n_loops < 1) return fail(COSIM_EINVAL, "n_loops must be >= 1 (got %d)", n_loops);
    if (!seg_off || !verts || !wire_a || !R) return fail(COSIM_EINVAL, "null input array");
    if (seg_off[0] != 0) return fail(COSIM_EINVAL, "seg_off[0] must be 0");
    for (int k = 0; k < n_loops; ++k)
        if (seg_off[k + 1] - seg_off[k] < 3)
            return fail(COSIM_EINVAL, "loop %d has fewer than 3 vertices", k);
    const int V = seg_off[n_loops];
    for (int i = 0; i < 3 * V; ++i)
        if (!std::isfinite(verts[i])) return fail(COSIM_EINVAL, "vertex coordinate %d is not finite", i);
    for (int k = 0; k < n_loops; ++k) {
        if (!(wire_a[k] > 0.0) || !std::isfinite(wire_a[k]))
            return fail(COSIM_EINVAL, "wire radius of loop %d must be positive and finite", k);
        if (!(R[k] >= 0.0) || !std::isfinite(R[k]))
            return fail(COSIM_EINVAL, "resistance of loop %d must be >= 0 and finite", k);
    }
    cosim_geom *g = new (std::nothrow) cosim_geom;
    if (!g) return fail(COSIM_ENOMEM, "host allocation failed");
    g->n = n_loops;
    g->V = V;
    g->seg_off.assign(seg_off, seg_off + n_loops + 1);
    g->verts.assign(verts, verts + 3 * (size_t)V);
    g->wire_a.assign(wire_a, wire_a + n_loops);
    g->R.assign(R, R + n_loops);
    g->area_z.resize(n_loops);
    // z-component of each loop's vector area (shoelace); the flux of a uniform
    // B_ext,z through the loop is exactly B_ext,z times this
    for (int k = 0; k < n_loops; ++k) {
        double acc = 0.0;
        const int v0 = seg_off[k], v1 = seg_off[k + 1];
        for (int v = v0; v < v1; ++v) {
            const int w = (v + 1 == v1) ? v0 : v + 1;
            acc += g->verts[3 * v] * g->verts[3 * w + 1] - g->verts[3 * w] * g->verts[3 * v + 1];
        }
        g->area_z[k] = 0.5 * acc;
    }
    *out = g;
    return COSIM_OK;
}

int cosim_geometry_destroy(cosim_geom_t g) {
    delete g;
    return COSIM_OK;
}

int cosim_geometry_size(cosim_geom_t g, int *n_loops, int *n_verts) {
    if (!g) return fail(COSIM_EINVAL, "null geometry");
    if (n_loops) *n_loops = g->n;
    if (n_verts) *n_verts = g->V;
    return COSIM_OK;
}

int cosim_assemble(cosim_geom_t g, int P, const double *pts_d, double bext_z, void *stream,
                   cosim_plan_t *out) {
    return cosim_assemble_ex(g, P, pts_d, bext_z, COSIM_PREC_ALL, stream, out);
}

int cosim_assemble_ex(cosim_geom_t g, int P, const double *pts_d, double bext_z, int precisions,
                      void *stream, cosim_plan_t *out) {
    return cosim_assemble_component(g, P, pts_d, bext_z, precisions, 2, stream, out);
}

int cosim_assemble_component(cosim_geom_t g, int P, const double *pts_d, double bext_z,
                             int precisions, int component, void *stream, cosim_plan_t *out) {
    if (!out) return fail(COSIM_EINVAL, "out is null");
    *out = nullptr;
    if (!g) return fail(COSIM_EINVAL, "null geometry");
    if (P < 1) return fail(COSIM_EINVAL, "P must be >= 1 (got %d)", P);
    if (!pts_d) return fail(COSIM_EINVAL, "pts_d is null");
    if (!std::isfinite(bext_z)) return fail(COSIM_EINVAL, "bext_z is not finite");
    if (component < 0 || component > 2)
        return fail(COSIM_EINVAL, "field component %d is not 0 (x), 1 (y) or 2 (z)", component);
    if (precisions <= 0 || (precisions & ~COSIM_PREC_ALL))
        return fail(COSIM_EINVAL, "precision mask %d is not a non-empty subset of %d", precisions,
                    COSIM_PREC_ALL);
    if (g->n > kMaxLoopsBig)
        return fail(COSIM_EUNSUPPORTED, "%d loops: this build supports up to %d loops per plan",
                    g->n, kMaxLoopsBig);
    hipStream_t st = (hipStream_t)stream;
    cosim_plan *p = new (std::nothrow) cosim_plan;
    if (!p) return fail(COSIM_ENOMEM, "host allocation failed");
    p->n = g->n;
    p->NP = padded_loops(g->n);
    p->P = P;
    // rows of G padded with zeros to whole 64-row tiles of the fused kernels
    // (and whole 32-point sub-tiles of the matrix-core contraction kernel)
    p->P_pad = (P + kPTile - 1) / kPTile * kPTile;
    p->bext_z = bext_z;
    p->component = component;
    p->phi_h.resize(g->n);
    for (int k = 0; k < g->n; ++k) p->phi_h[k] = bext_z * g->area_z[k];
    p->exc_h.assign(3 * (size_t)g->n, 0.0);
    std::copy(p->phi_h.begin(), p->phi_h.end(), p->exc_h.begin());
    p->R_geom = g->R;
    p->R_h = g->R;
    p->ldl_ok = true;
    for (int k = 0; k < g->n; ++k) p->ldl_ok = p->ldl_ok && g->R[k] > 0.0;
    p->prec_mask = precisions;
    const bool want64 = precisions & (1 << COSIM_FP64), want32 = precisions & (1 << COSIM_FP32);
    const bool want16 = precisions & (1 << COSIM_BF16X3);

    int32_t *seg_d = nullptr;
    double *verts_d = nullptr, *wa_d = nullptr;
    auto cleanup = [&](int code) {
        dfree(seg_d);
        dfree(verts_d);
        dfree(wa_d);
        if (code != COSIM_OK) {
            cosim_plan_destroy(p);
            (void)hipGetLastError();
        }
        return code;
    };
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
        return cleanup(fail(COSIM_EDEVICE, "hipGetDevice failed"));
    const size_t gsz = (size_t)p->P_pad * p->NP;
    const size_t n = (size_t)g->n;
    // every precision keeps G row-major and transposed: the fused kernels read
    // the bf16 transposed copy, the matrix-core contraction kernel every
    // precision's (the adjoint's operands are runs of points of one loop)
    if ((want64 && (hipMalloc((void **)&p->G64, gsz * sizeof(double)) != hipSuccess ||
                    hipMalloc((void **)&p->GT64, gsz * sizeof(double)) != hipSuccess)) ||
        (want32 && (hipMalloc((void **)&p->G32, gsz * sizeof(float)) != hipSuccess ||
                    hipMalloc((void **)&p->GT32, gsz * sizeof(float)) != hipSuccess)) ||
        (want16 && (hipMalloc((void **)&p->Ghi, gsz * sizeof(uint16_t)) != hipSuccess ||
                    hipMalloc((void **)&p->Glo, gsz * sizeof(uint16_t)) != hipSuccess ||
                    hipMalloc((void **)&p->GThi, gsz * sizeof(uint16_t)) != hipSuccess ||
                    hipMalloc((void **)&p->GTlo, gsz * sizeof(uint16_t)) != hipSuccess)) ||
        hipMalloc((void **)&p->M_d, n * n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&p->phi_d, 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&p->R_d, n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&p->T_ratio, (size_t)P * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&seg_d, (n + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&verts_d, 3 * (size_t)g->V * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&wa_d, n * sizeof(double)) != hipSuccess)
        return cleanup(fail(COSIM_ENOMEM, "device allocation for the operators failed"));
    hipError_t e = hipSuccess;
#define ASM_TRY(x)                                                                      \
    do {                                                                                \
        e = (x);                                                                        \
        if (e != hipSuccess)                                                            \
            return cleanup(fail(COSIM_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e))); \
    } while (0)
    ASM_TRY(hipMemcpyAsync(seg_d, g->seg_off.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ASM_TRY(hipMemcpyAsync(verts_d, g->verts.data(), 3 * (size_t)g->V * sizeof(double), hipMemcpyHostToDevice, st));
    ASM_TRY(hipMemcpyAsync(wa_d, g->wire_a.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    ASM_TRY(hipMemcpyAsync(p->R_d, g->R.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    ASM_TRY(hipMemcpyAsync(p->phi_d, p->exc_h.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice, st));
    ASM_TRY(launch_assemble_G(g->n, p->NP, P, p->P_pad, component, seg_d, verts_d, pts_d, p->G64,
                              p->G32, p->Ghi, p->Glo, p->GT64, p->GT32, p->GThi, p->GTlo, st));
    ASM_TRY(launch_assemble_M(g->n, seg_d, verts_d, wa_d, make_gl_rule(), p->M_d, st));
    p->M_h.resize(n * n);
    ASM_TRY(hipMemcpyAsync(p->M_h.data(), p->M_d, n * n * sizeof(double), hipMemcpyDeviceToHost, st));
    ASM_TRY(hipStreamSynchronize(st));
#undef ASM_TRY
    cleanup(COSIM_OK);
    *out = p;
    return COSIM_OK;
}

int cosim_plan_destroy(cosim_plan_t p) {
    if (!p) return COSIM_OK;
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    dfree(p->G64);
    dfree(p->GT64);
    dfree(p->G32);
    dfree(p->GT32);
    dfree(p->Ghi);
    dfree(p->Glo);
    dfree(p->GThi);
    dfree(p->GTlo);
    dfree(p->M_d);
    dfree(p->phi_d);
    dfree(p->R_d);
    dfree(p->T_ratio);
    plan_free_workspace(p);
    // the parameter-gradient workspace has its own lifetime: a growing regular
    // workspace must not free it while a call still holds its address
    dfree(p->mu_ws);
    dfree(p->gpar_ws);
    p->par_cap = 0;
    delete p;
    return COSIM_OK;
}

int cosim_plan_factorisations(cosim_plan_t p, long long *count) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!count) return fail(COSIM_EINVAL, "count is null");
    *count = p->factorisations;
    return COSIM_OK;
}

int cosim_plan_size(cosim_plan_t p, int *n_loops, int *n_points) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (n_loops) *n_loops = p->n;
    if (n_points) *n_points = p->P;
    return COSIM_OK;
}

int cosim_plan_reserve(cosim_plan_t p, int max_batch, int max_freq) {
    int rc = check_batch(p, max_batch, max_freq);
    if (rc) return rc;
    if ((rc = check_device(p))) return rc;
    const size_t S = (size_t)max_batch * max_freq;
    // partial-sum slots for every batch up to S: a smaller batch may use more
    // P-chunks (the fused kernels split P further to fill the chip)
    size_t parts = S, lparts = S;
    for (int pr = COSIM_FP64; pr <= COSIM_BF16X3; ++pr)
        for (int v = 0; v < plan_variants(p, (Prec)pr); ++v) {
            if (big_plan(p->NP)) {  // a smaller batch may split the points further
                const size_t ns = (size_t)mfma_systems_per_block((Prec)pr);
                for (size_t sb = 1; sb <= (S + ns - 1) / ns; ++sb) {
                    const size_t Sb = std::min(S, sb * ns);
                    const int c = chunks_for(p, (Prec)pr, Sb, v);
                    parts = std::max(parts, Sb * (size_t)c);
                    lparts = std::max(lparts, Sb * (size_t)loss_chunks(p, (Prec)pr, Sb, c));
                }
                continue;
            }
            const size_t per_block = (size_t)fused_systems_per_block((Prec)pr, p->NP, v);
            const size_t bxmax = (S + per_block - 1) / per_block;
            for (size_t bx = 1; bx <= bxmax; ++bx) {
                const size_t Sb = std::min(S, bx * per_block);
                parts = std::max(parts, Sb * (size_t)chunks_for(p, (Prec)pr, Sb, v));
            }
        }
    return ensure_workspace(p, S, 1, parts, lparts);
}

int cosim_plan_copy_G(cosim_plan_t p, double *G_d, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!G_d) return fail(COSIM_EINVAL, "G_d is null");
    int rc = check_assembled(p, COSIM_FP64);
    if (rc) return rc;
    if ((rc = check_device(p))) return rc;
    // the plan stores rows of NP (>= n) columns; copy the n leading columns
    HIP_TRY(hipMemcpy2DAsync(G_d, (size_t)p->n * sizeof(double), p->G64, (size_t)p->NP * sizeof(double),
                             (size_t)p->n * sizeof(double), (size_t)p->P, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_plan_copy_M(cosim_plan_t p, double *M) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!M) return fail(COSIM_EINVAL, "M is null");
    std::memcpy(M, p->M_h.data(), p->M_h.size() * sizeof(double));
    return COSIM_OK;
}

int cosim_plan_copy_phi(cosim_plan_t p, double *phi) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!phi) return fail(COSIM_EINVAL, "phi is null");
    std::memcpy(phi, p->phi_h.data(), p->phi_h.size() * sizeof(double));
    return COSIM_OK;
}

int cosim_plan_set_drive(cosim_plan_t p, int nport, const int32_t *loop, const double *power,
                         const double *phase, double z0, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    const int n = p->n;
    if (nport < 0 || nport > n) return fail(COSIM_EINVAL, "nport %d is not in [0, %d]", nport, n);
    if (nport > 0 && (!loop || !power)) return fail(COSIM_EINVAL, "loop or power is null");
    if (nport > 0 && !(std::isfinite(z0) && z0 > 0.0))
        return fail(COSIM_EINVAL, "z0 must be finite and > 0");
    std::vector<double> R = p->R_geom, exc(3 * (size_t)n, 0.0);
    std::copy(p->phi_h.begin(), p->phi_h.end(), exc.begin());
    std::vector<char> seen(n, 0);
    for (int i = 0; i < nport; ++i) {
        const int k = loop[i];
        if (k < 0 || k >= n) return fail(COSIM_EINVAL, "port %d: loop %d is not in [0, %d)", i, k, n);
        if (seen[k]) return fail(COSIM_EINVAL, "port %d: loop %d is driven twice", i, k);
        seen[k] = 1;
        const double pw = power[i], ph = phase ? phase[i] : 0.0;
        if (!(std::isfinite(pw) && pw >= 0.0))
            return fail(COSIM_EINVAL, "port %d: power must be finite and >= 0", i);
        if (!std::isfinite(ph)) return fail(COSIM_EINVAL, "port %d: phase is not finite", i);
        // the wave sqrt(z0 P) of Eq. 4 from a source of internal impedance z0:
        // Thevenin EMF 2 sqrt(z0 P) with z0 in series with the loop
        const double a = 2.0 * std::sqrt(z0 * pw);
        R[k] += z0;
        exc[(size_t)n + k] = a * std::cos(ph);
        exc[2 * (size_t)n + k] = a * std::sin(ph);
    }
    int rc;
    if ((rc = check_device(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(p->R_d, R.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->phi_d, exc.data(), 3 * (size_t)n * sizeof(double),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    p->R_h = std::move(R);
    p->exc_h = std::move(exc);
    p->n_drive = nport;
    p->rec_S = 0;  // a factor record of the old circuit no longer applies
    const bool was = p->ldl_ok;
    p->ldl_ok = true;
    for (int k = 0; k < n; ++k) p->ldl_ok = p->ldl_ok && p->R_h[k] > 0.0;
    // the blocked LDL^T workspace exists only for plans that can use it
    if (p->ldl_ok != was) plan_free_workspace(p);
    return COSIM_OK;
}

int cosim_plan_set_refinement(cosim_plan_t p, int enable, int max_iter, double tol) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (enable && (max_iter < 1 || max_iter > 64))
        return fail(COSIM_EINVAL, "max_iter %d is not in [1, 64]", max_iter);
    if (enable && !(tol >= 0.0 && tol < 1.0))
        return fail(COSIM_EINVAL, "tol must be in [0, 1) (0: chosen per precision)");
    int rc;
    if ((rc = check_device(p))) return rc;
    // The workspace is kept: the next call adds the FP32 factor slots if the
    // mode needs them and they are missing, and moves nothing else.
    const bool on = enable != 0;
    p->refine = on;
    p->refine_iter = on ? max_iter : 0;
    p->refine_tol = on ? tol : 0.0;
    return COSIM_OK;
}

// Partial-sum slots that cosim_field_backward needs for S systems in any
// precision (chunks of the matrix-core kernel times S).
static size_t vjp_parts(const cosim_plan *p, size_t S) {
    size_t parts = S;
    for (int pr = COSIM_FP64; pr <= COSIM_BF16X3; ++pr)
        parts = std::max(parts, S * (size_t)mfma_shape((Prec)pr, p->NP, (int)S, p->P_pad, p->cus).nchunk);
    return parts;
}

int cosim_solve(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                double *I_d, int32_t *status_d, void *stream) {
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if (B == 0 || F == 0) return COSIM_OK;  // empty batch: nothing to do
    if (!C_d || !omega_d || !I_d || !status_d) return fail(COSIM_EINVAL, "null device pointer");
    if ((rc = check_device(p))) return rc;
    const int S = B * F;
    // room for the record and for a later cosim_field_backward that replays it
    if ((rc = ensure_workspace(p, (size_t)S, 1, vjp_parts(p, (size_t)S)))) return rc;
    p->rec_S = 0;
    p->factorisations++;
    hipStream_t st = (hipStream_t)stream;
    double2 *I = (double2 *)I_d;
    if (big_plan(p->NP)) {
        const BigFactor bf = big_factor_args(p);
        const BigRefine rf = big_refine_args(p, COSIM_FP64);
        HIP_TRY(big_factor(bf, rf, p->NP, p->n, S, F, p->M_d, p->R_d, C_d, omega_d, p->fac.L,
                           p->fac.piv_row, status_d, st));
        HIP_TRY(big_solve(bf, rf, p->NP, p->n, S, F, p->M_d, p->R_d, p->phi_d, C_d, omega_d,
                          p->fac.L, p->fac.piv_row, I, kRhsExcitation, nullptr, 0, 0.0, nullptr,
                          status_d, st));
    } else if (p->ldl_ok) {
        HIP_TRY(launch_ldl(p->NP, p->n, S, F, p->M_d, p->R_d, C_d, omega_d, p->phi_d, p->fac, I,
                           status_d, st));
        HIP_TRY(launch_solve_fallback(p->NP, p->n, S, F, p->M_d, p->R_d, p->phi_d, C_d, omega_d,
                                      I, status_d, p->fac, st));
    } else {
        HIP_TRY(launch_solve_forward(p->NP, p->n, S, F, p->M_d, p->R_d, p->phi_d, C_d, omega_d,
                                     I, status_d, p->fac, st));
    }
    // the forward status travels with the record: the adjoint replay starts from it
    HIP_TRY(hipMemcpyAsync(p->rec_status, status_d, (size_t)S * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st));
    p->rec_B = B;
    p->rec_F = F;
    p->rec_S = (size_t)S;
    return COSIM_OK;
}

int cosim_field(cosim_plan_t p, int B, int F, const double *I_d, int precision, int add_incident,
                void *Bz_d, void *stream) {
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if (B == 0 || F == 0) return COSIM_OK;  // empty batch: nothing to do
    if ((rc = check_prec(precision))) return rc;
    if ((rc = check_assembled(p, precision))) return rc;
    if (add_incident && p->component != 2)
        return fail(COSIM_EINVAL, "the uniform incident field has no x or y part (this plan holds "
                                  "component %d)", p->component);
    if (!I_d || !Bz_d) return fail(COSIM_EINVAL, "null device pointer");
    if ((rc = check_device(p))) return rc;
    const int S = B * F;
    const Prec prec = (Prec)precision;
    const MfmaShape sh = mfma_shape(prec, p->NP, S, p->P_pad, p->cus);
    MfmaArgs a = mfma_args(p, prec, S, sh);
    a.I = (const double2 *)I_d;
    a.Bout = Bz_d;
    a.inc = add_incident ? p->bext_z : 0.0;
    HIP_TRY(launch_mfma(prec, kMfmaField, 0, a, sh.waves, (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_field_backward(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                         const double *I_d, const double *gBz_d, int precision, int reuse,
                         double *gC_d, int32_t *status_d, void *stream) {
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if (B == 0 || F == 0) return COSIM_OK;  // empty batch: nothing to do
    if ((rc = check_prec(precision))) return rc;
    if ((rc = check_assembled(p, precision))) return rc;
    if (!C_d || !omega_d || !I_d || !gBz_d || !gC_d || !status_d)
        return fail(COSIM_EINVAL, "null device pointer");
    const size_t S = (size_t)B * F;
    if (reuse && !(p->rec_S == S && p->rec_B == B && p->rec_F == F))
        return fail(COSIM_EINVAL, "no factor record of a %d x %d cosim_solve to reuse (another "
                                  "call has used the plan's workspace since, or the shape "
                                  "differs)", B, F);
    if ((rc = check_device(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Prec prec = (Prec)precision;
    const MfmaShape sh = mfma_shape(prec, p->NP, (int)S, p->P_pad, p->cus);
    if (!reuse) {
        if ((rc = ensure_workspace(p, S, sh.nchunk))) return rc;
        p->rec_S = 0;
        p->factorisations++;
    } else if (S * (size_t)sh.nchunk > p->cap_parts) {
        return fail(COSIM_EINVAL, "the workspace lacks room for the partial sums");  // not reached
    }
    // r = G^T gBz per chunk of points; gBz = 2 dL/d conj(B), so conj(w) = conj(gBz) / 2
    MfmaArgs a = mfma_args(p, prec, (int)S, sh);
    a.gB = (const double2 *)gBz_d;
    HIP_TRY(launch_mfma(prec, kMfmaVjp, 0, a, sh.waves, st));
    double2 *I = (double2 *)I_d;  // read only by the adjoint solves
    if (reuse) {
        // the forward status is where the replay starts
        HIP_TRY(hipMemcpyAsync(status_d, p->rec_status, S * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
        if (big_plan(p->NP)) {
            const BigFactor bf = big_factor_args(p);
            const BigRefine rf = big_refine_args(p, COSIM_FP64);
            HIP_TRY(big_solve(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d,
                              omega_d, p->fac.L, p->fac.piv_row, I, kRhsPairs, p->rpart,
                              sh.nchunk, 0.5, p->gsys, status_d, st));
        } else {
            HIP_TRY(launch_replay_adjoint(p->NP, p->n, (int)S, F, p->fac, C_d, omega_d, I,
                                          p->rpart, sh.nchunk, 0.5, p->gsys, nullptr, status_d,
                                          st));
        }
    } else if (big_plan(p->NP)) {
        const BigFactor bf = big_factor_args(p);
        const BigRefine rf = big_refine_args(p, COSIM_FP64);
        HIP_TRY(big_factor(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, C_d, omega_d,
                           p->fac.L, p->fac.piv_row, status_d, st));
        HIP_TRY(big_solve(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d, omega_d,
                          p->fac.L, p->fac.piv_row, I, kRhsPairs, p->rpart, sh.nchunk, 0.5,
                          p->gsys, status_d, st));
    } else {
        HIP_TRY(launch_solve_adjoint(p->NP, p->n, (int)S, F, p->M_d, p->R_d, C_d, omega_d, I,
                                     p->rpart, sh.nchunk, 0.5, p->gsys, nullptr, status_d, false,
                                     st));
    }
    HIP_TRY(launch_reduce(p->n, B, F, 0, p->gsys, nullptr, 0.0, gC_d, nullptr, st));
    return COSIM_OK;
}

// The body of cosim_loss_and_grad; mu (optional, [S][n]) receives the adjoint
// solutions for the gradients of the other circuit variables.
// Operands of the fused contraction (64 loops or fewer) for S systems.
static FusedArgs fused_args(const cosim_plan *p, int precision, int S, int nchunk, int tpc,
                            const double *T_d, double inc) {
    FusedArgs a;
    a.G = precision == COSIM_FP64 ? (const void *)p->G64
          : precision == COSIM_FP32 ? (const void *)p->G32
                                    : (const void *)p->Ghi;
    a.Glo = p->Glo;
    a.GThi = p->GThi;
    a.GTlo = p->GTlo;
    a.T = T_d;
    a.inc = inc;
    a.P = p->P;
    a.P_pad = p->P_pad;
    a.nchunk = nchunk;
    a.rows_per_chunk = tpc * kPTile;
    a.I = p->I_ws;
    a.S = S;
    a.n = p->n;
    a.rpart = p->rpart;
    a.lpart = p->lpart;
    return a;
}

// Device buffers of one call on the path of 64 loops or fewer: the plan's
// own workspace, or views into caller-provided scratch memory.
struct SmallWs {
    double2 *I = nullptr;      // [S][n] currents
    double2 *rpart = nullptr;  // [nchunk][S][NP] adjoint partial sums
    double *lpart = nullptr;   // [nchunk][S] loss partial sums
    double *gsys = nullptr;    // [S][n] per-system gradient terms
    GJFactor fac;              // factor records
};

// Bytes of scratch memory that a call of S systems with nchunk P-chunks uses
// on the path of 64 loops or fewer, each view aligned to 256 bytes.
static size_t small_ws_bytes(const cosim_plan *p, size_t S, int nchunk, size_t *off) {
    const size_t NP = (size_t)p->NP, n = (size_t)p->n;
    const size_t sz[8] = {S * n * sizeof(double2),       S * nchunk * NP * sizeof(double2),
                          S * nchunk * sizeof(double),   S * n * sizeof(double),
                          S * NP * NP * sizeof(double2), S * NP * sizeof(int),
                          S * NP * sizeof(double2),      S * sizeof(int)};
    size_t at = 0;
    for (int i = 0; i < 8; ++i) {
        if (off) off[i] = at;
        at += (sz[i] + 255) / 256 * 256;
    }
    return at;
}

static int loss_and_grad_impl(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                       const double *T_d, int loss_mode, int precision, double *loss_d,
                       double *grad_d, int32_t *status_d, void *stream, double2 *mu,
                       void *scratch = nullptr, size_t scratch_bytes = 0) {
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if (B == 0 || F == 0) return COSIM_OK;  // empty batch: nothing to do
    if ((rc = check_prec(precision))) return rc;
    if ((rc = check_assembled(p, precision))) return rc;
    if ((rc = check_loss_mode(p, loss_mode))) return rc;
    if (!C_d || !omega_d || !T_d || !loss_d || !status_d)
        return fail(COSIM_EINVAL, "null device pointer");
    if ((rc = check_device(p))) return rc;
    const size_t S = (size_t)B * F;
    const Prec prec = (Prec)precision;
    const int variant = p->variant[precision];
    int tpc = 1;
    const int nchunk = chunks_for(p, prec, S, variant, &tpc);
    SmallWs w;
    if (scratch) {
        // caller-provided memory: nothing is allocated, the plan's workspace is
        // not touched, no phase timing
        if (big_plan(p->NP))
            return fail(COSIM_EUNSUPPORTED, "the scratch-memory call covers plans of at most %d "
                                            "loops (this plan has %d)", kMaxLoops, p->n);
        size_t off[8];
        const size_t need = small_ws_bytes(p, S, nchunk, off);
        if (need > scratch_bytes)
            return fail(COSIM_EINVAL, "%zu systems of %d loops need %zu bytes of scratch memory; "
                                      "the limit is %zu", S, p->n, need, scratch_bytes);
        char *b = (char *)scratch;
        w.I = (double2 *)(b + off[0]);
        w.rpart = (double2 *)(b + off[1]);
        w.lpart = (double *)(b + off[2]);
        w.gsys = (double *)(b + off[3]);
        w.fac.L = (double2 *)(b + off[4]);
        w.fac.piv_row = (int *)(b + off[5]);
        w.fac.piv_val = (double2 *)(b + off[6]);
        w.fac.fmt = (int *)(b + off[7]);
    } else {
        if ((rc = ensure_workspace(p, S, nchunk, 0, S * (size_t)loss_chunks(p, prec, S, nchunk))))
            return rc;
        p->rec_S = 0;  // the factor record of a cosim_solve is overwritten
        w.I = p->I_ws;
        w.rpart = p->rpart;
        w.lpart = p->lpart;
        w.gsys = p->gsys;
        w.fac = p->fac;
    }
    p->factorisations++;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t *ev = nullptr;
    if (!scratch && p->timing_used < p->timing_cap)
        ev = &p->events[(size_t)p->timing_used++ * (COSIM_PHASES + 1)];
    if (ev) HIP_TRY(hipEventRecord(ev[0], st));
    // Z is factorised once and the factorisation recorded; the forward solve and
    // the adjoint solve both replay the record.  With every R_k > 0 the
    // unpivoted LDL^T path runs and hands systems with a small pivot to the
    // pivoted Gauss-Jordan fallback; otherwise Gauss-Jordan runs for all.
    const bool grad = grad_d != nullptr;
    double scale = 1.0 / ((double)F * (double)p->P);
    // enhancement factor: the magnitude loss of the total field bext_z + B_z
    // against beta |bext_z|, scaled by 1 / bext_z^2
    const bool ratio = loss_mode == COSIM_LOSS_RATIO;
    if (ratio) {
        HIP_TRY(launch_scale((size_t)p->P, std::fabs(p->bext_z), T_d, p->T_ratio, st));
        T_d = p->T_ratio;
        scale /= p->bext_z * p->bext_z;
    }
    if (big_plan(p->NP)) {
        // factor, GEMM contractions with the loss epilogue between, solves
        const BigFactor bf = big_factor_args(p);
        const BigRefine rf = big_refine_args(p, precision);
        HIP_TRY(big_factor(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, C_d, omega_d,
                           p->fac.L, p->fac.piv_row, status_d, st));
        HIP_TRY(big_solve(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d, omega_d,
                          p->fac.L, p->fac.piv_row, p->I_ws, kRhsExcitation, nullptr, 0, 0.0,
                          nullptr, status_d, st));
        if (ev) HIP_TRY(hipEventRecord(ev[1], st));
        HIP_TRY(big_contract(p, prec, loss_mode, grad, (int)S, p->I_ws, T_d,
                             ratio ? p->bext_z : 0.0, st));
        if (ev) HIP_TRY(hipEventRecord(ev[2], st));
        if (grad)
            HIP_TRY(big_solve(bf, rf, p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d,
                              omega_d, p->fac.L, p->fac.piv_row, p->I_ws, kRhsPairs, p->rpart,
                              nchunk, scale, p->gsys, status_d, st, mu));
        if (ev) HIP_TRY(hipEventRecord(ev[3], st));
        HIP_TRY(launch_reduce(p->n, B, F, loss_chunks(p, prec, S, nchunk),
                              grad ? p->gsys : nullptr, p->lpart, scale, grad_d, loss_d, st));
        if (ev) HIP_TRY(hipEventRecord(ev[4], st));
        return COSIM_OK;
    }
    if (p->ldl_ok) {
        HIP_TRY(launch_ldl(p->NP, p->n, (int)S, F, p->M_d, p->R_d, C_d, omega_d, p->phi_d,
                           w.fac, w.I, status_d, st));
        HIP_TRY(launch_solve_fallback(p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d,
                                      omega_d, w.I, status_d, w.fac, st));
    } else {
        HIP_TRY(launch_solve_forward(p->NP, p->n, (int)S, F, p->M_d, p->R_d, p->phi_d, C_d,
                                     omega_d, w.I, status_d, w.fac, st));
    }
    if (ev) HIP_TRY(hipEventRecord(ev[1], st));
    FusedArgs a = fused_args(p, precision, (int)S, nchunk, tpc, T_d, ratio ? p->bext_z : 0.0);
    a.I = w.I;
    a.rpart = w.rpart;
    a.lpart = w.lpart;
    HIP_TRY(launch_fused(prec, p->NP, variant, loss_mode, grad, a, st));
    if (ev) HIP_TRY(hipEventRecord(ev[2], st));
    if (grad)
        HIP_TRY(launch_replay_adjoint(p->NP, p->n, (int)S, F, w.fac, C_d, omega_d, w.I,
                                      w.rpart, nchunk, scale, w.gsys, mu, status_d, st));
    if (ev) HIP_TRY(hipEventRecord(ev[3], st));
    HIP_TRY(launch_reduce(p->n, B, F, nchunk, grad ? w.gsys : nullptr, w.lpart, scale, grad_d,
                          loss_d, st));
    if (ev) HIP_TRY(hipEventRecord(ev[4], st));
    return COSIM_OK;
}

int cosim_loss_and_grad(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                        const double *T_d, int loss_mode, int precision, double *loss_d,
                        double *grad_d, int32_t *status_d, void *stream) {
    return loss_and_grad_impl(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss_d, grad_d,
                              status_d, stream, nullptr);
}

}  // extern "C"

int cosim::loss_and_grad_scratch(cosim_plan_t p, int B, int F, const double *C_d,
                                 const double *omega_d, const double *T_d, int loss_mode,
                                 int precision, double *loss_d, double *grad_d, int32_t *status_d,
                                 void *stream, void *scratch, size_t scratch_bytes) {
    if (!scratch) return fail(COSIM_EINVAL, "no scratch memory");
    return loss_and_grad_impl(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss_d, grad_d,
                              status_d, stream, nullptr, scratch, scratch_bytes);
}

int cosim::set_error(int code, const char *msg) { return fail(code, "%s", msg); }

int cosim::plan_device(const cosim_plan *p, int *device) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    int rc = check_device(p);
    if (rc) return rc;
    *device = p->device;
    return COSIM_OK;
}

extern "C" {

int cosim_loss_and_grad_params(cosim_plan_t p, int B, int F, const double *C_d,
                               const double *omega_d, const double *T_d, int loss_mode,
                               int precision, double *loss_d, double *gC_d, double *gR_d,
                               double *gL_d, double *gomega_d, int32_t *status_d, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!gC_d) return fail(COSIM_EINVAL, "null capacitance gradient (the adjoint always runs)");
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if (B == 0 || F == 0) return COSIM_OK;
    if (!gR_d && !gL_d && !gomega_d)
        return loss_and_grad_impl(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss_d, gC_d,
                                  status_d, stream, nullptr);
    if ((rc = check_device(p))) return rc;
    const size_t S = (size_t)B * F, n = (size_t)p->n;
    if (S > p->par_cap) {
        dfree(p->mu_ws);
        dfree(p->gpar_ws);
        p->par_cap = 0;
        if (hipMalloc((void **)&p->mu_ws, S * n * sizeof(double2)) != hipSuccess ||
            hipMalloc((void **)&p->gpar_ws, (2 * S * n + S) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(COSIM_ENOMEM, "parameter-gradient workspace for %zu systems failed", S);
        }
        p->par_cap = S;
    }
    if ((rc = loss_and_grad_impl(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss_d, gC_d,
                                 status_d, stream, p->mu_ws)))
        return rc;
    // workspace: R terms [S][n], L terms [S][n], then S values of dL/dw when the
    // caller does not want them
    double *gw = gomega_d ? gomega_d : p->gpar_ws + 2 * S * n;
    HIP_TRY(launch_param_grads(p->n, B, F, p->I_ws, p->mu_ws, C_d, omega_d, p->phi_d, p->M_d,
                               p->gpar_ws, p->gpar_ws + S * n, gR_d, gL_d, gw,
                               (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_resonant_capacitance(cosim_plan_t p, int F, const double *omega_d, int coupled,
                               double *Cr_d, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (F < 0) return fail(COSIM_EINVAL, "F = %d", F);
    if (F == 0) return COSIM_OK;
    if (!omega_d || !Cr_d) return fail(COSIM_EINVAL, "null device pointer");
    int rc = check_device(p);
    if (rc) return rc;
    HIP_TRY(launch_resonant_c(p->n, F, p->M_d, omega_d, coupled ? 1 : 0, Cr_d, (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_tanh_projection(int64_t count, const double *theta_d, double cmin, double cmax,
                          double *C_d, double *dC_d, void *stream) {
    if (count < 0) return fail(COSIM_EINVAL, "count = %lld", (long long)count);
    if (!(cmin < cmax) || !std::isfinite(cmin) || !std::isfinite(cmax))
        return fail(COSIM_EINVAL, "range [%g, %g]", cmin, cmax);
    if (count == 0) return COSIM_OK;
    if (!theta_d || !C_d) return fail(COSIM_EINVAL, "null device pointer");
    HIP_TRY(launch_tanh_project((size_t)count, theta_d, cmin, cmax, C_d, dC_d, (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_clip(int64_t count, double *x_d, double lo, double hi, void *stream) {
    if (count < 0) return fail(COSIM_EINVAL, "count = %lld", (long long)count);
    if (!(lo <= hi)) return fail(COSIM_EINVAL, "range [%g, %g]", lo, hi);
    if (count == 0) return COSIM_OK;
    if (!x_d) return fail(COSIM_EINVAL, "null device pointer");
    HIP_TRY(launch_clip((size_t)count, x_d, lo, hi, (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_adam_step(int count, double *C_d, const double *grad_d, double *m_d, double *v_d,
                    int32_t *step_d, double lr, double beta1, double beta2, double eps,
                    void *stream) {
    if (count < 0) return fail(COSIM_EINVAL, "count = %d", count);
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(COSIM_EINVAL, "betas must lie in [0, 1) (got %g, %g)", beta1, beta2);
    if (!std::isfinite(lr) || !(eps >= 0.0) || !std::isfinite(eps))
        return fail(COSIM_EINVAL, "lr must be finite and eps finite and >= 0");
    if (count == 0) return COSIM_OK;
    if (!C_d || !grad_d || !m_d || !v_d || !step_d) return fail(COSIM_EINVAL, "null device pointer");
    HIP_TRY(launch_adam(count, C_d, grad_d, m_d, v_d, step_d, lr, beta1, beta2, eps,
                        (hipStream_t)stream));
    return COSIM_OK;
}

// Arguments of one cosim_loss_and_grad_many call, for the group helpers.
struct ManyCall {
    const cosim_plan_t *plans;
    const int *B, *F;
    const double *const *C_d, *const *omega_d, *const *T_d;
    double *const *loss_d, *const *grad_d;
    int32_t *const *status_d;
    int loss_mode, precision, ns;
    StreamPool *pool;
    const std::vector<int> &chunks, &tpcs;
};

// Instances of 64 loops or fewer of one padded size (group `group`, stream k of
// the pool): factorisation with the forward solve, and the fallback, in shared launches on
// stream k, the contractions in one shared launch there too (or, unless every
// member uses variant 0, one per member on the other side streams), then the
// adjoint replay and the final sums.
static int enqueue_small_group(const ManyCall &mc, const std::vector<int> &g, int group, int k,
                               int &next_ev) {
    const cosim_plan_t *plans = mc.plans;
    const int *B = mc.B, *F = mc.F;
    const double *const *C_d = mc.C_d, *const *omega_d = mc.omega_d, *const *T_d = mc.T_d;
    double *const *loss_d = mc.loss_d, *const *grad_d = mc.grad_d;
    int32_t *const *status_d = mc.status_d;
    const std::vector<int> &chunks = mc.chunks;
    const int loss_mode = mc.loss_mode, precision = mc.precision, ns = mc.ns;
    const Prec prec = (Prec)precision;
    const bool grad = grad_d != nullptr, ratio = loss_mode == COSIM_LOSS_RATIO;
    StreamPool *pool = mc.pool;
    hipStream_t gs = pool->streams[k];
    const int NP = plans[g[0]]->NP;
    int first_rc = COSIM_OK;
    const std::vector<int> &tpcs = mc.tpcs;
    SmallGroup sg{};
    sg.count = (int)g.size();
    int Sg = 0;
    for (size_t m = 0; m < g.size(); ++m) {
        const int i = g[m];
        cosim_plan *p = plans[i];
        p->factorisations++;
        double sc = 1.0 / ((double)F[i] * (double)p->P);
        if (ratio) sc /= p->bext_z * p->bext_z;
        SmallInst &e = sg.in[m];
        e.M = p->M_d;
        e.R = p->R_d;
        e.phi = p->phi_d;
        e.C = C_d[i];
        e.omega = omega_d[i];
        e.I = p->I_ws;
        e.rpart = p->rpart;
        e.gsys = p->gsys;
        e.mu = nullptr;
        e.status = status_d[i];
        e.fac = p->fac;
        e.n = p->n;
        e.F = F[i];
        e.S = B[i] * F[i];
        e.nchunk = chunks[i];
        e.s0 = Sg;
        e.rscale = sc;
        Sg += e.S;
    }
    hipEvent_t ev_fwd = pool->extra[group];
    if (launch_small_group(NP, sg, Sg, SmallPhase::Factor, gs) != hipSuccess ||
        launch_small_group(NP, sg, Sg, SmallPhase::Fallback, gs) != hipSuccess ||
        hipEventRecord(ev_fwd, gs) != hipSuccess) {
        return fail(COSIM_EDEVICE, "grouped solve launch failed");
    }
    // contractions: one launch for the group when every member uses the
    // default variant, else one per member on the other side streams
    bool one = true;
    for (int i : g) one = one && plans[i]->variant[precision] == 0;
    if (one) {
        FusedGroup fg{};
        fg.count = (int)g.size();
        const int per_block = fused_systems_per_block(prec, NP, 0);
        int blocks = 0;
        bool ok = true;
        for (size_t m = 0; m < g.size() && ok; ++m) {
            const int i = g[m];
            cosim_plan *p = plans[i];
            const double *Ti = T_d[i];
            if (ratio) {
                ok = launch_scale((size_t)p->P, std::fabs(p->bext_z), T_d[i], p->T_ratio,
                                  gs) == hipSuccess;
                Ti = p->T_ratio;
            }
            fg.in[m] = fused_args(p, precision, B[i] * F[i], chunks[i], tpcs[i], Ti,
                                  ratio ? p->bext_z : 0.0);
            fg.first[m] = blocks;
            fg.bx[m] = (B[i] * F[i] + per_block - 1) / per_block;
            blocks += fg.bx[m] * chunks[i];
        }
        if (!ok || launch_fused_group(prec, NP, loss_mode, grad, fg, blocks, gs) != hipSuccess) {
            return fail(COSIM_EDEVICE, "grouped contraction launch failed");
        }
    }
    for (size_t m = 0; !one && m < g.size() && first_rc == COSIM_OK; ++m) {
        const int i = g[m];
        cosim_plan *p = plans[i];
        hipStream_t cs = pool->streams[(k + 1 + m) % ns];
        hipEvent_t ev_c = pool->extra[next_ev++];
        const double *Ti = T_d[i];
        bool ok = hipStreamWaitEvent(cs, ev_fwd, 0) == hipSuccess;
        if (ok && ratio) {
            ok = launch_scale((size_t)p->P, std::fabs(p->bext_z), T_d[i], p->T_ratio, cs) ==
                 hipSuccess;
            Ti = p->T_ratio;
        }
        const FusedArgs a = fused_args(p, precision, B[i] * F[i], chunks[i], tpcs[i], Ti,
                                       ratio ? p->bext_z : 0.0);
        ok = ok &&
             launch_fused(prec, NP, p->variant[precision], loss_mode, grad, a, cs) ==
                 hipSuccess &&
             hipEventRecord(ev_c, cs) == hipSuccess &&
             hipStreamWaitEvent(gs, ev_c, 0) == hipSuccess;
        if (!ok) first_rc = fail_instance(fail(COSIM_EDEVICE, "contraction launch failed"), i);
    }
    if (first_rc != COSIM_OK) return first_rc;
    if (grad && launch_small_group(NP, sg, Sg, SmallPhase::Adjoint, gs) != hipSuccess) {
        return fail(COSIM_EDEVICE, "grouped adjoint launch failed");
    }
    ReduceGroup rg{};
    rg.count = (int)g.size();
    int Bg = 0;
    for (size_t m = 0; m < g.size(); ++m) {
        const int i = g[m];
        rg.in[m] = {grad ? plans[i]->gsys : nullptr, plans[i]->lpart,
                    grad ? grad_d[i] : nullptr, loss_d[i], sg.in[m].rscale,
                    plans[i]->n, B[i], F[i], chunks[i], Bg};
        Bg += B[i];
    }
    if (launch_reduce_group(rg, Bg, gs) != hipSuccess)
        first_rc = fail(COSIM_EDEVICE, "grouped reduction launch failed");
    return first_rc;
}

// Instances above 64 loops of one padded size (group `group`, stream k of the
// pool): blocked LDL^T and forward solve in shared launches on stream k with
// factor records in the pool's group workspace (running offsets `off`), the
// GEMM contractions per member on the other side streams, then the adjoint
// solve and the final sums on stream k.
static int enqueue_big_group(const ManyCall &mc, const std::vector<int> &g, int group, int k,
                             int &next_ev, size_t (&off)[5]) {
    const cosim_plan_t *plans = mc.plans;
    const int *B = mc.B, *F = mc.F;
    const double *const *C_d = mc.C_d, *const *omega_d = mc.omega_d, *const *T_d = mc.T_d;
    double *const *loss_d = mc.loss_d, *const *grad_d = mc.grad_d;
    int32_t *const *status_d = mc.status_d;
    const std::vector<int> &chunks = mc.chunks;
    const int loss_mode = mc.loss_mode, precision = mc.precision, ns = mc.ns;
    const Prec prec = (Prec)precision;
    const bool grad = grad_d != nullptr, ratio = loss_mode == COSIM_LOSS_RATIO;
    StreamPool *pool = mc.pool;
    hipStream_t gs = pool->streams[k];
    const int NP = plans[g[0]]->NP;
    int first_rc = COSIM_OK;
    GroupArgs ga{};
    ga.count = (int)g.size();
    int Sg = 0;
    std::vector<double> scale(g.size());
    std::vector<const double *> Teff(g.size());
    for (size_t m = 0; m < g.size(); ++m) {
        const int i = g[m];
        cosim_plan *p = plans[i];
        scale[m] = 1.0 / ((double)F[i] * (double)p->P);
        Teff[m] = T_d[i];
        if (ratio) scale[m] /= p->bext_z * p->bext_z;
        p->factorisations++;
        GroupInst &e = ga.in[m];
        e.M = p->M_d;
        e.R = p->R_d;
        e.phi = p->phi_d;
        e.C = C_d[i];
        e.omega = omega_d[i];
        e.I = p->I_ws;
        e.rhs = p->rpart;
        e.gsys = p->gsys;
        e.mu = nullptr;
        e.status = status_d[i];
        e.n = p->n;
        e.F = F[i];
        e.S = B[i] * F[i];
        e.nchunk = chunks[i];
        e.s0 = Sg;
        e.rscale = scale[m];
        Sg += e.S;
    }
    BigFactor bf;
    bf.ldl = true;
    bf.fmt = pool->gFmt + off[4];
    bf.zmax = pool->gZmax + off[4];
    bf.wt = pool->gWt + off[1];
    bf.tinv = pool->gTinv + off[2];
    double2 *A = pool->gA + off[0];
    int *piv = pool->gPiv + off[3];
    off[0] += (size_t)Sg * NP * NP;
    off[1] += (size_t)Sg * 64 * NP;
    off[2] += (size_t)Sg * 64 * 64;
    off[3] += (size_t)Sg * NP;
    off[4] += (size_t)Sg;
    hipEvent_t ev_fwd = pool->extra[group];
    if (big_group_factor(bf, ga, NP, Sg, A, piv, gs) != hipSuccess ||
        big_group_solve(ga, NP, Sg, A, piv, kRhsExcitation, gs) != hipSuccess ||
        hipEventRecord(ev_fwd, gs) != hipSuccess) {
        return fail(COSIM_EDEVICE, "grouped solve launch failed");
    }
    // Contractions: the members on the matrix-core kernel path in one launch
    // on the group's stream, after its forward solve; members with enough
    // systems for the GEMM passes each on a side stream, joined by events.
    MfmaGroup mg;
    int mblocks = 0, mwaves = 0;
    for (size_t m = 0; m < g.size() && first_rc == COSIM_OK; ++m) {
        const int i = g[m];
        cosim_plan *p = plans[i];
        const int S = B[i] * F[i];
        const double *Ti = Teff[m];
        if (!gemm_path(prec, p->NP, S)) {
            if (ratio) {
                if (launch_scale((size_t)p->P, std::fabs(p->bext_z), T_d[i], p->T_ratio, gs) !=
                    hipSuccess) {
                    first_rc = fail_instance(fail(COSIM_EDEVICE, "target scaling failed"), i);
                    break;
                }
                Ti = p->T_ratio;
            }
            const MfmaShape sh = mfma_shape(prec, p->NP, S, p->P_pad, p->cus);
            MfmaArgs a = mfma_args(p, prec, S, sh);
            a.I = p->I_ws;
            a.T = Ti;
            a.inc = ratio ? p->bext_z : 0.0;
            mg.first[mg.count] = mblocks;
            mg.in[mg.count++] = a;
            mblocks += (sh.nchunk * sh.nsb + 7) / 8 * 8;
            mwaves = sh.waves;  // a function of the padded loop count, shared by the group
            continue;
        }
        hipStream_t cs = pool->streams[(k + 1 + m) % ns];
        hipEvent_t ev_c = pool->extra[next_ev++];
        bool ok = hipStreamWaitEvent(cs, ev_fwd, 0) == hipSuccess;
        if (ok && ratio) {
            ok = launch_scale((size_t)p->P, std::fabs(p->bext_z), T_d[i], p->T_ratio, cs) ==
                 hipSuccess;
            Ti = p->T_ratio;
        }
        ok = ok &&
             big_contract(p, prec, loss_mode, grad, S, p->I_ws, Ti, ratio ? p->bext_z : 0.0, cs) ==
                 hipSuccess &&
             hipEventRecord(ev_c, cs) == hipSuccess && hipStreamWaitEvent(gs, ev_c, 0) == hipSuccess;
        if (!ok) first_rc = fail_instance(fail(COSIM_EDEVICE, "contraction launch failed"), i);
    }
    if (first_rc == COSIM_OK && mg.count > 0 &&
        launch_mfma_group(prec, grad, loss_mode, mg, mblocks, mwaves, gs) != hipSuccess)
        first_rc = fail(COSIM_EDEVICE, "grouped contraction launch failed");
    if (first_rc != COSIM_OK) return first_rc;
    if (grad &&
        big_group_solve(ga, NP, Sg, A, piv, kRhsPairs, gs) != hipSuccess) {
        return fail(COSIM_EDEVICE, "grouped adjoint launch failed");
    }
    ReduceGroup rg{};
    rg.count = (int)g.size();
    int Bg = 0;
    for (size_t m = 0; m < g.size(); ++m) {
        const int i = g[m];
        rg.in[m] = {grad ? plans[i]->gsys : nullptr, plans[i]->lpart,
                    grad ? grad_d[i] : nullptr, loss_d[i], scale[m],
                    plans[i]->n, B[i], F[i],
                    loss_chunks(plans[i], prec, (size_t)B[i] * F[i], chunks[i]), Bg};
        Bg += B[i];
    }
    if (launch_reduce_group(rg, Bg, gs) != hipSuccess)
        first_rc = fail(COSIM_EDEVICE, "grouped reduction launch failed");
    return first_rc;
}

int cosim_loss_and_grad_many(int count, const cosim_plan_t *plans, const int *B, const int *F,
                             const double *const *C_d, const double *const *omega_d,
                             const double *const *T_d, int loss_mode, int precision,
                             double *const *loss_d, double *const *grad_d,
                             int32_t *const *status_d, void *stream) {
    if (count < 0) return fail(COSIM_EINVAL, "count = %d", count);
    if (count == 0) return COSIM_OK;
    if (!plans || !B || !F || !C_d || !omega_d || !T_d || !loss_d || !status_d)
        return fail(COSIM_EINVAL, "null host array");
    int rc = check_prec(precision);
    if (rc) return rc;
    if (loss_mode != COSIM_LOSS_MAG && loss_mode != COSIM_LOSS_COMPLEX &&
        loss_mode != COSIM_LOSS_RATIO)
        return fail(COSIM_EINVAL, "unknown loss mode %d", loss_mode);
    for (int i = 0; i < count; ++i)
        if (plans[i] && (rc = check_loss_mode(plans[i], loss_mode))) return fail_instance(rc, i);
    // every instance is checked before anything is enqueued
    for (int i = 0; i < count; ++i) {
        if ((rc = check_batch(plans[i], B[i], F[i])))
            return fail_instance(rc, i);
        if ((size_t)B[i] * F[i] == 0) continue;
        if ((rc = check_assembled(plans[i], precision)) || (rc = check_device(plans[i])))
            return fail_instance(rc, i);
        if (!C_d[i] || !omega_d[i] || !T_d[i] || !loss_d[i] || !status_d[i])
            return fail(COSIM_EINVAL, "instance %d: null device pointer", i);
    }
    for (int i = 0; i < count; ++i) plans[i]->rec_S = 0;  // workspaces are overwritten
    {  // a plan's workspace serves one instance at a time
        std::vector<cosim_plan_t> sorted(plans, plans + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(COSIM_EINVAL, "a plan appears more than once");
    }
    // instances run on side streams that wait for `stream` and that `stream`
    // waits for afterwards
    StreamPool *pool = nullptr;
    if ((rc = stream_pool(plans[0]->device, &pool))) return rc;
    std::lock_guard<std::mutex> pool_lock(pool->mu);
    hipStream_t st = (hipStream_t)stream;
    const int ns = std::min(kPoolStreams, count);
    // Instances with every R_k > 0 (no refinement, no phase timing) are
    // factored and solved together, up to kGroupMax (above 64 loops) or
    // kSmallGroupMax (64 or fewer) of one padded size per group: one launch per
    // solver step for all their systems, in place of one per instance.  Their
    // contractions stay per instance.
    // While the stream is captured, instances above 64 loops are not grouped:
    // ending a capture that held their grouped launches once crashed the HIP
    // runtime on the host, with no cause found, and such a capture has not
    // been run again.  Their groups would also keep factor records in the
    // pool's shared workspace, whose reuse across calls is ordered by the event
    // ws_free of the previous grouping call, recorded outside any capture.
    // Groups of 64 loops or fewer use only their plans' workspaces and events
    // recorded inside the call (and capture correctly), so they are grouped
    // under capture too.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cap));
    const bool captured = cap != hipStreamCaptureStatusNone;
    std::vector<std::vector<int>> groups;
    std::vector<char> grouped(count, 0);
    {
        std::vector<std::pair<int, int>> cand;  // (NP, instance)
        for (int i = 0; i < count; ++i) {
            const cosim_plan *p = plans[i];
            if ((size_t)B[i] * F[i] == 0 || !p->ldl_ok) continue;
            if (big_refine_args(p, precision).on || p->timing_used < p->timing_cap) continue;
            if (captured && big_plan(p->NP)) continue;
            cand.emplace_back(p->NP, i);
        }
        std::stable_sort(cand.begin(), cand.end(),
                         [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
                             return a.first < b.first;
                         });
        for (size_t j = 0; j < cand.size();) {
            size_t e = j;
            while (e < cand.size() && cand[e].first == cand[j].first) ++e;
            const size_t gmax = big_plan(cand[j].first) ? kGroupMax : kSmallGroupMax;
            if (e - j >= 2)  // a class of one instance gains nothing
                for (size_t k = j; k < e; k += gmax) {
                    std::vector<int> g;
                    for (size_t m = k; m < std::min(e, k + gmax); ++m) {
                        g.push_back(cand[m].second);
                        grouped[cand[m].second] = 1;
                    }
                    groups.push_back(g);
                }
            j = e;
        }
    }
    // workspaces first (allocation, when growing, happens before anything is enqueued)
    size_t nA = 0, nWt = 0, nTinv = 0, nPiv = 0, nSys = 0;
    std::vector<int> chunks(count, 0), tpcs(count, 1);
    bool big_groups = false;
    for (const std::vector<int> &g : groups)
        for (int i : g) {
            const size_t S = (size_t)B[i] * F[i], NP = (size_t)plans[i]->NP;
            chunks[i] = chunks_for(plans[i], (Prec)precision, S, plans[i]->variant[precision],
                                   &tpcs[i]);
            if ((rc = ensure_workspace(plans[i], S, chunks[i], 0,
                                       S * (size_t)loss_chunks(plans[i], (Prec)precision, S,
                                                               chunks[i]))))
                return fail_instance(rc, i);
            if (!big_plan((int)NP)) continue;  // its own factor record
            big_groups = true;
            nA += S * NP * NP;
            nWt += S * 64 * NP;
            nTinv += S * 64 * 64;
            nPiv += S * NP;
            nSys += S;
        }
    if (big_groups && (rc = pool_group_ws(pool, nA, nWt, nTinv, nPiv, nSys))) return rc;
    if (!groups.empty() && (rc = pool_events(pool, groups.size() + count))) return rc;
    HIP_TRY(hipEventRecord(pool->start, st));
    for (int k = 0; k < ns; ++k) {
        HIP_TRY(hipStreamWaitEvent(pool->streams[k], pool->start, 0));
        // the group workspace is shared by every call on the device: wait
        // until the previous call that used it has finished (never under
        // capture, where no group uses it)
        if (big_groups && pool->ws_used)
            HIP_TRY(hipStreamWaitEvent(pool->streams[k], pool->ws_free, 0));
    }
    // largest work first, each item to the stream with the least work so far
    // (work ~ systems x (NP^3 for the solves + P NP for the contraction); a
    // group counts as its largest member)
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
        const double S = (double)B[i] * F[i], np = (double)plans[i]->NP;
        cost[i] = S * (np * np * np + (double)plans[i]->P * np);
    }
    struct Item {
        double cost;
        int inst, group;  // one of them is -1
    };
    std::vector<Item> items;
    for (int g = 0; g < (int)groups.size(); ++g) {
        double c = 0.0;
        for (int i : groups[g]) c = std::max(c, cost[i]);
        items.push_back({c, -1, g});
    }
    for (int i = 0; i < count; ++i)
        if (!grouped[i]) items.push_back({cost[i], i, -1});
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &b) { return a.cost > b.cost; });
    std::vector<double> load(ns, 0.0);
    size_t off[5] = {0, 0, 0, 0, 0};  // running offsets into the group workspace
    int first_rc = COSIM_OK;
    int next_ev = (int)groups.size();
    const ManyCall mc{plans, B, F, C_d, omega_d, T_d, loss_d, grad_d, status_d,
                      loss_mode, precision, ns, pool, chunks, tpcs};
    for (const Item &it : items) {
        if (first_rc != COSIM_OK) break;
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += it.cost;
        hipStream_t gs = pool->streams[k];
        if (it.inst >= 0) {
            const int i = it.inst;
            if ((rc = cosim_loss_and_grad(plans[i], B[i], F[i], C_d[i], omega_d[i], T_d[i],
                                          loss_mode, precision, loss_d[i],
                                          grad_d ? grad_d[i] : nullptr, status_d[i], gs)))
                first_rc = fail_instance(rc, i);
            continue;
        }
        // a group: factor and forward solve on gs, contractions spread over the
        // pool, then adjoint solve and reductions on gs
        const std::vector<int> &g = groups[it.group];
        first_rc = big_plan(plans[g[0]]->NP) ? enqueue_big_group(mc, g, it.group, k, next_ev, off)
                                             : enqueue_small_group(mc, g, it.group, k, next_ev);
    }
    for (int k = 0; k < ns; ++k) {  // join even after an error
        HIP_TRY(hipEventRecord(pool->done[k], pool->streams[k]));
        HIP_TRY(hipStreamWaitEvent(st, pool->done[k], 0));
    }
    if (big_groups) {
        HIP_TRY(hipEventRecord(pool->ws_free, st));
        pool->ws_used = true;
    }
    return first_rc;
}

int cosim_plan_set_variant(cosim_plan_t p, int precision, int variant) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    int rc = check_prec(precision);
    if (rc) return rc;
    if (variant < 0 || variant >= plan_variants(p, (Prec)precision))
        return fail(COSIM_EINVAL, "variant %d out of range [0, %d)", variant,
                    plan_variants(p, (Prec)precision));
    p->variant[precision] = variant;
    return COSIM_OK;
}

int cosim_plan_get_variant(cosim_plan_t p, int precision, int *variant, int *n_variants) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    int rc = check_prec(precision);
    if (rc) return rc;
    if (variant) *variant = p->variant[precision];
    if (n_variants) *n_variants = plan_variants(p, (Prec)precision);
    return COSIM_OK;
}

int cosim_plan_autotune(cosim_plan_t p, int B, int F, const double *C_d, const double *omega_d,
                        const double *T_d, int loss_mode, int precision, int reps, void *stream,
                        double *ms_out) {
    int rc = check_batch(p, B, F);
    if (rc) return rc;
    if ((rc = check_prec(precision))) return rc;
    if ((rc = check_assembled(p, precision))) return rc;
    if (B == 0 || F == 0) return COSIM_OK;
    if (!C_d || !omega_d || !T_d) return fail(COSIM_EINVAL, "null device pointer");
    if (reps < 1) return fail(COSIM_EINVAL, "reps must be >= 1");
    if ((rc = check_device(p))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t S = (size_t)B * F;
    double *loss = nullptr, *grad = nullptr;
    int32_t *status = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](int code) {
        dfree(loss);
        dfree(grad);
        dfree(status);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return code;
    };
    if (hipMalloc((void **)&loss, (size_t)B * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&grad, (size_t)B * p->n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&status, S * sizeof(int32_t)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return done(fail(COSIM_ENOMEM, "autotune scratch allocation failed"));
    const int nv = plan_variants(p, (Prec)precision);
    int best = 0;
    float best_ms = 0.f;
    const int saved_timing = p->timing_cap;
    p->timing_cap = 0;  // tuning calls are not recorded
    for (int v = 0; v < nv; ++v) {
        p->variant[precision] = v;
        rc = cosim_loss_and_grad(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss, grad,
                                 status, stream);  // warm-up (and workspace growth)
        if (rc) { p->timing_cap = saved_timing; return done(rc); }
        if (hipEventRecord(e0, st) != hipSuccess) { p->timing_cap = saved_timing; return done(fail(COSIM_EDEVICE, "hipEventRecord failed")); }
        for (int r = 0; r < reps; ++r) {
            rc = cosim_loss_and_grad(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss, grad,
                                     status, stream);
            if (rc) { p->timing_cap = saved_timing; return done(rc); }
        }
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            p->timing_cap = saved_timing;
            return done(fail(COSIM_EDEVICE, "timing the variants failed"));
        }
        ms /= (float)reps;
        if (ms_out) ms_out[v] = ms;
        if (v == 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
    }
    p->timing_cap = saved_timing;
    p->variant[precision] = best;
    return done(COSIM_OK);
}

int cosim_plan_timing(cosim_plan_t p, int max_records) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (max_records < 0) return fail(COSIM_EINVAL, "max_records must be >= 0");
    int rc = check_device(p);
    if (rc) return rc;
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.clear();
    p->timing_cap = p->timing_used = 0;
    const size_t ne = (size_t)max_records * (COSIM_PHASES + 1);
    p->events.resize(ne, nullptr);
    for (size_t i = 0; i < ne; ++i) {
        if (hipEventCreate(&p->events[i]) != hipSuccess) {
            for (size_t j = 0; j < i; ++j) (void)hipEventDestroy(p->events[j]);
            p->events.clear();
            return fail(COSIM_EDEVICE, "hipEventCreate failed");
        }
    }
    p->timing_cap = max_records;
    return COSIM_OK;
}

int cosim_plan_timing_read(cosim_plan_t p, double *ms, int max_records, int *n_records) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (!n_records || (max_records > 0 && !ms)) return fail(COSIM_EINVAL, "null output");
    const int nr = std::min(p->timing_used, max_records);
    for (int r = 0; r < nr; ++r) {
        hipEvent_t *ev = &p->events[(size_t)r * (COSIM_PHASES + 1)];
        HIP_TRY(hipEventSynchronize(ev[COSIM_PHASES]));
        for (int ph = 0; ph < COSIM_PHASES; ++ph) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, ev[ph], ev[ph + 1]));
            ms[(size_t)r * COSIM_PHASES + ph] = (double)t;
        }
    }
    *n_records = nr;
    p->timing_used = 0;
    return COSIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// S-parameter pipeline (include/cosim_sparam.h)
// ---------------------------------------------------------------------------

struct cosim_sp {
    int device = -1;
    int N = 0, prec_mask = 0;
    SpDev d;
    SpWork w;
    size_t cap = 0;  // configurations the workspace holds
    void *blas = nullptr;
    std::vector<int> ix, iy;  // host copies of the index pairs
    ~cosim_sp() {
        dfree(d.S0);
        dfree(d.K);
        dfree(d.r0);
        dfree(d.exc);
        dfree(d.ix);
        dfree(d.iy);
        dfree(d.fields64);
        dfree(d.fields32);
        dfree(w.X);
        dfree(w.Xg);
        dfree(w.Y);
        dfree(w.Rp);
        dfree(w.lpart);
        sp_blas_destroy(blas);
    }
};

namespace {

std::once_flag g_sp_lds_once;
hipError_t g_sp_lds_err = hipSuccess;

int sp_check_device(const cosim_sp *p) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(COSIM_EINVAL, "current device %d differs from the S-parameter plan's device %d",
                    dev, p->device);
    return COSIM_OK;
}

// P-chunk of the contractions: about sqrt(P n0) rows (a multiple of 256), which
// balances the chunk of B_comb (S rows entries) against the per-chunk partial
// sums (S n0 P / rows entries), and at most 2^28 / S rows
int sp_rows(int P, int n0, size_t systems) {
    size_t rows = (size_t)std::ceil(std::sqrt((double)P * n0) / 256.0) * 256;
    const size_t cap = std::max<size_t>(256, (((size_t)1 << 28) / std::max<size_t>(systems, 1)) / 256 * 256);
    rows = std::min(std::max<size_t>(rows, 256), cap);
    return (int)std::min<size_t>(rows, (size_t)P);
}

int sp_ensure(cosim_sp *p, int B) {
    if ((size_t)B <= p->cap) return COSIM_OK;
    dfree(p->w.X);
    dfree(p->w.Xg);
    dfree(p->w.Y);
    dfree(p->w.Rp);
    dfree(p->w.lpart);
    p->cap = 0;
    const size_t S = (size_t)B * p->d.F, n0 = (size_t)p->d.n0;
    const int rows = sp_rows(p->d.P, p->d.n0, S);
    const int nchunk = (p->d.P + rows - 1) / rows;
    if (hipMalloc((void **)&p->w.X, S * n0 * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->w.Xg, S * n0 * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->w.Y, S * (size_t)rows * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->w.Rp, (size_t)nchunk * S * n0 * sizeof(double2)) != hipSuccess ||
        hipMalloc((void **)&p->w.lpart, (size_t)nchunk * S * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(COSIM_ENOMEM, "S-parameter workspace for %d configurations failed", B);
    }
    p->w.B = B;
    p->w.rows = rows;
    p->w.nchunk = nchunk;
    p->cap = (size_t)B;
    return COSIM_OK;
}

}  // namespace

extern "C" {

int cosim_sp_create(int n0, int n1, int F, int P, int ncomp, const double *S0_d,
                    const double *fields_d, const double *sc_const_d, int nvar,
                    const int32_t *idx_x, const int32_t *idx_y, const double *exc,
                    int precisions, void *stream, cosim_sp_t *out) {
    if (!out) return fail(COSIM_EINVAL, "null output pointer");
    *out = nullptr;
    if (n0 < 1 || n0 > COSIM_SP_MAX_PORTS)
        return fail(COSIM_EINVAL, "n0 = %d outside 1..%d", n0, (int)COSIM_SP_MAX_PORTS);
    if (n1 < 1 || n1 > COSIM_SP_MAX_EXTERNAL)
        return fail(COSIM_EINVAL, "n1 = %d outside 1..%d", n1, (int)COSIM_SP_MAX_EXTERNAL);
    if (F < 1 || P < 1) return fail(COSIM_EINVAL, "F = %d, P = %d (both must be >= 1)", F, P);
    if (ncomp < 1 || ncomp > 3) return fail(COSIM_EINVAL, "ncomp = %d outside 1..3", ncomp);
    if (!S0_d || !fields_d) return fail(COSIM_EINVAL, "null S0 or field pointer");
    if (nvar < 0 || (nvar > 0 && (!idx_x || !idx_y)))
        return fail(COSIM_EINVAL, "nvar = %d with null index arrays", nvar);
    if (!exc) return fail(COSIM_EINVAL, "null drive waves");
    if (precisions & (1 << COSIM_BF16X3))
        return fail(COSIM_EUNSUPPORTED, "BF16X3 contractions are not offered for S-parameter plans");
    if (precisions & ~((1 << COSIM_FP64) | (1 << COSIM_FP32)) || precisions == 0)
        return fail(COSIM_EINVAL, "precision mask %d", precisions);
    const int N = n0 + n1;
    for (int e = 0; e < nvar; ++e)
        if (idx_x[e] < 0 || idx_x[e] >= N || idx_y[e] < 0 || idx_y[e] >= N)
            return fail(COSIM_EINVAL, "index pair %d = (%d, %d) outside the %d x %d network", e,
                        idx_x[e], idx_y[e], N, N);
    if ((size_t)F * P * ncomp * n0 > ((size_t)1 << 31))
        return fail(COSIM_EUNSUPPORTED, "field tensor of %zu entries per plan exceeds 2^31",
                    (size_t)F * P * ncomp * n0);
    cosim_sp *p = new (std::nothrow) cosim_sp;
    if (!p) return fail(COSIM_ENOMEM, "host allocation failed");
    auto cleanup = [&](int code) {
        if (code != COSIM_OK) delete p;
        return code;
    };
#define SP_TRY(x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            (void)hipGetLastError();                                                        \
            return cleanup(fail(e_ == hipErrorOutOfMemory ? COSIM_ENOMEM : COSIM_EDEVICE,   \
                                "%s failed: %s", #x, hipGetErrorString(e_)));               \
        }                                                                                   \
    } while (0)
    hipStream_t st = (hipStream_t)stream;
    SP_TRY(hipGetDevice(&p->device));
    std::call_once(g_sp_lds_once, [] { g_sp_lds_err = sp_set_lds_limit(); });
    SP_TRY(g_sp_lds_err);
    p->N = N;
    p->prec_mask = precisions;
    SpDev &d = p->d;
    d.n0 = n0;
    d.n1 = n1;
    d.F = F;
    d.P = P;
    d.ncomp = ncomp;
    d.nvar = nvar;
    p->ix.assign(idx_x, idx_x + nvar);
    p->iy.assign(idx_y, idx_y + nvar);
    const size_t nf = (size_t)F * P * ncomp * n0;
    SP_TRY(hipMalloc((void **)&d.S0, (size_t)F * n0 * n0 * sizeof(double2)));
    SP_TRY(hipMalloc((void **)&d.K, (size_t)F * n0 * n0 * sizeof(double2)));
    SP_TRY(hipMalloc((void **)&d.r0, (size_t)F * n0 * sizeof(double2)));
    SP_TRY(hipMalloc((void **)&d.exc, (size_t)n1 * sizeof(double2)));
    SP_TRY(hipMalloc((void **)&d.ix, std::max(nvar, 1) * sizeof(int)));
    SP_TRY(hipMalloc((void **)&d.iy, std::max(nvar, 1) * sizeof(int)));
    SP_TRY(hipMalloc((void **)&d.fields64, nf * sizeof(double2)));
    if (precisions & (1 << COSIM_FP32)) SP_TRY(hipMalloc((void **)&d.fields32, nf * sizeof(float2)));
    SP_TRY(hipMemcpyAsync(d.S0, S0_d, (size_t)F * n0 * n0 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    SP_TRY(hipMemcpyAsync(d.fields64, fields_d, nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
    SP_TRY(hipMemcpyAsync(d.exc, exc, (size_t)n1 * sizeof(double2), hipMemcpyHostToDevice, st));
    if (nvar > 0) {
        SP_TRY(hipMemcpyAsync(d.ix, p->ix.data(), nvar * sizeof(int), hipMemcpyHostToDevice, st));
        SP_TRY(hipMemcpyAsync(d.iy, p->iy.data(), nvar * sizeof(int), hipMemcpyHostToDevice, st));
    }
    if (d.fields32) SP_TRY(sp_to_c64(nf, d.fields64, d.fields32, st));
    SP_TRY(sp_prep(d, (const double2 *)sc_const_d, st));
    SP_TRY(sp_blas_create(&p->blas));
    SP_TRY(hipStreamSynchronize(st));  // host index copies and the caller's inputs are done with
#undef SP_TRY
    *out = p;
    return COSIM_OK;
}

int cosim_sp_destroy(cosim_sp_t p) {
    delete p;
    return COSIM_OK;
}

int cosim_sp_reserve(cosim_sp_t p, int max_batch) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (max_batch < 0) return fail(COSIM_EINVAL, "max_batch = %d", max_batch);
    int rc = sp_check_device(p);
    if (rc != COSIM_OK) return rc;
    return sp_ensure(p, max_batch);
}

int cosim_sp_field(cosim_sp_t p, int B, const double *values_d, double *x_d, double *field_d,
                   int32_t *status_d, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (B < 0) return fail(COSIM_EINVAL, "B = %d", B);
    if (B == 0) return COSIM_OK;
    if ((p->d.nvar > 0 && !values_d) || !status_d)
        return fail(COSIM_EINVAL, "null values or status pointer");
    int rc = sp_check_device(p);
    if (rc != COSIM_OK) return rc;
    if ((rc = sp_ensure(p, B)) != COSIM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(sp_forward(p->d, B, (const double2 *)values_d, p->w.X, p->w.Xg, 0, status_d, st));
    const size_t S = (size_t)B * p->d.F;
    if (x_d)
        HIP_TRY(hipMemcpyAsync(x_d, p->w.X, S * p->d.n0 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    if (field_d) HIP_TRY(sp_field(p->blas, p->d, B, (const double2 *)p->w.Xg, (double2 *)field_d, st));
    return COSIM_OK;
}

int cosim_sp_loss_and_grad(cosim_sp_t p, int B, const double *values_d, const double *T_d,
                           int comp, int loss_mode, int precision, double *loss_d, double *grad_d,
                           int32_t *status_d, void *stream) {
    if (!p) return fail(COSIM_EINVAL, "null plan");
    if (B < 0) return fail(COSIM_EINVAL, "B = %d", B);
    if (comp < 0 || comp >= p->d.ncomp)
        return fail(COSIM_EINVAL, "component %d outside 0..%d", comp, p->d.ncomp - 1);
    if (loss_mode != COSIM_LOSS_MAG && loss_mode != COSIM_LOSS_COMPLEX)
        return fail(COSIM_EINVAL, "loss mode %d", loss_mode);
    if (precision == COSIM_BF16X3)
        return fail(COSIM_EUNSUPPORTED, "BF16X3 contractions are not offered for S-parameter plans");
    if (precision != COSIM_FP64 && precision != COSIM_FP32)
        return fail(COSIM_EINVAL, "precision %d", precision);
    if (!(p->prec_mask & (1 << precision)))
        return fail(COSIM_EINVAL, "the plan was created without precision %d", precision);
    if (B == 0) return COSIM_OK;
    if ((p->d.nvar > 0 && !values_d) || !T_d || !loss_d || !status_d)
        return fail(COSIM_EINVAL, "null values, target, loss or status pointer");
    int rc = sp_check_device(p);
    if (rc != COSIM_OK) return rc;
    if ((rc = sp_ensure(p, B)) != COSIM_OK) return rc;
    HIP_TRY(sp_loss_and_grad(p->blas, p->d, p->w, B, (const double2 *)values_d, T_d, comp, loss_mode,
                             precision == COSIM_FP64 ? 0 : 1, loss_d, (double2 *)grad_d, status_d,
                             (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_sp_rc(int B, int F, int n, const double *R_d, const double *C_d, const double *omega_d,
                double z0, double *gamma_d, int ld, void *stream) {
    if (B < 0 || F < 1 || n < 1) return fail(COSIM_EINVAL, "B = %d, F = %d, n = %d", B, F, n);
    if (ld < n) return fail(COSIM_EINVAL, "row stride %d below n = %d", ld, n);
    if (!(z0 > 0.0)) return fail(COSIM_EINVAL, "reference impedance %g", z0);
    if (B > 0 && (!R_d || !C_d || !omega_d || !gamma_d)) return fail(COSIM_EINVAL, "null pointer");
    HIP_TRY(sp_rc(B, F, n, R_d, C_d, omega_d, z0, (double2 *)gamma_d, ld, (hipStream_t)stream));
    return COSIM_OK;
}

int cosim_sp_rc_backward(int B, int F, int n, const double *R_d, const double *C_d,
                         const double *omega_d, double z0, const double *g_d, int ld, double *gC_d,
                         void *stream) {
    if (B < 0 || F < 1 || n < 1) return fail(COSIM_EINVAL, "B = %d, F = %d, n = %d", B, F, n);
    if (ld < n) return fail(COSIM_EINVAL, "row stride %d below n = %d", ld, n);
    if (!(z0 > 0.0)) return fail(COSIM_EINVAL, "reference impedance %g", z0);
    if (B > 0 && (!R_d || !C_d || !omega_d || !g_d || !gC_d)) return fail(COSIM_EINVAL, "null pointer");
    HIP_TRY(sp_rc_backward(B, F, n, R_d, C_d, omega_d, z0, (const double2 *)g_d, ld, gC_d,
                           (hipStream_t)stream));
    return COSIM_OK;
}

}  // extern "C"
