// Host side of the HOBI-PB library: the C ABI declared in hobi.h.
//
// Owns device memory and the stream, validates inputs, orders the surface spatially
// (Morton order of vertices and of triangle centroids, so that a wavefront's targets and
// a chunk's source nodes are compact in space), runs the per-molecule setup kernels,
// and drives the matvec, restarted GMRES and the energy on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hobi.h"
#include "hobi_host.h"
#include "trace.h"
#include "hobi_internal.h"

using namespace hobi;

namespace {

hobi_status fail(hobi_ctx ctx, hobi_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), e_ == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
}

// Grows a device buffer to hold at least n elements (contents are not kept).
template <class T>
hipError_t grow(T** p, size_t* cap, size_t n) {
    if (*p && *cap >= n) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t m = std::max<size_t>(n, 1);
    const hipError_t e = hipMalloc((void**)p, m * sizeof(T));
    if (e == hipSuccess) *cap = m;
    return e;
}

template <class T>
hipError_t grow_pinned(T** p, size_t* cap, size_t n) {
    if (*p && *cap >= n) return hipSuccess;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t m = std::max<size_t>(n, 1);
    const hipError_t e = hipHostMalloc((void**)p, m * sizeof(T));
    if (e == hipSuccess) *cap = m;
    return e;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

hipEvent_t take_event(hobi_problem pb) {
    if (!pb->event_pool.empty()) {
        hipEvent_t e = pb->event_pool.back();
        pb->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ScopedTimer {
    hobi_problem pb;
    Timer t{};
    bool on;
    ScopedTimer(hobi_problem p, int kind) : pb(p), on(p->ctx->profile) {
        if (!on) return;
        t.a = take_event(pb);
        t.b = take_event(pb);
        t.kind = kind;
        if (!t.a || !t.b) { on = false; return; }
        (void)hipEventRecord(t.a, pb->ctx->stream);
    }
    ~ScopedTimer() {
        if (!on) return;
        (void)hipEventRecord(t.b, pb->ctx->stream);
        pb->pending.push_back(t);
    }
};

hobi_status resolve_timers(hobi_problem pb) {
    if (pb->pending.empty()) return HOBI_OK;
    HIPCHK(pb->ctx, hipStreamSynchronize(pb->ctx->stream));
    for (const Timer& t : pb->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            pb->ms[t.kind] += ms;
            pb->cnt[t.kind] += 1;
        }
        pb->event_pool.push_back(t.a);
        pb->event_pool.push_back(t.b);
    }
    pb->pending.clear();
    return HOBI_OK;
}

// y = A u, both in internal order on the device: the treecode's operator when the problem
// has one, unless `dense`.
hobi_status matvec_internal(hobi_problem pb, const double* u, double* y, bool dense = false) {
    hipStream_t s = pb->ctx->stream;
    const bool mixed = pb->prm.precision == HOBI_MIXED;
    {
        ScopedTimer t(pb, T_GATHER);
        HIPCHK(pb->ctx, launch_gather(pb->d, u, mixed, s));
    }
    if (pb->d.tree.on && !dense) {
        {
            ScopedTimer t(pb, T_PAIR);
            HIPCHK(pb->ctx, launch_tree_proxies(pb->d, mixed, s));
            HIPCHK(pb->ctx, launch_tree_pairs(pb->d, mixed, s));
        }
        {
            ScopedTimer t(pb, T_COMBINE);
            HIPCHK(pb->ctx, launch_tree_combine(pb->d, u, y, mixed, s));
        }
        return HOBI_OK;
    }
    {
        ScopedTimer t(pb, T_PAIR);
        HIPCHK(pb->ctx, launch_pair(pb->d, mixed, s));
    }
    {
        ScopedTimer t(pb, T_COMBINE);
        HIPCHK(pb->ctx, launch_combine(pb->d, u, y, mixed, s));
    }
    return HOBI_OK;
}

void free_krylov(Krylov& k) {
    double* ptrs[] = {k.V, k.H, k.cs, k.sn, k.g, k.h1, k.h2, k.hn, k.yk, k.res, k.dpart, k.x, k.tmp, k.scal, k.xo, k.ro};
    for (double* p : ptrs)
        if (p) (void)hipFree(p);
    k = Krylov{};
}

hobi_status ensure_krylov(hobi_problem pb, int n, int m) {
    Krylov& k = pb->kr;
    if (k.n == n && k.m == m) return HOBI_OK;
    free_krylov(k);
    hobi_ctx c = pb->ctx;
    HIPCHK(c, dalloc(&k.V, (size_t)(m + 1) * n));
    HIPCHK(c, dalloc(&k.H, (size_t)(m + 1) * m));
    HIPCHK(c, dalloc(&k.cs, m));
    HIPCHK(c, dalloc(&k.sn, m));
    HIPCHK(c, dalloc(&k.g, m + 1));
    HIPCHK(c, dalloc(&k.h1, m + 1));
    HIPCHK(c, dalloc(&k.h2, m + 1));
    HIPCHK(c, dalloc(&k.hn, 1));
    HIPCHK(c, dalloc(&k.yk, m));
    HIPCHK(c, dalloc(&k.res, 1));
    HIPCHK(c, dalloc(&k.dpart, (size_t)kDotBlocks * (m + 1)));
    HIPCHK(c, dalloc(&k.x, n));
    HIPCHK(c, dalloc(&k.tmp, n));
    HIPCHK(c, dalloc(&k.scal, 4));
    if (pb->prm.tree_refine) {
        HIPCHK(c, dalloc(&k.xo, n));
        HIPCHK(c, dalloc(&k.ro, n));
    }
    k.n = n;
    k.m = m;
    return HOBI_OK;
}

hobi_status read_scalar(hobi_problem pb, const double* dev, double* out) {
    HIPCHK(pb->ctx, hipMemcpyAsync(pb->host_pinned, dev, sizeof(double), hipMemcpyDeviceToHost,
                                   pb->ctx->stream));
    HIPCHK(pb->ctx, hipStreamSynchronize(pb->ctx->stream));
    *out = pb->host_pinned[0];
    return HOBI_OK;
}

hobi_status norm2(hobi_problem pb, const double* v, int n, double* dev_out) {
    hipStream_t s = pb->ctx->stream;
    HIPCHK(pb->ctx, launch_dots(v, 0, 1, v, n, pb->kr.dpart, s));
    HIPCHK(pb->ctx, launch_reduce(pb->kr.dpart, 1, dev_out, 1, s));
    return HOBI_OK;
}

// Restarted GMRES(m) from x0 = 0 on A x = rhs (internal order), A the problem's operator
// (the treecode's when it has one), at most max_iter matvecs.  With `scaled` it is
// right-preconditioned by the diagonal D whose inverse launch_scaling left in d.dinv (the
// row blocks' constants, diag_scaling 1, or A's own diagonal, 2): the Krylov space is that
// of A D^-1 and the iterate is x = D^-1 y, so the residual it estimates is that of
// A x = rhs.  Classical Gram-Schmidt with a second pass, Givens rotations; stops when the
// estimate |g_{k+1}| / ||rhs|| <= rtol.  The iterate is left in k.x (ensure_krylov first).
hobi_status gmres_run(hobi_problem pb, const double* rhs, double rtol, int max_iter, bool scaled, int* iters,
                      double* est, bool* converged) {
    const int n = 2 * pb->d.nv;
    const int m = pb->kr.m;
    hobi_status st = HOBI_OK;
    Krylov& k = pb->kr;
    hipStream_t s = pb->ctx->stream;
    hobi_ctx c = pb->ctx;
    const double* b = rhs;
    HIPCHK(c, hipMemsetAsync(k.x, 0, sizeof(double) * n, s));
    if ((st = norm2(pb, b, n, k.scal)) != HOBI_OK) return st;
    double bnorm = 0;
    if ((st = read_scalar(pb, k.scal, &bnorm)) != HOBI_OK) return st;
    *iters = 0;
    *est = 0.0;
    *converged = true;
    if (!(bnorm > 0.0)) return std::isfinite(bnorm) ? HOBI_OK : fail(c, HOBI_E_NUMERIC, "non-finite rhs");
    int total = 0;
    while (true) {
        // r = b - A x
        const double* r = b;
        if (total > 0) {
            if ((st = matvec_internal(pb, k.x, k.tmp)) != HOBI_OK) return st;
            HIPCHK(c, launch_sub(b, k.tmp, k.tmp, n, s));
            r = k.tmp;
        }
        if ((st = norm2(pb, r, n, k.scal + 1)) != HOBI_OK) return st;
        double beta = 0;
        if ((st = read_scalar(pb, k.scal + 1, &beta)) != HOBI_OK) return st;
        if (!std::isfinite(beta)) return fail(c, HOBI_E_NUMERIC, "GMRES residual is not finite");
        *est = beta / bnorm;
        if (*est <= rtol || total >= max_iter) break;
        HIPCHK(c, launch_scale_copy(r, k.scal + 1, k.V, n, s));
        HIPCHK(c, launch_init_g(k.scal + 1, k.g, m, s));
        int kk = 0;
        bool stop = false;
        for (int j = 0; j < m; ++j) {
            double* w = k.V + (size_t)(j + 1) * n;
            const double* vj = k.V + (size_t)j * n;
            if (scaled) {
                HIPCHK(c, launch_diag_scale(vj, k.tmp, n, pb->d.dinv, s));
                vj = k.tmp;
            }
            if ((st = matvec_internal(pb, vj, w)) != HOBI_OK) return st;
            ++total;
            {
                ScopedTimer t(pb, T_KRYLOV);
                for (int pass = 0; pass < 2; ++pass) {
                    double* h = pass == 0 ? k.h1 : k.h2;
                    HIPCHK(c, launch_dots(k.V, n, j + 1, w, n, k.dpart, s));
                    HIPCHK(c, launch_reduce(k.dpart, j + 1, h, 0, s));
                    HIPCHK(c, launch_multi_axpy(k.V, n, j + 1, h, -1.0, w, n, s));
                }
                if ((st = norm2(pb, w, n, k.hn)) != HOBI_OK) return st;
                HIPCHK(c, launch_scale_copy(w, k.hn, w, n, s));
                HIPCHK(c, launch_givens(k.H, m + 1, j, k.h1, k.h2, k.hn, k.cs, k.sn, k.g, bnorm, k.res, s));
            }
            double res = 0;
            if ((st = read_scalar(pb, k.res, &res)) != HOBI_OK) return st;
            if (!std::isfinite(res)) return fail(c, HOBI_E_NUMERIC, "GMRES residual is not finite");
            *est = res;
            kk = j + 1;
            if (res <= rtol || total >= max_iter) {
                stop = true;
                break;
            }
        }
        HIPCHK(c, launch_trisolve(k.H, m + 1, kk, k.g, k.yk, s));
        if (scaled)
            HIPCHK(c, launch_multi_axpy_scaled(k.V, n, kk, k.yk, k.x, n, pb->d.dinv, s));
        else
            HIPCHK(c, launch_multi_axpy(k.V, n, kk, k.yk, 1.0, k.x, n, s));
        if (stop) break;
    }
    *iters = total;
    *converged = *est <= rtol;
    return HOBI_OK;
}

// tree_refine: the dense system A x = b by defect correction with the treecode operator T
// (iterative refinement with an approximate operator): from x = 0, each outer step solves
// T d = r by gmres_run, then x += d and r = b - A x with the dense matvec.  The first step
// solves to 100 rtol (at most 1/10): the dense residual after it is bounded by the
// treecode's own error anyway, and GMRES converges about linearly, so solving further there
// only moves iterations from the second step to the first.  Later steps solve to
// max(rtol/2 ||b|| / ||r||, rtol/2), at most 1/2, so that with T = A the next residual would
// be at most rtol/2 ||b||.  A step that shrinks ||r|| by less than a tenth ends the solve
// (the treecode is too far from A).  Stops as the ABI states; x is left in k.x and the last
// dense residual b - A x in k.ro.
hobi_status gmres_refined(hobi_problem pb, bool scaled, int* iters, double* est, bool* converged, int* steps,
                          int* dense_mv) {
    const int n = 2 * pb->d.nv;
    Krylov& k = pb->kr;
    hipStream_t s = pb->ctx->stream;
    hobi_ctx c = pb->ctx;
    const double* b = pb->d.rhs;
    const double rtol = pb->prm.rtol;
    const int max_iter = pb->prm.max_iter;
    hobi_status st = HOBI_OK;
    *iters = 0;
    *est = 0.0;
    *converged = true;
    *steps = 0;
    *dense_mv = 0;
    HIPCHK(c, hipMemsetAsync(k.xo, 0, sizeof(double) * n, s));
    HIPCHK(c, hipMemcpyAsync(k.ro, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if ((st = norm2(pb, b, n, k.scal + 2)) != HOBI_OK) return st;
    double bnorm = 0;
    if ((st = read_scalar(pb, k.scal + 2, &bnorm)) != HOBI_OK) return st;
    if (!std::isfinite(bnorm)) return fail(c, HOBI_E_NUMERIC, "non-finite rhs");
    if (bnorm > 0.0) {
        double rnorm = bnorm;
        int total = 0;
        while (true) {
            const double tol = *steps == 0 ? std::min(0.1, std::max(100.0 * rtol, 0.5 * rtol))
                                           : std::min(0.5, std::max(0.5 * rtol * bnorm / rnorm, 0.5 * rtol));
            int it = 0;
            double e_in = 0;
            bool c_in = false;
            if ((st = gmres_run(pb, k.ro, tol, max_iter - total, scaled, &it, &e_in, &c_in)) != HOBI_OK) return st;
            total += it;
            HIPCHK(c, launch_add(k.xo, k.x, k.xo, n, s));
            if ((st = matvec_internal(pb, k.xo, k.tmp, true)) != HOBI_OK) return st;
            HIPCHK(c, launch_sub(b, k.tmp, k.ro, n, s));
            ++*steps;
            ++*dense_mv;
            if ((st = norm2(pb, k.ro, n, k.scal + 2)) != HOBI_OK) return st;
            double rn = 0;
            if ((st = read_scalar(pb, k.scal + 2, &rn)) != HOBI_OK) return st;
            if (!std::isfinite(rn)) return fail(c, HOBI_E_NUMERIC, "refinement residual is not finite");
            *est = rn / bnorm;
            *iters = total;
            if (*est <= rtol || total >= max_iter || *steps >= kMaxRefineSteps || rn > 0.9 * rnorm) break;
            rnorm = rn;
        }
    }
    HIPCHK(c, hipMemcpyAsync(k.x, k.xo, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    *converged = *est <= rtol;
    return HOBI_OK;
}

// The solve's Krylov driver: GMRES on the problem's operator, or the defect correction of
// tree_refine.  refine_steps and dense_mv are 0 without it.
hobi_status gmres(hobi_problem pb, int* iters, double* est, bool* converged, int* refine_steps, int* dense_mv) {
    TraceRange trace_range("gmres");
    const int n = 2 * pb->d.nv;
    const int m = std::max(1, std::min(pb->prm.restart, pb->prm.max_iter));
    hobi_status st = ensure_krylov(pb, n, m);
    if (st != HOBI_OK) return st;
    const bool scaled = pb->prm.diag_scaling != 0;
    if (scaled) HIPCHK(pb->ctx, launch_scaling(pb->d, pb->prm.diag_scaling, pb->d.dinv, pb->ctx->stream));
    *refine_steps = 0;
    *dense_mv = 0;
    if (pb->prm.tree_refine && pb->d.tree.on) return gmres_refined(pb, scaled, iters, est, converged, refine_steps, dense_mv);
    return gmres_run(pb, pb->d.rhs, pb->prm.rtol, pb->prm.max_iter, scaled, iters, est, converged);
}

hobi_status to_internal(hobi_problem pb, const double* u, int on_device, double* dst) {
    const int nv = pb->d.nv;
    hipStream_t s = pb->ctx->stream;
    if (on_device) {
        HIPCHK(pb->ctx, launch_permute(u, dst, pb->d_vperm, nv, true, s));
    } else {
        std::vector<double> h(2 * (size_t)nv);
        for (int i = 0; i < nv; ++i) {
            h[i] = u[pb->vperm[i]];
            h[nv + i] = u[nv + pb->vperm[i]];
        }
        HIPCHK(pb->ctx, hipMemcpyAsync(dst, h.data(), sizeof(double) * 2 * nv, hipMemcpyHostToDevice, s));
        HIPCHK(pb->ctx, hipStreamSynchronize(s));
    }
    return HOBI_OK;
}

hobi_status from_internal(hobi_problem pb, const double* src, int on_device, double* y) {
    const int nv = pb->d.nv;
    hipStream_t s = pb->ctx->stream;
    if (on_device) {
        HIPCHK(pb->ctx, launch_permute(src, y, pb->d_vperm, nv, false, s));
    } else {
        std::vector<double> h(2 * (size_t)nv);
        HIPCHK(pb->ctx, hipMemcpyAsync(h.data(), src, sizeof(double) * 2 * nv, hipMemcpyDeviceToHost, s));
        HIPCHK(pb->ctx, hipStreamSynchronize(s));
        for (int i = 0; i < nv; ++i) {
            y[pb->vperm[i]] = h[i];
            y[nv + pb->vperm[i]] = h[nv + i];
        }
    }
    return HOBI_OK;
}

void free_problem(hobi_problem pb) {
    DeviceProblem& d = pb->d;
    void* ptrs[] = {d.xyz, d.nrm, d.vxyz, d.tri, d.qpos, d.q, d.qsoa, d.patch, d.node64, d.node32, d.node_vid,
                    d.blk_range, d.w,
                    d.tgt64, d.tgt32, d.inc_off, d.inc_ent, d.coef, d.rhs, d.dinv, d.partial, d.plan_tab,
                    pb->d_vperm, pb->u_in, pb->y_out, pb->phi_reac, pb->e_dev, pb->d_err};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    free_krylov(pb->kr);
    {
        TreePlan& t = d.tree;
        void* tp[] = {t.clu_range, t.clu_child, t.clu_box, t.prox64, t.prox32, t.items[0], t.items[1],
                      t.slot_row[0], t.slot_row[1], t.partial};
        for (void* p : tp)
            if (p) (void)hipFree(p);
        t = TreePlan{};
    }
    {
        FieldWork& f = pb->field;
        void* fp[] = {f.pts64, f.pts32, f.partial, f.gstart, f.out, f.inside, f.items, f.slot_row, f.order, f.outc,
                      f.insc, f.raw, f.keys, f.idx, f.sort_tmp, f.bbox};
        for (void* p : fp)
            if (p) (void)hipFree(p);
        if (f.hbox) (void)hipHostFree(f.hbox);
        f = FieldWork{};
    }
    if (pb->host_pinned) (void)hipHostFree(pb->host_pinned);
    for (const Timer& t : pb->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : pb->event_pool) (void)hipEventDestroy(e);
}

// Device part of the per-molecule setup on the resident inputs; returns the elapsed ms.
hobi_status run_device_setup(hobi_problem pb, float* ms_out) {
    hipStream_t s = pb->ctx->stream;
    DeviceProblem& d = pb->d;
    hipEvent_t e0 = take_event(pb), e1 = take_event(pb);
    d.s32 = d.kappa > 0 ? d.kappa : 1.0;
    if (e0) (void)hipEventRecord(e0, s);
    if (d.method == HOBI_LOWER_ORDER) {
        HIPCHK(pb->ctx, launch_lobi_nodes(d, s));
        HIPCHK(pb->ctx, launch_targets(d, s));
        HIPCHK(pb->ctx, launch_sources(d, s));
    } else {
        HIPCHK(pb->ctx, launch_patch(d, pb->d_err, s));
        HIPCHK(pb->ctx, launch_regular_nodes(d, s));
        HIPCHK(pb->ctx, launch_targets(d, s));
        HIPCHK(pb->ctx, launch_singular(d, s));
        HIPCHK(pb->ctx, launch_sources(d, s));
    }
    if (e1) (void)hipEventRecord(e1, s);
    HIPCHK(pb->ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    if (e0 && e1) (void)hipEventElapsedTime(&ms, e0, e1);
    if (e0) pb->event_pool.push_back(e0);
    if (e1) pb->event_pool.push_back(e1);
    *ms_out = ms;
    return HOBI_OK;
}

// The treecode's partition (hobi_params.tree_theta > 0), from the node and target positions
// in internal order.  Leaves: runs of tree_leaf consecutive nodes; parents: neighbours
// joined pairwise level by level (a last cluster without a neighbour moves up unchanged),
// stored after the leaves level by level.  Each cluster and batch (tree_batch consecutive
// targets) has the bounding sphere of its box (centre, half diagonal); a cluster's
// vertex-id range is that of its triangles (higher-order method) or its own node range
// (lower-order method: a centroid's node is left out of its own row only).  Each batch walks the tree from the root:
// accepted (far) when r_b + r_c <= theta |c_b - c_c| and the cluster's vertex-id range
// misses the batch's targets, else a leaf is near and a parent is opened (left child
// first).  Work items: for every target slot of each precision, its batch's far and near
// clusters in walk order.
// Device bytes of a treecode plan's buffers (the allocations below).
int64_t tree_plan_bytes(const TreeHostPlan& hp, int nprox, int nv) {
    int64_t b = (int64_t)hp.nclu * (2 * (int64_t)sizeof(int2) + 6 * (int64_t)sizeof(double)) +
                (int64_t)hp.nclu * nprox * (int64_t)(sizeof(ProxyD) + sizeof(ProxyF));
    for (int m = 0; m < 2; ++m)
        b += (int64_t)hp.nitems[m] * (int64_t)sizeof(int4) + 4LL * ((nv + hp.slot[m] - 1) / hp.slot[m] + 1);
    return b + 8 * (int64_t)hp.partial_elems;
}

// The treecode partition and its device buffers.  Fails with HOBI_E_OOM, and the buffers'
// size in *need, when they would take more than `limit` bytes.
hobi_status build_tree_plan(hobi_problem pb, int64_t limit, int64_t* need) {
    TraceRange trace_range("treecode plan");
    DeviceProblem& d = pb->d;
    TreePlan& t = d.tree;
    const hobi_params& prm = pb->prm;
    if (!(prm.tree_theta > 0)) return HOBI_OK;
    hobi_ctx ctx = pb->ctx;
    hipStream_t s = ctx->stream;
    const int nn = d.nn, nv = d.nv, nf = d.nf;
    std::vector<NodeD> nodes(nn);
    std::vector<double> tg(3 * (size_t)d.nv_pad);
    std::vector<int> tri(3 * (size_t)nf);
    HIPCHK(ctx, hipMemcpyAsync(nodes.data(), d.node64, sizeof(NodeD) * nn, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(tg.data(), d.tgt64, sizeof(double) * tg.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(tri.data(), d.tri, sizeof(int) * tri.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    t.degree = prm.tree_degree;
    t.nprox = (t.degree + 1) * (t.degree + 1) * (t.degree + 1);
    t.leaf = prm.tree_leaf;
    t.batch = prm.tree_batch;
    std::vector<double> nxyz(3 * (size_t)nn);
    for (int j = 0; j < nn; ++j) nxyz[3 * (size_t)j] = nodes[j].x, nxyz[3 * (size_t)j + 1] = nodes[j].y,
                                 nxyz[3 * (size_t)j + 2] = nodes[j].z;
    TreeHostPlan hp;
    std::string msg;
    if (!plan_tree(nn, nxyz.data(), nv, tg.data(), (size_t)d.nv_pad, nf, tri.data(),
                   d.method == HOBI_LOWER_ORDER ? 1 : 0, prm.tree_theta, t.leaf, t.batch, kTreeTpl64, &hp, &msg))
        return fail(ctx, HOBI_E_ARG, "%s", msg.c_str());
    const int64_t bytes = tree_plan_bytes(hp, t.nprox, nv);
    if (bytes > limit) {
        if (need) *need = bytes;
        return fail(ctx, HOBI_E_OOM, "treecode buffers (%lld bytes) exceed the %lld bytes allowed", (long long)bytes,
                    (long long)limit);
    }
    t.nleaf = hp.nleaf;
    t.nbatch = hp.nbatch;
    t.nlev = hp.nlev;
    std::copy(hp.lev_off, hp.lev_off + kTreeMaxLevels + 1, t.lev_off);
    t.root = hp.root;
    t.nclu = hp.nclu;
    t.nfar = hp.nfar;
    t.nnear = hp.nnear;
    t.h_cen = hp.ccen;
    t.h_rad = hp.crad;
    t.h_child.resize(t.nclu);
    for (int c = 0; c < t.nclu; ++c) t.h_child[c] = make_int2(hp.cchild[2 * (size_t)c], hp.cchild[2 * (size_t)c + 1]);
    for (int m = 0; m < 2; ++m) {
        t.tpl[m] = hp.tpl[m];
        t.slot[m] = hp.slot[m];
        t.nitems[m] = hp.nitems[m];
    }
    static_assert(sizeof(int2) == 2 * sizeof(int) && sizeof(int4) == 4 * sizeof(int), "packed index records");
    const std::vector<int>* items = hp.items;
    const std::vector<int>* srow = hp.slot_row;
    const size_t partial_elems = hp.partial_elems;
    const std::vector<int>& crange = hp.crange;
    const std::vector<int>& cchild = hp.cchild;
    const std::vector<double>& cbox = hp.cbox;
    HIPCHK(ctx, dalloc(&t.clu_range, t.nclu));
    HIPCHK(ctx, dalloc(&t.clu_child, t.nclu));
    HIPCHK(ctx, dalloc(&t.clu_box, 6 * (size_t)t.nclu));
    HIPCHK(ctx, dalloc(&t.prox64, (size_t)t.nclu * t.nprox));
    HIPCHK(ctx, dalloc(&t.prox32, (size_t)t.nclu * t.nprox));
    for (int m = 0; m < 2; ++m) {
        HIPCHK(ctx, dalloc(&t.items[m], items[m].size() / 4));
        HIPCHK(ctx, dalloc(&t.slot_row[m], srow[m].size()));
    }
    HIPCHK(ctx, dalloc(&t.partial, partial_elems));
    HIPCHK(ctx, hipMemcpyAsync(t.clu_range, crange.data(), sizeof(int) * crange.size(), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(t.clu_child, cchild.data(), sizeof(int) * cchild.size(), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(t.clu_box, cbox.data(), sizeof(double) * cbox.size(), hipMemcpyHostToDevice, s));
    for (int m = 0; m < 2; ++m) {
        HIPCHK(ctx, hipMemcpyAsync(t.items[m], items[m].data(), sizeof(int) * items[m].size(),
                                   hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyAsync(t.slot_row[m], srow[m].data(), sizeof(int) * srow[m].size(),
                                   hipMemcpyHostToDevice, s));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    t.on = 1;
    return HOBI_OK;
}

bool finite_all(const double* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

hobi_status validate_params(hobi_ctx ctx, const hobi_params& p) {
    if (!(p.eps1 > 0) || !(p.eps2 > 0) || !std::isfinite(p.eps1) || !std::isfinite(p.eps2))
        return fail(ctx, HOBI_E_ARG, "eps1 and eps2 must be positive and finite");
    if (!(p.kappa >= 0) || !std::isfinite(p.kappa)) return fail(ctx, HOBI_E_ARG, "kappa must be >= 0");
    if (!(p.rtol >= 0) || !std::isfinite(p.rtol)) return fail(ctx, HOBI_E_ARG, "rtol must be >= 0");
    if (p.max_iter < 1 || p.restart < 1) return fail(ctx, HOBI_E_ARG, "max_iter and restart must be >= 1");
    if (p.precision != HOBI_FP64 && p.precision != HOBI_MIXED)
        return fail(ctx, HOBI_E_ARG, "precision must be HOBI_FP64 or HOBI_MIXED");
    if (p.method != HOBI_HIGHER_ORDER && p.method != HOBI_LOWER_ORDER)
        return fail(ctx, HOBI_E_ARG, "method must be HOBI_HIGHER_ORDER or HOBI_LOWER_ORDER");
    if (p.diag_scaling < 0 || p.diag_scaling > 2) return fail(ctx, HOBI_E_ARG, "diag_scaling must be 0, 1 or 2");
    if (!(p.tree_theta >= 0) || !std::isfinite(p.tree_theta)) return fail(ctx, HOBI_E_ARG, "tree_theta must be >= 0");
    if (p.tree_degree < 1 || p.tree_degree > kTreeMaxDeg)
        return fail(ctx, HOBI_E_ARG, "tree_degree must be in 1..%d", kTreeMaxDeg);
    if (p.tree_leaf < 64 || p.tree_leaf > (1 << 24) || p.tree_leaf % 64 != 0)
        return fail(ctx, HOBI_E_ARG, "tree_leaf must be a multiple of 64 in [64, 2^24]");
    if (p.tree_batch != 128 && p.tree_batch != 256 && p.tree_batch != 512)
        return fail(ctx, HOBI_E_ARG, "tree_batch must be 128, 256 or 512");
    if (p.tree_refine != 0 && p.tree_refine != 1) return fail(ctx, HOBI_E_ARG, "tree_refine must be 0 or 1");
    if (p.tree_refine == 1 && !(p.tree_theta > 0))
        return fail(ctx, HOBI_E_ARG, "tree_refine needs the treecode (tree_theta > 0)");
    return HOBI_OK;
}

// Mesh validation (check_mesh of host_logic.cpp) with its message on the context.
hobi_status validate_mesh(hobi_ctx ctx, int nv, const double* xyz, std::vector<double>& nrm, int nf,
                          const int32_t* tri) {
    std::string msg;
    if (!check_mesh(nv, xyz, nrm, nf, tri, &msg)) return fail(ctx, HOBI_E_MESH, "%s", msg.c_str());
    return HOBI_OK;
}

}  // namespace

namespace hobi {

hobi_status host_from_internal(hobi_problem pb, const double* src, int on_device, double* y) {
    return from_internal(pb, src, on_device, y);
}

hobi_status host_fail(hobi_ctx ctx, hobi_status code, const char* msg) { return fail(ctx, code, "%s", msg); }

}  // namespace hobi

// ======================================================================= C ABI ======

extern "C" {

void hobi_params_default(hobi_params* p) {
    if (!p) return;
    p->eps1 = 1.0;
    p->eps2 = 80.0;
    p->kappa = 0.1257;
    p->rtol = 1e-6;
    p->max_iter = 200;
    p->restart = 200;
    p->precision = HOBI_FP64;
    p->method = HOBI_HIGHER_ORDER;
    p->diag_scaling = 2;
    p->tree_theta = 0.0;
    p->tree_degree = 5;
    p->tree_leaf = 256;
    p->tree_batch = 128;
    p->tree_refine = 0;
}

hobi_status hobi_ctx_create(int device, void* stream, hobi_ctx* out) {
    if (!out) return HOBI_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return HOBI_E_HIP;
    if (device < 0 || device >= ndev) return HOBI_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return HOBI_E_HIP;
    void* scratch = nullptr;
    if (hobi::static_scratch_address(device, &scratch) != hipSuccess) return HOBI_E_HIP;
    hobi_ctx c = new hobi_ctx_s();
    c->device = device;
    c->scratch = scratch;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return HOBI_E_HIP;
        }
        c->own_stream = true;
    }
    *out = c;
    return HOBI_OK;
}

void hobi_ctx_destroy(hobi_ctx ctx) {
    if (!ctx) return;
    if (ctx->own_stream && ctx->stream) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

const char* hobi_last_error(hobi_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hobi_status hobi_ctx_set_profiling(hobi_ctx ctx, int32_t enable) {
    if (!ctx) return HOBI_E_ARG;
    ctx->profile = enable != 0;
    return HOBI_OK;
}

void* hobi_ctx_stream(hobi_ctx ctx) { return ctx ? (void*)ctx->stream : nullptr; }

hobi_status hobi_problem_create(hobi_ctx ctx, int32_t nv, const double* xyz, const double* nrm_in,
                                int32_t nf, const int32_t* tri_in, int32_t nc, const double* qpos,
                                const double* q, const hobi_params* params, hobi_problem* out) {
    return hobi::problem_create_limited(ctx, nv, xyz, nrm_in, nf, tri_in, nc, qpos, q, params, out, INT64_MAX,
                                        nullptr);
}

}  // extern "C"

namespace hobi {

hobi_status problem_create_limited(hobi_ctx ctx, int32_t nv, const double* xyz, const double* nrm_in, int32_t nf,
                                   const int32_t* tri_in, int32_t nc, const double* qpos, const double* q,
                                   const hobi_params* params, hobi_problem* out, int64_t tree_limit,
                                   int64_t* tree_need) {
    TraceRange trace_range("hobi_problem_create");
    if (tree_need) *tree_need = 0;
    if (!ctx) return HOBI_E_ARG;
    if (!out) return fail(ctx, HOBI_E_ARG, "out is NULL");
    *out = nullptr;
    if (!xyz || !nrm_in || !tri_in || !qpos || !q) return fail(ctx, HOBI_E_ARG, "NULL input array");
    if (nv < 4 || nf < 4 || nc < 1) return fail(ctx, HOBI_E_ARG, "need nv >= 4, nf >= 4, nc >= 1");
    if ((int64_t)nf * 4 > (int64_t)0x7fffffff / 4) return fail(ctx, HOBI_E_ARG, "nf too large");
    hobi_params prm;
    hobi_params_default(&prm);
    if (params) prm = *params;
    hobi_status st = validate_params(ctx, prm);
    if (st != HOBI_OK) return st;
    if (!finite_all(xyz, 3 * (size_t)nv) || !finite_all(nrm_in, 3 * (size_t)nv) ||
        !finite_all(qpos, 3 * (size_t)nc) || !finite_all(q, nc))
        return fail(ctx, HOBI_E_NUMERIC, "non-finite input");
    std::vector<double> nrm(nrm_in, nrm_in + 3 * (size_t)nv);
    if ((st = validate_mesh(ctx, nv, xyz, nrm, nf, tri_in)) != HOBI_OK) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));

    // ---- spatial order ----
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], xyz[3 * i + d]);
            hi[d] = std::max(hi[d], xyz[3 * i + d]);
        }
    const double extent = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                    (hi[2] - lo[2]) * (hi[2] - lo[2]));
    if (!(prm.kappa * 2.0 * extent < kExpTabMaxZ))
        return fail(ctx, HOBI_E_ARG, "kappa times the surface's extent must stay below %g", kExpTabMaxZ / 2);
    std::vector<double> xv(xyz, xyz + 3 * (size_t)nv);
    std::vector<int> vperm = morton_order(xv, nv, lo, hi);
    std::vector<int> vinv(nv);
    for (int i = 0; i < nv; ++i) vinv[vperm[i]] = i;
    std::vector<double> cen(3 * (size_t)nf);
    for (int t = 0; t < nf; ++t)
        for (int d = 0; d < 3; ++d)
            cen[3 * t + d] = (xyz[3 * tri_in[3 * t] + d] + xyz[3 * tri_in[3 * t + 1] + d] +
                              xyz[3 * tri_in[3 * t + 2] + d]) / 3.0;
    std::vector<int> tperm = morton_order(cen, nf, lo, hi);
    std::vector<double> hx(3 * (size_t)nv), hn(3 * (size_t)nv);
    for (int i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d) {
            hx[3 * i + d] = xyz[3 * vperm[i] + d];
            hn[3 * i + d] = nrm[3 * vperm[i] + d];
        }
    std::vector<int> ht(3 * (size_t)nf);
    for (int t = 0; t < nf; ++t)
        for (int k = 0; k < 3; ++k) ht[3 * t + k] = vinv[tri_in[3 * tperm[t] + k]];
    // incidence lists: entries t*3+k with ht[t][k] == i, in increasing entry order
    std::vector<int> off(nv + 1, 0), ent(3 * (size_t)nf);
    for (int e = 0; e < 3 * nf; ++e) off[ht[e] + 1]++;
    for (int i = 0; i < nv; ++i) off[i + 1] += off[i];
    {
        std::vector<int> fill(off.begin(), off.end() - 1);
        for (int e = 0; e < 3 * nf; ++e) ent[fill[ht[e]]++] = e;
    }

    const bool lower = prm.method == HOBI_LOWER_ORDER;
    hobi_problem pb = new hobi_problem_s();
    pb->ctx = ctx;
    pb->prm = prm;
    pb->vperm = lower ? tperm : vperm;   // internal site -> caller's vertex (triangle) index
    pb->tperm = tperm;
    DeviceProblem& d = pb->d;
    d.method = prm.method;
    d.nverts = nv;
    d.nv = lower ? nf : nv;
    d.nf = nf;
    d.nc = nc;
    d.nn = lower ? nf : 4 * nf;
    d.eps1 = prm.eps1;
    d.eps2 = prm.eps2;
    d.kappa = prm.kappa;
    d.eps = prm.eps2 / prm.eps1;
    for (int k = 0; k < 3; ++k) d.center[k] = 0.5 * (lo[k] + hi[k]);
    d.extent = extent;
    d.nv_pad = round_up(d.nv, 2048);
    d.nc_pad = round_up(nc, 256);
    d.plan_pts = make_grid_plan(d.nc_pad, d.nn, 1);

    auto cleanup_fail = [&](hobi_status code) {
        free_problem(pb);
        delete pb;
        return code;
    };
#define PCHK(expr)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return cleanup_fail(fail(ctx, e_ == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP,  \
                                     "%s: %s", #expr, hipGetErrorString(e_)));                  \
    } while (0)

    // the pair plans: the split of the pair sum over the waves the device holds at once
    std::vector<int> ptab;
    {
        const int tpl32 = tpl32_for(d.nv_pad);
        const int r64 = pair_resident_waves(ctx->device, false, kTpl64);
        const int r32 = pair_resident_waves(ctx->device, true, tpl32);
        if (r64 < 1 || r32 < 1)
            return cleanup_fail(fail(ctx, HOBI_E_HIP, "pair kernel occupancy query failed"));
        if (!make_pair_plan(d.nv, d.nn, kTpl64, r64, 1, &d.plan64, &ptab) ||
            !make_pair_plan(d.nv, d.nn, tpl32, r32, kPairWaves, &d.plan32, &ptab))
            return cleanup_fail(fail(ctx, HOBI_E_ARG, "problem too large: %d sites x %d nodes", d.nv, d.nn));
        // the partial rows of the current precision's plan (hobi_problem_set_precision grows
        // the buffer for the other one when it needs more), and the point sums of the energy
        const size_t pts = (size_t)d.nc_pad * d.plan_pts.chunks;
        d.partial_need[0] = std::max((size_t)2 * d.plan64.slot * d.plan64.slots * d.plan64.rows, pts);
        d.partial_need[1] = std::max((size_t)2 * d.plan32.slot * d.plan32.slots * d.plan32.rows, pts);
        d.partial_elems = d.partial_need[prm.precision == HOBI_MIXED ? 1 : 0];
    }

    hipStream_t s = ctx->stream;
    const int ns = d.nv;   // sites
    PCHK(dalloc(&d.plan_tab, ptab.size()));
    PCHK(hipMemcpyAsync(d.plan_tab, ptab.data(), sizeof(int) * ptab.size(), hipMemcpyHostToDevice, s));
    d.plan64.gstart = d.plan_tab;
    d.plan32.gstart = d.plan_tab + (d.plan64.groups + 1);
    PCHK(dalloc(&d.xyz, 3 * (size_t)ns));
    PCHK(dalloc(&d.nrm, 3 * (size_t)ns));
    if (lower) PCHK(dalloc(&d.vxyz, 3 * (size_t)nv));
    PCHK(dalloc(&d.tri, 3 * (size_t)nf));
    PCHK(dalloc(&d.qpos, 3 * (size_t)nc));
    PCHK(dalloc(&d.q, nc));
    PCHK(dalloc(&d.qsoa, 3 * (size_t)d.nc_pad));
    if (!lower) PCHK(dalloc(&d.patch, 30 * (size_t)nf));
    PCHK(dalloc(&d.node64, d.nn));
    PCHK(dalloc(&d.node32, d.nn));
    PCHK(dalloc(&d.node_vid, d.nn));
    PCHK(dalloc(&d.blk_range, (d.nn + 63) / 64));
    PCHK(dalloc(&d.w, d.nn));
    PCHK(dalloc(&d.tgt64, 6 * (size_t)d.nv_pad));
    PCHK(dalloc(&d.tgt32, 6 * (size_t)d.nv_pad));
    PCHK(dalloc(&d.inc_off, ns + 1));
    PCHK(dalloc(&d.inc_ent, lower ? 1 : 3 * (size_t)nf));
    PCHK(dalloc(&d.coef, lower ? 1 : 36 * (size_t)nf));
    PCHK(dalloc(&d.rhs, 2 * (size_t)ns));
    PCHK(dalloc(&d.dinv, 2 * (size_t)ns));
    PCHK(dalloc(&d.partial, d.partial_elems));
    PCHK(dalloc(&pb->d_vperm, ns));
    PCHK(dalloc(&pb->u_in, 2 * (size_t)ns));
    PCHK(dalloc(&pb->y_out, 2 * (size_t)ns));
    PCHK(dalloc(&pb->phi_reac, nc));
    PCHK(dalloc(&pb->e_dev, 4));
    PCHK(hipHostMalloc((void**)&pb->host_pinned, 64));
    PCHK(dalloc(&pb->d_err, nf));

    std::vector<double> qs(3 * (size_t)d.nc_pad);
    for (int k = 0; k < d.nc_pad; ++k)
        for (int c = 0; c < 3; ++c) qs[(size_t)c * d.nc_pad + k] = qpos[3 * std::min(k, nc - 1) + c];

    if (lower) {
        // sites (centroids, face normals) are computed by the setup kernel from the vertices
        PCHK(hipMemcpyAsync(d.vxyz, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice, s));
        off.assign(ns + 1, 0);   // no incident (singular) entries
    } else {
        PCHK(hipMemcpyAsync(d.xyz, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice, s));
        PCHK(hipMemcpyAsync(d.nrm, hn.data(), sizeof(double) * hn.size(), hipMemcpyHostToDevice, s));
    }
    PCHK(hipMemcpyAsync(d.tri, ht.data(), sizeof(int) * ht.size(), hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync(d.qpos, qpos, sizeof(double) * 3 * nc, hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync(d.q, q, sizeof(double) * nc, hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync(d.qsoa, qs.data(), sizeof(double) * qs.size(), hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync(d.inc_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, s));
    if (!lower) PCHK(hipMemcpyAsync(d.inc_ent, ent.data(), sizeof(int) * ent.size(), hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync(pb->d_vperm, pb->vperm.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    // masked-id range of every 64-node block: the vertices of its 16 consecutive triangles
    // (higher-order), or its own 64 sites (lower-order: a node is masked for its own site)
    std::vector<int2> brange((d.nn + 63) / 64);
    for (size_t b = 0; b < brange.size(); ++b) {
        int lo = ns, hi = -1;
        if (lower) {
            lo = (int)(64 * b);
            hi = std::min(nf - 1, (int)(64 * b + 63));
        } else {
            for (int t = (int)(16 * b); t < std::min(nf, (int)(16 * b + 16)); ++t)
                for (int k = 0; k < 3; ++k) {
                    lo = std::min(lo, ht[3 * t + k]);
                    hi = std::max(hi, ht[3 * t + k]);
                }
        }
        brange[b] = make_int2(lo, hi);
    }
    PCHK(hipMemcpyAsync(d.blk_range, brange.data(), sizeof(int2) * brange.size(), hipMemcpyHostToDevice, s));
    PCHK(hipMemsetAsync(d.node64, 0, sizeof(NodeD) * d.nn, s));
    PCHK(hipMemsetAsync(d.node32, 0, sizeof(NodeF) * d.nn, s));
    PCHK(hipMemsetAsync(pb->d_err, 0, sizeof(int) * nf, s));
    PCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    if ((st = run_device_setup(pb, &ms)) != HOBI_OK) return cleanup_fail(st);
    if ((st = build_tree_plan(pb, tree_limit, tree_need)) != HOBI_OK) return cleanup_fail(st);
    std::vector<int> herr(nf);
    PCHK(hipMemcpyAsync(herr.data(), pb->d_err, sizeof(int) * nf, hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    for (int t = 0; t < nf; ++t)
        if (herr[t])
            return cleanup_fail(fail(ctx, HOBI_E_MESH, "triangle %d: a vertex normal is parallel to an edge",
                                     tperm[t]));
    pb->last.ms_setup = ms;

    // every charge must be enclosed: solid-angle fraction ~ 1 inside, ~ 0 outside
    double* frac = pb->phi_reac;
    PCHK(launch_solid_angle(d, frac, s));
    std::vector<double> hf(nc);
    PCHK(hipMemcpyAsync(hf.data(), frac, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    for (int k = 0; k < nc; ++k) {
        if (!std::isfinite(hf[k])) return cleanup_fail(fail(ctx, HOBI_E_NUMERIC, "charge %d: non-finite", k));
        if (hf[k] < 0.5)
            return cleanup_fail(fail(ctx, HOBI_E_CHARGE_OUTSIDE, "charge %d is outside the surface", k));
    }
#undef PCHK
    pb->last.pairs_per_matvec = (int64_t)d.nv * d.nn;
    *out = pb;
    return HOBI_OK;
}

}  // namespace hobi

extern "C" {

void hobi_problem_destroy(hobi_problem pb) {
    if (!pb) return;
    if (pb->ctx && pb->ctx->stream) (void)hipStreamSynchronize(pb->ctx->stream);
    free_problem(pb);
    delete pb;
}

hobi_status hobi_problem_set_precision(hobi_problem pb, int32_t precision) {
    if (!pb) return HOBI_E_ARG;
    hobi_ctx c = pb->ctx;
    if (precision != HOBI_FP64 && precision != HOBI_MIXED)
        return fail(c, HOBI_E_ARG, "precision must be HOBI_FP64 or HOBI_MIXED");
    DeviceProblem& d = pb->d;
    const size_t need = d.partial_need[precision == HOBI_MIXED ? 1 : 0];
    if (need > d.partial_elems) {
        // the other plan's partial rows do not fit: a larger buffer, once the work queued on
        // the old one is done
        HIPCHK(c, hipSetDevice(c->device));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double* grown = nullptr;
        const hipError_t e = dalloc(&grown, need);
        if (e != hipSuccess)
            return fail(c, e == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP, "partial-row buffer: %s",
                        hipGetErrorString(e));
        (void)hipFree(d.partial);
        d.partial = grown;
        d.partial_elems = need;
    }
    pb->prm.precision = precision;
    return HOBI_OK;
}

hobi_status hobi_problem_set_dielectric(hobi_problem pb, double eps1, double eps2, double kappa) {
    TraceRange trace_range("hobi_problem_set_dielectric");
    if (!pb) return HOBI_E_ARG;
    hobi_params p = pb->prm;
    p.eps1 = eps1;
    p.eps2 = eps2;
    p.kappa = kappa;
    hobi_status st = validate_params(pb->ctx, p);
    if (st != HOBI_OK) return st;
    if (!(kappa * 2.0 * pb->d.extent < kExpTabMaxZ))
        return fail(pb->ctx, HOBI_E_ARG, "kappa times the surface's extent must stay below %g", kExpTabMaxZ / 2);
    HIPCHK(pb->ctx, hipSetDevice(pb->ctx->device));
    pb->prm = p;
    DeviceProblem& d = pb->d;
    d.eps1 = eps1;
    d.eps2 = eps2;
    d.kappa = kappa;
    d.eps = eps2 / eps1;
    float ms = 0.f;
    if ((st = run_device_setup(pb, &ms)) != HOBI_OK) return st;
    pb->last.ms_setup = ms;
    return HOBI_OK;
}

hobi_status hobi_problem_set_solver(hobi_problem pb, double rtol, int32_t max_iter, int32_t restart) {
    if (!pb) return HOBI_E_ARG;
    hobi_params p = pb->prm;
    p.rtol = rtol;
    p.max_iter = max_iter;
    p.restart = restart;
    hobi_status st = validate_params(pb->ctx, p);
    if (st != HOBI_OK) return st;
    pb->prm = p;
    return HOBI_OK;
}

hobi_status hobi_matvec(hobi_problem pb, const double* u, double* y, int32_t on_device) {
    TraceRange trace_range("hobi_matvec");
    if (!pb) return HOBI_E_ARG;
    if (!u || !y) return fail(pb->ctx, HOBI_E_ARG, "NULL vector");
    HIPCHK(pb->ctx, hipSetDevice(pb->ctx->device));
    hobi_status st = to_internal(pb, u, on_device, pb->u_in);
    if (st != HOBI_OK) return st;
    if ((st = matvec_internal(pb, pb->u_in, pb->y_out)) != HOBI_OK) return st;
    return from_internal(pb, pb->y_out, on_device, y);
}

hobi_status hobi_matvec_noalloc(hobi_problem pb, const double* u, double* y) {
    if (!pb) return HOBI_E_ARG;
    hobi_ctx c = pb->ctx;
    if (!u || !y) return fail(c, HOBI_E_ARG, "NULL vector");
    if (pb->d.tree.on) return fail(c, HOBI_E_ARG, "hobi_matvec_noalloc takes the dense sum only (tree_theta = 0)");
    if (!c->scratch) return fail(c, HOBI_E_HIP, "static work space not resolved");
    const bool mixed = pb->prm.precision == HOBI_MIXED;
    PairPlan pl{};
    size_t row_bytes = 0;
    if (!make_static_pair_plan(mixed ? pb->d.plan32 : pb->d.plan64, pb->d.nn, &pl, &row_bytes))
        return fail(c, HOBI_E_ARG, "problem too large for the static work space: one node group needs %zu bytes "
                    "of partial rows, %zu are available", row_bytes, kStaticScratchBytes - kStaticTableBytes);
    int* tab = (int*)c->scratch;
    double* part = (double*)((char*)c->scratch + kStaticTableBytes);
    pl.gstart = tab;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const DeviceProblem& d = pb->d;
    HIPCHK(c, launch_permute(u, pb->u_in, pb->d_vperm, d.nv, true, s));
    HIPCHK(c, launch_group_starts(tab, pl.groups, d.nn, s));
    HIPCHK(c, launch_gather(d, pb->u_in, mixed, s));
    HIPCHK(c, launch_pair_plan(d, pl, part, mixed, s));
    HIPCHK(c, launch_combine_plan(d, pl, part, pb->u_in, pb->y_out, s));
    HIPCHK(c, launch_permute(pb->y_out, y, pb->d_vperm, d.nv, false, s));
    return HOBI_OK;
}

hobi_status hobi_device_math(hobi_ctx ctx, int32_t fn, int32_t n, const double* x, double* y) {
    if (!ctx) return HOBI_E_ARG;
    if (fn != HOBI_MATH_EXP_NEG && fn != HOBI_MATH_RSQRT) return fail(ctx, HOBI_E_ARG, "unknown function %d", fn);
    if (n < 0 || (n > 0 && (!x || !y))) return fail(ctx, HOBI_E_ARG, "need n >= 0 and non-NULL arrays");
    if (n == 0) return HOBI_OK;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || (fn == HOBI_MATH_EXP_NEG ? !(x[i] >= 0.0 && x[i] < kExpTabMaxZ) : !(x[i] > 0.0)))
            return fail(ctx, HOBI_E_ARG, "argument %d out of the function's domain", i);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    double* d = nullptr;
    HIPCHK(ctx, hipMallocAsync((void**)&d, sizeof(double) * 2 * (size_t)n, s));
    hipError_t e = hipMemcpyAsync(d, x, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_device_math(fn, d, d + n, n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(y, d + n, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    const hipError_t f = hipFreeAsync(d, s);
    if (e == hipSuccess) e = f;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ctx, HOBI_E_HIP, "device math: %s", hipGetErrorString(e));
    return HOBI_OK;
}

hobi_status hobi_energy(hobi_problem pb, const double* u, int32_t on_device, double* e_sol) {
    TraceRange trace_range("hobi_energy");
    if (!pb) return HOBI_E_ARG;
    if (!u || !e_sol) return fail(pb->ctx, HOBI_E_ARG, "NULL argument");
    HIPCHK(pb->ctx, hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    hobi_status st = to_internal(pb, u, on_device, pb->u_in);
    if (st != HOBI_OK) return st;
    HIPCHK(pb->ctx, launch_gather(pb->d, pb->u_in, false, s));
    HIPCHK(pb->ctx, launch_reaction_energy(pb->d, pb->phi_reac, pb->e_dev, s));
    return read_scalar(pb, pb->e_dev, e_sol);
}

hobi_status hobi_field(hobi_problem pb, const double* u, int32_t on_device, int32_t np, const double* points,
                       double* phi, double* field, double* reac, double* reac_field, int32_t* inside) {
    TraceRange trace_range("hobi_field");
    if (!pb) return HOBI_E_ARG;
    hobi_ctx c = pb->ctx;
    if (!u) return fail(c, HOBI_E_ARG, "NULL u");
    if (np < 0) return fail(c, HOBI_E_ARG, "np < 0");
    if (np == 0) return HOBI_OK;
    if (!points) return fail(c, HOBI_E_ARG, "NULL points");
    for (size_t i = 0; i < 3 * (size_t)np; ++i)
        if (!std::isfinite(points[i])) return fail(c, HOBI_E_NUMERIC, "non-finite point");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    DeviceProblem& d = pb->d;
    const bool mixed = pb->prm.precision == HOBI_MIXED;
    // node strengths of u
    hobi_status st = to_internal(pb, u, on_device, pb->u_in);
    if (st != HOBI_OK) return st;
    HIPCHK(c, launch_gather(d, pb->u_in, mixed, s));
    // the split over waves (dense sum) or the treecode's slots of points, points in Morton order
    // (the treecode form of the field sums is defined for the higher-order method's nodes)
    const bool tree = d.tree.on != 0 && d.method == HOBI_HIGHER_ORDER;
    PairPlan pl{};
    std::vector<int> gs;
    if (tree) {
        pl.tpl = mixed ? kFieldTpl32 : kFieldTpl64;
        pl.slot = 64 * pl.tpl;
        pl.slots = (np + pl.slot - 1) / pl.slot;
        pl.groups = 1;
    } else {
        const int res = field_resident_waves(c->device, mixed);
        if (res < 1) return fail(c, HOBI_E_HIP, "field kernel occupancy query failed");
        if (!make_pair_plan(np, d.nn, mixed ? kFieldTpl32 : kFieldTpl64, res, 1, &pl, &gs))
            return fail(c, HOBI_E_ARG, "too many points: %d", np);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < np; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], points[3 * i + k]);
            hi[k] = std::max(hi[k], points[3 * i + k]);
        }
    if (d.kappa > 0.0) {
        // kappa r must stay below kExpTabMaxZ for every (point, node) pair (the FP64 sums'
        // table-driven exponential): r is at most the distance from the surface's box centre
        // to the points' box's farthest corner plus half the surface's box diagonal
        double far2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double a = std::max(std::fabs(hi[k] - d.center[k]), std::fabs(lo[k] - d.center[k]));
            far2 += a * a;
        }
        if (!(d.kappa * (std::sqrt(far2) + 0.5 * d.extent) < 0.5 * kExpTabMaxZ))
            return fail(c, HOBI_E_ARG, "kappa times the points' distance from the surface must stay below %g",
                        0.5 * kExpTabMaxZ);
    }
    FieldWork& f = pb->field;
    f.np = np;
    f.np_pad = tree ? round_up(np, kFieldTreeBatch) : pl.slots * pl.slot;
    const int nb = (np + kFieldTreeBatch - 1) / kFieldTreeBatch;
    const size_t sort_bytes = point_sort_temp_bytes(np);
    if (sort_bytes == 0) return fail(c, HOBI_E_HIP, "radix-sort work space query failed");
    hipError_t e = hipSuccess;
    if ((e = grow(&f.raw, &f.cap_raw, 3 * (size_t)np)) != hipSuccess ||
        (e = grow(&f.keys, &f.cap_keys, 2 * (size_t)np)) != hipSuccess ||
        (e = grow(&f.idx, &f.cap_idx, (size_t)np)) != hipSuccess ||
        (e = grow(&f.order, &f.cap_order, (size_t)np)) != hipSuccess ||
        (e = grow((char**)&f.sort_tmp, &f.cap_sort_tmp, sort_bytes)) != hipSuccess ||
        (e = grow(&f.pts64, &f.cap_pts64, 3 * (size_t)f.np_pad)) != hipSuccess ||
        (e = grow(&f.pts32, &f.cap_pts32, 3 * (size_t)f.np_pad)) != hipSuccess ||
        (tree && (e = grow(&f.bbox, &f.cap_bbox, 6 * (size_t)nb)) != hipSuccess) ||
        (tree && (e = grow_pinned(&f.hbox, &f.cap_hbox, 6 * (size_t)nb)) != hipSuccess))
        return fail(c, e == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP, "field work space: %s",
                    hipGetErrorString(e));
    // the points in Morton order over their box (sorted position -> caller index in f.order),
    // staged on the device; with the treecode the box of each batch of sorted points
    HIPCHK(c, hipMemcpyAsync(f.raw, points, sizeof(double) * 3 * (size_t)np, hipMemcpyHostToDevice, s));
    HIPCHK(c, launch_point_order(f, lo, hi, d.center, d.s32, tree ? nb : 0, s));
    if (tree) {
        HIPCHK(c, hipMemcpyAsync(f.hbox, f.bbox, sizeof(double) * 6 * (size_t)nb, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    // treecode: each batch of kFieldTreeBatch points walks the cluster tree (accepted when
    // r_b + r_c <= theta |c_b - c_c|; the points are off the surface, so no incidence rule),
    // work items per slot in walk order
    std::vector<int4> items;
    std::vector<int> srow(1, 0);
    if (tree) {
        const TreePlan& t = d.tree;
        std::vector<std::vector<std::pair<int, int>>> walk(nb);
        f.tree_far = f.tree_near = 0;
        std::vector<int> stack;
        for (int bi = 0; bi < nb; ++bi) {
            const double* blo = f.hbox + 6 * (size_t)bi;
            const double* bhi = blo + 3;
            double cb[3], q = 0;
            for (int k = 0; k < 3; ++k) cb[k] = 0.5 * (blo[k] + bhi[k]), q += (bhi[k] - blo[k]) * (bhi[k] - blo[k]);
            const double rb = 0.5 * std::sqrt(q);
            stack.assign(1, t.root);
            while (!stack.empty()) {
                const int cc = stack.back();
                stack.pop_back();
                const double* cen = &t.h_cen[3 * (size_t)cc];
                const double dx = cb[0] - cen[0], dy = cb[1] - cen[1], dz = cb[2] - cen[2];
                if (rb + t.h_rad[cc] <= pb->prm.tree_theta * std::sqrt(dx * dx + dy * dy + dz * dz)) {
                    walk[bi].emplace_back(cc, 1);
                    ++f.tree_far;
                } else if (t.h_child[cc].x < 0) {
                    walk[bi].emplace_back(cc, 0);
                    ++f.tree_near;
                } else {
                    stack.push_back(t.h_child[cc].y);
                    stack.push_back(t.h_child[cc].x);
                }
            }
        }
        for (int sl = 0; sl < pl.slots; ++sl) {
            for (const auto& w : walk[sl * pl.slot / kFieldTreeBatch]) items.push_back(make_int4(sl, w.second, w.first, 0));
            if (items.size() > ((size_t)1 << 30)) return fail(c, HOBI_E_ARG, "too many points for the treecode: %d", np);
            srow.push_back((int)items.size());
        }
    }
    // treecode: passes over runs of slots whose partial rows fit kFieldTreeRows doubles
    std::vector<int> pass_start(1, 0);
    size_t pass_rows = 0;
    if (tree) {
        const size_t row = 5 * (size_t)pl.slot;
        for (int sl = 0; sl < pl.slots; ++sl) {
            const size_t rows_now = (size_t)(srow[sl + 1] - srow[pass_start.back()]);
            if (sl > pass_start.back() && rows_now * row > kFieldTreeRows) pass_start.push_back(sl);
            pass_rows = std::max(pass_rows, (size_t)(srow[sl + 1] - srow[pass_start.back()]));
        }
        pass_start.push_back(pl.slots);
    }
    const size_t nparts = (tree ? pass_rows : (size_t)pl.workers) * 5 * pl.slot;
    if ((e = grow(&f.partial, &f.cap_partial, nparts)) != hipSuccess ||
        (e = grow(&f.gstart, &f.cap_gstart, gs.size())) != hipSuccess ||
        (e = grow(&f.out, &f.cap_out, 9 * (size_t)np)) != hipSuccess ||
        (e = grow(&f.inside, &f.cap_inside, (size_t)np)) != hipSuccess ||
        (e = grow(&f.outc, &f.cap_outc, 8 * (size_t)np)) != hipSuccess ||
        (e = grow(&f.insc, &f.cap_insc, (size_t)np + 1)) != hipSuccess ||
        (tree && (e = grow(&f.items, &f.cap_items, pass_rows)) != hipSuccess) ||
        (tree && (e = grow(&f.slot_row, &f.cap_slot_row, srow.size())) != hipSuccess))
        return fail(c, e == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP, "field work space: %s",
                    hipGetErrorString(e));
    if (tree) {
        HIPCHK(c, hipMemcpyAsync(f.slot_row, srow.data(), sizeof(int) * srow.size(), hipMemcpyHostToDevice, s));
        HIPCHK(c, launch_tree_proxies(d, mixed, s));
        for (size_t k = 0; k + 1 < pass_start.size(); ++k) {
            const int s0 = pass_start[k], s1 = pass_start[k + 1];
            const int r0 = srow[s0], nrow = srow[s1] - srow[s0];
            if (k > 0) HIPCHK(c, hipStreamSynchronize(s));   // the previous pass is done with f.items
            HIPCHK(c, hipMemcpyAsync(f.items, items.data() + r0, sizeof(int4) * (size_t)nrow, hipMemcpyHostToDevice, s));
            {
                ScopedTimer t(pb, T_FIELD);
                HIPCHK(c, launch_field_tree_pairs(d, f, nrow, mixed, s));
            }
            HIPCHK(c, launch_field_combine(d, f, pl, mixed, s, f.slot_row, r0, s0 * pl.slot,
                                           std::min(s1 * pl.slot, np)));
        }
    } else {
        HIPCHK(c, hipMemcpyAsync(f.gstart, gs.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
        pl.gstart = f.gstart;
        {
            ScopedTimer t(pb, T_FIELD);
            HIPCHK(c, launch_field_pairs(d, f, pl, mixed, s));
        }
        HIPCHK(c, launch_field_combine(d, f, pl, mixed, s));
    }
    // outputs in the caller's order on the device, then straight into the caller's arrays
    HIPCHK(c, hipMemsetAsync(f.insc + np, 0, sizeof(int), s));
    HIPCHK(c, launch_field_scatter(f, s));
    const size_t n1 = (size_t)np;
    if (phi) HIPCHK(c, hipMemcpyAsync(phi, f.outc, sizeof(double) * n1, hipMemcpyDeviceToHost, s));
    if (field) HIPCHK(c, hipMemcpyAsync(field, f.outc + n1, sizeof(double) * 3 * n1, hipMemcpyDeviceToHost, s));
    if (reac) HIPCHK(c, hipMemcpyAsync(reac, f.outc + 4 * n1, sizeof(double) * n1, hipMemcpyDeviceToHost, s));
    if (reac_field)
        HIPCHK(c, hipMemcpyAsync(reac_field, f.outc + 5 * n1, sizeof(double) * 3 * n1, hipMemcpyDeviceToHost, s));
    if (inside) HIPCHK(c, hipMemcpyAsync(inside, f.insc, sizeof(int) * n1, hipMemcpyDeviceToHost, s));
    int* flag = (int*)pb->host_pinned;
    HIPCHK(c, hipMemcpyAsync(flag, f.insc + np, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (*flag) return fail(c, HOBI_E_NUMERIC, "non-finite field value (a point on the surface?)");
    return HOBI_OK;
}

hobi_status hobi_solve(hobi_problem pb, double* phi, double* dphi, double* e_sol, hobi_stats* stats) {
    TraceRange trace_range("hobi_solve");
    if (!pb) return HOBI_E_ARG;
    hobi_ctx c = pb->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int nv = pb->d.nv, n = 2 * nv;
    hipEvent_t ev[4];
    for (auto& e : ev) e = take_event(pb);
    for (auto& e : ev)
        if (!e) return fail(c, HOBI_E_HIP, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(ev[0], s));
    int iters = 0, refine_steps = 0, dense_mv = 0;
    double est = 0;
    bool conv = false;
    hobi_status st = gmres(pb, &iters, &est, &conv, &refine_steps, &dense_mv);
    if (st != HOBI_OK) return st;
    HIPCHK(c, hipEventRecord(ev[1], s));
    Krylov& k = pb->kr;
    // true residual (tree_refine: its last outer step's dense residual, already in k.ro)
    const double* rres = k.ro;
    if (refine_steps == 0) {
        if ((st = matvec_internal(pb, k.x, k.tmp)) != HOBI_OK) return st;
        HIPCHK(c, launch_sub(pb->d.rhs, k.tmp, k.tmp, n, s));
        rres = k.tmp;
    }
    if ((st = norm2(pb, rres, n, k.scal + 2)) != HOBI_OK) return st;
    if ((st = norm2(pb, pb->d.rhs, n, k.scal + 3)) != HOBI_OK) return st;
    // energy (FP64 nodes, FP64 reduction)
    HIPCHK(c, hipEventRecord(ev[2], s));
    HIPCHK(c, launch_gather(pb->d, k.x, false, s));
    HIPCHK(c, launch_reaction_energy(pb->d, pb->phi_reac, pb->e_dev, s));
    HIPCHK(c, hipEventRecord(ev[3], s));
    double hs[2];
    HIPCHK(c, hipMemcpyAsync(hs, k.scal + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    double E = 0;
    if ((st = read_scalar(pb, pb->e_dev, &E)) != HOBI_OK) return st;
    std::vector<double> hu(n);
    if ((st = from_internal(pb, k.x, 0, hu.data())) != HOBI_OK) return st;
    const double scale = 4.0 * kPi * 332.0716;
    if (phi)
        for (int i = 0; i < nv; ++i) phi[i] = scale * hu[i];
    if (dphi)
        for (int i = 0; i < nv; ++i) dphi[i] = scale * hu[nv + i];
    if (e_sol) *e_sol = E;
    float t_solve = 0, t_energy = 0;
    (void)hipEventElapsedTime(&t_solve, ev[0], ev[1]);
    (void)hipEventElapsedTime(&t_energy, ev[2], ev[3]);
    for (auto& e : ev) pb->event_pool.push_back(e);
    if ((st = resolve_timers(pb)) != HOBI_OK) return st;
    hobi_stats& L = pb->last;
    L.iterations = iters;
    L.converged = conv ? 1 : 0;
    L.est_residual = est;
    L.true_residual = hs[1] > 0 ? hs[0] / hs[1] : 0.0;
    L.ms_solve = t_solve;
    L.ms_energy = t_energy;
    L.ms_pair_kernel = pb->ms[T_PAIR];
    L.pair_launches = pb->cnt[T_PAIR];
    L.ms_gather = pb->ms[T_GATHER];
    L.ms_combine = pb->ms[T_COMBINE];
    L.ms_krylov = pb->ms[T_KRYLOV];
    L.ms_field_kernel = pb->ms[T_FIELD];
    L.field_launches = pb->cnt[T_FIELD];
    L.tree_far_pairs = pb->d.tree.nfar;
    L.field_tree_far_pairs = pb->field.tree_far;
    L.field_tree_near_pairs = pb->field.tree_near;
    L.tree_near_pairs = pb->d.tree.nnear;
    L.refine_steps = refine_steps;
    L.dense_matvecs = dense_mv;
    if (stats) *stats = L;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(hu[i])) return fail(c, HOBI_E_NUMERIC, "non-finite solution");
    if (!std::isfinite(E)) return fail(c, HOBI_E_NUMERIC, "non-finite energy");
    if (!conv) {
        if (refine_steps > 0)
            return fail(c, HOBI_E_NOCONV, "defect correction stopped after %d outer steps (%d treecode matvecs), "
                        "dense residual %.3e", refine_steps, iters, est);
        return fail(c, HOBI_E_NOCONV, "GMRES stopped at %d matvecs, residual %.3e", iters, est);
    }
    return HOBI_OK;
}

hobi_status hobi_get_nodes(hobi_problem pb, double* y, double* ny, double* w) {
    if (!pb) return HOBI_E_ARG;
    HIPCHK(pb->ctx, hipSetDevice(pb->ctx->device));
    const int nf = pb->d.nf, nn = pb->d.nn;
    std::vector<NodeD> nd(nn);
    std::vector<double> hw(nn);
    hipStream_t s = pb->ctx->stream;
    HIPCHK(pb->ctx, hipMemcpyAsync(nd.data(), pb->d.node64, sizeof(NodeD) * nn, hipMemcpyDeviceToHost, s));
    HIPCHK(pb->ctx, hipMemcpyAsync(hw.data(), pb->d.w, sizeof(double) * nn, hipMemcpyDeviceToHost, s));
    HIPCHK(pb->ctx, hipStreamSynchronize(s));
    const int per = nn / nf;   // nodes per triangle: 4 (higher-order) or 1 (lower-order)
    for (int t = 0; t < nf; ++t) {
        const int o = pb->tperm[t];
        for (int m = 0; m < per; ++m) {
            const NodeD& a = nd[per * t + m];
            const size_t b = per * (size_t)o + m;
            if (y) y[3 * b] = a.x, y[3 * b + 1] = a.y, y[3 * b + 2] = a.z;
            if (ny) ny[3 * b] = a.nx, ny[3 * b + 1] = a.ny, ny[3 * b + 2] = a.nz;
            if (w) w[b] = hw[per * t + m];
        }
    }
    return HOBI_OK;
}

hobi_status hobi_get_rhs(hobi_problem pb, double* b) {
    if (!pb || !b) return HOBI_E_ARG;
    HIPCHK(pb->ctx, hipSetDevice(pb->ctx->device));
    return from_internal(pb, pb->d.rhs, 0, b);
}

hobi_status hobi_reset_stats(hobi_problem pb) {
    if (!pb) return HOBI_E_ARG;
    hobi_status st = resolve_timers(pb);
    for (int k = 0; k < T_NKINDS; ++k) pb->ms[k] = 0, pb->cnt[k] = 0;
    return st;
}

hobi_status hobi_get_stats(hobi_problem pb, hobi_stats* out) {
    if (!pb || !out) return HOBI_E_ARG;
    hobi_status st = resolve_timers(pb);
    pb->last.ms_pair_kernel = pb->ms[T_PAIR];
    pb->last.pair_launches = pb->cnt[T_PAIR];
    pb->last.ms_gather = pb->ms[T_GATHER];
    pb->last.ms_combine = pb->ms[T_COMBINE];
    pb->last.ms_krylov = pb->ms[T_KRYLOV];
    pb->last.ms_field_kernel = pb->ms[T_FIELD];
    pb->last.field_launches = pb->cnt[T_FIELD];
    pb->last.tree_far_pairs = pb->d.tree.nfar;
    pb->last.field_tree_far_pairs = pb->field.tree_far;
    pb->last.field_tree_near_pairs = pb->field.tree_near;
    pb->last.tree_near_pairs = pb->d.tree.nnear;
    *out = pb->last;
    return st;
}

}  // extern "C"
