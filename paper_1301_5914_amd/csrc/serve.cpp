// Request server: continuous batching of HOBI-PB solves on one device (hobi_server_* in
// hobi.h).  One worker thread owns a stream; requests are admitted by device footprint,
// advance one GMRES iteration per tick with their matvecs batched into four launches
// (requests with the treecode run their own matvec launches in the same tick), and
// retire as soon as they converge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "hobi.h"
#include "hobi_host.h"
#include "hobi_internal.h"
#include "serve_internal.h"
#include "trace.h"

using namespace hobi;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket = 0;
    int nv = 0, nf = 0, nc = 0;
    int nu = 0;             // unknown sites: vertices, or triangles (lower-order method)
    std::vector<double> xyz, nrm, qpos, q;
    std::vector<int32_t> tri;
    hobi_params prm{};
    int64_t footprint = 0;  // bytes charged to the budget
    int64_t tree_charged = 0;   // of which the treecode buffers, once measured
    // device state while active
    hobi_problem pb = nullptr;
    PairPlan plan{};        // the problem's own pair plan (its partial-sum buffer is reused)
    double *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
    double *h1 = nullptr, *h2 = nullptr, *hn = nullptr, *yk = nullptr, *dpart = nullptr;
    double *x = nullptr, *scal = nullptr;
    double* z = nullptr;    // D^-1 v_k, the matvec input under diag_scaling
    int m = 0, k = 0;
    double bnorm = 0, est = 1;
    // tree_refine: the single-problem defect correction's state (outer iterate, dense
    // residual, dense matvec output), the right-hand side's norm, the last outer residual's
    // norm, the current correction's tolerance, treecode matvecs and outer steps so far
    double *xo = nullptr, *ro = nullptr, *tmp = nullptr;
    double bnorm_b = 0, rnorm = 0, tol_in = 0;
    int total = 0, steps = 0;
    Clock::time_point t_admit;
    // outcome
    hobi_status status = HOBI_OK;
    std::string message;
    std::vector<double> phi, dphi;
    double energy = 0;
    hobi_stats stats{};
};

template <class T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Device bytes of one admitted request (the allocations of hobi_problem_create plus the
// server's Krylov basis), from its sizes alone.
int64_t footprint_bytes(int device, int nv, int nf, int nc, int m, int method, bool mixed) {
    // the lower-order method has one site and one node per triangle (an upper bound below)
    if (method == HOBI_LOWER_ORDER) nv = std::max(nv, nf);
    const int64_t nv_pad = round_up(nv, 2048), nc_pad = round_up(nc, 256), nn = 4LL * nf;
    const GridPlan pp = make_grid_plan((int)nc_pad, (int)nn, 1);
    // pair plans: the group starts of both, and one partial row of 2 * slot doubles per
    // worker of the request's own precision (a served problem keeps its precision)
    int64_t pair_rows_elems = 0, tab_ints = 0;
    for (int mx = 0; mx < 2; ++mx) {
        const int tpl = mx ? tpl32_for((int)nv_pad) : kTpl64;
        PairPlan pl{};
        std::vector<int> gs;
        if (!make_pair_plan(nv, (int)nn, tpl, std::max(1, pair_resident_waves(device, mx != 0, tpl)),
                            mx ? kPairWaves : 1, &pl, &gs))
            return INT64_MAX;
        if (mx == (mixed ? 1 : 0)) pair_rows_elems = 2LL * pl.slot * pl.slots * pl.rows;
        tab_ints += (int64_t)gs.size();
    }
    int64_t b = 0;
    b += 8 * (6LL * nv + 4LL * nc + 3 * nc_pad + 30LL * nf + 4 * nn + 12 * nv_pad + 36LL * nf + 2LL * nv + 4LL * nv);
    b += (int64_t)sizeof(NodeD) * nn + (int64_t)sizeof(NodeF) * nn + 16 * nn + 8 * (nn / 64 + 1);
    b += 4 * (3LL * nf + nv + 1 + 3LL * nf + nv + nf) + 2LL * 4 * nv_pad;
    b += 8 * std::max<int64_t>(pair_rows_elems, nc_pad * pp.chunks) + 4 * tab_ints;
    const int64_t n = 2LL * nv;
    b += 8 * ((int64_t)(m + 1) * n + (int64_t)(m + 1) * m + 6LL * (m + 1) + kDotBlocks * (int64_t)(m + 1) + 2 * n + 8);
    return b;
}

// Device bytes of a built problem's treecode buffers (0 without the treecode).  They depend
// on the partition, so a request is admitted on its dense footprint and its problem is built
// with the rest of the budget as the limit for them; a request whose buffers do not fit
// waits at the head of the queue, charged their size, until they do (alone in the server, it
// fails with HOBI_E_OOM).
int64_t tree_bytes(const DeviceProblem& d) {
    const TreePlan& t = d.tree;
    if (!t.on) return 0;
    int64_t b = (int64_t)t.nclu * (2 * sizeof(int2) + 6 * sizeof(double)) +
                (int64_t)t.nclu * t.nprox * (sizeof(ProxyD) + sizeof(ProxyF));
    int64_t part = 0;
    for (int m = 0; m < 2; ++m) {
        b += (int64_t)t.nitems[m] * sizeof(int4) + 4LL * ((d.nv + t.slot[m] - 1) / t.slot[m] + 1);
        part = std::max<int64_t>(part, 2LL * t.nitems[m] * t.slot[m]);
    }
    return b + 8 * part;
}

void free_request_device(Request& r) {
    double* ptrs[] = {r.V, r.H, r.cs, r.sn, r.g, r.h1, r.h2, r.hn, r.yk, r.dpart, r.x, r.scal, r.z, r.xo, r.ro, r.tmp};
    for (double* p : ptrs)
        if (p) (void)hipFree(p);
    r.V = r.H = r.cs = r.sn = r.g = r.h1 = r.h2 = r.hn = r.yk = r.dpart = r.x = r.scal = r.z = nullptr;
    r.xo = r.ro = r.tmp = nullptr;
    if (r.pb) hobi_problem_destroy(r.pb);
    r.pb = nullptr;
}

}  // namespace

struct hobi_server_s {
    int device = 0;
    hobi_ctx ctx = nullptr;           // the worker's context (own stream)
    int64_t budget = 0;
    int max_slots = 1;
    bool use_graph = true;

    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<std::unique_ptr<Request>> pending;
    std::map<uint64_t, std::unique_ptr<Request>> done;
    std::set<uint64_t> in_flight;     // submitted, not finished yet
    std::string last_error;
    hobi_server_stats st{};
    // preparation: requests whose problem (host checks, ordering, device setup) is being
    // built on the preparation thread's own context, and those built and waiting for the
    // worker; their footprints are already counted in in_use
    std::condition_variable prep_cv;
    std::deque<std::unique_ptr<Request>> ready;
    int preparing = 0;
    int active_count = 0;             // the worker's active requests (guarded by mu)
    int64_t in_use = 0;
    hobi_ctx prep_ctx = nullptr;
    std::thread prep;

    // worker-only state
    std::vector<std::unique_ptr<Request>> active;
    double batch_sum = 0;
    ServeDesc* d_desc = nullptr;
    ServeItem* d_items = nullptr;     // gather | pair | combine item arrays
    int* d_counts = nullptr;          // [4] matvec item counts, then [kKrylovPhases + 1] Krylov counts
    ServeDesc* h_desc = nullptr;      // pinned staging
    ServeItem* h_items = nullptr;
    int* h_counts = nullptr;
    KrylovDesc* d_kdesc = nullptr;    // one Arnoldi step per active request
    KrylovDesc* h_kdesc = nullptr;
    double* d_res = nullptr;          // one residual per active request
    double* h_res = nullptr;
    size_t cap_desc = 0, cap_items = 0;
    hipGraph_t graph = nullptr;       // diagonal scaling and the batched matvec
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t kgraph = nullptr;      // the batched Gram-Schmidt and Givens phases
    hipGraphExec_t kgraph_exec = nullptr;
    bool graph_dirty = true;
    std::thread worker;
};

namespace {

void fail_request(Request& r, hobi_status code, const std::string& msg) {
    r.status = code;
    r.message = msg;
}

// Allocates the Krylov state of a request whose problem the preparation thread created and
// starts its GMRES (x0 = 0, v0 = b / |b|).
hobi_status admit(hobi_server sv, Request& r) {
    TraceRange trace_range("server admit");
    hobi_ctx c = sv->ctx;
    hipStream_t s = c->stream;
    r.t_admit = Clock::now();
    const bool mixed = r.prm.precision == HOBI_MIXED;
    const DeviceProblem& d = r.pb->d;
    r.plan = mixed ? d.plan32 : d.plan64;
    r.m = std::max(1, r.prm.max_iter);
    const int n = 2 * r.nu, m = r.m;
    hipError_t e = hipSuccess;
#define SA(expr)                                                                   \
    if ((e = (expr)) != hipSuccess) {                                              \
        fail_request(r, e == hipErrorOutOfMemory ? HOBI_E_OOM : HOBI_E_HIP, #expr); \
        return r.status;                                                           \
    }
    SA(dalloc(&r.V, (size_t)(m + 1) * n));
    SA(dalloc(&r.H, (size_t)(m + 1) * m));
    SA(dalloc(&r.cs, m));
    SA(dalloc(&r.sn, m));
    SA(dalloc(&r.g, m + 1));
    SA(dalloc(&r.h1, m + 1));
    SA(dalloc(&r.h2, m + 1));
    SA(dalloc(&r.hn, 1));
    SA(dalloc(&r.yk, m));
    SA(dalloc(&r.dpart, (size_t)kDotBlocks * (m + 1)));
    SA(dalloc(&r.x, n));
    SA(dalloc(&r.scal, 4));
    if (r.prm.diag_scaling) {
        SA(dalloc(&r.z, n));
        SA(launch_scaling(d, r.prm.diag_scaling, d.dinv, s));
    }
    SA(hipMemsetAsync(r.x, 0, sizeof(double) * n, s));
    SA(launch_dots(d.rhs, 0, 1, d.rhs, n, r.dpart, s));
    SA(launch_reduce(r.dpart, 1, r.scal, 1, s));
    SA(hipMemcpyAsync(sv->h_res, r.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    SA(hipStreamSynchronize(s));
    r.bnorm = sv->h_res[0];
    if (!std::isfinite(r.bnorm)) {
        fail_request(r, HOBI_E_NUMERIC, "non-finite right-hand side");
        return r.status;
    }
    SA(launch_scale_copy(d.rhs, r.scal, r.V, n, s));
    SA(launch_init_g(r.scal, r.g, m, s));
    if (r.prm.tree_refine) {
        // the first correction solves T d = b from d = 0: the Krylov start above
        SA(dalloc(&r.xo, n));
        SA(dalloc(&r.ro, n));
        SA(dalloc(&r.tmp, n));
        SA(hipMemsetAsync(r.xo, 0, sizeof(double) * n, s));
        r.bnorm_b = r.rnorm = r.bnorm;
        r.tol_in = std::min(0.1, std::max(100.0 * r.prm.rtol, 0.5 * r.prm.rtol));
        r.total = r.steps = 0;
    }
#undef SA
    r.k = 0;
    r.est = r.bnorm > 0 ? 1.0 : 0.0;
    r.stats.ms_setup = r.pb->last.ms_setup;
    r.stats.pairs_per_matvec = (int64_t)d.nv * d.nn;
    return HOBI_OK;
}

// Forms x = V y, the energy and the caller-order outputs; frees the device state.
void finish(hobi_server sv, Request& r, bool converged) {
    TraceRange trace_range("server finish");
    hobi_ctx c = sv->ctx;
    hipStream_t s = c->stream;
    const int n = 2 * r.nu;
    hipError_t e = hipSuccess;
    if (r.k > 0) {
        if ((e = launch_trisolve(r.H, r.m + 1, r.k, r.g, r.yk, s)) == hipSuccess) {
            if (r.prm.diag_scaling) {
                e = launch_multi_axpy_scaled(r.V, n, r.k, r.yk, r.x, n, r.pb->d.dinv, s);
            } else {
                e = launch_multi_axpy(r.V, n, r.k, r.yk, 1.0, r.x, n, s);
            }
        }
    }
    if (e == hipSuccess) e = launch_gather(r.pb->d, r.x, false, s);
    if (e == hipSuccess) e = launch_reaction_energy(r.pb->d, r.pb->phi_reac, r.pb->e_dev, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sv->h_res, r.pb->e_dev, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fail_request(r, HOBI_E_HIP, hipGetErrorString(e));
    } else {
        r.energy = sv->h_res[0];
        std::vector<double> hu(n);
        hobi_status st = host_from_internal(r.pb, r.x, 0, hu.data());
        if (st != HOBI_OK) {
            fail_request(r, st, c->err);
        } else {
            const double scale = 4.0 * kPi * 332.0716;
            r.phi.assign(hu.begin(), hu.begin() + r.nu);
            r.dphi.assign(hu.begin() + r.nu, hu.end());
            for (double& v : r.phi) v *= scale;
            for (double& v : r.dphi) v *= scale;
            bool finite = std::isfinite(r.energy);
            for (double v : hu) finite = finite && std::isfinite(v);
            if (!finite)
                fail_request(r, HOBI_E_NUMERIC, "non-finite solution");
            else if (!converged)
                fail_request(r, HOBI_E_NOCONV, "GMRES reached max_iter");
        }
    }
    r.stats.iterations = r.k;
    r.stats.converged = converged ? 1 : 0;
    r.stats.est_residual = r.est;
    r.stats.ms_solve = std::chrono::duration<double, std::milli>(Clock::now() - r.t_admit).count();
    free_request_device(r);
}

// tree_refine: the end of one correction (the request's inner GMRES met its tolerance or the
// matvec budget).  The single-problem driver's outer step, with its kernels in its order:
// d = D^-1 V y, x += d, r = b - A x by the dense matvec, ||r||.  Then either the request
// finishes (as the driver stops) or the next correction starts from d = 0 on T d = r.
// Returns true when the request is finished (finish() has run).
bool refine_step(hobi_server sv, Request& r) {
    TraceRange trace_range("server refine step");
    hobi_ctx c = sv->ctx;
    hipStream_t s = c->stream;
    const DeviceProblem& d = r.pb->d;
    const bool mixed = r.prm.precision == HOBI_MIXED;
    const int n = 2 * r.nu;
    r.total += r.k;
    hipError_t e = hipSuccess;
    if (r.k > 0) {
        e = launch_trisolve(r.H, r.m + 1, r.k, r.g, r.yk, s);
        if (e == hipSuccess)
            e = r.prm.diag_scaling ? launch_multi_axpy_scaled(r.V, n, r.k, r.yk, r.x, n, d.dinv, s)
                                   : launch_multi_axpy(r.V, n, r.k, r.yk, 1.0, r.x, n, s);
    }
    if (e == hipSuccess) e = launch_add(r.xo, r.x, r.xo, n, s);
    if (e == hipSuccess) e = launch_gather(d, r.xo, mixed, s);
    if (e == hipSuccess) e = launch_pair(d, mixed, s);
    if (e == hipSuccess) e = launch_combine(d, r.xo, r.tmp, mixed, s);
    if (e == hipSuccess) e = launch_sub(d.rhs, r.tmp, r.ro, n, s);
    if (e == hipSuccess) e = launch_dots(r.ro, 0, 1, r.ro, n, r.dpart, s);
    if (e == hipSuccess) e = launch_reduce(r.dpart, 1, r.scal, 1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sv->h_res, r.scal, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fail_request(r, HOBI_E_HIP, hipGetErrorString(e));
        free_request_device(r);
        return true;
    }
    const double rn = sv->h_res[0];
    r.steps += 1;
    if (!std::isfinite(rn)) {
        fail_request(r, HOBI_E_NUMERIC, "refinement residual is not finite");
        free_request_device(r);
        return true;
    }
    const double est = rn / r.bnorm_b;
    if (est <= r.prm.rtol || r.total >= r.m || r.steps >= kMaxRefineSteps || rn > 0.9 * r.rnorm) {
        const bool conv = est <= r.prm.rtol;
        e = hipMemcpyAsync(r.x, r.xo, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            fail_request(r, HOBI_E_HIP, hipGetErrorString(e));
            free_request_device(r);
            return true;
        }
        r.k = 0;                          // the solution is in x already
        r.est = est;
        finish(sv, r, conv);
        r.stats.iterations = r.total;
        r.stats.est_residual = r.stats.true_residual = est;
        r.stats.refine_steps = r.steps;
        r.stats.dense_matvecs = r.steps;
        if (!conv && r.status == HOBI_E_NOCONV)
            r.message = "defect correction stopped after " + std::to_string(r.steps) + " outer steps";
        return true;
    }
    // the next correction: T d = r from d = 0, to max(rtol/2 ||b|| / ||r||, rtol/2), at most 1/2
    r.rnorm = rn;
    r.bnorm = rn;
    r.tol_in = std::min(0.5, std::max(0.5 * r.prm.rtol * r.bnorm_b / rn, 0.5 * r.prm.rtol));
    r.k = 0;
    r.est = 1.0;
    if ((e = hipMemsetAsync(r.x, 0, sizeof(double) * n, s)) != hipSuccess ||
        (e = launch_scale_copy(r.ro, r.scal, r.V, n, s)) != hipSuccess ||
        (e = launch_init_g(r.scal, r.g, r.m, s)) != hipSuccess) {
        fail_request(r, HOBI_E_HIP, hipGetErrorString(e));
        free_request_device(r);
        return true;
    }
    return false;
}

hipError_t ensure_capacity(hobi_server sv, size_t ndesc, size_t nitems) {
    hipError_t e = hipSuccess;
    if (ndesc > sv->cap_desc) {
        size_t cap = std::max<size_t>(ndesc, 2 * sv->cap_desc);
        if (sv->d_desc) (void)hipFree(sv->d_desc);
        if (sv->h_desc) (void)hipHostFree(sv->h_desc);
        if (sv->d_kdesc) (void)hipFree(sv->d_kdesc);
        if (sv->h_kdesc) (void)hipHostFree(sv->h_kdesc);
        if (sv->d_res) (void)hipFree(sv->d_res);
        if (sv->h_res) (void)hipHostFree(sv->h_res);
        if ((e = hipMalloc((void**)&sv->d_desc, cap * sizeof(ServeDesc))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void**)&sv->h_desc, cap * sizeof(ServeDesc))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&sv->d_kdesc, cap * sizeof(KrylovDesc))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void**)&sv->h_kdesc, cap * sizeof(KrylovDesc))) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&sv->d_res, (cap + 1) * sizeof(double))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void**)&sv->h_res, (cap + 1) * sizeof(double))) != hipSuccess) return e;
        sv->cap_desc = cap;
        sv->graph_dirty = true;
    }
    if (nitems > sv->cap_items) {
        size_t cap = std::max<size_t>(nitems, 2 * sv->cap_items);
        if (sv->d_items) (void)hipFree(sv->d_items);
        if (sv->h_items) (void)hipHostFree(sv->h_items);
        if ((e = hipMalloc((void**)&sv->d_items, cap * sizeof(ServeItem))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void**)&sv->h_items, cap * sizeof(ServeItem))) != hipSuccess) return e;
        sv->cap_items = cap;
        sv->graph_dirty = true;
    }
    return e;
}

// One tick: every active request advances one Arnoldi step: the batched diagonal scaling
// and matvec (phase A), the treecode requests' own matvec launches, then the batched
// Gram-Schmidt passes, normalisation and Givens updates (phase B).
hobi_status tick(hobi_server sv) {
    TraceRange trace_range("server tick");
    hipStream_t s = sv->ctx->stream;
    const size_t na = sv->active.size();
    // work lists: gather items, FP32 pair items, FP64 pair items, combine items
    size_t cnt[4] = {0, 0, 0, 0};
    for (auto& rp : sv->active) {
        const DeviceProblem& d = rp->pb->d;
        if (d.tree.on) continue;              // launched on its own below
        cnt[0] += (d.nn + kServeBlock - 1) / kServeBlock;
        cnt[rp->prm.precision == HOBI_MIXED ? 1 : 2] += (size_t)rp->plan.blocks;
        cnt[3] += (d.nv + kCombineVerts - 1) / kCombineVerts;
    }
    // the four lists live at fixed offsets (quarters of the item buffer), so that the
    // captured launches stay valid until the buffer has to grow
    hipError_t e =
        ensure_capacity(sv, na, 4 * std::max<size_t>(1, std::max(std::max(cnt[0], cnt[1]), std::max(cnt[2], cnt[3]))));
    if (e != hipSuccess) return host_fail(sv->ctx, HOBI_E_OOM, "server work-list allocation failed");
    const size_t t4 = sv->cap_items / 4;
    ServeItem* hl[4];
    const ServeItem* dl[4];
    for (int l = 0; l < 4; ++l) {
        hl[l] = sv->h_items + l * t4;
        dl[l] = sv->d_items + l * t4;
    }
    size_t fill[4] = {0, 0, 0, 0};
    int kcnt[kKrylovPhases] = {0, 0, 0, 0, 0, 0};
    for (size_t q = 0; q < na; ++q) {
        Request& r = *sv->active[q];
        const DeviceProblem& d = r.pb->d;
        const int n = 2 * r.nu;
        ServeDesc& sd = sv->h_desc[q];
        sd.u = r.V + (size_t)r.k * n;
        sd.y = r.V + (size_t)(r.k + 1) * n;
        KrylovDesc& kd = sv->h_kdesc[q];
        kd.vk = sd.u;
        kd.z = r.prm.diag_scaling ? r.z : nullptr;
        kd.V = r.V;
        kd.w = sd.y;
        kd.dpart = r.dpart;
        kd.h1 = r.h1;
        kd.h2 = r.h2;
        kd.hn = r.hn;
        kd.H = r.H;
        kd.cs = r.cs;
        kd.sn = r.sn;
        kd.g = r.g;
        kd.res = sv->d_res + q;
        kd.dinv = nullptr;
        kd.bnorm = r.bnorm;
        kd.n = n;
        kd.nu = r.nu;
        kd.k = r.k;
        kd.ldh = r.m + 1;
        {
            // item counts of each phase (the implicit lists of serve_internal.h)
            const int blocks = (n + kServeBlock - 1) / kServeBlock;
            const int per[kKrylovPhases] = {r.prm.diag_scaling ? blocks : 0, kDotBlocks * (r.k + 1), r.k + 1, blocks,
                                            kDotBlocks, 1};
            for (int ph = 0; ph < kKrylovPhases; ++ph) {
                kd.off[ph] = kcnt[ph];
                kcnt[ph] += per[ph];
            }
        }
        if (r.prm.diag_scaling) {
            // the matvec of the scaled system takes D^-1 v_k (the single-problem path's scaling)
            kd.dinv = d.dinv;
            sd.u = r.z;
        }
        sd.tri = d.tri;
        sd.w = d.w;
        sd.node64 = d.node64;
        sd.node32 = d.node32;
        sd.node_vid = d.node_vid;
        sd.blk_range = d.blk_range;
        sd.tgt32 = d.tgt32;
        sd.tgt64 = d.tgt64;
        sd.partial = d.partial;
        sd.inc_off = d.inc_off;
        sd.inc_ent = d.inc_ent;
        sd.coef = d.coef;
        sd.kappa = d.kappa;
        sd.eps = d.eps;
        sd.s32 = d.s32;
        sd.nv = d.nv;
        sd.nv_pad = d.nv_pad;
        sd.nn = d.nn;
        sd.gstart = r.plan.gstart;
        sd.blocks = r.plan.blocks;
        sd.slots = r.plan.slots;
        sd.rows = r.plan.rows;
        sd.slot = r.plan.slot;
        sd.mixed = r.prm.precision == HOBI_MIXED ? 1 : 0;
        sd.tpl = r.plan.tpl;
        sd.method = d.method;
        sd.pad = 0;
        if (d.tree.on) continue;
        for (int blk = 0; blk < (d.nn + kServeBlock - 1) / kServeBlock; ++blk)
            hl[0][fill[0]++] = ServeItem{(int)q, blk, 0, 0};
        const int pl = sd.mixed ? 1 : 2;
        for (int b = 0; b < r.plan.blocks; ++b) hl[pl][fill[pl]++] = ServeItem{(int)q, b, 0, 0};
        for (int blk = 0; blk < (d.nv + kCombineVerts - 1) / kCombineVerts; ++blk)
            hl[3][fill[3]++] = ServeItem{(int)q, blk, 0, 0};
    }
    for (int l = 0; l < 4; ++l) sv->h_counts[l] = (int)cnt[l];
    for (int ph = 0; ph < kKrylovPhases; ++ph) sv->h_counts[4 + ph] = kcnt[ph];
    sv->h_counts[4 + kKrylovPhases] = (int)na;
    const int* d_kcounts = sv->d_counts + 4;
    if ((e = hipMemcpyAsync(sv->d_desc, sv->h_desc, na * sizeof(ServeDesc), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(sv->d_kdesc, sv->h_kdesc, na * sizeof(KrylovDesc), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
        return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    for (int l = 0; l < 4; ++l)
        if (cnt[l] && (e = hipMemcpyAsync((void*)dl[l], hl[l], cnt[l] * sizeof(ServeItem), hipMemcpyHostToDevice,
                                          s)) != hipSuccess)
            return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    if ((e = hipMemcpyAsync(sv->d_counts, sv->h_counts, kServeCounts * sizeof(int), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    // phase A: diagonal scaling of v_k and the batched matvec; phase B: the Gram-Schmidt passes,
    // normalisation and Givens updates of every request.  Each is one launch sequence over the
    // device-side lists, captured once into a graph and replayed while the buffers keep their
    // addresses (the host rewrites only the lists and counts).
    auto phase_a = [&]() -> hipError_t {
        hipError_t le = launch_batched_diag(sv->d_kdesc, d_kcounts, s);
        if (le == hipSuccess) le = launch_batched_matvec(sv->d_desc, dl, sv->d_counts, s);
        return le;
    };
    auto phase_b = [&]() -> hipError_t { return launch_batched_krylov(sv->d_kdesc, d_kcounts, s); };
    if (sv->use_graph && (sv->graph_dirty || !sv->graph_exec || !sv->kgraph_exec)) {
        if (sv->graph_exec) (void)hipGraphExecDestroy(sv->graph_exec);
        if (sv->graph) (void)hipGraphDestroy(sv->graph);
        if (sv->kgraph_exec) (void)hipGraphExecDestroy(sv->kgraph_exec);
        if (sv->kgraph) (void)hipGraphDestroy(sv->kgraph);
        sv->graph_exec = sv->kgraph_exec = nullptr;
        sv->graph = sv->kgraph = nullptr;
        for (int which = 0; which < 2; ++which) {
            hipGraph_t* g = which == 0 ? &sv->graph : &sv->kgraph;
            hipGraphExec_t* x = which == 0 ? &sv->graph_exec : &sv->kgraph_exec;
            if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
            const hipError_t le = which == 0 ? phase_a() : phase_b();
            e = hipStreamEndCapture(s, g);
            if (le != hipSuccess || e != hipSuccess)
                return host_fail(sv->ctx, HOBI_E_HIP, "graph capture of the batched tick failed");
            if ((e = hipGraphInstantiate(x, *g, nullptr, nullptr, 0)) != hipSuccess)
                return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
        }
        sv->graph_dirty = false;
    }
    e = sv->use_graph ? hipGraphLaunch(sv->graph_exec, s) : phase_a();
    if (e != hipSuccess) return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    // treecode requests: the single-problem sequence (gather, proxy charges, items, combine)
    for (size_t q = 0; q < na; ++q) {
        Request& r = *sv->active[q];
        const DeviceProblem& d = r.pb->d;
        if (!d.tree.on) continue;
        const ServeDesc& sd = sv->h_desc[q];
        const bool mixed = r.prm.precision == HOBI_MIXED;
        if ((e = launch_gather(d, sd.u, mixed, s)) != hipSuccess || (e = launch_tree_proxies(d, mixed, s)) != hipSuccess ||
            (e = launch_tree_pairs(d, mixed, s)) != hipSuccess ||
            (e = launch_tree_combine(d, sd.u, sd.y, mixed, s)) != hipSuccess)
            return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    }
    e = sv->use_graph ? hipGraphLaunch(sv->kgraph_exec, s) : phase_b();
    if (e != hipSuccess) return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    if ((e = hipMemcpyAsync(sv->h_res, sv->d_res, na * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return host_fail(sv->ctx, HOBI_E_HIP, hipGetErrorString(e));
    return HOBI_OK;
}

void worker_main(hobi_server sv) {
    (void)hipSetDevice(sv->device);
    while (true) {
        std::vector<std::unique_ptr<Request>> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty()) sv->cv.wait(lk, [&] { return sv->stop || !sv->ready.empty(); });
            if (sv->stop) break;
            // the requests the preparation thread has built, in FIFO order
            while (!sv->ready.empty()) {
                admitted.push_back(std::move(sv->ready.front()));
                sv->ready.pop_front();
            }
            sv->active_count = (int)(sv->active.size() + admitted.size());
        }
        const auto t0 = Clock::now();
        std::vector<std::unique_ptr<Request>> finished;
        for (auto& r : admitted) {
            if (!r->pb) {                     // its problem could not be built
                finished.push_back(std::move(r));
            } else if (admit(sv, *r) != HOBI_OK || r->bnorm == 0.0) {
                if (r->status == HOBI_OK) finish(sv, *r, true);   // b = 0: u = 0
                else free_request_device(*r);
                finished.push_back(std::move(r));
            } else {
                sv->active.push_back(std::move(r));
            }
        }
        if (!sv->active.empty()) {
            hobi_status ts = tick(sv);
            sv->batch_sum += (double)sv->active.size();
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->st.ticks += 1;
            }
            std::vector<std::unique_ptr<Request>> still;
            for (size_t q = 0; q < sv->active.size(); ++q) {
                auto& r = sv->active[q];
                if (ts != HOBI_OK) {
                    fail_request(*r, ts, sv->ctx->err);
                    free_request_device(*r);
                    finished.push_back(std::move(r));
                    continue;
                }
                const double res = sv->h_res[q];
                r->k += 1;
                r->est = res;
                if (!std::isfinite(res)) {
                    fail_request(*r, HOBI_E_NUMERIC, "GMRES residual is not finite");
                    free_request_device(*r);
                    finished.push_back(std::move(r));
                } else if (r->prm.tree_refine && (res <= r->tol_in || r->total + r->k >= r->m)) {
                    if (refine_step(sv, *r)) finished.push_back(std::move(r));
                    else still.push_back(std::move(r));
                } else if (!r->prm.tree_refine && (res <= r->prm.rtol || r->k >= r->m)) {
                    finish(sv, *r, res <= r->prm.rtol);
                    finished.push_back(std::move(r));
                } else {
                    still.push_back(std::move(r));
                }
            }
            sv->active = std::move(still);
        }
        const double busy = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->st.busy_ms += busy;
            for (auto& r : finished) {
                sv->in_use -= r->footprint;
                if (r->status == HOBI_OK || r->status == HOBI_E_NOCONV) sv->st.completed += 1;
                else sv->st.failed += 1;
                sv->in_flight.erase(r->ticket);
                sv->done[r->ticket] = std::move(r);
            }
            sv->st.active = (int32_t)sv->active.size();
            sv->active_count = (int)sv->active.size();
            sv->st.bytes_in_use = sv->in_use;
            sv->st.mean_batch = sv->st.ticks ? sv->batch_sum / (double)sv->st.ticks : 0.0;
        }
        sv->prep_cv.notify_all();             // slots and budget may have been freed
    }
    for (auto& r : sv->active) free_request_device(*r);
    sv->active.clear();
}

// Preparation thread: FIFO over the pending requests while a slot is free (active, ready
// and in preparation together below max_slots) and the head fits in the budget; builds
// each request's problem on its own context and stream (host checks and ordering, device
// setup), concurrently with the worker's ticks, then hands the problem to the worker's
// context.
void prep_main(hobi_server sv) {
    (void)hipSetDevice(sv->device);
    while (true) {
        std::unique_ptr<Request> r;
        int64_t tree_limit = 0;
        bool alone = false;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->prep_cv.wait(lk, [&] {
                return sv->stop ||
                       (!sv->pending.empty() &&
                        sv->active_count + (int)sv->ready.size() + sv->preparing < sv->max_slots &&
                        sv->in_use + sv->pending.front()->footprint <= sv->budget);
            });
            if (sv->stop) break;
            r = std::move(sv->pending.front());
            sv->pending.pop_front();
            alone = sv->in_use == 0;
            sv->in_use += r->footprint;
            // what the budget leaves for the treecode buffers beyond the footprint charged
            // so far (the dense footprint, or that and the buffers' size measured before)
            tree_limit = sv->budget - sv->in_use + r->tree_charged;
            sv->preparing += 1;
            sv->st.pending = (int32_t)sv->pending.size();
            sv->st.bytes_in_use = sv->in_use;
            sv->st.peak_bytes = std::max(sv->st.peak_bytes, sv->in_use);
        }
        int64_t need = 0;
        const hobi_status st = problem_create_limited(sv->prep_ctx, r->nv, r->xyz.data(), r->nrm.data(), r->nf,
                                                      r->tri.data(), r->nc, r->qpos.data(), r->q.data(), &r->prm,
                                                      &r->pb, tree_limit, &need);
        if (st == HOBI_E_OOM && need > 0 && !alone && r->tree_charged == 0) {
            // its treecode buffers do not fit next to the admitted requests: back to the head
            // of the queue, charged their size, until enough of the budget is free
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->in_use -= r->footprint;
            r->footprint += need;
            r->tree_charged = need;
            sv->preparing -= 1;
            sv->st.bytes_in_use = sv->in_use;
            sv->pending.push_front(std::move(r));
            sv->st.pending = (int32_t)sv->pending.size();
            continue;
        }
        if (st != HOBI_OK) {
            fail_request(*r, st, sv->prep_ctx->err);
            r->pb = nullptr;
        } else {
            r->pb->ctx = sv->ctx;             // built and synchronised: from now on the worker's
        }
        const int64_t extra = r->pb ? tree_bytes(r->pb->d) - r->tree_charged : 0;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            r->footprint += extra;
            sv->in_use += extra;
            sv->st.bytes_in_use = sv->in_use;
            sv->st.peak_bytes = std::max(sv->st.peak_bytes, sv->in_use);
            sv->preparing -= 1;
            sv->ready.push_back(std::move(r));
        }
        sv->cv.notify_all();
    }
}

}  // namespace

extern "C" {

hobi_status hobi_server_create(hobi_ctx ctx, int64_t hbm_budget_bytes, int32_t max_slots, int32_t use_graph,
                               hobi_server* out) {
    if (!ctx || !out) return HOBI_E_ARG;
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || max_slots < 1) return host_fail(ctx, HOBI_E_ARG, "budget and slots must be positive");
    hobi_server sv = new hobi_server_s();
    sv->device = ctx->device;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    sv->use_graph = use_graph != 0;
    if (hobi_ctx_create(ctx->device, nullptr, &sv->ctx) != HOBI_OK ||
        hobi_ctx_create(ctx->device, nullptr, &sv->prep_ctx) != HOBI_OK) {
        if (sv->ctx) hobi_ctx_destroy(sv->ctx);
        delete sv;
        return host_fail(ctx, HOBI_E_HIP, "could not create the server streams");
    }
    if (hipMalloc((void**)&sv->d_counts, kServeCounts * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&sv->h_counts, kServeCounts * sizeof(int)) != hipSuccess ||
        ensure_capacity(sv, 16, 3 * 4096) != hipSuccess) {
        hobi_server_destroy(sv);
        return host_fail(ctx, HOBI_E_OOM, "server buffers");
    }
    sv->worker = std::thread(worker_main, sv);
    sv->prep = std::thread(prep_main, sv);
    *out = sv;
    return HOBI_OK;
}

hobi_status hobi_server_submit(hobi_server sv, int32_t nv, const double* xyz, const double* nrm, int32_t nf,
                               const int32_t* tri, int32_t nc, const double* qpos, const double* q,
                               const hobi_params* params, uint64_t* ticket) {
    if (!sv || !ticket) return HOBI_E_ARG;
    if (!xyz || !nrm || !tri || !qpos || !q || nv < 4 || nf < 4 || nc < 1) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->last_error = "bad sizes or NULL inputs";
        return HOBI_E_ARG;
    }
    auto r = std::make_unique<Request>();
    r->nv = nv;
    r->nf = nf;
    r->nc = nc;
    r->xyz.assign(xyz, xyz + 3 * (size_t)nv);
    r->nrm.assign(nrm, nrm + 3 * (size_t)nv);
    r->tri.assign(tri, tri + 3 * (size_t)nf);
    r->qpos.assign(qpos, qpos + 3 * (size_t)nc);
    r->q.assign(q, q + nc);
    hobi_params_default(&r->prm);
    if (params) r->prm = *params;
    if (r->prm.tree_refine != 0 && (r->prm.tree_refine != 1 || !(r->prm.tree_theta > 0))) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->last_error = "tree_refine must be 0, or 1 with tree_theta > 0";
        return HOBI_E_ARG;
    }
    r->prm.restart = r->prm.max_iter;
    r->nu = r->prm.method == HOBI_LOWER_ORDER ? nf : nv;
    r->footprint = footprint_bytes(sv->device, nv, nf, nc, std::max(1, r->prm.max_iter), r->prm.method,
                                   r->prm.precision == HOBI_MIXED);
    if (r->prm.tree_refine) r->footprint += 3LL * 2 * r->nu * (int64_t)sizeof(double);   // xo, ro, tmp
    std::lock_guard<std::mutex> lk(sv->mu);
    if (r->footprint > sv->budget) {
        sv->last_error = "request footprint exceeds the server budget";
        return HOBI_E_OOM;
    }
    r->ticket = sv->next_ticket++;
    *ticket = r->ticket;
    sv->in_flight.insert(r->ticket);
    sv->pending.push_back(std::move(r));
    sv->st.submitted += 1;
    sv->st.pending = (int32_t)sv->pending.size();
    sv->prep_cv.notify_all();
    return HOBI_OK;
}

hobi_status hobi_server_poll(hobi_server sv, uint64_t ticket, double* phi, double* dphi, double* e_sol,
                             hobi_stats* st) {
    if (!sv) return HOBI_E_ARG;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->done.find(ticket);
        if (it == sv->done.end()) {
            if (sv->in_flight.count(ticket)) return HOBI_E_BUSY;
            sv->last_error = "unknown ticket";
            return HOBI_E_ARG;
        }
        r = std::move(it->second);
        sv->done.erase(it);
        if (r->status != HOBI_OK) sv->last_error = r->message;
    }
    if (phi && !r->phi.empty()) std::memcpy(phi, r->phi.data(), sizeof(double) * r->nu);
    if (dphi && !r->dphi.empty()) std::memcpy(dphi, r->dphi.data(), sizeof(double) * r->nu);
    if (e_sol) *e_sol = r->energy;
    if (st) *st = r->stats;
    return r->status;
}

hobi_status hobi_server_get_stats(hobi_server sv, hobi_server_stats* out) {
    if (!sv || !out) return HOBI_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    return HOBI_OK;
}

const char* hobi_server_last_error(hobi_server sv) { return sv ? sv->last_error.c_str() : "null server"; }

void hobi_server_destroy(hobi_server sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    sv->prep_cv.notify_all();
    if (sv->prep.joinable()) sv->prep.join();
    if (sv->worker.joinable()) sv->worker.join();
    for (auto& r : sv->ready) free_request_device(*r);
    sv->ready.clear();
    if (sv->ctx) (void)hipStreamSynchronize(sv->ctx->stream);
    if (sv->graph_exec) (void)hipGraphExecDestroy(sv->graph_exec);
    if (sv->graph) (void)hipGraphDestroy(sv->graph);
    if (sv->kgraph_exec) (void)hipGraphExecDestroy(sv->kgraph_exec);
    if (sv->kgraph) (void)hipGraphDestroy(sv->kgraph);
    if (sv->d_desc) (void)hipFree(sv->d_desc);
    if (sv->d_kdesc) (void)hipFree(sv->d_kdesc);
    if (sv->h_kdesc) (void)hipHostFree(sv->h_kdesc);
    if (sv->d_items) (void)hipFree(sv->d_items);
    if (sv->d_counts) (void)hipFree(sv->d_counts);
    if (sv->d_res) (void)hipFree(sv->d_res);
    if (sv->h_desc) (void)hipHostFree(sv->h_desc);
    if (sv->h_items) (void)hipHostFree(sv->h_items);
    if (sv->h_counts) (void)hipHostFree(sv->h_counts);
    if (sv->h_res) (void)hipHostFree(sv->h_res);
    if (sv->ctx) hobi_ctx_destroy(sv->ctx);
    if (sv->prep_ctx) hobi_ctx_destroy(sv->prep_ctx);
    delete sv;
}

}  // extern "C"
