/*
 * hobi.h -- C ABI of the MI355X implementation of the higher-order boundary-integral
 * Poisson-Boltzmann method (HOBI-PB, arXiv 1301.5914).
 *
 * Problem (Section 2, eqs. eq1-radiation with the linearised eq2): a closed molecular
 * surface Gamma given as a triangulation with unit outward vertex normals; Nc point
 * charges q_k at x_k inside it; dielectric eps1 inside, eps2 and inverse Debye length
 * kappa outside.  Results: the surface potential phi and its normal derivative
 * dphi/dn at the vertices (the unknowns of Section 2.2) and the electrostatic
 * solvation energy E_sol (eq. solvation_energy, Section 2.5).
 *
 * Conventions shared by every entry point:
 *  - Lengths in Angstrom, charges in units of e.  phi is returned in kcal/(mol e),
 *    dphi/dn in kcal/(mol e A), E_sol in kcal/mol (Coulomb constant 332.0716).
 *  - Internal vectors u = (phi_1..phi_Nv, dphi_1..dphi_Nv) used by hobi_matvec and
 *    hobi_energy are in internal units: Green's functions G0 = 1/(4 pi r) and
 *    Gk = exp(-kappa r)/(4 pi r) (eq. eq_potential) with charges in e, i.e. phi in e/A.
 *    Output phi = 4 pi * 332.0716 * internal phi.
 *  - eps = eps2 / eps1 in the kernels K1..K4 (eq. Eq_Ls; the printed eps1/eps2 is read
 *    as inverted) and the source terms S1, S2 (eq. Eq_Ss) carry a factor 1/eps1.
 *  - Arrays are row-major and contiguous.  The library copies every input during the
 *    call and never keeps a caller pointer after returning.  The caller owns every
 *    input and output buffer; handles own all device memory and free it on destroy.
 *  - Every call returns a hobi_status; on failure the message is available from
 *    hobi_last_error() on the context.  Inputs are never repaired silently, except
 *    that normals within 1e-6 of unit length are renormalised.
 *  - One context per host thread.  Calls on one context are serialised on its stream.
 */
#ifndef HOBI_H
#define HOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hobi_status {
    HOBI_OK = 0,
    HOBI_E_ARG = 1,             /* bad argument (null pointer, size, parameter range)      */
    HOBI_E_MESH = 2,            /* not a closed oriented 2-manifold, degenerate triangle,   */
                                /* a triangle whose orientation disagrees with the sum of */
                                /* its vertex normals, or a normal along an edge          */
    HOBI_E_CHARGE_OUTSIDE = 3,  /* a charge is not enclosed by the surface                  */
    HOBI_E_NOCONV = 4,          /* GMRES hit max_iter; outputs hold the last iterate        */
    HOBI_E_OOM = 5,             /* device allocation failed / over the serving budget      */
    HOBI_E_HIP = 6,             /* a HIP runtime call failed                                */
    HOBI_E_NUMERIC = 7,         /* NaN or Inf in the inputs or in a result                 */
    HOBI_E_BUSY = 8             /* serving: the request is not finished yet                */
} hobi_status;

/* Arithmetic of the dense pair sum (the regular far field, eqdbef3/eqdbef4). */
enum {
    HOBI_FP64 = 0,   /* every step in FP64                                              */
    HOBI_MIXED = 1   /* pair kernel in FP32, tile sums folded into FP64 accumulators;   */
                     /* singular correction, GMRES, sources and energy stay FP64        */
};

/* Discretisation of the integral equations. */
enum {
    HOBI_HIGHER_ORDER = 0,  /* curved 10-node triangles, unknowns at the vertices, 4-point    */
                            /* regular and 16-point singular rules (Sections 2.2-2.3)         */
    HOBI_LOWER_ORDER = 1    /* flat triangles, centroid collocation: one unknown pair and one */
                            /* quadrature point per triangle, the self term dropped           */
                            /* (the low-order scheme, eqdbef1/eqdbef2)                        */
};

typedef struct hobi_ctx_s* hobi_ctx;
typedef struct hobi_problem_s* hobi_problem;
typedef struct hobi_server_s* hobi_server;

typedef struct hobi_params {
    double eps1;        /* solute dielectric (> 0), default 1                               */
    double eps2;        /* solvent dielectric (> 0), default 80                             */
    double kappa;       /* inverse Debye length in 1/A (>= 0), default 0.1257; kappa times  */
                        /* the surface's bounding-box diagonal must stay below 2.5e6       */
    double rtol;        /* GMRES stop: ||b - A u|| / ||b|| <= rtol (estimated), default 1e-6*/
    int32_t max_iter;   /* total matvecs allowed, default 200                               */
    int32_t restart;    /* GMRES(m) restart length, default 200                             */
    int32_t precision;  /* HOBI_FP64 or HOBI_MIXED, default HOBI_FP64                       */
    int32_t method;     /* HOBI_HIGHER_ORDER (default) or HOBI_LOWER_ORDER                  */
    int32_t diag_scaling; /* right preconditioner of GMRES (same solution; the monitored     */
                        /* residual is still ||b - A u|| / ||b||).  2 (default): Jacobi, the  */
                        /* inverse of A's own diagonal (1/2 (1+eps) and 1/2 (1+1/eps) minus  */
                        /* each vertex's singular terms on its own unknowns; for the lower-  */
                        /* order method, which has none, as 1).  1: the two row blocks'      */
                        /* constants 1/(1/2 (1+eps)) and 1/(1/2 (1+1/eps)).  0: A u = b as   */
                        /* written                                                           */
    /* Treecode form of the regular (dense) sum, either method.  0 (default):
     * the dense sum.  > 0: a cluster-particle treecode with opening parameter tree_theta.
     * The quadrature nodes in order are cut into leaves of tree_leaf nodes, joined pairwise
     * level by level into a binary cluster tree; the target vertices in order into batches
     * of tree_batch.  Each batch walks the tree from the root: a cluster whose bounding
     * sphere and the batch's satisfy r_b + r_c <= tree_theta |c_b - c_c|, and which has no
     * triangle incident to a target of the batch, is taken by the Green's functions
     * interpolated in the source point on the (tree_degree + 1)^3 Chebyshev points of its
     * box; a leaf that fails is summed directly; a parent that fails is opened (with the
     * lower-order method a cluster is rejected for a batch whose sites overlap its nodes).
     * The partition is fixed at problem creation.  hobi_field takes the treecode with the
     * higher-order method only.                                                          */
    double tree_theta;  /* >= 0, default 0                                                  */
    int32_t tree_degree; /* interpolation degree n, 1..7, default 5                        */
    int32_t tree_leaf;  /* nodes per leaf, a multiple of 64 in [64, 2^24], default 256      */
    int32_t tree_batch; /* targets per batch: 128, 256 or 512, default 128                  */
    /* With tree_theta > 0, what hobi_solve solves.  0 (default): the treecode's own system
     * (GMRES with the treecode matvec; its residuals are the treecode operator's).  1: the
     * dense system A u = b of tree_theta = 0, by defect correction (iterative refinement
     * with an approximate operator): from u = 0, each outer step solves T d = r by GMRES
     * with the treecode matvec T (same preconditioner, restart and precision), to the
     * relative tolerance min(100 rtol, 1/10) in the first step and
     * max(rtol/2 ||b|| / ||r||, rtol/2), at most 1/2, after it, adds d to u and recomputes
     * r = b - A u with the dense matvec.  It stops when ||r|| / ||b|| <= rtol (converged:
     * a dense residual, not an estimate), when the inner matvecs reach max_iter, after 16
     * outer steps, or when an outer step shrinks ||r|| by less than a tenth
     * (HOBI_E_NOCONV for the last three).  hobi_stats.iterations counts the treecode
     * matvecs, refine_steps the outer steps and dense_matvecs the dense ones; the true
     * residual is the last outer residual (no extra matvec).  hobi_matvec and hobi_field
     * of such a problem still use the treecode.  The server takes it too:
     * each request's outer steps run between its ticks, with the same arithmetic, so a
     * served result equals hobi_solve's. */
    int32_t tree_refine; /* 0 or 1, default 0; 1 needs tree_theta > 0                       */
} hobi_params;

typedef struct hobi_stats {
    int32_t iterations;        /* matvecs inside GMRES                                      */
    int32_t converged;         /* 1 if the estimated residual reached rtol                  */
    double est_residual;       /* GMRES estimate of ||b - A u|| / ||b||                     */
    double true_residual;      /* recomputed ||b - A u|| / ||b|| (one extra matvec)         */
    double ms_setup;           /* geometry + quadrature + singular coefficients + sources   */
    double ms_solve;           /* GMRES wall time on the stream                             */
    double ms_energy;          /* solvation energy                                          */
    int64_t pairs_per_matvec;  /* Nv * 4 Nf (target vertex, regular node) pairs; Nf * Nf for  */
                               /* the lower-order method                                    */
    /* Per-kernel device time, accumulated over the calls since the last reset when the
     * context has profiling enabled (HIP events on the context's stream), else 0.        */
    double ms_pair_kernel;
    int64_t pair_launches;
    double ms_gather, ms_combine, ms_krylov;
    double ms_field_kernel;    /* pair sums of hobi_field (R, its gradient, solid angle)     */
    int64_t field_launches;
    int64_t tree_far_pairs;    /* treecode: (batch, cluster) pairs taken by the proxies      */
    int64_t tree_near_pairs;   /* and (batch, leaf) pairs summed directly (0 without it)     */
    int64_t field_tree_far_pairs;  /* the same for the last hobi_field call's point batches   */
    int64_t field_tree_near_pairs;
    int32_t refine_steps;      /* tree_refine: outer steps of the last solve (else 0)       */
    int32_t dense_matvecs;     /* tree_refine: dense matvecs of the last solve (else 0)      */
} hobi_stats;

/* Fills p with the defaults listed in hobi_params. */
void hobi_params_default(hobi_params* p);

/* ---- context ---------------------------------------------------------------------
 * device: HIP device ordinal.  stream: a hipStream_t to run on, or NULL for a stream
 * owned by the context.  Fails with HOBI_E_ARG / HOBI_E_HIP. */
hobi_status hobi_ctx_create(int device, void* stream, hobi_ctx* out);
void hobi_ctx_destroy(hobi_ctx ctx);
/* Message of the last failure on this context (valid until the next call). */
const char* hobi_last_error(hobi_ctx ctx);
/* Enables (1) or disables (0) per-kernel HIP-event timing into hobi_stats. */
hobi_status hobi_ctx_set_profiling(hobi_ctx ctx, int32_t enable);
/* The hipStream_t the context runs on. */
void* hobi_ctx_stream(hobi_ctx ctx);

/* ---- problem ---------------------------------------------------------------------
 * Copies and validates the inputs and runs the per-molecule setup on the context's
 * stream (routines (1)-(4) of Section 2.6): curved 10-node elements (Section 2.2),
 * 4-point Gauss-Radau nodes, the singular 16-point Duffy/Gauss-Legendre
 * coefficients (Section 2.3), source terms S1/S2 (eq. Eq_Ss) and the check that every
 * charge is enclosed.  With params->method = HOBI_LOWER_ORDER the setup is that of the
 * low-order scheme instead (flat triangles: centroids, face normals, areas), and every
 * per-unknown array below ("[nv]", "[2 nv]") has one entry per triangle ([nf], [2 nf], in
 * the caller's triangle order) instead of one per vertex.
 *   xyz [nv][3], nrm [nv][3]: vertex positions and unit outward normals (host).
 *   tri [nf][3]: 0-based vertex ids, counter-clockwise seen from outside (host).  The
 *        first vertex of each triangle is significant: the 4-point rule is anchored at
 *        it.
 *   qpos [nc][3], q [nc]: charges (host); nc >= 1.
 *   params: NULL for the defaults.
 * Errors: HOBI_E_ARG, HOBI_E_MESH, HOBI_E_CHARGE_OUTSIDE, HOBI_E_NUMERIC, HOBI_E_OOM,
 * HOBI_E_HIP. */
hobi_status hobi_problem_create(hobi_ctx ctx, int32_t nv, const double* xyz,
                                const double* nrm, int32_t nf, const int32_t* tri,
                                int32_t nc, const double* qpos, const double* q,
                                const hobi_params* params, hobi_problem* out);
void hobi_problem_destroy(hobi_problem pb);
/* Switches the pair-kernel arithmetic (HOBI_FP64 / HOBI_MIXED) of an existing problem.  The
 * problem holds the partial-sum rows of its current precision's pair plan; a switch to a
 * plan that needs more waits for the problem's queued work and reallocates them (HOBI_E_OOM
 * if that fails; the problem then keeps its precision).  HOBI_E_ARG for another value. */
hobi_status hobi_problem_set_precision(hobi_problem pb, int32_t precision);
/* Replaces eps1, eps2 and kappa and re-runs the whole device part of the setup (curved
 * elements, regular nodes, singular coefficients, source terms) on the resident surface
 * and charges, e.g. the same molecule in another solvent.  Synchronous.
 * Errors: HOBI_E_ARG, HOBI_E_HIP. */
hobi_status hobi_problem_set_dielectric(hobi_problem pb, double eps1, double eps2, double kappa);
/* Replaces rtol / max_iter / restart. */
hobi_status hobi_problem_set_solver(hobi_problem pb, double rtol, int32_t max_iter,
                                    int32_t restart);

/* ---- solve: GMRES on A u = (S1, S2), then the energy (Sections 2.2-2.5) ------------
 * phi, dphi: [nv] host outputs (nullable); e_sol: host output (nullable);
 * st: nullable.  Returns HOBI_E_NOCONV (outputs hold the last iterate) when the
 * estimated residual did not reach rtol within max_iter matvecs. */
hobi_status hobi_solve(hobi_problem pb, double* phi, double* dphi, double* e_sol,
                       hobi_stats* st);

/* ---- the hot path: y = A u (eqdbef3 + eqdbef4 + eqdbef5 + eqdbef6) ----------------
 * u, y: [2 nv] FP64 in internal units and the caller's vertex order.
 * on_device = 0: host pointers; 1: device pointers valid on the context's stream (the
 * call is asynchronous with respect to the host in that case). */
hobi_status hobi_matvec(hobi_problem pb, const double* u, double* y, int32_t on_device);

/* ---- allocation-free variant of hobi_matvec, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid it).
 * Computes the same y = A u as hobi_matvec for a dense-sum problem (tree_theta = 0), with
 * the pair sum's partial rows in a static work space of the library (64 MiB per device,
 * a 64 KiB table of node-group starts and the rows; it lives in the library's code object
 * and each device that runs the library holds it until the process ends) instead of the
 * problem's own buffer.  The node groups are cut down to what fits (fewer groups than
 * hobi_matvec on large problems), so the sum runs in a different order and the result
 * equals hobi_matvec's up to rounding, not bit for bit.  Allocates nothing and calls no
 * hipMalloc or hipFree; launches only kernels on the context's stream (asynchronous).
 * u, y: [2 nv] FP64 device pointers valid on the context's stream, internal units, the
 * caller's order (as hobi_matvec with on_device = 1); they may not alias.
 * Every call on a device shares that device's work space and overwrites it (the group
 * table is rewritten by each call): calls that overlap on one device -- on different
 * streams, contexts or host threads -- race and give wrong results.
 * Errors: HOBI_E_ARG (NULL vector; a treecode problem; a problem whose slots' partial rows
 * for a single row of node groups (one group in FP64, four in mixed precision) exceed the
 * work space, about nv > 4 million), HOBI_E_HIP. */
hobi_status hobi_matvec_noalloc(hobi_problem pb, const double* u, double* y);

/* ---- solvation energy of a given u (eq. solvation_energy, 4-point rule on every
 * triangle; Section 2.6 routine (6)).  u: [2 nv] internal units; e_sol: kcal/mol. */
hobi_status hobi_energy(hobi_problem pb, const double* u, int32_t on_device,
                        double* e_sol);

/* ---- potential and field at points off the surface (Section 2.1: the representation
 * formulas eqbim_1 in the solute and eqbim_2 in the solvent, combined with the jump
 * conditions into the kernels of eq. solvation_energy).  With the reaction potential
 *     R(x) = integral over the surface of K1 dphi/dnu + K2 phi
 * (the quadrature of the energy: the 4-point rule on every triangle, or the centroid rule
 * of the lower-order method) and S1(x) = sum_k q_k G0(x, x_k) / eps1:
 *     x inside the surface:   phi(x) = S1(x) + R(x)
 *     x outside (solvent):    phi(x) = (S1(x) + R(x)) / eps,      E = -grad phi.
 * The side is read from the double layer of a unit density (solid-angle fraction of the
 * surface seen from x, 1 inside and 0 outside): inside when it exceeds 1/2.  A charge
 * within 1e-6 A of a point is left out of that point's S1 (so q_k times reac_field at x_k
 * is the solvation force on charge k).
 * u: [2 nv] internal units (as for hobi_energy), host or device per on_device.
 * points: [np][3] host, A; np >= 0 (np = 0 is a no-op).
 * Outputs: host arrays in the points' order, each may be NULL:
 *   phi [np] total potential, kcal/(mol e);   field [np][3] E, kcal/(mol e A);
 *   reac [np] R;   reac_field [np][3] -grad R;   inside [np] 1 inside, 0 outside.
 * The pair sums run in the problem's precision (mixed: FP32 pairs, FP64 accumulation).
 * With tree_theta > 0 (higher-order method) the sums over the surface take the problem's
 * treecode: the points
 * in Morton order form batches of 256 that walk its cluster tree with the acceptance test
 * alone (no incidence rule off the surface); accepted clusters add R, grad R and the
 * solid angle from their proxy charges (the solid angle from the charge of the unit
 * double layer), near leaves their nodes directly.  Its partial sums take one row per
 * (slot of points, cluster) pair, about 6 KB per point at the default parameters; larger
 * maps run in passes of at most 4 GiB of rows.
 * There is no near-singular treatment: within about one edge length of the surface the
 * rule's error grows, and a point on the surface is not a valid argument.
 * Synchronous: returns when the outputs are written.  The work space it allocates on the
 * first call (and on larger calls) stays with the problem until destroy.
 * Errors: HOBI_E_ARG (NULL u, NULL points with np > 0, np < 0, too many points, points so
 * far from the surface that kappa times their distance from it could reach 2.5e6),
 * HOBI_E_NUMERIC (non-finite point), HOBI_E_OOM, HOBI_E_HIP. */
hobi_status hobi_field(hobi_problem pb, const double* u, int32_t on_device, int32_t np,
                       const double* points, double* phi, double* field, double* reac,
                       double* reac_field, int32_t* inside);

/* ---- the FP64 pair sums' own arithmetic, for checking it against a reference -------
 * y[i] = f(x[i]) on the context's device, with the routines the FP64 pair kernel uses:
 *   HOBI_MATH_EXP_NEG: exp(-x), 0 <= x < 5e6 (Tang's table-driven method, 256 table values);
 *   HOBI_MATH_RSQRT:   1 / sqrt(x), x > 0 (hardware estimate and one third-order step).
 * x, y: [n] host arrays, n >= 0.  Synchronous.
 * Errors: HOBI_E_ARG (unknown fn, NULL array, an argument outside the domain), HOBI_E_HIP. */
enum { HOBI_MATH_EXP_NEG = 0, HOBI_MATH_RSQRT = 1 };
hobi_status hobi_device_math(hobi_ctx ctx, int32_t fn, int32_t n, const double* x, double* y);

/* ---- inspection of the setup (for verification), caller's vertex/triangle order ---
 * y, ny: [nf][4][3] regular quadrature nodes and unit normals; w: [nf][4] weight times
 * Jacobian (Section 2.2); lower-order method: [nf][3], [nf][3], [nf] (centroid, face
 * normal, area).  Any pointer may be NULL. */
hobi_status hobi_get_nodes(hobi_problem pb, double* y, double* ny, double* w);
/* b: [2 nv] right-hand side (S1, S2) in internal units. */
hobi_status hobi_get_rhs(hobi_problem pb, double* b);
/* Zeroes the per-kernel timers reported in hobi_stats; hobi_get_stats reads them. */
hobi_status hobi_reset_stats(hobi_problem pb);
hobi_status hobi_get_stats(hobi_problem pb, hobi_stats* st);

/* ---- request server: continuous batching of many solves on one device -------------
 * Two threads, each with a stream of its own.  Submitted requests wait in FIFO order
 * until a slot is free and their device footprint (surface, quadrature data, Krylov basis
 * of max_iter + 1 vectors) fits in hbm_budget_bytes next to the admitted ones; the
 * preparation thread then builds the request's problem (host checks and ordering, device
 * setup) while the worker's ticks run, and the worker advances every built request one
 * GMRES iteration per scheduler tick, all together: each tick does one batched diagonal
 * scaling, gather, pair-sum and combine launch for every request, then one batched launch
 * per Gram-Schmidt, normalisation and Givens phase for every request (two launch sequences,
 * each captured once in a HIP graph when use_graph is 1).  A request with
 * tree_theta > 0 runs its own treecode matvec launches in the tick instead (the sequence of
 * hobi_matvec); it is admitted on its dense footprint, and its treecode buffers, which
 * depend on the partition, are charged when its problem is built with the budget's rest as
 * their limit: if they do not fit, the request returns to the head of the queue charged
 * their size and waits until they do, so bytes_in_use never exceeds the budget (a request
 * that cannot fit even alone fails with HOBI_E_OOM).  Requests
 * arriving during a tick join at the next one; finished requests leave at the end of the
 * tick that finished them.  A request's arithmetic depends only on that request (its
 * split over waves is fixed by its own size and the device), so its results are
 * bit-for-bit the same alone, in any mix, and as hobi_solve with restart = max_iter.
 * Served solves do not restart: max_iter bounds the Krylov basis.
 * Thread safety: submit, poll and get_stats may be called from any thread. */
typedef struct hobi_server_stats {
    int64_t submitted, completed, failed;  /* requests                                      */
    int64_t ticks;                         /* scheduler ticks so far                          */
    int32_t active, pending;               /* requests on the device / waiting               */
    double mean_batch;                     /* mean active requests per tick                   */
    int64_t bytes_in_use, peak_bytes;      /* admitted footprint, now and at its maximum      */
    double busy_ms;                        /* wall time the worker spent with work in hand    */
} hobi_server_stats;

/* device: from ctx (the server creates its own two streams and threads).
 * hbm_budget_bytes > 0; max_slots >= 1.  Errors: HOBI_E_ARG, HOBI_E_HIP. */
hobi_status hobi_server_create(hobi_ctx ctx, int64_t hbm_budget_bytes, int32_t max_slots,
                               int32_t use_graph, hobi_server* out);
/* Inputs as hobi_problem_create (copied during the call); params NULL for the defaults.
 * Returns a ticket.  HOBI_E_OOM if the request alone exceeds the budget, HOBI_E_ARG for
 * bad sizes/pointers; mesh and charge errors are reported by hobi_server_poll. */
hobi_status hobi_server_submit(hobi_server sv, int32_t nv, const double* xyz, const double* nrm,
                               int32_t nf, const int32_t* tri, int32_t nc, const double* qpos,
                               const double* q, const hobi_params* params, uint64_t* ticket);
/* HOBI_E_BUSY while the request waits or runs.  Once it has finished: copies phi, dphi
 * ([nv], kcal/(mol e) and kcal/(mol e A), nullable), e_sol (kcal/mol, nullable) and st
 * (nullable), forgets the ticket and returns the request's status (HOBI_OK,
 * HOBI_E_NOCONV with the last iterate, or the error that stopped it; the message is then
 * in hobi_server_last_error).  Unknown ticket: HOBI_E_ARG. */
hobi_status hobi_server_poll(hobi_server sv, uint64_t ticket, double* phi, double* dphi,
                             double* e_sol, hobi_stats* st);
hobi_status hobi_server_get_stats(hobi_server sv, hobi_server_stats* out);
const char* hobi_server_last_error(hobi_server sv);
/* Stops the worker (requests still waiting or running are dropped) and frees everything. */
void hobi_server_destroy(hobi_server sv);

#ifdef __cplusplus
}
#endif

#endif /* HOBI_H */
