// Device-side descriptors of the request server's batched matvec.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "hobi.h"
#include "hobi_device.h"

namespace hobi {

constexpr int kServeBlock = 256;       // threads per block of the batched kernels
constexpr int kServeGridPair = 2048;  // fixed grids: the kernels walk the item lists
constexpr int kServeGridSmall = 1024;
constexpr int kServeCounts = 11;   // 4 matvec list counts, 6 Krylov phase counts, requests

// One active request as the batched kernels see it during one tick.
struct ServeDesc {
    const double* u;        // Krylov vector v_k (internal order)
    double* y;              // output A v_k (the next Krylov slot)
    const int* tri;
    const double* w;
    NodeD* node64;
    NodeF* node32;
    const int4* node_vid;
    const int2* blk_range;
    const float* tgt32;
    const double* tgt64;
    double* partial;        // [workers][2][slot] (the pair plan's rows)
    const int* gstart;      // the pair plan's node-group starts
    const int* inc_off;
    const int* inc_ent;
    const double* coef;
    double kappa;
    double eps;
    double s32;             // scale of the FP32 positions
    int nv, nv_pad, nn;
    int blocks, slots, rows, slot;      // the pair plan (the single-problem plan)
    int mixed;
    int tpl;                // targets per lane of the request's pair plan (the single-problem plan)
    int method;             // HOBI_HIGHER_ORDER or HOBI_LOWER_ORDER
    int pad;
};

// One unit of work: request `req`; a = block of the pair plan for the pair kernels, node or
// vertex block for gather and combine.
struct ServeItem {
    int req, a, b, pad;
};

// Item lists and their counts, in launch order: gather, FP32 pair, FP64 pair, combine.
hipError_t launch_batched_matvec(const ServeDesc* desc, const ServeItem* const items[4], const int* counts,
                                 hipStream_t s);

// One active request's Arnoldi step as the batched Krylov kernels see it during one tick:
// the diagonal scaling of v_k before the matvec, then two classical Gram-Schmidt passes of
// w = A v_k against v_0 .. v_k, its normalisation and the Givens update, with the arithmetic
// of the single-problem GMRES (krylov_tile.h).  The kernels walk implicit item lists: phase
// p of request q holds items [off[p], off[p] + its count) of that phase, counts following
// from n and k (diag: ceil(n/256) if scaled, else 0; dots: 64 (k + 1); reduce: k + 1;
// axpy: ceil(n/256); norm dots: 64; single: 1).
constexpr int kKrylovPhases = 6;
static_assert(kServeCounts == 4 + kKrylovPhases + 1, "count layout");
struct KrylovDesc {
    const double* vk;       // v_k
    double* z;              // D^-1 v_k (the matvec's input) under diagonal scaling, else null
    const double* V;        // v_0 .. v_k, leading dimension n
    double* w;              // v_{k+1}: A v_k on entry to the Gram-Schmidt phases
    double* dpart;          // [(k + 1) * kDotBlocks] dot-product partials
    double *h1, *h2, *hn;   // the two passes' coefficients and the norm
    double *H, *cs, *sn, *g;
    double* res;            // the request's residual estimate |g[k+1]| / ||b||
    const double* dinv;     // the preconditioner's inverse diagonal (diag_scaling), else null
    double bnorm;
    int n, nu, k, ldh;
    int off[kKrylovPhases];
};

// counts: [kKrylovPhases] item totals, then the number of requests.  The diagonal scaling
// (before the matvec) and the Gram-Schmidt / Givens phases (after it).
hipError_t launch_batched_diag(const KrylovDesc* kd, const int* counts, hipStream_t s);
hipError_t launch_batched_krylov(const KrylovDesc* kd, const int* counts, hipStream_t s);

}  // namespace hobi
