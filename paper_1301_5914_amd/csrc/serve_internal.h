// Device-side descriptors of the request server's batched matvec.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "hobi.h"
#include "hobi_device.h"

namespace hobi {

constexpr int kServeBlock = 256;       // threads per block of the batched kernels
constexpr int kServeGridPair = 2048;  // fixed grids: the kernels walk the item lists
constexpr int kServeGridSmall = 1024;

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
    int workers, slots, groups, slot;   // the pair plan (the single-problem plan)
    int mixed;
    int tpl;                // targets per lane of the request's pair plan (the single-problem plan)
    int method;             // HOBI_HIGHER_ORDER or HOBI_LOWER_ORDER
    int pad;
};

// One unit of work: request `req`; a = workgroup of the pair plan's workers (waves
// 4a .. 4a + 3) for the pair kernels, node or vertex block for gather and combine.
struct ServeItem {
    int req, a, b, pad;
};

// Item lists and their counts, in launch order: gather, FP32 pair, FP64 pair, combine.
hipError_t launch_batched_matvec(const ServeDesc* desc, const ServeItem* const items[4], const int* counts,
                                 hipStream_t s);

}  // namespace hobi
