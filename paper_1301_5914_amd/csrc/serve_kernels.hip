// Batched matrix-vector products of the request server: one launch per phase (gather,
// dense pair sum, combine) for every active request.  The launches walk device-side work
// lists with a grid-stride loop, so their grids are fixed and the three launches can be
// captured once in a HIP graph; the host only rewrites the descriptor and item arrays
// between ticks.  Each item runs the same tile functions as the single-problem kernels,
// and a request's items depend only on that request, so its result does not depend on
// which other requests share the launch.
#include "hobi_internal.h"
#include "pair_tile.h"
#include "serve_internal.h"

namespace hobi {

static_assert(kServeBlock == kPairBlock, "served work items are pair-kernel blocks");

namespace {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ __launch_bounds__(kPairBlock) void batched_gather_kernel(const ServeDesc* __restrict__ desc,
                                                                  const ServeItem* __restrict__ items,
                                                                  const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        const int idx = item.a * kPairBlock + (int)threadIdx.x;
        if (idx < d.nn) gather_node(idx, d.u, d.nv, d.tri, d.w, d.node64, d.node32, d.mixed, d.eps, d.s32);
    }
}

__global__ __launch_bounds__(kPairBlock) void batched_pair_kernel(const ServeDesc* __restrict__ desc,
                                                                const ServeItem* __restrict__ items,
                                                                const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        if (d.mixed) {
            if (d.kappa == 0.0)
                pair_f32_tile<kServeTpl32, true>(d.tgt32, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.nn, d.chunk,
                                                 d.partial, item.a, item.b);
            else
                pair_f32_tile<kServeTpl32, false>(d.tgt32, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.nn, d.chunk,
                                                  d.partial, item.a, item.b);
        } else {
            if (d.kappa == 0.0)
                pair_f64_tile<kServeTpl64, true>(d.tgt64, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.nn, d.chunk, d.kappa, d.eps,
                                                 d.partial, item.a, item.b);
            else
                pair_f64_tile<kServeTpl64, false>(d.tgt64, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.nn, d.chunk, d.kappa, d.eps,
                                                  d.partial, item.a, item.b);
        }
    }
}

__global__ __launch_bounds__(kPairBlock) void batched_combine_kernel(const ServeDesc* __restrict__ desc,
                                                                   const ServeItem* __restrict__ items,
                                                                   const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        combine_tile(item.a, d.u, d.y, d.nv, d.nv_pad, d.partial, d.chunks, d.inc_off, d.inc_ent, d.tri, d.coef,
                     d.eps);
    }
}

}  // namespace

hipError_t launch_batched_matvec(const ServeDesc* desc, const ServeItem* gather_items, const int* n_gather,
                                 const ServeItem* pair_items, const int* n_pair, const ServeItem* comb_items,
                                 const int* n_comb, hipStream_t s) {
    hipLaunchKernelGGL(batched_gather_kernel, dim3(kServeGridSmall), dim3(kPairBlock), 0, s, desc, gather_items,
                       n_gather);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_pair_kernel, dim3(kServeGridPair), dim3(kPairBlock), 0, s, desc, pair_items,
                       n_pair);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_combine_kernel, dim3(kServeGridSmall), dim3(kPairBlock), 0, s, desc, comb_items,
                       n_comb);
    return hipGetLastError();
}

}  // namespace hobi
