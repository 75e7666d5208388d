// Batched matrix-vector products of the request server: one launch per phase (gather,
// dense pair sum, combine) for every active request.  The launches walk device-side work
// lists with a grid-stride loop, so their grids are fixed and the three launches can be
// captured once in a HIP graph; the host only rewrites the descriptor and item arrays
// between ticks.  Each item runs the same tile and worker functions as the single-problem
// kernels (a pair item is one workgroup's worth of the problem's own pair plan),
// and a request's items depend only on that request, so its result does not depend on
// which other requests share the launch.
#include "hobi_internal.h"
#include "pair_tile.h"
#include "serve_internal.h"

namespace hobi {

static_assert(kServeBlock == kPairBlock, "served work items are pair-kernel blocks");
static_assert(kTpl64 == 2, "served FP64 tiles use the single-problem plan");

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
        if (idx < d.nn) {
            if (d.method == HOBI_LOWER_ORDER)
                gather_site(idx, d.u, d.nv, d.w, d.node64, d.node32, d.mixed, d.eps, d.s32);
            else
                gather_node(idx, d.u, d.nv, d.tri, d.w, d.node64, d.node32, d.mixed, d.eps, d.s32);
        }
    }
}

// FP32 and FP64 items go to separate launches, so that each kernel's register budget is
// that of its own tile (the FP32 one then keeps the occupancy of the single-problem kernel).
// At most 128 registers: the four tile shapes share one kernel, which would otherwise take
// more registers than the largest of them and lose a wave per SIMD.
__global__ __launch_bounds__(kPairBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void batched_pair32_kernel(
    const ServeDesc* __restrict__ desc, const ServeItem* __restrict__ items, const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        const int w = item.a * (kPairBlock / kWave) + wave;
        if (w >= d.workers) continue;
        if (d.tpl == 8) {
            if (d.kappa == 0.0)
                pair_f32_worker<8, true>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                         d.partial, w);
            else
                pair_f32_worker<8, false>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                          d.partial, w);
        } else {
            if (d.kappa == 0.0)
                pair_f32_worker<4, true>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                         d.partial, w);
            else
                pair_f32_worker<4, false>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                          d.partial, w);
        }
    }
}

__global__ __launch_bounds__(kPairBlock) void batched_pair64_kernel(const ServeDesc* __restrict__ desc,
                                                                  const ServeItem* __restrict__ items,
                                                                  const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        const int w = item.a * (kPairBlock / kWave) + wave;
        if (w >= d.workers) continue;
        if (d.kappa == 0.0)
            pair_f64_worker<kTpl64, true>(d.tgt64, d.nv, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.kappa, d.eps,
                                          d.gstart, d.slots, d.partial, w);
        else
            pair_f64_worker<kTpl64, false>(d.tgt64, d.nv, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.kappa, d.eps,
                                           d.gstart, d.slots, d.partial, w);
    }
}

__global__ __launch_bounds__(kPairBlock) void batched_combine_kernel(const ServeDesc* __restrict__ desc,
                                                                   const ServeItem* __restrict__ items,
                                                                   const int* __restrict__ count) {
    const int n = as_constant(count)[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        combine_tile(item.a, d.u, d.y, d.nv, d.partial, d.slot, d.slots, d.groups, d.inc_off, d.inc_ent, d.tri,
                     d.coef, d.eps);
    }
}

}  // namespace

hipError_t launch_batched_matvec(const ServeDesc* desc, const ServeItem* const items[4], const int* counts,
                                 hipStream_t s) {
    hipLaunchKernelGGL(batched_gather_kernel, dim3(kServeGridSmall), dim3(kPairBlock), 0, s, desc, items[0], counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_pair32_kernel, dim3(kServeGridPair), dim3(kPairBlock), 0, s, desc, items[1],
                       counts + 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_pair64_kernel, dim3(kServeGridPair), dim3(kPairBlock), 0, s, desc, items[2],
                       counts + 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_combine_kernel, dim3(kServeGridSmall), dim3(kPairBlock), 0, s, desc, items[3],
                       counts + 3);
    return hipGetLastError();
}

}  // namespace hobi
