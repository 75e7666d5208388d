// Batched matrix-vector products of the request server: one launch per phase (gather,
// dense pair sum, combine) for every active request.  The launches walk device-side work
// lists with a grid-stride loop, so their grids are fixed and the three launches can be
// captured once in a HIP graph; the host only rewrites the descriptor and item arrays
// between ticks.  Each item runs the same tile and worker functions as the single-problem
// kernels (a pair item is one workgroup's worth of the problem's own pair plan),
// and a request's items depend only on that request, so its result does not depend on
// which other requests share the launch.
#include "hobi_internal.h"
#include "krylov_tile.h"
#include "pair_tile.h"
#include "serve_internal.h"

namespace hobi {

static_assert(kServeBlock == kPairBlock, "served work items are pair-kernel blocks");
static_assert(kPairBlock == kPairWaves * kWave, "a pair block is kPairWaves waves");

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
    __shared__ double red[kPairWaves * 2 * kWave * 8];
    const int n = as_constant(count)[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        const int b = uniform(item.a);
        if (d.tpl == 8) {
            if (d.kappa == 0.0)
                pair_f32_block<8, true>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                        d.partial, b, red);
            else
                pair_f32_block<8, false>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                         d.partial, b, red);
        } else {
            if (d.kappa == 0.0)
                pair_f32_block<4, true>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                        d.partial, b, red);
            else
                pair_f32_block<4, false>(d.tgt32, d.nv, d.nv_pad, d.node32, d.node_vid, d.blk_range, d.gstart, d.slots,
                                         d.partial, b, red);
        }
    }
}

__global__ __launch_bounds__(kPairBlock) void batched_pair64_kernel(const ServeDesc* __restrict__ desc,
                                                                  const ServeItem* __restrict__ items,
                                                                  const int* __restrict__ count) {
    __shared__ double etab[kExpTab];
    fill_exp_table(etab);
    const int n = as_constant(count)[0];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const const_as<ServeItem>& item = as_constant(items)[uniform(it)];
        const const_as<ServeDesc>& d = as_constant(desc)[uniform(item.req)];
        const int w = item.a * kPairWaves + wave;   // one row per worker (per_row 1)
        if (w >= d.rows * d.slots) continue;
        if (d.kappa == 0.0)
            pair_f64_worker<kTpl64, true>(d.tgt64, d.nv, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.kappa, etab,
                                          d.gstart, d.slots, d.partial, w);
        else
            pair_f64_worker<kTpl64, false>(d.tgt64, d.nv, d.nv_pad, d.node64, d.node_vid, d.blk_range, d.kappa, etab,
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
        combine_tile(item.a, d.u, d.y, d.nv, d.partial, d.slot, d.slots, d.rows, d.inc_off, d.inc_ent, d.tri,
                     d.coef, d.eps);
    }
}

// ---- batched Arnoldi steps ----

enum KrylovPhase { K_DIAG = 0, K_DOTS, K_REDUCE, K_AXPY, K_NORM_DOTS, K_SINGLE };

// The request holding item `it` of `phase` (block-uniform): the last one whose first item is
// at most it.
__device__ __forceinline__ int krylov_owner(const KrylovDesc* __restrict__ kd, int nreq, int phase, int it) {
    const const_as<KrylovDesc>* c = as_constant(kd);
    int lo = 0, hi = nreq;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (c[mid].off[phase] <= it) lo = mid;
        else hi = mid;
    }
    return uniform(lo);
}

__global__ __launch_bounds__(kKrylovBlock) void batched_diag_kernel(const KrylovDesc* __restrict__ kd,
                                                                    const int* __restrict__ counts) {
    const int n_items = as_constant(counts)[K_DIAG], nreq = as_constant(counts)[kKrylovPhases];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int q = krylov_owner(kd, nreq, K_DIAG, it);
        const KrylovDesc& d = kd[q];
        const int i = (it - d.off[K_DIAG]) * kKrylovBlock + (int)threadIdx.x;
        if (d.z && i < d.n) diag_scale_elem(d.vk, d.z, d.dinv, i);
    }
}

// Slice partials of the Gram-Schmidt dot products (norm = 0: V[j] . w for j <= k) or of w . w.
__global__ __launch_bounds__(kKrylovBlock) void batched_dots_kernel(const KrylovDesc* __restrict__ kd,
                                                                    const int* __restrict__ counts, int norm) {
    __shared__ double red[kKrylovBlock];
    const int phase = norm ? K_NORM_DOTS : K_DOTS;
    const int n_items = as_constant(counts)[phase], nreq = as_constant(counts)[kKrylovPhases];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int q = krylov_owner(kd, nreq, phase, it);
        const KrylovDesc& d = kd[q];
        const int local = it - d.off[phase];
        const int j = local / kDotSlices, b = local % kDotSlices;
        const double* v = norm ? d.w : d.V + (size_t)d.n * j;
        const double s = dot_slice(v, d.w, d.n, b, red);
        if (threadIdx.x == 0) d.dpart[(size_t)j * kDotSlices + b] = s;
    }
}

// norm = 0: h_pass[j] = sum of the slices of dot product j; norm = 1: hn = its square root.
__global__ __launch_bounds__(kDotSlices) void batched_reduce_kernel(const KrylovDesc* __restrict__ kd,
                                                                   const int* __restrict__ counts, int pass,
                                                                   int norm) {
    __shared__ double red[kDotSlices];
    const int phase = norm ? K_SINGLE : K_REDUCE;
    const int n_items = as_constant(counts)[phase], nreq = as_constant(counts)[kKrylovPhases];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int q = krylov_owner(kd, nreq, phase, it);
        const KrylovDesc& d = kd[q];
        const int j = it - d.off[phase];
        const double s = sum_slices(d.dpart + (size_t)j * kDotSlices, red, norm != 0);
        if (threadIdx.x == 0) (norm ? d.hn : pass == 0 ? d.h1 : d.h2)[j] = s;
    }
}

// scale = 0: w -= V h_pass (one Gram-Schmidt pass); scale = 1: w = w / hn.
__global__ __launch_bounds__(kKrylovBlock) void batched_axpy_kernel(const KrylovDesc* __restrict__ kd,
                                                                    const int* __restrict__ counts, int pass,
                                                                    int scale) {
    const int n_items = as_constant(counts)[K_AXPY], nreq = as_constant(counts)[kKrylovPhases];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int q = krylov_owner(kd, nreq, K_AXPY, it);
        const KrylovDesc& d = kd[q];
        const int i = (it - d.off[K_AXPY]) * kKrylovBlock + (int)threadIdx.x;
        if (i >= d.n) continue;
        if (scale)
            scale_copy_elem(d.w, d.hn[0], d.w, i);
        else
            multi_axpy_elem(d.V, d.n, d.k + 1, pass == 0 ? d.h1 : d.h2, -1.0, d.w, i);
    }
}

// One thread per request: column k of its Hessenberg matrix and rotation k.
__global__ void batched_givens_kernel(const KrylovDesc* __restrict__ kd, const int* __restrict__ counts) {
    const int nreq = as_constant(counts)[kKrylovPhases];
    for (int q = blockIdx.x * blockDim.x + (int)threadIdx.x; q < nreq; q += gridDim.x * blockDim.x) {
        const KrylovDesc& d = kd[q];
        givens_step(d.H, d.ldh, d.k, d.h1, d.h2, d.hn, d.cs, d.sn, d.g, d.bnorm, d.res);
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

hipError_t launch_batched_diag(const KrylovDesc* kd, const int* counts, hipStream_t s) {
    hipLaunchKernelGGL(batched_diag_kernel, dim3(kServeGridSmall), dim3(kKrylovBlock), 0, s, kd, counts);
    return hipGetLastError();
}

hipError_t launch_batched_krylov(const KrylovDesc* kd, const int* counts, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(batched_dots_kernel, dim3(kServeGridSmall), dim3(kKrylovBlock), 0, s, kd, counts, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(batched_reduce_kernel, dim3(kServeGridSmall), dim3(kDotSlices), 0, s, kd, counts, pass, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(batched_axpy_kernel, dim3(kServeGridSmall), dim3(kKrylovBlock), 0, s, kd, counts, pass, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batched_dots_kernel, dim3(kServeGridSmall), dim3(kKrylovBlock), 0, s, kd, counts, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_reduce_kernel, dim3(kServeGridSmall), dim3(kDotSlices), 0, s, kd, counts, 0, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_axpy_kernel, dim3(kServeGridSmall), dim3(kKrylovBlock), 0, s, kd, counts, 0, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(batched_givens_kernel, dim3(1), dim3(64), 0, s, kd, counts);
    return hipGetLastError();
}

}  // namespace hobi
