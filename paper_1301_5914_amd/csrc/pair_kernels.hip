// The matrix-vector product y = A u of the discretised well-posed formulation
// (Section 2.2 eqdbef3/eqdbef4 and Section 2.3 eqdbef5/eqdbef6), in three launches:
//
//   gather_kernel   -- u -> per-node strengths Gamma = w J L.dphi / (4 pi),
//                      Phi = w J L.phi / (4 pi) at the 4 Nf regular nodes
//   pair_f64/f32    -- the dense regular sum over every (vertex, node) pair except the
//                      nodes of the vertex's own triangles (those are singular):
//                      R1_i = sum K1 Gamma + K2 Phi, R2_i = sum K3 Gamma + K4 Phi,
//                      one wave per (target slot, node group), one FP64 partial row
//                      per wave
//   combine_kernel  -- sums a slot's partial rows in a fixed order, adds the singular
//                      correction (FP64 coefficients) and the diagonal 1/2 (1 + eps).
//
// Pair-kernel layout: each lane owns TPL target vertices in registers; the wavefront
// walks its range of source nodes in lock-step, so every node is one wave-uniform
// scalar load (64 or 128 bytes) broadcast to all 64 lanes -- no LDS traffic, no
// barriers, and each target's sum stays in its own lane (no cross-lane reduction).
// The launch fills whole passes of the waves the device keeps resident, all with the same
// work (the node groups differ by at most one node).
// exp and rsqrt are VALU transcendental instructions in the FP32 kernel.
#include "hobi_internal.h"
#include "pair_tile.h"

#include <algorithm>
#include <mutex>

namespace hobi {

// The allocation-free matvec's work space: one copy per device, alive until the process
// ends.  Host code refers to it only through the address hipGetSymbolAddress returns.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {

constexpr int kBlock = kPairBlock;

__global__ void gather_kernel(const double* __restrict__ u, int nv, const int* __restrict__ tri,
                              const double* __restrict__ w, int nn, NodeD* __restrict__ node64,
                              NodeF* __restrict__ node32, int mixed, double eps, double s32, int method) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    if (method == HOBI_LOWER_ORDER)
        gather_site(idx, u, nv, w, node64, node32, mixed, eps, s32);
    else
        gather_node(idx, u, nv, tri, w, node64, node32, mixed, eps, s32);
}

constexpr int kWavesPerBlock = kBlock / kWave;
static_assert(kWavesPerBlock == kPairWaves, "a pair-kernel workgroup holds one block of the plan");

// Workgroups are dispatched round-robin over the 8 XCDs by linear id.  Give each XCD a
// contiguous range of logical workgroups, so that the workers of a node group (consecutive
// logical ids) share that XCD's L2 while they read the group's nodes.
__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, p = blockIdx.x;
    const int x = p & 7, q = nb >> 3, rm = nb & 7;
    return x * q + min(x, rm) + (p >> 3);
}

// FP64: one wave per worker of the pair plan (per_row 1): logical workgroup b holds workers
// kWavesPerBlock * b + (its waves); waves past the last worker return at once.
template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void pair_f64_kernel(
    const double* __restrict__ tgt, int nv, int nv_pad, const NodeD* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, double kappa,
    const int* __restrict__ gstart, int slots, int workers, double* __restrict__ partial) {
    __shared__ double etab[kExpTab];
    if constexpr (!KAPPA0) fill_exp_table(etab);
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= workers) return;
    pair_f64_worker<TPL, KAPPA0>(tgt, nv, nv_pad, nodes, node_vid, blk_range, kappa, etab, gstart, slots, partial, w);
}

// FP32: one workgroup per block of the pair plan (per_row 4; logical workgroup b is block b);
// every block of the grid is a block of the plan.
template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void pair_f32_kernel(
    const float* __restrict__ tgt, int nv, int nv_pad, const NodeF* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, const int* __restrict__ gstart,
    int slots, double* __restrict__ partial) {
    __shared__ double red[kPairWaves * 2 * kWave * TPL];
    pair_f32_block<TPL, KAPPA0>(tgt, nv, nv_pad, nodes, node_vid, blk_range, gstart, slots, partial,
                                xcd_logical_block(), red);
}

__global__ void combine_kernel(const double* __restrict__ u, double* __restrict__ y, int nv,
                               const double* __restrict__ partial, int slot, int slots, int rows,
                               const int* __restrict__ inc_off, const int* __restrict__ inc_ent,
                               const int* __restrict__ tri, const double* __restrict__ coef,
                               double eps) {
    combine_tile(blockIdx.x, u, y, nv, partial, slot, slots, rows, inc_off, inc_ent, tri, coef, eps);
}

// Sums over every regular node at interior points (the charges):
//   MODE 0: reaction potential  sum K1 Gamma + K2 Phi  (eq. solvation_energy)
//   MODE 1: double-layer of a unit density  sum w (d.ny) / r^3  (solid angle * 4 pi)
template <int MODE>
__global__ __launch_bounds__(kBlock) void point_sum_kernel(
    const double* __restrict__ pts, int np_pad, const NodeD* __restrict__ nodes,
    const double* __restrict__ w, int nn, int chunk, double kappa, double eps,
    double* __restrict__ partial) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const double px = pts[p], py = pts[(size_t)np_pad + p], pz = pts[2 * (size_t)np_pad + p];
    const double em1 = eps - 1.0;
    const int s0 = blockIdx.y * chunk;
    const int s1 = min(s0 + chunk, nn);
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) {
        const NodeD nd = nodes[s];
        const double dx = px - nd.x, dy = py - nd.y, dz = pz - nd.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double rinv = rsqrt(r2);
        const double rinv3 = rinv * rinv * rinv;
        const double dny = dx * nd.nx + dy * nd.ny + dz * nd.nz;
        if (MODE == 1) {
            acc += w[s] * dny * rinv3;
        } else {
            double f0, f1, f2;
            f012_f64(kappa * (r2 * rinv), &f0, &f1, &f2);
            acc += f0 * rinv * nd.g + dny * rinv3 * (em1 - eps * f1) * nd.p;
        }
    }
    partial[(size_t)blockIdx.y * np_pad + p] = acc;
}

// One block per point p: the sum over chunks (thread t takes chunks t, t + 256, ... in
// order, then a fixed LDS tree).  MODE 0: out[p] = phi_reac[p]; MODE 1: out[p] = -sum / (4 pi).
template <int MODE>
__global__ __launch_bounds__(256) void point_reduce_kernel(const double* __restrict__ partial, int np_pad,
                                                           int chunks, double* __restrict__ out) {
    __shared__ double red[256];
    const int p = blockIdx.x;
    double v = 0.0;
    for (int c = threadIdx.x; c < chunks; c += 256) v += partial[(size_t)c * np_pad + p];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = MODE == 0 ? red[0] : -red[0] * kInv4Pi;
}

// E = 1/2 * 4 pi C * sum_p q_p phi_reac[p]; one block, fixed order.
__global__ __launch_bounds__(256) void energy_kernel(const double* __restrict__ phi_reac, const double* __restrict__ q,
                                                     int np, double* __restrict__ e_out) {
    __shared__ double red[256];
    double local = 0.0;
    for (int p = threadIdx.x; p < np; p += 256) local += q[p] * phi_reac[p];
    red[threadIdx.x] = local;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) e_out[0] = 0.5 * 4.0 * kPi * 332.0716 * red[0];
}

__global__ void permute_kernel(const double* __restrict__ in, double* __restrict__ out,
                               const int* __restrict__ perm, int nv, int to_internal) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int o = perm[i];
    if (to_internal) {
        out[i] = in[o];
        out[nv + i] = in[nv + o];
    } else {
        out[o] = in[i];
        out[nv + o] = in[nv + i];
    }
}

// Group starts of a pair plan: tab[g] = g * nn / groups (as make_pair_plan computes them).
__global__ void group_starts_kernel(int* __restrict__ tab, int groups, int nn) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= groups) tab[g] = (int)((int64_t)g * nn / groups);
}

// The FP64 pair kernel's arithmetic on given arguments: fn 0 = exp(-x) (table-driven,
// x >= 0), fn 1 = 1 / sqrt(x) (x > 0).
__global__ __launch_bounds__(kBlock) void device_math_kernel(int fn, const double* __restrict__ x,
                                                             double* __restrict__ y, int n) {
    __shared__ double etab[kExpTab];
    fill_exp_table(etab);
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i >= n) return;
    y[i] = fn == 0 ? exp_neg_tab_f64(x[i], etab) : rsqrt_f64(x[i]);
}

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

GridPlan make_grid_plan(int n_pad, int nn, int tpl) {
    GridPlan pl{};
    pl.tpl = tpl;
    pl.block = kBlock;
    pl.target_blocks = n_pad / (kBlock * tpl);
    if (pl.target_blocks < 1) pl.target_blocks = 1;
    // about 16 blocks per compute unit on 256 CUs; at least 256 nodes per chunk
    const int want = 4096;
    int chunks = (want + pl.target_blocks - 1) / pl.target_blocks;
    const int max_chunks = nn / 256 > 1 ? nn / 256 : 1;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    pl.chunk = (nn + chunks - 1) / chunks;
    pl.chunks = (nn + pl.chunk - 1) / pl.chunk;
    return pl;
}

bool make_pair_plan(int nv, int nn, int tpl, int resident_waves, int per_row, PairPlan* plan,
                    std::vector<int>* gstart) {
    if (nv < 1 || nn < 1 || resident_waves < 1 || (per_row != 1 && per_row != kPairWaves)) return false;
    PairPlan pl{};
    pl.tpl = tpl;
    pl.slot = kWave * tpl;
    pl.slots = (nv + pl.slot - 1) / pl.slot;
    // about kPairPasses passes of the resident waves, with at least kMinGroupNodes nodes per
    // group (a worker's partial row then costs the combine step little next to its pairs)
    const int max_groups = std::max(1, nn / kMinGroupNodes);
    const int64_t want = (int64_t)kPairPasses * resident_waves / pl.slots;
    const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(want, max_groups));
    pl.per_row = per_row;
    pl.rows = (int)((groups + per_row - 1) / per_row);
    pl.groups = pl.rows * per_row;
    if ((int64_t)pl.groups * pl.slots >= ((int64_t)1 << 31) / kPairWaves) return false;
    pl.workers = pl.groups * pl.slots;
    pl.blocks = (pl.workers + kWavesPerBlock - 1) / kWavesPerBlock;
    for (int g = 0; g <= pl.groups; ++g) gstart->push_back((int)((int64_t)g * nn / pl.groups));
    pl.gstart = nullptr;
    *plan = pl;
    return true;
}

int pair_resident_waves(int device, bool mixed, int tpl) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    hipError_t e;
    if (mixed)
        e = tpl == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pair_f32_kernel<8, false>, kBlock, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pair_f32_kernel<4, false>, kBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pair_f64_kernel<kTpl64, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1) return 0;
    return cus * per_cu * kWavesPerBlock;
}

hipError_t launch_gather(const DeviceProblem& p, const double* u, bool mixed, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3(nblk(p.nn, 256)), dim3(256), 0, s, u, p.nv, p.tri, p.w, p.nn,
                       p.node64, p.node32, mixed ? 1 : 0, p.eps, p.s32, p.method);
    return hipGetLastError();
}

hipError_t launch_pair_plan(const DeviceProblem& p, const PairPlan& pl, double* partial, bool mixed,
                            hipStream_t s) {
    const bool k0 = p.kappa == 0.0;
    if (mixed) {
#define HOBI_PAIR32(T, K0)                                                                                    \
    hipLaunchKernelGGL((pair_f32_kernel<T, K0>), dim3(pl.blocks), dim3(kBlock), 0, s, p.tgt32, p.nv, p.nv_pad, \
                       p.node32, p.node_vid, p.blk_range, pl.gstart, pl.slots, partial)
        if (pl.tpl == 8) {
            if (k0) HOBI_PAIR32(8, true); else HOBI_PAIR32(8, false);
        } else {
            if (k0) HOBI_PAIR32(4, true); else HOBI_PAIR32(4, false);
        }
#undef HOBI_PAIR32
    } else {
#define HOBI_PAIR64(K0)                                                                                          \
    hipLaunchKernelGGL((pair_f64_kernel<kTpl64, K0>), dim3(pl.blocks), dim3(kBlock), 0, s, p.tgt64, p.nv, p.nv_pad, \
                       p.node64, p.node_vid, p.blk_range, p.kappa, pl.gstart, pl.slots, pl.workers, partial)
        if (k0) HOBI_PAIR64(true); else HOBI_PAIR64(false);
#undef HOBI_PAIR64
    }
    return hipGetLastError();
}

hipError_t launch_pair(const DeviceProblem& p, bool mixed, hipStream_t s) {
    return launch_pair_plan(p, mixed ? p.plan32 : p.plan64, p.partial, mixed, s);
}

hipError_t launch_combine_plan(const DeviceProblem& p, const PairPlan& pl, const double* partial,
                               const double* u, double* y, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(nblk(p.nv, kCombineVerts)), dim3(kPairBlock), 0, s, u, y, p.nv,
                       partial, pl.slot, pl.slots, pl.rows, p.inc_off, p.inc_ent, p.tri, p.coef, p.eps);
    return hipGetLastError();
}

hipError_t launch_combine(const DeviceProblem& p, const double* u, double* y, bool mixed, hipStream_t s) {
    return launch_combine_plan(p, mixed ? p.plan32 : p.plan64, p.partial, u, y, s);
}

// ---- static work space of the allocation-free matvec ----

bool make_static_pair_plan(const PairPlan& base, int nn, PairPlan* out, size_t* row_bytes) {
    PairPlan pl = base;
    // one partial row per slot for every per_row node groups
    const size_t row_set = (size_t)base.slots * 2 * base.slot * sizeof(double);
    *row_bytes = row_set;
    const size_t fit = (kStaticScratchBytes - kStaticTableBytes) / row_set;
    const size_t table_max = (kStaticTableBytes / sizeof(int) - 1) / base.per_row;
    if (fit < 1 || nn < 1) return false;
    pl.rows = (int)std::min<size_t>({(size_t)base.rows, fit, table_max});
    pl.groups = pl.rows * base.per_row;
    pl.workers = pl.groups * pl.slots;
    pl.blocks = (pl.workers + kWavesPerBlock - 1) / kWavesPerBlock;
    pl.gstart = nullptr;
    *out = pl;
    return true;
}

hipError_t launch_group_starts(int* tab, int groups, int nn, hipStream_t s) {
    hipLaunchKernelGGL(group_starts_kernel, dim3(nblk(groups + 1, 256)), dim3(256), 0, s, tab, groups, nn);
    return hipGetLastError();
}

hipError_t static_scratch_address(int device, void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_reaction_energy(const DeviceProblem& p, double* phi_reac, double* e_out, hipStream_t s) {
    const GridPlan& pl = p.plan_pts;
    hipLaunchKernelGGL((point_sum_kernel<0>), dim3(pl.target_blocks, pl.chunks), dim3(kBlock), 0, s, p.qsoa,
                       p.nc_pad, p.node64, p.w, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((point_reduce_kernel<0>), dim3(p.nc), dim3(256), 0, s, p.partial, p.nc_pad, pl.chunks,
                       phi_reac);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(256), 0, s, phi_reac, p.q, p.nc, e_out);
    return hipGetLastError();
}

hipError_t launch_solid_angle(const DeviceProblem& p, double* frac, hipStream_t s) {
    const GridPlan& pl = p.plan_pts;
    hipLaunchKernelGGL((point_sum_kernel<1>), dim3(pl.target_blocks, pl.chunks), dim3(kBlock), 0, s, p.qsoa,
                       p.nc_pad, p.node64, p.w, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((point_reduce_kernel<1>), dim3(p.nc), dim3(256), 0, s, p.partial, p.nc_pad, pl.chunks,
                       frac);
    return hipGetLastError();
}

hipError_t launch_device_math(int fn, const double* x, double* y, int n, hipStream_t s) {
    hipLaunchKernelGGL(device_math_kernel, dim3(nblk(n, kBlock)), dim3(kBlock), 0, s, fn, x, y, n);
    return hipGetLastError();
}

hipError_t launch_permute(const double* in, double* out, const int* perm, int nv, bool to_internal,
                          hipStream_t s) {
    hipLaunchKernelGGL(permute_kernel, dim3(nblk(nv, 256)), dim3(256), 0, s, in, out, perm, nv,
                       to_internal ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hobi
