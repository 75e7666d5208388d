// Potential and field at points off the surface (Section 2.1: the representation formulas
// eqbim_1 and eqbim_2 combined with the jump conditions into the kernels of eq.
// solvation_energy).  With the surface strengths Gamma = w dphi/(4 pi), Phi = w phi/(4 pi)
// at the quadrature nodes (written by the gather, as for the matrix-vector product):
//
//   R(x)      = sum_y K1 Gamma + K2 Phi                                  (reaction potential)
//   grad R(x) = sum_y [(pa + pb f1) n_y - (f1 Gamma + (3 pa + pb f2) q) d] / r^3
//   Omega(x)  = -sum_y w (d.n_y) / (4 pi r^3)                        (solid-angle fraction)
//
// with d = x - y, q = (d.n_y)/r^2, pa = (eps - 1) Phi, pb = -eps Phi (the gradient of
// K1 = G0 - Gk and of K2 = eps dGk/dnu_y - dG0/dnu_y with the f-functions of the matvec).
// Then x is inside when Omega > 1/2, and
//   inside:   phi = S1 + R,          outside: phi = (S1 + R) / eps,     E = -grad phi,
// S1 = sum_k q_k G0(x, x_k) / eps1 (a charge within kCoincident of x left out).
//
// Layout as the pair sum: one wave per (slot of points, node group) of a pair plan, each
// writing a row of five partial sums per point (R, grad R, Omega); field_combine_kernel
// adds a point's rows in a fixed order, then the Coulomb part in FP64.
#include <hipcub/hipcub.hpp>

#include "hobi_internal.h"
#include "pair_tile.h"

namespace hobi {

namespace {

constexpr int kBlock = kPairBlock;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kParts = 5;                 // R, dR/dx, dR/dy, dR/dz, Omega
constexpr double kCoincident = 1e-6;      // A

__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, p = blockIdx.x;
    const int x = p & 7, q = nb >> 3, rm = nb & 7;
    return x * q + min(x, rm) + (p >> 3);
}

// FP32 sums over nodes [sb, se) for the lane's TPL points (positions in the scaled frame of
// the FP32 records; the gradient comes out in scaled units, times 1/s32).
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void field_f32_run(const const_as<NodeF>* cnodes, int sb, int se,
                                              const float (&tx)[TPL], const float (&ty)[TPL],
                                              const float (&tz)[TPL], float (&a)[kParts][TPL]) {
    NodeF n = load_node(cnodes, sb);
    for (int s = sb; s < se; ++s) {
        const NodeF next = load_node(cnodes, min(s + 1, se - 1));
        const float pa3 = 3.0f * n.pa;
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const float dx = tx[k] - n.x, dy = ty[k] - n.y, dz = tz[k] - n.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float rinv2 = rinv * rinv;
            const float rinv3 = rinv2 * rinv;
            const float dny = fmaf(dx, n.nx, fmaf(dy, n.ny, dz * n.nz));
            const float q = dny * rinv2;
            float c1, c2;
            if (KAPPA0) {
                a[0][k] = fmaf(dny * rinv3, n.pa, a[0][k]);
                c2 = n.pa;
                c1 = pa3 * q;
            } else {
                const float zp1 = fmaf(r2, rinv, 1.0f);                  // 1 + z
                const float e = __builtin_amdgcn_exp2f(fmaf(zp1, -kLog2E, kLog2E));   // exp(-z)
                const float f1 = fmaf(-e, zp1, 1.0f);
                const float f2 = fmaf(-e, fmaf(zp1, 3.0f, r2), 3.0f);
                c2 = fmaf(n.pb, f1, n.pa);                               // pa + pb f1
                a[0][k] = fmaf(rinv, fmaf(q, c2, fmaf(-e, n.g, n.g)), a[0][k]);
                c1 = fmaf(f1, n.g, fmaf(n.pb, f2, pa3) * q);             // f1 Gamma + (3 pa + pb f2) q
            }
            const float gn = rinv3 * c2, gd = -rinv3 * c1;
            a[1][k] = fmaf(gn, n.nx, fmaf(gd, dx, a[1][k]));
            a[2][k] = fmaf(gn, n.ny, fmaf(gd, dy, a[2][k]));
            a[3][k] = fmaf(gn, n.nz, fmaf(gd, dz, a[3][k]));
            a[4][k] = fmaf(n.pad, dny * rinv3, a[4][k]);
        }
        n = next;
    }
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void field_f32_wave(const float* __restrict__ pts, int np_pad,
                                               const NodeF* __restrict__ nodes, int base, int n0, int n1,
                                               double* __restrict__ prow, int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    float tx[TPL], ty[TPL], tz[TPL];
    double acc[kParts][TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = pts[t];
        ty[k] = pts[(size_t)np_pad + t];
        tz[k] = pts[2 * (size_t)np_pad + t];
#pragma unroll
        for (int c = 0; c < kParts; ++c) acc[c][k] = 0.0;
    }
    const const_as<NodeF>* cnodes = as_constant(nodes);
    for (int sb = n0, se; sb < n1; sb = se) {
        se = min((sb / kFold + 1) * kFold, n1);
        float a[kParts][TPL];
#pragma unroll
        for (int c = 0; c < kParts; ++c)
#pragma unroll
            for (int k = 0; k < TPL; ++k) a[c][k] = 0.0f;
        field_f32_run<TPL, KAPPA0>(cnodes, sb, se, tx, ty, tz, a);
#pragma unroll
        for (int c = 0; c < kParts; ++c)
#pragma unroll
            for (int k = 0; k < TPL; ++k) acc[c][k] += (double)a[c][k];
    }
#pragma unroll
    for (int c = 0; c < kParts; ++c)
#pragma unroll
        for (int k = 0; k < TPL; ++k) prow[(size_t)c * slot + lane + k * kWave] = acc[c][k];
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void field_f32_narrow(int live, const float* __restrict__ pts, int np_pad,
                                                 const NodeF* __restrict__ nodes, int base, int n0, int n1,
                                                 double* __restrict__ prow, int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            field_f32_narrow<TPL / 2, KAPPA0>(live, pts, np_pad, nodes, base, n0, n1, prow, slot);
            return;
        }
    }
    field_f32_wave<TPL, KAPPA0>(pts, np_pad, nodes, base, n0, n1, prow, slot);
}

template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void field_f32_kernel(const float* __restrict__ pts, int np, int np_pad,
                                                           const NodeF* __restrict__ nodes,
                                                           const int* __restrict__ gstart, int slots, int workers,
                                                           double* __restrict__ partial) {
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= workers) return;
    constexpr int kSlot = kWave * TPL;
    const int g = w / slots, s = w - g * slots;
    const const_as<int>* cg = as_constant(gstart);
    const int base = s * kSlot;
    field_f32_narrow<TPL, KAPPA0>(np - base, pts, np_pad, nodes, base, cg[g], cg[g + 1],
                                  partial + (size_t)w * (kParts * kSlot), kSlot);
}

// FP64 sums (unscaled frame) with the FP64 pair kernel's exponential (etab: the workgroup's
// table, fill_exp_table; not read when KAPPA0) and closed-form f-functions.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void field_f64_wave(const double* __restrict__ pts, int np_pad,
                                               const NodeD* __restrict__ nodes, double kappa,
                                               const double* __restrict__ etab, int base, int n0, int n1,
                                               double* __restrict__ prow, int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    double tx[TPL], ty[TPL], tz[TPL], a[kParts][TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = pts[t];
        ty[k] = pts[(size_t)np_pad + t];
        tz[k] = pts[2 * (size_t)np_pad + t];
#pragma unroll
        for (int c = 0; c < kParts; ++c) a[c][k] = 0.0;
    }
    const const_as<NodeD>* cnodes = as_constant(nodes);
    for (int s = n0; s < n1; ++s) {
        const NodeD nd = load_node(cnodes, s);
        const double pa3 = 3.0 * nd.pa;
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const double dx = tx[k] - nd.x, dy = ty[k] - nd.y, dz = tz[k] - nd.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double rinv2 = rinv * rinv;
            const double rinv3 = rinv2 * rinv;
            const double dny = fma(dx, nd.nx, fma(dy, nd.ny, dz * nd.nz));
            const double q = dny * rinv2;
            double c1, c2;
            if (KAPPA0) {
                a[0][k] = fma(dny * rinv3, nd.pa, a[0][k]);
                c2 = nd.pa;
                c1 = pa3 * q;
            } else {
                const double z = kappa * (r2 * rinv);
                const double e = exp_neg_tab_f64(z, etab);
                const double zp1 = z + 1.0;
                const double f1 = fma(-e, zp1, 1.0);                          // 1 - e (1 + z)
                const double f2 = fma(-e, fma(zp1, zp1 + 1.0, 1.0), 3.0);     // 3 - e (3 + 3z + z^2)
                c2 = fma(nd.pb, f1, nd.pa);
                a[0][k] = fma(rinv, fma(q, c2, fma(-e, nd.g, nd.g)), a[0][k]);   // Gamma (1 - e) = Gamma f0
                c1 = fma(f1, nd.g, fma(nd.pb, f2, pa3) * q);
            }
            const double gn = rinv3 * c2, gd = -rinv3 * c1;
            a[1][k] = fma(gn, nd.nx, fma(gd, dx, a[1][k]));
            a[2][k] = fma(gn, nd.ny, fma(gd, dy, a[2][k]));
            a[3][k] = fma(gn, nd.nz, fma(gd, dz, a[3][k]));
            a[4][k] = fma(nd.pad, dny * rinv3, a[4][k]);
        }
    }
#pragma unroll
    for (int c = 0; c < kParts; ++c)
#pragma unroll
        for (int k = 0; k < TPL; ++k) prow[(size_t)c * slot + lane + k * kWave] = a[c][k];
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void field_f64_narrow(int live, const double* __restrict__ pts, int np_pad,
                                                 const NodeD* __restrict__ nodes, double kappa,
                                                 const double* __restrict__ etab, int base, int n0, int n1,
                                                 double* __restrict__ prow, int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            field_f64_narrow<TPL / 2, KAPPA0>(live, pts, np_pad, nodes, kappa, etab, base, n0, n1, prow, slot);
            return;
        }
    }
    field_f64_wave<TPL, KAPPA0>(pts, np_pad, nodes, kappa, etab, base, n0, n1, prow, slot);
}

template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void field_f64_kernel(const double* __restrict__ pts, int np, int np_pad,
                                                           const NodeD* __restrict__ nodes, double kappa,
                                                           const int* __restrict__ gstart, int slots, int workers,
                                                           double* __restrict__ partial) {
    __shared__ double etab[kExpTab];
    if constexpr (!KAPPA0) fill_exp_table(etab);
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= workers) return;
    constexpr int kSlot = kWave * TPL;
    const int g = w / slots, s = w - g * slots;
    const const_as<int>* cg = as_constant(gstart);
    const int base = s * kSlot;
    field_f64_narrow<TPL, KAPPA0>(np - base, pts, np_pad, nodes, kappa, etab, base, cg[g], cg[g + 1],
                                  partial + (size_t)w * (kParts * kSlot), kSlot);
}

// Treecode far items (hobi_params.tree_theta > 0): the kWave * TPL points from `base`
// against one cluster's proxies s_k with the charges Q0, Qk, Qs (d = x - s_k, a = e^-kappa r):
//   R += sum Q0/r + a Qk/r,   grad R -= sum (Q0 + a (1 + kappa r) Qk) d / r^3,   Omega += sum Qs/r,
// rows as the direct waves'.  FP32: positions in the scaled frame, q0a = s32 Q0, qka = s32 Qk,
// qs = s32 Qs, so that the gradient comes out times 1/s32 like the direct rows.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_field_f32_wave(const float* __restrict__ pts, int np_pad,
                                                   const ProxyF* __restrict__ prox, int P, int base,
                                                   double* __restrict__ prow, int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    float tx[TPL], ty[TPL], tz[TPL];
    double acc[kParts][TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = pts[t];
        ty[k] = pts[(size_t)np_pad + t];
        tz[k] = pts[2 * (size_t)np_pad + t];
#pragma unroll
        for (int c = 0; c < kParts; ++c) acc[c][k] = 0.0;
    }
    const const_as<ProxyF>* cp = as_constant(prox);
    for (int k0 = 0; k0 < P; k0 += kFold) {
        const int k1 = min(k0 + kFold, P);
        float a[kParts][TPL];
#pragma unroll
        for (int c = 0; c < kParts; ++c)
#pragma unroll
            for (int k = 0; k < TPL; ++k) a[c][k] = 0.0f;
        ProxyF pr = load_proxy(cp, k0);
        for (int q = k0; q < k1; ++q) {
            const ProxyF next = load_proxy(cp, min(q + 1, k1 - 1));
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const float dx = tx[k] - pr.x, dy = ty[k] - pr.y, dz = tz[k] - pr.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float rinv3 = rinv * rinv * rinv;
                float c;
                if (KAPPA0) {
                    c = pr.q0a + pr.qka;
                    a[0][k] = fmaf(rinv, c, a[0][k]);
                } else {
                    const float zp1 = fmaf(r2, rinv, 1.0f);              // 1 + kappa r
                    const float e = __builtin_amdgcn_exp2f(fmaf(zp1, -kLog2E, kLog2E));   // exp(-kappa r)
                    a[0][k] = fmaf(rinv, fmaf(e, pr.qka, pr.q0a), a[0][k]);
                    c = fmaf(e * zp1, pr.qka, pr.q0a);
                }
                const float g = -rinv3 * c;
                a[1][k] = fmaf(g, dx, a[1][k]);
                a[2][k] = fmaf(g, dy, a[2][k]);
                a[3][k] = fmaf(g, dz, a[3][k]);
                a[4][k] = fmaf(rinv, pr.qs, a[4][k]);
            }
            pr = next;
        }
#pragma unroll
        for (int c = 0; c < kParts; ++c)
#pragma unroll
            for (int k = 0; k < TPL; ++k) acc[c][k] += (double)a[c][k];
    }
#pragma unroll
    for (int c = 0; c < kParts; ++c)
#pragma unroll
        for (int k = 0; k < TPL; ++k) prow[(size_t)c * slot + lane + k * kWave] = acc[c][k];
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_field_f32_narrow(int live, const float* __restrict__ pts, int np_pad,
                                                     const ProxyF* __restrict__ prox, int P, int base,
                                                     double* __restrict__ prow, int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            far_field_f32_narrow<TPL / 2, KAPPA0>(live, pts, np_pad, prox, P, base, prow, slot);
            return;
        }
    }
    far_field_f32_wave<TPL, KAPPA0>(pts, np_pad, prox, P, base, prow, slot);
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_field_f64_wave(const double* __restrict__ pts, int np_pad,
                                                   const ProxyD* __restrict__ prox, int P, double kappa,
                                                   const double* __restrict__ etab, int base,
                                                   double* __restrict__ prow, int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    double tx[TPL], ty[TPL], tz[TPL], a[kParts][TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = pts[t];
        ty[k] = pts[(size_t)np_pad + t];
        tz[k] = pts[2 * (size_t)np_pad + t];
#pragma unroll
        for (int c = 0; c < kParts; ++c) a[c][k] = 0.0;
    }
    const const_as<ProxyD>* cp = as_constant(prox);
    for (int q = 0; q < P; ++q) {
        const ProxyD pr = load_proxy(cp, q);
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const double dx = tx[k] - pr.x, dy = ty[k] - pr.y, dz = tz[k] - pr.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double rinv3 = rinv * rinv * rinv;
            double c;
            if (KAPPA0) {
                c = pr.q0 + pr.qk;
                a[0][k] = fma(rinv, c, a[0][k]);
            } else {
                const double z = kappa * (r2 * rinv);
                const double e = exp_neg_tab_f64(z, etab);
                a[0][k] = fma(rinv, fma(e, pr.qk, pr.q0), a[0][k]);
                c = fma(e * (1.0 + z), pr.qk, pr.q0);
            }
            const double g = -rinv3 * c;
            a[1][k] = fma(g, dx, a[1][k]);
            a[2][k] = fma(g, dy, a[2][k]);
            a[3][k] = fma(g, dz, a[3][k]);
            a[4][k] = fma(rinv, pr.qs, a[4][k]);
        }
    }
#pragma unroll
    for (int c = 0; c < kParts; ++c)
#pragma unroll
        for (int k = 0; k < TPL; ++k) prow[(size_t)c * slot + lane + k * kWave] = a[c][k];
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_field_f64_narrow(int live, const double* __restrict__ pts, int np_pad,
                                                     const ProxyD* __restrict__ prox, int P, double kappa,
                                                     const double* __restrict__ etab, int base,
                                                     double* __restrict__ prow, int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            far_field_f64_narrow<TPL / 2, KAPPA0>(live, pts, np_pad, prox, P, kappa, etab, base, prow, slot);
            return;
        }
    }
    far_field_f64_wave<TPL, KAPPA0>(pts, np_pad, prox, P, kappa, etab, base, prow, slot);
}

// One wave per treecode work item {slot, far, cluster, -} of the points; the item's partial
// rows are its index: near items sum the leaf's nodes directly, far items its proxies.
template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void field_tree_f32_kernel(const int4* __restrict__ items, int nitems,
                                                                const float* __restrict__ pts, int np, int np_pad,
                                                                const NodeF* __restrict__ nodes,
                                                                const int2* __restrict__ clu_range,
                                                                const ProxyF* __restrict__ prox, int P,
                                                                double* __restrict__ partial) {
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= nitems) return;
    constexpr int kSlot = kWave * TPL;
    const int4 it = make_int4(as_constant(items)[w].x, as_constant(items)[w].y, as_constant(items)[w].z, 0);
    const int base = it.x * kSlot;
    double* prow = partial + (size_t)w * (kParts * kSlot);
    if (it.y == 0)
        field_f32_narrow<TPL, KAPPA0>(np - base, pts, np_pad, nodes, base, as_constant(clu_range)[it.z].x,
                                      as_constant(clu_range)[it.z].y, prow, kSlot);
    else
        far_field_f32_narrow<TPL, KAPPA0>(np - base, pts, np_pad, prox + (size_t)it.z * P, P, base, prow, kSlot);
}

template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void field_tree_f64_kernel(const int4* __restrict__ items, int nitems,
                                                                const double* __restrict__ pts, int np, int np_pad,
                                                                const NodeD* __restrict__ nodes, double kappa,
                                                                const int2* __restrict__ clu_range,
                                                                const ProxyD* __restrict__ prox, int P,
                                                                double* __restrict__ partial) {
    __shared__ double etab[kExpTab];
    if constexpr (!KAPPA0) fill_exp_table(etab);
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= nitems) return;
    constexpr int kSlot = kWave * TPL;
    const int4 it = make_int4(as_constant(items)[w].x, as_constant(items)[w].y, as_constant(items)[w].z, 0);
    const int base = it.x * kSlot;
    double* prow = partial + (size_t)w * (kParts * kSlot);
    if (it.y == 0)
        field_f64_narrow<TPL, KAPPA0>(np - base, pts, np_pad, nodes, kappa, etab, base,
                                      as_constant(clu_range)[it.z].x, as_constant(clu_range)[it.z].y, prow, kSlot);
    else
        far_field_f64_narrow<TPL, KAPPA0>(np - base, pts, np_pad, prox + (size_t)it.z * P, P, kappa, etab, base,
                                          prow, kSlot);
}

// 64 points per block of 256 threads: wave k sums the point's rows of node groups k, k + 4,
// ... into two running sums by turn (fixed order), or, with slot_row, the rows of the
// point's slot's treecode items k, k + 4, ... in item order; the four waves' sums are added
// in a fixed order through LDS; then the frame scale of the gradient, the Coulomb part of the
// charges, the side and the outputs in kcal/(mol e) [A^-1]: out[p] = {phi, Ex, Ey, Ez, R,
// -dR/dx, -dR/dy, -dR/dz, Omega}, inside[p].
constexpr int kCombPts = 64, kCombWays = 4;

__global__ __launch_bounds__(kCombPts * kCombWays) void field_combine_kernel(
    const double* __restrict__ partial, const int* __restrict__ slot_row, int row_base, int p0, int np, int slot,
    int slots, int groups, double gscale,
    const double* __restrict__ pts, int np_pad, const double* __restrict__ qpos, const double* __restrict__ q,
    int nc, double eps1, double eps, double* __restrict__ out, int* __restrict__ inside) {
    __shared__ double red[kCombWays][kParts][kCombPts];
    const int lane = threadIdx.x % kCombPts, way = threadIdx.x / kCombPts;
    const int p = p0 + blockIdx.x * kCombPts + lane;
    double v[kParts];
#pragma unroll
    for (int c = 0; c < kParts; ++c) v[c] = 0.0;
    if (p < np && slot_row) {
        const int s = p / slot, o = p - s * slot;
        for (int r = slot_row[s] + way; r < slot_row[s + 1]; r += kCombWays) {
            const double* col = partial + (size_t)(r - row_base) * kParts * slot + o;
#pragma unroll
            for (int c = 0; c < kParts; ++c) v[c] += col[(size_t)c * slot];
        }
    } else if (p < np) {
        const int s = p / slot, o = p - s * slot;
        const size_t row_step = (size_t)slots * kParts * slot;   // next group, same slot
        const double* col = partial + ((size_t)way * slots + s) * kParts * slot + o;
        double a0[kParts], a1[kParts];
#pragma unroll
        for (int c = 0; c < kParts; ++c) a0[c] = a1[c] = 0.0;
        int g = way;
        for (; g + kCombWays < groups; g += 2 * kCombWays, col += 2 * kCombWays * row_step) {
#pragma unroll
            for (int c = 0; c < kParts; ++c) {
                a0[c] += col[(size_t)c * slot];
                a1[c] += col[kCombWays * row_step + (size_t)c * slot];
            }
        }
        if (g < groups) {
#pragma unroll
            for (int c = 0; c < kParts; ++c) a0[c] += col[(size_t)c * slot];
        }
#pragma unroll
        for (int c = 0; c < kParts; ++c) v[c] = a0[c] + a1[c];
    }
#pragma unroll
    for (int c = 0; c < kParts; ++c) red[way][c][lane] = v[c];
    __syncthreads();
    if (way != 0 || p >= np) return;
#pragma unroll
    for (int c = 0; c < kParts; ++c) v[c] = (red[0][c][lane] + red[1][c][lane]) + (red[2][c][lane] + red[3][c][lane]);
    const double R = v[0], gx = v[1] * gscale, gy = v[2] * gscale, gz = v[3] * gscale, om = v[4];
    const double x = pts[p], y = pts[(size_t)np_pad + p], z = pts[2 * (size_t)np_pad + p];
    double S = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int k = 0; k < nc; ++k) {
        const double dx = x - qpos[3 * k], dy = y - qpos[3 * k + 1], dz = z - qpos[3 * k + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < kCoincident * kCoincident) continue;
        const double rinv = 1.0 / sqrt(r2);
        const double t = q[k] * rinv;
        S += t;
        const double t3 = t * rinv * rinv;
        sx -= t3 * dx;
        sy -= t3 * dy;
        sz -= t3 * dz;
    }
    const double cs = kInv4Pi / eps1;
    S *= cs, sx *= cs, sy *= cs, sz *= cs;
    const bool in = om > 0.5;
    const double side = in ? 1.0 : 1.0 / eps;
    constexpr double kUnit = 4.0 * kPi * 332.0716;            // internal -> kcal/(mol e)
    double* o9 = out + (size_t)9 * p;
    o9[0] = kUnit * side * (S + R);
    o9[1] = -kUnit * side * (sx + gx);
    o9[2] = -kUnit * side * (sy + gy);
    o9[3] = -kUnit * side * (sz + gz);
    o9[4] = kUnit * R;
    o9[5] = -kUnit * gx;
    o9[6] = -kUnit * gy;
    o9[7] = -kUnit * gz;
    o9[8] = om;
    inside[p] = in ? 1 : 0;
}

__device__ __forceinline__ uint64_t spread3_bits(uint64_t v) {   // 21 bits -> every third bit
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

__global__ void morton_keys_kernel(const double* __restrict__ raw, int np, double lx, double ly, double lz, double ex,
                                   double ey, double ez, uint64_t* __restrict__ keys, int* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const double lo[3] = {lx, ly, lz}, ext[3] = {ex, ey, ez};
    uint64_t c = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = fmin(fmax((raw[3 * (size_t)i + d] - lo[d]) / ext[d], 0.0), 1.0);
        c |= spread3_bits((uint64_t)(f * 2097151.0)) << d;
    }
    keys[i] = c;
    idx[i] = i;
}

__global__ void stage_points_kernel(const double* __restrict__ raw, const int* __restrict__ order, int np, int np_pad,
                                    double cx, double cy, double cz, double s32, double* __restrict__ pts64,
                                    float* __restrict__ pts32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np_pad) return;
    const int src = order[min(j, np - 1)];
    const double c[3] = {cx, cy, cz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double x = raw[3 * (size_t)src + k];
        pts64[(size_t)k * np_pad + j] = x;
        pts32[(size_t)k * np_pad + j] = (float)((x - c[k]) * s32);
    }
}

// One block per batch of kFieldTreeBatch sorted points: the box of its points (exact min/max).
static_assert(kFieldTreeBatch == 256, "one thread per point of a batch");
__global__ __launch_bounds__(256) void batch_box_kernel(const double* __restrict__ pts64, int np, int np_pad,
                                                        double* __restrict__ bbox) {
    __shared__ double red[6][256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int i = b * kFieldTreeBatch + t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = i < np ? pts64[(size_t)k * np_pad + i] : pts64[(size_t)k * np_pad + b * kFieldTreeBatch];
        red[k][t] = v;
        red[3 + k][t] = v;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                red[k][t] = fmin(red[k][t], red[k][t + w]);
                red[3 + k][t] = fmax(red[3 + k][t], red[3 + k][t + w]);
            }
        }
        __syncthreads();
    }
    if (t < 6) bbox[6 * (size_t)b + t] = red[t][0];
}

// Sorted point p's outputs to the caller's index order[p], split into the ABI's arrays.
__global__ void field_scatter_kernel(const double* __restrict__ out9, const int* __restrict__ ins, int np,
                                     const int* __restrict__ order, double* __restrict__ outc, int* __restrict__ insc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int i = order[p];
    const double* o = out9 + 9 * (size_t)p;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 9; ++k) finite = finite && isfinite(o[k]);
    outc[i] = o[0];                                  // phi
    for (int k = 0; k < 3; ++k) outc[(size_t)np + 3 * (size_t)i + k] = o[1 + k];       // E
    outc[4 * (size_t)np + i] = o[4];                 // R
    for (int k = 0; k < 3; ++k) outc[5 * (size_t)np + 3 * (size_t)i + k] = o[5 + k];   // -grad R
    insc[i] = ins[p];
    if (!finite) insc[np] = 1;
}

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

size_t point_sort_temp_bytes(int np) {
    size_t bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, np, 0, 64) != hipSuccess)
        return 0;
    return std::max<size_t>(bytes, 1);
}

hipError_t launch_point_order(const FieldWork& f, const double lo[3], const double hi[3], const double center[3],
                              double s32, int nbatch, hipStream_t s) {
    double ext[3];
    for (int k = 0; k < 3; ++k) ext[k] = hi[k] - lo[k] > 0 ? hi[k] - lo[k] : 1.0;
    hipLaunchKernelGGL(morton_keys_kernel, dim3(nblk(f.np, 256)), dim3(256), 0, s, f.raw, f.np, lo[0], lo[1], lo[2],
                       ext[0], ext[1], ext[2], f.keys, f.idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = f.cap_sort_tmp;
    if ((e = hipcub::DeviceRadixSort::SortPairs(f.sort_tmp, bytes, f.keys, f.keys + f.np, f.idx, f.order, f.np, 0, 64,
                                                s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(stage_points_kernel, dim3(nblk(f.np_pad, 256)), dim3(256), 0, s, f.raw, f.order, f.np,
                       f.np_pad, center[0], center[1], center[2], s32, f.pts64, f.pts32);
    if (nbatch > 0)
        hipLaunchKernelGGL(batch_box_kernel, dim3(nbatch), dim3(256), 0, s, f.pts64, f.np, f.np_pad, f.bbox);
    return hipGetLastError();
}

hipError_t launch_field_scatter(const FieldWork& f, hipStream_t s) {
    hipLaunchKernelGGL(field_scatter_kernel, dim3(nblk(f.np, 256)), dim3(256), 0, s, f.out, f.inside, f.np, f.order,
                       f.outc, f.insc);
    return hipGetLastError();
}

int field_resident_waves(int device, bool mixed) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    const hipError_t e =
        mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, field_f32_kernel<kFieldTpl32, false>, kBlock, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, field_f64_kernel<kFieldTpl64, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1) return 0;
    return cus * per_cu * kWavesPerBlock;
}

hipError_t launch_field_pairs(const DeviceProblem& p, const FieldWork& f, const PairPlan& pl, bool mixed,
                              hipStream_t s) {
    const bool k0 = p.kappa == 0.0;
    if (mixed) {
        if (k0)
            hipLaunchKernelGGL((field_f32_kernel<kFieldTpl32, true>), dim3(pl.blocks), dim3(kBlock), 0, s, f.pts32,
                               f.np, f.np_pad, p.node32, pl.gstart, pl.slots, pl.workers, f.partial);
        else
            hipLaunchKernelGGL((field_f32_kernel<kFieldTpl32, false>), dim3(pl.blocks), dim3(kBlock), 0, s, f.pts32,
                               f.np, f.np_pad, p.node32, pl.gstart, pl.slots, pl.workers, f.partial);
    } else {
        if (k0)
            hipLaunchKernelGGL((field_f64_kernel<kFieldTpl64, true>), dim3(pl.blocks), dim3(kBlock), 0, s, f.pts64,
                               f.np, f.np_pad, p.node64, p.kappa, pl.gstart, pl.slots, pl.workers, f.partial);
        else
            hipLaunchKernelGGL((field_f64_kernel<kFieldTpl64, false>), dim3(pl.blocks), dim3(kBlock), 0, s, f.pts64,
                               f.np, f.np_pad, p.node64, p.kappa, pl.gstart, pl.slots, pl.workers, f.partial);
    }
    return hipGetLastError();
}

hipError_t launch_field_tree_pairs(const DeviceProblem& p, const FieldWork& f, int nitems, bool mixed,
                                   hipStream_t s) {
    const TreePlan& t = p.tree;
    const bool k0 = p.kappa == 0.0;
    const dim3 grid(nblk(nitems, kWavesPerBlock));
    if (mixed) {
        if (k0)
            hipLaunchKernelGGL((field_tree_f32_kernel<kFieldTpl32, true>), grid, dim3(kBlock), 0, s, f.items, nitems,
                               f.pts32, f.np, f.np_pad, p.node32, t.clu_range, t.prox32, t.nprox, f.partial);
        else
            hipLaunchKernelGGL((field_tree_f32_kernel<kFieldTpl32, false>), grid, dim3(kBlock), 0, s, f.items, nitems,
                               f.pts32, f.np, f.np_pad, p.node32, t.clu_range, t.prox32, t.nprox, f.partial);
    } else {
        if (k0)
            hipLaunchKernelGGL((field_tree_f64_kernel<kFieldTpl64, true>), grid, dim3(kBlock), 0, s, f.items, nitems,
                               f.pts64, f.np, f.np_pad, p.node64, p.kappa, t.clu_range, t.prox64, t.nprox, f.partial);
        else
            hipLaunchKernelGGL((field_tree_f64_kernel<kFieldTpl64, false>), grid, dim3(kBlock), 0, s, f.items, nitems,
                               f.pts64, f.np, f.np_pad, p.node64, p.kappa, t.clu_range, t.prox64, t.nprox, f.partial);
    }
    return hipGetLastError();
}

hipError_t launch_field_combine(const DeviceProblem& p, const FieldWork& f, const PairPlan& pl, bool mixed,
                                hipStream_t s, const int* slot_row, int row_base, int p0, int p1) {
    const double gscale = mixed ? p.s32 : 1.0;
    if (p1 < 0) p1 = f.np;
    if (p1 <= p0) return hipSuccess;
    hipLaunchKernelGGL(field_combine_kernel, dim3(nblk(p1 - p0, kCombPts)), dim3(kCombPts * kCombWays), 0, s,
                       f.partial, slot_row, row_base, p0, p1, pl.slot, pl.slots, pl.groups, gscale, f.pts64, f.np_pad, p.qpos, p.q,
                       p.nc, p.eps1, p.eps, f.out, f.inside);
    return hipGetLastError();
}

}  // namespace hobi
