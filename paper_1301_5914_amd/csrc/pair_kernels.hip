// The matrix-vector product y = A u of the discretised well-posed formulation
// (Section 2.2 eqdbef3/eqdbef4 and Section 2.3 eqdbef5/eqdbef6), in three launches:
//
//   gather_kernel   -- u -> per-node strengths Gamma = w J L.dphi / (4 pi),
//                      Phi = w J L.phi / (4 pi) at the 4 Nf regular nodes
//   pair_f64/f32    -- the dense regular sum over every (vertex, node) pair:
//                      R1_i = sum K1 Gamma + K2 Phi, R2_i = sum K3 Gamma + K4 Phi,
//                      split over source chunks, one FP64 partial per (chunk, vertex)
//   combine_kernel  -- sums the chunk partials in a fixed order, adds the singular
//                      correction (FP64 coefficients) and the diagonal 1/2 (1 + eps).
//
// Pair-kernel layout: each lane owns TPL target vertices in registers; the wavefront
// walks its chunk of source nodes in lock-step, so every node is one wave-uniform
// scalar load (32 or 64 bytes) broadcast to all 64 lanes -- no LDS traffic, no
// barriers, and each target's sum stays in its own lane (no cross-lane reduction).
// exp and rsqrt are VALU transcendental instructions in the FP32 kernel.
#include "hobi_internal.h"

namespace hobi {

namespace {

constexpr int kBlock = 256;
constexpr int kFold = 64;   // FP32 running sums are folded into FP64 every kFold nodes

// Workgroups are dispatched round-robin over the 8 XCDs by linear id.  Give each XCD a
// contiguous range of logical blocks (target block fastest) so that the blocks sharing a
// source chunk run on the same XCD and re-read the chunk from that XCD's L2.
__device__ __forceinline__ void xcd_block(int* tb, int* ch) {
    const int nx = gridDim.x, nb = gridDim.x * gridDim.y;
    const int lin = blockIdx.x + nx * blockIdx.y;
    const int x = lin & 7, slot = lin >> 3;
    const int q = nb >> 3, rm = nb & 7;
    const int logical = x * q + min(x, rm) + slot;
    *tb = logical % nx;
    *ch = logical / nx;
}

__global__ void gather_kernel(const double* __restrict__ u, int nv, const int* __restrict__ tri,
                              const double* __restrict__ w, int nn, NodeD* __restrict__ node64,
                              NodeF* __restrict__ node32, int mixed, double eps) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    const int j = idx >> 2, m = idx & 3;
    double r, s, wm;
    gauss_radau4(m, &r, &s, &wm);
    const double L0 = 1.0 - r - s, L1 = r, L2 = s;
    const int v0 = tri[3 * j], v1 = tri[3 * j + 1], v2 = tri[3 * j + 2];
    const double dp = L0 * u[nv + v0] + L1 * u[nv + v1] + L2 * u[nv + v2];
    const double pp = L0 * u[v0] + L1 * u[v1] + L2 * u[v2];
    const double sc = w[idx] * kInv4Pi;
    const double g = sc * dp, p = sc * pp;
    node64[idx].g = g;
    node64[idx].p = p;
    if (mixed) {
        NodeF& n = node32[idx];
        n.g = (float)g;
        n.p = (float)p;
        n.ga = (float)(-(1.0 - 1.0 / eps) * g);
        n.gb = (float)(-g / eps);
        n.pa = (float)((eps - 1.0) * p);
        n.pb = (float)(-eps * p);
    }
}

template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void pair_f64_kernel(
    const double* __restrict__ tgt, int nv_pad, const NodeD* __restrict__ nodes, int nn, int chunk,
    double kappa, double eps, double* __restrict__ partial) {
    int tb, ch;
    xcd_block(&tb, &ch);
    const int t0 = tb * (kBlock * TPL) + threadIdx.x;
    double tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL], a1[TPL], a2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kBlock;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        a1[k] = 0.0;
        a2[k] = 0.0;
    }
    const double em1 = eps - 1.0, ce3 = 1.0 - 1.0 / eps, ie = 1.0 / eps;
    const int s0 = ch * chunk;
    const int s1 = min(s0 + chunk, nn);
    for (int s = s0; s < s1; ++s) {
        const NodeD nd = nodes[s];
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const double dx = tx[k] - nd.x, dy = ty[k] - nd.y, dz = tz[k] - nd.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double rinv = rsqrt(r2);
            const double rinv3 = rinv * rinv * rinv;
            const double dny = dx * nd.nx + dy * nd.ny + dz * nd.nz;
            const double dnx = dx * tnx[k] + dy * tny[k] + dz * tnz[k];
            if (KAPPA0) {
                a1[k] += em1 * dny * rinv3 * nd.p;
                a2[k] -= ce3 * dnx * rinv3 * nd.g;
            } else {
                const double nxy = tnx[k] * nd.nx + tny[k] * nd.ny + tnz[k] * nd.nz;
                double f0, f1, f2;
                f012_f64(kappa * (r2 * rinv), &f0, &f1, &f2);
                const double K1 = f0 * rinv;
                const double K2 = dny * rinv3 * (em1 - eps * f1);
                const double K3 = -dnx * rinv3 * (ce3 + f1 * ie);
                const double K4 = (dnx * dny * f2 * (rinv * rinv) - nxy * f1) * rinv3;
                a1[k] += K1 * nd.g + K2 * nd.p;
                a2[k] += K3 * nd.g + K4 * nd.p;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kBlock;
        partial[(size_t)(2 * ch) * nv_pad + t] = a1[k];
        partial[(size_t)(2 * ch + 1) * nv_pad + t] = a2[k];
    }
}

// FP32 pairs, FP64 accumulation: running FP32 sums over kFold nodes are added into
// FP64 per-target accumulators.  Per pair (kappa > 0): 38 VALU operations plus one
// rsqrt and one exp2 on the transcendental unit.
template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void pair_f32_kernel(
    const float* __restrict__ tgt, int nv_pad, const NodeF* __restrict__ nodes, int nn, int chunk,
    float kappa, float kl2n, double* __restrict__ partial) {
    int tb, ch;
    xcd_block(&tb, &ch);
    const int t0 = tb * (kBlock * TPL) + threadIdx.x;
    float tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL];
    double d1[TPL], d2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kBlock;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        d1[k] = 0.0;
        d2[k] = 0.0;
    }
    const int s0 = ch * chunk;
    const int s1 = min(s0 + chunk, nn);
    for (int sb = s0; sb < s1; sb += kFold) {
        const int se = min(sb + kFold, s1);
        float a1[TPL], a2[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) a1[k] = a2[k] = 0.0f;
        for (int s = sb; s < se; ++s) {
            const NodeF n = nodes[s];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const float dx = tx[k] - n.x, dy = ty[k] - n.y, dz = tz[k] - n.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float rinv2 = rinv * rinv;
                const float rinv3 = rinv2 * rinv;
                const float dny = fmaf(dx, n.nx, fmaf(dy, n.ny, dz * n.nz));
                const float dnx = fmaf(dx, tnx[k], fmaf(dy, tny[k], dz * tnz[k]));
                if (KAPPA0) {
                    a1[k] = fmaf(dny * rinv3, n.pa, a1[k]);
                    a2[k] = fmaf(dnx * rinv3, n.ga, a2[k]);
                } else {
                    const float nxy = fmaf(tnx[k], n.nx, fmaf(tny[k], n.ny, tnz[k] * n.nz));
                    const float r = r2 * rinv;
                    const float e = __builtin_amdgcn_exp2f(kl2n * r);         // exp(-kappa r)
                    const float zp1 = fmaf(kappa, r, 1.0f);                  // 1 + z
                    const float f1 = fmaf(-e, zp1, 1.0f);                    // 1 - e (1 + z)
                    const float f2 = fmaf(-e, fmaf(zp1, zp1 + 1.0f, 1.0f), 3.0f);   // 3 - e (3 + 3z + z^2)
                    // row 1: K1 Gamma + K2 Phi = (Gamma - e Gamma)/r + (d.ny)/r^3 (pa + pb f1)
                    a1[k] = fmaf(dny * rinv3, fmaf(n.pb, f1, n.pa), a1[k]);
                    a1[k] = fmaf(fmaf(-e, n.g, n.g), rinv, a1[k]);
                    // row 2: K3 Gamma + K4 Phi = [(d.nx)(ga + gb f1) + Phi ((d.nx)(d.ny) f2 / r^2 - (nx.ny) f1)] / r^3
                    const float w = fmaf(dnx * dny * f2, rinv2, -nxy * f1);
                    a2[k] = fmaf(rinv3, fmaf(w, n.p, dnx * fmaf(n.gb, f1, n.ga)), a2[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            d1[k] += (double)a1[k];
            d2[k] += (double)a2[k];
        }
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kBlock;
        partial[(size_t)(2 * ch) * nv_pad + t] = d1[k];
        partial[(size_t)(2 * ch + 1) * nv_pad + t] = d2[k];
    }
}

__global__ void combine_kernel(const double* __restrict__ u, double* __restrict__ y, int nv, int nv_pad,
                               const double* __restrict__ partial, int chunks,
                               const int* __restrict__ inc_off, const int* __restrict__ inc_ent,
                               const int* __restrict__ tri, const double* __restrict__ coef,
                               double eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double r1 = 0.0, r2 = 0.0;
    for (int c = 0; c < chunks; ++c) {
        r1 += partial[(size_t)(2 * c) * nv_pad + i];
        r2 += partial[(size_t)(2 * c + 1) * nv_pad + i];
    }
    double c1 = 0.0, c2 = 0.0;
    for (int e = inc_off[i]; e < inc_off[i + 1]; ++e) {
        const int ent = inc_ent[e];
        const int j = ent / 3, k = ent - 3 * (ent / 3);
        const double* co = coef + 12 * (size_t)ent;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int v = tri[3 * j + (k + b) % 3];
            const double ph = u[v], dp = u[nv + v];
            c1 += co[b] * dp + co[3 + b] * ph;
            c2 += co[6 + b] * dp + co[9 + b] * ph;
        }
    }
    y[i] = 0.5 * (1.0 + eps) * u[i] - r1 - c1;
    y[nv + i] = 0.5 * (1.0 + 1.0 / eps) * u[nv + i] - r2 - c2;
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

// MODE 0: phi_reac[p] = sum over chunks; E = 1/2 * 4 pi C * sum_p q_p phi_reac[p].
// MODE 1: out[p] = -(sum over chunks) / (4 pi).  One block, fixed reduction order.
template <int MODE>
__global__ __launch_bounds__(256) void point_reduce_kernel(const double* __restrict__ partial, int np,
                                                           int np_pad, int chunks,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ out,
                                                           double* __restrict__ e_out) {
    __shared__ double red[256];
    double local = 0.0;
    for (int p = threadIdx.x; p < np; p += 256) {
        double v = 0.0;
        for (int c = 0; c < chunks; ++c) v += partial[(size_t)c * np_pad + p];
        if (MODE == 0) {
            out[p] = v;
            local += q[p] * v;
        } else {
            out[p] = -v * kInv4Pi;
        }
    }
    red[threadIdx.x] = local;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (MODE == 0 && threadIdx.x == 0) e_out[0] = 0.5 * 4.0 * kPi * 332.0716 * red[0];
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

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

PairPlan make_plan(int n_pad, int nn, int tpl) {
    PairPlan pl{};
    pl.tpl = tpl;
    pl.block = kBlock;
    pl.target_blocks = n_pad / (kBlock * tpl);
    if (pl.target_blocks < 1) pl.target_blocks = 1;
    // about 8 resident blocks per compute unit on 256 CUs; at least 256 nodes per chunk
    const int want = 2048;
    int chunks = (want + pl.target_blocks - 1) / pl.target_blocks;
    const int max_chunks = nn / 256 > 1 ? nn / 256 : 1;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    pl.chunk = (nn + chunks - 1) / chunks;
    pl.chunks = (nn + pl.chunk - 1) / pl.chunk;
    return pl;
}

hipError_t launch_gather(const DeviceProblem& p, const double* u, bool mixed, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3(nblk(p.nn, 256)), dim3(256), 0, s, u, p.nv, p.tri, p.w, p.nn,
                       p.node64, p.node32, mixed ? 1 : 0, p.eps);
    return hipGetLastError();
}

hipError_t launch_pair(const DeviceProblem& p, bool mixed, hipStream_t s) {
    const bool k0 = p.kappa == 0.0;
    if (mixed) {
        const PairPlan& pl = p.plan32;
        dim3 grid(pl.target_blocks, pl.chunks);
        const float kappa = (float)p.kappa, kl2n = (float)(-p.kappa * 1.4426950408889634074);
#define HOBI_PAIR32(T, K0)                                                                        \
    hipLaunchKernelGGL((pair_f32_kernel<T, K0>), grid, dim3(kBlock), 0, s, p.tgt32, p.nv_pad, p.node32, \
                       p.nn, pl.chunk, kappa, kl2n, p.partial)
        if (pl.tpl == 8) {
            if (k0) HOBI_PAIR32(8, true); else HOBI_PAIR32(8, false);
        } else {
            if (k0) HOBI_PAIR32(4, true); else HOBI_PAIR32(4, false);
        }
#undef HOBI_PAIR32
    } else {
        const PairPlan& pl = p.plan64;
        dim3 grid(pl.target_blocks, pl.chunks);
        if (k0)
            hipLaunchKernelGGL((pair_f64_kernel<2, true>), grid, dim3(kBlock), 0, s, p.tgt64, p.nv_pad,
                               p.node64, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
        else
            hipLaunchKernelGGL((pair_f64_kernel<2, false>), grid, dim3(kBlock), 0, s, p.tgt64, p.nv_pad,
                               p.node64, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
    }
    return hipGetLastError();
}

hipError_t launch_combine(const DeviceProblem& p, const double* u, double* y, bool mixed, hipStream_t s) {
    const int chunks = mixed ? p.plan32.chunks : p.plan64.chunks;
    hipLaunchKernelGGL(combine_kernel, dim3(nblk(p.nv, 256)), dim3(256), 0, s, u, y, p.nv, p.nv_pad,
                       p.partial, chunks, p.inc_off, p.inc_ent, p.tri, p.coef, p.eps);
    return hipGetLastError();
}

hipError_t launch_reaction_energy(const DeviceProblem& p, double* phi_reac, double* e_out, hipStream_t s) {
    const PairPlan& pl = p.plan_pts;
    hipLaunchKernelGGL((point_sum_kernel<0>), dim3(pl.target_blocks, pl.chunks), dim3(kBlock), 0, s, p.qsoa,
                       p.nc_pad, p.node64, p.w, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((point_reduce_kernel<0>), dim3(1), dim3(256), 0, s, p.partial, p.nc, p.nc_pad,
                       pl.chunks, p.q, phi_reac, e_out);
    return hipGetLastError();
}

hipError_t launch_solid_angle(const DeviceProblem& p, double* frac, hipStream_t s) {
    const PairPlan& pl = p.plan_pts;
    hipLaunchKernelGGL((point_sum_kernel<1>), dim3(pl.target_blocks, pl.chunks), dim3(kBlock), 0, s, p.qsoa,
                       p.nc_pad, p.node64, p.w, p.nn, pl.chunk, p.kappa, p.eps, p.partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((point_reduce_kernel<1>), dim3(1), dim3(256), 0, s, p.partial, p.nc, p.nc_pad,
                       pl.chunks, p.q, frac, (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_permute(const double* in, double* out, const int* perm, int nv, bool to_internal,
                          hipStream_t s) {
    hipLaunchKernelGGL(permute_kernel, dim3(nblk(nv, 256)), dim3(256), 0, s, in, out, perm, nv,
                       to_internal ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hobi
