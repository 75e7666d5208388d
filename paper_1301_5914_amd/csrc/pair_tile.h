// The dense pair sum of one wave ("worker"): one slot of targets against one contiguous
// range of source nodes.  Shared by the single-problem kernels and the batched
// kernels of the request server, so that a request's partial sums are bit-for-bit the
// same whichever launch computes them.
#pragma once

#include "exp2_table.h"
#include "hobi_device.h"

namespace hobi {

constexpr int kPairBlock = 256;
constexpr int kFold = 64;   // FP32 running sums are folded into FP64 every kFold nodes
constexpr int kWave = 64;
constexpr float kLog2E = 1.44269504088896340736f;   // exp(-z) = exp2(-z log2 e)

// Target slots.  Slot s holds the kWave * TPL targets from s * kWave * TPL, lane l holding
// (slot start) + kWave * k + l for k < TPL.  The wave holding the last slot narrows TPL to
// what that slot holds (halving while the real targets still fit), so the padding of the
// target count costs at most 63 targets' work.  Partials of padding targets are neither
// written nor read.

// Source records are read-only for the whole launch and every wave reads them at
// wave-uniform addresses: reading them through the constant address space makes each
// record a single scalar load (s_load) broadcast to the wave, also when the pointer
// itself was loaded from memory (the batched kernels' descriptors).
template <class T>
using const_as = const T __attribute__((address_space(4)));

template <class T>
__device__ __forceinline__ const const_as<T>* as_constant(const T* p) {
    return (const const_as<T>*)p;
}

__device__ __forceinline__ NodeF load_node(const const_as<NodeF>* p, int s) {
    NodeF n;
    n.x = p[s].x, n.y = p[s].y, n.z = p[s].z;
    n.nx = p[s].nx, n.ny = p[s].ny, n.nz = p[s].nz;
    n.g = p[s].g, n.p = p[s].p, n.ga = p[s].ga, n.gb = p[s].gb, n.pa = p[s].pa, n.pb = p[s].pb;
    n.qx = p[s].qx, n.qy = p[s].qy, n.qz = p[s].qz, n.pad = p[s].pad;
    return n;
}

__device__ __forceinline__ ProxyF load_proxy(const const_as<ProxyF>* p, int k) {
    ProxyF r;
    r.x = p[k].x, r.y = p[k].y, r.z = p[k].z, r.q0a = p[k].q0a;
    r.qka = p[k].qka, r.q0b = p[k].q0b, r.qk2b = p[k].qk2b, r.qs = p[k].qs;
    return r;
}

__device__ __forceinline__ ProxyD load_proxy(const const_as<ProxyD>* p, int k) {
    ProxyD r;
    r.x = p[k].x, r.y = p[k].y, r.z = p[k].z, r.q0 = p[k].q0, r.qk = p[k].qk, r.qk2 = p[k].qk2;
    r.qs = p[k].qs, r.pad = 0.0;
    return r;
}

__device__ __forceinline__ int4 load_vid(const const_as<int4>* p, int s) {
    return make_int4(p[s].x, p[s].y, p[s].z, 0);
}

// Lanes of target slot k (targets base + 64 k + lane) that are vertices of the node's
// triangle, as a wave-wide lane mask: vid holds the vertex ids and base is wave-uniform,
// so the mask is built with scalar instructions and applied with one conditional move per
// slot (the mask is the move's lane condition).
template <int K>
__device__ __forceinline__ uint64_t vertex_lanes(int4 vid, int base) {
    const unsigned ux = (unsigned)(vid.x - base), uy = (unsigned)(vid.y - base), uz = (unsigned)(vid.z - base);
    uint64_t m = 0;
    if ((ux >> 6) == (unsigned)K) m |= 1ull << (ux & 63);
    if ((uy >> 6) == (unsigned)K) m |= 1ull << (uy & 63);
    if ((uz >> 6) == (unsigned)K) m |= 1ull << (uz & 63);
    return m;
}

template <int TPL, int K = 0>
__device__ __forceinline__ void vertex_lane_masks(int4 vid, int base, uint64_t (&m)[TPL]) {
    m[K] = vertex_lanes<K>(vid, base);
    if constexpr (K + 1 < TPL) vertex_lane_masks<TPL, K + 1>(vid, base, m);
}

__device__ __forceinline__ NodeD load_node(const const_as<NodeD>* p, int s) {
    NodeD n;
    n.x = p[s].x, n.y = p[s].y, n.z = p[s].z, n.g = p[s].g;
    n.nx = p[s].nx, n.ny = p[s].ny, n.nz = p[s].nz, n.p = p[s].p;
    n.ga = p[s].ga, n.gb = p[s].gb, n.pa = p[s].pa, n.pb = p[s].pb;
    n.qx = p[s].qx, n.qy = p[s].qy, n.qz = p[s].qz, n.pad = p[s].pad;
    return n;
}

// FP32 pairs of nodes [sb, se) with the lane's TPL targets, added to FP32 running sums.
// Positions are in units of 1 / kappa when kappa > 0, so that z = kappa r = r: with
// zp1 = 1 + z = r^2 / r + 1, exp(-z) = exp2(log2 e (1 - zp1)) and 3 + 3z + z^2 = 3 zp1 + r^2
// (the strengths carry the matching powers of the unit).  Per pair (kappa > 0): 32 VALU
// operations plus one rsqrt and one exp2.  With
// q = (d.ny)/r^2, the two rows are
//   row 1: K1 Gamma + K2 Phi = [Gamma (1 - e) + q (pa + pb f1)] / r
//   row 2: K3 Gamma + K4 Phi = [(d.nx)(ga + gb f1 + p q f2) - (nx.P) f1] / r^3,  P = p ny,
// which is the kernel algebra with the node strengths folded in.  f2 is never formed: since
// f2 = 3 f1 - z^2 e and q z^2 = (d.ny) (z = r in this frame), the strength of row 2 is
// ga + f1 (gb + 3p q) - p (d.ny) e, where 3p is taken once per node for the lane's TPL
// targets.  With MASK, pairs of a vertex with its own triangles' nodes (they belong to the
// singular rule) are skipped.
template <int TPL, bool KAPPA0, bool MASK>
__device__ __forceinline__ void pair_f32_run(const const_as<NodeF>* cnodes, const const_as<int4>* cvid, int sb,
                                             int se, int base, const float (&tx)[TPL], const float (&ty)[TPL],
                                             const float (&tz)[TPL], const float (&tnx)[TPL],
                                             const float (&tny)[TPL], const float (&tnz)[TPL],
                                             float (&a1)[TPL], float (&a2)[TPL]) {
    NodeF n = load_node(cnodes, sb);
    for (int s = sb; s < se; ++s) {
        // the next record's scalar load is in flight while this one is used
        const NodeF next = load_node(cnodes, min(s + 1, se - 1));
        uint64_t vmask[TPL];
        if (MASK) vertex_lane_masks<TPL>(load_vid(cvid, s), base, vmask);
        const float p3 = 3.0f * n.p;
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const float dx = tx[k] - n.x, dy = ty[k] - n.y, dz = tz[k] - n.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            float rinv = __builtin_amdgcn_rsqf(r2);
            if (MASK && __builtin_amdgcn_inverse_ballot_w64(vmask[k])) rinv = 0.0f;
            const float rinv2 = rinv * rinv;
            const float dny = fmaf(dx, n.nx, fmaf(dy, n.ny, dz * n.nz));
            const float dnx = fmaf(dx, tnx[k], fmaf(dy, tny[k], dz * tnz[k]));
            if (KAPPA0) {
                const float rinv3 = rinv2 * rinv;
                a1[k] = fmaf(dny * rinv3, n.pa, a1[k]);
                a2[k] = fmaf(dnx * rinv3, n.ga, a2[k]);
            } else {
                const float pnxy = fmaf(tnx[k], n.qx, fmaf(tny[k], n.qy, tnz[k] * n.qz));
                const float zp1 = fmaf(r2, rinv, 1.0f);                  // 1 + z
                const float e = __builtin_amdgcn_exp2f(fmaf(zp1, -kLog2E, kLog2E));   // exp(-z)
                const float f1 = fmaf(-e, zp1, 1.0f);                    // 1 - e (1 + z)
                const float q = dny * rinv2;
                a1[k] = fmaf(rinv, fmaf(q, fmaf(n.pb, f1, n.pa), fmaf(-e, n.g, n.g)), a1[k]);
                const float t = fmaf(-(n.p * dny), e, fmaf(f1, fmaf(p3, q, n.gb), n.ga));
                a2[k] = fmaf(rinv2 * rinv, fmaf(-pnxy, f1, dnx * t), a2[k]);
            }
        }
        n = next;
    }
}

// FP32 pairs, FP64 accumulation, of the kWave * TPL targets from `base` (wave-uniform) with
// the kFold-aligned node blocks part, part + step, ... of the nodes [n0, n1) (all of them for
// part 0, step 1): running FP32 sums over the nodes of one kFold-aligned block are added
// into FP64 per-target accumulators, stored to row `prow` of the partial sums (row 1 sums
// at prow[t - base], row 2 sums at prow[slot + t - base]).  blk_range[b] = (min, max)
// vertex id of the triangles of nodes [kFold b, kFold b + kFold); a wave whose targets miss
// it runs the unmasked loop.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f32_wave(
    const float* __restrict__ tgt, int nv_pad, const NodeF* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, int base, int n0, int n1,
    double* __restrict__ prow, int slot, int part, int step) {
    const int lane = (int)(threadIdx.x % kWave);
    const int t0 = base + lane;
    float tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL];
    double d1[TPL], d2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kWave;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        d1[k] = 0.0;
        d2[k] = 0.0;
    }
    const const_as<NodeF>* cnodes = as_constant(nodes);
    const const_as<int4>* cvid = as_constant(node_vid);
    const const_as<int2>* crange = as_constant(blk_range);
    // the kFold-aligned node blocks part, part + step, part + 2 step, ... of [n0, n1)
    for (int f = n0 / kFold + part; f * kFold < n1; f += step) {
        const int sb = max(f * kFold, n0), se = min(f * kFold + kFold, n1);
        const int vlo = crange[f].x, vhi = crange[f].y;
        const bool near = (vhi >= base) & (vlo < base + kWave * TPL);
        float a1[TPL], a2[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) a1[k] = a2[k] = 0.0f;
        if (near)
            pair_f32_run<TPL, KAPPA0, true>(cnodes, cvid, sb, se, base, tx, ty, tz, tnx, tny, tnz, a1, a2);
        else
            pair_f32_run<TPL, KAPPA0, false>(cnodes, cvid, sb, se, base, tx, ty, tz, tnx, tny, tnz, a1, a2);
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            d1[k] += (double)a1[k];
            d2[k] += (double)a2[k];
        }
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        prow[lane + k * kWave] = d1[k];
        prow[slot + lane + k * kWave] = d2[k];
    }
}

// The slot from `base` with `live` = nv - base >= 1 real targets in it: the narrowest TPL
// (halving) whose kWave * TPL targets still cover them.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f32_narrow(
    int live, const float* __restrict__ tgt, int nv_pad, const NodeF* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, int base, int n0, int n1,
    double* __restrict__ prow, int slot, int part = 0, int step = 1) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            pair_f32_narrow<TPL / 2, KAPPA0>(live, tgt, nv_pad, nodes, node_vid, blk_range, base, n0, n1, prow, slot,
                                             part, step);
            return;
        }
    }
    pair_f32_wave<TPL, KAPPA0>(tgt, nv_pad, nodes, node_vid, blk_range, base, n0, n1, prow, slot, part, step);
}

// The kPairWaves rows of a block (row w at red + w * 2 * kSlot, in LDS) summed in wave order
// into the block's partial row, for the `live` real targets of the slot.  All threads of the
// block call it, after a barrier that follows the waves' writes.
template <int kSlot>
__device__ __forceinline__ void sum_wave_rows(const double* red, int live, double* __restrict__ row) {
    for (int j = (int)threadIdx.x; j < 2 * kSlot; j += kPairBlock) {
        if ((j < kSlot ? j : j - kSlot) < live) {
            double v = red[j];
#pragma unroll
            for (int w = 1; w < kPairWaves; ++w) v += red[w * 2 * kSlot + j];
            row[j] = v;
        }
    }
}

// Block b of a pair plan with per_row = kPairWaves, `slots` target slots and node groups
// [gstart[g], gstart[g + 1]): slot b % slots against the nodes of groups
// kPairWaves (b / slots) .. kPairWaves (b / slots) + kPairWaves - 1.  Wave w takes the
// kFold-aligned node blocks w, w + kPairWaves, ... of that range (so the waves meet the
// costlier masked blocks near the slot's own vertices in equal shares) into its LDS row, and
// the block writes the rows' sum to partial row b.  red: kPairWaves * 2 * kWave * TPL doubles of LDS.  b must be block-uniform and
// below slots * groups / kPairWaves; all threads of the block call it.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f32_block(
    const float* __restrict__ tgt, int nv, int nv_pad, const NodeF* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, const int* __restrict__ gstart,
    int slots, double* __restrict__ partial, int b, double* red) {
    constexpr int kSlot = kWave * TPL;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int q = b / slots, s = b - q * slots;
    const const_as<int>* cg = as_constant(gstart);
    const int base = s * kSlot;
    pair_f32_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, nodes, node_vid, blk_range, base, cg[q * kPairWaves],
                                 cg[q * kPairWaves + kPairWaves], red + wave * (2 * kSlot), kSlot, wave, kPairWaves);
    __syncthreads();
    sum_wave_rows<kSlot>(red, nv - base, partial + (size_t)b * (2 * kSlot));
    __syncthreads();   // red may be reused at once
}

// Node strengths Gamma = g, Phi = p (1/(4 pi) folded in) and the quantities derived from
// them into the FP64 and FP32 records of node idx.  The FP32 record's positions are in
// units of 1/s32; its strengths carry the matching powers of s32 (Gamma terms over r and
// (d.ny)/r^3 terms: s32, s32^2; the Phi term of K4: s32^3).
__device__ __forceinline__ void write_strengths(int idx, double g, double p, NodeD* __restrict__ node64,
                                                NodeF* __restrict__ node32, int mixed, double eps, double s32) {
    {
        NodeD& n = node64[idx];
        n.g = g;
        n.p = p;
        n.ga = -(1.0 - 1.0 / eps) * g;
        n.gb = -g / eps;
        n.pa = (eps - 1.0) * p;
        n.pb = -eps * p;
        n.qx = p * n.nx;
        n.qy = p * n.ny;
        n.qz = p * n.nz;
    }
    if (mixed) {
        const NodeD& d = node64[idx];
        NodeF& n = node32[idx];
        const double s2 = s32 * s32, s3 = s2 * s32;
        n.g = (float)(s32 * g);
        n.p = (float)(s3 * p);
        n.ga = (float)(-(1.0 - 1.0 / eps) * s2 * g);
        n.gb = (float)(-s2 * g / eps);
        n.pa = (float)((eps - 1.0) * s2 * p);
        n.pb = (float)(-eps * s2 * p);
        n.qx = (float)(s3 * p * d.nx);
        n.qy = (float)(s3 * p * d.ny);
        n.qz = (float)(s3 * p * d.nz);
    }
}

// Higher-order method: regular node idx = 4 j + m of triangle j interpolates the vertex
// unknowns linearly (W_{j,m,n} of eqdbef3/eqdbef4).
__device__ __forceinline__ void gather_node(int idx, const double* __restrict__ u, int nv,
                                            const int* __restrict__ tri, const double* __restrict__ w,
                                            NodeD* __restrict__ node64, NodeF* __restrict__ node32,
                                            int mixed, double eps, double s32) {
    const int j = idx >> 2, m = idx & 3;
    double r, s, wm;
    gauss_radau4(m, &r, &s, &wm);
    const double L0 = 1.0 - r - s, L1 = r, L2 = s;
    const int v0 = tri[3 * j], v1 = tri[3 * j + 1], v2 = tri[3 * j + 2];
    const double dp = L0 * u[nv + v0] + L1 * u[nv + v1] + L2 * u[nv + v2];
    const double pp = L0 * u[v0] + L1 * u[v1] + L2 * u[v2];
    const double sc = w[idx] * kInv4Pi;
    write_strengths(idx, sc * dp, sc * pp, node64, node32, mixed, eps, s32);
}

// Lower-order method: node j is site j (eqdbef1/eqdbef2), weight = triangle area.
__device__ __forceinline__ void gather_site(int j, const double* __restrict__ u, int nv,
                                            const double* __restrict__ w, NodeD* __restrict__ node64,
                                            NodeF* __restrict__ node32, int mixed, double eps, double s32) {
    const double sc = w[j] * kInv4Pi;
    write_strengths(j, sc * u[nv + j], sc * u[j], node64, node32, mixed, eps, s32);
}

// exp(-z) for 0 <= z < kExpTabMaxZ in FP64 by Tang's table-driven method (P. T. P. Tang, ACM
// TOMS 15, 1989), in the negated reduction: m = rint(-256 z log2(e)) = 256 k + j
// (0 <= j < 256, k <= 0), r = z + m ln2/256 with |r| <= ln2/512 (Cody-Waite: ln2/256 split
// into a 32-bit head, so m * head is exact, and a tail), and exp(-z) = 2^k * 2^(j/256) *
// exp(-r), so that j and k are the low byte and the arithmetic shift of m as it stands.  m
// comes from adding 1.5 * 2^52 to -256 z log2(e) in one fused multiply-add: the sum's rounding
// is the rounding to an integer, its low 32 bits are m, and subtracting the constant again
// gives m exactly.  The 256 values 2^(j/256), each the nearest double (exp2_table.h), sit in
// LDS (fill_exp_table, once per workgroup); exp(-r) - 1 is its Taylor polynomial to degree 4
// (truncation below 4e-17), added as T + T (exp(-r) - 1) by one fused multiply-add.  Measured against an
// extended-precision reference: within 1.3 units in the last place.  Past z = 745 the result
// underflows to 0; the problem checks (kappa times its extent) keep z below kExpTabMaxZ,
// where n fits an int.
constexpr int kExpTab = 256;

// Must be called by every thread of the workgroup (it synchronises them).
__device__ __forceinline__ void fill_exp_table(double* __restrict__ tab) {
    for (int j = (int)threadIdx.x; j < kExpTab; j += (int)blockDim.x) tab[j] = kExp2Tab256[j];
    __syncthreads();
}

__device__ __forceinline__ double exp_neg_tab_f64(double z, const double* __restrict__ tab) {
    constexpr double kC = kExpTab * 1.44269504088896340735992468100189214;   // 256 log2(e)
    constexpr double kShift = 0x1.8p52;                                        // 1.5 * 2^52
    const double y = fma(z, -kC, kShift);
    const double m = y - kShift;
    const int mi = (int)(unsigned)__builtin_bit_cast(unsigned long long, y);
    double r = fma(m, kLn2Step256Hi, z);
    r = fma(m, kLn2Step256Lo, r);
    double p = fma(r, 1.0 / 24.0, -1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, -1.0);
    const double q = p * r;                       // exp(-r) - 1
    const double t = tab[mi & (kExpTab - 1)];
    return __builtin_amdgcn_ldexp(fma(t, q, t), mi >> 8);
}

// FP64 pairs of nodes [sb, se) with the lane's TPL targets.  Per pair (kappa > 0) about 48
// FP64 operations: the reciprocal square root of hobi_device.h, the table-driven exponential
// above (etab: its LDS table), and the closed forms of f1 and 1 - e, whose cancellation
// for small z = kappa r costs an absolute error of a few units of 1e-16, the size of the
// rows' other rounding errors; the rows as in the FP32 tile, with the strengths
// pre-multiplied by the epsilon factors and f2 folded into the strength of row 2 as there:
// f2 = 3 f1 - z^2 e with q z^2 = kappa^2 (d.ny), the node factors 3 Phi and kappa^2 Phi
// taken once per node for the lane's TPL targets.  With MASK, pairs of a vertex with its own
// triangles' nodes are skipped.
template <int TPL, bool KAPPA0, bool MASK>
__device__ __forceinline__ void pair_f64_run(const const_as<NodeD>* cnodes, const const_as<int4>* cvid, int sb,
                                             int se, int base, const double (&tx)[TPL], const double (&ty)[TPL],
                                             const double (&tz)[TPL], const double (&tnx)[TPL],
                                             const double (&tny)[TPL], const double (&tnz)[TPL], double kappa,
                                             const double* __restrict__ etab, double (&a1)[TPL], double (&a2)[TPL]) {
    const double kappa2 = kappa * kappa;
    for (int s = sb; s < se; ++s) {
        const NodeD nd = load_node(cnodes, s);   // (a prefetched FP64 record would not fit the scalar registers)
        uint64_t vmask[TPL];
        if (MASK) vertex_lane_masks<TPL>(load_vid(cvid, s), base, vmask);
        const double p3 = 3.0 * nd.p, pk2 = nd.p * kappa2;
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const double dx = tx[k] - nd.x, dy = ty[k] - nd.y, dz = tz[k] - nd.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            double rinv = rsqrt_f64(r2);
            if (MASK && __builtin_amdgcn_inverse_ballot_w64(vmask[k])) rinv = 0.0;
            const double rinv2 = rinv * rinv;
            const double dny = fma(dx, nd.nx, fma(dy, nd.ny, dz * nd.nz));
            const double dnx = fma(dx, tnx[k], fma(dy, tny[k], dz * tnz[k]));
            if (KAPPA0) {
                const double rinv3 = rinv2 * rinv;
                a1[k] = fma(dny * rinv3, nd.pa, a1[k]);
                a2[k] = fma(dnx * rinv3, nd.ga, a2[k]);
            } else {
                const double pnxy = fma(tnx[k], nd.qx, fma(tny[k], nd.qy, tnz[k] * nd.qz));
                const double z = kappa * (r2 * rinv);
                const double e = exp_neg_tab_f64(z, etab);
                const double zp1 = z + 1.0;
                const double f1 = fma(-e, zp1, 1.0);                          // 1 - e (1 + z)
                // the FP32 tile's row algebra: q = (d.ny)/r^2, P = Phi ny
                const double q = dny * rinv2;
                a1[k] = fma(rinv, fma(q, fma(nd.pb, f1, nd.pa), fma(-e, nd.g, nd.g)), a1[k]);
                const double t = fma(-(pk2 * dny), e, fma(f1, fma(p3, q, nd.gb), nd.ga));
                a2[k] = fma(rinv2 * rinv, fma(-pnxy, f1, dnx * t), a2[k]);
            }
        }
    }
}

// FP64 pairs of the kWave * TPL targets from `base` with the node blocks part, part + step,
// ... of [n0, n1), stored to row `prow` as in the FP32 wave (same block-range test).
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f64_wave(
    const double* __restrict__ tgt, int nv_pad, const NodeD* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, double kappa,
    const double* __restrict__ etab, int base, int n0, int n1, double* __restrict__ prow, int slot, int part,
    int step) {
    const int lane = (int)(threadIdx.x % kWave);
    const int t0 = base + lane;
    double tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL], a1[TPL], a2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = t0 + k * kWave;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        a1[k] = 0.0;
        a2[k] = 0.0;
    }
    const const_as<NodeD>* cnodes = as_constant(nodes);
    const const_as<int4>* cvid = as_constant(node_vid);
    const const_as<int2>* crange = as_constant(blk_range);
    // the kFold-aligned node blocks part, part + step, part + 2 step, ... of [n0, n1)
    for (int f = n0 / kFold + part; f * kFold < n1; f += step) {
        const int sb = max(f * kFold, n0), se = min(f * kFold + kFold, n1);
        const int vlo = crange[f].x, vhi = crange[f].y;
        const bool near = (vhi >= base) & (vlo < base + kWave * TPL);
        if (near)
            pair_f64_run<TPL, KAPPA0, true>(cnodes, cvid, sb, se, base, tx, ty, tz, tnx, tny, tnz, kappa, etab, a1,
                                            a2);
        else
            pair_f64_run<TPL, KAPPA0, false>(cnodes, cvid, sb, se, base, tx, ty, tz, tnx, tny, tnz, kappa, etab, a1,
                                             a2);
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        prow[lane + k * kWave] = a1[k];
        prow[slot + lane + k * kWave] = a2[k];
    }
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f64_narrow(
    int live, const double* __restrict__ tgt, int nv_pad, const NodeD* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, double kappa,
    const double* __restrict__ etab, int base, int n0, int n1, double* __restrict__ prow, int slot, int part = 0,
    int step = 1) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            pair_f64_narrow<TPL / 2, KAPPA0>(live, tgt, nv_pad, nodes, node_vid, blk_range, kappa, etab, base, n0, n1,
                                              prow, slot, part, step);
            return;
        }
    }
    pair_f64_wave<TPL, KAPPA0>(tgt, nv_pad, nodes, node_vid, blk_range, kappa, etab, base, n0, n1, prow, slot, part,
                               step);
}

// Worker w of a pair plan with one row per node group (per_row 1): slot w % slots against
// group w / slots, into partial row w.  etab: the workgroup's exponential table
// (fill_exp_table; not read when KAPPA0).  w must be wave-uniform and below slots * groups.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void pair_f64_worker(
    const double* __restrict__ tgt, int nv, int nv_pad, const NodeD* __restrict__ nodes,
    const int4* __restrict__ node_vid, const int2* __restrict__ blk_range, double kappa,
    const double* __restrict__ etab, const int* __restrict__ gstart, int slots, double* __restrict__ partial,
    int w) {
    constexpr int kSlot = kWave * TPL;
    const int g = w / slots, s = w - g * slots;
    const const_as<int>* cg = as_constant(gstart);
    const int base = s * kSlot;
    pair_f64_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, nodes, node_vid, blk_range, kappa, etab, base, cg[g],
                                 cg[g + 1], partial + (size_t)w * (2 * kSlot), kSlot);
}

constexpr int kCombineWays = kPairBlock / kCombineVerts;  // waves splitting the sum over node groups
constexpr int kCombineUnroll = 8;

// Rows (i, i + nv) of y = A u for the kCombineVerts vertices of tile vb: the partial rows of
// their slot s (rows r * slots + s for r < rows, each 2 * slot doubles; wave k of the block
// sums rows k, k + 4, ... into eight running sums by turn, and the sums of each wave and
// then of the four waves are added in a fixed order),
// the singular correction and the diagonal.  slot is a multiple of kCombineVerts.  Must be called by all
// kPairBlock threads of the block (it synchronises them).
__device__ __forceinline__ void combine_tile(int vb, const double* __restrict__ u, double* __restrict__ y, int nv,
                                             const double* __restrict__ partial, int slot, int slots,
                                             int rows, const int* __restrict__ inc_off, const int* __restrict__ inc_ent,
                                             const int* __restrict__ tri, const double* __restrict__ coef,
                                             double eps) {
    static_assert(kCombineWays == 4, "four partial sums per vertex");
    __shared__ double red[2][kCombineWays][kCombineVerts];
    const int lane = threadIdx.x % kCombineVerts, way = threadIdx.x / kCombineVerts;
    const int i = vb * kCombineVerts + lane;
    const int s = vb * kCombineVerts / slot;
    const int o = i - s * slot;
    double r1 = 0.0, r2 = 0.0;
    if (i < nv) {
        // kCombineUnroll rows in flight per wave, into separate sums added in a fixed order
        double p1[kCombineUnroll], p2[kCombineUnroll];
#pragma unroll
        for (int j = 0; j < kCombineUnroll; ++j) p1[j] = p2[j] = 0.0;
        const double* col = partial + o;
        const size_t row_step = (size_t)kCombineWays * slots * 2 * slot;
        const double* q = col + ((size_t)way * slots + s) * 2 * slot;
        int g = way;
        for (; g + (kCombineUnroll - 1) * kCombineWays < rows; g += kCombineUnroll * kCombineWays) {
#pragma unroll
            for (int j = 0; j < kCombineUnroll; ++j) {
                p1[j] += q[j * row_step];
                p2[j] += q[j * row_step + slot];
            }
            q += kCombineUnroll * row_step;
        }
        for (; g < rows; g += kCombineWays, q += row_step) {
            p1[0] += q[0];
            p2[0] += q[slot];
        }
        static_assert(kCombineUnroll == 8, "fixed-order sum of eight");
        r1 = ((p1[0] + p1[1]) + (p1[2] + p1[3])) + ((p1[4] + p1[5]) + (p1[6] + p1[7]));
        r2 = ((p2[0] + p2[1]) + (p2[2] + p2[3])) + ((p2[4] + p2[5]) + (p2[6] + p2[7]));
    }
    __syncthreads();                           // the previous tile's sums have been read
    red[0][way][lane] = r1;
    red[1][way][lane] = r2;
    __syncthreads();
    if (way != 0 || i >= nv) return;
    r1 = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
    r2 = (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
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

}  // namespace hobi
