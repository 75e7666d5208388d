// Treecode matvec (optional, hobi_params.tree_theta > 0): the dense regular sum of the
// pair kernels replaced by a cluster-particle treecode.  The partition (built on the host
// at problem creation): leaves = consecutive runs of tree_leaf nodes in Morton order,
// joined pairwise level by level into a binary cluster tree; batches = consecutive runs of
// tree_batch targets.  Each batch walks the tree: a cluster with (r_b + r_c) <= theta
// |c_b - c_c| and no triangle incident to a target of the batch is far, a leaf that fails
// is near, a parent that fails is opened.  Per matvec, after the gather:
//
//   proxy_kernel   -- per leaf, the (n+1)^3 Chebyshev points of its box (grown by 1e-6 of
//                     the diagonal) and three charges per point,
//                       Q0  = sum_j  Gamma_j L_k(y_j) - Phi_j grad L_k(y_j).n_j
//                       Qk  = sum_j -Gamma_j L_k(y_j) + eps Phi_j grad L_k(y_j).n_j
//                       Qk2 = sum_j -Gamma_j L_k(y_j) / eps + Phi_j grad L_k(y_j).n_j
//                       Qs  = sum_j pad_j grad L_k(y_j).n_j   (pad = -w/(4 pi): the unit
//                                                              double layer of hobi_field)
//                     (L_k the tensor Lagrange basis, product form): the Green's functions
//                     interpolated in the source point, so that a far cluster's two rows
//                     are sum_k G0 Q0 + Gk Qk and sum_k dG0/dnu_x Q0 + dGk/dnu_x Qk2 at s_k
//   upward_kernel  -- per parent of one level, its charges from its two children's:
//                     Q_k = sum over the children's points s_j of L_k(s_j) Q_j, the same
//                     value as the sums over its nodes (each L_k of the parent is a
//                     tensor polynomial of degree n, which a child's degree-n
//                     interpolation reproduces together with its gradient)
//   tree_*_kernel  -- one wave per work item (slot of targets, cluster): near items run
//                     the masked pair loop over the leaf's nodes, far items the proxies;
//                     each item writes one partial row
//   tree_combine   -- a slot's rows in item order, then the singular correction and the
//                     diagonal (as combine_tile).
#include "hobi_internal.h"
#include "pair_tile.h"

namespace hobi {

namespace {

constexpr int kBlock = kPairBlock;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kChunk = 32;          // nodes per LDS round of the proxy kernel

__device__ __forceinline__ int xcd_logical_block() {
    const int nb = gridDim.x, p = blockIdx.x;
    const int x = p & 7, q = nb >> 3, rm = nb & 7;
    return x * q + min(x, rm) + (p >> 3);
}

// l_a(t) and l_a'(t) of the points p[0..n1) (product form, the derivative by the running
// product rule); inv[b] = 1 / (p[a] - p[b]).
__device__ __forceinline__ double lagrange_1d(const double* p, const double* inv, int n1, int a, double t,
                                              double* dl) {
    double l = 1.0, d = 0.0;
    for (int b = 0; b < n1; ++b) {
        if (b == a) continue;
        const double f = (t - p[b]) * inv[b];
        d = d * f + l * inv[b];
        l *= f;
    }
    *dl = d;
    return l;
}

// inv[d][a][b] = 1 / (pt[d][a] - pt[d][b]) for a != b, by the first 3 (n + 1)^2 threads
template <int M>
__device__ __forceinline__ void inverse_differences(const double (&pt)[3][M], double (&inv)[3][M][M], int n1) {
    if ((int)threadIdx.x < 3 * n1 * n1) {
        const int d = threadIdx.x / (n1 * n1), a = (threadIdx.x / n1) % n1, b = threadIdx.x % n1;
        inv[d][a][b] = a == b ? 0.0 : 1.0 / (pt[d][a] - pt[d][b]);
    }
}

// n1 Chebyshev points of the second kind on [lo, hi]
__device__ __forceinline__ double cheb_point(double lo, double hi, int a, int n) {
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * cos(kPi * a / n);
}

// The FP64 proxy record and its FP32 copy (positions in the frame of the FP32 targets).
__device__ __forceinline__ void write_proxy(ProxyD* __restrict__ prox64, ProxyF* __restrict__ prox32, size_t at,
                                            double x, double y, double z, double q0, double qk, double qk2,
                                            double qs, int mixed, double s32, double cx, double cy, double cz) {
    ProxyD pd{};
    pd.x = x, pd.y = y, pd.z = z, pd.q0 = q0, pd.qk = qk, pd.qk2 = qk2, pd.qs = qs;
    prox64[at] = pd;
    if (mixed) {
        ProxyF pf{};
        pf.x = (float)((x - cx) * s32);
        pf.y = (float)((y - cy) * s32);
        pf.z = (float)((z - cz) * s32);
        pf.q0a = (float)(s32 * q0);
        pf.qka = (float)(s32 * qk);
        pf.q0b = (float)(s32 * s32 * q0);
        pf.qk2b = (float)(s32 * s32 * qk2);
        pf.qs = (float)(s32 * qs);
        prox32[at] = pf;
    }
}

// One block per leaf.  Each round puts l_a(y_d) and l_a'(y_d) of kChunk nodes (every
// dimension d and index a) into LDS; then thread k accumulates the charges of proxies k and
// k + kBlock over the round's nodes in node order.
__global__ __launch_bounds__(kBlock) void proxy_kernel(const NodeD* __restrict__ nodes,
                                                       const int2* __restrict__ clu_range,
                                                       const double* __restrict__ clu_box, int n, double eps,
                                                       ProxyD* __restrict__ prox64, ProxyF* __restrict__ prox32,
                                                       int mixed, double s32, double cx, double cy, double cz) {
    __shared__ double pt[3][kTreeMaxDeg + 1];
    __shared__ double inv[3][kTreeMaxDeg + 1][kTreeMaxDeg + 1];
    __shared__ double lv[kChunk][3][kTreeMaxDeg + 1];
    __shared__ double dv[kChunk][3][kTreeMaxDeg + 1];
    __shared__ double ng[kChunk], np_[kChunk], nw[kChunk], nn3[kChunk][3];
    const int c = blockIdx.x;
    const int n1 = n + 1, P = n1 * n1 * n1;
    const int2 rg = clu_range[c];
    const double* box = clu_box + 6 * (size_t)c;
    if (threadIdx.x < 3 * n1) {
        const int d = threadIdx.x / n1, a = threadIdx.x % n1;
        const double lo = box[d], hi = box[3 + d];
        pt[d][a] = cheb_point(lo, hi, a, n);
    }
    __syncthreads();
    inverse_differences(pt, inv, n1);
    __syncthreads();
    const double ieps = 1.0 / eps;
    double q0[2] = {0.0, 0.0}, qk[2] = {0.0, 0.0}, qk2[2] = {0.0, 0.0}, qs[2] = {0.0, 0.0};
    int ka[2], kb[2], kc[2];
    for (int h = 0; h < 2; ++h) {
        const int k = threadIdx.x + h * kBlock;
        ka[h] = k / (n1 * n1);
        kb[h] = (k / n1) % n1;
        kc[h] = k % n1;
    }
    for (int j0 = rg.x; j0 < rg.y; j0 += kChunk) {
        const int m = min(kChunk, rg.y - j0);
        for (int e = threadIdx.x; e < 3 * n1 * m; e += kBlock) {
            const int i = e / (3 * n1), d = (e / n1) % 3, a = e % n1;
            const NodeD& nd = nodes[j0 + i];
            const double t = d == 0 ? nd.x : (d == 1 ? nd.y : nd.z);
            double dl;
            lv[i][d][a] = lagrange_1d(pt[d], inv[d][a], n1, a, t, &dl);
            dv[i][d][a] = dl;
        }
        if ((int)threadIdx.x < m) {
            const NodeD& nd = nodes[j0 + threadIdx.x];
            ng[threadIdx.x] = nd.g;
            np_[threadIdx.x] = nd.p;
            nw[threadIdx.x] = nd.pad;          // -w / (4 pi): the solid-angle weight
            nn3[threadIdx.x][0] = nd.nx;
            nn3[threadIdx.x][1] = nd.ny;
            nn3[threadIdx.x][2] = nd.nz;
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {
            if ((int)threadIdx.x + h * kBlock >= P) continue;
            for (int i = 0; i < m; ++i) {
                const double la = lv[i][0][ka[h]], lb = lv[i][1][kb[h]], lc = lv[i][2][kc[h]];
                const double L = la * lb * lc;
                const double G = dv[i][0][ka[h]] * lb * lc * nn3[i][0] + la * dv[i][1][kb[h]] * lc * nn3[i][1] +
                                 la * lb * dv[i][2][kc[h]] * nn3[i][2];
                const double gL = ng[i] * L, pG = np_[i] * G;
                q0[h] += gL - pG;
                qk[h] += -gL + eps * pG;
                qk2[h] += fma(-gL, ieps, pG);
                qs[h] += nw[i] * G;
            }
        }
        __syncthreads();
    }
    for (int h = 0; h < 2; ++h) {
        const int k = threadIdx.x + h * kBlock;
        if (k >= P) continue;
        write_proxy(prox64, prox32, (size_t)c * P + k, pt[0][ka[h]], pt[1][kb[h]], pt[2][kc[h]], q0[h], qk[h], qk2[h],
                    qs[h], mixed, s32, cx, cy, cz);
    }
}

// One block per parent c = first + blockIdx.x of one level: its proxy points from its box,
// and its charges from its two children's (computed by earlier launches):
//   Q_a = sum_{child} sum_{b} l_a1(s_b1) l_a2(s_b2) l_a3(s_b3) Q_b(child),
// as three one-dimensional contractions per child (over b3, then b2, then b1: n + 1 terms
// per output each), children in order.
__global__ __launch_bounds__(kBlock) void upward_kernel(int first, const int2* __restrict__ clu_child,
                                                        const double* __restrict__ clu_box, int n,
                                                        ProxyD* __restrict__ prox64, ProxyF* __restrict__ prox32,
                                                        int mixed, double s32, double cx, double cy, double cz) {
    constexpr int M = kTreeMaxDeg + 1, MP = M * M * M;
    __shared__ double pt[3][M];
    __shared__ double inv[3][M][M];
    __shared__ double cp[2][3][M];          // children's 1D points
    __shared__ double lt[2][3][M][M];       // l_a(parent) at the children's points b
    constexpr int NQ = 4;                   // charges: q0, qk, qk2, qs
    __shared__ double qc[NQ][MP];           // one child's charges
    __shared__ double t1[NQ][MP], t2[NQ][MP]; // partial contractions
    const int c = first + blockIdx.x;
    const int n1 = n + 1, n2 = n1 * n1, P = n2 * n1;
    const int2 ch = clu_child[c];
    const double* box = clu_box + 6 * (size_t)c;
    if (threadIdx.x < 3 * n1) {
        const int d = threadIdx.x / n1, a = threadIdx.x % n1;
        pt[d][a] = cheb_point(box[d], box[3 + d], a, n);
    }
    if (threadIdx.x < 2 * 3 * n1) {
        const int h = threadIdx.x / (3 * n1), d = (threadIdx.x / n1) % 3, b = threadIdx.x % n1;
        const ProxyD* q = prox64 + (size_t)(h ? ch.y : ch.x) * P;
        cp[h][d][b] = d == 0 ? q[b * n2].x : (d == 1 ? q[b * n1].y : q[b].z);
    }
    __syncthreads();
    inverse_differences(pt, inv, n1);
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * 3 * n2; e += kBlock) {
        const int h = e / (3 * n2), d = (e / n2) % 3, a = (e / n1) % n1, b = e % n1;
        double dl;
        lt[h][d][a][b] = lagrange_1d(pt[d], inv[d][a], n1, a, cp[h][d][b], &dl);
    }
    __syncthreads();
    double acc[2][NQ] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    for (int g = 0; g < 2; ++g) {
        for (int k = threadIdx.x; k < P; k += kBlock) {
            const ProxyD& q = prox64[(size_t)(g ? ch.y : ch.x) * P + k];
            qc[0][k] = q.q0;
            qc[1][k] = q.qk;
            qc[2][k] = q.qk2;
            qc[3][k] = q.qs;
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {            // t1[b1 b2 a3] = sum_b3 l_a3(b3) Q[b1 b2 b3]
            const int k = threadIdx.x + h * kBlock;
            if (k >= P) continue;
            const int j0 = k - k % n1, a3 = k % n1;
            double sq[NQ] = {0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < n1; ++b) {
                const double w = lt[g][2][a3][b];
#pragma unroll
                for (int m = 0; m < NQ; ++m) sq[m] += w * qc[m][j0 + b];
            }
#pragma unroll
            for (int m = 0; m < NQ; ++m) t1[m][k] = sq[m];
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {            // t2[b1 a2 a3] = sum_b2 l_a2(b2) t1[b1 b2 a3]
            const int k = threadIdx.x + h * kBlock;
            if (k >= P) continue;
            const int b1 = k / n2, a2 = (k / n1) % n1, a3 = k % n1;
            double sq[NQ] = {0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < n1; ++b) {
                const double w = lt[g][1][a2][b];
                const int j = b1 * n2 + b * n1 + a3;
#pragma unroll
                for (int m = 0; m < NQ; ++m) sq[m] += w * t1[m][j];
            }
#pragma unroll
            for (int m = 0; m < NQ; ++m) t2[m][k] = sq[m];
        }
        __syncthreads();
        for (int h = 0; h < 2; ++h) {            // Q[a1 a2 a3] += sum_b1 l_a1(b1) t2[b1 a2 a3]
            const int k = threadIdx.x + h * kBlock;
            if (k >= P) continue;
            const int a1 = k / n2, r = k % n2;
            for (int b = 0; b < n1; ++b) {
                const double w = lt[g][0][a1][b];
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc[h][m] += w * t2[m][b * n2 + r];
            }
        }
        __syncthreads();                         // qc, t1, t2 are rewritten for the next child
    }
    for (int h = 0; h < 2; ++h) {
        const int k = threadIdx.x + h * kBlock;
        if (k >= P) continue;
        const int ka = k / n2, kb = (k / n1) % n1, kc = k % n1;
        write_proxy(prox64, prox32, (size_t)c * P + k, pt[0][ka], pt[1][kb], pt[2][kc], acc[h][0], acc[h][1],
                    acc[h][2], acc[h][3], mixed, s32, cx, cy, cz);
    }
}

// FP32 far item: the kWave * TPL targets from `base` (scaled frame) against the cluster's
// proxies; FP32 running sums folded into FP64 every kFold proxies.
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_f32_wave(const float* __restrict__ tgt, int nv_pad,
                                             const ProxyF* __restrict__ prox, int P, int base,
                                             double* __restrict__ prow, int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    float tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL];
    double d1[TPL], d2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        d1[k] = d2[k] = 0.0;
    }
    const const_as<ProxyF>* cp = as_constant(prox);
    for (int k0 = 0; k0 < P; k0 += kFold) {
        const int k1 = min(k0 + kFold, P);
        float a1[TPL], a2[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) a1[k] = a2[k] = 0.0f;
        ProxyF pr = load_proxy(cp, k0);
        for (int q = k0; q < k1; ++q) {
            // the next record's scalar load is in flight while this one is used
            const ProxyF next = load_proxy(cp, min(q + 1, k1 - 1));
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const float dx = tx[k] - pr.x, dy = ty[k] - pr.y, dz = tz[k] - pr.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float dnx = fmaf(dx, tnx[k], fmaf(dy, tny[k], dz * tnz[k]));
                const float rinv3 = rinv * rinv * rinv;
                if (KAPPA0) {
                    a1[k] = fmaf(rinv, pr.q0a + pr.qka, a1[k]);
                    a2[k] = fmaf(-rinv3 * dnx, pr.q0b + pr.qk2b, a2[k]);
                } else {
                    const float zp1 = fmaf(r2, rinv, 1.0f);              // 1 + kappa r
                    const float e = __builtin_amdgcn_exp2f(fmaf(zp1, -kLog2E, kLog2E));   // exp(-kappa r)
                    a1[k] = fmaf(rinv, fmaf(e, pr.qka, pr.q0a), a1[k]);
                    a2[k] = fmaf(-rinv3 * dnx, fmaf(e * zp1, pr.qk2b, pr.q0b), a2[k]);
                }
            }
            pr = next;
        }
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

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_f32_narrow(int live, const float* __restrict__ tgt, int nv_pad,
                                               const ProxyF* __restrict__ prox, int P, int base,
                                               double* __restrict__ prow, int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            far_f32_narrow<TPL / 2, KAPPA0>(live, tgt, nv_pad, prox, P, base, prow, slot);
            return;
        }
    }
    far_f32_wave<TPL, KAPPA0>(tgt, nv_pad, prox, P, base, prow, slot);
}

// FP64 far item (unscaled frame).
template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_f64_wave(const double* __restrict__ tgt, int nv_pad,
                                             const ProxyD* __restrict__ prox, int P, double kappa,
                                             const double* __restrict__ etab, int base, double* __restrict__ prow,
                                             int slot) {
    const int lane = (int)(threadIdx.x % kWave);
    double tx[TPL], ty[TPL], tz[TPL], tnx[TPL], tny[TPL], tnz[TPL], a1[TPL], a2[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = base + lane + k * kWave;
        tx[k] = tgt[t];
        ty[k] = tgt[(size_t)nv_pad + t];
        tz[k] = tgt[2 * (size_t)nv_pad + t];
        tnx[k] = tgt[3 * (size_t)nv_pad + t];
        tny[k] = tgt[4 * (size_t)nv_pad + t];
        tnz[k] = tgt[5 * (size_t)nv_pad + t];
        a1[k] = a2[k] = 0.0;
    }
    const const_as<ProxyD>* cp = as_constant(prox);
    for (int q = 0; q < P; ++q) {
        const ProxyD pr = load_proxy(cp, q);
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
            const double dx = tx[k] - pr.x, dy = ty[k] - pr.y, dz = tz[k] - pr.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double rinv = rsqrt_f64(r2);
            const double dnx = fma(dx, tnx[k], fma(dy, tny[k], dz * tnz[k]));
            const double rinv3 = rinv * rinv * rinv;
            if (KAPPA0) {
                a1[k] = fma(rinv, pr.q0 + pr.qk, a1[k]);
                a2[k] = fma(-rinv3 * dnx, pr.q0 + pr.qk2, a2[k]);
            } else {
                const double z = kappa * (r2 * rinv);
                const double e = exp_neg_tab_f64(z, etab);
                a1[k] = fma(rinv, fma(e, pr.qk, pr.q0), a1[k]);
                a2[k] = fma(-rinv3 * dnx, fma(e * (1.0 + z), pr.qk2, pr.q0), a2[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        prow[lane + k * kWave] = a1[k];
        prow[slot + lane + k * kWave] = a2[k];
    }
}

template <int TPL, bool KAPPA0>
__device__ __forceinline__ void far_f64_narrow(int live, const double* __restrict__ tgt, int nv_pad,
                                               const ProxyD* __restrict__ prox, int P, double kappa,
                                               const double* __restrict__ etab, int base, double* __restrict__ prow,
                                               int slot) {
    if constexpr (TPL > 1) {
        if (live <= kWave * TPL / 2) {
            far_f64_narrow<TPL / 2, KAPPA0>(live, tgt, nv_pad, prox, P, kappa, etab, base, prow, slot);
            return;
        }
    }
    far_f64_wave<TPL, KAPPA0>(tgt, nv_pad, prox, P, kappa, etab, base, prow, slot);
}

// One wave per work item {slot, kind, cluster, -}: the item's partial row is its index.
template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void tree_f32_kernel(
    const int4* __restrict__ items, int nitems, const float* __restrict__ tgt, int nv, int nv_pad,
    const NodeF* __restrict__ nodes, const int4* __restrict__ node_vid, const int2* __restrict__ blk_range,
    const int2* __restrict__ clu_range, const ProxyF* __restrict__ prox, int P, double* __restrict__ partial) {
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= nitems) return;
    constexpr int kSlot = kWave * TPL;
    const int4 it = make_int4(as_constant(items)[w].x, as_constant(items)[w].y, as_constant(items)[w].z, 0);
    const int base = it.x * kSlot;
    double* prow = partial + (size_t)w * (2 * kSlot);
    if (it.y == 0) {
        const int n0 = as_constant(clu_range)[it.z].x, n1 = as_constant(clu_range)[it.z].y;
        pair_f32_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, nodes, node_vid, blk_range, base, n0, n1, prow, kSlot);
    } else {
        far_f32_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, prox + (size_t)it.z * P, P, base, prow, kSlot);
    }
}

template <int TPL, bool KAPPA0>
__global__ __launch_bounds__(kBlock) void tree_f64_kernel(
    const int4* __restrict__ items, int nitems, const double* __restrict__ tgt, int nv, int nv_pad,
    const NodeD* __restrict__ nodes, const int4* __restrict__ node_vid, const int2* __restrict__ blk_range,
    const int2* __restrict__ clu_range, const ProxyD* __restrict__ prox, int P, double kappa,
    double* __restrict__ partial) {
    __shared__ double etab[kExpTab];
    if constexpr (!KAPPA0) fill_exp_table(etab);
    const int w = xcd_logical_block() * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (w >= nitems) return;
    constexpr int kSlot = kWave * TPL;
    const int4 it = make_int4(as_constant(items)[w].x, as_constant(items)[w].y, as_constant(items)[w].z, 0);
    const int base = it.x * kSlot;
    double* prow = partial + (size_t)w * (2 * kSlot);
    if (it.y == 0) {
        const int n0 = as_constant(clu_range)[it.z].x, n1 = as_constant(clu_range)[it.z].y;
        pair_f64_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, nodes, node_vid, blk_range, kappa, etab, base, n0, n1,
                                     prow, kSlot);
    } else {
        far_f64_narrow<TPL, KAPPA0>(nv - base, tgt, nv_pad, prox + (size_t)it.z * P, P, kappa, etab, base, prow,
                                    kSlot);
    }
}

// Rows (i, i + nv) for the kCombineVerts targets of tile vb: the rows of their slot s
// (items slot_row[s] .. slot_row[s + 1] - 1; wave k sums rows k, k + 4, ..., the four sums
// added in a fixed order), then the singular correction and the diagonal.
__global__ __launch_bounds__(kBlock) void tree_combine_kernel(
    const double* __restrict__ u, double* __restrict__ y, int nv, const double* __restrict__ partial, int slot,
    const int* __restrict__ slot_row, const int* __restrict__ inc_off, const int* __restrict__ inc_ent, const int* __restrict__ tri,
    const double* __restrict__ coef, double eps) {
    __shared__ double red[2][4][kCombineVerts];
    const int vb = blockIdx.x;
    const int lane = threadIdx.x % kCombineVerts, way = threadIdx.x / kCombineVerts;
    const int i = vb * kCombineVerts + lane;
    const int s = vb * kCombineVerts / slot, o = i - s * slot;
    const int rb = slot_row[s], re = slot_row[s + 1];
    double r1 = 0.0, r2 = 0.0;
    if (i < nv) {
        // rows rb + way, rb + way + 4, ... summed in that order; the loads of kAhead rows are
        // issued before their sums, so that they are in flight together
        constexpr int kAhead = 8;
        int r = rb + way;
        for (; r + 4 * (kAhead - 1) < re; r += 4 * kAhead) {
            double a[kAhead], b[kAhead];
#pragma unroll
            for (int q = 0; q < kAhead; ++q) {
                a[q] = partial[(size_t)(2 * (r + 4 * q)) * slot + o];
                b[q] = partial[(size_t)(2 * (r + 4 * q) + 1) * slot + o];
            }
#pragma unroll
            for (int q = 0; q < kAhead; ++q) {
                r1 += a[q];
                r2 += b[q];
            }
        }
        for (; r < re; r += 4) {
            r1 += partial[(size_t)(2 * r) * slot + o];
            r2 += partial[(size_t)(2 * r + 1) * slot + o];
        }
    }
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

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_tree_proxies(const DeviceProblem& p, bool mixed, hipStream_t s) {
    const TreePlan& t = p.tree;
    hipLaunchKernelGGL(proxy_kernel, dim3(t.nleaf), dim3(kBlock), 0, s, p.node64, t.clu_range, t.clu_box, t.degree,
                       p.eps, t.prox64, t.prox32, mixed ? 1 : 0, p.s32, p.center[0], p.center[1], p.center[2]);
    for (int l = 0; l < t.nlev; ++l) {
        const int first = t.lev_off[l], count = t.lev_off[l + 1] - t.lev_off[l];
        hipLaunchKernelGGL(upward_kernel, dim3(count), dim3(kBlock), 0, s, first, t.clu_child, t.clu_box, t.degree,
                           t.prox64, t.prox32, mixed ? 1 : 0, p.s32, p.center[0], p.center[1], p.center[2]);
    }
    return hipGetLastError();
}

hipError_t launch_tree_pairs(const DeviceProblem& p, bool mixed, hipStream_t s) {
    const TreePlan& t = p.tree;
    const bool k0 = p.kappa == 0.0;
    const int m = mixed ? 1 : 0;
    const dim3 grid(nblk(t.nitems[m], kWavesPerBlock));
    if (mixed) {
#define HOBI_TREE32(T, K0)                                                                                       \
    hipLaunchKernelGGL((tree_f32_kernel<T, K0>), grid, dim3(kBlock), 0, s, t.items[1], t.nitems[1], p.tgt32, p.nv, \
                       p.nv_pad, p.node32, p.node_vid, p.blk_range, t.clu_range, t.prox32, t.nprox, t.partial)
        if (t.tpl[1] == 8) {
            if (k0) HOBI_TREE32(8, true); else HOBI_TREE32(8, false);
        } else if (t.tpl[1] == 4) {
            if (k0) HOBI_TREE32(4, true); else HOBI_TREE32(4, false);
        } else {
            if (k0) HOBI_TREE32(2, true); else HOBI_TREE32(2, false);
        }
#undef HOBI_TREE32
    } else {
        if (k0)
            hipLaunchKernelGGL((tree_f64_kernel<kTreeTpl64, true>), grid, dim3(kBlock), 0, s, t.items[0], t.nitems[0],
                               p.tgt64, p.nv, p.nv_pad, p.node64, p.node_vid, p.blk_range, t.clu_range, t.prox64,
                               t.nprox, p.kappa, t.partial);
        else
            hipLaunchKernelGGL((tree_f64_kernel<kTreeTpl64, false>), grid, dim3(kBlock), 0, s, t.items[0], t.nitems[0],
                               p.tgt64, p.nv, p.nv_pad, p.node64, p.node_vid, p.blk_range, t.clu_range, t.prox64,
                               t.nprox, p.kappa, t.partial);
    }
    return hipGetLastError();
}

hipError_t launch_tree_combine(const DeviceProblem& p, const double* u, double* y, bool mixed, hipStream_t s) {
    const TreePlan& t = p.tree;
    const int m = mixed ? 1 : 0;
    hipLaunchKernelGGL(tree_combine_kernel, dim3(nblk(p.nv, kCombineVerts)), dim3(kBlock), 0, s, u, y, p.nv,
                       t.partial, t.slot[m], t.slot_row[m], p.inc_off, p.inc_ent, p.tri, p.coef, p.eps);
    return hipGetLastError();
}

}  // namespace hobi
