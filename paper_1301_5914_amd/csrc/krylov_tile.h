// The arithmetic of one GMRES step's building blocks (every multiply-add written as an
// explicit fma, so that no kernel's contraction choices can differ), shared by the single-problem kernels
// (gmres_kernels.hip) and the request server's batched kernels (serve_kernels.hip), so that
// a served request's Krylov iterates are bit-for-bit those of hobi_solve: the same slices,
// the same fixed reduction trees, the same order of every sum.
#pragma once

#include "hobi_device.h"

namespace hobi {

constexpr int kKrylovBlock = 256;   // threads of a dot-product block
constexpr int kDotSlices = 64;      // blocks a dot product is split over (= kDotBlocks)

// Partial b of v . w: the sum over elements b * 256 + t, stepping 256 * 64, by the 256
// threads of the block, then a fixed LDS tree.  Returned to thread 0.  All threads of the
// block must call it (it synchronises them); red: kKrylovBlock doubles of LDS.
__device__ __forceinline__ double dot_slice(const double* __restrict__ v, const double* __restrict__ w, int n,
                                            int b, double* red) {
    double acc = 0.0;
    for (int i = b * kKrylovBlock + (int)threadIdx.x; i < n; i += kKrylovBlock * kDotSlices) acc = fma(v[i], w[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kKrylovBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();   // red may be reused at once
    return r;
}

// The sum of the kDotSlices partials of one dot product by the first kDotSlices threads of
// the block (a fixed LDS tree), optionally its square root.  Returned to thread 0.  All
// threads of the block must call it; red: kDotSlices doubles of LDS.
__device__ __forceinline__ double sum_slices(const double* __restrict__ partial, double* red, bool sqrt_out) {
    const int t = (int)threadIdx.x;
    if (t < kDotSlices) red[t] = partial[t];
    __syncthreads();
    for (int off = kDotSlices / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    const double r = sqrt_out ? sqrt(red[0]) : red[0];
    __syncthreads();
    return r;
}

// w[i] += sign * sum_j coef[j] V[j][i]
__device__ __forceinline__ void multi_axpy_elem(const double* __restrict__ V, size_t ld, int nvec,
                                                const double* __restrict__ coef, double sign, double* __restrict__ w,
                                                int i) {
    double acc = 0.0;
    for (int j = 0; j < nvec; ++j) acc = fma(coef[j], V[ld * j + i], acc);
    w[i] = fma(sign, acc, w[i]);
}

// out[i] = dinv[i] in[i] (the inverse diagonal of the right preconditioner)
__device__ __forceinline__ void diag_scale_elem(const double* __restrict__ in, double* __restrict__ out,
                                                const double* __restrict__ dinv, int i) {
    out[i] = dinv[i] * in[i];
}

__device__ __forceinline__ void scale_copy_elem(const double* __restrict__ in, double d, double* __restrict__ out,
                                                int i) {
    out[i] = d != 0.0 ? in[i] / d : 0.0;
}

// Column k of the Hessenberg matrix (column-major, leading dimension ldh = m + 1):
// H[0..k][k] = h1 + h2 (two Gram-Schmidt passes), H[k+1][k] = hnext.  Applies the k
// previous rotations, forms rotation k, updates g and writes |g[k+1]| / bnorm.  One thread.
__device__ __forceinline__ void givens_step(double* __restrict__ H, int ldh, int k, const double* __restrict__ h1,
                                            const double* __restrict__ h2, const double* __restrict__ hnext,
                                            double* __restrict__ cs, double* __restrict__ sn,
                                            double* __restrict__ g, double bnorm, double* __restrict__ res) {
    double* col = H + (size_t)k * ldh;
    for (int i = 0; i <= k; ++i) col[i] = h1[i] + h2[i];
    col[k + 1] = hnext[0];
    for (int i = 0; i < k; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = fma(cs[i], a, sn[i] * b);
        col[i + 1] = fma(-sn[i], a, cs[i] * b);
    }
    const double a = col[k], b = col[k + 1];
    const double den = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (den > 0.0) {
        c = a / den;
        s = b / den;
    }
    cs[k] = c;
    sn[k] = s;
    col[k] = den;
    col[k + 1] = 0.0;
    const double gk = g[k];
    g[k + 1] = -s * gk;
    g[k] = c * gk;
    res[0] = fabs(g[k + 1]) / bnorm;
}

}  // namespace hobi
