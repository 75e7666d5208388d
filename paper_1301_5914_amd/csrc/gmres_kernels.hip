// FP64 building blocks of restarted GMRES on the device: multi-vector dot products with
// a fixed two-stage reduction (deterministic), multi-vector updates for classical
// Gram-Schmidt with one re-orthogonalisation pass, and the small Hessenberg work
// (Givens rotations, back substitution) in single-lane kernels.
#include "hobi_internal.h"
#include "krylov_tile.h"

namespace hobi {

namespace {

constexpr int kT = kKrylovBlock;
static_assert(kDotSlices == kDotBlocks, "one dot-product split");

// partial[j * kDotBlocks + b] = slice b of V[j] . w
__global__ __launch_bounds__(kT) void dots_kernel(const double* __restrict__ V, size_t ld,
                                                 const double* __restrict__ w, int n,
                                                 double* __restrict__ partial) {
    __shared__ double red[kT];
    const int j = blockIdx.y;
    const double d = dot_slice(V + ld * j, w, n, blockIdx.x, red);
    if (threadIdx.x == 0) partial[(size_t)j * kDotBlocks + blockIdx.x] = d;
}

__global__ __launch_bounds__(kDotBlocks) void reduce_kernel(const double* __restrict__ partial,
                                                           double* __restrict__ out, int sqrt_out) {
    __shared__ double red[kDotBlocks];
    const int j = blockIdx.x;
    const double d = sum_slices(partial + (size_t)j * kDotBlocks, red, sqrt_out != 0);
    if (threadIdx.x == 0) out[j] = d;
}

// w[i] += sign * sum_j coef[j] V[j][i]
__global__ void multi_axpy_kernel(const double* __restrict__ V, size_t ld, int nvec,
                                  const double* __restrict__ coef, double sign, double* __restrict__ w,
                                  int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    multi_axpy_elem(V, ld, nvec, coef, sign, w, i);
}

__global__ void diag_scale_kernel(const double* __restrict__ in, double* __restrict__ out, int n,
                                  const double* __restrict__ dinv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    diag_scale_elem(in, out, dinv, i);
}

// x[i] += dinv[i] * sum_j coef[j] V[j][i]
__global__ void multi_axpy_scaled_kernel(const double* __restrict__ V, size_t ld, int nvec,
                                         const double* __restrict__ coef, double* __restrict__ x, int n,
                                         const double* __restrict__ dinv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < nvec; ++j) acc = fma(coef[j], V[ld * j + i], acc);
    x[i] = fma(dinv[i], acc, x[i]);
}

// The inverse diagonal of the right preconditioner.  mode 1: the constants 1 / (1/2 (1 + eps))
// and 1 / (1/2 (1 + 1/eps)) of the two row blocks.  mode 2 (Jacobi): the inverse of A's own
// diagonal, those constants' inverses minus the vertex's singular terms on its own unknowns
// (entry b = 0 of each incident entry's coefficients: K2 on phi_i in row i, K3 on dphi_i in row
// nv + i), summed in the combine step's order; a non-positive or non-finite value (not met on
// the surfaces tried) falls back to the constant.  The lower-order method has no singular
// terms, so its mode 2 is mode 1.
__global__ void scaling_kernel(int nv, const int* __restrict__ inc_off, const int* __restrict__ inc_ent,
                               const double* __restrict__ coef, double eps, int jacobi, double* __restrict__ dinv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const double a0 = 0.5 * (1.0 + eps), b0 = 0.5 * (1.0 + 1.0 / eps);
    double a = a0, b = b0;
    if (jacobi) {
        for (int e = inc_off[i]; e < inc_off[i + 1]; ++e) {
            const double* co = coef + 12 * (size_t)inc_ent[e];
            a -= co[3];
            b -= co[6];
        }
        if (!(a > 0.0) || !isfinite(a)) a = a0;
        if (!(b > 0.0) || !isfinite(b)) b = b0;
    }
    dinv[i] = 1.0 / a;
    dinv[nv + i] = 1.0 / b;
}

__global__ void scale_copy_kernel(const double* __restrict__ in, const double* __restrict__ denom,
                                  double* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    scale_copy_elem(in, denom[0], out, i);
}

__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                           int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

__global__ void add_kernel(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                           int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

// Column k of the Hessenberg matrix and rotation k (givens_step), one thread.
__global__ void givens_kernel(double* __restrict__ H, int ldh, int k, const double* __restrict__ h1,
                              const double* __restrict__ h2, const double* __restrict__ hnext,
                              double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                              double bnorm, double* __restrict__ res) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    givens_step(H, ldh, k, h1, h2, hnext, cs, sn, g, bnorm, res);
}

__global__ void init_g_kernel(const double* __restrict__ beta, double* __restrict__ g, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= m) g[i] = (i == 0) ? beta[0] : 0.0;
}

// Solves the k x k upper-triangular system H y = g (column-major H).
__global__ void trisolve_kernel(const double* __restrict__ H, int ldh, int k, const double* __restrict__ g,
                                double* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double acc = g[i];
        for (int l = i + 1; l < k; ++l) acc -= H[(size_t)l * ldh + i] * y[l];
        const double d = H[(size_t)i * ldh + i];
        y[i] = d != 0.0 ? acc / d : 0.0;
    }
}

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_dots(const double* V, size_t ld, int nvec, const double* w, int n, double* partial,
                       hipStream_t s) {
    hipLaunchKernelGGL(dots_kernel, dim3(kDotBlocks, nvec), dim3(kT), 0, s, V, ld, w, n, partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nvec, double* out, int sqrt_out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(nvec), dim3(kDotBlocks), 0, s, partial, out, sqrt_out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* V, size_t ld, int nvec, const double* coef, double sign,
                             double* w, int n, hipStream_t s) {
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, V, ld, nvec, coef, sign, w, n);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const double* in, const double* denom, double* out, int n, hipStream_t s) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, in, denom, out, n);
    return hipGetLastError();
}

hipError_t launch_diag_scale(const double* in, double* out, int n, const double* dinv, hipStream_t s) {
    hipLaunchKernelGGL(diag_scale_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, in, out, n, dinv);
    return hipGetLastError();
}

hipError_t launch_multi_axpy_scaled(const double* V, size_t ld, int nvec, const double* coef, double* x, int n,
                                    const double* dinv, hipStream_t s) {
    hipLaunchKernelGGL(multi_axpy_scaled_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, V, ld, nvec, coef, x, n, dinv);
    return hipGetLastError();
}

hipError_t launch_scaling(const DeviceProblem& p, int mode, double* dinv, hipStream_t s) {
    const bool jacobi = mode == 2 && p.method == HOBI_HIGHER_ORDER;
    hipLaunchKernelGGL(scaling_kernel, dim3(nblk(p.nv, kT)), dim3(kT), 0, s, p.nv, p.inc_off, p.inc_ent, p.coef, p.eps,
                       jacobi ? 1 : 0, dinv);
    return hipGetLastError();
}

hipError_t launch_sub(const double* a, const double* b, double* out, int n, hipStream_t s) {
    hipLaunchKernelGGL(sub_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, a, b, out, n);
    return hipGetLastError();
}

hipError_t launch_add(const double* a, const double* b, double* out, int n, hipStream_t s) {
    hipLaunchKernelGGL(add_kernel, dim3(nblk(n, kT)), dim3(kT), 0, s, a, b, out, n);
    return hipGetLastError();
}

hipError_t launch_givens(double* H, int ldh, int k, const double* h1, const double* h2, const double* hnext,
                         double* cs, double* sn, double* g, double bnorm, double* res, hipStream_t s) {
    hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, s, H, ldh, k, h1, h2, hnext, cs, sn, g, bnorm, res);
    return hipGetLastError();
}

hipError_t launch_init_g(const double* beta, double* g, int m, hipStream_t s) {
    hipLaunchKernelGGL(init_g_kernel, dim3(nblk(m + 1, kT)), dim3(kT), 0, s, beta, g, m);
    return hipGetLastError();
}

hipError_t launch_trisolve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s) {
    hipLaunchKernelGGL(trisolve_kernel, dim3(1), dim3(64), 0, s, H, ldh, k, g, y);
    return hipGetLastError();
}

}  // namespace hobi
