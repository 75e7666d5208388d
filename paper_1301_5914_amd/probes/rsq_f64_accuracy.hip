// Accuracy of the FP64 hardware reciprocal square root (v_rsq_f64) on gfx950: relative error
// of __builtin_amdgcn_rsq against a long-double reference on 2^20 values spread
// log-uniformly over [1e-4, 1e6] (the squared distances, in A^2, of the pair sums).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

__global__ void rsq_kernel(const double* __restrict__ x, double* __restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = __builtin_amdgcn_rsq(x[i]);
}

int main() {
    const int n = 1 << 20;
    std::vector<double> x(n), y(n);
    unsigned long long s = 88172645463325252ull;
    for (int i = 0; i < n; ++i) {
        s ^= s << 13, s ^= s >> 7, s ^= s << 17;   // xorshift64
        const double u = (double)(s >> 11) * 0x1.0p-53;
        x[i] = std::pow(10.0, -4.0 + 10.0 * u);
    }
    double *dx, *dy;
    if (hipMalloc(&dx, n * sizeof(double)) != hipSuccess || hipMalloc(&dy, n * sizeof(double)) != hipSuccess) return 1;
    if (hipMemcpy(dx, x.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 1;
    hipLaunchKernelGGL(rsq_kernel, dim3(n / 256), dim3(256), 0, 0, dx, dy, n);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 1;
    if (hipMemcpy(y.data(), dy, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
    long double worst = 0, sum = 0;
    double worst_ulp = 0;
    for (int i = 0; i < n; ++i) {
        const long double ref = 1.0L / sqrtl((long double)x[i]);
        const long double rel = fabsl((long double)y[i] - ref) / ref;
        sum += rel;
        if (rel > worst) worst = rel;
        const double ulp = std::fabs(y[i] - (double)ref) / (std::nextafter((double)ref, INFINITY) - (double)ref);
        if (ulp > worst_ulp) worst_ulp = ulp;
    }
    std::printf("v_rsq_f64 on %d values in [1e-4, 1e6]: max relative error %.3Le (%.1f ulp), mean %.3Le\n", n,
                worst, worst_ulp, sum / n);
    (void)hipFree(dx);
    (void)hipFree(dy);
    return 0;
}
