// Per-molecule setup (routines (2)-(4) and (1) of Section 2.6), all in FP64:
//   patch_kernel      -- flat triangle -> 10-node curved element (Section 2.2)
//   regular_kernel    -- 4-point Gauss-Radau nodes, normals and weight*Jacobian
//   targets_kernel    -- SoA target arrays (vertex positions and normals)
//   singular_kernel   -- 16-point Duffy/Gauss-Legendre coefficients of the triangles
//                        incident to each vertex (Section 2.3, eqdbef5/eqdbef6); the
//                        dense pair sum skips those triangles' regular nodes
//   sources_kernel    -- S1, S2 at every vertex (eq. Eq_Ss)
#include "hobi_internal.h"

namespace hobi {

namespace {

__device__ inline Vec3 load3(const double* a, int i) { return v3(a[3 * i], a[3 * i + 1], a[3 * i + 2]); }

__global__ void patch_kernel(const double* __restrict__ xyz, const double* __restrict__ nrm,
                             const int* __restrict__ tri, int nf, double* __restrict__ patch,
                             int* __restrict__ err) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nf) return;
    const int v0 = tri[3 * j], v1 = tri[3 * j + 1], v2 = tri[3 * j + 2];
    const Vec3 X1 = load3(xyz, v0), X2 = load3(xyz, v1), X3 = load3(xyz, v2);
    const Vec3 N1 = load3(nrm, v0), N2 = load3(nrm, v1), N3 = load3(nrm, v2);
    Vec3 node[10], n_unused;
    bool ok = true;
    node[0] = X1;
    node[1] = X2;
    node[2] = X3;
    // edge X1X2 at u = 1/3, 2/3 (v = 0); edge X1X3 at u = 1/3, 2/3 (v = 1)
    Vec3 y12, n12, y13, n13;
    ok &= arc_eval(X1, N1, X2, N2, 1.0 / 3.0, &node[3], &n_unused);
    ok &= arc_eval(X1, N1, X2, N2, 2.0 / 3.0, &y12, &n12);
    ok &= arc_eval(X1, N1, X3, N3, 1.0 / 3.0, &node[5], &n_unused);
    ok &= arc_eval(X1, N1, X3, N3, 2.0 / 3.0, &y13, &n13);
    node[4] = y12;
    node[6] = y13;
    // edge X2X3 (u = 1) at v = 1/3, 2/3
    ok &= arc_eval(X2, N2, X3, N3, 1.0 / 3.0, &node[7], &n_unused);
    ok &= arc_eval(X2, N2, X3, N3, 2.0 / 3.0, &node[8], &n_unused);
    // centroid (1/3, 1/3): u = 2/3, v = 1/2 on the arc between the two edge points
    ok &= arc_eval(y12, n12, y13, n13, 0.5, &node[9], &n_unused);
    double* out = patch + 30 * (size_t)j;
    for (int k = 0; k < 10; ++k) {
        out[3 * k] = node[k].x;
        out[3 * k + 1] = node[k].y;
        out[3 * k + 2] = node[k].z;
    }
    err[j] = ok ? 0 : 1;   // per-triangle flag, checked on the host
}

__global__ void regular_kernel(const double* __restrict__ patch, const int* __restrict__ tri, int nf,
                               NodeD* __restrict__ node64, NodeF* __restrict__ node32,
                               int4* __restrict__ node_vid, double* __restrict__ w, double cx,
                               double cy, double cz, double s32) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * nf) return;
    const int j = idx >> 2, m = idx & 3;
    double r, s, wm, J;
    gauss_radau4(m, &r, &s, &wm);
    Vec3 x, n;
    patch_eval(patch + 30 * (size_t)j, kRotPerm[0], r, s, &x, &J, &n);
    NodeD d{};
    d.x = x.x;
    d.y = x.y;
    d.z = x.z;
    d.nx = n.x;
    d.ny = n.y;
    d.nz = n.z;
    d.pad = -wm * J * kInv4Pi;                // solid-angle weight: -w / (4 pi)
    node64[idx] = d;
    NodeF f{};
    f.x = (float)((x.x - cx) * s32);
    f.y = (float)((x.y - cy) * s32);
    f.z = (float)((x.z - cz) * s32);
    f.nx = (float)n.x;
    f.ny = (float)n.y;
    f.nz = (float)n.z;
    f.pad = (float)(d.pad * s32 * s32);       // in the FP32 frame
    node32[idx] = f;
    node_vid[idx] = make_int4(tri[3 * j], tri[3 * j + 1], tri[3 * j + 2], 0);
    w[idx] = wm * J;
}

// Lower-order method (eqdbef1/eqdbef2): triangle j is one site and one node, at its
// centroid, with the flat triangle's unit normal and area; its node is masked for its own
// site only (ids j, j, j).
__global__ void lobi_nodes_kernel(const double* __restrict__ vxyz, const int* __restrict__ tri, int nf,
                                  NodeD* __restrict__ node64, NodeF* __restrict__ node32,
                                  int4* __restrict__ node_vid, double* __restrict__ w,
                                  double* __restrict__ sxyz, double* __restrict__ snrm, double cx, double cy,
                                  double cz, double s32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nf) return;
    const Vec3 A = load3(vxyz, tri[3 * j]), B = load3(vxyz, tri[3 * j + 1]), C = load3(vxyz, tri[3 * j + 2]);
    const Vec3 c = (1.0 / 3.0) * (A + B + C);
    const Vec3 cr = cross(B - A, C - A);
    const double a2 = norm(cr);
    const Vec3 n = (1.0 / a2) * cr;
    NodeD d{};
    d.x = c.x, d.y = c.y, d.z = c.z;
    d.nx = n.x, d.ny = n.y, d.nz = n.z;
    d.pad = -0.5 * a2 * kInv4Pi;              // solid-angle weight: -area / (4 pi)
    node64[j] = d;
    NodeF f{};
    f.x = (float)((c.x - cx) * s32);
    f.y = (float)((c.y - cy) * s32);
    f.z = (float)((c.z - cz) * s32);
    f.nx = (float)n.x, f.ny = (float)n.y, f.nz = (float)n.z;
    f.pad = (float)(d.pad * s32 * s32);
    node32[j] = f;
    node_vid[j] = make_int4(j, j, j, 0);
    w[j] = 0.5 * a2;
    sxyz[3 * j] = c.x, sxyz[3 * j + 1] = c.y, sxyz[3 * j + 2] = c.z;
    snrm[3 * j] = n.x, snrm[3 * j + 1] = n.y, snrm[3 * j + 2] = n.z;
}

__global__ void targets_kernel(const double* __restrict__ xyz, const double* __restrict__ nrm, int nv,
                               int nv_pad, double* __restrict__ t64, float* __restrict__ t32,
                               double cx, double cy, double cz, double s32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv_pad) return;
    const int src = i < nv ? i : nv - 1;   // padding lanes repeat the last vertex
    const double c[3] = {cx, cy, cz};
    for (int d = 0; d < 3; ++d) {
        const double x = xyz[3 * src + d], n = nrm[3 * src + d];
        t64[(size_t)d * nv_pad + i] = x;
        t64[(size_t)(3 + d) * nv_pad + i] = n;
        t32[(size_t)d * nv_pad + i] = (float)((x - c[d]) * s32);
        t32[(size_t)(3 + d) * nv_pad + i] = (float)n;
    }
}

// K1..K4 including their 1/(4 pi) (Section 2.1).
__device__ inline void kernels4(Vec3 x, Vec3 nx, Vec3 y, Vec3 ny, double kappa, double eps, double K[4]) {
    const Vec3 d = x - y;
    const double r2 = dot(d, d);
    const double r = sqrt(r2);
    const double rinv = 1.0 / r;
    const double rinv3 = rinv * rinv * rinv;
    const double dnx = dot(d, nx), dny = dot(d, ny), nxy = dot(nx, ny);
    double f0, f1, f2;
    f012_f64(kappa * r, &f0, &f1, &f2);
    K[0] = kInv4Pi * f0 * rinv;
    K[1] = kInv4Pi * dny * rinv3 * ((eps - 1.0) - eps * f1);
    K[2] = -kInv4Pi * dnx * rinv3 * ((1.0 - 1.0 / eps) + f1 / eps);
    K[3] = kInv4Pi * (-nxy * f1 + dnx * dny * f2 * rinv * rinv) * rinv3;
}

// One thread per (triangle j, local vertex k): target i = tri[j][k].
// coef[e][row*6 + kind*3 + b]: row 0 -> K1 (kind 0, dphi) / K2 (kind 1, phi),
// row 1 -> K3 / K4; b = slot of the relabelled triangle (vertex tri[j][(k+b)%3]).
__global__ void singular_kernel(const double* __restrict__ xyz, const double* __restrict__ nrm,
                                const int* __restrict__ tri, const double* __restrict__ patch,
                                int nf, double kappa, double eps, double* __restrict__ coef) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * nf) return;
    const int j = e / 3, k = e - 3 * (e / 3);
    const int i = tri[3 * j + k];
    const Vec3 x = load3(xyz, i), nx = load3(nrm, i);
    double c[12];
    for (int t = 0; t < 12; ++t) c[t] = 0.0;
    const double* pj = patch + 30 * (size_t)j;
    const int* perm = kRotPerm[k];
    for (int a = 0; a < 4; ++a) {
        double xi, gx;
        gauss_legendre4_01(a, &xi, &gx);
        for (int b = 0; b < 4; ++b) {
            double eta, gy;
            gauss_legendre4_01(b, &eta, &gy);
            const double r = (1.0 - eta) * xi, s = eta * xi;
            Vec3 y, ny;
            double J;
            patch_eval(pj, perm, r, s, &y, &J, &ny);
            double K[4];
            kernels4(x, nx, y, ny, kappa, eps, K);
            const double W = gx * gy * xi * J;
            const double L[3] = {1.0 - r - s, r, s};
            for (int q = 0; q < 3; ++q) {
                const double WL = W * L[q];
                c[0 + q] += WL * K[0];
                c[3 + q] += WL * K[1];
                c[6 + q] += WL * K[2];
                c[9 + q] += WL * K[3];
            }
        }
    }
    double* out = coef + 12 * (size_t)e;
    for (int t = 0; t < 12; ++t) out[t] = c[t];
}

__global__ void sources_kernel(const double* __restrict__ xyz, const double* __restrict__ nrm, int nv,
                               const double* __restrict__ qpos, const double* __restrict__ q, int nc,
                               double inv_eps1, double* __restrict__ rhs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const Vec3 x = load3(xyz, i), n = load3(nrm, i);
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nc; ++k) {
        const Vec3 d = x - load3(qpos, k);
        const double r = norm(d);
        const double qk = q[k];
        s1 += qk / r;
        s2 -= qk * dot(d, n) / (r * r * r);
    }
    rhs[i] = kInv4Pi * inv_eps1 * s1;
    rhs[nv + i] = kInv4Pi * inv_eps1 * s2;
}

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_patch(const DeviceProblem& p, int* d_err, hipStream_t s) {
    hipLaunchKernelGGL(patch_kernel, dim3(nblk(p.nf, 128)), dim3(128), 0, s, p.xyz, p.nrm, p.tri, p.nf,
                       p.patch, d_err);
    return hipGetLastError();
}

hipError_t launch_regular_nodes(const DeviceProblem& p, hipStream_t s) {
    hipLaunchKernelGGL(regular_kernel, dim3(nblk(4L * p.nf, 128)), dim3(128), 0, s, p.patch, p.tri, p.nf,
                       p.node64, p.node32, p.node_vid, p.w, p.center[0], p.center[1], p.center[2], p.s32);
    return hipGetLastError();
}

hipError_t launch_lobi_nodes(const DeviceProblem& p, hipStream_t s) {
    hipLaunchKernelGGL(lobi_nodes_kernel, dim3(nblk(p.nf, 128)), dim3(128), 0, s, p.vxyz, p.tri, p.nf, p.node64,
                       p.node32, p.node_vid, p.w, p.xyz, p.nrm, p.center[0], p.center[1], p.center[2], p.s32);
    return hipGetLastError();
}

hipError_t launch_targets(const DeviceProblem& p, hipStream_t s) {
    hipLaunchKernelGGL(targets_kernel, dim3(nblk(p.nv_pad, 256)), dim3(256), 0, s, p.xyz, p.nrm, p.nv,
                       p.nv_pad, p.tgt64, p.tgt32, p.center[0], p.center[1], p.center[2], p.s32);
    return hipGetLastError();
}

hipError_t launch_singular(const DeviceProblem& p, hipStream_t s) {
    hipLaunchKernelGGL(singular_kernel, dim3(nblk(3L * p.nf, 64)), dim3(64), 0, s, p.xyz, p.nrm, p.tri,
                       p.patch, p.nf, p.kappa, p.eps, p.coef);
    return hipGetLastError();
}

hipError_t launch_sources(const DeviceProblem& p, hipStream_t s) {
    hipLaunchKernelGGL(sources_kernel, dim3(nblk(p.nv, 256)), dim3(256), 0, s, p.xyz, p.nrm, p.nv, p.qpos,
                       p.q, p.nc, 1.0 / p.eps1, p.rhs);
    return hipGetLastError();
}

}  // namespace hobi
