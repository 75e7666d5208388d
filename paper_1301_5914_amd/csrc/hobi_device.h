// Device-side building blocks shared by the HIP kernels: node layouts, the curved
// element (Section 2.2), quadrature constants (Sections 2.2-2.3) and the kernels
// K1..K4 of the well-posed formulation (Section 2.1, eq. Eq_Ls).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hobi {

// Source node as the pair kernels read it: position, node normal, Gamma (interpolated
// dphi times quadrature weight, Jacobian and 1/(4 pi)) and Phi (same with phi).  The
// FP32 record also carries the strengths pre-scaled by the dielectric constants,
//   ga = -(1 - 1/eps) Gamma, gb = -Gamma / eps, pa = (eps - 1) Phi, pb = -eps Phi,
// so that K2 Phi = (d.ny)/r^3 (pa + pb f1) and K3 Gamma = (d.nx)/r^3 (ga + gb f1),
// and the three vertex ids of the node's triangle (its pairs with those vertices belong
// to the singular rule and are skipped by the dense sum).
// `pad` holds the node's solid-angle weight -w J / (4 pi) (times s32^2 in the FP32 frame),
// written by the setup: the double layer of a unit density at a point, which tells the
// field evaluation on which side of the surface the point lies.
// One node is one 64-byte record, i.e. one wave-uniform scalar load.
struct alignas(64) NodeF {
    float x, y, z, nx, ny, nz, g, p;
    float ga, gb, pa, pb;
    float qx, qy, qz, pad;   // p * (nx, ny, nz), solid-angle weight
};
struct alignas(128) NodeD {
    double x, y, z, g;
    double nx, ny, nz, p;
    double ga, gb, pa, pb;   // Gamma, Phi times the epsilon factors of K3, K2
    double qx, qy, qz, pad;  // Phi * (nx, ny, nz), solid-angle weight
};

constexpr int kCombineVerts = 64;   // vertices per tile of the combine step
constexpr int kPairWaves = 4;       // waves of a pair-kernel workgroup (an FP32 block: one slot, four node groups)

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);
// Largest kappa r the FP64 pair kernels' exponential takes (its table index stays an int);
// a problem's kappa times twice its bounding-box diagonal must stay below it.
constexpr double kExpTabMaxZ = 5.0e6;

struct Vec3 {
    double x, y, z;
};
__device__ __forceinline__ Vec3 v3(double x, double y, double z) { return Vec3{x, y, z}; }
__device__ __forceinline__ Vec3 operator+(Vec3 a, Vec3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ Vec3 operator-(Vec3 a, Vec3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ Vec3 operator*(double s, Vec3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Vec3 cross(Vec3 a, Vec3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double norm(Vec3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ Vec3 unit(Vec3 a) { return (1.0 / norm(a)) * a; }

// ---------------------------------------------------------------------------------
// Curved edges (Section 2.2).  Cubic arc through P and Q whose end tangents lie in the
// tangent planes of nP and nQ along the projected chord, both of length
// m = 2|d| / (1 + cos(theta/2)); normal along the arc = blend of the end normals made
// orthogonal to the arc tangent.  Returns false when a normal is along the chord.
// ---------------------------------------------------------------------------------
__device__ inline bool arc_eval(Vec3 P, Vec3 nP, Vec3 Q, Vec3 nQ, double t, Vec3* x, Vec3* n) {
    if (t == 0.0) { *x = P; *n = nP; return true; }
    if (t == 1.0) { *x = Q; *n = nQ; return true; }
    Vec3 d = Q - P;
    double ell = norm(d);
    double c = fmin(fmax(dot(nP, nQ), -1.0), 1.0);
    double m = 2.0 * ell / (1.0 + sqrt(0.5 * (1.0 + c)));
    Vec3 tP = d - dot(d, nP) * nP;
    Vec3 tQ = d - dot(d, nQ) * nQ;
    double lp = norm(tP), lq = norm(tQ);
    if (!(ell > 0.0) || lp < 1e-12 * ell || lq < 1e-12 * ell) return false;
    Vec3 TP = (m / lp) * tP;
    Vec3 TQ = (m / lq) * tQ;
    Vec3 c2 = 3.0 * d - 2.0 * TP - TQ;
    Vec3 c3 = TP + TQ - 2.0 * d;
    *x = P + t * (TP + t * (c2 + t * c3));
    Vec3 dx = TP + t * (2.0 * c2 + (3.0 * t) * c3);
    Vec3 tau = unit(dx);
    Vec3 nb = (1.0 - t) * nP + t * nQ;
    *n = unit(nb - dot(nb, tau) * tau);
    return true;
}

// Ten element nodes in the barycentric multi-index order
//   (3,0,0) (0,3,0) (0,0,3) (2,1,0) (1,2,0) (2,0,1) (1,0,2) (0,2,1) (0,1,2) (1,1,1)
// for L = (1-r-s, r, s).  rot_perm[k][i] = stored index of node i after relabelling the
// element so that stored vertex k becomes local vertex 1.
__constant__ const int kRotPerm[3][10] = {
    {0, 1, 2, 3, 4, 5, 6, 7, 8, 9},
    {1, 2, 0, 7, 8, 4, 3, 6, 5, 9},
    {2, 0, 1, 6, 5, 8, 7, 3, 4, 9},
};

// Cubic Lagrange basis: values and derivatives in r and s at (r, s).
__device__ inline void p3_basis(double r, double s, double N[10], double Nr[10], double Ns[10]) {
    const double L1 = 1.0 - r - s, L2 = r, L3 = s;
    // gradient w.r.t. (L1, L2, L3) of each basis function
    double g[10][3];
    auto vert = [](double L, double* val, double* dval) {
        *val = 0.5 * L * (3.0 * L - 1.0) * (3.0 * L - 2.0);
        *dval = 0.5 * (27.0 * L * L - 18.0 * L + 2.0);
    };
    double dv;
    vert(L1, &N[0], &dv); g[0][0] = dv; g[0][1] = 0.0; g[0][2] = 0.0;
    vert(L2, &N[1], &dv); g[1][0] = 0.0; g[1][1] = dv; g[1][2] = 0.0;
    vert(L3, &N[2], &dv); g[2][0] = 0.0; g[2][1] = 0.0; g[2][2] = dv;
    // edge nodes E(a, b) = 9/2 La Lb (3 La - 1)
    auto edge = [&](int k, int a, int b, const double* L) {
        N[k] = 4.5 * L[a] * L[b] * (3.0 * L[a] - 1.0);
        g[k][0] = g[k][1] = g[k][2] = 0.0;
        g[k][a] = 4.5 * L[b] * (6.0 * L[a] - 1.0);
        g[k][b] = 4.5 * L[a] * (3.0 * L[a] - 1.0);
    };
    const double L[3] = {L1, L2, L3};
    edge(3, 0, 1, L);
    edge(4, 1, 0, L);
    edge(5, 0, 2, L);
    edge(6, 2, 0, L);
    edge(7, 1, 2, L);
    edge(8, 2, 1, L);
    N[9] = 27.0 * L1 * L2 * L3;
    g[9][0] = 27.0 * L2 * L3; g[9][1] = 27.0 * L1 * L3; g[9][2] = 27.0 * L1 * L2;
    for (int k = 0; k < 10; ++k) {
        Nr[k] = g[k][1] - g[k][0];
        Ns[k] = g[k][2] - g[k][0];
    }
}

// Position, Jacobian |x_r x x_s| and unit normal of a patch (nodes [10][3], possibly
// relabelled through perm) at (r, s) (Section 2.2, quadrature on curved elements).
__device__ inline void patch_eval(const double* nodes, const int* perm, double r, double s,
                                  Vec3* x, double* J, Vec3* n) {
    double N[10], Nr[10], Ns[10];
    p3_basis(r, s, N, Nr, Ns);
    Vec3 p = v3(0, 0, 0), pr = v3(0, 0, 0), ps = v3(0, 0, 0);
    for (int k = 0; k < 10; ++k) {
        const double* q = nodes + 3 * perm[k];
        Vec3 v = v3(q[0], q[1], q[2]);
        p = p + N[k] * v;
        pr = pr + Nr[k] * v;
        ps = ps + Ns[k] * v;
    }
    Vec3 c = cross(pr, ps);
    *J = norm(c);
    *n = (1.0 / *J) * c;
    *x = p;
}

// ---------------------------------------------------------------------------------
// Quadrature rules on the unit right triangle.
// Regular (4-point Gauss-Radau, collapsed product anchored at local vertex 1):
//   u in {(6 -+ sqrt6)/10} with weights (9 -+ sqrt6)/36, v in {(3 -+ sqrt3)/6} with
//   weights 1/2; (r, s) = (u (1 - v), u v); node order (u0,v0) (u0,v1) (u1,v0) (u1,v1).
// Singular (Section 2.3): 4x4 Gauss-Legendre on [0,1]^2 mapped by r = (1 - y) x,
//   s = y x, weight gx gy x.
// ---------------------------------------------------------------------------------
__device__ inline void gauss_radau4(int m, double* r, double* s, double* w) {
    const double s6 = sqrt(6.0), s3 = sqrt(3.0);
    const double u = (m < 2) ? (6.0 - s6) / 10.0 : (6.0 + s6) / 10.0;
    const double wu = (m < 2) ? (9.0 - s6) / 36.0 : (9.0 + s6) / 36.0;
    const double v = (m & 1) ? (3.0 + s3) / 6.0 : (3.0 - s3) / 6.0;
    *r = u * (1.0 - v);
    *s = u * v;
    *w = 0.5 * wu;
}

__device__ inline void gauss_legendre4_01(int a, double* x, double* w) {
    const double t1 = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));   // inner
    const double t2 = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));   // outer
    const double wi = (18.0 + sqrt(30.0)) / 72.0, wo = (18.0 - sqrt(30.0)) / 72.0;
    switch (a) {
        case 0: *x = 0.5 * (1.0 - t2); *w = wo; break;
        case 1: *x = 0.5 * (1.0 - t1); *w = wi; break;
        case 2: *x = 0.5 * (1.0 + t1); *w = wi; break;
        default: *x = 0.5 * (1.0 + t2); *w = wo; break;
    }
}

// ---------------------------------------------------------------------------------
// Kernels K1..K4 without the 1/(4 pi) factor (it is folded into the source strengths).
// With d = x - y, z = kappa r, f0 = 1 - e^-z, f1 = 1 - e^-z (1+z),
// f2 = 3 - e^-z (3 + 3z + z^2):
//   K1 = f0 / r, K2 = (d.ny)/r^3 ((eps-1) - eps f1), K3 = -(d.nx)/r^3 ((1-1/eps) + f1/eps),
//   K4 = (-(nx.ny) f1 + (d.nx)(d.ny) f2 / r^2) / r^3.
// For small z the f's come from their Taylor series (no cancellation).
// ---------------------------------------------------------------------------------
// Taylor coefficients of z^k (k = 0..12), built at compile time:
//   f0 = sum_{k>=1} (-1)^(k+1) z^k / k!, f1 = sum_{k>=2} (-1)^k (k-1) z^k / k!,
//   f2 = sum_{k>=2} (-1)^(k+1) (k-1)(k-3) z^k / k!.
struct SeriesTable {
    double f0[13], f1[13], f2[13];
};
constexpr SeriesTable series_table() {
    SeriesTable t{};
    double fact = 1.0;
    for (int k = 1; k <= 12; ++k) {
        fact *= k;
        const double sg = (k & 1) ? 1.0 : -1.0;   // (-1)^(k+1)
        t.f0[k] = sg / fact;
        t.f1[k] = k >= 2 ? -sg * (k - 1) / fact : 0.0;
        t.f2[k] = k >= 2 ? sg * (k - 1) * (k - 3) / fact : 0.0;
    }
    return t;
}

// Treecode proxy records: a point of a cluster's proxy grid with its charges (the sums over
// the cluster's nodes of the strengths times the tensor basis and its normal derivative).
struct ProxyD {                      // proxy point and its charges (64 B); qs: solid angle
    double x, y, z, q0, qk, qk2, qs, pad;
};
struct ProxyF {                      // FP32 copy in the frame of the FP32 node records (32 B):
    float x, y, z;                   // positions shifted and scaled like the targets
    float q0a, qka;                  // s32 Q0, s32 Qk           (row 1)
    float q0b, qk2b;                 // s32^2 Q0, s32^2 Qk2      (row 2)
    float qs;                        // s32 Qs                   (solid angle)
};
constexpr double kSeriesZ64 = 0.1;

__device__ __forceinline__ void f012_f64(double z, double* f0, double* f1, double* f2) {
    if (z < kSeriesZ64) {
        // Horner in z, terms k = 1..12 (f0) and k = 2..12 (f1, f2); truncation < 1e-17 rel.
        constexpr SeriesTable T = series_table();
        double a0 = T.f0[12], a1 = T.f1[12], a2 = T.f2[12];
#pragma unroll
        for (int k = 11; k >= 2; --k) {
            a0 = a0 * z + T.f0[k];
            a1 = a1 * z + T.f1[k];
            a2 = a2 * z + T.f2[k];
        }
        a0 = a0 * z + T.f0[1];
        *f0 = a0 * z;
        *f1 = a1 * z * z;
        *f2 = a2 * z * z;
    } else {
        const double e = exp(-z);
        *f0 = 1.0 - e;
        *f1 = 1.0 - e * (1.0 + z);
        *f2 = 3.0 - e * (3.0 + z * (3.0 + z));
    }
}

// exp(-z) for z >= 0 in FP64, without the special-case handling of the library routine
// (the argument is finite and non-negative; it is clamped where exp(-z) would underflow).
// Cody-Waite reduction z = n ln2 - t with |t| <= ln2 / 2 (ln2 split into a 21-bit head, so
// n * head is exact, and a tail), then the Taylor polynomial of exp(t) to degree 12
// (truncation below 2e-16 relative) and a scaling by 2^-n.
__device__ __forceinline__ double exp_neg_f64(double z) {
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2Hi = 0x1.62e42p-1;
    constexpr double kLn2Lo = 0x1.fdf473de6af28p-22;
    z = fmin(z, 708.0);
    const double n = __builtin_rint(z * kLog2e);
    double t = fma(n, kLn2Hi, -z);
    t = fma(n, kLn2Lo, t);
    // Horner's scheme (fewest operations; callers have independent work to hide its latency)
    double p = 1.0 / 479001600.0;
    p = fma(p, t, 1.0 / 39916800.0);
    p = fma(p, t, 1.0 / 3628800.0);
    p = fma(p, t, 1.0 / 362880.0);
    p = fma(p, t, 1.0 / 40320.0);
    p = fma(p, t, 1.0 / 5040.0);
    p = fma(p, t, 1.0 / 720.0);
    p = fma(p, t, 1.0 / 120.0);
    p = fma(p, t, 1.0 / 24.0);
    p = fma(p, t, 1.0 / 6.0);
    p = fma(p, t, 0.5);
    p = fma(p, t, 1.0);
    p = fma(p, t, 1.0);
    return __builtin_amdgcn_ldexp(p, -(int)n);
}

// 1 / sqrt(x) for finite x > 0 in FP64: hardware estimate, then one third-order
// correction y (1 + h/2 + 3 h^2 / 8) with h = 1 - x y^2.
__device__ __forceinline__ double rsqrt_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = fma(-x * y, y, 1.0);
    return fma(y * h, fma(h, 0.375, 0.5), y);
}

}  // namespace hobi
