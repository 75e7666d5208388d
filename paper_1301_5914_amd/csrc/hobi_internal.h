// Internal declarations of the HOBI-PB library: device buffers of a problem and the
// host-side launch wrappers of every kernel.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hobi.h"
#include "hobi_device.h"

namespace hobi {

// Launch configuration of the dense pair sum, fixed per problem size only (so that the
// reduction order -- and hence every bit of the result -- depends only on the problem).
struct PairPlan {
    int tpl;            // targets per lane
    int block;          // threads per block
    int target_blocks;  // blocks along the targets
    int chunks;         // source chunks (split of the node range)
    int chunk;          // nodes per chunk
};

struct DeviceProblem {
    // nv counts the collocation sites, which carry the unknowns: the vertices (higher-order
    // method) or the triangles' centroids (lower-order method, then nv = nf and nn = nf)
    int nv = 0, nf = 0, nc = 0, nn = 0;     // sites, triangles, charges, quadrature nodes
    int method = HOBI_HIGHER_ORDER;
    int nverts = 0;                         // mesh vertices
    double* vxyz = nullptr;                 // [nverts][3] vertex positions (lower-order method only)
    double eps1 = 1, eps2 = 80, kappa = 0, eps = 80;
    double center[3] = {0, 0, 0};          // shift applied to the FP32 copies
    double s32 = 1;                         // scale of the FP32 positions: kappa log2(e) (1 if kappa = 0)
    // inputs in internal (spatially sorted) order
    double* xyz = nullptr;                  // [nv][3] site positions
    double* nrm = nullptr;                  // [nv][3] site normals
    int* tri = nullptr;                     // [nf][3]
    double* qpos = nullptr;                 // [nc][3]
    double* q = nullptr;                    // [nc]
    double* qsoa = nullptr;                 // [3][nc_pad] charge positions, SoA, padded
    int nc_pad = 0;
    // setup products
    double* patch = nullptr;                // [nf][10][3]
    NodeD* node64 = nullptr;                // [nn] positions, normals, Gamma, Phi
    NodeF* node32 = nullptr;                // [nn] FP32 copy (positions shifted by center)
    int4* node_vid = nullptr;               // [nn] vertex ids of each node's triangle (FP64 path)
    int2* blk_range = nullptr;              // [nn/64] min, max vertex id per 64-node block
    double* w = nullptr;                    // [nn] quadrature weight * Jacobian
    double* tgt64 = nullptr;                // [6][nv_pad] SoA targets x,y,z,nx,ny,nz
    float* tgt32 = nullptr;                 // [6][nv_pad] FP32 SoA (shifted)
    int* inc_off = nullptr;                 // [nv+1] incidence CSR (vertex -> entries)
    int* inc_ent = nullptr;                 // [3 nf] entry = tri * 3 + local vertex
    double* coef = nullptr;                 // [3 nf][12] singular (Duffy) coefficients
    double* rhs = nullptr;                  // [2 nv] (S1, S2)
    // per-matvec work space
    double* partial = nullptr;              // [chunks][2][nv_pad]
    int nv_pad = 0;
    PairPlan plan64{}, plan32{}, plan_pts{};
    size_t partial_elems = 0;
};

// ---- setup kernels (setup_kernels.hip) ----
hipError_t launch_patch(const DeviceProblem& p, int* d_err /*[nf]*/, hipStream_t s);
hipError_t launch_regular_nodes(const DeviceProblem& p, hipStream_t s);
hipError_t launch_targets(const DeviceProblem& p, hipStream_t s);
hipError_t launch_singular(const DeviceProblem& p, hipStream_t s);
hipError_t launch_sources(const DeviceProblem& p, hipStream_t s);
hipError_t launch_lobi_nodes(const DeviceProblem& p, hipStream_t s);

// ---- matvec kernels (pair_kernels.hip) ----
PairPlan make_plan(int n_pad, int nn, int tpl);
constexpr int kTpl64 = 2;   // targets per lane of the FP64 pair kernel
hipError_t launch_gather(const DeviceProblem& p, const double* u, bool mixed, hipStream_t s);
hipError_t launch_pair(const DeviceProblem& p, bool mixed, hipStream_t s);
hipError_t launch_combine(const DeviceProblem& p, const double* u, double* y, bool mixed,
                          hipStream_t s);
// reaction potential at the charges (nodes must hold Gamma/Phi of u) and the energy
hipError_t launch_reaction_energy(const DeviceProblem& p, double* phi_reac, double* e_out,
                                  hipStream_t s);
// solid-angle fraction seen from each charge (1 inside, 0 outside)
hipError_t launch_solid_angle(const DeviceProblem& p, double* frac, hipStream_t s);
hipError_t launch_permute(const double* in, double* out, const int* perm, int nv, bool to_internal,
                          hipStream_t s);

// ---- Krylov kernels (gmres_kernels.hip) ----
constexpr int kDotBlocks = 64;
hipError_t launch_dots(const double* V, size_t ld, int nvec, const double* w, int n,
                       double* partial, hipStream_t s);
hipError_t launch_reduce(const double* partial, int nvec, double* out, int sqrt_out,
                         hipStream_t s);
hipError_t launch_multi_axpy(const double* V, size_t ld, int nvec, const double* coef,
                             double sign, double* w, int n, hipStream_t s);
hipError_t launch_scale_copy(const double* in, const double* denom, double* out, int n,
                             hipStream_t s);
hipError_t launch_sub(const double* a, const double* b, double* out, int n, hipStream_t s);
hipError_t launch_givens(double* H, int ldh, int k, const double* h1, const double* h2,
                         const double* hnext, double* cs, double* sn, double* g,
                         double bnorm, double* res, hipStream_t s);
hipError_t launch_init_g(const double* beta, double* g, int m, hipStream_t s);
hipError_t launch_trisolve(const double* H, int ldh, int k, const double* g, double* y,
                           hipStream_t s);

}  // namespace hobi
