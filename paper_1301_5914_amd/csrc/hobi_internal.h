// Internal declarations of the HOBI-PB library: device buffers of a problem and the
// host-side launch wrappers of every kernel.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hobi.h"
#include "hobi_device.h"
#include "host_logic.h"

namespace hobi {

// Launch configuration of the point sums at the charges: blocks of targets by chunks of
// nodes, fixed per problem size only.
struct GridPlan {
    int tpl;            // targets per lane
    int block;          // threads per block
    int target_blocks;  // blocks along the targets
    int chunks;         // source chunks (split of the node range)
    int chunk;          // nodes per chunk
};

// Split of the dense pair sum over waves ("workers").  The targets are cut into slots of
// 64 * tpl (one wave's targets), the nodes into `groups` contiguous ranges of equal length
// (within one node; a multiple of per_row of them, some empty on tiny problems).  With
// per_row = 4 (the FP32 pair kernels) one workgroup of 4 waves takes block b: slot
// b % slots against groups 4 (b / slots) .. 4 (b / slots) + 3, the waves sharing out their
// 64-node blocks, and sums the waves' rows in LDS in wave order into one row of partial sums
// (2 * slot doubles, row b).  With per_row = 1 (the FP64 pair kernels and the off-surface
// field kernels) worker w takes slot w % slots against group w / slots into row w.  Either
// way there are `rows` = groups / per_row rows per slot.  groups is chosen so
// that the workers make about kPairPasses passes of the waves the device holds at once:
// short workers let the hardware's dispatch balance the load to the end of the launch (one
// long pass ends with many SIMDs idle), while each partial row is written once and read once
// by the combine step, so a group keeps at least kMinGroupNodes nodes (one 64-node block: a
// wave then always has a whole block to walk).  The blocks of one
// row index run side by side on one XCD and read the same nodes from its L2 at about the
// same time.  The split depends on the problem and the device only, and so does the order of
// every sum (results are reproducible bit for bit).
constexpr int kPairPasses = 16;
constexpr int kMinGroupNodes = 64;
struct PairPlan {
    int tpl;            // targets per lane
    int slot;           // targets per slot: 64 * tpl
    int slots;          // ceil(nv / slot)
    int groups;         // node groups, a multiple of per_row
    int per_row;        // node groups summed into one partial row: 4 or 1
    int rows;           // partial rows per slot: groups / per_row
    int workers;        // slots * groups waves
    int blocks;         // workgroups of a launch: ceil(workers / 4)
    const int* gstart;  // device [groups + 1]: node range of group g is [gstart[g], gstart[g + 1])
};

// Treecode form of the regular sum (hobi_params.tree_theta > 0; higher-order method).  The
// partition is geometric and built once at problem creation; the proxy charges depend on u
// and are rebuilt by every matvec.
struct TreePlan {
    int on = 0;
    int degree = 0, nprox = 0;       // n, (n + 1)^3
    int leaf = 0, batch = 0;
    int nleaf = 0, nclu = 0, nbatch = 0;   // leaves, all clusters (leaves first), batches
    int nlev = 0;                    // parent levels
    int lev_off[kTreeMaxLevels + 1] = {};  // parents of level l: clusters [lev_off[l], lev_off[l + 1])
    int64_t nfar = 0, nnear = 0;     // accepted (batch, cluster) and near (batch, leaf) pairs
    int2* clu_range = nullptr;       // [nclu] node range of each cluster
    double* clu_box = nullptr;       // [nclu][6] grown box: lo[3], hi[3]
    int2* clu_child = nullptr;       // [nclu] children of a parent ((-1, -1) for a leaf)
    int root = 0;                    // the root cluster
    std::vector<double> h_cen, h_rad;  // host copies: centre [nclu][3] and radius of each cluster
    std::vector<int2> h_child;         // and its children, for the walks of hobi_field
    ProxyD* prox64 = nullptr;        // [nclu][nprox]
    ProxyF* prox32 = nullptr;        // [nclu][nprox]
    int4* items[2] = {nullptr, nullptr};   // [0] FP64, [1] mixed: {slot, far, cluster, 0}, slot-major
    int* slot_row[2] = {nullptr, nullptr}; // [slots + 1]: items of slot s are [slot_row[s], slot_row[s + 1])
    int nitems[2] = {0, 0};
    int slot[2] = {0, 0};            // targets per slot
    int tpl[2] = {0, 0};
    double* partial = nullptr;       // [nitems][2][slot] (the larger of the two)
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
    double extent = 0;                      // diagonal of the vertices' bounding box
    double s32 = 1;                         // scale of the FP32 positions: kappa (1 if kappa = 0)
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
    double* dinv = nullptr;                 // [2 nv] the right preconditioner's inverse diagonal
    // per-matvec work space
    double* partial = nullptr;              // pair sums: [workers][2][slot]; point sums: [chunks][nc_pad]
    int nv_pad = 0;
    PairPlan plan64{}, plan32{};
    GridPlan plan_pts{};
    int* plan_tab = nullptr;                // device group starts of plan64, then of plan32
    size_t partial_elems = 0;               // allocated: what the current precision's plan needs
    size_t partial_need[2] = {0, 0};        // what the FP64 [0] and FP32 [1] plans need (with the point sums)
    TreePlan tree{};
};

// ---- setup kernels (setup_kernels.hip) ----
hipError_t launch_patch(const DeviceProblem& p, int* d_err /*[nf]*/, hipStream_t s);
hipError_t launch_regular_nodes(const DeviceProblem& p, hipStream_t s);
hipError_t launch_targets(const DeviceProblem& p, hipStream_t s);
hipError_t launch_singular(const DeviceProblem& p, hipStream_t s);
hipError_t launch_sources(const DeviceProblem& p, hipStream_t s);
hipError_t launch_lobi_nodes(const DeviceProblem& p, hipStream_t s);

// ---- matvec kernels (pair_kernels.hip) ----
GridPlan make_grid_plan(int n_pad, int nn, int tpl);
constexpr int kTpl64 = 4;      // targets per lane of the FP64 pair kernel (dense sum, single and served)
constexpr int kTreeTpl64 = 2;  // targets per lane of the treecode's FP64 tiles
constexpr int kMaxRefineSteps = 16;   // outer steps of the tree_refine defect correction
inline int tpl32_for(int nv_pad) { return nv_pad >= 16384 ? 8 : 4; }
// Waves of the FP32 (mixed) or FP64 pair kernel with `tpl` targets per lane that device
// `device` holds at once (occupancy of the kernel times the compute units); 0 on error.
int pair_resident_waves(int device, bool mixed, int tpl);
// The split of nv targets by nn nodes for a device holding resident_waves of the kernel at
// once; the group starts are appended to `gstart` (the plan's device pointer is left null).
bool make_pair_plan(int nv, int nn, int tpl, int resident_waves, int per_row, PairPlan* plan,
                    std::vector<int>* gstart);
hipError_t launch_gather(const DeviceProblem& p, const double* u, bool mixed, hipStream_t s);
hipError_t launch_pair(const DeviceProblem& p, bool mixed, hipStream_t s);
hipError_t launch_combine(const DeviceProblem& p, const double* u, double* y, bool mixed,
                          hipStream_t s);
// The same two launches on an explicit plan and partial-row buffer (the plan's gstart must
// be a device table of groups + 1 node starts).
hipError_t launch_pair_plan(const DeviceProblem& p, const PairPlan& pl, double* partial, bool mixed,
                            hipStream_t s);
hipError_t launch_combine_plan(const DeviceProblem& p, const PairPlan& pl, const double* partial,
                               const double* u, double* y, hipStream_t s);

// Static work space of the allocation-free matvec (hobi_matvec_noalloc): one array per
// device in the library's code object, holding a table of node-group starts
// (kStaticTableBytes) followed by the partial rows of the pair sum.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr size_t kStaticTableBytes = (size_t)64 << 10;
// The array's device address on `device`, which must be the current device.  Looked up
// once per device (hipGetSymbolAddress) and cached.
hipError_t static_scratch_address(int device, void** out);
// The dense-sum split of `base` (same slots) with its node groups cut down so that the
// partial rows and the group-start table fit in the static work space; false if not even
// one group fits (*row_bytes: bytes of one group's rows).  out->gstart is left null.
bool make_static_pair_plan(const PairPlan& base, int nn, PairPlan* out, size_t* row_bytes);
// tab[g] = g * nn / groups for g = 0 .. groups (the group starts of make_pair_plan).
hipError_t launch_group_starts(int* tab, int groups, int nn, hipStream_t s);

// reaction potential at the charges (nodes must hold Gamma/Phi of u) and the energy
hipError_t launch_reaction_energy(const DeviceProblem& p, double* phi_reac, double* e_out,
                                  hipStream_t s);
// y[i] = the FP64 pair kernel's exp(-x[i]) (fn 0) or 1 / sqrt(x[i]) (fn 1), device arrays
hipError_t launch_device_math(int fn, const double* x, double* y, int n, hipStream_t s);
// solid-angle fraction seen from each charge (1 inside, 0 outside)
hipError_t launch_solid_angle(const DeviceProblem& p, double* frac, hipStream_t s);

// ---- potential and field at points off the surface (field_kernels.hip) ----
constexpr int kFieldTpl32 = 4;   // points per lane of the FP32 field kernel
constexpr int kFieldTpl64 = 2;   // and of the FP64 one
// Work space of one field evaluation, kept by the problem and grown on demand.
struct FieldWork {
    int np = 0, np_pad = 0;       // points, points padded to whole slots
    double* pts64 = nullptr;      // [3][np_pad] SoA, Morton order
    float* pts32 = nullptr;       // [3][np_pad] in the frame of the FP32 node records
    double* partial = nullptr;    // [workers][5][slot]
    int* gstart = nullptr;        // [groups + 1]
    double* out = nullptr;        // [np][9] phi, E, R, -grad R, solid-angle fraction
    int* inside = nullptr;        // [np]
    int* order = nullptr;         // [np] caller index of each sorted point
    double* outc = nullptr;       // [8 np] outputs in caller order: phi, E (3), R, -grad R (3)
    int* insc = nullptr;          // [np + 1] sides in caller order, then the non-finite flag
    double* raw = nullptr;        // [3 np] the caller's points
    uint64_t* keys = nullptr;     // [2 np] Morton codes: unsorted, then sorted
    int* idx = nullptr;           // [np] 0 .. np - 1
    void* sort_tmp = nullptr;     // radix-sort work space
    double* bbox = nullptr;       // [nbatch][6] lo, hi of each treecode batch of sorted points
    double* hbox = nullptr;       // pinned host copy
    int4* items = nullptr;        // treecode: work items {slot, far, cluster, 0}, slot-major
    int* slot_row = nullptr;      // treecode: items of slot s are [slot_row[s], slot_row[s + 1])
    size_t cap_pts64 = 0, cap_pts32 = 0, cap_partial = 0, cap_gstart = 0, cap_out = 0, cap_inside = 0;
    size_t cap_items = 0, cap_slot_row = 0, cap_order = 0, cap_outc = 0, cap_insc = 0;
    size_t cap_raw = 0, cap_keys = 0, cap_idx = 0, cap_sort_tmp = 0, cap_bbox = 0, cap_hbox = 0;
    int64_t tree_far = 0, tree_near = 0;   // accepted and near (batch, cluster) pairs of the last call
};
// Waves of the mixed or FP64 field kernel the device holds at once (0 on error).
int field_resident_waves(int device, bool mixed);
// Pair sums of the plan's workers (strengths of u must be in the node records: launch_gather
// with the same precision), then the per-point combine.
hipError_t launch_field_pairs(const DeviceProblem& p, const FieldWork& f, const PairPlan& plan, bool mixed,
                              hipStream_t s);
// slot_row non-null: the rows of slot s are the treecode items slot_row[s] .. slot_row[s + 1] - 1,
// stored from row_base on; the points [p0, p1) (p1 < 0: all)
hipError_t launch_field_combine(const DeviceProblem& p, const FieldWork& f, const PairPlan& plan, bool mixed,
                                hipStream_t s, const int* slot_row = nullptr, int row_base = 0, int p0 = 0,
                                int p1 = -1);
// treecode field (proxy charges computed): one wave per item of f.items, nitems of them
constexpr int kFieldTreeBatch = 64 * kFieldTpl32;   // points per batch: one FP32 field slot
constexpr size_t kFieldTreeRows = (size_t)1 << 29;  // partial-row doubles of one pass (4 GiB)
hipError_t launch_field_tree_pairs(const DeviceProblem& p, const FieldWork& f, int nitems, bool mixed,
                                   hipStream_t s);
hipError_t launch_permute(const double* in, double* out, const int* perm, int nv, bool to_internal,
                          hipStream_t s);
// Bytes of radix-sort work space for np points (0 on error).
size_t point_sort_temp_bytes(int np);
// The points f.raw in Morton order over [lo, hi] (the rule of the problem's own ordering:
// 21 bits per coordinate, x lowest, ties in input order): f.order, then f.pts64 / f.pts32
// (SoA, padded to f.np_pad by repeating the last point; pts32 shifted by center, scaled by
// s32), and with nbatch > 0 the box of each run of kFieldTreeBatch sorted points in f.bbox.
hipError_t launch_point_order(const FieldWork& f, const double lo[3], const double hi[3], const double center[3],
                              double s32, int nbatch, hipStream_t s);
// f.out / f.inside (sorted points) -> f.outc / f.insc in the caller's order (f.order), and
// f.insc[np] = 1 if any output value is not finite (the caller clears it first)
hipError_t launch_field_scatter(const FieldWork& f, hipStream_t s);

// ---- treecode (tree_kernels.hip) ----
// proxy charges of every cluster (node strengths of u must be gathered, FP64 records)
hipError_t launch_tree_proxies(const DeviceProblem& p, bool mixed, hipStream_t s);
// one partial row per work item: near items the masked pair sum, far items the proxies
hipError_t launch_tree_pairs(const DeviceProblem& p, bool mixed, hipStream_t s);
// rows of each slot in item order, singular correction and diagonal
hipError_t launch_tree_combine(const DeviceProblem& p, const double* u, double* y, bool mixed, hipStream_t s);

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
// out = a + b
hipError_t launch_add(const double* a, const double* b, double* out, int n, hipStream_t s);
// out[i] = dinv[i] in[i], i < n
hipError_t launch_diag_scale(const double* in, double* out, int n, const double* dinv, hipStream_t s);
// x[i] += dinv[i] sum_j coef[j] V[j][i], i < n
hipError_t launch_multi_axpy_scaled(const double* V, size_t ld, int nvec, const double* coef, double* x, int n,
                                    const double* dinv, hipStream_t s);
// dinv [2 nv]: the inverse diagonal of the right preconditioner of diag_scaling mode 1 (the two
// row blocks' constants) or 2 (A's own diagonal; mode 1 for the lower-order method)
hipError_t launch_scaling(const DeviceProblem& p, int mode, double* dinv, hipStream_t s);
hipError_t launch_givens(double* H, int ldh, int k, const double* h1, const double* h2,
                         const double* hnext, double* cs, double* sn, double* g,
                         double bnorm, double* res, hipStream_t s);
hipError_t launch_init_g(const double* beta, double* g, int m, hipStream_t s);
hipError_t launch_trisolve(const double* H, int ldh, int k, const double* g, double* y,
                           hipStream_t s);

}  // namespace hobi
