// Host-side state shared by the C-ABI implementation files (problem API and request
// server).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hobi.h"
#include "hobi_internal.h"

struct hobi_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool profile = false;
    void* scratch = nullptr;   // this device's static work space (hobi_matvec_noalloc)
    std::string err;
};

namespace hobi {

enum TimerKind { T_GATHER = 0, T_PAIR, T_COMBINE, T_KRYLOV, T_FIELD, T_NKINDS };

struct Timer {
    hipEvent_t a, b;
    int kind;
};

struct Krylov {
    int n = 0, m = 0;
    double *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
    double *h1 = nullptr, *h2 = nullptr, *hn = nullptr, *yk = nullptr, *res = nullptr;
    double *dpart = nullptr, *x = nullptr, *tmp = nullptr, *scal = nullptr;
    double *xo = nullptr, *ro = nullptr;   // defect correction: outer iterate and dense residual
};

}  // namespace hobi

struct hobi_problem_s {
    hobi_ctx ctx = nullptr;
    hobi::DeviceProblem d;
    hobi_params prm{};
    std::vector<int> vperm, tperm;   // internal -> caller ids
    int* d_vperm = nullptr;          // [nv] internal -> caller vertex
    double* u_in = nullptr;          // [2 nv] internal-order work vectors
    double* y_out = nullptr;
    double* phi_reac = nullptr;      // [nc]
    double* e_dev = nullptr;         // [1]
    double* host_pinned = nullptr;   // small pinned buffer for scalar read-backs
    int* d_err = nullptr;            // [nf] per-triangle flags of the curved-edge construction
    hobi::Krylov kr;
    hobi::FieldWork field;           // potential / field evaluation work space
    std::vector<hobi::Timer> pending;
    std::vector<hipEvent_t> event_pool;
    double ms[hobi::T_NKINDS] = {};
    int64_t cnt[hobi::T_NKINDS] = {};
    hobi_stats last{};
};


namespace hobi {
// internal order (device) -> caller order (host or device) of a [2 nv] vector
hobi_status host_from_internal(hobi_problem pb, const double* src, int on_device, double* y);
// records a message on the context and returns code
hobi_status host_fail(hobi_ctx ctx, hobi_status code, const char* msg);
// hobi_problem_create whose treecode buffers may take at most tree_limit bytes: beyond it
// the call fails with HOBI_E_OOM and *tree_need (nullable) holds their size (0 on any other
// outcome).
hobi_status problem_create_limited(hobi_ctx ctx, int32_t nv, const double* xyz, const double* nrm, int32_t nf,
                                   const int32_t* tri, int32_t nc, const double* qpos, const double* q,
                                   const hobi_params* params, hobi_problem* out, int64_t tree_limit,
                                   int64_t* tree_need);
}  // namespace hobi
