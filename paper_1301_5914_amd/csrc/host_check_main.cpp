// Command-line driver of host_logic.cpp for the host-only test build (compiled by the
// tests with a host compiler and AddressSanitizer / UndefinedBehaviorSanitizer): runs the
// library's mesh validation, Morton ordering and treecode partition on inputs read from a
// binary file and writes what they return.
//   host_check mesh   IN          IN: int32 nv, nf; f64 xyz[nv][3], nrm[nv][3]; int32 tri[nf][3]
//                                 prints "ok" or "error: <message>"
//   host_check morton IN OUT      IN: int32 n; f64 pts[n][3], lo[3], hi[3];  OUT: int32 order[n]
//   host_check tree   IN OUT      IN: int32 nn, nv, nf, method, leaf, batch, tpl64; f64 theta;
//                                 f64 nodes[nn][3], tgt[3][nv]; int32 tri[nf][3]
//                                 OUT (text): "nfar nnear", then per batch "far c ... | near c ..."
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_logic.h"

namespace {

template <class T>
bool get(FILE* f, T* p, size_t n) {
    return std::fread(p, sizeof(T), n, f) == n;
}

int run_mesh(FILE* f) {
    int32_t nv = 0, nf = 0;
    if (!get(f, &nv, 1) || !get(f, &nf, 1) || nv < 1 || nf < 1) return 2;
    std::vector<double> xyz(3 * (size_t)nv), nrm(3 * (size_t)nv);
    std::vector<int32_t> tri(3 * (size_t)nf);
    if (!get(f, xyz.data(), xyz.size()) || !get(f, nrm.data(), nrm.size()) || !get(f, tri.data(), tri.size()))
        return 2;
    std::string msg;
    if (hobi::check_mesh(nv, xyz.data(), nrm, nf, tri.data(), &msg))
        std::printf("ok\n");
    else
        std::printf("error: %s\n", msg.c_str());
    return 0;
}

int run_morton(FILE* f, const char* out) {
    int32_t n = 0;
    if (!get(f, &n, 1) || n < 1) return 2;
    std::vector<double> pts(3 * (size_t)n);
    double lo[3], hi[3];
    if (!get(f, pts.data(), pts.size()) || !get(f, lo, 3) || !get(f, hi, 3)) return 2;
    const std::vector<int> ord = hobi::morton_order(pts, n, lo, hi);
    FILE* o = std::fopen(out, "wb");
    if (!o) return 2;
    const bool ok = std::fwrite(ord.data(), sizeof(int), ord.size(), o) == ord.size();
    std::fclose(o);
    return ok ? 0 : 2;
}

int run_tree(FILE* f, const char* out) {
    int32_t h[7];
    double theta = 0;
    if (!get(f, h, 7) || !get(f, &theta, 1)) return 2;
    const int nn = h[0], nv = h[1], nf = h[2], method = h[3], leaf = h[4], batch = h[5], tpl64 = h[6];
    if (nn < 1 || nv < 1 || nf < 1) return 2;
    std::vector<double> nodes(3 * (size_t)nn), tgt(3 * (size_t)nv);
    std::vector<int32_t> tri(3 * (size_t)nf);
    if (!get(f, nodes.data(), nodes.size()) || !get(f, tgt.data(), tgt.size()) || !get(f, tri.data(), tri.size()))
        return 2;
    hobi::TreeHostPlan p;
    std::string msg;
    if (!hobi::plan_tree(nn, nodes.data(), nv, tgt.data(), (size_t)nv, nf, tri.data(), method, theta, leaf, batch,
                         tpl64, &p, &msg)) {
        std::printf("error: %s\n", msg.c_str());
        return 0;
    }
    FILE* o = std::fopen(out, "w");
    if (!o) return 2;
    std::fprintf(o, "%lld %lld\n", (long long)p.nfar, (long long)p.nnear);
    for (const auto& w : p.walk) {
        std::fprintf(o, "far");
        for (const auto& e : w)
            if (e.second) std::fprintf(o, " %d", e.first);
        std::fprintf(o, " | near");
        for (const auto& e : w)
            if (!e.second) std::fprintf(o, " %d", e.first);
        std::fprintf(o, "\n");
    }
    // the slot-major item lists cover each slot's batch walk once per precision
    for (int m = 0; m < 2; ++m)
        std::fprintf(o, "items %d %d %zu\n", p.nitems[m], p.slot[m], p.partial_elems);
    std::fclose(o);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    FILE* f = std::fopen(argv[2], "rb");
    if (!f) return 2;
    int rc = 2;
    if (!std::strcmp(argv[1], "mesh")) rc = run_mesh(f);
    else if (!std::strcmp(argv[1], "morton") && argc > 3) rc = run_morton(f, argv[3]);
    else if (!std::strcmp(argv[1], "tree") && argc > 3) rc = run_tree(f, argv[3]);
    std::fclose(f);
    return rc;
}
