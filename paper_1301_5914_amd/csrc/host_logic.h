// Host-side logic of the library that needs no GPU: input validation, spatial ordering and
// the treecode's partition and walk.  Plain C++17 with no HIP types, so that it also builds
// with a host compiler alone (the sanitizer build of the tests: host_check_main.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace hobi {

constexpr int kTreeMaxDeg = 7;       // (n + 1)^3 <= 512 proxies per cluster
constexpr int kTreeMaxLevels = 40;
constexpr double kTreeGrow = 1e-6;   // proxy box = node box grown by this fraction of its diagonal (+ 1e-12 A)

// The 21 low bits of v spread to every third bit.
uint64_t spread3(uint64_t v);
// Indices 0..n-1 ordered by key, ties in index order (stable LSD radix sort).
std::vector<int> stable_key_order(const std::vector<uint64_t>& key);
// Morton order of n points ([n][3]) over the box [lo, hi]: each coordinate mapped to [0, 1]
// (an empty extent read as 1), clamped, times 2097151 truncated to 21 bits, interleaved
// with x lowest; ties keep the input order.
std::vector<int> morton_order(const std::vector<double>& pts, int n, const double lo[3], const double hi[3]);

// Closed, consistently oriented 2-manifold: every directed edge once and its reverse once,
// every vertex used, no repeated vertex in a triangle, no degenerate triangle, unit normals
// (to 1e-6, renormalised in place), and every triangle counter-clockwise with respect to
// the sum of its vertex normals.  On failure returns false with a message.
bool check_mesh(int nv, const double* xyz, std::vector<double>& nrm, int nf, const int32_t* tri,
                std::string* msg);

// The treecode's partition of nn quadrature nodes (positions in the library's order, [nn][3])
// into leaves of `leaf` consecutive nodes joined pairwise into a binary tree, and the walk of
// every batch of `batch` consecutive targets (x, y, z at tgt[q * tgt_stride + i]): a cluster
// with no triangle incident to the batch and rb + rc <= theta |cb - cc| is far, a leaf that
// fails is near, a parent that fails is opened (c0 before c1).  method 1 (lower order): node
// j is site j, a cluster is incident to a batch whose site range meets its node range.
struct TreeHostPlan {
    int nleaf = 0, nbatch = 0, nlev = 0, root = 0, nclu = 0;
    int lev_off[kTreeMaxLevels + 1] = {};
    std::vector<int> crange;     // [nclu][2] node range
    std::vector<int> cchild;     // [nclu][2] children ((-1, -1) for a leaf)
    std::vector<double> cbox;    // [nclu][6] grown box lo, hi
    std::vector<double> ccen;    // [nclu][3] box centre
    std::vector<double> crad;    // [nclu] half the box diagonal
    std::vector<std::vector<std::pair<int, int>>> walk;   // per batch: (cluster, far 1 / near 0)
    int64_t nfar = 0, nnear = 0;
    // work items {slot, far, cluster, 0} per precision ([0] FP64, [1] mixed), slot-major
    std::vector<int> items[2];
    std::vector<int> slot_row[2];   // items of slot s: [slot_row[s], slot_row[s + 1])
    int tpl[2] = {0, 0}, slot[2] = {0, 0}, nitems[2] = {0, 0};
    size_t partial_elems = 0;       // partial-row doubles of the larger plan
};
bool plan_tree(int nn, const double* node_xyz, int nv, const double* tgt, size_t tgt_stride, int nf,
               const int* tri, int method, double theta, int leaf, int batch, int tpl64, TreeHostPlan* out,
               std::string* msg);

}  // namespace hobi
