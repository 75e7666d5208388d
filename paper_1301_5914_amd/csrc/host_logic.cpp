// Host-side logic without HIP: validation, Morton ordering, the treecode partition and walk.
#include "host_logic.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <numeric>

namespace hobi {

namespace {

bool fail_msg(std::string* msg, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (msg) *msg = buf;
    return false;
}

}  // namespace

uint64_t spread3(uint64_t v) {   // 21 bits -> every third bit
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Indices 0..n-1 ordered by key, ties in index order: a least-significant-digit radix sort
// (each pass a stable counting sort on one digit; 16-bit digits for large inputs, 8-bit
// for small ones, passes whose digit is the same for every key skipped).
std::vector<int> stable_key_order(const std::vector<uint64_t>& key_in) {
    const size_t n = key_in.size();
    const int bits = n >= 65536 ? 16 : 8;
    const size_t radix = (size_t)1 << bits;
    const int passes = 64 / bits;
    std::vector<uint64_t> k(key_in), k2(n);
    std::vector<int> ord(n), o2(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::vector<uint32_t> hist((size_t)passes * radix, 0);
    for (size_t i = 0; i < n; ++i)
        for (int p = 0; p < passes; ++p) hist[p * radix + ((k[i] >> (bits * p)) & (radix - 1))]++;
    for (int p = 0; p < passes; ++p) {
        uint32_t* h = &hist[p * radix];
        if (*std::max_element(h, h + radix) == n) continue;
        uint32_t sum = 0;
        for (size_t d = 0; d < radix; ++d) {
            const uint32_t c = h[d];
            h[d] = sum;
            sum += c;
        }
        const int shift = bits * p;
        for (size_t i = 0; i < n; ++i) {
            const uint32_t at = h[(k[i] >> shift) & (radix - 1)]++;
            k2[at] = k[i];
            o2[at] = ord[i];
        }
        k.swap(k2);
        ord.swap(o2);
    }
    return ord;
}

std::vector<int> morton_order(const std::vector<double>& pts, int n, const double lo[3], const double hi[3]) {
    std::vector<uint64_t> code(n);
    for (int i = 0; i < n; ++i) {
        uint64_t c = 0;
        for (int d = 0; d < 3; ++d) {
            const double ext = hi[d] - lo[d] > 0 ? hi[d] - lo[d] : 1.0;
            double f = (pts[3 * i + d] - lo[d]) / ext;
            f = std::min(std::max(f, 0.0), 1.0);
            c |= spread3((uint64_t)(f * 2097151.0)) << d;
        }
        code[i] = c;
    }
    return stable_key_order(code);
}

bool check_mesh(int nv, const double* xyz, std::vector<double>& nrm, int nf, const int32_t* tri,
                std::string* msg) {
    for (int i = 0; i < nv; ++i) {
        double* n = &nrm[3 * i];
        const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (std::fabs(l - 1.0) > 1e-6) return fail_msg(msg, "normal %d is not unit length", i);
        n[0] /= l, n[1] /= l, n[2] /= l;
    }
    std::vector<uint64_t> keys;
    keys.reserve(3 * (size_t)nf);
    std::vector<char> used(nv, 0);
    int64_t disagree = 0;
    for (int t = 0; t < nf; ++t) {
        const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            return fail_msg(msg, "triangle %d: vertex id out of range", t);
        if (a == b || b == c || a == c) return fail_msg(msg, "triangle %d repeats a vertex", t);
        used[a] = used[b] = used[c] = 1;
        keys.push_back((uint64_t)a * nv + b);
        keys.push_back((uint64_t)b * nv + c);
        keys.push_back((uint64_t)c * nv + a);
        double e1[3], e2[3], cr[3], ns[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = xyz[3 * b + d] - xyz[3 * a + d];
            e2[d] = xyz[3 * c + d] - xyz[3 * a + d];
            ns[d] = nrm[3 * a + d] + nrm[3 * b + d] + nrm[3 * c + d];
        }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double area2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double l1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
        const double l2 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
        if (!(area2 > 1e-12 * std::max(l1, l2))) return fail_msg(msg, "triangle %d is degenerate", t);
        if (!(cr[0] * ns[0] + cr[1] * ns[1] + cr[2] * ns[2] > 0.0)) ++disagree;
    }
    // every triangle, counter-clockwise seen from outside, must agree with the outward
    // normals at its vertices (the curved element is built from them)
    if (disagree > 0)
        return fail_msg(msg, "%lld of %d triangles disagree with their vertex normals",
                    (long long)disagree, nf);
    for (int i = 0; i < nv; ++i)
        if (!used[i]) return fail_msg(msg, "vertex %d is not used by any triangle", i);
    std::vector<uint64_t> sorted(keys);
    std::sort(sorted.begin(), sorted.end());
    for (size_t i = 1; i < sorted.size(); ++i)
        if (sorted[i] == sorted[i - 1])
            return fail_msg(msg, "directed edge used twice (non-manifold or misoriented)");
    for (uint64_t k : sorted) {
        const uint64_t a = k / nv, b = k % nv;
        if (!std::binary_search(sorted.begin(), sorted.end(), b * nv + a))
            return fail_msg(msg, "open edge (%d, %d)", (int)a, (int)b);
    }
    return true;
}


bool plan_tree(int nn, const double* node_xyz, int nv, const double* tgt, size_t tgt_stride, int nf,
               const int* tri, int method, double theta, int leaf, int batch, int tpl64, TreeHostPlan* out,
               std::string* msg) {
    TreeHostPlan& t = *out;
    t = TreeHostPlan{};
    if (nn < 1 || nv < 1 || leaf < 1 || batch < 64 || batch % 64 != 0)
        return fail_msg(msg, "treecode plan: bad sizes");
    t.nleaf = (nn + leaf - 1) / leaf;
    t.nbatch = (nv + batch - 1) / batch;
    // clusters: node range, box (lo, hi, ungrown), vertex-id range, children
    struct Clu {
        int a, b, vlo, vhi, c0, c1;
        double lo[3], hi[3];
    };
    std::vector<Clu> cl(t.nleaf);
    for (int c = 0; c < t.nleaf; ++c) {
        Clu& k = cl[c];
        k.a = c * leaf;
        k.b = std::min(k.a + leaf, nn);
        k.c0 = k.c1 = -1;
        for (int q = 0; q < 3; ++q) k.lo[q] = 1e300, k.hi[q] = -1e300;
        for (int j = k.a; j < k.b; ++j)
            for (int q = 0; q < 3; ++q) {
                const double v = node_xyz[3 * (size_t)j + q];
                k.lo[q] = std::min(k.lo[q], v), k.hi[q] = std::max(k.hi[q], v);
            }
        if (method == 1) {
            k.vlo = k.a, k.vhi = k.b - 1;   // node j is site j, left out of its own row only
        } else {
            k.vlo = nv, k.vhi = -1;
            for (int f = k.a / 4; f < (k.b + 3) / 4 && f < nf; ++f)
                for (int q = 0; q < 3; ++q)
                    k.vlo = std::min(k.vlo, tri[3 * f + q]), k.vhi = std::max(k.vhi, tri[3 * f + q]);
        }
    }
    std::vector<int> level(t.nleaf);
    std::iota(level.begin(), level.end(), 0);
    t.nlev = 0;
    while (level.size() > 1) {
        if (t.nlev >= kTreeMaxLevels) return fail_msg(msg, "cluster tree too deep");
        t.lev_off[t.nlev] = (int)cl.size();
        std::vector<int> up;
        for (size_t i = 0; i < level.size(); i += 2) {
            if (i + 1 == level.size()) {
                up.push_back(level[i]);
                continue;
            }
            const Clu l = cl[level[i]], r = cl[level[i + 1]];
            Clu k;
            k.a = l.a, k.b = r.b, k.c0 = level[i], k.c1 = level[i + 1];
            k.vlo = std::min(l.vlo, r.vlo), k.vhi = std::max(l.vhi, r.vhi);
            for (int q = 0; q < 3; ++q) k.lo[q] = std::min(l.lo[q], r.lo[q]), k.hi[q] = std::max(l.hi[q], r.hi[q]);
            cl.push_back(k);
            up.push_back((int)cl.size() - 1);
        }
        level.swap(up);
        ++t.nlev;
    }
    t.lev_off[t.nlev] = (int)cl.size();
    t.root = level[0];
    t.nclu = (int)cl.size();
    // centre of the box [lo, hi] into c; returns its diagonal
    auto box_centre = [](const double lo[3], const double hi[3], double c[3]) {
        double q = 0;
        for (int k = 0; k < 3; ++k) {
            c[k] = 0.5 * (lo[k] + hi[k]);
            q += (hi[k] - lo[k]) * (hi[k] - lo[k]);
        }
        return std::sqrt(q);
    };
    t.crange.resize(2 * (size_t)t.nclu);
    t.cchild.resize(2 * (size_t)t.nclu);
    t.cbox.resize(6 * (size_t)t.nclu);
    t.ccen.resize(3 * (size_t)t.nclu);
    t.crad.resize(t.nclu);
    for (int c = 0; c < t.nclu; ++c) {
        const Clu& k = cl[c];
        const double diag = box_centre(k.lo, k.hi, &t.ccen[3 * (size_t)c]);
        t.crad[c] = 0.5 * diag;
        const double g = kTreeGrow * diag + 1e-12;
        for (int q = 0; q < 3; ++q)
            t.cbox[6 * (size_t)c + q] = k.lo[q] - g, t.cbox[6 * (size_t)c + 3 + q] = k.hi[q] + g;
        t.crange[2 * (size_t)c] = k.a, t.crange[2 * (size_t)c + 1] = k.b;
        t.cchild[2 * (size_t)c] = k.c0, t.cchild[2 * (size_t)c + 1] = k.c1;
    }
    // the walk of every batch: far (1) and near (0) clusters
    t.walk.assign(t.nbatch, {});
    std::vector<int> stack;
    for (int bi = 0; bi < t.nbatch; ++bi) {
        const int a = bi * batch, b = std::min(a + batch, nv);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int i = a; i < b; ++i)
            for (int q = 0; q < 3; ++q) {
                const double v = tgt[(size_t)q * tgt_stride + i];
                lo[q] = std::min(lo[q], v), hi[q] = std::max(hi[q], v);
            }
        double cb[3];
        const double rb = 0.5 * box_centre(lo, hi, cb);
        stack.assign(1, t.root);
        while (!stack.empty()) {
            const int c = stack.back();
            stack.pop_back();
            const bool touches = cl[c].vhi >= a && cl[c].vlo <= b - 1;
            const double* cc = &t.ccen[3 * (size_t)c];
            const double dx = cb[0] - cc[0], dy = cb[1] - cc[1], dz = cb[2] - cc[2];
            if (!touches && rb + t.crad[c] <= theta * std::sqrt(dx * dx + dy * dy + dz * dz)) {
                t.walk[bi].emplace_back(c, 1);
                ++t.nfar;
            } else if (cl[c].c0 < 0) {
                t.walk[bi].emplace_back(c, 0);
                ++t.nnear;
            } else {
                stack.push_back(cl[c].c1);
                stack.push_back(cl[c].c0);
            }
        }
    }
    for (int m = 0; m < 2; ++m) {
        t.tpl[m] = m ? batch / 64 : tpl64;
        t.slot[m] = 64 * t.tpl[m];
        const int slots = (nv + t.slot[m] - 1) / t.slot[m];
        t.slot_row[m].assign(1, 0);
        size_t count = 0;
        for (int sl = 0; sl < slots; ++sl) {
            const int bi = (int)((int64_t)sl * t.slot[m] / batch);
            for (const auto& w : t.walk[bi]) {
                t.items[m].insert(t.items[m].end(), {sl, w.second, w.first, 0});
                ++count;
            }
            if (count > ((size_t)1 << 30)) return fail_msg(msg, "treecode plan too large: raise tree_leaf or tree_theta");
            t.slot_row[m].push_back((int)count);
        }
        t.nitems[m] = (int)count;
        const size_t elems = (size_t)t.nitems[m] * 2 * t.slot[m];
        if (elems > ((size_t)1 << 31))
            return fail_msg(msg, "treecode plan too large (%d work items): raise tree_leaf or tree_theta", t.nitems[m]);
        t.partial_elems = std::max(t.partial_elems, elems);
    }
    return true;
}

}  // namespace hobi
