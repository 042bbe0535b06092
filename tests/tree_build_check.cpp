// The plan construction of tree_build.hpp against a plain serial construction (the
// library's previous one: index arrays into the coordinate planes, one thread):
// identical source trees and permutations, the same target batches (the same
// points, in the same order of batches), identical interaction lists at several
// thread counts.  Built with the address and undefined-behaviour sanitizers by
// tests/test_tree_build_cpu.py.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <cmath>
#include <random>
#include <vector>

#include "tree_build.hpp"

using namespace stokes::tree;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            ++failures;                                                       \
            if (failures < 20) printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
        }                                                                     \
    } while (0)

static void ref_build_sources(const std::vector<double>& xyz, int64_t n, std::vector<int64_t>& perm,
                          std::vector<Cluster>& cl, int leaf) {
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    struct Item { int64_t start, count; int32_t self; };
    cl.clear();
    cl.push_back(Cluster{});
    std::vector<Item> stack{{0, n, 0}};
    std::vector<int64_t> tmp;
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        Cluster& C = cl[it.self];
        C.start = it.start;
        C.count = it.count;
        for (int d = 0; d < 3; ++d) {
            C.lo[d] = INFINITY;
            C.hi[d] = -INFINITY;
        }
        for (int64_t k = it.start; k < it.start + it.count; ++k)
            for (int d = 0; d < 3; ++d) {
                const double v = xyz[d * n + perm[k]];
                C.lo[d] = std::min(C.lo[d], v);
                C.hi[d] = std::max(C.hi[d], v);
            }
        double emax = 0.0;
        for (int d = 0; d < 3; ++d) emax = std::max(emax, C.hi[d] - C.lo[d]);
        double r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            C.c[d] = 0.5 * (C.lo[d] + C.hi[d]);
            r2 += 0.25 * (C.hi[d] - C.lo[d]) * (C.hi[d] - C.lo[d]);
        }
        C.r = std::sqrt(r2);
        C.first_child = -1;
        C.n_child = 0;
        if (it.count <= leaf || emax == 0.0) continue;
        // split
        std::vector<std::pair<int64_t, int64_t>> groups{{it.start, it.count}};
        for (int d = 0; d < 3; ++d) {
            if (C.hi[d] - C.lo[d] < 0.5 * emax) continue;
            const double mid = C.c[d];
            std::vector<std::pair<int64_t, int64_t>> ng;
            for (auto g : groups) {
                auto b = perm.begin() + g.first, e = b + g.second;
                auto m = std::stable_partition(b, e, [&](int64_t q) { return xyz[d * n + q] <= mid; });
                const int64_t a = m - b;
                if (a == 0 || a == g.second) {
                    ng.push_back(g);
                } else {
                    ng.push_back({g.first, a});
                    ng.push_back({g.first + a, g.second - a});
                }
            }
            groups.swap(ng);
        }
        if (groups.size() < 2) continue;
        const int32_t first = (int32_t)cl.size();
        cl[it.self].first_child = first;
        cl[it.self].n_child = (int32_t)groups.size();
        for (size_t g = 0; g < groups.size(); ++g) {
            cl.push_back(Cluster{});
            stack.push_back({groups[g].first, groups[g].second, first + (int32_t)g});
        }
    }
}

// Median splits along the longest extent down to at most BATCH targets per batch.
static void ref_build_batches(const std::vector<double>& xyz, int64_t n, std::vector<int64_t>& perm,
                          std::vector<Batch>& bt) {
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    bt.clear();
    std::vector<std::pair<int64_t, int64_t>> stack{{0, n}};
    while (!stack.empty()) {
        const auto g = stack.back();
        stack.pop_back();
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = g.first; k < g.first + g.second; ++k)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], xyz[d * n + perm[k]]);
                hi[d] = std::max(hi[d], xyz[d * n + perm[k]]);
            }
        if (g.second <= BATCH) {
            Batch B{};
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                B.c[d] = 0.5 * (lo[d] + hi[d]);
                r2 += 0.25 * (hi[d] - lo[d]) * (hi[d] - lo[d]);
            }
            B.r = std::sqrt(r2);
            B.start = g.first;
            B.count = (int32_t)g.second;
            bt.push_back(B);
            continue;
        }
        int dm = 0;
        for (int d = 1; d < 3; ++d)
            if (hi[d] - lo[d] > hi[dm] - lo[dm]) dm = d;
        const int64_t half = g.second / 2;
        auto b = perm.begin() + g.first;
        std::nth_element(b, b + half, b + g.second,
                         [&](int64_t a, int64_t c) { return xyz[dm * n + a] < xyz[dm * n + c]; });
        stack.push_back({g.first, half});
        stack.push_back({g.first + half, g.second - half});
    }
}


static void ref_lists(const std::vector<Batch>& bt, const std::vector<Cluster>& cl, double theta, int P,
                      Lists& L) {
    std::vector<int32_t> px_off{0}, px_list, dr_off{0}, dr_count, slot_of(cl.size(), -1);
    std::vector<int64_t> dr_start;
    std::vector<int32_t> used;
    int64_t pairs_px = 0, pairs_dir = 0;
    std::vector<int32_t> stack;
    for (const Batch& B : bt) {
        stack.assign(1, 0);
        while (!stack.empty()) {
            const int32_t ci = stack.back();
            stack.pop_back();
            const Cluster& C = cl[ci];
            const double dx = B.c[0] - C.c[0], dy = B.c[1] - C.c[1], dz = B.c[2] - C.c[2];
            const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
            const bool far = B.r + C.r < theta * dist;
            if (far && C.count > P) {
                if (slot_of[ci] < 0) {
                    slot_of[ci] = (int32_t)used.size();
                    used.push_back(ci);
                }
                px_list.push_back(slot_of[ci]);
                pairs_px += (int64_t)B.count * P;
            } else if (C.n_child == 0 || far) {
                if (!dr_start.empty() && dr_off.size() == px_off.size() &&
                    (int64_t)dr_start.size() > dr_off.back() &&
                    dr_start.back() + dr_count.back() == C.start && dr_count.back() + C.count < (1 << 30)) {
                    dr_count.back() += (int32_t)C.count;      // adjacent ranges merge
                } else {
                    dr_start.push_back(C.start);
                    dr_count.push_back((int32_t)C.count);
                }
                pairs_dir += (int64_t)B.count * C.count;
            } else {
                for (int32_t k = C.n_child - 1; k >= 0; --k) stack.push_back(C.first_child + k);
            }
        }
        px_off.push_back((int32_t)px_list.size());
        dr_off.push_back((int32_t)dr_start.size());
    }
    L.px_off = px_off;
    L.px_list = px_list;
    L.used = used;
    L.dr_off = dr_off;
    L.dr_start = dr_start;
    L.dr_count = dr_count;
    L.pairs_px = pairs_px;
    L.pairs_dir = pairs_dir;
}

static bool same_cluster(const Cluster& a, const Cluster& b) {
    for (int d = 0; d < 3; ++d)
        if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d] || a.c[d] != b.c[d]) return false;
    return a.r == b.r && a.start == b.start && a.count == b.count && a.first_child == b.first_child &&
           a.n_child == b.n_child;
}

static void check_case(const std::vector<double>& xyz, int64_t n, int leaf, int degree, double theta) {
    std::vector<int64_t> p0, p1, q0, q1;
    std::vector<Cluster> c0, c1;
    std::vector<Batch> b0, b1;
    ref_build_sources(xyz, n, p0, c0, leaf);
    for (int T : {16, 3, 1}) {   // the last (serial) one is used below
        build_sources(xyz, n, p1, c1, leaf, T);
        CHECK(p0 == p1);
        CHECK(c0.size() == c1.size());
        for (size_t k = 0; k < std::min(c0.size(), c1.size()); ++k) CHECK(same_cluster(c0[k], c1[k]));
    }
    ref_build_batches(xyz, n, q0, b0);
    for (int T : {16, 3, 1}) {   // the last (serial) one is used below
    build_batches(xyz, n, q1, b1, T);
    CHECK(b0.size() == b1.size());
    for (size_t k = 0; k < std::min(b0.size(), b1.size()); ++k) {
        CHECK(b0[k].start == b1[k].start && b0[k].count == b1[k].count);
        for (int d = 0; d < 3; ++d) CHECK(b0[k].c[d] == b1[k].c[d]);
        CHECK(b0[k].r == b1[k].r);
        std::vector<int64_t> s0(q0.begin() + b0[k].start, q0.begin() + b0[k].start + b0[k].count);
        std::vector<int64_t> s1(q1.begin() + b1[k].start, q1.begin() + b1[k].start + b1[k].count);
        std::sort(s0.begin(), s0.end());
        std::sort(s1.begin(), s1.end());
        CHECK(s0 == s1);
    }
    }
    const int n1 = degree + 1, P = n1 * n1 * n1;
    Lists r;
    ref_lists(b1, c1, theta, P, r);
    for (int T : {1, 3, 16}) {
        Lists l;
        build_lists(b1, c1, theta, P, l, T);
        CHECK(l.px_off == r.px_off && l.px_list == r.px_list && l.used == r.used);
        CHECK(l.dr_off == r.dr_off && l.dr_start == r.dr_start && l.dr_count == r.dr_count);
        CHECK(l.pairs_px == r.pairs_px && l.pairs_dir == r.pairs_dir);
        // each batch takes every source exactly once, through proxies or directly:
        // the counts add up to n and the ranges (clusters are ranges of the sorted
        // sources) do not overlap
        for (size_t b = 0; b + 1 < l.px_off.size(); ++b) {
            std::vector<std::pair<int64_t, int64_t>> rg;
            for (int32_t k = l.dr_off[b]; k < l.dr_off[b + 1]; ++k) rg.push_back({l.dr_start[k], l.dr_count[k]});
            for (int32_t k = l.px_off[b]; k < l.px_off[b + 1]; ++k) {
                const Cluster& C = c1[l.used[l.px_list[k]]];
                rg.push_back({C.start, C.count});
            }
            std::sort(rg.begin(), rg.end());
            int64_t next = 0;
            bool ok = true;
            for (const auto& x : rg) {
                ok &= x.first == next;
                next = x.first + x.second;
            }
            CHECK(ok && next == n);
        }
    }
    // work parts: cuts from 0 to the entry count, non-decreasing, each part within one
    // entry of 1 / S of the batch's cost, and the cuts for S / 2 every other one
    {
        Lists s = r;
        split_ranges(s, 512);
        const int nb = (int)s.px_off.size() - 1;
        std::vector<std::vector<int32_t>> cuts;
        for (int S : {1, 2, 4, 8, 16}) cuts.push_back(part_cuts(s, P, S));
        for (int si = 0; si < 5; ++si) {
            const int S = 1 << si;
            const std::vector<int32_t>& c = cuts[si];
            CHECK((int)c.size() == nb * (S + 1));
            bool ok = true;
            for (int b = 0; b < nb && ok; ++b) {
                const int32_t np = s.px_off[b + 1] - s.px_off[b], nd = s.dr_off[b + 1] - s.dr_off[b];
                auto cost = [&](int32_t e) -> int64_t { return e < np ? P : s.dr_count[s.dr_off[b] + e - np]; };
                int64_t total = 0, most = 0;
                for (int32_t e = 0; e < np + nd; ++e) {
                    total += cost(e);
                    most = std::max(most, cost(e));
                }
                const int32_t* cb = &c[(size_t)b * (S + 1)];
                ok &= cb[0] == 0 && cb[S] == np + nd;
                for (int h = 0; h < S && ok; ++h) {
                    ok &= cb[h] <= cb[h + 1];
                    int64_t part = 0;
                    for (int32_t e = cb[h]; e < cb[h + 1]; ++e) part += cost(e);
                    ok &= part <= total / S + most + 1;
                }
                if (si > 0)
                    for (int h = 0; h <= S / 2 && ok; ++h) ok &= cuts[si - 1][(size_t)b * (S / 2 + 1) + h] == cb[2 * h];
            }
            CHECK(ok);
        }
    }
    // pieces of at most `most` sources: in order, covering each batch's ranges exactly
    for (int32_t most : {1, 64, 1000}) {
        Lists s = r;
        split_ranges(s, most);
        CHECK(s.dr_off.size() == r.dr_off.size());
        CHECK(s.px_off == r.px_off && s.px_list == r.px_list);
        for (size_t b = 0; b + 1 < r.dr_off.size() && b + 1 < s.dr_off.size(); ++b) {
            int32_t k = s.dr_off[b];
            bool ok = true;
            for (int32_t e = r.dr_off[b]; e < r.dr_off[b + 1]; ++e) {
                int64_t at = r.dr_start[e];
                while (at < r.dr_start[e] + r.dr_count[e]) {
                    ok &= k < s.dr_off[b + 1] && s.dr_start[k] == at && s.dr_count[k] >= 1 &&
                          s.dr_count[k] <= most;
                    if (!ok) break;
                    at += s.dr_count[k++];
                }
                ok &= at == r.dr_start[e] + r.dr_count[e];
                if (!ok) break;
            }
            CHECK(ok && k == s.dr_off[b + 1]);
        }
    }
}

int main() {
    std::mt19937_64 g(5);
    std::normal_distribution<double> N(0.0, 1.0);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    int cases = 0;
    for (int64_t n : {1, 2, 63, 64, 65, 129, 1000, 5000, 40000, 70001}) {
        // points in a ball
        std::vector<double> xyz(3 * n);
        for (int64_t k = 0; k < n; ++k) {
            double v[3], r2 = 2.0;
            while (r2 > 1.0) {
                for (double& c : v) c = U(g);
                r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            }
            for (int d = 0; d < 3; ++d) xyz[d * n + k] = 5.0 * v[d];
        }
        for (int leaf : {16, 128}) {
            check_case(xyz, n, leaf, 6, 0.7);
            ++cases;
        }
        // fiber-like: 16-point straight segments at random positions and directions
        std::vector<double> f(3 * n);
        for (int64_t k = 0; k < n; k += 16) {
            double c[3], t[3];
            for (int d = 0; d < 3; ++d) {
                c[d] = 4.0 * U(g);
                t[d] = N(g);
            }
            const double tn = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            for (int64_t j = k; j < std::min<int64_t>(n, k + 16); ++j)
                for (int d = 0; d < 3; ++d) f[d * n + j] = c[d] + 0.05 * (j - k) * t[d] / tn;
        }
        check_case(f, n, 128, 8, 0.5);
        ++cases;
    }
    // degenerate: every point on a plane and repeated points
    {
        const int64_t n = 3000;
        std::vector<double> xyz(3 * n);
        for (int64_t k = 0; k < n; ++k) {
            xyz[k] = (double)(k % 50);
            xyz[n + k] = (double)((k / 50) % 7);
            xyz[2 * n + k] = 0.0;
        }
        check_case(xyz, n, 32, 6, 0.7);
        ++cases;
    }
    printf("%d cases, %d failures\n", cases, failures);
    return failures ? 1 : 0;
}
