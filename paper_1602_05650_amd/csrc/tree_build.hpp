// Host-side construction of a treecode plan: the source cluster tree, the target
// batches and the interaction lists (which clusters a batch takes through their
// proxies, which source ranges it sums directly).  Plain C++ (no HIP headers), so the
// CPU tests compile it on their own, with the sanitizers, against a plain serial
// construction.
//
// The points are bisected as records holding their coordinates (not through an index
// array into the coordinate planes), and the interaction lists of the batches are
// traversed on several threads; the proxy slots are then numbered in batch order, in
// the order of first use, so the lists do not depend on the thread count.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <thread>
#include <utility>
#include <vector>

namespace stokes {
namespace tree {

constexpr int BATCH = 64;   // targets per batch

struct Cluster {
    double lo[3], hi[3], c[3], r;
    int64_t start, count;
    int32_t first_child, n_child;
};

struct Batch {
    double c[3], r;
    int64_t start;
    int32_t count;
};

// A point of the bisections: its coordinates and its index in the input.
struct Pt {
    double x[3];
    int64_t i;
};

inline std::vector<Pt> points_of(const std::vector<double>& xyz, int64_t n) {
    std::vector<Pt> p((size_t)n);
    for (int64_t k = 0; k < n; ++k) p[k] = Pt{{xyz[k], xyz[n + k], xyz[2 * n + k]}, k};
    return p;
}

// Octree-like midpoint splits: every dimension whose extent is at least half the
// largest is halved (a stable partition, points at the midpoint going low), until a
// cluster holds at most `leaf` points.  perm[k] = input index of sorted point k;
// clusters numbered as a stack walk creates them (cluster 0 the root; a split cluster's
// children get consecutive numbers when it is taken from the stack, and the last child
// is taken first), so a cluster's children are contiguous.
//
// With n_threads > 1 the subtrees below the first few levels are split on separate
// threads (each into its own list, numbered the same way from its root) and the whole
// tree is then numbered by the same walk, so the result does not depend on the thread
// count.
namespace detail {
// Bounds of points [start, start + count) and their split into groups (empty when
// the cluster is a leaf).
inline Cluster bound(std::vector<Pt>& p, int64_t start, int64_t count) {
    Cluster C{};
    C.start = start;
    C.count = count;
    for (int d = 0; d < 3; ++d) {
        C.lo[d] = INFINITY;
        C.hi[d] = -INFINITY;
    }
    for (int64_t k = start; k < start + count; ++k)
        for (int d = 0; d < 3; ++d) {
            C.lo[d] = std::min(C.lo[d], p[k].x[d]);
            C.hi[d] = std::max(C.hi[d], p[k].x[d]);
        }
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        C.c[d] = 0.5 * (C.lo[d] + C.hi[d]);
        r2 += 0.25 * (C.hi[d] - C.lo[d]) * (C.hi[d] - C.lo[d]);
    }
    C.r = sqrt(r2);
    C.first_child = -1;
    C.n_child = 0;
    return C;
}
// The split of cluster C: each dimension whose extent is at least half the largest is
// halved at its midpoint (points at the midpoint go low).  One stable counting pass by
// the code of the halves (x, then y, then z, each 0 low / 1 high over the halved
// dimensions) orders the points as successive stable partitions by x, y and z would;
// the non-empty codes, in order, are the groups (none when C is a leaf or would not
// split).  tmp: scratch of the points' size, the cluster's range [start, start +
// count) of it used (so clusters of disjoint ranges may split at once).
inline void split(std::vector<Pt>& p, const Cluster& C, int leaf, std::vector<std::pair<int64_t, int64_t>>& groups,
                  std::vector<Pt>& tmp) {
    groups.clear();
    double emax = 0.0;
    for (int d = 0; d < 3; ++d) emax = std::max(emax, C.hi[d] - C.lo[d]);
    if (C.count <= leaf || emax == 0.0) return;
    // a dimension that is not halved gets an infinite midpoint: every point goes low
    double mid[3];
    for (int d = 0; d < 3; ++d) mid[d] = (C.hi[d] - C.lo[d] < 0.5 * emax) ? INFINITY : C.c[d];
    const double m0 = mid[0], m1 = mid[1], m2 = mid[2];
    auto code = [m0, m1, m2](const Pt& q) {
        return 4 * (int)(q.x[0] > m0) + 2 * (int)(q.x[1] > m1) + (int)(q.x[2] > m2);
    };
    int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t s0 = C.start, s1 = C.start + C.count;
    for (int64_t k = s0; k < s1; ++k) ++cnt[code(p[k])];
    int64_t off[8], o = 0;
    for (int c = 0; c < 8; ++c) {
        off[c] = o;
        o += cnt[c];
    }
    for (int c = 0; c < 8; ++c) off[c] += s0;
    for (int64_t k = s0; k < s1; ++k) tmp[off[code(p[k])]++] = p[k];
    std::copy(tmp.begin() + s0, tmp.begin() + s1, p.begin() + s0);
    int64_t at = s0;
    for (int c = 0; c < 8; ++c) {
        if (cnt[c] > 0) groups.push_back({at, cnt[c]});
        at += cnt[c];
    }
    if (groups.size() < 2) groups.clear();
}
// The serial build of the subtree of points [start, start + count) into cl (root at
// cl[0]), stopping (no split) at clusters of depth >= cut, which it lists in `tasks`.
struct TaskRef {
    int32_t id;   // cluster number in cl
    int depth;
};
inline void build_from(std::vector<Pt>& p, std::vector<Pt>& tmp, int64_t start, int64_t count, int leaf, int cut,
                       std::vector<Cluster>& cl, std::vector<TaskRef>* tasks) {
    struct Item {
        int64_t start, count;
        int32_t self;
        int depth;
    };
    cl.clear();
    cl.push_back(Cluster{});
    std::vector<Item> stack{{start, count, 0, 0}};
    std::vector<std::pair<int64_t, int64_t>> groups;
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        cl[it.self] = bound(p, it.start, it.count);
        if (tasks && it.depth >= cut) {
            tasks->push_back({it.self, it.depth});
            continue;
        }
        split(p, cl[it.self], leaf, groups, tmp);
        if (groups.empty()) continue;
        const int32_t first = (int32_t)cl.size();
        cl[it.self].first_child = first;
        cl[it.self].n_child = (int32_t)groups.size();
        for (size_t g = 0; g < groups.size(); ++g) {
            cl.push_back(Cluster{});
            stack.push_back({groups[g].first, groups[g].second, first + (int32_t)g, it.depth + 1});
        }
    }
}
}  // namespace detail

inline void build_sources(const std::vector<double>& xyz, int64_t n, std::vector<int64_t>& perm,
                          std::vector<Cluster>& cl, int leaf, int n_threads = 1) {
    std::vector<Pt> p = points_of(xyz, n), tmp((size_t)n);
    int cut = 0;
    while (cut < 4 && (1 << (3 * cut)) < 4 * n_threads) ++cut;
    if (n_threads <= 1 || n <= 64 * (int64_t)leaf) {
        detail::build_from(p, tmp, 0, n, leaf, 0, cl, nullptr);
    } else {
        // the top levels, then each cluster at depth `cut` as a subtree of its own
        std::vector<Cluster> top;
        std::vector<detail::TaskRef> tasks;
        detail::build_from(p, tmp, 0, n, leaf, cut, top, &tasks);
        std::vector<std::vector<Cluster>> sub(tasks.size());
        const int T = std::max(1, std::min<int>(n_threads, (int)tasks.size()));
        auto run = [&](int t) {
            for (size_t k = (size_t)t; k < tasks.size(); k += (size_t)T) {
                const Cluster& R = top[tasks[k].id];
                detail::build_from(p, tmp, R.start, R.count, leaf, 0, sub[k], nullptr);
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back(run, t);
        run(0);
        for (auto& x : th) x.join();
        // number the whole tree by the serial walk: a node is (list, index), list -1 the
        // top tree, k >= 0 subtree k (whose root stands for top cluster tasks[k].id)
        std::vector<int32_t> task_of(top.size(), -1);
        for (size_t k = 0; k < tasks.size(); ++k) task_of[tasks[k].id] = (int32_t)k;
        struct Ref {
            int32_t list, idx;
        };
        auto node = [&](const Ref& r) -> const Cluster& { return r.list < 0 ? top[r.idx] : sub[r.list][r.idx]; };
        auto norm = [&](Ref r) {   // a top cluster cut off as a task is its subtree's root
            if (r.list < 0 && task_of[r.idx] >= 0) return Ref{task_of[r.idx], 0};
            return r;
        };
        cl.clear();
        cl.push_back(node(norm(Ref{-1, 0})));
        std::vector<std::pair<int32_t, Ref>> stack{{0, norm(Ref{-1, 0})}};
        while (!stack.empty()) {
            const auto e = stack.back();
            stack.pop_back();
            const Cluster& C = node(e.second);
            cl[e.first].first_child = -1;
            cl[e.first].n_child = 0;
            if (C.n_child == 0) continue;
            const int32_t first = (int32_t)cl.size();
            cl[e.first].first_child = first;
            cl[e.first].n_child = C.n_child;
            for (int32_t g = 0; g < C.n_child; ++g) {
                const Ref child = norm(Ref{e.second.list, C.first_child + g});
                cl.push_back(node(child));
                stack.push_back({first + g, child});
            }
        }
    }
    perm.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) perm[k] = p[k].i;
}

// Median splits along the longest extent down to at most BATCH targets per batch
// (the lower half takes floor(count / 2) points).  perm[k] = input index of sorted
// target k; batches in the order of a depth-first walk that takes the upper half
// first.  The splits below the first few levels run as independent subtrees on up
// to n_threads threads; their batch lists are joined in the walk's order, so the
// result does not depend on the thread count.
inline void build_batches(const std::vector<double>& xyz, int64_t n, std::vector<int64_t>& perm,
                          std::vector<Batch>& bt, int n_threads = 1) {
    std::vector<Pt> p = points_of(xyz, n);
    struct Node {
        int64_t start, count;
        int depth;
    };
    // one node: a batch (true) or a split into its two halves (pushed lower, upper)
    auto visit = [&p](const Node& g, std::vector<Node>& stack, std::vector<Batch>& out) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = g.start; k < g.start + g.count; ++k)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], p[k].x[d]);
                hi[d] = std::max(hi[d], p[k].x[d]);
            }
        if (g.count <= BATCH) {
            Batch B{};
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                B.c[d] = 0.5 * (lo[d] + hi[d]);
                r2 += 0.25 * (hi[d] - lo[d]) * (hi[d] - lo[d]);
            }
            B.r = sqrt(r2);
            B.start = g.start;
            B.count = (int32_t)g.count;
            out.push_back(B);
            return;
        }
        int dm = 0;
        for (int d = 1; d < 3; ++d)
            if (hi[d] - lo[d] > hi[dm] - lo[dm]) dm = d;
        const int64_t half = g.count / 2;
        auto b = p.begin() + g.start;
        std::nth_element(b, b + half, b + g.count, [dm](const Pt& u, const Pt& v) { return u.x[dm] < v.x[dm]; });
        stack.push_back({g.start, half, g.depth + 1});
        stack.push_back({g.start + half, g.count - half, g.depth + 1});
    };
    auto walk = [&visit](const Node& root, std::vector<Batch>& out) {
        std::vector<Node> stack{root};
        while (!stack.empty()) {
            const Node g = stack.back();
            stack.pop_back();
            visit(g, stack, out);
        }
    };
    bt.clear();
    // the first levels serially: nodes at depth `cut` become tasks, in walk order (a
    // task holds no batch yet: an entry of `order` with task >= 0)
    int cut = 0;
    while (cut < 6 && (1 << cut) < 4 * n_threads) ++cut;
    if (n_threads <= 1 || n <= 64 * BATCH) cut = 1 << 30;
    struct Entry {
        int task;
        Batch b;
    };
    std::vector<Entry> order;
    std::vector<Node> tasks;
    {
        // the nodes above depth `cut`, expanded level by level with the nodes of a level
        // on separate threads (they own disjoint ranges of p, so each sees what the
        // serial walk would show it), then walked in the serial walk's order (upper half
        // first) into batches and tasks
        struct Top {
            Node g;
            int kid = -1;        // first of its two children (lower, upper), or -1
            bool leaf = false;   // a batch
            Batch b{};
        };
        std::vector<Top> top{{Node{0, n, 0}}};
        std::vector<int> level{0};
        for (int depth = 0; depth < cut && !level.empty(); ++depth) {
            std::vector<std::vector<Node>> kids(level.size());
            auto expand = [&](size_t i) {
                std::vector<Node> stack;
                std::vector<Batch> one;
                visit(top[level[i]].g, stack, one);
                if (!one.empty()) {
                    top[level[i]].leaf = true;
                    top[level[i]].b = one[0];
                } else {
                    kids[i] = stack;             // lower, upper
                }
            };
            const int T = (int)std::max<int64_t>(1, std::min<int64_t>(n_threads, (int64_t)level.size()));
            if (T == 1) {
                for (size_t i = 0; i < level.size(); ++i) expand(i);
            } else {
                std::vector<std::thread> th;
                auto run = [&](int t) {
                    for (size_t i = (size_t)t; i < level.size(); i += (size_t)T) expand(i);
                };
                for (int t = 1; t < T; ++t) th.emplace_back(run, t);
                run(0);
                for (auto& x : th) x.join();
            }
            std::vector<int> next;
            for (size_t i = 0; i < level.size(); ++i) {
                if (kids[i].empty()) continue;
                top[level[i]].kid = (int)top.size();
                for (const Node& c : kids[i]) {
                    top.push_back({c});
                    if (c.depth < cut || c.count <= BATCH) next.push_back((int)top.size() - 1);
                }
            }
            level.swap(next);
        }
        std::vector<int> stack{0};
        while (!stack.empty()) {
            const Top& u = top[stack.back()];
            stack.pop_back();
            if (u.leaf) {
                order.push_back({-1, u.b});
            } else if (u.kid >= 0) {
                stack.push_back(u.kid);          // lower, then upper: the upper half is taken first
                stack.push_back(u.kid + 1);
            } else {
                order.push_back({(int)tasks.size(), Batch{}});
                tasks.push_back(u.g);
            }
        }
    }
    std::vector<std::vector<Batch>> res(tasks.size());
    if (!tasks.empty()) {
        const int T = std::max(1, std::min<int>(n_threads, (int)tasks.size()));
        std::vector<std::thread> th;
        auto run = [&](int t) {
            for (size_t k = (size_t)t; k < tasks.size(); k += (size_t)T) walk(tasks[k], res[k]);
        };
        for (int t = 1; t < T; ++t) th.emplace_back(run, t);
        run(0);
        for (auto& x : th) x.join();
    }
    for (const Entry& e : order) {
        if (e.task < 0)
            bt.push_back(e.b);
        else
            bt.insert(bt.end(), res[e.task].begin(), res[e.task].end());
    }
    perm.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) perm[k] = p[k].i;
}

// Interaction lists.  Batch b takes clusters through their proxies (px_list[px_off[b]
// .. px_off[b + 1]), slots into `used`, numbered by first use in batch order) and sums
// source ranges directly (dr_start / dr_count[dr_off[b] .. dr_off[b + 1]), adjacent
// ranges of one batch merged).  A cluster C is far from batch B when r_B + r_C <
// theta |c_B - c_C|; it goes through proxies if also count > P, else directly; a near
// cluster recurses into its children, a near leaf is summed directly.
struct Lists {
    std::vector<int32_t> px_off, px_list, used, dr_off, dr_count;
    std::vector<int64_t> dr_start;
    int64_t pairs_px = 0, pairs_dir = 0;
};

inline void build_lists(const std::vector<Batch>& bt, const std::vector<Cluster>& cl, double theta, int P,
                        Lists& L, int n_threads) {
    const int64_t nb = (int64_t)bt.size();
    struct Part {   // one thread's batches: cluster ids and ranges, per-batch offsets
        std::vector<int32_t> px_cl, px_n, dr_n, dr_count;
        std::vector<int64_t> dr_start;
        int64_t pairs_px = 0, pairs_dir = 0;
    };
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(n_threads, (nb + 63) / 64));
    std::vector<Part> parts((size_t)T);
    auto work = [&](int t) {
        Part& W = parts[t];
        const int64_t b0 = nb * t / T, b1 = nb * (t + 1) / T;
        std::vector<int32_t> stack;
        for (int64_t b = b0; b < b1; ++b) {
            const Batch& B = bt[b];
            const size_t px0 = W.px_cl.size(), dr0 = W.dr_start.size();
            stack.assign(1, 0);
            while (!stack.empty()) {
                const int32_t ci = stack.back();
                stack.pop_back();
                const Cluster& C = cl[ci];
                const double dx = B.c[0] - C.c[0], dy = B.c[1] - C.c[1], dz = B.c[2] - C.c[2];
                const double dist = sqrt(dx * dx + dy * dy + dz * dz);
                const bool far = B.r + C.r < theta * dist;
                if (far && C.count > P) {
                    W.px_cl.push_back(ci);
                    W.pairs_px += (int64_t)B.count * P;
                } else if (C.n_child == 0 || far) {
                    if (W.dr_start.size() > dr0 && W.dr_start.back() + W.dr_count.back() == C.start &&
                        W.dr_count.back() + C.count < (1 << 30)) {
                        W.dr_count.back() += (int32_t)C.count;   // adjacent ranges merge
                    } else {
                        W.dr_start.push_back(C.start);
                        W.dr_count.push_back((int32_t)C.count);
                    }
                    W.pairs_dir += (int64_t)B.count * C.count;
                } else {
                    for (int32_t k = C.n_child - 1; k >= 0; --k) stack.push_back(C.first_child + k);
                }
            }
            W.px_n.push_back((int32_t)(W.px_cl.size() - px0));
            W.dr_n.push_back((int32_t)(W.dr_start.size() - dr0));
        }
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back(work, t);
        work(0);
        for (auto& x : th) x.join();
    }
    // merge in batch order; proxy slots by first use
    L = Lists{};
    L.px_off.assign(1, 0);
    L.dr_off.assign(1, 0);
    std::vector<int32_t> slot_of(cl.size(), -1);
    for (const Part& W : parts) {
        size_t pi = 0, di = 0;
        for (size_t b = 0; b < W.px_n.size(); ++b) {
            for (int32_t q = 0; q < W.px_n[b]; ++q, ++pi) {
                const int32_t ci = W.px_cl[pi];
                if (slot_of[ci] < 0) {
                    slot_of[ci] = (int32_t)L.used.size();
                    L.used.push_back(ci);
                }
                L.px_list.push_back(slot_of[ci]);
            }
            for (int32_t q = 0; q < W.dr_n[b]; ++q, ++di) {
                L.dr_start.push_back(W.dr_start[di]);
                L.dr_count.push_back(W.dr_count[di]);
            }
            L.px_off.push_back((int32_t)L.px_list.size());
            L.dr_off.push_back((int32_t)L.dr_start.size());
        }
        L.pairs_px += W.pairs_px;
        L.pairs_dir += W.pairs_dir;
    }
}

// Direct ranges longer than `most` sources cut into pieces of `most` (the last piece
// shorter), so that a batch's entries can be shared out evenly between the waves that
// evaluate it (merged neighbouring leaves can make one range hold a large part of a
// batch's direct work).  The pieces stay in order, sorted by start and disjoint.
inline void split_ranges(Lists& L, int32_t most) {
    std::vector<int32_t> off{0}, count;
    std::vector<int64_t> start;
    for (size_t b = 0; b + 1 < L.dr_off.size(); ++b) {
        for (int32_t e = L.dr_off[b]; e < L.dr_off[b + 1]; ++e)
            for (int32_t o = 0; o < L.dr_count[e]; o += most) {
                start.push_back(L.dr_start[e] + o);
                count.push_back(std::min(most, L.dr_count[e] - o));
            }
        off.push_back((int32_t)start.size());
    }
    L.dr_off.swap(off);
    L.dr_start.swap(start);
    L.dr_count.swap(count);
}

// Work parts of the batches' evaluation: each batch's entries (its proxy clusters, then
// its direct ranges) cut into S parts of about equal pair counts, a proxy cluster
// counting P pairs per target and a direct range its sources.  Part h of batch b takes
// entries [cut[b (S + 1) + h], cut[b (S + 1) + h + 1]).  Cut h is the first entry whose
// midpoint lies past h / S of the batch's cost, so a part costs at most 1 / S of it plus
// one entry, and the cuts for S / 2 parts are every other one of these.
inline std::vector<int32_t> part_cuts(const Lists& L, int P, int S) {
    const size_t nb = L.px_off.size() - 1;
    std::vector<int32_t> cut(nb * (S + 1));
    for (size_t b = 0; b < nb; ++b) {
        const int32_t pa = L.px_off[b], np = L.px_off[b + 1] - pa, da = L.dr_off[b], nd = L.dr_off[b + 1] - da;
        auto cost = [&](int32_t e) -> int64_t { return e < np ? P : L.dr_count[da + e - np]; };
        int64_t total = 0;
        for (int32_t e = 0; e < np + nd; ++e) total += cost(e);
        int32_t* cb = &cut[b * (S + 1)];
        cb[0] = 0;
        cb[S] = np + nd;
        int32_t e = 0;
        int64_t acc = 0;
        for (int h = 1; h < S; ++h) {
            const int64_t goal = total * h / S;
            while (e < np + nd && 2 * acc + cost(e) <= 2 * goal) acc += cost(e++);
            cb[h] = e;
        }
    }
    return cut;
}

// Threads for a plan over n points: one per 4,096 points, at most the host's cores
// and 16 (measured on 65,536 points: 16 threads 5.3 ms, 4 threads 5.7 ms).
inline int plan_threads(int64_t n) {
    const unsigned h = std::thread::hardware_concurrency();
    const int64_t by_size = std::max<int64_t>(1, n / 4096);
    return (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)(h ? h : 1u), by_size}));
}

}  // namespace tree
}  // namespace stokes
