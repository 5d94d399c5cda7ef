// Sheet-based level-of-detail hierarchy of the mesh edges (Section 5,
// Section 5.1), host C++.  This is the preprocessing step in front of the
// render path: it produces the per-edge level `e_level` that Eq. 1 compares
// with the user's `lod`.
//
//  1. Edges and faces are deduplicated by bucketing on their smallest vertex
//     id; every cell gets its 12 edge ids and, per local face, the cell on
//     the other side (-1 on the mesh boundary).
//  2. Sheets: the four topologically parallel edges of each cell are joined
//     in a union-find over edges; a sheet is a class of edges, its component
//     the cells holding them.  Sheets are numbered in order of first
//     appearance (cells in order, then the three edge directions).
//  3. Components are sorted cell lists; each cell knows the (at most three)
//     live components containing it, so one pass over a component's cells
//     and their six faces yields its boundary size and, for every other
//     component it touches, the number of boundary faces a merge would make
//     interior (the numerator of Eq. 5), the tangent faces and whether cells
//     are shared: everything the priority needs.
//  4. Pairs live in a binary heap ordered by class (adjacent, hybrid,
//     intersecting), then by the Eq. 5 weight compared exactly as a ratio of
//     integers, then by the two ids; entries of merged components are
//     dropped when they surface.  A merge scans only the new component.
//  5. The edges of the tangent faces of each merge disappear at the current
//     level; a merge opens the next level when its result has more than
//     twice the cells of the larger component of the merge that opened the
//     current level.  Singular edges follow the exceptions of Section 5.1.
//
// Bucketing, the sheet scans and the per-merge passes over large components
// run on a pool of host threads; the merge order itself is sequential.
#include <algorithm>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <new>
#include <queue>
#include <thread>
#include <vector>

#include "hexfc.h"

namespace {

constexpr int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                              {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
constexpr int kDirFirst[3] = {0, 1, 8};  // first local edge of each direction
constexpr int kDirEdges[3][4] = {{0, 2, 4, 6}, {1, 3, 5, 7}, {8, 9, 10, 11}};
constexpr int kFace[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
// local edges along the rim of each local face
constexpr int kFaceEdge[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 9, 4, 8}, {1, 10, 5, 9}, {2, 11, 6, 10}, {3, 8, 7, 11}};

enum : uint8_t { ADJACENT = 0, HYBRID = 1, INTERSECTING = 2 };

// A fixed set of worker threads for one build; run() hands every thread the
// same job and returns when all have finished it.
class Pool {
  public:
    explicit Pool(int n) : n_(std::max(n, 1)) {
        for (int t = 1; t < n_; ++t) th_.emplace_back([this, t] { loop(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        wake_.notify_all();
        for (auto &x : th_) x.join();
    }
    int size() const { return n_; }
    void run(const std::function<void(int)> &job) {
        if (n_ == 1) {
            job(0);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &job;
            pending_ = n_ - 1;
            ++gen_;
        }
        wake_.notify_all();
        job(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
    }

  private:
    void loop(int t) {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                wake_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                job = job_;
            }
            (*job)(t);
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable wake_, done_;
    const std::function<void(int)> *job_ = nullptr;
    uint64_t gen_ = 0;
    int pending_ = 0;
    bool stop_ = false;
};

// fn(lo, hi, thread) over [0, n), split evenly over the pool (one thread
// when n is small).
template <class F> void parallel_for(Pool &pool, int64_t n, F &&fn, int64_t min_split = 4096) {
    if (pool.size() == 1 || n < min_split) {
        fn((int64_t)0, n, 0);
        return;
    }
    const int nt = pool.size();
    pool.run([&](int t) { fn(n * t / nt, n * (t + 1) / nt, t); });
}

// Counting sort of `n` items by key in [0, nkeys): bucket starts and the
// items' payloads grouped by key.  item(i) returns {key, payload}.  The order
// inside a bucket depends on the thread schedule; every caller sorts its
// buckets.
template <class T, class Item>
void bucket(Pool &pool, int64_t n, int64_t nkeys, Item &&item, std::vector<int64_t> &start, std::vector<T> &out) {
    std::vector<uint32_t> cnt(nkeys, 0);
    parallel_for(pool, n, [&](int64_t i0, int64_t i1, int) {
        for (int64_t i = i0; i < i1; ++i) __atomic_fetch_add(&cnt[item(i).first], 1u, __ATOMIC_RELAXED);
    });
    start.assign(nkeys + 1, 0);
    for (int64_t k = 0; k < nkeys; ++k) start[k + 1] = start[k] + cnt[k];
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    out.resize(n);
    parallel_for(pool, n, [&](int64_t i0, int64_t i1, int) {
        for (int64_t i = i0; i < i1; ++i) {
            const auto kv = item(i);
            out[__atomic_fetch_add(&pos[kv.first], (int64_t)1, __ATOMIC_RELAXED)] = kv.second;
        }
    });
}

struct Mesh {
    int64_t C = 0, V = 0, E = 0;
    std::vector<uint32_t> eid;    // [12C] global edge id of each local edge
    std::vector<int32_t> nbr;     // [6C] cell across each local face, -1 on the boundary
    std::vector<uint32_t> val;    // [E] incident cells
    std::vector<uint8_t> bnd;     // [E] 1 if the edge lies on a boundary face
};

hexfc_status build_edges(Pool &pool, const int32_t *hex, Mesh &m) {
    const int64_t n = 12 * m.C;
    // bucket by the smaller end; payload (larger end << 32) | local edge slot
    std::vector<int64_t> start;
    std::vector<uint64_t> ent;
    bucket<uint64_t>(pool, n, m.V, [&](int64_t s) {
        const int64_t c = s / 12;
        const int e = (int)(s - 12 * c);
        const uint32_t a = (uint32_t)hex[8 * c + kEdge[e][0]], b = (uint32_t)hex[8 * c + kEdge[e][1]];
        return std::pair<uint32_t, uint64_t>(std::min(a, b), ((uint64_t)std::max(a, b) << 32) | (uint64_t)s);
    }, start, ent);
    std::vector<uint32_t> nuniq(m.V);
    parallel_for(pool, m.V, [&](int64_t v0, int64_t v1, int) {
        for (int64_t v = v0; v < v1; ++v) {
            uint64_t *b = ent.data() + start[v], *e = ent.data() + start[v + 1];
            std::sort(b, e);
            uint32_t u = 0;
            for (uint64_t *q = b; q < e; ++q) u += (q == b || (*q >> 32) != (q[-1] >> 32));
            nuniq[v] = u;
        }
    });
    std::vector<int64_t> ebase(m.V + 1, 0);
    for (int64_t v = 0; v < m.V; ++v) ebase[v + 1] = ebase[v] + nuniq[v];
    m.E = ebase[m.V];
    m.eid.assign(n, 0);
    m.val.assign(m.E, 0);
    parallel_for(pool, m.V, [&](int64_t v0, int64_t v1, int) {
        for (int64_t v = v0; v < v1; ++v) {
            int64_t id = ebase[v] - 1;
            for (int64_t q = start[v]; q < start[v + 1]; ++q) {
                if (q == start[v] || (ent[q] >> 32) != (ent[q - 1] >> 32)) ++id;
                m.eid[(uint32_t)ent[q]] = (uint32_t)id;
                ++m.val[id];
            }
        }
    });
    return HEXFC_OK;
}

struct FaceEnt {
    uint32_t r[3];  // the three larger corner ids, ascending
    uint32_t slot;  // 6 * cell + local face
    bool operator<(const FaceEnt &o) const {
        if (r[0] != o.r[0]) return r[0] < o.r[0];
        if (r[1] != o.r[1]) return r[1] < o.r[1];
        if (r[2] != o.r[2]) return r[2] < o.r[2];
        return slot < o.slot;
    }
    bool same(const FaceEnt &o) const { return r[0] == o.r[0] && r[1] == o.r[1] && r[2] == o.r[2]; }
};

hexfc_status build_faces(Pool &pool, const int32_t *hex, Mesh &m) {
    const int64_t n = 6 * m.C;
    // bucket by the smallest corner
    std::vector<int64_t> start;
    std::vector<FaceEnt> ent;
    bucket<FaceEnt>(pool, n, m.V, [&](int64_t s) {
        const int64_t c = s / 6;
        const int f = (int)(s - 6 * c);
        uint32_t q[4];
        for (int i = 0; i < 4; ++i) q[i] = (uint32_t)hex[8 * c + kFace[f][i]];
        std::sort(q, q + 4);
        FaceEnt fe;
        fe.r[0] = q[1];
        fe.r[1] = q[2];
        fe.r[2] = q[3];
        fe.slot = (uint32_t)s;
        return std::pair<uint32_t, FaceEnt>(q[0], fe);
    }, start, ent);
    m.nbr.assign(n, -1);
    std::vector<uint8_t> bad(pool.size(), 0);
    parallel_for(pool, m.V, [&](int64_t v0, int64_t v1, int t) {
        for (int64_t v = v0; v < v1; ++v) {
            FaceEnt *b = ent.data() + start[v], *e = ent.data() + start[v + 1];
            std::sort(b, e);
            for (FaceEnt *p = b; p < e;) {
                FaceEnt *r = p + 1;
                while (r < e && p->same(*r)) ++r;
                if (r - p == 2) {
                    m.nbr[p[0].slot] = (int32_t)(p[1].slot / 6);
                    m.nbr[p[1].slot] = (int32_t)(p[0].slot / 6);
                } else if (r - p > 2) {
                    bad[t] = 1;
                }
                p = r;
            }
        }
    });
    for (uint8_t x : bad)
        if (x) return HEXFC_EINVAL;  // a face shared by more than two cells
    m.bnd.assign(m.E, 0);
    parallel_for(pool, m.C, [&](int64_t c0, int64_t c1, int) {
        for (int64_t c = c0; c < c1; ++c)
            for (int f = 0; f < 6; ++f)
                if (m.nbr[6 * c + f] < 0)
                    for (int i = 0; i < 4; ++i)
                        __atomic_store_n(&m.bnd[m.eid[12 * c + kFaceEdge[f][i]]], (uint8_t)1, __ATOMIC_RELAXED);
    });
    return HEXFC_OK;
}

struct UnionFind {
    std::vector<uint32_t> p;
    explicit UnionFind(int64_t n) : p(n) {
        for (int64_t i = 0; i < n; ++i) p[i] = (uint32_t)i;
    }
    uint32_t find(uint32_t x) {
        while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
        }
        return x;
    }
    void join(uint32_t a, uint32_t b) {
        a = find(a);
        b = find(b);
        if (a < b) p[b] = a;
        else if (b < a) p[a] = b;
    }
};

// One heap entry: the pair (a, b), a < b, with its class and Eq. 5 weight
// m / D, D = (|dA| + |dB|) (|A| + |B|).
struct Pair {
    uint64_t D;
    uint32_t m;
    uint8_t cls;
    int32_t a, b;
};
bool better(const Pair &x, const Pair &y) {
    if (x.cls != y.cls) return x.cls < y.cls;
    const unsigned __int128 l = (unsigned __int128)x.m * y.D, r = (unsigned __int128)y.m * x.D;
    if (l != r) return l > r;
    if (x.a != y.a) return x.a < y.a;
    return x.b < y.b;
}
struct Worse {
    bool operator()(const Pair &x, const Pair &y) const { return better(y, x); }
};

struct Hierarchy {
    const Mesh &m;
    Pool &pool;
    std::vector<int32_t> cc;                  // [3C] live components of each cell, -1 padded
    std::vector<std::vector<int32_t>> cells;  // per component: sorted cell ids
    std::vector<int64_t> size, bsize;
    std::vector<uint8_t> alive;
    // per-thread scan scratch, dense over component ids
    struct Scratch {
        std::vector<uint32_t> mrg, tan;
        std::vector<uint8_t> shr, seen;
        std::vector<int32_t> touched;
        int64_t bsize = 0;
    };
    std::vector<Scratch> scr;

    Hierarchy(const Mesh &mesh, Pool &workers, int64_t ncomp_max) : m(mesh), pool(workers) {
        cc.assign(3 * m.C, -1);
        cells.resize(ncomp_max);
        size.assign(ncomp_max, 0);
        bsize.assign(ncomp_max, 0);
        alive.assign(ncomp_max, 0);
        scr.resize(pool.size());
        for (auto &s : scr) {
            s.mrg.assign(ncomp_max, 0);
            s.tan.assign(ncomp_max, 0);
            s.shr.assign(ncomp_max, 0);
            s.seen.assign(ncomp_max, 0);
        }
    }
    bool has(int64_t c, int32_t k) const {
        const int32_t *p = &cc[3 * c];
        return p[0] == k || p[1] == k || p[2] == k;
    }

    // Scan cells [lo, hi) of component k into s (see the file comment).  For
    // a face between c (in k) and b, and another component x: the face is on
    // the boundary of k or of x and interior to their union exactly when
    //  * b is in k: x holds one of c, b but not both;
    //  * b is not in k (a boundary face of k): x holds b; the face is then
    //    also tangent when x does not hold c.
    // Interior faces of k are taken from their smaller cell only.
    void scan_range(int32_t k, int64_t lo, int64_t hi, Scratch &s) {
        const std::vector<int32_t> &L = cells[k];
        auto touch = [&](int32_t x) {
            if (!s.seen[x]) {
                s.seen[x] = 1;
                s.touched.push_back(x);
            }
        };
        auto in = [](const int32_t *p, int32_t x) { return p[0] == x || p[1] == x || p[2] == x; };
        for (int64_t q = lo; q < hi; ++q) {
            const int32_t c = L[q];
            const int32_t *kc = &cc[3 * (int64_t)c];
            for (int i = 0; i < 3; ++i)
                if (kc[i] >= 0 && kc[i] != k) {
                    touch(kc[i]);
                    s.shr[kc[i]] = 1;
                }
            const int32_t *nb = &m.nbr[6 * (int64_t)c];
            for (int f = 0; f < 6; ++f) {
                const int32_t b = nb[f];
                if (b < 0) {
                    ++s.bsize;
                    continue;
                }
                const int32_t *kb = &cc[3 * (int64_t)b];
                if (in(kb, k)) {
                    if (b < c) continue;
                    for (int i = 0; i < 3; ++i) {
                        const int32_t x = kc[i];
                        if (x >= 0 && x != k && !in(kb, x)) {
                            touch(x);
                            ++s.mrg[x];
                        }
                    }
                    for (int i = 0; i < 3; ++i) {
                        const int32_t x = kb[i];
                        if (x >= 0 && x != k && !in(kc, x)) {
                            touch(x);
                            ++s.mrg[x];
                        }
                    }
                } else {
                    ++s.bsize;
                    for (int i = 0; i < 3; ++i) {
                        const int32_t x = kb[i];
                        if (x < 0) continue;
                        touch(x);
                        ++s.mrg[x];
                        if (!in(kc, x)) ++s.tan[x];
                    }
                }
            }
        }
    }

    // Run fn(t, lo, hi) over [0, n) on one thread, or on all when n is large.
    template <class F> void split(int64_t n, F &&fn) {
        parallel_for(pool, n, [&](int64_t lo, int64_t hi, int t) { fn(t, lo, hi); }, 16384);
    }

    // Cells shared by components sm and ot, and the tangent faces between
    // them (a cell of only sm against a cell of only ot), seen from sm.
    int64_t tangent_faces(int32_t sm, int32_t ot, std::vector<std::pair<int32_t, int>> &out) {
        const std::vector<int32_t> &L = cells[sm];
        std::vector<std::vector<std::pair<int32_t, int>>> part(scr.size());
        std::vector<int64_t> shared(scr.size(), 0);
        split((int64_t)L.size(), [&](int t, int64_t lo, int64_t hi) {
            for (int64_t q = lo; q < hi; ++q) {
                const int32_t c = L[q];
                if (has(c, ot)) {
                    ++shared[t];
                    continue;
                }
                for (int f = 0; f < 6; ++f) {
                    const int32_t b = m.nbr[6 * (int64_t)c + f];
                    if (b >= 0 && has(b, ot) && !has(b, sm)) part[t].emplace_back(c, f);
                }
            }
        });
        int64_t ns = 0;
        out.clear();
        for (size_t t = 0; t < part.size(); ++t) {
            ns += shared[t];
            out.insert(out.end(), part[t].begin(), part[t].end());
        }
        return ns;
    }

    // Replace a and b by k in the component lists of the given cells.
    void relabel(const std::vector<int32_t> &L, int32_t a, int32_t b, int32_t k) {
        split((int64_t)L.size(), [&](int, int64_t lo, int64_t hi) {
            for (int64_t q = lo; q < hi; ++q) {
                int32_t *p = &cc[3 * (int64_t)L[q]];
                int32_t keep[3] = {k, -1, -1};
                int n = 1;
                for (int i = 0; i < 3; ++i)
                    if (p[i] >= 0 && p[i] != a && p[i] != b) keep[n++] = p[i];
                p[0] = keep[0];
                p[1] = keep[1];
                p[2] = keep[2];
            }
        });
    }

    // Turn the statistics gathered in s for component k into pairs (without
    // their weight denominators) and clear s.  Only x > k when `upper_only`.
    void collect(int32_t k, Scratch &s, bool upper_only, std::vector<Pair> &out) {
        for (int32_t x : s.touched) {
            if (s.mrg[x] > 0 && (!upper_only || x > k)) {
                Pair p;
                p.a = std::min(k, x);
                p.b = std::max(k, x);
                p.m = s.mrg[x];
                p.cls = !s.shr[x] ? ADJACENT : (s.tan[x] ? HYBRID : INTERSECTING);
                p.D = 0;
                out.push_back(p);
            }
            s.mrg[x] = s.tan[x] = 0;
            s.shr[x] = s.seen[x] = 0;
        }
        s.touched.clear();
        s.bsize = 0;
    }
    void set_weight(Pair &p) const {
        p.D = (uint64_t)(bsize[p.a] + bsize[p.b]) * (uint64_t)(size[p.a] + size[p.b]);
    }

    // All sheets at once, several sheets per thread: boundary sizes and the
    // pairs (x > k) of every sheet.
    void scan_sheets(int32_t S, std::vector<Pair> &out) {
        std::vector<std::vector<Pair>> part(scr.size());
        int32_t next = 0;
        auto work = [&](int t) {
            for (;;) {
                const int32_t k = __atomic_fetch_add(&next, 1, __ATOMIC_RELAXED);
                if (k >= S) break;
                scan_range(k, 0, (int64_t)cells[k].size(), scr[t]);
                bsize[k] = scr[t].bsize;
                collect(k, scr[t], true, part[t]);
            }
        };
        if (S < 2) work(0);
        else pool.run(work);
        for (auto &v : part) out.insert(out.end(), v.begin(), v.end());
        for (Pair &p : out) set_weight(p);
    }

    // Scan the new component k (split over threads when large): its boundary
    // size and its pairs with every live component.
    void scan_new(int32_t k, std::vector<Pair> &out) {
        const int64_t n = (int64_t)cells[k].size();
        split(n, [&](int t, int64_t lo, int64_t hi) { scan_range(k, lo, hi, scr[t]); });
        {
            Scratch &s0 = scr[0];  // fold the other threads' statistics into thread 0's
            for (size_t t = 1; t < scr.size(); ++t) {
                Scratch &s = scr[t];
                s0.bsize += s.bsize;
                s.bsize = 0;
                for (int32_t x : s.touched) {
                    if (!s0.seen[x]) {
                        s0.seen[x] = 1;
                        s0.touched.push_back(x);
                    }
                    s0.mrg[x] += s.mrg[x];
                    s0.tan[x] += s.tan[x];
                    s0.shr[x] |= s.shr[x];
                    s.mrg[x] = s.tan[x] = 0;
                    s.shr[x] = s.seen[x] = 0;
                }
                s.touched.clear();
            }
        }
        bsize[k] = scr[0].bsize;
        const size_t first = out.size();
        collect(k, scr[0], false, out);
        for (size_t i = first; i < out.size(); ++i) set_weight(out[i]);
    }
};

}  // namespace

extern "C" hexfc_status hexfc_build_lod(const int32_t *hex, int64_t C, int64_t V, int32_t n_threads,
                                        uint8_t *cell_edge_level, hexfc_lod_info *info) {
    try {
        if (info) std::memset(info, 0, sizeof(*info));
        if (C < 0 || (C > 0 && (!hex || V <= 0))) return HEXFC_EINVAL;
        if (C == 0) return HEXFC_OK;
        if (V >= (int64_t(1) << 31) || 12 * C >= (int64_t(1) << 32) - 1) return HEXFC_ERANGE;
        for (int64_t c = 0; c < C; ++c) {
            for (int i = 0; i < 8; ++i) {
                if (hex[8 * c + i] < 0 || hex[8 * c + i] >= V) return HEXFC_ERANGE;
                for (int j = 0; j < i; ++j)
                    if (hex[8 * c + i] == hex[8 * c + j]) return HEXFC_EINVAL;
            }
        }
        int nt = n_threads > 0 ? n_threads : (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
        nt = std::min(nt, 256);

        Pool pool(nt);
        Mesh m;
        m.C = C;
        m.V = V;
        hexfc_status st = build_edges(pool, hex, m);
        if (st != HEXFC_OK) return st;
        st = build_faces(pool, hex, m);
        if (st != HEXFC_OK) return st;

        // sheets
        UnionFind uf(m.E);
        for (int64_t c = 0; c < C; ++c)
            for (int d = 0; d < 3; ++d)
                for (int i = 1; i < 4; ++i) uf.join(m.eid[12 * c + kDirEdges[d][0]], m.eid[12 * c + kDirEdges[d][i]]);
        std::vector<int32_t> sid(m.E, -1);
        std::vector<int32_t> cell_sheet(3 * C);
        int32_t S = 0;
        for (int64_t c = 0; c < C; ++c)
            for (int d = 0; d < 3; ++d) {
                const uint32_t r = uf.find(m.eid[12 * c + kDirFirst[d]]);
                if (sid[r] < 0) sid[r] = S++;
                cell_sheet[3 * c + d] = sid[r];
            }
        const int64_t ncomp = 2 * (int64_t)S;
        Hierarchy h(m, pool, ncomp);
        for (int64_t c = 0; c < C; ++c) {
            int32_t *p = &h.cc[3 * c];
            int n = 0;
            for (int d = 0; d < 3; ++d) {
                const int32_t s = cell_sheet[3 * c + d];
                if (s != p[0] && s != p[1] && s != p[2]) p[n++] = s;
            }
            for (int i = 0; i < n; ++i) h.cells[p[i]].push_back((int32_t)c);
        }
        for (int32_t s = 0; s < S; ++s) {
            h.size[s] = (int64_t)h.cells[s].size();
            h.alive[s] = 1;
        }
        std::vector<Pair> pairs;
        h.scan_sheets(S, pairs);
        std::priority_queue<Pair, std::vector<Pair>, Worse> heap(Worse(), std::move(pairs));

        // merging
        std::vector<uint8_t> hidden(m.E, 0);  // level at which the edge disappeared, 0 = never
        int64_t level = 0, ref = 0, merges[3] = {0, 0, 0};
        int32_t next = S, live = S;
        std::vector<std::pair<int32_t, int>> tangent;
        std::vector<int32_t> merged_cells;
        while (!heap.empty()) {
            const Pair p = heap.top();
            heap.pop();
            if (!h.alive[p.a] || !h.alive[p.b]) continue;
            const int32_t sm = h.size[p.a] <= h.size[p.b] ? p.a : p.b, ot = sm == p.a ? p.b : p.a;
            const int64_t shared = h.tangent_faces(sm, ot, tangent);
            const int64_t usize = h.size[p.a] + h.size[p.b] - shared;
            if (level == 0 || usize > 2 * ref) {
                ++level;
                ref = std::max(h.size[p.a], h.size[p.b]);
                if (level > 255) return HEXFC_ERANGE;
            }
            for (auto &tf : tangent)
                for (int i = 0; i < 4; ++i) {
                    uint8_t &hv = hidden[m.eid[12 * (int64_t)tf.first + kFaceEdge[tf.second][i]]];
                    if (!hv) hv = (uint8_t)level;
                }
            const int32_t k = next++;
            merged_cells.clear();
            merged_cells.reserve(usize);
            std::set_union(h.cells[p.a].begin(), h.cells[p.a].end(), h.cells[p.b].begin(), h.cells[p.b].end(),
                           std::back_inserter(merged_cells));
            h.relabel(merged_cells, p.a, p.b, k);
            h.cells[k].swap(merged_cells);
            merged_cells.clear();
            std::vector<int32_t>().swap(h.cells[p.a]);
            std::vector<int32_t>().swap(h.cells[p.b]);
            h.alive[p.a] = h.alive[p.b] = 0;
            h.alive[k] = 1;
            h.size[k] = usize;
            ++merges[p.cls];
            --live;
            pairs.clear();
            h.scan_new(k, pairs);
            for (const Pair &q : pairs) heap.push(q);
        }
        const int64_t L = level;
        int64_t nsing = 0;
        std::vector<uint8_t> lvl(m.E);
        for (int64_t e = 0; e < m.E; ++e) {
            const bool singular = m.val[e] != (m.bnd[e] ? 2u : 4u);
            nsing += singular;
            if (m.val[e] == 1) lvl[e] = (uint8_t)L;
            else if (singular) lvl[e] = (uint8_t)(hidden[e] ? L - 1 : L);
            else lvl[e] = (uint8_t)(hidden[e] ? hidden[e] - 1 : L);
        }
        if (cell_edge_level)
            for (int64_t s = 0; s < 12 * C; ++s) cell_edge_level[s] = lvl[m.eid[s]];
        if (info) {
            info->sheets = S;
            info->edges = m.E;
            int64_t nf = 0;
            for (int64_t s = 0; s < 6 * C; ++s) nf += m.nbr[s] < 0 || m.nbr[s] > s / 6;
            info->faces = nf;
            info->singular_edges = nsing;
            for (int i = 0; i < 3; ++i) info->merges[i] = merges[i];
            info->levels = (int32_t)L;
            info->components_left = live;
        }
        return HEXFC_OK;
    } catch (const std::bad_alloc &) {
        return HEXFC_ENOMEM;
    } catch (...) {
        return HEXFC_EINVAL;
    }
}
