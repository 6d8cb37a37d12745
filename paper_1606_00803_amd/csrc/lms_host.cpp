// Host side of the smoothing library: adjacency build, host quality,
// orderings (ORI / BFS / RDR / random), multicolour schedule and relabelling.
//
// Compiled with -ffp-contract=off: the vertex qualities RDR sorts by are
// computed with exactly the IEEE operations written here, so any other code
// performing the same operations in the same order gets the same bits.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <exception>
#include <limits>
#include <numeric>
#include <thread>

#include <sched.h>

#include "lms_internal.hpp"

namespace lms {

void fail(lms_status code, const std::string &msg) { throw Error{code, msg}; }

namespace {

template <class T>
void resize_or_fail(std::vector<T> &v, size_t n) {
    try {
        v.assign(n, T());
    } catch (const std::bad_alloc &) {
        fail(LMS_ERR_ALLOC, "host allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
}


// CPUs this process may run on (its affinity mask), at least 1.
int host_cpus() {
    cpu_set_t set;
    CPU_ZERO(&set);
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        const int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    const unsigned hw = std::thread::hardware_concurrency();
    return hw == 0 ? 1 : int(hw);
}

int host_threads(int64_t work_items) {
    const int64_t t = std::min<int64_t>(std::min<int64_t>(host_cpus(), 16), std::max<int64_t>(1, work_items / 64));
    return int(std::max<int64_t>(1, t));
}

// Runs f(worker, first, last) over [0, items) split into contiguous runs,
// one thread each; rethrows the first exception.  When a thread cannot be
// started (a process or thread limit), the runs left over execute on the
// calling thread after the started ones, so the result is the same.
template <class F>
void parallel_runs(int64_t items, int workers, F f) {
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(static_cast<size_t>(workers));
    auto run = [&](int w) {
        const int64_t first = items * w / workers, last = items * (w + 1) / workers;
        try {
            f(w, first, last);
        } catch (...) {
            err[size_t(w)] = std::current_exception();
        }
    };
    int started = 0;
    try {
        th.reserve(size_t(workers));
        for (; started < workers; ++started) th.emplace_back(run, started);
    } catch (...) {
        // the std::thread of run `started` was never created
    }
    for (int w = started; w < workers; ++w) run(w);
    for (auto &t : th) t.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

}  // namespace

// Neighbours of Eq. 1: for every vertex, the distinct vertices sharing a
// triangle edge with it.  An edge seen in exactly one triangle is a boundary
// edge and fixes both endpoints (unless the caller gave a mask).
void build_mesh(Mesh &M, int32_t n, int64_t T, const int32_t *tri, const uint8_t *fixed,
                int32_t n_mesh, const int64_t *v_off, const int64_t *t_off) {
    if (n <= 0) fail(LMS_ERR_ARG, "n must be positive");
    if (T <= 0) fail(LMS_ERR_ARG, "n_tri must be positive");
    if (T > (int64_t(1) << 40)) fail(LMS_ERR_ARG, "n_tri too large (more than 2^40 triangles)");
    if (!tri) fail(LMS_ERR_ARG, "tri is NULL");
    M.n = n;
    M.T = T;
    M.n_mesh = n_mesh;
    M.v_off.assign(v_off, v_off + n_mesh + 1);
    M.t_off.assign(t_off, t_off + n_mesh + 1);

    resize_or_fail(M.tri0, size_t(3 * T));
    for (int32_t i = 0; i < n_mesh; ++i) {
        const int64_t vb = v_off[i], ve = v_off[i + 1];
        const int64_t nv = ve - vb;
        for (int64_t t = t_off[i]; t < t_off[i + 1]; ++t) {
            for (int c = 0; c < 3; ++c) {
                const int64_t v = tri[3 * t + c];
                if (v < 0 || v >= nv)
                    fail(LMS_ERR_MESH, "triangle " + std::to_string(t) + " refers to vertex " +
                                           std::to_string(v) + " outside [0, " + std::to_string(nv) + ")");
                M.tri0[3 * t + c] = int32_t(v + vb);
            }
            const int32_t *p = &M.tri0[3 * t];
            if (p[0] == p[1] || p[1] == p[2] || p[0] == p[2])
                fail(LMS_ERR_MESH, "triangle " + std::to_string(t) + " repeats a vertex");
        }
    }

    // triangles per vertex, and vertex -> triangle incidence (counting sort,
    // ascending triangle index within each vertex)
    resize_or_fail(M.tcount0, size_t(n));
    for (int64_t i = 0; i < 3 * T; ++i) M.tcount0[M.tri0[i]]++;
    for (int32_t v = 0; v < n; ++v)
        if (M.tcount0[v] == 0) fail(LMS_ERR_MESH, "vertex " + std::to_string(v) + " is not referenced by any triangle");
    resize_or_fail(M.vt_ptr0, size_t(n) + 1);
    for (int32_t v = 0; v < n; ++v) M.vt_ptr0[v + 1] = M.vt_ptr0[v] + M.tcount0[v];
    resize_or_fail(M.vt0, size_t(3 * T));
    {
        std::vector<int64_t> fill(M.vt_ptr0.begin(), M.vt_ptr0.end() - 1);
        for (int64_t t = 0; t < T; ++t)
            for (int c = 0; c < 3; ++c) M.vt0[fill[M.tri0[3 * t + c]]++] = int32_t(t);
    }

    // unique neighbours with edge multiplicities
    resize_or_fail(M.adj_ptr0, size_t(n) + 1);
    resize_or_fail(M.fixed0, size_t(n));
    std::vector<int32_t> buf;
    std::vector<int32_t> tmp;
    try {
        tmp.reserve(size_t(6 * T));
    } catch (const std::bad_alloc &) {
        fail(LMS_ERR_ALLOC, "host allocation for the adjacency failed");
    }
    for (int32_t v = 0; v < n; ++v) {
        buf.clear();
        for (int64_t i = M.vt_ptr0[v]; i < M.vt_ptr0[v + 1]; ++i) {
            const int32_t *p = &M.tri0[3 * int64_t(M.vt0[i])];
            for (int c = 0; c < 3; ++c)
                if (p[c] != v) buf.push_back(p[c]);
        }
        std::sort(buf.begin(), buf.end());
        bool on_boundary = false;
        for (size_t a = 0; a < buf.size();) {
            size_t b = a;
            while (b < buf.size() && buf[b] == buf[a]) ++b;
            const size_t mult = b - a;
            if (mult > 2)
                fail(LMS_ERR_MESH, "edge (" + std::to_string(v) + ", " + std::to_string(buf[a]) +
                                       ") is shared by more than two triangles");
            if (mult == 1) on_boundary = true;
            tmp.push_back(buf[a]);
            a = b;
        }
        M.adj_ptr0[v + 1] = int64_t(tmp.size());
        M.fixed0[v] = fixed ? uint8_t(fixed[v] != 0) : uint8_t(on_boundary);
    }
    M.adj0.swap(tmp);

    M.n_free = 0;
    M.max_degree = 0;
    int64_t nnz = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (M.fixed0[v]) continue;
        const int64_t d = M.adj_ptr0[v + 1] - M.adj_ptr0[v];
        if (d == 0) fail(LMS_ERR_MESH, "free vertex " + std::to_string(v) + " has no neighbours");
        M.n_free++;
        M.max_degree = std::max<int32_t>(M.max_degree, int32_t(d));
        nnz += d;
    }
    if (nnz >= (int64_t(1) << 31)) fail(LMS_ERR_ARG, "smoothing adjacency exceeds 2^31 entries");

    // Multicolour schedule: greedy first-fit over the graph induced on free
    // vertices, in ascending input label, smallest colour not taken by an
    // already coloured free neighbour.
    resize_or_fail(M.color0, size_t(n));
    std::fill(M.color0.begin(), M.color0.end(), -1);
    std::vector<int32_t> seen_at;  // seen_at[c] == v: colour c taken around v
    M.n_colors = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (M.fixed0[v]) continue;
        for (int64_t j = M.adj_ptr0[v]; j < M.adj_ptr0[v + 1]; ++j) {
            const int32_t c = M.color0[M.adj0[j]];
            if (c >= 0) {
                if (size_t(c) >= seen_at.size()) seen_at.resize(size_t(c) + 1, -1);
                seen_at[c] = v;
            }
        }
        int32_t c = 0;
        while (size_t(c) < seen_at.size() && seen_at[c] == v) ++c;
        M.color0[v] = c;
        M.n_colors = std::max(M.n_colors, c + 1);
    }

    std::vector<int32_t> ident(static_cast<size_t>(n));
    std::iota(ident.begin(), ident.end(), 0);
    relabel(M, LMS_ORI, std::move(ident));
}

// Section 3.2: triangle quality = shortest / longest Euclidean edge length
// (0 when the longest edge has length 0); vertex quality = mean over its
// triangles, summed in ascending triangle index.
void vertex_quality_host(const Mesh &M, const double *x, const double *y, double *q) {
    std::vector<double> qt(static_cast<size_t>(M.T));
    parallel_runs(M.T, host_threads(M.T / 1024), [&](int, int64_t first, int64_t last) {
        for (int64_t t = first; t < last; ++t) {
            const int32_t a = M.tri0[3 * t], b = M.tri0[3 * t + 1], c = M.tri0[3 * t + 2];
            double dx, dy;
            dx = x[b] - x[a];
            dy = y[b] - y[a];
            const double e0 = dx * dx + dy * dy;
            dx = x[c] - x[b];
            dy = y[c] - y[b];
            const double e1 = dx * dx + dy * dy;
            dx = x[a] - x[c];
            dy = y[a] - y[c];
            const double e2 = dx * dx + dy * dy;
            const double mn = std::min(std::min(e0, e1), e2);
            const double mx = std::max(std::max(e0, e1), e2);
            qt[size_t(t)] = mx > 0.0 ? std::sqrt(mn) / std::sqrt(mx) : 0.0;
        }
    });
    parallel_runs(M.n, host_threads(M.n / 1024), [&](int, int64_t first, int64_t last) {
        for (int64_t v = first; v < last; ++v) {
            double s = 0.0;
            for (int64_t i = M.vt_ptr0[size_t(v)]; i < M.vt_ptr0[size_t(v) + 1]; ++i) s += qt[size_t(M.vt0[size_t(i)])];
            q[v] = s / double(M.tcount0[size_t(v)]);
        }
    });
}

// Breadth-first search from label 0, neighbours in ascending label, restart
// at the smallest unvisited label.  Meshes of a batch are separate
// components in label order, so each one is ordered within its own range.
std::vector<int32_t> order_bfs(const Mesh &M) {
    std::vector<int32_t> out;
    out.reserve(size_t(M.n));
    std::vector<uint8_t> seen(size_t(M.n), 0);
    std::vector<int32_t> queue(size_t(M.n));
    for (int32_t s = 0; s < M.n; ++s) {
        if (seen[s]) continue;
        size_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = 1;
        while (head < tail) {
            const int32_t v = queue[head++];
            out.push_back(v);
            for (int64_t j = M.adj_ptr0[v]; j < M.adj_ptr0[v + 1]; ++j) {
                const int32_t u = M.adj0[j];
                if (!seen[u]) {
                    seen[u] = 1;
                    queue[tail++] = u;
                }
            }
        }
    }
    return out;
}

// Algorithm 2 (RDR), per mesh.  Vertices are compared by (quality, label).
// Starting from each not-yet-processed interior vertex in that order, the
// vertex is placed if it is not yet; then repeatedly: the unprocessed
// neighbours of the current vertex are taken in (quality, label) order, the
// ones not yet placed are appended, and the walk moves to the first of them
// (the worst-quality unprocessed neighbour), marking it processed.  The same
// loop then continues over the fixed vertices, which places the ones the
// interior loop never reaches (Theorem 1 misses a fixed vertex whose
// neighbours are all fixed and never walked onto).
namespace {

// A vertex and its quality; RDR's order is ascending (q, label).
struct QV {
    double q;
    int32_t v;
};
inline bool qv_less(const QV &a, const QV &b) { return a.q < b.q || (a.q == b.q && a.v < b.v); }

// Sort by (q, label): sorted runs on several threads, then rounds of pairwise
// merges.  Keys are distinct (labels are), so the result is the sorted order.
void parallel_sort_qv(std::vector<QV> &a) {
    const int64_t n = int64_t(a.size());
    const int P = host_threads(n / 4096);
    if (P <= 1) {
        std::sort(a.begin(), a.end(), qv_less);
        return;
    }
    std::vector<int64_t> bound(size_t(P) + 1);
    for (int i = 0; i <= P; ++i) bound[size_t(i)] = n * i / P;
    parallel_runs(P, P, [&](int, int64_t first, int64_t last) {
        for (int64_t r = first; r < last; ++r)
            std::sort(a.begin() + bound[size_t(r)], a.begin() + bound[size_t(r) + 1], qv_less);
    });
    std::vector<QV> tmp(a.size());
    for (int64_t width = 1; width < P; width *= 2) {
        std::vector<std::array<int64_t, 3>> jobs;
        for (int64_t i = 0; i < P; i += 2 * width)
            jobs.push_back({bound[size_t(i)], bound[size_t(std::min<int64_t>(i + width, P))],
                            bound[size_t(std::min<int64_t>(i + 2 * width, P))]});
        parallel_runs(int64_t(jobs.size()), int(jobs.size()), [&](int, int64_t first, int64_t last) {
            for (int64_t j = first; j < last; ++j) {
                const auto &[lo, mid, hi] = jobs[size_t(j)];
                std::merge(a.begin() + lo, a.begin() + mid, a.begin() + mid, a.begin() + hi, tmp.begin() + lo, qv_less);
            }
        });
        a.swap(tmp);
    }
}

}  // namespace

std::vector<int32_t> order_rdr(const Mesh &M, const double *q) {
    std::vector<int32_t> out;
    out.reserve(size_t(M.n));
    std::vector<uint8_t> processed(size_t(M.n), 0), placed(size_t(M.n), 0);
    std::vector<QV> cur;
    auto place = [&](int32_t v) {
        if (!placed[v]) {
            placed[v] = 1;
            out.push_back(v);
        }
    };
    // l of Algorithm 2: the unprocessed neighbours of w by increasing (q, label)
    auto unprocessed_neighbours = [&](int32_t w) {
        cur.clear();
        for (int64_t j = M.adj_ptr0[w]; j < M.adj_ptr0[w + 1]; ++j) {
            const int32_t u = M.adj0[j];
            if (!processed[u]) cur.push_back(QV{q[u], u});
        }
        std::sort(cur.begin(), cur.end(), qv_less);
    };
    auto start_from = [&](int32_t i) {
        if (processed[i]) return;
        place(i);
        processed[i] = 1;
        unprocessed_neighbours(i);
        while (!cur.empty()) {
            for (const QV &u : cur) place(u.v);
            const int32_t w = cur[0].v;
            processed[w] = 1;
            unprocessed_neighbours(w);
        }
    };
    std::vector<QV> seeds;
    for (int32_t mi = 0; mi < M.n_mesh; ++mi) {
        const int32_t vb = int32_t(M.v_off[mi]), ve = int32_t(M.v_off[mi + 1]);
        for (int pass = 0; pass < 2; ++pass) {
            seeds.clear();
            for (int32_t v = vb; v < ve; ++v)
                if ((M.fixed0[v] != 0) == (pass == 1)) seeds.push_back(QV{q[v], v});
            parallel_sort_qv(seeds);
            for (const QV &i : seeds) start_from(i.v);
        }
    }
    return out;
}

namespace {
// SplitMix64 (Steele, Lea, Flood 2014): Weyl sequence plus a mixing function.
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};
}  // namespace

// Fisher-Yates from the identity: for i = size-1 down to 1, swap element i
// with element next() mod (i+1).  Mesh i of a batch uses seed + i.
std::vector<int32_t> order_random(const Mesh &M, uint64_t seed) {
    std::vector<int32_t> out(static_cast<size_t>(M.n));
    for (int32_t mi = 0; mi < M.n_mesh; ++mi) {
        const int64_t vb = M.v_off[mi], ve = M.v_off[mi + 1];
        int32_t *p = out.data() + vb;
        const int64_t sz = ve - vb;
        for (int64_t i = 0; i < sz; ++i) p[i] = int32_t(vb + i);
        SplitMix64 g{seed + uint64_t(mi)};
        for (int64_t i = sz - 1; i >= 1; --i) {
            const uint64_t j = g.next() % uint64_t(i + 1);
            std::swap(p[i], p[j]);
        }
    }
    return out;
}

// Apply an ordering: rebuild every current-label array from the input ones.
// Triangles are relabelled and sorted by (smallest new vertex id, input
// index), which keeps the quality pass's gathers local under any ordering.
void relabel(Mesh &M, lms_ordering kind, std::vector<int32_t> new2old) {
    const int32_t n = M.n;
    std::vector<int32_t> old2new(static_cast<size_t>(n), -1);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t v = new2old[k];
        if (v < 0 || v >= n || old2new[v] != -1) fail(LMS_ERR_ARG, "ordering is not a permutation");
        old2new[v] = k;
    }
    std::vector<int32_t> row_ptr(size_t(n) + 1), col;
    std::vector<uint8_t> fx(static_cast<size_t>(n));
    std::vector<int32_t> color(static_cast<size_t>(n));
    int64_t nnz = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t v = new2old[k];
        fx[k] = M.fixed0[v];
        color[k] = M.color0[v];
        if (!fx[k]) nnz += M.adj_ptr0[v + 1] - M.adj_ptr0[v];
        row_ptr[k + 1] = int32_t(nnz);
    }
    resize_or_fail(col, size_t(nnz));
    // every row below is filled from the input arrays alone: rows, entries
    // and triangles split over threads give the same arrays
    const int row_workers = host_threads(n / 256);
    parallel_runs(n, row_workers, [&](int, int64_t first, int64_t last) {
        for (int64_t k = first; k < last; ++k) {
            if (fx[size_t(k)]) continue;
            const int32_t v = new2old[size_t(k)];
            int32_t *dst = col.data() + row_ptr[size_t(k)];
            int64_t d = 0;
            for (int64_t j = M.adj_ptr0[v]; j < M.adj_ptr0[v + 1]; ++j) dst[d++] = old2new[M.adj0[j]];
            std::sort(dst, dst + d);
        }
    });

    // padded copy of the smoothing adjacency for the offset-free sweep
    // variants, row-major (entry k of row v at ell[v*W + k], -1 past the
    // row's end): width 8, 12 or 16, the smallest that holds every row
    int32_t ell_w = 0;
    std::vector<int32_t> ell;
    if (M.max_degree <= 16) {
        ell_w = M.max_degree <= 8 ? 8 : (M.max_degree <= 12 ? 12 : 16);
        resize_or_fail(ell, size_t(ell_w) * size_t(n));
        parallel_runs(n, row_workers, [&](int, int64_t first, int64_t last) {
            std::fill(ell.begin() + first * ell_w, ell.begin() + last * ell_w, -1);
            for (int64_t k = first; k < last; ++k)
                for (int32_t j = row_ptr[size_t(k)]; j < row_ptr[size_t(k) + 1]; ++j)
                    ell[size_t(k) * size_t(ell_w) + size_t(j - row_ptr[size_t(k)])] = col[size_t(j)];
        });
    }

    // triangles: counting sort by smallest new id, stable in input index
    const int64_t T = M.T;
    std::vector<int64_t> bucket(size_t(n) + 1, 0);
    std::vector<int32_t> key(static_cast<size_t>(T));
    const int tri_workers = host_threads(T / 256);
    parallel_runs(T, tri_workers, [&](int, int64_t first, int64_t last) {
        for (int64_t t = first; t < last; ++t) {
            const int32_t a = old2new[M.tri0[3 * t]], b = old2new[M.tri0[3 * t + 1]], c = old2new[M.tri0[3 * t + 2]];
            key[size_t(t)] = std::min(a, std::min(b, c));
        }
    });
    for (int64_t t = 0; t < T; ++t) bucket[key[size_t(t)] + 1]++;
    for (int32_t k = 0; k < n; ++k) bucket[k + 1] += bucket[k];
    std::vector<int64_t> torder(static_cast<size_t>(T));
    for (int64_t t = 0; t < T; ++t) torder[bucket[key[t]]++] = t;
    std::vector<int32_t> ta(static_cast<size_t>(T)), tb(static_cast<size_t>(T)), tc(static_cast<size_t>(T)),
        tmesh(static_cast<size_t>(T));
    std::vector<double> tw(static_cast<size_t>(T));
    parallel_runs(T, tri_workers, [&](int, int64_t first, int64_t last) {
        for (int64_t i = first; i < last; ++i) {
            const int64_t t = torder[size_t(i)];
            const int32_t a = M.tri0[3 * t], b = M.tri0[3 * t + 1], c = M.tri0[3 * t + 2];
            ta[size_t(i)] = old2new[a];
            tb[size_t(i)] = old2new[b];
            tc[size_t(i)] = old2new[c];
            // weight of q_t in the global mean: (1/|V|) sum over its corners
            // of 1/|T(v)| (the 1/|V| is applied after the sum)
            tw[size_t(i)] = 1.0 / double(M.tcount0[a]) + 1.0 / double(M.tcount0[b]) + 1.0 / double(M.tcount0[c]);
            // mesh index: meshes own contiguous triangle ranges in input order
            tmesh[size_t(i)] = int32_t(std::upper_bound(M.t_off.begin(), M.t_off.end(), t) - M.t_off.begin() - 1);
        }
    });
    // packed 16-byte triangle record for the quality pass: the corners and the
    // three triangle counts, from which the pass recomputes w_t exactly as above
    std::vector<int32_t> trec;
    {
        bool small = true;
        for (int32_t v = 0; v < n && small; ++v) small = M.tcount0[v] <= 1023;
        if (small) {
            resize_or_fail(trec, size_t(4) * size_t(T));
            parallel_runs(T, tri_workers, [&](int, int64_t first, int64_t last) {
                for (int64_t i = first; i < last; ++i) {
                    const int64_t t = torder[size_t(i)];
                    const int32_t a = M.tri0[3 * t], b = M.tri0[3 * t + 1], c = M.tri0[3 * t + 2];
                    trec[size_t(4 * i)] = ta[size_t(i)];
                    trec[size_t(4 * i + 1)] = tb[size_t(i)];
                    trec[size_t(4 * i + 2)] = tc[size_t(i)];
                    trec[size_t(4 * i + 3)] = M.tcount0[a] | (M.tcount0[b] << 10) | (M.tcount0[c] << 20);
                }
            });
        }
    }
    std::vector<int32_t> vt_ptr(size_t(n) + 1, 0), vt(static_cast<size_t>(3 * T));
    for (int64_t i = 0; i < T; ++i) {
        vt_ptr[ta[i] + 1]++;
        vt_ptr[tb[i] + 1]++;
        vt_ptr[tc[i] + 1]++;
    }
    for (int32_t k = 0; k < n; ++k) vt_ptr[k + 1] += vt_ptr[k];
    {
        std::vector<int32_t> fill(vt_ptr.begin(), vt_ptr.end() - 1);
        for (int64_t i = 0; i < T; ++i) {
            vt[fill[ta[i]]++] = int32_t(i);
            vt[fill[tb[i]]++] = int32_t(i);
            vt[fill[tc[i]]++] = int32_t(i);
        }
    }

    adopt_relabel(M, kind, std::move(new2old), std::move(old2new), std::move(row_ptr), std::move(col), ell_w,
                  std::move(ell), std::move(fx), std::move(color), std::move(ta), std::move(tb), std::move(tc),
                  std::move(tw), std::move(trec), std::move(tmesh), std::move(vt_ptr), std::move(vt));
}

void adopt_relabel(Mesh &M, lms_ordering kind, std::vector<int32_t> new2old, std::vector<int32_t> old2new,
                   std::vector<int32_t> row_ptr, std::vector<int32_t> col, int32_t ell_w, std::vector<int32_t> ell,
                   std::vector<uint8_t> fx, std::vector<int32_t> color, std::vector<int32_t> ta,
                   std::vector<int32_t> tb, std::vector<int32_t> tc, std::vector<double> tw,
                   std::vector<int32_t> trec, std::vector<int32_t> tmesh, std::vector<int32_t> vt_ptr,
                   std::vector<int32_t> vt) {
    const int32_t n = M.n;
    std::vector<int32_t> color_ptr(size_t(M.n_colors) + 1, 0), color_list;
    for (int32_t k = 0; k < n; ++k)
        if (color[k] >= 0) color_ptr[color[k] + 1]++;
    for (int32_t c = 0; c < M.n_colors; ++c) color_ptr[c + 1] += color_ptr[c];
    color_list.resize(size_t(color_ptr[M.n_colors]));
    {
        std::vector<int32_t> fill(color_ptr.begin(), color_ptr.end() - 1);
        for (int32_t k = 0; k < n; ++k)
            if (color[k] >= 0) color_list[fill[color[k]]++] = k;
    }

    // colour-major padded copy for the multicolour sweep: one coalesced index
    // load per entry for the vertices of one colour
    std::vector<int32_t> color_ell;
    if (ell_w > 0) {
        resize_or_fail(color_ell, size_t(ell_w) * color_list.size());
        std::fill(color_ell.begin(), color_ell.end(), -1);
        for (int32_t c = 0; c < M.n_colors; ++c) {
            const int64_t base = int64_t(ell_w) * color_ptr[c], cnt = color_ptr[c + 1] - color_ptr[c];
            parallel_runs(cnt, host_threads(cnt / 256), [&](int, int64_t first, int64_t last) {
                for (int64_t i = first; i < last; ++i) {
                    const int32_t k = color_list[size_t(color_ptr[c] + i)];
                    for (int32_t j = row_ptr[k]; j < row_ptr[k + 1]; ++j)
                        color_ell[size_t(base + int64_t(j - row_ptr[k]) * cnt + i)] = col[size_t(j)];
                }
            });
        }
    }

    M.halo_plans.clear();
    M.tb_plans.clear();
    M.mc_plans.clear();
    M.patch_sets.clear();
    M.ordering = kind;
    M.new2old = std::move(new2old);
    M.old2new = std::move(old2new);
    M.row_ptr = std::move(row_ptr);
    M.col = std::move(col);
    M.ell_w = ell_w;
    M.ell = std::move(ell);
    M.fixed = std::move(fx);
    M.color = std::move(color);
    M.color_ptr = std::move(color_ptr);
    M.color_list = std::move(color_list);
    M.color_ell = std::move(color_ell);
    M.ta = std::move(ta);
    M.tb = std::move(tb);
    M.tc = std::move(tc);
    M.tw = std::move(tw);
    M.trec = std::move(trec);
    M.tmesh = std::move(tmesh);
    M.vt_ptr = std::move(vt_ptr);
    M.vt = std::move(vt);
    M.version++;
}

// Tile plan of the halo-staged sweep for tile size ts (see HaloPlan).  The
// entries keep the row's ascending neighbour order, so the staged sweep adds
// neighbours in the same order as every other variant.
const Mesh::HaloPlan &halo_plan(Mesh &M, int32_t ts) {
    for (const auto &h : M.halo_plans)
        if (h.ts == ts && h.version == M.version) return h;
    if (M.ell_w <= 0) fail(LMS_ERR_STATE, "no padded adjacency for a halo plan");
    Mesh::HaloPlan H;
    H.ts = ts;
    const int32_t n = M.n, W = M.ell_w;
    const int64_t tiles = (int64_t(n) + ts - 1) / ts;
    H.halo_ptr.assign(size_t(tiles) + 1, 0);
    resize_or_fail(H.lidx, size_t(tiles) * size_t(W) * size_t(ts));
    std::fill(H.lidx.begin(), H.lidx.end(), uint16_t(0xFFFF));
    std::vector<int32_t> outside;
    for (int64_t t = 0; t < tiles; ++t) {
        const int32_t b = int32_t(t * ts), e = int32_t(std::min<int64_t>(int64_t(n), (t + 1) * int64_t(ts)));
        outside.clear();
        for (int32_t j = M.row_ptr[b]; j < M.row_ptr[e]; ++j)
            if (M.col[j] < b || M.col[j] >= e) outside.push_back(M.col[j]);
        std::sort(outside.begin(), outside.end());
        outside.erase(std::unique(outside.begin(), outside.end()), outside.end());
        if (int64_t(ts) + int64_t(outside.size()) > 0xFFFF) fail(LMS_ERR_STATE, "tile halo too large for 16-bit slots");
        H.h_max = std::max<int32_t>(H.h_max, int32_t(outside.size()));
        uint16_t *lt = H.lidx.data() + size_t(t) * size_t(W) * size_t(ts);
        for (int32_t v = b; v < e; ++v)
            for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                const int32_t u = M.col[j];
                int32_t slot;
                if (u >= b && u < e) {
                    slot = u - b;
                } else {
                    slot = ts + int32_t(std::lower_bound(outside.begin(), outside.end(), u) - outside.begin());
                }
                lt[size_t(v - b) * size_t(W) + size_t(j - M.row_ptr[v])] = uint16_t(slot);
            }
        H.halo.insert(H.halo.end(), outside.begin(), outside.end());
        if (H.halo.size() >= (size_t(1) << 31)) fail(LMS_ERR_STATE, "halo lists exceed 2^31 entries");
        H.halo_ptr[size_t(t) + 1] = int32_t(H.halo.size());
    }
    // self-check: every slot names the CSR neighbour it stands for and lies
    // inside the tile's staging area (own rows + its halo)
    for (int64_t t = 0; t < tiles; ++t) {
        const int32_t b = int32_t(t * ts), e = int32_t(std::min<int64_t>(int64_t(n), (t + 1) * int64_t(ts)));
        const int32_t hb = H.halo_ptr[size_t(t)], hn = H.halo_ptr[size_t(t) + 1] - hb;
        const uint16_t *lt = H.lidx.data() + size_t(t) * size_t(W) * size_t(ts);
        for (int32_t r = 0; r < ts; ++r) {
            const int32_t v = b + r;
            const int32_t deg = v < e ? M.row_ptr[v + 1] - M.row_ptr[v] : 0;
            for (int32_t k = 0; k < W; ++k) {
                const uint16_t slot = lt[size_t(r) * size_t(W) + size_t(k)];
                if (k >= deg) {
                    if (slot != 0xFFFF) fail(LMS_ERR_STATE, "halo plan: padding slot in use");
                    continue;
                }
                if (slot >= ts + hn) fail(LMS_ERR_STATE, "halo plan: slot outside the staging area");
                const int32_t u = slot < ts ? b + slot : H.halo[size_t(hb + slot - ts)];
                if (u != M.col[size_t(M.row_ptr[v] + k)]) fail(LMS_ERR_STATE, "halo plan: slot names the wrong vertex");
            }
        }
    }
    H.version = M.version;
    M.halo_plans.push_back(std::move(H));
    return M.halo_plans.back();
}

namespace {

// Open-addressing map vertex id -> local slot for one tile at a time; clear()
// empties only the entries the last tile used.
class SlotMap {
   public:
    explicit SlotMap(size_t want) {
        size_t cap = 16;
        while (cap < 2 * want) cap *= 2;
        keys_.assign(cap, -1);
        vals_.assign(cap, 0);
        mask_ = cap - 1;
    }
    // inserts (v, slot) unless v is present; true when inserted
    bool insert(int32_t v, int32_t slot) {
        size_t h = hash(v);
        while (keys_[h] != -1) {
            if (keys_[h] == v) return false;
            h = (h + 1) & mask_;
        }
        keys_[h] = v;
        vals_[h] = slot;
        used_.push_back(h);
        return true;
    }
    bool contains(int32_t v) const { return find(v) != npos; }
    void set(int32_t v, int32_t slot) { vals_[find(v)] = slot; }
    int32_t get(int32_t v) const {
        const size_t h = find(v);
        return h == npos ? -1 : vals_[h];
    }
    void clear() {
        for (size_t h : used_) keys_[h] = -1;
        used_.clear();
    }

   private:
    static constexpr size_t npos = ~size_t(0);
    size_t hash(int32_t v) const { return size_t((uint32_t(v) * 2654435761u) >> 7) & mask_; }
    size_t find(int32_t v) const {
        size_t h = hash(v);
        while (keys_[h] != -1) {
            if (keys_[h] == v) return h;
            h = (h + 1) & mask_;
        }
        return npos;
    }
    std::vector<int32_t> keys_, vals_;
    std::vector<size_t> used_;
    size_t mask_ = 0;
};

// A temporal-blocking plan is given up (the variant is unusable) once the
// tiles built so far (at least a sixteenth of the rows, over all workers)
// stage more than this many rows per own row: sweeping the halo rings would
// cost far more than it saves (a random ordering stages dozens; RDR about 3
// at depth 2).
constexpr int64_t kTBMaxStagedPerRow = 6;

// The tiles one worker builds for a run of nominal tiles.
struct TBPart {
    bool fits = true;
    std::vector<int32_t> tile_end, ring, halo, halo_n, lidx_rows;
    std::vector<uint16_t> lidx;
    int32_t l_max = 0, u_max = 0;
};

}  // namespace

// Patches: from a seed, take up to ts free rows not yet taken, in
// breadth-first order over the adjacency.  The next seed is the first row,
// in the order found, that borders a finished patch and is still free, so
// patches grow outwards from those before them and leave few fragments
// behind them whatever the labels; a component with no such row starts at
// its lowest free label.  A patch may reach rows of any label, which
// gathers the scattered end of an ordering into the patches around it.
// Cached per tile size until the plans are dropped.
const Mesh::Patches &patch_set(Mesh &M, int32_t ts) {
    for (const auto &q : M.patch_sets)
        if (q.ts == ts && q.version == M.version) return q;
    const int32_t n = M.n;
    Mesh::Patches q;
    q.ts = ts;
    q.patch_ptr.assign(1, 0);
    resize_or_fail(q.patch_rows, size_t(M.n_free));
    q.patch_rows.clear();
    std::vector<uint8_t> taken(size_t(n), 0), queued(size_t(n), 0);
    std::vector<int32_t> grow, border;  // border holds each row once at most
    size_t border_head = 0;
    int32_t lowest = 0;
    auto free_row = [&](int32_t v) { return !M.fixed[size_t(v)] && !taken[size_t(v)]; };
    for (;;) {
        int32_t seed = -1;
        while (border_head < border.size()) {
            const int32_t c = border[border_head++];
            if (free_row(c)) {
                seed = c;
                break;
            }
        }
        if (seed < 0) {
            while (lowest < n && !free_row(lowest)) ++lowest;
            if (lowest == n) break;
            seed = lowest;
        }
        grow.assign(1, seed);
        taken[size_t(seed)] = 1;
        for (size_t h = 0; h < grow.size() && h < size_t(ts); ++h) {
            const int32_t v = grow[h];
            for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                const int32_t u = M.col[size_t(j)];
                if (free_row(u)) {
                    taken[size_t(u)] = 1;
                    grow.push_back(u);
                }
            }
        }
        for (size_t i = size_t(ts); i < grow.size(); ++i) taken[size_t(grow[i])] = 0;  // give the rest back
        grow.resize(std::min(grow.size(), size_t(ts)));
        for (const int32_t v : grow)
            for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                const int32_t u = M.col[size_t(j)];
                if (free_row(u) && !queued[size_t(u)]) {
                    queued[size_t(u)] = 1;
                    border.push_back(u);
                }
            }
        q.patch_rows.insert(q.patch_rows.end(), grow.begin(), grow.end());
        q.patch_ptr.push_back(int64_t(q.patch_rows.size()));
    }
    q.version = M.version;
    M.patch_sets.push_back(std::move(q));
    return M.patch_sets.back();
}

const Mesh::TBPlan &tb_plan(Mesh &M, int32_t ts, int32_t k, int32_t u_cap, int32_t l_cap, bool patches) {
    for (const auto &h : M.tb_plans)
        if (h.ts == ts && h.k == k && h.u_cap == u_cap && h.l_cap == l_cap && h.patches == patches &&
            h.version == M.version)
            return h;
    if (M.ell_w <= 0) fail(LMS_ERR_STATE, "no padded adjacency for a temporal-blocking plan");
    if (ts <= 0 || k < 1 || k > 8 || u_cap < 1 || l_cap < u_cap || l_cap >= 0xFFFF)
        fail(LMS_ERR_ARG, "temporal-blocking plan: bad tile size, depth or caps");
    const int32_t n = M.n, W = M.ell_w;
    const int64_t nominal = (int64_t(n) + ts - 1) / ts;
    static const Mesh::Patches no_patches{0, 0, std::vector<int64_t>(1, 0), {}};
    const Mesh::Patches &ps = patches ? patch_set(M, ts) : no_patches;
    const std::vector<int64_t> &patch_ptr = ps.patch_ptr;
    const std::vector<int32_t> &patch_rows = ps.patch_rows;
    const int64_t items = patches ? int64_t(patch_ptr.size()) - 1 : nominal;
    const int workers = host_threads(items);
    std::vector<TBPart> parts(static_cast<size_t>(workers));
    std::atomic<bool> give_up{false};
    std::atomic<int64_t> all_own{0}, all_staged{0};
    const int64_t sample = std::max<int64_t>(4096, int64_t(n) / 16);
    parallel_runs(items, workers, [&](int w, int64_t first, int64_t last) {
        TBPart &out = parts[size_t(w)];
        SlotMap slots(size_t(l_cap) + size_t(W) + 1);
        std::vector<int32_t> local;
        int32_t rc[9];
        // Stage the own rows (ascending) and k rings; false as soon as a cap
        // is exceeded.
        auto try_tile = [&](const int32_t *own, int32_t nown) {
            slots.clear();
            local.clear();
            for (int32_t i = 0; i < nown; ++i) {
                slots.insert(own[i], i);
                local.push_back(own[i]);
            }
            rc[0] = nown;
            if (rc[0] > l_cap) return false;
            size_t from = 0;  // first local row of the ring being expanded
            for (int32_t m = 1; m <= k; ++m) {
                const size_t to = local.size();
                for (size_t i = from; i < to; ++i) {
                    const int32_t v = local[i];
                    for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                        const int32_t u = M.col[size_t(j)];
                        if (slots.insert(u, -1)) local.push_back(u);
                    }
                    if (local.size() > size_t(l_cap)) return false;
                }
                std::sort(local.begin() + std::ptrdiff_t(to), local.end());
                for (size_t i = to; i < local.size(); ++i) slots.set(local[i], int32_t(i));
                rc[m] = int32_t(local.size());
                from = to;
            }
            return rc[k - 1] <= u_cap;
        };
        auto emit_tile = [&]() {
            const int32_t nown = rc[0];
            out.tile_end.push_back(patches ? nown : local[size_t(nown) - 1] + 1);
            out.ring.insert(out.ring.end(), rc, rc + k + 1);
            out.l_max = std::max(out.l_max, rc[k]);
            out.u_max = std::max(out.u_max, rc[k - 1]);
            out.halo.insert(out.halo.end(), local.begin() + (patches ? 0 : nown), local.end());
            out.halo_n.push_back(patches ? rc[k] : rc[k] - rc[0]);
            const size_t rows = size_t(rc[k - 1]);
            const size_t base = out.lidx.size();
            out.lidx.resize(base + rows * size_t(W), uint16_t(0xFFFF));
            for (size_t i = 0; i < rows; ++i) {
                const int32_t v = local[i];
                uint16_t *row = out.lidx.data() + base + i * size_t(W);
                for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                    const int32_t s = slots.get(M.col[size_t(j)]);
                    if (s < 0) fail(LMS_ERR_STATE, "temporal-blocking plan: neighbour not staged");
                    row[j - M.row_ptr[v]] = uint16_t(s);
                }
            }
            out.lidx_rows.push_back(int32_t(rows));
        };
        // count the tile; false (and give up everywhere) once the staged rows
        // per own row exceed the limit
        auto account = [&]() {
            const int64_t own = all_own.fetch_add(rc[0]) + rc[0];
            const int64_t staged = all_staged.fetch_add(rc[k]) + rc[k];
            if (own > sample && staged > kTBMaxStagedPerRow * own) {
                out.fits = false;
                give_up.store(true, std::memory_order_relaxed);
                return false;
            }
            return true;
        };
        auto fail_here = [&]() {
            out.fits = false;
            give_up.store(true, std::memory_order_relaxed);
        };
        if (!patches) {
            std::vector<std::pair<int32_t, int32_t>> todo;
            std::vector<int32_t> own;
            for (int64_t t = first; t < last && out.fits; ++t) {
                if (give_up.load(std::memory_order_relaxed)) {
                    out.fits = false;
                    break;
                }
                todo.emplace_back(int32_t(t * ts), int32_t(std::min<int64_t>(n, (t + 1) * ts)));
                while (!todo.empty()) {
                    const auto [b, e] = todo.back();
                    todo.pop_back();
                    own.resize(size_t(e - b));
                    for (int32_t v = b; v < e; ++v) own[size_t(v - b)] = v;
                    if (try_tile(own.data(), e - b)) {
                        emit_tile();
                        if (!account()) break;
                    } else if (e - b > 1) {  // halve; the left half goes first
                        const int32_t mid = b + (e - b) / 2;
                        todo.emplace_back(mid, e);
                        todo.emplace_back(b, mid);
                    } else {
                        fail_here();
                        break;
                    }
                }
            }
        } else {
            // each patch; while a cap is exceeded, split it into the first
            // and second half of its breadth-first order (the first half is a
            // smaller ball around the seed), first half first
            std::vector<std::pair<int64_t, int64_t>> todo;
            std::vector<int32_t> own;
            for (int64_t t = first; t < last && out.fits; ++t) {
                if (give_up.load(std::memory_order_relaxed)) {
                    out.fits = false;
                    break;
                }
                todo.emplace_back(patch_ptr[size_t(t)], patch_ptr[size_t(t) + 1]);
                while (!todo.empty()) {
                    const auto [b, e] = todo.back();
                    todo.pop_back();
                    own.assign(patch_rows.begin() + std::ptrdiff_t(b), patch_rows.begin() + std::ptrdiff_t(e));
                    std::sort(own.begin(), own.end());
                    if (try_tile(own.data(), int32_t(e - b))) {
                        emit_tile();
                        if (!account()) break;
                    } else if (e - b > 1) {
                        const int64_t mid = b + (e - b) / 2;
                        todo.emplace_back(mid, e);
                        todo.emplace_back(b, mid);
                    } else {
                        fail_here();
                        break;
                    }
                }
            }
        }
    });
    Mesh::TBPlan P;
    P.ts = ts;
    P.k = k;
    P.u_cap = u_cap;
    P.l_cap = l_cap;
    P.patches = patches;
    for (const auto &q : parts) P.fits = P.fits && q.fits;
    if (P.fits) {
        size_t tiles = 0, halo = 0, lidx = 0;
        for (const auto &q : parts) {
            tiles += q.tile_end.size();
            halo += q.halo.size();
            lidx += q.lidx.size();
        }
        if (tiles >= size_t(std::numeric_limits<int32_t>::max())) fail(LMS_ERR_STATE, "too many tiles");
        P.tiles = int32_t(tiles);
        P.tile_ptr.reserve(tiles + 1);
        P.halo_ptr.reserve(tiles + 1);
        P.lidx_ptr.reserve(tiles + 1);
        resize_or_fail(P.halo, halo);
        resize_or_fail(P.lidx, lidx);
        P.ring.reserve(tiles * size_t(k + 1));
        P.tile_ptr.push_back(0);
        P.halo_ptr.push_back(0);
        P.lidx_ptr.push_back(0);
        size_t ho = 0, lo = 0;
        for (auto &q : parts) {
            P.l_max = std::max(P.l_max, q.l_max);
            P.u_max = std::max(P.u_max, q.u_max);
            P.ring.insert(P.ring.end(), q.ring.begin(), q.ring.end());
            for (size_t t = 0; t < q.tile_end.size(); ++t) {
                P.tile_ptr.push_back(patches ? P.tile_ptr.back() + q.tile_end[t] : q.tile_end[t]);
                P.halo_ptr.push_back(P.halo_ptr.back() + q.halo_n[t]);
                P.lidx_ptr.push_back(P.lidx_ptr.back() + q.lidx_rows[t]);
            }
            std::copy(q.halo.begin(), q.halo.end(), P.halo.begin() + std::ptrdiff_t(ho));
            std::copy(q.lidx.begin(), q.lidx.end(), P.lidx.begin() + std::ptrdiff_t(lo));
            ho += q.halo.size();
            lo += q.lidx.size();
            q = TBPart{};
        }
        // self-check: tiles cover the rows in order (patches: every free row
        // once); each updated row's slots name its CSR neighbours in order,
        // inside the rows valid one sweep earlier (own + one more ring)
        if (P.tile_ptr.back() != (patches ? M.n_free : n))
            fail(LMS_ERR_STATE, "temporal-blocking plan: tiles do not cover the rows");
        if (patches) {
            std::vector<uint8_t> seen(size_t(n), 0);
            for (int32_t t = 0; t < P.tiles; ++t)
                for (int32_t i = 0; i < P.tile_ptr[size_t(t) + 1] - P.tile_ptr[size_t(t)]; ++i) {
                    const int32_t v = P.halo[size_t(P.halo_ptr[size_t(t)] + i)];
                    if (v < 0 || v >= n || M.fixed[size_t(v)] || seen[size_t(v)] ||
                        (i > 0 && v <= P.halo[size_t(P.halo_ptr[size_t(t)] + i - 1)]))
                        fail(LMS_ERR_STATE, "temporal-blocking plan: patch rows");
                    seen[size_t(v)] = 1;
                }
        }
        parallel_runs(P.tiles, host_threads(P.tiles), [&](int, int64_t first, int64_t last) {
            for (int64_t t = first; t < last; ++t) {
                const int32_t b = P.tile_ptr[size_t(t)], e = P.tile_ptr[size_t(t) + 1];
                const int32_t *r = P.ring.data() + size_t(t) * size_t(k + 1);
                const int64_t hb = P.halo_ptr[size_t(t)];
                if (e <= b || r[0] != e - b || r[k] > l_cap || r[k - 1] > u_cap ||
                    P.halo_ptr[size_t(t) + 1] - hb != int64_t(patches ? r[k] : r[k] - r[0]) ||
                    P.lidx_ptr[size_t(t) + 1] - P.lidx_ptr[size_t(t)] != int64_t(r[k - 1]))
                    fail(LMS_ERR_STATE, "temporal-blocking plan: tile counts");
                auto global_of = [&](int32_t li) {
                    if (patches) return P.halo[size_t(hb + li)];
                    return li < e - b ? b + li : P.halo[size_t(hb + li - (e - b))];
                };
                for (int32_t m = 0; m < k; ++m)
                    for (int32_t li = m == 0 ? 0 : r[m - 1]; li < r[m]; ++li) {
                        const int32_t v = global_of(li);
                        const uint16_t *row = P.lidx.data() + size_t(P.lidx_ptr[size_t(t)] + li) * size_t(W);
                        const int32_t deg = M.row_ptr[v + 1] - M.row_ptr[v];
                        for (int32_t q = 0; q < W; ++q) {
                            if (q >= deg) {
                                if (row[q] != 0xFFFF) fail(LMS_ERR_STATE, "temporal-blocking plan: padding slot in use");
                                continue;
                            }
                            if (row[q] >= r[m + 1]) fail(LMS_ERR_STATE, "temporal-blocking plan: slot outside its ring");
                            if (global_of(row[q]) != M.col[size_t(M.row_ptr[v] + q)])
                                fail(LMS_ERR_STATE, "temporal-blocking plan: slot names the wrong vertex");
                        }
                    }
            }
        });
    }
    P.version = M.version;
    M.tb_plans.push_back(std::move(P));
    return M.tb_plans.back();
}

namespace {

// Triangle records of a tile plan for the quality evaluated inside the sweep
// passes.  Every triangle with a free corner belongs to the tile owning its
// smallest free corner (tile_of(v)); slot_of(tile, v) gives a staged corner's
// slot (every corner is staged: the others are neighbours of that free corner).
// Records, four words each: slots a | b<<16, slot c, then the triangle's
// weight w_t (the double the quality pass uses, low word first).  Triangles
// with all corners fixed are listed apart with their weights.  False when a
// slot does not fit 16 bits.
template <class TileOf, class SlotOf>
bool tile_quality_records(const Mesh &M, int32_t tiles, TileOf tile_of, SlotOf slot_of,
                          std::vector<int64_t> &qtri_ptr, std::vector<uint32_t> &qtri, std::vector<int32_t> &qc_ids,
                          std::vector<double> &qc_w) {
    const int64_t T = M.T;
    std::vector<int32_t> owner(size_t(T), -1);
    std::vector<uint32_t> rec(size_t(4) * size_t(T), 0u);
    std::atomic<bool> fits{true};
    parallel_runs(T, host_threads(T / 256), [&](int, int64_t first, int64_t last) {
        for (int64_t t = first; t < last; ++t) {
            const int32_t c3[3] = {M.ta[size_t(t)], M.tb[size_t(t)], M.tc[size_t(t)]};
            int32_t own = -1;
            for (int32_t v : c3)
                if (!M.fixed[size_t(v)] && (own < 0 || v < own)) own = v;
            if (own < 0) continue;
            const int32_t tile = tile_of(own);
            uint32_t slot[3];
            for (int q = 0; q < 3; ++q) {
                const int32_t sl = slot_of(tile, c3[q]);
                if (sl < 0) fail(LMS_ERR_STATE, "quality plan: corner not staged");
                if (sl > 0xFFFF) fits = false;
                slot[q] = uint32_t(sl) & 0xFFFFu;
            }
            owner[size_t(t)] = tile;
            uint32_t wbits[2];
            std::memcpy(wbits, &M.tw[size_t(t)], sizeof(double));
            rec[size_t(4 * t)] = slot[0] | (slot[1] << 16);
            rec[size_t(4 * t + 1)] = slot[2];
            rec[size_t(4 * t + 2)] = wbits[0];
            rec[size_t(4 * t + 3)] = wbits[1];
        }
    });
    if (!fits) return false;
    // group by tile (stable: ascending triangle index inside a tile)
    qtri_ptr.assign(size_t(tiles) + 1, 0);
    qc_ids.clear();
    qc_w.clear();
    for (int64_t t = 0; t < T; ++t) {
        if (owner[size_t(t)] >= 0) {
            qtri_ptr[size_t(owner[size_t(t)]) + 1]++;
        } else {
            qc_ids.insert(qc_ids.end(), {M.ta[size_t(t)], M.tb[size_t(t)], M.tc[size_t(t)]});
            qc_w.push_back(M.tw[size_t(t)]);
        }
    }
    for (int32_t i = 0; i < tiles; ++i) qtri_ptr[size_t(i) + 1] += qtri_ptr[size_t(i)];
    resize_or_fail(qtri, size_t(4) * size_t(qtri_ptr.back()));
    std::vector<int64_t> fill(qtri_ptr.begin(), qtri_ptr.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
        const int32_t o = owner[size_t(t)];
        if (o < 0) continue;
        const int64_t at = fill[size_t(o)]++;
        for (int q = 0; q < 4; ++q) qtri[size_t(4 * at + q)] = rec[size_t(4 * t + q)];
    }
    if (qtri_ptr.back() + int64_t(qc_w.size()) != T) fail(LMS_ERR_STATE, "quality plan: triangle count");
    return true;
}

// A record's slots lie below `staged` and its weight is positive and finite.
bool quality_record_ok(const uint32_t *w, uint32_t staged) {
    double wt;
    std::memcpy(&wt, w + 2, sizeof(double));
    return (w[0] & 0xFFFFu) < staged && (w[0] >> 16) < staged && w[1] < staged && wt > 0.0 && std::isfinite(wt);
}

}  // namespace

void tb_quality_plan(const Mesh &M, Mesh::TBPlan &P) {
    if (P.q_built) return;
    if (!P.fits || P.version != M.version) fail(LMS_ERR_STATE, "quality plan of a stale or unusable tile plan");
    const int32_t k = P.k;
    P.q_built = true;
    // a corner outside the own rows sits in ring 1; both lists are ascending
    auto find = [](const int32_t *a, int32_t len, int32_t v) -> int32_t {
        const int32_t *it = std::lower_bound(a, a + len, v);
        return it == a + len || *it != v ? -1 : int32_t(it - a);
    };
    std::vector<int32_t> row_tile;
    if (P.patches) {
        row_tile.assign(size_t(M.n), -1);
        for (int32_t t = 0; t < P.tiles; ++t)
            for (int64_t i = P.halo_ptr[size_t(t)]; i < P.halo_ptr[size_t(t)] + P.ring[size_t(t) * size_t(k + 1)]; ++i)
                row_tile[size_t(P.halo[size_t(i)])] = t;
    }
    auto tile_of = [&](int32_t v) -> int32_t {
        if (P.patches) return row_tile[size_t(v)];
        return int32_t(std::upper_bound(P.tile_ptr.begin(), P.tile_ptr.end(), v) - P.tile_ptr.begin()) - 1;
    };
    auto slot_of = [&](int32_t tile, int32_t v) -> int32_t {
        const int32_t *r = P.ring.data() + size_t(tile) * size_t(k + 1);
        const int32_t *h = P.halo.data() + P.halo_ptr[size_t(tile)];
        if (P.patches) {
            const int32_t i = find(h, r[0], v);
            if (i >= 0) return i;
            const int32_t j = find(h + r[0], r[1] - r[0], v);
            return j < 0 ? -1 : r[0] + j;
        }
        const int32_t b = P.tile_ptr[size_t(tile)], e = P.tile_ptr[size_t(tile) + 1];
        if (v >= b && v < e) return v - b;
        const int32_t j = find(h, r[1] - r[0], v);
        return j < 0 ? -1 : r[0] + j;
    };
    P.q_fits = tile_quality_records(M, P.tiles, tile_of, slot_of, P.qtri_ptr, P.qtri, P.qc_ids, P.qc_w);
    if (!P.q_fits) return;
    // self-check: slots inside own + ring 1, weights positive and finite
    for (int32_t i = 0; i < P.tiles; ++i) {
        const int32_t *r = P.ring.data() + size_t(i) * size_t(k + 1);
        for (int64_t t = P.qtri_ptr[size_t(i)]; t < P.qtri_ptr[size_t(i) + 1]; ++t)
            if (!quality_record_ok(P.qtri.data() + 4 * t, uint32_t(r[1])))
                fail(LMS_ERR_STATE, "quality plan: record out of range");
    }
}

void mc_quality_plan(const Mesh &M, Mesh::MCPlan &P) {
    if (P.q_built) return;
    if (!P.fits || P.version != M.version) fail(LMS_ERR_STATE, "quality plan of a stale or unusable tile plan");
    P.q_built = true;
    // a corner outside the own rows sits in the tile's other staged rows;
    // both lists are ascending (a patch lists its own rows ahead of them)
    auto find = [](const int32_t *a, int32_t len, int32_t v) -> int32_t {
        const int32_t *it = std::lower_bound(a, a + len, v);
        return it == a + len || *it != v ? -1 : int32_t(it - a);
    };
    std::vector<int32_t> row_tile;
    if (P.patches) {
        row_tile.assign(size_t(M.n), -1);
        for (int32_t t = 0; t < P.tiles; ++t)
            for (int32_t i = 0; i < P.tile_ptr[size_t(t) + 1] - P.tile_ptr[size_t(t)]; ++i)
                row_tile[size_t(P.halo[size_t(P.halo_ptr[size_t(t)] + i)])] = t;
    }
    auto slot_of = [&](int32_t tile, int32_t v) -> int32_t {
        const int32_t b = P.tile_ptr[size_t(tile)], e = P.tile_ptr[size_t(tile) + 1], nown = e - b;
        const int32_t *h = P.halo.data() + P.halo_ptr[size_t(tile)];
        const int32_t nh = int32_t(P.halo_ptr[size_t(tile) + 1] - P.halo_ptr[size_t(tile)]);
        if (P.patches) {
            const int32_t i = find(h, nown, v);
            if (i >= 0) return i;
            const int32_t j = find(h + nown, nh - nown, v);
            return j < 0 ? -1 : nown + j;
        }
        if (v >= b && v < e) return v - b;
        const int32_t j = find(h, nh, v);
        return j < 0 ? -1 : nown + j;
    };
    auto tile_of = [&](int32_t v) -> int32_t {
        if (P.patches) return row_tile[size_t(v)];
        return int32_t(std::upper_bound(P.tile_ptr.begin(), P.tile_ptr.end(), v) - P.tile_ptr.begin()) - 1;
    };
    P.q_fits = tile_quality_records(M, P.tiles, tile_of, slot_of, P.qtri_ptr, P.qtri, P.qc_ids, P.qc_w);
    if (!P.q_fits) return;
    for (int32_t i = 0; i < P.tiles; ++i) {
        const uint32_t nst = uint32_t(P.halo_ptr[size_t(i) + 1] - P.halo_ptr[size_t(i)]) +
                             uint32_t(P.patches ? 0 : P.tile_ptr[size_t(i) + 1] - P.tile_ptr[size_t(i)]);
        for (int64_t t = P.qtri_ptr[size_t(i)]; t < P.qtri_ptr[size_t(i) + 1]; ++t)
            if (!quality_record_ok(P.qtri.data() + 4 * t, nst)) fail(LMS_ERR_STATE, "quality plan: record out of range");
    }
}

const Mesh::MCPlan &mc_plan(Mesh &M, int32_t ts, int32_t l_cap, int32_t u_cap, bool patches, int32_t k) {
    for (const auto &h : M.mc_plans)
        if (h.ts == ts && h.l_cap == l_cap && h.u_cap == u_cap && h.patches == patches && h.k == k &&
            h.version == M.version)
            return h;
    if (M.ell_w <= 0) fail(LMS_ERR_STATE, "no padded adjacency for a multicolour tile plan");
    if (ts <= 0 || l_cap < 1 || l_cap >= 0xFFFF || u_cap < 1 || k < 1 || k > 8)
        fail(LMS_ERR_ARG, "multicolour plan: bad tile size, cap or depth");
    const int32_t n = M.n, W = M.ell_w, C = M.n_colors;
    static const Mesh::Patches no_patches{0, 0, std::vector<int64_t>(1, 0), {}};
    const Mesh::Patches &ps = patches ? patch_set(M, ts) : no_patches;
    const int64_t nominal = patches ? int64_t(ps.patch_ptr.size()) - 1 : (int64_t(n) + ts - 1) / ts;
    struct Part {
        bool fits = true;
        std::vector<int32_t> tile_end, halo, halo_n;
        std::vector<int64_t> ucount;  // per tile and colour
        std::vector<uint16_t> urow, uidx;
        std::vector<uint8_t> umask;
        int32_t l_max = 0;
    };
    const int workers = host_threads(nominal);
    std::vector<Part> parts(static_cast<size_t>(workers));
    std::atomic<bool> give_up{false};
    std::atomic<int64_t> all_own{0}, all_staged{0};
    const int64_t sample = std::max<int64_t>(4096, int64_t(n) / 16);
    parallel_runs(nominal, workers, [&](int w, int64_t first, int64_t last) {
        Part &out = parts[size_t(w)];
        SlotMap slots(size_t(l_cap) + size_t(W) + 1);
        std::vector<int32_t> staged, upd, queue, seeds;
        std::vector<uint8_t> in_upd_mark;  // parallel to staged: bit t-1 set when updated in sweep t
        // Stage the own rows (ascending), the rows each sweep of the pass
        // updates, their neighbours; false when a cap is exceeded.  Sweep k
        // (the last) updates U_k: the own free rows and, closed downwards,
        // every lower-colour neighbour of an updated row (read at this
        // sweep's value).  Sweep t-1 updates U_{t-1}: the higher-colour
        // neighbours of U_t (U_t reads them at sweep t-1's value), closed
        // downwards the same way.  A pass of depth d runs sweeps k-d+1..k.
        auto try_tile = [&](const int32_t *own, int32_t nown) {
            slots.clear();
            staged.clear();
            in_upd_mark.clear();
            seeds.clear();
            for (int32_t i = 0; i < nown; ++i) {
                const int32_t v = own[i];
                slots.insert(v, i);
                staged.push_back(v);
                in_upd_mark.push_back(0);
                if (!M.fixed[size_t(v)]) seeds.push_back(v);
            }
            if (int64_t(staged.size()) > l_cap) return false;
            int64_t nupd = 0;  // rows updated in some sweep
            auto stage = [&](int32_t u) {
                int32_t su = slots.get(u);
                if (su < 0) {
                    su = int32_t(staged.size());
                    slots.insert(u, su);
                    staged.push_back(u);
                    in_upd_mark.push_back(0);
                }
                return su;
            };
            for (int32_t t = k; t >= 1; --t) {
                const uint8_t bit = uint8_t(1u << (t - 1));
                queue.clear();
                auto mark = [&](int32_t v, int32_t sv) {
                    if (in_upd_mark[size_t(sv)] & bit) return;
                    if (!in_upd_mark[size_t(sv)]) ++nupd;
                    in_upd_mark[size_t(sv)] |= bit;
                    queue.push_back(v);
                };
                for (int32_t v : seeds) mark(v, stage(v));
                for (size_t qi = 0; qi < queue.size(); ++qi) {
                    if (nupd > u_cap || int64_t(staged.size()) > l_cap) return false;
                    const int32_t v = queue[qi];
                    const int32_t cv = M.color[size_t(v)];
                    for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                        const int32_t u = M.col[size_t(j)];
                        const int32_t su = stage(u);
                        // u is read by v at this sweep's value when its colour comes first
                        if (!M.fixed[size_t(u)] && M.color[size_t(u)] < cv) mark(u, su);
                    }
                }
                if (nupd > u_cap || int64_t(staged.size()) > l_cap) return false;
                // rows of higher colour that U_t reads, at the previous sweep's value
                seeds.clear();
                if (t > 1)
                    for (int32_t v : queue)
                        for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                            const int32_t u = M.col[size_t(j)];
                            if (!M.fixed[size_t(u)] && M.color[size_t(u)] > M.color[size_t(v)]) seeds.push_back(u);
                        }
            }
            return nupd <= u_cap;
        };
        auto emit_tile = [&](const int32_t *own, int32_t nown) {
            // slots: own rows, then the others in ascending id
            std::vector<int32_t> others(staged.begin() + nown, staged.end());
            std::sort(others.begin(), others.end());
            for (size_t i = 0; i < others.size(); ++i) slots.set(others[i], nown + int32_t(i));
            // updated rows by colour, ascending slot inside a colour, with
            // the sweeps of the pass that update them
            std::vector<std::vector<std::pair<int32_t, uint8_t>>> by_colour(size_t(std::max(C, 1)));
            for (size_t i = 0; i < staged.size(); ++i)
                if (in_upd_mark[i]) {
                    const int32_t v = staged[i];
                    by_colour[size_t(M.color[size_t(v)])].emplace_back(slots.get(v), in_upd_mark[i]);
                }
            for (int32_t c = 0; c < C; ++c) {
                auto &rows = by_colour[size_t(c)];
                std::sort(rows.begin(), rows.end());
                out.ucount.push_back(int64_t(rows.size()));
                for (const auto &[sl, msk] : rows) {
                    const int32_t v = sl < nown ? own[sl] : others[size_t(sl - nown)];
                    out.urow.push_back(uint16_t(sl));
                    out.umask.push_back(msk);
                    const size_t base = out.uidx.size();
                    out.uidx.resize(base + size_t(W), uint16_t(0xFFFF));
                    for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
                        const int32_t su = slots.get(M.col[size_t(j)]);
                        if (su < 0) fail(LMS_ERR_STATE, "multicolour plan: neighbour not staged");
                        out.uidx[base + size_t(j - M.row_ptr[v])] = uint16_t(su);
                    }
                }
            }
            // patches list their own rows ahead of the other staged rows
            out.tile_end.push_back(patches ? nown : own[nown - 1] + 1);
            if (patches) out.halo.insert(out.halo.end(), own, own + nown);
            out.halo.insert(out.halo.end(), others.begin(), others.end());
            out.halo_n.push_back(int32_t(others.size()) + (patches ? nown : 0));
            out.l_max = std::max(out.l_max, int32_t(staged.size()));
        };
        // a range tile is halved in the middle, a patch along its
        // breadth-first order (the first half is a smaller ball around the seed)
        std::vector<std::pair<int64_t, int64_t>> todo;
        std::vector<int32_t> ownv;
        for (int64_t t = first; t < last && out.fits; ++t) {
            if (give_up.load(std::memory_order_relaxed)) {
                out.fits = false;
                break;
            }
            if (patches)
                todo.emplace_back(ps.patch_ptr[size_t(t)], ps.patch_ptr[size_t(t) + 1]);
            else
                todo.emplace_back(t * ts, std::min<int64_t>(n, (t + 1) * ts));
            while (!todo.empty()) {
                const auto [b, e] = todo.back();
                todo.pop_back();
                ownv.resize(size_t(e - b));
                for (int64_t i = b; i < e; ++i) ownv[size_t(i - b)] = patches ? ps.patch_rows[size_t(i)] : int32_t(i);
                if (patches) std::sort(ownv.begin(), ownv.end());
                if (try_tile(ownv.data(), int32_t(e - b))) {
                    emit_tile(ownv.data(), int32_t(e - b));
                    const int64_t own = all_own.fetch_add(e - b) + (e - b);
                    const int64_t st = all_staged.fetch_add(int64_t(staged.size())) + int64_t(staged.size());
                    if (own > sample && st > kTBMaxStagedPerRow * own) {  // the same bound as temporal blocking
                        out.fits = false;
                        give_up.store(true, std::memory_order_relaxed);
                        break;
                    }
                } else if (e - b > 1) {
                    const int64_t mid = b + (e - b) / 2;
                    todo.emplace_back(mid, e);
                    todo.emplace_back(b, mid);
                } else {
                    out.fits = false;
                    give_up.store(true, std::memory_order_relaxed);
                    break;
                }
            }
        }
    });
    Mesh::MCPlan P;
    P.ts = ts;
    P.l_cap = l_cap;
    P.u_cap = u_cap;
    P.patches = patches;
    P.k = k;
    P.colors = C;
    for (const auto &q : parts) P.fits = P.fits && q.fits;
    if (P.fits) {
        P.tile_ptr.push_back(0);
        P.halo_ptr.push_back(0);
        P.upd_ptr.push_back(0);
        for (auto &q : parts) {
            P.l_max = std::max(P.l_max, q.l_max);
            for (size_t t = 0; t < q.tile_end.size(); ++t) {
                P.tile_ptr.push_back(patches ? P.tile_ptr.back() + q.tile_end[t] : q.tile_end[t]);
                P.halo_ptr.push_back(P.halo_ptr.back() + q.halo_n[t]);
            }
            for (int64_t c : q.ucount) P.upd_ptr.push_back(P.upd_ptr.back() + c);
            P.halo.insert(P.halo.end(), q.halo.begin(), q.halo.end());
            P.urow.insert(P.urow.end(), q.urow.begin(), q.urow.end());
            P.uidx.insert(P.uidx.end(), q.uidx.begin(), q.uidx.end());
            P.umask.insert(P.umask.end(), q.umask.begin(), q.umask.end());
            q = Part{};
        }
        P.tiles = int32_t(P.tile_ptr.size() - 1);
        // upd_ptr holds tiles*C counts' running sums: give each tile C+1 entries
        std::vector<int64_t> up(size_t(P.tiles) * size_t(C + 1));
        for (int32_t t = 0; t < P.tiles; ++t)
            for (int32_t c = 0; c <= C; ++c) up[size_t(t) * size_t(C + 1) + size_t(c)] = P.upd_ptr[size_t(t) * size_t(C) + size_t(c)];
        P.upd_ptr = std::move(up);
        // self-check: tiles cover the rows (patches: every free row once);
        // every own free row is updated once, in its colour; every updated
        // row's slots name its neighbours in order
        if (P.tile_ptr.back() != (patches ? M.n_free : n))
            fail(LMS_ERR_STATE, "multicolour plan: tiles do not cover the rows");
        std::vector<uint8_t> owned(patches ? size_t(n) : 0, 0);
        for (int32_t t = 0; t < P.tiles; ++t) {
            const int32_t b = P.tile_ptr[size_t(t)], e = P.tile_ptr[size_t(t) + 1], nown = e - b;
            const int64_t hb = P.halo_ptr[size_t(t)];
            const int32_t nst = int32_t(P.halo_ptr[size_t(t) + 1] - hb) + (patches ? 0 : nown);
            if (nown <= 0 || nst < nown) fail(LMS_ERR_STATE, "multicolour plan: tile counts");
            auto global_of = [&](int32_t sl) {
                if (patches) return P.halo[size_t(hb + sl)];
                return sl < nown ? b + sl : P.halo[size_t(hb + sl - nown)];
            };
            if (patches)
                for (int32_t sl = 0; sl < nown; ++sl) {
                    const int32_t v = global_of(sl);
                    if (v < 0 || v >= n || M.fixed[size_t(v)] || owned[size_t(v)] || (sl > 0 && v <= global_of(sl - 1)))
                        fail(LMS_ERR_STATE, "multicolour plan: patch rows");
                    owned[size_t(v)] = 1;
                }
            std::vector<uint8_t> seen(size_t(nst), 0);  // sweep mask of each updated slot
            for (int64_t i = P.upd_ptr[size_t(t) * size_t(C + 1)]; i < P.upd_ptr[size_t(t) * size_t(C + 1) + size_t(C)];
                 ++i) {
                const int32_t sl = P.urow[size_t(i)];
                const uint8_t msk = P.umask[size_t(i)];
                if (sl >= nst || seen[size_t(sl)] || msk == 0 || (k < 8 && (msk >> k) != 0))
                    fail(LMS_ERR_STATE, "multicolour plan: bad updated row");
                seen[size_t(sl)] = msk;
            }
            for (int32_t c = 0; c < C; ++c)
                for (int64_t i = P.upd_ptr[size_t(t) * size_t(C + 1) + size_t(c)];
                     i < P.upd_ptr[size_t(t) * size_t(C + 1) + size_t(c) + 1]; ++i) {
                    const int32_t sl = P.urow[size_t(i)];
                    const uint8_t msk = P.umask[size_t(i)];
                    const int32_t v = global_of(sl);
                    if (M.fixed[size_t(v)] || M.color[size_t(v)] != c) fail(LMS_ERR_STATE, "multicolour plan: colour");
                    const int32_t deg = M.row_ptr[v + 1] - M.row_ptr[v];
                    for (int32_t q = 0; q < W; ++q) {
                        const uint16_t su = P.uidx[size_t(i) * size_t(W) + size_t(q)];
                        if (q >= deg) {
                            if (su != 0xFFFF) fail(LMS_ERR_STATE, "multicolour plan: padding slot in use");
                            continue;
                        }
                        if (su >= nst || global_of(su) != M.col[size_t(M.row_ptr[v] + q)])
                            fail(LMS_ERR_STATE, "multicolour plan: slot names the wrong vertex");
                        // in every sweep t it runs in, v reads a free lower-colour
                        // neighbour at sweep t's value and a higher-colour one at
                        // sweep t-1's (the staged value when t is the pass's first)
                        const int32_t u = M.col[size_t(M.row_ptr[v] + q)];
                        if (M.fixed[size_t(u)]) continue;
                        const uint8_t mu = seen[size_t(su)];
                        for (int32_t tt = 1; tt <= k; ++tt) {
                            if (!((msk >> (tt - 1)) & 1u)) continue;
                            if (M.color[size_t(u)] < c && !((mu >> (tt - 1)) & 1u))
                                fail(LMS_ERR_STATE, "multicolour plan: lower-colour neighbour not updated");
                            if (M.color[size_t(u)] > c && tt > 1 && !((mu >> (tt - 2)) & 1u))
                                fail(LMS_ERR_STATE, "multicolour plan: higher-colour neighbour not updated");
                        }
                    }
                }
            for (int32_t sl = 0; sl < nown; ++sl)
                if (!M.fixed[size_t(global_of(sl))] && !((seen[size_t(sl)] >> (k - 1)) & 1u))
                    fail(LMS_ERR_STATE, "multicolour plan: own row missed");
        }
    } else {
        P = Mesh::MCPlan{};
        P.ts = ts;
        P.l_cap = l_cap;
        P.u_cap = u_cap;
        P.patches = patches;
        P.k = k;
        P.fits = false;
    }
    P.version = M.version;
    M.mc_plans.push_back(std::move(P));
    return M.mc_plans.back();
}

// Locality profile of the current ordering: reuse distances of an access
// trace (a Fenwick tree over trace positions marks each item's last access;
// the distinct items since then are the marks after it), exact quantiles from
// their histogram, and cache-line spans per wavefront.
//
// trace 0 (one sweep of Eq. 1): every free vertex in ascending current label,
// then its neighbours in ascending label.  trace 1 (Algorithm 1's loop body,
// the smoothing of V[i] followed by the update of the global quality): the
// same, and after each vertex's neighbours, every triangle containing it in
// ascending current triangle index, as its three corners in ascending label
// followed by the triangle's own quality record.  Items are vertex labels
// 0..n-1 and triangle records n..n+T-1.
void reuse_profile(const Mesh &M, int32_t trace, const double *fractions, int32_t nfrac, int64_t *quantiles,
                   int32_t line_bytes, int32_t record_bytes, lms_reuse_stats &out) {
    if (nfrac < 0 || (nfrac > 0 && (!fractions || !quantiles)) || line_bytes <= 0 || record_bytes <= 0)
        fail(LMS_ERR_ARG, "reuse profile: bad fractions or sizes");
    if (trace != 0 && trace != 1) fail(LMS_ERR_ARG, "reuse profile: unknown trace");
    for (int32_t i = 0; i < nfrac; ++i)
        if (!(fractions[i] >= 0.0 && fractions[i] <= 1.0)) fail(LMS_ERR_ARG, "reuse profile: fraction outside [0, 1]");
    const int32_t n = M.n;
    const int64_t items = trace == 1 ? int64_t(n) + M.T : int64_t(n);
    // the trace, in order, to an access function
    auto walk = [&](auto &&emit) {
        for (int32_t v = 0; v < n; ++v) {
            if (M.fixed[size_t(v)]) continue;
            emit(int64_t(v));
            for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) emit(int64_t(M.col[size_t(j)]));
            if (trace == 1)
                for (int32_t e = M.vt_ptr[v]; e < M.vt_ptr[v + 1]; ++e) {
                    const int32_t t = M.vt[size_t(e)];
                    int32_t c[3] = {M.ta[size_t(t)], M.tb[size_t(t)], M.tc[size_t(t)]};
                    std::sort(c, c + 3);
                    emit(int64_t(c[0]));
                    emit(int64_t(c[1]));
                    emit(int64_t(c[2]));
                    emit(int64_t(n) + t);
                }
        }
    };
    int64_t L = 0;
    walk([&](int64_t) { ++L; });
    if (L >= (int64_t(1) << 31)) fail(LMS_ERR_STATE, "reuse profile: trace too long");
    std::vector<int32_t> fen(size_t(L) + 1, 0);  // 1-based Fenwick tree over trace positions
    auto add = [&](int64_t i, int32_t d) {
        for (++i; i <= L; i += i & -i) fen[size_t(i)] += d;
    };
    auto prefix = [&](int64_t i) {  // marks at positions [0, i)
        int64_t acc = 0;
        for (; i > 0; i -= i & -i) acc += fen[size_t(i)];
        return acc;
    };
    std::vector<int64_t> last(size_t(items), -1);
    std::vector<int64_t> hist(size_t(items) + 1, 0);
    int64_t t = 0, cold = 0, dmax = 0;
    double dsum = 0.0;
    walk([&](int64_t x) {
        const int64_t p = last[size_t(x)];
        if (p < 0) {
            ++cold;
        } else {
            const int64_t d = prefix(t) - prefix(p + 1);
            hist[size_t(d)]++;
            dsum += double(d);
            dmax = std::max(dmax, d);
            add(p, -1);
        }
        add(t, 1);
        last[size_t(x)] = t;
        ++t;
    });
    const int64_t total = L - cold;
    for (int32_t i = 0; i < nfrac; ++i) {
        int64_t q = 0;
        if (total > 0) {
            const int64_t need = std::max<int64_t>(1, int64_t(std::ceil(fractions[i] * double(total) - 1e-12)));
            int64_t cum = 0;
            for (q = 0; q <= items; ++q) {
                cum += hist[size_t(q)];
                if (cum >= need) break;
            }
        }
        quantiles[i] = q;
    }
    // cache lines touched by the neighbour reads of each wavefront of 64 rows
    std::vector<int64_t> lines;
    int64_t waves = 0, span_sum = 0, span_max = 0;
    for (int32_t w0 = 0; w0 < n; w0 += 64) {
        lines.clear();
        bool any_free = false;
        for (int32_t v = w0; v < std::min(n, w0 + 64); ++v) {
            if (M.fixed[size_t(v)]) continue;
            any_free = true;
            for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j)
                lines.push_back(int64_t(M.col[size_t(j)]) * record_bytes / line_bytes);
        }
        if (!any_free) continue;
        std::sort(lines.begin(), lines.end());
        const int64_t span = int64_t(std::unique(lines.begin(), lines.end()) - lines.begin());
        ++waves;
        span_sum += span;
        span_max = std::max(span_max, span);
    }
    out.accesses = L;
    out.cold = cold;
    out.max = dmax;
    out.mean = total > 0 ? dsum / double(total) : 0.0;
    out.lines_per_wave = waves > 0 ? double(span_sum) / double(waves) : 0.0;
    out.max_lines_per_wave = span_max;
}

}  // namespace lms
