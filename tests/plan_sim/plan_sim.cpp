// CPU simulation of the tile plans that the temporally blocked Jacobi pass
// and the one-pass multicolour sweep read (host logic, no GPU).
//
// A plan lists, per tile, the rows it stages, the rows each sweep of a pass
// updates and the staging slots of their neighbours.  This program runs the
// arithmetic of Eq. 1 exactly as those lists direct it (ascending CSR order,
// one division per row) on one scalar field and compares the result, bit for
// bit, with plain sweeps over the whole mesh:
//   - halo plans (one sweep per launch): one Jacobi sweep;
//   - temporally blocked plans: a pass of depth d against d Jacobi sweeps
//     (Algorithm 1, every free vertex reading the previous sweep);
//   - multicolour plans: a pass of depth d against d colour-by-colour sweeps
//     in place (the in-place form of Algorithm 1 under a vertex colouring).
// It also sums the mesh quality (Section 3.2, Algorithm 1) from each plan's
// triangle records over the staged input coordinates, as the quality-fused
// passes do, and compares it with the per-vertex definition (relative error
// q_err; the two sum in different orders).
//
// Usage: plan_sim <mesh file> <ori|bfs|rdr|random> [plant]
// Mesh file: int32 n, int64 T, int32 tri[3T], float64 x[n], float64 y[n].
// Prints one line per plan shape; exits 1 on any mismatch or library error.
// With "plant", each plan is simulated from a copy in which one own row of
// the first tile reads its own slot in place of its first neighbour, and the
// weight of the first triangle record counts one triangle too many at its
// second corner:
// every fitting shape must then report mismatches and a large q_err (a check
// of this checker).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <string>
#include <vector>

#include "lms_internal.hpp"

// The plan builders live beside the device runtime; these two hooks belong
// to it and have nothing to release here.
namespace lms {
void destroy_device_state(DeviceState *) {}
void destroy_reorder_state(ReorderState *) {}
}  // namespace lms

namespace {

using lms::Mesh;

// One row of Eq. 1 over the values `val` of its neighbours, in CSR order.
double row_mean(const Mesh &M, int32_t v, const std::vector<double> &val) {
    double a = 0.0;
    int c = 0;
    for (int32_t j = M.row_ptr[v]; j < M.row_ptr[v + 1]; ++j) {
        a += val[size_t(M.col[size_t(j)])];
        ++c;
    }
    return a / double(c);
}

std::vector<double> jacobi(const Mesh &M, std::vector<double> p, int sweeps) {
    for (int s = 0; s < sweeps; ++s) {
        std::vector<double> q = p;
        for (int32_t v = 0; v < M.n; ++v)
            if (!M.fixed[size_t(v)]) q[size_t(v)] = row_mean(M, v, p);
        p.swap(q);
    }
    return p;
}

std::vector<double> multicolour(const Mesh &M, std::vector<double> p, int sweeps) {
    for (int s = 0; s < sweeps; ++s)
        for (int32_t c = 0; c < M.n_colors; ++c)
            for (int32_t v = 0; v < M.n; ++v)
                if (!M.fixed[size_t(v)] && M.color[size_t(v)] == c) p[size_t(v)] = row_mean(M, v, p);
    return p;
}

// Mean over the padded slots of one plan row (0xFFFF ends the row).
double slot_mean(const uint16_t *slots, int W, const std::vector<double> &lds, bool &any) {
    double a = 0.0;
    int c = 0;
    for (int q = 0; q < W; ++q)
        if (slots[q] != 0xFFFFu) {
            a += lds[slots[q]];
            ++c;
        }
    any = c > 0;
    return any ? a / double(c) : 0.0;
}

long count_mismatches(const std::vector<double> &a, const std::vector<double> &b) {
    long bad = 0;
    for (size_t i = 0; i < a.size(); ++i) bad += a[i] != b[i];
    return bad;
}

// A temporally blocked pass of depth d from p0, as the plan directs it.
std::vector<double> tb_pass(const Mesh &M, const Mesh::TBPlan &P, const std::vector<double> &p0, int d) {
    const int W = M.ell_w, k = P.k;
    std::vector<double> out = p0;
    for (int32_t t = 0; t < P.tiles; ++t) {
        const int32_t *rc = &P.ring[size_t(t) * size_t(k + 1)];
        const int32_t nown = rc[0], nload = rc[d];
        const int64_t hb = P.halo_ptr[size_t(t)];
        auto row_of = [&](int32_t sl) {
            if (P.patches) return P.halo[size_t(hb + sl)];
            return sl < nown ? P.tile_ptr[size_t(t)] + sl : P.halo[size_t(hb + sl - nown)];
        };
        std::vector<double> lds(static_cast<size_t>(nload));
        for (int32_t sl = 0; sl < nload; ++sl) lds[size_t(sl)] = p0[size_t(row_of(sl))];
        const uint16_t *lx = P.lidx.data() + size_t(P.lidx_ptr[size_t(t)]) * size_t(W);
        for (int j = 1; j <= d; ++j) {
            const int32_t m = rc[d - j];  // rows this sweep updates
            std::vector<double> next = lds;
            for (int32_t i = 0; i < m; ++i) {
                bool any = false;
                const double v = slot_mean(lx + size_t(i) * size_t(W), W, lds, any);
                if (any) next[size_t(i)] = v;
            }
            lds.swap(next);
        }
        for (int32_t sl = 0; sl < nown; ++sl) {
            const int32_t v = row_of(sl);
            if (!M.fixed[size_t(v)]) out[size_t(v)] = lds[size_t(sl)];
        }
    }
    return out;
}

// One Jacobi sweep from p0 through a halo plan: tile t owns rows
// [t*ts, (t+1)*ts) at slots 0..ts-1 and stages its halo list after them.
std::vector<double> halo_sweep(const Mesh &M, const Mesh::HaloPlan &H, const std::vector<double> &p0) {
    const int W = M.ell_w, ts = H.ts;
    std::vector<double> out = p0;
    const int32_t tiles = int32_t(H.halo_ptr.size()) - 1;
    for (int32_t t = 0; t < tiles; ++t) {
        const int32_t b = t * ts, e = std::min(M.n, b + ts);
        const int32_t hb = H.halo_ptr[size_t(t)], nh = H.halo_ptr[size_t(t) + 1] - hb;
        std::vector<double> lds(static_cast<size_t>(ts + nh), 0.0);
        for (int32_t v = b; v < e; ++v) lds[size_t(v - b)] = p0[size_t(v)];
        for (int32_t i = 0; i < nh; ++i) lds[size_t(ts + i)] = p0[size_t(H.halo[size_t(hb + i)])];
        for (int32_t v = b; v < e; ++v) {
            bool any = false;
            const double m = slot_mean(H.lidx.data() + size_t(v) * size_t(W), W, lds, any);
            if (any) out[size_t(v)] = m;
        }
    }
    return out;
}

// A one-pass multicolour pass of depth d from p0: sweeps k-d+1..k of the
// plan, colour by colour in place in the tile's staging area.
std::vector<double> mc_pass(const Mesh &M, const Mesh::MCPlan &P, const std::vector<double> &p0, int d) {
    const int W = M.ell_w, C = M.n_colors, k = P.k;
    std::vector<double> out = p0;
    for (int32_t t = 0; t < P.tiles; ++t) {
        const int32_t nown = P.tile_ptr[size_t(t) + 1] - P.tile_ptr[size_t(t)];
        const int64_t hb = P.halo_ptr[size_t(t)];
        const int32_t nst = int32_t(P.halo_ptr[size_t(t) + 1] - hb) + (P.patches ? 0 : nown);
        auto row_of = [&](int32_t sl) {
            if (P.patches) return P.halo[size_t(hb + sl)];
            return sl < nown ? P.tile_ptr[size_t(t)] + sl : P.halo[size_t(hb + sl - nown)];
        };
        std::vector<double> lds(static_cast<size_t>(nst));
        for (int32_t sl = 0; sl < nst; ++sl) lds[size_t(sl)] = p0[size_t(row_of(sl))];
        const int64_t *u = &P.upd_ptr[size_t(t) * size_t(C + 1)];
        for (int s = k - d + 1; s <= k; ++s)
            for (int32_t c = 0; c < C; ++c)
                for (int64_t e = u[c]; e < u[c + 1]; ++e) {
                    if (k > 1 && !((P.umask[size_t(e)] >> (s - 1)) & 1u)) continue;
                    bool any = false;
                    const double v = slot_mean(P.uidx.data() + size_t(e) * size_t(W), W, lds, any);
                    if (any) lds[P.urow[size_t(e)]] = v;
                }
        for (int32_t sl = 0; sl < nown; ++sl) {
            const int32_t v = row_of(sl);
            if (!M.fixed[size_t(v)]) out[size_t(v)] = lds[size_t(sl)];
        }
    }
    return out;
}

// Edge-length ratio of a triangle: shortest over longest edge (Section 3.2).
double tri_q(double xa, double ya, double xb, double yb, double xc, double yc) {
    const double e[3] = {(xb - xa) * (xb - xa) + (yb - ya) * (yb - ya), (xc - xb) * (xc - xb) + (yc - yb) * (yc - yb),
                         (xa - xc) * (xa - xc) + (ya - yc) * (ya - yc)};
    const double mn = std::min({e[0], e[1], e[2]}), mx = std::max({e[0], e[1], e[2]});
    return mx > 0.0 ? std::sqrt(mn) / std::sqrt(mx) : 0.0;
}

// n times the mesh quality from its definition, in input labels: the sum
// over vertices of the mean quality of the triangles at each vertex.
double quality_sum_direct(const Mesh &M, const std::vector<double> &x, const std::vector<double> &y) {
    std::vector<double> s(size_t(M.n), 0.0);
    for (int64_t t = 0; t < M.T; ++t) {
        const int32_t a = M.tri0[size_t(3 * t)], b = M.tri0[size_t(3 * t + 1)], c = M.tri0[size_t(3 * t + 2)];
        const double q = tri_q(x[size_t(a)], y[size_t(a)], x[size_t(b)], y[size_t(b)], x[size_t(c)], y[size_t(c)]);
        s[size_t(a)] += q;
        s[size_t(b)] += q;
        s[size_t(c)] += q;
    }
    double total = 0.0;
    for (int32_t v = 0; v < M.n; ++v)
        if (M.tcount0[size_t(v)] > 0) total += s[size_t(v)] / double(M.tcount0[size_t(v)]);
    return total;
}

// The same sum from a plan's triangle records: each record names three
// staging slots of its tile and carries the triangle's weight (a double in
// its last two words); triangles with only fixed corners are listed apart
// with their weights.
double record_weight(const uint32_t *w) {
    double wt;
    std::memcpy(&wt, w + 2, sizeof(double));
    return wt;
}

template <class Plan, class RowOf>
double quality_sum_plan(const Plan &P, RowOf row_of, const std::vector<double> &xc, const std::vector<double> &yc) {
    double total = 0.0;
    for (int32_t t = 0; t < P.tiles; ++t)
        for (int64_t i = P.qtri_ptr[size_t(t)]; i < P.qtri_ptr[size_t(t) + 1]; ++i) {
            const uint32_t *w = P.qtri.data() + 4 * i;
            const int32_t a = row_of(t, int32_t(w[0] & 0xFFFFu)), b = row_of(t, int32_t(w[0] >> 16)),
                          c = row_of(t, int32_t(w[1]));
            const double q = tri_q(xc[size_t(a)], yc[size_t(a)], xc[size_t(b)], yc[size_t(b)], xc[size_t(c)],
                                   yc[size_t(c)]);
            total += q * record_weight(w);
        }
    for (size_t i = 0; i < P.qc_w.size(); ++i) {
        const int32_t a = P.qc_ids[3 * i], b = P.qc_ids[3 * i + 1], c = P.qc_ids[3 * i + 2];
        total += P.qc_w[i] *
                 tri_q(xc[size_t(a)], yc[size_t(a)], xc[size_t(b)], yc[size_t(b)], xc[size_t(c)], yc[size_t(c)]);
    }
    return total;
}

// The current-label arrays a relabelling installs, checked against the CSR
// and the input triangles: the padded and colour-major copies, the sorted
// triangle list with its weights and packed records, and the vertex ->
// triangle lists.  Returns the number of wrong entries.
long check_relabel(const Mesh &M) {
    const int32_t n = M.n, W = M.ell_w;
    long bad = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t deg = M.row_ptr[k + 1] - M.row_ptr[k];
        for (int32_t j = 0; j < W; ++j)
            bad += M.ell[size_t(k) * size_t(W) + size_t(j)] != (j < deg ? M.col[size_t(M.row_ptr[k] + j)] : -1);
    }
    for (int32_t c = 0; c < M.n_colors; ++c) {
        const int64_t cnt = M.color_ptr[c + 1] - M.color_ptr[c];
        for (int64_t i = 0; i < cnt; ++i) {
            const int32_t k = M.color_list[size_t(M.color_ptr[c] + i)];
            const int32_t deg = M.row_ptr[k + 1] - M.row_ptr[k];
            bad += M.color[size_t(k)] != c;
            for (int32_t j = 0; j < W; ++j)
                bad += M.color_ell[size_t(int64_t(W) * M.color_ptr[c] + j * cnt + i)] !=
                       (j < deg ? M.col[size_t(M.row_ptr[k] + j)] : -1);
        }
    }
    // triangles: ascending smallest corner, and back in input labels a
    // permutation of the input triangles
    std::vector<std::array<int32_t, 3>> back(size_t(M.T)), in(size_t(M.T));
    for (int64_t i = 0; i < M.T; ++i) {
        const int32_t a = M.ta[size_t(i)], b = M.tb[size_t(i)], c = M.tc[size_t(i)];
        if (i > 0) bad += std::min({a, b, c}) < std::min({M.ta[size_t(i - 1)], M.tb[size_t(i - 1)], M.tc[size_t(i - 1)]});
        const int32_t oa = M.new2old[size_t(a)], ob = M.new2old[size_t(b)], oc = M.new2old[size_t(c)];
        back[size_t(i)] = {oa, ob, oc};
        in[size_t(i)] = {M.tri0[size_t(3 * i)], M.tri0[size_t(3 * i + 1)], M.tri0[size_t(3 * i + 2)]};
        bad += M.tw[size_t(i)] != 1.0 / double(M.tcount0[size_t(oa)]) + 1.0 / double(M.tcount0[size_t(ob)]) +
                                      1.0 / double(M.tcount0[size_t(oc)]);
        if (!M.trec.empty())
            bad += M.trec[size_t(4 * i)] != a || M.trec[size_t(4 * i + 1)] != b || M.trec[size_t(4 * i + 2)] != c ||
                   M.trec[size_t(4 * i + 3)] !=
                       (M.tcount0[size_t(oa)] | (M.tcount0[size_t(ob)] << 10) | (M.tcount0[size_t(oc)] << 20));
    }
    std::sort(back.begin(), back.end());
    std::sort(in.begin(), in.end());
    bad += back != in;
    // vertex -> triangles: every triangle at its three corners, ascending
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = M.vt_ptr[v]; e < M.vt_ptr[v + 1]; ++e) {
            const int32_t t = M.vt[size_t(e)];
            bad += M.ta[size_t(t)] != v && M.tb[size_t(t)] != v && M.tc[size_t(t)] != v;
            if (e > M.vt_ptr[v]) bad += t <= M.vt[size_t(e - 1)];
        }
    bad += M.vt_ptr[n] != 3 * M.T;
    return bad;
}

// Wrong entries of a patch set: free rows in no patch or in two, fixed rows
// in a patch, patches over ts rows or empty, and patches whose rows are not
// all reached from their first row over the adjacency inside the patch.
long check_patches(const Mesh &M, const Mesh::Patches &ps, int ts) {
    long bad = 0;
    std::vector<int32_t> owner(size_t(M.n), -1);
    const int32_t np = int32_t(ps.patch_ptr.size()) - 1;
    for (int32_t p = 0; p < np; ++p) {
        const int64_t b = ps.patch_ptr[size_t(p)], e = ps.patch_ptr[size_t(p) + 1];
        bad += e - b > ts || e <= b;
        for (int64_t i = b; i < e; ++i) {
            const int32_t v = ps.patch_rows[size_t(i)];
            bad += M.fixed[size_t(v)] != 0 || owner[size_t(v)] >= 0;
            owner[size_t(v)] = p;
        }
    }
    for (int32_t v = 0; v < M.n; ++v) bad += !M.fixed[size_t(v)] && owner[size_t(v)] < 0;
    std::vector<uint8_t> seen(size_t(M.n), 0);
    for (int32_t p = 0; p < np; ++p) {
        const int64_t b = ps.patch_ptr[size_t(p)], e = ps.patch_ptr[size_t(p) + 1];
        if (e <= b) continue;
        std::vector<int32_t> queue(1, ps.patch_rows[size_t(b)]);
        seen[size_t(queue[0])] = 1;
        for (size_t h = 0; h < queue.size(); ++h)
            for (int32_t j = M.row_ptr[queue[h]]; j < M.row_ptr[queue[h] + 1]; ++j) {
                const int32_t u = M.col[size_t(j)];
                if (owner[size_t(u)] == p && !seen[size_t(u)]) {
                    seen[size_t(u)] = 1;
                    queue.push_back(u);
                }
            }
        bad += int64_t(queue.size()) != e - b;
    }
    return bad;
}

// The planted weight: the first triangle record's weight as if its second
// corner were in one triangle more.
template <class Plan, class RowOf>
void plant_weight(const Mesh &M, Plan &P, RowOf row_of) {
    int32_t t0 = 0;
    while (t0 < P.tiles && P.qtri_ptr[size_t(t0) + 1] == P.qtri_ptr[size_t(t0)]) ++t0;
    if (t0 == P.tiles) return;
    uint32_t *w = P.qtri.data() + 4 * P.qtri_ptr[size_t(t0)];
    const int32_t rows[3] = {row_of(t0, int32_t(w[0] & 0xFFFFu)), row_of(t0, int32_t(w[0] >> 16)),
                             row_of(t0, int32_t(w[1]))};
    double c[3];
    for (int q = 0; q < 3; ++q) c[q] = double(M.tcount0[size_t(M.new2old[size_t(rows[q])])]);
    const double wt = 1.0 / c[0] + 1.0 / (c[1] + 1.0) + 1.0 / c[2];
    std::memcpy(w + 2, &wt, sizeof(double));
}

// The planted mistakes: the first own row of tile 0 that has neighbours
// reads its own slot in place of its first neighbour.
void plant(Mesh::TBPlan &P, int W) {
    const int32_t nown = P.ring[0];
    for (int32_t i = 0; i < nown; ++i) {
        uint16_t *row = P.lidx.data() + size_t(P.lidx_ptr[0] + i) * size_t(W);
        if (row[0] != 0xFFFFu) {
            row[0] = uint16_t(i);
            return;
        }
    }
}

void plant(Mesh::MCPlan &P, int W) {
    const int32_t nown = P.tile_ptr[1] - P.tile_ptr[0];
    for (int64_t e = 0; e < P.upd_ptr[size_t(P.colors)]; ++e) {
        uint16_t *row = P.uidx.data() + size_t(e) * size_t(W);
        if (P.urow[size_t(e)] < nown && row[0] != 0xFFFFu) {
            row[0] = P.urow[size_t(e)];
            return;
        }
    }
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3 && !(argc == 4 && std::string(argv[3]) == "plant")) {
        std::fprintf(stderr, "usage: plan_sim <mesh file> <ori|bfs|rdr|random> [plant]\n");
        return 2;
    }
    const bool planted = argc == 4;
    std::ifstream f(argv[1], std::ios::binary);
    int32_t n = 0;
    int64_t T = 0;
    f.read(reinterpret_cast<char *>(&n), sizeof(n));
    f.read(reinterpret_cast<char *>(&T), sizeof(T));
    std::vector<int32_t> tri(static_cast<size_t>(3 * T));
    std::vector<double> x(static_cast<size_t>(n)), y(static_cast<size_t>(n));
    f.read(reinterpret_cast<char *>(tri.data()), std::streamsize(tri.size() * sizeof(int32_t)));
    f.read(reinterpret_cast<char *>(x.data()), std::streamsize(x.size() * sizeof(double)));
    f.read(reinterpret_cast<char *>(y.data()), std::streamsize(y.size() * sizeof(double)));
    if (!f) {
        std::fprintf(stderr, "plan_sim: short mesh file\n");
        return 2;
    }
    const std::string ord = argv[2];
    long total_bad = 0;
    try {
        Mesh M;
        const int64_t v_off[2] = {0, n}, t_off[2] = {0, T};
        lms::build_mesh(M, n, T, tri.data(), nullptr, 1, v_off, t_off);
        if (ord == "bfs") {
            lms::relabel(M, LMS_BFS, lms::order_bfs(M));
        } else if (ord == "rdr") {
            std::vector<double> q(static_cast<size_t>(n));
            lms::vertex_quality_host(M, x.data(), y.data(), q.data());
            lms::relabel(M, LMS_RDR, lms::order_rdr(M, q.data()));
        } else if (ord == "random") {
            lms::relabel(M, LMS_RANDOM, lms::order_random(M, 12345));
        } else if (ord != "ori") {
            std::fprintf(stderr, "plan_sim: unknown ordering %s\n", ord.c_str());
            return 2;
        }
        if (M.ell_w <= 0) {
            std::fprintf(stderr, "plan_sim: mesh has no padded adjacency\n");
            return 2;
        }
        const long relabel_bad = check_relabel(M);
        total_bad += relabel_bad;
        std::printf("relabel wrong=%ld\n", relabel_bad);
        // a field with no structure, so that any wrong neighbour or order shows
        std::mt19937_64 rng(7);
        std::uniform_real_distribution<double> U(-1.0, 1.0);
        std::vector<double> p0(static_cast<size_t>(n));
        for (auto &v : p0) v = U(rng);
        // the input coordinates in the current labels, and n times their quality
        std::vector<double> xc(static_cast<size_t>(n)), yc(static_cast<size_t>(n));
        for (int32_t v = 0; v < n; ++v) {
            xc[size_t(v)] = x[size_t(M.new2old[size_t(v)])];
            yc[size_t(v)] = y[size_t(M.new2old[size_t(v)])];
        }
        const double q_direct = quality_sum_direct(M, x, y);
        auto q_err = [&](double q_plan) { return std::fabs(q_plan - q_direct) / q_direct; };

        // the patches the patch plans grow from: every free row in exactly one
        // patch, at most ts rows each, each patch connected over the adjacency
        for (int ts : {256, 1024}) {
            const Mesh::Patches &ps = lms::patch_set(M, ts);
            const long bad = check_patches(M, ps, ts);
            total_bad += bad;
            std::printf("patches ts=%d count=%d wrong=%ld\n", ts, int(ps.patch_ptr.size()) - 1, bad);
        }

        // single-sweep halo plans: {tile size}
        for (int ts : {128, 256}) {
            Mesh::HaloPlan H = lms::halo_plan(M, ts);
            if (planted) {  // the first row with neighbours reads its own slot
                for (size_t r = 0; r < H.lidx.size(); r += size_t(M.ell_w))
                    if (H.lidx[r] != 0xFFFFu) {
                        H.lidx[r] = uint16_t((r / size_t(M.ell_w)) % size_t(ts));
                        break;
                    }
            }
            const long bad = count_mismatches(halo_sweep(M, H, p0), jacobi(M, p0, 1));
            total_bad += bad;
            std::printf("halo range ts=%d k=1 fits=1 tiles=%d mismatches=%ld q_fits=0 q_err=-1\n", ts,
                        int(H.halo_ptr.size()) - 1, bad);
        }
        // temporally blocked plans: {tile size, depth, update cap, staging cap}
        const int tb_shapes[][4] = {{256, 2, 512, 1024}, {512, 3, 1024, 2048}, {1024, 4, 2048, 2048}};
        for (int patches = 0; patches < 2; ++patches)
            for (const auto &c : tb_shapes) {
                Mesh::TBPlan P = lms::tb_plan(M, c[0], c[1], c[2], c[3], patches != 0);
                if (planted && P.fits) plant(P, M.ell_w);
                long bad = 0;
                double qe = -1.0;
                if (P.fits) {
                    for (int d = 1; d <= P.k; ++d) bad += count_mismatches(tb_pass(M, P, p0, d), jacobi(M, p0, d));
                    lms::tb_quality_plan(M, P);
                    auto row_of = [&](int32_t t, int32_t sl) {
                        const int32_t nown = P.ring[size_t(t) * size_t(P.k + 1)];
                        if (P.patches) return P.halo[size_t(P.halo_ptr[size_t(t)] + sl)];
                        return sl < nown ? P.tile_ptr[size_t(t)] + sl : P.halo[size_t(P.halo_ptr[size_t(t)] + sl - nown)];
                    };
                    if (planted && P.q_fits) plant_weight(M, P, row_of);
                    if (P.q_fits) qe = q_err(quality_sum_plan(P, row_of, xc, yc));
                }
                total_bad += bad;
                std::printf("tb %s ts=%d k=%d fits=%d tiles=%d mismatches=%ld q_fits=%d q_err=%.3e\n",
                            patches ? "patch" : "range", c[0], c[1], int(P.fits), P.tiles, bad, int(P.q_fits), qe);
            }
        // multicolour plans: {tile size, staging cap, update cap, sweeps per pass}
        const int mc_shapes[][4] = {{128, 1024, 512, 1}, {512, 2048, 1024, 1}, {512, 2048, 1024, 2},
                                    {256, 2048, 1024, 3}, {1024, 4096, 2048, 2}};
        for (int patches = 0; patches < 2; ++patches)
            for (const auto &c : mc_shapes) {
                Mesh::MCPlan P = lms::mc_plan(M, c[0], c[1], c[2], patches != 0, c[3]);
                if (planted && P.fits) plant(P, M.ell_w);
                long bad = 0;
                double qe = -1.0;
                if (P.fits) {
                    for (int d = 1; d <= P.k; ++d)
                        bad += count_mismatches(mc_pass(M, P, p0, d), multicolour(M, p0, d));
                    lms::mc_quality_plan(M, P);
                    auto row_of = [&](int32_t t, int32_t sl) {
                        const int32_t nown = P.tile_ptr[size_t(t) + 1] - P.tile_ptr[size_t(t)];
                        if (P.patches) return P.halo[size_t(P.halo_ptr[size_t(t)] + sl)];
                        return sl < nown ? P.tile_ptr[size_t(t)] + sl : P.halo[size_t(P.halo_ptr[size_t(t)] + sl - nown)];
                    };
                    if (planted && P.q_fits) plant_weight(M, P, row_of);
                    if (P.q_fits) qe = q_err(quality_sum_plan(P, row_of, xc, yc));
                }
                total_bad += bad;
                std::printf("mc %s ts=%d k=%d fits=%d tiles=%d mismatches=%ld q_fits=%d q_err=%.3e\n",
                            patches ? "patch" : "range", c[0], c[3], int(P.fits), P.tiles, bad, int(P.q_fits), qe);
            }
    } catch (const lms::Error &e) {
        std::printf("FAIL %s\n", e.msg.c_str());
        return 1;
    }
    return total_bad == 0 ? 0 : 1;
}
