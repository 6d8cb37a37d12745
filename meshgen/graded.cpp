// Graded triangle meshes by newest-vertex bisection (input generator only).
//
// Builds a base grid of (n0 x n0) points with cell size 4 in integer
// reference coordinates, each cell split along a given diagonal into two
// right isosceles triangles whose refinement edge is the diagonal.  Then every
// triangle whose centroid lies within band_w[k] of any of the given curves
// y = 0.5 + A sin(2 pi f x + phi) (unit-square coordinates) is bisected until
// it reaches band_level[k] bisections; conformity is kept by the usual
// newest-vertex-bisection closure (a triangle whose refinement edge is not
// shared as its neighbour's refinement edge first bisects that neighbour).
// Four bisections quarter the edge length, so all vertices stay on the
// integer lattice.  Vertices are numbered in creation order (base grid
// row-major first), triangles are the leaves in array order.
//
// This file holds no smoothing arithmetic; it only produces inputs.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

struct Tri {
    int32_t v[3];   // v[0] apex (newest vertex), v[1]-v[2] refinement edge
    int32_t nb[3];  // nb[k]: neighbour across the edge opposite v[k], -1 on the boundary
    int32_t level;
};

struct Gen {
    std::vector<int32_t> vx, vy;
    std::vector<Tri> tris;
    int ncurves = 0;
    const double *amp = nullptr, *freq = nullptr, *phase = nullptr;
    int nbands = 0;
    const double *band_w = nullptr;
    const int32_t *band_level = nullptr;
    double scale = 1.0;  // reference units per unit-square unit

    int32_t add_vertex(int32_t x, int32_t y) {
        vx.push_back(x);
        vy.push_back(y);
        return int32_t(vx.size() - 1);
    }

    void replace_nb(int32_t t, int32_t old_t, int32_t new_t) {
        if (t < 0) return;
        for (int k = 0; k < 3; ++k)
            if (tris[t].nb[k] == old_t) {
                tris[t].nb[k] = new_t;
                return;
            }
    }

    // Split t (apex a, refinement edge b-c) at vertex m into (m, a, b) kept in
    // slot t and (m, c, a) in a new slot.  Returns the new slot.  The links
    // across b-m and m-c are set by the caller.
    int32_t split(int32_t t, int32_t m) {
        const Tri old = tris[t];
        const int32_t a = old.v[0], b = old.v[1], c = old.v[2];
        const int32_t t2 = int32_t(tris.size());
        Tri c1, c2;
        c1.v[0] = m; c1.v[1] = a; c1.v[2] = b;
        c2.v[0] = m; c2.v[1] = c; c2.v[2] = a;
        c1.level = c2.level = old.level + 1;
        // c1 edges: opposite m = a-b (old nb[2]); opposite a = b-m (set later); opposite b = m-a (c2)
        c1.nb[0] = old.nb[2]; c1.nb[1] = -1; c1.nb[2] = t2;
        // c2 edges: opposite m = c-a (old nb[1]); opposite c = a-m (c1); opposite a = m-c (set later)
        c2.nb[0] = old.nb[1]; c2.nb[1] = t; c2.nb[2] = -1;
        tris[t] = c1;
        tris.push_back(c2);
        replace_nb(old.nb[1], t, t2);
        return t2;
    }

    void refine(int32_t t) {
        for (;;) {
            const int32_t s = tris[t].nb[0];
            if (s >= 0) {
                // compatible iff s's refinement edge is the same edge
                const Tri &S = tris[s];
                const int32_t b = tris[t].v[1], c = tris[t].v[2];
                const bool compat = (S.v[1] == c && S.v[2] == b) || (S.v[1] == b && S.v[2] == c);
                if (!compat) {
                    refine(s);
                    continue;  // t's neighbour across b-c changed: look again
                }
            }
            const int32_t b = tris[t].v[1], c = tris[t].v[2];
            const int32_t m = add_vertex((vx[b] + vx[c]) / 2, (vy[b] + vy[c]) / 2);
            const int32_t s2 = s;
            const int32_t t2 = split(t, m);  // t = (m,a,b), t2 = (m,c,a)
            if (s2 >= 0) {
                // the neighbour sees the edge as (c, b): its children are
                // (m, a', c) in slot s2 and (m, b, a') in slot u2
                const int32_t u2 = split(s2, m);
                // t (edge b-m, opposite a = index 1) <-> u2 (edge m-b, opposite a' = index 2)
                tris[t].nb[1] = u2;
                tris[u2].nb[2] = t;
                // t2 (edge m-c, opposite a = index 2) <-> s2 (edge c-m, opposite a' = index 1)
                tris[t2].nb[2] = s2;
                tris[s2].nb[1] = t2;
            }
            return;
        }
    }

    int target_level(const Tri &T) const {
        const double cx = (vx[T.v[0]] + vx[T.v[1]] + vx[T.v[2]]) / (3.0 * scale);
        const double cy = (vy[T.v[0]] + vy[T.v[1]] + vy[T.v[2]]) / (3.0 * scale);
        int lv = 0;
        for (int k = 0; k < ncurves; ++k) {
            const double w = 2.0 * M_PI * freq[k];
            const double yc = 0.5 + amp[k] * std::sin(w * cx + phase[k]);
            const double slope = amp[k] * w * std::cos(w * cx + phase[k]);
            const double d = std::fabs(cy - yc) / std::sqrt(1.0 + slope * slope);
            for (int b = 0; b < nbands; ++b)
                if (d <= band_w[b] && band_level[b] > lv) lv = band_level[b];
        }
        return lv;
    }
};

}  // namespace

extern "C" {

// Returns the number of vertices (>= 0) or -1 on bad arguments.  Results are
// kept until graded_fetch copies them out.
static Gen *g_last = nullptr;

int64_t graded_build(int32_t n0, const uint8_t *diag_ac, int32_t ncurves, const double *amp,
                     const double *freq, const double *phase, int32_t nbands, const double *band_w,
                     const int32_t *band_level, int64_t *n_tri_out) {
    if (n0 < 2 || ncurves < 0 || nbands < 0) return -1;
    delete g_last;
    g_last = new Gen();
    Gen &G = *g_last;
    G.ncurves = ncurves;
    G.amp = amp;
    G.freq = freq;
    G.phase = phase;
    G.nbands = nbands;
    G.band_w = band_w;
    G.band_level = band_level;
    const int32_t cell = 4;
    G.scale = double(cell) * double(n0 - 1);
    G.vx.reserve(size_t(n0) * n0 * 4);
    G.vy.reserve(size_t(n0) * n0 * 4);
    for (int32_t i = 0; i < n0; ++i)
        for (int32_t j = 0; j < n0; ++j) G.add_vertex(j * cell, i * cell);
    const int32_t nc = n0 - 1;
    G.tris.resize(size_t(2) * nc * nc);
    // cell (i,j): corners a=(i,j) b=(i,j+1) c=(i+1,j+1) d=(i+1,j); triangle
    // slots 2*(i*nc+j) and +1, all counter-clockwise (so two neighbours walk
    // their shared edge in opposite directions, and bisection keeps that).
    // Diagonal a-c: T0=(apex b; c,a) T1=(apex d; a,c).  Diagonal b-d:
    // T0=(apex a; b,d) T1=(apex c; d,b).  Edge neighbours are linked after
    // all triangles exist.
    for (int32_t i = 0; i < nc; ++i)
        for (int32_t j = 0; j < nc; ++j) {
            const int32_t a = i * n0 + j, b = a + 1, c = a + n0 + 1, d = a + n0;
            Tri &T0 = G.tris[2 * size_t(i * nc + j)];
            Tri &T1 = G.tris[2 * size_t(i * nc + j) + 1];
            if (diag_ac[size_t(i) * nc + j]) {
                T0 = Tri{{b, c, a}, {-1, -1, -1}, 0};
                T1 = Tri{{d, a, c}, {-1, -1, -1}, 0};
            } else {
                T0 = Tri{{a, b, d}, {-1, -1, -1}, 0};
                T1 = Tri{{c, d, b}, {-1, -1, -1}, 0};
            }
        }
    // neighbours: the two halves of a cell share the diagonal (opposite the
    // apex); axis edges pair with the adjacent cell's triangle on that edge
    auto tri_with_edge = [&](int32_t ci, int32_t cj, int32_t p, int32_t q, int32_t &slot, int &k) {
        for (int h = 0; h < 2; ++h) {
            const int32_t t = 2 * (ci * nc + cj) + h;
            const Tri &T = G.tris[t];
            for (int e = 0; e < 3; ++e) {
                const int32_t u = T.v[(e + 1) % 3], w = T.v[(e + 2) % 3];
                if ((u == p && w == q) || (u == q && w == p)) {
                    slot = t;
                    k = e;
                    return;
                }
            }
        }
        slot = -1;
        k = -1;
    };
    for (int32_t i = 0; i < nc; ++i)
        for (int32_t j = 0; j < nc; ++j) {
            const int32_t t0 = 2 * (i * nc + j), t1 = t0 + 1;
            G.tris[t0].nb[0] = t1;
            G.tris[t1].nb[0] = t0;
            const int32_t a = i * n0 + j, b = a + 1, d = a + n0;
            int32_t s1, s2;
            int k1, k2;
            if (j + 1 < nc) {  // vertical edge b-(b+n0) shared with cell (i, j+1)
                tri_with_edge(i, j, b, b + n0, s1, k1);
                tri_with_edge(i, j + 1, b, b + n0, s2, k2);
                G.tris[s1].nb[k1] = s2;
                G.tris[s2].nb[k2] = s1;
            }
            if (i + 1 < nc) {  // horizontal edge d-(d+1) shared with cell (i+1, j)
                tri_with_edge(i, j, d, d + 1, s1, k1);
                tri_with_edge(i + 1, j, d, d + 1, s2, k2);
                G.tris[s1].nb[k1] = s2;
                G.tris[s2].nb[k2] = s1;
            }
            (void)a;
        }
    // refine until every leaf reaches its target level
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t t = 0; t < G.tris.size(); ++t) {
            while (G.tris[t].level < G.target_level(G.tris[t])) {
                G.refine(int32_t(t));
                changed = true;
            }
        }
    }
    *n_tri_out = int64_t(G.tris.size());
    return int64_t(G.vx.size());
}

// Copy out the last mesh: vertex integer coordinates (x, y in units of
// 1/(4*(n0-1)) of the unit square) and triangles (counter-clockwise).
void graded_fetch(int32_t *x, int32_t *y, int32_t *tri) {
    Gen &G = *g_last;
    std::memcpy(x, G.vx.data(), sizeof(int32_t) * G.vx.size());
    std::memcpy(y, G.vy.data(), sizeof(int32_t) * G.vy.size());
    for (size_t t = 0; t < G.tris.size(); ++t) {
        const Tri &T = G.tris[t];
        const int64_t ax = G.vx[T.v[0]], ay = G.vy[T.v[0]];
        const int64_t bx = G.vx[T.v[1]], by = G.vy[T.v[1]];
        const int64_t cx = G.vx[T.v[2]], cy = G.vy[T.v[2]];
        const int64_t cross = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
        tri[3 * t] = T.v[0];
        tri[3 * t + 1] = cross > 0 ? T.v[1] : T.v[2];
        tri[3 * t + 2] = cross > 0 ? T.v[2] : T.v[1];
    }
}

// Shortest edge (reference units) of the triangles around each vertex,
// over the triangle list given (vertex ids < n).
void graded_min_edge(int64_t n, int64_t ntri, const int32_t *x, const int32_t *y, const int32_t *tri,
                     double *out) {
    for (int64_t v = 0; v < n; ++v) out[v] = 1e300;
    for (int64_t t = 0; t < ntri; ++t) {
        for (int e = 0; e < 3; ++e) {
            const int32_t a = tri[3 * t + e], b = tri[3 * t + (e + 1) % 3];
            const double dx = double(x[b]) - double(x[a]), dy = double(y[b]) - double(y[a]);
            const double len = std::sqrt(dx * dx + dy * dy);
            if (len < out[a]) out[a] = len;
            if (len < out[b]) out[b] = len;
        }
    }
}

void graded_free(void) {
    delete g_last;
    g_last = nullptr;
}

}  // extern "C"
