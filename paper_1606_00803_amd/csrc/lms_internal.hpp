// Internal state of a mesh handle, shared by the host logic (lms_host.cpp)
// and the device runtime (lms_device.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <deque>
#include <vector>

#include "lms.h"

namespace lms {

// Error carried from the internals to the C boundary.
struct Error {
    lms_status code;
    std::string msg;
};

[[noreturn]] void fail(lms_status code, const std::string &msg);

struct DeviceState;  // defined in lms_device.hip
void destroy_device_state(DeviceState *d);

struct DeviceDeleter {
    void operator()(DeviceState *d) const { destroy_device_state(d); }
};

struct ReorderState;  // defined in lms_reorder.hip
void destroy_reorder_state(ReorderState *r);

struct ReorderDeleter {
    void operator()(ReorderState *r) const { destroy_reorder_state(r); }
};

// Everything the host knows about a mesh.  Arrays suffixed 0 are in INPUT
// labels and never change after the build; the rest follow the current
// ordering and are rebuilt by relabel().
struct Mesh {
    // ---- input labelling ----
    int32_t n = 0;
    int64_t T = 0;
    std::vector<int32_t> tri0;              // 3T
    std::vector<uint8_t> fixed0;            // n
    std::vector<int64_t> adj_ptr0;          // n+1, full adjacency
    std::vector<int32_t> adj0;              // ascending neighbours
    std::vector<int32_t> tcount0;           // triangles per vertex
    std::vector<int64_t> vt_ptr0;           // vertex -> triangles (ascending triangle index)
    std::vector<int32_t> vt0;
    std::vector<int32_t> color0;            // -1 for fixed vertices
    int32_t n_colors = 0;
    int32_t n_free = 0;
    int32_t max_degree = 0;
    // batched layout (n_mesh == 1 for a plain mesh)
    int32_t n_mesh = 1;
    std::vector<int64_t> v_off, t_off;      // n_mesh+1 each

    // ---- current labelling ----
    lms_ordering ordering = LMS_ORI;
    std::vector<int32_t> new2old, old2new;
    std::vector<int32_t> row_ptr;           // n+1, smoothing adjacency
    std::vector<int32_t> col;               // nnz
    int32_t ell_w = 0;                      // padded width (8, 12 or 16), 0 = no padded copy
    std::vector<int32_t> ell;               // ell[v*ell_w + k]: entry k of row v, -1 past its end
    std::vector<uint8_t> fixed;             // n
    std::vector<int32_t> color;             // n
    std::vector<int32_t> color_ptr;         // n_colors+1
    std::vector<int32_t> color_list;        // free vertices grouped by colour, ascending
    std::vector<int32_t> color_ell;         // colour-major padded neighbours: for the vertex at
                                            // color_list[color_ptr[c] + i], entry k sits at
                                            // color_ell[ell_w*color_ptr[c] + k*cnt_c + i] (-1 past the row)
    std::vector<int32_t> ta, tb, tc;        // triangles (current labels), sorted for locality
    std::vector<double> tw;                 // per-triangle weight of the global mean
    std::vector<int32_t> trec;              // 4 per triangle: corners a, b, c and the three
                                            // triangle counts |T(v)| packed 10 bits each (empty
                                            // when a count exceeds 1023)
    std::vector<int32_t> tmesh;             // mesh index of each triangle (current order)
    std::vector<int32_t> vt_ptr, vt;        // vertex -> triangles in current labels/order

    // Tile plans of the halo-staged sweep, built on first use for a tile size
    // and dropped by relabel().  Tile t owns rows [t*ts, (t+1)*ts); its halo is
    // the sorted list of neighbours outside that range; lidx holds, per tile
    // row and entry k (row-major, lidx[(t*ts + r)*ell_w + k]), the neighbour's slot in
    // the tile's staging area: own rows at 0..ts-1, halo vertices from ts on,
    // 0xFFFF past the row's end.
    struct HaloPlan {
        int32_t ts = 0;
        int32_t h_max = 0;
        std::vector<int32_t> halo_ptr;  // tiles+1
        std::vector<int32_t> halo;      // concatenated halo lists
        std::vector<uint16_t> lidx;     // tiles * ell_w * ts
        uint64_t version = ~uint64_t(0);
    };
    std::deque<HaloPlan> halo_plans;  // deque: references stay valid as plans are added

    // Tile plan of the temporally blocked sweep (k Jacobi sweeps per pass).
    // Tiles are ranges of consecutive rows: nominally ts rows, halved until
    // the tile's first sweep updates at most u_cap rows and its staging area
    // holds at most l_cap rows.  Tile t stages its own rows (local slots
    // 0..own-1) and k halo rings: ring 1 holds the outside neighbours of its
    // rows, ring m+1 the neighbours of ring m's free rows not staged yet, each
    // ring in ascending id.  ring[t*(k+1)+m] counts the rows of own + rings
    // 1..m.  Sweep j of a pass of k' <= k sweeps updates the rows below
    // ring[t*(k+1)+k'-j]; their padded slots (0xFFFF past a row's end) come
    // first in the tile's lidx block.  fits is false when even a one-row
    // tile exceeds the caps (the plan is then empty).
    // Tiles are either ranges of consecutive rows (patches = false) or
    // compact patches of free rows grown breadth-first over the adjacency
    // (patches = true): then the own rows are listed too, ascending, ahead of
    // the rings in `halo`, and tile_ptr counts own rows.
    struct TBPlan {
        int32_t ts = 0, k = 0, u_cap = 0, l_cap = 0;
        bool patches = false;
        bool fits = true;
        int32_t tiles = 0;
        int32_t l_max = 0;  // largest staging area (rows), over tiles
        int32_t u_max = 0;  // largest first-sweep update set (rows), over tiles
        std::vector<int32_t> tile_ptr;  // tiles+1: first own row of each tile (patches: prefix of own counts)
        std::vector<int32_t> ring;      // tiles * (k+1)
        std::vector<int64_t> halo_ptr;  // tiles+1, into halo
        std::vector<int32_t> halo;      // per tile: rings 1..k (patches: own rows, then rings 1..k)
        std::vector<int64_t> lidx_ptr;  // tiles+1, in rows of ell_w slots
        std::vector<uint16_t> lidx;
        // Quality of each staged state (filled by tb_quality_plan): every
        // triangle with a free corner belongs to the tile that owns its
        // smallest free corner, whose neighbours (the other two corners) are
        // staged in its own rows or ring 1.  Record: 3 words, slots a | b<<16,
        // c | |T(a)|<<16, |T(b)| | |T(c)|<<16 (corners in the order of ta,
        // tb, tc).  Triangles whose corners are all fixed never change; they
        // are listed apart in current labels with their weights.
        bool q_built = false, q_fits = false;
        std::vector<int64_t> qtri_ptr;  // tiles+1, in triangles
        std::vector<uint32_t> qtri;     // 3 words per triangle
        std::vector<int32_t> qc_ids;    // 3 per all-fixed triangle
        std::vector<double> qc_w;       // its weight 1/|T(a)| + 1/|T(b)| + 1/|T(c)|
        uint64_t version = ~uint64_t(0);
    };
    std::deque<TBPlan> tb_plans;
    // breadth-first patches of up to ts free rows (shared by the plans of one
    // tile size): rows of patch i at patch_rows[patch_ptr[i] .. patch_ptr[i+1])
    struct Patches {
        int32_t ts = 0;
        uint64_t version = ~uint64_t(0);
        std::vector<int64_t> patch_ptr;
        std::vector<int32_t> patch_rows;
    };
    std::deque<Patches> patch_sets;

    // Tile plan of the multicolour sweep in one pass (all colours of one
    // sweep, tile by tile, in LDS).  Tiles are row ranges (ts rows, halved
    // until the staging area fits l_cap and the updated rows u_cap).  A tile updates its own free rows
    // and every free halo vertex that an updated vertex of a higher colour
    // reads (a closure along strictly decreasing colours), and stages the
    // neighbours of everything it updates.  Local slots: own rows first,
    // then the other staged vertices in ascending id.  The updated rows of
    // tile t are listed by colour: upd_ptr[t*(C+1)+c] .. upd_ptr[t*(C+1)+c+1]
    // index urow (their slot) and uidx (ell_w neighbour slots each, 0xFFFF
    // past the row's end, in the row's order).
    struct MCPlan {
        int32_t ts = 0, l_cap = 0, u_cap = 0;
        bool patches = false;  // tiles are breadth-first patches of free rows (as for TBPlan)
        int32_t k = 1;         // multicolour sweeps per pass (a pass of depth d runs the last d)
        bool fits = true;
        int32_t tiles = 0, l_max = 0, colors = 0;
        std::vector<int32_t> tile_ptr;  // tiles+1 (patches: prefix of own counts)
        std::vector<int64_t> halo_ptr;  // tiles+1
        std::vector<int32_t> halo;      // staged ids beyond the own rows (patches: own rows first)
        std::vector<int64_t> upd_ptr;   // tiles*(C+1)
        std::vector<uint16_t> urow, uidx;
        std::vector<uint8_t> umask;     // per updated row: bit t-1 set when sweep t of the pass updates it
        // quality evaluated in the pass (as for TBPlan, slots into this
        // plan's staging area); filled by mc_quality_plan
        bool q_built = false, q_fits = false;
        std::vector<int64_t> qtri_ptr;
        std::vector<uint32_t> qtri;
        std::vector<int32_t> qc_ids;
        std::vector<double> qc_w;
        uint64_t version = ~uint64_t(0);
    };
    std::deque<MCPlan> mc_plans;

    // generation counter: bumped whenever the current labelling changes so
    // that device copies and captured graphs are refreshed
    uint64_t version = 0;

    std::unique_ptr<DeviceState, DeviceDeleter> dev;
    std::unique_ptr<ReorderState, ReorderDeleter> rdev;  // input arrays for the device reorder
};

// ---- host logic (lms_host.cpp) ----
void build_mesh(Mesh &M, int32_t n, int64_t T, const int32_t *tri, const uint8_t *fixed,
                int32_t n_mesh, const int64_t *v_off, const int64_t *t_off);
void vertex_quality_host(const Mesh &M, const double *x, const double *y, double *q);
std::vector<int32_t> order_bfs(const Mesh &M);
std::vector<int32_t> order_rdr(const Mesh &M, const double *q);
std::vector<int32_t> order_random(const Mesh &M, uint64_t seed);
void relabel(Mesh &M, lms_ordering kind, std::vector<int32_t> new2old);
// Install the arrays of a new labelling (colour lists built here).
void adopt_relabel(Mesh &M, lms_ordering kind, std::vector<int32_t> new2old, std::vector<int32_t> old2new,
                   std::vector<int32_t> row_ptr, std::vector<int32_t> col, int32_t ell_w, std::vector<int32_t> ell,
                   std::vector<uint8_t> fx, std::vector<int32_t> color, std::vector<int32_t> ta,
                   std::vector<int32_t> tb, std::vector<int32_t> tc, std::vector<double> tw,
                   std::vector<int32_t> trec, std::vector<int32_t> tmesh, std::vector<int32_t> vt_ptr,
                   std::vector<int32_t> vt);
const Mesh::HaloPlan &halo_plan(Mesh &M, int32_t ts);
const Mesh::TBPlan &tb_plan(Mesh &M, int32_t ts, int32_t k, int32_t u_cap, int32_t l_cap, bool patches = false);
void tb_quality_plan(const Mesh &M, Mesh::TBPlan &P);
const Mesh::MCPlan &mc_plan(Mesh &M, int32_t ts, int32_t l_cap, int32_t u_cap, bool patches = false,
                            int32_t k = 1);
const Mesh::Patches &patch_set(Mesh &M, int32_t ts);
void mc_quality_plan(const Mesh &M, Mesh::MCPlan &P);
void reuse_profile(const Mesh &M, int32_t trace, const double *fractions, int32_t nfrac, int64_t *quantiles,
                   int32_t line_bytes, int32_t record_bytes, lms_reuse_stats &out);

// ---- device runtime (lms_device.hip) ----
void dev_permute(Mesh &M, const void *sx, const void *sy, void *dx, void *dy,
                 lms_precision p, int inverse, void *stream);
void dev_sweep(Mesh &M, const void *sx, const void *sy, void *dx, void *dy,
               lms_precision p, void *stream);
void dev_smooth(Mesh &M, void *x, void *y, void *tx, void *ty, lms_precision p,
                lms_scheme s, const lms_smooth_opts &o, void *stream, lms_smooth_result &r);
std::string dev_sweep_config(Mesh &M, lms_precision p);
// ---- device reorder (lms_reorder.hip) ----
void dev_reorder(Mesh &M, lms_ordering kind, const std::vector<int32_t> &given, void *stream,
                 std::vector<int32_t> &new2old_out);
void dev_quality(Mesh &M, const void *x, const void *y, lms_precision p, double *q_global,
                 double *q_vertex, double *q_mesh, void *stream);
void dev_quality_noalloc(Mesh &M, const void *x, const void *y, lms_precision p, double *q_global_dev,
                         void *stream);

}  // namespace lms
