// The C ABI (include/lms.h): argument checks, status codes and the
// thread-local error message around the host and device internals.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>

#include "lms_internal.hpp"

namespace {

thread_local std::string g_error;

template <class F>
lms_status guarded(F &&f) {
    try {
        g_error.clear();
        f();
        return LMS_OK;
    } catch (const lms::Error &e) {
        g_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_error = "host allocation failed";
        return LMS_ERR_ALLOC;
    } catch (const std::exception &e) {
        g_error = std::string("internal error: ") + e.what();
        return LMS_ERR_STATE;
    } catch (...) {
        g_error = "internal error";
        return LMS_ERR_STATE;
    }
}

lms::Mesh &mesh_of(lms_mesh_t m) {
    if (!m) lms::fail(LMS_ERR_ARG, "mesh handle is NULL");
    return *reinterpret_cast<lms::Mesh *>(m);
}

void check_finite(const double *a, int32_t n, const char *what) {
    for (int32_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) lms::fail(LMS_ERR_ARG, std::string(what) + " holds a non-finite value");
}

std::vector<int32_t> make_order(lms::Mesh &M, lms_ordering kind, uint64_t seed, const double *x0,
                                const double *y0, const double *q_given) {
    switch (kind) {
        case LMS_ORI: {
            std::vector<int32_t> p(static_cast<size_t>(M.n));
            for (int32_t i = 0; i < M.n; ++i) p[i] = i;
            return p;
        }
        case LMS_BFS:
            return lms::order_bfs(M);
        case LMS_RANDOM:
            return lms::order_random(M, seed);
        case LMS_RDR: {
            if (q_given) return lms::order_rdr(M, q_given);
            if (!x0 || !y0) lms::fail(LMS_ERR_ARG, "RDR needs the input coordinates x0, y0");
            check_finite(x0, M.n, "x0");
            check_finite(y0, M.n, "y0");
            std::vector<double> q(static_cast<size_t>(M.n));
            lms::vertex_quality_host(M, x0, y0, q.data());
            return lms::order_rdr(M, q.data());
        }
    }
    lms::fail(LMS_ERR_ARG, "unknown ordering");
}

}  // namespace

extern "C" {

void lms_smooth_opts_default(lms_smooth_opts *o) {
    if (!o) return;
    o->max_iters = 1000;
    o->check_quality = 1;
    o->tol = 5e-6;
    o->goal = std::numeric_limits<double>::infinity();
    o->q_prev = std::numeric_limits<double>::quiet_NaN();
}

lms_status lms_build_csr(int32_t n, int64_t n_tri, const int32_t *tri, const uint8_t *fixed, lms_mesh_t *out) {
    return guarded([&] {
        if (!out) lms::fail(LMS_ERR_ARG, "out is NULL");
        auto M = std::make_unique<lms::Mesh>();
        const int64_t v_off[2] = {0, n};
        const int64_t t_off[2] = {0, n_tri};
        lms::build_mesh(*M, n, n_tri, tri, fixed, 1, v_off, t_off);
        *out = reinterpret_cast<lms_mesh_t>(M.release());
    });
}

lms_status lms_build_csr_batched(int32_t n_mesh, const int64_t *v_off, const int64_t *t_off, const int32_t *tri,
                                 const uint8_t *fixed, lms_mesh_t *out) {
    return guarded([&] {
        if (!out) lms::fail(LMS_ERR_ARG, "out is NULL");
        if (n_mesh <= 0) lms::fail(LMS_ERR_ARG, "n_mesh must be positive");
        if (!v_off || !t_off) lms::fail(LMS_ERR_ARG, "v_off and t_off are required");
        if (v_off[0] != 0 || t_off[0] != 0) lms::fail(LMS_ERR_ARG, "v_off[0] and t_off[0] must be 0");
        for (int32_t i = 0; i < n_mesh; ++i) {
            if (v_off[i + 1] <= v_off[i]) lms::fail(LMS_ERR_ARG, "every mesh needs at least one vertex");
            if (t_off[i + 1] <= t_off[i]) lms::fail(LMS_ERR_ARG, "every mesh needs at least one triangle");
        }
        if (v_off[n_mesh] >= (int64_t(1) << 31)) lms::fail(LMS_ERR_ARG, "total vertex count must be < 2^31");
        auto M = std::make_unique<lms::Mesh>();
        lms::build_mesh(*M, int32_t(v_off[n_mesh]), t_off[n_mesh], tri, fixed, n_mesh, v_off, t_off);
        *out = reinterpret_cast<lms_mesh_t>(M.release());
    });
}

lms_status lms_reorder(lms_mesh_t m, lms_ordering kind, uint64_t seed, const double *x0, const double *y0,
                       int32_t *new2old) {
    return guarded([&] {
        lms::Mesh &M = mesh_of(m);
        std::vector<int32_t> p = make_order(M, kind, seed, x0, y0, nullptr);
        lms::relabel(M, kind, p);
        if (new2old) std::memcpy(new2old, p.data(), sizeof(int32_t) * size_t(M.n));
    });
}

lms_status lms_reorder_device(lms_mesh_t m, lms_ordering kind, uint64_t seed, const double *x0, const double *y0,
                              int32_t *new2old, void *stream) {
    return guarded([&] {
        lms::Mesh &M = mesh_of(m);
        std::vector<int32_t> given;
        if (kind != LMS_BFS) given = make_order(M, kind, seed, x0, y0, nullptr);
        std::vector<int32_t> p;
        lms::dev_reorder(M, kind, given, stream, p);
        if (new2old) std::memcpy(new2old, p.data(), sizeof(int32_t) * size_t(M.n));
    });
}

lms_status lms_reorder_with_quality(lms_mesh_t m, const double *q, int32_t *new2old) {
    return guarded([&] {
        lms::Mesh &M = mesh_of(m);
        if (!q) lms::fail(LMS_ERR_ARG, "q is NULL");
        check_finite(q, M.n, "q");
        std::vector<int32_t> p = make_order(M, LMS_RDR, 0, nullptr, nullptr, q);
        lms::relabel(M, LMS_RDR, p);
        if (new2old) std::memcpy(new2old, p.data(), sizeof(int32_t) * size_t(M.n));
    });
}

lms_status lms_permute(lms_mesh_t m, const void *sx, const void *sy, void *dx, void *dy, lms_precision p,
                       int32_t inverse, void *stream) {
    return guarded([&] { lms::dev_permute(mesh_of(m), sx, sy, dx, dy, p, inverse != 0, stream); });
}

lms_status lms_smooth(lms_mesh_t m, void *x, void *y, void *tx, void *ty, lms_precision p, lms_scheme s,
                      const lms_smooth_opts *o, void *stream, lms_smooth_result *r) {
    return guarded([&] {
        lms::Mesh &M = mesh_of(m);
        lms_smooth_opts opts;
        if (o)
            opts = *o;
        else
            lms_smooth_opts_default(&opts);
        lms_smooth_result res{};
        lms::dev_smooth(M, x, y, tx, ty, p, s, opts, stream, res);
        if (r) *r = res;
    });
}

lms_status lms_sweep(lms_mesh_t m, const void *sx, const void *sy, void *dx, void *dy, lms_precision p,
                     void *stream) {
    return guarded([&] { lms::dev_sweep(mesh_of(m), sx, sy, dx, dy, p, stream); });
}

lms_status lms_quality(lms_mesh_t m, const void *x, const void *y, lms_precision p, double *q_global,
                       double *q_vertex, void *stream) {
    return guarded([&] { lms::dev_quality(mesh_of(m), x, y, p, q_global, q_vertex, nullptr, stream); });
}

lms_status lms_quality_noalloc(lms_mesh_t m, const void *x, const void *y, lms_precision p, double *q_global,
                               void *stream) {
    return guarded([&] { lms::dev_quality_noalloc(mesh_of(m), x, y, p, q_global, stream); });
}

lms_status lms_quality_batched(lms_mesh_t m, const void *x, const void *y, lms_precision p, double *q_mesh,
                               void *stream) {
    return guarded([&] {
        if (!q_mesh) lms::fail(LMS_ERR_ARG, "q_mesh is NULL");
        lms::dev_quality(mesh_of(m), x, y, p, nullptr, nullptr, q_mesh, stream);
    });
}

lms_status lms_sweep_config(lms_mesh_t m, lms_precision p, char *buf, int32_t len) {
    return guarded([&] {
        if (!buf || len <= 0) lms::fail(LMS_ERR_ARG, "buffer is NULL or empty");
        const std::string s = lms::dev_sweep_config(mesh_of(m), p);
        const size_t k = std::min(s.size(), size_t(len - 1));
        std::memcpy(buf, s.data(), k);
        buf[k] = 0;
    });
}

lms_status lms_destroy(lms_mesh_t m) {
    return guarded([&] { delete reinterpret_cast<lms::Mesh *>(m); });
}

const char *lms_last_error(void) { return g_error.c_str(); }

lms_status lms_get_info(lms_mesh_t m, lms_mesh_info *info) {
    return guarded([&] {
        const lms::Mesh &M = mesh_of(m);
        if (!info) lms::fail(LMS_ERR_ARG, "info is NULL");
        info->n = M.n;
        info->n_free = M.n_free;
        info->n_mesh = M.n_mesh;
        info->n_colors = M.n_colors;
        info->n_tri = M.T;
        info->nnz_full = int64_t(M.adj0.size());
        info->nnz = int64_t(M.col.size());
        info->ordering = int32_t(M.ordering);
        info->max_degree = M.max_degree;
    });
}

lms_status lms_get_csr(lms_mesh_t m, int32_t *row_ptr, int32_t *col) {
    return guarded([&] {
        const lms::Mesh &M = mesh_of(m);
        if (row_ptr) std::memcpy(row_ptr, M.row_ptr.data(), sizeof(int32_t) * M.row_ptr.size());
        if (col && !M.col.empty()) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.col.size());
    });
}

lms_status lms_get_vertex_data(lms_mesh_t m, uint8_t *fixed, int32_t *color) {
    return guarded([&] {
        const lms::Mesh &M = mesh_of(m);
        if (fixed) std::memcpy(fixed, M.fixed.data(), size_t(M.n));
        if (color) std::memcpy(color, M.color.data(), sizeof(int32_t) * size_t(M.n));
    });
}

lms_status lms_get_order(lms_mesh_t m, int32_t *new2old) {
    return guarded([&] {
        const lms::Mesh &M = mesh_of(m);
        if (!new2old) lms::fail(LMS_ERR_ARG, "new2old is NULL");
        std::memcpy(new2old, M.new2old.data(), sizeof(int32_t) * size_t(M.n));
    });
}

lms_status lms_host_vertex_quality(lms_mesh_t m, const double *x, const double *y, double *q) {
    return guarded([&] {
        const lms::Mesh &M = mesh_of(m);
        if (!x || !y || !q) lms::fail(LMS_ERR_ARG, "null pointer");
        lms::vertex_quality_host(M, x, y, q);
    });
}

lms_status lms_reuse_profile(lms_mesh_t m, const double *fractions, int32_t nfrac, int64_t *quantiles,
                             int32_t line_bytes, int32_t record_bytes, lms_reuse_stats *stats) {
    return guarded([&] {
        if (!stats) lms::fail(LMS_ERR_ARG, "null stats");
        lms::reuse_profile(mesh_of(m), 0, fractions, nfrac, quantiles, line_bytes, record_bytes, *stats);
    });
}

lms_status lms_reuse_profile_trace(lms_mesh_t m, int32_t trace, const double *fractions, int32_t nfrac,
                                   int64_t *quantiles, int32_t line_bytes, int32_t record_bytes,
                                   lms_reuse_stats *stats) {
    return guarded([&] {
        if (!stats) lms::fail(LMS_ERR_ARG, "null stats");
        lms::reuse_profile(mesh_of(m), trace, fractions, nfrac, quantiles, line_bytes, record_bytes, *stats);
    });
}

}  // extern "C"
