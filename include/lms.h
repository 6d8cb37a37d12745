/*
 * lms.h -- Laplacian mesh smoothing on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the smoothing library.  The method is that of Aupy, Park and
 * Raghavan, "Locality-Aware Laplacian Mesh Smoothing" (arXiv 1606.00803):
 *
 *   - every free (interior) vertex of a 2D triangle mesh moves to the mean of
 *     its edge-adjacent neighbours (Eq. 1, Section 3.2), boundary vertices
 *     stay fixed, and sweeps repeat until the mesh quality stops improving
 *     by at least a tolerance, reaches a goal, or an iteration cap is hit
 *     (Algorithm 1; Section 5.1 uses a tolerance of 0.000005);
 *   - quality is the edge-length ratio (shortest / longest edge) per
 *     triangle, averaged per vertex over its triangles, averaged over all
 *     vertices (Section 3.2, Algorithm 1);
 *   - before smoothing, the vertices may be relabelled by one of four
 *     orderings: ORI (as generated), BFS, RDR (Algorithm 2, Section 4.2)
 *     or a random permutation (Figure 1).
 *
 * Conventions for every entry point:
 *   - Sizes and ids are int32 (vertex ids, n < 2^31) or int64 (counts of
 *     triangles and of adjacency entries).
 *   - "host" pointers are ordinary CPU memory owned by the caller; the library
 *     copies what it needs before returning.  "device" pointers are GPU
 *     memory (hipMalloc or a PyTorch CUDA tensor's data_ptr) owned by the
 *     caller.  Coordinates are structure-of-arrays: x[n] and y[n], float64
 *     (LMS_FP64) or float32 (LMS_FP32).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued on it.  Calls that return host results
 *     synchronise that stream before returning.
 *   - Every call returns an lms_status; on failure nothing the caller owns is
 *     modified, the handle keeps its previous state, and lms_last_error()
 *     describes the failure.  No C++ exception crosses this boundary.
 *   - A handle may be used by one thread at a time.  Calls on the same handle
 *     from several threads, or overlapping calls on different streams that
 *     share the handle's internal buffers, race.
 */
#ifndef LMS_H
#define LMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque mesh handle.  Owns the adjacency, orderings, colouring, triangle
 * data, device copies, scratch buffers and captured graphs; lms_destroy
 * frees all of them. */
typedef struct lms_mesh_s *lms_mesh_t;

typedef enum {
    LMS_OK = 0,
    LMS_ERR_ARG = 1,    /* null pointer, bad enum, size out of range, aliased buffers, non-finite input */
    LMS_ERR_MESH = 2,   /* malformed triangle list (see lms_build_csr) */
    LMS_ERR_ALLOC = 3,  /* host or device allocation failed */
    LMS_ERR_HIP = 4,    /* a HIP runtime call failed (no device, launch or copy failure) */
    LMS_ERR_STATE = 5   /* call not valid for this handle (e.g. a different current device) */
} lms_status;

typedef enum { LMS_ORI = 0, LMS_BFS = 1, LMS_RDR = 2, LMS_RANDOM = 3 } lms_ordering;
typedef enum { LMS_FP64 = 0, LMS_FP32 = 1 } lms_precision;
typedef enum { LMS_JACOBI = 0, LMS_MULTICOLOR = 1 } lms_scheme;
typedef enum { LMS_STOP_MAX_ITERS = 0, LMS_STOP_TOL = 1, LMS_STOP_GOAL = 2 } lms_stop_reason;

/* Options of lms_smooth (Algorithm 1's loop and stopping rule). */
typedef struct {
    int32_t max_iters;     /* cap on the number of sweeps, >= 0 */
    int32_t check_quality; /* 0: run exactly max_iters sweeps and compute no quality;
                              1: evaluate Q after every sweep and stop by the rule below */
    double tol;            /* stop after sweep k when Q_k - Q_{k-1} < tol (paper: 5e-6) */
    double goal;           /* stop when Q_k >= goal; +inf disables */
    double q_prev;         /* NaN: Q_0 is computed from the input coordinates;
                              otherwise it is taken as Q_{k-1} of the first sweep (resume) */
} lms_smooth_opts;

/* Result of lms_smooth. */
typedef struct {
    int32_t iters;       /* sweeps performed */
    int32_t stopped_by;  /* lms_stop_reason */
    double q0;           /* Q before the first sweep (q_prev when given, NaN when not checked) */
    double q_final;      /* Q after the last sweep (NaN when not checked) */
    double last_dq;      /* Q_iters - Q_{iters-1} (NaN when not available) */
} lms_smooth_result;

/* Sizes of a handle, in its current labelling. */
typedef struct {
    int32_t n;          /* vertices */
    int32_t n_free;     /* free (interior) vertices: the ones that move */
    int32_t n_mesh;     /* meshes in the handle (1 unless built batched) */
    int32_t n_colors;   /* colours of the multicolour schedule */
    int64_t n_tri;      /* triangles */
    int64_t nnz_full;   /* entries of the full adjacency (every vertex's neighbours) */
    int64_t nnz;        /* entries of the smoothing adjacency (free rows only) */
    int32_t ordering;   /* lms_ordering currently applied */
    int32_t max_degree; /* largest neighbour count of a free vertex */
} lms_mesh_info;

/* Fills *o with the paper's settings: max_iters 1000, check_quality 1,
 * tol 5e-6, goal +inf, q_prev NaN. */
void lms_smooth_opts_default(lms_smooth_opts *o);

/* Build a mesh handle from a triangle list (Algorithm 1's inputs V and T;
 * neighbours of Eq. 1).
 *   n      vertices, 1 <= n < 2^31
 *   n_tri  triangles, >= 1
 *   tri    host int32[3*n_tri], vertex ids of each triangle, any orientation
 *   fixed  host uint8[n] (nonzero = vertex never moves), or NULL: then a
 *          vertex is fixed iff it is an endpoint of a boundary edge (an edge
 *          with exactly one incident triangle)
 *   out    receives the handle (ordering ORI: the input labels)
 * Builds the neighbour lists (distinct edge-adjacent vertices, ascending),
 * the smoothing adjacency (free rows only), triangle counts and weights, and
 * the multicolour schedule.  Host-only: touches no GPU.
 * LMS_ERR_MESH when an id is out of range, a triangle repeats a vertex, an
 * edge lies in more than two triangles or a vertex is in no triangle. */
lms_status lms_build_csr(int32_t n, int64_t n_tri, const int32_t *tri,
                         const uint8_t *fixed, lms_mesh_t *out);

/* Build one handle holding n_mesh independent meshes back to back (Algorithm
 * 1's inputs V and T for each mesh; neighbours of Eq. 1 within each mesh).
 *   v_off  host int64[n_mesh+1], v_off[0] = 0, mesh i owns vertices
 *          v_off[i] .. v_off[i+1]-1 (total < 2^31)
 *   t_off  host int64[n_mesh+1], mesh i owns triangles t_off[i] .. t_off[i+1]-1
 *   tri    host int32[3*t_off[n_mesh]] with MESH-LOCAL vertex ids
 *   fixed  host uint8[v_off[n_mesh]] or NULL (boundary-edge rule)
 * The handle smooths all meshes together; results equal those of each mesh
 * smoothed alone.  Orderings apply within each mesh. */
lms_status lms_build_csr_batched(int32_t n_mesh, const int64_t *v_off, const int64_t *t_off,
                                 const int32_t *tri, const uint8_t *fixed, lms_mesh_t *out);

/* Relabel the handle's vertices by an ordering of the INPUT labels.
 *   kind     LMS_ORI (identity), LMS_BFS (breadth-first from label 0,
 *            neighbours ascending, restart at the smallest unvisited label),
 *            LMS_RDR (Algorithm 2 from the vertex qualities of (x0, y0); ties
 *            broken by label; fixed vertices Algorithm 2 leaves unordered are
 *            appended by continuing its loop over them), LMS_RANDOM
 *            (Fisher-Yates driven by SplitMix64(seed))
 *   seed     used by LMS_RANDOM only
 *   x0, y0   host float64[n] coordinates in INPUT labels (needed by LMS_RDR,
 *            ignored otherwise, may be NULL then)
 *   new2old  host int32[n] out, or NULL: position k holds input vertex new2old[k]
 * Replaces any earlier ordering (orderings do not compose).  Afterwards every
 * coordinate array passed to the handle must be in the new labels (see
 * lms_permute).  Batched handles order each mesh within its own range.
 * Host-only.  LMS_ERR_ARG when RDR lacks coordinates or they are not finite. */
lms_status lms_reorder(lms_mesh_t m, lms_ordering kind, uint64_t seed,
                       const double *x0, const double *y0, int32_t *new2old);

/* lms_reorder with the work on the GPU: LMS_BFS's breadth-first search
 * (level-synchronous, one search from the smallest label of every component
 * at once) and, for every kind, the relabelling of the handle's arrays (the
 * permutation apply of Algorithm 2's V_new <- V: smoothing adjacency, padded
 * copies, triangles, vertex-to-triangle lists).  RDR's walk and the random
 * shuffle stay sequential on the host.  The resulting ordering and every
 * array equal lms_reorder's, bit for bit.  Synchronous on `stream` (the
 * current device); same arguments and errors as lms_reorder. */
lms_status lms_reorder_device(lms_mesh_t m, lms_ordering kind, uint64_t seed,
                              const double *x0, const double *y0, int32_t *new2old, void *stream);

/* RDR (Algorithm 2) from given vertex qualities.
 *   q        host float64[n], quality per INPUT vertex
 *   new2old  host int32[n] out, or NULL
 * Same as lms_reorder(LMS_RDR) with q in place of the computed qualities. */
lms_status lms_reorder_with_quality(lms_mesh_t m, const double *q, int32_t *new2old);

/* Gather coordinates between input labels and the handle's current labels:
 * the permutation apply of Algorithm 2 (its V_new[next_num] <- V[i]) for
 * vertex data, so that the sweep of Eq. 1 runs on the reordered mesh, and its
 * inverse to bring results back (the Figure 4 caption: the smoothing itself
 * does not depend on the ordering).
 *   sx, sy  device source arrays [n];  dx, dy  device destinations [n]
 *   inverse 0: dx[k] = sx[new2old[k]] (input -> current labels)
 *           1: dx[new2old[k]] = sx[k] (current -> input labels)
 * Source and destination must not overlap. */
lms_status lms_permute(lms_mesh_t m, const void *sx, const void *sy, void *dx, void *dy,
                       lms_precision p, int32_t inverse, void *stream);

/* Smooth in place (Algorithm 1).
 *   x, y    device [n], current labels: P_0 in, final positions out
 *   tx, ty  device [n] scratch of the same precision for the Jacobi double
 *           buffer, or NULL (the handle allocates and keeps its own); must not
 *           overlap x, y.  Ignored by LMS_MULTICOLOR, which updates in place
 *           colour by colour (no two neighbours share a colour).
 *   p       LMS_FP64, or LMS_FP32 (coordinates stored and summed in float32;
 *           quality is always evaluated in float64)
 *   s       LMS_JACOBI (every free vertex reads the previous sweep's values)
 *           or LMS_MULTICOLOR
 *   o       options (NULL = lms_smooth_opts_default)
 *   r       host out, or NULL (filled on return)
 * Asynchronous on `stream`: x, y hold the result once the stream reaches the
 * end of the call.  Under the stopping rule the host reads the stop state
 * between chunks of sweeps, so that path waits for the stream as it runs.
 * Calls on one handle from different streams are ordered by the handle (each
 * waits for the previous call); the caller orders its own reads and writes of
 * x, y (and tx, ty) with the stream.
 * The first call per precision after a reorder tunes on the caller's stream
 * and waits for it: it times the sweep variants (and builds their tile plans
 * on the host), the one-launch path of a batch of small meshes, the one-pass
 * multicolour variants (LMS_MULTICOLOR), and, under the stopping rule, the
 * quality-fused passes.  Make that call before capturing work into a graph of
 * your own.  Every variant gives the same result bits. */
lms_status lms_smooth(lms_mesh_t m, void *x, void *y, void *tx, void *ty,
                      lms_precision p, lms_scheme s, const lms_smooth_opts *o,
                      void *stream, lms_smooth_result *r);

/* One Jacobi sweep (Eq. 1 for every free vertex) from (sx, sy) into (dx, dy),
 * device arrays [n] in current labels.  Fixed vertices of (dx, dy) are not
 * written.  Asynchronous on `stream`. */
lms_status lms_sweep(lms_mesh_t m, const void *sx, const void *sy, void *dx, void *dy,
                     lms_precision p, void *stream);

/* Mesh quality (Section 3.2, Algorithm 1) in float64.
 *   x, y      device [n], current labels
 *   q_global  host out: (1/n) * sum over vertices of the vertex qualities
 *             (for a batched handle: over all meshes together), or NULL
 *   q_vertex  device float64[n] out (current labels), or NULL
 * The stream is synchronised before return when q_global is requested. */
lms_status lms_quality(lms_mesh_t m, const void *x, const void *y, lms_precision p,
                       double *q_global, double *q_vertex, void *stream);

/* lms_quality for callers that cannot allocate device memory (code that a
 * caller captures into a graph, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating routine.  It
 * computes the global quality only, into device memory, and never waits for
 * the stream.
 *   x, y      device [n], current labels (float64 or float32 per p)
 *   q_global  device float64[1] out: the same value lms_quality returns, from
 *             the same kernels
 * Its partial sums live in a library-owned array of 8192 float64 (64 KiB)
 * that every GPU holds from the library's load until the process ends; every
 * mesh size fits it.  All calls on one GPU share that array, so calls that
 * overlap on one GPU (other streams, other threads, other handles) race:
 * order them.  The handle's mesh arrays must already be on the current
 * device: after building or reordering a handle, make one other device call
 * on it (lms_quality, lms_permute, lms_sweep or lms_smooth) first, else the
 * call fails with LMS_ERR_STATE.  LMS_ERR_ARG for a null pointer or an
 * unknown precision.  Asynchronous on `stream`. */
lms_status lms_quality_noalloc(lms_mesh_t m, const void *x, const void *y, lms_precision p,
                               double *q_global, void *stream);

/* Per-mesh quality of a batched handle (Section 3.2's mesh quality, Algorithm
 * 1's global mean, taken over each mesh's own vertices and triangles):
 * q_mesh host float64[n_mesh] out.  Same arguments and errors as lms_quality;
 * synchronises the stream. */
lms_status lms_quality_batched(lms_mesh_t m, const void *x, const void *y, lms_precision p,
                               double *q_mesh, void *stream);

/* Name of the sweep kernel variant a fixed-K Jacobi lms_smooth runs for
 * precision p (when that is a temporally blocked variant, k sweeps per pass,
 * the single-sweep variant used under the stopping rule follows it), then
 * the per-variant timings the autotuner measured, in microseconds per sweep
 * ("" until the first lms_smooth or lms_sweep of that precision since the
 * last reorder).  The first sweep call per precision and ordering times every
 * variant on the caller's stream (synchronously) and keeps the fastest; all
 * variants give identical results.  On a batched handle whose meshes all
 * have at most 4096 vertices, the last fixed-K Jacobi call may have run every
 * sweep in one launch (one workgroup per mesh); the name then starts with
 * "small/r<rows per thread>/one-launch".  The first such call times that
 * kernel against the tuned per-sweep path and keeps the faster.  Once the
 * stopping rule has run with the quality fused into temporally blocked
 * passes, " stop=<variant>" names the variant it timed fastest in that form.
 * Once LMS_MULTICOLOR has run, " colour=<variant>" names the multicolour
 * variant of a fixed K ("by-colour": one launch per colour; "mc/...": all
 * colours of k sweeps in one pass), followed by " colour_stop=<variant>" when
 * the stopping rule runs another (it needs passes of one sweep).
 * buf: host
 * char[len] out, NUL-terminated, truncated to len-1 characters. */
lms_status lms_sweep_config(lms_mesh_t m, lms_precision p, char *buf, int32_t len);

/* Free the handle and everything it owns.  NULL is accepted. */
lms_status lms_destroy(lms_mesh_t m);

/* Message of the last failed call on this thread (empty if none); valid
 * until the next call on this thread. */
const char *lms_last_error(void);

/* ---- introspection (host-only) -------------------------------------- */

lms_status lms_get_info(lms_mesh_t m, lms_mesh_info *info);

/* Smoothing adjacency in current labels: row_ptr host int32[n+1],
 * col host int32[nnz] (ascending per row; fixed rows are empty). */
lms_status lms_get_csr(lms_mesh_t m, int32_t *row_ptr, int32_t *col);

/* Per current vertex: fixed flag (host uint8[n]) and colour (host int32[n],
 * -1 for fixed vertices); either may be NULL. */
lms_status lms_get_vertex_data(lms_mesh_t m, uint8_t *fixed, int32_t *color);

/* Current ordering as new2old (host int32[n]). */
lms_status lms_get_order(lms_mesh_t m, int32_t *new2old);

/* Vertex qualities (Section 3.2: mean over a vertex's triangles of the
 * shortest / longest edge ratio) computed on the host in float64 from
 * INPUT-label coordinates, the qualities RDR sorts by (Algorithm 2):
 * q host float64[n] out. */
lms_status lms_host_vertex_quality(lms_mesh_t m, const double *x, const double *y, double *q);

/* Statistics of lms_reuse_profile. */
typedef struct lms_reuse_stats {
    int64_t accesses;           /* trace length */
    int64_t cold;               /* first accesses */
    int64_t max;                /* largest reuse distance */
    double mean;                /* mean reuse distance of the other accesses */
    double lines_per_wave;
    int64_t max_lines_per_wave;
} lms_reuse_stats;

/* Locality of the current ordering (Section 2, reuse distance and cache
 * misses; the quantiles of Table 2), computed on the host.  The trace is one
 * Jacobi sweep in storage order: each free vertex in ascending current label,
 * then its neighbours in ascending current label; items are current labels.
 * The reuse distance of an access is the number of distinct items accessed
 * since the previous access to the same item (first accesses are cold and
 * have none).  For the GPU, lines_per_wave is the mean number of distinct
 * cache lines of line_bytes bytes (records of record_bytes bytes stored by
 * current label) that the neighbour reads of 64 consecutive rows touch, over
 * the waves that hold a free row.
 *   fractions  host double[nfrac] in [0, 1]
 *   quantiles  host int64[nfrac] out: for each fraction X, the smallest d
 *              such that at least a fraction X of the distances are <= d
 *   stats      host out
 * Fails with LMS_ERR_ARG for a fraction outside [0, 1] or non-positive sizes,
 * and LMS_ERR_STATE when the trace exceeds 2^31 accesses. */
lms_status lms_reuse_profile(lms_mesh_t m, const double *fractions, int32_t nfrac, int64_t *quantiles,
                             int32_t line_bytes, int32_t record_bytes, lms_reuse_stats *stats);

/* lms_reuse_profile over a chosen access trace (Section 2's reuse distance;
 * Table 2 profiles its own code's full run, whose trace it does not spell
 * out).
 *   trace  LMS_TRACE_SWEEP (0): the trace of lms_reuse_profile;
 *          LMS_TRACE_ALGORITHM1 (1): Algorithm 1's loop body, the smoothing
 *          of V[i] (the vertex, then its neighbours in ascending current
 *          label) followed by the update of the global quality: every
 *          triangle containing the vertex, in ascending current triangle
 *          index, as its three corners in ascending label and then the
 *          triangle's quality record.  Items are vertex labels 0..n-1 and
 *          triangle records n..n+T-1.
 * Other arguments, outputs and errors as lms_reuse_profile (LMS_ERR_ARG for
 * an unknown trace); lines_per_wave counts the neighbour reads only. */
typedef enum { LMS_TRACE_SWEEP = 0, LMS_TRACE_ALGORITHM1 = 1 } lms_trace_kind;
lms_status lms_reuse_profile_trace(lms_mesh_t m, int32_t trace, const double *fractions, int32_t nfrac,
                                   int64_t *quantiles, int32_t line_bytes, int32_t record_bytes,
                                   lms_reuse_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* LMS_H */
