// Device side of the smoothing library for gfx950 (MI355X): kernels and the
// runtime around them (upload of the mesh arrays, scratch buffers, graph
// capture of the sweep loop, device-side stopping rule).
//
// Compiled with -ffp-contract=off: the sweep sums and the quality arithmetic
// are exactly the IEEE operations written (no fused multiply-add).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <string>
#include <vector>

#include "lms_internal.hpp"

namespace lms {

#define HIP_CHECK(expr)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(e_ == hipErrorOutOfMemory ? LMS_ERR_ALLOC : LMS_ERR_HIP,                  \
                 std::string(#expr) + " failed: " + hipGetErrorString(e_));                \
    } while (0)

// ---------------------------------------------------------------------------
// Device-side state of Algorithm 1's stopping rule.
struct StopState {
    int32_t done;        // nonzero: stop; later sweeps in a captured chunk do nothing
    int32_t iters;       // sweeps done so far (fused path: the last state evaluated)
    int32_t stopped_by;  // lms_stop_reason
    int32_t swept;       // fused path: state index held by the next pass's source copy
    double q0;
    double q_prev;       // Q_{k-1}
    double q_last;       // Q_k of the last evaluation
    double last_dq;
    double q_const;      // fused path: sum of w_t q_t over triangles whose corners are all fixed
    int32_t redo;        // fused path: sweeps from copy `src` that give the final state
    int32_t src;         // fused path: 0 / 1, the working copy the final state comes from
};

// Arguments of the stopping rule (Section 5.1) for the fused path.
struct StopArgs {
    double inv_n;         // 1 / |V|
    double tol, goal;
    double q_prev_given;  // replaces Q_0 when use_q_prev
    int32_t use_q_prev;
    int32_t max_iters;
    int32_t src_index;    // 0 / 1: the working copy this pass reads
    int32_t pad;
};

constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// Workgroups are dealt to the XCDs round-robin.  Remap the launch index so
// that each XCD walks one contiguous range of tiles: neighbouring tiles share
// halo cache lines, and this keeps the sharing inside one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / kXcds, r = nb % kXcds;
    const int xcd = b % kXcds, local = b / kXcds;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Tile walked by workgroup b of nb.  MAP = 0: tile b (consecutive tiles land
// on different XCDs, so all XCDs sweep one narrow window of the ids);
// MAP < 0: xcd_tile (each XCD one contiguous eighth); MAP = k > 0: each XCD
// takes runs of k consecutive tiles (neighbouring tiles share an L2, and the
// XCDs still advance together through the ids).  The tail that does not fill
// a whole round of 8 runs keeps tile = b.  Every mapping is a bijection.
template <int MAP>
__device__ __forceinline__ int tile_of(int b, int nb) {
    if constexpr (MAP == 0) {
        return b;
    } else if constexpr (MAP < 0) {
        return xcd_tile(b, nb);
    } else {
        constexpr int span = kXcds * MAP;
        const int full = (nb / span) * span;
        if (b >= full) return b;
        const int xcd = b % kXcds, local = b / kXcds;
        return ((local / MAP) * kXcds + xcd) * MAP + local % MAP;
    }
}

// ---------------------------------------------------------------------------
// Jacobi sweep, Eq. 1 for every free vertex: dst[v] = (sum of src[u] over the
// neighbours u of v, in ascending label) / deg(v).  Fixed rows are empty and
// are not written.
//
// One workgroup of BS threads owns BS consecutive rows.  Its slice of
// row_ptr goes to LDS; then the whole workgroup streams the slice's
// neighbour indices with coalesced loads and gathers the neighbour
// coordinates into LDS (edge-parallel: all gathers independent, CAP entries
// per pass); finally each thread sums its own row out of LDS in order and
// divides.  A slice with more than CAP entries takes several passes; the
// partial sums carry over, so the summation order stays the row's order.
template <typename T, int BS, int CAP, int MAP>
__global__ __launch_bounds__(BS) void k_jacobi(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               const T *__restrict__ sx, const T *__restrict__ sy,
                                               T *__restrict__ dx, T *__restrict__ dy, int32_t n,
                                               const StopState *__restrict__ st) {
    static_assert(CAP % BS == 0, "CAP must be a multiple of BS");
    constexpr int PER = CAP / BS;
    __shared__ int32_t s_rp[BS + 1];
    __shared__ T s_x[CAP];
    __shared__ T s_y[CAP];
    if (st && st->done) return;

    const int nb = int(gridDim.x);
    const int tile = tile_of<MAP>(int(blockIdx.x), nb);
    const int32_t r0 = tile * BS;
    const int tid = int(threadIdx.x);
    const int rows = min(BS, n - r0);
    for (int i = tid; i <= rows; i += BS) s_rp[i] = row_ptr[r0 + i];
    __syncthreads();
    const int32_t nz0 = s_rp[0], nz1 = s_rp[rows];
    const int32_t my_b = tid < rows ? s_rp[tid] : 0;
    const int32_t my_e = tid < rows ? s_rp[tid + 1] : 0;
    T ax = T(0), ay = T(0);
    for (int32_t base = nz0; base < nz1; base += CAP) {
        const int cnt = min(CAP, nz1 - base);
        int32_t u[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = tid + i * BS;
            u[i] = j < cnt ? __builtin_nontemporal_load(col + base + j) : 0;
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = tid + i * BS;
            if (j < cnt) {
                s_x[j] = sx[u[i]];
                s_y[j] = sy[u[i]];
            }
        }
        __syncthreads();
        const int32_t lo = max(my_b, base), hi = min(my_e, base + cnt);
        for (int32_t j = lo; j < hi; ++j) {
            ax += s_x[j - base];
            ay += s_y[j - base];
        }
        __syncthreads();
    }
    if (my_e > my_b) {
        const T c = T(my_e - my_b);
        dx[r0 + tid] = ax / c;
        dy[r0 + tid] = ay / c;
    }
}

template <bool NT>
__device__ __forceinline__ int32_t load_index(const int32_t *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Jacobi sweep, thread per row: each thread owns R rows (BS apart, so every
// load instruction of the wavefront is coalesced), issues all their
// neighbour-index loads U at a time, then all the coordinate gathers (all
// independent, so they are in flight together), and adds each row in order.
// No LDS and no barriers.  Sums in the same order as k_jacobi: same bits.
// NT: neighbour indices are loaded with the non-temporal hint.
template <typename T, int BS, int U, int R, int MAP, bool NT>
__global__ __launch_bounds__(BS) void k_jacobi_row(const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col,
                                                   const T *__restrict__ sx, const T *__restrict__ sy,
                                                   T *__restrict__ dx, T *__restrict__ dy, int32_t n,
                                                   const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int nb = int(gridDim.x);
    const int tile = tile_of<MAP>(int(blockIdx.x), nb);
    const int32_t v0 = tile * (BS * R) + int32_t(threadIdx.x);
    int32_t b[R], e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t v = v0 + r * BS;
        b[r] = v < n ? row_ptr[v] : 0;
        e[r] = v < n ? row_ptr[v + 1] : 0;
    }
    int32_t u[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < U; ++k) u[r][k] = b[r] + k < e[r] ? load_index<NT>(col + b[r] + k) : -1;
    T vx[R][U], vy[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < U; ++k) {
            vx[r][k] = u[r][k] >= 0 ? sx[u[r][k]] : T(0);
            vy[r][k] = u[r][k] >= 0 ? sy[u[r][k]] : T(0);
        }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (e[r] == b[r]) continue;
        T ax = T(0), ay = T(0);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (u[r][k] >= 0) {
                ax += vx[r][k];
                ay += vy[r][k];
            }
        // rows longer than U: the rest in order, U at a time
        for (int32_t j0 = b[r] + U; j0 < e[r]; j0 += U) {
            int32_t w[U];
#pragma unroll
            for (int k = 0; k < U; ++k) w[k] = j0 + k < e[r] ? load_index<NT>(col + j0 + k) : -1;
            T wx[U], wy[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                wx[k] = w[k] >= 0 ? sx[w[k]] : T(0);
                wy[k] = w[k] >= 0 ? sy[w[k]] : T(0);
            }
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (w[k] >= 0) {
                    ax += wx[k];
                    ay += wy[k];
                }
        }
        const T c = T(e[r] - b[r]);
        const int32_t v = v0 + r * BS;
        dx[v] = ax / c;
        dy[v] = ay / c;
    }
}

// Vector loads of one row's padded entries: a row of W int32 indices (W a
// multiple of 4, 16-byte aligned) or of W uint16 slots (W*2 bytes, 16-byte
// aligned for W = 8, 16 and 8-byte aligned for W = 12), with the
// non-temporal hint.  One or two loads per lane instead of W.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int W>
__device__ __forceinline__ void load_row_ids(const int32_t *__restrict__ row, int32_t (&u)[W]) {
    static_assert(W % 4 == 0, "padded width must be a multiple of 4");
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
        const i32x4 v = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(row) + q);
        u[4 * q] = v.x;
        u[4 * q + 1] = v.y;
        u[4 * q + 2] = v.z;
        u[4 * q + 3] = v.w;
    }
}

template <int W>
__device__ __forceinline__ void load_row_slots(const uint16_t *__restrict__ row, uint16_t (&s)[W]) {
    if constexpr (W % 8 == 0) {
#pragma unroll
        for (int q = 0; q < W / 8; ++q) {
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(row) + q);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                s[8 * q + 2 * i] = uint16_t(w[i] & 0xFFFFu);
                s[8 * q + 2 * i + 1] = uint16_t(w[i] >> 16);
            }
        }
    } else {
        static_assert(W % 4 == 0, "padded width must be a multiple of 4");
#pragma unroll
        for (int q = 0; q < W / 4; ++q) {
            const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(row) + q);
            s[4 * q] = uint16_t(v.x & 0xFFFFu);
            s[4 * q + 1] = uint16_t(v.x >> 16);
            s[4 * q + 2] = uint16_t(v.y & 0xFFFFu);
            s[4 * q + 3] = uint16_t(v.y >> 16);
        }
    }
}

// Jacobi sweep over the padded ("ELL") copy of the adjacency: row v's W
// entries sit together at ell[v*W ..] (-1 past the row's end), so a thread
// finds its neighbours without first reading row offsets, with W/4 16-byte
// loads that are coalesced across the wavefront.  Rows have at most W entries.  Each
// thread owns R rows BS apart.  Entries are in the CSR order: same bits.
template <typename T, int BS, int W, int R, int MAP>
__global__ __launch_bounds__(BS) void k_jacobi_ell(const int32_t *__restrict__ ell,
                                                   const T *__restrict__ sx, const T *__restrict__ sy,
                                                   T *__restrict__ dx, T *__restrict__ dy, int32_t n,
                                                   const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int nb = int(gridDim.x);
    const int tile = tile_of<MAP>(int(blockIdx.x), nb);
    const int32_t v0 = tile * (BS * R) + int32_t(threadIdx.x);
    int32_t u[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t v = v0 + r * BS;
        if (v < n) {
            load_row_ids<W>(ell + int64_t(v) * W, u[r]);
        } else {
#pragma unroll
            for (int k = 0; k < W; ++k) u[r][k] = -1;
        }
    }
    T vx[R][W], vy[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < W; ++k) {
            vx[r][k] = u[r][k] >= 0 ? sx[u[r][k]] : T(0);
            vy[r][k] = u[r][k] >= 0 ? sy[u[r][k]] : T(0);
        }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T ax = T(0), ay = T(0);
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (u[r][k] >= 0) {
                ax += vx[r][k];
                ay += vy[r][k];
                ++cnt;
            }
        if (cnt == 0) continue;
        const T c = T(cnt);
        const int32_t v = v0 + r * BS;
        dx[v] = ax / c;
        dy[v] = ay / c;
    }
}

// Interleaved (x, y) working copy: one 16-byte (float64) or 8-byte (float32)
// load per neighbour instead of two.
template <typename T>
struct Vec2Of;
template <>
struct Vec2Of<double> {
    using type = double2;
};
template <>
struct Vec2Of<float> {
    using type = float2;
};
template <typename T>
using vec2_t = typename Vec2Of<T>::type;

template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T *__restrict__ x, const T *__restrict__ y,
                                              vec2_t<T> *__restrict__ a, vec2_t<T> *__restrict__ b, int32_t n) {
    const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (i >= n) return;
    vec2_t<T> v;
    v.x = x[i];
    v.y = y[i];
    a[i] = v;
    if (b) b[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const vec2_t<T> *__restrict__ a, T *__restrict__ x,
                                                T *__restrict__ y, int32_t n) {
    const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (i >= n) return;
    const vec2_t<T> v = a[i];
    x[i] = v.x;
    y[i] = v.y;
}

// k_jacobi_ell on the interleaved copy: same order of additions, same bits.
template <typename T, int BS, int W, int R, int MAP>
__global__ __launch_bounds__(BS) void k_jacobi_ell2(const int32_t *__restrict__ ell,
                                                    const vec2_t<T> *__restrict__ src,
                                                    vec2_t<T> *__restrict__ dst, int32_t n,
                                                    const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int nb = int(gridDim.x);
    const int tile = tile_of<MAP>(int(blockIdx.x), nb);
    const int32_t v0 = tile * (BS * R) + int32_t(threadIdx.x);
    int32_t u[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t v = v0 + r * BS;
        if (v < n) {
            load_row_ids<W>(ell + int64_t(v) * W, u[r]);
        } else {
#pragma unroll
            for (int k = 0; k < W; ++k) u[r][k] = -1;
        }
    }
    vec2_t<T> p[R][W];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (u[r][k] >= 0) {
                p[r][k] = src[u[r][k]];
            } else {
                p[r][k].x = T(0);
                p[r][k].y = T(0);
            }
        }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T ax = T(0), ay = T(0);
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (u[r][k] >= 0) {
                ax += p[r][k].x;
                ay += p[r][k].y;
                ++cnt;
            }
        if (cnt == 0) continue;
        const T c = T(cnt);
        vec2_t<T> o;
        o.x = ax / c;
        o.y = ay / c;
        dst[v0 + r * BS] = o;
    }
}

// k_jacobi_row on the interleaved copy: row offsets and the unpadded index
// stream (4 bytes per entry fewer than the padded copy's empty slots), one
// load per neighbour.  Same order of additions, same bits.
template <typename T, int BS, int U, int R, int MAP>
__global__ __launch_bounds__(BS) void k_jacobi_row2(const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const vec2_t<T> *__restrict__ src,
                                                    vec2_t<T> *__restrict__ dst, int32_t n,
                                                    const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int nb = int(gridDim.x);
    const int tile = tile_of<MAP>(int(blockIdx.x), nb);
    const int32_t v0 = tile * (BS * R) + int32_t(threadIdx.x);
    int32_t b[R], e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t v = v0 + r * BS;
        b[r] = v < n ? row_ptr[v] : 0;
        e[r] = v < n ? row_ptr[v + 1] : 0;
    }
    int32_t u[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < U; ++k) u[r][k] = b[r] + k < e[r] ? __builtin_nontemporal_load(col + b[r] + k) : -1;
    vec2_t<T> p[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (u[r][k] >= 0) {
                p[r][k] = src[u[r][k]];
            } else {
                p[r][k].x = T(0);
                p[r][k].y = T(0);
            }
        }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (e[r] == b[r]) continue;
        T ax = T(0), ay = T(0);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (u[r][k] >= 0) {
                ax += p[r][k].x;
                ay += p[r][k].y;
            }
        for (int32_t j = b[r] + U; j < e[r]; ++j) {  // rows longer than U, in order
            const vec2_t<T> q = src[col[j]];
            ax += q.x;
            ay += q.y;
        }
        const T c = T(e[r] - b[r]);
        vec2_t<T> o;
        o.x = ax / c;
        o.y = ay / c;
        dst[v0 + r * BS] = o;
    }
}

// Multicolour sweep of one colour, in place: every vertex of the colour reads
// the current coordinates of its neighbours (none of which has this colour).
template <typename T>
__global__ __launch_bounds__(256) void k_colour(const int32_t *__restrict__ row_ptr,
                                                const int32_t *__restrict__ col,
                                                const int32_t *__restrict__ list, int32_t cnt, T *x,
                                                T *y, const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (i >= cnt) return;
    const int32_t v = list[i];
    const int32_t b = row_ptr[v], e = row_ptr[v + 1];
    T ax = T(0), ay = T(0);
    for (int32_t j = b; j < e; ++j) {
        const int32_t u = col[j];
        ax += x[u];
        ay += y[u];
    }
    const T c = T(e - b);
    x[v] = ax / c;
    y[v] = ay / c;
}

// Jacobi sweep with the tile's neighbourhood staged in LDS.  Workgroup t owns
// rows [t*TS, (t+1)*TS): it loads their coordinates (coalesced) and those of
// the tile's halo (the sorted outside neighbours, one load each) into LDS
// once; each row then reads its W neighbours from LDS through 16-bit
// tile-local slots (0xFFFF past the row's end; one 16-byte load per row for
// W = 8).  Every global gather of the
// other variants becomes an LDS read, and the index stream halves.  Entries
// keep the row's ascending order: same additions, same bits.
template <typename T, int TS, int W, int MAP>
__global__ __launch_bounds__(TS) void k_jacobi_halo(const int32_t *__restrict__ halo_ptr,
                                                    const int32_t *__restrict__ halo,
                                                    const uint16_t *__restrict__ lidx,
                                                    const vec2_t<T> *__restrict__ src,
                                                    vec2_t<T> *__restrict__ dst, int32_t n,
                                                    const StopState *__restrict__ st) {
    extern __shared__ unsigned char lds_raw[];
    vec2_t<T> *stage = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if (st && st->done) return;
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t v = tile * TS + tid;
    uint16_t li[W];
    load_row_slots<W>(lidx + (int64_t(tile) * TS + tid) * W, li);
    if (v < n) stage[tid] = src[v];
    const int32_t hb = halo_ptr[tile], he = halo_ptr[tile + 1];
    for (int32_t j0 = hb + tid; j0 < he; j0 += 4 * TS) {
        int32_t g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = j0 + q * TS < he ? halo[j0 + q * TS] : -1;
        T hx[4], hy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hx[q] = T(0);
            hy[q] = T(0);
            if (g[q] >= 0) {
                const vec2_t<T> h = src[g[q]];
                hx[q] = h.x;
                hy[q] = h.y;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (g[q] >= 0) {
                vec2_t<T> h;
                h.x = hx[q];
                h.y = hy[q];
                stage[TS + (j0 + q * TS - hb)] = h;
            }
    }
    __syncthreads();
    T ax = T(0), ay = T(0);
    int c = 0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        if (li[k] != 0xFFFF) {
            const vec2_t<T> p = stage[li[k]];
            ax += p.x;
            ay += p.y;
            ++c;
        }
    if (c > 0) {
        vec2_t<T> o;
        o.x = ax / T(c);
        o.y = ay / T(c);
        dst[v] = o;
    }
}

// The padded slots of one row, two 16-bit slots per word (slot 2q in the
// low half of word q).
template <int W>
__device__ __forceinline__ void load_slot_words(const uint16_t *__restrict__ row, uint32_t (&w)[W / 2]) {
    if constexpr (W % 8 == 0) {
#pragma unroll
        for (int q = 0; q < W / 8; ++q) {
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(row) + q);
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
    } else {
        static_assert(W % 4 == 0, "padded width must be a multiple of 4");
#pragma unroll
        for (int q = 0; q < W / 4; ++q) {
            const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(row) + q);
            w[2 * q] = v.x;
            w[2 * q + 1] = v.y;
        }
    }
}

__device__ __forceinline__ double tri_quality(double xa, double ya, double xb, double yb, double xc, double yc);
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *s_red);

// Temporally blocked Jacobi: k sweeps (Eq. 1, Algorithm 1) of the tile's
// own rows in one pass over memory.  Tile t (rows tile_ptr[t] ..
// tile_ptr[t+1]-1) stages its own rows and k halo
// rings of src in LDS (local slots in ring order).  Sweep j of the pass
// updates, in LDS, every row of the tile's own set and of rings 1..k-j: a
// row of ring m reads only rings up to m+1, which still hold values of the
// previous sweep.  So after k sweeps the own rows hold exactly what k
// separate sweeps give them; halo rows are computed redundantly, in the same
// order, with the same bits.  Each sweep computes into registers, waits,
// stores, waits; the last one writes the own free rows to dst.  Thread t
// owns local rows t, t+BS, ..., R of them; the plan guarantees that the
// rows updated by the first sweep fit (ring[k-1] <= BS*R) and that the
// staging area fits the dynamic LDS it is launched with.  TS (nominal tile
// size), KP (the plan's depth) and LCAP (its staging cap) name the variant
// whose plan the kernel reads; the tiles themselves come from tile_ptr.
//
// G (patch tiles): the tile's own rows are not a range but the first nown
// entries of its staged-row list (halo_ptr/halo then cover every staged row),
// read and written through it.
//
// QUAL (the stopping rule, Section 5.1): the pass also evaluates the quality
// (Section 3.2) of each state it starts a sweep from.  Before sweep j+1 the
// own rows and ring 1 hold state s+j, and every triangle of the tile (those
// whose smallest free corner is an own row) has its corners there; the
// tile's sum of w_t q_t goes to qpart[j*gridDim.x + tile].  The depth comes
// from the device state: k = min(KP, max_iters - swept), and a pass of depth
// 0 (all sweeps done) evaluates its source state only.
template <typename T, int BS, int W, int R, int MAP, int TS, int KP, int LCAP, bool QUAL, bool G>
__global__ __launch_bounds__(BS) void k_jacobi_tb(const int32_t *__restrict__ tile_ptr,
                                                  const int32_t *__restrict__ ring, int32_t k,
                                                  const int64_t *__restrict__ halo_ptr,
                                                  const int32_t *__restrict__ halo,
                                                  const int64_t *__restrict__ lidx_ptr,
                                                  const uint16_t *__restrict__ lidx,
                                                  const vec2_t<T> *__restrict__ src, vec2_t<T> *__restrict__ dst,
                                                  const int64_t *__restrict__ qtri_ptr,
                                                  const uint32_t *__restrict__ qtri, double *__restrict__ qpart,
                                                  const StopState *__restrict__ st, int32_t max_iters) {
    static_assert(W % 4 == 0, "padded width must be a multiple of 4");
    constexpr int QR = 2;     // triangle records per thread held in registers
    constexpr int NRCP = 64;  // 1/c for triangle counts c = 1..NRCP from a table (the same division)
    extern __shared__ unsigned char lds_raw[];
    __shared__ double s_red[BS / 64];
    __shared__ double s_rcp[QUAL ? NRCP + 1 : 1];
    vec2_t<T> *sp = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if constexpr (QUAL) {
        if (st->done) return;
        k = min(KP, max_iters - st->swept);
    }
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t b = G ? 0 : tile_ptr[tile];
    static_assert(KP >= 1 && KP <= 8 && TS > 0 && LCAP > 0, "plan shape");
    const int32_t *rc = ring + int64_t(tile) * (KP + 1);
    const int32_t nown = rc[0], nload = rc[k > 0 ? k : 1], nupd = k > 0 ? rc[k - 1] : 0;
    const int64_t hb = halo_ptr[tile], lb = lidx_ptr[tile];
    uint32_t qw[QUAL ? QR : 1][3];
    int64_t qb = 0, qe = 0;
    if constexpr (QUAL) {
        for (int c = tid; c <= NRCP; c += BS) s_rcp[c] = c == 0 ? 0.0 : 1.0 / double(c);
        qb = qtri_ptr[tile];
        qe = qtri_ptr[tile + 1];
#pragma unroll
        for (int r = 0; r < QR; ++r) {
            const int64_t t = qb + tid + BS * r;
            qw[r][0] = qw[r][1] = qw[r][2] = 0u;  // count 0: no triangle
            if (t < qe) {
                qw[r][0] = qtri[3 * t];
                qw[r][1] = qtri[3 * t + 1];
                qw[r][2] = qtri[3 * t + 2];
            }
        }
    }
    uint32_t wd[R][W / 2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t i = tid + BS * r;
        if (i < nupd) {
            load_slot_words<W>(lidx + (lb + i) * W, wd[r]);
        } else {
#pragma unroll
            for (int q = 0; q < W / 2; ++q) wd[r][q] = 0xFFFFFFFFu;
        }
    }
    if constexpr (!G)
        for (int32_t i = tid; i < nown; i += BS) sp[i] = src[b + i];
    const int32_t g0 = G ? 0 : nown;  // first staged row read through the list
    const int32_t nh = nload - g0;
    for (int32_t j0 = tid; j0 < nh; j0 += 4 * BS) {
        int32_t g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = j0 + q * BS < nh ? halo[hb + j0 + q * BS] : -1;
        T hx[4], hy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hx[q] = T(0);
            hy[q] = T(0);
            if (g[q] >= 0) {
                const vec2_t<T> h = src[g[q]];
                hx[q] = h.x;
                hy[q] = h.y;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (g[q] >= 0) {
                vec2_t<T> h;
                h.x = hx[q];
                h.y = hy[q];
                sp[g0 + j0 + q * BS] = h;
            }
    }
    __syncthreads();
    const int32_t passes = QUAL && k == 0 ? 1 : k;
    for (int32_t j = 1; j <= passes; ++j) {
        if constexpr (QUAL) {
            // quality of state s+j-1: every triangle of the tile, from LDS
            auto tri_term = [&](uint32_t w0, uint32_t w1, uint32_t w2) {
                const vec2_t<T> pa = sp[w0 & 0xFFFFu], pb = sp[w0 >> 16], pc = sp[w1 & 0xFFFFu];
                const double q = tri_quality(double(pa.x), double(pa.y), double(pb.x), double(pb.y), double(pc.x),
                                             double(pc.y));
                const uint32_t ca = w1 >> 16, cb = w2 & 0xFFFFu, cc = w2 >> 16;
                const double ra = ca <= NRCP ? s_rcp[ca] : 1.0 / double(ca);
                const double rb = cb <= NRCP ? s_rcp[cb] : 1.0 / double(cb);
                const double rc = cc <= NRCP ? s_rcp[cc] : 1.0 / double(cc);
                return q * (ra + rb + rc);
            };
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < QR; ++r)
                if ((qw[r][1] >> 16) != 0u) acc += tri_term(qw[r][0], qw[r][1], qw[r][2]);
            for (int64_t t = qb + QR * BS + tid; t < qe; t += BS)
                acc += tri_term(qtri[3 * t], qtri[3 * t + 1], qtri[3 * t + 2]);
            const double sum = block_sum<BS>(acc, s_red);
            if (tid == 0) qpart[int64_t(j - 1) * gridDim.x + tile] = sum;
            __syncthreads();  // s_red is reused by the next state's sum
            if (k == 0) break;
        }
        const int32_t m = rc[k - j];  // rows updated by this sweep
        vec2_t<T> o[R];
        bool w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w[r] = false;
            o[r].x = T(0);
            o[r].y = T(0);
            const int32_t i = tid + BS * r;
            if (BS * r >= m) continue;  // the same for the whole workgroup
            if (i >= m) continue;
            T ax = T(0), ay = T(0);
            int c = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t id = (wd[r][q / 2] >> (16 * (q % 2))) & 0xFFFFu;
                if (id != 0xFFFFu) {
                    const vec2_t<T> p = sp[id];
                    ax += p.x;
                    ay += p.y;
                    ++c;
                }
            }
            w[r] = c > 0;
            if (c > 0) {
                o[r].x = ax / T(c);
                o[r].y = ay / T(c);
            }
        }
        if (j == k) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (w[r]) dst[G ? halo[hb + tid + BS * r] : b + tid + BS * r] = o[r];
        } else {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (w[r]) sp[tid + BS * r] = o[r];
            __syncthreads();
        }
    }
}

// All K Jacobi sweeps of a batch of small meshes in one launch, one workgroup
// of 256 threads per mesh (Algorithm 1 per mesh).  A mesh's padded index is
// read once, turned into 16-bit slots local to the mesh (two per register)
// and kept in registers for every sweep; its coordinates sit in one LDS copy.
// Each sweep computes its rows' new positions into registers, waits for the
// whole workgroup, stores them and waits again, so no row reads a value of
// the sweep it is in.  Thread t owns rows t, t+256, ..., R rows at most.
// Same order of additions and the same divide as every other sweep kernel.
template <typename T, int W, int R>
__global__ __launch_bounds__(256) void k_small_meshes(const int64_t *__restrict__ v_off,
                                                      const int32_t *__restrict__ ell,
                                                      vec2_t<T> *__restrict__ a, vec2_t<T> *__restrict__ b,
                                                      int32_t K) {
    static_assert(W % 2 == 0, "slots are packed in pairs");
    extern __shared__ unsigned char lds_raw[];
    vec2_t<T> *sp = reinterpret_cast<vec2_t<T> *>(lds_raw);
    const int64_t vb = v_off[blockIdx.x];
    const int32_t nv = int32_t(v_off[blockIdx.x + 1] - vb);
    uint32_t slot[R][W / 2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t i = int32_t(threadIdx.x) + 256 * r;
#pragma unroll
        for (int q = 0; q < W / 2; ++q) slot[r][q] = 0xFFFFFFFFu;
        if (i < nv) {
            int32_t u[W];
            load_row_ids<W>(ell + (vb + i) * W, u);
#pragma unroll
            for (int q = 0; q < W / 2; ++q) {
                const uint32_t lo = u[2 * q] >= 0 ? uint32_t(u[2 * q] - vb) : 0xFFFFu;
                const uint32_t hi = u[2 * q + 1] >= 0 ? uint32_t(u[2 * q + 1] - vb) : 0xFFFFu;
                slot[r][q] = lo | (hi << 16);
            }
            sp[i] = a[vb + i];
        }
    }
    __syncthreads();
    for (int32_t k = 0; k < K; ++k) {
        vec2_t<T> o[R];
        bool w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w[r] = false;
            if (256 * r >= nv) continue;  // the same for the whole workgroup
            T ax = T(0), ay = T(0);
            int c = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t id = (slot[r][q / 2] >> (16 * (q % 2))) & 0xFFFFu;
                if (id != 0xFFFFu) {
                    const vec2_t<T> p = sp[id];
                    ax += p.x;
                    ay += p.y;
                    ++c;
                }
            }
            w[r] = c > 0;
            o[r].x = w[r] ? ax / T(c) : T(0);
            o[r].y = w[r] ? ay / T(c) : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (256 * r < nv && w[r]) sp[int32_t(threadIdx.x) + 256 * r] = o[r];
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t i = int32_t(threadIdx.x) + 256 * r;
        if (i < nv) {
            a[vb + i] = sp[i];
            b[vb + i] = sp[i];
        }
    }
}

// Multicolour sweep of one colour on the interleaved copy, in place.  The
// colour's vertices read their neighbours' current positions (none of which
// has this colour) through the colour-major padded index: entry k of the
// colour's i-th vertex at cell[k*cnt + i].  Same order of additions as
// k_colour, same bits.
template <typename T, int BS, int W>
__global__ __launch_bounds__(BS) void k_colour2(const int32_t *__restrict__ list, const int32_t *__restrict__ cell,
                                                int32_t cnt, vec2_t<T> *xy, const StopState *__restrict__ st) {
    if (st && st->done) return;
    const int32_t i = int32_t(blockIdx.x) * BS + int32_t(threadIdx.x);
    if (i >= cnt) return;
    int32_t u[W];
#pragma unroll
    for (int k = 0; k < W; ++k) u[k] = __builtin_nontemporal_load(cell + int64_t(k) * cnt + i);
    const int32_t v = list[i];
    vec2_t<T> p[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        if (u[k] >= 0) {
            p[k] = xy[u[k]];
        } else {
            p[k].x = T(0);
            p[k].y = T(0);
        }
    }
    T ax = T(0), ay = T(0);
    int c = 0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        if (u[k] >= 0) {
            ax += p[k].x;
            ay += p[k].y;
            ++c;
        }
    vec2_t<T> o;
    o.x = ax / T(c);
    o.y = ay / T(c);
    xy[v] = o;
}

// ---------------------------------------------------------------------------
// All colours of one multicolour sweep (the in-place form, colours in
// order) in one pass, tile by tile.  The tile stages its own rows and its
// staged halo from src (the state at the start of the sweep) and updates in
// LDS, colour by colour and in place, its own free rows and every halo
// vertex whose new value one of them reads; it recomputes those the same way
// their owner does, from the same values in the same order, so the bits are
// those of the colour-by-colour sweep.  No two vertices of one colour are
// adjacent, so the updates inside a colour do not race.  Own rows go to dst
// (fixed ones unchanged).
//
// QUAL (the stopping rule, Section 5.1): the pass first evaluates the
// quality of the state it sweeps from over the tile's triangles (their
// corners are all staged) into qpart[tile]; its depth (1, or 0 once all
// sweeps are done: quality only) comes from the device state.
template <typename T, int BS, int W, int R, int MAP, bool QUAL>
__global__ __launch_bounds__(BS) void k_colour_tiles(const int32_t *__restrict__ tile_ptr,
                                                     const int64_t *__restrict__ halo_ptr,
                                                     const int32_t *__restrict__ halo,
                                                     const int64_t *__restrict__ upd_ptr,
                                                     const uint16_t *__restrict__ urow,
                                                     const uint16_t *__restrict__ uidx, int32_t C,
                                                     const vec2_t<T> *__restrict__ src, vec2_t<T> *__restrict__ dst,
                                                     const StopState *__restrict__ st,
                                                     const int64_t *__restrict__ qtri_ptr,
                                                     const uint32_t *__restrict__ qtri, double *__restrict__ qpart,
                                                     int32_t max_iters) {
    extern __shared__ unsigned char lds_raw[];
    __shared__ double s_red[BS / 64];
    __shared__ double s_rcp[QUAL ? 65 : 1];
    vec2_t<T> *sp = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if (st && st->done) return;
    int32_t depth = 1;
    if constexpr (QUAL) {
        depth = min(1, max_iters - st->swept);
        for (int c = int(threadIdx.x); c <= 64; c += BS) s_rcp[c] = c == 0 ? 0.0 : 1.0 / double(c);
    }
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t b = tile_ptr[tile], nown = tile_ptr[tile + 1] - b;
    const int64_t hb = halo_ptr[tile];
    const int32_t nh = int32_t(halo_ptr[tile + 1] - hb);
    // this thread's updated rows (the tile's list, colour by colour): slot,
    // colour and neighbour slots, held in registers for the whole pass
    const int64_t *up = upd_ptr + int64_t(tile) * (C + 1);
    uint32_t wd[R][W / 2];
    int32_t row[R], colr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t e = up[0] + tid + BS * r;
        colr[r] = -1;
        row[r] = 0;
        if (e < up[C]) {
            load_slot_words<W>(uidx + e * W, wd[r]);
            row[r] = urow[e];
            int32_t c = 0;
            while (up[c + 1] <= e) ++c;
            colr[r] = c;
        }
    }
    for (int32_t i = tid; i < nown; i += BS) sp[i] = src[b + i];
    for (int32_t j0 = tid; j0 < nh; j0 += 4 * BS) {
        int32_t g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = j0 + q * BS < nh ? halo[hb + j0 + q * BS] : -1;
        T hx[4], hy[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hx[q] = T(0);
            hy[q] = T(0);
            if (g[q] >= 0) {
                const vec2_t<T> h = src[g[q]];
                hx[q] = h.x;
                hy[q] = h.y;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (g[q] >= 0) {
                vec2_t<T> h;
                h.x = hx[q];
                h.y = hy[q];
                sp[nown + j0 + q * BS] = h;
            }
    }
    __syncthreads();
    if constexpr (QUAL) {
        // quality of the source state: the tile's triangles, from LDS
        double acc = 0.0;
        for (int64_t t = qtri_ptr[tile] + tid; t < qtri_ptr[tile + 1]; t += BS) {
            const uint32_t w0 = qtri[3 * t], w1 = qtri[3 * t + 1], w2 = qtri[3 * t + 2];
            const vec2_t<T> pa = sp[w0 & 0xFFFFu], pb = sp[w0 >> 16], pc = sp[w1 & 0xFFFFu];
            const double q = tri_quality(double(pa.x), double(pa.y), double(pb.x), double(pb.y), double(pc.x),
                                         double(pc.y));
            const uint32_t ca = w1 >> 16, cb = w2 & 0xFFFFu, cc = w2 >> 16;
            const double ra = ca <= 64 ? s_rcp[ca] : 1.0 / double(ca);
            const double rb = cb <= 64 ? s_rcp[cb] : 1.0 / double(cb);
            const double rc = cc <= 64 ? s_rcp[cc] : 1.0 / double(cc);
            acc += q * (ra + rb + rc);
        }
        const double sum = block_sum<BS>(acc, s_red);
        if (tid == 0) qpart[tile] = sum;
        if (depth == 0) return;  // all sweeps done: the state was evaluated only
        __syncthreads();
    }
    for (int32_t c = 0; c < C; ++c) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (colr[r] != c) continue;
            T ax = T(0), ay = T(0);
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t id = (wd[r][q / 2] >> (16 * (q % 2))) & 0xFFFFu;
                if (id != 0xFFFFu) {
                    const vec2_t<T> p = sp[id];
                    ax += p.x;
                    ay += p.y;
                    ++cnt;
                }
            }
            if (cnt > 0) {
                vec2_t<T> o;
                o.x = ax / T(cnt);
                o.y = ay / T(cnt);
                sp[row[r]] = o;
            }
        }
        __syncthreads();
    }
    for (int32_t i = tid; i < nown; i += BS) dst[b + i] = sp[i];
}

// Quality (Section 3.2) of one triangle: shortest / longest Euclidean edge.
__device__ __forceinline__ double tri_quality(double xa, double ya, double xb, double yb, double xc,
                                              double yc) {
    double dx, dy;
    dx = xb - xa;
    dy = yb - ya;
    const double e0 = dx * dx + dy * dy;
    dx = xc - xb;
    dy = yc - yb;
    const double e1 = dx * dx + dy * dy;
    dx = xa - xc;
    dy = ya - yc;
    const double e2 = dx * dx + dy * dy;
    const double mn = fmin(fmin(e0, e1), e2);
    const double mx = fmax(fmax(e0, e1), e2);
    return mx > 0.0 ? sqrt(mn) / sqrt(mx) : 0.0;
}

// Coordinates of vertex i from structure-of-arrays x/y, or from the
// interleaved working copy when xy is given.
template <typename T>
__device__ __forceinline__ void coords(const T *__restrict__ x, const T *__restrict__ y,
                                       const vec2_t<T> *__restrict__ xy, int32_t i, double &px, double &py) {
    if (xy) {
        const vec2_t<T> v = xy[i];
        px = double(v.x);
        py = double(v.y);
    } else {
        px = double(x[i]);
        py = double(y[i]);
    }
}

template <typename T>
__device__ __forceinline__ double tri_quality_at(const T *__restrict__ x, const T *__restrict__ y,
                                                 const vec2_t<T> *__restrict__ xy, int32_t a, int32_t b,
                                                 int32_t c) {
    double xa, ya, xb, yb, xc, yc;
    coords(x, y, xy, a, xa, ya);
    coords(x, y, xy, b, xb, yb);
    coords(x, y, xy, c, xc, yc);
    return tri_quality(xa, ya, xb, yb, xc, yc);
}

template <int BS>
__device__ __forceinline__ double block_sum(double v, double *s_red) {
    // fixed-shape reduction: 64-lane wavefront butterfly, then the wave sums
    // in wave order -- the same result for the same inputs on every run
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / 64; ++w) t += s_red[w];
    return t;  // valid in thread 0
}

// Per-block partial sums of q_t * w_t over a grid-stride range of triangles,
// where w_t = sum over the corners of 1/|T(v)| (the 1/|V| of the global mean
// is applied by the final reduction).  Optionally stores q_t.  Each triangle
// is one 16-byte record (corners a, b, c; counts |T(v)| packed 10 bits each,
// from which w_t is recomputed in the same order as on the host); each thread
// takes four triangles per step, loads first.
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_quality(const int32_t *__restrict__ trec, const T *__restrict__ x,
                                                const T *__restrict__ y, const vec2_t<T> *__restrict__ xy,
                                                int64_t ntri, double *__restrict__ partials,
                                                double *__restrict__ qt_out, const StopState *__restrict__ st) {
    __shared__ double s_red[BS / 64];
    if (st && st->done) return;
    double acc = 0.0;
    const int64_t stride = int64_t(gridDim.x) * BS;
    for (int64_t t0 = int64_t(blockIdx.x) * BS + threadIdx.x; t0 < ntri; t0 += 4 * stride) {
        i32x4 r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t t = t0 + q * stride;
            if (t < ntri) r[q] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(trec) + t);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t t = t0 + q * stride;
            if (t < ntri) {
                const double qt = tri_quality_at(x, y, xy, r[q].x, r[q].y, r[q].z);
                const uint32_t cnt = uint32_t(r[q].w);
                const double w = 1.0 / double(cnt & 1023u) + 1.0 / double((cnt >> 10) & 1023u) +
                                 1.0 / double(cnt >> 20);
                if (qt_out) qt_out[t] = qt;
                acc += qt * w;
            }
        }
    }
    const double s = block_sum<BS>(acc, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// The same without the packed record (a vertex in more than 1023 triangles).
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_quality_wide(const int32_t *__restrict__ ta, const int32_t *__restrict__ tb,
                                                     const int32_t *__restrict__ tc, const double *__restrict__ tw,
                                                     const T *__restrict__ x, const T *__restrict__ y,
                                                     const vec2_t<T> *__restrict__ xy, int64_t ntri,
                                                     double *__restrict__ partials, double *__restrict__ qt_out,
                                                     const StopState *__restrict__ st) {
    __shared__ double s_red[BS / 64];
    if (st && st->done) return;
    double acc = 0.0;
    const int64_t stride = int64_t(gridDim.x) * BS;
    for (int64_t t = int64_t(blockIdx.x) * BS + threadIdx.x; t < ntri; t += stride) {
        const double q = tri_quality_at(x, y, xy, ta[t], tb[t], tc[t]);
        if (qt_out) qt_out[t] = q;
        acc += q * tw[t];
    }
    const double s = block_sum<BS>(acc, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Sum of the partials in a fixed order, times 1/|V|.
__device__ double reduce_partials(const double *__restrict__ partials, int nparts, double inv_n,
                                  double *s_red) {
    double acc = 0.0;
    for (int i = int(threadIdx.x); i < nparts; i += 256) acc += partials[i];
    const double s = block_sum<256>(acc, s_red);
    return s * inv_n;
}

// Stopping rule of Algorithm 1, evaluated on the device after each sweep
// (init: before the first sweep).  Single workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_stop(const double *__restrict__ partials, int nparts,
                                              double inv_n, StopState *st, int init, int use_q_prev,
                                              double q_prev_given, double tol, double goal,
                                              int32_t max_iters) {
    __shared__ double s_red[4];
    if (st->done) return;
    const double Q = reduce_partials(partials, nparts, inv_n, s_red);
    if (threadIdx.x != 0) return;
    if (init) {
        const double q0 = use_q_prev ? q_prev_given : Q;
        st->q0 = q0;
        st->q_prev = q0;
        st->q_last = q0;
        st->iters = 0;
        st->last_dq = __builtin_nan("");
        if (q0 >= goal) {
            st->stopped_by = LMS_STOP_GOAL;
            st->done = 1;
        } else if (max_iters <= 0) {
            st->stopped_by = LMS_STOP_MAX_ITERS;
            st->done = 1;
        }
        return;
    }
    const int32_t k = st->iters + 1;
    const double dq = Q - st->q_prev;
    st->iters = k;
    st->q_last = Q;
    st->last_dq = dq;
    if (Q >= goal) {
        st->stopped_by = LMS_STOP_GOAL;
        st->done = 1;
    } else if (dq < tol) {
        st->stopped_by = LMS_STOP_TOL;
        st->done = 1;
    } else if (k >= max_iters) {
        st->stopped_by = LMS_STOP_MAX_ITERS;
        st->done = 1;
    }
    st->q_prev = Q;
}

// The stopping rule for the fused path, after each quality-fused pass (one
// workgroup): apply the rule to each state the pass evaluated (s, s+1, ...,
// one per sweep it started, or s alone for a depth-0 pass), in order, from
// the tiles' partial sums plus the all-fixed constant.  On a stop at state
// s+j the final state is j sweeps past the pass's source copy: record both;
// else advance `swept` past the pass.  Each thread sums a fixed set of tiles
// (four independent loads in flight), so the order is the same every run.
// First level of the fused stopping rule's sum when there are many tiles:
// block b sums its fixed slice of the tiles' partials for each state the
// pass evaluated (the same shape every run, so the same order).
__global__ __launch_bounds__(256) void k_sum_tiles(const double *__restrict__ qpart, int32_t tiles, int32_t kp,
                                                   const StopState *__restrict__ st, int32_t max_iters,
                                                   double *__restrict__ out) {
    __shared__ double s_red[4];
    if (st->done) return;
    const int32_t k = min(kp, max_iters - st->swept);
    const int32_t nq = k > 0 ? k : 1;
    const int64_t P = gridDim.x, b = blockIdx.x;
    const int64_t lo = b * tiles / P, hi = (b + 1) * tiles / P;
    for (int32_t j = 0; j < nq; ++j) {
        const double *p = qpart + int64_t(j) * tiles;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * 256) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = i0 + q * 256 < hi ? p[i0 + q * 256] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += v[q];
        }
        const double sum = block_sum<256>((acc[0] + acc[1]) + (acc[2] + acc[3]), s_red);
        if (threadIdx.x == 0) out[int64_t(j) * P + b] = sum;
        __syncthreads();
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_stop_tb(const double *__restrict__ qpart, int32_t tiles, int32_t kp,
                                                StopState *st, StopArgs a) {
    __shared__ double s_red_arr[NT / 64];
    __shared__ int stop_flag;
    double *s_red = s_red_arr;
    int *stop = &stop_flag;
    if (st->done) return;
    const int32_t s0 = st->swept;
    const int32_t k = min(kp, a.max_iters - s0);
    const int32_t nq = k > 0 ? k : 1;
    if (threadIdx.x == 0) *stop = 0;
    for (int32_t j = 0; j < nq; ++j) {
        __syncthreads();
        const double *p = qpart + int64_t(j) * tiles;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int32_t i0 = int32_t(threadIdx.x); i0 < tiles; i0 += 4 * NT) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = i0 + q * NT < tiles ? p[i0 + q * NT] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += v[q];
        }
        const double sum = block_sum<NT>((acc[0] + acc[1]) + (acc[2] + acc[3]), s_red);
        if (threadIdx.x == 0) {
            const double Q = (sum + st->q_const) * a.inv_n;
            const int32_t it = s0 + j;
            bool done = false;
            if (it == 0) {
                const double q0 = a.use_q_prev ? a.q_prev_given : Q;
                st->q0 = q0;
                st->q_prev = q0;
                st->q_last = q0;
                st->iters = 0;
                st->last_dq = __builtin_nan("");
                if (q0 >= a.goal) {
                    st->stopped_by = LMS_STOP_GOAL;
                    done = true;
                } else if (a.max_iters <= 0) {
                    st->stopped_by = LMS_STOP_MAX_ITERS;
                    done = true;
                }
            } else {
                const double dq = Q - st->q_prev;
                st->iters = it;
                st->q_last = Q;
                st->last_dq = dq;
                if (Q >= a.goal) {
                    st->stopped_by = LMS_STOP_GOAL;
                    done = true;
                } else if (dq < a.tol) {
                    st->stopped_by = LMS_STOP_TOL;
                    done = true;
                } else if (it >= a.max_iters) {
                    st->stopped_by = LMS_STOP_MAX_ITERS;
                    done = true;
                }
                st->q_prev = Q;
            }
            if (done) {
                st->redo = j;
                st->src = a.src_index;
                st->done = 1;
                *stop = 1;
            }
        }
        __syncthreads();
        if (*stop) return;
    }
    if (threadIdx.x == 0) st->swept = s0 + k;
}

// Sum of w_t q_t over the triangles whose corners are all fixed (their
// quality never changes during smoothing) into st->q_const.
template <typename T>
__global__ __launch_bounds__(256) void k_qconst(const int32_t *__restrict__ ids, const double *__restrict__ w,
                                                int64_t cnt, const vec2_t<T> *__restrict__ xy, StopState *st) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < cnt; t += 256) {
        const vec2_t<T> a = xy[ids[3 * t]], b = xy[ids[3 * t + 1]], c = xy[ids[3 * t + 2]];
        acc += tri_quality(double(a.x), double(a.y), double(b.x), double(b.y), double(c.x), double(c.y)) * w[t];
    }
    const double sum = block_sum<256>(acc, s_red);
    if (threadIdx.x == 0) st->q_const = sum;
}

__global__ void k_stop_reset(StopState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->done = 0;
        st->iters = 0;
        st->stopped_by = LMS_STOP_MAX_ITERS;
        st->swept = 0;
        st->q0 = st->q_prev = st->q_last = st->last_dq = __builtin_nan("");
        st->q_const = 0.0;
        st->redo = 0;
        st->src = 0;
    }
}

__global__ __launch_bounds__(256) void k_reduce_out(const double *__restrict__ partials, int nparts,
                                                    double inv_n, double *out) {
    __shared__ double s_red[4];
    const double Q = reduce_partials(partials, nparts, inv_n, s_red);
    if (threadIdx.x == 0) *out = Q;
}

// Per-mesh quality of a batched handle: one workgroup per mesh, over the
// mesh's contiguous range of triangles.
template <typename T>
__global__ __launch_bounds__(256) void k_quality_mesh(const int32_t *__restrict__ ta,
                                                      const int32_t *__restrict__ tb,
                                                      const int32_t *__restrict__ tc,
                                                      const double *__restrict__ tw,
                                                      const T *__restrict__ x, const T *__restrict__ y,
                                                      const int64_t *__restrict__ t_off,
                                                      const int64_t *__restrict__ v_off,
                                                      double *__restrict__ out) {
    __shared__ double s_red[4];
    const int mesh = int(blockIdx.x);
    double acc = 0.0;
    for (int64_t t = t_off[mesh] + threadIdx.x; t < t_off[mesh + 1]; t += 256)
        acc += tri_quality_at<T>(x, y, nullptr, ta[t], tb[t], tc[t]) * tw[t];
    const double s = block_sum<256>(acc, s_red);
    if (threadIdx.x == 0) out[mesh] = s / double(v_off[mesh + 1] - v_off[mesh]);
}

// q_v = mean of q_t over the triangles containing v.
__global__ __launch_bounds__(256) void k_vertex_quality(const int32_t *__restrict__ vt_ptr,
                                                        const int32_t *__restrict__ vt,
                                                        const double *__restrict__ qt, int32_t n,
                                                        double *__restrict__ qv) {
    const int32_t v = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (v >= n) return;
    double s = 0.0;
    const int32_t b = vt_ptr[v], e = vt_ptr[v + 1];
    for (int32_t i = b; i < e; ++i) s += qt[vt[i]];
    qv[v] = s / double(e - b);
}

template <typename T>
__global__ __launch_bounds__(256) void k_permute(const int32_t *__restrict__ new2old,
                                                 const T *__restrict__ sx, const T *__restrict__ sy,
                                                 T *__restrict__ dx, T *__restrict__ dy, int32_t n,
                                                 int inverse) {
    const int32_t k = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (k >= n) return;
    const int32_t v = new2old[k];
    if (inverse) {
        dx[v] = sx[k];
        dy[v] = sy[k];
    } else {
        dx[k] = sx[v];
        dy[k] = sy[v];
    }
}

// ---------------------------------------------------------------------------
// Runtime

namespace {

constexpr int kQualBS = 256;
constexpr int kQualMaxBlocks = 8192;
constexpr int kChunk = 16;  // sweeps per captured chunk under the stopping rule (even)

struct GraphEntry {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

bool env_flag(const char *name, bool dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return !(v[0] == '0' || v[0] == 'n' || v[0] == 'N' || v[0] == 'f' || v[0] == 'F');
}

}  // namespace

struct DeviceState {
    int device = -1;
    uint64_t version = ~uint64_t(0);
    std::vector<void *> arrays;  // mesh arrays of the current version
    int32_t *row_ptr = nullptr, *col = nullptr, *color_list = nullptr, *new2old = nullptr;
    int32_t *ell = nullptr;  // padded adjacency (row-major), when the handle has one
    int32_t *color_ell = nullptr;  // colour-major padded adjacency
    struct HaloDev {
        int32_t ts = 0, h_max = 0;
        int32_t *halo_ptr = nullptr, *halo = nullptr;
        uint16_t *lidx = nullptr;
    };
    std::deque<HaloDev> halos;   // uploaded tile plans of the current version (stable references)
    struct TBDev {
        int32_t ts = 0, k = 0, u_cap = 0, l_cap = 0, tiles = 0, l_max = 0, u_max = 0;
        bool patches = false;
        bool fits = false;
        int32_t *tile_ptr = nullptr, *ring = nullptr, *halo = nullptr;
        int64_t *halo_ptr = nullptr, *lidx_ptr = nullptr;
        uint16_t *lidx = nullptr;
        // quality-fused form (uploaded on first use under the stopping rule)
        bool q_ready = false, q_fits = false;
        int64_t *qtri_ptr = nullptr;
        uint32_t *qtri = nullptr;
        double *qpart = nullptr;  // k x tiles partial sums
        double *qpart2 = nullptr; // k x nsum first-level sums (many tiles), else unused
        int32_t nsum = 0;
        int32_t *qc_ids = nullptr;
        double *qc_w = nullptr;
        int64_t n_qc = 0;
    };
    std::deque<TBDev> tbs;       // uploaded temporal-blocking plans of the current version
    struct MCDev {
        int32_t ts = 0, l_cap = 0, u_cap = 0, tiles = 0, l_max = 0, colors = 0;
        bool fits = false;
        int32_t *tile_ptr = nullptr, *halo = nullptr;
        int64_t *halo_ptr = nullptr, *upd_ptr = nullptr;
        uint16_t *urow = nullptr, *uidx = nullptr;
        bool q_ready = false, q_fits = false;
        int64_t *qtri_ptr = nullptr;
        uint32_t *qtri = nullptr;
        double *qpart = nullptr, *qpart2 = nullptr, *qc_w = nullptr;
        int32_t *qc_ids = nullptr;
        int32_t nsum = 0;
        int64_t n_qc = 0;
    };
    std::deque<MCDev> mcs;       // uploaded one-pass multicolour plans of the current version
    int mc_cfg[2] = {-2, -2};    // one-pass multicolour variant per precision; -1 = colour by colour; -2 = not tuned
    int small_cfg[2] = {-2, -2}; // batch of small meshes: 1 = all sweeps in one launch, 0 = per sweep; -2 = not decided
    float small_us[2] = {-1.f, -1.f};  // measured one-launch time per sweep (microseconds)
    bool small_used[2] = {false, false};  // the last fixed-K Jacobi call ran the one-launch path
    int32_t *ta = nullptr, *tb = nullptr, *tc = nullptr, *vt_ptr = nullptr, *vt = nullptr;
    double *tw = nullptr;
    int32_t *trec = nullptr;
    int64_t *t_off = nullptr, *v_off = nullptr;
    int64_t *v_cur = nullptr;    // per-mesh vertex offsets in the current labels
    // scratch, kept across versions
    double *partials = nullptr;
    int nparts = 0;
    double *qt = nullptr;
    size_t qt_cap = 0;
    double *qout = nullptr;
    double *qmesh = nullptr;
    StopState *st = nullptr;
    StopState *h_st = nullptr;  // two pinned host mirrors (the check of chunk i while chunk i+1 runs)
    hipEvent_t st_ev[2] = {nullptr, nullptr};
    void *tmp[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [precision][x|y]
    size_t tmp_n[2] = {0, 0};
    hipStream_t cap = nullptr;
    std::vector<GraphEntry> graphs;
    bool use_graphs = true;
    int sweep_cfg[2] = {-1, -1};     // separate-array sweep variant per precision, -1 = not tuned
    int smooth_cfg[2] = {-1, -1};    // variant lms_smooth uses (may sweep the interleaved copy)
    int tb_cfg[2] = {-1, -1};        // temporally blocked variant for fixed-K Jacobi, -1 = none
    int tb_best[2] = {-1, -1};       // fastest temporally blocked variant (the stopping rule's fused pass)
    // end of the handle's last device call: a call on another stream waits
    // for it (the handle's buffers are shared between calls), and nothing the
    // calls may use is freed before it
    hipEvent_t last_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool last_valid = false;
    void *pk[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [precision][ping|pong] interleaved copies
    size_t pk_n[2] = {0, 0};
    float tune_us[2][80] = {};       // measured time per variant (microseconds per sweep)
};

namespace {

void free_graphs(DeviceState *d) {
    for (auto &g : d->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    d->graphs.clear();
}

// Wait until the handle's last device call has finished on the device.
void wait_idle(DeviceState &d) {
    if (d.last_valid) HIP_CHECK(hipEventSynchronize(d.last_done));
}

// Order this call after the handle's last one when it ran on another stream.
void begin_call(DeviceState &d, hipStream_t s) {
    if (d.last_valid && d.last_stream != s) HIP_CHECK(hipStreamWaitEvent(s, d.last_done, 0));
}

void end_call(DeviceState &d, hipStream_t s) {
    HIP_CHECK(hipEventRecord(d.last_done, s));
    d.last_stream = s;
    d.last_valid = true;
}

// Free one array of the current version's set (it must be in d.arrays).
void free_array(DeviceState &d, const void *p) {
    if (!p) return;
    for (size_t i = 0; i < d.arrays.size(); ++i)
        if (d.arrays[i] == p) {
            (void)hipFree(d.arrays[i]);
            d.arrays.erase(d.arrays.begin() + std::ptrdiff_t(i));
            return;
        }
}

void free_arrays(DeviceState *d) {
    for (void *p : d->arrays) (void)hipFree(p);
    d->arrays.clear();
}

template <class T>
T *upload(DeviceState *d, const std::vector<T> &v) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    HIP_CHECK(hipMalloc(&p, bytes));
    d->arrays.push_back(p);
    if (!v.empty()) HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<T *>(p);
}

int quality_blocks(int64_t ntri) {
    const int64_t need = (ntri + 4 * kQualBS - 1) / (4 * kQualBS);
    return int(std::max<int64_t>(1, std::min<int64_t>(need, kQualMaxBlocks)));
}

// Make the device copy of the mesh current (first device call, or after a
// reorder) on the current device.
DeviceState &ensure_device(Mesh &M) {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    if (!M.dev) {
        M.dev.reset(new DeviceState());
        DeviceState *d = M.dev.get();
        d->device = dev;
        d->use_graphs = env_flag("LMS_GRAPH", true);
        HIP_CHECK(hipStreamCreateWithFlags(&d->cap, hipStreamNonBlocking));
        HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d->partials), sizeof(double) * kQualMaxBlocks));
        d->nparts = kQualMaxBlocks;
        HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d->qout), sizeof(double)));
        HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d->st), sizeof(StopState)));
        HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&d->h_st), 2 * sizeof(StopState), hipHostMallocDefault));
        for (auto &e : d->st_ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&d->last_done, hipEventDisableTiming));
    }
    DeviceState *d = M.dev.get();
    if (d->device != dev)
        fail(LMS_ERR_STATE, "handle lives on device " + std::to_string(d->device) + " but device " +
                                std::to_string(dev) + " is current");
    if (d->version != M.version) {
        wait_idle(*d);
        free_graphs(d);
        free_arrays(d);
        d->halos.clear();  // their arrays were in d->arrays
        d->tbs.clear();
        d->mcs.clear();
        d->mc_cfg[0] = d->mc_cfg[1] = -2;
        d->small_cfg[0] = d->small_cfg[1] = -2;
        d->small_us[0] = d->small_us[1] = -1.f;
        d->small_used[0] = d->small_used[1] = false;
        d->version = ~uint64_t(0);
        d->row_ptr = upload(d, M.row_ptr);
        d->col = upload(d, M.col);
        d->ell = M.ell_w > 0 ? upload(d, M.ell) : nullptr;
        d->color_ell = M.ell_w > 0 ? upload(d, M.color_ell) : nullptr;
        d->color_list = upload(d, M.color_list);
        d->new2old = upload(d, M.new2old);
        d->ta = upload(d, M.ta);
        d->tb = upload(d, M.tb);
        d->tc = upload(d, M.tc);
        d->tw = upload(d, M.tw);
        d->trec = M.trec.empty() ? nullptr : upload(d, M.trec);
        d->vt_ptr = upload(d, M.vt_ptr);
        d->vt = upload(d, M.vt);
        d->t_off = upload(d, M.t_off);
        d->v_off = upload(d, M.v_off);
        d->v_cur = upload(d, M.v_off);  // orderings stay within each mesh's range
        void *qm = nullptr;
        HIP_CHECK(hipMalloc(&qm, sizeof(double) * size_t(M.n_mesh)));
        d->arrays.push_back(qm);
        d->qmesh = static_cast<double *>(qm);
        d->sweep_cfg[0] = d->sweep_cfg[1] = -1;  // a new ordering is tuned afresh
        d->smooth_cfg[0] = d->smooth_cfg[1] = -1;
        d->tb_cfg[0] = d->tb_cfg[1] = -1;
        d->tb_best[0] = d->tb_best[1] = -1;
        d->version = M.version;
    }
    return *d;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

size_t elem_size(lms_precision p) { return p == LMS_FP64 ? sizeof(double) : sizeof(float); }

void check_precision(lms_precision p) {
    if (p != LMS_FP64 && p != LMS_FP32) fail(LMS_ERR_ARG, "unknown precision");
}

void launch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(LMS_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

// The sweep kernel variants the autotuner chooses from.  All of them sum each
// row in ascending neighbour order from 0, so they return identical bits.
// MAP is the tile order (see tile_of: 0 linear, -1 one range per XCD, k runs
// of k tiles per XCD).
//   ROW(id, BS, U, R, MAP, NT)   k_jacobi_row
//   LDS(id, BS, CAP, MAP)        k_jacobi
//   ELL(id, BS, W, R, MAP)       k_jacobi_ell (eligible when the padded width is W)
//   ELL2(id, BS, W, R, MAP)      k_jacobi_ell2 on the interleaved copy (lms_smooth only)
//   ROW2(id, BS, U, R, MAP)      k_jacobi_row2 on the interleaved copy (lms_smooth only)
//   HALO(id, TS, W, MAP)         k_jacobi_halo on the interleaved copy (lms_smooth only;
//                                eligible when the padded width is W and the staging fits)
#define LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO) \
    ROW(0, 256, 8, 1, -1, true)                  \
    ROW(1, 256, 8, 1, 0, true)                   \
    ROW(2, 64, 8, 1, -1, true)                   \
    ROW(3, 256, 8, 1, -1, false)                 \
    ROW(4, 256, 8, 2, -1, true)                  \
    ROW(5, 128, 8, 2, -1, false)                 \
    ROW(6, 256, 8, 1, 16, false)                 \
    LDS(7, 256, 2048, -1)                        \
    LDS(8, 128, 1024, -1)                        \
    LDS(9, 64, 512, -1)                          \
    ELL(10, 256, 8, 1, -1)                       \
    ELL(11, 256, 8, 2, -1)                       \
    ELL(12, 128, 8, 2, 0)                        \
    ELL(13, 64, 8, 1, -1)                        \
    ELL(14, 256, 8, 4, -1)                       \
    ELL(15, 256, 12, 1, -1)                      \
    ELL(16, 256, 12, 2, -1)                      \
    ELL(17, 256, 16, 1, -1)                      \
    ELL2(18, 256, 8, 1, -1)                      \
    ELL2(19, 128, 8, 2, 0)                       \
    ELL2(20, 64, 8, 1, -1)                       \
    ELL2(21, 256, 8, 2, -1)                      \
    ELL2(22, 128, 8, 1, 0)                       \
    ELL2(23, 256, 12, 1, -1)                     \
    ELL2(24, 256, 16, 1, -1)                     \
    ELL2(25, 128, 8, 1, 16)                      \
    ELL2(26, 128, 8, 2, 16)                      \
    ELL2(27, 256, 8, 1, 4)                       \
    ELL2(28, 128, 8, 1, 64)                      \
    ELL2(29, 256, 12, 1, 0)                      \
    ELL2(30, 256, 16, 1, 0)                      \
    ROW2(31, 256, 8, 1, 0)                       \
    ROW2(32, 128, 8, 2, 0)                       \
    ROW2(33, 256, 8, 1, -1)                      \
    ROW2(34, 128, 8, 1, 16)                      \
    ROW2(35, 64, 8, 1, 0)                        \
    HALO(36, 256, 8, 0)                          \
    HALO(37, 256, 8, 16)                         \
    HALO(38, 256, 8, -1)                         \
    HALO(39, 128, 8, 0)                          \
    HALO(40, 512, 8, 0)                          \
    HALO(41, 128, 8, 16)                         \
    HALO(42, 256, 12, 0)                         \
    HALO(43, 256, 16, 0)
constexpr int kNumSweepConfigs = 44;
constexpr int kDefaultSweepConfig = 0;

// Temporally blocked variants, k sweeps per pass over memory:
// TB(id, block size, padded width, rows per thread, MAP, nominal tile size,
//    k, staging cap in rows, patches).  A tile whose first sweep would update
// more than block size x rows per thread rows, or whose staging area would
// pass the cap, is halved until it fits.  patches = 0: a tile is a range of
// consecutive rows; 1: a compact patch of free rows grown breadth-first over
// the adjacency, its rows read and written through the staged-row list.  A
// range of an ordering whose walk restarts (RDR's) or that runs in long
// strips (ORI's) is spread out in the mesh and stages about 2.9 rows per own
// row at depth 2; a patch stages about 1.7.
#define LMS_TB_CONFIGS(TB)                   \
    TB(44, 128, 8, 2, 0, 128, 2, 512, 0)     \
    TB(45, 256, 8, 2, 0, 256, 2, 1024, 0)    \
    TB(46, 256, 8, 2, -1, 256, 2, 1024, 0)   \
    TB(47, 256, 8, 2, 16, 256, 2, 1024, 0)   \
    TB(48, 256, 8, 4, 0, 256, 2, 2048, 0)    \
    TB(49, 256, 8, 4, 0, 512, 2, 2048, 0)    \
    TB(50, 256, 8, 4, -1, 512, 2, 2048, 0)   \
    TB(51, 256, 8, 4, 0, 256, 3, 2048, 0)    \
    TB(52, 256, 8, 8, 0, 512, 3, 4096, 0)    \
    TB(53, 256, 8, 8, 0, 1024, 2, 4096, 0)   \
    TB(54, 512, 8, 8, 0, 512, 4, 4096, 0)    \
    TB(55, 128, 8, 2, 16, 128, 2, 512, 0)    \
    TB(56, 256, 12, 4, 0, 512, 2, 2048, 0)   \
    TB(57, 256, 12, 4, -1, 512, 2, 2048, 0)  \
    TB(58, 256, 12, 8, 0, 1024, 2, 4096, 0)  \
    TB(59, 256, 12, 4, 0, 256, 3, 2048, 0)   \
    TB(60, 256, 12, 2, 0, 256, 2, 1024, 0)   \
    TB(61, 256, 16, 4, 0, 512, 2, 2048, 0)   \
    TB(62, 256, 16, 2, 0, 256, 2, 1024, 0)   \
    TB(63, 256, 16, 4, -1, 512, 2, 2048, 0)  \
    TB(64, 256, 8, 2, 16, 256, 2, 1024, 1)   \
    TB(65, 256, 8, 4, 0, 512, 2, 2048, 1)    \
    TB(66, 256, 8, 4, 16, 256, 3, 1024, 1)   \
    TB(67, 256, 8, 8, 0, 512, 4, 2048, 1)    \
    TB(68, 512, 8, 4, 0, 512, 4, 2048, 1)    \
    TB(69, 512, 8, 4, 16, 512, 4, 2048, 1)   \
    TB(70, 512, 8, 4, 0, 512, 3, 2048, 1)    \
    TB(71, 512, 8, 4, 0, 768, 4, 2048, 1)    \
    TB(72, 256, 8, 4, 16, 256, 4, 1024, 1)   \
    TB(73, 1024, 8, 2, 0, 1024, 4, 2048, 1)  \
    TB(74, 1024, 8, 2, 16, 1024, 4, 2048, 1) \
    TB(75, 1024, 8, 3, 0, 1536, 4, 3072, 1)  \
    TB(76, 1024, 8, 4, 0, 2048, 4, 4096, 1)  \
    TB(77, 1024, 8, 3, 0, 1024, 6, 3072, 1)  \
    TB(78, 1024, 8, 4, 0, 1024, 8, 4096, 1)
constexpr int kFirstTBConfig = kNumSweepConfigs;
constexpr int kNumAllConfigs = 79;
static_assert(kNumAllConfigs <= 80, "tune_us holds 80 variants");

struct TBShape {
    int bs = 0, w = 0, r = 0, map = 0, ts = 0, k = 0, lcap = 0, g = 0;  // g: tiles are patches
};

bool is_tb_config(int cfg) { return cfg >= kFirstTBConfig && cfg < kNumAllConfigs; }

TBShape tb_shape(int cfg) {
    switch (cfg) {
#define TB(id, bs, w, r, map, ts, k, lcap, g) \
    case id:                                  \
        return TBShape{bs, w, r, map, ts, k, lcap, g};
        LMS_TB_CONFIGS(TB)
#undef TB
    }
    return TBShape{};
}

// Sweeps one launch of variant cfg performs.
int sweep_config_depth(int cfg) { return is_tb_config(cfg) ? tb_shape(cfg).k : 1; }

std::string map_name(int map) {
    return map == 0 ? "linear" : (map < 0 ? "xcd" : "xcd" + std::to_string(map));
}

std::string sweep_config_name(int cfg) {
    char buf[96];
    if (is_tb_config(cfg)) {
        const TBShape t = tb_shape(cfg);
        std::snprintf(buf, sizeof(buf), "tb/ts%d/k%d/bs%d/w%d/r%d/l%d/%s%s", t.ts, t.k, t.bs, t.w, t.r, t.lcap,
                      map_name(t.map).c_str(), t.g ? "/patch" : "");
        return buf;
    }
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt)                                                              \
    case id:                                                                                    \
        std::snprintf(buf, sizeof(buf), "row/bs%d/u%d/r%d/%s%s", bs, u, r, map_name(map).c_str(), \
                      nt ? "/nt" : "");                                                         \
        return buf;
#define LDS(id, bs, cap, map)                                                                    \
    case id:                                                                                     \
        std::snprintf(buf, sizeof(buf), "lds/bs%d/cap%d/%s", bs, cap, map_name(map).c_str());    \
        return buf;
#define ELL(id, bs, w, r, map)                                                                   \
    case id:                                                                                     \
        std::snprintf(buf, sizeof(buf), "ell/bs%d/w%d/r%d/%s", bs, w, r, map_name(map).c_str()); \
        return buf;
#define ELL2(id, bs, w, r, map)                                                                   \
    case id:                                                                                      \
        std::snprintf(buf, sizeof(buf), "ell2/bs%d/w%d/r%d/%s", bs, w, r, map_name(map).c_str()); \
        return buf;
#define ROW2(id, bs, u, r, map)                                                                   \
    case id:                                                                                      \
        std::snprintf(buf, sizeof(buf), "row2/bs%d/u%d/r%d/%s", bs, u, r, map_name(map).c_str()); \
        return buf;
#define HALO(id, ts, w, map)                                                                      \
    case id:                                                                                      \
        std::snprintf(buf, sizeof(buf), "halo/ts%d/w%d/%s", ts, w, map_name(map).c_str());       \
        return buf;
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
    }
    return "unknown";
}

// Padded width an ELL variant needs (0: not a padded-index variant).
int sweep_config_ell_width(int cfg) {
    if (is_tb_config(cfg)) return tb_shape(cfg).w;
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt) \
    case id:                       \
        return 0;
#define LDS(id, bs, cap, map) \
    case id:                  \
        return 0;
#define ELL(id, bs, w, r, map) \
    case id:                   \
        return w;
#define ELL2(id, bs, w, r, map) \
    case id:                    \
        return w;
#define ROW2(id, bs, u, r, map) \
    case id:                    \
        return 0;
#define HALO(id, ts, w, map) \
    case id:                 \
        return w;
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
    }
    return -1;
}

// Variants that sweep the interleaved (x, y) working copy.
bool sweep_config_packed(int cfg) {
    if (is_tb_config(cfg)) return true;
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt) \
    case id:                       \
        return false;
#define LDS(id, bs, cap, map) \
    case id:                  \
        return false;
#define ELL(id, bs, w, r, map) \
    case id:                   \
        return false;
#define ELL2(id, bs, w, r, map) \
    case id:                    \
        return true;
#define ROW2(id, bs, u, r, map) \
    case id:                    \
        return true;
#define HALO(id, ts, w, map) \
    case id:                 \
        return true;
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
    }
    return false;
}

int sweep_config_tile(int cfg) {
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt)
#define LDS(id, bs, cap, map)
#define ELL(id, bs, w, r, map)
#define ELL2(id, bs, w, r, map)
#define ROW2(id, bs, u, r, map)
#define HALO(id, ts, w, map) \
    case id:                 \
        return ts;
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
        default:
            return 0;
    }
}

bool sweep_config_eligible(int cfg, const Mesh &M) {
    const int w = sweep_config_ell_width(cfg);
    return w == 0 || (w > 0 && w == M.ell_w);
}

int grid_for(int64_t n, int rows_per_block) { return int((n + rows_per_block - 1) / rows_per_block); }

const DeviceState::HaloDev *find_halo(const DeviceState &d, int32_t ts) {
    for (const auto &h : d.halos)
        if (h.ts == ts) return &h;
    return nullptr;
}

// Build (host) and upload the tile plan of the halo-staged sweep for tile size ts.
const DeviceState::HaloDev &ensure_halo(DeviceState &d, Mesh &M, int32_t ts) {
    if (const DeviceState::HaloDev *h = find_halo(d, ts)) return *h;
    const Mesh::HaloPlan &P = halo_plan(M, ts);
    DeviceState::HaloDev h;
    h.ts = ts;
    h.h_max = P.h_max;
    h.halo_ptr = upload(&d, P.halo_ptr);
    h.halo = upload(&d, P.halo);
    h.lidx = upload(&d, P.lidx);
    d.halos.push_back(h);
    return d.halos.back();
}

const DeviceState::TBDev *find_tb(const DeviceState &d, const TBShape &t) {
    for (const auto &h : d.tbs)
        if (h.ts == t.ts && h.k == t.k && h.u_cap == t.bs * t.r && h.l_cap == t.lcap && h.patches == (t.g != 0))
            return &h;
    return nullptr;
}

// Build (host) and upload the temporal-blocking plan of variant shape t.
const DeviceState::TBDev &ensure_tb(DeviceState &d, Mesh &M, const TBShape &t) {
    if (const DeviceState::TBDev *h = find_tb(d, t)) return *h;
    const auto t0 = std::chrono::steady_clock::now();
    const Mesh::TBPlan &P = tb_plan(M, t.ts, t.k, t.bs * t.r, t.lcap, t.g != 0);
    if (env_flag("LMS_VERBOSE", false))
        std::fprintf(stderr, "[lms] tile plan %s ts=%d k=%d: %d tiles, %s, %.2f s\n", t.g ? "patches" : "ranges", t.ts,
                     t.k, P.tiles, P.fits ? "fits" : "does not fit",
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    DeviceState::TBDev h;
    h.ts = t.ts;
    h.k = t.k;
    h.patches = t.g != 0;
    h.u_cap = t.bs * t.r;
    h.l_cap = t.lcap;
    h.fits = P.fits;
    h.tiles = P.tiles;
    h.l_max = P.l_max;
    h.u_max = P.u_max;
    h.tile_ptr = upload(&d, P.tile_ptr);
    h.ring = upload(&d, P.ring);
    h.halo_ptr = upload(&d, P.halo_ptr);
    h.halo = upload(&d, P.halo);
    h.lidx_ptr = upload(&d, P.lidx_ptr);
    h.lidx = upload(&d, P.lidx);
    d.tbs.push_back(h);
    return d.tbs.back();
}

// The quality-fused form of a temporally blocked plan (false when some
// vertex lies in more than 65535 triangles).
bool ensure_tbq(DeviceState &d, Mesh &M, const TBShape &t) {
    DeviceState::TBDev *h = const_cast<DeviceState::TBDev *>(find_tb(d, t));
    if (!h || !h->fits) fail(LMS_ERR_STATE, "quality-fused pass without its tile plan");
    if (h->q_ready) return h->q_fits;
    Mesh::TBPlan *P = nullptr;
    for (auto &p : M.tb_plans)
        if (p.ts == t.ts && p.k == t.k && p.u_cap == t.bs * t.r && p.l_cap == t.lcap && p.patches == (t.g != 0) &&
            p.version == M.version)
            P = &p;
    if (!P) fail(LMS_ERR_STATE, "tile plan missing on the host");
    tb_quality_plan(M, *P);
    h->q_ready = true;
    h->q_fits = P->q_fits;
    if (!h->q_fits) return false;
    h->qtri_ptr = upload(&d, P->qtri_ptr);
    h->qtri = upload(&d, P->qtri);
    h->qc_ids = upload(&d, P->qc_ids);
    h->qc_w = upload(&d, P->qc_w);
    h->n_qc = int64_t(P->qc_w.size());
    h->qpart = upload(&d, std::vector<double>(size_t(t.k) * size_t(std::max(h->tiles, 1)), 0.0));
    // more than 8192 tiles: a first level of ~2048 tiles per block
    h->nsum = h->tiles > 8192 ? std::min(1024, (h->tiles + 2047) / 2048) : 0;
    h->qpart2 = upload(&d, std::vector<double>(size_t(t.k) * size_t(std::max(h->nsum, 1)), 0.0));
    return true;
}

int sweep_config_tile(int cfg);  // tile size of a halo-staged variant, 0 otherwise

// Whether variant cfg can run on this mesh in precision T (builds the tile
// plan of a halo-staged or temporally blocked variant on first use).
template <typename T>
bool sweep_config_usable(int cfg, DeviceState &d, Mesh &M) {
    if (!sweep_config_eligible(cfg, M)) return false;
    if (is_tb_config(cfg)) {
        if (!env_flag("LMS_TEMPORAL_BLOCKING", true) || M.n == 0) return false;
        const DeviceState::TBDev &h = ensure_tb(d, M, tb_shape(cfg));
        return h.fits && size_t(h.l_max) * sizeof(vec2_t<T>) <= size_t(64) * 1024;
    }
    const int ts = sweep_config_tile(cfg);
    if (ts == 0) return true;
    const DeviceState::HaloDev &h = ensure_halo(d, M, ts);
    return size_t(ts + h.h_max) * sizeof(vec2_t<T>) <= size_t(64) * 1024;
}

template <typename T>
void launch_sweep_cfg(int cfg, const DeviceState &d, const Mesh &M, const T *sx, const T *sy, T *dx, T *dy,
                      const StopState *st, hipStream_t s) {
    const int64_t n = M.n;
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt)                                                                         \
    case id:                                                                                               \
        k_jacobi_row<T, bs, u, r, map, nt><<<grid_for(n, bs * r), bs, 0, s>>>(d.row_ptr, d.col, sx, sy, dx, \
                                                                              dy, M.n, st);                 \
        break;
#define LDS(id, bs, cap, map)                                                                                 \
    case id:                                                                                                  \
        k_jacobi<T, bs, cap, map><<<grid_for(n, bs), bs, 0, s>>>(d.row_ptr, d.col, sx, sy, dx, dy, M.n, st);   \
        break;
#define ELL(id, bs, w, r, map)                                                                       \
    case id:                                                                                         \
        if (M.ell_w != w) fail(LMS_ERR_STATE, "padded adjacency width does not match the variant"); \
        k_jacobi_ell<T, bs, w, r, map><<<grid_for(n, bs * r), bs, 0, s>>>(d.ell, sx, sy, dx, dy, M.n, st); \
        break;
#define ELL2(id, bs, w, r, map)
#define ROW2(id, bs, u, r, map)
#define HALO(id, ts, w, map)
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
        default:
            fail(LMS_ERR_STATE, "interleaved or unknown variant launched on separate x, y arrays");
    }
}

// k (1 <= k <= the variant's depth) Jacobi sweeps src -> dst in one pass of
// a temporally blocked variant.  dst's fixed rows are not written.  With
// `qual`, the pass is the quality-fused form: its depth comes from the
// device state (k is ignored) and it writes the tiles' quality sums.
template <typename T>
void launch_tb_cfg(int cfg, const DeviceState &d, const Mesh &M, const vec2_t<T> *src, vec2_t<T> *dst, int32_t k,
                   hipStream_t s, bool qual = false, int32_t max_iters = 0) {
    const TBShape t = tb_shape(cfg);
    const DeviceState::TBDev *h = find_tb(d, t);
    if (!h || !h->fits || M.ell_w != t.w) fail(LMS_ERR_STATE, "temporally blocked variant launched without its plan");
    if (qual) {
        if (!h->q_ready || !h->q_fits) fail(LMS_ERR_STATE, "quality-fused pass without its triangle plan");
        k = t.k;
    }
    if (k < 1 || k > t.k) fail(LMS_ERR_STATE, "temporally blocked pass deeper than its plan");
    if (h->u_max > t.bs * t.r || size_t(h->l_max) * sizeof(vec2_t<T>) > size_t(64) * 1024)
        fail(LMS_ERR_STATE, "temporally blocked plan does not fit the variant");
    if (h->tiles == 0) return;
    const size_t lds = size_t(h->l_max) * sizeof(vec2_t<T>);
    switch (cfg) {
#define TB(id, bs, w, r, map, ts, kk, lcap, g)                                                                 \
    case id:                                                                                                   \
        if (qual)                                                                                              \
            k_jacobi_tb<T, bs, w, r, map, ts, kk, lcap, true, g != 0><<<h->tiles, bs, lds, s>>>(               \
                h->tile_ptr, h->ring, k, h->halo_ptr, h->halo, h->lidx_ptr, h->lidx, src, dst, h->qtri_ptr,     \
                h->qtri, h->qpart, d.st, max_iters);                                                           \
        else                                                                                                   \
            k_jacobi_tb<T, bs, w, r, map, ts, kk, lcap, false, g != 0><<<h->tiles, bs, lds, s>>>(              \
                h->tile_ptr, h->ring, k, h->halo_ptr, h->halo, h->lidx_ptr, h->lidx, src, dst, nullptr,        \
                nullptr, nullptr, nullptr, 0);                                                                 \
        break;
        LMS_TB_CONFIGS(TB)
#undef TB
        default:
            fail(LMS_ERR_STATE, "not a temporally blocked variant");
    }
}

template <typename T>
void launch_sweep2_cfg(int cfg, const DeviceState &d, const Mesh &M, const vec2_t<T> *src, vec2_t<T> *dst,
                       const StopState *st, hipStream_t s) {
    const int64_t n = M.n;
    if (is_tb_config(cfg)) {
        if (st) fail(LMS_ERR_STATE, "temporally blocked variants do not run under the stopping rule");
        launch_tb_cfg<T>(cfg, d, M, src, dst, 1, s);
        return;
    }
    switch (cfg) {
#define ROW(id, bs, u, r, map, nt)
#define LDS(id, bs, cap, map)
#define ELL(id, bs, w, r, map)
#define ELL2(id, bs, w, r, map)                                                                         \
    case id:                                                                                            \
        if (M.ell_w != w) fail(LMS_ERR_STATE, "padded adjacency width does not match the variant");    \
        k_jacobi_ell2<T, bs, w, r, map><<<grid_for(n, bs * r), bs, 0, s>>>(d.ell, src, dst, M.n, st);   \
        break;
#define ROW2(id, bs, u, r, map)                                                                           \
    case id:                                                                                              \
        k_jacobi_row2<T, bs, u, r, map><<<grid_for(n, bs * r), bs, 0, s>>>(d.row_ptr, d.col, src, dst,    \
                                                                           M.n, st);                      \
        break;
#define HALO(id, ts, w, map)                                                                               \
    case id: {                                                                                             \
        const DeviceState::HaloDev *h = find_halo(d, ts);                                                  \
        if (!h || M.ell_w != w) fail(LMS_ERR_STATE, "halo-staged variant launched without its tile plan"); \
        k_jacobi_halo<T, ts, w, map><<<grid_for(n, ts), ts, size_t(ts + h->h_max) * sizeof(vec2_t<T>), s>>>( \
            h->halo_ptr, h->halo, h->lidx, src, dst, M.n, st);                                             \
        break;                                                                                             \
    }
        LMS_SWEEP_CONFIGS(ROW, LDS, ELL, ELL2, ROW2, HALO)
#undef ROW
#undef LDS
#undef ELL
#undef ELL2
#undef ROW2
#undef HALO
        default:
            fail(LMS_ERR_STATE, "separate-array or unknown variant launched on the interleaved copy");
    }
}

template <typename T>
void launch_sweep(const DeviceState &d, const Mesh &M, const T *sx, const T *sy, T *dx, T *dy,
                  const StopState *st, hipStream_t s) {
    launch_sweep_cfg<T>(d.sweep_cfg[sizeof(T) == 8 ? 0 : 1], d, M, sx, sy, dx, dy, st, s);
}

// The handle's two interleaved working copies for precision T.
template <typename T>
vec2_t<T> *ensure_packed(DeviceState &d, int which, int32_t n) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (d.pk_n[pi] < size_t(n)) {
        wait_idle(d);
        for (int w = 0; w < 2; ++w) {
            if (d.pk[pi][w]) (void)hipFree(d.pk[pi][w]);
            d.pk[pi][w] = nullptr;
        }
        d.pk_n[pi] = 0;
        for (int w = 0; w < 2; ++w) HIP_CHECK(hipMalloc(&d.pk[pi][w], sizeof(vec2_t<T>) * size_t(n)));
        d.pk_n[pi] = size_t(n);
        free_graphs(&d);
    }
    return static_cast<vec2_t<T> *>(d.pk[pi][which]);
}

// One-pass multicolour variants: MC(id, tile size, staging cap, updated
// rows per thread R (256 threads), map).
#define LMS_MC_CONFIGS(MC)        \
    MC(0, 128, 1024, 2, 16)       \
    MC(1, 128, 1024, 2, 0)        \
    MC(2, 256, 2048, 4, 16)       \
    MC(3, 64, 512, 1, 16)
constexpr int kNumMcConfigs = 4;

struct MCShape {
    int ts = 0, lcap = 0, r = 0, map = 0;
};

MCShape mc_shape(int cfg) {
    switch (cfg) {
#define MC(id, ts, lcap, r, map) \
    case id:                     \
        return MCShape{ts, lcap, r, map};
        LMS_MC_CONFIGS(MC)
#undef MC
    }
    return MCShape{};
}

// Meshes from this many rows on drop, after each tuning, the tile plans that
// no tuned precision's chosen variants use (host and device): there each plan
// costs ~20-40 bytes per row, and the tuner builds a dozen.
constexpr int32_t kDropPlansFrom = 1 << 22;

void drop_unused_plans(DeviceState &d, Mesh &M) {
    std::vector<int> keep;
    for (int pi = 0; pi < 2; ++pi)
        for (int c : {d.sweep_cfg[pi], d.smooth_cfg[pi], d.tb_cfg[pi], d.tb_best[pi]})
            if (c >= 0) keep.push_back(c);
    auto keep_ts = [&](int32_t ts) {
        for (int c : keep)
            if (!is_tb_config(c) && sweep_config_tile(c) == ts) return true;
        return false;
    };
    auto keep_tb = [&](int32_t ts, int32_t k, int32_t u_cap, int32_t l_cap, bool patches) {
        for (int c : keep)
            if (is_tb_config(c)) {
                const TBShape t = tb_shape(c);
                if (t.ts == ts && t.k == k && t.bs * t.r == u_cap && t.lcap == l_cap && (t.g != 0) == patches)
                    return true;
            }
        return false;
    };
    wait_idle(d);
    for (auto it = d.halos.begin(); it != d.halos.end();) {
        if (keep_ts(it->ts)) {
            ++it;
            continue;
        }
        free_array(d, it->halo_ptr);
        free_array(d, it->halo);
        free_array(d, it->lidx);
        it = d.halos.erase(it);
    }
    for (auto it = d.tbs.begin(); it != d.tbs.end();) {
        if (keep_tb(it->ts, it->k, it->u_cap, it->l_cap, it->patches)) {
            ++it;
            continue;
        }
        for (const void *p : {static_cast<const void *>(it->tile_ptr), static_cast<const void *>(it->ring),
                              static_cast<const void *>(it->halo), static_cast<const void *>(it->halo_ptr),
                              static_cast<const void *>(it->lidx_ptr), static_cast<const void *>(it->lidx),
                              static_cast<const void *>(it->qtri_ptr), static_cast<const void *>(it->qtri),
                              static_cast<const void *>(it->qpart), static_cast<const void *>(it->qpart2),
                              static_cast<const void *>(it->qc_ids), static_cast<const void *>(it->qc_w)})
            free_array(d, p);
        it = d.tbs.erase(it);
    }
    // one-pass multicolour plans: keep the tuned precisions' choices
    auto keep_mc = [&](int32_t ts, int32_t l_cap, int32_t u_cap) {
        for (int pi = 0; pi < 2; ++pi)
            if (d.mc_cfg[pi] >= 0) {
                const MCShape t = mc_shape(d.mc_cfg[pi]);
                if (t.ts == ts && t.lcap == l_cap && 256 * t.r == u_cap) return true;
            }
        return false;
    };
    for (auto it = d.mcs.begin(); it != d.mcs.end();) {
        if (keep_mc(it->ts, it->l_cap, it->u_cap)) {
            ++it;
            continue;
        }
        for (const void *p : {static_cast<const void *>(it->tile_ptr), static_cast<const void *>(it->halo),
                              static_cast<const void *>(it->halo_ptr), static_cast<const void *>(it->upd_ptr),
                              static_cast<const void *>(it->urow), static_cast<const void *>(it->uidx),
                              static_cast<const void *>(it->qtri_ptr), static_cast<const void *>(it->qtri),
                              static_cast<const void *>(it->qpart), static_cast<const void *>(it->qpart2),
                              static_cast<const void *>(it->qc_ids), static_cast<const void *>(it->qc_w)})
            free_array(d, p);
        it = d.mcs.erase(it);
    }
    for (auto it = M.mc_plans.begin(); it != M.mc_plans.end();)
        it = keep_mc(it->ts, it->l_cap, it->u_cap) ? std::next(it) : M.mc_plans.erase(it);
    for (auto it = M.halo_plans.begin(); it != M.halo_plans.end();)
        it = keep_ts(it->ts) ? std::next(it) : M.halo_plans.erase(it);
    for (auto it = M.tb_plans.begin(); it != M.tb_plans.end();)
        it = keep_tb(it->ts, it->k, it->u_cap, it->l_cap, it->patches) ? std::next(it) : M.tb_plans.erase(it);
    M.patch_sets.clear();  // only needed to build plans; a later tuning grows them again
}

// Autotuner: time every sweep variant on this mesh (src -> dst, which leaves
// dst holding one sweep of src) and keep the fastest for the handle's current
// ordering and this precision.  LMS_SWEEP_CONFIG=<id> forces a variant;
// LMS_AUTOTUNE=0 keeps the default.
template <typename T>
void tune_sweep(DeviceState &d, Mesh &M, const T *sx, const T *sy, T *dx, T *dy, hipStream_t s) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (d.sweep_cfg[pi] >= 0) return;
    d.tb_cfg[pi] = d.tb_best[pi] = -1;
    if (const char *f = std::getenv("LMS_SWEEP_CONFIG")) {
        const int c = std::atoi(f);
        if (c < 0 || c >= kNumAllConfigs) fail(LMS_ERR_ARG, "LMS_SWEEP_CONFIG out of range");
        if (!sweep_config_usable<T>(c, d, M)) fail(LMS_ERR_ARG, "LMS_SWEEP_CONFIG names a variant this mesh cannot use");
        d.sweep_cfg[pi] = sweep_config_packed(c) ? kDefaultSweepConfig : c;
        d.smooth_cfg[pi] = is_tb_config(c) ? kDefaultSweepConfig : c;
        if (is_tb_config(c)) d.tb_cfg[pi] = d.tb_best[pi] = c;
        return;
    }
    if (!env_flag("LMS_AUTOTUNE", true)) {
        d.sweep_cfg[pi] = d.smooth_cfg[pi] = kDefaultSweepConfig;
        return;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(hipEventCreate(&e0));
    hipError_t ce = hipEventCreate(&e1);
    if (ce != hipSuccess) {
        (void)hipEventDestroy(e0);
        HIP_CHECK(ce);
    }
    const int64_t work = int64_t(M.n) + int64_t(M.col.size());
    const int reps = work > (int64_t(1) << 26) ? 3 : (work > (int64_t(1) << 22) ? 6 : 12);
    int best = kDefaultSweepConfig, best_all = kDefaultSweepConfig, best_tb = -1;
    float best_ms = 3.0e38f, best_all_ms = 3.0e38f, best_tb_ms = 3.0e38f;  // per sweep
    hipError_t err = hipSuccess;
    vec2_t<T> *pa = nullptr, *pb = nullptr;
    // From 4M rows on, the tuner times fewer temporally blocked variants:
    // each plan costs ~30-40 bytes per row on the host and the device, and
    // growing the patches of one tile size is a pass over the mesh whose
    // accesses follow the ordering (tens of seconds for a random ordering
    // at 64M rows).  There it skips variants over row ranges where patch
    // variants of the same padded width exist (patches won wherever both
    // were measured), and patch variants with tiles under 1024 or over 1536
    // rows (the larger tiles won on every mesh of 16M rows or more).
    auto has_patches = [](int w) {
        for (int c = kFirstTBConfig; c < kNumAllConfigs; ++c)
            if (tb_shape(c).g && tb_shape(c).w == w) return true;
        return false;
    };
    auto skip_large = [&](int c) {
        if (M.n < kDropPlansFrom || !is_tb_config(c)) return false;
        const TBShape t = tb_shape(c);
        return t.g ? (t.ts < 1024 || t.ts > 1536) : has_patches(t.w);
    };
    for (int c = 0; c < kNumAllConfigs && err == hipSuccess; ++c) {
        if (skip_large(c) || !sweep_config_usable<T>(c, d, M)) {
            d.tune_us[pi][c] = -1.f;
            continue;
        }
        const bool packed = sweep_config_packed(c);
        if (packed && !pa) {
            pa = ensure_packed<T>(d, 0, M.n);
            pb = ensure_packed<T>(d, 1, M.n);
            k_pack<T><<<(M.n + 255) / 256, 256, 0, s>>>(sx, sy, pa, pb, M.n);
        }
        const bool tb = is_tb_config(c);
        const int depth = sweep_config_depth(c);
        auto one = [&]() {
            if (tb)
                launch_tb_cfg<T>(c, d, M, pa, pb, depth, s);
            else if (packed)
                launch_sweep2_cfg<T>(c, d, M, pa, pb, nullptr, s);
            else
                launch_sweep_cfg<T>(c, d, M, sx, sy, dx, dy, nullptr, s);
        };
        one();
        one();
        err = hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) one();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ms /= float(reps * depth);
        if (err == hipSuccess && tb && ms < best_tb_ms) {
            best_tb_ms = ms;
            best_tb = c;
        }
        if (err == hipSuccess && !packed && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        if (err == hipSuccess && !tb && ms < best_all_ms) {
            best_all_ms = ms;
            best_all = c;
        }
        d.tune_us[pi][c] = ms * 1000.f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_CHECK(err);
    launch_check();
    d.sweep_cfg[pi] = best;
    d.smooth_cfg[pi] = best_all;
    d.tb_cfg[pi] = best_tb >= 0 && best_tb_ms < best_all_ms ? best_tb : -1;
    d.tb_best[pi] = best_tb;
    if (M.n >= kDropPlansFrom) drop_unused_plans(d, M);
    if (env_flag("LMS_VERBOSE", false)) {
        std::fprintf(stderr,
                     "[lms] sweep autotune (%s, n=%d): %s, %.2f us (separate arrays: %s, %.2f us; "
                     "temporally blocked: %s, %.2f us per sweep)\n",
                     pi == 0 ? "f64" : "f32", M.n, sweep_config_name(best_all).c_str(), double(best_all_ms) * 1000.0,
                     sweep_config_name(best).c_str(), double(best_ms) * 1000.0,
                     best_tb >= 0 ? sweep_config_name(best_tb).c_str() : "none",
                     best_tb >= 0 ? double(best_tb_ms) * 1000.0 : 0.0);
        for (int c = 0; c < kNumAllConfigs; ++c)
            if (d.tune_us[pi][c] >= 0.f)
                std::fprintf(stderr, "[lms]   %2d %-28s %9.2f us\n", c, sweep_config_name(c).c_str(),
                             double(d.tune_us[pi][c]));
    }
}

template <typename T>
void launch_colour_sweep(const DeviceState &d, const Mesh &M, T *x, T *y, const StopState *st,
                         hipStream_t s) {
    for (int32_t c = 0; c < M.n_colors; ++c) {
        const int32_t b = M.color_ptr[c], cnt = M.color_ptr[c + 1] - b;
        if (cnt == 0) continue;
        k_colour<T><<<(cnt + 255) / 256, 256, 0, s>>>(d.row_ptr, d.col, d.color_list + b, cnt, x, y, st);
    }
}

template <typename T>
void launch_colour_sweep2(const DeviceState &d, const Mesh &M, vec2_t<T> *xy, const StopState *st, hipStream_t s) {
    for (int32_t c = 0; c < M.n_colors; ++c) {
        const int32_t b = M.color_ptr[c], cnt = M.color_ptr[c + 1] - b;
        if (cnt == 0) continue;
        const int32_t *list = d.color_list + b;
        const int32_t *cell = d.color_ell + int64_t(M.ell_w) * b;
        const int g = (cnt + 255) / 256;
        switch (M.ell_w) {
            case 8:
                k_colour2<T, 256, 8><<<g, 256, 0, s>>>(list, cell, cnt, xy, st);
                break;
            case 12:
                k_colour2<T, 256, 12><<<g, 256, 0, s>>>(list, cell, cnt, xy, st);
                break;
            case 16:
                k_colour2<T, 256, 16><<<g, 256, 0, s>>>(list, cell, cnt, xy, st);
                break;
            default:
                fail(LMS_ERR_STATE, "no padded colour index for this mesh");
        }
    }
}

template <typename T>
void launch_quality(const DeviceState &d, const Mesh &M, const T *x, const T *y, double *qt_out,
                    const StopState *st, hipStream_t s, const vec2_t<T> *xy = nullptr) {
    if (d.trec)
        k_quality<T, kQualBS><<<quality_blocks(M.T), kQualBS, 0, s>>>(d.trec, x, y, xy, M.T, d.partials, qt_out, st);
    else
        k_quality_wide<T, kQualBS><<<quality_blocks(M.T), kQualBS, 0, s>>>(d.ta, d.tb, d.tc, d.tw, x, y, xy, M.T,
                                                                        d.partials, qt_out, st);
}

void launch_stop(const DeviceState &d, const Mesh &M, int init, const lms_smooth_opts &o, hipStream_t s) {
    const bool use_prev = !std::isnan(o.q_prev);
    k_stop<<<1, 256, 0, s>>>(d.partials, quality_blocks(M.T), 1.0 / double(M.n), d.st, init, use_prev ? 1 : 0,
                             use_prev ? o.q_prev : 0.0, o.tol, o.goal, o.max_iters);
}

// Run `body(stream)` either directly on `s`, or captured once into a graph
// (cached under `key`) that is then launched on `s`.
template <class F>
void run_maybe_graph(DeviceState &d, const std::string &key, hipStream_t s, F body) {
    if (!d.use_graphs) {
        body(s);
        launch_check();
        return;
    }
    for (auto &g : d.graphs)
        if (g.key == key) {
            HIP_CHECK(hipGraphLaunch(g.exec, s));
            return;
        }
    GraphEntry g;
    g.key = key;
    HIP_CHECK(hipStreamBeginCapture(d.cap, hipStreamCaptureModeRelaxed));
    body(d.cap);
    hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(d.cap, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        fail(LMS_ERR_HIP, std::string("kernel launch failed during capture: ") + hipGetErrorString(le));
    }
    if (ce != hipSuccess) fail(LMS_ERR_HIP, std::string("hipStreamEndCapture failed: ") + hipGetErrorString(ce));
    g.graph = graph;
    hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(LMS_ERR_HIP, std::string("hipGraphInstantiate failed: ") + hipGetErrorString(ie));
    }
    if (d.graphs.size() >= 16) {
        (void)hipGraphExecDestroy(d.graphs.front().exec);
        (void)hipGraphDestroy(d.graphs.front().graph);
        d.graphs.erase(d.graphs.begin());
    }
    d.graphs.push_back(g);
    HIP_CHECK(hipGraphLaunch(g.exec, s));
}

std::string ptr_key(const void *p) { return std::to_string(reinterpret_cast<uintptr_t>(p)); }

std::string dbl_key(double v) {
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(bits));
    return std::to_string(bits);
}

void *ensure_tmp(DeviceState &d, lms_precision p, int which, int32_t n) {
    const int pi = p == LMS_FP64 ? 0 : 1;
    if (d.tmp_n[pi] < size_t(n)) {
        wait_idle(d);
        for (int w = 0; w < 2; ++w) {
            if (d.tmp[pi][w]) (void)hipFree(d.tmp[pi][w]);
            d.tmp[pi][w] = nullptr;
        }
        d.tmp_n[pi] = 0;
        for (int w = 0; w < 2; ++w) HIP_CHECK(hipMalloc(&d.tmp[pi][w], elem_size(p) * size_t(n)));
        d.tmp_n[pi] = size_t(n);
        free_graphs(&d);  // graphs may have captured the old pointers
    }
    return d.tmp[pi][which];
}

bool overlaps(const void *a, const void *b, size_t bytes) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bytes && pb < pa + bytes;
}

// Rows per thread the one-launch small-mesh path needs for this batched
// handle (its largest mesh over 256 threads, rounded up to 1, 2, 4, 8 or 16),
// or 0 when the path does not apply: not a batch, no padded index, a mesh
// above 4096 vertices (16-bit slots, the registers and one LDS copy of at most
// 64 KB), or LMS_SMALL_BATCH=0.
int small_batch_rows(const Mesh &M) {
    if (M.n_mesh < 2 || (M.ell_w != 8 && M.ell_w != 12 && M.ell_w != 16)) return 0;
    if (!env_flag("LMS_SMALL_BATCH", true)) return 0;
    int64_t largest = 0;
    for (int32_t i = 0; i < M.n_mesh; ++i) largest = std::max<int64_t>(largest, M.v_off[i + 1] - M.v_off[i]);
    for (int r = 1; r <= 16; r *= 2)
        if (largest <= 256 * r) return r;
    return 0;
}

template <typename T>
void launch_small_meshes(DeviceState &d, const Mesh &M, vec2_t<T> *A, vec2_t<T> *B, int32_t K, int rows,
                         hipStream_t s) {
    int64_t largest = 0;
    for (int32_t i = 0; i < M.n_mesh; ++i) largest = std::max<int64_t>(largest, M.v_off[i + 1] - M.v_off[i]);
    if (rows < 1 || rows > 16 || largest > 256 * int64_t(rows)) fail(LMS_ERR_STATE, "small-mesh rows do not fit");
    const size_t lds = size_t(largest) * sizeof(vec2_t<T>);
    auto go = [&](auto kern) { kern<<<M.n_mesh, 256, lds, s>>>(d.v_cur, d.ell, A, B, K); };
#define LMS_SMALL_R(W)                          \
    switch (rows) {                             \
        case 1: go(k_small_meshes<T, W, 1>); break;   \
        case 2: go(k_small_meshes<T, W, 2>); break;   \
        case 4: go(k_small_meshes<T, W, 4>); break;   \
        case 8: go(k_small_meshes<T, W, 8>); break;   \
        case 16: go(k_small_meshes<T, W, 16>); break; \
        default: fail(LMS_ERR_STATE, "small-mesh rows per thread");   \
    }
    switch (M.ell_w) {
        case 8:
            LMS_SMALL_R(8)
            break;
        case 12:
            LMS_SMALL_R(12)
            break;
        case 16:
            LMS_SMALL_R(16)
            break;
        default:
            fail(LMS_ERR_STATE, "no padded index for the small-mesh path");
    }
#undef LMS_SMALL_R
    launch_check();
}

// Whether a batch of small meshes runs all its sweeps in one launch (one
// workgroup per mesh) or one launch per sweep.  The one-launch kernel wins
// with many meshes; with few, its workgroups leave most of the chip idle and
// the per-sweep path, tuned first, is faster.  So time the one-launch kernel
// over a few sweeps and keep it if its time per sweep beats the per-sweep
// path's tuned one.  LMS_SMALL_BATCH=1 forces the one-launch path, 0 turns it
// off.  Returns the rows per thread of the one-launch kernel, or 0.
template <typename T>
int choose_small_batch(DeviceState &d, Mesh &M, T *x, T *y, T *tx, T *ty, hipStream_t s) {
    const int rows = small_batch_rows(M);
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (rows == 0) return 0;
    if (const char *f = std::getenv("LMS_SMALL_BATCH"); f && *f) return rows;  // forced on (0 gave rows == 0)
    if (d.small_cfg[pi] == -2) {
        tune_sweep<T>(d, M, x, y, tx, ty, s);
        float per_sweep = 3.0e38f;
        for (int c : {d.tb_cfg[pi], d.smooth_cfg[pi]})
            if (c >= 0 && d.tune_us[pi][c] >= 0.f) per_sweep = std::min(per_sweep, d.tune_us[pi][c]);
        vec2_t<T> *A = ensure_packed<T>(d, 0, M.n);
        vec2_t<T> *B = ensure_packed<T>(d, 1, M.n);
        k_pack<T><<<(M.n + 255) / 256, 256, 0, s>>>(x, y, A, B, M.n);
        launch_check();
        constexpr int32_t kK = 8, kReps = 3;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_CHECK(hipEventCreate(&e0));
        hipError_t err = hipEventCreate(&e1);
        if (err != hipSuccess) {
            (void)hipEventDestroy(e0);
            HIP_CHECK(err);
        }
        launch_small_meshes<T>(d, M, A, B, 2, rows, s);
        err = hipEventRecord(e0, s);
        for (int r = 0; r < kReps && err == hipSuccess; ++r) launch_small_meshes<T>(d, M, A, B, kK, rows, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIP_CHECK(err);
        d.small_us[pi] = ms * 1000.f / float(kK * kReps);
        d.small_cfg[pi] = d.small_us[pi] < per_sweep ? 1 : 0;
        if (env_flag("LMS_VERBOSE", false))
            std::fprintf(stderr, "[lms] small-mesh batch (%s, %d meshes): one launch %.2f us per sweep, per sweep %.2f us: %s\n",
                         pi == 0 ? "f64" : "f32", M.n_mesh, double(d.small_us[pi]), double(per_sweep),
                         d.small_cfg[pi] == 1 ? "one launch" : "per sweep");
    }
    return d.small_cfg[pi] == 1 ? rows : 0;
}

// Runs the stopping rule's chunks and returns the final device state.  One
// chunk stays queued ahead of the host's check: chunk i+1 is issued before
// the state after chunk i is read back.  The stop flag never goes down and
// all work after it returns at once, so a chunk issued past the stop changes
// nothing.  `max_chunks` bounds the run (each chunk advances or ends it).
template <class F>
StopState run_stop_chunks(DeviceState &d, hipStream_t s, int64_t max_chunks, F issue_chunk) {
    issue_chunk();
    for (int64_t i = 0;; ++i) {
        StopState *slot = d.h_st + (i & 1);
        HIP_CHECK(hipMemcpyAsync(slot, d.st, sizeof(StopState), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipEventRecord(d.st_ev[i & 1], s));
        if (i <= max_chunks) issue_chunk();
        HIP_CHECK(hipEventSynchronize(d.st_ev[i & 1]));
        if (slot->done) return *slot;
        if (i > max_chunks) fail(LMS_ERR_STATE, "the stopping rule made no progress");
    }
}

// The stopping rule after one quality-fused pass: the tiles' sums, in one or
// two fixed-shape levels, then the rule.
void launch_stop_tiles(const DeviceState &d, double *qpart, int32_t tiles, double *qpart2, int32_t nsum, int32_t kp,
                       int32_t max_iters, const StopArgs &sa, hipStream_t s) {
    if (nsum > 0) {
        k_sum_tiles<<<nsum, 256, 0, s>>>(qpart, tiles, kp, d.st, max_iters, qpart2);
        k_stop_tb<1024><<<1, 1024, 0, s>>>(qpart2, nsum, kp, d.st, sa);
    } else {
        k_stop_tb<1024><<<1, 1024, 0, s>>>(qpart, tiles, kp, d.st, sa);
    }
}

void launch_stop_tb(const DeviceState &d, const DeviceState::TBDev &h, int32_t kp, int32_t max_iters,
                    const StopArgs &sa, hipStream_t s) {
    launch_stop_tiles(d, h.qpart, h.tiles, h.qpart2, h.nsum, kp, max_iters, sa, s);
}


// Passes per captured chunk of the quality-fused stopping rule (even, so that
// every chunk starts from copy A).
constexpr int kFusedChunk = 8;

// The temporally blocked variant whose quality-fused form runs the stopping
// rule, or -1 (then sweep and quality pass run separately).
template <typename T>
int fused_stop_cfg(DeviceState &d, Mesh &M) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    const int c = d.tb_best[pi];
    if (c < 0 || !env_flag("LMS_FUSED_QUALITY", true)) return -1;
    return ensure_tbq(d, M, tb_shape(c)) ? c : -1;
}

const DeviceState::MCDev &ensure_mc(DeviceState &d, Mesh &M, const MCShape &t) {
    for (const auto &h : d.mcs)
        if (h.ts == t.ts && h.l_cap == t.lcap && h.u_cap == 256 * t.r) return h;
    const Mesh::MCPlan &P = mc_plan(M, t.ts, t.lcap, 256 * t.r);
    DeviceState::MCDev h;
    h.ts = t.ts;
    h.l_cap = t.lcap;
    h.u_cap = 256 * t.r;
    h.fits = P.fits;
    h.tiles = P.tiles;
    h.l_max = P.l_max;
    h.colors = P.colors;
    if (P.fits) {
        h.tile_ptr = upload(&d, P.tile_ptr);
        h.halo_ptr = upload(&d, P.halo_ptr);
        h.halo = upload(&d, P.halo);
        h.upd_ptr = upload(&d, P.upd_ptr);
        h.urow = upload(&d, P.urow);
        h.uidx = upload(&d, P.uidx);
    }
    d.mcs.push_back(h);
    return d.mcs.back();
}

template <typename T>
bool mc_usable(DeviceState &d, Mesh &M, int cfg) {
    if (M.ell_w != 8 && M.ell_w != 12 && M.ell_w != 16) return false;
    if (M.n_colors < 1 || M.n == 0) return false;
    const DeviceState::MCDev &h = ensure_mc(d, M, mc_shape(cfg));
    return h.fits && h.tiles > 0 && size_t(h.l_max) * sizeof(vec2_t<T>) <= size_t(64) * 1024;
}

// One multicolour sweep src -> dst in one pass of variant cfg.
template <typename T>
void launch_mc_cfg(int cfg, DeviceState &d, const Mesh &M, const vec2_t<T> *src, vec2_t<T> *dst,
                   const StopState *st, hipStream_t s, bool qual = false, int32_t max_iters = 0) {
    const MCShape t = mc_shape(cfg);
    const DeviceState::MCDev *h = nullptr;
    for (const auto &x : d.mcs)
        if (x.ts == t.ts && x.l_cap == t.lcap && x.u_cap == 256 * t.r) h = &x;
    if (!h || !h->fits || h->colors != M.n_colors) fail(LMS_ERR_STATE, "one-pass multicolour variant without its plan");
    if (size_t(h->l_max) * sizeof(vec2_t<T>) > size_t(64) * 1024) fail(LMS_ERR_STATE, "multicolour plan too large");
    if (qual && (!h->q_ready || !h->q_fits || !st)) fail(LMS_ERR_STATE, "quality-fused multicolour pass without its plan");
    const size_t lds = size_t(h->l_max) * sizeof(vec2_t<T>);
    auto go = [&](auto plain, auto fused) {
        if (qual)
            fused<<<h->tiles, 256, lds, s>>>(h->tile_ptr, h->halo_ptr, h->halo, h->upd_ptr, h->urow, h->uidx,
                                             h->colors, src, dst, st, h->qtri_ptr, h->qtri, h->qpart, max_iters);
        else
            plain<<<h->tiles, 256, lds, s>>>(h->tile_ptr, h->halo_ptr, h->halo, h->upd_ptr, h->urow, h->uidx,
                                             h->colors, src, dst, st, nullptr, nullptr, nullptr, 0);
    };
#define LMS_MC_W(W)                                                                                    \
    switch (cfg) {                                                                                     \
        case 0: go(k_colour_tiles<T, 256, W, 2, 16, false>, k_colour_tiles<T, 256, W, 2, 16, true>); break; \
        case 1: go(k_colour_tiles<T, 256, W, 2, 0, false>, k_colour_tiles<T, 256, W, 2, 0, true>); break;   \
        case 2: go(k_colour_tiles<T, 256, W, 4, 16, false>, k_colour_tiles<T, 256, W, 4, 16, true>); break; \
        case 3: go(k_colour_tiles<T, 256, W, 1, 16, false>, k_colour_tiles<T, 256, W, 1, 16, true>); break; \
        default: fail(LMS_ERR_STATE, "unknown one-pass multicolour variant");                           \
    }
    switch (M.ell_w) {
        case 8:
            LMS_MC_W(8)
            break;
        case 12:
            LMS_MC_W(12)
            break;
        case 16:
            LMS_MC_W(16)
            break;
        default:
            fail(LMS_ERR_STATE, "no padded adjacency for the one-pass multicolour sweep");
    }
#undef LMS_MC_W
    launch_check();
}

// Choose, per precision, between the colour-by-colour sweep and the one-pass
// variants by timing one sweep of each (LMS_COLOUR_TILES=0 keeps colour by
// colour; LMS_COLOUR_CONFIG=<id> forces a one-pass variant).
template <typename T>
void tune_colour(DeviceState &d, Mesh &M, vec2_t<T> *A, vec2_t<T> *B, hipStream_t s) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (d.mc_cfg[pi] != -2) return;
    d.mc_cfg[pi] = -1;
    if (!env_flag("LMS_COLOUR_TILES", true) || M.ell_w == 0) return;
    if (const char *f = std::getenv("LMS_COLOUR_CONFIG")) {
        const int c = std::atoi(f);
        if (c < 0 || c >= kNumMcConfigs || !mc_usable<T>(d, M, c))
            fail(LMS_ERR_ARG, "LMS_COLOUR_CONFIG names a one-pass multicolour variant this mesh cannot use");
        d.mc_cfg[pi] = c;
        return;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(hipEventCreate(&e0));
    hipError_t ce = hipEventCreate(&e1);
    if (ce != hipSuccess) {
        (void)hipEventDestroy(e0);
        HIP_CHECK(ce);
    }
    const int reps = M.n > (1 << 22) ? 3 : 8;
    float best = 3.0e38f;
    hipError_t err = hipSuccess;
    for (int c = -1; c < kNumMcConfigs && err == hipSuccess; ++c) {
        if (c >= 0 && !mc_usable<T>(d, M, c)) continue;
        auto one = [&]() {
            if (c < 0)
                launch_colour_sweep2<T>(d, M, A, nullptr, s);
            else
                launch_mc_cfg<T>(c, d, M, A, B, nullptr, s);
        };
        one();
        err = hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) one();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && ms < best) {
            best = ms;
            d.mc_cfg[pi] = c;
        }
        if (env_flag("LMS_VERBOSE", false))
            std::fprintf(stderr, "[lms] multicolour %s: %.2f us per sweep\n",
                         c < 0 ? "colour by colour" : ("one pass, variant " + std::to_string(c)).c_str(),
                         double(ms) * 1000.0 / reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_CHECK(err);
    if (M.n >= kDropPlansFrom) drop_unused_plans(d, M);
}

// The quality-fused form of a one-pass multicolour plan (false when some
// vertex lies in more than 65535 triangles).
bool ensure_mcq(DeviceState &d, Mesh &M, const MCShape &t) {
    DeviceState::MCDev *h = nullptr;
    for (auto &x : d.mcs)
        if (x.ts == t.ts && x.l_cap == t.lcap && x.u_cap == 256 * t.r) h = &x;
    if (!h || !h->fits) fail(LMS_ERR_STATE, "quality-fused multicolour pass without its tile plan");
    if (h->q_ready) return h->q_fits;
    Mesh::MCPlan *P = nullptr;
    for (auto &p : M.mc_plans)
        if (p.ts == t.ts && p.l_cap == t.lcap && p.u_cap == 256 * t.r && p.version == M.version) P = &p;
    if (!P) fail(LMS_ERR_STATE, "multicolour tile plan missing on the host");
    mc_quality_plan(M, *P);
    h->q_ready = true;
    h->q_fits = P->q_fits;
    if (!h->q_fits) return false;
    h->qtri_ptr = upload(&d, P->qtri_ptr);
    h->qtri = upload(&d, P->qtri);
    h->qc_ids = upload(&d, P->qc_ids);
    h->qc_w = upload(&d, P->qc_w);
    h->n_qc = int64_t(P->qc_w.size());
    h->qpart = upload(&d, std::vector<double>(size_t(std::max(h->tiles, 1)), 0.0));
    h->nsum = h->tiles > 8192 ? std::min(1024, (h->tiles + 2047) / 2048) : 0;
    h->qpart2 = upload(&d, std::vector<double>(size_t(std::max(h->nsum, 1)), 0.0));
    return true;
}

// lms_smooth on the interleaved working copies: pack P_0 into both copies,
// sweep back and forth between them (graph-captured), unpack the last one.
template <typename T>
void smooth_packed(Mesh &M, DeviceState &d, T *x, T *y, lms_precision p, lms_scheme sch, const lms_smooth_opts &o,
                   hipStream_t s, lms_smooth_result &r, int small = 0) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    const bool colour = sch == LMS_MULTICOLOR;
    const int cfg = colour ? -1 : d.smooth_cfg[pi];
    const int tb = colour || o.check_quality ? -1 : d.tb_cfg[pi];
    vec2_t<T> *A = ensure_packed<T>(d, 0, M.n);
    vec2_t<T> *B = ensure_packed<T>(d, 1, M.n);
    if (colour) tune_colour<T>(d, M, A, B, s);  // before the pack: it sweeps the working copies
    const int mc = colour ? d.mc_cfg[pi] : -1;    // >= 0: multicolour in one pass per sweep, A/B ping-pong
    const bool in_place = colour && mc < 0;
    const int nb = (M.n + 255) / 256;
    k_pack<T><<<nb, 256, 0, s>>>(x, y, A, in_place ? nullptr : B, M.n);
    launch_check();
    const std::string base = std::string("packed|") + (p == LMS_FP64 ? "f64" : "f32") + "|" + ptr_key(A) + "|" +
                             ptr_key(B) + "|cfg" + std::to_string(cfg) + "|mc" + std::to_string(mc) + "|" +
                             std::to_string(int(sch));
    // one sweep src -> dst (Jacobi or one-pass multicolour), or colour by colour in place on A
    auto sweep_once = [&](vec2_t<T> *src, vec2_t<T> *dst, const StopState *st, hipStream_t cs) {
        if (in_place)
            launch_colour_sweep2<T>(d, M, A, st, cs);
        else if (colour)
            launch_mc_cfg<T>(mc, d, M, src, dst, st, cs);
        else
            launch_sweep2_cfg<T>(cfg, d, M, src, dst, st, cs);
    };
    int32_t iters = 0;
    bool in_b = false;  // the result sits in B
    const int small_rows = colour || o.check_quality ? 0 : small;
    if (small_rows > 0) {
        // every mesh of the batch fits in LDS: all K sweeps in one launch
        const int32_t K = o.max_iters;
        if (K > 0) launch_small_meshes<T>(d, M, A, B, K, small_rows, s);
        iters = K;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (tb >= 0) {
        // temporally blocked: passes of up to `depth` sweeps, ping-pong A/B
        const int32_t K = o.max_iters, depth = sweep_config_depth(tb);
        const int32_t passes = (K + depth - 1) / depth;
        if (K > 0)
            run_maybe_graph(d, "tb|" + base + "|tb" + std::to_string(tb) + "|" + std::to_string(K), s,
                            [&](hipStream_t cs) {
                                int32_t left = K;
                                for (int32_t q = 0; q < passes; ++q) {
                                    const int32_t kk = std::min(left, depth);
                                    launch_tb_cfg<T>(tb, d, M, q % 2 == 0 ? A : B, q % 2 == 0 ? B : A, kk, cs);
                                    left -= kk;
                                }
                            });
        iters = K;
        in_b = passes % 2 == 1;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (!o.check_quality) {
        const int32_t K = o.max_iters;
        if (K > 0)
            run_maybe_graph(d, "fixed|" + base + "|" + std::to_string(K), s, [&](hipStream_t cs) {
                for (int32_t k = 0; k < K; ++k) sweep_once(k % 2 == 0 ? A : B, k % 2 == 0 ? B : A, nullptr, cs);
            });
        iters = K;
        in_b = !in_place && K % 2 == 1;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (const int fq = colour ? -1 : fused_stop_cfg<T>(d, M); fq >= 0) {
        // stopping rule with the quality fused into the sweep passes: each
        // pass evaluates the states it sweeps from; a stop inside a pass is
        // reached again from the pass's source copy
        const TBShape t = tb_shape(fq);
        const DeviceState::TBDev *h = find_tb(d, t);
        k_stop_reset<<<1, 64, 0, s>>>(d.st);
        k_qconst<T><<<1, 256, 0, s>>>(h->qc_ids, h->qc_w, h->n_qc, A, d.st);
        launch_check();
        const bool use_prev = !std::isnan(o.q_prev);
        const std::string key = "stopq|" + base + "|tb" + std::to_string(fq) + "|" + dbl_key(o.tol) + "|" +
                                dbl_key(o.goal) + "|" + std::to_string(o.max_iters);
        // every chunk advances at least kFusedChunk*depth sweeps or ends the run
        const int64_t max_chunks = (int64_t(o.max_iters) + 1) / (int64_t(kFusedChunk) * t.k) + 2;
        const StopState hs = run_stop_chunks(d, s, max_chunks, [&]() {
            run_maybe_graph(d, key, s, [&](hipStream_t cs) {
                for (int q = 0; q < kFusedChunk; ++q) {
                    StopArgs sa{};
                    sa.inv_n = 1.0 / double(M.n);
                    sa.tol = o.tol;
                    sa.goal = o.goal;
                    sa.q_prev_given = use_prev ? o.q_prev : 0.0;
                    sa.use_q_prev = use_prev ? 1 : 0;
                    sa.max_iters = o.max_iters;
                    sa.src_index = q % 2;
                    launch_tb_cfg<T>(fq, d, M, q % 2 == 0 ? A : B, q % 2 == 0 ? B : A, 0, cs, true, o.max_iters);
                    launch_stop_tb(d, *h, t.k, o.max_iters, sa, cs);
                }
            });
        });
        vec2_t<T> *fsrc = hs.src == 0 ? A : B, *fother = hs.src == 0 ? B : A;
        if (hs.redo > 0) launch_tb_cfg<T>(fq, d, M, fsrc, fother, hs.redo, s);
        in_b = (hs.redo > 0 ? fother : fsrc) == B;
        iters = hs.iters;
        r.stopped_by = hs.stopped_by;
        r.q0 = hs.q0;
        r.q_final = hs.q_last;
        r.last_dq = hs.last_dq;
    } else if (colour && mc >= 0 && env_flag("LMS_FUSED_QUALITY", true) && ensure_mcq(d, M, mc_shape(mc))) {
        // multicolour, one pass per sweep, each pass evaluating the quality
        // of the state it sweeps from: a stop is at the source copy of the
        // pass that evaluated it
        const MCShape t = mc_shape(mc);
        const DeviceState::MCDev *h = nullptr;
        for (const auto &xh : d.mcs)
            if (xh.ts == t.ts && xh.l_cap == t.lcap && xh.u_cap == 256 * t.r) h = &xh;
        k_stop_reset<<<1, 64, 0, s>>>(d.st);
        k_qconst<T><<<1, 256, 0, s>>>(h->qc_ids, h->qc_w, h->n_qc, A, d.st);
        launch_check();
        const bool use_prev = !std::isnan(o.q_prev);
        const std::string key = "stopmc|" + base + "|" + dbl_key(o.tol) + "|" + dbl_key(o.goal) + "|" +
                                std::to_string(o.max_iters);
        const StopState hs = run_stop_chunks(d, s, (int64_t(o.max_iters) + 1) / kFusedChunk + 2, [&]() {
            run_maybe_graph(d, key, s, [&](hipStream_t cs) {
                for (int q = 0; q < kFusedChunk; ++q) {
                    StopArgs sa{};
                    sa.inv_n = 1.0 / double(M.n);
                    sa.tol = o.tol;
                    sa.goal = o.goal;
                    sa.q_prev_given = use_prev ? o.q_prev : 0.0;
                    sa.use_q_prev = use_prev ? 1 : 0;
                    sa.max_iters = o.max_iters;
                    sa.src_index = q % 2;
                    launch_mc_cfg<T>(mc, d, M, q % 2 == 0 ? A : B, q % 2 == 0 ? B : A, d.st, cs, true, o.max_iters);
                    launch_stop_tiles(d, h->qpart, h->tiles, h->qpart2, h->nsum, 1, o.max_iters, sa, cs);
                }
            });
        });
        in_b = hs.src == 1;
        iters = hs.iters;
        r.stopped_by = hs.stopped_by;
        r.q0 = hs.q0;
        r.q_final = hs.q_last;
        r.last_dq = hs.last_dq;
    } else {
        k_stop_reset<<<1, 64, 0, s>>>(d.st);
        launch_quality<T>(d, M, nullptr, nullptr, nullptr, nullptr, s, A);
        launch_stop(d, M, 1, o, s);
        launch_check();
        const std::string key = "stop|" + base + "|" + dbl_key(o.tol) + "|" + dbl_key(o.goal) + "|" +
                                std::to_string(o.max_iters);
        const StopState h = run_stop_chunks(d, s, int64_t(o.max_iters) / kChunk + 2, [&]() {
            run_maybe_graph(d, key, s, [&](hipStream_t cs) {
                for (int k = 0; k < kChunk; ++k) {
                    vec2_t<T> *src = k % 2 == 0 ? A : B, *dst = in_place ? A : (k % 2 == 0 ? B : A);
                    sweep_once(src, dst, d.st, cs);
                    launch_quality<T>(d, M, nullptr, nullptr, nullptr, d.st, cs, dst);
                    launch_stop(d, M, 0, o, cs);
                }
            });
        });
        iters = h.iters;
        r.stopped_by = h.stopped_by;
        r.q0 = h.q0;
        r.q_final = h.q_last;
        r.last_dq = h.last_dq;
        in_b = !in_place && iters % 2 == 1;
    }
    k_unpack<T><<<nb, 256, 0, s>>>(in_b ? B : A, x, y, M.n);
    launch_check();
    r.iters = iters;
}

template <typename T>
void smooth_typed(Mesh &M, DeviceState &d, T *x, T *y, T *tx, T *ty, lms_precision p, lms_scheme sch,
                  const lms_smooth_opts &o, hipStream_t s, lms_smooth_result &r) {
    if (sch == LMS_JACOBI) {
        const int pi = sizeof(T) == 8 ? 0 : 1;
        const int small = !o.check_quality && small_batch_rows(M) > 0
                              ? choose_small_batch<T>(d, M, x, y, tx, ty, s)
                              : 0;
        if (!o.check_quality) d.small_used[pi] = small > 0;
        if (small > 0) {
            smooth_packed<T>(M, d, x, y, p, sch, o, s, r, small);
            return;
        }
        tune_sweep<T>(d, M, x, y, tx, ty, s);
        if (sweep_config_packed(d.smooth_cfg[pi]) || (!o.check_quality && d.tb_cfg[pi] >= 0) ||
            (o.check_quality && fused_stop_cfg<T>(d, M) >= 0)) {
            smooth_packed<T>(M, d, x, y, p, sch, o, s, r);
            return;
        }
    } else if (M.ell_w > 0 && env_flag("LMS_PACKED_COLOUR", true)) {
        smooth_packed<T>(M, d, x, y, p, sch, o, s, r);
        return;
    }
    const std::string base = std::string(p == LMS_FP64 ? "f64" : "f32") + "|" + ptr_key(x) + "|" +
                             ptr_key(y) + "|" + ptr_key(tx) + "|" + ptr_key(ty) + "|cfg" +
                             std::to_string(d.sweep_cfg[sizeof(T) == 8 ? 0 : 1]);
    const size_t bytes = sizeof(T) * size_t(M.n);
    const bool jacobi = sch == LMS_JACOBI;
    if (jacobi) {
        // both buffers start as P_0: fixed vertices are then right in either
        HIP_CHECK(hipMemcpyAsync(tx, x, bytes, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(ty, y, bytes, hipMemcpyDeviceToDevice, s));
    }
    if (!o.check_quality) {
        const int32_t K = o.max_iters;
        if (K > 0) {
            run_maybe_graph(d, "fixed|" + base + "|" + std::to_string(int(sch)) + "|" + std::to_string(K), s,
                            [&](hipStream_t cs) {
                                for (int32_t k = 0; k < K; ++k) {
                                    if (!jacobi) {
                                        launch_colour_sweep<T>(d, M, x, y, nullptr, cs);
                                    } else if (k % 2 == 0) {
                                        launch_sweep<T>(d, M, x, y, tx, ty, nullptr, cs);
                                    } else {
                                        launch_sweep<T>(d, M, tx, ty, x, y, nullptr, cs);
                                    }
                                }
                            });
        }
        if (jacobi && (K % 2 == 1)) {
            HIP_CHECK(hipMemcpyAsync(x, tx, bytes, hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipMemcpyAsync(y, ty, bytes, hipMemcpyDeviceToDevice, s));
        }
        r.iters = K;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
        return;
    }
    // Stopping rule on the device: Q_0, then chunks of sweeps each followed by
    // a quality evaluation and the stop test; sweeps after the stop do nothing.
    k_stop_reset<<<1, 64, 0, s>>>(d.st);
    launch_quality<T>(d, M, x, y, nullptr, nullptr, s);
    launch_stop(d, M, 1, o, s);
    launch_check();
    const std::string key = "stop|" + base + "|" + std::to_string(int(sch)) + "|" + dbl_key(o.tol) + "|" + dbl_key(o.goal) +
                            "|" + std::to_string(o.max_iters);
    const StopState h = run_stop_chunks(d, s, int64_t(o.max_iters) / kChunk + 2, [&]() {
        run_maybe_graph(d, key, s, [&](hipStream_t cs) {
            for (int k = 0; k < kChunk; ++k) {
                const bool fwd = (k % 2 == 0);
                if (!jacobi) {
                    launch_colour_sweep<T>(d, M, x, y, d.st, cs);
                    launch_quality<T>(d, M, x, y, nullptr, d.st, cs);
                } else if (fwd) {
                    launch_sweep<T>(d, M, x, y, tx, ty, d.st, cs);
                    launch_quality<T>(d, M, tx, ty, nullptr, d.st, cs);
                } else {
                    launch_sweep<T>(d, M, tx, ty, x, y, d.st, cs);
                    launch_quality<T>(d, M, x, y, nullptr, d.st, cs);
                }
                launch_stop(d, M, 0, o, cs);
            }
        });
    });
    if (jacobi && (h.iters % 2 == 1)) {
        HIP_CHECK(hipMemcpyAsync(x, tx, bytes, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(y, ty, bytes, hipMemcpyDeviceToDevice, s));
    }
    r.iters = h.iters;
    r.stopped_by = h.stopped_by;
    r.q0 = h.q0;
    r.q_final = h.q_last;
    r.last_dq = h.last_dq;
}

}  // namespace

void destroy_device_state(DeviceState *d) {
    if (!d) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (d->device >= 0) (void)hipSetDevice(d->device);
    if (d->last_valid) (void)hipEventSynchronize(d->last_done);
    free_graphs(d);
    free_arrays(d);
    for (auto &pt : d->tmp)
        for (void *p : pt)
            if (p) (void)hipFree(p);
    for (auto &pt : d->pk)
        for (void *p : pt)
            if (p) (void)hipFree(p);
    if (d->partials) (void)hipFree(d->partials);
    if (d->qt) (void)hipFree(d->qt);
    if (d->qout) (void)hipFree(d->qout);
    if (d->st) (void)hipFree(d->st);
    if (d->h_st) (void)hipHostFree(d->h_st);
    for (auto e : d->st_ev)
        if (e) (void)hipEventDestroy(e);
    if (d->cap) (void)hipStreamDestroy(d->cap);
    if (d->last_done) (void)hipEventDestroy(d->last_done);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete d;
}

void dev_permute(Mesh &M, const void *sx, const void *sy, void *dx, void *dy, lms_precision p, int inverse,
                 void *stream) {
    check_precision(p);
    if (!sx || !sy || !dx || !dy) fail(LMS_ERR_ARG, "null coordinate pointer");
    const size_t bytes = elem_size(p) * size_t(M.n);
    if (overlaps(sx, dx, bytes) || overlaps(sx, dy, bytes) || overlaps(sy, dx, bytes) || overlaps(sy, dy, bytes))
        fail(LMS_ERR_ARG, "lms_permute source and destination overlap");
    DeviceState &d = ensure_device(M);
    hipStream_t s = as_stream(stream);
    begin_call(d, s);
    const int nb = (M.n + 255) / 256;
    if (p == LMS_FP64)
        k_permute<double><<<nb, 256, 0, s>>>(d.new2old, static_cast<const double *>(sx), static_cast<const double *>(sy),
                                             static_cast<double *>(dx), static_cast<double *>(dy), M.n, inverse);
    else
        k_permute<float><<<nb, 256, 0, s>>>(d.new2old, static_cast<const float *>(sx), static_cast<const float *>(sy),
                                            static_cast<float *>(dx), static_cast<float *>(dy), M.n, inverse);
    launch_check();
    end_call(d, s);
}

void dev_sweep(Mesh &M, const void *sx, const void *sy, void *dx, void *dy, lms_precision p, void *stream) {
    check_precision(p);
    if (!sx || !sy || !dx || !dy) fail(LMS_ERR_ARG, "null coordinate pointer");
    const size_t bytes = elem_size(p) * size_t(M.n);
    if (overlaps(sx, dx, bytes) || overlaps(sx, dy, bytes) || overlaps(sy, dx, bytes) || overlaps(sy, dy, bytes))
        fail(LMS_ERR_ARG, "a Jacobi sweep cannot run in place");
    DeviceState &d = ensure_device(M);
    hipStream_t s = as_stream(stream);
    begin_call(d, s);
    if (p == LMS_FP64) {
        tune_sweep<double>(d, M, static_cast<const double *>(sx), static_cast<const double *>(sy),
                           static_cast<double *>(dx), static_cast<double *>(dy), s);
        launch_sweep<double>(d, M, static_cast<const double *>(sx), static_cast<const double *>(sy),
                             static_cast<double *>(dx), static_cast<double *>(dy), nullptr, s);
    } else {
        tune_sweep<float>(d, M, static_cast<const float *>(sx), static_cast<const float *>(sy),
                          static_cast<float *>(dx), static_cast<float *>(dy), s);
        launch_sweep<float>(d, M, static_cast<const float *>(sx), static_cast<const float *>(sy),
                            static_cast<float *>(dx), static_cast<float *>(dy), nullptr, s);
    }
    launch_check();
    end_call(d, s);
}

void dev_smooth(Mesh &M, void *x, void *y, void *tx, void *ty, lms_precision p, lms_scheme sch,
                const lms_smooth_opts &o, void *stream, lms_smooth_result &r) {
    check_precision(p);
    if (sch != LMS_JACOBI && sch != LMS_MULTICOLOR) fail(LMS_ERR_ARG, "unknown scheme");
    if (!x || !y) fail(LMS_ERR_ARG, "null coordinate pointer");
    if (o.max_iters < 0) fail(LMS_ERR_ARG, "max_iters must be >= 0");
    if (std::isnan(o.tol) || std::isnan(o.goal)) fail(LMS_ERR_ARG, "tol and goal must not be NaN");
    const size_t bytes = elem_size(p) * size_t(M.n);
    if (overlaps(x, y, bytes)) fail(LMS_ERR_ARG, "x and y overlap");
    DeviceState &d = ensure_device(M);
    hipStream_t s = as_stream(stream);
    begin_call(d, s);
    if (sch == LMS_JACOBI) {
        if ((tx == nullptr) != (ty == nullptr)) fail(LMS_ERR_ARG, "give both tx and ty, or neither");
        if (!tx) {
            tx = ensure_tmp(d, p, 0, M.n);
            ty = ensure_tmp(d, p, 1, M.n);
        }
        if (overlaps(tx, ty, bytes) || overlaps(tx, x, bytes) || overlaps(tx, y, bytes) || overlaps(ty, x, bytes) ||
            overlaps(ty, y, bytes))
            fail(LMS_ERR_ARG, "Jacobi scratch buffers must not overlap the coordinates");
    }
    if (p == LMS_FP64)
        smooth_typed<double>(M, d, static_cast<double *>(x), static_cast<double *>(y), static_cast<double *>(tx),
                             static_cast<double *>(ty), p, sch, o, s, r);
    else
        smooth_typed<float>(M, d, static_cast<float *>(x), static_cast<float *>(y), static_cast<float *>(tx),
                            static_cast<float *>(ty), p, sch, o, s, r);
    end_call(d, s);
}

std::string dev_sweep_config(Mesh &M, lms_precision p) {
    check_precision(p);
    if (!M.dev || M.dev->version != M.version) return "";
    const int pi = p == LMS_FP64 ? 0 : 1;
    const int c = M.dev->smooth_cfg[pi];
    // a batch of small meshes that runs all sweeps in one launch names that first
    std::string small;
    if (M.dev->small_used[pi]) small = "small/r" + std::to_string(small_batch_rows(M)) + "/one-launch";
    if (c < 0) return small;
    // then the variant a fixed-K Jacobi lms_smooth runs, then the one it runs
    // under the stopping rule
    std::string out = M.dev->tb_cfg[pi] >= 0 ? sweep_config_name(M.dev->tb_cfg[pi]) + " " + sweep_config_name(c)
                                             : sweep_config_name(c);
    if (!small.empty()) out = small + " " + out;
    char buf[64];
    for (int i = 0; i < kNumAllConfigs; ++i) {
        std::snprintf(buf, sizeof(buf), "%s%d:%.2fus", i == 0 ? " tuned[" : " ", i,
                      double(M.dev->tune_us[p == LMS_FP64 ? 0 : 1][i]));
        out += buf;
    }
    return out + "]";
}

void dev_quality(Mesh &M, const void *x, const void *y, lms_precision p, double *q_global, double *q_vertex,
                 double *q_mesh, void *stream) {
    check_precision(p);
    if (!x || !y) fail(LMS_ERR_ARG, "null coordinate pointer");
    DeviceState &d = ensure_device(M);
    hipStream_t s = as_stream(stream);
    begin_call(d, s);
    if (q_mesh) {
        if (p == LMS_FP64)
            k_quality_mesh<double><<<M.n_mesh, 256, 0, s>>>(d.ta, d.tb, d.tc, d.tw, static_cast<const double *>(x),
                                                            static_cast<const double *>(y), d.t_off, d.v_off, d.qmesh);
        else
            k_quality_mesh<float><<<M.n_mesh, 256, 0, s>>>(d.ta, d.tb, d.tc, d.tw, static_cast<const float *>(x),
                                                           static_cast<const float *>(y), d.t_off, d.v_off, d.qmesh);
        launch_check();
        HIP_CHECK(hipMemcpyAsync(q_mesh, d.qmesh, sizeof(double) * size_t(M.n_mesh), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        end_call(d, s);
        return;
    }
    double *qt_out = nullptr;
    if (q_vertex) {
        if (d.qt_cap < size_t(M.T)) {
            wait_idle(d);
            if (d.qt) (void)hipFree(d.qt);
            d.qt = nullptr;
            d.qt_cap = 0;
            HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d.qt), sizeof(double) * size_t(M.T)));
            d.qt_cap = size_t(M.T);
        }
        qt_out = d.qt;
    }
    if (p == LMS_FP64)
        launch_quality<double>(d, M, static_cast<const double *>(x), static_cast<const double *>(y), qt_out, nullptr, s);
    else
        launch_quality<float>(d, M, static_cast<const float *>(x), static_cast<const float *>(y), qt_out, nullptr, s);
    launch_check();
    if (q_vertex) {
        k_vertex_quality<<<(M.n + 255) / 256, 256, 0, s>>>(d.vt_ptr, d.vt, d.qt, M.n, q_vertex);
        launch_check();
    }
    if (q_global) {
        k_reduce_out<<<1, 256, 0, s>>>(d.partials, quality_blocks(M.T), 1.0 / double(M.n), d.qout);
        launch_check();
        HIP_CHECK(hipMemcpyAsync(q_global, d.qout, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    end_call(d, s);
}

}  // namespace lms
