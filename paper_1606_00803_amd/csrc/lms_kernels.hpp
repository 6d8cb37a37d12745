// Kernels of the smoothing library for gfx950 (MI355X): the sweeps of
// Eq. 1 in their layouts, the temporally blocked and multicolour passes,
// the quality of Section 3.2 and the stopping rule of Section 5.1, layout
// and label changes.  Device code only; included by lms_device.hip, which
// holds the runtime that launches them.
//
// Compiled with -ffp-contract=off: the sweep sums and the quality arithmetic
// are exactly the IEEE operations written (no fused multiply-add).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lms_divide.hpp"
#include "lms_internal.hpp"

namespace lms {

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

// Sum over a row's neighbours in LDS, in slot order (the row's ascending
// neighbour order), from 0, and their count.  slot(q) is the row's q-th
// 16-bit slot, 0xFFFF past its end.  Each read sits behind its own branch and
// waits for its value: the reads of the other waves on the SIMD cover that
// wait.  A form with all of a row's reads in flight at once needed ~20 more
// registers, which let one 1024-thread workgroup per CU run instead of two,
// and measured slower on every ordering.
template <typename T, int W, class Slot>
__device__ __forceinline__ int lds_row_sum(const vec2_t<T> *sp, Slot slot, T &ax, T &ay) {
    T sx = T(0), sy = T(0);
    int c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const uint32_t id = slot(q);
        if (id != 0xFFFFu) {
            const vec2_t<T> p = sp[id];
            sx += p.x;
            sy += p.y;
            ++c;
        }
    }
    ax = sx;
    ay = sy;
    return c;
}

// The same from byte offsets into sp, two per word (offset 2q in the low half
// of word q, 0xFFFF past the row's end): the address is the offset itself.
template <typename T, int W>
__device__ __forceinline__ int lds_row_sum_bytes(const vec2_t<T> *sp, const uint32_t (&wd)[W / 2], T &ax, T &ay) {
    const unsigned char *base = reinterpret_cast<const unsigned char *>(sp);
    T sx = T(0), sy = T(0);
    int c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const uint32_t off = (wd[q / 2] >> (16 * (q % 2))) & 0xFFFFu;
        if (off != 0xFFFFu) {
            const vec2_t<T> p = *reinterpret_cast<const vec2_t<T> *>(base + off);
            sx += p.x;
            sy += p.y;
            ++c;
        }
    }
    ax = sx;
    ay = sy;
    return c;
}

// Slots packed two per word -> byte offsets into an array of vec2_t<T>
// (0xFFFF stays): a staging area of at most 4096 rows keeps every offset
// below 0xFFFF.
template <typename T, int W>
__device__ __forceinline__ void slots_to_bytes(uint32_t (&wd)[W / 2]) {
    constexpr uint32_t s = uint32_t(sizeof(vec2_t<T>));
#pragma unroll
    for (int q = 0; q < W / 2; ++q) {
        const uint32_t lo = wd[q] & 0xFFFFu, hi = wd[q] >> 16;
        wd[q] = (lo == 0xFFFFu ? lo : lo * s) | ((hi == 0xFFFFu ? hi : hi * s) << 16);
    }
}

// The same for slots packed two per word (slot 2q in the low half of word q).
template <typename T, int W>
__device__ __forceinline__ int lds_row_sum_words(const vec2_t<T> *sp, const uint32_t (&wd)[W / 2], T &ax, T &ay) {
    return lds_row_sum<T, W>(sp, [&](int q) { return (wd[q / 2] >> (16 * (q % 2))) & 0xFFFFu; }, ax, ay);
}

// Stage rows ids[0..cnt) of src into sp[base + j], four per thread per step:
// the ids, then the coordinates, each as four loads in flight together.  An
// index past cnt is clamped to cnt-1, so that lane loads and stores entry
// cnt-1's own value again: no branch holds a load back.
template <typename T, int BS>
__device__ __forceinline__ void stage_rows(const int32_t *__restrict__ ids, int32_t cnt,
                                           const vec2_t<T> *__restrict__ src, vec2_t<T> *sp, int32_t base,
                                           int tid) {
    for (int32_t j0 = tid; j0 < cnt; j0 += 4 * BS) {
        int32_t j[4], g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) j[q] = min(j0 + q * BS, cnt - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = ids[j[q]];
        vec2_t<T> h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = src[g[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q) sp[base + j[q]] = h[q];
    }
}

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

// The same in patch order: position i of the working copies holds label[i].
template <typename T>
__global__ __launch_bounds__(256) void k_pack_pm(const T *__restrict__ x, const T *__restrict__ y,
                                                 const int32_t *__restrict__ label, vec2_t<T> *__restrict__ a,
                                                 vec2_t<T> *__restrict__ b, int32_t n) {
    const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (i >= n) return;
    const int32_t v = label[i];
    vec2_t<T> p;
    p.x = x[v];
    p.y = y[v];
    a[i] = p;
    if (b) b[i] = p;
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack_pm(const vec2_t<T> *__restrict__ a, const int32_t *__restrict__ label,
                                                   T *__restrict__ x, T *__restrict__ y, int32_t n) {
    const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
    if (i >= n) return;
    const vec2_t<T> p = a[i];
    const int32_t v = label[i];
    x[v] = p.x;
    y[v] = p.y;
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
    extern __shared__ __align__(16) unsigned char lds_raw[];
    vec2_t<T> *stage = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if (st && st->done) return;
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t v = tile * TS + tid;
    uint16_t li[W];
    load_row_slots<W>(lidx + (int64_t(tile) * TS + tid) * W, li);
    if (v < n) stage[tid] = src[v];
    const int32_t hb = halo_ptr[tile], he = halo_ptr[tile + 1];
    stage_rows<T, TS>(halo + hb, he - hb, src, stage, TS, tid);
    __syncthreads();
    T ax, ay;
    const int c = lds_row_sum<T, W>(stage, [&](int q) { return uint32_t(li[q]); }, ax, ay);
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

// w_t q_t of one triangle of a tile from its 16-byte record (slots a | b<<16,
// slot c, then w_t = 1/|T(a)| + 1/|T(b)| + 1/|T(c)| as a double, the value
// the host computed for the quality pass): the corners come from LDS.
template <typename T>
__device__ __forceinline__ double tri_record_term(const vec2_t<T> *sp, const u32x4 &w) {
    const vec2_t<T> pa = sp[w.x & 0xFFFFu], pb = sp[w.x >> 16], pc = sp[w.y];
    const double q = tri_quality(double(pa.x), double(pa.y), double(pb.x), double(pb.y), double(pc.x), double(pc.y));
    return q * __hiloint2double(int(w.w), int(w.z));
}
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
// G (patch tiles): the working copies are stored patch by patch (position p
// holds label pm_label[p]): tile t's own rows are positions tile_ptr[t] ..
// tile_ptr[t+1]-1, read and written as one contiguous run, and its staged-row
// list (halo_ptr/halo, in positions) starts with those own rows, then its
// rings.  Range tiles store rows by label (pm_label null) and list only their
// rings.
//
// ox, oy (non-null only for the last pass of a fixed-K call without quality):
// the last sweep writes the own free rows to these separate x and y arrays,
// by label, instead of dst, so no unpack of dst follows.
//
// float64, and the quality-fused form in either precision: a row's slots are
// kept as byte offsets and decoded again in every sweep, and the quotient
// comes from div_by_count with 1/c from an LDS table.  The compiler would
// otherwise keep every slot's address in its own register across the sweeps,
// which takes a variant with three rows per thread past 64 registers, so that
// only one 1024-thread workgroup fits on a CU; this way it holds ~50 and two
// fit.  Plain float32 rows fit either way and keep the hoisted addresses and
// the plain division, which measured faster.
//
// QUAL (the stopping rule, Section 5.1): the pass also evaluates the quality
// (Section 3.2) of each state it starts a sweep from.  Before sweep j+1 the
// own rows and ring 1 hold state s+j, and every triangle of the tile (those
// whose smallest free corner is an own row) has its corners there; the
// tile's sum of w_t q_t goes to qpart[j*gridDim.x + tile].  The depth comes
// from the device state: k = min(KP, max_iters - swept), and a pass of depth
// 0 (all sweeps done) evaluates its source state only.
template <typename T, int BS, int W, int R, int MAP, int TS, int KP, int LCAP, bool QUAL, bool G>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(QUAL && R <= 2 && BS == 1024 ? 8 : 1))) void
k_jacobi_tb(const int32_t *__restrict__ tile_ptr,
                                                  const int32_t *__restrict__ ring, int32_t k,
                                                  const int64_t *__restrict__ halo_ptr,
                                                  const int32_t *__restrict__ halo,
                                                  const int64_t *__restrict__ lidx_ptr,
                                                  const uint16_t *__restrict__ lidx,
                                                  const vec2_t<T> *__restrict__ src, vec2_t<T> *__restrict__ dst,
                                                  T *__restrict__ ox, T *__restrict__ oy,
                                                  const int32_t *__restrict__ pm_label,
                                                  const int64_t *__restrict__ qtri_ptr,
                                                  const uint32_t *__restrict__ qtri, double *__restrict__ qpart,
                                                  const StopState *__restrict__ st, int32_t max_iters) {
    static_assert(W % 4 == 0, "padded width must be a multiple of 4");
    // the quality-fused form on 1024 threads and two rows per thread reads its
    // triangle records from memory for every state and is held to 64
    // registers, so that two workgroups fit on a CU; the others keep QR
    // records per thread in registers
    constexpr bool FIT2 = QUAL && R <= 2 && BS == 1024;
    constexpr int QR = FIT2 ? 0 : 2;
    constexpr bool BYTES = sizeof(T) == 8 || QUAL;  // slots as byte offsets, quotient by div_by_count
    static_assert(!BYTES || LCAP * sizeof(vec2_t<T>) <= 65536, "byte offsets fit 16 bits");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double s_red[BS / 64];
    __shared__ T s_inv[BYTES ? W + 1 : 1];  // RN(1/c), c = 1..W
    vec2_t<T> *sp = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if constexpr (BYTES)
        if (threadIdx.x <= W) s_inv[threadIdx.x] = threadIdx.x == 0 ? T(0) : T(1) / T(int(threadIdx.x));
    if constexpr (QUAL) {
        if (st->done) return;
        k = min(KP, max_iters - st->swept);
    }
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t b = tile_ptr[tile];  // first own row (a position, for patches)
    static_assert(KP >= 1 && KP <= 8 && TS > 0 && LCAP > 0, "plan shape");
    const int32_t *rc = ring + int64_t(tile) * (KP + 1);
    const int32_t nown = rc[0], nload = rc[k > 0 ? k : 1], nupd = k > 0 ? rc[k - 1] : 0;
    const int64_t hb = halo_ptr[tile], lb = lidx_ptr[tile];
    u32x4 qw[QUAL && QR > 0 ? QR : 1];
    int64_t qb = 0, qe = 0;
    if constexpr (QUAL) {
        qb = qtri_ptr[tile];
        qe = qtri_ptr[tile + 1];
#pragma unroll
        for (int r = 0; r < QR; ++r) {
            const int64_t t = qb + tid + BS * r;
            qw[r] = u32x4{0u, 0u, 0u, 0u};  // weight 0: no triangle
            if (t < qe) qw[r] = reinterpret_cast<const u32x4 *>(qtri)[t];
        }
    }
    uint32_t wd[R][W / 2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t i = tid + BS * r;
        if (i < nupd) {
            load_slot_words<W>(lidx + (lb + i) * W, wd[r]);
            if constexpr (BYTES) slots_to_bytes<T, W>(wd[r]);
        } else {
#pragma unroll
            for (int q = 0; q < W / 2; ++q) wd[r][q] = 0xFFFFFFFFu;
        }
    }
    for (int32_t i = tid; i < nown; i += BS) sp[i] = src[b + i];
    // the rings, through the list (which, for patches, starts with the own rows)
    stage_rows<T, BS>(halo + hb + (G ? nown : 0), nload - nown, src, sp, nown, tid);
    __syncthreads();
    const int32_t passes = QUAL && k == 0 ? 1 : k;
    for (int32_t j = 1; j <= passes; ++j) {
        if constexpr (QUAL) {
            // quality of state s+j-1: every triangle of the tile, from LDS
            auto tri_term = [&](const u32x4 &w) { return tri_record_term<T>(sp, w); };
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < QR; ++r)
                if (qw[r].w != 0u) acc += tri_term(qw[r]);
            for (int64_t t = qb + QR * BS + tid; t < qe; t += BS)
                acc += tri_term(reinterpret_cast<const u32x4 *>(qtri)[t]);
            const double sum = block_sum<BS>(acc, s_red);
            if (tid == 0) qpart[int64_t(j - 1) * gridDim.x + tile] = sum;
            __syncthreads();  // s_red is reused by the next state's sum
            if (k == 0) break;
        }
        const int32_t m = rc[k - j];  // rows updated by this sweep
        if constexpr (BYTES) {
            // the words are opaque to the compiler here, so it decodes them in
            // each sweep instead of holding W addresses per row
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < W / 2; ++q) asm volatile("" : "+v"(wd[r][q]));
        }
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
            T ax, ay;
            const int c = BYTES ? lds_row_sum_bytes<T, W>(sp, wd[r], ax, ay) : lds_row_sum_words<T, W>(sp, wd[r], ax, ay);
            w[r] = c > 0;
            if (c > 0) {
                if constexpr (BYTES) {
                    const T y = s_inv[c];
                    o[r].x = div_by_count(ax, T(c), y);
                    o[r].y = div_by_count(ay, T(c), y);
                } else {
                    o[r].x = ax / T(c);
                    o[r].y = ay / T(c);
                }
            }
        }
        if (j == k) {
            if (ox) {
                int32_t lab[R];
#pragma unroll
                for (int r = 0; r < R; ++r)  // labels of the own rows, loads in flight together
                    lab[r] = G ? pm_label[b + min(tid + BS * r, nown - 1)] : b + tid + BS * r;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (w[r]) {
                        ox[lab[r]] = o[r].x;
                        oy[lab[r]] = o[r].y;
                    }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (w[r]) dst[b + tid + BS * r] = o[r];
            }
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
    extern __shared__ __align__(16) unsigned char lds_raw[];
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
            T ax, ay;
            const int c = lds_row_sum_words<T, W>(sp, slot[r], ax, ay);
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
//
// G (patch tiles): the own rows are the first nown entries of the staged
// list (halo_ptr/halo cover every staged row), read and written through it.
//
// KP > 1 (several sweeps per pass): sweep t of the plan (t = 1..KP) updates
// the rows whose mask has bit t-1: the last sweep the own free rows and the
// lower-colour rows they read at its value; each earlier sweep the
// higher-colour rows the next one reads at the previous value, closed the same
// way.  A pass of depth d runs sweeps KP-d+1..KP, in LDS, colour by colour.
template <typename T, int BS, int W, int R, int MAP, bool QUAL, bool G, int KP>
__global__ __launch_bounds__(BS) void k_colour_tiles(const int32_t *__restrict__ tile_ptr,
                                                     const int64_t *__restrict__ halo_ptr,
                                                     const int32_t *__restrict__ halo,
                                                     const int64_t *__restrict__ upd_ptr,
                                                     const uint16_t *__restrict__ urow,
                                                     const uint16_t *__restrict__ uidx,
                                                     const uint8_t *__restrict__ umask, int32_t C, int32_t depth,
                                                     const vec2_t<T> *__restrict__ src, vec2_t<T> *__restrict__ dst,
                                                     const StopState *__restrict__ st,
                                                     const int64_t *__restrict__ qtri_ptr,
                                                     const uint32_t *__restrict__ qtri, double *__restrict__ qpart,
                                                     int32_t max_iters) {
    static_assert(KP >= 1 && KP <= 8, "sweeps per pass");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double s_red[BS / 64];
    vec2_t<T> *sp = reinterpret_cast<vec2_t<T> *>(lds_raw);
    if (st && st->done) return;
    if constexpr (QUAL) depth = min(1, max_iters - st->swept);
    const int tile = tile_of<MAP>(int(blockIdx.x), int(gridDim.x));
    const int tid = int(threadIdx.x);
    const int32_t b = tile_ptr[tile], nown = tile_ptr[tile + 1] - b;
    const int64_t hb = halo_ptr[tile];
    const int32_t nh = int32_t(halo_ptr[tile + 1] - hb);  // rows read through the list
    const int32_t g0 = G ? 0 : nown;                      // slot of its first entry
    // this thread's updated rows (the tile's list, colour by colour): slot,
    // colour and neighbour slots, held in registers for the whole pass
    const int64_t *up = upd_ptr + int64_t(tile) * (C + 1);
    uint32_t wd[R][W / 2];
    int32_t row[R], colr[R];
    uint32_t msk[KP > 1 ? R : 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t e = up[0] + tid + BS * r;
        colr[r] = -1;
        row[r] = 0;
        if constexpr (KP > 1) msk[r] = 0u;
        if (e < up[C]) {
            load_slot_words<W>(uidx + e * W, wd[r]);
            row[r] = urow[e];
            if constexpr (KP > 1) msk[r] = umask[e];
            int32_t c = 0;
            while (up[c + 1] <= e) ++c;
            colr[r] = c;
        }
    }
    if constexpr (!G)
        for (int32_t i = tid; i < nown; i += BS) sp[i] = src[b + i];
    stage_rows<T, BS>(halo + hb, nh, src, sp, g0, tid);
    __syncthreads();
    if constexpr (QUAL) {
        // quality of the source state: the tile's triangles, from LDS
        double acc = 0.0;
        for (int64_t t = qtri_ptr[tile] + tid; t < qtri_ptr[tile + 1]; t += BS)
            acc += tri_record_term<T>(sp, reinterpret_cast<const u32x4 *>(qtri)[t]);
        const double sum = block_sum<BS>(acc, s_red);
        if (tid == 0) qpart[tile] = sum;
        if (depth == 0) return;  // all sweeps done: the state was evaluated only
        __syncthreads();
    }
    for (int32_t t = KP - depth + 1; t <= KP; ++t) {
        for (int32_t c = 0; c < C; ++c) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (colr[r] != c) continue;
                if constexpr (KP > 1)
                    if (!((msk[r] >> (t - 1)) & 1u)) continue;
                T ax, ay;
                const int cnt = lds_row_sum_words<T, W>(sp, wd[r], ax, ay);
                if (cnt > 0) {
                    vec2_t<T> o;
                    o.x = ax / T(cnt);
                    o.y = ay / T(cnt);
                    sp[row[r]] = o;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t i = tid; i < nown; i += BS) dst[G ? halo[hb + i] : b + i] = sp[i];
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
    // q = sqrt(mn / mx) in [0, 1]: 1/mx from the hardware estimate and two
    // Newton steps, then the square root of the ratio from the hardware
    // reciprocal-square-root estimate and a coupled Newton refinement of
    // sqrt and 1/(2 sqrt); a few units in the last place from the correctly
    // rounded sqrt(mn) / sqrt(mx).  Outside the range where the estimates
    // are exact enough (tiny or huge squared lengths), the rounded operations.
    if (!(mx > 0.0)) return 0.0;
    if (mx < 0x1p-900 || mx > 0x1p900 || mn < 0x1p-900) return sqrt(mn) / sqrt(mx);
    double r = __builtin_amdgcn_rcp(mx);
    r = fma(r, fma(-mx, r, 1.0), r);
    r = fma(r, fma(-mx, r, 1.0), r);
    const double s = mn * r;
    if (s < 0x1p-1000) return sqrt(mn) / sqrt(mx);
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, s);
    return fma(d, h, g);
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
// from which w_t is recomputed in the same order as on the host: 1/c from a
// 64-entry table filled by the same division, beyond it divided); each
// thread takes four triangles per step, loads first.
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_quality(const int32_t *__restrict__ trec, const T *__restrict__ x,
                                                const T *__restrict__ y, const vec2_t<T> *__restrict__ xy,
                                                int64_t ntri, double *__restrict__ partials,
                                                double *__restrict__ qt_out, const StopState *__restrict__ st) {
    __shared__ double s_red[BS / 64];
    __shared__ double s_rcp[65];
    if (st && st->done) return;
    for (int c = int(threadIdx.x); c <= 64; c += BS) s_rcp[c] = c == 0 ? 0.0 : 1.0 / double(c);
    __syncthreads();
    auto rcp = [&](uint32_t c) { return c <= 64u ? s_rcp[c] : 1.0 / double(c); };
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
                const double w = rcp(cnt & 1023u) + rcp((cnt >> 10) & 1023u) + rcp(cnt >> 20);
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

}  // namespace lms
