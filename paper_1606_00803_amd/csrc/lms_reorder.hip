// Reordering on the GPU (gfx950): the breadth-first ordering and the
// relabelling of every array that follows the current labels (the
// permutation apply of Algorithm 2's V_new <- V).  Both give exactly what
// the host path gives (order_bfs and relabel), bit for bit; the host then
// adopts the arrays.
//
// Breadth-first order (the BFS baseline of Sections 1 and 5.2.1): from label
// 0, neighbours in ascending label, restarting at the smallest unvisited
// label.  Components are visited in the order of their smallest label, so
// one multi-source level-synchronous search from every component's smallest
// label gives each component's queue order, if each newly reached vertex is
// claimed by the earliest frontier position that reaches it (a 64-bit
// atomicMin on (level, position)) and then placed in its claimer's
// ascending neighbour order.  The order is then component by component,
// level by level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "lms_internal.hpp"

namespace lms {

#define RHIP_CHECK(expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(e_ == hipErrorOutOfMemory ? LMS_ERR_ALLOC : LMS_ERR_HIP,                  \
                 std::string(#expr) + " failed: " + hipGetErrorString(e_));                \
    } while (0)

namespace {

void rlaunch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(LMS_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
}

constexpr int kBS = 256;
int blocks_for(int64_t n) { return int(std::max<int64_t>(1, (n + kBS - 1) / kBS)); }

// ---- exclusive scan (int64), out[n] = total ------------------------------
constexpr int kScanIPT = 16;
constexpr int kScanItems = kBS * kScanIPT;

__global__ __launch_bounds__(kBS) void k_scan_block(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                    int64_t n, int64_t *__restrict__ block_sums) {
    __shared__ int64_t s[kBS];
    const int64_t base = int64_t(blockIdx.x) * kScanItems + int64_t(threadIdx.x) * kScanIPT;
    int64_t v[kScanIPT];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanIPT; ++q) {
        v[q] = base + q < n ? in[base + q] : 0;
        sum += v[q];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kBS; off <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
        const int64_t t = threadIdx.x >= unsigned(off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - sum;  // exclusive prefix of this thread
#pragma unroll
    for (int q = 0; q < kScanIPT; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == kBS - 1) block_sums[blockIdx.x] = s[kBS - 1];
}

__global__ __launch_bounds__(kBS) void k_scan_add(int64_t *__restrict__ out, int64_t n,
                                                  const int64_t *__restrict__ offsets) {
    const int64_t i = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (i < n) out[i] += offsets[i / kScanItems];
}

__global__ void k_scan_total(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ in) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

// out[0..n] = exclusive scan of in[0..n), out[n] the total.  in and out may
// not overlap.
void scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (n + kScanItems - 1) / kScanItems);
    int64_t *sums = nullptr, *offs = nullptr;
    RHIP_CHECK(hipMalloc(&sums, sizeof(int64_t) * size_t(nb)));
    RHIP_CHECK(hipMalloc(&offs, sizeof(int64_t) * size_t(nb + 1)));
    k_scan_block<<<int(nb), kBS, 0, s>>>(in, out, n, sums);
    rlaunch_check();
    if (nb > 1) {
        scan(sums, offs, nb, s);
        k_scan_add<<<blocks_for(n), kBS, 0, s>>>(out, n, offs);
        rlaunch_check();
    }
    k_scan_total<<<1, 64, 0, s>>>(out, n, in);
    rlaunch_check();
    RHIP_CHECK(hipStreamSynchronize(s));
    (void)hipFree(sums);
    (void)hipFree(offs);
}

// ---- small per-segment sorts (rows of neighbours, triangle lists) --------
// Ascending sort of a[0..m): insertion sort for short segments, heapsort
// beyond (a vertex of high degree).
template <typename K>
__device__ void seg_sort(K *a, int64_t m) {
    if (m <= 32) {
        for (int64_t i = 1; i < m; ++i) {
            const K x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) {
                a[j + 1] = a[j];
                --j;
            }
            a[j + 1] = x;
        }
        return;
    }
    auto sift = [&](int64_t root, int64_t end) {
        while (2 * root + 1 < end) {
            int64_t c = 2 * root + 1;
            if (c + 1 < end && a[c] < a[c + 1]) ++c;
            if (!(a[root] < a[c])) return;
            const K t = a[root];
            a[root] = a[c];
            a[c] = t;
            root = c;
        }
    };
    for (int64_t i = m / 2 - 1; i >= 0; --i) sift(i, m);
    for (int64_t end = m - 1; end > 0; --end) {
        const K t = a[0];
        a[0] = a[end];
        a[end] = t;
        sift(0, end);
    }
}

// ---- connected components: every vertex gets its component's smallest label
__global__ void k_cc_init(int32_t *comp, int32_t n) {
    const int32_t v = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (v < n) comp[v] = v;
}

// hook: for each edge (v, u) with comp[u] < comp[v] and comp[v] a root, move
// that root under comp[u] (atomicMin: a root only ever moves to a smaller id)
__global__ void k_cc_hook(const int64_t *__restrict__ ptr, const int32_t *__restrict__ adj, int32_t *comp,
                          int32_t n, int32_t *changed) {
    const int32_t v = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (v >= n) return;
    const int32_t cv = comp[v];
    for (int64_t j = ptr[v]; j < ptr[v + 1]; ++j) {
        const int32_t cu = comp[adj[j]];
        if (cu < cv && comp[cv] == cv) {
            if (atomicMin(&comp[cv], cu) > cu) *changed = 1;
        }
    }
}

// shortcut: comp[v] <- comp[comp[v]] until every vertex points at a root
__global__ void k_cc_shortcut(int32_t *comp, int32_t n, int32_t *changed) {
    const int32_t v = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (v >= n) return;
    int32_t c = comp[v];
    while (comp[c] != c) c = comp[c];
    if (comp[v] != c) {
        comp[v] = c;
        *changed = 1;
    }
}

// ---- breadth-first search ------------------------------------------------
// root flags and component sizes; a wavefront whose vertices all lie in one
// component (the usual case) adds its count with one atomic instead of 64
__global__ void k_root_flags(const int32_t *__restrict__ comp, int64_t *flag, int64_t *size_at_root, int32_t n) {
    const int32_t v = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    const bool valid = v < n;
    const int32_t c = valid ? comp[v] : -1;
    if (valid) flag[v] = c == v ? 1 : 0;
    const int32_t c0 = __shfl(c, 0, 64);
    const bool uniform = __all(!valid || c == c0);
    if (uniform) {
        const int cnt = __popcll(__ballot(valid));
        if ((threadIdx.x & 63) == 0 && c0 >= 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&size_at_root[c0]), (unsigned long long)cnt);
    } else if (valid) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&size_at_root[c]), 1ull);
    }
}

// frontier 0: the roots in ascending label; claim[root] = (0 << 32) | position
__global__ void k_seed(const int32_t *__restrict__ comp, const int64_t *__restrict__ rank, int32_t *frontier,
                       uint64_t *claim, int32_t n) {
    const int32_t v = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (v >= n) return;
    claim[v] = ~uint64_t(0);
    if (comp[v] == v) {
        frontier[rank[v]] = v;
        claim[v] = uint64_t(rank[v]);
    }
}

// ---- the whole level loop in one workgroup --------------------------------
// Frontiers of these meshes hold hundreds to tens of thousands of vertices
// over thousands of levels, so one workgroup runs every level, with workgroup
// barriers between the phases instead of a launch (and a host round trip for
// the next frontier's size) per level.  A frontier of up to kFrontLds
// vertices, the next frontier of a frontier of at most one chunk, stays in
// LDS; any other goes to global memory.  Per level, in
// frontier order:
//   1. place each entry after its component's earlier levels, at its offset
//      from the first entry of its component in this level (the frontier
//      keeps components in rank order, each contiguous), and claim every
//      neighbour for the earliest position that reaches it (atomicMin on
//      (level, position));
//   2. the last entry of each component adds the level's count to it, each
//      entry counts the neighbours it claimed, an exclusive scan gives its
//      offset in the next frontier, and it appends them in ascending label.
// Claims and component counts are read and written with device-scope
// atomics; a frontier in global memory is read after a device-scope fence on
// each side of the barrier.

constexpr int kOneBS = 1024;
constexpr int kFrontLds = 7936;  // two LDS frontiers within 64 KiB

enum class ScanOp { Sum, Max };

// Inclusive scan of v over the workgroup (wave shuffles, then the wave
// totals in LDS); *total receives the reduction of the whole workgroup.
template <ScanOp OP>
__device__ int64_t wg_scan_incl(int64_t v, int64_t *s_w, int64_t *total) {
    const int lane = int(threadIdx.x) & 63, w = int(threadIdx.x) >> 6;
    auto op = [](int64_t a, int64_t b) { return OP == ScanOp::Sum ? a + b : (a > b ? a : b); };
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t t = __shfl_up(v, off, 64);
        if (lane >= off) v = op(v, t);
    }
    if (lane == 63) s_w[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = OP == ScanOp::Sum ? 0 : -1;
        for (int i = 0; i < kOneBS / 64; ++i) {
            const int64_t t = s_w[i];
            s_w[i] = run;  // what the waves before wave i hold
            run = op(run, t);
        }
        s_w[kOneBS / 64] = run;
    }
    __syncthreads();
    const int64_t r = op(s_w[w], v);
    *total = s_w[kOneBS / 64];
    __syncthreads();  // s_w is reused by the next scan
    return r;
}

__device__ __forceinline__ int64_t load_done(int64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_claim(uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kOneBS) void k_bfs_one_group(const int64_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ adj,
                                                         const int32_t *__restrict__ comp,
                                                         const int64_t *__restrict__ comp_start, int64_t *done,
                                                         uint64_t *claim, int32_t *ga, int32_t *gb, int64_t m0,
                                                         int32_t *order, int32_t n, int32_t *bad,
                                                         int64_t *placed_out) {
    __shared__ int64_t s_w[kOneBS / 64 + 1];
    __shared__ int32_t s_front[2][kFrontLds];
    const int tid = int(threadIdx.x);
    // the first frontier (the roots) arrives in ga
    int32_t *front = ga;
    int64_t m = m0, placed = 0;
    for (uint64_t level = 0; m > 0; ++level) {
        if (level > uint64_t(n)) {  // cannot happen: every level places at least one vertex
            if (tid == 0) *bad = 1;
            break;
        }
        const uint64_t tag = (level + 1) << 32;
        // 1. placement and claims
        int64_t carry = -1;  // first position of the component running into this chunk
        for (int64_t base = 0; base < m; base += kOneBS) {
            const int64_t p = base + tid;
            const bool valid = p < m;
            const int32_t v = valid ? front[p] : 0;
            const int32_t c = valid ? comp[v] : -1;
            const bool head = valid && (p == 0 || comp[front[p - 1]] != c);
            int64_t chunk_max;
            int64_t first = wg_scan_incl<ScanOp::Max>(head ? p : -1, s_w, &chunk_max);
            if (first < 0) first = carry;
            carry = chunk_max >= 0 ? chunk_max : carry;
            if (valid) {
                const int64_t at = comp_start[c] + load_done(&done[c]) + (p - first);
                if (first < 0 || at < comp_start[c] || at >= comp_start[c + 1] || at >= n)
                    *bad = 1;
                else
                    order[at] = v;
                const uint64_t want = tag | uint64_t(p);
                for (int64_t j = ptr[v]; j < ptr[v + 1]; ++j)
                    atomicMin(reinterpret_cast<unsigned long long *>(&claim[adj[j]]), (unsigned long long)want);
            }
        }
        __threadfence();  // the claims are complete before any is counted
        __syncthreads();
        // 2. claimed neighbours and the next frontier: its size is known
        // before any entry is written when the frontier is one chunk, and the
        // next frontier stays in LDS if it fits; otherwise it goes to the
        // global buffer the current frontier does not use
        int32_t *lds_next = front == s_front[0] ? s_front[1] : s_front[0];
        int32_t *glb_next = front == ga ? gb : ga;
        int32_t *nf = glb_next;
        int64_t cap = n;
        int64_t total = 0;  // the next frontier's size
        for (int64_t base = 0; base < m; base += kOneBS) {
            const int64_t p = base + tid;
            const bool valid = p < m;
            int64_t cnt = 0;
            int32_t v = 0;
            int64_t j0 = 0, j1 = 0;
            uint32_t mine = 0;  // which of the first 32 neighbours this entry claimed
            const uint64_t want = tag | uint64_t(p);
            if (valid) {
                v = front[p];
                j0 = ptr[v];
                j1 = ptr[v + 1];
                for (int64_t j = j0; j < j1; ++j)
                    if (load_claim(&claim[adj[j]]) == want) {
                        ++cnt;
                        if (j - j0 < 32) mine |= 1u << (j - j0);
                    }
            }
            int64_t chunk_total;
            const int64_t o0 = total + wg_scan_incl<ScanOp::Sum>(cnt, s_w, &chunk_total) - cnt;
            total += chunk_total;
            if (m <= kOneBS && total <= kFrontLds) {  // the same for every thread
                nf = lds_next;
                cap = kFrontLds;
            }
            if (valid) {
                int64_t o = o0;
                for (int64_t j = j0; j < j1; ++j) {
                    const int32_t u = adj[j];
                    if (j - j0 < 32 ? ((mine >> (j - j0)) & 1u) != 0 : load_claim(&claim[u]) == want) {
                        if (o < cap)
                            nf[o] = u;
                        else
                            *bad = 1;
                        ++o;
                    }
                }
            }
        }
        // the component counts, once every placement of the level has read them
        __syncthreads();
        int64_t carry2 = -1;
        for (int64_t base = 0; base < m; base += kOneBS) {
            const int64_t p = base + tid;
            const bool valid = p < m;
            const int32_t c = valid ? comp[front[p]] : -1;
            const bool head = valid && (p == 0 || comp[front[p - 1]] != c);
            int64_t chunk_max;
            int64_t first = wg_scan_incl<ScanOp::Max>(head ? p : -1, s_w, &chunk_max);
            if (first < 0) first = carry2;
            carry2 = chunk_max >= 0 ? chunk_max : carry2;
            if (valid && (p + 1 == m || comp[front[p + 1]] != c))
                __hip_atomic_fetch_add(&done[c], p - first + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();  // a frontier in global memory, and the counts, are complete
        __syncthreads();
        if (nf == glb_next) __threadfence();  // and no stale copy of it stays in this CU's cache
        placed += m;
        front = nf;
        m = total <= cap ? total : 0;
    }
    if (tid == 0) *placed_out = placed;
}

// ---- relabelling -----------------------------------------------------------
__global__ void k_inverse(const int32_t *__restrict__ new2old, int32_t *old2new, int32_t n, int32_t *bad) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= n) return;
    const int32_t v = new2old[k];
    if (v < 0 || v >= n || atomicCAS(&old2new[v], -1, k) != -1) *bad = 1;
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (i < n) a[i] = v;
}

// per new row: fixed flag, colour, and the smoothing degree (0 when fixed)
__global__ void k_row_meta(const int32_t *__restrict__ new2old, const uint8_t *__restrict__ fixed0,
                           const int32_t *__restrict__ color0, const int64_t *__restrict__ ptr0, uint8_t *fx,
                           int32_t *color, int64_t *deg, int32_t n) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= n) return;
    const int32_t v = new2old[k];
    fx[k] = fixed0[v];
    color[k] = color0[v];
    deg[k] = fixed0[v] ? 0 : ptr0[v + 1] - ptr0[v];
}

// row k of the smoothing adjacency: its input neighbours mapped to new
// labels, ascending
__global__ void k_row_fill(const int32_t *__restrict__ new2old, const int32_t *__restrict__ old2new,
                           const int64_t *__restrict__ ptr0, const int32_t *__restrict__ adj0,
                           const int64_t *__restrict__ row64, int32_t *col, int32_t n) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= n) return;
    const int64_t b = row64[k], m = row64[k + 1] - b;
    if (m == 0) return;
    const int32_t v = new2old[k];
    for (int64_t j = 0; j < m; ++j) col[b + j] = old2new[adj0[ptr0[v] + j]];
    seg_sort(col + b, m);
}

__global__ void k_row_ptr32(const int64_t *__restrict__ row64, int32_t *row_ptr, int32_t n) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k <= n) row_ptr[k] = int32_t(row64[k]);
}

// padded row-major copy: entry j of row k at ell[k*W + j], -1 past the row
__global__ void k_ell(const int64_t *__restrict__ row64, const int32_t *__restrict__ col, int32_t *ell, int32_t n,
                      int32_t W) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= n) return;
    const int64_t b = row64[k], m = row64[k + 1] - b;
    for (int32_t j = 0; j < W; ++j) ell[int64_t(k) * W + j] = j < m ? col[b + j] : -1;
}

// triangles: key = smallest new corner; bucket counts
__global__ void k_tri_key(const int32_t *__restrict__ tri0, const int32_t *__restrict__ old2new, int64_t T,
                          int32_t *key, int64_t *bucket) {
    const int64_t t = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (t >= T) return;
    const int32_t a = old2new[tri0[3 * t]], b = old2new[tri0[3 * t + 1]], c = old2new[tri0[3 * t + 2]];
    const int32_t k = min(a, min(b, c));
    key[t] = k;
    atomicAdd(reinterpret_cast<unsigned long long *>(&bucket[k]), 1ull);
}

// scatter into the key's bucket (any order), then sort each bucket by input
// index: the counting sort's stable order
__global__ void k_tri_scatter(const int32_t *__restrict__ key, int64_t T, const int64_t *__restrict__ start,
                              int64_t *cursor, int64_t *torder) {
    const int64_t t = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (t >= T) return;
    const int32_t k = key[t];
    const int64_t at = start[k] + int64_t(atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[k]), 1ull));
    torder[at] = t;
}

__global__ void k_seg_sort_i64(const int64_t *__restrict__ start, int64_t *a, int32_t nseg) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= nseg) return;
    seg_sort(a + start[k], start[k + 1] - start[k]);
}

__global__ void k_seg_sort_i32(const int64_t *__restrict__ start, int32_t *a, int32_t nseg) {
    const int32_t k = int32_t(blockIdx.x) * kBS + int32_t(threadIdx.x);
    if (k >= nseg) return;
    seg_sort(a + start[k], start[k + 1] - start[k]);
}

// triangle i of the sorted order: corners, weight (the host's operation
// order), mesh index, packed record
__global__ void k_tri_gather(const int64_t *__restrict__ torder, const int32_t *__restrict__ tri0,
                             const int32_t *__restrict__ old2new, const int32_t *__restrict__ tcount0,
                             const int64_t *__restrict__ t_off, int32_t n_mesh, int64_t T, int32_t *ta, int32_t *tb,
                             int32_t *tc, double *tw, int32_t *tmesh, int32_t *trec) {
    const int64_t i = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (i >= T) return;
    const int64_t t = torder[i];
    const int32_t a = tri0[3 * t], b = tri0[3 * t + 1], c = tri0[3 * t + 2];
    ta[i] = old2new[a];
    tb[i] = old2new[b];
    tc[i] = old2new[c];
    tw[i] = 1.0 / double(tcount0[a]) + 1.0 / double(tcount0[b]) + 1.0 / double(tcount0[c]);
    int32_t lo = 0, hi = n_mesh;  // mesh m owns triangles [t_off[m], t_off[m+1])
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) / 2;
        if (t_off[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    tmesh[i] = lo;
    if (trec) {
        trec[4 * i] = ta[i];
        trec[4 * i + 1] = tb[i];
        trec[4 * i + 2] = tc[i];
        trec[4 * i + 3] = tcount0[a] | (tcount0[b] << 10) | (tcount0[c] << 20);
    }
}

__global__ void k_vt_count(const int32_t *__restrict__ ta, const int32_t *__restrict__ tb,
                           const int32_t *__restrict__ tc, int64_t T, int64_t *cnt) {
    const int64_t i = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (i >= T) return;
    atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[ta[i]]), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[tb[i]]), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long *>(&cnt[tc[i]]), 1ull);
}

__global__ void k_vt_scatter(const int32_t *__restrict__ ta, const int32_t *__restrict__ tb,
                             const int32_t *__restrict__ tc, int64_t T, const int64_t *__restrict__ start,
                             int64_t *cursor, int32_t *vt) {
    const int64_t i = int64_t(blockIdx.x) * kBS + threadIdx.x;
    if (i >= T) return;
    const int32_t c3[3] = {ta[i], tb[i], tc[i]};
    for (int q = 0; q < 3; ++q) {
        const int32_t v = c3[q];
        vt[start[v] + int64_t(atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[v]), 1ull))] = int32_t(i);
    }
}

// ---- buffers ---------------------------------------------------------------
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    void alloc(size_t count) {
        RHIP_CHECK(hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T)));
        n = count;
    }
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    void up(const std::vector<T> &v, hipStream_t s) {
        if (!v.empty()) RHIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void down(std::vector<T> &v, size_t count, hipStream_t s) const {
        v.resize(count);
        if (count) RHIP_CHECK(hipMemcpyAsync(v.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

}  // namespace

// Input-label arrays of the handle on the device, uploaded on the first
// device reorder and kept (they never change after the build).
struct ReorderState {
    int device = -1;
    DBuf<int64_t> ptr0, t_off;
    DBuf<int32_t> adj0, tri0, color0, tcount0;
    DBuf<uint8_t> fixed0;
};

void destroy_reorder_state(ReorderState *r) {
    if (!r) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (r->device >= 0) (void)hipSetDevice(r->device);
    delete r;
    if (cur >= 0) (void)hipSetDevice(cur);
}

namespace {

ReorderState &ensure_reorder_state(Mesh &M, hipStream_t s) {
    int dev = 0;
    RHIP_CHECK(hipGetDevice(&dev));
    if (M.rdev && M.rdev->device != dev) fail(LMS_ERR_STATE, "handle's device reorder state lives on another device");
    if (!M.rdev) {
        std::unique_ptr<ReorderState, ReorderDeleter> r(new ReorderState());
        r->device = dev;
        r->ptr0.alloc(M.adj_ptr0.size());
        r->ptr0.up(M.adj_ptr0, s);
        r->adj0.alloc(M.adj0.size());
        r->adj0.up(M.adj0, s);
        r->tri0.alloc(M.tri0.size());
        r->tri0.up(M.tri0, s);
        r->color0.alloc(M.color0.size());
        r->color0.up(M.color0, s);
        r->tcount0.alloc(M.tcount0.size());
        r->tcount0.up(M.tcount0, s);
        r->fixed0.alloc(M.fixed0.size());
        r->fixed0.up(M.fixed0, s);
        r->t_off.alloc(M.t_off.size());
        r->t_off.up(M.t_off, s);
        RHIP_CHECK(hipStreamSynchronize(s));
        M.rdev = std::move(r);
    }
    return *M.rdev;
}

// Breadth-first order of the whole handle on the device (new2old).
void bfs_device(Mesh &M, ReorderState &R, hipStream_t s, DBuf<int32_t> &order) {
    const int32_t n = M.n;
    DBuf<int32_t> comp(static_cast<size_t>(n)), changed(1);
    k_cc_init<<<blocks_for(n), kBS, 0, s>>>(comp.p, n);
    rlaunch_check();
    for (int it = 0;; ++it) {
        if (it > n + 2) fail(LMS_ERR_STATE, "components did not converge");  // each round merges two trees
        RHIP_CHECK(hipMemsetAsync(changed.p, 0, sizeof(int32_t), s));
        k_cc_hook<<<blocks_for(n), kBS, 0, s>>>(R.ptr0.p, R.adj0.p, comp.p, n, changed.p);
        k_cc_shortcut<<<blocks_for(n), kBS, 0, s>>>(comp.p, n, changed.p);
        rlaunch_check();
        int32_t h = 0;
        RHIP_CHECK(hipMemcpyAsync(&h, changed.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        RHIP_CHECK(hipStreamSynchronize(s));
        if (!h) break;
    }
    // roots (component minima) in ascending label and component start offsets
    DBuf<int64_t> flag(static_cast<size_t>(n)), rank(static_cast<size_t>(n) + 1), size_at(static_cast<size_t>(n)), comp_start(static_cast<size_t>(n) + 1);
    RHIP_CHECK(hipMemsetAsync(size_at.p, 0, sizeof(int64_t) * size_t(n), s));
    k_root_flags<<<blocks_for(n), kBS, 0, s>>>(comp.p, flag.p, size_at.p, n);
    rlaunch_check();
    scan(flag.p, rank.p, n, s);
    scan(size_at.p, comp_start.p, n, s);
    int64_t roots = 0;
    RHIP_CHECK(hipMemcpyAsync(&roots, rank.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RHIP_CHECK(hipStreamSynchronize(s));
    DBuf<int32_t> fa(static_cast<size_t>(n)), fb(static_cast<size_t>(n));
    DBuf<uint64_t> claim(static_cast<size_t>(n));
    DBuf<int64_t> done(static_cast<size_t>(n)), placed_d(1);
    k_seed<<<blocks_for(n), kBS, 0, s>>>(comp.p, rank.p, fa.p, claim.p, n);
    rlaunch_check();
    RHIP_CHECK(hipMemsetAsync(done.p, 0, sizeof(int64_t) * size_t(n), s));
    RHIP_CHECK(hipMemsetAsync(changed.p, 0, sizeof(int32_t), s));  // reused as the placement check
    RHIP_CHECK(hipMemsetAsync(placed_d.p, 0, sizeof(int64_t), s));
    k_bfs_one_group<<<1, kOneBS, 0, s>>>(R.ptr0.p, R.adj0.p, comp.p, comp_start.p, done.p, claim.p, fa.p, fb.p,
                                         roots, order.p, n, changed.p, placed_d.p);
    rlaunch_check();
    int64_t placed = 0;
    int32_t hbad = 0;
    RHIP_CHECK(hipMemcpyAsync(&placed, placed_d.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RHIP_CHECK(hipMemcpyAsync(&hbad, changed.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RHIP_CHECK(hipStreamSynchronize(s));
    if (placed != n || hbad) fail(LMS_ERR_STATE, "breadth-first search misplaced vertices");
}

}  // namespace

// Reorder with the breadth-first search (kind LMS_BFS, new2old ignored) or
// the given order on the device, relabel there, and adopt the results; the
// host arrays come out as relabel() makes them.
void dev_reorder(Mesh &M, lms_ordering kind, const std::vector<int32_t> &given, void *stream,
                 std::vector<int32_t> &new2old_out) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n = M.n;
    const int64_t T = M.T;
    ReorderState &R = ensure_reorder_state(M, s);
    DBuf<int32_t> n2o(static_cast<size_t>(n));
    if (kind == LMS_BFS) {
        bfs_device(M, R, s, n2o);
    } else {
        if (given.size() != size_t(n)) fail(LMS_ERR_ARG, "ordering has the wrong length");
        n2o.up(given, s);
    }
    // inverse and permutation check
    DBuf<int32_t> o2n(static_cast<size_t>(n)), bad(1);
    k_fill_i32<<<blocks_for(n), kBS, 0, s>>>(o2n.p, n, -1);
    RHIP_CHECK(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    k_inverse<<<blocks_for(n), kBS, 0, s>>>(n2o.p, o2n.p, n, bad.p);
    rlaunch_check();
    int32_t hbad = 0;
    RHIP_CHECK(hipMemcpyAsync(&hbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RHIP_CHECK(hipStreamSynchronize(s));
    if (hbad) fail(LMS_ERR_ARG, "ordering is not a permutation");
    // smoothing adjacency
    DBuf<uint8_t> fx(static_cast<size_t>(n));
    DBuf<int32_t> color(static_cast<size_t>(n)), row_ptr(static_cast<size_t>(n) + 1);
    DBuf<int64_t> deg(static_cast<size_t>(n)), row64(static_cast<size_t>(n) + 1);
    k_row_meta<<<blocks_for(n), kBS, 0, s>>>(n2o.p, R.fixed0.p, R.color0.p, R.ptr0.p, fx.p, color.p, deg.p, n);
    rlaunch_check();
    scan(deg.p, row64.p, n, s);
    int64_t nnz = 0;
    RHIP_CHECK(hipMemcpyAsync(&nnz, row64.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RHIP_CHECK(hipStreamSynchronize(s));
    if (nnz >= (int64_t(1) << 31)) fail(LMS_ERR_STATE, "adjacency exceeds 2^31 entries");
    DBuf<int32_t> col(static_cast<size_t>(nnz));
    k_row_fill<<<blocks_for(n), kBS, 0, s>>>(n2o.p, o2n.p, R.ptr0.p, R.adj0.p, row64.p, col.p, n);
    k_row_ptr32<<<blocks_for(int64_t(n) + 1), kBS, 0, s>>>(row64.p, row_ptr.p, n);
    rlaunch_check();
    int32_t ell_w = 0;
    DBuf<int32_t> ell;
    if (M.max_degree <= 16) {
        ell_w = M.max_degree <= 8 ? 8 : (M.max_degree <= 12 ? 12 : 16);
        ell.alloc(size_t(ell_w) * size_t(n));
        k_ell<<<blocks_for(n), kBS, 0, s>>>(row64.p, col.p, ell.p, n, ell_w);
        rlaunch_check();
    }
    // triangles: counting sort by smallest new corner, stable in input index
    DBuf<int32_t> key(static_cast<size_t>(T));
    DBuf<int64_t> bucket(static_cast<size_t>(n)), bstart(static_cast<size_t>(n) + 1), cursor(static_cast<size_t>(n)), torder(static_cast<size_t>(T));
    RHIP_CHECK(hipMemsetAsync(bucket.p, 0, sizeof(int64_t) * size_t(n), s));
    k_tri_key<<<blocks_for(T), kBS, 0, s>>>(R.tri0.p, o2n.p, T, key.p, bucket.p);
    rlaunch_check();
    scan(bucket.p, bstart.p, n, s);
    RHIP_CHECK(hipMemsetAsync(cursor.p, 0, sizeof(int64_t) * size_t(n), s));
    k_tri_scatter<<<blocks_for(T), kBS, 0, s>>>(key.p, T, bstart.p, cursor.p, torder.p);
    k_seg_sort_i64<<<blocks_for(n), kBS, 0, s>>>(bstart.p, torder.p, n);
    rlaunch_check();
    bool small = true;
    for (int32_t v = 0; v < n && small; ++v) small = M.tcount0[size_t(v)] <= 1023;
    DBuf<int32_t> ta(static_cast<size_t>(T)), tb(static_cast<size_t>(T)), tc(static_cast<size_t>(T)), tmesh(static_cast<size_t>(T)), trec;
    DBuf<double> tw(static_cast<size_t>(T));
    if (small) trec.alloc(size_t(4) * size_t(T));
    k_tri_gather<<<blocks_for(T), kBS, 0, s>>>(torder.p, R.tri0.p, o2n.p, R.tcount0.p, R.t_off.p, M.n_mesh, T, ta.p,
                                               tb.p, tc.p, tw.p, tmesh.p, small ? trec.p : nullptr);
    rlaunch_check();
    // vertex -> triangles, ascending triangle index per vertex
    DBuf<int64_t> vcnt(static_cast<size_t>(n)), vstart(static_cast<size_t>(n) + 1);
    DBuf<int32_t> vt(static_cast<size_t>(3) * size_t(T)), vt_ptr(static_cast<size_t>(n) + 1);
    RHIP_CHECK(hipMemsetAsync(vcnt.p, 0, sizeof(int64_t) * size_t(n), s));
    k_vt_count<<<blocks_for(T), kBS, 0, s>>>(ta.p, tb.p, tc.p, T, vcnt.p);
    rlaunch_check();
    scan(vcnt.p, vstart.p, n, s);
    RHIP_CHECK(hipMemsetAsync(cursor.p, 0, sizeof(int64_t) * size_t(n), s));
    k_vt_scatter<<<blocks_for(T), kBS, 0, s>>>(ta.p, tb.p, tc.p, T, vstart.p, cursor.p, vt.p);
    k_seg_sort_i32<<<blocks_for(n), kBS, 0, s>>>(vstart.p, vt.p, n);
    k_row_ptr32<<<blocks_for(int64_t(n) + 1), kBS, 0, s>>>(vstart.p, vt_ptr.p, n);
    rlaunch_check();

    // adopt
    std::vector<int32_t> h_n2o, h_o2n, h_row_ptr, h_col, h_ell, h_color, h_ta, h_tb, h_tc, h_trec, h_tmesh,
        h_vt_ptr, h_vt;
    std::vector<uint8_t> h_fx;
    std::vector<double> h_tw;
    n2o.down(h_n2o, size_t(n), s);
    o2n.down(h_o2n, size_t(n), s);
    row_ptr.down(h_row_ptr, size_t(n) + 1, s);
    col.down(h_col, size_t(nnz), s);
    if (ell_w > 0) ell.down(h_ell, size_t(ell_w) * size_t(n), s);
    fx.down(h_fx, size_t(n), s);
    color.down(h_color, size_t(n), s);
    ta.down(h_ta, size_t(T), s);
    tb.down(h_tb, size_t(T), s);
    tc.down(h_tc, size_t(T), s);
    tw.down(h_tw, size_t(T), s);
    tmesh.down(h_tmesh, size_t(T), s);
    if (small) trec.down(h_trec, size_t(4) * size_t(T), s);
    vt_ptr.down(h_vt_ptr, size_t(n) + 1, s);
    vt.down(h_vt, size_t(3) * size_t(T), s);
    RHIP_CHECK(hipStreamSynchronize(s));
    adopt_relabel(M, kind, std::move(h_n2o), std::move(h_o2n), std::move(h_row_ptr), std::move(h_col), ell_w,
                  std::move(h_ell), std::move(h_fx), std::move(h_color), std::move(h_ta), std::move(h_tb),
                  std::move(h_tc), std::move(h_tw), std::move(h_trec), std::move(h_tmesh), std::move(h_vt_ptr),
                  std::move(h_vt));
    new2old_out = M.new2old;
}

}  // namespace lms
