// Device side of the smoothing library for gfx950 (MI355X): the runtime
// around the kernels of lms_kernels.hpp (upload of the mesh arrays, scratch
// buffers, tile plans on the device, the autotuners, graph capture of the
// sweep loop, the device-side stopping rule).
//
// Compiled with -ffp-contract=off, like the kernels it includes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "lms_internal.hpp"
#include "lms_kernels.hpp"

// Scratch of lms_quality_noalloc (see dev_quality_noalloc below): 8192
// partial sums, 64 KiB on every GPU the library runs on.
constexpr int kScratchDoubles = 8192;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace lms {

#define HIP_CHECK(expr)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(e_ == hipErrorOutOfMemory ? LMS_ERR_ALLOC : LMS_ERR_HIP,                  \
                 std::string(#expr) + " failed: " + hipGetErrorString(e_));                \
    } while (0)

// ---------------------------------------------------------------------------
// Runtime

namespace {

constexpr int kQualBS = 256;
constexpr int kQualMaxBlocks = 8192;
constexpr int kChunk = 16;  // sweeps per captured chunk under the stopping rule (even)
constexpr size_t kMaxGraphs = 16;  // captured graphs cached per handle

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
        // patch plans: the working copies are stored patch by patch, position
        // p holding label pm_label[p] (halo and qc_ids then hold positions)
        int32_t *pm_label = nullptr;
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
        bool patches = false;
        int32_t k = 1;
        bool fits = false;
        int32_t *tile_ptr = nullptr, *halo = nullptr;
        int64_t *halo_ptr = nullptr, *upd_ptr = nullptr;
        uint16_t *urow = nullptr, *uidx = nullptr;
        uint8_t *umask = nullptr;
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
    int mc1_cfg[2] = {-1, -1};   // the fastest of one sweep per pass (the stopping rule runs it)
    float mc_us[2] = {-1.f, -1.f};  // mc_cfg's measured time per sweep (microseconds; -1 = not timed)
    int small_cfg[2] = {-2, -2}; // batch of small meshes: 1 = all sweeps in one launch, 0 = per sweep; -2 = not decided
    float small_us[2] = {-1.f, -1.f};  // measured one-launch time per sweep (microseconds)
    bool small_used[2] = {false, false};  // the last fixed-K Jacobi call ran the one-launch path
    int tbq_cfg[2] = {-2, -2};   // variant whose quality-fused form runs the stopping rule; -1 none; -2 not tuned
    float tbq_us[2] = {-1.f, -1.f};  // its measured time per sweep (microseconds)
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
    // x, y of the last fixed-K packed lms_smooth: a call on the same arrays
    // issues the pack and the unpack with the passes (in their graph, if any)
    const void *io_x = nullptr, *io_y = nullptr;
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
        d->mc1_cfg[0] = d->mc1_cfg[1] = -1;
        d->small_cfg[0] = d->small_cfg[1] = -2;
        d->small_us[0] = d->small_us[1] = -1.f;
        d->small_used[0] = d->small_used[1] = false;
        d->tbq_cfg[0] = d->tbq_cfg[1] = -2;
        d->tbq_us[0] = d->tbq_us[1] = -1.f;
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

// Patch-major order of a patch plan: tile t's own rows (in its list order)
// at positions tile_ptr[t] .. tile_ptr[t+1]-1, then the rows no tile owns
// (the fixed vertices) in ascending label.  label[p] is the label stored at
// position p, pos its inverse.
void patch_major(const Mesh &M, const Mesh::TBPlan &P, std::vector<int32_t> &label, std::vector<int32_t> &pos) {
    const int32_t n = M.n;
    label.assign(size_t(n), -1);
    pos.assign(size_t(n), -1);
    for (int32_t t = 0; t < P.tiles; ++t) {
        const int32_t nown = P.tile_ptr[size_t(t) + 1] - P.tile_ptr[size_t(t)];
        for (int32_t i = 0; i < nown; ++i) {
            const int32_t v = P.halo[size_t(P.halo_ptr[size_t(t)]) + size_t(i)];
            const int32_t p = P.tile_ptr[size_t(t)] + i;
            if (v < 0 || v >= n || p >= n || pos[size_t(v)] >= 0) fail(LMS_ERR_STATE, "patch plan: own rows");
            label[size_t(p)] = v;
            pos[size_t(v)] = p;
        }
    }
    int32_t next = P.tiles > 0 ? P.tile_ptr[size_t(P.tiles)] : 0;
    for (int32_t v = 0; v < n; ++v)
        if (pos[size_t(v)] < 0) {
            if (!M.fixed[size_t(v)]) fail(LMS_ERR_STATE, "patch plan: a free row no tile owns");
            label[size_t(next)] = v;
            pos[size_t(v)] = next++;
        }
    if (next != n) fail(LMS_ERR_STATE, "patch plan: positions");
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
    if (h.patches && P.fits) {
        std::vector<int32_t> label, pos;
        patch_major(M, P, label, pos);
        std::vector<int32_t> halo(P.halo.size());
        for (size_t j = 0; j < halo.size(); ++j) halo[j] = pos[size_t(P.halo[j])];
        h.halo = upload(&d, halo);
        h.pm_label = upload(&d, label);
    } else {
        h.halo = upload(&d, P.halo);
    }
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
    if (h->patches) {
        std::vector<int32_t> label, pos;
        patch_major(M, *P, label, pos);
        std::vector<int32_t> ids(P->qc_ids.size());
        for (size_t j = 0; j < ids.size(); ++j) ids[j] = pos[size_t(P->qc_ids[j])];
        h->qc_ids = upload(&d, ids);
    } else {
        h->qc_ids = upload(&d, P->qc_ids);
    }
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
                   hipStream_t s, bool qual = false, int32_t max_iters = 0, T *ox = nullptr, T *oy = nullptr) {
    const TBShape t = tb_shape(cfg);
    const DeviceState::TBDev *h = find_tb(d, t);
    if (!h || !h->fits || M.ell_w != t.w) fail(LMS_ERR_STATE, "temporally blocked variant launched without its plan");
    if (qual) {
        if (!h->q_ready || !h->q_fits) fail(LMS_ERR_STATE, "quality-fused pass without its triangle plan");
        k = t.k;
    }
    if (k < 1 || k > t.k) fail(LMS_ERR_STATE, "temporally blocked pass deeper than its plan");
    if ((ox == nullptr) != (oy == nullptr) || (qual && ox))
        fail(LMS_ERR_STATE, "temporally blocked pass: separate outputs need both arrays and no quality");
    if (h->u_max > t.bs * t.r || size_t(h->l_max) * sizeof(vec2_t<T>) > size_t(64) * 1024)
        fail(LMS_ERR_STATE, "temporally blocked plan does not fit the variant");
    if (h->patches && !h->pm_label) fail(LMS_ERR_STATE, "patch plan without its patch order");
    if (h->tiles == 0) return;
    const size_t lds = size_t(h->l_max) * sizeof(vec2_t<T>);
    switch (cfg) {
#define TB(id, bs, w, r, map, ts, kk, lcap, g)                                                                 \
    case id:                                                                                                   \
        if (qual)                                                                                              \
            k_jacobi_tb<T, bs, w, r, map, ts, kk, lcap, true, g != 0><<<h->tiles, bs, lds, s>>>(               \
                h->tile_ptr, h->ring, k, h->halo_ptr, h->halo, h->lidx_ptr, h->lidx, src, dst, nullptr,        \
                nullptr, h->pm_label, h->qtri_ptr, h->qtri, h->qpart, d.st, max_iters);                        \
        else                                                                                                   \
            k_jacobi_tb<T, bs, w, r, map, ts, kk, lcap, false, g != 0><<<h->tiles, bs, lds, s>>>(              \
                h->tile_ptr, h->ring, k, h->halo_ptr, h->halo, h->lidx_ptr, h->lidx, src, dst, ox, oy,         \
                h->pm_label, nullptr, nullptr, nullptr, nullptr, 0);                                           \
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
        // a patch variant keeps its copies in patch order, which this caller's do not follow
        if (tb_shape(cfg).g) fail(LMS_ERR_STATE, "patch variants run only in their own passes");
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

// One-pass multicolour variants: MC(id, block size, tile size, staging cap,
// updated rows per thread R, map, patches, sweeps per pass k).  A tile
// updates at most block size x R rows.  patches = 1: tiles are breadth-first
// patches of free rows, as for the temporally blocked sweep.  k > 1: a pass
// runs up to k multicolour sweeps in LDS.
#define LMS_MC_CONFIGS(MC)                  \
    MC(0, 256, 128, 1024, 2, 16, 0, 1)      \
    MC(1, 256, 128, 1024, 2, 0, 0, 1)       \
    MC(2, 256, 256, 2048, 4, 16, 0, 1)      \
    MC(3, 256, 64, 512, 1, 16, 0, 1)        \
    MC(4, 256, 256, 1024, 2, 16, 1, 1)      \
    MC(5, 256, 512, 2048, 4, 0, 1, 1)       \
    MC(6, 256, 512, 2048, 4, 16, 1, 1)      \
    MC(7, 256, 1024, 4096, 8, 0, 1, 1)      \
    MC(8, 512, 512, 2048, 2, 0, 1, 1)       \
    MC(9, 1024, 1024, 2048, 2, 0, 1, 1)     \
    MC(10, 1024, 2048, 4096, 4, 0, 1, 1)    \
    MC(11, 256, 512, 2048, 4, 0, 1, 2)      \
    MC(12, 256, 384, 2048, 4, 16, 1, 2)     \
    MC(13, 512, 1024, 4096, 4, 0, 1, 2)     \
    MC(14, 256, 256, 2048, 4, 16, 1, 3)
constexpr int kNumMcConfigs = 15;

struct MCShape {
    int bs = 0, ts = 0, lcap = 0, r = 0, map = 0, g = 0, k = 1;
};

MCShape mc_shape(int cfg) {
    switch (cfg) {
#define MC(id, bs, ts, lcap, r, map, g, k) \
    case id:                               \
        return MCShape{bs, ts, lcap, r, map, g, k};
        LMS_MC_CONFIGS(MC)
#undef MC
    }
    return MCShape{};
}

// Name of a multicolour variant as lms_sweep_config reports it.
std::string mc_config_name(int cfg) {
    if (cfg < 0) return "by-colour";
    const MCShape t = mc_shape(cfg);
    char buf[96];
    std::snprintf(buf, sizeof(buf), "mc/ts%d/k%d/bs%d/r%d/l%d/%s%s", t.ts, t.k, t.bs, t.r, t.lcap,
                  map_name(t.map).c_str(), t.g ? "/patch" : "");
    return buf;
}

// Whether a resident multicolour plan is the one of shape t.
template <class P>
bool mc_plan_is(const P &p, const MCShape &t) {
    return p.ts == t.ts && p.l_cap == t.lcap && p.u_cap == t.bs * t.r && p.patches == (t.g != 0) && p.k == t.k;
}

// Meshes from this many rows on drop, after each tuning, the tile plans that
// no tuned precision's chosen variants use (host and device): there each plan
// costs ~20-40 bytes per row, and the tuner builds a dozen.
constexpr int32_t kDropPlansFrom = 1 << 22;

void drop_unused_plans(DeviceState &d, Mesh &M) {
    std::vector<int> keep;
    for (int pi = 0; pi < 2; ++pi) {
        for (int c : {d.sweep_cfg[pi], d.smooth_cfg[pi], d.tb_cfg[pi], d.tb_best[pi], d.tbq_cfg[pi]})
            if (c >= 0) keep.push_back(c);
        // the three fastest temporally blocked variants stay candidates for
        // the quality-fused stopping rule
        std::vector<std::pair<float, int>> tb;
        for (int c = kFirstTBConfig; c < kNumAllConfigs; ++c)
            if (d.tune_us[pi][c] >= 0.f) tb.emplace_back(d.tune_us[pi][c], c);
        std::sort(tb.begin(), tb.end());
        for (size_t i = 0; i < tb.size() && i < 3; ++i) keep.push_back(tb[i].second);
    }
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
    auto keep_mc = [&](const auto &plan) {
        for (int pi = 0; pi < 2; ++pi)
            for (int c : {d.mc_cfg[pi], d.mc1_cfg[pi]})
                if (c >= 0 && mc_plan_is(plan, mc_shape(c))) return true;
        return false;
    };
    for (auto it = d.mcs.begin(); it != d.mcs.end();) {
        if (keep_mc(*it)) {
            ++it;
            continue;
        }
        for (const void *p : {static_cast<const void *>(it->tile_ptr), static_cast<const void *>(it->halo),
                              static_cast<const void *>(it->halo_ptr), static_cast<const void *>(it->upd_ptr),
                              static_cast<const void *>(it->urow), static_cast<const void *>(it->uidx),
                              static_cast<const void *>(it->umask),
                              static_cast<const void *>(it->qtri_ptr), static_cast<const void *>(it->qtri),
                              static_cast<const void *>(it->qpart), static_cast<const void *>(it->qpart2),
                              static_cast<const void *>(it->qc_ids), static_cast<const void *>(it->qc_w)})
            free_array(d, p);
        it = d.mcs.erase(it);
    }
    for (auto it = M.mc_plans.begin(); it != M.mc_plans.end();)
        it = keep_mc(*it) ? std::next(it) : M.mc_plans.erase(it);
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
// A fixed-K call whose launches each run at least this long is issued launch
// by launch: the host stays ahead of the device, and the end of a graph costs
// more (about 8 us per call, measured on the 708k-vertex mesh) than the
// launches it saves.
constexpr float kDirectLaunchUs = 10.f;

template <class F>
void run_maybe_graph(DeviceState &d, const std::string &key, hipStream_t s, F body, bool direct = false) {
    if (!d.use_graphs || direct) {
        body(s);
        launch_check();
        return;
    }
    for (size_t i = 0; i < d.graphs.size(); ++i)
        if (d.graphs[i].key == key) {
            // least recently used last out: a hit moves to the back
            if (i + 1 != d.graphs.size()) {
                GraphEntry g = d.graphs[i];
                d.graphs.erase(d.graphs.begin() + std::ptrdiff_t(i));
                d.graphs.push_back(g);
            }
            HIP_CHECK(hipGraphLaunch(d.graphs.back().exec, s));
            return;
        }
    GraphEntry g;
    g.key = key;
    HIP_CHECK(hipStreamBeginCapture(d.cap, hipStreamCaptureModeRelaxed));
    try {
        body(d.cap);
    } catch (...) {
        // end the capture whatever body threw, so the capture stream stays usable
        hipGraph_t partial = nullptr;
        (void)hipStreamEndCapture(d.cap, &partial);
        if (partial) (void)hipGraphDestroy(partial);
        (void)hipGetLastError();
        throw;
    }
    hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(d.cap, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (le != hipSuccess)
            fail(LMS_ERR_HIP, std::string("kernel launch failed during capture: ") + hipGetErrorString(le));
        fail(LMS_ERR_HIP, std::string("hipStreamEndCapture failed: ") + hipGetErrorString(ce));
    }
    g.graph = graph;
    hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(LMS_ERR_HIP, std::string("hipGraphInstantiate failed: ") + hipGetErrorString(ie));
    }
    if (d.graphs.size() >= kMaxGraphs) {
        // the evicted graph may still run: from an earlier call (last_done)
        // or from this call on s.  Wait for both before destroying it.
        hipError_t we = hipSuccess;
        if (d.last_valid) we = hipEventSynchronize(d.last_done);
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (we == hipSuccess) we = hipStreamIsCapturing(s, &cs);
        if (we == hipSuccess && cs == hipStreamCaptureStatusNone) we = hipStreamSynchronize(s);
        if (we != hipSuccess) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
            HIP_CHECK(we);
        }
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
// rule, or -1 (then sweep and quality pass run separately).  Once tuned
// (tune_fused_stop) the choice stands; before, the fastest plain variant.
template <typename T>
int fused_stop_cfg(DeviceState &d, Mesh &M) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (!env_flag("LMS_FUSED_QUALITY", true)) return -1;
    if (d.tbq_cfg[pi] != -2) return d.tbq_cfg[pi];
    const int c = d.tb_best[pi];
    if (c < 0) return -1;
    return ensure_tbq(d, M, tb_shape(c)) ? c : -1;
}

// Candidates timed for the quality-fused stopping rule.
constexpr size_t kFusedCandidates = 6;

// A quality-fused pass holds more registers than the plain one (triangle
// records, the float64 quality), so the fastest plain variant need not be
// the fastest fused one: time the fused form of the fastest temporally
// blocked variants whose plans are resident (a full pass from P_0 in the
// working copies, with the stop state cleared) and keep the fastest per
// sweep.  A variant forced with LMS_SWEEP_CONFIG, or LMS_AUTOTUNE=0, keeps
// the plain choice.
template <typename T>
void tune_fused_stop(DeviceState &d, Mesh &M, const T *x, const T *y, hipStream_t s) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (d.tbq_cfg[pi] != -2) return;
    d.tbq_cfg[pi] = -1;
    if (d.tb_best[pi] < 0 || !env_flag("LMS_FUSED_QUALITY", true)) return;
    std::vector<std::pair<float, int>> cand;
    const char *forced = std::getenv("LMS_SWEEP_CONFIG");
    if ((forced && *forced) || !env_flag("LMS_AUTOTUNE", true)) {
        cand.emplace_back(0.f, d.tb_best[pi]);
    } else {
        for (int c = kFirstTBConfig; c < kNumAllConfigs; ++c)
            if (d.tune_us[pi][c] >= 0.f && find_tb(d, tb_shape(c))) cand.emplace_back(d.tune_us[pi][c], c);
        std::sort(cand.begin(), cand.end());
        if (cand.size() > kFusedCandidates) cand.resize(kFusedCandidates);
    }
    if (cand.size() == 1) {
        d.tbq_cfg[pi] = ensure_tbq(d, M, tb_shape(cand[0].second)) ? cand[0].second : -1;
        return;
    }
    vec2_t<T> *A = ensure_packed<T>(d, 0, M.n);
    vec2_t<T> *B = ensure_packed<T>(d, 1, M.n);
    k_pack<T><<<(M.n + 255) / 256, 256, 0, s>>>(x, y, A, B, M.n);
    launch_check();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        HIP_CHECK(err);
    }
    const int reps = M.n > (1 << 22) ? 2 : 6;
    float best = 3.0e38f;
    for (const auto &[us, c] : cand) {
        if (err != hipSuccess) break;
        if (!ensure_tbq(d, M, tb_shape(c))) continue;
        const int kk = tb_shape(c).k;
        k_stop_reset<<<1, 64, 0, s>>>(d.st);
        launch_tb_cfg<T>(c, d, M, A, B, kk, s, true, 1 << 30);
        err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r) launch_tb_cfg<T>(c, d, M, A, B, kk, s, true, 1 << 30);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        const float per = ms * 1000.f / float(reps * kk);
        if (err == hipSuccess && per < best) {
            best = per;
            d.tbq_cfg[pi] = c;
            d.tbq_us[pi] = per;
        }
        if (env_flag("LMS_VERBOSE", false))
            std::fprintf(stderr, "[lms] quality-fused %-44s %9.2f us per sweep (plain %.2f)\n",
                         sweep_config_name(c).c_str(), double(per), double(us));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_CHECK(err);
    launch_check();
}

const DeviceState::MCDev &ensure_mc(DeviceState &d, Mesh &M, const MCShape &t) {
    for (const auto &h : d.mcs)
        if (mc_plan_is(h, t)) return h;
    const auto t0 = std::chrono::steady_clock::now();
    const Mesh::MCPlan &P = mc_plan(M, t.ts, t.lcap, t.bs * t.r, t.g != 0, t.k);
    if (env_flag("LMS_VERBOSE", false))
        std::fprintf(stderr, "[lms] multicolour plan %s ts=%d k=%d: %d tiles, %s, %.2f s\n",
                     t.g ? "patches" : "ranges", t.ts, t.k, P.tiles, P.fits ? "fits" : "does not fit",
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    DeviceState::MCDev h;
    h.ts = t.ts;
    h.l_cap = t.lcap;
    h.u_cap = t.bs * t.r;
    h.patches = t.g != 0;
    h.k = t.k;
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
        h.umask = upload(&d, P.umask);
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

// The plain and quality-fused kernels of one-pass multicolour variant cfg
// at padded width W, handed to go.
template <typename T, int W, class Go>
void mc_dispatch(int cfg, Go &&go) {
    switch (cfg) {
#define MC(id, bs, ts, lcap, r, map, g, k)                                                          \
    case id:                                                                                        \
        go(bs, k_colour_tiles<T, bs, W, r, map, false, g != 0, k>,                                  \
           k_colour_tiles<T, bs, W, r, map, true, g != 0, k>);                                      \
        break;
        LMS_MC_CONFIGS(MC)
#undef MC
        default:
            fail(LMS_ERR_STATE, "unknown one-pass multicolour variant");
    }
}

// One pass of variant cfg src -> dst: `depth` multicolour sweeps (the last
// `depth` of its plan; under the stopping rule, with qual, one).
template <typename T>
void launch_mc_cfg(int cfg, DeviceState &d, const Mesh &M, const vec2_t<T> *src, vec2_t<T> *dst,
                   const StopState *st, hipStream_t s, bool qual = false, int32_t max_iters = 0, int32_t depth = 1) {
    const MCShape t = mc_shape(cfg);
    const DeviceState::MCDev *h = nullptr;
    for (const auto &x : d.mcs)
        if (mc_plan_is(x, t)) h = &x;
    if (!h || !h->fits || h->colors != M.n_colors) fail(LMS_ERR_STATE, "one-pass multicolour variant without its plan");
    if (size_t(h->l_max) * sizeof(vec2_t<T>) > size_t(64) * 1024) fail(LMS_ERR_STATE, "multicolour plan too large");
    if (qual && (!h->q_ready || !h->q_fits || !st)) fail(LMS_ERR_STATE, "quality-fused multicolour pass without its plan");
    const size_t lds = size_t(h->l_max) * sizeof(vec2_t<T>);
    if (depth < 1 || depth > t.k) fail(LMS_ERR_STATE, "multicolour pass deeper than its plan");
    auto go = [&](int bs, auto plain, auto fused) {
        if (qual)
            fused<<<h->tiles, bs, lds, s>>>(h->tile_ptr, h->halo_ptr, h->halo, h->upd_ptr, h->urow, h->uidx,
                                            h->umask, h->colors, 1, src, dst, st, h->qtri_ptr, h->qtri, h->qpart,
                                            max_iters);
        else
            plain<<<h->tiles, bs, lds, s>>>(h->tile_ptr, h->halo_ptr, h->halo, h->upd_ptr, h->urow, h->uidx,
                                            h->umask, h->colors, depth, src, dst, st, nullptr, nullptr, nullptr, 0);
    };
    switch (M.ell_w) {
        case 8:
            mc_dispatch<T, 8>(cfg, go);
            break;
        case 12:
            mc_dispatch<T, 12>(cfg, go);
            break;
        case 16:
            mc_dispatch<T, 16>(cfg, go);
            break;
        default:
            fail(LMS_ERR_STATE, "no padded adjacency for the one-pass multicolour sweep");
    }
    launch_check();
}

// Choose, per precision, between the colour-by-colour sweep and the one-pass
// variants by timing one sweep of each (LMS_COLOUR_TILES=0 keeps colour by
// colour; LMS_COLOUR_CONFIG=<id> forces a one-pass variant).
template <typename T>
void tune_colour(DeviceState &d, Mesh &M, vec2_t<T> *A, vec2_t<T> *B, hipStream_t s) {
    const int pi = sizeof(T) == 8 ? 0 : 1;
    if (d.mc_cfg[pi] != -2) return;
    d.mc_cfg[pi] = d.mc1_cfg[pi] = -1;
    d.mc_us[pi] = -1.f;
    if (!env_flag("LMS_COLOUR_TILES", true) || M.ell_w == 0) return;
    if (const char *f = std::getenv("LMS_COLOUR_CONFIG")) {
        const int c = std::atoi(f);
        if (c < 0 || c >= kNumMcConfigs || !mc_usable<T>(d, M, c))
            fail(LMS_ERR_ARG, "LMS_COLOUR_CONFIG names a one-pass multicolour variant this mesh cannot use");
        d.mc_cfg[pi] = d.mc1_cfg[pi] = c;  // a deeper variant runs passes of depth 1 under the stopping rule
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
    float best = 3.0e38f, best1 = 3.0e38f;  // per sweep: every variant, and one sweep per pass
    hipError_t err = hipSuccess;
    // from 4M rows on, only patch variants are timed (as for the sweep tuner:
    // patches won wherever both were measured, and every plan costs memory)
    for (int c = -1; c < kNumMcConfigs && err == hipSuccess; ++c) {
        if (c >= 0 && M.n >= kDropPlansFrom && !mc_shape(c).g) continue;
        if (c >= 0 && !mc_usable<T>(d, M, c)) continue;
        const int kk = c < 0 ? 1 : mc_shape(c).k;  // sweeps per timed pass
        auto one = [&]() {
            if (c < 0)
                launch_colour_sweep2<T>(d, M, A, nullptr, s);
            else
                launch_mc_cfg<T>(c, d, M, A, B, nullptr, s, false, 0, kk);
        };
        one();
        err = hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) one();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ms /= float(kk);
        if (err == hipSuccess && ms < best) {
            best = ms;
            d.mc_cfg[pi] = c;
            d.mc_us[pi] = ms * 1000.f / float(reps);
        }
        if (err == hipSuccess && kk == 1 && ms < best1) {
            best1 = ms;
            d.mc1_cfg[pi] = c;
        }
        if (env_flag("LMS_VERBOSE", false))
            std::fprintf(stderr, "[lms] multicolour %s: %.2f us per sweep\n",
                         c < 0 ? "colour by colour"
                               : ("one pass, variant " + std::to_string(c) + " (" + std::to_string(kk) +
                                  " sweeps per pass)").c_str(),
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
        if (mc_plan_is(x, t)) h = &x;
    if (!h || !h->fits) fail(LMS_ERR_STATE, "quality-fused multicolour pass without its tile plan");
    if (h->q_ready) return h->q_fits;
    Mesh::MCPlan *P = nullptr;
    for (auto &p : M.mc_plans)
        if (mc_plan_is(p, t) && p.version == M.version) P = &p;
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
    // >= 0: multicolour in one-pass sweeps, A/B ping-pong (under the stopping
    // rule the fastest of one sweep per pass)
    const int mc = colour ? (o.check_quality ? d.mc1_cfg[pi] : d.mc_cfg[pi]) : -1;
    const int mck = mc >= 0 ? mc_shape(mc).k : 1;  // sweeps per pass for fixed K
    const bool in_place = colour && mc < 0;
    const int nb = (M.n + 255) / 256;
    const int small_rows = colour || o.check_quality ? 0 : small;
    // A fixed-K call on the same x, y as the previous one issues the pack (and
    // the unpack, where one is needed) with the passes, in one graph keyed by
    // x and y (or launch by launch when the launches are long), which removes
    // the gaps around them; other calls pack and unpack around the passes, so
    // arrays that change from call to call capture no new graph.
    const bool fixed_k = !o.check_quality && o.max_iters > 0 && small_rows == 0;
    const bool io_in_graph = fixed_k && d.io_x == x && d.io_y == y;
    if (fixed_k) {
        d.io_x = x;
        d.io_y = y;
    }
    // the variant whose passes run this call, when they are temporally
    // blocked: a patch variant keeps the working copies in its patch order
    const int fq = !colour && o.check_quality && small_rows == 0 ? fused_stop_cfg<T>(d, M) : -1;
    const int layout_cfg = small_rows > 0 ? -1 : tb >= 0 ? tb : fq;
    const int32_t *pm = nullptr;
    if (layout_cfg >= 0 && tb_shape(layout_cfg).g) {
        const DeviceState::TBDev *lh = find_tb(d, tb_shape(layout_cfg));
        if (!lh || !lh->pm_label) fail(LMS_ERR_STATE, "patch variant without its patch order");
        pm = lh->pm_label;
    }
    auto pack = [&](hipStream_t cs) {
        if (pm)
            k_pack_pm<T><<<nb, 256, 0, cs>>>(x, y, pm, A, in_place ? nullptr : B, M.n);
        else
            k_pack<T><<<nb, 256, 0, cs>>>(x, y, A, in_place ? nullptr : B, M.n);
    };
    auto unpack = [&](const vec2_t<T> *src, hipStream_t cs) {
        if (pm)
            k_unpack_pm<T><<<nb, 256, 0, cs>>>(src, pm, x, y, M.n);
        else
            k_unpack<T><<<nb, 256, 0, cs>>>(src, x, y, M.n);
    };
    if (!io_in_graph) {
        pack(s);
        launch_check();
    }
    const std::string base = std::string("packed|") + (p == LMS_FP64 ? "f64" : "f32") + "|" + ptr_key(A) + "|" +
                             ptr_key(B) + "|cfg" + std::to_string(cfg) + "|mc" + std::to_string(mc) + "|" +
                             std::to_string(int(sch)) +
                             (io_in_graph ? "|io|" + ptr_key(x) + "|" + ptr_key(y) : std::string());
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
    bool in_b = false;        // the result sits in B
    bool xy_written = false;  // the last pass wrote the result to x, y
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
        const bool direct = d.tune_us[pi][tb] * float(depth) >= kDirectLaunchUs;
        // the last pass writes the result to x, y itself when no graph keeps
        // x, y beyond this call under a key that does not name them
        const bool to_xy = io_in_graph || direct || !d.use_graphs;
        if (K > 0)
            run_maybe_graph(d, "tb|" + base + "|tb" + std::to_string(tb) + "|" + std::to_string(K), s,
                            [&](hipStream_t cs) {
                                if (io_in_graph) pack(cs);
                                int32_t left = K;
                                for (int32_t q = 0; q < passes; ++q) {
                                    const int32_t kk = std::min(left, depth);
                                    const bool last = to_xy && q == passes - 1;
                                    launch_tb_cfg<T>(tb, d, M, q % 2 == 0 ? A : B, q % 2 == 0 ? B : A, kk, cs, false,
                                                     0, last ? x : nullptr, last ? y : nullptr);
                                    left -= kk;
                                }
                            },
                            direct);
        iters = K;
        in_b = passes % 2 == 1;
        xy_written = K > 0 && to_xy;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (!o.check_quality && mck > 1) {
        // multicolour, passes of up to mck sweeps, ping-pong A/B
        const int32_t K = o.max_iters;
        const int32_t passes = (K + mck - 1) / mck;
        const bool direct = d.mc_us[pi] * float(mck) >= kDirectLaunchUs;
        if (K > 0)
            run_maybe_graph(d, "mcp|" + base + "|" + std::to_string(K), s, [&](hipStream_t cs) {
                if (io_in_graph) pack(cs);
                int32_t left = K;
                for (int32_t q = 0; q < passes; ++q) {
                    const int32_t kk = std::min(left, mck);
                    launch_mc_cfg<T>(mc, d, M, q % 2 == 0 ? A : B, q % 2 == 0 ? B : A, nullptr, cs, false, 0, kk);
                    left -= kk;
                }
                if (io_in_graph) unpack(passes % 2 == 1 ? B : A, cs);
            }, direct);
        iters = K;
        in_b = passes % 2 == 1;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (!o.check_quality) {
        const int32_t K = o.max_iters;
        // one launch per sweep (colour by colour: one per colour, kept in a graph)
        const bool direct = colour ? mc >= 0 && d.mc_us[pi] >= kDirectLaunchUs
                                   : cfg >= 0 && d.tune_us[pi][cfg] >= kDirectLaunchUs;
        if (K > 0)
            run_maybe_graph(d, "fixed|" + base + "|" + std::to_string(K), s, [&](hipStream_t cs) {
                if (io_in_graph) pack(cs);
                for (int32_t k = 0; k < K; ++k) sweep_once(k % 2 == 0 ? A : B, k % 2 == 0 ? B : A, nullptr, cs);
                if (io_in_graph) unpack(!in_place && K % 2 == 1 ? B : A, cs);
            }, direct);
        iters = K;
        in_b = !in_place && K % 2 == 1;
        r.stopped_by = LMS_STOP_MAX_ITERS;
        r.q0 = r.q_final = r.last_dq = std::numeric_limits<double>::quiet_NaN();
    } else if (fq >= 0) {
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
            if (mc_plan_is(xh, t)) h = &xh;
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
    if (!io_in_graph && !xy_written) {
        unpack(in_b ? B : A, s);
        launch_check();
    }
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
        if (o.check_quality) tune_fused_stop<T>(d, M, x, y, s);
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
    std::string out;
    if (M.dev->small_used[pi]) out = "small/r" + std::to_string(small_batch_rows(M)) + "/one-launch";
    auto add = [&out](const std::string &w) { out += (out.empty() ? "" : " ") + w; };
    // then the variant a fixed-K Jacobi lms_smooth runs, then the one it runs
    // under the stopping rule
    if (c >= 0) {
        if (M.dev->tb_cfg[pi] >= 0) add(sweep_config_name(M.dev->tb_cfg[pi]));
        add(sweep_config_name(c));
        if (M.dev->tbq_cfg[pi] >= 0) add("stop=" + sweep_config_name(M.dev->tbq_cfg[pi]));
    }
    // the multicolour variant of a fixed K, and the one of the stopping rule if another
    if (M.dev->mc_cfg[pi] != -2) {
        add("colour=" + mc_config_name(M.dev->mc_cfg[pi]));
        if (M.dev->mc1_cfg[pi] != M.dev->mc_cfg[pi]) add("colour_stop=" + mc_config_name(M.dev->mc1_cfg[pi]));
    }
    if (c < 0) return out;
    char buf[64];
    for (int i = 0; i < kNumAllConfigs; ++i) {
        std::snprintf(buf, sizeof(buf), "%s%d:%.2fus", i == 0 ? " tuned[" : " ", i, double(M.dev->tune_us[pi][i]));
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

// ---------------------------------------------------------------------------
// Allocation-free quality (lms_quality_noalloc)
//
// The per-block partial sums of the quality pass live in `scratch`, a
// file-scope array of which every GPU holds its own copy from the library's
// load until the process ends.  In host code the array's name only stands for
// the symbol: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch.  Calls on
// one GPU share the array (and keep its last contents), so calls that overlap
// on one GPU race.  Nothing needs clearing: a pass writes every partial the
// reduction after it reads.

namespace {

static_assert(kScratchDoubles >= kQualMaxBlocks, "the scratch array holds every partial sum");

std::mutex g_scratch_mu;
std::vector<double *> g_scratch;  // device address of `scratch`, per device (nullptr: not looked up)

double *scratch_on_current_device() {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch.size() <= size_t(dev)) g_scratch.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch[size_t(dev)]) {
        void *p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(LMS_ERR_HIP, "hipGetSymbolAddress returned no address for the quality scratch array");
        g_scratch[size_t(dev)] = static_cast<double *>(p);
    }
    return g_scratch[size_t(dev)];
}

}  // namespace

void dev_quality_noalloc(Mesh &M, const void *x, const void *y, lms_precision p, double *q_global_dev,
                         void *stream) {
    check_precision(p);
    if (!x || !y || !q_global_dev) fail(LMS_ERR_ARG, "null device pointer");
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    // the handle's device arrays must already be current: uploading them
    // would allocate
    if (!M.dev || M.dev->device != dev || M.dev->version != M.version)
        fail(LMS_ERR_STATE,
             "the handle's mesh arrays are not on the current device: make one device call on this handle "
             "(lms_quality, lms_permute, lms_sweep or lms_smooth) after the last reorder first");
    const int blocks = quality_blocks(M.T);
    if (blocks > kScratchDoubles)
        fail(LMS_ERR_ARG, "the quality pass needs " + std::to_string(blocks) + " partial sums; the scratch array holds " +
                              std::to_string(kScratchDoubles));
    double *part = scratch_on_current_device();
    DeviceState &d = *M.dev;
    hipStream_t s = as_stream(stream);
    begin_call(d, s);
    if (p == LMS_FP64) {
        const double *xd = static_cast<const double *>(x), *yd = static_cast<const double *>(y);
        if (d.trec)
            k_quality<double, kQualBS><<<blocks, kQualBS, 0, s>>>(d.trec, xd, yd, nullptr, M.T, part, nullptr, nullptr);
        else
            k_quality_wide<double, kQualBS><<<blocks, kQualBS, 0, s>>>(d.ta, d.tb, d.tc, d.tw, xd, yd, nullptr, M.T,
                                                                      part, nullptr, nullptr);
    } else {
        const float *xf = static_cast<const float *>(x), *yf = static_cast<const float *>(y);
        if (d.trec)
            k_quality<float, kQualBS><<<blocks, kQualBS, 0, s>>>(d.trec, xf, yf, nullptr, M.T, part, nullptr, nullptr);
        else
            k_quality_wide<float, kQualBS><<<blocks, kQualBS, 0, s>>>(d.ta, d.tb, d.tc, d.tw, xf, yf, nullptr, M.T,
                                                                     part, nullptr, nullptr);
    }
    launch_check();
    k_reduce_out<<<1, 256, 0, s>>>(part, blocks, 1.0 / double(M.n), q_global_dev);
    launch_check();
    end_call(d, s);
}

}  // namespace lms
