// Host runtime of the transport library: grid upload and set-up, job
// registration, batched persistent launches, tally read-back.  Implements the
// C ABI declared in include/colt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "colt.h"
#include "colt_internal.h"
#include "colt_launch.h"

using namespace colt;

namespace {

thread_local std::string g_error;
thread_local hipEvent_t g_t0 = nullptr, g_t1 = nullptr;
thread_local bool g_timed = false;

colt_status fail(colt_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(COLT_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Octree neighbour links: for every leaf and face (2 axis + (step > 0)), the
// node across that face at the leaf's own level, or the coarser leaf that
// covers it there.  A leaf across (same level or coarser) is stored as its leaf
// index with how many levels coarser it is, kRopeLeaf | (up << 27) | leaf, so
// a crossing reads no node table; a refined node across (its children are
// finer than the leaf) is stored as the node, which the crossing descends.
// kRopeEdge marks the domain face and kRopeSearch a case the encoding cannot
// hold (the transport then searches from the root).  Built with exact integer
// coordinates in units of the finest cell.
constexpr uint32_t kRopeEdge = 0xFFFFFFFFu, kRopeSearch = 0xFFFFFFFEu, kRopeLeaf = 0x80000000u;

// child: the device node table (a leaf holds -(leaf index + 1)).
void build_ropes(const int32_t *child, int64_t nn, const std::vector<int32_t> &depth,
                 const std::vector<int64_t> &order, const std::vector<int64_t> &leaf_src,
                 std::vector<uint32_t> &rope)
{
    int dmax = 0;
    for (int64_t i = 0; i < nn; ++i) dmax = std::max(dmax, depth[i]);
    std::vector<int64_t> lo((size_t)nn * 3, 0);
    for (int64_t i : order) {                 // parents before children
        const int32_t c = child[i];
        if (c < 0) continue;
        const int64_t half = int64_t(1) << (dmax - depth[i] - 1);
        for (int o = 0; o < 8; ++o)
            for (int d = 0; d < 3; ++d)
                lo[(size_t)(c + o) * 3 + d] = lo[(size_t)i * 3 + d] + (((o >> d) & 1) ? half : 0);
    }
    const int64_t extent = int64_t(1) << dmax;
    const int64_t nl = (int64_t)leaf_src.size();
    rope.assign((size_t)nl * 6, kRopeSearch);
    auto work = [&](int64_t j0, int64_t j1) {
        for (int64_t j = j0; j < j1; ++j) {
            const int64_t leaf = leaf_src[j];
            const int dl = depth[leaf];
            const int64_t size = int64_t(1) << (dmax - dl);
            for (int face = 0; face < 6; ++face) {
                const int a = face >> 1;
                int64_t q[3] = {lo[leaf * 3], lo[leaf * 3 + 1], lo[leaf * 3 + 2]};
                q[a] = (face & 1) ? q[a] + size : q[a] - 1;      // first unit across
                if (q[a] < 0 || q[a] >= extent) {
                    rope[(size_t)j * 6 + face] = kRopeEdge;
                    continue;
                }
                int64_t node = 0;
                int lvl = 0;
                int64_t nlo[3] = {0, 0, 0};
                while (child[node] >= 0 && lvl < dl) {
                    const int64_t half = int64_t(1) << (dmax - lvl - 1);
                    int oct = 0;
                    for (int d = 0; d < 3; ++d)
                        if (q[d] - nlo[d] >= half) { oct |= 1 << d; nlo[d] += half; }
                    node = child[node] + oct;
                    ++lvl;
                }
                const int up = dl - lvl;
                if (child[node] < 0) {
                    // up <= 14 keeps clear of the two marker values
                    const int64_t lf = -(int64_t)child[node] - 1;
                    if (lf < (int64_t(1) << 27) && up <= 14)
                        rope[(size_t)j * 6 + face] = kRopeLeaf | ((uint32_t)up << 27) | (uint32_t)lf;
                } else if (node < (int64_t(1) << 27) && up == 0) {
                    rope[(size_t)j * 6 + face] = (uint32_t)node;
                }
            }
        }
    };
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(16, std::thread::hardware_concurrency()));
    if (nl < 4096 || nt == 1) {
        work(0, nl);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t)
        th.emplace_back(work, nl * t / nt, nl * (t + 1) / nt);
    for (auto &x : th) x.join();
}

// Breadth-first walk of a caller's octree: every node reached exactly once
// from the root, child indices in range, depth per node and the walk order.
colt_status octree_walk(const int32_t *child, int64_t nn, std::vector<int32_t> &depth,
                        std::vector<int64_t> &order)
{
    depth.assign(nn, -1);
    order.clear();
    order.reserve(nn);
    depth[0] = 0;
    order.push_back(0);
    for (size_t h = 0; h < order.size(); ++h) {
        const int64_t i = order[h];
        const int32_t c = child[i];
        if (c < 0) continue;
        if ((int64_t)c + 7 >= nn || c <= 0)
            return fail(COLT_ERR_ARG, "node %lld has child index %d out of range",
                        (long long)i, c);
        for (int o = 0; o < 8; ++o) {
            if (depth[c + o] >= 0) return fail(COLT_ERR_ARG, "node %d reached twice", c + o);
            depth[c + o] = depth[i] + 1;
            order.push_back(c + o);
        }
        if (depth[i] + 1 > 40) return fail(COLT_ERR_ARG, "octree deeper than 40");
    }
    if ((int64_t)order.size() != nn)
        return fail(COLT_ERR_ARG, "%lld nodes unreachable from the root",
                    (long long)(nn - (int64_t)order.size()));
    return COLT_OK;
}

// The device node table (a leaf holds -(leaf index + 1), leaves numbered in
// node order) and the caller's node of every leaf.
void node_table(const int32_t *child, int64_t nn, std::vector<int32_t> &child_dev,
                std::vector<int64_t> &leaf_src)
{
    child_dev.assign(nn, 0);
    leaf_src.clear();
    for (int64_t i = 0; i < nn; ++i) {
        if (child[i] >= 0) {
            child_dev[i] = child[i];
        } else {
            child_dev[i] = -(int32_t)leaf_src.size() - 1;
            leaf_src.push_back(i);
        }
    }
}

// Device memory from the caller's allocator (or hipMalloc), remembered for release.
struct DevMem {
    colt_allocator alloc{};
    bool custom = false;
    std::vector<void *> ptrs;
    size_t bytes = 0;

    void *get(size_t n)
    {
        n = (n + 255) & ~size_t(255);
        if (n == 0) n = 256;
        void *p = nullptr;
        if (custom) {
            p = alloc.alloc(n, alloc.user);
        } else if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
        }
        if (p) {
            ptrs.push_back(p);
            bytes += n;
        }
        return p;
    }
    void release_all()
    {
        for (void *p : ptrs) {
            if (custom) alloc.free(p, alloc.user);
            else (void)hipFree(p);
        }
        ptrs.clear();
        bytes = 0;
    }
};

// Device memory from an allocator (NULL or incomplete: hipMalloc) and its release.
void *dev_alloc(const colt_allocator &a, bool custom, size_t n)
{
    void *p = nullptr;
    if (custom) return a.alloc(n, a.user);
    return (hipMalloc(&p, n) == hipSuccess) ? p : nullptr;
}

void dev_free(const colt_allocator &a, bool custom, void *p)
{
    if (!p) return;
    if (custom) a.free(p, a.user);
    else (void)hipFree(p);
}

// Reusable launch tables: device memory from the jobs' allocator plus pinned
// host staging, recycled once the event recorded after their launch has
// completed.  Tables are kept per allocator and are never returned to it.
// Small tables come in batches cut from one device and one pinned host
// allocation, so a burst of launches in flight (steps queued on several
// streams) does not allocate per launch.  A table handed out is busy until its
// event is recorded, so concurrent callers never share one.
struct LaunchBuf {
    void *dev = nullptr;
    void *host = nullptr;
    size_t size = 0;
    hipEvent_t done = nullptr;
    colt_allocator alloc{};
    bool custom = false;
    bool busy = false;
};
std::mutex g_pool_mu;
std::vector<LaunchBuf *> g_pool;
constexpr size_t kLaunchSlot = 16384;     // bytes of a small table
constexpr int kLaunchBatch = 16;          // small tables allocated together

bool same_allocator(const LaunchBuf *b, const colt_allocator &a, bool custom)
{
    if (b->custom != custom) return false;
    return !custom || (b->alloc.alloc == a.alloc && b->alloc.free == a.free &&
                       b->alloc.user == a.user);
}

LaunchBuf *acquire_launch_buf(size_t bytes, const colt_allocator &a, bool custom)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (LaunchBuf *b : g_pool) {
        if (!b->busy && b->size >= bytes && same_allocator(b, a, custom) &&
            hipEventQuery(b->done) == hipSuccess) {
            b->busy = true;
            return b;
        }
    }
    const bool small = bytes <= kLaunchSlot;
    const size_t slot = small ? kLaunchSlot : std::max<size_t>((bytes + 4095) & ~size_t(4095), 4096);
    const int n = small ? kLaunchBatch : 1;
    void *dev = dev_alloc(a, custom, slot * n);
    if (!dev) return nullptr;
    void *host = nullptr;
    if (hipHostMalloc(&host, slot * n, hipHostMallocDefault) != hipSuccess) {
        dev_free(a, custom, dev);
        return nullptr;
    }
    LaunchBuf *first = nullptr;
    for (int k = 0; k < n; ++k) {
        LaunchBuf *b = new LaunchBuf();
        b->size = slot;
        b->dev = (char *)dev + (size_t)k * slot;
        b->host = (char *)host + (size_t)k * slot;
        b->alloc = a;
        b->custom = custom;
        if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
            delete b;
            break;
        }
        g_pool.push_back(b);
        if (!first) first = b;
    }
    if (!first) {               // nothing refers to the memory: give it back
        dev_free(a, custom, dev);
        (void)hipHostFree(host);
        return nullptr;
    }
    first->busy = true;
    return first;
}

// Holds a table for one launch: on release its event has been recorded on the
// launch's stream (here, if an error cut the launch short), so the table is
// reused only after everything queued with it has run.
struct LaunchHold {
    LaunchBuf *b = nullptr;
    hipStream_t s = nullptr;
    bool recorded = false;
    ~LaunchHold()
    {
        if (!b) return;
        if (!recorded) (void)hipEventRecord(b->done, s);
        std::lock_guard<std::mutex> lk(g_pool_mu);
        b->busy = false;
    }
};

// Host stop words (colt_stop_set): pinned, device-mapped, coherent memory the
// transport kernel polls.
std::mutex g_stop_mu;
int *g_stop_words = nullptr;

int *stop_words()
{
    std::lock_guard<std::mutex> lk(g_stop_mu);
    if (!g_stop_words) {
        void *p = nullptr;
        if (hipHostMalloc(&p, kStopTokens * sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            return nullptr;
        std::memset(p, 0, kStopTokens * sizeof(int));
        g_stop_words = (int *)p;
    }
    return g_stop_words;
}

int cu_count()
{
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n = 256;
    }
    return n;
}

bool finite_pos(double v) { return std::isfinite(v); }

// Lanes a launch may keep resident on this device.
uint64_t resident_lanes() { return (uint64_t)cu_count() * kMaxLanesPerCU; }

// Slots per sub-buffer of a camera job's march-task buffer: `req` slots in
// all (0: four times what the lanes of a full launch can still add after a
// stop request -- two events of n_cams marches each, in chunks -- at least
// 2^20 and at most 2^26), rounded to whole chunks.
uint64_t task_sub_slots(uint64_t n_photons, int n_cams, uint64_t req)
{
    if (req == 0) {
        const uint64_t lanes = std::min<uint64_t>(std::max<uint64_t>(n_photons, 64), resident_lanes());
        const uint64_t per_lane = ((2 * (uint64_t)n_cams + kTaskChunk - 1) / kTaskChunk + 1) * kTaskChunk;
        req = std::min<uint64_t>(std::max<uint64_t>(4 * lanes * per_lane, 1ull << 20), 1ull << 26);
    }
    return std::max<uint64_t>((req / kTaskSubs + kTaskChunk - 1) / kTaskChunk * kTaskChunk,
                              (uint64_t)kTaskChunk);
}

}  // namespace

struct colt_grid_s {
    DevMem mem;
    GridView view{};               // cells/aux point at the FP64 records
    void *rec_d = nullptr, *aux_d = nullptr, *rec_f = nullptr, *aux_f = nullptr;
    double *n_dev = nullptr;       // n_HI per cell / leaf (for the non-local estimate)
    std::vector<int32_t> child_host, base_host;   // octree tables as uploaded
    int32_t kind = 0;
    int64_t n_leaves = 0;
    double dx_cm = 0.0;
    double box_min[3] = {0, 0, 0};
    std::atomic<int> jobs{0};
    hipStream_t stream = nullptr;
};

struct colt_graph_s {
    std::vector<colt_job> jobs;
    void *dev = nullptr;
    colt_allocator alloc{};
    bool custom = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t quota = 0;
    bool may_stop = false;
};

struct colt_job_s {
    DevMem mem;
    colt_grid grid = nullptr;
    JobView view{};
    colt_job_params params{};
    // host view of the device cursor: photons reserved by launches so far; it
    // is exact unless a launch that can stop has run since the last refresh
    uint64_t h_cursor = 0;
    uint64_t h_susp = 0;             // suspended photons at the last refresh
    bool uncertain = false;          // a launch that may have stopped is pending
    // one event per stream the job's launches ran on (tally and release wait
    // on all of them), taken first from events created with the job
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
    std::vector<hipEvent_t> spare_ev;
};

namespace {

// The job's completion event for stream s: the one it already has there, else
// one created with the job, else (when allowed) a new one.
hipError_t job_event(colt_job j, hipStream_t s, hipEvent_t *out, bool may_create = true)
{
    for (auto &e : j->ev)
        if (e.first == s) { *out = e.second; return hipSuccess; }
    hipEvent_t e = nullptr;
    if (!j->spare_ev.empty()) {
        e = j->spare_ev.back();
        j->spare_ev.pop_back();
    } else {
        if (!may_create) return hipErrorOutOfMemory;
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
    }
    j->ev.emplace_back(s, e);
    *out = e;
    return hipSuccess;
}

hipError_t job_wait(colt_job j)
{
    for (auto &e : j->ev) {
        const hipError_t r = hipEventSynchronize(e.second);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// hipSuccess when every launch of the job has ended, hipErrorNotReady if not.
hipError_t job_query(colt_job j)
{
    for (auto &e : j->ev) {
        const hipError_t r = hipEventQuery(e.second);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// Waits for the job's launches and reads its device cursor and suspended count.
hipError_t job_refresh(colt_job j)
{
    hipError_t r = job_wait(j);
    if (r != hipSuccess) return r;
    JobCtl c;
    r = hipMemcpy(&c, j->view.ctl, sizeof(JobCtl), hipMemcpyDeviceToHost);
    if (r != hipSuccess) return r;
    j->h_cursor = c.cursor;
    j->h_susp = c.n_in;
    j->uncertain = false;
    return hipSuccess;
}

// Photons a launch of the job may hand out (exact when not uncertain).
uint64_t job_work_bound(colt_job j, uint64_t quota)
{
    const uint64_t left = j->params.n_photons - std::min(j->h_cursor, j->params.n_photons);
    const uint64_t take = (quota && quota < left) ? quota : left;
    return take + (j->uncertain ? (uint64_t)j->view.susp_cap : j->h_susp);
}

}  // namespace

extern "C" {

const char *colt_last_error(void) { return g_error.c_str(); }

colt_status colt_init_grid(const colt_grid_desc *d, const colt_allocator *alloc, void *stream,
                           colt_grid *out)
{
    if (!d || !out) return fail(COLT_ERR_ARG, "null descriptor or output");
    *out = nullptr;
    if (d->kind != 0 && d->kind != 1) return fail(COLT_ERR_ARG, "grid kind must be 0 or 1");
    if (!d->n_HI || !d->T) return fail(COLT_ERR_ARG, "n_HI and T are required");
    double ext[3];
    for (int i = 0; i < 3; ++i) {
        ext[i] = d->box_max[i] - d->box_min[i];
        if (!(ext[i] > 0.0) || !finite_pos(ext[i]))
            return fail(COLT_ERR_ARG, "box extent must be positive on every axis");
    }
    if (!(d->escape_radius >= 0.0)) return fail(COLT_ERR_ARG, "escape_radius must be >= 0");
    if (!(d->dust_albedo >= 0.0 && d->dust_albedo <= 1.0))
        return fail(COLT_ERR_ARG, "dust_albedo must lie in [0, 1]");
    colt_grid g = new colt_grid_s();
    g->kind = d->kind;
    g->stream = (hipStream_t)stream;
    if (alloc && alloc->alloc && alloc->free) {
        g->mem.alloc = *alloc;
        g->mem.custom = true;
    }
    for (int i = 0; i < 3; ++i) g->box_min[i] = d->box_min[i];

    // leaf list (index into the caller's arrays) and device node table
    std::vector<int64_t> leaf_src;
    std::vector<int32_t> child_dev, base_dev;
    std::vector<uint32_t> rope_dev;
    int nb = 0;
    if (d->kind == 0) {
        if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0)
            return delete g, fail(COLT_ERR_ARG, "Cartesian dimensions must be positive");
        const int64_t n = (int64_t)d->nx * d->ny * d->nz;
        if (d->n_cells != n)
            return delete g, fail(COLT_ERR_ARG, "n_cells %lld != nx*ny*nz %lld",
                                  (long long)d->n_cells, (long long)n);
        if (n > INT32_MAX) return delete g, fail(COLT_ERR_ARG, "too many cells");
        const double wx = ext[0] / d->nx, wy = ext[1] / d->ny, wz = ext[2] / d->nz;
        if (std::fabs(wy / wx - 1.0) > 1e-9 || std::fabs(wz / wx - 1.0) > 1e-9)
            return delete g, fail(COLT_ERR_ARG, "cells must be cubes");
        g->dx_cm = wx;
        g->view.n[0] = d->nx; g->view.n[1] = d->ny; g->view.n[2] = d->nz;
        g->n_leaves = n;
        leaf_src.resize(n);
        for (int64_t i = 0; i < n; ++i) leaf_src[i] = i;
    } else {
        const int64_t nn = d->n_cells;
        if (nn <= 0 || !d->child) return delete g, fail(COLT_ERR_ARG, "octree needs nodes and child");
        if (nn > INT32_MAX / 2) return delete g, fail(COLT_ERR_ARG, "too many octree nodes");
        if (std::fabs(ext[1] / ext[0] - 1.0) > 1e-9 || std::fabs(ext[2] / ext[0] - 1.0) > 1e-9)
            return delete g, fail(COLT_ERR_ARG, "octree root box must be a cube");
        std::vector<int32_t> depth;
        std::vector<int64_t> order;
        if (octree_walk(d->child, nn, depth, order) != COLT_OK) return delete g, COLT_ERR_ARG;
        // base level: deepest level above which every node is refined (<= 7)
        int min_leaf_depth = 1 << 30;
        for (int64_t i = 0; i < nn; ++i)
            if (d->child[i] < 0) min_leaf_depth = std::min(min_leaf_depth, depth[i]);
        const int Lb = std::min(min_leaf_depth, 7);
        nb = 1 << Lb;
        g->dx_cm = ext[0] / nb;
        g->view.n[0] = g->view.n[1] = g->view.n[2] = nb;
        node_table(d->child, nn, child_dev, leaf_src);
        g->n_leaves = (int64_t)leaf_src.size();
        build_ropes(child_dev.data(), nn, depth, order, leaf_src, rope_dev);
        base_dev.resize((size_t)nb * nb * nb);
        for (int iz = 0; iz < nb; ++iz)
            for (int iy = 0; iy < nb; ++iy)
                for (int ix = 0; ix < nb; ++ix) {
                    int64_t node = 0;
                    for (int lv = Lb - 1; lv >= 0; --lv) {
                        const int oct = ((ix >> lv) & 1) | (((iy >> lv) & 1) << 1) |
                                        (((iz >> lv) & 1) << 2);
                        node = d->child[node] + oct;
                    }
                    base_dev[((size_t)iz * nb + iy) * nb + ix] = (int32_t)node;
                }
    }
    const int64_t nl = g->n_leaves;
    // gather the gas of the leaves and validate it
    std::vector<double> raw((size_t)nl * 7);
    double *h_n = raw.data(), *h_T = h_n + nl, *h_kd = h_T + nl, *h_nl = h_kd + nl,
           *h_v = h_nl + nl;
    for (int64_t j = 0; j < nl; ++j) {
        const int64_t i = leaf_src[j];
        h_n[j] = d->n_HI[i];
        h_T[j] = d->T[i];
        h_kd[j] = d->k_dust ? d->k_dust[i] : 0.0;
        h_nl[j] = d->atau_nl ? d->atau_nl[i] : 0.0;
        for (int c = 0; c < 3; ++c) h_v[3 * j + c] = d->v ? d->v[3 * i + c] : 0.0;
        if (!(h_n[j] >= 0.0) || !std::isfinite(h_n[j]) || !(h_T[j] > 0.0) ||
            !std::isfinite(h_T[j]) || !(h_kd[j] >= 0.0) || !std::isfinite(h_kd[j]) ||
            !(h_nl[j] >= 0.0) || !std::isfinite(h_nl[j]) || !std::isfinite(h_v[3 * j]) ||
            !std::isfinite(h_v[3 * j + 1]) || !std::isfinite(h_v[3 * j + 2])) {
            delete g;
            return fail(COLT_ERR_ARG, "cell %lld has invalid gas values", (long long)i);
        }
    }
    hipStream_t s = g->stream;
    void *stage = g->mem.get(raw.size() * sizeof(double));
    void *rd = g->mem.get((size_t)nl * sizeof(CellRec<double>));
    void *ad = g->mem.get((size_t)nl * sizeof(CellAux<double>));
    // FP32 octree records share a 64-byte line with the leaf's six links, so a
    // crossing reads one line for the leaf it leaves and the leaf it enters
    const int rf_stride = (d->kind == 1) ? 2 : 1;
    static_assert(sizeof(CellRec<float>) == 32, "an FP32 record is half a 64-byte line");
    void *rf = g->mem.get((size_t)nl * rf_stride * sizeof(CellRec<float>));
    void *af = g->mem.get((size_t)nl * sizeof(CellAux<float>));
    g->n_dev = (double *)g->mem.get((size_t)nl * sizeof(double));
    void *dchild = nullptr, *dbase = nullptr, *drope = nullptr;
    if (d->kind == 1) {
        dchild = g->mem.get(child_dev.size() * sizeof(int32_t));
        dbase = g->mem.get(base_dev.size() * sizeof(int32_t));
        drope = g->mem.get(rope_dev.size() * sizeof(uint32_t));
    }
    if (!stage || !rd || !ad || !rf || !af || !g->n_dev ||
        (d->kind == 1 && (!dchild || !dbase || !drope))) {
        g->mem.release_all();
        delete g;
        return fail(COLT_ERR_NOMEM, "device allocation for the grid failed");
    }
    auto cleanup = [&]() { g->mem.release_all(); delete g; };
    hipError_t e = hipMemcpyAsync(stage, raw.data(), raw.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && d->kind == 1) {
        e = hipMemcpyAsync(dchild, child_dev.data(), child_dev.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dbase, base_dev.data(), base_dev.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(drope, rope_dev.data(), rope_dev.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s);
    }
    const double *sd = (const double *)stage;
    if (e == hipSuccess)
        e = launch_cell_setup(nl, sd, sd + nl, sd + 4 * nl, sd + 2 * nl, sd + 3 * nl, g->dx_cm,
                              rd, ad, rf, rf_stride, af, s);
    if (e == hipSuccess && d->kind == 1 && nl > 0)
        e = hipMemcpy2DAsync((char *)rf + sizeof(CellRec<float>), 2 * sizeof(CellRec<float>),
                             rope_dev.data(), 6 * sizeof(uint32_t), 6 * sizeof(uint32_t),
                             (size_t)nl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->n_dev, sd, (size_t)nl * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cleanup();
        return fail(COLT_ERR_HIP, "grid upload or set-up failed: %s", hipGetErrorString(e));
    }
    // the staging buffer is not needed any more
    if (g->mem.custom) g->mem.alloc.free(stage, g->mem.alloc.user);
    else (void)hipFree(stage);
    g->mem.ptrs.erase(std::find(g->mem.ptrs.begin(), g->mem.ptrs.end(), stage));
    g->mem.bytes -= ((raw.size() * sizeof(double) + 255) & ~size_t(255));

    GridView &v = g->view;
    v.kind = d->kind;
    v.rec_stride = 1;          // the FP64 records and the separate link table
    v.rope_stride = 6;
    v.cells = rd;
    v.aux = ad;
    v.child = (const int32_t *)dchild;
    v.base = (const int32_t *)dbase;
    v.rope = (const uint32_t *)drope;
    for (int i = 0; i < 3; ++i) v.centre[i] = 0.5 * ext[i] / g->dx_cm;
    v.esc_r = d->escape_radius / g->dx_cm;
    v.albedo = d->dust_albedo;
    g->rec_d = rd; g->aux_d = ad; g->rec_f = rf; g->aux_f = af;
    if (d->kind == 1) {
        g->child_host = std::move(child_dev);
        g->base_host = std::move(base_dev);
    }
    *out = g;
    return COLT_OK;
}

colt_status colt_grid_nonlocal(colt_grid g, double f_nl, void *stream)
{
    if (!g) return fail(COLT_ERR_ARG, "null grid");
    if (!(f_nl >= 0.0) || !std::isfinite(f_nl)) return fail(COLT_ERR_ARG, "f_nl must be >= 0");
    if (g->jobs.load() > 0) return fail(COLT_ERR_STATE, "grid has live jobs");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nl = g->n_leaves;
    double *boxes = nullptr;
    if (g->kind == 1) {
        // lower corner and size of every leaf, in base-cell units
        std::vector<double> hb((size_t)nl * 4);
        const int nb = g->view.n[0];
        struct Item { int32_t node; double lo[3]; double size; };
        std::vector<Item> stack;
        for (int iz = 0; iz < nb; ++iz)
            for (int iy = 0; iy < nb; ++iy)
                for (int ix = 0; ix < nb; ++ix) {
                    stack.push_back({g->base_host[((size_t)iz * nb + iy) * nb + ix],
                                     {(double)ix, (double)iy, (double)iz}, 1.0});
                    while (!stack.empty()) {
                        Item it = stack.back();
                        stack.pop_back();
                        const int32_t c = g->child_host[it.node];
                        if (c < 0) {
                            double *o = &hb[(size_t)(-c - 1) * 4];
                            o[0] = it.lo[0]; o[1] = it.lo[1]; o[2] = it.lo[2]; o[3] = it.size;
                            continue;
                        }
                        const double h = 0.5 * it.size;
                        for (int oc = 0; oc < 8; ++oc)
                            stack.push_back({c + oc,
                                             {it.lo[0] + ((oc & 1) ? h : 0.0),
                                              it.lo[1] + ((oc & 2) ? h : 0.0),
                                              it.lo[2] + ((oc & 4) ? h : 0.0)}, h});
                    }
                }
        boxes = (double *)dev_alloc(g->mem.alloc, g->mem.custom, hb.size() * sizeof(double));
        if (!boxes) return fail(COLT_ERR_NOMEM, "leaf boxes allocation failed");
        hipError_t e = hipMemcpyAsync(boxes, hb.data(), hb.size() * sizeof(double),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            dev_free(g->mem.alloc, g->mem.custom, boxes);
            return fail(COLT_ERR_HIP, "leaf boxes upload: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = launch_nonlocal(g->view, g->n_dev, boxes, nl, f_nl, g->aux_d, g->aux_f, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(g->mem.alloc, g->mem.custom, boxes);
    if (e != hipSuccess) return fail(COLT_ERR_HIP, "non-local estimate: %s", hipGetErrorString(e));
    return COLT_OK;
}

colt_status colt_release_grid(colt_grid g)
{
    if (!g) return COLT_OK;
    if (g->jobs.load() > 0) return fail(COLT_ERR_STATE, "grid still referenced by %d jobs",
                                        g->jobs.load());
    g->mem.release_all();
    delete g;
    return COLT_OK;
}

size_t colt_grid_bytes(colt_grid g) { return g ? g->mem.bytes : 0; }

colt_status colt_octree_links(const int32_t *child, int64_t n_nodes, uint32_t *links,
                              int64_t *n_leaves)
{
    if (!child || n_nodes <= 0 || !n_leaves)
        return fail(COLT_ERR_ARG, "child, n_nodes > 0 and n_leaves are required");
    if (n_nodes > INT32_MAX / 2) return fail(COLT_ERR_ARG, "too many octree nodes");
    std::vector<int32_t> depth;
    std::vector<int64_t> order;
    const colt_status st = octree_walk(child, n_nodes, depth, order);
    if (st != COLT_OK) return st;
    std::vector<int32_t> child_dev;
    std::vector<int64_t> leaf_src;
    node_table(child, n_nodes, child_dev, leaf_src);
    *n_leaves = (int64_t)leaf_src.size();
    if (!links) return COLT_OK;
    std::vector<uint32_t> rope;
    build_ropes(child_dev.data(), n_nodes, depth, order, leaf_src, rope);
    std::memcpy(links, rope.data(), rope.size() * sizeof(uint32_t));
    return COLT_OK;
}

colt_status colt_grid_fields(colt_grid g, double *out)
{
    if (!g || !out) return fail(COLT_ERR_ARG, "null grid or output");
    const int64_t n = g->n_leaves;
    std::vector<CellRec<double>> rec(n);
    std::vector<CellAux<double>> aux(n);
    HIP_TRY(hipStreamSynchronize(g->stream));
    HIP_TRY(hipMemcpy(rec.data(), g->rec_d, n * sizeof(CellRec<double>), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(aux.data(), g->aux_d, n * sizeof(CellAux<double>), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        double *o = out + 11 * i;
        o[0] = rec[i].k0 / g->dx_cm;
        o[1] = rec[i].a;
        o[2] = kVthRef / rec[i].s;
        o[3] = rec[i].ux; o[4] = rec[i].uy; o[5] = rec[i].uz;
        o[6] = rec[i].kd / g->dx_cm;
        o[7] = rec[i].xcw;
        o[8] = aux[i].g;
        o[9] = aux[i].atau_nl;
        o[10] = aux[i].atau_j;
    }
    return COLT_OK;
}

colt_status colt_emit(colt_grid g, const colt_source_desc *src, const colt_job_params *p,
                      colt_job *out)
{
    if (!g || !src || !p || !out) return fail(COLT_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->precision != COLT_FP64 && p->precision != COLT_FP32_BULK)
        return fail(COLT_ERR_ARG, "precision must be COLT_FP64 or COLT_FP32_BULK");
    if (p->xcrit_mode < 0 || p->xcrit_mode > 3) return fail(COLT_ERR_ARG, "xcrit_mode 0..3");
    if (p->xcrit_mode == 1 && !(p->atau0 >= 0.0)) return fail(COLT_ERR_ARG, "atau0 must be >= 0");
    if (p->n_bins < 0 || (p->n_bins > 0 && !(p->x_max > p->x_min)))
        return fail(COLT_ERR_ARG, "spectrum needs n_bins >= 0 and x_max > x_min");
    if (p->n_cams < 0 || p->n_cams > kMaxCams) return fail(COLT_ERR_ARG, "0 <= n_cams <= 64");
    if (p->n_cams > 0) {
        if (!p->cam_dir) return fail(COLT_ERR_ARG, "cam_dir required");
        if (p->cam_nbins < 0 || (p->cam_nbins > 0 && !(p->cam_xmax > p->cam_xmin)))
            return fail(COLT_ERR_ARG, "camera spectrum needs cam_xmax > cam_xmin");
        if (p->cam_npix < 0 || (p->cam_npix > 0 && !(p->cam_fov > 0.0)))
            return fail(COLT_ERR_ARG, "camera images need cam_fov > 0");
        if (!(p->tau_peel_max > 0.0)) return fail(COLT_ERR_ARG, "tau_peel_max must be > 0");
    }
    if (src->n_src < 1 || !src->pos) return fail(COLT_ERR_ARG, "at least one source position");
    if (src->kind < 0 || src->kind > 2) return fail(COLT_ERR_ARG, "source kind 0..2");
    if (src->kind != 2 && src->n_src != 1) return fail(COLT_ERR_ARG, "kinds 0, 1 take one source");
    if (src->kind == 1 && !(src->sigma >= 0.0)) return fail(COLT_ERR_ARG, "sigma must be >= 0");
    if (src->freq_mode != 0 && src->freq_mode != 1) return fail(COLT_ERR_ARG, "freq_mode 0 or 1");
    if (p->march_tasks > (1ull << 28)) return fail(COLT_ERR_ARG, "march_tasks above 2^28");

    colt_job j = new colt_job_s();
    j->grid = g;
    j->params = *p;
    j->params.cam_dir = nullptr;
    j->mem.alloc = g->mem.alloc;
    j->mem.custom = g->mem.custom;
    const int nc = p->n_cams;
    // host tables: sources in grid units, cumulative weights, cameras
    std::vector<double> hpos(3 * src->n_src), hcdf(src->n_src);
    double wsum = 0.0;
    for (int i = 0; i < src->n_src; ++i) {
        const double w = src->weight ? src->weight[i] : 1.0;
        if (!(w >= 0.0)) { delete j; return fail(COLT_ERR_ARG, "negative source weight"); }
        wsum += w;
        for (int c = 0; c < 3; ++c) hpos[3 * i + c] = (src->pos[3 * i + c] - g->box_min[c]) / g->dx_cm;
    }
    if (!(wsum > 0.0)) { delete j; return fail(COLT_ERR_ARG, "source weights sum to zero"); }
    double acc = 0.0;
    for (int i = 0; i < src->n_src; ++i) {
        acc += src->weight ? src->weight[i] : 1.0;
        hcdf[i] = acc / wsum;
    }
    std::vector<double> hcam(12 * std::max(nc, 1), 0.0);
    for (int i = 0; i < nc; ++i) {
        double dv[3] = {p->cam_dir[3 * i], p->cam_dir[3 * i + 1], p->cam_dir[3 * i + 2]};
        const double n = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (!(n > 0.0) || !std::isfinite(n)) { delete j; return fail(COLT_ERR_ARG, "camera %d direction", i); }
        for (double &c : dv) c /= n;
        double up[3] = {0.0, 0.0, 1.0};
        if (std::fabs(dv[2]) > 0.999) { up[1] = 1.0; up[2] = 0.0; }
        double eu[3] = {up[1] * dv[2] - up[2] * dv[1], up[2] * dv[0] - up[0] * dv[2],
                        up[0] * dv[1] - up[1] * dv[0]};
        const double m = std::sqrt(eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2]);
        for (double &c : eu) c /= m;
        const double ev[3] = {dv[1] * eu[2] - dv[2] * eu[1], dv[2] * eu[0] - dv[0] * eu[2],
                              dv[0] * eu[1] - dv[1] * eu[0]};
        double *o = &hcam[12 * i];
        for (int c = 0; c < 3; ++c) {
            o[c] = dv[c];
            o[3 + c] = (dv[c] != 0.0) ? 1.0 / dv[c] : 0.0;
            o[6 + c] = eu[c];
            o[9 + c] = ev[c];
        }
    }
    const uint64_t N = p->n_photons;
    const size_t nbins = (size_t)p->n_bins + 2;
    const size_t ncs = (size_t)nc * p->cam_nbins, nimg = (size_t)nc * p->cam_npix * p->cam_npix;
    JobView &v = j->view;
    v.g = g->view;
    if (p->precision == COLT_FP32_BULK) {
        v.g.cells = g->rec_f;
        v.g.aux = g->aux_f;
        if (g->kind == 1) {
            v.g.rec_stride = 2;
            v.g.rope = (const uint32_t *)((const char *)g->rec_f + sizeof(CellRec<float>));
            v.g.rope_stride = 16;
        }
    }
    v.src_kind = src->kind;
    v.n_src = src->n_src;
    v.freq_mode = src->freq_mode;
    v.sigma = src->sigma / g->dx_cm;
    v.seed = p->seed;
    v.n_photons = N;
    v.max_events = p->max_events ? p->max_events : (uint64_t)1 << 62;
    v.xcrit_mode = p->xcrit_mode;
    v.recoil = p->recoil ? 1 : 0;
    v.isotropic = p->isotropic ? 1 : 0;
    v.n_bins = p->n_bins;
    v.xcrit_global = (p->atau0 < 1.0) ? 0.0 : std::cbrt(p->atau0) / 5.0;
    v.xcrit_global_f = (float)v.xcrit_global;
    v.x_min = p->x_min;
    v.x_max = p->x_max;
    v.n_cams = nc;
    v.cam_nbins = p->cam_nbins;
    v.npix = p->cam_npix;
    v.record = p->record ? 1 : 0;
    v.cam_xmin = p->cam_xmin;
    v.cam_xmax = p->cam_xmax;
    v.fov = (p->cam_fov > 0.0) ? p->cam_fov / g->dx_cm : 1.0;
    v.tau_peel_max = p->tau_peel_max;
    v.dx_cm = g->dx_cm;
    for (int c = 0; c < 3; ++c) v.box_min_cm[c] = g->box_min[c];

    DevMem &m = j->mem;
    double *d_pos = (double *)m.get(hpos.size() * sizeof(double));
    double *d_cdf = (double *)m.get(hcdf.size() * sizeof(double));
    double *d_cam = (double *)m.get(hcam.size() * sizeof(double));
    v.spectrum = (unsigned long long *)m.get(nbins * sizeof(unsigned long long));
    v.cam_spec = (double *)m.get(std::max<size_t>(ncs, 1) * sizeof(double));
    v.cam_img = (double *)m.get(std::max<size_t>(nimg, 1) * sizeof(double));
    v.counters = (unsigned long long *)m.get(kCounterSlots * kNumCounters * sizeof(unsigned long long));
    bool ok = d_pos && d_cdf && d_cam && v.spectrum && v.cam_spec && v.cam_img && v.counters;
    if (p->record && ok) {
        const size_t n1 = std::max<uint64_t>(N, 1);
        v.rec_x = (double *)m.get(n1 * sizeof(double));
        v.rec_nscat = (int32_t *)m.get(n1 * sizeof(int32_t));
        v.rec_status = (int32_t *)m.get(n1 * sizeof(int32_t));
        v.rec_pos = (double *)m.get(3 * n1 * sizeof(double));
        v.rec_peel = (double *)m.get(std::max<size_t>(n1 * nc, 1) * sizeof(double));
        ok = v.rec_x && v.rec_nscat && v.rec_status && v.rec_pos && v.rec_peel;
    }
    // control block and the two suspend arrays (a job's suspended photons
    // never outnumber the lanes a launch keeps resident)
    v.susp_cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(N, resident_lanes()));
    if (ok) {
        v.ctl = (JobCtl *)m.get(sizeof(JobCtl));
        v.susp[0] = (SuspRec *)m.get((size_t)v.susp_cap * sizeof(SuspRec));
        v.susp[1] = (SuspRec *)m.get((size_t)v.susp_cap * sizeof(SuspRec));
        ok = v.ctl && v.susp[0] && v.susp[1];
    }
    // march tasks of the next-event estimator: by default four times what the
    // lanes of a full launch can still add after a stop request (two events of
    // n_cams marches each, in chunks), at least 2^20 and at most 2^26 slots
    if (ok && nc > 0) {
        const uint64_t sub = task_sub_slots(N, nc, p->march_tasks);
        v.task_sub_cap = (uint32_t)sub;
        const size_t nt = sub * kTaskSubs;
        const size_t rb = (p->precision == COLT_FP64) ? 8 : 4;
        TaskSoA &T = v.task;
        T.rx = (double *)m.get(nt * 8);
        T.ry = (double *)m.get(nt * 8);
        T.rz = (double *)m.get(nt * 8);
        T.lox = (float *)m.get(nt * 4);
        T.loy = (float *)m.get(nt * 4);
        T.loz = (float *)m.get(nt * 4);
        T.size = (float *)m.get(nt * 4);
        T.cell = (int32_t *)m.get(nt * 4);
        T.cam = (int32_t *)m.get(nt * 4);
        T.xl = m.get(nt * rb);
        T.W = m.get(nt * rb);
        T.id = (unsigned long long *)m.get(nt * 8);
        ok = T.rx && T.ry && T.rz && T.lox && T.loy && T.loz && T.size && T.cell && T.cam &&
             T.xl && T.W && T.id;
    }
    if (!ok) {
        m.release_all();
        delete j;
        return fail(COLT_ERR_NOMEM, "device allocation for the job failed");
    }
    v.src_pos = d_pos;
    v.src_cdf = d_cdf;
    v.cam = d_cam;
    hipStream_t s = g->stream;
    hipError_t e = hipMemcpyAsync(d_pos, hpos.data(), hpos.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_cdf, hcdf.data(), hcdf.size() * sizeof(double),
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_cam, hcam.data(), hcam.size() * sizeof(double),
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(v.spectrum, 0, nbins * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(v.cam_spec, 0, std::max<size_t>(ncs, 1) * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(v.cam_img, 0, std::max<size_t>(nimg, 1) * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(v.counters, 0, kCounterSlots * kNumCounters * 8, s);
    if (e == hipSuccess && p->record)
        e = hipMemsetAsync(v.rec_peel, 0, std::max<size_t>(std::max<uint64_t>(N, 1) * nc, 1) * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(v.ctl, 0, sizeof(JobCtl), s);
    for (int i = 0; e == hipSuccess && i < kJobEvents; ++i) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) j->spare_ev.push_back(ev);
    }
    // host tables must outlive the asynchronous copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        for (hipEvent_t ev : j->spare_ev) (void)hipEventDestroy(ev);
        m.release_all();
        delete j;
        return fail(COLT_ERR_HIP, "job set-up failed: %s", hipGetErrorString(e));
    }
    g->jobs.fetch_add(1);
    *out = j;
    return COLT_OK;
}

size_t colt_job_bytes(colt_job j) { return j ? j->mem.bytes : 0; }

size_t colt_job_footprint(const colt_job_params *p, int32_t n_src)
{
    if (!p || n_src < 1) return 0;
    auto up = [](size_t n) { return std::max<size_t>((n + 255) & ~size_t(255), 256); };
    const uint64_t N = p->n_photons;
    const size_t nc = (size_t)std::max(p->n_cams, 0);
    size_t b = up(24 * (size_t)n_src) + up(8 * (size_t)n_src) + up(96 * std::max<size_t>(nc, 1));
    b += up(8 * ((size_t)std::max(p->n_bins, 0) + 2));
    b += up(8 * std::max<size_t>(nc * std::max(p->cam_nbins, 0), 1));
    b += up(8 * std::max<size_t>(nc * std::max(p->cam_npix, 0) * std::max(p->cam_npix, 0), 1));
    b += up(8 * kCounterSlots * kNumCounters);
    if (p->record) {
        const size_t n1 = std::max<uint64_t>(N, 1);
        b += up(8 * n1) + 2 * up(4 * n1) + up(24 * n1) + up(8 * std::max<size_t>(n1 * nc, 1));
    }
    const size_t cap = (size_t)std::max<uint64_t>(1, std::min<uint64_t>(N, resident_lanes()));
    b += up(sizeof(JobCtl)) + 2 * up(cap * sizeof(SuspRec));
    if (nc > 0) {
        const size_t nt = task_sub_slots(N, (int)nc, p->march_tasks) * kTaskSubs;
        const size_t rb = (p->precision == COLT_FP64) ? 8 : 4;
        b += 4 * up(nt * 8) + 6 * up(nt * 4) + 2 * up(nt * rb);
    }
    return b;
}

colt_status colt_job_status(colt_job j, uint64_t *launched, uint64_t *total)
{
    if (!j) return fail(COLT_ERR_ARG, "null job");
    if (j->uncertain) {
        const hipError_t e = job_refresh(j);
        if (e != hipSuccess) return fail(COLT_ERR_HIP, "job status: %s", hipGetErrorString(e));
    }
    if (launched) *launched = j->h_cursor - j->h_susp;
    if (total) *total = j->params.n_photons;
    return COLT_OK;
}

colt_status colt_job_pending(colt_job j, uint64_t *next_id, uint64_t *n_suspended,
                             uint64_t *ids, uint64_t ids_cap)
{
    if (!j) return fail(COLT_ERR_ARG, "null job");
    const hipError_t e = job_refresh(j);
    if (e != hipSuccess) return fail(COLT_ERR_HIP, "job progress: %s", hipGetErrorString(e));
    if (next_id) *next_id = j->h_cursor;
    if (n_suspended) *n_suspended = j->h_susp;
    const uint64_t n = std::min<uint64_t>(j->h_susp, ids ? ids_cap : 0);
    if (n) {
        JobCtl c;
        HIP_TRY(hipMemcpy(&c, j->view.ctl, sizeof(JobCtl), hipMemcpyDeviceToHost));
        std::vector<SuspRec> rec(n);
        HIP_TRY(hipMemcpy(rec.data(), c.cur ? j->view.susp[1] : j->view.susp[0],
                          n * sizeof(SuspRec), hipMemcpyDeviceToHost));
        for (uint64_t i = 0; i < n; ++i) ids[i] = rec[i].id;
        std::sort(ids, ids + n);
    }
    return COLT_OK;
}

void colt_release_job(colt_job j)
{
    if (!j) return;
    (void)job_wait(j);
    for (auto &e : j->ev) (void)hipEventDestroy(e.second);
    for (hipEvent_t e : j->spare_ev) (void)hipEventDestroy(e);
    j->mem.release_all();
    if (j->grid) j->grid->jobs.fetch_sub(1);
    delete j;
}

colt_status colt_stop_set(int32_t token, int32_t value)
{
    if (token < 1 || token >= kStopTokens) return fail(COLT_ERR_ARG, "stop token 1..%d", kStopTokens - 1);
    int *w = stop_words();
    if (!w) return fail(COLT_ERR_NOMEM, "stop words allocation failed");
    __atomic_store_n(&w[token], value ? 1 : 0, __ATOMIC_SEQ_CST);
    return COLT_OK;
}

static int march_min_of(const colt_launch *launch, int precision)
{
    const int m = (launch && launch->march_min > 0)
                      ? launch->march_min
                      : ((precision == COLT_FP64) ? kDefaultMarchMinFp64 : kDefaultMarchMinFp32);
    return m > 64 ? 64 : m;
}

namespace {

// Byte offsets of one launch's table in device memory.
struct TableLayout {
    size_t jobs, prefix, first, rprefix, peel_work, queue, rqueue, stop, bytes;
};

TableLayout table_layout(int nj)
{
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    TableLayout t{};
    size_t o = 0;
    t.jobs = o; o += up(sizeof(JobView) * nj);
    t.prefix = o; o += up(8 * (size_t)(nj + 1));
    t.first = o; o += up(8 * (size_t)nj);
    t.rprefix = o; o += up(4 * (size_t)(nj + 1));
    t.peel_work = o; o += up(8 * (size_t)nj);
    t.queue = o; o += 256;          // the three words polled or hit by atomics
    t.rqueue = o; o += 256;         // each have a cache line of their own
    t.stop = o; o += 256;
    t.bytes = o;
    return t;
}

LaunchView table_view(char *dev, const TableLayout &t, int nj, uint64_t quota, int march_min,
                      const int *stop_host, int tail_live)
{
    LaunchView L{};
    L.jobs = (JobView *)(dev + t.jobs);
    L.prefix = (uint64_t *)(dev + t.prefix);
    L.first_id = (uint64_t *)(dev + t.first);
    L.rprefix = (uint32_t *)(dev + t.rprefix);
    L.peel_work = (unsigned long long *)(dev + t.peel_work);
    L.queue = (unsigned long long *)(dev + t.queue);
    L.rqueue = (unsigned long long *)(dev + t.rqueue);
    L.stop_dev = (unsigned int *)(dev + t.stop);
    L.stop_host = stop_host;
    L.quota = quota;
    L.n_jobs = nj;
    L.march_min = march_min;
    L.tail_live = tail_live;
    return L;
}

// Launch shape of a transport launch over `views` (a host bound on the photons
// it hands out in `work`): workgroups of `block` lanes, at most the resident
// limit per CU, no more than the work needs, and few enough lanes that every
// camera job's task buffer keeps room for what its lanes add after a stop.
// Sets each camera job's high-water mark for this shape.
colt_status launch_shape(int prec, bool cams, std::vector<JobView> &views, uint64_t work,
                         int block, int per_cu, int *grid_out)
{
    const int nj = (int)views.size();
    if (per_cu <= 0) {
        hipError_t e = transport_occupancy(prec, cams, nj == 1, nj == 1 ? views[0].g.kind : -1,
                                           block, &per_cu);
        if (e != hipSuccess) return fail(COLT_ERR_HIP, "occupancy: %s", hipGetErrorString(e));
        if (per_cu <= 0) per_cu = 1;
    }
    uint64_t grid = (uint64_t)cu_count() * per_cu;
    grid = std::min<uint64_t>(grid, (uint64_t)cu_count() * kMaxLanesPerCU / block);
    const uint64_t lanes_needed = (work + 63) / 64 * 64;
    grid = std::min<uint64_t>(grid, (lanes_needed + block - 1) / block);
    for (const JobView &v : views) {
        if (!v.task_sub_cap) continue;
        const uint64_t per_lane = ((2 * (uint64_t)v.n_cams + kTaskChunk - 1) / kTaskChunk + 1) * kTaskChunk;
        const uint64_t max_lanes = (uint64_t)v.task_sub_cap / 2 * kTaskSubs / per_lane;
        if (max_lanes < 64) return fail(COLT_ERR_ARG, "march-task buffer too small for one wave");
        grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, max_lanes / block));
    }
    if (grid < 1) grid = 1;
    const uint64_t lanes = grid * block;
    for (JobView &v : views) {
        if (!v.task_sub_cap) continue;
        const uint64_t per_lane = ((2 * (uint64_t)v.n_cams + kTaskChunk - 1) / kTaskChunk + 1) * kTaskChunk;
        const uint64_t head = (lanes + kTaskSubs - 1) / kTaskSubs * per_lane;
        v.task_hw = (uint32_t)(v.task_sub_cap - std::min<uint64_t>(head, v.task_sub_cap));
    }
    *grid_out = (int)grid;
    return COLT_OK;
}

// The kernels of one launch on stream s: plan, transport, the deferred
// next-event marches of every camera job, advance.
hipError_t launch_sequence(int prec, bool cams, const LaunchView &L,
                           const std::vector<JobView> &views, int grid, int block,
                           hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    hipError_t e = launch_plan(L, false, s);
    if (e == hipSuccess && t0) e = hipEventRecord(t0, s);
    if (e == hipSuccess)
        e = launch_transport(prec, cams, L, views.size() == 1 ? views[0] : JobView{}, grid, block, s);
    if (e == hipSuccess && t1) e = hipEventRecord(t1, s);
    for (size_t j = 0; e == hipSuccess && j < views.size(); ++j) {
        if (!views[j].task_sub_cap) continue;
        int per_cu = 0;
        e = peel_occupancy(prec, views[j].g.kind, &per_cu);
        if (e == hipSuccess)
            e = launch_peel(prec, views[j], L.peel_work + j, cu_count() * std::max(per_cu, 1), s);
    }
    if (e == hipSuccess) e = launch_plan(L, true, s);
    return e;
}

}  // namespace

namespace {

// Both transport entry points.  fixed: the launch table is the device's fixed
// array (colt_transport_static) and nothing is allocated -- no launch table,
// no stop words, no timing events, no job events beyond those made with the
// jobs; otherwise the table comes from the jobs' allocator through the pool.
colt_status transport_impl(const colt_job *jobs, int32_t n_jobs, const colt_launch *launch,
                           void *stream, bool fixed)
{
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(COLT_ERR_ARG, "bad job list");
    hipStream_t s = (hipStream_t)stream;
    int block = (launch && launch->block) ? launch->block : 256;
    if (block < 64 || block > 256 || block % 64)
        return fail(COLT_ERR_ARG, "block must be 64, 128, 192 or 256");
    const uint64_t quota = launch ? launch->photons_per_job : 0;
    bool timed = launch && launch->time_kernel;
    const int token = launch ? launch->stop_token : 0;
    if (token < 0 || token >= kStopTokens) return fail(COLT_ERR_ARG, "stop token 0..%d", kStopTokens - 1);
    const int tail_live = launch ? launch->tail_live : 0;
    if (tail_live < 0 || tail_live > 64) return fail(COLT_ERR_ARG, "tail_live must lie in 0..64");
    const int reps = (launch && launch->launches > 0) ? launch->launches : 1;
    if (launch && launch->launches < 0) return fail(COLT_ERR_ARG, "launches must not be negative");
    const int *stop_host = nullptr;
    if (token) {
        if (fixed) {
            std::lock_guard<std::mutex> lk(g_stop_mu);
            if (!g_stop_words)
                return fail(COLT_ERR_STATE, "stop words not allocated yet (call colt_stop_set first)");
        }
        int *w = stop_words();
        if (!w) return fail(COLT_ERR_NOMEM, "stop words allocation failed");
        int *dw = nullptr;
        HIP_TRY(hipHostGetDevicePointer((void **)&dw, w, 0));
        stop_host = dw + token;
    }
    for (int i = 0; i < n_jobs; ++i) {
        if (!jobs[i]) return fail(COLT_ERR_ARG, "null job %d", i);
        for (int k = 0; k < i; ++k)
            if (jobs[k] == jobs[i]) return fail(COLT_ERR_ARG, "job %d listed twice", i);
    }
    for (int prec = 0; prec < 2; ++prec) {
        std::vector<JobView> views;
        std::vector<colt_job> members;
        bool cams = false;
        uint64_t work = 0;
        for (int i = 0; i < n_jobs; ++i) {
            colt_job j = jobs[i];
            if (j->params.precision != prec) continue;
            const uint64_t w = job_work_bound(j, quota);
            if (w == 0 && !j->uncertain) continue;
            views.push_back(j->view);
            members.push_back(j);
            cams = cams || j->params.n_cams > 0;
            work += w;
        }
        if (members.empty()) continue;
        const int nj = (int)members.size();
        const bool may_stop = token != 0 || cams || tail_live > 0;
        // a launch that may stop, or a job another such launch may have left
        // suspended photons to, must follow the job's launches on other streams
        for (colt_job j : members) {
            if (!(may_stop || j->uncertain)) continue;
            for (auto &e : j->ev)
                if (e.first != s) HIP_TRY(hipStreamWaitEvent(s, e.second, 0));
        }
        if (fixed) {
            // every job must have an event for this stream before anything runs
            for (colt_job j : members) {
                bool ok = !j->spare_ev.empty();
                for (auto &e : j->ev) ok = ok || e.first == s;
                if (!ok) return fail(COLT_ERR_STATE, "a job launched on more than %d streams", kJobEvents);
            }
        }
        int grid = 0;
        const colt_status st = launch_shape(prec, cams, views, work, block,
                                            launch ? launch->blocks_per_cu : 0, &grid);
        if (st != COLT_OK) return st;
        const TableLayout t = table_layout(nj);
        LaunchHold hold;
        LaunchBuf *b = nullptr;
        char *table = nullptr;
        if (fixed) {
            if (nj > kStaticJobs || t.bytes > kStaticTableBytes)
                return fail(COLT_ERR_ARG, "at most %d jobs of one precision per call", kStaticJobs);
            void *p = nullptr;
            HIP_TRY(static_table(&p));
            table = (char *)p;
            HIP_TRY(put_views(views.data(), nj, (JobView *)(table + t.jobs), s));
        } else {
            b = acquire_launch_buf(t.bytes, members[0]->mem.alloc, members[0]->mem.custom);
            if (!b) return fail(COLT_ERR_NOMEM, "launch table allocation failed");
            hold.b = b;
            hold.s = s;
            std::memset(b->host, 0, t.bytes);
            std::memcpy((char *)b->host + t.jobs, views.data(), sizeof(JobView) * nj);
            HIP_TRY(hipMemcpyAsync(b->dev, b->host, t.bytes, hipMemcpyHostToDevice, s));
            table = (char *)b->dev;
        }
        const LaunchView L = table_view(table, t, nj, quota, march_min_of(launch, prec), stop_host,
                                        tail_live);
        if (fixed) timed = false;
        if (timed && !g_t0) {
            HIP_TRY(hipEventCreate(&g_t0));
            HIP_TRY(hipEventCreate(&g_t1));
        }
        // the timing events bracket the first to the last transport kernel
        for (int rep = 0; rep < reps; ++rep)
            HIP_TRY(launch_sequence(prec, cams, L, views, grid, block, s,
                                    (timed && rep == 0) ? g_t0 : nullptr,
                                    (timed && rep == reps - 1) ? g_t1 : nullptr));
        if (timed) g_timed = true;
        if (b) {
            HIP_TRY(hipEventRecord(b->done, s));
            hold.recorded = true;
        }
        for (colt_job j : members) {
            if (!j->uncertain && !may_stop) {
                const uint64_t left = j->params.n_photons - j->h_cursor;
                j->h_cursor += (quota && quota < left) ? quota : left;
                j->h_susp = 0;
            } else {
                j->uncertain = true;
            }
            hipEvent_t ev = nullptr;
            const hipError_t e = job_event(j, s, &ev, !fixed);
            if (e == hipErrorOutOfMemory && fixed)
                return fail(COLT_ERR_STATE, "a job launched on more than %d streams", kJobEvents);
            HIP_TRY(e);
            HIP_TRY(hipEventRecord(ev, s));
        }
    }
    return COLT_OK;
}

}  // namespace

colt_status colt_transport(const colt_job *jobs, int32_t n_jobs, const colt_launch *launch,
                           void *stream)
{
    return transport_impl(jobs, n_jobs, launch, stream, false);
}

colt_status colt_transport_static(const colt_job *jobs, int32_t n_jobs,
                                  const colt_launch *launch, void *stream)
{
    return transport_impl(jobs, n_jobs, launch, stream, true);
}

colt_status colt_graph_create(const colt_job *jobs, int32_t n_jobs, const colt_launch *launch,
                              void *capture_stream, colt_graph *out)
{
    if (!out) return fail(COLT_ERR_ARG, "null output");
    *out = nullptr;
    if (n_jobs < 1 || !jobs) return fail(COLT_ERR_ARG, "a graph needs at least one job");
    if (!capture_stream) return fail(COLT_ERR_ARG, "capture needs a non-default stream");
    const int prec = jobs[0] ? jobs[0]->params.precision : 0;
    bool cams = false;
    std::vector<JobView> views;
    for (int i = 0; i < n_jobs; ++i) {
        if (!jobs[i]) return fail(COLT_ERR_ARG, "null job %d", i);
        if (jobs[i]->params.precision != prec)
            return fail(COLT_ERR_ARG, "all jobs of a graph share one precision");
        for (int k = 0; k < i; ++k)
            if (jobs[k] == jobs[i]) return fail(COLT_ERR_ARG, "job %d listed twice", i);
        cams = cams || jobs[i]->params.n_cams > 0;
        views.push_back(jobs[i]->view);
    }
    const int block = (launch && launch->block) ? launch->block : 256;
    if (block < 64 || block > 256 || block % 64) return fail(COLT_ERR_ARG, "block 64..256");
    const int token = launch ? launch->stop_token : 0;
    if (token < 0 || token >= kStopTokens) return fail(COLT_ERR_ARG, "stop token 0..%d", kStopTokens - 1);
    const int tail_live = launch ? launch->tail_live : 0;
    if (tail_live < 0 || tail_live > 64) return fail(COLT_ERR_ARG, "tail_live must lie in 0..64");
    if (launch && launch->launches < 0) return fail(COLT_ERR_ARG, "launches must not be negative");
    const int reps = (launch && launch->launches > 0) ? launch->launches : 1;
    const int *stop_host = nullptr;
    if (token) {
        int *w = stop_words();
        if (!w) return fail(COLT_ERR_NOMEM, "stop words allocation failed");
        int *dw = nullptr;
        HIP_TRY(hipHostGetDevicePointer((void **)&dw, w, 0));
        stop_host = dw + token;
    }
    const int nj = n_jobs;
    int grid = 0;
    // a replay's work is not known when it is captured: size for a full device
    const colt_status st = launch_shape(prec, cams, views, ~0ull >> 8, block,
                                        launch ? launch->blocks_per_cu : 0, &grid);
    if (st != COLT_OK) return st;
    const TableLayout t = table_layout(nj);
    std::vector<char> h(t.bytes, 0);
    std::memcpy(h.data() + t.jobs, views.data(), sizeof(JobView) * nj);
    colt_graph gr = new colt_graph_s();
    gr->jobs.assign(jobs, jobs + nj);
    gr->quota = launch ? launch->photons_per_job : 0;
    gr->may_stop = token != 0 || cams || tail_live > 0;
    gr->alloc = jobs[0]->mem.alloc;
    gr->custom = jobs[0]->mem.custom;
    gr->dev = dev_alloc(gr->alloc, gr->custom, t.bytes);
    if (!gr->dev) {
        delete gr;
        return fail(COLT_ERR_NOMEM, "graph tables allocation failed");
    }
    hipStream_t s = (hipStream_t)capture_stream;
    hipError_t e = hipMemcpyAsync(gr->dev, h.data(), t.bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const LaunchView L = table_view((char *)gr->dev, t, nj, gr->quota, march_min_of(launch, prec),
                                    stop_host, tail_live);
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = hipSuccess;
        for (int rep = 0; rep < reps && e1 == hipSuccess; ++rep)
            e1 = launch_sequence(prec, cams, L, views, grid, block, s, nullptr, nullptr);
        e = hipStreamEndCapture(s, &gr->graph);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        dev_free(gr->alloc, gr->custom, gr->dev);
        delete gr;
        return fail(COLT_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = gr;
    return COLT_OK;
}

colt_status colt_graph_launch(colt_graph gr, void *stream)
{
    if (!gr) return fail(COLT_ERR_ARG, "null graph");
    hipStream_t s = (hipStream_t)stream;
    for (colt_job j : gr->jobs) {
        if (!(gr->may_stop || j->uncertain)) continue;
        for (auto &e : j->ev)
            if (e.first != s) HIP_TRY(hipStreamWaitEvent(s, e.second, 0));
    }
    HIP_TRY(hipGraphLaunch(gr->exec, s));
    for (colt_job j : gr->jobs) {        // host mirror of the device plan
        if (!j->uncertain && !gr->may_stop) {
            const uint64_t left = j->params.n_photons - j->h_cursor;
            j->h_cursor += (gr->quota && gr->quota < left) ? gr->quota : left;
            j->h_susp = 0;
        } else {
            j->uncertain = true;
        }
        hipEvent_t ev = nullptr;
        HIP_TRY(job_event(j, s, &ev));
        HIP_TRY(hipEventRecord(ev, s));
    }
    return COLT_OK;
}

void colt_graph_release(colt_graph gr)
{
    if (!gr) return;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    (void)hipDeviceSynchronize();
    dev_free(gr->alloc, gr->custom, gr->dev);
    delete gr;
}

double colt_last_kernel_ms(void)
{
    if (!g_timed) return -1.0;
    float ms = -1.0f;
    if (hipEventSynchronize(g_t1) != hipSuccess) return -1.0;
    if (hipEventElapsedTime(&ms, g_t0, g_t1) != hipSuccess) return -1.0;
    return ms;
}

colt_status colt_tally(colt_job j, colt_tally_out *o, int32_t wait)
{
    if (!j || !o) return fail(COLT_ERR_ARG, "null job or output");
    if (wait) {
        const hipError_t e = job_wait(j);
        if (e != hipSuccess) return fail(COLT_ERR_HIP, "job wait: %s", hipGetErrorString(e));
    } else {
        const hipError_t q = job_query(j);
        if (q == hipErrorNotReady) return fail(COLT_ERR_BUSY, "job still running");
        if (q != hipSuccess) return fail(COLT_ERR_HIP, "event query: %s", hipGetErrorString(q));
    }
    HIP_TRY(hipStreamSynchronize(j->grid->stream));
    {
        JobCtl c;
        HIP_TRY(hipMemcpy(&c, j->view.ctl, sizeof(JobCtl), hipMemcpyDeviceToHost));
        if (c.overflow)
            return fail(COLT_ERR_STATE, "%u suspended photons or next-event marches found no "
                        "room (results incomplete)", c.overflow);
    }
    const colt_job_params &p = j->params;
    const JobView &v = j->view;
    const size_t nbins = (size_t)p.n_bins + 2;
    if (o->spectrum) {
        std::vector<unsigned long long> tmp(nbins);
        HIP_TRY(hipMemcpy(tmp.data(), v.spectrum, nbins * 8, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < nbins; ++i) o->spectrum[i] = (double)tmp[i];
    }
    const size_t ncs = (size_t)p.n_cams * p.cam_nbins;
    const size_t nimg = (size_t)p.n_cams * p.cam_npix * p.cam_npix;
    if (o->cam_spec && ncs) HIP_TRY(hipMemcpy(o->cam_spec, v.cam_spec, ncs * 8, hipMemcpyDeviceToHost));
    if (o->cam_img && nimg) HIP_TRY(hipMemcpy(o->cam_img, v.cam_img, nimg * 8, hipMemcpyDeviceToHost));
    {
        std::vector<unsigned long long> c(kCounterSlots * kNumCounters);
        HIP_TRY(hipMemcpy(c.data(), v.counters, c.size() * 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < COLT_N_COUNTERS; ++i) {
            uint64_t t = 0;
            for (int s = 0; s < kCounterSlots; ++s) t += c[s * kNumCounters + i];
            o->counters[i] = t;
        }
    }
    if (p.record) {
        const size_t N = p.n_photons;
        if (N) {
            if (o->rec_x) HIP_TRY(hipMemcpy(o->rec_x, v.rec_x, N * 8, hipMemcpyDeviceToHost));
            if (o->rec_nscat) HIP_TRY(hipMemcpy(o->rec_nscat, v.rec_nscat, N * 4, hipMemcpyDeviceToHost));
            if (o->rec_status) HIP_TRY(hipMemcpy(o->rec_status, v.rec_status, N * 4, hipMemcpyDeviceToHost));
            if (o->rec_pos) HIP_TRY(hipMemcpy(o->rec_pos, v.rec_pos, 3 * N * 8, hipMemcpyDeviceToHost));
            if (o->rec_peel && p.n_cams)
                HIP_TRY(hipMemcpy(o->rec_peel, v.rec_peel, N * p.n_cams * 8, hipMemcpyDeviceToHost));
        }
    }
    return COLT_OK;
}

colt_status colt_eval_voigt(int32_t precision, const double *a, const double *x, int64_t n,
                            double *out, void *stream)
{
    if (n < 0 || (n > 0 && (!a || !x || !out))) return fail(COLT_ERR_ARG, "bad arrays");
    if (precision != 0 && precision != 1) return fail(COLT_ERR_ARG, "precision 0 or 1");
    if (n == 0) return COLT_OK;
    hipStream_t s = (hipStream_t)stream;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, 3 * n * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, a, n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d + n, x, n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_voigt(precision, n, d, d + n, d + 2 * n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d + 2 * n, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(COLT_ERR_HIP, "voigt check failed: %s", hipGetErrorString(e));
    return COLT_OK;
}

colt_status colt_sample(int32_t what, int32_t precision, double p0, double p1, double p2,
                        uint64_t seed, int64_t n, double *out, int32_t *draws, void *stream)
{
    const bool upar = what == 0 || what == 4 || what == 5 || what == 6;
    if (what < 0 || what > 7 || n < 0 || (n > 0 && !out) || (upar && n > 0 && !draws))
        return fail(COLT_ERR_ARG, "bad sampler request");
    if (precision != 0 && precision != 1) return fail(COLT_ERR_ARG, "precision 0 or 1");
    if (what == 3 && !(p0 >= 1.0 && p0 <= 4096.0)) return fail(COLT_ERR_ARG, "1..4096 draws");
    if (what == 7 && !(p0 >= 0.0 && p0 <= 4096.0)) return fail(COLT_ERR_ARG, "0..4096 skipped");
    if (n == 0) return COLT_OK;
    const int64_t per = (what == 1) ? 2 : ((what == 3) ? (int64_t)p0 : ((what == 7) ? 5 : 1));
    hipStream_t s = (hipStream_t)stream;
    double *d = nullptr;
    int32_t *dd = nullptr;
    HIP_TRY(hipMalloc(&d, n * per * sizeof(double)));
    hipError_t e = hipMalloc(&dd, n * sizeof(int32_t));
    if (e == hipSuccess) e = launch_sample(precision, what, p0, p1, p2, seed, n, d, dd, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, n * per * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && upar)
        e = hipMemcpyAsync(draws, dd, n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (dd) (void)hipFree(dd);
    if (e != hipSuccess) return fail(COLT_ERR_HIP, "sampler check failed: %s", hipGetErrorString(e));
    return COLT_OK;
}

}  // extern "C"
