// Device-side views shared by the host runtime and the HIP kernels of the
// transport library.  Lengths are in grid units (one base cell = 1), with the
// origin at the lower box corner; frequencies in Doppler widths.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace colt {

constexpr double kVthRef = 12.85;          // km/s, thermal speed at 1e4 K (Sec. 2)
constexpr int kCounterSlots = 64;          // counter copies per job (spread atomics)
constexpr int kNumCounters = 16;
constexpr int kMaxCams = 64;
// Lanes per CU a transport launch may keep resident (the grid is clamped to
// it); it bounds the photons in flight, hence a job's suspended photons.
constexpr int kMaxLanesPerCU = 1024;
// Sub-buffers of a camera job's march-task buffer (spread append atomics).
constexpr int kTaskSubs = 32;
// Slots a lane reserves in a task sub-buffer at a time.
constexpr int kTaskChunk = 8;
// Host stop words (colt_stop_set tokens 1 .. kStopTokens-1).
constexpr int kStopTokens = 64;
// Completion events created with each job, so that launches on up to this many
// streams record them without creating any.
constexpr int kJobEvents = 4;
// The allocation-free launch path (colt_transport_static): jobs per launch and
// bytes of its per-device launch table.
constexpr int kStaticJobs = 64;
constexpr size_t kStaticTableBytes = 40960;
// Lanes in flight that keep a wave ray tracing (measured best on the 64^3
// dusty sphere: 16 of 64 lanes).
constexpr int kDefaultMarchMinFp32 = 16;
constexpr int kDefaultMarchMinFp64 = 16;

// Line data of one cell for the march: opacity at line centre per grid unit,
// damping parameter, v_ref / v_th, dust opacity per grid unit, bulk velocity
// in units of the cell's v_th, and the core-wing crossover frequency.
template <typename R>
struct alignas(8 * sizeof(R)) CellRec {
    R k0, a, s, kd;
    R ux, uy, uz, xcw;
};

// Data only needed at scattering events: recoil parameter, non-local a*tau,
// Jeans a*tau.
template <typename R>
struct alignas(4 * sizeof(R)) CellAux {
    R g, atau_nl, atau_j, pad;
};

// A photon between launches: its state at a pass boundary of the wave loop,
// where every live photon is in flight with its optical depth to go (128 B).
// The direction and frequency are kept in double for both precisions (FP32
// values convert exactly); the generator's cached words are recomputed from
// the draw index.
struct SuspRec {
    double r[3];
    double tau;
    double lo[3];
    double size;
    double k[3];
    double x;
    unsigned long long events, id, rng_k;
    int32_t cell, nscat;
};
static_assert(sizeof(SuspRec) == 128, "suspended photon record is one 128-byte line");

// Per-job control block in device memory.
struct JobCtl {
    unsigned long long cursor;      // next photon id not yet handed to a launch
    unsigned int n_in;              // suspended photons to resume, in susp[cur]
    unsigned int n_out;             // suspended by the running launch, in susp[cur ^ 1]
    unsigned int cur;
    unsigned int overflow;          // photons or march tasks that found no room (error)
    unsigned int pad[10];
    unsigned int tn[kTaskSubs * 16];   // march-task slots reserved per sub-buffer (64 B apart)
};

// Deferred next-event marches of a camera job, structure of arrays: a march
// starts at the event's position in the event's cell with zero optical depth.
// Slots whose cam is -1 are unused.
struct TaskSoA {
    double *rx, *ry, *rz;
    float *lox, *loy, *loz, *size;     // cell box in base-cell units (exact dyadics)
    int32_t *cell, *cam;
    void *xl, *W;                      // lab frequency and phase weight (R)
    unsigned long long *id;
};

struct GridView {
    int32_t kind;              // 0 Cartesian, 1 octree
    int32_t n[3];              // Cartesian cells per axis / octree base cells per axis
    int32_t rec_stride;        // cell records between consecutive cells (2: FP32 octree,
                               // whose leaf's links fill the second half of its 64-byte line)
    int32_t rope_stride;       // uint32 words between consecutive leaves' links (6 or 16)
    const void *cells;         // CellRec<R>[n_cells * rec_stride] (leaf order for octrees)
    const void *aux;           // CellAux<R>[n_cells]
    const int32_t *child;      // octree: >= 0 first child, < 0 -(leaf + 1)
    const int32_t *base;       // octree: node at the base level per base cell
    const uint32_t *rope;      // octree: per leaf and face, the leaf or node across (cross())
    double centre[3];          // box centre
    double esc_r;              // escape sphere radius (0 = box faces)
    double albedo;             // dust scattering probability per dust event
};

struct JobView {
    GridView g;
    // sources (Sec. 3.1.1)
    int32_t src_kind, n_src, freq_mode, pad0;
    const double *src_pos;     // 3 per source, grid units
    const double *src_cdf;     // cumulative weights
    double sigma;              // Gaussian width, grid units
    // physics options
    uint64_t seed, n_photons, max_events;
    int32_t xcrit_mode, recoil, isotropic, n_bins;
    double xcrit_global;
    float xcrit_global_f, pad1;     // the same in single precision (a scalar operand)
    double x_min, x_max;
    // next-event estimator (Sec. 6.1)
    int32_t n_cams, cam_nbins, npix, record;
    const double *cam;         // 12 per camera: direction, 1/direction, image u, image v
    double cam_xmin, cam_xmax, fov, tau_peel_max;
    // outputs (device)
    unsigned long long *spectrum;   // n_bins + 2
    double *cam_spec;               // n_cams * cam_nbins
    double *cam_img;                // n_cams * npix * npix
    unsigned long long *counters;   // kCounterSlots * kNumCounters
    double *rec_x;
    int32_t *rec_nscat;
    int32_t *rec_status;
    double *rec_pos;
    double *rec_peel;
    double dx_cm;                   // grid unit in cm (for recorded positions)
    double box_min_cm[3];
    // preemption and deferred marches
    JobCtl *ctl;
    SuspRec *susp[2];
    uint32_t susp_cap;              // records per suspend array
    uint32_t task_sub_cap;          // slots per task sub-buffer (0: no cameras)
    uint32_t task_hw;               // reserve beyond this in a sub-buffer: stop the launch
    uint32_t pad2;
    TaskSoA task;
};

// One persistent launch, planned on the device (k_plan) from the jobs'
// control blocks: jobs[j] resumes its suspended photons as resume indices
// [rprefix[j], rprefix[j+1]) and takes new photons as queue indices
// [prefix[j], prefix[j+1]), ids first_id[j] + (index - prefix[j]).  Resumes
// are handed out first (rqueue), then new photons (queue).  The tables live in
// device memory, so a captured graph re-plans them on every replay.
struct LaunchView {
    JobView *jobs;
    uint64_t *prefix;
    uint64_t *first_id;
    uint32_t *rprefix;
    unsigned long long *queue;
    unsigned long long *rqueue;
    unsigned int *stop_dev;     // set on the device (a task buffer near full)
    const int *stop_host;       // pinned host word (colt_stop_set), or null
    unsigned long long *peel_work;  // per job: march tasks handed out by k_peel
    uint64_t quota;             // new photons per job (0: all that remain)
    int32_t n_jobs;
    int32_t march_min;          // a wave keeps stepping while this many lanes are in flight
    int32_t tail_live;          // > 0: drained waves with fewer live photons suspend them
};

// A launch that starts with fewer photons (new and resumed) than this runs to
// the end whatever tail_live asks, so repeated launches always finish a job.
constexpr uint64_t kTailMinWork = 16384;

}  // namespace colt
