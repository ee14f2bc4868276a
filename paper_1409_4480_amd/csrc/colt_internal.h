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

// Data only needed at scattering events: recoil parameter, non-local a*tau.
template <typename R>
struct alignas(2 * sizeof(R)) CellAux {
    R g, atau_nl;
};

struct GridView {
    int32_t kind;              // 0 Cartesian, 1 octree
    int32_t n[3];              // Cartesian cells per axis / octree base cells per axis
    const void *cells;         // CellRec<R>[n_cells] (leaf order for octrees)
    const void *aux;           // CellAux<R>[n_cells]
    const int32_t *child;      // octree: >= 0 first child, < 0 -(leaf + 1)
    const int32_t *base;       // octree: node at the base level per base cell
    const uint32_t *rope;      // octree: per leaf and face, the node across (see cross())
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
};

// One persistent launch: jobs[j] takes global queue indices
// [prefix[j], prefix[j+1]) as photon ids first_id[j] + (index - prefix[j]);
// prefix[n_jobs] is the number of photons of the launch.  The tables live in
// device memory, so a captured graph can re-plan them on every replay.
struct LaunchView {
    const JobView *jobs;
    const uint64_t *prefix;
    const uint64_t *first_id;
    unsigned long long *queue;
    int32_t n_jobs;
    int32_t march_min;          // a wave keeps stepping while this many lanes are in flight
};

// Device-side planning of a graph replay: each job takes up to `quota`
// photons from its cursor; the cursors advance after the transport.
struct PlanView {
    int32_t n_jobs, pad;
    uint64_t quota;
    const uint64_t *n_photons;
    uint64_t *cursor;
    uint64_t *prefix;
    uint64_t *first_id;
    unsigned long long *queue;
};

}  // namespace colt
