/*
 * colt.h -- C ABI of the MI355X Monte-Carlo Lyman-alpha transport library.
 *
 * The library transports photon packets through neutral hydrogen (and grey
 * dust) on Cartesian or octree grids, following the method of Smith,
 * Safranek-Shrader, Bromm & Milosavljevic (2014, arXiv:1409.4480):
 *   - optical-depth draws tau = -ln R against the Voigt profile (Sec. 3.1.2,
 *     eq. lnR) with H(a,x) from the appendix approximation (eq. AB);
 *   - cell-by-cell ray tracing with the bulk-velocity / temperature frequency
 *     transform between cells (Sec. 3.1.2);
 *   - scattering with the atom-velocity draw (parallel component by rejection,
 *     Sec. 3.2.3; perpendicular components Gaussian, Sec. 3.1.3), the phase
 *     function (eq. phaseW) and frequency redistribution with recoil (eq. x_f);
 *   - optional core-skipping (Sec. 3.2.4, eq. xcrit, eq. atau0min);
 *   - next-event (peel-off) tallies into camera spectra and images (Sec. 6.1,
 *     eq. SB), and the angle-averaged escape spectrum (Sec. 4).
 * Grey dust competes with H I at each interaction point; it is not part of the
 * paper's method and is an extension of this library.
 *
 * Conventions
 *   - Units: cm, cm^-3, K, km/s.  Frequencies are x = (nu - nu0)/Delta nu_D;
 *     spectra are binned in the lab-frame x measured in Doppler widths at
 *     T_ref = 1e4 K (v_th,ref = 12.85 km/s), positive towards the blue.
 *   - Every call returns a colt_status (0 = COLT_OK, < 0 = error); the message
 *     of the last error on the calling thread is colt_last_error().  No C++
 *     exception crosses this interface.
 *   - Descriptor and array arguments are HOST pointers, borrowed for the call
 *     only; data is copied to the device.  Handles are owned by the library
 *     until released.  Output buffers of colt_tally are owned by the caller.
 *   - Device memory of grids, jobs, launch tables and graphs comes from the
 *     allocator given to colt_init_grid (NULL = hipMalloc); the device checks
 *     at the end of this file allocate their temporaries with hipMalloc.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls are
 *     asynchronous on it unless stated otherwise.
 *   - Random numbers: photon i of a job draws uniform number k from
 *     Philox4x32-10 (Salmon et al. 2011) with key = job seed (64 bit) and
 *     counter = (block lo, block hi, i lo, i hi), one draw order per photon;
 *     results do not depend on launch shape, job batching, kernel variant or
 *     where a launch was stopped.
 *   - Preemption: a transport launch can stop at the end of a pass of its
 *     wave loop (colt_stop_set, or a camera job's next-event task buffer near
 *     full).  Photons in flight are then suspended in the job's device memory
 *     and the next launch of the job resumes them first; every photon's
 *     history and every tally equal those of an uninterrupted run.
 */
#ifndef COLT_H
#define COLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t colt_status;
#define COLT_OK          0
#define COLT_ERR_ARG    -1   /* invalid argument or descriptor                  */
#define COLT_ERR_NOMEM  -2   /* device allocation failed or budget exceeded     */
#define COLT_ERR_HIP    -3   /* a HIP runtime call failed                       */
#define COLT_ERR_STATE  -4   /* call not valid in the object's current state    */
#define COLT_ERR_BUSY   -5   /* work still in flight                            */

#define COLT_N_COUNTERS 16
/* counter slots of colt_tally_out.counters */
#define COLT_C_EMITTED        0
#define COLT_C_ESCAPED        1
#define COLT_C_ABSORBED       2
#define COLT_C_SCAT_HI        3   /* executed H I scatterings (core-skipped ones are not events) */
#define COLT_C_SCAT_DUST      4
#define COLT_C_CROSSINGS      5   /* cell crossings of the transport march           */
#define COLT_C_PEELS          6   /* next-event evaluations (event x camera)          */
#define COLT_C_UPAR_TRIES     7   /* candidate draws of the u_par rejection sampler   */
#define COLT_C_PEEL_CROSSINGS 8   /* cell crossings of next-event marches             */
#define COLT_C_CAPPED         9   /* photons stopped by the per-photon event cap      */
#define COLT_C_UPAR_ROUNDS   10   /* cooperative u_par rounds, summed over waves      */
#define COLT_C_PASSES        11   /* transport-loop passes, summed over waves         */

typedef struct colt_grid_s *colt_grid;
typedef struct colt_job_s *colt_job;
typedef struct colt_graph_s *colt_graph;

/* Device allocator (e.g. a framework's caching allocator).  alloc returns a
 * device pointer of at least `bytes` bytes, 256-byte aligned, or NULL. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} colt_allocator;

/* Gas on a grid of cells of uniform density, temperature and bulk velocity
 * (Sec. 3, introduction: initial conditions of v, n, T for each cell of a 3-D
 * grid with adaptive refinement).
 * kind 0 (Cartesian): nx*ny*nz cells, index (k*ny + j)*nx + i, x fastest.
 *   Cells must be cubes: (box_max-box_min)/n equal on all axes.
 * kind 1 (octree): n_cells nodes; node 0 is the root spanning the (cubic)
 *   box; child[i] is the index of the first of node i's eight children, or -1
 *   for a leaf; child c + o holds octant o = ox + 2 oy + 4 oz.  Field arrays
 *   have one entry per node; entries of internal nodes are ignored.
 * Photons escape at the box faces, or at the sphere of radius escape_radius
 * about the box centre when escape_radius > 0. */
typedef struct {
    int32_t kind;
    int32_t nx, ny, nz;
    double box_min[3], box_max[3];        /* cm                                   */
    int64_t n_cells;                      /* Cartesian: nx*ny*nz; octree: nodes   */
    const int32_t *child;                 /* octree only                          */
    const double *n_HI;                   /* cm^-3                                */
    const double *T;                      /* K, > 0                               */
    const double *v;                      /* km/s, 3 per cell interleaved; NULL=0 */
    const double *k_dust;                 /* cm^-1 grey extinction; NULL = none   */
    const double *atau_nl;                /* non-local a*tau per cell; NULL = 0   */
    double dust_albedo;                   /* scattering probability per dust event */
    double escape_radius;                 /* cm; 0 = box faces                    */
} colt_grid_desc;

/* Photon sources (Sec. 3.1.1).  kind 0: point at pos[0]; kind 1: Gaussian
 * blob of width sigma about pos[0]; kind 2: n_src points chosen with
 * probability proportional to weight (NULL = equal).  freq_mode 0 emits at
 * comoving line centre x = 0; freq_mode 1 draws x = x_nat + k.u_atom with a
 * Lorentzian x_nat and a thermal atom velocity (eq. init_freq). */
typedef struct {
    int32_t kind;
    int32_t n_src;
    const double *pos;                    /* 3*n_src, cm                          */
    const double *weight;                 /* n_src or NULL                        */
    double sigma;                         /* cm (kind 1)                          */
    int32_t freq_mode;
} colt_source_desc;

#define COLT_FP64      0   /* all arithmetic in double precision                */
#define COLT_FP32_BULK 1   /* Voigt, sampling, directions in float; position,   */
                           /* optical depth and tallies in double              */

typedef struct {
    uint64_t n_photons;
    uint64_t seed;
    int32_t precision;                    /* COLT_FP64 or COLT_FP32_BULK          */
    int32_t xcrit_mode;                   /* 0 off; 1 global: x_crit(atau0);      */
                                          /* 2 local: a tau_cell + atau_nl[cell]; */
                                          /* 3 Jeans: a tau_J of the cell         */
    double atau0;                         /* a*tau0 for xcrit_mode 1              */
    int32_t recoil;                       /* recoil term g(mu - 1) of eq. x_f     */
    int32_t isotropic;                    /* 1: isotropic H I scattering          */
    int32_t n_bins;                       /* escape spectrum bins over [x_min,x_max) */
    double x_min, x_max;
    int32_t n_cams;                       /* next-event observers (<= 64)         */
    const double *cam_dir;                /* 3*n_cams unit vectors (host)         */
    int32_t cam_nbins;
    double cam_xmin, cam_xmax;
    int32_t cam_npix;                     /* images of cam_npix^2 pixels          */
    double cam_fov;                       /* cm, image side about the box centre  */
    double tau_peel_max;                  /* next-event cut-off (paper: 50)       */
    int32_t record;                       /* 1: keep per-photon records           */
    uint64_t max_events;                  /* per-photon event cap; 0 = 2^62       */
    uint64_t march_tasks;                 /* next-event task slots (cameras); 0 = */
                                          /* sized from n_photons and n_cams      */
} colt_job_params;

/* Launch shape of colt_transport; NULL or zero fields take defaults. */
typedef struct {
    int32_t block;                        /* threads per workgroup: 64, 128, 192  */
                                          /* or 256 (0 = 256)                     */
    int32_t blocks_per_cu;                /* resident workgroups per CU (grid size) */
    uint64_t photons_per_job;             /* photons taken from each job per call; */
                                          /* 0 = all that remain                   */
    int32_t time_kernel;                  /* 1: time the transport kernel with    */
                                          /* events (see colt_last_kernel_ms)      */
    int32_t march_min;                    /* a wave keeps ray tracing while at     */
                                          /* least this many of its 64 lanes are   */
                                          /* in flight (with fewer than 64 live    */
                                          /* photons, a quarter of them); 0 =      */
                                          /* default (16), 1 = every flight ends   */
                                          /* within its pass                       */
    int32_t stop_token;                   /* 1..63: the launch stops when          */
                                          /* colt_stop_set(token, 1); 0 = none     */
    int32_t tail_live;                    /* 0 = off; 1..64: once a launch has     */
                                          /* handed out all its photons, a wave    */
                                          /* with fewer live photons suspends them */
                                          /* and exits, so the last long histories */
                                          /* of a job do not hold the device; a    */
                                          /* later launch resumes them in full     */
                                          /* waves.  A launch that starts with     */
                                          /* fewer than 16384 photons runs to the  */
                                          /* end.                                  */
    int32_t launches;                     /* launch sequences the call enqueues    */
                                          /* (0 = 1), each planned on the device   */
                                          /* from the jobs' control blocks; one    */
                                          /* that finds nothing left returns at    */
                                          /* once                                  */
} colt_launch;

typedef struct {
    double *spectrum;     /* n_bins + 2 photon counts: [0] below x_min,           */
                          /* [1..n_bins] bins, [n_bins+1] at or above x_max       */
    double *cam_spec;     /* n_cams * cam_nbins, sum of W exp(-tau)                */
    double *cam_img;      /* n_cams * npix * npix, row v, column u                 */
    uint64_t counters[COLT_N_COUNTERS];
    /* per-photon records (job created with record = 1; NULL skips a field)    */
    double *rec_x;        /* n_photons, final lab-frame x                          */
    int32_t *rec_nscat;   /* n_photons, H I scatterings                            */
    int32_t *rec_status;  /* n_photons, 1 escaped, 2 absorbed, 3 capped            */
    double *rec_pos;      /* 3*n_photons, final position (cm)                      */
    double *rec_peel;     /* n_photons*n_cams, summed W exp(-tau) per camera        */
} colt_tally_out;

/* Copies the gas of `desc` to the device and derives per-cell line
 * quantities (Sec. 2: v_th, a, sigma_0; Sec. 3.2.2: x_cw; eq. recoil_parameter)
 * with a device kernel on `stream`.  The descriptor arrays may be reused on
 * return.  Errors: COLT_ERR_ARG (bad shape, non-cubic cells, malformed
 * octree), COLT_ERR_NOMEM, COLT_ERR_HIP. */
colt_status colt_init_grid(const colt_grid_desc *desc, const colt_allocator *alloc,
                           void *stream, colt_grid *out);

/* Computes the non-local a*tau estimate of every cell on the device (Sec.
 * 3.2.4, eq. atauNL): six coordinate-axis paths start at the centres of the
 * cell's faces and run outward, summing a * tau0 = a n_HI sigma0 l over the
 * cells crossed while |n_HI - n_HI,start| < f_nl n_HI,start (stopping at the
 * domain edge); the estimate is the smallest sum.  It replaces the grid's
 * aτ_NL array, which local core-skipping adds to a tau_cell.  f_nl = 0 gives
 * zeros.  Synchronous on `stream`.  Errors: COLT_ERR_ARG (f_nl < 0),
 * COLT_ERR_STATE (jobs registered on the grid), COLT_ERR_HIP. */
colt_status colt_grid_nonlocal(colt_grid grid, double f_nl, void *stream);

/* Registers a transfer job on a grid: the emission of Sec. 3.1.1 (sources,
 * N_ph photon packets of equal weight, each with an isotropic direction and
 * the frequency of eq. init_freq or x = 0), the physics options of Secs.
 * 3.1.3 and 3.2.4 (recoil, phase function, core-skipping mode) and the tally
 * layout of Sec. 6.1 (observers, spectral and image bins).  Photon i is
 * generated lazily by the transport from (seed, i).  Allocates and zeroes the
 * job's device tallies, its control block, two suspend arrays of min(N_ph,
 * resident lanes) records and, with cameras, its next-event task buffer, on
 * the grid's stream.  The job keeps a reference to the grid.  `src` and `p`
 * are borrowed for the call.
 * Errors: COLT_ERR_ARG (invalid option or source), COLT_ERR_NOMEM, COLT_ERR_HIP. */
colt_status colt_emit(colt_grid grid, const colt_source_desc *src,
                      const colt_job_params *params, colt_job *out);

/* Transports photons of n_jobs jobs in one persistent launch per precision
 * mode on `stream` (asynchronous): each photon is traced cell by cell against
 * its optical depth drawn by eq. lnR, with the Doppler and temperature
 * frequency transform between cells (Sec. 3.1.2), and scatters off H I with
 * the atom velocity of Secs. 3.1.3 and 3.2.3, the phase function eq. phaseW,
 * the redistribution eq. x_f and core-skipping (Sec. 3.2.4), or off grey dust,
 * until it escapes or is absorbed; every event adds its next-event estimate
 * for each camera (Sec. 6.1).  Each job first resumes its suspended photons,
 * then contributes its next `photons_per_job` new photons (all remaining if
 * 0); lanes that finish a photon take the next one from a shared queue, so
 * jobs of uneven cost share the device.  The launch is planned on the device
 * from each job's control block.  A launch may stop early (stop_token, or a
 * camera job's task buffer near full, or tail_live): its photons in flight are
 * suspended and colt_job_status reports the job unfinished until a later
 * launch completes it.  A launch that can stop, and any launch of a job a stopped launch may
 * have left unfinished, waits for the job's launches on other streams.  `jobs`
 * is borrowed for the call.  Errors: COLT_ERR_ARG (list, block, token or a
 * task buffer too small for one wave), COLT_ERR_NOMEM (launch table),
 * COLT_ERR_HIP. */
colt_status colt_transport(const colt_job *jobs, int32_t n_jobs, const colt_launch *launch,
                           void *stream);

/* colt_transport for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, but nothing is allocated.  The launch table lives in a
 * fixed device array of 40 KB that each GPU holds until the process ends
 * (found once per device on the first call); job views reach it through
 * kernel arguments.  Limits: at most 64 jobs of one precision per call; a job
 * may be launched this way on at most 4 streams (the completion events made
 * with the job); stop_token only once colt_stop_set has been called;
 * time_kernel is ignored.  Every call on one GPU shares its table, which keeps
 * the last call's contents: calls that overlap on one GPU (other streams, not
 * yet complete) race, so order them on one stream or synchronise.  Errors as
 * colt_transport, plus COLT_ERR_ARG (more than 64 jobs) and COLT_ERR_STATE
 * (a fifth stream, or stop words not yet made). */
colt_status colt_transport_static(const colt_job *jobs, int32_t n_jobs,
                                  const colt_launch *launch, void *stream);

/* Sets (value != 0) or clears the stop word `token` (1..63).  Transport
 * launches started with that stop_token stop within about 32 passes of their
 * wave loop, suspending their photons in flight; a launch started while the
 * word is set does one pass and stops.  Errors: COLT_ERR_ARG, COLT_ERR_NOMEM. */
colt_status colt_stop_set(int32_t token, int32_t value);

/* Captures one transport epoch over n_jobs jobs (one precision) into a HIP
 * graph: a planning kernel takes up to photons_per_job photons (all if 0) from
 * each job's device-side cursor, the persistent transport kernel runs them,
 * and a second kernel advances the cursors.  Every colt_graph_launch replays
 * one epoch, so repeated launches walk through the jobs without host work
 * beyond the launch; replays after a job is complete do nothing for it.
 * Capture needs a non-default stream.  The jobs must outlive the graph and
 * must not be passed to colt_transport while the graph is in use.
 * Errors: COLT_ERR_ARG, COLT_ERR_NOMEM, COLT_ERR_HIP. */
colt_status colt_graph_create(const colt_job *jobs, int32_t n_jobs, const colt_launch *launch,
                              void *capture_stream, colt_graph *out);
/* Replays one epoch on `stream` (asynchronous). */
colt_status colt_graph_launch(colt_graph graph, void *stream);
void colt_graph_release(colt_graph graph);

/* Copies a job's tallies to caller buffers (sizes from its params): the
 * angle-averaged escape spectrum of Sec. 4 (photon counts per lab-frame
 * frequency bin, with under- and overflow), each camera's spectrum and
 * orthographic image of summed W exp(-tau_esc) (Sec. 6.1, eq. SB: multiply by
 * L/(4 pi N_ph d_L^2 Omega_pix) for surface brightness), the event counters
 * and, for record = 1 jobs, the per-photon records.  With wait = 1 it first
 * waits for every launch of the job (on every stream); with wait = 0 it
 * returns COLT_ERR_BUSY if any is still running.  Tallies of a job with
 * suspended photons cover the work done so far.  Errors: COLT_ERR_ARG,
 * COLT_ERR_BUSY, COLT_ERR_STATE (suspended photons or next-event marches
 * found no room: the results are incomplete), COLT_ERR_HIP. */
colt_status colt_tally(colt_job job, colt_tally_out *out, int32_t wait);

/* Photons taken by transport and not suspended (*launched), and the job's
 * total; the job is complete once every launch has ended and *launched ==
 * *total.  Exact without waiting unless a launch that can stop ran since the
 * last call; then it waits for the job's launches. */
colt_status colt_job_status(colt_job job, uint64_t *launched, uint64_t *total);

/* Unfinished photons of a job (waits for its launches): ids >= *next_id were
 * never started, and *n_suspended photons wait to resume; their ids (up to
 * ids_cap of them, sorted) go to `ids` when it is not NULL. */
colt_status colt_job_pending(colt_job job, uint64_t *next_id, uint64_t *n_suspended,
                             uint64_t *ids, uint64_t ids_cap);

/* Device bytes held by a grid or a job (for admission control). */
size_t colt_grid_bytes(colt_grid grid);
size_t colt_job_bytes(colt_job job);
/* Device bytes colt_emit would allocate for a job with these parameters and
 * n_src sources (0 for invalid arguments); exact for the library's own
 * allocations, before the allocator's rounding. */
size_t colt_job_footprint(const colt_job_params *p, int32_t n_src);

/* Duration in ms of the last transport kernel launched with time_kernel = 1
 * on the calling thread (synchronises on its end event); < 0 if none. */
double colt_last_kernel_ms(void);

void colt_release_job(colt_job job);
/* COLT_ERR_STATE if jobs still reference the grid. */
colt_status colt_release_grid(colt_grid grid);
const char *colt_last_error(void);

/* ---- device checks of the building blocks (host arrays in and out) ---- */

/* Per-cell derived fields as computed on the device, 11 doubles per cell:
 * k0 (cm^-1), a, v_th (km/s), u_x, u_y, u_z (bulk velocity / v_th),
 * k_dust (cm^-1), x_cw, g, atau_nl, atau_J (eq. atau0J). */
colt_status colt_grid_fields(colt_grid grid, double *out);

/* The neighbour links the library builds for an octree grid (host only, no
 * device use), for inspection.  child is the grid's node table as given to
 * colt_init_grid (-1 for a leaf); leaves are numbered in node order.  For leaf
 * j and face f = 2 axis + (step > 0), links[6 j + f] is
 *   0xFFFFFFFF                   the face is the domain edge;
 *   0xFFFFFFFE                   no link (a crossing there searches the tree);
 *   0x80000000 | up << 27 | l    leaf l lies across, up levels coarser;
 *   n                            node n lies across at the leaf's own level and
 *                                is refined (a crossing descends into it).
 * The point across is the first finest-level cell beyond the face at the
 * leaf's lowest corner.  links == NULL only reports n_leaves; otherwise it
 * holds 6 n_leaves entries, owned by the caller.  COLT_ERR_ARG for an invalid
 * tree (as colt_init_grid). */
colt_status colt_octree_links(const int32_t *child, int64_t n_nodes, uint32_t *links,
                              int64_t *n_leaves);

/* H(a, x) (eq. AB) evaluated on the device in the given precision. */
colt_status colt_eval_voigt(int32_t precision, const double *a, const double *x, int64_t n,
                            double *out, void *stream);

/* Draws n samples of one sampler on the device; sample i uses photon stream
 * (seed, i) from its first draw, exactly as in transport.
 *   what 0: u_par for (a = p0, x = p1, x_cw = p2) with the wave-cooperative
 *           sampler used in transport      out[n], draws[n] = draw index after
 *   what 1: u_perp pair with cut-off p0              out[2n]
 *   what 2: mu for W ~ 1 + p0 mu^2                    out[n]
 *   what 3: uniform numbers (k = 0 .. p0-1 of stream i) out[n*p0]
 *   what 4: as 0 with x_i = p1 + 0.41 (i mod 23) (-1)^i (mixed requests in a wave)
 *   what 5: as 0 with the one-lane sequential sampler
 *   what 6: as 4 with the one-lane sequential sampler
 *   what 7: after p0 single draws (0..4096), the five draws of a scattering
 *           (u_perp pair, mu, phi, next tau) as transport takes them: in FP32
 *           from a block boundary its two generator blocks are computed
 *           together; equal to draws p0 .. p0+4 of what 3  out[5n] */
colt_status colt_sample(int32_t what, int32_t precision, double p0, double p1, double p2,
                        uint64_t seed, int64_t n, double *out, int32_t *draws, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* COLT_H */
