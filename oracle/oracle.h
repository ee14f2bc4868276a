/*
 * Plain FP64 CPU oracle of the Monte-Carlo Lyman-alpha transfer method of
 * Smith, Safranek-Shrader, Bromm & Milosavljevic (2014), "The Lyman-alpha
 * signature of the first galaxies" (arXiv:1409.4480).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP transport
 * library against the paper.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU path; the two agree only on the written
 * specification (units, draw order, tie rules) stated in the design notes.
 *
 * Everything is scalar double precision, written for readability: one photon
 * at a time, the steps of Sec. 3.1 (emission, ray tracing, scattering) with the
 * schemes of Sec. 3.2 (H(a,x) approximation, x_cw, the u_par sampler,
 * core-skipping) and the next-event estimator of Sec. 6.1.
 *
 * Units: lengths in cm, densities in cm^-3, temperatures in K, velocities in
 * km/s.  Frequencies are dimensionless x = (nu - nu0)/Delta nu_D.  A photon's
 * frequency is carried in the lab (grid) frame in units of the Doppler width
 * at T_ref = 1e4 K; the comoving frequency of a cell is derived from it.
 */
#ifndef COLT_ORACLE_H
#define COLT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Grid of cells with uniform (n_HI, T, v, k_dust) per cell (Sec. 3, intro). */
typedef struct {
    int32_t kind;              /* 0 = Cartesian, 1 = octree                          */
    int32_t nx, ny, nz;        /* Cartesian cell counts                              */
    double box_min[3];         /* cm                                                 */
    double box_max[3];         /* cm; cells (Cartesian) / root (octree) are cubes     */
    int64_t n_nodes;           /* octree node count (root = node 0)                  */
    const int32_t *child;      /* octree: first of 8 children (x fastest) or -1      */
    const double *n_HI;        /* per cell / node, cm^-3                             */
    const double *T;           /* per cell / node, K                                 */
    const double *v;           /* per cell / node, 3 interleaved, km/s; NULL = 0     */
    const double *k_dust;      /* per cell / node, cm^-1 extinction; NULL = 0        */
    const double *atau_nl;     /* per cell / node non-local a*tau estimate; NULL = 0 */
    double dust_albedo;        /* probability that a dust interaction scatters       */
    double escape_radius;      /* cm about the box centre; 0 = escape at box faces   */
} orc_grid;

typedef struct {
    int32_t kind;              /* 0 point, 1 Gaussian blob, 2 list of point sources   */
    int32_t n_src;
    const double *pos;         /* 3 * n_src, cm                                       */
    const double *weight;      /* n_src relative weights; NULL = equal                */
    double sigma;              /* Gaussian width (cm) for kind 1                      */
    int32_t freq_mode;         /* 0: comoving x = 0; 1: Lorentzian + thermal draw      */
} orc_source;

typedef struct {
    uint64_t n_photons;        /* photon ids 0 .. n_photons-1 form the job            */
    uint64_t id_begin, id_end; /* the oracle runs the id range [begin, end)           */
    uint64_t seed;
    int32_t xcrit_mode;        /* 0 off, 1 global a*tau0, 2 local a*tau_cell + NL,    */
                               /* 3 Jeans a*tau_J of the cell (eq. atau0J)            */
    double atau0;              /* for xcrit_mode 1                                    */
    int32_t recoil;            /* include the recoil term g (eq. x_f)                 */
    int32_t isotropic;         /* isotropic phase function instead of eq. phaseW       */
    int32_t n_bins;            /* escape spectrum in lab x over [x_min, x_max)        */
    double x_min, x_max;
    int32_t n_cams;            /* next-event estimator observers                      */
    const double *cam_dir;     /* 3 * n_cams unit vectors                             */
    int32_t cam_nbins;
    double cam_xmin, cam_xmax;
    int32_t cam_npix;          /* square images of cam_npix^2 pixels                   */
    double cam_fov;            /* cm, image side, centred on the box centre           */
    double tau_peel_max;       /* next-event march cut-off (Sec. 6.1 uses 50)         */
    uint64_t max_events;       /* stop a photon (status 3) after this many cell
                                  crossings plus interactions; 0 = no limit           */
} orc_params;

enum {
    ORC_EMITTED = 0, ORC_ESCAPED, ORC_ABSORBED, ORC_SCAT_HI, ORC_SCAT_DUST,
    ORC_CROSSINGS, ORC_PEELS, ORC_UPAR_TRIES, ORC_PEEL_CROSSINGS, ORC_CAPPED,
    ORC_N_COUNTERS = 16
};

typedef struct {
    double *spectrum;          /* n_bins + 2: [0] underflow, [1..n_bins], [n+1] over  */
    double *cam_spec;          /* n_cams * cam_nbins                                  */
    double *cam_img;           /* n_cams * cam_npix * cam_npix (row = v, col = u)     */
    uint64_t counters[ORC_N_COUNTERS];
    /* optional per-photon records indexed by (id - id_begin); NULL = off            */
    double *rec_x;             /* final lab x                                         */
    int32_t *rec_nscat;        /* executed HI scatterings                             */
    int32_t *rec_status;       /* 1 escaped, 2 absorbed, 3 stopped by max_events      */
    double *rec_pos;           /* 3 per photon, final position (cm)                   */
    double *rec_peel;          /* n_cams per photon, summed W exp(-tau)               */
    double *rec_len;           /* path length travelled from emission to the end (cm) */
    int32_t *rec_ndust;        /* dust scatterings                                    */
} orc_out;

/* Runs photons [id_begin, id_end) with n_threads worker threads; returns 0 or <0. */
int orc_run(const orc_grid *g, const orc_source *s, const orc_params *p, orc_out *o,
            int n_threads);

/* Non-local a*tau per cell (Sec. 3.2.4, eq. atauNL) with density threshold
 * f_NL; out has one entry per cell (Cartesian) or node (octree). */
void orc_nonlocal(const orc_grid *g, double f_nl, double *out);

/* Building blocks exported for the pin tests. */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint64_t seed, uint64_t photon, uint64_t k);
double orc_H(double a, double x);
double orc_xcw(double a);
double orc_xcrit(double atau0);
double orc_atau_jeans(double T, double n_HI);
void   orc_cell_constants(double T, double n_HI, double *a, double *sigma0, double *k0,
                          double *vth, double *xcw, double *g);
/* Samplers driven by the photon stream (seed, photon) starting at draw k;
 * each writes n samples and the number of uniforms consumed per sample. */
void orc_sample_upar(double a, double x, double xcw, uint64_t seed, int64_t n,
                     double *out, int32_t *draws);
double orc_sample_upar_one(double a, double x, double xcw, uint64_t seed, uint64_t photon,
                           int32_t *draws);
void orc_sample_uperp(double xcrit_eff, uint64_t seed, int64_t n, double *out2);
void orc_sample_mu(double rW, uint64_t seed, int64_t n, double *out);
double orc_upar_split(double a, double x, double xcw, double *u0);
/* x_crit of an H I scattering at r (moving along k, comoving frequency x) as
 * the transport computes it for the job's mode; -1 outside the domain. */
double orc_xcrit_at(const orc_grid *g, const orc_params *p, const double r[3],
                    const double k[3], double x);
/* One H I scattering as the transport performs it (stream (seed, photon) from
 * draw 0, gas at temperature T, core-skipping frequency xcrit as used). */
void orc_scatter_once(double T, double x, const double k_in[3], double xcrit, int recoil,
                      int isotropic, uint64_t seed, uint64_t photon, double *x_f,
                      double k_f[3], double *u_par);

#ifdef __cplusplus
}
#endif
#endif
