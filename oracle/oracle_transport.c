/*
 * Oracle transport: one photon at a time through emission (Sec. 3.1.1), ray
 * tracing (Sec. 3.1.2), scattering (Sec. 3.1.3 with the schemes of Sec. 3.2)
 * and the next-event estimator (Sec. 6.1, eq. SB).  Dust is an extra grey
 * opacity competing with H I at each interaction point.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Pins: every step is checked against a closed form, a limit or an exact
 * invariant in the tests (dust at any albedo through the coupling of its
 * histories to the albedo-1 ones; bulk flows through Galilean invariance, the
 * unscattered Doppler shift and the expanding sphere's mirror symmetry).  The
 * wind and turbulent workloads have no spectra in the paper to compare with,
 * but every function they exercise is among those pinned.
 *
 * Draw order of one photon's stream (the written contract both
 * implementations follow):
 *   emission : [source choice if n_src > 1] [4 for a Gaussian blob offset]
 *              mu, phi, [x_nat, 4 for the atom velocity if freq_mode = 1], tau
 *   per event: [dust R if k_dust > 0] then
 *              dust   : [albedo R], mu, phi, tau
 *              H I    : u_par draws, u_perp R1 R2, mu, phi, tau
 */
#include "oracle.h"
#include "oracle_internal.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Per-cell quantities derived once from (n_HI, T, v, k_dust) (Sec. 2), with
 * the non-local and Jeans a*tau of Sec. 3.2.4. */
typedef struct {
    double *a, *k0, *vth, *xcw, *g, *kd, *v, *atau_nl, *atau_j;
} orc_cells;

static int64_t n_cells_of(const orc_grid *g)
{
    return (g->kind == 0) ? (int64_t)g->nx * g->ny * g->nz : g->n_nodes;
}

static void cells_init(const orc_grid *g, orc_cells *C)
{
    int64_t nc = n_cells_of(g);
    C->a = calloc(nc, sizeof(double));   C->k0 = calloc(nc, sizeof(double));
    C->vth = calloc(nc, sizeof(double)); C->xcw = calloc(nc, sizeof(double));
    C->g = calloc(nc, sizeof(double));   C->kd = calloc(nc, sizeof(double));
    C->v = calloc(3 * nc, sizeof(double)); C->atau_nl = calloc(nc, sizeof(double));
    C->atau_j = calloc(nc, sizeof(double));
    for (int64_t i = 0; i < nc; ++i) {
        double sigma0;
        orc_cell_constants(g->T[i], g->n_HI[i], &C->a[i], &sigma0, &C->k0[i], &C->vth[i],
                           &C->xcw[i], &C->g[i]);
        C->kd[i] = g->k_dust ? g->k_dust[i] : 0.0;
        C->atau_nl[i] = g->atau_nl ? g->atau_nl[i] : 0.0;
        C->atau_j[i] = orc_atau_jeans(g->T[i], g->n_HI[i]);
        for (int d = 0; d < 3; ++d) C->v[3 * i + d] = g->v ? g->v[3 * i + d] : 0.0;
    }
}

static void cells_free(orc_cells *C)
{
    free(C->a); free(C->k0); free(C->vth); free(C->xcw); free(C->g); free(C->kd);
    free(C->v); free(C->atau_nl); free(C->atau_j);
}

typedef struct {
    double *spectrum, *cam_spec, *cam_img;
    uint64_t counters[ORC_N_COUNTERS];
} orc_tally;

typedef struct {
    const orc_grid *g;
    const orc_source *s;
    const orc_params *p;
    orc_out *o;
    orc_cells cells;
    double centre[3];
    double cam_eu[3 * 64], cam_ev[3 * 64];
    double *src_cdf;
    uint64_t next;              /* next photon id to hand out */
    pthread_mutex_t lock;
    orc_tally *tallies;
} orc_job;

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Comoving frequency in a cell from the lab frequency x_lab (units of the
 * Doppler width at 1e4 K): the cell-to-cell rule of Sec. 3.1.2 written against
 * a fixed reference frame, x = (x_lab v_ref - k.v) / v_th. */
static double comoving_x(const orc_cells *C, int64_t c, double x_lab, const double k[3])
{
    const double *v = &C->v[3 * c];
    return (x_lab * ORC_VTH_REF - (k[0] * v[0] + k[1] * v[1] + k[2] * v[2])) / C->vth[c];
}

static double lab_x(const orc_cells *C, int64_t c, double x, const double k[3])
{
    const double *v = &C->v[3 * c];
    return (x * C->vth[c] + (k[0] * v[0] + k[1] * v[1] + k[2] * v[2])) / ORC_VTH_REF;
}

static int bin_of(double x, double lo, double hi, int n)
{
    if (x < lo) return 0;
    double t = (x - lo) / (hi - lo) * n;
    if (t >= n) return n + 1;
    return 1 + (int)t;
}

/* Optical depth from r along direction d to the domain edge for a photon of
 * lab frequency x_lab; returns -1 once it exceeds tau_max (Sec. 6.1). */
static double peel_tau(const orc_job *J, orc_cell c, const double r0[3], const double d[3],
                       double x_lab, orc_tally *T)
{
    const orc_grid *g = J->g;
    double r[3] = { r0[0], r0[1], r0[2] };
    double tau = 0.0;
    for (;;) {
        int axis, by_sphere;
        double l = orc_exit_distance(g, &c, r, d, &axis, &by_sphere);
        double x = comoving_x(&J->cells, c.id, x_lab, d);
        double kt = J->cells.k0[c.id] * orc_H(J->cells.a[c.id], x) + J->cells.kd[c.id];
        tau += kt * l;
        T->counters[ORC_PEEL_CROSSINGS] += 1;
        if (tau > J->p->tau_peel_max) return -1.0;
        if (by_sphere) return tau;
        for (int e = 0; e < 3; ++e) r[e] += l * d[e];
        if (!orc_cross(g, &c, r, d, axis)) return tau;
    }
}

/* Adds one next-event contribution for every camera: phase weight W toward
 * the camera times exp(-tau_esc), binned in lab frequency and projected
 * position.  xcam[i] is the comoving frequency the photon would have toward
 * camera i. */
static void peel_off(const orc_job *J, const orc_cell *c, const double r[3],
                     const double *xcam, const double *W, orc_tally *T, double *rec_peel)
{
    const orc_params *p = J->p;
    for (int i = 0; i < p->n_cams; ++i) {
        const double *d = &p->cam_dir[3 * i];
        double x_lab = lab_x(&J->cells, c->id, xcam[i], d);
        T->counters[ORC_PEELS] += 1;
        double tau = peel_tau(J, *c, r, d, x_lab, T);
        if (tau < 0.0) continue;
        double w = W[i] * exp(-tau);
        if (rec_peel) rec_peel[i] += w;
        int b = bin_of(x_lab, p->cam_xmin, p->cam_xmax, p->cam_nbins);
        if (b >= 1 && b <= p->cam_nbins)
            T->cam_spec[(size_t)i * p->cam_nbins + (b - 1)] += w;
        double rc[3] = { r[0] - J->centre[0], r[1] - J->centre[1], r[2] - J->centre[2] };
        double pu = dot3(rc, &J->cam_eu[3 * i]) / p->cam_fov + 0.5;
        double pv = dot3(rc, &J->cam_ev[3 * i]) / p->cam_fov + 0.5;
        if (pu >= 0.0 && pu < 1.0 && pv >= 0.0 && pv < 1.0) {
            int iu = (int)(pu * p->cam_npix), iv = (int)(pv * p->cam_npix);
            if (iu >= p->cam_npix) iu = p->cam_npix - 1;
            if (iv >= p->cam_npix) iv = p->cam_npix - 1;
            T->cam_img[((size_t)i * p->cam_npix + iv) * p->cam_npix + iu] += w;
        }
    }
}

static void isotropic_dir(orc_stream *s, double k[3])
{
    double mu = 2.0 * orc_draw(s) - 1.0;
    double phi = 2.0 * ORC_PI * orc_draw(s);
    double st = sqrt(1.0 - mu * mu);
    k[0] = st * cos(phi); k[1] = st * sin(phi); k[2] = mu;
}

/* Core-skipping frequency at an H I scattering (Sec. 3.2.4): eq. xcrit of the
 * a*tau0 the job's mode names -- 1: the job's global value; 2: the local
 * a*tau_cell of eq. atau0min, with l_cell the shortest distance from the
 * scattering point to the boundary of its cell, plus the cell's non-local
 * estimate (eq. atauNL); 3: the Jeans estimate of eq. atau0J from the cell's
 * density and temperature -- and no cut-off for a photon already in the wing
 * (|x| >= x_cw). */
static double event_xcrit(const orc_params *p, const orc_cells *C, int64_t ci,
                          const orc_cell *c, const double r[3], double x)
{
    double xcrit = 0.0;
    if (p->xcrit_mode == 1) {
        xcrit = orc_xcrit(p->atau0);
    } else if (p->xcrit_mode == 2) {
        double l_cell = orc_min_face_distance(c, r);
        xcrit = orc_xcrit(C->a[ci] * C->k0[ci] * l_cell + C->atau_nl[ci]);
    } else if (p->xcrit_mode == 3) {
        xcrit = orc_xcrit(C->atau_j[ci]);
    }
    if (fabs(x) >= C->xcw[ci]) xcrit = 0.0;
    return xcrit;
}

/* What one H I scattering leaves: the parallel atom velocity, the atom
 * velocity vector, the phase-function parameter r_W used, the new direction
 * and the redistributed comoving frequency. */
typedef struct {
    double u_par, u_atom[3], rW, kf[3], x_f;
    int64_t tries;
} orc_scatter;

/* One H I scattering (Sec. 3.1.3) of a photon of comoving frequency x moving
 * along k in a cell with damping a, crossover x_cw and recoil parameter g_rec
 * (0 when recoil is off): u_par by rejection (Sec. 3.2.3), the perpendicular
 * components truncated below xcrit (Sec. 3.2.4), the direction from the phase
 * function of eq. phaseW about k (core mixture for |x| < x_cw, wing dipole
 * otherwise, or isotropic), and x_f of eq. x_f.  Draw order: u_par, u_perp
 * (2), mu, phi. */
static void scatter_hi(double a, double xcw, double g_rec, double xcrit, int isotropic,
                       double x, const double k[3], orc_stream *st, orc_scatter *o)
{
    o->tries = 0;
    o->u_par = orc_draw_upar(a, x, xcw, st, &o->tries);
    double u1, u2;
    orc_draw_uperp(xcrit, st, &u1, &u2);
    double e1[3], e2[3];
    orc_perp_basis(k, e1, e2);
    for (int d = 0; d < 3; ++d) o->u_atom[d] = o->u_par * k[d] + u1 * e1[d] + u2 * e2[d];
    o->rW = isotropic ? 0.0 : ((fabs(x) < xcw) ? 3.0 / 11.0 : 1.0);
    double mu = orc_draw_mu(o->rW, st);
    double phi = 2.0 * ORC_PI * orc_draw(st);
    double st_ = sqrt(1.0 - mu * mu);
    for (int d = 0; d < 3; ++d)
        o->kf[d] = mu * k[d] + st_ * (cos(phi) * e1[d] + sin(phi) * e2[d]);
    double nk = sqrt(dot3(o->kf, o->kf));
    for (int d = 0; d < 3; ++d) o->kf[d] /= nk;
    o->x_f = x - o->u_par + dot3(o->kf, o->u_atom) + g_rec * (mu - 1.0);   /* eq. x_f */
}

static void run_photon(orc_job *J, uint64_t id, orc_tally *T)
{
    const orc_grid *g = J->g;
    const orc_source *S = J->s;
    const orc_params *p = J->p;
    orc_out *o = J->o;
    const orc_cells *C = &J->cells;
    orc_stream st = { p->seed, id, 0 };
    uint64_t slot = id - p->id_begin;
    double *rec_peel = o->rec_peel ? &o->rec_peel[slot * p->n_cams] : NULL;
    double xcam[64], W[64];

    /* ---- emission (Sec. 3.1.1) ---- */
    int src = 0;
    if (S->n_src > 1) {
        double R = orc_draw(&st);
        while (src < S->n_src - 1 && R > J->src_cdf[src]) ++src;
    }
    double r[3] = { S->pos[3 * src], S->pos[3 * src + 1], S->pos[3 * src + 2] };
    if (S->kind == 1) {                         /* Gaussian blob: N(0, sigma^2) offsets */
        double R1 = orc_draw(&st), R2 = orc_draw(&st), R3 = orc_draw(&st), R4 = orc_draw(&st);
        double q1 = sqrt(-2.0 * log(R1)), q2 = sqrt(-2.0 * log(R3));
        r[0] += S->sigma * q1 * cos(2.0 * ORC_PI * R2);
        r[1] += S->sigma * q1 * sin(2.0 * ORC_PI * R2);
        r[2] += S->sigma * q2 * cos(2.0 * ORC_PI * R4);
    }
    double k[3];
    isotropic_dir(&st, k);
    T->counters[ORC_EMITTED] += 1;
    orc_cell c;
    int32_t nscat = 0;
    int status;
    double x_lab = 0.0;
    double path = 0.0;                          /* distance travelled (record only) */
    int32_t ndust = 0;                          /* dust scatterings (record only) */
    if (!orc_locate(g, r, k, &c)) {             /* born outside the domain: escapes */
        status = 1;
        T->counters[ORC_ESCAPED] += 1;
        goto done;
    }
    {
        double x = 0.0, u_atom[3] = { 0.0, 0.0, 0.0 };
        if (S->freq_mode == 1) {                /* eq. init_freq */
            double a = C->a[c.id];
            double x_nat = a * tan(ORC_PI * (orc_draw(&st) - 0.5));
            double R1 = orc_draw(&st), R2 = orc_draw(&st), R3 = orc_draw(&st), R4 = orc_draw(&st);
            double q1 = sqrt(-log(R1)), q2 = sqrt(-log(R3));
            u_atom[0] = q1 * cos(2.0 * ORC_PI * R2);
            u_atom[1] = q1 * sin(2.0 * ORC_PI * R2);
            u_atom[2] = q2 * cos(2.0 * ORC_PI * R4);
            x = x_nat + dot3(k, u_atom);
            for (int i = 0; i < p->n_cams; ++i)
                xcam[i] = x_nat + dot3(&p->cam_dir[3 * i], u_atom);
        } else {
            for (int i = 0; i < p->n_cams; ++i) xcam[i] = 0.0;
        }
        x_lab = lab_x(C, c.id, x, k);
        for (int i = 0; i < p->n_cams; ++i) W[i] = 1.0;
        if (p->n_cams > 0) peel_off(J, &c, r, xcam, W, T, rec_peel);
    }
    double tau = -log(orc_draw(&st));           /* eq. lnR */

    /* ---- ray tracing and scattering ---- */
    uint64_t events = 0;
    const uint64_t cap = p->max_events ? p->max_events : UINT64_MAX;
    for (;;) {
        int64_t ci = c.id;
        double x = comoving_x(C, ci, x_lab, k);
        int axis, by_sphere;
        double l_exit = orc_exit_distance(g, &c, r, k, &axis, &by_sphere);
        double k_HI = C->k0[ci] * orc_H(C->a[ci], x);
        double k_tot = k_HI + C->kd[ci];
        double tau_cell = k_tot * l_exit;
        if (tau > tau_cell) {                   /* leave the cell with tau spent */
            tau -= tau_cell;
            for (int d = 0; d < 3; ++d) r[d] += l_exit * k[d];
            path += l_exit;
            T->counters[ORC_CROSSINGS] += 1;
            if (++events >= cap) { status = 3; break; }
            if (by_sphere || !orc_cross(g, &c, r, k, axis)) { status = 1; break; }
            continue;
        }
        double l = tau / k_tot;                 /* interaction inside this cell */
        for (int d = 0; d < 3; ++d) r[d] += l * k[d];
        path += l;
        if (++events >= cap) { status = 3; break; }

        if (C->kd[ci] > 0.0 && orc_draw(&st) < C->kd[ci] / k_tot) {
            if (orc_draw(&st) >= g->dust_albedo) { status = 2; break; }
            isotropic_dir(&st, k);              /* grey isotropic dust scattering */
            x_lab = lab_x(C, ci, x, k);         /* comoving frequency unchanged */
            T->counters[ORC_SCAT_DUST] += 1;
            ++ndust;
            if (p->n_cams > 0) {
                for (int i = 0; i < p->n_cams; ++i) { xcam[i] = x; W[i] = 1.0; }
                peel_off(J, &c, r, xcam, W, T, rec_peel);
            }
            tau = -log(orc_draw(&st));
            continue;
        }

        /* H I scattering (Sec. 3.1.3) */
        double a = C->a[ci], xcw = C->xcw[ci];
        double g_rec = p->recoil ? C->g[ci] : 0.0;
        /* x_crit does not depend on u_par's draws, so it may be taken first */
        double xcrit = event_xcrit(p, C, ci, &c, r, x);
        orc_scatter sc;
        scatter_hi(a, xcw, g_rec, xcrit, p->isotropic, x, k, &st, &sc);
        T->counters[ORC_UPAR_TRIES] += (uint64_t)sc.tries;
        nscat += 1;
        T->counters[ORC_SCAT_HI] += 1;
        if (p->n_cams > 0) {
            double wn = 1.0 + sc.rW / 3.0;
            for (int i = 0; i < p->n_cams; ++i) {
                const double *dc = &p->cam_dir[3 * i];
                double muc = dot3(k, dc);
                W[i] = (1.0 + sc.rW * muc * muc) / wn;
                xcam[i] = x - sc.u_par + dot3(dc, sc.u_atom) + g_rec * (muc - 1.0);
            }
            peel_off(J, &c, r, xcam, W, T, rec_peel);
        }
        for (int d = 0; d < 3; ++d) k[d] = sc.kf[d];
        x_lab = lab_x(C, ci, sc.x_f, k);
        tau = -log(orc_draw(&st));
    }
    if (status == 1) T->counters[ORC_ESCAPED] += 1;
    else if (status == 2) T->counters[ORC_ABSORBED] += 1;
    else T->counters[ORC_CAPPED] += 1;
done:
    if (status == 1 && p->n_bins > 0)
        T->spectrum[bin_of(x_lab, p->x_min, p->x_max, p->n_bins)] += 1.0;
    if (o->rec_x) o->rec_x[slot] = x_lab;
    if (o->rec_nscat) o->rec_nscat[slot] = nscat;
    if (o->rec_status) o->rec_status[slot] = status;
    if (o->rec_pos) for (int d = 0; d < 3; ++d) o->rec_pos[3 * slot + d] = r[d];
    if (o->rec_len) o->rec_len[slot] = path;
    if (o->rec_ndust) o->rec_ndust[slot] = ndust;
}

typedef struct { orc_job *J; int t; } orc_worker_arg;

static void *worker(void *arg)
{
    orc_worker_arg *w = (orc_worker_arg *)arg;
    orc_job *J = w->J;
    orc_tally *T = &J->tallies[w->t];
    const uint64_t chunk = 16;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        uint64_t b = J->next;
        J->next = (b + chunk < J->p->id_end) ? b + chunk : J->p->id_end;
        uint64_t e = J->next;
        pthread_mutex_unlock(&J->lock);
        if (b >= e) break;
        for (uint64_t id = b; id < e; ++id) run_photon(J, id, T);
    }
    return NULL;
}

int orc_run(const orc_grid *g, const orc_source *s, const orc_params *p, orc_out *o,
            int n_threads)
{
    if (p->n_cams > 64 || p->id_end < p->id_begin || p->xcrit_mode < 0 || p->xcrit_mode > 3)
        return -1;
    if (g->kind == 1 && !g->child) return -1;
    orc_job J;
    memset(&J, 0, sizeof J);
    J.g = g; J.s = s; J.p = p; J.o = o;
    cells_init(g, &J.cells);
    for (int d = 0; d < 3; ++d) J.centre[d] = 0.5 * (g->box_min[d] + g->box_max[d]);
    for (int i = 0; i < p->n_cams; ++i) {           /* camera image axes */
        const double *dc = &p->cam_dir[3 * i];
        double up[3] = { 0.0, 0.0, 1.0 };
        if (fabs(dc[2]) > 0.999) { up[1] = 1.0; up[2] = 0.0; }
        double eu[3] = { up[1] * dc[2] - up[2] * dc[1], up[2] * dc[0] - up[0] * dc[2],
                         up[0] * dc[1] - up[1] * dc[0] };
        double n = sqrt(dot3(eu, eu));
        for (int d = 0; d < 3; ++d) eu[d] /= n;
        double ev[3] = { dc[1] * eu[2] - dc[2] * eu[1], dc[2] * eu[0] - dc[0] * eu[2],
                         dc[0] * eu[1] - dc[1] * eu[0] };
        for (int d = 0; d < 3; ++d) { J.cam_eu[3 * i + d] = eu[d]; J.cam_ev[3 * i + d] = ev[d]; }
    }
    J.src_cdf = calloc(s->n_src > 0 ? s->n_src : 1, sizeof(double));
    {
        double tot = 0.0, acc = 0.0;
        for (int i = 0; i < s->n_src; ++i) tot += s->weight ? s->weight[i] : 1.0;
        for (int i = 0; i < s->n_src; ++i) {
            acc += s->weight ? s->weight[i] : 1.0;
            J.src_cdf[i] = acc / tot;
        }
    }
    if (n_threads < 1) n_threads = 1;
    size_t ns = (size_t)p->n_bins + 2, ncs = (size_t)p->n_cams * p->cam_nbins;
    size_t nimg = (size_t)p->n_cams * p->cam_npix * p->cam_npix;
    J.tallies = calloc(n_threads, sizeof(orc_tally));
    for (int t = 0; t < n_threads; ++t) {
        J.tallies[t].spectrum = calloc(ns, sizeof(double));
        J.tallies[t].cam_spec = calloc(ncs ? ncs : 1, sizeof(double));
        J.tallies[t].cam_img = calloc(nimg ? nimg : 1, sizeof(double));
    }
    J.next = p->id_begin;
    pthread_mutex_init(&J.lock, NULL);
    pthread_t *th = calloc(n_threads, sizeof(pthread_t));
    orc_worker_arg *args = calloc(n_threads, sizeof(orc_worker_arg));
    for (int t = 0; t < n_threads; ++t) {
        args[t].J = &J; args[t].t = t;
        pthread_create(&th[t], NULL, worker, &args[t]);
    }
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    /* fixed-order reduction of the per-thread tallies */
    for (int t = 0; t < n_threads; ++t) {
        orc_tally *T = &J.tallies[t];
        if (o->spectrum) for (size_t i = 0; i < ns; ++i) o->spectrum[i] += T->spectrum[i];
        if (o->cam_spec) for (size_t i = 0; i < ncs; ++i) o->cam_spec[i] += T->cam_spec[i];
        if (o->cam_img) for (size_t i = 0; i < nimg; ++i) o->cam_img[i] += T->cam_img[i];
        for (int i = 0; i < ORC_N_COUNTERS; ++i) o->counters[i] += T->counters[i];
        free(T->spectrum); free(T->cam_spec); free(T->cam_img);
    }
    free(J.tallies); free(th); free(args); free(J.src_cdf);
    cells_free(&J.cells);
    return 0;
}

/* x_crit at an H I scattering of comoving frequency x at r, moving along k,
 * as the transport computes it (event_xcrit); -1 if r is outside the domain. */
double orc_xcrit_at(const orc_grid *g, const orc_params *p, const double r[3],
                    const double k[3], double x)
{
    orc_cell c;
    if (!orc_locate(g, r, k, &c)) return -1.0;
    orc_cells C;
    cells_init(g, &C);
    double xc = event_xcrit(p, &C, c.id, &c, r, x);
    cells_free(&C);
    return xc;
}

/* One H I scattering as the transport performs it (scatter_hi), for a photon
 * of comoving frequency x moving along the unit vector k_in in gas at
 * temperature T, with core-skipping frequency xcrit (as used: the wing rule
 * already applied), recoil on or off, from stream (seed, photon) at draw 0.
 * Outputs x_f, k_f and u_par. */
void orc_scatter_once(double T, double x, const double k_in[3], double xcrit, int recoil,
                      int isotropic, uint64_t seed, uint64_t photon, double *x_f,
                      double k_f[3], double *u_par)
{
    double a, sigma0, k0, vth, xcw, g;
    orc_cell_constants(T, 1.0, &a, &sigma0, &k0, &vth, &xcw, &g);
    orc_stream st = { seed, photon, 0 };
    orc_scatter sc;
    scatter_hi(a, xcw, recoil ? g : 0.0, xcrit, isotropic, x, k_in, &st, &sc);
    *x_f = sc.x_f;
    for (int d = 0; d < 3; ++d) k_f[d] = sc.kf[d];
    *u_par = sc.u_par;
}
