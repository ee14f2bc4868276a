/*
 * Oracle geometry: cell location and cell-by-cell ray tracing on a Cartesian
 * grid or an octree (Sec. 3 intro: a 3-D grid with adaptive refinement; Sec.
 * 3.1.2: trace to the point where the photon exits the current cell).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Tie rules (the paper is silent): cells are half-open [lo, hi); a point lying
 * exactly on a face belongs to the cell the photon is moving into.  Distances
 * are clamped at zero.  Among equal face distances the first axis (x, y, z)
 * is crossed.
 */
#include "oracle.h"
#include "oracle_internal.h"

#include <math.h>

static int side_of(double r, double mid, double k)
{
    if (r > mid) return 1;
    if (r < mid) return 0;
    return (k < 0.0) ? 0 : 1;
}

static int outside_box(const orc_grid *g, const double r[3], const double k[3])
{
    for (int d = 0; d < 3; ++d) {
        if (r[d] < g->box_min[d] || r[d] > g->box_max[d]) return 1;
        if (r[d] == g->box_max[d] && k[d] >= 0.0) return 1;
        if (r[d] == g->box_min[d] && k[d] < 0.0) return 1;
    }
    return 0;
}

static int outside_sphere(const orc_grid *g, const double r[3])
{
    if (g->escape_radius <= 0.0) return 0;
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double c = 0.5 * (g->box_min[d] + g->box_max[d]);
        d2 += (r[d] - c) * (r[d] - c);
    }
    return d2 >= g->escape_radius * g->escape_radius;
}

static void cartesian_bounds(const orc_grid *g, orc_cell *c)
{
    int n[3] = { g->nx, g->ny, g->nz };
    for (int d = 0; d < 3; ++d) {
        double w = (g->box_max[d] - g->box_min[d]) / n[d];
        c->lo[d] = g->box_min[d] + c->ijk[d] * w;
        c->hi[d] = g->box_min[d] + (c->ijk[d] + 1) * w;
    }
    c->id = ((int64_t)c->ijk[2] * g->ny + c->ijk[1]) * g->nx + c->ijk[0];
}

/* Finds the cell holding r for a photon moving along k; returns 0 if r lies
 * outside the domain (box or escape sphere). */
int orc_locate(const orc_grid *g, const double r[3], const double k[3], orc_cell *c)
{
    if (outside_box(g, r, k) || outside_sphere(g, r)) return 0;
    if (g->kind == 0) {
        int n[3] = { g->nx, g->ny, g->nz };
        for (int d = 0; d < 3; ++d) {
            double w = (g->box_max[d] - g->box_min[d]) / n[d];
            double t = (r[d] - g->box_min[d]) / w;
            int i = (int)floor(t);
            if (t == (double)i && k[d] < 0.0) i -= 1;
            if (i < 0) i = 0;
            if (i >= n[d]) i = n[d] - 1;
            c->ijk[d] = i;
        }
        cartesian_bounds(g, c);
        return 1;
    }
    /* octree: descend from the root through the child holding r; faces and
     * midpoints are lattice points X(I) = box_min + I * (side / 2^40) */
    const double unit = (g->box_max[0] - g->box_min[0]) / (double)((int64_t)1 << ORC_OCT_DEPTH);
    int64_t node = 0;
    int64_t I[3] = { 0, 0, 0 };
    int64_t S = (int64_t)1 << ORC_OCT_DEPTH;
    while (g->child[node] >= 0) {
        int64_t half = S / 2;
        int oct = 0;
        for (int d = 0; d < 3; ++d) {
            double mid = g->box_min[d] + (double)(I[d] + half) * unit;
            int b = side_of(r[d], mid, k[d]);
            if (b) I[d] += half;
            oct |= b << d;
        }
        node = g->child[node] + oct;
        S = half;
    }
    c->id = node;
    c->S = S;
    for (int d = 0; d < 3; ++d) {
        c->I[d] = I[d];
        c->lo[d] = g->box_min[d] + (double)I[d] * unit;
        c->hi[d] = g->box_min[d] + (double)(I[d] + S) * unit;
        c->ijk[d] = 0;
    }
    return 1;
}

/* Distance along k from r to where the photon leaves cell c: the nearest face
 * or, when an escape radius is set, the escape sphere. */
double orc_exit_distance(const orc_grid *g, const orc_cell *c, const double r[3],
                         const double k[3], int *axis, int *by_sphere)
{
    double best = INFINITY;
    int best_axis = 0;
    for (int d = 0; d < 3; ++d) {
        double t;
        if (k[d] > 0.0) t = (c->hi[d] - r[d]) / k[d];
        else if (k[d] < 0.0) t = (c->lo[d] - r[d]) / k[d];
        else continue;
        if (t < 0.0) t = 0.0;
        if (t < best) { best = t; best_axis = d; }
    }
    *axis = best_axis;
    *by_sphere = 0;
    if (g->escape_radius > 0.0) {
        double rc[3], b = 0.0, rr = 0.0;
        for (int d = 0; d < 3; ++d) {
            rc[d] = r[d] - 0.5 * (g->box_min[d] + g->box_max[d]);
            b += rc[d] * k[d];
            rr += rc[d] * rc[d];
        }
        double disc = b * b - (rr - g->escape_radius * g->escape_radius);
        double t = (disc > 0.0) ? -b + sqrt(disc) : 0.0;
        if (t < 0.0) t = 0.0;
        if (t <= best) { best = t; *by_sphere = 1; }
    }
    return best;
}

/* Moves a photon that has reached the exit face on `axis` into the next cell.
 * The position component on that axis is set exactly to the face.  Returns 0
 * when the photon leaves the domain. */
int orc_cross(const orc_grid *g, orc_cell *c, double r[3], const double k[3], int axis)
{
    r[axis] = (k[axis] > 0.0) ? c->hi[axis] : c->lo[axis];
    if (g->kind == 0) {
        int n[3] = { g->nx, g->ny, g->nz };
        int i = c->ijk[axis] + ((k[axis] > 0.0) ? 1 : -1);
        if (i < 0 || i >= n[axis]) return 0;
        c->ijk[axis] = i;
        cartesian_bounds(g, c);
        return 1;
    }
    return orc_locate(g, r, k, c);
}

/* Shortest distance from r to the boundary of cell c (local a*tau, Sec. 3.2.4). */
double orc_min_face_distance(const orc_cell *c, const double r[3])
{
    double m = INFINITY;
    for (int d = 0; d < 3; ++d) {
        double a = r[d] - c->lo[d], b = c->hi[d] - r[d];
        if (a < m) m = a;
        if (b < m) m = b;
    }
    return (m < 0.0) ? 0.0 : m;
}

/* Non-local a*tau estimate of Sec. 3.2.4 (eq. atauNL): for every cell, six
 * paths along the coordinate axes start at the centre of one of the cell's
 * faces and run outward, summing a * tau0 = a n_HI sigma0 l over the cells
 * crossed while |n_HI - n_HI,start| < f_NL n_HI,start; the estimate is the
 * smallest of the six sums.  f_NL = 0 gives zero everywhere.  Octree output
 * is per node (internal nodes get 0). */
static double nonlocal_cell(const orc_grid *g, const orc_cell *c0, double f_nl)
{
    double n_start = g->n_HI[c0->id];
    double best = INFINITY;
    for (int d = 0; d < 3; ++d) {
        for (int s = -1; s <= 1; s += 2) {
            double p[3], k[3] = { 0.0, 0.0, 0.0 };
            k[d] = (double)s;
            for (int e = 0; e < 3; ++e) p[e] = 0.5 * (c0->lo[e] + c0->hi[e]);
            if (g->kind == 1) {          /* octree: the centre as a lattice point */
                const double unit = (g->box_max[0] - g->box_min[0]) /
                                    (double)((int64_t)1 << ORC_OCT_DEPTH);
                for (int e = 0; e < 3; ++e)
                    p[e] = g->box_min[e] + (double)(c0->I[e] + c0->S / 2) * unit;
            }
            p[d] = (s > 0) ? c0->hi[d] : c0->lo[d];
            double sum = 0.0;
            orc_cell c;
            if (orc_locate(g, p, k, &c)) {
                for (;;) {
                    double n = g->n_HI[c.id];
                    if (!(fabs(n - n_start) < f_nl * n_start)) break;
                    double a, sigma0, k0, vth, xcw, gr;
                    orc_cell_constants(g->T[c.id], n, &a, &sigma0, &k0, &vth, &xcw, &gr);
                    int axis, by_sphere;
                    double l = orc_exit_distance(g, &c, p, k, &axis, &by_sphere);
                    sum += a * k0 * l;
                    if (by_sphere) break;
                    p[d] += l * k[d];
                    if (!orc_cross(g, &c, p, k, axis)) break;
                }
            }
            if (sum < best) best = sum;
        }
    }
    return best;
}

static void nonlocal_octree(const orc_grid *g, int64_t node, int64_t I[3], int64_t S,
                            double unit, double f_nl, double *out)
{
    if (g->child[node] >= 0) {
        int64_t half = S / 2;
        for (int o = 0; o < 8; ++o) {
            int64_t J[3] = { I[0] + ((o & 1) ? half : 0), I[1] + ((o & 2) ? half : 0),
                             I[2] + ((o & 4) ? half : 0) };
            nonlocal_octree(g, g->child[node] + o, J, half, unit, f_nl, out);
        }
        return;
    }
    orc_cell c;
    c.id = node;
    c.S = S;
    for (int d = 0; d < 3; ++d) {
        c.I[d] = I[d];
        c.ijk[d] = 0;
        c.lo[d] = g->box_min[d] + (double)I[d] * unit;
        c.hi[d] = g->box_min[d] + (double)(I[d] + S) * unit;
    }
    out[node] = nonlocal_cell(g, &c, f_nl);
}

void orc_nonlocal(const orc_grid *g, double f_nl, double *out)
{
    if (g->kind == 0) {
        int n[3] = { g->nx, g->ny, g->nz };
        for (int iz = 0; iz < n[2]; ++iz)
            for (int iy = 0; iy < n[1]; ++iy)
                for (int ix = 0; ix < n[0]; ++ix) {
                    orc_cell c;
                    c.ijk[0] = ix; c.ijk[1] = iy; c.ijk[2] = iz;
                    for (int d = 0; d < 3; ++d) {
                        double w = (g->box_max[d] - g->box_min[d]) / n[d];
                        c.lo[d] = g->box_min[d] + c.ijk[d] * w;
                        c.hi[d] = g->box_min[d] + (c.ijk[d] + 1) * w;
                    }
                    c.id = ((int64_t)iz * n[1] + iy) * n[0] + ix;
                    out[c.id] = nonlocal_cell(g, &c, f_nl);
                }
        return;
    }
    for (int64_t i = 0; i < g->n_nodes; ++i) out[i] = 0.0;
    const double unit = (g->box_max[0] - g->box_min[0]) / (double)((int64_t)1 << ORC_OCT_DEPTH);
    int64_t I[3] = { 0, 0, 0 };
    nonlocal_octree(g, 0, I, (int64_t)1 << ORC_OCT_DEPTH, unit, f_nl, out);
}
