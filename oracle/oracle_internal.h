/* Private declarations of the oracle (TEST INFRASTRUCTURE ONLY, see oracle.h). */
#ifndef COLT_ORACLE_INTERNAL_H
#define COLT_ORACLE_INTERNAL_H

#include <stdint.h>

#define ORC_PI       3.14159265358979323846
#define ORC_SQRT_PI  1.77245385090551602730
#define ORC_VTH_REF  12.85          /* km/s, thermal speed at T = 1e4 K (Sec. 2) */

/* One photon's random stream: uniform number k of (seed, photon). */
typedef struct { uint64_t seed, photon, k; } orc_stream;

double orc_draw(orc_stream *s);
double orc_draw_upar(double a, double x, double xcw, orc_stream *s, int64_t *tries);
void   orc_draw_uperp(double xcrit_eff, orc_stream *s, double *u1, double *u2);
double orc_draw_mu(double rW, orc_stream *s);
void   orc_perp_basis(const double k[3], double e1[3], double e2[3]);

/* Cell reached by a photon: Cartesian (i,j,k) or octree leaf, with its box. */
typedef struct {
    int64_t id;          /* flat Cartesian index or octree node index */
    int32_t ijk[3];      /* Cartesian indices                          */
    int64_t I[3], S;     /* octree: lower corner and size on the lattice of
                            2^ORC_OCT_DEPTH steps per root side          */
    double lo[3], hi[3]; /* cell bounds in cm                          */
} orc_cell;

/* Octree faces are evaluated as one function of an integer lattice
 * coordinate, so neighbouring cells see bit-identical shared faces. */
#define ORC_OCT_DEPTH 40

/* Geometry helpers (oracle_grid.c). */
int    orc_locate(const orc_grid *g, const double r[3], const double k[3], orc_cell *c);
double orc_exit_distance(const orc_grid *g, const orc_cell *c, const double r[3],
                         const double k[3], int *axis, int *by_sphere);
int    orc_cross(const orc_grid *g, orc_cell *c, double r[3], const double k[3], int axis);
double orc_min_face_distance(const orc_cell *c, const double r[3]);

#endif
