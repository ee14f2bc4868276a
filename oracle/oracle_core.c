/*
 * Oracle building blocks: random numbers, line constants, H(a,x), x_cw, and the
 * scattering samplers.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the paper in its notation; scalar FP64, libm transcendentals.
 */
#include "oracle.h"
#include "oracle_internal.h"

#include <math.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the description in Salmon, Moraes, Dror & Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11), Sec. 4: each round  */
/* multiplies words 0 and 2 by fixed 32-bit constants, swaps halves and xors */
/* with the round key; the key is bumped by the Weyl constants each round.   */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform number k of photon `photon` in the job keyed by `seed`, on (0, 1].
 * Block k/2 of the photon's counter space gives four words; the even draw uses
 * words (0,1), the odd draw words (2,3); 53 bits are kept. */
double orc_uniform(uint64_t seed, uint64_t photon, uint64_t k)
{
    uint64_t block = k >> 1;
    uint32_t ctr[4] = { (uint32_t)block, (uint32_t)(block >> 32),
                        (uint32_t)photon, (uint32_t)(photon >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int h = (int)(k & 1);
    uint64_t bits = ((uint64_t)w[2 * h + 1] << 32) | (uint64_t)w[2 * h];
    uint64_t m = bits >> 11;                     /* 53 random bits */
    return ((double)m + 1.0) * 0x1.0p-53;        /* (0, 1] so that -ln R is finite */
}

double orc_draw(orc_stream *s)
{
    return orc_uniform(s->seed, s->photon, s->k++);
}

/* ------------------------------------------------------------------------- */
/* Line constants, Sec. 2: v_th, a, sigma_0 and the recoil parameter g all   */
/* scale with T4^(-1/2) (or T4^(1/2) for v_th).                              */
/* ------------------------------------------------------------------------- */
void orc_cell_constants(double T, double n_HI, double *a, double *sigma0, double *k0,
                        double *vth, double *xcw, double *g)
{
    double T4 = T / 1.0e4;
    double sq = sqrt(T4);
    *vth = ORC_VTH_REF * sq;            /* 12.85 T4^(1/2) km/s */
    *a = 4.702e-4 / sq;                 /* damping parameter   */
    *sigma0 = 5.898e-14 / sq;           /* line-centre cross section, cm^2 */
    *k0 = n_HI * (*sigma0);             /* opacity at line centre, cm^-1 */
    *xcw = orc_xcw(*a);
    *g = 2.536e-4 / sq;                 /* recoil parameter */
}

/* Core-to-wing crossover frequency: rational fit in ln a (Sec. 3.2.2). */
double orc_xcw(double a)
{
    return 6.9184721 + 81.766279 / (log(a) - 14.651253);
}

/* Approximation of the Hjerting-Voigt function H(a,x) to first order in a, in
 * three regions of z = x^2 with the continued fractions and coefficients of
 * the appendix (eq. AB, table AB). */
double orc_H(double a, double x)
{
    static const double A0 = 15.75328153963877, A1 = 286.9341762324778,
                        A2 = 19.05706700907019, A3 = 28.22644017233441,
                        A4 = 9.526399802414186, A5 = 35.29217026286130,
                        A6 = 0.8681020834678775;
    static const double B0 = 0.0003300469163682737, B1 = 0.5403095364583999,
                        B2 = 2.676724102580895, B3 = 12.82026082606220,
                        B4 = 3.21166435627278, B5 = 32.032981933420,
                        B6 = 9.0328158696, B7 = 23.7489999060, B8 = 1.82106170570;
    double z = x * x;
    if (z <= 3.0) {
        double cf = A1 / (z - A2 + A3 / (z - A4 + A5 / (z - A6)));
        return exp(-z) * (1.0 - a * (A0 + cf));
    } else if (z < 25.0) {
        double cf = B1 / (z - B2 + B3 / (z + B4 + B5 / (z - B6 + B7 / (z - B8))));
        return exp(-z) + a * (B0 + cf);
    } else {
        return (a / ORC_SQRT_PI) / (z - 1.5 - 1.5 / (z - 3.5 - 5.0 / (z - 5.5)));
    }
}

/* Critical frequency for core-skipping, eq. xcrit. */
double orc_xcrit(double atau0)
{
    if (atau0 < 1.0) return 0.0;
    return cbrt(atau0) / 5.0;
}

/* Jeans estimate of a*tau0 for core-skipping (Sec. 3.2.4, eq. atau0J): the
 * optical depth parameter across one Jeans length of primordial gas of the
 * cell's density and temperature, 6.428e4 T4^(-1/2) (n_HI / cm^-3)^(1/2). */
double orc_atau_jeans(double T, double n_HI)
{
    return 6.428e4 / sqrt(T / 1.0e4) * sqrt(n_HI);
}

/* ------------------------------------------------------------------------- */
/* Parallel atom velocity (Sec. 3.2.3).  Target f(u) ~ exp(-u^2)/(a^2+(x-u)^2) */
/* (eq. uparf).  For |x| <= 1: Lorentzian proposal, accept exp(-u^2).  For    */
/* 1 < |x| < 9: the two-part comparison function split at u0 (u0,core below  */
/* x_cw, u0,wing above), with p the probability of the part below u0; on      */
/* rejection the part is drawn again.  For |x| >= 9: Gaussian of mean 1/x     */
/* (variance 1/2, that of exp(-u^2)).  Negative x uses f(-x,u) = f(x,-u).     */
/* ------------------------------------------------------------------------- */
double orc_upar_split(double a, double X, double xcw, double *u0_out)
{
    double u0;
    if (X < xcw)
        u0 = X - 1.0 / (X + exp(1.0 - X * X) / a);          /* u0,core */
    else
        u0 = xcw - 1.0 / xcw + 0.15 * (X - xcw);             /* u0,wing */
    double theta0 = atan((u0 - X) / a);
    double e0 = exp(-u0 * u0);
    double p = (theta0 + ORC_PI / 2.0) /
               ((1.0 - e0) * theta0 + (1.0 + e0) * ORC_PI / 2.0);
    *u0_out = u0;
    return p;
}

/* Draw layout: the sampler starts on a fresh counter block (an even draw
 * index); each candidate of the |x| <= 1 proposal takes one block (two
 * draws), each candidate of the two-part proposal two blocks (three draws
 * used, the fourth left unused), the |x| >= 9 Gaussian one block. */
double orc_draw_upar(double a, double x, double xcw, orc_stream *s, int64_t *tries)
{
    double sgn = (x < 0.0) ? -1.0 : 1.0;
    double X = fabs(x);
    double u;
    s->k = (s->k + 1) & ~(uint64_t)1;
    if (X <= 1.0) {
        for (;;) {
            double theta = ORC_PI * (orc_draw(s) - 0.5);
            u = a * tan(theta) + X;
            double Racc = orc_draw(s);
            ++*tries;
            if (Racc < exp(-u * u)) break;
        }
    } else if (X < 9.0) {
        double u0;
        double p = orc_upar_split(a, X, xcw, &u0);
        double theta0 = atan((u0 - X) / a);
        for (;;) {
            double R = orc_draw(s);
            double Rth = orc_draw(s);
            double accept;
            if (R <= p) {                                    /* u <= u0 part */
                double theta = -ORC_PI / 2.0 + Rth * (theta0 + ORC_PI / 2.0);
                u = a * tan(theta) + X;
                accept = exp(-u * u);
            } else {                                         /* u > u0 part  */
                double theta = theta0 + Rth * (ORC_PI / 2.0 - theta0);
                u = a * tan(theta) + X;
                accept = exp(u0 * u0 - u * u);
            }
            double Racc = orc_draw(s);
            s->k += 1;                                       /* unused fourth draw */
            ++*tries;
            if (Racc < accept) break;
        }
    } else {
        double R1 = orc_draw(s), R2 = orc_draw(s);
        u = 1.0 / X + sqrt(-log(R1)) * cos(2.0 * ORC_PI * R2);
    }
    return sgn * u;
}

/* Perpendicular components (Sec. 3.1.3, 3.2.4): Box-Muller on exp(-u^2)/sqrt(pi)
 * per component, truncated below x_crit in magnitude when core-skipping. */
void orc_draw_uperp(double xcrit_eff, orc_stream *s, double *u1, double *u2)
{
    double R1 = orc_draw(s), R2 = orc_draw(s);
    double rho = sqrt(xcrit_eff * xcrit_eff - log(R1));
    *u1 = rho * cos(2.0 * ORC_PI * R2);
    *u2 = rho * sin(2.0 * ORC_PI * R2);
}

/* Cosine of the scattering angle from W(mu) ~ 1 + rW mu^2 on [-1, 1]
 * (eq. phaseW; rW = R/Q for a pure transition, 3/11 for the core mixture).
 * Inverts the CDF, a cubic in mu, with Cardano's formula. */
double orc_draw_mu(double rW, orc_stream *s)
{
    double R = orc_draw(s);
    if (rW == 0.0) return 2.0 * R - 1.0;
    /* CDF: (mu + rW mu^3/3 + 1 + rW/3) / (2 + 2 rW/3) = R
     *  <=> mu^3 + p mu + q = 0 with p = 3/rW, q = (1 + 3/rW)(1 - 2R). */
    double p = 3.0 / rW;
    double q = (1.0 + 3.0 / rW) * (1.0 - 2.0 * R);
    double D = 0.25 * q * q + p * p * p / 27.0;
    double c = cbrt(0.5 * fabs(q) + sqrt(D));
    if (q > 0.0) c = -c;
    double mu = c - p / (3.0 * c);
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Orthonormal pair (e1, e2) perpendicular to the unit vector k. */
void orc_perp_basis(const double k[3], double e1[3], double e2[3])
{
    if (fabs(k[2]) <= 0.9) {                 /* e1 = k x z / |k x z| */
        double n = sqrt(k[0] * k[0] + k[1] * k[1]);
        e1[0] = k[1] / n; e1[1] = -k[0] / n; e1[2] = 0.0;
    } else {                                  /* e1 = k x x / |k x x| */
        double n = sqrt(k[1] * k[1] + k[2] * k[2]);
        e1[0] = 0.0; e1[1] = k[2] / n; e1[2] = -k[1] / n;
    }
    e2[0] = k[1] * e1[2] - k[2] * e1[1];
    e2[1] = k[2] * e1[0] - k[0] * e1[2];
    e2[2] = k[0] * e1[1] - k[1] * e1[0];
}

/* Sampler entry points for the pin tests: n samples, photon i uses stream
 * (seed, i) from draw 0. */
void orc_sample_upar(double a, double x, double xcw, uint64_t seed, int64_t n,
                     double *out, int32_t *draws)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_stream s = { seed, (uint64_t)i, 0 };
        int64_t tries = 0;
        out[i] = orc_draw_upar(a, x, xcw, &s, &tries);
        if (draws) draws[i] = (int32_t)s.k;
    }
}

double orc_sample_upar_one(double a, double x, double xcw, uint64_t seed, uint64_t photon,
                           int32_t *draws)
{
    orc_stream s = { seed, photon, 0 };
    int64_t tries = 0;
    double u = orc_draw_upar(a, x, xcw, &s, &tries);
    if (draws) *draws = (int32_t)s.k;
    return u;
}

void orc_sample_uperp(double xcrit_eff, uint64_t seed, int64_t n, double *out2)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_stream s = { seed, (uint64_t)i, 0 };
        orc_draw_uperp(xcrit_eff, &s, &out2[2 * i], &out2[2 * i + 1]);
    }
}

void orc_sample_mu(double rW, uint64_t seed, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_stream s = { seed, (uint64_t)i, 0 };
        out[i] = orc_draw_mu(rW, &s);
    }
}
