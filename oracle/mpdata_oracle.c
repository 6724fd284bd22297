/*
 * mpdata_oracle.c -- plain FP64 CPU oracle of one MPDATA time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP path is
 * compared against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the product library never links,
 * calls or includes anything from here, and this file includes nothing
 * from the product.
 *
 * What it computes.  The paper (section 5.2, "Introduction to MPDATA")
 * describes one MPDATA time step as a chain of dependent stencil stages
 * that turns five input matrices into one output matrix, shows one of the
 * stages (a 7-point neighbourhood maximum, Listing 1) and defers the
 * equations to the MPDATA literature it cites (Smolarkiewicz 1984 for the
 * upwind pass and the antidiffusive pseudo-velocities, Smolarkiewicz &
 * Grabowski 1990 for the non-oscillatory limiter, Smolarkiewicz & Margolin
 * 1998 for the density-weighted form).  The five inputs are the scalar
 * psi, the three face Courant numbers u1, u2, u3 and the density h; the
 * output is psi at the next time level.
 *
 * The step is written out stage by stage on whole arrays, in the order of
 * the scheme, with no fusion, blocking or reordering:
 *   S1+S2  donor-cell (upwind) pass          -> psi1
 *   S3     antidiffusive pseudo-velocities    -> V1, V2, V3 on faces
 *   S4     limiter bounds (7-point max/min)   -> mx, mn
 *   S5     limiter factors                    -> beta_up, beta_dn
 *   S6     limited pseudo-velocities          -> Vt1, Vt2, Vt3
 *   S7     corrective donor-cell pass         -> psi at n+1
 * plus the mass sum  M = sum_c h_c * psi_c.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - eps regularises every ratio denominator (A, B and beta); default 1e-15.
 *   - the face density is the arithmetic mean of the two cell densities.
 *   - limiter bounds run over psi^n and psi1 at the cell and its 6 face
 *     neighbours (Listing 1 shows the single-field 7-point maximum); a
 *     further corrective pass adds each further iterate of the step.
 *   - periodic boundaries wrap cell indices; face n along an axis is the
 *     same face as face 0 (the caller supplies equal values).
 *   - open boundaries are zero-gradient: a ghost cell takes the value of
 *     the nearest interior cell; the antidiffusive velocity normal to an
 *     open boundary is zero.
 *   - sums of three axis contributions are taken x, then y, then z;
 *     four-term averages are taken as (a+b)+(c+d).
 *
 * Option vsign (fields of variable sign, from the MPDATA literature the
 * paper cites -- Smolarkiewicz & Margolin 1998): the ratios A and B of S3
 * take |psi1| in place of psi1, so their denominators cannot vanish where
 * the field changes sign; every other stage is unchanged.
 *
 * Option iord > 2 (Smolarkiewicz 1984: the corrective pass repeated): pass
 * k = 2 .. iord-1 runs S3-S7 again on the result psi^(k) of pass k-1, with
 * the (limited) antidiffusive velocity of pass k-1 in the place of the
 * Courant numbers; h, eps and the options are the same in every pass.
 *
 * Option div (flows that are not divergence-free, Smolarkiewicz 1984; the
 * density-weighted form of Smolarkiewicz & Margolin 1998): the donor-cell
 * pass of a divergent flow leaves a first-order error proportional to psi
 * times the divergence, which the pseudo-velocity takes back with the term
 *   -(1/4) (U/G) dv
 * on every face, dv the centred divergence of the pass's velocity field
 * across the face: along the face's own axis the difference of the faces
 * beyond b and below a, along each transverse axis the upper faces of a and
 * b minus their lower faces (own axis, then the transverse axes in the
 * cyclic order).  In a later pass the velocity field is the previous pass's
 * antidiffusive velocity, which is divergent in general.
 *
 * Option time-dependent velocity (orc_step_tv; the generalised MPDATA of the
 * literature the paper cites, for flows that change in time): the step from
 * level n to n+1 is given the Courant numbers at both levels, U at n (which
 * the donor-cell pass and every other term use) and W at n+1.  Holding U at
 * level n over the step leaves a first-order error, the flux
 * (1/2) dt (dU/dt) psi, on every face; the first corrective pass takes it
 * back with the term
 *   +(1/2) (W - U)
 * added to the pseudo-velocity of every face (after the divergent-flow term,
 * before the limiter), zero on boundary-normal faces of an open domain like
 * the rest of V.  Later corrective passes (iord > 2) correct their own pass,
 * whose velocity does not change within the step, and add nothing.  With
 * W = U the term is an exact zero.
 *
 * Layout: cell arrays are [k][j][i] with i fastest, nx*ny*nz doubles.
 * Face arrays hold n+1 faces along their own axis: u1[k][j][i'] with
 * i' = 0..nx (face i' lies between cells i'-1 and i'), u2[k][j'][i],
 * u3[k'][j][i].  Positive Courant numbers carry mass toward +axis.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math, no FMA
 * contraction), so every operation below rounds exactly as written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "mpdata_oracle.h"

/* ---------------------------------------------------------------- indexing */

/* Boundary resolution of a cell coordinate: periodic wraps, open clamps. */
static int res(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

typedef struct {
    int nx, ny, nz, bc;
} grid;

static long cell(const grid *g, int i, int j, int k)
{
    i = res(i, g->nx, g->bc);
    j = res(j, g->ny, g->bc);
    k = res(k, g->nz, g->bc);
    return ((long)k * g->ny + j) * g->nx + i;
}

/* Face arrays: the own-axis coordinate is a face index 0..n, the other two
 * are resolved cell coordinates. */
static long xface(const grid *g, int f, int j, int k)
{
    j = res(j, g->ny, g->bc);
    k = res(k, g->nz, g->bc);
    return ((long)k * g->ny + j) * (g->nx + 1) + f;
}

static long yface(const grid *g, int i, int f, int k)
{
    i = res(i, g->nx, g->bc);
    k = res(k, g->nz, g->bc);
    return ((long)k * (g->ny + 1) + f) * g->nx + i;
}

static long zface(const grid *g, int i, int j, int f)
{
    i = res(i, g->nx, g->bc);
    j = res(j, g->ny, g->bc);
    return ((long)f * g->ny + j) * g->nx + i;
}

static double pos(double x) { return x > 0.0 ? x : 0.0; }
static double neg(double x) { return x < 0.0 ? x : 0.0; }

/* Upwind (donor-cell) flux through a face between a lower cell holding
 * value l and an upper cell holding value r, for face Courant number c.
 * Smolarkiewicz 1984, the donor-cell flux function. */
static double donor(double l, double r, double c)
{
    return pos(c) * l + neg(c) * r;
}

/* -------------------------------------------------------- S1+S2: upwind pass
 * out_c = in_c - ( dF1 + dF2 + dF3 ) / h_c with dFd = F(upper face) -
 * F(lower face) along axis d and F = donor(in_lower, in_upper, c_face).
 * Used twice per step: with the Courant numbers (first-order pass) and with
 * the limited antidiffusive velocities (corrective pass). */
static void donor_cell_pass(const grid *g, const double *in, const double *c1,
                            const double *c2, const double *c3, const double *h,
                            double *out)
{
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double vc = in[cell(g, i, j, k)];
                double f1lo = donor(in[cell(g, i - 1, j, k)], vc, c1[xface(g, i, j, k)]);
                double f1hi = donor(vc, in[cell(g, i + 1, j, k)], c1[xface(g, i + 1, j, k)]);
                double f2lo = donor(in[cell(g, i, j - 1, k)], vc, c2[yface(g, i, j, k)]);
                double f2hi = donor(vc, in[cell(g, i, j + 1, k)], c2[yface(g, i, j + 1, k)]);
                double f3lo = donor(in[cell(g, i, j, k - 1)], vc, c3[zface(g, i, j, k)]);
                double f3hi = donor(vc, in[cell(g, i, j, k + 1)], c3[zface(g, i, j, k + 1)]);
                double div = ((f1hi - f1lo) + (f2hi - f2lo)) + (f3hi - f3lo);
                out[cell(g, i, j, k)] = vc - div / h[cell(g, i, j, k)];
            }
}

/* ----------------------------------------- S3: antidiffusive pseudo-velocity
 * On the x-face between a = (i-1, j, k) and b = (i, j, k):
 *   G   = (h_a + h_b)/2
 *   A   = (p_b - p_a) / (p_b + p_a + eps)
 *   U2m = ((u2(a, j) + u2(a, j+1)) + (u2(b, j) + u2(b, j+1))) / 4
 *   B2  = ((p_b,j+1 + p_a,j+1) - (p_b,j-1 + p_a,j-1)) / 2
 *         / ((p_b,j+1 + p_a,j+1) + (p_b,j-1 + p_a,j-1) + eps)
 *   U3m, B3 likewise along k
 *   V1  = (|U1| - U1*U1/G) * A - (U1/G) * (U2m*B2 + U3m*B3)
 * (Smolarkiewicz 1984 for the form; the division of U by the face density
 * G follows Smolarkiewicz & Margolin 1998.)  The y- and z-faces follow by
 * the cyclic permutation x -> y -> z -> x.  With open boundaries the
 * velocity on a boundary-normal face is zero. */

/* The shared formula, written for a face along axis "n" with the two
 * transverse axes "s" and "t". */
static double pseudo_velocity(double U, double G, double pa, double pb,
                              double us_a, double us_b, double ps_a_hi, double ps_b_hi,
                              double ps_a_lo, double ps_b_lo,
                              double ut_a, double ut_b, double pt_a_hi, double pt_b_hi,
                              double pt_a_lo, double pt_b_lo, double eps, int div,
                              double dv)
{
    double A = (pb - pa) / (pb + pa + eps);
    double Us = 0.25 * (us_a + us_b);
    double s_hi = ps_b_hi + ps_a_hi, s_lo = ps_b_lo + ps_a_lo;
    double Bs = 0.5 * (s_hi - s_lo) / (s_hi + s_lo + eps);
    double Ut = 0.25 * (ut_a + ut_b);
    double t_hi = pt_b_hi + pt_a_hi, t_lo = pt_b_lo + pt_a_lo;
    double Bt = 0.5 * (t_hi - t_lo) / (t_hi + t_lo + eps);
    double V = (fabs(U) - U * U / G) * A - (U / G) * (Us * Bs + Ut * Bt);
    if (div) V = V - 0.25 * (U / G) * dv;
    return V;
}

/* Face index f along an axis of n cells, for the neighbouring faces the
 * divergence estimate reads: periodic wraps (face n is face 0), open clamps
 * (only boundary-normal faces, whose V is zero anyway, reach past the ends). */
static int fres(int f, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        f %= n;
        return f < 0 ? f + n : f;
    }
    return f < 0 ? 0 : (f > n ? n : f);
}

static void pseudo_velocities(const grid *g, const double *p, const double *u1,
                              const double *u2, const double *u3, const double *h,
                              double eps, int div, double *v1, double *v2, double *v3)
{
    const int open = g->bc == ORC_BC_OPEN;
    const int bc = g->bc;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int f = 0; f <= g->nx; ++f) {
                long o = xface(g, f, j, k);
                if (open && (f == 0 || f == g->nx)) { v1[o] = 0.0; continue; }
                int a = f - 1, b = f;
                /* column sums of the transverse Courant numbers of cells a, b */
                double sa2 = u2[yface(g, a, j, k)] + u2[yface(g, a, j + 1, k)];
                double sb2 = u2[yface(g, b, j, k)] + u2[yface(g, b, j + 1, k)];
                double sa3 = u3[zface(g, a, j, k)] + u3[zface(g, a, j, k + 1)];
                double sb3 = u3[zface(g, b, j, k)] + u3[zface(g, b, j, k + 1)];
                double dv = 0.0;
                if (div)
                    dv = ((u1[xface(g, fres(f + 1, g->nx, bc), j, k)] -
                           u1[xface(g, fres(f - 1, g->nx, bc), j, k)]) +
                          ((u2[yface(g, a, j + 1, k)] + u2[yface(g, b, j + 1, k)]) -
                           (u2[yface(g, a, j, k)] + u2[yface(g, b, j, k)]))) +
                         ((u3[zface(g, a, j, k + 1)] + u3[zface(g, b, j, k + 1)]) -
                          (u3[zface(g, a, j, k)] + u3[zface(g, b, j, k)]));
                v1[o] = pseudo_velocity(
                    u1[o], 0.5 * (h[cell(g, a, j, k)] + h[cell(g, b, j, k)]),
                    p[cell(g, a, j, k)], p[cell(g, b, j, k)],
                    sa2, sb2, p[cell(g, a, j + 1, k)], p[cell(g, b, j + 1, k)],
                    p[cell(g, a, j - 1, k)], p[cell(g, b, j - 1, k)],
                    sa3, sb3, p[cell(g, a, j, k + 1)], p[cell(g, b, j, k + 1)],
                    p[cell(g, a, j, k - 1)], p[cell(g, b, j, k - 1)], eps, div, dv);
            }
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int f = 0; f <= g->ny; ++f)
            for (int i = 0; i < g->nx; ++i) {
                long o = yface(g, i, f, k);
                if (open && (f == 0 || f == g->ny)) { v2[o] = 0.0; continue; }
                int a = f - 1, b = f;
                /* transverse axes of a y-face: z then x (cyclic order) */
                double sa3 = u3[zface(g, i, a, k)] + u3[zface(g, i, a, k + 1)];
                double sb3 = u3[zface(g, i, b, k)] + u3[zface(g, i, b, k + 1)];
                double sa1 = u1[xface(g, i, a, k)] + u1[xface(g, i + 1, a, k)];
                double sb1 = u1[xface(g, i, b, k)] + u1[xface(g, i + 1, b, k)];
                double dv = 0.0;
                if (div)
                    dv = ((u2[yface(g, i, fres(f + 1, g->ny, bc), k)] -
                           u2[yface(g, i, fres(f - 1, g->ny, bc), k)]) +
                          ((u3[zface(g, i, a, k + 1)] + u3[zface(g, i, b, k + 1)]) -
                           (u3[zface(g, i, a, k)] + u3[zface(g, i, b, k)]))) +
                         ((u1[xface(g, i + 1, a, k)] + u1[xface(g, i + 1, b, k)]) -
                          (u1[xface(g, i, a, k)] + u1[xface(g, i, b, k)]));
                v2[o] = pseudo_velocity(
                    u2[o], 0.5 * (h[cell(g, i, a, k)] + h[cell(g, i, b, k)]),
                    p[cell(g, i, a, k)], p[cell(g, i, b, k)],
                    sa3, sb3, p[cell(g, i, a, k + 1)], p[cell(g, i, b, k + 1)],
                    p[cell(g, i, a, k - 1)], p[cell(g, i, b, k - 1)],
                    sa1, sb1, p[cell(g, i + 1, a, k)], p[cell(g, i + 1, b, k)],
                    p[cell(g, i - 1, a, k)], p[cell(g, i - 1, b, k)], eps, div, dv);
            }
    int f;
#pragma omp parallel for schedule(static)
    for (f = 0; f <= g->nz; ++f)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                long o = zface(g, i, j, f);
                if (open && (f == 0 || f == g->nz)) { v3[o] = 0.0; continue; }
                int a = f - 1, b = f;
                /* transverse axes of a z-face: x then y (cyclic order) */
                double sa1 = u1[xface(g, i, j, a)] + u1[xface(g, i + 1, j, a)];
                double sb1 = u1[xface(g, i, j, b)] + u1[xface(g, i + 1, j, b)];
                double sa2 = u2[yface(g, i, j, a)] + u2[yface(g, i, j + 1, a)];
                double sb2 = u2[yface(g, i, j, b)] + u2[yface(g, i, j + 1, b)];
                double dv = 0.0;
                if (div)
                    dv = ((u3[zface(g, i, j, fres(f + 1, g->nz, bc))] -
                           u3[zface(g, i, j, fres(f - 1, g->nz, bc))]) +
                          ((u1[xface(g, i + 1, j, a)] + u1[xface(g, i + 1, j, b)]) -
                           (u1[xface(g, i, j, a)] + u1[xface(g, i, j, b)]))) +
                         ((u2[yface(g, i, j + 1, a)] + u2[yface(g, i, j + 1, b)]) -
                          (u2[yface(g, i, j, a)] + u2[yface(g, i, j, b)]));
                v3[o] = pseudo_velocity(
                    u3[o], 0.5 * (h[cell(g, i, j, a)] + h[cell(g, i, j, b)]),
                    p[cell(g, i, j, a)], p[cell(g, i, j, b)],
                    sa1, sb1, p[cell(g, i + 1, j, a)], p[cell(g, i + 1, j, b)],
                    p[cell(g, i - 1, j, a)], p[cell(g, i - 1, j, b)],
                    sa2, sb2, p[cell(g, i, j + 1, a)], p[cell(g, i, j + 1, b)],
                    p[cell(g, i, j - 1, a)], p[cell(g, i, j - 1, b)], eps, div, dv);
            }
}

/* ------------------------------------------- S3': time-variation term
 * V_d += (W_d - U_d) / 2 on every face of every axis: W are the Courant
 * numbers at the end of the step, U those at its start (option
 * time-dependent velocity).  Boundary-normal faces of an open domain keep
 * V = 0. */
static void time_variation_term(const grid *g, const double *u1, const double *u2,
                                const double *u3, const double *w1, const double *w2,
                                const double *w3, double *v1, double *v2, double *v3)
{
    const int open = g->bc == ORC_BC_OPEN;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int f = 0; f <= g->nx; ++f) {
                if (open && (f == 0 || f == g->nx)) continue;
                long o = xface(g, f, j, k);
                v1[o] = v1[o] + 0.5 * (w1[o] - u1[o]);
            }
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int f = 0; f <= g->ny; ++f)
            for (int i = 0; i < g->nx; ++i) {
                if (open && (f == 0 || f == g->ny)) continue;
                long o = yface(g, i, f, k);
                v2[o] = v2[o] + 0.5 * (w2[o] - u2[o]);
            }
    int f;
#pragma omp parallel for schedule(static)
    for (f = 0; f <= g->nz; ++f) {
        if (open && (f == 0 || f == g->nz)) continue;
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                long o = zface(g, i, j, f);
                v3[o] = v3[o] + 0.5 * (w3[o] - u3[o]);
            }
    }
}

/* ------------------------------------------------------------ S4: bounds
 * mx_c (mn_c) is the maximum (minimum), over the cell and its six face
 * neighbours, of every field in fields[0 .. nf-1] -- the paper's stage 8
 * (Listing 1) is this 7-point maximum for one field.  Smolarkiewicz &
 * Grabowski 1990 take it over the old solution and the first-order one; a
 * later corrective pass adds each further iterate of the step, so the
 * fields are psi^n, psi^(1), ..., psi^(k) for the pass that corrects
 * psi^(k). */
static void bounds(const grid *g, const double *const *fields, int nf, double *mx,
                   double *mn)
{
    static const int off[7][3] = {{0, 0, 0},  {-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                  {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double hi = -INFINITY, lo = INFINITY;
                for (int q = 0; q < 7; ++q) {
                    long o = cell(g, i + off[q][0], j + off[q][1], k + off[q][2]);
                    for (int f = 0; f < nf; ++f) {
                        hi = fmax(hi, fields[f][o]);
                        lo = fmin(lo, fields[f][o]);
                    }
                }
                mx[cell(g, i, j, k)] = hi;
                mn[cell(g, i, j, k)] = lo;
            }
}

/* --------------------------------------------------- S5: limiter factors
 * With FA = donor(p1_lower, p1_upper, V) on every face,
 *   IN_c  = sum_d [ pos(FA(lower face)) - neg(FA(upper face)) ]
 *   OUT_c = sum_d [ pos(FA(upper face)) - neg(FA(lower face)) ]
 *   beta_up_c = (mx_c - p1_c) * h_c / (IN_c + eps)
 *   beta_dn_c = (p1_c - mn_c) * h_c / (OUT_c + eps)
 * (Smolarkiewicz & Grabowski 1990, density-weighted as the upwind pass). */
static void limiter_factors(const grid *g, const double *p1, const double *v1,
                            const double *v2, const double *v3, const double *mx,
                            const double *mn, const double *h, double eps,
                            double *bup, double *bdn)
{
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                double pc = p1[cell(g, i, j, k)];
                double x_lo = donor(p1[cell(g, i - 1, j, k)], pc, v1[xface(g, i, j, k)]);
                double x_hi = donor(pc, p1[cell(g, i + 1, j, k)], v1[xface(g, i + 1, j, k)]);
                double y_lo = donor(p1[cell(g, i, j - 1, k)], pc, v2[yface(g, i, j, k)]);
                double y_hi = donor(pc, p1[cell(g, i, j + 1, k)], v2[yface(g, i, j + 1, k)]);
                double z_lo = donor(p1[cell(g, i, j, k - 1)], pc, v3[zface(g, i, j, k)]);
                double z_hi = donor(pc, p1[cell(g, i, j, k + 1)], v3[zface(g, i, j, k + 1)]);
                double in = ((pos(x_lo) - neg(x_hi)) + (pos(y_lo) - neg(y_hi))) +
                            (pos(z_lo) - neg(z_hi));
                double out = ((pos(x_hi) - neg(x_lo)) + (pos(y_hi) - neg(y_lo))) +
                             (pos(z_hi) - neg(z_lo));
                long c = cell(g, i, j, k);
                bup[c] = (mx[c] - pc) * h[c] / (in + eps);
                bdn[c] = (pc - mn[c]) * h[c] / (out + eps);
            }
}

/* ------------------------------------------- S6: limited pseudo-velocity
 * On a face between lower cell a and upper cell b:
 *   Vt = min(1, beta_dn_a, beta_up_b) * pos(V) + min(1, beta_up_a, beta_dn_b) * neg(V)
 * (Smolarkiewicz & Grabowski 1990). */
static double limited(double v, double bup_a, double bdn_a, double bup_b, double bdn_b)
{
    return fmin(1.0, fmin(bdn_a, bup_b)) * pos(v) + fmin(1.0, fmin(bup_a, bdn_b)) * neg(v);
}

static void limit_velocities(const grid *g, const double *bup, const double *bdn,
                             double *v1, double *v2, double *v3)
{
    const int open = g->bc == ORC_BC_OPEN;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int f = 0; f <= g->nx; ++f) {
                long o = xface(g, f, j, k);
                if (open && (f == 0 || f == g->nx)) continue;
                long a = cell(g, f - 1, j, k), b = cell(g, f, j, k);
                v1[o] = limited(v1[o], bup[a], bdn[a], bup[b], bdn[b]);
            }
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int f = 0; f <= g->ny; ++f)
            for (int i = 0; i < g->nx; ++i) {
                long o = yface(g, i, f, k);
                if (open && (f == 0 || f == g->ny)) continue;
                long a = cell(g, i, f - 1, k), b = cell(g, i, f, k);
                v2[o] = limited(v2[o], bup[a], bdn[a], bup[b], bdn[b]);
            }
    int f;
#pragma omp parallel for schedule(static)
    for (f = 0; f <= g->nz; ++f)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                long o = zface(g, i, j, f);
                if (open && (f == 0 || f == g->nz)) continue;
                long a = cell(g, i, j, f - 1), b = cell(g, i, j, f);
                v3[o] = limited(v3[o], bup[a], bdn[a], bup[b], bdn[b]);
            }
}

/* ---------------------------------------------------------------- API */

int orc_check(const orc_params *p)
{
    if (!p) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->bc != ORC_BC_PERIODIC && p->bc != ORC_BC_OPEN) return -1;
    if (p->iord < 1 || p->iord > ORC_MAX_IORD) return -1;
    if (p->nonos != 0 && p->nonos != 1) return -1;
    if (p->vsign != 0 && p->vsign != 1) return -1;
    if (p->div != 0 && p->div != 1) return -1;
    if (!(p->eps > 0.0)) return -1;
    return 0;
}

int orc_step(const orc_params *p, const double *psi, const double *u1,
             const double *u2, const double *u3, const double *h, double *out,
             orc_stages *st)
{
    return orc_step_tv(p, psi, u1, u2, u3, 0, 0, 0, h, out, st);
}

int orc_step_tv(const orc_params *p, const double *psi, const double *u1,
                const double *u2, const double *u3, const double *w1,
                const double *w2, const double *w3, const double *h, double *out,
                orc_stages *st)
{
    if (orc_check(p)) return -1;
    if ((w1 != 0) != (w2 != 0) || (w1 != 0) != (w3 != 0)) return -1;
    grid g = {p->nx, p->ny, p->nz, p->bc};
    long n = (long)p->nx * p->ny * p->nz;
    long n1 = (long)(p->nx + 1) * p->ny * p->nz;
    long n2 = (long)p->nx * (p->ny + 1) * p->nz;
    long n3 = (long)p->nx * p->ny * (p->nz + 1);
    const int npass = p->iord - 1;  /* corrective passes */

    /* iterates of the step: it[0] = psi^n, it[k] = psi^(k) */
    const double *it[ORC_MAX_IORD + 1];
    double *own[ORC_MAX_IORD + 1] = {0};
    /* velocities: the pass being corrected (c) and the new one (v) */
    double *va[3] = {0}, *vb[3] = {0};
    double *mx = 0, *mn = 0, *bu = 0, *bd = 0, *a1 = 0;
    int rc = -2;
    it[0] = psi;
    for (int k = 1; k <= p->iord; ++k)
        if (!(own[k] = malloc(sizeof(double) * n))) goto done;
    if (npass > 0) {
        long nf[3] = {n1, n2, n3};
        for (int d = 0; d < 3; ++d)
            if (!(va[d] = malloc(sizeof(double) * nf[d])) ||
                !(vb[d] = malloc(sizeof(double) * nf[d])))
                goto done;
        if (!(mx = malloc(sizeof(double) * n)) || !(mn = malloc(sizeof(double) * n)) ||
            !(bu = malloc(sizeof(double) * n)) || !(bd = malloc(sizeof(double) * n)))
            goto done;
        if (p->vsign && !(a1 = malloc(sizeof(double) * n))) goto done;
    }

    donor_cell_pass(&g, psi, u1, u2, u3, h, own[1]);                  /* S1+S2 */
    it[1] = own[1];
    if (st && st->psi1) memcpy(st->psi1, own[1], sizeof(double) * n);

    /* Corrective pass k (k = 1 .. iord-1) corrects psi^(k): its velocity
     * field is the Courant numbers for k = 1 and the (limited)
     * antidiffusive velocity of pass k-1 after that (Smolarkiewicz 1984). */
    const double *c1 = u1, *c2 = u2, *c3 = u3;
    for (int k = 1; k <= npass; ++k) {
        const double *cur = it[k];
        double **v = (k & 1) ? va : vb;
        if (p->vsign) {
            /* S3 on |psi^(k)| (option vsign); the limiter and S7 keep psi^(k) */
            for (long c = 0; c < n; ++c) a1[c] = fabs(cur[c]);
            pseudo_velocities(&g, a1, c1, c2, c3, h, p->eps, p->div, v[0], v[1], v[2]);
        } else {
            pseudo_velocities(&g, cur, c1, c2, c3, h, p->eps, p->div, v[0], v[1], v[2]); /* S3 */
        }
        if (k == 1 && w1)                                                   /* S3' */
            time_variation_term(&g, u1, u2, u3, w1, w2, w3, v[0], v[1], v[2]);
        const int last = k == npass;
        if (last && st && st->v1) memcpy(st->v1, v[0], sizeof(double) * n1);
        if (last && st && st->v2) memcpy(st->v2, v[1], sizeof(double) * n2);
        if (last && st && st->v3) memcpy(st->v3, v[2], sizeof(double) * n3);
        if (p->nonos) {
            bounds(&g, it, k + 1, mx, mn);                                        /* S4 */
            limiter_factors(&g, cur, v[0], v[1], v[2], mx, mn, h, p->eps, bu, bd); /* S5 */
            if (last && st && st->mx) memcpy(st->mx, mx, sizeof(double) * n);
            if (last && st && st->mn) memcpy(st->mn, mn, sizeof(double) * n);
            if (last && st && st->beta_up) memcpy(st->beta_up, bu, sizeof(double) * n);
            if (last && st && st->beta_dn) memcpy(st->beta_dn, bd, sizeof(double) * n);
            limit_velocities(&g, bu, bd, v[0], v[1], v[2]);                       /* S6 */
        }
        donor_cell_pass(&g, cur, v[0], v[1], v[2], h, own[k + 1]);                /* S7 */
        it[k + 1] = own[k + 1];
        c1 = v[0];
        c2 = v[1];
        c3 = v[2];
    }
    memcpy(out, it[p->iord], sizeof(double) * n);
    rc = 0;
done:
    for (int k = 1; k <= p->iord; ++k) free(own[k]);
    for (int d = 0; d < 3; ++d) {
        free(va[d]);
        free(vb[d]);
    }
    free(mx); free(mn); free(bu); free(bd); free(a1);
    return rc;
}

int orc_run(const orc_params *p, double *psi, const double *u1, const double *u2,
            const double *u3, const double *h, int nsteps)
{
    if (orc_check(p) || nsteps < 0) return -1;
    long n = (long)p->nx * p->ny * p->nz;
    double *tmp = malloc(sizeof(double) * n);
    if (!tmp) return -2;
    for (int s = 0; s < nsteps; ++s) {
        int rc = orc_step(p, psi, u1, u2, u3, h, tmp, NULL);
        if (rc) { free(tmp); return rc; }
        memcpy(psi, tmp, sizeof(double) * n);
    }
    free(tmp);
    return 0;
}

/* Mass M = sum_c h_c * psi_c, computed with the compensated dot product
 * "Dot2" of Ogita, Rump & Oishi (SIAM J. Sci. Comput. 26, 2005): each
 * product is split exactly into p + e with an FMA (TwoProduct), the running
 * sum is split exactly with Knuth's TwoSum, and all rounding errors are
 * accumulated separately and added at the end.  The result is as accurate
 * as a dot product evaluated in twice the working precision. */
double orc_mass(long n, const double *h, const double *psi)
{
    double s = 0.0, c = 0.0;
    for (long i = 0; i < n; ++i) {
        double prod = h[i] * psi[i];
        double perr = fma(h[i], psi[i], -prod);
        double t = s + prod;
        double bb = t - s;
        double serr = (s - (t - bb)) + (prod - bb);
        s = t;
        c = c + (perr + serr);
    }
    return s + c;
}

/* Mass flowing in through the six faces of an open (zero-gradient) domain
 * during the first-order pass: at a boundary face the ghost cell equals the
 * boundary cell, so the upwind flux there is c * psi_boundary whichever way
 * the flow goes.  Returned as the net inflow (positive = mass gained).  The
 * corrective pass adds nothing because V is zero on those faces. */
double orc_open_inflow(const orc_params *p, const double *psi, const double *u1,
                       const double *u2, const double *u3)
{
    grid g = {p->nx, p->ny, p->nz, ORC_BC_OPEN};
    double in = 0.0;
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j) {
            in += u1[xface(&g, 0, j, k)] * psi[cell(&g, 0, j, k)];
            in -= u1[xface(&g, g.nx, j, k)] * psi[cell(&g, g.nx - 1, j, k)];
        }
    for (int k = 0; k < g.nz; ++k)
        for (int i = 0; i < g.nx; ++i) {
            in += u2[yface(&g, i, 0, k)] * psi[cell(&g, i, 0, k)];
            in -= u2[yface(&g, i, g.ny, k)] * psi[cell(&g, i, g.ny - 1, k)];
        }
    for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
            in += u3[zface(&g, i, j, 0)] * psi[cell(&g, i, j, 0)];
            in -= u3[zface(&g, i, j, g.nz)] * psi[cell(&g, i, j, g.nz - 1)];
        }
    return in;
}

/* Number of OpenMP threads the stage loops run on (1 without OpenMP).  The
 * results do not depend on it: every output element is computed by one
 * thread from inputs that no thread writes. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of the stage loops (n >= 1; ignored
 * without OpenMP); returns the number now in effect. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return orc_threads();
}
