/*
 * synth_pack.c -- overlap-removal sweeps of the seeded cell placement (host input generator).
 *
 * Pure geometry for synth.py: rigid ellipsoids with shape matrices A = s^2 Q diag(a^2) Q^T (s
 * the current scale of the semi-axes) are moved and turned until no pair, and no pair of a
 * cell and a wall mesh point (a sphere of radius a_wall), is below a target of the
 * Perram-Wertheim contact function at lambda = 1/2,
 *     c = r^T (A_i + A_j)^-1 r / 2        (c >= 1: no contact).
 * None of the simulated model's arithmetic is here.
 *
 * One sweep is a damped Jacobi projection: for every contact below the target t^2, with
 * x = (A_i + A_j)^-1 r, the contact function's gradient is x with respect to the centre R_i
 * and g_i = x cross (A_i x) with respect to a small lab-frame rotation of cell i. The
 * minimum-norm move that lifts the linearised c to t^2, rotations weighted by kappa =
 * 1 / (s a_max)^2, is dR_i = tau x, dR_j = -tau x, dtheta_i = kappa tau g_i, dtheta_j =
 * kappa tau g_j with tau = (t^2 - c) / (2 x.x + kappa (g_i.g_i + g_j.g_j)); a wall contact
 * moves the cell alone. Each cell sums the moves of its contacts, scales the sum by
 * damp / sqrt(contacts), caps it, and applies it unless its centre would leave the fluid.
 * Every cell's update is computed from the state before the sweep, in a fixed order, so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Fewer cells than this sweep on one thread: a parallel region per sweep costs more, and far
 * more when several placements run in parallel processes. */
#define PAR_MIN_CELLS 4096

typedef struct {
    int n[3];
    double edge[3];
    int *off, *ids;   /* CSR: off[ncells + 1], ids ascending per cell */
} grid_t;

static int coord(double v, int a, const grid_t *g)
{
    int c = (int)floor(v / g->edge[a]);
    if (c < 0) c = 0;
    if (c >= g->n[a]) c = g->n[a] - 1;
    return c;
}

static void grid_build(grid_t *g, const double *box, double rc, const double *P, int m)
{
    int nc = 1;
    for (int a = 0; a < 3; ++a) {
        int k = (int)floor(box[a] / rc);
        if (k < 1) k = 1;
        g->n[a] = k;
        g->edge[a] = box[a] / k;
        nc *= k;
    }
    g->off = (int *)calloc((size_t)nc + 1, sizeof(int));
    g->ids = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    int *cid = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m; ++i) {
        const double *p = P + 3 * i;
        cid[i] = coord(p[0], 0, g) + g->n[0] * (coord(p[1], 1, g) + g->n[1] * coord(p[2], 2, g));
        g->off[cid[i] + 1]++;
    }
    for (int c = 0; c < nc; ++c) g->off[c + 1] += g->off[c];
    int *fill = (int *)calloc((size_t)nc, sizeof(int));
    for (int i = 0; i < m; ++i) g->ids[g->off[cid[i]] + fill[cid[i]]++] = i;
    free(fill);
    free(cid);
}

static void grid_free(grid_t *g)
{
    free(g->off);
    free(g->ids);
}

/* neighbour cell q (0..26) of cell coordinates cc; -1 outside a non-periodic face. Axes with
 * fewer than three cells list each of their cells once. */
static int nb_cell(const grid_t *g, const int *per, const int *cc, int q)
{
    const int d[3] = {q % 3, (q / 3) % 3, q / 9};
    int v[3];
    for (int a = 0; a < 3; ++a) {
        const int m = g->n[a];
        if (m < 3) {
            if (d[a] >= m) return -1;
            v[a] = d[a];
        } else {
            int x = cc[a] + d[a] - 1;
            if (x < 0 || x >= m) {
                if (!per[a]) return -1;
                x = (x + m) % m;
            }
            v[a] = x;
        }
    }
    return v[0] + g->n[0] * (v[1] + g->n[1] * v[2]);
}

static double min_img(double d, double L, int per)
{
    if (per) d -= L * nearbyint(d / L);
    return d;
}

/* x = H^-1 r for symmetric positive definite H (cofactors) */
static void solve3(const double *H, const double *r, double *x)
{
    const double c00 = H[4] * H[8] - H[5] * H[7], c01 = H[5] * H[6] - H[3] * H[8], c02 = H[3] * H[7] - H[4] * H[6];
    const double det = H[0] * c00 + H[1] * c01 + H[2] * c02;
    const double i00 = c00, i01 = H[2] * H[7] - H[1] * H[8], i02 = H[1] * H[5] - H[2] * H[4];
    const double i10 = c01, i11 = H[0] * H[8] - H[2] * H[6], i12 = H[2] * H[3] - H[0] * H[5];
    const double i20 = c02, i21 = H[1] * H[6] - H[0] * H[7], i22 = H[0] * H[4] - H[1] * H[3];
    const double id = 1.0 / det;
    x[0] = (i00 * r[0] + i01 * r[1] + i02 * r[2]) * id;
    x[1] = (i10 * r[0] + i11 * r[1] + i12 * r[2]) * id;
    x[2] = (i20 * r[0] + i21 * r[1] + i22 * r[2]) * id;
}

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void mv(const double *A, const double *v, double *o)
{
    for (int r = 0; r < 3; ++r) o[r] = A[3 * r] * v[0] + A[3 * r + 1] * v[1] + A[3 * r + 2] * v[2];
}

static int centre_fluid(const double *c, const uint8_t *fluid, const int *dims, const int *per)
{
    int v[3];
    for (int a = 0; a < 3; ++a) {
        int k = (int)floor(c[a] + 0.5);
        if (per[a]) k = ((k % dims[a]) + dims[a]) % dims[a];
        else if (k < 0 || k >= dims[a]) return 0;
        v[a] = k;
    }
    return fluid[(size_t)v[0] + (size_t)dims[0] * ((size_t)v[1] + (size_t)dims[1] * v[2])] != 0;
}

/* Up to nsweeps sweeps at scale s, stopping after a sweep that found no pair contact below
 * s_acc^2 and no wall contact below s_wacc^2. R: [3n] centres (wrapped on periodic axes), Q:
 * [9n] row-major orientations (columns = body axes), both updated in place. wall: [3 nw]
 * wall points. fluid: [nx ny nz] 1 = fluid node. stats[0] = smallest pair contact value of the
 * last sweep, stats[1] = violations counted in it. Returns the number of sweeps done. */
int pack_sweeps(int n, double *R, double *Q, const double *axes, const int *dims, const int *per,
                const double *wall, int nw, double a_wall, const uint8_t *fluid, double s,
                double t_pair, double t_wall, double s_acc, double s_wacc, double damp, double dmax,
                double thmax, int nsweeps, double *stats)
{
    const double box[3] = {(double)dims[0], (double)dims[1], (double)dims[2]};
    const double amax = fmax(axes[0], fmax(axes[1], axes[2]));
    const double rpair = 2.0 * amax * s;
    const double rwall = sqrt(2.0 * (s * s * amax * amax + a_wall * a_wall));
    const double kap = 1.0 / (s * amax * s * amax);
    const double tp2 = t_pair * t_pair, tw2 = t_wall * t_wall, sa2 = s_acc * s_acc, swa2 = s_wacc * s_wacc;
    grid_t wg;
    grid_build(&wg, box, rwall, wall, nw);
    double *A = (double *)malloc(sizeof(double) * 9 * (size_t)(n > 0 ? n : 1));
    double *dR = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *dT = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int *hits = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int done = 0;
    double worst = INFINITY;
    long long nbad = 0;
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int i = 0; i < n; ++i) {
            const double *q = Q + 9 * i;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double v = 0.0;
                    for (int k = 0; k < 3; ++k) v += q[3 * r + k] * axes[k] * axes[k] * q[3 * c + k];
                    A[9 * i + 3 * r + c] = s * s * v;
                }
        }
        grid_t cg;
        grid_build(&cg, box, rpair, R, n);
        worst = INFINITY;
        nbad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(min : worst) reduction(+ : nbad) if (n >= PAR_MIN_CELLS)
        for (int i = 0; i < n; ++i) {
            const double *Ri = R + 3 * i, *Ai = A + 9 * i;
            double acc[3] = {0, 0, 0}, rot[3] = {0, 0, 0};
            int h = 0;
            int cc[3];
            for (int a = 0; a < 3; ++a) cc[a] = coord(Ri[a], a, &cg);
            for (int q = 0; q < 27; ++q) {
                const int cell = nb_cell(&cg, per, cc, q);
                if (cell < 0) continue;
                for (int k = cg.off[cell]; k < cg.off[cell + 1]; ++k) {
                    const int j = cg.ids[k];
                    if (j == i) continue;
                    double d[3];
                    for (int a = 0; a < 3; ++a) d[a] = min_img(Ri[a] - R[3 * j + a], box[a], per[a]);
                    if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] >= rpair * rpair) continue;
                    double H[9], x[3];
                    for (int a = 0; a < 9; ++a) H[a] = Ai[a] + A[9 * j + a];
                    solve3(H, d, x);
                    const double c = 0.5 * (d[0] * x[0] + d[1] * x[1] + d[2] * x[2]);
                    if (j > i) {
                        if (c < worst) worst = c;
                        if (c < sa2) nbad++;
                    }
                    if (c >= tp2) continue;
                    double ax[3], gi[3], gj[3];
                    mv(Ai, x, ax);
                    cross(x, ax, gi);
                    mv(A + 9 * j, x, ax);
                    cross(x, ax, gj);
                    const double den = 2.0 * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) +
                                       kap * (gi[0] * gi[0] + gi[1] * gi[1] + gi[2] * gi[2] +
                                              gj[0] * gj[0] + gj[1] * gj[1] + gj[2] * gj[2]);
                    const double tau = (tp2 - c) / den;
                    for (int a = 0; a < 3; ++a) {
                        acc[a] += tau * x[a];
                        rot[a] += kap * tau * gi[a];
                    }
                    h++;
                }
            }
            if (nw > 0) {
                int wc[3];
                for (int a = 0; a < 3; ++a) wc[a] = coord(Ri[a], a, &wg);
                for (int q = 0; q < 27; ++q) {
                    const int cell = nb_cell(&wg, per, wc, q);
                    if (cell < 0) continue;
                    for (int k = wg.off[cell]; k < wg.off[cell + 1]; ++k) {
                        const int p = wg.ids[k];
                        double d[3];
                        for (int a = 0; a < 3; ++a) d[a] = min_img(Ri[a] - wall[3 * p + a], box[a], per[a]);
                        if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] >= rwall * rwall) continue;
                        double H[9], x[3];
                        for (int a = 0; a < 9; ++a) H[a] = Ai[a] + (a % 4 == 0 ? a_wall * a_wall : 0.0);
                        solve3(H, d, x);
                        const double c = 0.5 * (d[0] * x[0] + d[1] * x[1] + d[2] * x[2]);
                        if (c < swa2) nbad++;
                        if (c >= tw2) continue;
                        double ax[3], g[3];
                        mv(Ai, x, ax);
                        cross(x, ax, g);
                        const double den = (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) +
                                           kap * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                        const double tau = (tw2 - c) / den;
                        for (int a = 0; a < 3; ++a) {
                            acc[a] += tau * x[a];
                            rot[a] += kap * tau * g[a];
                        }
                        h++;
                    }
                }
            }
            hits[i] = h;
            const double f = h ? damp / sqrt((double)h) : 0.0;
            double ln = 0.0, la = 0.0;
            for (int a = 0; a < 3; ++a) {
                acc[a] *= f;
                rot[a] *= f;
                ln += acc[a] * acc[a];
                la += rot[a] * rot[a];
            }
            ln = sqrt(ln);
            la = sqrt(la);
            const double cr = ln > dmax * s ? dmax * s / ln : 1.0, ca = la > thmax ? thmax / la : 1.0;
            for (int a = 0; a < 3; ++a) {
                dR[3 * i + a] = acc[a] * cr;
                dT[3 * i + a] = rot[a] * ca;
            }
        }
        grid_free(&cg);
        done = sw + 1;
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_CELLS)
        for (int i = 0; i < n; ++i) {
            if (!hits[i]) continue;
            double c[3];
            for (int a = 0; a < 3; ++a) {
                c[a] = R[3 * i + a] + dR[3 * i + a];
                if (per[a]) c[a] -= box[a] * floor(c[a] / box[a]);
            }
            if (centre_fluid(c, fluid, dims, per))
                for (int a = 0; a < 3; ++a) R[3 * i + a] = c[a];
            /* Q <- Rot(dtheta) Q (Rodrigues) */
            const double *th = dT + 3 * i;
            const double ang = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
            if (ang > 0.0) {
                const double k0 = th[0] / ang, k1 = th[1] / ang, k2 = th[2] / ang;
                const double sn = sin(ang), cs = 1.0 - cos(ang);
                const double K[9] = {0, -k2, k1, k2, 0, -k0, -k1, k0, 0};
                double K2[9], M[9], Qn[9];
                for (int r = 0; r < 3; ++r)
                    for (int cc2 = 0; cc2 < 3; ++cc2) {
                        double v = 0.0;
                        for (int k = 0; k < 3; ++k) v += K[3 * r + k] * K[3 * k + cc2];
                        K2[3 * r + cc2] = v;
                    }
                for (int a = 0; a < 9; ++a) M[a] = (a % 4 == 0 ? 1.0 : 0.0) + sn * K[a] + cs * K2[a];
                double *q = Q + 9 * i;
                for (int r = 0; r < 3; ++r)
                    for (int cc2 = 0; cc2 < 3; ++cc2)
                        Qn[3 * r + cc2] = M[3 * r] * q[cc2] + M[3 * r + 1] * q[3 + cc2] + M[3 * r + 2] * q[6 + cc2];
                memcpy(q, Qn, sizeof Qn);
            }
        }
        if (nbad == 0) break;
    }
    grid_free(&wg);
    free(A);
    free(dR);
    free(dT);
    free(hits);
    stats[0] = worst;
    stats[1] = (double)nbad;
    return done;
}
