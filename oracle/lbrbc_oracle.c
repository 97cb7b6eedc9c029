/*
 * lbrbc_oracle.c -- plain FP64 CPU oracle of the coupled plasma / rigid red-blood-cell
 * time step (S. Melchionna, 2011). TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Written for reading, not for speed: every step is a direct loop over nodes or cells in
 * the order of the paper, in double precision, with no blocking, fusion or reordering.
 * Where the paper is silent, garbled or inconsistent, the reading taken is stated at the
 * place it is used.
 *
 * One time step n -> n+1 (the paper gives the pieces, not their order; this order is
 * the reading taken):
 *   1. rigid-body first half (App. A steps 1-4)
 *   2. cell list of the cell centres (Gay-Berne neighbour search)
 *   3. node -> cell coverage map
 *   4. interpolation of u, vorticity and stress onto each cell (Eqs. 17-21)
 *   5. Gay-Berne cell-cell and cell-wall forces and torques (Eqs. 24-28, App. B)
 *   6. rigid-body second half (App. A steps 5-7) and the hydrodynamic force/torque
 *   7. spread back-reaction G and local relaxation time (Sec. II B, Eq. 23)
 *   8. pull stream + BGK collision with body force (Eqs. 1-8), halfway bounce-back
 * Steps 4 uses the velocity and stress stored by step 8 of the previous step.
 *
 * The stress torque T^S of step 4 (Eq. 16) is pinned by its symmetries, its sign, its
 * linearity in alpha and a four-node configuration whose value is worked out by hand.
 */
#include "lbrbc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer nodes or cells than these run on one thread: a parallel region per step
 * costs more than such loops, and far more when several processes share the cores. Every
 * iteration is independent, so the thread count changes no result. */
#define ORC_PAR_NODES 16384
#define ORC_PAR_CELLS 64

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from here on (the timing of the oracle on 1 and on N cores). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------------------- */
/* D3Q19 lattice (Sec. II A): c0 = 0 (w = 1/3), six first neighbours (w = 1/18), twelve
 * second neighbours (w = 1/36). The paper leaves the order inside each group open; the
 * order here puts opposite speeds next to each other. */
static const int CV[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double WV[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c^2, squared lattice sound speed */

static int opposite(int p)
{
    int q;
    for (q = 0; q < 19; ++q)
        if (CV[q][0] == -CV[p][0] && CV[q][1] == -CV[p][1] && CV[q][2] == -CV[p][2])
            return q;
    return -1;
}

void orc_lattice(int c[19][3], double w[19])
{
    int p, a;
    for (p = 0; p < 19; ++p) {
        for (a = 0; a < 3; ++a) c[p][a] = CV[p][a];
        w[p] = WV[p];
    }
}

/* Eq. (3): second-order equilibrium. */
double orc_feq(double rho, const double u[3], int p)
{
    double uc = u[0] * CV[p][0] + u[1] * CV[p][1] + u[2] * CV[p][2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return WV[p] * rho * (1.0 + uc / CS2 + (uc * uc - CS2 * uu) / (2.0 * CS2 * CS2));
}

/* Body-force term added after the BGK relaxation (Eq. 2 with Eq. 4, h = 1).
 * The spread quantity is a force density g (the printed rho*G, Sec. II B), so Eq. 4's
 * rho*G is g here. forcing = 1 is Eq. 4 as printed. forcing = 0 is the second-order
 * form of the reference the paper cites for Eq. 6 (Guo et al. 2002): prefactor
 * (1 - 1/(2T)) and 1/c^4 on the second-order term. Only the latter injects exactly g
 * of momentum per step together with the half-force velocity shift of Eq. 6. */
double orc_force_term(int forcing, double T, const double g[3], const double u[3], int p)
{
    double gc = g[0] * CV[p][0] + g[1] * CV[p][1] + g[2] * CV[p][2];
    double uc = u[0] * CV[p][0] + u[1] * CV[p][1] + u[2] * CV[p][2];
    double gu = g[0] * u[0] + g[1] * u[1] + g[2] * u[2];
    if (forcing == 1)
        return WV[p] * (gc / CS2 + (gc * uc - CS2 * gu) / (2.0 * CS2 * CS2));
    return (1.0 - 1.0 / (2.0 * T)) * WV[p] * (gc / CS2 + (gc * uc - CS2 * gu) / (CS2 * CS2));
}

/* Shape function, Sec. II B (Eqs. 10-11). The printed 1-D profile is negative on part
 * of its support and jumps at |y/xi| = 1/2, so it cannot be the normalised kernel the
 * text describes. This is the four-point kernel of the cited reference (Peskin 2002)
 * at r = 2|y|/xi, which has the stated properties: support |y| < xi, 64 mesh points at
 * xi = 2, unit sum at xi = 2. */
double orc_peskin(double r)
{
    r = fabs(r);
    if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
    if (r < 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
    return 0.0;
}

/* ---------------------------------------------------------------------------------- */
struct orc_sim {
    orc_params P;
    int nx, ny, nz;
    long N;
    uint8_t* solid;
    double* f;     /* post-collision populations of the last step, f[p*N+n] */
    double* fnew;
    double* u;     /* velocity of the last step (Eq. 6) [n*3+a] */
    double* sig;   /* shear stress of the last step (Eq. 8) [n*6+k] */
    double* g;     /* force density spread in the last step [n*3+a] */
    double* Trel;  /* local relaxation time of the last step [n] */
    double wall_mom[3];

    int nrbc;
    double *R, *Q, *V, *Om;
    double *Fcomb, *Tcomb;   /* lab force, body torque */
    double *Vh, *Omh;        /* after the first half */
    double *S, *ut, *wt, *TS;
    double *Fhyd, *Thyd;     /* lab */
    double *Fmech, *Tmech;   /* lab force, body torque */

    double rc;
    int ncell[3];
    double cedge[3];
    int* cell_off;
    int* cell_ids;

    int nwall;
    int* wall_xyz;
    int* wcell_off;
    int* wcell_ids;

    long* map_off;
    int* map_ids;
    long map_len, map_alloc;

    int nwn;          /* wall-adjacent fluid nodes */
    long* wn_node;
    double* wn_nrm;   /* unit wall normal per wall-adjacent node (towards the wall) */
    long step;
};

static int wrapi(int v, int L) { return ((v % L) + L) % L; }

/* Node index of integer position (x, y, z); -1 if outside a non-periodic face. */
static long node_at(const orc_sim* s, int x, int y, int z)
{
    if (x < 0 || x >= s->nx) { if (!s->P.periodic[0]) return -1; x = wrapi(x, s->nx); }
    if (y < 0 || y >= s->ny) { if (!s->P.periodic[1]) return -1; y = wrapi(y, s->ny); }
    if (z < 0 || z >= s->nz) { if (!s->P.periodic[2]) return -1; z = wrapi(z, s->nz); }
    return (long)x + (long)s->nx * ((long)y + (long)s->ny * z);
}

static int fluid_at(const orc_sim* s, int x, int y, int z)
{
    long n = node_at(s, x, y, z);
    return n >= 0 && !s->solid[n];
}

static void node_xyz(const orc_sim* s, long n, int* x, int* y, int* z)
{
    *x = (int)(n % s->nx);
    *y = (int)((n / s->nx) % s->ny);
    *z = (int)(n / ((long)s->nx * s->ny));
}

static double box_len(const orc_sim* s, int a) { return a == 0 ? s->nx : (a == 1 ? s->ny : s->nz); }

/* Minimum image of a lab-frame displacement on the periodic axes. */
static void min_image(const orc_sim* s, double d[3])
{
    int a;
    for (a = 0; a < 3; ++a) {
        double L = box_len(s, a);
        if (!s->P.periodic[a]) continue;
        if (d[a] > 0.5 * L) d[a] -= L;
        else if (d[a] < -0.5 * L) d[a] += L;
    }
}

static int open_plane(const orc_sim* s, int z)
{
    return s->P.open_z && (z == 0 || z == s->nz - 1);
}

/* ---------------------------------------------------------------------------------- */
/* Shape function of cell i at the node with integer position xn (already wrapped).
 * The printed argument (Q x) mixes frames: with v' = Q v mapping body to lab, the body
 * coordinates of the lab displacement d are Q^T d. Each component is accumulated left to
 * right without fused multiply-add so that the support test is reproducible. */
static void body_coords(const orc_sim* s, int i, const int xn[3], double y[3])
{
    const double* Q = s->Q + 9 * i;
    double d[3];
    int a;
    for (a = 0; a < 3; ++a) d[a] = (double)xn[a] - s->R[3 * i + a];
    min_image(s, d);
    for (a = 0; a < 3; ++a) {
        double t0 = Q[0 * 3 + a] * d[0];
        double t1 = Q[1 * 3 + a] * d[1];
        double t2 = Q[2 * 3 + a] * d[2];
        y[a] = (t0 + t1) + t2;
    }
}

/* Support test: |y_a| < xi_a on every body axis. */
static int inside(const orc_sim* s, int i, const int xn[3])
{
    double y[3];
    body_coords(s, i, xn, y);
    return fabs(y[0]) < s->P.xi[0] && fabs(y[1]) < s->P.xi[1] && fabs(y[2]) < s->P.xi[2];
}

/* Unnormalised shape function: product of three 1-D kernels in body coordinates. */
static double delta_raw(const orc_sim* s, int i, const int xn[3])
{
    double y[3];
    body_coords(s, i, xn, y);
    return orc_peskin(2.0 * y[0] / s->P.xi[0]) * orc_peskin(2.0 * y[1] / s->P.xi[1]) *
           orc_peskin(2.0 * y[2] / s->P.xi[2]);
}

/* Normalised shape function. The unit sum of Eq. 12 holds only for xi = 2 on an
 * unobstructed lattice; the reading taken normalises explicitly over the fluid nodes
 * (S_i = sum of the raw kernel over fluid nodes) and sets the kernel to zero on solid
 * nodes. (x, y, z) may be unwrapped; outside a non-periodic face the kernel is zero. */
static double delta_hat(const orc_sim* s, int i, int x, int y, int z)
{
    long n = node_at(s, x, y, z);
    int xn[3];
    if (n < 0 || s->solid[n]) return 0.0;
    node_xyz(s, n, &xn[0], &xn[1], &xn[2]);
    return delta_raw(s, i, xn) / s->S[i];
}

/* Gradient of the normalised kernel by central differences on the lattice. With this
 * discrete derivative the identities of Eq. 13 hold exactly on a periodic lattice. */
static void grad_delta_hat(const orc_sim* s, int i, int x, int y, int z, double gr[3])
{
    gr[0] = 0.5 * (delta_hat(s, i, x + 1, y, z) - delta_hat(s, i, x - 1, y, z));
    gr[1] = 0.5 * (delta_hat(s, i, x, y + 1, z) - delta_hat(s, i, x, y - 1, z));
    gr[2] = 0.5 * (delta_hat(s, i, x, y, z + 1) - delta_hat(s, i, x, y, z - 1));
}

/* Half-width of a cube around a cell centre that contains its support plus one node. */
static int support_halfwidth(const orc_sim* s)
{
    double r = sqrt(s->P.xi[0] * s->P.xi[0] + s->P.xi[1] * s->P.xi[1] + s->P.xi[2] * s->P.xi[2]);
    return (int)ceil(r) + 2;
}

/* ---------------------------------------------------------------------------------- */
static void mat_vec(const double* M, const double* v, double* out)
{
    int r;
    for (r = 0; r < 3; ++r) out[r] = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
}
static void matT_vec(const double* M, const double* v, double* out)
{
    int c;
    for (c = 0; c < 3; ++c) out[c] = M[c] * v[0] + M[3 + c] * v[1] + M[6 + c] * v[2];
}
static void cross(const double* a, const double* b, double* out)
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}
static int inv3(const double* M, double* Mi)
{
    double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                 M[2] * (M[3] * M[7] - M[4] * M[6]);
    if (det == 0.0) return 1;
    Mi[0] = (M[4] * M[8] - M[5] * M[7]) / det;
    Mi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    Mi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    Mi[3] = (M[5] * M[6] - M[3] * M[8]) / det;
    Mi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    Mi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    Mi[6] = (M[3] * M[7] - M[4] * M[6]) / det;
    Mi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    Mi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    return 0;
}

/* ---------------------------------------------------------------------------------- */
/* Gay-Berne repulsion (Sec. II E, Eqs. 24-28; App. B).
 * A = Q S^2 Q^T, H = A_i + A_j, phi = R^.H^-1.R^/2, sigma = phi^-1/2,
 * rho = (R - sigma + sigma_min)/sigma_min, u = 4 eps0 (rho^-12 - rho^-6) + eps0 while
 * rho^6 <= 2 (zero beyond; u and the force vanish at the cut-off).
 * R_ij = R_i - R_j and F_ij = -grad_{R_i} u is the force on i. The force follows Eq. B1.
 * The printed torques (Eqs. B5, B6) are off by a factor 1/R_ij and, for j, by a sign
 * against -du/d(rotation angle); this uses tau_i = (1/R) R_ci x f_k and
 * tau_j = -(1/R) R_cj x f_k in the lab frame, with R_ci = -A_i k and R_cj = A_j k, which
 * satisfies the stated sum rule tau_i + tau_j = -R_ij x F_ij. A wall particle j is a
 * sphere of radius a_wall (A_j = a_wall^2 1) with sigma_min = sigmin_wall. */
static int gb_pair_core(const orc_params* P, const double rij[3], const double* Qi,
                        const double* Qj, int wall, double* U, double F[3], double ti[3],
                        double tj[3])
{
    double Ai[9], Aj[9], H[9], Hi[9], kap[3], Aik[3], Ajk[3], rhat[3], fk[3];
    double R, phi, sigma, smin, rho, dudr, dudphi, kr;
    int r, c, k;
    double amin_i, amin_j;
    F[0] = F[1] = F[2] = ti[0] = ti[1] = ti[2] = tj[0] = tj[1] = tj[2] = 0.0;
    *U = 0.0;
    for (r = 0; r < 3; ++r)
        for (c = 0; c < 3; ++c) {
            double a = 0.0, b = 0.0;
            for (k = 0; k < 3; ++k) {
                a += Qi[3 * r + k] * P->axes[k] * P->axes[k] * Qi[3 * c + k];
                if (!wall) b += Qj[3 * r + k] * P->axes[k] * P->axes[k] * Qj[3 * c + k];
            }
            if (wall) b = (r == c) ? P->a_wall * P->a_wall : 0.0;
            Ai[3 * r + c] = a;
            Aj[3 * r + c] = b;
            H[3 * r + c] = a + b;
        }
    if (inv3(H, Hi)) return ORC_EOVERLAP;
    R = sqrt(rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2]);
    if (R == 0.0) return ORC_EOVERLAP;
    for (k = 0; k < 3; ++k) rhat[k] = rij[k] / R;
    mat_vec(Hi, rij, kap); /* kappa = H^-1 R_ij */
    phi = 0.5 * (rhat[0] * kap[0] + rhat[1] * kap[1] + rhat[2] * kap[2]) / R;
    sigma = 1.0 / sqrt(phi);
    amin_i = fmin(P->axes[0], fmin(P->axes[1], P->axes[2]));
    amin_j = amin_i;
    smin = wall ? P->sigmin_wall : sqrt(2.0 * (amin_i * amin_i + amin_j * amin_j));
    rho = (R - sigma + smin) / smin;
    if (rho <= 0.0) return ORC_EOVERLAP;
    if (pow(rho, 6.0) > 2.0) return ORC_OK;
    *U = 4.0 * P->eps0 * (pow(rho, -12.0) - pow(rho, -6.0)) + P->eps0;
    dudr = -24.0 * P->eps0 * (2.0 * pow(rho, -13.0) - pow(rho, -7.0)) / smin;
    dudphi = -24.0 * P->eps0 * (2.0 * pow(rho, -13.0) - pow(rho, -7.0)) * sigma * sigma * sigma /
             (2.0 * smin);
    kr = kap[0] * rhat[0] + kap[1] * rhat[1] + kap[2] * rhat[2];
    for (k = 0; k < 3; ++k)
        F[k] = -dudr * rhat[k] - dudphi / (R * R) * (kap[k] - kr * rhat[k]);
    mat_vec(Ai, kap, Aik);
    mat_vec(Aj, kap, Ajk);
    for (k = 0; k < 3; ++k) fk[k] = -dudphi / R * kap[k];
    {
        double Rci[3], Rcj[3], ci[3], cj[3];
        for (k = 0; k < 3; ++k) { Rci[k] = -Aik[k]; Rcj[k] = Ajk[k]; }
        cross(Rci, fk, ci);
        cross(Rcj, fk, cj);
        for (k = 0; k < 3; ++k) { ti[k] = ci[k] / R; tj[k] = -cj[k] / R; }
    }
    return ORC_OK;
}

int orc_gb_pair(const orc_params* prm, const double Ri[3], const double Qi[9],
                const double Rj[3], const double Qj[9], int wall, double* U, double F[3],
                double taui[3], double tauj[3])
{
    double rij[3];
    int k;
    for (k = 0; k < 3; ++k) rij[k] = Ri[k] - Rj[k];
    return gb_pair_core(prm, rij, Qi, Qj, wall, U, F, taui, tauj);
}

/* ---------------------------------------------------------------------------------- */
/* Rigid-body integrator (App. A). Translation in the lab frame, rotation in the body
 * frame. Readings: the garbled subscripts of steps 2, 6 and 7 mean "apply to the
 * running value"; the printed skew(v) is the negative of the cross-product matrix used
 * by the Euler equation (A2), so Q' = Q hat(Omega) is taken, for which the free
 * sub-rotation about body axis k by phi = f h Omega_k is R = Rot_k(-phi):
 * pi <- R pi, Q <- Q R^T. */
static void rot_axis(int k, double ang, double* M)
{
    double c = cos(ang), s = sin(ang);
    int a;
    for (a = 0; a < 9; ++a) M[a] = 0.0;
    if (k == 0) { M[0] = 1; M[4] = c; M[5] = -s; M[7] = s; M[8] = c; }
    if (k == 1) { M[4] = 1; M[0] = c; M[2] = s; M[6] = -s; M[8] = c; }
    if (k == 2) { M[8] = 1; M[0] = c; M[1] = -s; M[3] = s; M[4] = c; }
}

static void first_half(const orc_params* P, const double L[3], const int per[3],
                       double R[3], double Q[9], double V[3], double Om[3],
                       const double Fc[3], const double Tc[3])
{
    static const int axis_seq[5] = {0, 1, 2, 1, 0};
    static const double frac[5] = {0.5, 0.5, 1.0, 0.5, 0.5};
    const double h = 1.0;
    double eT = exp(-P->gammaT * h / 2.0), eR = exp(-P->gammaR * h / 2.0);
    int a, st;
    /* step 1: half kick with the combined force and torque */
    for (a = 0; a < 3; ++a) {
        V[a] += h / (2.0 * P->mass) * Fc[a];
        Om[a] += h / 2.0 * Tc[a] / P->inertia[a];
    }
    /* step 2: friction over half a step */
    for (a = 0; a < 3; ++a) { V[a] *= eT; Om[a] *= eR; }
    /* step 3: drift; positions wrapped into [0, L) on periodic axes */
    for (a = 0; a < 3; ++a) {
        R[a] += h * V[a];
        if (per[a]) {
            if (R[a] >= L[a]) R[a] -= L[a];
            else if (R[a] < 0.0) R[a] += L[a];
        }
    }
    /* step 4: five free sub-rotations n/2, t/2, g, t/2, n/2 */
    for (st = 0; st < 5; ++st) {
        int k = axis_seq[st];
        double phi = frac[st] * h * Om[k];
        double M[9], pi[3], pin[3], Qn[9];
        int r, c, m;
        rot_axis(k, -phi, M);
        for (a = 0; a < 3; ++a) pi[a] = P->inertia[a] * Om[a];
        mat_vec(M, pi, pin);
        for (a = 0; a < 3; ++a) Om[a] = pin[a] / P->inertia[a];
        for (r = 0; r < 3; ++r)
            for (c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (m = 0; m < 3; ++m) acc += Q[3 * r + m] * M[3 * c + m]; /* Q M^T */
                Qn[3 * r + c] = acc;
            }
        memcpy(Q, Qn, sizeof Qn);
    }
}

static void second_half(const orc_params* P, double V[3], double Om[3], const double Fc[3],
                        const double Tc[3])
{
    const double h = 1.0;
    double eT = exp(-P->gammaT * h / 2.0), eR = exp(-P->gammaR * h / 2.0);
    int a;
    /* step 6: friction over half a step */
    for (a = 0; a < 3; ++a) { V[a] *= eT; Om[a] *= eR; }
    /* step 7: half kick with the new combined force and torque */
    for (a = 0; a < 3; ++a) {
        V[a] += h / (2.0 * P->mass) * Fc[a];
        Om[a] += h / 2.0 * Tc[a] / P->inertia[a];
    }
}

void orc_rigid_step(const orc_params* prm, double R[3], double Q[9], double V[3],
                    double Om[3], const double F[3], const double T[3])
{
    double L[3] = {prm->nx, prm->ny, prm->nz};
    first_half(prm, L, prm->periodic, R, Q, V, Om, F, T);
    second_half(prm, V, Om, F, T);
}

/* ---------------------------------------------------------------------------------- */
/* Cell list. Cut-off: sigma_ij <= sqrt(2 (amax_i^2 + amax_j^2)), so a pair (cell-cell or
 * cell-wall) interacts only within r_c = max over pair kinds of that bound plus
 * (2^(1/6) - 1) sigma_min. Cells per axis = floor(L / r_c) (at least 1), edge L / count;
 * a centre falls in cell floor(R_a / edge_a), clamped to the grid. */
static void setup_cell_grid(orc_sim* s)
{
    const orc_params* P = &s->P;
    double amax = fmax(P->axes[0], fmax(P->axes[1], P->axes[2]));
    double amin = fmin(P->axes[0], fmin(P->axes[1], P->axes[2]));
    double sm = sqrt(2.0 * (amin * amin + amin * amin));
    double rc_cc = sqrt(2.0 * (amax * amax + amax * amax)) + (pow(2.0, 1.0 / 6.0) - 1.0) * sm;
    double rc_cw = sqrt(2.0 * (amax * amax + P->a_wall * P->a_wall)) +
                   (pow(2.0, 1.0 / 6.0) - 1.0) * P->sigmin_wall;
    int a;
    s->rc = fmax(rc_cc, rc_cw);
    for (a = 0; a < 3; ++a) {
        double L = box_len(s, a);
        int n = (int)floor(L / s->rc);
        if (n < 1) n = 1;
        s->ncell[a] = n;
        s->cedge[a] = L / n;
    }
}

static int cell_coord(const orc_sim* s, int a, double x)
{
    int c = (int)floor(x / s->cedge[a]);
    if (c < 0) c = 0;
    if (c >= s->ncell[a]) c = s->ncell[a] - 1;
    return c;
}

static int cell_index(const orc_sim* s, const double r[3])
{
    int cx = cell_coord(s, 0, r[0]), cy = cell_coord(s, 1, r[1]), cz = cell_coord(s, 2, r[2]);
    return cx + s->ncell[0] * (cy + s->ncell[1] * cz);
}

/* Counting sort of the cell centres; ids ascend within each cell. */
static void build_cell_list(orc_sim* s)
{
    int nc = s->ncell[0] * s->ncell[1] * s->ncell[2];
    int i, c;
    int* cnt = (int*)calloc((size_t)nc, sizeof(int));
    for (i = 0; i < s->nrbc; ++i) cnt[cell_index(s, s->R + 3 * i)]++;
    s->cell_off[0] = 0;
    for (c = 0; c < nc; ++c) s->cell_off[c + 1] = s->cell_off[c] + cnt[c];
    for (c = 0; c < nc; ++c) cnt[c] = 0;
    for (i = 0; i < s->nrbc; ++i) {
        int ci = cell_index(s, s->R + 3 * i);
        s->cell_ids[s->cell_off[ci] + cnt[ci]++] = i;
    }
    free(cnt);
}

/* Neighbouring cells of cell (cx, cy, cz): offsets -1..1 per axis, wrapped on periodic
 * axes; an axis with fewer than three cells lists each of its cells once. */
static int neighbour_cells(const orc_sim* s, int cx, int cy, int cz, int* out)
{
    int lst[3][3], cnt[3], a, n = 0, i, j, k;
    int cc[3] = {cx, cy, cz};
    for (a = 0; a < 3; ++a) {
        int m = s->ncell[a];
        cnt[a] = 0;
        if (m < 3) {
            for (i = 0; i < m; ++i) lst[a][cnt[a]++] = i;
        } else {
            for (i = -1; i <= 1; ++i) {
                int v = cc[a] + i;
                if (v < 0 || v >= m) {
                    if (!s->P.periodic[a]) continue;
                    v = wrapi(v, m);
                }
                lst[a][cnt[a]++] = v;
            }
        }
    }
    for (k = 0; k < cnt[2]; ++k)
        for (j = 0; j < cnt[1]; ++j)
            for (i = 0; i < cnt[0]; ++i)
                out[n++] = lst[0][i] + s->ncell[0] * (lst[1][j] + s->ncell[1] * lst[2][k]);
    return n;
}

/* Wall particles: solid nodes with at least one fluid D3Q19 neighbour. */
static void build_walls(orc_sim* s)
{
    long n;
    int nc = s->ncell[0] * s->ncell[1] * s->ncell[2];
    int w, c, *cnt;
    s->nwall = 0;
    for (n = 0; n < s->N; ++n) {
        int x, y, z, p, adj = 0;
        if (!s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        for (p = 1; p < 19; ++p)
            if (fluid_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2])) adj = 1;
        if (adj) s->nwall++;
    }
    s->wall_xyz = (int*)malloc(sizeof(int) * 3 * (size_t)(s->nwall + 1));
    w = 0;
    for (n = 0; n < s->N; ++n) {
        int x, y, z, p, adj = 0;
        if (!s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        for (p = 1; p < 19; ++p)
            if (fluid_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2])) adj = 1;
        if (adj) {
            s->wall_xyz[3 * w] = x; s->wall_xyz[3 * w + 1] = y; s->wall_xyz[3 * w + 2] = z;
            ++w;
        }
    }
    s->wcell_off = (int*)calloc((size_t)nc + 1, sizeof(int));
    s->wcell_ids = (int*)malloc(sizeof(int) * (size_t)(s->nwall + 1));
    cnt = (int*)calloc((size_t)nc, sizeof(int));
    for (w = 0; w < s->nwall; ++w) {
        double r[3] = {s->wall_xyz[3 * w], s->wall_xyz[3 * w + 1], s->wall_xyz[3 * w + 2]};
        cnt[cell_index(s, r)]++;
    }
    for (c = 0; c < nc; ++c) s->wcell_off[c + 1] = s->wcell_off[c] + cnt[c];
    for (c = 0; c < nc; ++c) cnt[c] = 0;
    for (w = 0; w < s->nwall; ++w) {
        double r[3] = {s->wall_xyz[3 * w], s->wall_xyz[3 * w + 1], s->wall_xyz[3 * w + 2]};
        int ci = cell_index(s, r);
        s->wcell_ids[s->wcell_off[ci] + cnt[ci]++] = w;
    }
    free(cnt);
}

/* Wall-adjacent fluid nodes and their unit wall normal: the normalised sum of w_p c_p
 * over the directions p whose neighbour x + c_p is solid (points into the wall). */
static void build_wall_nodes(orc_sim* s)
{
    long n;
    int k = 0;
    s->nwn = 0;
    for (n = 0; n < s->N; ++n) {
        int x, y, z, p, adj = 0;
        if (s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        for (p = 1; p < 19; ++p)
            if (!fluid_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2]) &&
                node_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2]) >= 0) adj = 1;
        if (adj) s->nwn++;
    }
    s->wn_node = (long*)malloc(sizeof(long) * (size_t)(s->nwn + 1));
    s->wn_nrm = (double*)malloc(sizeof(double) * 3 * (size_t)(s->nwn + 1));
    for (n = 0; n < s->N; ++n) {
        int x, y, z, p, adj = 0;
        double v[3] = {0, 0, 0}, len;
        if (s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        for (p = 1; p < 19; ++p)
            if (!fluid_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2]) &&
                node_at(s, x + CV[p][0], y + CV[p][1], z + CV[p][2]) >= 0) {
                adj = 1;
                v[0] += WV[p] * CV[p][0]; v[1] += WV[p] * CV[p][1]; v[2] += WV[p] * CV[p][2];
            }
        if (!adj) continue;
        len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        s->wn_node[k] = n;
        if (len > 0.0) { v[0] /= len; v[1] /= len; v[2] /= len; }
        s->wn_nrm[3 * k] = v[0]; s->wn_nrm[3 * k + 1] = v[1]; s->wn_nrm[3 * k + 2] = v[2];
        ++k;
    }
}

/* ---------------------------------------------------------------------------------- */
/* Step 3: node -> cell coverage. A fluid node is covered by cell i if it, or one of its
 * six axis neighbours that is fluid, lies inside the support of i: exactly the nodes
 * where the normalised kernel or its central-difference gradient can be non-zero. Cells
 * are visited in ascending order, so each node's list ascends. */
static int covered(const orc_sim* s, int i, int x, int y, int z)
{
    static const int nb[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                 {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    int k;
    if (!fluid_at(s, x, y, z)) return 0;
    for (k = 0; k < 7; ++k) {
        long m = node_at(s, x + nb[k][0], y + nb[k][1], z + nb[k][2]);
        int xn[3];
        if (m < 0 || s->solid[m]) continue;
        node_xyz(s, m, &xn[0], &xn[1], &xn[2]);
        if (inside(s, i, xn)) return 1;
    }
    return 0;
}

static void build_map(orc_sim* s)
{
    int hw = support_halfwidth(s);
    int i, pass;
    long n;
    long* cnt = (long*)calloc((size_t)s->N, sizeof(long));
    for (pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            s->map_off[0] = 0;
            for (n = 0; n < s->N; ++n) s->map_off[n + 1] = s->map_off[n] + cnt[n];
            s->map_len = s->map_off[s->N];
            if (s->map_len > s->map_alloc) {
                free(s->map_ids);
                s->map_alloc = s->map_len + 1024;
                s->map_ids = (int*)malloc(sizeof(int) * (size_t)s->map_alloc);
            }
            memset(cnt, 0, sizeof(long) * (size_t)s->N);
        }
        for (i = 0; i < s->nrbc; ++i) {
            int cx = (int)floor(s->R[3 * i]), cy = (int)floor(s->R[3 * i + 1]),
                cz = (int)floor(s->R[3 * i + 2]);
            int dx, dy, dz;
            for (dz = -hw; dz <= hw; ++dz)
                for (dy = -hw; dy <= hw; ++dy)
                    for (dx = -hw; dx <= hw; ++dx) {
                        long m = node_at(s, cx + dx, cy + dy, cz + dz);
                        int xn[3];
                        if (m < 0) continue;
                        node_xyz(s, m, &xn[0], &xn[1], &xn[2]);
                        if (!covered(s, i, xn[0], xn[1], xn[2])) continue;
                        if (pass == 1) s->map_ids[s->map_off[m] + cnt[m]] = i;
                        cnt[m]++;
                    }
        }
    }
    free(cnt);
}

/* ---------------------------------------------------------------------------------- */
/* Step 4: smeared fields (Eqs. 20-21) and the elongational torque (Eqs. 16, 19).
 * Vorticity is the curl of u (Sec. II B) by second-order central differences, with u = 0
 * on solid nodes. n^ = grad(delta)/|grad(delta)| (0 where the gradient vanishes) and
 * T^S = alpha sum delta (sigma . n^) x (x - R), as printed. */
static void u_at(const orc_sim* s, int x, int y, int z, double out[3])
{
    long n = node_at(s, x, y, z);
    if (n < 0 || s->solid[n]) { out[0] = out[1] = out[2] = 0.0; return; }
    out[0] = s->u[3 * n]; out[1] = s->u[3 * n + 1]; out[2] = s->u[3 * n + 2];
}

static void vorticity_at(const orc_sim* s, int x, int y, int z, double w[3])
{
    double xp[3], xm[3], yp[3], ym[3], zp[3], zm[3];
    u_at(s, x + 1, y, z, xp); u_at(s, x - 1, y, z, xm);
    u_at(s, x, y + 1, z, yp); u_at(s, x, y - 1, z, ym);
    u_at(s, x, y, z + 1, zp); u_at(s, x, y, z - 1, zm);
    w[0] = 0.5 * (yp[2] - ym[2]) - 0.5 * (zp[1] - zm[1]);
    w[1] = 0.5 * (zp[0] - zm[0]) - 0.5 * (xp[2] - xm[2]);
    w[2] = 0.5 * (xp[1] - xm[1]) - 0.5 * (yp[0] - ym[0]);
}

static void interpolate_cell(orc_sim* s, int i)
{
    int hw = support_halfwidth(s);
    int cx = (int)floor(s->R[3 * i]), cy = (int)floor(s->R[3 * i + 1]),
        cz = (int)floor(s->R[3 * i + 2]);
    int dx, dy, dz, a;
    double S = 0.0, ut[3] = {0, 0, 0}, wt[3] = {0, 0, 0}, ts[3] = {0, 0, 0};
    /* normalisation over the fluid nodes of the support */
    for (dz = -hw; dz <= hw; ++dz)
        for (dy = -hw; dy <= hw; ++dy)
            for (dx = -hw; dx <= hw; ++dx) {
                long m = node_at(s, cx + dx, cy + dy, cz + dz);
                int xn[3];
                if (m < 0 || s->solid[m]) continue;
                node_xyz(s, m, &xn[0], &xn[1], &xn[2]);
                if (inside(s, i, xn)) S += delta_raw(s, i, xn);
            }
    s->S[i] = S;
    for (dz = -hw; dz <= hw; ++dz)
        for (dy = -hw; dy <= hw; ++dy)
            for (dx = -hw; dx <= hw; ++dx) {
                int x = cx + dx, y = cy + dy, z = cz + dz;
                long m = node_at(s, x, y, z);
                double dh, w[3], gr[3], gl, nh[3], t[3], d[3], c[3];
                const double* sg;
                int xn[3];
                if (m < 0 || s->solid[m]) continue;
                node_xyz(s, m, &xn[0], &xn[1], &xn[2]);
                if (!inside(s, i, xn)) continue;
                dh = delta_hat(s, i, x, y, z);
                for (a = 0; a < 3; ++a) ut[a] += dh * s->u[3 * m + a];
                vorticity_at(s, x, y, z, w);
                for (a = 0; a < 3; ++a) wt[a] += dh * w[a];
                grad_delta_hat(s, i, x, y, z, gr);
                gl = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
                for (a = 0; a < 3; ++a) nh[a] = gl > 0.0 ? gr[a] / gl : 0.0;
                sg = s->sig + 6 * m; /* xx yy zz xy xz yz */
                t[0] = sg[0] * nh[0] + sg[3] * nh[1] + sg[4] * nh[2];
                t[1] = sg[3] * nh[0] + sg[1] * nh[1] + sg[5] * nh[2];
                t[2] = sg[4] * nh[0] + sg[5] * nh[1] + sg[2] * nh[2];
                for (a = 0; a < 3; ++a) d[a] = (double)xn[a] - s->R[3 * i + a];
                min_image(s, d);
                cross(t, d, c);
                for (a = 0; a < 3; ++a) ts[a] += s->P.alpha * dh * c[a];
            }
    for (a = 0; a < 3; ++a) {
        s->ut[3 * i + a] = ut[a];
        s->wt[3 * i + a] = wt[a];
        s->TS[3 * i + a] = ts[a];
    }
}

/* ---------------------------------------------------------------------------------- */
/* Step 5: Gay-Berne forces (lab) and torques (body frame) of every cell. */
static int collide_one(orc_sim* s, int i, int brute, double F[3], double T[3])
{
    double tl[3] = {0, 0, 0};
    int k, st;
    F[0] = F[1] = F[2] = 0.0;
    if (brute) {
        int j, w;
        for (j = 0; j < s->nrbc; ++j) {
            double rij[3], U, f[3], ti[3], tj[3];
            if (j == i) continue;
            for (k = 0; k < 3; ++k) rij[k] = s->R[3 * i + k] - s->R[3 * j + k];
            min_image(s, rij);
            st = gb_pair_core(&s->P, rij, s->Q + 9 * i, s->Q + 9 * j, 0, &U, f, ti, tj);
            if (st) return st;
            for (k = 0; k < 3; ++k) { F[k] += f[k]; tl[k] += ti[k]; }
        }
        if (s->P.wall_particles)
            for (w = 0; w < s->nwall; ++w) {
                double rij[3], U, f[3], ti[3], tj[3];
                for (k = 0; k < 3; ++k) rij[k] = s->R[3 * i + k] - s->wall_xyz[3 * w + k];
                min_image(s, rij);
                st = gb_pair_core(&s->P, rij, s->Q + 9 * i, NULL, 1, &U, f, ti, tj);
                if (st) return st;
                for (k = 0; k < 3; ++k) { F[k] += f[k]; tl[k] += ti[k]; }
            }
    } else {
        int cells[27], nn, c;
        int cx = cell_coord(s, 0, s->R[3 * i]), cy = cell_coord(s, 1, s->R[3 * i + 1]),
            cz = cell_coord(s, 2, s->R[3 * i + 2]);
        nn = neighbour_cells(s, cx, cy, cz, cells);
        for (c = 0; c < nn; ++c) {
            int e;
            for (e = s->cell_off[cells[c]]; e < s->cell_off[cells[c] + 1]; ++e) {
                int j = s->cell_ids[e];
                double rij[3], U, f[3], ti[3], tj[3], r2;
                if (j == i) continue;
                for (k = 0; k < 3; ++k) rij[k] = s->R[3 * i + k] - s->R[3 * j + k];
                min_image(s, rij);
                r2 = rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2];
                if (r2 > s->rc * s->rc) continue; /* beyond every possible cut-off */
                st = gb_pair_core(&s->P, rij, s->Q + 9 * i, s->Q + 9 * j, 0, &U, f, ti, tj);
                if (st) return st;
                for (k = 0; k < 3; ++k) { F[k] += f[k]; tl[k] += ti[k]; }
            }
            if (!s->P.wall_particles) continue;
            for (e = s->wcell_off[cells[c]]; e < s->wcell_off[cells[c] + 1]; ++e) {
                int w = s->wcell_ids[e];
                double rij[3], U, f[3], ti[3], tj[3], r2;
                for (k = 0; k < 3; ++k) rij[k] = s->R[3 * i + k] - s->wall_xyz[3 * w + k];
                min_image(s, rij);
                r2 = rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2];
                if (r2 > s->rc * s->rc) continue;
                st = gb_pair_core(&s->P, rij, s->Q + 9 * i, NULL, 1, &U, f, ti, tj);
                if (st) return st;
                for (k = 0; k < 3; ++k) { F[k] += f[k]; tl[k] += ti[k]; }
            }
        }
    }
    matT_vec(s->Q + 9 * i, tl, T); /* torque to the body frame */
    return ORC_OK;
}

static int collide_all(orc_sim* s, int brute)
{
    int i, err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : err) if (s->nrbc >= ORC_PAR_CELLS)
    for (i = 0; i < s->nrbc; ++i) {
        int st = collide_one(s, i, brute, s->Fmech + 3 * i, s->Tmech + 3 * i);
        if (st > err) err = st;
    }
    return err;
}

/* ---------------------------------------------------------------------------------- */
/* Step 6 pieces. Combined force/torque (App. A, step 5), with two readings: the
 * translational/rotational friction carries the mass and inertia (F = -M gT (V - u~),
 * T^A = -gR I (Omega - Q^T w~)), as the integrator's M gT u~ and I gR w~ terms require;
 * and tau^comb includes the elongational torque Q^T T^S, without which alpha would have
 * no effect on the cell. A constant external force (lab) and torque (body) on every cell,
 * as a drag experiment applies (Sec. III, single-cell mobilities), add to the mechanical
 * ones. */
static void combined(const orc_sim* s, int i, double Fc[3], double Tc[3])
{
    const orc_params* P = &s->P;
    double wb[3], tsb[3];
    int a;
    matT_vec(s->Q + 9 * i, s->wt + 3 * i, wb);
    matT_vec(s->Q + 9 * i, s->TS + 3 * i, tsb);
    for (a = 0; a < 3; ++a) {
        Fc[a] = s->Fmech[3 * i + a] + P->ext_force[a] + P->gammaT * P->mass * s->ut[3 * i + a];
        Tc[a] = s->Tmech[3 * i + a] + P->ext_torque[a] + tsb[a] +
                P->gammaR * P->inertia[a] * P->vort_scale * wb[a];
    }
}

/* Force and torque the cell receives from the plasma (lab frame), from the mid-step
 * V and Omega of this step: F^hyd = -M gT (V - u~), T^hyd = Q [-gR I (Omega - s Q^T w~)] + T^S. */
static void hydrodynamic(orc_sim* s, int i, const double* V, const double* Om)
{
    const orc_params* P = &s->P;
    double wb[3], tb[3], tl[3];
    int a;
    matT_vec(s->Q + 9 * i, s->wt + 3 * i, wb);
    for (a = 0; a < 3; ++a) {
        s->Fhyd[3 * i + a] = -P->mass * P->gammaT * (V[a] - s->ut[3 * i + a]);
        tb[a] = -P->gammaR * P->inertia[a] * (Om[a] - P->vort_scale * wb[a]);
    }
    mat_vec(s->Q + 9 * i, tb, tl);
    for (a = 0; a < 3; ++a) s->Thyd[3 * i + a] = tl[a] + s->TS[3 * i + a];
}

/* ---------------------------------------------------------------------------------- */
/* Step 7: back-reaction and local relaxation time at every fluid node.
 * G = g_ext - sum_i [F_i delta_i - (1/2) T_i x grad(delta_i)] over the covering cells in
 * ascending order. The torque term's sign is the reading taken: with the printed
 * "+ (1/2) T x grad(delta)" inside the bracket the plasma's angular momentum about R_i
 * (sum of (x - R_i) x G) changes by +T_i, i.e. in the same sense as the cell's; the
 * paper's own derivation of Eq. 22 drops the minus sign of G and uses c x (x - R), the
 * negative of the angular momentum. The sign here gives -T_i, the opposite reaction the
 * text states (exact on a periodic lattice, see Eq. 13).
 * Viscosity contrast, Eq. 23: T(x) = T0 + Delta sum_i [1 - (1 - delta_i)^kappa] with the
 * unnormalised kernel (centre value 1/8 gives theta = 0.93 at kappa = 20, i.e. "theta ~ 1
 * inside"; the normalised kernel would give about 0.6). */
static void spread(orc_sim* s)
{
    long n;
#pragma omp parallel for schedule(static) if (s->N >= ORC_PAR_NODES)
    for (n = 0; n < s->N; ++n) {
        int x, y, z, a;
        long e;
        double g[3], theta = 0.0;
        if (s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        for (a = 0; a < 3; ++a) g[a] = s->P.g_ext[a];
        for (e = s->map_off[n]; e < s->map_off[n + 1]; ++e) {
            int i = s->map_ids[e];
            int xn[3] = {x, y, z};
            double dh = delta_hat(s, i, x, y, z), gr[3], txg[3], draw;
            grad_delta_hat(s, i, x, y, z, gr);
            cross(s->Thyd + 3 * i, gr, txg);
            for (a = 0; a < 3; ++a) g[a] -= s->Fhyd[3 * i + a] * dh - 0.5 * txg[a];
            draw = delta_raw(s, i, xn);
            theta += 1.0 - pow(1.0 - draw, s->P.kappa);
        }
        for (a = 0; a < 3; ++a) s->g[3 * n + a] = g[a];
        s->Trel[n] = s->P.tau0 + s->P.delta_visc * theta;
    }
}

/* ---------------------------------------------------------------------------------- */
/* Step 8: pull streaming (Eq. 1) with halfway bounce-back on resting walls, moments
 * (Eqs. 5-6), BGK relaxation with the body-force term (Eqs. 2-4) at the local T, and the
 * shear stress of the non-equilibrium part (Eq. 8). Eq. 8 as printed has the sign of
 * +sum c c (f - f^eq), opposite to its left-hand side nu rho (du + du^T); the stored
 * stress is sigma = -(1 - 1/(2T)) sum c c (f - f^eq), with nu/(c^2 T) = 1 - 1/(2T). */
/* Velocity of the wall at a solid (or outside) source row ys: the solid nodes below the box's
 * mid-plane y = ny/2 move with wall_u_lo, the others with wall_u_hi (both zero: resting walls). */
static const double* wall_velocity(const orc_sim* s, int ys)
{
    return 2 * ys < s->ny ? s->P.wall_u_lo : s->P.wall_u_hi;
}

/* Halfway bounce-back from a wall moving with velocity u_w (Ladd 1994): the population that
 * left x towards the wall along -c_p comes back along c_p with the momentum the wall hands it,
 * f_p(x) = f*_{opp(p)}(x) + 2 w_p rho_w (c_p . u_w) / c^2, with the wall density rho_w = 1. */
static double bounce_back_term(const orc_sim* s, int p, int ys)
{
    const double* uw = wall_velocity(s, ys);
    return 2.0 * WV[p] * (CV[p][0] * uw[0] + CV[p][1] * uw[1] + CV[p][2] * uw[2]) / CS2;
}

static void pulled(const orc_sim* s, long n, int x, int y, int z, double f[19])
{
    int p;
    for (p = 0; p < 19; ++p) {
        long src = node_at(s, x - CV[p][0], y - CV[p][1], z - CV[p][2]);
        if (src < 0 || s->solid[src])
            f[p] = s->f[(long)opposite(p) * s->N + n] + bounce_back_term(s, p, y - CV[p][1]);
        else f[p] = s->f[(long)p * s->N + src];
    }
}

static void moments(const double f[19], double* rho, double m[3])
{
    int p;
    *rho = 0.0; m[0] = m[1] = m[2] = 0.0;
    for (p = 0; p < 19; ++p) {
        *rho += f[p];
        m[0] += f[p] * CV[p][0]; m[1] += f[p] * CV[p][1]; m[2] += f[p] * CV[p][2];
    }
}

static int stream_collide(orc_sim* s)
{
    long n;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) if (s->N >= ORC_PAR_NODES)
    for (n = 0; n < s->N; ++n) {
        int x, y, z, p, a;
        double f[19], rho, m[3], u[3], T, Pn[6] = {0, 0, 0, 0, 0, 0}, k;
        const double* g = s->g + 3 * n;
        if (s->solid[n]) continue;
        node_xyz(s, n, &x, &y, &z);
        if (open_plane(s, z)) continue; /* done below */
        pulled(s, n, x, y, z, f);
        moments(f, &rho, m);
        for (a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * g[a]) / rho;
        T = s->Trel[n];
        for (p = 0; p < 19; ++p) {
            double fe = orc_feq(rho, u, p), neq = f[p] - fe;
            const int* c = CV[p];
            s->fnew[(long)p * s->N + n] =
                f[p] - (f[p] - fe) / T + orc_force_term(s->P.forcing, T, g, u, p);
            Pn[0] += c[0] * c[0] * neq; Pn[1] += c[1] * c[1] * neq; Pn[2] += c[2] * c[2] * neq;
            Pn[3] += c[0] * c[1] * neq; Pn[4] += c[0] * c[2] * neq; Pn[5] += c[1] * c[2] * neq;
        }
        k = -(1.0 - 1.0 / (2.0 * T));
        for (a = 0; a < 6; ++a) s->sig[6 * n + a] = k * Pn[a];
        for (a = 0; a < 3; ++a) s->u[3 * n + a] = u[a];
        if (!(rho > 0.0) || !(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 0.09)) bad = 1;
    }
    /* Open z faces: non-equilibrium extrapolation (Guo, Zheng & Shi 2002). The boundary
     * node takes the prescribed density, the velocity of its interior z-neighbour and
     * that neighbour's non-equilibrium part, relaxed at the boundary node's T. */
    if (s->P.open_z) {
        for (n = 0; n < s->N; ++n) {
            int x, y, z, p, a, zi;
            long ni;
            double f[19], rho, m[3], u[3], rb, T;
            const double* g;
            if (s->solid[n]) continue;
            node_xyz(s, n, &x, &y, &z);
            if (!open_plane(s, z)) continue;
            zi = (z == 0) ? 1 : s->nz - 2;
            ni = node_at(s, x, y, zi);
            rb = (z == 0) ? s->P.rho_in : s->P.rho_out;
            T = s->Trel[n];
            if (ni < 0 || s->solid[ni]) {
                for (p = 0; p < 19; ++p) {
                    double zero[3] = {0, 0, 0};
                    s->fnew[(long)p * s->N + n] = orc_feq(rb, zero, p);
                }
                for (a = 0; a < 3; ++a) s->u[3 * n + a] = 0.0;
                for (a = 0; a < 6; ++a) s->sig[6 * n + a] = 0.0;
                continue;
            }
            pulled(s, ni, x, y, zi, f);
            moments(f, &rho, m);
            g = s->g + 3 * ni;
            for (a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * g[a]) / rho;
            for (p = 0; p < 19; ++p)
                s->fnew[(long)p * s->N + n] =
                    orc_feq(rb, u, p) + (1.0 - 1.0 / T) * (f[p] - orc_feq(rho, u, p));
            for (a = 0; a < 3; ++a) s->u[3 * n + a] = u[a];
            for (a = 0; a < 6; ++a) s->sig[6 * n + a] = 0.0;
        }
    }
    /* momentum handed to the walls by bounce-back in this step */
    {
        double wm[3] = {0, 0, 0};
        for (n = 0; n < s->N; ++n) {
            int x, y, z, p;
            if (s->solid[n]) continue;
            node_xyz(s, n, &x, &y, &z);
            if (open_plane(s, z)) continue;
            for (p = 1; p < 19; ++p) {
                long src = node_at(s, x - CV[p][0], y - CV[p][1], z - CV[p][2]);
                if (src < 0 || s->solid[src]) {
                    /* the fluid gains c_p (f_back + f_out): the wall takes the opposite */
                    const double fo = s->f[(long)opposite(p) * s->N + n];
                    const double fb = fo + bounce_back_term(s, p, y - CV[p][1]);
                    wm[0] -= (fo + fb) * CV[p][0];
                    wm[1] -= (fo + fb) * CV[p][1];
                    wm[2] -= (fo + fb) * CV[p][2];
                }
            }
        }
        s->wall_mom[0] = wm[0]; s->wall_mom[1] = wm[1]; s->wall_mom[2] = wm[2];
    }
    {
        double* t = s->f; s->f = s->fnew; s->fnew = t;
    }
    return bad ? ORC_EUNSTABLE : ORC_OK;
}

/* ---------------------------------------------------------------------------------- */
static int couple_cells(orc_sim* s)
{
    int i;
    build_cell_list(s);
    build_map(s);
#pragma omp parallel for schedule(dynamic, 4) if (s->nrbc >= ORC_PAR_CELLS)
    for (i = 0; i < s->nrbc; ++i) interpolate_cell(s, i);
    return ORC_OK;
}

static int one_step(orc_sim* s)
{
    int i, st;
    /* 1 */
    for (i = 0; i < s->nrbc; ++i) {
        double L[3] = {s->nx, s->ny, s->nz};
        first_half(&s->P, L, s->P.periodic, s->R + 3 * i, s->Q + 9 * i, s->V + 3 * i,
                   s->Om + 3 * i, s->Fcomb + 3 * i, s->Tcomb + 3 * i);
        memcpy(s->Vh + 3 * i, s->V + 3 * i, 3 * sizeof(double));
        memcpy(s->Omh + 3 * i, s->Om + 3 * i, 3 * sizeof(double));
    }
    /* 2, 3, 4 */
    couple_cells(s);
    /* 5 */
    st = collide_all(s, 0);
    if (st) return st;
    /* 6 */
    for (i = 0; i < s->nrbc; ++i) {
        combined(s, i, s->Fcomb + 3 * i, s->Tcomb + 3 * i);
        hydrodynamic(s, i, s->Vh + 3 * i, s->Omh + 3 * i);
        second_half(&s->P, s->V + 3 * i, s->Om + 3 * i, s->Fcomb + 3 * i, s->Tcomb + 3 * i);
    }
    /* 7 */
    spread(s);
    /* 8 */
    st = stream_collide(s);
    s->step++;
    return st;
}

int orc_step(orc_sim* s, int nsteps)
{
    int k, st;
    for (k = 0; k < nsteps; ++k) {
        st = one_step(s);
        if (st) return st;
    }
    return ORC_OK;
}

int orc_couple(orc_sim* s)
{
    int i;
    couple_cells(s);
    for (i = 0; i < s->nrbc; ++i) hydrodynamic(s, i, s->V + 3 * i, s->Om + 3 * i);
    spread(s);
    return ORC_OK;
}

int orc_collide(orc_sim* s, int brute, double* F, double* T)
{
    int st;
    build_cell_list(s);
    st = collide_all(s, brute);
    if (F) memcpy(F, s->Fmech, sizeof(double) * 3 * (size_t)s->nrbc);
    if (T) memcpy(T, s->Tmech, sizeof(double) * 3 * (size_t)s->nrbc);
    return st;
}

/* ---------------------------------------------------------------------------------- */
orc_sim* orc_create(const orc_params* prm, const uint8_t* solid, int n_rbc, const double* R,
                    const double* Q, const double* V, const double* Om, int* status)
{
    orc_sim* s;
    long n;
    int p, i, a, nc;
    *status = ORC_EINVAL;
    if (prm->nx < 1 || prm->ny < 1 || prm->nz < 1 || !(prm->tau0 > 0.5) || n_rbc < 0)
        return NULL;
    if (n_rbc > 0 && (!(prm->mass > 0) || !(prm->inertia[0] > 0) || !(prm->inertia[1] > 0) ||
                      !(prm->inertia[2] > 0) || !(prm->xi[0] > 0) || !(prm->xi[1] > 0) ||
                      !(prm->xi[2] > 0) || !(prm->eps0 > 0)))
        return NULL;
    if (prm->open_z && prm->periodic[2]) return NULL;
    s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->P = *prm;
    s->nx = prm->nx; s->ny = prm->ny; s->nz = prm->nz;
    s->N = (long)prm->nx * prm->ny * prm->nz;
    s->solid = (uint8_t*)malloc((size_t)s->N);
    memcpy(s->solid, solid, (size_t)s->N);
    s->f = (double*)malloc(sizeof(double) * 19 * (size_t)s->N);
    s->fnew = (double*)malloc(sizeof(double) * 19 * (size_t)s->N);
    s->u = (double*)calloc(3 * (size_t)s->N, sizeof(double));
    s->sig = (double*)calloc(6 * (size_t)s->N, sizeof(double));
    s->g = (double*)calloc(3 * (size_t)s->N, sizeof(double));
    s->Trel = (double*)malloc(sizeof(double) * (size_t)s->N);
    for (p = 0; p < 19; ++p)
        for (n = 0; n < s->N; ++n) {
            s->f[(long)p * s->N + n] = WV[p];
            s->fnew[(long)p * s->N + n] = WV[p];
        }
    for (n = 0; n < s->N; ++n) {
        s->Trel[n] = prm->tau0;
        for (a = 0; a < 3; ++a) s->g[3 * n + a] = solid[n] ? 0.0 : prm->g_ext[a];
    }
    s->nrbc = n_rbc;
#define ALLOCN(ptr, k) ptr = (double*)calloc((size_t)(k) * (size_t)(n_rbc + 1), sizeof(double))
    ALLOCN(s->R, 3); ALLOCN(s->Q, 9); ALLOCN(s->V, 3); ALLOCN(s->Om, 3);
    ALLOCN(s->Fcomb, 3); ALLOCN(s->Tcomb, 3); ALLOCN(s->Vh, 3); ALLOCN(s->Omh, 3);
    ALLOCN(s->S, 1); ALLOCN(s->ut, 3); ALLOCN(s->wt, 3); ALLOCN(s->TS, 3);
    ALLOCN(s->Fhyd, 3); ALLOCN(s->Thyd, 3); ALLOCN(s->Fmech, 3); ALLOCN(s->Tmech, 3);
#undef ALLOCN
    if (n_rbc > 0) {
        memcpy(s->R, R, sizeof(double) * 3 * (size_t)n_rbc);
        memcpy(s->Q, Q, sizeof(double) * 9 * (size_t)n_rbc);
        if (V) memcpy(s->V, V, sizeof(double) * 3 * (size_t)n_rbc);
        if (Om) memcpy(s->Om, Om, sizeof(double) * 3 * (size_t)n_rbc);
    }
    setup_cell_grid(s);
    nc = s->ncell[0] * s->ncell[1] * s->ncell[2];
    for (a = 0; a < 3; ++a)
        if (s->P.periodic[a] && n_rbc > 0 &&
            box_len(s, a) < 2.0 * (double)(support_halfwidth(s) + 1) + 1.0) {
            orc_destroy(s);
            return NULL;
        }
    s->cell_off = (int*)calloc((size_t)nc + 1, sizeof(int));
    s->cell_ids = (int*)malloc(sizeof(int) * (size_t)(n_rbc + 1));
    build_walls(s);
    build_wall_nodes(s);
    s->map_off = (long*)calloc((size_t)s->N + 1, sizeof(long));
    s->map_alloc = 1024;
    s->map_ids = (int*)malloc(sizeof(int) * (size_t)s->map_alloc);
    /* start-up pass: F^comb(0) = F^mech(0), tau^comb(0) = tau^mech(0) (fluid at rest) */
    if (n_rbc > 0) {
        int st;
        for (i = 0; i < n_rbc; ++i)
            for (a = 0; a < 3; ++a)
                if (s->P.periodic[a]) {
                    double L = box_len(s, a);
                    if (s->R[3 * i + a] >= L) s->R[3 * i + a] -= L;
                    else if (s->R[3 * i + a] < 0.0) s->R[3 * i + a] += L;
                }
        build_cell_list(s);
        st = collide_all(s, 0);
        if (st) {
            orc_destroy(s);
            *status = st;
            return NULL;
        }
        for (int i = 0; i < n_rbc; ++i)
            for (int a = 0; a < 3; ++a) {
                s->Fcomb[3 * i + a] = s->Fmech[3 * i + a] + s->P.ext_force[a];
                s->Tcomb[3 * i + a] = s->Tmech[3 * i + a] + s->P.ext_torque[a];
            }
    }
    *status = ORC_OK;
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->solid); free(s->f); free(s->fnew); free(s->u); free(s->sig); free(s->g);
    free(s->Trel);
    free(s->R); free(s->Q); free(s->V); free(s->Om); free(s->Fcomb); free(s->Tcomb);
    free(s->Vh); free(s->Omh); free(s->S); free(s->ut); free(s->wt); free(s->TS);
    free(s->Fhyd); free(s->Thyd); free(s->Fmech); free(s->Tmech);
    free(s->cell_off); free(s->cell_ids); free(s->wall_xyz); free(s->wcell_off);
    free(s->wcell_ids); free(s->map_off); free(s->map_ids); free(s->wn_node);
    free(s->wn_nrm);
    free(s);
}

int orc_set_fields(orc_sim* s, const double* f, const double* u, const double* sig)
{
    if (f) memcpy(s->f, f, sizeof(double) * 19 * (size_t)s->N);
    if (u) memcpy(s->u, u, sizeof(double) * 3 * (size_t)s->N);
    if (sig) memcpy(s->sig, sig, sizeof(double) * 6 * (size_t)s->N);
    return ORC_OK;
}

long orc_num_nodes(const orc_sim* s) { return s->N; }
long orc_num_fluid(const orc_sim* s)
{
    long n, c = 0;
    for (n = 0; n < s->N; ++n) c += !s->solid[n];
    return c;
}
void orc_get_f(const orc_sim* s, double* f) { memcpy(f, s->f, sizeof(double) * 19 * (size_t)s->N); }
void orc_get_u(const orc_sim* s, double* u) { memcpy(u, s->u, sizeof(double) * 3 * (size_t)s->N); }
void orc_get_sigma(const orc_sim* s, double* g) { memcpy(g, s->sig, sizeof(double) * 6 * (size_t)s->N); }
void orc_get_force(const orc_sim* s, double* g) { memcpy(g, s->g, sizeof(double) * 3 * (size_t)s->N); }
void orc_get_relax(const orc_sim* s, double* T) { memcpy(T, s->Trel, sizeof(double) * (size_t)s->N); }
void orc_get_rbc(const orc_sim* s, double* R, double* Q, double* V, double* Om)
{
    size_t n = (size_t)s->nrbc;
    if (R) memcpy(R, s->R, sizeof(double) * 3 * n);
    if (Q) memcpy(Q, s->Q, sizeof(double) * 9 * n);
    if (V) memcpy(V, s->V, sizeof(double) * 3 * n);
    if (Om) memcpy(Om, s->Om, sizeof(double) * 3 * n);
}
void orc_get_coupling(const orc_sim* s, double* o)
{
    int i, a;
    for (i = 0; i < s->nrbc; ++i) {
        double* r = o + 22 * i;
        r[0] = s->S[i];
        for (a = 0; a < 3; ++a) {
            r[1 + a] = s->ut[3 * i + a];
            r[4 + a] = s->wt[3 * i + a];
            r[7 + a] = s->TS[3 * i + a];
            r[10 + a] = s->Fhyd[3 * i + a];
            r[13 + a] = s->Thyd[3 * i + a];
            r[16 + a] = s->Fcomb[3 * i + a];
            r[19 + a] = s->Tcomb[3 * i + a];
        }
    }
}
void orc_cell_grid(const orc_sim* s, int ncell[3], double edge[3])
{
    int a;
    for (a = 0; a < 3; ++a) { ncell[a] = s->ncell[a]; edge[a] = s->cedge[a]; }
}
void orc_get_cells(const orc_sim* s, int* off, int* ids)
{
    int nc = s->ncell[0] * s->ncell[1] * s->ncell[2];
    memcpy(off, s->cell_off, sizeof(int) * ((size_t)nc + 1));
    memcpy(ids, s->cell_ids, sizeof(int) * (size_t)s->nrbc);
}
long orc_get_map(const orc_sim* s, int* off, int* ids)
{
    long n;
    if (off)
        for (n = 0; n <= s->N; ++n) off[n] = (int)s->map_off[n];
    if (ids) memcpy(ids, s->map_ids, sizeof(int) * (size_t)s->map_len);
    return s->map_len;
}
int orc_num_wall_particles(const orc_sim* s) { return s->nwall; }

static double node_wss(const orc_sim* s, int k)
{
    const double* sg = s->sig + 6 * s->wn_node[k];
    const double* nw = s->wn_nrm + 3 * k;
    double t[3], tn, r[3];
    t[0] = sg[0] * nw[0] + sg[3] * nw[1] + sg[4] * nw[2];
    t[1] = sg[3] * nw[0] + sg[1] * nw[1] + sg[5] * nw[2];
    t[2] = sg[4] * nw[0] + sg[5] * nw[1] + sg[2] * nw[2];
    tn = t[0] * nw[0] + t[1] * nw[1] + t[2] * nw[2];
    r[0] = t[0] - tn * nw[0]; r[1] = t[1] - tn * nw[1]; r[2] = t[2] - tn * nw[2];
    return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

int orc_wall_shear_stress(const orc_sim* s, long* node, double* wss)
{
    int k;
    for (k = 0; k < s->nwn; ++k) {
        if (node) node[k] = s->wn_node[k];
        if (wss) wss[k] = node_wss(s, k);
    }
    return s->nwn;
}

/* Observables. Flow rate: mean over z-slices of the summed u_z. Apparent viscosity of a
 * straight tube along z from Poiseuille's law, eta = pi R^4 g_z / (8 Q), with R the radius
 * of the disc that has the mean fluid cross-section (the paper's "eta proportional to Q"
 * inverts Poiseuille's law at fixed drive; relative viscosity is Q_0 / Q_H). */
/* Neumaier compensated summation, so that sums over millions of nodes keep FP64 accuracy. */
typedef struct { double s, c; } ksum;
static void kadd(ksum* k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

void orc_observe(const orc_sim* s, double* out)
{
    long n;
    int p, k;
    ksum mass = {0, 0}, mom[3] = {{0, 0}, {0, 0}, {0, 0}}, uz = {0, 0}, wsum = {0, 0};
    double area, Rt, wmax = 0;
    long nf = 0;
    for (n = 0; n < s->N; ++n) {
        double m = 0, mx = 0, my = 0, mz = 0;
        if (s->solid[n]) continue;
        nf++;
        for (p = 0; p < 19; ++p) {
            double fp = s->f[(long)p * s->N + n];
            m += fp;
            mx += fp * CV[p][0]; my += fp * CV[p][1]; mz += fp * CV[p][2];
        }
        kadd(&mass, m);
        kadd(&mom[0], mx); kadd(&mom[1], my); kadd(&mom[2], mz);
        kadd(&uz, s->u[3 * n + 2]);
    }
    out[0] = kval(&mass);
    out[1] = kval(&mom[0]); out[2] = kval(&mom[1]); out[3] = kval(&mom[2]);
    out[4] = kval(&uz) / s->nz;
    area = (double)nf / s->nz;
    Rt = sqrt(area / M_PI);
    out[5] = out[4] != 0.0 ? M_PI * pow(Rt, 4.0) * s->P.g_ext[2] / (8.0 * out[4]) : 0.0;
    for (k = 0; k < s->nwn; ++k) {
        double w = node_wss(s, k);
        kadd(&wsum, w);
        if (w > wmax) wmax = w;
    }
    out[6] = s->nwn ? kval(&wsum) / s->nwn : 0.0;
    out[7] = wmax;
    out[8] = s->nwn;
}

void orc_wall_momentum(const orc_sim* s, double out3[3])
{
    out3[0] = s->wall_mom[0]; out3[1] = s->wall_mom[1]; out3[2] = s->wall_mom[2];
}
