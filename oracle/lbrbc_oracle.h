/*
 * lbrbc_oracle.h -- plain FP64 CPU oracle for the coupled plasma / rigid red-blood-cell
 * time step of S. Melchionna, "A model for red blood cells in simulations of large-scale
 * blood flows" (2011).
 *
 * TEST INFRASTRUCTURE ONLY. This oracle exists to check the HIP library. Only the test
 * suite, the package's smoke check and the CPU-baseline leg of the benchmark load it. It
 * shares no code, header, table or helper with the HIP library; both sides receive the
 * same seeded inputs (geometry mask and cell state) and nothing else.
 *
 * Units: lattice units throughout (time step h = 1, mesh spacing 1, c^2 = 1/3).
 * Layouts: node index n = x + nx*(y + ny*z); populations f[p*N + n]; vectors per node
 * [n*3 + a]; stress per node [n*6 + k] with k = xx, yy, zz, xy, xz, yz; orientation Q is
 * row-major 3x3 whose columns are the body axes n, t, g in the lab frame (Sec. II B).
 */
#ifndef LBRBC_ORACLE_H
#define LBRBC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_EUNSTABLE = 4, ORC_EOVERLAP = 5 };

typedef struct orc_params {
    int nx, ny, nz;
    int periodic[3];      /* 1: periodic axis; 0: the box face is a wall (outside = solid) */
    int forcing;          /* 0: second-order (Guo) body-force term; 1: the term as printed */
    double tau0;          /* plasma relaxation time T0 (> 1/2) */
    double delta_visc;    /* viscosity enhancement factor Delta */
    double kappa;         /* smoothness exponent kappa of the cell indicator */
    double g_ext[3];      /* uniform external body-force density on fluid nodes */
    double gammaT, gammaR;/* translational / rotational coupling rates */
    double alpha;         /* elongational (tank-treading) torque factor */
    double mass;          /* cell mass M */
    double inertia[3];    /* body-frame principal moments of inertia */
    double vort_scale;    /* factor applied to the smeared vorticity (1 = full curl) */
    double xi[3];         /* shape-function radii (body frame) */
    double axes[3];       /* Gay-Berne semi-axes (body frame) */
    double eps0;          /* Gay-Berne energy scale */
    double a_wall;        /* radius of the spherical wall particles */
    double sigmin_wall;   /* sigma_min of a cell-wall pair */
    int wall_particles;   /* 1: wall mesh points repel the cells */
    int open_z;           /* 1: z faces are pressure boundaries (inlet z=0, outlet z=nz-1) */
    double rho_in, rho_out;
    double ext_force[3];  /* external force on every cell, lab frame (drag experiments) */
    double ext_torque[3]; /* external torque on every cell, body frame */
    double wall_u_lo[3];  /* velocity of the solid nodes with y < ny/2 (moving walls) */
    double wall_u_hi[3];  /* velocity of the solid nodes with y >= ny/2 */
} orc_params;

typedef struct orc_sim orc_sim;

/* Create a simulation at rest (f = w, u = sigma = 0). solid: nx*ny*nz bytes, 1 = solid.
 * Cell arrays (may be NULL when n_rbc == 0): R[3n], Q[9n], V[3n], Om[3n] (Om body frame).
 * Returns NULL and sets *status on failure. */
orc_sim* orc_create(const orc_params* prm, const uint8_t* solid, int n_rbc,
                    const double* R, const double* Q, const double* V, const double* Om,
                    int* status);
void orc_destroy(orc_sim* s);

/* Advance nsteps full coupled steps. Returns ORC_OK or an error (state then undefined). */
int orc_step(orc_sim* s, int nsteps);

/* Coupling only, at the current state: cell list, node->cell map, interpolation sums,
 * hydrodynamic force/torque from the current V, Omega, and the spread force field and
 * local relaxation time. No time advance. */
int orc_couple(orc_sim* s);
/* Cell list + Gay-Berne forces at the current positions. F: lab force [3n];
 * T: body-frame torque [3n]. brute != 0 uses all pairs and all wall points. */
int orc_collide(orc_sim* s, int brute, double* F, double* T);

/* Overwrite the fluid state. f: f*[19*N] (may be NULL), u: [3N], sig: [6N] (may be NULL). */
int orc_set_fields(orc_sim* s, const double* f, const double* u, const double* sig);

/* Getters (caller-allocated). */
long orc_num_nodes(const orc_sim* s);
long orc_num_fluid(const orc_sim* s);
void orc_get_f(const orc_sim* s, double* f);
void orc_get_u(const orc_sim* s, double* u);
void orc_get_sigma(const orc_sim* s, double* sig);
void orc_get_force(const orc_sim* s, double* g);    /* last spread force density [3N] */
void orc_get_relax(const orc_sim* s, double* T);    /* last local relaxation time [N] */
void orc_get_rbc(const orc_sim* s, double* R, double* Q, double* V, double* Om);
/* Per cell: S (raw shape sum), u~[3], w~[3], T^S[3] (lab), F^hyd[3] (lab), T^hyd[3] (lab),
 * F^comb[3] (lab), tau^comb[3] (body): 22 doubles per cell. */
void orc_get_coupling(const orc_sim* s, double* out22);
void orc_cell_grid(const orc_sim* s, int ncell[3], double edge[3]);
/* Cell-list CSR: off[ncells+1], ids[n_rbc] ascending within a cell. */
void orc_get_cells(const orc_sim* s, int* off, int* ids);
/* Node->cell map CSR over all nodes: off[N+1]; returns entry count (ids sized by caller
 * after a first call with ids == NULL). Ids ascending per node. */
long orc_get_map(const orc_sim* s, int* off, int* ids);
int  orc_num_wall_particles(const orc_sim* s);
/* Observables: out[0] mass, [1..3] momentum (post-collision), [4] flow rate along z,
 * [5] apparent viscosity, [6] mean WSS, [7] max WSS, [8] number of wall-adjacent nodes. */
void orc_observe(const orc_sim* s, double* out9);
/* Wall shear stress at the wall-adjacent fluid nodes (ascending node index): node[],
 * wss[]. Returns the count (arrays may be NULL to query it). */
int orc_wall_shear_stress(const orc_sim* s, long* node, double* wss);
/* Momentum exchanged with the walls by bounce-back during the last step (lab). */
void orc_wall_momentum(const orc_sim* s, double out3[3]);

/* Threads the oracle's parallel loops use (OpenMP; 1 without it). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Primitives exposed for closed-form tests. */
void   orc_lattice(int c[19][3], double w[19]);
double orc_peskin(double r);
double orc_feq(double rho, const double u[3], int p);
double orc_force_term(int forcing, double T, const double g[3], const double u[3], int p);
/* Gay-Berne pair: lab-frame force on i and lab-frame torques on i and j.
 * wall != 0: j is a sphere of radius a_wall with sigma_min = sigmin_wall.
 * Returns 0 (interacting or beyond cut-off: all zero), ORC_EOVERLAP if rho <= 0. */
int orc_gb_pair(const orc_params* prm, const double Ri[3], const double Qi[9],
                const double Rj[3], const double Qj[9], int wall,
                double* U, double F[3], double taui[3], double tauj[3]);
/* One rigid-body step with given combined force (lab) and torque (body), both halves,
 * no fluid: used for integrator closed forms. Forces are held fixed over the step. */
void orc_rigid_step(const orc_params* prm, double R[3], double Q[9], double V[3],
                    double Om[3], const double F[3], const double T[3]);

#ifdef __cplusplus
}
#endif
#endif
