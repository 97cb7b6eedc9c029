/*
 * lbrbc.h -- C ABI of the MI355X (gfx950) library for the coupled plasma / rigid red-blood-
 * cell time step of S. Melchionna, "A model for red blood cells in simulations of
 * large-scale blood flows" (2011).
 *
 * One time step advances, on the GPU and on the caller's HIP stream:
 *   rigid-body first half (App. A, steps 1-4) -> cell list -> node->cell coverage map ->
 *   interpolation of velocity, vorticity and stress onto each cell (Sec. II B, Eqs. 16-21)
 *   -> Gay-Berne cell-cell and cell-wall forces (Sec. II E, Eqs. 24-28; App. B) ->
 *   rigid-body second half (App. A, steps 5-7) -> fused spreading of the back-reaction G
 *   with the local relaxation time (Sec. II B; Sec. II D, Eq. 23) and D3Q19 pull
 *   stream-collide with body force and halfway bounce-back (Sec. II A, Eqs. 1-8).
 *
 * Conventions (all lattice units, h = 1, mesh spacing 1, c^2 = 1/3):
 *   - node (x, y, z) has flat index n = x + nx*(y + ny*z) and sits at the point (x, y, z);
 *   - host arrays: solid[n] (uint8, 1 = solid); per node vectors [n*3 + a]; stress per node
 *     [n*6 + k], k = xx, yy, zz, xy, xz, yz; populations [p*N + n] (unshifted f). Host
 *     arrays are in this lattice order whatever storage layout the device uses
 *     (lb_config.layout);
 *   - D3Q19 order: 0 rest; 1-6 = +x, -x, +y, -y, +z, -z; 7-18 = (+1,+1,0), (-1,-1,0),
 *     (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1), (-1,0,+1), (0,+1,+1),
 *     (0,-1,-1), (0,+1,-1), (0,-1,+1);
 *   - a cell's orientation Q is row-major 3x3 whose columns are the body axes n, t, g in
 *     the lab frame (Sec. II B, Eq. 9); V is lab frame, Omega is body frame.
 *
 * Ownership: every host pointer is read or written only during the call. Device memory
 * comes from the caller as one arena (e.g. a torch uint8 tensor) of at least
 * lb_query_footprint() bytes; the library never allocates or frees device memory, and the
 * arena and the stream must outlive the context. lb_destroy frees host state only.
 *
 * Errors: every call returns lb_status; nothing throws across the ABI. Invalid arguments
 * give LB_EINVAL synchronously. Faults found on the device (non-finite or non-positive
 * density, |u| > 0.3, a Gay-Berne pair at rho_ij <= 0, a full coverage slot) set a flag
 * word in the arena; the next synchronising call (lb_sync, lb_observe, any getter)
 * returns it, after which the context answers LB_ESTATE to lb_step until lb_load or
 * lb_set_fields. lb_last_error() gives a message for the last failure.
 */
#ifndef LBRBC_H
#define LBRBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx_s* lb_ctx;
typedef struct lb_graph_s* lb_graph;

typedef enum {
    LB_OK = 0,
    LB_EINVAL = 1,
    LB_ENOMEM = 2,      /* arena too small */
    LB_EHIP = 3,        /* a HIP runtime call failed */
    LB_EUNSTABLE = 4,   /* non-finite or non-positive density, or |u| > 0.3 */
    LB_EOVERLAP = 5,    /* Gay-Berne pair or cell-wall pair at rho <= 0 (singular) */
    LB_ECAPACITY = 6,   /* more covering cells at a node than map_cap, or support too big */
    LB_ESTATE = 7       /* context poisoned by an earlier device fault */
} lb_status;

typedef enum { LB_F64 = 0, LB_F32 = 1, LB_BF16 = 2, LB_F16 = 3 } lb_storage;

typedef struct lb_config {
    int nx, ny, nz;
    int periodic[3];      /* 1: periodic axis; 0: box faces are walls (outside = solid) */
    int storage;          /* lb_storage of the shifted populations f - w; F64 computes in
                             double, the others in float */
    double f16_scale;     /* LB_F16: stored value = scale * (f - w); a power of two in
                             [2^10, 2^40], else LB_EINVAL. Below about 2^10 the populations of a
                             slow flow (|f - w| ~ 1e-5) fall into FP16's subnormal range and
                             their per-step increments round to zero without any error; above
                             2^17 a fast flow (|f - w| ~ 0.3) overflows, which the step reports
                             as LB_EUNSTABLE */
    int forcing;          /* 0: second-order (Guo) body-force term; 1: Eq. 4 as printed */
    double tau0;          /* plasma relaxation time T0 > 1/2 (nu = (T0 - 1/2)/3) */
    double delta_visc;    /* viscosity enhancement Delta (Eq. 23) */
    double kappa;         /* smoothness exponent kappa (Eq. 23) */
    double g_ext[3];      /* uniform body-force density on fluid nodes */
    double gammaT, gammaR;/* coupling rates (Eqs. 14-15), per unit mass / inertia */
    double alpha;         /* elongational torque factor (Eq. 16) */
    double mass;          /* cell mass M */
    double inertia[3];    /* body-frame principal moments */
    double vort_scale;    /* factor on the smeared vorticity (1: full curl as printed) */
    double xi[3];         /* shape-function radii (support |y_a| < xi_a in body frame) */
    double axes[3];       /* Gay-Berne semi-axes (body frame) */
    double eps0;          /* Gay-Berne energy scale */
    double a_wall;        /* wall particle radius */
    double sigmin_wall;   /* sigma_min of a cell-wall pair */
    int wall_particles;   /* 1: wall mesh points repel the cells (Sec. II E, last par.) */
    int open_z;           /* 1: z faces are pressure boundaries (inlet z = 0, outlet top) */
    double rho_in, rho_out;
    int map_cap;          /* coverage slots per node, 1..12 (0 = 12) */
    int bf16_nearest;     /* BF16 storage rounding: 0 = stochastic (unbiased; the random bits are
                             a hash of node, direction and value, so results stay deterministic);
                             1 = round to nearest even, which loses the increments of slow flows */
    double ext_force[3];  /* constant external force on every cell, lab frame, added to the
                             combined force (drag experiments of Sec. III; 0 = none) */
    double ext_torque[3]; /* constant external torque on every cell, body frame, added to the
                             combined torque (spin experiments of Sec. III; 0 = none) */
    double wall_u_lo[3];  /* moving walls: velocity of the solid nodes with y < ny/2 (lab) */
    double wall_u_hi[3];  /* velocity of the solid nodes with y >= ny/2. Nonzero velocities make
                             the halfway bounce-back hand the fluid the wall's momentum (Ladd's
                             rule, wall density 1): the wall-bounded shear cell of the
                             tank-treading experiments (Sec. III). Not with open_z (LB_EINVAL) */
    int cand_cap;         /* test hook: candidate nodes per cell that the one-wavefront map pass
                             holds (0 = a sampled bound, above every orientation met in
                             practice). Smaller values, raised to at least tile_max^2, send
                             more cells to the full-tile pass; the results do not change */
    int layout;           /* storage of the per-node planes: 0 = automatic, 1 = dense (every node,
                             index x + nx (y + ny z)), 2 = compact (only the 64-node row segments
                             that hold a fluid node, with a neighbour table per segment). The
                             automatic choice is compact when under 60% of the row segments hold
                             fluid. Field accessors work in lattice order either way;
                             checkpoints hold the storage order, so one loads only into a
                             context of the same layout */
} lb_config;

typedef struct lb_rbc {
    double R[3];          /* centre, lab frame */
    double Q[9];          /* orientation, row-major, columns = body axes */
    double V[3];          /* velocity, lab frame */
    double Omega[3];      /* angular velocity, body frame */
} lb_rbc;

typedef struct lb_observables {
    double mass;          /* sum of populations over fluid nodes */
    double momentum[3];   /* sum of f c over fluid nodes (post-collision) */
    double flow_rate;     /* mean over z-slices of the summed u_z */
    double eta_app;       /* pi R^4 g_z / (8 Q), R from the mean fluid cross-section */
    double wss_mean;      /* wall shear stress over wall-adjacent fluid nodes */
    double wss_max;
    double wss_time_mean; /* time average of wss_mean since lb_wss_accumulate(ctx, 1) */
    long long step;
    unsigned flags;       /* device fault bits: 1 unstable, 2 overlap, 4 capacity */
    long long n_fluid;
    int n_wall_nodes;
    int n_rbc;
    int compact;          /* storage layout in use: 1 compact, 0 dense */
    long long n_stored;   /* storage slots per plane (nodes, or 64 per stored row segment) */
} lb_observables;

/* Bytes of device arena needed for this configuration (solid: host, nx*ny*nz bytes). */
lb_status lb_query_footprint(const lb_config* cfg, const uint8_t* solid, int n_rbc,
                             size_t* arena_bytes);

/* Build a context: fluid at rest (f = w, u = sigma = 0), cells from `cells` (host, copied),
 * F^comb(0) and tau^comb(0) from the Gay-Berne forces at t = 0 (the fluid is at rest).
 * arena: device pointer, >= footprint bytes, 256-byte aligned. hip_stream: hipStream_t
 * (NULL = default stream). Synchronises the stream before returning. */
lb_status lb_init(const lb_config* cfg, const uint8_t* solid, const lb_rbc* cells, int n_rbc,
                  void* arena, size_t arena_bytes, void* hip_stream, lb_ctx* out);

/* Enqueue nsteps full coupled steps on the stream (asynchronous). */
lb_status lb_step(lb_ctx ctx, int nsteps);

/* Coupling only, at the current state, no time advance (asynchronous): cell list,
 * coverage map (the support of Sec. II B, Eqs. 10-12, plus the one-node halo of its
 * central-difference gradient), interpolation sums S, u~, w~, T^S (Sec. II B, Eqs. 16-21;
 * Sec. II C, Eq. 16 for T^S), hydrodynamic force/torque from the current V and Omega
 * (Eqs. 14-15), and the spread force density G (Sec. II B, back-reaction) and local
 * relaxation time (Sec. II D, Eq. 23) per node, readable with lb_get_fields. */
lb_status rbc_couple(lb_ctx ctx);

/* Cell list and Gay-Berne cell-cell and cell-wall forces and torques at the current
 * positions (Sec. II E, Eqs. 24-28; App. B, with the torques of App. B corrected as stated
 * in the library's notes: tau_i = (1/R) R_ci x f_k, tau_j = -(1/R) R_cj x f_k); synchronous.
 * F: host [3*n_rbc] lab force; T: host [3*n_rbc] body-frame torque. Either may be NULL.
 * A pair at rho_ij <= 0 returns LB_EOVERLAP. */
lb_status rbc_collide(lb_ctx ctx, double* F, double* T);

/* rbc_collide without any device memory of its own, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels write the Gay-Berne force (lab, F[3*i + a]) and torque (body, T[3*i + a]) of every
 * cell into the caller's DEVICE arrays, asynchronously on the context's stream. The cell list
 * it needs is built in a static device array of the library (about 10 MiB per GPU, held until
 * the process ends), not in the arena. At most 262,144 cells and 1,048,576 grid cells, else
 * LB_EINVAL. Calls that overlap on one GPU (other streams or threads) share that array and
 * race; an overlapping pair (rho_ij <= 0) is reported by the next synchronising call. */
lb_status rbc_collide_static(lb_ctx ctx, double* F, double* T);

/* Synchronous reads of the observables of Sec. III: mass and momentum (sums of f and f c
 * over fluid nodes, Eqs. 5-6), the flow rate Q (mean over z-slices of the summed u_z), the
 * apparent viscosity pi R^4 g / (8 Q) of a body-force-driven tube (Poiseuille's law, which
 * the paper's viscosity comparisons assume) and the wall shear stress of
 * lb_wall_shear_stress. FP64 reductions in a fixed order. */
lb_status lb_observe(lb_ctx ctx, lb_observables* out);
/* Wall shear stress at each wall-adjacent fluid node (the quantity Sec. III reports for the
 * bifurcation), from the deviatoric stress of Eq. 8: with the wall normal n_w =
 * normalize(sum over solid neighbours x + c_p of w_p c_p) and the traction t = sigma n_w,
 * WSS = |t - (t . n_w) n_w|, in FP64. Ascending node index. wss: host [*n] or NULL to query
 * the count; node: host [*n] or NULL. With time != 0, the time average since
 * lb_wss_accumulate(ctx, 1). */
lb_status lb_wall_shear_stress(lb_ctx ctx, int time, double* wss, long long* node, int* n);
/* The apparent viscosity of lb_observe alone (Sec. III, the viscosity of a tube flow). */
lb_status lb_apparent_viscosity(lb_ctx ctx, double* eta_app);
/* Start (on != 0, resetting the sums) or stop per-step FP64 accumulation of the WSS. */
lb_status lb_wss_accumulate(lb_ctx ctx, int on);

/* Host copies of the fields; any pointer may be NULL. f: [19*N] unshifted populations
 * (post-collision of the last step); u: [3N]; sigma: [6N]; g: [3N] spread force density
 * and relax: [N] local relaxation time from the last rbc_couple. The device keeps u and
 * sigma in the compute precision, or in 16 bits for the 16-bit storages (BF16 rounded to
 * nearest even; FP16 holding 4096 times the value): the values returned, and those
 * lb_set_fields stores, carry that rounding. */
lb_status lb_get_fields(lb_ctx ctx, double* f, double* u, double* sigma, double* g,
                        double* relax);
/* Overwrite the fluid state from host arrays (any may be NULL); clears a device fault. */
lb_status lb_set_fields(lb_ctx ctx, const double* f, const double* u, const double* sigma);

lb_status rbc_get_state(lb_ctx ctx, lb_rbc* out, int n);
lb_status rbc_set_state(lb_ctx ctx, const lb_rbc* in, int n);
/* Per cell, 22 doubles: S, u~[3], w~[3], T^S[3] (lab), F^hyd[3] (lab), T^hyd[3] (lab),
 * F^comb[3] (lab), tau^comb[3] (body). */
lb_status rbc_get_coupling(lb_ctx ctx, double* out22, int n);
/* Cell grid and list: ncell[3]; off[ncells + 1]; ids[n_rbc] ascending per cell. */
lb_status rbc_get_cells(lb_ctx ctx, int* ncell, int* off, int* ids);
/* Coverage map (the cells covering each node) as CSR over all nodes, ids ascending per
 * node: off[N + 1] (may be NULL), ids[*len] (NULL to query *len). It is the map of the last
 * rbc_couple call: call rbc_couple first to read the map of the current state (a time step
 * consumes the per-node counts of its own map). */
lb_status rbc_get_map(lb_ctx ctx, int* off, int* ids, long long* len);

/* Checkpoint of the full dynamic state (populations in storage precision, fields, cells,
 * combined forces, step count). buf == NULL: *bytes = size needed. */
lb_status lb_save(lb_ctx ctx, void* buf, size_t* bytes);
lb_status lb_load(lb_ctx ctx, const void* buf, size_t bytes);

/* Serving (not in the paper, whose method is one simulation at a time): enqueue nsteps[i]
 * steps of the same coupled time step (the steps of lb_step) for each of n contexts
 * (asynchronous).
 * - When all contexts share one stream and one storage type, and none has open boundaries,
 *   WSS accumulation or kernel timing on, each stage of a step is ONE launch over all the
 *   contexts still stepping (fused multi-lattice kernels, up to 64 contexts per launch);
 *   the results are bitwise those of stepping each context alone. The Gay-Berne stage and the
 *   kick run on a second stream of the library's (one per device, default priority, created
 *   at the first batch call), forked from and joined back into the contexts' stream by events;
 *   the call returns with the contexts' stream holding all its work.
 * - Otherwise the contexts' steps are interleaved step by step on their own streams, so
 *   their kernels can overlap on the device.
 * nsteps[i] < 0 or a NULL context: LB_EINVAL; a poisoned context: LB_ESTATE (nothing is
 * enqueued in either case). */
lb_status lb_batch_step(lb_ctx* ctxs, const int* nsteps, int n);

/* Serving with captured HIP graphs (scheduling only, no paper passage): record nsteps (even,
 * >= 2) fused steps of the n contexts, the same launches lb_batch_step issues for a fused
 * batch, into a HIP graph on their common stream; nothing runs and no context changes. The
 * contexts must share one stream and one storage, without open boundaries, WSS accumulation
 * or timing (else LB_EINVAL), and stay alive and on that stream while the graph exists.
 * Every replay first clears the contexts' coverage counts, so it is valid whatever ran before.
 * lb_graph_launch enqueues one replay (asynchronous; LB_ESTATE if a context is poisoned) and
 * advances the contexts' step counters; lb_graph_destroy waits for the graph's last replay to
 * finish (that replay only, not the rest of the stream) and frees it. */
lb_status lb_batch_capture(lb_ctx* ctxs, int n, int nsteps, lb_graph* out);
lb_status lb_graph_launch(lb_graph graph);
void lb_graph_destroy(lb_graph graph);

/* Move the context's later work to another HIP stream (not NULL). The caller orders it after
 * the work already enqueued (e.g. an event recorded on the old stream and waited on by the
 * new one); the library does not. Used to put contexts on one stream for fused batches and
 * to take a finished one off it. NULL context or stream: LB_EINVAL. */
lb_status lb_set_stream(lb_ctx ctx, void* hip_stream);

/* Second stream for the cells' own work (no paper passage: scheduling only). With 2048 or
 * more cells a step runs the Gay-Berne pass, and after the map pass the kick and the next
 * step's first half and cell list, on a second stream beside the stream-collide, ordered by
 * events. By default the library creates that stream at lb_init (default priority); this
 * call hands it a caller-owned one instead (e.g. a torch stream), which must outlive the
 * context, or, with NULL, runs every kernel on the main stream. Results are bitwise the same
 * in every case. Synchronises the context's streams first. */
lb_status lb_set_side_stream(lb_ctx ctx, void* hip_stream);

/* Wait for the context's stream and report device faults (LB_EUNSTABLE, LB_EOVERLAP,
 * LB_ECAPACITY) raised since the last check; after a fault the context is poisoned. */
lb_status lb_sync(lb_ctx ctx);
const char* lb_last_error(lb_ctx ctx);
void lb_destroy(lb_ctx ctx);

/* Measurement (no paper passage): with lb_set_timing(ctx, 1), HIP events on the main stream
 * bracket every stream-collide launch and the whole lb_step calls; lb_kernel_time gives the
 * average stream-collide duration and the average step duration (ms) since timing was
 * switched on, 0 if none. */
lb_status lb_set_timing(lb_ctx ctx, int on);
lb_status lb_kernel_time(lb_ctx ctx, double* sc_ms, double* step_ms);
/* The same events also bracket the map pass of every step (the one-wavefront pass and the
 * full-tile pass behind it): its average duration (ms) since timing was switched on, 0 if none. */
lb_status lb_map_time(lb_ctx ctx, double* map_ms);

#ifdef __cplusplus
}
#endif
#endif
