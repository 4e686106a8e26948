/*
 * fp.h -- C ABI of libfpgpu.so: the cubic Fokker-Planck particle step on one MI355X.
 *
 * The method is the particle cubic-FP model of Gorji et al. as restated in Roohi,
 * "Accelerating Kinetic Fokker-Planck Simulations via a GPU-Native Deep Neural Network
 * Surrogate": every step bins the particles into cells, gathers central velocity
 * moments per cell, solves the 9x9 moment-matching system for the drift coefficients
 * (C, Gamma), updates velocities with the mixed Ornstein-Uhlenbeck/Euler scheme and
 * moves the particles (Algorithm "Baseline Physics Simulation Loop").
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers owned by the caller, on the device that was
 *     current at fp_init.  The library owns only the context and its scratch memory.
 *   - Every call is asynchronous on the given HIP stream and never synchronises the
 *     host, except fp_init, fp_destroy and fp_error_count.
 *   - Return value 0 (FP_OK) or a negative error code.  FP_EDEVICE keeps the HIP error
 *     text for fp_last_error.  Numerical trouble inside a cell is NOT a call error: it
 *     is reported through the per-cell status array (FP_CELL_*).
 *   - Use one context per stream; calls on one context must not overlap.
 *
 * Memory layouts (all row-major, one row per cell):
 *   mom[ncell][32] doubles: [N, U1 U2 U3, theta, P11 P12 P13 P22 P23 P33,
 *       T111 T112 T113 T122 T123 T133 T222 T223 T233 T333,
 *       R11 R12 R13 R22 R23 R33, W1 W2 W3, H, 0]
 *     with c = v - U, P_ij = <c_i c_j>, T_ijk = <c_i c_j c_k>, R_ij = <c_i c_j |c|^2>,
 *     W_i = <c_i |c|^4>, H = <|c|^6>, theta = tr(P)/3, averages with 1/N.
 *   rec[ncell][16] doubles: [Ct11 Ct12 Ct13 Ct22 Ct23 Ct33, G1 G2 G3, tau, theta, E,
 *       eps2, sigma, status, 0] where the drift is A = -c/tau + N with
 *       N = Ct c + G (|c|^2 - 3 theta) - eps2 (c |c|^2 - S), S_i = T_ikk
 *       (eqs. cubic_drift and update_N; the paper's c^(1) equals Ct - I/tau),
 *       E = exp(-dt/tau), sigma = sqrt(theta (1 - exp(-2 dt/tau))).
 *   samp[ncell][16] doubles: [sum N, sum v_i (3), sum v_i v_j (11 12 13 22 23 33),
 *       sum v_i |v|^2 (3), number of samples, 0].
 */
#ifndef FP_H
#define FP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define FP_OK 0
#define FP_EINVAL (-1)     /* bad argument: null pointer, size, configuration */
#define FP_ENOMEM (-2)     /* device allocation failed */
#define FP_EDEVICE (-3)    /* a HIP call failed; text in fp_last_error */
#define FP_ECAPACITY (-4)  /* more particles than the context's capacity */

enum fp_geometry { FP_COUETTE1D = 0, FP_CAVITY2D = 1, FP_CYLINDER2D = 2 };
enum fp_precision { FP_F32 = 0, FP_F64 = 1 };
enum fp_conserve { FP_EXACT = 0, FP_PAPER = 1 };

/* per-cell status written by the closure calls */
enum fp_cell_status {
    FP_CELL_OK = 0,          /* exact 9x9 solve */
    FP_CELL_EMPTY = 1,       /* N <= 1 or theta = 0: the update leaves the cell alone */
    FP_CELL_FEW = 2,         /* N < n_min: Langevin drift (Ct = G = 0, no cubic term) */
    FP_CELL_SINGULAR = 3,    /* |pivot| < pivot_tol or non-finite solution: Langevin */
    FP_CELL_NONFINITE = 4,   /* non-finite moments: the update leaves the cell alone */
    FP_CELL_NN = 5,          /* learned closure accepted */
    FP_CELL_NN_FALLBACK = 6  /* learned closure rejected, exact solve used */
};

/* fp_step flags */
#define FP_STEP_COLLIDE 1u   /* velocity update (eqs. update_vel, update_N) + conservation */
#define FP_STEP_MOVE 2u      /* free flight (eq. update_pos), diffuse walls, new cell key */
#define FP_STEP_KEYS 4u      /* only recompute cell keys from the stored positions */
#define FP_STEP_ADVANCE 8u   /* fp_step_dev only: add 1 to *step_dev once the step is done */

typedef struct fp_config {
    int32_t geometry;        /* fp_geometry */
    int32_t precision;       /* fp_precision: storage and update arithmetic of particles */
    int32_t conserve;        /* fp_conserve */
    int32_t nx, ny;          /* cells along x, y (ny = 1 for the 1-D channel) */
    int32_t n_min;           /* cells with fewer particles use the Langevin drift */
    int32_t max_bounces;     /* wall interactions per particle and step */
    int32_t lanes;           /* lanes per cell of the per-cell kernels: 4, 8, 16, 32 or 64;
                                0 = chosen from the particle and cell counts */
    int32_t moment_order;    /* 5 (or 0): moment records through fifth order (the exact
                                closure needs them); 3: only N, U, theta, P and T are
                                gathered (R, W, H written as 0), for a closure from
                                low-order moments (fp_closure_nn unchecked); fp_closure_solve
                                and the checked fp_closure_nn then refuse the records */
    int32_t reserved0;       /* 0 */
    int64_t capacity;        /* largest particle count any call will see, <= 2^29 - 64 */
    double x0, y0;           /* domain origin [m] */
    double lx, ly;           /* domain extent [m] */
    double dx, dy;           /* cell size [m] */
    double dt;               /* time step [s] */
    double kB, mass;         /* Boltzmann constant [J/K], molecular mass [kg] */
    double mu_ref, T_ref, omega;  /* viscosity law mu = mu_ref (T/T_ref)^omega */
    double fnum_over_vol;    /* real molecules per particle / cell volume [1/m^3] */
    double eps_hat;          /* cubic stabiliser: eps^2 = eps_hat / (theta tau) */
    double pivot_tol;        /* pivot threshold of the normalised 9x9 system */
    double T_wall[4];        /* wall temperatures: x = x0, x = x0+lx, y = y0, y = y0+ly */
    double u_wall[4][3];     /* wall velocities, same order */
    uint64_t seed;           /* Philox4x32-10 key */
    /* open domain around a cylinder (FP_CYLINDER2D): the box boundaries are open (a
     * particle whose flight ends outside is deleted), free stream enters by fp_inject */
    double circle[3];        /* cylinder centre x, y and radius [m] */
    double T_body;           /* cylinder wall temperature [K] (diffuse, isothermal) */
    double n_inf;            /* free-stream number density [1/m^3] */
    double u_inf[3];         /* free-stream velocity [m/s] */
    double T_inf;            /* free-stream temperature [K] */
    double fnum;             /* real molecules per particle (cylinder: density uses the
                                gas volume of each cut cell; fnum_over_vol is ignored) */
    double depth;            /* extent along z [m] */
} fp_config;

/* Particle arrays in structure-of-arrays form.  x, y, vx, vy, vz are float
 * (FP_F32) or double (FP_F64); y may be NULL in 1-D.  pid is a unique particle id
 * (the Philox counter); key is the cell index (row-major, ky*nx + kx).
 *
 * The number of particles is either the host value n, or, when n_dev is set, the value
 * *n_dev on the device at the moment the kernels of a call run (so that a loop whose
 * count changes on the device, as the open domain's deletion and injection make it,
 * needs no host read and can be captured in a HIP graph).  Then capacity is the number
 * of slots the arrays hold (kernels never touch a slot at or beyond it; at most the
 * context's capacity) and n is only a hint of the count for launch shapes.  fp_bin and
 * fp_rebin write the number of particles they keep to dst->n_dev (when set; it must not
 * be src->n_dev), fp_inject_dev appends at *n_dev and advances it. */
typedef struct fp_particles {
    void *x, *y, *vx, *vy, *vz;
    uint32_t* pid;
    int32_t* key;
    int64_t n;               /* number of particles (host), or the hint with n_dev */
    int64_t* n_dev;          /* device count (one int64, caller-owned) or NULL */
    int64_t capacity;        /* slots of the arrays when n_dev is set (ignored otherwise) */
} fp_particles;

typedef struct fp_ctx fp_ctx;

/* Create a context on the current device; allocates scratch for cfg->capacity
 * particles and nx*ny cells.  Synchronous. */
int fp_init(const fp_config* cfg, fp_ctx** out);
/* Free the context and its scratch (synchronises the device). */
void fp_destroy(fp_ctx* ctx);
/* Text of the last FP_EDEVICE/FP_EINVAL error of this context ("" if none). */
const char* fp_last_error(const fp_ctx* ctx);
/* Number of invalid keys met by fp_bin since fp_init (synchronous read-back). */
int64_t fp_error_count(fp_ctx* ctx, hipStream_t s);

/* Stable counting sort by cell key (the sort of "sort_and_calc_moments" in Algorithm
 * "Baseline Physics Simulation Loop"): dst receives the particles of src ordered by
 * key, particles of one cell in their order in src.  offsets[ncell+1] receives the
 * cell start indices; offsets[ncell] is the number of particles kept.  perm (optional,
 * may be NULL) receives for every slot of dst the index in src it came from.  src and
 * dst must not alias.  Particles with key == ncell (deleted) are dropped; keys outside
 * [0, ncell] are counted by fp_error_count and dropped as well. */
int fp_bin(fp_ctx* ctx, const fp_particles* src, fp_particles* dst, int32_t* offsets,
           int32_t* perm, hipStream_t s);

/* The sort of fp_bin (the same result, bit for bit) for particles that were sorted by cell
 * one step earlier: the first src_offsets[ncell] particles of src are grouped by their
 * previous cell, those of cell c at [src_offsets[c], src_offsets[c+1]) (src_offsets is
 * what fp_bin or fp_rebin wrote then; fp_step has since given them new keys), and any
 * particles after them (e.g. injected ones) are in no particular order.  A particle
 * whose new cell is one of the 3 x 3 cells around its previous one is placed from
 * per-cell direction counts, without global atomics; the others take a general path
 * that is slower per particle: a destination ranks its arrivals from outside its 3 x 3
 * neighbourhood by comparing them with one another, a cost that grows with the square of
 * their number, so the call is meant for steps after which almost every particle is still
 * within one cell of its old one (the step length of the method ensures it; use fp_bin
 * after a step that scatters the particles).  src_offsets and offsets must not alias (keep two
 * offsets arrays and alternate them); src_offsets must be non-decreasing with
 * src_offsets[0] >= 0 and src_offsets[ncell] <= src->n.  mom (optional, may be NULL)
 * receives the moment records of the sorted cells, as fp_moments of dst would compute
 * them (up to the order of the sums), gathered in the same pass.  samp (optional, needs
 * mom) then receives the time-average sums of those records exactly as fp_sample would
 * add them.  On a context with an adaptive tree the leaves count as one row of cells (the
 * leaves before and after a leaf in depth-first order are its side neighbours; any other
 * move takes the general path), and the call is refused (FP_EINVAL) until an fp_bin has
 * sorted by the current leaves, i.e. after fp_amr_init and after every fp_amr_adapt. */
int fp_rebin(fp_ctx* ctx, const fp_particles* src, const int32_t* src_offsets,
             fp_particles* dst, int32_t* offsets, int32_t* perm, double* mom, double* samp,
             hipStream_t s);

/* Central moments of every cell of particles sorted by cell (moments u^(p) entering
 * eq. system9x9 and Table matrix_system; layout mom above). */
int fp_moments(fp_ctx* ctx, const fp_particles* p, const int32_t* offsets, double* mom,
               hipStream_t s);
/* fp_moments and fp_sample in one pass (the "average_results" step of Algorithm "Baseline
 * Physics Simulation Loop" on the freshly gathered moments): mom as fp_moments writes it,
 * and its raw sums added to samp0 and, when samp1 is not NULL, to samp1, bit for bit as
 * fp_sample(mom, samp0) and fp_sample(mom, samp1) would add them (layout samp above; a loop
 * that keeps two sets of sums, e.g. the quadtree's adaptation sums beside the output
 * averages, reads the records once).  samp0 is required, samp1 must differ from it;
 * FP_EINVAL otherwise. */
int fp_moments_sample(fp_ctx* ctx, const fp_particles* p, const int32_t* offsets, double* mom,
                      double* samp0, double* samp1, hipStream_t s);

/* Exact closure of every cell: the 9x9 moment-matching system (eq. system9x9, Table
 * matrix_system) in theta-normalised form, solved by LU with partial pivoting in FP64;
 * tau = 2 mu / p (eq. tau).  Writes rec and status[ncell]. */
int fp_closure_solve(fp_ctx* ctx, const double* mom, double* rec, int32_t* status,
                     hipStream_t s);

/* Per-particle step on particles sorted by cell, as selected by flags (in the open
 * cylinder domain MOVE also reflects diffusely off the body at T_body and gives a
 * particle whose flight ends outside the box the key ncell):
 *   FP_STEP_COLLIDE  eq. update_vel with N of eq. update_N, Philox normals with counter
 *                    (pid, step, 3, 0); then every cell is recentred on U and its energy
 *                    restored exactly (FP_EXACT) or by alpha of eq. update_alpha
 *                    (FP_PAPER).  Cells with status EMPTY or NONFINITE are untouched.
 *   FP_STEP_MOVE     x += v dt (eq. update_pos) in FP64 with diffuse isothermal walls
 *                    (re-emission draws from counter (pid, step, 4, bounce)), then key.
 *   FP_STEP_KEYS     key from the stored position only.
 * mom/rec may be NULL when COLLIDE is not set; offsets may be NULL for MOVE/KEYS only. */
int fp_step(fp_ctx* ctx, fp_particles* p, const int32_t* offsets, const double* mom,
            const double* rec, uint64_t step, uint32_t flags, hipStream_t s);

/* fp_step with the step number read from device memory (*step_dev, one uint32) when the
 * kernels run, so that a whole step can be captured once in a HIP graph and replayed
 * for successive steps.  With FP_STEP_ADVANCE the step itself adds 1 to *step_dev after
 * every kernel of the step has read it (with COLLIDE | MOVE the last kernel does it, so
 * no launch is added); without it advance the counter with fp_counter_add.  step_dev
 * must then be writable device memory that no other work uses during the step. */
int fp_step_dev(fp_ctx* ctx, fp_particles* p, const int32_t* offsets, const double* mom,
                const double* rec, const uint32_t* step_dev, uint32_t flags, hipStream_t s);
/* *ctr += inc on the device, ordered on the stream (a kernel, no memset: capturable). */
int fp_counter_add(fp_ctx* ctx, uint32_t* ctr, uint32_t inc, hipStream_t s);

/* Free-stream inflow of the open cylinder domain (boundary step of the loop).
 * Candidates are drawn uniformly in a buffer frame of width
 * (|u_inf| + 4 sqrt(2 R T_inf)) dt around the box (four rectangles: x-low, x-high, y-low,
 * y-high) with Maxwellian(u_inf, T_inf) velocities (Philox counter (pid, step, 5, 0|2);
 * the count of rectangle r is floor(lambda_r) plus a Bernoulli remainder drawn with
 * counter (r, step, 5, 1), lambda_r = n_inf area_r depth / fnum); they fly for dt and
 * those ending inside the box are kept.  fp_inject writes fp_inject_slots(ctx) slots at
 * indices [at, at + slots) of p (capacity must allow it): kept candidates with their
 * cell key, the rest with key = ncell so that the next fp_bin drops them.  pid_next
 * (device, one uint32) is the id of the first candidate and advances by the number of
 * candidates.  Returns FP_EINVAL for other geometries. */
int fp_inject(fp_ctx* ctx, fp_particles* p, int64_t at, uint32_t* pid_next, uint64_t step,
              hipStream_t s);
/* fp_inject for a particle count and a step number kept on the device (a loop captured
 * in a HIP graph): the slots start at *p->n_dev (p->n_dev required), the step number is
 * *step_dev (one uint32) when the kernels run, and afterwards *p->n_dev has advanced by
 * fp_inject_slots(ctx); with FP_STEP_ADVANCE in flags *step_dev also advances by 1 (in the
 * call's last kernel, after every kernel has read it).  If the slots would reach beyond
 * p->capacity nothing is written, *p->n_dev keeps its value and the overflow is counted
 * on the device (fp_capacity_overflows). */
int fp_inject_dev(fp_ctx* ctx, fp_particles* p, uint32_t* pid_next, uint32_t* step_dev,
                  uint32_t flags, hipStream_t s);
/* Number of fp_inject_dev calls since fp_init that found no room (synchronous read-back). */
int64_t fp_capacity_overflows(fp_ctx* ctx, hipStream_t s);
/* Number of slots fp_inject writes per call (a configuration constant). */
int64_t fp_inject_slots(const fp_ctx* ctx);
/* Gas volume of every cell [m^3] into vol[ncell] (device): cylinder cells lose the part
 * covered by the body (exact disk-rectangle areas, cells covered up to 1e-12 of their
 * area count as solid, volume 0); box geometries dx dy (1 m depth). */
int fp_cell_volumes(fp_ctx* ctx, double* vol, hipStream_t s);

/* Normalised high-order fields of the averaged particle fields (the cavity's high-order
 * diagnostics: R_ij = <c_i c_j |c|^2>, Delta_4 = <|c|^4> - 15 theta^2, DM6 = <|c|^6>, over
 * the local Maxwellian scales).  fp_sample_high adds, for every cell with particles,
 * [N, N theta, N R_ij (11 12 13 22 23 33), N <|c|^4>, N <|c|^6>] of one step's moment
 * records (mom, moments through fifth order) to hsamp[ncell][16] (device, caller-owned,
 * entries 10..15 untouched).  fp_high_order writes out[ncell][8] = (R_ij / theta^2 (6),
 * <|c|^4> / theta^2 - 15, <|c|^6> / theta^3) of the particle-weighted averages
 * (theta = sum N theta / sum N, ...): 5 delta_ij, 0 and 105 for a Maxwellian; NaN for
 * cells without particles or temperature. */
int fp_sample_high(fp_ctx* ctx, const double* mom, double* hsamp, hipStream_t s);
int fp_high_order(fp_ctx* ctx, const double* hsamp, double* out, hipStream_t s);

/* Surface sampling of the cylinder (for the C_p, C_f, C_h distributions of Sec.
 * "Extension to External Aerodynamics"): while sums is set, every diffuse re-emission at
 * the body during fp_step (MOVE) adds its exchange to sums[nbins][4] (device doubles,
 * caller-owned, zeroed by the caller): hits, normal momentum v_out.n - v_in.n, tangential
 * momentum towards the rear (v_in - v_out).t, energy (|v_in|^2 - |v_out|^2)/2, per unit
 * molecular mass, n the outward normal, t the tangent along decreasing theta, in bins of
 * the surface angle theta (0 at the rear point, pi at the front stagnation point; both
 * halves of the circle share a bin): a hit goes to bin b when
 * cos((b + 1) pi / nbins) < n_x <= cos(b pi / nbins), decided by comparing cos(theta) = n_x
 * with edges the host computes once (so every implementation bins a hit point alike,
 * which the last bits of an arctangent would not guarantee).  FP64 atomic adds (their
 * order, and so the last bits of the sums, vary from run to run).  sums = NULL stops;
 * the caller keeps sums allocated until then (the context holds only the pointer).  A HIP
 * graph captured meanwhile keeps the pointer.  FP_EINVAL for other geometries or
 * nbins outside [1, 65536]. */
int fp_wall_sampling(fp_ctx* ctx, double* sums, int32_t nbins);
/* Surface coefficients from such sums gathered over a time t_total [s]: out[nbins][4]
 * (device) = (bin-centre theta in degrees, C_p, C_f, C_h) with A = 2 R (pi / nbins) depth,
 * p = m fnum S_n / (A t), tau = m fnum S_t / (A t), q = m fnum S_e / (A t),
 * C_p = (p - p_inf) / (rho_inf U^2 / 2), C_f = tau / (rho_inf U^2 / 2),
 * C_h = q / (rho_inf U^3 / 2), rho_inf = n_inf m, p_inf = n_inf k_B T_inf, U = |u_inf|. */
int fp_surface_coefficients(fp_ctx* ctx, const double* sums, int32_t nbins, double t_total,
                            double* out, hipStream_t s);

/* ---- adaptive quadtree of the cylinder domain -----------------------------------------
 * Sec. "Extension to External Aerodynamics", Problem Description: hierarchical Cartesian
 * quadtree, cells split on the normalised deviation |phi - phi_parent| / (|phi| + eps)
 * of density, temperature and pressure from the parent (tau_grad), on a particle-count
 * limit (N_max) and on shock pressure (P > factor p_inf); four sibling leaves merge when
 * all deviations are below tau_coarse, the merged count is low and every sibling has been
 * unchanged for age_min steps.  The grid of the context (nx, ny) is the finest level; the
 * base grid has (nx >> max_level) x (ny >> max_level) cells.  With a tree, "cell" in every
 * other entry point means leaf: ncell = fp_ncell(ctx) leaves, numbered depth first (base
 * cells row-major, children (0,0) (1,0) (0,1) (1,1)); keys computed from positions
 * (fp_step, fp_inject) are leaf ids; fp_cell_volumes gives leaf gas volumes; fp_rebin
 * is refused (its neighbour structure is that of the uniform grid), fp_bin sorts. */
typedef struct fp_amr_params {
    double tau_grad;      /* split: largest deviation from the parent above this (0.10) */
    double tau_coarse;    /* merge: every sibling's deviation below this (0.05) */
    double shock_factor;  /* split: pressure above shock_factor p_inf (1.2) */
    double p_inf;         /* free-stream pressure [Pa] */
    double n_max;         /* split: mean particles per sampled step above this; merge: the
                             merged cell's mean at most this */
    double n_grad;        /* fewer sampled particles: no gradient or shock test (a sibling
                             with fewer counts as no deviation) */
    double eps;           /* regularisation of the deviation */
    int32_t age_min;      /* steps unchanged before a leaf may merge (2000) */
    int32_t reserved;     /* must be 0 */
} fp_amr_params;

/* Give a FP_CYLINDER2D context a tree of base cells only (all leaves at level 0,
 * ages 0), 0 <= max_level <= 4, nx and ny multiples of 2^max_level.  Synchronous. */
int fp_amr_init(fp_ctx* ctx, int32_t max_level);
/* One adaptation (synchronous on s: returns once the new leaf count is known).  acc
 * [ncell][16] (device) holds the sampling sums (layout of samp, e.g. from fp_sample) of
 * the current leaves over the steps since the last adaptation; the fields behind the
 * criteria are rho = (sum N / samples) fnum / V, U = sum v / sum N, theta = (sum |v|^2 /
 * sum N - |U|^2) / 3, P = rho m theta, a parent's from the sums of its children.  One
 * level per call: flagged leaves split, flagged parents of four leaves merge; ages of
 * unchanged leaves advance by steps.  Afterwards acc is zeroed for the new leaves; samp
 * (optional) is carried over (a new child takes its parent's sums scaled by its share of
 * the parent's gas volume, a merged cell the sum of its children's, the sample count
 * kept); p (optional, its n slots) gets the keys of the new leaves from the positions,
 * and key = ncell for slots whose key was not a cell (deleted, unused).  FP_EINVAL
 * without a tree. */
int fp_amr_adapt(fp_ctx* ctx, const fp_amr_params* prm, double* acc, double* samp,
                 fp_particles* p, int32_t steps, hipStream_t s);
/* Number of cells (leaves with a tree, else nx ny). */
int32_t fp_ncell(const fp_ctx* ctx);
/* Number of tree nodes (all levels; 0 without a tree). */
int64_t fp_amr_nodes(const fp_ctx* ctx);
/* Copies of the tree (device buffers, each optional): state[nodes] (0 absent, 1 leaf,
 * 2 refined; level-major, row-major in a level), age[nodes], leafmap[nx ny] (leaf of
 * every fine cell), leaf_node[ncell] (node of every leaf). */
int fp_amr_tree(fp_ctx* ctx, int8_t* state, int32_t* age, int32_t* leafmap, int32_t* leaf_node,
                hipStream_t s);

/* Time averaging (the "average_results" step): adds the raw sums of every cell,
 * reconstructed from mom, to samp (layout samp above). */
int fp_sample(fp_ctx* ctx, const double* mom, double* samp, hipStream_t s);

/* Diagnostics of the time-averaged fields in samp (after the loop): the averaged state
 * (ratios of the cumulative sums), the normalised stress Theta_ij / theta - delta_ij, the
 * normalised heat flux q^_i = <c_i |c|^2> / (2 theta^1.5), and the covariance-based
 * entropy proxies of Sec. "Covariance-based entropy-proxy audit on the stagnation line and
 * cylinder surface" (eqs. cyl_theta_def, cyl_entropy_eq, cyl_DG, cyl_entropy_kinG):
 * ds_eq = 3/2 log(theta/theta_inf) - log(n/n_inf), D_G = -1/2 log det(Theta/theta),
 * ds_kinG = ds_eq - (D_G - dg_inf), D_q = |q^|^2 / 5.  theta_inf [m^2/s^2] and n_inf
 * [1/m^3] are the caller's reference state (e.g. the free stream), dg_inf its D_G.
 * diag[ncell][FP_DIAG_STRIDE] doubles: 0 particles per sample, 1 number density [1/m^3]
 * (cut-cell gas volume on the cylinder), 2-4 U [m/s], 5 theta, 6 T [K], 7-12 stress
 * (11 12 13 22 23 33), 13-15 q^, 16 ds_eq, 17 D_G, 18 ds_kinG, 19 D_q, 20-23 zero;
 * entries 2-19 are NaN for cells without particles or with theta <= 0, D_G and ds_kinG
 * also where det(Theta/theta) <= 1e-12 (a singular sample covariance: fewer than four
 * particles, say). */
#define FP_DIAG_STRIDE 24
int fp_diagnostics(fp_ctx* ctx, const double* samp, double theta_inf, double n_inf,
                   double dg_inf, double* diag, hipStream_t s);


/* ---- learned closure (project extension) -------------------------------------------
 * The paper replaces the closure build and solve by a dense network evaluated on the GPU
 * with standardised inputs and outputs (Secs. "Phase 1-2", "Phase 3", Algorithm
 * "Accelerated ML Simulation Loop").  Here: 27 features of the theta-normalised moments
 *   [P/th - I (6), T/th^1.5 (10), R/th^2 - 5I (6), W/th^2.5 (3), eps_hat, log10 N]
 * -> 128 -> 128 -> 128 (SiLU) -> 9 normalised coefficients
 *   [tau Ct - 5 eps_hat I (6), tau sqrt(theta) Gamma (3)],
 * zero padded to 32 inputs and 16 outputs, BF16 MFMA with FP32 accumulation.
 *
 * Parameter vector: FP_NN_PARAMS floats, device memory, owned by the caller:
 *   W1[128][32] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[16][128] b4[16]
 *   x_mean[32] x_std[32] y_mean[16] y_std[16]
 * (W[out][in] row-major; the first FP_NN_TRAIN floats are trained, the scalers fixed). */
#define FP_NN_PARAMS 39408
#define FP_NN_TRAIN 39312
#define FP_NN_FEATURES 32
#define FP_NN_OUTPUTS 16
#define FP_LOSS_MSE 0        /* mean over samples of the squared error of standardised targets */
#define FP_LOSS_RESIDUAL 1   /* mean over samples of |A y - b|^2 of the normalised 9x9 system */

typedef struct fp_nn fp_nn;

/* Create a network handle on ctx with training scratch for batches up to max_batch
 * (0: inference only).  Synchronous. */
int fp_nn_create(fp_ctx* ctx, int64_t max_batch, fp_nn** out);
void fp_nn_destroy(fp_nn* net);
/* Convert params (FP_NN_PARAMS floats, device, read only) into the network's BF16 image
 * held by net (Sec. "Phase 3": the trained weights, biases and scalers are exported once
 * and then evaluated forward only inside the loop).  Weights are rounded to bfloat16 (nearest
 * even) and laid out for the MFMA fragments; the biases and the scalers stay FP32.  Must be
 * called before any inference on net and again after params change; asynchronous on s.
 * FP_EINVAL for a null pointer or a handle made on another context. */
int fp_nn_load(fp_ctx* ctx, fp_nn* net, const float* params, hipStream_t s);
/* Learned closure of every cell (Algorithm "Accelerated ML Simulation Loop"): network
 * outputs de-standardised, then checked against the cell's own normalised 9x9 system;
 * accepted if |A y - b| <= tol_abs + tol_rel |b| (status FP_CELL_NN), otherwise solved
 * exactly (FP_CELL_NN_FALLBACK).  tol_abs = +infinity skips the check (and the assembly
 * of the system): every finite output is accepted, non-finite ones fall back (on a
 * context with moment_order 3, which has no system to solve, they take the Langevin drift:
 * FP_CELL_SINGULAR; such a context accepts only tol_abs = +infinity).  relax in (0, 1]:
 * accepted coefficients are blended with the cell's previous ones in rec, C = relax C_net
 * + (1 - relax) C_prev, the same for Gamma, when that record carries coefficients (the
 * temporal under-relaxation of the cylinder deployment, Sec. "Extension to External
 * Aerodynamics"); 1
 * takes the network's values.  Cells that are EMPTY/NONFINITE/FEW are treated as in
 * fp_closure_solve.  Same rec layout. */
int fp_closure_nn(fp_ctx* ctx, const fp_nn* net, const double* mom, double* rec,
                  int32_t* status, double tol_abs, double tol_rel, double relax, hipStream_t s);
/* fp_closure_nn for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results, bit for bit, but the network outputs pass between the two kernels through a
 * fixed library array of FP_NN_NOALLOC_CELLS x 16 floats (16 MiB, one per GPU, held until
 * the process ends; its device address is looked up by fp_nn_create) instead of the
 * handle's buffer.  The call itself allocates nothing.  FP_EINVAL if the context has more
 * than FP_NN_NOALLOC_CELLS cells.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other contexts) race and must be serialised by
 * the caller; each call writes every entry it reads, so nothing needs clearing.
 * fp_nn_outputs still returns the outputs of the last fp_closure_nn, not of this call. */
#define FP_NN_NOALLOC_CELLS 262144
int fp_closure_nn_noalloc(fp_ctx* ctx, const fp_nn* net, const double* mom, double* rec,
                          int32_t* status, double tol_abs, double tol_rel, double relax,
                          hipStream_t s);
/* Coefficient-sensitivity probe (Sec. "Heuristic coefficient-sensitivity probe"): npass
 * >= 1 forward passes of the network on every cell's moments (mom [ncell][32], device)
 * with inference-time dropout of rate p in [0, 1) on the three hidden layers (inverted:
 * kept activations scaled by 1/(1-p); hidden unit u of layer l is dropped in pass k of
 * cell c when word u % 4 of Philox4x32-10 with key (seed low, seed high) and counter
 * (c, k, 6, 32 (l-1) + u / 4) is below floor(p 2^32)).  Per cell the standard deviation
 * (1/npass) over the passes of each de-standardised normalised coefficient (the targets
 * above), and sens[c] = (sigma_Stress, sigma_Heat), the Euclidean norms over the six
 * stress and the three heat-flux coefficients (device, [ncell][2] doubles, caller-owned);
 * cells with N <= 1 or theta <= 0 get zeros.  Not a deployment path: the closure itself
 * never drops units.  FP_EINVAL for a bad argument. */
int fp_nn_sensitivity(fp_ctx* ctx, const fp_nn* net, const double* mom, int32_t npass,
                      double p, uint64_t seed, double* sens, hipStream_t s);
/* The network alone (no check, no de-normalisation): standardised outputs of every cell's
 * moments into y[ncell][16] floats (device, caller-owned); rows 9..15 zero, cells with
 * N <= 1 or theta <= 0 evaluated on zero features. */
int fp_nn_infer(fp_ctx* ctx, const fp_nn* net, const double* mom, float* y, hipStream_t s);
/* Copy the standardised network outputs of the last fp_closure_nn ([ncell][16]). */
int fp_nn_outputs(fp_ctx* ctx, const fp_nn* net, float* y, hipStream_t s);
/* Raw (unstandardised) features of n moment records: feats[n][32] floats. */
int fp_nn_features(fp_ctx* ctx, const double* mom, int64_t n, float* feats, hipStream_t s);
/* Normalised 9x9 systems of n moment records (eq. system9x9 with the entries of Table
 * matrix_system, as fp_closure_solve assembles them, divided by the cell's theta powers so
 * that the unknowns are the normalised coefficients [tau Ct - 5 eps_hat I, tau sqrt(theta)
 * Gamma]): mom[n][32] device doubles in, sys[n][90] device doubles out (caller-owned), A
 * row-major then b.  The training data of the residual loss.  Only records with theta > 0
 * give finite systems (the caller filters the others out, as the training set builders
 * do).  FP_EINVAL for n < 0 or a null pointer; n = 0 does nothing. */
int fp_closure_build(fp_ctx* ctx, const double* mom, int64_t n, double* sys, hipStream_t s);
/* Gradient of the loss w.r.t. the trainable parameters for a batch of B samples (Sec.
 * "Phase 1-2": standardised inputs and targets, a mean-squared-error loss; the residual
 * loss is this library's alternative, the same system the deployment check of Algorithm
 * "Accelerated ML Simulation Loop" evaluates).  feats[B][32] raw features; targets[B][16]
 * raw normalised targets (FP_LOSS_MSE) or sys[B][90] (FP_LOSS_RESIDUAL); all device, read
 * only.  Writes the trainable prefix of grad[FP_NN_PARAMS] (the scaler tail is left as
 * it is) and *loss (device float).  B in [1, max_batch of net], else FP_EINVAL.  Fixed-order
 * reductions: bitwise reproducible. */
int fp_nn_grad(fp_ctx* ctx, fp_nn* net, const float* params, const float* feats,
               const float* targets, const double* sys, int64_t B, int32_t loss_kind,
               float* grad, float* loss, hipStream_t s);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) step t >= 1 on the trainable prefix. */
int fp_nn_adam(fp_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t t,
               float lr, hipStream_t s);
/* fp_nn_grad followed by fp_nn_adam (Sec. "Phase 1-2": Adam on the loss), in place on
 * params, m and v (device, caller-owned, FP_NN_PARAMS floats each, m and v zero before
 * t = 1). */
int fp_nn_train_step(fp_ctx* ctx, fp_nn* net, float* params, float* m, float* v, int64_t t,
                     float lr, const float* feats, const float* targets, const double* sys,
                     int64_t B, int32_t loss_kind, float* loss, hipStream_t s);

/* ---- the paper's LITE surrogate -------------------------------------------------------
 * Secs. "Phase 1-2", "Neural Network Architecture" and "Phase 3": a 16-256-256-256-256-9
 * network with ReLU hidden layers and a linear output, on 16 low-order inputs of the cell
 *   [rho, T, U_x, U_y, U_z, Pi_11, Pi_12, Pi_13, Pi_22, Pi_23, Pi_33, q_x, q_y, q_z, DM2, nu]
 * with rho = N fnum / V m, T = theta m / k_B, Pi_ij = rho (P_ij - theta delta_ij),
 * q_i = rho S_i / 2, DM2 = <|c|^2> = 3 theta, nu = 1 / tau (eq. tau), predicting the
 * coefficients of the update record [Ct (6), Gamma (3)] in solver units; inputs and
 * outputs standardised.  It needs moments through third order only: on a context with
 * moment_order 3 (the high-order gather skipped) it runs unchecked.  BF16 MFMA with FP32
 * accumulation; inference in one kernel with the layers' weights staged through LDS.
 *
 * Parameter vector: FP_LITE_PARAMS floats, device memory, owned by the caller:
 *   W1[256][16] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[256][256] b4[256]
 *   W5[16][256] b5[16] x_mean[16] x_std[16] y_mean[16] y_std[16]
 * (W[out][in] row-major; output rows 9..15 are padding and should be zero; the first
 * FP_LITE_TRAIN floats are trained, the scalers fixed).  The paper's 204,041 trainable
 * parameters are this prefix without the padded output rows. */
#define FP_LITE_PARAMS 205904
#define FP_LITE_TRAIN 205840
#define FP_LITE_FEATURES 16
typedef struct fp_lite fp_lite;
/* Create a LITE network on ctx with training scratch for batches up to max_batch (0:
 * inference only).  Synchronous. */
int fp_lite_create(fp_ctx* ctx, int64_t max_batch, fp_lite** out);
void fp_lite_destroy(fp_lite* net);
/* Convert params (FP_LITE_PARAMS floats, device, read only) into the network's BF16 image
 * (Sec. "Phase 3": weights, biases and scalers exported once for forward-only use); same
 * rules as fp_nn_load. */
int fp_lite_load(fp_ctx* ctx, fp_lite* net, const float* params, hipStream_t s);
/* Standardised network outputs of every cell's moments: y[ncell][16] floats (rows 9..15
 * zero; cells with N <= 1 or theta <= 0 are evaluated on zero inputs). */
int fp_lite_infer(fp_ctx* ctx, const fp_lite* net, const double* mom, float* y, hipStream_t s);
/* Learned closure of every cell with the LITE network: same contract, checks, statuses,
 * fallback and relax as fp_closure_nn (Algorithm "Accelerated ML Simulation Loop"). */
int fp_closure_lite(fp_ctx* ctx, const fp_lite* net, const double* mom, double* rec,
                    int32_t* status, double tol_abs, double tol_rel, double relax, hipStream_t s);
/* Raw inputs of n moment records: feats[n][16] floats; nvol[n] (device, optional): real
 * molecules per particle over the cell volume of each record (NULL: fnum_over_vol). */
int fp_lite_features(fp_ctx* ctx, const double* mom, const double* nvol, int64_t n, float* feats,
                     hipStream_t s);
/* Raw targets [Ct (6), Gamma (3), 0 (7)] of n update records: targets[n][16] floats. */
int fp_lite_targets(fp_ctx* ctx, const double* rec, int64_t n, float* targets, hipStream_t s);
/* Gradient of the mean over the batch of the squared error of the standardised targets
 * (the paper's MSE) w.r.t. the trainable parameters: grad[FP_LITE_PARAMS] (trainable
 * prefix written) and *loss (device float); fixed-order reductions, bitwise reproducible. */
int fp_lite_grad(fp_ctx* ctx, fp_lite* net, const float* params, const float* feats,
                 const float* targets, int64_t B, float* grad, float* loss, hipStream_t s);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) step t >= 1 on the trainable prefix. */
int fp_lite_adam(fp_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t t,
                 float lr, hipStream_t s);
/* fp_lite_grad followed by fp_lite_adam (Sec. "Phase 1-2": Adam on the MSE). */
int fp_lite_train_step(fp_ctx* ctx, fp_lite* net, float* params, float* m, float* v, int64_t t,
                       float lr, const float* feats, const float* targets, int64_t B, float* loss,
                       hipStream_t s);

/* Per-column mean and population standard deviation of x[n][k] (device floats; k <= 4096)
 * into mean[k], stdev[k] (device doubles): the standardising scalers of the networks'
 * inputs and targets (Sec. "Phase 3": means and scales; Sec. "Phase 1-2": StandardScaler).
 * FP64 sums in a fixed order: bitwise reproducible. */
int fp_column_stats(fp_ctx* ctx, const float* x, int64_t n, int32_t k, double* mean, double* stdev,
                    hipStream_t s);

/* ---- differentiation (project extension) -------------------------------------------
 * Reverse mode through fp_moments and fp_closure_solve for the map
 *   particle velocities -> cell coefficients (Ct, Gamma) of rec entries 0..8,
 * including the dependence of tau (eq. tau) and of the normalisation on theta. */

/* ybar[ncell][16]: gradient w.r.t. rec entries 0..8 (others ignored).  Writes
 * mombar[ncell][32], the gradient w.r.t. the moment record (theta folded into the
 * diagonal of P; zero rows for cells whose status is not FP_CELL_OK). */
int fp_closure_solve_backward(fp_ctx* ctx, const double* mom, const double* rec,
                              const double* ybar, double* mombar, hipStream_t s);
/* Gradient w.r.t. every particle velocity of a scalar whose gradient w.r.t. the moment
 * records is mombar (entries U, theta, P, T, R, W, H are honoured), recomputed from the
 * velocities: vbar_p = (1/N) (G(c_p) - <G>) + Ubar / N with G = sum_k mbar_k grad f_k.
 * vbar_* are double arrays in the order of p. */
int fp_moments_backward(fp_ctx* ctx, const fp_particles* p, const int32_t* offsets,
                        const double* mom, const double* mombar, double* vbar_x,
                        double* vbar_y, double* vbar_z, hipStream_t s);
/* Normalised training targets [tau Ct - 5 eps_hat I, tau sqrt(theta) Gamma] of n update
 * records: targets[n][16] floats (entries 9..15 zero). */
int fp_nn_targets(fp_ctx* ctx, const double* rec, int64_t n, float* targets, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif /* FP_H */
