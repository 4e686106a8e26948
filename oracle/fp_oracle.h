/*
 * fp_oracle.h -- plain FP64 CPU oracle of the cubic Fokker-Planck particle step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code, header or constant
 * table with the GPU library; it is written from the paper's equations:
 *   - cubic drift (Sec. "Formulation of the cubic-FP model", eq. cubic_drift),
 *   - isotropic diffusion and its Ito form (eqs. cubic_diffusion, sde_vel),
 *   - the 9x9 moment-matching system (eq. system9x9, Table matrix_system),
 *   - the mixed OU/Euler velocity update (eqs. update_vel, update_N, update_alpha),
 *   - the position update (eq. update_pos),
 *   - the loop order of Algorithm "Baseline Physics Simulation Loop".
 * Everything is double precision.  Where a storage precision of float is configured,
 * stored particle values are rounded to float at exactly the points the GPU path
 * stores them, so that discrete decisions (cell keys, wall hits) are taken on the
 * same stored numbers.
 */
#ifndef FP_ORACLE_H
#define FP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* geometry kinds */
enum { OR_COUETTE1D = 0, OR_CAVITY2D = 1, OR_CYLINDER2D = 2 };
/* particle storage precision */
enum { OR_F32 = 0, OR_F64 = 1 };
/* conservation mode after the velocity update */
enum { OR_EXACT = 0, OR_PAPER = 1 };
/* per-cell closure status */
enum { OR_OK = 0, OR_EMPTY = 1, OR_FEW = 2, OR_SINGULAR = 3, OR_NONFINITE = 4,
       OR_NN = 5, OR_NN_FALLBACK = 6 };
/* Philox stream purposes (third counter word) */
enum { OR_PURPOSE_COLLISION = 3, OR_PURPOSE_WALL = 4, OR_PURPOSE_INJECT = 5 };

/* Cell record layout, 32 doubles per cell:
 * [N, U1..3, theta, P11 P12 P13 P22 P23 P33,
 *  T111 T112 T113 T122 T123 T133 T222 T223 T233 T333,
 *  R11 R12 R13 R22 R23 R33, W1..3, H, pad]                                             */
#define OR_MOM_STRIDE 32
/* Update record layout, 16 doubles per cell:
 * [Ct11 Ct12 Ct13 Ct22 Ct23 Ct33, G1..3, tau, theta, E, eps2, sigma, status, pad]   */
#define OR_REC_STRIDE 16
/* Sampling sums, 16 doubles per cell:
 * [sum N, sum v1..3, sum v_i v_j (11 12 13 22 23 33), sum v_i |v|^2 (3), n_samples, pad] */
#define OR_SAMP_STRIDE 16

typedef struct or_config {
    int32_t geometry;       /* OR_COUETTE1D or OR_CAVITY2D */
    int32_t precision;      /* OR_F32 or OR_F64 */
    int32_t conserve;       /* OR_EXACT or OR_PAPER */
    int32_t nx, ny;         /* cells along x and y (ny = 1 for 1-D) */
    int32_t n_min;          /* fewer particles than this: Langevin fallback */
    int32_t max_bounces;    /* wall interactions per particle per step */
    double x0, y0;          /* domain origin */
    double lx, ly;          /* domain extent */
    double dx, dy;          /* cell size */
    double dt;              /* time step */
    double kB, mass;        /* Boltzmann constant, molecular mass */
    double mu_ref, T_ref, omega;   /* VHS viscosity law mu = mu_ref (T/T_ref)^omega */
    double fnum_over_vol;   /* real molecules per particle divided by cell volume */
    double eps_hat;         /* dimensionless cubic stabiliser, eps^2 = eps_hat/(theta tau) */
    double pivot_tol;       /* |pivot| below this in the normalised system: singular */
    double T_wall[4];       /* wall temperatures: x_lo, x_hi, y_lo, y_hi */
    double u_wall[4][3];    /* wall velocities */
    uint64_t seed;
    /* cylinder in an open domain (OR_CYLINDER2D) */
    double circle[3];       /* centre x, centre y, radius */
    double T_body;          /* cylinder wall temperature */
    double n_inf;           /* free-stream number density */
    double u_inf[3];        /* free-stream velocity */
    double T_inf;           /* free-stream temperature */
    double fnum;            /* real molecules per simulator particle */
    double depth;           /* extent along z */
} or_config;

/* Philox4x32-10 of Salmon et al. (SC'11): one block of four 32-bit outputs. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* uniforms u_k = (out_k + 1/2) 2^-32 from the block with counter (pid, step, purpose, sub),
 * key (seed low word, seed high word). */
void or_uniforms(uint64_t seed, uint32_t pid, uint32_t step, uint32_t purpose, uint32_t sub,
                 double u[4]);
/* three standard normals by Box-Muller on (u0,u1) and (u2,u3) */
void or_normals3(uint64_t seed, uint32_t pid, uint32_t step, uint32_t purpose, uint32_t sub,
                 double z[3]);

/* cell key from a stored position; row-major, clamped to the grid */
void or_keys(const or_config* cfg, int64_t n, const double* x, const double* y, int32_t* key);
/* stable counting sort by key: perm[j] = source index placed at slot j; offsets[ncell+1] */
void or_bin(int32_t ncell, int64_t n, const int32_t* key, int64_t* perm, int32_t* offsets);
/* central moments of each cell, record layout above */
void or_moments(int32_t ncell, const int32_t* offsets, const double* vx, const double* vy,
                const double* vz, double* mom);
/* cell gas state: tau = 2 mu / p (eq. tau), eps^2; nvol = real molecules per particle
 * divided by the cell volume (cfg->fnum_over_vol for uniform cells) */
void or_cell_params(const or_config* cfg, const double* mom_cell, double nvol, double* tau,
                    double* eps2);
/* gas volume of every cell (cylinder: the part of the cell outside the circle, times the
 * depth; box geometries: dx dy times 1) */
void or_cell_volumes(const or_config* cfg, double* vol);
/* normalised 9x9 system of one cell: A (row major 81) and b (9) */
void or_closure_system(const double* mom_cell, double eps_hat, double* A, double* b);
/* exact closure of every cell: update records and status; nvol[ncell] (real molecules
 * per particle / cell volume) or NULL for cfg->fnum_over_vol everywhere */
void or_closure(const or_config* cfg, int32_t ncell, const double* mom, const double* nvol,
                double* rec, int32_t* status);
/* velocity update of eq. update_vel with conservation (in place) */
void or_update(const or_config* cfg, int32_t ncell, const int32_t* offsets, double* vx,
               double* vy, double* vz, const uint32_t* pid, const double* mom,
               const double* rec, uint32_t step);
/* free flight of eq. update_pos with diffuse walls, then the new key (in place); in the
 * open cylinder domain a particle leaving the box gets key = ncell (deleted) */
void or_move(const or_config* cfg, int64_t n, double* x, double* y, double* vx, double* vy,
             double* vz, const uint32_t* pid, int32_t* key, uint32_t step);
/* or_move that also adds the exchange of every re-emission at the cylinder to
 * wall[nbins][4] (per unit molecular mass, bins of the surface angle theta from the rear
 * point by the edges cos(k pi / nbins) of cos theta = n_x): hits, normal momentum,
 * tangential momentum towards the rear, energy given to the wall.  wall = NULL: plain
 * or_move. */
void or_move_wall(const or_config* cfg, int64_t n, double* x, double* y, double* vx,
                  double* vy, double* vz, const uint32_t* pid, int32_t* key, uint32_t step,
                  double* wall, int32_t nbins);
/* Inflow through the open boundaries of the cylinder domain: candidates drawn uniformly
 * in a buffer frame of width (|u_inf| + 4 sqrt(2 R T_inf)) dt around the domain with a
 * Maxwellian(u_inf, T_inf) velocity fly for dt; those ending inside the domain are
 * appended (x, y, v, pid = *pid_next + candidate index, key).  Returns the number
 * appended, or -1 if more than room would be needed; *pid_next advances by the number
 * of candidates. */
int64_t or_inject(const or_config* cfg, uint32_t step, uint32_t* pid_next, int64_t room,
                  double* x, double* y, double* vx, double* vy, double* vz, uint32_t* pid,
                  int32_t* key);
/* add raw particle sums of each cell to samp */
void or_sample(int32_t ncell, const int32_t* offsets, const double* vx, const double* vy,
               const double* vz, double* samp);
/* Full loop: for each step s in [step0, step0+nsteps): bin, moments, sample if
 * s >= n_skip, closure, update, move.  Arrays are overwritten with the final state
 * (in sorted order of the last bin followed by the last move).  mom/rec/status hold
 * the last step's values; samp accumulates.  Returns 0, or -1 on allocation failure. */
int or_run(const or_config* cfg, int64_t n, double* x, double* y, double* vx, double* vy,
           double* vz, uint32_t* pid, int32_t* key, uint32_t step0, int32_t nsteps,
           uint32_t n_skip, double* mom, double* rec, int32_t* status, double* samp);
/* The same loop for the open cylinder domain: arrays have room for `capacity`
 * particles, *n is updated (deletions at the boundaries, injection after the move).
 * Returns 0, -1 on allocation failure, -2 if the capacity is exceeded. */
int or_run_open(const or_config* cfg, int64_t capacity, int64_t* n, double* x, double* y,
                double* vx, double* vy, double* vz, uint32_t* pid, int32_t* key,
                uint32_t* pid_next, uint32_t step0, int32_t nsteps, uint32_t n_skip,
                double* mom, double* rec, int32_t* status, double* samp);

/* Threads of the loops split across threads (n <= 0 keeps the OpenMP default); returns
 * the number in use (1 without OpenMP). */
int or_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
