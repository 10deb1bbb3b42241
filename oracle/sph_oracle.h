/*
 * FP64 CPU oracle for the 2-D weakly-compressible SPH particle update of
 * Pourabdian, Omidvar & Morad, "Numerical simulation of liquid jet breakup using
 * smoothed particle hydrodynamics (SPH)".
 *
 * TEST INFRASTRUCTURE ONLY. This code exists to check the HIP library: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it. It
 * shares no source, header, table or helper with the HIP library. It is plain
 * and slow on purpose: every array is in particle-id order, neighbour lists are
 * built with a textbook cell linked list (head/next chains, Section 2-7) and
 * re-sorted by id, and each particle sum follows its equation term by term.
 *
 * Conventions: r_ab = r_a - r_b, v_ab = v_a - v_b; grad_a W_ab = F(r) r_ab.
 * Particle types: 0 fluid, 1 fixed wall, 2 piston, 3 inactive.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t kernel;        /* 0 Wendland (eq. 28), 1 cubic spline (eq. 27) */
    int32_t density;       /* 0 continuity (eq. 7), 1 summation (eq. 6) for fluid particles */
    double h;              /* smoothing length */
    double rho0, c0, gamma;/* Tait reference density, sound speed, exponent (eq. 26) */
    double alpha;          /* artificial-viscosity coefficient (eq. 10) */
    double eta2_h2;        /* eta^2 / h^2 (eq. 10) */
    double sigma;          /* surface-tension coefficient (eq. 12, 24) */
    double eps_h;          /* eps * h, normal filter threshold (eq. 20) */
    double gravity[2];
    double courant;        /* Cr (eq. 32) */
    double dt_fixed;       /* > 0: use this step instead of eq. 30-32 */
    double box_lo[2], box_hi[2];   /* fluid leaving this box becomes inactive */
    double cell_size;      /* cell edge of the linked-list grid */
    double piston_dir[2], piston_u, piston_amp, piston_omega;
    int32_t boundary;      /* 0 dynamic boundary particles, 1 repulsive-force walls (eq. 29) */
    int32_t gravity_plane; /* 1: g acts only on fluid with r . g/|g| >= gravity_from */
    double wall_spacing;   /* spacing of the wall particles (repulsive walls) */
    double gravity_from;
} orc_params;

enum { ORC_FLUID = 0, ORC_WALL = 1, ORC_PISTON = 2, ORC_INACTIVE = 3 };

/* Outputs of one evaluation of the right-hand sides. Arrays sized n (or 2n for
 * vectors, interleaved x,y), per-system arrays sized n_sys. Any pointer may be
 * NULL to skip that output. */
typedef struct {
    double *colour;    /* C_a, eq. 14 (self included) */
    double *drho;      /* d rho_a / dt, eq. 7 */
    double *apv;       /* pressure + viscous acceleration, eq. 9-10 */
    double *nrm;       /* n_a, eq. 18 */
    int32_t *nflag;    /* N_a, eq. 20 */
    double *kappa;     /* kappa_a, eq. 23 */
    double *asurf;     /* (a_s)_a, eq. 24 */
    double *acc;       /* total acceleration, eq. 25 */
    double *vsig;      /* max_b |h v_ab . r_ab / r_ab^2|, eq. 31 */
    int32_t *nnb;      /* neighbour count (b != a) */
    double *s_drho;    /* absolute-sum scales for error bounds */
    double *s_acc;
    double *s_nrm;
    double *dt_f, *dt_cv, *dt;  /* per system, eq. 30-32 */
    double *rho;       /* density used by this evaluation (eq. 6 where summed) */
} orc_eval_out;

/* Kernel value W(r,h) and F(r,h) with grad_a W = F r_ab (2-D). */
double orc_kernel_w(int kernel, double r, double h);
double orc_kernel_f(int kernel, double r, double h);

/* Tait pressure and sound speed per particle (eq. 26). */
void orc_eos(const orc_params* p, int64_t n, const double* rho, double* P, double* c);

/* Grid geometry of one system's linked-list cells. */
void orc_grid(const orc_params* p, int64_t* nx, int64_t* ny);

/* Neighbour lists: all active b != a of the same system with r_ab^2 < (2h)^2,
 * ascending id. start has n+1 entries. Returns the total number of pairs; nbr is
 * filled only if it is non-NULL and cap is large enough. brute != 0 uses the
 * O(N^2) definition instead of the cell list. */
int64_t orc_neighbors(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
                      const int32_t* type, int brute, int64_t* start, int32_t* nbr, int64_t cap);

/* Cell keys and the sorted order: key = (cell offset of the system) + cx*ny + cy,
 * inactive particles get the key one past the last cell. perm lists particle
 * ids ordered by (key, id); keys_sorted the matching keys. */
void orc_sort(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
              const int32_t* type, uint64_t* keys_sorted, int64_t* perm);

/* One evaluation of every right-hand side at the given state. wall_normal
 * (2n, may be NULL): the unit normal, into the fluid, of every boundary
 * particle of a system with repulsive-force walls (boundary = 1). */
int orc_eval(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
             const double* vel, const double* rho, const double* mass, const int32_t* type,
             const double* wall_normal, const orc_eval_out* out);

/* nsteps predictor-corrector steps in place (time per system advanced). dt_out
 * (n_sys, may be NULL) receives the last step's dt. */
int orc_step(int n_sys, const orc_params* p, const int64_t* off, double* pos, double* vel,
             double* rho, const double* mass, int32_t* type, const double* wall_normal,
             double* time, int nsteps, double* dt_out);

/* Breakup length (Section 3-2): per system, the fluid particles whose
 * coordinate along `axis`, xi = x axis_x + y axis_y (no FMA), is at least
 * xi_start[s] are taken in order of xi; the jet is broken at the first pair of
 * consecutive particles more than gap_h * h apart, and length[s] is the
 * coordinate of the nearer one minus xi_start[s] (broken[s] = 1). Without such
 * a gap, length[s] is that of the farthest particle (broken[s] = 0); without
 * any such particle 0. */
void orc_breakup(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
                 const int32_t* type, const double* axis, const double* xi_start, double gap_h,
                 double* length, int32_t* broken);

/* Number of OpenMP threads the oracle runs on, and a way to change it. */
int orc_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
