/*
 * sph.h -- C-ABI of libsphjet, the MI355X (gfx950) particle update of a 2-D
 * weakly-compressible SPH solver with surface tension, after Pourabdian, Omidvar
 * & Morad, "Numerical simulation of liquid jet breakup using smoothed particle
 * hydrodynamics (SPH)".
 *
 * One call of sph_step advances every particle system of a context by one
 * predictor-corrector step (Section 2-8) made of:
 *   - a cell-linked-list neighbour search (Section 2-7): particles are binned in
 *     square cells and counting-sorted by cell, so every neighbourhood is a few
 *     contiguous ranges of the particle arrays;
 *   - three neighbour sweeps per evaluation: colour function (eq. 14);
 *     continuity (eq. 7), Tait pressure (eq. 26), momentum with artificial
 *     viscosity (eq. 9-10) and interface normal (eq. 18); normal filter,
 *     curvature and surface-tension acceleration (eq. 20-25);
 *   - the time-step limit of eq. 30-32, reduced on the device, and the
 *     predictor and corrector updates.
 *
 * Conventions
 *   - Every function returns an sph_status (0 = success, < 0 = error); no C++
 *     exception crosses this boundary. On error, sph_last_error(ctx) holds a
 *     message (for a NULL or not-yet-created context, sph_last_error(NULL)
 *     returns the thread's last message).
 *   - Host arrays passed in are read during the call and never retained; the
 *     caller keeps ownership. Device memory is never allocated by the library:
 *     the caller supplies one device workspace of sph_workspace_bytes() bytes
 *     and keeps it alive, unmoved, until sph_free() (sph_init_static instead
 *     takes it from a static device array the library holds).
 *   - Particle arrays are FP64 on the host, in the caller's order; that order
 *     defines the particle id (0 .. n-1). 2-vectors are interleaved (x0, y0,
 *     x1, y1, ...). Systems are contiguous id ranges given by offsets[n_sys+1].
 *     Particles of different systems never interact.
 *   - On the device positions are kept in FP64; velocities, densities and all
 *     derived quantities in the context's dtype (32 or 64 bits). Density is
 *     stored as rho - rho0, so a 32-bit context rounds each input once to
 *     float: vel -> float, mass -> float, (rho - rho0) -> float.
 *   - Work is enqueued on the HIP stream given to sph_init; sph_step returns
 *     without waiting. sph_read, sph_neighbors and sph_sync wait for the stream.
 *   - A context is used by one host thread at a time.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 2

/* Largest total particle count of a context: every per-particle array is
 * addressed with 32-bit byte offsets (16-byte records, a few padding slots). */
#define SPH_MAX_PARTICLES ((int64_t)(1 << 28) - 4096)

typedef enum {
    SPH_OK = 0,
    SPH_EINVAL = -1,     /* bad argument: NULL pointer, size, parameter out of range */
    SPH_ENOMEM = -2,     /* workspace smaller than sph_workspace_bytes() */
    SPH_EDEVICE = -3,    /* a HIP runtime call failed (message in sph_last_error) */
    SPH_EUNSTABLE = -4,  /* the device flagged a non-finite value, a density outside
                            [rho0/2, 2 rho0], or a particle that moved farther within
                            half a step than the widest rescan covers (see cell_size);
                            data was still copied out */
    SPH_ECAPACITY = -5,  /* output buffer too small (sph_neighbors) */
    SPH_ESTATE = -6      /* call not valid in the context's current state */
} sph_status;

/* Smoothing kernels, both with support 2h (Section 2-5). */
enum { SPH_WENDLAND = 0,   /* eq. 28, normalised: 7/(4 pi h^2) (1 - q/2)^4 (1 + 2q) */
       SPH_CUBIC = 1 };    /* eq. 27, 10/(7 pi h^2) times the cubic B-spline */

/* Particle types. Walls and the piston are dynamic boundary particles standing
 * in for the paper's repulsive wall (Section 2-6): they enter every neighbour
 * sum of a fluid particle; their own density obeys eq. 7 summed over fluid
 * neighbours only, is held at or above rho0 (so they push fluid away but never
 * pull it) and sets their pressure through eq. 26; walls do not move, the
 * piston follows its prescribed motion. A fluid particle that
 * leaves its system's box at the end of a step becomes INACTIVE for good and is
 * excluded from every sum. */
enum { SPH_FLUID = 0, SPH_WALL = 1, SPH_PISTON = 2, SPH_INACTIVE = 3 };

/* Per-system physical parameters (SI or nondimensional, caller's choice). */
typedef struct sph_params {
    int32_t kernel;        /* SPH_WENDLAND or SPH_CUBIC */
    int32_t closure;       /* 0: curvature from eq. 23; 1: learned closure (sph_set_closure) */
    double h;              /* smoothing length (the paper uses 1.3 dx) */
    double rho0;           /* reference density (eq. 26) */
    double c0;             /* numerical sound speed, B = rho0 c0^2 / gamma (eq. 26) */
    double gamma;          /* Tait exponent, 7 for a liquid (eq. 26) */
    double alpha;          /* artificial-viscosity coefficient alpha_vis (eq. 10) */
    double eta2_h2;        /* eta^2 / h^2, 0.01 in eq. 10 */
    double sigma;          /* surface-tension coefficient (eq. 12, 24) */
    double eps_h;          /* eps * h for the normal filter, 0.01 in eq. 20 */
    double gravity[2];     /* g (eq. 25) */
    double courant;        /* Cr in eq. 32 (0.2 in the paper), 0 < Cr <= 1 */
    double dt_fixed;       /* > 0: fixed step; otherwise dt from eq. 30-32 */
    double box_lo[2];      /* fluid outside [box_lo, box_hi] becomes inactive; */
    double box_hi[2];      /*   the box also spans the cell grid */
    double cell_size;      /* cell edge s; must exceed h (reach 2) or 2h (reach 1).
                              The neighbour search scans (2R+1)^2 cells, R = 1 if
                              s > 2h else 2, and the half step reuses the pairs
                              within R s found at the step's start while no particle
                              moves more than (R s - 2h)/2 in half a step. A system
                              in which one does scans its cells again for the half
                              step, with the reach that covers the largest
                              displacement (exact; FLAGS bit 8); beyond a reach of
                              6 cells pairs may be missed (FLAGS bit 4, SPH_EUNSTABLE) */
    double piston_dir[2];  /* unit direction of the piston's motion */
    double piston_u;       /* piston speed U: U (1 + piston_amp sin(piston_omega t)) */
    double piston_amp;
    double piston_omega;
    double closure_tol;    /* closure only: relative deviation from the plain
                              curvature above which the plain value is used (0.2) */
    int32_t density;       /* 0: density from the continuity equation (eq. 7);
                              1: density summation (eq. 6) for fluid particles --
                              at every evaluation rho_a = sum_b m_b W_ab over every
                              active particle of the system, itself included,
                              before the pressure; the integrator keeps the density
                              of the latest evaluation; the density check then has
                              no lower bound (a lone particle has m W(0)) */
    int32_t boundary;      /* 0: dynamic boundary particles (see the particle types);
                              1: repulsive-force walls (eq. 29, see sph_set_wall_normals):
                              boundary particles stay out of the cells and sums, and
                              the system's NACTIVE counts its fluid only */
    double wall_spacing;   /* repulsive walls: spacing of the wall particles along
                              the wall (0: h / 1.3) */
    int32_t gravity_plane; /* 0: g acts on every fluid particle; 1: only on those whose
                              coordinate along g, r . g/|g|, is at least gravity_from
                              (a jet whose nozzle imposes its inflow speed, with g
                              acting on the free jet beyond the nozzle exit) */
    int32_t pad_;
    double gravity_from;
} sph_params;

/* Per-context options. Zero-initialised options select the defaults. */
typedef struct sph_options {
    int32_t dtype_bits;    /* 32 or 64 (0 = 32) */
    int32_t block_sweep;   /* threads per block, neighbour sweeps: 64, 128, 192 or 256 (0 = 256) */
    int32_t block_stream;  /* threads per block, per-particle kernels (0 = 256) */
    int32_t use_graph;     /* 1: sph_step replays captured hipGraphs; 0: plain launches; -1: default (1) */
    int32_t xcd_remap;     /* 1: map workgroups so each XCD sweeps one contiguous range; -1: default (1) */
    int32_t graph_steps;   /* steps per replayed graph with use_graph (even, 0 = 8); odd remainders
                              replay a one-step graph */
    int32_t reserved[2];
} sph_options;

/* Result of sph_autotune. */
typedef struct sph_tune_result {
    double cell_factor;    /* chosen cell size as a multiple of each system's h */
    int32_t block_sweep;   /* chosen threads per block of the neighbour sweeps */
    int32_t n_tried;       /* configurations timed (0 when served from the cache) */
    double ms_per_step;    /* measured time per step of the chosen configuration */
    int32_t from_cache;    /* 1: an earlier call on the same problem class decided */
    int32_t pad_;
} sph_tune_result;

typedef struct sph_ctx sph_ctx;

/* Readable fields (sph_read). Per-particle fields come back in id order as FP64
 * (or int32/int64 where noted), whatever the storage dtype. Derivative fields
 * (DRHODT .. NFLAG) are those of the most recent evaluation: after sph_step the
 * corrector's (half-step) evaluation, after sph_evaluate the current state's. */
enum {
    SPH_F_POS = 0,        /* n x 2 */
    SPH_F_VEL = 1,        /* n x 2 */
    SPH_F_RHO = 2,        /* n */
    SPH_F_PRESSURE = 3,   /* n, eq. 26 */
    SPH_F_MASS = 4,       /* n */
    SPH_F_TYPE = 5,       /* n, int32 */
    SPH_F_DRHODT = 6,     /* n, eq. 7 */
    SPH_F_ACCEL = 7,      /* n x 2, total acceleration of eq. 25 (0 for boundaries) */
    SPH_F_COLOUR = 8,     /* n, eq. 14 */
    SPH_F_NORMAL = 9,     /* n x 2, eq. 18 (0 for boundaries) */
    SPH_F_CURV = 10,      /* n, curvature used in eq. 24 (0 where N_a = 0) */
    SPH_F_NFLAG = 11,     /* n, int32, N_a of eq. 20 */
    SPH_F_DT = 12,        /* n_sys, the last step's dt (after sph_evaluate: eq. 32 at the current state) */
    SPH_F_TIME = 13,      /* n_sys */
    SPH_F_NACTIVE = 14,   /* n_sys, int64 */
    SPH_F_SORT_KEYS = 15, /* n, uint64, cell key of each slot of the sorted arrays */
    SPH_F_SORT_PERM = 16, /* n, int64, particle id held by each slot of the sorted arrays */
    SPH_F_FLAGS = 17,     /* 1, int32, instability bits (1 non-finite, 2 density, 4 a half-step
                             displacement beyond the widest rescan) and 8, informational: some
                             half step was rescanned (see cell_size); sticky until sph_restore */
    SPH_F_CURV_PLAIN = 18,/* n, curvature of eq. 23 (equals CURV unless the closure is on) */
    SPH_F_STENCIL = 19,   /* n x 64, closure input of every particle the closure saw at the last
                             evaluation (BF16 values as FP64), zeros elsewhere */
    SPH_F_CLOSURE = 20,   /* n x 4, network output (n_1, n_2, kappa h, 1) of those particles,
                             zeros elsewhere (the last entry marks the listed particles) */
    SPH_F_FALLBACK = 21,  /* n, int32, 1 where the plain curvature replaced the network's */
    SPH_F_ALL_STATE = 22, /* sph_state_bytes() bytes: the checkpoint blob (see sph_restore) */
    SPH_F_COUNT = 23
};

/* Bytes of device workspace a context with these systems needs.
 *   opt: options (NULL = defaults); n_sys >= 1; p: n_sys parameter records;
 *   offsets: n_sys + 1 ascending particle offsets, offsets[0] = 0, total in
 *            [1, SPH_MAX_PARTICLES].
 * Errors: SPH_EINVAL for invalid parameters (see sph_params). */
sph_status sph_workspace_bytes(const sph_options* opt, int32_t n_sys, const sph_params* p,
                               const int64_t* offsets, size_t* bytes_out);

/* Create a context: copies the initial state to the device (on `stream`), sorts
 * it into cells and, with use_graph, captures the step graphs.
 *   pos, vel: 2n FP64; rho, mass: n FP64; type: n int32 (SPH_FLUID..SPH_INACTIVE)
 *   d_workspace: device pointer, 256-byte aligned, at least ws_bytes >= sph_workspace_bytes()
 *   stream: hipStream_t (NULL = the null stream)
 * Errors: SPH_EINVAL (bad pointer, parameters or type), SPH_ENOMEM (workspace too
 * small), SPH_EDEVICE. On error *out is NULL. */
sph_status sph_init(const sph_options* opt, int32_t n_sys, const sph_params* p,
                    const int64_t* offsets, const double* pos, const double* vel,
                    const double* rho, const double* mass, const int32_t* type,
                    void* d_workspace, size_t ws_bytes, void* stream, sph_ctx** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_init
 * without a workspace argument. The context is carved from a static device
 * array of SPH_STATIC_WORKSPACE_BYTES that the library holds on every device it
 * runs on until the process ends; this call allocates no device memory (no
 * hipMalloc, no graph instantiation: opt->use_graph is taken as 0, so
 * sph_step launches its kernels directly and a caller may capture them).
 *   Arguments as for sph_init, the stream's device being the current device.
 *   One such context per device at a time: its state lives in that device's
 *   array until sph_free; the array keeps the last context's contents, and
 *   sph_init_static clears what must start at zero.
 * Errors: those of sph_init; SPH_ENOMEM if the systems need more than
 * SPH_STATIC_WORKSPACE_BYTES (sph_workspace_bytes with use_graph = 0 tells);
 * SPH_ESTATE if a context created by this call is still alive on the device
 * (two such contexts would share the array and race). */
#define SPH_STATIC_WORKSPACE_BYTES (128u << 20)
sph_status sph_init_static(const sph_options* opt, int32_t n_sys, const sph_params* p,
                           const int64_t* offsets, const double* pos, const double* vel,
                           const double* rho, const double* mass, const int32_t* type,
                           void* stream, sph_ctx** out);

/* Enqueue n_steps >= 0 predictor-corrector steps; returns after enqueueing. */
sph_status sph_step(sph_ctx* ctx, int32_t n_steps);

/* Re-sort the current state and evaluate every right-hand side (eq. 7-25) and
 * the eq. 30-32 time step without advancing time (for inspection and tests). */
sph_status sph_evaluate(sph_ctx* ctx);

/* Copy one field to host memory (waits for the stream). bytes must equal the
 * field's size (n, 2n or n_sys elements of 4 or 8 bytes, see SPH_F_*).
 * Returns SPH_EUNSTABLE, after copying, if the device raised an instability flag. */
sph_status sph_read(sph_ctx* ctx, int32_t field, void* host_dst, size_t bytes);

/* Checkpoint and resume. The state of Section 2-2 (position, velocity,
 * density and mass of every particle) plus each system's time and last dt --
 * everything a step starts from, the piston's phase being its time -- as one
 * blob: sph_read(ctx, SPH_F_ALL_STATE, buf, sph_state_bytes) fills it, and
 * sph_restore loads it into a context, which may be a different one with the
 * same dtype, system count and particle count (for example one created with a
 * smaller Courant number to recover from SPH_EUNSTABLE). The blob holds the
 * stored values themselves (positions FP64; velocity, rho - rho0 and mass in
 * the context's dtype; types), in particle-id order, after a small header, so a
 * restored context continues bit for bit as the one it was read from. Derived
 * fields (DRHODT .. CURV) read zero until the next sph_step or sph_evaluate;
 * instability flags are cleared.
 * sph_state_bytes: *bytes_out = size of the blob of this context.
 * sph_restore: waits for the stream; SPH_EINVAL if bytes differs from
 * sph_state_bytes or the header does not match this context. */
sph_status sph_state_bytes(const sph_ctx* ctx, size_t* bytes_out);
sph_status sph_restore(sph_ctx* ctx, const void* state, size_t bytes);

/* Neighbour lists at the current state (Section 2-7; waits for the stream):
 * for every particle id a, the ids b != a of its system with
 * |r_a - r_b|^2 < (2h)^2, ascending. start: n + 1 int64; nbr: cap int32.
 * *total receives the number of pairs; SPH_ECAPACITY (start still filled) if
 * cap < *total. These are the pairs the sweeps visit: the call sorts the
 * current state into cells (as sph_evaluate does), runs the colour sweep that
 * records each particle's candidate mask, and walks those masks as the main
 * and surface sweeps do, with the exact pair predicate. */
sph_status sph_neighbors(sph_ctx* ctx, int64_t* start, int32_t* nbr, int64_t cap, int64_t* total);

/* Repulsive-force walls (Section 2-6, eq. 29) for the systems with
 * boundary = 1: the unit normal, pointing into the fluid, of every wall and
 * piston particle (normals: 2n FP64 in particle-id order; entries of other
 * particles are ignored; a boundary particle with a zero normal exerts no
 * force). In such a system the boundary particles stay out of every SPH sum
 * and exert on each fluid particle within 2h the force per unit mass
 * f = n R(psi) P(xi) eps(z, u_perp) of eq. 29, whose functions the paper names
 * without defining; they are taken from the published form of the method it
 * cites (psi = (r_a - r_k) . n_k, xi the distance along the wall, c_a the
 * fluid particle's sound speed, db = wall_spacing):
 *   R = 0.01 c_a^2 / h (1 - q) / sqrt(q), q = psi / (2h), for 0 < psi < 2h;
 *   P = (1 + cos(pi xi / db)) / 2 for xi < db (they sum to 1 along a straight
 *       wall of spacing db);
 *   eps = 1 + min(|20 u_perp| / c0, 1) for an approaching particle,
 *       u_perp = (v_a - v_k) . n_k < 0, else 1.
 * Wall densities do not evolve. The call records the boundary particles'
 * current positions (pistons keep their prescribed motion); until it is made
 * the walls exert no force. Waits for the stream. Errors: SPH_ESTATE (no
 * system with boundary = 1), SPH_EINVAL (NULL, a non-zero normal that is not
 * a unit vector). */
sph_status sph_set_wall_normals(sph_ctx* ctx, const double* normals);

/* Breakup length of every system at the current state (Section 3-2: the jet
 * is broken where two particles consecutive along it are more than 1.5 h
 * apart). The fluid particles whose coordinate along `axis` (2 FP64,
 * xi = x axis[0] + y axis[1], no FMA) is at least xi_start[s] (the nozzle exit)
 * are taken in order of xi; system s is broken where two consecutive ones are
 * more than gap_h * h apart: length[s] is then the coordinate of the nearer one
 * minus xi_start[s] and broken[s] = 1. Otherwise length[s] reaches the
 * farthest such particle (0 if there is none) and broken[s] = 0.
 *   axis: 2 doubles, a unit vector; xi_start, length: n_sys doubles; broken:
 *   n_sys int32; gap_h >= 1 (the paper: 1.5).
 * Waits for the stream; uses workspace of its own (bins of gap_h h / 2 along
 * each system's box). Errors: SPH_EINVAL (NULL, an axis that is not a finite
 * unit vector, a start that is not finite, gap_h < 1), SPH_ECAPACITY (fluid
 * outside its box, which a step deactivates, reaching past the bins). */
sph_status sph_breakup(sph_ctx* ctx, const double* axis, const double* xi_start, double gap_h,
                       double* length, int32_t* broken);

/* Wait for all enqueued work. */
sph_status sph_sync(sph_ctx* ctx);

/* Per-kernel timing over n_steps steps launched eagerly with a HIP event pair
 * around every kernel, on the context's stream (advances the simulation).
 * names/avg_ms/calls: arrays of max_stats entries; *n_stats receives the count. */
sph_status sph_profile(sph_ctx* ctx, int32_t n_steps, int32_t max_stats, const char** names,
                       double* avg_ms, int64_t* calls, int32_t* n_stats);

/* Pick the cell size and sweep block shape for these systems by timing: for
 * cell sizes 1.05, 1.1, 1.2 h (5 x 5 cell blocks) and 2.05, 2.2 h (3 x 3) and
 * block_sweep 256 and 128, a throwaway context is built from the given initial
 * state inside d_workspace (the caller's arrays are not modified), run for two
 * warm-up steps and two windows of trial_steps timed steps (the faster window
 * counts), and freed. A configuration later in that order replaces the best so
 * far only when it is more than 2% faster. Configurations whose
 * workspace exceeds ws_bytes are skipped; size the workspace with
 * sph_workspace_bytes() at cell_size = 1.05 h to allow all of them. The winner
 * is cached per process by (dtype, number of systems, log2 of the particle
 * count, kernels used) and reused without timing. Arguments as for sph_init;
 * opt's other fields are kept. Errors: those of sph_init; SPH_ENOMEM if no
 * configuration fits. */
sph_status sph_autotune(const sph_options* opt, int32_t n_sys, const sph_params* p, const int64_t* offsets,
                        const double* pos, const double* vel, const double* rho, const double* mass,
                        const int32_t* type, void* d_workspace, size_t ws_bytes, void* stream,
                        int32_t trial_steps, sph_tune_result* out);

/* ------------------------------------------------------------------------
 * Learned curvature closure (for systems with sph_params.closure = 1)
 *
 * For every fluid particle that passes the normal filter (eq. 20), the
 * closure builds a stencil -- the relative positions (r_b - r_a)/h of its
 * fluid neighbours within 2h, the 32 nearest (ties by particle id), written in
 * the particle's own frame e1 = n_a/|n_a| (the colour gradient of eq. 18,
 * pointing into the liquid), e2 = e1 turned by +90 degrees, ordered by their
 * angle in that frame in (-pi, pi] (ties: nearer, then lower id), zero-padded
 * to 32 pairs -- and feeds it to a 64 -> 64 -> 64 -> 3 network (tanh hidden
 * layers, linear output (n_1, n_2, kappa h): the interface normal in the
 * frame (e1, e2) and the curvature) evaluated on BF16 matrix cores with FP32
 * accumulation. The network's curvature and unit normal replace those of
 * eq. 21-23 in the surface-tension acceleration of eq. 24,
 * a_s = -(sigma / rho_a) kappa |n_a| n_hat, except where the network's
 * curvature differs from the plain estimate of eq. 23 by more than
 * closure_tol times its magnitude: there the plain estimate is used.
 *
 * Parameters are a flat FP32 vector of SPH_MLP_NPARAMS values: W1 (64 x 64,
 * row-major, input index first), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 3),
 * b3 (3). They are rounded to BF16 for the matrix products; biases stay FP32.
 * ------------------------------------------------------------------------ */
#define SPH_MLP_NPARAMS 8515

/* Install network parameters (host array of SPH_MLP_NPARAMS floats, copied)
 * in a context; until called, a closure context's network is all zeros. */
sph_status sph_set_closure(sph_ctx* ctx, const float* params);

/* Trainer: FP32 master parameters, Adam moments and BF16 working copies on the
 * device, and the forward / backward kernels. Device arrays: x (m x 64 BF16
 * stencils, row-major), targets t and outputs y (m x 3 FP32), all in device
 * memory owned by the caller; m <= max_batch. Loss is the mean squared error
 * over the m rows and 3 outputs. */
typedef struct sph_mlp sph_mlp;
sph_status sph_mlp_workspace_bytes(int64_t max_batch, size_t* bytes_out);
sph_status sph_mlp_create(const float* params, int64_t max_batch, void* d_workspace, size_t ws_bytes,
                          void* stream, sph_mlp** out);
sph_status sph_mlp_forward(sph_mlp* t, const uint16_t* d_x, int64_t m, float* d_y);
/* Gradient of the loss w.r.t. the parameters (d_grad: SPH_MLP_NPARAMS FP32,
 * flat order above) and the loss itself (d_loss: one FP32; may be NULL). */
sph_status sph_mlp_gradient(sph_mlp* t, const uint16_t* d_x, const float* d_t, int64_t m, float* d_grad,
                            float* d_loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * masters with learning rate lr; the BF16 copies follow. */
sph_status sph_mlp_train_step(sph_mlp* t, const uint16_t* d_x, const float* d_t, int64_t m, float lr,
                              float* d_loss);
/* Copy the FP32 master parameters to host memory (SPH_MLP_NPARAMS floats). */
sph_status sph_mlp_params(sph_mlp* t, float* params);
void sph_mlp_free(sph_mlp* t);

/* Release the context (waits for the stream; the workspace is the caller's). */
void sph_free(sph_ctx* ctx);

/* Message of the last error on ctx (or of the calling thread if ctx is NULL). */
const char* sph_last_error(const sph_ctx* ctx);

int32_t sph_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
