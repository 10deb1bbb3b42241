/*
 * FP64 CPU oracle for the 2-D WCSPH particle update (Pourabdian, Omidvar & Morad).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path. Plain C, FP64, no FMA
 * contraction (built with -ffp-contract=off), OpenMP over particles.
 *
 * Readings of the paper used here (where it is silent or garbled):
 *  - Wendland kernel (eq. 28): the printed 2-D constant does not normalise the
 *    printed polynomial; the unit-integral constant 7/(64 pi) of the
 *    (1+2q)(2-q)^4 form is used.
 *  - Self contributions (b = a) are included in the W sums of eq. 14 and the
 *    denominator of eq. 23; gradient sums exclude them (grad W_aa = 0).
 *  - eq. 18 uses the smoothed colour of eq. 14 for C_b and C_a.
 *  - eq. 24 uses the constant sigma and the un-normalised n_a.
 *  - eq. 31 is read as |h v_ab . r_ab| / r_ab^2 with c_s = c_a.
 *  - |f_a| in eq. 30 is the total acceleration (eq. 25) of a fluid particle.
 *  - Boundaries are dynamic particles: they enter every sum of a fluid
 *    particle; their own density follows eq. 7 summed over fluid neighbours only
 *    (a boundary interacts with the fluid, never with another boundary, as in a
 *    force-type wall) and eq. 26, and it is held at or above rho0 after every
 *    update so a boundary pushes fluid away but never pulls it (the paper's
 *    wall of Section 2-6 is a purely repulsive force); walls stay fixed, the
 *    piston follows its prescribed motion, and boundaries carry no normal
 *    (N = 0) or surface force.
 *  - Density summation (eq. 6), a per-system option: at every evaluation a
 *    fluid particle's density is rho_a = sum_b m_b W_ab over every active
 *    particle of its system, itself included, from the positions alone; it
 *    replaces the continuity equation for that particle (the integrator keeps
 *    the density of the latest evaluation). Boundary particles keep the rule
 *    above.
 *  - The predictor-corrector (Section 2-8 cites it without equations):
 *    half step phi_1/2 = phi_n + dt/2 D_n; full step rho_{n+1} = rho_n + dt Drho_1/2,
 *    v_{n+1} = v_n + dt a_1/2, r_{n+1} = r_n + dt (v_n + dt/2 a_1/2); dt from
 *    the evaluation at state n.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- kernels */

/* Cubic spline, eq. 27: W = (10/(7 pi h^2)) f(q); Wendland, eq. 28:
 * W = (7/(64 pi h^2)) (1+2q)(2-q)^4, both with support q = r/h < 2. */
static double w_poly(int kernel, double q) {
    if (q >= 2.0) return 0.0;
    if (kernel == 1) {
        if (q <= 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
        double t = 2.0 - q;
        return 0.25 * t * t * t;
    }
    double t = 2.0 - q;
    return (1.0 + 2.0 * q) * t * t * t * t;
}

/* d/dq of the polynomial above. */
static double dw_poly(int kernel, double q) {
    if (q >= 2.0) return 0.0;
    if (kernel == 1) {
        if (q <= 1.0) return -3.0 * q + 2.25 * q * q;
        double t = 2.0 - q;
        return -0.75 * t * t;
    }
    double t = 2.0 - q;
    /* d/dq[(1+2q)(2-q)^4] = 2(2-q)^4 - 4(1+2q)(2-q)^3 */
    return 2.0 * t * t * t * t - 4.0 * (1.0 + 2.0 * q) * t * t * t;
}

static double norm_const(int kernel, double h) {
    if (kernel == 1) return 10.0 / (7.0 * PI * h * h);
    return 7.0 / (64.0 * PI * h * h);
}

double orc_kernel_w(int kernel, double r, double h) {
    return norm_const(kernel, h) * w_poly(kernel, r / h);
}

/* grad_a W_ab = dW/dr * r_ab / r = (norm/h) dW/dq * r_ab / r  =>  F = norm dW/dq / (h r). */
double orc_kernel_f(int kernel, double r, double h) {
    if (r <= 0.0) return 0.0;
    return norm_const(kernel, h) * dw_poly(kernel, r / h) / (h * r);
}

/* --------------------------------------------------------------------- EOS */

static double tait_B(const orc_params* p) { return p->rho0 * p->c0 * p->c0 / p->gamma; }

/* eq. 26: P = B [(rho/rho0)^gamma - 1]; sound speed c^2 = dP/drho. */
static double tait_p(const orc_params* p, double rho) {
    return tait_B(p) * (pow(rho / p->rho0, p->gamma) - 1.0);
}
static double tait_c(const orc_params* p, double rho) {
    return p->c0 * pow(rho / p->rho0, 0.5 * (p->gamma - 1.0));
}

void orc_eos(const orc_params* p, int64_t n, const double* rho, double* P, double* c) {
    for (int64_t i = 0; i < n; ++i) {
        if (P) P[i] = tait_p(p, rho[i]);
        if (c) c[i] = tait_c(p, rho[i]);
    }
}

/* ------------------------------------------------------------- cell lists */

void orc_grid(const orc_params* p, int64_t* nx, int64_t* ny) {
    double inv = 1.0 / p->cell_size;
    *nx = (int64_t)floor((p->box_hi[0] - p->box_lo[0]) * inv) + 1;
    *ny = (int64_t)floor((p->box_hi[1] - p->box_lo[1]) * inv) + 1;
}

static int64_t cell_coord(double x, double lo, double inv, int64_t ncell) {
    double t = floor((x - lo) * inv);
    if (!(t >= 0.0)) t = 0.0; /* also catches NaN */
    if (t > (double)(ncell - 1)) t = (double)(ncell - 1);
    return (int64_t)t;
}

/* Whether a particle enters the SPH sums of its system: every active one, but
 * for repulsive-force walls (eq. 29) only the fluid -- walls act on the fluid
 * through the wall force alone. */
static int in_sums(const orc_params* p, int32_t t) {
    return t != ORC_INACTIVE && !(p->boundary == 1 && t != ORC_FLUID);
}

/* The pair predicate: r_ab^2 < (2h)^2 in FP64, squares summed left to right. */
static int within(const double* pos, int64_t a, int64_t b, double R2) {
    double dx = pos[2 * b] - pos[2 * a];
    double dy = pos[2 * b + 1] - pos[2 * a + 1];
    double r2 = dx * dx + dy * dy;
    return r2 < R2;
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/* Neighbours of each particle of one system [o0, o1), via a head/next cell
 * linked list or by brute force. Pass 1 (nbr == NULL) counts, pass 2 fills. */
static void system_neighbors(const orc_params* p, int64_t o0, int64_t o1, const double* pos,
                             const int32_t* type, int brute, int64_t* count_or_start,
                             int32_t* nbr, int fill) {
    int64_t n = o1 - o0;
    double R2 = (2.0 * p->h) * (2.0 * p->h);
    if (n <= 0) return;
    if (brute) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t a = o0; a < o1; ++a) {
            if (!in_sums(p, type[a])) { if (!fill) count_or_start[a] = 0; continue; }
            int64_t k = fill ? count_or_start[a] : 0;
            for (int64_t b = o0; b < o1; ++b) {
                if (b == a || !in_sums(p, type[b])) continue;
                if (within(pos, a, b, R2)) {
                    if (fill) nbr[k] = (int32_t)b;
                    ++k;
                }
            }
            if (!fill) count_or_start[a] = k;
        }
        return;
    }
    int64_t nx, ny;
    orc_grid(p, &nx, &ny);
    double inv = 1.0 / p->cell_size;
    int reach = (int)ceil(2.0 * p->h / p->cell_size);
    if (reach < 1) reach = 1;
    int64_t ncell = nx * ny;
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* cx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* cy = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t a = o0; a < o1; ++a) {
        int64_t i = a - o0;
        cx[i] = cell_coord(pos[2 * a], p->box_lo[0], inv, nx);
        cy[i] = cell_coord(pos[2 * a + 1], p->box_lo[1], inv, ny);
        if (!in_sums(p, type[a])) { next[i] = -2; continue; }
        int64_t c = cx[i] * ny + cy[i];
        next[i] = head[c];
        head[c] = i;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = o0; a < o1; ++a) {
        int64_t i = a - o0;
        if (!in_sums(p, type[a])) { if (!fill) count_or_start[a] = 0; continue; }
        int64_t k0 = fill ? count_or_start[a] : 0, k = k0;
        for (int64_t X = cx[i] - reach; X <= cx[i] + reach; ++X) {
            if (X < 0 || X >= nx) continue;
            for (int64_t Y = cy[i] - reach; Y <= cy[i] + reach; ++Y) {
                if (Y < 0 || Y >= ny) continue;
                for (int64_t j = head[X * ny + Y]; j >= 0; j = next[j]) {
                    int64_t b = j + o0;
                    if (b == a) continue;
                    if (within(pos, a, b, R2)) {
                        if (fill) nbr[k] = (int32_t)b;
                        ++k;
                    }
                }
            }
        }
        if (fill) qsort(nbr + k0, (size_t)(k - k0), sizeof(int32_t), cmp_i32);
        else count_or_start[a] = k;
    }
    free(head); free(next); free(cx); free(cy);
}

int64_t orc_neighbors(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
                      const int32_t* type, int brute, int64_t* start, int32_t* nbr, int64_t cap) {
    int64_t n = off[n_sys];
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int s = 0; s < n_sys; ++s)
        system_neighbors(&p[s], off[s], off[s + 1], pos, type, brute, cnt, NULL, 0);
    start[0] = 0;
    for (int64_t a = 0; a < n; ++a) start[a + 1] = start[a] + cnt[a];
    int64_t total = start[n];
    if (nbr && total <= cap) {
        for (int64_t a = 0; a < n; ++a) cnt[a] = start[a];
        for (int s = 0; s < n_sys; ++s)
            system_neighbors(&p[s], off[s], off[s + 1], pos, type, brute, cnt, nbr, 1);
    }
    free(cnt);
    return total;
}

/* -------------------------------------------------------------- cell sort */

typedef struct { uint64_t key; int64_t id; } key_id;

static int cmp_key_id(const void* x, const void* y) {
    const key_id* a = (const key_id*)x;
    const key_id* b = (const key_id*)y;
    if (a->key != b->key) return (a->key > b->key) - (a->key < b->key);
    return (a->id > b->id) - (a->id < b->id);
}

void orc_sort(int n_sys, const orc_params* p, const int64_t* off, const double* pos,
              const int32_t* type, uint64_t* keys_sorted, int64_t* perm) {
    int64_t n = off[n_sys];
    uint64_t base = 0;
    uint64_t* sys_base = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_sys);
    for (int s = 0; s < n_sys; ++s) {
        int64_t nx, ny;
        orc_grid(&p[s], &nx, &ny);
        sys_base[s] = base;
        base += (uint64_t)(nx * ny);
    }
    uint64_t trash = base;
    key_id* kv = (key_id*)malloc(sizeof(key_id) * (size_t)n);
    for (int s = 0; s < n_sys; ++s) {
        int64_t nx, ny;
        orc_grid(&p[s], &nx, &ny);
        double inv = 1.0 / p[s].cell_size;
        for (int64_t a = off[s]; a < off[s + 1]; ++a) {
            kv[a].id = a;
            if (!in_sums(&p[s], type[a])) { kv[a].key = trash; continue; }
            int64_t X = cell_coord(pos[2 * a], p[s].box_lo[0], inv, nx);
            int64_t Y = cell_coord(pos[2 * a + 1], p[s].box_lo[1], inv, ny);
            kv[a].key = sys_base[s] + (uint64_t)(X * ny + Y);
        }
    }
    qsort(kv, (size_t)n, sizeof(key_id), cmp_key_id);
    for (int64_t j = 0; j < n; ++j) {
        if (keys_sorted) keys_sorted[j] = kv[j].key;
        if (perm) perm[j] = kv[j].id;
    }
    free(kv);
    free(sys_base);
}

/* ------------------------------------------------------------ repulsive walls */

/* Force per unit mass on fluid particle a from the repulsive-force walls of its
 * system (eq. 29, f = n R(psi) P(xi) eps(z, u_perp)). The paper names the three
 * functions without defining them (its references are missing); they are read
 * as the published forms of those references:
 *   psi = (r_a - r_k) . n_k (normal distance), xi = |(r_a - r_k) - psi n_k|;
 *   R(psi) = A (1 - q) / sqrt(q), q = psi / (2h), A = 0.01 c_a^2 / h, for 0 < psi < 2h;
 *   P(xi) = (1 + cos(pi xi / db)) / 2 for xi < db, db the wall-particle spacing, so
 *   that the P of equally spaced wall particles sum to 1 wherever the fluid
 *   particle is along a straight wall (the force does not ripple along it);
 *   eps = eps(z) + eps(u_perp), eps(z) = 1 (no still-water depth in these runs),
 *   eps(u_perp) = 0 for u_perp = (v_a - v_k) . n_k >= 0, else min(|20 u_perp| / c0, 1).
 * sf receives the sum of the magnitudes (error scale). */
static void wall_force(const orc_params* p, int64_t o0, int64_t o1, int64_t a, const double* pos,
                       const double* vel, const int32_t* type, const double* wn, double c_a,
                       double* fx, double* fy, double* sf) {
    double h = p->h, db = p->wall_spacing > 0.0 ? p->wall_spacing : h / 1.3;
    double A = 0.01 * c_a * c_a / h;
    for (int64_t k = o0; k < o1; ++k) {
        if (type[k] != ORC_WALL && type[k] != ORC_PISTON) continue;
        double nx = wn[2 * k], ny = wn[2 * k + 1];
        double dx = pos[2 * a] - pos[2 * k], dy = pos[2 * a + 1] - pos[2 * k + 1];
        double psi = dx * nx + dy * ny;
        if (!(psi > 0.0 && psi < 2.0 * h)) continue;
        double tx = dx - psi * nx, ty = dy - psi * ny;
        double xi = sqrt(tx * tx + ty * ty);
        if (!(xi < db)) continue;
        double q = psi / (2.0 * h);
        double R = A * (1.0 - q) / sqrt(q);
        double P = 0.5 * (1.0 + cos(PI * xi / db));
        double up = (vel[2 * a] - vel[2 * k]) * nx + (vel[2 * a + 1] - vel[2 * k + 1]) * ny;
        double eu = up >= 0.0 ? 0.0 : fmin(fabs(20.0 * up) / p->c0, 1.0);
        double f = R * P * (1.0 + eu);
        *fx += f * nx;
        *fy += f * ny;
        *sf += fabs(f);
    }
}

/* ------------------------------------------------------------ evaluation */

static double dot2(double ax, double ay, double bx, double by) { return ax * bx + ay * by; }

int orc_eval(int n_sys, const orc_params* prm, const int64_t* off, const double* pos,
             const double* vel, const double* rho_in, const double* mass, const int32_t* type,
             const double* wall_normal, const orc_eval_out* out) {
    int64_t n = off[n_sys];
    int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t total = orc_neighbors(n_sys, prm, off, pos, type, 0, start, NULL, 0);
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    orc_neighbors(n_sys, prm, off, pos, type, 0, start, nbr, total);

    double* P = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* C = (double*)malloc(sizeof(double) * (size_t)n);
    double* nv = (double*)calloc((size_t)(2 * n), sizeof(double));
    double* snrm = (double*)calloc((size_t)n, sizeof(double));
    double* nhat = (double*)calloc((size_t)(2 * n), sizeof(double));
    int32_t* N = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    double* kap = (double*)calloc((size_t)n, sizeof(double));
    double* as = (double*)calloc((size_t)(2 * n), sizeof(double));
    double* apv = (double*)calloc((size_t)(2 * n), sizeof(double));
    double* acc = (double*)calloc((size_t)(2 * n), sizeof(double));
    double* dr = (double*)calloc((size_t)n, sizeof(double));
    double* vs = (double*)calloc((size_t)n, sizeof(double));
    double* sdr = (double*)calloc((size_t)n, sizeof(double));
    double* sacc = (double*)calloc((size_t)n, sizeof(double));
    double* rho = (double*)malloc(sizeof(double) * (size_t)n);
    memcpy(rho, rho_in, sizeof(double) * (size_t)n);

    for (int s = 0; s < n_sys; ++s) {
        const orc_params* p = &prm[s];
        int64_t o0 = off[s], o1 = off[s + 1];
        double h = p->h;
        int K = p->kernel;
        double eps = p->eps_h / h;                 /* eq. 20 threshold eps = 0.01/h */
        double eta2 = p->eta2_h2 * h * h;          /* eq. 10 */
        double W0 = orc_kernel_w(K, 0.0, h);

        /* Density summation (eq. 6) over every active particle, self included,
         * for the fluid particles of a system that uses it. */
        if (p->density == 1) {
#pragma omp parallel for schedule(dynamic, 128)
            for (int64_t a = o0; a < o1; ++a) {
                if (type[a] != ORC_FLUID) continue;
                double sum = mass[a] * W0;
                for (int64_t k = start[a]; k < start[a + 1]; ++k) {
                    int64_t b = nbr[k];
                    double rx = pos[2 * a] - pos[2 * b], ry = pos[2 * a + 1] - pos[2 * b + 1];
                    sum += mass[b] * orc_kernel_w(K, sqrt(rx * rx + ry * ry), h);
                }
                rho[a] = sum;
            }
        }

        /* Tait pressure and sound speed (eq. 26). */
        for (int64_t a = o0; a < o1; ++a) { P[a] = tait_p(p, rho[a]); c[a] = tait_c(p, rho[a]); }

        /* Colour function, eq. 14, over every active particle, self included. */
#pragma omp parallel for schedule(dynamic, 128)
        for (int64_t a = o0; a < o1; ++a) {
            if (!in_sums(p, type[a])) { C[a] = 0.0; continue; }
            double sum = mass[a] / rho[a] * W0;
            for (int64_t k = start[a]; k < start[a + 1]; ++k) {
                int64_t b = nbr[k];
                double rx = pos[2 * a] - pos[2 * b], ry = pos[2 * a + 1] - pos[2 * b + 1];
                double r = sqrt(rx * rx + ry * ry);
                sum += mass[b] / rho[b] * orc_kernel_w(K, r, h);
            }
            C[a] = sum;
        }

        /* Continuity (eq. 7), momentum with artificial viscosity (eq. 9-10),
         * interface normal (eq. 18) and the signal term of eq. 31. */
#pragma omp parallel for schedule(dynamic, 128)
        for (int64_t a = o0; a < o1; ++a) {
            if (!in_sums(p, type[a])) continue;
            int fluid = type[a] == ORC_FLUID;
            double d = 0.0, sd = 0.0, ax = 0.0, ay = 0.0, sa = 0.0;
            double nx = 0.0, ny = 0.0, sn = 0.0, vmax = 0.0;
            for (int64_t k = start[a]; k < start[a + 1]; ++k) {
                int64_t b = nbr[k];
                /* a boundary particle's density responds to the fluid only */
                if (!fluid && type[b] != ORC_FLUID) continue;
                double rx = pos[2 * a] - pos[2 * b], ry = pos[2 * a + 1] - pos[2 * b + 1];
                double r2 = rx * rx + ry * ry;
                double r = sqrt(r2);
                double F = orc_kernel_f(K, r, h);
                double gx = F * rx, gy = F * ry;           /* grad_a W_ab */
                double vx = vel[2 * a] - vel[2 * b], vy = vel[2 * a + 1] - vel[2 * b + 1];
                double vdotr = dot2(vx, vy, rx, ry);
                double t = mass[b] * dot2(vx, vy, gx, gy);
                d += t;
                sd += fabs(t);
                double sig = fabs(h * vdotr / r2);
                if (sig > vmax) vmax = sig;
                if (!fluid) continue;
                double pa = P[a] / (rho[a] * rho[a]), pb = P[b] / (rho[b] * rho[b]);
                double Pi = 0.0;
                if (vdotr < 0.0) {
                    double cbar = 0.5 * (c[a] + c[b]);
                    double rbar = 0.5 * (rho[a] + rho[b]);
                    Pi = -p->alpha * h * cbar * vdotr / (rbar * (r2 + eta2));
                }
                double coef = mass[b] * (pa + pb + Pi);
                ax -= coef * gx;
                ay -= coef * gy;
                sa += mass[b] * (fabs(pa) + fabs(pb) + fabs(Pi)) * sqrt(gx * gx + gy * gy);
                double vol = mass[b] / rho[b];
                nx += vol * (C[b] - C[a]) * gx;
                ny += vol * (C[b] - C[a]) * gy;
                sn += vol * (fabs(C[b]) + fabs(C[a])) * sqrt(gx * gx + gy * gy);
            }
            dr[a] = d; sdr[a] = sd; vs[a] = vmax;
            apv[2 * a] = ax; apv[2 * a + 1] = ay; sacc[a] = sa;
            nv[2 * a] = nx; nv[2 * a + 1] = ny; snrm[a] = sn;
        }

        /* Normal filter and unit normal, eq. 20-21 (fluid only). */
        for (int64_t a = o0; a < o1; ++a) {
            N[a] = 0; nhat[2 * a] = 0.0; nhat[2 * a + 1] = 0.0;
            if (type[a] != ORC_FLUID) continue;
            double m = sqrt(nv[2 * a] * nv[2 * a] + nv[2 * a + 1] * nv[2 * a + 1]);
            if (m > eps) {
                N[a] = 1;
                nhat[2 * a] = nv[2 * a] / m;
                nhat[2 * a + 1] = nv[2 * a + 1] / m;
            }
        }

        /* Filtered, normalised curvature (eq. 22-23), surface-tension
         * acceleration (eq. 24) and the total acceleration (eq. 25). */
#pragma omp parallel for schedule(dynamic, 128)
        for (int64_t a = o0; a < o1; ++a) {
            if (type[a] != ORC_FLUID) continue;
            double k_a = 0.0, sx = 0.0, sy = 0.0, scale_k = 0.0;
            if (N[a]) {
                double num = 0.0, den = mass[a] / rho[a] * W0, snum = 0.0;
                double ma = sqrt(nv[2 * a] * nv[2 * a] + nv[2 * a + 1] * nv[2 * a + 1]);
                for (int64_t k = start[a]; k < start[a + 1]; ++k) {
                    int64_t b = nbr[k];
                    if (!N[b]) continue;                  /* min(N_a, N_b) = 0 */
                    double rx = pos[2 * a] - pos[2 * b], ry = pos[2 * a + 1] - pos[2 * b + 1];
                    double r = sqrt(rx * rx + ry * ry);
                    double F = orc_kernel_f(K, r, h);
                    double vol = mass[b] / rho[b];
                    double dnx = nhat[2 * b] - nhat[2 * a], dny = nhat[2 * b + 1] - nhat[2 * a + 1];
                    num += vol * F * dot2(dnx, dny, rx, ry);
                    den += vol * orc_kernel_w(K, r, h);
                    double mb = sqrt(nv[2 * b] * nv[2 * b] + nv[2 * b + 1] * nv[2 * b + 1]);
                    snum += vol * fabs(F) * r * (2.0 + snrm[a] / ma + snrm[b] / mb);
                }
                k_a = num / den;
                double f = -p->sigma / rho[a] * k_a;
                sx = f * nv[2 * a];
                sy = f * nv[2 * a + 1];
                scale_k = p->sigma / rho[a] * (ma * (snum + fabs(k_a) * den) / den + fabs(k_a) * snrm[a]);
            }
            kap[a] = k_a;
            as[2 * a] = sx; as[2 * a + 1] = sy;
            /* repulsive-force walls (eq. 29) */
            double fx = 0.0, fy = 0.0, sf = 0.0;
            if (p->boundary == 1 && wall_normal) wall_force(p, o0, o1, a, pos, vel, type, wall_normal, c[a], &fx, &fy, &sf);
            /* gravity everywhere, or beyond a plane normal to g */
            double gx = p->gravity[0], gy = p->gravity[1];
            if (p->gravity_plane) {
                double gn = hypot(gx, gy);
                if (!(pos[2 * a] * (gx / gn) + pos[2 * a + 1] * (gy / gn) >= p->gravity_from)) gx = gy = 0.0;
            }
            acc[2 * a] = apv[2 * a] + sx + gx + fx;
            acc[2 * a + 1] = apv[2 * a + 1] + sy + gy + fy;
            sacc[a] += scale_k + sqrt(gx * gx + gy * gy) + sf;
        }

        /* Time-step limits, eq. 30-32. */
        double dtf = INFINITY, dtcv = INFINITY;
        for (int64_t a = o0; a < o1; ++a) {
            if (!in_sums(p, type[a])) continue;
            double v = h / (c[a] + vs[a]);
            if (v < dtcv) dtcv = v;
            if (type[a] != ORC_FLUID) continue;
            double am = sqrt(acc[2 * a] * acc[2 * a] + acc[2 * a + 1] * acc[2 * a + 1]);
            if (am > 0.0) {
                double v2 = sqrt(h / am);
                if (v2 < dtf) dtf = v2;
            }
        }
        if (out->dt_f) out->dt_f[s] = dtf;
        if (out->dt_cv) out->dt_cv[s] = dtcv;
        if (out->dt) {
            /* a system without active particles has no limit: it does not advance */
            double d = p->dt_fixed > 0.0 ? p->dt_fixed : p->courant * fmin(dtf, dtcv);
            out->dt[s] = isfinite(d) ? d : 0.0;
        }
    }

    if (out->colour) memcpy(out->colour, C, sizeof(double) * (size_t)n);
    if (out->drho) memcpy(out->drho, dr, sizeof(double) * (size_t)n);
    if (out->apv) memcpy(out->apv, apv, sizeof(double) * (size_t)(2 * n));
    if (out->nrm) memcpy(out->nrm, nv, sizeof(double) * (size_t)(2 * n));
    if (out->nflag) memcpy(out->nflag, N, sizeof(int32_t) * (size_t)n);
    if (out->kappa) memcpy(out->kappa, kap, sizeof(double) * (size_t)n);
    if (out->asurf) memcpy(out->asurf, as, sizeof(double) * (size_t)(2 * n));
    if (out->acc) memcpy(out->acc, acc, sizeof(double) * (size_t)(2 * n));
    if (out->vsig) memcpy(out->vsig, vs, sizeof(double) * (size_t)n);
    if (out->s_drho) memcpy(out->s_drho, sdr, sizeof(double) * (size_t)n);
    if (out->s_acc) memcpy(out->s_acc, sacc, sizeof(double) * (size_t)n);
    if (out->s_nrm) memcpy(out->s_nrm, snrm, sizeof(double) * (size_t)n);
    if (out->nnb)
        for (int64_t a = 0; a < n; ++a) out->nnb[a] = (int32_t)(start[a + 1] - start[a]);
    if (out->rho) memcpy(out->rho, rho, sizeof(double) * (size_t)n);

    free(rho);
    free(start); free(nbr); free(P); free(c); free(C); free(nv); free(snrm); free(nhat);
    free(N); free(kap); free(as); free(apv); free(acc); free(dr); free(vs); free(sdr); free(sacc);
    return 0;
}

/* ------------------------------------------------------------ integrator */

/* Piston travel X(t) for the speed U (1 + A sin(w t)) along piston_dir. */
static double piston_travel(const orc_params* p, double t) {
    if (p->piston_omega == 0.0) return p->piston_u * t;
    return p->piston_u * (t + p->piston_amp * (1.0 - cos(p->piston_omega * t)) / p->piston_omega);
}
static double piston_speed(const orc_params* p, double t) {
    return p->piston_u * (1.0 + p->piston_amp * sin(p->piston_omega * t));
}

int orc_step(int n_sys, const orc_params* prm, const int64_t* off, double* pos, double* vel,
             double* rho, const double* mass, int32_t* type, const double* wall_normal, double* time,
             int nsteps, double* dt_out) {
    int64_t n = off[n_sys];
    double* ph = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    double* vh = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    double* rh = (double*)malloc(sizeof(double) * (size_t)n);
    double* d0 = (double*)malloc(sizeof(double) * (size_t)n);
    double* a0 = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    double* d1 = (double*)malloc(sizeof(double) * (size_t)n);
    double* a1 = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    double* dt = (double*)malloc(sizeof(double) * (size_t)n_sys);
    double* dt_unused = (double*)malloc(sizeof(double) * (size_t)n_sys);
    double* re0 = (double*)malloc(sizeof(double) * (size_t)n);   /* densities of the two evaluations */
    double* re1 = (double*)malloc(sizeof(double) * (size_t)n);

    for (int step = 0; step < nsteps; ++step) {
        orc_eval_out o0;
        memset(&o0, 0, sizeof o0);
        o0.drho = d0; o0.acc = a0; o0.dt = dt; o0.rho = re0;
        orc_eval(n_sys, prm, off, pos, vel, rho, mass, type, wall_normal, &o0);

        /* predictor: half step */
        for (int s = 0; s < n_sys; ++s) {
            const orc_params* p = &prm[s];
            double hdt = 0.5 * dt[s];
            double dX = piston_travel(p, time[s] + hdt) - piston_travel(p, time[s]);
            double U = piston_speed(p, time[s] + hdt);
            for (int64_t a = off[s]; a < off[s + 1]; ++a) {
                ph[2 * a] = pos[2 * a]; ph[2 * a + 1] = pos[2 * a + 1];
                vh[2 * a] = vel[2 * a]; vh[2 * a + 1] = vel[2 * a + 1];
                rh[a] = rho[a];
                if (type[a] == ORC_INACTIVE) continue;
                /* a summed density is recomputed by the next evaluation; a
                 * repulsive wall's density does not evolve */
                if (p->density == 1 && type[a] == ORC_FLUID) rh[a] = re0[a];
                else if (p->boundary == 1 && type[a] != ORC_FLUID) rh[a] = rho[a];
                else rh[a] = rho[a] + hdt * d0[a];
                if (type[a] != ORC_FLUID && rh[a] < p->rho0) rh[a] = p->rho0;  /* walls only repel */
                if (type[a] == ORC_FLUID) {
                    ph[2 * a] = pos[2 * a] + hdt * vel[2 * a];
                    ph[2 * a + 1] = pos[2 * a + 1] + hdt * vel[2 * a + 1];
                    vh[2 * a] = vel[2 * a] + hdt * a0[2 * a];
                    vh[2 * a + 1] = vel[2 * a + 1] + hdt * a0[2 * a + 1];
                } else if (type[a] == ORC_PISTON) {
                    ph[2 * a] = pos[2 * a] + p->piston_dir[0] * dX;
                    ph[2 * a + 1] = pos[2 * a + 1] + p->piston_dir[1] * dX;
                    vh[2 * a] = p->piston_dir[0] * U;
                    vh[2 * a + 1] = p->piston_dir[1] * U;
                }
            }
        }

        orc_eval_out o1;
        memset(&o1, 0, sizeof o1);
        o1.drho = d1; o1.acc = a1; o1.dt = dt_unused; o1.rho = re1;
        orc_eval(n_sys, prm, off, ph, vh, rh, mass, type, wall_normal, &o1);

        /* corrector: full step from state n with the half-step derivatives */
        for (int s = 0; s < n_sys; ++s) {
            const orc_params* p = &prm[s];
            double T = dt[s];
            double dX = piston_travel(p, time[s] + T) - piston_travel(p, time[s]);
            double U = piston_speed(p, time[s] + T);
            for (int64_t a = off[s]; a < off[s + 1]; ++a) {
                if (type[a] == ORC_INACTIVE) continue;
                /* summation: the density of the latest (half-step) evaluation */
                if (p->density == 1 && type[a] == ORC_FLUID) rho[a] = re1[a];
                else if (p->boundary == 1 && type[a] != ORC_FLUID) rho[a] = rho[a];
                else rho[a] = rho[a] + T * d1[a];
                if (type[a] != ORC_FLUID && rho[a] < p->rho0) rho[a] = p->rho0;  /* walls only repel */
                if (type[a] == ORC_FLUID) {
                    double vx = vel[2 * a], vy = vel[2 * a + 1];
                    pos[2 * a] = pos[2 * a] + T * (vx + 0.5 * T * a1[2 * a]);
                    pos[2 * a + 1] = pos[2 * a + 1] + T * (vy + 0.5 * T * a1[2 * a + 1]);
                    vel[2 * a] = vx + T * a1[2 * a];
                    vel[2 * a + 1] = vy + T * a1[2 * a + 1];
                    if (pos[2 * a] < p->box_lo[0] || pos[2 * a] > p->box_hi[0] ||
                        pos[2 * a + 1] < p->box_lo[1] || pos[2 * a + 1] > p->box_hi[1])
                        type[a] = ORC_INACTIVE;
                } else if (type[a] == ORC_PISTON) {
                    pos[2 * a] += p->piston_dir[0] * dX;
                    pos[2 * a + 1] += p->piston_dir[1] * dX;
                    vel[2 * a] = p->piston_dir[0] * U;
                    vel[2 * a + 1] = p->piston_dir[1] * U;
                }
            }
            time[s] += T;
            if (dt_out) dt_out[s] = T;
        }
    }
    free(ph); free(vh); free(rh); free(d0); free(a0); free(d1); free(a1); free(dt); free(dt_unused);
    free(re0); free(re1);
    return 0;
}

/* ------------------------------------------------------------ breakup */

static int cmp_f64(const void* x, const void* y) {
    double a = *(const double*)x, b = *(const double*)y;
    return (a > b) - (a < b);
}

/* The breakup criterion of Section 3-2: two particles consecutive along the
 * jet farther apart than the gap (1.5 h in the paper). Plain definition: sort
 * the coordinates and look at consecutive differences. */
void orc_breakup(int n_sys, const orc_params* prm, const int64_t* off, const double* pos,
                 const int32_t* type, const double* axis, const double* xi_start, double gap_h,
                 double* length, int32_t* broken) {
    for (int s = 0; s < n_sys; ++s) {
        int64_t o0 = off[s], o1 = off[s + 1], m = 0;
        double* xi = (double*)malloc(sizeof(double) * (size_t)(o1 - o0 + 1));
        for (int64_t a = o0; a < o1; ++a) {
            if (type[a] != ORC_FLUID) continue;
            double t = pos[2 * a] * axis[0] + pos[2 * a + 1] * axis[1];
            if (t >= xi_start[s]) xi[m++] = t;
        }
        qsort(xi, (size_t)m, sizeof(double), cmp_f64);
        double gap = gap_h * prm[s].h;
        length[s] = m ? xi[m - 1] - xi_start[s] : 0.0;
        broken[s] = 0;
        for (int64_t i = 0; i + 1 < m; ++i) {
            if (xi[i + 1] - xi[i] > gap) {
                length[s] = xi[i] - xi_start[s];
                broken[s] = 1;
                break;
            }
        }
        free(xi);
    }
}
