/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the binary-fluid lattice Boltzmann
 * update of He, Yang, Qin, Wen & Zhang, "The roles of wettability and surface
 * tension in droplet formation during inkjet printing" (arXiv:1702.04487),
 * Methods, Eqs. (1)-(10), with the actuation of the Results section
 * ("Actuation modeling", Fig. 1) and the wetting wall of "Reproducing the
 * experiment".
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no source, header, table or helper with the GPU library.
 *
 * Storage: array of structures in double precision,
 *   f[(y*nx + x)*9 + i]  (D2Q9, mean density n),
 *   g[(y*nx + x)*5 + i]  (D2Q5, order parameter phi).
 * Lattice units dx = dt = 1, c_s^2 = 1/3 (the 3, 9/2, 3/2 of Eq. 5).
 * Velocities c_0=(0,0) c_1=(1,0) c_2=(0,1) c_3=(-1,0) c_4=(0,-1)
 *            c_5=(1,1) c_6=(-1,1) c_7=(-1,-1) c_8=(1,-1); D2Q5 = c_0..c_4.
 *
 * Readings of passages the paper leaves silent (each is listed in the design
 * notes of the repository):
 *   chemical potential (Eq. 7's mu_phi, closure of Ref. 30 not printed):
 *       mu = 4 beta phi (phi^2 - phi*^2) - kappa lap(phi);
 *   interface width W and tension sigma -> beta = 3 sigma/(4 W phi*^4),
 *       kappa = 3 sigma W/(8 phi*^2)  (profile phi* tanh(2z/W));
 *   velocity with the Guo shift: n u = sum_i c_i f_i + F/2  (needed by Eq. 4);
 *   per-phase relaxation: C = clamp((phi/phi*+1)/2,0,1),
 *       tau_n = tau_amb + C (tau_ink - tau_amb);
 *   Eq. (10)'s index "1" is the rest direction 0;
 *   gradient stencils: isotropic nine-point sums;
 *   Eq. (8): dt = 1, g_i(x + c_i, t) is the pre-collision value stored at the
 *       destination, i.e. new g_i(y) = h_i(y - c_i) + (1-q) g_i(y) with
 *       h = g* - (1-q) g;
 *   walls: halfway bounce-back; wetting ghost phi_s = mean of its fluid axis
 *       neighbours (diagonal ones if none) + 2 Omega phi_star / W, with
 *       cos(theta) = [(1+Omega)^1.5 - (1-Omega)^1.5]/2;
 *   "fully developed" top/bottom rows: after streaming, unknown incoming
 *       populations are copied from the adjacent interior row, and the
 *       stencil mirrors phi across the open edge;
 *   driving force: +F_pos for t in [0,T_pos), -F_neg for [T_pos,T_pos+T_neg),
 *       then idle; optionally periodic; along +y on fluid nodes y < force_rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Discrete velocities and weights of the D2Q9 model, Eq. (6). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* Every field is 8 bytes wide so that a ctypes mirror needs no padding rules. */
typedef struct o_params {
    int64_t nx, ny;
    int64_t bc_y;          /* 0: periodic in y; 1: open ("fully developed") rows */
    int64_t force_rows;    /* F_b acts on fluid nodes with y < force_rows */
    int64_t t_pos, t_neg, t_idle, periodic_pulse;
    double rho_ink, rho_amb, sigma, width, gamma;
    double tau_ink, tau_amb, tau_phi;
    double theta_inner, theta_outer; /* degrees, measured through the ink */
    double f_pos, f_neg;             /* magnitudes of the +/- force pulses */
} o_params;

typedef struct o_sim {
    o_params p;
    int nx, ny;
    double phi_star, n0, beta, kappa, q;
    double wet[3];        /* omega/kappa for wall classes 1 (inner) and 2 (outer) */
    uint8_t *wall;        /* 0 fluid, 1 inner-wall solid, 2 outer-wall solid */
    double *f, *g;        /* pre-collision distributions at time t */
    double *fs, *h;       /* post-collision f* and h = g* - (1-q) g */
    double *fn, *gn;      /* next state */
    double *phi;          /* phi at fluid nodes, wetting ghost at solid nodes */
    long t;
} o_sim;

/* ---------------------------------------------------------------- closures */

/* Wetting parameter Omega for a contact angle theta (degrees), inverse of
 * cos(theta) = [(1+Omega)^{3/2} - (1-Omega)^{3/2}]/2 (Cahn wetting with the
 * phi^4 closure).  Wall of Results "Reproducing the experiment", Ref. 29. */
double o_omega_of_theta(double theta_deg)
{
    double th = theta_deg * M_PI / 180.0;
    double s = sin(th);
    double alpha = acos(s * s);
    double c = cos(alpha / 3.0);
    double mag = 2.0 * sqrt(c * (1.0 - c));
    if (theta_deg < 90.0) return mag;
    if (theta_deg > 90.0) return -mag;
    return 0.0;
}

/* cos(theta) as a function of Omega (the forward relation). */
double o_cos_theta_of_omega(double om)
{
    return 0.5 * (pow(1.0 + om, 1.5) - pow(1.0 - om, 1.5));
}

/* Driving force amplitude at step t: Fig. 1 / "Actuation modeling". */
double o_pulse(const o_params *p, long t)
{
    long period = (long)(p->t_pos + p->t_neg + p->t_idle);
    long tt = t;
    if (p->periodic_pulse && period > 0) tt = t % period;
    if (tt < p->t_pos) return p->f_pos;
    if (tt < p->t_pos + p->t_neg) return -p->f_neg;
    return 0.0;
}

/* ------------------------------------------------------------ lattice maps */

static int is_fluid(const o_sim *s, int x, int y) { return s->wall[(size_t)y * s->nx + x] == 0; }

/* Neighbour (x+dx, y+dy) with x periodic; y periodic or off-lattice.
 * Returns 0 when the neighbour is outside an open row. */
static int neighbour(const o_sim *s, int x, int y, int dx, int dy, int *xn, int *yn)
{
    int a = x + dx, b = y + dy;
    a = ((a % s->nx) + s->nx) % s->nx;
    if (b < 0 || b >= s->ny) {
        if (s->p.bc_y == 0)
            b = ((b % s->ny) + s->ny) % s->ny;
        else
            return 0;
    }
    *xn = a;
    *yn = b;
    return 1;
}

/* phi seen by a stencil: across an open row the field is mirrored
 * (zero normal gradient, "fully developed"). */
static double phi_stencil(const o_sim *s, int x, int y)
{
    x = ((x % s->nx) + s->nx) % s->nx;
    if (y < 0 || y >= s->ny) {
        if (s->p.bc_y == 0)
            y = ((y % s->ny) + s->ny) % s->ny;
        else
            y = (y < 0) ? 0 : s->ny - 1;
    }
    return s->phi[(size_t)y * s->nx + x];
}

/* ------------------------------------------------------- macroscopic fields */

/* phi = sum_i g_i at fluid nodes (Eq. 9 zeroth moment), then the wetting
 * ghost on every solid node that touches fluid. */
static void compute_phi(o_sim *s)
{
    int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (s->wall[k]) continue;
            double sum = 0.0;
            for (int i = 0; i < 5; i++) sum += s->g[k * 5 + i];
            s->phi[k] = sum;
        }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (!s->wall[k]) continue;
            double sum = 0.0;
            int cnt = 0;
            for (int pass = 0; pass < 2 && cnt == 0; pass++) {
                int i0 = pass == 0 ? 1 : 5, i1 = pass == 0 ? 5 : 9;
                for (int i = i0; i < i1; i++) {
                    int xn, yn;
                    if (!neighbour(s, x, y, CX[i], CY[i], &xn, &yn)) continue;
                    if (!is_fluid(s, xn, yn)) continue;
                    sum += s->phi[(size_t)yn * nx + xn];
                    cnt++;
                }
            }
            s->phi[k] = cnt ? sum / cnt + s->wet[s->wall[k]] : 0.0;
        }
}

typedef struct {
    double n, phi, dphix, dphiy, lap, mu, Fx, Fy, ux, uy, tau;
} node_t;

/* Gradient, Laplacian, chemical potential, force, velocity and relaxation
 * time at fluid node (x,y).  Needs compute_phi() first.  sF is the driving
 * force amplitude of the current step. */
static void node_fields(const o_sim *s, int x, int y, double sF, node_t *o)
{
    size_t k = (size_t)y * s->nx + x;
    const double *f = s->f + k * 9;
    double ph = s->phi[k];

    /* isotropic stencils: grad = (1/cs2) sum w_i c_i phi(x+c_i),
     * lap = (2/cs2) sum w_i [phi(x+c_i) - phi(x)] */
    double gx = 0.0, gy = 0.0, lap = 0.0;
    for (int i = 1; i < 9; i++) {
        double pn = phi_stencil(s, x + CX[i], y + CY[i]);
        gx += WT[i] * CX[i] * pn / CS2;
        gy += WT[i] * CY[i] * pn / CS2;
        lap += 2.0 * WT[i] * (pn - ph) / CS2;
    }

    /* chemical potential of the phi^4 free energy */
    double mu = 4.0 * s->beta * ph * (ph * ph - s->phi_star * s->phi_star) - s->kappa * lap;

    /* force of Eq. (4): mu_phi grad(phi) + F_b */
    double Fx = mu * gx, Fy = mu * gy;
    if (y < s->p.force_rows) Fy += sF;

    double n = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; i++) {
        n += f[i];
        jx += CX[i] * f[i];
        jy += CY[i] * f[i];
    }
    double C = (ph / s->phi_star + 1.0) * 0.5;
    if (C < 0.0) C = 0.0;
    if (C > 1.0) C = 1.0;

    o->n = n;
    o->phi = ph;
    o->dphix = gx;
    o->dphiy = gy;
    o->lap = lap;
    o->mu = mu;
    o->Fx = Fx;
    o->Fy = Fy;
    o->ux = (jx + 0.5 * Fx) / n;
    o->uy = (jy + 0.5 * Fy) / n;
    o->tau = s->p.tau_amb + C * (s->p.tau_ink - s->p.tau_amb);
}

/* Equilibria: Eqs. (5)-(6) for f, Eqs. (9)-(10) for g. */
static void feq(double n, double phi, double mu, double ux, double uy, double out[9])
{
    double A0 = 9.0 * n / 4.0 - 15.0 * (phi * mu + n / 3.0) / 4.0;
    double Ai = 3.0 * (phi * mu + n / 3.0);
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double cu = CX[i] * ux + CY[i] * uy;
        double A = i == 0 ? A0 : Ai;
        out[i] = WT[i] * A + WT[i] * n * (3.0 * cu - 1.5 * uu + 4.5 * cu * cu);
    }
}

static void geq(double phi, double mu, double ux, double uy, double Gam, double q, double out[5])
{
    for (int i = 0; i < 5; i++) {
        double A = i == 0 ? -2.0 * Gam * mu : 0.5 * Gam * mu;
        double B = i == 0 ? 1.0 : 0.0;
        double C = 1.0 / (2.0 * q);
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = A + B * phi + C * phi * cu;
    }
}

/* ------------------------------------------------------------ public API */

void o_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int o_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Create a simulation; wall is ny*nx bytes (0 fluid, 1 inner wall, 2 outer
 * wall).  Returns NULL on invalid input (err receives a code). */
o_sim *o_create(const o_params *p, const uint8_t *wall, int *err)
{
    *err = 0;
    if (p->nx < 3 || p->ny < 3 || p->tau_ink <= 0.5 || p->tau_amb <= 0.5 || p->tau_phi <= 0.5 ||
        p->width <= 0.0 || p->rho_ink <= p->rho_amb || p->rho_amb <= 0.0 || p->sigma < 0.0) {
        *err = 1;
        return NULL;
    }
    int nx = (int)p->nx, ny = (int)p->ny;
    size_t N = (size_t)nx * ny;
    /* an open row must have fluid directly inside it */
    if (p->bc_y == 1)
        for (int x = 0; x < nx; x++) {
            if (wall[x] == 0 && wall[(size_t)nx + x] != 0) *err = 2;
            if (wall[(size_t)(ny - 1) * nx + x] == 0 && wall[(size_t)(ny - 2) * nx + x] != 0) *err = 2;
        }
    for (size_t k = 0; k < N; k++)
        if (wall[k] > 2) *err = 3;
    if (*err) return NULL;

    o_sim *s = (o_sim *)calloc(1, sizeof(o_sim));
    s->p = *p;
    s->nx = nx;
    s->ny = ny;
    /* composition variables of Eq. (1)/(7): n = (rho_A+rho_B)/2, phi = (rho_A-rho_B)/2 */
    s->phi_star = 0.5 * (p->rho_ink - p->rho_amb);
    s->n0 = 0.5 * (p->rho_ink + p->rho_amb);
    double ps2 = s->phi_star * s->phi_star;
    s->beta = 3.0 * p->sigma / (4.0 * p->width * ps2 * ps2);
    s->kappa = 3.0 * p->sigma * p->width / (8.0 * ps2);
    s->q = 1.0 / (p->tau_phi + 0.5); /* Eq. (8) */
    s->wet[0] = 0.0;
    s->wet[1] = 2.0 * o_omega_of_theta(p->theta_inner) * s->phi_star / p->width;
    s->wet[2] = 2.0 * o_omega_of_theta(p->theta_outer) * s->phi_star / p->width;
    s->wall = (uint8_t *)malloc(N);
    memcpy(s->wall, wall, N);
    s->f = (double *)calloc(N * 9, sizeof(double));
    s->fs = (double *)calloc(N * 9, sizeof(double));
    s->fn = (double *)calloc(N * 9, sizeof(double));
    s->g = (double *)calloc(N * 5, sizeof(double));
    s->h = (double *)calloc(N * 5, sizeof(double));
    s->gn = (double *)calloc(N * 5, sizeof(double));
    s->phi = (double *)calloc(N, sizeof(double));
    s->t = 0;
    return s;
}

void o_destroy(o_sim *s)
{
    if (!s) return;
    free(s->wall);
    free(s->f);
    free(s->fs);
    free(s->fn);
    free(s->g);
    free(s->h);
    free(s->gn);
    free(s->phi);
    free(s);
}

/* Derived constants: phi*, n0, beta, kappa, q, ghost offsets, mobility. */
void o_derived(const o_sim *s, double out[8])
{
    out[0] = s->phi_star;
    out[1] = s->n0;
    out[2] = s->beta;
    out[3] = s->kappa;
    out[4] = s->q;
    out[5] = s->wet[1];
    out[6] = s->wet[2];
    /* mobility of Eq. (7) from the Chapman-Enskog expansion of Eq. (8) */
    out[7] = s->p.gamma * s->q * (s->q * s->p.tau_phi - 0.5);
}

/* Initial state: given phi (ny*nx; solid entries ignored) and optional
 * velocity (NULL = 0), n = n0 everywhere; f = f_eq, g = g_eq with mu from
 * the initial phi including wetting ghosts. */
void o_init_phi(o_sim *s, const double *phi, const double *ux, const double *uy)
{
    int nx = s->nx, ny = s->ny;
    size_t N = (size_t)nx * ny;
    /* write g so that sum_i g_i = phi, then build the ghosts */
    memset(s->g, 0, N * 5 * sizeof(double));
    memset(s->f, 0, N * 9 * sizeof(double));
    for (size_t k = 0; k < N; k++)
        if (!s->wall[k]) {
            s->g[k * 5] = phi[k];
            s->f[k * 9] = s->n0; /* only sum_i f_i = n0 matters for node_fields' n */
        }
    compute_phi(s);
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (s->wall[k]) continue;
            node_t nd;
            node_fields(s, x, y, 0.0, &nd);
            double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0;
            feq(s->n0, nd.phi, nd.mu, vx, vy, s->fn + k * 9);
            geq(nd.phi, nd.mu, vx, vy, s->p.gamma, s->q, s->gn + k * 5);
        }
    memcpy(s->f, s->fn, N * 9 * sizeof(double));
    memcpy(s->g, s->gn, N * 5 * sizeof(double));
    memset(s->fn, 0, N * 9 * sizeof(double));
    memset(s->gn, 0, N * 5 * sizeof(double));
    s->t = 0;
}

/* Initial state from a signed distance d to the ink region (positive inside):
 * phi = phi* tanh(2 d / W), the equilibrium planar profile of width W. */
void o_init_distance(o_sim *s, const double *d)
{
    size_t N = (size_t)s->nx * s->ny;
    double *phi = (double *)malloc(N * sizeof(double));
    for (size_t k = 0; k < N; k++) phi[k] = s->phi_star * tanh(2.0 * d[k] / s->p.width);
    o_init_phi(s, phi, NULL, NULL);
    free(phi);
}

/* One time step (Eqs. 3, 4, 8): collide every fluid node, stream with
 * bounce-back at solids, then fill the open rows. */
static void step_once(o_sim *s)
{
    int nx = s->nx, ny = s->ny;
    double sF = o_pulse(&s->p, s->t);
    double q = s->q;
    compute_phi(s);

    /* collisions */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (s->wall[k]) continue;
            node_t nd;
            node_fields(s, x, y, sF, &nd);
            double fe[9], ge[5];
            feq(nd.n, nd.phi, nd.mu, nd.ux, nd.uy, fe);
            geq(nd.phi, nd.mu, nd.ux, nd.uy, s->p.gamma, q, ge);
            double pref = 1.0 - 1.0 / (2.0 * nd.tau);
            for (int i = 0; i < 9; i++) {
                double cu = CX[i] * nd.ux + CY[i] * nd.uy;
                /* Guo source of Eq. (4) */
                double vx = (CX[i] - nd.ux) + cu * CX[i] / CS2;
                double vy = (CY[i] - nd.uy) + cu * CY[i] / CS2;
                double Si = pref * WT[i] / CS2 * (vx * nd.Fx + vy * nd.Fy);
                s->fs[k * 9 + i] = s->f[k * 9 + i] + (fe[i] - s->f[k * 9 + i]) / nd.tau + Si;
            }
            for (int i = 0; i < 5; i++) {
                double gstar = s->g[k * 5 + i] + (ge[i] - s->g[k * 5 + i]) / s->p.tau_phi;
                s->h[k * 5 + i] = gstar - (1.0 - q) * s->g[k * 5 + i];
            }
        }

    /* streaming, pull form: every fluid destination collects from y - c_i */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (s->wall[k]) continue;
            for (int i = 0; i < 9; i++) {
                int xs, ys;
                if (!neighbour(s, x, y, -CX[i], -CY[i], &xs, &ys)) continue; /* open row: below */
                size_t ks = (size_t)ys * nx + xs;
                if (s->wall[ks]) {
                    /* halfway bounce-back */
                    s->fn[k * 9 + i] = s->fs[k * 9 + OPP[i]];
                    if (i < 5) s->gn[k * 5 + i] = s->h[k * 5 + OPP[i]] + (1.0 - q) * s->g[k * 5 + i];
                } else {
                    s->fn[k * 9 + i] = s->fs[ks * 9 + i];
                    if (i < 5) s->gn[k * 5 + i] = s->h[ks * 5 + i] + (1.0 - q) * s->g[k * 5 + i];
                }
            }
        }

    /* open rows: copy the unknown incoming populations from the adjacent row */
    if (s->p.bc_y == 1) {
        for (int x = 0; x < nx; x++) {
            size_t kb = (size_t)x, kb1 = (size_t)nx + x;
            size_t kt = (size_t)(ny - 1) * nx + x, kt1 = (size_t)(ny - 2) * nx + x;
            for (int i = 0; i < 9; i++) {
                if (CY[i] > 0 && !s->wall[kb]) {
                    s->fn[kb * 9 + i] = s->fn[kb1 * 9 + i];
                    if (i < 5) s->gn[kb * 5 + i] = s->gn[kb1 * 5 + i];
                }
                if (CY[i] < 0 && !s->wall[kt]) {
                    s->fn[kt * 9 + i] = s->fn[kt1 * 9 + i];
                    if (i < 5) s->gn[kt * 5 + i] = s->gn[kt1 * 5 + i];
                }
            }
        }
    }

    double *tmp = s->f;
    s->f = s->fn;
    s->fn = tmp;
    tmp = s->g;
    s->g = s->gn;
    s->gn = tmp;
    s->t += 1;
}

void o_step(o_sim *s, long nsteps)
{
    for (long k = 0; k < nsteps; k++) step_once(s);
}

long o_time(const o_sim *s) { return s->t; }

/* Fields at the current time (pre-collision state, current pulse value).
 * Each output is ny*nx doubles or NULL; solid nodes get 0, except
 * phi_tilde which holds the ghost there. */
void o_fields(o_sim *s, double *n, double *phi, double *ux, double *uy, double *phi_tilde,
              double *dphix, double *dphiy, double *lap, double *mu, double *Fx, double *Fy)
{
    int nx = s->nx, ny = s->ny;
    double sF = o_pulse(&s->p, s->t);
    compute_phi(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (phi_tilde) phi_tilde[k] = s->phi[k];
            node_t nd;
            memset(&nd, 0, sizeof nd);
            if (!s->wall[k]) node_fields(s, x, y, sF, &nd);
            if (n) n[k] = nd.n;
            if (phi) phi[k] = nd.phi;
            if (ux) ux[k] = nd.ux;
            if (uy) uy[k] = nd.uy;
            if (dphix) dphix[k] = nd.dphix;
            if (dphiy) dphiy[k] = nd.dphiy;
            if (lap) lap[k] = nd.lap;
            if (mu) mu[k] = nd.mu;
            if (Fx) Fx[k] = nd.Fx;
            if (Fy) Fy[k] = nd.Fy;
        }
}

/* State in structure-of-arrays order: f[i*N + y*nx + x], g[i*N + ...]. */
void o_get_state(const o_sim *s, double *f, double *g)
{
    size_t N = (size_t)s->nx * s->ny;
    for (size_t k = 0; k < N; k++) {
        for (int i = 0; i < 9; i++) f[i * N + k] = s->f[k * 9 + i];
        for (int i = 0; i < 5; i++) g[i * N + k] = s->g[k * 5 + i];
    }
}

void o_set_state(o_sim *s, const double *f, const double *g, long t)
{
    size_t N = (size_t)s->nx * s->ny;
    for (size_t k = 0; k < N; k++) {
        for (int i = 0; i < 9; i++) s->f[k * 9 + i] = s->wall[k] ? 0.0 : f[i * N + k];
        for (int i = 0; i < 5; i++) s->g[k * 5 + i] = s->wall[k] ? 0.0 : g[i * N + k];
    }
    s->t = t;
}

/* Diagnostic sums at the current time.
 *   rec[0] = sum n, rec[1] = sum phi, rec[2] = sum_x sum_i c_ix f_i,
 *   rec[3] = sum_x sum_i c_iy f_i, rec[4] = max |u|, rec[5] = count of fluid
 *   nodes with a non-finite n, phi or u.
 *   For rows y >= row0: row_count[y] = #{fluid x: phi > 0} (ink indicator),
 *   row_uy[y] = sum of u_y over those nodes.  Rows below row0 are zeroed. */
void o_diag(o_sim *s, long row0, double rec[6], int64_t *row_count, double *row_uy)
{
    int nx = s->nx, ny = s->ny;
    double sF = o_pulse(&s->p, s->t);
    compute_phi(s);
    double sn = 0, sp = 0, sjx = 0, sjy = 0, umax = 0, bad = 0;
    for (int y = 0; y < ny; y++) {
        int64_t cnt = 0;
        double suy = 0.0;
        for (int x = 0; x < nx; x++) {
            size_t k = (size_t)y * nx + x;
            if (s->wall[k]) continue;
            node_t nd;
            node_fields(s, x, y, sF, &nd);
            const double *f = s->f + k * 9;
            double jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; i++) {
                jx += CX[i] * f[i];
                jy += CY[i] * f[i];
            }
            sn += nd.n;
            sp += nd.phi;
            sjx += jx;
            sjy += jy;
            double um = sqrt(nd.ux * nd.ux + nd.uy * nd.uy);
            /* the stability guard's count: a non-finite value, or a density
             * that is not positive (n <= 0 has no meaning in Eq. 1) */
            if (!isfinite(nd.n) || !isfinite(nd.phi) || !isfinite(um) || !(nd.n > 0.0))
                bad += 1;
            else if (um > umax)
                umax = um;
            if (y >= row0 && nd.phi > 0.0) {
                cnt++;
                suy += nd.uy;
            }
        }
        row_count[y] = y >= row0 ? cnt : 0;
        row_uy[y] = y >= row0 ? suy : 0.0;
    }
    rec[0] = sn;
    rec[1] = sp;
    rec[2] = sjx;
    rec[3] = sjy;
    rec[4] = umax;
    rec[5] = bad;
}
