/*
 * lbm3d_oracle.c -- plain FP64 CPU oracle of the three-dimensional form of the
 * binary-fluid lattice Boltzmann update of He, Yang, Qin, Wen & Zhang
 * (arXiv:1702.04487), Methods, Eqs. (1)-(10), with the pulsed actuation of
 * Results, "Actuation modeling" (Fig. 1), and the wetting walls of
 * "Reproducing the experiment".  The paper works in two dimensions; this file
 * writes the same update on D3Q19 (f) and D3Q7 (g) so that a round nozzle
 * can be modelled.
 *
 * TEST INFRASTRUCTURE ONLY.  The slow, obviously-correct reference that the
 * GPU library's 3-D path is checked against.  Only the test-suite and the
 * CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no source, header, table or helper with the GPU library,
 * nor with the two-dimensional oracle.
 *
 * Storage: array of structures in double precision,
 *   f[((y*nz + z)*nx + x)*19 + i],  g[(...)*7 + i].
 * Lattice units dx = dt = 1, c_s^2 = 1/3.  Axes: x periodic (width), y the
 * jet direction (periodic or open rows), z periodic (depth).
 * Velocities: 0 rest; 1..6 = +x, +y, -x, -y, +z, -z (D3Q7 = 0..6);
 *   7..10 = (1,1,0) (-1,1,0) (-1,-1,0) (1,-1,0);
 *   11..14 = (1,0,1) (-1,0,1) (-1,0,-1) (1,0,-1);
 *   15..18 = (0,1,1) (0,-1,1) (0,-1,-1) (0,1,-1).
 * Weights 1/3, 1/18 (axes), 1/36 (edges).  Summed along any one axis they
 * give the D2Q9 weights 4/9, 1/9, 1/36 of Eq. (6), and D3Q7 gives D2Q5, so a
 * state that does not vary along that axis evolves exactly as the
 * two-dimensional update.
 *
 * Readings (the paper's two-dimensional readings carried to three
 * dimensions; each is listed in the design notes of the repository):
 *   mu = 4 beta phi (phi^2 - phi*^2) - kappa lap(phi), beta and kappa from
 *       sigma and W as in two dimensions (planar profile phi* tanh(2z/W));
 *   f equilibrium of Eqs. (5)-(6): w_i [A_i + n (3 c.u + 9/2 (c.u)^2 - 3/2 u^2)]
 *       with A_i = 3p off rest and A_0 = (n - 3p (1 - w_0)) / w_0 at rest,
 *       p = n/3 + phi mu, so that sum f = n and sum c c f = p I + n u u;
 *   g equilibrium of Eqs. (9)-(10) on D3Q7: g_0 = phi - 3 Gamma mu,
 *       g_i = Gamma mu / 2 + phi c_i.u / (2q) (moments phi, phi u / q,
 *       Gamma mu I);
 *   n u = sum_i c_i f_i + F/2; Guo source
 *       (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F;
 *   C = clamp((phi/phi* + 1)/2, 0, 1), tau_n = tau_amb + C (tau_ink - tau_amb);
 *   gradient and Laplacian: isotropic sums over the 18 D3Q19 neighbours,
 *       grad = 3 sum w_i c_i phi(x + c_i), lap = 6 sum w_i (phi(x + c_i) - phi);
 *   Eq. (8): new g_i(y) = h_i(y - c_i) + (1 - q) g_i(y), h = g* - (1-q) g;
 *   walls: halfway bounce-back; wetting ghost phi_s = mean of its fluid axis
 *       neighbours (the 12 edge neighbours if none) + 2 Omega phi* / W;
 *   open rows (y = 0 and y = ny-1): after streaming, unknown incoming
 *       populations are copied from the adjacent interior row, and the
 *       stencil mirrors phi across the open edge;
 *   driving force along +y on fluid nodes with y < force_rows, with the
 *       +F_pos / -F_neg / idle pulse of Fig. 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define QG 7

static const int CX[Q] = {0, 1, 0, -1, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, -1, 1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
static const double CS2 = 1.0 / 3.0;

static double weight(int i)
{
    int m = abs(CX[i]) + abs(CY[i]) + abs(CZ[i]);
    return m == 0 ? 1.0 / 3.0 : (m == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* opposite direction: the one with every component negated */
static int opposite(int i)
{
    for (int j = 0; j < Q; j++)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

typedef struct o3_params {
    int64_t nx, ny, nz;
    int64_t bc_y;          /* 0: periodic in y; 1: open rows at y = 0 and ny-1 */
    int64_t force_rows;    /* F_b acts on fluid nodes with y < force_rows */
    int64_t t_pos, t_neg, t_idle, periodic_pulse;
    double rho_ink, rho_amb, sigma, width, gamma;
    double tau_ink, tau_amb, tau_phi;
    double theta_inner, theta_outer; /* degrees, through the ink */
    double f_pos, f_neg;
} o3_params;

typedef struct o3_sim {
    o3_params p;
    int nx, ny, nz;
    size_t N;
    double phi_star, n0, beta, kappa, q;
    double wet[3];
    double w[Q];
    int opp[Q];
    uint8_t *wall;
    double *f, *g, *fs, *h, *fn, *gn, *phi;
    long t;
} o3_sim;

/* Cahn wetting with the phi^4 closure: Omega for a contact angle theta,
 * inverse of cos(theta) = [(1+Omega)^{3/2} - (1-Omega)^{3/2}]/2. */
static double omega_of_theta(double theta_deg)
{
    double th = theta_deg * M_PI / 180.0;
    double s = sin(th);
    double c = cos(acos(s * s) / 3.0);
    double mag = 2.0 * sqrt(c * (1.0 - c));
    if (theta_deg < 90.0) return mag;
    if (theta_deg > 90.0) return -mag;
    return 0.0;
}

double o3_pulse(const o3_params *p, long t)
{
    long period = (long)(p->t_pos + p->t_neg + p->t_idle);
    long tt = t;
    if (p->periodic_pulse && period > 0) tt = t % period;
    if (tt < p->t_pos) return p->f_pos;
    if (tt < p->t_pos + p->t_neg) return -p->f_neg;
    return 0.0;
}

static size_t node(const o3_sim *s, int x, int y, int z) { return ((size_t)y * s->nz + z) * s->nx + x; }

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Neighbour (x+dx, y+dy, z+dz) with x, z periodic; 0 when it lies beyond an
 * open row. */
static int neighbour(const o3_sim *s, int x, int y, int z, int dx, int dy, int dz, size_t *k)
{
    int b = y + dy;
    if (b < 0 || b >= s->ny) {
        if (s->p.bc_y == 0)
            b = wrap(b, s->ny);
        else
            return 0;
    }
    *k = node(s, wrap(x + dx, s->nx), b, wrap(z + dz, s->nz));
    return 1;
}

/* phi seen by a stencil: mirrored across an open row */
static double phi_stencil(const o3_sim *s, int x, int y, int z)
{
    if (y < 0 || y >= s->ny) {
        if (s->p.bc_y == 0)
            y = wrap(y, s->ny);
        else
            y = y < 0 ? 0 : s->ny - 1;
    }
    return s->phi[node(s, wrap(x, s->nx), y, wrap(z, s->nz))];
}

/* phi = sum_i g_i at fluid nodes, then the wetting ghost at every solid node
 * that touches fluid (axis neighbours first, edge neighbours if none). */
static void compute_phi(o3_sim *s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int z = 0; z < nz; z++)
            for (int x = 0; x < nx; x++) {
                size_t k = node(s, x, y, z);
                if (s->wall[k]) continue;
                double sum = 0.0;
                for (int i = 0; i < QG; i++) sum += s->g[k * QG + i];
                s->phi[k] = sum;
            }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int z = 0; z < nz; z++)
            for (int x = 0; x < nx; x++) {
                size_t k = node(s, x, y, z);
                if (!s->wall[k]) continue;
                double sum = 0.0;
                int cnt = 0;
                for (int pass = 0; pass < 2 && cnt == 0; pass++) {
                    int i0 = pass == 0 ? 1 : 7, i1 = pass == 0 ? 7 : Q;
                    for (int i = i0; i < i1; i++) {
                        size_t kn;
                        if (!neighbour(s, x, y, z, CX[i], CY[i], CZ[i], &kn)) continue;
                        if (s->wall[kn]) continue;
                        sum += s->phi[kn];
                        cnt++;
                    }
                }
                s->phi[k] = cnt ? sum / cnt + s->wet[s->wall[k]] : 0.0;
            }
}

typedef struct {
    double n, phi, lap, mu, F[3], u[3], tau;
} node3_t;

static void node_fields(const o3_sim *s, int x, int y, int z, double sF, node3_t *o)
{
    size_t k = node(s, x, y, z);
    const double *f = s->f + k * Q;
    double ph = s->phi[k];
    double gr[3] = {0.0, 0.0, 0.0}, lap = 0.0;
    for (int i = 1; i < Q; i++) {
        double pn = phi_stencil(s, x + CX[i], y + CY[i], z + CZ[i]);
        gr[0] += s->w[i] * CX[i] * pn / CS2;
        gr[1] += s->w[i] * CY[i] * pn / CS2;
        gr[2] += s->w[i] * CZ[i] * pn / CS2;
        lap += 2.0 * s->w[i] * (pn - ph) / CS2;
    }
    double mu = 4.0 * s->beta * ph * (ph * ph - s->phi_star * s->phi_star) - s->kappa * lap;
    double F[3] = {mu * gr[0], mu * gr[1], mu * gr[2]};
    if (y < s->p.force_rows) F[1] += sF;
    double n = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        n += f[i];
        j[0] += CX[i] * f[i];
        j[1] += CY[i] * f[i];
        j[2] += CZ[i] * f[i];
    }
    double C = (ph / s->phi_star + 1.0) * 0.5;
    if (C < 0.0) C = 0.0;
    if (C > 1.0) C = 1.0;
    o->n = n;
    o->phi = ph;
    o->lap = lap;
    o->mu = mu;
    for (int a = 0; a < 3; a++) {
        o->F[a] = F[a];
        o->u[a] = (j[a] + 0.5 * F[a]) / n;
    }
    o->tau = s->p.tau_amb + C * (s->p.tau_ink - s->p.tau_amb);
}

static double cdotu(int i, const double u[3]) { return CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2]; }

static void feq(const o3_sim *s, double n, double phi, double mu, const double u[3], double out[Q])
{
    double p = n / 3.0 + phi * mu;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; i++) {
        double A = i == 0 ? (n - 3.0 * p * (1.0 - s->w[0])) / s->w[0] : 3.0 * p;
        double cu = cdotu(i, u);
        out[i] = s->w[i] * A + s->w[i] * n * (3.0 * cu - 1.5 * uu + 4.5 * cu * cu);
    }
}

static void geq(const o3_sim *s, double phi, double mu, const double u[3], double out[QG])
{
    for (int i = 0; i < QG; i++) {
        if (i == 0)
            out[i] = phi - 3.0 * s->p.gamma * mu;
        else
            out[i] = 0.5 * s->p.gamma * mu + phi * cdotu(i, u) / (2.0 * s->q);
    }
}

/* ------------------------------------------------------------ public API */

void o3_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* wall: ny*nz*nx bytes (0 fluid, 1 inner wall, 2 outer wall) */
o3_sim *o3_create(const o3_params *p, const uint8_t *wall, int *err)
{
    *err = 0;
    if (p->nx < 3 || p->ny < 3 || p->nz < 3 || p->tau_ink <= 0.5 || p->tau_amb <= 0.5 || p->tau_phi <= 0.5 ||
        p->width <= 0.0 || p->rho_ink <= p->rho_amb || p->rho_amb <= 0.0 || p->sigma < 0.0) {
        *err = 1;
        return NULL;
    }
    o3_sim *s = (o3_sim *)calloc(1, sizeof(o3_sim));
    s->p = *p;
    s->nx = (int)p->nx;
    s->ny = (int)p->ny;
    s->nz = (int)p->nz;
    s->N = (size_t)s->nx * s->ny * s->nz;
    for (size_t k = 0; k < s->N; k++)
        if (wall[k] > 2) *err = 3;
    if (p->bc_y == 1)
        for (int z = 0; z < s->nz; z++)
            for (int x = 0; x < s->nx; x++) {
                if (!wall[node(s, x, 0, z)] && wall[node(s, x, 1, z)]) *err = 2;
                if (!wall[node(s, x, s->ny - 1, z)] && wall[node(s, x, s->ny - 2, z)]) *err = 2;
            }
    if (*err) {
        free(s);
        return NULL;
    }
    for (int i = 0; i < Q; i++) {
        s->w[i] = weight(i);
        s->opp[i] = opposite(i);
    }
    s->phi_star = 0.5 * (p->rho_ink - p->rho_amb);
    s->n0 = 0.5 * (p->rho_ink + p->rho_amb);
    double ps2 = s->phi_star * s->phi_star;
    s->beta = 3.0 * p->sigma / (4.0 * p->width * ps2 * ps2);
    s->kappa = 3.0 * p->sigma * p->width / (8.0 * ps2);
    s->q = 1.0 / (p->tau_phi + 0.5);
    s->wet[0] = 0.0;
    s->wet[1] = 2.0 * omega_of_theta(p->theta_inner) * s->phi_star / p->width;
    s->wet[2] = 2.0 * omega_of_theta(p->theta_outer) * s->phi_star / p->width;
    s->wall = (uint8_t *)malloc(s->N);
    memcpy(s->wall, wall, s->N);
    s->f = (double *)calloc(s->N * Q, sizeof(double));
    s->fs = (double *)calloc(s->N * Q, sizeof(double));
    s->fn = (double *)calloc(s->N * Q, sizeof(double));
    s->g = (double *)calloc(s->N * QG, sizeof(double));
    s->h = (double *)calloc(s->N * QG, sizeof(double));
    s->gn = (double *)calloc(s->N * QG, sizeof(double));
    s->phi = (double *)calloc(s->N, sizeof(double));
    return s;
}

void o3_destroy(o3_sim *s)
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

/* phi*, n0, beta, kappa, q, inner and outer ghost offsets */
void o3_derived(const o3_sim *s, double out[7])
{
    out[0] = s->phi_star;
    out[1] = s->n0;
    out[2] = s->beta;
    out[3] = s->kappa;
    out[4] = s->q;
    out[5] = s->wet[1];
    out[6] = s->wet[2];
}

/* The velocity set, for tests: c[i*3 + a], w[i], opp[i]. */
void o3_velocity_set(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; i++) {
        c[i * 3 + 0] = CX[i];
        c[i * 3 + 1] = CY[i];
        c[i * 3 + 2] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Initial state from phi (N values; solid entries ignored) and an optional
 * velocity (NULL = 0): n = n0, f = f_eq, g = g_eq with mu from the initial
 * phi including the wetting ghosts. */
void o3_init_phi(o3_sim *s, const double *phi, const double *ux, const double *uy, const double *uz)
{
    memset(s->f, 0, s->N * Q * sizeof(double));
    memset(s->g, 0, s->N * QG * sizeof(double));
    for (size_t k = 0; k < s->N; k++)
        if (!s->wall[k]) {
            s->g[k * QG] = phi[k];
            s->f[k * Q] = s->n0;
        }
    compute_phi(s);
    for (int y = 0; y < s->ny; y++)
        for (int z = 0; z < s->nz; z++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = node(s, x, y, z);
                if (s->wall[k]) continue;
                node3_t nd;
                node_fields(s, x, y, z, 0.0, &nd);
                double u[3] = {ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, uz ? uz[k] : 0.0};
                feq(s, s->n0, nd.phi, nd.mu, u, s->fn + k * Q);
                geq(s, nd.phi, nd.mu, u, s->gn + k * QG);
            }
    memcpy(s->f, s->fn, s->N * Q * sizeof(double));
    memcpy(s->g, s->gn, s->N * QG * sizeof(double));
    memset(s->fn, 0, s->N * Q * sizeof(double));
    memset(s->gn, 0, s->N * QG * sizeof(double));
    s->t = 0;
}

/* One step: collide every fluid node (Eqs. 4, 8), pull-stream with
 * halfway bounce-back, then fill the open rows. */
static void step_once(o3_sim *s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const double sF = o3_pulse(&s->p, s->t), q = s->q;
    compute_phi(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int z = 0; z < nz; z++)
            for (int x = 0; x < nx; x++) {
                size_t k = node(s, x, y, z);
                if (s->wall[k]) continue;
                node3_t nd;
                node_fields(s, x, y, z, sF, &nd);
                double fe[Q], ge[QG];
                feq(s, nd.n, nd.phi, nd.mu, nd.u, fe);
                geq(s, nd.phi, nd.mu, nd.u, ge);
                double pref = 1.0 - 1.0 / (2.0 * nd.tau);
                for (int i = 0; i < Q; i++) {
                    double cu = cdotu(i, nd.u);
                    double v0 = (CX[i] - nd.u[0]) + cu * CX[i] / CS2;
                    double v1 = (CY[i] - nd.u[1]) + cu * CY[i] / CS2;
                    double v2 = (CZ[i] - nd.u[2]) + cu * CZ[i] / CS2;
                    double Si = pref * s->w[i] / CS2 * (v0 * nd.F[0] + v1 * nd.F[1] + v2 * nd.F[2]);
                    s->fs[k * Q + i] = s->f[k * Q + i] + (fe[i] - s->f[k * Q + i]) / nd.tau + Si;
                }
                for (int i = 0; i < QG; i++) {
                    double gstar = s->g[k * QG + i] + (ge[i] - s->g[k * QG + i]) / s->p.tau_phi;
                    s->h[k * QG + i] = gstar - (1.0 - q) * s->g[k * QG + i];
                }
            }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int z = 0; z < nz; z++)
            for (int x = 0; x < nx; x++) {
                size_t k = node(s, x, y, z);
                if (s->wall[k]) continue;
                for (int i = 0; i < Q; i++) {
                    size_t ks;
                    if (!neighbour(s, x, y, z, -CX[i], -CY[i], -CZ[i], &ks)) continue;
                    if (s->wall[ks]) {
                        s->fn[k * Q + i] = s->fs[k * Q + s->opp[i]];
                        if (i < QG) s->gn[k * QG + i] = s->h[k * QG + s->opp[i]] + (1.0 - q) * s->g[k * QG + i];
                    } else {
                        s->fn[k * Q + i] = s->fs[ks * Q + i];
                        if (i < QG) s->gn[k * QG + i] = s->h[ks * QG + i] + (1.0 - q) * s->g[k * QG + i];
                    }
                }
            }
    if (s->p.bc_y == 1)
        for (int z = 0; z < nz; z++)
            for (int x = 0; x < nx; x++) {
                size_t kb = node(s, x, 0, z), kb1 = node(s, x, 1, z);
                size_t kt = node(s, x, ny - 1, z), kt1 = node(s, x, ny - 2, z);
                for (int i = 0; i < Q; i++) {
                    if (CY[i] > 0 && !s->wall[kb]) {
                        s->fn[kb * Q + i] = s->fn[kb1 * Q + i];
                        if (i < QG) s->gn[kb * QG + i] = s->gn[kb1 * QG + i];
                    }
                    if (CY[i] < 0 && !s->wall[kt]) {
                        s->fn[kt * Q + i] = s->fn[kt1 * Q + i];
                        if (i < QG) s->gn[kt * QG + i] = s->gn[kt1 * QG + i];
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

void o3_step(o3_sim *s, long nsteps)
{
    for (long k = 0; k < nsteps; k++) step_once(s);
}

long o3_time(const o3_sim *s) { return s->t; }

/* Fields of the current state (N doubles each, NULL = skip); solid nodes
 * read 0 except phi_tilde, which holds the ghost there. */
void o3_fields(o3_sim *s, double *n, double *phi, double *ux, double *uy, double *uz, double *phi_tilde,
               double *mu)
{
    const double sF = o3_pulse(&s->p, s->t);
    compute_phi(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < s->ny; y++)
        for (int z = 0; z < s->nz; z++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = node(s, x, y, z);
                node3_t nd;
                memset(&nd, 0, sizeof nd);
                if (!s->wall[k]) node_fields(s, x, y, z, sF, &nd);
                if (n) n[k] = nd.n;
                if (phi) phi[k] = nd.phi;
                if (ux) ux[k] = nd.u[0];
                if (uy) uy[k] = nd.u[1];
                if (uz) uz[k] = nd.u[2];
                if (phi_tilde) phi_tilde[k] = s->phi[k];
                if (mu) mu[k] = nd.mu;
            }
}

/* State as structure of arrays: f[i*N + k], g[i*N + k]. */
void o3_get_state(const o3_sim *s, double *f, double *g)
{
    for (size_t k = 0; k < s->N; k++) {
        for (int i = 0; i < Q; i++) f[i * s->N + k] = s->f[k * Q + i];
        for (int i = 0; i < QG; i++) g[i * s->N + k] = s->g[k * QG + i];
    }
}

void o3_set_state(o3_sim *s, const double *f, const double *g, long t)
{
    for (size_t k = 0; k < s->N; k++) {
        for (int i = 0; i < Q; i++) s->f[k * Q + i] = s->wall[k] ? 0.0 : f[i * s->N + k];
        for (int i = 0; i < QG; i++) s->g[k * QG + i] = s->wall[k] ? 0.0 : g[i * s->N + k];
    }
    s->t = t;
}

/* Diagnostic sums of the current state.
 *   rec = {sum n, sum phi, sum_x sum_i c_ix f_i, ... c_iy ..., ... c_iz ...,
 *          max |u|, fluid nodes with a non-finite n, phi or u}.
 *   For rows (x-z slices) y >= row0: row_count[y] = #{fluid nodes: phi > 0},
 *   row_uy[y] = sum of u_y over them; rows below row0 read 0. */
void o3_diag(o3_sim *s, long row0, double rec[7], int64_t *row_count, double *row_uy)
{
    const double sF = o3_pulse(&s->p, s->t);
    compute_phi(s);
    double sn = 0, sp = 0, sj[3] = {0, 0, 0}, umax = 0, bad = 0;
    for (int y = 0; y < s->ny; y++) {
        int64_t cnt = 0;
        double suy = 0.0;
        for (int z = 0; z < s->nz; z++)
            for (int x = 0; x < s->nx; x++) {
                size_t k = node(s, x, y, z);
                if (s->wall[k]) continue;
                node3_t nd;
                node_fields(s, x, y, z, sF, &nd);
                const double *f = s->f + k * Q;
                for (int i = 0; i < Q; i++) {
                    sj[0] += CX[i] * f[i];
                    sj[1] += CY[i] * f[i];
                    sj[2] += CZ[i] * f[i];
                }
                sn += nd.n;
                sp += nd.phi;
                double um = sqrt(nd.u[0] * nd.u[0] + nd.u[1] * nd.u[1] + nd.u[2] * nd.u[2]);
                /* non-finite, or a density that is not positive */
                if (!isfinite(nd.n) || !isfinite(nd.phi) || !isfinite(um) || !(nd.n > 0.0))
                    bad += 1;
                else if (um > umax)
                    umax = um;
                if (y >= row0 && nd.phi > 0.0) {
                    cnt++;
                    suy += nd.u[1];
                }
            }
        row_count[y] = y >= row0 ? cnt : 0;
        row_uy[y] = y >= row0 ? suy : 0.0;
    }
    rec[0] = sn;
    rec[1] = sp;
    rec[2] = sj[0];
    rec[3] = sj[1];
    rec[4] = sj[2];
    rec[5] = umax;
    rec[6] = bad;
}
