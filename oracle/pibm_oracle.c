/*
 * pibm_oracle.c -- plain FP64 CPU oracle of the coupled thermal LBM-PIBM-DEM
 * time step of Zhang, Yuan, Trias, Yu, Tan & Oliva, "Particulate immersed
 * boundary method for complex fluid-particle interaction problems with heat
 * transfer" (arXiv 1502.01159).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Nothing in the product
 * path may include, link or call it; it shares no code, header, table or
 * constant with the HIP library.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * Everything is double precision, lattice units (h = dt = c = 1, rho0 = 1),
 * array-of-structures (population index fastest), plain loops in the order the
 * paper states the method:
 *
 *   1. stream (pull) with halfway bounce-back / anti-bounce-back walls
 *      -- Sec. 2.1, Eqs. (lbm2), (lbm2.5);
 *   2. raw moments rho = sum f, j = sum e f, S = sum g        -- Sec. 2.1;
 *   3. Lagrange interpolation of rho, j, S to the Lagrangian points
 *      -- Sec. 2.2, Eqs. (lbm5), (lbm5.5), (lbm6) with i_max = 2 (or 4);
 *   4. point exchange F_l = 2(rho_l U_l - j_l), Q_l = 2 kappa (T_p - T_l)
 *      -- Sec. 2.2, Eqs. (lbm7), (lbm7.5), (lbm8) summed over directions;
 *   5. per-particle reactions  F = -sum F_l A_l, tau = -sum r x F_l A_l,
 *      H = sum Q_l A_l                                     -- Eq. (lbm13);
 *   6. spreading with the cosine kernel  -- Eqs. (lbm10), (lbm11), (lbm12),
 *      (lbm12.6);
 *   7. BGK collision with Guo forcing and heat source, buoyancy
 *      -- Eqs. (lbm2), (lbm2.5), (lbm3), (lbm9), (lbm12.5) and the moment
 *      definitions after (lbm3.5);
 *   8. DEM: Newton-Euler with Hertz normal and Mindlin-Deresiewicz tangential
 *      contact, n_sub semi-implicit Euler sub-steps   -- Sec. 2.3, Eq. (demgov);
 *   9. lumped heat balance of thermosensitive particles  -- Sec. 3.4.
 *
 * The readings of the garbled or silent passages are listed in the design
 * notes; each is marked "reading:" where it is used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Public parameter block (mirrored by oracle/oracle.py as a ctypes struct).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim, nx, ny, nz;
    int periodic[3];
    double T_wall[6];        /* faces -x,+x,-y,+y,-z,+z */
    double T_init, T_ref;
    double tau_f, tau_g;     /* relaxation times (already derived) */
    double gbeta;            /* Boussinesq coefficient g*beta in lattice units */
    double gravity;          /* particle gravity magnitude, along -e_up */
    double kappa_T;          /* thermal exchange prefactor */
    double E_star, poisson, mu_fric;
    int n_sub;
    double beta_p, c_r;      /* thermosensitive density slope, heat-capacity ratio */
    int marker_mode;         /* 0 surface element, 1 A = pi s^2/4, 2 one point */
    double marker_spacing;
    int interp_order;        /* Lagrange nodes per axis in Eq. (lbm6): 2 (0 means 2) or 4 */
    int lattice;             /* 3D flow velocity set: 19 (0 means 19) or 15 (Sec. 2.1's D3Q15) */
    int thermal_model;       /* 0: D2Q5 / D3Q7, linear g^eq; 1: the flow lattice, quadratic g^eq */
} orc_params;

enum { ORC_FIXED = 1, ORC_THERMO = 2 };

#define ORC_MAX_CONTACTS 64

typedef struct {
    int partner;           /* particle index, or -1-face for a wall */
    double xi[3];          /* tangential spring displacement */
} orc_contact;

typedef struct {
    double x[3], u[3], om[3], th[3];
    double R, rho_r, T;
    int flags;
    int nm;                /* number of Lagrangian points */
    double *off;           /* nm*3 offsets r_k from the centre */
    double *area;          /* nm weights A_k */
    int nc;
    orc_contact c[ORC_MAX_CONTACTS];
    double F[3], tq[3], H, dTA;   /* last step's reactions */
} orc_particle;

typedef struct {
    orc_params p;
    int Q, Qg;
    int e[19][3], eg[19][3];
    double w[19], wg[19], csg2;
    int opp[19], oppg[19];
    long N;
    double *f, *g;           /* post-collision populations, [node][q] */
    double *fs, *gs;         /* scratch: post-stream populations */
    double *rho, *j, *S;     /* raw post-stream moments */
    double *FB, *QB;         /* spread force [node][3] and heat source */
    int np;
    orc_particle *pt;
    long step;
    int error;
} orc_state;

/* ------------------------------------------------------------------------ */
/* Lattices.  D2Q9 / D3Q19 for the flow, or the D3Q15 of Sec. 2.1 (rest,    */
/* six faces, eight corners; w = 2/9, 1/9, 1/72); D2Q5 / D3Q7 for           */
/* temperature (reading: linear equilibrium, c_sg^2 = 1/3 in 2D, 1/4 in 3D). */
/* ------------------------------------------------------------------------ */
static void set_lattice(orc_state *s)
{
    static const int d2q9[9][2] = {{0,0},{1,0},{0,1},{-1,0},{0,-1},{1,1},{-1,1},{-1,-1},{1,-1}};
    static const int d3q19[19][3] = {
        {0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},
        {1,1,0},{-1,-1,0},{1,-1,0},{-1,1,0},{1,0,1},{-1,0,-1},{1,0,-1},{-1,0,1},
        {0,1,1},{0,-1,-1},{0,1,-1},{0,-1,1}};
    static const int d3q15[15][3] = {
        {0,0,0},{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1},
        {1,1,1},{-1,-1,-1},{1,1,-1},{-1,-1,1},{1,-1,1},{-1,1,-1},{-1,1,1},{1,-1,-1}};
    memset(s->e, 0, sizeof s->e);
    memset(s->eg, 0, sizeof s->eg);
    if (s->p.dim == 2) {
        s->Q = 9; s->Qg = 5;
        for (int a = 0; a < 9; a++) { s->e[a][0] = d2q9[a][0]; s->e[a][1] = d2q9[a][1]; }
        for (int a = 0; a < 9; a++) {
            int n2 = s->e[a][0]*s->e[a][0] + s->e[a][1]*s->e[a][1];
            s->w[a] = n2 == 0 ? 4.0/9.0 : (n2 == 1 ? 1.0/9.0 : 1.0/36.0);
        }
        for (int a = 0; a < 5; a++) {
            s->eg[a][0] = d2q9[a][0]; s->eg[a][1] = d2q9[a][1];
            s->wg[a] = a == 0 ? 1.0/3.0 : 1.0/6.0;
        }
        s->csg2 = 1.0/3.0;
    } else if (s->p.lattice == 15) {
        s->Q = 15; s->Qg = 7;
        for (int a = 0; a < 15; a++) {
            for (int d = 0; d < 3; d++) s->e[a][d] = d3q15[a][d];
            int n2 = s->e[a][0]*s->e[a][0] + s->e[a][1]*s->e[a][1] + s->e[a][2]*s->e[a][2];
            s->w[a] = n2 == 0 ? 2.0/9.0 : (n2 == 1 ? 1.0/9.0 : 1.0/72.0);
        }
        for (int a = 0; a < 7; a++) {
            for (int d = 0; d < 3; d++) s->eg[a][d] = d3q19[a][d];
            s->wg[a] = a == 0 ? 1.0/4.0 : 1.0/8.0;
        }
        s->csg2 = 1.0/4.0;
    } else {
        s->Q = 19; s->Qg = 7;
        for (int a = 0; a < 19; a++) {
            for (int d = 0; d < 3; d++) s->e[a][d] = d3q19[a][d];
            int n2 = s->e[a][0]*s->e[a][0] + s->e[a][1]*s->e[a][1] + s->e[a][2]*s->e[a][2];
            s->w[a] = n2 == 0 ? 1.0/3.0 : (n2 == 1 ? 1.0/18.0 : 1.0/36.0);
        }
        for (int a = 0; a < 7; a++) {
            for (int d = 0; d < 3; d++) s->eg[a][d] = d3q19[a][d];
            s->wg[a] = a == 0 ? 1.0/4.0 : 1.0/8.0;
        }
        s->csg2 = 1.0/4.0;
    }
    if (s->p.thermal_model == 1) {
        /* Sec. 2.1 as printed: temperature on the flow lattice with the same
         * weights and c_s^2 = 1/3 (its equilibrium is quadratic, see geq) */
        s->Qg = s->Q;
        for (int a = 0; a < s->Q; a++) {
            for (int d = 0; d < 3; d++) s->eg[a][d] = s->e[a][d];
            s->wg[a] = s->w[a];
        }
        s->csg2 = 1.0/3.0;
    }
    for (int a = 0; a < s->Q; a++)
        for (int b = 0; b < s->Q; b++)
            if (s->e[b][0] == -s->e[a][0] && s->e[b][1] == -s->e[a][1] && s->e[b][2] == -s->e[a][2])
                s->opp[a] = b;
    for (int a = 0; a < s->Qg; a++)
        for (int b = 0; b < s->Qg; b++)
            if (s->eg[b][0] == -s->eg[a][0] && s->eg[b][1] == -s->eg[a][1] && s->eg[b][2] == -s->eg[a][2])
                s->oppg[a] = b;
}

static int nsz(const orc_state *s, int d) { return d == 0 ? s->p.nx : (d == 1 ? s->p.ny : s->p.nz); }

static long node_index(const orc_state *s, int i, int j, int k)
{
    return ((long)k * s->p.ny + j) * s->p.nx + i;
}

/* Map a lattice coordinate on axis d: wrap on periodic axes; return -1 when
 * the coordinate lies outside a wall. */
static int map_coord(const orc_state *s, int d, int c)
{
    int n = nsz(s, d);
    if (s->p.periodic[d]) { c %= n; if (c < 0) c += n; return c; }
    return (c < 0 || c >= n) ? -1 : c;
}

/* Clamp (walls) or wrap (periodic) for the interpolation stencil. */
static int clamp_coord(const orc_state *s, int d, int c)
{
    int n = nsz(s, d);
    if (s->p.periodic[d]) { c %= n; if (c < 0) c += n; return c; }
    if (c < 0) return 0;
    if (c >= n) return n - 1;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Lagrangian point templates.                                               */
/*   2D: ring of N = round(pi D / s) points at angles 2 pi k / N.            */
/*   3D: Fibonacci sphere of N = round(pi D^2 / s^2) points.                 */
/* Weights: surface element pi D / N or pi D^2 / N (marker_mode 0); the     */
/* paper's cross-section of a Lagrangian particle of diameter d = s          */
/* (mode 1): A_p = pi d^2 / 4 in 3D, A_p = d per unit depth in 2D (Sec. 2.2,  */
/* after Eq. lbm12.6); or one point at the centre carrying the body's own    */
/* cross-section (mode 2, the sub-grid particle of Sec. 2.2).                */
/* ------------------------------------------------------------------------ */
static void make_markers(const orc_state *s, orc_particle *q)
{
    const double pi = 3.14159265358979323846;
    int mode = s->p.marker_mode;
    double sp = s->p.marker_spacing > 0 ? s->p.marker_spacing : 1.0;
    double D = 2.0 * q->R;
    if (mode == 2) {
        q->nm = 1;
        q->off = calloc(3, sizeof(double));
        q->area = malloc(sizeof(double));
        q->area[0] = s->p.dim == 2 ? D : 0.25 * pi * D * D;
        return;
    }
    int n;
    if (s->p.dim == 2) n = (int)lround(pi * D / sp);
    else n = (int)lround(pi * D * D / (sp * sp));
    if (n < 1) n = 1;
    q->nm = n;
    q->off = calloc((size_t)n * 3, sizeof(double));
    q->area = malloc((size_t)n * sizeof(double));
    double golden = pi * (3.0 - sqrt(5.0));
    for (int k = 0; k < n; k++) {
        if (s->p.dim == 2) {
            double th = 2.0 * pi * k / n;
            q->off[3*k+0] = q->R * cos(th);
            q->off[3*k+1] = q->R * sin(th);
            q->off[3*k+2] = 0.0;
            q->area[k] = mode == 0 ? pi * D / n : sp;
        } else {
            double z = 1.0 - (2.0 * k + 1.0) / n;
            double rr = sqrt(1.0 - z * z);
            double ph = k * golden;
            q->off[3*k+0] = q->R * rr * cos(ph);
            q->off[3*k+1] = q->R * rr * sin(ph);
            q->off[3*k+2] = q->R * z;
            q->area[k] = mode == 0 ? pi * D * D / n : 0.25 * pi * sp * sp;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibria and sources.                                                   */
/* ------------------------------------------------------------------------ */
/* Eq. (lbm3). */
static double feq(const orc_state *s, int a, double rho, const double u[3])
{
    double eu = s->e[a][0]*u[0] + s->e[a][1]*u[1] + s->e[a][2]*u[2];
    double uu = u[0]*u[0] + u[1]*u[1] + u[2]*u[2];
    return rho * s->w[a] * (1.0 + 3.0*eu + 4.5*eu*eu - 1.5*uu);
}

/* Thermal equilibrium on the D2Q5 / D3Q7 lattice (reading: linear in u). */
static double geq(const orc_state *s, int a, double T, const double u[3])
{
    double eu = s->eg[a][0]*u[0] + s->eg[a][1]*u[1] + s->eg[a][2]*u[2];
    if (s->p.thermal_model == 1) {
        /* the flow's equilibrium form with T in place of rho (Sec. 2.1) */
        double uu = u[0]*u[0] + u[1]*u[1] + u[2]*u[2];
        return s->wg[a] * T * (1.0 + 3.0*eu + 4.5*eu*eu - 1.5*uu);
    }
    return s->wg[a] * T * (1.0 + eu / s->csg2);
}

/* Guo forcing, Eq. (lbm9), with the total force F (reading: buoyancy
 * included, so that u and the momentum source agree). */
static double guo(const orc_state *s, int a, const double u[3], const double F[3])
{
    double eu = s->e[a][0]*u[0] + s->e[a][1]*u[1] + s->e[a][2]*u[2];
    double acc = 0.0;
    for (int d = 0; d < 3; d++)
        acc += (3.0 * (s->e[a][d] - u[d]) + 9.0 * eu * s->e[a][d]) * F[d];
    return (1.0 - 0.5 / s->p.tau_f) * s->w[a] * acc;
}

/* Cosine kernel, Eq. (lbm12). */
double orc_delta_h(double a)
{
    const double pi = 3.14159265358979323846;
    if (fabs(a) > 2.0) return 0.0;
    return 0.25 * (1.0 + cos(0.5 * pi * a));
}

/* ------------------------------------------------------------------------ */
/* Creation / destruction / state access.                                    */
/* ------------------------------------------------------------------------ */
/* pdata per particle: x[3] u[3] om[3] R rho_r T flags  (13 doubles). */
orc_state *orc_create(const orc_params *p, int np, const double *pdata)
{
    orc_state *s = calloc(1, sizeof *s);
    s->p = *p;
    if (s->p.dim == 2) s->p.nz = 1;
    set_lattice(s);
    s->N = (long)s->p.nx * s->p.ny * s->p.nz;
    s->f = malloc(sizeof(double) * s->N * s->Q);
    s->g = malloc(sizeof(double) * s->N * s->Qg);
    s->fs = malloc(sizeof(double) * s->N * s->Q);
    s->gs = malloc(sizeof(double) * s->N * s->Qg);
    s->rho = malloc(sizeof(double) * s->N);
    s->j = malloc(sizeof(double) * s->N * 3);
    s->S = malloc(sizeof(double) * s->N);
    s->FB = malloc(sizeof(double) * s->N * 3);
    s->QB = malloc(sizeof(double) * s->N);
    /* Initial state: f = w rho0, g = w T_init (u = 0). */
    for (long n = 0; n < s->N; n++) {
        for (int a = 0; a < s->Q; a++) s->f[n*s->Q + a] = s->w[a];
        for (int a = 0; a < s->Qg; a++) s->g[n*s->Qg + a] = s->wg[a] * s->p.T_init;
    }
    s->np = np;
    s->pt = calloc(np > 0 ? np : 1, sizeof(orc_particle));
    for (int i = 0; i < np; i++) {
        const double *d = pdata + 13 * (long)i;
        orc_particle *q = &s->pt[i];
        for (int c = 0; c < 3; c++) { q->x[c] = d[c]; q->u[c] = d[3+c]; q->om[c] = d[6+c]; }
        q->R = d[9]; q->rho_r = d[10]; q->T = d[11]; q->flags = (int)d[12];
        make_markers(s, q);
    }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    for (int i = 0; i < s->np; i++) { free(s->pt[i].off); free(s->pt[i].area); }
    free(s->pt);
    free(s->f); free(s->g); free(s->fs); free(s->gs);
    free(s->rho); free(s->j); free(s->S); free(s->FB); free(s->QB);
    free(s);
}

long orc_num_nodes(const orc_state *s) { return s->N; }
int orc_num_markers(const orc_state *s, int i) { return s->pt[i].nm; }
int orc_error(const orc_state *s) { return s->error; }
long orc_step_count(const orc_state *s) { return s->step; }

/* Populations are exchanged as [q][node] (q slowest) to keep the Python side
 * simple; internally they are [node][q]. */
void orc_get_populations(const orc_state *s, double *f, double *g)
{
    for (long n = 0; n < s->N; n++) {
        for (int a = 0; a < s->Q; a++) f[a * s->N + n] = s->f[n*s->Q + a];
        for (int a = 0; a < s->Qg; a++) g[a * s->N + n] = s->g[n*s->Qg + a];
    }
}

void orc_set_populations(orc_state *s, const double *f, const double *g)
{
    for (long n = 0; n < s->N; n++) {
        for (int a = 0; a < s->Q; a++) s->f[n*s->Q + a] = f[a * s->N + n];
        for (int a = 0; a < s->Qg; a++) s->g[n*s->Qg + a] = g[a * s->N + n];
    }
}

/* Per particle 16 doubles: x[3] u[3] om[3] th[3] R rho_r T flags. */
void orc_get_particles(const orc_state *s, double *out)
{
    for (int i = 0; i < s->np; i++) {
        const orc_particle *q = &s->pt[i];
        double *o = out + 16 * (long)i;
        for (int c = 0; c < 3; c++) { o[c] = q->x[c]; o[3+c] = q->u[c]; o[6+c] = q->om[c]; o[9+c] = q->th[c]; }
        o[12] = q->R; o[13] = q->rho_r; o[14] = q->T; o[15] = q->flags;
    }
}

/* pdata as in orc_create; keeps markers and contact history. */
void orc_set_particles(orc_state *s, const double *pdata)
{
    for (int i = 0; i < s->np; i++) {
        const double *d = pdata + 13 * (long)i;
        orc_particle *q = &s->pt[i];
        for (int c = 0; c < 3; c++) { q->x[c] = d[c]; q->u[c] = d[3+c]; q->om[c] = d[6+c]; }
        q->rho_r = d[10]; q->T = d[11]; q->flags = (int)d[12];
    }
}

/* Per particle 8 doubles: F[3] tau[3] H sum_l (T_p - T_l) A_l. */
void orc_get_reactions(const orc_state *s, double *out)
{
    for (int i = 0; i < s->np; i++) {
        const orc_particle *q = &s->pt[i];
        double *o = out + 8 * (long)i;
        for (int c = 0; c < 3; c++) { o[c] = q->F[c]; o[3+c] = q->tq[c]; }
        o[6] = q->H; o[7] = q->dTA;
    }
}

/* Lagrangian points of particle i: nm * 4 doubles (r_k[3], A_k). */
void orc_get_markers(const orc_state *s, int i, double *out)
{
    const orc_particle *q = &s->pt[i];
    for (int k = 0; k < q->nm; k++) {
        out[4*k+0] = q->off[3*k+0]; out[4*k+1] = q->off[3*k+1];
        out[4*k+2] = q->off[3*k+2]; out[4*k+3] = q->area[k];
    }
}

/* ------------------------------------------------------------------------ */
/* 1. Streaming (pull) with walls.                                           */
/*   flow:    f_a(x) = f*_a(x - e_a), or f*_abar(x) beyond a wall             */
/*            (halfway bounce-back, stationary no-slip wall);                 */
/*   thermal: g_a(x) = g*_a(x - e_a), or -g*_abar(x) + 2 w_a T_wall          */
/*            (anti-bounce-back, Dirichlet wall temperature).                 */
/* reading: the paper prescribes no-slip, cold walls without a scheme.       */
/* ------------------------------------------------------------------------ */
static void stream(orc_state *s)
{
    const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int jj = 0; jj < ny; jj++)
            for (int i = 0; i < nx; i++) {
                long n = node_index(s, i, jj, k);
                int xc[3] = {i, jj, k};
                for (int a = 0; a < s->Q; a++) {
                    int src[3], wall = 0;
                    for (int d = 0; d < 3; d++) {
                        if (d == 2 && s->p.dim == 2) { src[d] = 0; continue; }
                        src[d] = map_coord(s, d, xc[d] - s->e[a][d]);
                        if (src[d] < 0) wall = 1;
                    }
                    if (wall) s->fs[n*s->Q + a] = s->f[n*s->Q + s->opp[a]];
                    else s->fs[n*s->Q + a] = s->f[node_index(s, src[0], src[1], src[2])*s->Q + a];
                }
                for (int a = 0; a < s->Qg; a++) {
                    int src[3], face = -1;
                    for (int d = 0; d < 3; d++) {
                        if (d == 2 && s->p.dim == 2) { src[d] = 0; continue; }
                        src[d] = map_coord(s, d, xc[d] - s->eg[a][d]);
                        if (src[d] < 0) face = 2*d + (s->eg[a][d] > 0 ? 0 : 1);
                    }
                    if (face >= 0)
                        s->gs[n*s->Qg + a] = -s->g[n*s->Qg + s->oppg[a]] + 2.0 * s->wg[a] * s->p.T_wall[face];
                    else
                        s->gs[n*s->Qg + a] = s->g[node_index(s, src[0], src[1], src[2])*s->Qg + a];
                }
            }
}

/* 2. Raw moments of the streamed populations (reading: no half-force terms
 * in the values handed to the interpolation). */
static void moments(orc_state *s)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < s->N; n++) {
        double r = 0, jx = 0, jy = 0, jz = 0, t = 0;
        for (int a = 0; a < s->Q; a++) {
            double v = s->fs[n*s->Q + a];
            r += v; jx += s->e[a][0]*v; jy += s->e[a][1]*v; jz += s->e[a][2]*v;
        }
        for (int a = 0; a < s->Qg; a++) t += s->gs[n*s->Qg + a];
        s->rho[n] = r; s->j[3*n] = jx; s->j[3*n+1] = jy; s->j[3*n+2] = jz; s->S[n] = t;
    }
}

/* Eqs. (lbm10)-(lbm12): spread a point's force F_l A_l and heat Q_l A_l to
 * every node within |a| < 2 of X on each axis (the nodes floor(X) - 1 ..
 * floor(X) + 2); nodes beyond a wall are dropped, periodic axes wrap. */
static void spread_point(orc_state *s, const double X[3], const double FA[3], double QA)
{
    const int dim = s->p.dim;
    int b[3];
    for (int d = 0; d < 3; d++) b[d] = (int)floor(X[d]);
    int nf = dim == 2 ? 16 : 64;
    for (int c = 0; c < nf; c++) {
        int o[3] = {c & 3, (c >> 2) & 3, (c >> 4) & 3};
        double W = 1.0; int idx[3] = {0, 0, 0}, out = 0;
        for (int d = 0; d < dim; d++) {
            int gc = b[d] - 1 + o[d];
            W *= orc_delta_h((double)gc - X[d]);
            idx[d] = map_coord(s, d, gc);
            if (idx[d] < 0) out = 1;
        }
        if (out) continue;
        long n = node_index(s, idx[0], idx[1], idx[2]);
        for (int d = 0; d < 3; d++) s->FB[3*n + d] += FA[d] * W;
        s->QB[n] += QA * W;
    }
}

/* 3.-6. Interpolation, exchange, reactions and spreading, one particle and
 * one Lagrangian point at a time. */
static void pibm(orc_state *s, int record_reactions)
{
    const int dim = s->p.dim;
    memset(s->FB, 0, sizeof(double) * s->N * 3);
    memset(s->QB, 0, sizeof(double) * s->N);
    for (int ip = 0; ip < s->np; ip++) {
        orc_particle *q = &s->pt[ip];
        double Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0}, Hs = 0, dTs = 0;
        for (int k = 0; k < q->nm; k++) {
            const double *r = &q->off[3*k];
            double X[3], U[3];
            for (int d = 0; d < 3; d++) X[d] = q->x[d] + r[d];
            /* U_l = U_p + Omega x r (2D: Omega is the z component). */
            U[0] = q->u[0] + q->om[1]*r[2] - q->om[2]*r[1];
            U[1] = q->u[1] + q->om[2]*r[0] - q->om[0]*r[2];
            U[2] = q->u[2] + q->om[0]*r[1] - q->om[1]*r[0];
            if (dim == 2) { X[2] = 0; U[2] = 0; }
            int b[3]; double t[3];
            for (int d = 0; d < 3; d++) { b[d] = (int)floor(X[d]); t[d] = X[d] - b[d]; }
            double rl = 0, jl[3] = {0, 0, 0}, Tl = 0;
            if (s->p.interp_order == 4) {
                /* Eq. (lbm6) with i_max = j_max = k_max = 4: the tensor product
                 * of the cubic Lagrange polynomials through the nodes
                 * b - 1 .. b + 2 of each axis, l_k(t) = prod_{m != k}
                 * (t - m) / (k - m) over k, m in {-1, 0, 1, 2}. */
                double L[3][4];
                for (int d = 0; d < 3; d++)
                    for (int k = 0; k < 4; k++) {
                        double w = 1.0;
                        for (int m = 0; m < 4; m++)
                            if (m != k) w *= (t[d] - (m - 1)) / (double)(k - m);
                        L[d][k] = w;
                    }
                int nc = dim == 2 ? 16 : 64;
                for (int c = 0; c < nc; c++) {
                    int o[3] = {c & 3, (c >> 2) & 3, (c >> 4) & 3};
                    double W = 1.0;
                    int idx[3] = {0, 0, 0};
                    for (int d = 0; d < dim; d++) {
                        W *= L[d][o[d]];
                        idx[d] = clamp_coord(s, d, b[d] - 1 + o[d]);
                    }
                    long n = node_index(s, idx[0], idx[1], idx[2]);
                    rl += W * s->rho[n];
                    for (int d = 0; d < 3; d++) jl[d] += W * s->j[3*n + d];
                    Tl += W * s->S[n];
                }
            } else {
                /* Eq. (lbm6) with i_max = j_max = k_max = 2: multilinear weights on
                 * the corners of the lattice cell holding X_l. */
                int nc = dim == 2 ? 4 : 8;
                for (int c = 0; c < nc; c++) {
                    int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                    double W = 1.0;
                    int idx[3] = {0, 0, 0};
                    for (int d = 0; d < dim; d++) {
                        W *= o[d] ? t[d] : 1.0 - t[d];
                        idx[d] = clamp_coord(s, d, b[d] + o[d]);
                    }
                    long n = node_index(s, idx[0], idx[1], idx[2]);
                    rl += W * s->rho[n];
                    for (int d = 0; d < 3; d++) jl[d] += W * s->j[3*n + d];
                    Tl += W * s->S[n];
                }
            }
            /* Eqs. (lbm7)-(lbm8): bouncing every direction back at the point
             * and summing e_beta (f_beta - f_alpha) gives 2(rho_l U_l - j_l).
             * reading: rho_f of Eq. (lbm7) is the interpolated rho_l. */
            double Fl[3];
            for (int d = 0; d < 3; d++) Fl[d] = 2.0 * (rl * U[d] - jl[d]);
            if (dim == 2) Fl[2] = 0.0;
            /* Eqs. (lbm7.5), (lbm12.6): heat source density; reading: the
             * prefactor is kappa_T (1 by default). */
            double Ql = 2.0 * s->p.kappa_T * (q->T - Tl);
            double A = q->area[k];
            double FA[3] = {Fl[0]*A, Fl[1]*A, Fl[2]*A}, QA = Ql * A;
            /* Eq. (lbm13): reaction on the particle. */
            for (int d = 0; d < 3; d++) Fs[d] -= FA[d];
            Ts[0] -= r[1]*FA[2] - r[2]*FA[1];
            Ts[1] -= r[2]*FA[0] - r[0]*FA[2];
            Ts[2] -= r[0]*FA[1] - r[1]*FA[0];
            Hs += QA;
            dTs += (q->T - Tl) * A;
            spread_point(s, X, FA, QA);
        }
        if (record_reactions) {
            for (int d = 0; d < 3; d++) { q->F[d] = Fs[d]; q->tq[d] = Ts[d]; }
            if (dim == 2) { q->F[2] = 0; q->tq[0] = 0; q->tq[1] = 0; }
            q->H = Hs; q->dTA = dTs;
        }
    }
}

/* Macroscopic values used by the collision (Sec. 2.1, after Eq. lbm3.5):
 * T = S + Q_B/2 (reading: the e_alpha in the printed T moment is a typo),
 * F = F_B + g beta (T - T_ref) e_up, u = (j + F/2) / rho. */
static void macro(const orc_state *s, long n, double *rho, double u[3], double *T, double F[3])
{
    int up = s->p.dim == 2 ? 1 : 2;
    *rho = s->rho[n];
    *T = s->S[n] + 0.5 * s->QB[n];
    for (int d = 0; d < 3; d++) F[d] = s->FB[3*n + d];
    F[up] += s->p.gbeta * (*T - s->p.T_ref);
    if (s->p.dim == 2) F[2] = 0.0;
    for (int d = 0; d < 3; d++) u[d] = (s->j[3*n + d] + 0.5 * F[d]) / *rho;
}

/* 7. BGK collision, Eqs. (lbm2), (lbm2.5) with sources (lbm9), (lbm12.5). */
static void collide(orc_state *s)
{
    const double tf = s->p.tau_f, tg = s->p.tau_g;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < s->N; n++) {
        double rho, u[3], T, F[3];
        macro(s, n, &rho, u, &T, F);
        for (int a = 0; a < s->Q; a++) {
            double fa = s->fs[n*s->Q + a];
            s->f[n*s->Q + a] = fa - (fa - feq(s, a, rho, u)) / tf + guo(s, a, u, F);
        }
        double Qb = s->QB[n];
        for (int a = 0; a < s->Qg; a++) {
            double ga = s->gs[n*s->Qg + a];
            s->g[n*s->Qg + a] = ga - (ga - geq(s, a, T, u)) / tg + (1.0 - 0.5 / tg) * s->wg[a] * Qb;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 8. DEM (Sec. 2.3).                                                        */
/* ------------------------------------------------------------------------ */
static double volume(const orc_state *s, double R)
{
    const double pi = 3.14159265358979323846;
    return s->p.dim == 2 ? pi * R * R : 4.0 / 3.0 * pi * R * R * R;
}

/* Minimum-image separation on periodic axes. */
static void separation(const orc_state *s, const double *xi, const double *xj, double d[3])
{
    for (int c = 0; c < 3; c++) {
        d[c] = xj[c] - xi[c];
        if (c == 2 && s->p.dim == 2) { d[c] = 0; continue; }
        if (s->p.periodic[c]) {
            double L = nsz(s, c);
            if (d[c] > 0.5 * L) d[c] -= L;
            else if (d[c] < -0.5 * L) d[c] += L;
        }
    }
}

static double *find_xi(orc_particle *q, int partner)
{
    for (int c = 0; c < q->nc; c++) if (q->c[c].partner == partner) return q->c[c].xi;
    return NULL;
}

/* One contact seen from particle i: Hertz normal force (Sec. 2.3), and the
 * tangential spring.  reading: the loading-history weights theta_k of the
 * Mindlin-Deresiewicz increment are taken in the no-slip limit, giving the
 * stiffness 8 G* r_a with r_a = sqrt(R* delta_n), capped by Coulomb friction
 * |F_t| <= mu F_n; 1/G* = sum (2 - nu)/G with G = E / (2 (1 + nu)). */
static void contact_force(const orc_state *s, const orc_particle *qi, const double n[3], double delta,
                          double Rstar, const double vrel[3], const double *xi_old,
                          double Fc[3], double Tc[3], double xi_new[3])
{
    double E = s->p.E_star, nu = s->p.poisson;
    double G = (1.0 - nu) * E / (2.0 * (2.0 - nu));   /* G* for equal materials */
    double Fn = 4.0 / 3.0 * E * sqrt(Rstar) * delta * sqrt(delta);
    double vn = vrel[0]*n[0] + vrel[1]*n[1] + vrel[2]*n[2];
    double vt[3] = {vrel[0] - vn*n[0], vrel[1] - vn*n[1], vrel[2] - vn*n[2]};
    double xi[3] = {0, 0, 0};
    if (xi_old) { xi[0] = xi_old[0]; xi[1] = xi_old[1]; xi[2] = xi_old[2]; }
    double xn = xi[0]*n[0] + xi[1]*n[1] + xi[2]*n[2];
    double dts = 1.0 / s->p.n_sub;
    for (int c = 0; c < 3; c++) xi[c] = xi[c] - xn * n[c] + vt[c] * dts;
    double kt = 8.0 * G * sqrt(Rstar * delta);
    double Ft[3] = {-kt * xi[0], -kt * xi[1], -kt * xi[2]};
    double ft = sqrt(Ft[0]*Ft[0] + Ft[1]*Ft[1] + Ft[2]*Ft[2]);
    double cap = s->p.mu_fric * Fn;
    if (ft > cap) {
        double sc = cap / ft;
        for (int c = 0; c < 3; c++) { Ft[c] *= sc; xi[c] = -Ft[c] / kt; }
    }
    for (int c = 0; c < 3; c++) { Fc[c] = -Fn * n[c] + Ft[c]; xi_new[c] = xi[c]; }
    double rn[3] = {qi->R * n[0], qi->R * n[1], qi->R * n[2]};
    Tc[0] = rn[1]*Ft[2] - rn[2]*Ft[1];
    Tc[1] = rn[2]*Ft[0] - rn[0]*Ft[2];
    Tc[2] = rn[0]*Ft[1] - rn[1]*Ft[0];
}

/* Contact list of particle i: every j != i with overlap, in ascending j, by
 * brute force over all pairs (obviously complete). */
static int contacts_of(const orc_state *s, int i, int *list)
{
    int n = 0;
    for (int jp = 0; jp < s->np; jp++) {
        if (jp == i) continue;
        double d[3];
        separation(s, s->pt[i].x, s->pt[jp].x, d);
        double dist = sqrt(d[0]*d[0] + d[1]*d[1] + d[2]*d[2]);
        if (dist < s->pt[i].R + s->pt[jp].R) list[n++] = jp;
    }
    return n;
}

static void dem_substep(orc_state *s, double (*Fc)[3], double (*Tc)[3], orc_contact (*hist)[ORC_MAX_CONTACTS], int *nh)
{
    const int dim = s->p.dim;
    int overflow = 0;
    /* Each particle's contacts are found and evaluated independently: the
     * iteration for i reads the shared state and writes only slot i, so the
     * particles are shared among threads without changing any result. */
#pragma omp parallel reduction(|:overflow)
    {
    int *list = malloc(sizeof(int) * (s->np > 0 ? s->np : 1));
#pragma omp for schedule(dynamic, 16)
    for (int i = 0; i < s->np; i++) {
        orc_particle *qi = &s->pt[i];
        for (int c = 0; c < 3; c++) { Fc[i][c] = 0; Tc[i][c] = 0; }
        nh[i] = 0;
        int nl = contacts_of(s, i, list);
        for (int m = 0; m < nl; m++) {
            int jp = list[m];
            orc_particle *qj = &s->pt[jp];
            double d[3];
            separation(s, qi->x, qj->x, d);
            double dist = sqrt(d[0]*d[0] + d[1]*d[1] + d[2]*d[2]);
            double n[3] = {d[0]/dist, d[1]/dist, d[2]/dist};
            double delta = qi->R + qj->R - dist;
            double Rstar = qi->R * qj->R / (qi->R + qj->R);
            /* relative velocity of i's contact point with respect to j's */
            double wi[3], wj[3];
            double ri[3] = {qi->R*n[0], qi->R*n[1], qi->R*n[2]};
            double rj[3] = {qj->R*n[0], qj->R*n[1], qj->R*n[2]};
            wi[0] = qi->om[1]*ri[2] - qi->om[2]*ri[1];
            wi[1] = qi->om[2]*ri[0] - qi->om[0]*ri[2];
            wi[2] = qi->om[0]*ri[1] - qi->om[1]*ri[0];
            wj[0] = qj->om[1]*rj[2] - qj->om[2]*rj[1];
            wj[1] = qj->om[2]*rj[0] - qj->om[0]*rj[2];
            wj[2] = qj->om[0]*rj[1] - qj->om[1]*rj[0];
            double vrel[3];
            for (int c = 0; c < 3; c++) vrel[c] = (qi->u[c] - qj->u[c]) + (wi[c] + wj[c]);
            double F[3], T[3], xn[3];
            contact_force(s, qi, n, delta, Rstar, vrel, find_xi(qi, jp), F, T, xn);
            for (int c = 0; c < 3; c++) { Fc[i][c] += F[c]; Tc[i][c] += T[c]; }
            if (nh[i] < ORC_MAX_CONTACTS) {
                hist[i][nh[i]].partner = jp;
                memcpy(hist[i][nh[i]].xi, xn, sizeof xn);
                nh[i]++;
            } else overflow = 1;
        }
        /* Walls: halfway planes at -1/2 and n - 1/2 on non-periodic axes, same
         * material as the particles, R* = R_i. */
        for (int ax = 0; ax < dim; ax++) {
            if (s->p.periodic[ax]) continue;
            for (int side = 0; side < 2; side++) {
                double gap = side == 0 ? qi->x[ax] + 0.5 : (nsz(s, ax) - 0.5) - qi->x[ax];
                double delta = qi->R - gap;
                if (!(delta > 0)) continue;
                double n[3] = {0, 0, 0};
                n[ax] = side == 0 ? -1.0 : 1.0;
                double ri[3] = {qi->R*n[0], qi->R*n[1], qi->R*n[2]}, wi[3];
                wi[0] = qi->om[1]*ri[2] - qi->om[2]*ri[1];
                wi[1] = qi->om[2]*ri[0] - qi->om[0]*ri[2];
                wi[2] = qi->om[0]*ri[1] - qi->om[1]*ri[0];
                double vrel[3];
                for (int c = 0; c < 3; c++) vrel[c] = qi->u[c] + wi[c];
                int partner = -1 - (2*ax + side);
                double F[3], T[3], xn[3];
                contact_force(s, qi, n, delta, qi->R, vrel, find_xi(qi, partner), F, T, xn);
                for (int c = 0; c < 3; c++) { Fc[i][c] += F[c]; Tc[i][c] += T[c]; }
                if (nh[i] < ORC_MAX_CONTACTS) {
                    hist[i][nh[i]].partner = partner;
                    memcpy(hist[i][nh[i]].xi, xn, sizeof xn);
                    nh[i]++;
                } else overflow = 1;
            }
        }
    }
    free(list);
    }
    if (overflow) s->error = 1;
    /* Install the new histories (pairs no longer in contact are dropped). */
    for (int i = 0; i < s->np; i++) {
        s->pt[i].nc = nh[i];
        memcpy(s->pt[i].c, hist[i], sizeof(orc_contact) * nh[i]);
    }
    /* Eq. (demgov), semi-implicit Euler; reading: the gravity term carries
     * the particle mass, m a = m (1 - rho_f / rho_p) g + F. */
    const double dts = 1.0 / s->p.n_sub;
    const int up = dim == 2 ? 1 : 2;
    for (int i = 0; i < s->np; i++) {
        orc_particle *q = &s->pt[i];
        if (q->flags & ORC_FIXED) continue;
        double V = volume(s, q->R);
        double m = q->rho_r * V;
        double I = dim == 2 ? 0.5 * m * q->R * q->R : 0.4 * m * q->R * q->R;
        double rho_p = q->rho_r;
        if (q->flags & ORC_THERMO) rho_p = q->rho_r * (1.0 - s->p.beta_p * (q->T - s->p.T_ref));
        double gv[3] = {0, 0, 0};
        gv[up] = -s->p.gravity * (1.0 - 1.0 / rho_p);
        for (int c = 0; c < dim; c++) {
            q->u[c] += dts * ((q->F[c] + Fc[i][c]) / m + gv[c]);
            q->x[c] += dts * q->u[c];
        }
        if (dim == 2) {
            q->om[2] += dts * (q->tq[2] + Tc[i][2]) / I;
            q->th[2] += dts * q->om[2];
        } else {
            for (int c = 0; c < 3; c++) {
                q->om[c] += dts * (q->tq[c] + Tc[i][c]) / I;
                q->th[c] += dts * q->om[c];
            }
        }
    }
}

static void dem(orc_state *s)
{
    if (s->np == 0) return;
    double (*Fc)[3] = malloc(sizeof(double[3]) * s->np);
    double (*Tc)[3] = malloc(sizeof(double[3]) * s->np);
    orc_contact (*hist)[ORC_MAX_CONTACTS] = malloc(sizeof(orc_contact[ORC_MAX_CONTACTS]) * s->np);
    int *nh = malloc(sizeof(int) * s->np);
    for (int k = 0; k < s->p.n_sub; k++) dem_substep(s, Fc, Tc, hist, nh);
    free(Fc); free(Tc); free(hist); free(nh);
}

/* 9. Thermosensitive particles (Sec. 3.4; reading: lumped capacitance,
 * rho_r c_r V dT_p = -H_p per step, H_p being the heat handed to the fluid). */
static void thermo(orc_state *s)
{
    for (int i = 0; i < s->np; i++) {
        orc_particle *q = &s->pt[i];
        if (!(q->flags & ORC_THERMO)) continue;
        q->T -= q->H / (q->rho_r * s->p.c_r * volume(s, q->R));
    }
}

/* ------------------------------------------------------------------------ */
/* Driver entry points.                                                       */
/* ------------------------------------------------------------------------ */
void orc_step(orc_state *s, int nsteps)
{
    for (int it = 0; it < nsteps; it++) {
        stream(s);
        moments(s);
        pibm(s, 1);
        collide(s);
        dem(s);
        thermo(s);
        s->step++;
    }
}

/* One step of the one-point mode with prescribed reactions in place of the
 * Lagrangian-point exchange (a learned closure supplies them): FH holds 4
 * doubles per particle, the force F_p on the particle and the heat H_p it
 * gives the fluid.  The fluid receives F_l A_l = -F_p and Q_l A_l = H_p
 * spread from the centre (Eqs. lbm10-lbm12.6 for one point); the particle
 * receives F_p and no fluid torque (a point has no lever arm, Eq. lbm13);
 * the reactions record F_p, 0, H_p and sum (T_p - T_l) A = H_p / (2 kappa_T).
 * Collision, DEM and the thermosensitive update follow as in orc_step. */
void orc_step_prescribed(orc_state *s, const double *FH)
{
    stream(s);
    moments(s);
    memset(s->FB, 0, sizeof(double) * s->N * 3);
    memset(s->QB, 0, sizeof(double) * s->N);
    for (int ip = 0; ip < s->np; ip++) {
        orc_particle *q = &s->pt[ip];
        const double *r = FH + 4 * (long)ip;
        double X[3] = {q->x[0], q->x[1], s->p.dim == 2 ? 0.0 : q->x[2]};
        double FA[3] = {-r[0], -r[1], s->p.dim == 2 ? 0.0 : -r[2]};
        spread_point(s, X, FA, r[3]);
        for (int d = 0; d < 3; d++) { q->F[d] = -FA[d]; q->tq[d] = 0.0; }
        q->H = r[3];
        q->dTA = s->p.kappa_T != 0.0 ? r[3] / (2.0 * s->p.kappa_T) : 0.0;
    }
    collide(s);
    dem(s);
    thermo(s);
    s->step++;
}

/* DEM only (no fluid): advance n_steps * n_sub sub-steps with the stored
 * hydrodynamic reactions (zero unless a fluid step ran). */
void orc_dem_only(orc_state *s, int nsteps)
{
    for (int it = 0; it < nsteps; it++) dem(s);
}

void orc_clear_reactions(orc_state *s)
{
    for (int i = 0; i < s->np; i++) {
        orc_particle *q = &s->pt[i];
        memset(q->F, 0, sizeof q->F); memset(q->tq, 0, sizeof q->tq); q->H = 0; q->dTA = 0;
    }
}

/* Macroscopic fields (rho, u[3], T per node, node index x fastest) that the
 * next collision would use; the state is left untouched.  Also returns the
 * forcing fields when FB / QB are non-NULL. */
void orc_fields(orc_state *s, double *rho, double *u, double *T, double *FB, double *QB)
{
    stream(s);
    moments(s);
    pibm(s, 0);
    for (long n = 0; n < s->N; n++) {
        double r, uu[3], t, F[3];
        macro(s, n, &r, uu, &t, F);
        if (rho) rho[n] = r;
        if (u) { u[3*n] = uu[0]; u[3*n+1] = uu[1]; u[3*n+2] = uu[2]; }
        if (T) T[n] = t;
        if (FB) { FB[3*n] = s->FB[3*n]; FB[3*n+1] = s->FB[3*n+1]; FB[3*n+2] = s->FB[3*n+2]; }
        if (QB) QB[n] = s->QB[n];
    }
}

/* Raw post-stream moments of the current state (the exchange's inputs,
 * Sec. 2.2): rho[N], j[3N], S[N] with S = sum g; the state is not advanced. */
void orc_raw_moments(orc_state *s, double *rho, double *j, double *S)
{
    stream(s);
    moments(s);
    for (long n = 0; n < s->N; n++) {
        rho[n] = s->rho[n];
        j[3*n] = s->j[3*n]; j[3*n+1] = s->j[3*n+1]; j[3*n+2] = s->j[3*n+2];
        S[n] = s->S[n];
    }
}

/* The Lagrangian-point exchange and reactions (Eqs. lbm5-lbm8, lbm13) of the
 * current state, recorded as the reactions; the state is not advanced. */
void orc_exchange(orc_state *s)
{
    stream(s);
    moments(s);
    pibm(s, 1);
}

/* Lagrange weight of one corner (for pins): product over axes of the i_max=2
 * polynomial of Eq. (lbm6). */
double orc_lagrange2(double X, int node, int other)
{
    return (X - other) / (double)(node - other);
}

/* Contact list of particle i by brute force (for pins of neighbour search). */
int orc_contacts(const orc_state *s, int i, int *out)
{
    return contacts_of(s, i, out);
}

/* Sum of the raw moments over the lattice (for conservation pins): after
 * stream + moments of the current state; out = {sum rho, sum j[3], sum S}. */
void orc_totals(orc_state *s, double *out)
{
    stream(s);
    moments(s);
    double r = 0, jx = 0, jy = 0, jz = 0, t = 0;
    for (long n = 0; n < s->N; n++) {
        r += s->rho[n]; jx += s->j[3*n]; jy += s->j[3*n+1]; jz += s->j[3*n+2]; t += s->S[n];
    }
    out[0] = r; out[1] = jx; out[2] = jy; out[3] = jz; out[4] = t;
}

/* Threads of the OpenMP loops from now on (n < 1: leave unchanged). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
