/*
 * lbm_ref.c -- plain, slow, FP64 CPU oracle of the fused lattice-Boltzmann
 * LES forest-canopy time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product (the HIP
 * library) never links, loads or calls it, and the two share no code,
 * header, table or helper.
 *
 * Method: Shao, Camps Santasmasas, Xue, Niu, Davidson, Revell, Yao,
 * "Near-wall approximations to speed up simulations for atmosphere boundary
 * layers in the presence of forests using lattice Boltzmann method on GPU",
 * arXiv 2206.15454.
 *
 *   lattice Boltzmann equation with forcing ......... Sec. 2.1, Eq. (lbe)
 *   BGK collision .................................... Sec. 2.1, Eq. (bgk)
 *   second-order equilibrium ......................... Sec. 2.1, Eq. (local_eq)
 *   Guo forcing term ................................. Sec. 2.1, Eq. (bodyforce)
 *   density, momentum, momentum flux ................. Sec. 2.1, Eqs. (density),
 *                                                      (momentum), (tensor)
 *   Smagorinsky eddy viscosity, total tau ............ Sec. 2.2
 *   forest drag force ................................ Sec. 2.3, Eq. (forestForce)
 *   leaf-area-density profile ........................ Sec. 2.3, Eq. (af_theory)
 *   order of operations inside a step ................ Sec. 3, Algorithm 1
 *
 * Readings taken where the paper is silent or garbled (each is marked
 * "reading" where it is used):
 *   R1  Eq. (lbe)/(bgk) print the collision with a "+" sign; relaxation
 *       towards equilibrium needs f* = f - (f - feq)/tau + F_i.
 *   R2  The lattice tables are not printed: standard D3Q19, weights
 *       1/3, 1/18, 1/36, c_s^2 = 1/3, lattice units dx = dt = 1.
 *   R3  F in Eqs. (bodyforce)/(momentum) is a force density: F = rho * a,
 *       where a is the driving acceleration g plus the canopy drag
 *       acceleration.  The drag of Eq. (forestForce) is an acceleration.
 *   R4  The Guo prefactor (1 - 1/(2 tau)) uses the total relaxation time,
 *       since Sec. 2.2 replaces tau by tau_total in the collision.
 *   R5  The strain magnitude follows Eq. (strain) with c = dx = delta = 1;
 *       nu_t = C_smag |S| (Delta = 1) and tau_total = tau0 + 3 nu_t, which
 *       is tau_total = (tau0 + sqrt(tau0^2 + 18 sqrt2 C_smag Q^(1/2)/rho))/2.
 *       (The printed tau_total drops the rho inside the root.)
 *   R6  Pi_neq = Pi - Pi_eq(rho, u) with the force-corrected u, no extra
 *       forcing correction.
 *   R7  The drag acts on x only (the paper: "added in the streamwise
 *       direction") with |u| the full speed; an optional flag applies it to
 *       all three components.
 *   R8  The drag is evaluated explicitly from u* = (j + rho g/2)/rho, then
 *       the velocity is corrected with half the drag (Algorithm 1: calculate
 *       u, calculate the forest force, correct u).  No iteration.
 *   R9  Walls: halfway bounce-back (no-slip, wall half a cell below the first
 *       cell centre); free-slip is specular reflection; x and z periodic.
 *       The forced-equilibrium boundary of Sec. 5.1 ("moves with the free-
 *       stream velocity") supplies f_eq(1, u_wall) for every population
 *       entering from it; populations leaving through it are lost.
 *   R10 The LAD is evaluated at cell centres y_j = j + 1/2; n = 6 below y_m,
 *       1/2 from y_m to h; zero at and above h.
 *   R11 Initial state: f* = feq(rho0, u0), taken as post-collision at t = 0.
 *   R12 Moments reported at time t are those of the collision of step t
 *       (rho, the corrected u, nu_t).
 *
 * State: post-collision populations f*_q(x, t), two FP64 arrays (pull scheme,
 * double buffered), layout [q][z][y][x], x fastest.  OpenMP over z only; no
 * reduction inside a step, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

/* D3Q19 velocities in the interface order: rest; +x,-x,+y,-y,+z,-z; then
 * the twelve edge vectors, each directly followed by its opposite. (R2) */
static const int CV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared (R2) */

static double weight(int q) {
    int n2 = CV[q][0] * CV[q][0] + CV[q][1] * CV[q][1] + CV[q][2] * CV[q][2];
    if (n2 == 0) return 1.0 / 3.0;
    if (n2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* direction whose velocity is -c_q */
static int opposite(int q) {
    for (int p = 0; p < NQ; ++p)
        if (CV[p][0] == -CV[q][0] && CV[p][1] == -CV[q][1] && CV[p][2] == -CV[q][2]) return p;
    return -1;
}

/* direction whose velocity is c_q with its y component reversed */
static int mirror_y(int q) {
    for (int p = 0; p < NQ; ++p)
        if (CV[p][0] == CV[q][0] && CV[p][1] == -CV[q][1] && CV[p][2] == CV[q][2]) return p;
    return -1;
}

enum { BC_PERIODIC = 0, BC_BOUNCEBACK = 1, BC_FREESLIP = 2, BC_EQUILIBRIUM = 3 };

/* ------------------------------------------------------------------------ */
/* pure per-cell formulas                                                    */
/* ------------------------------------------------------------------------ */

int ref_lattice(int *c, double *w) {
    for (int q = 0; q < NQ; ++q) {
        for (int a = 0; a < 3; ++a) c[3 * q + a] = CV[q][a];
        w[q] = weight(q);
    }
    return NQ;
}

/* Eq. (local_eq): feq_i = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)] */
void ref_feq(double rho, const double *u, double *feq) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < NQ; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        feq[q] = weight(q) * rho *
                 (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Eq. (bodyforce): F_i = (1 - 1/(2 tau)) w_i [(c_i - u)/cs2 + (c_i.u) c_i/cs2^2] . F */
void ref_guo(double tau, const double *u, const double *F, double *Fi) {
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int q = 0; q < NQ; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            double va = (CV[q][a] - u[a]) / CS2 + cu * CV[q][a] / (CS2 * CS2);
            s += va * F[a];
        }
        Fi[q] = pref * weight(q) * s;
    }
}

/* Eqs. (density), (tensor): rho = sum f, j = sum f c, Pi = sum f c c (3x3) */
void ref_moments_of(const double *f, double *rho, double *j, double *Pi) {
    double r = 0.0, m[3] = {0, 0, 0}, P[9] = {0};
    for (int q = 0; q < NQ; ++q) {
        r += f[q];
        for (int a = 0; a < 3; ++a) {
            m[a] += f[q] * CV[q][a];
            for (int b = 0; b < 3; ++b) P[3 * a + b] += f[q] * CV[q][a] * CV[q][b];
        }
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) j[a] = m[a];
    for (int k = 0; k < 9; ++k) Pi[k] = P[k];
}

/* Sec. 2.2 with reading R5.  Pineq is the full 3x3 non-equilibrium momentum
 * flux.  Returns tau_total; *nut receives nu_t. */
double ref_smag(double tau0, double csmag, double rho, const double *Pineq, double *nut) {
    double q2 = 0.0;
    for (int k = 0; k < 9; ++k) q2 += Pineq[k] * Pineq[k];
    double Qh = sqrt(q2); /* Q^(1/2) = sqrt(Pi_neq : Pi_neq) */
    double nt = 0.0;
    if (csmag > 0.0) {
        /* Eq. (strain) with c = dx = delta = 1:
         *   |S| = (-a + sqrt(a^2 + b)) / (6 rho C),  a = tau0 rho,
         *   b = 18 sqrt(2) rho C Q^(1/2),
         * evaluated in the identical rationalised form b / ((sqrt(a^2+b) + a) 6 rho C),
         * which avoids the cancellation of -a + sqrt(a^2 + b) when b << a^2. */
        double a = tau0 * rho;
        double b = 18.0 * sqrt(2.0) * rho * csmag * Qh;
        double S = b / ((sqrt(a * a + b) + a) * (6.0 * rho * csmag));
        nt = csmag * S; /* Eq. (nu_t), Delta = 1 */
    }
    if (nut) *nut = nt;
    /* nu_total = nu0 + nu_t and nu = cs2 (tau - 1/2): tau_total = tau0 + nu_t / cs2 */
    return tau0 + nt / CS2;
}

/* Eq. (af_theory), evaluated at cell centres y_j = j + 1/2 (R10).  With
 * lai > 0 the profile is rescaled so that its sum over cells equals lai
 * (leaf-area index per unit ground area, one-cell spacing); otherwise the
 * peak value is afm. */
int ref_lad_lalic(double h, double ym, double afm, double lai, int ny, double *out) {
    if (ny < 1 || !(h > 0.0) || !(ym >= 0.0) || !(ym < h)) return 1;
    double sum = 0.0;
    for (int j = 0; j < ny; ++j) {
        double y = j + 0.5;
        double a = 0.0;
        if (y < h) {
            double n = (y < ym) ? 6.0 : 0.5;
            double r = (h - ym) / (h - y);
            a = pow(r, n) * exp(n * (1.0 - r));
        }
        out[j] = a;
        sum += a;
    }
    double scale = afm;
    if (lai > 0.0) {
        if (!(sum > 0.0)) return 1;
        scale = lai / sum;
    }
    for (int j = 0; j < ny; ++j) out[j] *= scale;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* simulation context                                                        */
/* ------------------------------------------------------------------------ */

struct mlp_ref; /* learned closure, oracle side (mlp_ref.c) */
double ref_mlp_closure_nut(const struct mlp_ref *m, const double *feat, int *used_fallback,
                           double smag_nut);
int ref_mlp_features(const struct mlp_ref *m, double tau0, double rho, const double *Pineq,
                     double yh, double lad, double *feat);

typedef struct {
    int nx, ny, nz;
    size_t n;
    double tau0, csmag, g[3];
    int bc_lo, bc_hi;
    double u_wall[3]; /* velocity of the forced-equilibrium boundary (density 1) */
    double cd;
    double *lad;
    double *lad_cell; /* [nz][ny][nx] LAD of a heterogeneous forest, or NULL */
    int vector_drag;
    double canopy_h; /* canopy height in cells, used only by the learned closure's y/h feature */
    double *fa, *fb; /* post-collision populations [q][z][y][x] */
    double *rho, *u, *nut;
    int64_t t;
    double impulse[3];
    int stats_every;
    int64_t stats_n;
    double *stats; /* [ny][10] sums over samples and x-z */
    const struct mlp_ref *mlp;
    int64_t mlp_fallback; /* cells that fell back in the last evaluation of the network */
    int closure_every;    /* evaluate the learned closure every this many steps */
    int closure_lag;      /* steps since its last evaluation (0: evaluate next step) */
} ref_ctx;

static size_t cell(const ref_ctx *c, int i, int j, int k) {
    return ((size_t)k * c->ny + j) * c->nx + i;
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

void *ref_create(int nx, int ny, int nz, double tau0, double csmag, double gx, double gy,
                 double gz, int bc_lo, int bc_hi) {
    if (nx < 1 || ny < 1 || nz < 1 || !(tau0 > 0.5) || csmag < 0.0) return NULL;
    if (bc_lo < 0 || bc_lo > 3 || bc_hi < 0 || bc_hi > 3) return NULL;
    if ((bc_lo == BC_PERIODIC) != (bc_hi == BC_PERIODIC)) return NULL;
    ref_ctx *c = (ref_ctx *)calloc(1, sizeof(ref_ctx));
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->n = (size_t)nx * ny * nz;
    c->tau0 = tau0; c->csmag = csmag;
    c->g[0] = gx; c->g[1] = gy; c->g[2] = gz;
    c->bc_lo = bc_lo; c->bc_hi = bc_hi;
    c->lad = (double *)calloc(ny, sizeof(double));
    c->fa = (double *)calloc(NQ * c->n, sizeof(double));
    c->fb = (double *)calloc(NQ * c->n, sizeof(double));
    c->rho = (double *)calloc(c->n, sizeof(double));
    c->u = (double *)calloc(3 * c->n, sizeof(double));
    c->nut = (double *)calloc(c->n, sizeof(double));
    c->stats = (double *)calloc(10 * (size_t)ny, sizeof(double));
    c->canopy_h = 1.0;
    c->closure_every = 1;
    if (!c->lad || !c->fa || !c->fb || !c->rho || !c->u || !c->nut || !c->stats) {
        free(c->lad); free(c->fa); free(c->fb); free(c->rho); free(c->u); free(c->nut);
        free(c->stats); free(c);
        return NULL;
    }
    return c;
}

void ref_destroy(void *h) {
    ref_ctx *c = (ref_ctx *)h;
    if (!c) return;
    free(c->lad); free(c->fa); free(c->fb); free(c->rho); free(c->u); free(c->nut);
    free(c->stats); free(c->lad_cell); free(c);
}

int ref_set_canopy(void *h, double cd, const double *lad, int ny, int vector_drag) {
    ref_ctx *c = (ref_ctx *)h;
    if (ny != c->ny) return 1;
    c->cd = cd;
    for (int j = 0; j < ny; ++j) c->lad[j] = lad ? lad[j] : 0.0;
    c->vector_drag = vector_drag;
    free(c->lad_cell);
    c->lad_cell = NULL;
    return 0;
}

double ref_forest_lad(uint32_t code, double afm, int constant);

/* Heterogeneous forest (Sec. 3, Algorithm 1): the LAD of every cell from
 * its forest code (forest_ref.c); replaces the per-row profile until the
 * next ref_set_canopy. */
int ref_set_forest(void *h, double cd, double afm, int constant, const uint32_t *codes,
                   int vector_drag) {
    ref_ctx *c = (ref_ctx *)h;
    double *l = (double *)malloc(c->n * sizeof(double));
    if (!l) return 1;
    for (size_t x = 0; x < c->n; ++x) l[x] = ref_forest_lad(codes[x], afm, constant);
    free(c->lad_cell);
    c->lad_cell = l;
    c->cd = cd;
    c->vector_drag = vector_drag;
    return 0;
}

double ref_mlp_canopy_h(const void *m);

/* learned closure (NULL restores Smagorinsky); the blob fixes the canopy
 * height used by the y/h feature */
/* velocity imposed by a forced-equilibrium boundary (Sec. 5.1: the upper
 * boundary moves with the free-stream velocity) */
void ref_set_wall_velocity(void *h, double ux, double uy, double uz) {
    ref_ctx *c = (ref_ctx *)h;
    c->u_wall[0] = ux;
    c->u_wall[1] = uy;
    c->u_wall[2] = uz;
}

void ref_set_closure(void *h, const void *mlp) {
    ref_ctx *c = (ref_ctx *)h;
    c->mlp = (const struct mlp_ref *)mlp;
    c->canopy_h = mlp ? ref_mlp_canopy_h(mlp) : 1.0;
    c->closure_lag = 0;
}

/* Learned closure evaluated on every `every`-th step only, its nu_t reused
 * by the steps in between (a cost saving of this implementation, not of
 * the paper); the next step evaluates. */
int ref_set_closure_interval(void *h, int every) {
    ref_ctx *c = (ref_ctx *)h;
    if (every < 1) return 1;
    c->closure_every = every;
    c->closure_lag = 0;
    return 0;
}

/* R11: f*(x, 0) = feq(rho0, u0); moments before any step are rho0, u0, 0 */
int ref_init(void *h, const double *rho, const double *u) {
    ref_ctx *c = (ref_ctx *)h;
    size_t n = c->n;
    for (size_t x = 0; x < n; ++x) {
        double uu[3] = {u[x], u[n + x], u[2 * n + x]}, feq[NQ];
        ref_feq(rho[x], uu, feq);
        for (int q = 0; q < NQ; ++q) c->fa[q * n + x] = feq[q];
        c->rho[x] = rho[x];
        for (int a = 0; a < 3; ++a) c->u[a * n + x] = uu[a];
        c->nut[x] = 0.0;
    }
    c->t = 0;
    c->impulse[0] = c->impulse[1] = c->impulse[2] = 0.0;
    c->mlp_fallback = 0;
    c->closure_lag = 0;
    return 0;
}

/* overwrite the post-collision populations at the current time */
void ref_set_f(void *h, const double *f) {
    ref_ctx *c = (ref_ctx *)h;
    memcpy(c->fa, f, NQ * c->n * sizeof(double));
    c->closure_lag = 0;
}

void ref_get_f(const void *h, double *f) {
    const ref_ctx *c = (const ref_ctx *)h;
    memcpy(f, c->fa, NQ * c->n * sizeof(double));
}

/* Streaming with boundaries (Algorithm 1, "Stream"; R9): the population that
 * arrives at (i,j,k) in direction q. */
static double pull(const ref_ctx *c, const double *fp, int q, int i, int j, int k) {
    int si = wrap(i - CV[q][0], c->nx);
    int sk = wrap(k - CV[q][2], c->nz);
    int sj = j - CV[q][1];
    size_t n = c->n;
    if (sj >= 0 && sj < c->ny) return fp[q * n + cell(c, si, sj, sk)];
    int bc = (sj < 0) ? c->bc_lo : c->bc_hi;
    int wall_row = (sj < 0) ? 0 : c->ny - 1;
    switch (bc) {
    case BC_PERIODIC:
        return fp[q * n + cell(c, si, wrap(sj, c->ny), sk)];
    case BC_BOUNCEBACK: /* the population that left this cell towards the wall */
        return fp[opposite(q) * n + cell(c, i, j, k)];
    case BC_EQUILIBRIUM: { /* forced equilibrium at the wall velocity, density 1 */
        double feq[NQ];
        ref_feq(1.0, c->u_wall, feq);
        return feq[q];
    }
    default: /* free-slip: left the wall row of the upstream column moving towards the wall */
        return fp[mirror_y(q) * n + cell(c, si, wall_row, sk)];
    }
}

/* streamed populations (the pre-collision inputs of the next step) */
void ref_pull(const void *h, double *fin) {
    const ref_ctx *c = (const ref_ctx *)h;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i)
                for (int q = 0; q < NQ; ++q)
                    fin[q * c->n + cell(c, i, j, k)] = pull(c, c->fa, q, i, j, k);
}

/* One cell of one step in the order of Algorithm 1.  fin: streamed
 * populations; writes post-collision fout, moments, the body force. */
static void collide_cell(const ref_ctx *c, int jrow, size_t xc, int eval, const double *fin,
                         double *fout, double *rho_o, double *u_o, double *nut_o, double *F_o,
                         int *fallback) {
    double rho, jm[3], Pi[9];
    ref_moments_of(fin, &rho, jm, Pi);

    /* "Calculate local cell velocity": Eq. (momentum) with the driving force only (R8) */
    double F[3], us[3], u[3];
    for (int a = 0; a < 3; ++a) {
        F[a] = rho * c->g[a];
        us[a] = (jm[a] + 0.5 * F[a]) / rho;
        u[a] = us[a];
    }
    double lad = c->lad_cell ? c->lad_cell[xc] : c->lad[jrow];
    if (lad > 0.0) { /* "if cell x is forest" */
        /* "Calculate forest force", Eq. (forestForce) as an acceleration (R3, R7) */
        double speed = sqrt(us[0] * us[0] + us[1] * us[1] + us[2] * us[2]);
        double ad[3] = {-c->cd * lad * speed * us[0], 0.0, 0.0};
        if (c->vector_drag) {
            ad[1] = -c->cd * lad * speed * us[1];
            ad[2] = -c->cd * lad * speed * us[2];
        }
        /* "Correct the local cell velocity using the forest force" */
        for (int a = 0; a < 3; ++a) {
            F[a] = rho * (c->g[a] + ad[a]);
            u[a] = (jm[a] + 0.5 * F[a]) / rho;
        }
    }

    double feq[NQ];
    ref_feq(rho, u, feq);
    /* Pi = Pi_eq + Pi_neq with Pi_eq the momentum flux of feq (R6) */
    double rho_e, j_e[3], Pi_eq[9], Pineq[9];
    ref_moments_of(feq, &rho_e, j_e, Pi_eq);
    for (int k = 0; k < 9; ++k) Pineq[k] = Pi[k] - Pi_eq[k];

    double nut;
    double tau = ref_smag(c->tau0, c->csmag, rho, Pineq, &nut);
    if (c->mlp && !eval) {
        nut = c->nut[xc]; /* the learned nu_t of the last evaluation */
        tau = c->tau0 + nut / CS2;
    } else if (c->mlp) {
        double feat[9];
        double yh = (jrow + 0.5) / c->canopy_h;
        ref_mlp_features(c->mlp, c->tau0, rho, Pineq, yh, lad, feat);
        int fb = 0;
        nut = ref_mlp_closure_nut(c->mlp, feat, &fb, nut);
        *fallback += fb;
        tau = c->tau0 + nut / CS2;
    }

    double Fi[NQ];
    ref_guo(tau, u, F, Fi); /* R4: total tau in the prefactor */
    for (int q = 0; q < NQ; ++q)
        fout[q] = fin[q] - (fin[q] - feq[q]) / tau + Fi[q]; /* Eqs. (lbe), (bgk), R1 */

    *rho_o = rho;
    for (int a = 0; a < 3; ++a) {
        u_o[a] = u[a];
        F_o[a] = F[a];
    }
    *nut_o = nut;
}

static void sample_stats(ref_ctx *c) {
    size_t n = c->n;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                size_t x = cell(c, i, j, k);
                double u = c->u[x], v = c->u[n + x], w = c->u[2 * n + x];
                double *s = c->stats + 10 * (size_t)j;
                s[0] += u; s[1] += v; s[2] += w;
                s[3] += u * u; s[4] += v * v; s[5] += w * w;
                s[6] += u * v; s[7] += u * w; s[8] += v * w;
                s[9] += c->nut[x];
            }
    c->stats_n += 1;
}

int ref_step(void *h, int64_t nsteps) {
    ref_ctx *c = (ref_ctx *)h;
    size_t n = c->n;
    double *Fsum = (double *)calloc(3 * (size_t)c->nz, sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t fb_total = 0;
        const int eval = c->closure_lag == 0;
#pragma omp parallel for schedule(static) reduction(+ : fb_total)
        for (int k = 0; k < c->nz; ++k) {
            double Fz[3] = {0, 0, 0};
            int fb = 0;
            for (int j = 0; j < c->ny; ++j)
                for (int i = 0; i < c->nx; ++i) {
                    double fin[NQ], fout[NQ], uo[3], Fo[3], r, nt;
                    for (int q = 0; q < NQ; ++q) fin[q] = pull(c, c->fa, q, i, j, k);
                    size_t x = cell(c, i, j, k);
                    collide_cell(c, j, x, eval, fin, fout, &r, uo, &nt, Fo, &fb);
                    for (int q = 0; q < NQ; ++q) c->fb[q * n + x] = fout[q];
                    c->rho[x] = r;
                    for (int a = 0; a < 3; ++a) {
                        c->u[a * n + x] = uo[a];
                        Fz[a] += Fo[a];
                    }
                    c->nut[x] = nt;
                }
            for (int a = 0; a < 3; ++a) Fsum[3 * (size_t)k + a] = Fz[a];
            fb_total += fb;
        }
        /* impulse of the body force, summed in a fixed order */
        for (int k = 0; k < c->nz; ++k)
            for (int a = 0; a < 3; ++a) c->impulse[a] += Fsum[3 * (size_t)k + a];
        if (c->mlp && eval) c->mlp_fallback = fb_total;
        if (c->mlp) c->closure_lag = (c->closure_lag + 1) % c->closure_every;
        double *tmp = c->fa;
        c->fa = c->fb;
        c->fb = tmp;
        c->t += 1;
        if (c->stats_every > 0 && c->t % c->stats_every == 0) sample_stats(c);
    }
    free(Fsum);
    return 0;
}

/* moments of the latest step (R12) and global diagnostics.
 * diag: mass, mom[3], impulse[3], max|u|, t, nonfinite, mlp_fallback */
int ref_moments(const void *h, double *rho, double *u, double *nut, double *diag) {
    const ref_ctx *c = (const ref_ctx *)h;
    size_t n = c->n;
    if (rho) memcpy(rho, c->rho, n * sizeof(double));
    if (u) memcpy(u, c->u, 3 * n * sizeof(double));
    if (nut) memcpy(nut, c->nut, n * sizeof(double));
    if (diag) {
        double mass = 0, mom[3] = {0, 0, 0}, umax = 0;
        int64_t bad = 0;
        for (size_t x = 0; x < n; ++x) {
            double r = c->rho[x], a = c->u[x], b = c->u[n + x], w = c->u[2 * n + x];
            if (!isfinite(r) || !isfinite(a) || !isfinite(b) || !isfinite(w) ||
                !isfinite(c->nut[x])) {
                bad++;
                continue;
            }
            mass += r;
            mom[0] += r * a; mom[1] += r * b; mom[2] += r * w;
            double sp = sqrt(a * a + b * b + w * w);
            if (sp > umax) umax = sp;
        }
        diag[0] = mass;
        diag[1] = mom[0]; diag[2] = mom[1]; diag[3] = mom[2];
        diag[4] = c->impulse[0]; diag[5] = c->impulse[1]; diag[6] = c->impulse[2];
        diag[7] = umax;
        diag[8] = (double)c->t;
        diag[9] = (double)bad;
        diag[10] = (double)c->mlp_fallback;
    }
    return 0;
}

/* plane statistics: op 0 reset, 1 enable (sample when t % every == 0 after a
 * step; every = 0 disables), 2 read means [ny][10]:
 * <u> <v> <w> <uu> <vv> <ww> <uv> <uw> <vw> <nu_t> */
int ref_stats(void *h, int op, int every, double *prof, int64_t *nsamples) {
    ref_ctx *c = (ref_ctx *)h;
    if (op == 0) {
        memset(c->stats, 0, 10 * (size_t)c->ny * sizeof(double));
        c->stats_n = 0;
    } else if (op == 1) {
        if (every < 0) return 1;
        c->stats_every = every;
    } else if (op == 2) {
        double denom = (double)c->stats_n * c->nx * c->nz;
        for (int k = 0; k < 10 * c->ny; ++k) prof[k] = c->stats_n ? c->stats[k] / denom : 0.0;
    } else {
        return 1;
    }
    if (nsamples) *nsamples = c->stats_n;
    return 0;
}

int ref_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
