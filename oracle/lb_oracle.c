/*
 * lb_oracle.c -- plain FP64 CPU oracle for the coupled cross-diffusion-fluid
 * lattice Boltzmann model of Zhan, Chai & Shi, "A lattice Boltzmann model for
 * the coupled cross-diffusion-fluid system" (arXiv 2101.03055).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or helper with the GPU library; the two are compared
 * on the same seeded inputs.
 *
 * Structure: two population arrays and push streaming.  Every node is
 * collided in the order the paper presents the model (Sec. 2):
 *   scalar moments (Eq. sum-phi) -> body force F(phi) -> fluid velocity
 *   (Eq. sum-u) -> pressure (Eq. sum-p, appendix A) -> diffusion matrix D(phi)
 *   and relaxation matrix from Eq. omega-D -> source S(phi) -> equilibria
 *   (Eqs. feq-phi, heq) -> discrete source (Eq. source), auxiliary source
 *   (Eq. Gi) and discrete force (Eq. force) -> evolution (Eqs. evolution12,
 *   evolution3) -> streaming with the boundary rules of Sec. 3.
 *
 * Lattice units throughout: dx = dt = 1, cs^2 = 1/3 (D2Q5 and D2Q9 tables,
 * Sec. 2).  Readings of the paper (all listed in the design notes):
 *   - vartheta = 0 in Eq. feq-phi (the linear equilibrium Case 2 permits, and
 *     the only one D2Q5 can carry).  lambda is a parameter (Sec. 3 uses
 *     lambda = I).  On D2Q5 the lambda part of Eq. feq-phi is rescaled so that
 *     its second moment is (lambda phi - phi) cs^2 I as the moment condition
 *     of Sec. 2.1 requires: the printed 1/(2 cs^4) assumes a lattice whose
 *     weights satisfy sum_i W_i c_ix^2 c_iy^2 = cs^4, which D2Q5 does not
 *     (there it gives half the required moment).
 *   - varphi is a parameter of Eq. force (Sec. 3 uses varphi = 0).  The
 *     pressure takes the first form of the appendix-A result,
 *     p = cs^2/(1 - W_0) [sum_{i>0} h_i - W_0 u.u/(2 cs^2) + dt (1/omega - 1/2) F_0],
 *     F_0 being the rest component of Eq. force (its second, expanded form
 *     and Eq. sum-p drop the factor W_0 and disagree in sign).  varphi != 0
 *     needs BGK (the correction uses the single fluid rate).
 *   - D-bar of Eq. evolution12, delta d/dt + gamma c_i . grad on the discrete
 *     source S_i = W_i S (Eq. source): d/dt S by the first-order backward
 *     difference (text after Eq. source), S_old at t = 0 being S(phi0); gamma
 *     is diagonal (gamma[a]; 0 in the paper's runs).  The paper gives no
 *     discretisation of c_i . grad S_i: it is taken as W_i c_i . grad S with
 *     grad S by central differences of the previous step's source field
 *     S(x +- e_d, t - dt), the field the step already keeps; across a wall
 *     the node's own value stands in for the missing neighbour (periodic
 *     sides wrap).
 *   - Initial populations: scalar equilibrium of (phi0, u0); fluid equilibrium
 *     of (p0, u0 - F(phi0)/2), so that Eq. sum-u gives u0 at t = 0.
 *   - Half-way walls; anti-bounce-back f_opp = -f*_i + 2 W_i phi_w for
 *     Dirichlet scalars, half-way bounce-back for no-flux scalars and no-slip
 *     fluid, specular reflection for a free-slip fluid wall; a link leaving
 *     the domain through a corner (two walls) bounces back.
 *   - MRT (an option the paper does not define) uses the Lallemand-Luo D2Q9
 *     moment basis; with all rates equal to omega it is BGK.
 *
 * CASE 1 (model 2, the convection cross-diffusion equation without a fluid,
 * Sec. 2): the velocity u(x) is prescribed and constant in time; there are no
 * fluid populations.  The auxiliary source is G_i = (I - omega/2) W_i c_i .
 * d_t(phi u) / cs^2 with the time derivative taken by the first-order backward
 * difference the paper points to, u (phi(t) - phi(t - dt)) / dt; phi(-dt) is
 * phi0, so G vanishes at the first step.  For this model the h array holds,
 * per node, u_x, u_y in planes 0, 1 and phi(t - dt) in planes 2 .. 2 + m - 1;
 * those values stay at their node (no streaming).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXM 4

/* ---- configuration (the oracle's own record; filled by its Python wrapper) */
typedef struct orc_cfg {
    int32_t nx, ny, m;
    int32_t model;          /* 0: linear closures  (D const, S = K phi, F = F0 + Fphi phi)
                               1: chemotaxis closures (Sec. 3.1)
                               2: no fluid (Case 1 of Sec. 2): prescribed constant velocity,
                                  linear closures without force; see CASE 1 below */
    int32_t collision;      /* 0: BGK (Eq. evolution3), 1: MRT */
    int32_t r_kind;         /* chemotaxis cut-off: 0 step, 1 regularised (Sec. 3.1.2) */
    int32_t mutation;       /* 0 = faithful; k > 0 plants mistake k (pin self-test only) */
    int32_t fluid_bc[4];    /* sides x-, x+, y-, y+: 0 periodic, 1 no-slip, 2 free-slip */
    int32_t scalar_bc[4][ORC_MAXM]; /* [side][alpha]: 0 periodic, 1 no-flux, 2 Dirichlet */
    int32_t pad_;
    double tau_f;           /* fluid relaxation time, omega = 1/tau_f */
    double rho0;            /* constant of the fluid equilibrium (Eq. heq) */
    double mrt_s[9];        /* MRT rates in the moment order rho,e,eps,jx,qx,jy,qy,pxx,pxy */
    double D[ORC_MAXM * ORC_MAXM];      /* constant diffusion matrix, row-major */
    double F0[2];                       /* constant body force */
    double Fphi[ORC_MAXM * 2];          /* F += Fphi[alpha] * phi_alpha */
    double K[ORC_MAXM * ORC_MAXM];      /* linear source S = K phi (model 0) */
    double chi, beta, cstar, eps;       /* chemotaxis: D12 -= chi r(c) n, S_c = -beta r(c) n */
    double wall[4 * ORC_MAXM];          /* Dirichlet values [side][alpha] */
    double lam[ORC_MAXM * ORC_MAXM];    /* lambda of Eq. feq-phi, row-major (identity in Sec. 3) */
    double varphi;                      /* varphi of Eq. force (0 in Sec. 3) */
    double gamma[ORC_MAXM];             /* diagonal of gamma in D-bar of Eq. evolution12 (0 in Sec. 3) */
} orc_cfg;

/* ---- lattices (Sec. 2, D2Q5 and D2Q9 tables) ---------------------------- */
static const int e9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                             {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
/* weights kept as exact fractions num/den: W_i x is evaluated as (x num)/den so
 * that each product is correctly rounded (a rounded constant 1/3 would bias
 * every sum over i the same way and drift the conserved totals) */
static const double W9num[9] = {4, 1, 1, 1, 1, 1, 1, 1, 1};
static const double W9den[9] = {9, 9, 9, 9, 9, 36, 36, 36, 36};
static const int e5[5][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}};
static const double W5num[5] = {1, 1, 1, 1, 1};
static const double W5den[5] = {3, 6, 6, 6, 6};
static double W9x(int i, double x) { return x * W9num[i] / W9den[i]; }
static double W5x(int i, double x) { return x * W5num[i] / W5den[i]; }
static const double cs2 = 1.0 / 3.0;
static const double dt = 1.0;

/* index of the velocity equal to (cx, cy) in a set, -1 if none */
static int find_dir(const int (*e)[2], int q, int cx, int cy) {
    for (int i = 0; i < q; ++i)
        if (e[i][0] == cx && e[i][1] == cy) return i;
    return -1;
}

/* ---- small dense linear algebra (plain Gauss-Jordan, partial pivoting) --- */
/* inverts the n x n row-major matrix a into ainv; returns 0 if singular */
static int mat_inverse(int n, const double *a, double *ainv) {
    double w[ORC_MAXM * 2 * ORC_MAXM];
    int cols = 2 * n;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < cols; ++c)
            w[r * cols + c] = (c < n) ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(w[r * cols + k]) > fabs(w[piv * cols + k])) piv = r;
        if (w[piv * cols + k] == 0.0) return 0;
        if (piv != k)
            for (int c = 0; c < cols; ++c) {
                double t = w[k * cols + c];
                w[k * cols + c] = w[piv * cols + c];
                w[piv * cols + c] = t;
            }
        double d = w[k * cols + k];
        for (int c = 0; c < cols; ++c) w[k * cols + c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            double s = w[r * cols + k];
            if (s != 0.0)
                for (int c = 0; c < cols; ++c) w[r * cols + c] -= s * w[k * cols + c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) ainv[r * n + c] = w[r * cols + n + c];
    return 1;
}

/* ---- MRT moment basis (Lallemand & Luo 2000, D2Q9) ----------------------- */
/* rows: rho, e, eps, jx, qx, jy, qy, pxx, pxy, in the velocity order of e9 */
static const double Mmrt[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* 9x9 Gauss-Jordan for the MRT basis (separate from mat_inverse: larger n) */
static int mat_inverse9(const double a[9][9], double ainv[9][9]) {
    double w[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c) w[r][c] = (c < 9) ? a[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int k = 0; k < 9; ++k) {
        int piv = k;
        for (int r = k + 1; r < 9; ++r)
            if (fabs(w[r][k]) > fabs(w[piv][k])) piv = r;
        if (w[piv][k] == 0.0) return 0;
        if (piv != k)
            for (int c = 0; c < 18; ++c) {
                double t = w[k][c];
                w[k][c] = w[piv][c];
                w[piv][c] = t;
            }
        double d = w[k][k];
        for (int c = 0; c < 18; ++c) w[k][c] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == k) continue;
            double s = w[r][k];
            if (s != 0.0)
                for (int c = 0; c < 18; ++c) w[r][c] -= s * w[k][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) ainv[r][c] = w[r][9 + c];
    return 1;
}

/* ---- closures ------------------------------------------------------------ */
/* chemotaxis cut-off r(c): Heaviside step with r(c*) = 1 (Sec. 3.1.3), or the
 * regularised form of Sec. 3.1.2 */
static double cutoff_r(const orc_cfg *cfg, double c) {
    if (cfg->r_kind == 0) return (c >= cfg->cstar) ? 1.0 : 0.0;
    double d = c - cfg->cstar;
    return 0.5 * (1.0 + d / sqrt(d * d + cfg->eps * cfg->eps));
}

/* diffusion matrix D(phi): constant for model 0; for the chemotaxis model the
 * matrix [[D_n, -chi r(c) n], [0, delta]] (Sec. 3.1, dimensionless system) */
static void diffusion_matrix(const orc_cfg *cfg, const double *phi, double *Dm) {
    int m = cfg->m;
    for (int k = 0; k < m * m; ++k) Dm[k] = cfg->D[k];
    if (cfg->model == 1) Dm[0 * m + 1] += -cfg->chi * cutoff_r(cfg, phi[1]) * phi[0];
}

/* source S(phi): K phi for model 0; (0, -beta r(c) n) for chemotaxis */
static void source_S(const orc_cfg *cfg, const double *phi, double *S) {
    int m = cfg->m;
    if (cfg->model == 1) {
        S[0] = 0.0;
        S[1] = -cfg->beta * cutoff_r(cfg, phi[1]) * phi[0];
        return;
    }
    for (int a = 0; a < m; ++a) {
        S[a] = 0.0;
        for (int b = 0; b < m; ++b) S[a] += cfg->K[a * m + b] * phi[b];
    }
}

/* body force F(phi) = F0 + sum_a Fphi_a phi_a (DDC buoyancy RaPr(T + Nc C) z,
 * chemotaxis -Sc gamma n z are both of this form) */
static void body_force(const orc_cfg *cfg, const double *phi, double *F) {
    F[0] = cfg->F0[0];
    F[1] = cfg->F0[1];
    for (int a = 0; a < cfg->m; ++a) {
        F[0] += cfg->Fphi[2 * a + 0] * phi[a];
        F[1] += cfg->Fphi[2 * a + 1] * phi[a];
    }
}

/* relaxation matrix from Eq. omega-D:
 * D = (omega^-1 - I/2) lambda cs^2 dt  =>  omega = (D lambda^-1 / (cs^2 dt) + I/2)^-1.
 * lam_left != 0 plants the mistake lambda^-1 D (pin self-test only). */
static int relaxation_matrix(int m, const double *Dm, const double *lam, int lam_left, double *omega) {
    double li[ORC_MAXM * ORC_MAXM], A[ORC_MAXM * ORC_MAXM];
    if (!mat_inverse(m, lam, li)) return 0;
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double dl = 0.0;
            for (int c = 0; c < m; ++c)
                dl += lam_left ? li[a * m + c] * Dm[c * m + b] : Dm[a * m + c] * li[c * m + b];
            A[a * m + b] = dl / (cs2 * dt) + (a == b ? 0.5 : 0.0);
        }
    return mat_inverse(m, A, omega);
}

/* ---- equilibria, force and sources (exported for the single-node pins) -- */

/* Factor that gives the lambda part of Eq. feq-phi, W_i X cs^2 I:(c_i c_i - cs^2 I)/(2 cs^4),
 * the second moment X cs^2 I the moment condition of Sec. 2.1 asks for.  Its
 * second moment is X/(2 cs^2) sum_i W_i c_ix^2 (|c_i|^2 - 2 cs^2) per unit factor:
 * cs^2 X on D2Q9, cs^2 X / 2 on D2Q5, so the factor is 2 here. */
static double lam_norm(void) {
    double mom = 0.0;
    for (int i = 0; i < 5; ++i) {
        double cc = e5[i][0] * e5[i][0] + e5[i][1] * e5[i][1];
        mom += W5x(i, e5[i][0] * e5[i][0] * (cc - 2.0 * cs2)) / (2.0 * cs2);
    }
    return cs2 / mom;
}

/* Eq. feq-phi on D2Q5 with vartheta = 0:
 * f^eq_{i,a} = W_i [phi_a + c_i.phi_a u / cs^2
 *                   + (k (lambda phi - phi)_a cs^2 I + vartheta phi_a uu):(c_i c_i - cs^2 I)/(2 cs^4)]
 * with k = lam_norm() (k = 1 plants the mistake of the printed D2Q9 form) */
static void feq_node(int m, const double *lam, double k, const double *phi, const double *u,
                     double *feq /*[m][5]*/) {
    const double vartheta = 0.0;
    for (int a = 0; a < m; ++a) {
        double X = -phi[a];
        for (int b = 0; b < m; ++b) X += lam[a * m + b] * phi[b];
        for (int i = 0; i < 5; ++i) {
            double cu = e5[i][0] * u[0] + e5[i][1] * u[1];
            double Q[2][2] = {{k * X * cs2 + vartheta * phi[a] * u[0] * u[0], vartheta * phi[a] * u[0] * u[1]},
                              {vartheta * phi[a] * u[1] * u[0], k * X * cs2 + vartheta * phi[a] * u[1] * u[1]}};
            double contr = 0.0;
            for (int r = 0; r < 2; ++r)
                for (int s = 0; s < 2; ++s)
                    contr += Q[r][s] * (e5[i][r] * e5[i][s] - (r == s ? cs2 : 0.0));
            feq[a * 5 + i] = W5x(i, phi[a] + phi[a] * cu / cs2 + contr / (2.0 * cs2 * cs2));
        }
    }
}

void orc_feq(int m, const double *lam, const double *phi, const double *u, double *feq /*[m][5]*/) {
    feq_node(m, lam, lam_norm(), phi, u, feq);
}

/* Eq. heq with sigma_0 = (W_0 - 1) p / cs^2 + rho0, sigma_i = W_i p / cs^2 */
void orc_heq(double p, const double *u, double rho0, double *heq /*[9]*/) {
    for (int i = 0; i < 9; ++i) {
        double sigma = (i == 0) ? (W9x(0, p) - p) / cs2 + rho0 : W9x(i, p) / cs2;
        double cu = e9[i][0] * u[0] + e9[i][1] * u[1];
        double uu_cc = 0.0;
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s)
                uu_cc += u[r] * u[s] * (e9[i][r] * e9[i][s] - (r == s ? cs2 : 0.0));
        heq[i] = sigma + W9x(i, cu / cs2 + uu_cc / (2.0 * cs2 * cs2));
    }
}

/* Eq. force: F_i = W_i [c_i.F / cs^2 + varphi (uF + Fu):(c_i c_i - cs^2 I)/(2 cs^4)] */
void orc_force_pop(const double *F, const double *u, double varphi, double *Fi /*[9]*/) {
    for (int i = 0; i < 9; ++i) {
        double T2 = 0.0;
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s)
                T2 += (u[r] * F[s] + F[r] * u[s]) * (e9[i][r] * e9[i][s] - (r == s ? cs2 : 0.0));
        Fi[i] = W9x(i, (e9[i][0] * F[0] + e9[i][1] * F[1]) / cs2 + varphi * T2 / (2.0 * cs2 * cs2));
    }
}

/* Eq. Gi: G_{i,a} = sum_b (delta_ab - omega_ab / 2) W_i c_i.(u S_b + phi_b F) / cs^2 */
void orc_aux_source(int m, const double *omega, const double *phi, const double *S,
                    const double *u, const double *F, double *G /*[m][5]*/) {
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 5; ++i) {
            double g = 0.0;
            for (int b = 0; b < m; ++b) {
                double coef = (a == b ? 1.0 : 0.0) - 0.5 * omega[a * m + b];
                double vx = u[0] * S[b] + phi[b] * F[0];
                double vy = u[1] * S[b] + phi[b] * F[1];
                g += coef * W5x(i, e5[i][0] * vx + e5[i][1] * vy) / cs2;
            }
            G[a * 5 + i] = g;
        }
}

/* Eq. source with M_1S = 0: S_{i,a} = W_i S_a */
void orc_source_pop(int m, const double *S, double *Si /*[m][5]*/) {
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 5; ++i) Si[a * 5 + i] = W5x(i, S[a]);
}

/* relaxation matrix for a constant D (exported for the pins) */
int orc_relaxation_matrix(int m, const double *Dm, const double *lam, double *omega) {
    return relaxation_matrix(m, Dm, lam, 0, omega);
}

/* Lallemand-Luo basis and its inverse (exported for the pins) */
int orc_mrt_basis(double *M /*[9][9]*/, double *Minv /*[9][9]*/) {
    double inv[9][9];
    if (!mat_inverse9(Mmrt, inv)) return 0;
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            M[r * 9 + c] = Mmrt[r][c];
            Minv[r * 9 + c] = inv[r][c];
        }
    return 1;
}

/* ---- node-level macroscopic quantities (Eq. sum) ------------------------- */
typedef struct node_macro {
    double phi[ORC_MAXM];
    double F[2];
    double u[2];
    double p;
} node_macro;

static void node_moments(const orc_cfg *cfg, const double *f /*[m][5]*/, const double *h /*[9]*/,
                         node_macro *mc) {
    int m = cfg->m;
    /* Eq. sum-phi */
    for (int a = 0; a < m; ++a) {
        mc->phi[a] = 0.0;
        for (int i = 0; i < 5; ++i) mc->phi[a] += f[a * 5 + i];
    }
    if (cfg->model == 2) { /* Case 1: prescribed velocity, no force, no pressure */
        mc->F[0] = mc->F[1] = 0.0;
        mc->u[0] = h[0];
        mc->u[1] = h[1];
        mc->p = 0.0;
        return;
    }
    body_force(cfg, mc->phi, mc->F);
    /* Eq. sum-u */
    double half = (cfg->mutation == 4) ? 0.0 : dt / 2.0;
    for (int d = 0; d < 2; ++d) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += e9[i][d] * h[i];
        mc->u[d] = s + half * mc->F[d];
    }
    /* pressure, appendix A: p = cs2/(1 - W_0) [sum_{i>0} h_i - W_0 u.u/(2 cs2)
     * + dt (1/omega - 1/2) F_0], F_0 the rest component of Eq. force (0 for varphi = 0) */
    double s = 0.0;
    for (int i = 1; i < 9; ++i) s += h[i];
    double uu = mc->u[0] * mc->u[0] + mc->u[1] * mc->u[1];
    double w0term = (cfg->mutation == 6) ? 0.0 : W9x(0, uu) / (2.0 * cs2);
    double Fi[9];
    orc_force_pop(mc->F, mc->u, cfg->varphi, Fi);
    double corr = dt * (cfg->tau_f - 0.5) * Fi[0];
    if (cfg->mutation == 13) corr = -corr;
    /* cs2 / (1 - W_0) with W_0 = 4/9 */
    mc->p = cs2 * W9den[0] / (W9den[0] - W9num[0]) * (s - w0term + corr);
}

/* ---- collision of one node ----------------------------------------------- */
static int collide_node(const orc_cfg *cfg, const double Minv[9][9], const double *f,
                        const double *h, const double *Sold, const double *gradS, double *fs, double *hs,
                        double *Snew) {
    int m = cfg->m;
    node_macro mc;
    node_moments(cfg, f, h, &mc);

    double Dm[ORC_MAXM * ORC_MAXM], omega[ORC_MAXM * ORC_MAXM];
    diffusion_matrix(cfg, mc.phi, Dm);
    if (cfg->mutation == 10) { /* planted: omega = (D/cs2 + I)^-1 */
        double A[ORC_MAXM * ORC_MAXM];
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) A[a * m + b] = Dm[a * m + b] / cs2 + (a == b ? 1.0 : 0.0);
        if (!mat_inverse(m, A, omega)) return 0;
    } else if (!relaxation_matrix(m, Dm, cfg->lam, cfg->mutation == 12, omega)) {
        return 0;
    }
    if (cfg->mutation == 2) { /* planted: transposed relaxation matrix */
        double t[ORC_MAXM * ORC_MAXM];
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) t[a * m + b] = omega[b * m + a];
        memcpy(omega, t, sizeof(double) * m * m);
    }

    double S[ORC_MAXM];
    source_S(cfg, mc.phi, S);

    double feq[ORC_MAXM * 5], heq[9], Fi[9], Gi[ORC_MAXM * 5], Si[ORC_MAXM * 5], Si_old[ORC_MAXM * 5];
    double ueq[2] = {mc.u[0], mc.u[1]};
    if (cfg->mutation == 8) { ueq[0] = -ueq[0]; ueq[1] = -ueq[1]; }
    feq_node(m, cfg->lam, (cfg->mutation == 11) ? 1.0 : lam_norm(), mc.phi, ueq, feq);
    orc_heq(mc.p, mc.u, cfg->rho0, heq);
    orc_force_pop(mc.F, mc.u, (cfg->mutation == 14) ? 0.0 : cfg->varphi, Fi);
    if (cfg->model == 2) {
        /* Case 1: G_i = (I - omega/2) W_i c_i . u (phi - phi_prev) / (dt cs^2) */
        for (int a = 0; a < m; ++a) {
            double g[2] = {0.0, 0.0};
            for (int b = 0; b < m; ++b) {
                double cf = (a == b ? 1.0 : 0.0) - omega[a * m + b] / 2.0;
                double dphi = (mc.phi[b] - h[2 + b]) / dt;
                g[0] += cf * mc.u[0] * dphi;
                g[1] += cf * mc.u[1] * dphi;
            }
            for (int i = 0; i < 5; ++i) Gi[a * 5 + i] = W5x(i, e5[i][0] * g[0] + e5[i][1] * g[1]) / cs2;
        }
    } else {
        orc_aux_source(m, omega, mc.phi, S, mc.u, mc.F, Gi);
    }
    if (cfg->mutation == 1)
        for (int k = 0; k < m * 5; ++k) Gi[k] = 0.0;
    orc_source_pop(m, S, Si);
    orc_source_pop(m, Sold, Si_old);

    /* Eq. evolution12: (dt^2/2) Dbar_{ab} S_{i,b} with Dbar = delta d/dt + gamma c_i . grad:
     * d/dt S_i = (S_i(t) - S_i(t - dt))/dt and, gamma being diagonal,
     * gamma_a c_i . grad S_{i,a} = gamma_a W_i c_i . grad S_a (S_i = W_i S, Eq. source) */
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 5; ++i) {
            double coll = 0.0;
            for (int b = 0; b < m; ++b) coll += omega[a * m + b] * (f[b * 5 + i] - feq[b * 5 + i]);
            double dS = (cfg->mutation == 3) ? 0.0 : (Si[a * 5 + i] - Si_old[a * 5 + i]);
            double cgrad = e5[i][0] * gradS[a * 2] + e5[i][1] * gradS[a * 2 + 1];
            double gam = (cfg->mutation == 15) ? -cfg->gamma[a] : cfg->gamma[a];
            double dbar = dS / dt + gam * W5x(i, cgrad);
            fs[a * 5 + i] = f[a * 5 + i] - coll + dt * Si[a * 5 + i] + dt * Gi[a * 5 + i]
                            + (dt * dt / 2.0) * dbar;
        }
    for (int a = 0; a < m; ++a) Snew[a] = S[a];

    if (cfg->model == 2) { /* Case 1: no fluid; remember phi(t) for the next difference */
        for (int i = 0; i < 9; ++i) hs[i] = h[i];
        for (int a = 0; a < m; ++a) hs[2 + a] = mc.phi[a];
        return 1;
    }
    /* Eq. evolution3 (BGK), or its MRT counterpart */
    double w = 1.0 / cfg->tau_f;
    double fcoef = (cfg->mutation == 5) ? (1.0 + w / 2.0) : (1.0 - w / 2.0);
    if (cfg->collision == 0) {
        for (int i = 0; i < 9; ++i) hs[i] = h[i] - w * (h[i] - heq[i]) + dt * fcoef * Fi[i];
    } else {
        double s[9];
        for (int k = 0; k < 9; ++k) s[k] = cfg->mrt_s[k];
        s[7] = w; /* the stress moments carry the viscosity nu = (1/w - 1/2) cs2 dt */
        s[8] = w;
        double mneq[9], mF[9], mstar[9];
        for (int k = 0; k < 9; ++k) {
            double a1 = 0.0, a2 = 0.0;
            for (int i = 0; i < 9; ++i) {
                a1 += Mmrt[k][i] * (h[i] - heq[i]);
                a2 += Mmrt[k][i] * Fi[i];
            }
            mneq[k] = a1;
            mF[k] = a2;
        }
        for (int k = 0; k < 9; ++k) mstar[k] = -s[k] * mneq[k] + dt * (1.0 - s[k] / 2.0) * mF[k];
        for (int i = 0; i < 9; ++i) {
            double acc = 0.0;
            for (int k = 0; k < 9; ++k) acc += Minv[i][k] * mstar[k];
            hs[i] = h[i] + acc;
        }
    }
    return 1;
}

/* ---- geometry ------------------------------------------------------------ */
/* side crossed when leaving the domain along one axis: 0 x-, 1 x+, 2 y-, 3 y+ */
static int side_of(int axis, int coord, int n) {
    if (coord < 0) return axis == 0 ? 0 : 2;
    if (coord >= n) return axis == 0 ? 1 : 3;
    return -1;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

static size_t nidx(const orc_cfg *cfg, int x, int y) { return (size_t)y * cfg->nx + x; }

/* ---- public entry points --------------------------------------------------- */
/* layout: f[a][i][y][x] (m x 5 planes), h[i][y][x] (9 planes), Sold[a][y][x] */

int orc_init(const orc_cfg *cfg, const double *phi0, const double *u0, const double *p0,
             double *f, double *h, double *Sold) {
    int nx = cfg->nx, ny = cfg->ny, m = cfg->m;
    size_t N = (size_t)nx * ny;
    if (cfg->varphi != 0.0 && cfg->collision != 0) return 0; /* the p correction is BGK's */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = nidx(cfg, x, y);
            double phi[ORC_MAXM], u[2], feq[ORC_MAXM * 5], heq[9], S[ORC_MAXM];
            for (int a = 0; a < m; ++a) phi[a] = phi0[a * N + n];
            u[0] = u0[n];
            u[1] = u0[N + n];
            double p = p0 ? p0[n] : 0.0;
            feq_node(m, cfg->lam, lam_norm(), phi, u, feq);
            /* fluid: equilibrium at the momentum sum c_i h_i = u0 - (dt/2) F(phi0), so that
             * Eq. sum-u returns the prescribed u0 at t = 0 */
            double F[2], j[2];
            body_force(cfg, phi, F);
            j[0] = u[0] - dt / 2.0 * F[0];
            j[1] = u[1] - dt / 2.0 * F[1];
            orc_heq(p, j, cfg->rho0, heq);
            source_S(cfg, phi, S);
            for (int a = 0; a < m; ++a) {
                for (int i = 0; i < 5; ++i) f[(a * 5 + i) * N + n] = feq[a * 5 + i];
                Sold[a * N + n] = S[a];
            }
            for (int i = 0; i < 9; ++i) h[i * N + n] = heq[i];
            if (cfg->model == 2) { /* Case 1: prescribed velocity and phi(-dt) = phi0 */
                for (int i = 0; i < 9; ++i) h[i * N + n] = 0.0;
                h[0 * N + n] = u[0];
                h[1 * N + n] = u[1];
                for (int a = 0; a < m; ++a) h[(2 + a) * N + n] = phi[a];
            }
        }
    return 1;
}

/* destination of the post-collision fluid population i leaving (x, y):
 * returns the plane and node it lands in at t + dt */
static void fluid_dest(const orc_cfg *cfg, int x, int y, int i, int *plane, size_t *node) {
    int nx = cfg->nx, ny = cfg->ny;
    int tx = x + e9[i][0], ty = y + e9[i][1];
    int sx = side_of(0, tx, nx), sy = side_of(1, ty, ny);
    if (sx >= 0 && cfg->fluid_bc[sx] == 0) { tx = wrap(tx, nx); sx = -1; }
    if (sy >= 0 && cfg->fluid_bc[sy] == 0) { ty = wrap(ty, ny); sy = -1; }
    int opp = find_dir(e9, 9, -e9[i][0], -e9[i][1]);
    if (sx < 0 && sy < 0) { *plane = i; *node = nidx(cfg, tx, ty); return; }
    if (sx >= 0 && sy >= 0) { *plane = opp; *node = nidx(cfg, x, y); return; } /* corner link */
    int side = sx >= 0 ? sx : sy;
    if (cfg->fluid_bc[side] == 2 && cfg->mutation != 9) {
        /* specular reflection: the normal component flips, the tangential move is kept */
        int mx = e9[i][0], my = e9[i][1], rx = x, ry = y;
        if (sx >= 0) { mx = -mx; ry = y + e9[i][1]; } else { my = -my; rx = x + e9[i][0]; }
        int ssx = side_of(0, rx, nx), ssy = side_of(1, ry, ny);
        if (ssx >= 0 && cfg->fluid_bc[ssx] == 0) { rx = wrap(rx, nx); ssx = -1; }
        if (ssy >= 0 && cfg->fluid_bc[ssy] == 0) { ry = wrap(ry, ny); ssy = -1; }
        if (ssx < 0 && ssy < 0) {
            *plane = find_dir(e9, 9, mx, my);
            *node = nidx(cfg, rx, ry);
            return;
        }
    }
    *plane = opp; /* half-way bounce-back */
    *node = nidx(cfg, x, y);
}

int orc_step(const orc_cfg *cfg, double *f, double *h, double *Sold, int64_t nsteps) {
    int nx = cfg->nx, ny = cfg->ny, m = cfg->m;
    size_t N = (size_t)nx * ny;
    double *f2 = (double *)malloc(sizeof(double) * N * 5 * m);
    double *h2 = (double *)malloc(sizeof(double) * N * 9);
    if (!f2 || !h2) { free(f2); free(h2); return 0; }
    double M[81], Minvf[81], Minv[9][9];
    if (!orc_mrt_basis(M, Minvf)) { free(f2); free(h2); return 0; }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) Minv[r][c] = Minvf[r * 9 + c];
    /* the previous step's source field S(x, t - dt), read at the neighbours
     * by the gamma term (Sold itself is overwritten node by node) */
    double *Sprev = (double *)malloc(sizeof(double) * N * m);
    if (!Sprev) { free(f2); free(h2); return 0; }
    int ok = 1;
    for (int64_t s = 0; s < nsteps && ok; ++s) {
        memcpy(Sprev, Sold, sizeof(double) * N * m);
#pragma omp parallel for schedule(static) reduction(&& : ok)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = nidx(cfg, x, y);
                double fl[ORC_MAXM * 5], hl[9], so[ORC_MAXM], fs[ORC_MAXM * 5], hs[9], sn[ORC_MAXM];
                double gs[ORC_MAXM * 2];
                for (int a = 0; a < m; ++a) {
                    for (int i = 0; i < 5; ++i) fl[a * 5 + i] = f[(a * 5 + i) * N + n];
                    so[a] = Sold[a * N + n];
                    /* central differences; a wall side takes the node's own value */
                    for (int d = 0; d < 2; ++d) {
                        int len = d == 0 ? nx : ny, c = d == 0 ? x : y;
                        int wall_lo = d == 0 ? cfg->scalar_bc[0][a] != 0 : cfg->scalar_bc[2][a] != 0;
                        int wall_hi = d == 0 ? cfg->scalar_bc[1][a] != 0 : cfg->scalar_bc[3][a] != 0;
                        int cp = c + 1, cm = c - 1;
                        if (cp >= len) cp = wall_hi ? c : 0;
                        if (cm < 0) cm = wall_lo ? c : len - 1;
                        size_t np_ = d == 0 ? nidx(cfg, cp, y) : nidx(cfg, x, cp);
                        size_t nm_ = d == 0 ? nidx(cfg, cm, y) : nidx(cfg, x, cm);
                        gs[a * 2 + d] = (Sprev[a * N + np_] - Sprev[a * N + nm_]) / 2.0;
                    }
                }
                for (int i = 0; i < 9; ++i) hl[i] = h[i * N + n];
                if (!collide_node(cfg, Minv, fl, hl, so, gs, fs, hs, sn)) ok = 0;
                for (int a = 0; a < m; ++a) Sold[a * N + n] = sn[a];
                /* fluid streaming (Case 1: the per-node values stay in place) */
                if (cfg->model == 2) {
                    for (int i = 0; i < 9; ++i) h2[i * N + n] = hs[i];
                } else {
                    for (int i = 0; i < 9; ++i) {
                        int pl;
                        size_t dn;
                        fluid_dest(cfg, x, y, i, &pl, &dn);
                        h2[pl * N + dn] = hs[i];
                    }
                }
                /* scalar streaming: D2Q5 links cross at most one wall */
                for (int a = 0; a < m; ++a)
                    for (int i = 0; i < 5; ++i) {
                        int tx = x + e5[i][0], ty = y + e5[i][1];
                        int sx = side_of(0, tx, nx), sy = side_of(1, ty, ny);
                        int side = sx >= 0 ? sx : sy;
                        double v = fs[a * 5 + i];
                        if (side < 0 || cfg->scalar_bc[side][a] == 0) {
                            tx = wrap(tx, nx);
                            ty = wrap(ty, ny);
                            f2[(a * 5 + i) * N + nidx(cfg, tx, ty)] = v;
                            continue;
                        }
                        int opp = find_dir(e5, 5, -e5[i][0], -e5[i][1]);
                        if (cfg->scalar_bc[side][a] == 1) {
                            f2[(a * 5 + opp) * N + n] = v; /* half-way bounce-back: no flux */
                        } else {
                            /* anti-bounce-back (Dirichlet phi_w at the half-way wall) */
                            double sgn = (cfg->mutation == 7) ? 1.0 : -1.0;
                            f2[(a * 5 + opp) * N + n] = sgn * v + 2.0 * W5x(i, cfg->wall[side * ORC_MAXM + a]);
                        }
                    }
            }
        memcpy(f, f2, sizeof(double) * N * 5 * m);
        memcpy(h, h2, sizeof(double) * N * 9);
    }
    free(Sprev);
    free(f2);
    free(h2);
    return ok;
}

/* macroscopic fields phi[a][y][x], u[2][y][x], p[y][x] (Eq. sum) */
int orc_moments(const orc_cfg *cfg, const double *f, const double *h, double *phi, double *u,
                double *p) {
    int m = cfg->m;
    size_t N = (size_t)cfg->nx * cfg->ny;
    for (size_t n = 0; n < N; ++n) {
        double fl[ORC_MAXM * 5], hl[9];
        for (int a = 0; a < m; ++a)
            for (int i = 0; i < 5; ++i) fl[a * 5 + i] = f[(a * 5 + i) * N + n];
        for (int i = 0; i < 9; ++i) hl[i] = h[i * N + n];
        node_macro mc;
        node_moments(cfg, fl, hl, &mc);
        for (int a = 0; a < m; ++a) phi[a * N + n] = mc.phi[a];
        u[n] = mc.u[0];
        u[N + n] = mc.u[1];
        p[n] = mc.p;
    }
    return 1;
}

/* number of threads the parallel step loop uses (for the CPU baseline record) */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sets the number of threads of the parallel step loop (n > 0); results do
   not depend on it: every node's update is independent of the others */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

size_t orc_cfg_size(void) { return sizeof(orc_cfg); }

/* the chemotaxis cut-off r(c) of the record (for pin tests) */
double orc_cutoff(const orc_cfg *cfg, double c) { return cutoff_r(cfg, c); }
