/*
 * lb3_oracle.c -- plain FP64 CPU oracle for the three-dimensional form of the
 * coupled cross-diffusion-fluid lattice Boltzmann model of Zhan, Chai & Shi
 * (arXiv 2101.03055): one D3Q7 lattice per scalar and a D3Q19 lattice for the
 * fluid, with the lattice tables of Sec. 2.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or helper with the GPU library (nor with the 2-D
 * oracle); the two are compared on the same seeded inputs.
 *
 * Per node, in the order of Sec. 2: scalar moments (Eq. sum-phi) -> body force
 * -> fluid velocity (Eq. sum-u) -> pressure (Eq. sum-p, varphi = 0) -> relaxation
 * matrix from Eq. omega-D -> source -> equilibria (Eqs. feq-phi, heq) ->
 * discrete source (Eq. source), auxiliary source (Eq. Gi) and discrete force
 * (Eq. force) -> evolution (Eqs. evolution12, evolution3) -> push streaming with
 * the wall rules, into a second array.
 *
 * Lattice units: dx = dt = 1.  The two lattices have different sound speeds:
 * cs^2 = 1/4 on D3Q7 (its table in Sec. 2) and 1/3 on D3Q19, and every
 * formula uses the sound speed of its own lattice, so Eq. omega-D reads
 * omega = (D / cs7^2 + I/2)^-1 = (4 D + I/2)^-1 here.
 * Readings (as in two dimensions): lambda = I, vartheta = 0, varphi = 0,
 * gamma = 0 with the first-order difference for d/dt S and S_old(t = 0) =
 * S(phi0); half-way walls; initial scalar equilibrium of (phi0, u0) and fluid
 * equilibrium of (p0, u0 - F(phi0)/2); a D3Q19 link that leaves through one or
 * two walls (an edge) bounces back; D3Q7 links cross at most one wall.
 * Fluid sides are periodic or no-slip; scalar sides periodic, no-flux
 * (bounce-back) or Dirichlet (anti-bounce-back f_opp = -f*_i + 2 W_i phi_w).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O3_MAXM 4

typedef struct orc3_cfg {
    int32_t nx, ny, nz, m;
    int32_t mutation;                 /* 0 = faithful; k > 0 plants mistake k (pin self-test only) */
    int32_t fluid_bc[6];              /* sides x-, x+, y-, y+, z-, z+: 0 periodic, 1 no-slip */
    int32_t scalar_bc[6][O3_MAXM];    /* 0 periodic, 1 no-flux, 2 Dirichlet */
    int32_t pad_;
    double tau_f, rho0;
    double D[O3_MAXM * O3_MAXM];      /* constant diffusion matrix, row-major */
    double K[O3_MAXM * O3_MAXM];      /* linear source S = K phi */
    double F0[3];                     /* constant body force */
    double Fphi[O3_MAXM * 3];         /* F += Fphi[alpha] * phi_alpha */
    double wall[6 * O3_MAXM];         /* Dirichlet values [side][alpha] */
} orc3_cfg;

/* ---- lattices, in the column order of the Sec. 2 tables ------------------ */
static const int e7[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
static const double W7num[7] = {2, 1, 1, 1, 1, 1, 1};
static const double W7den[7] = {8, 8, 8, 8, 8, 8, 8};
static const int e19[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
                               {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19num[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
static const double W19den[19] = {36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36, 36};
static double W7x(int i, double x) { return x * W7num[i] / W7den[i]; }
static double W19x(int i, double x) { return x * W19num[i] / W19den[i]; }
static const double cs2_7 = 0.25;       /* D3Q7 */
static const double cs2_19 = 1.0 / 3.0; /* D3Q19 */

static int find_dir(const int (*e)[3], int q, int cx, int cy, int cz) {
    for (int i = 0; i < q; ++i)
        if (e[i][0] == cx && e[i][1] == cy && e[i][2] == cz) return i;
    return -1;
}

/* Gauss-Jordan inverse with partial pivoting; 0 if singular */
static int inverse(int n, const double *a, double *ainv) {
    double w[O3_MAXM][2 * O3_MAXM];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c) w[r][c] = (c < n) ? a[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(w[r][k]) > fabs(w[piv][k])) piv = r;
        if (w[piv][k] == 0.0) return 0;
        for (int c = 0; c < 2 * n; ++c) {
            double t = w[k][c];
            w[k][c] = w[piv][c];
            w[piv][c] = t;
        }
        double d = w[k][k];
        for (int c = 0; c < 2 * n; ++c) w[k][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            double s = w[r][k];
            for (int c = 0; c < 2 * n; ++c) w[r][c] -= s * w[k][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) ainv[r * n + c] = w[r][n + c];
    return 1;
}

/* Eq. omega-D with lambda = I on D3Q7: omega = (D / (cs7^2 dt) + I/2)^-1.
 * mutation 2 plants the D2Q5/D3Q19 sound speed 1/3 instead of 1/4. */
static int relaxation(const orc3_cfg *cfg, double *omega) {
    int m = cfg->m;
    double cs2 = (cfg->mutation == 2) ? 1.0 / 3.0 : cs2_7;
    double A[O3_MAXM * O3_MAXM];
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) A[a * m + b] = cfg->D[a * m + b] / cs2 + (a == b ? 0.5 : 0.0);
    return inverse(m, A, omega);
}

/* ---- equilibria, force and sources (exported for the single-node pins) -- */
/* Eq. feq-phi on D3Q7 (lambda = I, vartheta = 0): W_i [phi + c_i.phi u / cs7^2] */
void orc3_feq(int m, const double *phi, const double *u, double *feq /*[m][7]*/) {
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 7; ++i) {
            double cu = e7[i][0] * u[0] + e7[i][1] * u[1] + e7[i][2] * u[2];
            feq[a * 7 + i] = W7x(i, phi[a] + phi[a] * cu / cs2_7);
        }
}

/* Eq. heq on D3Q19: sigma_0 = (W_0 - 1) p / cs^2 + rho0, sigma_i = W_i p / cs^2 */
void orc3_heq(double p, const double *u, double rho0, double *heq /*[19]*/) {
    for (int i = 0; i < 19; ++i) {
        double sigma = (i == 0) ? (W19x(0, p) - p) / cs2_19 + rho0 : W19x(i, p) / cs2_19;
        double cu = e19[i][0] * u[0] + e19[i][1] * u[1] + e19[i][2] * u[2];
        double uu_cc = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) uu_cc += u[r] * u[s] * (e19[i][r] * e19[i][s] - (r == s ? cs2_19 : 0.0));
        heq[i] = sigma + W19x(i, cu / cs2_19 + uu_cc / (2.0 * cs2_19 * cs2_19));
    }
}

/* Eq. force with varphi = 0: F_i = W_i c_i.F / cs^2 (mutation 3 drops the 1/cs^2) */
static void force_pop(const orc3_cfg *cfg, const double *F, double *Fi) {
    double k = (cfg && cfg->mutation == 3) ? 1.0 : 1.0 / cs2_19;
    for (int i = 0; i < 19; ++i) Fi[i] = W19x(i, e19[i][0] * F[0] + e19[i][1] * F[1] + e19[i][2] * F[2]) * k;
}
void orc3_force_pop(const double *F, double *Fi /*[19]*/) { force_pop(NULL, F, Fi); }

/* Eq. Gi: G_{i,a} = sum_b (delta_ab - omega_ab/2) W_i c_i.(u S_b + phi_b F) / cs7^2 */
void orc3_aux_source(int m, const double *omega, const double *phi, const double *S, const double *u,
                     const double *F, double *G /*[m][7]*/) {
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 7; ++i) {
            double g = 0.0;
            for (int b = 0; b < m; ++b) {
                double coef = (a == b ? 1.0 : 0.0) - 0.5 * omega[a * m + b];
                double cv = 0.0;
                for (int d = 0; d < 3; ++d) cv += e7[i][d] * (u[d] * S[b] + phi[b] * F[d]);
                g += coef * W7x(i, cv) / cs2_7;
            }
            G[a * 7 + i] = g;
        }
}

int orc3_relaxation_matrix(int m, const double *Dm, double *omega) {
    orc3_cfg c;
    memset(&c, 0, sizeof c);
    c.m = m;
    memcpy(c.D, Dm, sizeof(double) * m * m);
    return relaxation(&c, omega);
}

/* ---- one node ------------------------------------------------------------- */
typedef struct macro3 {
    double phi[O3_MAXM], F[3], u[3], p;
} macro3;

static void node_moments(const orc3_cfg *cfg, const double *f, const double *h, macro3 *mc) {
    int m = cfg->m;
    for (int a = 0; a < m; ++a) {
        mc->phi[a] = 0.0;
        for (int i = 0; i < 7; ++i) mc->phi[a] += f[a * 7 + i];
    }
    for (int d = 0; d < 3; ++d) {
        mc->F[d] = cfg->F0[d];
        for (int a = 0; a < m; ++a) mc->F[d] += cfg->Fphi[3 * a + d] * mc->phi[a];
    }
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int i = 0; i < 19; ++i) s += e19[i][d] * h[i];
        mc->u[d] = s + 0.5 * mc->F[d];
    }
    /* Eq. sum-p (varphi = 0): p = cs^2/(1 - W_0) [sum_{i>0} h_i - W_0 u.u/(2 cs^2)] */
    double s = 0.0;
    for (int i = 1; i < 19; ++i) s += h[i];
    double uu = mc->u[0] * mc->u[0] + mc->u[1] * mc->u[1] + mc->u[2] * mc->u[2];
    mc->p = cs2_19 * W19den[0] / (W19den[0] - W19num[0]) * (s - W19x(0, uu) / (2.0 * cs2_19));
}

static int collide(const orc3_cfg *cfg, const double *f, const double *h, const double *Sold, double *fs,
                   double *hs, double *Snew) {
    int m = cfg->m;
    macro3 mc;
    node_moments(cfg, f, h, &mc);
    double omega[O3_MAXM * O3_MAXM];
    if (!relaxation(cfg, omega)) return 0;
    double S[O3_MAXM];
    for (int a = 0; a < m; ++a) {
        S[a] = 0.0;
        for (int b = 0; b < m; ++b) S[a] += cfg->K[a * m + b] * mc.phi[b];
    }
    double feq[O3_MAXM * 7], G[O3_MAXM * 7], heq[19], Fi[19];
    orc3_feq(m, mc.phi, mc.u, feq);
    orc3_aux_source(m, omega, mc.phi, S, mc.u, mc.F, G);
    if (cfg->mutation == 1)
        for (int k = 0; k < m * 7; ++k) G[k] = 0.0;
    orc3_heq(mc.p, mc.u, cfg->rho0, heq);
    force_pop(cfg, mc.F, Fi);
    /* Eq. evolution12, gamma = 0: + dt S_i + (dt/2)(S_i(t) - S_i(t - dt)) + dt G_i */
    for (int a = 0; a < m; ++a)
        for (int i = 0; i < 7; ++i) {
            double coll = 0.0;
            for (int b = 0; b < m; ++b) coll += omega[a * m + b] * (f[b * 7 + i] - feq[b * 7 + i]);
            double Si = W7x(i, S[a]), Si_old = W7x(i, Sold[a]);
            fs[a * 7 + i] = f[a * 7 + i] - coll + Si + G[a * 7 + i] + 0.5 * (Si - Si_old);
        }
    for (int a = 0; a < m; ++a) Snew[a] = S[a];
    /* Eq. evolution3 (BGK) */
    double w = 1.0 / cfg->tau_f;
    for (int i = 0; i < 19; ++i) hs[i] = h[i] - w * (h[i] - heq[i]) + (1.0 - w / 2.0) * Fi[i];
    return 1;
}

/* ---- geometry ------------------------------------------------------------- */
static int wrap(int v, int n) { return ((v % n) + n) % n; }
static size_t nid(const orc3_cfg *cfg, int x, int y, int z) {
    return ((size_t)z * cfg->ny + y) * cfg->nx + x;
}
/* side crossed by coordinate c on axis d (0 x, 1 y, 2 z), -1 if inside */
static int side_of(int d, int c, int n) { return c < 0 ? 2 * d : (c >= n ? 2 * d + 1 : -1); }

/* ---- entry points ---------------------------------------------------------- */
/* layout: f[a][i][z][y][x] (7m planes), h[i][z][y][x] (19), Sold[a][z][y][x] */
int orc3_init(const orc3_cfg *cfg, const double *phi0, const double *u0, const double *p0, double *f, double *h,
              double *Sold) {
    int m = cfg->m;
    size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
    for (size_t n = 0; n < N; ++n) {
        double phi[O3_MAXM], u[3], feq[O3_MAXM * 7], heq[19], F[3], j[3];
        for (int a = 0; a < m; ++a) phi[a] = phi0[a * N + n];
        for (int d = 0; d < 3; ++d) u[d] = u0[d * N + n];
        orc3_feq(m, phi, u, feq);
        for (int d = 0; d < 3; ++d) {
            F[d] = cfg->F0[d];
            for (int a = 0; a < m; ++a) F[d] += cfg->Fphi[3 * a + d] * phi[a];
            j[d] = u[d] - 0.5 * F[d];
        }
        orc3_heq(p0 ? p0[n] : 0.0, j, cfg->rho0, heq);
        for (int a = 0; a < m; ++a) {
            for (int i = 0; i < 7; ++i) f[(a * 7 + i) * N + n] = feq[a * 7 + i];
            double s = 0.0;
            for (int b = 0; b < m; ++b) s += cfg->K[a * m + b] * phi[b];
            Sold[a * N + n] = s;
        }
        for (int i = 0; i < 19; ++i) h[i * N + n] = heq[i];
    }
    return 1;
}

int orc3_step(const orc3_cfg *cfg, double *f, double *h, double *Sold, int64_t nsteps) {
    int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, m = cfg->m;
    int dims[3] = {nx, ny, nz};
    size_t N = (size_t)nx * ny * nz;
    double *f2 = (double *)malloc(sizeof(double) * N * 7 * m);
    double *h2 = (double *)malloc(sizeof(double) * N * 19);
    if (!f2 || !h2) {
        free(f2);
        free(h2);
        return 0;
    }
    int ok = 1;
    for (int64_t s = 0; s < nsteps && ok; ++s) {
#pragma omp parallel for schedule(static) reduction(&& : ok)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t n = nid(cfg, x, y, z);
                    int pos[3] = {x, y, z};
                    double fl[O3_MAXM * 7], hl[19], so[O3_MAXM], fs[O3_MAXM * 7], hs[19], sn[O3_MAXM];
                    for (int a = 0; a < m; ++a) {
                        for (int i = 0; i < 7; ++i) fl[a * 7 + i] = f[(a * 7 + i) * N + n];
                        so[a] = Sold[a * N + n];
                    }
                    for (int i = 0; i < 19; ++i) hl[i] = h[i * N + n];
                    if (!collide(cfg, fl, hl, so, fs, hs, sn)) ok = 0;
                    for (int a = 0; a < m; ++a) Sold[a * N + n] = sn[a];
                    /* fluid: stream, or bounce back when any wall is crossed (edges too) */
                    for (int i = 0; i < 19; ++i) {
                        int t[3], walled = 0;
                        for (int d = 0; d < 3; ++d) {
                            t[d] = pos[d] + e19[i][d];
                            int sd = side_of(d, t[d], dims[d]);
                            if (sd < 0) continue;
                            if (cfg->fluid_bc[sd] == 0)
                                t[d] = wrap(t[d], dims[d]);
                            else
                                walled = 1;
                        }
                        if (walled && cfg->mutation != 4) {
                            int opp = find_dir(e19, 19, -e19[i][0], -e19[i][1], -e19[i][2]);
                            h2[opp * N + n] = hs[i];
                        } else {
                            for (int d = 0; d < 3; ++d) t[d] = wrap(t[d], dims[d]);
                            h2[i * N + nid(cfg, t[0], t[1], t[2])] = hs[i];
                        }
                    }
                    /* scalars: D3Q7 links cross at most one wall */
                    for (int a = 0; a < m; ++a)
                        for (int i = 0; i < 7; ++i) {
                            int t[3], side = -1;
                            for (int d = 0; d < 3; ++d) {
                                t[d] = pos[d] + e7[i][d];
                                int sd = side_of(d, t[d], dims[d]);
                                if (sd >= 0 && cfg->scalar_bc[sd][a] != 0) side = sd;
                                t[d] = wrap(t[d], dims[d]);
                            }
                            double v = fs[a * 7 + i];
                            if (side < 0) {
                                f2[(a * 7 + i) * N + nid(cfg, t[0], t[1], t[2])] = v;
                                continue;
                            }
                            int opp = find_dir(e7, 7, -e7[i][0], -e7[i][1], -e7[i][2]);
                            if (cfg->scalar_bc[side][a] == 1)
                                f2[(a * 7 + opp) * N + n] = v;
                            else
                                f2[(a * 7 + opp) * N + n] = -v + 2.0 * W7x(i, cfg->wall[side * O3_MAXM + a]);
                        }
                }
        memcpy(f, f2, sizeof(double) * N * 7 * m);
        memcpy(h, h2, sizeof(double) * N * 19);
    }
    free(f2);
    free(h2);
    return ok;
}

int orc3_moments(const orc3_cfg *cfg, const double *f, const double *h, double *phi, double *u, double *p) {
    int m = cfg->m;
    size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
    for (size_t n = 0; n < N; ++n) {
        double fl[O3_MAXM * 7], hl[19];
        for (int a = 0; a < m; ++a)
            for (int i = 0; i < 7; ++i) fl[a * 7 + i] = f[(a * 7 + i) * N + n];
        for (int i = 0; i < 19; ++i) hl[i] = h[i * N + n];
        macro3 mc;
        node_moments(cfg, fl, hl, &mc);
        for (int a = 0; a < m; ++a) phi[a * N + n] = mc.phi[a];
        for (int d = 0; d < 3; ++d) u[d * N + n] = mc.u[d];
        p[n] = mc.p;
    }
    return 1;
}

size_t orc3_cfg_size(void) { return sizeof(orc3_cfg); }
