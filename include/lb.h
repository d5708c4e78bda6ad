/*
 * lb.h -- C ABI of the MI355X (gfx950) library for the lattice Boltzmann model
 * of the coupled cross-diffusion-fluid system (Zhan, Chai & Shi, arXiv
 * 2101.03055).
 *
 * Problem (Sec. 1, Eq. CDF): m scalars phi_a (a = 1..m, m <= 4) transported by
 * an incompressible flow u,
 *     d_t phi_a + div(phi_a u) = div(D_ab grad phi_b) + S_a,
 *     div u = 0,   d_t u + div(uu) = -grad p + div(nu grad u) + F,
 * solved with one D2Q5 lattice per scalar and one D2Q9 fluid lattice
 * (Sec. 2, Eqs. evolution12 and evolution3).  The scalar collision is the
 * matrix relaxation omega_ab = (D/(cs^2 dt) + I/2)^-1 (Eq. omega-D with
 * lambda = I), whose off-diagonal entries carry the cross-diffusion; the
 * auxiliary source G of Eq. Gi cancels the numerical diffusion of convection;
 * the source carries its time-derivative correction (Eq. source; the gamma
 * part of D-bar is a parameter, 0 by default as in the paper's runs);
 * the fluid is BGK (Eq. evolution3) with the force term of Eq. force
 * (varphi = 0) and the pressure scheme of appendix A, or MRT.
 *
 * Units: lattice units, dx = dt = 1, cs^2 = 1/3.
 * Grid: nx * ny nodes, node (x, y) at the cell centre; walls are half-way
 * between the last node and the next (Sec. 3: half-way bounce-back).
 * Sides: 0 = x-, 1 = x+, 2 = y-, 3 = y+.
 *
 * Host arrays are row-major, x fastest:
 *   phi[a][y][x] (m planes), u[d][y][x] (2 planes), p[y][x],
 *   f[a][i][y][x] (m*5 planes, D2Q5 order 0,(1,0),(0,1),(-1,0),(0,-1)),
 *   h[i][y][x]    (9 planes, D2Q9 order 0,(1,0),(0,1),(-1,0),(0,-1),
 *                  (1,1),(-1,1),(-1,-1),(1,-1)).
 *
 * Ownership: the caller owns the device workspace (any device allocation of
 * at least lb_workspace_bytes() bytes, 256-byte aligned) and every host
 * array.  The handle holds no other device memory; lb_free() releases the
 * handle only, never the workspace.  All work is enqueued on the stream given
 * to lb_init (a hipStream_t, NULL for the default stream).
 *
 * Errors: every call returns an lb_status; nothing throws or aborts across
 * the ABI.  lb_last_error() returns a thread-local description of the last
 * failure on the calling thread.
 */
#ifndef LBCDF_LB_H
#define LBCDF_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_MAX_M 4

typedef enum lb_status {
    LB_OK = 0,
    LB_EINVAL = -1,      /* invalid argument or parameter set */
    LB_ENOMEM = -2,      /* workspace too small or host allocation failed */
    LB_EDEVICE = -3,     /* a HIP call failed */
    LB_ENONFINITE = -4,  /* a non-finite value was found (inputs or fields) */
    LB_ESTATE = -5       /* call not valid in the handle's current state */
} lb_status;

/* closures */
enum { LB_MODEL_LINEAR = 0,      /* D constant, S = K phi, F = F0 + sum_a Fphi[a] phi_a  (DDC, Sec. 3.2) */
       LB_MODEL_CHEMOTAXIS = 1,  /* m = 2, (n, c): D = [[D00, D01 - chi r(c) n], [D10, D11]],
                                    S = (0, -beta r(c) n), F = F0 + sum_a Fphi[a] phi_a  (Sec. 3.1) */
       LB_MODEL_CDE = 2 };       /* Case 1 of Sec. 2, no fluid: the convection cross-diffusion equation
                                    with a prescribed velocity (u0 of lb_init, constant in time); D
                                    constant, S = K phi, no force (F0, Fphi must be 0).  The auxiliary
                                    source uses d_t(phi u) = u (phi(t) - phi(t - dt)) / dt, phi(-dt) =
                                    phi0.  Storage F64 or F32, BGK only, one step per launch, not in
                                    batches; lb_moments returns the prescribed u and p = 0, lb_mass
                                    returns 0 for the fluid sum, lb_populations fills h with 0;
                                    lb_wall_flux and lb_copy_state are not available. */
/* population storage in device memory */
enum { LB_STORE_F64 = 0,         /* raw populations, FP64 arithmetic */
       LB_STORE_F32 = 1,         /* deviations f - W_i phi_ref, h - rho0 delta_i0 in FP32, FP32 arithmetic;
                                    each species' rest population takes the FP64 remainder of its
                                    post-collision mass (no systematic drift of the scalar totals) */
       LB_STORE_F16 = 2 };       /* the same deviations times fp16_scale in binary16, stochastically
                                    rounded (reproducible counter-based dither), FP32 arithmetic */
/* fluid collision */
enum { LB_COLL_BGK = 0, LB_COLL_MRT = 1 };
/* chemotaxis cut-off r(c) */
enum { LB_R_STEP = 0,            /* r = 1 if c >= cstar else 0 (Sec. 3.1.3) */
       LB_R_SMOOTH = 1 };        /* r = (1 + (c - cstar)/sqrt((c - cstar)^2 + eps^2))/2 (Sec. 3.1.2) */
/* fluid boundary per side */
enum { LB_BC_PERIODIC = 0, LB_BC_NOSLIP = 1 /* half-way bounce-back */, LB_BC_FREESLIP = 2 /* specular */ };
/* scalar boundary per side and species */
enum { LB_SBC_PERIODIC = 0, LB_SBC_NOFLUX = 1 /* half-way bounce-back */,
       LB_SBC_DIRICHLET = 2 /* anti-bounce-back, value wall[side][a] */ };

typedef struct lb_params {
    int32_t nx, ny;              /* grid, each >= 2, nx ny < 2^31 and (nx + 64)(9 + 5m) < 2^31
                                    (LB_EINVAL otherwise) */
    int32_t m;                   /* number of scalars, 1..4 (2 for the chemotaxis model) */
    int32_t model;               /* LB_MODEL_* */
    int32_t storage;             /* LB_STORE_* */
    int32_t collision;           /* LB_COLL_* */
    int32_t r_kind;              /* LB_R_* */
    int32_t fluid_bc[4];         /* LB_BC_* per side; periodic only in pairs (0,1) / (2,3) */
    int32_t scalar_bc[4][LB_MAX_M]; /* LB_SBC_* per side and species; periodic must match the fluid */
    int32_t fused_steps;         /* 0 or 1: one AA-pattern launch per step (single population array);
                                    2: two steps per launch, temporally blocked through LDS (two
                                    population arrays: twice the population memory, half the HBM
                                    traffic per step) */
    double tau_f;                /* fluid relaxation time (> 1/2); nu = (tau_f - 1/2)/3 */
    double rho0;                 /* constant of the fluid equilibrium (Eq. heq) */
    double mrt_s[9];             /* MRT rates, moment order rho,e,eps,jx,qx,jy,qy,pxx,pxy;
                                    the stress rates (7, 8) are replaced by 1/tau_f */
    double D[LB_MAX_M * LB_MAX_M]; /* diffusion matrix, row-major m x m (constant part) */
    double K[LB_MAX_M * LB_MAX_M]; /* linear source matrix (LINEAR model), row-major m x m */
    double F0[2];                /* constant body force */
    double Fphi[LB_MAX_M][2];    /* buoyancy coefficients: F += Fphi[a] * phi_a */
    double chi, beta, cstar, eps;/* chemotaxis closure coefficients (lattice units) */
    double wall[4][LB_MAX_M];    /* Dirichlet wall values [side][species] */
    double phi_ref[LB_MAX_M];    /* reference level subtracted in reduced-precision storage */
    double fp16_scale;           /* multiplier of the scalar deviations in LB_STORE_F16 (> 0) */
    double fp16_scale_h;         /* multiplier of the fluid deviations in LB_STORE_F16 (> 0) */
    double lam[LB_MAX_M * LB_MAX_M]; /* lambda of Eq. feq-phi, row-major m x m; all zeros means the
                                    identity (Sec. 3).  With lambda != I the relaxation matrix is
                                    omega = (3 D lambda^-1 + I/2)^-1 (Eq. omega-D) and the D2Q5
                                    equilibrium gains (lambda phi - phi)_a x (-2/3, 1/6, 1/6, 1/6, 1/6):
                                    the lambda part of Eq. feq-phi scaled so that its second moment
                                    is cs^2 (lambda phi - phi) I (Sec. 2.1), twice the printed
                                    D2Q9 form.  LINEAR and CDE models only; the eigenvalues of lambda
                                    need real parts in (0, 3/2) (positive rest weight) and those of
                                    D lambda^-1 positive real parts */
    double varphi;               /* varphi of Eq. force (0 in Sec. 3): F_i gains
                                    varphi W_i (uF + Fu):(c_i c_i - cs^2 I)/(2 cs^4) and the pressure
                                    dt (1/omega - 1/2) F_0 inside the bracket of appendix A.  BGK only;
                                    not for the no-fluid model */
    double gamma_s[LB_MAX_M];    /* diagonal of gamma in D-bar = delta d/dt + gamma c_i . grad of
                                    Eq. evolution12 (0 in Sec. 3): the step adds (1/2) gamma_a W_i c_i .
                                    grad S_a, grad S_a by central differences of the previous step's
                                    source field (S(x +- e_d, t - dt); across a wall the node's own
                                    value).  Non-zero values need the linear or chemotaxis model,
                                    one step per launch, and no batch */
} lb_params;

typedef struct lb_handle lb_handle;

/* Bytes of device workspace lb_init needs for these parameters.
 * Layout (documented for debugging only; opaque to callers): populations as
 * 9 + 5m planes [plane][ny][nx] of the storage type, the previous-step source
 * planes, the residual snapshot, a staging area and the reduction scratch. */
lb_status lb_workspace_bytes(const lb_params* params, size_t* bytes);

/* Validates the parameters (tau_f > 1/2, Re(eig D) > 0 so that eig(omega) lies in
 * (0, 2), m range, boundary codes, finite inputs), then initialises
 * f = f^eq(phi0, u0), h = h^eq(p0, u0 - F(phi0)/2) and S_old = S(phi0) at t = 0, so
 * that the velocity of Eq. sum-u is the prescribed u0 (reading of the paper: it
 * does not state the initial populations).  phi0: host [m][ny][nx];
 * u0: host [2][ny][nx]; p0: host [ny][nx] or NULL (p0 = 0).  Synchronises the
 * stream before returning.  *out receives a new handle. */
lb_status lb_init(const lb_params* params, void* dev_workspace, size_t workspace_bytes,
                  void* hip_stream, const double* phi0, const double* u0, const double* p0,
                  lb_handle** out);

/* Advances n >= 0 time steps (Eqs. evolution12 and evolution3 with the boundary
 * rules of Sec. 3), asynchronously on the handle's stream.  Any n, odd or even. */
lb_status lb_step(lb_handle* h, int64_t n);

/* Macroscopic fields at the current time (Eq. sum): phi [m][ny][nx], u [2][ny][nx]
 * (u = sum_i c_i h_i + F/2), p [ny][nx] (appendix A, with the varphi term).  Host arrays;
 * any may be NULL.  Synchronises the stream. */
lb_status lb_moments(lb_handle* h, double* phi, double* u, double* p);

/* Same fields written to caller-owned DEVICE buffers (FP64, same layouts),
 * asynchronously on the handle's stream; any may be NULL. */
lb_status lb_moments_device(lb_handle* h, double* d_phi, double* d_u, double* d_p);

/* Steady-state residual since the previous call (reading of the criterion of
 * Sec. 3.1.1 with absolute values): res[q] = sum|q - q_prev| / sum|q| for
 * q = u_x, u_y, phi_1..phi_m (m + 2 values); res[q] = 0 when both sums vanish.
 * The first call after lb_init/lb_load stores the snapshot and returns +inf.
 * Returns LB_ENONFINITE (with res filled) if any field is not finite.
 * Synchronises the stream. */
lb_status lb_residual(lb_handle* h, double* res);

/* lb_residual for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid it):
 * the same kernels, result and error behaviour, but the reduction's partial
 * records and result record live in a library-held device array of fixed size
 * (128.5 KiB: 1024 partial records of 16 doubles plus 64 doubles) instead of
 * the handle's workspace.  Allocates nothing; grids of any size fit (the first
 * pass uses at most 1024 workgroups), a larger request would return LB_EINVAL.
 * Each GPU holds one copy of the array until the process ends, shared by every
 * call on that GPU and keeping the last call's contents (every value a call
 * reads it first writes).  Calls through this entry point on one GPU are
 * serialised by a host lock held until the call's stream has finished with the
 * array; work that wrote the array concurrently (another process has its own
 * copy) would race.  Synchronises the stream. */
lb_status lb_residual_noalloc(lb_handle* h, double* res);

/* Steady solve: repeats { lb_step(check_every); lb_residual } until every
 * residual component is below tol (criterion of Sec. 3.1.1, absolute values),
 * or max_steps steps have been taken, or a field turns non-finite.
 * *steps_out = steps taken by this call; res_out[m + 2] = last residual (may be
 * NULL).  Returns LB_OK when converged, LB_ESTATE when max_steps was reached
 * first, LB_ENONFINITE on divergence. */
lb_status lb_solve_steady(lb_handle* h, double tol, int64_t check_every, int64_t max_steps,
                          int64_t* steps_out, double* res_out);

/* Mean inward diffusive flux of every species through a Dirichlet wall:
 * flux[a] = -(1/D_aa) sum_b D_ab dphi_b/dn averaged along the wall, with the
 * normal derivative per unit cavity length (lattice spacing x nodes across the
 * cavity) by the second-order one-sided difference through the half-way wall
 * value and the first two nodes.  For the double-diffusive cavity of Sec. 3.2
 * (D = [[1, D_CT], [S_TC/Le, 1/Le]]) at the hot wall (side 0) these are the
 * mean Nusselt and Sherwood numbers.  Uses the constant part of D.
 * Synchronises the stream. */
lb_status lb_wall_flux(lb_handle* h, int32_t side, double* flux);

/* Totals: mass[a] = sum_x phi_a (a < m), mass[m] = sum_x sum_i h_i (= N rho0 for the
 * incompressible equilibrium).  FP64, deterministic.  Synchronises the stream. */
lb_status lb_mass(lb_handle* h, double* mass);

/* Populations at the current time, pre-collision, in canonical order and raw
 * (un-shifted) FP64: f [m][5][ny][nx], hpop [9][ny][nx]; either may be NULL.
 * Synchronises the stream. */
lb_status lb_populations(lb_handle* h, double* f, double* hpop);

/* Time step counter (number of steps taken since lb_init). */
lb_status lb_time(lb_handle* h, int64_t* t);

/* Checkpoint: size of the blob, save into / restore from a host buffer.
 * lb_load requires a handle created with identical parameters.  A run of n
 * steps equals k steps + save + load + (n - k) steps bit for bit. */
lb_status lb_state_bytes(lb_handle* h, size_t* bytes);
lb_status lb_save(lb_handle* h, void* host_buf, size_t bytes);
lb_status lb_load(lb_handle* h, const void* host_buf, size_t bytes);

/* Copies the state of src into dst (both initialised, same parameters except
 * storage, phi_ref and the FP16 scales), converting the storage on the device:
 * populations, previous-step source and time counter.  Used to finish an FP32
 * or FP16 run in FP64 (mixed-precision steady solve).  dst's residual snapshot
 * is reset.  Synchronises both streams. */
lb_status lb_copy_state(lb_handle* dst, lb_handle* src);

/* Fluid reference pressure per row (a storage detail; results are unchanged in
 * exact arithmetic).  With a reference P(y) the stored fluid populations of
 * row y are h_i minus the rest equilibrium at pressure P(y) (Eq. heq at u = 0:
 * r_0 = -(5/3) P, r_i = 3 W_i P for i > 0, so sum_i r_i = 0 and no moment but
 * the pressure changes), and values that stream between rows change reference
 * on the way.  A flow close to hydrostatic balance (Sec. 3.1: buoyancy balanced
 * by a vertical pressure gradient) then stores only its departure from that
 * balance, so FP32 storage rounds a much smaller number.
 * mode 1: P(y) = the row mean of the current pressure (FP64 sums, fixed order,
 * then rounded to the storage's arithmetic type), and every stored fluid value
 * is moved to it; call again to follow a changing balance.  mode 0: back to no
 * reference.  lb_moments, lb_populations, lb_save/lb_load and lb_copy_state see
 * and keep the absolute values.  Not for the no-fluid model or fused_steps = 2
 * (LB_EINVAL).  Synchronises the stream. */
lb_status lb_fluid_reference(lb_handle* h, int32_t mode);

/* Launch shape of the step kernel: tile_x * tile_y threads per workgroup,
 * tile_x a multiple of 64 (one wavefront per row segment), product <= 1024.
 * (0, 0) restores the default.  Used by the autotuner. */
lb_status lb_set_tile(lb_handle* h, int32_t tile_x, int32_t tile_y);

/* Releases the handle (never the workspace).  NULL is accepted. */
lb_status lb_free(lb_handle* h);

/* ---- batched parameter sweep ------------------------------------------------
 * count independent cavities of uneven size (each its own lb_params: grid,
 * tau_f, D, forces, walls, boundary kinds) advanced together: every time step
 * is ONE launch over a list of tiles of all running cavities, each workgroup
 * reading its cavity's parameter record from device memory.  All cavities
 * must share m, model, storage, collision and r_kind.  Residuals are reduced
 * per cavity (FP64, deterministic); converged, diverged or capped cavities are
 * retired from the tile list and keep their final state.
 * Per-cavity status: 0 running, 1 converged, 2 diverged (non-finite). */
typedef struct lbb_handle lbb_handle;

/* Workspace bytes for the batch (validates every record). */
lb_status lbb_workspace_bytes(const lb_params* params, int32_t count, size_t* bytes);

/* Initialises every cavity at equilibrium of its host fields phi0[c] ([m][ny][nx]),
 * u0[c] ([2][ny][nx]) and p0[c] ([ny][nx]; p0 or p0[c] may be NULL).  Synchronises. */
lb_status lbb_init(const lb_params* params, int32_t count, void* dev_workspace, size_t workspace_bytes,
                   void* hip_stream, const double* const* phi0, const double* const* u0, const double* const* p0,
                   lbb_handle** out);

/* Advances every running cavity by n steps (n launches), asynchronously. */
lb_status lbb_step(lbb_handle* b, int64_t n);

/* Runs until every cavity is retired or max_steps steps were taken by this call:
 * windows of check_every steps (rounded up to even) followed by the per-cavity
 * residual of lb_residual; a cavity retires when all its residual components
 * are below tol or when a field turns non-finite.  Cavities still running at
 * the end keep status 0 and continue in the next call (a call sequence is a
 * long run with progress points).  Outputs (any may be NULL): steps_out[count]
 * (total steps per cavity), status_out[count], res_out[count][m + 2] (last
 * residual).  Synchronises. */
lb_status lbb_run(lbb_handle* b, double tol, int64_t check_every, int64_t max_steps, int64_t* steps_out,
                  int32_t* status_out, double* res_out);

/* Copies cavity j of src into cavity i of dst (same parameters except storage,
 * phi_ref and the FP16 scales), converting the storage on the device; cavity i
 * becomes running with src's step count.  dst must be at an even batch step.
 * Used for the FP64 finish of an FP32 sweep.  Synchronises both streams. */
lb_status lbb_copy_cavity(lbb_handle* dst, int32_t i, lbb_handle* src, int32_t j);

/* Fields of cavity i (host arrays as in lb_moments; any may be NULL).  Synchronises. */
lb_status lbb_moments(lbb_handle* b, int32_t i, double* phi, double* u, double* p);

/* Steps taken by cavity i and its status. */
lb_status lbb_time(lbb_handle* b, int32_t i, int64_t* steps, int32_t* status);

/* Tile shape of the batched step for every cavity: one of 32x4, 32x8, 64x2,
 * 64x4, 128x1, 128x2, 256x1. */
lb_status lbb_set_tile(lbb_handle* b, int32_t tile_x, int32_t tile_y);

/* Autotuner: times trial_steps steps (rounded up to even, plus 2 warm-up steps)
 * of every supported tile shape on the live batch and keeps the fastest for
 * all cavities (tile_x, tile_y); then, one cavity width at a time, tries the
 * other shapes of the same workgroup size for the cavities of that width and
 * keeps one when it saves more than 1 % of the step time (lbb_cavity_tile reads
 * the result).  The timed steps are real steps of every running cavity (counted
 * in their step totals; results do not depend on the tile shapes).  us_per_step
 * is the best step time seen.  Outputs may be NULL. */
lb_status lbb_autotune(lbb_handle* b, int32_t trial_steps, int32_t* tile_x, int32_t* tile_y, double* us_per_step);

/* Tile shape of cavity i alone (one of the shapes above with the batch's
 * workgroup size, tile_x * tile_y of the last lbb_set_tile; LB_EINVAL otherwise),
 * and the shape in use for cavity i. */
lb_status lbb_set_cavity_tile(lbb_handle* b, int32_t i, int32_t tile_x, int32_t tile_y);
lb_status lbb_cavity_tile(lbb_handle* b, int32_t i, int32_t* tile_x, int32_t* tile_y);

/* Releases the batch handle (never the workspace).  NULL is accepted. */
lb_status lbb_free(lbb_handle* b);

/* Thread-local text of the last error, "" if none. */
const char* lb_last_error(void);

/* sizeof(lb_params) as compiled into the library (lets bindings check their
 * mirror of the record). */
size_t lb_params_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* LBCDF_LB_H */
