/*
 * lb3.h -- C ABI of the three-dimensional form of the coupled
 * cross-diffusion-fluid lattice Boltzmann model (Zhan, Chai & Shi, arXiv
 * 2101.03055): one D3Q7 lattice per scalar and a D3Q19 lattice for the
 * fluid, with the lattice tables of Sec. 2 (cs^2 = 1/4 on D3Q7, 1/3 on D3Q19).
 *
 * The evolution is that of Eqs. evolution12 and evolution3 with the linear
 * closures of the LB_MODEL_LINEAR model of lb.h: constant diffusion matrix D
 * (omega = (D / cs7^2 + I/2)^-1 = (4 D + I/2)^-1, Eq. omega-D with lambda = I),
 * linear source S = K phi with the first-order time-derivative correction
 * (Eq. source, gamma = 0), auxiliary source G of Eq. Gi with the D3Q7 sound
 * speed, body force F = F0 + sum_a Fphi[a] phi_a with the forcing of Eq. force
 * (varphi = 0), BGK fluid, pressure of Eq. sum-p.  Boundaries per side
 * (x-, x+, y-, y+, z-, z+): periodic (in pairs) or half-way walls; the fluid
 * bounces back on a wall (no slip; a D3Q19 link leaving through an edge
 * bounces back too), each scalar takes no flux (bounce-back) or a Dirichlet
 * value (anti-bounce-back f_opp = -f*_i + 2 W_i phi_w).
 *
 * Same conventions as lb.h: the caller owns the device workspace and every
 * host array; calls return lb_status and never abort; lb3_last_error gives
 * the message of the last failure on the calling thread.  Fields are
 * host arrays in FP64, x fastest: phi [m][nz][ny][nx], u [3][nz][ny][nx],
 * p [nz][ny][nx].  Storage LB_STORE_F64, or LB_STORE_F32 holding deviations
 * from W_i phi_ref (scalars) and rho0 (rest fluid population), with each
 * species' rest population set to the FP64 remainder of its post-collision
 * mass.  Grids need nx ny nz < 2^31 and (nx + 64)(19 + 7m) < 2^31.
 */
#ifndef LB3_H
#define LB3_H

#include <stddef.h>
#include <stdint.h>

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb3_params {
    int32_t nx, ny, nz;              /* grid, each >= 2; nx ny nz < 2^31 */
    int32_t m;                       /* scalars, 1..4 */
    int32_t storage;                 /* LB_STORE_F64 | LB_STORE_F32 */
    int32_t fluid_bc[6];             /* LB_BC_PERIODIC | LB_BC_NOSLIP per side */
    int32_t scalar_bc[6][LB_MAX_M];  /* LB_SBC_* per side and species; periodic must match the fluid */
    int32_t pad_;
    double tau_f;                    /* fluid relaxation time (> 1/2); nu = (tau_f - 1/2)/3 */
    double rho0;                     /* constant of the fluid equilibrium (Eq. heq) */
    double D[LB_MAX_M * LB_MAX_M];   /* diffusion matrix, row-major m x m */
    double K[LB_MAX_M * LB_MAX_M];   /* linear source matrix, row-major m x m */
    double F0[3];                    /* constant body force */
    double Fphi[LB_MAX_M][3];        /* F += Fphi[a] * phi_a */
    double wall[6][LB_MAX_M];        /* Dirichlet wall values [side][species] */
    double phi_ref[LB_MAX_M];        /* reference level of the F32 deviation storage */
} lb3_params;

typedef struct lb3_handle lb3_handle;

/* Bytes of device workspace for these parameters (validates them first). */
lb_status lb3_workspace_bytes(const lb3_params* params, size_t* bytes);

/* Validates (tau_f > 1/2, Re eig(D) > 0, codes, periodic pairs, finite
 * values), then sets f = f^eq(phi0, u0), h = h^eq(p0, u0 - F(phi0)/2) and
 * S_old = S(phi0) at t = 0.  dev_workspace: device memory of at least
 * lb3_workspace_bytes, 256-byte aligned, owned by the caller and not freed by
 * the library.  p0 may be NULL (p0 = 0).  Synchronises the stream. */
lb_status lb3_init(const lb3_params* params, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                   const double* phi0, const double* u0, const double* p0, lb3_handle** out);

/* Advances n >= 0 time steps asynchronously on the handle's stream (AA-pattern
 * in-place streaming: even steps read and write each node's own slots, odd
 * steps its neighbours'). */
lb_status lb3_step(lb3_handle* h, int64_t n);

/* Macroscopic fields (Eq. sum) at the current time into host arrays (any may
 * be NULL).  Synchronises the stream. */
lb_status lb3_moments(lb3_handle* h, double* phi, double* u, double* p);

/* Canonical populations at the current time (post-streaming, pre-collision):
 * f [m][7][nz][ny][nx] and h [19][nz][ny][nx] in the velocity order of the
 * Sec. 2 tables, with any storage shift added back.  Host arrays; either may
 * be NULL.  Synchronises the stream. */
lb_status lb3_populations(lb3_handle* h, double* f, double* hpop);

/* Totals: mass[a] = sum phi_a for a < m, mass[m] = sum_i h_i; deterministic
 * FP64 reduction.  LB_ENONFINITE if any total is not finite.  Synchronises. */
lb_status lb3_mass(lb3_handle* h, double* mass);

/* Steps taken since lb3_init. */
lb_status lb3_time(lb3_handle* h, int64_t* t);

/* Workgroup shape: tile_x x tile_y nodes of one z-plane (tile_x * tile_y <= 256,
 * a multiple of 64).  Results do not depend on it. */
lb_status lb3_set_tile(lb3_handle* h, int32_t tile_x, int32_t tile_y);

/* Releases the handle (not the workspace).  NULL is accepted. */
lb_status lb3_free(lb3_handle* h);

const char* lb3_last_error(void);

/* sizeof(lb3_params) as compiled into the library. */
size_t lb3_params_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* LB3_H */
