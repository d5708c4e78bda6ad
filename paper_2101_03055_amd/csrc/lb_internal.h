// lb_internal.h -- shared declarations between the C ABI (lb_api.hip) and the
// gfx950 kernels (lb_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lb.h"

namespace lbk {

// Kernel-side parameter block, in the arithmetic type T of the storage mode
// (double for LB_STORE_F64, float otherwise).  Passed by value.
template <class T>
struct KParams {
    int nx, ny;
    int px, py;           // periodic in x / y
    int fbc[4];           // fluid boundary code per side
    int sbc[4][LB_MAX_M]; // scalar boundary code per side and species
    int r_kind;
    int src_mask;         // species carrying a source (need S_old)
    T wallr[4][LB_MAX_M]; // Dirichlet value minus phi_ref
    T omega_f;            // 1 / tau_f
    T rho0_eff;           // constant in sigma_0 as seen by the stored h_0
    T h0_shift;           // stored h_0 = h_0 - h0_shift
    T omega[LB_MAX_M * LB_MAX_M]; // constant relaxation matrix (linear model)
    T Dc[4];              // chemotaxis: constant part of D (2 x 2)
    T K[LB_MAX_M * LB_MAX_M];
    T Dflux[LB_MAX_M * LB_MAX_M]; // constant diffusion matrix (wall-flux diagnostics)
    T F0[2];
    T Fphi[LB_MAX_M][2];
    T chi, beta, cstar, eps;
    T mrt_s[9];
    T phi_ref[LB_MAX_M];
    T scale, inv_scale;   // storage scale of the scalar planes (F16 only; 1 otherwise)
    T scale_h, inv_scale_h; // storage scale of the fluid planes (F16 only; 1 otherwise)
    int lam_on;           // lambda != I in the scalar equilibrium (linear and no-fluid models)
    T lamm[LB_MAX_M * LB_MAX_M]; // lambda - I, row-major
    T varphi;             // varphi of Eq. force (0: the force term of Sec. 3)
    T vp_p;               // pressure correction per u.F: (tau_f - 1/2) (4/3) varphi
    int gam_on;           // gamma != 0 in D-bar (Eq. evolution12) for a species with a source
    T gam12[LB_MAX_M];    // gamma_a / 12: the auxiliary-source vector gains gamma_a grad S_a / 6,
                          // with grad S_a = (S(x + e) - S(x - e)) / 2
    const T* pref;        // fluid reference pressure per row, or NULL (lb_fluid_reference)
};

struct Layout {
    size_t N;             // nodes
    size_t elem;          // bytes per stored population value
    size_t plane;         // nodes rounded up to whole storage blocks (64)
    size_t npop;          // population planes, 9 + 5m
    size_t nsrc;          // S_old planes
    size_t pop_off, sold_off, snap_off, stage_off, part_off, res_off, total;
    size_t pop2_off, sold2_off;  // second population / source arrays (two-step launches; the source
                                 // planes also when gamma != 0: the step reads the previous source
                                 // field at the neighbours while writing the new one)
    size_t naux, aux_off;        // no-fluid model: prescribed u (2 planes) and previous phi - phi_ref (m planes)
    size_t pref_off;             // fluid reference pressure per row (ny values of the arithmetic type)
    size_t tstep_off;            // step count read by replayed FP16 step graphs (one int64)
};

constexpr int kRedBlocks = 1024;   // blocks of the first reduction pass (upper bound)
constexpr int kRedWidth = 16;      // doubles per partial record

struct Launch {
    int tile_x, tile_y;
    int nt;  // non-temporal population accesses: bit 0 in even steps, bit 1 in odd steps
};

// launchers (lb_kernels.hip); all return hipError_t of the launch
hipError_t launch_init(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                       const KParams<float>& kf, int has_p0, hipStream_t s);
hipError_t launch_step(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                       const KParams<float>& kf, bool odd, Launch lc, int64_t step, hipStream_t s);
// two steps per launch: canonical state of L.pop_off / L.sold_off at t into
// L.pop2_off / L.sold2_off at t + 2
hipError_t launch_step2(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                        const KParams<float>& kf, int64_t step, hipStream_t s);
// fluid reference pressure: row means of the pressure (FP64, ny values), and the
// move of the stored fluid values from the reference in kp.pref to pnew (ny values of
// the arithmetic type)
hipError_t launch_row_pressure(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                               const KParams<float>& kf, bool odd, double* out, hipStream_t s);
hipError_t launch_reref(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                        const KParams<float>& kf, const void* pnew, hipStream_t s);
hipError_t launch_to_float(const double* src, float* dst, long long n, hipStream_t s);
hipError_t build_step_graph(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                            const KParams<float>& kf, Launch lc, int steps, const long long* tstep, hipGraph_t* out);
// *tstep = step (a one-thread kernel: ordered on the stream before a graph replay)
hipError_t launch_set_step(long long* tstep, long long step, hipStream_t s);
int reduce_blocks(size_t N);
hipError_t launch_reduce_final(int Q, const double* part, int nblocks, double* out, int mode, hipStream_t s);
// no-fluid model (lb_cde.hip)
hipError_t launch_cde_init(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                           const KParams<float>& kf, hipStream_t s);
hipError_t launch_cde_step(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                           const KParams<float>& kf, bool odd, Launch lc, hipStream_t s);
hipError_t build_cde_step_graph(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                                const KParams<float>& kf, Launch lc, int steps, hipGraph_t* out);
hipError_t launch_cde_moments(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                              const KParams<float>& kf, bool odd, double* phi, double* u, double* pr, hipStream_t s);
hipError_t launch_cde_export(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                             const KParams<float>& kf, bool odd, int plane_begin, int plane_count, double* out,
                             hipStream_t s);
// part / res: partial records (reduce_blocks(L.N) x kRedWidth doubles) and the
// result record; nullptr selects the workspace's own (L.part_off, L.res_off)
hipError_t launch_cde_reduce(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                             const KParams<float>& kf, bool odd, int mode, hipStream_t s, double* part = nullptr,
                             double* res = nullptr);
hipError_t launch_wall_flux(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                            const KParams<float>& kf, bool odd, int side, double* out, hipStream_t s);
hipError_t launch_moments(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                          const KParams<float>& kf, bool odd, double* phi, double* u, double* pr,
                          hipStream_t s);
hipError_t launch_export(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, bool odd, int plane_begin, int plane_count,
                         double* out, hipStream_t s);
// writes planes [plane_begin, plane_begin + count) of canonical raw FP64
// populations (as produced by launch_export) into the own-slot layout
hipError_t launch_import(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, int plane_begin, int plane_count, const double* in,
                         hipStream_t s);
// converts the previous-step source planes between storage modes
hipError_t launch_copy_sold(const lb_params& ps, const Layout& Ls, void* wss, const lb_params& pd,
                            const Layout& Ld, void* wsd, hipStream_t s);
// mode 0: residual (updates the snapshot), mode 1: snapshot only, mode 2: mass;
// part / res as for launch_cde_reduce
hipError_t launch_reduce(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, bool odd, int mode, hipStream_t s, double* part = nullptr,
                         double* res = nullptr);

// ---- batched sweep ---------------------------------------------------------
// Per-cavity record visible to the batched kernels (offsets in bytes from the
// workspace base).
struct CavRec {
    long long pop_off, sold_off, snap_off;
    int tiles_x, tiles_y;
    int tile_x, tile_y;   // the cavity's tile shape (tile_x * tile_y = the launch's workgroup size)
};

// one step of every listed tile: tiles[k] = (cavity, tile index in the cavity)
hipError_t build_bstep_graph(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                             int ntiles, Launch lc, int steps, const long long* tstep, hipGraph_t* out);
hipError_t launch_bstep(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                        int ntiles, bool odd, Launch lc, int64_t step, hipStream_t s);
// per-tile partial sums (mode 0 residual + snapshot, 1 snapshot only, 2 mass),
// then per-cavity totals: ranges[k] = (cavity, first tile, tile count, 0);
// out[cavity][3 (m + 2) + 1]: diff sums, norms, non-finite count, residuals
hipError_t launch_breduce(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                          int ntiles, const int4* ranges, int nranges, bool odd, Launch lc, int mode, double* part,
                          double* out, hipStream_t s);

}  // namespace lbk
