// lb_cde.hip -- Case 1 of the model (Sec. 2): the convection cross-diffusion
// equation without a fluid.  The velocity field is prescribed (given at
// initialisation, constant in time); only the m D2Q5 scalar lattices evolve.
// The auxiliary source follows the Case 1 form
//   G_{i,a} = sum_b (delta_ab - omega_ab / 2) W_i c_i . d_t(phi_b u) / cs^2,
// with d_t(phi u) = u (phi(t) - phi(t - dt)) / dt, the first-order backward
// difference the paper points to; phi(-dt) = phi0.  Closures are the linear
// ones (constant D, S = K phi); there is no body force.
//
// Storage: the scalar populations in the blocked layout of lb_device.h with
// 5m populations per block; per node, in the arithmetic type, the prescribed
// velocity (2 planes) and the previous phi - phi_ref (m planes) follow the
// S_old planes.
#include <hip/hip_runtime.h>

#include "lb_internal.h"
#include "lb_device.h"

namespace lbk {

template <int M>
__device__ __forceinline__ long long cidx(int q, long long n) {
    constexpr int NQ = 5 * M;
    return ((n >> kBlkShift) * (NQ << kBlkShift) + (n & (kBlk - 1))) + ((long long)q << kBlkShift);
}

// canonical pre-collision scalar populations of node (x, y); PULL as in gather()
template <class S, int M, bool PULL, bool NT = false, class T>
__device__ __forceinline__ void gather_f(const KParams<T>& kp, const S* __restrict__ pop, int x, int y,
                                         T f[M][5]) {
    const long long n = (long long)y * kp.nx + x;
    if constexpr (!PULL) {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) f[a][i] = ld<NT>(pop + cidx<M>(5 * a + i, n), kp, false);
    } else {
        Nbr nb(kp, x, y);
        if (__all(no_wall_link(kp, x, y))) {
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    f[a][i] = ld<NT>(pop + cidx<M>(5 * a + OPP5[i], nb.at(-CX5[i], -CY5[i])), kp, false);
            return;
        }
        const WallFlags wf(kp, x, y);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const int cx = CX5[i], cy = CY5[i];
                const bool out = wf.out_x(-cx) || wf.out_y(-cy);
                const int side = wf.out_x(-cx) ? (cx > 0 ? 0 : 1) : (cy > 0 ? 2 : 3);
                const long long src = out ? n : nb.at(-cx, -cy);
                const T v = ld<NT>(pop + cidx<M>(5 * a + (out ? i : OPP5[i]), src), kp, false);
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                f[a][i] = dir ? -v + T(2) * w5<T>(i) * kp.wallr[side][a] : v;
            }
    }
}

// post-collision scalar populations of node (x, y); PUSH as in scatter()
template <class S, int M, bool PUSH, bool NT = false, class T>
__device__ __forceinline__ void scatter_f(const KParams<T>& kp, S* __restrict__ pop, int x, int y, const T f[M][5]) {
    const long long n = (long long)y * kp.nx + x;
    if constexpr (!PUSH) {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) st<NT>(pop, cidx<M>(5 * a + OPP5[i], n), f[a][i], kp, false, 0u);
    } else {
        Nbr nb(kp, x, y);
        if (__all(no_wall_link(kp, x, y))) {
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 5; ++i) st<NT>(pop, cidx<M>(5 * a + i, nb.at(CX5[i], CY5[i])), f[a][i], kp, false, 0u);
            return;
        }
        const WallFlags wf(kp, x, y);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const int cx = CX5[i], cy = CY5[i];
                const bool out = wf.out_x(cx) || wf.out_y(cy);
                const int side = wf.out_x(cx) ? (cx > 0 ? 1 : 0) : (cy > 0 ? 3 : 2);
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                const T v = dir ? -f[a][i] + T(2) * w5<T>(i) * kp.wallr[side][a] : f[a][i];
                const long long dst = out ? n : nb.at(cx, cy);
                st<NT>(pop, cidx<M>(5 * a + (out ? OPP5[i] : i), dst), v, kp, false, 0u);
            }
    }
}

// one node: moments, linear source, Case 1 auxiliary source, matrix collision
// (Eq. evolution12 with the linear equilibrium of Eq. feq-phi, deviation form)
// CONS (FP32 storage): the rest populations take the remainder of each
// species' post-collision mass in FP64 (as in the fluid model's collision).
template <class T, int M, bool CONS = false>
__device__ __forceinline__ void collide_cde(const KParams<T>& kp, T f[M][5], const T u[2], const T prevd[M],
                                            const T Sold[M], T phid[M], T Snew[M]) {
    double mass_in[M];
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a)
            mass_in[a] = (((double)f[a][0] + (double)f[a][1]) + ((double)f[a][2] + (double)f[a][3])) + (double)f[a][4];
    }
    T phi[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        phid[a] = ((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + f[a][4];
        phi[a] = kp.phi_ref[a] + phid[a];
    }
    T S[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        S[a] = T(0);
        if (kp.src_mask >> a & 1) {
#pragma unroll
            for (int b = 0; b < M; ++b) S[a] += kp.K[a * M + b] * phi[b];
        }
    }
    // g_a = sum_b (delta_ab - omega_ab/2) u (phi_b(t) - phi_b(t - dt))
    T g[M][2];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        T s = T(0);
#pragma unroll
        for (int b = 0; b < M; ++b) s += ((a == b ? T(1) : T(0)) - T(0.5) * kp.omega[a * M + b]) * (phid[b] - prevd[b]);
        g[a][0] = s * u[0];
        g[a][1] = s * u[1];
    }
    T src[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        src[a] = T(1.5) * S[a] - T(0.5) * Sold[a];
        Snew[a] = S[a];
    }
    T feq[M][5], wsrc[M][5];
#pragma unroll
    for (int b = 0; b < M; ++b) {
        T pd = phid[b];
        if (kp.lam_on) pd += lam_excess<T, M>(kp, phi, b);  // lambda != I (D2Q5 form)
        const T iso = pd * (T(1) / T(6));
        const T adv = T(0.5) * phi[b];
        feq[b][1] = iso + adv * u[0];
        feq[b][3] = iso - adv * u[0];
        feq[b][2] = iso + adv * u[1];
        feq[b][4] = iso - adv * u[1];
        feq[b][0] = phid[b] - T(4) * iso;
        const T s6 = src[b] * (T(1) / T(6));
        wsrc[b][1] = wsrc[b][2] = wsrc[b][3] = wsrc[b][4] = s6;
        wsrc[b][0] = src[b] - T(4) * s6;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const T wi = w5<T>(i);
        T neq[M];
#pragma unroll
        for (int b = 0; b < M; ++b) neq[b] = f[b][i] - feq[b][i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            T coll = T(0);
#pragma unroll
            for (int b = 0; b < M; ++b) coll += kp.omega[a * M + b] * neq[b];
            const T cg = T(CX5[i]) * g[a][0] + T(CY5[i]) * g[a][1];
            f[a][i] = f[a][i] - coll + wsrc[a][i] + T(3) * wi * cg;
        }
    }
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double moving = ((double)f[a][1] + (double)f[a][2]) + ((double)f[a][3] + (double)f[a][4]);
            f[a][0] = T((mass_in[a] + (double)src[a]) - moving);
        }
    }
}

template <class S, int M, bool ODD, bool NT>
__global__ __launch_bounds__(256) void k_cde_step(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                                  typename St<S>::T* __restrict__ sold,
                                                  typename St<S>::T* __restrict__ aux, int tile_x, int tile_y,
                                                  int tiles_x) {
    using T = typename St<S>::T;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % tiles_x, by = b / tiles_x;
    const int x = bx * tile_x + (int)(threadIdx.x % tile_x);
    const int y = by * tile_y + (int)(threadIdx.x / tile_x);
    if (x >= kp.nx || y >= kp.ny) return;
    const long long N = (long long)kp.nx * kp.ny, n = (long long)y * kp.nx + x;
    T f[M][5], u[2], prevd[M], Sold[M], phid[M], Snew[M];
    gather_f<S, M, ODD, NT>(kp, pop, x, y, f);
    u[0] = load_raw<NT>(&aux[n]);
    u[1] = load_raw<NT>(&aux[N + n]);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        prevd[a] = load_raw<NT>(&aux[(2 + a) * N + n]);
        Sold[a] = T(0);
        if (kp.src_mask >> a & 1) Sold[a] = load_raw<NT>(&sold[(long long)(k++) * N + n]);
    }
    collide_cde<T, M, std::is_same_v<S, float>>(kp, f, u, prevd, Sold, phid, Snew);
    k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        store_raw<NT>(phid[a], &aux[(2 + a) * N + n]);
        if (kp.src_mask >> a & 1) store_raw<NT>(Snew[a], &sold[(long long)(k++) * N + n]);
    }
    scatter_f<S, M, ODD, NT>(kp, pop, x, y, f);
}

// equilibrium initialisation from the staged FP64 fields phi0 [M][N], u0 [2][N]
template <class S, int M>
__global__ __launch_bounds__(256) void k_cde_init(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                                  typename St<S>::T* __restrict__ sold,
                                                  typename St<S>::T* __restrict__ aux,
                                                  const double* __restrict__ stage) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T phi[M], u[2];
#pragma unroll
    for (int a = 0; a < M; ++a) phi[a] = T(stage[a * N + n]);
    u[0] = T(stage[M * N + n]);
    u[1] = T(stage[(M + 1) * N + n]);
    aux[n] = u[0];
    aux[N + n] = u[1];
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const T phid = phi[a] - kp.phi_ref[a];
        T pd = phid;
        if (kp.lam_on) pd += lam_excess<T, M>(kp, phi, a);
        const T iso = pd * (T(1) / T(6));
        const T adv = T(0.5) * phi[a];
        st(pop, cidx<M>(5 * a + 1, n), iso + adv * u[0], kp, false, 0u);
        st(pop, cidx<M>(5 * a + 3, n), iso - adv * u[0], kp, false, 0u);
        st(pop, cidx<M>(5 * a + 2, n), iso + adv * u[1], kp, false, 0u);
        st(pop, cidx<M>(5 * a + 4, n), iso - adv * u[1], kp, false, 0u);
        st(pop, cidx<M>(5 * a + 0, n), phid - T(4) * iso, kp, false, 0u);
        aux[(2 + a) * N + n] = phid;
        if (kp.src_mask >> a & 1) {
            T s = T(0);
#pragma unroll
            for (int b = 0; b < M; ++b) s += kp.K[a * M + b] * phi[b];
            sold[(long long)(k++) * N + n] = s;
        }
    }
}

template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_cde_moments(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                     const typename St<S>::T* __restrict__ aux,
                                                     double* __restrict__ phi, double* __restrict__ u,
                                                     double* __restrict__ pr) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T f[M][5];
    gather_f<S, M, ODD>(kp, pop, (int)(n % kp.nx), (int)(n / kp.nx), f);
    if (phi)
#pragma unroll
        for (int a = 0; a < M; ++a)
            phi[a * N + n] = double(kp.phi_ref[a]) + double(((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + f[a][4]);
    if (u) {
        u[n] = double(aux[n]);
        u[N + n] = double(aux[N + n]);
    }
    if (pr) pr[n] = 0.0;
}

// raw canonical scalar populations, planes [plane_begin, plane_begin + count)
// of the sequence f_{1,0}..f_{m,4}, into out[k][N]
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_cde_export(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                    int plane_begin, int count, double* __restrict__ out) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T f[M][5];
    gather_f<S, M, ODD>(kp, pop, (int)(n % kp.nx), (int)(n / kp.nx), f);
#pragma unroll
    for (int k = 0; k < 5 * M; ++k) {
        if (k < plane_begin || k >= plane_begin + count) continue;
        const int a = k / 5, i = k % 5;
        out[(long long)(k - plane_begin) * N + n] = double(f[a][i]) + double(w5<T>(i)) * double(kp.phi_ref[a]);
    }
}

// first reduction pass, same partial records as k_reduce: residual / snapshot
// of q = (u_x, u_y, phi_a) (modes 0, 1), or masses [phi_a (M), 0 (no fluid)] (mode 2)
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_cde_reduce(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                    const typename St<S>::T* __restrict__ aux,
                                                    double* __restrict__ snap, double* __restrict__ part, int mode) {
    using T = typename St<S>::T;
    constexpr int Q = M + 2;
    const long long N = (long long)kp.nx * kp.ny;
    double acc[2 * Q + 1];
#pragma unroll
    for (int k = 0; k < 2 * Q + 1; ++k) acc[k] = 0.0;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        T f[M][5];
        gather_f<S, M, ODD>(kp, pop, (int)(n % kp.nx), (int)(n / kp.nx), f);
        double q[Q];
        q[0] = double(aux[n]);
        q[1] = double(aux[N + n]);
#pragma unroll
        for (int a = 0; a < M; ++a)
            q[2 + a] = double(kp.phi_ref[a]) + double(((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + f[a][4]);
        bool bad = false;
        if (mode == 2) {
#pragma unroll
            for (int a = 0; a < M; ++a) {
                acc[a] += q[2 + a];
                bad |= !isfinite(q[2 + a]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double old = snap[(long long)k * N + n];
                acc[k] += fabs(q[k] - old);
                acc[Q + k] += fabs(q[k]);
                snap[(long long)k * N + n] = q[k];
                bad |= !isfinite(q[k]);
            }
        }
        acc[2 * Q] += bad ? 1.0 : 0.0;
    }
    block_sum<2 * Q + 1>(acc, part + (long long)blockIdx.x * kRedWidth);
}

// ---- launchers ---------------------------------------------------------------
template <class Fn>
static hipError_t dispatch_cde(const lb_params& p, Fn&& fn) {
    auto by_m = [&](auto sTag) -> hipError_t {
        using S = decltype(sTag);
        switch (p.m) {
            case 1: return fn.template operator()<S, 1>();
            case 2: return fn.template operator()<S, 2>();
            case 3: return fn.template operator()<S, 3>();
            case 4: return fn.template operator()<S, 4>();
        }
        return hipErrorInvalidValue;
    };
    if (p.model != LB_MODEL_CDE) return hipErrorInvalidValue;
    switch (p.storage) {
        case LB_STORE_F64: return by_m(double{});
        case LB_STORE_F32: return by_m(float{});
    }
    return hipErrorInvalidValue;
}

hipError_t launch_cde_init(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                           const KParams<float>& kf, hipStream_t s) {
    return dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        hipLaunchKernelGGL((k_cde_init<S, M>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                           (S*)at(ws, L.pop_off), (T*)at(ws, L.sold_off), (T*)at(ws, L.aux_off),
                           (const double*)at(ws, L.stage_off));
        return hipGetLastError();
    });
}

hipError_t launch_cde_step(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                           const KParams<float>& kf, bool odd, Launch lc, hipStream_t s) {
    const int tiles_x = (p.nx + lc.tile_x - 1) / lc.tile_x;
    const int tiles_y = (p.ny + lc.tile_y - 1) / lc.tile_y;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)(lc.tile_x * lc.tile_y));
    return dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at(ws, L.pop_off);
        T* sold = (T*)at(ws, L.sold_off);
        T* aux = (T*)at(ws, L.aux_off);
        const bool nt = (lc.nt >> (odd ? 1 : 0) & 1) != 0;
        const void* const fns[4] = {reinterpret_cast<const void*>(&k_cde_step<S, M, false, false>),
                                    reinterpret_cast<const void*>(&k_cde_step<S, M, false, true>),
                                    reinterpret_cast<const void*>(&k_cde_step<S, M, true, false>),
                                    reinterpret_cast<const void*>(&k_cde_step<S, M, true, true>)};
        KParams<T> kp = kpar<S>(kd, kf);
        int tx = lc.tile_x, ty = lc.tile_y, tsx = tiles_x;
        void* args[] = {&kp, &pop, &sold, &aux, &tx, &ty, &tsx};
        hipError_t e = hipLaunchKernel(fns[(odd ? 2 : 0) + (nt ? 1 : 0)], grid, block, args, 0, s);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    });
}

// A graph of `steps` (even) no-fluid step launches, even parity first, chained; built node
// by node like the fluid model's step graph (the arguments are the same for every launch of
// a parity: the previous-phi planes are updated in place)
hipError_t build_cde_step_graph(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                                const KParams<float>& kf, Launch lc, int steps, hipGraph_t* out) {
    if (steps < 2 || steps % 2) return hipErrorInvalidValue;
    const int tiles_x = (p.nx + lc.tile_x - 1) / lc.tile_x;
    const int tiles_y = (p.ny + lc.tile_y - 1) / lc.tile_y;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)(lc.tile_x * lc.tile_y));
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    e = dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at(ws, L.pop_off);
        T* sold = (T*)at(ws, L.sold_off);
        T* aux = (T*)at(ws, L.aux_off);
        KParams<T> kp = kpar<S>(kd, kf);
        int tx = lc.tile_x, ty = lc.tile_y, tsx = tiles_x;
        void* args[] = {&kp, &pop, &sold, &aux, &tx, &ty, &tsx};
        void* fe = reinterpret_cast<void*>((lc.nt & 1) ? &k_cde_step<S, M, false, true> : &k_cde_step<S, M, false, false>);
        void* fo = reinterpret_cast<void*>((lc.nt & 2) ? &k_cde_step<S, M, true, true> : &k_cde_step<S, M, true, false>);
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < steps; ++k) {
            hipKernelNodeParams np{};
            np.func = (k & 1) ? fo : fe;
            np.gridDim = grid;
            np.blockDim = block;
            np.sharedMemBytes = 0;
            np.kernelParams = args;
            np.extra = nullptr;
            hipGraphNode_t node;
            hipError_t ee = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
            if (ee != hipSuccess) return ee;
            prev = node;
        }
        return hipSuccess;
    });
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    *out = g;
    return hipSuccess;
}

hipError_t launch_cde_moments(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                              const KParams<float>& kf, bool odd, double* phi, double* u, double* pr, hipStream_t s) {
    return dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        const S* pop = (const S*)at(ws, L.pop_off);
        const T* aux = (const T*)at(ws, L.aux_off);
        if (odd)
            hipLaunchKernelGGL((k_cde_moments<S, M, true>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, aux, phi, u, pr);
        else
            hipLaunchKernelGGL((k_cde_moments<S, M, false>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, aux, phi, u, pr);
        return hipGetLastError();
    });
}

hipError_t launch_cde_export(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                             const KParams<float>& kf, bool odd, int plane_begin, int plane_count, double* out,
                             hipStream_t s) {
    return dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k_cde_export<S, M, true>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, plane_begin, plane_count, out);
        else
            hipLaunchKernelGGL((k_cde_export<S, M, false>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, plane_begin, plane_count, out);
        return hipGetLastError();
    });
}

hipError_t launch_cde_reduce(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                             const KParams<float>& kf, bool odd, int mode, hipStream_t s, double* part, double* res) {
    const int nb = reduce_blocks(L.N);
    if (!part) part = (double*)at(ws, L.part_off);
    if (!res) res = (double*)at(ws, L.res_off);
    hipError_t e = dispatch_cde(p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        const S* pop = (const S*)at(ws, L.pop_off);
        const T* aux = (const T*)at(ws, L.aux_off);
        double* snap = (double*)at(ws, L.snap_off);
        if (odd)
            hipLaunchKernelGGL((k_cde_reduce<S, M, true>), dim3(nb), dim3(256), 0, s, kpar<S>(kd, kf), pop, aux, snap,
                               part, mode);
        else
            hipLaunchKernelGGL((k_cde_reduce<S, M, false>), dim3(nb), dim3(256), 0, s, kpar<S>(kd, kf), pop, aux,
                               snap, part, mode);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return launch_reduce_final(p.m + 2, part, nb, res, mode, s);
}

}  // namespace lbk
