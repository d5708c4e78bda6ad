// lb3.hip -- the three-dimensional form of the model (include/lb3.h): D3Q7
// scalar lattices (cs^2 = 1/4) and a D3Q19 fluid lattice (cs^2 = 1/3) with
// the lattice tables of Sec. 2, linear closures, BGK fluid.
//
// Same design as the 2-D path: one fused collide-and-stream kernel per step in
// the AA pattern (even steps read and write each node's own slots, odd steps
// pull from and push to the neighbours), populations in blocks of 64 nodes
// (within a block the 19 + 7m populations follow each other as runs of 64
// values), wall links resolved with selects, a wave-uniform fast path for
// interior wavefronts, deviation storage in FP32, non-temporal population
// accesses chosen by working-set size, XCD-aware workgroup placement.
// Algorithmic traffic per node update: 2 (19 + 7m) b bytes (+ 2 b per source
// plane): 528 B in FP64 and 264 B in FP32 for m = 2.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lb3.h"
#include "lb3_index.h"
#include "lb_device.h"

namespace lb3k {

using lbk::load_raw;
using lbk::St;
using lbk::store_raw;
using lbk::xcd_remap;

// ---- lattices (Sec. 2 tables) ------------------------------------------------
__device__ constexpr int CX19[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0};
__device__ constexpr int CY19[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int CZ19[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
__device__ constexpr int OPP19[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
__device__ constexpr int CX7[7] = {0, 1, 0, 0, -1, 0, 0};
__device__ constexpr int CY7[7] = {0, 0, 1, 0, 0, -1, 0};
__device__ constexpr int CZ7[7] = {0, 0, 0, 1, 0, 0, -1};
__device__ constexpr int OPP7[7] = {0, 4, 5, 6, 1, 2, 3};

template <class T>
__device__ __forceinline__ T w19(int i) {
    return i == 0 ? T(1) / T(3) : (i < 7 ? T(1) / T(18) : T(1) / T(36));
}

// kernel parameters, in the arithmetic type T
template <class T>
struct K3 {
    int nx, ny, nz;
    int px, py, pz;                // periodic axes
    int sbc[6][LB_MAX_M];
    int src_mask;                  // species with a source (S_old planes)
    T wallr[6][LB_MAX_M];          // Dirichlet value minus phi_ref
    T omega_f, rho0_eff;
    T omega[LB_MAX_M * LB_MAX_M];
    T K[LB_MAX_M * LB_MAX_M];
    T F0[3];
    T Fphi[LB_MAX_M][3];
    T phi_ref[LB_MAX_M];
};

struct Walls3 {
    bool lo[3], hi[3];
    template <class T>
    __device__ __forceinline__ Walls3(const K3<T>& kp, int x, int y, int z) {
        lo[0] = !kp.px && x == 0;
        hi[0] = !kp.px && x == kp.nx - 1;
        lo[1] = !kp.py && y == 0;
        hi[1] = !kp.py && y == kp.ny - 1;
        lo[2] = !kp.pz && z == 0;
        hi[2] = !kp.pz && z == kp.nz - 1;
    }
    // node + d (d in -1, 0, 1) lies beyond a wall on axis a
    __device__ __forceinline__ bool out(int a, int d) const { return (d < 0 && lo[a]) || (d > 0 && hi[a]); }
};

template <class T>
__device__ __forceinline__ bool interior(const K3<T>& kp, int x, int y, int z) {
    const bool ox = kp.px || ((x > 0) & (x < kp.nx - 1));
    const bool oy = kp.py || ((y > 0) & (y < kp.ny - 1));
    const bool oz = kp.pz || ((z > 0) & (z < kp.nz - 1));
    return ox & oy & oz;
}

template <bool NT, class S, class T>
__device__ __forceinline__ T ld3(const S* p) {
    return T(load_raw<NT>(p));
}
template <bool NT, class S, class T>
__device__ __forceinline__ void st3(S* p, T v) {
    store_raw<NT>(S(v), p);
}

// ---- gather: canonical pre-collision populations of one node ----------------
template <class S, int M, bool PULL, bool NT, class T>
__device__ __forceinline__ void gather3(const K3<T>& kp, const S* __restrict__ pop, int x, int y, int z, long long n,
                                        T h[19], T f[M][7]) {
    if constexpr (!PULL) {
#pragma unroll
        for (int i = 0; i < 19; ++i) h[i] = ld3<NT, S, T>(pop + p3<M>(i, n));
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 7; ++i) f[a][i] = ld3<NT, S, T>(pop + p3<M>(19 + 7 * a + i, n));
    } else {
        const Nb3E<M> nb(kp, x, y, z);
        if (__all(interior(kp, x, y, z))) {
#pragma unroll
            for (int i = 0; i < 19; ++i)
                h[i] = ld3<NT, S, T>(pop + nb.at(-CX19[i], -CY19[i], -CZ19[i]) + ((long long)(OPP19[i]) << 6));
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 7; ++i)
                    f[a][i] = ld3<NT, S, T>(pop + nb.at(-CX7[i], -CY7[i], -CZ7[i]) + ((long long)(19 + 7 * a + OPP7[i]) << 6));
            return;
        }
        const Walls3 w(kp, x, y, z);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            // the upstream node x - c_i beyond a wall (face or edge): bounce-back,
            // the node's own value of direction opp(i), kept in its slot i
            const bool out = w.out(0, -CX19[i]) || w.out(1, -CY19[i]) || w.out(2, -CZ19[i]);
            const long long src = out ? nb.at(0, 0, 0) : nb.at(-CX19[i], -CY19[i], -CZ19[i]);
            h[i] = ld3<NT, S, T>(pop + src + ((long long)(out ? i : OPP19[i]) << 6));
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const int cx = CX7[i], cy = CY7[i], cz = CZ7[i];
                const bool ox = w.out(0, -cx), oy = w.out(1, -cy), oz = w.out(2, -cz);
                const bool out = ox || oy || oz;
                const int side = ox ? (cx > 0 ? 0 : 1) : (oy ? (cy > 0 ? 2 : 3) : (cz > 0 ? 4 : 5));
                const long long src = out ? nb.at(0, 0, 0) : nb.at(-cx, -cy, -cz);
                const T v = ld3<NT, S, T>(pop + src + ((long long)(19 + 7 * a + (out ? i : OPP7[i])) << 6));
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                f[a][i] = dir ? -v + T(0.25) * kp.wallr[side][a] : v;  // 2 W_i phi_w, W_i = 1/8
            }
    }
}

// ---- scatter: post-collision values of one node -------------------------------
template <class S, int M, bool PUSH, bool NT, class T>
__device__ __forceinline__ void scatter3(const K3<T>& kp, S* __restrict__ pop, int x, int y, int z, long long n,
                                         const T h[19], const T f[M][7]) {
    if constexpr (!PUSH) {
#pragma unroll
        for (int i = 0; i < 19; ++i) st3<NT>(pop + p3<M>(OPP19[i], n), h[i]);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 7; ++i) st3<NT>(pop + p3<M>(19 + 7 * a + OPP7[i], n), f[a][i]);
    } else {
        const Nb3E<M> nb(kp, x, y, z);
        if (__all(interior(kp, x, y, z))) {
#pragma unroll
            for (int i = 0; i < 19; ++i) st3<NT>(pop + nb.at(CX19[i], CY19[i], CZ19[i]) + ((long long)(i) << 6), h[i]);
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 7; ++i) st3<NT>(pop + nb.at(CX7[i], CY7[i], CZ7[i]) + ((long long)(19 + 7 * a + i) << 6), f[a][i]);
            return;
        }
        const Walls3 w(kp, x, y, z);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const bool out = w.out(0, CX19[i]) || w.out(1, CY19[i]) || w.out(2, CZ19[i]);
            const long long dst = out ? nb.at(0, 0, 0) : nb.at(CX19[i], CY19[i], CZ19[i]);
            st3<NT>(pop + dst + ((long long)(out ? OPP19[i] : i) << 6), h[i]);
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                const int cx = CX7[i], cy = CY7[i], cz = CZ7[i];
                const bool ox = w.out(0, cx), oy = w.out(1, cy), oz = w.out(2, cz);
                const bool out = ox || oy || oz;
                const int side = ox ? (cx > 0 ? 1 : 0) : (oy ? (cy > 0 ? 3 : 2) : (cz > 0 ? 5 : 4));
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                const T v = dir ? -f[a][i] + T(0.25) * kp.wallr[side][a] : f[a][i];
                const long long dst = out ? nb.at(0, 0, 0) : nb.at(cx, cy, cz);
                st3<NT>(pop + dst + ((long long)(19 + 7 * a + (out ? OPP7[i] : i)) << 6), v);
            }
    }
}

// ---- macroscopic quantities (Eq. sum) in deviation form ------------------------
template <class T, int M>
struct Mac3 {
    T phid[M], phi[M], F[3], u[3], p;
};

template <class T, int M>
__device__ __forceinline__ void macro3(const K3<T>& kp, const T h[19], const T f[M][7], Mac3<T, M>& mc) {
#pragma unroll
    for (int a = 0; a < M; ++a) {
        mc.phid[a] = (((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + ((f[a][4] + f[a][5]) + f[a][6]));
        mc.phi[a] = kp.phi_ref[a] + mc.phid[a];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        mc.F[d] = kp.F0[d];
#pragma unroll
        for (int a = 0; a < M; ++a) mc.F[d] += kp.Fphi[a][d] * mc.phi[a];
    }
    T j[3] = {T(0), T(0), T(0)};
    T s = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (CX19[i]) j[0] += T(CX19[i]) * h[i];
        if (CY19[i]) j[1] += T(CY19[i]) * h[i];
        if (CZ19[i]) j[2] += T(CZ19[i]) * h[i];
        s += h[i];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) mc.u[d] = j[d] + T(0.5) * mc.F[d];
    const T usq = mc.u[0] * mc.u[0] + mc.u[1] * mc.u[1] + mc.u[2] * mc.u[2];
    // p = cs2/(1 - W0) [sum_{i>0} h_i - W0 u.u/(2 cs2)] with W0 = 1/3: (1/2)(s - u.u/2)
    mc.p = T(0.5) * (s - T(0.5) * usq);
}

// ---- the node update: Eqs. evolution12 (D3Q7) and evolution3 (D3Q19, BGK) -------
// CONS (FP32 storage): the scalar rest populations take the remainder of
// each species' post-collision mass in FP64 (sum_i f*_a,i = sum_i f_a,i + src_a
// up to one final rounding), as in the 2-D kernels.
template <class T, int M, bool CONS = false>
__device__ __forceinline__ void collide3(const K3<T>& kp, T h[19], T f[M][7], const T Sold[M], T Snew[M]) {
    double mass_in[M];
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) s += (double)f[a][i];
            mass_in[a] = s;
        }
    }
    Mac3<T, M> mc;
    macro3<T, M>(kp, h, f, mc);
    T S[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        S[a] = T(0);
        if (kp.src_mask >> a & 1) {
#pragma unroll
            for (int b = 0; b < M; ++b) S[a] += kp.K[a * M + b] * mc.phi[b];
        }
    }
    // Eq. Gi with cs7^2 = 1/4: G_i = W_i c_i.g / cs7^2 = c_i.g / 2, g_a = sum_b (delta - omega/2)_ab (u S_b + phi_b F)
    T g[M][3];
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
        for (int d = 0; d < 3; ++d) g[a][d] = T(0);
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const T cf = (a == b ? T(1) : T(0)) - T(0.5) * kp.omega[a * M + b];
#pragma unroll
            for (int d = 0; d < 3; ++d) g[a][d] += cf * (mc.u[d] * S[b] + mc.phi[b] * mc.F[d]);
        }
    }
    // f^eq (Eq. feq-phi, lambda = I, vartheta = 0) in deviation form: W_i (phid + 4 phi c.u);
    // the rest direction takes the remainder so that mass is exact
    T feq[M][7], wsrc[M][7], srcv[M];
#pragma unroll
    for (int b = 0; b < M; ++b) {
        const T iso = mc.phid[b] * T(0.125);
        const T adv = T(0.5) * mc.phi[b];  // 4 W_i phi
        feq[b][1] = iso + adv * mc.u[0];
        feq[b][4] = iso - adv * mc.u[0];
        feq[b][2] = iso + adv * mc.u[1];
        feq[b][5] = iso - adv * mc.u[1];
        feq[b][3] = iso + adv * mc.u[2];
        feq[b][6] = iso - adv * mc.u[2];
        feq[b][0] = mc.phid[b] - T(6) * iso;
        const T src = T(1.5) * S[b] - T(0.5) * Sold[b];  // dt S_i + (dt/2)(S_i - S_i(t - dt)) over W_i
        srcv[b] = src;
        Snew[b] = S[b];
        const T s8 = src * T(0.125);
#pragma unroll
        for (int i = 1; i < 7; ++i) wsrc[b][i] = s8;
        wsrc[b][0] = src - T(6) * s8;
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        T neq[M];
#pragma unroll
        for (int b = 0; b < M; ++b) neq[b] = f[b][i] - feq[b][i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            T coll = T(0);
#pragma unroll
            for (int b = 0; b < M; ++b) coll += kp.omega[a * M + b] * neq[b];
            const T cg = T(CX7[i]) * g[a][0] + T(CY7[i]) * g[a][1] + T(CZ7[i]) * g[a][2];
            f[a][i] = f[a][i] - coll + wsrc[a][i] + T(0.5) * cg;
        }
    }
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double moving = 0.0;
#pragma unroll
            for (int i = 1; i < 7; ++i) moving += (double)f[a][i];
            f[a][0] = T((mass_in[a] + (double)srcv[a]) - moving);
        }
    }
    // fluid: h^eq of Eq. heq (rest value by difference: sum_i h^eq = rho0), F_i = 3 W_i c.F
    const T usq = mc.u[0] * mc.u[0] + mc.u[1] * mc.u[1] + mc.u[2] * mc.u[2];
    T heq[19];
    T hsum = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const T cu = T(CX19[i]) * mc.u[0] + T(CY19[i]) * mc.u[1] + T(CZ19[i]) * mc.u[2];
        heq[i] = w19<T>(i) * (T(3) * mc.p + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
        hsum += heq[i];
    }
    heq[0] = kp.rho0_eff - hsum;
    const T w = kp.omega_f, fc = T(1) - T(0.5) * w;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const T cF = T(CX19[i]) * mc.F[0] + T(CY19[i]) * mc.F[1] + T(CZ19[i]) * mc.F[2];
        h[i] = h[i] - w * (h[i] - heq[i]) + fc * (T(3) * w19<T>(i) * cF);
    }
}

// ---- kernels -----------------------------------------------------------------
struct Geo {
    int tile_x, tile_y, tiles_x, tiles_y;
};

__device__ __forceinline__ bool node_of(const Geo& g, int nx, int ny, int& x, int& y, int& z) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % g.tiles_x, r = b / g.tiles_x;
    const int by = r % g.tiles_y;
    z = r / g.tiles_y;
    x = bx * g.tile_x + (int)(threadIdx.x % g.tile_x);
    y = by * g.tile_y + (int)(threadIdx.x / g.tile_x);
    return x < nx && y < ny;
}

template <class S, int M, bool ODD, bool NT>
__global__ __launch_bounds__(256) void k3_step(K3<typename St<S>::T> kp, S* __restrict__ pop,
                                               typename St<S>::T* __restrict__ sold, Geo geo) {
    using T = typename St<S>::T;
    int x, y, z;
    if (!node_of(geo, kp.nx, kp.ny, x, y, z)) return;
    const long long N = (long long)kp.nx * kp.ny * kp.nz;
    const long long n = ((long long)z * kp.ny + y) * kp.nx + x;
    T h[19], f[M][7], So[M], Sn[M];
    gather3<S, M, ODD, NT>(kp, pop, x, y, z, n, h, f);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) So[a] = (kp.src_mask >> a & 1) ? load_raw<NT>(sold + (long long)(k++) * N + n) : T(0);
    collide3<T, M, std::is_same_v<S, float>>(kp, h, f, So, Sn);
    k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a)
        if (kp.src_mask >> a & 1) store_raw<NT>(Sn[a], sold + (long long)(k++) * N + n);
    scatter3<S, M, ODD, NT>(kp, pop, x, y, z, n, h, f);
}

// stage: phi0 [m][N], u0 [3][N], p0 [N] (FP64)
template <class S, int M>
__global__ __launch_bounds__(256) void k3_init(K3<typename St<S>::T> kp, S* __restrict__ pop,
                                               typename St<S>::T* __restrict__ sold, const double* __restrict__ stage,
                                               int has_p0) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny * kp.nz;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T phi[M], u[3];
#pragma unroll
    for (int a = 0; a < M; ++a) phi[a] = T(stage[a * N + n]);
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = T(stage[(M + d) * N + n]);
    const T p = has_p0 ? T(stage[(M + 3) * N + n]) : T(0);
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const T phid = phi[a] - kp.phi_ref[a];
        const T iso = phid * T(0.125), adv = T(0.5) * phi[a];
        st3<false>(pop + p3<M>(19 + 7 * a + 1, n), iso + adv * u[0]);
        st3<false>(pop + p3<M>(19 + 7 * a + 4, n), iso - adv * u[0]);
        st3<false>(pop + p3<M>(19 + 7 * a + 2, n), iso + adv * u[1]);
        st3<false>(pop + p3<M>(19 + 7 * a + 5, n), iso - adv * u[1]);
        st3<false>(pop + p3<M>(19 + 7 * a + 3, n), iso + adv * u[2]);
        st3<false>(pop + p3<M>(19 + 7 * a + 6, n), iso - adv * u[2]);
        st3<false>(pop + p3<M>(19 + 7 * a + 0, n), phid - T(6) * iso);
    }
    // fluid equilibrium at the momentum u0 - F(phi0)/2 (Eq. sum-u then returns u0)
    T j[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        j[d] = u[d] - T(0.5) * kp.F0[d];
#pragma unroll
        for (int a = 0; a < M; ++a) j[d] -= T(0.5) * kp.Fphi[a][d] * phi[a];
    }
    const T usq = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    T hsum = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const T cu = T(CX19[i]) * j[0] + T(CY19[i]) * j[1] + T(CZ19[i]) * j[2];
        const T v = w19<T>(i) * (T(3) * p + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
        hsum += v;
        st3<false>(pop + p3<M>(i, n), v);
    }
    st3<false>(pop + p3<M>(0, n), kp.rho0_eff - hsum);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        if (!(kp.src_mask >> a & 1)) continue;
        T s = T(0);
#pragma unroll
        for (int b = 0; b < M; ++b) s += kp.K[a * M + b] * phi[b];
        sold[(long long)(k++) * N + n] = s;
    }
}

// canonical populations of planes [q0, q0 + nq) into out [nq][N] (FP64, shift
// added back: W_i phi_ref for scalars, rho0 for the rest fluid population)
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k3_export(K3<typename St<S>::T> kp, const S* __restrict__ pop, Geo geo, int q0,
                                                 int nq, double rho0_shift, double* __restrict__ out) {
    using T = typename St<S>::T;
    int x, y, z;
    if (!node_of(geo, kp.nx, kp.ny, x, y, z)) return;
    const long long N = (long long)kp.nx * kp.ny * kp.nz;
    const long long n = ((long long)z * kp.ny + y) * kp.nx + x;
    T h[19], f[M][7];
    gather3<S, M, ODD, false>(kp, pop, x, y, z, n, h, f);
    for (int q = q0; q < q0 + nq; ++q) {
        double v;
        if (q < 19) {
            v = double(h[q]) + (q == 0 ? rho0_shift : 0.0);
        } else {
            const int a = (q - 19) / 7, i = (q - 19) % 7;
            T fv = T(0);
#pragma unroll
            for (int aa = 0; aa < M; ++aa)
#pragma unroll
                for (int ii = 0; ii < 7; ++ii)
                    if (aa == a && ii == i) fv = f[aa][ii];
            v = double(fv) + double(kp.phi_ref[a]) * (i == 0 ? 0.25 : 0.125);
        }
        out[(long long)(q - q0) * N + n] = v;
    }
}

// moments: phi [m][N], u [3][N], p [N] (FP64) into out
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k3_moments(K3<typename St<S>::T> kp, const S* __restrict__ pop, Geo geo,
                                                  double* __restrict__ out) {
    using T = typename St<S>::T;
    int x, y, z;
    if (!node_of(geo, kp.nx, kp.ny, x, y, z)) return;
    const long long N = (long long)kp.nx * kp.ny * kp.nz;
    const long long n = ((long long)z * kp.ny + y) * kp.nx + x;
    T h[19], f[M][7];
    gather3<S, M, ODD, false>(kp, pop, x, y, z, n, h, f);
    Mac3<T, M> mc;
    macro3<T, M>(kp, h, f, mc);
#pragma unroll
    for (int a = 0; a < M; ++a) out[(long long)a * N + n] = double(mc.phi[a]);
#pragma unroll
    for (int d = 0; d < 3; ++d) out[(long long)(M + d) * N + n] = double(mc.u[d]);
    out[(long long)(M + 3) * N + n] = double(mc.p);
}

// per-block totals of phi_a (shifted back) and of the stored h_i; partial [block][M + 1]
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k3_mass(K3<typename St<S>::T> kp, const S* __restrict__ pop, Geo geo,
                                               double* __restrict__ partial) {
    using T = typename St<S>::T;
    int x, y, z;
    double v[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) v[k] = 0.0;
    if (node_of(geo, kp.nx, kp.ny, x, y, z)) {
        const long long n = ((long long)z * kp.ny + y) * kp.nx + x;
        T h[19], f[M][7];
        gather3<S, M, ODD, false>(kp, pop, x, y, z, n, h, f);
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) s += double(f[a][i]);
            v[a] = s + double(kp.phi_ref[a]);
        }
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) s += double(h[i]);
        v[M] = s;
    }
    lbk::block_sum<M + 1>(v, partial + (long long)blockIdx.x * (M + 1));
}

}  // namespace lb3k

// =============================================================================
// host side
// =============================================================================
namespace {

using namespace lb3k;

thread_local std::string g_err3;

lb_status fail3(lb_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lb_status fail3(lb_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err3 = buf;
    return st;
}

#define HIP3(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail3(LB_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                                \
    } while (0)

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout3 {
    size_t N, elem, npop, nsrc, pop_off, sold_off, stage_off, total;
    int stage_planes;
};

int src_mask3(const lb3_params& p) {
    int mask = 0;
    for (int a = 0; a < p.m; ++a)
        for (int b = 0; b < p.m; ++b)
            if (p.K[a * p.m + b] != 0.0) mask |= 1 << a;
    return mask;
}

Layout3 layout3(const lb3_params& p) {
    Layout3 L{};
    L.N = (size_t)p.nx * p.ny * p.nz;
    L.elem = p.storage == LB_STORE_F64 ? 8 : 4;
    L.npop = 19 + 7 * (size_t)p.m;
    int ns = 0;
    for (int a = 0; a < p.m; ++a) ns += (src_mask3(p) >> a) & 1;
    L.nsrc = ns;
    L.stage_planes = p.m + 4;  // init fields; moments; export chunks
    size_t off = 0;
    L.pop_off = off;
    off = round_up(off + round_up(L.N, 64) * L.npop * L.elem, 4096);
    L.sold_off = off;
    off = round_up(off + L.nsrc * L.N * L.elem, 4096);
    L.stage_off = off;
    off = round_up(off + (size_t)L.stage_planes * L.N * 8, 4096);
    L.total = off;
    return L;
}

bool finite_all3(const double* v, size_t n) {
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

// real parts of the eigenvalues of a small matrix (m <= 4), from the
// characteristic polynomial (Faddeev-LeVerrier) and Durand-Kerner roots
void eig_real_parts(int m, const double* A, double* re) {
    double c[LB_MAX_M + 1];
    double Mk[LB_MAX_M * LB_MAX_M] = {0};
    c[0] = 1.0;
    for (int k = 1; k <= m; ++k) {
        double Mn[LB_MAX_M * LB_MAX_M];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double s = (i == j) ? c[k - 1] : 0.0;
                for (int l = 0; l < m; ++l) s += A[i * m + l] * Mk[l * m + j];
                Mn[i * m + j] = s;
            }
        std::memcpy(Mk, Mn, sizeof Mn);
        double tr = 0.0;
        for (int i = 0; i < m; ++i)
            for (int l = 0; l < m; ++l) tr += A[i * m + l] * Mk[l * m + i];
        c[k] = -tr / k;
    }
    std::complex<double> z[LB_MAX_M];
    double scale = 1e-300;
    for (int k = 0; k < m * m; ++k) scale = std::max(scale, std::fabs(A[k]));
    for (int k = 0; k < m; ++k) z[k] = scale * std::pow(std::complex<double>(0.4, 0.9), k);
    for (int it = 0; it < 500; ++it)
        for (int k = 0; k < m; ++k) {
            std::complex<double> num = 1.0, den = 1.0;
            for (int j = 1; j <= m; ++j) num = num * z[k] + c[j];
            for (int j = 0; j < m; ++j)
                if (j != k) den *= (z[k] - z[j]);
            if (std::abs(den) > 0) z[k] -= num / den;
        }
    for (int k = 0; k < m; ++k) re[k] = z[k].real();
}

bool invert3(int m, const double* A, double* out) {
    double w[LB_MAX_M][2 * LB_MAX_M];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 2 * m; ++j) w[i][j] = j < m ? A[i * m + j] : (j - m == i ? 1.0 : 0.0);
    for (int k = 0; k < m; ++k) {
        int pv = k;
        for (int i = k + 1; i < m; ++i)
            if (std::fabs(w[i][k]) > std::fabs(w[pv][k])) pv = i;
        if (w[pv][k] == 0.0) return false;
        for (int j = 0; j < 2 * m; ++j) std::swap(w[k][j], w[pv][j]);
        const double d = w[k][k];
        for (int j = 0; j < 2 * m; ++j) w[k][j] /= d;
        for (int i = 0; i < m; ++i)
            if (i != k) {
                const double s = w[i][k];
                for (int j = 0; j < 2 * m; ++j) w[i][j] -= s * w[k][j];
            }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) out[i * m + j] = w[i][m + j];
    return true;
}

lb_status validate3(const lb3_params* p) {
    if (!p) return fail3(LB_EINVAL, "params is NULL");
    if (p->nx < 2 || p->ny < 2 || p->nz < 2)
        return fail3(LB_EINVAL, "grid %d x %d x %d: each side must be >= 2", p->nx, p->ny, p->nz);
    if ((long long)p->nx * p->ny * p->nz > (1ll << 31) - 1) return fail3(LB_EINVAL, "grid too large");
    if (p->m < 1 || p->m > LB_MAX_M) return fail3(LB_EINVAL, "m = %d outside 1..%d", p->m, LB_MAX_M);
    // neighbour offsets within a row are formed in 32-bit arithmetic
    if (((long long)p->nx + 64) * (19 + 7 * p->m) > (1ll << 31) - 1)
        return fail3(LB_EINVAL, "grid %d wide: (nx + 64) (19 + 7m) must stay below 2^31", p->nx);
    if (p->storage != LB_STORE_F64 && p->storage != LB_STORE_F32) return fail3(LB_EINVAL, "storage must be F64 or F32");
    if (!(p->tau_f > 0.5) || !std::isfinite(p->tau_f)) return fail3(LB_EINVAL, "tau_f = %g must be > 1/2", p->tau_f);
    if (!std::isfinite(p->rho0)) return fail3(LB_EINVAL, "rho0 not finite");
    for (int s = 0; s < 6; ++s) {
        if (p->fluid_bc[s] != LB_BC_PERIODIC && p->fluid_bc[s] != LB_BC_NOSLIP)
            return fail3(LB_EINVAL, "fluid_bc[%d]: periodic or no-slip", s);
        for (int a = 0; a < p->m; ++a) {
            if (p->scalar_bc[s][a] < 0 || p->scalar_bc[s][a] > 2) return fail3(LB_EINVAL, "scalar_bc[%d][%d] invalid", s, a);
            if (!std::isfinite(p->wall[s][a])) return fail3(LB_EINVAL, "wall[%d][%d] not finite", s, a);
        }
    }
    for (int axis = 0; axis < 3; ++axis) {
        const int s0 = 2 * axis, s1 = s0 + 1;
        const bool per = p->fluid_bc[s0] == LB_BC_PERIODIC;
        if ((p->fluid_bc[s1] == LB_BC_PERIODIC) != per)
            return fail3(LB_EINVAL, "periodic fluid sides must come in pairs (axis %d)", axis);
        for (int a = 0; a < p->m; ++a)
            if ((p->scalar_bc[s0][a] == LB_SBC_PERIODIC) != per || (p->scalar_bc[s1][a] == LB_SBC_PERIODIC) != per)
                return fail3(LB_EINVAL, "scalar %d periodicity on axis %d must match the fluid", a, axis);
    }
    const int m = p->m;
    if (!finite_all3(p->D, (size_t)m * m) || !finite_all3(p->K, (size_t)m * m) || !finite_all3(p->F0, 3) ||
        !finite_all3(&p->Fphi[0][0], (size_t)m * 3) || !finite_all3(p->phi_ref, (size_t)m))
        return fail3(LB_EINVAL, "D, K, F or phi_ref not finite");
    double re[LB_MAX_M];
    eig_real_parts(m, p->D, re);
    for (int k = 0; k < m; ++k)
        if (!(re[k] > 0.0)) return fail3(LB_EINVAL, "D has an eigenvalue with real part %g <= 0", re[k]);
    return LB_OK;
}

template <class T>
void fill3(const lb3_params& p, K3<T>& k) {
    std::memset(&k, 0, sizeof k);
    const bool shifted = p.storage != LB_STORE_F64;
    k.nx = p.nx;
    k.ny = p.ny;
    k.nz = p.nz;
    k.px = p.fluid_bc[0] == LB_BC_PERIODIC;
    k.py = p.fluid_bc[2] == LB_BC_PERIODIC;
    k.pz = p.fluid_bc[4] == LB_BC_PERIODIC;
    for (int s = 0; s < 6; ++s)
        for (int a = 0; a < p.m; ++a) {
            k.sbc[s][a] = p.scalar_bc[s][a];
            k.wallr[s][a] = T(p.wall[s][a] - (shifted ? p.phi_ref[a] : 0.0));
        }
    k.src_mask = src_mask3(p);
    k.omega_f = T(1.0 / p.tau_f);
    k.rho0_eff = T(shifted ? 0.0 : p.rho0);
    const int m = p.m;
    double A[LB_MAX_M * LB_MAX_M], om[LB_MAX_M * LB_MAX_M];
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) A[a * m + b] = 4.0 * p.D[a * m + b] + (a == b ? 0.5 : 0.0);  // D / cs7^2 + I/2
    invert3(m, A, om);
    for (int q = 0; q < m * m; ++q) {
        k.omega[q] = T(om[q]);
        k.K[q] = T(p.K[q]);
    }
    for (int d = 0; d < 3; ++d) k.F0[d] = T(p.F0[d]);
    for (int a = 0; a < m; ++a) {
        for (int d = 0; d < 3; ++d) k.Fphi[a][d] = T(p.Fphi[a][d]);
        k.phi_ref[a] = T(shifted ? p.phi_ref[a] : 0.0);
    }
}

// per-species kernel dispatch: S in {double, float}, M in 1..4
template <class F>
hipError_t dispatch3(const lb3_params& p, F&& fn) {
    auto by_m = [&]<class S>() -> hipError_t {
        switch (p.m) {
            case 1: return fn.template operator()<S, 1>();
            case 2: return fn.template operator()<S, 2>();
            case 3: return fn.template operator()<S, 3>();
            default: return fn.template operator()<S, 4>();
        }
    };
    return p.storage == LB_STORE_F64 ? by_m.template operator()<double>() : by_m.template operator()<float>();
}

constexpr size_t kNtMax3 = size_t(64) << 20;

}  // namespace

struct lb3_handle {
    lb3_params p;
    Layout3 L;
    K3<double> kd;
    K3<float> kf;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    int64_t t;
    int tile_x, tile_y;
    int nt_bits;  // bit 0: hint on even steps, bit 1: on odd steps
    std::vector<double> part_host;  // per-block totals of lb3_mass
    // cached graph of kGraphSteps3 step launches (even parity first) for long runs; rebuilt
    // when the tile shape changes
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_tx = 0, g_ty = 0;
    ~lb3_handle() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

void* at3(void* base, size_t off) { return static_cast<char*>(base) + off; }

template <class S>
const K3<typename St<S>::T>& kpar3(const lb3_handle* h) {
    if constexpr (std::is_same_v<typename St<S>::T, double>)
        return h->kd;
    else
        return h->kf;
}

Geo geo_of(const lb3_handle* h) {
    Geo g;
    g.tile_x = h->tile_x;
    g.tile_y = h->tile_y;
    g.tiles_x = (h->p.nx + h->tile_x - 1) / h->tile_x;
    g.tiles_y = (h->p.ny + h->tile_y - 1) / h->tile_y;
    return g;
}

unsigned grid_of(const lb3_handle* h, const Geo& g) { return (unsigned)(g.tiles_x * g.tiles_y * h->p.nz); }

hipError_t launch3_step(lb3_handle* h, bool odd) {
    const Geo g = geo_of(h);
    const dim3 grid(grid_of(h, g)), block((unsigned)(h->tile_x * h->tile_y));
    const bool nt = (h->nt_bits >> (odd ? 1 : 0)) & 1;
    return dispatch3(h->p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at3(h->ws, h->L.pop_off);
        T* sold = (T*)at3(h->ws, h->L.sold_off);
        const auto& kp = kpar3<S>(h);
        if (odd) {
            if (nt)
                hipLaunchKernelGGL((k3_step<S, M, true, true>), grid, block, 0, h->stream, kp, pop, sold, g);
            else
                hipLaunchKernelGGL((k3_step<S, M, true, false>), grid, block, 0, h->stream, kp, pop, sold, g);
        } else {
            if (nt)
                hipLaunchKernelGGL((k3_step<S, M, false, true>), grid, block, 0, h->stream, kp, pop, sold, g);
            else
                hipLaunchKernelGGL((k3_step<S, M, false, false>), grid, block, 0, h->stream, kp, pop, sold, g);
        }
        return hipGetLastError();
    });
}

// a graph of `steps` (even) step launches, even parity first, chained, built node by node
// (the launches of one parity have the same arguments: populations and sources in place)
constexpr int kGraphSteps3 = 64;
hipError_t build3_step_graph(lb3_handle* h, int steps, hipGraph_t* out) {
    const Geo g = geo_of(h);
    const dim3 grid(grid_of(h, g)), block((unsigned)(h->tile_x * h->tile_y));
    hipGraph_t gr = nullptr;
    hipError_t e = hipGraphCreate(&gr, 0);
    if (e != hipSuccess) return e;
    e = dispatch3(h->p, [&]<class S, int M>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at3(h->ws, h->L.pop_off);
        T* sold = (T*)at3(h->ws, h->L.sold_off);
        K3<T> kp = kpar3<S>(h);
        Geo geo = g;
        void* args[] = {&kp, &pop, &sold, &geo};
        void* fe = reinterpret_cast<void*>((h->nt_bits & 1) ? &k3_step<S, M, false, true> : &k3_step<S, M, false, false>);
        void* fo = reinterpret_cast<void*>((h->nt_bits & 2) ? &k3_step<S, M, true, true> : &k3_step<S, M, true, false>);
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
            hipError_t ee = hipGraphAddKernelNode(&node, gr, prev ? &prev : nullptr, prev ? 1 : 0, &np);
            if (ee != hipSuccess) return ee;
            prev = node;
        }
        return hipSuccess;
    });
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return e;
    }
    *out = gr;
    return hipSuccess;
}

lb_status check_handle(lb3_handle* h) {
    if (!h) return fail3(LB_EINVAL, "handle is NULL");
    return LB_OK;
}

}  // namespace

extern "C" {

const char* lb3_last_error(void) { return g_err3.c_str(); }
size_t lb3_params_bytes(void) { return sizeof(lb3_params); }

lb_status lb3_workspace_bytes(const lb3_params* params, size_t* bytes) {
    lb_status st = validate3(params);
    if (st != LB_OK) return st;
    if (!bytes) return fail3(LB_EINVAL, "bytes is NULL");
    *bytes = layout3(*params).total;
    return LB_OK;
}

lb_status lb3_init(const lb3_params* params, void* ws, size_t ws_bytes, void* stream, const double* phi0,
                   const double* u0, const double* p0, lb3_handle** out) {
    if (out) *out = nullptr;
    lb_status st = validate3(params);
    if (st != LB_OK) return st;
    if (!out || !phi0 || !u0) return fail3(LB_EINVAL, "out, phi0 and u0 are required");
    if (!ws) return fail3(LB_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail3(LB_EINVAL, "workspace must be 256-byte aligned");
    const Layout3 L = layout3(*params);
    if (ws_bytes < L.total) return fail3(LB_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
    const size_t N = L.N;
    const int m = params->m;
    if (!finite_all3(phi0, (size_t)m * N) || !finite_all3(u0, 3 * N) || (p0 && !finite_all3(p0, N)))
        return fail3(LB_ENONFINITE, "initial fields are not finite");
    lb3_handle* h = new (std::nothrow) lb3_handle();
    if (!h) return fail3(LB_ENOMEM, "no host memory for the handle");
    h->p = *params;
    h->L = L;
    h->ws = ws;
    h->ws_bytes = ws_bytes;
    h->stream = (hipStream_t)stream;
    h->t = 0;
    // measured at 256^3: FP64 best with whole 256-node rows (1569 us; 64 x 4: 1575 us),
    // FP32 with 64 x 4 (771 us; 256 x 1: 788 us)
    h->tile_x = (params->nx >= 256 && params->storage == LB_STORE_F64) ? 256 : 64;
    h->tile_y = 256 / h->tile_x;
    h->nt_bits = round_up(N, 64) * L.npop * L.elem <= kNtMax3 ? 3 : 1;
    fill3(*params, h->kd);
    fill3(*params, h->kf);
    double* stage = (double*)at3(ws, L.stage_off);
    auto bail = [&](lb_status s) {
        delete h;
        return s;
    };
    hipError_t e = hipMemcpyAsync(stage, phi0, (size_t)m * N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + (size_t)m * N, u0, 3 * N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && p0) e = hipMemcpyAsync(stage + (size_t)(m + 3) * N, p0, N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        e = dispatch3(*params, [&]<class S, int M>() -> hipError_t {
            using T = typename St<S>::T;
            hipLaunchKernelGGL((k3_init<S, M>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, h->stream, kpar3<S>(h),
                               (S*)at3(ws, L.pop_off), (T*)at3(ws, L.sold_off), (const double*)stage, p0 ? 1 : 0);
            return hipGetLastError();
        });
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(fail3(LB_EDEVICE, "lb3_init: %s", hipGetErrorString(e)));
    *out = h;
    return LB_OK;
}

lb_status lb3_step(lb3_handle* h, int64_t n) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    if (n < 0) return fail3(LB_EINVAL, "n = %lld < 0", (long long)n);
    // long runs: replay a prebuilt graph of kGraphSteps3 launches (one host call each)
    if (n >= kGraphSteps3 + (h->t & 1)) {
        if (h->t & 1) {
            HIP3(launch3_step(h, true));
            ++h->t;
            --n;
        }
        if (!h->gexec || h->g_tx != h->tile_x || h->g_ty != h->tile_y) {
            if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
            if (h->graph) (void)hipGraphDestroy(h->graph);
            h->gexec = nullptr;
            h->graph = nullptr;
            HIP3(build3_step_graph(h, kGraphSteps3, &h->graph));
            HIP3(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
            h->g_tx = h->tile_x;
            h->g_ty = h->tile_y;
        }
        for (; n >= kGraphSteps3; n -= kGraphSteps3) {
            HIP3(hipGraphLaunch(h->gexec, h->stream));
            h->t += kGraphSteps3;
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        HIP3(launch3_step(h, (h->t & 1) != 0));
        ++h->t;
    }
    return LB_OK;
}

lb_status lb3_time(lb3_handle* h, int64_t* t) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    if (!t) return fail3(LB_EINVAL, "t is NULL");
    *t = h->t;
    return LB_OK;
}

lb_status lb3_set_tile(lb3_handle* h, int32_t tile_x, int32_t tile_y) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    const int th = tile_x * tile_y;
    if (tile_x < 1 || tile_y < 1 || th > 256 || th % 64)
        return fail3(LB_EINVAL, "tile %d x %d: product must be a multiple of 64, at most 256", tile_x, tile_y);
    h->tile_x = tile_x;
    h->tile_y = tile_y;
    return LB_OK;
}

lb_status lb3_moments(lb3_handle* h, double* phi, double* u, double* p) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    const size_t N = h->L.N;
    const int m = h->p.m;
    double* stage = (double*)at3(h->ws, h->L.stage_off);
    const Geo g = geo_of(h);
    const bool odd = (h->t & 1) != 0;  // an even number of steps leaves the canonical layout
    HIP3(dispatch3(h->p, [&]<class S, int M>() -> hipError_t {
        const S* pop = (const S*)at3(h->ws, h->L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k3_moments<S, M, true>), dim3(grid_of(h, g)), dim3(h->tile_x * h->tile_y), 0, h->stream,
                               kpar3<S>(h), pop, g, stage);
        else
            hipLaunchKernelGGL((k3_moments<S, M, false>), dim3(grid_of(h, g)), dim3(h->tile_x * h->tile_y), 0,
                               h->stream, kpar3<S>(h), pop, g, stage);
        return hipGetLastError();
    }));
    if (phi) HIP3(hipMemcpyAsync(phi, stage, (size_t)m * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (u) HIP3(hipMemcpyAsync(u, stage + (size_t)m * N, 3 * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (p) HIP3(hipMemcpyAsync(p, stage + (size_t)(m + 3) * N, N * 8, hipMemcpyDeviceToHost, h->stream));
    HIP3(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status lb3_populations(lb3_handle* h, double* f, double* hpop) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    const size_t N = h->L.N;
    const int m = h->p.m;
    double* stage = (double*)at3(h->ws, h->L.stage_off);
    const Geo g = geo_of(h);
    const bool odd = (h->t & 1) != 0;
    const double shift = h->p.storage == LB_STORE_F64 ? 0.0 : h->p.rho0;
    const int total = 19 + 7 * m, chunk = h->L.stage_planes;
    for (int q0 = 0; q0 < total; q0 += chunk) {
        const int nq = std::min(chunk, total - q0);
        HIP3(dispatch3(h->p, [&]<class S, int M>() -> hipError_t {
            const S* pop = (const S*)at3(h->ws, h->L.pop_off);
            if (odd)
                hipLaunchKernelGGL((k3_export<S, M, true>), dim3(grid_of(h, g)), dim3(h->tile_x * h->tile_y), 0,
                                   h->stream, kpar3<S>(h), pop, g, q0, nq, shift, stage);
            else
                hipLaunchKernelGGL((k3_export<S, M, false>), dim3(grid_of(h, g)), dim3(h->tile_x * h->tile_y), 0,
                                   h->stream, kpar3<S>(h), pop, g, q0, nq, shift, stage);
            return hipGetLastError();
        }));
        for (int q = q0; q < q0 + nq; ++q) {
            double* dst = q < 19 ? (hpop ? hpop + (size_t)q * N : nullptr) : (f ? f + (size_t)(q - 19) * N : nullptr);
            if (dst) HIP3(hipMemcpyAsync(dst, stage + (size_t)(q - q0) * N, N * 8, hipMemcpyDeviceToHost, h->stream));
        }
        HIP3(hipStreamSynchronize(h->stream));
    }
    return LB_OK;
}

lb_status lb3_mass(lb3_handle* h, double* mass) {
    if (lb_status s = check_handle(h); s != LB_OK) return s;
    if (!mass) return fail3(LB_EINVAL, "mass is NULL");
    const int m = h->p.m;
    const Geo g = geo_of(h);
    const unsigned nb = grid_of(h, g);
    // the per-block partial sums use the stage area: (m + 1) doubles per block
    // fit, since a block covers at least 64 nodes and the stage holds m + 4
    // doubles per node
    double* part = (double*)at3(h->ws, h->L.stage_off);
    const bool odd = (h->t & 1) != 0;
    HIP3(dispatch3(h->p, [&]<class S, int M>() -> hipError_t {
        const S* pop = (const S*)at3(h->ws, h->L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k3_mass<S, M, true>), dim3(nb), dim3(h->tile_x * h->tile_y), 0, h->stream, kpar3<S>(h),
                               pop, g, part);
        else
            hipLaunchKernelGGL((k3_mass<S, M, false>), dim3(nb), dim3(h->tile_x * h->tile_y), 0, h->stream, kpar3<S>(h),
                               pop, g, part);
        return hipGetLastError();
    }));
    h->part_host.resize((size_t)nb * (m + 1));
    HIP3(hipMemcpyAsync(h->part_host.data(), part, h->part_host.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIP3(hipStreamSynchronize(h->stream));
    for (int k = 0; k <= m; ++k) mass[k] = 0.0;
    for (unsigned b = 0; b < nb; ++b)
        for (int k = 0; k <= m; ++k) mass[k] += h->part_host[(size_t)b * (m + 1) + k];
    if (h->p.storage != LB_STORE_F64) mass[m] += h->p.rho0 * (double)h->L.N;
    for (int k = 0; k <= m; ++k)
        if (!std::isfinite(mass[k])) return fail3(LB_ENONFINITE, "total %d is not finite", k);
    return LB_OK;
}

lb_status lb3_free(lb3_handle* h) {
    delete h;
    return LB_OK;
}

}  // extern "C"
