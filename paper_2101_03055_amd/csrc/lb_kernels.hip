// lb_kernels.hip -- gfx950 kernels of the coupled cross-diffusion-fluid lattice
// Boltzmann step (Zhan, Chai & Shi, arXiv 2101.03055, Sec. 2).
//
// One thread updates one node: it gathers the 9 fluid and 5m scalar
// populations, forms the moments (Eq. sum), the relaxation matrix (Eq. omega-D),
// the source with its time-derivative correction (Eq. source), the auxiliary
// source (Eq. Gi) and the force term (Eq. force), collides (Eqs. evolution12,
// evolution3 or MRT) and scatters the results.  Streaming is the in-place AA
// pattern over a structure-of-arrays layout [plane][ny][nx]:
//   even step: read own slots i, write post-collision values to own slots opp(i);
//   odd step : read slot opp(i) of the upstream neighbour x - c_i, write slot i
//              of the downstream neighbour x + c_i.
// Each node reads and writes the same set of locations in both steps, so one
// array suffices and no two threads touch the same word.  Wall links are
// resolved only in the odd step: at the read (a population that would come
// from outside is the reflected post-collision value the even step left in
// the node's own slot) and at the write (a population leaving through a wall
// is written where the next even step reads its reflection).
//
// Reduced-precision storage keeps deviations: f - W_i phi_ref and h - rho0
// delta_i0 (the He-Shi-Guo equilibrium carries rho0 in sigma_0 only), in FP32,
// or scaled by fp16_scale in binary16.  The arithmetic then runs on
// deviations in FP32: it is the FP64 update with phi_ref and rho0 moved out.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lb_device.h"

namespace lbk {

// ---- kernels ------------------------------------------------------------------
// REF: the odd (streaming) parity re-references fluid values that cross rows
// to a per-row pressure (kp.pref non-null); the even parity never crosses rows
template <class S, int M, int MODEL, int COLL, bool ODD, bool NT, bool REF>
__global__ __launch_bounds__(256) void k_step(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                              const typename St<S>::T* sold, typename St<S>::T* sold_out,
                                              int tile_x, int tile_y, int tiles_x, uint32_t salt,
                                              const long long* __restrict__ tstep) {
    using T = typename St<S>::T;
    salt = launch_salt<S>(salt, tstep);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % tiles_x, by = b / tiles_x;
    const int x = bx * tile_x + (int)(threadIdx.x % tile_x);
    const int y = by * tile_y + (int)(threadIdx.x / tile_x);
    if (x >= kp.nx || y >= kp.ny) return;
    const long long n = (long long)y * kp.nx + x;

    const long long N = (long long)kp.nx * kp.ny;
    T h[9], f[M][5], Sold[M], Snew[M];
    gather<S, M, ODD, NT, REF>(kp, pop, x, y, h, f);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        Sold[a] = T(0);
        if (kp.src_mask >> a & 1) Sold[a] = load_raw<NT>(&sold[(long long)(k++) * N + n]);
    }
    // gamma of D-bar (Eq. evolution12): central differences of the previous
    // step's source field (`sold`, not written by this launch when gamma != 0);
    // across a wall the node's own value stands in for the missing neighbour
    T gS[M][2];
#pragma unroll
    for (int a = 0; a < M; ++a) gS[a][0] = gS[a][1] = T(0);
    if (kp.gam_on) {
        k = 0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            if (kp.src_mask >> a & 1) {
                const T* pl = sold + (long long)(k++) * N;
                const long long xp = x + 1 < kp.nx ? n + 1 : (kp.sbc[1][a] == LB_SBC_PERIODIC ? n + 1 - kp.nx : n);
                const long long xm = x > 0 ? n - 1 : (kp.sbc[0][a] == LB_SBC_PERIODIC ? n - 1 + kp.nx : n);
                const long long yp = y + 1 < kp.ny ? n + kp.nx : (kp.sbc[3][a] == LB_SBC_PERIODIC ? n + kp.nx - N : n);
                const long long ym = y > 0 ? n - kp.nx : (kp.sbc[2][a] == LB_SBC_PERIODIC ? n - kp.nx + N : n);
                gS[a][0] = kp.gam12[a] * (pl[xp] - pl[xm]);
                gS[a][1] = kp.gam12[a] * (pl[yp] - pl[ym]);
            }
        }
    }
    collide<T, M, MODEL, COLL, std::is_same_v<S, float>>(kp, h, f, Sold, Snew, gS);
    k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a)
        if (kp.src_mask >> a & 1) store_raw<NT>(Snew[a], &sold_out[(long long)(k++) * N + n]);
    scatter<S, M, ODD, NT, REF>(kp, pop, x, y, h, f, salt);
}

// the step kernel for a collision kind, parity, cache hint and fluid reference
template <class S, int M, int MODEL>
static const void* step_kernel(bool mrt, bool odd, bool nt, bool ref) {
    const void* const fns[12] = {
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, false, false, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, false, true, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, true, false, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, true, true, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, false, false, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, false, true, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, true, false, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, true, true, false>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, true, false, true>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_BGK, true, true, true>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, true, false, true>),
        reinterpret_cast<const void*>(&k_step<S, M, MODEL, LB_COLL_MRT, true, true, true>)};
    if (odd && ref) return fns[8 + (mrt ? 2 : 0) + (nt ? 1 : 0)];
    return fns[(mrt ? 4 : 0) + (odd ? 2 : 0) + (nt ? 1 : 0)];
}

// ---- two steps per launch (temporal blocking through LDS) -----------------
// Reads the canonical state at t (own slots) of a tile plus a 2-node ring
// from `src`, collides every node of that region (step 1) into LDS buffer 1,
// streams inside LDS (with the wall rules) and collides the tile plus a
// 1-node ring (step 2) into LDS buffer 2, then streams once more and writes
// the canonical state at t + 2 of the tile to `dst` (own slots).  src/dst and
// the previous-step source planes are ping-pong pairs: neighbouring
// workgroups read the ring of this tile from `src` while it is updated.
// Each state value therefore crosses HBM once per two steps.
template <int TX, int TY>
struct Tb2Geom {
    static constexpr int RX = TX + 4, RY = TY + 4;  // region of step 1 (ring 2)
    static constexpr int R1X = TX + 2, R1Y = TY + 2;  // region of step 2 (ring 1)
};

__device__ __forceinline__ bool node_exists(int& gx, int& gy, int nx, int ny, int px, int py) {
    const bool inx = wrap_in(gx, nx, px), iny = wrap_in(gy, ny, py);
    return inx && iny;
}

// Pull of the pre-collision populations of local node (lx, ly) from the
// post-collision values in an LDS buffer of pitch BX (rows) with origin
// (ox, oy) relative to the step-1 region; ex(lx, ly) tells whether a local
// node exists in the domain.  Same wall rules as gather<.., true>.
template <class T, int M, int NQ, class ExFn>
__device__ __forceinline__ void lds_pull(const KParams<T>& kp, const T* __restrict__ buf, int BX, int BN, int lx,
                                         int ly, ExFn&& ex, T h[9], T f[M][5]) {
    auto at = [&](int q, int x, int y) -> T { return buf[q * BN + y * BX + x]; };
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = lx - CX9[i], sy = ly - CY9[i];
        int ox, oy;
        const int e = ex(sx, sy, ox, oy);  // bit 0: exists; ox, oy: side flags
        T v;
        if (e) {
            v = at(i, sx, sy);
        } else {
            v = at(OPP9[i], lx, ly);  // bounce-back
            if ((ox >= 0) != (oy >= 0)) {
                const int side = ox >= 0 ? ox : oy;
                if (kp.fbc[side] == LB_BC_FREESLIP) {
                    int ax, ay;
                    if (oy >= 0) {
                        if (ex(lx - CX9[i], ly, ax, ay)) v = at(MIRY9[i], lx - CX9[i], ly);
                    } else {
                        if (ex(lx, ly - CY9[i], ax, ay)) v = at(MIRX9[i], lx, ly - CY9[i]);
                    }
                }
            }
        }
        h[i] = v;
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const int sx = lx - CX5[i], sy = ly - CY5[i];
            int ox, oy;
            if (ex(sx, sy, ox, oy)) {
                f[a][i] = at(9 + 5 * a + i, sx, sy);
            } else {
                const int side = ox >= 0 ? ox : oy;
                T v = at(9 + 5 * a + OPP5[i], lx, ly);
                if (kp.sbc[side][a] == LB_SBC_DIRICHLET) v = -v + T(2) * w5<T>(i) * kp.wallr[side][a];
                f[a][i] = v;
            }
        }
}

template <class S, int M, int MODEL, int COLL, int TX, int TY>
__global__ __launch_bounds__(256) void k_step2(KParams<typename St<S>::T> kp, const S* __restrict__ src,
                                               S* __restrict__ dst, const typename St<S>::T* __restrict__ sold_src,
                                               typename St<S>::T* __restrict__ sold_dst, int tiles_x,
                                               uint32_t salt) {
    using T = typename St<S>::T;
    using G = Tb2Geom<TX, TY>;
    constexpr int NQ = 9 + 5 * M;
    constexpr int N1 = G::RX * G::RY, N2 = G::R1X * G::R1Y;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T* buf1 = reinterpret_cast<T*>(smem);    // [NQ][RY][RX] post-collision, step 1
    T* buf2 = buf1 + NQ * N1;                 // [NQ][R1Y][R1X] post-collision, step 2
    T* sb = buf2 + NQ * N2;                   // [M][RY][RX] source after step 1 / [M][R1Y][R1X] after step 2
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % tiles_x, by = b / tiles_x;
    const int x0 = bx * TX - 2, y0 = by * TY - 2;  // global origin of the step-1 region
    const int nx = kp.nx, ny = kp.ny;
    const long long N = (long long)nx * ny;
    // existence of a step-1-region node, with the side it lies beyond on each axis (-1: inside/periodic)
    auto ex1 = [&](int lx, int ly, int& ox, int& oy) -> int {
        int gx = x0 + lx, gy = y0 + ly;
        const bool inx = wrap_in(gx, nx, kp.px), iny = wrap_in(gy, ny, kp.py);
        ox = inx ? -1 : side_x(gx);
        oy = iny ? -1 : side_y(gy);
        return inx & iny;
    };

    // phase A: load + collide (step 1) on the ring-2 region
    for (int r = threadIdx.x; r < N1; r += blockDim.x) {
        const int lx = r % G::RX, ly = r / G::RX;
        int gx = x0 + lx, gy = y0 + ly;
        if (!node_exists(gx, gy, nx, ny, kp.px, kp.py)) continue;
        const long long n = (long long)gy * nx + gx;
        T h[9], f[M][5], So[M], Sn[M];
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = ld(src + pidx<M>(i, n), kp, true);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) f[a][i] = ld(src + pidx<M>((9 + 5 * a + i), n), kp, false);
        int k = 0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
            So[a] = T(0);
            if (kp.src_mask >> a & 1) So[a] = sold_src[(long long)(k++) * N + n];
        }
        collide<T, M, MODEL, COLL, std::is_same_v<S, float>>(kp, h, f, So, Sn);
#pragma unroll
        for (int i = 0; i < 9; ++i) buf1[i * N1 + r] = h[i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
#pragma unroll
            for (int i = 0; i < 5; ++i) buf1[(9 + 5 * a + i) * N1 + r] = f[a][i];
            sb[a * N1 + r] = Sn[a];
        }
    }
    __syncthreads();
    // phase B: stream (in LDS) + collide (step 2) on the ring-1 region
    T* sb2 = sb + M * N1;
    for (int r = threadIdx.x; r < N2; r += blockDim.x) {
        const int lx = 1 + r % G::R1X, ly = 1 + r / G::R1X;
        int ox, oy;
        if (!ex1(lx, ly, ox, oy)) continue;
        T h[9], f[M][5], So[M], Sn[M];
        lds_pull<T, M, NQ>(kp, buf1, G::RX, N1, lx, ly, ex1, h, f);
#pragma unroll
        for (int a = 0; a < M; ++a) So[a] = sb[a * N1 + ly * G::RX + lx];
        collide<T, M, MODEL, COLL, std::is_same_v<S, float>>(kp, h, f, So, Sn);
#pragma unroll
        for (int i = 0; i < 9; ++i) buf2[i * N2 + r] = h[i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
#pragma unroll
            for (int i = 0; i < 5; ++i) buf2[(9 + 5 * a + i) * N2 + r] = f[a][i];
            sb2[a * N2 + r] = Sn[a];
        }
    }
    __syncthreads();
    // phase C: stream (in LDS) into the tile and write the canonical state at t + 2
    auto ex2 = [&](int lx, int ly, int& ox, int& oy) -> int { return ex1(lx + 1, ly + 1, ox, oy); };
    for (int r = threadIdx.x; r < TX * TY; r += blockDim.x) {
        const int tx = r % TX, ty = r / TX;
        const int gx = x0 + 2 + tx, gy = y0 + 2 + ty;
        if (gx >= nx || gy >= ny) continue;
        const long long n = (long long)gy * nx + gx;
        T h[9], f[M][5];
        lds_pull<T, M, NQ>(kp, buf2, G::R1X, N2, tx + 1, ty + 1, ex2, h, f);
#pragma unroll
        for (int i = 0; i < 9; ++i) st(dst, pidx<M>(i, n), h[i], kp, true, salt);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) st(dst, pidx<M>((9 + 5 * a + i), n), f[a][i], kp, false, salt);
        int k = 0;
#pragma unroll
        for (int a = 0; a < M; ++a)
            if (kp.src_mask >> a & 1) sold_dst[(long long)(k++) * N + n] = sb2[a * N2 + (ty + 1) * G::R1X + tx + 1];
    }
}

// initial state: f = f^eq(phi0, u0), h = h^eq(p0, u0), S_old = S(phi0)
template <class S, int M, int MODEL>
__global__ __launch_bounds__(256) void k_init(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                              typename St<S>::T* __restrict__ sold,
                                              const double* __restrict__ stage, int has_p0) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    T phi[M], u[2];
#pragma unroll
    for (int a = 0; a < M; ++a) phi[a] = T(stage[a * N + n]);
    u[0] = T(stage[M * N + n]);
    u[1] = T(stage[(M + 1) * N + n]);
    // the fluid values are stored relative to the row's reference equilibrium (pressure P(y)),
    // and h^eq is linear in p: the stored equilibrium is h^eq at p - P(y)
    const T p = (has_p0 ? T(stage[(M + 2) * N + n]) : T(0)) - (kp.pref ? kp.pref[n / kp.nx] : T(0));
    const uint32_t salt = 0x51ed270bu;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const T phid = phi[a] - kp.phi_ref[a];
        T pd = phid;
        if constexpr (MODEL != LB_MODEL_CHEMOTAXIS)
            if (kp.lam_on) pd += lam_excess<T, M>(kp, phi, a);
        const T iso = pd * (T(1) / T(6));
        const T adv = T(0.5) * phi[a];
        st(pop, pidx<M>((9 + 5 * a + 1), n), iso + adv * u[0], kp, false, salt);
        st(pop, pidx<M>((9 + 5 * a + 3), n), iso - adv * u[0], kp, false, salt);
        st(pop, pidx<M>((9 + 5 * a + 2), n), iso + adv * u[1], kp, false, salt);
        st(pop, pidx<M>((9 + 5 * a + 4), n), iso - adv * u[1], kp, false, salt);
        st(pop, pidx<M>((9 + 5 * a + 0), n), phid - T(4) * iso, kp, false, salt);
    }
    // fluid equilibrium at the momentum c_i h_i = u0 - F(phi0)/2 so that the
    // velocity of Eq. sum-u equals the prescribed u0 at t = 0
    T j[2] = {u[0] - T(0.5) * kp.F0[0], u[1] - T(0.5) * kp.F0[1]};
#pragma unroll
    for (int a = 0; a < M; ++a) {
        j[0] -= T(0.5) * kp.Fphi[a][0] * phi[a];
        j[1] -= T(0.5) * kp.Fphi[a][1] * phi[a];
    }
    const T usq = j[0] * j[0] + j[1] * j[1];
    T hsum = T(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const T cu = T(CX9[i]) * j[0] + T(CY9[i]) * j[1];
        const T v = w9<T>(i) * (T(3) * p + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
        hsum += v;
        st(pop, pidx<M>(i, n), v, kp, true, salt);
    }
    st(pop, pidx<M>(0, n), kp.rho0_eff - hsum, kp, true, salt);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        if (!(kp.src_mask >> a & 1)) continue;
        T s = T(0);
        if constexpr (MODEL == LB_MODEL_CHEMOTAXIS) {
            s = (a == 1) ? -kp.beta * cutoff_r(kp, phi[1]) * phi[0] : T(0);
        } else {
#pragma unroll
            for (int b = 0; b < M; ++b) s += kp.K[a * M + b] * phi[b];
        }
        sold[(long long)(k++) * N + n] = s;
    }
}

template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_moments(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                 double* __restrict__ phi, double* __restrict__ u,
                                                 double* __restrict__ pr) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % kp.nx), y = (int)(n / kp.nx);
    T h[9], f[M][5];
    gather<S, M, ODD>(kp, pop, x, y, h, f);
    Macro<T, M> mc;
    macro<T, M>(kp, h, f, mc);
    if (phi)
#pragma unroll
        for (int a = 0; a < M; ++a) phi[a * N + n] = double(kp.phi_ref[a]) + double(mc.phid[a]);
    if (u) {
        u[n] = double(mc.u[0]);
        u[N + n] = double(mc.u[1]);
    }
    if (pr) pr[n] = double(mc.p) + (kp.pref ? double(kp.pref[y]) : 0.0);
}

// raw canonical populations, planes [plane_begin, plane_begin + count) of the
// sequence h_0..h_8, f_{1,0}..f_{m,4}, into out[k][N]
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_export(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                int plane_begin, int count, double* __restrict__ out) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % kp.nx), y = (int)(n / kp.nx);
    T h[9], f[M][5];
    gather<S, M, ODD>(kp, pop, x, y, h, f);
#pragma unroll
    for (int k = 0; k < 9 + 5 * M; ++k) {
        if (k < plane_begin || k >= plane_begin + count) continue;
        double v;
        if (k < 9) {
            v = double(h[k]) + (k == 0 ? double(kp.h0_shift) : 0.0);
            if (kp.pref) v += double(href_r<T>(k, kp.pref[y]));
        } else {
            const int a = (k - 9) / 5, i = (k - 9) % 5;
            v = double(f[a][i]) + double(w5<T>(i)) * double(kp.phi_ref[a]);
        }
        out[(long long)(k - plane_begin) * N + n] = v;
    }
}

// inverse of k_export: raw canonical FP64 planes into the own-slot layout
template <class S, int M>
__global__ __launch_bounds__(256) void k_import(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                                int plane_begin, int count, const double* __restrict__ in) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t salt = 0x2545f491u;
#pragma unroll
    for (int k = 0; k < 9 + 5 * M; ++k) {
        if (k < plane_begin || k >= plane_begin + count) continue;
        const double v = in[(long long)(k - plane_begin) * N + n];
        if (k < 9) {
            const double r = kp.pref ? double(href_r<T>(k, kp.pref[n / kp.nx])) : 0.0;
            st(pop, pidx<M>(k, n), T(v - (k == 0 ? double(kp.h0_shift) : 0.0) - r), kp, true, salt);
        } else {
            const int a = (k - 9) / 5, i = (k - 9) % 5;
            st(pop, pidx<M>(k, n), T(v - double(w5<T>(i)) * double(kp.phi_ref[a])), kp, false, salt);
        }
    }
}

// mean pressure of every row (one workgroup per row, fixed-order sums): the
// reference that lb_fluid_reference sets
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_row_pressure(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                      double* __restrict__ out) {
    using T = typename St<S>::T;
    const int y = blockIdx.x;
    double acc[1] = {0.0};
    for (int x = threadIdx.x; x < kp.nx; x += blockDim.x) {
        T h[9], f[M][5];
        gather<S, M, ODD>(kp, pop, x, y, h, f);
        Macro<T, M> mc;
        macro<T, M>(kp, h, f, mc);
        acc[0] += double(mc.p) + (kp.pref ? double(kp.pref[y]) : 0.0);
    }
    block_sum<1>(acc, out + y);
    if (threadIdx.x == 0) out[y] /= double(kp.nx);   // the thread that wrote the sum
}

// the stored fluid values of every node moved from the row reference in kp.pref
// (NULL: none) to pnew: + r_i(P_old) - r_i(P_new), each slot by its own node's
// row (in both AA layouts a slot's value is relative to the row of its node)
template <class S, int M>
__global__ __launch_bounds__(256) void k_reref(KParams<typename St<S>::T> kp, S* __restrict__ pop,
                                               const typename St<S>::T* __restrict__ pnew) {
    using T = typename St<S>::T;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int y = (int)(n / kp.nx);
    const T d = (kp.pref ? kp.pref[y] : T(0)) - pnew[y];
    const uint32_t salt = 0x7a3c9e21u;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        S* q = pop + pidx<M>(i, n);
        st(pop, pidx<M>(i, n), ld(q, kp, true) + href_r<T>(i, d), kp, true, salt);
    }
}

template <class TS, class TD>
__global__ __launch_bounds__(256) void k_convert(const TS* __restrict__ src, TD* __restrict__ dst, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = TD(src[k]);
}

// first reduction pass; mode 0 residual + snapshot, 1 snapshot only, 2 mass.
// Partial record per block: [diff_q (Q), norm_q (Q), nonfinite] (Q = M + 2),
// or [mass_a (M), sum h, nonfinite] for mode 2.
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_reduce(KParams<typename St<S>::T> kp, const S* __restrict__ pop,
                                                double* __restrict__ snap, double* __restrict__ part, int mode) {
    using T = typename St<S>::T;
    constexpr int Q = M + 2;
    const long long N = (long long)kp.nx * kp.ny;
    double acc[2 * Q + 1];
#pragma unroll
    for (int k = 0; k < 2 * Q + 1; ++k) acc[k] = 0.0;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(n % kp.nx), y = (int)(n / kp.nx);
        T h[9], f[M][5];
        gather<S, M, ODD>(kp, pop, x, y, h, f);
        Macro<T, M> mc;
        macro<T, M>(kp, h, f, mc);
        double q[Q];
        q[0] = double(mc.u[0]);
        q[1] = double(mc.u[1]);
#pragma unroll
        for (int a = 0; a < M; ++a) q[2 + a] = double(kp.phi_ref[a]) + double(mc.phid[a]);
        if (mode == 2) {
#pragma unroll
            for (int a = 0; a < M; ++a) acc[a] += q[2 + a];
            double hs = double(kp.h0_shift);
#pragma unroll
            for (int i = 0; i < 9; ++i) hs += double(h[i]);
            acc[M] += hs;
            bool bad = !isfinite(hs);
#pragma unroll
            for (int a = 0; a < M; ++a) bad |= !isfinite(q[2 + a]);
            acc[2 * Q] += bad ? 1.0 : 0.0;
        } else {
            bool bad = false;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double old = snap[(long long)k * N + n];
                acc[k] += fabs(q[k] - old);
                acc[Q + k] += fabs(q[k]);
                snap[(long long)k * N + n] = q[k];
                bad |= !isfinite(q[k]);
            }
            acc[2 * Q] += bad ? 1.0 : 0.0;
        }
    }
    block_sum<2 * Q + 1>(acc, part + (long long)blockIdx.x * kRedWidth);
}

// second pass: one block sums the partial records in a fixed order; in
// residual mode it also forms res_q = sum|q - q_prev| / sum|q| (0 if both vanish)
template <int Q>
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int nblocks,
                                                      double* __restrict__ out, int mode) {
    constexpr int NV = 2 * Q + 1;
    __shared__ double tot[NV];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += part[(long long)b * kRedWidth + k];
    block_sum<NV>(acc, tot);
    __syncthreads();
    if (threadIdx.x < NV) out[threadIdx.x] = tot[threadIdx.x];
    if (mode == 0 && threadIdx.x < Q) {
        const double d = tot[threadIdx.x], s = tot[Q + threadIdx.x];
        out[NV + threadIdx.x] = s > 0.0 ? d / s : (d == 0.0 ? 0.0 : __builtin_huge_val());
    }
}

// Mean inward diffusive flux through a Dirichlet wall (Sec. 3.2: Nu and Sh).
// For species a: flux_a(s) = -sum_b D_ab dphi_b/dn / D_aa along the inward normal,
// dphi/dn by the second-order one-sided difference through the wall value
// (half-way, distance 0) and the first two nodes (distances 1/2 and 3/2):
// (-8 phi_w + 9 phi_0 - phi_1) / 3 per lattice spacing; averaged along the
// wall and multiplied by the number of nodes across the cavity (unit length).
template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_wall_flux(KParams<typename St<S>::T> kp, const S* __restrict__ pop, int side,
                                                   double* __restrict__ out) {
    using T = typename St<S>::T;
    const bool xwall = side < 2;
    const int len = xwall ? kp.ny : kp.nx;        // nodes along the wall
    const int depth = xwall ? kp.nx : kp.ny;      // nodes across the cavity
    double acc[M];
#pragma unroll
    for (int a = 0; a < M; ++a) acc[a] = 0.0;
    for (int j = threadIdx.x; j < len; j += blockDim.x) {
        double ph[2][M];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            int x, y;
            if (xwall) {
                y = j;
                x = side == 0 ? d : kp.nx - 1 - d;
            } else {
                x = j;
                y = side == 2 ? d : kp.ny - 1 - d;
            }
            T h[9], f[M][5];
            gather<S, M, ODD>(kp, pop, x, y, h, f);
#pragma unroll
            for (int a = 0; a < M; ++a)
                ph[d][a] = double(kp.phi_ref[a]) + double(((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + f[a][4]);
        }
        double g[M];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double w = double(kp.wallr[side][a]) + double(kp.phi_ref[a]);
            g[a] = (-8.0 * w + 9.0 * ph[0][a] - ph[1][a]) / 3.0;
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < M; ++b) s += double(kp.Dflux[a * M + b]) * g[b];
            acc[a] += -s / double(kp.Dflux[a * M + a]);
        }
    }
    __shared__ double tot[M];
    block_sum<M>(acc, tot);
    __syncthreads();
    if (threadIdx.x < M) out[threadIdx.x] = tot[threadIdx.x] / len * depth;
}

hipError_t launch_wall_flux(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                            const KParams<float>& kf, bool odd, int side, double* out, hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k_wall_flux<S, M, true>), dim3(1), dim3(256), 0, s, kpar<S>(kd, kf), pop, side, out);
        else
            hipLaunchKernelGGL((k_wall_flux<S, M, false>), dim3(1), dim3(256), 0, s, kpar<S>(kd, kf), pop, side, out);
        return hipGetLastError();
    });
}

hipError_t launch_init(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                       const KParams<float>& kf, int has_p0, hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        hipLaunchKernelGGL((k_init<S, M, MODEL>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                           (S*)at(ws, L.pop_off), (T*)at(ws, L.sold_off), (const double*)at(ws, L.stage_off),
                           has_p0);
        return hipGetLastError();
    });
}

hipError_t launch_step(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                       const KParams<float>& kf, bool odd, Launch lc, int64_t step, hipStream_t s) {
    const uint32_t salt = step_salt(step);
    const int tiles_x = (p.nx + lc.tile_x - 1) / lc.tile_x;
    const int tiles_y = (p.ny + lc.tile_y - 1) / lc.tile_y;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)(lc.tile_x * lc.tile_y));
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at(ws, L.pop_off);
        T* sold = (T*)at(ws, L.sold_off);
        KParams<T> kp = kpar<S>(kd, kf);
        // with gamma != 0 the new source field goes to the second buffer (the
        // caller swaps the two after the launch); otherwise in place
        T* sold_out = kp.gam_on ? (T*)at(ws, L.sold2_off) : sold;
        int tx = lc.tile_x, ty = lc.tile_y, tsx = tiles_x;
        uint32_t sl = salt;
        const long long* tsp = nullptr;
        void* args[] = {&kp, &pop, &sold, &sold_out, &tx, &ty, &tsx, &sl, &tsp};
        const void* fn = step_kernel<S, M, MODEL>(p.collision == LB_COLL_MRT, odd, (lc.nt >> (odd ? 1 : 0) & 1) != 0,
                                                  kp.pref != nullptr);
        return hipLaunchKernel(fn, grid, block, args, 0, s);
    });
}

// A graph of `steps` (even) single-step launches, even parity first, each
// node depending on the previous one.  Built node by node (no stream
// capture), so it can be launched on any stream, including the null stream.
// FP16: launch k of a replay takes the stochastic-rounding salt of step
// *tstep + k, *tstep set to the step count before each replay (launch_set_step).
hipError_t build_step_graph(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                            const KParams<float>& kf, Launch lc, int steps, const long long* tstep, hipGraph_t* out) {
    if (steps < 2 || steps % 2) return hipErrorInvalidValue;
    const int tiles_x = (p.nx + lc.tile_x - 1) / lc.tile_x;
    const int tiles_y = (p.ny + lc.tile_y - 1) / lc.tile_y;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)(lc.tile_x * lc.tile_y));
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    e = dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        S* pop = (S*)at(ws, L.pop_off);
        // source planes: launch k reads buffer k % 2 and writes the other one
        // (the same buffer twice unless gamma != 0)
        KParams<T> kp = kpar<S>(kd, kf);
        T* sbuf[2] = {(T*)at(ws, L.sold_off), (T*)at(ws, kp.gam_on ? L.sold2_off : L.sold_off)};
        int tx = lc.tile_x, ty = lc.tile_y, tsx = tiles_x;
        uint32_t salt = 0;   // launch k: its offset k from *tstep (FP16)
        const long long* tsp = p.storage == LB_STORE_F16 ? tstep : nullptr;
        void* args[2][9] = {{&kp, &pop, &sbuf[0], &sbuf[1], &tx, &ty, &tsx, &salt, &tsp},
                            {&kp, &pop, &sbuf[1], &sbuf[0], &tx, &ty, &tsx, &salt, &tsp}};
        const bool mrt = p.collision == LB_COLL_MRT;
        const bool ref = kp.pref != nullptr;
        void* fe = const_cast<void*>(step_kernel<S, M, MODEL>(mrt, false, (lc.nt & 1) != 0, ref));
        void* fo = const_cast<void*>(step_kernel<S, M, MODEL>(mrt, true, (lc.nt & 2) != 0, ref));
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < steps; ++k) {
            salt = (uint32_t)k;   // the node copies the argument values
            hipKernelNodeParams np{};
            np.func = (k & 1) ? fo : fe;
            np.gridDim = grid;
            np.blockDim = block;
            np.sharedMemBytes = 0;
            np.kernelParams = args[k & 1];
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

template <class S, int M, int MODEL, int COLL, int TX, int TY>
static hipError_t launch_step2_t(const KParams<typename St<S>::T>& kp, const Layout& L, void* ws, uint32_t salt,
                                 hipStream_t s) {
    using T = typename St<S>::T;
    using G = Tb2Geom<TX, TY>;
    const size_t lds = sizeof(T) * (9 + 5 * M + M) * (G::RX * G::RY + G::R1X * G::R1Y);
    auto kern = k_step2<S, M, MODEL, COLL, TX, TY>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int tiles_x = (kp.nx + TX - 1) / TX, tiles_y = (kp.ny + TY - 1) / TY;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles_x * tiles_y)), dim3(256), lds, s, kp,
                       (const S*)at(ws, L.pop_off), (S*)at(ws, L.pop2_off), (const T*)at(ws, L.sold_off),
                       (T*)at(ws, L.sold2_off), tiles_x, salt);
    return hipGetLastError();
}

hipError_t launch_step2(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                        const KParams<float>& kf, int64_t step, hipStream_t s) {
    const uint32_t salt = mix32((uint32_t)step ^ (uint32_t)(step >> 32) * 0x632be5abu ^ 0x2b2b2b2bu);
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const auto& kp = kpar<S>(kd, kf);
        if constexpr (std::is_same<S, double>::value) {
            if (p.collision == LB_COLL_MRT) return launch_step2_t<S, M, MODEL, LB_COLL_MRT, 32, 4>(kp, L, ws, salt, s);
            return launch_step2_t<S, M, MODEL, LB_COLL_BGK, 32, 4>(kp, L, ws, salt, s);
        } else {
            if (p.collision == LB_COLL_MRT) return launch_step2_t<S, M, MODEL, LB_COLL_MRT, 64, 4>(kp, L, ws, salt, s);
            return launch_step2_t<S, M, MODEL, LB_COLL_BGK, 64, 4>(kp, L, ws, salt, s);
        }
    });
}

hipError_t launch_moments(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                          const KParams<float>& kf, bool odd, double* phi, double* u, double* pr,
                          hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k_moments<S, M, true>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, phi, u, pr);
        else
            hipLaunchKernelGGL((k_moments<S, M, false>), dim3(blocks_for(L.N)), dim3(256), 0, s,
                               kpar<S>(kd, kf), pop, phi, u, pr);
        return hipGetLastError();
    });
}

hipError_t launch_export(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, bool odd, int plane_begin, int plane_count, double* out,
                         hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k_export<S, M, true>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, plane_begin, plane_count, out);
        else
            hipLaunchKernelGGL((k_export<S, M, false>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                               pop, plane_begin, plane_count, out);
        return hipGetLastError();
    });
}

hipError_t launch_import(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, int plane_begin, int plane_count, const double* in,
                         hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        hipLaunchKernelGGL((k_import<S, M>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                           (S*)at(ws, L.pop_off), plane_begin, plane_count, in);
        return hipGetLastError();
    });
}

hipError_t launch_row_pressure(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                               const KParams<float>& kf, bool odd, double* out, hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        if (odd)
            hipLaunchKernelGGL((k_row_pressure<S, M, true>), dim3((unsigned)p.ny), dim3(256), 0, s, kpar<S>(kd, kf), pop, out);
        else
            hipLaunchKernelGGL((k_row_pressure<S, M, false>), dim3((unsigned)p.ny), dim3(256), 0, s, kpar<S>(kd, kf), pop, out);
        return hipGetLastError();
    });
}

__global__ void k_set_step(long long* __restrict__ tstep, long long step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *tstep = step;
}

hipError_t launch_set_step(long long* tstep, long long step, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, tstep, step);
    return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_reref(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                        const KParams<float>& kf, const void* pnew, hipStream_t s) {
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        hipLaunchKernelGGL((k_reref<S, M>), dim3(blocks_for(L.N)), dim3(256), 0, s, kpar<S>(kd, kf),
                           (S*)at(ws, L.pop_off), (const T*)pnew);
        return hipGetLastError();
    });
}

hipError_t launch_copy_sold(const lb_params& ps, const Layout& Ls, void* wss, const lb_params& pd,
                            const Layout& Ld, void* wsd, hipStream_t s) {
    const long long n = (long long)(Ls.nsrc * Ls.N);
    if (n == 0) return hipSuccess;
    const bool s64 = ps.storage == LB_STORE_F64, d64 = pd.storage == LB_STORE_F64;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    void* src = at(wss, Ls.sold_off);
    void* dst = at(wsd, Ld.sold_off);
    if (s64 && d64)
        hipLaunchKernelGGL((k_convert<double, double>), g, b, 0, s, (const double*)src, (double*)dst, n);
    else if (s64)
        hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, s, (const double*)src, (float*)dst, n);
    else if (d64)
        hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, s, (const float*)src, (double*)dst, n);
    else
        hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, s, (const float*)src, (float*)dst, n);
    return hipGetLastError();
}

hipError_t launch_reduce_final(int Q, const double* part, int nblocks, double* out, int mode, hipStream_t s) {
    switch (Q) {
        case 3: hipLaunchKernelGGL((k_reduce_final<3>), dim3(1), dim3(256), 0, s, part, nblocks, out, mode); break;
        case 4: hipLaunchKernelGGL((k_reduce_final<4>), dim3(1), dim3(256), 0, s, part, nblocks, out, mode); break;
        case 5: hipLaunchKernelGGL((k_reduce_final<5>), dim3(1), dim3(256), 0, s, part, nblocks, out, mode); break;
        case 6: hipLaunchKernelGGL((k_reduce_final<6>), dim3(1), dim3(256), 0, s, part, nblocks, out, mode); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int reduce_blocks(size_t N) {
    const size_t b = (N + 255) / 256;
    return (int)(b < (size_t)kRedBlocks ? b : (size_t)kRedBlocks);
}

hipError_t launch_reduce(const lb_params& p, const Layout& L, void* ws, const KParams<double>& kd,
                         const KParams<float>& kf, bool odd, int mode, hipStream_t s, double* part, double* res) {
    const int nb = reduce_blocks(L.N);
    if (!part) part = (double*)at(ws, L.part_off);
    if (!res) res = (double*)at(ws, L.res_off);
    return dispatch(p, [&]<class S, int M, int MODEL>() -> hipError_t {
        const S* pop = (const S*)at(ws, L.pop_off);
        double* snap = (double*)at(ws, L.snap_off);
        if (odd)
            hipLaunchKernelGGL((k_reduce<S, M, true>), dim3(nb), dim3(256), 0, s, kpar<S>(kd, kf), pop, snap, part,
                               mode);
        else
            hipLaunchKernelGGL((k_reduce<S, M, false>), dim3(nb), dim3(256), 0, s, kpar<S>(kd, kf), pop, snap,
                               part, mode);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_reduce_final<M + 2>), dim3(1), dim3(256), 0, s, part, nb, res, mode);
        return hipGetLastError();
    });
}

}  // namespace lbk
