// lb_batch.hip -- batched parameter sweep: many independent cavities of
// uneven size advanced by one launch per time step.
//
// The grid is a list of tiles (cavity, tile index) over every cavity still
// running; each workgroup updates one tile of one cavity with the same fused
// AA-pattern update as the single-domain kernel, reading that cavity's own
// parameter record (relaxation matrix, forces, walls, grid size) from device
// memory.  Tiles of a cavity are contiguous in the list and the XCD-aware
// remap keeps them on one XCD.  Residuals are reduced per tile and then per
// cavity in a fixed order (deterministic FP64), so converged or diverged
// cavities can be retired from the list between launches.
#include <hip/hip_runtime.h>

#include "lb_device.h"

namespace lbk {

template <class S, int M, int MODEL, int COLL, bool ODD, bool NT>
__global__ __launch_bounds__(256) void k_bstep(const KParams<typename St<S>::T>* __restrict__ kps,
                                               const CavRec* __restrict__ cav, const int2* __restrict__ tiles,
                                               int ntiles, char* __restrict__ ws, uint32_t salt,
                                               const long long* __restrict__ tstep) {
    using T = typename St<S>::T;
    salt = launch_salt<S>(salt, tstep);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b >= ntiles) return;
    const int2 t = tiles[b];
    const KParams<T>& kp = kps[t.x];
    const CavRec cr = cav[t.x];
    // the cavity's own tile shape (every shape of a launch has blockDim.x threads)
    const int bx = t.y % cr.tiles_x, by = t.y / cr.tiles_x;
    const int x = bx * cr.tile_x + (int)(threadIdx.x % cr.tile_x);
    const int y = by * cr.tile_y + (int)(threadIdx.x / cr.tile_x);
    if (x >= kp.nx || y >= kp.ny) return;
    const long long N = (long long)kp.nx * kp.ny;
    const long long n = (long long)y * kp.nx + x;
    S* pop = reinterpret_cast<S*>(ws + cr.pop_off);
    T* sold = reinterpret_cast<T*>(ws + cr.sold_off);

    T h[9], f[M][5], Sold[M], Snew[M];
    gather<S, M, ODD, NT, false>(kp, pop, x, y, h, f);
    int k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        Sold[a] = T(0);
        if (kp.src_mask >> a & 1) Sold[a] = load_raw<NT>(&sold[(long long)(k++) * N + n]);
    }
    collide<T, M, MODEL, COLL, std::is_same_v<S, float>>(kp, h, f, Sold, Snew);
    k = 0;
#pragma unroll
    for (int a = 0; a < M; ++a)
        if (kp.src_mask >> a & 1) store_raw<NT>(Snew[a], &sold[(long long)(k++) * N + n]);
    scatter<S, M, ODD, NT, false>(kp, pop, x, y, h, f, salt);
}

// the batched step kernel for a collision kind, parity and cache hint
template <class S, int M, int MODEL>
static const void* bstep_kernel(bool mrt, bool odd, bool nt) {
    const void* const fns[8] = {
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_BGK, false, false>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_BGK, false, true>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_BGK, true, false>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_BGK, true, true>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_MRT, false, false>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_MRT, false, true>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_MRT, true, false>),
        reinterpret_cast<const void*>(&k_bstep<S, M, MODEL, LB_COLL_MRT, true, true>)};
    return fns[(mrt ? 4 : 0) + (odd ? 2 : 0) + (nt ? 1 : 0)];
}

template <class S, int M, bool ODD>
__global__ __launch_bounds__(256) void k_breduce(const KParams<typename St<S>::T>* __restrict__ kps,
                                                 const CavRec* __restrict__ cav, const int2* __restrict__ tiles,
                                                 int ntiles, char* __restrict__ ws, double* __restrict__ part, int mode) {
    using T = typename St<S>::T;
    constexpr int Q = M + 2;
    double acc[2 * Q + 1];
#pragma unroll
    for (int k = 0; k < 2 * Q + 1; ++k) acc[k] = 0.0;
    const int2 t = tiles[blockIdx.x];
    const KParams<T>& kp = kps[t.x];
    const CavRec cr = cav[t.x];
    const int bx = t.y % cr.tiles_x, by = t.y / cr.tiles_x;
    const int x = bx * cr.tile_x + (int)(threadIdx.x % cr.tile_x);
    const int y = by * cr.tile_y + (int)(threadIdx.x / cr.tile_x);
    if (x < kp.nx && y < kp.ny) {
        const long long N = (long long)kp.nx * kp.ny;
        const long long n = (long long)y * kp.nx + x;
        const S* pop = reinterpret_cast<const S*>(ws + cr.pop_off);
        double* snap = reinterpret_cast<double*>(ws + cr.snap_off);
        T h[9], f[M][5];
        gather<S, M, ODD, false, false>(kp, pop, x, y, h, f);
        Macro<T, M> mc;
        macro<T, M>(kp, h, f, mc);
        double q[Q];
        q[0] = double(mc.u[0]);
        q[1] = double(mc.u[1]);
#pragma unroll
        for (int a = 0; a < M; ++a) q[2 + a] = double(kp.phi_ref[a]) + double(mc.phid[a]);
        bool bad = false;
        if (mode == 2) {
#pragma unroll
            for (int a = 0; a < M; ++a) acc[a] = q[2 + a];
            double hs = double(kp.h0_shift);
#pragma unroll
            for (int i = 0; i < 9; ++i) hs += double(h[i]);
            acc[M] = hs;
            bad = !isfinite(hs);
#pragma unroll
            for (int a = 0; a < M; ++a) bad |= !isfinite(q[2 + a]);
        } else {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                acc[k] = fabs(q[k] - snap[(long long)k * N + n]);
                acc[Q + k] = fabs(q[k]);
                snap[(long long)k * N + n] = q[k];
                bad |= !isfinite(q[k]);
            }
        }
        acc[2 * Q] = bad ? 1.0 : 0.0;
    }
    block_sum<2 * Q + 1>(acc, part + (long long)blockIdx.x * kRedWidth);
}

template <int Q>
__global__ __launch_bounds__(256) void k_bfinal(const int4* __restrict__ ranges, const double* __restrict__ part,
                                                double* __restrict__ out, int mode) {
    constexpr int NV = 2 * Q + 1;
    __shared__ double tot[NV];
    const int4 r = ranges[blockIdx.x];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < r.z; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += part[(long long)(r.y + b) * kRedWidth + k];
    block_sum<NV>(acc, tot);
    __syncthreads();
    double* o = out + (long long)r.x * 64;
    if (threadIdx.x < NV) o[threadIdx.x] = tot[threadIdx.x];
    if (mode == 0 && threadIdx.x < Q) {
        const double d = tot[threadIdx.x], s = tot[Q + threadIdx.x];
        o[NV + threadIdx.x] = s > 0.0 ? d / s : (d == 0.0 ? 0.0 : __builtin_huge_val());
    }
}

hipError_t launch_bstep(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                        int ntiles, bool odd, Launch lc, int64_t step, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const uint32_t salt = step_salt(step);
    const dim3 grid((unsigned)ntiles), block((unsigned)(lc.tile_x * lc.tile_y));
    return dispatch(p0, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        const KParams<T>* kp = static_cast<const KParams<T>*>(kparams);
        char* w = static_cast<char*>(ws);
        const CavRec* cv = cav;
        const int2* tl = tiles;
        int nt = ntiles;
        uint32_t sl = salt;
        const long long* tsp = nullptr;
        void* args[] = {&kp, &cv, &tl, &nt, &w, &sl, &tsp};
        const void* fn = bstep_kernel<S, M, MODEL>(p0.collision == LB_COLL_MRT, odd, (lc.nt >> (odd ? 1 : 0) & 1) != 0);
        return hipLaunchKernel(fn, grid, block, args, 0, s);
    });
}

// Graph of `steps` (even) batched single-step launches, even parity first,
// chained; same arguments as launch_bstep.  FP16: launch k of a replay takes
// the stochastic-rounding salt of step *tstep + k (*tstep set before each replay).
hipError_t build_bstep_graph(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                             int ntiles, Launch lc, int steps, const long long* tstep, hipGraph_t* out) {
    if (steps < 2 || steps % 2 || ntiles <= 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)ntiles), block((unsigned)(lc.tile_x * lc.tile_y));
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    e = dispatch(p0, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        const KParams<T>* kp = static_cast<const KParams<T>*>(kparams);
        char* w = static_cast<char*>(ws);
        const CavRec* cv = cav;
        const int2* tl = tiles;
        int nt = ntiles;
        uint32_t salt = 0;   // launch k: its offset k from *tstep (FP16)
        const long long* tsp = p0.storage == LB_STORE_F16 ? tstep : nullptr;
        void* args[] = {&kp, &cv, &tl, &nt, &w, &salt, &tsp};
        const bool mrt = p0.collision == LB_COLL_MRT;
        void* fe = const_cast<void*>(bstep_kernel<S, M, MODEL>(mrt, false, (lc.nt & 1) != 0));
        void* fo = const_cast<void*>(bstep_kernel<S, M, MODEL>(mrt, true, (lc.nt & 2) != 0));
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < steps; ++k) {
            salt = (uint32_t)k;   // the node copies the argument values
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

hipError_t launch_breduce(const lb_params& p0, void* ws, const void* kparams, const CavRec* cav, const int2* tiles,
                          int ntiles, const int4* ranges, int nranges, bool odd, Launch lc, int mode, double* part,
                          double* out, hipStream_t s) {
    if (ntiles <= 0 || nranges <= 0) return hipSuccess;
    const dim3 grid((unsigned)ntiles), block((unsigned)(lc.tile_x * lc.tile_y));
    return dispatch(p0, [&]<class S, int M, int MODEL>() -> hipError_t {
        using T = typename St<S>::T;
        const KParams<T>* kp = static_cast<const KParams<T>*>(kparams);
        char* w = static_cast<char*>(ws);
        if (odd)
            hipLaunchKernelGGL((k_breduce<S, M, true>), grid, block, 0, s, kp, cav, tiles, ntiles, w, part, mode);
        else
            hipLaunchKernelGGL((k_breduce<S, M, false>), grid, block, 0, s, kp, cav, tiles, ntiles, w, part, mode);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_bfinal<M + 2>), dim3((unsigned)nranges), dim3(256), 0, s, ranges, part, out, mode);
        return hipGetLastError();
    });
}

}  // namespace lbk
