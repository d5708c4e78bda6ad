// lb_device.h -- device-side building blocks of the fused lattice Boltzmann
// update (lattices, storage traits, AA-pattern gather/scatter with the wall
// rules, moments and the collision), shared by the single-domain kernels
// (lb_kernels.hip) and the batched sweep kernels (lb_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "lb_internal.h"

namespace lbk {

// ---- lattices (Sec. 2: D2Q5 for the scalars, D2Q9 for the fluid) ---------
__device__ constexpr int CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr int MIRY9[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};  // c_y -> -c_y
__device__ constexpr int MIRX9[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};  // c_x -> -c_x
__device__ constexpr int CX5[5] = {0, 1, 0, -1, 0};
__device__ constexpr int CY5[5] = {0, 0, 1, 0, -1};
__device__ constexpr int OPP5[5] = {0, 3, 4, 1, 2};

template <class T>
__device__ __forceinline__ T w9(int i) {
    return i == 0 ? T(4) / T(9) : (i < 5 ? T(1) / T(9) : T(1) / T(36));
}
template <class T>
__device__ __forceinline__ T w5(int i) {
    return i == 0 ? T(1) / T(3) : T(1) / T(6);
}

// Lallemand-Luo D2Q9 moment basis (rows rho, e, eps, jx, qx, jy, qy, pxx, pxy);
// rows are orthogonal, so M^-1 = M^T diag(1/|row|^2).
__device__ constexpr int MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},     {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1}, {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},  {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},  {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
__device__ constexpr int MNORM[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};

// ---- storage traits --------------------------------------------------------
template <class S>
struct St;
template <>
struct St<double> {
    using T = double;
    static constexpr bool scaled = false;
};
template <>
struct St<float> {
    using T = float;
    static constexpr bool scaled = false;
};
template <>
struct St<_Float16> {
    using T = float;
    static constexpr bool scaled = true;
};

// FP16 deviations carry one scale for the fluid planes (0..8) and one for
// the scalar planes; FP32/FP64 are unscaled
// Population loads and stores, plain or with the non-temporal hint (NT).  The
// hint pays on launches whose working set stays in the caches (every value is
// read once and written once per step; the plume step at 512 x 256 went from
// 4.9 to 4.45 us) but costs bandwidth on grids far beyond them (4096^2 FP32:
// 463 -> 500 us, the odd step's shifted accesses share cache lines between
// neighbouring wavefronts), so the launcher chooses it by working-set size.
template <bool NT, class S>
__device__ __forceinline__ S load_raw(const S* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, class S>
__device__ __forceinline__ void store_raw(S v, S* p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT = false, class S, class T>
__device__ __forceinline__ T ld(const S* p, const KParams<T>& kp, bool fluid) {
    if constexpr (St<S>::scaled)  // fma with a zero addend: one mixed-precision fma (f16 operand) on gfx950
        return __builtin_fmaf(T(load_raw<NT>(p)), fluid ? kp.inv_scale_h : kp.inv_scale, T(0));
    else
        return T(load_raw<NT>(p));
}
// 32-bit integer mixer (Wellons' "lowbias32"), used as a counter-based
// generator for stochastic rounding
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
// the stochastic-rounding salt of time step `step` (one value per launch)
__host__ __device__ __forceinline__ uint32_t step_salt(long long step) {
    return mix32((uint32_t)step ^ (uint32_t)(step >> 32) * 0x632be5abu);
}
// the salt of a launch: given directly, or (tstep non-null: launches replayed from a graph,
// whose arguments are fixed) as the offset of the launch from the step count in *tstep
template <class S>
__device__ __forceinline__ uint32_t launch_salt(uint32_t salt, const long long* tstep) {
    if constexpr (St<S>::scaled) {
        if (tstep) return step_salt(*tstep + (long long)salt);
    }
    return salt;
}

// binary16 with stochastic rounding: adding uniform random bits below the 10
// kept mantissa bits to the magnitude and truncating rounds up with
// probability equal to the discarded fraction, so increments smaller than
// half an ulp survive in expectation.  gfx950 does this in one instruction
// (v_cvt_sr_f16_f32), which takes the top 13 bits of its 32-bit random word as
// the dither (checked on the GPU against the add-and-truncate definition: equal
// on every binary16-normal value; subnormal results are dithered too).
__device__ __forceinline__ _Float16 to_half_sr(float v, uint32_t rnd) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t z = {_Float16(0), _Float16(0)};
    return __builtin_amdgcn_cvt_sr_f16_f32(z, v, rnd, false)[0];
}

// The random word of element idx in a step with salt s (a lowbias32 hash of
// the step number): (idx xor s) times the 32-bit golden-ratio constant
// (Knuth's multiplicative hashing), whose top bits serve as the dither; used
// by the set-up kernels and the two-steps-per-launch kernel (the single-step
// kernels use the per-node words of sr_node below).  Uniform over steps for
// every element (xor with a uniform salt, then a bijection of the 32-bit
// words); reproducible.
__device__ __forceinline__ uint32_t sr_dither(long long idx, uint32_t salt) {
    return ((uint32_t)idx ^ salt) * 0x9e3779b9u;
}

template <bool NT = false, class S, class T>
__device__ __forceinline__ void st(S* base, long long idx, T v, const KParams<T>& kp, bool fluid, uint32_t salt) {
    if constexpr (St<S>::scaled)
        store_raw<NT>(to_half_sr(v * (fluid ? kp.scale_h : kp.scale), sr_dither(idx, salt)), base + idx);
    else
        store_raw<NT>(S(v), base + idx);
}

// The random words of the values a node stores in a step with salt s: value q
// of node n takes (32 n + q + s) times the golden-ratio constant, i.e. one
// multiply per node and one add per value (an integer multiply per value
// was a sixth of the FP16 step's issue time).  Within a step the words of
// distinct values are distinct terms of the golden-ratio (Weyl) sequence, so
// their top bits are evenly spread; over steps each word is uniform (the salt
// is a hash of the step number and multiplication by an odd constant is a
// bijection).  Runs are reproducible.
__device__ __forceinline__ uint32_t sr_node(long long n, uint32_t salt) {
    return ((uint32_t)n * 32u + salt) * 0x9e3779b9u;
}
__device__ __forceinline__ uint32_t sr_word(uint32_t node_word, int q) { return node_word + (uint32_t)q * 0x9e3779b9u; }

// store of one population value; rnd is the stochastic-rounding word (FP16)
template <bool NT = false, class S, class T>
__device__ __forceinline__ void st_r(S* p, T v, const KParams<T>& kp, bool fluid, uint32_t rnd) {
    if constexpr (St<S>::scaled)
        store_raw<NT>(to_half_sr(v * (fluid ? kp.scale_h : kp.scale), rnd), p);
    else
        store_raw<NT>(S(v), p);
}

// ---- geometry helpers -------------------------------------------------------
// wraps c into [0, n) on a periodic axis; returns false when c is outside a
// non-periodic axis
__device__ __forceinline__ bool wrap_in(int& c, int n, int periodic) {
    if (c < 0) {
        if (!periodic) return false;
        c += n;
    } else if (c >= n) {
        if (!periodic) return false;
        c -= n;
    }
    return true;
}
__device__ __forceinline__ int side_x(int c) { return c < 0 ? 0 : 1; }
__device__ __forceinline__ int side_y(int c) { return c < 0 ? 2 : 3; }

// Population storage: nodes (n = y nx + x) in blocks of kBlk; within a block
// the 9 + 5m populations follow each other as runs of kBlk values (h_0..h_8,
// then f_{a,0..4} per species).  A wavefront of 64 nodes reads or writes 64
// consecutive values per population, and the 19+ runs of one block are
// contiguous, so the memory system sees few long streams instead of one
// stream per population plane.
constexpr int kBlkShift = 6;
constexpr int kBlk = 1 << kBlkShift;

template <int M>
__host__ __device__ __forceinline__ long long pidx(int q, long long n) {
    constexpr int NQ = 9 + 5 * M;
    // node part first, population part last: the node part is shared by all
    // populations of a node and the population part folds into the load offset
    return ((n >> kBlkShift) * (NQ << kBlkShift) + (n & (kBlk - 1))) + ((long long)q << kBlkShift);
}

// true when no link of node (x, y) crosses a wall: interior on every walled
// axis (a periodic axis has no walls)
template <class T>
__device__ __forceinline__ bool no_wall_link(const KParams<T>& kp, int x, int y) {
    const bool okx = kp.px || ((x > 0) & (x < kp.nx - 1));
    const bool oky = kp.py || ((y > 0) & (y < kp.ny - 1));
    return okx & oky;
}

// node indices of the 3 x 3 neighbourhood of (x, y), wrapped on periodic
// axes; valid for nodes with no_wall_link()
struct Nbr {
    long long row[3];
    int col[3];
    template <class T>
    __host__ __device__ __forceinline__ Nbr(const KParams<T>& kp, int x, int y) {
        const int nx = kp.nx, ny = kp.ny;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        row[0] = (long long)ym * nx;
        row[1] = (long long)y * nx;
        row[2] = (long long)yp * nx;
        col[0] = x == 0 ? nx - 1 : x - 1;
        col[1] = x;
        col[2] = x == nx - 1 ? 0 : x + 1;
    }
    __host__ __device__ __forceinline__ long long at(int dx, int dy) const { return row[dy + 1] + col[dx + 1]; }
};

// Element offsets (population 0) of the 3 x 3 neighbourhood of (x, y) in the
// blocked layout, wrapped on periodic axes; valid for nodes with
// no_wall_link(), and for the node itself and its in-domain neighbours
// otherwise.  Same value as pidx<M>(0, n') for the neighbour n', computed
// with 32-bit node arithmetic: for the first node R of a row, the neighbour
// R + c lies in block (R >> 6) + ((R & 63) + c) >> 6 at lane ((R & 63) + c) & 63,
// so one 64-bit product per row ((R >> 6) times the block size) and a 24-bit
// product per neighbour replace a 64-bit multiply per neighbour.  Needs
// nx * ny < 2^31 and nx * (9 + 5m) + 64 (9 + 5m) < 2^31 (checked by the host).
template <int M>
struct NbrE {
    static constexpr int Q = (9 + 5 * M) << kBlkShift;  // values per block
    long long rb[3];  // rows y - 1, y, y + 1: element offset of the block holding the row's first node
    int rm[3];        // lane of the row's first node in that block
    int col[3];       // columns x - 1, x, x + 1
    template <class T>
    __host__ __device__ __forceinline__ NbrE(const KParams<T>& kp, int x, int y) {
        const int nx = kp.nx, ny = kp.ny;
        const int r1 = y * nx;
        const int r0 = y == 0 ? (ny - 1) * nx : r1 - nx;
        const int r2 = y == ny - 1 ? 0 : r1 + nx;
        rb[0] = (long long)(r0 >> kBlkShift) * Q;
        rb[1] = (long long)(r1 >> kBlkShift) * Q;
        rb[2] = (long long)(r2 >> kBlkShift) * Q;
        rm[0] = r0 & (kBlk - 1);
        rm[1] = r1 & (kBlk - 1);
        rm[2] = r2 & (kBlk - 1);
        col[0] = x == 0 ? nx - 1 : x - 1;
        col[1] = x;
        col[2] = x == nx - 1 ? 0 : x + 1;
    }
    __host__ __device__ __forceinline__ long long at(int dx, int dy) const {
        const int t = rm[dy + 1] + col[dx + 1];
        // both factors below 2^24 (masks are no-ops under the host's limits): a
        // full-rate 24-bit multiply on the GPU
        const unsigned blk = (unsigned)(t >> kBlkShift) & 0xffffffu;
        return rb[dy + 1] + (long long)(blk * (unsigned)Q + (unsigned)(t & (kBlk - 1)));
    }
};

// walls next to node (x, y): out_x(d) is true when x + d (d in -1, 0, 1) lies
// beyond a wall (never on a periodic axis); likewise out_y
struct WallFlags {
    bool x0, x1, y0, y1;
    template <class T>
    __device__ __forceinline__ WallFlags(const KParams<T>& kp, int x, int y)
        : x0(!kp.px && x == 0), x1(!kp.px && x == kp.nx - 1), y0(!kp.py && y == 0), y1(!kp.py && y == kp.ny - 1) {}
    __device__ __forceinline__ bool out_x(int d) const { return (d < 0 && x0) || (d > 0 && x1); }
    __device__ __forceinline__ bool out_y(int d) const { return (d < 0 && y0) || (d > 0 && y1); }
};

// ---- gather ---------------------------------------------------------------
// Canonical pre-collision populations of node (x, y).  PULL = false: the own
// slots (state after an odd step or initialisation).  PULL = true: the state
// left by an even step, read from the upstream neighbours with the wall rules.
// Fluid reference pressure (kp.pref, REF kernels only): with a per-row reference P(y)
// the stored fluid values of a node in row y are h_i - r_i(P(y)), r_i the
// equilibrium at pressure P and rest (r_0 = -(5/3) P, r_i = 3 W_i P; sum_i r_i = 0),
// so a value that streams between rows changes its reference by
// r_i(P(y_from)) - r_i(P(y_to)) = 3 W_i (P(y_from) - P(y_to)).
template <class T>
__device__ __forceinline__ T href_r(int i, T P) {   // r_i(P)
    return i == 0 ? -(T(5) / T(3)) * P : T(3) * w9<T>(i) * P;
}
template <class T>
__device__ __forceinline__ T pref_at(const KParams<T>& kp, int y) {
    return kp.pref[y];
}
__device__ __forceinline__ int wrap_row(int y, int ny) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); }

template <class S, int M, bool PULL, bool NT = false, bool REF = true, class T>
__device__ __forceinline__ void gather(const KParams<T>& kp, const S* __restrict__ pop, int x, int y,
                                       T h[9], T f[M][5]) {
    const int nx = kp.nx;
    const long long n = (long long)y * nx + x;
    if constexpr (!PULL) {
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = ld<NT>(pop + pidx<M>(i, n), kp, true);
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) f[a][i] = ld<NT>(pop + pidx<M>((9 + 5 * a + i), n), kp, false);
        return;
    } else {
        if (__all(no_wall_link(kp, x, y))) {  // wave-uniform choice: no lane pays for both paths
            const NbrE<M> nb(kp, x, y);
#pragma unroll
            for (int i = 0; i < 9; ++i) h[i] = ld<NT>(pop + nb.at(-CX9[i], -CY9[i]) + ((long long)(OPP9[i]) << kBlkShift), kp, true);
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    f[a][i] = ld<NT>(pop + nb.at(-CX5[i], -CY5[i]) + ((long long)(9 + 5 * a + OPP5[i]) << kBlkShift), kp, false);
            if (REF && kp.pref) {   // values pulled from rows y -+ 1, to this row's reference
                const int ny = kp.ny;
                const T P0 = pref_at(kp, y);
                const T dm = T(3) * (pref_at(kp, y == 0 ? ny - 1 : y - 1) - P0);
                const T dp = T(3) * (pref_at(kp, y == ny - 1 ? 0 : y + 1) - P0);
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    if (CY9[i] > 0) h[i] += w9<T>(i) * dm;
                    if (CY9[i] < 0) h[i] += w9<T>(i) * dp;
                }
            }
            return;
        }
        // nodes next to a wall: every link resolved with selects (no load in a
        // divergent branch); wall rules by side: bounce-back, specular
        // reflection (free slip), anti-bounce-back (Dirichlet scalars)
        const WallFlags wf(kp, x, y);
        const NbrE<M> nb(kp, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int cx = CX9[i], cy = CY9[i];
            const bool ox = wf.out_x(-cx), oy = wf.out_y(-cy);  // source x - c_i beyond a wall
            long long src = nb.at(-cx, -cy);
            int pl = OPP9[i];
            int dys = -cy;  // row of the source relative to y
            if (ox || oy) {
                src = nb.at(0, 0);  // bounce-back: the node's own reflected value (also corners)
                pl = i;
                dys = 0;
                if (ox != oy && kp.fbc[ox ? (cx > 0 ? 0 : 1) : (cy > 0 ? 2 : 3)] == LB_BC_FREESLIP) {
                    if (oy) {  // specular across a y-wall: from (x - c_x, y), direction mirrored
                        src = nb.at(-cx, 0);
                        pl = OPP9[MIRY9[i]];
                    } else {  // across an x-wall: from (x, y - c_y)
                        src = nb.at(0, -cy);
                        pl = OPP9[MIRX9[i]];
                        dys = -cy;
                    }
                }
            }
            h[i] = ld<NT>(pop + src + ((long long)(pl) << kBlkShift), kp, true);
            if (REF && kp.pref && dys != 0)
                h[i] += w9<T>(i) * (T(3) * (pref_at(kp, wrap_row(y + dys, kp.ny)) - pref_at(kp, y)));
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const int cx = CX5[i], cy = CY5[i];
                const bool out = wf.out_x(-cx) || wf.out_y(-cy);
                const int side = wf.out_x(-cx) ? (cx > 0 ? 0 : 1) : (cy > 0 ? 2 : 3);
                const long long src = out ? nb.at(0, 0) : nb.at(-cx, -cy);
                const T v = ld<NT>(pop + src + ((long long)(9 + 5 * a + (out ? i : OPP5[i])) << kBlkShift), kp, false);
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                f[a][i] = dir ? -v + T(2) * w5<T>(i) * kp.wallr[side][a] : v;
            }
    }
}

// ---- scatter ---------------------------------------------------------------
// PUSH = false: even step, post-collision value of direction i to own slot
// opp(i).  PUSH = true: odd step, to slot i of x + c_i, or by the wall rules.
template <class S, int M, bool PUSH, bool NT = false, bool REF = true, class T>
__device__ __forceinline__ void scatter(const KParams<T>& kp, S* __restrict__ pop, int x, int y,
                                        const T h[9], const T f[M][5], uint32_t salt) {
    const int nx = kp.nx;
    const long long n = (long long)y * nx + x;
    const uint32_t rw = sr_node(n, salt);  // FP16 only: random words of this node's values
    if constexpr (!PUSH) {
#pragma unroll
        for (int i = 0; i < 9; ++i) st_r<NT>(pop + pidx<M>(OPP9[i], n), h[i], kp, true, sr_word(rw, i));
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) st_r<NT>(pop + pidx<M>((9 + 5 * a + OPP5[i]), n), f[a][i], kp, false, sr_word(rw, 9 + 5 * a + i));
        return;
    } else {
        if (__all(no_wall_link(kp, x, y))) {  // wave-uniform choice: no lane pays for both paths
            const NbrE<M> nb(kp, x, y);
            if (REF && kp.pref) {   // a value pushed to row y + c_y is stored relative to that row's reference
                const int ny = kp.ny;
                const T P0 = pref_at(kp, y);
                const T dm = T(3) * (pref_at(kp, y == 0 ? ny - 1 : y - 1) - P0);
                const T dp = T(3) * (pref_at(kp, y == ny - 1 ? 0 : y + 1) - P0);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const T v = CY9[i] > 0 ? h[i] - w9<T>(i) * dp : (CY9[i] < 0 ? h[i] - w9<T>(i) * dm : h[i]);
                    st_r<NT>(pop + nb.at(CX9[i], CY9[i]) + ((long long)(i) << kBlkShift), v, kp, true, sr_word(rw, i));
                }
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st_r<NT>(pop + nb.at(CX9[i], CY9[i]) + ((long long)(i) << kBlkShift), h[i], kp, true, sr_word(rw, i));
            }
#pragma unroll
            for (int a = 0; a < M; ++a)
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    st_r<NT>(pop + nb.at(CX5[i], CY5[i]) + ((long long)(9 + 5 * a + i) << kBlkShift), f[a][i], kp, false,
                         sr_word(rw, 9 + 5 * a + i));
            return;
        }
        const WallFlags wf(kp, x, y);
        const NbrE<M> nb(kp, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int cx = CX9[i], cy = CY9[i];
            const bool ox = wf.out_x(cx), oy = wf.out_y(cy);  // target x + c_i beyond a wall
            long long dst = nb.at(cx, cy);
            int pl = i;
            int dyd = cy;  // row of the destination relative to y
            if (ox || oy) {
                dst = nb.at(0, 0);  // bounce-back into the node's own opposite slot (also corners)
                pl = OPP9[i];
                dyd = 0;
                if (ox != oy && kp.fbc[ox ? (cx > 0 ? 1 : 0) : (cy > 0 ? 3 : 2)] == LB_BC_FREESLIP) {
                    if (oy) {
                        dst = nb.at(cx, 0);
                        pl = MIRY9[i];
                    } else {
                        dst = nb.at(0, cy);
                        pl = MIRX9[i];
                        dyd = cy;
                    }
                }
            }
            T v = h[i];
            if (REF && kp.pref && dyd != 0)
                v -= w9<T>(i) * (T(3) * (pref_at(kp, wrap_row(y + dyd, kp.ny)) - pref_at(kp, y)));
            st_r<NT>(pop + dst + ((long long)(pl) << kBlkShift), v, kp, true, sr_word(rw, i));
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const int cx = CX5[i], cy = CY5[i];
                const bool out = wf.out_x(cx) || wf.out_y(cy);
                const int side = wf.out_x(cx) ? (cx > 0 ? 1 : 0) : (cy > 0 ? 3 : 2);
                const bool dir = out && kp.sbc[side][a] == LB_SBC_DIRICHLET;
                const T v = dir ? -f[a][i] + T(2) * w5<T>(i) * kp.wallr[side][a] : f[a][i];
                const long long dst = out ? nb.at(0, 0) : nb.at(cx, cy);
                st_r<NT>(pop + dst + ((long long)(9 + 5 * a + (out ? OPP5[i] : i)) << kBlkShift), v, kp, false,
                        sr_word(rw, 9 + 5 * a + i));
            }
    }
}

// ---- closures ---------------------------------------------------------------
template <class T>
__device__ __forceinline__ T cutoff_r(const KParams<T>& kp, T c) {
    if (kp.r_kind == LB_R_STEP) return c >= kp.cstar ? T(1) : T(0);
    const T d = c - kp.cstar;
    return T(0.5) * (T(1) + d / sqrt(d * d + kp.eps * kp.eps));
}

// Macroscopic quantities of one node (Eq. sum) in deviation form.
template <class T, int M>
struct Macro {
    T phid[M];  // phi - phi_ref
    T phi[M];
    T F[2];
    T u[2];
    T p;
};

template <class T, int M>
__device__ __forceinline__ void macro(const KParams<T>& kp, const T h[9], const T f[M][5], Macro<T, M>& mc) {
#pragma unroll
    for (int a = 0; a < M; ++a) {
        mc.phid[a] = ((f[a][0] + f[a][1]) + (f[a][2] + f[a][3])) + f[a][4];
        mc.phi[a] = kp.phi_ref[a] + mc.phid[a];
    }
    mc.F[0] = kp.F0[0];
    mc.F[1] = kp.F0[1];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        mc.F[0] += kp.Fphi[a][0] * mc.phi[a];
        mc.F[1] += kp.Fphi[a][1] * mc.phi[a];
    }
    const T jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const T jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    mc.u[0] = jx + T(0.5) * mc.F[0];
    mc.u[1] = jy + T(0.5) * mc.F[1];
    const T s = ((h[1] + h[2]) + (h[3] + h[4])) + ((h[5] + h[6]) + (h[7] + h[8]));
    const T usq = mc.u[0] * mc.u[0] + mc.u[1] * mc.u[1];
    // p = cs2/(1 - W0) [sum_{i>0} h_i - W0 u.u/(2 cs2) + (1/omega - 1/2) F_0] (appendix A)
    //   = (3/5)(s - (2/3) u.u - (tau_f - 1/2)(4/3) varphi u.F)
    T corr = T(0);
    if (kp.varphi != T(0)) corr = kp.vp_p * (mc.u[0] * mc.F[0] + mc.u[1] * mc.F[1]);
    mc.p = T(0.6) * ((s - (T(2) / T(3)) * usq) - corr);
}

// (lambda phi - phi)_b of Eq. feq-phi: zero unless lambda != I
template <class T, int M>
__device__ __forceinline__ T lam_excess(const KParams<T>& kp, const T phi[M], int b) {
    T x = T(0);
#pragma unroll
    for (int c = 0; c < M; ++c) x += kp.lamm[b * M + c] * phi[c];
    return x;
}

// ---- the node update ------------------------------------------------------
// CONS (FP32 storage): the scalar rest populations take the remainder of the
// species' post-collision mass in FP64, see below.
// gS (may be NULL; read only when kp.gam_on): gamma_a grad S_a / 6 per species
// and axis, the term of D-bar (Eq. evolution12) that acts like the auxiliary
// source.  Callers pass their local array itself, never a pointer chosen at run
// time: an array whose address is selected at run time lives in scratch memory.
template <class T, int M, int MODEL, int COLL, bool CONS = false>
__device__ __forceinline__ void collide(const KParams<T>& kp, T h[9], T f[M][5], const T Sold[M], T Snew[M],
                                        const T (*gS)[2] = nullptr) {
    Macro<T, M> mc;
    macro<T, M>(kp, h, f, mc);
    double mass_in[M];  // exact sums of the stored (FP32) input populations
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a)
            mass_in[a] = (((double)f[a][0] + (double)f[a][1]) + ((double)f[a][2] + (double)f[a][3])) + (double)f[a][4];
    }

    // relaxation matrix, Eq. omega-D with lambda = I: omega = (3 D + I/2)^-1
    T om[M][M];
    T S[M];
    if constexpr (MODEL == LB_MODEL_CHEMOTAXIS) {
        const T r = cutoff_r(kp, mc.phi[1]);
        const T a = T(3) * kp.Dc[0] + T(0.5);
        const T b = T(3) * (kp.Dc[1] - kp.chi * r * mc.phi[0]);
        const T c = T(3) * kp.Dc[2];
        const T d = T(3) * kp.Dc[3] + T(0.5);
        T idet;
        if constexpr (std::is_same_v<T, float>)
            idet = __builtin_amdgcn_rcpf(a * d - b * c);  // 1-ulp reciprocal: the FP32 paths carry ~1e-7 anyway
        else
            idet = T(1) / (a * d - b * c);
        om[0][0] = d * idet;
        om[0][1] = -b * idet;
        om[1][0] = -c * idet;
        om[1][1] = a * idet;
        S[0] = T(0);
        S[1] = -kp.beta * r * mc.phi[0];
    } else {
#pragma unroll
        for (int a = 0; a < M; ++a) {
#pragma unroll
            for (int b = 0; b < M; ++b) om[a][b] = kp.omega[a * M + b];
            S[a] = T(0);
            if (kp.src_mask >> a & 1) {
#pragma unroll
                for (int b = 0; b < M; ++b) S[a] += kp.K[a * M + b] * mc.phi[b];
            }
        }
    }

    // auxiliary source, Eq. Gi: G_{i,a} = 3 W_i c_i . g_a with
    // g_a = sum_b (delta_ab - omega_ab/2)(u S_b + phi_b F)
    T g[M][2];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        g[a][0] = T(0);
        g[a][1] = T(0);
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const T cf = (a == b ? T(1) : T(0)) - T(0.5) * om[a][b];
            g[a][0] += cf * (mc.u[0] * S[b] + mc.phi[b] * mc.F[0]);
            g[a][1] += cf * (mc.u[1] * S[b] + mc.phi[b] * mc.F[1]);
        }
    }
    // gamma of D-bar: (dt^2/2) gamma_a c_i . grad S_{i,a} with S_i = W_i S (Eq. source)
    // is 3 W_i c_i . (gamma_a grad S_a / 6), the form of G_i above
    if (gS && kp.gam_on) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            g[a][0] += gS[a][0];
            g[a][1] += gS[a][1];
        }
    }
    // source with its time-derivative correction (Eq. source, gamma = 0):
    // dt S_i + (dt/2)(S_i(t) - S_i(t - dt)) = W_i (3/2 S - 1/2 S_old)
    T src[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        src[a] = T(1.5) * S[a] - T(0.5) * Sold[a];
        Snew[a] = S[a];
    }

    // scalar matrix collision (Eq. evolution12), f^eq of Eq. feq-phi with
    // vartheta = 0 in deviation form: W_i (phid + 3 phi c.u), plus (lambda phi -
    // phi)/6 on the moving directions when lambda != I (the D2Q5 form whose
    // second moment is cs2 (lambda phi - phi)).  The rest direction takes the
    // remainder, f^eq_0 = phid - sum_{i>0} f^eq_i (and likewise for W_i S):
    // with rounded weights sum_i W_i != 1, which would create or destroy mass
    // by the same fraction at every step.
    // The non-equilibrium part f - f^eq is formed first (with omega close to 2
    // the expanded (1 - omega) f + omega f^eq loses accuracy in FP32); the
    // source and auxiliary-source terms are node constants per species and
    // direction, W_i src_a + 3 W_i c_i . g_a = src_a/6 +- g_a,x/2 or +- g_a,y/2
    // on the moving directions.
    T feq[M][5], add[M][5];
#pragma unroll
    for (int b = 0; b < M; ++b) {
        T pd = mc.phid[b];
        if constexpr (MODEL != LB_MODEL_CHEMOTAXIS)
            if (kp.lam_on) pd += lam_excess<T, M>(kp, mc.phi, b);
        const T iso = pd * (T(1) / T(6));
        const T adv = T(0.5) * mc.phi[b];  // 3 W_i phi for i > 0
        feq[b][1] = iso + adv * mc.u[0];
        feq[b][3] = iso - adv * mc.u[0];
        feq[b][2] = iso + adv * mc.u[1];
        feq[b][4] = iso - adv * mc.u[1];
        feq[b][0] = mc.phid[b] - T(4) * iso;
        const T s6 = src[b] * (T(1) / T(6));
        const T gx = T(0.5) * g[b][0], gy = T(0.5) * g[b][1];
        add[b][1] = s6 + gx;
        add[b][3] = s6 - gx;
        add[b][2] = s6 + gy;
        add[b][4] = s6 - gy;
        add[b][0] = src[b] - T(4) * s6;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        T neq[M];
#pragma unroll
        for (int b = 0; b < M; ++b) neq[b] = f[b][i] - feq[b][i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            T acc = f[a][i] + add[a][i];
#pragma unroll
            for (int b = 0; b < M; ++b) acc -= om[a][b] * neq[b];
            f[a][i] = acc;
        }
    }
    // In exact arithmetic the collision changes the mass of species a by its
    // source only, sum_i f*_a,i = sum_i f_a,i + src_a.  Evaluated in FP32 its
    // rounding errors are deterministic functions of smooth fields and add up
    // coherently over nodes and steps (a slow systematic drift of the mass).
    // With FP32 storage the rest population takes the remainder computed in
    // FP64 from the stored inputs and the other four outputs, which are exact
    // in FP64, so that the only error left is the final rounding of f*_0.
    if constexpr (CONS) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double moving = ((double)f[a][1] + (double)f[a][2]) + ((double)f[a][3] + (double)f[a][4]);
            f[a][0] = T((mass_in[a] + (double)src[a]) - moving);
        }
    }

    // fluid: h^eq of Eq. heq, F_i of Eq. force
    const T usq = mc.u[0] * mc.u[0] + mc.u[1] * mc.u[1];
    // h^eq_0 = rho0 - sum_{i>0} h^eq_i (Eq. momentNS: sum_i h^eq_i = rho0), which
    // equals sigma_0 - W_0 u.u/(2 cs2) of Eq. heq without a rounding bias
    T heq[9], Fi[9];
    T hsum = T(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const T wi = w9<T>(i);
        const T cu = T(CX9[i]) * mc.u[0] + T(CY9[i]) * mc.u[1];
        heq[i] = wi * (T(3) * mc.p + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
        hsum += heq[i];
    }
    heq[0] = kp.rho0_eff - hsum;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T cF = T(CX9[i]) * mc.F[0] + T(CY9[i]) * mc.F[1];
        Fi[i] = T(3) * w9<T>(i) * cF;
    }
    if (kp.varphi != T(0)) {
        // varphi W_i (uF + Fu):(c c - cs2 I)/(2 cs2^2) = varphi W_i (9 (c.u)(c.F) - 3 u.F)
        const T uF = mc.u[0] * mc.F[0] + mc.u[1] * mc.F[1];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T cF = T(CX9[i]) * mc.F[0] + T(CY9[i]) * mc.F[1];
            const T cu = T(CX9[i]) * mc.u[0] + T(CY9[i]) * mc.u[1];
            Fi[i] += kp.varphi * w9<T>(i) * (T(9) * cu * cF - T(3) * uF);
        }
    }
    const T w = kp.omega_f;
    if constexpr (COLL == LB_COLL_BGK) {
        const T fc = T(1) - T(0.5) * w;
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = h[i] - w * (h[i] - heq[i]) + fc * Fi[i];
    } else {
        T dm[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            T mne = T(0), mf = T(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (MM[k][i] != 0) {
                    mne += T(MM[k][i]) * (h[i] - heq[i]);
                    mf += T(MM[k][i]) * Fi[i];
                }
            }
            const T s = (k >= 7) ? w : kp.mrt_s[k];
            dm[k] = (-s * mne + (T(1) - T(0.5) * s) * mf) / T(MNORM[k]);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < 9; ++k)
                if (MM[k][i] != 0) acc += T(MM[k][i]) * dm[k];
            h[i] = h[i] + acc;
        }
    }
}

// ---- XCD-aware block placement ----------------------------------------------
// Workgroups are dealt round-robin to the 8 XCDs.  Remap so that each XCD
// processes one contiguous run of tiles: neighbouring tiles (which share
// cache lines of the shifted odd-step accesses) then sit in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// deterministic block reduction of NV doubles (wave64 shuffles, then LDS)
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV], double* __restrict__ dst) {
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[wid][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x, nw = (int)(blockDim.x + 63) >> 6;  // 1..4 wavefronts
        double t = red[0][k];
        for (int w = 1; w < nw; ++w) t += red[w][k];
        dst[k] = t;
    }
}

// ---- launch helpers ----------------------------------------------------------
static inline void* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

template <class S>
static const KParams<typename St<S>::T>& kpar(const KParams<double>& kd, const KParams<float>& kf) {
    if constexpr (std::is_same<typename St<S>::T, double>::value)
        return kd;
    else
        return kf;
}

// calls fn.template operator()<S, M, MODEL>() for the runtime storage/m/model
template <class Fn>
static hipError_t dispatch(const lb_params& p, Fn&& fn) {
    auto by_m = [&](auto sTag) -> hipError_t {
        using S = decltype(sTag);
        if (p.model == LB_MODEL_CHEMOTAXIS) return fn.template operator()<S, 2, LB_MODEL_CHEMOTAXIS>();
        switch (p.m) {
            case 1: return fn.template operator()<S, 1, LB_MODEL_LINEAR>();
            case 2: return fn.template operator()<S, 2, LB_MODEL_LINEAR>();
            case 3: return fn.template operator()<S, 3, LB_MODEL_LINEAR>();
            case 4: return fn.template operator()<S, 4, LB_MODEL_LINEAR>();
        }
        return hipErrorInvalidValue;
    };
    if (p.model != LB_MODEL_LINEAR && p.model != LB_MODEL_CHEMOTAXIS) return hipErrorInvalidValue;
    switch (p.storage) {
        case LB_STORE_F64: return by_m(double{});
        case LB_STORE_F32: return by_m(float{});
        case LB_STORE_F16: return by_m(_Float16{});
    }
    return hipErrorInvalidValue;
}

static inline unsigned blocks_for(size_t N) { return (unsigned)((N + 255) / 256); }

}  // namespace lbk
