// sg_kernels.hip -- CNN surrogate on the gfx950 matrix cores: 3x3 convolutions
// as implicit GEMMs with bfloat16 operands and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), fused bias/SiLU epilogues, weight gradients by
// split-K implicit GEMM with a deterministic reduction, MSE loss and Adam.
//
// Tensors are channels-last: pixel p = (b H + y) W + x, channel contiguous.
// A convolution  z[p][co] = b[co] + sum_{tap, ci} w[co][tap][ci] x[p + off(tap)][ci]
// is the GEMM  Z[M = pixels][N = co] = A[M][K = (tap, ci)] B[K][N]  with
// A gathered from the shifted input (zero outside the image) and B the
// weights; the data gradient is the same GEMM with the transposed, flipped
// weights, and the weight gradient is  dW[co][(tap, ci)] = sum_p dZ[p][co]
// x[p + off(tap)][ci]  (K = pixels, split over workgroups).
//
// Workgroup tile 64 x 64 (4 wavefronts of 32 x 32, each 2 x 2 MFMA blocks of
// 16 x 16), K step 32 staged through LDS.  MFMA operand layout (16x16x32):
// lane l holds A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16], j < 8,
// and D[4 (l / 16) + j][l % 16], j < 4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sg.h"

namespace sgk {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));

constexpr int kLayers = SG_LAYERS;
constexpr int kCin[kLayers] = {15, 64, 128, 64, 64, 64};
constexpr int kCout[kLayers] = {64, 128, 64, 64, 64, 4};
constexpr int kCinPad[kLayers] = {32, 64, 128, 64, 64, 64};
constexpr int kCoutPad[kLayers] = {64, 128, 64, 64, 64, 64};
constexpr int kMaxC = 128;
constexpr int kFeat = 15;
constexpr int kSplit = 128;     // split-K factor of the weight gradient
constexpr int kRed = 256;       // blocks of the first pass of small reductions
constexpr int kMseBlocks = 1024;  // blocks of the loss pass (four per CU: its loads need the parallelism)
constexpr int kIdxSteps = 256;  // batches of sample indices the workspace holds (training epochs upload them at once)
constexpr int LDSK = 32;        // LDS row pitch in bf16 of the convolution tiles (32 channels, no pad)

// Offset (bf16) of the 16-byte segment seg (8 channels) of row `row` in a
// convolution tile: the segment index is XOR-swizzled with ((row >> 1) ^
// (row >> 3)) & 3, so that the segment stores of two adjacent rows and the
// MFMA operand reads (16 rows, one segment) spread over distinct LDS banks.
__device__ __forceinline__ int tile_off(int row, int seg) {
    return row * LDSK + (((seg ^ (row >> 1) ^ (row >> 3)) & 3) << 3);
}

// ---- features ------------------------------------------------------------
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ params, const int* __restrict__ idx,
                                                  int nb, int H, int W, bf16* __restrict__ x) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long P = (long long)nb * H * W;
    if (p >= P) return;
    const int b = (int)(p / ((long long)H * W));
    const int rem = (int)(p % ((long long)H * W));
    const int yi = rem / W, xi = rem % W;
    const float* pr = params + (long long)idx[b] * SG_IN_PARAMS;
    const float xc = (xi + 0.5f) / W, yc = (yi + 0.5f) / H;
    const float pi = 3.14159265358979f;
    float f[kFeat] = {pr[0], pr[1], pr[2], pr[3], pr[4], xc, yc,
                      sinf(pi * xc), cosf(pi * xc), sinf(2 * pi * xc), cosf(2 * pi * xc),
                      sinf(pi * yc), cosf(pi * yc), sinf(2 * pi * yc), cosf(2 * pi * yc)};
    bf16* o = x + p * kCinPad[0];
#pragma unroll
    for (int c = 0; c < kCinPad[0]; ++c) o[c] = bf16(c < kFeat ? f[c] : 0.0f);
}

// SiLU and its derivative with gfx950's 1-ulp reciprocal instead of a correctly
// rounded division: the results are stored in bfloat16 (8 mantissa bits), and the
// division's scale/fixup sequence was ~10 % of the convolutions' time (forward
// 42 -> 39 us, data gradient 39 -> 35 us at 64 channels, 16 x 128^2)
__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---- implicit-GEMM convolution -------------------------------------------
// MODE 0 (forward): z = acc + bias; Zout = z; Yout = bf16(act ? SiLU(z) : z).
// MODE 1 (data gradient): Yout = bf16(acc * SiLU'(Zprev)).
template <int MODE>
__global__ __launch_bounds__(256) void k_conv(const bf16* __restrict__ X, const bf16* __restrict__ Wk,
                                              const float* __restrict__ bias, const float* __restrict__ Zprev,
                                              float* __restrict__ Zout, bf16* __restrict__ Yout, int H, int W,
                                              int Cin, int Cout, int act) {
    __shared__ __attribute__((aligned(16))) bf16 As[64 * LDSK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[64 * LDSK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_per_row = W >> 6;
    const int img_row = blockIdx.x / tiles_per_row;  // b * H + y
    const int x0 = (blockIdx.x % tiles_per_row) << 6;
    const int y = img_row % H;
    const int n0 = blockIdx.y << 6;
    const int sj = tid >> 2, sq = tid & 3;
    const int wr = (wave >> 1) << 5, wc = (wave & 1) << 5;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int yy = y + dy, xx = x0 + sj + dx;
        const bool in = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W);
        const long long src = ((long long)(img_row + dy) * W + xx) * Cin;
        const long long wsrc = ((long long)(n0 + sj) * 9 + tap) * Cin;
        for (int c0 = 0; c0 < Cin; c0 += 32) {
            uint4 va = make_uint4(0u, 0u, 0u, 0u);
            if (in) va = *reinterpret_cast<const uint4*>(X + src + c0 + 8 * sq);
            *reinterpret_cast<uint4*>(&As[tile_off(sj, sq)]) = va;
            *reinterpret_cast<uint4*>(&Bs[tile_off(sj, sq)]) =
                *reinterpret_cast<const uint4*>(Wk + wsrc + c0 + 8 * sq);
            __syncthreads();
            const int r = lane & 15;
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&As[tile_off(wr + r, lane >> 4)]);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&As[tile_off(wr + 16 + r, lane >> 4)]);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&Bs[tile_off(wc + r, lane >> 4)]);
            const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&Bs[tile_off(wc + 16 + r, lane >> 4)]);
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
            __syncthreads();
        }
    }
    const long long pbase = (long long)img_row * W + x0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = wr + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + wc + 16 * j + (lane & 15);
                const long long o = (pbase + m) * Cout + n;
                const float v = acc[i][j][e];
                if constexpr (MODE == 0) {
                    const float z = v + bias[n];
                    if (Zout) Zout[o] = z;
                    if (Yout) Yout[o] = bf16(act ? silu(z) : z);
                } else {
                    Yout[o] = bf16(v * silu_grad(Zprev[o]));
                }
            }
}

// Same convolution with a workgroup tile of 128 pixels (one image row of 128
// or half a longer one) x 64 output channels: each wavefront computes 32
// pixels x 64 channels, so every K step issues 8 MFMAs per 6 LDS operand reads
// (4 per 4 in k_conv).  Needs W % 128 == 0.
// 16 zero bytes: the source of the LDS DMA loads of pixels outside the image
__device__ const uint4 kZero16 = {0u, 0u, 0u, 0u};

typedef __attribute__((address_space(3))) void lds_void;

// wait until at most N vector-memory operations of this wave are outstanding
// (LDS DMA loads count there until their data is in LDS); other counters untouched
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

constexpr int kStages = 3;                          // LDS ring depth of k_conv128
constexpr int kStageElems = (128 + 64) * LDSK;      // bf16 per stage: A tile, then B tile
// LDS DMA loads per thread and stage in k_conv128: one load of a wavefront
// fills 16 tile rows (64 lanes x 16 bytes, 4 lanes per 64-byte row), so the
// 128-row A tile takes 2 per wavefront and the 64-row B tile 1 (4 wavefronts).
// compute() waits for all but the loads of the later stages: kLoadsPerStage
// times the number of stages issued after its own.
constexpr int kWaves128 = 4, kRowsPerLoad = 16;
constexpr int kLoadsA = 128 / (kRowsPerLoad * kWaves128), kLoadsB = 64 / (kRowsPerLoad * kWaves128);
constexpr int kLoadsPerStage = kLoadsA + kLoadsB;
static_assert(kLoadsA * kRowsPerLoad * kWaves128 == 128 && kLoadsB * kRowsPerLoad * kWaves128 == 64,
              "the tiles must be whole multiples of the rows one round of loads fills");
static_assert(kLoadsPerStage * (kStages - 1) < 16, "wait_vm takes counts below 16 here");

template <int MODE>
__global__ __launch_bounds__(256) void k_conv128(const bf16* __restrict__ X, const bf16* __restrict__ Wk,
                                                 const float* __restrict__ bias, const float* __restrict__ Zprev,
                                                 float* __restrict__ Zout, bf16* __restrict__ Yout, int H, int W,
                                                 int Cin, int Cout, int act) {
    // kStages LDS stages (A: 128 pixels x 32 channels, B: 64 output channels x
    // 32 channels), filled by LDS DMA (global_load_lds): kStages - 1 K steps
    // are in flight while the matrix cores work on one, with no staging registers
    __shared__ __attribute__((aligned(16))) bf16 Sbuf[kStages * kStageElems];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_per_row = W >> 7;
    const int img_row = blockIdx.x / tiles_per_row;  // b * H + y
    const int x0 = (blockIdx.x % tiles_per_row) << 7;
    const int y = img_row % H;
    const int n0 = blockIdx.y << 6;
    const int wr = wave << 5;
    floatx4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // A DMA load writes 64 lanes x 16 bytes = 16 tile rows at the wave's base;
    // lane l fills row 16 c + l / 4, LDS segment l % 4, from global segment
    // (l % 4) ^ swz(row), which is where tile_off() looks for it
    const int rsub = lane >> 2, pseg = lane & 3;
    const int nc = Cin >> 5, nsteps = 9 * nc;
    auto issue = [&](int st, bf16* As, bf16* Bs) {
        const int tap = st / nc, c0 = (st - tap * nc) << 5;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int yy = y + dy;
        const bool rowin = (yy >= 0) & (yy < H);
#pragma unroll
        for (int q = 0; q < kLoadsA; ++q) {
            const int blk = wave + kWaves128 * q;          // 16-row block of the A tile
            const int row = kRowsPerLoad * blk + rsub;     // pixel x0 + row
            const int seg = (pseg ^ (row >> 1) ^ (row >> 3)) & 3;
            const int xx = x0 + row + dx;
            const bool in = rowin & (xx >= 0) & (xx < W);
            const void* src = in ? (const void*)(X + ((long long)(img_row + dy) * W + xx) * Cin + c0 + 8 * seg)
                                 : (const void*)&kZero16;
            __builtin_amdgcn_global_load_lds(src, (lds_void*)(As + (kRowsPerLoad * blk) * LDSK), 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < kLoadsB; ++q) {
            const int blk = wave + kWaves128 * q;          // 16-row block of the B tile
            const int row = kRowsPerLoad * blk + rsub;     // output channel n0 + row
            const int seg = (pseg ^ (row >> 1) ^ (row >> 3)) & 3;
            __builtin_amdgcn_global_load_lds((const void*)(Wk + ((long long)(n0 + row) * 9 + tap) * Cin + c0 + 8 * seg),
                                             (lds_void*)(Bs + (kRowsPerLoad * blk) * LDSK), 16, 0, 0);
        }
    };
    auto lds_addr = [](const bf16* p) { return (uint32_t)(uintptr_t)p; };
    // later: stages issued after this one (their kLoadsPerStage loads each may still be in flight)
    auto compute = [&](const bf16* As, const bf16* Bs, int later) {
        // this wave's loads of this stage have landed, later stages may still be in flight ...
        static_assert(kStages - 1 <= 2, "extend the cases below with the ring depth");
        switch (later) {
            case 2: wait_vm<2 * kLoadsPerStage>(); break;
            case 1: wait_vm<kLoadsPerStage>(); break;
            default: wait_vm<0>(); break;
        }
        __builtin_amdgcn_s_barrier();  // ... and every other wave's
        const int r = lane & 15, sg = lane >> 4;
        // The six operand reads are written as one asm block that waits for
        // them itself: as plain loads, the compiler cannot tell them from the
        // LDS DMA writes still in flight to the other stages and waits for
        // all vector-memory operations first (vmcnt(0)), which serialises the
        // pipeline.
        bf16x8 a0, a1, b0, b1, b2, b3;
        asm volatile(
            "ds_read_b128 %0, %6\n\t"
            "ds_read_b128 %1, %7\n\t"
            "ds_read_b128 %2, %8\n\t"
            "ds_read_b128 %3, %9\n\t"
            "ds_read_b128 %4, %10\n\t"
            "ds_read_b128 %5, %11\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(a0), "=&v"(a1), "=&v"(b0), "=&v"(b1), "=&v"(b2), "=&v"(b3)
            : "v"(lds_addr(&As[tile_off(wr + r, sg)])), "v"(lds_addr(&As[tile_off(wr + 16 + r, sg)])),
              "v"(lds_addr(&Bs[tile_off(r, sg)])), "v"(lds_addr(&Bs[tile_off(16 + r, sg)])),
              "v"(lds_addr(&Bs[tile_off(32 + r, sg)])), "v"(lds_addr(&Bs[tile_off(48 + r, sg)]))
            : "memory");
        const bf16x8 bj[4] = {b0, b1, b2, b3};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bj[j], acc[0][j], 0, 0, 0);
            acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bj[j], acc[1][j], 0, 0, 0);
        }
        __builtin_amdgcn_s_barrier();  // every wave is done reading this stage before it is refilled
    };
    auto stage_a = [&](int st) { return Sbuf + (st % kStages) * kStageElems; };
    auto stage_b = [&](int st) { return Sbuf + (st % kStages) * kStageElems + 128 * LDSK; };
#pragma unroll
    for (int k = 0; k < kStages - 1; ++k)
        if (k < nsteps) issue(k, stage_a(k), stage_b(k));
    for (int st = 0; st < nsteps; ++st) {
        if (st + kStages - 1 < nsteps) issue(st + kStages - 1, stage_a(st + kStages - 1), stage_b(st + kStages - 1));
        const int later = min(kStages - 1, nsteps - 1 - st);  // stages issued after this one
        compute(stage_a(st), stage_b(st), later);
    }
    const long long pbase = (long long)img_row * W + x0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = wr + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + 16 * j + (lane & 15);
                const long long o = (pbase + m) * Cout + n;
                const float v = acc[i][j][e];
                if constexpr (MODE == 0) {
                    const float z = v + bias[n];
                    if (Zout) Zout[o] = z;
                    if (Yout) Yout[o] = bf16(act ? silu(z) : z);
                } else {
                    Yout[o] = bf16(v * silu_grad(Zprev[o]));
                }
            }
}

// ---- persistent row-streaming convolution (width 128, K channels 32 or 64) ----
// One workgroup owns 64 output channels and a run of whole image rows of 128
// pixels.  Its weights (all 9 taps) stay in LDS for the whole run; the input
// rows pass through a ring of 4 LDS slots.  Eight wavefronts form two groups of
// four that take alternate output rows, out of phase: in each step group A
// computes row Ra and then stores it, while group B first stores its row of the
// previous step and then computes row Ra + 1, so that one group's epilogue
// (bias, SiLU, BF16 conversion, stores) runs beside the other group's matrix
// work.  Wavefront w of a group computes pixels 32 w .. 32 w + 31 x 64 channels
// on the 32x32x16 bf16 MFMA, its operand reads issued two K steps ahead of the
// MFMAs that take them; the outputs leave straight from the accumulator layout
// (per element, two runs of 32 consecutive channels).  The rows of the next
// step come in through plain loads held in registers during the step and are
// written to the two slots that the step has finished with (two barriers per
// step of two rows).
constexpr int kRowW = 128;       // image width handled by the row kernels
constexpr int kRowPx = kRowW + 2;   // an input row with its two halo pixels
// 16-byte segment swizzle of LDS rows of CK bf16 (pixels of an input row, or output channels of a
// weight tap): consecutive rows that would start on the same banks get different segments, so that
// 16 lanes reading one logical segment of 16 consecutive rows hit 64 distinct banks
template <int CK> __device__ __forceinline__ int swz(int row) { return (row / (128 / CK)) & (CK / 8 - 1); }

// MODE 0 (forward): z = acc + bias, stored when ZO; y = bf16(act ? SiLU(z) : z), stored when YO.
// MODE 1 (data gradient): y = bf16(acc * SiLU'(Zprev)) (ZO false, YO true).
// The K channels of a tap are X's channels koff .. koff + CK - 1 of xcs (the weights' K stride
// is xcs too).  KS = 0: all of them in one launch.  With more K channels than the LDS holds
// beside the ring, two forward launches: KS = 1 stores the raw sums of the first CK channels
// to Zpart (FP32, [pixel][Cout]); KS = 2 adds them to its own before the bias.
template <int MODE, int CK, bool ZO, bool YO, int KS>
__global__ __launch_bounds__(512, 1) void k_conv_rows(const bf16* __restrict__ X, const bf16* __restrict__ Wk,
        const float* __restrict__ bias, const float* __restrict__ Zprev, float* __restrict__ Zout,
        bf16* __restrict__ Yout, float* __restrict__ Zpart, int H, int rows_total, int rows_per_wg, int Cout, int act,
        int xcs, int koff) {
    static_assert(CK == 32 || CK == 64, "the K channels of a tap are 32 or 64");
    static_assert(MODE == 0 || (!ZO && YO), "the data gradient stores y only");
    static_assert(KS != 1 || (!ZO && !YO), "the first of two K launches stores the partial sums only");
    static_assert(KS == 0 || MODE == 0, "two K launches for the forward only");
    constexpr int S = CK / 8;                       // 16-byte segments per pixel / per weight row
    constexpr int kWts = 9 * 64 * CK;               // bf16 of the workgroup's weights
    constexpr int kSlot = kRowPx * CK;              // bf16 per ring slot
    constexpr int kPieces = kRowPx * S;             // 16-byte pieces per input row
    constexpr int kPer = (kPieces + 255) / 256;     // pieces per thread of a group (the last round partial)
    __shared__ __attribute__((aligned(16))) bf16 Wts[kWts];
    __shared__ __attribute__((aligned(16))) bf16 Ring[4 * kSlot];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = wave >> 2, pw = wave & 3, gtid = tid & 255;
    const int n0 = blockIdx.y << 6;
    const int R0 = blockIdx.x * rows_per_wg;
    const int R1 = min(R0 + rows_per_wg, rows_total);
    if (R0 >= R1) return;

    // weights of the workgroup's 64 output channels: piece q = (tap 64 + co) S + s holds the
    // 8 channels (s ^ swz(co)); the rounds in an order rotated per workgroup, since all
    // workgroups read the same weights and starting on the same lines would queue on the same
    // L2 channels
    constexpr int kWPieces = kWts / 8, kWRounds = (kWPieces + 511) / 512;
    for (int rr = 0; rr < kWRounds; ++rr) {
        const int r = (rr + (int)blockIdx.x) % kWRounds;
        const int q = r * 512 + tid;
        if (q < kWPieces) {
            const int tap = q / (64 * S), co = (q / S) % 64, ps = q % S;
            const int ls = ps ^ swz<CK>(co);
            *reinterpret_cast<uint4*>(Wts + (size_t)q * 8) =
                *reinterpret_cast<const uint4*>(Wk + ((long long)(n0 + co) * 9 + tap) * xcs + koff + 8 * ls);
        }
    }
    // input row Rg (zero outside 0..rows_total-1) by one group: piece q = px S + s, pixel px
    // of the row with halo (image column px - 1), segment s holding the channels (s ^ swz(px))
    auto fetch_row = [&](int Rg, uint4 (&v)[kPer]) {
        const bool rin = Rg >= 0 && Rg < rows_total;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int q = r * 256 + gtid;
            const int px = q / S, ls = (q % S) ^ swz<CK>(px);
            const int x = px - 1;
            const bool in = rin && q < kPieces && x >= 0 && x < kRowW;
            v[r] = in ? *reinterpret_cast<const uint4*>(X + ((long long)Rg * kRowW + x) * xcs + koff + 8 * ls)
                      : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto put_row = [&](int Rg, const uint4 (&v)[kPer]) {   // into ring slot Rg & 3
        bf16* slot = Ring + (size_t)(Rg & 3) * kSlot;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int q = r * 256 + gtid;
            if (q < kPieces) *reinterpret_cast<uint4*>(slot + (size_t)q * 8) = v[r];
        }
    };
    {
        uint4 v[kPer];
        fetch_row(R0 - 1 + grp, v);
        put_row(R0 - 1 + grp, v);
        fetch_row(R0 + 1 + grp, v);
        put_row(R0 + 1 + grp, v);
    }
    __syncthreads();

    const int l32 = lane & 31, kg = lane >> 5;
    const int swzw = swz<CK>(l32);   // weight-row swizzle (output channels l32 and 32 + l32 alike)
    const float bc0 = MODE == 0 ? bias[n0 + l32] : 0.f, bc1 = MODE == 0 ? bias[n0 + 32 + l32] : 0.f;
    // accumulator element j of lane l: output pixel 32 pw + 8 (j >> 2) + 4 kg + (j & 3) of the
    // row, channels l32 (first accumulator) and 32 + l32 (second)
    auto out_off = [&](int Rp, int j) {
        return ((long long)Rp * kRowW + 32 * pw + 8 * (j >> 2) + 4 * kg + (j & 3)) * Cout + n0 + l32;
    };
    auto compute = [&](int R, floatx16& acc0, floatx16& acc1) {
#pragma unroll
        for (int e = 0; e < 16; ++e) acc0[e] = acc1[e] = 0.f;
        constexpr int PD = 2;                        // operand reads run PD K steps ahead
        constexpr int HS = CK / 16, NS = 9 * HS;     // K steps per tap, per row
        auto ld = [&](int st, bf16x8& a, bf16x8& b0, bf16x8& b1) {
            const int t = st / HS, h = st % HS, dyi = t / 3, dxi = t % 3;
            const bf16* slot = Ring + (size_t)((R + dyi - 1) & 3) * kSlot;
            const int pxi = 32 * pw + l32 + dxi;    // pixel (with halo) feeding output pixel 32 pw + l32
            a = *reinterpret_cast<const bf16x8*>(slot + (size_t)pxi * CK + 8 * ((2 * h + kg) ^ swz<CK>(pxi)));
            const bf16* brow0 = Wts + (size_t)(t * 64 + l32) * CK;
            b0 = *reinterpret_cast<const bf16x8*>(brow0 + 8 * ((2 * h + kg) ^ swzw));
            b1 = *reinterpret_cast<const bf16x8*>(brow0 + (size_t)32 * CK + 8 * ((2 * h + kg) ^ swzw));
        };
        const int y = R % H;
        if (y > 0 && y < H - 1) {
            bf16x8 A[PD + 1], B0[PD + 1], B1[PD + 1];
#pragma unroll
            for (int st = 0; st < PD; ++st) ld(st, A[st], B0[st], B1[st]);
            __builtin_amdgcn_sched_group_barrier(0x100, 3 * PD, 0);   // the first PD steps' LDS reads
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                constexpr int NB = PD + 1;
                if (st + PD < NS) ld(st + PD, A[(st + PD) % NB], B0[(st + PD) % NB], B1[(st + PD) % NB]);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[st % NB], B0[st % NB], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[st % NB], B1[st % NB], acc1, 0, 0, 0);
                // keep the order: the reads of step st + PD, then the two MFMAs of step st
                if (st + PD < NS) __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            }
        } else {   // first or last row of an image: the tap row outside contributes nothing
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                const int dyi = (st / HS) / 3;
                if ((dyi == 0 && y == 0) || (dyi == 2 && y == H - 1)) continue;
                bf16x8 a, b0, b1;
                ld(st, a, b0, b1);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
            }
        }
    };
    // pre-activations of row Rp (data gradient), or the first K launch's sums (forward, KS = 2)
    auto load_z = [&](int Rp, float (&z0)[16], float (&z1)[16]) {
        const float* src = MODE == 1 ? Zprev : Zpart;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const long long o = out_off(Rp, j);
            z0[j] = src[o];
            z1[j] = src[o + 32];
        }
    };
    constexpr bool kLoadZ = MODE == 1 || KS == 2;
    auto epi = [&](int Rp, const floatx16& a0, const floatx16& a1, const float (&z0)[16], const float (&z1)[16]) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const long long o = out_off(Rp, j);
            if constexpr (KS == 1) {
                Zpart[o] = a0[j];
                Zpart[o + 32] = a1[j];
            } else if constexpr (MODE == 0) {
                const float v0 = (KS == 2 ? a0[j] + z0[j] : a0[j]) + bc0, v1 = (KS == 2 ? a1[j] + z1[j] : a1[j]) + bc1;
                if constexpr (ZO) {
                    Zout[o] = v0;
                    Zout[o + 32] = v1;
                }
                if constexpr (YO) {
                    Yout[o] = bf16(act ? silu(v0) : v0);
                    Yout[o + 32] = bf16(act ? silu(v1) : v1);
                }
            } else {
                Yout[o] = bf16(a0[j] * silu_grad(z0[j]));
                Yout[o + 32] = bf16(a1[j] * silu_grad(z1[j]));
            }
        }
    };

    floatx16 acc0, acc1;   // group A: this step's row; group B: its row, stored at the next step
    float z0[16], z1[16];  // data gradient: the pre-activations of the same row
    for (int Ra = R0; Ra < R1; Ra += 2) {
        const int Rb = Ra + 1;
        // rows Ra + 3 (group A) and Ra + 4 (group B) for the next step, which reads rows
        // Ra + 1 .. Ra + 4; loaded now, written after every wave is done with rows Ra - 1, Ra
        const int Rn = Ra + 3 + grp;
        uint4 pre[kPer];
        fetch_row(Ra + 2 < R1 ? Rn : -1, pre);
        if (grp == 0) {
            if constexpr (kLoadZ) load_z(Ra, z0, z1);
            compute(Ra, acc0, acc1);
            epi(Ra, acc0, acc1, z0, z1);
        } else {
            if (Ra > R0) epi(Ra - 1, acc0, acc1, z0, z1);
            if (Rb < R1) {
                if constexpr (kLoadZ) load_z(Rb, z0, z1);
                compute(Rb, acc0, acc1);
            }
        }
        __syncthreads();
        put_row(Rn, pre);   // into the slots of rows Ra - 1 and Ra
        __syncthreads();
    }
    if (grp == 1 && ((R1 - R0) & 1) == 0) epi(R1 - 1, acc0, acc1, z0, z1);
}

// ---- weight gradient: split-K implicit GEMM -------------------------------
// part[s][tap][co][ci] = sum over the 64-pixel chunks of split s of dZ[p][co] x[p + off(tap)][ci].
// Both operands are channels-last, the reduction runs over pixels, so tiles are
// transposed on the way into LDS: each thread loads 8 channels of two adjacent
// pixels (two 16-byte loads per operand) and writes 8 packed pixel pairs
// ([channel][pixel] layout, 32-bit stores).  The next chunk's global loads are
// in flight while the matrix cores work on the current one.
constexpr int LDSW = 72;  // LDS row pitch (bf16) of the 64-pixel wgrad tiles: 64 + 8 pad, 16-byte rows

__device__ __forceinline__ uint32_t pack_bf16x2(bf16 lo, bf16 hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

__global__ __launch_bounds__(256) void k_wgrad(const bf16* __restrict__ dZ, const bf16* __restrict__ X,
                                               float* __restrict__ part, int H, int W, int P, int Ci, int Co) {
    // one workgroup: the three taps dx = -1, 0, +1 of one dy share the
    // transposed dZ tile (A), each with its own shifted input tile (B)
    __shared__ __attribute__((aligned(16))) bf16 As[64 * LDSW];
    __shared__ __attribute__((aligned(16))) bf16 Bs[3][64 * LDSW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x << 6, n0 = blockIdx.y << 6;
    const int dy = (int)(blockIdx.z % 3) - 1, s = blockIdx.z / 3;
    const int chunks = P >> 6;
    const int c_begin = (int)((long long)s * chunks / kSplit), c_end = (int)((long long)(s + 1) * chunks / kSplit);
    const int pp = tid >> 3, cg = tid & 7;  // pixel pair (0..31), 8-channel group (0..7)
    const int wr = (wave >> 1) << 5, wc = (wave & 1) << 5;
    const bool bcol = n0 + 8 * cg < Ci;
    floatx4 acc[3][2][2];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[t][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint4 va[2], vb[3][2];
    auto load = [&](int c) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const long long p = ((long long)c << 6) + 2 * pp + q;
            va[q] = *reinterpret_cast<const uint4*>(dZ + p * Co + m0 + 8 * cg);
            const int img_row = (int)(p / W), xi = (int)(p % W), yi = img_row % H;
            const int yy = yi + dy;
            const bool rowin = bcol && yy >= 0 && yy < H;
            const bf16* xrow = X + (long long)(img_row + dy) * W * Ci + n0 + 8 * cg;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int xx = xi + t - 1;
                vb[t][q] = make_uint4(0u, 0u, 0u, 0u);
                if (rowin && xx >= 0 && xx < W) vb[t][q] = *reinterpret_cast<const uint4*>(xrow + (long long)xx * Ci);
            }
        }
    };
    if (c_begin < c_end) load(c_begin);
    for (int c = c_begin; c < c_end; ++c) {
        // row 8 cg + e, pixel pair pp: its 8-pixel group pp / 4 is XOR-swizzled
        // with the row's cg (rows 8 apart would otherwise share LDS banks)
        const int col = ((((pp >> 2) ^ cg) & 7) << 3) | ((pp & 3) << 1);
        {
            const bf16* a0 = reinterpret_cast<const bf16*>(&va[0]);
            const bf16* a1 = reinterpret_cast<const bf16*>(&va[1]);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint32_t*>(&As[(8 * cg + e) * LDSW + col]) = pack_bf16x2(a0[e], a1[e]);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const bf16* b0 = reinterpret_cast<const bf16*>(&vb[t][0]);
            const bf16* b1 = reinterpret_cast<const bf16*>(&vb[t][1]);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint32_t*>(&Bs[t][(8 * cg + e) * LDSW + col]) = pack_bf16x2(b0[e], b1[e]);
        }
        __syncthreads();
        if (c + 1 < c_end) load(c + 1);
        const int r = lane & 15, kq = (lane >> 4) * 8;
        // the 8-pixel group (kk + kq) / 8 of row R sits at group ((kk + kq) / 8) ^ ((R / 8) & 7)
        auto at = [&](const bf16* base, int R, int k) -> bf16x8 {
            return *reinterpret_cast<const bf16x8*>(&base[R * LDSW + ((((k >> 3) ^ (R >> 3)) & 7) << 3)]);
        };
#pragma unroll
        for (int kk = 0; kk < 64; kk += 32) {
            const bf16x8 x0 = at(As, wr + r, kk + kq);
            const bf16x8 x1 = at(As, wr + 16 + r, kk + kq);
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const bf16x8 y0 = at(Bs[t], wc + r, kk + kq);
                const bf16x8 y1 = at(Bs[t], wc + 16 + r, kk + kq);
                acc[t][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y0, acc[t][0][0], 0, 0, 0);
                acc[t][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y1, acc[t][0][1], 0, 0, 0);
                acc[t][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y0, acc[t][1][0], 0, 0, 0);
                acc[t][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y1, acc[t][1][1], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int tap = 3 * (dy + 1) + t;
        float* dst = part + ((long long)s * 9 + tap) * Co * Ci;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = m0 + wr + 16 * i + 4 * (lane >> 4) + e;
                    const int ci = n0 + wc + 16 * j + (lane & 15);
                    if (ci < Ci) dst[(long long)co * Ci + ci] = acc[t][i][j][e];
                }
    }
}

// ---- weight gradient: persistent row streaming (width 128) ----------------
// part[s][tap][co][ci] for the 64 x CI block (co c0.., ci i0..) = the sum over the
// image rows of split s of dZ[p][co] x[p + off(tap)][ci]; all nine taps at once.
// A workgroup streams its run of whole rows through LDS rings (dZ rows in three
// slots, input rows with their halo pixels in five), two rows ahead, one barrier
// per row.  One wavefront only moves the rows in (LDS DMA) and eight compute:
// the computing wavefronts never have DMA of their own in flight, so their LDS
// reads are plain loads that the compiler schedules against the MFMAs (it
// waits for all DMA in flight before any LDS read of a wavefront that issued
// some).  The reduction runs over pixels, and the channels-last rows become
// MFMA operands with pixels along K through gfx950's transposing LDS read
// (ds_read_b64_tr_b16: lane 4a + b of each 16-lane group receives element b of
// the 8-byte chunks addressed by lanes a, a + 4, a + 8, a + 12).  Lane
// L = 16 G + a + 4 t addresses the 4 channels 16 (G & 1) + 4 a.. of pixel
// 8 (G >> 1) + t, so lane l receives channel l & 31 of pixels 8 (l >> 5) + 0..3
// (+ 4..7 with a second read at pixel + 4): the operand layout of the 32x32x16
// MFMA (row l & 31, k = 8 (l >> 5) + j).  The dx taps read the same input row at
// pixel offsets 0, 1, 2 of the halo row.
// Computing wavefront w: quadrant q = w & 3, taps 0-4 (w < 4) or 5-8.  CI = 64:
// quadrant q is co 32 (q & 1).. x ci 32 (q >> 1)..  CI = 32 (the first layer):
// co 32 (q & 1).. x all 32 ci over every other 16-pixel K step (from 16 (q >> 1)),
// written as separate partials (split index 2 s + (q >> 1)).
// The ci-block-0 workgroups also sum dZ over their rows, from the dZ operands
// of the taps-0-4 wavefronts: bpart[s][co].
constexpr int kWgWaves = 9;   // 8 computing wavefronts and the one that moves rows in

template <int CI>
__global__ __launch_bounds__(64 * kWgWaves, 1) void k_wgrad_rows(const bf16* __restrict__ dZ, const bf16* __restrict__ X,
        float* __restrict__ part, float* __restrict__ bpart, int H, int rows_total, int rows_per_wg, int Ci, int Co) {
    static_assert(CI == 32 || CI == 64, "input blocks of 32 or 64 channels");
    constexpr int KH = 64 / CI;                 // K-step phases of one (co, ci) quadrant
    constexpr int SX = CI / 8;                  // 16-byte segments per input pixel
    constexpr int kZSlot = kRowW * 64;          // dZ row: 128 px x 64 co
    constexpr int kXSlot = kRowPx * CI;         // input row: 130 px (halo) x CI
    constexpr int kZSlots = 3, kXSlots = 5;     // rows R .. R + 2 of dZ, R - 1 .. R + 3 of the input
    constexpr int kZLoads = kZSlot / (64 * 8);  // DMA instructions per dZ row (64 lanes x 16 bytes each)
    constexpr int kXPieces = kRowPx * SX;
    constexpr int kXLoads = (kXPieces + 63) / 64;
    constexpr int kXTail = kXPieces - 64 * (kXLoads - 1);   // lanes of the last input-row instruction
    constexpr int kRowLoads = kZLoads + kXLoads;            // per row, all issued by the moving wavefront
    static_assert(kRowLoads < 64, "wait_vm counts below 64");
    __shared__ __attribute__((aligned(16))) bf16 Zr[kZSlots * kZSlot];
    __shared__ __attribute__((aligned(16))) bf16 Xr[kXSlots * kXSlot];
    __shared__ float bred[4][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s = blockIdx.x, c0 = blockIdx.y << 6, i0 = blockIdx.z * CI;
    const int R0 = s * rows_per_wg, R1 = min(R0 + rows_per_wg, rows_total);
    const bool bias = blockIdx.z == 0;
    auto zslot = [&](int Rg) { return Zr + (size_t)((Rg + kZSlots) % kZSlots) * kZSlot; };
    auto xslot = [&](int Rg) { return Xr + (size_t)((Rg + kXSlots) % kXSlots) * kXSlot; };   // Rg >= -1
    if (wave == 8) {
        // dZ row Rg: piece q = px 8 + ps holds the 8 channels (ps ^ swz<64>(px)); input row Rg:
        // piece q = px SX + ps, halo pixel px (image column px - 1)
        auto load_z = [&](int Rg) {
            bf16* slot = zslot(Rg);
            const bool rin = Rg >= 0 && Rg < rows_total;
#pragma unroll
            for (int r = 0; r < kZLoads; ++r) {
                const int q = r * 64 + lane;
                const int px = q >> 3, ls = (q & 7) ^ swz<64>(px);
                const void* src = rin ? (const void*)(dZ + ((long long)Rg * kRowW + px) * Co + c0 + 8 * ls) : (const void*)&kZero16;
                __builtin_amdgcn_global_load_lds(src, (lds_void*)(slot + (size_t)r * 64 * 8), 16, 0, 0);
            }
        };
        auto load_x = [&](int Rg) {
            bf16* slot = xslot(Rg);
            const bool rin = Rg >= 0 && Rg < rows_total;
#pragma unroll
            for (int r = 0; r < kXLoads; ++r) {
                const bool on = r < kXLoads - 1 || lane < kXTail;
                const int q = r * 64 + lane;
                const int px = q / SX, ls = (q % SX) ^ swz<CI>(px);
                const int x = px - 1;
                const bool in = rin && on && x >= 0 && x < kRowW;
                const void* src = in ? (const void*)(X + ((long long)Rg * kRowW + x) * Ci + i0 + 8 * ls) : (const void*)&kZero16;
                if (on) __builtin_amdgcn_global_load_lds(src, (lds_void*)(slot + (size_t)r * 64 * 8), 16, 0, 0);
            }
        };
        if (R0 < R1) {
            load_x(R0 - 1);
            load_x(R0);
            load_x(R0 + 1);
            load_z(R0);
            if (R0 + 1 < R1) {
                load_x(R0 + 2);
                load_z(R0 + 1);
            }
        }
        for (int R = R0; R < R1; ++R) {
            // rows R + 1 (input) and R (dZ) have landed; the loads of rows R + 2 and R + 1,
            // issued one row earlier (when R + 1 < R1), may still be in flight
            if (R + 1 < R1) wait_vm<kRowLoads>(); else wait_vm<0>();
            __builtin_amdgcn_s_barrier();
            if (R + 2 < R1) {   // into the slots of rows R - 2 (input) and R - 1 (dZ), which no wave reads any more
                load_x(R + 3);
                load_z(R + 2);
            }
        }
        __syncthreads();    // pairs with the computing wavefronts' barrier before the bias sums
        return;
    }
    const int q = wave & 3, g = wave >> 2;
    const int cw = 32 * (q & 1);
    const int iw = KH == 1 ? 32 * (q >> 1) : 0;
    const int kh = KH == 1 ? 0 : q >> 1;
    const bool bsums = bias && g == 0 && (KH == 2 || q < 2);
    constexpr int kSteps = kRowW / (16 * KH);   // this wavefront's 16-pixel K steps per row
    floatx16 acc[5];
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.f;
    float bsum = 0.f;
    const int G = lane >> 4, ta = lane & 3, tt = (lane >> 2) & 3;
    const int tpx = 8 * (G >> 1) + tt;        // pixel of the addressed chunk within a 16-pixel K step
    const int tch = 16 * (G & 1) + 4 * ta;    // its first channel within the wave's 32
    typedef __attribute__((address_space(3))) short lshort;
    typedef __attribute__((address_space(3))) v4s lv4s;
    // the 8-byte chunk of channels ch.. ch + 3 (ch a multiple of 4) of pixel px, transposed
    auto ztr = [&](const bf16* base, int px, int ch) {
        const bf16* p = base + (size_t)px * 64 + 8 * ((ch >> 3) ^ swz<64>(px)) + (ch & 4);
        return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lv4s*)(lshort*)p);
    };
    auto xtr = [&](const bf16* base, int px, int ch) {
        const bf16* p = base + (size_t)px * CI + 8 * ((ch >> 3) ^ swz<CI>(px)) + (ch & 4);
        return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lv4s*)(lshort*)p);
    };
    // two 4-element reads side by side as one 8-element operand (a bit cast of the whole
    // vector: this compiler reads element 0 for a bit cast of a vector-element lvalue)
    auto pack = [](v4s lo, v4s hi) {
        const v8s c = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_bit_cast(bf16x8, c);
    };
    auto xop = [&](const bf16* xr, int px, int dxi) { return pack(xtr(xr, px + dxi, iw + tch), xtr(xr, px + dxi + 4, iw + tch)); };
    for (int R = R0; R < R1; ++R) {
        const int y = R % H;
        __builtin_amdgcn_s_barrier();   // the moving wavefront has seen rows R + 1 (input) and R (dZ) land
        const bf16* zrow = zslot(R);
        const bf16* xr0 = xslot(R - 1);
        const bf16* xr1 = xslot(R);
        const bf16* xr2 = xslot(R + 1);
        const bool up = y > 0, dn = y + 1 < H;   // outside the image the taps read zeros
        if (g == 0) {
#pragma unroll 2
            for (int i = 0; i < kSteps; ++i) {
                const int px = 16 * (kh + KH * i) + tpx;
                const bf16x8 A = pack(ztr(zrow, px, cw + tch), ztr(zrow, px + 4, cw + tch));
                if (bsums) {   // dZ of channel cw + (l & 31) at pixels k0 + 8 (l >> 5) + 0..7
#pragma unroll
                    for (int j = 0; j < 8; ++j) bsum += float(A[j]);
                }
                if (up) {
                    acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr0, px, 0), acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr0, px, 1), acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr0, px, 2), acc[2], 0, 0, 0);
                }
                acc[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr1, px, 0), acc[3], 0, 0, 0);
                acc[4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr1, px, 1), acc[4], 0, 0, 0);
            }
        } else {
#pragma unroll 2
            for (int i = 0; i < kSteps; ++i) {
                const int px = 16 * (kh + KH * i) + tpx;
                const bf16x8 A = pack(ztr(zrow, px, cw + tch), ztr(zrow, px + 4, cw + tch));
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr1, px, 2), acc[0], 0, 0, 0);
                if (dn) {
                    acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr2, px, 0), acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr2, px, 1), acc[2], 0, 0, 0);
                    acc[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, xop(xr2, px, 2), acc[3], 0, 0, 0);
                }
            }
        }
    }
    // this wavefront's partial sums; acc element e of lane l is D[8 (e >> 2) + 4 (l >> 5) + (e & 3)][l & 31]
    const int t0 = g == 0 ? 0 : 5, nt = g == 0 ? 5 : 4;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        if (t < nt) {
            float* dst = part + ((((long long)s * KH + kh) * 9 + t0 + t) * Co + c0 + cw) * Ci + i0 + iw;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int m = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                dst[(long long)m * Ci + (lane & 31)] = acc[t][e];
            }
        }
    }
    if (g == 0) bred[q][lane] = bsum;
    __syncthreads();
    if (bias && tid < 64) {
        // channel co: quadrant co >> 5 (and + 2: the other K phase, CI = 32), lanes co & 31 (pixels
        // 0..7 of each K step) and + 32 (8..15); fixed order
        const int h = tid >> 5, l = tid & 31;
        float v = bred[h][l] + bred[h][l + 32];
        if (KH == 2) v += bred[h + 2][l] + bred[h + 2][l + 32];
        bpart[(long long)s * kMaxC + c0 + tid] = v;
    }
}

// dW[co][tap][ci] (packed) = sum_s part[s][tap][co][ci], fixed order
// dW = sum over the ns partials, in a fixed order: a workgroup covers 64
// outputs, its wave g sums partials [g ns / 4, (g + 1) ns / 4) of them, then
// the four wave sums are added in wave order
// dW[co][tap][ci] = the fixed-order sum of the ns split partials (eight runs, one per wavefront,
// added in order); the grid's last workgroup adds up the bias partials instead: db[co] = the sum
// of bpart[0 .. nb-1][co], in four runs added in order
constexpr int kRedWaves = 8;
__global__ __launch_bounds__(64 * kRedWaves) void k_wgrad_reduce(const float* __restrict__ part, int ns, int Ci, int Co,
                                                                 float* __restrict__ dW, const float* __restrict__ bpart,
                                                                 int nb, float* __restrict__ db) {
    __shared__ float red[kRedWaves - 1][kMaxC];
    if (blockIdx.x == gridDim.x - 1) {
        constexpr int G = 64 * kRedWaves / kMaxC;   // runs of the bias partials
        const int co = (int)threadIdx.x % kMaxC, g = (int)threadIdx.x / kMaxC;
        const int b0 = g * nb / G, b1 = (g + 1) * nb / G;
        float t = 0.f;
        if (co < Co) {
#pragma unroll 8
            for (int q = b0; q < b1; ++q) t += bpart[(long long)q * kMaxC + co];
        }
        if (g > 0) red[g - 1][co] = t;
        __syncthreads();
        if (g == 0 && co < Co) {
#pragma unroll
            for (int k = 0; k < G - 1; ++k) t += red[k][co];
            db[co] = t;
        }
        return;
    }
    const int j = threadIdx.x & 63, g = threadIdx.x >> 6;
    const long long k = ((long long)blockIdx.x << 6) + j;
    const long long n = 9ll * Co * Ci;
    const bool live = k < n;
    float s = 0.f;
    if (live) {
        const int q0 = g * ns / kRedWaves, q1 = (g + 1) * ns / kRedWaves;
        const float* src = part + k;
#pragma unroll 8
        for (int q = q0; q < q1; ++q) s += src[(long long)q * n];
    }
    if (g > 0) red[g - 1][j] = s;
    __syncthreads();
    if (g == 0 && live) {
#pragma unroll
        for (int w = 0; w < kRedWaves - 1; ++w) s += red[w][j];
        const int tap = (int)(k / ((long long)Co * Ci));
        const long long rem = k % ((long long)Co * Ci);
        const int co = (int)(rem / Ci), ci = (int)(rem % Ci);
        dW[((long long)co * 9 + tap) * Ci + ci] = s;
    }
}

// bias gradient, two passes: part[block][co] over contiguous pixel ranges
// (16-byte loads of 8 channels, fixed-order reduction through LDS), then a
// fixed-order sum over the blocks
__global__ __launch_bounds__(256) void k_bgrad_part(const bf16* __restrict__ dZ, long long P, int Co,
                                                    float* __restrict__ part) {
    const int groups = Co >> 3;  // 8 channels per thread; Co is 64 or 128
    const int g = (int)threadIdx.x % groups, lp = (int)threadIdx.x / groups, per = 256 / groups;
    const long long b0 = P * blockIdx.x / gridDim.x, b1 = P * (blockIdx.x + 1) / gridDim.x;
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
    for (long long p = b0 + lp; p < b1; p += per) {
        const uint4 v = *reinterpret_cast<const uint4*>(dZ + p * Co + 8 * g);
        const bf16* e = reinterpret_cast<const bf16*>(&v);
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += float(e[k]);
    }
    __shared__ float red[256][9];
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    if ((int)threadIdx.x < Co) {
        const int gg = (int)threadIdx.x >> 3, k = (int)threadIdx.x & 7;
        float t = 0.f;
        for (int l = 0; l < per; ++l) t += red[l * groups + gg][k];
        part[(long long)blockIdx.x * kMaxC + threadIdx.x] = t;
    }
}

// MSE over the SG_OUTPUTS real channels: dZ = 2 (z - t) / count (bf16, zero on
// padded channels); per-block partial sums of (z - t)^2 in FP64
static_assert(SG_OUTPUTS <= 8, "k_mse keeps the real output channels in the first 8-channel group");
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Z, const float* __restrict__ fields,
                                             const int* __restrict__ idx, int nb, int H, int W, int Co,
                                             bf16* __restrict__ dZ, double* __restrict__ part) {
    __shared__ double red[256];
    const long long P = (long long)nb * H * W;
    const double inv = 2.0 / (double)(P * SG_OUTPUTS);
    const long long HW = (long long)H * W;
    const int groups = Co >> 3;  // a thread writes 8 channels of one pixel (one 16-byte store)
    double acc = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < P * groups;
         e += (long long)gridDim.x * blockDim.x) {
        const long long p = e / groups;
        const int cg = (int)(e - p * groups);
        uint4 pk = make_uint4(0u, 0u, 0u, 0u);
        if (cg == 0) {  // the real channels 0 .. SG_OUTPUTS - 1
            bf16* g = reinterpret_cast<bf16*>(&pk);
            const int b = (int)(p / HW);
            const long long pix = p - b * HW;
#pragma unroll
            for (int c = 0; c < SG_OUTPUTS; ++c) {
                const float d = Z[p * Co + c] - fields[((long long)idx[b] * SG_OUTPUTS + c) * HW + pix];
                acc += (double)d * d;
                g[c] = bf16((float)(inv * d));
            }
        }
        *reinterpret_cast<uint4*>(dZ + p * Co + 8 * cg) = pk;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
// the batch loss; with acc, also acc += the loss (as rounded to FP32), a running sum over steps.
// One workgroup of 64 threads: thread t sums the t-th run of nb / 64 partials in order, thread 0
// adds the 64 run sums in order (fixed order, deterministic)
__global__ __launch_bounds__(64) void k_mse_final(const double* __restrict__ part, int nb, double count,
                                                  float* __restrict__ loss, double* __restrict__ acc) {
    __shared__ double red[64];
    const int t = (int)threadIdx.x;
    const int b0 = t * nb / 64, b1 = (t + 1) * nb / 64;
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += part[b];
    red[t] = s;
    __syncthreads();
    if (t != 0) return;
    s = 0.0;
    for (int k = 0; k < 64; ++k) s += red[k];
    const float l = (float)(s / count);
    *loss = l;
    if (acc) *acc += (double)l;
}

// where each layer's weights sit in the packed vector and their two BF16 copies
struct PackMap {
    long long woff[kLayers];
    int ci[kLayers], co[kLayers];
    bf16* wk[kLayers];
    bf16* wt[kLayers];
};

// weight k of the packed vector (value v) into the BF16 copies of its layer: the forward
// GEMM's [co][tap][ci] and the data-gradient GEMM's [ci][8 - tap][co] (transposed and
// flipped); biases have no copy
__device__ __forceinline__ void pack_one(const PackMap& pm, long long k, float v) {
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
        const long long r = k - pm.woff[l];
        const int Ci = pm.ci[l], Co = pm.co[l];
        if (r >= 0 && r < 9ll * Co * Ci) {
            const int co = (int)(r / (9ll * Ci));
            const long long rem = r % (9ll * Ci);
            const int tap = (int)(rem / Ci), ci = (int)(rem % Ci);
            const bf16 b = bf16(v);
            pm.wk[l][r] = b;
            pm.wt[l][((long long)ci * 9 + (8 - tap)) * Co + co] = b;
        }
    }
}

// Adam (bias-corrected) on the FP32 master weights, then their BF16 copies
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2, PackMap pm) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    w[k] = wk;
    pack_one(pm, k, wk);
}

// the BF16 copies of every layer's weights (after weights are set)
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ w, long long n, PackMap pm) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) pack_one(pm, k, w[k]);
}

// [p][Co] (first SG_OUTPUTS channels) -> out[b][c][y][x]
__global__ __launch_bounds__(256) void k_unpack_out(const float* __restrict__ Z, int nb, int H, int W, int Co,
                                                    float* __restrict__ out) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long P = (long long)nb * H * W;
    if (p >= P) return;
    const int b = (int)(p / ((long long)H * W));
    const long long pix = p % ((long long)H * W);
#pragma unroll
    for (int c = 0; c < SG_OUTPUTS; ++c) out[((long long)b * SG_OUTPUTS + c) * H * W + pix] = Z[p * Co + c];
}

// separable [1 2 1]/4 filter per plane, edge values replicated; it removes
// the grid-scale (Nyquist) content of a prediction exactly
__global__ __launch_bounds__(256) void k_smooth(const float* __restrict__ in, float* __restrict__ out,
                                                long long planes, int H, int W) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= planes * H * W) return;
    const long long pl = k / ((long long)H * W);
    const int rem = (int)(k % ((long long)H * W));
    const int y = rem / W, x = rem % W;
    const float* q = in + pl * H * W;
    const float wt[3] = {0.25f, 0.5f, 0.25f};
    float s = 0.f;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = min(max(y + dy, 0), H - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = min(max(x + dx, 0), W - 1);
            s += wt[dy + 1] * wt[dx + 1] * q[yy * W + xx];
        }
    }
    out[k] = s;
}

// Removes the lattice-staggered parts of a velocity field, one workgroup per
// field set [u, v, T, C]: u -= <u (-1)^x> (-1)^x and v -= <v (-1)^y> (-1)^y,
// means over the whole plane, accumulated in FP64 in a fixed order.
__global__ __launch_bounds__(256) void k_destagger(float* __restrict__ f, int H, int W) {
    float* u = f + (long long)blockIdx.x * 4 * H * W;
    float* v = u + (long long)H * W;
    const int HW = H * W;
    double su = 0.0, sv = 0.0;
    for (int k = threadIdx.x; k < HW; k += blockDim.x) {
        const int y = k / W, x = k % W;
        su += (x & 1) ? -double(u[k]) : double(u[k]);
        sv += (y & 1) ? -double(v[k]) : double(v[k]);
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = su;
    red[1][threadIdx.x] = sv;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    const float cu = float(red[0][0] / HW), cv = float(red[1][0] / HW);
    for (int k = threadIdx.x; k < HW; k += blockDim.x) {
        const int y = k / W, x = k % W;
        u[k] -= (x & 1) ? -cu : cu;
        v[k] -= (y & 1) ? -cv : cv;
    }
}

}  // namespace sgk

// ============================================================================
// host side
// ============================================================================
using namespace sgk;

namespace {
thread_local std::string g_sgerr;
lb_status sgfail(lb_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_sgerr = buf;
    return st;
}
#define SGCHK(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return sgfail(LB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

size_t rup(size_t v) { return (v + 255) / 256 * 256; }

struct Plan {
    size_t P;
    long long nw[kLayers], woff[kLayers], boff[kLayers], npacked;
    size_t w_off, m_off, v_off, g_off, wk_off[kLayers], wt_off[kLayers], x0_off, z_off[kLayers], y_off[kLayers],
        dz_off[2], part_off, bpart_off, lpart_off, loss_off, lsum_off, idx_off, total;
};

Plan make_plan(const sg_config& c) {
    Plan pl{};
    pl.P = (size_t)c.batch * c.height * c.width;
    long long off = 0;
    for (int l = 0; l < kLayers; ++l) {
        pl.nw[l] = 9ll * kCoutPad[l] * kCinPad[l];
        pl.woff[l] = off;
        off += pl.nw[l];
        pl.boff[l] = off;
        off += kCoutPad[l];
    }
    pl.npacked = off;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = rup(o + bytes);
        return r;
    };
    pl.w_off = take(4 * pl.npacked);
    pl.m_off = take(4 * pl.npacked);
    pl.v_off = take(4 * pl.npacked);
    pl.g_off = take(4 * pl.npacked);
    for (int l = 0; l < kLayers; ++l) {
        pl.wk_off[l] = take(2 * pl.nw[l]);
        pl.wt_off[l] = take(2 * pl.nw[l]);
    }
    pl.x0_off = take(2 * pl.P * kCinPad[0]);
    for (int l = 0; l < kLayers; ++l) {
        pl.z_off[l] = take(4 * pl.P * kCoutPad[l]);
        pl.y_off[l] = take(2 * pl.P * kCoutPad[l]);
    }
    pl.dz_off[0] = take(2 * pl.P * kMaxC);
    pl.dz_off[1] = take(2 * pl.P * kMaxC);
    pl.part_off = take(4ull * kSplit * 9 * kMaxC * kMaxC);
    pl.bpart_off = take(4ull * kRed * kMaxC);
    pl.lpart_off = take(8ull * kMseBlocks);
    pl.loss_off = take(8);
    pl.lsum_off = take(8);
    pl.idx_off = take(4ull * c.batch * kIdxSteps);
    pl.total = o;
    return pl;
}
}  // namespace

struct sg_handle {
    sg_config c;
    Plan pl;
    char* ws;
    hipStream_t s;
    long long t;  // Adam step counter
    int nb_last;  // samples in the last forward pass
    bool z_valid; // the last forward pass stored every layer's pre-activation
};

namespace {
template <class T>
T* ptr(sg_handle* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

PackMap pack_map(sg_handle* h) {
    PackMap pm{};
    for (int l = 0; l < kLayers; ++l) {
        pm.woff[l] = h->pl.woff[l];
        pm.ci[l] = kCinPad[l];
        pm.co[l] = kCoutPad[l];
        pm.wk[l] = ptr<bf16>(h, h->pl.wk_off[l]);
        pm.wt[l] = ptr<bf16>(h, h->pl.wt_off[l]);
    }
    return pm;
}

lb_status pack_weights(sg_handle* h) {
    const long long n = h->pl.npacked;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->s, ptr<float>(h, h->pl.w_off), n,
                       pack_map(h));
    SGCHK(hipGetLastError());
    return LB_OK;
}

// one convolution of layer l over P pixels: mode 0 forward (x -> z, y), mode 1
// data gradient (g = dL/dz_l, zprev = z_{l-1} -> y = dL/dz_{l-1})
lb_status launch_conv(sg_handle* h, int l, int mode, long long P, const bf16* x, const float* zprev, float* z,
                      bf16* y) {
    const int H = h->c.height, W = h->c.width;
    const int Ci = mode == 0 ? kCinPad[l] : kCoutPad[l];   // K channels (per tap)
    const int Co = mode == 0 ? kCoutPad[l] : kCinPad[l];   // output channels
    const bf16* wk = ptr<bf16>(h, mode == 0 ? h->pl.wk_off[l] : h->pl.wt_off[l]);
    const float* bias = mode == 0 ? ptr<float>(h, h->pl.w_off) + h->pl.boff[l] : nullptr;
    const int act = mode == 0 && l + 1 < kLayers ? 1 : 0;
    if (!y && (mode == 1 || !z)) return sgfail(LB_EINVAL, "launch_conv: no output");
    const int rows_total = (int)(P / W);
    // forward with 128 K channels: two K launches of 64 channels through the FP32 partial buffer
    // (free outside the weight gradient) when the partial sums fit.  Not for the data gradient:
    // against its tile kernel's 86-89 us the two launches took 102 us with the pre-activations
    // held beside the partial sums (spilled) and 94-98 us with both read in the epilogue
    // (where the forward gains 90 -> 75 us)
    const bool ksplit = mode == 0 && W == kRowW && Ci == 128 && Co == 64 &&
                        4ull * (size_t)P * Co <= 4ull * kSplit * 9 * kMaxC * kMaxC;
    if (W == kRowW && (Ci == 32 || Ci == 64 || ksplit)) {
        const int nblk = Co / 64;
        const int nwg = std::max(1, std::min(rows_total, 256 / nblk));   // one workgroup per CU
        const int rpw = (rows_total + nwg - 1) / nwg;
        const dim3 grid((unsigned)nwg, (unsigned)nblk);
        float* zpart = ptr<float>(h, h->pl.part_off);
        auto go = [&](auto kern, int koff) {
            hipLaunchKernelGGL(kern, grid, dim3(512), 0, h->s, x, wk, bias, zprev, z, y, zpart, H, rows_total, rpw, Co, act,
                               Ci, koff);
        };
        if (ksplit) {
            go(k_conv_rows<0, 64, false, false, 1>, 0);
            if (z && y) go(k_conv_rows<0, 64, true, true, 2>, 64);
            else if (y) go(k_conv_rows<0, 64, false, true, 2>, 64);
            else go(k_conv_rows<0, 64, true, false, 2>, 64);
        } else {
            // z and y, y only (prediction) or z only (the output layer)
            auto fwd = [&](auto ck) {
                constexpr int CK = decltype(ck)::value;
                if (z && y) go(k_conv_rows<0, CK, true, true, 0>, 0);
                else if (y) go(k_conv_rows<0, CK, false, true, 0>, 0);
                else go(k_conv_rows<0, CK, true, false, 0>, 0);
            };
            auto bwd = [&](auto ck) {
                constexpr int CK = decltype(ck)::value;
                go(k_conv_rows<1, CK, false, true, 0>, 0);
            };
            if (mode == 0) {
                if (Ci == 32) fwd(std::integral_constant<int, 32>{});
                else fwd(std::integral_constant<int, 64>{});
            } else {
                if (Ci == 32) bwd(std::integral_constant<int, 32>{});
                else bwd(std::integral_constant<int, 64>{});
            }
        }
    } else if (W % 128 == 0) {
        const dim3 grid((unsigned)(P / 128), (unsigned)(Co / 64));
        if (mode == 0)
            hipLaunchKernelGGL(k_conv128<0>, grid, dim3(256), 0, h->s, x, wk, bias, zprev, z, y, H, W, Ci, Co, act);
        else
            hipLaunchKernelGGL(k_conv128<1>, grid, dim3(256), 0, h->s, x, wk, bias, zprev, z, y, H, W, Ci, Co, act);
    } else {
        const dim3 grid((unsigned)(P / 64), (unsigned)(Co / 64));
        if (mode == 0)
            hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, h->s, x, wk, bias, zprev, z, y, H, W, Ci, Co, act);
        else
            hipLaunchKernelGGL(k_conv<1>, grid, dim3(256), 0, h->s, x, wk, bias, zprev, z, y, H, W, Ci, Co, act);
    }
    SGCHK(hipGetLastError());
    return LB_OK;
}

// weight and bias gradients of layer l over P pixels (split-K partials in the
// workspace, then fixed-order reductions)
lb_status launch_wgrad(sg_handle* h, int l, long long P, const bf16* dz, const bf16* xin, float* dw, float* db) {
    const int H = h->c.height, W = h->c.width;
    const int Ci = kCinPad[l], Co = kCoutPad[l];
    const long long n = 9ll * Co * Ci;
    float* part = ptr<float>(h, h->pl.part_off);
    float* bpart = ptr<float>(h, h->pl.bpart_off);
    if (W == kRowW && (Ci == 32 || Ci % 64 == 0)) {
        // one workgroup per CU over the (co, ci) blocks, each with a run of whole rows
        const int rows_total = (int)(P / W);
        const int cib = Ci == 32 ? 1 : Ci / 64, blocks = (Co / 64) * cib;
        int nwg = std::max(1, std::min(rows_total, 256 / blocks));
        const int rpw = (rows_total + nwg - 1) / nwg;
        nwg = (rows_total + rpw - 1) / rpw;   // no workgroup without rows
        const int ns = Ci == 32 ? 2 * nwg : nwg;
        if ((long long)ns * n > (long long)kSplit * 9 * kMaxC * kMaxC || nwg > kRed) return LB_ENOMEM;
        const dim3 grid((unsigned)nwg, (unsigned)(Co / 64), (unsigned)cib);
        if (Ci == 32)
            hipLaunchKernelGGL(k_wgrad_rows<32>, grid, dim3(64 * kWgWaves), 0, h->s, dz, xin, part, bpart, H, rows_total, rpw, Ci, Co);
        else
            hipLaunchKernelGGL(k_wgrad_rows<64>, grid, dim3(64 * kWgWaves), 0, h->s, dz, xin, part, bpart, H, rows_total, rpw, Ci, Co);
        SGCHK(hipGetLastError());
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 63) / 64 + 1)), dim3(64 * kRedWaves), 0, h->s, part, ns, Ci, Co, dw,
                           bpart, nwg, db);
        SGCHK(hipGetLastError());
        return LB_OK;
    }
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)(Co / 64), (unsigned)((Ci + 63) / 64), 3u * kSplit), dim3(256), 0, h->s,
                       dz, xin, part, H, W, (int)P, Ci, Co);
    SGCHK(hipGetLastError());
    hipLaunchKernelGGL(k_bgrad_part, dim3(kRed), dim3(256), 0, h->s, dz, P, Co, bpart);
    SGCHK(hipGetLastError());
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 63) / 64 + 1)), dim3(64 * kRedWaves), 0, h->s, part, kSplit, Ci, Co, dw,
                       bpart, kRed, db);
    SGCHK(hipGetLastError());
    return LB_OK;
}

// forward pass of nb samples listed in the device index array; keep_z = false
// (prediction) skips the FP32 pre-activation store of the hidden layers, which
// only the backward pass reads
lb_status forward(sg_handle* h, const float* d_params, int nb, bool keep_z = true, const int* idx = nullptr) {
    if (!idx) idx = ptr<int>(h, h->pl.idx_off);
    const int H = h->c.height, W = h->c.width;
    const long long P = (long long)nb * H * W;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, h->s, d_params,
                       idx, nb, H, W, ptr<bf16>(h, h->pl.x0_off));
    SGCHK(hipGetLastError());
    const bf16* x = ptr<bf16>(h, h->pl.x0_off);
    for (int l = 0; l < kLayers; ++l) {
        float* z = keep_z || l + 1 == kLayers ? ptr<float>(h, h->pl.z_off[l]) : nullptr;
        // the output layer's BF16 copy feeds nothing (the loss and the prediction read z)
        bf16* y = l + 1 < kLayers ? ptr<bf16>(h, h->pl.y_off[l]) : nullptr;
        lb_status st = launch_conv(h, l, 0, P, x, nullptr, z, y);
        if (st != LB_OK) return st;
        x = y;
    }
    h->nb_last = nb;
    h->z_valid = keep_z;
    return LB_OK;
}

lb_status set_indices(sg_handle* h, const int32_t* host_idx, int nb) {
    SGCHK(hipMemcpyAsync(ptr<int>(h, h->pl.idx_off), host_idx, 4ull * nb, hipMemcpyHostToDevice, h->s));
    return LB_OK;
}

// loss + gradients of every layer into the packed gradient vector
// loss_host: the batch loss, read back (synchronising); lsum: device running sum of the
// batch losses (no synchronisation)
lb_status backward(sg_handle* h, const float* d_fields, int nb, float* loss_host, const int* idx = nullptr,
                   double* lsum = nullptr) {
    if (!idx) idx = ptr<int>(h, h->pl.idx_off);
    const int H = h->c.height, W = h->c.width;
    const long long P = (long long)nb * H * W;
    const int L = kLayers - 1;
    bf16* dz = ptr<bf16>(h, h->pl.dz_off[0]);
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, h->s, ptr<float>(h, h->pl.z_off[L]), d_fields,
                       idx, nb, H, W, kCoutPad[L], dz, ptr<double>(h, h->pl.lpart_off));
    SGCHK(hipGetLastError());
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, h->s, ptr<double>(h, h->pl.lpart_off), kMseBlocks,
                       (double)(P * SG_OUTPUTS), ptr<float>(h, h->pl.loss_off), lsum);
    SGCHK(hipGetLastError());
    float* grads = ptr<float>(h, h->pl.g_off);
    for (int l = L; l >= 0; --l) {
        const bf16* xin = l == 0 ? ptr<bf16>(h, h->pl.x0_off) : ptr<bf16>(h, h->pl.y_off[l - 1]);
        lb_status st = launch_wgrad(h, l, P, dz, xin, grads + h->pl.woff[l], grads + h->pl.boff[l]);
        if (st != LB_OK) return st;
        if (l > 0) {
            bf16* dzn = ptr<bf16>(h, h->pl.dz_off[(L - l + 1) & 1]);
            st = launch_conv(h, l, 1, P, dz, ptr<float>(h, h->pl.z_off[l - 1]), nullptr, dzn);
            if (st != LB_OK) return st;
            dz = dzn;
        }
    }
    if (loss_host) {
        SGCHK(hipMemcpyAsync(loss_host, ptr<float>(h, h->pl.loss_off), 4, hipMemcpyDeviceToHost, h->s));
        SGCHK(hipStreamSynchronize(h->s));
    }
    return LB_OK;
}

lb_status adam(sg_handle* h) {
    h->t += 1;
    const float c1 = 1.f - powf(h->c.beta1, (float)h->t), c2 = 1.f - powf(h->c.beta2, (float)h->t);
    const long long n = h->pl.npacked;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->s, ptr<float>(h, h->pl.w_off),
                       ptr<float>(h, h->pl.g_off), ptr<float>(h, h->pl.m_off), ptr<float>(h, h->pl.v_off), n, h->c.lr,
                       h->c.beta1, h->c.beta2, h->c.eps, c1, c2, pack_map(h));
    SGCHK(hipGetLastError());
    return LB_OK;
}

lb_status check_idx(sg_handle* h, const int32_t* idx) {
    if (!idx) return sgfail(LB_EINVAL, "host_idx is NULL");
    for (int b = 0; b < h->c.batch; ++b)
        if (idx[b] < 0) return sgfail(LB_EINVAL, "negative sample index");
    return LB_OK;
}
}  // namespace

extern "C" {

lb_status sg_layer_info(int32_t layer, int32_t* cin, int32_t* cout, int32_t* cin_pad, int32_t* cout_pad) {
    if (layer < 0 || layer >= kLayers) return sgfail(LB_EINVAL, "layer out of range");
    if (cin) *cin = kCin[layer];
    if (cout) *cout = kCout[layer];
    if (cin_pad) *cin_pad = kCinPad[layer];
    if (cout_pad) *cout_pad = kCoutPad[layer];
    return LB_OK;
}

lb_status sg_param_count(int64_t* packed, int64_t* real) {
    long long p = 0, r = 0;
    for (int l = 0; l < kLayers; ++l) {
        p += 9ll * kCoutPad[l] * kCinPad[l] + kCoutPad[l];
        r += 9ll * kCout[l] * kCin[l] + kCout[l];
    }
    if (packed) *packed = p;
    if (real) *real = r;
    return LB_OK;
}

lb_status sg_workspace_bytes(const sg_config* cfg, size_t* bytes) {
    if (!cfg || !bytes) return sgfail(LB_EINVAL, "NULL argument");
    if (cfg->batch < 1 || cfg->height < 1 || cfg->width < 64 || cfg->width % 64 || cfg->reserved != 0)
        return sgfail(LB_EINVAL, "batch >= 1, height >= 1, width a multiple of 64 required");
    if (!(cfg->lr >= 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
        !(cfg->eps > 0.f))
        return sgfail(LB_EINVAL, "invalid Adam hyper-parameters");
    *bytes = make_plan(*cfg).total;
    return LB_OK;
}

lb_status sg_create(const sg_config* cfg, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                    sg_handle** out) {
    if (!out) return sgfail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    lb_status st = sg_workspace_bytes(cfg, &need);
    if (st != LB_OK) return st;
    if (!dev_workspace || reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return sgfail(LB_EINVAL, "workspace NULL or not 256-byte aligned");
    if (workspace_bytes < need) return sgfail(LB_ENOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
    sg_handle* h = new (std::nothrow) sg_handle();
    if (!h) return sgfail(LB_ENOMEM, "host allocation failed");
    h->c = *cfg;
    h->pl = make_plan(*cfg);
    h->ws = static_cast<char*>(dev_workspace);
    h->s = static_cast<hipStream_t>(hip_stream);
    h->t = 0;
    h->nb_last = 0;
    h->z_valid = false;
    *out = h;
    return LB_OK;
}

lb_status sg_set_weights(sg_handle* h, const float* host_packed) {
    if (!h || !host_packed) return sgfail(LB_EINVAL, "NULL argument");
    const size_t n = (size_t)h->pl.npacked;
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(host_packed[k])) return sgfail(LB_ENONFINITE, "non-finite weight");
    SGCHK(hipMemcpyAsync(ptr<float>(h, h->pl.w_off), host_packed, 4 * n, hipMemcpyHostToDevice, h->s));
    SGCHK(hipMemsetAsync(ptr<float>(h, h->pl.m_off), 0, 4 * n, h->s));
    SGCHK(hipMemsetAsync(ptr<float>(h, h->pl.v_off), 0, 4 * n, h->s));
    h->t = 0;
    lb_status st = pack_weights(h);
    if (st != LB_OK) return st;
    SGCHK(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status sg_get_weights(sg_handle* h, float* host_packed) {
    if (!h || !host_packed) return sgfail(LB_EINVAL, "NULL argument");
    SGCHK(hipMemcpyAsync(host_packed, ptr<float>(h, h->pl.w_off), 4ull * h->pl.npacked, hipMemcpyDeviceToHost, h->s));
    SGCHK(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status sg_gradients(sg_handle* h, const float* d_params, const float* d_fields, const int32_t* host_idx,
                       float* loss_out, float* grads_out) {
    if (!h || !d_params || !d_fields) return sgfail(LB_EINVAL, "NULL argument");
    lb_status st = check_idx(h, host_idx);
    if (st == LB_OK) st = set_indices(h, host_idx, h->c.batch);
    if (st == LB_OK) st = forward(h, d_params, h->c.batch);
    if (st == LB_OK) st = backward(h, d_fields, h->c.batch, loss_out);
    if (st != LB_OK) return st;
    if (grads_out) {
        SGCHK(hipMemcpyAsync(grads_out, ptr<float>(h, h->pl.g_off), 4ull * h->pl.npacked, hipMemcpyDeviceToHost, h->s));
        SGCHK(hipStreamSynchronize(h->s));
    }
    return LB_OK;
}

lb_status sg_train_step(sg_handle* h, const float* d_params, const float* d_fields, const int32_t* host_idx,
                        float* loss_out) {
    lb_status st = sg_gradients(h, d_params, d_fields, host_idx, loss_out, nullptr);
    if (st != LB_OK) return st;
    return adam(h);
}

lb_status sg_train_epochs(sg_handle* h, const float* d_params, const float* d_fields, int32_t n, int32_t epochs,
                          uint64_t seed, float* losses_out) {
    if (!h || !d_params || !d_fields || n < h->c.batch || epochs < 0)
        return sgfail(LB_EINVAL, "need the parameter and field arrays, n >= batch and epochs >= 0");
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::mt19937_64 rng(seed);
    const int B = h->c.batch, nbatch = n / B;
    int* idx = ptr<int>(h, h->pl.idx_off);
    double* lsum = ptr<double>(h, h->pl.lsum_off);
    for (int e = 0; e < epochs; ++e) {
        for (int k = n - 1; k > 0; --k) {  // Fisher-Yates with the seeded generator
            const int j = (int)(rng() % (uint64_t)(k + 1));
            std::swap(order[k], order[j]);
        }
        // the steps run back to back: the indices go up kIdxSteps batches at a time (stream
        // ordered after the steps that read the previous ones) and the batch losses are summed
        // on the device, in step order, and read once per epoch
        SGCHK(hipMemsetAsync(lsum, 0, sizeof(double), h->s));
        for (int b0 = 0; b0 < nbatch; b0 += kIdxSteps) {
            const int nb = std::min(kIdxSteps, nbatch - b0);
            SGCHK(hipMemcpyAsync(idx, order.data() + (size_t)b0 * B, 4ull * B * nb, hipMemcpyHostToDevice, h->s));
            for (int b = 0; b < nb; ++b) {
                const int* ib = idx + (size_t)b * B;
                lb_status st = forward(h, d_params, B, true, ib);
                if (st == LB_OK) st = backward(h, d_fields, B, nullptr, ib, lsum);
                if (st == LB_OK) st = adam(h);
                if (st != LB_OK) return st;
            }
        }
        double sum = 0.0;
        SGCHK(hipMemcpyAsync(&sum, lsum, sizeof(double), hipMemcpyDeviceToHost, h->s));
        SGCHK(hipStreamSynchronize(h->s));
        if (losses_out) losses_out[e] = (float)(sum / nbatch);
    }
    SGCHK(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status sg_predict(sg_handle* h, const float* d_params, int32_t n, float* d_out) {
    if (!h || !d_params || !d_out || n < 0) return sgfail(LB_EINVAL, "bad argument");
    const int H = h->c.height, W = h->c.width, L = kLayers - 1;
    std::vector<int32_t> idx((size_t)h->c.batch);
    for (int s0 = 0; s0 < n; s0 += h->c.batch) {
        const int nb = std::min(h->c.batch, n - s0);
        for (int b = 0; b < nb; ++b) idx[b] = s0 + b;
        lb_status st = set_indices(h, idx.data(), nb);
        if (st == LB_OK) st = forward(h, d_params, nb, false);
        if (st != LB_OK) return st;
        const long long P = (long long)nb * H * W;
        hipLaunchKernelGGL(k_unpack_out, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, h->s,
                           ptr<float>(h, h->pl.z_off[L]), nb, H, W, kCoutPad[L],
                           d_out + (long long)s0 * SG_OUTPUTS * H * W);
        SGCHK(hipGetLastError());
        SGCHK(hipStreamSynchronize(h->s));  // the index staging buffer is reused by the next chunk
    }
    return LB_OK;
}

lb_status sg_layer_output(sg_handle* h, int32_t layer, float* host_out) {
    if (!h || !host_out || layer < 0 || layer >= kLayers) return sgfail(LB_EINVAL, "bad argument");
    if (!h->z_valid && layer + 1 < kLayers)
        return sgfail(LB_ESTATE, "the last forward pass (a prediction) kept only the output layer's pre-activation");
    const size_t n = (size_t)h->nb_last * h->c.height * h->c.width * kCoutPad[layer];
    SGCHK(hipMemcpyAsync(host_out, ptr<float>(h, h->pl.z_off[layer]), 4 * n, hipMemcpyDeviceToHost, h->s));
    SGCHK(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status sg_layer_input(sg_handle* h, int32_t layer, float* host_out) {
    if (!h || !host_out || layer < 0 || layer >= kLayers) return sgfail(LB_EINVAL, "bad argument");
    const size_t n = (size_t)h->nb_last * h->c.height * h->c.width * kCinPad[layer];
    const size_t off = layer == 0 ? h->pl.x0_off : h->pl.y_off[layer - 1];
    std::vector<uint16_t> tmp(n);
    SGCHK(hipMemcpyAsync(tmp.data(), h->ws + off, 2 * n, hipMemcpyDeviceToHost, h->s));
    SGCHK(hipStreamSynchronize(h->s));
    for (size_t k = 0; k < n; ++k) {
        const uint32_t bits = (uint32_t)tmp[k] << 16;
        std::memcpy(&host_out[k], &bits, 4);
    }
    return LB_OK;
}

lb_status sg_conv(sg_handle* h, int32_t layer, int32_t mode, int32_t nb, const void* d_in, const float* d_zprev,
                  float* d_z, void* d_out) {
    if (!h || layer < 0 || layer >= kLayers || (mode != 0 && mode != 1)) return sgfail(LB_EINVAL, "bad argument");
    if (nb < 1 || nb > h->c.batch) return sgfail(LB_EINVAL, "nb must lie in 1..batch");
    if (!d_in || !d_out) return sgfail(LB_EINVAL, "d_in and d_out are required");
    if (mode == 1 && (layer == 0 || !d_zprev)) return sgfail(LB_EINVAL, "the data gradient needs layer >= 1 and d_zprev");
    const long long P = (long long)nb * h->c.height * h->c.width;
    return launch_conv(h, layer, mode, P, static_cast<const bf16*>(d_in), mode == 1 ? d_zprev : nullptr,
                       mode == 0 ? d_z : nullptr, static_cast<bf16*>(d_out));
}

lb_status sg_weight_grad(sg_handle* h, int32_t layer, int32_t nb, const void* d_g, const void* d_x, float* d_dw,
                         float* d_db) {
    if (!h || layer < 0 || layer >= kLayers) return sgfail(LB_EINVAL, "bad argument");
    if (nb < 1 || nb > h->c.batch) return sgfail(LB_EINVAL, "nb must lie in 1..batch");
    if (!d_g || !d_x || !d_dw || !d_db) return sgfail(LB_EINVAL, "NULL device array");
    const long long P = (long long)nb * h->c.height * h->c.width;
    return launch_wgrad(h, layer, P, static_cast<const bf16*>(d_g), static_cast<const bf16*>(d_x), d_dw, d_db);
}

lb_status sg_smooth(const float* d_in, float* d_out, int32_t planes, int32_t height, int32_t width,
                    void* hip_stream) {
    if (!d_in || !d_out || d_in == d_out || planes < 0 || height < 1 || width < 1)
        return sgfail(LB_EINVAL, "bad argument (the filter is not in place)");
    const long long n = (long long)planes * height * width;
    if (n == 0) return LB_OK;
    hipLaunchKernelGGL(k_smooth, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       d_in, d_out, (long long)planes, height, width);
    SGCHK(hipGetLastError());
    return LB_OK;
}

lb_status sg_destagger(float* d_fields, int32_t count, int32_t height, int32_t width, void* hip_stream) {
    if (!d_fields || count < 0 || height < 1 || width < 1) return sgfail(LB_EINVAL, "bad argument");
    if ((long long)height * width > (1LL << 30)) return sgfail(LB_EINVAL, "plane too large");
    if (count == 0) return LB_OK;
    hipLaunchKernelGGL(k_destagger, dim3((unsigned)count), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_fields,
                       height, width);
    SGCHK(hipGetLastError());
    return LB_OK;
}

lb_status sg_free(sg_handle* h) {
    delete h;
    return LB_OK;
}

const char* sg_last_error(void) { return g_sgerr.c_str(); }

}  // extern "C"
