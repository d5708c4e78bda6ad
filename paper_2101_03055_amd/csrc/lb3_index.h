// lb3_index.h -- node and population indexing of the 3-D path (lb3.hip) in
// the blocked layout: nodes n = (z ny + y) nx + x in blocks of 64, within a
// block the 19 + 7m populations as runs of 64 values.  Host-callable so the
// offsets can be checked on the CPU.
#pragma once

#include <hip/hip_runtime.h>

namespace lb3k {

constexpr int kBlk = 64;

// element index of population q of node n
template <int M>
__host__ __device__ __forceinline__ long long p3(int q, long long n) {
    constexpr int NQ = 19 + 7 * M;
    return ((n >> 6) * (NQ << 6) + (n & (kBlk - 1))) + ((long long)q << 6);
}

// 3 x 3 x 3 neighbourhood node indices, wrapped on periodic axes (on a walled
// axis the wrapped index is never used: links through a wall take the node
// itself).  KP: any record with int nx, ny, nz.
struct Nb3 {
    long long xo[3], yo[3], zo[3];
    template <class KP>
    __host__ __device__ __forceinline__ Nb3(const KP& kp, int x, int y, int z) {
        const long long sx = 1, sy = kp.nx, sz = (long long)kp.nx * kp.ny;
        xo[0] = (x == 0 ? kp.nx - 1 : x - 1) * sx;
        xo[1] = x * sx;
        xo[2] = (x == kp.nx - 1 ? 0 : x + 1) * sx;
        yo[0] = (y == 0 ? kp.ny - 1 : y - 1) * sy;
        yo[1] = y * sy;
        yo[2] = (y == kp.ny - 1 ? 0 : y + 1) * sy;
        zo[0] = (z == 0 ? kp.nz - 1 : z - 1) * sz;
        zo[1] = z * sz;
        zo[2] = (z == kp.nz - 1 ? 0 : z + 1) * sz;
    }
    __host__ __device__ __forceinline__ long long at(int dx, int dy, int dz) const {
        return zo[dz + 1] + yo[dy + 1] + xo[dx + 1];
    }
};

// The same neighbourhood as element offsets of population 0 (p3<M>(0, n') of
// the neighbour n'), with 32-bit node arithmetic: the first node R of each of
// the nine rows (y + dy, z + dz) gives one 64-bit product, (R >> 6) times the
// block size; the neighbour R + c then lies in block (R >> 6) + ((R & 63) + c)
// >> 6 at lane ((R & 63) + c) & 63, a 24-bit product.  Needs nx ny nz < 2^31
// and (nx + 64) (19 + 7m) < 2^31 (checked by the host).
template <int M>
struct Nb3E {
    static constexpr int Q = (19 + 7 * M) << 6;  // values per block
    long long rb[3][3];  // [dz + 1][dy + 1]: element offset of the block holding the row's first node
    int rm[3][3];        // lane of the row's first node in that block
    int col[3];          // columns x - 1, x, x + 1
    template <class KP>
    __host__ __device__ __forceinline__ Nb3E(const KP& kp, int x, int y, int z) {
        const int nx = kp.nx, ny = kp.ny, nz = kp.nz;
        const int yv[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
        const int zv[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int r = (zv[c] * ny + yv[b]) * nx;
                rb[c][b] = (long long)(r >> 6) * Q;
                rm[c][b] = r & (kBlk - 1);
            }
        col[0] = x == 0 ? nx - 1 : x - 1;
        col[1] = x;
        col[2] = x == nx - 1 ? 0 : x + 1;
    }
    __host__ __device__ __forceinline__ long long at(int dx, int dy, int dz) const {
        const int t = rm[dz + 1][dy + 1] + col[dx + 1];
        const unsigned blk = (unsigned)(t >> 6) & 0xffffffu;  // below 2^24 under the host's limits
        return rb[dz + 1][dy + 1] + (long long)(blk * (unsigned)Q + (unsigned)(t & (kBlk - 1)));
    }
};

}  // namespace lb3k
