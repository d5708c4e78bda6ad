// Host-side check of the step kernels' neighbour addressing: for every node
// of a set of grids (ragged widths, wrapped rows and columns, the widest and
// largest grids the host accepts), the 32-bit neighbour offsets of NbrE (2-D)
// and Nb3E (3-D) must equal the 64-bit blocked-layout index of the wrapped
// neighbour node.
// Runs on the CPU only (no kernel launch); prints one line per grid and
// exits non-zero on the first mismatch.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lb3_index.h"
#include "lb_device.h"

using namespace lbk;

template <int M>
static long long check_rows(int nx, int ny, const std::vector<int>& rows, const std::vector<int>& cols) {
    KParams<double> kp{};
    kp.nx = nx;
    kp.ny = ny;
    long long checked = 0;
    for (int y : rows) {
        for (int x : cols) {
            const NbrE<M> e(kp, x, y);
            const Nbr n(kp, x, y);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const long long want = pidx<M>(0, n.at(dx, dy));
                    const long long got = e.at(dx, dy);
                    if (want != got) {
                        std::printf("MISMATCH M=%d grid %dx%d node (%d,%d) d=(%d,%d): %lld != %lld\n", M, nx, ny, x,
                                    y, dx, dy, got, want);
                        std::exit(1);
                    }
                    ++checked;
                }
        }
    }
    return checked;
}

// every row and column when all is set; otherwise the edge rows and a middle
// row, and the first, last and middle 200 columns
template <int M>
static void grid(int nx, int ny, bool all) {
    std::vector<int> rows, cols;
    if (all) {
        for (int y = 0; y < ny; ++y) rows.push_back(y);
        for (int x = 0; x < nx; ++x) cols.push_back(x);
    } else {
        for (int y : {0, 1, 2, ny / 2, ny - 3, ny - 2, ny - 1})
            if (y >= 0 && y < ny) rows.push_back(y);
        for (int x = 0; x < nx; ++x) {
            if (x >= 200 && x < nx / 2 - 100) x = nx / 2 - 100;
            if (x >= nx / 2 + 100 && x < nx - 200) x = nx - 200;
            cols.push_back(x);
        }
    }
    const long long c = check_rows<M>(nx, ny, rows, cols);
    std::printf("ok M=%d grid %dx%d: %lld offsets\n", M, nx, ny, c);
}

template <int M>
static void all_grids() {
    const int small[][2] = {{2, 2}, {3, 5}, {63, 7}, {64, 4}, {65, 9}, {67, 45}, {127, 3}, {128, 130}, {300, 11}};
    for (const auto& g : small) grid<M>(g[0], g[1], true);
    grid<M>(4096, 4096, false);
    grid<M>(46340, 46340, false);  // nx ny just below 2^31
    const int widest = (int)((((1ll << 31) - 1) / (9 + 5 * M)) - 64);  // the host's width limit
    grid<M>(widest, 2, false);
    grid<M>((int)(((1ll << 31) - 1) / widest), widest, false);  // tall, near 2^31 nodes
}

struct Grid3 {
    int nx, ny, nz;
};

// 3-D: every node of small boxes; edge planes and a middle plane of large ones
template <int M>
static void box(int nx, int ny, int nz, bool all) {
    const Grid3 g{nx, ny, nz};
    std::vector<int> xs, ys, zs;
    auto pick = [&](int n, std::vector<int>& v) {
        if (all) {
            for (int i = 0; i < n; ++i) v.push_back(i);
        } else {
            for (int i : {0, 1, 2, n / 2, n - 3, n - 2, n - 1})
                if (i >= 0 && i < n) v.push_back(i);
        }
    };
    pick(nx, xs);
    pick(ny, ys);
    pick(nz, zs);
    if (!all) {  // first, middle and last 130 columns
        xs.clear();
        for (int x = 0; x < nx; ++x) {
            if (x >= 130 && x < nx / 2 - 65) x = nx / 2 - 65;
            if (x >= nx / 2 + 65 && x < nx - 130) x = nx - 130;
            xs.push_back(x);
        }
    }
    long long checked = 0;
    for (int z : zs)
        for (int y : ys)
            for (int x : xs) {
                const lb3k::Nb3E<M> e(g, x, y, z);
                const lb3k::Nb3 n(g, x, y, z);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const long long want = lb3k::p3<M>(0, n.at(dx, dy, dz));
                            const long long got = e.at(dx, dy, dz);
                            if (want != got) {
                                std::printf("MISMATCH 3-D M=%d box %dx%dx%d node (%d,%d,%d) d=(%d,%d,%d): %lld != %lld\n",
                                            M, nx, ny, nz, x, y, z, dx, dy, dz, got, want);
                                std::exit(1);
                            }
                            ++checked;
                        }
            }
    std::printf("ok 3-D M=%d box %dx%dx%d: %lld offsets\n", M, nx, ny, nz, checked);
}

template <int M>
static void all_boxes() {
    const int small[][3] = {{2, 2, 2}, {3, 5, 4}, {21, 13, 11}, {64, 3, 2}, {65, 7, 5}, {130, 4, 3}};
    for (const auto& b : small) box<M>(b[0], b[1], b[2], true);
    box<M>(256, 256, 256, false);
    box<M>(1290, 1290, 1290, false);  // nx ny nz just below 2^31
    const int widest = (int)((((1ll << 31) - 1) / (19 + 7 * M)) - 64);  // the host's width limit
    box<M>(widest, 2, 2, false);
    box<M>(5, 20000, 20000, false);
}

int main() {
    all_grids<1>();
    all_grids<2>();
    all_grids<3>();
    all_grids<4>();
    all_boxes<1>();
    all_boxes<2>();
    all_boxes<3>();
    all_boxes<4>();
    std::printf("all neighbour offsets agree\n");
    return 0;
}
