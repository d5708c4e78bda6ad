// Host-side check of the step kernels' neighbour addressing: for every node
// of a set of grids (ragged widths, wrapped rows and columns, the widest and
// largest grids the host accepts), the 32-bit neighbour offsets of NbrE must
// equal the 64-bit blocked-layout index of the wrapped neighbour node.
// Runs on the CPU only (no kernel launch); prints one line per grid and
// exits non-zero on the first mismatch.
#include <cstdio>
#include <cstdlib>
#include <vector>

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

int main() {
    all_grids<1>();
    all_grids<2>();
    all_grids<3>();
    all_grids<4>();
    std::printf("all neighbour offsets agree\n");
    return 0;
}
