// Host-side check of the brick tables that the force kernels rely on (compiled and run by
// tests/test_host_grid.py; no GPU is touched).
//
// For many box shapes, densities and list radii it builds the grid with the library's own
// make_grid and checks, brick by brick:
//   - the brick's extent fields and cells (contiguous, a box-aligned block of cells);
//   - the centring bit of an axis is set exactly when the axis holds at least (brick cells + 2)
//     cells, and the stored centre is the middle of the brick's cells;
//   - by sampling: a particle of the brick (at a build position in one of its cells, since
//     moved by less than skin/2) and a partner closer than r_cut, both wrapped into [0, L), give
//     their minimum-image difference on every centred axis when both are moved to their image
//     nearest the centre, and on every wrap-free axis as the plain difference.
// Prints "ok <bricks checked> <pairs checked>" or the first failures, and exits non-zero then.

#include "../paper_1308_5587_amd/csrc/ljmd_host.h"

#include <cmath>
#include <cstdio>
#include <random>

using namespace ljmd;

namespace {

double near_image(double x, double c, double L) {
    const double k = std::rint((x - c) * (1.0 / L));
    return std::fma(-k, L, x);
}

double wrap(double x, double L) {
    x -= L * std::floor(x / L);
    return x >= L ? 0.0 : x;
}

int failures = 0;

void fail(const char *what, double L, int b, int a, double v0, double v1) {
    if (failures < 20)
        std::printf("FAIL %s: L %.6g brick %d axis %d: %.17g vs %.17g\n", what, L, b, a, v0, v1);
    ++failures;
}

}  // namespace

int main() {
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long bricks_checked = 0, pairs_checked = 0;
    for (int trial = 0; trial < 400; ++trial) {
        const double rc = 1.0 + 2.0 * U(rng);
        const double skin = (trial % 7 == 0) ? 0.0 : 0.6 * U(rng);
        const double rl = rc + skin;
        double L[3];
        for (int a = 0; a < 3; ++a) {
            // 2 to 14 cells per axis (2 to 4 in a third of the trials: boxes of at most 27
            // cells and axes of fewer than 3 cells), a random fraction of a cell on top
            const int k = 2 + (int)(U(rng) * (trial % 3 == 0 ? 3 : 13));
            L[a] = rl * (1.0 + 1e-9) * (k + 0.99 * U(rng));
        }
        const double rho = 0.3 + 1.2 * U(rng);
        const int64_t n = (int64_t)(rho * L[0] * L[1] * L[2]) + 1;
        ReplicaGrid g;
        if (make_grid(L, rl, &g, n, TILE_TARGET) != LJMD_OK) continue;  // box below 2 r_L
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = L[a] / g.nc[a];
        for (int b = 0; b < g.nbrick; ++b) {
            const BrickInfo &bi = g.bricks[b];
            int lo[3] = {1 << 20, 1 << 20, 1 << 20}, hi[3] = {-1, -1, -1};
            for (int c = bi.first_cell; c < bi.first_cell + bi.ncell; ++c) {
                const int p = g.xyz[c];
                const int xyz[3] = {p & 1023, (p >> 10) & 1023, (p >> 20) & 1023};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], xyz[a]);
                    hi[a] = std::max(hi[a], xyz[a]);
                }
            }
            int nb[3];
            for (int a = 0; a < 3; ++a) nb[a] = hi[a] - lo[a] + 1;
            if (nb[0] * nb[1] * nb[2] != bi.ncell) fail("cells form a block", L[0], b, 0, bi.ncell, 0);
            for (int a = 0; a < 3; ++a) {
                const bool centred = (bi.dims >> (CENTER_SHIFT + a)) & 1;
                const bool want = g.nc[a] >= nb[a] + 2;
                if (centred != want) fail("centring bit", L[a], b, a, centred, want);
                if (centred) {
                    const int field = (bi.dims >> (12 + 4 * a)) & 15;
                    if (field != nb[a]) fail("extent field", L[a], b, a, field, nb[a]);
                    const double c = (lo[a] + 0.5 * nb[a]) * w[a];
                    if (std::fabs(bi.centre[a] - c) > 1e-12 * L[a])
                        fail("centre", L[a], b, a, bi.centre[a], c);
                }
            }
            ++bricks_checked;
            // sampled pairs: i built in one of the brick's cells, moved by less than skin/2;
            // j closer than r_cut
            for (int s = 0; s < 24; ++s) {
                double xi[3], d[3];
                double dn = 0.0, mv = 0.0;
                double mvv[3];
                for (int a = 0; a < 3; ++a) {
                    const int cell = lo[a] + (int)(U(rng) * nb[a]);
                    xi[a] = (cell + U(rng)) * w[a];
                    mvv[a] = (2.0 * U(rng) - 1.0);
                    mv += mvv[a] * mvv[a];
                    d[a] = (2.0 * U(rng) - 1.0);
                    dn += d[a] * d[a];
                }
                const double ms = 0.4999 * skin / std::sqrt(mv > 0 ? mv : 1.0) * U(rng);
                const double ds = 0.9999 * rc / std::sqrt(dn > 0 ? dn : 1.0) * U(rng);
                for (int a = 0; a < 3; ++a) {
                    const double xa = xi[a] + ms * mvv[a];
                    const double da = ds * d[a];
                    const double wi = wrap(xa, L[a]), wj = wrap(xa + da, L[a]);
                    const bool centred = (bi.dims >> (CENTER_SHIFT + a)) & 1;
                    const bool free_ax = (bi.dims >> (MI_FREE_SHIFT + a)) & 1;
                    if (free_ax) {
                        if (std::fabs((wj - wi) - da) > 1e-9) fail("wrap-free axis", L[a], b, a, wj - wi, da);
                    } else if (centred) {
                        const double got = near_image(wj, bi.centre[a], L[a]) -
                                            near_image(wi, bi.centre[a], L[a]);
                        if (std::fabs(got - da) > 1e-9) fail("centred axis", L[a], b, a, got, da);
                    }
                }
                ++pairs_checked;
            }
        }
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok %ld %ld\n", bricks_checked, pairs_checked);
    return 0;
}
