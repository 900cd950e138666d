// Host-side helpers shared by the single-system and batch entry points of libljmd.
#include "ljmd_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace ljmd {

thread_local std::string g_last_error;

int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ------------------------------------------------------------------ device memory

int DeviceArena::get(void **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 256;
    if (alloc) {
        *p = alloc(n, stream, ctx);
        if (!*p) return set_err(LJMD_E_NOMEM, "allocator returned NULL for %zu bytes", n);
    } else {
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess || !*p)
            return set_err(LJMD_E_NOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
    }
    blocks.emplace_back(*p, n);
    bytes += (int64_t)n;
    return LJMD_OK;
}

void DeviceArena::put(void *p) {
    if (!p) return;
    for (size_t k = 0; k < blocks.size(); ++k) {
        if (blocks[k].first == p) {
            const size_t n = blocks[k].second;
            if (free)
                free(p, n, stream, ctx);
            else
                (void)hipFree(p);
            bytes -= (int64_t)n;
            blocks.erase(blocks.begin() + (long)k);
            return;
        }
    }
}

void DeviceArena::release_all() {
    while (!blocks.empty()) put(blocks.back().first);
}

// ------------------------------------------------------------------ pair table

void make_pair_table(int nt, const double *eps, const double *sig, const double *rc,
                     double skin, PairTable *out) {
    out->coef.assign((size_t)nt * nt, PairCoef{});
    out->rl2.assign((size_t)nt * nt, 0.0);
    out->rl_max = 0.0;
    for (int k = 0; k < nt * nt; ++k) {
        PairCoef c{};
        const double e = eps[k], sg = sig[k], r = rc[k];
        if (r > 0.0) {
            const double rl = r + skin;
            c.rc2 = r * r;
            c.rl2 = rl * rl;
            out->rl_max = std::max(out->rl_max, rl);
            const double s6 = sg * sg * sg * sg * sg * sg;
            const double s12 = s6 * s6;
            c.lj1 = 48.0 * e * s12;
            c.lj2 = 24.0 * e * s6;
            c.lj3 = 4.0 * e * s12;
            c.lj4 = 4.0 * e * s6;
            const double q2 = (sg * sg) / c.rc2;
            const double q6 = q2 * q2 * q2;
            c.shift = 4.0 * e * (q6 * q6 - q6);
        }
        out->coef[k] = c;
        out->rl2[k] = c.rl2;
    }
}

void make_form_table(int nt, int style, const double *par, const double *rc, double skin,
                     PairTable *out) {
    out->coef.assign((size_t)nt * nt, PairCoef{});
    out->rl2.assign((size_t)nt * nt, 0.0);
    out->rl_max = 0.0;
    for (int k = 0; k < nt * nt; ++k) {
        PairCoef c{};
        const double *p = par + 4 * (size_t)k;
        const double r = rc[k];
        if (r > 0.0) {
            const double rl = r + skin;
            c.rc2 = r * r;
            c.rl2 = rl * rl;
            out->rl_max = std::max(out->rl_max, rl);
            if (style == STYLE_MIE) {
                const double e = p[0], sg = p[1], n = p[2], m = p[3];
                const double cm = (n / (n - m)) * std::pow(n / m, m / (n - m));
                c.lj1 = cm * e * n * std::pow(sg, n);
                c.lj2 = cm * e * m * std::pow(sg, m);
                c.lj3 = 0.5 * n;
                c.lj4 = 0.5 * m;
                c.shift = cm * e * (std::pow(sg / r, n) - std::pow(sg / r, m));
            } else if (style == STYLE_GAUSS) {
                const double e = p[0], sg = p[1];
                c.lj1 = e / (sg * sg);
                c.lj2 = -1.0 / (2.0 * sg * sg);
                c.lj3 = e;
                c.shift = e * std::exp(-c.rc2 / (2.0 * sg * sg));
            } else {  // Yukawa
                const double e = p[0], kappa = p[1];
                c.lj1 = e;
                c.lj2 = kappa;
                c.shift = e * std::exp(-kappa * r) / r;
            }
        }
        out->coef[k] = c;
        out->rl2[k] = c.rl2;
    }
}

void apply_force_shift(int style, const double *rc, PairTable *pt) {
    for (size_t k = 0; k < pt->coef.size(); ++k) {
        PairCoef &c = pt->coef[k];
        const double r = rc[k];
        if (!(r > 0.0)) continue;
        const double r2 = c.rc2;
        double f;  // the force factor at r_cut, as the kernels evaluate it
        if (style == STYLE_LJ) {
            const double r2i = 1.0 / r2;
            const double r6i = r2i * r2i * r2i;
            f = r2i * r6i * (c.lj1 * r6i - c.lj2);
        } else if (style == STYLE_MIE) {
            const double lr = std::log(r2);
            f = (c.lj1 * std::exp(-c.lj3 * lr) - c.lj2 * std::exp(-c.lj4 * lr)) / r2;
        } else if (style == STYLE_GAUSS) {
            f = c.lj1 * std::exp(c.lj2 * r2);
        } else {
            f = c.lj1 * std::exp(-c.lj2 * r) * (1.0 + c.lj2 * r) / (r2 * r);
        }
        c.fcut = f * r;
        c.shift += r * c.fcut;
    }
}

// ------------------------------------------------------------------ cell grid and bricks

static uint64_t spread3(uint64_t v) {  // 10-bit value -> every third bit
    uint64_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

// Boxes of at most 27 cells: every cell neighbours every other one, so each brick's halo is
// the whole box (its distinct cells) and the list build scans all of them with the branch-form
// minimum image. The bricks are the z-layers of cells: a few workgroups per replica, each
// with a share of the atoms comparable to a 2 x 2 x 2 brick of a large box.
static int make_small_box_grid(const int nc[3], const double L[3], ReplicaGrid *g) {
    const int ncell = nc[0] * nc[1] * nc[2];
    const int per = nc[0] * nc[1];
    const int nbrick = nc[2];
    g->rank.assign(ncell, 0);
    g->xyz.assign(ncell, 0);
    g->bricks.assign(nbrick, BrickInfo{});
    g->halo.assign((size_t)nbrick * HALO_MAX, HaloCell{0, 0});
    for (int x = 0; x < nc[0]; ++x)
        for (int y = 0; y < nc[1]; ++y)
            for (int z = 0; z < nc[2]; ++z) {
                const int r = z * per + x * nc[1] + y;
                g->rank[(x * nc[1] + y) * nc[2] + z] = r;
                g->xyz[r] = x | (y << 10) | (z << 20);
            }
    for (int b = 0; b < nbrick; ++b) {
        BrickInfo &bi = g->bricks[b];
        bi.first_cell = b * per;
        bi.ncell = per;
        bi.nhalo = ncell;
        // the stencil-walk fields are unused here. x and y span the box, so only z can be
        // centred (three or more layers); the brick is one layer thick (extent field ez)
        bi.dims = (1 << 20) | (nc[2] >= 3 ? 1 << (CENTER_SHIFT + 2) : 0);
        bi.rep = 0;
        bi.centre[2] = (b + 0.5) * L[2] / nc[2];
        for (int r = 0; r < ncell; ++r) g->halo[(size_t)b * HALO_MAX + r] = HaloCell{r, 21};
    }
    for (int a = 0; a < 3; ++a) g->nc[a] = nc[a];
    g->canonical = true;
    g->ncell = ncell;
    g->nbrick = nbrick;
    g->max_halo = ncell;
    return LJMD_OK;
}

int make_grid(const double L[3], double rl_max, ReplicaGrid *g, int64_t n_atoms, int tile_limit) {
    for (int a = 0; a < 3; ++a)
        if (rl_max > 0.5 * L[a])
            return set_err(LJMD_E_BOX, "r_cut + skin = %g exceeds half the box edge %g", rl_max, L[a]);
    // cell width >= the largest list radius (a relative margin keeps it strictly larger, so
    // rounding in the binning can never hide a pair)
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        const double r = rl_max > 0.0 ? rl_max * (1.0 + 1e-12) : L[a] / 3.0;
        long v = (long)std::floor(L[a] / r);
        v = std::max(1L, std::min(1023L, v));
        nc[a] = (int)v;
    }
    const int ncell = nc[0] * nc[1] * nc[2];
    if (ncell <= 27) return make_small_box_grid(nc, L, g);
    // Bricks of up to 2 x 2 x 2 cells (one cell wide on an axis with fewer than 4 cells,
    // single cells when some axis has fewer than 3), bricks in Morton order, cells in Morton
    // order inside their brick: every brick is a contiguous range of cells.
    const bool canonical = nc[0] < 3 || nc[1] < 3 || nc[2] < 3;
    int ext[3], nb[3];
    for (int a = 0; a < 3; ++a) ext[a] = (!canonical && nc[a] >= 4) ? 2 : 1;
    if (n_atoms > 0 && tile_limit > 0) {
        // while the tile capacity this density asks for (choose_tile_cap's headroom) would
        // exceed the limit, halve the brick along z, then y, then x: 64 halo cells, 48, 36, 27
        const double per_cell = (double)n_atoms / ncell;
        for (int a = 2; a >= 0; --a) {
            const int halo = (ext[0] + 2) * (ext[1] + 2) * (ext[2] + 2);
            if (1.05 * halo * per_cell + 128.0 <= tile_limit) break;
            ext[a] = 1;
        }
    }
    for (int a = 0; a < 3; ++a) nb[a] = (nc[a] + ext[a] - 1) / ext[a];
    const int nbrick = nb[0] * nb[1] * nb[2];
    std::vector<std::pair<uint64_t, int>> bmort(nbrick);
    for (int x = 0; x < nb[0]; ++x)
        for (int y = 0; y < nb[1]; ++y)
            for (int z = 0; z < nb[2]; ++z) {
                const int lin = (x * nb[1] + y) * nb[2] + z;
                bmort[lin] = {spread3(x) | (spread3(y) << 1) | (spread3(z) << 2), lin};
            }
    std::sort(bmort.begin(), bmort.end());
    g->rank.assign(ncell, 0);
    g->xyz.assign(ncell, 0);
    g->bricks.assign(nbrick, BrickInfo{});
    std::vector<int> brick_lo(3 * nbrick), brick_n(3 * nbrick);
    int next = 0;
    for (int bo = 0; bo < nbrick; ++bo) {
        const int lin = bmort[bo].second;
        const int bz = lin % nb[2], by = (lin / nb[2]) % nb[1], bx = lin / (nb[1] * nb[2]);
        const int lo[3] = {bx * ext[0], by * ext[1], bz * ext[2]};
        int cn[3];
        for (int a = 0; a < 3; ++a) cn[a] = std::min(ext[a], nc[a] - lo[a]);
        BrickInfo &bi = g->bricks[bo];
        bi.first_cell = next;
        bi.ncell = 0;
        bi.rep = 0;
        for (int c = 0; c < 8; ++c) {
            const int l[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            if (l[0] >= cn[0] || l[1] >= cn[1] || l[2] >= cn[2]) continue;
            const int x = lo[0] + l[0], y = lo[1] + l[1], z = lo[2] + l[2];
            g->rank[(x * nc[1] + y) * nc[2] + z] = next;
            g->xyz[next] = x | (y << 10) | (z << 20);
            ++next;
            ++bi.ncell;
        }
        for (int a = 0; a < 3; ++a) {
            brick_lo[3 * bo + a] = lo[a];
            brick_n[3 * bo + a] = cn[a];
        }
    }
    // halo of each brick: cells lo-1 .. lo+n per axis, seen in the periodic image given by
    // the wrap; duplicates (fewer than 3 cells on an axis) keep their first occurrence
    g->halo.assign((size_t)nbrick * HALO_MAX, HaloCell{0, 0});
    int max_halo = 0;
    for (int bo = 0; bo < nbrick; ++bo) {
        BrickInfo &bi = g->bricks[bo];
        int hd[3];
        for (int a = 0; a < 3; ++a) hd[a] = brick_n[3 * bo + a] + 2;
        bi.dims = hd[0] | (hd[1] << 4) | (hd[2] << 8) | (brick_n[3 * bo] << 12) |
                  (brick_n[3 * bo + 1] << 16) | (brick_n[3 * bo + 2] << 20);
        for (int a = 0; a < 3; ++a) {
            const int lo = brick_lo[3 * bo + a], hi = lo + brick_n[3 * bo + a];
            if (!canonical && nc[a] >= 10 && lo - 1 >= 1 && hi <= nc[a] - 2)
                bi.dims |= 1 << (MI_FREE_SHIFT + a);
            if (nc[a] >= brick_n[3 * bo + a] + 2) bi.dims |= 1 << (CENTER_SHIFT + a);
            bi.centre[a] = (lo + 0.5 * brick_n[3 * bo + a]) * L[a] / nc[a];
        }

        int nh = 0;
        for (int hx = 0; hx < hd[0]; ++hx)
            for (int hy = 0; hy < hd[1]; ++hy)
                for (int hz = 0; hz < hd[2]; ++hz) {
                    const int hc[3] = {hx, hy, hz};
                    int e[3], code = 0;
                    for (int a = 0; a < 3; ++a) {
                        int v = brick_lo[3 * bo + a] + hc[a] - 1;
                        int sh = 0;
                        if (v < 0) { v += nc[a]; sh = -1; }
                        else if (v >= nc[a]) { v -= nc[a]; sh = 1; }
                        e[a] = v;
                        code |= (sh + 1) << (2 * a);
                    }
                    const int r = g->rank[(e[0] * nc[1] + e[1]) * nc[2] + e[2]];
                    bool dup = false;
                    if (canonical)
                        for (int u = 0; u < nh; ++u) dup |= g->halo[(size_t)bo * HALO_MAX + u].rank == r;
                    if (dup) continue;
                    g->halo[(size_t)bo * HALO_MAX + nh] = HaloCell{r, code};
                    ++nh;
                }
        bi.nhalo = nh;
        max_halo = std::max(max_halo, nh);
    }
    for (int a = 0; a < 3; ++a) g->nc[a] = nc[a];
    g->canonical = canonical;
    g->ncell = ncell;
    g->nbrick = nbrick;
    g->max_halo = max_halo;
    return LJMD_OK;
}

int grid_tile_cap(const ReplicaGrid &g, int64_t n_atoms, int max_ntypes, size_t lds_limit) {
    if (g.max_halo < g.ncell)
        return choose_tile_cap((double)n_atoms / g.ncell, g.max_halo, max_ntypes, lds_limit);
    // every halo is the whole box: the tile holds exactly n atoms, no headroom needed
    const int lds_cap = choose_tile_cap(1e9, HALO_MAX, max_ntypes, lds_limit);
    const int64_t want = std::max<int64_t>(64, (n_atoms + 63) & ~63LL);
    return (int)std::min<int64_t>(want, lds_cap);
}

int tile_limit_for(int max_ntypes, size_t lds_limit) {
    return std::min(TILE_TARGET, choose_tile_cap(1e9, HALO_MAX, max_ntypes, lds_limit));
}

int choose_tile_cap(double atoms_per_cell, int max_halo, int max_ntypes, size_t lds_limit) {
    const double expect = max_halo * atoms_per_cell;
    // clamp before converting: a huge request (the largest tile the LDS allows) must not
    // overflow the integer
    int cap = (int)std::ceil(std::min(1.05 * expect + 128.0, (double)TILE_MAX));
    cap = std::min((cap + 63) & ~63, TILE_MAX);
    const size_t limit = std::min<size_t>(lds_limit, 64 * 1024) - 4096;
    while (cap > 64 && std::max(force_lds_bytes(cap, max_ntypes), nlist_lds_bytes(cap, max_ntypes)) > limit)
        cap -= 64;
    return cap;
}

}  // namespace ljmd
