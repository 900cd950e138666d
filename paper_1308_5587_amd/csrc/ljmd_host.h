// Host-side helpers shared by the single-system and batch entry points of libljmd:
// error reporting, device allocation through the configured allocator, and the per-replica
// tables (pair coefficients, cell grid, bricks and halos) that the kernels read.
#pragma once

#include "ljmd_internal.h"
#include "ljmd.h"

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace ljmd {

// Thread-local message returned by ljmd_last_error; set_err formats it and returns code.
extern thread_local std::string g_last_error;
int set_err(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::ljmd::set_err(LJMD_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

#define CHK(expr)                     \
    do {                              \
        int r_ = (expr);              \
        if (r_ != LJMD_OK) return r_; \
    } while (0)

// Device memory through the user's allocator (or hipMalloc), with a record for freeing.
struct DeviceArena {
    ljmd_alloc_fn alloc = nullptr;
    ljmd_free_fn free = nullptr;
    void *ctx = nullptr;
    hipStream_t stream = nullptr;
    std::vector<std::pair<void *, size_t>> blocks;
    int64_t bytes = 0;

    int get(void **p, size_t n);
    void put(void *p);
    void release_all();
    template <class T>
    int get_t(T **p, size_t count) {
        return get(reinterpret_cast<void **>(p), count * sizeof(T));
    }
};

// Pair coefficients of one replica: ntypes x ntypes rows (row-major), list radii squared,
// and the largest list radius. Pairs with r_cut == 0 are disabled.
struct PairTable {
    std::vector<PairCoef> coef;
    std::vector<double> rl2;
    double rl_max = 0.0;
};
void make_pair_table(int ntypes, const double *eps, const double *sig, const double *rc,
                     double skin, PairTable *out);
// The table of another pair form (STYLE_MIE, STYLE_GAUSS, STYLE_YUKAWA) from its parameters,
// 4 per pair: (eps, sigma, n, m), (eps, sigma), (eps, kappa).
void make_form_table(int ntypes, int style, const double *par, const double *rc, double skin,
                     PairTable *out);
// The shifted-force variant of a table (style one of STYLE_LJ .. STYLE_YUKAWA): per pair,
// fcut = F(r_cut) (the force factor at r_cut times r_cut) and the shift raised by r_cut fcut,
// so that the kernels' f - fcut / r and u + r fcut - shift vanish at r_cut.
void apply_force_shift(int style, const double *rc, PairTable *pt);

// Cell grid, bricks and halos of one replica, with replica-local cell indices.
struct ReplicaGrid {
    int nc[3] = {0, 0, 0};
    bool canonical = false;          // fewer than 3 cells on some axis
    int ncell = 0, nbrick = 0, max_halo = 0;
    std::vector<int> rank;           // local linear cell index -> local cell index
    std::vector<int> xyz;            // local cell index -> packed (cx | cy << 10 | cz << 20)
    std::vector<BrickInfo> bricks;   // first_cell local, rep unset
    std::vector<HaloCell> halo;      // HALO_MAX per brick, ranks local
};
// Returns LJMD_E_BOX when r_L,max exceeds half a box edge. With n_atoms and tile_limit
// (atoms an LDS tile can hold) given, bricks shrink to single cells when a 2 x 2 x 2 brick's
// halo would not fit the tile at the mean density.
int make_grid(const double L[3], double rl_max, ReplicaGrid *g, int64_t n_atoms = 0,
              int tile_limit = 0);

// Tile capacity (atoms staged in LDS) for a mean occupancy of atoms_per_cell.
int choose_tile_cap(double atoms_per_cell, int max_halo, int max_ntypes, size_t lds_limit);

// Tile capacity for a replica's grid: exact when every halo is the whole box.
int grid_tile_cap(const ReplicaGrid &g, int64_t n_atoms, int max_ntypes, size_t lds_limit);

// The tile capacity bricks are shaped for: what fits the LDS, and at most TILE_TARGET.
int tile_limit_for(int max_ntypes, size_t lds_limit);

}  // namespace ljmd
