// Internal definitions shared by the device kernels and the host side of libljmd.
// Not part of the public C ABI (that is include/ljmd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ljmd {

// Per type pair coefficients of the truncated-and-shifted pair form, FP64.
// rc2 = r_cut^2 and rl2 = (r_cut + skin)^2 are 0 for a disabled pair. For the LJ form:
struct PairCoef {
    double rc2;
    double rl2;
    double lj1;    // 48 eps sig^12   force:  f = r^-2 r^-6 (lj1 r^-6 - lj2)
    double lj2;    // 24 eps sig^6
    double lj3;    // 4 eps sig^12    energy: u = r^-6 (lj3 r^-6 - lj4) - shift
    double lj4;    // 4 eps sig^6
    double shift;  // 4 eps ((sig/r_cut)^12 - (sig/r_cut)^6), the energy at r_cut (shifted
                   // force: that plus r_cut fcut)
    double fcut;   // shifted force only: F(r_cut), the pair force magnitude at the cutoff
};
// (the other forms keep their coefficients in lj1..lj4 too: see form64 in ljmd_force.h)

// Device status block (one per system or batch). Rebuild requests live in a separate
// per-replica array: req[2 r + b] for replica r, b the position buffer just written.
struct DevStatus {
    int status;              // ST_* bits
    int max_count;           // longest list seen at a build
    unsigned long long builds;
    unsigned long long entries;  // list entries written at the last build
    int debug;               // first failed check of a debug build (DBG_*), else 0
};

// Parameters of one replica (a single system is a batch of one). Replica r owns particles
// [poff, poff + n), cells [coff, coff + ncell] (ncell + 1 entries of cell_start), bricks
// [boff, boff + nbrick) and the pair table rows [pair_off, pair_off + ntypes^2).
struct RepParams {
    double L[3], invL[3], inv_w[3];
    double dt, half_dt, lim2;
    double single_rl2;       // (r_cut + skin)^2 of pair (0,0)
    double pad0;
    int nc[3];
    int poff, n;
    int coff, ncell;
    int boff, nbrick;
    int canonical;           // some axis has fewer than 3 cells
    int ntypes, pair_off;
    int active;              // 0 for a free slot
    int tile_cap;            // the replica's own tile capacity: a brick's tile is staged in
                             // the force kernels only if it fits this (and the launch's LDS),
                             // so the choice never depends on what shares a batch
};

enum { ST_OVERFLOW = 1, ST_NONFINITE = 2, ST_TILE = 4, ST_DEBUG = 8 };

// Debug builds (LJMD_DEBUG_CHECKS=1) check indices and capacities on the device; a failed
// check sets ST_DEBUG and records its code (the first one), and the access is skipped.
#ifndef LJMD_DEBUG_CHECKS
#define LJMD_DEBUG_CHECKS 0
#endif
enum {
    DBG_CELL = 1,       // a particle's cell outside its replica's cells (binning)
    DBG_SCATTER = 2,    // a particle's sorted slot outside its replica's range
    DBG_TILE = 3,       // a list entry written outside the brick's tile
    DBG_SLOT = 4,       // a list slot outside the list allocation
    DBG_READ = 5,       // a list entry read outside the brick's tile (force kernel)
    DBG_DANGEROUS = 6,  // forces at a position half the skin or more from the list's build
};

// Bricks: aligned groups of up to 2 x 2 x 2 cells whose cells are consecutive in the cell
// order. A brick's halo is every cell within one cell of it (up to 4 x 4 x 4 = 64 cells);
// the atoms of the halo, concatenated in halo order, form the brick's tile, and list
// entries are 16-bit indices into that tile.
struct BrickInfo {
    int first_cell;  // global index of the brick's first cell (its (0,0,0) corner)
    int ncell;       // cells in the brick (1..8)
    int nhalo;       // halo cells (<= HALO_MAX)
    int dims;        // halo extents hx | hy << 4 | hz << 8, brick extents ex << 12 | ey << 16 | ez << 20,
                     // bit 24 + a: axis a needs no minimum image (see MI_FREE),
                     // bit 27 + a: axis a is centred while staging (see CENTER)
    int rep;         // replica, -1 for an unused brick
    int pad;
    double centre[3];  // the brick's centre (box units), read on the centred axes
};
// Bit 24 + a of BrickInfo::dims is set when, on axis a, the brick's halo lies in cells
// 1 .. n_cell - 2 and n_cell >= 10. Between builds no particle moves more than skin/2 <
// one cell, so no halo particle can have wrapped, and every listed pair is closer than
// 4 cells + skin < L/2 on that axis: the plain difference x_j - x_i already is the minimum
// image, bit for bit.
constexpr int MI_FREE_SHIFT = 24;
// Bit 27 + a of BrickInfo::dims is set when the axis holds at least (brick cells + 2) cells.
// Let c be the brick's centre on that axis and w >= r_cut + skin the cell width. A brick
// particle lies within (brick cells) w / 2 + skin / 2 of c, so a partner closer than r_cut
// lies, in its nearest image, within (brick cells) w / 2 + w - skin / 2 < L / 2 of c. Moving
// every staged atom and the brick's own particles to their image nearest c,
// x - L rint((x - c) / L), therefore puts every pair that can interact at its minimum image,
// and the pair loop takes the plain difference on that axis. Any other pair is at least
// r_cut apart in every image and stays beyond the cutoff.
constexpr int CENTER_SHIFT = 27;
// Per-brick tile table written by the list build: offsets off[0..64], starts start[0..63],
// halo count.
constexpr int TILE_TAB = 2 * 64 + 2;
// Halo cell: its rank and the periodic image it is seen in from the brick, per axis a
// value in {-1, 0, 1} stored as (s + 1) in two bits: sx | sy << 2 | sz << 4.
struct HaloCell {
    int rank;
    int shift;
};
constexpr int HALO_MAX = 64;
constexpr int TILE_MAX = 2560;        // tile atoms staged in LDS at most (32 B each: 80 KiB)
// Tile capacity bricks are shaped for: 1536 atoms (48 KiB) plus the build's 3.9 KiB of static
// LDS lets three 512-thread workgroups share a CU's 160 KiB.
constexpr int TILE_TARGET = 1536;
constexpr int LJMD_MAX_TYPES_DEVICE = 16;     // type count the kernels' tables allow
constexpr size_t LDS_MAX_BYTES = 160 * 1024;  // LDS of one workgroup on gfx950
constexpr int TILE_INDEX_MAX = 65535; // 16-bit tile indices
constexpr int FORCE_BATCH = 2;  // neighbour positions requested together (1, 2, 4, 8)
constexpr int BUILD_BATCH = 2;  // candidate rounds tested together in the build
constexpr int FLAT_ROUNDS = 12; // rounds of 64 candidates a wavefront-per-particle build item holds
constexpr int FLAT_RING = 128;  // list entries a build wavefront holds before writing them out

enum { MODE_EVAL = 0, MODE_FUSED = 1, MODE_FINAL = 2 };
// Pair forms (one per system; the batch uses LJ). The PairCoef fields lj1..lj4 hold each
// form's coefficients (see form64 in ljmd_force.h).
enum { STYLE_LJ = 0, STYLE_MIE = 1, STYLE_GAUSS = 2, STYLE_YUKAWA = 3, STYLE_COUNT = 4 };
// Flag on a style: its shifted-force variant (force less F(r_cut), energy less the matching
// linear term; PairCoef::fcut).
constexpr int STYLE_SF = 8;
enum { PREC_FP64 = 0, PREC_MIXED = 1 };

constexpr int LJMD_MAX_TYPES_DEV = 16; // equals LJMD_MAX_TYPES of the public header
constexpr int RED_BLOCK = 256;       // reduction workgroup size
constexpr int RED_QUANT = 8;         // U, W[6], K
constexpr int SORT_LDS = 1024;       // in-cell sort capacity per workgroup
constexpr int SCAN_TILE = 8192;      // counts per LDS tile of the scan (multiple of 1024)
constexpr int WORK_SORT_MAX = 1024;  // bricks with more atoms keep their particles in order

// Dynamic LDS of the force kernel: the tile as double4 records (x, y, z, type), then the
// pair table when there are several types.
__host__ __device__ inline size_t force_lds_bytes(int tile_cap, int ntypes) {
    size_t b = (size_t)tile_cap * 4 * sizeof(double);
    if (ntypes > 1) b += (size_t)ntypes * ntypes * sizeof(PairCoef);
    return b;
}

// Dynamic LDS of the list build: the tile as double4 records, then the list radii squared
// when there are several types.
__host__ __device__ inline size_t nlist_lds_bytes(int tile_cap, int ntypes) {
    size_t b = (size_t)tile_cap * 4 * sizeof(double);
    if (ntypes > 1) b += (size_t)ntypes * ntypes * sizeof(double);
    return b;
}

// Arguments of the force kernel family (by value). The grid covers bricks [0, nbrick);
// each brick reads its replica's parameters.
struct ForceArgs {
    const RepParams *reps;
    const double4 *pos_in;   // x, y, z, type (as double); sorted order
    double4 *pos_out;        // MODE_FUSED: positions after the drift
    double4 *vel;            // vx, vy, vz, 1/m
    int4 *img;               // image counters x, y, z and the tag in w
    const double4 *xb;       // positions at the last build
    double4 *force;          // MODE_EVAL / MODE_FINAL output
    const int *nl_count;
    const uint16_t *nlist;   // 16-bit tile indices
    const int32_t *nlist32;  // tree lists: 32-bit sorted-order indices (k_force_glist)
    const uint16_t *work;    // per brick: order in which its particles are taken
    const BrickInfo *bricks;
    const int *cell_start;
    const int *tile_tab;     // TILE_TAB ints per brick, written by the build
    double *u_out;           // per-particle energy half-sums (ENERGY)
    double *w_out;           // per-particle virial half-sums, 6 per particle (ENERGY)
    double *ke_out;          // per-particle kinetic energy at the full step (ENERGY, FUSED)
    const PairCoef *pair;    // pair rows of all replicas
    int *req;                // rebuild requests, 2 per replica
    int *rem;                // MODE_FUSED with step limits: steps left, 2 per replica (or null)
    const int *only;         // replica mask (null: all replicas)
    int *status;
    int *rep_status;         // per-replica status bits (or null)
    int cur;                 // position buffer read (0/1): req/rem parity
    int npad, cap, lshift, nbrick, tile_cap, max_ntypes;
};

// NVT thermostat scalars on the device (doubles): the state at the last step boundary
// (xi, eta), the scale factor of the last end-of-step thermostat half step that the stored
// velocities still lack (1 between calls), the thermostat half step that opens the next step
// (its scale factor, and xi and eta after it), and the kinetic energy after the last scaling.
enum { TH_XI = 0, TH_ETA = 1, TH_SPEND = 2, TH_SB = 3, TH_XIB = 4, TH_ETAB = 5, TH_K = 6,
       TH_COUNT = 8 };

struct NvtParams {
    double dt;
    double invQ;   // 1 / Q, Q = N_f kT tau^2; 0 for zero coupling
    double g;      // N_f kT
    int np;        // partial sums to reduce
    int begin_only;
};

struct KickDriftArgs {
    const RepParams *reps;
    const double *scale;     // NVT: velocities are first scaled by scale[0] * scale[1] (or null)
    const int *prep;         // replica of each particle (null: replica 0)
    const double4 *pos_in;
    double4 *pos_out;
    double4 *vel;
    int4 *img;
    const double4 *xb;
    const double4 *force;
    int *req;
    const int *only;         // replica mask (null: all)
    int cur;
    int n;                   // particle slots [0, n)
};

struct RebuildArgs {
    const RepParams *reps;
    const int *prep;         // replica of each particle (null: replica 0)
    const int *crep;         // replica of each cell (null: replica 0)
    const int *go;           // replica r rebuilds only if go[r * go_stride] != 0
    int go_stride;
    const double *rl2_table; // pair rows of all replicas: list radii squared
    double4 *pos;            // current positions (sorted order); rewritten in new order
    double4 *pos_scr;
    double4 *vel, *vel_scr;
    int4 *img, *img_scr;
    double4 *xb;
    int *key, *slot, *perm;
    int *cell_count;         // zero between builds
    int *cell_start;         // ncell + 1 entries per replica
    int *cell_lo;            // per cell: members in the lower z half of the cell (cell method;
                             // null for the tree method's sort grid)
    int split_halves;        // list build items may be half cells (bricks of few cells)
    const int *cell_rank;    // per replica: local linear cell index -> global cell index
    const int *cell_xyz;     // global cell -> packed local (cx | cy << 10 | cz << 20)
    int *nl_count;
    uint16_t *nlist;
    uint16_t *work;          // per brick: its particles by decreasing list length (local index)
    const BrickInfo *bricks;
    const HaloCell *halo;
    int *tile_tab;
    DevStatus *st;
    int *rep_status;         // per-replica status bits (or null)
    int n, ncell, nbrick, nrep;   // slot counts of the arrays
    int npad, cap, lshift, tile_cap, max_ntypes;
    // tree (BVH) lists: the sort grid's cells are (type, cx, cy, cz), type-major, so each
    // type's particles are contiguous; the gather then records each particle's cell
    int typed_cells;              // spatial cells per type (0: cells are spatial only)
    int *cell_of;                 // cell of each particle in the new order (or null)
};

// Tree (BVH) neighbour lists, one tree per particle type over the type's particles in their
// sorted order: the Karras construction on the keys (cell << 32 | index), the children's boxes
// of every node from range reductions over box tables, and one traversal per particle and tree.
constexpr int BVH_LEAF = 1 << 30;   // child code: a leaf (particle index | BVH_LEAF)
// A tree node as a walk reads it, one 64-byte record per internal node: per child 24 bytes,
// the exact build position (3 doubles) of a leaf child or the box of an internal child in
// FP32 rounded outwards (lo x y z, hi x y z: the box only ever grows, so a walk never skips a
// neighbour), then the two child codes.
struct alignas(64) BvhNode {
    union {
        double pos[3];
        float box[6];
    } child[2];
    int left, right;
    int pad[2];
};
constexpr int BVH_STACK = 64;       // traversal stack (tree depth is at most the 64 key bits)
struct BvhArgs {
    const RepParams *reps;
    const int *go;           // rebuild gate (go[0])
    double4 *pos, *pos_scr, *vel, *vel_scr, *xb;
    int4 *img, *img_scr;
    const int *cell_start;   // typed cells: type t is [cell_start[t ncs], cell_start[(t+1) ncs])
    const int *cell_of;
    int *left, *right;       // internal node children (node of type t at s_t + local index)
    int *rlo, *rsplit, *rhi; // internal node's leaves [rlo, rhi]; the left child's end rsplit
    double *blk;             // per 64 leaves (sorted order): their box, lo x y z, hi x y z
    double *sblk;            // per 4096 leaves: their box
    BvhNode *node;           // per internal node: what a walk reads
    const double *rl2_table; // list radii squared per type pair (0: pair disabled)
    int *nl_count;
    int32_t *nlist32;        // 32-bit sorted-order indices, 4 per 16-byte chunk (see slot32)
    DevStatus *st;
    int n, ntypes, ncs, npad, cap, lshift;
    // the order in which the walk kernel's threads take the types' particle ranges: the
    // types with the widest list radii (the longest walks) first, so they do not form a tail
    int type_order[LJMD_MAX_TYPES_DEVICE];
};

// ---------------------------------------------------------------- launchers
hipError_t launch_upload(hipStream_t s, const double *pos, const double *vel, const int *type,
                         const double *mass, double4 *pos4, double4 *vel4, int4 *img, int n,
                         const double L[3], int set_vel, int set_img, const int *img_in,
                         int poff);
hipError_t launch_kick_drift(hipStream_t s, const KickDriftArgs &a);
hipError_t launch_force(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                        bool energy, int block, int style = STYLE_LJ);
hipError_t launch_force_lj(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                           bool energy, int block);
hipError_t launch_force_mie(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                            bool energy, int block);
hipError_t launch_force_gauss(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                              bool energy, int block);
hipError_t launch_force_yukawa(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                               bool energy, int block);
// the shifted-force variants (STYLE_SF)
hipError_t launch_force_lj_sf(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                              bool energy, int block);
hipError_t launch_force_mie_sf(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                               bool energy, int block);
hipError_t launch_force_gauss_sf(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                                 bool energy, int block);
hipError_t launch_force_yukawa_sf(hipStream_t s, const ForceArgs &a, int prec, int tpp,
                                  int mode, bool energy, int block);
hipError_t launch_rebuild(hipStream_t s, const RebuildArgs &a, hipEvent_t *ev = nullptr);
// The sort of launch_rebuild (bin, scan, scatter, gather) over the typed sort grid, then the
// tree build and traversal; ev as for launch_rebuild (the tree kernels in the last slot).
hipError_t launch_rebuild_bvh(hipStream_t s, const RebuildArgs &a, const BvhArgs &b,
                              hipEvent_t *ev = nullptr);
hipError_t launch_sort_cells(hipStream_t s, const RebuildArgs &a, hipEvent_t *ev);
hipError_t launch_force_glist(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                              bool energy, int block);
hipError_t launch_reduce(hipStream_t s, const double *u, const double *w, const double *ke,
                         const double4 *vel, int poff, int n, double *partials, int nblocks_max,
                         double *out);
hipError_t launch_ke_partials(hipStream_t s, const double4 *vel, int poff, int n,
                              double *partials, int nblocks_max, int *np_out);
hipError_t launch_nvt_thermo(hipStream_t s, const double *partials, const NvtParams &p,
                             double *th);
hipError_t launch_nvt_finalize(hipStream_t s, double4 *vel, int poff, int n, double *th);
hipError_t launch_thermo_nvt_k(hipStream_t s, double *row, const double *th);
hipError_t launch_negate_vel(hipStream_t s, double4 *vel, int poff, int n);
hipError_t launch_unsort_vec(hipStream_t s, const double4 *src, const int4 *img, int poff,
                             int n, double *dst);
hipError_t launch_unsort_img(hipStream_t s, const int4 *img, int poff, int n, int *dst);
hipError_t launch_unsort_scalar(hipStream_t s, const double *src, int width, const int4 *img,
                                int poff, int n, double *dst);
hipError_t launch_fill_status(hipStream_t s, DevStatus *st);
hipError_t launch_fill_int(hipStream_t s, int *p, int n, int value);
hipError_t launch_decode_list(hipStream_t s, const RebuildArgs &a, int *out);

}  // namespace ljmd
