// Device helpers shared by the kernel translation units of libljmd (gfx950, wave64):
// minimum-image and distance arithmetic in the canonical operation order, the list-slot
// layout, and the brick tiles staged in LDS. Every file including this is compiled with
// -ffp-contract=off, so no multiply-add below is fused unless written explicitly.
#pragma once

#include "ljmd_internal.h"

namespace ljmd {

// A failed check of a debug build: the status bit, and the code of the first failure.
__device__ __forceinline__ void debug_fail(DevStatus *st, int code) {
    atomicOr(&st->status, ST_DEBUG);
    atomicCAS(&st->debug, 0, code);
}

// ---------------------------------------------------------------- arithmetic helpers

// Minimum image of a coordinate difference d in (-L, L): subtract k L with k = rint(d/L).
// For |d| away from L/2 by more than a few ulps this equals the branch form "if d >= L/2
// subtract L, else if d < -L/2 add L" bit for bit (fma(-k, L, d) rounds d - L once, as the
// branch form does); within a few ulps of L/2 the two may pick different images, both of
// length ~L/2, which is beyond every cutoff and list radius.
__device__ __forceinline__ double mi_rint(double d, double L, double invL) {
    double k = __builtin_rint(d * invL);
    return __builtin_fma(-k, L, d);
}

// Branch form of the minimum image, used where a list radius may reach L/2.
__device__ __forceinline__ double mi_branch(double d, double L) {
    double h = 0.5 * L;
    double up = d - L;
    double dn = d + L;
    return d >= h ? up : (d < -h ? dn : d);
}

__device__ __forceinline__ double r2_canon(double x, double y, double z) {
    double xx = x * x;
    double yy = y * y;
    double zz = z * z;
    double t = xx + yy;
    return t + zz;
}

// 1/x in FP64: the hardware reciprocal estimate (relative error below 5e-8 on gfx950) refined
// by one Newton step, which squares the error: below 3e-15 relative (measured over 2^20
// arguments in [0.3, 12]; a second step reproduces the correctly rounded quotient).
__device__ __forceinline__ double rcp64(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// The image of coordinate x nearest c: x - L rint((x - c) / L), rounded once; x itself when
// it already is that image.
__device__ __forceinline__ double near_image(double x, double c, double L, double invL) {
    const double k = __builtin_rint((x - c) * invL);
    return __builtin_fma(-k, L, x);
}

// Workgroup b of nb is dispatched to XCD (b mod 8). Map each XCD to a contiguous range
// of logical tiles so that spatial neighbours share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    int per = nb >> 3, rem = nb & 7;
    int x = b & 7, idx = b >> 3;
    return x * per + (x < rem ? x : rem) + idx;
}

__device__ __forceinline__ void wrap_coord(double &x, int &im, double L) {
    if (x >= L) {
        x = x - L;
        im += 1;
    } else if (x < 0.0) {
        x = x + L;
        im -= 1;
        if (x >= L) {  // x + L rounded up to L: the particle sits at 0 in its old image
            x = 0.0;
            im += 1;
        }
    }
}

// List slot of entry k of particle q with 2^ls lanes per particle: lanes own chunks of 8
// consecutive 16-bit entries, lane l holds chunks l, l + 2^ls, ...; for chunk index c the
// lanes of consecutive particles are adjacent, so a wavefront reads 64 x 16 contiguous bytes.
// In closed form: slot = (k >> (3 + ls)) * (npad << (3 + ls)) + (q << (3 + ls))
//                        + (k & (2^(3 + ls) - 1)).
__device__ __forceinline__ size_t nl_slot(int q, int k, int npad, int ls) {
    const int sh = 3 + ls;
    return (size_t)((unsigned)k >> sh) * ((size_t)npad << sh) + ((size_t)q << sh) +
           (size_t)(k & ((1 << sh) - 1));
}

// ---------------------------------------------------------------- brick tiles

// Offsets of a brick's tile: tile atom k belongs to halo cell h with off[h] <= k < off[h+1]
// and is the particle start[h] + (k - off[h]) of the sorted order.
struct TileSmem {
    int off[HALO_MAX + 1];
    int start[HALO_MAX];
    int shift[HALO_MAX];
    int nhalo;
    int total;
};

// Wavefront 0 reads the halo cells (lane h, h < nhalo) and scans their atom counts; with
// lo_out, also each halo cell's count of lower-z-half members (cell_lo).
__device__ __forceinline__ void tile_setup(const BrickInfo &bi, const HaloCell *halo_b,
                                           const int *cell_start, TileSmem &t,
                                           int *lo_out = nullptr, const int *cell_lo = nullptr) {
    if (threadIdx.x < 64) {
        const int h = threadIdx.x;
        int cnt = 0;
        if (h < bi.nhalo) {
            const HaloCell hc = halo_b[h];
            const int st = cell_start[hc.rank];
            cnt = cell_start[hc.rank + 1] - st;
            t.start[h] = st;
            t.shift[h] = hc.shift;
            if (lo_out) lo_out[h] = cell_lo[hc.rank];
        }
        int v = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o);
            if (h >= o) v += u;
        }
        t.off[h + 1] = v;
        if (h == 0) {
            t.off[0] = 0;
            t.nhalo = bi.nhalo;
        }
        if (h == 63) t.total = v;
    }
    __syncthreads();
}

// Halo cell of tile atom k (0 <= k < total): the h with off[h] <= k < off[h+1].
__device__ __forceinline__ int tile_cell(const TileSmem &t, int k) {
    int lo = 0, hi = t.nhalo;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t.off[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int tile_global(const TileSmem &t, int k) {
    const int h = tile_cell(t, k);
    return t.start[h] + (k - t.off[h]);
}

// Brick centre and the axes to centre while staging (CENTER bits not already wrap-free).
struct Centre {
    double c[3];
    int mask;
};

__device__ __forceinline__ Centre brick_centre(const BrickInfo &bi) {
    Centre ce;
    ce.mask = ((bi.dims >> CENTER_SHIFT) & 7) & ~((bi.dims >> MI_FREE_SHIFT) & 7);
    for (int a = 0; a < 3; ++a) ce.c[a] = bi.centre[a];
    return ce;
}

__device__ __forceinline__ double4 centred(double4 p, const Centre &ce, const RepParams &P) {
    if (ce.mask & 1) p.x = near_image(p.x, ce.c[0], P.L[0], P.invL[0]);
    if (ce.mask & 2) p.y = near_image(p.y, ce.c[1], P.L[1], P.invL[1]);
    if (ce.mask & 4) p.z = near_image(p.z, ce.c[2], P.L[2], P.invL[2]);
    return p;
}

// The same with the axes fixed at compile time (CM = the centring mask).
template <int CM>
__device__ __forceinline__ double4 centred_t(double4 p, const Centre &ce, const RepParams &P) {
    if (CM & 1) p.x = near_image(p.x, ce.c[0], P.L[0], P.invL[0]);
    if (CM & 2) p.y = near_image(p.y, ce.c[1], P.L[1], P.invL[1]);
    if (CM & 4) p.z = near_image(p.z, ce.c[2], P.L[2], P.invL[2]);
    return p;
}

// Copy the tile's atoms (x, y, z, type) into LDS as double4 records: blockDim / 64
// consecutive threads copy one halo cell's atoms (consecutive in memory). The coordinates
// on the axes in CM are moved to their image nearest the brick centre.
template <int CM = 0>
__device__ __forceinline__ void tile_stage(const TileSmem &t, const double4 *pos, double4 *st,
                                           const Centre *ce = nullptr,
                                           const RepParams *P = nullptr) {
    const int per = blockDim.x >= 64 ? (int)blockDim.x / 64 : 1;
    const int sub = threadIdx.x % per;
    for (int h = threadIdx.x / per; h < t.nhalo; h += (int)blockDim.x / per) {
        const int o = t.off[h];
        const int m = t.off[h + 1] - o;
        const double4 *src = pos + t.start[h];
        // four loads in flight per thread before the LDS stores (an index past the cell
        // reads its first atom, k0 < m, and is not stored)
        for (int k0 = sub; k0 < m; k0 += 4 * per) {
            const int k1 = k0 + per, k2 = k0 + 2 * per, k3 = k0 + 3 * per;
            double4 p0 = src[k0];
            double4 p1 = src[k1 < m ? k1 : k0];
            double4 p2 = src[k2 < m ? k2 : k0];
            double4 p3 = src[k3 < m ? k3 : k0];
            if (CM) {
                p0 = centred_t<CM>(p0, *ce, *P);
                p1 = centred_t<CM>(p1, *ce, *P);
                p2 = centred_t<CM>(p2, *ce, *P);
                p3 = centred_t<CM>(p3, *ce, *P);
            }
            st[o + k0] = p0;
            if (k1 < m) st[o + k1] = p1;
            if (k2 < m) st[o + k2] = p2;
            if (k3 < m) st[o + k3] = p3;
        }
    }
    __syncthreads();
}

// Load a brick's tile offsets from the table written by the list build.
__device__ __forceinline__ void tile_load(const int *tab, TileSmem &t) {
    for (int k = threadIdx.x; k < TILE_TAB; k += blockDim.x) {
        const int v = tab[k];
        if (k <= 64) t.off[k] = v;
        else if (k < 129) t.start[k - 65] = v;
        else t.nhalo = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) t.total = t.off[t.nhalo];
    __syncthreads();
}

// Store a brick's tile offsets for the force kernels (after tile_setup).
__device__ __forceinline__ void tile_save(const TileSmem &t, int *tab) {
    for (int k = threadIdx.x; k < TILE_TAB; k += blockDim.x) {
        int v;
        if (k <= 64) v = t.off[k];
        else if (k < 129) v = (k - 65 < t.nhalo) ? t.start[k - 65] : 0;
        else v = t.nhalo;
        tab[k] = v;
    }
}

// A tile capacity or type count outside the kernels' assumptions is refused before launch
// (the LDS carve-up and the pair-table offset are derived from them).
static inline bool lds_args_ok(int tile_cap, int max_ntypes, size_t smem) {
    return tile_cap >= 64 && tile_cap <= TILE_MAX && max_ntypes >= 1 &&
           max_ntypes <= LJMD_MAX_TYPES_DEVICE && smem <= LDS_MAX_BYTES;
}

}  // namespace ljmd
