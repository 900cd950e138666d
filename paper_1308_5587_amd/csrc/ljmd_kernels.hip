// Device kernels of the LJ MD hot path for gfx950 (CDNA4, wave64).
//
// This file is compiled with -ffp-contract=off: every fused multiply-add below is written
// explicitly, and the squared distance that decides list membership and the cutoff is
// formed as (dx*dx + dy*dy) + dz*dz with separate roundings, the operation order that
// defines the neighbour list bit for bit.
//
// Data layout (sorted order: particles grouped by cell; cells grouped into 2 x 2 x 2
// bricks, bricks in Morton order, cells in Morton order inside a brick):
//   pos    double4 (x, y, z, type)        two buffers, the step kernel reads one and
//                                          writes the other
//   vel    double4 (vx, vy, vz, 1/m)
//   img    int4    (image x, y, z, tag)
//   xb     double4 positions at the last list build
//   nlist  uint16 indices into the particle's brick tile (see nl_slot for the layout).
#include "ljmd_internal.h"

namespace ljmd {

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

// Wavefront 0 reads the halo cells (lane h, h < nhalo) and scans their atom counts.
__device__ __forceinline__ void tile_setup(const BrickInfo &bi, const HaloCell *halo_b,
                                           const int *cell_start, TileSmem &t) {
    if (threadIdx.x < 64) {
        const int h = threadIdx.x;
        int cnt = 0;
        if (h < bi.nhalo) {
            const HaloCell hc = halo_b[h];
            const int st = cell_start[hc.rank];
            cnt = cell_start[hc.rank + 1] - st;
            t.start[h] = st;
            t.shift[h] = hc.shift;
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

// ---------------------------------------------------------------- upload (create / set_state)

// Host arrays (tag order) -> device SoA in tag order at slots poff + q, positions wrapped
// into [0, L): k = floor(x / L) whole boxes are removed, then one-box rounding fix-ups.
__global__ void k_upload(const double *__restrict__ pos, const double *__restrict__ vel,
                         const int *__restrict__ type, const double *__restrict__ mass,
                         double4 *pos4, double4 *vel4, int4 *img, int n, double L0, double L1,
                         double L2, int set_vel, int set_img, const int *__restrict__ img_in,
                         int poff) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double Ls[3] = {L0, L1, L2};
    double x[3];
    int im[3];
    for (int a = 0; a < 3; ++a) {
        double v = pos[3 * q + a];
        double L = Ls[a];
        double k = floor(v / L);
        double kl = k * L;
        v = v - kl;
        int m = (int)k;
        if (v >= L) { v = v - L; m += 1; }
        if (v < 0.0) { v = v + L; m -= 1; if (v >= L) { v = 0.0; m += 1; } }
        x[a] = v;
        im[a] = m + (img_in ? img_in[3 * q + a] : 0);
    }
    const int t = type ? type[q] : 0;
    pos4[poff + q] = make_double4(x[0], x[1], x[2], (double)t);
    if (set_vel) {
        double m = mass ? mass[q] : 1.0;
        vel4[poff + q] = make_double4(vel[3 * q], vel[3 * q + 1], vel[3 * q + 2], 1.0 / m);
    }
    if (set_img) img[poff + q] = make_int4(im[0], im[1], im[2], q);
}

hipError_t launch_upload(hipStream_t s, const double *pos, const double *vel, const int *type,
                         const double *mass, double4 *pos4, double4 *vel4, int4 *img, int n,
                         const double L[3], int set_vel, int set_img, const int *img_in,
                         int poff) {
    int b = 256;
    hipLaunchKernelGGL(k_upload, dim3((n + b - 1) / b), dim3(b), 0, s, pos, vel, type, mass,
                       pos4, vel4, img, n, L[0], L[1], L[2], set_vel, set_img, img_in, poff);
    return hipGetLastError();
}

// ---------------------------------------------------------------- kick + drift

// First half of a velocity-Verlet step from stored forces: v += dt/(2m) F, x += dt v,
// wrap, then raise the replica's rebuild request if |x - x_build| (min image) >= skin/2.
__global__ void __launch_bounds__(256) k_kick_drift(const KickDriftArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    bool exceed = false;
    int rep = -1;
    if (q < a.n) {
        rep = a.prep ? a.prep[q] : 0;
        if (rep >= 0 && a.reps[rep].active && !(a.only && !a.only[rep])) {
            const RepParams &P = a.reps[rep];
            if (q == P.poff) a.req[2 * rep + a.cur] = 0;  // the other buffer's request
            double4 x = a.pos_in[q];
            double4 v = a.vel[q];
            const double4 f = a.force[q];
            const double hm = P.half_dt * v.w;
            v.x = __builtin_fma(hm, f.x, v.x);
            v.y = __builtin_fma(hm, f.y, v.y);
            v.z = __builtin_fma(hm, f.z, v.z);
            int4 im = a.img[q];
            const int4 im0 = im;
            x.x = __builtin_fma(P.dt, v.x, x.x);
            x.y = __builtin_fma(P.dt, v.y, x.y);
            x.z = __builtin_fma(P.dt, v.z, x.z);
            wrap_coord(x.x, im.x, P.L[0]);
            wrap_coord(x.y, im.y, P.L[1]);
            wrap_coord(x.z, im.z, P.L[2]);
            a.pos_out[q] = x;
            a.vel[q] = v;
            if (im.x != im0.x || im.y != im0.y || im.z != im0.z) a.img[q] = im;
            const double4 b = a.xb[q];
            const double dx = mi_rint(x.x - b.x, P.L[0], P.invL[0]);
            const double dy = mi_rint(x.y - b.y, P.L[1], P.invL[1]);
            const double dz = mi_rint(x.z - b.z, P.L[2], P.invL[2]);
            exceed = r2_canon(dx, dy, dz) >= P.lim2;
        }
    }
    if (exceed) atomicOr(&a.req[2 * rep + (a.cur ^ 1)], 1);
}

hipError_t launch_kick_drift(hipStream_t s, const KickDriftArgs &a) {
    int b = 256;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.n + b - 1) / b), dim3(b), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- force kernel family

template <int TPP>
__device__ __forceinline__ double lane_sum(double v) {
#pragma unroll
    for (int o = TPP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, TPP);
    return v;
}
template <int TPP>
__device__ __forceinline__ float lane_sum(float v) {
#pragma unroll
    for (int o = TPP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, TPP);
    return v;
}

// Accumulators of one lane. FP64 path: everything double. Mixed path: force in FP32,
// energy and virial in FP64.
template <int PREC>
struct Acc;
template <>
struct Acc<PREC_FP64> {
    double fx = 0, fy = 0, fz = 0;
};
template <>
struct Acc<PREC_MIXED> {
    float fx = 0, fy = 0, fz = 0;
};

// One pair inside the cutoff: add the LJ force on i (and, with ENERGY, half the pair
// energy and virial) for the displacement d = x_j - x_i with r2 = |d|^2.
template <int PREC, bool ENERGY>
__device__ __forceinline__ void pair_term(const PairCoef &c, double dx, double dy, double dz,
                                          double r2, Acc<PREC> &acc, double &ue, double &w0,
                                          double &w1, double &w2, double &w3, double &w4,
                                          double &w5) {
    if (PREC == PREC_FP64) {
        const double r2i = rcp64(r2);
        const double r6i = r2i * r2i * r2i;
        const double ff = r2i * r6i * __builtin_fma(c.lj1, r6i, -c.lj2);
        // force on i is ff * (x_i - x_j) = -ff * d
        acc.fx = __builtin_fma(-ff, dx, acc.fx);
        acc.fy = __builtin_fma(-ff, dy, acc.fy);
        acc.fz = __builtin_fma(-ff, dz, acc.fz);
        if (ENERGY) {
            ue += 0.5 * (r6i * __builtin_fma(c.lj3, r6i, -c.lj4) - c.shift);
            const double hf = 0.5 * ff;
            w0 = __builtin_fma(hf * dx, dx, w0);
            w1 = __builtin_fma(hf * dx, dy, w1);
            w2 = __builtin_fma(hf * dx, dz, w2);
            w3 = __builtin_fma(hf * dy, dy, w3);
            w4 = __builtin_fma(hf * dy, dz, w4);
            w5 = __builtin_fma(hf * dz, dz, w5);
        }
    } else {
        // FP32 pair arithmetic on the exactly formed FP64 displacement
        const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
        const float fr2 = (float)r2;
        const float r2i = __builtin_amdgcn_rcpf(fr2);
        const float r6i = r2i * r2i * r2i;
        const float l1 = (float)c.lj1, l2 = (float)c.lj2;
        const float ff = r2i * r6i * __builtin_fmaf(l1, r6i, -l2);
        acc.fx = __builtin_fmaf(-ff, fdx, acc.fx);
        acc.fy = __builtin_fmaf(-ff, fdy, acc.fy);
        acc.fz = __builtin_fmaf(-ff, fdz, acc.fz);
        if (ENERGY) {
            const float l3 = (float)c.lj3, l4 = (float)c.lj4;
            const float up = r6i * __builtin_fmaf(l3, r6i, -l4);
            ue += 0.5 * ((double)up - c.shift);
            const double hf = 0.5 * (double)ff;
            w0 = __builtin_fma(hf * (double)fdx, (double)fdx, w0);
            w1 = __builtin_fma(hf * (double)fdx, (double)fdy, w1);
            w2 = __builtin_fma(hf * (double)fdx, (double)fdz, w2);
            w3 = __builtin_fma(hf * (double)fdy, (double)fdy, w3);
            w4 = __builtin_fma(hf * (double)fdy, (double)fdz, w4);
            w5 = __builtin_fma(hf * (double)fdz, (double)fdz, w5);
        }
    }
}

// The particle passes of one brick; STAGED selects neighbour positions from the LDS tile
// (plain LDS reads) or, for a tile larger than the LDS allocation, from global memory.
// MIF: bit a set when no pair of the brick can wrap on axis a (the minimum image is skipped
// there; subtracting 0 x L would give the same bits).
template <int PREC, int TPP, int MODE, bool ENERGY, bool MULTI, bool STAGED, int MIF>
__device__ __forceinline__ void force_passes(const ForceArgs &a, const TileSmem &t,
                                             const double4 *__restrict__ st,
                                             const PairCoef *s_pair, const PairCoef &single,
                                             const RepParams &P, const Centre &ce, int rep,
                                             bool last, int first, int natoms) {
    const int per_pass = blockDim.x / TPP;
    const int g = threadIdx.x / TPP;
    const int lane = threadIdx.x & (TPP - 1);
    const double L0 = P.L[0], L1 = P.L[1], L2 = P.L[2];
    const double iL0 = P.invL[0], iL1 = P.invL[1], iL2 = P.invL[2];
    typedef int v4i __attribute__((ext_vector_type(4)));
    const size_t cstride = (size_t)a.npad << a.lshift;  // 16-byte chunks between rounds

    for (int p0 = 0; p0 < natoms; p0 += per_pass) {
        const int p = p0 + g;
        const bool active = p < natoms;
        const int q = first + (active ? (int)a.work[first + p] : 0);
        const double4 xi = a.pos_in[q];
        // the staged tile is centred on the brick: so is the particle in the pair loop
        const double4 xc = STAGED ? centred(xi, ce, P) : xi;
        const int ti = MULTI ? (int)xi.w : 0;
        int cnt = active ? a.nl_count[q] : 0;
        cnt = cnt < a.cap ? cnt : a.cap;

        // the integration state (velocity, build position, images) is read after the pair
        // loop: holding it across the loop would cost 20 registers per lane and occupancy

        Acc<PREC> acc;
        double ue = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0, w5 = 0.0;
        const v4i *row = reinterpret_cast<const v4i *>(a.nlist) + ((size_t)q << a.lshift) + lane;
        int k0 = lane * 8;
        v4i nxt = {0, 0, 0, 0};
        if (k0 < cnt) nxt = __builtin_nontemporal_load(row);
        for (; k0 < cnt; k0 += 8 * TPP) {
            const v4i cur = nxt;
            row += cstride;
            if (k0 + 8 * TPP < cnt) nxt = __builtin_nontemporal_load(row);
            const int e[8] = {cur.x & 0xffff, (cur.x >> 16) & 0xffff, cur.y & 0xffff,
                              (cur.y >> 16) & 0xffff, cur.z & 0xffff, (cur.z >> 16) & 0xffff,
                              cur.w & 0xffff, (cur.w >> 16) & 0xffff};
            // entries in groups of FB: all neighbour positions of the group are requested
            // first, then the arithmetic runs on them
            constexpr int FB = FORCE_BATCH;
#pragma unroll
            for (int u0 = 0; u0 < 8; u0 += FB) {
                double px[FB], py[FB], pz[FB];
                int pt[FB];
                bool pv[FB];
#pragma unroll
                for (int v = 0; v < FB; ++v) {
                    const int u = u0 + v;
                    pv[v] = k0 + u < cnt && e[u] < t.total;
                    const int idx = pv[v] ? e[u] : 0;
                    pt[v] = 0;
                    if (STAGED) {
                        const double4 pj = st[idx];
                        px[v] = pj.x;
                        py[v] = pj.y;
                        pz[v] = pj.z;
                        if (MULTI) pt[v] = (int)pj.w;
                    } else {
                        const double4 pj = a.pos_in[tile_global(t, idx)];
                        px[v] = pj.x;
                        py[v] = pj.y;
                        pz[v] = pj.z;
                        pt[v] = (int)pj.w;
                    }
                }
#pragma unroll
                for (int v = 0; v < FB; ++v) {
                    const double dx = (MIF & 1) ? px[v] - xc.x : mi_rint(px[v] - xc.x, L0, iL0);
                    const double dy = (MIF & 2) ? py[v] - xc.y : mi_rint(py[v] - xc.y, L1, iL1);
                    const double dz = (MIF & 4) ? pz[v] - xc.z : mi_rint(pz[v] - xc.z, L2, iL2);
                    const double r2 = r2_canon(dx, dy, dz);
                    const PairCoef &c = MULTI ? s_pair[ti * P.ntypes + pt[v]] : single;
                    if (pv[v] && r2 < c.rc2)
                        pair_term<PREC, ENERGY>(c, dx, dy, dz, r2, acc, ue, w0, w1, w2, w3, w4, w5);
                }
            }
        }

        double fx, fy, fz;
        if (PREC == PREC_FP64) {
            fx = lane_sum<TPP>((double)acc.fx);
            fy = lane_sum<TPP>((double)acc.fy);
            fz = lane_sum<TPP>((double)acc.fz);
        } else {
            fx = (double)lane_sum<TPP>((float)acc.fx);
            fy = (double)lane_sum<TPP>((float)acc.fy);
            fz = (double)lane_sum<TPP>((float)acc.fz);
        }
        if (ENERGY) {
            ue = lane_sum<TPP>(ue);
            w0 = lane_sum<TPP>(w0);
            w1 = lane_sum<TPP>(w1);
            w2 = lane_sum<TPP>(w2);
            w3 = lane_sum<TPP>(w3);
            w4 = lane_sum<TPP>(w4);
            w5 = lane_sum<TPP>(w5);
        }
        bool exceed = false;
        if (active && lane == 0) {
            const bool finite =
                __builtin_isfinite(fx) && __builtin_isfinite(fy) && __builtin_isfinite(fz);
            if (!finite) {
                atomicOr(a.status, ST_NONFINITE);
                if (a.rep_status) atomicOr(&a.rep_status[rep], ST_NONFINITE);
            }
            if (ENERGY) {
                a.u_out[q] = ue;
                double *w = a.w_out + 6 * (size_t)q;
                w[0] = w0; w[1] = w1; w[2] = w2; w[3] = w3; w[4] = w4; w[5] = w5;
            }
            if (MODE == MODE_EVAL) {
                a.force[q] = make_double4(fx, fy, fz, 0.0);
            } else {
                double4 v = a.vel[q];
                const double hm = P.half_dt * v.w;
                // second half kick of the current step: full-step velocity
                v.x = __builtin_fma(hm, fx, v.x);
                v.y = __builtin_fma(hm, fy, v.y);
                v.z = __builtin_fma(hm, fz, v.z);
                if (MODE == MODE_FINAL || last) {
                    // the replica's last step: no drift; the position stays in place
                    a.vel[q] = v;
                    a.force[q] = make_double4(fx, fy, fz, 0.0);
                    if (MODE == MODE_FUSED) a.pos_out[q] = xi;
                } else {
                    if (ENERGY) {
                        const double m = 1.0 / v.w;
                        a.ke_out[q] = 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z);
                    }
                    // first half kick and drift of the next step
                    v.x = __builtin_fma(hm, fx, v.x);
                    v.y = __builtin_fma(hm, fy, v.y);
                    v.z = __builtin_fma(hm, fz, v.z);
                    double4 x = xi;
                    x.x = __builtin_fma(P.dt, v.x, x.x);
                    x.y = __builtin_fma(P.dt, v.y, x.y);
                    x.z = __builtin_fma(P.dt, v.z, x.z);
                    int4 im = a.img[q];
                    const int4 im0 = im;
                    wrap_coord(x.x, im.x, L0);
                    wrap_coord(x.y, im.y, L1);
                    wrap_coord(x.z, im.z, L2);
                    a.pos_out[q] = x;
                    a.vel[q] = v;
                    if (im.x != im0.x || im.y != im0.y || im.z != im0.z) a.img[q] = im;
                    const double4 b_pre = a.xb[q];
                    const double ex = mi_rint(x.x - b_pre.x, L0, iL0);
                    const double ey = mi_rint(x.y - b_pre.y, L1, iL1);
                    const double ez = mi_rint(x.z - b_pre.z, L2, iL2);
                    exceed = r2_canon(ex, ey, ez) >= P.lim2;
                }
            }
        }
        if (MODE == MODE_FUSED) {
            // all particles of the workgroup belong to one replica: one atomic per wavefront
            const unsigned long long vote = __ballot(exceed);
            if (exceed && (threadIdx.x & 63) == __ffsll((long long)vote) - 1)
                atomicOr(&a.req[2 * rep + (a.cur ^ 1)], 1);
        }
    }
}

// One workgroup per brick. The brick's tile (the atoms of its halo cells, double4 records,
// moved to their image nearest the brick centre on the centred axes) is staged in LDS; TPP
// lanes per particle of the brick stride through the particle's list of 16-bit tile
// indices, 8 per 16-byte load, gathering neighbour positions from LDS. Forces are reduced
// across the lanes with wavefront shuffles; lane 0 then finishes the particle according to
// MODE. If a tile is larger than the replica's own tile capacity (or the LDS allocation),
// the positions are read from global memory through the tile offsets instead, with the
// minimum image on every axis; the capacity is the replica's, so a replica takes the same
// path alone and in a batch.
// Occupancy: a 48 KiB tile lets three 512-thread workgroups share a CU, which needs at most
// 80 VGPRs (6 waves per SIMD); the single-type variants without energy fit that without
// spilling and are held to it, the others keep their natural register count.
template <int PREC, int TPP, int MODE, bool ENERGY, bool MULTI>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu((ENERGY || MULTI || TPP >= 8) ? 1 : 6)))
k_force(const ForceArgs a) {
    extern __shared__ double4 dyn_tile[];
    __shared__ TileSmem t;
    // one system: XCD-contiguous brick ranges share halos in L2. A batch (the only caller
    // with per-replica status words) launches a grid rounded up past its live bricks, so
    // contiguous ranges would leave the XCDs of the tail idle: consecutive bricks go to
    // different XCDs there (the dispatcher's round robin)
    const int b = a.rep_status ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const BrickInfo bi = a.bricks[b];
    const int rep = bi.rep;
    if (rep < 0) return;
    const RepParams &P = a.reps[rep];
    if (!P.active || (a.only && !a.only[rep])) return;
    // steps left for this replica: >= 2 full step, 1 last step, 0 finished (positions kept)
    int r_in = 2;
    if (MODE == MODE_FUSED) {
        if (a.rem) r_in = a.rem[2 * rep + a.cur];
        if (b == P.boff && threadIdx.x == 0) {
            if (a.rem) a.rem[2 * rep + (a.cur ^ 1)] = r_in > 0 ? r_in - 1 : 0;
            a.req[2 * rep + a.cur] = 0;  // the request for this buffer was served
        }
    }
    const int first = a.cell_start[bi.first_cell];
    const int natoms = a.cell_start[bi.first_cell + bi.ncell] - first;
    if (MODE == MODE_FUSED && r_in <= 0) {
        for (int k = threadIdx.x; k < natoms; k += blockDim.x)
            a.pos_out[first + k] = a.pos_in[first + k];
        return;
    }
    double4 *st = dyn_tile;
    PairCoef *s_pair = reinterpret_cast<PairCoef *>(st + a.tile_cap);
    if (MULTI)
        for (int k = threadIdx.x; k < P.ntypes * P.ntypes; k += blockDim.x)
            s_pair[k] = a.pair[P.pair_off + k];
    const PairCoef single = a.pair[P.pair_off];
    tile_load(a.tile_tab + (size_t)b * TILE_TAB, t);
    const bool staged = t.total <= a.tile_cap && t.total <= P.tile_cap;
    const Centre ce = brick_centre(bi);
    if (staged) {
        switch (ce.mask) {
            case 1: tile_stage<1>(t, a.pos_in, st, &ce, &P); break;
            case 2: tile_stage<2>(t, a.pos_in, st, &ce, &P); break;
            case 3: tile_stage<3>(t, a.pos_in, st, &ce, &P); break;
            case 4: tile_stage<4>(t, a.pos_in, st, &ce, &P); break;
            case 5: tile_stage<5>(t, a.pos_in, st, &ce, &P); break;
            case 6: tile_stage<6>(t, a.pos_in, st, &ce, &P); break;
            case 7: tile_stage<7>(t, a.pos_in, st, &ce, &P); break;
            default: tile_stage(t, a.pos_in, st); break;
        }
    }
    const bool last = MODE == MODE_FUSED && r_in == 1;
    // axes on which the pair loop takes the plain difference: wrap-free or centred (the
    // variants that still take the minimum image there get k = 0 and the same bits)
    const int mif = ((bi.dims >> MI_FREE_SHIFT) | (bi.dims >> CENTER_SHIFT)) & 7;
#define LJMD_PASSES(M) \
    force_passes<PREC, TPP, MODE, ENERGY, MULTI, true, M>(a, t, st, s_pair, single, P, ce, rep, last, first, natoms)
    if (!staged) {
        force_passes<PREC, TPP, MODE, ENERGY, MULTI, false, 0>(
            a, t, st, s_pair, single, P, ce, rep, last, first, natoms);
    } else if (MODE == MODE_FUSED) {
        // the step kernel: a variant per set of wrap-free axes
        switch (mif) {
            case 7: LJMD_PASSES(7); break;
            case 6: LJMD_PASSES(6); break;
            case 5: LJMD_PASSES(5); break;
            case 3: LJMD_PASSES(3); break;
            case 4: LJMD_PASSES(4); break;
            case 2: LJMD_PASSES(2); break;
            case 1: LJMD_PASSES(1); break;
            default: LJMD_PASSES(0); break;
        }
    } else if (mif == 7) {
        LJMD_PASSES(7);
    } else {
        LJMD_PASSES(0);
    }
#undef LJMD_PASSES
}

// A tile capacity or type count outside the kernels' assumptions is refused before launch
// (the LDS carve-up and the pair-table offset are derived from them).
static bool lds_args_ok(int tile_cap, int max_ntypes, size_t smem) {
    return tile_cap >= 64 && tile_cap <= TILE_MAX && max_ntypes >= 1 &&
           max_ntypes <= LJMD_MAX_TYPES_DEVICE && smem <= LDS_MAX_BYTES;
}

template <int PREC, int TPP, int MODE, bool ENERGY>
static hipError_t launch_force_t(hipStream_t s, const ForceArgs &a, int block) {
    const size_t smem = force_lds_bytes(a.tile_cap, a.max_ntypes);
    if (!lds_args_ok(a.tile_cap, a.max_ntypes, smem)) return hipErrorInvalidValue;
    if (a.max_ntypes > 1)
        hipLaunchKernelGGL((k_force<PREC, TPP, MODE, ENERGY, true>), dim3(a.nbrick), dim3(block),
                           smem, s, a);
    else
        hipLaunchKernelGGL((k_force<PREC, TPP, MODE, ENERGY, false>), dim3(a.nbrick), dim3(block),
                           smem, s, a);
    return hipGetLastError();
}

template <int PREC, int TPP>
static hipError_t launch_force_m(hipStream_t s, const ForceArgs &a, int mode, bool energy,
                                 int block) {
    switch (mode) {
        case MODE_EVAL:
            return energy ? launch_force_t<PREC, TPP, MODE_EVAL, true>(s, a, block)
                          : launch_force_t<PREC, TPP, MODE_EVAL, false>(s, a, block);
        case MODE_FUSED:
            return energy ? launch_force_t<PREC, TPP, MODE_FUSED, true>(s, a, block)
                          : launch_force_t<PREC, TPP, MODE_FUSED, false>(s, a, block);
        default:
            return launch_force_t<PREC, TPP, MODE_FINAL, false>(s, a, block);
    }
}

template <int PREC>
static hipError_t launch_force_p(hipStream_t s, const ForceArgs &a, int tpp, int mode,
                                 bool energy, int block) {
    switch (tpp) {
        case 1: return launch_force_m<PREC, 1>(s, a, mode, energy, block);
        case 2: return launch_force_m<PREC, 2>(s, a, mode, energy, block);
        case 4: return launch_force_m<PREC, 4>(s, a, mode, energy, block);
        case 8: return launch_force_m<PREC, 8>(s, a, mode, energy, block);
        case 16: return launch_force_m<PREC, 16>(s, a, mode, energy, block);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_force(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                        bool energy, int block) {
    if (block < 64 || block > 512 || (block & 63)) return hipErrorInvalidValue;
    return prec == PREC_MIXED ? launch_force_p<PREC_MIXED>(s, a, tpp, mode, energy, block)
                              : launch_force_p<PREC_FP64>(s, a, tpp, mode, energy, block);
}

// ---------------------------------------------------------------- rebuild: cell binning

// Cell coordinate of a scaled position, clamped into [0, nc - 1] (also for a NaN, which
// fails the comparison and lands in cell 0).
__device__ __forceinline__ int cell_coord(double f, int nc) {
    return f > 0.0 ? (int)fmin(f, (double)(nc - 1)) : 0;
}

// Replica of particle q / cell c and whether it takes part in this rebuild.
__device__ __forceinline__ bool rebuilds(const RebuildArgs &a, int rep) {
    return rep >= 0 && a.reps[rep].active && a.go[rep * a.go_stride] != 0;
}

// Cell of each particle; the slot inside its cell comes from an integer atomic counter
// (the order is made deterministic afterwards by k_cell_gather). Particles are still in the
// previous build's cell order, so equal cells come in runs along a wavefront: each run
// takes its slots with one atomic add by its first lane.
__global__ void __launch_bounds__(256) k_bin(const RebuildArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int wl = threadIdx.x & 63;
    int r = -1;
    if (q < a.n) {
        const int rep = a.prep ? a.prep[q] : 0;
        if (rebuilds(a, rep)) {
            const RepParams &P = a.reps[rep];
            const double4 x = a.pos[q];
            const int cx = cell_coord(x.x * P.inv_w[0], P.nc[0]);
            const int cy = cell_coord(x.y * P.inv_w[1], P.nc[1]);
            const int cz = cell_coord(x.z * P.inv_w[2], P.nc[2]);
            r = a.cell_rank[P.coff + (cx * P.nc[1] + cy) * P.nc[2] + cz];
        }
    }
    const int prev = __shfl_up(r, 1);
    const bool head = (wl == 0) || (r != prev);
    const unsigned long long heads = __ballot(head);
    const unsigned long long le = (wl == 63) ? ~0ull : ((2ull << wl) - 1ull);
    const int leader = 63 - __clzll(heads & le);
    const unsigned long long after = heads & ~le;
    const int next = after ? (__ffsll((long long)after) - 1) : 64;
    int base = 0;
    if (head && r >= 0) base = atomicAdd(&a.cell_count[r], next - wl);
    base = __shfl(base, leader);
    if (r >= 0) {
        a.key[q] = r;
        a.slot[q] = base + (wl - leader);
    }
}

// Exclusive scan of a replica's cell counts into cell_start[coff .. coff + ncell], starting
// at its first particle slot. One workgroup of 1024 threads per replica, in tiles of
// SCAN_TILE counts staged through LDS with coalesced loads; the counts are zeroed for the
// next build.
__global__ void __launch_bounds__(1024) k_scan(const RebuildArgs a) {
    const int rep = blockIdx.x;
    if (!rebuilds(a, rep)) return;
    const RepParams &P = a.reps[rep];
    __shared__ int s_val[SCAN_TILE];
    __shared__ int s_sum[1024];
    __shared__ int s_carry;
    const int T = blockDim.x;
    const int t = threadIdx.x;
    constexpr int PER = SCAN_TILE / 1024;
    if (t == 0) {
        s_carry = P.poff;
        if (rep == 0) a.st->entries = 0ull;
    }
    int *cs = a.cell_start + P.coff;
    int *cc = a.cell_count + P.coff;
    for (int base = 0; base < P.ncell; base += SCAN_TILE) {
        const int len = min(SCAN_TILE, P.ncell - base);
        for (int u = t; u < SCAN_TILE; u += T) {
            int v = 0;
            if (u < len) {
                v = cc[base + u];
                cc[base + u] = 0;
            }
            s_val[u] = v;
        }
        __syncthreads();
        int sum = 0;
        for (int u = 0; u < PER; ++u) sum += s_val[t * PER + u];
        s_sum[t] = sum;
        __syncthreads();
        for (int o = 1; o < T; o <<= 1) {
            const int v = t >= o ? s_sum[t - o] : 0;
            __syncthreads();
            s_sum[t] += v;
            __syncthreads();
        }
        int run = s_carry + s_sum[t] - sum;
        for (int u = 0; u < PER; ++u) {
            const int k = s_val[t * PER + u];
            s_val[t * PER + u] = run;
            run += k;
        }
        __syncthreads();
        for (int u = t; u < len; u += T) cs[base + u] = s_val[u];
        __syncthreads();
        if (t == T - 1) s_carry += s_sum[T - 1];
        __syncthreads();
    }
    if (t == 0) cs[P.ncell] = s_carry;
}

__global__ void __launch_bounds__(256) k_scatter(const RebuildArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    if (!rebuilds(a, a.prep ? a.prep[q] : 0)) return;
    a.perm[a.cell_start[a.key[q]] + a.slot[q]] = q;
}

// Order each cell's members by their previous sorted index (a stable counting sort) and
// gather their state into the new order. One workgroup of 64 lanes per cell (grid-stride);
// the rank of a member is the number of members with a smaller index.
__device__ __forceinline__ void gather_member(const RebuildArgs &a, int dst, int k) {
    a.pos_scr[dst] = a.pos[k];
    a.vel_scr[dst] = a.vel[k];
    a.img_scr[dst] = a.img[k];
}

__global__ void __launch_bounds__(64) k_cell_gather(const RebuildArgs a) {
    __shared__ int s_in[SORT_LDS];
    for (int c = blockIdx.x; c < a.ncell; c += gridDim.x) {
        if (!rebuilds(a, a.crep ? a.crep[c] : 0)) continue;  // uniform per workgroup
        const int beg = a.cell_start[c];
        const int m = a.cell_start[c + 1] - beg;
        __syncthreads();  // s_in of the previous cell is no longer read
        if (m <= SORT_LDS) {
            for (int t = threadIdx.x; t < m; t += blockDim.x) s_in[t] = a.perm[beg + t];
            __syncthreads();
            for (int t = threadIdx.x; t < m; t += blockDim.x) {
                const int v = s_in[t];
                int rank = 0;
                for (int u = 0; u < m; ++u) rank += s_in[u] < v;
                gather_member(a, beg + rank, v);
            }
        } else {
            if (threadIdx.x == 0) {
                // pathological occupancy: insertion sort in place by one lane
                for (int t = 1; t < m; ++t) {
                    const int v = a.perm[beg + t];
                    int u = t - 1;
                    while (u >= 0 && a.perm[beg + u] > v) {
                        a.perm[beg + u + 1] = a.perm[beg + u];
                        --u;
                    }
                    a.perm[beg + u + 1] = v;
                }
            }
            __syncthreads();
            for (int t = threadIdx.x; t < m; t += blockDim.x)
                gather_member(a, beg + t, a.perm[beg + t]);
        }
    }
}

// ---------------------------------------------------------------- rebuild: Verlet list

// Candidates of one stencil cell for the particles of a wavefront's groups: each group of
// Ln lanes takes Ln atoms of the cell at a time and appends the hits of its particle in
// lane order. MIK selects the minimum-image form, fixed per cell: 0 none (the halo cell is
// in the primary image), 1 a constant shift of the halo cell's periodic image, 2 the branch
// form (fewer than 3 cells on some axis).
template <bool MULTI, bool STAGED, int MIK, bool SOLO>
__device__ __forceinline__ void nlist_scan_cell(const RebuildArgs &a,
                                                const double4 *__restrict__ st,
                                                const double *s_rl2, const RepParams &P, int o,
                                                int m, int jst, double shx, double shy,
                                                double shz, const double4 &xi, int ti, int q,
                                                bool active, int Ln, int lane,
                                                unsigned long long gmask, int &count) {
    // list slots (nl_slot in closed form with the particle's part precomputed)
    const int sh = 3 + a.lshift;
    // the round stride npad << sh fits 32 bits (the host keeps npad x 8 x lanes < 2^32), so
    // the slot is one 32 x 32 + 64-bit multiply-add
    const uint32_t rstride = (uint32_t)a.npad << sh;
    const uint64_t qbase = (uint64_t)q << sh;
    // BUILD_BATCH rounds of Ln candidates per iteration: their positions are read and their
    // distances tested before any append, so the LDS reads and FP64 chains of the rounds
    // overlap; the appends then run round by round, in the order of a plain loop
    for (int t0 = 0; t0 < m; t0 += Ln * BUILD_BATCH) {
        bool hv[BUILD_BATCH];
        int ttv[BUILD_BATCH];
#pragma unroll
        for (int u = 0; u < BUILD_BATCH; ++u) {
            const int tt = t0 + u * Ln + lane;
            const bool valid = active && tt < m;
            const int tv = valid ? tt : 0;
            double xjx, xjy, xjz;
            int tj = 0;
            if (STAGED) {
                const double4 pj = st[o + tv];
                xjx = pj.x;
                xjy = pj.y;
                xjz = pj.z;
                if (MULTI) tj = (int)pj.w;
            } else {
                const double4 pj = a.pos_scr[jst + tv];
                xjx = pj.x;
                xjy = pj.y;
                xjz = pj.z;
                tj = (int)pj.w;
            }
            double dx = xjx - xi.x, dy = xjy - xi.y, dz = xjz - xi.z;
            if (MIK == 2) {
                dx = mi_branch(dx, P.L[0]);
                dy = mi_branch(dy, P.L[1]);
                dz = mi_branch(dz, P.L[2]);
            } else if (MIK == 1) {
                dx = dx + shx;  // adding 0.0 on an unshifted axis is exact
                dy = dy + shy;
                dz = dz + shz;
            }
            const double r2 = r2_canon(dx, dy, dz);
            const double rl2 = MULTI ? s_rl2[ti * P.ntypes + tj] : P.single_rl2;
            hv[u] = valid && (jst + tt) != q && r2 < rl2;
            ttv[u] = tt;
        }
#pragma unroll
        for (int u = 0; u < BUILD_BATCH; ++u) {
            const bool hit = hv[u];
            if (SOLO) {
                // one lane per particle: its hits are appended in order, no group prefix
                if (hit) {
                    if (count < a.cap) {
                        const uint64_t slot = (uint64_t)((uint32_t)count >> sh) * rstride +
                                              qbase + (size_t)(count & ((1 << sh) - 1));
                        a.nlist[slot] = (uint16_t)(o + ttv[u]);
                    }
                    ++count;
                }
                continue;
            }
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(hit) & gmask;
            if (hit) {
                // hits of lower lanes of the group: mbcnt counts the set bits of bal below
                // this lane
                const int k = count + (int)__builtin_amdgcn_mbcnt_hi(
                                          (unsigned)(bal >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                if (k < a.cap) {
                    const uint64_t slot = (uint64_t)((uint32_t)k >> sh) * rstride + qbase +
                                          (size_t)(k & ((1 << sh) - 1));
                    a.nlist[slot] = (uint16_t)(o + ttv[u]);
                }
            }
            count += __popcll(bal);
        }
    }
}

// The minimum-image form of a stencil cell: branch form for small boxes, else the halo cell's
// shift code (21: no shift on any axis).
template <bool MULTI, bool STAGED, bool SOLO>
__device__ __forceinline__ void nlist_scan_dispatch(const RebuildArgs &a,
                                                    const double4 *__restrict__ st,
                                                    const double *s_rl2, const RepParams &P,
                                                    int o, int m, int jst, int code,
                                                    const double4 &xi, int ti, int q, bool active,
                                                    int Ln, int lane, unsigned long long gmask,
                                                    int &count) {
    if (P.canonical) {
        nlist_scan_cell<MULTI, STAGED, 2, SOLO>(a, st, s_rl2, P, o, m, jst, 0.0, 0.0, 0.0, xi, ti,
                                                q, active, Ln, lane, gmask, count);
    } else if (code != 21) {
        const double shx = (double)((code & 3) - 1) * P.L[0];
        const double shy = (double)(((code >> 2) & 3) - 1) * P.L[1];
        const double shz = (double)(((code >> 4) & 3) - 1) * P.L[2];
        nlist_scan_cell<MULTI, STAGED, 1, SOLO>(a, st, s_rl2, P, o, m, jst, shx, shy, shz, xi, ti,
                                                q, active, Ln, lane, gmask, count);
    } else {
        nlist_scan_cell<MULTI, STAGED, 0, SOLO>(a, st, s_rl2, P, o, m, jst, 0.0, 0.0, 0.0, xi, ti,
                                                q, active, Ln, lane, gmask, count);
    }
}

// The cells of one brick, one wavefront per cell; STAGED selects candidate positions from
// the LDS tile or, for a tile larger than the LDS allocation, from global memory.
template <bool MULTI, bool STAGED>
__device__ __forceinline__ void nlist_cells(const RebuildArgs &a, const TileSmem &t,
                                            const BrickInfo &bi, const double4 *__restrict__ st,
                                            const double *s_rl2, const RepParams &P,
                                            int first, uint16_t *s_cnt, int &my_max,
                                            unsigned long long &my_entries) {
    const int hy = (bi.dims >> 4) & 15, hz = (bi.dims >> 8) & 15;
    const int fpk = a.cell_xyz[bi.first_cell];
    const int wl = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int nst = P.canonical ? t.nhalo : 27;
    for (int ci = wave; ci < bi.ncell; ci += nwave) {
        const int rank = bi.first_cell + ci;
        const int pk = a.cell_xyz[rank];
        const int lx = (pk & 1023) - (fpk & 1023);
        const int ly = ((pk >> 10) & 1023) - ((fpk >> 10) & 1023);
        const int lz = ((pk >> 20) & 1023) - ((fpk >> 20) & 1023);
        const int beg = __builtin_amdgcn_readfirstlane(a.cell_start[rank]);
        const int cnt = __builtin_amdgcn_readfirstlane(a.cell_start[rank + 1]) - beg;
        if (cnt == 0) continue;
        int Ln = 64 / cnt;
        Ln = Ln < 1 ? 1 : (Ln > 32 ? 32 : Ln);
        const int G = 64 / Ln;
        const int group = wl / Ln;
        const int lane = wl - group * Ln;
        const unsigned long long gmask =
            group < G ? (((1ull << Ln) - 1ull) << (group * Ln)) : 0ull;
        for (int p0 = 0; p0 < cnt; p0 += G) {
            const int p = p0 + group;
            const bool active = group < G && p < cnt;
            const int q = beg + (active ? p : 0);
            const double4 xi = a.pos_scr[q];
            const int ti = MULTI ? (int)xi.w : 0;
            int count = 0;
            for (int s = 0; s < nst; ++s) {
                const int h = P.canonical
                                  ? s
                                  : ((lx + s / 9) * hy + (ly + (s / 3) % 3)) * hz + (lz + s % 3);
                // the stencil cell is the same for every lane of the wavefront: keep its
                // bounds in scalar registers (uniform loop control, no per-lane masks)
                const int o = __builtin_amdgcn_readfirstlane(t.off[h]);
                const int m = __builtin_amdgcn_readfirstlane(t.off[h + 1]) - o;
                const int jst = __builtin_amdgcn_readfirstlane(t.start[h]);
                const int code = __builtin_amdgcn_readfirstlane(t.shift[h]);
                if (Ln == 1)
                    nlist_scan_dispatch<MULTI, STAGED, true>(a, st, s_rl2, P, o, m, jst, code, xi,
                                                             ti, q, active, Ln, lane, gmask, count);
                else
                    nlist_scan_dispatch<MULTI, STAGED, false>(a, st, s_rl2, P, o, m, jst, code, xi,
                                                              ti, q, active, Ln, lane, gmask, count);
            }
            if (active && lane == 0) {
                a.nl_count[q] = count;
                if (q - first < WORK_SORT_MAX) s_cnt[q - first] = (uint16_t)(count < 65535 ? count : 65535);
                if (count > a.cap) {
                    atomicOr(&a.st->status, ST_OVERFLOW);
                    if (a.rep_status) atomicOr(&a.rep_status[bi.rep], ST_OVERFLOW);
                }
                my_max = count > my_max ? count : my_max;
                my_entries += (unsigned long long)(count < a.cap ? count : a.cap);
            }
        }
    }
}

// One workgroup per brick: the brick's tile (its halo cells' atoms at the new sorted order)
// is staged in LDS, then each wavefront takes the brick's cells in turn. A cell's particles
// are split into groups of L lanes, L = 64 / (particles in the cell) clamped to [1, 32],
// so nearly every lane has work. Each group walks the atoms of the particle's 27 stencil
// cells (the brick's distinct halo cells when an axis has fewer than 3 cells) L at a time,
// reading them from LDS (all groups read the same atoms at once), and appends the tile index
// of every j != i with r^2 < (r_cut + skin)^2. Appends of one group are compacted with a
// wavefront ballot, so the entry order (stencil cell, then index) is deterministic. The
// workgroup also copies its particles' permuted state back into the main arrays and records
// the build positions.
//
// Distances: for an axis with at least 3 cells the periodic image of a halo cell is known,
// and fl(fl(x_j - x_i) + s) with s in {-L, 0, L} equals the branch-form minimum image bit
// for bit for every pair that can be listed; unshifted halo cells need no addition at all.
// With fewer than 3 cells on some axis the branch form is applied directly.
// Order in which the force kernels take a brick's particles: by decreasing number of
// 8-entry list chunks (a counting sort on LDS bins), so that the particles sharing a wavefront
// have lists of similar length. Any order gives the same results: a particle's sum does not
// depend on the lanes it runs on.
__device__ __forceinline__ void work_order(const RebuildArgs &a, int first, int natoms,
                                           const uint16_t *s_cnt, int *s_bin) {
    if (natoms > WORK_SORT_MAX) {
        for (int p = threadIdx.x; p < natoms; p += blockDim.x) a.work[first + p] = (uint16_t)p;
        return;
    }
    for (int k = threadIdx.x; k < 256; k += blockDim.x) s_bin[k] = 0;
    __syncthreads();  // also: every count is in s_cnt
    for (int p = threadIdx.x; p < natoms; p += blockDim.x) {
        const int chunks = (s_cnt[p] + 7) >> 3;
        atomicAdd(&s_bin[255 - (chunks < 255 ? chunks : 255)], 1);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // exclusive scan of the 256 bins, 4 per lane
        const int l = threadIdx.x;
        const int v0 = s_bin[4 * l], v1 = s_bin[4 * l + 1], v2 = s_bin[4 * l + 2],
                  v3 = s_bin[4 * l + 3];
        const int tot = v0 + v1 + v2 + v3;
        int inc = tot;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(inc, o);
            if (l >= o) inc += u;
        }
        const int ex = inc - tot;
        s_bin[4 * l] = ex;
        s_bin[4 * l + 1] = ex + v0;
        s_bin[4 * l + 2] = ex + v0 + v1;
        s_bin[4 * l + 3] = ex + v0 + v1 + v2;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < natoms; p += blockDim.x) {
        const int chunks = (s_cnt[p] + 7) >> 3;
        const int at = atomicAdd(&s_bin[255 - (chunks < 255 ? chunks : 255)], 1);
        a.work[first + at] = (uint16_t)p;
    }
}

// Three workgroups of 512 per CU when the tile allows it: registers capped at 80 per lane.
template <bool MULTI>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
k_nlist(const RebuildArgs a) {
    // one system: every brick builds, and XCD-contiguous brick ranges share halos in L2. A
    // batch: only the bricks of replicas that asked for a build do work, and each replica's
    // bricks are contiguous, so consecutive bricks go to different XCDs instead (the
    // dispatcher's round robin) to spread the builders of one step over the whole chip
    const int b = a.nrep > 1 ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    const BrickInfo bi = a.bricks[b];
    if (!rebuilds(a, bi.rep)) return;
    const RepParams &P = a.reps[bi.rep];
    extern __shared__ double4 dyn_tile[];
    __shared__ TileSmem t;
    double4 *st = dyn_tile;
    double *s_rl2 = reinterpret_cast<double *>(st + a.tile_cap);
    if (MULTI)
        for (int k = threadIdx.x; k < P.ntypes * P.ntypes; k += blockDim.x)
            s_rl2[k] = a.rl2_table[P.pair_off + k];
    if (b == P.boff && threadIdx.x == 0) atomicAdd(&a.st->builds, 1ull);
    tile_setup(bi, a.halo + (size_t)b * HALO_MAX, a.cell_start, t);
    tile_save(t, a.tile_tab + (size_t)b * TILE_TAB);
    // the permuted state of the brick's particles becomes the main state and the new build
    // point (coalesced copy; tile staging below reads pos_scr, not pos)
    {
        const int first = a.cell_start[bi.first_cell];
        const int last = a.cell_start[bi.first_cell + bi.ncell];
        for (int q = first + (int)threadIdx.x; q < last; q += blockDim.x) {
            const double4 x = a.pos_scr[q];
            a.pos[q] = x;
            a.xb[q] = x;
            a.vel[q] = a.vel_scr[q];
            a.img[q] = a.img_scr[q];
        }
        if (t.total > TILE_INDEX_MAX) {
            // 16-bit tile indices cannot address this tile: no list for the brick
            for (int q = first + (int)threadIdx.x; q < last; q += blockDim.x) {
                a.nl_count[q] = 0;
                a.work[q] = (uint16_t)(q - first);
            }
            if (threadIdx.x == 0) {
                atomicOr(&a.st->status, ST_TILE);
                if (a.rep_status) atomicOr(&a.rep_status[bi.rep], ST_TILE);
            }
            return;
        }
    }
    const bool staged = t.total <= a.tile_cap;
    if (staged) tile_stage(t, a.pos_scr, st);

    const int wl = threadIdx.x & 63;
    int my_max = 0;
    unsigned long long my_entries = 0ull;
    __shared__ uint16_t s_cnt[WORK_SORT_MAX];
    __shared__ int s_bin[256];
    const int first = a.cell_start[bi.first_cell];
    const int natoms = a.cell_start[bi.first_cell + bi.ncell] - first;
    if (staged)
        nlist_cells<MULTI, true>(a, t, bi, st, s_rl2, P, first, s_cnt, my_max, my_entries);
    else
        nlist_cells<MULTI, false>(a, t, bi, st, s_rl2, P, first, s_cnt, my_max, my_entries);
    work_order(a, first, natoms, s_cnt, s_bin);

    // wavefront reductions of the build statistics, one atomic each per wavefront
    for (int o = 32; o > 0; o >>= 1) {
        const int om = __shfl_xor(my_max, o);
        my_max = om > my_max ? om : my_max;
        my_entries += __shfl_xor(my_entries, o);
    }
    if (wl == 0 && my_max > 0) {
        atomicMax(&a.st->max_count, my_max);
        atomicAdd(&a.st->entries, my_entries);
    }
}

// Global indices of every list entry (for inspection): out[q * cap + k].
__global__ void __launch_bounds__(256) k_decode_list(const RebuildArgs a, int *out) {
    __shared__ TileSmem t;
    const BrickInfo bi = a.bricks[blockIdx.x];
    if (bi.rep < 0 || !a.reps[bi.rep].active) return;
    tile_setup(bi, a.halo + (size_t)blockIdx.x * HALO_MAX, a.cell_start, t);
    const int first = a.cell_start[bi.first_cell];
    const int natoms = a.cell_start[bi.first_cell + bi.ncell] - first;
    for (int p = threadIdx.x; p < natoms; p += blockDim.x) {
        const int q = first + p;
        int cnt = a.nl_count[q];
        cnt = cnt < a.cap ? cnt : a.cap;
        for (int k = 0; k < cnt; ++k)
            out[(size_t)q * a.cap + k] = tile_global(t, a.nlist[nl_slot(q, k, a.npad, a.lshift)]);
    }
}

hipError_t launch_decode_list(hipStream_t s, const RebuildArgs &a, int *out) {
    hipLaunchKernelGGL(k_decode_list, dim3(a.nbrick), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_rebuild(hipStream_t s, const RebuildArgs &a) {
    if (!lds_args_ok(a.tile_cap, a.max_ntypes, nlist_lds_bytes(a.tile_cap, a.max_ntypes)))
        return hipErrorInvalidValue;
    const int b = 256;
    const int g = (a.n + b - 1) / b;
    hipLaunchKernelGGL(k_bin, dim3(g), dim3(b), 0, s, a);
    hipLaunchKernelGGL(k_scan, dim3(a.nrep), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(b), 0, s, a);
    hipLaunchKernelGGL(k_cell_gather, dim3(a.ncell < 8192 ? a.ncell : 8192), dim3(64), 0, s, a);
    const size_t smem = nlist_lds_bytes(a.tile_cap, a.max_ntypes);
    if (a.max_ntypes > 1)
        hipLaunchKernelGGL(k_nlist<true>, dim3(a.nbrick), dim3(512), smem, s, a);
    else
        hipLaunchKernelGGL(k_nlist<false>, dim3(a.nbrick), dim3(512), smem, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions

// Deterministic FP64 sums of U, W[6] and K over particles [poff, poff + n): each workgroup
// adds a fixed strided subset in a fixed order and tree-reduces it in LDS; one workgroup
// then reduces the partials the same way. K is taken from ke[] when given, else from the
// stored velocities.
__global__ void __launch_bounds__(RED_BLOCK) k_reduce_partials(const double *u, const double *w,
                                                                const double *ke,
                                                                const double4 *vel, int poff,
                                                                int n, double *partials) {
    __shared__ double s[RED_QUANT][RED_BLOCK];
    double acc[RED_QUANT];
    for (int c = 0; c < RED_QUANT; ++c) acc[c] = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const size_t q = (size_t)poff + k;
        acc[0] += u[q];
        for (int c = 0; c < 6; ++c) acc[1 + c] += w[6 * q + c];
        if (ke) {
            acc[7] += ke[q];
        } else {
            const double4 v = vel[q];
            const double m = 1.0 / v.w;
            acc[7] += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z);
        }
    }
    for (int c = 0; c < RED_QUANT; ++c) s[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = RED_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < RED_QUANT; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < RED_QUANT; ++c) partials[RED_QUANT * blockIdx.x + c] = s[c][0];
}

__global__ void __launch_bounds__(RED_BLOCK) k_reduce_final(const double *partials, int np,
                                                             double *out) {
    __shared__ double s[RED_QUANT][RED_BLOCK];
    double acc[RED_QUANT];
    for (int c = 0; c < RED_QUANT; ++c) acc[c] = 0.0;
    for (int p = threadIdx.x; p < np; p += blockDim.x)
        for (int c = 0; c < RED_QUANT; ++c) acc[c] += partials[RED_QUANT * p + c];
    for (int c = 0; c < RED_QUANT; ++c) s[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = RED_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int c = 0; c < RED_QUANT; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < RED_QUANT; ++c) out[c] = s[c][0];
}

hipError_t launch_reduce(hipStream_t s, const double *u, const double *w, const double *ke,
                         const double4 *vel, int poff, int n, double *partials, int nblocks_max,
                         double *out) {
    int g = (n + RED_BLOCK - 1) / RED_BLOCK;
    if (g > nblocks_max) g = nblocks_max;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_reduce_partials, dim3(g), dim3(RED_BLOCK), 0, s, u, w, ke, vel, poff, n,
                       partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_BLOCK), 0, s, partials, g, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- outputs in tag order

// Particles [poff, poff + n) hold tags 0 .. n-1 (in img.w); outputs are written by tag.
__global__ void k_unsort_vec(const double4 *src, const int4 *img, int poff, int n, double *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double4 v = src[poff + k];
    const int t = img[poff + k].w;
    dst[3 * (size_t)t] = v.x;
    dst[3 * (size_t)t + 1] = v.y;
    dst[3 * (size_t)t + 2] = v.z;
}

__global__ void k_unsort_img(const int4 *img, int poff, int n, int *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int4 v = img[poff + k];
    dst[3 * (size_t)v.w] = v.x;
    dst[3 * (size_t)v.w + 1] = v.y;
    dst[3 * (size_t)v.w + 2] = v.z;
}

__global__ void k_unsort_scalar(const double *src, int width, const int4 *img, int poff, int n,
                                double *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int t = img[poff + k].w;
    for (int c = 0; c < width; ++c)
        dst[(size_t)width * t + c] = src[(size_t)width * (poff + k) + c];
}

hipError_t launch_unsort_vec(hipStream_t s, const double4 *src, const int4 *img, int poff, int n,
                             double *dst) {
    hipLaunchKernelGGL(k_unsort_vec, dim3((n + 255) / 256), dim3(256), 0, s, src, img, poff, n,
                       dst);
    return hipGetLastError();
}

hipError_t launch_unsort_img(hipStream_t s, const int4 *img, int poff, int n, int *dst) {
    hipLaunchKernelGGL(k_unsort_img, dim3((n + 255) / 256), dim3(256), 0, s, img, poff, n, dst);
    return hipGetLastError();
}

hipError_t launch_unsort_scalar(hipStream_t s, const double *src, int width, const int4 *img,
                                int poff, int n, double *dst) {
    hipLaunchKernelGGL(k_unsort_scalar, dim3((n + 255) / 256), dim3(256), 0, s, src, width, img,
                       poff, n, dst);
    return hipGetLastError();
}

__global__ void k_fill_status(DevStatus *st) {
    if (threadIdx.x == 0) {
        st->status = 0;
        st->max_count = 0;
        st->builds = 0ull;
        st->entries = 0ull;
        st->pad = 0;
    }
}

hipError_t launch_fill_status(hipStream_t s, DevStatus *st) {
    hipLaunchKernelGGL(k_fill_status, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

__global__ void k_fill_int(int *p, int n, int value) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = value;
}

hipError_t launch_fill_int(hipStream_t s, int *p, int n, int value) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

}  // namespace ljmd
