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
//
// The force kernels themselves are in ljmd_force.h (one translation unit per pair form).
#include "ljmd_device.h"

namespace ljmd {

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
            if (a.scale) {
                // NVT: the thermostat half steps between the last kick and this one
                const double S = a.scale[0] * a.scale[1];
                v.x = S * v.x;
                v.y = S * v.y;
                v.z = S * v.z;
            }
            v.x = __builtin_fma(hm, f.x, v.x);
            v.y = __builtin_fma(hm, f.y, v.y);
            v.z = __builtin_fma(hm, f.z, v.z);
            x.x = __builtin_fma(P.dt, v.x, x.x);
            x.y = __builtin_fma(P.dt, v.y, x.y);
            x.z = __builtin_fma(P.dt, v.z, x.z);
            // the image counters are read and written only where a coordinate wraps
            int4 d = make_int4(0, 0, 0, 0);
            wrap_coord(x.x, d.x, P.L[0]);
            wrap_coord(x.y, d.y, P.L[1]);
            wrap_coord(x.z, d.z, P.L[2]);
            a.pos_out[q] = x;
            a.vel[q] = v;
            if (d.x | d.y | d.z) {
                int4 im = a.img[q];
                im.x += d.x;
                im.y += d.y;
                im.z += d.z;
                a.img[q] = im;
            }
            const double4 b = a.xb[q];
            const double dx = mi_rint(x.x - b.x, P.L[0], P.invL[0]);
            const double dy = mi_rint(x.y - b.y, P.L[1], P.invL[1]);
            const double dz = mi_rint(x.z - b.z, P.L[2], P.invL[2]);
            exceed = r2_canon(dx, dy, dz) >= P.lim2;
        }
    }
    // lanes may belong to different replicas; a plain read first spares the atomic once the
    // request is set (nothing clears it during this kernel)
    if (exceed && __hip_atomic_load(&a.req[2 * rep + (a.cur ^ 1)], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(&a.req[2 * rep + (a.cur ^ 1)], 1);
}

hipError_t launch_kick_drift(hipStream_t s, const KickDriftArgs &a) {
    int b = 256;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.n + b - 1) / b), dim3(b), 0, s, a);
    return hipGetLastError();
}


hipError_t launch_force(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                        bool energy, int block, int style) {
    switch (style) {
        case STYLE_LJ: return launch_force_lj(s, a, prec, tpp, mode, energy, block);
        case STYLE_MIE: return launch_force_mie(s, a, prec, tpp, mode, energy, block);
        case STYLE_GAUSS: return launch_force_gauss(s, a, prec, tpp, mode, energy, block);
        case STYLE_YUKAWA: return launch_force_yukawa(s, a, prec, tpp, mode, energy, block);
        case STYLE_LJ | STYLE_SF: return launch_force_lj_sf(s, a, prec, tpp, mode, energy, block);
        case STYLE_MIE | STYLE_SF:
            return launch_force_mie_sf(s, a, prec, tpp, mode, energy, block);
        case STYLE_GAUSS | STYLE_SF:
            return launch_force_gauss_sf(s, a, prec, tpp, mode, energy, block);
        case STYLE_YUKAWA | STYLE_SF:
            return launch_force_yukawa_sf(s, a, prec, tpp, mode, energy, block);
        default: return hipErrorInvalidValue;
    }
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

// 1 when a particle at z lies in the upper half of its cell cz: the scaled coordinate
// z / w, the value k_bin bins by, is at least cz + 1/2 (exact: the difference of two
// nearby doubles).
__device__ __forceinline__ int upper_half(double z, double inv_w, int cz) {
    return (z * inv_w - (double)cz) >= 0.5 ? 1 : 0;
}

// Cell of each particle; the slot inside its cell comes from an integer atomic counter
// (the order is made deterministic afterwards by k_cell_gather). Particles are still in the
// previous build's cell order, so equal cells come in runs along a wavefront: each run
// takes its slots with one atomic add by its first lane.
__global__ void __launch_bounds__(256) k_bin(const RebuildArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int wl = threadIdx.x & 63;
    int r = -1, up = 0;
    if (q < a.n) {
        const int rep = a.prep ? a.prep[q] : 0;
        if (rebuilds(a, rep)) {
            const RepParams &P = a.reps[rep];
            const double4 x = a.pos[q];
            const int cx = cell_coord(x.x * P.inv_w[0], P.nc[0]);
            const int cy = cell_coord(x.y * P.inv_w[1], P.nc[1]);
            const int cz = cell_coord(x.z * P.inv_w[2], P.nc[2]);
            const int tcell = a.typed_cells ? (int)x.w * a.typed_cells : 0;
            r = a.cell_rank[P.coff + tcell + (cx * P.nc[1] + cy) * P.nc[2] + cz];
            if (LJMD_DEBUG_CHECKS && (r < P.coff || r >= P.coff + P.ncell)) {
                debug_fail(a.st, DBG_CELL);
                r = -1;
            }
            if (a.cell_lo) up = upper_half(x.z, P.inv_w[2], cz);
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
        a.slot[q] = (base + (wl - leader)) | (up << 30);  // the z half rides in bit 30
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
    // perm holds 2 q + (upper z half): particle slots are below 2^26
    const int sl = a.slot[q];
    const int dst = a.cell_start[a.key[q]] + (sl & 0x3FFFFFFF);
    if (LJMD_DEBUG_CHECKS) {
        const RepParams &P = a.reps[a.prep ? a.prep[q] : 0];
        if (dst < P.poff || dst >= P.poff + P.n) {
            debug_fail(a.st, DBG_SCATTER);
            return;
        }
    }
    a.perm[dst] = (q << 1) | (sl >> 30);
}

// Order each cell's members and gather their state into the new order. One workgroup of 64
// lanes per cell (grid-stride). The cell method orders members by (z half, previous sorted
// index): k_bin marks the particles whose scaled z coordinate lies in the upper half of their
// cell, k_scatter carries the mark into perm (2 q + mark), lower-half members come first and
// cell_lo records how many; the list build uses the split to skip, for a particle in one
// half, the far half of the cells above or below it. The tree method's sort grid orders by
// previous index only. The rank of a member is the number of members with a smaller key.
__device__ __forceinline__ void gather_member(const RebuildArgs &a, int dst, int k, int c) {
    a.pos_scr[dst] = a.pos[k];
    a.vel_scr[dst] = a.vel[k];
    a.img_scr[dst] = a.img[k];
    if (a.cell_of) a.cell_of[dst] = c;
}

__global__ void __launch_bounds__(64) k_cell_gather(const RebuildArgs a) {
    __shared__ int s_key[SORT_LDS];
    __shared__ int s_lo;
    for (int c = blockIdx.x; c < a.ncell; c += gridDim.x) {
        if (!rebuilds(a, a.crep ? a.crep[c] : 0)) continue;  // uniform per workgroup
        const int beg = a.cell_start[c];
        const int m = a.cell_start[c + 1] - beg;
        __syncthreads();  // s_key of the previous cell is no longer read
        if (m <= SORT_LDS) {
            if (threadIdx.x == 0) s_lo = 0;
            __syncthreads();
            // the key (half, index) as one int: half in bit 30, the index below 2^26
            for (int t = threadIdx.x; t < m; t += blockDim.x) {
                const int pv = a.perm[beg + t];
                s_key[t] = ((pv & 1) << 30) | (pv >> 1);
                if (!(pv & 1)) atomicAdd(&s_lo, 1);
            }
            __syncthreads();
            for (int t = threadIdx.x; t < m; t += blockDim.x) {
                const int kt = s_key[t];
                int rank = 0;
                for (int u = 0; u < m; ++u) rank += s_key[u] < kt;
                gather_member(a, beg + rank, kt & 0x3FFFFFFF, c);
            }
            if (a.cell_lo && threadIdx.x == 0) a.cell_lo[c] = s_lo;
        } else {
            if (threadIdx.x == 0) {
                // pathological occupancy: insertion sort in place by one lane, on the key
                // (half, index), which orders as the encoded value with the half bit on top
                auto key = [](int pv) { return ((pv & 1) << 30) | (pv >> 1); };
                int lo = 0;
                for (int t = 0; t < m; ++t) lo += !(a.perm[beg + t] & 1);
                for (int t = 1; t < m; ++t) {
                    const int v = a.perm[beg + t];
                    const int kv = key(v);
                    int u = t - 1;
                    while (u >= 0 && key(a.perm[beg + u]) > kv) {
                        a.perm[beg + u + 1] = a.perm[beg + u];
                        --u;
                    }
                    a.perm[beg + u + 1] = v;
                }
                if (a.cell_lo) a.cell_lo[c] = lo;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < m; t += blockDim.x)
                gather_member(a, beg + t, a.perm[beg + t] >> 1, c);
        }
    }
}

// ---------------------------------------------------------------- rebuild: Verlet list

// The replica parameters the list build reads inside its loops, held in scalar registers for
// the whole workgroup: a parameter load in the loops would wait (vmcnt) for every list store
// still in flight.
struct BuildParams {
    double L[3];
    double rl2;  // (r_cut + skin)^2 of pair (0,0)
    int canonical, ntypes;
    int narrow;  // npad < 2^24 and every list slot below 2^31 (byte offsets fit 32 bits)
    int tile_total;  // atoms of the brick's tile (debug checks)
};

__device__ __forceinline__ double uniform_f64(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ BuildParams build_params(const RepParams &P) {
    BuildParams u;
    for (int k = 0; k < 3; ++k) u.L[k] = uniform_f64(P.L[k]);
    u.rl2 = uniform_f64(P.single_rl2);
    u.canonical = __builtin_amdgcn_readfirstlane(P.canonical);
    u.ntypes = __builtin_amdgcn_readfirstlane(P.ntypes);
    return u;
}

// The z shifts of a stencil column whose three cells lie in different periodic images along
// z: the second and third cells start at tile indices b1 and b2.
struct ColumnShift {
    int b1, b2;
    double shz1, shz2;
};

// Writes entry k of particle q's list (nl_slot in closed form with the particle's part
// precomputed). The round stride npad << sh fits 32 bits (the host keeps npad x 8 x lanes
// < 2^32), so the slot is one 32 x 32 + 64-bit multiply-add; for a list of less than 4 GiB
// with npad < 2^24 (narrow) it is a 24-bit multiply and 32-bit byte offsets from the list base.
struct ListWriter {
    uint16_t *nlist;
    uint32_t npad, rstride, qb32, lmask;
    uint64_t qbase, limit;  // limit: slots of the allocation (debug checks)
    int sh, narrow;
    DevStatus *st;
    __device__ __forceinline__ ListWriter(const RebuildArgs &a, const BuildParams &P, int q) {
        nlist = a.nlist;
        st = a.st;
        limit = (uint64_t)a.npad * (uint64_t)a.cap;
        sh = 3 + a.lshift;
        npad = (uint32_t)a.npad;
        rstride = npad << sh;
        qbase = (uint64_t)q << sh;
        qb32 = (uint32_t)q << sh;
        lmask = (1u << sh) - 1u;
        narrow = P.narrow;
    }
    // eight entries 8g .. 8g + 7 of a narrow list (consecutive slots within one chunk,
    // 16-byte aligned)
    __device__ __forceinline__ void store8_narrow(int g, const uint4 &v) const {
        const uint32_t k = (uint32_t)g << 3;
        const uint32_t e = __umul24(k >> sh, npad);
        const uint32_t slot = (e << sh) + qb32 + (k & lmask);
        if (LJMD_DEBUG_CHECKS && slot + 8 > limit) {
            debug_fail(st, DBG_SLOT);
            return;
        }
        *reinterpret_cast<uint4 *>(reinterpret_cast<char *>(nlist) + (slot << 1)) = v;
    }
    __device__ __forceinline__ void operator()(int k, int v) const {
        if (narrow) {
            const uint32_t e = __umul24((uint32_t)k >> sh, npad);
            const uint32_t slot = (e << sh) + qb32 + ((uint32_t)k & lmask);
            if (LJMD_DEBUG_CHECKS && slot >= limit) {
                debug_fail(st, DBG_SLOT);
                return;
            }
            *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(nlist) + (slot << 1)) =
                (uint16_t)v;
        } else {
            const uint64_t slot =
                (uint64_t)((uint32_t)k >> sh) * rstride + qbase + (size_t)((uint32_t)k & lmask);
            if (LJMD_DEBUG_CHECKS && slot >= limit) {
                debug_fail(st, DBG_SLOT);
                return;
            }
            nlist[slot] = (uint16_t)v;
        }
    }
};

// Candidates of one range of tile atoms (a stencil cell, or a column of them) for the
// particles of a wavefront's groups: each group of Ln lanes takes Ln atoms of the range at a
// time and appends the hits of its particle in lane order, so entries follow the tile order.
// MIK selects the minimum-image form, fixed per range: 0 none (the halo cells are in the
// primary image), 1 a constant shift of their periodic image, 2 the branch form (fewer than
// 3 cells on some axis).
template <bool MULTI, bool STAGED, int MIK, bool SOLO>
__device__ __forceinline__ void nlist_scan_cell(const RebuildArgs &a,
                                                const double4 *__restrict__ st,
                                                const double *s_rl2, const BuildParams &P, int o,
                                                int m, int jst, double shx, double shy,
                                                double shz, const ColumnShift &cz,
                                                const double4 &xi, int ti, int q, int self,
                                                bool active, int Ln, int lane,
                                                unsigned long long gmask, int &count) {
    const ListWriter store(a, P, q);
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
            } else if (MIK == 3) {
                // a column whose cells lie in different z images: the z shift of the
                // candidate's own cell (tile index below b1: the first cell, below b2: the
                // second, else the third)
                const int k = o + tv;
                dx = dx + shx;
                dy = dy + shy;
                dz = dz + (k < cz.b1 ? shz : (k < cz.b2 ? cz.shz1 : cz.shz2));
            }
            const double r2 = r2_canon(dx, dy, dz);
            const double rl2 = MULTI ? s_rl2[ti * P.ntypes + tj] : P.rl2;
            // the particle itself: its tile index (staged) or its sorted index
            hv[u] = valid && (STAGED ? o + tt : jst + tt) != self && r2 < rl2;
            ttv[u] = tt;
        }
#pragma unroll
        for (int u = 0; u < BUILD_BATCH; ++u) {
            const bool hit = hv[u];
            if (LJMD_DEBUG_CHECKS && hit && STAGED && o + ttv[u] >= P.tile_total)
                debug_fail(a.st, DBG_TILE);
            if (SOLO) {
                // one lane per particle: its hits are appended in order, no group prefix
                if (hit) {
                    if (count < a.cap) store(count, o + ttv[u]);
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
                if (k < a.cap) store(k, o + ttv[u]);
            }
            count += __popcll(bal);
        }
    }
}

// The minimum-image form of a range: branch form for small boxes, else the halo cells' shift
// code (21: no shift on any axis), or for a column across the box's z boundary the shift
// code of its first cell and the z shifts of the others (cz.b1 >= 0).
template <bool MULTI, bool STAGED, bool SOLO>
__device__ __forceinline__ void nlist_scan_dispatch(const RebuildArgs &a,
                                                    const double4 *__restrict__ st,
                                                    const double *s_rl2, const BuildParams &P,
                                                    int o, int m, int jst, int code,
                                                    const ColumnShift &cz, const double4 &xi,
                                                    int ti, int q, int self, bool active, int Ln,
                                                    int lane, unsigned long long gmask,
                                                    int &count) {
    if (P.canonical) {
        nlist_scan_cell<MULTI, STAGED, 2, SOLO>(a, st, s_rl2, P, o, m, jst, 0.0, 0.0, 0.0, cz, xi,
                                                ti, q, self, active, Ln, lane, gmask, count);
        return;
    }
    const double shx = (double)((code & 3) - 1) * P.L[0];
    const double shy = (double)(((code >> 2) & 3) - 1) * P.L[1];
    const double shz = (double)(((code >> 4) & 3) - 1) * P.L[2];
    if (cz.b1 >= 0)
        nlist_scan_cell<MULTI, STAGED, 3, SOLO>(a, st, s_rl2, P, o, m, jst, shx, shy, shz, cz, xi,
                                                ti, q, self, active, Ln, lane, gmask, count);
    else if (code != 21)
        nlist_scan_cell<MULTI, STAGED, 1, SOLO>(a, st, s_rl2, P, o, m, jst, shx, shy, shz, cz, xi,
                                                ti, q, self, active, Ln, lane, gmask, count);
    else
        nlist_scan_cell<MULTI, STAGED, 0, SOLO>(a, st, s_rl2, P, o, m, jst, 0.0, 0.0, 0.0, cz, xi,
                                                ti, q, self, active, Ln, lane, gmask, count);
}

template <bool MULTI, bool STAGED>
__device__ __forceinline__ void nlist_scan(const RebuildArgs &a, const double4 *__restrict__ st,
                                           const double *s_rl2, const BuildParams &P, int o,
                                           int m, int jst, int code, const ColumnShift &cz,
                                           const double4 &xi, int ti, int q, int self,
                                           bool active, int Ln, int lane,
                                           unsigned long long gmask, int &count) {
    if (Ln == 1)
        nlist_scan_dispatch<MULTI, STAGED, true>(a, st, s_rl2, P, o, m, jst, code, cz, xi, ti, q,
                                                 self, active, Ln, lane, gmask, count);
    else
        nlist_scan_dispatch<MULTI, STAGED, false>(a, st, s_rl2, P, o, m, jst, code, cz, xi, ti,
                                                  q, self, active, Ln, lane, gmask, count);
}

// A particle's list is complete: its count, its work-order key, the overflow flags and the
// wavefront's build statistics (one lane per particle).
__device__ __forceinline__ void finish_particle(const RebuildArgs &a, int rep, int first, int q,
                                                int count, uint8_t *s_cnt, int &my_max,
                                                unsigned long long &my_entries) {
    a.nl_count[q] = count;
    if (q - first < WORK_SORT_MAX) {
        const int chunks = (count + 7) >> 3;  // 8-entry list chunks, the work order's key
        s_cnt[q - first] = (uint8_t)(chunks < 255 ? chunks : 255);
    }
    if (count > a.cap) {
        atomicOr(&a.st->status, ST_OVERFLOW);
        if (a.rep_status) atomicOr(&a.rep_status[rep], ST_OVERFLOW);
    }
    my_max = count > my_max ? count : my_max;
    my_entries += (unsigned long long)(count < a.cap ? count : a.cap);
}

// The tile range [o, e) of stencil column h0 (its cells h0, h0 + 1, h0 + 2: z below, level,
// above) that a work item needs: all of it, or with the z-half split (half 0 or 1) without the
// far half of the cell above or below.
__device__ __forceinline__ void column_bounds(const TileSmem &t, const int *s_lo, int h0,
                                              int half, int &o, int &e) {
    o = __builtin_amdgcn_readfirstlane(t.off[h0]);
    e = __builtin_amdgcn_readfirstlane(t.off[h0 + 3]);
    if (half == 1) o += __builtin_amdgcn_readfirstlane(s_lo[h0]);
    if (half == 0)
        e = __builtin_amdgcn_readfirstlane(t.off[h0 + 2]) +
            __builtin_amdgcn_readfirstlane(s_lo[h0 + 2]);
}

// One particle's list built by a whole wavefront, 64 candidates a round: the ballot and the
// running count are the same on every lane (scalar registers). Hits go to the wavefront's ring
// of FLAT_RING entries in LDS (entry k at k mod FLAT_RING); whole groups of eight entries are
// written to the list with one 16-byte store per group, once 64 entries are pending and when
// the particle is done, instead of one 2-byte store per hit and round. Narrow lists only
// (32-bit byte offsets).
struct RingList {
    const ListWriter list;
    uint16_t *ring;
    int cap8;             // whole groups of eight below the cap
    int count = 0;        // entries found (uniform)
    int done = 0;         // groups of eight written (uniform)
    __device__ __forceinline__ RingList(const RebuildArgs &a, const BuildParams &P, int q,
                                        uint16_t *ring_)
        : list(a, P, q), ring(ring_), cap8(a.cap >> 3) {}
    // groups [done, g_end) of the ring to the list, one lane per group. The list's allocation
    // holds the cap rounded up to whole chunks, so a last partial group may carry stale ring
    // entries past the count (never read).
    __device__ __forceinline__ void flush(int g_end, int wl) {
        g_end = g_end < cap8 ? g_end : cap8;
        const int g = done + wl;
        if (g < g_end)
            list.store8_narrow(g, reinterpret_cast<const uint4 *>(ring)[g & (FLAT_RING / 8 - 1)]);
        done = __builtin_amdgcn_readfirstlane(g_end);
    }
    // one round: every lane writes, without a branch, a hit to its entry's slot and the others
    // to the slot of entry count + 64, which no pending entry holds (at most 64 + 7 are
    // pending) and a later hit overwrites before it is written out
    __device__ __forceinline__ void round(bool hit, int value, int wl) {
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(hit);
        const int k = (int)__builtin_amdgcn_mbcnt_hi(
            (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, (unsigned)count));
        ring[(hit ? k : count + 64) & (FLAT_RING - 1)] = (uint16_t)value;
        count += __popcll(bal);
        if (__builtin_amdgcn_readfirstlane(count - (done << 3)) >= 64) flush(count >> 3, wl);
    }
    __device__ __forceinline__ void finish(int wl) { flush((count + 7) >> 3, wl); }
};

// One work item with a whole wavefront per particle. The item's nine column ranges laid end
// to end are its particles' common candidate list, in the order the columns give one after
// another; lane l holds its candidates l, l + 64, ... as tile byte offsets in registers, and
// each of the item's particles takes all 64 lanes over that list, appending through the
// wavefront's ring as RingList does (written out inline here: the list build's hottest loop).
// The entries are those of the column-by-column scan, in the same order. Used for narrow lists
// and items whose stencil cells all lie in the primary image and whose candidates fit
// FLAT_ROUNDS rounds.
template <bool MULTI>
__device__ __forceinline__ void nlist_item_flat(const RebuildArgs &a,
                                                const double4 *__restrict__ st,
                                                const double *s_rl2, const BuildParams &P,
                                                const int (&co)[9], const int (&ce)[9], int M,
                                                int own, int beg, int cnt, int first, int rep,
                                                uint16_t *ring, uint8_t *s_cnt, int &my_max,
                                                unsigned long long &my_entries) {
    const int wl = threadIdx.x & 63;
    int tab[FLAT_ROUNDS];
#pragma unroll
    for (int r = 0; r < FLAT_ROUNDS; ++r) {
        // candidate f of the list: column c's atom co[c] + (f - start of column c)
        const int f = r * 64 + wl;
        int d = co[0], pre = ce[0] - co[0];
#pragma unroll
        for (int c = 1; c < 9; ++c) {
            d = f >= pre ? co[c] - pre : d;
            pre += ce[c] - co[c];
        }
        // byte offset in the tile; past the end: any tile atom (never a hit)
        tab[r] = (f < M ? f + d : own) * (int)sizeof(double4);
    }
    const char *const stb = reinterpret_cast<const char *>(st);
    const uint4 *const ring8 = reinterpret_cast<const uint4 *>(ring);
    // entries below the cap, in whole groups of eight: the list's allocation holds the cap
    // rounded up to whole chunks, so a last partial group may carry stale ring entries past
    // the count (never read)
    const int cap8 = a.cap >> 3;
    for (int p = 0; p < cnt; ++p) {
        const double4 xi = st[own + p];
        const int ti = MULTI ? (int)xi.w : 0;
        const int self_b = (own + p) * (int)sizeof(double4);
        const int q = beg + p;
        const ListWriter list(a, P, q);
        int count = 0, done = 0;  // entries found, groups of eight written (both uniform)
        auto flush = [&](int g_end) {
            const int g = done + wl;
            if (g < g_end) list.store8_narrow(g, ring8[g & (FLAT_RING / 8 - 1)]);
            done = __builtin_amdgcn_readfirstlane(g_end);
        };
        // the next round's candidates are read before this round's appends (LDS latency)
        double4 pn = *reinterpret_cast<const double4 *>(stb + tab[0]);
#pragma unroll
        for (int r = 0; r < FLAT_ROUNDS; ++r) {
            if (r * 64 >= M) break;
            const double4 pj = pn;
            if (r + 1 < FLAT_ROUNDS && (r + 1) * 64 < M)
                pn = *reinterpret_cast<const double4 *>(stb + tab[r + 1 < FLAT_ROUNDS ? r + 1 : r]);
            const double r2 = r2_canon(pj.x - xi.x, pj.y - xi.y, pj.z - xi.z);
            const double rl2 = MULTI ? s_rl2[ti * P.ntypes + (int)pj.w] : P.rl2;
            const bool hit = r * 64 + wl < M && tab[r] != self_b && r2 < rl2;
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(hit);
            // every lane writes, without a branch: a hit to its entry's slot, the others to
            // the slot of entry count + 64, which no pending entry holds (at most 64 + 7 are
            // pending) and a later hit overwrites before it is written out
            const int k = (int)__builtin_amdgcn_mbcnt_hi(
                (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, (unsigned)count));
            if (LJMD_DEBUG_CHECKS && hit && tab[r] / (int)sizeof(double4) >= P.tile_total)
                debug_fail(a.st, DBG_TILE);
            ring[(hit ? k : count + 64) & (FLAT_RING - 1)] =
                (uint16_t)(tab[r] / (int)sizeof(double4));
            count += __popcll(bal);
            // at most 64 + 7 entries pending: the ring never wraps onto unwritten ones
            if (__builtin_amdgcn_readfirstlane(count - (done << 3)) >= 64) {
                const int g_end = count >> 3;
                flush(g_end < cap8 ? g_end : cap8);
            }
        }
        {
            const int g_end = (count + 7) >> 3;
            flush(g_end < cap8 ? g_end : cap8);
        }
        if (wl == 0) finish_particle(a, rep, first, q, count, s_cnt, my_max, my_entries);
    }
}

// A brick of a box too small for the stencil's fixed images (fewer than three cells on some
// axis): every particle's candidates are the brick's whole tile, in tile order, with the
// branch-form minimum image, as the cell-by-cell scan takes them. The wavefronts take the
// brick's particles in turn, each with the whole wavefront (RingList), so a brick of many
// particles is spread over all of them instead of one wavefront per cell.
template <bool MULTI>
__device__ __forceinline__ void nlist_brick_whole(const RebuildArgs &a, const TileSmem &t,
                                                  const BrickInfo &bi,
                                                  const double4 *__restrict__ st,
                                                  const double *s_rl2, const BuildParams &P,
                                                  int first, uint16_t *ring, uint8_t *s_cnt,
                                                  int &my_max, unsigned long long &my_entries) {
    const int wl = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    const int total = t.total;
    const int R = (total + 63) >> 6;
    for (int ci = 0; ci < bi.ncell; ++ci) {
        const int rank = bi.first_cell + ci;
        const int cbeg = __builtin_amdgcn_readfirstlane(a.cell_start[rank]);
        const int ccnt = __builtin_amdgcn_readfirstlane(a.cell_start[rank + 1]) - cbeg;
        if (ccnt == 0) continue;
        // the cell as a halo cell: the one holding its range
        int hc = 0;
        for (int h = 0; h < t.nhalo; ++h)
            if (t.start[h] == cbeg && t.off[h + 1] - t.off[h] == ccnt) hc = h;
        const int own = __builtin_amdgcn_readfirstlane(t.off[hc]);
        for (int p = wave; p < ccnt; p += nwave) {
            const int self = own + p;
            const double4 xi = st[self];
            const int ti = MULTI ? (int)xi.w : 0;
            const int q = cbeg + p;
            RingList rl(a, P, q, ring);
            double4 pn = st[wl < total ? wl : total - 1];
            for (int r = 0; r < R; ++r) {
                const int j = r * 64 + wl;
                const double4 pj = pn;
                if (r + 1 < R) pn = st[j + 64 < total ? j + 64 : total - 1];
                const double dx = mi_branch(pj.x - xi.x, P.L[0]);
                const double dy = mi_branch(pj.y - xi.y, P.L[1]);
                const double dz = mi_branch(pj.z - xi.z, P.L[2]);
                const double r2 = r2_canon(dx, dy, dz);
                const double rl2 = MULTI ? s_rl2[ti * P.ntypes + (int)pj.w] : P.rl2;
                rl.round(j < total && j != self && r2 < rl2, j, wl);
            }
            rl.finish(wl);
            if (wl == 0) finish_particle(a, bi.rep, first, q, rl.count, s_cnt, my_max, my_entries);
        }
    }
}

// The cells of one brick, one wavefront per work item; STAGED selects candidate positions
// from the LDS tile or, for a tile larger than the LDS allocation, from global memory. With
// the z-half split (s_lo: each halo cell's lower-half count) a work item is one half of a
// cell: its particles need, of the stencil cells below them, only the upper half when they
// are in the upper half, and of the cells above them only the lower half when they are in
// the lower half (the far half lies beyond a cell width, at least the list radius, on z).
// Without it (boxes with fewer than three cells on an axis) an item is a whole cell.
template <bool MULTI, bool STAGED>
__device__ __forceinline__ void nlist_cells(const RebuildArgs &a, const TileSmem &t,
                                            const int *s_lo, const BrickInfo &bi,
                                            const double4 *__restrict__ st,
                                            const double *s_rl2, const BuildParams &P,
                                            int first, uint16_t *s_ring, uint8_t *s_cnt, int &my_max,
                                            unsigned long long &my_entries) {
    const int hy = (bi.dims >> 4) & 15, hz = (bi.dims >> 8) & 15;
    const int fpk = a.cell_xyz[bi.first_cell];
    const int wl = threadIdx.x & 63;
    // the wavefront index is uniform: so are the item, its cell and every range bound below
    // (scalar loop control)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    const int nst = P.canonical ? t.nhalo : 27;
    // split cells in halves only where whole cells would leave wavefronts idle (bricks of
    // fewer cells than wavefronts) and the caller allows it (split_halves): halves double the
    // ranges of an item's particles, and each range costs a fixed setup. The list is the
    // same either way: a split only skips atoms beyond the list radius, and entries keep the
    // tile order within each column
    if (STAGED && P.canonical && P.narrow) {
        nlist_brick_whole<MULTI>(a, t, bi, st, s_rl2, P, first, s_ring + wave * FLAT_RING,
                                 s_cnt, my_max, my_entries);
        return;
    }
    const bool split = s_lo != nullptr && a.split_halves && !P.canonical && bi.ncell < nwave;
    const int nitem = split ? 2 * bi.ncell : bi.ncell;
    for (int it = wave; it < nitem; it += nwave) {
        const int ci = split ? it >> 1 : it;
        const int half = split ? (it & 1) : -1;
        const int rank = bi.first_cell + ci;
        const int pk = a.cell_xyz[rank];
        const int lx = (pk & 1023) - (fpk & 1023);
        const int ly = ((pk >> 10) & 1023) - ((fpk >> 10) & 1023);
        const int lz = ((pk >> 20) & 1023) - ((fpk >> 20) & 1023);
        const int cbeg = __builtin_amdgcn_readfirstlane(a.cell_start[rank]);
        const int ccnt = __builtin_amdgcn_readfirstlane(a.cell_start[rank + 1]) - cbeg;
        // the cell as a halo cell: at the brick-relative offset (1, 1, 1) of its stencil, or
        // in a small box the distinct halo cell holding the cell's range
        int hc = ((lx + 1) * hy + (ly + 1)) * hz + (lz + 1);
        if (P.canonical)
            for (int h = 0; h < t.nhalo; ++h)
                if (t.start[h] == cbeg && t.off[h + 1] - t.off[h] == ccnt) hc = h;
        const int clo = split ? __builtin_amdgcn_readfirstlane(s_lo[hc]) : 0;
        // the item's particles: the cell's lower-half members, its upper-half ones, or all
        const int pb = half == 1 ? clo : 0;
        const int cnt = half == 0 ? clo : ccnt - pb;
        if (cnt == 0) continue;
        const int beg = cbeg + pb;
        const int own = STAGED ? __builtin_amdgcn_readfirstlane(t.off[hc]) + pb : 0;
        if (STAGED && !P.canonical) {
            int co[9], ce[9], M = 0;
            bool plain = true;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const int h0 = ((lx + c / 3) * hy + (ly + c % 3)) * hz + lz;
                plain = plain && __builtin_amdgcn_readfirstlane(t.shift[h0]) == 21 &&
                        __builtin_amdgcn_readfirstlane(t.shift[h0 + 1]) == 21 &&
                        __builtin_amdgcn_readfirstlane(t.shift[h0 + 2]) == 21;
                column_bounds(t, s_lo, h0, half, co[c], ce[c]);
                M += ce[c] - co[c];
            }
            if (plain && P.narrow && M <= FLAT_ROUNDS * 64) {
                nlist_item_flat<MULTI>(a, st, s_rl2, P, co, ce, M, own, beg, cnt, first, bi.rep,
                                       s_ring + wave * FLAT_RING, s_cnt, my_max, my_entries);
                continue;
            }
        }
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
            const double4 xi = STAGED ? st[own + (active ? p : 0)] : a.pos_scr[q];
            const int ti = MULTI ? (int)xi.w : 0;
            const int self = STAGED ? own + (active ? p : 0) : q;
            int count = 0;
            if (STAGED && !P.canonical) {
                // the stencil by columns (dx, dy): a column's three cells (z below, level,
                // above) are consecutive in the tile, and so is the part of them the item
                // needs, so a column is one range (same entry order as cell by cell); across
                // the box's z boundary its cells differ in their z image only
                for (int c = 0; c < 9; ++c) {
                    const int h0 = ((lx + c / 3) * hy + (ly + c % 3)) * hz + lz;
                    const int code = __builtin_amdgcn_readfirstlane(t.shift[h0]);
                    const int code1 = __builtin_amdgcn_readfirstlane(t.shift[h0 + 1]);
                    const int code2 = __builtin_amdgcn_readfirstlane(t.shift[h0 + 2]);
                    ColumnShift cz{-1, -1, 0.0, 0.0};
                    if (code != code1 || code != code2) {
                        cz.b1 = __builtin_amdgcn_readfirstlane(t.off[h0 + 1]);
                        cz.b2 = __builtin_amdgcn_readfirstlane(t.off[h0 + 2]);
                        cz.shz1 = (double)(((code1 >> 4) & 3) - 1) * P.L[2];
                        cz.shz2 = (double)(((code2 >> 4) & 3) - 1) * P.L[2];
                    }
                    int o, e;
                    column_bounds(t, s_lo, h0, half, o, e);
                    nlist_scan<MULTI, STAGED>(a, st, s_rl2, P, o, e - o, 0, code, cz, xi, ti, q,
                                              self, active, Ln, lane, gmask, count);
                }
            } else {
                for (int s = 0; s < nst; ++s) {
                    const int h =
                        P.canonical ? s
                                    : ((lx + s / 9) * hy + (ly + (s / 3) % 3)) * hz + (lz + s % 3);
                    // the stencil cell is the same for every lane of the wavefront: keep its
                    // bounds in scalar registers (uniform loop control, no per-lane masks)
                    int o = __builtin_amdgcn_readfirstlane(t.off[h]);
                    int m = __builtin_amdgcn_readfirstlane(t.off[h + 1]) - o;
                    int jst = __builtin_amdgcn_readfirstlane(t.start[h]);
                    const int code = __builtin_amdgcn_readfirstlane(t.shift[h]);
                    if (split && s % 3 != 1) {
                        const int lo_h = __builtin_amdgcn_readfirstlane(s_lo[h]);
                        if (half == 0 && s % 3 == 2) {
                            m = lo_h;  // the cell above: its lower half
                        } else if (half == 1 && s % 3 == 0) {
                            o += lo_h;  // the cell below: its upper half
                            jst += lo_h;
                            m -= lo_h;
                        }
                    }
                    const ColumnShift none{-1, -1, 0.0, 0.0};
                    nlist_scan<MULTI, STAGED>(a, st, s_rl2, P, o, m, jst, code, none, xi, ti, q,
                                              self, active, Ln, lane, gmask, count);
                }
            }
            if (active && lane == 0)
                finish_particle(a, bi.rep, first, q, count, s_cnt, my_max, my_entries);
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
                                           const uint8_t *s_cnt, int *s_bin) {
    if (natoms > WORK_SORT_MAX) {
        for (int p = threadIdx.x; p < natoms; p += blockDim.x) a.work[first + p] = (uint16_t)p;
        return;
    }
    for (int k = threadIdx.x; k < 256; k += blockDim.x) s_bin[k] = 0;
    __syncthreads();  // also: every count is in s_cnt
    for (int p = threadIdx.x; p < natoms; p += blockDim.x) {
        atomicAdd(&s_bin[255 - s_cnt[p]], 1);
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
        const int at = atomicAdd(&s_bin[255 - s_cnt[p]], 1);
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
    const RepParams &P = a.reps[__builtin_amdgcn_readfirstlane(bi.rep)];
    BuildParams U = build_params(P);
    // every slot of an entry k < cap is below npad x (cap rounded up to a whole round)
    U.narrow = a.npad < (1 << 24) &&
               (uint64_t)a.npad * (uint64_t)(a.cap + (8 << a.lshift)) <= 0x7FFFFFFFull;
    extern __shared__ double4 dyn_tile[];
    __shared__ TileSmem t;
    double4 *st = dyn_tile;
    double *s_rl2 = reinterpret_cast<double *>(st + a.tile_cap);
    if (MULTI)
        for (int k = threadIdx.x; k < P.ntypes * P.ntypes; k += blockDim.x)
            s_rl2[k] = a.rl2_table[P.pair_off + k];
    if (b == P.boff && threadIdx.x == 0) atomicAdd(&a.st->builds, 1ull);
    __shared__ int s_lo[HALO_MAX];
    tile_setup(bi, a.halo + (size_t)b * HALO_MAX, a.cell_start, t, a.cell_lo ? s_lo : nullptr,
               a.cell_lo);
    tile_save(t, a.tile_tab + (size_t)b * TILE_TAB);
    U.tile_total = t.total;
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
    __shared__ uint8_t s_cnt[WORK_SORT_MAX];
    // the wavefronts' list rings during the scan (8 x FLAT_RING entries), then the work
    // order's 256 bins
    __shared__ uint4 s_share[8 * FLAT_RING * sizeof(uint16_t) / sizeof(uint4)];
    static_assert(sizeof(s_share) >= 256 * sizeof(int), "bins fit the shared array");
    uint16_t *s_ring = reinterpret_cast<uint16_t *>(s_share);
    int *s_bin = reinterpret_cast<int *>(s_share);
    const int first = a.cell_start[bi.first_cell];
    const int natoms = a.cell_start[bi.first_cell + bi.ncell] - first;
    if (staged)
        nlist_cells<MULTI, true>(a, t, a.cell_lo ? s_lo : nullptr, bi, st, s_rl2, U, first,
                                 s_ring, s_cnt, my_max, my_entries);
    else
        nlist_cells<MULTI, false>(a, t, a.cell_lo ? s_lo : nullptr, bi, st, s_rl2, U, first,
                                  s_ring, s_cnt, my_max, my_entries);
    work_order(a, first, natoms, s_cnt, s_bin);

    // The build statistics, reduced over the wavefront, then over the workgroup, then one
    // atomic add per workgroup, and an atomic max only where the workgroup's longest list is
    // longer than the one recorded. Atomics on one word from every wavefront of the chip
    // serialise, and a wavefront does not retire before its atomics are acknowledged: per
    // wavefront they held the workgroup slots idle for most of the build.
    for (int o = 32; o > 0; o >>= 1) {
        const int om = __shfl_xor(my_max, o);
        my_max = om > my_max ? om : my_max;
        my_entries += __shfl_xor(my_entries, o);
    }
    __syncthreads();  // the work order is done with the shared array
    int *s_wmax = reinterpret_cast<int *>(s_share);
    unsigned long long *s_went = reinterpret_cast<unsigned long long *>(s_share) + 8;
    const int wave = threadIdx.x >> 6;
    if (wl == 0) {
        s_wmax[wave] = my_max;
        s_went[wave] = my_entries;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int mx = 0;
        unsigned long long ent = 0ull;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            mx = s_wmax[w] > mx ? s_wmax[w] : mx;
            ent += s_went[w];
        }
        if (mx > __hip_atomic_load(&a.st->max_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&a.st->max_count, mx);
        if (ent) atomicAdd(&a.st->entries, ent);
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

// The sort of a rebuild: bin, scan, scatter and in-cell gather; ev (optional): the first five
// of the six events around a rebuild's kernels, for measurement.
hipError_t launch_sort_cells(hipStream_t s, const RebuildArgs &a, hipEvent_t *ev) {
    const int b = 256;
    const int g = (a.n + b - 1) / b;
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_bin, dim3(g), dim3(b), 0, s, a);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(k_scan, dim3(a.nrep), dim3(1024), 0, s, a);
    if (ev) (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(b), 0, s, a);
    if (ev) (void)hipEventRecord(ev[3], s);
    hipLaunchKernelGGL(k_cell_gather, dim3(a.ncell < 8192 ? a.ncell : 8192), dim3(64), 0, s, a);
    if (ev) (void)hipEventRecord(ev[4], s);
    return hipGetLastError();
}

hipError_t launch_rebuild(hipStream_t s, const RebuildArgs &a, hipEvent_t *ev) {
    if (!lds_args_ok(a.tile_cap, a.max_ntypes, nlist_lds_bytes(a.tile_cap, a.max_ntypes)))
        return hipErrorInvalidValue;
    // ev (optional): six events around the five kernels, for measurement
    const hipError_t e = launch_sort_cells(s, a, ev);
    if (e != hipSuccess) return e;
    const size_t smem = nlist_lds_bytes(a.tile_cap, a.max_ntypes);
    if (a.max_ntypes > 1)
        hipLaunchKernelGGL(k_nlist<true>, dim3(a.nbrick), dim3(512), smem, s, a);
    else
        hipLaunchKernelGGL(k_nlist<false>, dim3(a.nbrick), dim3(512), smem, s, a);
    if (ev) (void)hipEventRecord(ev[5], s);
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

// ---------------------------------------------------------------- NVT thermostat

// Kinetic energy partial sums (one per workgroup, fixed order) of particles [poff, poff + n).
__global__ void __launch_bounds__(RED_BLOCK) k_ke_partials(const double4 *vel, int poff, int n,
                                                            double *partials) {
    __shared__ double s[RED_BLOCK];
    double acc = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double4 v = vel[(size_t)poff + k];
        const double m = 1.0 / v.w;
        acc += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = RED_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// One thermostat half step of length dt/2 from kinetic energy K: xi += dt/4 G(K),
// eta += dt/2 xi, scale s = exp(-dt/2 xi) (K becomes s^2 K), xi += dt/4 G(K), with
// G(K) = (2K - N_f kT) / Q. Returns s.
__device__ double nvt_half(double &xi, double &eta, double &K, const NvtParams &p) {
    xi += 0.25 * p.dt * (2.0 * K - p.g) * p.invQ;
    eta += 0.5 * p.dt * xi;
    const double sc = exp(-0.5 * p.dt * xi);
    K = sc * sc * K;
    xi += 0.25 * p.dt * (2.0 * K - p.g) * p.invQ;
    return sc;
}

// One workgroup: the kinetic energy from the partials, then the thermostat. At the end of a
// step (begin_only = 0) K is that of the velocities after the second kick: the end half step
// runs from the state the step opened with (xi_b, eta_b) and is committed, with its scale
// factor left pending for the stored velocities; the half step that opens the next step is
// then taken from the scaled K. With begin_only the half step that opens the next step is
// taken from the committed state and the K of the stored velocities.
__global__ void __launch_bounds__(RED_BLOCK) k_nvt_thermo(const double *partials, NvtParams p,
                                                           double *th) {
    __shared__ double s[RED_BLOCK];
    double acc = 0.0;
    for (int k = threadIdx.x; k < p.np; k += blockDim.x) acc += partials[k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = RED_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double K = s[0];
    double xi, eta;
    if (p.begin_only) {
        xi = th[TH_XI];
        eta = th[TH_ETA];
        th[TH_SPEND] = 1.0;
        th[TH_K] = K;
    } else {
        xi = th[TH_XIB];
        eta = th[TH_ETAB];
        const double s1 = nvt_half(xi, eta, K, p);
        th[TH_XI] = xi;
        th[TH_ETA] = eta;
        th[TH_SPEND] = s1;
        th[TH_K] = K;
    }
    const double s2 = nvt_half(xi, eta, K, p);
    th[TH_SB] = s2;
    th[TH_XIB] = xi;
    th[TH_ETAB] = eta;
}

// A thermo sample of an NVT step: its kinetic energy is the thermostat's, after the closing
// half step (the stored velocities are scaled only when the next step opens).
__global__ void k_thermo_nvt_k(double *row, const double *th) {
    if (threadIdx.x == 0 && blockIdx.x == 0) row[RED_QUANT - 1] = th[TH_K];
}

hipError_t launch_thermo_nvt_k(hipStream_t s, double *row, const double *th) {
    hipLaunchKernelGGL(k_thermo_nvt_k, dim3(1), dim3(64), 0, s, row, th);
    return hipGetLastError();
}

// End of a call: the stored velocities take the pending scale factor ...
__global__ void k_nvt_scale(double4 *vel, int poff, int n, const double *th) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double sc = th[TH_SPEND];
    double4 v = vel[(size_t)poff + k];
    v.x = sc * v.x;
    v.y = sc * v.y;
    v.z = sc * v.z;
    vel[(size_t)poff + k] = v;
}

// ... and only then is it cleared (a separate launch: every workgroup above has read it).
__global__ void k_nvt_clear_pending(double *th) {
    if (threadIdx.x == 0 && blockIdx.x == 0) th[TH_SPEND] = 1.0;
}

__global__ void k_negate_vel(double4 *vel, int poff, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double4 v = vel[(size_t)poff + k];
    v.x = -v.x;
    v.y = -v.y;
    v.z = -v.z;
    vel[(size_t)poff + k] = v;
}

hipError_t launch_negate_vel(hipStream_t s, double4 *vel, int poff, int n) {
    hipLaunchKernelGGL(k_negate_vel, dim3((n + 255) / 256), dim3(256), 0, s, vel, poff, n);
    return hipGetLastError();
}

hipError_t launch_ke_partials(hipStream_t s, const double4 *vel, int poff, int n,
                              double *partials, int nblocks_max, int *np_out) {
    int g = (n + RED_BLOCK - 1) / RED_BLOCK;
    if (g > nblocks_max) g = nblocks_max;
    if (g < 1) g = 1;
    *np_out = g;
    hipLaunchKernelGGL(k_ke_partials, dim3(g), dim3(RED_BLOCK), 0, s, vel, poff, n, partials);
    return hipGetLastError();
}

hipError_t launch_nvt_thermo(hipStream_t s, const double *partials, const NvtParams &p,
                             double *th) {
    hipLaunchKernelGGL(k_nvt_thermo, dim3(1), dim3(RED_BLOCK), 0, s, partials, p, th);
    return hipGetLastError();
}

hipError_t launch_nvt_finalize(hipStream_t s, double4 *vel, int poff, int n, double *th) {
    hipLaunchKernelGGL(k_nvt_scale, dim3((n + 255) / 256), dim3(256), 0, s, vel, poff, n, th);
    hipLaunchKernelGGL(k_nvt_clear_pending, dim3(1), dim3(64), 0, s, th);
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
        st->debug = 0;
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