// The force kernel family of libljmd for gfx950: one workgroup per brick, the brick's tile in
// LDS, lanes per particle striding its 16-bit list, wavefront shuffles for the per-particle
// sums, and the velocity-Verlet epilogue of the fused step. Templated on the pair form; each
// form is instantiated in a translation unit of its own (ljmd_force_<form>.hip), which defines
// that form's launcher. Compiled with -ffp-contract=off.
#pragma once

#include "ljmd_device.h"

namespace ljmd {

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

// The pair form's force factor f (force on i = f (x_i - x_j)) and, with ENERGY, its shifted
// energy u, at squared distance r2 inside the cutoff. Coefficients per form (PairCoef):
//   LJ      lj1 = 48 eps s^12, lj2 = 24 eps s^6, lj3 = 4 eps s^12, lj4 = 4 eps s^6:
//           f = r^-2 r^-6 (lj1 r^-6 - lj2), u = r^-6 (lj3 r^-6 - lj4) - shift
//   Mie     lj1 = C eps n s^n, lj2 = C eps m s^m, lj3 = n/2, lj4 = m/2:
//           f = (lj1 r^-n - lj2 r^-m) / r^2, u = lj1 r^-n / n - lj2 r^-m / m - shift
//   Gauss   lj1 = eps / s^2, lj2 = -1 / (2 s^2), lj3 = eps:
//           f = lj1 exp(lj2 r^2), u = lj3 exp(lj2 r^2) - shift
//   Yukawa  lj1 = eps, lj2 = kappa: f = eps exp(-kappa r) (1 + kappa r) / r^3,
//           u = eps exp(-kappa r) / r - shift
template <int FORM, bool ENERGY>
__device__ __forceinline__ double form64(const PairCoef &c, double r2, double &u) {
    constexpr int STYLE = FORM & 7;
    if (STYLE == STYLE_LJ) {
        const double r2i = rcp64(r2);
        const double r6i = r2i * r2i * r2i;
        if (ENERGY) u = r6i * __builtin_fma(c.lj3, r6i, -c.lj4) - c.shift;
        return r2i * r6i * __builtin_fma(c.lj1, r6i, -c.lj2);
    } else if (STYLE == STYLE_MIE) {
        const double lr = log(r2);
        const double rn = exp(-c.lj3 * lr);
        const double rm = exp(-c.lj4 * lr);
        if (ENERGY) u = (c.lj1 * rn) / (2.0 * c.lj3) - (c.lj2 * rm) / (2.0 * c.lj4) - c.shift;
        return (c.lj1 * rn - c.lj2 * rm) / r2;
    } else if (STYLE == STYLE_GAUSS) {
        const double g = exp(c.lj2 * r2);
        if (ENERGY) u = c.lj3 * g - c.shift;
        return c.lj1 * g;
    } else {
        const double r = sqrt(r2);
        const double e = c.lj1 * exp(-c.lj2 * r);
        if (ENERGY) u = e / r - c.shift;
        return e * __builtin_fma(c.lj2, r, 1.0) / (r2 * r);
    }
}

// The same in FP32 (the mixed path); the energy shift is applied in FP64 by the caller.
template <int FORM, bool ENERGY>
__device__ __forceinline__ float form32(const PairCoef &c, float r2, float &u) {
    constexpr int STYLE = FORM & 7;
    if (STYLE == STYLE_LJ) {
        const float r2i = __builtin_amdgcn_rcpf(r2);
        const float r6i = r2i * r2i * r2i;
        if (ENERGY) u = r6i * __builtin_fmaf((float)c.lj3, r6i, -(float)c.lj4);
        return r2i * r6i * __builtin_fmaf((float)c.lj1, r6i, -(float)c.lj2);
    } else if (STYLE == STYLE_MIE) {
        const float lr = logf(r2);
        const float rn = expf(-(float)c.lj3 * lr);
        const float rm = expf(-(float)c.lj4 * lr);
        if (ENERGY) u = ((float)c.lj1 * rn) / (2.0f * (float)c.lj3) -
                        ((float)c.lj2 * rm) / (2.0f * (float)c.lj4);
        return ((float)c.lj1 * rn - (float)c.lj2 * rm) / r2;
    } else if (STYLE == STYLE_GAUSS) {
        const float g = expf((float)c.lj2 * r2);
        if (ENERGY) u = (float)c.lj3 * g;
        return (float)c.lj1 * g;
    } else {
        const float r = sqrtf(r2);
        const float e = (float)c.lj1 * expf(-(float)c.lj2 * r);
        if (ENERGY) u = e / r;
        return e * __builtin_fmaf((float)c.lj2, r, 1.0f) / (r2 * r);
    }
}

// One pair inside the cutoff: add the force on i (and, with ENERGY, half the pair energy and
// virial) for the displacement d = x_j - x_i with r2 = |d|^2. With STYLE_SF in STYLE, the
// shifted-force variant: f - F(r_cut) / r, and u + r F(r_cut) (the shift holds the constant
// part, u(r_cut) + r_cut F(r_cut)), so that both vanish at r_cut.
template <int STYLE, int PREC, bool ENERGY>
__device__ __forceinline__ void pair_term(const PairCoef &c, double dx, double dy, double dz,
                                          double r2, Acc<PREC> &acc, double &ue, double &w0,
                                          double &w1, double &w2, double &w3, double &w4,
                                          double &w5) {
    if (PREC == PREC_FP64) {
        double u = 0.0;
        double ff = form64<STYLE, ENERGY>(c, r2, u);
        if (STYLE & STYLE_SF) {
            const double r = __builtin_sqrt(r2);
            ff = __builtin_fma(-c.fcut, rcp64(r), ff);
            if (ENERGY) u = __builtin_fma(c.fcut, r, u);
        }
        // force on i is ff * (x_i - x_j) = -ff * d
        acc.fx = __builtin_fma(-ff, dx, acc.fx);
        acc.fy = __builtin_fma(-ff, dy, acc.fy);
        acc.fz = __builtin_fma(-ff, dz, acc.fz);
        if (ENERGY) {
            ue += 0.5 * u;
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
        float up = 0.0f;
        float ff = form32<STYLE, ENERGY>(c, fr2, up);
        float fr = 0.0f;
        if (STYLE & STYLE_SF) {
            fr = __builtin_sqrtf(fr2);
            ff = __builtin_fmaf(-(float)c.fcut, __builtin_amdgcn_rcpf(fr), ff);
        }
        acc.fx = __builtin_fmaf(-ff, fdx, acc.fx);
        acc.fy = __builtin_fmaf(-ff, fdy, acc.fy);
        acc.fz = __builtin_fmaf(-ff, fdz, acc.fz);
        if (ENERGY) {
            ue += 0.5 * ((double)up - c.shift + ((STYLE & STYLE_SF) ? c.fcut * (double)fr : 0.0));
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

// The end of a particle's pass: its force (and, with ENERGY, energy and virial halves) summed
// over its TPP lanes with wavefront shuffles, then, on lane 0, the finish MODE asks for: the
// force stored (MODE_EVAL), or the velocity-Verlet epilogue (MODE_FINAL: second half kick;
// MODE_FUSED: second half kick, first half kick of the next step, drift, wrap and the
// displacement check, which is returned).
template <int PREC, int TPP, int MODE, bool ENERGY>
__device__ __forceinline__ bool finish_particle(const ForceArgs &a, const RepParams &P, int q,
                                                int rep, bool active, int lane, bool last,
                                                const double4 &xi, const Acc<PREC> &acc,
                                                double ue, double w0, double w1, double w2,
                                                double w3, double w4, double w5) {
    const double L0 = P.L[0], L1 = P.L[1], L2 = P.L[2];
    const double iL0 = P.invL[0], iL1 = P.invL[1], iL2 = P.invL[2];
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
                // the image counters change only where a coordinate wraps: they are read
                // and written there alone
                int4 d = make_int4(0, 0, 0, 0);
                wrap_coord(x.x, d.x, L0);
                wrap_coord(x.y, d.y, L1);
                wrap_coord(x.z, d.z, L2);
                a.pos_out[q] = x;
                a.vel[q] = v;
                if (d.x | d.y | d.z) {
                    int4 im = a.img[q];
                    im.x += d.x;
                    im.y += d.y;
                    im.z += d.z;
                    a.img[q] = im;
                }
                const double4 b_pre = a.xb[q];
                if (LJMD_DEBUG_CHECKS) {
                    // the forces were taken at xi: within half the skin of the list's build
                    const double ox = mi_rint(xi.x - b_pre.x, L0, iL0);
                    const double oy = mi_rint(xi.y - b_pre.y, L1, iL1);
                    const double oz = mi_rint(xi.z - b_pre.z, L2, iL2);
                    if (r2_canon(ox, oy, oz) >= P.lim2)
                        debug_fail(reinterpret_cast<DevStatus *>(a.status), DBG_DANGEROUS);
                }
                const double ex = mi_rint(x.x - b_pre.x, L0, iL0);
                const double ey = mi_rint(x.y - b_pre.y, L1, iL1);
                const double ez = mi_rint(x.z - b_pre.z, L2, iL2);
                exceed = r2_canon(ex, ey, ez) >= P.lim2;
            }
        }
    }
    return exceed;
}

// The particle passes of one brick; STAGED selects neighbour positions from the LDS tile
// (plain LDS reads) or, for a tile larger than the LDS allocation, from global memory.
// MIF: bit a set when no pair of the brick can wrap on axis a (the minimum image is skipped
// there; subtracting 0 x L would give the same bits).
template <int STYLE, int PREC, int TPP, int MODE, bool ENERGY, bool MULTI, bool STAGED, int MIF>
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
            // first, then the arithmetic runs on them. The builder writes only tile indices;
            // an entry is clamped to the tile (not tested against it) so that the read stays
            // inside the tile whatever the word holds: one compare and one clamp per entry.
            constexpr int FB = FORCE_BATCH;
            const int left = cnt - k0;
            const int top = t.total - 1;
#pragma unroll
            for (int u0 = 0; u0 < 8; u0 += FB) {
                double px[FB], py[FB], pz[FB];
                int pt[FB];
                bool pv[FB];
#pragma unroll
                for (int v = 0; v < FB; ++v) {
                    const int u = u0 + v;
                    pv[v] = u < left;
                    if (LJMD_DEBUG_CHECKS && pv[v] && e[u] > top)
                        debug_fail(reinterpret_cast<DevStatus *>(a.status), DBG_READ);
                    const int idx = e[u] < top ? e[u] : top;
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
                    // fused: the force kernel's r^2 may differ from the canonical one by a
                    // rounding (the list decision stays canonical in the build)
                    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                    const PairCoef &c = MULTI ? s_pair[ti * P.ntypes + pt[v]] : single;
                    if (pv[v] && r2 < c.rc2)
                        pair_term<STYLE, PREC, ENERGY>(c, dx, dy, dz, r2, acc, ue, w0, w1, w2, w3, w4, w5);
                }
            }
        }

        const bool exceed = finish_particle<PREC, TPP, MODE, ENERGY>(
            a, P, q, rep, active, lane, last, xi, acc, ue, w0, w1, w2, w3, w4, w5);
        if (MODE == MODE_FUSED) {
            // all particles of the workgroup belong to one replica: one atomic per wavefront
            const unsigned long long vote = __ballot(exceed);
            // set once: a plain read first spares the atomic once another wavefront set it
            if (exceed && (threadIdx.x & 63) == __ffsll((long long)vote) - 1 &&
                __hip_atomic_load(&a.req[2 * rep + (a.cur ^ 1)], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) == 0)
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
template <int STYLE, int PREC, int TPP, int MODE, bool ENERGY, bool MULTI>
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
    force_passes<STYLE, PREC, TPP, MODE, ENERGY, MULTI, true, M>(a, t, st, s_pair, single, P, ce, rep, last, first, natoms)
    if (!staged) {
        force_passes<STYLE, PREC, TPP, MODE, ENERGY, MULTI, false, 0>(
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


template <int STYLE, int PREC, int TPP, int MODE, bool ENERGY>
static hipError_t launch_force_t(hipStream_t s, const ForceArgs &a, int block) {
    const size_t smem = force_lds_bytes(a.tile_cap, a.max_ntypes);
    if (!lds_args_ok(a.tile_cap, a.max_ntypes, smem)) return hipErrorInvalidValue;
    if (a.max_ntypes > 1)
        hipLaunchKernelGGL((k_force<STYLE, PREC, TPP, MODE, ENERGY, true>), dim3(a.nbrick), dim3(block),
                           smem, s, a);
    else
        hipLaunchKernelGGL((k_force<STYLE, PREC, TPP, MODE, ENERGY, false>), dim3(a.nbrick), dim3(block),
                           smem, s, a);
    return hipGetLastError();
}

template <int STYLE, int PREC, int TPP>
static hipError_t launch_force_m(hipStream_t s, const ForceArgs &a, int mode, bool energy,
                                 int block) {
    switch (mode) {
        case MODE_EVAL:
            return energy ? launch_force_t<STYLE, PREC, TPP, MODE_EVAL, true>(s, a, block)
                          : launch_force_t<STYLE, PREC, TPP, MODE_EVAL, false>(s, a, block);
        case MODE_FUSED:
            return energy ? launch_force_t<STYLE, PREC, TPP, MODE_FUSED, true>(s, a, block)
                          : launch_force_t<STYLE, PREC, TPP, MODE_FUSED, false>(s, a, block);
        default:
            return launch_force_t<STYLE, PREC, TPP, MODE_FINAL, false>(s, a, block);
    }
}

template <int STYLE, int PREC>
static hipError_t launch_force_p(hipStream_t s, const ForceArgs &a, int tpp, int mode,
                                 bool energy, int block) {
    switch (tpp) {
        case 1: return launch_force_m<STYLE, PREC, 1>(s, a, mode, energy, block);
        case 2: return launch_force_m<STYLE, PREC, 2>(s, a, mode, energy, block);
        case 4: return launch_force_m<STYLE, PREC, 4>(s, a, mode, energy, block);
        case 8: return launch_force_m<STYLE, PREC, 8>(s, a, mode, energy, block);
        case 16: return launch_force_m<STYLE, PREC, 16>(s, a, mode, energy, block);
        default: return hipErrorInvalidValue;
    }
}

// All launches of one pair form: precision, lanes per particle, mode and energy are runtime
// choices dispatched to the instantiated kernels.
template <int STYLE>
static hipError_t launch_force_style(hipStream_t s, const ForceArgs &a, int prec, int tpp,
                                     int mode, bool energy, int block) {
    if (block < 64 || block > 512 || (block & 63)) return hipErrorInvalidValue;
    return prec == PREC_MIXED ? launch_force_p<STYLE, PREC_MIXED>(s, a, tpp, mode, energy, block)
                              : launch_force_p<STYLE, PREC_FP64>(s, a, tpp, mode, energy, block);
}

}  // namespace ljmd
