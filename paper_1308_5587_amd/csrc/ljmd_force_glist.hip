// Force kernels over tree (BVH) lists: 32-bit sorted-order neighbour indices, so neighbour
// positions come from global memory (L2) rather than a brick tile, with the minimum image on
// every axis. TPP lanes per particle stride its list 4 entries per 16-byte load and reduce
// with wavefront shuffles; the particle's finish (stored force, or the velocity-Verlet
// epilogue) is the brick kernels' (finish_particle). LJ form; one system (replica 0).
#include "ljmd_force.h"

namespace ljmd {

template <int PREC, int TPP, int MODE, bool ENERGY, bool MULTI>
__global__ void __launch_bounds__(512) k_force_glist(const ForceArgs a) {
    extern __shared__ PairCoef s_pair[];
    const RepParams &P = a.reps[0];
    if (MULTI) {
        for (int k = threadIdx.x; k < P.ntypes * P.ntypes; k += blockDim.x)
            s_pair[k] = a.pair[P.pair_off + k];
        __syncthreads();
    }
    const PairCoef single = a.pair[P.pair_off];
    if (MODE == MODE_FUSED && blockIdx.x == 0 && threadIdx.x == 0)
        a.req[a.cur] = 0;  // the request for this buffer was served
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = gid & (TPP - 1);
    const bool active = gid / TPP < P.n;
    const int q = active ? gid / TPP : 0;
    const double4 xi = a.pos_in[q];
    const int ti = MULTI ? (int)xi.w : 0;
    int cnt = active ? a.nl_count[q] : 0;
    cnt = cnt < a.cap ? cnt : a.cap;
    const double L0 = P.L[0], L1 = P.L[1], L2 = P.L[2];
    const double iL0 = P.invL[0], iL1 = P.invL[1], iL2 = P.invL[2];
    typedef int v4i __attribute__((ext_vector_type(4)));
    const size_t cstride = (size_t)a.npad << a.lshift;  // 16-byte chunks between rounds
    const v4i *row = reinterpret_cast<const v4i *>(a.nlist32) + ((size_t)q << a.lshift) + lane;
    Acc<PREC> acc;
    double ue = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0, w4 = 0.0, w5 = 0.0;
    for (int k0 = lane * 4; k0 < cnt; k0 += 4 * TPP) {
        const v4i cur = __builtin_nontemporal_load(row);
        row += cstride;
        const int e[4] = {cur.x, cur.y, cur.z, cur.w};
        double px[4], py[4], pz[4];
        int pt[4];
        bool pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pv[u] = k0 + u < cnt;
            const double4 pj = a.pos_in[pv[u] ? e[u] : q];
            px[u] = pj.x;
            py[u] = pj.y;
            pz[u] = pj.z;
            pt[u] = (int)pj.w;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double dx = mi_rint(px[u] - xi.x, L0, iL0);
            const double dy = mi_rint(py[u] - xi.y, L1, iL1);
            const double dz = mi_rint(pz[u] - xi.z, L2, iL2);
            // fused, as in the cell-list force kernel (the list decision stays canonical)
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const PairCoef &c = MULTI ? s_pair[ti * P.ntypes + pt[u]] : single;
            if (pv[u] && r2 < c.rc2)
                pair_term<STYLE_LJ, PREC, ENERGY>(c, dx, dy, dz, r2, acc, ue, w0, w1, w2, w3, w4,
                                                  w5);
        }
    }
    const bool exceed = finish_particle<PREC, TPP, MODE, ENERGY>(
        a, P, q, 0, active, lane, false, xi, acc, ue, w0, w1, w2, w3, w4, w5);
    if (MODE == MODE_FUSED) {
        const unsigned long long vote = __ballot(exceed);
        if (exceed && (threadIdx.x & 63) == __ffsll((long long)vote) - 1 &&
            __hip_atomic_load(&a.req[a.cur ^ 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            atomicOr(&a.req[a.cur ^ 1], 1);
    }
}

template <int PREC, int TPP, int MODE, bool ENERGY>
static hipError_t launch_glist_t(hipStream_t s, const ForceArgs &a, int block) {
    const size_t nthreads = (size_t)a.npad * TPP;
    const dim3 grid((unsigned)((nthreads + block - 1) / block));
    if (a.max_ntypes > 1)
        hipLaunchKernelGGL((k_force_glist<PREC, TPP, MODE, ENERGY, true>), grid, dim3(block),
                           (size_t)a.max_ntypes * a.max_ntypes * sizeof(PairCoef), s, a);
    else
        hipLaunchKernelGGL((k_force_glist<PREC, TPP, MODE, ENERGY, false>), grid, dim3(block), 0,
                           s, a);
    return hipGetLastError();
}

template <int PREC, int TPP>
static hipError_t launch_glist_m(hipStream_t s, const ForceArgs &a, int mode, bool energy,
                                 int block) {
    switch (mode) {
        case MODE_EVAL:
            return energy ? launch_glist_t<PREC, TPP, MODE_EVAL, true>(s, a, block)
                          : launch_glist_t<PREC, TPP, MODE_EVAL, false>(s, a, block);
        case MODE_FUSED:
            return energy ? launch_glist_t<PREC, TPP, MODE_FUSED, true>(s, a, block)
                          : launch_glist_t<PREC, TPP, MODE_FUSED, false>(s, a, block);
        default:
            return launch_glist_t<PREC, TPP, MODE_FINAL, false>(s, a, block);
    }
}

template <int PREC>
static hipError_t launch_glist_p(hipStream_t s, const ForceArgs &a, int tpp, int mode,
                                 bool energy, int block) {
    switch (tpp) {
        case 1: return launch_glist_m<PREC, 1>(s, a, mode, energy, block);
        case 2: return launch_glist_m<PREC, 2>(s, a, mode, energy, block);
        case 4: return launch_glist_m<PREC, 4>(s, a, mode, energy, block);
        case 8: return launch_glist_m<PREC, 8>(s, a, mode, energy, block);
        case 16: return launch_glist_m<PREC, 16>(s, a, mode, energy, block);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_force_glist(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                              bool energy, int block) {
    if (block < 64 || block > 512 || (block & 63)) return hipErrorInvalidValue;
    if (a.max_ntypes < 1 || a.max_ntypes > LJMD_MAX_TYPES_DEVICE) return hipErrorInvalidValue;
    return prec == PREC_MIXED ? launch_glist_p<PREC_MIXED>(s, a, tpp, mode, energy, block)
                              : launch_glist_p<PREC_FP64>(s, a, tpp, mode, energy, block);
}

}  // namespace ljmd
