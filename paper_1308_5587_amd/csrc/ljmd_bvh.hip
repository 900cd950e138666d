// Tree (bounding volume hierarchy) neighbour lists for size-disperse systems (the paper's
// nlist.tree, Section "Performance": a cell list sized for the largest cutoff makes small
// particles scan many cells to find few neighbours).
//
// After the sort of a rebuild (typed sort grid: the particles of each type are contiguous and
// in Morton order of fine cells), every type gets a binary radix tree over its particles built
// by the Karras construction on the unique sorted keys (cell << 32 | index); every internal
// node then stores the boxes of its two children, each the bounding box of the child's
// contiguous leaf range, reduced from per-64 and per-4096-leaf box tables (no atomics and no
// device-wide fences: each node's boxes are formed independently); then each particle
// walks every type's tree with its list radius for that type pair and appends, as 32-bit sorted
// indices, the particles j with r^2 < (r_cut + skin)^2 in the canonical FP64 arithmetic. The
// walk order is fixed by the tree, so the list order is deterministic.
//
// Periodic images: a particle near a face also walks the tree with its position shifted by a
// box length (at most 8 images); a leaf is accepted only in the image the minimum image of the
// pair selects, so no pair is listed twice. Compiled with -ffp-contract=off.
#include "ljmd_device.h"

namespace ljmd {

__device__ __forceinline__ bool bvh_go(const BvhArgs &b) {
    return b.reps[0].active && b.go[0] != 0;
}

// Entry k of particle q in the 32-bit list: chunks of 4 entries per lane, lane l holds chunks
// l, l + 2^ls, ...; for chunk index c the lanes of consecutive particles are adjacent.
__device__ __forceinline__ size_t slot32(int q, int k, int npad, int ls) {
    const int sh = 2 + ls;
    return (size_t)((unsigned)k >> sh) * ((size_t)npad << sh) + ((size_t)q << sh) +
           (size_t)(k & ((1 << sh) - 1));
}

// The type of sorted particle i and its type's range [s, e).
__device__ __forceinline__ int bvh_type_range(const BvhArgs &b, int i, int &s, int &e) {
    int t = 0;
    while (t + 1 < b.ntypes && b.cell_start[(t + 1) * b.ncs] <= i) ++t;
    s = b.cell_start[t * b.ncs];
    e = b.cell_start[(t + 1) * b.ncs];
    return t;
}

// The permuted state becomes the main state and the build positions.
__global__ void __launch_bounds__(256) k_bvh_copy(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) atomicAdd(&b.st->builds, 1ull);
    if (q >= b.n) return;
    const double4 x = b.pos_scr[q];
    b.pos[q] = x;
    b.xb[q] = x;
    b.vel[q] = b.vel_scr[q];
    b.img[q] = b.img_scr[q];
}

// Length of the common prefix of the keys of local leaves i and j of a type's range, or -1
// when j is outside it. Keys (cell << 32 | global index) are unique and sorted.
__device__ __forceinline__ int bvh_delta(const BvhArgs &b, int s, int nt, int i, int j) {
    if (j < 0 || j >= nt) return -1;
    const unsigned long long ki = ((unsigned long long)(unsigned)b.cell_of[s + i] << 32) |
                                  (unsigned)(s + i);
    const unsigned long long kj = ((unsigned long long)(unsigned)b.cell_of[s + j] << 32) |
                                  (unsigned)(s + j);
    return __clzll((long long)(ki ^ kj));
}

// Internal node i (local to its type's range) of the Karras construction: the direction of
// its range from the prefix lengths to its neighbours, the range's other end by a doubling
// then halving search, and the split where the prefix length drops.
__global__ void __launch_bounds__(256) k_bvh_nodes(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b.n) return;
    int s, e;
    bvh_type_range(b, g, s, e);
    const int nt = e - s;
    const int i = g - s;
    if (i >= nt - 1) return;  // a one-particle type has no internal node
    const int node = s + i;
    const int dr = bvh_delta(b, s, nt, i, i + 1), dl = bvh_delta(b, s, nt, i, i - 1);
    const int d = dr > dl ? 1 : -1;
    const int dmin = d > 0 ? dl : dr;
    int lmax = 2;
    while (bvh_delta(b, s, nt, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (bvh_delta(b, s, nt, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = bvh_delta(b, s, nt, i, j);
    int sp = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (bvh_delta(b, s, nt, i, i + (sp + t) * d) > dnode) sp += t;
    } while (t > 1);
    const int gamma = i + sp * d + (d < 0 ? -1 : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    b.left[node] = lo == gamma ? ((s + gamma) | BVH_LEAF) : s + gamma;
    b.right[node] = hi == gamma + 1 ? ((s + gamma + 1) | BVH_LEAF) : s + gamma + 1;
    b.rlo[node] = s + lo;
    b.rsplit[node] = s + gamma;
    b.rhi[node] = s + hi;
}

// Box tables over the build positions in sorted order: blk[k] bounds leaves [64k, 64k + 64)
// (one wavefront per block, shuffle reductions), sblk[k] bounds leaves [4096k, 4096k + 4096)
// (one wavefront per 64 blocks). A block may straddle two types' ranges; a node's range query
// uses only the blocks that lie inside it.
__device__ __forceinline__ void wave_minmax(double lo[3], double hi[3]) {
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
        }
}

__global__ void __launch_bounds__(256) k_bvh_blocks(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = g >> 6;
    if (k >= (b.n + 63) / 64) return;  // whole wavefronts: 64 divides the workgroup
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (g < b.n) {
        const double4 x = b.xb[g];
        lo[0] = hi[0] = x.x;
        lo[1] = hi[1] = x.y;
        lo[2] = hi[2] = x.z;
    }
    wave_minmax(lo, hi);
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            b.blk[6 * (size_t)k + a] = lo[a];
            b.blk[6 * (size_t)k + 3 + a] = hi[a];
        }
}

__global__ void __launch_bounds__(256) k_bvh_sblocks(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = (b.n + 63) / 64;
    const int k = g >> 6;
    if (k >= (b.n + 4095) / 4096) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (g < nb)
        for (int a = 0; a < 3; ++a) {
            lo[a] = b.blk[6 * (size_t)g + a];
            hi[a] = b.blk[6 * (size_t)g + 3 + a];
        }
    wave_minmax(lo, hi);
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            b.sblk[6 * (size_t)k + a] = lo[a];
            b.sblk[6 * (size_t)k + 3 + a] = hi[a];
        }
}

// The bounding box of the build positions of sorted leaves [i, e]: single leaves up to a block
// boundary, whole blocks up to a 4096 boundary, whole 4096-blocks, then blocks and leaves
// again (at most 63 + 63 + n/4096 + 63 + 63 reads). Minimum and maximum are exact, so this is
// the box of the range itself.
__device__ __forceinline__ void range_box(const BvhArgs &b, int i, int e, double *out) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    auto leaf = [&](int k) {
        const double4 x = b.xb[k];
        const double c[3] = {x.x, x.y, x.z};
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], c[a]);
            hi[a] = fmax(hi[a], c[a]);
        }
    };
    auto box = [&](const double *t) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], t[a]);
            hi[a] = fmax(hi[a], t[3 + a]);
        }
    };
    while (i <= e && (i & 63)) leaf(i++);
    while (i + 63 <= e && (i & 4095)) {
        box(b.blk + 6 * (size_t)(i >> 6));
        i += 64;
    }
    while (i + 4095 <= e) {
        box(b.sblk + 6 * (size_t)(i >> 12));
        i += 4096;
    }
    while (i + 63 <= e) {
        box(b.blk + 6 * (size_t)(i >> 6));
        i += 64;
    }
    while (i <= e) leaf(i++);
    for (int a = 0; a < 3; ++a) {
        out[a] = lo[a];
        out[3 + a] = hi[a];
    }
}

// Each internal node's record (BvhNode): per child, a leaf's exact build position or an
// internal child's box rounded outwards to FP32, the box of its leaf range [rlo, rsplit] on
// the left and [rsplit + 1, rhi] on the right; then the child codes. A walk reads one 64-byte
// record per node it opens and tests both children from it.
__global__ void __launch_bounds__(256) k_bvh_boxes(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b.n) return;
    int s, e;
    bvh_type_range(b, g, s, e);
    if (g - s >= e - s - 1) return;  // the type's last leaf index has no internal node
    BvhNode nd;
    nd.left = b.left[g];
    nd.right = b.right[g];
    nd.pad[0] = nd.pad[1] = 0;
    const int sp = b.rsplit[g];
    const int code[2] = {nd.left, nd.right};
    const int lo[2] = {b.rlo[g], sp + 1}, hi[2] = {sp, b.rhi[g]};
    for (int u = 0; u < 2; ++u) {
        if (code[u] & BVH_LEAF) {
            const double4 x = b.xb[code[u] & ~BVH_LEAF];
            nd.child[u].pos[0] = x.x;
            nd.child[u].pos[1] = x.y;
            nd.child[u].pos[2] = x.z;
        } else {
            double bx[6];
            range_box(b, lo[u], hi[u], bx);
            for (int a = 0; a < 3; ++a) {
                nd.child[u].box[a] = __double2float_rd(bx[a]);
                nd.child[u].box[3 + a] = __double2float_ru(bx[3 + a]);
            }
        }
    }
    b.node[g] = nd;
}

// Squared distance from q to a box (0 inside).
__device__ __forceinline__ double box_dist2(const double q[3], const double lo[3],
                                            const double hi[3]) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double d = q[a] < lo[a] ? lo[a] - q[a] : (q[a] > hi[a] ? q[a] - hi[a] : 0.0);
        d2 = __builtin_fma(d, d, d2);
    }
    return d2;
}

// The image the branch-form minimum image of d picks: +1 when d >= L/2 (x_j lies near
// x_i + L), -1 when d < -L/2, else 0; and the minimum-image difference.
__device__ __forceinline__ int mi_side(double d, double L, double &out) {
    const double h = 0.5 * L;
    if (d >= h) {
        out = d - L;
        return 1;
    }
    if (d < -h) {
        out = d + L;
        return -1;
    }
    out = d;
    return 0;
}

// A leaf j at (xjx, xjy, xjz) seen from particle p at xi in the image (sx, sy, sz): listed when
// the minimum image of the pair is that image and the canonical squared distance is below rl2.
__device__ __forceinline__ void try_leaf(const double4 &xi, double xjx, double xjy, double xjz,
                                         int j, int sx, int sy, int sz, double rl2,
                                         const RepParams &P, const BvhArgs &b, int p, int &count) {
    double dx, dy, dz;
    const int kx = mi_side(xjx - xi.x, P.L[0], dx);
    const int ky = mi_side(xjy - xi.y, P.L[1], dy);
    const int kz = mi_side(xjz - xi.z, P.L[2], dz);
    if (kx != sx || ky != sy || kz != sz) return;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const double r2 = (xx + yy) + zz;
    if (r2 < rl2) {
        if (count < b.cap) b.nlist32[slot32(p, count, b.npad, b.lshift)] = j;
        ++count;
    }
}

// One thread per particle: every type's tree, in every periodic image the particle's list
// sphere reaches, in a fixed depth-first order.
__global__ void __launch_bounds__(256) k_bvh_list(const BvhArgs b) {
    if (!bvh_go(b)) return;
    const RepParams &P = b.reps[0];
    // thread g takes the g-th particle of the types' ranges in type_order
    int p = b.n;
    {
        int g = blockIdx.x * blockDim.x + threadIdx.x;
        for (int k = 0; k < b.ntypes; ++k) {
            const int t = b.type_order[k];
            const int s = b.cell_start[t * b.ncs], e = b.cell_start[(t + 1) * b.ncs];
            if (g < e - s) {
                p = s + g;
                break;
            }
            g -= e - s;
        }
    }
    int count = 0;
    if (p < b.n) {
        const double4 xi = b.xb[p];
        const int ti = (int)xi.w;
        const double xq[3] = {xi.x, xi.y, xi.z};
        // depth-first walk: the stack never holds more than the tree depth + 1 nodes, and the
        // depth is at most the number of key bits that vary (cells < 2^22, indices < 2^26)
        int stack[BVH_STACK];
        for (int t = 0; t < b.ntypes; ++t) {
            const double rl2 = b.rl2_table[ti * b.ntypes + t];
            const int s = b.cell_start[t * b.ncs], e = b.cell_start[(t + 1) * b.ncs];
            if (!(rl2 > 0.0) || e <= s) continue;
            const double rl = sqrt(rl2);
            // box test with a relative margin: a box is never skipped for rounding
            const double rl2_box = rl2 * (1.0 + 1e-12) + 1e-300;
            const int root = (e - s == 1) ? (s | BVH_LEAF) : s;
            int lo_img[3], hi_img[3];
            for (int a = 0; a < 3; ++a) {
                lo_img[a] = xq[a] >= P.L[a] - rl ? -1 : 0;
                hi_img[a] = xq[a] < rl ? 1 : 0;
            }
            for (int sx = lo_img[0]; sx <= hi_img[0]; ++sx)
                for (int sy = lo_img[1]; sy <= hi_img[1]; ++sy)
                    for (int sz = lo_img[2]; sz <= hi_img[2]; ++sz) {
                        const double q[3] = {xq[0] + sx * P.L[0], xq[1] + sy * P.L[1],
                                             xq[2] + sz * P.L[2]};
                        if (root & BVH_LEAF) {  // a one-particle tree
                            const int j = root & ~BVH_LEAF;
                            if (j != p) {
                                const double4 xj = b.xb[j];
                                try_leaf(xi, xj.x, xj.y, xj.z, j, sx, sy, sz, rl2, P, b, p, count);
                            }
                            continue;
                        }
                        // the next node to open is kept in a register: a descent needs no stack
                        // round trip; the right child waits on the stack while the left
                        // subtree is walked (the same depth-first order as pushing both)
                        int top = 0;
                        int c = root;
                        while (true) {
                            if (c < 0) {
                                if (top == 0) break;
                                c = stack[--top];
                            }
                            const BvhNode nd = b.node[c];
                            const int ch[2] = {nd.left, nd.right};
                            // leaves are tested at once, in child order
                            for (int u = 0; u < 2; ++u) {
                                if (!(ch[u] & BVH_LEAF)) continue;
                                const int j = ch[u] & ~BVH_LEAF;
                                if (j == p) continue;
                                try_leaf(xi, nd.child[u].pos[0], nd.child[u].pos[1],
                                         nd.child[u].pos[2], j, sx, sy, sz, rl2, P, b, p, count);
                            }
                            bool go[2];
                            for (int u = 0; u < 2; ++u) {
                                const float *f = nd.child[u].box;
                                const double lo[3] = {(double)f[0], (double)f[1], (double)f[2]};
                                const double hi[3] = {(double)f[3], (double)f[4], (double)f[5]};
                                go[u] = !(ch[u] & BVH_LEAF) && box_dist2(q, lo, hi) <= rl2_box;
                            }
                            if (go[0]) {
                                if (go[1] && top < BVH_STACK) stack[top++] = ch[1];
                                c = ch[0];
                            } else {
                                c = go[1] ? ch[1] : -1;
                            }
                        }
                    }
        }
        b.nl_count[p] = count;
        if (count > b.cap) atomicOr(&b.st->status, ST_OVERFLOW);
    }
    // build statistics, reduced over the workgroup: one atomic add per workgroup, an atomic
    // max only where its longest list beats the recorded one (atomics on one word from every
    // wavefront serialise, and a wavefront retires only once its atomics are acknowledged)
    int mx = count;
    unsigned long long ent = (unsigned long long)(count < b.cap ? count : b.cap);
    for (int o = 32; o > 0; o >>= 1) {
        const int om = __shfl_xor(mx, o);
        mx = om > mx ? om : mx;
        ent += __shfl_xor(ent, o);
    }
    __shared__ int s_mx[4];
    __shared__ unsigned long long s_ent[4];
    if ((threadIdx.x & 63) == 0) {
        s_mx[threadIdx.x >> 6] = mx;
        s_ent[threadIdx.x >> 6] = ent;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            mx = s_mx[w] > mx ? s_mx[w] : mx;
            ent += s_ent[w];
        }
        if (mx > __hip_atomic_load(&b.st->max_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&b.st->max_count, mx);
        if (ent) atomicAdd(&b.st->entries, ent);
    }
}

hipError_t launch_rebuild_bvh(hipStream_t s, const RebuildArgs &a, const BvhArgs &b,
                              hipEvent_t *ev) {
    hipError_t e = launch_sort_cells(s, a, ev);
    if (e != hipSuccess) return e;
    const int g = (b.n + 255) / 256;
    const int nb = (b.n + 63) / 64;
    hipLaunchKernelGGL(k_bvh_copy, dim3(g), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bvh_nodes, dim3(g), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bvh_blocks, dim3((nb + 3) / 4), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bvh_sblocks, dim3(((b.n + 4095) / 4096 + 3) / 4), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bvh_boxes, dim3(g), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bvh_list, dim3(g), dim3(256), 0, s, b);
    if (ev) (void)hipEventRecord(ev[5], s);
    return hipGetLastError();
}

}  // namespace ljmd
