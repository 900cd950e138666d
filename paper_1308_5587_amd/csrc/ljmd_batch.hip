// Batched replicas: many independent LJ systems of uneven size advanced together, with
// continuous admission and retirement (the batch C ABI of include/ljmd.h).
//
// Layout. All replicas share one set of device arrays: replica r owns the particle slots
// [poff, poff + n), the cell entries [coff, coff + ncell] (ncell + 1: the cell-start scan
// writes an end marker), the bricks [boff, boff + nbrick) and the pair rows
// [pair_off, pair_off + ntypes^2), all recorded in its RepParams row. Per-particle and per-
// cell replica tags (prep, crep; -1 for a free slot) and BrickInfo::rep route every thread
// to its replica's parameters, so one launch of each kernel serves all replicas, and each
// replica runs exactly the arithmetic it would run alone.
//
// Phase. Between blocks every running replica sits in the middle of a step: positions
// x(t+1) and velocities v(t+1/2) after the kick-drift, with a list valid for x(t+1). A block
// is block_steps fused units (force, second half kick, next kick-drift, rebuild request)
// each followed by the gated rebuild, captured in one HIP graph. A per-replica counter of
// steps left (two words, one per position buffer) makes the fused kernel stop a replica
// exactly at its count: the last step ends with the forces and full-step velocities and
// no drift, after which the replica idles until it is retired.
//
// Recovery. The state of every replica is snapshotted before a block. A replica whose list
// overflowed during the block is restored, its list is rebuilt with a larger capacity and
// the block is run again for it alone (the others keep their results: the list slot of an
// entry does not depend on the capacity, so growing the list buffer keeps their lists). A
// replica whose forces became non-finite is restored and retired with an error.
#include "ljmd_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace ljmd;

// Staging of ljmd_batch_read_noalloc: a file-scope device array, so that the call allocates
// nothing. Each GPU the library runs on holds its own copy until the process ends. In host
// code the name `scratch` is only a stand-in: its device address is taken once per device with
// hipGetSymbolAddress (scratch_address) and only that address is passed to kernels and copies.
constexpr size_t NOALLOC_STAGE_BYTES = (size_t)8 << 20;
constexpr size_t NOALLOC_STAGE_DOUBLES = NOALLOC_STAGE_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[NOALLOC_STAGE_DOUBLES];

namespace {

constexpr int PAIR_ROWS = LJMD_MAX_TYPES * LJMD_MAX_TYPES;  // pair rows reserved per slot

// Device bytes per particle slot: positions x2, scratch, velocities, scratch, forces, build
// positions (7 x 32), image counters and scratch (2 x 16), key/slot/perm/prep/count (5 x 4),
// work order (2),
// energy, virial and kinetic per particle (8 + 48 + 8), the block snapshot (2 x 32 + 16).
constexpr int64_t PER_PARTICLE = 7 * 32 + 2 * 16 + 5 * 4 + 2 + 64 + 2 * 32 + 16;
// per cell entry: rank, xyz, count, start, lower-half count, replica tag
constexpr int64_t PER_CELL = 6 * 4;
// per brick: BrickInfo, halo cells, tile table
constexpr int64_t PER_BRICK = (int64_t)sizeof(BrickInfo) + HALO_MAX * (int64_t)sizeof(HaloCell) +
                              TILE_TAB * 4;

// First-fit allocator of index ranges in [0, capacity).
struct RangeAlloc {
    int capacity = 0;
    std::map<int, int> free_;  // offset -> length

    void init(int cap) {
        capacity = cap;
        free_.clear();
        if (cap > 0) free_[0] = cap;
    }
    bool get(int len, int *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= len) {
                *off = it->first;
                const int rest = it->second - len;
                const int roff = it->first + len;
                free_.erase(it);
                if (rest > 0) free_[roff] = rest;
                return true;
            }
        return false;
    }
    void put(int off, int len) {
        if (len <= 0) return;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    // one past the last used index
    int high_water() const {
        if (free_.empty()) return capacity;
        auto last = std::prev(free_.end());
        return last->first + last->second == capacity ? last->first : capacity;
    }
};

struct Slot {
    bool used = false;
    bool done = false;
    int error = LJMD_OK;    // non-zero: retired with this status
    int64_t nsteps = 0;
    int64_t rem = 0;        // steps left (mirror of the device counter at block start)
    int poff = 0, n = 0, coff = 0, ncell = 0, boff = 0, nbrick = 0;
    int ntypes = 1;
    int64_t bytes = 0;
    RepParams P{};
};

struct GraphKey {
    int cur, p_ext, c_ext, b_ext, cap, tpp, block, tile_cap, max_ntypes, steps;
    void *nlist;
    bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof *this) == 0; }
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

struct ljmd_batch {
    ljmd_batch_config cfg{};
    hipStream_t stream = nullptr, cap_stream = nullptr;
    DeviceArena mem;
    int device = 0;
    size_t lds_limit = 64 * 1024;
    int prec = PREC_FP64;
    int max_slots = 0;
    int p_cap = 0, npad = 0, c_cap = 0, b_cap = 0;
    RangeAlloc palloc, calloc_, balloc;
    int p_ext = 0, c_ext = 0, b_ext = 0;
    int cap = 0, cap_assumed = 128;
    int tpp = 0, lshift = 0, block = 0, tile_cap = 64, max_ntypes = 1;
    bool layout_fixed = false;  // lanes and workgroup size final (after the first block)
    int block_steps = 100;
    int cur = 0;
    int64_t used_bytes = 0;
    std::vector<Slot> slots;
    std::vector<int> h_status, h_mask;
    // device arrays
    RepParams *d_reps = nullptr;
    PairCoef *d_pair = nullptr;
    double *d_rl2 = nullptr;
    int *d_req = nullptr, *d_rem = nullptr, *d_only = nullptr, *d_go = nullptr,
        *d_rep_status = nullptr;
    int *d_prep = nullptr, *d_crep = nullptr;
    int *d_cell_rank = nullptr, *d_cell_xyz = nullptr, *d_cell_count = nullptr,
        *d_cell_start = nullptr, *d_cell_lo = nullptr;
    BrickInfo *d_bricks = nullptr;
    HaloCell *d_halo = nullptr;
    int *d_tile_tab = nullptr;
    double4 *d_pos[2]{}, *d_pos_scr = nullptr, *d_vel = nullptr, *d_vel_scr = nullptr,
            *d_force = nullptr, *d_xb = nullptr;
    int4 *d_img = nullptr, *d_img_scr = nullptr;
    int *d_key = nullptr, *d_slot = nullptr, *d_perm = nullptr, *d_count = nullptr;
    uint16_t *d_nlist = nullptr;
    uint16_t *d_work = nullptr;
    size_t nlist_alloc = 0;
    double *d_u = nullptr, *d_w = nullptr, *d_ke = nullptr, *d_partials = nullptr,
           *d_red = nullptr;
    double *d_stage = nullptr;
    size_t stage_alloc = 0;  // doubles
    double *d_noalloc_stage = nullptr;  // this device's `scratch` (NOALLOC_STAGE_DOUBLES)
    double4 *d_snap_pos = nullptr, *d_snap_vel = nullptr;
    int4 *d_snap_img = nullptr;
    DevStatus *d_st = nullptr;
    hipGraphExec_t graph = nullptr;
    GraphKey gkey{};
    int red_blocks = 1024;
    int64_t blocks = 0, overflow_reruns = 0;
};

namespace {

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_addr;  // device -> address of its copy of `scratch`

// The device address of `scratch` on device `dev` (the current device), resolved once per
// device.
int scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return LJMD_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_err(LJMD_E_DEVICE, "address of the no-allocation staging array on device %d: %s",
                       dev, hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<double *>(p);
    *out = static_cast<double *>(p);
    return LJMD_OK;
}

}  // namespace

namespace {

int launch_chk(hipError_t e, const char *what) {
    if (e != hipSuccess) return set_err(LJMD_E_DEVICE, "launch of %s: %s", what, hipGetErrorString(e));
    return LJMD_OK;
}

void drop_graph(ljmd_batch *b) {
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
}

int sync(ljmd_batch *b) {
    HIPCHK(hipStreamSynchronize(b->stream));
    return LJMD_OK;
}

// The pair table and cell grid of a replica request, validated.
int describe(const ljmd_batch *b, const ljmd_replica_spec *sp, PairTable *pt, ReplicaGrid *g) {
    if (!sp) return set_err(LJMD_E_INVAL, "null replica spec");
    if (sp->n < 1 || sp->n > (int64_t)(1 << 24))
        return set_err(LJMD_E_INVAL, "replica n = %lld out of range", (long long)sp->n);
    if (!sp->pos || !sp->vel || !sp->eps || !sp->sigma || !sp->r_cut)
        return set_err(LJMD_E_INVAL, "replica arrays must not be NULL (type may be)");
    if (sp->ntypes < 1 || sp->ntypes > LJMD_MAX_TYPES)
        return set_err(LJMD_E_INVAL, "ntypes = %d out of range [1, %d]", sp->ntypes, LJMD_MAX_TYPES);
    if (sp->nsteps < 1 || sp->nsteps > 2000000000LL)
        return set_err(LJMD_E_INVAL, "nsteps must be in [1, 2e9]");
    for (int a = 0; a < 3; ++a)
        if (!(sp->box[a] > 0.0) || !std::isfinite(sp->box[a]))
            return set_err(LJMD_E_INVAL, "box edge %d must be finite and > 0", a);
    const int nt = sp->ntypes;
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < nt; ++j) {
            const int k = i * nt + j, kt = j * nt + i;
            const double e = sp->eps[k], s = sp->sigma[k], r = sp->r_cut[k];
            if (!std::isfinite(e) || !(s > 0.0) || !std::isfinite(s) || !(r >= 0.0) || !std::isfinite(r))
                return set_err(LJMD_E_INVAL, "pair (%d,%d): need finite epsilon, sigma > 0, r_cut >= 0", i, j);
            if (e != sp->eps[kt] || s != sp->sigma[kt] || r != sp->r_cut[kt])
                return set_err(LJMD_E_INVAL, "pair table is not symmetric at (%d,%d)", i, j);
        }
    make_pair_table(nt, sp->eps, sp->sigma, sp->r_cut, b->cfg.skin, pt);
    return make_grid(sp->box, pt->rl_max, g, sp->n,
                     tile_limit_for(std::max(b->max_ntypes, sp->ntypes), b->lds_limit));
}

// list entries a replica is expected to need: neighbours within the largest list radius at
// its mean density, with headroom
int expected_cap(const ljmd_replica_spec *sp, double rl_max) {
    const double vol = sp->box[0] * sp->box[1] * sp->box[2];
    const double nbar = sp->n / vol * 4.18879020478639 * rl_max * rl_max * rl_max;
    const double c = std::min(1.3 * nbar + 24.0, (double)std::max<int64_t>(16, (sp->n + 15) & ~15));
    return std::max(8, (int)std::ceil(c));
}

int64_t footprint(const ljmd_batch *b, int64_t n, int ncell, int nbrick) {
    return n * (PER_PARTICLE + 2 * (int64_t)b->cap_assumed) + (int64_t)(ncell + 1) * PER_CELL +
           (int64_t)nbrick * PER_BRICK;
}

// Capacity of the list (entries per particle), rounded to whole chunks of 8 per lane. The
// slot of entry k does not depend on the capacity, so the old buffer's contents are kept.
int grow_list(ljmd_batch *b, int want) {
    // the list build addresses rounds of 8 x lanes entries with a 32-bit stride
    if (((uint64_t)b->npad << (3 + b->lshift)) > 0xFFFFFFFFull)
        return set_err(LJMD_E_INVAL, "%d lanes per particle is too many for %d particle slots",
                       1 << b->lshift, b->p_cap);
    const int unit = 8 << b->lshift;
    want = std::max(unit, round_up(want, unit));
    if (want <= b->cap && b->d_nlist) return LJMD_OK;
    want = std::max(want, b->cap);
    const size_t need = (size_t)want * (size_t)b->npad;
    if (need > b->nlist_alloc) {
        uint16_t *nl = nullptr;
        CHK(b->mem.get_t(&nl, need));
        if (b->d_nlist) {
            HIPCHK(hipMemcpyAsync(nl, b->d_nlist, (size_t)b->cap * b->npad * sizeof(uint16_t),
                                  hipMemcpyDeviceToDevice, b->stream));
            CHK(sync(b));
            b->mem.put(b->d_nlist);
        }
        b->d_nlist = nl;
        b->nlist_alloc = need;
    }
    b->cap = want;
    drop_graph(b);
    return LJMD_OK;
}

int ensure_stage(ljmd_batch *b, size_t doubles) {
    if (doubles <= b->stage_alloc) return LJMD_OK;
    CHK(sync(b));
    b->mem.put(b->d_stage);
    b->d_stage = nullptr;
    b->stage_alloc = 0;
    CHK(b->mem.get_t(&b->d_stage, doubles));
    b->stage_alloc = doubles;
    return LJMD_OK;
}

// Launch extents: the high-water mark of each range allocator rounded up to a power of two
// (at least a minimum), so that the block graph is captured again only when an extent doubles
// or halves.
int pow2_extent(int hw, int lo, int cap) {
    int e = lo;
    while (e < hw && e < cap) e <<= 1;
    return std::min(e, cap);
}

void update_extents(ljmd_batch *b) {
    const int pe = pow2_extent(b->palloc.high_water(), 4096, b->p_cap);
    const int ce = pow2_extent(b->calloc_.high_water(), 1024, b->c_cap);
    const int be = pow2_extent(b->balloc.high_water(), 256, b->b_cap);
    if (pe != b->p_ext || ce != b->c_ext || be != b->b_ext) drop_graph(b);
    b->p_ext = pe;
    b->c_ext = ce;
    b->b_ext = be;
}

// ------------------------------------------------------------ argument blocks

RebuildArgs rebuild_args(ljmd_batch *b, const int *go, int go_stride, int cur) {
    RebuildArgs a{};
    a.reps = b->d_reps;
    a.prep = b->d_prep;
    a.crep = b->d_crep;
    a.go = go;
    a.go_stride = go_stride;
    a.rl2_table = b->d_rl2;
    a.pos = b->d_pos[cur];
    a.pos_scr = b->d_pos_scr;
    a.vel = b->d_vel;
    a.vel_scr = b->d_vel_scr;
    a.img = b->d_img;
    a.img_scr = b->d_img_scr;
    a.xb = b->d_xb;
    a.key = b->d_key;
    a.slot = b->d_slot;
    a.perm = b->d_perm;
    a.cell_count = b->d_cell_count;
    a.cell_start = b->d_cell_start;
    a.cell_lo = b->d_cell_lo;
    a.cell_rank = b->d_cell_rank;
    a.cell_xyz = b->d_cell_xyz;
    a.nl_count = b->d_count;
    a.nlist = b->d_nlist;
    a.work = b->d_work;
    a.bricks = b->d_bricks;
    a.halo = b->d_halo;
    a.tile_tab = b->d_tile_tab;
    a.st = b->d_st;
    a.rep_status = b->d_rep_status;
    a.n = b->p_ext;
    a.ncell = b->c_ext;
    a.nbrick = b->b_ext;
    a.nrep = b->max_slots;
    a.npad = b->npad;
    a.cap = b->cap;
    a.lshift = b->lshift;
    a.tile_cap = b->tile_cap;
    a.max_ntypes = b->max_ntypes;
    return a;
}

ForceArgs force_args(ljmd_batch *b, int cur, const int *only, bool with_rem) {
    ForceArgs a{};
    a.reps = b->d_reps;
    a.pos_in = b->d_pos[cur];
    a.pos_out = b->d_pos[cur ^ 1];
    a.vel = b->d_vel;
    a.img = b->d_img;
    a.xb = b->d_xb;
    a.force = b->d_force;
    a.nl_count = b->d_count;
    a.nlist = b->d_nlist;
    a.work = b->d_work;
    a.bricks = b->d_bricks;
    a.cell_start = b->d_cell_start;
    a.tile_tab = b->d_tile_tab;
    a.u_out = b->d_u;
    a.w_out = b->d_w;
    a.ke_out = b->d_ke;
    a.pair = b->d_pair;
    a.req = b->d_req;
    a.rem = with_rem ? b->d_rem : nullptr;
    a.only = only;
    a.status = &b->d_st->status;
    a.rep_status = b->d_rep_status;
    a.cur = cur;
    a.npad = b->npad;
    a.cap = b->cap;
    a.lshift = b->lshift;
    a.nbrick = b->b_ext;
    a.tile_cap = b->tile_cap;
    a.max_ntypes = b->max_ntypes;
    return a;
}

// mask[r] = 1 for r == slot, else 0 (slot < 0: all zero)
int set_single_mask(ljmd_batch *b, int *mask, int slot) {
    CHK(launch_chk(launch_fill_int(b->stream, mask, b->max_slots, 0), "fill"));
    if (slot >= 0) CHK(launch_chk(launch_fill_int(b->stream, mask + slot, 1, 1), "fill"));
    return LJMD_OK;
}

int upload_mask(ljmd_batch *b, int *mask, const std::vector<int> &h) {
    HIPCHK(hipMemcpyAsync(mask, h.data(), sizeof(int) * b->max_slots, hipMemcpyHostToDevice, b->stream));
    return sync(b);  // the host vector may change after this
}

int write_params(ljmd_batch *b, int s) {
    HIPCHK(hipMemcpyAsync(b->d_reps + s, &b->slots[s].P, sizeof(RepParams), hipMemcpyHostToDevice,
                          b->stream));
    return sync(b);  // the host row may change after this
}

int read_status(ljmd_batch *b) {
    HIPCHK(hipMemcpyAsync(b->h_status.data(), b->d_rep_status, sizeof(int) * b->max_slots,
                          hipMemcpyDeviceToHost, b->stream));
    if (LJMD_DEBUG_CHECKS) {
        // the device checks of a debug build report through the batch's status block
        DevStatus st{};
        HIPCHK(hipMemcpyAsync(&st, b->d_st, sizeof st, hipMemcpyDeviceToHost, b->stream));
        CHK(sync(b));
        if (st.status & ST_DEBUG)
            return set_err(LJMD_E_DEVICE, "device check %d failed (debug build)", st.debug);
        return LJMD_OK;
    }
    return sync(b);
}

int clear_status(ljmd_batch *b) {
    HIPCHK(hipMemsetAsync(b->d_rep_status, 0, sizeof(int) * b->max_slots, b->stream));
    HIPCHK(hipMemsetAsync(&b->d_st->status, 0, 2 * sizeof(int), b->stream));
    return LJMD_OK;
}

// Unconditional rebuild of the replicas in d_go at the current positions, growing the list
// until it fits. Returns E_BOX for a tile beyond 16-bit indices.
int forced_rebuild(ljmd_batch *b, const std::vector<int> &which) {
    for (int attempt = 0; attempt < 8; ++attempt) {
        CHK(clear_status(b));
        CHK(launch_chk(launch_rebuild(b->stream, rebuild_args(b, b->d_go, 1, b->cur)), "rebuild"));
        CHK(read_status(b));
        bool over = false;
        for (int s : which) {
            if (b->h_status[s] & ST_TILE)
                return set_err(LJMD_E_BOX, "a brick of replica %d holds more than %d atoms in its "
                                           "halo cells", s, TILE_INDEX_MAX);
            over |= (b->h_status[s] & ST_OVERFLOW) != 0;
        }
        if (!over) return LJMD_OK;
        DevStatus st{};
        HIPCHK(hipMemcpyAsync(&st, b->d_st, sizeof st, hipMemcpyDeviceToHost, b->stream));
        CHK(sync(b));
        CHK(grow_list(b, (int)std::ceil(1.25 * st.max_count + 8)));
    }
    return set_err(LJMD_E_DEVICE, "neighbour list did not fit after repeated growth");
}

double time_evals(ljmd_batch *b, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    const ForceArgs fa = force_args(b, b->cur, b->d_only, false);
    bool ok = true;
    for (int r = 0; r < 3 && ok; ++r)
        ok = launch_force(b->stream, fa, b->prec, b->tpp, MODE_EVAL, false, b->block) == hipSuccess;
    double best = 1e30;
    if (ok) {
        (void)hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && ok; ++r)
            ok = launch_force(b->stream, fa, b->prec, b->tpp, MODE_EVAL, false, b->block) == hipSuccess;
        (void)hipEventRecord(e1, b->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

void set_tpp(ljmd_batch *b, int t) {
    b->tpp = t;
    for (b->lshift = 0; (1 << b->lshift) < t; ++b->lshift) {}
}

// Lanes per particle and workgroup size, timed on the force evaluation of the replicas in
// `which` (d_go and d_only select them). Each lane count needs its own list layout, so the
// lists of those replicas are rebuilt for every trial and once more for the choice; a rebuild
// at fixed positions is valid at any time (it only moves the next rebuild).
int tune(ljmd_batch *b, const std::vector<int> &which) {
    const int want_tpp = b->cfg.threads_per_particle, want_block = b->cfg.block_size;
    const int tpps[] = {1, 2, 4, 8};
    const int blocks[] = {128, 192, 256, 320, 384, 448, 512};
    double best = 1e30;
    int bt = want_tpp ? want_tpp : 2, bb = want_block ? want_block : 256;
    for (int t : tpps) {
        if (want_tpp && t != want_tpp) continue;
        int ls = 0;
        while ((1 << ls) < t) ++ls;
        if (((uint64_t)b->npad << (3 + ls)) > 0xFFFFFFFFull) continue;
        set_tpp(b, t);
        CHK(grow_list(b, b->cap));
        CHK(forced_rebuild(b, which));
        for (int k : blocks) {
            if (want_block && k != want_block) continue;
            b->block = k;
            const double ms = time_evals(b, 5);
            if (ms < best) {
                best = ms;
                bt = t;
                bb = k;
            }
        }
    }
    set_tpp(b, bt);
    b->block = bb;
    CHK(grow_list(b, b->cap));
    CHK(forced_rebuild(b, which));
    drop_graph(b);
    return LJMD_OK;
}

int release_slot(ljmd_batch *b, int s) {
    Slot &sl = b->slots[s];
    if (!sl.used) return LJMD_OK;
    sl.P.active = 0;
    CHK(write_params(b, s));
    CHK(launch_chk(launch_fill_int(b->stream, b->d_prep + sl.poff, sl.n, -1), "fill"));
    CHK(launch_chk(launch_fill_int(b->stream, b->d_crep + sl.coff, sl.ncell + 1, -1), "fill"));
    CHK(launch_chk(launch_fill_int(b->stream, reinterpret_cast<int *>(b->d_bricks + sl.boff),
                                   sl.nbrick * (int)(sizeof(BrickInfo) / sizeof(int)), -1),
                   "fill"));
    CHK(sync(b));
    b->palloc.put(sl.poff, sl.n);
    b->calloc_.put(sl.coff, sl.ncell + 1);
    b->balloc.put(sl.boff, sl.nbrick);
    b->used_bytes -= sl.bytes;
    sl = Slot{};
    update_extents(b);
    return LJMD_OK;
}

// Snapshot of every particle slot in use (one copy per array over the launch extent).
int snapshot_all(ljmd_batch *b) {
    const size_t n = (size_t)b->p_ext;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    HIPCHK(hipMemcpyAsync(b->d_snap_pos, b->d_pos[b->cur], n * sizeof(double4), k, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_snap_vel, b->d_vel, n * sizeof(double4), k, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_snap_img, b->d_img, n * sizeof(int4), k, b->stream));
    return LJMD_OK;
}

// Copy a replica's particle range between the live state and the block snapshot.
int copy_range(ljmd_batch *b, const Slot &sl, bool to_snapshot) {
    const size_t o = (size_t)sl.poff, n = (size_t)sl.n;
    double4 *pos = b->d_pos[b->cur];
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (to_snapshot) {
        HIPCHK(hipMemcpyAsync(b->d_snap_pos + o, pos + o, n * sizeof(double4), k, b->stream));
        HIPCHK(hipMemcpyAsync(b->d_snap_vel + o, b->d_vel + o, n * sizeof(double4), k, b->stream));
        HIPCHK(hipMemcpyAsync(b->d_snap_img + o, b->d_img + o, n * sizeof(int4), k, b->stream));
    } else {
        HIPCHK(hipMemcpyAsync(pos + o, b->d_snap_pos + o, n * sizeof(double4), k, b->stream));
        HIPCHK(hipMemcpyAsync(b->d_vel + o, b->d_snap_vel + o, n * sizeof(double4), k, b->stream));
        HIPCHK(hipMemcpyAsync(b->d_img + o, b->d_snap_img + o, n * sizeof(int4), k, b->stream));
    }
    return LJMD_OK;
}

// One block of fused units starting at buffer cur; only == nullptr runs every replica
// (from the graph when possible), else the masked replicas unit by unit.
int enqueue_block(ljmd_batch *b, hipStream_t st, const int *only) {
    int c = b->cur;
    for (int u = 0; u < b->block_steps; ++u) {
        const ForceArgs fa = force_args(b, c, only, true);
        CHK(launch_chk(launch_force(st, fa, b->prec, b->tpp, MODE_FUSED, false, b->block), "fused step"));
        CHK(launch_chk(launch_rebuild(st, rebuild_args(b, b->d_req + (c ^ 1), 2, c ^ 1)), "rebuild"));
        c ^= 1;
    }
    return LJMD_OK;
}

int ensure_graph(ljmd_batch *b) {
    GraphKey k{};
    std::memset(&k, 0, sizeof k);
    k.cur = b->cur;
    k.p_ext = b->p_ext;
    k.c_ext = b->c_ext;
    k.b_ext = b->b_ext;
    k.cap = b->cap;
    k.tpp = b->tpp;
    k.block = b->block;
    k.tile_cap = b->tile_cap;
    k.max_ntypes = b->max_ntypes;
    k.steps = b->block_steps;
    k.nlist = b->d_nlist;
    if (b->graph && k == b->gkey) return LJMD_OK;
    drop_graph(b);
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_block(b, b->cap_stream, nullptr);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != LJMD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_err(LJMD_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return set_err(LJMD_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    b->gkey = k;
    return LJMD_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int ljmd_batch_create(const ljmd_batch_config *cfg, ljmd_batch **out) {
    if (out) *out = nullptr;
    if (!cfg || !out) return set_err(LJMD_E_INVAL, "null argument");
    if (cfg->max_slots < 1 || cfg->max_slots > 65536)
        return set_err(LJMD_E_INVAL, "max_slots must be in [1, 65536]");
    if (cfg->precision != LJMD_FP64 && cfg->precision != LJMD_MIXED)
        return set_err(LJMD_E_INVAL, "unknown precision %d", cfg->precision);
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return set_err(LJMD_E_INVAL, "dt must be > 0");
    if (!(cfg->skin >= 0.0) || !std::isfinite(cfg->skin)) return set_err(LJMD_E_INVAL, "skin must be >= 0");
    if (cfg->block_steps != 0 && (cfg->block_steps < 2 || cfg->block_steps % 2 || cfg->block_steps > 100000))
        return set_err(LJMD_E_INVAL, "block_steps must be 0 or an even number in [2, 100000]");
    const int tpp = cfg->threads_per_particle;
    if (tpp != 0 && tpp != 1 && tpp != 2 && tpp != 4 && tpp != 8 && tpp != 16)
        return set_err(LJMD_E_INVAL, "threads_per_particle must be 0, 1, 2, 4, 8 or 16");
    if (cfg->block_size != 0 && (cfg->block_size < 64 || cfg->block_size > 512 || cfg->block_size % 64))
        return set_err(LJMD_E_INVAL, "block_size must be 0 or a multiple of 64 up to 512");
    if (cfg->nlist_capacity < 0) return set_err(LJMD_E_INVAL, "nlist_capacity must be >= 0");
    if (!!cfg->alloc != !!cfg->free) return set_err(LJMD_E_INVAL, "alloc and free must be given together");
    const int cap_assumed = cfg->nlist_capacity > 0 ? cfg->nlist_capacity : 128;
    const int64_t per = PER_PARTICLE + 2 * (int64_t)cap_assumed + PER_CELL / 4 + PER_BRICK / 16;
    const int64_t pc = cfg->budget_bytes / per;
    if (pc < 64) return set_err(LJMD_E_INVAL, "budget_bytes too small (%lld)", (long long)cfg->budget_bytes);
    if (pc > (int64_t)(1 << 26)) return set_err(LJMD_E_INVAL, "budget_bytes too large for 2^26 particle slots");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return set_err(LJMD_E_DEVICE, "no HIP device available");

    ljmd_batch *b = new (std::nothrow) ljmd_batch();
    if (!b) return set_err(LJMD_E_NOMEM, "host allocation failed");
    b->cfg = *cfg;
    (void)hipGetDevice(&b->device);
    {
        // once per device, with it current: the address of this device's staging array for
        // ljmd_batch_read_noalloc
        const int rc0 = scratch_address(b->device, &b->d_noalloc_stage);
        if (rc0 != LJMD_OK) {
            delete b;
            return rc0;
        }
    }
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) == hipSuccess && v > 0)
            b->lds_limit = (size_t)v;
    }
    b->stream = (hipStream_t)cfg->stream;
    b->mem.alloc = cfg->alloc;
    b->mem.free = cfg->free;
    b->mem.ctx = cfg->alloc_ctx;
    b->mem.stream = b->stream;
    b->prec = cfg->precision == LJMD_MIXED ? PREC_MIXED : PREC_FP64;
    b->max_slots = cfg->max_slots;
    b->cap_assumed = cap_assumed;
    b->block_steps = cfg->block_steps ? cfg->block_steps : 100;
    b->p_cap = (int)pc;
    b->npad = round_up(b->p_cap, 64);
    b->c_cap = b->p_cap / 4 + 32 * b->max_slots;
    b->b_cap = b->p_cap / 16 + 27 * b->max_slots;
    b->palloc.init(b->p_cap);
    b->calloc_.init(b->c_cap);
    b->balloc.init(b->b_cap);
    b->slots.assign(b->max_slots, Slot{});
    b->h_status.assign(b->max_slots, 0);
    b->h_mask.assign(b->max_slots, 0);
    if (tpp) set_tpp(b, tpp);
    b->block = cfg->block_size;

    const size_t P = (size_t)b->p_cap, C = (size_t)b->c_cap, B = (size_t)b->b_cap;
    const size_t S = (size_t)b->max_slots;
    int rc = LJMD_OK;
    auto get = [&](auto **p, size_t count) {
        if (rc == LJMD_OK) rc = b->mem.get_t(p, count);
    };
    get(&b->d_reps, S);
    get(&b->d_pair, S * PAIR_ROWS);
    get(&b->d_rl2, S * PAIR_ROWS);
    get(&b->d_req, 2 * S);
    get(&b->d_rem, 2 * S);
    get(&b->d_only, S);
    get(&b->d_go, S);
    get(&b->d_rep_status, S);
    get(&b->d_prep, P);
    get(&b->d_crep, C);
    get(&b->d_cell_rank, C);
    get(&b->d_cell_xyz, C);
    get(&b->d_cell_count, C);
    get(&b->d_cell_start, C);
    get(&b->d_cell_lo, C);
    get(&b->d_bricks, B);
    get(&b->d_halo, B * HALO_MAX);
    get(&b->d_tile_tab, B * TILE_TAB);
    get(&b->d_pos[0], P);
    get(&b->d_pos[1], P);
    get(&b->d_pos_scr, P);
    get(&b->d_vel, P);
    get(&b->d_vel_scr, P);
    get(&b->d_force, P);
    get(&b->d_xb, P);
    get(&b->d_img, P);
    get(&b->d_img_scr, P);
    get(&b->d_key, P);
    get(&b->d_slot, P);
    get(&b->d_perm, P);
    get(&b->d_count, (size_t)b->npad);
    get(&b->d_work, P);
    get(&b->d_u, P);
    get(&b->d_w, 6 * P);
    get(&b->d_ke, P);
    get(&b->d_partials, (size_t)RED_QUANT * b->red_blocks);
    get(&b->d_red, (size_t)RED_QUANT);
    get(&b->d_snap_pos, P);
    get(&b->d_snap_vel, P);
    get(&b->d_snap_img, P);
    get(&b->d_st, 1);
    if (rc != LJMD_OK) {
        ljmd_batch_destroy(b);
        return rc;
    }
    // every slot free: replica tags -1, parameter rows inactive, counters zero
    std::vector<RepParams> rows(S);
    for (auto &r : rows) r = RepParams{};
    auto fail = [&](int code) {
        ljmd_batch_destroy(b);
        return code;
    };
    if (hipMemcpyAsync(b->d_reps, rows.data(), S * sizeof(RepParams), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_req, 0, 2 * S * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_rem, 0, 2 * S * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_only, 0, S * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_go, 0, S * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_rep_status, 0, S * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_prep, 0xff, P * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_crep, 0xff, C * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_cell_count, 0, C * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_cell_start, 0, C * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_bricks, 0xff, B * sizeof(BrickInfo), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_count, 0, (size_t)b->npad * sizeof(int), b->stream) != hipSuccess ||
        launch_fill_status(b->stream, b->d_st) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return fail(set_err(LJMD_E_DEVICE, "batch initialisation failed"));
    update_extents(b);
    *out = b;
    return LJMD_OK;
}

void ljmd_batch_destroy(ljmd_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    b->mem.release_all();
    delete b;
}

int ljmd_batch_footprint(const ljmd_batch *b, const ljmd_replica_spec *spec, int64_t *bytes) {
    if (!b || !spec || !bytes) return set_err(LJMD_E_INVAL, "null argument");
    PairTable pt;
    ReplicaGrid g;
    CHK(describe(b, spec, &pt, &g));
    *bytes = footprint(b, spec->n, g.ncell, g.nbrick);
    return LJMD_OK;
}

int ljmd_batch_admit(ljmd_batch *b, const ljmd_replica_spec *sp, int32_t *slot_out) {
    if (slot_out) *slot_out = -1;
    if (!b || !sp || !slot_out) return set_err(LJMD_E_INVAL, "null argument");
    PairTable pt;
    ReplicaGrid g;
    CHK(describe(b, sp, &pt, &g));
    const int n = (int)sp->n, nt = sp->ntypes;
    for (int64_t i = 0; i < 3 * sp->n; ++i)
        if (!std::isfinite(sp->pos[i]) || !std::isfinite(sp->vel[i]))
            return set_err(LJMD_E_INVAL, "non-finite position or velocity");
    if (sp->type)
        for (int64_t i = 0; i < sp->n; ++i)
            if (sp->type[i] < 0 || sp->type[i] >= nt)
                return set_err(LJMD_E_INVAL, "type[%lld] = %d out of range", (long long)i, sp->type[i]);
    const int64_t bytes = footprint(b, sp->n, g.ncell, g.nbrick);
    if (b->used_bytes + bytes > b->cfg.budget_bytes)
        return set_err(LJMD_E_CAPACITY, "replica needs %lld bytes, %lld of the budget left",
                       (long long)bytes, (long long)(b->cfg.budget_bytes - b->used_bytes));
    int s = -1;
    for (int k = 0; k < b->max_slots; ++k)
        if (!b->slots[k].used) {
            s = k;
            break;
        }
    if (s < 0) return set_err(LJMD_E_CAPACITY, "no free slot");
    int poff = 0, coff = 0, boff = 0;
    if (!b->palloc.get(n, &poff)) return set_err(LJMD_E_CAPACITY, "no room for %d particles", n);
    if (!b->calloc_.get(g.ncell + 1, &coff)) {
        b->palloc.put(poff, n);
        return set_err(LJMD_E_CAPACITY, "no room for %d cells", g.ncell);
    }
    if (!b->balloc.get(g.nbrick, &boff)) {
        b->palloc.put(poff, n);
        b->calloc_.put(coff, g.ncell + 1);
        return set_err(LJMD_E_CAPACITY, "no room for %d bricks", g.nbrick);
    }
    Slot &sl = b->slots[s];
    sl = Slot{};
    sl.used = true;
    sl.nsteps = sp->nsteps;
    sl.rem = sp->nsteps;
    sl.poff = poff;
    sl.n = n;
    sl.coff = coff;
    sl.ncell = g.ncell;
    sl.boff = boff;
    sl.nbrick = g.nbrick;
    sl.ntypes = nt;
    sl.bytes = bytes;
    b->used_bytes += bytes;
    update_extents(b);

    RepParams &P = sl.P;
    for (int a = 0; a < 3; ++a) {
        P.L[a] = sp->box[a];
        P.invL[a] = 1.0 / sp->box[a];
        P.inv_w[a] = (double)g.nc[a] / sp->box[a];
        P.nc[a] = g.nc[a];
    }
    P.dt = b->cfg.dt;
    P.half_dt = 0.5 * b->cfg.dt;
    const double lim = 0.5 * b->cfg.skin;
    P.lim2 = lim * lim;
    P.single_rl2 = pt.coef[0].rl2;
    P.poff = poff;
    P.n = n;
    P.coff = coff;
    P.ncell = g.ncell;
    P.boff = boff;
    P.nbrick = g.nbrick;
    P.canonical = g.canonical ? 1 : 0;
    P.ntypes = nt;
    P.pair_off = s * PAIR_ROWS;
    P.active = 1;
    // the capacity the replica would have alone (its own type count): whether a brick's tile
    // is staged is then the same alone and batched
    P.tile_cap = grid_tile_cap(g, n, nt, b->lds_limit);

    // global cell and brick indices of the replica's tables
    for (auto &r : g.rank) r += coff;
    for (auto &br : g.bricks) {
        br.first_cell += coff;
        br.rep = s;
    }
    for (auto &h : g.halo) h.rank += coff;
    // layout-wide settings that depend on the replicas present
    const int old_ntypes = b->max_ntypes;
    b->max_ntypes = std::max(b->max_ntypes, nt);
    const int tc_limit = choose_tile_cap(1e9, HALO_MAX, b->max_ntypes, b->lds_limit);
    const int tc = grid_tile_cap(g, n, b->max_ntypes, b->lds_limit);
    const int new_tc = std::min(std::max(b->tile_cap, tc), tc_limit);
    if (new_tc != b->tile_cap || old_ntypes != b->max_ntypes) drop_graph(b);
    b->tile_cap = new_tc;

    int rc = LJMD_OK;
    auto undo = [&](int code) {
        const std::string msg = g_last_error;
        (void)release_slot(b, s);
        g_last_error = msg;
        return code;
    };
    const size_t N = (size_t)n;
    rc = ensure_stage(b, 8 * N);
    if (rc != LJMD_OK) return undo(rc);
    double *st_pos = b->d_stage, *st_vel = b->d_stage + 3 * N;
    int *st_type = (int *)(b->d_stage + 6 * N);
    std::vector<int> zeros;
    if (!sp->type) zeros.assign(N, 0);
    std::vector<PairCoef> coef(PAIR_ROWS);
    std::vector<double> rl2(PAIR_ROWS, 0.0);
    std::copy(pt.coef.begin(), pt.coef.end(), coef.begin());
    std::copy(pt.rl2.begin(), pt.rl2.end(), rl2.begin());
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    if (hipMemcpyAsync(st_pos, sp->pos, 3 * N * sizeof(double), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(st_vel, sp->vel, 3 * N * sizeof(double), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(st_type, sp->type ? sp->type : zeros.data(), N * sizeof(int), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_pair + P.pair_off, coef.data(), PAIR_ROWS * sizeof(PairCoef), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_rl2 + P.pair_off, rl2.data(), PAIR_ROWS * sizeof(double), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_cell_rank + coff, g.rank.data(), g.ncell * sizeof(int), h2d, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_cell_xyz + coff, g.xyz.data(), g.ncell * sizeof(int), h2d, b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_cell_count + coff, 0, (g.ncell + 1) * sizeof(int), b->stream) != hipSuccess ||
        hipMemcpyAsync(b->d_halo + (size_t)boff * HALO_MAX, g.halo.data(),
                       g.halo.size() * sizeof(HaloCell), h2d, b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_req + 2 * s, 0, 2 * sizeof(int), b->stream) != hipSuccess ||
        hipMemsetAsync(b->d_count + poff, 0, N * sizeof(int), b->stream) != hipSuccess ||
        launch_fill_int(b->stream, b->d_prep + poff, n, s) != hipSuccess ||
        launch_fill_int(b->stream, b->d_crep + coff, g.ncell, s) != hipSuccess ||
        launch_fill_int(b->stream, b->d_crep + coff + g.ncell, 1, -1) != hipSuccess ||
        launch_upload(b->stream, st_pos, st_vel, st_type, nullptr, b->d_pos[b->cur], b->d_vel,
                      b->d_img, n, sp->box, 1, 1, nullptr, poff) != hipSuccess ||
        hipMemcpyAsync(b->d_bricks + boff, g.bricks.data(), g.nbrick * sizeof(BrickInfo), h2d,
                       b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return undo(set_err(LJMD_E_DEVICE, "replica upload failed"));
    rc = write_params(b, s);
    if (rc != LJMD_OK) return undo(rc);

    // first list build, with the lane layout chosen on the first replica
    rc = set_single_mask(b, b->d_go, s);
    if (rc == LJMD_OK) rc = set_single_mask(b, b->d_only, s);
    if (rc != LJMD_OK) return undo(rc);
    // until the first block tunes them, lanes and workgroup size take the given values or
    // defaults (2, 256)
    if (!b->tpp) set_tpp(b, 2);
    if (!b->block) b->block = 256;
    rc = grow_list(b, b->cfg.nlist_capacity > 0 ? b->cfg.nlist_capacity : expected_cap(sp, pt.rl_max));
    if (rc != LJMD_OK) return undo(rc);
    rc = forced_rebuild(b, {s});
    if (rc != LJMD_OK) return undo(rc);
    // before the first block tunes lanes or workgroup size, keep the sorted state at t = 0:
    // the tuning trials rebuild lists at the drifted positions, so the first half step is
    // taken again afterwards from this state (redo_first_half_step)
    if (!b->layout_fixed && (!b->cfg.threads_per_particle || !b->cfg.block_size)) {
        rc = copy_range(b, b->slots[s], true);
        if (rc != LJMD_OK) return undo(rc);
    }

    // forces at the initial positions, then the first half step
    rc = clear_status(b);
    if (rc == LJMD_OK)
        rc = launch_chk(launch_force(b->stream, force_args(b, b->cur, b->d_only, false), b->prec,
                                     b->tpp, MODE_EVAL, false, b->block), "force eval");
    if (rc == LJMD_OK) rc = read_status(b);
    if (rc != LJMD_OK) return undo(rc);
    if (b->h_status[s] & ST_NONFINITE)
        return undo(set_err(LJMD_E_NONFINITE, "non-finite force at the initial positions"));
    KickDriftArgs ka{};
    ka.reps = b->d_reps;
    ka.prep = b->d_prep;
    ka.pos_in = b->d_pos[b->cur];
    ka.pos_out = b->d_pos[b->cur ^ 1];
    ka.vel = b->d_vel;
    ka.img = b->d_img;
    ka.xb = b->d_xb;
    ka.force = b->d_force;
    ka.req = b->d_req;
    ka.only = b->d_only;
    ka.cur = b->cur;
    ka.n = b->p_ext;
    rc = launch_chk(launch_kick_drift(b->stream, ka), "kick-drift");
    if (rc != LJMD_OK) return undo(rc);
    // the batch's current buffer is cur: bring the drifted positions there, then serve the
    // rebuild request the drift raised (it sits in the other buffer's word)
    if (hipMemcpyAsync(b->d_pos[b->cur] + poff, b->d_pos[b->cur ^ 1] + poff, N * sizeof(double4),
                       hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
        launch_fill_int(b->stream, b->d_go, b->max_slots, 0) != hipSuccess ||
        hipMemcpyAsync(b->d_go + s, b->d_req + 2 * s + (b->cur ^ 1), sizeof(int),
                       hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
        return undo(set_err(LJMD_E_DEVICE, "admission copy failed"));
    rc = clear_status(b);
    if (rc == LJMD_OK)
        rc = launch_chk(launch_rebuild(b->stream, rebuild_args(b, b->d_go, 1, b->cur)), "rebuild");
    if (rc == LJMD_OK) rc = read_status(b);
    if (rc != LJMD_OK) return undo(rc);
    if (b->h_status[s] & ST_TILE)
        return undo(set_err(LJMD_E_BOX, "a brick holds more than %d atoms in its halo cells", TILE_INDEX_MAX));
    if (b->h_status[s] & ST_OVERFLOW) {
        // the list at the drifted positions does not fit: grow it and build again there
        DevStatus st{};
        if (hipMemcpyAsync(&st, b->d_st, sizeof st, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return undo(set_err(LJMD_E_DEVICE, "status copy failed"));
        rc = grow_list(b, (int)std::ceil(1.25 * st.max_count + 8));
        if (rc == LJMD_OK) rc = set_single_mask(b, b->d_go, s);
        if (rc == LJMD_OK) rc = forced_rebuild(b, {s});
        if (rc != LJMD_OK) return undo(rc);
    }
    // requests served; steps left counted from the current buffer
    if (hipMemsetAsync(b->d_req + 2 * s, 0, 2 * sizeof(int), b->stream) != hipSuccess ||
        launch_fill_int(b->stream, b->d_rem + 2 * s + b->cur, 1, (int)sp->nsteps) != hipSuccess ||
        launch_fill_int(b->stream, b->d_rem + 2 * s + (b->cur ^ 1), 1, 0) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return undo(set_err(LJMD_E_DEVICE, "admission counters failed"));
    *slot_out = s;
    return LJMD_OK;
}

namespace {

// Replicas admitted before the first block took their first force evaluation and half step
// with the default lanes per particle, and the tuning trials then rebuilt their lists (new
// order and build points) at the drifted positions. The lane count orders each particle's
// force sum, so once the block has tuned the lanes these steps are taken again with them,
// from the sorted state kept at admission: every replica then follows the trajectory its
// alone run computes with the same lanes. The sequence is admission's, for all of them at once: build, forces,
// kick and drift, drifted positions into the current buffer, the builds the drift asks for.
int redo_first_half_step(ljmd_batch *b, const std::vector<int> &which) {
    for (int s : which) CHK(copy_range(b, b->slots[s], false));
    std::fill(b->h_mask.begin(), b->h_mask.end(), 0);
    for (int s : which) b->h_mask[s] = 1;
    CHK(upload_mask(b, b->d_go, b->h_mask));
    CHK(upload_mask(b, b->d_only, b->h_mask));
    CHK(forced_rebuild(b, which));
    CHK(clear_status(b));
    CHK(launch_chk(launch_force(b->stream, force_args(b, b->cur, b->d_only, false), b->prec,
                                b->tpp, MODE_EVAL, false, b->block), "force eval"));
    CHK(read_status(b));
    for (int s : which)
        if (b->h_status[s] & ST_NONFINITE)
            return set_err(LJMD_E_NONFINITE, "non-finite force at the initial positions of slot %d", s);
    KickDriftArgs ka{};
    ka.reps = b->d_reps;
    ka.prep = b->d_prep;
    ka.pos_in = b->d_pos[b->cur];
    ka.pos_out = b->d_pos[b->cur ^ 1];
    ka.vel = b->d_vel;
    ka.img = b->d_img;
    ka.xb = b->d_xb;
    ka.force = b->d_force;
    ka.req = b->d_req;
    ka.only = b->d_only;
    ka.cur = b->cur;
    ka.n = b->p_ext;
    HIPCHK(hipMemsetAsync(b->d_req, 0, 2 * sizeof(int) * b->max_slots, b->stream));
    CHK(launch_chk(launch_kick_drift(b->stream, ka), "kick-drift"));
    CHK(launch_chk(launch_fill_int(b->stream, b->d_go, b->max_slots, 0), "fill"));
    for (int s : which) {
        const Slot &sl = b->slots[s];
        HIPCHK(hipMemcpyAsync(b->d_pos[b->cur] + sl.poff, b->d_pos[b->cur ^ 1] + sl.poff,
                              (size_t)sl.n * sizeof(double4), hipMemcpyDeviceToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->d_go + s, b->d_req + 2 * s + (b->cur ^ 1), sizeof(int),
                              hipMemcpyDeviceToDevice, b->stream));
    }
    return forced_rebuild(b, which);  // gated by the go words just written
}

}  // namespace

int ljmd_batch_run_block(ljmd_batch *b) {
    if (!b) return set_err(LJMD_E_INVAL, "null handle");
    std::vector<int> running;
    for (int s = 0; s < b->max_slots; ++s)
        if (b->slots[s].used && !b->slots[s].done) running.push_back(s);
    if (running.empty()) return LJMD_OK;
    if (!b->layout_fixed) {
        // the first block: tune lanes and workgroup size on the replicas present
        if (!b->cfg.threads_per_particle || !b->cfg.block_size) {
            std::fill(b->h_mask.begin(), b->h_mask.end(), 0);
            for (int s : running) b->h_mask[s] = 1;
            CHK(upload_mask(b, b->d_go, b->h_mask));
            CHK(upload_mask(b, b->d_only, b->h_mask));
            CHK(tune(b, running));
            // the trials re-sorted the replicas and moved their build points: every one
            // takes its first half step again from its state at t = 0
            CHK(redo_first_half_step(b, running));
            HIPCHK(hipMemsetAsync(b->d_req, 0, 2 * sizeof(int) * b->max_slots, b->stream));
        }
        b->layout_fixed = true;
    }
    CHK(snapshot_all(b));
    CHK(clear_status(b));
    CHK(ensure_graph(b));
    HIPCHK(hipGraphLaunch(b->graph, b->stream));
    CHK(read_status(b));
    b->blocks += 1;
    std::vector<int> overflowed;
    for (int s : running) {
        Slot &sl = b->slots[s];
        const int st = b->h_status[s];
        if (st & (ST_NONFINITE | ST_TILE)) {
            // retire with the state of the block start
            CHK(copy_range(b, sl, false));
            sl.done = true;
            sl.error = (st & ST_TILE) ? LJMD_E_BOX : LJMD_E_NONFINITE;
            sl.P.active = 0;
            CHK(write_params(b, s));
        } else if (st & ST_OVERFLOW) {
            overflowed.push_back(s);
        }
    }
    // run the block again for the replicas whose list overflowed, from their snapshot
    for (int attempt = 0; !overflowed.empty(); ++attempt) {
        if (attempt >= 8) return set_err(LJMD_E_DEVICE, "list overflow persisted after growth");
        DevStatus st{};
        HIPCHK(hipMemcpyAsync(&st, b->d_st, sizeof st, hipMemcpyDeviceToHost, b->stream));
        CHK(sync(b));
        CHK(grow_list(b, (int)std::ceil(1.25 * st.max_count + 8)));
        std::fill(b->h_mask.begin(), b->h_mask.end(), 0);
        for (int s : overflowed) {
            CHK(copy_range(b, b->slots[s], false));
            b->h_mask[s] = 1;
        }
        b->overflow_reruns += (int64_t)overflowed.size();
        CHK(upload_mask(b, b->d_go, b->h_mask));
        CHK(upload_mask(b, b->d_only, b->h_mask));
        CHK(forced_rebuild(b, overflowed));
        // every request is stale or served: the re-run must rebuild only what it requests
        HIPCHK(hipMemsetAsync(b->d_req, 0, 2 * sizeof(int) * b->max_slots, b->stream));
        for (int s : overflowed) {
            CHK(launch_chk(launch_fill_int(b->stream, b->d_rem + 2 * s + b->cur, 1, (int)b->slots[s].rem), "fill"));
        }
        CHK(clear_status(b));
        CHK(enqueue_block(b, b->stream, b->d_only));
        CHK(read_status(b));
        std::vector<int> again;
        for (int s : overflowed) {
            Slot &sl = b->slots[s];
            const int stt = b->h_status[s];
            if (stt & (ST_NONFINITE | ST_TILE)) {
                CHK(copy_range(b, sl, false));
                sl.done = true;
                sl.error = (stt & ST_TILE) ? LJMD_E_BOX : LJMD_E_NONFINITE;
                sl.P.active = 0;
                CHK(write_params(b, s));
            } else if (stt & ST_OVERFLOW) {
                again.push_back(s);
            }
        }
        overflowed.swap(again);
    }
    // steps left after the block; finished replicas stop taking part in launches
    for (int s : running) {
        Slot &sl = b->slots[s];
        if (sl.done) continue;
        sl.rem = std::max<int64_t>(0, sl.rem - b->block_steps);
        if (sl.rem == 0) {
            sl.done = true;
            sl.P.active = 0;
            CHK(write_params(b, s));
        }
    }
    return LJMD_OK;
}

int ljmd_batch_poll(ljmd_batch *b, int32_t *done, int32_t *ndone) {
    if (!b || !ndone) return set_err(LJMD_E_INVAL, "null argument");
    int k = 0;
    for (int s = 0; s < b->max_slots; ++s)
        if (b->slots[s].used && b->slots[s].done) {
            if (done) done[k] = s;
            ++k;
        }
    *ndone = k;
    return LJMD_OK;
}

int ljmd_batch_slot_steps(ljmd_batch *b, int32_t s, int64_t *steps) {
    if (!b || !steps) return set_err(LJMD_E_INVAL, "null argument");
    if (s < 0 || s >= b->max_slots || !b->slots[s].used) return set_err(LJMD_E_STATE, "slot %d is empty", s);
    const Slot &sl = b->slots[s];
    *steps = sl.error ? 0 : sl.nsteps - sl.rem;
    return LJMD_OK;
}

int ljmd_batch_slot_status(ljmd_batch *b, int32_t s, int32_t *status) {
    if (!b || !status) return set_err(LJMD_E_INVAL, "null argument");
    if (s < 0 || s >= b->max_slots || !b->slots[s].used) return set_err(LJMD_E_STATE, "slot %d is empty", s);
    *status = b->slots[s].error;
    return LJMD_OK;
}

namespace {

int check_readable(ljmd_batch *b, int32_t s) {
    if (!b) return set_err(LJMD_E_INVAL, "null handle");
    if (s < 0 || s >= b->max_slots || !b->slots[s].used) return set_err(LJMD_E_STATE, "slot %d is empty", s);
    const Slot &sl = b->slots[s];
    if (!sl.done) return set_err(LJMD_E_STATE, "replica in slot %d has not finished", s);
    if (sl.error) return set_err(sl.error, "replica in slot %d was retired with status %d", s, sl.error);
    return LJMD_OK;
}

// Results of a finished slot through `stage` (3 n doubles of device staging): positions,
// velocities and forces are put in tag order there, then copied to the host; energy and virial
// come from a force evaluation of the replica alone and the fixed-order reductions, in the
// batch's own buffers.
int read_slot(ljmd_batch *b, int32_t s, double *stage, double *pos, double *vel, double *force,
              double *energy, double *virial) {
    Slot &sl = b->slots[s];
    const size_t N = (size_t)sl.n;
    auto fetch = [&](const double4 *src, double *out) {
        CHK(launch_chk(launch_unsort_vec(b->stream, src, b->d_img, sl.poff, sl.n, stage), "unsort"));
        HIPCHK(hipMemcpyAsync(out, stage, 3 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        return sync(b);
    };
    if (pos) CHK(fetch(b->d_pos[b->cur], pos));
    if (vel) CHK(fetch(b->d_vel, vel));
    if (force) CHK(fetch(b->d_force, force));
    if (energy || virial) {
        // the replica is inactive once finished: evaluate it alone, then retire it again
        sl.P.active = 1;
        CHK(write_params(b, s));
        CHK(set_single_mask(b, b->d_only, s));
        int rc = launch_chk(launch_force(b->stream, force_args(b, b->cur, b->d_only, false), b->prec,
                                         b->tpp, MODE_EVAL, true, b->block), "force eval");
        if (rc == LJMD_OK)
            rc = launch_chk(launch_reduce(b->stream, b->d_u, b->d_w, nullptr, b->d_vel, sl.poff, sl.n,
                                          b->d_partials, b->red_blocks, b->d_red), "reduce");
        double red[RED_QUANT];
        if (rc == LJMD_OK &&
            (hipMemcpyAsync(red, b->d_red, sizeof red, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
             hipStreamSynchronize(b->stream) != hipSuccess))
            rc = set_err(LJMD_E_DEVICE, "reduction copy failed");
        sl.P.active = 0;
        CHK(write_params(b, s));
        CHK(rc);
        if (energy) {
            energy[0] = red[0];
            energy[1] = red[7];
        }
        if (virial)
            for (int c = 0; c < 6; ++c) virial[c] = red[1 + c];
    }
    return LJMD_OK;
}

}  // namespace

int ljmd_batch_read(ljmd_batch *b, int32_t s, double *pos, double *vel, double *force,
                    double *energy, double *virial) {
    CHK(check_readable(b, s));
    CHK(ensure_stage(b, 3 * (size_t)b->slots[s].n));
    return read_slot(b, s, b->d_stage, pos, vel, force, energy, virial);
}

int ljmd_batch_read_noalloc(ljmd_batch *b, int32_t s, double *pos, double *vel, double *force,
                            double *energy, double *virial) {
    CHK(check_readable(b, s));
    if (3 * (size_t)b->slots[s].n > NOALLOC_STAGE_DOUBLES)
        return set_err(LJMD_E_INVAL, "replica of %d particles exceeds the no-allocation staging "
                                     "(at most %zu particles)",
                       b->slots[s].n, NOALLOC_STAGE_DOUBLES / 3);
    return read_slot(b, s, b->d_noalloc_stage, pos, vel, force, energy, virial);
}

int ljmd_batch_get_stats(ljmd_batch *b, ljmd_batch_stats *out) {
    if (!b || !out) return set_err(LJMD_E_INVAL, "null argument");
    DevStatus st{};
    HIPCHK(hipMemcpyAsync(&st, b->d_st, sizeof st, hipMemcpyDeviceToHost, b->stream));
    CHK(sync(b));
    std::memset(out, 0, sizeof *out);
    for (const Slot &sl : b->slots) {
        out->resident += sl.used ? 1 : 0;
        out->running += (sl.used && !sl.done) ? 1 : 0;
    }
    out->blocks = b->blocks;
    out->overflow_reruns = b->overflow_reruns;
    out->rebuilds = (int64_t)st.builds;
    out->nlist_capacity = b->cap;
    out->threads_per_particle = b->tpp;
    out->block_size = b->block;
    out->tile_capacity = b->tile_cap;
    out->device_bytes = b->mem.bytes;
    out->used_bytes = b->used_bytes;
    out->budget_bytes = b->cfg.budget_bytes;
    return LJMD_OK;
}

int ljmd_batch_release(ljmd_batch *b, int32_t s) {
    if (!b) return set_err(LJMD_E_INVAL, "null handle");
    if (s < 0 || s >= b->max_slots || !b->slots[s].used) return set_err(LJMD_E_STATE, "slot %d is empty", s);
    return release_slot(b, s);
}

}  // extern "C"
