// Host side of libljmd: the single-system C ABI of include/ljmd.h. For the kernels a
// system is a batch of one replica (a parameter table of one entry, all offsets 0).
//
// Step structure (velocity Verlet, NVE). With x(t), v(t) and F(t) on the device:
//   kick-drift kernel        v += dt/2m F(t); x(t+1) = x + dt v, wrapped, written into the
//                            other position buffer; raises the rebuild request if needed.
//   gated rebuild kernels    bin -> scan -> scatter -> in-cell sort and gather -> Verlet
//                            build; every kernel returns at once unless the request is set.
//   n-1 times: fused kernel  F(t+1) at x(t+1); v += dt/2m F (full step); v += dt/2m F;
//                            x(t+2) into the other buffer; rebuild request; gated rebuild.
//   final kernel             F(t+n); v += dt/2m F; F stored.
// The repeating unit (fused kernel + gated rebuild) is captured once per starting buffer
// into a HIP graph of `graph_steps` units. Host and device meet once per call, at the end,
// to read the status word: on list overflow the call restores its starting state, grows
// the list and runs again; on a non-finite force it restores and returns an error.
#include "ljmd_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

using namespace ljmd;

namespace {

struct TuneKey {
    int prec, multi, nbucket;
    bool operator<(const TuneKey &o) const {
        return std::tie(prec, multi, nbucket) < std::tie(o.prec, o.multi, o.nbucket);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;  // -> (tpp, block)

}  // namespace

constexpr int EV_PER_UNIT = 8;  // step kernel (2 events) + five rebuild kernels (6 events)

struct ljmd_system {
    ljmd_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    DeviceArena mem;
    size_t lds_limit = 64 * 1024;
    int n = 0, npad = 0;
    double L[3]{};
    int ntypes = 1;
    std::vector<double> eps, sig, rc;
    std::vector<char> is_set;
    // pair form of the system (all set pairs share it) and each pair's form parameters
    int style = STYLE_LJ;
    int shift_force = 0;  // LJMD_SHIFT_FORCE: the shifted-force variant of the form
    std::vector<int> pform;       // form of each set pair
    std::vector<double> par;      // 4 per pair
    std::vector<int32_t> h_type;
    std::vector<double> h_mass;
    bool table_dirty = true;
    double rl_max = 0.0;
    RepParams rep{};  // host copy of the replica parameters
    // device memory
    RepParams *d_rep = nullptr;
    PairCoef *d_pair = nullptr;
    double *d_rl2 = nullptr;
    int *d_req = nullptr;  // rebuild requests, one per position buffer
    int *d_one = nullptr;  // constant 1: the go word of an unconditional rebuild
    int ncell = 0, ncell_alloc = 0;
    int *d_cell_rank = nullptr, *d_cell_xyz = nullptr, *d_cell_count = nullptr,
        *d_cell_start = nullptr, *d_cell_lo = nullptr;
    BrickInfo *d_bricks = nullptr;
    HaloCell *d_halo = nullptr;
    int *d_tile_tab = nullptr;
    int nbrick = 0, nbrick_alloc = 0, tile_cap = 0;
    double4 *d_pos[2]{}, *d_pos_scr = nullptr, *d_vel = nullptr, *d_vel_scr = nullptr,
            *d_force = nullptr, *d_xb = nullptr;
    int4 *d_img = nullptr, *d_img_scr = nullptr;
    int *d_key = nullptr, *d_slot = nullptr, *d_perm = nullptr;
    int *d_count = nullptr;
    uint16_t *d_nlist = nullptr;
    uint16_t *d_work = nullptr;
    int cap = 0;
    size_t nlist_alloc = 0;
    double *d_u = nullptr, *d_w = nullptr, *d_ke = nullptr, *d_partials = nullptr,
           *d_red = nullptr;
    double *d_stage = nullptr;  // n x 10 doubles of upload/download staging
    double4 *d_snap_pos = nullptr, *d_snap_vel = nullptr;
    int4 *d_snap_img = nullptr;
    // neighbour-list method: cell-list bricks (16-bit tile lists) or one tree per type
    // (32-bit lists, LJMD_NLIST_TREE); the tree method's typed sort grid has ncs spatial cells
    int nlist_method = LJMD_NLIST_CELL;
    int ncs = 0;
    int *d_cell_of = nullptr, *d_bvh_left = nullptr, *d_bvh_right = nullptr,
        *d_bvh_rlo = nullptr, *d_bvh_rsplit = nullptr, *d_bvh_rhi = nullptr;
    BvhNode *d_bvh_node = nullptr;
    double *d_bvh_blk = nullptr, *d_bvh_sblk = nullptr;
    int32_t *d_nlist32 = nullptr;
    size_t nlist32_alloc = 0;
    // NVT thermostat: device scalars (TH_*), their snapshot, kinetic-energy partials
    bool nvt = false;
    bool nvt_ready = false;  // the half step opening the next step is on the device
    double nvt_kT = 0.0, nvt_invQ = 0.0, nvt_g = 0.0;
    double *d_th = nullptr, *d_snap_th = nullptr, *d_kpart = nullptr;
    DevStatus *d_st = nullptr;
    // thermodynamic samples (ljmd_set_thermo): U, W[6], K of every period-th step, reduced on
    // the device into a ring of thermo_cap rows; the step of each row is kept on the host
    int thermo_period = 0, thermo_cap = 0;
    double *d_thermo = nullptr;
    std::vector<int64_t> thermo_step;
    int64_t thermo_written = 0;
    int cur = 0;
    bool list_valid = false, force_valid = false;
    int64_t steps = 0, overflow_retries = 0;
    int tpp = 4, lshift = 2, block = 128;
    int graph_steps = 64;
    hipGraphExec_t graph[2]{nullptr, nullptr};
    // timing: per unit EV_PER_UNIT events (around the step's force kernel, then around the
    // five rebuild kernels), and every recorded duration by kernel kind
    bool timing = false;
    std::vector<float> dur[LJMD_KERNEL_KINDS];
    std::vector<hipEvent_t> ev;
    int64_t t_launches = 0;
    double t_ms = 0.0;
    int red_blocks = 1024;
};

namespace {

template <class T>
int dalloc_t(ljmd_system *s, T **p, size_t count) {
    return s->mem.get_t(p, count);
}

void dfree(ljmd_system *s, void *p) { s->mem.put(p); }

void drop_graphs(ljmd_system *s) {
    for (int c = 0; c < 2; ++c)
        if (s->graph[c]) {
            (void)hipGraphExecDestroy(s->graph[c]);
            s->graph[c] = nullptr;
        }
}

int sync_status(ljmd_system *s, DevStatus *out) {
    HIPCHK(hipMemcpyAsync(out, s->d_st, sizeof(DevStatus), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (out->status & ST_DEBUG)
        return set_err(LJMD_E_DEVICE, "device check %d failed (debug build)", out->debug);
    return LJMD_OK;
}

int clear_status_bits(ljmd_system *s) {
    // status and max_count words only; the counters stay
    HIPCHK(hipMemsetAsync(&s->d_st->status, 0, 2 * sizeof(int), s->stream));
    return LJMD_OK;
}

int precision(ljmd_system *s) { return s->cfg.precision == LJMD_MIXED ? PREC_MIXED : PREC_FP64; }

int launch_chk(hipError_t e, const char *what) {
    if (e != hipSuccess) return set_err(LJMD_E_DEVICE, "launch of %s: %s", what, hipGetErrorString(e));
    return LJMD_OK;
}

// ------------------------------------------------------------ pair table and cell grid

// The tree method's sort grid: fine cells of about four particles, at most 1023 per axis and
// 2^22 in all with the type as the slowest index; cells in Morton order within each type, so
// each type's particles end up contiguous and spatially ordered (the trees' leaf order).
int make_sort_grid(ljmd_system *s, double rl_max, ReplicaGrid *g) {
    for (int a = 0; a < 3; ++a)
        if (rl_max > 0.5 * s->L[a])
            return set_err(LJMD_E_BOX, "r_cut + skin = %g exceeds half the box edge %g", rl_max,
                           s->L[a]);
    const double vol = s->L[0] * s->L[1] * s->L[2];
    double w = std::cbrt(4.0 * vol / std::max(1, s->n));
    int nc[3];
    for (;;) {
        int64_t tot = s->ntypes;
        for (int a = 0; a < 3; ++a) {
            nc[a] = (int)std::max(1.0, std::min(1023.0, std::floor(s->L[a] / w)));
            tot *= nc[a];
        }
        if (tot <= ((int64_t)1 << 22)) break;
        w *= 1.25;
    }
    const int ncs = nc[0] * nc[1] * nc[2];
    std::vector<std::pair<uint64_t, int>> order(ncs);
    for (int x = 0; x < nc[0]; ++x)
        for (int y = 0; y < nc[1]; ++y)
            for (int z = 0; z < nc[2]; ++z) {
                uint64_t code = 0;
                for (int bit = 0; bit < 10; ++bit)
                    code |= ((uint64_t)((x >> bit) & 1) << (3 * bit + 2)) |
                            ((uint64_t)((y >> bit) & 1) << (3 * bit + 1)) |
                            ((uint64_t)((z >> bit) & 1) << (3 * bit));
                const int lin = (x * nc[1] + y) * nc[2] + z;
                order[lin] = {code, lin};
            }
    std::sort(order.begin(), order.end());
    g->rank.assign((size_t)ncs * s->ntypes, 0);
    g->xyz.assign((size_t)ncs * s->ntypes, 0);
    for (int r = 0; r < ncs; ++r)
        for (int t = 0; t < s->ntypes; ++t) g->rank[(size_t)t * ncs + order[r].second] = t * ncs + r;
    for (int a = 0; a < 3; ++a) g->nc[a] = nc[a];
    g->canonical = false;
    g->ncell = ncs * s->ntypes;
    g->nbrick = 0;
    g->max_halo = 0;
    s->ncs = ncs;
    return LJMD_OK;
}

int ensure_tree_arrays(ljmd_system *s);

int setup_table(ljmd_system *s) {
    const int nt = s->ntypes;
    for (int k = 0; k < nt * nt; ++k)
        if (!s->is_set[k])
            return set_err(LJMD_E_STATE, "pair (%d,%d) has not been set", k / nt, k % nt);
    PairTable pt;
    if (s->style == STYLE_LJ)
        make_pair_table(nt, s->eps.data(), s->sig.data(), s->rc.data(), s->cfg.skin, &pt);
    else
        make_form_table(nt, s->style, s->par.data(), s->rc.data(), s->cfg.skin, &pt);
    if (s->shift_force) apply_force_shift(s->style, s->rc.data(), &pt);
    ReplicaGrid g;
    if (s->nlist_method == LJMD_NLIST_TREE) {
        if (s->style != STYLE_LJ || s->shift_force)
            return set_err(LJMD_E_INVAL,
                           "tree neighbour lists evaluate the LJ form with the energy shift only");
        CHK(make_sort_grid(s, pt.rl_max, &g));
    } else {
        CHK(make_grid(s->L, pt.rl_max, &g, s->n, tile_limit_for(nt, s->lds_limit)));
    }
    const int ncell = g.ncell;
    if (ncell + 1 > s->ncell_alloc) {
        dfree(s, s->d_cell_rank);
        dfree(s, s->d_cell_xyz);
        dfree(s, s->d_cell_count);
        dfree(s, s->d_cell_start);
        dfree(s, s->d_cell_lo);
        s->d_cell_rank = s->d_cell_xyz = s->d_cell_count = s->d_cell_start = s->d_cell_lo =
            nullptr;
        s->ncell_alloc = 0;
        CHK(dalloc_t(s, &s->d_cell_rank, ncell + 1));
        CHK(dalloc_t(s, &s->d_cell_xyz, ncell + 1));
        CHK(dalloc_t(s, &s->d_cell_count, ncell + 1));
        CHK(dalloc_t(s, &s->d_cell_start, ncell + 1));
        CHK(dalloc_t(s, &s->d_cell_lo, ncell + 1));
        s->ncell_alloc = ncell + 1;
    }
    if (g.nbrick > 0 && g.nbrick > s->nbrick_alloc) {
        dfree(s, s->d_bricks);
        dfree(s, s->d_halo);
        dfree(s, s->d_tile_tab);
        s->d_bricks = nullptr;
        s->d_halo = nullptr;
        s->d_tile_tab = nullptr;
        s->nbrick_alloc = 0;
        CHK(dalloc_t(s, &s->d_bricks, g.nbrick));
        CHK(dalloc_t(s, &s->d_halo, (size_t)g.nbrick * HALO_MAX));
        CHK(dalloc_t(s, &s->d_tile_tab, (size_t)g.nbrick * TILE_TAB));
        s->nbrick_alloc = g.nbrick;
    }
    RepParams &P = s->rep;
    P = RepParams{};
    for (int a = 0; a < 3; ++a) {
        P.L[a] = s->L[a];
        P.invL[a] = 1.0 / s->L[a];
        P.inv_w[a] = (double)g.nc[a] / s->L[a];
        P.nc[a] = g.nc[a];
    }
    P.dt = s->cfg.dt;
    P.half_dt = 0.5 * s->cfg.dt;
    const double lim = 0.5 * s->cfg.skin;
    P.lim2 = lim * lim;
    P.single_rl2 = pt.coef[0].rl2;
    P.poff = 0;
    P.n = s->n;
    P.coff = 0;
    P.ncell = ncell;
    P.boff = 0;
    P.nbrick = g.nbrick;
    P.canonical = g.canonical ? 1 : 0;
    P.ntypes = nt;
    P.pair_off = 0;
    P.active = 1;
    P.tile_cap = g.nbrick > 0 ? grid_tile_cap(g, s->n, nt, s->lds_limit) : 64;
    HIPCHK(hipMemcpyAsync(s->d_rep, &P, sizeof(RepParams), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->d_pair, pt.coef.data(), sizeof(PairCoef) * nt * nt,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->d_rl2, pt.rl2.data(), sizeof(double) * nt * nt, hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_cell_rank, g.rank.data(), sizeof(int) * ncell, hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_cell_xyz, g.xyz.data(), sizeof(int) * ncell, hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemsetAsync(s->d_cell_count, 0, sizeof(int) * (ncell + 1), s->stream));
    if (g.nbrick > 0) {
        HIPCHK(hipMemcpyAsync(s->d_bricks, g.bricks.data(), sizeof(BrickInfo) * g.nbrick,
                              hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->d_halo, g.halo.data(),
                              sizeof(HaloCell) * (size_t)g.nbrick * HALO_MAX,
                              hipMemcpyHostToDevice, s->stream));
    }
    if (s->nlist_method == LJMD_NLIST_TREE) CHK(ensure_tree_arrays(s));
    HIPCHK(hipStreamSynchronize(s->stream));  // host vectors go out of scope
    s->rl_max = pt.rl_max;
    s->ncell = ncell;
    s->nbrick = g.nbrick;
    s->tile_cap = P.tile_cap;
    s->table_dirty = false;
    s->list_valid = false;
    s->force_valid = false;
    drop_graphs(s);
    return LJMD_OK;
}

// The tree method's node, record and cell arrays (n each; 6 box doubles per block of 64 and
// of 4096 leaves).
int ensure_tree_arrays(ljmd_system *s) {
    if (s->d_cell_of) return LJMD_OK;
    const size_t N = (size_t)s->n;
    CHK(dalloc_t(s, &s->d_cell_of, N));
    CHK(dalloc_t(s, &s->d_bvh_left, N));
    CHK(dalloc_t(s, &s->d_bvh_right, N));
    CHK(dalloc_t(s, &s->d_bvh_rlo, N));
    CHK(dalloc_t(s, &s->d_bvh_rsplit, N));
    CHK(dalloc_t(s, &s->d_bvh_rhi, N));
    CHK(dalloc_t(s, &s->d_bvh_node, N));
    CHK(dalloc_t(s, &s->d_bvh_blk, 6 * ((N + 63) / 64)));
    CHK(dalloc_t(s, &s->d_bvh_sblk, 6 * ((N + 4095) / 4096)));
    return LJMD_OK;
}

// The list build addresses rounds of 8 x lanes entries (16-bit lists) or 4 x lanes entries
// (32-bit tree lists) with a 32-bit stride.
bool lanes_fit(int npad, int lshift) { return ((uint64_t)npad << (3 + lshift)) <= 0xFFFFFFFFull; }

int ensure_list_alloc(ljmd_system *s, int cap) {
    if (!lanes_fit(s->npad, s->lshift))
        return set_err(LJMD_E_INVAL, "%d lanes per particle is too many for %d particles",
                       1 << s->lshift, s->n);
    // a multiple of (entries per chunk) x lanes per particle (whole chunks per lane) keeps
    // every slot of k < cap inside cap * npad
    const bool tree = s->nlist_method == LJMD_NLIST_TREE;
    const int unit = (tree ? 4 : 8) << s->lshift;
    cap = std::max(unit, (cap + unit - 1) / unit * unit);
    const size_t need = (size_t)cap * (size_t)s->npad;
    if (tree && need > s->nlist32_alloc) {
        dfree(s, s->d_nlist32);
        s->d_nlist32 = nullptr;
        s->nlist32_alloc = 0;
        CHK(dalloc_t(s, &s->d_nlist32, need));
        s->nlist32_alloc = need;
    }
    if (!tree && need > s->nlist_alloc) {
        dfree(s, s->d_nlist);
        s->d_nlist = nullptr;
        s->nlist_alloc = 0;
        CHK(dalloc_t(s, &s->d_nlist, need));
        s->nlist_alloc = need;
    }
    if (cap != s->cap) drop_graphs(s);
    s->cap = cap;
    return LJMD_OK;
}

int round_cap(double v) { return std::max(8, (int)std::ceil(v)); }

// ------------------------------------------------------------ argument blocks

// go[0] is the rebuild's gate: a request word, or d_one for an unconditional rebuild
RebuildArgs rebuild_args(ljmd_system *s, const int *go, int cur) {
    RebuildArgs a{};
    a.reps = s->d_rep;
    a.prep = nullptr;  // every particle, cell and brick belongs to replica 0
    a.crep = nullptr;
    a.go = go;
    a.go_stride = 0;
    a.rl2_table = s->d_rl2;
    a.pos = s->d_pos[cur];
    a.pos_scr = s->d_pos_scr;
    a.vel = s->d_vel;
    a.vel_scr = s->d_vel_scr;
    a.img = s->d_img;
    a.img_scr = s->d_img_scr;
    a.xb = s->d_xb;
    a.key = s->d_key;
    a.slot = s->d_slot;
    a.perm = s->d_perm;
    a.cell_count = s->d_cell_count;
    a.cell_start = s->d_cell_start;
    a.cell_rank = s->d_cell_rank;
    a.cell_xyz = s->d_cell_xyz;
    a.nl_count = s->d_count;
    a.nlist = s->d_nlist;
    a.work = s->d_work;
    a.bricks = s->d_bricks;
    a.halo = s->d_halo;
    a.tile_tab = s->d_tile_tab;
    a.st = s->d_st;
    a.n = s->n;
    a.ncell = s->ncell;
    a.nbrick = s->nbrick;
    a.nrep = 1;
    a.npad = s->npad;
    a.cap = s->cap;
    a.lshift = s->lshift;
    a.tile_cap = s->tile_cap;
    a.max_ntypes = s->ntypes;
    const bool tree = s->nlist_method == LJMD_NLIST_TREE;
    a.typed_cells = tree ? s->ncs : 0;
    a.cell_of = tree ? s->d_cell_of : nullptr;
    a.cell_lo = tree ? nullptr : s->d_cell_lo;
    // half-cell work items for bricks of fewer cells than wavefronts (the batch keeps whole
    // cells: there, over many small replicas at once, halves measured slower)
    a.split_halves = 1;
    return a;
}

BvhArgs bvh_args(ljmd_system *s, const int *go, int cur) {
    BvhArgs b{};
    b.reps = s->d_rep;
    b.go = go;
    b.pos = s->d_pos[cur];
    b.pos_scr = s->d_pos_scr;
    b.vel = s->d_vel;
    b.vel_scr = s->d_vel_scr;
    b.xb = s->d_xb;
    b.img = s->d_img;
    b.img_scr = s->d_img_scr;
    b.cell_start = s->d_cell_start;
    b.cell_of = s->d_cell_of;
    b.left = s->d_bvh_left;
    b.right = s->d_bvh_right;
    b.rlo = s->d_bvh_rlo;
    b.rsplit = s->d_bvh_rsplit;
    b.rhi = s->d_bvh_rhi;
    b.blk = s->d_bvh_blk;
    b.sblk = s->d_bvh_sblk;
    b.node = s->d_bvh_node;
    b.rl2_table = s->d_rl2;
    b.nl_count = s->d_count;
    b.nlist32 = s->d_nlist32;
    b.st = s->d_st;
    b.n = s->n;
    b.ntypes = s->ntypes;
    b.ncs = s->ncs;
    b.npad = s->npad;
    b.cap = s->cap;
    b.lshift = s->lshift;
    // types by decreasing widest list radius (ties by index): the longest walks start first
    const int nt = s->ntypes;
    std::vector<double> widest(nt, 0.0);
    for (int a = 0; a < nt; ++a)
        for (int c = 0; c < nt; ++c) widest[a] = std::max(widest[a], s->rc[a * nt + c]);
    for (int k = 0; k < nt; ++k) b.type_order[k] = k;
    std::stable_sort(b.type_order, b.type_order + nt,
                     [&](int x, int y) { return widest[x] > widest[y]; });
    return b;
}

// The rebuild kernels of the system's list method at buffer cur, gated by go[0].
hipError_t launch_list_rebuild(ljmd_system *s, hipStream_t st, const int *go, int cur,
                               hipEvent_t *ev = nullptr) {
    RebuildArgs ra = rebuild_args(s, go, cur);
    if (s->nlist_method == LJMD_NLIST_TREE)
        return launch_rebuild_bvh(st, ra, bvh_args(s, go, cur), ev);
    return launch_rebuild(st, ra, ev);
}

ForceArgs force_args(ljmd_system *s, int cur) {
    ForceArgs a{};
    a.reps = s->d_rep;
    a.pos_in = s->d_pos[cur];
    a.pos_out = s->d_pos[cur ^ 1];
    a.vel = s->d_vel;
    a.img = s->d_img;
    a.xb = s->d_xb;
    a.force = s->d_force;
    a.nl_count = s->d_count;
    a.nlist = s->d_nlist;
    a.nlist32 = s->d_nlist32;
    a.work = s->d_work;
    a.bricks = s->d_bricks;
    a.cell_start = s->d_cell_start;
    a.tile_tab = s->d_tile_tab;
    a.u_out = s->d_u;
    a.w_out = s->d_w;
    a.ke_out = s->d_ke;
    a.pair = s->d_pair;
    a.req = s->d_req;
    a.rem = nullptr;  // no step budget: every fused step is a full step
    a.only = nullptr;
    a.status = &s->d_st->status;
    a.cur = cur;
    a.npad = s->npad;
    a.cap = s->cap;
    a.lshift = s->lshift;
    a.nbrick = s->nbrick;
    a.tile_cap = s->tile_cap;
    a.max_ntypes = s->ntypes;
    return a;
}

KickDriftArgs kick_drift_args(ljmd_system *s, int cur) {
    KickDriftArgs a{};
    a.reps = s->d_rep;
    a.prep = nullptr;
    a.pos_in = s->d_pos[cur];
    a.pos_out = s->d_pos[cur ^ 1];
    a.vel = s->d_vel;
    a.img = s->d_img;
    a.xb = s->d_xb;
    a.force = s->d_force;
    a.req = s->d_req;
    a.only = nullptr;
    a.cur = cur;
    a.n = s->n;
    return a;
}

// unconditional rebuild at the current positions
int enqueue_forced_rebuild(ljmd_system *s) {
    return launch_chk(launch_list_rebuild(s, s->stream, s->d_one, s->cur), "rebuild");
}

// The force kernel of the system's list method and pair form.
hipError_t launch_forces(ljmd_system *s, hipStream_t st, const ForceArgs &fa, int mode,
                         bool energy) {
    if (s->nlist_method == LJMD_NLIST_TREE)
        return launch_force_glist(st, fa, precision(s), s->tpp, mode, energy, s->block);
    return launch_force(st, fa, precision(s), s->tpp, mode, energy, s->block,
                        s->style | (s->shift_force ? STYLE_SF : 0));
}

int enqueue_eval(ljmd_system *s, bool energy) {
    ForceArgs a = force_args(s, s->cur);
    return launch_chk(launch_forces(s, s->stream, a, MODE_EVAL, energy), "force eval");
}

// Build the list at the current positions, growing the capacity until it fits.
int build_list(ljmd_system *s) {
    if (s->cap == 0) {
        int cap = s->cfg.nlist_capacity;
        if (cap <= 0) {
            // expected neighbours in the list radius at the mean density, with headroom
            const double vol = s->L[0] * s->L[1] * s->L[2];
            const double rho = s->n / vol;
            const double rl = s->rl_max;
            const double nbar = rho * 4.18879020478639 * rl * rl * rl;
            cap = round_cap(1.3 * nbar + 24.0);
            cap = std::min(cap, std::max(16, ((s->n + 15) & ~15)));
        }
        CHK(ensure_list_alloc(s, cap));
    }
    for (int attempt = 0; attempt < 8; ++attempt) {
        CHK(clear_status_bits(s));
        // a fresh list makes any pending rebuild request moot
        HIPCHK(hipMemsetAsync(s->d_req, 0, 2 * sizeof(int), s->stream));
        CHK(enqueue_forced_rebuild(s));
        DevStatus st{};
        CHK(sync_status(s, &st));
        if (st.status & ST_TILE)
            return set_err(LJMD_E_BOX, "a brick holds more than %d atoms in its halo cells: "
                                       "particle density too high for 16-bit tile indices",
                           TILE_INDEX_MAX);
        if (!(st.status & ST_OVERFLOW)) {
            s->list_valid = true;
            s->force_valid = false;
            return LJMD_OK;
        }
        CHK(ensure_list_alloc(s, round_cap(1.25 * st.max_count + 8)));
        s->overflow_retries += 1;
    }
    return set_err(LJMD_E_DEVICE, "neighbour list did not fit after repeated growth");
}

int tune(ljmd_system *s);

int ensure_ready(ljmd_system *s) {
    if (s->table_dirty) CHK(setup_table(s));
    if (s->tpp == 0 || s->block == 0) CHK(tune(s));
    if (!s->list_valid) CHK(build_list(s));
    if (!s->force_valid) {
        CHK(clear_status_bits(s));
        CHK(enqueue_eval(s, false));
        DevStatus st{};
        CHK(sync_status(s, &st));
        if (st.status & ST_NONFINITE)
            return set_err(LJMD_E_NONFINITE, "non-finite force at the current positions");
        s->force_valid = true;
    }
    return LJMD_OK;
}

// ------------------------------------------------------------ autotuner

double time_evals(ljmd_system *s, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    double best = 1e30;
    bool ok = true;
    for (int r = 0; r < 3 && ok; ++r) ok = enqueue_eval(s, false) == LJMD_OK;  // clocks up
    if (ok) {
        (void)hipEventRecord(e0, s->stream);
        for (int r = 0; r < reps && ok; ++r) ok = enqueue_eval(s, false) == LJMD_OK;
        (void)hipEventRecord(e1, s->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// Choose lanes per particle and workgroup size for the force kernel by timing the
// force evaluation on this system. Results are kept per (precision, multi-type, size
// bucket) for the life of the process.
int tune(ljmd_system *s) {
    const int want_tpp = s->cfg.threads_per_particle;
    const int want_block = s->cfg.block_size;
    int nb = 0;
    for (int v = s->n; v > 1; v >>= 1) ++nb;
    TuneKey key{precision(s), s->ntypes > 1 ? 1 : 0, nb};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        int ls = 0;
        if (it != g_tune.end())
            while ((1 << ls) < (want_tpp ? want_tpp : it->second.first)) ++ls;
        // a stored choice whose lane count this system cannot address is tuned afresh
        if (it != g_tune.end() && lanes_fit(s->npad, ls)) {
            s->tpp = want_tpp ? want_tpp : it->second.first;
            s->block = want_block ? want_block : it->second.second;
            for (s->lshift = 0; (1 << s->lshift) < s->tpp; ++s->lshift) {}
            if (s->cap) CHK(ensure_list_alloc(s, s->cap));
            s->list_valid = false;
            return LJMD_OK;
        }
    }
    const int tpps[] = {1, 2, 4, 8};
    const int blocks[] = {128, 192, 256, 320, 384, 448, 512};
    double best = 1e30;
    int bt = 4, bb = 128;
    for (int t : tpps) {
        if (want_tpp && t != want_tpp) continue;
        int ls = 0;
        while ((1 << ls) < t) ++ls;
        if (!lanes_fit(s->npad, ls)) continue;
        s->tpp = t;
        for (s->lshift = 0; (1 << s->lshift) < t; ++s->lshift) {}
        s->block = 256;
        s->list_valid = false;
        if (s->cap) CHK(ensure_list_alloc(s, s->cap));  // re-round for this lane count
        CHK(build_list(s));
        for (int b : blocks) {
            if (want_block && b != want_block) continue;
            s->block = b;
            const double ms = time_evals(s, 5);
            if (ms < best) {
                best = ms;
                bt = t;
                bb = b;
            }
        }
    }
    s->tpp = bt;
    s->block = bb;
    for (s->lshift = 0; (1 << s->lshift) < bt; ++s->lshift) {}
    if (s->cap) CHK(ensure_list_alloc(s, s->cap));
    s->list_valid = false;
    s->force_valid = false;
    drop_graphs(s);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {bt, bb};
    return LJMD_OK;
}

// ------------------------------------------------------------ stepping

NvtParams nvt_params(ljmd_system *s, int np, bool begin_only) {
    NvtParams p{};
    p.dt = s->cfg.dt;
    p.invQ = s->nvt_invQ;
    p.g = s->nvt_g;
    p.np = np;
    p.begin_only = begin_only ? 1 : 0;
    return p;
}

// The thermostat half step that opens the next step, from the stored velocities.
// Whether the step that ends at absolute step number `step` is sampled.
bool thermo_due(const ljmd_system *s, int64_t step) {
    return s->thermo_period > 0 && step > 0 && step % s->thermo_period == 0;
}

// The sample of a full step whose per-particle energies and virials are in d_u and d_w: K
// from the full-step kinetic energies of the fused step kernel (ke), else from the stored
// velocities; with NVT, K is then replaced by the thermostat's kinetic energy after its
// closing half step (the stored velocities still owe that half step's scaling).
int enqueue_thermo_sample(ljmd_system *s, hipStream_t st, int64_t step, const double *ke) {
    const int slot = (int)(s->thermo_written % s->thermo_cap);
    double *row = s->d_thermo + (size_t)slot * RED_QUANT;
    CHK(launch_chk(launch_reduce(st, s->d_u, s->d_w, ke, s->d_vel, 0, s->n, s->d_partials,
                                 s->red_blocks, row),
                   "thermo reduce"));
    if (s->nvt) CHK(launch_chk(launch_thermo_nvt_k(st, row, s->d_th), "thermo K"));
    s->thermo_step[slot] = step;
    s->thermo_written += 1;
    return LJMD_OK;
}

int enqueue_nvt_begin(ljmd_system *s, hipStream_t st) {
    int np = 0;
    CHK(launch_chk(launch_ke_partials(st, s->d_vel, 0, s->n, s->d_kpart, s->red_blocks, &np),
                   "kinetic energy"));
    return launch_chk(launch_nvt_thermo(st, s->d_kpart, nvt_params(s, np, true), s->d_th),
                      "thermostat");
}

// One NVT step from a full-step state at buffer cur (forces current): the opening thermostat
// half step's scaling with the first kick and the drift, the gated rebuild, the forces and
// second kick, then the kinetic energy and the thermostat (end half step, and the opening
// half step of the next one).
// `sample` >= 0: the step number this unit completes, sampled into the thermo ring.
int enqueue_nvt_unit(ljmd_system *s, hipStream_t st, int cur, bool timed, int ev_index,
                     int64_t sample) {
    KickDriftArgs ka = kick_drift_args(s, cur);
    ka.scale = s->d_th + TH_SPEND;  // TH_SPEND, TH_SB
    CHK(launch_chk(launch_kick_drift(st, ka), "kick-drift"));
    hipEvent_t *rev = timed ? &s->ev[EV_PER_UNIT * ev_index + 2] : nullptr;
    CHK(launch_chk(launch_list_rebuild(s, st, s->d_req + (cur ^ 1), cur ^ 1, rev), "rebuild"));
    ForceArgs fa = force_args(s, cur ^ 1);
    if (timed) HIPCHK(hipEventRecord(s->ev[EV_PER_UNIT * ev_index], st));
    CHK(launch_chk(launch_forces(s, st, fa, MODE_FINAL, false), "force"));
    if (timed) HIPCHK(hipEventRecord(s->ev[EV_PER_UNIT * ev_index + 1], st));
    // a sampled step: the energies and virials at the same positions (an evaluation that
    // rewrites the same forces)
    if (sample >= 0) CHK(launch_chk(launch_forces(s, st, fa, MODE_EVAL, true), "thermo eval"));
    int np = 0;
    CHK(launch_chk(launch_ke_partials(st, s->d_vel, 0, s->n, s->d_kpart, s->red_blocks, &np),
                   "kinetic energy"));
    CHK(launch_chk(launch_nvt_thermo(st, s->d_kpart, nvt_params(s, np, false), s->d_th),
                   "thermostat"));
    if (sample >= 0) CHK(enqueue_thermo_sample(s, st, sample, nullptr));
    return LJMD_OK;
}

int enqueue_unit(ljmd_system *s, hipStream_t st, int cur, bool timed, int ev_index,
                 int64_t sample = -1) {
    if (s->nvt) return enqueue_nvt_unit(s, st, cur, timed, ev_index, sample);
    ForceArgs fa = force_args(s, cur);
    if (timed) HIPCHK(hipEventRecord(s->ev[EV_PER_UNIT * ev_index], st));
    CHK(launch_chk(launch_forces(s, st, fa, MODE_FUSED, sample >= 0), "fused step"));
    if (timed) HIPCHK(hipEventRecord(s->ev[EV_PER_UNIT * ev_index + 1], st));
    if (sample >= 0) CHK(enqueue_thermo_sample(s, st, sample, s->d_ke));
    hipEvent_t *rev = timed ? &s->ev[EV_PER_UNIT * ev_index + 2] : nullptr;
    return launch_chk(launch_list_rebuild(s, st, s->d_req + (cur ^ 1), cur ^ 1, rev), "rebuild");
}

int capture_graph(ljmd_system *s, int cur) {
    if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    int c = cur;
    int rc = LJMD_OK;
    for (int u = 0; u < s->graph_steps && rc == LJMD_OK; ++u) {
        rc = enqueue_unit(s, s->cap_stream, c, false, 0);
        c ^= 1;
    }
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (rc != LJMD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_err(LJMD_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_err(LJMD_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    s->graph[cur] = ex;
    return LJMD_OK;
}

int ensure_events(ljmd_system *s, int64_t count) {
    while ((int64_t)s->ev.size() < EV_PER_UNIT * count) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        s->ev.push_back(e);
    }
    return LJMD_OK;
}

int snapshot(ljmd_system *s) {
    const size_t n = (size_t)s->n;
    HIPCHK(hipMemcpyAsync(s->d_snap_pos, s->d_pos[s->cur], n * sizeof(double4),
                          hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->d_snap_vel, s->d_vel, n * sizeof(double4), hipMemcpyDeviceToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_snap_img, s->d_img, n * sizeof(int4), hipMemcpyDeviceToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_snap_th, s->d_th, TH_COUNT * sizeof(double),
                          hipMemcpyDeviceToDevice, s->stream));
    return LJMD_OK;
}

int restore(ljmd_system *s, int cur0) {
    const size_t n = (size_t)s->n;
    s->cur = cur0;
    HIPCHK(hipMemcpyAsync(s->d_pos[s->cur], s->d_snap_pos, n * sizeof(double4),
                          hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->d_vel, s->d_snap_vel, n * sizeof(double4), hipMemcpyDeviceToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_img, s->d_snap_img, n * sizeof(int4), hipMemcpyDeviceToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->d_th, s->d_snap_th, TH_COUNT * sizeof(double),
                          hipMemcpyDeviceToDevice, s->stream));
    s->list_valid = false;
    s->force_valid = false;
    return LJMD_OK;
}

int collect_timing(ljmd_system *s, int64_t units) {
    for (int64_t u = 0; u < units; ++u) {
        const hipEvent_t *e = &s->ev[EV_PER_UNIT * u];
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
        s->t_ms += ms;
        s->dur[LJMD_KERNEL_STEP].push_back(ms);
        for (int k = 0; k < 5; ++k) {
            HIPCHK(hipEventElapsedTime(&ms, e[2 + k], e[3 + k]));
            s->dur[LJMD_KERNEL_BIN + k].push_back(ms);
        }
    }
    s->t_launches += units;
    return LJMD_OK;
}

// NVT: every step is one unit (no fused kick-kick-drift: the thermostat needs the kinetic
// energy between the two kicks); at the end the stored velocities take the pending scale.
int run_nvt_steps(ljmd_system *s, int64_t nsteps, bool *overflow, bool *nonfinite) {
    if (!s->nvt_ready) {
        CHK(enqueue_nvt_begin(s, s->stream));
        s->nvt_ready = true;
    }
    // sampled runs launch step by step (a graph's steps have no fixed step numbers)
    const bool use_graph = s->graph_steps > 0 && !s->timing && s->thermo_period == 0;
    if (s->timing) CHK(ensure_events(s, nsteps));
    int64_t done = 0;
    while (done < nsteps) {
        if (use_graph && nsteps - done >= s->graph_steps) {
            if (!s->graph[s->cur]) CHK(capture_graph(s, s->cur));
            HIPCHK(hipGraphLaunch(s->graph[s->cur], s->stream));
            done += s->graph_steps;
        } else {
            const int64_t step = s->steps + done + 1;
            CHK(enqueue_nvt_unit(s, s->stream, s->cur, s->timing, (int)done,
                                 thermo_due(s, step) ? step : -1));
            s->cur ^= 1;
            done += 1;
        }
    }
    CHK(launch_chk(launch_nvt_finalize(s->stream, s->d_vel, 0, s->n, s->d_th), "thermostat"));
    DevStatus st{};
    CHK(sync_status(s, &st));
    if (s->timing) CHK(collect_timing(s, nsteps));
    *overflow = (st.status & ST_OVERFLOW) != 0;
    *nonfinite = (st.status & (ST_NONFINITE | ST_TILE)) != 0;
    return LJMD_OK;
}

// One attempt at nsteps >= 1 steps from a ready state; reports overflow and non-finite
// forces through the flags.
int run_steps(ljmd_system *s, int64_t nsteps, bool *overflow, bool *nonfinite) {
    *overflow = false;
    *nonfinite = false;
    CHK(clear_status_bits(s));
    if (s->nvt) return run_nvt_steps(s, nsteps, overflow, nonfinite);
    // first half step from the stored forces
    {
        KickDriftArgs ka = kick_drift_args(s, s->cur);
        CHK(launch_chk(launch_kick_drift(s->stream, ka), "kick-drift"));
        s->cur ^= 1;
        CHK(launch_chk(launch_list_rebuild(s, s->stream, s->d_req + s->cur, s->cur), "rebuild"));
    }
    const int64_t units = nsteps - 1;
    // sampled runs launch step by step (a graph's steps have no fixed step numbers)
    const bool use_graph = s->graph_steps > 0 && !s->timing && s->thermo_period == 0;
    if (s->timing) CHK(ensure_events(s, units));
    int64_t done = 0;
    while (done < units) {
        if (use_graph && units - done >= s->graph_steps) {
            if (!s->graph[s->cur]) CHK(capture_graph(s, s->cur));
            HIPCHK(hipGraphLaunch(s->graph[s->cur], s->stream));
            done += s->graph_steps;  // graph_steps is even: cur is unchanged
        } else {
            // the fused kernel of unit `done` completes step s->steps + done + 1
            const int64_t step = s->steps + done + 1;
            CHK(enqueue_unit(s, s->stream, s->cur, s->timing, (int)done,
                             thermo_due(s, step) ? step : -1));
            s->cur ^= 1;
            done += 1;
        }
    }
    ForceArgs fa = force_args(s, s->cur);
    const int64_t last = s->steps + nsteps;
    CHK(launch_chk(launch_forces(s, s->stream, fa, MODE_FINAL, false), "final"));
    if (thermo_due(s, last)) {
        CHK(launch_chk(launch_forces(s, s->stream, fa, MODE_EVAL, true), "thermo eval"));
        CHK(enqueue_thermo_sample(s, s->stream, last, nullptr));
    }
    DevStatus st{};
    CHK(sync_status(s, &st));
    if (s->timing) CHK(collect_timing(s, units));
    *overflow = (st.status & ST_OVERFLOW) != 0;
    *nonfinite = (st.status & (ST_NONFINITE | ST_TILE)) != 0;
    return LJMD_OK;
}

bool finite_array(const double *p, size_t k) {
    for (size_t i = 0; i < k; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int fetch_vec(ljmd_system *s, const double4 *src, double *out) {
    CHK(launch_chk(launch_unsort_vec(s->stream, src, s->d_img, 0, s->n, s->d_stage), "unsort"));
    HIPCHK(hipMemcpyAsync(out, s->d_stage, 3 * (size_t)s->n * sizeof(double), hipMemcpyDeviceToHost,
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return LJMD_OK;
}

int eval_thermo(ljmd_system *s, double red[RED_QUANT]) {
    CHK(ensure_ready(s));
    CHK(enqueue_eval(s, true));
    CHK(launch_chk(launch_reduce(s->stream, s->d_u, s->d_w, nullptr, s->d_vel, 0, s->n,
                                 s->d_partials, s->red_blocks, s->d_red),
                   "reduce"));
    HIPCHK(hipMemcpyAsync(red, s->d_red, RED_QUANT * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return LJMD_OK;
}

// The current list with every entry as a sorted-order particle index: cnt[q] entries of row
// q at ent[q * cap ...]; img gives the tag of each sorted index (img[q].w).
int decode_list(ljmd_system *s, std::vector<int> &cnt, std::vector<int> &ent,
                std::vector<int4> &img) {
    CHK(ensure_ready(s));
    const size_t N = (size_t)s->n;
    if (s->nlist_method == LJMD_NLIST_TREE) {
        // 32-bit lists hold sorted indices already: copy and reorder rows on the host
        std::vector<int32_t> raw((size_t)s->cap * s->npad);
        cnt.assign(N, 0);
        img.assign(N, int4{});
        HIPCHK(hipMemcpyAsync(cnt.data(), s->d_count, N * sizeof(int), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipMemcpyAsync(img.data(), s->d_img, N * sizeof(int4), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipMemcpyAsync(raw.data(), s->d_nlist32, raw.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        ent.assign(N * (size_t)s->cap, 0);
        const int sh = 2 + s->lshift;
        for (size_t q = 0; q < N; ++q) {
            const int c = std::min(cnt[q], s->cap);
            for (int k = 0; k < c; ++k) {
                const size_t slot = (size_t)((unsigned)k >> sh) * ((size_t)s->npad << sh) +
                                    (q << sh) + (size_t)(k & ((1 << sh) - 1));
                ent[q * (size_t)s->cap + k] = raw[slot];
            }
        }
        return LJMD_OK;
    }
    int *d_out = nullptr;
    CHK(dalloc_t(s, &d_out, N * (size_t)s->cap));
    RebuildArgs ra = rebuild_args(s, s->d_one, s->cur);
    int rc = launch_chk(launch_decode_list(s->stream, ra, d_out), "decode list");
    cnt.assign(N, 0);
    ent.assign(N * (size_t)s->cap, 0);
    img.assign(N, int4{});
    if (rc == LJMD_OK &&
        (hipMemcpyAsync(cnt.data(), s->d_count, N * sizeof(int), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
         hipMemcpyAsync(img.data(), s->d_img, N * sizeof(int4), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
         hipMemcpyAsync(ent.data(), d_out, ent.size() * sizeof(int), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
         hipStreamSynchronize(s->stream) != hipSuccess))
        rc = set_err(LJMD_E_DEVICE, "copy of the decoded list failed");
    dfree(s, d_out);
    return rc;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

const char *ljmd_last_error(void) { return ljmd::g_last_error.c_str(); }

const char *ljmd_version(void) {
    return LJMD_DEBUG_CHECKS ? "ljmd 0.2 (gfx950, debug checks)" : "ljmd 0.2 (gfx950)";
}

int ljmd_tuning_get(ljmd_tuning_entry *out, int32_t capacity, int32_t *count) {
    if (!count || capacity < 0 || (capacity > 0 && !out))
        return set_err(LJMD_E_INVAL, "count must be non-null and out non-null when capacity > 0");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int32_t k = 0;
    for (const auto &kv : g_tune) {  // std::map: ordered by key
        if (k < capacity)
            out[k] = ljmd_tuning_entry{kv.first.prec == PREC_MIXED ? LJMD_MIXED : LJMD_FP64,
                                       kv.first.multi, kv.first.nbucket, kv.second.first,
                                       kv.second.second};
        ++k;
    }
    *count = k;
    return LJMD_OK;
}

int ljmd_tuning_set(const ljmd_tuning_entry *entries, int32_t n) {
    if (n < 0 || (n > 0 && !entries))
        return set_err(LJMD_E_INVAL, "entries must be non-null when n > 0");
    for (int32_t k = 0; k < n; ++k) {
        const ljmd_tuning_entry &e = entries[k];
        const int t = e.threads_per_particle;
        if ((e.precision != LJMD_FP64 && e.precision != LJMD_MIXED) ||
            (e.multi_type != 0 && e.multi_type != 1) || e.size_bucket < 0 ||
            e.size_bucket > 26 || !(t == 1 || t == 2 || t == 4 || t == 8) ||
            e.block_size < 128 || e.block_size > 512 || e.block_size % 64)
            return set_err(LJMD_E_INVAL, "tuning entry %d is out of range", (int)k);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int32_t k = 0; k < n; ++k) {
        const ljmd_tuning_entry &e = entries[k];
        const int prec = e.precision == LJMD_MIXED ? PREC_MIXED : PREC_FP64;
        g_tune[TuneKey{prec, e.multi_type, e.size_bucket}] = {e.threads_per_particle,
                                                              e.block_size};
    }
    return LJMD_OK;
}

int ljmd_system_create(const ljmd_config *cfg, int64_t n, const double *pos, const double *vel,
                       const int32_t *type, const double *mass, ljmd_system **out) {
    if (out) *out = nullptr;
    if (!cfg || !pos || !vel || !type || !out) return set_err(LJMD_E_INVAL, "null argument");
    if (n < 1 || n > (int64_t)(1 << 26)) return set_err(LJMD_E_INVAL, "n = %lld out of range", (long long)n);
    if (cfg->ntypes < 1 || cfg->ntypes > LJMD_MAX_TYPES)
        return set_err(LJMD_E_INVAL, "ntypes = %d out of range [1, %d]", cfg->ntypes, LJMD_MAX_TYPES);
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return set_err(LJMD_E_INVAL, "dt must be > 0");
    if (!(cfg->skin >= 0.0) || !std::isfinite(cfg->skin)) return set_err(LJMD_E_INVAL, "skin must be >= 0");
    for (int a = 0; a < 3; ++a)
        if (!(cfg->box[a] > 0.0) || !std::isfinite(cfg->box[a]))
            return set_err(LJMD_E_INVAL, "box edge %d must be finite and > 0", a);
    if (cfg->precision != LJMD_FP64 && cfg->precision != LJMD_MIXED)
        return set_err(LJMD_E_INVAL, "unknown precision %d", cfg->precision);
    const int tpp = cfg->threads_per_particle;
    if (tpp != 0 && tpp != 1 && tpp != 2 && tpp != 4 && tpp != 8 && tpp != 16)
        return set_err(LJMD_E_INVAL, "threads_per_particle must be 0, 1, 2, 4, 8 or 16");
    if (cfg->block_size != 0 && (cfg->block_size < 64 || cfg->block_size > 512 || cfg->block_size % 64))
        return set_err(LJMD_E_INVAL, "block_size must be 0 or a multiple of 64 up to 512");
    if (cfg->graph_steps != 0 && cfg->graph_steps != -1 && (cfg->graph_steps < 2 || cfg->graph_steps % 2))
        return set_err(LJMD_E_INVAL, "graph_steps must be 0, -1 or an even number >= 2");
    if (cfg->nlist_capacity < 0) return set_err(LJMD_E_INVAL, "nlist_capacity must be >= 0");
    if (!!cfg->alloc != !!cfg->free) return set_err(LJMD_E_INVAL, "alloc and free must be given together");
    if (!finite_array(pos, 3 * (size_t)n) || !finite_array(vel, 3 * (size_t)n))
        return set_err(LJMD_E_INVAL, "non-finite position or velocity");
    for (int64_t i = 0; i < n; ++i)
        if (type[i] < 0 || type[i] >= cfg->ntypes)
            return set_err(LJMD_E_INVAL, "type[%lld] = %d out of range", (long long)i, type[i]);
    if (mass)
        for (int64_t i = 0; i < n; ++i)
            if (!(mass[i] > 0.0) || !std::isfinite(mass[i]))
                return set_err(LJMD_E_INVAL, "mass[%lld] must be > 0", (long long)i);

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return set_err(LJMD_E_DEVICE, "no HIP device available");

    ljmd_system *s = new (std::nothrow) ljmd_system();
    if (!s) return set_err(LJMD_E_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) ==
                hipSuccess &&
            v > 0)
            s->lds_limit = (size_t)v;

    }
    s->stream = (hipStream_t)cfg->stream;
    s->mem.alloc = cfg->alloc;
    s->mem.free = cfg->free;
    s->mem.ctx = cfg->alloc_ctx;
    s->mem.stream = s->stream;
    s->n = (int)n;
    s->npad = (int)((n + 63) & ~63LL);
    for (int a = 0; a < 3; ++a) s->L[a] = cfg->box[a];
    s->ntypes = cfg->ntypes;
    const int nt2 = s->ntypes * s->ntypes;
    s->eps.assign(nt2, 0.0);
    s->sig.assign(nt2, 1.0);
    s->rc.assign(nt2, 0.0);
    s->is_set.assign(nt2, 0);
    s->pform.assign(nt2, STYLE_LJ);
    s->par.assign(4 * (size_t)nt2, 0.0);
    s->h_type.assign(type, type + n);
    if (mass) s->h_mass.assign(mass, mass + n);
    s->tpp = tpp;
    s->block = cfg->block_size;
    if (s->tpp) for (s->lshift = 0; (1 << s->lshift) < s->tpp; ++s->lshift) {}
    s->graph_steps = cfg->graph_steps == 0 ? 64 : (cfg->graph_steps < 0 ? 0 : cfg->graph_steps);

    const size_t N = (size_t)n;
    int rc = LJMD_OK;
    rc = rc ? rc : dalloc_t(s, &s->d_rep, 1);
    rc = rc ? rc : dalloc_t(s, &s->d_pair, nt2);
    rc = rc ? rc : dalloc_t(s, &s->d_rl2, nt2);
    rc = rc ? rc : dalloc_t(s, &s->d_req, 2);
    rc = rc ? rc : dalloc_t(s, &s->d_one, 1);
    rc = rc ? rc : dalloc_t(s, &s->d_pos[0], N);
    rc = rc ? rc : dalloc_t(s, &s->d_pos[1], N);
    rc = rc ? rc : dalloc_t(s, &s->d_pos_scr, N);
    rc = rc ? rc : dalloc_t(s, &s->d_vel, N);
    rc = rc ? rc : dalloc_t(s, &s->d_vel_scr, N);
    rc = rc ? rc : dalloc_t(s, &s->d_force, N);
    rc = rc ? rc : dalloc_t(s, &s->d_xb, N);
    rc = rc ? rc : dalloc_t(s, &s->d_img, N);
    rc = rc ? rc : dalloc_t(s, &s->d_img_scr, N);
    rc = rc ? rc : dalloc_t(s, &s->d_key, N);
    rc = rc ? rc : dalloc_t(s, &s->d_slot, N);
    rc = rc ? rc : dalloc_t(s, &s->d_perm, N);
    rc = rc ? rc : dalloc_t(s, &s->d_count, (size_t)s->npad);
    rc = rc ? rc : dalloc_t(s, &s->d_work, N);
    rc = rc ? rc : dalloc_t(s, &s->d_u, N);
    rc = rc ? rc : dalloc_t(s, &s->d_w, 6 * N);
    rc = rc ? rc : dalloc_t(s, &s->d_ke, N);
    rc = rc ? rc : dalloc_t(s, &s->d_partials, (size_t)RED_QUANT * s->red_blocks);
    rc = rc ? rc : dalloc_t(s, &s->d_red, (size_t)RED_QUANT);
    rc = rc ? rc : dalloc_t(s, &s->d_stage, 10 * N);
    rc = rc ? rc : dalloc_t(s, &s->d_snap_pos, N);
    rc = rc ? rc : dalloc_t(s, &s->d_snap_vel, N);
    rc = rc ? rc : dalloc_t(s, &s->d_snap_img, N);
    rc = rc ? rc : dalloc_t(s, &s->d_st, 1);
    rc = rc ? rc : dalloc_t(s, &s->d_th, TH_COUNT);
    rc = rc ? rc : dalloc_t(s, &s->d_snap_th, TH_COUNT);
    rc = rc ? rc : dalloc_t(s, &s->d_kpart, (size_t)s->red_blocks);
    if (rc != LJMD_OK) {
        ljmd_system_destroy(s);
        return rc;
    }
    // upload through the staging area: pos (3N) | vel (3N) | mass (N) | type (N ints)
    double *st_pos = s->d_stage, *st_vel = s->d_stage + 3 * N, *st_mass = s->d_stage + 6 * N;
    int *st_type = (int *)(s->d_stage + 7 * N);
    auto fail = [&](int code) {
        ljmd_system_destroy(s);
        return code;
    };
    static const int one = 1;
    static const double th0[TH_COUNT] = {0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    if (hipMemcpyAsync(st_pos, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_th, th0, sizeof th0, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(st_vel, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(st_type, type, N * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_one, &one, sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemsetAsync(s->d_req, 0, 2 * sizeof(int), s->stream) != hipSuccess ||
        (mass && hipMemcpyAsync(st_mass, mass, N * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess))
        return fail(set_err(LJMD_E_DEVICE, "host-to-device copy failed"));
    if (launch_upload(s->stream, st_pos, st_vel, st_type, mass ? st_mass : nullptr, s->d_pos[0],
                      s->d_vel, s->d_img, s->n, s->L, 1, 1, nullptr, 0) != hipSuccess ||
        launch_fill_status(s->stream, s->d_st) != hipSuccess)
        return fail(set_err(LJMD_E_DEVICE, "upload kernel failed"));
    if (hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(set_err(LJMD_E_DEVICE, "synchronisation after upload failed"));
    s->cur = 0;
    *out = s;
    return LJMD_OK;
}

void ljmd_system_destroy(ljmd_system *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    s->mem.release_all();
    delete s;
}

namespace {

// Store pair (a, b) of form `style` with parameters p[4] and cutoff rc (validated).
int store_pair(ljmd_system *s, int32_t a, int32_t b, int style, const double *p, double rc) {
    const int nt = s->ntypes;
    for (int k = 0; k < nt * nt; ++k) {
        const int x = k / nt, y = k % nt;
        const bool this_pair = (x == a && y == b) || (x == b && y == a);
        if (!this_pair && s->is_set[k] && s->pform[k] != style)
            return set_err(LJMD_E_INVAL, "pair (%d,%d) already uses another pair form: the "
                                         "kernels evaluate one form per system", x, y);
    }
    const int k1 = a * nt + b, k2 = b * nt + a;
    for (int k : {k1, k2}) {
        s->eps[k] = p[0];
        s->sig[k] = style == STYLE_YUKAWA ? 1.0 : p[1];
        s->rc[k] = rc;
        s->is_set[k] = 1;
        s->pform[k] = style;
        for (int c = 0; c < 4; ++c) s->par[4 * (size_t)k + c] = p[c];
    }
    s->style = style;
    s->table_dirty = true;
    s->list_valid = false;
    s->force_valid = false;
    return LJMD_OK;
}

}  // namespace

int ljmd_pair_lj_set(ljmd_system *s, int32_t a, int32_t b, double epsilon, double sigma, double r_cut) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (a < 0 || b < 0 || a >= s->ntypes || b >= s->ntypes)
        return set_err(LJMD_E_INVAL, "type pair (%d,%d) out of range", a, b);
    if (!std::isfinite(epsilon) || !(sigma > 0.0) || !std::isfinite(sigma) || !(r_cut >= 0.0) ||
        !std::isfinite(r_cut))
        return set_err(LJMD_E_INVAL, "need finite epsilon, sigma > 0, r_cut >= 0");
    const double p[4] = {epsilon, sigma, 0.0, 0.0};
    return store_pair(s, a, b, STYLE_LJ, p, r_cut);
}

int ljmd_pair_set(ljmd_system *s, int32_t a, int32_t b, int32_t form, const double *params,
                  int32_t nparams, double r_cut) {
    if (!s || !params) return set_err(LJMD_E_INVAL, "null argument");
    if (a < 0 || b < 0 || a >= s->ntypes || b >= s->ntypes)
        return set_err(LJMD_E_INVAL, "type pair (%d,%d) out of range", a, b);
    const int need = form == LJMD_PAIR_MIE ? 4 : 2;
    if (form < LJMD_PAIR_LJ || form > LJMD_PAIR_WCA)
        return set_err(LJMD_E_INVAL, "unknown pair form %d", form);
    if (nparams != need) return set_err(LJMD_E_INVAL, "pair form %d takes %d parameters", form, need);
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < need; ++c) {
        if (!std::isfinite(params[c])) return set_err(LJMD_E_INVAL, "non-finite parameter");
        p[c] = params[c];
    }
    if (form == LJMD_PAIR_WCA) {
        if (r_cut != 0.0) return set_err(LJMD_E_INVAL, "WCA takes r_cut = 0 (its cut is 2^(1/6) sigma)");
        if (!(p[1] > 0.0)) return set_err(LJMD_E_INVAL, "need sigma > 0");
        return store_pair(s, a, b, STYLE_LJ, p, std::pow(2.0, 1.0 / 6.0) * p[1]);
    }
    if (!(r_cut >= 0.0) || !std::isfinite(r_cut)) return set_err(LJMD_E_INVAL, "need r_cut >= 0");
    switch (form) {
        case LJMD_PAIR_LJ:
            if (!(p[1] > 0.0)) return set_err(LJMD_E_INVAL, "need sigma > 0");
            return store_pair(s, a, b, STYLE_LJ, p, r_cut);
        case LJMD_PAIR_MIE:
            if (!(p[1] > 0.0) || !(p[3] > 0.0) || !(p[2] > p[3]))
                return set_err(LJMD_E_INVAL, "Mie needs sigma > 0 and n > m > 0");
            return store_pair(s, a, b, STYLE_MIE, p, r_cut);
        case LJMD_PAIR_GAUSS:
            if (!(p[1] > 0.0)) return set_err(LJMD_E_INVAL, "need sigma > 0");
            return store_pair(s, a, b, STYLE_GAUSS, p, r_cut);
        default:
            if (!(p[1] >= 0.0)) return set_err(LJMD_E_INVAL, "Yukawa needs kappa >= 0");
            return store_pair(s, a, b, STYLE_YUKAWA, p, r_cut);
    }
}

int ljmd_step(ljmd_system *s, int64_t nsteps) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (nsteps < 0) return set_err(LJMD_E_INVAL, "nsteps must be >= 0");
    CHK(ensure_ready(s));
    const int64_t seg = 1000000;
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t k = std::min(left, seg);
        const int cur0 = s->cur;
        if (s->nvt && !s->nvt_ready) {
            // the thermostat half step opening the first step, before the snapshot that a
            // re-run after a list overflow restores
            CHK(enqueue_nvt_begin(s, s->stream));
            s->nvt_ready = true;
        }
        CHK(snapshot(s));
        const int64_t thermo0 = s->thermo_written;
        for (int attempt = 0;; ++attempt) {
            bool over = false, nonfin = false;
            s->thermo_written = thermo0;  // a re-run rewrites the samples of the failed one
            CHK(run_steps(s, k, &over, &nonfin));
            if (nonfin) {
                DevStatus st{};
                CHK(sync_status(s, &st));
                CHK(restore(s, cur0));
                s->thermo_written = thermo0;
                if (st.status & ST_TILE)
                    return set_err(LJMD_E_BOX, "a brick holds more than %d atoms in its halo "
                                               "cells; state restored", TILE_INDEX_MAX);
                return set_err(LJMD_E_NONFINITE, "non-finite force during the step; state restored");
            }
            if (!over) break;
            if (attempt >= 8) return set_err(LJMD_E_DEVICE, "list overflow persisted after growth");
            DevStatus st{};
            CHK(sync_status(s, &st));
            CHK(restore(s, cur0));
            CHK(ensure_list_alloc(s, round_cap(1.25 * st.max_count + 8)));
            s->overflow_retries += 1;
            CHK(ensure_ready(s));
        }
        s->steps += k;
        left -= k;
    }
    return LJMD_OK;
}

int ljmd_get_forces(ljmd_system *s, double *out) {
    if (!s || !out) return set_err(LJMD_E_INVAL, "null argument");
    CHK(ensure_ready(s));
    return fetch_vec(s, s->d_force, out);
}

int ljmd_get_energy(ljmd_system *s, double *potential, double *kinetic) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    double red[RED_QUANT];
    CHK(eval_thermo(s, red));
    if (potential) *potential = red[0];
    if (kinetic) *kinetic = red[7];
    return LJMD_OK;
}

int ljmd_get_virial(ljmd_system *s, double *out6) {
    if (!s || !out6) return set_err(LJMD_E_INVAL, "null argument");
    double red[RED_QUANT];
    CHK(eval_thermo(s, red));
    for (int c = 0; c < 6; ++c) out6[c] = red[1 + c];
    return LJMD_OK;
}

int ljmd_get_per_particle(ljmd_system *s, double *u, double *w) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    CHK(ensure_ready(s));
    CHK(enqueue_eval(s, true));
    const size_t N = (size_t)s->n;
    if (u) {
        CHK(launch_chk(launch_unsort_scalar(s->stream, s->d_u, 1, s->d_img, 0, s->n, s->d_stage), "unsort"));
        HIPCHK(hipMemcpyAsync(u, s->d_stage, N * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    if (w) {
        CHK(launch_chk(launch_unsort_scalar(s->stream, s->d_w, 6, s->d_img, 0, s->n, s->d_stage), "unsort"));
        HIPCHK(hipMemcpyAsync(w, s->d_stage, 6 * N * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return LJMD_OK;
}

int ljmd_get_state(ljmd_system *s, double *pos, double *vel, int32_t *img, int64_t *step) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (pos) CHK(fetch_vec(s, s->d_pos[s->cur], pos));
    if (vel) CHK(fetch_vec(s, s->d_vel, vel));
    if (img) {
        CHK(launch_chk(launch_unsort_img(s->stream, s->d_img, 0, s->n, (int *)s->d_stage), "unsort"));
        HIPCHK(hipMemcpyAsync(img, s->d_stage, 3 * (size_t)s->n * sizeof(int), hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    if (step) *step = s->steps;
    return LJMD_OK;
}

int ljmd_set_state(ljmd_system *s, const double *pos, const double *vel, const int32_t *img,
                   const int64_t *step) {
    if (!s || !pos || !vel) return set_err(LJMD_E_INVAL, "positions and velocities are required");
    const size_t N = (size_t)s->n;
    if (!finite_array(pos, 3 * N) || !finite_array(vel, 3 * N))
        return set_err(LJMD_E_INVAL, "non-finite position or velocity");
    double *st_pos = s->d_stage, *st_vel = s->d_stage + 3 * N, *st_mass = s->d_stage + 6 * N;
    int *st_type = (int *)(s->d_stage + 7 * N);
    int *st_img = (int *)(s->d_stage + 8 * N);
    HIPCHK(hipMemcpyAsync(st_pos, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(st_vel, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(st_type, s->h_type.data(), N * sizeof(int), hipMemcpyHostToDevice, s->stream));
    if (!s->h_mass.empty())
        HIPCHK(hipMemcpyAsync(st_mass, s->h_mass.data(), N * sizeof(double), hipMemcpyHostToDevice, s->stream));
    if (img) HIPCHK(hipMemcpyAsync(st_img, img, 3 * N * sizeof(int), hipMemcpyHostToDevice, s->stream));
    s->cur = 0;
    CHK(launch_chk(launch_upload(s->stream, st_pos, st_vel, st_type, s->h_mass.empty() ? nullptr : st_mass,
                                 s->d_pos[0], s->d_vel, s->d_img, s->n, s->L, 1, 1, img ? st_img : nullptr, 0),
                   "upload"));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (step) s->steps = *step;
    s->list_valid = false;
    s->force_valid = false;
    s->nvt_ready = false;  // new velocities: the opening thermostat half step is redone
    return LJMD_OK;
}

int ljmd_set_nvt(ljmd_system *s, double kT, double tau) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (!(kT > 0.0) || !std::isfinite(kT) || !(tau > 0.0) || std::isnan(tau))
        return set_err(LJMD_E_INVAL, "need kT > 0 and tau > 0 (tau may be infinite)");
    if (s->n < 2) return set_err(LJMD_E_INVAL, "NVT needs at least two particles");
    const double ndof = 3.0 * (double)s->n - 3.0;
    s->nvt = true;
    s->nvt_kT = kT;
    s->nvt_g = ndof * kT;
    s->nvt_invQ = std::isinf(tau) ? 0.0 : 1.0 / (ndof * kT * tau * tau);
    s->nvt_ready = false;
    drop_graphs(s);
    static const double th0[TH_COUNT] = {0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    HIPCHK(hipMemcpyAsync(s->d_th, th0, sizeof th0, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return LJMD_OK;
}

int ljmd_set_nve(ljmd_system *s) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (s->nvt) drop_graphs(s);
    s->nvt = false;
    s->nvt_ready = false;
    return LJMD_OK;
}

int ljmd_get_thermostat(ljmd_system *s, double *xi, double *eta, double *energy) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    double th[TH_COUNT];
    HIPCHK(hipMemcpyAsync(th, s->d_th, sizeof th, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (!s->nvt) th[TH_XI] = th[TH_ETA] = 0.0;
    if (xi) *xi = th[TH_XI];
    if (eta) *eta = th[TH_ETA];
    if (energy)
        *energy = (s->nvt && s->nvt_invQ > 0.0)
                      ? 0.5 * th[TH_XI] * th[TH_XI] / s->nvt_invQ + s->nvt_g * th[TH_ETA]
                      : 0.0;
    return LJMD_OK;
}

int ljmd_set_thermostat(ljmd_system *s, double xi, double eta) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (!std::isfinite(xi) || !std::isfinite(eta)) return set_err(LJMD_E_INVAL, "non-finite value");
    if (!s->nvt) return set_err(LJMD_E_STATE, "the system is not under NVT (ljmd_set_nvt)");
    const double v[2] = {xi, eta};
    HIPCHK(hipMemcpyAsync(s->d_th + TH_XI, v, sizeof v, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->nvt_ready = false;
    return LJMD_OK;
}

int ljmd_negate_velocities(ljmd_system *s) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    CHK(launch_chk(launch_negate_vel(s->stream, s->d_vel, 0, s->n), "negate"));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->nvt_ready = false;
    return LJMD_OK;
}

int ljmd_set_pair_shift(ljmd_system *s, int32_t mode) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (mode != LJMD_SHIFT_ENERGY && mode != LJMD_SHIFT_FORCE)
        return set_err(LJMD_E_INVAL, "unknown shift mode %d", mode);
    if ((mode == LJMD_SHIFT_FORCE) == (s->shift_force != 0)) return LJMD_OK;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->shift_force = mode == LJMD_SHIFT_FORCE;
    s->table_dirty = true;  // coefficients change; the list radii do not
    s->force_valid = false;
    drop_graphs(s);
    return LJMD_OK;
}

int ljmd_set_thermo(ljmd_system *s, int32_t period, int32_t capacity) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (period < 0) return set_err(LJMD_E_INVAL, "thermo period %d is negative", period);
    if (period > 0 && (capacity < 1 || capacity > LJMD_THERMO_MAX_ROWS))
        return set_err(LJMD_E_INVAL, "thermo capacity %d outside [1, %d]", capacity,
                       LJMD_THERMO_MAX_ROWS);
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->d_thermo) dfree(s, s->d_thermo);
    s->d_thermo = nullptr;
    s->thermo_period = 0;
    s->thermo_cap = 0;
    s->thermo_written = 0;
    s->thermo_step.clear();
    if (period == 0) return LJMD_OK;
    CHK(dalloc_t(s, &s->d_thermo, (size_t)capacity * RED_QUANT));
    s->thermo_step.assign((size_t)capacity, 0);
    s->thermo_period = period;
    s->thermo_cap = capacity;
    return LJMD_OK;
}

int ljmd_get_thermo(ljmd_system *s, double *rows, int32_t max_rows, int32_t *nrows) {
    if (!s || !nrows) return set_err(LJMD_E_INVAL, "null argument");
    const int avail = (int)std::min<int64_t>(s->thermo_written, s->thermo_cap);
    if (!rows) {
        *nrows = avail;
        return LJMD_OK;
    }
    if (max_rows < 0) return set_err(LJMD_E_INVAL, "max_rows %d is negative", max_rows);
    const int take = std::min(avail, (int)max_rows);
    *nrows = take;
    if (take == 0) return LJMD_OK;
    std::vector<double> raw((size_t)s->thermo_cap * RED_QUANT);
    HIPCHK(hipMemcpyAsync(raw.data(), s->d_thermo, raw.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const double vol = s->L[0] * s->L[1] * s->L[2];
    const double ndof = 3.0 * (double)s->n - 3.0;
    for (int r = 0; r < take; ++r) {
        // the most recent `take` samples, oldest first
        const int64_t idx = s->thermo_written - take + r;
        const int slot = (int)(idx % s->thermo_cap);
        const double *q = raw.data() + (size_t)slot * RED_QUANT;  // U, W[6], K
        double *o = rows + (size_t)r * LJMD_THERMO_COLS;
        const double U = q[0], K = q[7];
        o[0] = (double)s->thermo_step[slot];
        o[1] = K;
        o[2] = U;
        o[3] = K + U;
        o[4] = ndof > 0.0 ? 2.0 * K / ndof : 0.0;
        o[5] = (2.0 * K + q[1] + q[4] + q[6]) / (3.0 * vol);
        for (int c = 0; c < 6; ++c) o[6 + c] = q[1 + c];
    }
    return LJMD_OK;
}

int ljmd_set_nlist(ljmd_system *s, int32_t method) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (method != LJMD_NLIST_CELL && method != LJMD_NLIST_TREE)
        return set_err(LJMD_E_INVAL, "unknown neighbour-list method %d", method);
    if (method == s->nlist_method) return LJMD_OK;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->nlist_method = method;
    s->cap = 0;  // the list is sized afresh for the method's layout
    s->table_dirty = true;
    s->list_valid = false;
    s->force_valid = false;
    drop_graphs(s);
    return LJMD_OK;
}

int ljmd_get_neighbor_pairs(ljmd_system *s, int64_t *count, int32_t *pairs, double *build_pos) {
    if (!s || !count) return set_err(LJMD_E_INVAL, "null argument");
    std::vector<int> cnt, ent;
    std::vector<int4> img;
    CHK(decode_list(s, cnt, ent, img));
    const size_t N = (size_t)s->n;
    std::vector<std::pair<int, int>> pr;
    for (size_t q = 0; q < N; ++q) {
        const int c = std::min(cnt[q], s->cap);
        for (int k = 0; k < c; ++k) {
            const int j = ent[q * (size_t)s->cap + k];
            const int a = img[q].w, b = img[j].w;
            if (a < b) pr.emplace_back(a, b);
        }
    }
    std::sort(pr.begin(), pr.end());
    *count = (int64_t)pr.size();
    if (pairs)
        for (size_t p = 0; p < pr.size(); ++p) {
            pairs[2 * p] = pr[p].first;
            pairs[2 * p + 1] = pr[p].second;
        }
    if (build_pos) CHK(fetch_vec(s, s->d_xb, build_pos));
    return LJMD_OK;
}

int ljmd_get_neighbor_list(ljmd_system *s, int32_t *counts, int64_t *total, int32_t *neighbors,
                           double *build_pos) {
    if (!s || !total) return set_err(LJMD_E_INVAL, "null argument");
    std::vector<int> cnt, ent;
    std::vector<int4> img;
    CHK(decode_list(s, cnt, ent, img));
    const size_t N = (size_t)s->n;
    // rows by tag: the sorted index of each tag
    std::vector<int> at(N);
    for (size_t q = 0; q < N; ++q) at[(size_t)img[q].w] = (int)q;
    int64_t tot = 0;
    for (size_t t = 0; t < N; ++t) {
        const int c = std::min(cnt[at[t]], s->cap);
        if (counts) counts[t] = c;
        if (neighbors)
            for (int k = 0; k < c; ++k)
                neighbors[tot + k] = img[ent[(size_t)at[t] * s->cap + k]].w;
        tot += c;
    }
    *total = tot;
    if (build_pos) CHK(fetch_vec(s, s->d_xb, build_pos));
    return LJMD_OK;
}

int ljmd_get_stats(ljmd_system *s, ljmd_stats *out) {
    if (!s || !out) return set_err(LJMD_E_INVAL, "null argument");
    DevStatus st{};
    CHK(sync_status(s, &st));
    std::memset(out, 0, sizeof *out);
    out->steps = s->steps;
    out->rebuilds = (int64_t)st.builds;
    out->max_neighbors = st.max_count;
    out->nlist_capacity = s->cap;
    out->overflow_retries = s->overflow_retries;
    out->threads_per_particle = s->tpp;
    out->block_size = s->block;
    for (int a = 0; a < 3; ++a) out->ncell[a] = s->rep.nc[a];
    out->graph_steps = s->graph_steps;
    out->device_bytes = s->mem.bytes;
    out->list_entries = (int64_t)st.entries;
    return LJMD_OK;
}

int ljmd_set_kernel_timing(ljmd_system *s, int32_t on) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    s->timing = on != 0;
    s->t_launches = 0;
    s->t_ms = 0.0;
    for (auto &d : s->dur) d.clear();
    return LJMD_OK;
}

int ljmd_kernel_time(ljmd_system *s, int64_t *launches, double *total_ms) {
    if (!s) return set_err(LJMD_E_INVAL, "null handle");
    if (launches) *launches = s->t_launches;
    if (total_ms) *total_ms = s->t_ms;
    return LJMD_OK;
}

int ljmd_kernel_durations(ljmd_system *s, int32_t kind, int64_t *count, float *ms) {
    if (!s || !count) return set_err(LJMD_E_INVAL, "null argument");
    if (kind < 0 || kind >= LJMD_KERNEL_KINDS) return set_err(LJMD_E_INVAL, "unknown kernel kind %d", kind);
    const std::vector<float> &d = s->dur[kind];
    *count = (int64_t)d.size();
    if (ms && !d.empty()) std::memcpy(ms, d.data(), d.size() * sizeof(float));
    return LJMD_OK;
}

}  // extern "C"
