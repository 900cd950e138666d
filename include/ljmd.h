/*
 * ljmd.h -- C ABI of the MI355X (gfx950) Lennard-Jones molecular-dynamics hot path.
 *
 * The calls follow the paper's statement of an MD simulation (Section "Capabilities",
 * Molecular dynamics listing; Section "Python package"): build a system from a periodic
 * box and particles, set Lennard-Jones epsilon, sigma and r_cut per type pair through a
 * cell-list neighbour list, set the time step, run a number of NVE steps, and read the
 * force, energy and virial that the paper's pair-force unit test checks (Section "Software
 * engineering", Testing).
 *
 * Definitions used throughout (the paper names the method; these are the textbook forms):
 *   minimum image  d = x_j - x_i per axis, reduced into [-L/2, L/2) by adding or
 *                  subtracting one box length.
 *   pair energy    u(r) = 4 eps ((s/r)^12 - (s/r)^6) - 4 eps ((s/r_cut)^12 - (s/r_cut)^6)
 *                  for r < r_cut, else 0 (truncated and shifted).
 *   pair force     on i from j: 24 eps (2 (s/r)^12 - (s/r)^6) / r^2 * (x_i - x_j), not
 *                  shifted, zero for r >= r_cut.
 *   virial         W_ab = sum over pairs (i<j) of (x_i - x_j)_a F_ij,b, stored as
 *                  (xx, xy, xz, yy, yz, zz).
 *   neighbour list all j with r^2 < (r_cut_ab + skin)^2, rebuilt when any particle has
 *                  moved (minimum image) at least skin/2 since the last build.
 *   step           velocity Verlet: v += dt/(2m) F; x += dt v (wrapped into [0, L), image
 *                  counters updated); F recomputed; v += dt/(2m) F.
 *
 * Conventions
 *   - Every function returns LJMD_OK (0) or a negative LJMD_E_* status; ljmd_last_error()
 *     then gives a message. No C++ exception crosses this interface.
 *   - Host arrays passed in are copied; the caller keeps ownership. Output arrays are
 *     allocated by the caller, host memory, in input (tag) order: particle k of the
 *     arrays given to ljmd_system_create is particle k of every output.
 *   - Device state is owned by the handle and allocated through the configured allocator
 *     on the configured stream. All device work is enqueued on that stream.
 *   - A handle must be used by one host thread at a time.
 *   - Array shapes: positions, velocities and forces are n x 3 doubles, row-major
 *     (x0 y0 z0 x1 ...); per-particle virials are n x 6 doubles in (xx,xy,xz,yy,yz,zz).
 */
#ifndef LJMD_H
#define LJMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LJMD_OK 0
#define LJMD_E_INVAL -1     /* null pointer, n < 1, type out of range, dt <= 0, sigma <= 0,
                               r_cut < 0, non-finite input, unknown option */
#define LJMD_E_NOMEM -2     /* the allocator returned NULL */
#define LJMD_E_DEVICE -3    /* no usable GPU, or a HIP runtime error */
#define LJMD_E_BOX -4       /* max over pairs of (r_cut + skin) exceeds half a box edge */
#define LJMD_E_NONFINITE -5 /* a force became non-finite (for example overlapping particles) */
#define LJMD_E_STATE -6     /* a type pair has not been set, or a batch slot is not ready */
#define LJMD_E_CAPACITY -7  /* batch admission: no free slot or not enough memory budget */

/* precision of the pair arithmetic */
#define LJMD_FP64 0  /* everything in FP64 */
#define LJMD_MIXED 1 /* FP32 pair arithmetic; FP64 positions, velocities, integration and
                        energy/virial sums */

/* Device memory callbacks. alloc returns device memory of at least `bytes` usable on
 * `stream`, or NULL; free releases it. With both NULL the library uses hipMalloc/hipFree. */
typedef void *(*ljmd_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*ljmd_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);

typedef struct ljmd_config {
    double box[3];          /* orthorhombic box edges L_x, L_y, L_z (> 0) */
    int32_t ntypes;         /* number of particle types, 1..LJMD_MAX_TYPES */
    double dt;              /* time step (> 0), reduced units */
    double skin;            /* Verlet skin r_s (>= 0) */
    int32_t precision;      /* LJMD_FP64 or LJMD_MIXED */
    int32_t nlist_capacity; /* entries per particle; 0 = sized from the first build */
    int32_t threads_per_particle; /* lanes per particle in the force kernel: 1,2,4,8,16
                                     or 0 = autotuned */
    int32_t block_size;     /* force kernel workgroup size: a multiple of 64 up to 512;
                               0 = autotuned */
    int32_t graph_steps;    /* steps per captured HIP graph block (even, >= 2); 0 = 64;
                               -1 disables graphs */
    void *stream;           /* hipStream_t; NULL = the default stream */
    ljmd_alloc_fn alloc;    /* NULL = hipMalloc */
    ljmd_free_fn free;      /* NULL = hipFree */
    void *alloc_ctx;        /* passed through to alloc/free */
} ljmd_config;

#define LJMD_MAX_TYPES 16

typedef struct ljmd_stats {
    int64_t steps;            /* steps taken since create */
    int64_t rebuilds;         /* neighbour-list builds (from the device counter) */
    int32_t max_neighbors;    /* largest list length seen at a build */
    int32_t nlist_capacity;   /* current entries per particle */
    int64_t overflow_retries; /* step segments re-run after growing the list */
    int32_t threads_per_particle;
    int32_t block_size;
    int32_t ncell[3];         /* cells per axis */
    int32_t graph_steps;
    int64_t device_bytes;     /* device memory held by the handle */
    int64_t list_entries;     /* entries stored by the last list build (sum over particles) */
} ljmd_stats;

typedef struct ljmd_system ljmd_system;

/* Create a system of n particles, 1 <= n <= 2^26. pos, vel: n x 3 host doubles (positions
 * may lie outside the box; they are wrapped, with image counters). type: n host int32 in [0, ntypes).
 * mass: n host doubles (> 0) or NULL for unit masses. Pair coefficients must then be set
 * with ljmd_pair_lj_set for every type pair before stepping or reading. *out receives the
 * handle, or NULL on error. Errors: INVAL, NOMEM, DEVICE. */
int ljmd_system_create(const ljmd_config *cfg, int64_t n, const double *pos,
                       const double *vel, const int32_t *type, const double *mass,
                       ljmd_system **out);

/* Frees all device memory through the same allocator. NULL is ignored. */
void ljmd_system_destroy(ljmd_system *sys);

/* Set the LJ pair (a, b), symmetric in a and b. r_cut = 0 disables the pair. May be
 * called at any time (the paper's unit test changes parameters between evaluations); the
 * list and forces are rebuilt before the next step or read. Errors: INVAL. */
int ljmd_pair_lj_set(ljmd_system *sys, int32_t a, int32_t b, double epsilon, double sigma,
                     double r_cut);

/* Pair forms on the same skeleton (the paper lists Gaussian, Mie, WCA and Yukawa among its
 * pair potentials, Section "Capabilities"). Each is truncated at r_cut with its energy
 * shifted to 0 there and its force not shifted; F on i = f(r) (x_i - x_j):
 *   LJMD_PAIR_LJ      params (eps, sigma): the LJ form above (as ljmd_pair_lj_set)
 *   LJMD_PAIR_MIE     params (eps, sigma, n, m), n > m > 0:
 *                     u = C eps ((s/r)^n - (s/r)^m), C = (n/(n-m)) (n/m)^(m/(n-m))
 *   LJMD_PAIR_GAUSS   params (eps, sigma): u = eps exp(-r^2 / (2 sigma^2))
 *   LJMD_PAIR_YUKAWA  params (eps, kappa): u = eps exp(-kappa r) / r
 *   LJMD_PAIR_WCA     params (eps, sigma), r_cut = 0: the LJ form cut at 2^(1/6) sigma
 *                     (purely repulsive; the shift is +eps)
 * Every set pair of a system uses one form (the kernels evaluate one form per system);
 * batches use the LJ form. Errors: INVAL (unknown form, wrong parameter count, out-of-range
 * parameter, a second form in one system). */
#define LJMD_PAIR_LJ 0
#define LJMD_PAIR_MIE 1
#define LJMD_PAIR_GAUSS 2
#define LJMD_PAIR_YUKAWA 3
#define LJMD_PAIR_WCA 4
int ljmd_pair_set(ljmd_system *sys, int32_t a, int32_t b, int32_t form, const double *params,
                  int32_t nparams, double r_cut);

/* Advance nsteps velocity-Verlet steps (NVE, or NVT after ljmd_set_nvt) on the configured
 * stream and synchronise once at the end to report status. nsteps = 0 only makes the list
 * and forces current.
 * Errors: INVAL, STATE (pair unset), BOX, NONFINITE, NOMEM, DEVICE. On NONFINITE the
 * state is restored to what it was when the call began. */
int ljmd_step(ljmd_system *sys, int64_t nsteps);

/* NVT: the integrator of the paper's MD listing (Section "Capabilities": integrate.nvt with
 * kT and tau, built on the Martyna-Tobias-Klein method). One Nose-Hoover thermostat
 * variable xi (with "position" eta) of mass Q = N_f kT tau^2, N_f = 3n - 3, acting on
 *   dx/dt = v,  dv/dt = F/m - xi v,  dxi/dt = (2K - N_f kT) / Q,  deta/dt = xi,
 * integrated by the symmetric (time-reversible) splitting: each step is a thermostat half
 * step, the velocity-Verlet step, and another thermostat half step, where a half step of
 * length dt/2 is xi += (dt/4) G; eta += (dt/2) xi; v *= exp(-(dt/2) xi) (K scales by the
 * square); xi += (dt/4) G, with G = (2K - N_f kT) / Q. K + U + Q xi^2 / 2 + N_f kT eta is
 * conserved. tau = +infinity means zero coupling (the NVE step). Sets xi = eta = 0.
 * Errors: INVAL (kT <= 0, tau <= 0, n < 2). */
int ljmd_set_nvt(ljmd_system *sys, double kT, double tau);

/* Back to NVE steps (the thermostat variables are kept but no longer used). */
int ljmd_set_nve(ljmd_system *sys);

/* Thermostat state at the current step: xi, eta and its share of the conserved quantity,
 * Q xi^2 / 2 + N_f kT eta (all 0 under NVE or zero coupling); pointers may be NULL. */
int ljmd_get_thermostat(ljmd_system *sys, double *xi, double *eta, double *energy);

/* Set xi and eta (checkpoint/resume, reversibility checks). Errors: INVAL, STATE (not NVT). */
int ljmd_set_thermostat(ljmd_system *sys, double xi, double eta);

/* v -> -v for every particle (time-reversal checks); forces stay valid. */
int ljmd_negate_velocities(ljmd_system *sys);

/* Forces at the current positions, n x 3 host doubles, tag order. */
int ljmd_get_forces(ljmd_system *sys, double *out);

/* Total shifted LJ potential energy and kinetic energy (sum of m v^2 / 2 over full-step
 * velocities); either pointer may be NULL. Reduced in FP64 in a fixed order. */
int ljmd_get_energy(ljmd_system *sys, double *potential, double *kinetic);

/* Virial tensor W (6 doubles, xx xy xz yy yz zz), reduced in FP64 in a fixed order. */
int ljmd_get_virial(ljmd_system *sys, double *out6);

/* Per-particle halves of each pair's energy (n doubles) and virial (n x 6 doubles), tag
 * order; either pointer may be NULL. */
int ljmd_get_per_particle(ljmd_system *sys, double *u, double *w);

/* Checkpoint: positions (wrapped, n x 3), velocities (n x 3), image counters (n x 3 int32)
 * and the step counter; any pointer may be NULL. */
int ljmd_get_state(ljmd_system *sys, double *pos, double *vel, int32_t *img, int64_t *step);

/* Resume: replace positions (required; wrapped on upload), velocities (required), image
 * counters (NULL = all zero; added to the images the wrap produces) and the step counter
 * (NULL = keep). Types and masses are those given at create. Forces a list rebuild. */
int ljmd_set_state(ljmd_system *sys, const double *pos, const double *vel, const int32_t *img,
                   const int64_t *step);

/* Neighbour-list method (Section "Performance": the cell list, and the bounding volume
 * hierarchy of nlist.tree for size-disperse systems, where a cell list sized for the largest
 * cutoff makes small particles scan many cells to find few neighbours):
 *   LJMD_NLIST_CELL  (default) cells at least as wide as the largest list radius, grouped into
 *                    bricks whose halo atoms are staged in LDS; 16-bit tile-index lists.
 *   LJMD_NLIST_TREE  one binary radix tree per particle type over that type's particles (in
 *                    Morton order of fine cells), walked by each particle with its list radius
 *                    for that type pair; 32-bit index lists. LJ form only.
 * Both produce the same pair set (the definition above); list order, and hence the rounding
 * of the force sums, differs. Changing the method rebuilds the list before the next step or
 * read. Errors: INVAL (unknown method; the tree with another pair form at the next step). */
#define LJMD_NLIST_CELL 0
#define LJMD_NLIST_TREE 1
int ljmd_set_nlist(ljmd_system *sys, int32_t method);

/* How every pair form of the system is truncated at its r_cut:
 *   LJMD_SHIFT_ENERGY  (default) the energy is shifted to 0 at r_cut, the force is not (it
 *                      jumps to 0 there), as the paper's LJ pair force does by default.
 *   LJMD_SHIFT_FORCE   shifted force, for tighter energy conservation: with F(r) the pair
 *                      force magnitude (positive when repulsive) and F_c = F(r_cut), the
 *                      force is F(r) - F_c and the energy u(r) - u(r_cut) + (r - r_cut) F_c,
 *                      so both vanish at r_cut and the force stays -du/dr.
 * Applies to the LJ form and to every form of ljmd_pair_set; the next step or read uses it.
 * Errors: INVAL (unknown mode; the tree lists with the shifted force, at the next step). */
#define LJMD_SHIFT_ENERGY 0
#define LJMD_SHIFT_FORCE 1
int ljmd_set_pair_shift(ljmd_system *sys, int32_t mode);

/* Thermodynamic samples during ljmd_step (Section "Python package": a run's system
 * quantities followed over time). With period > 0, every step whose number (the step
 * counter, see ljmd_get_state) is a positive multiple of period is sampled on the device,
 * with no host round trip: the potential energy, the virial and the kinetic energy at that
 * full step, reduced in FP64 in a fixed order into a ring of `capacity` rows that keeps the
 * latest ones. In NVT runs K is the thermostat's, after its closing half step. Sampled runs
 * launch their steps one by one instead of as graphs. period = 0 turns sampling off;
 * (re)configuring clears the ring. Errors: INVAL (period < 0, capacity outside
 * [1, LJMD_THERMO_MAX_ROWS] with period > 0). */
#define LJMD_THERMO_MAX_ROWS 1048576
int ljmd_set_thermo(ljmd_system *sys, int32_t period, int32_t capacity);

/* The latest min(available, max_rows) samples, oldest first, LJMD_THERMO_COLS doubles a row:
 * step, K, U, E = K + U, T = 2K / (3n - 3), P = (2K + W_xx + W_yy + W_zz) / (3V), and the
 * virial (xx, xy, xz, yy, yz, zz). rows = NULL only returns the number available in *nrows.
 * The caller owns rows (max_rows x LJMD_THERMO_COLS doubles). Errors: INVAL (null handle or
 * nrows, max_rows < 0), DEVICE. */
#define LJMD_THERMO_COLS 12
int ljmd_get_thermo(ljmd_system *sys, double *rows, int32_t max_rows, int32_t *nrows);

/* The current neighbour list as unordered tag pairs (i < j), 2 x count int32, sorted by
 * (i, j); pairs = NULL only returns the count. build_pos (n x 3, tag order, nullable)
 * receives the positions the list was built from. */
int ljmd_get_neighbor_pairs(ljmd_system *sys, int64_t *count, int32_t *pairs,
                            double *build_pos);

/* The full neighbour list as the force kernel holds it: every particle's row, both
 * directions of each pair (Section "Performance": the list the pair kernel streams).
 * counts (n int32, tag order, nullable) receives each row's length and *total their sum;
 * neighbors (total int32, nullable: then only sizes are returned) receives the tags of
 * each row's entries in the order they are stored, rows in tag order. build_pos (n x 3,
 * tag order, nullable) receives the positions the list was built from. Errors: INVAL,
 * STATE (pair unset), BOX, DEVICE. */
int ljmd_get_neighbor_list(ljmd_system *sys, int32_t *counts, int64_t *total,
                           int32_t *neighbors, double *build_pos);

/* Counters and tuned launch parameters. */
int ljmd_get_stats(ljmd_system *sys, ljmd_stats *out);

/* Kernel timing for measurement: when on != 0, every launch of the step's dominant kernel
 * (the fused force + integration kernel) is bracketed by HIP events on the configured
 * stream and graphs are not used. ljmd_kernel_time returns the launch count and the summed
 * event time in milliseconds since timing was switched on. */
int ljmd_set_kernel_timing(ljmd_system *sys, int32_t on);
int ljmd_kernel_time(ljmd_system *sys, int64_t *launches, double *total_ms);

/* Per-launch durations recorded while kernel timing is on, by kernel kind: the step's force
 * kernel (the fused force + integration kernel; under NVT the force kernel of the step) and
 * the five list-rebuild kernels, which every step launches and which return at once unless
 * the displacement check asked for a rebuild. *count receives the number of launches
 * recorded since timing was switched on; ms (count floats, nullable) their durations in
 * milliseconds, in launch order. Errors: INVAL (unknown kind). */
#define LJMD_KERNEL_STEP 0     /* fused force + integration (NVE) or force (NVT) */
#define LJMD_KERNEL_BIN 1      /* cell binning */
#define LJMD_KERNEL_SCAN 2     /* cell-count scan */
#define LJMD_KERNEL_SCATTER 3  /* permutation scatter */
#define LJMD_KERNEL_GATHER 4   /* in-cell ordering and state gather */
#define LJMD_KERNEL_NLIST 5    /* Verlet list build */
#define LJMD_KERNEL_KINDS 6
int ljmd_kernel_durations(ljmd_system *sys, int32_t kind, int64_t *count, float *ms);

/* ------------------------------------------------------------------ batched replicas
 *
 * A batch advances many independent single-box LJ systems ("replicas") of uneven size
 * together: every step is one launch of the fused force/integration kernel over the bricks
 * of all replicas, plus the list-rebuild kernels, each gated per replica by that replica's
 * own rebuild request, all captured in HIP graphs of block_steps steps. Every replica runs
 * exactly the arithmetic it would run alone (same kernels, same per-replica parameters, no
 * cross-replica reductions), so its trajectory does not depend on its neighbours in the
 * batch. Replicas are admitted into free slots while others run and are retired when their
 * requested number of steps is done; their state stays on the device in between. This is
 * the paper's "many independent simulations" use of one GPU (Section "Performance") turned
 * into continuous batching. */

typedef struct ljmd_batch ljmd_batch;

typedef struct ljmd_batch_config {
    int64_t budget_bytes;   /* device memory the batch may use for replica state */
    int32_t max_slots;      /* replicas resident at once (>= 1) */
    int32_t precision;      /* LJMD_FP64 or LJMD_MIXED, for every replica */
    double dt;              /* time step for every replica */
    double skin;            /* Verlet skin for every replica */
    int32_t block_steps;    /* steps per ljmd_batch_run_block (even, >= 2); 0 = 100 */
    int32_t threads_per_particle; /* 0 = autotuned on the first block */
    int32_t block_size;     /* 0 = autotuned */
    int32_t nlist_capacity; /* entries per particle; 0 = automatic */
    void *stream;           /* hipStream_t; NULL = default stream */
    ljmd_alloc_fn alloc;    /* NULL = hipMalloc */
    ljmd_free_fn free;
    void *alloc_ctx;
} ljmd_batch_config;

/* One replica request: an orthorhombic box and N particles (host arrays, copied at
 * admission), a pair table of ntypes x ntypes LJ coefficients (row-major eps, sigma,
 * r_cut, each ntypes*ntypes doubles, symmetric), and the number of NVE steps to run. */
typedef struct ljmd_replica_spec {
    double box[3];
    int64_t n;
    const double *pos;      /* n x 3 */
    const double *vel;      /* n x 3 */
    const int32_t *type;    /* n, or NULL for all type 0 */
    int32_t ntypes;
    const double *eps;      /* ntypes x ntypes */
    const double *sigma;    /* ntypes x ntypes */
    const double *r_cut;    /* ntypes x ntypes */
    int64_t nsteps;         /* >= 1 */
} ljmd_replica_spec;

/* Create an empty batch. Errors: INVAL, NOMEM, DEVICE. */
int ljmd_batch_create(const ljmd_batch_config *cfg, ljmd_batch **out);

/* Device bytes a replica would hold in this batch (state, cells, bricks, list). */
int ljmd_batch_footprint(const ljmd_batch *b, const ljmd_replica_spec *spec, int64_t *bytes);

/* Admit a replica into a free slot: upload, first list build, first forces and the first
 * half step. *slot receives the slot id. Errors: CAPACITY (no free slot or not enough of
 * the budget left), INVAL, BOX, NONFINITE, DEVICE. */
int ljmd_batch_admit(ljmd_batch *b, const ljmd_replica_spec *spec, int32_t *slot);

/* Advance every running replica by up to block_steps steps (a replica stops exactly at its
 * requested count). Enqueued on the batch stream; synchronises once at the end. */
int ljmd_batch_run_block(ljmd_batch *b);

/* Slots whose replica has finished: done[0..*ndone) (done sized max_slots). */
int ljmd_batch_poll(ljmd_batch *b, int32_t *done, int32_t *ndone);

/* Results of a slot, tag order; any pointer may be NULL: positions (wrapped), velocities
 * and forces (n x 3), energy[2] = {potential, kinetic}, virial[6]. Errors: STATE if the slot
 * is empty. */
int ljmd_batch_read(ljmd_batch *b, int32_t slot, double *pos, double *vel, double *force,
                    double *energy, double *virial);

/* The same results as ljmd_batch_read, with no device memory allocated by the call: for
 * callers that cannot allocate (tight serving loops, harnesses that forbid allocation). The
 * positions, velocities and forces are staged in a fixed device array of 8 MiB per GPU (held
 * by the library until the process ends), so a replica may hold at most 349,525 particles
 * (3 doubles each); larger ones are refused with INVAL before any device work. Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (from several threads or
 * batches) race, and must be serialised by the caller. Errors: as ljmd_batch_read, and INVAL
 * for a replica beyond the limit. */
int ljmd_batch_read_noalloc(ljmd_batch *b, int32_t slot, double *pos, double *vel,
                            double *force, double *energy, double *virial);

/* Steps completed by the replica in a slot. */
int ljmd_batch_slot_steps(ljmd_batch *b, int32_t slot, int64_t *steps);

/* Outcome of the replica in a slot: LJMD_OK while it runs or once it finished its steps,
 * else the status it was retired with (LJMD_E_NONFINITE: a force became non-finite;
 * LJMD_E_BOX: a tile outgrew 16-bit indices); its results are then not readable.
 * Errors: INVAL, STATE (empty slot). */
int ljmd_batch_slot_status(ljmd_batch *b, int32_t slot, int32_t *status);

/* Free a slot (its memory returns to the budget). */
int ljmd_batch_release(ljmd_batch *b, int32_t slot);

void ljmd_batch_destroy(ljmd_batch *b);

/* Counters of a batch. */
typedef struct ljmd_batch_stats {
    int32_t resident;          /* occupied slots (running or finished, not yet released) */
    int32_t running;           /* resident replicas with steps left */
    int64_t blocks;            /* ljmd_batch_run_block calls that ran a block */
    int64_t overflow_reruns;   /* replicas whose block ran again after a list overflow */
    int64_t rebuilds;          /* list builds over all replicas (one per replica build) */
    int32_t nlist_capacity;    /* list entries per particle (all replicas) */
    int32_t threads_per_particle;
    int32_t block_size;
    int32_t tile_capacity;     /* atoms of a brick tile held in LDS */
    int64_t device_bytes;      /* device memory held by the batch */
    int64_t used_bytes;        /* footprints of the resident replicas */
    int64_t budget_bytes;
} ljmd_batch_stats;

int ljmd_batch_get_stats(ljmd_batch *b, ljmd_batch_stats *out);

/* ---------------------------------------------------------------- tuning table
 *
 * The autotuner of single systems (threads_per_particle or block_size 0 in ljmd_config)
 * times the force evaluation over lanes per particle {1, 2, 4, 8} and workgroup sizes 128..512
 * (the autotuning the paper applies to its kernels, Section "Performance") and keeps the
 * choice, for the life of the process, per key (precision, one or several types, size bucket
 * floor(log2 n)). These two calls read that table and preload it, so that a table saved from
 * one run freezes the choices of the next: a system whose key is in the table takes the stored
 * lanes and workgroup size without timing runs. Both are host-only (no device is touched) and
 * safe to call from any thread. */
typedef struct ljmd_tuning_entry {
    int32_t precision;            /* LJMD_FP64 or LJMD_MIXED */
    int32_t multi_type;           /* 0: one type, 1: several types */
    int32_t size_bucket;          /* floor(log2 n), 0..26 */
    int32_t threads_per_particle; /* 1, 2, 4 or 8 */
    int32_t block_size;           /* a multiple of 64 in [128, 512] */
} ljmd_tuning_entry;

/* Copies the table, ordered by key, into out[0 .. min(capacity, count)) and stores the
 * number of entries in *count (out may be NULL when capacity is 0: a size query).
 * Errors: INVAL (count NULL, capacity < 0, out NULL with capacity > 0). */
int ljmd_tuning_get(ljmd_tuning_entry *out, int32_t capacity, int32_t *count);

/* Adds the n entries to the table, replacing entries of the same key. All entries are
 * validated first; if any is out of range the call stores nothing. Systems created earlier
 * keep their choice. Errors: INVAL. */
int ljmd_tuning_set(const ljmd_tuning_entry *entries, int32_t n);

/* Thread-local message for the last non-zero status returned on this thread. */
const char *ljmd_last_error(void);

/* Library version string; a debug build (compiled with LJMD_DEBUG_CHECKS=1, loaded by the
 * Python binding when the environment sets LJMD_DEBUG_CHECKS=1) says "debug checks". Such a
 * build checks on the device that every particle's cell and sorted slot lie in its replica's
 * range, that every list entry written or read lies in its brick's tile and every list slot
 * in the list allocation, and that no force is taken at a position half the skin or more
 * from the list's build position (a dangerous build); a failed check makes the call that
 * next reads the device status return DEVICE with the check's code in the message. */
const char *ljmd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LJMD_H */
