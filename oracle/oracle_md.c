/*
 * oracle_md.c -- plain, slow FP64 CPU reference of the Lennard-Jones MD hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or calls this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header, table or helper with the GPU path.
 *
 * What it computes (the paper names the method -- a cell-list neighbour list feeding a
 * truncated Lennard-Jones pair force, driven by an NVE integrator, Section "Capabilities",
 * Molecular dynamics listing; Section "Performance" -- and fixes no formulas, so the
 * textbook definitions are written out here):
 *
 *   state       orthorhombic box L, positions wrapped into [0, L) with integer image
 *               counters, velocities, masses, types, a per-type-pair (eps, sigma, r_cut)
 *               table, a Verlet skin r_s and a time step dt.
 *   min image   d = x_j - x_i per axis; if d >= L/2 then d -= L, else if d < -L/2 then
 *               d += L.  Valid because every list radius r_L = r_cut + r_s is <= L/2.
 *   distance    r2 = (dx*dx + dy*dy) + dz*dz, in that order, no fused multiply-add
 *               (this file must be compiled with -ffp-contract=off).
 *   pair        U_LJ(r) = 4 eps ((s/r)^12 - (s/r)^6); u(r) = U_LJ(r) - U_LJ(r_cut) when
 *               r2 < r_cut^2, else 0 (truncated and shifted energy).  The force is not
 *               shifted: F on i from j = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2 * (x_i - x_j).
 *   list        P = { (i, j) : i < j, r2 < (r_cut_ab + r_s)^2 }, the squared threshold
 *               rounded once in FP64 from (r_cut + r_s); built from a cell list with
 *               n_cell = floor(L / max r_L) cells per axis and a 27-cell stencil reduced to
 *               its distinct cells when n_cell < 3.
 *   sums        F_i = sum over pairs with r2 < r_cut^2; U = sum u; W_ab = sum d_a F_b with
 *               d = x_i - x_j; per-particle energy and virial take half of each pair.
 *   step        velocity Verlet (NVE): v += dt/(2m) F; x += dt v, wrap and count images;
 *               rebuild the list when max |x - x_build|^2 (min image) >= (r_s/2)^2;
 *               recompute F; v += dt/(2m) F.
 *   other pair  forms on the same skeleton (Section "Capabilities" lists Gaussian, Mie, WCA
 *   potentials  and Yukawa among its pair potentials), each truncated at r_cut with the
 *               energy shifted to 0 there and the force not shifted; f is the factor with
 *               F on i = f (x_i - x_j), f = -(du/dr) / r:
 *                 Mie(eps, sigma, n, m): u = C eps ((s/r)^n - (s/r)^m),
 *                   C = (n / (n - m)) (n / m)^(m / (n - m)); f = C eps (n (s/r)^n - m (s/r)^m) / r^2
 *                 Gaussian(eps, sigma): u = eps exp(-r^2 / (2 s^2)); f = eps / s^2 exp(-r^2 / (2 s^2))
 *                 Yukawa(eps, kappa): u = eps exp(-kappa r) / r; f = eps exp(-kappa r) (1 + kappa r) / r^3
 *               WCA is the LJ form cut at 2^(1/6) sigma (the shift then is +eps).
 *   shifted     (an option per system, for tighter energy conservation): the force is
 *   force       shifted as well, so that both vanish at r_cut. With F(r) = f(r) r the
 *               pair force magnitude (positive when repulsive) and F_c = F(r_cut):
 *                 u_sf(r) = u(r) - u(r_cut) + (r - r_cut) F_c,  f_sf(r) = f(r) - F_c / r,
 *               so that F_sf = F - F_c = -du_sf/dr, and u_sf(r_cut) = F_sf(r_cut) = 0.
 *   NVT         (the integrator of the paper's MD listing, built on the Martyna-Tobias-
 *               Klein method, Section "Capabilities"): one Nose-Hoover thermostat
 *               variable xi with "position" eta and mass Q = N_f kT tau^2, N_f = 3N - 3.
 *               The equations of motion dx/dt = v, dv/dt = F/m - xi v,
 *               dxi/dt = (2K - N_f kT)/Q, deta/dt = xi are split symmetrically (the
 *               time-reversible factorisation of Martyna, Tuckerman, Tobias and Klein,
 *               chain length one): each step is a thermostat half step, the velocity-
 *               Verlet step above, and another thermostat half step. A thermostat half
 *               step of length dt/2 is: xi += (dt/4) G(K); eta += (dt/2) xi; every v is
 *               scaled by s = exp(-(dt/2) xi), so K becomes s^2 K; xi += (dt/4) G(K), with
 *               G(K) = (2K - N_f kT) / Q and K = sum m v^2 / 2. The conserved quantity is
 *               K + U + Q xi^2 / 2 + N_f kT eta. tau = +infinity is zero coupling: xi and
 *               eta stay 0, s = 1, and the step is the NVE step.
 *
 * Every function below is a direct statement of one of these definitions, with no
 * blocking, fusion or reordering beyond what the definition states.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EBOX -4
#define ORC_ENONFINITE -5
#define ORC_ESTATE -6

typedef struct {
    int64_t n;
    int32_t ntypes;
    double L[3];
    double dt, skin;
    double *x, *v, *f, *m;   /* n*3, n*3, n*3, n */
    int32_t *type, *img;     /* n, n*3 */
    double *xb;              /* positions at the last list build, n*3 */
    double *eps, *sig, *rc;  /* ntypes*ntypes */
    int32_t *is_set;         /* ntypes*ntypes */
    int32_t *style;          /* ntypes*ntypes: ORC_LJ, ORC_MIE, ORC_GAUSS, ORC_YUKAWA */
    double *par;             /* ntypes*ntypes*4 form parameters (LJ: eps, sigma) */
    /* neighbour list: half list of index pairs (i < j) */
    int64_t npairs, cap;
    int32_t *pi, *pj;
    int list_valid, force_valid;
    int64_t builds, steps;
    /* results of the last force evaluation */
    double U, W[6];
    double *u_i, *w_i;       /* n, n*6 */
    /* NVT thermostat (nvt = 0: NVE) */
    int nvt;
    double kT, invQ, xi, eta;
    int shift_force;         /* 1: shifted force (see the header), 0: shifted energy only */
} orc_sys;

/* ---------------------------------------------------------------- basic definitions */

static double min_image(double d, double L)
{
    double h = 0.5 * L;
    if (d >= h) return d - L;
    if (d < -h) return d + L;
    return d;
}

/* squared min-image distance from i to j, canonical operation order */
static double dist2(const orc_sys *s, int64_t i, int64_t j, double d[3])
{
    for (int a = 0; a < 3; ++a) d[a] = min_image(s->x[3 * j + a] - s->x[3 * i + a], s->L[a]);
    double xx = d[0] * d[0];
    double yy = d[1] * d[1];
    double zz = d[2] * d[2];
    double t = xx + yy;
    return t + zz;
}

static double lj_energy(double eps, double sig, double r2)
{
    double sr2 = (sig * sig) / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    return 4.0 * eps * (sr12 - sr6);
}

/* magnitude factor f with F_on_i = f * (x_i - x_j) */
static double lj_force_factor(double eps, double sig, double r2)
{
    double sr2 = (sig * sig) / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    return 24.0 * eps * (2.0 * sr12 - sr6) / r2;
}

#define ORC_LJ 0
#define ORC_MIE 1
#define ORC_GAUSS 2
#define ORC_YUKAWA 3

/* energy of the other forms (see the header), before truncation and shift */
static double form_energy(int style, const double *p, double r2)
{
    if (style == ORC_MIE) {
        double n = p[2], m = p[3];
        double c = (n / (n - m)) * pow(n / m, m / (n - m));
        double sr2 = (p[1] * p[1]) / r2;
        return c * p[0] * (pow(sr2, 0.5 * n) - pow(sr2, 0.5 * m));
    }
    if (style == ORC_GAUSS) return p[0] * exp(-r2 / (2.0 * p[1] * p[1]));
    /* Yukawa */
    double r = sqrt(r2);
    return p[0] * exp(-p[1] * r) / r;
}

/* force factor f of the other forms: F on i = f (x_i - x_j) */
static double form_force_factor(int style, const double *p, double r2)
{
    if (style == ORC_MIE) {
        double n = p[2], m = p[3];
        double c = (n / (n - m)) * pow(n / m, m / (n - m));
        double sr2 = (p[1] * p[1]) / r2;
        return c * p[0] * (n * pow(sr2, 0.5 * n) - m * pow(sr2, 0.5 * m)) / r2;
    }
    if (style == ORC_GAUSS) return p[0] / (p[1] * p[1]) * exp(-r2 / (2.0 * p[1] * p[1]));
    double r = sqrt(r2);
    return p[0] * exp(-p[1] * r) * (1.0 + p[1] * r) / (r2 * r);
}

static int pair_index(const orc_sys *s, int32_t a, int32_t b) { return a * s->ntypes + b; }

static double list_threshold2(const orc_sys *s, int32_t a, int32_t b)
{
    int k = pair_index(s, a, b);
    if (s->rc[k] <= 0.0) return 0.0;          /* disabled pair: never listed */
    double rl = s->rc[k] + s->skin;
    return rl * rl;
}

static double max_list_radius(const orc_sys *s)
{
    double r = 0.0;
    for (int k = 0; k < s->ntypes * s->ntypes; ++k)
        if (s->rc[k] > 0.0 && s->rc[k] + s->skin > r) r = s->rc[k] + s->skin;
    return r;
}

static void wrap_coordinate(double *x, int32_t *img, double L)
{
    if (*x >= L) {
        *x -= L;
        *img += 1;
    } else if (*x < 0.0) {
        *x += L;
        *img -= 1;
        if (*x >= L) { /* x + L rounded up to L: the particle sits at 0 in its old image */
            *x = 0.0;
            *img += 1;
        }
    }
}

/* ---------------------------------------------------------------- create / destroy */

void oracle_destroy(orc_sys *s)
{
    if (!s) return;
    free(s->x); free(s->v); free(s->f); free(s->m); free(s->type); free(s->img);
    free(s->xb); free(s->eps); free(s->sig); free(s->rc); free(s->is_set);
    free(s->style); free(s->par);
    free(s->pi); free(s->pj); free(s->u_i); free(s->w_i);
    free(s);
}

orc_sys *oracle_create(int64_t n, const double *box, const double *pos, const double *vel,
                       const int32_t *type, const double *mass, int32_t ntypes, double dt,
                       double skin)
{
    if (n < 1 || !box || !pos || !vel || !type || ntypes < 1 || !(dt > 0.0) || !(skin >= 0.0))
        return NULL;
    for (int a = 0; a < 3; ++a)
        if (!(box[a] > 0.0) || !isfinite(box[a])) return NULL;
    orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
    if (!s) return NULL;
    s->n = n;
    s->ntypes = ntypes;
    for (int a = 0; a < 3; ++a) s->L[a] = box[a];
    s->dt = dt;
    s->skin = skin;
    size_t nt2 = (size_t)ntypes * (size_t)ntypes;
    s->x = (double *)malloc(sizeof(double) * 3 * n);
    s->v = (double *)malloc(sizeof(double) * 3 * n);
    s->f = (double *)calloc(3 * n, sizeof(double));
    s->m = (double *)malloc(sizeof(double) * n);
    s->type = (int32_t *)malloc(sizeof(int32_t) * n);
    s->img = (int32_t *)calloc(3 * n, sizeof(int32_t));
    s->xb = (double *)malloc(sizeof(double) * 3 * n);
    s->eps = (double *)calloc(nt2, sizeof(double));
    s->sig = (double *)calloc(nt2, sizeof(double));
    s->rc = (double *)calloc(nt2, sizeof(double));
    s->is_set = (int32_t *)calloc(nt2, sizeof(int32_t));
    s->style = (int32_t *)calloc(nt2, sizeof(int32_t));
    s->par = (double *)calloc(4 * nt2, sizeof(double));
    s->u_i = (double *)calloc(n, sizeof(double));
    s->w_i = (double *)calloc(6 * n, sizeof(double));
    if (!s->x || !s->v || !s->f || !s->m || !s->type || !s->img || !s->xb || !s->eps ||
        !s->sig || !s->rc || !s->is_set || !s->style || !s->par || !s->u_i || !s->w_i) {
        oracle_destroy(s);
        return NULL;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] < 0 || type[i] >= ntypes) { oracle_destroy(s); return NULL; }
        s->type[i] = type[i];
        s->m[i] = mass ? mass[i] : 1.0;
        if (!(s->m[i] > 0.0)) { oracle_destroy(s); return NULL; }
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * i + a], L = s->L[a];
            if (!isfinite(x) || !isfinite(vel[3 * i + a])) { oracle_destroy(s); return NULL; }
            /* bring into [0, L): k = floor(x / L) whole boxes, then fix rounding */
            double k = floor(x / L);
            double kl = k * L;
            x = x - kl;
            int32_t im = (int32_t)k;
            if (x >= L) { x -= L; im += 1; }
            if (x < 0.0) { x += L; im -= 1; if (x >= L) { x = 0.0; im += 1; } }
            s->x[3 * i + a] = x;
            s->img[3 * i + a] = im;
            s->v[3 * i + a] = vel[3 * i + a];
        }
    }
    return s;
}

int oracle_set_pair(orc_sys *s, int32_t a, int32_t b, double eps, double sig, double rc)
{
    if (!s || a < 0 || b < 0 || a >= s->ntypes || b >= s->ntypes) return ORC_EINVAL;
    if (!(sig > 0.0) || !(rc >= 0.0) || !isfinite(eps) || !isfinite(rc)) return ORC_EINVAL;
    int k1 = pair_index(s, a, b), k2 = pair_index(s, b, a);
    s->eps[k1] = s->eps[k2] = eps;
    s->sig[k1] = s->sig[k2] = sig;
    s->rc[k1] = s->rc[k2] = rc;
    s->is_set[k1] = s->is_set[k2] = 1;
    s->style[k1] = s->style[k2] = ORC_LJ;
    s->list_valid = 0;
    s->force_valid = 0;
    return ORC_OK;
}

/* a pair of one of the other forms: params holds (eps, sigma, n, m) for Mie, (eps, sigma)
 * for Gaussian, (eps, kappa) for Yukawa */
int oracle_set_pair_style(orc_sys *s, int32_t a, int32_t b, int32_t style, const double *params,
                          double rc)
{
    if (!s || !params || a < 0 || b < 0 || a >= s->ntypes || b >= s->ntypes) return ORC_EINVAL;
    if (style == ORC_LJ) return oracle_set_pair(s, a, b, params[0], params[1], rc);
    if (style != ORC_MIE && style != ORC_GAUSS && style != ORC_YUKAWA) return ORC_EINVAL;
    if (!(rc >= 0.0) || !isfinite(rc) || !isfinite(params[0])) return ORC_EINVAL;
    if (style == ORC_MIE && !(params[1] > 0.0 && params[3] > 0.0 && params[2] > params[3]))
        return ORC_EINVAL;
    if (style == ORC_GAUSS && !(params[1] > 0.0)) return ORC_EINVAL;
    if (style == ORC_YUKAWA && !(params[1] >= 0.0)) return ORC_EINVAL;
    int k1 = pair_index(s, a, b), k2 = pair_index(s, b, a);
    s->rc[k1] = s->rc[k2] = rc;
    s->is_set[k1] = s->is_set[k2] = 1;
    s->style[k1] = s->style[k2] = style;
    for (int c = 0; c < 4; ++c) s->par[4 * k1 + c] = s->par[4 * k2 + c] = params[c];
    s->list_valid = 0;
    s->force_valid = 0;
    return ORC_OK;
}

/* mode 0: energy shifted to 0 at r_cut, force not shifted; mode 1: shifted force */
int oracle_set_shift_mode(orc_sys *s, int32_t mode)
{
    if (!s || (mode != 0 && mode != 1)) return ORC_EINVAL;
    s->shift_force = mode;
    s->force_valid = 0;
    return ORC_OK;
}

static int check_ready(const orc_sys *s)
{
    for (int k = 0; k < s->ntypes * s->ntypes; ++k)
        if (!s->is_set[k]) return ORC_ESTATE;
    double rl = max_list_radius(s);
    for (int a = 0; a < 3; ++a)
        if (rl > 0.5 * s->L[a]) return ORC_EBOX;
    return ORC_OK;
}

/* ---------------------------------------------------------------- neighbour list */

static int push_pair(orc_sys *s, int32_t i, int32_t j)
{
    if (s->npairs == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 1024;
        int32_t *a = (int32_t *)realloc(s->pi, sizeof(int32_t) * nc);
        if (!a) return ORC_ENOMEM;
        s->pi = a;
        int32_t *b = (int32_t *)realloc(s->pj, sizeof(int32_t) * nc);
        if (!b) return ORC_ENOMEM;
        s->pj = b;
        s->cap = nc;
    }
    s->pi[s->npairs] = i;
    s->pj[s->npairs] = j;
    s->npairs += 1;
    return ORC_OK;
}

/* Cell list: cell c = (cx, cy, cz), cx = floor(x / w) clamped to n_cell - 1, w = L / n_cell.
 * Members of each cell are kept in a plain array of index lists (head/next chaining). */
static int build_list(orc_sys *s)
{
    double rl = max_list_radius(s);
    s->npairs = 0;
    memcpy(s->xb, s->x, sizeof(double) * 3 * s->n);
    s->builds += 1;
    s->list_valid = 1;
    if (rl <= 0.0) return ORC_OK; /* every pair disabled */
    int64_t nc[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int64_t)floor(s->L[a] / rl);
        if (nc[a] < 1) nc[a] = 1;
        w[a] = s->L[a] / (double)nc[a];
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * s->n);
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * s->n);
    if (!head || !next || !cell_of) { free(head); free(next); free(cell_of); return ORC_ENOMEM; }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    /* insert in descending index order so that each chain lists ascending indices */
    for (int64_t i = s->n - 1; i >= 0; --i) {
        int64_t cc[3];
        for (int a = 0; a < 3; ++a) {
            cc[a] = (int64_t)floor(s->x[3 * i + a] / w[a]);
            if (cc[a] > nc[a] - 1) cc[a] = nc[a] - 1;
            if (cc[a] < 0) cc[a] = 0;
        }
        int64_t c = (cc[0] * nc[1] + cc[1]) * nc[2] + cc[2];
        cell_of[i] = c;
        next[i] = head[c];
        head[c] = i;
    }
    int rc = ORC_OK;
    for (int64_t i = 0; i < s->n && rc == ORC_OK; ++i) {
        int64_t c = cell_of[i];
        int64_t cz = c % nc[2], cy = (c / nc[2]) % nc[1], cx = c / (nc[1] * nc[2]);
        /* the distinct cells of the 27-cell stencil around c */
        int64_t stencil[27];
        int ns = 0;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t ex = ((cx + dx) % nc[0] + nc[0]) % nc[0];
                    int64_t ey = ((cy + dy) % nc[1] + nc[1]) % nc[1];
                    int64_t ez = ((cz + dz) % nc[2] + nc[2]) % nc[2];
                    int64_t e = (ex * nc[1] + ey) * nc[2] + ez;
                    int seen = 0;
                    for (int t = 0; t < ns; ++t)
                        if (stencil[t] == e) seen = 1;
                    if (!seen) stencil[ns++] = e;
                }
        for (int t = 0; t < ns && rc == ORC_OK; ++t) {
            for (int64_t j = head[stencil[t]]; j >= 0; j = next[j]) {
                if (j <= i) continue;
                double d[3];
                double r2 = dist2(s, i, j, d);
                if (r2 < list_threshold2(s, s->type[i], s->type[j])) {
                    rc = push_pair(s, (int32_t)i, (int32_t)j);
                    if (rc != ORC_OK) break;
                }
            }
        }
    }
    free(head); free(next); free(cell_of);
    return rc;
}

/* ---------------------------------------------------------------- forces */

static int compute_forces(orc_sys *s)
{
    int rc = check_ready(s);
    if (rc != ORC_OK) return rc;
    if (!s->list_valid) {
        rc = build_list(s);
        if (rc != ORC_OK) return rc;
    }
    memset(s->f, 0, sizeof(double) * 3 * s->n);
    memset(s->u_i, 0, sizeof(double) * s->n);
    memset(s->w_i, 0, sizeof(double) * 6 * s->n);
    s->U = 0.0;
    for (int k = 0; k < 6; ++k) s->W[k] = 0.0;
    for (int64_t p = 0; p < s->npairs; ++p) {
        int64_t i = s->pi[p], j = s->pj[p];
        double d[3];
        double r2 = dist2(s, i, j, d);         /* d = x_j - x_i */
        int k = pair_index(s, s->type[i], s->type[j]);
        double rcut2 = s->rc[k] * s->rc[k];
        if (!(r2 < rcut2)) continue;
        double ff, u, ffc;
        if (s->style[k] == ORC_LJ) {
            ff = lj_force_factor(s->eps[k], s->sig[k], r2);
            u = lj_energy(s->eps[k], s->sig[k], r2) -
                lj_energy(s->eps[k], s->sig[k], rcut2);
            ffc = lj_force_factor(s->eps[k], s->sig[k], rcut2);
        } else {
            const double *p = s->par + 4 * k;
            ff = form_force_factor(s->style[k], p, r2);
            u = form_energy(s->style[k], p, r2) - form_energy(s->style[k], p, rcut2);
            ffc = form_force_factor(s->style[k], p, rcut2);
        }
        if (s->shift_force) {
            /* F_c = f(r_cut) r_cut; u_sf = u + (r - r_cut) F_c; f_sf = f - F_c / r */
            double r = sqrt(r2);
            double fc = ffc * s->rc[k];
            u = u + (r - s->rc[k]) * fc;
            ff = ff - fc / r;
        }
        double rij[3] = {-d[0], -d[1], -d[2]};  /* x_i - x_j */
        for (int a = 0; a < 3; ++a) {
            s->f[3 * i + a] += ff * rij[a];
            s->f[3 * j + a] -= ff * rij[a];
        }
        /* W_ab = r_a F_b with F = ff * r */
        double wp[6] = {rij[0] * ff * rij[0], rij[0] * ff * rij[1], rij[0] * ff * rij[2],
                        rij[1] * ff * rij[1], rij[1] * ff * rij[2], rij[2] * ff * rij[2]};
        s->U += u;
        s->u_i[i] += 0.5 * u;
        s->u_i[j] += 0.5 * u;
        for (int c = 0; c < 6; ++c) {
            s->W[c] += wp[c];
            s->w_i[6 * i + c] += 0.5 * wp[c];
            s->w_i[6 * j + c] += 0.5 * wp[c];
        }
    }
    for (int64_t q = 0; q < 3 * s->n; ++q)
        if (!isfinite(s->f[q])) return ORC_ENONFINITE;
    s->force_valid = 1;
    return ORC_OK;
}

int oracle_compute(orc_sys *s)
{
    if (!s) return ORC_EINVAL;
    if (s->force_valid) return ORC_OK;
    return compute_forces(s);
}

/* force a fresh list build at the current positions, then forces */
int oracle_rebuild(orc_sys *s)
{
    if (!s) return ORC_EINVAL;
    int rc = check_ready(s);
    if (rc != ORC_OK) return rc;
    rc = build_list(s);
    if (rc != ORC_OK) return rc;
    return compute_forces(s);
}

/* ---------------------------------------------------------------- integration */

static double kinetic_energy(const orc_sys *s)
{
    double k = 0.0;
    for (int64_t i = 0; i < s->n; ++i)
        for (int a = 0; a < 3; ++a) k += 0.5 * s->m[i] * s->v[3 * i + a] * s->v[3 * i + a];
    return k;
}

/* degrees of freedom of the thermostatted motion: 3N - 3 (total momentum is conserved) */
static double dof(const orc_sys *s) { return 3.0 * (double)s->n - 3.0; }

/* one thermostat half step of length dt/2 (see the header) */
static void thermostat_half(orc_sys *s)
{
    double g = dof(s) * s->kT;
    double K = kinetic_energy(s);
    s->xi += 0.25 * s->dt * (2.0 * K - g) * s->invQ;
    s->eta += 0.5 * s->dt * s->xi;
    double sc = exp(-0.5 * s->dt * s->xi);
    for (int64_t q = 0; q < 3 * s->n; ++q) s->v[q] *= sc;
    K = sc * sc * K;
    s->xi += 0.25 * s->dt * (2.0 * K - g) * s->invQ;
}

/* NVT at temperature kT with thermostat time constant tau (Q = N_f kT tau^2); tau may be
 * +infinity (zero coupling). The thermostat variables start at 0. */
int oracle_set_nvt(orc_sys *s, double kT, double tau)
{
    if (!s || s->n < 2 || !(kT > 0.0) || !isfinite(kT) || !(tau > 0.0)) return ORC_EINVAL;
    s->nvt = 1;
    s->kT = kT;
    s->invQ = isinf(tau) ? 0.0 : 1.0 / (dof(s) * kT * tau * tau);
    s->xi = 0.0;
    s->eta = 0.0;
    return ORC_OK;
}

int oracle_set_nve(orc_sys *s)
{
    if (!s) return ORC_EINVAL;
    s->nvt = 0;
    s->xi = 0.0;
    s->eta = 0.0;
    return ORC_OK;
}

/* xi, eta and the thermostat's share of the conserved quantity, Q xi^2 / 2 + N_f kT eta
 * (0 for NVE or zero coupling); any pointer may be NULL */
int oracle_get_thermostat(const orc_sys *s, double *xi, double *eta, double *energy)
{
    if (!s) return ORC_EINVAL;
    if (xi) *xi = s->xi;
    if (eta) *eta = s->eta;
    if (energy) {
        double e = 0.0;
        if (s->nvt && s->invQ > 0.0)
            e = 0.5 * s->xi * s->xi / s->invQ + dof(s) * s->kT * s->eta;
        *energy = e;
    }
    return ORC_OK;
}

int oracle_set_thermostat(orc_sys *s, double xi, double eta)
{
    if (!s || !isfinite(xi) || !isfinite(eta)) return ORC_EINVAL;
    s->xi = xi;
    s->eta = eta;
    return ORC_OK;
}

/* velocities v -> -v (for reversibility checks) */
int oracle_negate_velocities(orc_sys *s)
{
    if (!s) return ORC_EINVAL;
    for (int64_t q = 0; q < 3 * s->n; ++q) s->v[q] = -s->v[q];
    return ORC_OK;
}

static int needs_rebuild(const orc_sys *s)
{
    double lim = 0.5 * s->skin;
    double lim2 = lim * lim;
    for (int64_t i = 0; i < s->n; ++i) {
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = min_image(s->x[3 * i + a] - s->xb[3 * i + a], s->L[a]);
        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (r2 >= lim2) return 1;
    }
    return 0;
}

int oracle_step(orc_sys *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return ORC_EINVAL;
    int rc = oracle_compute(s);
    if (rc != ORC_OK) return rc;
    double h = 0.5 * s->dt;
    for (int64_t t = 0; t < nsteps; ++t) {
        if (s->nvt) thermostat_half(s);
        for (int64_t i = 0; i < s->n; ++i)
            for (int a = 0; a < 3; ++a) s->v[3 * i + a] += h * s->f[3 * i + a] / s->m[i];
        for (int64_t i = 0; i < s->n; ++i)
            for (int a = 0; a < 3; ++a) {
                s->x[3 * i + a] += s->dt * s->v[3 * i + a];
                wrap_coordinate(&s->x[3 * i + a], &s->img[3 * i + a], s->L[a]);
            }
        if (needs_rebuild(s)) s->list_valid = 0;
        s->force_valid = 0;
        rc = compute_forces(s);
        if (rc != ORC_OK) return rc;
        for (int64_t i = 0; i < s->n; ++i)
            for (int a = 0; a < 3; ++a) s->v[3 * i + a] += h * s->f[3 * i + a] / s->m[i];
        if (s->nvt) thermostat_half(s);
        s->steps += 1;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- readers */

int oracle_get_forces(orc_sys *s, double *out)
{
    int rc = oracle_compute(s);
    if (rc != ORC_OK) return rc;
    memcpy(out, s->f, sizeof(double) * 3 * s->n);
    return ORC_OK;
}

int oracle_get_energy(orc_sys *s, double *potential, double *kinetic)
{
    int rc = oracle_compute(s);
    if (rc != ORC_OK) return rc;
    if (potential) *potential = s->U;
    if (kinetic) *kinetic = kinetic_energy(s);
    return ORC_OK;
}

int oracle_get_virial(orc_sys *s, double *out6)
{
    int rc = oracle_compute(s);
    if (rc != ORC_OK) return rc;
    for (int c = 0; c < 6; ++c) out6[c] = s->W[c];
    return ORC_OK;
}

int oracle_get_per_particle(orc_sys *s, double *u, double *w)
{
    int rc = oracle_compute(s);
    if (rc != ORC_OK) return rc;
    if (u) memcpy(u, s->u_i, sizeof(double) * s->n);
    if (w) memcpy(w, s->w_i, sizeof(double) * 6 * s->n);
    return ORC_OK;
}

int oracle_get_state(const orc_sys *s, double *pos, double *vel, int32_t *img, int64_t *step)
{
    if (!s) return ORC_EINVAL;
    if (pos) memcpy(pos, s->x, sizeof(double) * 3 * s->n);
    if (vel) memcpy(vel, s->v, sizeof(double) * 3 * s->n);
    if (img) memcpy(img, s->img, sizeof(int32_t) * 3 * s->n);
    if (step) *step = s->steps;
    return ORC_OK;
}

/* the current list as (i < j) index pairs; pairs == NULL only reports the count */
int oracle_get_pairs(orc_sys *s, int64_t *count, int32_t *pairs, double *build_pos)
{
    if (!s || !count) return ORC_EINVAL;
    int rc = check_ready(s);
    if (rc != ORC_OK) return rc;
    if (!s->list_valid) {
        rc = build_list(s);
        if (rc != ORC_OK) return rc;
        s->force_valid = 0;
    }
    *count = s->npairs;
    if (pairs)
        for (int64_t p = 0; p < s->npairs; ++p) {
            pairs[2 * p] = s->pi[p];
            pairs[2 * p + 1] = s->pj[p];
        }
    if (build_pos) memcpy(build_pos, s->xb, sizeof(double) * 3 * s->n);
    return ORC_OK;
}

int oracle_get_counters(const orc_sys *s, int64_t *steps, int64_t *builds)
{
    if (!s) return ORC_EINVAL;
    if (steps) *steps = s->steps;
    if (builds) *builds = s->builds;
    return ORC_OK;
}
