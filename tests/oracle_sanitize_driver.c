/* Drives the CPU oracle through every entry point on small random systems, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py): LJ and the other
 * pair forms, both shift modes, NVE and NVT steps with rebuilds, every getter, the error
 * paths, and destruction. Exits 0 when every call behaves; the sanitizers abort on any
 * invalid access or undefined operation. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_sys orc_sys;
orc_sys *oracle_create(int64_t n, const double *box, const double *pos, const double *vel,
                       const int32_t *type, const double *mass, int32_t ntypes, double dt,
                       double skin);
void oracle_destroy(orc_sys *s);
int oracle_set_pair(orc_sys *s, int32_t a, int32_t b, double eps, double sig, double rc);
int oracle_set_pair_style(orc_sys *s, int32_t a, int32_t b, int32_t style, const double *params,
                          double rc);
int oracle_set_shift_mode(orc_sys *s, int32_t mode);
int oracle_compute(orc_sys *s);
int oracle_rebuild(orc_sys *s);
int oracle_set_nvt(orc_sys *s, double kT, double tau);
int oracle_set_nve(orc_sys *s);
int oracle_get_thermostat(const orc_sys *s, double *xi, double *eta, double *energy);
int oracle_set_thermostat(orc_sys *s, double xi, double eta);
int oracle_negate_velocities(orc_sys *s);
int oracle_step(orc_sys *s, int64_t nsteps);
int oracle_get_forces(orc_sys *s, double *out);
int oracle_get_energy(orc_sys *s, double *potential, double *kinetic);
int oracle_get_virial(orc_sys *s, double *out6);
int oracle_get_per_particle(orc_sys *s, double *u, double *w);
int oracle_get_state(const orc_sys *s, double *pos, double *vel, int32_t *img, int64_t *step);
int oracle_get_pairs(orc_sys *s, int64_t *count, int32_t *pairs, double *build_pos);
int oracle_get_counters(const orc_sys *s, int64_t *steps, int64_t *builds);

static uint64_t rng = 88172645463325252ull;
static double uniform(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(x)                                                              \
    do {                                                                      \
        if ((x) != 0) {                                                       \
            fprintf(stderr, "failed: %s (line %d)\n", #x, __LINE__);          \
            return 1;                                                         \
        }                                                                     \
    } while (0)

/* one system of n particles on a jittered lattice in a cubic box of side L */
static int run(int64_t n, double L, int ntypes, int style, int shift, int nvt)
{
    double box[3] = {L, L, L};
    double *pos = malloc(sizeof(double) * 3 * n), *vel = malloc(sizeof(double) * 3 * n);
    int32_t *type = malloc(sizeof(int32_t) * n);
    int side = (int)ceil(cbrt((double)n));
    double a = L / side;
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix = i / (side * side), iy = (i / side) % side, iz = i % side;
        pos[3 * i] = (ix + 0.5 + 0.1 * (uniform() - 0.5)) * a;
        pos[3 * i + 1] = (iy + 0.5 + 0.1 * (uniform() - 0.5)) * a;
        pos[3 * i + 2] = (iz + 0.5 + 0.1 * (uniform() - 0.5)) * a;
        for (int c = 0; c < 3; ++c) vel[3 * i + c] = uniform() - 0.5;
        type[i] = (int32_t)(i % ntypes);
    }
    orc_sys *s = oracle_create(n, box, pos, vel, type, NULL, ntypes, 0.005, 0.4);
    if (!s) return 1;
    for (int p = 0; p < ntypes; ++p)
        for (int q = p; q < ntypes; ++q) {
            if (style == 0) {
                CHECK(oracle_set_pair(s, p, q, 1.0, 1.0, 2.5));
            } else {
                double par[4] = {1.0, 1.0, 14.0, 7.0};
                if (style == 3) par[1] = 1.1; /* Yukawa: (eps, kappa) */
                CHECK(oracle_set_pair_style(s, p, q, style, par, 2.5));
            }
        }
    CHECK(oracle_set_shift_mode(s, shift));
    if (nvt) CHECK(oracle_set_nvt(s, 1.2, 1.0));
    CHECK(oracle_compute(s));
    CHECK(oracle_step(s, 40));
    CHECK(oracle_rebuild(s));
    double *f = malloc(sizeof(double) * 3 * n), *u = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * 6 * n), U, K, W[6], xi, eta, e;
    int32_t *img = malloc(sizeof(int32_t) * 3 * n);
    int64_t step, steps, builds, count;
    CHECK(oracle_get_forces(s, f));
    CHECK(oracle_get_energy(s, &U, &K));
    CHECK(oracle_get_virial(s, W));
    CHECK(oracle_get_per_particle(s, u, w));
    CHECK(oracle_get_state(s, pos, vel, img, &step));
    CHECK(oracle_get_counters(s, &steps, &builds));
    CHECK(oracle_get_pairs(s, &count, NULL, NULL));
    int32_t *pairs = malloc(sizeof(int32_t) * 2 * (count + 1));
    CHECK(oracle_get_pairs(s, &count, pairs, pos));
    CHECK(oracle_get_thermostat(s, &xi, &eta, &e));
    CHECK(oracle_set_thermostat(s, xi, eta));
    CHECK(oracle_negate_velocities(s));
    CHECK(oracle_step(s, 5));
    CHECK(oracle_set_nve(s));
    /* error paths: they must return an error, not crash */
    if (oracle_set_pair(s, ntypes, 0, 1.0, 1.0, 2.5) == 0) return 1;
    if (oracle_set_shift_mode(s, 7) == 0) return 1;
    if (oracle_set_nvt(s, -1.0, 1.0) == 0) return 1;
    oracle_destroy(s);
    free(pos); free(vel); free(type); free(f); free(u); free(w); free(img); free(pairs);
    return 0;
}

int main(void)
{
    /* a small box (fewer than three cells per axis), a larger one, two types, other forms */
    if (run(64, 6.0, 1, 0, 0, 0)) return 1;
    if (run(500, 8.4, 1, 0, 1, 1)) return 1;
    if (run(700, 9.6, 2, 0, 0, 1)) return 1;
    for (int style = 1; style <= 3; ++style)
        if (run(343, 7.6, 1, style, style & 1, 0)) return 1;
    if (oracle_create(0, NULL, NULL, NULL, NULL, NULL, 1, 0.005, 0.4) != NULL) return 1;
    printf("ok\n");
    return 0;
}
