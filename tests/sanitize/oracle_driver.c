/* Exercises every entry of the CPU oracle on small grids, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure): 2D and
 * 3D Voronoi-like label fields, steps with the taxicab and the Euclidean
 * re-initialization, both predictor-correction terms, intermediates, grain
 * replacement, labels, volumes, areas, coarsening and the stand-alone pieces.
 * Exits non-zero on any failed call. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gg_oracle.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__);    \
            exit(1);                                                    \
        }                                                               \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

/* nearest of G random seeds under the periodic metric */
static int32_t *voronoi(int dim, const int32_t n[3], int G) {
    double *s = malloc(sizeof(double) * 3 * G);
    for (int k = 0; k < G; ++k)
        for (int a = 0; a < 3; ++a) s[3 * k + a] = a < dim ? urand() * n[a] : 0.0;
    const long long m = (long long)n[0] * n[1] * n[2];
    int32_t *lab = malloc(sizeof(int32_t) * m);
    for (long long v = 0; v < m; ++v) {
        const long long x = v % n[0], y = (v / n[0]) % n[1], z = v / ((long long)n[0] * n[1]);
        const double p[3] = {x + 0.5, y + 0.5, z + 0.5};
        double best = 1e300;
        int id = 0;
        for (int k = 0; k < G; ++k) {
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                double d = p[a] - s[3 * k + a];
                d -= n[a] * nearbyint(d / n[a]);
                d2 += d * d;
            }
            if (d2 < best) {
                best = d2;
                id = k;
            }
        }
        lab[v] = id;
    }
    free(s);
    return lab;
}

static void run(int dim, int N, int G, double W, double sigma) {
    const int32_t n[3] = {N, N, dim == 3 ? N : 1};
    int32_t *lab = voronoi(dim, n, G);
    orc_sim *s = orc_create(dim, n, W, lab, G);
    CHECK(s);
    double *quat = malloc(sizeof(double) * 4 * G), *energy = malloc(sizeof(double) * G);
    for (int k = 0; k < G; ++k) {
        double q[4], nrm = 0.0;
        for (int a = 0; a < 4; ++a) nrm += (q[a] = urand() - 0.5) * q[a];
        for (int a = 0; a < 4; ++a) quat[4 * k + a] = q[a] / sqrt(nrm);
        energy[k] = 100.0 + 1000.0 * urand();
    }
    CHECK(orc_set_physics(s, 3, quat, 15.0, energy, 2e-5, 0.3) == 0);
    const double dt = sigma * sigma / (2.0 * N * N);
    orc_keep_intermediates(s, 1);
    for (int t = 0; t < 3; ++t) CHECK(orc_step(s, dt) == 0);
    CHECK(orc_set_redistance(s, 1) == 0);
    CHECK(orc_step(s, dt) == 0);
    CHECK(orc_set_redistance(s, 0) == 0);
    const long long m = (long long)n[0] * n[1] * n[2];
    int32_t *labels = malloc(sizeof(int32_t) * m);
    double *vol = malloc(sizeof(double) * G), *area = malloc(sizeof(double) * G), *wa = malloc(sizeof(double) * G);
    CHECK(orc_labels(s, labels) == 0);
    CHECK(orc_volumes(s, vol) == 0);
    CHECK(orc_grain_areas(s, area, wa) == 0);
    double total = 0.0;
    for (int k = 0; k < G; ++k) total += vol[k];
    CHECK(fabs(total - (double)m) < 5e-3 * m);
    /* per-grain queries, and replacing a grain with its own state */
    for (int k = 0; k < G; ++k) {
        int32_t lo[3], ext[3];
        const int alive = orc_get_box(s, k, lo, ext);
        CHECK(alive >= 0);
        if (!alive) continue;
        const long long e = (long long)ext[0] * ext[1] * ext[2];
        double *phi = malloc(sizeof(double) * e);
        int32_t *io = malloc(sizeof(int32_t) * e);
        CHECK(orc_get_phi(s, k, phi, e) == 0);
        CHECK(orc_get_iota(s, k, io, e) == 0);
        CHECK(orc_set_grain(s, k, 1, lo, ext, phi, io) == 0);
        free(phi);
        free(io);
        if (orc_get_prev_box(s, k, lo, ext) == 1) {
            const long long pe = (long long)ext[0] * ext[1] * ext[2];
            double *buf = malloc(sizeof(double) * pe);
            CHECK(orc_get_psi(s, k, buf, pe) == 0);
            CHECK(orc_get_phic(s, k, buf, pe) == 0);
            free(buf);
        }
    }
    CHECK(orc_step(s, dt) == 0);
    /* coarsening by 2 (when the coarse grid keeps 4P + 2 voxels), then a step */
    const int P = (int)ceil(W);
    if (N / 2 >= 4 * P + 2) {
        const int32_t np[3] = {N / 2, N / 2, dim == 3 ? N / 2 : 1};
        CHECK(orc_coarsen(s, np) == 0);
        CHECK(orc_step(s, dt * 0.25) == 0);
    }
    CHECK(orc_alive_count(s) >= 1 && orc_grain_count(s) == G);
    orc_destroy(s);
    /* the stand-alone pieces on a wrapping box */
    {
        const int32_t lo[3] = {N - 3, 1, 0}, ext[3] = {N / 2, N, dim == 3 ? 5 : 1};
        const long long e = (long long)ext[0] * ext[1] * ext[2];
        double *f = malloc(sizeof(double) * e), *out = malloc(sizeof(double) * e);
        for (long long i = 0; i < e; ++i) f[i] = W * (2.0 * urand() - 1.0);
        CHECK(orc_convolve_box(dim, n, W, sigma, lo, ext, f, out) > 0); /* returns R */
        CHECK(orc_redistance_box(dim, n, W, lo, ext, f, out) == 0);
        CHECK(orc_redistance_box_euclid(dim, n, W, lo, ext, f, out) == 0);
        free(f);
        free(out);
    }
    double mob;
    CHECK(orc_pair_weight(orc_misorientation_deg(quat, quat + 4), 15.0, &mob) >= 0.0);
    CHECK(orc_euclid_sweeps(dim, W) >= 2);
    free(quat);
    free(energy);
    free(labels);
    free(vol);
    free(area);
    free(wa);
    free(lab);
}

int main(void) {
    orc_set_num_threads(2);
    run(2, 64, 12, 6.0, 1.5);
    run(3, 40, 20, 4.0, 1.5);
    printf("oracle driver ok\n");
    return 0;
}
