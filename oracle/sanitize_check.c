/*
 * sanitize_check.c -- TEST INFRASTRUCTURE: a standalone driver that runs the
 * oracle's entry points on seeded synthetic sweeps, built with the host's
 * address and undefined-behaviour sanitizers by tests/test_oracle_sanitize.py.
 * It checks no values (the pinned tests do that); it exercises the edges that
 * stress indexing: empty and one-point sweeps, open and closed cylinders, one
 * ring, sub-sampling, reported rings (some beyond the lattice), non-finite and
 * out-of-range points, duplicated returns, point labels, segment removal, the
 * cosine test and edge scores at several radii.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static const double PI = 3.14159265358979323846;

int oracle_mesh_segment_ex(const float* xyz, const uint8_t* ring_ids, int64_t n, int32_t H, int32_t W, int32_t s,
                           int32_t wrap, const double* elev, double az0, double r_min, double r_max, int32_t pred,
                           const double* thr, double cos_min, int32_t min_segment, float* vertices, float* normals,
                           int32_t* labels, int32_t* triangles, int32_t* vertex_point, int64_t* counts,
                           double* normals64, int32_t* point_labels);
void oracle_edge_scores(int32_t H, int32_t Wp, int32_t wrap, const int32_t* label, const int32_t* truth,
                        int32_t R, int64_t* out);

static uint64_t rng_state = 88172645463325252ull;
static double uniform(void) {  /* xorshift64, in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

/* A sweep of a sensor at the origin over a ground plane z = -1.7 and a wall
 * y = 6: ring i fires at elevation elev[i], firing j at azimuth az0 + 2 pi j / W;
 * each ray's first hit within 80 m is emitted with range noise, some rays drop. */
static int64_t make_sweep(int32_t H, int32_t W, const double* elev, double az0, double drop, float* xyz,
                          uint8_t* rings) {
    int64_t n = 0;
    for (int32_t j = 0; j < W; ++j) {
        const double phi = az0 + 2.0 * PI * j / W;
        for (int32_t i = 0; i < H; ++i) {
            if (uniform() < drop) continue;
            const double ux = cos(elev[i]) * cos(phi), uy = cos(elev[i]) * sin(phi), uz = sin(elev[i]);
            double t = 1e30;
            if (uz < 0) t = fmin(t, -1.7 / uz);
            if (uy > 0) t = fmin(t, 6.0 / uy);
            if (t > 80.0) continue;
            t += 0.01 * (uniform() - 0.5);
            xyz[3 * n] = (float)(t * ux);
            xyz[3 * n + 1] = (float)(t * uy);
            xyz[3 * n + 2] = (float)(t * uz);
            rings[n] = (uint8_t)i;
            ++n;
        }
    }
    return n;
}

static int run_case(int32_t H, int32_t W, int32_t s, int32_t wrap, int32_t pred, int32_t min_segment,
                    int use_rings, int extras, double drop) {
    double* elev = malloc(sizeof(double) * (size_t)H);
    for (int32_t i = 0; i < H; ++i) elev[i] = (H == 1 ? 0.0 : (10.0 - 30.0 * i / (H - 1))) * PI / 180.0;
    const int64_t cap = (int64_t)H * W + 16;
    float* xyz = malloc(sizeof(float) * 3 * (size_t)cap * 2);
    uint8_t* rings = malloc((size_t)cap * 2);
    int64_t n = make_sweep(H, W, elev, 0.05, drop, xyz, rings);
    if (extras && n > 4) {
        /* duplicates of the first returns, a NaN, an infinity, a point too close, one far away */
        const int64_t m = n;
        for (int64_t q = 0; q < 4; ++q, ++n) {
            for (int d = 0; d < 3; ++d) xyz[3 * n + d] = xyz[3 * q + d];
            rings[n] = rings[q];
        }
        xyz[0] = NAN;
        xyz[4] = INFINITY;
        xyz[3 * (m - 1)] = 0.1f; xyz[3 * (m - 1) + 1] = 0.0f; xyz[3 * (m - 1) + 2] = 0.0f;
        xyz[3 * (m - 2)] = 500.0f;
        rings[m - 3] = (uint8_t)(H + 3);   /* a reported ring beyond the lattice */
    }
    const int32_t Wp = W / s;
    const int64_t cells = (int64_t)H * Wp;
    float* vertices = malloc(sizeof(float) * 3 * (size_t)(cells + 1));
    float* normals = malloc(sizeof(float) * 3 * (size_t)(cells + 1));
    double* normals64 = malloc(sizeof(double) * 3 * (size_t)(cells + 1));
    int32_t* labels = malloc(sizeof(int32_t) * (size_t)(cells + 1));
    int32_t* triangles = malloc(sizeof(int32_t) * 3 * (size_t)(2 * cells + 1));
    int32_t* vpoint = malloc(sizeof(int32_t) * (size_t)(cells + 1));
    int32_t* plabels = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t counts[3] = {0, 0, 0};
    const double thr[3] = {0.2, 0.2, 0.2};
    int rc = oracle_mesh_segment_ex(xyz, use_rings ? rings : NULL, n, H, W, s, wrap, elev, 0.05, 1.0, 60.0, pred,
                                    thr, 0.95, min_segment, vertices, normals, labels, triangles, vpoint, counts,
                                    normals64, plabels);
    if (rc == 0) {
        /* edge scores on a lattice filled from the vertices in order (every third
           cell left empty), truth = ground or wall */
        int32_t* clab = malloc(sizeof(int32_t) * (size_t)(cells + 1));
        int32_t* ctru = malloc(sizeof(int32_t) * (size_t)(cells + 1));
        for (int64_t c = 0; c < cells; ++c) clab[c] = ctru[c] = -1;
        int64_t v = 0;
        for (int64_t c = 0; c < cells && v < counts[0]; ++c) {
            if (c % 3 == 0) continue;  /* leave some cells empty */
            clab[c] = labels[v];
            ctru[c] = vertices[3 * v + 2] < -1.6f ? 0 : 1;
            ++v;
        }
        int64_t out[4];
        for (int32_t R = 0; R <= 3; ++R) oracle_edge_scores(H, Wp, wrap, clab, ctru, R, out);
        free(clab);
        free(ctru);
    }
    free(elev); free(xyz); free(rings); free(vertices); free(normals); free(normals64); free(labels);
    free(triangles); free(vpoint); free(plabels);
    return rc;
}

int main(void) {
    int failures = 0;
    /* H, W, s, wrap, pred, min_segment, reported rings, extra points, dropout */
    const int cases[][8] = {
        {16, 360, 1, 1, 0, 0, 0, 0}, {16, 360, 2, 1, 0, 3, 1, 1}, {16, 360, 5, 0, 1, 0, 0, 1},
        {1, 90, 1, 1, 0, 0, 0, 0},   {2, 4, 1, 0, 0, 2, 1, 1},    {5, 3, 1, 1, 1, 0, 0, 0},
        {33, 101, 1, 0, 0, 0, 1, 1}, {64, 256, 4, 1, 1, 5, 1, 1},
    };
    for (size_t k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k) {
        const int* c = cases[k];
        for (int d = 0; d < 2; ++d) {
            const int rc = run_case(c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], d ? 0.3 : 0.0);
            if (rc != 0) {
                fprintf(stderr, "case %zu: oracle returned %d\n", k, rc);
                ++failures;
            }
        }
    }
    /* an empty sweep */
    {
        const double elev[4] = {0.1, 0.0, -0.1, -0.2};
        float v[3];
        int32_t l[1], t[3], vp[1], pl[1];
        int64_t counts[3];
        const double thr[3] = {0.2, 0.2, 0.2};
        if (oracle_mesh_segment_ex(NULL, NULL, 0, 4, 8, 1, 1, elev, 0.0, 1.0, 60.0, 0, thr, 0.0, 0, v, v, l, t, vp,
                                   counts, NULL, pl) != 0 || counts[0] != 0)
            ++failures;
    }
    printf("sanitize check: %d failures\n", failures);
    return failures ? 1 : 0;
}
