/*
 * Seeded synthetic inputs for K-NN descent on the probability simplex.
 *
 * This module only draws inputs.  It holds none of the method's arithmetic
 * (no divergence, no neighbor lists, no stop test); both the GPU library and
 * the CPU oracle consume the bytes it writes.
 *
 * Points are i.i.d. Dirichlet(1,...,1) on the simplex with D = d+1 stored
 * coordinates, the distribution the paper draws its test points from
 * (Section 4, scaling experiment; Table 4).  A Dirichlet(1^D) vector is a
 * vector of D i.i.d. unit exponentials divided by their sum.
 *
 * Randomness is counter based: every draw is mix64-hashed from
 * (seed, tag, a, b), so any point can be regenerated on its own and the
 * bytes do not depend on threading.  mix64 is the SplitMix64 finalizer
 * (Steele, Lea and Flood, OOPSLA 2014; constants of Stafford's "variant 13").
 *
 * Tags used by this module: 5 = batched instance parameters,
 * 6 = point coordinates, 7 = recall subsample.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static uint64_t synth_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_hash(uint64_t s, uint64_t t, uint64_t a, uint64_t b)
{
    uint64_t h = synth_mix64(s ^ (t * 0x9E3779B97F4A7C15ULL));
    h = synth_mix64(h ^ a);
    return synth_mix64(h ^ b);
}

/* floor(h * m / 2^64): an integer in [0, m) from a 64-bit hash. */
uint64_t synth_bound(uint64_t h, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)h * m) >> 64);
}

/* One Dirichlet(1^D) point into w[0..D-1] (FP64, clamped below at 1e-12). */
static void synth_point(uint64_t data_seed, int64_t j, int D, double *w)
{
    double sum = 0.0;
    for (int i = 0; i < D; ++i) {
        uint64_t h = synth_hash(data_seed, 6, (uint64_t)j, (uint64_t)i);
        /* u in (0, 1]: 53 random bits, offset by one ulp so log(u) is finite */
        double u = (double)((h >> 11) + 1) * 0x1.0p-53;
        w[i] = -log(u);
        sum += w[i];
    }
    for (int i = 0; i < D; ++i) {
        double x = w[i] / sum;
        w[i] = x < 1e-12 ? 1e-12 : x;
    }
}

/* n points, D coordinates each, row-major FP64.  D <= 4096. */
int synth_dirichlet_f64(uint64_t data_seed, int64_t n, int D, double *out)
{
    if (D < 1 || D > 4096 || n < 0 || !out) return -1;
    for (int64_t j = 0; j < n; ++j) synth_point(data_seed, j, D, out + (size_t)j * D);
    return 0;
}

/* Same points, each coordinate rounded to nearest FP32 (no renormalisation). */
int synth_dirichlet_f32(uint64_t data_seed, int64_t n, int D, float *out)
{
    double w[4096];
    if (D < 1 || D > 4096 || n < 0 || !out) return -1;
    for (int64_t j = 0; j < n; ++j) {
        synth_point(data_seed, j, D, w);
        for (int i = 0; i < D; ++i) out[(size_t)j * D + i] = (float)w[i];
    }
    return 0;
}

/* Parameters of batched instance b drawn from base seed `base`:
 * n in [500, 20000], d in [3, 20], K in {8, 16, 32}, plus the data seed and
 * the algorithm seed of that instance. */
void synth_instance(uint64_t base, int64_t b, int64_t *n, int32_t *d, int32_t *K,
                    uint64_t *data_seed, uint64_t *seed)
{
    static const int32_t ks[3] = {8, 16, 32};
    *n = 500 + (int64_t)synth_bound(synth_hash(base, 5, (uint64_t)b, 0), 19501);
    *d = 3 + (int32_t)synth_bound(synth_hash(base, 5, (uint64_t)b, 1), 18);
    *K = ks[synth_bound(synth_hash(base, 5, (uint64_t)b, 2), 3)];
    *data_seed = synth_hash(base, 5, (uint64_t)b, 3);
    *seed = synth_hash(base, 5, (uint64_t)b, 4);
}

/* m distinct query indices in [0, n), in draw order (m <= n). */
int synth_subsample(uint64_t seed, int64_t n, int64_t m, unsigned char *seen, int64_t *out)
{
    if (m > n || m < 0) return -1;
    for (int64_t i = 0; i < n; ++i) seen[i] = 0;
    int64_t got = 0;
    for (uint64_t a = 0; got < m; ++a) {
        int64_t q = (int64_t)synth_bound(synth_hash(seed, 7, 0, a), (uint64_t)n);
        if (!seen[q]) { seen[q] = 1; out[got++] = q; }
    }
    return 0;
}
