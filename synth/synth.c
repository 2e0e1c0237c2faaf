/* synth.c - seeded synthetic point sets (see synth.h).  No hull arithmetic. */
#include "synth.h"

#include <math.h>
#include <stddef.h>

#define PCG_MULT 6364136223846793005ULL

void synth_pcg32_seed(synth_pcg32* g, uint64_t initstate, uint64_t initseq) {
    g->state = 0u;
    g->inc = (initseq << 1u) | 1u;
    (void)synth_pcg32_next(g);
    g->state += initstate;
    (void)synth_pcg32_next(g);
}

uint32_t synth_pcg32_next(synth_pcg32* g) {
    uint64_t old = g->state;
    g->state = old * PCG_MULT + g->inc;
    uint32_t xs = (uint32_t)(((old >> 18u) ^ old) >> 27u);
    uint32_t rot = (uint32_t)(old >> 59u);
    return (xs >> rot) | (xs << ((-rot) & 31u));
}

double synth_u53(synth_pcg32* g) {
    uint32_t a = synth_pcg32_next(g) >> 5;   /* 27 bits */
    uint32_t b = synth_pcg32_next(g) >> 6;   /* 26 bits */
    return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

uint32_t synth_bounded(synth_pcg32* g, uint32_t bound) {
    uint32_t threshold = (uint32_t)(-bound) % bound;
    for (;;) {
        uint32_t r = synth_pcg32_next(g);
        if (r >= threshold) return r % bound;
    }
}

int synth_square(double* xy, int64_t n, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = 0; i < n; ++i) {
        xy[2 * i] = synth_u53(&g);
        xy[2 * i + 1] = synth_u53(&g);
    }
    return 0;
}

int synth_disk(double* xy, int64_t n, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = 0; i < n;) {
        double x = 2.0 * synth_u53(&g) - 1.0;
        double y = 2.0 * synth_u53(&g) - 1.0;
        double r2 = x * x;
        r2 = r2 + y * y;
        if (r2 < 1.0) {
            xy[2 * i] = x;
            xy[2 * i + 1] = y;
            ++i;
        }
    }
    return 0;
}

int synth_annulus(double* xy, int64_t n, double r_in, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy) || !(r_in >= 0.0 && r_in <= 1.0)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    const double two_pi = 6.283185307179586;
    const double a = r_in * r_in;
    for (int64_t i = 0; i < n; ++i) {
        double th = two_pi * synth_u53(&g);
        double r = sqrt(a + synth_u53(&g) * (1.0 - a));
        xy[2 * i] = r * cos(th);
        xy[2 * i + 1] = r * sin(th);
    }
    return 0;
}

/* One pair of independent standard normals (Marsaglia polar method). */
static void polar_pair(synth_pcg32* g, double* z0, double* z1) {
    for (;;) {
        double u = 2.0 * synth_u53(g) - 1.0;
        double v = 2.0 * synth_u53(g) - 1.0;
        double s = u * u;
        s = s + v * v;
        if (s < 1.0 && s > 0.0) {
            double f = sqrt(-2.0 * log(s) / s);
            *z0 = u * f;
            *z1 = v * f;
            return;
        }
    }
}

int synth_gaussian(double* xy, int64_t n, double sigma, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = 0; i < n; ++i) {
        double a, b;
        polar_pair(&g, &a, &b);
        xy[2 * i] = sigma * a;
        xy[2 * i + 1] = sigma * b;
    }
    return 0;
}

int synth_ngon(double* xy, int64_t n, int log2k, uint64_t s0, uint64_t s1) {
    if (log2k < 2 || log2k > 30) return -1;
    int64_t K = (int64_t)1 << log2k;
    if (n < K || !xy) return -1;
    const double two_pi = 6.283185307179586;
    for (int64_t k = 0; k < K; ++k) {
        double th = two_pi * (double)k / (double)K;
        xy[2 * k] = cos(th);
        xy[2 * k + 1] = sin(th);
    }
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = K; i < n; ++i) {
        int64_t k = (int64_t)synth_bounded(&g, (uint32_t)K);
        xy[2 * i] = xy[2 * k];
        xy[2 * i + 1] = xy[2 * k + 1];
    }
    return 0;
}

int synth_shuffle(double* xy, int64_t n, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy) || n > (int64_t)UINT32_MAX) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)synth_bounded(&g, (uint32_t)(i + 1));
        double tx = xy[2 * i], ty = xy[2 * i + 1];
        xy[2 * i] = xy[2 * j];
        xy[2 * i + 1] = xy[2 * j + 1];
        xy[2 * j] = tx;
        xy[2 * j + 1] = ty;
    }
    return 0;
}

int synth_grid(double* xy, int side, int copies, uint64_t s0, uint64_t s1) {
    if (side < 1 || copies < 1 || !xy) return -1;
    int64_t i = 0;
    for (int c = 0; c < copies; ++c)
        for (int a = 0; a < side; ++a)
            for (int b = 0; b < side; ++b) {
                xy[2 * i] = (double)a;
                xy[2 * i + 1] = (double)b;
                ++i;
            }
    return synth_shuffle(xy, i, s0, s1);
}

int synth_grid_draws(double* xy, int64_t n, int side, uint64_t s0, uint64_t s1) {
    if (n < 0 || side < 1 || (n > 0 && !xy)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    for (int64_t i = 0; i < n; ++i) {
        xy[2 * i] = (double)synth_bounded(&g, (uint32_t)side);
        xy[2 * i + 1] = (double)synth_bounded(&g, (uint32_t)side);
    }
    return 0;
}

int synth_mixture(double* xy, int64_t n, uint64_t s0, uint64_t s1) {
    if (n < 0 || (n > 0 && !xy)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, s1);
    int K = 1 + (int)(synth_pcg32_next(&g) % 8u);
    double cum[8], mx[8], my[8], c[8], s[8], sminor[8];
    double total = 0.0;
    for (int k = 0; k < K; ++k) {
        double w = -log(1.0 - synth_u53(&g));  /* exponential(1) */
        total += w;
        cum[k] = total;
        mx[k] = -10.0 + 20.0 * synth_u53(&g);
        my[k] = -10.0 + 20.0 * synth_u53(&g);
        double rot = 3.141592653589793 * synth_u53(&g);
        c[k] = cos(rot);
        s[k] = sin(rot);
        double r = exp(log(50.0) * synth_u53(&g));
        sminor[k] = 1.0 / r;
    }
    for (int k = 0; k < K; ++k) cum[k] /= total;
    cum[K - 1] = 1.0;
    for (int64_t i = 0; i < n; ++i) {
        double u = synth_u53(&g);
        int k = 0;
        while (k < K - 1 && u >= cum[k]) ++k;
        double a, b;
        polar_pair(&g, &a, &b);
        double px = a;             /* sigma_major = 1 */
        double py = b * sminor[k];
        double rx = c[k] * px;
        rx = rx - s[k] * py;
        double ry = s[k] * px;
        ry = ry + c[k] * py;
        xy[2 * i] = mx[k] + rx;
        xy[2 * i + 1] = my[k] + ry;
    }
    return 0;
}

int synth_batch_sizes(int64_t* sizes, int S, double lo, double hi, uint64_t s0) {
    if (S < 0 || (S > 0 && !sizes) || !(lo >= 1.0) || !(hi >= lo)) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, 0u);
    double a = log(lo), b = log(hi / lo);
    for (int i = 0; i < S; ++i) {
        int64_t v = (int64_t)floor(exp(a + synth_u53(&g) * b));
        if (v < (int64_t)lo) v = (int64_t)lo;
        sizes[i] = v;
    }
    return 0;
}

int synth_batch_set(double* xy, int64_t n, uint64_t s0, int set_id) {
    if (n < 0 || (n > 0 && !xy) || set_id < 0) return -1;
    synth_pcg32 g;
    synth_pcg32_seed(&g, s0, (uint64_t)set_id + 1u);
    int kind = (int)(synth_pcg32_next(&g) % 4u);
    /* The point stream continues from the state after the kind draw. */
    uint64_t st = (uint64_t)synth_pcg32_next(&g) << 32;
    st |= synth_pcg32_next(&g);
    int rc;
    switch (kind) {
        case 0: rc = synth_square(xy, n, st, (uint64_t)set_id + 1u); break;
        case 1: rc = synth_disk(xy, n, st, (uint64_t)set_id + 1u); break;
        case 2: rc = synth_gaussian(xy, n, 1.0, st, (uint64_t)set_id + 1u); break;
        default: rc = synth_annulus(xy, n, 0.999, st, (uint64_t)set_id + 1u); break;
    }
    return rc == 0 ? kind : -1;
}

uint64_t synth_hash(const double* xy, int64_t n) {
    const unsigned char* p = (const unsigned char*)xy;
    uint64_t h = 1469598103934665603ULL;
    size_t bytes = (size_t)(n > 0 ? n : 0) * 16u;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= p[i];
        h *= 1099511628211ULL;
    }
    return h;
}
