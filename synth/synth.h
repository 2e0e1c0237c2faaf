/*
 * synth.h - seeded synthetic point sets for exact 2D convex-hull workloads.
 *
 * This module only draws random numbers and places points; it holds none of
 * the hull method's arithmetic (no orientation tests, no angles, no sorting by
 * geometry).  Both the CPU oracle tests and the GPU benchmark take their input
 * bytes from here, so that the two sides always see identical points.
 *
 * Random source: PCG32 (M. E. O'Neill, "PCG: A Family of Simple Fast
 * Space-Efficient Statistically Good Algorithms for Random Number
 * Generation", 2014), the XSH-RR 64/32 member, written from its published
 * definition: a 64-bit LCG state with multiplier 6364136223846793005 and an
 * odd increment, output = rotate32(((s >> 18) ^ s) >> 27, s >> 59).
 *
 * All point buffers are row-major float64 [n][2] (x then y).  Functions that
 * fill a buffer never allocate; the caller owns every buffer.  Return value:
 * 0 on success, -1 on a bad argument.
 */
#ifndef SYNTH_H
#define SYNTH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { uint64_t state, inc; } synth_pcg32;

/* Seeding as in the PCG paper: inc = 2*initseq+1, state = step(step(0)+initstate). */
void     synth_pcg32_seed(synth_pcg32* g, uint64_t initstate, uint64_t initseq);
uint32_t synth_pcg32_next(synth_pcg32* g);
/* Uniform double in [0,1) with 53 random bits: ((a>>5)*2^26 + (b>>6)) * 2^-53. */
double   synth_u53(synth_pcg32* g);
/* Unbiased integer in [0, bound) by threshold rejection; bound >= 1. */
uint32_t synth_bounded(synth_pcg32* g, uint32_t bound);

/* n points uniform in [0,1)^2. */
int synth_square(double* xy, int64_t n, uint64_t s0, uint64_t s1);
/* n points uniform in the open unit disk: (2u-1, 2v-1) kept when x^2+y^2 < 1. */
int synth_disk(double* xy, int64_t n, uint64_t s0, uint64_t s1);
/* n points uniform in the annulus r in [r_in, 1]: theta = 2*pi*u,
 * r = sqrt(r_in^2 + u'*(1-r_in^2)). */
int synth_annulus(double* xy, int64_t n, double r_in, uint64_t s0, uint64_t s1);
/* n points with independent N(0, sigma^2) coordinates (Marsaglia polar method). */
int synth_gaussian(double* xy, int64_t n, double sigma, uint64_t s0, uint64_t s1);
/* n >= 2^log2k points: every vertex (cos 2*pi*k/K, sin 2*pi*k/K), K = 2^log2k,
 * once in order, then n-K vertices drawn uniformly with repetition. */
int synth_ngon(double* xy, int64_t n, int log2k, uint64_t s0, uint64_t s1);
/* Fisher-Yates shuffle of n points in place. */
int synth_shuffle(double* xy, int64_t n, uint64_t s0, uint64_t s1);
/* side x side integer grid (values 0..side-1), every cell `copies` times,
 * shuffled; fills side*side*copies points. */
int synth_grid(double* xy, int side, int copies, uint64_t s0, uint64_t s1);
/* n draws from a side x side integer grid, with repetition. */
int synth_grid_draws(double* xy, int64_t n, int side, uint64_t s0, uint64_t s1);
/* n points from a mixture of K = 1 + (draw mod 8) anisotropic Gaussians:
 * weights from normalised exponentials, means uniform in [-10,10]^2,
 * rotation uniform in [0, pi), sigma_major = 1, sigma_minor = 1/r with
 * r log-uniform in [1, 50]. */
int synth_mixture(double* xy, int64_t n, uint64_t s0, uint64_t s1);
/* Batch layout: S set sizes floor(exp(ln lo + u*ln(hi/lo))) from stream (s0, 0). */
int synth_batch_sizes(int64_t* sizes, int S, double lo, double hi, uint64_t s0);
/* One batch member from stream (s0, set_id+1): first draw mod 4 picks the
 * distribution {0 square, 1 disk, 2 Gaussian sigma=1, 3 annulus [0.999,1]}.
 * Returns the kind (0..3) or -1. */
int synth_batch_set(double* xy, int64_t n, uint64_t s0, int set_id);

/* 64-bit FNV-1a over the raw bytes of n points (input content hash). */
uint64_t synth_hash(const double* xy, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
