/* Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure): every entry point on small deterministic
 * inputs, among them repeats, collinear sets, grids and tiny sizes.  Exits 0
 * when every call succeeds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static uint64_t g_state = 88172645463325252ull;
static double next_unit(void) {  /* xorshift64*, 53-bit uniform in [0, 1) */
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 2685821657736338717ull) >> 11) * 0x1p-53;
}

static int run(const double* xy, int64_t n) {
    int32_t* out = malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* srt = malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* r2 = malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* hl = malloc((size_t)(n + 1) * sizeof(int32_t));
    uint8_t* k1 = malloc((size_t)(n + 1));
    int8_t* reg = malloc((size_t)(n + 1));
    int32_t* kept = malloc((size_t)(n + 1) * sizeof(int32_t));
    int64_t h = 0;
    int bad = 0;
    bad |= oracle_hull(xy, n, out, n + 1, &h) != 0;
    for (int64_t chunk = -1; chunk <= 3; ++chunk) {
        oracle_model_result m = {0};
        m.round1_keep = k1;
        m.sorted = srt;
        m.round2 = r2;
        m.hull = hl;
        bad |= oracle_model(xy, n, chunk, &m) != 0;
        bad |= m.h != h;
    }
    oracle_chain_result c = {0};
    c.region = reg;
    c.kept = kept;
    c.hull = hl;
    bad |= oracle_chain(xy, n, &c) != 0;
    bad |= c.h != h;
    double dirs[16 * 2];
    for (int j = 0; j < 16; ++j) {
        dirs[2 * j] = next_unit() - 0.5;
        dirs[2 * j + 1] = next_unit() - 0.5;
    }
    int32_t cand[20];
    int64_t m1 = 0;
    bad |= oracle_learned_round1(xy, n, dirs, 16, k1, cand, &m1) != 0;
    free(out); free(srt); free(r2); free(hl); free(k1); free(reg); free(kept);
    return bad;
}

int main(void) {
    int bad = 0;
    for (int64_t n = 0; n <= 9; ++n) {  /* tiny sizes, random points */
        double xy[18];
        for (int64_t i = 0; i < 2 * n; ++i) xy[i] = next_unit();
        bad |= run(xy, n);
    }
    const int64_t N = 3000;
    double* xy = malloc((size_t)(2 * N) * sizeof(double));
    for (int kind = 0; kind < 5; ++kind) {
        for (int64_t i = 0; i < N; ++i) {
            double x = next_unit(), y = next_unit();
            if (kind == 1) { x = (double)(i % 7); y = (double)((i / 7) % 5); }          /* grid, repeats */
            if (kind == 2) { x = (double)(i % 100); y = 2.0 * x - 3.0; }                  /* collinear */
            if (kind == 3) { x = 0.25; y = 0.75; }                                        /* all equal */
            if (kind == 4) { x = 2.0 * x - 1.0; y = 2.0 * y - 1.0; if (x * x + y * y > 1.0) { x = 0.0; y = 0.0; } }
            xy[2 * i] = x;
            xy[2 * i + 1] = y;
        }
        bad |= run(xy, N);
    }
    free(xy);
    printf("sanitized oracle: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
