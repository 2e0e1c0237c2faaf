// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer host build of
// the library's exact predicates (exact.hpp): the adaptive orientation
// against its exact expansion, and the angle and turn keys, on random and
// near-degenerate inputs across the input domain.  Exits 0 when the adaptive
// and exact orientations agree everywhere.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "exact.hpp"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double next_unit() {
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 2685821657736338717ull) >> 11) * 0x1p-53;
}

int main() {
    int bad = 0;
    unsigned sink = 0;
    for (int t = 0; t < 200000; ++t) {
        const double s = std::ldexp(1.0, (int)(next_unit() * 500.0) - 250);
        double ax = (next_unit() - 0.5) * s, ay = (next_unit() - 0.5) * s;
        double bx = (next_unit() - 0.5) * s, by = (next_unit() - 0.5) * s;
        const double u = next_unit() * 3.0 - 1.0;
        double cx = ax + u * (bx - ax), cy = ay + u * (by - ay);
        if (t & 1) cx = std::nextafter(cx, (t & 2) ? INFINITY : -INFINITY);
        const int a = hx::orient(ax, ay, bx, by, cx, cy);
        const int e = hx::orient_exact(ax, ay, bx, by, cx, cy);
        bad |= a != e;
        if (cy > ay || (cy == ay && cx > ax)) sink += hx::angle_key(cx, cy, ax, ay);
        if (cx != bx || cy != by) sink += hx::turn_key(cx, cy, bx, by);
    }
    std::printf("sanitized exact predicates: %s (%u)\n", bad ? "FAILED" : "ok", sink);
    return bad;
}
