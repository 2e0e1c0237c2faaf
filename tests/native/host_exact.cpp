// Host build of the library's exact predicates (exact.hpp), so the CPU test
// suite can check them against rational arithmetic without a GPU.
#include "exact.hpp"

extern "C" {
int hx_orient(double ax, double ay, double bx, double by, double cx, double cy) {
    return hx::orient(ax, ay, bx, by, cx, cy);
}
int hx_orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
    return hx::orient_exact(ax, ay, bx, by, cx, cy);
}
unsigned hx_angle_key(double x, double y, double x0, double y0) {
    return hx::angle_key(x, y, x0, y0);
}
int hx_key_at_least(double x, double y, double x0, double y0, double k) {
    return hx::key_at_least(x, y, x0, y0, x - x0 >= 0.0, k) ? 1 : 0;
}
}

extern "C" unsigned hx_turn_key(double px, double py, double cx, double cy) {
    return hx::turn_key(px, py, cx, cy);
}
