// kernels_learned.hip - the learned-filter variant of Steps 1-2 (not in the
// paper) and the training kernels of its network.
//
// Proposal (per hull, before the first round), k_front, one workgroup:
//   32 x 32 occupancy histogram of a sample (every point up to 4096, else 16
//   evenly spaced blocks of 256 points) over the sample's bounding box; the
//   1024 -> 256 -> 256 -> 32 network (bfloat16 weights and layer inputs,
//   float32 sums): 16 directions; the sample point farthest along each
//   (fma(x, ux, y * uy), ties: smallest index).  The final Step-1 block
//   (kernels_filter.hip) then takes the exact convex hull of these 16
//   points and the four Step-1 extremes: the discard polygon, which
//   contains the quadrilateral, so the first round stays conservative
//   whatever the network says.
// k_sample_bbox, k_sample_hist, k_hist_to_x and k_mlp_layer compute the
// histogram and the network as separate kernels for the standalone entry
// points (k_front's outputs equal theirs bit for bit).
// Training (float32, off the timed path): tiled GEMM with bias / ReLU
// epilogues, mean-squared-error gradient, column sums, Adam.
#include "exact.hpp"
#include "kernels.hpp"
#include "steps.hpp"

namespace hx {
namespace {

constexpr int kHB = 256;        // threads of the histogram and network kernels
constexpr int kDirs = kMlpDirs;

__device__ inline bool finite_d(double v) { return fabs(v) <= DBL_MAX; }

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// The sample: every point when n <= 4096, otherwise 16 blocks of 256
// consecutive points, block b starting at floor(b n / 16): 4096 points for
// any larger n, so the network reads histograms of one density whatever the
// set size (a 65,536-point set gives every 16th block of 256).  Sample
// position s maps to point (s >> 8) n / 16 + (s & 255).
__host__ __device__ inline int64_t sample_size(int64_t n) { return n < 4096 ? n : 4096; }

__device__ inline int64_t sample_point(int64_t s, int64_t n) {
    return n <= 4096 ? s : ((s >> 8) * n) / 16 + (s & 255);
}

__global__ __launch_bounds__(kHB) void k_sample_bbox(const double2* __restrict__ xy, int64_t n,
                                                     double* __restrict__ part,
                                                     uint32_t* __restrict__ hist) {
    __shared__ double s_v[4][kHB / 64];
    if (blockIdx.x == 0)
        for (int i = (int)threadIdx.x; i < kMlpIn; i += kHB) hist[i] = 0;
    double lo_x = INFINITY, lo_y = INFINITY, hi_x = -INFINITY, hi_y = -INFINITY;
    const int64_t slots = sample_size(n);
    for (int64_t s = (int64_t)blockIdx.x * kHB + threadIdx.x; s < slots; s += (int64_t)gridDim.x * kHB) {
        const int64_t i = sample_point(s, n);
        {
            const double2 p = xy[i];
            lo_x = fmin(lo_x, p.x);
            lo_y = fmin(lo_y, p.y);
            hi_x = fmax(hi_x, p.x);
            hi_y = fmax(hi_y, p.y);
        }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        lo_x = fmin(lo_x, __shfl_xor(lo_x, m));
        lo_y = fmin(lo_y, __shfl_xor(lo_y, m));
        hi_x = fmax(hi_x, __shfl_xor(hi_x, m));
        hi_y = fmax(hi_y, __shfl_xor(hi_y, m));
    }
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (lane == 0) {
        s_v[0][wave] = lo_x;
        s_v[1][wave] = lo_y;
        s_v[2][wave] = hi_x;
        s_v[3][wave] = hi_y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kHB / 64; ++w) {
            lo_x = fmin(lo_x, s_v[0][w]);
            lo_y = fmin(lo_y, s_v[1][w]);
            hi_x = fmax(hi_x, s_v[2][w]);
            hi_y = fmax(hi_y, s_v[3][w]);
        }
        part[4 * blockIdx.x + 0] = lo_x;
        part[4 * blockIdx.x + 1] = lo_y;
        part[4 * blockIdx.x + 2] = hi_x;
        part[4 * blockIdx.x + 3] = hi_y;
    }
}

__device__ inline int cell_of(double v, double lo, double sc) {
    const double c = floor((v - lo) * sc);
    if (!(c >= 0.0)) return 0;  // also catches NaN
    return c > 31.0 ? 31 : (int)c;
}

__global__ __launch_bounds__(kHB) void k_sample_hist(const double2* __restrict__ xy, int64_t n,
                                                     const double* __restrict__ part, int nparts,
                                                     uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[kMlpIn];
    __shared__ double s_box[4];
    __shared__ double s_v[4][kHB / 64];
    for (int i = (int)threadIdx.x; i < kMlpIn; i += kHB) s_h[i] = 0;
    {
        double lo_x = INFINITY, lo_y = INFINITY, hi_x = -INFINITY, hi_y = -INFINITY;
        for (int b = (int)threadIdx.x; b < nparts; b += kHB) {
            lo_x = fmin(lo_x, part[4 * b + 0]);
            lo_y = fmin(lo_y, part[4 * b + 1]);
            hi_x = fmax(hi_x, part[4 * b + 2]);
            hi_y = fmax(hi_y, part[4 * b + 3]);
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            lo_x = fmin(lo_x, __shfl_xor(lo_x, m));
            lo_y = fmin(lo_y, __shfl_xor(lo_y, m));
            hi_x = fmax(hi_x, __shfl_xor(hi_x, m));
            hi_y = fmax(hi_y, __shfl_xor(hi_y, m));
        }
        const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
        if (lane == 0) {
            s_v[0][wave] = lo_x;
            s_v[1][wave] = lo_y;
            s_v[2][wave] = hi_x;
            s_v[3][wave] = hi_y;
        }
        __syncthreads();
        if (threadIdx.x != 0) goto binned;
        for (int w = 1; w < kHB / 64; ++w) {
            lo_x = fmin(lo_x, s_v[0][w]);
            lo_y = fmin(lo_y, s_v[1][w]);
            hi_x = fmax(hi_x, s_v[2][w]);
            hi_y = fmax(hi_y, s_v[3][w]);
        }
        s_box[0] = lo_x;
        s_box[1] = lo_y;
        const double wx = hi_x - lo_x, wy = hi_y - lo_y;
        s_box[2] = wx > 0.0 ? 32.0 / wx : 0.0;
        s_box[3] = wy > 0.0 ? 32.0 / wy : 0.0;
    }
binned:
    __syncthreads();
    const double lo_x = s_box[0], lo_y = s_box[1], sx = s_box[2], sy = s_box[3];
    const int64_t slots = sample_size(n);
    for (int64_t s = (int64_t)blockIdx.x * kHB + threadIdx.x; s < slots; s += (int64_t)gridDim.x * kHB) {
        const int64_t i = sample_point(s, n);
        {
            const double2 p = xy[i];
            atomicAdd(&s_h[cell_of(p.y, lo_y, sy) * 32 + cell_of(p.x, lo_x, sx)], 1u);
        }
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < kMlpIn; i += kHB)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// Histogram counts -> the network's float inputs (count * 1024 / sample size).
__global__ void k_hist_to_x(const uint32_t* __restrict__ hist, int64_t n, float* __restrict__ x) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= kMlpIn) return;
    const int64_t ns = sample_size(n);
    x[i] = ns > 0 ? (float)((double)hist[i] * (1024.0 / (double)ns)) : 0.0f;
}

// One layer for rows of inputs (blockIdx.y = row): out = act(W in + b), one
// wave per output unit, lane l summing inputs 2l + 128k and 2l + 1 + 128k for
// k = 0, 1, ... in that order (one 4-byte load per pair of bfloat16 weights
// [out][in], layer input rounded to bfloat16, float32 sums).  act: ReLU then
// bfloat16 rounding (hidden layers), or none (the output layer).
constexpr int kMlpWaves = 4;  // output units per workgroup

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_layer(const float* __restrict__ in, int n_in,
                                                             const uint16_t* __restrict__ W,
                                                             const float* __restrict__ bias, int n_out,
                                                             int hidden, float* __restrict__ out) {
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    const int o = (int)blockIdx.x * kMlpWaves + wave;
    if (o >= n_out) return;
    const float* x = in + (size_t)blockIdx.y * n_in;
    const uint16_t* w = W + (size_t)o * n_in;
    float acc = 0.f;
    for (int i = 2 * lane; i < n_in; i += 128) {
        const uint32_t w2 = *reinterpret_cast<const uint32_t*>(w + i);  // inputs i, i + 1
        acc = fmaf(from_bf16(to_bf16(x[i])), from_bf16((uint16_t)(w2 & 0xFFFFu)), acc);
        acc = fmaf(from_bf16(to_bf16(x[i + 1])), from_bf16((uint16_t)(w2 >> 16)), acc);
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) {
        acc += bias[o];
        out[(size_t)blockIdx.y * n_out + o] = hidden ? from_bf16(to_bf16(fmaxf(acc, 0.f))) : acc;
    }
}

// The whole proposal in one workgroup of kFB threads: the sample's bounding
// box and histogram (as k_sample_bbox / k_sample_hist), the network inputs
// (as k_hist_to_x), the three layers (each output unit summed by one wave in
// the order of k_mlp_layer) and the directions, so the
// outputs equal those of the separate kernels bit for bit.
constexpr int kFB = 1024;

// out[o] = act(W[o] . in + b[o]) for every unit o (in, out in LDS): wave w
// takes the kU units o = w + 16 u, all their loads in flight together, each
// lane summing its inputs in the order k_mlp_layer does; the 64 lane sums of a
// unit are then added by a tree in LDS (s[l] += s[l + m], m = 32 .. 1) that
// associates them as k_mlp_layer's butterfly does for lane 0, so each output
// equals k_mlp_layer's bit for bit.  s_r: [kMlpHidden][64] floats.
template <int kIn, int kU>
__device__ inline void front_layer(const float* in, const uint16_t* __restrict__ W,
                                   const float* __restrict__ bias, bool hidden, float* out,
                                   float (*s_r)[64]) {
    constexpr int kOut = 16 * kU;
    const int t = (int)threadIdx.x, lane = (int)__lane_id(), wave = t >> 6;
    float acc[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) acc[u] = 0.f;
#pragma unroll 2
    for (int i = 2 * lane; i < kIn; i += 128) {
        const float x0 = from_bf16(to_bf16(in[i])), x1 = from_bf16(to_bf16(in[i + 1]));
        uint32_t w2[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            w2[u] = *reinterpret_cast<const uint32_t*>(W + (size_t)(wave + 16 * u) * kIn + i);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            acc[u] = fmaf(x0, from_bf16((uint16_t)(w2[u] & 0xFFFFu)), acc[u]);
            acc[u] = fmaf(x1, from_bf16((uint16_t)(w2[u] >> 16)), acc[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) s_r[wave + 16 * u][lane] = acc[u];
    __syncthreads();
    for (int m = 32; m > 0; m >>= 1) {
        for (int e = t; e < kOut * m; e += kFB) {
            const int o = e / m, l = e - o * m;
            s_r[o][l] = s_r[o][l] + s_r[o][l + m];
        }
        __syncthreads();
    }
    for (int o = t; o < kOut; o += kFB) {
        const float a = s_r[o][0] + bias[o];
        out[o] = hidden ? from_bf16(to_bf16(fmaxf(a, 0.f))) : a;
    }
}

__global__ __launch_bounds__(kFB) void k_front(const double2* __restrict__ xy, int64_t n, MlpDev W,
                                               LearnOut* __restrict__ lo) {
    constexpr int NW = kFB / 64;
    constexpr int PT = 4096 / kFB;  // sample points per thread
    __shared__ uint32_t s_h[kMlpIn];
    __shared__ float s_x[kMlpIn], s_h1[kMlpHidden], s_h2[kMlpHidden], s_y[kMlpOut];
    __shared__ float s_r[kMlpHidden][64];  // a layer's lane sums
    __shared__ double2 s_pt[4096];         // the sample, by sample position
    __shared__ double s_v[4][NW];
    __shared__ double s_box[4];
    const int t = (int)threadIdx.x;
    for (int i = t; i < kMlpIn; i += kFB) s_h[i] = 0;
    const int64_t ns = sample_size(n);
    double2 p[PT];
    double lo_x = INFINITY, lo_y = INFINITY, hi_x = -INFINITY, hi_y = -INFINITY;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int64_t sl = t + (int64_t)u * kFB;
        if (sl < ns) {
            p[u] = xy[sample_point(sl, n)];
            s_pt[sl] = p[u];
            lo_x = fmin(lo_x, p[u].x);
            lo_y = fmin(lo_y, p[u].y);
            hi_x = fmax(hi_x, p[u].x);
            hi_y = fmax(hi_y, p[u].y);
        }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        lo_x = fmin(lo_x, __shfl_xor(lo_x, m));
        lo_y = fmin(lo_y, __shfl_xor(lo_y, m));
        hi_x = fmax(hi_x, __shfl_xor(hi_x, m));
        hi_y = fmax(hi_y, __shfl_xor(hi_y, m));
    }
    const int lane = (int)__lane_id(), wave = t >> 6;
    if (lane == 0) {
        s_v[0][wave] = lo_x;
        s_v[1][wave] = lo_y;
        s_v[2][wave] = hi_x;
        s_v[3][wave] = hi_y;
    }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < NW; ++w) {
            lo_x = fmin(lo_x, s_v[0][w]);
            lo_y = fmin(lo_y, s_v[1][w]);
            hi_x = fmax(hi_x, s_v[2][w]);
            hi_y = fmax(hi_y, s_v[3][w]);
        }
        s_box[0] = lo_x;
        s_box[1] = lo_y;
        const double wx = hi_x - lo_x, wy = hi_y - lo_y;
        s_box[2] = wx > 0.0 ? 32.0 / wx : 0.0;
        s_box[3] = wy > 0.0 ? 32.0 / wy : 0.0;
    }
    __syncthreads();
    {
        const double bx = s_box[0], by = s_box[1], sx = s_box[2], sy = s_box[3];
#pragma unroll
        for (int u = 0; u < PT; ++u)
            if (t + (int64_t)u * kFB < ns) atomicAdd(&s_h[cell_of(p[u].y, by, sy) * 32 + cell_of(p[u].x, bx, sx)], 1u);
    }
    __syncthreads();
    for (int i = t; i < kMlpIn; i += kFB)
        s_x[i] = ns > 0 ? (float)((double)s_h[i] * (1024.0 / (double)ns)) : 0.0f;
    __syncthreads();
    static_assert(kFB / 64 == 16 && kMlpHidden % 16 == 0 && kMlpOut % 16 == 0, "16 waves");
    front_layer<kMlpIn, kMlpHidden / 16>(s_x, W.w1, W.b1, true, s_h1, s_r);
    __syncthreads();
    front_layer<kMlpHidden, kMlpHidden / 16>(s_h1, W.w2, W.b2, true, s_h2, s_r);
    __syncthreads();
    front_layer<kMlpHidden, kMlpOut / 16>(s_h2, W.w3, W.b3, false, s_y, s_r);
    __syncthreads();
    __shared__ double s_u[2 * kDirs];
    if (t < kDirs) {
        double ux = (double)s_y[2 * t], uy = (double)s_y[2 * t + 1];
        if (!finite_d(ux) || !finite_d(uy) || (ux == 0.0 && uy == 0.0)) {
            const double a = 6.283185307179586 * (double)t / (double)kDirs;
            ux = cos(a);
            uy = sin(a);
        }
        s_u[2 * t] = ux;
        s_u[2 * t + 1] = uy;
    }
    __syncthreads();
    // the sample point farthest along each direction (fma(x, ux, y * uy),
    // ties: smallest index, that is smallest sample position): wave d takes
    // direction d, lane l the positions l, l + 64, ... (consecutive lanes,
    // consecutive LDS words)
    __shared__ int32_t s_c[kDirs];
    static_assert(NW == kDirs, "wave d: direction d");
    {
        const int d = wave;
        const double ux = s_u[2 * d], uy = s_u[2 * d + 1];
        double bv = -INFINITY;
        int32_t bs = INT32_MAX;
#pragma unroll 8
        for (int sl = lane; sl < (int)ns; sl += 64) {
            const double2 q = s_pt[sl];
            const double v = fma(q.x, ux, q.y * uy);
            const bool tk = v > bv;
            bv = tk ? v : bv;
            bs = tk ? sl : bs;
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double ov = __shfl_xor(bv, m);
            const int32_t os = __shfl_xor(bs, m);
            dir_take(bv, bs, ov, os);
        }
        if (lane == 0) s_c[d] = bs;
    }
    __syncthreads();
    // the hull of the direction candidates alone: the final discard polygon
    // (their hull with the Step-1 extremes) contains it, so the Step-1 pass
    // can already drop the points strictly inside it
    __shared__ double s_cx[kDirs], s_cy[kDirs];
    __shared__ int32_t s_cu[kDirs];
    __shared__ Poly s_sp;
    if (t < kDirs) {
        const int32_t sl = s_c[t];
        const double2 q = sl == INT32_MAX ? make_double2(0.0, 0.0) : s_pt[sl];
        s_cx[t] = q.x;
        s_cy[t] = q.y;
        s_cu[t] = sl != INT32_MAX && finite_d(q.x) && finite_d(q.y);
    }
    __syncthreads();
    hull_of_points<kDirs>(s_cx, s_cy, s_cu, s_sp);
    // every global store at the end: a barrier waits for outstanding stores
    static_assert(sizeof(Poly) % 8 == 0, "double copies");
    for (int i = t; i < (int)(sizeof(Poly) / 8); i += kFB)
        reinterpret_cast<double*>(&lo->spoly)[i] = reinterpret_cast<const double*>(&s_sp)[i];
    if (t < kMlpOut) lo->y[t] = s_y[t];
    if (t >= 64 && t < 64 + 2 * kDirs) lo->dirs[t - 64] = s_u[t - 64];
    if (t >= 128 && t < 128 + kDirs) {
        const int d = t - 128;
        const int32_t sl = s_c[d];
        lo->cand[4 + d] = sl == INT32_MAX ? INT32_MAX : (int32_t)sample_point(sl, n);
        const double2 q = sl == INT32_MAX ? make_double2(0.0, 0.0) : s_pt[sl];
        lo->cxy[2 * d] = q.x;
        lo->cxy[2 * d + 1] = q.y;
    }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
constexpr int kGT = 64;   // output tile (rows and columns)
constexpr int kGK = 16;   // depth per step

// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (then ReLU, or times (mask[m][n] > 0)),
// A(m,k) = tA ? A[k*lda + m] : A[m*lda + k], B(k,n) = tB ? B[n*ldb + k] : B[k*ldb + n].
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              int tA, const float* __restrict__ B, int ldb, int tB,
                                              const float* __restrict__ bias, int relu,
                                              const float* __restrict__ mask, float* __restrict__ C,
                                              int ldc) {
    __shared__ float s_a[kGK][kGT + 1];
    __shared__ float s_b[kGK][kGT + 1];
    const int t = (int)threadIdx.x;
    const int tm = (t >> 4) * 4, tn = (t & 15) * 4;
    const int m0 = (int)blockIdx.y * kGT, n0 = (int)blockIdx.x * kGT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += kGK) {
        for (int e = t; e < kGK * kGT; e += 256) {
            const int kk = e / kGT, r = e % kGT;
            const int m = m0 + r, n = n0 + r, k = k0 + kk;
            s_a[kk][r] = (m < M && k < K) ? (tA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]) : 0.f;
            s_b[kk][r] = (n < N && k < K) ? (tB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = s_a[kk][tm + i];
                b[i] = s_b[kk][tn + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + tm + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tn + j;
            if (n >= N) continue;
            float v = acc[i][j];
            if (bias) v += bias[n];
            if (relu) v = fmaxf(v, 0.f);
            if (mask && !(mask[(size_t)m * ldc + n] > 0.f)) v = 0.f;
            C[(size_t)m * ldc + n] = v;
        }
    }
}

// d = 2 (y - t) / count and the loss sum (one workgroup).
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ y, const float* __restrict__ tg,
                                              int count, float* __restrict__ d,
                                              float* __restrict__ loss) {
    __shared__ double s_w[16];
    double acc = 0.0;
    for (int i = (int)threadIdx.x; i < count; i += 1024) {
        const float e = y[i] - tg[i];
        d[i] = 2.f * e / (float)count;
        acc += (double)e * (double)e;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
    if (lane == 0) s_w[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += s_w[w];
        *loss = (float)(s / (double)count);
    }
}

// out[n] = sum_m d[m][n]
__global__ void k_colsum(const float* __restrict__ d, int M, int N, float* __restrict__ out) {
    const int n = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += d[(size_t)m * N + n];
    out[n] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// master float32 -> bfloat16 (same [out][in] layout)
__global__ void k_to_bf16(const float* __restrict__ w, int64_t count, uint16_t* __restrict__ wb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) wb[e] = to_bf16(w[e]);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int learned_grid(int64_t n, int cu_count) {
    const int64_t g = (sample_size(n) + kHB - 1) / kHB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cu_count));
}

hipError_t launch_histogram_sample(const double* xy, int64_t n, double* part, int grid, uint32_t* hist,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_sample_bbox, dim3(grid), dim3(kHB), 0, s, reinterpret_cast<const double2*>(xy),
                       n, part, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sample_hist, dim3(grid), dim3(kHB), 0, s, reinterpret_cast<const double2*>(xy),
                       n, part, grid, hist);
    return hipGetLastError();
}

hipError_t launch_hist_to_x(const uint32_t* hist, int64_t n, float* x, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_to_x, dim3(kMlpIn / 256), dim3(256), 0, s, hist, n, x);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* x, int rows, const MlpDev& W, float* h1, float* h2, float* y,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_layer, dim3(kMlpHidden / kMlpWaves, rows), dim3(64 * kMlpWaves), 0, s, x,
                       kMlpIn, W.w1, W.b1, kMlpHidden, 1, h1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_layer, dim3(kMlpHidden / kMlpWaves, rows), dim3(64 * kMlpWaves), 0, s, h1,
                       kMlpHidden, W.w2, W.b2, kMlpHidden, 1, h2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_layer, dim3(kMlpOut / kMlpWaves, rows), dim3(64 * kMlpWaves), 0, s, h2,
                       kMlpHidden, W.w3, W.b3, kMlpOut, 0, y);
    return hipGetLastError();
}

hipError_t launch_front(const double* xy, int64_t n, const MlpDev& W, LearnOut* lo, hipStream_t s) {
    hipLaunchKernelGGL(k_front, dim3(1), dim3(kFB), 0, s, reinterpret_cast<const double2*>(xy), n, W, lo);
    return hipGetLastError();
}



hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int tA, const float* B, int ldb,
                       int tB, const float* bias, int relu, const float* mask, float* C, int ldc,
                       hipStream_t s) {
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, lda, tA, B, ldb, tB, bias, relu, mask, C, ldc);
    return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, int count, float* d, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, y, t, count, d, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, d, M, N, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, g, m, v, count,
                       lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* w, int64_t count, uint16_t* wb, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, w, count, wb);
    return hipGetLastError();
}

}  // namespace hx
