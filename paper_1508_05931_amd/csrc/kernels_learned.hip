// kernels_learned.hip - the learned-filter variant of Steps 1-2 (not in the
// paper) and the training kernels of its network.
//
// Proposal (per hull, before the first round):
//   k_sample_bbox, k_sample_hist  32 x 32 occupancy histogram of a sample
//                                 (16 evenly spaced blocks of 256 points)
//                                 over the sample's bounding box
//   k_mlp_layer ×3, k_mlp_dirs    1024 -> 256 -> 256 -> 32 network, bfloat16
//                                 weights and layer inputs, float32 sums, one
//                                 wave per output unit: 16 directions
//   k_extremes<16>, k_poly        the point farthest along each direction
//                                 (fma(x, ux, y * uy), ties: smallest index;
//                                 in the same pass as Step 1), and the exact
//                                 convex hull of those 16
//                                 points and the four Step-1 extremes: the
//                                 discard polygon, which contains the
//                                 quadrilateral, so the first round stays
//                                 conservative whatever the network says
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
// wave per output unit, each lane summing every 64th input (bfloat16 weights
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
    for (int i = lane; i < n_in; i += 64) acc = fmaf(from_bf16(to_bf16(x[i])), from_bf16(w[i]), acc);
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) {
        acc += bias[o];
        out[(size_t)blockIdx.y * n_out + o] = hidden ? from_bf16(to_bf16(fmaxf(acc, 0.f))) : acc;
    }
}

// The 16 directions of one row of outputs (non-finite or zero: the evenly
// spaced direction of that slot).
__global__ void k_mlp_dirs(const float* __restrict__ y, LearnOut* __restrict__ lo) {
    const int t = (int)threadIdx.x;
    if (t >= kDirs) return;
    double ux = (double)y[2 * t], uy = (double)y[2 * t + 1];
    if (!finite_d(ux) || !finite_d(uy) || (ux == 0.0 && uy == 0.0)) {
        const double a = 6.283185307179586 * (double)t / (double)kDirs;
        ux = cos(a);
        uy = sin(a);
    }
    lo->y[2 * t] = y[2 * t];
    lo->y[2 * t + 1] = y[2 * t + 1];
    lo->dirs[2 * t] = ux;
    lo->dirs[2 * t + 1] = uy;
}


// The candidates and their exact convex hull (Andrew's monotone chain on at
// most 20 points, one thread): the discard polygon.
__global__ __launch_bounds__(64 * kDirs) void k_poly(const DirBest* __restrict__ part, int nparts,
                                                    const double2* __restrict__ xy,
                                                    const Params* __restrict__ prm,
                                                    LearnOut* __restrict__ lo) {
    __shared__ int32_t s_c[kPolyMax];
    const int t = (int)threadIdx.x;
    {
        // wave j reduces direction j over the block partials
        const int lane = (int)__lane_id(), j = t >> 6;
        double v = -INFINITY;
        int32_t i = INT32_MAX;
        for (int b = lane; b < nparts; b += 64) dir_take(v, i, part[(size_t)b * kDirs + j].v, part[(size_t)b * kDirs + j].i);
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            const double ov = __shfl_xor(v, m);
            const int32_t oi = __shfl_xor(i, m);
            dir_take(v, i, ov, oi);
        }
        if (lane == 0) s_c[4 + j] = i;
    }
    if (t < 4) s_c[t] = prm->ext[t].i;
    __syncthreads();
    // the candidates' coordinates, loaded in parallel
    __shared__ double s_x[kPolyMax], s_y[kPolyMax];
    if (t < kPolyMax && s_c[t] != INT32_MAX) {
        const double2 p = xy[s_c[t]];
        s_x[t] = p.x;
        s_y[t] = p.y;
    }
    __syncthreads();
    // one thread builds the hull with its arrays in LDS (no scratch), then
    // every thread copies the polygon out
    __shared__ Poly Q;
    __shared__ double cx[kPolyMax], cy[kPolyMax], hx_[2 * kPolyMax + 1], hy_[2 * kPolyMax + 1];
    if (t == 0) {
        Q.pad = 0;
        Q.nv = 0;
        int nc = 0;
        const bool ok = prm->flags == 0u;
        for (int j = 0; j < kPolyMax; ++j) {
            lo->cand[j] = s_c[j];
            if (!ok || s_c[j] == INT32_MAX) continue;
            const double px = s_x[j], py = s_y[j];
            // insertion by (x, y), dropping repeats
            bool dup = false;
            for (int a = 0; a < nc; ++a) dup |= (cx[a] == px && cy[a] == py);
            if (dup) continue;
            int k = nc;
            while (k > 0 && (cx[k - 1] > px || (cx[k - 1] == px && cy[k - 1] > py))) {
                cx[k] = cx[k - 1];
                cy[k] = cy[k - 1];
                --k;
            }
            cx[k] = px;
            cy[k] = py;
            ++nc;
        }
        int h = 0;
        if (nc >= 3) {
            for (int i = 0; i < nc; ++i) {
                while (h >= 2 && orient(hx_[h - 2], hy_[h - 2], hx_[h - 1], hy_[h - 1], cx[i], cy[i]) <= 0) --h;
                hx_[h] = cx[i];
                hy_[h] = cy[i];
                ++h;
            }
            const int base = h;
            for (int i = nc - 2; i >= 0; --i) {
                while (h > base && orient(hx_[h - 2], hy_[h - 2], hx_[h - 1], hy_[h - 1], cx[i], cy[i]) <= 0) --h;
                hx_[h] = cx[i];
                hy_[h] = cy[i];
                ++h;
            }
            --h;  // the last point repeats the first
        }
        Q.nv = h >= 3 ? h : 0;
        // every corner and point lies in the Step-1 bounding box W x H
        const double W = prm->ext[2].x - prm->ext[0].x, H = prm->ext[3].y - prm->ext[1].y;
        Q.qb = 9.0 * kEps * W * H;
    }
    __syncthreads();
    if (t < kPolyMax) {
        const int nv = Q.nv, j = t;
        const int j1 = j + 1 < nv ? j + 1 : 0;
        Q.px[j] = j < nv ? hx_[j] : 0.0;
        Q.py[j] = j < nv ? hy_[j] : 0.0;
        Q.ex[j] = j < nv ? hx_[j1] - hx_[j] : 0.0;
        Q.ey[j] = j < nv ? hy_[j1] - hy_[j] : 0.0;
    }
    __syncthreads();
    static_assert(sizeof(Poly) % 8 == 0, "double copies");
    for (int i = t; i < (int)(sizeof(Poly) / 8); i += (int)blockDim.x)
        reinterpret_cast<double*>(&lo->poly)[i] = reinterpret_cast<const double*>(&Q)[i];
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
                            LearnOut* lo, hipStream_t s) {
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
    e = hipGetLastError();
    if (e != hipSuccess || !lo) return e;
    hipLaunchKernelGGL(k_mlp_dirs, dim3(1), dim3(64), 0, s, y, lo);
    return hipGetLastError();
}

hipError_t launch_poly(const double* xy, const Params* prm, LearnOut* lo, const DirBest* dpart,
                       int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_poly, dim3(1), dim3(64 * kDirs), 0, s, dpart, grid,
                       reinterpret_cast<const double2*>(xy), prm, lo);
    return hipGetLastError();
}

size_t dir_part_bytes(int grid) { return (size_t)grid * kDirs * sizeof(DirBest); }

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
