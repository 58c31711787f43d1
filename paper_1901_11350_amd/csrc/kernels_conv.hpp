// kernels_conv.hpp -- BF16 matrix-core (MFMA) kernels of the learned
// dipole-field surrogate: a stack of zero-padded 3x3 convolutions with SiLU
// between layers, trained by its own forward/backward kernels and Adam.
//
// Layout: activations NHWC with the channel dimension padded to 32
// (x[b][y][x][32] bf16); weights in "kernel layout" wk[tap][n][k] bf16
// (tap = 3 ky + kx, n = output channel, k = input channel), master weights
// w[tap][ci][co] FP32 with Adam moments beside them.  Padded channels hold
// zeros and receive zero gradients.
//
// Contract (mirrored by the FP64 oracle): activations, weights and
// back-propagated gradients are rounded to bf16 before they are multiplied;
// products are accumulated in FP32 by v_mfma_f32_16x16x32_bf16 (16 pixels x
// 16 channels x 32 input channels per instruction).
//
// A convolution is an implicit GEMM: M = pixels, N = output channels,
// K = 9 taps x 32 input channels.  A 256-thread workgroup owns a 16 x 16
// pixel tile; the tile plus its 1-pixel halo (zero outside the image) and
// all weights sit in LDS; each of the 4 wavefronts computes 4 rows of 16
// pixels for all 32 output channels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCP = 32;      // padded channels
constexpr int kTile = 16;    // tile side (pixels)
constexpr int kHalo = kTile + 2;

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

enum { CONV_SILU = 0, CONV_LINEAR = 1, CONV_SILU_NOZ = 2 };

// One 3x3 convolution layer (or the dgrad of one, with tap-flipped weights).
//   MODE CONV_SILU:     z (FP32) and y = bf16(silu(z))
//   MODE CONV_LINEAR:   z (FP32) only
//   MODE CONV_SILU_NOZ: y only (inference)
// TR: tile rows (16, or 4 for small grids: four times the workgroups, one
// row per wavefront); per accumulator the taps and instructions are the
// same, so both give the same bits.
template <int MODE, int TR = kTile>
__global__ void __launch_bounds__(256) k_conv3x3(int H, int W, const __bf16* __restrict__ x,
                                                 const __bf16* __restrict__ wk, const float* __restrict__ bias,
                                                 float* __restrict__ z, __bf16* __restrict__ y) {
    static_assert(TR % 4 == 0 && TR <= kTile, "four wavefronts of whole rows");
    constexpr int RPW = TR / 4;   // rows per wavefront
    __shared__ __attribute__((aligned(16))) __bf16 sX[(TR + 2) * kHalo * kCP];
    __shared__ __attribute__((aligned(16))) __bf16 sW[9 * kCP * kCP];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * TR;
    const int tid = threadIdx.x;
    // weights: 9*32*32 bf16 = 1152 vectors of 8
    for (int v = tid; v < 9 * kCP * kCP / 8; v += 256)
        reinterpret_cast<bf16x8*>(sW)[v] = reinterpret_cast<const bf16x8*>(wk)[v];
    // input tile with halo: (TR+2) x 18 pixels x 4 vectors of 8 channels
    for (int v = tid; v < (TR + 2) * kHalo * 4; v += 256) {
        const int p = v >> 2, q = v & 3;
        const int hy = p / kHalo, hx = p - hy * kHalo;
        const int gy = y0 + hy - 1, gx = x0 + hx - 1;
        bf16x8 val;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            val = reinterpret_cast<const bf16x8*>(x + (((size_t)b * H + gy) * W + gx) * kCP)[q];
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) val[j] = (__bf16)0.0f;
        }
        reinterpret_cast<bf16x8*>(sX)[v] = val;
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int lm = lane & 15, lk = lane >> 4;   // fragment row/col, k group
    f32x4 acc[RPW][2];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[r][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        bf16x8 bw[2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            bw[nb] = *reinterpret_cast<const bf16x8*>(sW + (tap * kCP + lm + 16 * nb) * kCP + 8 * lk);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int row = wave * RPW + r;
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(sX + ((row + ky) * kHalo + lm + kx) * kCP + 8 * lk);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[nb], acc[r][nb], 0, 0, 0);
        }
    }
    // D fragment: lane holds pixels 4*lk + j (j = 0..3) of the row, channel lm + 16 nb
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int gy = y0 + wave * RPW + r;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int c = lm + 16 * nb;
            const float bc = bias ? bias[c] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int gx = x0 + 4 * lk + j;
                const size_t o = (((size_t)b * H + gy) * W + gx) * kCP + c;
                const float v = acc[r][nb][j] + bc;
                if (MODE != CONV_SILU_NOZ) z[o] = v;
                if (MODE != CONV_LINEAR) y[o] = (__bf16)silu_f(v);
            }
        }
    }
}

// Weight gradient (split over pixel tiles) and bias gradient of one layer:
// dw[tap][ci][co] = sum_pixels x[p + tap offset][ci] dz[p][co], db[co] = sum dz[p][co].
// Each workgroup writes the partial sums of its 16x16 tile (9*32*32 + 32 floats).
__global__ void __launch_bounds__(256) k_conv3x3_wgrad(int H, int W, const __bf16* __restrict__ x,
                                                       const __bf16* __restrict__ dz, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) __bf16 sXc[kCP * kHalo * kHalo];   // channel-major, halo tile
    __shared__ __attribute__((aligned(16))) __bf16 sDc[kCP * kTile * kTile];   // channel-major, tile
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    const int tid = threadIdx.x;
    for (int v = tid; v < kHalo * kHalo * kCP; v += 256) {
        const int p = v / kCP, c = v - p * kCP;
        const int hy = p / kHalo, hx = p - hy * kHalo;
        const int gy = y0 + hy - 1, gx = x0 + hx - 1;
        __bf16 val = (__bf16)0.0f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) val = x[(((size_t)b * H + gy) * W + gx) * kCP + c];
        sXc[c * kHalo * kHalo + p] = val;
    }
    for (int v = tid; v < kTile * kTile * kCP; v += 256) {
        const int p = v / kCP, c = v - p * kCP;
        const int ty = p / kTile, tx = p - ty * kTile;
        sDc[c * kTile * kTile + p] = dz[(((size_t)b * H + y0 + ty) * W + x0 + tx) * kCP + c];
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int lm = lane & 15, lk = lane >> 4;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    const int blk = (b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* out = part + (size_t)blk * (9 * kCP * kCP + kCP);
    // taps of this wave: wave, wave+4, wave+8
    for (int tap = wave; tap < 9; tap += 4) {
        const int ky = tap / 3, kx = tap - 3 * (tap / 3);
        f32x4 acc[2][2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        // K = 256 tile pixels in blocks of 32 (two rows); lane group lk takes pixels 8*lk..8*lk+7
        for (int kb = 0; kb < 8; ++kb) {
            const int row = 2 * kb + (lk >> 1);
            const int xs = 8 * (lk & 1);
            bf16x8 bfr[2], afr[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                bfr[nb] = *reinterpret_cast<const bf16x8*>(sDc + (lm + 16 * nb) * kTile * kTile + row * kTile + xs);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const __bf16* src = sXc + (lm + 16 * mb) * kHalo * kHalo + (row + ky) * kHalo + xs + kx;
#pragma unroll
                for (int j = 0; j < 8; ++j) afr[mb][j] = src[j];
            }
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[mb], bfr[nb], acc[mb][nb], 0, 0, 0);
        }
        // D: rows = ci (4*lk + j + 16 mb), cols = co (lm + 16 nb)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    out[(tap * kCP + 4 * lk + j + 16 * mb) * kCP + lm + 16 * nb] = acc[mb][nb][j];
    }
    if (tid < kCP) {
        float s = 0.0f;
        for (int p = 0; p < kTile * kTile; ++p) s += (float)sDc[tid * kTile * kTile + p];
        out[9 * kCP * kCP + tid] = s;
    }
    (void)nblk;
}

// Fixed-order sum of per-tile partials: out[k] = sum_p part[p][k].
// Sum of n_parts rows of length len, in two fixed-order stages: group g
// (blockIdx.y) of k_sum_partials_stage adds rows [g*chunk, (g+1)*chunk) into
// stage[g]; k_sum_partials then adds the groups in order.
__global__ void __launch_bounds__(256) k_sum_partials_stage(int n_parts, int len, int chunk,
                                                            const float* __restrict__ part,
                                                            float* __restrict__ stage) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= len) return;
    const int p0 = blockIdx.y * chunk, p1 = min(n_parts, p0 + chunk);
    float s = 0.0f;
    for (int p = p0; p < p1; ++p) s += part[(size_t)p * len + k];
    stage[(size_t)blockIdx.y * len + k] = s;
}

__global__ void __launch_bounds__(256) k_sum_partials(int n_parts, int len, const float* __restrict__ part,
                                                      float* __restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= len) return;
    float s = 0.0f;
    for (int p = 0; p < n_parts; ++p) s += part[(size_t)p * len + k];
    out[k] = s;
}

// dz_prev = bf16(dx * silu'(z_prev)) for the layer below.
__global__ void __launch_bounds__(256) k_silu_backward(int64_t n, const float* __restrict__ dx,
                                                       const float* __restrict__ zprev, __bf16* __restrict__ dz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    dz[i] = (__bf16)(dx[i] * silu_grad_f(zprev[i]));
}

// Loss sum_b |y_b - t_b|^2 / |t_b|^2 over the first n_out channels: gradient
// dz = 2 (y - t) / |t_b|^2 (bf16) and per-block loss partials (FP64).
__global__ void __launch_bounds__(256) k_loss_grad(int64_t pix_per_sample, int n_out, const float* __restrict__ yout,
                                                   const float* __restrict__ target, const double* __restrict__ tnorm2,
                                                   __bf16* __restrict__ dz, double* __restrict__ loss_part) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;   // pixel over the batch
    const int b = (int)(blockIdx.x * 256 / pix_per_sample);
    double l = 0.0;
    const double inv = 1.0 / tnorm2[b];
    for (int c = 0; c < kCP; ++c) {
        const size_t o = (size_t)p * kCP + c;
        float g = 0.0f;
        if (c < n_out) {
            const float d = yout[o] - target[(size_t)p * n_out + c];
            l += (double)d * d * inv;
            g = (float)(2.0 * d * inv);
        }
        dz[o] = (__bf16)g;
    }
    // block sum
    __shared__ double red[256];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam on the FP32 master parameters (Kingma and Ba); c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void __launch_bounds__(256) k_adam(int n, float* __restrict__ p, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Kernel-layout bf16 weights from the FP32 master w[tap][ci][co]:
// forward wf[tap][co][ci] = w[tap][ci][co]; dgrad wb[tap][ci][co] = w[8 - tap][ci][co].
__global__ void __launch_bounds__(256) k_prep_weights(const float* __restrict__ w, __bf16* __restrict__ wf,
                                                      __bf16* __restrict__ wb) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= 9 * kCP * kCP) return;
    const int tap = k / (kCP * kCP), r = k - tap * kCP * kCP;
    const int ci = r / kCP, co = r - ci * kCP;
    wf[(tap * kCP + co) * kCP + ci] = (__bf16)w[k];
    if (wb) wb[((8 - tap) * kCP + ci) * kCP + co] = (__bf16)w[k];
}

// Spins of a film (SoA, N = H*W*L sites, site = x + W*(y + H*layer)) to the
// network input x[b][y][x][c], c = 3*layer + component (bf16, zero padded).
template <typename T>
__global__ void __launch_bounds__(256) k_spins_to_nhwc(int H, int W, int L, const T* __restrict__ n,
                                                       __bf16* __restrict__ x, int64_t stride_n, int b0) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;   // pixel within sample
    const int b = blockIdx.y;
    if (t >= (int64_t)H * W) return;
    const T* nb = n + (size_t)b * stride_n;
    const int64_t N = (int64_t)H * W * L;
    __bf16* o = x + ((size_t)(b0 + b) * H * W + t) * kCP;
    for (int c = 0; c < kCP; ++c) {
        float v = 0.0f;
        if (c < 3 * L) {
            const int layer = c / 3, comp = c - 3 * layer;
            v = (float)nb[(size_t)comp * N + (size_t)layer * H * W + t];
        }
        o[c] = (__bf16)v;
    }
}

// Network output y[b][y][x][c] (FP32) to the dipole gradient of the film,
// g[comp][site] = scale * y[c = 3*layer + comp].
template <typename T>
__global__ void __launch_bounds__(256) k_nhwc_to_field(int H, int W, int L, const float* __restrict__ y, float scale,
                                                       T* __restrict__ g) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)H * W) return;
    const int64_t N = (int64_t)H * W * L;
    for (int c = 0; c < 3 * L; ++c) {
        const int layer = c / 3, comp = c - 3 * layer;
        g[(size_t)comp * N + (size_t)layer * H * W + t] = (T)(scale * y[t * kCP + c]);
    }
}

// Dipole gradient of a film (SoA, meV) to the training target
// t[b][y][x][c] = g[comp][layer*H*W + pixel] / scale, c = 3*layer + comp.
template <typename T>
__global__ void __launch_bounds__(256) k_field_to_target(int H, int W, int L, const T* __restrict__ g, float inv_scale,
                                                         float* __restrict__ t, int64_t stride_g, int b0) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (p >= (int64_t)H * W) return;
    const T* gb = g + (size_t)b * stride_g;
    const int64_t N = (int64_t)H * W * L;
    float* o = t + ((size_t)(b0 + b) * H * W + p) * (3 * L);
    for (int c = 0; c < 3 * L; ++c) {
        const int layer = c / 3, comp = c - 3 * layer;
        o[c] = inv_scale * (float)gb[(size_t)comp * N + (size_t)layer * H * W + p];
    }
}

// |t_b|^2 of each sample (one workgroup per sample, FP64 tree).
// Squared norm of each sample (blockIdx.y) of length len: block x of
// kNormChunks adds its contiguous chunk (FP64, fixed-order tree) into
// part[sample * kNormChunks + x]; k_sample_norm2_final adds the chunks in order.
constexpr int kNormChunks = 64;
__global__ void __launch_bounds__(256) k_sample_norm2(int64_t len, const float* __restrict__ t,
                                                      double* __restrict__ part) {
    const int64_t chunk = (len + kNormChunks - 1) / kNormChunks;
    const int64_t k0 = (int64_t)blockIdx.x * chunk, k1 = k0 + chunk < len ? k0 + chunk : len;
    const float* tb = t + (size_t)blockIdx.y * len;
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += (double)tb[k] * tb[k];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * kNormChunks + blockIdx.x] = red[0];
}

__global__ void k_sample_norm2_final(int B, const double* __restrict__ part, double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int k = 0; k < kNormChunks; ++k) s += part[(size_t)b * kNormChunks + k];
    out[b] = s;
}

constexpr int kSitesPerGroup = 4;
constexpr int kSiteSlices = 16;

// Residual check of a surrogate field at sampled sites: relative error
// |g_s - exact_s| / |exact_s| over the samples; *need = (error > tol).
// exact_s = scale * (sum of the kSiteSlices slice sums of
// k_dipole_at_sites_part, in slice order).
// stats: [evaluations, fallbacks, last error, max error].
// Sampled sites are offset + s * stride, s < n_sites.
// One workgroup of 256 threads; thread t covers samples t, t + 256, ...; the
// sums are reduced in a fixed-order tree.
template <typename T>
__global__ void __launch_bounds__(256) k_surrogate_check(int N, int n_sites, int offset, int stride,
                                                         const double* __restrict__ part, double scale,
                                                         const T* __restrict__ g, double tol,
                                                         int* __restrict__ need, double* __restrict__ stats) {
    double num = 0.0, den = 0.0;
    for (int s = threadIdx.x; s < n_sites; s += 256) {
        const int i = offset + s * stride;
        double v[kSiteSlices * 3];   // every slice sum of the site in flight at once
#pragma unroll
        for (int k = 0; k < kSiteSlices * 3; ++k) v[k] = part[(size_t)s * kSiteSlices * 3 + k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kSiteSlices; ++k) t += v[3 * k + c];
            const double ex = scale * t;
            const double d = (double)g[(size_t)c * N + i] - ex;
            num += d * d;
            den += ex * ex;
        }
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = num;
    red[1][threadIdx.x] = den;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[0][threadIdx.x] += red[0][threadIdx.x + st];
            red[1][threadIdx.x] += red[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    num = red[0][0];
    den = red[1][0];
    const double err = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? 1e300 : 0.0);
    const int f = (err > tol || !(err == err)) ? 1 : 0;
    *need = f;
    stats[0] += 1.0;
    stats[1] += (double)f;
    stats[2] = err;
    stats[3] = fmax(stats[3], err);
}

// Exact dipole gradient (direct sum over all sources, in units of C_dd mu^2) at the n_sites
// target sites offset + s * stride, the reference of the surrogate's
// residual check: workgroup (g, k) takes the
// kSitesPerGroup sites of group g and the k-th of kSiteSlices source
// slices, so each source read serves every site of the group; each thread
// accumulates its sources in FP32, the workgroup adds the per-thread sums
// in FP64 (fixed-order tree) into part[(site * kSiteSlices + k) * 3 + c],
// and the check adds the slices in order.

template <typename T>
__global__ void __launch_bounds__(256) k_dipole_at_sites_part(int N, const T* __restrict__ pos,
                                                               const T* __restrict__ n, int offset, int stride,
                                                               int n_sites, double* __restrict__ part) {
    const int g = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
    T px[kSitesPerGroup], py[kSitesPerGroup], pz[kSitesPerGroup];
    T acc[kSitesPerGroup][3];
#pragma unroll
    for (int q = 0; q < kSitesPerGroup; ++q) {
        const int s = min(g * kSitesPerGroup + q, n_sites - 1);
        const int i = offset + s * stride;
        px[q] = pos[i];
        py[q] = pos[N + i];
        pz[q] = pos[2 * N + i];
        acc[q][0] = acc[q][1] = acc[q][2] = T(0);
    }
    const int j0 = (int)((long long)N * k / kSiteSlices), j1 = (int)((long long)N * (k + 1) / kSiteSlices);
    for (int j = j0 + tid; j < j1; j += 256) {
        const T sx = pos[j], sy = pos[N + j], sz = pos[2 * N + j];
        const T mx = n[j], my = n[N + j], mz = n[2 * N + j];
#pragma unroll
        for (int q = 0; q < kSitesPerGroup; ++q) {
            const T rx = sx - px[q], ry = sy - py[q], rz = sz - pz[q];
            const T d2 = rx * rx + ry * ry + rz * rz;
            T inv;
            if constexpr (sizeof(T) == 4) {
                inv = d2 > T(0) ? __builtin_amdgcn_rsqf(d2) : T(0);
            } else {
                inv = d2 > T(0) ? T(1) / sqrt(d2) : T(0);
            }
            const T inv3 = inv * inv * inv;
            const T sdot = T(3) * (mx * rx + my * ry + mz * rz) * inv * inv;
            acc[q][0] += (mx - sdot * rx) * inv3;
            acc[q][1] += (my - sdot * ry) * inv3;
            acc[q][2] += (mz - sdot * rz) * inv3;
        }
    }
    __shared__ double red[kSitesPerGroup * 3][256];
#pragma unroll
    for (int q = 0; q < kSitesPerGroup; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) red[3 * q + c][tid] = (double)acc[q][c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st)
            for (int v = 0; v < kSitesPerGroup * 3; ++v) red[v][tid] += red[v][tid + st];
        __syncthreads();
    }
    if (tid < kSitesPerGroup * 3) {
        const int s = g * kSitesPerGroup + tid / 3;
        if (s < n_sites) part[((size_t)s * kSiteSlices + k) * 3 + tid % 3] = red[tid][0];
    }
}

}  // namespace sp
