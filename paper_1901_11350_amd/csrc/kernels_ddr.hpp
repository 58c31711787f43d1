// kernels_ddr.hpp -- residual form of the learned dipole field (not in the
// paper; a stand-in for its costliest term, the dipolar sum of Sec. III.A).
//
// The film (one-atom simple cubic, NA x NB cells, NC layers, lattice
// constant a) is cut into blocks of B x B cells and every layer; block
// (qa, qb) is pixel (qb, qa) of a block grid.  With u_i = sum_j K(r_j - r_i)
// n_j, K(r) = (1 - 3 r^ r^)/|r|^3 (the dipole gradient in units of C_dd mu^2):
//   backbone: exact pair sums over the sites of the blocks within `reach`
//             blocks of i's block (along a and b), and one dipole
//             M_b = sum_{j in b} n_j at the block centroid R_b for every
//             other block;
//   learned:  a 3x3-convolution network on the block grid maps the block
//             moments (M_b, and the first moments Q_b[g][c] =
//             sum_j (r_jg - R_bg) n_jc) to per-block coefficients of the
//             backbone's error, c0_b + (r_i - R_b) . c1_b, trained on the
//             least-squares fit of (direct sum - backbone) per block.
// Channel layout of a block pixel: M or c0 at c = 0..2, Q or c1 at
// 3 + 3 g + c.
#pragma once

#include <type_traits>

#include "kernels_conv.hpp"

namespace sp {

struct DdrGeo {
    int NA, NB, NC, B;      // cells and block side
    int QA, QB;             // block grid (NA / B, NB / B)
    int reach;              // exact blocks on each side
    float a;                // lattice constant (Angstrom)
    float ca, cb, cc;       // centroid of a block relative to its first cell, in cells
};

// Block moments of sample b: network input (bf16, NHWC, channels padded to
// kCP) scaled by in_s0 (moment) and in_s1 (first moments), and the moments
// themselves (FP32, [b][qb][qa][3]) for the backbone's far field.  One
// wavefront per block, one site per lane (B * B * NC == 64), sums by a
// fixed butterfly of lane exchanges; four blocks per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) k_ddr_moments(DdrGeo G, const T* __restrict__ n, int64_t stride_n,
                                                     float in_s0, float in_s1, __bf16* __restrict__ x0, int b0,
                                                     float* __restrict__ M0) {
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int b = blockIdx.y;
    if (q >= G.QA * G.QB) return;   // the whole wavefront
    const int qa = q % G.QA, qb = q / G.QA;
    const int la = l % G.B, lb = (l / G.B) % G.B, lc = l / (G.B * G.B);
    const int64_t N = (int64_t)G.NA * G.NB * G.NC;
    const T* nb = n + (size_t)b * stride_n;
    const int64_t i = (qa * G.B + la) + (int64_t)G.NA * ((qb * G.B + lb) + (int64_t)G.NB * lc);
    const float v[3] = {(float)nb[i], (float)nb[N + i], (float)nb[2 * N + i]};
    const float d[3] = {(la - G.ca) * G.a, (lb - G.cb) * G.a, (lc - G.cc) * G.a};
    // acc[c] = m_c, acc[3 + 3 g + c] = Q_gc = sum d_g v_c
    float acc[12];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = v[c];
#pragma unroll
        for (int g = 0; g < 3; ++g) acc[3 + 3 * g + c] = d[g] * v[c];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] += __shfl_xor(acc[k], o, 64);
    if (M0 && l < 3) M0[((size_t)b * G.QA * G.QB + q) * 3 + l] = acc[l];
    if (x0 && l < kCP) {
        float v0 = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            if (l == k) v0 = (k < 3 ? in_s0 : in_s1) * acc[k];
        x0[((size_t)(b0 + b) * G.QA * G.QB + q) * kCP + l] = (__bf16)v0;
    }
}

// u += K(r) v, r from the field point to the source; r = 0 adds nothing
// (NZ: the caller guarantees r != 0, and the test is left out).
template <bool NZ = false>
__device__ __forceinline__ void ddr_add(float rx, float ry, float rz, float vx, float vy, float vz, float& ux,
                                        float& uy, float& uz) {
    const float d2 = rx * rx + ry * ry + rz * rz;
    float inv;
    if constexpr (NZ)
        inv = __builtin_amdgcn_rsqf(d2);
    else
        inv = d2 > 0.f ? __builtin_amdgcn_rsqf(d2) : 0.f;
    const float inv2 = inv * inv;
    const float inv3 = inv2 * inv;
    const float s = (vx * rx + vy * ry + vz * rz) * (3.f * inv2);
    ux += (vx - s * rx) * inv3;
    uy += (vy - s * ry) * inv3;
    uz += (vz - s * rz) * inv3;
}

constexpr int kDdrMaxNear = 1600;     // staged near sources of one target block (25 blocks of 64)
constexpr int kDdrChunk = 1024;       // far-block moments staged per pass

// Backbone field (units of C_dd mu^2) of every site of one target block
// (blockIdx.x) of sample blockIdx.y: 256 threads = 8 source slices x 32
// lanes, each lane two targets (sites t and t + 32 of the block), so each
// source read from LDS serves two targets.  The sources of the near blocks
// are staged in LDS (spin, and position relative to the target block's
// first cell); slice k takes every eighth staged source.  The far blocks'
// moments are staged in LDS a chunk of block rows at a time; slice k takes
// every eighth block row, each row as the column ranges left and right of
// the near window (no test per block).  The eight partial sums are added in
// a fixed order.  Requires B * B * NC == 64 and reach <= 2.
template <typename T>
__global__ void __launch_bounds__(256) k_ddr_backbone(DdrGeo G, const T* __restrict__ n, int64_t stride_n,
                                                      const float* __restrict__ M0, float* __restrict__ u,
                                                      int64_t stride_u) {
    constexpr int NS = 8;   // source slices
    __shared__ float4 sv[kDdrMaxNear];
    __shared__ float4 sp[kDdrMaxNear];
    __shared__ float4 sm[kDdrChunk];
    __shared__ float red[NS - 1][6][32];
    const int q = blockIdx.x, b = blockIdx.y;
    const int qa = q % G.QA, qb = q / G.QA;
    const int64_t N = (int64_t)G.NA * G.NB * G.NC;
    const T* nb = n + (size_t)b * stride_n;
    const float* Mb = M0 + (size_t)b * G.QA * G.QB * 3;
    const int tid = threadIdx.x, lane = tid & 31, k = tid >> 5;
    const int a0 = qa * G.B, b0 = qb * G.B;
    const int oa0 = max(0, qa - G.reach), oa1 = min(G.QA - 1, qa + G.reach);
    const int ob0 = max(0, qb - G.reach), ob1 = min(G.QB - 1, qb + G.reach);
    const int nwa = oa1 - oa0 + 1;
    const int n_near = nwa * (ob1 - ob0 + 1) * 64;
    // stage the near sources (block-major, 64 sites per block)
    for (int s = tid; s < n_near; s += 256) {
        const int blk = s >> 6, l = s & 63;
        const int sa = oa0 + blk % nwa, sb = ob0 + blk / nwa;
        const int la = l % G.B, lb = (l / G.B) % G.B, lc = l / (G.B * G.B);
        const int ga = sa * G.B + la, gb = sb * G.B + lb;
        const int64_t j = ga + (int64_t)G.NA * (gb + (int64_t)G.NB * lc);
        sv[s] = make_float4((float)nb[j], (float)nb[N + j], (float)nb[2 * N + j], 0.f);
        sp[s] = make_float4((ga - a0) * G.a, (gb - b0) * G.a, lc * G.a, 0.f);
    }
    __syncthreads();
    // the lane's two targets: sites t0 = lane and t1 = lane + 32 of the block
    const int t0 = lane, t1 = lane + 32;
    const int ta0 = t0 % G.B, tb0 = (t0 / G.B) % G.B, tc0 = t0 / (G.B * G.B);
    const int ta1 = t1 % G.B, tb1 = (t1 / G.B) % G.B, tc1 = t1 / (G.B * G.B);
    const float px0 = ta0 * G.a, py0 = tb0 * G.a, pz0 = tc0 * G.a;
    const float px1 = ta1 * G.a, py1 = tb1 * G.a, pz1 = tc1 * G.a;
    float ux0 = 0.f, uy0 = 0.f, uz0 = 0.f, ux1 = 0.f, uy1 = 0.f, uz1 = 0.f;
    // staged sources [s0, s1) of this slice (s0, s1 multiples of NS); only the
    // target block's own sources can sit at r = 0 (the site itself adds 0)
    auto near = [&](int s0, int s1, auto nz) {
        constexpr bool NZ = decltype(nz)::value;
        int s = s0 + k;
        for (; s + NS < s1; s += 2 * NS) {
            const float4 v0 = sv[s], r0 = sp[s], v1 = sv[s + NS], r1 = sp[s + NS];
            ddr_add<NZ>(r0.x - px0, r0.y - py0, r0.z - pz0, v0.x, v0.y, v0.z, ux0, uy0, uz0);
            ddr_add<NZ>(r0.x - px1, r0.y - py1, r0.z - pz1, v0.x, v0.y, v0.z, ux1, uy1, uz1);
            ddr_add<NZ>(r1.x - px0, r1.y - py0, r1.z - pz0, v1.x, v1.y, v1.z, ux0, uy0, uz0);
            ddr_add<NZ>(r1.x - px1, r1.y - py1, r1.z - pz1, v1.x, v1.y, v1.z, ux1, uy1, uz1);
        }
        for (; s < s1; s += NS) {
            const float4 v = sv[s], r = sp[s];
            ddr_add<NZ>(r.x - px0, r.y - py0, r.z - pz0, v.x, v.y, v.z, ux0, uy0, uz0);
            ddr_add<NZ>(r.x - px1, r.y - py1, r.z - pz1, v.x, v.y, v.z, ux1, uy1, uz1);
        }
    };
    const int own0 = ((qa - oa0) + (qb - ob0) * nwa) * 64;
    near(0, own0, std::true_type{});
    near(own0, own0 + 64, std::false_type{});
    near(own0 + 64, n_near, std::true_type{});
    // far blocks: one dipole at the centroid, staged a chunk of rows at a time
    const float step = G.B * G.a;
    const float cx0 = (G.ca - ta0) * G.a - qa * step, cy0 = (G.cb - tb0) * G.a - qb * step, cz0 = (G.cc - tc0) * G.a;
    const float cx1 = (G.ca - ta1) * G.a - qa * step, cy1 = (G.cb - tb1) * G.a - qb * step, cz1 = (G.cc - tc1) * G.a;
    const int rows_per_chunk = max(1, kDdrChunk / G.QA);
    for (int r0 = 0; r0 < G.QB; r0 += rows_per_chunk) {
        const int r1 = min(G.QB, r0 + rows_per_chunk);
        __syncthreads();   // the previous chunk is no longer read
        for (int m = tid; m < (r1 - r0) * G.QA; m += 256) {
            const float* mm = Mb + 3 * ((size_t)r0 * G.QA + m);
            sm[m] = make_float4(mm[0], mm[1], mm[2], 0.f);
        }
        __syncthreads();
        for (int fb = r0 + k; fb < r1; fb += NS) {
            const float ry0 = fb * step + cy0, ry1 = fb * step + cy1;
            const float4* row = sm + (fb - r0) * G.QA;
            const bool in_rows = fb >= ob0 && fb <= ob1;
            const int gap0 = in_rows ? oa0 : G.QA, gap1 = in_rows ? oa1 + 1 : G.QA;
            // a far block's centroid is at least reach + 1/2 blocks away: r != 0
            for (int fa = 0; fa < gap0; ++fa) {
                const float4 m = row[fa];
                ddr_add<true>(fa * step + cx0, ry0, cz0, m.x, m.y, m.z, ux0, uy0, uz0);
                ddr_add<true>(fa * step + cx1, ry1, cz1, m.x, m.y, m.z, ux1, uy1, uz1);
            }
            for (int fa = gap1; fa < G.QA; ++fa) {
                const float4 m = row[fa];
                ddr_add<true>(fa * step + cx0, ry0, cz0, m.x, m.y, m.z, ux0, uy0, uz0);
                ddr_add<true>(fa * step + cx1, ry1, cz1, m.x, m.y, m.z, ux1, uy1, uz1);
            }
        }
    }
    if (k > 0) {
        float* r = &red[k - 1][0][0];
        r[0 * 32 + lane] = ux0;
        r[1 * 32 + lane] = uy0;
        r[2 * 32 + lane] = uz0;
        r[3 * 32 + lane] = ux1;
        r[4 * 32 + lane] = uy1;
        r[5 * 32 + lane] = uz1;
    }
    __syncthreads();
    if (k == 0) {
        for (int j = 0; j < NS - 1; ++j) {
            ux0 += red[j][0][lane];
            uy0 += red[j][1][lane];
            uz0 += red[j][2][lane];
            ux1 += red[j][3][lane];
            uy1 += red[j][4][lane];
            uz1 += red[j][5][lane];
        }
        float* ub = u + (size_t)b * stride_u;
        const int64_t i0 = (a0 + ta0) + (int64_t)G.NA * ((b0 + tb0) + (int64_t)G.NB * tc0);
        const int64_t i1 = (a0 + ta1) + (int64_t)G.NA * ((b0 + tb1) + (int64_t)G.NB * tc1);
        ub[i0] = ux0;
        ub[N + i0] = uy0;
        ub[2 * N + i0] = uz0;
        ub[i1] = ux1;
        ub[N + i1] = uy1;
        ub[2 * N + i1] = uz1;
    }
}

// Training target of sample b: the per-block least-squares coefficients of
// r = field / scale - backbone (field in meV, scale = C_dd mu^2), divided by
// out_s0 (c0) and out_s1 (c1).  For a full block with its centroid at the
// origin the normal equations are diagonal: c0 = mean r, c1_g =
// sum d_g r / sum d_g^2.  One thread per block.
template <typename T>
__global__ void __launch_bounds__(256) k_ddr_target(DdrGeo G, const T* __restrict__ field, int64_t stride_f,
                                                    float inv_scale, const float* __restrict__ u, int64_t stride_u,
                                                    float out_s0, float out_s1, float* __restrict__ target, int b0) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (q >= G.QA * G.QB) return;
    const int qa = q % G.QA, qb = q / G.QA;
    const int64_t N = (int64_t)G.NA * G.NB * G.NC;
    const T* fb = field + (size_t)b * stride_f;
    const float* ub = u + (size_t)b * stride_u;
    float s0[3] = {0.f, 0.f, 0.f}, s1[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float dd[3] = {0.f, 0.f, 0.f};
    for (int lc = 0; lc < G.NC; ++lc)
        for (int lb = 0; lb < G.B; ++lb)
            for (int la = 0; la < G.B; ++la) {
                const int64_t i = (qa * G.B + la) + (int64_t)G.NA * ((qb * G.B + lb) + (int64_t)G.NB * lc);
                const float d[3] = {(la - G.ca) * G.a, (lb - G.cb) * G.a, (lc - G.cc) * G.a};
#pragma unroll
                for (int g = 0; g < 3; ++g) dd[g] += d[g] * d[g];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float r = inv_scale * (float)fb[(size_t)c * N + i] - ub[(size_t)c * N + i];
                    s0[c] += r;
#pragma unroll
                    for (int g = 0; g < 3; ++g) s1[3 * g + c] += d[g] * r;
                }
            }
    float* o = target + ((size_t)(b0 + b) * G.QA * G.QB + q) * 12;
    const float cnt = (float)(G.B * G.B * G.NC);
    for (int c = 0; c < 3; ++c) o[c] = s0[c] / cnt / out_s0;
    for (int g = 0; g < 3; ++g)
        for (int c = 0; c < 3; ++c) o[3 + 3 * g + c] = (dd[g] > 0.f ? s1[3 * g + c] / dd[g] : 0.f) / out_s1;
}

// The field of the residual form: g_i = scale (u_i + c0_b + (r_i - R_b) . c1_b)
// with c0 = out_s0 z[0..2], c1 = out_s1 z[3..11] of the network output z
// (FP32, NHWC with kCP channels).  One thread per site.
template <typename T>
__global__ void __launch_bounds__(256) k_ddr_apply(DdrGeo G, const float* __restrict__ u, const float* __restrict__ z,
                                                   float out_s0, float out_s1, float scale, T* __restrict__ g) {
    const int64_t N = (int64_t)G.NA * G.NB * G.NC;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int ga = (int)(i % G.NA), gb = (int)((i / G.NA) % G.NB), gc = (int)(i / ((int64_t)G.NA * G.NB));
    const int qa = ga / G.B, qb = gb / G.B;
    const float* zb = z + ((size_t)qb * G.QA + qa) * kCP;
    const float d[3] = {(ga - qa * G.B - G.ca) * G.a, (gb - qb * G.B - G.cb) * G.a, (gc - G.cc) * G.a};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v = u[(size_t)c * N + i] + out_s0 * zb[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) v += out_s1 * d[k] * zb[3 + 3 * k + c];
        g[(size_t)c * N + i] = (T)(scale * v);
    }
}

}  // namespace sp
