// kernels_stencil.hpp -- the stand-alone stencil field kernel (sp_gradient on
// one-atom 2D lattices with a compile-time stencil; the shapes and field
// routine of kernels_fused2d.hpp) and the observables on the same tiles.
#pragma once

#include "kernels_fused2d.hpp"
#include "kernels_reduce.hpp"

namespace sp {

// Stand-alone stencil field: dH/dn of exchange, DMI, anisotropy and Zeeman
// (Sec. III.A) for one-atom 2D lattices with a compile-time stencil.  The
// TX x TY tile plus an R halo is staged in LDS as 16/32-byte cells from
// coalesced row loads of the three SoA planes; each thread forms the field
// of its site from immediate-offset LDS reads and writes it once.  HBM:
// read n (12 B per FP32 site, the halo mostly from L2), write g (12 B).
template <typename T, int S, int NDMI, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_gradient_shape(ShapeCoef<T> C, Site2D<T> Q, TileMap M,
                                                       const T* __restrict__ n, T* __restrict__ g) {
    constexpr int R = ShapeTab<S>::R, W = TX + 2 * R, H = TY + 2 * R, P = W * H, PT = TX * TY;
    static_assert(PT % NT == 0, "tile sites must divide evenly over the threads");
    constexpr int KPT = PT / NT, KST = (P + NT - 1) / NT;
    __shared__ V4<T> sN[P];
    const int ntiles = M.tiles_x * M.tiles_y;
    int tile = blockIdx.x;
    if (M.xcd_bands) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int tyi = tile / M.tiles_x;
    const int x0 = (tile - tyi * M.tiles_x) * TX, y0 = tyi * TY;
    const int N = Q.na * Q.nb;
    const int tid = threadIdx.x;
    // every load of the tile in flight before the first LDS write
    V4<T> st[KST];
#pragma unroll
    for (int k = 0; k < KST; ++k) {
        const int idx = tid + k * NT;
        st[k] = V4<T>{T(0), T(0), T(0), T(0)};
        if (idx < P) {
            const int ly = idx / W, lx = idx - ly * W;
            bool in = true;
            const int gx = wrap_once(x0 - R + lx, Q.na, Q.per_a, in);
            const int gy = wrap_once(y0 - R + ly, Q.nb, Q.per_b, in);
            if (in) {
                const int q = gx + gy * Q.na;
                st[k] = V4<T>{n[q], n[N + q], n[2 * N + q], T(0)};
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KST; ++k) {
        const int idx = tid + k * NT;
        if (idx < P) sN[idx] = st[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const int t = tid + j * NT;
        const int ty = t / TX, tx = t - ty * TX;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= Q.na || gy >= Q.nb) continue;
        const int c = (ty + R) * W + (tx + R);
        const V3<T> gv = shape_field_aos<T, S, NDMI, W>(C, Q, sN, c, lds_cell_xyz(sN, c));
        const int gi = gx + gy * Q.na;
        store_out(g + gi, gv.x);
        store_out(g + N + gi, gv.y);
        store_out(g + 2 * N + gi, gv.z);
    }
}

// The same field for FP32 lattices whose sides divide into 64 x 64 tiles,
// with 16-byte global accesses: each plane's rows of the tile are loaded as
// float4 (16 per row), only the R halo columns as single floats, and each
// thread forms the fields of four consecutive sites of one row and stores
// them as one float4 per plane.  (16-byte lanes move ~20 % more bytes per
// second than 4-byte lanes in a device copy on MI355X.)
template <int S, int NDMI>
__global__ void __launch_bounds__(1024) k_gradient_shape_v4(ShapeCoef<float> C, Site2D<float> Q, TileMap M,
                                                            const float* __restrict__ n, float* __restrict__ g) {
    constexpr int TX = 64, TY = 64, NT = 1024;
    constexpr int R = ShapeTab<S>::R, W = TX + 2 * R, H = TY + 2 * R, P = W * H;
    constexpr int NV = 3 * H * (TX / 4);                   // float4 loads of the tile rows, three planes
    constexpr int NS = 3 * H * 2 * R;                      // single loads of the halo columns
    constexpr int KV = (NV + NT - 1) / NT, KS = (NS + NT - 1) / NT;
    __shared__ V4<float> sN[P];
    const int ntiles = M.tiles_x * M.tiles_y;
    int tile = blockIdx.x;
    if (M.xcd_bands) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int tyi = tile / M.tiles_x;
    const int x0 = (tile - tyi * M.tiles_x) * TX, y0 = tyi * TY;
    const int N = Q.na * Q.nb;
    const int tid = threadIdx.x;
    float4 vv[KV];
    float sv[KS];
    // every load of the tile in flight before the first LDS write
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int idx = tid + k * NT;
        vv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (idx < NV) {
            const int comp = idx / (H * 16), r = idx - comp * (H * 16);
            const int ly = r >> 4, cx = r & 15;
            bool in = true;
            const int gy = wrap_once(y0 - R + ly, Q.nb, Q.per_b, in);
            if (in) vv[k] = *reinterpret_cast<const float4*>(n + (size_t)comp * N + (size_t)gy * Q.na + x0 + 4 * cx);
        }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        sv[k] = 0.f;
        if (idx < NS) {
            const int comp = idx / (H * 2 * R), r = idx - comp * (H * 2 * R);
            const int ly = r / (2 * R), h = r - ly * (2 * R);
            const int lx = h < R ? h : TX + h;
            bool in = true;
            const int gx = wrap_once(x0 - R + lx, Q.na, Q.per_a, in);
            const int gy = wrap_once(y0 - R + ly, Q.nb, Q.per_b, in);
            if (in) sv[k] = n[(size_t)comp * N + (size_t)gy * Q.na + gx];
        }
    }
    float* sf = reinterpret_cast<float*>(sN);   // component c of cell i at sf[4 i + c]
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int idx = tid + k * NT;
        if (idx < NV) {
            const int comp = idx / (H * 16), r = idx - comp * (H * 16);
            const int ly = r >> 4, cx = r & 15;
            const int cell = ly * W + R + 4 * cx;
            sf[4 * cell + comp] = vv[k].x;
            sf[4 * (cell + 1) + comp] = vv[k].y;
            sf[4 * (cell + 2) + comp] = vv[k].z;
            sf[4 * (cell + 3) + comp] = vv[k].w;
        }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        if (idx < NS) {
            const int comp = idx / (H * 2 * R), r = idx - comp * (H * 2 * R);
            const int ly = r / (2 * R), h = r - ly * (2 * R);
            const int lx = h < R ? h : TX + h;
            sf[4 * (ly * W + lx) + comp] = sv[k];
        }
    }
    __syncthreads();
    const int ty = tid >> 4, cx = tid & 15;
    float ox[4], oy[4], oz[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = (ty + R) * W + (R + 4 * cx + u);
        const V3<float> gv = shape_field_aos<float, S, NDMI, W>(C, Q, sN, c, lds_cell_xyz(sN, c));
        ox[u] = gv.x;
        oy[u] = gv.y;
        oz[u] = gv.z;
    }
    const size_t gi = (size_t)(y0 + ty) * Q.na + x0 + 4 * cx;
    *reinterpret_cast<float4*>(g + gi) = make_float4(ox[0], ox[1], ox[2], ox[3]);
    *reinterpret_cast<float4*>(g + N + gi) = make_float4(oy[0], oy[1], oy[2], oy[3]);
    *reinterpret_cast<float4*>(g + 2 * (size_t)N + gi) = make_float4(oz[0], oz[1], oz[2], oz[3]);
}

// The four local terms of dH/dn at LDS cell c, kept apart for the energy
// per term: the same sums as shape_field (Sec. III.A).
template <typename T, int S, int NDMI, int W>
__device__ __forceinline__ FieldTerms<T> shape_terms(const ShapeCoef<T>& C, const Site2D<T>& Q,
                                                     const V4<T>* __restrict__ sv, int c, V3<T> ni) {
    using SH = ShapeTab<S>;
    V3<T> acc[SH::NS];
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) acc[s] = V3<T>{T(0), T(0), T(0)};
    V3<T> d{T(0), T(0), T(0)};   // sum of n_j x D over the DMI bonds, D = (Dx, Dy, 0)
#pragma unroll
    for (int q = 0; q < SH::NB; ++q) {
        const V3<T> nj = lds_cell_xyz(sv, c + SH::da[q] + SH::db[q] * W);
        acc[SH::sh[q]] = acc[SH::sh[q]] + nj;
        if (q < NDMI) {
            d.x -= nj.z * C.Dy[q];
            d.y += nj.z * C.Dx[q];
            d.z += nj.x * C.Dy[q] - nj.y * C.Dx[q];
        }
    }
    FieldTerms<T> f;
    f.z = V3<T>{Q.gZ[0], Q.gZ[1], Q.gZ[2]};
    const V3<T> ax{Q.Kax[0], Q.Kax[1], Q.Kax[2]};
    f.k = (-Q.K2 * dot(ax, ni)) * ax;
    V3<T> j{T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) j = j - C.J[s] * acc[s];
    f.j = j;
    f.d = T(-1) * d;
    f.q = V3<T>{T(0), T(0), T(0)};
    return f;
}

// Stage 1 of the observables (kernels_reduce.hpp) on the tiles of the
// stencil path: each workgroup stages TX x TY tiles plus an R halo in LDS, as
// k_gradient_shape does, and folds the energy per term, torque, mean spin and
// norm deviation of their sites into one row of partials.  Workgroups take
// tiles blockIdx.x, blockIdx.x + gridDim.x, ...; k_observe_final reduces
// the gridDim.x rows.  No dipole term and no on-site potentials on this
// path.
template <typename T, int S, int NDMI, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_observe_shape(ShapeCoef<T> C, Site2D<T> Q, TileMap M,
                                                      const T* __restrict__ n, double* __restrict__ partials) {
    static_assert(NT % 64 == 0, "whole wavefronts");
    constexpr int R = ShapeTab<S>::R, W = TX + 2 * R, H = TY + 2 * R, P = W * H, PT = TX * TY;
    static_assert(PT % NT == 0, "tile sites must divide evenly over the threads");
    constexpr int KPT = PT / NT, KST = (P + NT - 1) / NT;
    __shared__ V4<T> sN[P];
    const int ntiles = M.tiles_x * M.tiles_y;
    const int N = Q.na * Q.nb;
    const int tid = threadIdx.x;
    double acc[OBS_NVALS];
#pragma unroll
    for (int k = 0; k < OBS_NVALS; ++k) acc[k] = 0.0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tyi = tile / M.tiles_x;
        const int x0 = (tile - tyi * M.tiles_x) * TX, y0 = tyi * TY;
        V4<T> st[KST];
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            const int idx = tid + k * NT;
            st[k] = V4<T>{T(0), T(0), T(0), T(0)};
            if (idx < P) {
                const int ly = idx / W, lx = idx - ly * W;
                bool in = true;
                const int gx = wrap_once(x0 - R + lx, Q.na, Q.per_a, in);
                const int gy = wrap_once(y0 - R + ly, Q.nb, Q.per_b, in);
                if (in) {
                    const int q = gx + gy * Q.na;
                    st[k] = V4<T>{n[q], n[N + q], n[2 * N + q], T(0)};
                }
            }
        }
        __syncthreads();   // the previous tile's cells are no longer read
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            const int idx = tid + k * NT;
            if (idx < P) sN[idx] = st[k];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int t = tid + j * NT;
            const int ty = t / TX, tx = t - ty * TX;
            if (x0 + tx >= Q.na || y0 + ty >= Q.nb) continue;
            const int c = (ty + R) * W + (tx + R);
            const V3<T> ni = lds_cell_xyz(sN, c);
            const FieldTerms<T> f = shape_terms<T, S, NDMI, W>(C, Q, sN, c, ni);
            const V3<T> g = f.z + f.k + f.j + f.d;
            const double nx = ni.x, ny = ni.y, nz = ni.z;
            acc[OBS_EZ] += nx * f.z.x + ny * f.z.y + nz * f.z.z;
            acc[OBS_EK] += 0.5 * (nx * f.k.x + ny * f.k.y + nz * f.k.z);
            acc[OBS_EJ] += 0.5 * (nx * f.j.x + ny * f.j.y + nz * f.j.z);
            acc[OBS_ED] += 0.5 * (nx * f.d.x + ny * f.d.y + nz * f.d.z);
            const double tx_ = ny * g.z - nz * g.y, ty_ = nz * g.x - nx * g.z, tz_ = nx * g.y - ny * g.x;
            const double t2 = tx_ * tx_ + ty_ * ty_ + tz_ * tz_;
            if (!isfinite(t2)) {
                acc[OBS_NONFINITE] += 1.0;
            } else {
                acc[OBS_TMAX] = fmax(acc[OBS_TMAX], sqrt(t2));
                acc[OBS_T2] += t2;
            }
            acc[OBS_MX] += nx;
            acc[OBS_MY] += ny;
            acc[OBS_MZ] += nz;
            const double nn = sqrt(nx * nx + ny * ny + nz * nz);
            acc[OBS_NDEV] = fmax(acc[OBS_NDEV], fabs(nn - 1.0));
        }
    }
    block_reduce<NT / 64>(acc);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) partials[blockIdx.x * OBS_NVALS + k] = acc[k];
    }
}

}  // namespace sp
