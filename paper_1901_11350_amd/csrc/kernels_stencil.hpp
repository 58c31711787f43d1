// kernels_stencil.hpp -- the stand-alone stencil field kernel (sp_gradient on
// one-atom 2D lattices with a compile-time stencil; the shapes and field
// routine of kernels_fused2d.hpp).
#pragma once

#include "kernels_fused2d.hpp"

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

}  // namespace sp
