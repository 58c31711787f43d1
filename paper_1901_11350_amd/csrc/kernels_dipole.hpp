// kernels_dipole.hpp -- dipole-dipole gradient by direct summation over all
// pairs of the sample (the O(N^2) form of the dipolar term of the
// Hamiltonian, Sec. III.A):
//   g_dd_i = C_dd mu_i sum_{j != i} mu_j [n_j - 3 (n_j . r_ij) r_ij] / r_ij^3.
//
// This is a matrix-free product with a kernel generated on the fly (one
// right-hand side), so it runs on the vector ALUs, not the matrix cores.
// Workgroups own IPT*256 target sites i and one of S slices of the sources j;
// each 256-source tile (positions and moments mu_j n_j) is staged in LDS and
// broadcast to all threads.  Within a tile the sum is accumulated separately
// and then added to the running total (two-level summation).  The S slice
// results are summed in a fixed order by a second kernel.
#pragma once

#include "device_common.hpp"

namespace sp {

template <typename T>
struct DipoleArgs {
    int N;
    int cells;           // sites per sublattice
    int slices;          // S
    int slice_len;       // sources per slice (multiple of 256)
    T mu[kMaxBasis];
};

// gate: when non-null and *gate == 0 the kernel does nothing (the surrogate's
// fallback launches the direct sum unconditionally and lets the device-side
// residual check decide).
template <typename T, int IPT>
__global__ void __launch_bounds__(256) k_dipole_partial(DipoleArgs<T> a, const T* __restrict__ pos,
                                                        const T* __restrict__ n, T* __restrict__ part,
                                                        const int* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ T sp_[6][256];
    const int N = a.N;
    const int i0 = blockIdx.x * (256 * IPT) + threadIdx.x;
    T px[IPT], py[IPT], pz[IPT], gx[IPT], gy[IPT], gz[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int i = i0 + u * 256;
        const int ii = i < N ? i : N - 1;
        px[u] = pos[ii];
        py[u] = pos[N + ii];
        pz[u] = pos[2 * N + ii];
        gx[u] = gy[u] = gz[u] = T(0);
    }
    const int jbeg = blockIdx.y * a.slice_len;
    const int jend = min(N, jbeg + a.slice_len);
    for (int jt = jbeg; jt < jend; jt += 256) {
        __syncthreads();
        {
            const int j = jt + threadIdx.x;
            if (j < jend) {
                const T m = a.mu[j / a.cells];
                sp_[0][threadIdx.x] = pos[j];
                sp_[1][threadIdx.x] = pos[N + j];
                sp_[2][threadIdx.x] = pos[2 * N + j];
                sp_[3][threadIdx.x] = m * n[j];
                sp_[4][threadIdx.x] = m * n[N + j];
                sp_[5][threadIdx.x] = m * n[2 * N + j];
            } else {
                // zero moment: contributes exactly zero
                sp_[0][threadIdx.x] = T(0);
                sp_[1][threadIdx.x] = T(0);
                sp_[2][threadIdx.x] = T(0);
                sp_[3][threadIdx.x] = T(0);
                sp_[4][threadIdx.x] = T(0);
                sp_[5][threadIdx.x] = T(0);
            }
        }
        __syncthreads();
        T tx[IPT], ty[IPT], tz[IPT];
#pragma unroll
        for (int u = 0; u < IPT; ++u) tx[u] = ty[u] = tz[u] = T(0);
        for (int jj = 0; jj < 256; ++jj) {
            const T qx = sp_[0][jj], qy = sp_[1][jj], qz = sp_[2][jj];
            const T mx = sp_[3][jj], my = sp_[4][jj], mz = sp_[5][jj];
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                const T rx = qx - px[u], ry = qy - py[u], rz = qz - pz[u];
                const T d2 = rx * rx + ry * ry + rz * rz;
                T inv;
                if constexpr (sizeof(T) == 4) {
                    inv = d2 > T(0) ? __builtin_amdgcn_rsqf(d2) : T(0);
                } else {
                    inv = d2 > T(0) ? T(1) / sqrt(d2) : T(0);
                }
                const T inv2 = inv * inv;
                const T inv3 = inv2 * inv;
                const T s = T(3) * (mx * rx + my * ry + mz * rz) * inv2;
                tx[u] += (mx - s * rx) * inv3;
                ty[u] += (my - s * ry) * inv3;
                tz[u] += (mz - s * rz) * inv3;
            }
        }
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            gx[u] += tx[u];
            gy[u] += ty[u];
            gz[u] += tz[u];
        }
    }
    T* out = part + (size_t)blockIdx.y * 3 * N;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int i = i0 + u * 256;
        if (i < N) {
            out[i] = gx[u];
            out[N + i] = gy[u];
            out[2 * N + i] = gz[u];
        }
    }
}

// Sum the S slices in order and scale by C_dd mu_i.
template <typename T>
__global__ void __launch_bounds__(256) k_dipole_finish(DipoleArgs<T> a, T Cdd, const T* __restrict__ part,
                                                       T* __restrict__ gdd, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N;
    if (t >= 3 * N) return;
    const int i = t % N;
    T s = T(0);
    for (int k = 0; k < a.slices; ++k) s += part[(size_t)k * 3 * N + t];
    gdd[t] = Cdd * a.mu[i / a.cells] * s;
}

}  // namespace sp
