// kernels_mc.hpp -- Metropolis Monte Carlo with cone trial moves (Sec. III.B).
// The paper's sweep picks every spin once, one after another, in random
// order.  Here a sweep is a multi-colour pass: the host colours the sites
// periodically -- colour(i) = table[a mod ma][b mod mb][c mod mc][beta] --
// so that no bond joins two sites of one colour (two colours, the
// checkerboard, for the simple-cubic nearest-neighbour lattice; three or
// more for triangular, second-neighbour or basis lattices), and one launch
// updates a whole colour in parallel; every site is still tried once per
// sweep and each trial sees the current state of every spin it interacts
// with, so the chain samples the same Boltzmann distribution (checked
// statistically against the sequential random-order sweep).
//
// Trial at site i of sweep s: Philox block of counter (i, s_lo, s_hi,
// replica), u_k = (x_k + 1/2) 2^-32; phi = 2 pi u0, cos(theta) = 1 - u1 (1 -
// cos(cone)); new spin cos(theta) n + sin(theta) (cos(phi) e1 + sin(phi) e2),
// e1 = unit(n x r) with r = z if |n_z| < 0.9 else x, e2 = n x e1; accepted
// if u2 < exp(-dE / k_B T).  dE needs only the terms containing site i:
// Zeeman and the pair terms are linear in n_i (dn . coefficient), the
// anisotropy and the on-site Gaussians are evaluated at both spins.
// Adaptive cone: after every sweep the cone is multiplied by
// 1 + a - a* (a the sweep's acceptance ratio, a* the target), at most 180
// degrees, on the device.
#pragma once

#include "kernels_field.hpp"

namespace sp {

template <typename T>
struct McArgs {
    T kT;            // k_B T (meV)
    T cos_cone;
    ThermalKey key;  // seed, sweep number (step words), replica
    int colour;
    const double* cone_dev;   // adaptive cone (degrees) on the device, or null: cos_cone
    const unsigned char* col; // colour of (a mod cm[0], b mod cm[1], c mod cm[2], beta), row-major
    int cm[3];
};

template <typename T>
__device__ __forceinline__ void mc_uniforms(const U4& x, T u[3]) {
    if constexpr (sizeof(T) == 4) {
        u[0] = fmaf((float)x.x, 0x1p-32f, 0x1p-33f);
        u[1] = fmaf((float)x.y, 0x1p-32f, 0x1p-33f);
        u[2] = fmaf((float)x.z, 0x1p-32f, 0x1p-33f);
    } else {
        u[0] = ((double)x.x + 0.5) * 0x1p-32;
        u[1] = ((double)x.y + 0.5) * 0x1p-32;
        u[2] = ((double)x.z + 0.5) * 0x1p-32;
    }
}

template <typename T>
__device__ __forceinline__ V3<T> mc_trial(V3<T> n, const T u[3], T cos_cone) {
    const V3<T> r = fabs(n.z) < T(0.9) ? V3<T>{T(0), T(0), T(1)} : V3<T>{T(1), T(0), T(0)};
    const V3<T> e1 = normalize3(cross(n, r));
    const V3<T> e2 = cross(n, e1);
    T sp, cp;
    if constexpr (sizeof(T) == 4) {
        sp = __builtin_amdgcn_sinf(u[0]);   // argument in revolutions
        cp = __builtin_amdgcn_cosf(u[0]);
    } else {
        sincospi(T(2) * u[0], &sp, &cp);
    }
    const T ct = T(1) - u[1] * (T(1) - cos_cone);
    const T st = sqrt(fmax(T(0), T(1) - ct * ct));
    return V3<T>{ct * n.x + st * (cp * e1.x + sp * e2.x), ct * n.y + st * (cp * e1.y + sp * e2.y),
                 ct * n.z + st * (cp * e1.z + sp * e2.z)};
}

// One colour of one sweep.  acc_part[block] accumulates the
// accepted trials of this workgroup's sites over the launches of a run.
// The accept/reject decision is taken in FP64 for every engine precision
// (the precision of the FP64 reference): trial spin, energy difference and
// Metropolis test from the stored spins (type T) with FP64 couplings; an
// accepted trial is stored rounded to T.
template <typename T>
__global__ void __launch_bounds__(256) k_mc_colour(Lattice L, BondCoef<double> C, Phys<double> P,
                                                   McArgs<double> M, T* __restrict__ n,
                                                   unsigned int* __restrict__ acc_part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    bool accepted = false;
    if (i < L.N) {
        const int a = i % L.n[0];
        const int rem = i / L.n[0];
        const int b = rem % L.n[1];
        const int rem2 = rem / L.n[1];
        const int c = rem2 % L.n[2];
        const int beta = rem2 / L.n[2];
        const int cell = ((a % M.cm[0]) * M.cm[1] + b % M.cm[1]) * M.cm[2] + c % M.cm[2];
        if (M.col[cell * L.nb + beta] == M.colour) {
            const V3<double> ni{(double)n[i], (double)n[L.N + i], (double)n[2 * L.N + i]};
            double u[3];
            mc_uniforms<double>(thermal_bits(M.key, (uint32_t)i), u);
            const double cos_cone = M.cone_dev ? cos(*M.cone_dev * (3.141592653589793 / 180.0)) : M.cos_cone;
            const V3<double> nn = mc_trial(ni, u, cos_cone);
            const FieldTerms<double> f = site_terms<double, T>(L, C, P, n, i, ni);
            const V3<double> lin = f.z + f.j + f.d;
            const V3<double> ax{P.Kax[beta][0], P.Kax[beta][1], P.Kax[beta][2]};
            const double k0 = dot(ax, ni), k1 = dot(ax, nn);
            const double dE = dot(nn - ni, lin) - 0.5 * P.K2[beta] * (k1 * k1 - k0 * k0) +
                              (gauss_energy(P, nn) - gauss_energy(P, ni));
            if (u[2] < exp(-dE / M.kT)) {
                store3(n, L.N, i, V3<T>{(T)nn.x, (T)nn.y, (T)nn.z});
                accepted = true;
            }
        }
    }
    const unsigned long long mask = __ballot(accepted);
    __shared__ unsigned int cnt[4];
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = (unsigned int)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) acc_part[blockIdx.x] += cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Feedback of the adaptive cone after one sweep: the sweep's accepted trials
// are the growth of the run's per-workgroup counts (summed in a fixed
// order) since the previous sweep; state[0] is the cone in degrees,
// state[1] the count at the previous sweep.
__global__ void __launch_bounds__(256) k_mc_adapt(const unsigned int* __restrict__ acc_part, int blocks,
                                                  long long n_sites, double target, double* __restrict__ state) {
    __shared__ unsigned long long red[256];
    unsigned long long t = 0;
    for (int b = threadIdx.x; b < blocks; b += 256) t += acc_part[b];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double total = (double)red[0];
        const double a = n_sites > 0 ? (total - state[1]) / (double)n_sites : 0.0;
        const double c = state[0] * (1.0 + a - target);
        state[0] = c > 180.0 ? 180.0 : c;
        state[1] = total;
    }
}

}  // namespace sp
