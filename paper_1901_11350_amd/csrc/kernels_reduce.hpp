// kernels_reduce.hpp -- double-precision reductions of the observables:
// energy per term (Zeeman linear, the rest quadratic: E = sum n.(g_Z + g_rest/2),
// the linear + quadratic split of the Hamiltonian), maximum and RMS torque
// |n x g|, mean spin, maximum | |n| - 1 |, and a count of non-finite torques.
//
// Stage 1: every workgroup reduces a grid-stride slice of sites (wavefront
// shuffles, then LDS across the four wavefronts) into one row of partials.
// Stage 2: one workgroup reduces the rows in a fixed order, so results are
// bit-reproducible run to run.
#pragma once

#include "kernels_field.hpp"

namespace sp {

enum {
    OBS_EZ = 0, OBS_EK, OBS_EJ, OBS_ED, OBS_EDD,
    OBS_TMAX, OBS_MX, OBS_MY, OBS_MZ, OBS_NDEV, OBS_T2, OBS_NONFINITE,
    OBS_NVALS
};

__device__ __forceinline__ bool is_max_slot(int k) { return k == OBS_TMAX || k == OBS_NDEV; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Reduce acc[OBS_NVALS] across a workgroup of NW wavefronts; thread 0 gets
// the result.
template <int NW = 4>
__device__ __forceinline__ void block_reduce(double* acc) {
    __shared__ double red[NW][OBS_NVALS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < OBS_NVALS; ++k) {
        const double v = is_max_slot(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) {
            double v = red[0][k];
            for (int w = 1; w < NW; ++w) v = is_max_slot(k) ? fmax(v, red[w][k]) : v + red[w][k];
            acc[k] = v;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_observe_partial(Lattice L, BondCoef<T> C, Phys<T> P,
                                                         const T* __restrict__ n,
                                                         const T* __restrict__ gdd,
                                                         double* __restrict__ partials) {
    double acc[OBS_NVALS];
#pragma unroll
    for (int k = 0; k < OBS_NVALS; ++k) acc[k] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L.N; i += gridDim.x * blockDim.x) {
        const V3<T> ni = load3(n, L.N, i);
        const FieldTerms<T> f = site_terms(L, C, P, n, i, ni);
        V3<T> g = total(f);
        double edd = 0.0;
        if (gdd) {
            const V3<T> gd = load3(gdd, L.N, i);
            edd = 0.5 * ((double)ni.x * gd.x + (double)ni.y * gd.y + (double)ni.z * gd.z);
            g = g + gd;
        }
        const double nx = ni.x, ny = ni.y, nz = ni.z;
        acc[OBS_EZ] += nx * f.z.x + ny * f.z.y + nz * f.z.z;
        acc[OBS_EK] += 0.5 * (nx * f.k.x + ny * f.k.y + nz * f.k.z) + gauss_energy(P, ni);
        acc[OBS_EJ] += 0.5 * (nx * f.j.x + ny * f.j.y + nz * f.j.z);
        acc[OBS_ED] += 0.5 * (nx * f.d.x + ny * f.d.y + nz * f.d.z);
        acc[OBS_EDD] += edd;
        const double tx = ny * g.z - nz * g.y, ty = nz * g.x - nx * g.z, tz = nx * g.y - ny * g.x;
        const double t2 = tx * tx + ty * ty + tz * tz;
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
    block_reduce(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) partials[blockIdx.x * OBS_NVALS + k] = acc[k];
    }
}

// Final stage: rows of partials -> out[OBS_NVALS]; raises *abort_flag when a
// non-finite torque was seen, and records the step in abort_step.
// Run control flags (abort_flag): 0 running; 1 a non-finite torque was seen
// (the run aborts); 2 the convergence test passed (the run stops).  Step
// kernels return at once while the flag is nonzero.
enum { RUN_GO = 0, RUN_NONFINITE = 1, RUN_CONVERGED = 2 };

// Stage 2.  With abort_flag set, the observation also decides whether the
// run goes on: a non-finite torque aborts it; with tol > 0, a maximum torque
// |n x g| below tol (the convergence test, in FP64) stops it.  *abort_step
// records the step of that observation: `step`, or *step_dev + step_off in
// a replayed graph.
__global__ void __launch_bounds__(256) k_observe_final(const double* __restrict__ partials, int rows,
                                                       double* __restrict__ out, int* __restrict__ abort_flag,
                                                       long long* __restrict__ abort_step, long long step,
                                                       const unsigned long long* __restrict__ step_dev,
                                                       int step_off, double tol) {
    double acc[OBS_NVALS];
#pragma unroll
    for (int k = 0; k < OBS_NVALS; ++k) acc[k] = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) {
            const double v = partials[r * OBS_NVALS + k];
            acc[k] = is_max_slot(k) ? fmax(acc[k], v) : acc[k] + v;
        }
    }
    block_reduce(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) out[k] = acc[k];
        if (abort_flag && *abort_flag == RUN_GO) {
            const long long s = step_dev ? (long long)(*step_dev + (unsigned long long)step_off) : step;
            if (acc[OBS_NONFINITE] > 0.0) {
                *abort_flag = RUN_NONFINITE;
                *abort_step = s;
            } else if (tol > 0.0 && acc[OBS_TMAX] < tol) {
                *abort_flag = RUN_CONVERGED;
                *abort_step = s;
            }
        }
    }
}

// Start of a run: clear the run flag and set the device step and the index
// of the next observation row (a kernel rather than memsets, so that the
// same values reach the device in stream order on every path).
__global__ void k_set_run_ctl(int* __restrict__ flag, long long* __restrict__ abort_step,
                              unsigned long long* __restrict__ step_dev, long long* __restrict__ obs_index,
                              unsigned long long step, long long index) {
    if (threadIdx.x != 0) return;
    *flag = RUN_GO;
    *abort_step = 0;
    *step_dev = step;
    *obs_index = index;
}

// End of a replayed chunk of `steps` steps: advance the device step and,
// when the chunk ends with an observation, move it from the staging row to
// the next row of the run's observation array (rows past cap are dropped).
__global__ void k_run_chunk_end(unsigned long long* __restrict__ step_dev, long long* __restrict__ obs_index,
                                const double* __restrict__ stage, double* __restrict__ obs, long long cap,
                                int steps) {
    if (threadIdx.x != 0) return;
    if (stage) {
        const long long q = *obs_index;
        if (q < cap)
            for (int k = 0; k < OBS_NVALS; ++k) obs[q * OBS_NVALS + k] = stage[k];
        *obs_index = q + 1;
    }
    *step_dev += (unsigned long long)steps;
}

}  // namespace sp
