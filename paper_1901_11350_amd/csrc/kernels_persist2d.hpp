// kernels_persist2d.hpp -- many Depondt steps in one launch for one-atom 2D
// lattices with a compile-time stencil (the shapes of kernels_fused2d.hpp).
//
// One workgroup per TX x TY tile, one thread per tile site, every workgroup
// resident at once (cooperative launch).  A thread keeps its site's spin in
// registers from step to step; only the 2R-wide halo of a tile is read from
// HBM each step, out of the spins its eight neighbour tiles wrote at the end
// of the previous step.  Each tile publishes "finished step s" in a flag word
// of its own (one agent-scope release by one thread after a workgroup
// barrier that follows every thread's spin stores); a tile starts
// reading its halo for step s+1 once its neighbours' flags say so (agent-scope
// acquire).  Spins alternate between two buffers by step parity: a tile
// overwrites the buffer that holds n(s-1) only after every neighbour has
// finished step s-1, i.e. has read everything it needed from it.
//
// Per step, the arithmetic is that of the fused one-launch-per-step kernel:
// the same predictor, corrector and base-field routines on the same cells.  The order of the work hides the halo
// traffic: the predictor of the sites at least R from the tile edge needs no
// halo and runs while the neighbours' flags are awaited; the halo is then
// loaded, the edge sites and the R-ring of predictor cells are computed, and
// the corrector follows.
//
// Every wait is bounded: after `spin_limit` polls, or when another workgroup
// has reported a failure in *status, the workgroup reports failure and
// leaves, so every wave of the grid ends.
#pragma once

#include "kernels_fused2d.hpp"

namespace sp {

constexpr int kFlagStride = 32;   // flag words one 128-byte line apart

struct PersistMap {
    int tiles_x, tiles_y;
    int xcd_bands;     // same tile order as the one-step kernel
    int n_steps;
    uint32_t gen;      // flags hold gen + (steps finished in this launch)
    int spin_limit;
};

__device__ __forceinline__ uint32_t persist_flag_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-wide wait until every lane's neighbour flag reaches `target` (lanes
// with nbr < 0 have none).  Returns false on time-out or reported failure.
__device__ __forceinline__ bool persist_wait(const uint32_t* flags, int* status, int nbr, uint32_t target,
                                             int limit) {
    for (int it = 0;; ++it) {
        bool ready = true;
        if (nbr >= 0) ready = (int)(persist_flag_load(flags + (size_t)nbr * kFlagStride) - target) >= 0;
        if (__all(ready)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if (it >= limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_or(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((it & 63) == 63 && __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

template <typename T, int S, int NDMI, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_persist2d(StepCoef<T> C, Site2D<T> Q, LLGArgs<T> A, PersistMap M,
                                                        const int* __restrict__ abort_flag, T* b0, T* b1,
                                                        uint32_t* flags, int* status) {
    using TL = TileLDS<T, S, TX, TY>;
    constexpr int R = TL::R, WN = TL::WN, PN = TL::PN, PP = TL::PP, PT = TL::PT, NT = TX * TY;
    constexpr int RING = PP - PT;                  // predictor cells around the tile
    constexpr int HALO = PN - PT;                  // staged cells around the tile
    constexpr int KH = (HALO + NT - 1) / NT;
    constexpr int IX = TX - 2 * R, IY = TY - 2 * R;   // inner sites: no halo in their stencil
    static_assert(IX > 0 && IY > 0 && RING <= IX * IY, "ring cells are computed by inner-site threads");
    if (abort_flag && *abort_flag) return;   // set before this launch: the same for every workgroup

    __shared__ TL L;
    __shared__ int s_fail;
    const int ntiles = M.tiles_x * M.tiles_y;
    int tile = blockIdx.x;
    if (M.xcd_bands) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int tyi = tile / M.tiles_x, txi = tile - tyi * M.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int N = Q.na * Q.nb;
    const int tid = threadIdx.x;
    const int ty = tid / TX, tx = tid - ty * TX;
    const int own_c = (ty + 2 * R) * WN + (tx + 2 * R);
    const int gsite = (x0 + tx) + (y0 + ty) * Q.na;
    const bool inner = tx >= R && tx < TX - R && ty >= R && ty < TY - R;
    const int rank = inner ? (ty - R) * IX + (tx - R) : -1;
    int rpx = 0, rpy = 0;
    if (rank >= 0 && rank < RING) ring_cell<R, TX, TY>(rank, rpx, rpy);

    // neighbour tile watched by lanes 0..7 of wave 0
    int nbr = -1;
    if (tid < 8) {
        const int k = tid < 4 ? tid : tid + 1;   // the 3 x 3 block without its centre
        int nx = txi + k % 3 - 1, ny = tyi + k / 3 - 1;
        bool ok = true;
        if (nx < 0 || nx >= M.tiles_x) {
            if (Q.per_a) nx = (nx + M.tiles_x) % M.tiles_x;
            else ok = false;
        }
        if (ny < 0 || ny >= M.tiles_y) {
            if (Q.per_b) ny = (ny + M.tiles_y) % M.tiles_y;
            else ok = false;
        }
        if (ok) nbr = nx + ny * M.tiles_x;
    }
    // halo cells staged by this thread: LDS cell and source site (-1: zero pad)
    int hcell[KH], hsrc[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        const int h = tid + k * NT;
        hcell[k] = -1;
        hsrc[k] = -1;
        if (h < HALO) {
            int px, py;
            ring_cell<2 * R, TX, TY>(h, px, py);
            hcell[k] = py * WN + px;
            bool in = true;
            const int gx = wrap_once(x0 - 2 * R + px, Q.na, Q.per_a, in);
            const int gy = wrap_once(y0 - 2 * R + py, Q.nb, Q.per_b, in);
            if (in) hsrc[k] = gx + gy * Q.na;
        }
    }

    const unsigned long long step0 = ((unsigned long long)A.key.step_hi << 32) | A.key.step_lo;
    auto set_step = [&](int s) {
        const unsigned long long st = step0 + (unsigned long long)s;
        A.key.step_lo = (uint32_t)st;
        A.key.step_hi = (uint32_t)(st >> 32);
    };
    V3<T> own{b0[gsite], b0[N + gsite], b0[2 * N + gsite]};
    L.sN[own_c] = V4<T>{own.x, own.y, own.z, T(0)};
    set_step(0);
    V3<T> Bown = cell_base<T, S, TX, TY>(C, Q, A, x0, y0, tx + R, ty + R);
    V3<T> Bring{T(0), T(0), T(0)};
    if (rank >= 0 && rank < RING) Bring = cell_base<T, S, TX, TY>(C, Q, A, x0, y0, rpx, rpy);
    if (tid == 0) s_fail = 0;
    __syncthreads();

    for (int s = 0; s < M.n_steps; ++s) {
        // b0 and b1 are written and read by other workgroups during the
        // launch: plain pointers, no restrict
        const T* nin = (s & 1) ? b1 : b0;
        T* nout = (s & 1) ? b0 : b1;
        // 1) predictor of the inner sites (own spins only)
        V3<T> keepA{T(0), T(0), T(0)};
        if (inner) keepA = predict_cell<T, S, NDMI, TX, TY, SOLVER_DEPONDT>(C, Q, A, x0, y0, tx + R, ty + R, L, Bown);
        // 2) the neighbours' n(s) must be in HBM before the halo is read
        if (s > 0 && tid < 64) {
            const bool ok = persist_wait(flags, status, nbr, M.gen + (uint32_t)s, M.spin_limit);
            if (!ok && tid == 0) s_fail = 1;
        }
        __syncthreads();
        if (s_fail) return;
        // 3) halo of n(s)
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            if (hcell[k] < 0) continue;
            V4<T> v{T(0), T(0), T(0), T(0)};
            if (hsrc[k] >= 0) v = V4<T>{nin[hsrc[k]], nin[N + hsrc[k]], nin[2 * N + hsrc[k]], T(0)};
            L.sN[hcell[k]] = v;
        }
        __syncthreads();
        // 4) predictor of the edge sites and of the R-ring around the tile
        if (!inner)
            keepA = predict_cell<T, S, NDMI, TX, TY, SOLVER_DEPONDT>(C, Q, A, x0, y0, tx + R, ty + R, L, Bown);
        else if (rank < RING)
            predict_cell<T, S, NDMI, TX, TY, SOLVER_DEPONDT>(C, Q, A, x0, y0, rpx, rpy, L, Bring);
        __syncthreads();
        // 5) corrector: n(s+1) stays in registers and in the LDS cell of the
        //    site (no other thread reads that cell in this phase) and goes to HBM
        own = correct_cell<T, S, NDMI, TX, TY, SOLVER_DEPONDT>(C, Q, A, tx, ty, L, keepA, Bown);
        L.sN[own_c] = V4<T>{own.x, own.y, own.z, T(0)};
        // agent-scope stores go through to the device coherence point, so
        // the release below finds few dirty L2 lines to write back
        __hip_atomic_store(nout + gsite, own.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(nout + N + gsite, own.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(nout + 2 * N + gsite, own.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // external plus thermal fields of the next step while the stores drain
        if (s + 1 < M.n_steps) {
            set_step(s + 1);
            Bown = cell_base<T, S, TX, TY>(C, Q, A, x0, y0, tx + R, ty + R);
            if (rank >= 0 && rank < RING) Bring = cell_base<T, S, TX, TY>(C, Q, A, x0, y0, rpx, rpy);
        }
        // every wave's stores precede the barrier; the one agent-scope
        // release of the flag store then covers the whole tile
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(flags + (size_t)tile * kFlagStride, M.gen + (uint32_t)(s + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace sp
