// kernels_tile.hpp -- fused Depondt step on LDS tiles for lattices with a
// basis (Sec. III.A: Bravais lattice with basis), 2D or 3D, with a runtime
// bond table; also 3D one-atom lattices whose bonds match no compile-time
// stencil.
//
// Depondt, Heun or SIB (template SOLVER), as the other fused kernels.
//
// Sites are stored basis-major, i = a + Na (b + Nb (c + Nc beta)), so every
// basis atom is a block of its own.  A workgroup owns a TX x TY x TZ tile of
// cells and all NB atoms in it, one thread per owned site (NB * TX * TY * TZ
// threads; thread t works on atom t / (TX TY TZ), so the atom, and with it
// the bond list, is wavefront-uniform).  Per step:
//   1. stage n(t) of every atom on the tile plus a (2R, 2R, 2RC) halo in LDS
//      as 16-byte cells (periodic axes wrap; beyond an open boundary a zero
//      spin, which adds nothing to a field), every load issued before the
//      first LDS write; the thermal field of the owned site is drawn while
//      the loads are in flight;
//   2. predictor of the owned site (its rotation vector, or Heun slope, and
//      thermal field stay in registers) and of the ring of cells within
//      (R, R, RC) of the tile,
//      spread over the workgroup;
//   3. corrector of the owned site from the predictor field; n(t+dt) is
//      written once.
// HBM traffic: one read and one write of the spins per step.  Bond q of atom
// beta couples it to atom bj[q] of the cell (da[q], db[q], dc[q]) away.
#pragma once

#include "kernels_fused2d.hpp"

namespace sp {

constexpr int kMaxStencilB = 48;   // directed bonds of all basis atoms together

// Bond q of atom beta (bstart[beta] <= q < bstart[beta + 1]) reaches the
// LDS cell offN[q] (spin frame) or offP[q] (predictor frame) away from the
// site's own cell; the host forms both from the bond's target atom and
// cell offset and the frames' pitches.  Each atom's list is padded to a
// multiple of four with bonds of zero coupling to the site's own cell
// (they add exactly zero), so the field loop takes four bonds at a time.
template <typename T>
struct StencilB {
    int nb;
    int bstart[kMaxBasis + 1];
    int offN[kMaxStencilB];
    int offP[kMaxStencilB];
    T J[kMaxStencilB];
    T D[kMaxStencilB][3];
};

template <typename T>
struct SiteB {
    int n[3];
    int per[3];
    T inv_mumuB[kMaxBasis];
    T gZ[kMaxBasis][3];
    T K2[kMaxBasis];
    T Kax[kMaxBasis][3];
    T sigma[kMaxBasis];
};

// Field of atom beta at cell c of an LDS frame whose bond offsets are off[].
// beta is wavefront-uniform, so the bond data are scalar loads.
template <typename T>
__device__ __forceinline__ V3<T> tile_field(const StencilB<T>& S, const SiteB<T>& Q, int beta,
                                            const V4<T>* __restrict__ s, const int* off, int c, V3<T> ni) {
    V3<T> g{Q.gZ[beta][0], Q.gZ[beta][1], Q.gZ[beta][2]};
    const T kn = Q.K2[beta] * (Q.Kax[beta][0] * ni.x + Q.Kax[beta][1] * ni.y + Q.Kax[beta][2] * ni.z);
    g.x -= kn * Q.Kax[beta][0];
    g.y -= kn * Q.Kax[beta][1];
    g.z -= kn * Q.Kax[beta][2];
    const int q1 = S.bstart[beta + 1];
    for (int q0 = S.bstart[beta]; q0 < q1; q0 += 4) {
        // four full-width 16-byte reads in flight together: one empty asm
        // keeps every padding word live (else the compiler narrows each read
        // to 12 bytes), placed after all four so they are not serialised
        V4<T> v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = s[c + off[q0 + k]];
        T J[4], D[4][3];   // the coefficients' scalar loads overlap the LDS reads
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            J[k] = S.J[q0 + k];
            D[k][0] = S.D[q0 + k][0];
            D[k][1] = S.D[q0 + k][1];
            D[k][2] = S.D[q0 + k][2];
        }
        if constexpr (sizeof(T) == 4) asm volatile("" ::"v"(v[0].w), "v"(v[1].w), "v"(v[2].w), "v"(v[3].w));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const V3<T> nj{v[k].x, v[k].y, v[k].z};
            g.x -= J[k] * nj.x + (nj.y * D[k][2] - nj.z * D[k][1]);
            g.y -= J[k] * nj.y + (nj.z * D[k][0] - nj.x * D[k][2]);
            g.z -= J[k] * nj.z + (nj.x * D[k][1] - nj.y * D[k][0]);
        }
    }
    return g;
}

// Wraps a coordinate on a periodic axis (a full modulo: a tile plus halo can
// be wider than a small lattice); false when it leaves an open one.
__device__ __forceinline__ bool tile_coord(int& t, int n, int per) {
    if (t >= 0 && t < n) return true;
    if (!per) return false;
    t %= n;
    if (t < 0) t += n;
    return true;
}

// Ring cell h of the predictor frame (0 <= h < PP - PT): the RC planes
// below and above the tile, then, in each tile plane, R rows above and
// below the tile and R columns either side of each tile row.
template <int TX, int TY, int TZ, int R, int RC>
__device__ __forceinline__ void tile_ring_cell(int h, int& px, int& py, int& pz) {
    constexpr int WP = TX + 2 * R, HP = TY + 2 * R;
    constexpr int SLAB = 2 * RC * WP * HP;
    constexpr int RING2 = 2 * R * WP + 2 * R * TY;
    if (h < SLAB) {
        const int s = h / (WP * HP), r = h - s * (WP * HP);
        pz = s < RC ? s : TZ + s;
        py = r / WP;
        px = r - py * WP;
        return;
    }
    const int k0 = h - SLAB;
    const int layer = k0 / RING2, k = k0 - layer * RING2;
    pz = RC + layer;
    if (k < 2 * R * WP) {
        const int r = k / WP;
        px = k - r * WP;
        py = r < R ? r : TY + r;
    } else {
        const int k2 = k - 2 * R * WP;
        const int r = k2 / (2 * R), q = k2 - r * (2 * R);
        py = R + r;
        px = q < R ? q : TX + q;
    }
}

// One predictor of a cell with field g and thermal field Bth: the spin the
// corrector's field is evaluated on, and (returned through keep) what the
// corrector needs of the site: Depondt n^p = R(A) n, keeps the rotation
// vector w = B + alpha n x B (A = -gp w); Heun n^p = (n + dt n x A)/|...|,
// keeps n x A; SIB the midpoint of the implicit stage with A frozen
// (Appendix C).
template <typename T, int SOLVER>
__device__ __forceinline__ V3<T> tile_predict(V3<T> ni, V3<T> B, const LLGArgs<T>& A, V3<T>& keep) {
    if constexpr (SOLVER == SOLVER_HEUN) {
        keep = cross(ni, llg_A(ni, B, A.gp, A.alpha));
        return normalize3(ni + A.dt * keep);
    } else if constexpr (SOLVER == SOLVER_SIB) {
        return T(0.5) * (ni + sib_stage(ni, llg_A(ni, B, A.gp, A.alpha), A.dt));
    } else {
        keep = llg_w(ni, B, A.alpha);
        return rotate_half(ni, keep, rot_half_factor(A.gp, A.dt));
    }
}

template <typename T, int TX, int TY, int TZ, int R, int RC, int NB, int SOLVER>
__global__ void __launch_bounds__(NB * TX * TY * TZ) k_fused_tile(StencilB<T> S, SiteB<T> Q, LLGArgs<T> A_arg,
                                                                  const int* __restrict__ abort_flag,
                                                                  const T* __restrict__ n, T* __restrict__ nout) {
    constexpr int WN = TX + 4 * R, HN = TY + 4 * R, DN = TZ + 4 * RC;   // spins with the 2R halo
    constexpr int WP = TX + 2 * R, HP = TY + 2 * R, DP = TZ + 2 * RC;   // predictor with the R halo
    constexpr int PN = WN * HN * DN, PP = WP * HP * DP, PT = TX * TY * TZ;
    constexpr int NT = NB * PT;
    constexpr int RING = PP - PT;
    constexpr int RINGP = (RING + 63) / 64 * 64;   // padded so a wavefront's ring cells share one atom
    constexpr int KS = (NB * PN + NT - 1) / NT;    // staged cells per thread
    static_assert(PT % 64 == 0, "a tile must hold whole wavefronts of each atom");
    __shared__ V4<T> sN[NB * PN];
    __shared__ V4<T> sP[NB * PP];
    if (abort_flag && *abort_flag) return;
    const LLGArgs<T> A = resolve_step(A_arg);
    const int na = Q.n[0], nbc = Q.n[1], nc = Q.n[2];
    const int block = na * nbc * nc;
    const int N = block * NB;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int tid = threadIdx.x;

    // 1) issue the loads of n(t) (tile plus 2R halo, every atom)
    V3<T> ld[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        ld[k] = V3<T>{T(0), T(0), T(0)};
        if (idx < NB * PN) {
            const int b = idx / PN, r = idx - b * PN;
            const int lz = r / (WN * HN), rr = r - lz * (WN * HN);
            const int ly = rr / WN, lx = rr - ly * WN;
            int gx = x0 - 2 * R + lx, gy = y0 - 2 * R + ly, gz = z0 - 2 * RC + lz;
            if (tile_coord(gx, na, Q.per[0]) & tile_coord(gy, nbc, Q.per[1]) & tile_coord(gz, nc, Q.per[2])) {
                const int g = gx + na * (gy + nbc * gz) + b * block;
                ld[k] = V3<T>{n[g], n[N + g], n[2 * N + g]};
            }
        }
    }
    // the owned site (its predictor-frame cell wraps like any other)
    const int beta = __builtin_amdgcn_readfirstlane(tid / PT), t = tid - beta * PT;
    const int tz = t / (TX * TY), tr = t - tz * (TX * TY);
    const int ty = tr / TX, tx = tr - ty * TX;
    int ox = x0 + tx, oy = y0 + ty, oz = z0 + tz;
    const bool own_site = ox < na && oy < nbc && oz < nc;
    const bool own_in = tile_coord(ox, na, Q.per[0]) & tile_coord(oy, nbc, Q.per[1]) & tile_coord(oz, nc, Q.per[2]);
    V3<T> Bth{T(0), T(0), T(0)};
    if (A.thermal && own_in) {
        const uint32_t site = (uint32_t)(ox + na * (oy + nbc * oz) + beta * block);
        Bth = Q.sigma[beta] * normals3(thermal_bits(A.key, site), T(0));
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        if (idx < NB * PN) sN[idx] = V4<T>{ld[k].x, ld[k].y, ld[k].z, T(0)};
    }
    __syncthreads();

    // 2) predictor: the owned site, then the ring
    V3<T> keep{T(0), T(0), T(0)};
    {
        const int pc = ((tz + RC) * HP + (ty + R)) * WP + (tx + R);
        V4<T> out{T(0), T(0), T(0), T(0)};
        if (own_in) {
            const int c = ((tz + 2 * RC) * HN + (ty + 2 * R)) * WN + (tx + 2 * R);
            const V3<T> ni = lds_cell_xyz(sN, beta * PN + c);
            const V3<T> g = tile_field(S, Q, beta, sN, S.offN, c, ni);
            const V3<T> o = tile_predict<T, SOLVER>(ni, (-Q.inv_mumuB[beta]) * g + Bth, A, keep);
            out = V4<T>{o.x, o.y, o.z, T(0)};
        }
        sP[beta * PP + pc] = out;
    }
    for (int idx = tid; idx < NB * RINGP; idx += NT) {
        const int b = __builtin_amdgcn_readfirstlane(idx / RINGP), h = idx - b * RINGP;
        if (h >= RING) continue;
        int px, py, pz;
        tile_ring_cell<TX, TY, TZ, R, RC>(h, px, py, pz);
        int gx = x0 - R + px, gy = y0 - R + py, gz = z0 - RC + pz;
        V4<T> out{T(0), T(0), T(0), T(0)};
        if (tile_coord(gx, na, Q.per[0]) & tile_coord(gy, nbc, Q.per[1]) & tile_coord(gz, nc, Q.per[2])) {
            const int c = ((pz + RC) * HN + (py + R)) * WN + (px + R);
            const V3<T> ni = lds_cell_xyz(sN, b * PN + c);
            const V3<T> g = tile_field(S, Q, b, sN, S.offN, c, ni);
            V3<T> B = (-Q.inv_mumuB[b]) * g;
            if (A.thermal) {
                const uint32_t site = (uint32_t)(gx + na * (gy + nbc * gz) + b * block);
                B = B + Q.sigma[b] * normals3(thermal_bits(A.key, site), T(0));
            }
            V3<T> unused;
            const V3<T> o = tile_predict<T, SOLVER>(ni, B, A, unused);
            out = V4<T>{o.x, o.y, o.z, T(0)};
        }
        sP[b * PP + ((pz * HP) + py) * WP + px] = out;
    }
    __syncthreads();

    // 3) corrector of the owned site
    if (!own_site) return;
    const int pc = ((tz + RC) * HP + (ty + R)) * WP + (tx + R);
    const V3<T> npi = lds_cell_xyz(sP, beta * PP + pc);
    const V3<T> g = tile_field(S, Q, beta, sP, S.offP, pc, npi);
    const V3<T> B = (-Q.inv_mumuB[beta]) * g + Bth;
    const V3<T> ni = lds_cell_xyz(sN, beta * PN + ((tz + 2 * RC) * HN + (ty + 2 * R)) * WN + (tx + 2 * R));
    V3<T> o;
    if constexpr (SOLVER == SOLVER_HEUN) {
        o = normalize3(ni + (T(0.5) * A.dt) * (keep + cross(npi, llg_A(npi, B, A.gp, A.alpha))));
    } else if constexpr (SOLVER == SOLVER_SIB) {
        o = renorm_if_float(sib_stage(ni, llg_A(npi, B, A.gp, A.alpha), A.dt));
    } else {
        // about the mean rotation vector: the sum by half the angle factor
        o = renorm_if_float(rotate_half(ni, keep + llg_w(npi, B, A.alpha), T(0.5) * rot_half_factor(A.gp, A.dt)));
    }
    const int gi = ox + na * (oy + nbc * oz) + beta * block;
    store_out(nout + gi, o.x);
    store_out(nout + N + gi, o.y);
    store_out(nout + 2 * N + gi, o.z);
}

// Stand-alone field g = dH/dn (sp_gradient) of the same lattices: every
// atom's tile plus an (R, R, RC) halo staged in LDS as 16-byte cells, every
// load issued before the first LDS write, one thread per owned site; one
// read of n and one write of g per site (24 B per FP32 site).
template <typename T, int TX, int TY, int TZ, int R, int RC, int NB>
__global__ void __launch_bounds__(NB * TX * TY * TZ) k_gradient_tile(StencilB<T> S, SiteB<T> Q,
                                                                     const T* __restrict__ n, T* __restrict__ g) {
    constexpr int WN = TX + 2 * R, HN = TY + 2 * R, DN = TZ + 2 * RC;
    constexpr int PN = WN * HN * DN, PT = TX * TY * TZ, NT = NB * PT;
    constexpr int KS = (NB * PN + NT - 1) / NT;
    static_assert(PT % 64 == 0, "a tile must hold whole wavefronts of each atom");
    __shared__ V4<T> sN[NB * PN];
    const int na = Q.n[0], nbc = Q.n[1], nc = Q.n[2];
    const int block = na * nbc * nc;
    const int N = block * NB;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    const int tid = threadIdx.x;
    V3<T> ld[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        ld[k] = V3<T>{T(0), T(0), T(0)};
        if (idx < NB * PN) {
            const int b = idx / PN, r = idx - b * PN;
            const int lz = r / (WN * HN), rr = r - lz * (WN * HN);
            const int ly = rr / WN, lx = rr - ly * WN;
            int gx = x0 - R + lx, gy = y0 - R + ly, gz = z0 - RC + lz;
            if (tile_coord(gx, na, Q.per[0]) & tile_coord(gy, nbc, Q.per[1]) & tile_coord(gz, nc, Q.per[2])) {
                const int gi = gx + na * (gy + nbc * gz) + b * block;
                ld[k] = V3<T>{n[gi], n[N + gi], n[2 * N + gi]};
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int idx = tid + k * NT;
        if (idx < NB * PN) sN[idx] = V4<T>{ld[k].x, ld[k].y, ld[k].z, T(0)};
    }
    __syncthreads();
    const int beta = __builtin_amdgcn_readfirstlane(tid / PT), t = tid - beta * PT;
    const int tz = t / (TX * TY), tr = t - tz * (TX * TY);
    const int ty = tr / TX, tx = tr - ty * TX;
    const int ox = x0 + tx, oy = y0 + ty, oz = z0 + tz;
    if (ox >= na || oy >= nbc || oz >= nc) return;
    const int c = ((tz + RC) * HN + (ty + R)) * WN + (tx + R);
    const V3<T> gv = tile_field(S, Q, beta, sN, S.offN, c, lds_cell_xyz(sN, beta * PN + c));
    const int gi = ox + na * (oy + nbc * oz) + beta * block;
    store_out(g + gi, gv.x);
    store_out(g + N + gi, gv.y);
    store_out(g + 2 * N + gi, gv.z);
}

}  // namespace sp
