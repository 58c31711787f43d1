// kernels_fused3d.hpp -- fused LLG step (Depondt, Heun or SIB) for one-atom
// simple-cubic lattices with a compile-time neighbour stencil, streamed
// plane by plane along c (2.5D blocking).
//
// A workgroup owns a TX x TY column of the lattice over ZC consecutive
// planes.  It marches along c keeping rings of four planes in LDS: n(t) with
// a 2R halo in a and b, and three planes of predictor output with an R halo.  Iteration
// k stores n(t) plane k+1 (loaded into registers one iteration earlier) and
// issues the loads of plane k+2, computes the predictor of plane k (tile + R
// halo; needs n(t) planes k-1..k+1) and the corrector of plane k-1 (needs
// predictor planes k-2..k), which is written once to HBM.  Only two extra
// predictor planes per column are recomputed (instead of a full 3D halo),
// and each thread keeps the rotation vector (Depondt) or slope (Heun) and the thermal
// field of its own site from the predictor of a plane to its corrector one
// iteration later.
#pragma once

#include "kernels_fused2d.hpp"
#include "kernels_reduce.hpp"

namespace sp {

enum Shape3D { SH3_SC1 = 0, SH3_SC2, SH3_SC3, SH3_COUNT };

template <int S>
struct ShapeTab3;

// simple cubic: shells at 1, sqrt2, sqrt3 lattice constants
template <>
struct ShapeTab3<SH3_SC1> {
    static constexpr int NB = 6, NS = 1, R = 1, NB0 = 6;
    static constexpr int da[NB] = {1, -1, 0, 0, 0, 0};
    static constexpr int db[NB] = {0, 0, 1, -1, 0, 0};
    static constexpr int dc[NB] = {0, 0, 0, 0, 1, -1};
    static constexpr int sh[NB] = {0, 0, 0, 0, 0, 0};
};
template <>
struct ShapeTab3<SH3_SC2> {
    static constexpr int NB = 18, NS = 2, R = 1, NB0 = 6;
    static constexpr int da[NB] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int db[NB] = {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int dc[NB] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int sh[NB] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
};
template <>
struct ShapeTab3<SH3_SC3> {
    static constexpr int NB = 26, NS = 3, R = 1, NB0 = 6;
    static constexpr int da[NB] = {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                   1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int db[NB] = {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                   1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int dc[NB] = {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                   1, -1, -1, 1, 1, -1, 1, -1};
    static constexpr int sh[NB] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                   2, 2, 2, 2, 2, 2, 2, 2};
};

// Run-time coefficients in shape order (DMI vectors may point anywhere).
template <typename T>
struct ShapeCoef3 {
    T J[4];
    T Dx[8], Dy[8], Dz[8];   // first-shell bonds only
    T D0;                    // the bulk form: D_b = D0 r_b on the six first-shell bonds
};

// The same coefficients divided by mu mu_B, for the step kernel: its bond
// sums then give the field B = -dH/dn / (mu mu_B) in Tesla directly, with
// the external field as their starting value.
template <typename T>
struct StepCoef3 {
    T J[4];
    T Dx[8], Dy[8], Dz[8];
    T D0;
    T K2;        // 2K / (mu mu_B)
    T Bext[3];   // external field (Tesla)
};

// DMI of the streamed step kernel: none; any vectors on the first shell; or
// the bulk form D0 r_b (r_b the bond direction) on the six nearest
// neighbours, whose sum over the bonds is
//   sum_b n_b x D0 r_b = D0 [(n_+x - n_-x) x x + (n_+y - n_-y) x y + (n_+z - n_-z) x z]
// (three differences instead of six cross products).
enum Dmi3 { DK_NONE = 0, DK_GENERAL = 1, DK_BULK = 2 };

struct Site3D {
    int nc, per_c;
    int zc;                  // planes per workgroup
    int tiles_x, tiles_y;
    int xcd_bands;           // 1: each XCD gets a contiguous range of work items (count divisible by 8)
};

template <typename T, int S, int TX, int TY>
struct PlaneLDS {
    static constexpr int R = ShapeTab3<S>::R;
    static constexpr int WN = TX + 4 * R, HN = TY + 4 * R, PN = WN * HN;   // n(t) plane + 2R halo
    static constexpr int WP = TX + 2 * R, HP = TY + 2 * R, PP = WP * HP;   // predictor plane + R halo
    V4<T> sN[4][PN];
    V4<T> sP[3][PP];   // predictor plane k lives in slot k mod 3
};

// Field B = -dH/dn / (mu mu_B) (Tesla) of one site from its 3 x 3 x 3
// neighbourhood in LDS, starting from base (the external plus thermal
// field): bm, b0 and bp point at cell (-1, -1) of the site's row in the
// planes below, at and above it (row pitch W), so every neighbour is a
// non-negative compile-time offset from one of three base addresses.
// Neighbours are read six at a time as full 16-byte cells, with one empty
// asm after each group keeping the padding words live (else each read is
// narrowed to 12 bytes); a group's reads are in flight together.  Shell
// sums start from their first neighbour; each coefficient (a scalar
// register) then enters one multiply-add per component.  AN: the
// anisotropy term is formed (off when K = 0).
template <typename T, int S, int DK, int W, bool AN>
__device__ __forceinline__ V3<T> shape_B3(const StepCoef3<T>& C, const Site2D<T>& Q, const V4<T>* __restrict__ bm,
                                          const V4<T>* __restrict__ b0, const V4<T>* __restrict__ bp, V3<T> ni,
                                          V3<T> base) {
    using SH = ShapeTab3<S>;
    static_assert(SH::da[0] == 1 && SH::da[1] == -1 && SH::db[2] == 1 && SH::db[3] == -1 && SH::dc[4] == 1 &&
                      SH::dc[5] == -1,
                  "first six bonds are +x, -x, +y, -y, +z, -z");
    constexpr int G = 6;
    V3<T> acc[SH::NS];
    V3<T> B = base;
    V3<T> nn[6];
#pragma unroll
    for (int q0 = 0; q0 < SH::NB; q0 += G) {
        V4<T> v[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int q = q0 + k;
            if (q < SH::NB) {
                const V4<T>* b = SH::dc[q] < 0 ? bm : (SH::dc[q] > 0 ? bp : b0);
                v[k] = b[(SH::da[q] + 1) + (SH::db[q] + 1) * W];
            } else {
                v[k] = v[0];
            }
        }
        if constexpr (sizeof(T) == 4)
            asm volatile("" ::"v"(v[0].w), "v"(v[1].w), "v"(v[2].w), "v"(v[3].w), "v"(v[4].w), "v"(v[5].w));
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int q = q0 + k;
            if (q < SH::NB) {
                const V3<T> x{v[k].x, v[k].y, v[k].z};
                const int s = SH::sh[q];
                if (first_of_shell<SH>(q)) {
                    acc[s] = x;
                } else {
                    acc[s].x += x.x;
                    acc[s].y += x.y;
                    acc[s].z += x.z;
                }
                if constexpr (DK == DK_GENERAL) {
                    if (q < SH::NB0) {
                        // + n_j x D
                        B.x += x.y * C.Dz[q] - x.z * C.Dy[q];
                        B.y += x.z * C.Dx[q] - x.x * C.Dz[q];
                        B.z += x.x * C.Dy[q] - x.y * C.Dx[q];
                    }
                }
                if (q < 6) nn[q] = x;
            }
        }
    }
    if constexpr (DK == DK_BULK) {
        B.x += C.D0 * ((nn[4].y - nn[5].y) - (nn[2].z - nn[3].z));
        B.y += C.D0 * ((nn[0].z - nn[1].z) - (nn[4].x - nn[5].x));
        B.z += C.D0 * ((nn[2].x - nn[3].x) - (nn[0].y - nn[1].y));
    }
    if constexpr (AN) {
        const T kn = C.K2 * (Q.Kax[0] * ni.x + Q.Kax[1] * ni.y + Q.Kax[2] * ni.z);
        B.x += kn * Q.Kax[0];
        B.y += kn * Q.Kax[1];
        B.z += kn * Q.Kax[2];
    }
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) {
        B.x += C.J[s] * acc[s].x;
        B.y += C.J[s] * acc[s].y;
        B.z += C.J[s] * acc[s].z;
    }
    return B;
}

// Plane index with periodic wrap, or in = false outside an open lattice.
__device__ __forceinline__ int wrap_plane(int z, int nc, int per, bool& in) {
    if (z >= 0 && z < nc) return z;
    if (!per) {
        in = false;
        return 0;
    }
    z %= nc;
    return z < 0 ? z + nc : z;
}

// PER: every axis periodic (the lattice wraps, no cell is ever outside it),
// so the boundary tests and the zero fills of outside cells are compiled
// out; the host takes it only when 3N floats have 32-bit byte offsets, so
// sites are addressed by 32-bit offsets from the three component bases
// (scalar base + vector offset loads and stores, no 64-bit address math).
template <typename T, int S, int DK, int TX, int TY, int SOLVER, bool AN, bool PER = false>
__global__ void __launch_bounds__(TX * TY) k_fused3d_shape(StepCoef3<T> C, Site2D<T> Q, Site3D Z, LLGArgs<T> A_arg,
                                                            const int* __restrict__ abort_flag,
                                                            const T* __restrict__ n, T* __restrict__ nout) {
    // The abort word and the step of a replayed graph are both consumed (by
    // an empty asm) before the branch on the first, so their loads are in
    // flight together instead of one after the other.
    int abort_now = 0;
    if (abort_flag) abort_now = *abort_flag;
    const LLGArgs<T> A = resolve_step(A_arg);
    asm volatile("" ::"s"(abort_now), "s"(A.key.step_lo), "s"(A.key.step_hi));
    if (abort_now) return;
    const T hrot = rot_half_factor(A.gp, A.dt);
    const V3<T> Bext{C.Bext[0], C.Bext[1], C.Bext[2]};
    using PL = PlaneLDS<T, S, TX, TY>;
    constexpr int R = PL::R, WN = PL::WN, PN = PL::PN, WP = PL::WP, PP = PL::PP;
    static_assert(R == 1, "one-cell stencil reach");
    constexpr int NT = TX * TY;
    constexpr int RING = PP - TX * TY;
    constexpr int KST = (PN + NT - 1) / NT;
    constexpr int KRG = (RING + NT - 1) / NT;
    __shared__ PL L;
    const int tid = threadIdx.x;
    const int tiles_xy = Z.tiles_x * Z.tiles_y;
    // workgroups are dealt to the 8 XCDs round-robin: give each XCD a
    // contiguous range of (chunk, tile) items, so that neighbouring columns,
    // which stream through the planes in step, share one L2 for their halos
    int item = blockIdx.x;
    if (Z.xcd_bands) item = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int zchunk = item / tiles_xy;
    const int txy = item - zchunk * tiles_xy;
    const int ty0 = txy / Z.tiles_x;
    const int x0 = (txy - ty0 * Z.tiles_x) * TX, y0 = ty0 * TY;
    const int z0 = zchunk * Z.zc;
    const int z1 = min(z0 + Z.zc, Z.nc);
    const int NA = Q.na, NBB = Q.nb;
    const long long plane = (long long)NA * NBB;
    const long long N = plane * Z.nc;
    const int tx = tid % TX, tyy = tid / TX;
    const T* const nx = n;
    const T* const ny = n + N;
    const T* const nz = n + 2 * N;
    T* const ox_ = nout;
    T* const oy_ = nout + N;
    T* const oz_ = nout + 2 * N;
    // predictor ring slot of plane z (z >= -2)
    auto pslot = [](int z) { return (z + 3) % 3; };

    // Everything in a and b is the same on every plane: the staged cells'
    // in-plane offsets and in-sample flags, the predictor cells this thread
    // owns (its site and its ring cells) and their LDS positions.
    const int per_a = PER ? 1 : Q.per_a, per_b = PER ? 1 : Q.per_b, per_c = PER ? 1 : Z.per_c;
    long long ld_off[KST];
    bool ld_in[KST];
#pragma unroll
    for (int k = 0; k < KST; ++k) {
        const int idx = tid + k * NT;
        const int ly = idx / WN, lx = idx - ly * WN;
        bool in = idx < PN;
        const int gx = wrap_once(x0 - 2 * R + lx, NA, per_a, in);
        const int gy = wrap_once(y0 - 2 * R + ly, NBB, per_b, in);
        ld_off[k] = gx + (long long)NA * gy;
        ld_in[k] = in;
    }
    // predictor cell (px, py): LDS cell of its n(t) (pitch WN, halo 2R), of
    // its output (pitch WP, halo R), in-plane offset and flag
    bool pi_in = true;
    long long pi_off;
    {
        const int gx = wrap_once(x0 + tx, NA, per_a, pi_in);
        const int gy = wrap_once(y0 + tyy, NBB, per_b, pi_in);
        pi_off = gx + (long long)NA * gy;
    }
    int rg_px[KRG], rg_py[KRG];
    bool rg_in[KRG];
    long long rg_off[KRG];
#pragma unroll
    for (int q = 0; q < KRG; ++q) {
        const int h = tid + q * NT;
        rg_in[q] = h < RING;
        int px = 0, py = 0;
        if (rg_in[q]) ring_cell<R, TX, TY>(h, px, py);
        const int gx = wrap_once(x0 - R + px, NA, per_a, rg_in[q]);
        const int gy = wrap_once(y0 - R + py, NBB, per_b, rg_in[q]);
        rg_px[q] = px;
        rg_py[q] = py;
        rg_off[q] = gx + (long long)NA * gy;
    }
    const bool own_site = x0 + tx < NA && y0 + tyy < NBB;

    // n(t) of plane z (tile + 2R halo): load into registers, later store into
    // ring slot z & 3 (the loads of plane k+2 fly while planes k and k-1 are
    // computed)
    auto load_plane = [&](int z, V3<T>* st) {
        bool zin = true;
        const long long gz = wrap_plane(z, Z.nc, per_c, zin) * plane;
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            // (cells past the staged frame are never stored)
            if constexpr (!PER) st[k] = V3<T>{T(0), T(0), T(0)};
            if (zin && ld_in[k]) {
                if constexpr (PER) {
                    const uint32_t b = ((uint32_t)ld_off[k] + (uint32_t)gz) * (uint32_t)sizeof(T);
                    st[k] = V3<T>{at_byte(nx, b), at_byte(ny, b), at_byte(nz, b)};
                } else {
                    const long long g = ld_off[k] + gz;
                    st[k] = V3<T>{n[g], n[N + g], n[2 * N + g]};
                }
            }
        }
    };
    auto store_plane = [&](int z, const V3<T>* st) {
        V4<T>* dst = L.sN[z & 3];
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            const int idx = tid + k * NT;
            if (idx < PN) dst[idx] = V4<T>{st[k].x, st[k].y, st[k].z, T(0)};
        }
    };
    // thermal field of a predictor cell of plane z (in-plane offset off)
    auto thermal = [&](bool in, long long off, long long gz) -> V3<T> {
        if (!A.thermal || !in) return V3<T>{T(0), T(0), T(0)};
        return Q.sigma * normals3(thermal_bits(A.key, (uint32_t)(off + gz)), T(0));
    };
    // predictor of predictor cell (px, py) of plane z into predictor slot
    // pslot(z), base the cell's external plus thermal field; returns what
    // the corrector needs of the site
    auto predict = [&](int px, int py, bool in, int z, V3<T> base) -> V3<T> {
        V4<T> out{T(0), T(0), T(0), T(0)};
        V3<T> keep{T(0), T(0), T(0)};
        if (in) {
            const int c = (py + R) * WN + (px + R);
            const V3<T> ni = lds_cell_xyz(L.sN[z & 3], c);
            const int cb = c - WN - 1;
            const V3<T> B = shape_B3<T, S, DK, WN, AN>(C, Q, L.sN[(z - 1) & 3] + cb, L.sN[z & 3] + cb,
                                                       L.sN[(z + 1) & 3] + cb, ni, base);
            V3<T> o;
            if constexpr (SOLVER == SOLVER_HEUN) {
                keep = cross(ni, llg_A(ni, B, A.gp, A.alpha));
                o = normalize3(ni + A.dt * keep);
            } else if constexpr (SOLVER == SOLVER_SIB) {
                o = T(0.5) * (ni + sib_stage(ni, llg_A(ni, B, A.gp, A.alpha), A.dt));
            } else {
                keep = llg_w(ni, B, A.alpha);
                o = rotate_half(ni, keep, hrot);
            }
            out = V4<T>{o.x, o.y, o.z, T(0)};
        }
        L.sP[pslot(z)][py * WP + px] = out;
        return keep;
    };

    // pipeline: predictor planes z0-1 .. z1, corrector planes z0 .. z1-1.
    // The first three planes are loaded together: at launch every workgroup
    // waits for them, so their loads share one memory round trip.
    V3<T> st[KST];
    {
        V3<T> s0[KST], s1[KST];
        load_plane(z0 - 2, s0);
        load_plane(z0 - 1, s1);
        load_plane(z0, st);
        store_plane(z0 - 2, s0);
        store_plane(z0 - 1, s1);
    }
    V3<T> keepA{T(0), T(0), T(0)}, keepB{T(0), T(0), T(0)};   // of the previous plane (keepB: base field)
    const int cP = (tyy + R) * WP + (tx + R);                  // the site's predictor cell
    const int cN = (tyy + 2 * R) * WN + (tx + 2 * R);          // the site's n(t) cell
    for (int k = z0 - 1; k <= z1; ++k) {
        bool zin = true;
        const long long gz = wrap_plane(k, Z.nc, per_c, zin) * plane;
        // external plus thermal fields of this thread's cells of plane k,
        // then stage n(t) plane k+1.  The empty asm keeps the thermal draws
        // inside the branch: left
        // free, the compiler moves the ring cells' draw into the predictor and
        // runs it at T = 0 too, selecting zero afterwards.
        V3<T> bI = Bext;
        V3<T> bR[KRG];
#pragma unroll
        for (int q = 0; q < KRG; ++q) bR[q] = Bext;
        if (A.thermal) {
            bI = Bext + thermal(zin && pi_in, pi_off, gz);
#pragma unroll
            for (int q = 0; q < KRG; ++q) {
                bR[q] = Bext + thermal(zin && rg_in[q], rg_off[q], gz);
                asm volatile("" : "+v"(bR[q].x), "+v"(bR[q].y), "+v"(bR[q].z));
            }
        }
        store_plane(k + 1, st);
        if (k + 2 <= z1 + 1) load_plane(k + 2, st);
        __syncthreads();
        const V3<T> aI = predict(tx + R, tyy + R, zin && pi_in, k, bI);
#pragma unroll
        for (int q = 0; q < KRG; ++q)
            if (tid + q * NT < RING) predict(rg_px[q], rg_py[q], PER || (zin && rg_in[q]), k, bR[q]);
        __syncthreads();
        // corrector of plane k-1
        const int zc = k - 1;
        if (zc >= z0 && zc < z1 && own_site) {
            const V3<T> npi = lds_cell_xyz(L.sP[pslot(zc)], cP);
            const int cb = cP - WP - 1;
            const V3<T> B = shape_B3<T, S, DK, WP, AN>(C, Q, L.sP[pslot(zc - 1)] + cb, L.sP[pslot(zc)] + cb,
                                                       L.sP[pslot(zc + 1)] + cb, npi, keepB);
            const V3<T> ni = lds_cell_xyz(L.sN[zc & 3], cN);
            V3<T> o;
            if constexpr (SOLVER == SOLVER_HEUN) {
                o = normalize3(ni + (T(0.5) * A.dt) * (keepA + cross(npi, llg_A(npi, B, A.gp, A.alpha))));
            } else if constexpr (SOLVER == SOLVER_SIB) {
                o = renorm_if_float(sib_stage(ni, llg_A(npi, B, A.gp, A.alpha), A.dt));
            } else {
                // about the mean rotation vector: the sum by half the angle factor
                o = renorm_if_float(rotate_half(ni, keepA + llg_w(npi, B, A.alpha), T(0.5) * hrot));
            }
            if constexpr (PER) {
                const uint32_t b = ((uint32_t)pi_off + (uint32_t)zc * (uint32_t)plane) * (uint32_t)sizeof(T);
                store_out(ptr_byte(ox_, b), o.x);
                store_out(ptr_byte(oy_, b), o.y);
                store_out(ptr_byte(oz_, b), o.z);
            } else {
                const long long gi = pi_off + (long long)zc * plane;
                store_out(nout + gi, o.x);
                store_out(nout + N + gi, o.y);
                store_out(nout + 2 * N + gi, o.z);
            }
        }
        keepA = aI;
        keepB = bI;
    }
}

// The four local terms of dH/dn of a site whose own plane sits in slot 1 of
// `planes` (slots 0 and 2: planes c - 1 and c + 1) at LDS cell c (pitch W),
// kept apart for the energy per term: the sums of shape_field3 (Sec. III.A).
template <typename T, int S, int NDMI, int W, int PL>
__device__ __forceinline__ FieldTerms<T> shape_terms3(const ShapeCoef3<T>& C, const Site2D<T>& Q,
                                                      const V4<T> (*planes)[PL], int c, V3<T> ni) {
    using SH = ShapeTab3<S>;
    V3<T> acc[SH::NS];
#pragma unroll
    for (int s = 0; s < SH::NS; ++s) acc[s] = V3<T>{T(0), T(0), T(0)};
    V3<T> dm{T(0), T(0), T(0)};   // sum of n_j x D over the DMI bonds
#pragma unroll
    for (int q = 0; q < SH::NB; ++q) {
        const V3<T> v = lds_cell_xyz(planes[1 + SH::dc[q]], c + SH::da[q] + SH::db[q] * W);
        acc[SH::sh[q]] = acc[SH::sh[q]] + v;
        if (q < NDMI) {
            dm.x += v.y * C.Dz[q] - v.z * C.Dy[q];
            dm.y += v.z * C.Dx[q] - v.x * C.Dz[q];
            dm.z += v.x * C.Dy[q] - v.y * C.Dx[q];
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
    f.d = T(-1) * dm;
    f.q = V3<T>{T(0), T(0), T(0)};
    return f;
}

// Stage 1 of the observables (kernels_reduce.hpp) for one-atom simple-cubic
// lattices with a compile-time stencil: a work item is a TX x TY tile of one
// plane c, staged with planes c - 1 and c + 1 and a one-cell halo in LDS;
// workgroups take items blockIdx.x, blockIdx.x + gridDim.x, ... and fold the
// energy per term, torque, mean spin and norm deviation of their sites into
// one row of partials.  No dipole term and no on-site potentials on this
// path.
template <typename T, int S, int NDMI, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_observe_shape3(ShapeCoef3<T> C, Site2D<T> Q, int nc, int per_c,
                                                             int tiles_x, int tiles_y, const T* __restrict__ n,
                                                             double* __restrict__ partials) {
    constexpr int NT = TX * TY;
    static_assert(ShapeTab3<S>::R == 1, "one-cell halo");
    static_assert(NT % 64 == 0, "whole wavefronts");
    constexpr int W = TX + 2, H = TY + 2, P = W * H, KST = (3 * P + NT - 1) / NT;
    __shared__ V4<T> sN[3][P];
    const int ntiles = tiles_x * tiles_y;
    const long long items = (long long)ntiles * nc;
    const long long plane = (long long)Q.na * Q.nb;
    const long long N = plane * nc;
    const int tid = threadIdx.x;
    const int ty = tid / TX, tx = tid - ty * TX;
    double acc[OBS_NVALS];
#pragma unroll
    for (int k = 0; k < OBS_NVALS; ++k) acc[k] = 0.0;
    for (long long w = blockIdx.x; w < items; w += gridDim.x) {
        const int z = (int)(w / ntiles), tile = (int)(w - (long long)z * ntiles);
        const int tyi = tile / tiles_x;
        const int x0 = (tile - tyi * tiles_x) * TX, y0 = tyi * TY;
        V4<T> st[KST];
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            const int idx = tid + k * NT;
            st[k] = V4<T>{T(0), T(0), T(0), T(0)};
            if (idx < 3 * P) {
                const int s = idx / P, r = idx - s * P;
                const int ly = r / W, lx = r - ly * W;
                bool in = true;
                const int gz = wrap_plane(z - 1 + s, nc, per_c, in);
                const int gx = wrap_once(x0 - 1 + lx, Q.na, Q.per_a, in);
                const int gy = wrap_once(y0 - 1 + ly, Q.nb, Q.per_b, in);
                if (in) {
                    const long long q = gx + (long long)Q.na * gy + plane * gz;
                    st[k] = V4<T>{n[q], n[N + q], n[2 * N + q], T(0)};
                }
            }
        }
        __syncthreads();   // the previous item's cells are no longer read
#pragma unroll
        for (int k = 0; k < KST; ++k) {
            const int idx = tid + k * NT;
            if (idx < 3 * P) sN[idx / P][idx % P] = st[k];
        }
        __syncthreads();
        if (x0 + tx >= Q.na || y0 + ty >= Q.nb) continue;
        const int c = (ty + 1) * W + (tx + 1);
        const V3<T> ni = lds_cell_xyz(sN[1], c);
        const FieldTerms<T> f = shape_terms3<T, S, NDMI, W, P>(C, Q, sN, c, ni);
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
    block_reduce<NT / 64>(acc);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < OBS_NVALS; ++k) partials[blockIdx.x * OBS_NVALS + k] = acc[k];
    }
}

}  // namespace sp
