// kernels_field.hpp -- effective-field (energy-gradient) evaluation and the
// Depondt LLG step kernels.
//
// The gradient g_i = dH/dn_i of the extended Heisenberg Hamiltonian
// (Sec. III.A) in the embedding space:
//   Zeeman      -mu_i mu_B B
//   anisotropy  -2 K_i (K_hat_i . n_i) K_hat_i
//   exchange    -sum_j J_ij n_j
//   DMI         -sum_j n_j x D_ij
//   dipole      C_dd mu_i sum_j mu_j [n_j - 3 (n_j . r_ij) r_ij] / r_ij^3
// The effective field in Tesla is B_i = -g_i / (mu_i mu_B).
//
// Two step paths:
//   * "twopass": any lattice/basis/boundary, plus the dipole term.  One
//     kernel computes the predictor (and stores A_i), a second computes the
//     corrector.  Neighbour lookups wrap/drop through integer coordinates.
//   * "fused2d": one-atom-basis 2D lattices.  One kernel per step: a
//     workgroup stages its spin tile plus a 2R halo in LDS, computes the
//     predictor on the tile plus an R halo into LDS, then the corrector on
//     the tile, writing n(t+dt) once.  HBM traffic is one read and one write
//     of the spin array per step.
#pragma once

#include "device_common.hpp"

namespace sp {

constexpr int kMaxGauss = 16;

// Per-basis physical constants in engine precision.
template <typename T>
struct Phys {
    int nb;
    int ng;                 // on-site Gaussian potentials (same on every site)
    T ga[kMaxGauss];        // amplitude a_k (meV)
    T gis2[kMaxGauss];      // 1 / sigma_k^2
    T gc[kMaxGauss][3];     // unit centre directions
    T mumuB[kMaxBasis];     // mu_b mu_B (meV/T)
    T gZ[kMaxBasis][3];     // Zeeman gradient -mu_b mu_B B
    T K2[kMaxBasis];        // 2 K_b
    T Kax[kMaxBasis][3];    // unit anisotropy axes
    T sigma[kMaxBasis];     // thermal field std-dev per component (Tesla), 0 at T = 0
};

template <typename T>
struct LLGArgs {
    T gp;      // gamma / (1 + alpha^2)
    T alpha;
    T dt;
    int thermal;
    ThermalKey key;
    // Replayed step graphs: when set, the Philox step is *step_dev + step_off
    // (the launch's place in its chunk) instead of the step words of key.
    const unsigned long long* step_dev;
    unsigned int step_off;
};

// The launch's own copy of the LLG arguments with the step of a replayed
// graph filled in (one uniform load; unchanged when step_dev is null).
template <typename T>
__device__ __forceinline__ LLGArgs<T> resolve_step(LLGArgs<T> A) {
    if (A.step_dev) {
        const unsigned long long s = *A.step_dev + A.step_off;
        A.key.step_lo = (uint32_t)s;
        A.key.step_hi = (uint32_t)(s >> 32);
    }
    return A;
}

// Generic lattice: bonds of basis atom b are bond[bstart[b] .. bstart[b+1]).
struct Lattice {
    int n[3];
    int per[3];
    int nb;
    int N;
    const int4* bond;   // (beta_j, da, db, dc)
    const int* bstart;
};

template <typename T>
struct BondCoef {
    const T* J;   // [n_bonds]
    const T* D;   // [3 * n_bonds]
};

template <typename T>
struct FieldTerms {
    V3<T> z, k, j, d;
    V3<T> q;   // on-site Gaussian potentials (not quadratic: energy formed separately)
};

__device__ __forceinline__ int wrap_coord(int t, int n, int per, bool& ok) {
    if (t >= 0 && t < n) return t;
    if (!per) {
        ok = false;
        return 0;
    }
    t %= n;
    return t < 0 ? t + n : t;
}

template <typename T>
__device__ __forceinline__ V3<T> load3(const T* __restrict__ v, int N, int i) {
    return V3<T>{v[i], v[N + i], v[2 * N + i]};
}

template <typename T>
__device__ __forceinline__ void store3(T* __restrict__ v, int N, int i, V3<T> a) {
    v[i] = a.x;
    v[N + i] = a.y;
    v[2 * N + i] = a.z;
}

// Local field terms of site i from the bond table (generic lattice), in
// arithmetic type T from spins stored as S (S = T except where an FP32
// engine takes a decision in FP64).
template <typename T, typename S = T>
__device__ FieldTerms<T> site_terms(const Lattice& L, const BondCoef<T>& C, const Phys<T>& P,
                                    const S* __restrict__ n, int i, V3<T> ni) {
    const int na = L.n[0], nbc = L.n[1], nc = L.n[2];
    const int a = i % na;
    const int rem = i / na;
    const int b = rem % nbc;
    const int rem2 = rem / nbc;
    const int c = rem2 % nc;
    const int beta = rem2 / nc;
    FieldTerms<T> f;
    f.z = V3<T>{P.gZ[beta][0], P.gZ[beta][1], P.gZ[beta][2]};
    const V3<T> ax{P.Kax[beta][0], P.Kax[beta][1], P.Kax[beta][2]};
    f.k = (-P.K2[beta] * dot(ax, ni)) * ax;
    f.q = gauss_gradient(P, ni);
    V3<T> gj{T(0), T(0), T(0)}, gd{T(0), T(0), T(0)};
    for (int q = L.bstart[beta]; q < L.bstart[beta + 1]; ++q) {
        const int4 bd = L.bond[q];
        bool ok = true;
        const int ta = wrap_coord(a + bd.y, na, L.per[0], ok);
        const int tb = wrap_coord(b + bd.z, nbc, L.per[1], ok);
        const int tc = wrap_coord(c + bd.w, nc, L.per[2], ok);
        if (!ok) continue;
        const int j = ta + na * (tb + nbc * (tc + nc * bd.x));
        if (j == i) continue;
        const V3<T> nj{(T)n[j], (T)n[L.N + j], (T)n[2 * L.N + j]};
        const T J = C.J[q];
        const V3<T> D{C.D[3 * q], C.D[3 * q + 1], C.D[3 * q + 2]};
        gj = gj - J * nj;
        gd = gd - cross(nj, D);
    }
    f.j = gj;
    f.d = gd;
    return f;
}

template <typename T>
__device__ __forceinline__ V3<T> total(const FieldTerms<T>& f) {
    return f.z + f.k + f.j + f.d + f.q;
}

// On-site Gaussian potentials (the single-spin landscape of Appendix G):
// E = sum_k a_k exp(-(1 - n.c_k)^2 / (2 sigma_k^2)), gradient
// sum_k a_k exp(...) (1 - n.c_k) / sigma_k^2 c_k.
template <typename T>
__device__ __forceinline__ V3<T> gauss_gradient(const Phys<T>& P, V3<T> n) {
    V3<T> g{T(0), T(0), T(0)};
    for (int k = 0; k < P.ng; ++k) {
        const V3<T> c{P.gc[k][0], P.gc[k][1], P.gc[k][2]};
        const T d = T(1) - dot(n, c);
        const T f = P.ga[k] * exp(T(-0.5) * d * d * P.gis2[k]) * d * P.gis2[k];
        g = g + f * c;
    }
    return g;
}

template <typename T>
__device__ __forceinline__ double gauss_energy(const Phys<T>& P, V3<T> n) {
    double e = 0.0;
    for (int k = 0; k < P.ng; ++k) {
        const V3<T> c{P.gc[k][0], P.gc[k][1], P.gc[k][2]};
        const T d = T(1) - dot(n, c);
        e += (double)(P.ga[k] * exp(T(-0.5) * d * d * P.gis2[k]));
    }
    return e;
}

__device__ __forceinline__ int basis_of(const Lattice& L, int i) {
    return i / (L.n[0] * L.n[1] * L.n[2]);
}

// g = dH/dn for every site (plus an optional precomputed dipole gradient).
template <typename T>
__global__ void __launch_bounds__(256) k_gradient(Lattice L, BondCoef<T> C, Phys<T> P,
                                                  const T* __restrict__ n, const T* __restrict__ gdd,
                                                  T* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.N) return;
    const V3<T> ni = load3(n, L.N, i);
    V3<T> gi = total(site_terms(L, C, P, n, i, ni));
    if (gdd) gi = gi + load3(gdd, L.N, i);
    store3(g, L.N, i, gi);
}

// ----------------------------------------------------------- two-pass path
// Predictor, with A_i = -gp (B_i + alpha n_i x B_i), B_i = -g_i/(mu_i mu_B)
// + sigma_i eta_i:
//   Depondt: np = R(A_i(n)) n_i, Aout = A_i;
//   Heun:    np = normalised n_i + dt n_i x A_i, Aout = n_i x A_i;
//   SIB:     np = midpoint (n_i + x_i)/2 with x_i the implicit-midpoint
//            stage with A_i frozen (Appendix C); Aout unused.
template <typename T, int SOLVER>
__global__ void __launch_bounds__(256) k_predict(Lattice L, BondCoef<T> C, Phys<T> P, LLGArgs<T> A_arg,
                                                 const int* __restrict__ abort_flag,
                                                 const T* __restrict__ n, const T* __restrict__ gdd,
                                                 T* __restrict__ np, T* __restrict__ Aout) {
    if (abort_flag && *abort_flag) return;
    const LLGArgs<T> A = resolve_step(A_arg);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.N) return;
    const int beta = basis_of(L, i);
    const V3<T> ni = load3(n, L.N, i);
    V3<T> g = total(site_terms(L, C, P, n, i, ni));
    if (gdd) g = g + load3(gdd, L.N, i);
    const T inv_m = T(1) / P.mumuB[beta];
    V3<T> B = (-inv_m) * g;
    if (A.thermal) B = B + P.sigma[beta] * normals3(thermal_bits(A.key, (uint32_t)i), T(0));
    const V3<T> Ai = llg_A(ni, B, A.gp, A.alpha);
    if constexpr (SOLVER == SOLVER_HEUN) {
        const V3<T> f = cross(ni, Ai);
        store3(Aout, L.N, i, f);
        store3(np, L.N, i, normalize3(ni + A.dt * f));
    } else if constexpr (SOLVER == SOLVER_SIB) {
        store3(np, L.N, i, T(0.5) * (ni + sib_stage(ni, Ai, A.dt)));
    } else {
        store3(Aout, L.N, i, Ai);
        store3(np, L.N, i, renorm_if_float(rotate(ni, (T(-1)) * Ai, A.dt)));
    }
}

// Corrector: A^p from (np, g(np), same eta), then
//   Depondt: n(t+dt) = R((A + A^p)/2) n;
//   Heun:    n(t+dt) = normalised n + dt (f + np x A^p)/2;
//   SIB:     n(t+dt) = midpoint stage of n with A(m) frozen (np holds m).
template <typename T, int SOLVER>
__global__ void __launch_bounds__(256) k_correct(Lattice L, BondCoef<T> C, Phys<T> P, LLGArgs<T> A_arg,
                                                 const int* __restrict__ abort_flag,
                                                 const T* __restrict__ n, const T* __restrict__ np,
                                                 const T* __restrict__ gddp, const T* __restrict__ Ain,
                                                 T* __restrict__ nout) {
    if (abort_flag && *abort_flag) return;
    const LLGArgs<T> A = resolve_step(A_arg);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.N) return;
    const int beta = basis_of(L, i);
    const V3<T> npi = load3(np, L.N, i);
    V3<T> g = total(site_terms(L, C, P, np, i, npi));
    if (gddp) g = g + load3(gddp, L.N, i);
    const T inv_m = T(1) / P.mumuB[beta];
    V3<T> B = (-inv_m) * g;
    if (A.thermal) B = B + P.sigma[beta] * normals3(thermal_bits(A.key, (uint32_t)i), T(0));
    const V3<T> Ap = llg_A(npi, B, A.gp, A.alpha);
    const V3<T> ni = load3(n, L.N, i);
    if constexpr (SOLVER == SOLVER_HEUN) {
        const V3<T> f0 = load3(Ain, L.N, i);
        store3(nout, L.N, i, normalize3(ni + (T(0.5) * A.dt) * (f0 + cross(npi, Ap))));
    } else if constexpr (SOLVER == SOLVER_SIB) {
        store3(nout, L.N, i, renorm_if_float(sib_stage(ni, Ap, A.dt)));
    } else {
        const V3<T> A0 = load3(Ain, L.N, i);
        const V3<T> w = (T(-0.5)) * (A0 + Ap);
        store3(nout, L.N, i, renorm_if_float(rotate(ni, w, A.dt)));
    }
}

// ------------------------------------------------------------ fused 2D path
// One-atom basis, n_cells[2] == 1.  The stencil (bond offsets and
// coefficients) travels in the kernel arguments so every bond's data is
// wavefront-uniform (scalar registers).
template <typename T>
struct Stencil2D {
    int nbond;
    int da[kMaxStencil];
    int db[kMaxStencil];
    T J[kMaxStencil];
    T D[kMaxStencil][3];
};

template <typename T>
struct Site2D {
    int na, nb;
    int per_a, per_b;
    T mumuB, inv_mumuB;
    T gZ[3];
    T K2;
    T Kax[3];
    T sigma;
};

// Field of one site from a tile of spins in LDS (pitch W, SoA planes of size
// PL); centre at LDS index c.  Out-of-sample sites hold zero spins, so open
// boundaries need no test.
template <typename T>
__device__ __forceinline__ V3<T> lds_field(const Stencil2D<T>& S, const Site2D<T>& Q, const T* sx,
                                           const T* sy, const T* sz, int c, int W, V3<T> ni) {
    V3<T> g{Q.gZ[0], Q.gZ[1], Q.gZ[2]};
    const T kn = Q.K2 * (Q.Kax[0] * ni.x + Q.Kax[1] * ni.y + Q.Kax[2] * ni.z);
    g.x -= kn * Q.Kax[0];
    g.y -= kn * Q.Kax[1];
    g.z -= kn * Q.Kax[2];
    for (int q = 0; q < S.nbond; ++q) {
        const int o = c + S.da[q] + S.db[q] * W;
        const T jx = sx[o], jy = sy[o], jz = sz[o];
        const T J = S.J[q];
        const T Dx = S.D[q][0], Dy = S.D[q][1], Dz = S.D[q][2];
        // -J n_j - n_j x D
        g.x -= J * jx + (jy * Dz - jz * Dy);
        g.y -= J * jy + (jz * Dx - jx * Dz);
        g.z -= J * jz + (jx * Dy - jy * Dx);
    }
    return g;
}

template <typename T, int TX, int TY, int R>
__global__ void __launch_bounds__(256) k_depondt_fused2d(Stencil2D<T> S, Site2D<T> Q, LLGArgs<T> A_arg,
                                                         const int* __restrict__ abort_flag,
                                                         const T* __restrict__ n, T* __restrict__ nout) {
    if (abort_flag && *abort_flag) return;
    const LLGArgs<T> A = resolve_step(A_arg);
    constexpr int WN = TX + 4 * R, HN = TY + 4 * R;   // spin tile with 2R halo
    constexpr int WP = TX + 2 * R, HP = TY + 2 * R;   // predictor tile with R halo
    constexpr int PN = WN * HN, PP = WP * HP, PT = TX * TY;
    __shared__ T sN[3 * PN];
    __shared__ T sP[3 * PP];
    __shared__ T sA[3 * PT];
    __shared__ T sB[3 * PT];
    const int N = Q.na * Q.nb;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tid = threadIdx.x;

    // 1) stage n(t) on the tile plus 2R halo; periodic axes wrap, open axes pad with zeros
    for (int idx = tid; idx < PN; idx += 256) {
        const int ly = idx / WN, lx = idx - ly * WN;
        int gx = x0 - 2 * R + lx, gy = y0 - 2 * R + ly;
        bool in = true;
        if (gx < 0 || gx >= Q.na) {
            if (Q.per_a) { gx %= Q.na; if (gx < 0) gx += Q.na; } else in = false;
        }
        if (gy < 0 || gy >= Q.nb) {
            if (Q.per_b) { gy %= Q.nb; if (gy < 0) gy += Q.nb; } else in = false;
        }
        T vx = T(0), vy = T(0), vz = T(0);
        if (in) {
            const int g = gx + gy * Q.na;
            vx = n[g];
            vy = n[N + g];
            vz = n[2 * N + g];
        }
        sN[idx] = vx;
        sN[PN + idx] = vy;
        sN[2 * PN + idx] = vz;
    }
    __syncthreads();

    // 2) predictor on tile plus R halo
    for (int idx = tid; idx < PP; idx += 256) {
        const int py = idx / WP, px = idx - py * WP;
        int gx = x0 - R + px, gy = y0 - R + py;
        bool in = true;
        if (gx < 0 || gx >= Q.na) {
            if (Q.per_a) { gx %= Q.na; if (gx < 0) gx += Q.na; } else in = false;
        }
        if (gy < 0 || gy >= Q.nb) {
            if (Q.per_b) { gy %= Q.nb; if (gy < 0) gy += Q.nb; } else in = false;
        }
        V3<T> out{T(0), T(0), T(0)};
        if (in) {
            const int c = (py + R) * WN + (px + R);
            const V3<T> ni{sN[c], sN[PN + c], sN[2 * PN + c]};
            const V3<T> g = lds_field(S, Q, sN, sN + PN, sN + 2 * PN, c, WN, ni);
            V3<T> B = (-Q.inv_mumuB) * g;
            V3<T> Bth{T(0), T(0), T(0)};
            if (A.thermal) {
                Bth = Q.sigma * normals3(thermal_bits(A.key, (uint32_t)(gx + gy * Q.na)), T(0));
                B = B + Bth;
            }
            const V3<T> Ai = llg_A(ni, B, A.gp, A.alpha);
            out = renorm_if_float(rotate(ni, T(-1) * Ai, A.dt));
            const int tx = px - R, ty = py - R;
            if (tx >= 0 && tx < TX && ty >= 0 && ty < TY) {
                const int t = ty * TX + tx;
                sA[t] = Ai.x; sA[PT + t] = Ai.y; sA[2 * PT + t] = Ai.z;
                sB[t] = Bth.x; sB[PT + t] = Bth.y; sB[2 * PT + t] = Bth.z;
            }
        }
        sP[idx] = out.x;
        sP[PP + idx] = out.y;
        sP[2 * PP + idx] = out.z;
    }
    __syncthreads();

    // 3) corrector on the tile
    for (int t = tid; t < PT; t += 256) {
        const int ty = t / TX, tx = t - ty * TX;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= Q.na || gy >= Q.nb) continue;
        const int c = (ty + R) * WP + (tx + R);
        const V3<T> npi{sP[c], sP[PP + c], sP[2 * PP + c]};
        const V3<T> g = lds_field(S, Q, sP, sP + PP, sP + 2 * PP, c, WP, npi);
        const V3<T> B = (-Q.inv_mumuB) * g + V3<T>{sB[t], sB[PT + t], sB[2 * PT + t]};
        const V3<T> Ap = llg_A(npi, B, A.gp, A.alpha);
        const V3<T> w{T(-0.5) * (sA[t] + Ap.x), T(-0.5) * (sA[PT + t] + Ap.y), T(-0.5) * (sA[2 * PT + t] + Ap.z)};
        const int cn = (ty + 2 * R) * WN + (tx + 2 * R);
        const V3<T> ni{sN[cn], sN[PN + cn], sN[2 * PN + cn]};
        const V3<T> o = renorm_if_float(rotate(ni, w, A.dt));
        const int gi = gx + gy * Q.na;
        nout[gi] = o.x;
        nout[N + gi] = o.y;
        nout[2 * N + gi] = o.z;
    }
}

// Normals exactly as the LLG kernels draw them (for generator tests).
template <typename T>
__global__ void k_normals(ThermalKey key, uint32_t site0, int n_sites, T* __restrict__ eta,
                          uint32_t* __restrict__ raw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_sites) return;
    const U4 b = thermal_bits(key, site0 + (uint32_t)i);
    const V3<T> e = normals3(b, T(0));
    eta[i] = e.x;
    eta[n_sites + i] = e.y;
    eta[2 * n_sites + i] = e.z;
    if (raw) {
        raw[4 * i] = b.x;
        raw[4 * i + 1] = b.y;
        raw[4 * i + 2] = b.z;
        raw[4 * i + 3] = b.w;
    }
}

}  // namespace sp
