// kernels_gneb.hpp -- geodesic nudged elastic band on the GPU (Sec. III.D;
// Appendix F for tangents, distances and projections; Appendix D for the
// velocity-projection minimiser).
//
// The chain holds M images of N spins, image-major, each image SoA.  Images 0
// and M-1 are fixed.  Per velocity-projection iteration (five launches):
//   k_gneb_move       [projection of the previous iteration: v <- (v.F/F.F) F
//                     if v.F > 0 else 0, F_prev <- F]  then
//                     x <- normalise(x + dt v + dt^2/(2m) F_prev)    (interior)
//   k_gneb_grad       g = dH/dn per image, energy partials per block
//                     (k_gneb_grad_shape on the stencil path's tiles)
//   k_gneb_tangent    E of the image and its neighbours from the partials;
//                     improved tangent, per-spin projection; partials of
//                     |tau|^2, g.tau, and squared geodesic angles to image v+1
//   k_gneb_force      |tau|^2, g.tau, l^2 from the partials;
//                     F = -g + (g.t)t, per-spin projected, + k (l_v - l_{v-1}) t
//                     (climbing images: -g + 2 (g.t)t, falling: -g, no spring)
//                     with t = tau/|tau|; v <- v + dt/(2m)(F_prev + F);
//                     chain-wide partials of v.F and F.F
//   k_gneb_sum        v.F, F.F
// k_gneb_project applies the last projection when a run of iterations ends.
// Every reduction is a fixed-order FP64 tree: a row of partials is summed by
// the same thread-strided loop and tree in every workgroup that needs it
// (bit-reproducible, identical everywhere).
#pragma once

#include "kernels_field.hpp"
#include "kernels_reduce.hpp"
#include "kernels_stencil.hpp"

namespace sp {

template <int NV>
__device__ __forceinline__ void block_sums(double* acc) {
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    }
}

// Sum of row `row` of NV-value partials (nblk per row), fixed order; every
// thread receives the result.
template <int NV>
__device__ __forceinline__ void row_sum(const double* __restrict__ part, int nblk, int row, double* out) {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += part[((size_t)row * nblk + b) * NV + k];
    }
    block_sums<NV>(acc);
    __shared__ double bc[NV];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) bc[k] = acc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = bc[k];
    __syncthreads();
}

// Maximum over the block (thread 0 receives it).
__device__ __forceinline__ double block_max(double v) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    return v;
}

struct GnebDims {
    int M;         // images
    int N;         // spins per image
    int nblk;      // blocks per image in the per-site kernels
};

template <typename T>
__global__ void __launch_bounds__(256) k_gneb_move(GnebDims d, T dt, T half_dt2_m, int project,
                                                   const double* __restrict__ vf_ff, const T* __restrict__ F,
                                                   T* __restrict__ x, T* __restrict__ v, T* __restrict__ Fp,
    const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int im = blockIdx.y + 1;   // interior images only
    if (i >= d.N) return;
    const size_t base = (size_t)im * 3 * d.N;
    T scale = T(0);
    if (project) {
        const double vf = vf_ff[0], ff = vf_ff[1];
        scale = (vf > 0.0 && ff > 0.0) ? (T)(vf / ff) : T(0);
    }
    T n[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t q = base + (size_t)c * d.N + i;
        T vq, fq;
        if (project) {
            fq = F[q];
            vq = scale * fq;
            v[q] = vq;
            Fp[q] = fq;
        } else {
            vq = v[q];
            fq = Fp[q];
        }
        n[c] = x[q] + dt * vq + half_dt2_m * fq;
    }
    const T r = T(1) / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) x[base + (size_t)c * d.N + i] = n[c] * r;
}

// Gradient of every image and per-block energy partials (Zeeman linear,
// the other local terms quadratic: e_i = n.(g_Z + (g_K + g_J + g_D)/2)).
template <typename T>
__global__ void __launch_bounds__(256) k_gneb_grad(GnebDims d, Lattice L, BondCoef<double> C, Phys<double> P,
                                                   const T* __restrict__ x, T* __restrict__ g,
                                                   double* __restrict__ part,
    const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    // field and energy in FP64 from the stored spins (type T): the image
    // energies decide the tangent's branch, so they are formed in the
    // reference's precision for both engine precisions; g is stored as T
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int im = blockIdx.y;
    const T* xi = x + (size_t)im * 3 * d.N;
    double acc[1] = {0.0};
    if (i < d.N) {
        const V3<double> ni{(double)xi[i], (double)xi[d.N + i], (double)xi[2 * d.N + i]};
        const FieldTerms<double> f = site_terms<double, T>(L, C, P, xi, i, ni);
        const V3<double> gt = total(f);
        store3(g + (size_t)im * 3 * d.N, d.N, i, V3<T>{(T)gt.x, (T)gt.y, (T)gt.z});
        acc[0] = ni.x * f.z.x + ni.y * f.z.y + ni.z * f.z.z +
                 0.5 * (ni.x * (f.k.x + f.j.x + f.d.x) + ni.y * (f.k.y + f.j.y + f.d.y) +
                        ni.z * (f.k.z + f.j.z + f.d.z)) +
                 gauss_energy(P, ni);
    }
    block_sums<1>(acc);
    if (threadIdx.x == 0) part[(size_t)im * d.nblk + blockIdx.x] = acc[0];
}

// The same gradient and energy partials on the stencil path's tiles, for
// one-atom 2D images with a compile-time stencil whose sides divide into
// 64 x 4 tiles: tile t of an image (256 sites, one per thread) is partial t
// of its row, as block t is in k_gneb_grad.  The image is staged in LDS with
// an R halo as FP64 cells; the terms are those of shape_terms, in FP64 from
// the stored spins.
template <typename T, int S, int NDMI>
__global__ void __launch_bounds__(256) k_gneb_grad_shape(GnebDims d, ShapeCoef<double> C, Site2D<double> Q,
                                                         int tiles_x, const T* __restrict__ x, T* __restrict__ g,
                                                         double* __restrict__ part,
    const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    constexpr int TX = 64, TY = 4, NT = 256;
    constexpr int R = ShapeTab<S>::R, W = TX + 2 * R, H = TY + 2 * R, P = W * H, KST = (P + NT - 1) / NT;
    __shared__ V4<double> sN[P];
    const int im = blockIdx.y, tile = blockIdx.x;
    const int tyi = tile / tiles_x;
    const int x0 = (tile - tyi * tiles_x) * TX, y0 = tyi * TY;
    const int N = d.N, tid = threadIdx.x;
    const T* xi = x + (size_t)im * 3 * N;
    V4<double> st[KST];
#pragma unroll
    for (int k = 0; k < KST; ++k) {
        const int idx = tid + k * NT;
        st[k] = V4<double>{0.0, 0.0, 0.0, 0.0};
        if (idx < P) {
            const int ly = idx / W, lx = idx - ly * W;
            bool in = true;
            const int gx = wrap_once(x0 - R + lx, Q.na, Q.per_a, in);
            const int gy = wrap_once(y0 - R + ly, Q.nb, Q.per_b, in);
            if (in) {
                const int q = gx + gy * Q.na;
                st[k] = V4<double>{(double)xi[q], (double)xi[N + q], (double)xi[2 * N + q], 0.0};
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KST; ++k) {
        const int idx = tid + k * NT;
        if (idx < P) sN[idx] = st[k];
    }
    __syncthreads();
    const int ty = tid / TX, tx = tid - ty * TX;
    const int c = (ty + R) * W + (tx + R);
    const V3<double> ni = lds_cell_xyz(sN, c);
    const FieldTerms<double> f = shape_terms<double, S, NDMI, W>(C, Q, sN, c, ni);
    const V3<double> gt = f.z + f.k + f.j + f.d;
    store3(g + (size_t)im * 3 * N, N, (x0 + tx) + (y0 + ty) * Q.na, V3<T>{(T)gt.x, (T)gt.y, (T)gt.z});
    double acc[1] = {ni.x * f.z.x + ni.y * f.z.y + ni.z * f.z.z +
                     0.5 * (ni.x * (f.k.x + f.j.x + f.d.x) + ni.y * (f.k.y + f.j.y + f.d.y) +
                            ni.z * (f.k.z + f.j.z + f.d.z))};
    block_sums<1>(acc);
    if (tid == 0) part[(size_t)im * d.nblk + tile] = acc[0];
}

// Sum NV-value partials of each of `rows` rows (blocks per row = nblk) in a
// fixed order: out[row*NV + k].
template <int NV>
__global__ void __launch_bounds__(256) k_gneb_sum(const double* __restrict__ part, int nblk, double* __restrict__ out,
    const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    const int row = blockIdx.x;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += part[((size_t)row * nblk + b) * NV + k];
    }
    block_sums<NV>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[row * NV + k] = acc[k];
    }
}

// Tangent of interior images (unnormalised, per-spin projected) and partials
// of |tau|^2, g.tau and the squared great-circle angle to image im+1.
template <typename T>
__global__ void __launch_bounds__(256) k_gneb_tangent(GnebDims d, const T* __restrict__ x, const T* __restrict__ g,
                                                      const double* __restrict__ epart, double* __restrict__ E,
                                                      T* __restrict__ tau, double* __restrict__ part,
    const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int im = blockIdx.y;
    // energies of this image and its neighbours
    double Em = 0.0, E0 = 0.0, Ep = 0.0;
    row_sum<1>(epart, d.nblk, im, &E0);
    if (im > 0 && im + 1 < d.M) {
        row_sum<1>(epart, d.nblk, im - 1, &Em);
        row_sum<1>(epart, d.nblk, im + 1, &Ep);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) E[im] = E0;
    double acc[3] = {0.0, 0.0, 0.0};
    if (i < d.N) {
        const size_t L3 = (size_t)3 * d.N;
        const V3<T> n0 = load3(x + im * L3, d.N, i);
        if (im + 1 < d.M) {
            const V3<T> n1 = load3(x + (im + 1) * L3, d.N, i);
            const V3<T> c = cross(n0, n1);
            // angle in working precision (its inputs are), squared sum in FP64
            const double ang = (double)atan2(sqrt(dot(c, c)), dot(n0, n1));
            acc[2] = ang * ang;
        }
        if (im > 0 && im + 1 < d.M) {
            const V3<T> nm = load3(x + (im - 1) * L3, d.N, i);
            const V3<T> np = load3(x + (im + 1) * L3, d.N, i);
            double wp, wm;
            if (Ep > E0 && E0 > Em) {
                wp = 1.0; wm = 0.0;
            } else if (Ep < E0 && E0 < Em) {
                wp = 0.0; wm = 1.0;
            } else {
                const double d1 = fabs(Ep - E0), d2 = fabs(Em - E0);
                const double dmax = d1 > d2 ? d1 : d2, dmin = d1 > d2 ? d2 : d1;
                if (Ep > Em) { wp = dmax; wm = dmin; } else { wp = dmin; wm = dmax; }
            }
            V3<T> t = T(wp) * (np - n0) + T(wm) * (n0 - nm);
            t = t - dot(t, n0) * n0;
            store3(tau + im * L3, d.N, i, t);
            const V3<T> gi = load3(g + im * L3, d.N, i);
            acc[0] = (double)dot(t, t);
            acc[1] = (double)dot(gi, t);
        }
    }
    block_sums<3>(acc);
    if (threadIdx.x == 0) {
        double* o = part + ((size_t)im * d.nblk + blockIdx.x) * 3;
        o[0] = acc[0];
        o[1] = acc[1];
        o[2] = acc[2];
    }
}

// Forces of interior images, velocity update, chain-wide v.F and F.F partials.
// s3[v] = (|tau|^2, g.tau, l^2) from k_gneb_sum<3>.
// Image types: 0 normal, 1 climbing (no spring, F = -g + 2 (g.t) t),
// 2 falling (no spring, F = -g); all per-spin projected.
template <typename T>
__global__ void __launch_bounds__(256) k_gneb_force(GnebDims d, T k_spring, T dt_2m, int update_v,
                                                    const T* __restrict__ x, const T* __restrict__ g,
                                                    const T* __restrict__ tau, const double* __restrict__ tpart,
                                                    double* __restrict__ s3, const int* __restrict__ types,
                                                    T* __restrict__ F, const T* __restrict__ Fp, T* __restrict__ v,
                                                    double* __restrict__ part,
    double* __restrict__ fmax_part, const int* __restrict__ stop) {
    if (stop && *stop) return;   // the chain has converged: the rest of the run is skipped
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int im = blockIdx.y + 1;
    // |tau|^2, g.tau, l^2 of this image and of the one before
    double s_im[3], s_prev[3];
    row_sum<3>(tpart, d.nblk, im, s_im);
    row_sum<3>(tpart, d.nblk, im - 1, s_prev);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) s3[im * 3 + k] = s_im[k];
        if (im == 1)
            for (int k = 0; k < 3; ++k) s3[k] = s_prev[k];
    }
    double acc[2] = {0.0, 0.0};
    if (i < d.N) {
        const size_t off = (size_t)im * 3 * d.N;
        const double tn2 = s_im[0];
        const double inv = tn2 > 0.0 ? 1.0 / sqrt(tn2) : 0.0;
        const int type = types[im];
        const T cpar = type == 1 ? T(2) : (type == 2 ? T(0) : T(1));
        const T gt = cpar * (T)(s_im[1] * inv);
        const T fs = type == 0 ? (T)(k_spring * (sqrt(s_im[2]) - sqrt(s_prev[2]))) : T(0);
        const V3<T> n = load3(x + off, d.N, i);
        const V3<T> t = T(inv) * load3(tau + off, d.N, i);
        const V3<T> gi = load3(g + off, d.N, i);
        V3<T> fe = gt * t - gi;
        fe = fe - dot(fe, n) * n;
        const V3<T> f = fe + fs * t;
        store3(F + off, d.N, i, f);
        if (update_v) {
            const V3<T> vn = load3(v + off, d.N, i) + dt_2m * (load3(Fp + off, d.N, i) + f);
            store3(v + off, d.N, i, vn);
            acc[0] = (double)dot(vn, f);
        }
        acc[1] = (double)dot(f, f);
    }
    const double f2 = acc[1];
    block_sums<2>(acc);
    if (fmax_part) {
        const double m = block_max(f2);
        if (threadIdx.x == 0) fmax_part[(size_t)(im - 1) * d.nblk + blockIdx.x] = m;
    }
    if (threadIdx.x == 0) {
        double* o = part + ((size_t)(im - 1) * d.nblk + blockIdx.x) * 2;
        o[0] = acc[0];
        o[1] = acc[1];
    }
}

// Convergence test of a chain relaxation: the largest per-spin force
// |F_{v,i}| over the interior images below tol (compared as squares).  Sets
// *stop and records the iteration that passed; later launches of the run
// see *stop and return.
__global__ void __launch_bounds__(256) k_gneb_converged(const double* __restrict__ fmax_part, int n,
                                                        double tol2, int* __restrict__ stop,
                                                        int* __restrict__ stop_iter, int iter) {
    if (*stop) return;
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) m = fmax(m, fmax_part[k]);
    m = block_max(m);
    if (threadIdx.x == 0 && m < tol2) {
        *stop = 1;
        *stop_iter = iter;
    }
}

// Start of a run with a convergence test.
__global__ void k_gneb_clear_stop(int* __restrict__ stop, int* __restrict__ stop_iter) {
    if (threadIdx.x == 0) {
        *stop = 0;
        *stop_iter = -1;
    }
}

// Velocity projection: v <- (v.F / F.F) F if v.F > 0, else 0; F_prev <- F.
template <typename T>
__global__ void __launch_bounds__(256) k_gneb_project(GnebDims d, const double* __restrict__ vf_ff,
                                                      T* __restrict__ v, const T* __restrict__ F,
                                                      T* __restrict__ Fp) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int im = blockIdx.y + 1;
    if (i >= d.N) return;
    const double vf = vf_ff[0], ff = vf_ff[1];
    const T scale = (vf > 0.0 && ff > 0.0) ? (T)(vf / ff) : T(0);
    const size_t off = (size_t)im * 3 * d.N;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t q = off + (size_t)c * d.N + i;
        v[q] = scale * F[q];
        Fp[q] = F[q];
    }
}

}  // namespace sp
