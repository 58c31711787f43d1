// kernels_fft.hpp -- dipole-dipole gradient by FFT convolution (Sec. III.A:
// the dipolar term as a convolution over lattice translations, with one
// interaction kernel per pair of planes).
//
// Sites i = a + Na (b + Nb p) with plane p = c + Nc beta.  The pair vector
// r_j - r_i depends on (a_j - a_i, b_j - b_i) and on the plane pair, so
//   g_i = C_dd mu_i sum_{p'} sum_{a', b'} W_{p p'}(a - a', b - b') mu_{p'} n_{p'}(a', b')
// is, for every plane pair, a 2D linear convolution with the symmetric
// tensor W = (1 - 3 r^ r^) / r^3 (W = 0 for i = j).  Zero padding to
// La >= 2 Na - 1, Lb >= 2 Nb - 1 (powers of two) makes the circular
// convolution of the FFT equal to the linear one: only pairs inside the
// sample interact, exactly as in the direct sum.
//
// Per evaluation: the 3P real channels (component x plane) are packed two
// per complex array, transformed along a then b, unpacked into channel
// spectra, mixed per frequency by the P x P plane-pair kernel spectra,
// repacked two per complex array and transformed back.
//
// The 1D transforms are radix-2 Stockham passes in LDS (the self-sorting
// formulation of Govindaraju et al., SC'08): each workgroup transforms C
// lines of length L, twiddles exp(-2 pi i m / L) come from a table built in
// double precision on the host.
#pragma once

#include "device_common.hpp"

namespace sp {

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Lines of length L = 2^logL: line l of batch q starts at q * batch_stride +
// l * line_stride, element e sits e * elem_stride further.  A workgroup
// transforms C lines; its threads step through the C * L / 2 butterflies of
// a stage.  LINE_FAST (lines adjacent in memory, e.g. the columns of a
// row-major grid): the line index runs fastest over the threads, so a wave
// reads C adjacent elements of each of 64 / C rows, and the LDS copy is
// element-major (index e C + l), so the lanes of a wave touch consecutive
// LDS words in every stage.  Otherwise (contiguous lines) the element index
// runs fastest and the LDS copy is line-major.  inverse: conjugated
// twiddles, no scaling.
template <typename T, bool LINE_FAST>
__global__ void __launch_bounds__(1024) k_fft_lines(Cx<T>* __restrict__ data, const Cx<T>* __restrict__ tw, int logL,
                                                    int C, int n_lines, long long line_stride, long long elem_stride,
                                                    long long batch_stride, int inverse) {
    extern __shared__ unsigned char fft_smem[];
    const int L = 1 << logL, H = L >> 1;
    Cx<T>* x = reinterpret_cast<Cx<T>*>(fft_smem);
    Cx<T>* y = x + C * L;
    const int nthr = blockDim.x;
    auto at = [&](int lo, int e) { return LINE_FAST ? e * C + lo : lo * L + e; };
    Cx<T>* base = data + (long long)blockIdx.y * batch_stride;
    const int line0 = blockIdx.x * C;
    for (int u = threadIdx.x; u < C * L; u += nthr) {
        const int lo = LINE_FAST ? u % C : u / L;
        const int e = LINE_FAST ? u / C : u % L;
        if (line0 + lo < n_lines) x[at(lo, e)] = base[(long long)(line0 + lo) * line_stride + (long long)e * elem_stride];
    }
    __syncthreads();
    for (int s = 0; s < logL; ++s) {
        const int Ns = 1 << s;
        for (int u = threadIdx.x; u < C * H; u += nthr) {
            const int lo = LINE_FAST ? u % C : u / H;
            const int j = LINE_FAST ? u / C : u % H;
            const int k = j & (Ns - 1);
            Cx<T> w = tw[k << (logL - 1 - s)];
            if (inverse) w.im = -w.im;
            const Cx<T> a = x[at(lo, j)];
            const Cx<T> b = cmul(x[at(lo, j + H)], w);
            const int o = ((j - k) << 1) + k;
            y[at(lo, o)] = Cx<T>{a.re + b.re, a.im + b.im};
            y[at(lo, o + Ns)] = Cx<T>{a.re - b.re, a.im - b.im};
        }
        __syncthreads();
        Cx<T>* sw = x;
        x = y;
        y = sw;
    }
    for (int u = threadIdx.x; u < C * L; u += nthr) {
        const int lo = LINE_FAST ? u % C : u / L;
        const int e = LINE_FAST ? u / C : u % L;
        if (line0 + lo < n_lines) base[(long long)(line0 + lo) * line_stride + (long long)e * elem_stride] = x[at(lo, e)];
    }
}

struct FftDims {
    int Na, Nb, P;        // lattice extent along a, b; planes (Nc x basis)
    int La, Lb;           // padded transform lengths
    int Q;                // complex arrays holding the 3P real channels
    int Nc, Nbas;         // plane = c + Nc beta
};

// mu_p n -> complex arrays Z_q = X_{2q} + i X_{2q+1} on the padded grid,
// channel ch = 3 p + component; zero outside the sample.
template <typename T>
__global__ void k_dd_pack(FftDims d, const T* __restrict__ n, const T* __restrict__ mu_plane, Cx<T>* __restrict__ Z) {
    const long long F = (long long)d.La * d.Lb;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)d.Q * F) return;
    const int q = (int)(t / F);
    const long long f = t - (long long)q * F;
    const int b = (int)(f / d.La), a = (int)(f - (long long)b * d.La);
    Cx<T> z{T(0), T(0)};
    if (a < d.Na && b < d.Nb) {
        const long long N = (long long)d.Na * d.Nb * d.P;
        const int C3 = 3 * d.P;
        const int c0 = 2 * q, c1 = 2 * q + 1;
        {
            const int p = c0 / 3, comp = c0 - 3 * p;
            const long long i = a + (long long)d.Na * (b + (long long)d.Nb * p);
            z.re = mu_plane[p] * n[comp * N + i];
        }
        if (c1 < C3) {
            const int p = c1 / 3, comp = c1 - 3 * p;
            const long long i = a + (long long)d.Na * (b + (long long)d.Nb * p);
            z.im = mu_plane[p] * n[comp * N + i];
        }
    }
    Z[t] = z;
}

// Channel spectra from the packed spectra: with Z = X0 + i X1 (X0, X1 real),
// X0^(k) = (Z^(k) + conj Z^(-k)) / 2 and X1^(k) = (Z^(k) - conj Z^(-k)) / (2i).
template <typename T>
__global__ void k_dd_unpack_spec(FftDims d, const Cx<T>* __restrict__ Z, Cx<T>* __restrict__ X) {
    const long long F = (long long)d.La * d.Lb;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)d.Q * F) return;
    const int q = (int)(t / F);
    const long long f = t - (long long)q * F;
    const int kb = (int)(f / d.La), ka = (int)(f - (long long)kb * d.La);
    const int ma = ka == 0 ? 0 : d.La - ka, mb = kb == 0 ? 0 : d.Lb - kb;
    const Cx<T> zk = Z[t];
    const Cx<T> zm = Z[(long long)q * F + ma + (long long)d.La * mb];
    // conj(zm) = (zm.re, -zm.im)
    X[(long long)(2 * q) * F + f] = Cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
    if (2 * q + 1 < 3 * d.P) {
        // (zk - conj zm) / (2i) = ((zk.im + zm.im) - i (zk.re - zm.re)) / 2
        X[(long long)(2 * q + 1) * F + f] = Cx<T>{T(0.5) * (zk.im + zm.im), T(-0.5) * (zk.re - zm.re)};
    }
}

__device__ __forceinline__ int sym6(int a, int b) {
    // xx xy xz yy yz zz
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
}

// Output channel spectra G_{3p+alpha} = sum_{p', beta} W^_{p p'}^{alpha beta} X_{3p'+beta},
// repacked two per complex array (Y_q = G_{2q} + i G_{2q+1}).
// W^ layout: [offset][sym6][frequency], offset = (c' - c + Nc - 1) Nbas^2 + beta Nbas + beta'.
template <typename T>
__global__ void k_dd_mix(FftDims d, const Cx<T>* __restrict__ What, const Cx<T>* __restrict__ X,
                         Cx<T>* __restrict__ Y) {
    const long long F = (long long)d.La * d.Lb;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)d.Q * F) return;
    const int q = (int)(t / F);
    const long long f = t - (long long)q * F;
    Cx<T> g[2] = {{T(0), T(0)}, {T(0), T(0)}};
    for (int h = 0; h < 2; ++h) {
        const int ch = 2 * q + h;
        if (ch >= 3 * d.P) break;
        const int p = ch / 3, alpha = ch - 3 * p;
        const int c = p % d.Nc, beta = p / d.Nc;
        Cx<T> acc{T(0), T(0)};
        for (int p2 = 0; p2 < d.P; ++p2) {
            const int c2 = p2 % d.Nc, beta2 = p2 / d.Nc;
            const int off = (c2 - c + d.Nc - 1) * d.Nbas * d.Nbas + beta * d.Nbas + beta2;
            const Cx<T>* Wo = What + (long long)off * 6 * F + f;
#pragma unroll
            for (int bc = 0; bc < 3; ++bc) {
                const Cx<T> w = Wo[(long long)sym6(alpha, bc) * F];
                const Cx<T> x = X[(long long)(3 * p2 + bc) * F + f];
                acc.re += w.re * x.re - w.im * x.im;
                acc.im += w.re * x.im + w.im * x.re;
            }
        }
        g[h] = acc;
    }
    // Y = G0 + i G1
    Y[t] = Cx<T>{g[0].re - g[1].im, g[0].im + g[1].re};
}

// Real channels back from the inverse transform, scaled by C_dd mu_i / (La Lb).
template <typename T>
__global__ void k_dd_out(FftDims d, const Cx<T>* __restrict__ Y, const T* __restrict__ mu_plane, T scale,
                         T* __restrict__ gdd) {
    const long long N = (long long)d.Na * d.Nb * d.P;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * N) return;
    const int comp = (int)(t / N);
    const long long i = t - (long long)comp * N;
    const int a = (int)(i % d.Na);
    const long long r = i / d.Na;
    const int b = (int)(r % d.Nb);
    const int p = (int)(r / d.Nb);
    const int ch = 3 * p + comp;
    const Cx<T> y = Y[(long long)(ch >> 1) * d.La * d.Lb + a + (long long)d.La * b];
    gdd[t] = scale * mu_plane[p] * ((ch & 1) ? y.im : y.re);
}

// Kernel tensor W on the padded grid for every plane-pair offset (double on
// the device, converted to the engine precision): index (ia, ib) holds the
// translation (da, db) = (a_i - a_j, b_i - b_j) with da = ia or ia - La.
template <typename T>
__global__ void k_dd_kernel_grid(FftDims d, const double* __restrict__ geo, Cx<T>* __restrict__ W) {
    // geo: A1[3], A2[3], A3[3] (Angstrom), then basis[3 * Nbas] (Angstrom)
    const long long F = (long long)d.La * d.Lb;
    const int noff = (2 * d.Nc - 1) * d.Nbas * d.Nbas;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)noff * F) return;
    const int off = (int)(t / F);
    const long long f = t - (long long)off * F;
    const int ib = (int)(f / d.La), ia = (int)(f - (long long)ib * d.La);
    const int nb2 = d.Nbas * d.Nbas;
    const int dc = off / nb2 - (d.Nc - 1);      // c' - c
    const int beta = (off % nb2) / d.Nbas, beta2 = off % d.Nbas;
    int da = ia < d.Na ? ia : ia - d.La;
    int db = ib < d.Nb ? ib : ib - d.Lb;
    const bool inside = (ia < d.Na || ia > d.La - d.Na) && (ib < d.Nb || ib > d.Lb - d.Nb);
    double w[6] = {0, 0, 0, 0, 0, 0};
    if (inside) {
        // r = r_j - r_i = -da A1 - db A2 + dc A3 + basis_beta' - basis_beta
        double r[3];
        for (int k = 0; k < 3; ++k)
            r[k] = -da * geo[k] - db * geo[3 + k] + dc * geo[6 + k] + geo[9 + 3 * beta2 + k] - geo[9 + 3 * beta + k];
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (r2 > 0.0) {
            const double inv = 1.0 / sqrt(r2);
            const double inv3 = inv * inv * inv;
            const double e[3] = {r[0] * inv, r[1] * inv, r[2] * inv};
            w[0] = (1.0 - 3.0 * e[0] * e[0]) * inv3;
            w[1] = -3.0 * e[0] * e[1] * inv3;
            w[2] = -3.0 * e[0] * e[2] * inv3;
            w[3] = (1.0 - 3.0 * e[1] * e[1]) * inv3;
            w[4] = -3.0 * e[1] * e[2] * inv3;
            w[5] = (1.0 - 3.0 * e[2] * e[2]) * inv3;
        }
    }
    for (int s = 0; s < 6; ++s) W[((long long)off * 6 + s) * F + f] = Cx<T>{(T)w[s], T(0)};
}

}  // namespace sp
