// device_common.hpp -- device helpers shared by the engine's kernels:
// Philox4x32-10 counter-based normals, the Rodrigues rotation used by
// Depondt's scheme, and the LLG map from effective field to rotation vector.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp {

constexpr int kMaxBasis = 8;
constexpr int kMaxStencil = 40;   // bonds per basis atom in the kernel-argument stencil

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
    return V3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return V3<T>{a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return V3<T>{a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return V3<T>{s * a.x, s * a.y, s * a.z}; }

// --------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products on counter words 0 and 2, a word permutation, and
// xors with the key, which advances by the Weyl increments after each round.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        U4 o;
        o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        o.y = (uint32_t)p1;
        o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        o.w = (uint32_t)p0;
        c = o;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

struct ThermalKey {
    uint32_t seed_lo, seed_hi, step_lo, step_hi, replica;
};

__device__ __forceinline__ U4 thermal_bits(const ThermalKey& k, uint32_t site) {
    return philox4x32_10(U4{site, k.step_lo, k.step_hi, k.replica}, k.seed_lo, k.seed_hi);
}

// Three standard normals from one Philox block: u = (x + 1/2) 2^-32, then
// Box-Muller on (u0, u1) and (u2, u3), keeping the first three.
__device__ __forceinline__ V3<float> normals3(U4 b, float) {
    const float s = 0x1p-32f, h = 0x1p-33f;
    const float u0 = fmaf((float)b.x, s, h), u1 = fmaf((float)b.y, s, h);
    const float u2 = fmaf((float)b.z, s, h), u3 = fmaf((float)b.w, s, h);
    // -2 ln u = -2 ln2 * log2(u); v_log_f32 is log2, v_sin/v_cos take revolutions.
    // Raw v_sqrt_f32: its argument is zero or a normal number (2^-33 <= u <= 1).
    const float r0 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u2));
    return V3<float>{r0 * __builtin_amdgcn_cosf(u1), r0 * __builtin_amdgcn_sinf(u1),
                     r1 * __builtin_amdgcn_cosf(u3)};
}

__device__ __forceinline__ V3<double> normals3(U4 b, double) {
    const double s = 0x1p-32, h = 0x1p-33;
    const double u0 = (double)b.x * s + h, u1 = (double)b.y * s + h;
    const double u2 = (double)b.z * s + h, u3 = (double)b.w * s + h;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    return V3<double>{r0 * c1, r0 * s1, r1 * c3};
}

// --------------------------------------------------------------- rotation
// n rotated about omega by the angle |omega| dt.  1 - cos(theta) is formed as
// 2 sin^2(theta/2) so that small angles keep full relative precision.
template <typename T>
__device__ __forceinline__ V3<T> rotate(V3<T> n, V3<T> w, T dt) {
    const T w2 = dot(w, w);
    if (!(w2 > T(0))) return n;
    const T wn = sqrt(w2);
    const T inv = T(1) / wn;
    const V3<T> e = inv * w;
    const T half = T(0.5) * wn * dt;
    T sh, ch;
    if constexpr (sizeof(T) == 4) {
        __sincosf(half, &sh, &ch);
        // __sincosf loses accuracy only for large arguments; rotation angles per
        // step are far below one radian, where the hardware result is fine.
    } else {
        sincos(half, &sh, &ch);
    }
    const T st = T(2) * sh * ch;
    const T omc = T(2) * sh * sh;
    const V3<T> exn = cross(e, n);
    const T en = dot(e, n);
    return V3<T>{n.x + st * exn.x + omc * (en * e.x - n.x),
                 n.y + st * exn.y + omc * (en * e.y - n.y),
                 n.z + st * exn.z + omc * (en * e.z - n.z)};
}

// LLG (terms i and ii) written as dn/dt = n x A:
//   A = -gamma/(1+alpha^2) (B + alpha n x B), B in Tesla.
template <typename T>
__device__ __forceinline__ V3<T> llg_A(V3<T> n, V3<T> B, T gp, T alpha) {
    const V3<T> nxB = cross(n, B);
    return V3<T>{-gp * (B.x + alpha * nxB.x), -gp * (B.y + alpha * nxB.y), -gp * (B.z + alpha * nxB.z)};
}

// Integrators of the LLG equation dn/dt = n x A (Sec. III.C; Appendices B, C).
enum Solver { SOLVER_DEPONDT = 0, SOLVER_HEUN = 1, SOLVER_SIB = 2 };

template <typename T>
__device__ __forceinline__ V3<T> normalize3(V3<T> v) {
    const T r2 = v.x * v.x + v.y * v.y + v.z * v.z;
    T r;
    if constexpr (sizeof(T) == 4) {
        r = __builtin_amdgcn_rsqf(r2);
    } else {
        r = T(1) / sqrt(r2);
    }
    return V3<T>{v.x * r, v.y * r, v.z * r};
}

// Implicit-midpoint stage with the rotation vector A frozen: the x solving
// x = n + dt (n + x)/2 x A, i.e. (I + [w]x) x = n + n x w with w = A dt/2
// (Appendix C).  The 3x3 system is the Cayley transform of w; its inverse is
// (I - [w]x + w w^T) / (1 + |w|^2).
template <typename T>
__device__ __forceinline__ V3<T> sib_stage(V3<T> n, V3<T> A, T dt) {
    const V3<T> w = (T(0.5) * dt) * A;
    const V3<T> a = n + cross(n, w);
    const V3<T> wxa = cross(w, a);
    const T wa = dot(w, a);
    const T inv = T(1) / (T(1) + dot(w, w));
    return V3<T>{(a.x - wxa.x + w.x * wa) * inv, (a.y - wxa.y + w.y * wa) * inv, (a.z - wxa.z + w.z * wa) * inv};
}

template <typename T>
__device__ __forceinline__ V3<T> renorm_if_float(V3<T> n) {
    if constexpr (sizeof(T) == 4) {
        const float r = __builtin_amdgcn_rsqf(n.x * n.x + n.y * n.y + n.z * n.z);
        return V3<T>{n.x * r, n.y * r, n.z * r};
    } else {
        return n;
    }
}

}  // namespace sp
