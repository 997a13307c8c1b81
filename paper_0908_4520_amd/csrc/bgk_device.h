// bgk_device.h -- device building blocks of the BGK step: storage codec, moment
// projection, N-th order Hermite equilibrium and relaxation, fused per cell.
//
// Stored value v_a of population a ("v-space"):
//   full storages (FP64, FP32):  v_a = f_a
//   deviation storages (*_DEV):  v_a = f_a - w_a rho0,      rho0 = 1
//   scaled deviation (FP16_DEV): v_a = (f_a - w_a rho0) / w_a
// so f_a - a_a = m_a v_a with a_a = w_a rho0 [dev], m_a = w_a [scaled] or 1.
//
// Collision (paper, section 2.2, Eq. 2order, with the moments of Eq. an and the
// Hermite equilibrium of Eq. demoeq generalised to order N <= 4):
//   d = sum_a m_a v_a  (= rho, or rho - rho0 for deviations),  j = sum_a xi_a m_a v_a,
//   rho = rho0 [dev] + d,  u = j / rho,  q = u.u,  s_a = xi_a.u,
//   f^eq_a = w_a rho P_N(s_a, q),
//   P_N = 1 + s + (s^2 - q)/2 + (s^3 - 3 s q)/6 + (s^4 - 6 s^2 q + 3 q^2)/24 (truncated),
//   f*_a = f_a - omega (f_a - f^eq_a).
// In v-space, with e_a = w_a (or 1 when scaled):
//   v^eq_a = e_a (d + rho (P_N(s_a) - 1)),   v*_a = v_a + omega (v^eq_a - v_a),
// and P_N - 1 is the polynomial a0' + a1 s + a2 s^2 + a3 s^3 + a4 s^4 whose coefficients
// depend only on q, so each population costs one dot product and a Horner chain.
// The relaxation keeps v_a with coefficient exactly 1: written as (1 - omega) v + omega v^eq,
// the rounded 1 - omega and omega would not sum to 1 and every step would scale the state by
// 1 + O(2^-24), a bias that is large against the slow decay of a shear wave.  For the same
// reason the equilibrium's mass and linear (momentum) terms are corrected for the rounding of
// the weights and abscissae to the compute type: with the rounded constants sum_a w_a and
// sum_a w_a xi_ax^2 differ from 1 by ~1e-8, which the corrections delta0, delta1 (computed at
// compile time from the rounded values) remove, so the FP32 collision conserves mass and
// momentum up to rounding noise instead of drifting systematically.  The corrections are
// below half an ulp of v^eq itself, so they are added to the non-equilibrium difference
// v^eq - v (small, so finely resolved), not to v^eq or its coefficients.
// With omega = 0 every term added to v_a is an exact zero, so a collisionless step moves
// the stored values bit for bit.
//
// Body force (section 2.1, force expansion; Eq. 2order with its forcing term).  The stored
// populations are then the shifted variable f~ of Eq. 2order; with G = g dt (here along x)
//   rho u = j + rho G/2,
//   f*_a = f~_a - omega (f~_a - f^eq_a) + (1 - omega/2) F_a,
// (Kn dt/(Kn + dt/2) = (1 - omega/2) dt), and the force term of order N, with the expansion
// coefficients of the equilibrium a^(m) = rho u^{(x)m}, is the derivative of the equilibrium
// along G at fixed rho:
//   F_a = w_a rho [(xi_a.G) P_{N-1}(s_a) - (u.G) P_{N-2}(s_a)],   P_{-1} = 0,
// because d/du of u^{(x)n}:chi^(n)/n! is the n-1 term contracted with chi^(n), and in the
// (s, q) form dP_N/ds = P_{N-1}, dP_N/dq = -P_{N-2}/2.  The physical distribution behind f~
// is f = f^eq + (1 - omega/2)(f~ - f^eq + F/2) (inverting the definition of f~), whose
// xy (xz) moment is the shear stress the forced kernels can also sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "lattices.inc"

namespace lbm {

enum Storage : int { ST_FP64 = 0, ST_FP32 = 1, ST_FP32_DEV = 2, ST_FP16_DEV = 3, ST_BF16_DEV = 4 };

// ------------------------------------------------------------------ compile-time loop
template <int I>
using ic = std::integral_constant<int, I>;

template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(ic<Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------------ random bits
// 32-bit integer finaliser (xorshift-multiply, "lowbias32" constants by C. Wellons).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// ------------------------------------------------------------------ storage codec
template <int S>
struct Codec;

template <>
struct Codec<ST_FP64> {
    using raw = double;
    using T = double;
    static constexpr bool dev = false, scaled = false, lowp = false;
    __device__ static T dec(raw r) { return r; }
    __device__ static double dec64(raw r) { return r; }
    template <bool SR>
    __device__ static raw enc(T v, uint32_t) { return v; }
};

template <>
struct Codec<ST_FP32> {
    using raw = float;
    using T = float;
    static constexpr bool dev = false, scaled = false, lowp = false;
    __device__ static T dec(raw r) { return r; }
    __device__ static double dec64(raw r) { return (double)r; }
    template <bool SR>
    __device__ static raw enc(T v, uint32_t) { return v; }
};

template <>
struct Codec<ST_FP32_DEV> : Codec<ST_FP32> {
    static constexpr bool dev = true;
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <>
struct Codec<ST_BF16_DEV> {
    using raw = uint16_t;
    using T = float;
    static constexpr bool dev = true, scaled = false, lowp = true;
    __device__ static T dec(raw r) { return __builtin_bit_cast(float, (uint32_t)r << 16); }
    __device__ static double dec64(raw r) { return (double)dec(r); }
    template <bool SR>
    __device__ static raw enc(T v, uint32_t rnd) {
        if constexpr (SR) {
            // the conversion writes the low half and keeps the high half of its first operand:
            // start from v's own bits, so no register has to be cleared for it
            bf16x2 p = __builtin_bit_cast(bf16x2, v);
            p = __builtin_amdgcn_cvt_sr_bf16_f32(p, v, rnd, false);
            return __builtin_bit_cast(uint16_t, p[0]);
        } else {
            return __builtin_bit_cast(uint16_t, (__bf16)v);   // round to nearest even
        }
    }
};

template <>
struct Codec<ST_FP16_DEV> {
    using raw = uint16_t;
    using T = float;
    static constexpr bool dev = true, scaled = true, lowp = true;
    __device__ static T dec(raw r) { return (float)__builtin_bit_cast(_Float16, r); }
    __device__ static double dec64(raw r) { return (double)dec(r); }
    template <bool SR>
    __device__ static raw enc(T v, uint32_t rnd) {
        if constexpr (SR) {
            f16x2 p = __builtin_bit_cast(f16x2, v);   // as for BF16: no cleared register
            p = __builtin_amdgcn_cvt_sr_f16_f32(p, v, rnd, false);
            return __builtin_bit_cast(uint16_t, p[0]);
        } else {
            return __builtin_bit_cast(uint16_t, (_Float16)v);  // round to nearest even
        }
    }
};

// m_a: factor from stored value to f_a - a_a; e_a: factor from (f^eq_a - a_a)/w_a to v-space.
template <class L, int S, int A>
constexpr double moment_factor() {
    return Codec<S>::scaled ? L::w[A] : 1.0;
}
template <class L, int S, int A>
constexpr double eq_factor() {
    return Codec<S>::scaled ? 1.0 : L::w[A];
}

// ------------------------------------------------------------------ moments + collision
// Index of the population with velocity -xi_a (every set here is symmetric under inversion).
template <class L>
constexpr int opposite(int a) {
    for (int b = 0; b < L::Q; ++b)
        if (L::xi[b][0] == -L::xi[a][0] && L::xi[b][1] == -L::xi[a][1] && L::xi[b][2] == -L::xi[a][2]) return b;
    return -1;
}

template <class T>
struct Moments {
    T d, jx, jy, jz;
};

template <class L, int S, class T>
__device__ __forceinline__ Moments<T> project(const T (&v)[L::Q]) {
    // per velocity pair (xi, -xi): the sum feeds the density, the difference the momentum.
    Moments<T> m{T(0), T(0), T(0), T(0)};
    static_for<L::Q>([&](auto I) {
        constexpr int a = decltype(I)::value;
        constexpr int b = opposite<L>(a);
        static_assert(b >= 0, "velocity set without inversion symmetry");
        if constexpr (b >= a) {
            constexpr double mf = moment_factor<L, S, a>();
            static_assert(mf == moment_factor<L, S, b>(), "opposite velocities with different weights");
            if constexpr (b == a) {                 // xi = 0
                m.d += (mf == 1.0) ? v[a] : T(mf) * v[a];
            } else {
                const T sum = v[a] + v[b], dif = v[a] - v[b];
                const T gs = (mf == 1.0) ? sum : T(mf) * sum, gd = (mf == 1.0) ? dif : T(mf) * dif;
                m.d += gs;
                if constexpr (L::xi[a][0] != 0.0) m.jx += T(L::xi[a][0]) * gd;
                if constexpr (L::xi[a][1] != 0.0) m.jy += T(L::xi[a][1]) * gd;
                if constexpr (L::D == 3 && L::xi[a][2] != 0.0) m.jz += T(L::xi[a][2]) * gd;
            }
        }
    });
    return m;
}

// Sums of the velocity-set constants after rounding to the compute type T.
template <class L, class T>
constexpr double rounded_mass_sum() {
    double s = 0.0;
    for (int a = 0; a < L::Q; ++a) s += (double)(T)L::w[a];
    return s;
}
template <class L, class T>
constexpr double rounded_momentum_sum() {   // sum_a w_a xi_ax^2 (the same for every axis)
    double s = 0.0;
    for (int a = 0; a < L::Q; ++a) s += (double)(T)L::w[a] * (double)(T)L::xi[a][0] * (double)(T)L::xi[a][0];
    return s;
}

// Relax the Q values in place; omega = 1/tau (0 = collisionless).  With FORCED, Gx is the
// body force times dt at this cell and sigma receives the physical shear stresses
// sum_a xi_ax xi_ay (f_a - f^eq_a) and, in 3-D, sum_a xi_ax xi_az (f_a - f^eq_a).
template <class L, int N, int S, class T, bool FORCED>
__device__ __forceinline__ void collide_impl(T (&v)[L::Q], T omega, T Gx, T (&sigma)[2]) {
    static_assert(N >= 1 && N <= 4, "Hermite order 1..4");
    constexpr double delta0 = 1.0 / rounded_mass_sum<L, T>() - 1.0;
    constexpr double delta1 = 1.0 / rounded_momentum_sum<L, T>() - 1.0;
    const Moments<T> m = project<L, S>(v);
    const T rho = Codec<S>::dev ? T(1) + m.d : m.d;
    const T inv = T(1) / rho;
    T ux = m.jx * inv;
    if constexpr (FORCED) ux += T(0.5) * Gx;
    const T uy = m.jy * inv, uz = (L::D == 3) ? m.jz * inv : T(0);
    const T q = ux * ux + uy * uy + uz * uz;
    // P_N(s) - 1 = a0m + a1 s + a2 s^2 + a3 s^3 + a4 s^4
    T a0m = T(0), a1 = T(1), a2 = T(0);
    if constexpr (N >= 2) { a0m = T(-0.5) * q; a2 = T(0.5); }
    if constexpr (N >= 3) { a1 = T(1) - T(0.5) * q; }
    if constexpr (N >= 4) { a0m = q * (T(0.125) * q - T(0.5)); a2 = T(0.5) - T(0.25) * q; }
    const T C0 = m.d + rho * a0m;
    const T C1 = rho * a1;
    const T D0 = m.d * T(delta0), D1 = C1 * T(delta1);   // conservation corrections
    const T C2 = rho * a2;
    const T C3 = rho * T(1.0 / 6.0);
    const T C4 = rho * T(1.0 / 24.0);
    // force: F_a / e_a = rG xi_ax P_{N-1}(s) - rGu P_{N-2}(s), with
    // P_0 = 1, P_1 = 1 + s, P_2 = b0 + s + s^2/2, P_3 = b0 + b0 s + s^2/2 + s^3/6, b0 = 1 - q/2
    const T rG = rho * Gx, rGu = rho * Gx * ux, b0 = T(1) - T(0.5) * q;
    const T kf = T(1) - T(0.5) * omega;
    T sxy = T(0), sxz = T(0);
    if constexpr (Codec<S>::lowp && !FORCED) {
        // 16-bit storages: the polynomial per velocity pair (xi, -xi), P(+-s) = E(s^2) +- s O(s^2).
        // Its rounding differs from the per-population Horner form in the last bits of FP32, far
        // below the storage's 8 or 11 bits (where FP32 storage needs the per-population form:
        // the two roundings fl(E + sO), fl(E - sO) round E's low bits alike, so a pair's mass
        // errors no longer cancel).
        static_for<L::Q>([&](auto I) {
            constexpr int a = decltype(I)::value;
            constexpr int b = opposite<L>(a);
            constexpr double ef = eq_factor<L, S, a>();
            if constexpr (b == a) {
                const T neq = (ef == 1.0) ? (C0 - v[a]) + D0 : (T(ef) * C0 - v[a]) + T(ef) * D0;
                v[a] = v[a] + omega * neq;
            } else if constexpr (b > a) {
                T s = T(0);
                if constexpr (L::xi[a][0] != 0.0) s += T(L::xi[a][0]) * ux;
                if constexpr (L::xi[a][1] != 0.0) s += T(L::xi[a][1]) * uy;
                if constexpr (L::D == 3 && L::xi[a][2] != 0.0) s += T(L::xi[a][2]) * uz;
                const T s2 = s * s;
                T E = C0, O = C1;
                if constexpr (N == 2 || N == 3) E = C0 + s2 * C2;
                if constexpr (N == 4) E = C0 + s2 * (C2 + s2 * C4);
                if constexpr (N >= 3) O = C1 + s2 * C3;
                const T sO = s * O, sD = s * D1;
                const T pa = E + sO, pb = E - sO, ca = D0 + sD, cb = D0 - sD;
                T na, nb;
                if constexpr (ef == 1.0) {
                    na = (pa - v[a]) + ca;
                    nb = (pb - v[b]) + cb;
                } else {
                    na = (T(ef) * pa - v[a]) + T(ef) * ca;
                    nb = (T(ef) * pb - v[b]) + T(ef) * cb;
                }
                v[a] = v[a] + omega * na;
                v[b] = v[b] + omega * nb;
            }
        });
        return;
    }
    static_for<L::Q>([&](auto I) {
        constexpr int a = decltype(I)::value;
        T s = T(0);
        if constexpr (L::xi[a][0] != 0.0) s += T(L::xi[a][0]) * ux;
        if constexpr (L::xi[a][1] != 0.0) s += T(L::xi[a][1]) * uy;
        if constexpr (L::D == 3 && L::xi[a][2] != 0.0) s += T(L::xi[a][2]) * uz;
        T p;
        if constexpr (N == 1) p = C1;
        if constexpr (N == 2) p = C1 + s * C2;
        if constexpr (N == 3) p = C1 + s * (C2 + s * C3);
        if constexpr (N == 4) p = C1 + s * (C2 + s * (C3 + s * C4));
        p = C0 + s * p;
        const T corr = D0 + s * D1;
        constexpr double ef = eq_factor<L, S, a>();
        T neq;                                      // v^eq - v, corrected
        if constexpr (ef == 1.0)
            neq = (p - v[a]) + corr;
        else
            neq = (T(ef) * p - v[a]) + T(ef) * corr;
        if constexpr (FORCED) {
            T pm1, pm2;                             // P_{N-1}(s), P_{N-2}(s)
            if constexpr (N == 1) { pm1 = T(1); pm2 = T(0); }
            if constexpr (N == 2) { pm1 = T(1) + s; pm2 = T(1); }
            if constexpr (N == 3) { pm1 = b0 + s * (T(1) + s * T(0.5)); pm2 = T(1) + s; }
            if constexpr (N == 4) {
                pm1 = b0 + s * (b0 + s * (T(0.5) + s * T(1.0 / 6.0)));
                pm2 = b0 + s * (T(1) + s * T(0.5));
            }
            T fa = -(rGu * pm2);
            if constexpr (L::xi[a][0] != 0.0) fa += T(L::xi[a][0]) * rG * pm1;
            if constexpr (ef != 1.0) fa *= T(ef);
            // f_a - f^eq_a = m_a (v_a - v^eq_a) in v-space units
            constexpr double mxy = moment_factor<L, S, a>() * L::xi[a][0] * L::xi[a][1];
            constexpr double mxz = moment_factor<L, S, a>() * L::xi[a][0] * L::xi[a][2];
            if constexpr (mxy != 0.0) sxy += T(mxy) * (T(0.5) * fa - neq);
            if constexpr (L::D == 3 && mxz != 0.0) sxz += T(mxz) * (T(0.5) * fa - neq);
            v[a] = v[a] + omega * neq + kf * fa;
        } else {
            v[a] = v[a] + omega * neq;
        }
    });
    if constexpr (FORCED) {
        sigma[0] = kf * sxy;
        sigma[1] = kf * sxz;
    }
}

template <class L, int N, int S, class T>
__device__ __forceinline__ void collide(T (&v)[L::Q], T omega) {
    T unused[2];
    collide_impl<L, N, S, T, false>(v, omega, T(0), unused);
}

// ------------------------------------------------------------------ equilibrium (init)
// v-space equilibrium values for given rho, u (FP64), used to initialise and encode.
template <class L, int N, int S>
__device__ __forceinline__ void equilibrium_v(double rho, double ux, double uy, double uz,
                                              double (&out)[L::Q]) {
    const double q = ux * ux + uy * uy + uz * uz;
    const double d = Codec<S>::dev ? rho - 1.0 : rho;
    static_for<L::Q>([&](auto I) {
        constexpr int a = decltype(I)::value;
        const double s = L::xi[a][0] * ux + L::xi[a][1] * uy + L::xi[a][2] * uz;
        double pm1 = s;   // P_N - 1, term by term
        if constexpr (N >= 2) pm1 += 0.5 * (s * s - q);
        if constexpr (N >= 3) pm1 += (s * s * s - 3.0 * s * q) / 6.0;
        if constexpr (N >= 4) pm1 += (s * s * s * s - 6.0 * s * s * q + 3.0 * q * q) / 24.0;
        out[a] = eq_factor<L, S, a>() * (d + rho * pm1);
    });
}

}  // namespace lbm
