// collide.hpp -- BGK / TRT collision with the Guo body force, in registers.
//
// The paper's solver uses a two-relaxation-time (TRT) collision (Sec. 10,
// ref. [15]) and does not print an operator.  With
//   rho = sum f_i,  j = sum c_i f_i,  u = (j + rho g / 2) / rho
//   f_i^eq = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)
//   S_i    = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . (rho g)              (Guo, Zheng & Shi 2002)
// and the even/odd parts of a pair of opposite directions i, i',
//   a^+ = (a_i + a_i')/2,  a^- = (a_i - a_i')/2,
// the update is
//   f_i* = f_i - w+ (f^+ - eq^+) - w- (f^- - eq^-) + (1 - w+/2) S^+ + (1 - w-/2) S^-
// with w+ = omega (viscosity nu = (1/omega - 1/2)/3) and w- set by the
// parameter Lambda = (1/w+ - 1/2)(1/w- - 1/2).  BGK is the case w- = w+,
// evaluated by the same code, so BGK and TRT with equal rates agree bit for
// bit.  The even and odd parts of the equilibrium and of the source are
// formed directly (they are the terms of even and odd degree in c_i).
//
// SHIFTED = true works on v_i = sigma (f_i - w_i) (the FP16 storage form):
//   rho = 1 + sum v / sigma, j = sum c v / sigma,
//   v_i^eq = sigma w_i (rho - 1 + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)),
//   v_i* = v_i - omega (v_i - v_i^eq) + sigma S_i,
// which equals sigma (f_i* - w_i) in exact arithmetic.
//
// Evaluation: the pair sums A = v_i + v_i' and differences B = v_i - v_i'
// give the moments and the even and odd parts at once; every factor that
// does not depend on the node is folded on the host (collide_params), so a
// pair costs about 15 FP operations.
#pragma once

#include "d3q19.hpp"

namespace lbm {

template <typename T>
struct CollideParams {
    T gx, gy, gz;        // body-force acceleration g
    T g9x, g9y, g9z;     // 9 g
    T hp, hm;            // w+/2, w-/2
    T a1[2], a2[2];      // w+ sc w_c and sc (1 - w+/2) w_c   (c = 0: |c_i| = 1, c = 1: |c_i|^2 = 2)
    T b1[2], b2[2];      // 3 w- sc w_c (times rho per node) and sc (1 - w-/2) w_c / 3
    T sc, inv_sc;        // sigma and 1/sigma for the shifted forms, else 1
};

// The node-independent factors, formed once in FP64 on the host and rounded
// to the compute type.
template <typename T>
__host__ __device__ inline CollideParams<T> collide_params(double wp, double wm, double gx, double gy, double gz,
                                                           double sc)
{
    CollideParams<T> p;
    p.gx = (T)gx;
    p.gy = (T)gy;
    p.gz = (T)gz;
    p.g9x = (T)(9.0 * gx);
    p.g9y = (T)(9.0 * gy);
    p.g9z = (T)(9.0 * gz);
    p.hp = (T)(0.5 * wp);
    p.hm = (T)(0.5 * wm);
    for (int c = 0; c < 2; ++c) {
        const double w = c == 0 ? 1.0 / 18.0 : 1.0 / 36.0;
        p.a1[c] = (T)(wp * sc * w);
        p.a2[c] = (T)(sc * (1.0 - 0.5 * wp) * w);
        p.b1[c] = (T)(3.0 * wm * sc * w);
        p.b2[c] = (T)(sc * (1.0 - 0.5 * wm) * w / 3.0);
    }
    p.sc = (T)sc;
    p.inv_sc = (T)(1.0 / sc);
    return p;
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float recip_(float x) { return __builtin_amdgcn_rcpf(x); } // within 1 ulp
__device__ __forceinline__ double recip_(double x) { return 1.0 / x; }

// Running signed sum over compile-time signs; the first term initialises it
// (no addition of a zero, which floating point cannot drop).
template <typename T>
struct SignedSum {
    T v;
    bool any = false;
    __device__ __forceinline__ void add(int sign, T x)
    {
        if (sign == 0) return;
        if (!any) {
            v = sign > 0 ? x : -x;
            any = true;
        } else {
            v = sign > 0 ? v + x : v - x;
        }
    }
    __device__ __forceinline__ T get() const { return any ? v : T(0); }
};

template <typename T, bool SHIFTED>
__device__ __forceinline__ void collide_node(T (&v)[Q], const CollideParams<T> &p)
{
    // No implicit contraction: every operation rounds as written (the fused
    // multiply-adds are explicit), so every kernel this is inlined into
    // computes identical bits and all schemes, layouts and addressings
    // produce bit-identical states.
#pragma clang fp contract(off)
    // sums and differences of the 9 pairs of opposite directions (i, i + 1)
    T A[9], B[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        A[q] = v[2 * q + 1] + v[2 * q + 2];
        B[q] = v[2 * q + 1] - v[2 * q + 2];
    }
    // moments, fixed summation order: mass from the pair sums, momentum from
    // the pair differences
    T s = v[0];
#pragma unroll
    for (int q = 0; q < 9; ++q) s += A[q];
    SignedSum<T> sx, sy, sz;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        sx.add(cx(2 * q + 1), B[q]);
        sy.add(cy(2 * q + 1), B[q]);
        sz.add(cz(2 * q + 1), B[q]);
    }
    T jx = sx.get(), jy = sy.get(), jz = sz.get();
    T rho, base; // base = rho (plain) or rho - 1 (shifted)
    if constexpr (SHIFTED) {
        base = s * p.inv_sc;
        rho = T(1) + base;
        jx *= p.inv_sc;
        jy *= p.inv_sc;
        jz *= p.inv_sc;
    } else {
        rho = s;
        base = s;
    }
    const T inv_rho = recip_(rho);
    const T hr = T(0.5) * rho;
    const T ux = fma_(hr, p.gx, jx) * inv_rho;
    const T uy = fma_(hr, p.gy, jy) * inv_rho;
    const T uz = fma_(hr, p.gz, jz) * inv_rho;
    const T F9x = rho * p.g9x, F9y = rho * p.g9y, F9z = rho * p.g9z; // 9 F, F = rho g
    const T uu = fma_(uz, uz, fma_(uy, uy, ux * ux));
    const T ug = fma_(uz, p.gz, fma_(uy, p.gy, ux * p.gx));
    const T U3 = (T(3) * rho) * ug;                        // 3 u.F
    const T T0 = fma_(-(T(1.5) * rho), uu, base);          // base - 3/2 rho u.u
    const T r45 = T(4.5) * rho;
    const T b1r[2] = {p.b1[0] * rho, p.b1[1] * rho};

    // Per pair (i, i'), with cu = c_i.u and cF9 = 9 c_i.F:
    //   X  = base + rho (9/2 cu^2 - 3/2 u.u)     even equilibrium / (sc w)
    //   Y  = 9 cu cF - 3 u.F                      even Guo term / (sc w)
    //   Ep = w+ eq^+ + (1 - w+/2) S^+ = a1 X + a2 Y
    //   Do = w- eq^- + (1 - w-/2) S^- = b1 rho cu + b2 cF9
    //   R  = w+ f^+ - Ep,  M = w- f^- - Do
    //   f_i* = f_i - R - M,  f_i'* = f_i' - R + M
    SignedSum<T> moving;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int i = 2 * q + 1;
        const int c = (i <= 6) ? 0 : 1;
        SignedSum<T> su, sf;
        su.add(cx(i), ux);
        su.add(cy(i), uy);
        su.add(cz(i), uz);
        sf.add(cx(i), F9x);
        sf.add(cy(i), F9y);
        sf.add(cz(i), F9z);
        const T cu = su.get(), cF9 = sf.get();
        const T X = fma_(r45 * cu, cu, T0);
        const T Y = fma_(cu, cF9, -U3);
        const T Ep = fma_(p.a1[c], X, p.a2[c] * Y);
        const T Do = fma_(b1r[c], cu, p.b2[c] * cF9);
        const T R = fma_(p.hp, A[q], -Ep);
        const T M = fma_(p.hm, B[q], -Do);
        const T vi = (v[i] - R) - M;
        const T vk = (v[i + 1] - R) + M;
        v[i] = vi;
        v[i + 1] = vk;
        moving.add(1, vi + vk);
    }
    // Rest direction by mass conservation: the collision with the Guo term
    // leaves sum_i f_i unchanged, so f_0* = rho - sum_{i>0} f_i* (shifted:
    // v_0* = sigma (rho - 1) - sum_{i>0} v_i*).  Equal to the direct formula
    // in exact arithmetic; in floating point it keeps the rounded weights
    // from creating mass every step.
    v[0] = (SHIFTED ? p.sc * base : base) - moving.get();
}

} // namespace lbm
