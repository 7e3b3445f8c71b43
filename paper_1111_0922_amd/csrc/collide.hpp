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
#pragma once

#include "d3q19.hpp"

namespace lbm {

template <typename T>
struct CollideParams {
    T omega, gx, gy, gz;   // omega = w+ (shear relaxation)
    T sigma, inv_sigma;
    T omega_minus;         // w- (odd moments); equal to omega for BGK
};

template <typename T, bool SHIFTED>
__device__ __forceinline__ void collide_bgk(T (&v)[Q], const CollideParams<T> &p)
{
    // No implicit contraction: every operation rounds as written, so every
    // kernel this is inlined into computes identical bits and all schemes,
    // layouts and addressings produce bit-identical states.
#pragma clang fp contract(off)
    // moments, fixed summation order
    T s = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        s += v[i];
        if (cx(i) > 0) jx += v[i];
        if (cx(i) < 0) jx -= v[i];
        if (cy(i) > 0) jy += v[i];
        if (cy(i) < 0) jy -= v[i];
        if (cz(i) > 0) jz += v[i];
        if (cz(i) < 0) jz -= v[i];
    }
    T rho, drho;
    if constexpr (SHIFTED) {
        drho = s * p.inv_sigma;
        rho = T(1) + drho;
        jx *= p.inv_sigma;
        jy *= p.inv_sigma;
        jz *= p.inv_sigma;
    } else {
        rho = s;
        drho = T(0);
    }
    const T inv_rho = T(1) / rho;
    const T ux = (jx + T(0.5) * rho * p.gx) * inv_rho;
    const T uy = (jy + T(0.5) * rho * p.gy) * inv_rho;
    const T uz = (jz + T(0.5) * rho * p.gz) * inv_rho;
    const T Fx = rho * p.gx, Fy = rho * p.gy, Fz = rho * p.gz;
    const T uu = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    const T om = p.omega;                        // w+
    const T omm = p.omega_minus;                 // w-
    const T kf = T(1) - T(0.5) * om;             // Guo prefactor of the even source part (1 - w+/2)
    const T kfm = T(1) - T(0.5) * omm;           // and of the odd part (1 - w-/2)
    const T sc = SHIFTED ? p.sigma : T(1);       // scale of the stored form
    const T base = SHIFTED ? drho : rho;         // rho (plain) or rho - 1 (shifted)

    // moving directions, in pairs of opposites; the sum of the new values is
    // kept to close the rest direction below
    T moving = T(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int k = i + 1; // opposite of i
        const T w = (i <= 6) ? T(1.0 / 18.0) : T(1.0 / 36.0);
        T cu = T(0), cF = T(0);
        if (cx(i) > 0) { cu += ux; cF += Fx; }
        if (cx(i) < 0) { cu -= ux; cF -= Fx; }
        if (cy(i) > 0) { cu += uy; cF += Fy; }
        if (cy(i) < 0) { cu -= uy; cF -= Fy; }
        if (cz(i) > 0) { cu += uz; cF += Fz; }
        if (cz(i) < 0) { cu -= uz; cF -= Fz; }
        const T eq_even = sc * w * (base + rho * (T(4.5) * cu * cu - T(1.5) * uu));
        const T eq_odd = sc * w * rho * T(3) * cu;
        const T src_even = sc * kf * w * (T(9) * cu * cF - T(3) * uF);
        const T src_odd = sc * kfm * w * T(3) * cF;
        const T vi = v[i], vk = v[k];
        const T ve = T(0.5) * (vi + vk), vo = T(0.5) * (vi - vk);
        // relaxation of the even and odd parts: r = w+ (f^+ - eq^+), s = w- (f^- - eq^-)
        const T r = om * (ve - eq_even);
        const T q = omm * (vo - eq_odd);
        v[i] = ((vi - r) - q) + (src_even + src_odd);
        v[k] = ((vk - r) + q) + (src_even - src_odd);
        moving += v[i] + v[k];
    }
    // Rest direction by mass conservation: the BGK update with the Guo term
    // leaves sum_i f_i unchanged, so f_0* = rho - sum_{i>0} f_i* (shifted:
    // v_0* = sigma (rho - 1) - sum_{i>0} v_i*).  Equal to the direct formula
    // in exact arithmetic; in floating point it keeps the rounded weights
    // (whose FP32 sum exceeds 1 by 1.5e-8) from creating mass every step.
    v[0] = sc * base - moving;
}

} // namespace lbm
