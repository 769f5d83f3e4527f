// fslbm_math.hpp -- per-cell arithmetic of the FSLBM step on shifted populations
// d_i = f_i - w_i: equilibrium, Guo forcing, SRT/TRT collision, moments, and
// the Parker-Youngs stencil.  Written for the device; T is double or float.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// c_i . v over the nonzero components of c_i (each +-1), so that a direction
// with zero components costs no multiplication: without fast-math a product
// 0 * v cannot be folded away (v may be NaN or -0).  The rest direction gives 0.
template <typename T>
__device__ __forceinline__ T cdot(int i, T vx, T vy, T vz) {
    T s = T(0);
    bool any = false;
    auto add = [&](int c, T v) {
        if (c == 0) return;
        const T t = c > 0 ? v : -v;
        s = any ? s + t : t;
        any = true;
    };
    add(cx(i), vx);
    add(cy(i), vy);
    add(cz(i), vz);
    return s;
}

// Equilibrium (Sec. 2.1) minus its weight: f_eq_i(rho,u) - w_i with c_s^2 = 1/3.
template <typename T>
__device__ __forceinline__ T feq_shift(int i, T rho, T drho, T ux, T uy, T uz, T uu) {
    T uc = cdot<T>(i, ux, uy, uz);
    return wgt<T>(i) * (drho + rho * (T(3) * uc + T(4.5) * uc * uc - T(1.5) * uu));
}

// Guo forcing term without its (1 - omega/2) prefactor (Sec. 2.1).
template <typename T>
__device__ __forceinline__ T guo_hat(int i, T ux, T uy, T uz, T Fx, T Fy, T Fz) {
    T uc = cdot<T>(i, ux, uy, uz);
    T cF = cdot<T>(i, Fx, Fy, Fz);
    T uF = ux * Fx + uy * Fy + uz * Fz;
    return wgt<T>(i) * (T(3) * (cF - uF) + T(9) * uc * cF);
}

// Collision of one cell in place on shifted populations (Sec. 2.1): rho and the
// half-force-shifted velocity, F = rho g, SRT (relaxation towards equilibrium)
// or TRT (symmetric/antisymmetric split with rates om and omm).
// COLL: bit 0 selects TRT (else SRT), bit 1 the Smagorinsky turbulence model
// (Sec. 2.1): the relaxation time tau0 = 1/om becomes
// tau = (tau0 + sqrt(tau0^2 + les_k Qbar / rho)) / 2, les_k = 2 C_S^2 / c_s^4,
// Qbar = sqrt(2 Q:Q) of the non-equilibrium momentum flux of the incoming
// populations; with TRT om- then follows from lambda.
template <typename T, int COLL>
__device__ __forceinline__ void collide(T (&d)[Q], T om, T omm, T gx, T gy, T gz, T les_k = T(0),
                                        T lambda = T(0)) {
    T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += d[i];
        if (cx(i)) jx += T(cx(i)) * d[i];
        if (cy(i)) jy += T(cy(i)) * d[i];
        if (cz(i)) jz += T(cz(i)) * d[i];
    }
    T rho = T(1) + drho;
    T Fx = rho * gx, Fy = rho * gy, Fz = rho * gz;
    T ir = T(1) / rho;
    T ux = (jx + T(0.5) * Fx) * ir, uy = (jy + T(0.5) * Fy) * ir, uz = (jz + T(0.5) * Fz) * ir;
    T uu = ux * ux + uy * uy + uz * uz;
    if (COLL & 2) {
        // momentum flux of the non-equilibrium part (the shift w_i cancels)
        T qxx = T(0), qyy = T(0), qzz = T(0), qxy = T(0), qxz = T(0), qyz = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T ne = d[i] - feq_shift<T>(i, rho, drho, ux, uy, uz, uu);
            if (cx(i)) qxx += ne;
            if (cy(i)) qyy += ne;
            if (cz(i)) qzz += ne;
            if (cx(i) * cy(i)) qxy += T(cx(i) * cy(i)) * ne;
            if (cx(i) * cz(i)) qxz += T(cx(i) * cz(i)) * ne;
            if (cy(i) * cz(i)) qyz += T(cy(i) * cz(i)) * ne;
        }
        const T qq = qxx * qxx + qyy * qyy + qzz * qzz + T(2) * (qxy * qxy + qxz * qxz + qyz * qyz);
        const T qbar = sqrt(T(2) * qq);
        const T tau0 = T(1) / om;
        const T tau = T(0.5) * (tau0 + sqrt(tau0 * tau0 + les_k * qbar * ir));
        om = T(1) / tau;
        if (COLL & 1) omm = T(1) / (T(0.5) + lambda / (tau - T(0.5)));
    }
    // Per pair (i, opp(i)) the equilibrium and the Guo term split into a part
    // even in c_i and one odd in c_i; with uc = c_i.u and cF = c_i.F:
    //   f_eq - w = w (A + 4.5 rho uc^2) +- 3 w rho uc,   A = (rho - 1) - 1.5 rho u.u
    //   F^      = w (9 uc cF - 3 u.F)   +- 3 w cF
    // The relaxation then needs, per weight class w (faces 1/18, edges 1/36),
    //   even:  om (f_eq - w)_even + pf+ F^_even = K0 + K1 uc^2 + K2 uc cF
    //   odd:   om' (f_eq - w)_odd + pf' F^_odd  = K3 uc + K4 cF
    // (om' = om, pf' = pf+ for SRT; omega-, pf- for TRT), so each pair costs
    // one uc, one cF and a handful of fused multiply-adds.
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    const T A = drho - T(1.5) * rho * uu;
    const T pfp = T(1) - T(0.5) * om;
    const T omo = (COLL & 1) ? omm : om;
    const T pfo = T(1) - T(0.5) * omo;
    {
        const T w0 = wgt<T>(0);
        d[0] = d[0] - om * (d[0] - w0 * A) - pfp * (w0 * (T(3) * uF));
    }
    T K0[2], K1[2], K2[2], K3[2], K4[2];
#pragma unroll
    for (int cl = 0; cl < 2; ++cl) {
        const T w = cl == 0 ? wgt<T>(1) : wgt<T>(7);
        K0[cl] = om * (w * A) - pfp * (w * (T(3) * uF));
        K1[cl] = om * (w * (T(4.5) * rho));
        K2[cl] = pfp * (T(9) * w);
        K3[cl] = omo * (w * (T(3) * rho));
        K4[cl] = pfo * (T(3) * w);
    }
    const T keep = T(1) - om;
    const T hp = T(0.5) * om, hm = T(0.5) * omm;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int k = i + 1, cl = i <= 6 ? 0 : 1;
        const T uc = cdot<T>(i, ux, uy, uz), cF = cdot<T>(i, Fx, Fy, Fz);
        const T P = K0[cl] + K1[cl] * (uc * uc) + K2[cl] * (uc * cF);   // even part
        const T M = K3[cl] * uc + K4[cl] * cF;                           // odd part
        if ((COLL & 1) == 0) {
            d[i] = keep * d[i] + (P + M);
            d[k] = keep * d[k] + (P - M);
        } else {
            // symmetric and antisymmetric relaxation of (d_i + d_k)/2, (d_i - d_k)/2
            const T rs = P - hp * (d[i] + d[k]);
            const T ra = M - hm * (d[i] - d[k]);
            d[i] = d[i] + rs + ra;
            d[k] = d[k] + rs - ra;
        }
    }
}

// rho and velocity of stored post-collision populations (u = j/rho - g/2).
template <typename T>
__device__ __forceinline__ void moments_post(const T (&d)[Q], double gx, double gy, double gz,
                                             double &rho, double &ux, double &uy, double &uz) {
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double v = double(d[i]);
        drho += v;
        if (cx(i)) jx += cx(i) * v;
        if (cy(i)) jy += cy(i) * v;
        if (cz(i)) jz += cz(i) * v;
    }
    rho = 1.0 + drho;
    ux = jx / rho - 0.5 * gx;
    uy = jy / rho - 0.5 * gy;
    uz = jz / rho - 0.5 * gz;
}

// The 13 pairs (c, -c) of the 3x3x3 Parker-Youngs stencil, weights 4/2/1.
__host__ __device__ constexpr int pyx(int k) {
    constexpr int t[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
    return t[k];
}
__host__ __device__ constexpr int pyy(int k) {
    constexpr int t[13] = {0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
    return t[k];
}
__host__ __device__ constexpr int pyz(int k) {
    constexpr int t[13] = {0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return t[k];
}
__host__ __device__ constexpr double pyw(int k) { return k < 3 ? 4.0 : (k < 9 ? 2.0 : 1.0); }

// Parker-Youngs gradient of a per-cell double field at cell c (global id gid):
// central differences of each stencil pair; a pair with a wall at either end
// is dropped and its weight removed from the axis normaliser (wall narrowing).
// `val(k)` returns the field at global cell k.
template <typename F>
__device__ __forceinline__ void py_gradient(const Geom &g, const Cell &c, F val, double &gx,
                                            double &gy, double &gz) {
#pragma clang fp contract(off)
    double ax = 0.0, ay = 0.0, az = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    const long long base = (long long)c.b * g.N;
    // all 26 loads first (walls read the cell itself and are masked below)
    double vp[13], vm[13];
    bool ok[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) {
        const int p = nb_local(g, c.x, c.y, c.z, pyx(k), pyy(k), pyz(k));
        const int m = nb_local(g, c.x, c.y, c.z, -pyx(k), -pyy(k), -pyz(k));
        ok[k] = p >= 0 && m >= 0;
        vp[k] = val(base + (p >= 0 ? p : c.n));
        vm[k] = val(base + (m >= 0 ? m : c.n));
    }
#pragma unroll
    for (int k = 0; k < 13; ++k) {
        if (ok[k]) {
            const double dv = vp[k] - vm[k];
            if (pyx(k)) { ax += pyw(k) * pyx(k) * dv; wx += 2.0 * pyw(k); }
            if (pyy(k)) { ay += pyw(k) * pyy(k) * dv; wy += 2.0 * pyw(k); }
            if (pyz(k)) { az += pyw(k) * pyz(k) * dv; wz += 2.0 * pyw(k); }
        }
    }
    gx = wx > 0.0 ? ax / wx : 0.0;
    gy = wy > 0.0 ? ay / wy : 0.0;
    gz = wz > 0.0 ? az / wz : 0.0;
}

}  // namespace fslbm
