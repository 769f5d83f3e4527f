// fslbm_math.hpp -- per-cell arithmetic of the FSLBM step on shifted populations
// d_i = f_i - w_i: equilibrium, Guo forcing, SRT/TRT collision, moments, and
// the Parker-Youngs stencil.  Written for the device; T is double or float.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// Equilibrium (Sec. 2.1) minus its weight: f_eq_i(rho,u) - w_i with c_s^2 = 1/3.
template <typename T>
__device__ __forceinline__ T feq_shift(int i, T rho, T drho, T ux, T uy, T uz, T uu) {
    T uc = T(cx(i)) * ux + T(cy(i)) * uy + T(cz(i)) * uz;
    return wgt<T>(i) * (drho + rho * (T(3) * uc + T(4.5) * uc * uc - T(1.5) * uu));
}

// Guo forcing term without its (1 - omega/2) prefactor (Sec. 2.1).
template <typename T>
__device__ __forceinline__ T guo_hat(int i, T ux, T uy, T uz, T Fx, T Fy, T Fz) {
    T uc = T(cx(i)) * ux + T(cy(i)) * uy + T(cz(i)) * uz;
    T cF = T(cx(i)) * Fx + T(cy(i)) * Fy + T(cz(i)) * Fz;
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
    if ((COLL & 1) == 0) {
        T pf = T(1) - T(0.5) * om;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T e = feq_shift<T>(i, rho, drho, ux, uy, uz, uu);
            d[i] = d[i] - om * (d[i] - e) + pf * guo_hat<T>(i, ux, uy, uz, Fx, Fy, Fz);
        }
    } else {
        T pfp = T(1) - T(0.5) * om, pfm = T(1) - T(0.5) * omm;
        {
            T e = feq_shift<T>(0, rho, drho, ux, uy, uz, uu);
            d[0] = d[0] - om * (d[0] - e) + pfp * guo_hat<T>(0, ux, uy, uz, Fx, Fy, Fz);
        }
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const int k = i + 1;
            T ei = feq_shift<T>(i, rho, drho, ux, uy, uz, uu);
            T ek = feq_shift<T>(k, rho, drho, ux, uy, uz, uu);
            T Fi = guo_hat<T>(i, ux, uy, uz, Fx, Fy, Fz);
            T Fk = guo_hat<T>(k, ux, uy, uz, Fx, Fy, Fz);
            T fs = T(0.5) * (d[i] + d[k]), fa = T(0.5) * (d[i] - d[k]);
            T es = T(0.5) * (ei + ek), ea = T(0.5) * (ei - ek);
            T Fs = T(0.5) * (Fi + Fk), Fa = T(0.5) * (Fi - Fk);
            T rs = -om * (fs - es) + pfp * Fs;
            T ra = -omm * (fa - ea) + pfm * Fa;
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
