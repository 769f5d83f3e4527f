// step_kernels.hip -- the kernels of one FSLBM time step on gfx950.
//
// Per step (parity p = steps done mod 2; layout A before even steps, B before
// odd ones, see fslbm_device.hpp):
//   [sigma != 0]  k_band -> k_normals -> k_curvature    (Sec. 2.2, curvature)
//   k_mass_exchange     interface list: mass flux, m(t+1), interface velocity
//   k_stream_collide    every cell: in-place stream + bounce-back + anti-bounce-
//                       back + fill level + conversion marks + collision
//   k_resolve           interface list: conflict rules, new/from-liquid lists
//   k_refill<scheme>    new-interface list: one of the five schemes (Sec. 3.1)
//   k_apply             conversions, next interface list, excess mass
//   k_excess_gather     converted list: receiver counts (Sec. 2.2, excess mass)
//   k_excess_scatter    next interface list: gather shares, reservoir, phi,
//                       forced filling/emptying classes
// Only the bulk kernel touches every cell; the others walk compacted int32
// lists with grid-stride loops whose lengths live in device memory, so the
// whole sequence can be captured once and replayed as a HIP graph.
#include "fslbm_kernels.hpp"
#include "fslbm_math.hpp"

namespace fslbm {
namespace {   // every kernel has internal linkage; only the launchers are exported

// Grid-stride loop over a device-resident list length, clamped to the list
// capacity (appends beyond it are dropped and flagged, never read).
#define FOR_LIST(k, count)                                                             \
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x,               \
                   k##_end = (count) < a.cap ? (long long)(count) : a.cap;             \
         k < k##_end; k += (long long)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ helpers

// Shifted PDF at a slot, decoded to double.
template <int ST>
__device__ __forceinline__ double load_slot(const StepArgs &a, Slot s) {
    using C = Codec<ST>;
    const typename C::M *pdf = static_cast<const typename C::M *>(a.pdf);
    return double(C::load(pdf + slot_index(a.g, s)));
}
template <int ST>
__device__ __forceinline__ void store_slot(const StepArgs &a, Slot s, double v) {
    using C = Codec<ST>;
    typename C::M *pdf = static_cast<typename C::M *>(a.pdf);
    C::store(pdf + slot_index(a.g, s), typename C::T(v));
}

// Shifted post-collision populations of a cell in the given layout.
template <int ST>
__device__ __forceinline__ void load_cell(const StepArgs &a, int layoutB, long long gid,
                                          double (&d)[Q]) {
    Cell c = decode(a.g, gid);
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = load_slot<ST>(a, slot_of(a.g, layoutB, c, gid, i));
}

__device__ __forceinline__ int fclass(uint8_t fl) {
    return (fl & F_NOFLUID) ? 1 : ((fl & F_NOEMPTY) ? 2 : 0);
}

// Mass flux of an interface-interface link after the forced filling/emptying
// table (Thuerey): fin flows into the cell, fout out of it.
__device__ __forceinline__ double link_flux(int cc, int cn, double fin, double fout) {
    if (cc == cn) return fin - fout;
    if (cc == 0) return cn == 1 ? fin : -fout;
    if (cc == 1) return -fout;
    return fin;
}

// ------------------------------------------------------------------ surface

// Mark the band (interface cells and their 3x3x3 neighbours) once and list it.
__global__ void k_band(StepArgs a) {
    const int32_t nold = a.cnt[C_IF0 + a.parity];
    FOR_LIST(k, nold) {
        long long gid = a.list_old[k];
        Cell c = decode(a.g, gid);
        long long base = (long long)c.b * a.g.N;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    long long q = nb_local(a.g, c.x, c.y, c.z, dx, dy, dz);
                    if (q < 0) continue;
                    long long cell = base + q;
                    unsigned int bit = 1u << (cell & 31);
                    unsigned int old = atomicOr(a.band + (cell >> 5), bit);
                    if (!(old & bit)) {
                        int32_t pos = atomicAdd(a.cnt + C_BAND, 1);
                        if (pos < a.cap) a.list_band[pos] = int32_t(cell);
                        else atomicOr(a.cnt + C_ERR, E_LIST_OVERFLOW);
                    }
                }
    }
}

// Unit normal n^ = grad(phi)/|grad(phi)| on the band (Parker-Youngs).
__global__ void k_normals(StepArgs a) {
    const int32_t nb = a.cnt[C_BAND];
    const long long BN = a.g.BN;
    FOR_LIST(k, nb) {
        long long gid = a.list_band[k];
        Cell c = decode(a.g, gid);
        double gx, gy, gz;
        py_gradient(a.g, c, [&](long long q) { return a.phi[q]; }, gx, gy, gz);
        double len = sqrt(gx * gx + gy * gy + gz * gz);
        a.normal[gid] = len > 0.0 ? gx / len : 0.0;
        a.normal[BN + gid] = len > 0.0 ? gy / len : 0.0;
        a.normal[2 * BN + gid] = len > 0.0 ? gz / len : 0.0;
        atomicAnd(a.band + (gid >> 5), ~(1u << (gid & 31)));
    }
}

// Mean curvature kappa_m = -div(n^)/2 and gas density rho_G = 3 (p_V + 2 sigma kappa_m).
__global__ void k_curvature(StepArgs a) {
    const int32_t nold = a.cnt[C_IF0 + a.parity];
    const long long BN = a.g.BN;
    FOR_LIST(k, nold) {
        long long gid = a.list_old[k];
        Cell c = decode(a.g, gid);
        double d0, d1, d2, t;
        py_gradient(a.g, c, [&](long long q) { return a.normal[q]; }, d0, t, t);
        py_gradient(a.g, c, [&](long long q) { return a.normal[BN + q]; }, t, d1, t);
        py_gradient(a.g, c, [&](long long q) { return a.normal[2 * BN + q]; }, t, t, d2);
        double km = -0.5 * ((d0 + d1) + d2);
        a.rhoG[gid] = 3.0 * (a.p_volume + 2.0 * a.sigma * km);
    }
}

// ------------------------------------------------------------------ mass exchange

// Interface mass exchange over the current interface list (Sec. 2.2 mass flux
// with the forced filling/emptying table), plus the velocity of each interface
// cell from its stored post-collision populations for the anti-bounce-back
// condition.  Block 0 also resets this step's list counters and carries the
// reservoir over; a second loop clears the previous step's conversion marks.
template <int ST>
__global__ void k_mass_exchange(StepArgs a) {
    const int p = a.parity;
    if (blockIdx.x == 0) {
        for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
            // mass that found no receiver is kept while the domain has no interface
            double carry = a.nif_dom[(1 - p) * a.B + b] > 0 ? 0.0 : a.res[(1 - p) * a.B + b];
            a.res[p * a.B + b] = carry;
            a.nif_dom[p * a.B + b] = 0;
        }
        if (threadIdx.x == 0) {
            a.cnt[C_IF0 + (1 - p)] = 0;
            a.cnt[C_NEWG] = 0;
            a.cnt[C_FROML] = 0;
            a.cnt[C_CONV0 + p] = 0;
        }
    }
    const int layoutB = p;   // layout before this step
    const int32_t nold = a.cnt[C_IF0 + p];
    const long long BN = a.g.BN;
    FOR_LIST(k, nold) {
        long long gid = a.list_old[k];
        Cell c = decode(a.g, gid);
        uint8_t fl = a.flags[gid];
        int cc = fclass(fl);
        double phx = a.phi[gid];
        double dm = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long nbg = nb_dir(a.g, c, i);
            if (nbg < 0) continue;
            uint8_t fn = a.flags[nbg];
            if (fn & F_GAS) continue;
            // the two populations crossing the link x <-> x + c_i, unshifted: the
            // one-sided fluxes of the forced classes need absolute values
            Slot sin_ = layoutB ? Slot{opp(i), gid} : Slot{i, nbg};   // f*_opp(i)(x + c_i)
            Slot sout = layoutB ? Slot{i, nbg} : Slot{opp(i), gid};   // f*_i(x)
            const double w = wgt<double>(i);
            double fin = w + load_slot<ST>(a, sin_), fout = w + load_slot<ST>(a, sout);
            if (fn & F_LIQ) dm += fin - fout;
            else dm += 0.5 * (phx + a.phi[nbg]) * link_flux(cc, fclass(fn), fin, fout);
        }
        a.m[gid] = a.m[gid] + dm;
        double d[Q];
        load_cell<ST>(a, layoutB, gid, d);
        const double *gr = a.grav + 3 * c.b;
        double rho, ux, uy, uz;
        moments_post(d, gr[0], gr[1], gr[2], rho, ux, uy, uz);
        a.uif[gid] = ux;
        a.uif[BN + gid] = uy;
        a.uif[2 * BN + gid] = uz;
    }
    const int32_t nconv = a.cnt[C_CONV0 + (1 - p)];
    FOR_LIST(k, nconv) {
        long long gid = a.list_conv_prev[k];
        a.flags[gid] = uint8_t(a.flags[gid] & ~F_CONV);
    }
}

// ------------------------------------------------------------------ bulk

// Fused stream + boundary conditions + collision for every cell (Sec. 2.1,
// 2.2).  PAR = 0: layout A -> B (pull from neighbours' slots, push into
// neighbours' slots); PAR = 1: layout B -> A (local slots only).  Gas cells
// exit after the flag read.  Interface cells additionally rebuild PDFs
// arriving from gas with the anti-bounce-back condition, update their fill
// level phi = m/rho and mark fill levels beyond the conversion thresholds.
template <int ST, int COLL, int PAR>
__global__ __launch_bounds__(256) void k_stream_collide(StepArgs a) {
    using C = Codec<ST>;
    using T = typename C::T;
    using Mem = typename C::M;
    const Geom g = a.g;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= g.BN) return;
    const uint8_t fl = a.flags[gid];
    if (!(fl & (F_LIQ | F_IF))) return;
    const Cell c = decode(g, gid);
    Mem *base = static_cast<Mem *>(a.pdf) + (long long)c.b * Q * g.N;
    const long long n = c.n;
    const long long N = g.N;

    // neighbour coordinates per axis (-1 = wall)
    int xs[3], ys[3], zs[3];
    xs[1] = c.x; ys[1] = c.y; zs[1] = c.z;
    xs[0] = c.x > 0 ? c.x - 1 : (g.per[0] ? g.nx - 1 : -1);
    xs[2] = c.x < g.nx - 1 ? c.x + 1 : (g.per[0] ? 0 : -1);
    ys[0] = c.y > 0 ? c.y - 1 : (g.per[1] ? g.ny - 1 : -1);
    ys[2] = c.y < g.ny - 1 ? c.y + 1 : (g.per[1] ? 0 : -1);
    zs[0] = c.z > 0 ? c.z - 1 : (g.per[2] ? g.nz - 1 : -1);
    zs[2] = c.z < g.nz - 1 ? c.z + 1 : (g.per[2] ? 0 : -1);
    auto nbl = [&](int dx, int dy, int dz) -> long long {
        int X = xs[dx + 1], Y = ys[dy + 1], Z = zs[dz + 1];
        if (X < 0 || Y < 0 || Z < 0) return -1;
        return ((long long)Z * g.ny + Y) * g.nx + X;
    };

    T d[Q];
    d[0] = C::load(base + n);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (PAR == 0) {
            long long s = nbl(-cx(i), -cy(i), -cz(i));
            // wall: the redirected f*_opp(i)(x) sits in (i, x)
            d[i] = s < 0 ? C::load(base + i * N + n) : C::load(base + opp(i) * N + s);
        } else {
            d[i] = C::load(base + i * N + n);
        }
    }

    if (fl & F_IF) {
        const long long BN = g.BN;
        const double ux = a.uif[gid], uy = a.uif[BN + gid], uz = a.uif[2 * BN + gid];
        const double rg = a.rhoG ? a.rhoG[gid] : 3.0 * a.p_volume;
        const double uu = ux * ux + uy * uy + uz * uz;
        const uint8_t *fb = a.flags + (long long)c.b * N;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long s = nbl(-cx(i), -cy(i), -cz(i));
            if (s >= 0 && (fb[s] & F_GAS)) {
                // anti-bounce-back: f_i = f_eq_i + f_eq_opp(i) - f*_opp(i)(x)
                double fo = PAR == 0 ? double(C::load(base + i * N + n))
                                     : double(C::load(base + opp(i) * N + s));
                double uc = cx(i) * ux + cy(i) * uy + cz(i) * uz;
                double w = wgt<double>(i);
                double e2 = 2.0 * w * rg * (1.0 + 4.5 * uc * uc - 1.5 * uu);
                d[i] = T(e2 - 2.0 * w - fo);
            }
        }
        double drho = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) drho += double(d[i]);
        const double ph = a.m[gid] / (1.0 + drho);
        a.phi[gid] = ph;
        uint8_t mark = ph > 1.0 + a.eps_phi ? F_MARK_A : (ph < -a.eps_phi ? F_MARK_B : 0);
        if (mark) a.flags[gid] = uint8_t(fl | mark);
    }

    const double *gr = a.grav + 3 * c.b;
    const T om = T(a.omega[c.b]);
    T omm = om;
    if (COLL == 1) {
        double op = a.omega[c.b];
        omm = T(1.0 / (0.5 + a.trt_lambda / (1.0 / op - 0.5)));
    }
    collide<T, COLL>(d, om, omm, T(gr[0]), T(gr[1]), T(gr[2]));

    C::store(base + n, d[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (PAR == 0) {
            long long t = nbl(cx(i), cy(i), cz(i));
            if (t < 0) C::store(base + opp(i) * N + n, d[i]);   // bounce-back at write
            else C::store(base + i * N + t, d[i]);
        } else {
            C::store(base + opp(i) * N + n, d[i]);
        }
    }
}

// ------------------------------------------------------------------ conversion

// Conflict rules over the interface list: gas next to a cell filling over
// 1+eps becomes a new interface cell; a cell emptying under -eps next to a
// filling cell stays interface; liquid next to a remaining emptying cell
// becomes interface.  Each rule reads only the fill marks, so one pass does all.
__global__ void k_resolve(StepArgs a) {
    const int32_t nold = a.cnt[C_IF0 + a.parity];
    FOR_LIST(k, nold) {
        long long gid = a.list_old[k];
        Cell c = decode(a.g, gid);
        uint8_t fl = a.flags[gid];
        if (fl & F_MARK_A) {
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                long long q = nb_dir(a.g, c, i);
                bool add = false;
                if (q >= 0 && (a.flags[q] & F_GAS)) add = !(flag_or(a.flags, q, F_MARK_A) & F_MARK_A);
                wave_append(add, int32_t(q), a.list_newg, a.cnt + C_NEWG, a.cap, a.cnt + C_ERR);
            }
        } else if (fl & F_MARK_B) {
            bool near_fill = false;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                long long q = nb_dir(a.g, c, i);
                if (q >= 0) {
                    uint8_t fq = a.flags[q];
                    near_fill |= (fq & F_IF) && (fq & F_MARK_A);
                }
            }
            if (near_fill) {
                flag_clear(a.flags, gid, F_MARK_B);
            } else {
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    long long q = nb_dir(a.g, c, i);
                    bool add = false;
                    if (q >= 0 && (a.flags[q] & F_LIQ))
                        add = !(flag_or(a.flags, q, F_MARK_B) & F_MARK_B);
                    wave_append(add, int32_t(q), a.list_froml, a.cnt + C_FROML, a.cap,
                                a.cnt + C_ERR);
                }
            }
        }
    }
}

// Valid refill source: liquid, or interface that is not emptying (new
// interface cells are still gas-typed at this point).
__device__ __forceinline__ bool refill_source(uint8_t f) {
    return (f & F_LIQ) || ((f & F_IF) && !(f & F_MARK_B));
}

// Refill every new interface cell (Sec. 3.1) and write its populations into
// the slots of the layout after this step.
template <int ST, int SCHEME>
__global__ void k_refill(StepArgs a) {
    const int32_t nn = a.cnt[C_NEWG];
    const int layoutB = 1 - a.parity;   // layout after this step
    FOR_LIST(k, nn) {
        long long gid = a.list_newg[k];
        Cell c = decode(a.g, gid);
        const double *gr = a.grav + 3 * c.b;
        bool val[Q];
        int nv = 0;
        double rs = 0.0, usx = 0.0, usy = 0.0, usz = 0.0;
        // face neighbours' velocities for GEQ
        double fu[7][3];
        double avg[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) avg[i] = 0.0;
        val[0] = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long q = nb_dir(a.g, c, i);
            val[i] = q >= 0 && refill_source(a.flags[q]);
            if (val[i]) {
                ++nv;
                double d[Q];
                load_cell<ST>(a, layoutB, q, d);
                double r, ux, uy, uz;
                moments_post(d, gr[0], gr[1], gr[2], r, ux, uy, uz);
                rs += r; usx += ux; usy += uy; usz += uz;
                if (i <= 6) { fu[i][0] = ux; fu[i][1] = uy; fu[i][2] = uz; }
                if (SCHEME == 4) {
#pragma unroll
                    for (int j = 0; j < Q; ++j) avg[j] += d[j];
                }
            }
        }
        double out[Q];
        double rb = 1.0, ub[3] = {0.0, 0.0, 0.0};
        if (nv > 0) {
            rb = rs / nv;
            ub[0] = usx / nv; ub[1] = usy / nv; ub[2] = usz / nv;
        }
        {
            double uu = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
#pragma unroll
            for (int i = 0; i < Q; ++i)
                out[i] = feq_shift<double>(i, rb, rb - 1.0, ub[0], ub[1], ub[2], uu);
        }
        int cn = -1;
        if ((SCHEME == 1 || SCHEME == 3) && nv > 0) {
            double nx_, ny_, nz_;
            py_gradient(a.g, c, [&](long long q) { return a.phi[q]; }, nx_, ny_, nz_);
            double sc[Q], best = -1e300;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                sc[i] = val[i] ? __dadd_rn(__dadd_rn(__dmul_rn(double(cx(i)), nx_),
                                                     __dmul_rn(double(cy(i)), ny_)),
                                           __dmul_rn(double(cz(i)), nz_))
                               : -1e300;
                best = sc[i] > best ? sc[i] : best;
            }
            double tol = 1e-12 * (fabs(nx_) + fabs(ny_) + fabs(nz_));
#pragma unroll
            for (int i = Q - 1; i >= 1; --i)
                if (val[i] && sc[i] >= best - tol) cn = i;
        }
        // offsets of c^n and the first cell along it
        int ddx = 0, ddy = 0, ddz = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if (i == cn) { ddx = cx(i); ddy = cy(i); ddz = cz(i); }
        long long k1 = -1;
        if (cn > 0) k1 = (long long)c.b * a.g.N + nb_local(a.g, c.x, c.y, c.z, ddx, ddy, ddz);
        if (SCHEME == 1 && cn > 0) {
            // EQ+NEQ: add the non-equilibrium part of the neighbour along c^n
            double d[Q];
            load_cell<ST>(a, layoutB, k1, d);
            double r, ux, uy, uz;
            moments_post(d, gr[0], gr[1], gr[2], r, ux, uy, uz);
            double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
            for (int i = 0; i < Q; ++i) out[i] += d[i] - feq_shift<double>(i, r, r - 1.0, ux, uy, uz, uu);
        } else if (SCHEME == 2 && nv > 0) {
            // GEQ: Grad's approximation from finite-difference velocity gradients
            double du[3][3];   // du[al][be] = d u_al / d x_be
#pragma unroll
            for (int be = 0; be < 3; ++be) {
                const int ip = 1 + 2 * be, im = 2 + 2 * be;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    if (val[ip] && val[im]) du[al][be] = (fu[ip][al] - fu[im][al]) / 2.0;
                    else if (val[ip]) du[al][be] = fu[ip][al] - ub[al];
                    else if (val[im]) du[al][be] = ub[al] - fu[im][al];
                    else du[al][be] = 0.0;
                }
            }
            const double tau = 1.0 / a.omega[c.b];
            const double cs2 = 1.0 / 3.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int ci[3] = {cx(i), cy(i), cz(i)};
                double s = 0.0;
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = 0; be < 3; ++be)
                        s += (du[al][be] + du[be][al]) *
                             (cs2 * (al == be ? 1.0 : 0.0) - double(ci[al] * ci[be]));
                out[i] += wgt<double>(i) * rb * tau / (2.0 * cs2) * s;
            }
        } else if (SCHEME == 3 && cn > 0) {
            // EXT: extrapolation along c^n, order limited by the run of valid cells
            Cell c1 = decode(a.g, k1);
            long long k2 = -1, k3 = -1;
            long long q2 = nb_local(a.g, c1.x, c1.y, c1.z, ddx, ddy, ddz);
            if (q2 >= 0) q2 += (long long)c.b * a.g.N;
            if (q2 >= 0 && refill_source(a.flags[q2])) {
                k2 = q2;
                Cell c2 = decode(a.g, k2);
                long long q3 = nb_local(a.g, c2.x, c2.y, c2.z, ddx, ddy, ddz);
                if (q3 >= 0) q3 += (long long)c.b * a.g.N;
                if (q3 >= 0 && refill_source(a.flags[q3])) k3 = q3;
            }
            double d1[Q], d2[Q];
            load_cell<ST>(a, layoutB, k1, d1);
            if (k2 >= 0) load_cell<ST>(a, layoutB, k2, d2);
            if (k3 >= 0) {
                double d3[Q];
                load_cell<ST>(a, layoutB, k3, d3);
#pragma unroll
                for (int i = 0; i < Q; ++i) out[i] = 3.0 * d1[i] - 3.0 * d2[i] + d3[i];
            } else if (k2 >= 0) {
#pragma unroll
                for (int i = 0; i < Q; ++i) out[i] = 2.0 * d1[i] - d2[i];
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) out[i] = d1[i];
            }
        } else if (SCHEME == 4 && nv > 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) out[i] = avg[i] / nv;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) store_slot<ST>(a, slot_of(a.g, layoutB, c, gid, i), out[i]);
        a.m[gid] = 0.0;
        a.phi[gid] = 0.0;
    }
}

// Density sum_i f*_i of a cell in the layout after this step.
template <int ST>
__device__ __forceinline__ double rho_after(const StepArgs &a, long long gid) {
    double d[Q];
    load_cell<ST>(a, 1 - a.parity, gid, d);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += d[i];
    return 1.0 + s;
}

// Apply the conversions (Sec. 2.2): filled cells become liquid and emptied
// cells gas (their excess mass is kept in mex), new and from-liquid cells
// become interface; the next interface list is built on the way.
template <int ST>
__global__ void k_apply(StepArgs a) {
    const int p = a.parity;
    auto clamp = [&](int32_t v) { return v < a.cap ? v : int32_t(a.cap); };
    const int32_t nold = clamp(a.cnt[C_IF0 + p]), nng = clamp(a.cnt[C_NEWG]),
                  nfl = clamp(a.cnt[C_FROML]);
    const long long total = (long long)nold + nng + nfl;
    const long long stride = (long long)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations so the
    // wave-level appends stay convergent
    const long long first = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long iters = (total + stride - 1) / stride;
    for (long long it = 0; it < iters; ++it) {
        long long k = first + it * stride;
        bool in = k < total;
        bool is_if = false, conv = false;
        long long gid = 0;
        if (in) {
            if (k < nold) {
                gid = a.list_old[k];
                uint8_t fl = a.flags[gid];
                if (fl & F_MARK_A) {
                    a.mex[gid] = a.m[gid] - rho_after<ST>(a, gid);
                    a.flags[gid] = uint8_t(F_LIQ | F_CONV);
                    a.phi[gid] = 1.0;
                    a.m[gid] = 0.0;
                    conv = true;
                } else if (fl & F_MARK_B) {
                    a.mex[gid] = a.m[gid];
                    a.flags[gid] = uint8_t(F_GAS | F_CONV);
                    a.phi[gid] = 0.0;
                    a.m[gid] = 0.0;
                    conv = true;
                } else {
                    is_if = true;
                }
            } else if (k < (long long)nold + nng) {
                gid = a.list_newg[k - nold];
                a.flags[gid] = F_IF;
                is_if = true;
            } else {
                gid = a.list_froml[k - nold - nng];
                a.m[gid] = rho_after<ST>(a, gid);
                a.phi[gid] = 1.0;
                a.flags[gid] = F_IF;
                is_if = true;
            }
        }
        wave_append(conv, int32_t(gid), a.list_conv, a.cnt + C_CONV0 + p, a.cap, a.cnt + C_ERR);
        wave_append(is_if, int32_t(gid), a.list_new, a.cnt + C_IF0 + (1 - p), a.cap, a.cnt + C_ERR);
        // interface cells per domain (one atomic per wave when it is one domain)
        int b = is_if ? int(gid / a.g.N) : -1;
        unsigned long long mask = __ballot(is_if);
        if (mask) {
            int lead = __ffsll((long long)mask) - 1;
            int b0 = __shfl(b, lead);
            bool same = __ballot(is_if && b != b0) == 0;
            if (same) {
                if (__lane_id() == lead) atomicAdd(a.nif_dom + p * a.B + b0, __popcll(mask));
            } else if (is_if) {
                atomicAdd(a.nif_dom + p * a.B + b, 1);
            }
        }
    }
}

// Receivers of each converted cell's excess mass: its D3Q19 neighbours that are
// interface after the conversion.  No receiver: the mass goes to the reservoir.
__global__ void k_excess_gather(StepArgs a) {
    const int p = a.parity;
    const int32_t nc = a.cnt[C_CONV0 + p];
    FOR_LIST(k, nc) {
        long long gid = a.list_conv[k];
        Cell c = decode(a.g, gid);
        int nr = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long q = nb_dir(a.g, c, i);
            if (q >= 0 && (a.flags[q] & F_IF)) ++nr;
        }
        if (nr == 0) {
            atomicAdd(a.res + p * a.B + c.b, a.mex[gid]);
            a.mex[gid] = 0.0;
        } else {
            a.mex[gid] = a.mex[gid] / nr;
        }
    }
}

// Every interface cell gathers the shares of its converted neighbours and the
// reservoir share, refreshes phi = m/rho if its mass changed, and gets its
// forced filling/emptying class for the next step.
template <int ST>
__global__ void k_excess_scatter(StepArgs a) {
    const int p = a.parity;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt[C_BAND] = 0;
    const int32_t nn = a.cnt[C_IF0 + (1 - p)];
    FOR_LIST(k, nn) {
        long long gid = a.list_new[k];
        Cell c = decode(a.g, gid);
        double add = 0.0;
        bool touched = false, has_liq = false, has_gas = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long q = nb_dir(a.g, c, i);
            if (q < 0) continue;
            uint8_t fq = a.flags[q];
            if (fq & F_CONV) {
                // a converted neighbour that had receivers (it has at least this one)
                add += a.mex[q];
                touched = true;
            }
            has_liq |= (fq & F_LIQ) != 0;
            has_gas |= (fq & F_GAS) != 0;
        }
        double r = a.res[p * a.B + c.b];
        int nd = a.nif_dom[p * a.B + c.b];
        double m = a.m[gid];
        if (touched) m = m + add;
        if (r != 0.0 && nd > 0) {
            m = m + r / nd;
            touched = true;
        }
        if (touched) {
            a.m[gid] = m;
            a.phi[gid] = m / rho_after<ST>(a, gid);
        }
        a.flags[gid] = uint8_t(F_IF | (!has_liq ? F_NOFLUID : (!has_gas ? F_NOEMPTY : 0)));
    }
}

// ------------------------------------------------------------------ launchers

static int list_blocks(long long cap) {
    long long b = (cap + 255) / 256;
    return int(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

template <int ST>
static void launch_step_t(const StepArgs &a, int collision, int scheme, hipStream_t s,
                          const BulkEvents *ev) {
    const int lb = list_blocks(a.cap);
    if (a.rhoG) {
        hipLaunchKernelGGL(k_band, dim3(lb), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_normals, dim3(lb), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_curvature, dim3(lb), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_mass_exchange<ST>, dim3(lb), dim3(256), 0, s, a);
    const unsigned nblk = unsigned((a.g.BN + 255) / 256);
    if (ev) (void)hipEventRecord(ev->before, s);
    if (collision == 0) {
        if (a.parity == 0) hipLaunchKernelGGL((k_stream_collide<ST, 0, 0>), dim3(nblk), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_stream_collide<ST, 0, 1>), dim3(nblk), dim3(256), 0, s, a);
    } else {
        if (a.parity == 0) hipLaunchKernelGGL((k_stream_collide<ST, 1, 0>), dim3(nblk), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_stream_collide<ST, 1, 1>), dim3(nblk), dim3(256), 0, s, a);
    }
    if (ev) (void)hipEventRecord(ev->after, s);
    hipLaunchKernelGGL(k_resolve, dim3(lb), dim3(256), 0, s, a);
    switch (scheme) {
        case 0: hipLaunchKernelGGL((k_refill<ST, 0>), dim3(lb), dim3(256), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_refill<ST, 1>), dim3(lb), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_refill<ST, 2>), dim3(lb), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_refill<ST, 3>), dim3(lb), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((k_refill<ST, 4>), dim3(lb), dim3(256), 0, s, a); break;
    }
    hipLaunchKernelGGL(k_apply<ST>, dim3(lb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_excess_gather, dim3(lb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_excess_scatter<ST>, dim3(lb), dim3(256), 0, s, a);
}

}  // namespace

#if defined(FSLBM_UNIT_STORAGE)
template <>
void launch_step_storage<FSLBM_UNIT_STORAGE>(const StepArgs &a, int collision, int scheme,
                                             hipStream_t s, const BulkEvents *ev) {
    launch_step_t<FSLBM_UNIT_STORAGE>(a, collision, scheme, s, ev);
}
#endif

#if defined(FSLBM_UNIT_DISPATCH)
void launch_step(const StepArgs &a, int storage, int collision, int scheme, hipStream_t s,
                 const BulkEvents *ev) {
    switch (storage) {
        case ST_F64: launch_step_storage<ST_F64>(a, collision, scheme, s, ev); break;
        case ST_F32: launch_step_storage<ST_F32>(a, collision, scheme, s, ev); break;
        case ST_F16: launch_step_storage<ST_F16>(a, collision, scheme, s, ev); break;
        default: launch_step_storage<ST_BF16>(a, collision, scheme, s, ev); break;
    }
}
#endif

}  // namespace fslbm
