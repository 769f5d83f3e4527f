// adjoint_kernels.hip -- reverse mode of one FSLBM step (FP64, SRT collision,
// EQ refilling, no surface tension) with the cell-type sequence frozen from the
// forward run.
//
// The forward step t -> t+1 on the canonical state (post-collision PDFs f*,
// interface mass m, fill level phi, cell types, reservoir) is
//   S1  streaming with bounce-back at walls (Sec. 2.1) and anti-bounce-back
//       from gas cells (Sec. 2.2, with the cell's velocity from f*(t) and the
//       gas density rho_G = 3 p_V); interface mass exchange
//       m' = m + sum_i dm_i(f*(t), phi(t), forced classes) (Sec. 2.2, mass
//       flux equation); phi' = m' / rho with rho the streamed density
//   S2  SRT collision with Guo forcing, F = rho g (Sec. 2.1)
//   S5  EQ refilling of new interface cells from the mean density and velocity
//       of their valid neighbours (Sec. 3.1)
//   S6  conversions: a filled cell's excess is m' - rho*, an emptied cell's is
//       m'; a cell that leaves the liquid gets m = rho* (Sec. 2.2)
//   S7  excess shares to the interface neighbours after S6, or to the
//       domain's reservoir, which is spread over all interface cells;
//       phi = m / rho* on every cell whose mass changed (Sec. 2.2, excess-mass
//       equation).
// Its reverse runs S7/S6 (k_adj_receivers, k_adj_converted), S5
// (k_adj_refill), then S2 with phi' and S1 in one pass that pushes each
// streamed population's adjoint back to its origin (k_adj_collide_stream, with
// k_adj_abb_velocity for the anti-bounce-back's velocity term).  Which cells converted, and which interface cells
// received excess mass, is read off the two canonical type fields; the
// conversion decisions themselves are held fixed.
#include <algorithm>

#include "adjoint.hpp"

namespace fslbm {
namespace {

constexpr int BS = 256;

__device__ __forceinline__ Cell cell_of(const Geom &g, int b, int n) {
    Cell c;
    c.b = b;
    c.n = n;
    const uint32_t r = g.dx.div(uint32_t(n));
    const uint32_t z = g.dy.div(r);
    c.x = n - int(r) * g.nx;
    c.y = int(r) - int(z) * g.ny;
    c.z = int(z);
    return c;
}

// Flat index of PDF i of cell n in domain b ([B][19][N]).
__device__ __forceinline__ long long pidx(const Geom &g, int b, int i, int n) {
    return ((long long)b * Q + i) * g.N + n;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// dst[k] += sum over the workgroup of v[k] (fixed order; every thread calls).
__device__ __forceinline__ void block_add4(double (&v)[4], double *dst) {
    __shared__ double sh[BS / 64][4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) dst[k] += (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    }
}

enum { STD = 0, NOFLUID = 1, NOEMPTY = 2 };

// Forced filling/emptying class of an interface cell from the types around it.
__device__ __forceinline__ int type_class(const Geom &g, const uint8_t *fl, const Cell &c) {
    bool liq = false, gas = false;
    const long long cb = (long long)c.b * g.N;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int q = nb_local(g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        if (q < 0) continue;
        liq |= fl[cb + q] == F_LIQ;
        gas |= fl[cb + q] == F_GAS;
    }
    return !liq ? NOFLUID : (!gas ? NOEMPTY : STD);
}

// The interface-interface link flux under the forced classes is
// ca * fin + cb * fout (cc: the cell's class, cn: the neighbour's).
__device__ __forceinline__ void flux_coef(int cc, int cn, double &ca, double &cb) {
    if (cc == cn) { ca = 1.0; cb = -1.0; }
    else if (cc == STD) { if (cn == NOFLUID) { ca = 1.0; cb = 0.0; } else { ca = 0.0; cb = -1.0; } }
    else if (cc == NOFLUID) { ca = 0.0; cb = -1.0; }
    else { ca = 1.0; cb = 0.0; }
}

// Streamed (pre-collision) populations of fluid cell c at t+1 from f*(t).
__device__ __forceinline__ void stream_in(const AdjArgs &a, const Cell &c, double (&fin)[Q]) {
    const double *f0 = a.s0.f;
    const uint8_t *fl = a.s0.fl;
    const long long cb = (long long)c.b * a.g.N;
    // the cell's populations, and every source's flag and population, in one
    // round of loads (the cell itself stands in for a wall source; unused)
    double fs[Q], fp[Q];
    int src[Q];
    uint8_t fls[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fs[i] = f0[pidx(a.g, c.b, i, c.n)];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        src[i] = nb_local(a.g, c.x, c.y, c.z, -cx(i), -cy(i), -cz(i));
        const int sc = src[i] < 0 ? c.n : src[i];
        fls[i] = fl[cb + sc];
        fp[i] = f0[pidx(a.g, c.b, i, sc)];
    }
    issue_fence();
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r += fs[i];
        jx += cx(i) * fs[i]; jy += cy(i) * fs[i]; jz += cz(i) * fs[i];
    }
    const double *gr = a.grav + 3 * c.b;
    const double ux = jx / r - 0.5 * gr[0], uy = jy / r - 0.5 * gr[1], uz = jz / r - 0.5 * gr[2];
    const double uu = ux * ux + uy * uy + uz * uz;
    fin[0] = fs[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (src[i] < 0) {
            fin[i] = fs[opp(i)];
        } else if (fls[i] == F_GAS) {
            const double uc = cx(i) * ux + cy(i) * uy + cz(i) * uz;
            fin[i] = 2.0 * wgt<double>(i) * a.rhoG * (1.0 + 4.5 * uc * uc - 1.5 * uu) - fs[opp(i)];
        } else {
            fin[i] = fp[i];
        }
    }
}

// ------------------------------------------------------------------ kernels

// Forced classes of the interface cells at t.
// They are also listed (ifcnt by the parity of t + 1), for the kernels that
// only act on interface cells; the other parity's count is cleared for the
// next reverse step.
__global__ __launch_bounds__(BS) void k_adj_classes(AdjArgs a) {
    const int b = blockIdx.y, n = blockIdx.x * BS + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.sum_lm[b] = 0.0;
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) a.ifcnt[1 - (a.t1 & 1)] = 0;
    const long long gid = (long long)b * a.g.N + n;
    const bool itf = n < a.g.N && a.s0.fl[gid] == F_IF;
    if (n < a.g.N) a.cls[gid] = itf ? uint8_t(type_class(a.g, a.s0.fl, cell_of(a.g, b, n))) : 0;
    wave_append(itf, int32_t(gid), a.iflist, a.ifcnt + (a.t1 & 1), (long long)a.B * a.g.N, a.ifcnt + 2);
}

// Item k of the interface list as (domain, cell).
__device__ __forceinline__ void if_item(const AdjArgs &a, long long k, int &b, int &n) {
    const int32_t gid = a.iflist[k];
    b = int(a.g.dN.div(uint32_t(gid)));
    n = int(gid - (long long)b * a.g.N);
}

// S7 reverse on the cells that are interface at t+1.  The loss adds its
// fill-level adjoint on the probe plane.  A cell whose mass changed (a
// converted neighbour, or the domain's reservoir spread) had phi = m / rho*:
// that adjoint moves to m and f*.  An unchanged cell that was already
// interface keeps phi = phi'.
__global__ __launch_bounds__(BS) void k_adj_receivers(AdjArgs a) {
    const int b = blockIdx.y, n = blockIdx.x * BS + threadIdx.x;
    if (n >= a.g.N) return;
    const long long gid = (long long)b * a.g.N + n;
    const uint8_t ty0 = a.s0.fl[gid], ty1 = a.s1.fl[gid];
    double lphis = 0.0;
    if (ty1 == F_IF) {
        const Cell c = cell_of(a.g, b, n);
        const long long cb = (long long)b * a.g.N;
        const bool spread = a.s1.R[b] != 0.0 && a.s1.nif[b] > 0;
        double lp = a.lphi1[gid];
        if (c.x == a.x_probe)
            lp += 2.0 * (a.h[(long long)b * (a.T + 1) + a.t1] - a.target[(long long)b * a.T + (a.t1 - 1)]) /
                  a.T * a.dloss[b];
        bool touched = spread;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int q = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
            if (q < 0) continue;
            touched |= a.s0.fl[cb + q] == F_IF && a.s1.fl[cb + q] != F_IF;
        }
        if (touched) {
            double rs = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) rs += a.s1.f[pidx(a.g, b, i, n)];
            const double lm = a.lm1[gid] + lp / rs;
            a.lm1[gid] = lm;
            const double dr = -lp * a.s1.m[gid] / (rs * rs);
#pragma unroll
            for (int i = 0; i < Q; ++i) a.lf1[pidx(a.g, b, i, n)] += dr;
            if (spread) atomicAdd(a.sum_lm + b, lm);
        } else if (ty0 == F_IF) {
            lphis = lp;
        }
    }
    a.lphis[gid] = lphis;
}

// S6/S7 reverse on converted cells and on cells that left the liquid; sets the
// adjoint of m' of every cell that was interface at t, and of the reservoir.
__global__ __launch_bounds__(BS) void k_adj_converted(AdjArgs a) {
    const int b = blockIdx.y, n = blockIdx.x * BS + threadIdx.x;
    if (n >= a.g.N) return;
    const long long gid = (long long)b * a.g.N + n;
    const bool spread = a.s1.R[b] != 0.0 && a.s1.nif[b] > 0;
    // the reservoir after S7 is 0 when spread, else reservoir + unreceived excess
    const double lR = spread ? a.sum_lm[b] / a.s1.nif[b] : a.lres1[b];
    if (n == 0) a.lres0[b] = lR;
    const uint8_t ty0 = a.s0.fl[gid], ty1 = a.s1.fl[gid];
    double lmt = 0.0;
    if (ty0 == F_LIQ && ty1 == F_IF) {
        const double l = a.lm1[gid];   // m = rho* (+ shares)
#pragma unroll
        for (int i = 0; i < Q; ++i) a.lf1[pidx(a.g, b, i, n)] += l;
    } else if (ty0 == F_IF && ty1 != F_IF) {
        const Cell c = cell_of(a.g, b, n);
        const long long cb = (long long)b * a.g.N;
        int nr = 0;
        double s = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int q = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
            if (q < 0 || a.s1.fl[cb + q] != F_IF) continue;
            ++nr;
            s += a.lm1[cb + q];
        }
        const double lmex = nr > 0 ? s / nr : lR;
        lmt = lmex;   // the excess is m' - rho* (filled) or m' (emptied)
        if (ty1 == F_LIQ) {
#pragma unroll
            for (int i = 0; i < Q; ++i) a.lf1[pidx(a.g, b, i, n)] -= lmex;
        }
    } else if (ty0 == F_IF && ty1 == F_IF) {
        lmt = a.lm1[gid];
        // phi(t+1) = phi' = m' / rho on an interface cell whose mass no
        // excess touched (lphis, set by k_adj_receivers), with rho the
        // streamed density
        // (the collision keeps the density: rho = sum f*(t+1))
        const double lp = a.lphis[gid];
        if (lp != 0.0) {
            double rho = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) rho += a.s1.f[pidx(a.g, b, i, n)];
            lmt += lp / rho;
        }
    }
    a.lmt[gid] = lmt;
}

// S5 reverse (EQ refilling): the new cell's PDFs are f_eq(rho_bar, u_bar) over
// its valid neighbours v (liquid, or interface and not emptied, at t), with
// rho(v) = sum f*(v) and u(v) = sum c f*(v) / rho(v) - g/2 at t+1.  A source
// can feed several new cells, so its adjoint is accumulated atomically.
__device__ __forceinline__ bool refill_source(const AdjArgs &a, long long cb, int q) {
    if (q < 0) return false;
    const uint8_t t0 = a.s0.fl[cb + q], t1 = a.s1.fl[cb + q];
    return t0 == F_LIQ || (t0 == F_IF && t1 != F_GAS);
}

// Density and velocity sum c f* / rho - g/2 of cell q at t+1.
__device__ __forceinline__ void moments1(const AdjArgs &a, int b, int q, const double *gr, double &r,
                                         double (&u)[3]) {
    double j[3] = {0.0, 0.0, 0.0};
    r = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const double v = a.s1.f[pidx(a.g, b, k, q)];
        r += v;
        j[0] += cx(k) * v; j[1] += cy(k) * v; j[2] += cz(k) * v;
    }
    for (int d = 0; d < 3; ++d) u[d] = j[d] / r - 0.5 * gr[d];
}

__global__ __launch_bounds__(BS) void k_adj_refill(AdjArgs a) {
    const int b = blockIdx.y, n = blockIdx.x * BS + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long gid = (long long)b * a.g.N + n;
    const bool mine = n < a.g.N && a.s0.fl[gid] == F_GAS && a.s1.fl[gid] == F_IF;
    const long long cb = (long long)b * a.g.N;
    const double *gr = a.grav + 3 * b;
    const int lane = __lane_id();
    // The wavefront's new cells one after the other, each by the whole
    // wavefront: lane j in 1..18 takes the source x + c_j (its moments, and at
    // the end its 19 adjoint contributions), lane i in 0..18 the refilled
    // population i.  A cell's sources are then read in one round, not one
    // after the other.
    unsigned long long todo = __ballot(mine);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int cn = __shfl(n, leader);
        const Cell c = cell_of(a.g, b, cn);
        const bool has = lane >= 1 && lane < Q;
        const int q = has ? nb_local(a.g, c.x, c.y, c.z, k_cx[lane], k_cy[lane], k_cz[lane]) : -1;
        const bool valid = refill_source(a, cb, q);
        double r = 1.0, u[3] = {0.0, 0.0, 0.0};
        if (valid) moments1(a, b, q, gr, r, u);
        const double nv = wave_sum(valid ? 1.0 : 0.0);
        if (nv > 0.0) {
            const double rb = wave_sum(valid ? r : 0.0) / nv;
            const double ub[3] = {wave_sum(valid ? u[0] : 0.0) / nv, wave_sum(valid ? u[1] : 0.0) / nv,
                                  wave_sum(valid ? u[2] : 0.0) / nv};
            const double uu = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
            // adjoint of the equilibrium refill f_i = f_eq_i(rho_bar, u_bar)
            double pl = 0.0, pu[3] = {0.0, 0.0, 0.0};
            if (lane < Q) {
                const int ci[3] = {k_cx[lane], k_cy[lane], k_cz[lane]};
                const double l = a.lf1[pidx(a.g, b, lane, cn)];
                const double uc = ci[0] * ub[0] + ci[1] * ub[1] + ci[2] * ub[2];
                const double w = lane == 0 ? 1.0 / 3.0 : (lane <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
                pl = l * w * (1.0 + 3.0 * uc + 4.5 * uc * uc - 1.5 * uu);
                for (int d = 0; d < 3; ++d) pu[d] = l * w * rb * (3.0 * ci[d] + 9.0 * uc * ci[d] - 3.0 * ub[d]);
            }
            const double lrb = wave_sum(pl);
            const double lub[3] = {wave_sum(pu[0]), wave_sum(pu[1]), wave_sum(pu[2])};
            const double lr = lrb / nv;
            const double lu[3] = {lub[0] / nv, lub[1] / nv, lub[2] / nv};
            // rho(v) and u(v) = sum c f*(v) / rho(v) - g/2 of every source v
            if (valid) {
                const double ir = 1.0 / r;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    const int ck[3] = {cx(k), cy(k), cz(k)};
                    double v = lr;
                    for (int d = 0; d < 3; ++d) v += lu[d] * (ck[d] - (u[d] + 0.5 * gr[d])) * ir;
                    atomicAdd(a.lf1 + pidx(a.g, b, k, q), v);
                }
            }
            if (lane == 0)
                for (int d = 0; d < 3; ++d) acc[1 + d] += -0.5 * lub[d];
        }
    }
    block_add4(acc, a.gpart + ((long long)b * a.nblk + blockIdx.x) * 4);
}

// S2 reverse (SRT collision with Guo forcing, and phi' = m' / rho) and S1
// reverse in one pass over the cell x that the populations stream into.  The
// collision's adjoint at x gives the adjoint lfin_i of every streamed
// population f_i(x), which goes back to where that population came from: the
// source cell y = x - c_i's entry i (f*_i(y)), with the mass-exchange terms of
// the link between y and x, or x's own entry opp(i) at a wall (bounce-back) or
// under anti-bounce-back from gas.  So every entry of the adjoint at t has one
// writer: entry (j, y) is written by y + c_j when that cell is fluid, else by
// y.  A cell's own terms are formed by its thread: the adjoints of m and phi
// at t (gathered over its links) and the anti-bounce-back velocity term, which
// touches all 19 of its entries and so is added afterwards (k_adj_abb_velocity,
// from the sum this kernel leaves in lua).  The mass adjoints lmt read here
// are final (k_adj_converted).
__global__ __launch_bounds__(BS) void k_adj_collide_stream(AdjArgs a) {
    const int b = blockIdx.y, n = blockIdx.x * BS + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long gid = (long long)b * a.g.N + n;
    if (n < a.g.N) {
        const uint8_t ty0 = a.s0.fl[gid];
        if (ty0 == F_GAS) {
#pragma unroll
            for (int i = 0; i < Q; ++i) a.lf0[pidx(a.g, b, i, n)] = 0.0;
            a.lm0[gid] = 0.0;
            a.lphi0[gid] = 0.0;
        } else {
            const Cell c = cell_of(a.g, b, n);
            const long long cb = (long long)b * a.g.N;
            const double *gr = a.grav + 3 * b;
            const bool xif = ty0 == F_IF;
            // streamed populations (as stream_in): every source's flag and
            // population in one round of loads (the cell's own slot at a wall);
            // the cell's own f*(t) is only needed next to a wall or gas
            double fin[Q];
            uint8_t fls[Q];
            int src[Q];
            bool special = false;   // a wall or gas source
            fin[0] = a.s0.f[pidx(a.g, b, 0, n)];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                src[i] = nb_local(a.g, c.x, c.y, c.z, -cx(i), -cy(i), -cz(i));
                const int sc = src[i] < 0 ? n : src[i];
                fls[i] = src[i] < 0 ? uint8_t(0) : a.s0.fl[cb + sc];
                fin[i] = a.s0.f[pidx(a.g, b, i, sc)];
            }
            issue_fence();
#pragma unroll
            for (int i = 1; i < Q; ++i) special |= fls[i] == 0 || fls[i] == F_GAS;
            // u(x) from f*(t), the velocity of the anti-bounce-back
            double ua[3] = {0.0, 0.0, 0.0};
            if (special) {
                double fs[Q];
                double rs = 0.0, js[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    fs[i] = a.s0.f[pidx(a.g, b, i, n)];
                    rs += fs[i];
                    js[0] += cx(i) * fs[i]; js[1] += cy(i) * fs[i]; js[2] += cz(i) * fs[i];
                }
                for (int d = 0; d < 3; ++d) ua[d] = js[d] / rs - 0.5 * gr[d];
                const double uu = ua[0] * ua[0] + ua[1] * ua[1] + ua[2] * ua[2];
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (fls[i] == 0) {
                        fin[i] = fs[opp(i)];
                    } else if (fls[i] == F_GAS) {
                        const double uc = cx(i) * ua[0] + cy(i) * ua[1] + cz(i) * ua[2];
                        fin[i] = 2.0 * wgt<double>(i) * a.rhoG * (1.0 + 4.5 * uc * uc - 1.5 * uu) - fs[opp(i)];
                    }
                }
            }
            // S2 reverse: lfin = (d f*(t+1) / d fin)^T lf1(x)
            const double om = a.omega[b];
            double rho = 0.0, J[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                rho += fin[i];
                J[0] += cx(i) * fin[i]; J[1] += cy(i) * fin[i]; J[2] += cz(i) * fin[i];
            }
            const double F[3] = {rho * gr[0], rho * gr[1], rho * gr[2]};
            // one reciprocal for the many divisions by rho below (FP64
            // division is a long instruction sequence on this part)
            const double irho = 1.0 / rho;
            const double u[3] = {J[0] * irho + 0.5 * gr[0], J[1] * irho + 0.5 * gr[1], J[2] * irho + 0.5 * gr[2]};
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
            const double pf = 1.0 - 0.5 * om;
            double lrho = 0.0, lu[3] = {0.0, 0.0, 0.0}, lF[3] = {0.0, 0.0, 0.0}, lom = 0.0;
            double lam[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double l = a.lf1[pidx(a.g, b, i, n)];
                lam[i] = l;
                const int ci[3] = {cx(i), cy(i), cz(i)};
                const double w = wgt<double>(i);
                const double uc = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
                const double feq = w * rho * (1.0 + 3.0 * uc + 4.5 * uc * uc - 1.5 * uu);
                const double cF = ci[0] * F[0] + ci[1] * F[1] + ci[2] * F[2];
                const double Fh = w * (3.0 * (cF - uF) + 9.0 * uc * cF);
                lom += l * (-(fin[i] - feq) - 0.5 * Fh);
                lrho += l * om * feq * irho;
                for (int d = 0; d < 3; ++d) {
                    lu[d] += l * (om * w * rho * (3.0 * ci[d] + 9.0 * uc * ci[d] - 3.0 * u[d]) +
                                  pf * w * (-3.0 * F[d] + 9.0 * ci[d] * cF));
                    lF[d] += l * pf * w * (3.0 * (ci[d] - u[d]) + 9.0 * uc * ci[d]);
                }
            }
            for (int d = 0; d < 3; ++d) lrho += lF[d] * gr[d];   // F = rho g
            // phi(t+1) = phi' = m' / rho: its adjoint adds dr to every streamed
            // population's (its m' part is in lmt already)
            double dr = 0.0;
            if (xif) {
                const double lp = a.lphis[gid];
                if (lp != 0.0) dr = -lp * a.s1.phi[gid] * irho;
            }
            acc[0] = lom;
            for (int d = 0; d < 3; ++d) acc[1 + d] = lF[d] * rho + 0.5 * lu[d];
            // S1 reverse, pushed back to each population's origin (the
            // mass-exchange terms are added by k_adj_mass)
            double lua[3] = {0.0, 0.0, 0.0};
            // lam becomes the adjoint of the streamed populations, lfin
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int ci[3] = {cx(i), cy(i), cz(i)};
                double v = (1.0 - om) * lam[i] + lrho + dr;
                for (int d = 0; d < 3; ++d) v += lu[d] * (ci[d] - (u[d] - 0.5 * gr[d])) * irho;
                lam[i] = v;
            }
            // bounce-back (f_i(x) = f*_opp(i)(x)) and anti-bounce-back from gas
            // (f_i(x) = feq_i + feq_opp(i) at (rho_G, u(x)) - f*_opp(i)(x)) go to
            // the cell's own entry opp(i); a streamed f_i(x) = f*_i(y) to y's entry i
            a.lf0[pidx(a.g, b, 0, n)] = lam[0];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const double li = lam[i];
                const bool gas = src[i] >= 0 && fls[i] == F_GAS;
                const bool own = src[i] < 0 || gas;
                a.lf0[own ? pidx(a.g, b, opp(i), n) : pidx(a.g, b, i, src[i])] = gas ? -li : li;
                const double lg = gas ? li : 0.0;
                const double uc = cx(i) * ua[0] + cy(i) * ua[1] + cz(i) * ua[2];
                const double k2 = 2.0 * wgt<double>(i) * a.rhoG;
                lua[0] += lg * k2 * (9.0 * uc * cx(i) - 3.0 * ua[0]);
                lua[1] += lg * k2 * (9.0 * uc * cy(i) - 3.0 * ua[1]);
                lua[2] += lg * k2 * (9.0 * uc * cz(i) - 3.0 * ua[2]);
            }
            if (xif) {
                // (zero without a gas neighbour)
                for (int d = 0; d < 3; ++d) {
                    a.lua[3 * gid + d] = lua[d];
                    acc[1 + d] += -0.5 * lua[d];
                }
            } else {
                a.lm0[gid] = 0.0;
                a.lphi0[gid] = 0.0;
            }
        }
    }
    block_add4(acc, a.gpart + ((long long)b * a.nblk + blockIdx.x) * 4);
}

// The mass-exchange part of S1 reverse, run by the interface cells.  An entry
// (i, y) of the adjoint at t that k_adj_collide_stream wrote from x = y + c_i
// carries the link between y and x, whose terms depend on m' of whichever of
// the two is interface.  Interface cell x adds them to the entries it wrote
// (every fluid source y = x - c_i), and to its own entry (i, x) where x + c_i
// is liquid (that entry's writer has no terms to add).  So each entry is
// updated by one thread.  x also sets its own adjoints of m and phi at t.
__device__ __forceinline__ void adj_mass_cell(const AdjArgs &a, const int b, const int n) {
    const long long gid = (long long)b * a.g.N + n;
    const Cell c = cell_of(a.g, b, n);
    const long long cb = (long long)b * a.g.N;
    // the neighbours x + c_i (the source of direction opp(i) is x + c_i) and,
    // in rounds of loads issued together, their types, then their fill
    // levels, mass adjoints, classes and populations, then the entries to
    // update (the cell itself stands in for a wall; unused there)
    int qs[Q];
    uint8_t tq[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        qs[i] = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        tq[i] = qs[i] < 0 ? uint8_t(0) : a.s0.fl[cb + qs[i]];
    }
    const double phx = a.s0.phi[gid];
    const double lmtx = a.lmt[gid];
    const int clx = a.cls[gid];
    issue_fence();
    double lphi = 0.0;
    // two halves of nine directions, so that a half's loads fit the registers
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        constexpr int H = 9;
        double phq[H], lmq[H], fq[H], fx[H], e_src[H], e_own[H];
        int clq[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int i = 1 + h * H + k;
            const int q = qs[i] < 0 ? n : qs[i];
            const long long qg = cb + q;
            phq[k] = a.s0.phi[qg];
            lmq[k] = a.lmt[qg];
            clq[k] = a.cls[qg];
            fq[k] = a.s0.f[pidx(a.g, b, opp(i), q)];   // f*_opp(i)(x + c_i)
            fx[k] = a.s0.f[pidx(a.g, b, i, n)];        // f*_i(x)
            e_src[k] = a.lf0[pidx(a.g, b, opp(i), q)]; // entry (opp(i), x + c_i), streamed into x
            e_own[k] = a.lf0[pidx(a.g, b, i, n)];      // entry (i, x), streamed into x + c_i
        }
        issue_fence();
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int i = 1 + h * H + k;
            if (qs[i] < 0) continue;
            const int q = qs[i];
            if (tq[i] == F_LIQ) {
                // with a liquid neighbour q: f*_opp(i)(q) in, f*_i(x) out
                a.lf0[pidx(a.g, b, opp(i), q)] = e_src[k] + lmtx;
                a.lf0[pidx(a.g, b, i, n)] = e_own[k] - lmtx;
            } else if (tq[i] == F_IF) {
                // entry (opp(i), q): link opp(i) of q (out) and link i of x (in)
                double ca, cbf, v;
                flux_coef(clq[k], clx, ca, cbf);
                v = lmq[k] * 0.5 * (phq[k] + phx) * cbf;
                flux_coef(clx, clq[k], ca, cbf);
                v += lmtx * 0.5 * (phx + phq[k]) * ca;
                a.lf0[pidx(a.g, b, opp(i), q)] = e_src[k] + v;
                // the fill-level adjoint of the link: link i of x (fin =
                // f*_opp(i)(q), fout = f*_i(x)) and link opp(i) of q (fin =
                // f*_i(x), fout = f*_opp(i)(q))
                flux_coef(clx, clq[k], ca, cbf);
                lphi += lmtx * 0.5 * (ca * fq[k] + cbf * fx[k]);
                flux_coef(clq[k], clx, ca, cbf);
                lphi += lmq[k] * 0.5 * (ca * fx[k] + cbf * fq[k]);
            }
        }
    }
    a.lm0[gid] = lmtx;
    a.lphi0[gid] = lphi;
}

__global__ __launch_bounds__(BS) void k_adj_mass(AdjArgs a) {
    const long long cnt = a.ifcnt[a.t1 & 1];
    for (long long k = (long long)blockIdx.x * BS + threadIdx.x; k < cnt; k += (long long)gridDim.x * BS) {
        int b, n;
        if_item(a, k, b, n);
        adj_mass_cell(a, b, n);
    }
}

// The anti-bounce-back velocity term of the interface cells next to gas: u(x)
// = sum c f*(x) / rho*(x) - g/2 enters every one of x's 19 entries.  lua is
// zero on interface cells without a gas neighbour.
__device__ __forceinline__ void adj_abb_cell(const AdjArgs &a, const int b, const int n) {
    const long long gid = (long long)b * a.g.N + n;
    const double lua[3] = {a.lua[3 * gid], a.lua[3 * gid + 1], a.lua[3 * gid + 2]};
    if (lua[0] == 0.0 && lua[1] == 0.0 && lua[2] == 0.0) return;
    const double *gr = a.grav + 3 * b;
    double fs[Q];
    double rs = 0.0, js[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fs[i] = a.s0.f[pidx(a.g, b, i, n)];
        rs += fs[i];
        js[0] += cx(i) * fs[i]; js[1] += cy(i) * fs[i]; js[2] += cz(i) * fs[i];
    }
    const double ua[3] = {js[0] / rs - 0.5 * gr[0], js[1] / rs - 0.5 * gr[1], js[2] / rs - 0.5 * gr[2]};
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int cj[3] = {cx(j), cy(j), cz(j)};
        double v = 0.0;
        for (int d = 0; d < 3; ++d) v += lua[d] * (cj[d] - (ua[d] + 0.5 * gr[d])) / rs;
        a.lf0[pidx(a.g, b, j, n)] += v;
    }
}

__global__ __launch_bounds__(BS) void k_adj_abb_velocity(AdjArgs a) {
    const long long cnt = a.ifcnt[a.t1 & 1];
    for (long long k = (long long)blockIdx.x * BS + threadIdx.x; k < cnt; k += (long long)gridDim.x * BS) {
        int b, n;
        if_item(a, k, b, n);
        adj_abb_cell(a, b, n);
    }
}

// Interface height: h = sum of phi over the plane x = x_probe, one workgroup
// per domain, fixed summation order.
__global__ __launch_bounds__(BS) void k_height(Geom g, const double *phi, int x_probe, double *h,
                                               long long stride, int t) {
    const int b = blockIdx.x;
    const long long plane = (long long)g.ny * g.nz;
    double s = 0.0;
    for (long long k = threadIdx.x; k < plane; k += BS) s += phi[(long long)b * g.N + k * g.nx + x_probe];
    __shared__ double sh[BS];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[(long long)b * stride + t] = sh[0];
}

__global__ __launch_bounds__(BS) void k_reduce_params(const double *gpart, int nblk, double *out) {
    const int b = blockIdx.x;
    __shared__ double sh[BS];
    for (int k = 0; k < 4; ++k) {
        double s = 0.0;
        for (int j = threadIdx.x; j < nblk; j += BS) s += gpart[((long long)b * nblk + j) * 4 + k];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = BS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[4 * b + k] = sh[0];
        __syncthreads();
    }
}

__global__ void k_save_scalars(const double *res, const int32_t *nif_dom, int B, int p_last, int p_cur,
                               double *R, int32_t *nif, double *reservoir) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    R[b] = p_last >= 0 ? res[p_last * B + b] : 0.0;
    nif[b] = p_last >= 0 ? nif_sum(nif_dom, p_last, B, b) : 0;
    reservoir[b] = res[p_cur * B + b];
}

}  // namespace

void launch_save_scalars(const double *res, const int32_t *nif_dom, int B, int p_last, int p_cur,
                         double *R, int32_t *nif, double *reservoir, hipStream_t s) {
    hipLaunchKernelGGL(k_save_scalars, dim3(unsigned((B + 255) / 256)), dim3(256), 0, s, res, nif_dom, B,
                       p_last, p_cur, R, nif, reservoir);
}

void launch_adjoint_step(const AdjArgs &a, hipStream_t s) {
    const dim3 grid(unsigned(a.nblk), unsigned(a.B));
    hipLaunchKernelGGL(k_adj_classes, grid, dim3(BS), 0, s, a);
    hipLaunchKernelGGL(k_adj_receivers, grid, dim3(BS), 0, s, a);
    hipLaunchKernelGGL(k_adj_converted, grid, dim3(BS), 0, s, a);
    hipLaunchKernelGGL(k_adj_refill, grid, dim3(BS), 0, s, a);
    hipLaunchKernelGGL(k_adj_collide_stream, grid, dim3(BS), 0, s, a);
    // the interface-cell kernels stride over the list (a fixed grid: its
    // length is only known on the device)
    const long long cells = (long long)a.B * a.g.N;
    const unsigned nl = unsigned(std::min<long long>((cells + BS - 1) / BS, 1024));
    hipLaunchKernelGGL(k_adj_mass, dim3(nl), dim3(BS), 0, s, a);
    hipLaunchKernelGGL(k_adj_abb_velocity, dim3(nl), dim3(BS), 0, s, a);
}

void launch_height(const Geom &g, int B, const double *phi, int x_probe, double *h, long long stride,
                   int t, hipStream_t s) {
    hipLaunchKernelGGL(k_height, dim3(unsigned(B)), dim3(BS), 0, s, g, phi, x_probe, h, stride, t);
}

void launch_reduce_params(const double *gpart, int B, int nblk, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_params, dim3(unsigned(B)), dim3(BS), 0, s, gpart, nblk, out);
}

}  // namespace fslbm
