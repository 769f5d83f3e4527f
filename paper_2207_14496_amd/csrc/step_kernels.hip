// step_kernels.hip -- the kernels of one FSLBM time step on gfx950.
//
// Per step (parity p = steps done mod 2; layout A before even steps, B before
// odd ones, see fslbm_device.hpp), five kernels plus three for surface tension:
//   [sigma != 0]  k_band -> k_normals -> k_curvature    (Sec. 2.2, curvature)
//   k_stream_collide  fluid tiles: liquid cells get the in-place stream +
//                     bounce-back + collide; interface cells are listed by
//                     groups of neighbouring tiles
//   k_interface       interface list: the same update plus the mass exchange
//                     (Sec. 2.2 mass flux with the forced filling/emptying
//                     table), the anti-bounce-back condition, phi = m/rho and
//                     the conversion marks; marked cells are listed
//   k_resolve         marked cells: conflict rules -> new / from-liquid lists
//   k_convert         new cells: refilling (Sec. 3.1), 32 lanes per cell;
//                     marked cells: conversions, excess mass, receivers
//                     (Sec. 2.2); from-liquid cells
//   k_excess          receivers: gather excess shares (and the reservoir);
//                     phi; forced filling/emptying classes of every interface
//                     cell; bookkeeping for the next step
// Inside a multi-step call a step's k_excess work runs in extra workgroups of
// the next step's bulk kernel (k_excess_stream_collide); the call's last step
// runs k_excess on its own.  Only the bulk kernel walks the domain (the tiles
// that ever held fluid); the others walk compacted int32 lists whose lengths
// live in device memory, so the whole sequence can be captured once and
// replayed as a HIP graph.
//
// On MI355X a kernel boundary inside the graph leaves a gap of about a
// microsecond, and each kernel starts with cold per-XCD caches; the short list
// kernels are bound by their chains of dependent memory round trips, so work
// that can share a kernel does, and inside the list kernels every load that
// does not depend on another is issued first, with clamped in-bounds
// addresses for walls, and only then selected.
#include <hip/hip_ext.h>

#include <type_traits>

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

// The same over [0, count) without clamping, but every lane runs the same
// number of iterations (lanes past the end see in == false), so wavefront-wide
// ballots and shuffles inside stay convergent.
#define FOR_UNIFORM(k, in, count)                                                      \
    for (long long k##_end = (count), k##_str = (long long)gridDim.x * blockDim.x,     \
                   k##_it = 0, k##_n = (k##_end + k##_str - 1) / k##_str,              \
                   k = (long long)blockIdx.x * blockDim.x + threadIdx.x;               \
         k##_it < k##_n; ++k##_it, k += k##_str)                                       \
        if (const bool in = k < k##_end; true)

__device__ __forceinline__ long long clamp_cap(const StepArgs &a, int32_t v) {
    return v < a.cap ? (long long)v : a.cap;
}

// ------------------------------------------------------------------ helpers

// Shifted PDF at a flat slot index, decoded to double.
template <int ST>
__device__ __forceinline__ double load_slot(const StepArgs &a, long long off) {
    using C = Codec<ST>;
    return double(C::load(static_cast<const typename C::M *>(a.pdf) + off));
}
template <int ST>
__device__ __forceinline__ void store_slot(const StepArgs &a, long long off, double v) {
    using C = Codec<ST>;
    C::store(static_cast<typename C::M *>(a.pdf) + off, typename C::T(v));
}
// Outgoing-population copy of interface cell gid, direction i in 1..18.
template <int ST>
__device__ __forceinline__ void store_fo(const StepArgs &a, int i, long long gid, double v) {
    using C = Codec<ST>;
    C::store(static_cast<typename C::M *>(a.fo) + fo_index(gid, i), typename C::T(v));
}

// Shifted post-collision populations of a cell in the given layout (SLIP as
// for slot_flat).
template <int ST, int SLIP = -1>
__device__ __forceinline__ void load_cell(const StepArgs &a, int layoutB, const Cell &c,
                                          double (&d)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = load_slot<ST>(a, slot_flat<SLIP>(a.g, layoutB, c, i));
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

// Cell type after this step's conversions, read from a flag byte in either
// the encoding before k_convert rewrites it or the one after.
__device__ __forceinline__ uint8_t type_after(uint8_t f) {
    if (!(f & F_TYPE)) return 0;   // no cell (wall)
    if (f & F_IF) return (f & F_MARK_A) ? F_LIQ : ((f & F_MARK_B) ? F_GAS : F_IF);
    if (f & F_GAS) return (f & F_MARK_A) ? F_IF : F_GAS;
    return (f & F_MARK_B) ? F_IF : F_LIQ;   // liquid (possibly CONV-marked)
}

// Valid refill source: liquid, or interface that is not emptying (new
// interface cells are still gas-typed while k_convert runs).  Holds for the
// flag encodings both before and after k_convert's own rewrites.
__device__ __forceinline__ bool refill_source(uint8_t f) {
    return (f & F_LIQ) || ((f & F_IF) && !(f & F_MARK_B));
}

// Neighbour local indices of cell c along the 18 D3Q19 directions (-1 = wall).
__device__ __forceinline__ void neighbours(const Geom &g, const Cell &c, int (&nb)[Q]) {
    nb[0] = c.n;
#pragma unroll
    for (int i = 1; i < Q; ++i) nb[i] = nb_local(g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
}

// Append the entries val(i) of every lane whose bit i is set in sel (i < 32)
// to list[*count] with one atomic per wavefront.  Must be called by all lanes
// of the wavefront that are active in the enclosing loop.
template <int NI, typename V>
__device__ __forceinline__ void wave_append_sel(uint32_t sel, V val, int32_t *list, int32_t *count,
                                                long long cap, int32_t *err) {
    unsigned long long masks[NI];
    int pre[NI];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        masks[i] = __ballot((sel >> i) & 1u);
        pre[i] = tot;
        tot += __popcll(masks[i]);
    }
    if (tot == 0) return;
    const unsigned long long active = __ballot(1);
    const int lane = __lane_id();
    const int leader = __ffsll((long long)active) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, tot);
    base = __shfl(base, leader);
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        if ((sel >> i) & 1u) {
            long long pos = (long long)base + pre[i] + __popcll(masks[i] & below);
            if (pos < cap) list[pos] = val(i);
            else atomicOr(err, E_LIST_OVERFLOW);
        }
    }
}

// Sum of v over each aligned group of 32 lanes (every lane gets the sum).
__device__ __forceinline__ double group32_sum(double v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 32);
    return v;
}
__device__ __forceinline__ double group32_max(double v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off, 32);
        v = o > v ? o : v;
    }
    return v;
}

// f_eq_i(rho,u) - w_i for a runtime direction i (one lane per direction).
__device__ __forceinline__ double feq_shift_rt(int i, double rho, double ux, double uy, double uz) {
    const double uc = k_cx[i] * ux + k_cy[i] * uy + k_cz[i] * uz;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    return w * ((rho - 1.0) + rho * (3.0 * uc + 4.5 * uc * uc - 1.5 * uu));
}

// ------------------------------------------------------------------ surface

// The interface cells at the start of the step, before the bulk kernel lists
// them: the last step's list entries that are still interface, then the last
// step's new and from-liquid cells.  Item k of n0 + n1 + n2; false if the entry
// is no longer an interface cell.
__device__ __forceinline__ bool start_interface(const StepArgs &a, const SView &prev, long long k,
                                                long long n0, long long n1, long long &gid) {
    if (k < n0) {
        gid = sview_at(prev, k);
        return (a.flags[gid] & F_TYPE) == F_IF;
    }
    gid = k - n0 < n1 ? a.list_newg[k - n0] : a.list_froml[k - n0 - n1];
    return true;
}
#define START_COUNTS                                                                   \
    __shared__ int32_t pref_[257];                                                     \
    const SView prev = slist_view(a.list_if_prev, pref_);                              \
    const long long n0 = prev.total, n1 = clamp_cap(a, a.cnt[C_NEWG]),                 \
                    n2 = clamp_cap(a, a.cnt[C_FROML])

// Mark the band (interface cells and their 3x3x3 neighbours) once and list it.
__global__ __launch_bounds__(256) void k_band(StepArgs a) {
    START_COUNTS;
    FOR_UNIFORM(k, in, n0 + n1 + n2) {
        uint32_t sel = 0;
        long long cells[27];
        long long gid = 0;
        if (in && start_interface(a, prev, k, n0, n1, gid)) {
            const Cell c = decode(a.g, gid);
            const long long base = (long long)c.b * a.g.N;
            unsigned int olds[27], bits[27];
#pragma unroll
            for (int j = 0; j < 27; ++j) {
                const int q = nb_local(a.g, c.x, c.y, c.z, j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1);
                cells[j] = base + (q >= 0 ? q : c.n);
                bits[j] = 1u << (cells[j] & 31);
                olds[j] = q >= 0 ? atomicOr(a.band + (cells[j] >> 5), bits[j]) : bits[j];
            }
#pragma unroll
            for (int j = 0; j < 27; ++j) sel |= (olds[j] & bits[j]) ? 0u : (1u << j);
        }
        slist_append_sel<27>(a.list_band, sel, [&](int j) { return int32_t(cells[j]); }, a.cnt + C_ERR);
    }
}

// Unit normal n^ = grad(phi)/|grad(phi)| on the band (Parker-Youngs), phi(t).
__global__ __launch_bounds__(256) void k_normals(StepArgs a) {
    const long long BN = a.g.BN;
    __shared__ int32_t pref[257];
    const SView band = slist_view(a.list_band, pref);
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < band.total;
         k += (long long)gridDim.x * blockDim.x) {
        const long long gid = sview_at(band, k);
        const Cell c = decode(a.g, gid);
        double gx, gy, gz;
        py_gradient(a.g, c, [&](long long q) { return a.phi_cur[q]; }, gx, gy, gz);
        const double len = sqrt(gx * gx + gy * gy + gz * gz);
        a.normal[gid] = len > 0.0 ? gx / len : 0.0;
        a.normal[BN + gid] = len > 0.0 ? gy / len : 0.0;
        a.normal[2 * BN + gid] = len > 0.0 ? gz / len : 0.0;
        atomicAnd(a.band + (gid >> 5), ~(1u << (gid & 31)));
    }
}

// Mean curvature kappa_m = -div(n^)/2 and gas density rho_G = 3 (p_V + 2 sigma kappa_m).
__global__ __launch_bounds__(256) void k_curvature(StepArgs a) {
    const long long BN = a.g.BN;
    START_COUNTS;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n0 + n1 + n2;
         k += (long long)gridDim.x * blockDim.x) {
        long long gid;
        if (!start_interface(a, prev, k, n0, n1, gid)) continue;
        const Cell c = decode(a.g, gid);
        double d0, d1, d2, t;
        py_gradient(a.g, c, [&](long long q) { return a.normal[q]; }, d0, t, t);
        py_gradient(a.g, c, [&](long long q) { return a.normal[BN + q]; }, t, d1, t);
        py_gradient(a.g, c, [&](long long q) { return a.normal[2 * BN + q]; }, t, t, d2);
        const double km = -0.5 * ((d0 + d1) + d2);
        a.rhoG[gid] = 3.0 * ((a.pbub ? a.pbub[gid] : a.p_volume) + 2.0 * a.sigma * km);
    }
}

// ------------------------------------------------------------------ bulk

// Interface part of the update of cell gid (Sec. 2.2): mass exchange over the
// 18 links with the populations that just streamed in (d, before any
// reconstruction) and the cell's own outgoing populations of the last step
// (fo buffer); anti-bounce-back for populations arriving from gas, with the
// cell's velocity of the last step; phi = m/rho; conversion marks.
template <int ST, int PAR, bool SLIP>
__device__ __forceinline__ bool interface_part(const StepArgs &a, const long long gid, const uint8_t fl,
                                               const Cell &c, const int (&src)[Q],
                                               typename Codec<ST>::T (&d)[Q]) {
    using C = Codec<ST>;
    using T = typename C::T;
    const long long BN = a.g.BN, N = a.g.N;
    const long long cbase = (long long)c.b * N;
    const typename C::M *fob = static_cast<const typename C::M *>(a.fo);
    // own outgoing populations f*_i(x, t), i = 1..18, and neighbour flags
    // (every load of a round is issued before the first use; the fences keep
    // the compiler from sinking loads into the branches that use them, where
    // each would wait on its own)
    T fo[Q];
    uint8_t fn[Q];   // flag of the cell x - c_i (source of direction i)
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        fo[i] = C::load(fob + fo_index(gid, i));
        fn[i] = a.flags[cbase + (src[i] >= 0 ? src[i] : c.n)];   // own flag at walls: unused
    }
    const double m0 = a.m[gid];
    const double phx = a.phi_cur[gid];
    const double rg = a.rhoG ? a.rhoG[gid] : 3.0 * (a.pbub ? a.pbub[gid] : a.p_volume);
    issue_fence();
#pragma unroll
    for (int i = 1; i < Q; ++i) fn[i] = src[i] >= 0 ? fn[i] : uint8_t(0);
    // mass exchange: the neighbour x + c_i is the source of direction opp(i)
    const int cc = fclass(fl);
    // fill levels of the interface neighbours, loads in flight together (the
    // cell's own where the neighbour is not interface; unused there); with
    // FP64 populations in two batches of nine directions, which keeps the
    // free-slip interface update within 256 registers
    constexpr int NB = sizeof(T) == 8 ? 2 : 1;
    double dm = 0.0;
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const int i0 = 1 + h * (18 / NB), i1 = 1 + (h + 1) * (18 / NB);
        double phn[Q];
#pragma unroll
        for (int i = i0; i < i1; ++i) {
            const int o = opp(i);
            const bool itf = src[o] >= 0 && !(fn[o] & (F_GAS | F_LIQ));
            phn[i] = a.phi_cur[itf ? cbase + src[o] : gid];
        }
        issue_fence();
#pragma unroll
        for (int i = i0; i < i1; ++i) {
            const int o = opp(i);
            const uint8_t f = fn[o];
            // (no wall link; a free-slip path back into this cell exchanges nothing)
            if (src[o] < 0 || (SLIP && src[o] == c.n) || (f & F_GAS)) continue;
            const double w = wgt<double>(i);
            const double fin = w + double(d[o]);    // f*_opp(i)(x + c_i, t)
            const double fout = w + double(fo[i]);  // f*_i(x, t)
            if (f & F_LIQ) {
                dm += fin - fout;
            } else {
                dm += 0.5 * (phx + phn[i]) * link_flux(cc, fclass(f), fin, fout);
            }
        }
    }
    // velocity of the cell at the last step from its post-collision populations
    double r0 = 1.0 + double(d[0]), jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double v = double(fo[i]);
        r0 += v;
        if (cx(i)) jx += cx(i) * v;
        if (cy(i)) jy += cy(i) * v;
        if (cz(i)) jz += cz(i) * v;
    }
    const double *gr = a.grav + 3 * c.b;
    const double ux = jx / r0 - 0.5 * gr[0], uy = jy / r0 - 0.5 * gr[1], uz = jz / r0 - 0.5 * gr[2];
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (src[i] >= 0 && (fn[i] & F_GAS)) {
            // anti-bounce-back: f_i = f_eq_i + f_eq_opp(i) - f*_opp(i)(x)
            const double uc = cx(i) * ux + cy(i) * uy + cz(i) * uz;
            const double w = wgt<double>(i);
            const double e2 = 2.0 * w * rg * (1.0 + 4.5 * uc * uc - 1.5 * uu);
            d[i] = T(e2 - 2.0 * w - double(fo[opp(i)]));
        }
    }
    const double m1 = m0 + dm;
    double drho = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) drho += double(d[i]);
    const double ph = m1 / (1.0 + drho);
    a.m[gid] = m1;
    a.phi_next[gid] = ph;
    const uint8_t mark = ph > 1.0 + a.eps_phi ? F_MARK_A : (ph < -a.eps_phi ? F_MARK_B : 0);
    if (mark) a.flags[gid] = uint8_t(fl | mark);
    return mark != 0;
}

// Fused stream + boundary conditions + collision of one liquid (IF = false) or
// interface (IF = true) cell (Sec. 2.1, 2.2).  PAR = 0: layout A -> B (pull
// from neighbours' slots, push into neighbours' slots); PAR = 1: layout B -> A
// (local slots only).  Every cell reads and writes only its own slot set, so
// cells may be updated in any order and by different kernels.
template <int ST, int COLL, int PAR, bool IF>
__device__ __forceinline__ bool update_cell(const StepArgs &a, const long long gid, const uint8_t fl) {
    using C = Codec<ST>;
    using T = typename C::T;
    using Mem = typename C::M;
    const Geom &g = a.g;
    const Cell c = decode(g, gid);
    Mem *base = static_cast<Mem *>(a.pdf) + (long long)c.b * Q * g.N;
    const int n = c.n;
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
    auto nbl = [&](int dx, int dy, int dz) -> int {
        int X = xs[dx + 1], Y = ys[dy + 1], Z = zs[dz + 1];
        if (X < 0 || Y < 0 || Z < 0) return -1;
        return (Z * g.ny + Y) * g.nx + X;
    };
    constexpr bool SLIPC = (COLL & 4) != 0;   // free-slip walls
    const uint32_t N32 = uint32_t(N);      // slot offsets fit 32 bits (N * 19 < 2^32)
    // source cell x - c_i of each incoming population (-1 = no-slip wall) and
    // its population: the direction it was sent in is i, or at a free-slip
    // wall the reflected direction from the cell the specular path comes from
    // (used at once, so that no per-direction array of it stays live)
    int src[Q];
    T d[Q];
    src[0] = n;
    d[0] = C::load(base + n);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int sc = nbl(-cx(i), -cy(i), -cz(i));
        int sd = i;
        if (SLIPC && sc < 0) {
            int rx, ry, rz;
            sc = slip_target(g, c.x, c.y, c.z, -cx(i), -cy(i), -cz(i), rx, ry, rz);
            sd = dir_index(-rx, -ry, -rz);
        }
        src[i] = sc;
        if (PAR == 0) {
            // no-slip wall: the redirected f*_opp(i)(x) sits in (i, x); free-slip
            // wall: f*_sd(src) sits in (opp(sd), src) like any layout-A value
            const uint32_t off = sc < 0 ? uint32_t(i) * N32 + uint32_t(n) : uint32_t(opp(sd)) * N32 + uint32_t(sc);
            d[i] = C::load(base + off);
        } else {
            d[i] = C::load(base + uint32_t(i) * N32 + uint32_t(n));
        }
    }

    bool marked = false;
    if (IF) marked = interface_part<ST, PAR, SLIPC>(a, gid, fl, c, src, d);

    const double *gr = a.grav + 3 * c.b;
    const T om = T(a.omega[c.b]);
    const T omm = (COLL & 1) ? T(a.omega_m[c.b]) : om;
    collide<T, COLL>(d, om, omm, T(gr[0]), T(gr[1]), T(gr[2]), T(a.les_k), T(a.trt_lambda));

    C::store(base + n, d[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (PAR == 0) {
            int t = nbl(cx(i), cy(i), cz(i));
            // a no-slip wall neighbour gets the bounce-back slot (opp(i), x)
            // instead; a free-slip one the arrival slot of the reflection
            uint32_t off = t < 0 ? uint32_t(opp(i) * N + n) : uint32_t(i * N + t);
            if (SLIPC && t < 0) {
                int rx, ry, rz;
                const int m = slip_target(g, c.x, c.y, c.z, cx(i), cy(i), cz(i), rx, ry, rz);
                off = uint32_t(dir_index(rx, ry, rz) * N + m);
            }
            C::store(base + off, d[i]);
        } else {
            C::store(base + opp(i) * N + n, d[i]);
        }
    }
    if (IF) {
        typename C::M *fob = static_cast<typename C::M *>(a.fo);
#pragma unroll
        for (int i = 1; i < Q; ++i) C::store(fob + fo_index(gid, i), d[i]);
        // the density after this step as a read-back of the stored populations sums it
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += double(codec_round<ST>(d[i]));
        a.rho_if[gid] = 1.0 + s;
    }
    return marked;
}

// Global-memory pointer (address space 1), so that accesses through it are
// global, not flat, instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

// A global pointer that is the same on every lane of the wavefront, held in
// scalar registers and opaque to the compiler's address folding: an access at
// it plus a 32-bit lane byte offset is then one global instruction with a
// scalar base and a vector offset, with no per-lane 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ gptr<T> wave_ptr(T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (gptr<T>)((uint64_t(hi) << 32) | uint64_t(lo));
}
template <typename T>
__device__ __forceinline__ gptr<T> at_bytes(gptr<T> base, uint32_t off) {
    return (gptr<T>)((__attribute__((address_space(1))) char *)base + off);
}

// Update of the liquid cells of a plain tile (see tile_is_plain; lane l takes
// cell n0 + l of domain b): every lane reads and writes at fixed offsets from
// its own cell, so slot (d, n + delta) is base_d[n] with a per-direction base
// that is the same for the whole wavefront.  All accesses share one 32-bit
// lane byte offset (the domain's populations take less than 4 GiB: pdf_off32)
// and the domain's omega and g are scalar loads.  Only liquid lanes load and
// store.  (Issuing the population loads of all lanes together with the flag
// loads, so that no load waits for the cell types, was measured slower on
// partly liquid tiles and no faster on full ones.)  Returns the lane's cell
// type (as type_after reads it).  Arithmetic as update_cell.
template <int ST, int COLL, int PAR>
__device__ __forceinline__ uint8_t update_plain_tile(const StepArgs &a, const int b, const uint32_t n0) {
    using C = Codec<ST>;
    using T = typename C::T;
    using Mem = typename C::M;
    const Geom &g = a.g;
    const long long N = g.N;
    const uint32_t n = n0 + uint32_t(__lane_id());
    // cell offset of the neighbour x + c_i (no wall and no periodic wrap here)
    auto delta = [&](int i) -> long long {
        return (long long)cx(i) + (long long)cy(i) * g.nx + (long long)cz(i) * g.nx * g.ny;
    };
    Mem *pb = static_cast<Mem *>(a.pdf) + (long long)b * Q * N;
    const uint32_t off = n * uint32_t(sizeof(Mem));
    const uint8_t fl = *at_bytes(wave_ptr(a.flags + (long long)b * N), n);
    const uint8_t ty = type_after(fl);
    if (ty != F_LIQ) return ty;
    T d[Q];
    {
        d[0] = C::decode(*at_bytes(wave_ptr(pb), off));
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            // PAR 0 pulls f*_i(x - c_i) from slot (opp(i), x - c_i); PAR 1 reads (i, x)
            Mem *bi = PAR == 0 ? pb + (long long)opp(i) * N - delta(i) : pb + (long long)i * N;
            d[i] = C::decode(*at_bytes(wave_ptr(bi), off));
        }
    }
    const double *gr = a.grav + 3 * b;
    const T om = T(a.omega[b]);
    const T omm = (COLL & 1) ? T(a.omega_m[b]) : om;
    collide<T, COLL>(d, om, omm, T(gr[0]), T(gr[1]), T(gr[2]), T(a.les_k), T(a.trt_lambda));
    *at_bytes(wave_ptr(pb), off) = C::encode(d[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        // PAR 0 pushes into (i, x + c_i); PAR 1 writes (opp(i), x)
        Mem *bi = PAR == 0 ? pb + (long long)i * N + delta(i) : pb + (long long)opp(i) * N;
        *at_bytes(wave_ptr(bi), off) = C::encode(d[i]);
    }
    return ty;
}

// A tile (64 consecutive cells from gid0) is plain when every lane's update
// reads and writes only slots at fixed offsets from its own cell: for the
// layout A -> B step (PAR 0) the tile lies inside one row with no cell on a
// face of the box (so no wall and no periodic wrap among the neighbours); for
// the layout B -> A step (PAR 1, local slots only) it lies inside one domain.
template <int PAR>
__device__ __forceinline__ bool tile_is_plain(const StepArgs &a, uint32_t gid0, int &b, uint32_t &n0) {
    const Geom &g = a.g;
    if (!a.pdf_off32) return false;
    const uint32_t bb = g.dN.div(gid0);
    n0 = gid0 - bb * uint32_t(g.N);
    b = int(bb);
    if (PAR == 1) return (long long)n0 + TILE <= g.N;
    const uint32_t r = g.dx.div(n0);
    const uint32_t z = g.dy.div(r);
    const int x0 = int(n0 - r * uint32_t(g.nx)), y0 = int(r - z * uint32_t(g.ny));
    return x0 >= 1 && x0 + TILE <= g.nx - 1 && y0 >= 1 && y0 + 1 < g.ny && int(z) >= 1 && int(z) + 1 < g.nz;
}

// Bulk kernel: one thread per cell, one wavefront per tile of 64 consecutive
// cells (x fastest, so every PDF access of a wavefront is a contiguous row
// segment).  Only tiles that ever held fluid are listed; the wavefronts stride
// over that list, so a mostly empty domain does not pay for its gas, and a
// wavefront never loads a row segment without fluid.  Liquid cells get the full
// stream-collide update (plain tiles through update_liquid_plain).  Interface
// cells are listed for k_interface in groups from eight neighbouring tiles, so
// the list kernels of the step read neighbouring cells from neighbouring lanes.
// Cell types are read through type_after: with the last step's excess-mass
// work running in the same grid, a new interface cell may still carry its
// gas-typed flag while this kernel reads it.
template <int ST, int COLL, int PAR>
__device__ __forceinline__ void bulk_part(const StepArgs &a, const int wg, const int nwg) {
    const int p = a.parity;
    if (wg == 0) {
        // this step's conversion and mark lists start empty (the other lists
        // are cleared by k_interface, after the last step's excess work)
        if (threadIdx.x == 0) a.cnt[C_CONV0 + p] = 0;
        slist_reset(a.list_mark);
    }
    static_assert(TILE == 64, "one tile per wavefront");
    const int32_t ntiles = int32_t(tile_count(a.g.BN));
    const int32_t nt = min(a.cnt[C_TILES], ntiles);
    const int32_t nw = int32_t(blockDim.x >> 6);
    // the wavefront's index is the same on all its lanes; say so, so that the
    // tile index and everything derived from it live in scalar registers
    const int32_t wave = __builtin_amdgcn_readfirstlane(int32_t(threadIdx.x >> 6));
    for (int32_t k = wg * nw + wave; k < nt; k += nwg * nw) {
        const int32_t tile = __builtin_amdgcn_readfirstlane(a.tiles[k]);
        const long long gid = ((long long)tile << TILE_SHIFT) + __lane_id();
        int b;
        uint32_t n0;
        uint8_t ty;
        if (tile_is_plain<PAR>(a, uint32_t(tile) << TILE_SHIFT, b, n0)) {
            ty = update_plain_tile<ST, COLL, PAR>(a, b, n0);
        } else {
            const bool valid = gid < a.g.BN;
            const uint8_t fl = valid ? a.flags[gid] : uint8_t(0);
            ty = type_after(fl);
            if (ty == F_LIQ) update_cell<ST, COLL, PAR, false>(a, gid, fl);
        }
        // the interface cells of eight consecutive list tiles share a slot, and
        // the slots of such groups are scattered by a multiplicative hash:
        // k_interface's wavefronts then take cells of a few neighbouring rows,
        // while the wavefronts that run at the same time work far apart (with
        // the list in tile order and the wavefront's slot, k_interface on the
        // 512x512x96 cylinder in FP64 took 60 us instead of 45)
        slist_append(a.list_if, ty == F_IF, int32_t(gid), a.cnt + C_ERR,
                     int((uint32_t(k >> 3) * 2654435761u) >> 8));
    }
}

// Two-byte storage moves half the bytes per wavefront of FP32, so it needs
// more wavefronts in flight to keep HBM busy: at least five per SIMD (measured
// on the dense pool: 511 -> 444 us per FP16 bulk launch; the same bound makes
// FP32 slower, 710 -> 724 us, as its register budget then spills).
template <int ST>
constexpr int bulk_min_waves() { return ST >= ST_F16 ? 5 : 1; }

template <int ST, int COLL, int PAR>
__global__ __launch_bounds__(256, bulk_min_waves<ST>()) void k_stream_collide(StepArgs a) {
    bulk_part<ST, COLL, PAR>(a, int(blockIdx.x), int(gridDim.x));
}

// Add v (per lane) to the sharded interface count of the lane's domain; one
// atomic per wavefront when its lanes share a domain.  All lanes call.
__device__ __forceinline__ void count_interface(const StepArgs &a, int v, long long gid) {
    const int b = v ? int(a.g.dN.div(uint32_t(gid))) : -1;
    const unsigned long long mask = __ballot(v != 0);
    if (!mask) return;
    const int lead = __ffsll((long long)mask) - 1;
    const int b0 = __shfl(b, lead);
    const int shard = int(((blockIdx.x * blockDim.x + threadIdx.x) >> 6) % unsigned(ND_SHARDS));
    if (__ballot(v != 0 && b != b0) == 0) {
        int sum = v;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (__lane_id() == lead) atomicAdd(nif_slot(a.nif_dom, a.parity, a.B, b0, shard), sum);
    } else if (v) {
        atomicAdd(nif_slot(a.nif_dom, a.parity, a.B, b, shard), v);
    }
}

// Interface cells of the list: the same update plus mass exchange,
// anti-bounce-back, fill level and conversion marks; marked cells are listed.
template <int ST, int COLL, int PAR>
__global__ __launch_bounds__(256) void k_interface(StepArgs a) {
    if (blockIdx.x == 0) {
        // the conversion lists of this step start empty (the last step's
        // stayed readable through its excess work); the next step's interface
        // list too
        if (threadIdx.x == 0) {
            a.cnt[C_NEWG] = 0;
            a.cnt[C_FROML] = 0;
            a.cnt[C_RECV] = 0;
        }
        slist_reset(a.list_if_prev);
    }
    __shared__ int32_t pref[257];
    const SView lst = slist_view(a.list_if, pref);
    FOR_UNIFORM(k, in, lst.total) {
        long long gid = 0;
        bool marked = false;
        if (in) {
            gid = sview_at(lst, k);
            marked = update_cell<ST, COLL, PAR, true>(a, gid, a.flags[gid]);
        }
        slist_append(a.list_mark, marked, int32_t(gid), a.cnt + C_ERR);
        count_interface(a, in ? 1 : 0, gid);
    }
}

// ------------------------------------------------------------------ conversion

// Conflict rules over the marked interface cells: gas next to a cell filling over
// 1+eps becomes a new interface cell; a cell emptying under -eps next to a
// filling cell stays interface; liquid next to a remaining emptying cell
// becomes interface.  Each rule reads only the fill marks, so one pass does all.
// The same pass clears the conversion bit of the cells converted in the last
// step.
__global__ __launch_bounds__(256) void k_resolve(StepArgs a) {
    const long long N = a.g.N;
    __shared__ int32_t pref[257];
    const SView marks = slist_view(a.list_mark, pref);
    // the marks, then the cells converted in the last step (disjoint flag
    // bits, byte-atomic updates: one index space, side by side)
    const long long nmk = marks.total, ncp = clamp_cap(a, a.cnt[C_CONV0 + (1 - a.parity)]);
    FOR_UNIFORM(k, in, nmk + ncp) {
        uint32_t sel_g = 0, sel_l = 0;
        long long cbase = 0;
        int nb[Q];
        if (in && k >= nmk) {
            flag_clear(a.flags, a.list_conv_prev[k - nmk], F_CONV);
        } else if (in) {
            const long long gid = sview_at(marks, k);
            const Cell c = decode(a.g, gid);
            cbase = (long long)c.b * N;
            neighbours(a.g, c, nb);
            const uint8_t fl = a.flags[gid];
            uint8_t fn[Q];
#pragma unroll
            for (int i = 1; i < Q; ++i) fn[i] = a.flags[cbase + (nb[i] >= 0 ? nb[i] : c.n)];
            // the neighbours to mark (gas next to a filling cell, liquid next
            // to an emptying cell that no filling neighbour cancels)
            uint8_t bit = 0;
            uint32_t tmask = 0;
            if (fl & F_MARK_A) {
                bit = F_MARK_A;
#pragma unroll
                for (int i = 1; i < Q; ++i) tmask |= (nb[i] >= 0 && (fn[i] & F_GAS)) ? (1u << i) : 0u;
            } else if (fl & F_MARK_B) {
                bool near_fill = false;
#pragma unroll
                for (int i = 1; i < Q; ++i)
                    near_fill |= nb[i] >= 0 && (fn[i] & F_IF) && (fn[i] & F_MARK_A);
                if (near_fill) {
                    flag_clear(a.flags, gid, F_MARK_B);
                } else {
                    bit = F_MARK_B;
#pragma unroll
                    for (int i = 1; i < Q; ++i) tmask |= (nb[i] >= 0 && (fn[i] & F_LIQ)) ? (1u << i) : 0u;
                }
            }
            if (bit) {
                // one atomic per direction, issued without branches so that all
                // are in flight together (an OR of 0 where there is nothing to
                // mark); a cell is listed by the lane that set its mark
                uint8_t old[Q];
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const bool t = (tmask >> i) & 1u;
                    old[i] = flag_or(a.flags, nb[i] >= 0 ? cbase + nb[i] : gid, t ? bit : uint8_t(0));
                }
                uint32_t sel = 0;
#pragma unroll
                for (int i = 1; i < Q; ++i) sel |= (((tmask >> i) & 1u) && !(old[i] & bit)) ? (1u << i) : 0u;
                if (bit == F_MARK_A) sel_g = sel;
                else sel_l = sel;
            }
        }
        wave_append_sel<Q>(sel_g, [&](int i) { return int32_t(cbase + nb[i]); }, a.list_newg,
                           a.cnt + C_NEWG, a.cap, a.cnt + C_ERR);
        wave_append_sel<Q>(sel_l, [&](int i) { return int32_t(cbase + nb[i]); }, a.list_froml,
                           a.cnt + C_FROML, a.cap, a.cnt + C_ERR);
    }
}

// Refilling of one new interface cell x by 32 cooperating lanes (Sec. 3.1).
// Lane j in 1..18 loads neighbour x + c_j; lane i in 0..18 produces f_i.
// Returns nothing; writes the populations in the layout after this step and
// the cell's outgoing copy, and sets m = 0.
template <int ST, int SCHEME, int SLIP>
__device__ __forceinline__ void refill_group(const StepArgs &a, const long long gid, const int lane,
                                             const bool active) {
    const int layoutB = 1 - a.parity;   // layout after this step
    const long long N = a.g.N;
    const Cell c = decode(a.g, gid);
    const long long cbase = (long long)c.b * N;
    const double *gr = a.grav + 3 * c.b;
    const int j = lane;
    const bool has = active && j >= 1 && j < Q;
    const int ox = has ? k_cx[j] : 0, oy = has ? k_cy[j] : 0, oz = has ? k_cz[j] : 0;
    const int q = has ? nb_local(a.g, c.x, c.y, c.z, ox, oy, oz) : -1;
    // the neighbour's flag and populations are loaded together (the cell's
    // own at a wall or on an idle lane); values of cells that are not valid
    // sources are masked out below, never multiplied in
    const long long qg = cbase + (q >= 0 ? q : c.n);
    // EQ+NEQ and EXT need the fill-level gradient after streaming at the new
    // cell; it is taken before the neighbour's populations are loaded, so that
    // its 26 fill levels and those populations are not live together
    double nx_ = 0.0, ny_ = 0.0, nz_ = 0.0;
    if ((SCHEME == 1 || SCHEME == 3) && active)
        py_gradient(a.g, c, [&](long long k) { return a.phi_next[k]; }, nx_, ny_, nz_);
    const uint8_t fq = a.flags[qg];
    double d[Q];
    load_cell<ST, SLIP>(a, layoutB, decode(a.g, qg), d);
    issue_fence();
    const bool valid = q >= 0 && refill_source(fq);
    double r, ux, uy, uz;
    moments_post(d, gr[0], gr[1], gr[2], r, ux, uy, uz);
    const double vw = valid ? 1.0 : 0.0;
    const double nv = group32_sum(vw);
    const double rs = group32_sum(valid ? r : 0.0);
    const double usx = group32_sum(valid ? ux : 0.0), usy = group32_sum(valid ? uy : 0.0),
                 usz = group32_sum(valid ? uz : 0.0);
    double rb = 1.0, ubx = 0.0, uby = 0.0, ubz = 0.0;
    if (nv > 0.0) {
        rb = rs / nv;
        ubx = usx / nv; uby = usy / nv; ubz = usz / nv;
    }
    const int i = lane < Q ? lane : 0;   // output direction of this lane
    double out = feq_shift_rt(i, rb, ubx, uby, ubz);   // EQ

    if (SCHEME == 1 || SCHEME == 3) {
        // c^n: the valid direction best aligned with grad(phi) after streaming;
        // scores within rounding of the best tie and the lowest index wins
        const double sc = valid ? __dadd_rn(__dadd_rn(__dmul_rn(double(ox), nx_), __dmul_rn(double(oy), ny_)),
                                            __dmul_rn(double(oz), nz_))
                                : -1e300;
        const double best = group32_max(sc);
        const double tol = 1e-12 * (fabs(nx_) + fabs(ny_) + fabs(nz_));
        const unsigned long long cand = __ballot(valid && sc >= best - tol);
        const int gbase = __lane_id() & 32;
        const unsigned int gcand = unsigned((cand >> gbase) & 0xffffffffull);
        const int cn = gcand ? __ffs(gcand) - 1 : -1;   // lane index = direction
        if (SCHEME == 1 && cn > 0) {
            // EQ+NEQ: add the non-equilibrium part of the neighbour along c^n,
            // f*_i(y) - f_eq_i(rho(y), u(y)), y = x + c^n
            const int src = gbase + cn;
            const double rn = __shfl(r, src), uxn = __shfl(ux, src), uyn = __shfl(uy, src),
                         uzn = __shfl(uz, src);
            double mine = 0.0;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const double v = __shfl(d[k], src);
                if (k == i) mine = v;
            }
            out += mine - feq_shift_rt(i, rn, uxn, uyn, uzn);
        } else if (SCHEME == 3 && cn > 0) {
            // EXT: extrapolation along c^n, order limited by the run of valid cells
            const int ddx = k_cx[cn], ddy = k_cy[cn], ddz = k_cz[cn];
            const int k1 = nb_local(a.g, c.x, c.y, c.z, ddx, ddy, ddz);
            const Cell c1 = decode(a.g, cbase + k1);
            const int k2 = nb_local(a.g, c1.x, c1.y, c1.z, ddx, ddy, ddz);
            const bool v2 = k2 >= 0 && refill_source(a.flags[cbase + k2]);
            const Cell c2 = decode(a.g, cbase + (v2 ? k2 : k1));
            const int k3 = v2 ? nb_local(a.g, c2.x, c2.y, c2.z, ddx, ddy, ddz) : -1;
            const bool v3 = k3 >= 0 && refill_source(a.flags[cbase + k3]);
            const Cell c3 = decode(a.g, cbase + (v3 ? k3 : k1));
            const double f1 = load_slot<ST>(a, slot_flat_rt<SLIP>(a.g, layoutB, c1, i));
            const double f2 = load_slot<ST>(a, slot_flat_rt<SLIP>(a.g, layoutB, c2, i));
            const double f3 = load_slot<ST>(a, slot_flat_rt<SLIP>(a.g, layoutB, c3, i));
            out = (v2 && v3) ? 3.0 * f1 - 3.0 * f2 + f3 : (v2 ? 2.0 * f1 - f2 : f1);
        }
    } else if (SCHEME == 2) {
        // GEQ: Grad's approximation from finite-difference velocity gradients
        // (central if both face neighbours are valid, else one-sided with u(x) = u_bar)
        const int gb = __lane_id() & 32;
        double fu[7][3];
        bool fv[7];
#pragma unroll
        for (int f = 1; f <= 6; ++f) {
            fu[f][0] = __shfl(ux, gb + f);
            fu[f][1] = __shfl(uy, gb + f);
            fu[f][2] = __shfl(uz, gb + f);
            fv[f] = __shfl(vw, gb + f) > 0.0;
        }
        const double ub[3] = {ubx, uby, ubz};
        double du[3][3];
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            const int ip = 1 + 2 * be, im = 2 + 2 * be;
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                if (fv[ip] && fv[im]) du[al][be] = (fu[ip][al] - fu[im][al]) / 2.0;
                else if (fv[ip]) du[al][be] = fu[ip][al] - ub[al];
                else if (fv[im]) du[al][be] = ub[al] - fu[im][al];
                else du[al][be] = 0.0;
            }
        }
        const double tau = 1.0 / a.omega[c.b];
        const double cs2 = 1.0 / 3.0;
        const int ci[3] = {k_cx[i], k_cy[i], k_cz[i]};
        double s = 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
            for (int be = 0; be < 3; ++be)
                s += (du[al][be] + du[be][al]) * (cs2 * (al == be ? 1.0 : 0.0) - double(ci[al] * ci[be]));
        const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
        out += w * rb * tau / (2.0 * cs2) * s;
    } else if (SCHEME == 4) {
        // AVG: mean of the valid neighbours' populations, direction by direction
        double mine = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const double sk = group32_sum(valid ? d[k] : 0.0);
            if (k == i) mine = sk;
        }
        if (nv > 0.0) out = mine / nv;
    }
    if (active && lane < Q) {
        store_slot<ST>(a, slot_flat_rt<SLIP>(a.g, layoutB, c, i), out);
        if (i > 0) store_fo<ST>(a, i, gid, out);
    }
    // density after this step: the stored populations summed in direction order
    const double rt = lane < Q ? double(codec_round<ST>(typename Codec<ST>::T(out))) : 0.0;
    const int gl = __lane_id() & 32;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) s += __shfl(rt, gl + k);
    if (active && lane == 0) {
        a.m[gid] = 0.0;
        a.rho_if[gid] = 1.0 + s;
    }
}

// Density sum_i f*_i of a cell in the layout after this step, also returned
// as shifted populations.
template <int ST, int SLIP>
__device__ __forceinline__ double rho_after(const StepArgs &a, const Cell &c, double (&d)[Q]) {
    load_cell<ST, SLIP>(a, 1 - a.parity, c, d);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += d[i];
    return 1.0 + s;
}

// Conversions (Sec. 2.2, 3.1).  Work items: first every new interface cell
// (refilled by a group of 32 lanes), then every marked interface cell (filled
// cells become liquid, emptied cells gas; their excess mass is split over the
// receivers, which are claimed and listed, or sent to the reservoir; cells
// whose emptying was cancelled stay), then every from-liquid cell (mass = its
// density).  The per-domain interface counts are corrected on the way.  The
// new cells keep their gas-typed flag until k_excess, so the refill sources
// read the same validity throughout.
template <int ST, int SCHEME, int SLIP>
__global__ __launch_bounds__(256) void k_convert(StepArgs a) {
    const int p = a.parity;
    const long long N = a.g.N;
    __shared__ int32_t pref[257];
    const SView marks = slist_view(a.list_mark, pref);
    const long long nng = clamp_cap(a, a.cnt[C_NEWG]), nmk = marks.total, nfl = clamp_cap(a, a.cnt[C_FROML]);
    const long long R = (nng * 32 + 63) / 64 * 64;   // refill lanes, whole wavefronts
    FOR_UNIFORM(t, in, R + nmk + nfl) {
        bool conv = false;
        int dn = 0;            // change of the domain's interface count
        long long gid = 0, cbase = 0;
        uint32_t sel = 0;      // receivers claimed by this lane
        int nb[Q];
        if (t < R) {
            // refill: a wavefront never mixes with the items below
            const long long cell = t >> 5;
            const bool active = in && cell < nng;
            const long long g0 = active ? a.list_newg[cell] : 0;
            refill_group<ST, SCHEME, SLIP>(a, g0, int(t & 31), active);
            gid = g0;
            if (active && (t & 31) == 0) {
                // a new interface cell may sit in a tile that never held fluid
                activate_tile(a.tiles, a.tile_bits, a.cnt + C_TILES, int32_t(g0 >> TILE_SHIFT),
                              int32_t(tile_count(a.g.BN)));
                dn = 1;
            }
        } else if (in) {
            const long long k = t - R;
            gid = k < nmk ? sview_at(marks, k) : a.list_froml[k - nmk];
            const Cell c = decode(a.g, gid);
            cbase = (long long)c.b * N;
            if (k < nmk) {
                const uint8_t fl = a.flags[gid];
                if (fl & (F_MARK_A | F_MARK_B)) {
                    const bool fill = (fl & F_MARK_A) != 0;
                    neighbours(a.g, c, nb);
                    uint8_t fq[Q];
#pragma unroll
                    for (int i = 1; i < Q; ++i) fq[i] = a.flags[cbase + (nb[i] >= 0 ? nb[i] : c.n)];
                    double d[Q];
                    const double mx = fill ? a.m[gid] - rho_after<ST, SLIP>(a, c, d) : a.m[gid];
                    int nr = 0;
                    uint32_t recv = 0;
#pragma unroll
                    for (int i = 1; i < Q; ++i)
                        if (nb[i] >= 0 && type_after(fq[i]) == F_IF) { ++nr; recv |= 1u << i; }
                    if (nr == 0) {
                        atomicAdd(a.res + p * a.B + c.b, mx);
                        a.mex[gid] = 0.0;
                    } else {
                        a.mex[gid] = mx / nr;
                        // claim the receivers (each is listed once); one atomic
                        // per direction without branches, as in k_resolve
                        uint8_t old[Q];
#pragma unroll
                        for (int i = 1; i < Q; ++i)
                            old[i] = flag_or(a.claim, nb[i] >= 0 ? cbase + nb[i] : gid,
                                             ((recv >> i) & 1u) ? uint8_t(1) : uint8_t(0));
#pragma unroll
                        for (int i = 1; i < Q; ++i)
                            sel |= (((recv >> i) & 1u) && !(old[i] & 1)) ? (1u << i) : 0u;
                    }
                    a.flags[gid] = uint8_t((fill ? F_LIQ : F_GAS) | F_CONV);
                    a.m[gid] = 0.0;
                    conv = true;
                    dn = -1;
                }
            } else {
                // from liquid: mass = density; keep a copy of its populations
                double d[Q];
                const double rho = rho_after<ST, SLIP>(a, c, d);
                a.m[gid] = rho;
                a.rho_if[gid] = rho;
#pragma unroll
                for (int i = 1; i < Q; ++i) store_fo<ST>(a, i, gid, d[i]);
                a.flags[gid] = F_IF;
                dn = 1;
            }
        }
        wave_append(conv, int32_t(gid), a.list_conv, a.cnt + C_CONV0 + p, a.cap, a.cnt + C_ERR);
        wave_append_sel<Q>(sel, [&](int i) { return int32_t(cbase + nb[i]); }, a.list_recv,
                           a.cnt + C_RECV, a.cap, a.cnt + C_ERR);
        count_interface(a, dn, gid);
    }
}

// Excess mass of one receiver (Sec. 2.2): the shares of its converted
// neighbours plus the reservoir share r; phi = m/rho* if its mass changed.
template <int ST>
__device__ __forceinline__ void receive(const StepArgs &a, long long gid, double r) {
    const Cell c = decode(a.g, gid);
    const long long cbase = (long long)c.b * a.g.N;
    int nb[Q];
    neighbours(a.g, c, nb);
    // (the excess-mass work mostly runs inside the bulk kernel, where its
    // latency is hidden and its register count sets the bulk's occupancy:
    // these loads are left as dependent as the compiler makes them)
    uint8_t fq[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) fq[i] = nb[i] >= 0 ? a.flags[cbase + nb[i]] : uint8_t(0);
    double add = 0.0;
    bool touched = false;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (fq[i] & F_CONV) {
            // a converted neighbour that had receivers (it has at least this one)
            add += a.mex[cbase + nb[i]];
            touched = true;
        }
    }
    double m = a.m[gid];
    if (touched) m = m + add;
    if (r != 0.0) {
        m = m + r;
        touched = true;
    }
    if (touched) {
        a.m[gid] = m;
        a.phi_next[gid] = m / a.rho_if[gid];
    }
}

// Excess-mass redistribution and the end of the step.  Receivers gather the
// shares of their converted neighbours.  Every interface cell after the
// conversions (this step's list entries that are still interface, the new and
// the from-liquid cells) gets its type and forced class, and in a domain whose
// reservoir is spread its share of it (receivers of such a domain are left to
// this loop).  Converted cells get phi in {0, 1} in both fill-level buffers.
// Workgroup 0 carries the reservoir over and clears the interface counts the
// next step accumulates.  wg / nwg: this workgroup's index among the nwg
// workgroups that share the work (the whole grid, or a part of the next
// step's bulk grid).
template <int ST>
__device__ __forceinline__ void excess_part(const StepArgs &a, const int wg, const int nwg) {
    const int p = a.parity;
    const double *res = a.res + p * a.B;
    // the reservoir is spread when it holds mass and the domain has interface cells
    auto spreads = [&](int b) { return res[b] != 0.0 && nif_sum(a.nif_dom, p, a.B, b) > 0; };
    if (wg == 0) {
        for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
            // mass that found no receiver is kept while the domain has no interface
            a.res[(1 - p) * a.B + b] = spreads(b) ? 0.0 : res[b];
        }
        for (int k = threadIdx.x; k < a.B * ND_SHARDS; k += blockDim.x)
            *nif_slot(a.nif_dom, 1 - p, a.B, k / ND_SHARDS, k % ND_SHARDS) = 0;
        if (a.rhoG) slist_reset(a.list_band);   // the band list exists with surface tension only
    }
    bool spread_any = false;
    for (int b = threadIdx.x; b < a.B; b += blockDim.x) spread_any |= spreads(b);
    spread_any = __syncthreads_or(spread_any);
    __shared__ int32_t pref[257];
    const SView lst = slist_view(a.list_if, pref);
    // The three kinds of work items below touch disjoint data, so they share
    // one index space and run side by side: receivers, then every interface
    // cell after the conversions (this step's list entries, the new and the
    // from-liquid cells), then the converted cells.
    const long long nr = clamp_cap(a, a.cnt[C_RECV]);
    const long long n0 = lst.total, n1 = clamp_cap(a, a.cnt[C_NEWG]), n2 = clamp_cap(a, a.cnt[C_FROML]);
    const long long nif = n0 + n1 + n2, ncv = clamp_cap(a, a.cnt[C_CONV0 + p]);
    for (long long t = (long long)wg * blockDim.x + threadIdx.x; t < nr + nif + ncv;
         t += (long long)nwg * blockDim.x) {
        if (t < nr) {
            const long long gid = a.list_recv[t];
            a.claim[gid] = 0;
            if (!spread_any || !spreads(int(a.g.dN.div(uint32_t(gid))))) receive<ST>(a, gid, 0.0);
            continue;
        }
        if (t >= nr + nif) {
            // converted cells: phi in {0, 1} in both fill-level buffers
            const long long gid = a.list_conv[t - nr - nif];
            const double v = (a.flags[gid] & F_LIQ) ? 1.0 : 0.0;
            a.phi_cur[gid] = v;
            a.phi_next[gid] = v;
            continue;
        }
        // an interface cell after the conversions: its forced filling/emptying
        // class (Thuerey) from the final neighbour types, and in a domain
        // whose reservoir is spread its share
        const long long k = t - nr;
        long long gid;
        if (k < n0) {
            gid = sview_at(lst, k);
            if (type_after(a.flags[gid]) != F_IF) continue;
        } else {
            gid = k - n0 < n1 ? a.list_newg[k - n0] : a.list_froml[k - n0 - n1];
        }
        const Cell c = decode(a.g, gid);
        const long long cbase = (long long)c.b * a.g.N;
        int nb[Q];
        neighbours(a.g, c, nb);
        bool has_liq = false, has_gas = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint8_t ty = nb[i] >= 0 ? type_after(a.flags[cbase + nb[i]]) : uint8_t(0);
            has_liq |= ty == F_LIQ;
            has_gas |= ty == F_GAS;
        }
        a.flags[gid] = uint8_t(F_IF | (!has_liq ? F_NOFLUID : (!has_gas ? F_NOEMPTY : 0)));
        if (spread_any && spreads(c.b)) receive<ST>(a, gid, res[c.b] / nif_sum(a.nif_dom, p, a.B, c.b));
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_excess(StepArgs a) {
    excess_part<ST>(a, int(blockIdx.x), int(gridDim.x));
}

// Workgroups of the last step's excess-mass work ahead of the bulk grid.
constexpr int EXCESS_WG = 512;

// The bulk kernel of this step (a) fused with the excess-mass work of the last
// step (ae).  The two touch disjoint data: the excess work writes mass, fill
// levels, the flag bytes of interface cells (type-preserving) and its own
// counters; the bulk work writes the populations of liquid cells only (every
// cell's slot set is its own).  Its latency-bound chains overlap the
// bandwidth-bound bulk instead of running as a kernel of their own.
template <int ST, int COLL, int PAR>
__global__ __launch_bounds__(256, bulk_min_waves<ST>()) void k_excess_stream_collide(StepArgs a, StepArgs ae) {
    if (blockIdx.x < EXCESS_WG)
        excess_part<ST>(ae, int(blockIdx.x), EXCESS_WG);
    else
        bulk_part<ST, COLL, PAR>(a, int(blockIdx.x) - EXCESS_WG, int(gridDim.x) - EXCESS_WG);
}


// ------------------------------------------------------------------ launchers

// List kernels get a fixed grid (the list lengths are only known on the
// device); 2048 workgroups cover 512k items per pass.
static int list_blocks(long long cap) {
    long long b = (cap + 255) / 256;
    return int(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

template <typename K>
static void launch_bulk(K kernel, const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.bulk_grid)), dim3(256), 0, s, a);
}

// With ev, the bulk kernel is launched with start and stop events that its
// dispatch itself stamps (hipExtLaunchKernelGGL), so the timed duration is the
// kernel's alone, without the gaps around it.
template <int ST, int COLL, int PAR>
static void launch_bulk_t(const StepArgs &a, const StepArgs *pending, hipStream_t s, const BulkEvents *ev) {
    const dim3 fused(unsigned(EXCESS_WG + a.bulk_grid)), plain(unsigned(a.bulk_grid));
    if (ev && pending)
        hipExtLaunchKernelGGL((k_excess_stream_collide<ST, COLL, PAR>), fused, dim3(256), 0, s, ev->before,
                              ev->after, 0, a, *pending);
    else if (ev)
        hipExtLaunchKernelGGL((k_stream_collide<ST, COLL, PAR>), plain, dim3(256), 0, s, ev->before, ev->after,
                              0, a);
    else if (pending)
        hipLaunchKernelGGL((k_excess_stream_collide<ST, COLL, PAR>), fused, dim3(256), 0, s, a, *pending);
    else
        launch_bulk(k_stream_collide<ST, COLL, PAR>, a, s);
}

// Calls f(C, P) with the collision variant and the step parity as
// compile-time constants (std::integral_constant).
template <int ST, typename F>
static void launch_coll(int coll, int parity, F &&f) {
    using std::integral_constant;
    auto par = [&](auto C) {
        if (parity == 0) f(C, integral_constant<int, 0>{});
        else f(C, integral_constant<int, 1>{});
    };
    switch (coll) {
        case 0: par(integral_constant<int, 0>{}); break;
        case 1: par(integral_constant<int, 1>{}); break;
        case 2: par(integral_constant<int, 2>{}); break;
        case 3: par(integral_constant<int, 3>{}); break;
        case 4: par(integral_constant<int, 4>{}); break;
        case 5: par(integral_constant<int, 5>{}); break;
        case 6: par(integral_constant<int, 6>{}); break;
        default: par(integral_constant<int, 7>{}); break;
    }
}

template <int ST>
static void launch_step_t(const StepArgs &a, int collision, int scheme, hipStream_t s,
                          const BulkEvents *ev, const StepArgs *pending, bool finish,
                          const StepHook *after_bulk) {
    const int lb = list_blocks(a.cap);
    if (pending && a.rhoG) {
        hipLaunchKernelGGL(k_excess<ST>, dim3(lb), dim3(256), 0, s, *pending);
        pending = nullptr;
    }
    if (a.rhoG) {
        hipLaunchKernelGGL(k_band, dim3(lb), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_normals, dim3(lb), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_curvature, dim3(lb), dim3(256), 0, s, a);
    }
    // collision variant: bit 0 TRT, bit 1 Smagorinsky turbulence model, bit 2
    // free-slip walls
    const int coll = (collision ? 1 : 0) | (a.les_k > 0.0 ? 2 : 0) | (a.g.slip ? 4 : 0);
    launch_coll<ST>(coll, a.parity, [&](auto C, auto P) {
        launch_bulk_t<ST, decltype(C)::value, decltype(P)::value>(a, pending, s, ev);
    });
    if (after_bulk) after_bulk->fn(after_bulk->arg, s);
    launch_coll<ST>(coll, a.parity, [&](auto C, auto P) {
        hipLaunchKernelGGL((k_interface<ST, decltype(C)::value, decltype(P)::value>), dim3(lb), dim3(256), 0,
                           s, a);
    });
    hipLaunchKernelGGL(k_resolve, dim3(lb), dim3(256), 0, s, a);
    auto convert = [&](auto SL) {
        constexpr int SLIP = decltype(SL)::value;
        switch (scheme) {
            case 0: hipLaunchKernelGGL((k_convert<ST, 0, SLIP>), dim3(lb), dim3(256), 0, s, a); break;
            case 1: hipLaunchKernelGGL((k_convert<ST, 1, SLIP>), dim3(lb), dim3(256), 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_convert<ST, 2, SLIP>), dim3(lb), dim3(256), 0, s, a); break;
            case 3: hipLaunchKernelGGL((k_convert<ST, 3, SLIP>), dim3(lb), dim3(256), 0, s, a); break;
            default: hipLaunchKernelGGL((k_convert<ST, 4, SLIP>), dim3(lb), dim3(256), 0, s, a); break;
        }
    };
    if (a.g.slip) convert(std::integral_constant<int, 1>{});
    else convert(std::integral_constant<int, 0>{});
    if (finish) hipLaunchKernelGGL(k_excess<ST>, dim3(lb), dim3(256), 0, s, a);
}

}  // namespace

#if defined(FSLBM_UNIT_STORAGE)
template <>
void launch_step_storage<FSLBM_UNIT_STORAGE>(const StepArgs &a, int collision, int scheme,
                                             hipStream_t s, const BulkEvents *ev,
                                             const StepArgs *pending, bool finish,
                                             const StepHook *after_bulk) {
    launch_step_t<FSLBM_UNIT_STORAGE>(a, collision, scheme, s, ev, pending, finish, after_bulk);
}
template <>
void launch_excess_storage<FSLBM_UNIT_STORAGE>(const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_excess<FSLBM_UNIT_STORAGE>, dim3(list_blocks(a.cap)), dim3(256), 0, s, a);
}
#endif

#if defined(FSLBM_UNIT_DISPATCH)
void launch_step(const StepArgs &a, int storage, int collision, int scheme, hipStream_t s,
                 const BulkEvents *ev, const StepArgs *pending, bool finish, const StepHook *after_bulk) {
    switch (storage) {
        case ST_F64: launch_step_storage<ST_F64>(a, collision, scheme, s, ev, pending, finish, after_bulk); break;
        case ST_F32: launch_step_storage<ST_F32>(a, collision, scheme, s, ev, pending, finish, after_bulk); break;
        case ST_F16: launch_step_storage<ST_F16>(a, collision, scheme, s, ev, pending, finish, after_bulk); break;
        default: launch_step_storage<ST_BF16>(a, collision, scheme, s, ev, pending, finish, after_bulk); break;
    }
}
void launch_excess(const StepArgs &a, int storage, hipStream_t s) {
    switch (storage) {
        case ST_F64: launch_excess_storage<ST_F64>(a, s); break;
        case ST_F32: launch_excess_storage<ST_F32>(a, s); break;
        case ST_F16: launch_excess_storage<ST_F16>(a, s); break;
        default: launch_excess_storage<ST_BF16>(a, s); break;
    }
}
#endif

}  // namespace fslbm
