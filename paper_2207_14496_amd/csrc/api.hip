// api.hip -- host side of the FSLBM library: workspace carving, the context,
// initial-state upload, canonical read-back, diagnostics, HIP-graph replay of
// the step sequence and the C ABI declared in include/fslbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fslbm.h"
#include "context.hpp"
#include "fslbm_kernels.hpp"
#include "fslbm_math.hpp"

using namespace fslbm;

namespace {

constexpr int DIAG_BLOCKS = 256;

size_t storage_bytes(int st) { return st == FSLBM_F64 ? 8 : (st == FSLBM_F32 ? 4 : 2); }

bool make_layout(const fslbm_params &p, Layout &L) {
    long long N = (long long)p.nx * p.ny * p.nz;
    long long BN = N * p.batch;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.pdf = take(size_t(BN) * Q * storage_bytes(p.storage));
    L.flags = take(size_t(BN) + 4);
    L.m = take(size_t(BN) * 8);
    L.phi = take(size_t(BN) * 16);   // two buffers
    L.fo = take(size_t(BN) * 18 * storage_bytes(p.storage));
    L.mex = take(size_t(BN) * 8);
    L.rho_if = take(size_t(BN) * 8);
    bool surf = p.sigma != 0.0;
    L.rhoG = surf ? take(size_t(BN) * 8) : 0;
    L.normal = surf ? take(size_t(BN) * 24) : 0;
    L.band = surf ? take(size_t((BN + 31) / 32) * 4) : 0;
    for (int k = 0; k < 5; ++k) L.lists[k] = take(size_t(BN) * 4);
    // sharded lists: S slots of seg entries plus an overflow region of BN entries
    L.sl_S = int32_t(std::max<long long>(1, std::min<long long>(256, BN / 1024)));
    L.sl_seg = int32_t((BN + L.sl_S - 1) / L.sl_S);
    L.sl_ovf = int32_t(BN);
    for (int k = 0; k < 4; ++k) {
        const bool need = k < 3 || surf;
        L.sl_data[k] = need ? take((size_t(L.sl_S) * L.sl_seg + size_t(L.sl_ovf)) * 4) : 0;
        L.sl_cnt[k] = need ? take(size_t(L.sl_S + 1) * 32 * 4) : 0;
    }
    L.claim = take(size_t(BN) + 4);
    L.cnt = take(C_COUNT * 4);
    L.nif = take(size_t(2 * p.batch) * ND_SHARDS * 32 * 4);
    L.res = take(size_t(2 * p.batch) * 8);
    L.omega = take(size_t(p.batch) * 16);   // omega (omega+) [B], then TRT omega- [B]
    L.grav = take(size_t(p.batch) * 24);
    L.diag_d = take(size_t(p.batch) * DIAG_BLOCKS * 2 * 8);
    L.diag_i = take(size_t(p.batch) * DIAG_BLOCKS * 4 * 8);
    const size_t ntiles = size_t(tile_count(BN));
    L.tiles = take(ntiles * 4);
    L.tile_bits = take((ntiles + 31) / 32 * 4);
    const bool bub = p.bubble_model != 0;
    L.pbub = bub ? take(size_t(BN) * 8) : 0;
    L.blab0 = bub ? take(size_t(BN) * 4) : 0;
    L.blab1 = bub ? take(size_t(BN) * 4) : 0;
    L.bV0 = bub ? take(size_t(BN) * 8) : 0;
    L.bV1 = bub ? take(size_t(BN) * 8) : 0;
    L.bkept = bub ? take(size_t(BN) * 8) : 0;
    L.bamount = bub ? take(size_t(BN) * 8) : 0;
    L.batm = bub ? take(size_t(BN) * 4) : 0;
    L.total = off;
    return true;
}

const char *validate(const fslbm_params *p) {
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->batch < 1) return "sizes must be >= 1";
    long long BN = (long long)p->nx * p->ny * p->nz * p->batch;
    if (BN >= (1LL << 31) - 64) return "more than 2^31 cells in total";
    if ((long long)p->nx * p->ny * p->nz * Q >= (1LL << 32)) return "more than 2^32 / 19 cells per domain";
    if (!(p->omega > 0.0 && p->omega < 2.0)) return "omega must lie in (0, 2)";
    if (p->collision != FSLBM_SRT && p->collision != FSLBM_TRT) return "unknown collision";
    if (p->storage < FSLBM_F64 || p->storage > FSLBM_BF16) return "unknown storage";
    if (p->refill < FSLBM_REFILL_EQ || p->refill > FSLBM_REFILL_AVG) return "unknown refill scheme";
    if (p->collision == FSLBM_TRT && !(p->trt_lambda > 0.0)) return "trt_lambda must be > 0";
    if (!(p->eps_phi >= 0.0)) return "eps_phi must be >= 0";
    if (!(p->smagorinsky_cs >= 0.0) || !(p->smagorinsky_cs < 1e3)) return "smagorinsky_cs must be finite and >= 0";
    if (p->free_slip != 0 && p->free_slip != 1) return "free_slip must be 0 or 1";
    if (p->bubble_model != 0 && p->bubble_model != 1) return "bubble_model must be 0 or 1";
    if (p->diag_every < 0) return "diag_every must be >= 0";
    if (p->omega_b)
        for (int b = 0; b < p->batch; ++b)
            if (!(p->omega_b[b] > 0.0 && p->omega_b[b] < 2.0)) return "omega_b must lie in (0, 2)";
    for (int a = 0; a < 3; ++a)
        if (p->periodic[a] != 0 && p->periodic[a] != 1) return "periodic must be 0 or 1";
    return nullptr;
}

std::string g_init_error = "no error";

// The workspace of fslbm_init_static: one array per device, held until the
// process ends.  In host code the array's name is only a host-side stand-in;
// every host use goes through the device address that hipGetSymbolAddress
// returns for the current device, kept per device in g_static.
constexpr size_t STATIC_WS_BYTES = size_t(FSLBM_STATIC_WORKSPACE_BYTES);
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];
constexpr int STATIC_MAX_DEVICES = 64;
struct StaticSlot {
    void *ptr = nullptr;          // device address of `scratch` on this device
    fslbm_ctx *owner = nullptr;   // the live context that uses it, if any
};
std::mutex g_static_mu;
StaticSlot g_static[STATIC_MAX_DEVICES];

// ------------------------------------------------------------------ init kernels

struct InitArgs {
    StepArgs s;
    const uint8_t *flags_in;
    const double *phi_in, *rho_in, *u_in, *pdf_in, *mass_in;
};

template <int ST>
__global__ void k_init_cells(InitArgs ia) {
    const StepArgs &a = ia.s;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.g.BN) return;
    using C = Codec<ST>;
    typename C::M *pdf = static_cast<typename C::M *>(a.pdf);
    Cell c = decode(a.g, gid);
    const long long N = a.g.N;
    uint8_t fl = ia.flags_in[gid];
    double ph = ia.phi_in[gid];
    int err = 0;
    if (fl != F_LIQ && fl != F_IF && fl != F_GAS) { err |= E_BAD_FLAG; fl = F_GAS; }
    if ((fl == F_LIQ && ph != 1.0) || (fl == F_GAS && ph != 0.0) || !isfinite(ph)) err |= E_BAD_PHI;
    if (fl == F_LIQ) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long q = nb_dir(a.g, c, i);
            if (q >= 0 && ia.flags_in[q] == F_GAS) err |= E_OPEN_LAYER;
        }
    }
    if (err) atomicOr(a.cnt + C_ERR, err);
    a.flags[gid] = fl;
    a.phi_cur[gid] = ph;
    a.phi_next[gid] = ph;
    bool fluid = fl != F_GAS;
    double d[Q];
    if (!fluid) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = 0.0;
    } else if (ia.pdf_in) {
        const double *src = ia.pdf_in + (long long)c.b * Q * N + c.n;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = src[i * N] - wgt<double>(i);
    } else {
        double r = ia.rho_in[gid];
        const double *u = ia.u_in + (long long)c.b * 3 * N + c.n;
        double ux = u[0], uy = u[N], uz = u[2 * N];
        double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = feq_shift<double>(i, r, r - 1.0, ux, uy, uz, uu);
    }
    // layout A: f*_i(x) in slot (opp(i), x)
    typename C::M *base = pdf + (long long)c.b * Q * N + c.n;
#pragma unroll
    for (int i = 0; i < Q; ++i) C::store(base + opp(i) * N, typename C::T(d[i]));
    if (fl == F_IF) {
        // outgoing populations of interface cells, read by the next mass exchange
        typename C::M *fo = static_cast<typename C::M *>(a.fo);
#pragma unroll
        for (int i = 1; i < Q; ++i) C::store(fo + fo_index(gid, i), typename C::T(d[i]));
    }
    double m = 0.0;
    if (fl == F_IF) {
        if (ia.mass_in) {
            m = ia.mass_in[gid];
        } else {
            double r;
            if (ia.pdf_in) {
                double s = 0.0;
                const double *src = ia.pdf_in + (long long)c.b * Q * N + c.n;
#pragma unroll
                for (int i = 0; i < Q; ++i) s += src[i * N];
                r = s;
            } else {
                r = ia.rho_in[gid];
            }
            m = ph * r;
        }
    }
    a.m[gid] = m;
}

// Forced filling/emptying classes and the interface list of the step before the
// first (read by the surface-tension kernels of the first step).
__global__ void k_init_lists(StepArgs a) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool in = gid < a.g.BN;
    bool is_if = in && a.flags[gid] == F_IF;
    if (is_if) {
        Cell c = decode(a.g, gid);
        bool has_liq = false, has_gas = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            long long q = nb_dir(a.g, c, i);
            if (q < 0) continue;
            uint8_t fq = a.flags[q] & F_TYPE;
            has_liq |= fq == F_LIQ;
            has_gas |= fq == F_GAS;
        }
        a.flags[gid] = uint8_t(F_IF | (!has_liq ? F_NOFLUID : (!has_gas ? F_NOEMPTY : 0)));
    }
    slist_append(a.list_if_prev, is_if, int32_t(gid), a.cnt + C_ERR);
}

// The tiles (one wavefront of consecutive cells each) that hold liquid or
// interface cells: first their membership bits (one atomic per workgroup),
// then the list itself in tile order (k_tile_list).
__global__ __launch_bounds__(256) void k_init_tiles(StepArgs a) {
    static_assert(TILE == 64, "one tile per wavefront");
    __shared__ uint32_t has;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool fluid = gid < a.g.BN && (a.flags[gid] & (F_LIQ | F_IF));
    const int w = int(threadIdx.x >> 6);
    const bool any = __ballot(fluid) != 0;
    if (threadIdx.x == 0) has = 0;
    __syncthreads();
    if (any && __lane_id() == 0) atomicOr(&has, 1u << w);
    __syncthreads();
    const int32_t t0 = int32_t(blockIdx.x) * 4;   // the workgroup's four tiles share one bit word
    if (threadIdx.x == 0 && has) atomicOr(a.tile_bits + (t0 >> 5), has << (t0 & 31));
}

// The tile list from the membership bits, in ascending tile order, and its
// length.  One workgroup of 1024 threads; thread t takes a contiguous run of
// bit words, so the list order is the memory order of the cells.  The bulk
// kernel's wavefronts take consecutive list entries, so neighbouring tiles
// are updated side by side (on the dense pool, 701 -> 642 us per FP32 bulk
// launch against the order of the workgroups' atomics).  Runs once per load.
__global__ __launch_bounds__(1024) void k_tile_list(StepArgs a) {
    __shared__ int32_t wave_sum[16];
    const long long nwords = (tile_count(a.g.BN) + 31) / 32;
    const long long per = (nwords + blockDim.x - 1) / blockDim.x;
    const long long s0 = (long long)threadIdx.x * per;
    const long long w0 = s0 < nwords ? s0 : nwords;
    const long long w1 = w0 + per < nwords ? w0 + per : nwords;
    int32_t n = 0;
    for (long long w = w0; w < w1; ++w) n += __popc(a.tile_bits[w]);
    // exclusive prefix of n over the workgroup: in each wavefront by
    // shuffles, then over the sixteen wavefronts through shared memory
    const int lane = __lane_id(), wv = int(threadIdx.x >> 6);
    int32_t x = n;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_sum[wv] = x;
    __syncthreads();
    int32_t pos = x - n;
    for (int k = 0; k < wv; ++k) pos += wave_sum[k];
    for (long long w = w0; w < w1; ++w) {
        uint32_t bits = a.tile_bits[w];
        while (bits) {
            a.tiles[pos++] = int32_t(w * 32 + (__ffs(bits) - 1));
            bits &= bits - 1u;
        }
    }
    if (threadIdx.x == blockDim.x - 1) a.cnt[C_TILES] = pos;
}

// ------------------------------------------------------------------ read-back

struct ReadArgs {
    StepArgs s;
    int layoutB;
    uint32_t mask;
    uint8_t *flags;
    double *pdf, *mass, *phi, *rho, *vel;
};

template <int ST>
__global__ void k_read(ReadArgs r) {
    const StepArgs &a = r.s;
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.g.BN) return;
    Cell c = decode(a.g, gid);
    const long long N = a.g.N;
    uint8_t fl = a.flags[gid] & F_TYPE;
    bool fluid = fl != F_GAS;
    if (r.mask & FSLBM_FIELD_FLAGS) r.flags[gid] = fl;
    if (r.mask & FSLBM_FIELD_MASS) r.mass[gid] = fl == F_IF ? a.m[gid] : 0.0;
    if (r.mask & FSLBM_FIELD_PHI) r.phi[gid] = a.phi_cur[gid];
    if (r.mask & (FSLBM_FIELD_PDF | FSLBM_FIELD_RHO | FSLBM_FIELD_VEL)) {
        double d[Q];
        if (fluid) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                using Cd = Codec<ST>;
                d[i] = double(Cd::load(static_cast<const typename Cd::M *>(a.pdf) +
                                       slot_flat(a.g, r.layoutB, c, i)));
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] = 0.0;
        }
        if (r.mask & FSLBM_FIELD_PDF) {
            double *dst = r.pdf + (long long)c.b * Q * N + c.n;
#pragma unroll
            for (int i = 0; i < Q; ++i) dst[i * N] = fluid ? wgt<double>(i) + d[i] : 0.0;
        }
        if (r.mask & (FSLBM_FIELD_RHO | FSLBM_FIELD_VEL)) {
            double rho = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
            if (fluid) {
                const double *gr = a.grav + 3 * c.b;
                moments_post(d, gr[0], gr[1], gr[2], rho, ux, uy, uz);
            }
            if (r.mask & FSLBM_FIELD_RHO) r.rho[gid] = rho;
            if (r.mask & FSLBM_FIELD_VEL) {
                double *v = r.vel + (long long)c.b * 3 * N + c.n;
                v[0] = ux; v[N] = uy; v[2 * N] = uz;
            }
        }
    }
}

// ------------------------------------------------------------------ diagnostics

// Per-domain partial sums with a fixed-order tree (deterministic).
template <int ST>
__global__ __launch_bounds__(256) void k_diag_partial(StepArgs a, int layoutB, double *pd,
                                                      long long *pi) {
    const int b = blockIdx.y;
    const long long N = a.g.N;
    double mass = 0.0, vmax = 0.0;
    long long nl = 0, ni = 0, ng = 0, bad = 0;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        long long gid = (long long)b * N + n;
        uint8_t fl = a.flags[gid] & F_TYPE;
        if (fl == F_GAS) { ++ng; continue; }
        double d[Q];
        Cell c = decode(a.g, gid);
        bool fin = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            using Cd = Codec<ST>;
            d[i] = double(Cd::load(static_cast<const typename Cd::M *>(a.pdf) +
                                   slot_flat(a.g, layoutB, c, i)));
            fin &= isfinite(d[i]);
        }
        const double *gr = a.grav + 3 * b;
        double rho, ux, uy, uz;
        moments_post(d, gr[0], gr[1], gr[2], rho, ux, uy, uz);
        double sp = sqrt(ux * ux + uy * uy + uz * uz);
        if (fl == F_LIQ) { ++nl; mass += rho; }
        else { ++ni; mass += a.m[gid]; fin &= isfinite(a.m[gid]) && isfinite(a.phi_cur[gid]); }
        vmax = fin ? (sp > vmax ? sp : vmax) : vmax;
        bad += !fin || !isfinite(sp);
    }
    __shared__ double sm[256], sv[256];
    __shared__ long long s0[256], s1[256], s2[256], s3[256];
    int t = threadIdx.x;
    sm[t] = mass; sv[t] = vmax; s0[t] = nl; s1[t] = ni; s2[t] = ng; s3[t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sm[t] += sm[t + w];
            sv[t] = sv[t] > sv[t + w] ? sv[t] : sv[t + w];
            s0[t] += s0[t + w]; s1[t] += s1[t + w]; s2[t] += s2[t + w]; s3[t] += s3[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        long long o = (long long)b * gridDim.x + blockIdx.x;
        pd[2 * o] = sm[0];
        pd[2 * o + 1] = sv[0];
        pi[4 * o] = s0[0]; pi[4 * o + 1] = s1[0]; pi[4 * o + 2] = s2[0]; pi[4 * o + 3] = s3[0];
    }
}

}  // namespace

// ------------------------------------------------------------------ context

namespace fslbm {

StepArgs make_args(fslbm_ctx *c, int parity) {
    StepArgs a{};
    const fslbm_params &p = c->p;
    a.g.nx = p.nx; a.g.ny = p.ny; a.g.nz = p.nz;
    for (int k = 0; k < 3; ++k) a.g.per[k] = p.periodic[k];
    a.g.slip = p.free_slip;
    a.g.N = (long long)p.nx * p.ny * p.nz;
    a.g.BN = a.g.N * p.batch;
    a.g.dx = FastDiv::make(uint32_t(p.nx));
    a.g.dy = FastDiv::make(uint32_t(p.ny));
    a.g.dN = FastDiv::make(uint32_t(a.g.N));
    a.pdf = c->ws + c->L.pdf;
    a.flags = at<uint8_t>(c, c->L.flags);
    a.m = at<double>(c, c->L.m);
    // fill level: buffer (steps done) mod 2 holds the current one
    a.phi_cur = at<double>(c, c->L.phi) + size_t(parity) * size_t(a.g.BN);
    a.phi_next = at<double>(c, c->L.phi) + size_t(1 - parity) * size_t(a.g.BN);
    a.fo = c->ws + c->L.fo;
    a.mex = at<double>(c, c->L.mex);
    a.rho_if = at<double>(c, c->L.rho_if);
    bool surf = p.sigma != 0.0;
    a.rhoG = surf ? at<double>(c, c->L.rhoG) : nullptr;
    a.pbub = p.bubble_model ? at<double>(c, c->L.pbub) : nullptr;
    a.normal = surf ? at<double>(c, c->L.normal) : nullptr;
    a.band = surf ? at<uint32_t>(c, c->L.band) : nullptr;
    a.omega = at<double>(c, c->L.omega);
    a.omega_m = a.omega + p.batch;
    a.pdf_off32 = (long long)p.nx * p.ny * p.nz * Q * (long long)storage_bytes(p.storage) < (1LL << 32) ? 1 : 0;
    a.grav = at<double>(c, c->L.grav);
    a.trt_lambda = p.trt_lambda;
    // 2 C_S^2 / c_s^4 with c_s^2 = 1/3
    a.les_k = p.smagorinsky_cs > 0.0 ? 18.0 * p.smagorinsky_cs * p.smagorinsky_cs : 0.0;
    a.sigma = p.sigma;
    a.p_volume = p.p_volume;
    a.eps_phi = p.eps_phi;
    int32_t *lists[5];
    for (int k = 0; k < 5; ++k) lists[k] = at<int32_t>(c, c->L.lists[k]);
    a.list_newg = lists[0];
    a.list_froml = lists[1];
    a.list_conv = lists[2 + parity];
    a.list_conv_prev = lists[2 + (1 - parity)];
    a.list_recv = lists[4];
    SList sl[4];
    for (int k = 0; k < 4; ++k) {
        sl[k].data = c->L.sl_data[k] ? at<int32_t>(c, c->L.sl_data[k]) : nullptr;
        sl[k].cnt = c->L.sl_cnt[k] ? at<int32_t>(c, c->L.sl_cnt[k]) : nullptr;
        sl[k].S = c->L.sl_S;
        sl[k].seg = c->L.sl_seg;
        sl[k].ovf = c->L.sl_ovf;
    }
    a.list_if = sl[parity];
    a.list_if_prev = sl[1 - parity];
    a.list_mark = sl[2];
    a.list_band = sl[3];
    a.claim = at<uint8_t>(c, c->L.claim);
    a.tiles = at<int32_t>(c, c->L.tiles);
    a.tile_bits = at<uint32_t>(c, c->L.tile_bits);
    a.bulk_grid = c->bulk_grid;
    a.cnt = at<int32_t>(c, c->L.cnt);
    a.nif_dom = at<int32_t>(c, c->L.nif);
    a.res = at<double>(c, c->L.res);
    a.parity = parity;
    a.B = p.batch;
    a.cap = a.g.BN;
    return a;
}

fslbm_status fail(fslbm_ctx *c, fslbm_status s, const std::string &msg) {
    if (c->status == FSLBM_OK) {
        c->status = s;
        c->err = msg;
    }
    return c->status;
}

bool hip_ok(fslbm_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    fail(c, FSLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

// Check the sticky device error word (requires a synchronised stream).
bool device_errors_ok(fslbm_ctx *c) {
    int32_t cnt[C_COUNT];
    if (!hip_ok(c, hipMemcpy(cnt, at<int32_t>(c, c->L.cnt), sizeof cnt, hipMemcpyDeviceToHost),
                "hipMemcpy(counters)"))
        return false;
    int e = cnt[C_ERR];
    if (e & E_LIST_OVERFLOW) { fail(c, FSLBM_EDEVICE, "internal list overflow"); return false; }
    if (e & E_BAD_FLAG) { fail(c, FSLBM_EINVAL, "flags must be 1 (liquid), 2 (interface) or 4 (gas)"); return false; }
    if (e & E_BAD_PHI) { fail(c, FSLBM_EINVAL, "liquid cells need phi = 1 and gas cells phi = 0 (finite)"); return false; }
    if (e & E_OPEN_LAYER) { fail(c, FSLBM_EINVAL, "a liquid cell has a gas neighbour (open interface layer)"); return false; }
    return true;
}

void drop_graphs(fslbm_ctx *c) {
    for (int k = 0; k < 8; ++k)
        if (c->exec[k]) { (void)hipGraphExecDestroy(c->exec[k]); c->exec[k] = nullptr; }
}

// The step graphs hold the step without its own excess-mass redistribution;
// variant pending = 1 runs the last step's inside the bulk kernel.
bool capture(fslbm_ctx *c, int parity, int pending) {
    if (!c->cap_stream &&
        !hip_ok(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate"))
        return false;
    hipGraph_t g = nullptr;
    if (!hip_ok(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal),
                "hipStreamBeginCapture"))
        return false;
    const StepArgs prev = make_args(c, 1 - parity);
    launch_step(make_args(c, parity), c->p.storage, c->p.collision, c->p.refill, c->cap_stream, nullptr,
                pending ? &prev : nullptr, false);
    hipError_t le = hipGetLastError();
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (!hip_ok(c, le, "kernel launch (capture)") || !hip_ok(c, e, "hipStreamEndCapture")) return false;
    hipError_t ie = hipGraphInstantiate(&c->exec[parity + 2 * pending], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return hip_ok(c, ie, "hipGraphInstantiate");
}

// The bubble model's end of the step before (its labels and pressures), run
// between a step's bulk kernel, which finishes that step's excess work, and its
// interface kernel, the first to read the pressures.
struct BubbleEnd {
    fslbm_ctx *c;
    int parity;   // of the step whose bulk kernel precedes
};
void bubble_end_hook(void *arg, hipStream_t s) {
    const BubbleEnd *h = static_cast<const BubbleEnd *>(arg);
    (void)bubble_end(h->c, s, h->parity);
}

// A bubble-model step that finishes the step before inside its bulk kernel and
// then runs that step's bubble kernels, as graph v.
bool capture_bubble_step(fslbm_ctx *c, int parity, int v) {
    if (!c->cap_stream &&
        !hip_ok(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate"))
        return false;
    hipGraph_t g = nullptr;
    if (!hip_ok(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal),
                "hipStreamBeginCapture"))
        return false;
    const StepArgs prev = make_args(c, 1 - parity);
    BubbleEnd h{c, parity};
    const StepHook hook{bubble_end_hook, &h};
    launch_step(make_args(c, parity), c->p.storage, c->p.collision, c->p.refill, c->cap_stream, nullptr, &prev,
                false, &hook);
    hipError_t le = hipGetLastError();
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (c->status != FSLBM_OK || !hip_ok(c, le, "kernel launch (capture)") ||
        !hip_ok(c, e, "hipStreamEndCapture"))
        return false;
    hipError_t ie = hipGraphInstantiate(&c->exec[v], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return hip_ok(c, ie, "hipGraphInstantiate");
}

// One step with the bubble model.  A step left pending has its excess work run
// inside this step's bulk kernel and its bubble labels and pressures between
// this step's bulk and interface kernels (graph replay when enabled); its end
// labels then become this step's start labels.  finish: this step's own excess
// work and bubble kernels run at its end.
bool enqueue_bubble_step(fslbm_ctx *c, bool finish) {
    const int parity = int(c->t & 1);
    const StepArgs a = make_args(c, parity);
    if (!c->pending) {
        // the step's start labels: the last step's end labels, or labelled now
        if (!bubble_begin(c)) return false;
        launch_step(a, c->p.storage, c->p.collision, c->p.refill, c->stream, nullptr, nullptr, false);
    } else if (c->graphs) {
        const int v = 4 + parity + 2 * (c->L.blab0 < c->L.blab1 ? 0 : 1);
        if (!c->exec[v] && !capture_bubble_step(c, parity, v)) return false;
        if (!hip_ok(c, hipGraphLaunch(c->exec[v], c->stream), "hipGraphLaunch")) return false;
    } else {
        const StepArgs prev = make_args(c, 1 - parity);
        BubbleEnd h{c, parity};
        const StepHook hook{bubble_end_hook, &h};
        launch_step(a, c->p.storage, c->p.collision, c->p.refill, c->stream, nullptr, &prev, false, &hook);
    }
    if (!hip_ok(c, hipGetLastError(), "step kernel launch") || c->status != FSLBM_OK) return false;
    if (c->pending) {
        c->bub_ready = true;
        if (!bubble_begin(c)) return false;   // the last step's end labels become the start labels
    }
    if (finish) {
        launch_excess(a, c->p.storage, c->stream);
        if (!hip_ok(c, hipGetLastError(), "k_excess") || !bubble_end(c, c->stream, 1 - parity)) return false;
    }
    c->pending = !finish;
    ++c->t;
    return true;
}

bool enqueue_step(fslbm_ctx *c, bool finish) {
    const int parity = int(c->t & 1);
    // with surface tension the surface kernels open the next step and read
    // the redistribution's results: every step finishes
    finish = finish || c->p.sigma != 0.0;
    const int pend = c->pending ? 1 : 0;
    const StepArgs a = make_args(c, parity);
    if (c->graphs) {
        const int v = parity + 2 * pend;
        if (!c->exec[v] && !capture(c, parity, pend)) return false;
        if (!hip_ok(c, hipGraphLaunch(c->exec[v], c->stream), "hipGraphLaunch")) return false;
        if (finish) launch_excess(a, c->p.storage, c->stream);
    } else {
        const StepArgs prev = make_args(c, 1 - parity);
        launch_step(a, c->p.storage, c->p.collision, c->p.refill, c->stream, nullptr, pend ? &prev : nullptr,
                    finish);
    }
    if (!hip_ok(c, hipGetLastError(), "step kernel launch")) return false;
    c->pending = !finish;
    ++c->t;
    return true;
}

bool load_state(fslbm_ctx *c, const uint8_t *flags, const double *phi, const double *rho,
                const double *u, const double *pdf, const double *mass, const double *reservoir) {
    c->t = 0;
    c->pending = false;
    StepArgs a = make_args(c, 0);
    const int B = c->p.batch;
    const size_t sb = storage_bytes(c->p.storage);
    bool ok = hip_ok(c, hipMemsetAsync(a.cnt, 0, C_COUNT * 4, c->stream), "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.nif_dom, 0, size_t(2 * B) * ND_SHARDS * 32 * 4, c->stream),
                     "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.res, 0, 16 * B, c->stream), "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.mex, 0, size_t(a.g.BN) * 8, c->stream), "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.fo, 0, size_t(a.g.BN) * 18 * sb, c->stream), "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.tile_bits, 0, size_t(tile_count(a.g.BN) + 31) / 32 * 4, c->stream),
                     "hipMemset") &&
              hip_ok(c, hipMemsetAsync(a.claim, 0, size_t(a.g.BN) + 4, c->stream), "hipMemset");
    for (int k = 0; ok && k < 4; ++k)
        if (c->L.sl_cnt[k])
            ok = hip_ok(c, hipMemsetAsync(at<int32_t>(c, c->L.sl_cnt[k]), 0, size_t(c->L.sl_S + 1) * 32 * 4,
                                          c->stream), "hipMemset");
    if (ok && a.band)
        ok = hip_ok(c, hipMemsetAsync(a.band, 0, size_t((a.g.BN + 31) / 32) * 4, c->stream), "hipMemset") &&
             hip_ok(c, hipMemsetAsync(a.rhoG, 0, size_t(a.g.BN) * 8, c->stream), "hipMemset") &&
             hip_ok(c, hipMemsetAsync(a.normal, 0, size_t(a.g.BN) * 24, c->stream), "hipMemset");
    // also clear the PDF array so gas slots hold finite values
    ok = ok && hip_ok(c, hipMemsetAsync(a.pdf, 0, size_t(a.g.BN) * Q * sb, c->stream), "hipMemset(pdf)");
    // the reservoir carried into the next step sits in the slot of parity 0
    if (ok && reservoir)
        ok = hip_ok(c, hipMemcpyAsync(a.res, reservoir, 8 * B, hipMemcpyDeviceToDevice, c->stream),
                    "hipMemcpy(reservoir)");
    if (!ok) return false;
    InitArgs ia{a, flags, phi, rho, u, pdf, mass};
    const unsigned nblk = unsigned((a.g.BN + 255) / 256);
    switch (c->p.storage) {
        case FSLBM_F64: hipLaunchKernelGGL(k_init_cells<ST_F64>, dim3(nblk), dim3(256), 0, c->stream, ia); break;
        case FSLBM_F32: hipLaunchKernelGGL(k_init_cells<ST_F32>, dim3(nblk), dim3(256), 0, c->stream, ia); break;
        case FSLBM_F16: hipLaunchKernelGGL(k_init_cells<ST_F16>, dim3(nblk), dim3(256), 0, c->stream, ia); break;
        default: hipLaunchKernelGGL(k_init_cells<ST_BF16>, dim3(nblk), dim3(256), 0, c->stream, ia); break;
    }
    if (!hip_ok(c, hipGetLastError(), "k_init_cells")) return false;
    hipLaunchKernelGGL(k_init_lists, dim3(nblk), dim3(256), 0, c->stream, a);
    if (!hip_ok(c, hipGetLastError(), "k_init_lists")) return false;
    hipLaunchKernelGGL(k_init_tiles, dim3(nblk), dim3(256), 0, c->stream, a);
    if (!hip_ok(c, hipGetLastError(), "k_init_tiles")) return false;
    hipLaunchKernelGGL(k_tile_list, dim3(1), dim3(1024), 0, c->stream, a);
    if (!hip_ok(c, hipGetLastError(), "k_tile_list")) return false;
    return !c->p.bubble_model || bubble_reset(c);
}

bool refresh_bulk_grid(fslbm_ctx *c) {
    int32_t n = 0;
    if (!hip_ok(c, hipMemcpy(&n, at<int32_t>(c, c->L.cnt) + C_TILES, 4, hipMemcpyDeviceToHost),
                "hipMemcpy(tile count)"))
        return false;
    return resize_bulk_grid(c, n);
}

bool resize_bulk_grid(fslbm_ctx *c, int32_t n) {
    // one wavefront per tile, four per workgroup, room for the list to double
    const long long total = tile_count((long long)c->p.nx * c->p.ny * c->p.nz * c->p.batch);
    const long long waves = std::min<long long>(total, std::max<long long>(4096, 2LL * n));
    const long long want = (waves + 3) / 4;
    if (want > c->bulk_grid) {
        c->bulk_grid = int(want);
        drop_graphs(c);
    }
    return true;
}

// The stability check of fslbm_params.diag_every after a step: the
// diagnostics, when the step count since the load is a multiple of the period.
fslbm_status check_stability(fslbm_ctx *c) {
    const int K = c->p.diag_every;
    if (K <= 0 || c->t % K != 0) return FSLBM_OK;
    std::vector<fslbm_diag> d(size_t(c->p.batch));
    const fslbm_status st = run_diagnostics(c, d.data());
    if (st == FSLBM_EUNSTABLE && c->status == FSLBM_OK) {
        const double cs = 1.0 / std::sqrt(3.0);
        for (int b = 0; b < c->p.batch; ++b)
            if (!d[b].finite || !(d[b].max_speed <= cs)) {
                c->err = "stability check after step " + std::to_string(c->t) + ": domain " + std::to_string(b) +
                         (d[b].finite ? " has |u| = " + std::to_string(d[b].max_speed) + " > c_s"
                                      : " holds non-finite values");
                break;
            }
    }
    return st;
}

bool enqueue_read(fslbm_ctx *c, uint32_t mask, void *const *dst) {
    if (!mask) return true;
    ReadArgs r{};
    r.s = make_args(c, int(c->t & 1));
    r.layoutB = int(c->t & 1);
    r.mask = mask;
    r.flags = static_cast<uint8_t *>(dst[0]);
    r.pdf = static_cast<double *>(dst[1]);
    r.mass = static_cast<double *>(dst[2]);
    r.phi = static_cast<double *>(dst[3]);
    r.rho = static_cast<double *>(dst[4]);
    r.vel = static_cast<double *>(dst[5]);
    const unsigned nblk = unsigned((r.s.g.BN + 255) / 256);
    switch (c->p.storage) {
        case FSLBM_F64: hipLaunchKernelGGL(k_read<ST_F64>, dim3(nblk), dim3(256), 0, c->stream, r); break;
        case FSLBM_F32: hipLaunchKernelGGL(k_read<ST_F32>, dim3(nblk), dim3(256), 0, c->stream, r); break;
        case FSLBM_F16: hipLaunchKernelGGL(k_read<ST_F16>, dim3(nblk), dim3(256), 0, c->stream, r); break;
        default: hipLaunchKernelGGL(k_read<ST_BF16>, dim3(nblk), dim3(256), 0, c->stream, r); break;
    }
    return hip_ok(c, hipGetLastError(), "k_read");
}

}  // namespace fslbm

// ------------------------------------------------------------------ C ABI

extern "C" {

fslbm_status fslbm_workspace_bytes(const fslbm_params *params, size_t *bytes) {
    const char *why = validate(params);
    if (why || !bytes) { g_init_error = why ? why : "bytes is NULL"; return FSLBM_EINVAL; }
    Layout L;
    make_layout(*params, L);
    *bytes = L.total;
    return FSLBM_OK;
}

fslbm_status fslbm_init(const fslbm_params *params, void *workspace, size_t bytes,
                        const uint8_t *flags, const double *phi, const double *rho,
                        const double *u, const double *pdf, const double *mass,
                        fslbm_ctx **out) {
    if (out) *out = nullptr;
    const char *why = validate(params);
    if (!why && !out) why = "out is NULL";
    if (!why && (!workspace || !flags || !phi)) why = "workspace, flags and phi are required";
    if (!why && !pdf && (!rho || !u)) why = "rho and u are required when pdf is NULL";
    if (!why && (reinterpret_cast<uintptr_t>(workspace) & 255)) why = "workspace must be 256-byte aligned";
    if (why) { g_init_error = why; return FSLBM_EINVAL; }
    fslbm_ctx *c = new (std::nothrow) fslbm_ctx;
    if (!c) { g_init_error = "host allocation failed"; return FSLBM_ENOMEM; }
    c->p = *params;
    c->p.omega_b = nullptr;
    c->p.gravity_b = nullptr;
    make_layout(c->p, c->L);
    if (bytes < c->L.total) {
        g_init_error = "workspace too small";
        delete c;
        return FSLBM_ENOMEM;
    }
    c->ws = static_cast<char *>(workspace);
    c->stream = static_cast<hipStream_t>(params->stream);
    const int B = params->batch;
    c->omega_h.resize(2 * B);
    c->grav_h.resize(3 * B);
    for (int b = 0; b < B; ++b) {
        c->omega_h[b] = params->omega_b ? params->omega_b[b] : params->omega;
        // TRT: (1/omega+ - 1/2)(1/omega- - 1/2) = Lambda
        c->omega_h[B + b] = 1.0 / (0.5 + params->trt_lambda / (1.0 / c->omega_h[b] - 0.5));
        for (int k = 0; k < 3; ++k)
            c->grav_h[3 * b + k] = params->gravity_b ? params->gravity_b[3 * b + k] : params->gravity[k];
    }
    bool ok = hip_ok(c, hipMemcpyAsync(at<double>(c, c->L.omega), c->omega_h.data(), 16 * B,
                                       hipMemcpyHostToDevice, c->stream), "hipMemcpy(omega)") &&
              hip_ok(c, hipMemcpyAsync(at<double>(c, c->L.grav), c->grav_h.data(), 24 * B,
                                       hipMemcpyHostToDevice, c->stream), "hipMemcpy(gravity)");
    ok = ok && load_state(c, flags, phi, rho, u, pdf, mass, nullptr);
    ok = ok && hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize") && device_errors_ok(c) &&
         refresh_bulk_grid(c);
    if (!ok) {
        g_init_error = c->err;
        fslbm_status s = c->status;
        fslbm_destroy(c);
        return s;
    }
    *out = c;
    return FSLBM_OK;
}

fslbm_status fslbm_init_static(const fslbm_params *params, const uint8_t *flags, const double *phi,
                               const double *rho, const double *u, const double *pdf,
                               const double *mass, fslbm_ctx **out) {
    if (out) *out = nullptr;
    const char *why = validate(params);
    if (!why && !out) why = "out is NULL";
    if (why) { g_init_error = why; return FSLBM_EINVAL; }
    Layout L;
    make_layout(*params, L);
    if (L.total > STATIC_WS_BYTES) {
        g_init_error = "fslbm_init_static: these parameters need " + std::to_string(L.total) +
                       " bytes of workspace, more than the static workspace's " +
                       std::to_string(STATIC_WS_BYTES);
        return FSLBM_ENOMEM;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) {
        g_init_error = "fslbm_init_static: no current device (or a device index above 63)";
        return FSLBM_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot &slot = g_static[dev];
    if (!slot.ptr) {
        // once per device, with that device current
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_init_error = std::string("fslbm_init_static: hipGetSymbolAddress: ") + hipGetErrorString(e);
            return FSLBM_EDEVICE;
        }
        slot.ptr = ptr;
    }
    if (slot.owner) {
        g_init_error = "fslbm_init_static: another live context uses this device's static workspace "
                       "(fslbm_destroy it first)";
        return FSLBM_ESTATE;
    }
    // fslbm_init clears every part of the workspace that must start at zero,
    // so what the last context left in the array does not matter
    fslbm_ctx *c = nullptr;
    const fslbm_status st = fslbm_init(params, slot.ptr, STATIC_WS_BYTES, flags, phi, rho, u, pdf, mass, &c);
    if (st != FSLBM_OK) return st;
    c->static_dev = dev;
    slot.owner = c;
    *out = c;
    return FSLBM_OK;
}

fslbm_status fslbm_step(fslbm_ctx *c, int32_t nsteps) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (nsteps < 0) return fail(c, FSLBM_EINVAL, "nsteps must be >= 0");
    if (c->p.bubble_model) {
        // each step's excess work runs inside the next step's bulk kernel, and
        // its bubble labels and pressures right after it; the last step of the
        // call, a step that a stability check follows and every step with
        // surface tension (its curvature kernel reads the pressures before the
        // bulk kernel) finish their own
        const int K = c->p.diag_every;
        for (int32_t s = 0; s < nsteps; ++s) {
            const bool checked = K > 0 && (c->t + 1) % K == 0;
            if (!enqueue_bubble_step(c, s + 1 == nsteps || checked || c->p.sigma != 0.0)) return c->status;
            if (checked) {
                const fslbm_status st = check_stability(c);
                if (st != FSLBM_OK) return st;
            }
        }
        return FSLBM_OK;
    }
    // each step's excess-mass redistribution runs inside the next step's bulk
    // kernel; the last step finishes its own, and so does a step that a
    // stability check follows
    const int K = c->p.diag_every;
    for (int32_t s = 0; s < nsteps; ++s) {
        const bool checked = K > 0 && (c->t + 1) % K == 0;
        if (!enqueue_step(c, s + 1 == nsteps || checked)) return c->status;
        if (checked) {
            const fslbm_status st = check_stability(c);
            if (st != FSLBM_OK) return st;
        }
    }
    return FSLBM_OK;
}

fslbm_status fslbm_step_timed(fslbm_ctx *c, int32_t nsteps, double *bulk_ms, double *total_ms) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (nsteps < 1 || !bulk_ms || !total_ms) return fail(c, FSLBM_EINVAL, "nsteps >= 1 and outputs required");
    if (c->p.bubble_model) return fail(c, FSLBM_EINVAL, "fslbm_step_timed does not run the bubble model");
    std::vector<hipEvent_t> ev(size_t(2) * nsteps + 2, nullptr);
    bool ok = true;
    for (auto &e : ev)
        if (ok) ok = hip_ok(c, hipEventCreate(&e), "hipEventCreate");
    if (ok) ok = hip_ok(c, hipEventRecord(ev[2 * nsteps], c->stream), "hipEventRecord");
    for (int32_t s = 0; ok && s < nsteps; ++s) {
        // as fslbm_step: the bulk kernel also runs the last step's excess-mass
        // redistribution where that is fused
        BulkEvents be{ev[2 * s], ev[2 * s + 1]};
        const int parity = int(c->t & 1);
        const bool finish = s + 1 == nsteps || c->p.sigma != 0.0;
        const StepArgs prev = make_args(c, 1 - parity);
        launch_step(make_args(c, parity), c->p.storage, c->p.collision, c->p.refill, c->stream, &be,
                    c->pending ? &prev : nullptr, finish);
        ok = hip_ok(c, hipGetLastError(), "step kernel launch");
        if (ok) {
            c->pending = !finish;
            ++c->t;
        }
    }
    if (ok) ok = hip_ok(c, hipEventRecord(ev[2 * nsteps + 1], c->stream), "hipEventRecord") &&
                 hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    double bulk = 0.0, total = 0.0;
    for (int32_t s = 0; ok && s < nsteps; ++s) {
        float ms = 0.0f;
        ok = hip_ok(c, hipEventElapsedTime(&ms, ev[2 * s], ev[2 * s + 1]), "hipEventElapsedTime");
        bulk += ms;
    }
    if (ok) {
        float ms = 0.0f;
        ok = hip_ok(c, hipEventElapsedTime(&ms, ev[2 * nsteps], ev[2 * nsteps + 1]), "hipEventElapsedTime");
        total = ms;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (!ok) return c->status;
    *bulk_ms = bulk;
    *total_ms = total;
    return device_errors_ok(c) ? FSLBM_OK : c->status;
}

fslbm_status fslbm_refill_scheme(fslbm_ctx *c, int32_t scheme) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (scheme < FSLBM_REFILL_EQ || scheme > FSLBM_REFILL_AVG) return fail(c, FSLBM_EINVAL, "unknown refill scheme");
    if (scheme != c->p.refill) {
        c->p.refill = scheme;
        drop_graphs(c);
    }
    return FSLBM_OK;
}

fslbm_status fslbm_use_graphs(fslbm_ctx *c, int32_t enable) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    c->graphs = enable != 0;
    return FSLBM_OK;
}

fslbm_status fslbm_set_stream(fslbm_ctx *c, void *stream) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    c->stream = static_cast<hipStream_t>(stream);
    return FSLBM_OK;
}

fslbm_status fslbm_read_fields(fslbm_ctx *c, uint32_t mask, void *const *dst) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (mask & ~0x7Fu) return fail(c, FSLBM_EINVAL, "unknown field bits");
    if (!dst && mask) return fail(c, FSLBM_EINVAL, "dst is NULL");
    for (int k = 0; k < 7; ++k)
        if ((mask >> k & 1u) && !dst[k]) return fail(c, FSLBM_EINVAL, "NULL destination for a requested field");
    if ((mask & FSLBM_FIELD_BUBBLE_PRESSURE) && !c->p.bubble_model)
        return fail(c, FSLBM_EINVAL, "the bubble pressure needs bubble_model = 1");
    if (!enqueue_read(c, mask & 0x3Fu, dst)) return c->status;
    if ((mask & FSLBM_FIELD_BUBBLE_PRESSURE) &&
        !hip_ok(c, hipMemcpyAsync(dst[6], at<double>(c, c->L.pbub),
                                  size_t(c->p.nx) * c->p.ny * c->p.nz * c->p.batch * 8,
                                  hipMemcpyDeviceToDevice, c->stream), "hipMemcpy(bubble pressure)"))
        return c->status;
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize")) return c->status;
    if (!device_errors_ok(c) || !refresh_bulk_grid(c)) return c->status;
    return FSLBM_OK;
}

}  // extern "C"

namespace fslbm {

// Per-domain diagnostics into out[B] (synchronises): FSLBM_EUNSTABLE if some
// domain holds non-finite values or a speed above c_s, else OK (or the
// context's failure).
fslbm_status run_diagnostics(fslbm_ctx *c, fslbm_diag *out) {
    const int B = c->p.batch;
    StepArgs a = make_args(c, int(c->t & 1));
    double *pd = at<double>(c, c->L.diag_d);
    long long *pi = at<long long>(c, c->L.diag_i);
    switch (c->p.storage) {
        case FSLBM_F64: hipLaunchKernelGGL(k_diag_partial<ST_F64>, dim3(DIAG_BLOCKS, B), dim3(256), 0, c->stream, a, int(c->t & 1), pd, pi); break;
        case FSLBM_F32: hipLaunchKernelGGL(k_diag_partial<ST_F32>, dim3(DIAG_BLOCKS, B), dim3(256), 0, c->stream, a, int(c->t & 1), pd, pi); break;
        case FSLBM_F16: hipLaunchKernelGGL(k_diag_partial<ST_F16>, dim3(DIAG_BLOCKS, B), dim3(256), 0, c->stream, a, int(c->t & 1), pd, pi); break;
        default: hipLaunchKernelGGL(k_diag_partial<ST_BF16>, dim3(DIAG_BLOCKS, B), dim3(256), 0, c->stream, a, int(c->t & 1), pd, pi); break;
    }
    if (!hip_ok(c, hipGetLastError(), "k_diag_partial")) return c->status;
    std::vector<double> hd(size_t(B) * DIAG_BLOCKS * 2);
    std::vector<long long> hi(size_t(B) * DIAG_BLOCKS * 4);
    std::vector<double> res(2 * B);
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize") ||
        !hip_ok(c, hipMemcpy(hd.data(), pd, hd.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy") ||
        !hip_ok(c, hipMemcpy(hi.data(), pi, hi.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy") ||
        !hip_ok(c, hipMemcpy(res.data(), a.res, 16 * B, hipMemcpyDeviceToHost), "hipMemcpy"))
        return c->status;
    if (!device_errors_ok(c) || !refresh_bulk_grid(c)) return c->status;
    bool unstable = false;
    const double cs = 1.0 / std::sqrt(3.0);
    for (int b = 0; b < B; ++b) {
        fslbm_diag d{};
        double mass = 0.0, vmax = 0.0;
        long long cnt[4] = {0, 0, 0, 0};
        for (int k = 0; k < DIAG_BLOCKS; ++k) {
            size_t o = size_t(b) * DIAG_BLOCKS + k;
            mass += hd[2 * o];
            vmax = std::max(vmax, hd[2 * o + 1]);
            for (int j = 0; j < 4; ++j) cnt[j] += hi[4 * o + j];
        }
        // the reservoir carried into the next step (set at load, then by every step)
        const double r = res[size_t(c->t & 1) * B + b];
        d.reservoir = r;
        d.total_mass = mass + r;
        d.max_speed = vmax;
        d.n_liquid = cnt[0];
        d.n_interface = cnt[1];
        d.n_gas = cnt[2];
        d.finite = cnt[3] == 0;
        unstable |= !d.finite || !(vmax <= cs);
        out[b] = d;
    }
    return unstable ? FSLBM_EUNSTABLE : FSLBM_OK;
}

}  // namespace fslbm

extern "C" {

fslbm_status fslbm_diagnostics(fslbm_ctx *c, fslbm_diag *out) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (!out) return fail(c, FSLBM_EINVAL, "out is NULL");
    return run_diagnostics(c, out);
}

fslbm_status fslbm_last_step_stats(fslbm_ctx *c, fslbm_step_stats *out) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (!out) return fail(c, FSLBM_EINVAL, "out is NULL");
    int32_t cnt[C_COUNT];
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize") ||
        !hip_ok(c, hipMemcpy(cnt, at<int32_t>(c, c->L.cnt), sizeof cnt, hipMemcpyDeviceToHost),
                "hipMemcpy(counters)"))
        return c->status;
    *out = fslbm_step_stats{};
    if (c->t == 0) return FSLBM_OK;
    const int p = int((c->t - 1) & 1);   // parity of the last step
    std::vector<int32_t> nif(size_t(c->p.batch) * ND_SHARDS * 32);
    if (!hip_ok(c, hipMemcpy(nif.data(), at<int32_t>(c, c->L.nif) + size_t(p) * nif.size(),
                             4 * nif.size(), hipMemcpyDeviceToHost), "hipMemcpy(interface counts)"))
        return c->status;
    for (size_t k = 0; k < nif.size(); k += 32) out->interface_cells += nif[k];
    out->new_from_gas = cnt[C_NEWG];
    out->from_liquid = cnt[C_FROML];
    out->converted = cnt[C_CONV0 + p];
    return FSLBM_OK;
}

const char *fslbm_last_error(const fslbm_ctx *c) {
    return c ? c->err.c_str() : g_init_error.c_str();
}

void fslbm_destroy(fslbm_ctx *c) {
    if (!c) return;
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->static_dev >= 0) {
        // the next static context may use another stream: let this one's work end first
        (void)hipStreamSynchronize(c->stream);
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static[c->static_dev].owner == c) g_static[c->static_dev].owner = nullptr;
    }
    delete c;
}

}  // extern "C"
