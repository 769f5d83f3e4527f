// fslbm_device.hpp -- device-side building blocks of the FSLBM step for gfx950:
// the D3Q19 lattice, PDF storage codecs, the in-place (AA) slot map, cell
// geometry and the per-launch argument block shared by all kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fslbm {

// ------------------------------------------------------------------ lattice
// D3Q19 (Sec. 2.1): rest, 6 faces, 12 edges; opposite directions adjacent.
constexpr int Q = 19;
// All direction loops are fully unrolled, so these fold to constants.
__host__ __device__ constexpr int cx(int i) {
    constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
template <typename T>
__host__ __device__ constexpr T wgt(int i) {
    return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

// ------------------------------------------------------------------ flag bits
// Low three bits are the canonical cell types.  The rest are internal:
//   NOFLUID / NOEMPTY  forced emptying / filling classes of interface cells
//   MARK_A  interface: fill level above 1+eps (to liquid); gas: new interface
//   MARK_B  interface: fill level below -eps (to gas); liquid: becomes interface
//   CONV    liquid or gas cell that was interface before this step's conversion
enum : uint8_t {
    F_LIQ = 1, F_IF = 2, F_GAS = 4, F_TYPE = 7,
    F_NOFLUID = 8, F_NOEMPTY = 16,
    F_MARK_A = 32, F_MARK_B = 64, F_CONV = 128
};

// ------------------------------------------------------------------ storage
// PDFs are kept as shifted populations d_i = s (f_i - w_i).
enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

template <int S> struct Codec;
// decode / encode convert one stored value; load / store do it through memory.
template <> struct Codec<ST_F64> {
    using T = double;      // arithmetic type
    using M = double;      // memory type
    __device__ static T decode(M m) { return m; }
    __device__ static M encode(T v) { return v; }
    __device__ static T load(const M *p) { return *p; }
    __device__ static void store(M *p, T v) { *p = v; }
};
template <> struct Codec<ST_F32> {
    using T = float;
    using M = float;
    __device__ static T decode(M m) { return m; }
    __device__ static M encode(T v) { return v; }
    __device__ static T load(const M *p) { return *p; }
    __device__ static void store(M *p, T v) { *p = v; }
};
template <> struct Codec<ST_F16> {
    using T = float;
    using M = _Float16;
    static constexpr float S = 1024.0f, IS = 1.0f / 1024.0f;  // exact powers of two
    __device__ static T decode(M m) { return float(m) * IS; }
    __device__ static M encode(T v) { return (_Float16)(v * S); }
    __device__ static T load(const M *p) { return decode(*p); }
    __device__ static void store(M *p, T v) { *p = encode(v); }
};
template <> struct Codec<ST_BF16> {
    using T = float;
    using M = uint16_t;
    __device__ static T decode(M m) { return __uint_as_float(uint32_t(m) << 16); }
    __device__ static M encode(T v) {
        // round to nearest even on the upper 16 bits (finite inputs)
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    __device__ static T load(const M *p) { return decode(*p); }
    __device__ static void store(M *p, T v) { *p = encode(v); }
};

// A value as it reads back after a store in storage type ST.
template <int ST>
__device__ __forceinline__ typename Codec<ST>::T codec_round(typename Codec<ST>::T v) {
    typename Codec<ST>::M m;
    Codec<ST>::store(&m, v);
    return Codec<ST>::load(&m);
}

// Keeps the loads issued above it from being moved below it (into the
// branches that use them), so that they are all in flight at once.  Emits no
// instruction and no wait.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// ------------------------------------------------------------------ geometry
// Unsigned division of n < 2^31 by an invariant d >= 1 with one 32x32->64
// multiply and a shift (Granlund & Montgomery): m = ceil(2^(31+l) / d) with
// l = ceil(log2 d); then n / d == (n * m) >> (31 + l) for every n < 2^31.
struct FastDiv {
    uint32_t d, m;
    int s;
    __host__ static FastDiv make(uint32_t d) {
        int l = 0;
        while ((1ull << l) < d) ++l;
        FastDiv f;
        f.d = d;
        f.m = uint32_t(((1ull << (31 + l)) + d - 1) / d);
        f.s = 31 + l;
        return f;
    }
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        return uint32_t((uint64_t(n) * m) >> s);
    }
};

struct Geom {
    int nx, ny, nz;
    int per[3];
    int slip;         // walls: 0 no-slip (bounce-back), 1 free-slip (specular)
    long long N;      // cells per domain
    long long BN;     // cells in all domains (< 2^31)
    FastDiv dx, dy, dN;
};

// Neighbour of cell (x,y,z) shifted by (ox,oy,oz) inside the same domain:
// returns the domain-local cell index or -1 for a wall.
__device__ __forceinline__ int nb_local(const Geom &g, int x, int y, int z, int ox, int oy, int oz) {
    x += ox; y += oy; z += oz;
    if (x < 0 || x >= g.nx) { if (!g.per[0]) return -1; x = x < 0 ? x + g.nx : x - g.nx; }
    if (y < 0 || y >= g.ny) { if (!g.per[1]) return -1; y = y < 0 ? y + g.ny : y - g.ny; }
    if (z < 0 || z >= g.nz) { if (!g.per[2]) return -1; z = z < 0 ? z + g.nz : z - g.nz; }
    return (z * g.ny + y) * g.nx + x;
}

struct Cell {
    int b, x, y, z;
    int n;        // domain-local index
};

// Where a population leaving cell (x,y,z) along (ox,oy,oz) goes next when
// that cell lies in a wall and the walls are free-slip (Sec. 2.1, specular
// reflection): the wall-crossing components are reversed and the population
// arrives in the cell shifted by the others.  Returns the domain-local cell;
// (rx,ry,rz) receives the arrival direction.  Only called for a move that hits
// a wall.
__device__ __forceinline__ int slip_target(const Geom &g, int x, int y, int z, int ox, int oy, int oz,
                                           int &rx, int &ry, int &rz) {
    auto axis = [](int p, int o, int n, int per, int &r) -> int {
        int q = p + o;
        r = o;
        if (q >= 0 && q < n) return q;
        if (per) return q < 0 ? q + n : q - n;
        r = -o;   // reflected: stays in this layer
        return p;
    };
    const int X = axis(x, ox, g.nx, g.per[0], rx);
    const int Y = axis(y, oy, g.ny, g.per[1], ry);
    const int Z = axis(z, oz, g.nz, g.per[2], rz);
    return (Z * g.ny + Y) * g.nx + X;
}

__device__ __forceinline__ Cell decode(const Geom &g, long long gid) {
    Cell c;
    uint32_t u = uint32_t(gid);
    uint32_t b = g.dN.div(u);
    uint32_t n = u - b * uint32_t(g.N);
    uint32_t r = g.dx.div(n);
    uint32_t z = g.dy.div(r);
    c.b = int(b);
    c.n = int(n);
    c.x = int(n - r * uint32_t(g.nx));
    c.y = int(r - z * uint32_t(g.ny));
    c.z = int(z);
    return c;
}

// Global index of the neighbour along c_i, or -1 for a wall.
__device__ __forceinline__ long long nb_dir(const Geom &g, const Cell &c, int i) {
    int k = nb_local(g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
    return k < 0 ? -1 : (long long)c.b * g.N + k;
}

// ------------------------------------------------------------------ AA slots
// In-place streaming (AA pattern, Bailey et al. 2009).  After an even number of
// steps ("layout A") f*_i(x) sits in slot (opp(i), x).  After an odd number
// ("layout B") it sits in slot (i, x + c_i), or, when x + c_i is a wall, in
// (opp(i), x) with no-slip walls and in (j, m) with free-slip walls, m and j
// being the cell and direction of its specular reflection (slip_target).
// Slot (d, n) of domain b is pdf[(b*19 + d)*N + n].

// The lattice again as tables, for the few places that index a direction with
// a runtime value (one lane per direction).
__device__ __constant__ const int8_t k_cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ __constant__ const int8_t k_cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ __constant__ const int8_t k_cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Direction index of lattice velocity (x, y, z) (a D3Q19 velocity).
__device__ __forceinline__ int dir_index(int x, int y, int z) {
    int k = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) k = (cx(i) == x && cy(i) == y && cz(i) == z) ? i : k;
    return k;
}

// Flat index of the slot holding f*_i of cell c in the given layout (after
// an odd number of steps a population that went into a free-slip wall sits
// in its reflected arrival slot), for a runtime direction i.
// SLIP: 1 free-slip walls, 0 no-slip walls, -1 as the geometry says (the
// kernels that run every step fix it at compile time).
template <int SLIP = -1>
__device__ __forceinline__ long long slot_flat_rt(const Geom &g, int layoutB, const Cell &c, int i) {
    const long long base = (long long)c.b * Q * g.N;
    if (layoutB && i > 0) {
        int k = nb_local(g, c.x, c.y, c.z, k_cx[i], k_cy[i], k_cz[i]);
        if (k >= 0) return base + (long long)i * g.N + k;
        if (SLIP == 1 || (SLIP < 0 && g.slip)) {
            int rx, ry, rz;
            const int m = slip_target(g, c.x, c.y, c.z, k_cx[i], k_cy[i], k_cz[i], rx, ry, rz);
            return base + (long long)dir_index(rx, ry, rz) * g.N + m;
        }
    }
    const int o = i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
    return base + (long long)o * g.N + c.n;
}

// Flat index of the slot holding f*_i of cell c in the given layout.
template <int SLIP = -1>
__device__ __forceinline__ long long slot_flat(const Geom &g, int layoutB, const Cell &c, int i) {
    const long long base = (long long)c.b * Q * g.N;
    if (layoutB) {
        int k = nb_local(g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        if (k >= 0) return base + (long long)i * g.N + k;
        if (i > 0 && (SLIP == 1 || (SLIP < 0 && g.slip))) {
            int rx, ry, rz;
            const int m = slip_target(g, c.x, c.y, c.z, cx(i), cy(i), cz(i), rx, ry, rz);
            return base + (long long)dir_index(rx, ry, rz) * g.N + m;
        }
    }
    return base + (long long)opp(i) * g.N + c.n;
}

// ------------------------------------------------------------------ lists
// Append-only int32 list whose length is split over S counters, one 128-byte
// line each.  On MI355X atomics on a single address serialise (about 11 ns
// each), so thousands of wavefronts appending to one counter would take
// hundreds of microseconds; here wavefront w appends to slot w mod S, which
// owns a segment of `seg` entries.  Entries that do not fit their segment go
// to a shared overflow region, so the list holds S * seg + ovf entries in any
// distribution.  Slot s's length is cnt[32 s] (clamped to seg when read); the
// overflow length is cnt[32 S].
struct SList {
    int32_t *data;     // [S * seg + ovf]
    int32_t *cnt;      // [(S + 1) * 32]
    int32_t S, seg, ovf;
};

// Interface cells per domain, split over ND_SHARDS counters per domain (one
// 128-byte line each): [2 parities][B][ND_SHARDS][32].
constexpr int ND_SHARDS = 64;

// ------------------------------------------------------------------ arguments
struct StepArgs {
    Geom g;
    void *pdf;
    void *fo;              // [BN][18] (storage type) outgoing populations f*_i, i = 1..18,
                           // of every interface cell at the end of the last step
    uint8_t *flags;
    double *m;             // [BN] interface mass
    double *phi_cur;       // [BN] fill level at the start of this step
    double *phi_next;      // [BN] fill level at the end of this step (the other buffer)
    double *rhoG;          // [BN] gas density at interface cells (sigma != 0), else null
    const double *pbub;    // [BN] bubble pressure of every gas and interface cell (bubble
                           // model), else null: the volume pressure p_volume everywhere
    double *mex;           // [BN] excess mass share of converted cells
    double *rho_if;        // [BN] density after this step, sum_i f*_i as stored, of every
                           // interface cell after the conversions (set by its update,
                           // refill or conversion from liquid; read by the excess step)
    double *normal;        // [3][BN] unit normals on the band (sigma != 0)
    uint32_t *band;        // [ceil(BN/32)] band membership bits (sigma != 0)
    const double *omega;   // [B]
    const double *omega_m; // [B] TRT omega- (from omega+ and trt_lambda)
    const double *grav;    // [B][3]
    double trt_lambda;
    double les_k;          // Smagorinsky: 2 C_S^2 / c_s^4 (0 = no turbulence model)
    double sigma, p_volume, eps_phi;
    SList list_if;          // interface cells of this step, built by the bulk kernel by tile groups
    SList list_if_prev;     // the same list of the last step
    SList list_mark;        // interface cells marked for filling or emptying this step
    SList list_band;        // surface band (sigma != 0)
    int32_t *list_newg, *list_froml, *list_conv, *list_conv_prev;
    int32_t *list_recv;     // interface cells that receive excess mass this step
    uint8_t *claim;         // [BN] receiver claim bytes, zero between steps
    int32_t *tiles;        // tiles (TILE consecutive cells) that ever held fluid
    uint32_t *tile_bits;   // membership bits of that list
    int bulk_grid;         // workgroups of the bulk kernel (its wavefronts stride over the tiles)
    int pdf_off32;         // 1 if one domain's populations take less than 4 GiB (32-bit byte offsets)
    int32_t *cnt;          // device counters, see Counter
    int32_t *nif_dom;      // sharded interface cells per domain (see ND_SHARDS): counted by
                           // the interface kernel, then corrected by the step's conversions
    double *res;           // [2][B] reservoir of excess mass
    int parity;            // step parity: 0 = layout A -> B, 1 = layout B -> A
    int B;
    long long cap;         // capacity of every list
};

// Counter slots in StepArgs::cnt.  Index by parity where noted.
enum Counter {
    C_NEWG = 2, C_FROML = 3,     // this step's conversion lists
    C_CONV0 = 4, C_CONV1 = 5,    // converted interface cells (by step parity)
    C_ERR = 7,                   // sticky device error bits
    C_TILES = 8,                 // length of the tile list
    C_RECV = 10,                 // excess-mass receivers
    C_COUNT = 11
};
enum DeviceError { E_LIST_OVERFLOW = 1, E_OPEN_LAYER = 2, E_BAD_FLAG = 4, E_BAD_PHI = 8 };

// Append `v` to list[*count] with one atomic per wavefront.
__device__ __forceinline__ void wave_append(bool pred, int32_t v, int32_t *list, int32_t *count,
                                            long long cap, int32_t *err) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        unsigned long long below = mask & ((1ull << lane) - 1ull);
        long long pos = (long long)base + __popcll(below);
        if (pos < cap) list[pos] = v;
        else atomicOr(err, E_LIST_OVERFLOW);
    }
}

// ------------------------------------------------------------------ sharded lists

// Zero the counters of a sharded list (all threads of one workgroup).
__device__ __forceinline__ void slist_reset(const SList &L) {
    for (int t = threadIdx.x; t <= L.S; t += blockDim.x) L.cnt[32 * t] = 0;
}

// Append the entries val(i) of every lane whose bit i is set in sel (i < NI),
// one reservation per wavefront.  The slot is the wavefront's global index
// modulo S, or key modulo S for a key >= 0 (the same on all lanes), which sets
// where in the list's order the entries land.  Must be called by all lanes of
// the wavefront that are active in the enclosing loop.
template <int NI, typename V>
__device__ __forceinline__ void slist_append_sel(const SList &L, uint32_t sel, V val, int32_t *err, int key = -1) {
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
    const int slot = key >= 0 ? int(unsigned(key) % unsigned(L.S))
                              : int(((blockIdx.x * blockDim.x + threadIdx.x) >> 6) % unsigned(L.S));
    int base = 0, obase = 0;
    if (lane == leader) {
        base = atomicAdd(L.cnt + 32 * slot, tot);
        const int spill = base + tot - (base > L.seg ? base : L.seg);
        if (spill > 0) obase = atomicAdd(L.cnt + 32 * L.S, spill);
    }
    base = __shfl(base, leader);
    obase = __shfl(obase, leader);
    const int first_spill = base > L.seg ? base : L.seg;   // first position past the segment
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        if ((sel >> i) & 1u) {
            const int pos = base + pre[i] + __popcll(masks[i] & below);
            if (pos < L.seg) {
                L.data[(long long)slot * L.seg + pos] = val(i);
            } else {
                const int o = obase + (pos - first_spill);
                if (o < L.ovf) L.data[(long long)L.S * L.seg + o] = val(i);
                else atomicOr(err, E_LIST_OVERFLOW);
            }
        }
    }
}

__device__ __forceinline__ void slist_append(const SList &L, bool pred, int32_t v, int32_t *err, int key = -1) {
    slist_append_sel<1>(L, pred ? 1u : 0u, [&](int) { return v; }, err, key);
}

// Read side: prefix sums of the clamped slot lengths in shared memory (every
// thread of the workgroup calls slist_view; blockDim.x == 256 >= S).
struct SView {
    const int32_t *data;
    const int32_t *pref;   // [S + 1] in shared memory
    int32_t S, seg;
    long long nseg, total;
};

__device__ __forceinline__ SView slist_view(const SList &L, int32_t *pref) {
    __shared__ int32_t wave_total[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // both counter loads in flight together
    int v = 0;
    if (t < L.S) v = L.cnt[32 * t];
    int o = L.cnt[32 * L.S];
    v = v < L.seg ? v : L.seg;
    // inclusive scan: within each wavefront by shuffles, then across the
    // four wavefronts through shared memory
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_total[wv] = x;
    __syncthreads();
    for (int k = 0; k < wv; ++k) x += wave_total[k];
    pref[t + 1] = x;
    if (t == 0) pref[0] = 0;
    __syncthreads();
    SView w;
    w.data = L.data;
    w.pref = pref;
    w.S = L.S;
    w.seg = L.seg;
    w.nseg = pref[L.S];
    o = o < L.ovf ? o : L.ovf;
    w.total = w.nseg + o;
    return w;
}

// Entry k < total of the list.
__device__ __forceinline__ int32_t sview_at(const SView &w, long long k) {
    if (k >= w.nseg) return w.data[(long long)w.S * w.seg + (k - w.nseg)];
    int lo = 0, hi = w.S;   // pref[lo] <= k < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w.pref[mid] <= k) lo = mid;
        else hi = mid;
    }
    return w.data[(long long)lo * w.seg + (k - w.pref[lo])];
}

// Sharded per-domain interface counts.
__device__ __forceinline__ int32_t *nif_slot(int32_t *nif, int p, int B, int b, int shard) {
    return nif + (((long long)p * B + b) * ND_SHARDS + shard) * 32;
}
__device__ __forceinline__ int32_t nif_sum(const int32_t *nif, int p, int B, int b) {
    int32_t s = 0;
    for (int k = 0; k < ND_SHARDS; ++k) s += nif[(((long long)p * B + b) * ND_SHARDS + k) * 32];
    return s;
}

// Slot of direction i (1..18) in the outgoing-population copy of interface
// cell gid.  A cell's 18 values are contiguous, so an interface cell costs one
// or two cache lines wherever the interface cells of a wavefront lie.
__host__ __device__ inline long long fo_index(long long gid, int i) { return gid * 18 + (i - 1); }

// Cells per tile of the bulk kernel's work list: one wavefront's worth of
// consecutive cells (x fastest), so a wavefront never loads a row it has no
// fluid in.
constexpr int TILE = 64;
constexpr int TILE_SHIFT = 6;
__host__ __device__ inline long long tile_count(long long BN) { return (BN + TILE - 1) / TILE; }

// Add tile t to the fluid-tile list unless it is there already.
__device__ __forceinline__ void activate_tile(int32_t *tiles, uint32_t *bits, int32_t *count, int32_t t,
                                              int32_t ntiles) {
    const uint32_t bit = 1u << (t & 31);
    if (atomicOr(bits + (t >> 5), bit) & bit) return;
    const int32_t pos = atomicAdd(count, 1);
    if (pos < ntiles) tiles[pos] = t;
}

// Byte-granular atomic OR on a byte array whose base is 4-byte aligned (the
// workspace arrays are 256-byte aligned) and padded to whole words.  Returns
// the previous byte value.  The word is addressed by pointer arithmetic on
// the array itself, so the compiler keeps the global address space (global,
// not flat, atomics: several can be in flight at once).
__device__ __forceinline__ uint8_t flag_or(uint8_t *flags, long long i, uint8_t bits) {
    unsigned int *w = reinterpret_cast<unsigned int *>(flags + (i & ~3LL));
    const int sh = int(i & 3) * 8;
    const unsigned int old = atomicOr(w, (unsigned int)bits << sh);
    return uint8_t(old >> sh);
}
// Byte-granular atomic clear of `bits` (same layout rules).
__device__ __forceinline__ void flag_clear(uint8_t *flags, long long i, uint8_t bits) {
    unsigned int *w = reinterpret_cast<unsigned int *>(flags + (i & ~3LL));
    const int sh = int(i & 3) * 8;
    atomicAnd(w, ~((unsigned int)bits << sh));
}

}  // namespace fslbm
