// bubble.hip -- the bubble model (Sec. 2.2: the volume pressure of an
// enclosed gas volume, p_V(t) = p_V(0) V(0) / V(t), tracked through
// coalescence and segmentation).
//
// A bubble is a connected set of gas and interface cells over D3Q19 links; a
// cell holds the gas volume max(0, 1 - phi) and a bubble V, the sum over its
// cells.  A set that reaches the top layer (z = nz - 1) is the atmosphere and
// stays at p_volume.  Every other bubble carries the amount p V.  At the end
// of a step each bubble b of the step's start hands p_b V_b to the bubbles of
// the step's end, shared by the gas volume of b's cells that each of them
// holds, and p_k = n_k / V_k: a bubble without a topology change keeps p V
// (Boyle's law), a merge adds amounts, the parts of a split share one pressure.
//
// Labels are global cell indices: every set ends up labelled with its
// smallest cell index.  They come from passes of label propagation (each cell
// takes the smallest label around it, then the label of the cell its label
// names) until a pass changes nothing.  Every pass has its own change flag and
// returns at once when the pass before it changed nothing, so the host
// launches a batch of passes (as many as the last labelling took) and reads
// the flags once.  Per-label sums are double atomics.  The model runs with
// direct launches between the steps (fslbm_step), for the runs with enclosed gas.
#include <algorithm>
#include <utility>
#include <vector>

#include "context.hpp"

namespace fslbm {
namespace {

constexpr int BS = 256;

__device__ __forceinline__ bool gas_phase(uint8_t f) { return (f & (F_IF | F_GAS)) != 0; }
__device__ __forceinline__ double gas_volume(double phi) { return phi < 1.0 ? 1.0 - phi : 0.0; }

// Adds v of every lane whose label l >= 0 into dst[l].  Lanes that share a
// label (most of a wavefront: its cells are neighbours) are summed in
// registers first, so there is one atomic per label and wavefront: atomics on
// one address serialise, and a bubble's cells all add to one.  Every lane of
// the wavefront calls it.
__device__ __forceinline__ void wave_add_by_label(int32_t l, double v, double *dst) {
    unsigned long long todo = __ballot(l >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int32_t lk = __shfl(l, leader);
        const bool mine = l == lk;
        double sum = mine ? v : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (__lane_id() == leader) atomicAdd(dst + lk, sum);
        todo &= ~__ballot(mine);
    }
}

// Every gas and interface cell labelled with its own index, liquid -1; the
// passes' change flags and the per-label sums of this labelling cleared.
__global__ __launch_bounds__(BS) void k_bub_seed(StepArgs a, int32_t *lab, int32_t *flags, int nflags,
                                                 double *z0, double *z1, double *z2, int32_t *z3) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    for (long long i = gid; i < nflags; i += (long long)gridDim.x * BS) flags[i] = 0;
    if (gid >= a.g.BN) return;
    lab[gid] = gas_phase(a.flags[gid]) ? int32_t(gid) : -1;
    if (z0) z0[gid] = 0.0;
    if (z1) z1[gid] = 0.0;
    if (z2) z2[gid] = 0.0;
    if (z3) z3[gid] = 0;
}

// Propagation pass k.  Labels only ever name gas or interface cells of the
// same set and only fall, so the fixed point is each set's smallest index.
// A pass after one that changed nothing has nothing to do.
__global__ __launch_bounds__(BS) void k_bub_pass(StepArgs a, int32_t *lab, int32_t *flags, int k) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    if (gid >= a.g.BN || (k > 0 && flags[k - 1] == 0)) return;
    const int32_t l0 = lab[gid];
    if (l0 < 0) return;
    const Cell c = decode(a.g, gid);
    const long long cb = (long long)c.b * a.g.N;
    int32_t m = l0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int q = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        const int32_t lq = q >= 0 ? lab[cb + q] : -1;
        m = (lq >= 0 && lq < m) ? lq : m;
    }
    const int32_t mm = lab[m];   // the label of the cell m (a gas or interface cell)
    m = (mm >= 0 && mm < m) ? mm : m;
    if (m < l0) {
        lab[gid] = m;
        flags[k] = 1;
    }
}

// Gas volume per label of lab1; with atm, the labels that reach the top layer;
// with lab0, the gas volume of every start bubble's cells that are still gas
// or interface.
__global__ __launch_bounds__(BS) void k_bub_volume(StepArgs a, const int32_t *lab1, const double *phi,
                                                   double *V, int32_t *atm, const int32_t *lab0,
                                                   double *kept) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    const int32_t l = gid < a.g.BN ? lab1[gid] : -1;
    const double gv = l >= 0 ? gas_volume(phi[gid]) : 0.0;
    wave_add_by_label(l, gv, V);
    if (l >= 0 && atm && decode(a.g, gid).z == a.g.nz - 1) atm[l] = 1;
    if (lab0) {
        const int32_t b = l >= 0 ? lab0[gid] : -1;
        wave_add_by_label(b, gv, kept);
    }
}

// Each start bubble's amount p V, handed to the end bubbles by gas volume.
__global__ __launch_bounds__(BS) void k_bub_amount(StepArgs a, const int32_t *lab0, const int32_t *lab1,
                                                   const double *phi, const double *pbub, const double *V0,
                                                   const double *kept, double *amount) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    const int32_t b = gid < a.g.BN ? lab0[gid] : -1;
    int32_t k = gid < a.g.BN ? lab1[gid] : -1;
    double v = 0.0;
    if (b < 0 || k < 0 || !(kept[b >= 0 ? b : 0] > 0.0)) k = -1;
    else v = pbub[b] * V0[b] * gas_volume(phi[gid]) / kept[b];
    wave_add_by_label(k, v, amount);
}

// The pressures of the end bubbles (0 on liquid cells).
__global__ __launch_bounds__(BS) void k_bub_assign(StepArgs a, const int32_t *lab1, const double *V1,
                                                   const double *amount, const int32_t *atm, double *pbub) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    if (gid >= a.g.BN) return;
    const int32_t k = lab1[gid];
    double p = 0.0;
    if (k >= 0) p = (atm[k] || !(V1[k] > 0.0) || !(amount[k] > 0.0)) ? a.p_volume : amount[k] / V1[k];
    pbub[gid] = p;
}

__global__ __launch_bounds__(BS) void k_bub_reset(StepArgs a, double *pbub) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    if (gid >= a.g.BN) return;
    pbub[gid] = gas_phase(a.flags[gid]) ? a.p_volume : 0.0;
}

unsigned blocks(const StepArgs &a) { return unsigned((a.g.BN + BS - 1) / BS); }

// Label the gas and interface sets of the current flags into lab and clear
// the sums z0..z3 (each BN entries, or null).  With tiles, also read back the
// fluid-tile count in the same synchronisation and resize the bulk grid.
bool label(fslbm_ctx *c, const StepArgs &a, int32_t *lab, double *z0, double *z1, double *z2, int32_t *z3,
           bool tiles) {
    int32_t *flags = at<int32_t>(c, c->L.bflag);
    const int cap = int(bubble_pass_cap(c->p));
    hipLaunchKernelGGL(k_bub_seed, dim3(blocks(a)), dim3(BS), 0, c->stream, a, lab, flags, cap, z0, z1, z2, z3);
    if (!hip_ok(c, hipGetLastError(), "k_bub_seed")) return false;
    std::vector<int32_t> h;
    int done = 0, batch = std::max(2, c->bub_passes);
    while (done < cap) {
        const int n = std::min(batch, cap - done);
        for (int j = 0; j < n; ++j)
            hipLaunchKernelGGL(k_bub_pass, dim3(blocks(a)), dim3(BS), 0, c->stream, a, lab, flags, done + j);
        h.assign(size_t(n) + 1, 0);
        if (!hip_ok(c, hipGetLastError(), "k_bub_pass") ||
            !hip_ok(c, hipMemcpyAsync(h.data(), flags + done, size_t(n) * 4, hipMemcpyDeviceToHost, c->stream),
                    "hipMemcpy(bubble flags)") ||
            (tiles && !hip_ok(c, hipMemcpyAsync(&h[n], at<int32_t>(c, c->L.cnt) + C_TILES, 4,
                                                hipMemcpyDeviceToHost, c->stream), "hipMemcpy(tile count)")) ||
            !hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize"))
            return false;
        const int first_zero = int(std::find(h.begin(), h.begin() + n, 0) - h.begin());
        if (first_zero < n) {
            c->bub_passes = done + first_zero + 1;
            return !tiles || resize_bulk_grid(c, h[n]);
        }
        done += n;
        batch *= 2;
    }
    fail(c, FSLBM_EDEVICE, "bubble labels did not settle");
    return false;
}

}  // namespace

bool bubble_begin(fslbm_ctx *c) {
    if (c->bub_ready) {
        // the step's start is the last step's end: its labels and volumes
        std::swap(c->L.blab0, c->L.blab1);
        std::swap(c->L.bV0, c->L.bV1);
        c->bub_ready = false;
        return true;
    }
    const StepArgs a = make_args(c, int(c->t & 1));
    int32_t *lab0 = at<int32_t>(c, c->L.blab0);
    double *V0 = at<double>(c, c->L.bV0);
    if (!label(c, a, lab0, V0, nullptr, nullptr, nullptr, false)) return false;
    hipLaunchKernelGGL(k_bub_volume, dim3(blocks(a)), dim3(BS), 0, c->stream, a, lab0, a.phi_cur, V0,
                       static_cast<int32_t *>(nullptr), static_cast<const int32_t *>(nullptr),
                       static_cast<double *>(nullptr));
    return hip_ok(c, hipGetLastError(), "k_bub_volume");
}

bool bubble_end(fslbm_ctx *c) {
    // after the step: phi_cur of the next step's arguments is the step's result
    const StepArgs a = make_args(c, int(c->t & 1));
    int32_t *lab0 = at<int32_t>(c, c->L.blab0), *lab1 = at<int32_t>(c, c->L.blab1);
    int32_t *atm = at<int32_t>(c, c->L.batm);
    double *V0 = at<double>(c, c->L.bV0), *V1 = at<double>(c, c->L.bV1);
    double *kept = at<double>(c, c->L.bkept), *amount = at<double>(c, c->L.bamount);
    double *pbub = at<double>(c, c->L.pbub);
    // the refills may have opened tiles: the bulk grid is resized from the
    // tile count read with the labels
    if (!label(c, a, lab1, V1, kept, amount, atm, true)) return false;
    const unsigned nb = blocks(a);
    hipLaunchKernelGGL(k_bub_volume, dim3(nb), dim3(BS), 0, c->stream, a, lab1, a.phi_cur, V1, atm,
                       static_cast<const int32_t *>(lab0), kept);
    hipLaunchKernelGGL(k_bub_amount, dim3(nb), dim3(BS), 0, c->stream, a, lab0, lab1, a.phi_cur,
                       static_cast<const double *>(pbub), static_cast<const double *>(V0),
                       static_cast<const double *>(kept), amount);
    hipLaunchKernelGGL(k_bub_assign, dim3(nb), dim3(BS), 0, c->stream, a, lab1, static_cast<const double *>(V1),
                       static_cast<const double *>(amount), static_cast<const int32_t *>(atm), pbub);
    if (!hip_ok(c, hipGetLastError(), "bubble kernels")) return false;
    c->bub_ready = true;
    return true;
}

long long bubble_pass_cap(const fslbm_params &p) {
    // each pass lowers at least one label while any is not final; pointer
    // jumping makes the passes far fewer than a set's diameter
    return 8LL * (p.nx + p.ny + p.nz) + 1024;
}

bool bubble_reset(fslbm_ctx *c) {
    c->bub_ready = false;
    const StepArgs a = make_args(c, int(c->t & 1));
    hipLaunchKernelGGL(k_bub_reset, dim3(blocks(a)), dim3(BS), 0, c->stream, a, at<double>(c, c->L.pbub));
    return hip_ok(c, hipGetLastError(), "k_bub_reset");
}

}  // namespace fslbm
