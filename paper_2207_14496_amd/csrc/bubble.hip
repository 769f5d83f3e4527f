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
// smallest cell index.  They come from a union-find over parent pointers that
// only ever fall and always name a cell of the same set.  A seed pass points
// every cell at its smallest neighbour of the set; two propagation passes
// lower each pointer to the smallest label around the cell, then to that
// label's own label, which shortens the trees; a merge pass joins the two
// trees of every link (the lock-free linking by atomic minimum of Playne and
// Hawick, IEEE TPDS 2018, with path halving); a last pass takes each cell's
// root, the smallest index of its tree, and adds its gas volume to it.  A
// fixed number of launches, whatever the sets' shapes, and no host
// synchronisation.  Per-label sums are double atomics.  The model runs
// between the steps (fslbm_step), for the runs with enclosed gas; a step whose
// start labels are the last step's end labels replays the step and these
// launches as one HIP graph.
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

// Parent pointers: every gas or interface cell points at the smallest index
// among itself and its gas or interface D3Q19 neighbours, liquid -1.  The
// per-label sums of this labelling are cleared where they can be read: V,
// amount and atm (indexed by this labelling) on its gas and interface cells,
// kept (indexed by the start labels lab0) on the cells lab0 labels.
__global__ __launch_bounds__(BS) void k_bub_seed(StepArgs a, int32_t *lab, const int32_t *lab0, double *V,
                                                 double *kept, double *amount, int32_t *atm) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    if (gid >= a.g.BN) return;
    if (kept && lab0[gid] >= 0) kept[gid] = 0.0;
    if (!gas_phase(a.flags[gid])) {
        lab[gid] = -1;
        return;
    }
    const Cell c = decode(a.g, gid);
    const long long cb = (long long)c.b * a.g.N;
    uint8_t fq[Q];
    int q[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        q[i] = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        fq[i] = a.flags[cb + (q[i] >= 0 ? q[i] : c.n)];
    }
    int32_t m = int32_t(gid);
#pragma unroll
    for (int i = 1; i < Q; ++i)
        if (q[i] >= 0 && gas_phase(fq[i]) && int32_t(cb + q[i]) < m) m = int32_t(cb + q[i]);
    lab[gid] = m;
    if (V) V[gid] = 0.0;
    if (amount) amount[gid] = 0.0;
    if (atm) atm[gid] = 0;
}

// Root of x's tree.  Parents are read past the per-CU cache: an older value
// is only a larger parent of the same set, so it delays nothing but a retry.
__device__ __forceinline__ int32_t uf_root(int32_t *lab, int32_t x) {
    int32_t p = __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != x) {
        const int32_t gp = __hip_atomic_load(lab + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp == p) return p;
        // path halving: x now points at its grandparent, an ancestor of the same set
        atomicMin(lab + x, gp);
        x = gp;
        p = __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return x;
}

// Join the trees of x and y: the larger root is pointed at the smaller one by
// an atomic minimum.  If that root had meanwhile been given a parent (old), it
// now points at the smaller root instead, and the join continues with old, so
// that old's tree is joined as well.  The larger of the two roots falls with
// every retry, so the loop ends.
__device__ __forceinline__ void uf_join(int32_t *lab, int32_t x, int32_t y) {
    for (;;) {
        x = uf_root(lab, x);
        y = uf_root(lab, y);
        if (x == y) return;
        if (x > y) {
            const int32_t t = x;
            x = y;
            y = t;
        }
        const int32_t old = atomicMin(lab + y, x);
        if (old == y) return;
        y = old;
    }
}

// Propagation: the smallest label among the cell's and its gas or interface
// neighbours', then the label of the cell that label names.  Labels only fall
// and only name cells of the same set, so a neighbour's label read before or
// after its own update is valid either way.
__device__ __forceinline__ void bub_prop_cell(const StepArgs &a, int32_t *lab, const long long gid,
                                              const Cell &c, const long long cb) {
    const int32_t l0 = lab[gid];
    int32_t m = l0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int q = nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i));
        const int32_t lq = q >= 0 ? lab[cb + q] : -1;
        m = (lq >= 0 && lq < m) ? lq : m;
    }
    const int32_t mm = lab[m];
    m = (mm >= 0 && mm < m) ? mm : m;
    if (m < l0) lab[gid] = m;
}

// After the seed, for every gas or interface cell: NPROP propagation rounds
// (each pass one launch: a merge must not run beside a propagation round,
// whose plain store could undo the merge's link), or with MERGE the merge of
// the two trees of every link (from the cell whose direction index is the
// lower of the pair).  Two propagation rounds in one launch time the same as
// two launches; three cost 1.7%.
template <int NPROP, bool MERGE>
__global__ __launch_bounds__(BS) void k_bub_link(StepArgs a, int32_t *lab) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    if (gid >= a.g.BN || lab[gid] < 0) return;
    const Cell c = decode(a.g, gid);
    const long long cb = (long long)c.b * a.g.N;
#pragma unroll
    for (int r = 0; r < NPROP; ++r) bub_prop_cell(a, lab, gid, c, cb);
    if (!MERGE) return;
    int32_t lq[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int q = i < opp(i) ? nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i)) : -1;
        lq[i] = q >= 0 ? lab[cb + q] : -1;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i)
        if (i < opp(i) && lq[i] >= 0)
            uf_join(lab, int32_t(gid), int32_t(cb + nb_local(a.g, c.x, c.y, c.z, cx(i), cy(i), cz(i))));
}

// Each cell's label (its root) into lab1, its gas volume added to its label's
// V; with atm, the labels that reach the top layer; with lab0, the gas volume
// of every start bubble's cells that are still gas or interface.
__global__ __launch_bounds__(BS) void k_bub_volume(StepArgs a, int32_t *lab1, const double *phi, double *V,
                                                   int32_t *atm, const int32_t *lab0, double *kept) {
    const long long gid = (long long)blockIdx.x * BS + threadIdx.x;
    int32_t l = gid < a.g.BN ? lab1[gid] : -1;
    if (l >= 0) {
        l = uf_root(lab1, int32_t(gid));
        lab1[gid] = l;
    }
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

// Label the gas and interface sets of the current flags into lab (roots and
// volumes: k_bub_volume), clearing the sums V, amount, atm and, with lab0,
// kept (each BN entries, or null).
bool label(fslbm_ctx *c, hipStream_t st, const StepArgs &a, int32_t *lab, const int32_t *lab0, double *V,
           double *kept, double *amount, int32_t *atm) {
    hipLaunchKernelGGL(k_bub_seed, dim3(blocks(a)), dim3(BS), 0, st, a, lab, lab0, V, kept, amount, atm);
    hipLaunchKernelGGL((k_bub_link<1, false>), dim3(blocks(a)), dim3(BS), 0, st, a, lab);
    hipLaunchKernelGGL((k_bub_link<1, false>), dim3(blocks(a)), dim3(BS), 0, st, a, lab);
    hipLaunchKernelGGL((k_bub_link<0, true>), dim3(blocks(a)), dim3(BS), 0, st, a, lab);
    return hip_ok(c, hipGetLastError(), "bubble labels");
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
    if (!label(c, c->stream, a, lab0, nullptr, V0, nullptr, nullptr, nullptr)) return false;
    hipLaunchKernelGGL(k_bub_volume, dim3(blocks(a)), dim3(BS), 0, c->stream, a, lab0, a.phi_cur, V0,
                       static_cast<int32_t *>(nullptr), static_cast<const int32_t *>(nullptr),
                       static_cast<double *>(nullptr));
    return hip_ok(c, hipGetLastError(), "k_bub_volume");
}

bool bubble_end(fslbm_ctx *c, hipStream_t st, int parity) {
    // after the step: phi_cur of the next step's arguments (parity: the next
    // step's) is the step's result
    const StepArgs a = make_args(c, parity);
    int32_t *lab0 = at<int32_t>(c, c->L.blab0), *lab1 = at<int32_t>(c, c->L.blab1);
    int32_t *atm = at<int32_t>(c, c->L.batm);
    double *V0 = at<double>(c, c->L.bV0), *V1 = at<double>(c, c->L.bV1);
    double *kept = at<double>(c, c->L.bkept), *amount = at<double>(c, c->L.bamount);
    double *pbub = at<double>(c, c->L.pbub);
    if (!label(c, st, a, lab1, lab0, V1, kept, amount, atm)) return false;
    const unsigned nb = blocks(a);
    hipLaunchKernelGGL(k_bub_volume, dim3(nb), dim3(BS), 0, st, a, lab1, a.phi_cur, V1, atm,
                       static_cast<const int32_t *>(lab0), kept);
    hipLaunchKernelGGL(k_bub_amount, dim3(nb), dim3(BS), 0, st, a, lab0, lab1, a.phi_cur,
                       static_cast<const double *>(pbub), static_cast<const double *>(V0),
                       static_cast<const double *>(kept), amount);
    hipLaunchKernelGGL(k_bub_assign, dim3(nb), dim3(BS), 0, st, a, lab1, static_cast<const double *>(V1),
                       static_cast<const double *>(amount), static_cast<const int32_t *>(atm), pbub);
    if (!hip_ok(c, hipGetLastError(), "bubble kernels")) return false;
    c->bub_ready = true;
    return true;
}

bool bubble_reset(fslbm_ctx *c) {
    c->bub_ready = false;
    const StepArgs a = make_args(c, int(c->t & 1));
    hipLaunchKernelGGL(k_bub_reset, dim3(blocks(a)), dim3(BS), 0, c->stream, a, at<double>(c, c->L.pbub));
    return hip_ok(c, hipGetLastError(), "k_bub_reset");
}

}  // namespace fslbm
