// adjoint_api.hip -- host side of the reverse mode: checkpointed forward run of
// a loss window, segment-wise recomputation and the reverse sweep, behind the
// fslbm_adjoint_* entry points of include/fslbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/fslbm.h"
#include "adjoint.hpp"
#include "context.hpp"

using namespace fslbm;

namespace {

// One canonical state record inside the adjoint workspace.
struct Record {
    uint8_t *fl;
    double *f, *m, *phi;
    double *R;          // [B] reservoir + unreceived excess of the step that made it
    int32_t *nif;       // [B] interface cells after that step
    double *res;        // [B] reservoir carried into the next step
};

struct AdjLayout {
    int T, K, S;          // window, checkpoints actually used, segment length
    int nblk;             // workgroups per domain
    size_t rec_bytes;
    size_t h, dloss, ck, seg, fin;
    size_t lf[2], lm[2], lphi[2], lres[2], lua, lmt, lphis, cls, iflist, ifcnt, sum_lm, gpart, gred;
    size_t total;
};

const char *check_config(const fslbm_ctx *c) {
    const fslbm_params &p = c->p;
    if (p.storage != FSLBM_F64) return "the adjoint needs FSLBM_F64 storage";
    if (p.collision != FSLBM_SRT) return "the adjoint needs SRT collision";
    if (p.sigma != 0.0) return "the adjoint needs sigma = 0";
    if (p.smagorinsky_cs != 0.0) return "the adjoint needs smagorinsky_cs = 0";
    if (p.free_slip != 0) return "the adjoint needs no-slip walls";
    if (p.bubble_model != 0) return "the adjoint needs the constant volume pressure (bubble_model = 0)";
    if (p.refill != FSLBM_REFILL_EQ) return "the adjoint needs EQ refilling";
    if (p.batch > 65535) return "the adjoint supports at most 65535 domains";
    return nullptr;
}

const char *check_spec(const fslbm_ctx *c, const fslbm_adjoint_spec *s) {
    if (!s) return "spec is NULL";
    if (s->nsteps < 1) return "spec.nsteps must be >= 1";
    if (s->n_checkpoints < 0) return "spec.n_checkpoints must be >= 0";
    if (s->x_probe < 0 || s->x_probe >= c->p.nx) return "spec.x_probe outside [0, nx)";
    if (!s->target) return "spec.target is NULL";
    return nullptr;
}

AdjLayout make_adj_layout(const fslbm_ctx *c, const fslbm_adjoint_spec &s) {
    AdjLayout L{};
    const size_t B = size_t(c->p.batch);
    const size_t N = size_t(c->p.nx) * c->p.ny * c->p.nz;
    const size_t BN = B * N;
    L.T = s.nsteps;
    int K = s.n_checkpoints > 0 ? s.n_checkpoints : int(std::ceil(std::sqrt(double(L.T))));
    K = std::max(1, std::min(K, L.T));
    L.S = (L.T + K - 1) / K;
    L.K = (L.T + L.S - 1) / L.S;
    L.nblk = int((N + 255) / 256);
    L.rec_bytes = align256(BN) + align256(BN * Q * 8) + 2 * align256(BN * 8) + 2 * align256(B * 8) +
                  align256(B * 4);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.h = take(B * size_t(L.T + 1) * 8);
    L.dloss = take(B * 8);
    L.ck = take(L.rec_bytes * size_t(L.K));
    L.seg = take(L.rec_bytes * size_t(L.S));
    L.fin = take(L.rec_bytes);
    for (int k = 0; k < 2; ++k) {
        L.lf[k] = take(BN * Q * 8);
        L.lm[k] = take(BN * 8);
        L.lphi[k] = take(BN * 8);
        L.lres[k] = take(B * 8);
    }
    L.lua = take(BN * 3 * 8);
    L.lmt = take(BN * 8);
    L.lphis = take(BN * 8);
    L.cls = take(BN);
    L.iflist = take(BN * 4);
    L.ifcnt = take(16);
    L.sum_lm = take(B * 8);
    L.gpart = take(B * size_t(L.nblk) * 4 * 8);
    L.gred = take(B * 4 * 8);
    L.total = off;
    return L;
}

Record record_at(const fslbm_ctx *c, char *base) {
    const size_t B = size_t(c->p.batch);
    const size_t BN = B * size_t(c->p.nx) * c->p.ny * c->p.nz;
    Record r;
    size_t o = 0;
    r.fl = reinterpret_cast<uint8_t *>(base + o); o += align256(BN);
    r.f = reinterpret_cast<double *>(base + o); o += align256(BN * Q * 8);
    r.m = reinterpret_cast<double *>(base + o); o += align256(BN * 8);
    r.phi = reinterpret_cast<double *>(base + o); o += align256(BN * 8);
    r.R = reinterpret_cast<double *>(base + o); o += align256(B * 8);
    r.res = reinterpret_cast<double *>(base + o); o += align256(B * 8);
    r.nif = reinterpret_cast<int32_t *>(base + o);
    return r;
}

// Write the engine's current canonical state (and its per-domain scalars).
bool save_record(fslbm_ctx *c, const Record &r) {
    void *dst[6] = {r.fl, r.f, r.m, r.phi, nullptr, nullptr};
    if (!enqueue_read(c, FSLBM_FIELD_FLAGS | FSLBM_FIELD_PDF | FSLBM_FIELD_MASS | FSLBM_FIELD_PHI, dst))
        return false;
    StepArgs a = make_args(c, int(c->t & 1));
    const int p_last = c->t > 0 ? int((c->t - 1) & 1) : -1;
    launch_save_scalars(a.res, a.nif_dom, c->p.batch, p_last, int(c->t & 1), r.R, r.nif, r.res, c->stream);
    return hip_ok(c, hipGetLastError(), "k_save_scalars");
}

bool load_record(fslbm_ctx *c, const Record &r) {
    return load_state(c, r.fl, r.phi, nullptr, nullptr, r.f, r.m, r.res);
}

bool height(fslbm_ctx *c, const AdjLayout &L, char *ws, int x_probe, int t) {
    StepArgs a = make_args(c, int(c->t & 1));
    launch_height(a.g, c->p.batch, a.phi_cur, x_probe, reinterpret_cast<double *>(ws + L.h), L.T + 1, t,
                  c->stream);
    return hip_ok(c, hipGetLastError(), "k_height");
}

AdjState state_of(const Record &r) {
    return AdjState{r.fl, r.f, r.m, r.phi, r.R, r.nif};
}

fslbm_status start(fslbm_ctx *c, const fslbm_adjoint_spec *spec, void *ws, size_t bytes, AdjLayout &L) {
    if (const char *why = check_config(c)) return fail(c, FSLBM_EINVAL, why);
    if (const char *why = check_spec(c, spec)) return fail(c, FSLBM_EINVAL, why);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(c, FSLBM_EINVAL, "adjoint workspace must be non-NULL and 256-byte aligned");
    L = make_adj_layout(c, *spec);
    if (bytes < L.total) return fail(c, FSLBM_ENOMEM, "adjoint workspace too small");
    return FSLBM_OK;
}

}  // namespace

extern "C" {

fslbm_status fslbm_adjoint_workspace_bytes(fslbm_ctx *c, const fslbm_adjoint_spec *spec,
                                           size_t *bytes) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (!bytes) return fail(c, FSLBM_EINVAL, "bytes is NULL");
    if (const char *why = check_config(c)) return fail(c, FSLBM_EINVAL, why);
    if (const char *why = check_spec(c, spec)) return fail(c, FSLBM_EINVAL, why);
    *bytes = make_adj_layout(c, *spec).total;
    return FSLBM_OK;
}

fslbm_status fslbm_adjoint_forward(fslbm_ctx *c, const fslbm_adjoint_spec *spec, void *workspace,
                                   size_t bytes, double *loss, double *height_out) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (!loss) return fail(c, FSLBM_EINVAL, "loss is NULL");
    AdjLayout L;
    if (start(c, spec, workspace, bytes, L) != FSLBM_OK) return c->status;
    c->adj = AdjointRun{};
    char *ws = static_cast<char *>(workspace);
    const int B = c->p.batch;
    for (int t = 0; t < L.T; ++t) {
        if (t % L.S == 0) {
            // checkpoint: write the state out and continue from what was written
            const Record r = record_at(c, ws + L.ck + L.rec_bytes * size_t(t / L.S));
            if (!save_record(c, r) || !load_record(c, r)) return c->status;
        }
        if (t == 0 && !height(c, L, ws, spec->x_probe, 0)) return c->status;
        if (!enqueue_step(c) || !height(c, L, ws, spec->x_probe, t + 1)) return c->status;
    }
    if (!save_record(c, record_at(c, ws + L.fin))) return c->status;
    std::vector<double> h(size_t(B) * (L.T + 1)), tg(size_t(B) * L.T);
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize") || !device_errors_ok(c) ||
        !hip_ok(c, hipMemcpy(h.data(), ws + L.h, h.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy(height)") ||
        !hip_ok(c, hipMemcpy(tg.data(), spec->target, tg.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy(target)"))
        return c->status;
    for (int b = 0; b < B; ++b) {
        double s = 0.0;
        for (int t = 1; t <= L.T; ++t) {
            const double d = h[size_t(b) * (L.T + 1) + t] - tg[size_t(b) * L.T + (t - 1)];
            s += d * d;
        }
        loss[b] = s / L.T;
    }
    if (height_out) std::copy(h.begin(), h.end(), height_out);
    c->adj.valid = true;
    c->adj.ws = workspace;
    c->adj.T = L.T;
    c->adj.K = L.K;
    c->adj.S = L.S;
    c->adj.x_probe = spec->x_probe;
    c->adj.target = spec->target;
    return FSLBM_OK;
}

fslbm_status fslbm_adjoint_backward(fslbm_ctx *c, const fslbm_adjoint_spec *spec, void *workspace,
                                    size_t bytes, const double *dloss, double *grad_omega,
                                    double *grad_gravity, double *grad_pdf0, double *grad_mass0,
                                    double *grad_phi0) {
    if (!c) return FSLBM_EINVAL;
    if (c->status != FSLBM_OK) return c->status;
    if (!grad_omega || !grad_gravity) return fail(c, FSLBM_EINVAL, "grad_omega and grad_gravity are required");
    AdjLayout L;
    if (start(c, spec, workspace, bytes, L) != FSLBM_OK) return c->status;
    const AdjointRun &run = c->adj;
    if (!run.valid || run.ws != workspace || run.T != L.T || run.K != L.K || run.x_probe != spec->x_probe ||
        run.target != spec->target)
        return fail(c, FSLBM_EINVAL, "no matching fslbm_adjoint_forward on this context and workspace");
    char *ws = static_cast<char *>(workspace);
    const int B = c->p.batch;
    const size_t BN = size_t(B) * c->p.nx * c->p.ny * c->p.nz;
    std::vector<double> dl(B, 1.0);
    if (dloss) std::copy(dloss, dloss + B, dl.begin());
    auto D = [&](size_t off) { return reinterpret_cast<double *>(ws + off); };
    bool ok = hip_ok(c, hipMemcpyAsync(D(L.dloss), dl.data(), 8 * B, hipMemcpyHostToDevice, c->stream),
                     "hipMemcpy(dloss)");
    // adjoint of the state at the end of the window: zero (the loss enters per step)
    int cur = 0;
    ok = ok && hip_ok(c, hipMemsetAsync(D(L.lf[0]), 0, BN * Q * 8, c->stream), "hipMemset") &&
         hip_ok(c, hipMemsetAsync(D(L.lm[0]), 0, BN * 8, c->stream), "hipMemset") &&
         hip_ok(c, hipMemsetAsync(D(L.lphi[0]), 0, BN * 8, c->stream), "hipMemset") &&
         hip_ok(c, hipMemsetAsync(D(L.lres[0]), 0, size_t(B) * 8, c->stream), "hipMemset") &&
         hip_ok(c, hipMemsetAsync(D(L.gpart), 0, size_t(B) * L.nblk * 4 * 8, c->stream), "hipMemset") &&
         hip_ok(c, hipMemsetAsync(ws + L.ifcnt, 0, 16, c->stream), "hipMemset");
    if (!ok) return c->status;

    StepArgs sa = make_args(c, 0);
    AdjArgs a{};
    a.g = sa.g;
    a.B = B;
    a.nblk = L.nblk;
    a.omega = sa.omega;
    a.grav = sa.grav;
    a.rhoG = 3.0 * c->p.p_volume;
    a.lua = D(L.lua);
    a.lmt = D(L.lmt);
    a.lphis = D(L.lphis);
    a.cls = reinterpret_cast<uint8_t *>(ws + L.cls);
    a.iflist = reinterpret_cast<int32_t *>(ws + L.iflist);
    a.ifcnt = reinterpret_cast<int32_t *>(ws + L.ifcnt);
    a.sum_lm = D(L.sum_lm);
    a.gpart = D(L.gpart);
    a.h = D(L.h);
    a.target = spec->target;
    a.dloss = D(L.dloss);
    a.x_probe = spec->x_probe;
    a.T = L.T;

    for (int k = L.K - 1; k >= 0; --k) {
        const int t0 = k * L.S, t1 = std::min(L.T, t0 + L.S);
        const Record ck = record_at(c, ws + L.ck + L.rec_bytes * size_t(k));
        // recompute the segment: slot j holds the state at t0 + 1 + j
        if (!load_record(c, ck)) return c->status;
        for (int s = t0; s < t1; ++s)
            if (!enqueue_step(c) || !save_record(c, record_at(c, ws + L.seg + L.rec_bytes * size_t(s - t0))))
                return c->status;
        for (int s = t1 - 1; s >= t0; --s) {
            a.s0 = state_of(s == t0 ? ck : record_at(c, ws + L.seg + L.rec_bytes * size_t(s - 1 - t0)));
            a.s1 = state_of(record_at(c, ws + L.seg + L.rec_bytes * size_t(s - t0)));
            a.lf1 = D(L.lf[cur]);
            a.lm1 = D(L.lm[cur]);
            a.lphi1 = D(L.lphi[cur]);
            a.lres1 = D(L.lres[cur]);
            a.lf0 = D(L.lf[1 - cur]);
            a.lm0 = D(L.lm[1 - cur]);
            a.lphi0 = D(L.lphi[1 - cur]);
            a.lres0 = D(L.lres[1 - cur]);
            a.t1 = s + 1;
            launch_adjoint_step(a, c->stream);
            if (!hip_ok(c, hipGetLastError(), "adjoint step")) return c->status;
            cur = 1 - cur;
        }
    }
    launch_reduce_params(D(L.gpart), B, L.nblk, D(L.gred), c->stream);
    if (!hip_ok(c, hipGetLastError(), "k_reduce_params")) return c->status;
    ok = (!grad_pdf0 || hip_ok(c, hipMemcpyAsync(grad_pdf0, D(L.lf[cur]), BN * Q * 8, hipMemcpyDeviceToDevice,
                                                 c->stream), "hipMemcpy(grad_pdf0)")) &&
         (!grad_mass0 || hip_ok(c, hipMemcpyAsync(grad_mass0, D(L.lm[cur]), BN * 8, hipMemcpyDeviceToDevice,
                                                  c->stream), "hipMemcpy(grad_mass0)")) &&
         (!grad_phi0 || hip_ok(c, hipMemcpyAsync(grad_phi0, D(L.lphi[cur]), BN * 8, hipMemcpyDeviceToDevice,
                                                 c->stream), "hipMemcpy(grad_phi0)"));
    if (!ok || !load_record(c, record_at(c, ws + L.fin))) return c->status;
    std::vector<double> g(size_t(B) * 4);
    if (!hip_ok(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize") || !device_errors_ok(c) ||
        !hip_ok(c, hipMemcpy(g.data(), D(L.gred), g.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy(grads)"))
        return c->status;
    for (int b = 0; b < B; ++b) {
        grad_omega[b] = g[4 * b];
        for (int d = 0; d < 3; ++d) grad_gravity[3 * b + d] = g[4 * b + 1 + d];
    }
    return FSLBM_OK;
}

}  // extern "C"
