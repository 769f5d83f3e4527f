// adjoint.hpp -- argument block and launchers of the reverse-mode FSLBM step.
//
// Every adjoint kernel runs on a 2-D grid: blockIdx.y is the domain, blockIdx.x
// covers that domain's cells in groups of 256, so no workgroup spans two
// domains and per-domain parameter gradients reduce without atomics.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// One canonical state record (what the forward stores per saved time level).
struct AdjState {
    const uint8_t *fl;     // [B][N] cell types (1 liquid, 2 interface, 4 gas)
    const double *f;       // [B][19][N] post-collision PDFs (0 in gas)
    const double *m;       // [B][N] interface mass
    const double *phi;     // [B][N] fill level
    const double *R;       // [B] reservoir plus unreceived excess of the step that made this state
    const int32_t *nif;    // [B] interface cells after that step
};

struct AdjArgs {
    Geom g;
    int B;
    int nblk;              // workgroups per domain (ceil(N / 256))
    AdjState s0, s1;       // states at t and t+1
    const double *omega;   // [B]
    const double *grav;    // [B][3]
    double rhoG;           // gas density 3 p_V (no surface tension)
    // adjoints of the state at t+1: f and m are updated in place
    double *lf1, *lm1;
    const double *lphi1, *lres1;
    // adjoints of the state at t (outputs)
    double *lf0, *lm0, *lphi0, *lres0;
    // per-step scratch
    double *lua;           // [BN][3] anti-bounce-back velocity adjoint of interface cells next to gas
    double *lmt;           // [BN] adjoint of the mass after the exchange, m'
    double *lphis;         // [BN] adjoint of the fill level after streaming, phi'
    uint8_t *cls;          // [BN] forced filling/emptying class at t
    int32_t *iflist;       // [BN] the interface cells at t (k_adj_classes)
    int32_t *ifcnt;        // [3] list length by the parity of t + 1; [2] unused error slot
    double *sum_lm;        // [B] sum of interface-mass adjoints (reservoir spreading)
    double *gpart;         // [B][nblk][4] running (omega, gx, gy, gz) gradient partials
    // loss L_b = (1/T) sum_{t=1..T} (h_b(t) - h*_b(t))^2, h = sum of phi over x = x_probe
    const double *h;       // [B][T+1]
    const double *target;  // [B][T]
    const double *dloss;   // [B] incoming adjoint of L_b
    int x_probe, t1, T;
};

void launch_adjoint_step(const AdjArgs &a, hipStream_t s);

// h[b * stride + t] = sum over the plane x = x_probe of phi (one workgroup per
// domain, fixed summation order).
void launch_height(const Geom &g, int B, const double *phi, int x_probe, double *h, long long stride,
                   int t, hipStream_t s);

// out[b][k] = sum over blocks of gpart[b][blk][k] (fixed order).
void launch_reduce_params(const double *gpart, int B, int nblk, double *out, hipStream_t s);

// Copy the per-domain scalars of the engine after a step into a state record:
// R = res[p_last], nif = the interface count of that step (sharded counters),
// reservoir = res[p_cur]; with no step done yet (p_last < 0) R and nif are zero.
void launch_save_scalars(const double *res, const int32_t *nif_dom, int B, int p_last, int p_cur,
                         double *R, int32_t *nif, double *reservoir, hipStream_t s);

}  // namespace fslbm
