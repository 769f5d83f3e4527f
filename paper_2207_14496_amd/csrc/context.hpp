// context.hpp -- the host-side library context shared by the C-ABI translation
// units (forward step in api.hip, reverse mode in adjoint_api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fslbm.h"
#include "fslbm_kernels.hpp"

namespace fslbm {

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    size_t pdf, fo, flags, m, phi, mex, rho_if, rhoG, normal, band;
    size_t lists[5];   // newg, froml, conv0, conv1, recv
    size_t sl_data[4], sl_cnt[4];   // sharded lists: interface (even / odd step), marks, band
    int32_t sl_S, sl_seg, sl_ovf;
    size_t claim;
    size_t cnt, nif, res, omega, grav, diag_d, diag_i;
    size_t tiles, tile_bits;
    // bubble model: per-cell pressure (the state), labels at the step's start
    // and end, per-label sums
    size_t pbub, blab0, blab1, bV0, bV1, bkept, bamount, batm;
    size_t total;
};

// Bookkeeping of the last fslbm_adjoint_forward (what the backward sweep needs).
struct AdjointRun {
    bool valid = false;
    const void *ws = nullptr;      // adjoint workspace it used
    int T = 0, K = 0, S = 0, x_probe = 0;
    const double *target = nullptr;
};

}  // namespace fslbm

struct fslbm_ctx {
    fslbm_params p{};
    fslbm::Layout L{};
    char *ws = nullptr;
    std::vector<double> omega_h, grav_h;
    long long t = 0;                 // steps done since the state was loaded
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    bool graphs = true;
    // [parity + 2 * pending]; with the bubble model [4 + parity + 2 * (label buffers swapped)]
    hipGraphExec_t exec[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool pending = false;            // the last step's excess-mass redistribution has not run yet
    int bulk_grid = 1024;            // workgroups of the bulk kernel (tile-list stride)
    bool bub_ready = false;          // the bubble labels and volumes of the last step's end
                                     // are those of the next step's start
    fslbm::AdjointRun adj;
    int static_dev = -1;             // device whose static workspace backs this context
                                     // (fslbm_init_static), else -1
    fslbm_status status = FSLBM_OK;
    std::string err = "no error";
};

namespace fslbm {

template <typename T>
T *at(fslbm_ctx *c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }

// Kernel arguments of a step with the given parity.
StepArgs make_args(fslbm_ctx *c, int parity);

// Record the first error (sticky) and return the context status.
fslbm_status fail(fslbm_ctx *c, fslbm_status s, const std::string &msg);
bool hip_ok(fslbm_ctx *c, hipError_t e, const char *what);
// Check the device error word (the stream must be synchronised).
bool device_errors_ok(fslbm_ctx *c);

// Enqueue a FSLBM step on the context's stream (graph replay or direct).
// finish = false lets the step end with its excess-mass redistribution
// pending (without surface tension it then runs inside the next step's bulk
// kernel); every API call that returns to the caller ends with none pending.
bool enqueue_step(fslbm_ctx *c, bool finish = true);

// Load a canonical state (device arrays, layouts of fslbm_init) into the
// context and restart its step count at 0.  reservoir: device [B] or null (0).
// Enqueued on the context's stream; validation errors surface at the next
// device_errors_ok.
bool load_state(fslbm_ctx *c, const uint8_t *flags, const double *phi, const double *rho,
                const double *u, const double *pdf, const double *mass, const double *reservoir);

// Grow the bulk kernel's grid to twice the fluid-tile count (capped by the
// tile total) if the list has outgrown it.  Needs a synchronised stream; drops
// the captured graphs when the grid changes.
bool refresh_bulk_grid(fslbm_ctx *c);
// The same from a fluid-tile count the caller has read back.
bool resize_bulk_grid(fslbm_ctx *c, int32_t fluid_tiles);

// Per-domain diagnostics into out[B] (synchronises); FSLBM_EUNSTABLE if some
// domain holds non-finite values or a speed above c_s.
fslbm_status run_diagnostics(fslbm_ctx *c, fslbm_diag *out);

// Enqueue the canonical read-back of the fields in `mask` (no synchronisation).
bool enqueue_read(fslbm_ctx *c, uint32_t mask, void *const *dst);

// Bubble model (bubble_model = 1): the bubbles and their volumes at the start
// of a step, and their pressures at its end (launches only, no waits).
bool bubble_begin(fslbm_ctx *c);
bool bubble_end(fslbm_ctx *c, hipStream_t st, int parity);
// Every gas and interface cell at p_volume (after a state is loaded).
bool bubble_reset(fslbm_ctx *c);

}  // namespace fslbm
