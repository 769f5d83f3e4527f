// fslbm_kernels.hpp -- host-callable launchers of the step kernels.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// Optional events recorded on the stream right before and after the bulk
// stream-collide kernel of a step.
struct BulkEvents {
    hipEvent_t before, after;
};

// Work enqueued between a step's bulk kernel and its interface kernel: fn(arg, s).
struct StepHook {
    void (*fn)(void *arg, hipStream_t s);
    void *arg;
};

// Enqueue one FSLBM step with the given arguments.
//   pending:    the arguments of the last step if its excess-mass
//               redistribution has not run yet (it then runs inside this
//               step's bulk kernel), else null;
//   finish:     run this step's own excess-mass redistribution at its end;
//               otherwise the step is left pending for the next launch_step or
//               for launch_excess;
//   after_bulk: enqueued after the bulk kernel (so after a pending
//               redistribution), before the interface kernel.
// With surface tension a pending redistribution runs on its own first (the
// surface kernels read its results).
void launch_step(const StepArgs &a, int storage, int collision, int scheme, hipStream_t s,
                 const BulkEvents *ev = nullptr, const StepArgs *pending = nullptr,
                 bool finish = true, const StepHook *after_bulk = nullptr);

// Enqueue the excess-mass redistribution of a step left pending.
void launch_excess(const StepArgs &a, int storage, hipStream_t s);

// The same for one PDF storage type (one translation unit per type).
template <int ST>
void launch_step_storage(const StepArgs &a, int collision, int scheme, hipStream_t s,
                         const BulkEvents *ev, const StepArgs *pending, bool finish,
                         const StepHook *after_bulk);
template <int ST>
void launch_excess_storage(const StepArgs &a, hipStream_t s);

}  // namespace fslbm
