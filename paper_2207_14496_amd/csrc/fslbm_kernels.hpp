// fslbm_kernels.hpp -- host-callable launchers of the step kernels.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// Optional events recorded on the stream right before and after the bulk
// stream-collide kernel of a step.
struct BulkEvents {
    hipEvent_t before, after;
};

// Enqueue one full FSLBM step (all sub-steps) with the given arguments.
void launch_step(const StepArgs &a, int storage, int collision, int scheme, hipStream_t s,
                 const BulkEvents *ev = nullptr);

// The same for one PDF storage type (one translation unit per type).
template <int ST>
void launch_step_storage(const StepArgs &a, int collision, int scheme, hipStream_t s,
                         const BulkEvents *ev);

}  // namespace fslbm
