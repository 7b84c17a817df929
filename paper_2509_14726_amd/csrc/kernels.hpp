// Launch entry points of the device code (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace mppi {

// Convert the problem tables of a context to the device layout.
hipError_t launch_setup(const KArgs &a, bool fp64, hipStream_t st);

// Enqueue one MPPI step: sample (with the head), rollout, average (+ tail).
// acc64 selects binary64 accumulation of the weighted average.
// When ev is non-null, ev[0..3] are recorded before the sample, rollout and
// average kernels and after the average kernel.
hipError_t launch_solve(const KArgs &a, bool fp64, bool acc64, hipStream_t st, hipEvent_t *ev = nullptr);

// Device address of the fixed solve workspace (kScratchBytes, 256-byte
// aligned) on the current device.  The first call on a device resolves it
// (with that device current) and later calls return the cached address.
hipError_t scratch_address(void **ptr);

// Launch shape of one batch group.
struct BatchLaunch {
    int objective;
    bool fp64, acc64;
    int rollout_waves;    // 1..4 (see mppi_batch_cfg)
    int ring4_b;          // four-wave chunk (binary32): 4, one workgroup per CU; 2, two
    int rollout_groups;   // persistent rollout workgroups
    int sample_groups;    // grid-stride workgroups of the sample kernel
    int final_groups;     // grid-stride workgroups of the weighted-average kernel
    int ctrl_groups;      // grid-stride workgroups of the control-cost kernel (0: no item has the term)
};

// Enqueue one batched MPPI step over the items described in device memory.
hipError_t launch_batch(const BArgs &b, const BatchLaunch &L, hipStream_t st);

}  // namespace mppi
