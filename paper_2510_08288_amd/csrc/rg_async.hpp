// Launches of the asynchronous RG step (rg_step_async): the kernels that move
// its inputs and outputs between caller device memory and the step's records.
#pragma once

#include "rg_internal.hpp"

namespace rg {

// Asynchronous RG step: x [n], r, v_prev and the step counter t from device
// memory into the state record; the result record's v, kappa and status out to
// device memory (kappa_out, status_out may be null) and t advanced by one.
hipError_t launch_async_in(const DevBuffers& b, const double* x, const double* r,
                           const double* v_prev, const uint32_t* t, int n, hipStream_t st);
hipError_t launch_async_out(const DevBuffers& b, double* v_out, double* kappa_out,
                            int32_t* status_out, uint32_t* t, hipStream_t st);

}  // namespace rg
