// Kernels of the asynchronous RG step (rg_step_async).  The step itself is the
// launch sequence of a blocking step; these two kernels replace its host
// upload of (x_t, r_t, v_{t-1}, t) and its host read of the result record.
#include <hip/hip_runtime.h>

#include "rg_async.hpp"

namespace rg {

// Asynchronous RG step: the step's inputs from caller device memory into the
// state record (as the host upload of a blocking step writes it), and the
// result record out to caller device memory with the step counter advanced.
__global__ void __launch_bounds__(64) k_async_in(DevState* st, const double* __restrict__ x,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ v_prev,
                                                 const uint32_t* __restrict__ t, int n) {
  for (int i = threadIdx.x; i < kMaxN; i += blockDim.x) st->x[i] = i < n ? x[i] : 0.0;
  if (threadIdx.x == 0) {
    st->v_prev = *v_prev;
    st->r = *r;
    st->t = *t;
    st->cl_index = 0;
    st->cl_len = 0;
    st->gen_lo = 0;
    st->gen_hi = 0;
    st->gen_n = 0;
  }
}

__global__ void __launch_bounds__(64) k_async_out(const DevResult* __restrict__ res,
                                                  double* v_out, double* kappa_out,
                                                  int32_t* status_out, uint32_t* t) {
  if (threadIdx.x == 0) {
    const DevResult R = res[0];
    *v_out = R.v;
    if (kappa_out) *kappa_out = R.kappa;
    if (status_out) *status_out = R.status;
    *t = R.t + 1u;
  }
}

hipError_t launch_async_in(const DevBuffers& b, const double* x, const double* r,
                           const double* v_prev, const uint32_t* t, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_async_in, dim3(1), dim3(64), 0, st, b.st, x, r, v_prev, t, n);
  return hipGetLastError();
}

hipError_t launch_async_out(const DevBuffers& b, double* v_out, double* kappa_out,
                            int32_t* status_out, uint32_t* t, hipStream_t st) {
  hipLaunchKernelGGL(k_async_out, dim3(1), dim3(64), 0, st, b.res, v_out, kappa_out, status_out,
                     t);
  return hipGetLastError();
}

}  // namespace rg
