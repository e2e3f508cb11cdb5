// Time bookkeeping shared by host and kernels: the time of a step is
// t_base + (ctr + step_add) * dt, where ctr is an optional device counter
// advanced inside captured graphs (nullptr for eager launches).
#pragma once
#include <hip/hip_runtime.h>

namespace dgw {
struct StepTime {
  const long long* ctr;   // device step counter or nullptr
  double t_base;          // time of step 0
  double dt;              // step size
  int step_add;           // steps added to the counter
  double t_off;           // offset inside the step (LSRK stage: c_i dt)
  __host__ __device__ double tn() const {
#if defined(__HIP_DEVICE_COMPILE__)
    const long long c = ctr ? *ctr : 0;
#else
    const long long c = 0;
#endif
    return t_base + (double)(c + step_add) * dt;
  }
};
}  // namespace dgw
