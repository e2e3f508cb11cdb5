// Prescribed exterior state of boundary faces (DGW_BC_PRESCRIBED): a
// superposition of plane waves p = A cos(k.x - omega t + phi),
// v = p k / (|k| Z), evaluated once per operator launch at that launch's
// time into a compact per-face buffer that the operator kernel reads.  The
// operator applies the flux to the stage state (LSRK, operator apply: the
// data at the stage time) or to the time-integrated Taylor sum (ADER update:
// the data integrated over the step).
#include <hip/hip_runtime.h>

#include "dgw_exterior.hpp"

namespace dgw {

__global__ void __launch_bounds__(256) exterior_kernel(ExteriorParams q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q.nslots * q.nf) return;
  const int64_t slot = i / q.nf;
  const int t = (int)(i - slot * q.nf);
  const int d = q.dim;
  const int64_t face = q.faces[slot];
  // unit outward normal from the area vector a = w detJ J^-T n_ref
  const double* a = q.geo_face + face * (int64_t)((d + 2) * q.nf) + t;
  double nrm[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0}, aa = 0.0;
  for (int e = 0; e < d; ++e) {
    nrm[e] = a[e * q.nf];
    aa = fma(nrm[e], nrm[e], aa);
    x[e] = q.bx[(slot * d + e) * q.nf + t];
  }
  const double ia = 1.0 / sqrt(aa);
  for (int e = 0; e < d; ++e) nrm[e] *= ia;
  const double tn = q.time.tn() + (q.integral ? 0.0 : q.time.t_off);
  const double dt = q.time.dt;
  double pe = 0.0, vne = 0.0;
  for (int j = 0; j < q.n_waves; ++j) {
    const double* w = q.waves + 7 * j;
    double th = w[5], kk = 0.0, kn = 0.0;
    for (int e = 0; e < d; ++e) {
      th = fma(w[1 + e], x[e], th);
      kk = fma(w[1 + e], w[1 + e], kk);
      kn = fma(w[1 + e], nrm[e], kn);
    }
    const double om = w[4];
    double val;
    if (q.integral) {
      // int_{tn}^{tn+dt} cos(th - om s) ds = 2 cos(th - om (tn + dt/2)) sin(om dt / 2) / om
      const double fac = om == 0.0 ? dt : 2.0 * sin(0.5 * om * dt) / om;
      val = w[0] * fac * cos(th - om * (tn + 0.5 * dt));
    } else {
      val = w[0] * cos(th - om * tn);
    }
    pe += val;
    vne += val * kn / (sqrt(kk) * w[6]);
  }
  q.ext[(slot * 2) * q.nf + t] = pe;
  q.ext[(slot * 2 + 1) * q.nf + t] = vne;
}

hipError_t launch_exterior(const ExteriorParams& q, hipStream_t s) {
  const int64_t n = q.nslots * q.nf;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(exterior_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q);
  return hipGetLastError();
}

}  // namespace dgw
