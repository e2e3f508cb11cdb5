// Parameters and launcher of the prescribed-exterior evaluation kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dgw_params_time.hpp"

namespace dgw {

struct ExteriorParams {
  const int64_t* faces;    // [nslots]: face id cell * 2d + f of each prescribed face
  const double* bx;        // [nslots][d][nf] face point coordinates
  const double* geo_face;  // [nc][2d][d+2][nf] (area vectors for the normals)
  const double* waves;     // [n_waves][7]: A, k (3), omega, phi, Z
  double* ext;             // out: [nslots][2][nf] p+, v+.n
  int64_t nslots;
  int dim, nf, n_waves;
  int integral;            // 1: integral over [tn, tn + dt] (ADER update), 0: value at tn + t_off
  StepTime time;
};

hipError_t launch_exterior(const ExteriorParams& q, hipStream_t s);

}  // namespace dgw
