// Launch wrappers and the launcher table for one (dim, precision) pair; the
// including translation unit defines DGW_DIM, DGW_T and DGW_INST_NAME.
#pragma once
#include "kernels.hpp"

namespace dgw {

template <typename K>
static hipError_t ensure_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int D, int N, typename T, int EPI>
hipError_t launch_op(const OpParams& p, int nth, hipStream_t s) {
  const size_t lds = (size_t)p.cpw * OpLayout<D, N, T>::per_cell * sizeof(T);
  hipError_t e = ensure_lds(op_kernel<D, N, T, EPI>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((op_kernel<D, N, T, EPI>), dim3(p.groups * p.B), dim3(nth), lds, s, p);
  return hipGetLastError();
}

template <int D, int N, typename T, bool R>
hipError_t launch_tck(const TckParams& p, int nth, hipStream_t s) {
  const size_t lds = (size_t)p.cpw * TckLayout<D, N, T>::bytes_per_cell;
  hipError_t e = ensure_lds(tck_kernel<D, N, T, R>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tck_kernel<D, N, T, R>), dim3(p.groups * p.B), dim3(nth), lds, s, p);
  return hipGetLastError();
}

template <int D, int N, typename T>
hipError_t launch_energy(const EnergyParams& p, int nth, hipStream_t s) {
  const size_t lds = (size_t)p.cpw * (D + 1) * ipow(N, D) * sizeof(T);
  hipError_t e = ensure_lds(energy_kernel<D, N, T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((energy_kernel<D, N, T>), dim3(p.groups * p.B), dim3(nth), lds, s, p);
  return hipGetLastError();
}

template <int D, int N, typename T>
const Launchers* make_launchers() {
  static const Launchers L = {
      {launch_op<D, N, T, EPI_STORE>, launch_op<D, N, T, EPI_LSRK>, launch_op<D, N, T, EPI_ADD>},
      {launch_tck<D, N, T, true>, launch_tck<D, N, T, false>},
      launch_energy<D, N, T>,
      (int)(OpLayout<D, N, T>::per_cell * sizeof(T)),
      TckLayout<D, N, T>::bytes_per_cell,
      (int)((D + 1) * ipow(N, D) * sizeof(T))};
  return &L;
}

}  // namespace dgw

#define DGW_DEFINE_INST(NAME, DIM, TYPE)                          \
  namespace dgw {                                                 \
  const Launchers* NAME(int n) {                                  \
    switch (n) {                                                  \
      case 2: return make_launchers<DIM, 2, TYPE>();              \
      case 3: return make_launchers<DIM, 3, TYPE>();              \
      case 4: return make_launchers<DIM, 4, TYPE>();              \
      case 5: return make_launchers<DIM, 5, TYPE>();              \
      case 6: return make_launchers<DIM, 6, TYPE>();              \
      case 7: return make_launchers<DIM, 7, TYPE>();              \
      case 8: return make_launchers<DIM, 8, TYPE>();              \
      case 9: return make_launchers<DIM, 9, TYPE>();              \
      default: return nullptr;                                    \
    }                                                             \
  }                                                               \
  }
