// Launch wrappers and the launcher table for one (dim, precision) pair; the
// including translation unit defines DGW_DIM, DGW_T and DGW_INST_NAME.
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace dgw {

template <typename K>
static hipError_t ensure_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int D, int N, typename T, int EPI, int SEL, bool GB = false, int MB = 1, bool GOUT = GB>
hipError_t launch_op(const OpParams& p, hipStream_t s) {
  constexpr int CPW = cells_per_group(D, N, SEL);
  if (p.cpw != CPW) return hipErrorInvalidValue;
  const size_t lds = (size_t)CPW * OpLayout<D, N, T>::per_cell * sizeof(T);
  hipError_t e = ensure_lds(op_kernel<D, N, T, EPI, CPW, GB, MB, GOUT>, lds);
  if (e != hipSuccess) return e;
  const int nmb = (p.B + MB - 1) / MB;
  hipLaunchKernelGGL((op_kernel<D, N, T, EPI, CPW, GB, MB, GOUT>), dim3(p.groups * nmb), dim3(op_threads(D, N)),
                     lds, s, p);
  return hipGetLastError();
}

// Member-block launchers (kMemberBlock batch members per workgroup, the
// geometry loaded once): 3D, GL storage basis only.
template <int D, int N, typename T, int EPI, int SEL>
constexpr OpLaunch member_block_op() {
  if constexpr (D == 3)
    return launch_op<D, N, T, EPI, SEL, false, kMemberBlock>;
  else
    return nullptr;
}

template <int D, int N, typename T, int R, int SEL, bool HDG = false, bool GS = false>
hipError_t launch_tck(const TckParams& p, hipStream_t s) {
  constexpr int CPW = cells_per_group(D, N, SEL);
  if (p.cpw != CPW) return hipErrorInvalidValue;
  const size_t lds = (size_t)CPW * TckLayout<D, N, T>::bytes_per_cell(R);
  hipError_t e = ensure_lds(tck_kernel<D, N, T, R, CPW, HDG, GS>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tck_kernel<D, N, T, R, CPW, HDG, GS>), dim3(p.groups * p.B), dim3(tck_threads(D, N)), lds, s,
                     p);
  return hipGetLastError();
}

template <int D, int N, typename T, bool GS = false>
hipError_t launch_energy(const EnergyParams& p, hipStream_t s) {
  const size_t lds = (size_t)p.cpw * (D + 1) * ipow(N, D) * sizeof(T);
  hipError_t e = ensure_lds(energy_kernel<D, N, T, GS>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((energy_kernel<D, N, T, GS>), dim3(p.groups * p.B), dim3(op_threads(D, N)), lds, s, p);
  return hipGetLastError();
}

// Launchers of one storage basis (GS: Gauss): the operator per epilogue, the
// TCK per reduction period, HDG-ADER and the energy.  In the Gauss basis the
// ADER update reads the TCK sum I in the GL basis (the face nodes of the
// neighbours, as with GL storage) and writes u at the Gauss points.
template <int D, int N, typename T, bool GS>
constexpr BasisLaunchers basis_launchers() {
  return {{{launch_op<D, N, T, EPI_STORE, 0, GS>, launch_op<D, N, T, EPI_STORE, 1, GS>},
           {launch_op<D, N, T, EPI_LSRK, 0, GS>, launch_op<D, N, T, EPI_LSRK, 1, GS>},
           {launch_op<D, N, T, EPI_ADD, 0, false, 1, GS>, launch_op<D, N, T, EPI_ADD, 1, false, 1, GS>}},
          {{launch_tck<D, N, T, 0, 0, false, GS>, launch_tck<D, N, T, 0, 1, false, GS>},
           {launch_tck<D, N, T, 1, 0, false, GS>, launch_tck<D, N, T, 1, 1, false, GS>},
           {launch_tck<D, N, T, 2, 0, false, GS>, launch_tck<D, N, T, 2, 1, false, GS>},
           {launch_tck<D, N, T, 3, 0, false, GS>, launch_tck<D, N, T, 3, 1, false, GS>}},
          {launch_tck<D, N, T, 2, 0, true, GS>, launch_tck<D, N, T, 2, 1, true, GS>},
          launch_energy<D, N, T, GS>};
}

template <int D, int N, typename T>
const Launchers* make_launchers() {
  static const Launchers L = {
      {basis_launchers<D, N, T, false>(), basis_launchers<D, N, T, true>()},
      {{member_block_op<D, N, T, EPI_STORE, 0>(), member_block_op<D, N, T, EPI_STORE, 1>()},
       {member_block_op<D, N, T, EPI_LSRK, 0>(), member_block_op<D, N, T, EPI_LSRK, 1>()},
       {member_block_op<D, N, T, EPI_ADD, 0>(), member_block_op<D, N, T, EPI_ADD, 1>()}},
      {cells_per_group(D, N, 0), cells_per_group(D, N, 1)},
      (int)(OpLayout<D, N, T>::per_cell * sizeof(T)),
      {TckLayout<D, N, T>::bytes_per_cell(0), TckLayout<D, N, T>::bytes_per_cell(1),
       TckLayout<D, N, T>::bytes_per_cell(2), TckLayout<D, N, T>::bytes_per_cell(3)},
      (int)((D + 1) * ipow(N, D) * sizeof(T))};
  return &L;
}

}  // namespace dgw

#define DGW_DEFINE_INST(NAME, DIM, TYPE)                          \
  namespace dgw {                                                 \
  hipError_t NAME##_upload(const double* t64, const float* t32) { \
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab64), t64,    \
                                     kTabTotal * sizeof(double)); \
    if (e != hipSuccess) return e;                                \
    return hipMemcpyToSymbol(HIP_SYMBOL(c_tab32), t32,            \
                             kTabTotal * sizeof(float));          \
  }                                                               \
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
