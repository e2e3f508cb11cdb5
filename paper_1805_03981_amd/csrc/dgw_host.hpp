// Host-side internals of the dgw library: the mesh object, setup routines
// and error reporting.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dgw.h"
#include "dgw_params.hpp"

namespace dgw {

void set_error(const std::string& msg);
dgw_status fail(dgw_status code, const std::string& msg);
#define DGW_HIP(call)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return ::dgw::fail(DGW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// 1D rule on [0,1] in long double (nodes ascending).
struct Rule {
  std::vector<long double> x, w;
};
Rule gauss_rule(int n);
Rule gauss_lobatto_rule(int n);
long double lagrange_value(const std::vector<long double>& nodes, int j, long double x);
long double lagrange_deriv(const std::vector<long double>& nodes, int j, long double x);
// Tables in the layout of dgw_params.hpp (tab_*) for n nodes per direction.
std::vector<double> build_tables(int n);

// Host copy of the setup (FP64).
struct HostSetup {
  int dim = 0, k = 0, n = 0, q = 0;
  int64_t nc = 0;
  std::vector<double> geo_nodes;           // [nc][(q+1)^d][d]
  std::vector<int32_t> nb;                 // [nc][2d]
  std::vector<int32_t> fo;                 // [nc][2d] 8 f' + o, or empty (standard faces)
  std::vector<double> cell;                // [nc][d*d+2][np]
  std::vector<double> face;                // [nc][2d][d+2][nf]
  std::vector<std::vector<double>> level;  // [l] (l >= 1): [nc][d*d+2][m_l^d]
  std::vector<double> hK, cK;
  bool prescribed = false;                 // some face is DGW_BC_PRESCRIBED
  std::vector<double> face_x;              // [nc][2d][d][nf] face point coordinates (only if prescribed)
  std::vector<double> waves;               // [n][7]: A, k (3), omega, phi, Z
  double dt_unit = 0, h_min = 0, c_max = 0;
  dgw_material_fn material = nullptr;
  void* material_ctx = nullptr;
};
dgw_status build_setup(const dgw_mesh_desc& desc, HostSetup& hs);
// Face pairing: the neighbour's face of face f of cell c, the orientation
// code of the pair, and the index on the neighbour's face of own face point p.
int face_of_neighbor(const HostSetup& hs, int64_t c, int f);
int orient_of(const HostSetup& hs, int64_t c, int f);
int orient_face_index(int d, int n, int o, int p);
// Metric and mass factors at the m^d Gauss points of every cell (layout of
// HostSetup::level), for the reduced TCK levels of another period.
dgw_status build_level_metric(const HostSetup& hs, int m, std::vector<double>& out);
// Physical coordinates of the GL nodes, [nc][np][d].
void node_coords(const HostSetup& hs, std::vector<double>& out);
// Evaluate the map of one cell at a reference point: x[d], J[d][d].
void map_point(const HostSetup& hs, int64_t cell, const double* xi, double* x, double* J);

// Which compiled launch shape (cells per workgroup) a kernel family uses.
struct LaunchShape {
  int sel = 0;
};

}  // namespace dgw

struct dgw_mesh {
  dgw::HostSetup hs;
  int precision = 0, flux = 0, device = -1, max_batch = 1;
  int basis = 0;  // DGW_BASIS_GL or DGW_BASIS_GAUSS
  int np = 0, nf = 0, ncomp = 0, nlev = 0;
  std::vector<int> level_pts;
  const dgw::Launchers* L = nullptr;
  // device memory owned by the mesh
  double* d_cell = nullptr;
  double* d_face = nullptr;
  double* d_level[dgw::kMaxLevels] = {};     // reduced levels of period 2 (n - 2l points)
  double* d_level_pts[dgw::kMaxLevels + 1] = {};  // other periods' levels, by points per direction
  int32_t* d_nb = nullptr;
  int32_t* d_fo = nullptr;  // face orientation codes, nullptr for the standard faces
  // prescribed faces (slots in face order): face ids, face point
  // coordinates, plane waves, and the exterior state of the current launch
  int64_t n_pslots = 0;
  int64_t* d_pfaces = nullptr;
  double* d_bx = nullptr;
  double* d_waves = nullptr;
  double* d_ext = nullptr;
  double* d_partial = nullptr;  // energy partial sums [max_batch][groups]
  int64_t device_bytes = 0;
  dgw::LaunchShape op_shape, tck_shape;
  int op_sel_epi[3] = {-1, -1, -1};  // per operator epilogue (store, LSRK, ADER update); -1: op_shape
  bool tuned = false;
  std::mutex mtx;
};

struct dgw_sources {
  dgw_mesh* mesh = nullptr;
  int n = 0;
  std::vector<int> cell;
  int* d_cell = nullptr;
  double* d_gvec = nullptr;
  double* d_glev[dgw::kMaxLevels] = {};
  double* d_wave = nullptr;
};
