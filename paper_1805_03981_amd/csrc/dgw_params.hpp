// Kernel parameter blocks and the launcher table shared by the host code and
// the per-(dim, precision) kernel instantiation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "dgw_params_time.hpp"

namespace dgw {

constexpr int kMaxLevels = 9;  // TCK levels: up to k+1 with the reduction every derivative

// Boundary codes of the neighbour table (DGW_BC_WALL, DGW_BC_ABSORBING).
constexpr int kBcWall = -1, kBcAbsorbing = -2, kBcPrescribed = -3;
constexpr int kMaxPlaneWaves = 8;

// Threads per workgroup for dimension d and n points per direction.  The
// kernels run one cell per workgroup once a cell has more than 256 points;
// a wider workgroup then gives the cell more waves, which pays only where
// the LDS already limits a CU to one or two cells and the registers do not
// cut that further (measured on 40^3 meshes, k = 6..8): the operator sweep
// widens for 9^3 points, the TCK for 8^3 and 9^3.
__host__ __device__ constexpr int op_threads(int d, int n) {
  const int np = d == 2 ? n * n : n * n * n;
  return np <= 512 ? 256 : 1024;
}
__host__ __device__ constexpr int tck_threads(int d, int n) {
  const int np = d == 2 ? n * n : n * n * n;
  return np <= 343 ? 256 : (np <= 512 ? 512 : 1024);
}  // Gauss sets of the degree reduction: k+1, k-1, ... (k <= 8)

// Epilogues of the fused operator sweep.
enum Epilogue { EPI_STORE = 0, EPI_LSRK = 1, EPI_ADD = 2 };
// Batch members per workgroup of the member-block operator variant.
constexpr int kMemberBlock = 8;

struct SourceParams {
  const int* cell;        // [B] source cell of each member, or nullptr (no sources)
  const double* gvec;     // [B][np] GL coefficients of g (pressure component)
  const double* glev[kMaxLevels];  // [B][m_l^d] g at the level-l Gauss points (ADER)
  const double* wave;     // [B][3]: f, t0, amp of the Ricker wavelet
};

struct OpParams {
  const double* u;        // input state, GL, [B][nc][d+1][np]
  double* out;            // EPI_STORE: L u
  double* du;             // EPI_LSRK: stage register (in/out)
  const double* u_base;   // EPI_ADD: u_n (the result is u_base + L u)
  double* u_next;         // EPI_LSRK / EPI_ADD: new state
  const double* geo_cell; // [nc][d*d+2][np]: w detJ J^-1 (b*d+a), mu_v, mu_p
  const double* geo_face; // [nc][2d][d+2][n^(d-1)]: a (d), Z-, Z+
  const int* nb;          // [nc][2d]
  const int* fo;          // [nc][2d] 8 f' + o (neighbour face, orientation) or nullptr (f' = f^1, o = 0)
  const double* ext;      // [slot][2][n^(d-1)]: p+, v+.n of the prescribed faces for this launch, or
                          // nullptr; nb holds kBcPrescribed - slot for such a face
  int64_t nc;
  int cpw;                // cells per workgroup
  int groups;             // ceil(nc / cpw)
  int B;
  int central;            // 1: central flux, 0: upwind
  double acoef, bcoef, dt;  // LSRK: du <- acoef du + dt (L u + s g); u_next <- u + bcoef du
  int two_r;              // LSRK 2R form: k = dt (L u + s g); du <- du + bcoef k (du := u in the
                          // first stage); u_next <- du + acoef k
  int first;              // 2R: first stage of the step
  StepTime time;          // LSRK: source at tn + t_off; ADER update: int_{tn}^{tn+dt} s * g
  SourceParams src;
};

struct TckParams {
  const double* u;        // [B][nc][d+1][np] GL (HDG-ADER: W = L u, may alias I)
  double* I;              // [B][nc][d+1][np] GL, time-integrated Taylor sum
  const double* u_base;   // HDG-ADER only: u, for the dt u term of I
  const double* geo_lev[kMaxLevels];  // level 0 = geo_cell; [nc][d*d+2][m_l^d]
  int64_t nc;
  int cpw, groups, B;
  double dt;
  StepTime time;          // tn = time at the start of the step (source derivatives)
  SourceParams src;
};

struct EnergyParams {
  const double* u;
  const double* geo_cell;
  double* partial;        // [B][groups]
  int64_t nc;
  int cpw, groups, B;
};

using OpLaunch = hipError_t (*)(const OpParams&, hipStream_t);
using TckLaunch = hipError_t (*)(const TckParams&, hipStream_t);
using EnergyLaunch = hipError_t (*)(const EnergyParams&, hipStream_t);

// Kernels are compiled for two launch shapes (sel 0/1: cells per workgroup
// cpw[sel]); p.cpw must equal cpw[sel] of the launcher that is called.
// The kernels of one storage basis.
struct BasisLaunchers {
  OpLaunch op[3][2];      // [Epilogue][sel]
  TckLaunch tck[4][2];    // [reduction period 0 (none), 1, 2 (Alg. 3), 3][sel]
  TckLaunch tck_hdg[2];   // HDG-ADER variant (with reduction) [sel]
  EnergyLaunch energy;
};

struct Launchers {
  BasisLaunchers basis[2];  // [DGW_BASIS_GL, DGW_BASIS_GAUSS]
  OpLaunch op_mb[3][2];   // kMemberBlock batch members per workgroup, [Epilogue][sel]; 3D, GL only (else nullptr)
  int cpw[2];
  int op_lds_per_cell;    // bytes of LDS per cell
  int tck_lds_per_cell[4];  // per reduction period
  int energy_lds_per_cell;
};

// precision: 0 = FP64, 1 = FP32 split.  nullptr if (dim, n) is unsupported.
const Launchers* launchers(int dim, int n, int precision);

// Table layout (element offsets) of the 1D matrices for n = k+1 nodes.
// S (n x n), S^-1 (n x n), D (n x n), LF0 (n), LF1 (n); then, for each
// reduction period r of the TCK (r = 2 first, then 1 and 3), per reduced
// level l = 1.. with m = n - r l >= 1 points and mp = m + r: D_l (m x m)
// collocation derivative, P_l (m x mp) projection from level l-1, E_l
// (mp x m) interpolation back to level l-1, F_l (m x n) evaluation of a
// level-0 Gauss polynomial at the level-l points, Q_l (n x m) evaluation of
// a level-l Gauss polynomial at the n GL nodes.
__host__ __device__ constexpr int tab_S(int) { return 0; }
__host__ __device__ constexpr int tab_Sinv(int n) { return n * n; }
__host__ __device__ constexpr int tab_D(int n) { return 2 * n * n; }
__host__ __device__ constexpr int tab_LF0(int n) { return 3 * n * n; }
__host__ __device__ constexpr int tab_LF1(int n) { return 3 * n * n + n; }
// levels l = 0.. of period r with n - r l >= 1 points (r = 0: no reduction)
__host__ __device__ constexpr int num_levels_r(int n, int r) { return r == 0 ? 1 : (n - 1) / r + 1; }
__host__ __device__ constexpr int levels_block(int n, int r) {
  int sz = 0;
  for (int l = 1; l < num_levels_r(n, r); ++l) {
    const int m = n - r * l, mp = m + r;
    sz += m * m + m * mp + mp * m + 2 * m * n;
  }
  return sz;
}
__host__ __device__ constexpr int tab_levels_start(int n, int r) {
  const int base = 3 * n * n + 2 * n;
  return r == 2 ? base : (r == 1 ? base + levels_block(n, 2) : base + levels_block(n, 2) + levels_block(n, 1));
}
__host__ __device__ constexpr int tab_level(int n, int l, int r = 2) {
  int off = tab_levels_start(n, r);
  for (int j = 1; j < l; ++j) {
    const int m = n - r * j, mp = m + r;
    off += m * m + m * mp + mp * m + 2 * m * n;
  }
  return off;
}
__host__ __device__ constexpr int tab_level_D(int n, int l, int r = 2) { return tab_level(n, l, r); }
__host__ __device__ constexpr int tab_level_P(int n, int l, int r = 2) {
  return tab_level(n, l, r) + (n - r * l) * (n - r * l);
}
__host__ __device__ constexpr int tab_level_E(int n, int l, int r = 2) {
  return tab_level_P(n, l, r) + (n - r * l) * (n - r * (l - 1));
}
__host__ __device__ constexpr int tab_level_F(int n, int l, int r = 2) {
  return tab_level_E(n, l, r) + (n - r * (l - 1)) * (n - r * l);
}
__host__ __device__ constexpr int tab_level_Q(int n, int l, int r = 2) { return tab_level_F(n, l, r) + (n - r * l) * n; }
__host__ __device__ constexpr int num_levels(int n) { return num_levels_r(n, 2); }  // n, n-2, ... >= 1
__host__ __device__ constexpr int tab_size(int n) { return tab_levels_start(n, 3) + levels_block(n, 3); }
// All degrees share one constant-memory table: n = 2..9 back to back.
constexpr int kMinN = 2, kMaxN = 9;
__host__ __device__ constexpr int tab_base(int n) {
  int off = 0;
  for (int m = kMinN; m < n; ++m) off += tab_size(m);
  return off;
}
constexpr int kTabTotal = tab_base(kMaxN + 1);

// Uploads the 1D tables of every degree to the constant memory of the
// current device, for the kernels of one (dim, precision) unit.
using TableUpload = hipError_t (*)(const double* t64, const float* t32);

}  // namespace dgw
