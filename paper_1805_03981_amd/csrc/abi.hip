// C-ABI entry points of libdgw: mesh lifecycle, operator application, the
// LSRK(5,4) and ADER steppers, point sources, energy and the batch solver.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <tuple>
#include <vector>

#include "dgw_exterior.hpp"
#include "dgw_host.hpp"

namespace dgw {

const Launchers* launchers_d2_f64(int n);
const Launchers* launchers_d2_f32(int n);
const Launchers* launchers_d3_f64(int n);
const Launchers* launchers_d3_f32(int n);
hipError_t launchers_d2_f64_upload(const double*, const float*);
hipError_t launchers_d2_f32_upload(const double*, const float*);
hipError_t launchers_d3_f64_upload(const double*, const float*);
hipError_t launchers_d3_f32_upload(const double*, const float*);

const Launchers* launchers(int dim, int n, int precision) {
  if (dim == 2) return precision ? launchers_d2_f32(n) : launchers_d2_f64(n);
  if (dim == 3) return precision ? launchers_d3_f32(n) : launchers_d3_f64(n);
  return nullptr;
}

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
dgw_status fail(dgw_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

__global__ void advance_counter(long long* ctr, int by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] += by;
}

// Five-stage fourth-order 2N-storage Runge-Kutta (Carpenter & Kennedy 1994),
// Williamson form; the paper's LSRK4(5) family (Sec. 2.2).
struct Lsrk54 {
  double A[5], B[5], C[5];
  Lsrk54() {
    const long double a[5][2] = {{0, 1},
                                 {-567301805773.0L, 1357537059087.0L},
                                 {-2404267990393.0L, 2016746695238.0L},
                                 {-3550918686646.0L, 2091501179385.0L},
                                 {-1275806237668.0L, 842570457699.0L}};
    const long double b[5][2] = {{1432997174477.0L, 9575080441755.0L},
                                 {5161836677717.0L, 13612068292357.0L},
                                 {1720146321549.0L, 2090206949498.0L},
                                 {3134564353537.0L, 4481467310338.0L},
                                 {2277821191437.0L, 14882151754819.0L}};
    const long double c[5][2] = {{0, 1},
                                 {1432997174477.0L, 9575080441755.0L},
                                 {2526269341429.0L, 6820363962896.0L},
                                 {2006345519317.0L, 3224310063776.0L},
                                 {2802321613138.0L, 2924317926251.0L}};
    for (int i = 0; i < 5; ++i) {
      A[i] = (double)(a[i][0] / a[i][1]);
      B[i] = (double)(b[i][0] / b[i][1]);
      C[i] = (double)(c[i][0] / c[i][1]);
    }
  }
};
static const Lsrk54 kLsrk;

// LSRK5(9) in two-register form: subdiagonal alpha (8) and weights b (9) of
// the Butcher tableau (a_ij = b_j for j < i-1), the root of the 17 order-5
// conditions named by a 10-digit key, refined by Newton's method in long
// double with derivatives by complex steps (exact for polynomials).
struct Lsrk59 {
  double alpha[8], b[9], c[9];
  bool ok = false;
  template <typename X>
  static void conditions(const X* x, X* r) {
    X a[9][9] = {}, c[9], ac[9], ac2[9], ac3[9], aac[9], acac[9], aac2[9], aaac[9], bb[9];
    for (int j = 0; j < 9; ++j) bb[j] = x[8 + j];
    for (int i = 1; i < 9; ++i) {
      for (int j = 0; j + 1 < i; ++j) a[i][j] = bb[j];
      a[i][i - 1] = x[i - 1];
    }
    for (int i = 0; i < 9; ++i) {
      c[i] = X(0);
      for (int j = 0; j < 9; ++j) c[i] += a[i][j];
    }
    auto mv = [&](const X* v, X* out) {
      for (int i = 0; i < 9; ++i) {
        out[i] = X(0);
        for (int j = 0; j < 9; ++j) out[i] += a[i][j] * v[j];
      }
    };
    X c2[9], c3[9], cac[9];
    for (int i = 0; i < 9; ++i) {
      c2[i] = c[i] * c[i];
      c3[i] = c2[i] * c[i];
    }
    mv(c, ac);
    mv(c2, ac2);
    mv(c3, ac3);
    mv(ac, aac);
    for (int i = 0; i < 9; ++i) cac[i] = c[i] * ac[i];
    mv(cac, acac);
    mv(ac2, aac2);
    mv(aac, aaac);
    auto dot = [&](auto f) {
      X acc(0);
      for (int j = 0; j < 9; ++j) acc += bb[j] * f(j);
      return acc;
    };
    r[0] = dot([&](int) { return X(1); }) - X(1.0L);
    r[1] = dot([&](int j) { return c[j]; }) - X(1.0L / 2);
    r[2] = dot([&](int j) { return c2[j]; }) - X(1.0L / 3);
    r[3] = dot([&](int j) { return ac[j]; }) - X(1.0L / 6);
    r[4] = dot([&](int j) { return c3[j]; }) - X(1.0L / 4);
    r[5] = dot([&](int j) { return cac[j]; }) - X(1.0L / 8);
    r[6] = dot([&](int j) { return ac2[j]; }) - X(1.0L / 12);
    r[7] = dot([&](int j) { return aac[j]; }) - X(1.0L / 24);
    r[8] = dot([&](int j) { return c2[j] * c2[j]; }) - X(1.0L / 5);
    r[9] = dot([&](int j) { return c2[j] * ac[j]; }) - X(1.0L / 10);
    r[10] = dot([&](int j) { return c[j] * ac2[j]; }) - X(1.0L / 15);
    r[11] = dot([&](int j) { return c[j] * aac[j]; }) - X(1.0L / 30);
    r[12] = dot([&](int j) { return ac[j] * ac[j]; }) - X(1.0L / 20);
    r[13] = dot([&](int j) { return ac3[j]; }) - X(1.0L / 20);
    r[14] = dot([&](int j) { return acac[j]; }) - X(1.0L / 40);
    r[15] = dot([&](int j) { return aac2[j]; }) - X(1.0L / 60);
    r[16] = dot([&](int j) { return aaac[j]; }) - X(1.0L / 120);
  }
  Lsrk59() {
    using L = long double;
    using Cx = std::complex<long double>;
    L x[17] = {0.1702644982L, -0.09676474868L, 0.0244514839L, 0.1382907685L, 0.2294641842L, 0.5748250612L,
               -0.1211285367L, 0.09183392377L, 0.1804864076L, 0.622352667L, -0.4110536782L, -0.01125784998L,
               0.009612188747L, 0.1576014651L, 0.1129031225L, 0.08522852155L, 0.2541271558L};
    const L h = 1e-40L;
    for (int it = 0; it < 30; ++it) {
      L r[17], J[17][18];
      conditions<L>(x, r);
      L rmax = 0;
      for (L v : r) rmax = std::max(rmax, std::fabs(v));
      if (rmax < 1e-18L) {
        ok = true;
        break;
      }
      for (int j = 0; j < 17; ++j) {
        Cx xc[17], rc[17];
        for (int i = 0; i < 17; ++i) xc[i] = Cx(x[i], i == j ? h : 0.0L);
        conditions<Cx>(xc, rc);
        for (int i = 0; i < 17; ++i) J[i][j] = rc[i].imag() / h;
      }
      for (int i = 0; i < 17; ++i) J[i][17] = -r[i];
      // Gaussian elimination with partial pivoting
      for (int col = 0; col < 17; ++col) {
        int piv = col;
        for (int i = col + 1; i < 17; ++i)
          if (std::fabs(J[i][col]) > std::fabs(J[piv][col])) piv = i;
        for (int k = 0; k < 18; ++k) std::swap(J[col][k], J[piv][k]);
        for (int i = col + 1; i < 17; ++i) {
          const L f = J[i][col] / J[col][col];
          for (int k = col; k < 18; ++k) J[i][k] -= f * J[col][k];
        }
      }
      L dx[17];
      for (int i = 16; i >= 0; --i) {
        L acc = J[i][17];
        for (int k = i + 1; k < 17; ++k) acc -= J[i][k] * dx[k];
        dx[i] = acc / J[i][i];
      }
      for (int i = 0; i < 17; ++i) x[i] += dx[i];
    }
    L cc[9] = {0};
    for (int i = 1; i < 9; ++i) {
      for (int j = 0; j + 1 < i; ++j) cc[i] += x[8 + j];
      cc[i] += x[i - 1];
    }
    for (int i = 0; i < 8; ++i) alpha[i] = (double)x[i];
    for (int i = 0; i < 9; ++i) {
      b[i] = (double)x[8 + i];
      c[i] = (double)cc[i];
    }
  }
};
static const Lsrk59 kLsrk59;

static int ipw(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

static int64_t state_elems(const dgw_mesh* m) { return m->hs.nc * m->ncomp * m->np; }

static const int64_t kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950

static LaunchShape default_shape(const Launchers* L, int lds_per_cell) {
  LaunchShape s;
  // the larger group when two of them still fit a CU twice over
  s.sel = (int64_t)L->cpw[1] * lds_per_cell * 2 <= kLdsLimit ? 1 : 0;
  return s;
}

// The 1D tables of every degree go to each kernel unit's constant memory,
// once per device.
static dgw_status ensure_tables(int device) {
  static std::mutex mtx;
  static std::vector<int> done;
  std::lock_guard<std::mutex> lk(mtx);
  if (std::find(done.begin(), done.end(), device) != done.end()) return DGW_OK;
  std::vector<double> t64(kTabTotal, 0.0);
  for (int n = kMinN; n <= kMaxN; ++n) {
    const std::vector<double> t = build_tables(n);
    std::copy(t.begin(), t.end(), t64.begin() + tab_base(n));
  }
  std::vector<float> t32(t64.begin(), t64.end());
  const TableUpload up[4] = {launchers_d2_f64_upload, launchers_d2_f32_upload, launchers_d3_f64_upload,
                             launchers_d3_f32_upload};
  for (auto f : up) DGW_HIP(f(t64.data(), t32.data()));
  done.push_back(device);
  return DGW_OK;
}

static dgw_status check_mesh(const dgw_mesh* m) {
  if (!m) return fail(DGW_EINVAL, "mesh is NULL");
  if (m->device < 0) return fail(DGW_EINVAL, "mesh was created without a device (DGW_DEVICE_NONE)");
  return DGW_OK;
}

// HDG-ADER takes its first derivative from the operator at the step start;
// the time derivatives of prescribed exterior data are not part of it.
static dgw_status check_hdg_faces(const dgw_mesh* m, int flags) {
  if ((flags & DGW_ADER_HDG) && m->hs.prescribed)
    return fail(DGW_EUNSUPPORTED, "DGW_ADER_HDG is not available with DGW_BC_PRESCRIBED faces");
  return DGW_OK;
}

// The kernels of the mesh's storage basis.
static const BasisLaunchers& basis_launchers(const dgw_mesh* m) {
  return m->L->basis[m->basis == DGW_BASIS_GAUSS ? 1 : 0];
}

// The operator launcher for epilogue epi and launch shape sel in the mesh's
// storage basis.  Operator launch shape index: bit 0 selects the compiled
// cells per workgroup, bit 1 the member-block variant (kMemberBlock batch
// members per workgroup with the geometry loaded once; GL storage basis
// only) instead of one member per group.
static OpLaunch op_launch(const dgw_mesh* m, int epi, int shape) {
  const int sel = shape & 1;
  if (shape & 2) return m->basis == DGW_BASIS_GAUSS ? nullptr : m->L->op_mb[epi][sel];
  return basis_launchers(m).op[epi][sel];
}

// One operator launch; on a mesh with prescribed faces the exterior state
// of this launch (at p.time, or integrated over the step for the ADER
// update) is evaluated first on the same stream.
static hipError_t run_op(const dgw_mesh* m, int epi, int sel, OpParams p, hipStream_t s) {
  if ((sel & 2) && (p.B == 1 || !op_launch(m, epi, sel))) sel &= 1;  // one member: the plain kernel
  p.cpw = m->L->cpw[sel & 1];
  p.groups = (int)((m->hs.nc + p.cpw - 1) / p.cpw);
  if (m->d_ext) {
    ExteriorParams q;
    std::memset(&q, 0, sizeof(q));
    q.faces = m->d_pfaces;
    q.bx = m->d_bx;
    q.geo_face = m->d_face;
    q.waves = m->d_waves;
    q.ext = m->d_ext;
    q.nslots = m->n_pslots;
    q.dim = m->hs.dim;
    q.nf = m->nf;
    q.n_waves = (int)(m->hs.waves.size() / 7);
    q.integral = epi == EPI_ADD;
    q.time = p.time;
    const hipError_t e = launch_exterior(q, s);
    if (e != hipSuccess) return e;
  }
  return op_launch(m, epi, sel)(p, s);
}

// Launch shape of the operator with epilogue epi: the one tuned for that
// epilogue, else the mesh's operator shape.
static int op_sel(const dgw_mesh* m, int epi) {
  const int s = m->op_sel_epi[epi];
  return s >= 0 ? s : m->op_shape.sel;
}
static hipError_t run_op(const dgw_mesh* m, int epi, const OpParams& p, hipStream_t s) {
  return run_op(m, epi, op_sel(m, epi), p, s);
}

static dgw_status set_device(const dgw_mesh* m) {
  DGW_HIP(hipSetDevice(m->device));
  return DGW_OK;
}

static void fill_sources(SourceParams& sp, const dgw_sources* src) {
  std::memset(&sp, 0, sizeof(sp));
  if (!src) return;
  sp.cell = src->d_cell;
  sp.gvec = src->d_gvec;
  for (int l = 0; l < kMaxLevels; ++l) sp.glev[l] = src->d_glev[l];
  sp.wave = src->d_wave;
}

static OpParams op_params(const dgw_mesh* m, int B, const dgw_sources* src) {
  OpParams p;
  std::memset(&p, 0, sizeof(p));
  p.geo_cell = m->d_cell;
  p.geo_face = m->d_face;
  p.nb = m->d_nb;
  p.fo = m->d_fo;
  p.ext = m->d_ext;
  p.nc = m->hs.nc;
  p.cpw = m->L->cpw[m->op_shape.sel];
  p.groups = (int)((m->hs.nc + p.cpw - 1) / p.cpw);
  p.B = B;
  p.central = m->flux == DGW_FLUX_CENTRAL;
  fill_sources(p.src, src);
  return p;
}

// Device metric of the m^d Gauss set: a level of the mesh's own reduction
// (period 2, built with the mesh) or one built for another period.
static const double* level_metric(const dgw_mesh* m, int pts) {
  const int n = m->hs.n;
  if (pts == n) return m->d_cell;
  if ((n - pts) % 2 == 0 && m->d_level[(n - pts) / 2]) return m->d_level[(n - pts) / 2];
  return m->d_level_pts[pts];
}

static TckParams tck_params(const dgw_mesh* m, int B, const dgw_sources* src, int period = 2) {
  TckParams p;
  std::memset(&p, 0, sizeof(p));
  for (int l = 0; l < num_levels_r(m->hs.n, period) && l < kMaxLevels; ++l)
    p.geo_lev[l] = level_metric(m, m->hs.n - period * l);
  p.nc = m->hs.nc;
  p.cpw = m->L->cpw[m->tck_shape.sel];
  p.groups = (int)((m->hs.nc + p.cpw - 1) / p.cpw);
  p.B = B;
  fill_sources(p.src, src);
  return p;
}

static dgw_status check_batch(const dgw_mesh* m, int B, const dgw_sources* src) {
  if (B < 1 || B > m->max_batch) return fail(DGW_EINVAL, "B must be in 1..max_batch");
  if ((int64_t)B * (m->hs.nc + 1) > INT32_MAX)
    return fail(DGW_EINVAL, "grid too large");
  if (src) {
    if (src->mesh != m) return fail(DGW_EINVAL, "sources were created for another mesh");
    if (src->n < B) return fail(DGW_EINVAL, "fewer sources than batch members");
  }
  return DGW_OK;
}

// One LSRK step (fused stages: 5 of the 2N LSRK4(5), or 9 of the 2R
// LSRK5(9)).  cur/oth: ping-pong state buffers; returns with the new state
// in *cur.
static int lsrk_stages(int scheme) { return scheme == DGW_SCHEME_LSRK59 ? 9 : 5; }

// Coefficients of fused stage i.  2N LSRK4(5): du <- A_i du + k,
// u <- u + B_i du.  2R LSRK5(9): du holds the accumulated solution U,
// U <- U + b_i k, and u_next the next stage state Y = U + (alpha_{i+1} - b_i) k
// (= U after the last stage).
static void set_lsrk_stage(OpParams& p, int scheme, int i, double dt) {
  if (scheme == DGW_SCHEME_LSRK59) {
    p.two_r = 1;
    p.first = i == 0;
    p.bcoef = kLsrk59.b[i];
    p.acoef = i < 8 ? kLsrk59.alpha[i] - kLsrk59.b[i] : 0.0;
    p.time.t_off = kLsrk59.c[i] * dt;
  } else {
    p.two_r = 0;
    p.first = 0;
    p.acoef = kLsrk.A[i];
    p.bcoef = kLsrk.B[i];
    p.time.t_off = kLsrk.C[i] * dt;
  }
}

static dgw_status lsrk_step(dgw_mesh* m, int B, const dgw_sources* src, double t0, double dt, int step_add,
                            const long long* ctr, double*& cur, double*& oth, double* du, hipStream_t s,
                            int scheme = DGW_SCHEME_LSRK54) {
  OpParams p = op_params(m, B, src);
  p.dt = dt;
  p.du = du;
  p.time = StepTime{ctr, t0, dt, step_add, 0.0};
  for (int i = 0; i < lsrk_stages(scheme); ++i) {
    p.u = cur;
    p.u_next = oth;
    set_lsrk_stage(p, scheme, i, dt);
    DGW_HIP(run_op(m, EPI_LSRK, p, s));
    std::swap(cur, oth);
  }
  return DGW_OK;
}

// Vector updates of an LSRK stage outside the operator sweep (the unfused
// variants, Sec. 4.3): merged, one pass over du, r = L u and u (the paper's
// optimized updater); standard, three BLAS-1 passes.  A stage coefficient
// A_i = 0 means du is not read (the work buffer may hold anything).
__global__ void __launch_bounds__(256) vu_merged(double* __restrict__ u, double* __restrict__ du,
                                                 const double* __restrict__ r, double a, double dt, double b,
                                                 int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (a != 0.0 ? a * du[i] : 0.0) + dt * r[i];
    du[i] = d;
    u[i] += b * d;
  }
}
__global__ void __launch_bounds__(256) vu_scale(double* __restrict__ x, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = a != 0.0 ? a * x[i] : 0.0;
}
__global__ void __launch_bounds__(256) vu_axpy(double* __restrict__ y, const double* __restrict__ x, double a,
                                               int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

static dgw_status lsrk_vector_update(int scheme, int stage, double dt, double* u, double* du, const double* r,
                                     int64_t n, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 16384);
  const double a = kLsrk.A[stage], b = kLsrk.B[stage];
  if (scheme == DGW_SCHEME_LSRK54_MERGED_VU) {
    hipLaunchKernelGGL(vu_merged, dim3(blocks), dim3(256), 0, s, u, du, r, a, dt, b, n);
  } else {
    hipLaunchKernelGGL(vu_scale, dim3(blocks), dim3(256), 0, s, du, a, n);
    hipLaunchKernelGGL(vu_axpy, dim3(blocks), dim3(256), 0, s, du, r, dt, n);
    hipLaunchKernelGGL(vu_axpy, dim3(blocks), dim3(256), 0, s, u, du, b, n);
  }
  DGW_HIP(hipGetLastError());
  return DGW_OK;
}

static dgw_status check_ader_flags(int flags, const dgw_sources* src) {
  const int periods = DGW_ADER_NOREDUCE | DGW_ADER_REDUCE_EVERY_STEP | DGW_ADER_REDUCE_EVERY_THIRD;
  if (flags & ~(periods | DGW_ADER_HDG)) return fail(DGW_EINVAL, "unknown ADER flags");
  const int pf = flags & periods;
  if (pf & (pf - 1)) return fail(DGW_EINVAL, "at most one of the reduction flags");
  if ((flags & DGW_ADER_HDG) && pf)
    return fail(DGW_EUNSUPPORTED, "HDG-ADER is built with the reduction every second derivative only");
  if ((flags & DGW_ADER_HDG) && src) return fail(DGW_EUNSUPPORTED, "HDG-ADER takes no sources");
  if ((flags & (DGW_ADER_REDUCE_EVERY_STEP | DGW_ADER_REDUCE_EVERY_THIRD)) && src)
    return fail(DGW_EUNSUPPORTED, "sources need the reduction every second derivative (or none)");
  return DGW_OK;
}

// reduction period of the TCK selected by the ADER flags
static int ader_period(int flags) {
  if (flags & DGW_ADER_NOREDUCE) return 0;
  if (flags & DGW_ADER_REDUCE_EVERY_STEP) return 1;
  if (flags & DGW_ADER_REDUCE_EVERY_THIRD) return 3;
  return 2;
}

// Builds (once) the metric of the reduced levels of a period other than the
// mesh's own (host evaluation of the map and the material, then upload).
static dgw_status ensure_period_levels(dgw_mesh* m, int period) {
  const int n = m->hs.n;
  for (int l = 1; l < num_levels_r(n, period); ++l) {
    const int pts = n - period * l;
    if (level_metric(m, pts)) continue;
    std::vector<double> host;
    dgw_status st = build_level_metric(m->hs, pts, host);
    if (st) return st;
    double* d = nullptr;
    DGW_HIP(hipMalloc(&d, host.size() * sizeof(double)));
    const hipError_t e = hipMemcpy(d, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(DGW_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    m->d_level_pts[pts] = d;
    m->device_bytes += (int64_t)(host.size() * sizeof(double));
  }
  return DGW_OK;
}

// launch shape of the TCK for a period: the tuned one unless its LDS (the
// every-derivative sums live there) does not fit
static int tck_sel(const dgw_mesh* m, int period) {
  const int sel = m->tck_shape.sel;
  return (int64_t)m->L->cpw[sel] * m->L->tck_lds_per_cell[period] <= kLdsLimit ? sel : 0;
}

static dgw_status ader_step(dgw_mesh* m, int flags, int B, const dgw_sources* src, double t0, double dt,
                            int step_add, const long long* ctr, double*& cur, double*& oth, double* I,
                            hipStream_t s) {
  const int period = ader_period(flags);
  TckParams tp = tck_params(m, B, src, period);
  const int sel = tck_sel(m, period);
  tp.cpw = m->L->cpw[sel];
  tp.groups = (int)((m->hs.nc + tp.cpw - 1) / tp.cpw);
  tp.u = cur;
  tp.I = I;
  tp.dt = dt;
  tp.time = StepTime{ctr, t0, dt, step_add, 0.0};
  if (flags & DGW_ADER_HDG) {
    // W = L u into I, then the TCK sweep in place on I (each workgroup reads
    // only its own cells before it writes them)
    OpParams w = op_params(m, B, nullptr);
    w.u = cur;
    w.out = I;
    DGW_HIP(run_op(m, EPI_STORE, w, s));
    tp.u = I;
    tp.u_base = cur;
    DGW_HIP(basis_launchers(m).tck_hdg[sel](tp, s));
  } else {
    DGW_HIP(basis_launchers(m).tck[period][sel](tp, s));
  }
  OpParams p = op_params(m, B, src);
  p.u = I;
  p.u_base = cur;
  p.u_next = oth;
  p.time = StepTime{ctr, t0, dt, step_add, 0.0};
  DGW_HIP(run_op(m, EPI_ADD, p, s));
  std::swap(cur, oth);
  return DGW_OK;
}

static dgw_status energy_impl(dgw_mesh* m, const double* u, int B, double* host_out, hipStream_t s) {
  EnergyParams p;
  std::memset(&p, 0, sizeof(p));
  p.u = u;
  p.geo_cell = m->d_cell;
  p.partial = m->d_partial;
  p.nc = m->hs.nc;
  p.cpw = std::max(1, std::min(16, 16384 / m->L->energy_lds_per_cell));
  p.groups = (int)((m->hs.nc + p.cpw - 1) / p.cpw);
  p.B = B;
  DGW_HIP(basis_launchers(m).energy(p, s));
  std::vector<double> part((size_t)B * p.groups);
  DGW_HIP(hipMemcpyAsync(part.data(), m->d_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  DGW_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b) {
    double acc = 0;
    for (int g = 0; g < p.groups; ++g) acc += part[(size_t)b * p.groups + g];
    host_out[b] = acc;
  }
  return DGW_OK;
}

// Autotuner of the launch shapes (cells per workgroup) of the operator, per
// epilogue, and of the TCK: each compiled candidate that fits the LDS is
// timed on scratch buffers of the mesh's size and batch, and the fastest is
// kept (the paper's throughput depends on how many cells are processed
// together, Sec. 4.4; the best choice here depends on k, d, precision, the
// epilogue's register use and the batch).  Results are kept per process and,
// when the environment variable DGW_AUTOTUNE_CACHE names a file, in that file
// as JSON lines keyed by device architecture, d, k, precision, storage basis,
// batch size and cell count, so that later processes skip the timing.
namespace {
struct TuneResult {
  int op[3] = {0, 0, 0};  // store, LSRK, ADER update
  int tck = 0;
};

std::string tune_key(const dgw_mesh* m, int B) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  return arch + "|d" + std::to_string(m->hs.dim) + "|k" + std::to_string(m->hs.k) +
         (m->precision == DGW_FP32_SPLIT ? "|fp32" : "|fp64") + (m->basis == DGW_BASIS_GAUSS ? "|gauss" : "|gl") +
         "|B" + std::to_string(B) + "|nc" + std::to_string(m->hs.nc);
}

// integer field `name` of one JSON line, -1 if absent
int json_int(const std::string& line, const char* name) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return -1;
  return std::atoi(line.c_str() + at + pat.size());
}

bool cache_file_lookup(const std::string& key, TuneResult& r) {
  const char* path = std::getenv("DGW_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char buf[1024];
  bool found = false;
  const std::string kpat = "\"key\":\"" + key + "\"";
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string line;
    for (const char* c = buf; *c; ++c)  // keys and values hold no blanks: drop them all
      if (*c != ' ' && *c != '\t') line += *c;
    if (line.find(kpat) == std::string::npos) continue;
    const int v[4] = {json_int(line, "op_store"), json_int(line, "op_lsrk"), json_int(line, "op_ader_update"),
                      json_int(line, "tck")};
    if (v[0] < 0 || v[0] > 3 || v[1] < 0 || v[1] > 3 || v[2] < 0 || v[2] > 3 || v[3] < 0 || v[3] > 1) continue;
    r.op[0] = v[0];
    r.op[1] = v[1];
    r.op[2] = v[2];
    r.tck = v[3];
    found = true;  // the last matching line wins
  }
  std::fclose(f);
  return found;
}

void cache_file_append(const std::string& key, const TuneResult& r, float (&ms)[4][4]) {
  const char* path = std::getenv("DGW_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  for (auto& row : ms)
    for (float& t : row)
      if (t >= 1e29f) t = -1.0f;  // not timed (does not fit, or no such variant)
  static std::mutex file_mtx;
  std::lock_guard<std::mutex> lk(file_mtx);
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\":\"%s\",\"op_store\":%d,\"op_lsrk\":%d,\"op_ader_update\":%d,\"tck\":%d,"
               "\"ms\":{\"op_store\":[%.4f,%.4f,%.4f,%.4f],\"op_lsrk\":[%.4f,%.4f,%.4f,%.4f],"
               "\"op_ader_update\":[%.4f,%.4f,%.4f,%.4f],\"tck\":[%.4f,%.4f]}}\n",
               key.c_str(), r.op[0], r.op[1], r.op[2], r.tck, ms[0][0], ms[0][1], ms[0][2], ms[0][3], ms[1][0],
               ms[1][1], ms[1][2], ms[1][3], ms[2][0], ms[2][1], ms[2][2], ms[2][3], ms[3][0], ms[3][1]);
  std::fclose(f);
}

void apply_tuning(dgw_mesh* m, const TuneResult& r) {
  for (int e = 0; e < 3; ++e) m->op_sel_epi[e] = r.op[e];
  m->op_shape.sel = r.op[EPI_STORE] & 1;
  m->tck_shape.sel = r.tck;
  m->tuned = true;
}
}  // namespace

static dgw_status autotune(dgw_mesh* m, int B, hipStream_t s) {
  static std::mutex cache_mtx;
  static std::map<std::string, TuneResult> cache;
  const std::string key = tune_key(m, B);
  {
    std::lock_guard<std::mutex> lk(cache_mtx);
    auto it = cache.find(key);
    TuneResult r;
    if (it != cache.end() || cache_file_lookup(key, r)) {
      if (it != cache.end()) r = it->second;
      bool fits = (int64_t)m->L->cpw[r.tck] * m->L->tck_lds_per_cell[2] <= kLdsLimit;
      for (int e = 0; e < 3; ++e)
        fits = fits && (int64_t)m->L->cpw[r.op[e] & 1] * m->L->op_lds_per_cell <= kLdsLimit &&
               op_launch(m, e, r.op[e]) != nullptr;
      if (fits) {
        cache[key] = r;
        apply_tuning(m, r);
        return DGW_OK;
      }
    }
  }
  const int64_t ne = state_elems(m) * B;
  double* buf[3] = {nullptr, nullptr, nullptr};
  for (auto*& b : buf)
    if (hipMalloc(&b, ne * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      for (auto* q : buf) (void)hipFree(q);
      return fail(DGW_ENOMEM, "autotune scratch");
    }
  for (auto* b : buf) DGW_HIP(hipMemsetAsync(b, 0, ne * sizeof(double), s));
  hipEvent_t e0, e1;
  DGW_HIP(hipEventCreate(&e0));
  DGW_HIP(hipEventCreate(&e1));
  float ms[4][4] = {{1e30f, 1e30f, 1e30f, 1e30f}, {1e30f, 1e30f, 1e30f, 1e30f}, {1e30f, 1e30f, 1e30f, 1e30f},
                    {1e30f, 1e30f, 1e30f, 1e30f}};
  // every candidate (kernel, shape) with the slot of its time
  struct Cand {
    float* slot;
    std::function<hipError_t()> launch;
    bool ok;
  };
  std::vector<Cand> cands;
  const bool gauss = m->basis == DGW_BASIS_GAUSS;
  const int nshape = B > 1 && !gauss ? 4 : 2;  // member blocks only pay with more than one member
  for (int shape = 0; shape < nshape; ++shape) {
    const int sel = shape & 1;
    if ((int64_t)m->L->cpw[sel] * m->L->op_lds_per_cell <= kLdsLimit) {
      for (int epi = 0; epi < 3; ++epi) {
        if (!op_launch(m, epi, shape)) continue;
        OpParams p = op_params(m, B, nullptr);
        p.u = buf[0];
        if (epi == EPI_STORE) {
          p.out = buf[1];
        } else if (epi == EPI_LSRK) {
          p.du = buf[2];
          p.u_next = buf[1];
          p.dt = 1e-3;
          set_lsrk_stage(p, DGW_SCHEME_LSRK54, 1, 1e-3);  // a stage that reads du
        } else {
          p.u_base = buf[2];
          p.u_next = buf[1];
          p.dt = 1e-3;
        }
        cands.push_back({&ms[epi][shape], [=]() { return run_op(m, epi, shape, p, s); }, true});
      }
    }
    if (shape < 2 && (int64_t)m->L->cpw[sel] * m->L->tck_lds_per_cell[2] <= kLdsLimit) {
      TckParams p = tck_params(m, B, nullptr);
      p.cpw = m->L->cpw[sel];
      p.groups = (int)((m->hs.nc + p.cpw - 1) / p.cpw);
      p.u = buf[0];
      p.I = buf[1];
      p.dt = 1e-3;
      cands.push_back({&ms[3][sel], [=]() { return basis_launchers(m).tck[2][sel](p, s); }, true});
    }
  }
  // round robin over the candidates, keeping each one's fastest round: a
  // clock ramp or a noisy neighbour then does not favour whichever shape
  // happens to be timed last
  constexpr int kRounds = 3, kLaunches = 3;
  for (int round = 0; round < kRounds; ++round)
    for (auto& c : cands) {
      if (round == 0) c.ok = c.launch() == hipSuccess;  // warm-up
      if (!c.ok) continue;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < kLaunches; ++r) (void)c.launch();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float t = 0;
      (void)hipEventElapsedTime(&t, e0, e1);
      *c.slot = std::min(*c.slot, t / kLaunches);
    }
  (void)hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (auto* b : buf) (void)hipFree(b);
  TuneResult r;
  for (int e = 0; e < 3; ++e)
    for (int sh = 1; sh < 4; ++sh)
      if (ms[e][sh] < ms[e][r.op[e]]) r.op[e] = sh;
  r.tck = ms[3][1] < ms[3][0] ? 1 : 0;
  apply_tuning(m, r);
  std::lock_guard<std::mutex> lk(cache_mtx);
  cache[key] = r;
  cache_file_append(key, r, ms);
  return DGW_OK;
}

static dgw_status upload(dgw_mesh* m) {
  auto& hs = m->hs;
  auto alloc_copy = [&](auto*& dst, const auto* src, size_t count) -> dgw_status {
    using E = std::remove_pointer_t<std::remove_reference_t<decltype(dst)>>;
    const size_t bytes = count * sizeof(E);
    if (hipMalloc(reinterpret_cast<void**>(&dst), std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      dst = nullptr;
      return fail(DGW_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    m->device_bytes += bytes;
    if (bytes) DGW_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return DGW_OK;
  };
  dgw_status st;
  if ((st = alloc_copy(m->d_cell, hs.cell.data(), hs.cell.size()))) return st;
  if ((st = alloc_copy(m->d_face, hs.face.data(), hs.face.size()))) return st;
  {
    // device neighbour table: a prescribed face carries kBcPrescribed - slot
    std::vector<int32_t> nbd(hs.nb);
    std::vector<int64_t> pfaces;
    for (size_t i = 0; i < nbd.size(); ++i)
      if (nbd[i] == kBcPrescribed) {
        nbd[i] = kBcPrescribed - (int32_t)pfaces.size();
        pfaces.push_back((int64_t)i);
      }
    if ((st = alloc_copy(m->d_nb, nbd.data(), nbd.size()))) return st;
    m->n_pslots = (int64_t)pfaces.size();
    if (!pfaces.empty()) {
      const int d = hs.dim, nf = m->nf;
      std::vector<double> bxp((size_t)pfaces.size() * d * nf);
      for (size_t j = 0; j < pfaces.size(); ++j)
        std::copy(hs.face_x.begin() + (size_t)pfaces[j] * d * nf, hs.face_x.begin() + (size_t)(pfaces[j] + 1) * d * nf,
                  bxp.begin() + j * d * nf);
      if ((st = alloc_copy(m->d_pfaces, pfaces.data(), pfaces.size()))) return st;
      if ((st = alloc_copy(m->d_bx, bxp.data(), bxp.size()))) return st;
      if ((st = alloc_copy(m->d_waves, hs.waves.data(), hs.waves.size()))) return st;
      std::vector<double> zeros((size_t)pfaces.size() * 2 * nf, 0.0);
      if ((st = alloc_copy(m->d_ext, zeros.data(), zeros.size()))) return st;
    }
  }
  if (!hs.fo.empty() && (st = alloc_copy(m->d_fo, hs.fo.data(), hs.fo.size()))) return st;
  for (int l = 1; l < m->nlev; ++l)
    if ((st = alloc_copy(m->d_level[l], hs.level[l].data(), hs.level[l].size()))) return st;
  if ((st = ensure_tables(m->device))) return st;
  const int cpw_e = std::max(1, std::min(16, 16384 / m->L->energy_lds_per_cell));
  const size_t groups_e = (size_t)((hs.nc + cpw_e - 1) / cpw_e);
  std::vector<double> zeros((size_t)m->max_batch * groups_e, 0.0);
  if ((st = alloc_copy(m->d_partial, zeros.data(), zeros.size()))) return st;
  return DGW_OK;
}

static void release(dgw_mesh* m) {
  if (!m) return;
  if (m->device >= 0) {
    (void)hipSetDevice(m->device);
    (void)hipFree(m->d_cell);
    (void)hipFree(m->d_face);
    (void)hipFree(m->d_nb);
    (void)hipFree(m->d_fo);
    (void)hipFree(m->d_pfaces);
    (void)hipFree(m->d_bx);
    (void)hipFree(m->d_waves);
    (void)hipFree(m->d_ext);
    for (auto* p : m->d_level) (void)hipFree(p);
    for (auto* p : m->d_level_pts) (void)hipFree(p);
    (void)hipFree(m->d_partial);
  }
  delete m;
}

}  // namespace dgw

using namespace dgw;

extern "C" {

const char* dgw_last_error(void) { return g_last_error.c_str(); }
const char* dgw_version(void) { return "dgw 0.1 (gfx950)"; }

dgw_status dgw_basis_1d(int n, int what, double* out) {
  if (n < 1 || n > 9 || !out) return fail(DGW_EINVAL, "n must be in 1..9");
  const Rule g = gauss_rule(n);
  switch (what) {
    case 0:
    case 1:
      for (int i = 0; i < n; ++i) out[i] = (double)(what == 0 ? g.x[i] : g.w[i]);
      return DGW_OK;
    case 2:
    case 3: {
      if (n < 2) return fail(DGW_EINVAL, "Gauss-Lobatto needs n >= 2");
      const Rule gl = gauss_lobatto_rule(n);
      for (int i = 0; i < n; ++i) out[i] = (double)(what == 2 ? gl.x[i] : gl.w[i]);
      return DGW_OK;
    }
    case 4:
    case 5:
    case 6: {
      if (n < 2) return fail(DGW_EINVAL, "n >= 2 needed");
      const std::vector<double> t = build_tables(n);
      const int off = what == 4 ? tab_S(n) : (what == 5 ? tab_Sinv(n) : tab_D(n));
      std::copy(t.begin() + off, t.begin() + off + n * n, out);
      return DGW_OK;
    }
  }
  return fail(DGW_EINVAL, "unknown table");
}

dgw_status dgw_lsrk_coefficients(int scheme, double* out) {
  if (!out) return fail(DGW_EINVAL, "out is NULL");
  if (scheme == DGW_SCHEME_LSRK54) {
    for (int i = 0; i < 5; ++i) {
      out[i] = kLsrk.A[i];
      out[5 + i] = kLsrk.B[i];
      out[10 + i] = kLsrk.C[i];
    }
    return DGW_OK;
  }
  if (scheme == DGW_SCHEME_LSRK59) {
    if (!kLsrk59.ok) return fail(DGW_EDEVICE, "LSRK5(9) coefficients did not converge");
    for (int i = 0; i < 8; ++i) out[i] = kLsrk59.alpha[i];
    for (int i = 0; i < 9; ++i) {
      out[8 + i] = kLsrk59.b[i];
      out[17 + i] = kLsrk59.c[i];
    }
    return DGW_OK;
  }
  return fail(DGW_EINVAL, "scheme has no Runge-Kutta coefficients");
}

dgw_status dgw_mesh_create(const dgw_mesh_desc* desc, dgw_mesh** out) {
  if (!out) return fail(DGW_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(DGW_EINVAL, "desc is NULL");
  if (desc->dim != 2 && desc->dim != 3) return fail(DGW_EUNSUPPORTED, "dim must be 2 or 3");
  if (desc->degree < 1 || desc->degree > 8) return fail(DGW_EUNSUPPORTED, "degree must be in 1..8");
  if (desc->n_cells < 1) return fail(DGW_EINVAL, "n_cells must be >= 1");
  if (!desc->geo_nodes || !desc->neighbors || !desc->material)
    return fail(DGW_EINVAL, "geo_nodes, neighbors and material are required");
  if (desc->flux != DGW_FLUX_UPWIND && desc->flux != DGW_FLUX_CENTRAL) return fail(DGW_EINVAL, "bad flux");
  if (desc->precision != DGW_FP64 && desc->precision != DGW_FP32_SPLIT) return fail(DGW_EINVAL, "bad precision");
  if (desc->max_batch < 1) return fail(DGW_EINVAL, "max_batch must be >= 1");
  if (desc->n_cells > (int64_t)1 << 30) return fail(DGW_EUNSUPPORTED, "too many cells");
  if (desc->storage_basis != DGW_BASIS_GL && desc->storage_basis != DGW_BASIS_GAUSS)
    return fail(DGW_EINVAL, "storage_basis must be DGW_BASIS_GL or DGW_BASIS_GAUSS");
  std::unique_ptr<dgw_mesh> m(new (std::nothrow) dgw_mesh);
  if (!m) return fail(DGW_ENOMEM, "host allocation");
  m->precision = desc->precision;
  m->flux = desc->flux;
  m->device = desc->device;
  m->max_batch = desc->max_batch;
  m->basis = desc->storage_basis;
  const int n = desc->degree + 1;
  m->np = ipw(n, desc->dim);
  m->nf = ipw(n, desc->dim - 1);
  m->ncomp = desc->dim + 1;
  m->nlev = num_levels(n);
  for (int l = 0; l < m->nlev; ++l) m->level_pts.push_back(n - 2 * l);
  m->L = launchers(desc->dim, n, desc->precision);
  if (!m->L) return fail(DGW_EUNSUPPORTED, "no kernels for this dim/degree");
  try {
    dgw_status st = build_setup(*desc, m->hs);
    if (st) return st;
  } catch (const std::bad_alloc&) {
    return fail(DGW_ENOMEM, "host allocation during setup");
  }
  m->op_shape = default_shape(m->L, m->L->op_lds_per_cell);
  m->tck_shape = default_shape(m->L, m->L->tck_lds_per_cell[2]);
  if (m->device >= 0) {
    if (hipSetDevice(m->device) != hipSuccess) return fail(DGW_EDEVICE, "hipSetDevice failed");
    dgw_status st = upload(m.get());
    if (st) {
      release(m.release());
      return st;
    }
    // the host copy of the bulk geometry is not needed once uploaded
    std::vector<double>().swap(m->hs.cell);
    std::vector<double>().swap(m->hs.face);
    std::vector<double>().swap(m->hs.face_x);
    for (auto& v : m->hs.level) std::vector<double>().swap(v);
  }
  *out = m.release();
  return DGW_OK;
}

void dgw_mesh_destroy(dgw_mesh* mesh) { release(mesh); }

dgw_status dgw_mesh_info_get(const dgw_mesh* m, dgw_mesh_info* info) {
  if (!m || !info) return fail(DGW_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->dim = m->hs.dim;
  info->degree = m->hs.k;
  info->n1d = m->hs.n;
  info->nodes_per_cell = m->np;
  info->n_comp = m->ncomp;
  info->geo_degree = m->hs.q;
  info->n_cells = m->hs.nc;
  info->dofs = state_elems(m);
  info->state_bytes = info->dofs * 8;
  info->lsrk_work_bytes = 2 * info->state_bytes;
  info->ader_work_bytes = 2 * info->state_bytes;
  info->device_bytes = m->device_bytes;
  info->n_levels = m->nlev;
  for (int l = 0; l < m->nlev && l < 8; ++l) info->level_points[l] = m->level_pts[l];
  info->h_min = m->hs.h_min;
  info->c_max = m->hs.c_max;
  info->dt_unit = m->hs.dt_unit;
  info->precision = m->precision;
  info->flux = m->flux;
  info->max_batch = m->max_batch;
  info->device = m->device;
  return DGW_OK;
}

dgw_status dgw_mesh_get(const dgw_mesh* m, int what, double* host_out, int64_t count) {
  if (!m || !host_out) return fail(DGW_EINVAL, "NULL argument");
  const auto& hs = m->hs;
  const int d = hs.dim;
  auto fetch = [&](const std::vector<double>& h, const double* dev, size_t n) -> dgw_status {
    if ((int64_t)n != count) return fail(DGW_EINVAL, "count must be " + std::to_string(n));
    if (!h.empty()) {
      std::copy(h.begin(), h.end(), host_out);
      return DGW_OK;
    }
    if (!dev) return fail(DGW_EINVAL, "no such data");
    DGW_HIP(hipSetDevice(m->device));
    DGW_HIP(hipMemcpy(host_out, dev, n * sizeof(double), hipMemcpyDeviceToHost));
    return DGW_OK;
  };
  if (what == DGW_GET_NODE_COORDS) {
    std::vector<double> x;
    node_coords(hs, x);
    if ((int64_t)x.size() != count) return fail(DGW_EINVAL, "count must be " + std::to_string(x.size()));
    std::copy(x.begin(), x.end(), host_out);
    return DGW_OK;
  }
  if (what == DGW_GET_CELL_METRIC) return fetch(hs.cell, m->d_cell, (size_t)hs.nc * (d * d + 2) * m->np);
  if (what == DGW_GET_FACE) return fetch(hs.face, m->d_face, (size_t)hs.nc * 2 * d * (d + 2) * m->nf);
  if (what > DGW_GET_LEVEL0 && what < DGW_GET_LEVEL0 + m->nlev) {
    const int l = what - DGW_GET_LEVEL0;
    const size_t sz = (size_t)hs.nc * (d * d + 2) * ipw(m->level_pts[l], d);
    return fetch(l < (int)hs.level.size() ? hs.level[l] : std::vector<double>(), m->d_level[l], sz);
  }
  return fail(DGW_EINVAL, "unknown item");
}

dgw_status dgw_operator_apply(dgw_mesh* m, const double* u, double* out, int B, void* stream) {
  dgw_status st = check_mesh(m);
  if (st) return st;
  if (!u || !out) return fail(DGW_EINVAL, "NULL state pointer");
  if ((st = check_batch(m, B, nullptr))) return st;
  const int64_t bytes = state_elems(m) * 8 * B;
  if ((const char*)u < (const char*)out + bytes && (const char*)out < (const char*)u + bytes)
    return fail(DGW_EINVAL, "u and out must not alias");
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  OpParams p = op_params(m, B, nullptr);
  p.u = u;
  p.out = out;
  DGW_HIP(run_op(m, EPI_STORE, p, (hipStream_t)stream));
  return DGW_OK;
}

static dgw_status check_step(dgw_mesh* m, double dt, int nsteps, double* u, double* work, int B,
                             const dgw_sources* src) {
  dgw_status st = check_mesh(m);
  if (st) return st;
  if (!u || !work) return fail(DGW_EINVAL, "NULL state or work pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DGW_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return fail(DGW_EINVAL, "nsteps must be >= 0");
  if ((st = check_batch(m, B, src))) return st;
  const int64_t bytes = state_elems(m) * 8 * B;
  if ((char*)u < (char*)work + 2 * bytes && (char*)work < (char*)u + bytes)
    return fail(DGW_EINVAL, "u and work must not alias");
  return DGW_OK;
}

dgw_status dgw_step_lsrk(dgw_mesh* m, int scheme, double t0, double dt, int nsteps, double* u, double* work,
                         int B, const dgw_sources* src, void* stream) {
  if (scheme != DGW_SCHEME_LSRK54 && scheme != DGW_SCHEME_LSRK54_MERGED_VU &&
      scheme != DGW_SCHEME_LSRK54_STANDARD_VU && scheme != DGW_SCHEME_LSRK59)
    return fail(DGW_EUNSUPPORTED, "scheme must be one of the DGW_SCHEME_LSRK54 variants or DGW_SCHEME_LSRK59");
  if (scheme == DGW_SCHEME_LSRK59 && !kLsrk59.ok) return fail(DGW_EDEVICE, "LSRK5(9) coefficients did not converge");
  const bool fused = scheme == DGW_SCHEME_LSRK54 || scheme == DGW_SCHEME_LSRK59;
  if (!fused && src) return fail(DGW_EUNSUPPORTED, "the unfused LSRK variants take no sources");
  dgw_status st = check_step(m, dt, nsteps, u, work, B, src);
  if (st) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  hipStream_t s = (hipStream_t)stream;
  if (!fused) {
    // operator sweep stores r = L u into the second work register; the
    // vector update then advances u in place
    double* du = work;
    double* r = work + state_elems(m) * B;
    OpParams p = op_params(m, B, nullptr);
    p.u = u;
    p.out = r;
    for (int k = 0; k < nsteps; ++k)
      for (int i = 0; i < 5; ++i) {
        p.time = StepTime{nullptr, t0, dt, k, kLsrk.C[i] * dt};  // prescribed data at the stage time
        DGW_HIP(run_op(m, EPI_STORE, p, s));
        if ((st = lsrk_vector_update(scheme, i, dt, u, du, r, state_elems(m) * B, s))) return st;
      }
    return DGW_OK;
  }
  double* du = work;
  double* cur = u;
  double* oth = work + state_elems(m) * B;
  for (int k = 0; k < nsteps; ++k)
    if ((st = lsrk_step(m, B, src, t0, dt, k, nullptr, cur, oth, du, s, scheme))) return st;
  if (cur != u) DGW_HIP(hipMemcpyAsync(u, cur, state_elems(m) * 8 * B, hipMemcpyDeviceToDevice, s));
  return DGW_OK;
}

dgw_status dgw_step_ader(dgw_mesh* m, int flags, double t0, double dt, int nsteps, double* u, double* work, int B,
                         const dgw_sources* src, void* stream) {
  dgw_status st = check_ader_flags(flags, src);
  if (st) return st;
  if ((st = check_step(m, dt, nsteps, u, work, B, src))) return st;
  if ((st = check_hdg_faces(m, flags))) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  if ((st = ensure_period_levels(m, ader_period(flags)))) return st;
  hipStream_t s = (hipStream_t)stream;
  double* I = work;
  double* cur = u;
  double* oth = work + state_elems(m) * B;
  for (int k = 0; k < nsteps; ++k)
    if ((st = ader_step(m, flags, B, src, t0, dt, k, nullptr, cur, oth, I, s))) return st;
  if (cur != u) DGW_HIP(hipMemcpyAsync(u, cur, state_elems(m) * 8 * B, hipMemcpyDeviceToDevice, s));
  return DGW_OK;
}

// ------------------------------------------------------- no-alloc ADER step
// Work registers of dgw_step_ader_noalloc (the TCK sum I and the ping-pong
// state of every member) in a static device array: each device that runs the
// call holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel: its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static constexpr int64_t kNoAllocScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / 8];

static dgw_status scratch_address(int device, double** out) {
  static std::mutex mtx;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lk(mtx);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DGW_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = addr.emplace(device, static_cast<double*>(p)).first;
  }
  *out = it->second;
  return DGW_OK;
}

static bool period_levels_ready(const dgw_mesh* m, int period) {
  for (int l = 1; l < num_levels_r(m->hs.n, period); ++l)
    if (!level_metric(m, m->hs.n - period * l)) return false;
  return true;
}

dgw_status dgw_step_ader_noalloc(dgw_mesh* m, int flags, double t0, double dt, int nsteps, double* u, int B,
                                 const dgw_sources* src, void* stream) {
  dgw_status st = check_ader_flags(flags, src);
  if (st) return st;
  if ((st = check_mesh(m))) return st;
  if (!u) return fail(DGW_EINVAL, "NULL state pointer");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DGW_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return fail(DGW_EINVAL, "nsteps must be >= 0");
  if ((st = check_batch(m, B, src))) return st;
  if ((st = check_hdg_faces(m, flags))) return st;
  const int64_t ne = state_elems(m) * B;
  if (2 * ne * (int64_t)sizeof(double) > kNoAllocScratchBytes)
    return fail(DGW_EINVAL, "dgw_step_ader_noalloc: 2 * B * state bytes = " +
                                std::to_string(2 * ne * (int64_t)sizeof(double)) + " exceed the " +
                                std::to_string(kNoAllocScratchBytes) + "-byte device scratch");
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  if (!period_levels_ready(m, ader_period(flags)))
    return fail(DGW_EUNSUPPORTED, "the reduced levels of this reduction period are not built yet "
                                  "(one dgw_step_ader call with these flags builds them)");
  double* base = nullptr;
  if ((st = scratch_address(m->device, &base))) return st;
  hipStream_t s = (hipStream_t)stream;
  double* I = base;
  double* cur = u;
  double* oth = base + ne;
  for (int k = 0; k < nsteps; ++k)
    if ((st = ader_step(m, flags, B, src, t0, dt, k, nullptr, cur, oth, I, s))) return st;
  if (cur != u) DGW_HIP(hipMemcpyAsync(u, cur, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DGW_OK;
}

dgw_status dgw_step_profile(dgw_mesh* m, int scheme, int flags, double t0, double dt, int nsteps, double* u,
                            double* work, int B, const dgw_sources* src, void* stream, dgw_profile* out) {
  if (!out) return fail(DGW_EINVAL, "out is NULL");
  const bool unfused = scheme == DGW_SCHEME_LSRK54_MERGED_VU || scheme == DGW_SCHEME_LSRK54_STANDARD_VU;
  if (scheme != DGW_SCHEME_LSRK54 && scheme != DGW_SCHEME_LSRK59 && scheme != DGW_SCHEME_ADER && !unfused)
    return fail(DGW_EINVAL, "bad scheme");
  if (unfused && src) return fail(DGW_EUNSUPPORTED, "the unfused LSRK variants take no sources");
  const bool hdg = scheme == DGW_SCHEME_ADER && (flags & DGW_ADER_HDG);
  if (scheme == DGW_SCHEME_ADER) {
    dgw_status fs = check_ader_flags(flags, src);
    if (fs) return fs;
  }
  dgw_status st = check_step(m, dt, nsteps, u, work, B, src);
  if (st) return st;
  if (scheme == DGW_SCHEME_ADER && (st = check_hdg_faces(m, flags))) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  if (scheme == DGW_SCHEME_ADER && (st = ensure_period_levels(m, ader_period(flags)))) return st;
  hipStream_t s = (hipStream_t)stream;
  std::memset(out, 0, sizeof(*out));
  const char* names[3] = {"operator_lsrk", nullptr, nullptr};
  if (scheme == DGW_SCHEME_ADER) names[0] = "tck", names[1] = "operator_ader_update";
  if (hdg) names[2] = "operator_store";
  if (unfused) names[0] = "operator_store", names[1] = "vector_update";
  out->n = names[2] ? 3 : (names[1] ? 2 : 1);
  for (int c = 0; c < out->n; ++c) std::snprintf(out->names[c], 32, "%s", names[c]);
  // (component, start event, end event) of every timed launch group
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> rec;
  auto timed = [&](int c, auto&& launch) -> dgw_status {
    hipEvent_t a, b;
    DGW_HIP(hipEventCreate(&a));
    DGW_HIP(hipEventCreate(&b));
    rec.push_back({c, {a, b}});
    DGW_HIP(hipEventRecord(a, s));
    dgw_status e = launch();
    if (e) return e;
    DGW_HIP(hipEventRecord(b, s));
    return DGW_OK;
  };
  double* cur = u;
  double* oth = work + state_elems(m) * B;
  double* aux = work;
  for (int k = 0; k < nsteps && !st; ++k) {
    if (unfused) {
      OpParams p = op_params(m, B, nullptr);
      p.u = u;
      p.out = oth;
      for (int i = 0; i < 5 && !st; ++i) {
        p.time = StepTime{nullptr, t0, dt, k, kLsrk.C[i] * dt};
        st = timed(0, [&]() -> dgw_status {
          DGW_HIP(run_op(m, EPI_STORE, p, s));
          return DGW_OK;
        });
        if (!st) st = timed(1, [&] { return lsrk_vector_update(scheme, i, dt, u, aux, oth, state_elems(m) * B, s); });
      }
    } else if (scheme == DGW_SCHEME_LSRK54 || scheme == DGW_SCHEME_LSRK59) {
      OpParams p = op_params(m, B, src);
      p.dt = dt;
      p.du = aux;
      p.time = StepTime{nullptr, t0, dt, k, 0.0};
      for (int i = 0; i < lsrk_stages(scheme) && !st; ++i) {
        p.u = cur;
        p.u_next = oth;
        set_lsrk_stage(p, scheme, i, dt);
        st = timed(0, [&]() -> dgw_status {
          DGW_HIP(run_op(m, EPI_LSRK, p, s));
          return DGW_OK;
        });
        std::swap(cur, oth);
      }
    } else {
      const int period = ader_period(flags);
      const int sel = tck_sel(m, period);
      TckParams tp = tck_params(m, B, src, period);
      tp.cpw = m->L->cpw[sel];
      tp.groups = (int)((m->hs.nc + tp.cpw - 1) / tp.cpw);
      tp.u = cur;
      tp.I = aux;
      tp.dt = dt;
      tp.time = StepTime{nullptr, t0, dt, k, 0.0};
      if (hdg) {
        OpParams w = op_params(m, B, nullptr);
        w.u = cur;
        w.out = aux;
        st = timed(2, [&]() -> dgw_status {
          DGW_HIP(run_op(m, EPI_STORE, w, s));
          return DGW_OK;
        });
        tp.u = aux;
        tp.u_base = cur;
      }
      if (!st)
        st = timed(0, [&]() -> dgw_status {
          if (hdg)
            DGW_HIP(basis_launchers(m).tck_hdg[sel](tp, s));
          else
            DGW_HIP(basis_launchers(m).tck[period][sel](tp, s));
          return DGW_OK;
        });
      OpParams p = op_params(m, B, src);
      p.u = aux;
      p.u_base = cur;
      p.u_next = oth;
      p.time = StepTime{nullptr, t0, dt, k, 0.0};
      if (!st)
        st = timed(1, [&]() -> dgw_status {
          DGW_HIP(run_op(m, EPI_ADD, p, s));
          return DGW_OK;
        });
      std::swap(cur, oth);
    }
  }
  if (!st && hipStreamSynchronize(s) != hipSuccess) st = fail(DGW_EDEVICE, "stream synchronize failed");
  for (auto& r : rec) {
    float ms = 0;
    if (!st && hipEventElapsedTime(&ms, r.second.first, r.second.second) == hipSuccess) {
      out->ms[r.first] += ms;
      out->launches[r.first] += 1;
    }
    (void)hipEventDestroy(r.second.first);
    (void)hipEventDestroy(r.second.second);
  }
  if (st) return st;
  for (int c = 0; c < out->n; ++c)
    if (out->launches[c]) out->ms[c] /= (double)out->launches[c];
  if (cur != u) DGW_HIP(hipMemcpyAsync(u, cur, state_elems(m) * 8 * B, hipMemcpyDeviceToDevice, s));
  DGW_HIP(hipStreamSynchronize(s));
  return DGW_OK;
}

dgw_status dgw_autotune(dgw_mesh* m, int B, void* stream) {
  dgw_status st = check_mesh(m);
  if (st) return st;
  if ((st = check_batch(m, B, nullptr))) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  return autotune(m, B, (hipStream_t)stream);
}

dgw_status dgw_launch_shape(dgw_mesh* m, int which, int* cells_per_group, int* threads) {
  if (!m || !cells_per_group || !threads || which < 0 || which > 6) return fail(DGW_EINVAL, "bad argument");
  if (which >= 4) {  // batch members per workgroup of the store (4), LSRK (5), ADER update (6) operator
    if (*cells_per_group > 0) return fail(DGW_EINVAL, "which = 4..6 only report a member count");
    *cells_per_group = (op_sel(m, which - 4) & 2) ? kMemberBlock : 1;
    *threads = op_threads(m->hs.dim, m->hs.n);
    return DGW_OK;
  }
  if (which >= 2) {  // read the shape of the LSRK (2) or ADER update (3) epilogue
    if (*cells_per_group > 0) return fail(DGW_EINVAL, "which = 2, 3 only report a shape");
    *cells_per_group = m->L->cpw[op_sel(m, which == 2 ? EPI_LSRK : EPI_ADD) & 1];
    *threads = op_threads(m->hs.dim, m->hs.n);
    return DGW_OK;
  }
  LaunchShape& sh = which == 0 ? m->op_shape : m->tck_shape;
  if (*cells_per_group > 0) {
    const int per_cell = which == 0 ? m->L->op_lds_per_cell : m->L->tck_lds_per_cell[2];
    int sel = -1;
    for (int c = 0; c < 2; ++c)
      if (m->L->cpw[c] == *cells_per_group && (int64_t)m->L->cpw[c] * per_cell <= kLdsLimit) sel = c;
    const int nt = which == 0 ? op_threads(m->hs.dim, m->hs.n) : tck_threads(m->hs.dim, m->hs.n);
    if (sel < 0 || (*threads > 0 && *threads != nt))
      return fail(DGW_EINVAL, "cells_per_group must be one of the compiled shapes (" + std::to_string(m->L->cpw[0]) +
                                  ", " + std::to_string(m->L->cpw[1]) + ") and fit the LDS; threads must be " +
                                  std::to_string(nt));
    sh.sel = sel;
    if (which == 0)
      for (int e = 0; e < 3; ++e) m->op_sel_epi[e] = -1;  // every epilogue takes this shape
  }
  *cells_per_group = m->L->cpw[sh.sel];
  *threads = which == 0 ? op_threads(m->hs.dim, m->hs.n) : tck_threads(m->hs.dim, m->hs.n);
  return DGW_OK;
}

dgw_status dgw_energy(dgw_mesh* m, const double* u, int B, double* host_out, void* stream) {
  dgw_status st = check_mesh(m);
  if (st) return st;
  if (!u || !host_out) return fail(DGW_EINVAL, "NULL argument");
  if ((st = check_batch(m, B, nullptr))) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  return energy_impl(m, u, B, host_out, (hipStream_t)stream);
}

// ---------------------------------------------------------------- sources
dgw_status dgw_sources_create(dgw_mesh* m, const dgw_source_desc* desc, dgw_sources** out) {
  if (!out) return fail(DGW_EINVAL, "out is NULL");
  *out = nullptr;
  dgw_status st = check_mesh(m);
  if (st) return st;
  if (!desc || desc->n < 1 || !desc->position || !desc->frequency) return fail(DGW_EINVAL, "bad source desc");
  const auto& hs = m->hs;
  const int d = hs.dim, n = hs.n, np = m->np, ng = ipw(hs.q + 1, d);
  std::unique_ptr<dgw_sources> S(new dgw_sources);
  S->mesh = m;
  S->n = desc->n;
  // bounding boxes of the geometry nodes (with a margin for curved faces)
  std::vector<double> lo((size_t)hs.nc * d), hi((size_t)hs.nc * d);
  for (int64_t c = 0; c < hs.nc; ++c)
    for (int a = 0; a < d; ++a) {
      double mn = 1e300, mx = -1e300;
      for (int g = 0; g < ng; ++g) {
        const double v = hs.geo_nodes[(c * ng + g) * d + a];
        mn = std::min(mn, v);
        mx = std::max(mx, v);
      }
      const double pad = 0.1 * (mx - mn) + 1e-12;
      lo[c * d + a] = mn - pad;
      hi[c * d + a] = mx + pad;
    }
  const Rule g = gauss_rule(n);
  const std::vector<double> tab = build_tables(n);
  std::vector<double> gvec((size_t)S->n * np), wave((size_t)S->n * 3);
  std::vector<std::vector<double>> glev(m->nlev);
  for (int l = 0; l < m->nlev; ++l) glev[l].assign((size_t)S->n * ipw(m->level_pts[l], d), 0.0);
  S->cell.resize(S->n);
  std::vector<double> mu(np);
  for (int i = 0; i < S->n; ++i) {
    const double* xs = desc->position + (size_t)i * d;
    int64_t found = -1;
    double xi[3] = {0.5, 0.5, 0.5};
    for (int64_t c = 0; c < hs.nc && found < 0; ++c) {
      bool in = true;
      for (int a = 0; a < d; ++a) in = in && xs[a] >= lo[c * d + a] && xs[a] <= hi[c * d + a];
      if (!in) continue;
      double z[3] = {0.5, 0.5, 0.5};
      bool ok = false;
      for (int it = 0; it < 50; ++it) {
        double x[3], J[9], Ji[9], r[3];
        map_point(hs, c, z, x, J);
        double err = 0;
        for (int a = 0; a < d; ++a) {
          r[a] = x[a] - xs[a];
          err = std::max(err, std::fabs(r[a]));
        }
        if (err < 1e-12) {
          ok = true;
          break;
        }
        // z -= J^-1 r
        if (d == 2) {
          const double det = J[0] * J[3] - J[1] * J[2];
          Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
        } else {
          const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
          const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
          Ji[0] = c00 / det; Ji[3] = c01 / det; Ji[6] = c02 / det;
          Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det; Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
          Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det; Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
          Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det; Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
        }
        bool far = false;
        for (int a = 0; a < d; ++a) {
          double s = 0;
          for (int b = 0; b < d; ++b) s += Ji[a * d + b] * r[b];
          z[a] -= s;
          far = far || std::fabs(z[a] - 0.5) > 2.0;
        }
        if (far) break;
      }
      bool inside = ok;
      for (int a = 0; a < d; ++a) inside = inside && z[a] >= -1e-10 && z[a] <= 1 + 1e-10;
      if (inside) {
        found = c;
        for (int a = 0; a < d; ++a) xi[a] = std::min(1.0, std::max(0.0, z[a]));
      }
    }
    if (found < 0) return fail(DGW_EINVAL, "source " + std::to_string(i) + " is outside the mesh");
    S->cell[i] = (int)found;
    double x[3], J[9];
    map_point(hs, found, xi, x, J);
    double rho, c;
    hs.material(x, 1, d, &rho, &c, hs.material_ctx);
    // mu_p of the source cell (from the device copy of the metric)
    DGW_HIP(hipSetDevice(m->device));
    DGW_HIP(hipMemcpy(mu.data(), m->d_cell + ((size_t)found * (d * d + 2) + d * d + 1) * np, np * sizeof(double),
                      hipMemcpyDeviceToHost));
    // g in the collocated basis: mu_p * l^G(xi_s) / (rho c^2); then S^-1 to
    // GL unless the state is stored at the Gauss points
    std::vector<double> lg((size_t)d * n);
    for (int a = 0; a < d; ++a)
      for (int j = 0; j < n; ++j) lg[a * n + j] = (double)lagrange_value(g.x, j, (long double)xi[a]);
    std::vector<double> gG(np), tmp(np);
    for (int qq = 0; qq < np; ++qq) {
      int t = qq;
      double v = 1.0;
      for (int a = 0; a < d; ++a) {
        v *= lg[a * n + t % n];
        t /= n;
      }
      gG[qq] = mu[qq] * v / (rho * c * c);
    }
    // apply a 1D matrix along every direction (host, small)
    auto apply = [&](const std::vector<double>& in, int mi, const double* M, int mo) {
      std::vector<double> cur = in;
      int ext[3] = {mi, mi, d == 3 ? mi : 1};
      for (int e = 0; e < d; ++e) {
        int eo[3] = {ext[0], ext[1], ext[2]};
        eo[e] = mo;
        std::vector<double> nxt((size_t)eo[0] * eo[1] * eo[2]);
        for (int k2 = 0; k2 < eo[2]; ++k2)
          for (int k1 = 0; k1 < eo[1]; ++k1)
            for (int k0 = 0; k0 < eo[0]; ++k0) {
              int kk[3] = {k0, k1, k2};
              const int row = kk[e];
              double acc = 0;
              for (int j = 0; j < ext[e]; ++j) {
                kk[e] = j;
                acc += M[row * ext[e] + j] * cur[kk[0] + ext[0] * (kk[1] + ext[1] * kk[2])];
              }
              nxt[k0 + eo[0] * (k1 + eo[1] * k2)] = acc;
            }
        cur.swap(nxt);
        ext[0] = eo[0];
        ext[1] = eo[1];
        ext[2] = eo[2];
      }
      return cur;
    };
    const std::vector<double> gl = m->basis == DGW_BASIS_GAUSS ? gG : apply(gG, n, tab.data() + tab_Sinv(n), n);
    std::copy(gl.begin(), gl.end(), gvec.begin() + (size_t)i * np);
    std::copy(gG.begin(), gG.end(), glev[0].begin() + (size_t)i * np);
    for (int l = 1; l < m->nlev; ++l) {
      const int ml = m->level_pts[l];
      const std::vector<double> gl_l = apply(gG, n, tab.data() + tab_level_F(n, l), ml);
      std::copy(gl_l.begin(), gl_l.end(), glev[l].begin() + (size_t)i * ipw(ml, d));
    }
    const double f = desc->frequency[i];
    wave[i * 3 + 0] = f;
    wave[i * 3 + 1] = desc->t0 ? desc->t0[i] : 1.2 / f;
    wave[i * 3 + 2] = desc->amplitude ? desc->amplitude[i] : 1.0;
  }
  DGW_HIP(hipMalloc(&S->d_cell, S->n * sizeof(int)));
  DGW_HIP(hipMemcpy(S->d_cell, S->cell.data(), S->n * sizeof(int), hipMemcpyHostToDevice));
  DGW_HIP(hipMalloc(&S->d_gvec, gvec.size() * sizeof(double)));
  DGW_HIP(hipMemcpy(S->d_gvec, gvec.data(), gvec.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int l = 0; l < m->nlev; ++l) {
    DGW_HIP(hipMalloc(&S->d_glev[l], glev[l].size() * sizeof(double)));
    DGW_HIP(hipMemcpy(S->d_glev[l], glev[l].data(), glev[l].size() * sizeof(double), hipMemcpyHostToDevice));
  }
  DGW_HIP(hipMalloc(&S->d_wave, wave.size() * sizeof(double)));
  DGW_HIP(hipMemcpy(S->d_wave, wave.data(), wave.size() * sizeof(double), hipMemcpyHostToDevice));
  *out = S.release();
  return DGW_OK;
}

void dgw_sources_destroy(dgw_sources* s) {
  if (!s) return;
  (void)hipFree(s->d_cell);
  (void)hipFree(s->d_gvec);
  for (auto* p : s->d_glev) (void)hipFree(p);
  (void)hipFree(s->d_wave);
  delete s;
}

// ---------------------------------------------------------------- solve
dgw_status dgw_solve_batch(dgw_mesh* m, const dgw_solve_desc* desc, double* u, double* work, int B,
                           dgw_solve_report* report) {
  if (!desc) return fail(DGW_EINVAL, "desc is NULL");
  dgw_status st = check_mesh(m);
  if (st) return st;
  if (desc->scheme != DGW_SCHEME_LSRK54 && desc->scheme != DGW_SCHEME_LSRK59 && desc->scheme != DGW_SCHEME_ADER)
    return fail(DGW_EINVAL, "bad scheme");
  if (desc->scheme == DGW_SCHEME_ADER && (st = check_ader_flags(desc->ader_flags, desc->sources))) return st;
  if (desc->scheme == DGW_SCHEME_ADER && (st = check_hdg_faces(m, desc->ader_flags))) return st;
  const double span = desc->t_end - desc->t0;
  if (!(span > 0) || !std::isfinite(span)) return fail(DGW_EINVAL, "t_end must exceed t0");
  double dt = desc->dt > 0 ? desc->dt : desc->courant * m->hs.dt_unit;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(DGW_EINVAL, "dt or courant must be positive");
  const int64_t nsteps = (int64_t)std::ceil(span / dt - 1e-12);
  dt = span / (double)nsteps;
  if ((st = check_step(m, dt, 0, u, work, B, desc->sources))) return st;
  std::lock_guard<std::mutex> lk(m->mtx);
  if ((st = set_device(m))) return st;
  hipStream_t s = (hipStream_t)desc->stream;
  if (desc->autotune && !m->tuned)
    if ((st = autotune(m, B, s))) return st;
  if (desc->scheme == DGW_SCHEME_ADER && (st = ensure_period_levels(m, ader_period(desc->ader_flags)))) return st;
  const int64_t ne = state_elems(m) * B;
  double* cur = u;
  double* oth = work + ne;
  double* aux = work;  // du (LSRK) or I (ADER)
  const dgw_sources* src = desc->sources;
  double e0 = 0, e1 = 0;
  std::vector<double> en(B), en0(B, 0.0);
  if (desc->watchdog_every > 0 || report) {
    if ((st = energy_impl(m, cur, B, en.data(), s))) return st;
    e0 = en[0];
    en0 = en;
  }
  const double growth = desc->watchdog_growth > 0 ? desc->watchdog_growth : 10.0;
  // every member: a non-finite energy trips; a member that started with
  // positive energy trips when it exceeds growth times that energy (one that
  // starts at rest, driven by a source, is checked for a finite energy only)
  auto unstable = [&]() {
    for (int b = 0; b < B; ++b)
      if (!std::isfinite(en[b]) || (en0[b] > 0 && !(en[b] <= growth * en0[b]))) return true;
    return false;
  };
  auto one = [&](int64_t k, const long long* ctr, int add) -> dgw_status {
    return desc->scheme != DGW_SCHEME_ADER
               ? lsrk_step(m, B, src, desc->t0, dt, (int)(ctr ? add : k), ctr, cur, oth, aux, s, desc->scheme)
               : ader_step(m, desc->ader_flags, B, src, desc->t0, dt, (int)(ctr ? add : k), ctr, cur, oth, aux, s);
  };
  DGW_HIP(hipStreamSynchronize(s));
  const auto tstart = std::chrono::steady_clock::now();
  int64_t k = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  long long* d_ctr = nullptr;
  if (desc->use_graph && nsteps >= 2) {
    // Capture needs a stream of our own (the legacy default stream cannot be
    // captured); two steps per graph keep the ping-pong buffers in place
    // between replays; the device step counter advances inside the graph.
    hipStream_t gs = nullptr;
    DGW_HIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    hipStream_t caller = s;
    s = gs;
    auto cleanup = [&]() {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (graph) (void)hipGraphDestroy(graph);
      if (d_ctr) (void)hipFree(d_ctr);
      (void)hipStreamSynchronize(gs);
      (void)hipStreamDestroy(gs);
    };
    if (hipMalloc(&d_ctr, sizeof(long long)) != hipSuccess) {
      cleanup();
      return fail(DGW_ENOMEM, "graph step counter");
    }
    const long long zero = 0;
    if (hipMemcpyAsync(d_ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, gs) != hipSuccess ||
        hipStreamSynchronize(gs) != hipSuccess) {
      cleanup();
      return fail(DGW_EDEVICE, "graph step counter init");
    }
    double* c0 = cur;
    double* o0 = oth;
    if (hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      cleanup();
      return fail(DGW_EDEVICE, "hipStreamBeginCapture failed");
    }
    dgw_status cst = one(0, d_ctr, 0);
    if (!cst) cst = one(1, d_ctr, 1);
    hipLaunchKernelGGL(advance_counter, dim3(1), dim3(64), 0, gs, d_ctr, 2);
    const hipError_t ce = hipStreamEndCapture(gs, &graph);
    if (cst || ce != hipSuccess || hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
      cleanup();
      return cst ? cst : fail(DGW_EDEVICE, "graph capture failed");
    }
    cur = c0;  // the capture swapped the pointers twice: back where they were
    oth = o0;
    const int64_t pairs = nsteps / 2;
    for (int64_t r = 0; r < pairs && !st; ++r) {
      if (hipGraphLaunch(gexec, gs) != hipSuccess) {
        st = fail(DGW_EDEVICE, "hipGraphLaunch failed");
        break;
      }
      k += 2;
      if (desc->watchdog_every > 0 && (k % desc->watchdog_every) < 2) {
        if ((st = energy_impl(m, cur, B, en.data(), gs))) break;
        if (unstable()) st = fail(DGW_EUNSTABLE, "energy grew beyond the watchdog limit (time step too large?)");
      }
    }
    cleanup();
    s = caller;
    gexec = nullptr;
    graph = nullptr;
    d_ctr = nullptr;
    if (st) return st;
  }
  for (; k < nsteps; ++k) {
    if ((st = one(k, nullptr, 0))) return st;
    if (desc->watchdog_every > 0 && (k + 1) % desc->watchdog_every == 0) {
      if ((st = energy_impl(m, cur, B, en.data(), s))) return st;
      if (unstable()) return fail(DGW_EUNSTABLE, "energy grew beyond the watchdog limit (time step too large?)");
    }
  }
  if (cur != u) DGW_HIP(hipMemcpyAsync(u, cur, ne * 8, hipMemcpyDeviceToDevice, s));
  DGW_HIP(hipStreamSynchronize(s));
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - tstart).count();
  if (report) {
    if ((st = energy_impl(m, u, B, en.data(), s))) return st;
    e1 = en[0];
    report->steps = nsteps;
    report->dt = dt;
    report->wall_s = wall;
    report->dof_steps_per_s = (double)ne * (double)nsteps / std::max(wall, 1e-12);
    report->energy0 = e0;
    report->energy_end = e1;
  }
  return DGW_OK;
}

}  // extern "C"
