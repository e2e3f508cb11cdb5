// Host setup in FP64 (long double for the 1D rules): quadrature rules, the 1D
// matrices of the basis change / collocation derivative / degree reduction,
// and the per-point geometry and material data of the curved mesh.
//
// Paper references: Gauss quadrature on k+1 points and the G / GL Lagrange
// bases (Sec. 3, Sec. 3.1); the collocated derivative and the basis change
// (Sec. 3.2, Alg. 2); the projection to a degree two lower and the reduced
// Gauss sets with their pre-computed inverse Jacobians (Sec. 3.3, Alg. 3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "dgw_host.hpp"

static_assert(DGW_BC_WALL == dgw::kBcWall && DGW_BC_ABSORBING == dgw::kBcAbsorbing &&
                  DGW_BC_PRESCRIBED == dgw::kBcPrescribed && DGW_MAX_PLANE_WAVES == dgw::kMaxPlaneWaves,
              "boundary codes");

namespace dgw {

using ld = long double;

// ---------------------------------------------------------------- 1D rules
static void legendre(int n, ld x, ld& p, ld& dp) {
  // P_n and P_n' by the three-term recurrence
  ld p0 = 1, p1 = x;
  if (n == 0) {
    p = 1;
    dp = 0;
    return;
  }
  for (int j = 2; j <= n; ++j) {
    const ld p2 = ((2 * j - 1) * x * p1 - (j - 1) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = (std::fabs(x) < 1) ? n * (x * p1 - p0) / (x * x - 1) : (x > 0 ? 1 : ((n % 2) ? 1 : -1)) * n * (n + 1) / 2.0L;
}

Rule gauss_rule(int n) {
  Rule r;
  r.x.resize(n);
  r.w.resize(n);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld x = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(n, x, p, dp);
      const ld dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    ld p, dp;
    legendre(n, x, p, dp);
    r.x[i] = 0.5L * (x + 1);
    r.w[i] = 1.0L / ((1 - x * x) * dp * dp);  // 2/((1-x^2) P'^2), halved for [0,1]
  }
  return r;
}

Rule gauss_lobatto_rule(int n) {
  Rule r;
  r.x.resize(n);
  r.w.resize(n);
  const ld pi = 3.141592653589793238462643383279502884L;
  const int m = n - 1;  // interior nodes are the roots of P_m'
  for (int i = 0; i < n; ++i) {
    ld x;
    if (i == 0)
      x = -1;
    else if (i == n - 1)
      x = 1;
    else {
      x = -std::cos(pi * i / m);
      for (int it = 0; it < 100; ++it) {
        ld p, dp;
        legendre(m, x, p, dp);
        const ld d2p = (2 * x * dp - m * (m + 1) * p) / (1 - x * x);
        const ld dx = dp / d2p;
        x -= dx;
        if (std::fabs(dx) < 1e-19L) break;
      }
    }
    ld p, dp;
    legendre(m, x, p, dp);
    r.x[i] = 0.5L * (x + 1);
    r.w[i] = 1.0L / (n * m * p * p);  // 2/(n(n-1) P_{n-1}^2), halved
  }
  return r;
}

long double lagrange_value(const std::vector<ld>& nodes, int j, ld x) {
  ld v = 1;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
  return v;
}

long double lagrange_deriv(const std::vector<ld>& nodes, int j, ld x) {
  ld s = 0;
  const int n = (int)nodes.size();
  for (int m = 0; m < n; ++m) {
    if (m == j) continue;
    ld t = 1 / (nodes[j] - nodes[m]);
    for (int l = 0; l < n; ++l)
      if (l != j && l != m) t *= (x - nodes[l]) / (nodes[j] - nodes[l]);
    s += t;
  }
  return s;
}

std::vector<double> build_tables(int n) {
  std::vector<double> t(tab_size(n), 0.0);
  const Rule g = gauss_rule(n), gl = gauss_lobatto_rule(n);
  for (int q = 0; q < n; ++q)
    for (int j = 0; j < n; ++j) {
      t[tab_S(n) + q * n + j] = (double)lagrange_value(gl.x, j, g.x[q]);     // GL coeff -> G value
      t[tab_Sinv(n) + q * n + j] = (double)lagrange_value(g.x, j, gl.x[q]);  // G value -> GL coeff
      t[tab_D(n) + q * n + j] = (double)lagrange_deriv(g.x, j, g.x[q]);      // l^G_j'(xi_q)
    }
  for (int j = 0; j < n; ++j) {
    t[tab_LF0(n) + j] = (double)lagrange_value(g.x, j, 0.0L);
    t[tab_LF1(n) + j] = (double)lagrange_value(g.x, j, 1.0L);
  }
  for (int r = 1; r <= 3; ++r)
    for (int l = 1; l < num_levels_r(n, r); ++l) {
      const int m = n - r * l, mp = m + r;
      const Rule rm = gauss_rule(m), rp = gauss_rule(mp);
      for (int q = 0; q < m; ++q)
        for (int j = 0; j < m; ++j)
          t[tab_level_D(n, l, r) + q * m + j] = m > 1 ? (double)lagrange_deriv(rm.x, j, rm.x[q]) : 0.0;
      // unweighted L2 projection on the reference element, collocated form
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < mp; ++b)
          t[tab_level_P(n, l, r) + a * mp + b] = (double)(rp.w[b] * lagrange_value(rm.x, a, rp.x[b]) / rm.w[a]);
      for (int q = 0; q < mp; ++q)
        for (int a = 0; a < m; ++a)
          t[tab_level_E(n, l, r) + q * m + a] = (double)lagrange_value(rm.x, a, rp.x[q]);
      for (int q = 0; q < m; ++q)
        for (int j = 0; j < n; ++j) t[tab_level_F(n, l, r) + q * n + j] = (double)lagrange_value(g.x, j, rm.x[q]);
      // level-l Gauss interpolant at the GL nodes: the embeddings back to
      // level 0 (exact on the lower degree) followed by S^-1, in one matrix
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < m; ++a) t[tab_level_Q(n, l, r) + i * m + a] = (double)lagrange_value(rm.x, a, gl.x[i]);
    }
  return t;
}

// ---------------------------------------------------------------- geometry
namespace {

int ipw(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

struct GeoMats {
  // value and derivative of the equispaced Lagrange polynomials at 1D points
  std::vector<double> V, W;
  int m = 0;
};

GeoMats geo_mats(int q, const std::vector<ld>& pts) {
  std::vector<ld> nodes(q + 1);
  for (int j = 0; j <= q; ++j) nodes[j] = (ld)j / q;
  GeoMats g;
  g.m = (int)pts.size();
  g.V.resize(g.m * (q + 1));
  g.W.resize(g.m * (q + 1));
  for (int i = 0; i < g.m; ++i)
    for (int j = 0; j <= q; ++j) {
      g.V[i * (q + 1) + j] = (double)lagrange_value(nodes, j, pts[i]);
      g.W[i * (q + 1) + j] = (double)lagrange_deriv(nodes, j, pts[i]);
    }
  return g;
}

// One sum-factorized pass along direction dir of a tensor of d-vectors:
// in has extents E[3] (x fastest, the d components innermost), the m x E[dir]
// matrix M replaces extent dir by m; out[point * ostride + a * cstride].
static void map_pass(int d, const int* E, int dir, const double* in, const double* M, int m, double* out,
                     int ostride, int cstride) {
  int eo[3] = {E[0], E[1], E[2]};
  eo[dir] = m;
  const int si[3] = {1, E[0], E[0] * E[1]};
  const int so[3] = {1, eo[0], eo[0] * eo[1]};
  const int n = E[dir];
  for (int k2 = 0; k2 < eo[2]; ++k2)
    for (int k1 = 0; k1 < eo[1]; ++k1)
      for (int k0 = 0; k0 < eo[0]; ++k0) {
        int kk[3] = {k0, k1, k2};
        const int io = k0 * so[0] + k1 * so[1] + k2 * so[2];
        const int row = kk[dir];
        kk[dir] = 0;
        const double* src = in + (size_t)(kk[0] * si[0] + kk[1] * si[1] + kk[2] * si[2]) * d;
        const double* mr = M + (size_t)row * n;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < n; ++j) {
          const double w = mr[j];
          const double* v = src + (size_t)j * si[dir] * d;
          for (int a = 0; a < d; ++a) acc[a] += w * v[a];
        }
        for (int a = 0; a < d; ++a) out[(size_t)io * ostride + a * cstride] = acc[a];
      }
}

// x [P][d] and J [P][d][d] (J[p][a][b] = dx_a/dxi_b) of one cell at the tensor
// point set given by per-direction matrices (V values, W derivatives of the
// 1D geometry Lagrange polynomials).  All d coordinates in one pass, and the
// passes shared between the map and its derivatives: in 3D, V0/W0 along x,
// then V1 on both and W1 on the V0 branch, then the last direction.
//
// The passes run on the nodes relative to the cell's first node: J does not
// depend on a translation, and a small cell far from the origin would
// otherwise lose digits in the sums of its derivatives (absolute coordinates
// of order 1 cancelling down to a cell size of order 1/n); x gets that node
// back at the end.
void eval_map(int d, int q, const double* X_abs, const std::vector<const GeoMats*>& gm, double* x, double* J,
              std::vector<double>& comp, std::vector<double>& res, std::vector<double>& t1,
              std::vector<double>& t2) {
  const int Q = q + 1;
  const int m0 = gm[0]->m, m1 = gm[1]->m;
  int E[3] = {Q, Q, d == 3 ? Q : 1};
  const int ng = Q * Q * (d == 3 ? Q : 1);
  thread_local std::vector<double> rel;
  rel.resize((size_t)ng * d);
  for (int g = 0; g < ng; ++g)
    for (int a = 0; a < d; ++a) rel[(size_t)g * d + a] = X_abs[(size_t)g * d + a] - X_abs[a];
  const double* X = rel.data();
  const int npts = m0 * m1 * (d == 3 ? gm[2]->m : 1);
  auto shift_back = [&]() {
    for (int p = 0; p < npts; ++p)
      for (int a = 0; a < d; ++a) x[(size_t)p * d + a] += X_abs[a];
  };
  // direction 0: A = V0 X, B = W0 X
  const int nA = m0 * Q * (d == 3 ? Q : 1);
  comp.resize((size_t)nA * d);
  res.resize((size_t)nA * d);
  map_pass(d, E, 0, X, gm[0]->V.data(), m0, comp.data(), d, 1);
  map_pass(d, E, 0, X, gm[0]->W.data(), m0, res.data(), d, 1);
  E[0] = m0;
  if (d == 2) {
    // direction 1: x = V1 A, dx/dxi1 = W1 A, dx/dxi0 = V1 B
    map_pass(d, E, 1, comp.data(), gm[1]->V.data(), m1, x, d, 1);
    map_pass(d, E, 1, comp.data(), gm[1]->W.data(), m1, J + 1, d * d, d);
    map_pass(d, E, 1, res.data(), gm[1]->V.data(), m1, J + 0, d * d, d);
    shift_back();
    return;
  }
  const int m2 = gm[2]->m;
  // direction 1: AA = V1 A, AW = W1 A, BV = V1 B
  const int nB = m0 * m1 * Q;
  t1.resize((size_t)2 * nB * d);
  t2.resize((size_t)nB * d);
  double* AA = t1.data();
  double* AW = t1.data() + (size_t)nB * d;
  double* BV = t2.data();
  map_pass(d, E, 1, comp.data(), gm[1]->V.data(), m1, AA, d, 1);
  map_pass(d, E, 1, comp.data(), gm[1]->W.data(), m1, AW, d, 1);
  map_pass(d, E, 1, res.data(), gm[1]->V.data(), m1, BV, d, 1);
  E[1] = m1;
  // direction 2: x = V2 AA, dx/dxi2 = W2 AA, dx/dxi1 = V2 AW, dx/dxi0 = V2 BV
  map_pass(d, E, 2, AA, gm[2]->V.data(), m2, x, d, 1);
  map_pass(d, E, 2, AA, gm[2]->W.data(), m2, J + 2, d * d, d);
  map_pass(d, E, 2, AW, gm[2]->V.data(), m2, J + 1, d * d, d);
  map_pass(d, E, 2, BV, gm[2]->V.data(), m2, J + 0, d * d, d);
  shift_back();
}

double det_inv(int d, const double* J, double* Ji) {
  if (d == 2) {
    const double det = J[0] * J[3] - J[1] * J[2];
    Ji[0] = J[3] / det;
    Ji[1] = -J[1] / det;
    Ji[2] = -J[2] / det;
    Ji[3] = J[0] / det;
    return det;
  }
  const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  Ji[0] = c00 / det;
  Ji[3] = c01 / det;
  Ji[6] = c02 / det;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
  return det;
}

// Smallest singular value of J (eigenvalues of J^T J by Jacobi rotations).
double sigma_min(int d, const double* J) {
  double A[9] = {0};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0;
      for (int k = 0; k < d; ++k) s += J[k * d + i] * J[k * d + j];
      A[i * 3 + j] = s;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) off += A[i * 3 + j] * A[i * 3 + j];
    if (off < 1e-40) break;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) {
        if (std::fabs(A[i * 3 + j]) < 1e-300) continue;
        const double th = 0.5 * std::atan2(2 * A[i * 3 + j], A[j * 3 + j] - A[i * 3 + i]);
        const double c = std::cos(th), s = std::sin(th);
        for (int k = 0; k < d; ++k) {  // rotate rows/cols i, j
          const double aki = A[k * 3 + i], akj = A[k * 3 + j];
          A[k * 3 + i] = c * aki - s * akj;
          A[k * 3 + j] = s * aki + c * akj;
        }
        for (int k = 0; k < d; ++k) {
          const double aik = A[i * 3 + k], ajk = A[j * 3 + k];
          A[i * 3 + k] = c * aik - s * ajk;
          A[j * 3 + k] = s * aik + c * ajk;
        }
      }
  }
  double mn = A[0];
  for (int i = 1; i < d; ++i) mn = std::min(mn, A[i * 3 + i]);
  return std::sqrt(std::max(mn, 0.0));
}

template <class F>
void parallel_for(int64_t n, F&& f) {
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 64) nt = 1;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int64_t i = t; i < n; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

void map_point(const HostSetup& hs, int64_t cell, const double* xi, double* x, double* J) {
  std::vector<GeoMats> gm(hs.dim);
  std::vector<const GeoMats*> gp(hs.dim);
  for (int e = 0; e < hs.dim; ++e) {
    gm[e] = geo_mats(hs.q, {(ld)xi[e]});
    gp[e] = &gm[e];
  }
  std::vector<double> comp, res, t1, t2;
  const int ng = ipw(hs.q + 1, hs.dim);
  eval_map(hs.dim, hs.q, hs.geo_nodes.data() + cell * ng * hs.dim, gp, x, J, comp, res, t1, t2);
}

void node_coords(const HostSetup& hs, std::vector<double>& out) {
  const int d = hs.dim, n = hs.n, np = ipw(n, d), ng = ipw(hs.q + 1, d);
  const Rule gl = gauss_lobatto_rule(n);
  const GeoMats gm = geo_mats(hs.q, gl.x);
  std::vector<const GeoMats*> gp(d, &gm);
  out.resize((size_t)hs.nc * np * d);
  parallel_for(hs.nc, [&](int64_t c) {
    std::vector<double> comp, res, t1, t2, J((size_t)np * d * d);
    eval_map(d, hs.q, hs.geo_nodes.data() + c * ng * d, gp, out.data() + c * np * d, J.data(), comp, res, t1, t2);
  });
}

// Neighbour face of face f of cell c, and the orientation of the pair.
int face_of_neighbor(const HostSetup& hs, int64_t c, int f) {
  return hs.fo.empty() ? (f ^ 1) : hs.fo[c * 2 * hs.dim + f] / 8;
}
int orient_of(const HostSetup& hs, int64_t c, int f) { return hs.fo.empty() ? 0 : hs.fo[c * 2 * hs.dim + f] % 8; }

// Index on the neighbour's face (n points per direction, the first
// tangential direction fastest) of own face point p under orientation o:
// bit 2 swaps the two tangential indices first, bit 0 reverses the first,
// bit 1 the second (2D: bit 0 reverses the only one).  The Gauss and GL
// point sets are symmetric, so a reversal is i -> n-1-i.
int orient_face_index(int d, int n, int o, int p) {
  if (d == 2) return (o & 1) ? n - 1 - p : p;
  int i = p % n, j = p / n;
  if (o & 4) std::swap(i, j);
  if (o & 1) i = n - 1 - i;
  if (o & 2) j = n - 1 - j;
  return i + n * j;
}

dgw_status build_setup(const dgw_mesh_desc& desc, HostSetup& hs) {
  const int d = desc.dim, k = desc.degree, n = k + 1;
  const int q = desc.geo_degree > 0 ? desc.geo_degree : k;
  if (q < 1 || q > 8) return fail(DGW_EUNSUPPORTED, "geo_degree must be in 1..8");
  hs.dim = d;
  hs.k = k;
  hs.n = n;
  hs.q = q;
  hs.nc = desc.n_cells;
  hs.material = desc.material;
  hs.material_ctx = desc.material_ctx;
  const int64_t nc = desc.n_cells;
  const int np = ipw(n, d), nf = ipw(n, d - 1), ng = ipw(q + 1, d), nface = 2 * d;
  const int ncomp_geo = d * d + 2;
  // neighbours: conforming; negative entries are boundary codes
  hs.nb.resize(nc * nface);
  for (int64_t c = 0; c < nc; ++c)
    for (int f = 0; f < nface; ++f) {
      const int64_t o = desc.neighbors[c * nface + f];
      if (o < 0 && o != DGW_BC_WALL && o != DGW_BC_ABSORBING && o != DGW_BC_PRESCRIBED)
        return fail(DGW_EINVAL, "negative neighbor entries must be DGW_BC_WALL, DGW_BC_ABSORBING or DGW_BC_PRESCRIBED");
      if (o == DGW_BC_PRESCRIBED) hs.prescribed = true;
      if (o >= nc) return fail(DGW_EINVAL, "neighbor index out of range");
      hs.nb[c * nface + f] = (int32_t)o;
    }
  if (desc.n_plane_waves < 0 || desc.n_plane_waves > DGW_MAX_PLANE_WAVES ||
      (desc.n_plane_waves > 0 && !desc.plane_waves))
    return fail(DGW_EINVAL, "n_plane_waves must be in 0..DGW_MAX_PLANE_WAVES with plane_waves given");
  if (hs.prescribed && desc.n_plane_waves < 1)
    return fail(DGW_EINVAL, "DGW_BC_PRESCRIBED faces need plane_waves (the exterior state)");
  hs.waves.clear();
  for (int j = 0; j < desc.n_plane_waves; ++j) {
    const dgw_plane_wave& w = desc.plane_waves[j];
    const double kk = w.k[0] * w.k[0] + w.k[1] * w.k[1] + (d == 3 ? w.k[2] * w.k[2] : 0.0);
    const double v[7] = {w.amplitude, w.k[0], w.k[1], d == 3 ? w.k[2] : 0.0, w.omega, w.phase, w.impedance};
    for (double x : v)
      if (!std::isfinite(x)) return fail(DGW_EINVAL, "plane wave parameters must be finite");
    if (!(kk > 0) || !(w.impedance > 0)) return fail(DGW_EINVAL, "plane waves need |k| > 0 and impedance > 0");
    hs.waves.insert(hs.waves.end(), v, v + 7);
  }
  if (desc.face_orient) {
    hs.fo.assign(desc.face_orient, desc.face_orient + nc * nface);
    const int norient = d == 3 ? 8 : 2;
    for (int64_t c = 0; c < nc; ++c)
      for (int f = 0; f < nface; ++f) {
        const int code = hs.fo[c * nface + f];
        if (code < 0 || code / 8 >= nface || code % 8 >= norient)
          return fail(DGW_EINVAL, "face_orient code out of range");
      }
  }
  for (int64_t c = 0; c < nc; ++c)
    for (int f = 0; f < nface; ++f) {
      const int64_t o = desc.neighbors[c * nface + f];
      if (o < 0) continue;
      const int fn = face_of_neighbor(hs, c, f);
      if (desc.neighbors[o * nface + fn] != c || face_of_neighbor(hs, o, fn) != f)
        return fail(DGW_EINVAL, "neighbor table is not conforming (the neighbour's face does not point back)");
      // the orientation back must undo the orientation there
      for (int p = 0; p < ipw(n, d - 1); ++p)
        if (orient_face_index(d, n, orient_of(hs, o, fn), orient_face_index(d, n, orient_of(hs, c, f), p)) != p)
          return fail(DGW_EINVAL, "face orientations of a face pair do not invert each other");
    }
  hs.geo_nodes.assign(desc.geo_nodes, desc.geo_nodes + nc * ng * d);

  const Rule g = gauss_rule(n);
  // 1D map matrices at the point sets
  const GeoMats gm_cell = geo_mats(q, g.x);
  const GeoMats gm_lo = geo_mats(q, {0.0L}), gm_hi = geo_mats(q, {1.0L});
  const int nlev = num_levels(n);
  std::vector<Rule> lrule(nlev);
  std::vector<GeoMats> gm_lev(nlev);
  for (int l = 1; l < nlev; ++l) {
    lrule[l] = gauss_rule(n - 2 * l);
    gm_lev[l] = geo_mats(q, lrule[l].x);
  }
  hs.cell.assign((size_t)nc * ncomp_geo * np, 0.0);
  hs.face.assign((size_t)nc * nface * (d + 2) * nf, 0.0);
  if (hs.prescribed) hs.face_x.assign((size_t)nc * nface * d * nf, 0.0);
  hs.level.assign(nlev, {});
  for (int l = 1; l < nlev; ++l) hs.level[l].assign((size_t)nc * ncomp_geo * ipw(n - 2 * l, d), 0.0);
  hs.hK.assign(nc, 0.0);
  hs.cK.assign(nc, 0.0);
  std::vector<double> Zown((size_t)nc * nface * nf);
  // weights of the tensor rules
  auto tensor_w = [&](const Rule& r, int dims, std::vector<double>& w) {
    const int m = (int)r.x.size();
    const int P = ipw(m, dims);
    w.assign(P, 1.0);
    for (int p = 0; p < P; ++p) {
      int t = p;
      long double acc = 1;
      for (int e = 0; e < dims; ++e) {
        acc *= r.w[t % m];
        t /= m;
      }
      w[p] = (double)acc;
    }
  };
  std::vector<double> wcell, wface;
  tensor_w(g, d, wcell);
  tensor_w(g, d - 1, wface);
  std::vector<std::vector<double>> wlev(nlev);
  for (int l = 1; l < nlev; ++l) tensor_w(lrule[l], d, wlev[l]);

  // point sets: 0 = cell, 1..2d = faces, 2d+l = level l
  const int nsets = 1 + nface + (nlev - 1);
  std::vector<int> set_pts(nsets);
  std::vector<std::vector<const GeoMats*>> set_mats(nsets, std::vector<const GeoMats*>(d));
  for (int e = 0; e < d; ++e) set_mats[0][e] = &gm_cell;
  set_pts[0] = np;
  for (int f = 0; f < nface; ++f) {
    for (int e = 0; e < d; ++e) set_mats[1 + f][e] = (e == f / 2) ? ((f & 1) ? &gm_hi : &gm_lo) : &gm_cell;
    set_pts[1 + f] = nf;
  }
  for (int l = 1; l < nlev; ++l) {
    for (int e = 0; e < d; ++e) set_mats[nface + l][e] = &gm_lev[l];
    set_pts[nface + l] = ipw(n - 2 * l, d);
  }
  int pts_per_cell = 0;
  std::vector<int> set_off(nsets);
  for (int s = 0; s < nsets; ++s) {
    set_off[s] = pts_per_cell;
    pts_per_cell += set_pts[s];
  }

  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nc, (64ll << 20) / (8ll * pts_per_cell * (d + d * d))));
  std::vector<double> X, Jb, rho, cc;
  std::string err;
  std::mutex err_mtx;
  for (int64_t c0 = 0; c0 < nc; c0 += chunk) {
    const int64_t cn = std::min(chunk, nc - c0);
    X.resize((size_t)cn * pts_per_cell * d);
    Jb.resize((size_t)cn * pts_per_cell * d * d);
    parallel_for(cn, [&](int64_t i) {
      std::vector<double> comp, res, t1, t2;
      const double* Xn = hs.geo_nodes.data() + (c0 + i) * ng * d;
      for (int s = 0; s < nsets; ++s)
        eval_map(d, q, Xn, set_mats[s], X.data() + ((size_t)i * pts_per_cell + set_off[s]) * d,
                 Jb.data() + ((size_t)i * pts_per_cell + set_off[s]) * d * d, comp, res, t1, t2);
    });
    rho.resize((size_t)cn * pts_per_cell);
    cc.resize((size_t)cn * pts_per_cell);
    if (desc.material == dgw_material_fourier) {
      // the library's own material is thread-safe: one block of cells per
      // call; a caller's callback is called from this thread only
      parallel_for(cn, [&](int64_t i) {
        const size_t o = (size_t)i * pts_per_cell;
        desc.material(X.data() + o * d, pts_per_cell, d, rho.data() + o, cc.data() + o, desc.material_ctx);
      });
    } else {
      desc.material(X.data(), cn * pts_per_cell, d, rho.data(), cc.data(), desc.material_ctx);
    }
    parallel_for(cn, [&](int64_t i) {
      const int64_t cell = c0 + i;
      double Ji[9];
      double hmin = 1e300, cmax = 0;
      for (int s = 0; s < nsets; ++s) {
        for (int p = 0; p < set_pts[s]; ++p) {
          const size_t pp = (size_t)i * pts_per_cell + set_off[s] + p;
          const double* J = Jb.data() + pp * d * d;
          const double det = det_inv(d, J, Ji);
          const double r = rho[pp], c = cc[pp];
          if (!(det > 0) || !(r > 0) || !(c > 0)) {
            std::lock_guard<std::mutex> lk(err_mtx);
            if (err.empty())
              err = !(det > 0) ? "non-positive Jacobian determinant in cell " + std::to_string(cell)
                               : "non-positive rho or c in cell " + std::to_string(cell);
            return;
          }
          if (s == 0) {
            const double wd = wcell[p] * det;
            double* G = hs.cell.data() + (size_t)cell * ncomp_geo * np;
            for (int b = 0; b < d; ++b)
              for (int a = 0; a < d; ++a) G[(b * d + a) * np + p] = wd * Ji[b * d + a];
            G[(d * d) * np + p] = 1.0 / (wd * r);
            G[(d * d + 1) * np + p] = r * c * c / wd;
            hmin = std::min(hmin, sigma_min(d, J));
            cmax = std::max(cmax, c);
          } else if (s <= nface) {
            const int f = s - 1, dir = f / 2;
            const double sgn = (f & 1) ? 1.0 : -1.0;
            const double wd = wface[p] * det * sgn;
            double* F = hs.face.data() + ((size_t)cell * nface + f) * (d + 2) * nf;
            for (int a = 0; a < d; ++a) F[a * nf + p] = wd * Ji[dir * d + a];
            F[d * nf + p] = r * c;
            Zown[((size_t)cell * nface + f) * nf + p] = r * c;
            if (hs.prescribed) {
              const double* xp = X.data() + pp * d;
              for (int a = 0; a < d; ++a) hs.face_x[(((size_t)cell * nface + f) * d + a) * nf + p] = xp[a];
            }
          } else {
            const int l = s - nface;
            const int m = set_pts[s];
            const double wd = wlev[l][p] * det;
            double* G = hs.level[l].data() + (size_t)cell * ncomp_geo * m;
            for (int b = 0; b < d; ++b)
              for (int a = 0; a < d; ++a) G[(b * d + a) * m + p] = wd * Ji[b * d + a];
            G[(d * d) * m + p] = 1.0 / (wd * r);
            G[(d * d + 1) * m + p] = r * c * c / wd;
          }
        }
      }
      hs.hK[cell] = hmin;
      hs.cK[cell] = cmax;
    });
    if (!err.empty()) return fail(DGW_EINVAL, err);
  }
  // impedance of the neighbour at the shared face point (its own sample, at
  // the point its face orientation maps to); on a boundary face the own one
  for (int64_t c = 0; c < nc; ++c)
    for (int f = 0; f < nface; ++f) {
      const int64_t o = hs.nb[c * nface + f];
      double* F = hs.face.data() + ((size_t)c * nface + f) * (d + 2) * nf;
      if (o < 0) {
        const double* Zo = Zown.data() + ((size_t)c * nface + f) * nf;
        for (int p = 0; p < nf; ++p) F[(d + 1) * nf + p] = Zo[p];
      } else {
        const double* Zo = Zown.data() + ((size_t)o * nface + face_of_neighbor(hs, c, f)) * nf;
        const int ori = orient_of(hs, c, f);
        for (int p = 0; p < nf; ++p) F[(d + 1) * nf + p] = Zo[orient_face_index(d, n, ori, p)];
      }
    }
  double dtu = 1e300, hmin = 1e300, cmax = 0;
  for (int64_t c = 0; c < nc; ++c) {
    dtu = std::min(dtu, hs.hK[c] / hs.cK[c]);
    hmin = std::min(hmin, hs.hK[c]);
    cmax = std::max(cmax, hs.cK[c]);
  }
  hs.dt_unit = dtu / std::pow((double)k, 1.5);
  hs.h_min = hmin;
  hs.c_max = cmax;
  return DGW_OK;
}

// Metric and mass factors at the m^d tensor Gauss points of every cell, in
// the layout of hs.level: [nc][d*d+2][m^d] (w detJ J^-1 at b*d+a, then
// 1/(w detJ rho), rho c^2/(w detJ)).  For the reduced TCK levels of another
// reduction period than the one built with the mesh; evaluates the map and
// the material callback again.
dgw_status build_level_metric(const HostSetup& hs, int m, std::vector<double>& out) {
  const int d = hs.dim, q = hs.q, ng = ipw(q + 1, d), P = ipw(m, d), ncomp = d * d + 2;
  const int64_t nc = hs.nc;
  const Rule r = gauss_rule(m);
  const GeoMats gm = geo_mats(q, r.x);
  std::vector<const GeoMats*> mats(d, &gm);
  std::vector<double> w(P, 1.0);
  for (int p = 0; p < P; ++p) {
    int t = p;
    long double acc = 1;
    for (int e = 0; e < d; ++e) {
      acc *= r.w[t % m];
      t /= m;
    }
    w[p] = (double)acc;
  }
  out.assign((size_t)nc * ncomp * P, 0.0);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nc, (64ll << 20) / (8ll * P * (d + d * d))));
  std::vector<double> X, Jb, rho, cc;
  std::string err;
  std::mutex err_mtx;
  for (int64_t c0 = 0; c0 < nc; c0 += chunk) {
    const int64_t cn = std::min(chunk, nc - c0);
    X.resize((size_t)cn * P * d);
    Jb.resize((size_t)cn * P * d * d);
    parallel_for(cn, [&](int64_t i) {
      std::vector<double> comp, res, t1, t2;
      eval_map(d, q, hs.geo_nodes.data() + (c0 + i) * ng * d, mats, X.data() + (size_t)i * P * d,
               Jb.data() + (size_t)i * P * d * d, comp, res, t1, t2);
    });
    rho.resize((size_t)cn * P);
    cc.resize((size_t)cn * P);
    hs.material(X.data(), cn * P, d, rho.data(), cc.data(), hs.material_ctx);
    parallel_for(cn, [&](int64_t i) {
      double Ji[9];
      double* G = out.data() + (size_t)(c0 + i) * ncomp * P;
      for (int p = 0; p < P; ++p) {
        const size_t pp = (size_t)i * P + p;
        const double det = det_inv(d, Jb.data() + pp * d * d, Ji);
        const double rr = rho[pp], c = cc[pp];
        if (!(det > 0) || !(rr > 0) || !(c > 0)) {
          std::lock_guard<std::mutex> lk(err_mtx);
          if (err.empty()) err = "non-positive Jacobian, rho or c in cell " + std::to_string(c0 + i);
          return;
        }
        const double wd = w[p] * det;
        for (int b = 0; b < d; ++b)
          for (int a = 0; a < d; ++a) G[(b * d + a) * P + p] = wd * Ji[b * d + a];
        G[(d * d) * P + p] = 1.0 / (wd * rr);
        G[(d * d + 1) * P + p] = rr * c * c / wd;
      }
    });
    if (!err.empty()) return fail(DGW_EINVAL, err);
  }
  return DGW_OK;
}

}  // namespace dgw
