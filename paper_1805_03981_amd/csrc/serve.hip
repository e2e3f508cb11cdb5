// Box mesh helper, the built-in Fourier material, and the request server:
// requests (a seeded curved periodic box, degree, scheme, final time) arrive
// over time, are admitted while their device footprint fits the budget, run
// concurrently on their own streams (one time step per request per
// scheduling round, so work from different requests overlaps on the GPU) and
// retire with their latency recorded.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <future>
#include <memory>
#include <thread>
#include <vector>

#include "dgw_host.hpp"

using namespace dgw;

extern "C" {

void dgw_material_fourier(const double* x, int64_t npts, int dim, double* rho, double* c, void* ctx) {
  const dgw_fourier_material* f = static_cast<const dgw_fourier_material*>(ctx);
  const double two_pi = 2.0 * M_PI;
  const double scale = f->amp / std::sqrt((double)f->nmodes);
  for (int64_t i = 0; i < npts; ++i) {
    double s = 0.0;
    for (int m = 0; m < f->nmodes; ++m) {
      double arg = 0.0;
      for (int a = 0; a < dim; ++a) arg += (double)f->m[m][a] * x[i * dim + a];
      s += f->a[m] * std::cos(two_pi * arg + f->phi[m]);
    }
    c[i] = std::min(f->cmax, std::max(f->cmin, f->c0 + scale * s));
    rho[i] = f->rho0;
  }
}

dgw_status dgw_mesh_create_box(int dim, int ncell, int degree, double amp, dgw_material_fn material,
                               void* material_ctx, int flux, int precision, int device, int max_batch,
                               int storage_basis, dgw_mesh** out) {
  if (dim != 2 && dim != 3) return fail(DGW_EUNSUPPORTED, "dim must be 2 or 3");
  if (ncell < 1 || ncell > 1024) return fail(DGW_EINVAL, "ncell must be in 1..1024");
  if (degree < 1 || degree > 8) return fail(DGW_EUNSUPPORTED, "degree must be in 1..8");
  const int q = degree, ng1 = q + 1;
  int64_t nc = 1, ng = 1;
  for (int a = 0; a < dim; ++a) {
    nc *= ncell;
    ng *= ng1;
  }
  std::vector<double> nodes;
  std::vector<int64_t> nb;
  try {
    nodes.resize((size_t)nc * ng * dim);
    nb.resize((size_t)nc * 2 * dim);
  } catch (const std::bad_alloc&) {
    return fail(DGW_ENOMEM, "host allocation");
  }
  const double h = 1.0 / ncell, two_pi = 2.0 * M_PI;
  for (int64_t c = 0; c < nc; ++c) {
    int64_t idx[3] = {c % ncell, (c / ncell) % ncell, dim == 3 ? c / ((int64_t)ncell * ncell) : 0};
    for (int64_t g = 0; g < ng; ++g) {
      const int64_t loc[3] = {g % ng1, (g / ng1) % ng1, dim == 3 ? g / (ng1 * ng1) : 0};
      double X[3];
      double prod = 1.0;
      for (int a = 0; a < dim; ++a) {
        X[a] = ((double)idx[a] + (double)loc[a] / q) * h;
        prod *= std::sin(two_pi * X[a]);
      }
      for (int a = 0; a < dim; ++a) nodes[((size_t)c * ng + g) * dim + a] = X[a] + amp * prod;
    }
    for (int a = 0; a < dim; ++a)
      for (int s = 0; s < 2; ++s) {
        int64_t j[3] = {idx[0], idx[1], idx[2]};
        j[a] = (j[a] + (s ? 1 : ncell - 1)) % ncell;
        nb[(size_t)c * 2 * dim + 2 * a + s] = j[0] + ncell * (j[1] + (int64_t)ncell * j[2]);
      }
  }
  dgw_mesh_desc d;
  std::memset(&d, 0, sizeof(d));
  d.dim = dim;
  d.degree = degree;
  d.n_cells = nc;
  d.geo_degree = q;
  d.geo_nodes = nodes.data();
  d.neighbors = nb.data();
  d.material = material;
  d.material_ctx = material_ctx;
  d.flux = flux;
  d.precision = precision;
  d.device = device;
  d.max_batch = max_batch;
  d.storage_basis = storage_basis;
  return dgw_mesh_create(&d, out);
}

int64_t dgw_request_footprint(const dgw_request* r) {
  if (!r || r->dim < 2 || r->dim > 3 || r->degree < 1 || r->degree > 8 || r->ncell < 1) return -1;
  if (r->scheme != DGW_SCHEME_LSRK54 && r->scheme != DGW_SCHEME_LSRK59 && r->scheme != DGW_SCHEME_ADER) return -1;
  const int d = r->dim, n = r->degree + 1;
  int64_t nc = 1, np = 1, nf = 1;
  for (int a = 0; a < d; ++a) {
    nc *= r->ncell;
    np *= n;
  }
  for (int a = 0; a < d - 1; ++a) nf *= n;
  const int64_t state = nc * (d + 1) * np * 8;
  int64_t geo = nc * ((int64_t)(d * d + 2) * np + 2 * d * (d + 2) * nf) * 8 + nc * 2 * d * 4;
  for (int m = n - 2; m >= 1; m -= 2) {
    int64_t pts = 1;
    for (int a = 0; a < d; ++a) pts *= m;
    geo += nc * (d * d + 2) * pts * 8;
  }
  return geo + 3 * state;  // state + two work registers
}

namespace {

// DoF-steps per stepping call of a live request (about a millisecond of
// GPU time at the solver's rates)
constexpr int64_t kChunkDofSteps = 10000000;

struct Live {
  int idx = -1;
  dgw_mesh* mesh = nullptr;
  double* u = nullptr;
  double* work = nullptr;
  hipStream_t stream = nullptr;
  int64_t steps = 0, done = 0, dofs = 0, footprint = 0;
  double dt = 0;
};

double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

// Gaussian pressure pulse (minimum-image distance), v = 0, at the GL nodes.
void initial_state(dgw_mesh* m, const dgw_request& r, std::vector<double>& u) {
  std::vector<double> x;
  node_coords(m->hs, x);
  const int d = r.dim, np = m->np;
  u.assign((size_t)m->hs.nc * (d + 1) * np, 0.0);
  for (int64_t c = 0; c < m->hs.nc; ++c)
    for (int q = 0; q < np; ++q) {
      double r2 = 0;
      for (int a = 0; a < d; ++a) {
        double dx = x[((size_t)c * np + q) * d + a] - r.ic_center[a];
        dx -= std::round(dx);
        r2 += dx * dx;
      }
      u[((size_t)c * (d + 1) + d) * np + q] = std::exp(-r2 / (2 * r.ic_width * r.ic_width));
    }
}

// A request whose mesh and initial state are being built on a worker thread
// (the host setup of a large curved mesh takes seconds; the live requests
// keep stepping meanwhile).
struct Prep {
  int idx = 0;
  int64_t footprint = 0;
  dgw_mesh* mesh = nullptr;
  std::vector<double> u0;
  std::future<dgw_status> done;
};

std::shared_ptr<Prep> prepare(const dgw_request& r, int idx, int64_t fp, int device) {
  auto P = std::make_shared<Prep>();
  P->idx = idx;
  P->footprint = fp;
  P->done = std::async(std::launch::async, [P, r, device]() -> dgw_status {
    dgw_fourier_material mat = r.material;  // read during the setup only
    const dgw_status st = dgw_mesh_create_box(r.dim, r.ncell, r.degree, r.deform_amp, dgw_material_fourier, &mat,
                                              DGW_FLUX_UPWIND, r.precision, device, 1, DGW_BASIS_GL, &P->mesh);
    if (st) return st;
    initial_state(P->mesh, r, P->u0);
    return DGW_OK;
  });
  return P;
}

}  // namespace

dgw_status dgw_serve(const dgw_server_desc* desc, const dgw_request* reqs, int n, dgw_result* out,
                     dgw_serve_report* report) {
  if (!desc || (!reqs && n > 0) || (!out && n > 0)) return fail(DGW_EINVAL, "NULL argument");
  if (!(desc->hbm_budget_bytes > 0)) return fail(DGW_EINVAL, "hbm_budget_bytes must be positive");
  DGW_HIP(hipSetDevice(desc->device));
  const int max_live = std::max(1, desc->max_live);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  for (int i = 0; i < n; ++i) {
    double* keep = out[i].state_host;
    std::memset(&out[i], 0, sizeof(dgw_result));
    out[i].state_host = keep;
    out[i].t_arrive = desc->realtime ? reqs[i].arrival_s : 0.0;
  }
  std::deque<int> pending(order.begin(), order.end());
  std::vector<Live> live;
  std::vector<std::shared_ptr<Prep>> preparing;
  double used = 0;
  int64_t dof_steps = 0;
  std::vector<double> lat;
  double max_wait = 0;
  int failed = 0;
  const auto t_start = std::chrono::steady_clock::now();
  auto now = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
  auto retire = [&](Live& L, dgw_status st) {
    dgw_result& R = out[L.idx];
    R.status = st;
    if (!st) {
      double e = 0;
      if (dgw_energy(L.mesh, L.u, 1, &e, L.stream) == DGW_OK) R.energy_end = e;
      if (R.state_host)
        (void)hipMemcpyAsync(R.state_host, L.u, L.dofs * 8, hipMemcpyDeviceToHost, L.stream);
      (void)hipStreamSynchronize(L.stream);
    } else {
      ++failed;
    }
    R.t_done = now();
    R.steps = L.done;
    lat.push_back(R.t_done - R.t_arrive);
    if (desc->progress) {
      std::fprintf(stderr, "[serve] request %d: status %d, %lld steps, %lld DoF, latency %.3f s (%zu finished)\n",
                   L.idx, st, (long long)L.done, (long long)L.dofs, R.t_done - R.t_arrive, lat.size());
      std::fflush(stderr);
    }
    (void)hipFree(L.u);
    (void)hipFree(L.work);
    (void)hipStreamDestroy(L.stream);
    dgw_mesh_destroy(L.mesh);
    used -= (double)L.footprint;
  };
  while (!pending.empty() || !live.empty() || !preparing.empty()) {
    // admission: arrived requests, in arrival order, while the budget allows;
    // the budget is reserved now and the mesh is built on a worker thread
    while (!pending.empty() && (int)(live.size() + preparing.size()) < max_live) {
      const int i = pending.front();
      const dgw_request& r = reqs[i];
      if (desc->realtime && r.arrival_s > now()) break;
      const int64_t fp = dgw_request_footprint(&r);
      if (fp < 0 || (double)fp > desc->hbm_budget_bytes) {
        pending.pop_front();
        out[i].status = fp < 0 ? DGW_EINVAL : DGW_ENOMEM;
        out[i].t_admit = out[i].t_done = now();
        ++failed;
        continue;
      }
      if (used + (double)fp > desc->hbm_budget_bytes) break;  // wait for memory
      pending.pop_front();
      out[i].t_admit = now();
      max_wait = std::max(max_wait, out[i].t_admit - out[i].t_arrive);
      used += (double)fp;
      preparing.push_back(prepare(r, i, fp, desc->device));
    }
    // requests whose mesh is ready: device state, then live
    for (size_t j = 0; j < preparing.size();) {
      Prep& P = *preparing[j];
      if (P.done.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
        ++j;
        continue;
      }
      const dgw_status st = P.done.get();
      const int i = P.idx;
      const dgw_request& r = reqs[i];
      if (st) {
        if (P.mesh) dgw_mesh_destroy(P.mesh);
        out[i].status = st;
        out[i].t_done = now();
        ++failed;
        used -= (double)P.footprint;
        preparing.erase(preparing.begin() + j);
        continue;
      }
      Live L;
      L.idx = i;
      L.footprint = P.footprint;
      L.mesh = P.mesh;
      dgw_mesh_info info;
      dgw_mesh_info_get(L.mesh, &info);
      L.dofs = info.dofs;
      out[i].dofs = info.dofs;
      const double dt0 = r.courant * info.dt_unit;
      L.steps = std::max<int64_t>(1, (int64_t)std::ceil(r.t_end / dt0 - 1e-12));
      L.dt = r.t_end / (double)L.steps;
      if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
          hipMalloc(&L.u, L.dofs * 8) != hipSuccess || hipMalloc(&L.work, 2 * L.dofs * 8) != hipSuccess) {
        (void)hipGetLastError();
        retire(L, fail(DGW_ENOMEM, "device allocation for a request"));
        preparing.erase(preparing.begin() + j);
        continue;
      }
      (void)hipMemcpyAsync(L.u, P.u0.data(), L.dofs * 8, hipMemcpyHostToDevice, L.stream);
      (void)hipStreamSynchronize(L.stream);
      double e0 = 0;
      (void)dgw_energy(L.mesh, L.u, 1, &e0, L.stream);
      out[i].energy0 = e0;
      live.push_back(L);
      preparing.erase(preparing.begin() + j);
    }
    if (live.empty()) {
      if (!preparing.empty()) {
        preparing.front()->done.wait_for(std::chrono::milliseconds(2));
      } else if (!pending.empty() && desc->realtime) {
        const double wait = reqs[pending.front()].arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
      }
      continue;
    }
    // a chunk of steps of every live request, each on its own stream: about
    // kChunkDofSteps of work per call, so that a small request does not
    // pay a host round trip per step while a large one advances one step
    // per round (its steps are long enough to keep the GPU busy)
    for (auto& L : live) {
      const dgw_request& r = reqs[L.idx];
      const double t0 = (double)L.done * L.dt;
      const int64_t chunk =
          std::max<int64_t>(1, std::min<int64_t>(L.steps - L.done, kChunkDofSteps / std::max<int64_t>(1, L.dofs)));
      const dgw_status st =
          r.scheme == DGW_SCHEME_ADER
              ? dgw_step_ader(L.mesh, 0, t0, L.dt, (int)chunk, L.u, L.work, 1, nullptr, L.stream)
              : dgw_step_lsrk(L.mesh, r.scheme, t0, L.dt, (int)chunk, L.u, L.work, 1, nullptr, L.stream);
      if (st) {
        L.done = -1 - L.done;  // mark failed
        continue;
      }
      L.done += chunk;
      dof_steps += L.dofs * chunk;
    }
    // retire finished or failed requests (query streams without blocking others)
    for (size_t j = 0; j < live.size();) {
      Live& L = live[j];
      if (L.done < 0) {
        L.done = -1 - L.done;
        retire(L, DGW_EDEVICE);
        live.erase(live.begin() + j);
      } else if (L.done >= L.steps) {
        retire(L, DGW_OK);
        live.erase(live.begin() + j);
      } else {
        ++j;
      }
    }
  }
  if (report) {
    report->n_done = n - failed;
    report->n_failed = failed;
    report->wall_s = now();
    report->p50_s = quantile(lat, 0.5);
    report->p99_s = quantile(lat, 0.99);
    report->dof_steps_per_s = (double)dof_steps / std::max(report->wall_s, 1e-12);
    report->max_wait_s = max_wait;
  }
  return DGW_OK;
}

}  // extern "C"
