// HIP kernels of the matrix-free DG acoustic operator for gfx950.
//
// One workgroup owns `cpw` consecutive cells of one batch member.  Each cell's
// (d+1) x n^d tile lives in LDS; every 1D contraction (the "tensor product
// kernel" of Sec. 3) is done line by line: a thread loads one line of n values
// into registers, multiplies by the n x n matrix (uniform across the
// wavefront, so its entries come through the scalar cache) and writes the
// line back.  Steps of the fused operator sweep (Sec. 3.1, Sec. 4.3):
//   A  coalesced load of the cell tiles and gather of the neighbours' GL face
//      nodes (n^(d-1) values per face and component, Sec. 3.1)
//   B  GL -> G basis change, d passes (u_G = u_GL, Sec. 3.2); tangential
//      GL -> G interpolation of the neighbour traces
//   C  per direction b: volume fluxes w detJ J^-1 applied pointwise in FP64,
//      transposed collocation derivative (Sec. 3, collocation), and the two
//      faces normal to b (own trace by contraction with l^G(0), l^G(1);
//      upwind flux; lift, rank one in the normal direction)
//   D  inverse mass in the collocated basis: pointwise 1/(w detJ rho),
//      rho c^2/(w detJ), then G -> GL (Sec. 3.1, inverse via basis change)
//   E  epilogue: store, fused low-storage Runge-Kutta update, or ADER update
#pragma once
#include <hip/hip_runtime.h>

#include "dgw_params.hpp"

namespace dgw {

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Workgroup id -> logical id so that each XCD (workgroups are dispatched round
// robin over the 8 XCDs) processes one contiguous range of logical ids: the
// cells it touches, their neighbours' faces and (for batches) the shared
// geometry stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  constexpr int NX = 8;
  const int q = nblk / NX, r = nblk % NX;
  const int x = bid % NX, local = bid / NX;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Index geometry of a 1D pass along direction DIR of a D-dimensional tensor.
// Extents of the other directions: A0, A1, A2 (entry DIR ignored); the passed
// direction has MI entries on input and MO on output.
template <int D, int DIR, int MI, int MO, int A0, int A1, int A2>
struct Pass {
  static constexpr int ext(int e, int m) { return e == DIR ? m : (e == 0 ? A0 : (e == 1 ? A1 : A2)); }
  static constexpr int stride(int e, int m) { return e == 0 ? 1 : stride(e - 1, m) * ext(e - 1, m); }
  static constexpr int size(int m) { return stride(D - 1, m) * ext(D - 1, m); }
  static constexpr int nlines() {
    int r = 1;
    for (int e = 0; e < D; ++e)
      if (e != DIR) r *= ext(e, MI);
    return r;
  }
  static constexpr int SIN = size(MI), SOUT = size(MO), NL = nlines();
  static constexpr int STEP_IN = stride(DIR, MI), STEP_OUT = stride(DIR, MO);
  __device__ static __forceinline__ void base(int L, int& bi, int& bo) {
    bi = 0;
    bo = 0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (e == DIR) continue;
      const int x = ext(e, MI);
      const int c = L % x;
      L /= x;
      bi += c * stride(e, MI);
      bo += c * stride(e, MO);
    }
  }
};

enum PassMode { PM_STORE = 0, PM_ADD_SCALED = 1 };

// out = M in along DIR, for nslices independent tensors (cells x components).
// in and out may be the same buffer when MI == MO (each line is read whole
// before it is written, and lines are disjoint).
template <int D, int DIR, int MI, int MO, int A0, int A1, int A2, int MODE, typename TM, typename TI,
          typename TO>
__device__ __forceinline__ void tpass(const TI* in, TO* out, int nslices, const TM* __restrict__ M,
                                      double scale = 1.0) {
  using P = Pass<D, DIR, MI, MO, A0, A1, A2>;
  const int total = nslices * P::NL;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int s = w / P::NL;
    const int L = w - s * P::NL;
    int bi, bo;
    P::base(L, bi, bo);
    const TI* src = in + s * P::SIN + bi;
    TO* dst = out + s * P::SOUT + bo;
    TM x[MI];
#pragma unroll
    for (int j = 0; j < MI; ++j) x[j] = (TM)src[j * P::STEP_IN];
#pragma unroll
    for (int i = 0; i < MO; ++i) {
      TM acc = M[i * MI] * x[0];
#pragma unroll
      for (int j = 1; j < MI; ++j) acc = fma(M[i * MI + j], x[j], acc);
      if constexpr (MODE == PM_STORE)
        dst[i * P::STEP_OUT] = (TO)acc;
      else
        dst[i * P::STEP_OUT] += (TO)(scale * (double)acc);
    }
  }
}

// Apply the same n x n matrix along all D directions in place (square passes).
template <int D, int N, typename TM, typename TT>
__device__ __forceinline__ void tensor_apply_inplace(TT* buf, int nslices, const TM* M) {
  tpass<D, 0, N, N, N, N, N, PM_STORE, TM>(buf, buf, nslices, M);
  __syncthreads();
  tpass<D, 1, N, N, N, N, N, PM_STORE, TM>(buf, buf, nslices, M);
  __syncthreads();
  if constexpr (D == 3) {
    tpass<D, 2, N, N, N, N, N, PM_STORE, TM>(buf, buf, nslices, M);
    __syncthreads();
  }
}

// Ricker wavelet and its l-th time derivative:
// s^(l)(t) = -amp/(2a) (-sqrt a)^(l+2) H_{l+2}(sqrt(a) tau) exp(-a tau^2).
__device__ inline double ricker_deriv(const double* w, double t, int l) {
  const double f = w[0], t0 = w[1], amp = w[2];
  const double a = M_PI * M_PI * f * f, sa = sqrt(a), tau = t - t0, x = sa * tau;
  double h0 = 1.0, h1 = 2.0 * x;
  for (int m = 1; m < l + 2; ++m) {
    const double h2 = 2.0 * x * h1 - 2.0 * m * h0;
    h0 = h1;
    h1 = h2;
  }
  double pw = 1.0;
  for (int m = 0; m < l + 2; ++m) pw *= -sa;
  return -amp / (2.0 * a) * pw * h1 * exp(-a * tau * tau);
}
__device__ inline double ricker_integral(const double* w, double t1, double t2) {
  const double t0 = w[1], amp = w[2], a = M_PI * M_PI * w[0] * w[0];
  const double x1 = t1 - t0, x2 = t2 - t0;
  return amp * (x2 * exp(-a * x2 * x2) - x1 * exp(-a * x1 * x1));
}

// ------------------------------------------------------------------------
// Fused operator sweep: L u = -M^-1 K u with an epilogue.
// ------------------------------------------------------------------------
template <int D, int N, typename T>
struct OpLayout {
  static constexpr int NC = D + 1, NP = ipow(N, D), NF = ipow(N, D - 1), NFACE = 2 * D;
  static constexpr int per_cell = 2 * NC * NP + NFACE * NC * NF;  // elements of T
};

template <int D, int N, typename T, int DIR>
__device__ __forceinline__ void op_direction(const OpParams& p, const T* sU, T* sR, const T* sN,
                                             int64_t cell0, int ncl) {
  using Lay = OpLayout<D, N, T>;
  constexpr int NC = Lay::NC, NP = Lay::NP, NF = Lay::NF, NFACE = Lay::NFACE;
  using P = Pass<D, DIR, N, N, N, N, N>;
  const T* tab = static_cast<const T*>(p.tab);
  const T* Dm = tab + tab_D(N);
  const T* LF0 = tab + tab_LF0(N);
  const T* LF1 = tab + tab_LF1(N);
  const int total = ncl * NF;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int c = w / NF;
    const int L = w - c * NF;
    const int64_t cell = cell0 + c;
    int bq, bq2;
    P::base(L, bq, bq2);
    const T* su = sU + c * NC * NP;
    T x[NC][N];
#pragma unroll
    for (int v = 0; v < NC; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) x[v][j] = su[v * NP + bq + j * P::STEP_IN];
    // volume fluxes in FP64 metric: F_{v_a} = G_{ba} p, F_p = sum_a G_{ba} v_a
    const double* G = p.geo_cell + cell * (int64_t)((D * D + 2) * NP) + bq;
    T F[NC][N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double pj = (double)x[D][j];
      double fp = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double g = G[(DIR * D + a) * NP + j * P::STEP_IN];
        F[a][j] = (T)(g * pj);
        fp = fma(g, (double)x[a][j], fp);
      }
      F[D][j] = (T)fp;
    }
    // R_i = sum_j D[j][i] F_j  (transposed collocation derivative)
    T R[NC][N];
#pragma unroll
    for (int v = 0; v < NC; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = Dm[i] * F[v][0];
#pragma unroll
        for (int j = 1; j < N; ++j) acc = fma(Dm[j * N + i], F[v][j], acc);
        R[v][i] = acc;
      }
    // the two faces normal to DIR
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* LF = s == 0 ? LF0 : LF1;
      const int f = 2 * DIR + s;
      double um[NC], up[NC];
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        T acc = LF[0] * x[v][0];
#pragma unroll
        for (int j = 1; j < N; ++j) acc = fma(LF[j], x[v][j], acc);
        um[v] = (double)acc;
        up[v] = (double)sN[((c * NFACE + f) * NC + v) * NF + L];
      }
      const double* fg = p.geo_face + ((cell * NFACE + f) * (int64_t)(D + 2)) * NF + L;
      double a[D];
      double area2 = 0.0, vnm = 0.0, vnp = 0.0;
#pragma unroll
      for (int e = 0; e < D; ++e) {
        a[e] = fg[e * NF];
        area2 = fma(a[e], a[e], area2);
        vnm = fma(a[e], um[e], vnm);
        vnp = fma(a[e], up[e], vnp);
      }
      const double area = sqrt(area2);
      vnm /= area;
      vnp /= area;
      double ps, vs;
      if (p.central) {
        ps = 0.5 * (um[D] + up[D]);
        vs = 0.5 * (vnm + vnp);
      } else {
        const double Zm = fg[D * NF], Zp = fg[(D + 1) * NF];
        const double inv = 1.0 / (Zm + Zp);
        ps = (Zp * um[D] + Zm * up[D] + Zm * Zp * (vnm - vnp)) * inv;
        vs = (Zm * vnm + Zp * vnp + um[D] - up[D]) * inv;
      }
      T fl[NC];
#pragma unroll
      for (int e = 0; e < D; ++e) fl[e] = (T)(-a[e] * ps);
      fl[D] = (T)(-area * vs);
#pragma unroll
      for (int v = 0; v < NC; ++v)
#pragma unroll
        for (int i = 0; i < N; ++i) R[v][i] = fma(LF[i], fl[v], R[v][i]);
    }
    T* sr = sR + c * NC * NP;
#pragma unroll
    for (int v = 0; v < NC; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int q = v * NP + bq + i * P::STEP_IN;
        if constexpr (DIR == 0)
          sr[q] = R[v][i];
        else
          sr[q] += R[v][i];
      }
  }
}

template <int D, int N, typename T, int EPI>
__global__ void __launch_bounds__(256) op_kernel(OpParams p) {
  using Lay = OpLayout<D, N, T>;
  constexpr int NC = Lay::NC, NP = Lay::NP, NF = Lay::NF, NFACE = Lay::NFACE;
  extern __shared__ __align__(16) unsigned char smem[];
  T* sU = reinterpret_cast<T*>(smem);
  T* sR = sU + p.cpw * NC * NP;
  T* sN = sR + p.cpw * NC * NP;
  const T* tab = static_cast<const T*>(p.tab);

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int member = logical % p.B;
  const int group = logical / p.B;
  const int64_t cell0 = (int64_t)group * p.cpw;
  const int ncl = (int)min((int64_t)p.cpw, p.nc - cell0);
  const int64_t moff = (int64_t)member * p.nc * NC * NP;
  const double* u = p.u + moff;

  // A: cell tiles (contiguous) and neighbour GL face nodes
  {
    const double* src = u + cell0 * NC * NP;
    for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) sU[i] = (T)src[i];
    const int tot = ncl * NFACE * NC * NF;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) {
      const int t = i % NF;
      int r = i / NF;
      const int v = r % NC;
      r /= NC;
      const int f = r % NFACE;
      const int c = r / NFACE;
      const int nbc = p.nb[(cell0 + c) * NFACE + f];
      // GL node on the neighbour's face opposite to f, tangential index t
      const int fo = f ^ 1, dir = fo >> 1, side = fo & 1;
      const int st = dir == 0 ? 1 : (dir == 1 ? N : N * N);
      const int q = (t % st) + (side ? (N - 1) * st : 0) + (t / st) * st * N;
      sN[i] = (T)u[(int64_t)nbc * NC * NP + v * NP + q];
    }
  }
  __syncthreads();
  // B: GL -> G of the cell tiles; tangential GL -> G of the neighbour traces
  {
    const T* S = tab + tab_S(N);
    tpass<D, 0, N, N, N, N, N, PM_STORE, T>(sU, sU, ncl * NC, S);
    if constexpr (D == 2) tpass<1, 0, N, N, N, N, N, PM_STORE, T>(sN, sN, ncl * NFACE * NC, S);
    if constexpr (D == 3) tpass<2, 0, N, N, N, N, N, PM_STORE, T>(sN, sN, ncl * NFACE * NC, S);
    __syncthreads();
    tpass<D, 1, N, N, N, N, N, PM_STORE, T>(sU, sU, ncl * NC, S);
    if constexpr (D == 3) tpass<2, 1, N, N, N, N, N, PM_STORE, T>(sN, sN, ncl * NFACE * NC, S);
    __syncthreads();
    if constexpr (D == 3) {
      tpass<D, 2, N, N, N, N, N, PM_STORE, T>(sU, sU, ncl * NC, S);
      __syncthreads();
    }
  }
  // C: volume and face integrals, one direction at a time
  op_direction<D, N, T, 0>(p, sU, sR, sN, cell0, ncl);
  __syncthreads();
  op_direction<D, N, T, 1>(p, sU, sR, sN, cell0, ncl);
  __syncthreads();
  if constexpr (D == 3) {
    op_direction<D, N, T, 2>(p, sU, sR, sN, cell0, ncl);
    __syncthreads();
  }
  // D: inverse mass (pointwise, FP64 factors) then G -> GL
  {
    for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) {
      const int q = i % NP;
      const int r = i / NP;
      const int v = r % NC;
      const int c = r / NC;
      const double mu = p.geo_cell[(cell0 + c) * (int64_t)((D * D + 2) * NP) + (D * D + (v == D)) * NP + q];
      sR[i] = (T)(mu * (double)sR[i]);
    }
    __syncthreads();
    tensor_apply_inplace<D, N, T>(sR, ncl * NC, tab + tab_Sinv(N));
  }
  // E: epilogue (coalesced)
  {
    const int64_t gofs = moff + cell0 * NC * NP;
    int scell = -1;
    if (p.src.cell) scell = p.src.cell[member];
    const bool has_src = scell >= cell0 && scell < cell0 + ncl;
    double sval = 0.0;
    if (has_src) {
      const double tn = p.time.tn();
      if constexpr (EPI == EPI_LSRK) sval = ricker_deriv(p.src.wave + 3 * member, tn + p.time.t_off, 0);
      if constexpr (EPI == EPI_ADD) sval = ricker_integral(p.src.wave + 3 * member, tn, tn + p.time.dt);
    }
    for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) {
      double val = (double)sR[i];
      const int64_t gi = gofs + i;
      if constexpr (EPI == EPI_STORE) {
        p.out[gi] = val;
      } else {
        double add = 0.0;
        if (has_src) {
          const int c = i / (NC * NP);
          const int v = (i / NP) % NC;
          if (cell0 + c == scell && v == D) add = sval * p.src.gvec[(int64_t)member * NP + (i % NP)];
        }
        if constexpr (EPI == EPI_LSRK) {
          const double d = (p.acoef == 0.0 ? 0.0 : p.acoef * p.du[gi]) + p.dt * (val + add);
          p.du[gi] = d;
          p.u_next[gi] = p.u[gi] + p.bcoef * d;
        } else {
          p.u_next[gi] = p.u_base[gi] + val + add;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------
// ADER sweep 1: Taylor-Cauchy-Kowalevski sum in the collocated Gauss basis
// with the degree reduction (Sec. 3.2, 3.3).  Buffers: three T tiles
// (current derivative, next derivative, scratch) and the FP64 accumulator.
// ------------------------------------------------------------------------
template <int D, int N, typename T>
struct TckLayout {
  static constexpr int NC = D + 1, NP = ipow(N, D);
  static constexpr int bytes_per_cell = 3 * NC * NP * (int)sizeof(T) + NC * NP * 8;
};

template <int D, int N, typename T, bool REDUCE, int M, int NL, int CUR>
struct TckStep {
  __device__ static void run(const TckParams& p, T* const* bufs, double* sI, int64_t cell0, int ncl,
                             int member) {
    constexpr int NC = D + 1, NP = ipow(N, D), NPL = ipow(NL, D);
    if constexpr (M > N || NL < 1) {
      return;
    } else {
      constexpr int LVL = (N - NL) / 2;  // index of the Gauss set with NL points
      constexpr int NXT = (CUR + 1) % 3, SCR = (CUR + 2) % 3;
      const T* tab = static_cast<const T*>(p.tab);
      T* cur = bufs[CUR];
      T* w = bufs[NXT];
      const double* G = p.geo_lev[LVL];
      // w = -S_loc cur: accumulate over directions G_{ba} d_b p and sum_a G_{ba} d_b v_a
      if constexpr (NL > 1) {
        const T* Dl = tab + (LVL == 0 ? tab_D(N) : tab_level_D(N, LVL));
        tck_deriv<0>(p, cur, w, G, Dl, cell0, ncl);
        __syncthreads();
        tck_deriv<1>(p, cur, w, G, Dl, cell0, ncl);
        __syncthreads();
        if constexpr (D == 3) {
          tck_deriv<2>(p, cur, w, G, Dl, cell0, ncl);
          __syncthreads();
        }
      }
      // scale by -1/(w detJ rho), -rho c^2/(w detJ); source injection s^(M-1)(t) g
      {
        int scell = -1;
        if (p.src.cell) scell = p.src.cell[member];
        double sd = 0.0;
        if (scell >= cell0 && scell < cell0 + ncl) sd = ricker_deriv(p.src.wave + 3 * member, p.time.tn(), M - 1);
        for (int i = threadIdx.x; i < ncl * NC * NPL; i += blockDim.x) {
          const int q = i % NPL;
          const int r = i / NPL;
          const int v = r % NC;
          const int c = r / NC;
          double val = 0.0;
          if constexpr (NL > 1) {
            const double mu = G[(cell0 + c) * (int64_t)((D * D + 2) * NPL) + (D * D + (v == D)) * NPL + q];
            val = -mu * (double)w[(c * NC + v) * NP + q];
          }
          if (v == D && cell0 + c == scell) val += sd * p.src.glev[LVL][(int64_t)member * NPL + q];
          w[(c * NC + v) * NP + q] = (T)val;
        }
        __syncthreads();
      }
      constexpr double coef = taylor_coef(M);
      if constexpr (REDUCE && (M % 2 == 0)) {
        constexpr int NR = NL - 2;
        if constexpr (NR >= 1) {
          // project w (NL^D) to NR^D, ping-pong w -> cur -> w (-> cur)
          const T* Pm = tab + tab_level_P(N, LVL + 1);
          project<NR>(w, cur, ncl, Pm);
          constexpr int RES = (D == 3) ? CUR : NXT;
          accumulate<NR, RES>(p, bufs, sI, ncl, coef * dtpow<M + 1>(p.dt), LVL + 1);
          TckStep<D, N, T, REDUCE, M + 1, NR, RES>::run(p, bufs, sI, cell0, ncl, member);
        }
      } else {
        accumulate<NL, NXT>(p, bufs, sI, ncl, coef * dtpow<M + 1>(p.dt), LVL);
        TckStep<D, N, T, REDUCE, M + 1, NL, NXT>::run(p, bufs, sI, cell0, ncl, member);
      }
    }
  }

  static constexpr double taylor_coef(int m) {
    double f = 1.0;
    for (int j = 2; j <= m + 1; ++j) f *= j;
    return 1.0 / f;
  }
  template <int E>
  __device__ static __forceinline__ double dtpow(double dt) {
    double r = 1.0;
#pragma unroll
    for (int j = 0; j < E; ++j) r *= dt;
    return r;
  }

  template <int DIR>
  __device__ static __forceinline__ void tck_deriv(const TckParams& p, const T* cur, T* w, const double* G,
                                                   const T* Dl, int64_t cell0, int ncl) {
    constexpr int NC = D + 1, NP = ipow(N, D), NPL = ipow(NL, D);
    using P = Pass<D, DIR, NL, NL, NL, NL, NL>;
    const int total = ncl * P::NL;
    for (int wi = threadIdx.x; wi < total; wi += blockDim.x) {
      const int c = wi / P::NL;
      const int L = wi - c * P::NL;
      int bq, bq2;
      P::base(L, bq, bq2);
      T x[NC][NL];
#pragma unroll
      for (int v = 0; v < NC; ++v)
#pragma unroll
        for (int j = 0; j < NL; ++j) x[v][j] = cur[(c * NC + v) * NP + bq + j * P::STEP_IN];
      T dx[NC][NL];
#pragma unroll
      for (int v = 0; v < NC; ++v)
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          T acc = Dl[i * NL] * x[v][0];
#pragma unroll
          for (int j = 1; j < NL; ++j) acc = fma(Dl[i * NL + j], x[v][j], acc);
          dx[v][i] = acc;
        }
      const double* g = G + (cell0 + c) * (int64_t)((D * D + 2) * NPL) + bq;
      T* wc = w + c * NC * NP + bq;
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int q = i * P::STEP_IN;
        double dv = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double gba = g[(DIR * D + a) * NPL + q];
          const T va = (T)(gba * (double)dx[D][i]);
          dv = fma(gba, (double)dx[a][i], dv);
          if constexpr (DIR == 0)
            wc[a * NP + q] = va;
          else
            wc[a * NP + q] += va;
        }
        if constexpr (DIR == 0)
          wc[D * NP + q] = (T)dv;
        else
          wc[D * NP + q] += (T)dv;
      }
    }
  }

  // Projection P (NR x NL) along every direction: src (NL^D) -> ... ; the
  // intermediate tensors use the NP-strided slices of the two buffers.
  template <int NR>
  __device__ static __forceinline__ void project(T* w, T* cur, int ncl, const T* Pm) {
    constexpr int NC = D + 1, NP = ipow(N, D);
    // slices are NP apart; Pass uses dense sub-tensors of its own extents
    proj_pass<0, NL, NL, NL, NR>(w, cur, ncl, Pm);
    __syncthreads();
    proj_pass<1, NR, NL, NL, NR>(cur, w, ncl, Pm);
    __syncthreads();
    if constexpr (D == 3) {
      proj_pass<2, NR, NR, NL, NR>(w, cur, ncl, Pm);
      __syncthreads();
    }
    (void)NC;
    (void)NP;
  }

  // One pass of a size-changing 1D matrix (MO x MI) along DIR between two
  // buffers whose cell-component slices are NP apart.
  template <int DIR, int E0, int E1, int E2, int MO>
  __device__ static __forceinline__ void proj_pass(const T* in, T* out, int ncl, const T* Mx) {
    constexpr int NC = D + 1, NP = ipow(N, D);
    constexpr int MI = DIR == 0 ? E0 : (DIR == 1 ? E1 : E2);
    using P = Pass<D, DIR, MI, MO, E0, E1, E2>;
    const int total = ncl * NC * P::NL;
    for (int wi = threadIdx.x; wi < total; wi += blockDim.x) {
      const int s = wi / P::NL;
      const int L = wi - s * P::NL;
      int bi, bo;
      P::base(L, bi, bo);
      const T* src = in + s * NP + bi;
      T* dst = out + s * NP + bo;
      T x[MI];
#pragma unroll
      for (int j = 0; j < MI; ++j) x[j] = src[j * P::STEP_IN];
#pragma unroll
      for (int i = 0; i < MO; ++i) {
        T acc = Mx[i * MI] * x[0];
#pragma unroll
        for (int j = 1; j < MI; ++j) acc = fma(Mx[i * MI + j], x[j], acc);
        dst[i * P::STEP_OUT] = acc;
      }
    }
  }

  // sI += scale * E (level NLm -> N) of bufs[RES]; uses the two other buffers
  // as scratch for the size-changing passes.
  template <int NLm, int RES>
  __device__ static __forceinline__ void accumulate(const TckParams& p, T* const* bufs, double* sI, int ncl,
                                                    double scale, int lvl) {
    constexpr int NC = D + 1, NP = ipow(N, D);
    const T* src = bufs[RES];
    if constexpr (NLm == N) {
      for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) sI[i] += scale * (double)src[i];
      __syncthreads();
    } else {
      const T* tab = static_cast<const T*>(p.tab);
      const T* E = tab + tab_level_E(N, (N - NLm) / 2);
      T* s1 = bufs[(RES + 1) % 3];
      T* s2 = bufs[(RES + 2) % 3];
      proj_pass<0, NLm, NLm, NLm, N>(src, s1, ncl, E);
      __syncthreads();
      if constexpr (D == 2) {
        emb_last<1, N, NLm, 1>(s1, sI, ncl, E, scale);
        __syncthreads();
      } else {
        proj_pass<1, N, NLm, NLm, N>(s1, s2, ncl, E);
        __syncthreads();
        emb_last<2, N, N, NLm>(s2, sI, ncl, E, scale);
        __syncthreads();
      }
    }
    (void)lvl;
  }

  template <int DIR, int E0, int E1, int E2>
  __device__ static __forceinline__ void emb_last(const T* in, double* sI, int ncl, const T* Mx, double scale) {
    constexpr int NC = D + 1, NP = ipow(N, D);
    constexpr int MI = DIR == 0 ? E0 : (DIR == 1 ? E1 : E2);
    using P = Pass<D, DIR, MI, N, E0, E1, E2>;
    const int total = ncl * NC * P::NL;
    for (int wi = threadIdx.x; wi < total; wi += blockDim.x) {
      const int s = wi / P::NL;
      const int L = wi - s * P::NL;
      int bi, bo;
      P::base(L, bi, bo);
      const T* src = in + s * NP + bi;
      double* dst = sI + s * NP + bo;
      T x[MI];
#pragma unroll
      for (int j = 0; j < MI; ++j) x[j] = src[j * P::STEP_IN];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = Mx[i * MI] * x[0];
#pragma unroll
        for (int j = 1; j < MI; ++j) acc = fma(Mx[i * MI + j], x[j], acc);
        dst[i * P::STEP_OUT] += scale * (double)acc;
      }
    }
  }
};

template <int D, int N, typename T, bool REDUCE>
__global__ void __launch_bounds__(256) tck_kernel(TckParams p) {
  constexpr int NC = D + 1, NP = ipow(N, D);
  extern __shared__ __align__(16) unsigned char smem[];
  double* sI = reinterpret_cast<double*>(smem);
  T* b0 = reinterpret_cast<T*>(sI + p.cpw * NC * NP);
  T* bufs[3] = {b0, b0 + p.cpw * NC * NP, b0 + 2 * p.cpw * NC * NP};
  const T* tab = static_cast<const T*>(p.tab);

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int member = logical % p.B;
  const int group = logical / p.B;
  const int64_t cell0 = (int64_t)group * p.cpw;
  const int ncl = (int)min((int64_t)p.cpw, p.nc - cell0);
  const int64_t gofs = (int64_t)member * p.nc * NC * NP + cell0 * NC * NP;

  for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) bufs[0][i] = (T)p.u[gofs + i];
  __syncthreads();
  tensor_apply_inplace<D, N, T>(bufs[0], ncl * NC, tab + tab_S(N));
  for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) sI[i] = p.dt * (double)bufs[0][i];
  __syncthreads();
  TckStep<D, N, T, REDUCE, 1, N, 0>::run(p, bufs, sI, cell0, ncl, member);
  // G -> GL of the FP64 accumulator, then store
  tensor_apply_inplace<D, N, double>(sI, ncl * NC, p.tab64 + tab_Sinv(N));
  for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) p.I[gofs + i] = sI[i];
}

// ------------------------------------------------------------------------
// Energy sum_q |v|^2 / mu_v + p^2 / mu_p at the Gauss points (per group).
// ------------------------------------------------------------------------
template <int D, int N, typename T>
__global__ void __launch_bounds__(256) energy_kernel(EnergyParams p) {
  constexpr int NC = D + 1, NP = ipow(N, D);
  extern __shared__ __align__(16) unsigned char smem[];
  T* sU = reinterpret_cast<T*>(smem);
  __shared__ double red[256];
  const T* tab = static_cast<const T*>(p.tab);
  const int logical = blockIdx.x;
  const int member = logical % p.B;
  const int group = logical / p.B;
  const int64_t cell0 = (int64_t)group * p.cpw;
  const int ncl = (int)min((int64_t)p.cpw, p.nc - cell0);
  const int64_t gofs = (int64_t)member * p.nc * NC * NP + cell0 * NC * NP;
  for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) sU[i] = (T)p.u[gofs + i];
  __syncthreads();
  tensor_apply_inplace<D, N, T>(sU, ncl * NC, tab + tab_S(N));
  double acc = 0.0;
  for (int i = threadIdx.x; i < ncl * NC * NP; i += blockDim.x) {
    const int q = i % NP;
    const int r = i / NP;
    const int v = r % NC;
    const int c = r / NC;
    const double mu = p.geo_cell[(cell0 + c) * (int64_t)((D * D + 2) * NP) + (D * D + (v == D)) * NP + q];
    const double x = (double)sU[i];
    acc += x * x / mu;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.partial[(int64_t)member * p.groups + group] = red[0];
}

}  // namespace dgw
