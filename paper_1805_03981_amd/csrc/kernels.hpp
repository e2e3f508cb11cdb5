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
//      upwind flux; lift, rank one in the normal direction); the residual
//      is summed over the directions in registers of the point's thread
//   D  inverse mass in the collocated basis: pointwise 1/(w detJ rho),
//      rho c^2/(w detJ), then G -> GL (Sec. 3.1, inverse via basis change)
//   E  epilogue: store, fused low-storage Runge-Kutta update, or ADER update
#pragma once
#include <hip/hip_runtime.h>

#include "dgw_params.hpp"

namespace dgw {

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Threads per workgroup (op_threads, tck_threads in dgw_params.hpp): 256,
// wider for the largest 3D cells.  Below, NT is the thread count of the
// kernel being compiled.

// 1D tables of every degree (layout tab_base / tab_*) in constant memory:
// uniform reads of the matrix entries go through the scalar cache.  Each
// translation unit has its own copy, filled by its upload function.
static __constant__ double c_tab64[kTabTotal];
static __constant__ float c_tab32[kTabTotal];
template <typename T>
__device__ __forceinline__ const T* ctab(int n);
template <>
__device__ __forceinline__ const double* ctab<double>(int n) {
  return c_tab64 + tab_base(n);
}
template <>
__device__ __forceinline__ const float* ctab<float>(int n) {
  return c_tab32 + tab_base(n);
}

// Cells per workgroup of the two compiled launch shapes: sel 0 gives about
// one cell point per thread of a 256-thread group (one cell for larger
// cells, whatever the group width), sel 1 twice as many cells.
__host__ __device__ constexpr int cells_per_group(int d, int n, int sel) {
  return (256 / ipow(n, d) > 1 ? 256 / ipow(n, d) : 1) * (sel + 1);
}

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
  // extents of the input (direction DIR has MI entries) and output (MO)
  static constexpr int EI0 = DIR == 0 ? MI : A0, EI1 = DIR == 1 ? MI : A1, EI2 = DIR == 2 ? MI : A2;
  static constexpr int EO0 = DIR == 0 ? MO : A0, EO1 = DIR == 1 ? MO : A1, EO2 = DIR == 2 ? MO : A2;
  // strides (x fastest), plain constants: no recursion for the compiler to keep
  static constexpr int SI0 = 1, SI1 = EI0, SI2 = EI0 * EI1;
  static constexpr int SO0 = 1, SO1 = EO0, SO2 = EO0 * EO1;
  static constexpr int SIN = D == 1 ? EI0 : (D == 2 ? EI0 * EI1 : EI0 * EI1 * EI2);
  static constexpr int SOUT = D == 1 ? EO0 : (D == 2 ? EO0 * EO1 : EO0 * EO1 * EO2);
  static constexpr int NL = SIN / MI;  // lines: product of the other input extents
  static constexpr int STEP_IN = DIR == 0 ? SI0 : (DIR == 1 ? SI1 : SI2);
  static constexpr int STEP_OUT = DIR == 0 ? SO0 : (DIR == 1 ? SO1 : SO2);
  // input / output offset of the start of line L (the other coordinates in
  // increasing direction order, first fastest)
  __device__ static __forceinline__ void base(int L, int& bi, int& bo) {
    if constexpr (D == 1) {
      bi = 0;
      bo = 0;
    } else if constexpr (D == 2) {
      if constexpr (DIR == 0) {
        bi = L * SI1;
        bo = L * SO1;
      } else {
        bi = L;
        bo = L;
      }
    } else {
      if constexpr (DIR == 0) {
        const int c1 = L % EI1, c2 = L / EI1;
        bi = c1 * SI1 + c2 * SI2;
        bo = c1 * SO1 + c2 * SO2;
      } else if constexpr (DIR == 1) {
        const int c0 = L % EI0, c2 = L / EI0;
        bi = c0 + c2 * SI2;
        bo = c0 + c2 * SO2;
      } else {
        const int c0 = L % EI0, c1 = L / EI0;
        bi = c0 + c1 * SI1;
        bo = c0 + c1 * SO1;
      }
    }
  }
};

enum PassMode { PM_STORE = 0, PM_ADD_SCALED = 1 };

// acc = M x for an MO x MI matrix (row-major), written column by column so
// that the MO accumulations are independent chains (FMA latency overlaps).
template <int MI, int MO, typename TM>
__device__ __forceinline__ void contract(const TM* __restrict__ M, const TM (&x)[MI], TM (&acc)[MO]) {
#pragma unroll
  for (int i = 0; i < MO; ++i) acc[i] = M[i * MI] * x[0];
#pragma unroll
  for (int j = 1; j < MI; ++j)
#pragma unroll
    for (int i = 0; i < MO; ++i) acc[i] = fma(M[i * MI + j], x[j], acc[i]);
}

// Zero, opaque to the compiler (a scalar register it cannot see through).
// A phase that addresses its matrix with it loads the entries itself: they
// are not merged with the same entries loaded by an earlier phase, whose
// values would otherwise be kept in scalar registers across the kernel and,
// at n >= 7 where one n x n FP64 matrix alone exceeds the scalar register
// file, spilled to vector lanes and read back entry by entry.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Whether the operator sweep addresses each 1D phase's matrix with its own
// opaque zero and visits the phase's lines in unrolled rounds: where an
// n x n matrix fills most of the scalar registers (FP64 from n = 7, FP32
// from n = 8).  Measured A/B on one box: at k = 6, 7, 8 in FP64 the LSRK
// stage ran 1.3x, 2.3x, 2.2x and the ADER update 1.4x, 1.6x, 1.8x faster,
// in FP32 at k = 7, 8 by 1-5 %; at k = 5 the same change cost 2-6 %, so
// smaller matrices keep the plain loops.
template <int N, typename T>
constexpr bool op_phase_tables() {
  return N >= (sizeof(T) == 8 ? 7 : 8);
}

// out = M in along DIR, for nslices independent tensors (cells x components).
// in and out may be the same buffer when MI == MO (each line is read whole
// before it is written, and lines are disjoint).  MAXS > 0: nslices is at
// most MAXS, and the lines are visited in a fixed number of unrolled rounds
// (the matrix entries are then loaded where they are used, not hoisted out
// of a loop and spilled); MAXS = 0: a loop over any number of slices.
template <int NT, int D, int DIR, int MI, int MO, int A0, int A1, int A2, int MODE, int MAXS, typename TM,
          typename TI, typename TO>
__device__ __forceinline__ void tpass(const TI* in, TO* out, int nslices, const TM* __restrict__ M,
                                      double scale = 1.0) {
  using P = Pass<D, DIR, MI, MO, A0, A1, A2>;
  const int total = nslices * P::NL;
  auto line = [&](int w) {
    const int s = w / P::NL;
    const int L = w - s * P::NL;
    int bi, bo;
    P::base(L, bi, bo);
    const TI* src = in + s * P::SIN + bi;
    TO* dst = out + s * P::SOUT + bo;
    TM x[MI];
#pragma unroll
    for (int j = 0; j < MI; ++j) x[j] = (TM)src[j * P::STEP_IN];
    TM acc[MO];
    contract<MI, MO>(M, x, acc);
#pragma unroll
    for (int i = 0; i < MO; ++i) {
      if constexpr (MODE == PM_STORE)
        dst[i * P::STEP_OUT] = (TO)acc[i];
      else
        dst[i * P::STEP_OUT] += (TO)(scale * (double)acc[i]);
    }
  };
  if constexpr (MAXS > 0) {
#pragma unroll
    for (int it = 0; it < cdiv(MAXS * P::NL, NT); ++it) {
      const int w = threadIdx.x + it * NT;
      if (w >= total) break;
      line(w);
    }
  } else {
    for (int w = threadIdx.x; w < total; w += NT) line(w);
  }
}

// Apply the same n x n matrix along all D directions in place (square passes);
// MAXS as in tpass.
template <int NT, int D, int N, int MAXS, typename TM, typename TT>
__device__ __forceinline__ void tensor_apply_inplace(TT* buf, int nslices, const TM* M) {
  tpass<NT, D, 0, N, N, N, N, N, PM_STORE, MAXS, TM>(buf, buf, nslices, M);
  __syncthreads();
  tpass<NT, D, 1, N, N, N, N, N, PM_STORE, MAXS, TM>(buf, buf, nslices, M);
  __syncthreads();
  if constexpr (D == 3) {
    tpass<NT, D, 2, N, N, N, N, N, PM_STORE, MAXS, TM>(buf, buf, nslices, M);
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
//
// Every global operand of the sweep (the workgroup's state tile, the
// neighbours' GL face nodes, the metric and mass factors of every point, the
// face area vectors and impedances) is requested in one batch at the start.
// The geometry stays in registers of the thread that owns the point
// (thread-per-point phases) or the face point, so its memory latency
// overlaps the basis-change passes and only one memory round trip per
// workgroup is exposed before the sweep; the epilogue's second state
// operand is requested after the sweep, its latency hidden by phase D.
// ------------------------------------------------------------------------
template <int D, int N, typename T>
struct OpLayout {
  static constexpr int NC = D + 1, NP = ipow(N, D), NF = ipow(N, D - 1), NFACE = 2 * D;
  // state and flux tiles, neighbour traces (elements of T); the residual
  // is accumulated in registers of the point's thread
  static constexpr int per_cell = 2 * NC * NP + NFACE * NC * NF;
};

// Register budget of the operator sweep: with one cell point per thread of
// a 256-thread group it is compiled for the waves per SIMD that its LDS
// allows, capped at 6 (80 VGPRs) and at 5 (96 VGPRs) for the FP64 LSRK
// epilogue, which keeps the stage state in registers across the sweep (at 6
// it would spill 44 bytes per lane).  The member-block variant (MB > 1)
// keeps its geometry registers live across its loop over members and gets
// no budget (measured on the 64-source batch at k = 5 FP32: capped at 5
// waves it spills and runs 1.7x slower than one member per workgroup).
template <int D, int N, typename T, int EPI, int CPW, int MB = 1>
constexpr int op_waves_per_simd() {
  if (MB != 1 || op_threads(D, N) != 256 || cdiv(CPW * ipow(N, D), 256) > 1) return 1;
  const int wg = (160 * 1024) / (CPW * OpLayout<D, N, T>::per_cell * (int)sizeof(T));
  const int cap = (EPI == EPI_LSRK && sizeof(T) == 8) ? 5 : 6;
  return wg < 1 ? 1 : (wg > cap ? cap : wg);
}

__device__ __forceinline__ int dir_stride(int n, int dir) { return dir == 0 ? 1 : (dir == 1 ? n : n * n); }

// Offset of the start of the line along `dir` through tangential face index
// t (the other coordinates in increasing direction order, first fastest):
// (t % st) + (t / st) st N with st = N^dir, written with constant divisors.
template <int D, int N>
__device__ __forceinline__ int face_line_base(int dir, int t) {
  if constexpr (D == 2) return dir == 0 ? t * N : t;
  return dir == 0 ? t * N : (dir == 1 ? (t % N) + (t / N) * N * N : t);
}

// Tangential index on the neighbour's face of own face index t under
// orientation o: bit 2 swaps the two tangential indices, then bit 0 reverses
// the first and bit 1 the second (2D: bit 0 reverses the only one).  The GL
// nodes are symmetric about the cell centre, so a reversal is i -> N-1-i.
template <int D, int N>
__device__ __forceinline__ int orient_face(int o, int t) {
  if constexpr (D == 2) return (o & 1) ? N - 1 - t : t;
  int i = t % N, j = t / N;
  if (o & 4) {
    const int x = i;
    i = j;
    j = x;
  }
  if (o & 1) i = N - 1 - i;
  if (o & 2) j = N - 1 - j;
  return i + N * j;
}

// C2 of the operator: D_b^T F along the b-lines plus the lifts of the two
// face fluxes of direction b (rank one in the normal direction), written
// over F in sT (a line is read whole before it is written; lines are
// disjoint).  The point phase that follows adds it to the residual.
template <int D, int N, typename T, int DIR>
__device__ __forceinline__ void op_lines(const T* __restrict__ tab, T* sT, const T* sN, int ncl) {
  constexpr int NC = D + 1, NP = ipow(N, D), NF = ipow(N, D - 1), NFACE = 2 * D;
  using P = Pass<D, DIR, N, N, N, N, N>;
  const T* Dm = tab + tab_D(N);
  const T* LF0 = tab + tab_LF0(N);
  const T* LF1 = tab + tab_LF1(N);
  constexpr int NT = op_threads(D, N);
  for (int w = threadIdx.x; w < ncl * NC * NF; w += NT) {
    const int sl = w / NF;  // c * NC + v
    const int L = w - sl * NF;
    const int c = sl / NC, v = sl - c * NC;
    int bq, bq2;
    P::base(L, bq, bq2);
    T* ln = sT + sl * NP + bq;
    T F[N];
#pragma unroll
    for (int j = 0; j < N; ++j) F[j] = ln[j * P::STEP_IN];
    const T f0 = sN[((c * NFACE + 2 * DIR) * NC + v) * NF + L];
    const T f1 = sN[((c * NFACE + 2 * DIR + 1) * NC + v) * NF + L];
    T acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = fma(LF1[i], f1, LF0[i] * f0);
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = fma(Dm[j * N + i], F[j], acc[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) ln[i * P::STEP_IN] = acc[i];
  }
}

// op_lines for large matrices (op_phase_tables): the phase loads its own
// matrix entries (an opaque zero offset) and visits its lines in a fixed
// number of unrolled rounds.
template <int D, int N, typename T, int DIR, int CPW>
__device__ __forceinline__ void op_lines_pt(const T* __restrict__ tab, T* sT, const T* sN, int ncl) {
  constexpr int NC = D + 1, NP = ipow(N, D), NF = ipow(N, D - 1), NFACE = 2 * D;
  using P = Pass<D, DIR, N, N, N, N, N>;
  const int off = opaque_zero();
  const T* Dm = tab + tab_D(N) + off;
  const T* LF0 = tab + tab_LF0(N) + off;
  const T* LF1 = tab + tab_LF1(N) + off;
  constexpr int NT = op_threads(D, N);
  constexpr int ROUNDS = cdiv(CPW * NC * NF, NT);
#pragma unroll
  for (int it = 0, w = threadIdx.x; it < ROUNDS && w < ncl * NC * NF; ++it, w += NT) {
    const int sl = w / NF;  // c * NC + v
    const int L = w - sl * NF;
    const int c = sl / NC, v = sl - c * NC;
    int bq, bq2;
    P::base(L, bq, bq2);
    T* ln = sT + sl * NP + bq;
    T F[N];
#pragma unroll
    for (int j = 0; j < N; ++j) F[j] = ln[j * P::STEP_IN];
    const T f0 = sN[((c * NFACE + 2 * DIR) * NC + v) * NF + L];
    const T f1 = sN[((c * NFACE + 2 * DIR + 1) * NC + v) * NF + L];
    T acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = fma(LF1[i], f1, LF0[i] * f0);
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = fma(Dm[j * N + i], F[j], acc[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) ln[i * P::STEP_IN] = acc[i];
  }
}

// C1 of the operator: the residual of the previous direction's lines (in sT
// at the point) is added to the registers R, then the pointwise volume
// fluxes of direction b in FP64, F_{v_a} = G_{ba} p, F_p = sum_a G_{ba} v_a
// with G = w det J J^-1, are written over it.
template <int D, int N, typename T, int PS, int DIR>
__device__ __forceinline__ void op_points(const double (&g)[PS][D * D + 2], const T* sU, T* sT, T (&R)[PS][D + 1],
                                          int ncl) {
  constexpr int NC = D + 1, NP = ipow(N, D), NT = op_threads(D, N);
#pragma unroll
  for (int s = 0; s < PS; ++s) {
    const int i = threadIdx.x + s * NT;
    if (i < ncl * NP) {
      const int c = i / NP, q = i - c * NP;
      const T* su = sU + c * NC * NP + q;
      T* st = sT + c * NC * NP + q;
      if constexpr (DIR == 1) {
#pragma unroll
        for (int v = 0; v < NC; ++v) R[s][v] = st[v * NP];
      } else if constexpr (DIR > 1) {
#pragma unroll
        for (int v = 0; v < NC; ++v) R[s][v] += st[v * NP];
      }
      const double pq = (double)su[D * NP];
      double fp = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double gba = g[s][DIR * D + a];
        st[a * NP] = (T)(gba * pq);
        fp = fma(gba, (double)su[a * NP], fp);
      }
      st[D * NP] = (T)fp;
    }
  }
}

// GB selects the storage basis of u: false = Lagrange polynomials in the GL
// points (nodes on the faces; the operator changes to the Gauss basis and
// back), true = Lagrange polynomials in the Gauss points (the collocated
// basis of Sec. 3.1: no basis change, diagonal mass, but a neighbour's trace
// needs its whole line of values along the face normal).  GOUT: the result
// (and the epilogue's other state operands) at the Gauss points, without
// the final G -> GL passes; the ADER update of a Gauss-basis mesh reads the
// TCK sum I in the GL basis and writes u at the Gauss points.
template <int D, int N, typename T, int EPI, int CPW, bool GB = false, int MB = 1, bool GOUT = GB>
__global__ void __launch_bounds__(op_threads(D, N))
__attribute__((amdgpu_waves_per_eu(op_waves_per_simd<D, N, T, EPI, CPW, MB>()))) op_kernel(OpParams p) {
  using Lay = OpLayout<D, N, T>;
  constexpr int NC = Lay::NC, NP = Lay::NP, NF = Lay::NF, NFACE = Lay::NFACE, G2 = D * D + 2;
  constexpr int NT = op_threads(D, N);
  constexpr int PS = cdiv(CPW * NP, NT);             // cell points per thread
  constexpr int FS = cdiv(CPW * NFACE * NF, NT);     // face points per thread
  constexpr int ES = cdiv(CPW * NC * NP, NT);        // tile elements per thread
  constexpr int NS = cdiv(CPW * NFACE * NC * NF, NT);  // neighbour trace values per thread
  extern __shared__ __align__(16) unsigned char smem[];
  T* sU = reinterpret_cast<T*>(smem);
  T* sT = sU + CPW * NC * NP;
  T* sN = sT + CPW * NC * NP;
  const T* tab = ctab<T>(N);
  const int tid = threadIdx.x;

  // workgroup -> (cell group, block of MB batch members): the cell geometry
  // is loaded once into registers and applied to each member of the block in
  // turn (members share mesh, geometry and material); MB = 1 makes the batch
  // a plain grid dimension
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int nmb = (p.B + MB - 1) / MB;
  const int mblock = logical % nmb;
  const int group = logical / nmb;
  const int64_t cell0 = (int64_t)group * CPW;
  const int ncl = (int)min((int64_t)CPW, p.nc - cell0);
  const int nel = ncl * NC * NP;

  // ---- A: the sweep's global operands, in dependency order: the neighbour
  // table and the geometry once, then per member its state and the
  // neighbours' face nodes
  int nbi[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = tid + s * NT;
    nbi[s] = 0;
    if (i < ncl * NFACE * NC * NF) {
      const int cf = i / (NC * NF);  // c * NFACE + f
      nbi[s] = p.nb[cell0 * NFACE + cf];
    }
  }
  double g[PS][G2];
#pragma unroll
  for (int s = 0; s < PS; ++s) {
    const int i = tid + s * NT;
    const int c = i / NP, q = i - (i / NP) * NP;
    const double* gp = p.geo_cell + (cell0 + c) * (int64_t)(G2 * NP) + q;
#pragma unroll
    for (int e = 0; e < G2; ++e) g[s][e] = i < ncl * NP ? gp[e * NP] : 0.0;
  }
  int fnb[FS];  // neighbour (or boundary code) of the face of each face point
#pragma unroll
  for (int s = 0; s < FS; ++s) {
    const int i = tid + s * NT;
    fnb[s] = 0;
    if (i < ncl * NFACE * NF) fnb[s] = p.nb[cell0 * NFACE + i / NF];
  }
  double fg[FS][D + 2];
#pragma unroll
  for (int s = 0; s < FS; ++s) {
    const int i = tid + s * NT;
    const int cf = i / NF, t = i - (i / NF) * NF;  // cf = c * NFACE + f
    const double* fp = p.geo_face + (cell0 * NFACE + cf) * (int64_t)((D + 2) * NF) + t;
#pragma unroll
    for (int e = 0; e < D + 2; ++e) fg[s][e] = i < ncl * NFACE * NF ? fp[e * NF] : 1.0;
  }
#pragma unroll 1
  for (int mm = 0; mm < MB; ++mm) {
    const int member = mblock * MB + mm;
    if (MB > 1 && member >= p.B) break;
    const int64_t moff = (int64_t)member * p.nc * NC * NP;
    const int64_t gofs = moff + cell0 * NC * NP;
    double ev[ES];
#pragma unroll
    for (int s = 0; s < ES; ++s) {
      const int i = tid + s * NT;
      ev[s] = i < nel ? p.u[gofs + i] : 0.0;
    }
    double nv[NS];
    double glf0[GB ? N : 1], glf1[GB ? N : 1];  // Gauss basis: face values of the 1D Lagrange polynomials
    if constexpr (GB) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        glf0[j] = (double)tab[tab_LF0(N) + j];
        glf1[j] = (double)tab[tab_LF1(N) + j];
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = tid + s * NT;
      nv[s] = 0.0;
      if (i < ncl * NFACE * NC * NF && nbi[s] >= 0) {  // boundary faces: exterior state built in F
        const int t = i % NF;
        const int r = i / NF;
        const int v = r % NC;
        const int cf = r / NC;  // c * NFACE + f
        // GL node of the neighbour's face f' that meets own tangential index t:
        // f' = f^1 with aligned coordinates unless the mesh gives orientations
        int fn = (cf % NFACE) ^ 1, tn = t;
        if (p.fo) {
          const int code = p.fo[cell0 * NFACE + cf];
          fn = code >> 3;
          tn = orient_face<D, N>(code & 7, t);
        }
        const int dir = fn >> 1, side = fn & 1;
        const double* un = p.u + moff + (int64_t)nbi[s] * NC * NP + v * NP;
        if constexpr (GB) {  // interpolate the neighbour's normal line to its face
          const int q0 = face_line_base<D, N>(dir, tn), st = dir_stride(N, dir);
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j) acc = fma(side ? glf1[j] : glf0[j], un[q0 + j * st], acc);
          nv[s] = acc;
        } else {
          nv[s] = un[face_line_base<D, N>(dir, tn) + (side ? (N - 1) * dir_stride(N, dir) : 0)];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < ES; ++s) {
      const int i = tid + s * NT;
      if (i < nel) sU[i] = (T)ev[s];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = tid + s * NT;
      if (i < ncl * NFACE * NC * NF) sN[i] = (T)nv[s];
    }
    __syncthreads();

    // ---- B: GL -> G of the cell tiles; tangential GL -> G of the neighbour traces
    if constexpr (!GB) {
      // with op_phase_tables each pass addresses S with its own opaque zero
      constexpr bool PT = op_phase_tables<N, T>();
      constexpr int MU = PT ? CPW * NC : 0, MN = PT ? CPW * NFACE * NC : 0;
      const T* S = tab + tab_S(N) + (PT ? opaque_zero() : 0);
      tpass<NT, D, 0, N, N, N, N, N, PM_STORE, MU, T>(sU, sU, ncl * NC, S);
      if constexpr (D == 2) tpass<NT, 1, 0, N, N, N, N, N, PM_STORE, MN, T>(sN, sN, ncl * NFACE * NC, S);
      if constexpr (D == 3) tpass<NT, 2, 0, N, N, N, N, N, PM_STORE, MN, T>(sN, sN, ncl * NFACE * NC, S);
      __syncthreads();
      if constexpr (PT) S = tab + tab_S(N) + opaque_zero();
      tpass<NT, D, 1, N, N, N, N, N, PM_STORE, MU, T>(sU, sU, ncl * NC, S);
      if constexpr (D == 3) tpass<NT, 2, 1, N, N, N, N, N, PM_STORE, MN, T>(sN, sN, ncl * NFACE * NC, S);
      __syncthreads();
      if constexpr (D == 3) {
        if constexpr (PT) S = tab + tab_S(N) + opaque_zero();
        tpass<NT, D, 2, N, N, N, N, N, PM_STORE, MU, T>(sU, sU, ncl * NC, S);
        __syncthreads();
      }
    }
    // ---- F: numerical fluxes at every face point, written over the neighbour traces
    {
      T lf0[N], lf1[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        lf0[j] = tab[tab_LF0(N) + j];
        lf1[j] = tab[tab_LF1(N) + j];
      }
#pragma unroll
      for (int s = 0; s < FS; ++s) {
        const int i = tid + s * NT;
        if (i < ncl * NFACE * NF) {
          const int cf = i / NF, t = i - (i / NF) * NF;
          const int c = cf / NFACE, f = cf - c * NFACE;
          const int dir = f >> 1, side = f & 1;
          const int st = dir_stride(N, dir);
          const T* su = sU + c * NC * NP + face_line_base<D, N>(dir, t);
          double um[NC], up[NC];
#pragma unroll
          for (int v = 0; v < NC; ++v) {
            T acc = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) acc = fma(side ? lf1[j] : lf0[j], su[v * NP + j * st], acc);
            um[v] = (double)acc;
            up[v] = (double)sN[(cf * NC + v) * NF + t];
          }
          double area2 = 0.0, vnm = 0.0, vnp = 0.0;
#pragma unroll
          for (int e = 0; e < D; ++e) {
            area2 = fma(fg[s][e], fg[s][e], area2);
            vnm = fma(fg[s][e], um[e], vnm);
            vnp = fma(fg[s][e], up[e], vnp);
          }
          const double area = sqrt(area2), inv_area = 1.0 / area;
          vnm *= inv_area;
          vnp *= inv_area;
          double pp = up[D];
          if (fnb[s] < 0) {  // boundary: mirror state (wall), else zero state (absorbing;
                             // prescribed data are added below)
            pp = fnb[s] == kBcWall ? um[D] : 0.0;
            vnp = fnb[s] == kBcWall ? -vnm : 0.0;
          }
          double ps, vs;
          if (p.central) {
            ps = 0.5 * (um[D] + pp);
            vs = 0.5 * (vnm + vnp);
          } else {
            const double Zm = fg[s][D], Zp = fg[s][D + 1];
            const double inv = 1.0 / (Zm + Zp);
            ps = (Zp * um[D] + Zm * pp + Zm * Zp * (vnm - vnp)) * inv;
            vs = (Zm * vnm + Zp * vnp + um[D] - pp) * inv;
          }
#pragma unroll
          for (int e = 0; e < D; ++e) sN[(cf * NC + e) * NF + t] = (T)(-fg[s][e] * ps);
          sN[(cf * NC + D) * NF + t] = (T)(-area * vs);
        }
      }
      // Prescribed faces (device neighbour entry kBcPrescribed - slot): both
      // fluxes are linear in the exterior state, so the flux of the given data
      // (p+, v+.n, evaluated for this launch into ext[slot][2][NF]) is added to
      // the zero-state flux written above.  Same thread as above for each face
      // point; operands re-read from memory so that this rare path takes no
      // registers from the loop above.
      if (p.ext) {
#pragma unroll 1
        for (int i = tid; i < ncl * NFACE * NF; i += NT) {
          const int cf = i / NF, t = i - (i / NF) * NF;
          const int code = p.nb[cell0 * NFACE + cf];
          if (code > kBcPrescribed) continue;
          const double* ex = p.ext + (int64_t)(kBcPrescribed - code) * 2 * NF + t;
          const double pe = ex[0], vne = ex[NF];
          const double* fp = p.geo_face + (cell0 * NFACE + cf) * (int64_t)((D + 2) * NF) + t;
          double area2 = 0.0;
#pragma unroll
          for (int e = 0; e < D; ++e) area2 = fma(fp[e * NF], fp[e * NF], area2);
          double dps, dvs;
          if (p.central) {
            dps = 0.5 * pe;
            dvs = 0.5 * vne;
          } else {
            const double Zm = fp[D * NF], Zp = fp[(D + 1) * NF];
            const double inv = 1.0 / (Zm + Zp);
            dps = (Zm * pe - Zm * Zp * vne) * inv;
            dvs = (Zp * vne - pe) * inv;
          }
#pragma unroll
          for (int e = 0; e < D; ++e) sN[(cf * NC + e) * NF + t] += (T)(-fp[e * NF] * dps);
          sN[(cf * NC + D) * NF + t] += (T)(-sqrt(area2) * dvs);
        }
      }
    }
    __syncthreads();
    // ---- C: per direction, pointwise fluxes then lines (derivative + lifts);
    // the residual of each direction is added in the next point phase
    T R[PS][NC];
    op_points<D, N, T, PS, 0>(g, sU, sT, R, ncl);
    __syncthreads();
    if constexpr (op_phase_tables<N, T>())
      op_lines_pt<D, N, T, 0, CPW>(tab, sT, sN, ncl);
    else
      op_lines<D, N, T, 0>(tab, sT, sN, ncl);
    __syncthreads();
    op_points<D, N, T, PS, 1>(g, sU, sT, R, ncl);
    __syncthreads();
    if constexpr (op_phase_tables<N, T>())
      op_lines_pt<D, N, T, 1, CPW>(tab, sT, sN, ncl);
    else
      op_lines<D, N, T, 1>(tab, sT, sN, ncl);
    __syncthreads();
    if constexpr (D == 3) {
      op_points<D, N, T, PS, 2>(g, sU, sT, R, ncl);
      __syncthreads();
      if constexpr (op_phase_tables<N, T>())
      op_lines_pt<D, N, T, 2, CPW>(tab, sT, sN, ncl);
    else
      op_lines<D, N, T, 2>(tab, sT, sN, ncl);
      __syncthreads();
    }
    // the epilogue's second state operand, requested after the sweep so that
    // its registers are free during it; its latency overlaps phase D
    double eb[ES];
#pragma unroll
    for (int s = 0; s < ES; ++s) {
      const int i = tid + s * NT;
      eb[s] = 0.0;
      if constexpr (EPI == EPI_ADD)
        if (i < nel) eb[s] = p.u_base[gofs + i];
      if constexpr (EPI == EPI_LSRK)
        if (i < nel && (p.two_r ? !p.first : p.acoef != 0.0)) eb[s] = p.du[gofs + i];
    }
    // ---- D: last direction's residual, inverse mass (pointwise FP64
    // factors) into sT, G -> GL
#pragma unroll
    for (int s = 0; s < PS; ++s) {
      const int i = tid + s * NT;
      if (i < ncl * NP) {
        const int c = i / NP, q = i - c * NP;
        T* r = sT + c * NC * NP + q;
#pragma unroll
        for (int v = 0; v < NC; ++v) {
          const T rv = R[s][v] + r[v * NP];
          r[v * NP] = (T)(g[s][D * D + (v == D)] * (double)rv);
        }
      }
    }
    __syncthreads();
    if constexpr (!GOUT && !op_phase_tables<N, T>()) {
      tensor_apply_inplace<NT, D, N, 0, T>(sT, ncl * NC, tab + tab_Sinv(N));
    } else if constexpr (!GOUT) {
      constexpr int MU = CPW * NC;
      tpass<NT, D, 0, N, N, N, N, N, PM_STORE, MU, T>(sT, sT, ncl * NC, tab + tab_Sinv(N) + opaque_zero());
      __syncthreads();
      tpass<NT, D, 1, N, N, N, N, N, PM_STORE, MU, T>(sT, sT, ncl * NC, tab + tab_Sinv(N) + opaque_zero());
      __syncthreads();
      if constexpr (D == 3) {
        tpass<NT, D, 2, N, N, N, N, N, PM_STORE, MU, T>(sT, sT, ncl * NC, tab + tab_Sinv(N) + opaque_zero());
        __syncthreads();
      }
    }
    // ---- E: epilogue (coalesced; u from A, the second operand from D)
    {
      int scell = -1;
      if (p.src.cell) scell = p.src.cell[member];
      const bool has_src = scell >= cell0 && scell < cell0 + ncl;
      double sval = 0.0;
      if (has_src) {
        const double tn = p.time.tn();
        if constexpr (EPI == EPI_LSRK) sval = ricker_deriv(p.src.wave + 3 * member, tn + p.time.t_off, 0);
        if constexpr (EPI == EPI_ADD) sval = ricker_integral(p.src.wave + 3 * member, tn, tn + p.time.dt);
      }
#pragma unroll
      for (int s = 0; s < ES; ++s) {
        const int i = tid + s * NT;
        if (i >= nel) continue;
        const double val = (double)sT[i];
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
            if (p.two_r) {  // accumulated solution in du, next stage state in u_next
              const double k = p.dt * (val + add);
              const double un = (p.first ? ev[s] : eb[s]) + p.bcoef * k;
              p.du[gi] = un;
              p.u_next[gi] = un + p.acoef * k;
            } else {
              const double d = p.acoef * eb[s] + p.dt * (val + add);
              p.du[gi] = d;
              p.u_next[gi] = ev[s] + p.bcoef * d;
            }
          } else {
            p.u_next[gi] = eb[s] + val + add;
          }
        }
      }
    }
  }  // member
}

// ------------------------------------------------------------------------
// ADER sweep 1: the Taylor-Cauchy-Kowalevski sum in the collocated Gauss
// basis with the degree reduction (Sec. 3.2, 3.3, Alg. 3).
//
// Per time derivative m at the level with NL points per direction: one line
// phase computes the collocated derivative along all d directions of every
// component (tiles Db[0..d-1]); one point phase applies the metric of the
// level (held in registers of the point's thread), scales by the mass
// factors and adds the source term, giving ut^m.  Every second derivative is
// projected to NL-2 points; the metric of the coarser level is requested
// into the same registers as soon as the last point phase of the finer level
// is done, so its latency overlaps the projection passes.  The Taylor sum is
// accumulated per level in FP64 registers: I = A_0 + E(A_1 + E(A_2 + ...)),
// embedded level by level at the end (E between consecutive Gauss sets is
// exact on the lower degree).  LDS: the current derivative C and d
// derivative tiles, nothing else, so that more workgroups fit on a CU.
// ------------------------------------------------------------------------
template <int D, int N, typename T>
struct TckLayout {
  static constexpr int NC = D + 1, NP = ipow(N, D), G2 = D * D + 2;
  static constexpr int tiles = 1 + D;  // C and the d derivative tiles (an FP64 tile fits in Db)
  // FP64 Taylor sums of the reduced levels kept in LDS (reduction every
  // derivative: up to N levels, too many for registers), per cell
  static constexpr int acc_elems(int rp) {
    int e = 0;
    if (rp == 1)
      for (int l = 1; N - l >= 1; ++l) e += NC * ipow(N - l, D);
    return e;
  }
  static constexpr int bytes_per_cell(int rp) { return tiles * NC * NP * (int)sizeof(T) + 8 * acc_elems(rp); }
};

// RP: reduction period of the TCK (0: none, Alg. 2; 2: every second
// derivative, Alg. 3; 1 and 3: every derivative / every third, the
// ablation of Sec. 3.3); level L has N - RP L points per direction.
template <int D, int N, int CPW, int RP>
struct TckRegs {
  static constexpr int G2 = D * D + 2, NC = D + 1;
  static constexpr int NLV = num_levels_r(N, RP);
  static constexpr bool ACC_LDS = RP == 1;  // sums of levels >= 1 in LDS
  static constexpr int NT = tck_threads(D, N);
  static constexpr int PS0 = cdiv(CPW * ipow(N, D), NT);
  double g[PS0][G2];                       // metric and mass factors of the current level
  double A[ACC_LDS ? 1 : NLV][PS0][NC];    // Taylor sums per level (FP64)
  double* acc;                             // LDS: sums of levels >= 1 when ACC_LDS
};

// metric and mass factors of level L (N - RP L points per direction) of the
// group's cells into the registers of the threads that own the points
template <int D, int N, int CPW, int RP, int L>
__device__ __forceinline__ void tck_load_geo(TckRegs<D, N, CPW, RP>& R, const TckParams& p, int64_t cell0,
                                             int ncl) {
  constexpr int G2 = D * D + 2, NPL = ipow(N - RP * L, D), NT = tck_threads(D, N);
  constexpr int PSL = cdiv(CPW * NPL, NT);
#pragma unroll
  for (int s = 0; s < PSL; ++s) {
    const int i = threadIdx.x + s * NT;
    const int c = i / NPL, q = i - c * NPL;
    const double* gp = p.geo_lev[L] + (cell0 + c) * (int64_t)(G2 * NPL) + q;
#pragma unroll
    for (int e = 0; e < G2; ++e) R.g[s][e] = i < ncl * NPL ? gp[e * NPL] : 0.0;
  }
}

template <int D, int N, typename T, int RP, int CPW>
struct Tck {
  static constexpr int NC = D + 1, NP = ipow(N, D), G2 = D * D + 2, NT = tck_threads(D, N);
  using Regs = TckRegs<D, N, CPW, RP>;

  static constexpr double inv_fact(int m) {  // 1/(m+1)!
    double f = 1.0;
    for (int j = 2; j <= m + 1; ++j) f *= j;
    return 1.0 / f;
  }
  static constexpr int npl(int L) { return ipow(N - RP * L, D); }
  // offset of level L >= 1 in the LDS sums (elements per cell and component)
  static constexpr int acc_before(int L) {
    int e = 0;
    for (int j = 1; j < L; ++j) e += npl(j);
    return e;
  }
  // FP64 Taylor sum of level L at the s-th point (cell c, point q) of this thread
  template <int L>
  __device__ static __forceinline__ double& accum(Regs& R, int s, int c, int q, int v) {
    if constexpr (L == 0 || !Regs::ACC_LDS)
      return R.A[L][s][v];
    else
      return R.acc[CPW * NC * acc_before(L) + (c * NC + v) * npl(L) + q];
  }

  // metric entry e of the s-th point of this thread on the current level
  __device__ static __forceinline__ double geo(const Regs& R, int s, int e) { return R.g[s][e]; }
  static constexpr int psl(int L) { return cdiv(CPW * npl(L), NT); }

  // derivative of every component along every direction at level NL: C -> Db
  // (the d derivative tiles are contiguous, TILE elements apart)
  template <int NL>
  __device__ static __forceinline__ void lines(const T* C, T* Db0, const T* __restrict__ Dl, int ncl) {
    constexpr int NLL = ipow(NL, D - 1);
    constexpr int TILE = CPW * NC * NP;
    constexpr int PER_DIR = CPW * NC * NLL;  // compile-time: no runtime division
    constexpr int ITERS = cdiv(D * PER_DIR, NT);
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int wi = threadIdx.x + it * NT;
      if (wi >= D * PER_DIR) break;
      const int dir = wi / PER_DIR;
      const int r = wi - dir * PER_DIR;
      const int sl = r / NLL;
      const int L = r - sl * NLL;
      if (sl >= ncl * NC) continue;  // ragged last group
      // line base and stride inside the NL^D tensor (x fastest)
      const int st = dir == 0 ? 1 : (dir == 1 ? NL : NL * NL);
      const int base = face_line_base<D, NL>(dir, L);
      const T* src = C + sl * NP + base;
      T* dst = Db0 + dir * TILE + sl * NP + base;
      T x[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) x[j] = src[j * st];
      T acc[NL];
      contract<NL, NL>(Dl, x, acc);
#pragma unroll
      for (int i = 0; i < NL; ++i) dst[i * st] = acc[i];
    }
  }

  // size-changing pass (MO x MI matrix) along DIR between buffers with
  // NP-strided cell-component slices.  Here and in the final phase the lines
  // are visited in a fixed number of unrolled rounds rather than a loop over
  // the group's cells: a loop would have its matrix entries hoisted into
  // scalar registers ahead of it and spilled (the kernel ran 10 % slower)
  template <int DIR, int E0, int E1, int E2, int MO, typename TI, typename TO>
  __device__ static __forceinline__ void pass(const TI* in, TO* out, int ncl, const T* __restrict__ Mx) {
    constexpr int MI = DIR == 0 ? E0 : (DIR == 1 ? E1 : E2);
    using P = Pass<D, DIR, MI, MO, E0, E1, E2>;
#pragma unroll
    for (int it = 0; it < cdiv(CPW * NC * P::NL, NT); ++it) {
      const int wi = threadIdx.x + it * NT;
      if (wi >= ncl * NC * P::NL) break;
      const int s = wi / P::NL;
      const int L = wi - s * P::NL;
      int bi, bo;
      P::base(L, bi, bo);
      const TI* src = in + s * NP + bi;
      TO* dst = out + s * NP + bo;
      T x[MI];
#pragma unroll
      for (int j = 0; j < MI; ++j) x[j] = (T)src[j * P::STEP_IN];
      T acc[MO];
      contract<MI, MO>(Mx, x, acc);
#pragma unroll
      for (int i = 0; i < MO; ++i) dst[i * P::STEP_OUT] = (TO)acc[i];
    }
  }

  // separable map of a level-NI tensor to a level-NO tensor with the same
  // matrix in every direction, buf0 -> ... -> buf0 through buf1, buf2
  template <int NI, int NO>
  __device__ static __forceinline__ void tensor_map(T* b0, T* b1, T* b2, int ncl, const T* Mx) {
    pass<0, NI, NI, NI, NO>(b0, b1, ncl, Mx);
    __syncthreads();
    if constexpr (D == 2) {
      pass<1, NO, NI, 1, NO>(b1, b0, ncl, Mx);
      __syncthreads();
    } else {
      pass<1, NO, NI, NI, NO>(b1, b2, ncl, Mx);
      __syncthreads();
      pass<2, NO, NO, NI, NO>(b2, b0, ncl, Mx);
      __syncthreads();
    }
  }

  // time derivative M at level index L (NL = N - 2L points), current in C.
  // A derivative that would be projected below one point per direction is
  // zero (and so is every later one): the recursion stops before it.
  template <int M, int L>
  __device__ static __forceinline__ void step(const TckParams& p, T* C, T* const* Db, Regs& R, int64_t cell0,
                                              int ncl, int member) {
    constexpr int NL = N - RP * L;
    constexpr bool PROJECT = RP > 0 && M % (RP > 0 ? RP : 1) == 0;
    if constexpr (M <= N && NL >= 1 && !(PROJECT && NL - RP < 1)) {
      constexpr int NPL = ipow(NL, D);
      constexpr int PSL = cdiv(CPW * NPL, NT);
      const T* tab = ctab<T>(N);
      double dtp = 1.0;
#pragma unroll
      for (int j = 0; j <= M; ++j) dtp *= p.dt;
      const double coef = inv_fact(M) * dtp;
      if constexpr (NL > 1) {
        lines<NL>(C, Db[0], tab + (L == 0 ? tab_D(N) : tab_level_D(N, L, RP)), ncl);
        __syncthreads();
      }
      // point phase: ut^M = -mu * metric(derivatives) + s^(M-1)(t) g, into C
      int scell = -1;
      if (p.src.cell) scell = p.src.cell[member];
      double sd = 0.0;
      if (scell >= cell0 && scell < cell0 + ncl) sd = ricker_deriv(p.src.wave + 3 * member, p.time.tn(), M - 1);
#pragma unroll
      for (int s = 0; s < PSL; ++s) {
        const int i = threadIdx.x + s * NT;
        if (i < ncl * NPL) {
          const int c = i / NPL, q = i - c * NPL;
          double w[NC];
#pragma unroll
          for (int v = 0; v < NC; ++v) w[v] = 0.0;
          if constexpr (NL > 1) {
#pragma unroll
            for (int b = 0; b < D; ++b) {
              const T* t = Db[b] + c * NC * NP + q;
              const double dp = (double)t[D * NP];
#pragma unroll
              for (int a = 0; a < D; ++a) {
                const double gba = geo(R, s, b * D + a);
                w[a] = fma(gba, dp, w[a]);
                w[D] = fma(gba, (double)t[a * NP], w[D]);
              }
            }
#pragma unroll
            for (int v = 0; v < NC; ++v) w[v] *= -geo(R, s, D * D + (v == D));
          }
          if (cell0 + c == scell) w[D] += sd * p.src.glev[L][(int64_t)member * NPL + q];
#pragma unroll
          for (int v = 0; v < NC; ++v) {
            const T wt = (T)w[v];
            C[(c * NC + v) * NP + q] = wt;
            if constexpr (!PROJECT) accum<L>(R, s, c, q, v) += coef * (double)wt;
          }
        }
      }
      // the last use of this level's metric: request the next level's
      if constexpr (PROJECT && NL - RP >= 1) tck_load_geo<D, N, CPW, RP, L + 1>(R, p, cell0, ncl);
      __syncthreads();
      if constexpr (PROJECT) {
        constexpr int NR = NL - RP;
        if constexpr (NR >= 1) {
          tensor_map<NL, NR>(C, Db[0], Db[1], ncl, tab + tab_level_P(N, L + 1, RP));
          constexpr int PSR = cdiv(CPW * ipow(NR, D), NT);
#pragma unroll
          for (int s = 0; s < PSR; ++s) {
            const int i = threadIdx.x + s * NT;
            if (i < ncl * ipow(NR, D)) {
              const int c = i / ipow(NR, D), q = i - c * ipow(NR, D);
#pragma unroll
              for (int v = 0; v < NC; ++v) accum<L + 1>(R, s, c, q, v) += coef * (double)C[(c * NC + v) * NP + q];
            }
          }
          step<M + 1, L + 1>(p, C, Db, R, cell0, ncl, member);
        }
      } else {
        step<M + 1, L>(p, C, Db, R, cell0, ncl, member);
      }
    }
  }

  // ---- final phase in FP64: I_GL = sum_l Q_l^(x d) A_l, with Q_l (N x m_l)
  // the level-l Gauss interpolant evaluated at the GL nodes (the embeddings
  // to level 0 and S^-1 in one matrix per level).  One pass per direction
  // over all levels at once; the last pass sums the levels and stores I.
  static constexpr int NLV_ALL = Regs::NLV;
  static constexpr int mlev(int L) { return N - RP * L; }
  static constexpr int fin_elems(int stage) {  // FP64 elements per cell and component of A / T / U
    int e = 0;
    for (int L = 0; L < NLV_ALL; ++L) {
      const int m = mlev(L);
      e += stage == 0 ? ipow(m, D) : (stage == 1 ? N * ipow(m, D - 1) : N * N * ipow(m, D - 2));
    }
    return e;
  }
  static constexpr int fin_off(int stage, int L) {  // offset of level L inside stage `stage`
    int e = 0;
    for (int j = 0; j < L; ++j) {
      const int m = mlev(j);
      e += stage == 0 ? ipow(m, D) : (stage == 1 ? N * ipow(m, D - 1) : N * N * ipow(m, D - 2));
    }
    return e;
  }
  // LDS use of the final phase (bytes per cell): A and T at once, then T and U
  static constexpr int fin_bytes() {
    const int a = fin_elems(0), t = fin_elems(1), u = D == 3 ? fin_elems(2) : 0;
    const int p1 = a + t, p2 = t + u;
    return 8 * NC * (p1 > p2 ? p1 : p2);
  }
  static constexpr bool FUSED_FINAL = sizeof(T) == 8 && !Regs::ACC_LDS &&
                                      fin_bytes() <= TckLayout<D, N, T>::bytes_per_cell(RP);

  // level L's 1D matrix of the final phase (N x m_L): S^-1 for level 0
  __device__ static __forceinline__ const double* qmat(int L) {
    return L == 0 ? ctab<double>(N) + tab_Sinv(N) : ctab<double>(N) + tab_level_Q(N, L, RP);
  }

  template <int L>
  __device__ static __forceinline__ void fin_write_A(double* A, Regs& R, int ncl) {
    if constexpr (L < NLV_ALL) {
      constexpr int NPL = ipow(mlev(L), D);
      double* a = A + CPW * NC * fin_off(0, L);
#pragma unroll
      for (int s = 0; s < psl(L); ++s) {
        const int i = threadIdx.x + s * NT;
        if (i < ncl * NPL) {
          const int c = i / NPL, q = i - c * NPL;
#pragma unroll
          for (int v = 0; v < NC; ++v) a[(c * NC + v) * NPL + q] = R.A[L][s][v];
        }
      }
      fin_write_A<L + 1>(A, R, ncl);
    }
  }

  // pass along DIR (0: x, 1: y) of every level, from stage DIR to stage DIR+1
  template <int DIR, int L>
  __device__ static __forceinline__ void fin_pass(const double* in, double* out, int ncl) {
    if constexpr (L < NLV_ALL) {
      constexpr int m = mlev(L);
      // extents of the input: direction < DIR already N, the others m
      using P = Pass<D, DIR, m, N, (DIR > 0 ? N : m), (DIR > 1 ? N : m), m>;
      const double* src0 = in + CPW * NC * fin_off(DIR, L);
      double* dst0 = out + CPW * NC * fin_off(DIR + 1, L);
      const double* Q = qmat(L);
#pragma unroll
      for (int it = 0; it < cdiv(CPW * NC * P::NL, NT); ++it) {
        const int w = threadIdx.x + it * NT;
        if (w >= ncl * NC * P::NL) break;
        const int sl = w / P::NL;
        const int Ln = w - sl * P::NL;
        int bi, bo;
        P::base(Ln, bi, bo);
        const double* src = src0 + sl * P::SIN + bi;
        double* dst = dst0 + sl * P::SOUT + bo;
        double x[m];
#pragma unroll
        for (int j = 0; j < m; ++j) x[j] = src[j * P::STEP_IN];
        double acc[N];
        contract<m, N>(Q, x, acc);
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i * P::STEP_OUT] = acc[i];
      }
      fin_pass<DIR, L + 1>(in, out, ncl);
    }
  }

  // last direction: sum over the levels of Q_L along D-1, into acc
  template <int L>
  __device__ static __forceinline__ void fin_last(const double* in, int sl, int t, double (&acc)[N]) {
    if constexpr (L < NLV_ALL) {
      constexpr int m = mlev(L);
      constexpr int SL = ipow(N, D - 1) * m;  // elements of one slice of this level
      const double* src = in + CPW * NC * fin_off(D - 1, L) + sl * SL + t;
      const double* Q = qmat(L);
#pragma unroll
      for (int j = 0; j < m; ++j) {
        const double xj = src[j * ipow(N, D - 1)];
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = fma(Q[i * m + j], xj, acc[i]);
      }
      fin_last<L + 1>(in, sl, t, acc);
    }
  }

  // the whole final phase; smem holds at least fin_bytes() per cell
  template <bool HDG_ADD>
  __device__ static __forceinline__ void final_fused(const TckParams& p, double* sm, Regs& R, int ncl,
                                                     int64_t gofs) {
    constexpr int EA = fin_elems(0), EU = D == 3 ? fin_elems(2) : 0;
    constexpr int LOW = (EA > EU ? EA : EU) * CPW * NC;  // A and U share the start, T follows
    double* A = sm;
    double* Tt = sm + LOW;
    double* U = sm;
    fin_write_A<0>(A, R, ncl);
    __syncthreads();
    fin_pass<0, 0>(A, Tt, ncl);
    __syncthreads();
    const double* last = Tt;
    if constexpr (D == 3) {
      fin_pass<1, 0>(Tt, U, ncl);
      __syncthreads();
      last = U;
    }
    // one thread per output line along the last direction: (cell, component, tangential t)
    constexpr int NT1 = ipow(N, D - 1);
    constexpr int ST = ipow(N, D - 1);
#pragma unroll
    for (int it = 0; it < cdiv(CPW * NC * NT1, NT); ++it) {
      const int w = threadIdx.x + it * NT;
      if (w >= ncl * NC * NT1) break;
      const int sl = w / NT1;
      const int t = w - sl * NT1;
      double acc[N];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = 0.0;
      fin_last<0>(last, sl, t, acc);
      const int64_t g0 = gofs + (int64_t)sl * NP + t;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double val = acc[i];
        if constexpr (HDG_ADD) val += p.dt * p.u_base[g0 + i * ST];
        p.I[g0 + i * ST] = val;
      }
    }
  }

  // I_G = A_0 + E(A_1 + E(A_2 + ...)): from the coarsest level L upwards,
  // leaving level L-1's partial sum in tile C
  template <int L>
  __device__ static __forceinline__ void collapse(const TckParams& p, T* C, T* const* Db, Regs& R, int ncl) {
    constexpr int NLV = Regs::NLV;
    if constexpr (L >= 1 && L < NLV) {
      constexpr int NPL = npl(L);
      // tile <- A_L (+ the embedded sum of the coarser levels already in C)
#pragma unroll
      for (int s = 0; s < psl(L); ++s) {
        const int i = threadIdx.x + s * NT;
        if (i < ncl * NPL) {
          const int c = i / NPL, q = i - c * NPL;
#pragma unroll
          for (int v = 0; v < NC; ++v) {
            T* x = C + (c * NC + v) * NP + q;
            const double prev = (L == NLV - 1) ? 0.0 : (double)*x;
            *x = (T)(prev + accum<L>(R, s, c, q, v));
          }
        }
      }
      __syncthreads();
      const T* tab = ctab<T>(N);
      tensor_map<N - RP * L, N - RP * (L - 1)>(C, Db[0], Db[1], ncl, tab + tab_level_E(N, L, RP));
      collapse<L - 1>(p, C, Db, R, ncl);
    }
  }
};

// Register budget of the TCK: with one point per thread the kernel is
// compiled for the waves per SIMD that the LDS of one workgroup allows (a
// 256-thread group puts one wave on each SIMD; 160 KiB of LDS per CU),
// capped at 5 (at most 96 VGPRs) in FP64 and 6 (80 VGPRs) with FP32 tiles,
// so that the registers limit occupancy as little as they can without
// spilling much (FP32 at 6 waves spills 12 bytes per lane and still runs 8 %
// faster at k = 5; 8 waves spills 72 and runs 30 % slower).  With more
// points per thread the registers hold several metric sets and no budget is
// imposed (it would spill).
template <int D, int N, typename T, int CPW, int RP>
constexpr int tck_waves_per_simd() {
  if (tck_threads(D, N) != 256 || cdiv(CPW * ipow(N, D), 256) > 1) return 1;
  const int wg = (160 * 1024) / (CPW * TckLayout<D, N, T>::bytes_per_cell(RP));
  const int cap = sizeof(T) == 4 ? 6 : 5;
  return wg < 1 ? 1 : (wg > cap ? cap : wg);
}

// HDG = true: the HDG-ADER variant (Sec. 2.4, eq. hdg-ader).  p.u holds the
// DG derivative W = L u (the first time derivative), the recursion starts at
// the second derivative, and I = dt u + sum_{m>=1} dt^{m+1}/(m+1)! ut^m with
// the dt u term added from p.u_base.  GS: u (and u_base) in the Gauss
// storage basis, so no basis change on the way in; I always leaves in the GL
// basis, whose face nodes the update sweep gathers from the neighbours (the
// HDG dt u term then joins the level-0 sum before its S^-1).
template <int D, int N, typename T, int RP, int CPW, bool HDG = false, bool GS = false>
__global__ void __launch_bounds__(tck_threads(D, N))
__attribute__((amdgpu_waves_per_eu(tck_waves_per_simd<D, N, T, CPW, RP>()))) tck_kernel(TckParams p) {
  using K = Tck<D, N, T, RP, CPW>;
  using Regs = TckRegs<D, N, CPW, RP>;
  constexpr int NC = D + 1, NP = ipow(N, D), NT = tck_threads(D, N);
  constexpr int ES = cdiv(CPW * NC * NP, NT);
  constexpr int PS0 = cdiv(CPW * NP, NT);
  extern __shared__ __align__(16) unsigned char smem[];
  T* C = reinterpret_cast<T*>(smem);
  T* Db[3] = {C + CPW * NC * NP, C + 2 * CPW * NC * NP, C + 3 * CPW * NC * NP};
  const T* tab = ctab<T>(N);

  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int member = logical % p.B;
  const int group = logical / p.B;
  const int64_t cell0 = (int64_t)group * CPW;
  const int ncl = (int)min((int64_t)CPW, p.nc - cell0);
  const int64_t gofs = (int64_t)member * p.nc * NC * NP + cell0 * NC * NP;
  const int nel = ncl * NC * NP;

  double ev[ES];
#pragma unroll
  for (int s = 0; s < ES; ++s) {
    const int i = threadIdx.x + s * NT;
    ev[s] = i < nel ? p.u[gofs + i] : 0.0;
  }
  Regs R;
  tck_load_geo<D, N, CPW, RP, 0>(R, p, cell0, ncl);
#pragma unroll
  for (int l = 0; l < (Regs::ACC_LDS ? 1 : Regs::NLV); ++l)
#pragma unroll
    for (int s = 0; s < PS0; ++s)
#pragma unroll
      for (int v = 0; v < NC; ++v) R.A[l][s][v] = 0.0;
  R.acc = reinterpret_cast<double*>(C + (1 + D) * CPW * NC * NP);  // after the tiles (8-byte aligned)
  if constexpr (Regs::ACC_LDS)
    for (int i = threadIdx.x; i < CPW * TckLayout<D, N, T>::acc_elems(RP); i += NT) R.acc[i] = 0.0;
#pragma unroll
  for (int s = 0; s < ES; ++s) {
    const int i = threadIdx.x + s * NT;
    if (i < nel) C[i] = (T)ev[s];
  }
  __syncthreads();
  if constexpr (!GS) tensor_apply_inplace<NT, D, N, CPW * NC, T>(C, ncl * NC, tab + tab_S(N));
  // first term of the sum: dt u_G (ADER), dt^2/2 W_G (HDG-ADER)
  const double c0 = HDG ? 0.5 * p.dt * p.dt : p.dt;
#pragma unroll
  for (int s = 0; s < PS0; ++s) {
    const int i = threadIdx.x + s * NT;
    if (i < ncl * NP) {
      const int c = i / NP, q = i - c * NP;
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        R.A[0][s][v] = c0 * (double)C[(c * NC + v) * NP + q];
        if constexpr (HDG && GS) R.A[0][s][v] += p.dt * p.u_base[gofs + (c * NC + v) * NP + q];
      }
    }
  }
  if constexpr (HDG)
    K::template step<2, 0>(p, C, Db, R, cell0, ncl, member);
  else
    K::template step<1, 0>(p, C, Db, R, cell0, ncl, member);
  __syncthreads();  // the last accumulation may still read C
  if constexpr (K::FUSED_FINAL) {
    K::template final_fused<HDG && !GS>(p, reinterpret_cast<double*>(smem), R, ncl, gofs);
  } else {
    // collapse the coarser levels into level 0, add A_0 in FP64, then G -> GL
    // in FP64
    K::template collapse<Regs::NLV - 1>(p, C, Db, R, ncl);
    double* sI = reinterpret_cast<double*>(Db[0]);  // FP64 tile over the derivative tiles
#pragma unroll
    for (int s = 0; s < PS0; ++s) {
      const int i = threadIdx.x + s * NT;
      if (i < ncl * NP) {
        const int c = i / NP, q = i - c * NP;
#pragma unroll
        for (int v = 0; v < NC; ++v) {
          const double lower = Regs::NLV > 1 ? (double)C[(c * NC + v) * NP + q] : 0.0;
          sI[(c * NC + v) * NP + q] = R.A[0][s][v] + lower;
        }
      }
    }
    __syncthreads();
    tensor_apply_inplace<NT, D, N, CPW * NC, double>(sI, ncl * NC, ctab<double>(N) + tab_Sinv(N));
    if constexpr (HDG && !GS) {
      for (int i = threadIdx.x; i < nel; i += NT) p.I[gofs + i] = sI[i] + p.dt * p.u_base[gofs + i];
    } else {
      for (int i = threadIdx.x; i < nel; i += NT) p.I[gofs + i] = sI[i];
    }
  }
}

// ------------------------------------------------------------------------
// Energy sum_q |v|^2 / mu_v + p^2 / mu_p at the Gauss points (per group);
// GS: the state is already at the Gauss points.
// ------------------------------------------------------------------------
template <int D, int N, typename T, bool GS = false>
__global__ void __launch_bounds__(op_threads(D, N)) energy_kernel(EnergyParams p) {
  constexpr int NC = D + 1, NP = ipow(N, D), NT = op_threads(D, N);
  extern __shared__ __align__(16) unsigned char smem[];
  T* sU = reinterpret_cast<T*>(smem);
  __shared__ double red[NT];
  const T* tab = ctab<T>(N);
  const int logical = blockIdx.x;
  const int member = logical % p.B;
  const int group = logical / p.B;
  const int64_t cell0 = (int64_t)group * p.cpw;
  const int ncl = (int)min((int64_t)p.cpw, p.nc - cell0);
  const int64_t gofs = (int64_t)member * p.nc * NC * NP + cell0 * NC * NP;
  for (int i = threadIdx.x; i < ncl * NC * NP; i += NT) sU[i] = (T)p.u[gofs + i];
  __syncthreads();
  if constexpr (!GS) tensor_apply_inplace<NT, D, N, 0, T>(sU, ncl * NC, tab + tab_S(N));
  double acc = 0.0;
  for (int i = threadIdx.x; i < ncl * NC * NP; i += NT) {
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
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.partial[(int64_t)member * p.groups + group] = red[0];
}

}  // namespace dgw
