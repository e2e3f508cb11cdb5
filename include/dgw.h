/*
 * dgw -- matrix-free discontinuous Galerkin solver for first-order acoustics
 * on curved quadrilateral / hexahedral meshes, for AMD Instinct MI355X (gfx950).
 *
 * Method: Schoeder, Kormann, Wall, Kronbichler, "Efficient explicit time
 * stepping of high order discontinuous Galerkin schemes for waves",
 * arXiv:1805.03981.  Section references below are to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - dim d in {2,3}; degree k in 1..8; n = k+1 nodes per direction;
 *    np = n^d nodes per cell; components (v_1..v_d, p), d+1 of them.
 *  - Reference cell [0,1]^d.  The solution is stored in the Lagrange basis on
 *    the Gauss-Lobatto (GL) nodes (Sec. 3.1: nodes on the faces keep face
 *    access at n^(d-1) values), lexicographic with x fastest.
 *  - State layout (device memory, FP64): u[B][n_cells][d+1][np]; B is the
 *    batch of independent solutions (right-hand sides) sharing one mesh.
 *  - Cell geometry: (q+1)^d nodes per cell at the equispaced reference points
 *    j/q, lexicographic with x fastest (a degree-q map; q = k by default).
 *  - Faces are numbered -x,+x,-y,+y,-z,+z.  Neighbour tables list, per cell
 *    and face, the cell across it; the neighbour's matching face is the
 *    opposite one with the same tangential orientation.
 *  - Weak form (Sec. 2.1, eq. weak-form) with the material in a weighted
 *    mass: (phi, rho dv/dt) = (grad phi, p) - <phi n, p*>,
 *    (phi, dp/dt / (rho c^2)) = (grad phi, v) - <phi, v*.n>; Gauss quadrature
 *    on n points per direction (Sec. 3); upwind flux = the paper's HDG flux
 *    with tau = 1/(rho c) (Sec. 2.4), or central flux.
 *  - Device pointers are caller-owned, 256-byte aligned and must not alias
 *    unless stated.  Streams are hipStream_t passed as void* (NULL = the
 *    null stream).  Calls that take a stream are asynchronous on it.
 *  - Errors: every call returns a dgw_status.  Validation happens before any
 *    launch: on an error nothing has been written.  dgw_last_error() gives
 *    the text of the last error of the calling thread.  A mesh must not be
 *    used from two host threads at once.
 */
#ifndef DGW_H
#define DGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dgw_status;
#define DGW_OK 0
#define DGW_EINVAL (-1)        /* invalid argument or mesh                        */
#define DGW_ENOMEM (-2)        /* device or host allocation failed / over budget  */
#define DGW_EDEVICE (-3)       /* HIP runtime error                               */
#define DGW_EUNSUPPORTED (-4)  /* valid but not supported (degree, boundary, ...) */
#define DGW_EUNSTABLE (-5)     /* energy watchdog tripped (time step too large)   */
#define DGW_EBUSY (-6)         /* resource in use                                 */

enum { DGW_FLUX_UPWIND = 0, DGW_FLUX_CENTRAL = 1 };
/* Precision of the operator arithmetic.  DGW_FP32_SPLIT: 1D contractions and
 * flux arithmetic in FP32; state, stage and Taylor sums, metric terms and the
 * inverse mass factors in FP64. */
enum { DGW_FP64 = 0, DGW_FP32_SPLIT = 1 };
enum { DGW_SCHEME_LSRK54 = 0, DGW_SCHEME_ADER = 1 };
/* Unfused LSRK(5,4) variants, for the ablation of the fused vector update
 * (Sec. 4.3): the operator sweep stores L u and a separate pass updates the
 * registers, merged into one pass over du, L u and u (the paper's optimized
 * updater) or as three BLAS-1 passes (its standard one).  dgw_step_lsrk and
 * dgw_step_profile only; no sources. */
enum { DGW_SCHEME_LSRK54_MERGED_VU = 2, DGW_SCHEME_LSRK54_STANDARD_VU = 3 };
/* LSRK5(9): nine stages, order five, two registers (Sec. 2.2; the reference's
 * coefficients are not printed).  Two-register (2R) form: the Butcher tableau
 * has a_ij = b_j for j < i-1 and a free subdiagonal alpha; with U the
 * accumulated solution and Y the stage state, stage i computes
 * k = dt (L Y + s(t + c_i dt) g), U <- U + b_i k, Y <- U + (alpha_{i+1} - b_i) k.
 * The 17 coefficients are the real root of the 17 order-5 conditions named
 * by the 10-digit key alpha = (0.1702644982, -0.09676474868, 0.0244514839,
 * 0.1382907685, 0.2294641842, 0.5748250612, -0.1211285367, 0.09183392377),
 * b = (0.1804864076, 0.622352667, -0.4110536782, -0.01125784998,
 * 0.009612188747, 0.1576014651, 0.1129031225, 0.08522852155, 0.2541271558),
 * refined by Newton's method when the library loads.  Fused into the
 * operator sweep like DGW_SCHEME_LSRK54 (dgw_step_lsrk, dgw_step_profile,
 * dgw_solve_batch; sources allowed). */
enum { DGW_SCHEME_LSRK59 = 4 };
/* ADER flags: DGW_ADER_NOREDUCE evaluates every time derivative at k+1
 * points per direction (Alg. 2 without the degree reduction of Sec. 3.3).
 * DGW_ADER_HDG selects the HDG-ADER variant (Sec. 2.4, eq. hdg-ader): the
 * first element-local derivative of the Taylor sum is replaced by the DG
 * operator, u <- u + L(dt u + sum_{j>=1} dt^{j+1}/(j+1)! (-S)^{j-1} L u),
 * two operator sweeps and one TCK sweep per step; with the degree reduction
 * only (DGW_ADER_HDG | DGW_ADER_NOREDUCE: DGW_EUNSUPPORTED) and without
 * sources (DGW_EUNSUPPORTED). */
enum { DGW_ADER_REDUCE = 0, DGW_ADER_NOREDUCE = 1, DGW_ADER_HDG = 2 };
/* Reduction period of the TCK for the ablation of Sec. 3.3 (at most one of
 * these and DGW_ADER_NOREDUCE): DGW_ADER_REDUCE_EVERY_STEP projects every
 * time derivative by one point per direction (the variant the section
 * starts from), DGW_ADER_REDUCE_EVERY_THIRD every third derivative by three;
 * the default projects every second by two (Alg. 3).  The metric of those
 * reduced Gauss sets is built on the host at the first step that needs it
 * (the mesh's material callback and context must still be valid then), and
 * kept with the mesh.  No sources, no HDG-ADER (DGW_EUNSUPPORTED). */
enum { DGW_ADER_REDUCE_EVERY_STEP = 4, DGW_ADER_REDUCE_EVERY_THIRD = 8 };
/* Boundary codes of the neighbour table.  The paper leaves the boundary
 * conditions open (Sec. 2); the exterior state of a boundary face is built
 * from the own trace and goes through the interior flux with the own
 * impedance: DGW_BC_WALL is a rigid (sound-hard) wall, mirror state
 * p+ = p-, v+ = v- - 2 (v-.n) n (so v*.n = 0); DGW_BC_ABSORBING a first-order
 * absorbing face, zero exterior state (with the upwind flux only the outgoing
 * characteristic passes).  Both are linear in the trace, so the ADER update
 * applies them to the time-integrated Taylor sum unchanged. */
#define DGW_BC_WALL (-1)
#define DGW_BC_ABSORBING (-2)
/* DGW_BC_PRESCRIBED: the exterior state is given data, a superposition of
 * the plane waves of dgw_mesh_desc.plane_waves at the face point x:
 * p+ = sum A cos(k.x - omega t + phi), v+ = sum A cos(...) k / (|k| Z).  The
 * time t is the stage time in dgw_step_lsrk; dgw_step_ader uses the exact
 * time integral of that state over each step (the ADER update applies the
 * operator to the time-integrated Taylor sum, so its exterior state is the
 * integrated data); dgw_operator_apply takes t = 0.  Not with DGW_ADER_HDG. */
#define DGW_BC_PRESCRIBED (-3)
#define DGW_MAX_PLANE_WAVES 8
typedef struct dgw_plane_wave {
  double amplitude;          /* A                                               */
  double k[3];               /* wave vector, |k| > 0 (k[2] unused in 2D)        */
  double omega;              /* angular frequency (c |k| for a solution)        */
  double phase;              /* phi                                             */
  double impedance;          /* Z = rho c of the wave's medium, > 0             */
} dgw_plane_wave;
/* device = DGW_DEVICE_NONE builds the host-side setup only (no device
 * memory): the mesh can be inspected with dgw_mesh_get but not stepped. */
#define DGW_DEVICE_NONE (-1)

/* Storage basis of the state (Sec. 3.1 compares the two for the Runge-Kutta
 * operator).  DGW_BASIS_GL: Lagrange polynomials in the k+1 Gauss-Lobatto
 * points per direction, nodes on the faces; the kernels change to the Gauss
 * basis and back (Sec. 3.2).  DGW_BASIS_GAUSS: Lagrange polynomials in the
 * k+1 Gauss points (the collocated setup): u holds the values at the cell's
 * Gauss points in the same lexicographic order, the mass matrix is diagonal,
 * but a face trace needs the neighbour's whole line of values along the face
 * normal.  Same discrete operator: L_Gauss = S L_GL S^-1 with S the
 * tensor-product interpolation from the GL nodes to the Gauss points.  Every
 * call accepts either basis, in both precisions: states and source vectors
 * are in the mesh's storage basis.  With DGW_BASIS_GAUSS the ADER TCK reads
 * u without a basis change, its sum I (in the work buffer) stays in the GL
 * basis so that the update sweep gathers the neighbours' face nodes as with
 * GL storage, and the update writes u at the Gauss points without the final
 * basis change; the energy needs none either.
 * dgw_mesh_get(DGW_GET_NODE_COORDS) returns the GL nodes in both cases. */
#define DGW_BASIS_GL 0
#define DGW_BASIS_GAUSS 1

/* Material callback, evaluated on the host at mapped points during setup.
 * x: [npts][dim] physical points; writes rho[npts], c[npts]. */
typedef void (*dgw_material_fn)(const double* x, int64_t npts, int dim, double* rho, double* c,
                                void* ctx);

typedef struct dgw_mesh dgw_mesh;
typedef struct dgw_sources dgw_sources;

/* ---------------------------------------------------------------- b1 ---- */
typedef struct dgw_mesh_desc {
  int dim;                   /* 2 or 3                                          */
  int degree;                /* k, 1..8 (else DGW_EUNSUPPORTED)                 */
  int64_t n_cells;           /* >= 1                                            */
  int geo_degree;            /* q, 1..8; 0 = k                                  */
  const double* geo_nodes;   /* host [n_cells][(q+1)^dim][dim]; copied          */
  const int64_t* neighbors;  /* host [n_cells][2*dim]; a negative entry marks a */
                             /* boundary face: DGW_BC_WALL, DGW_BC_ABSORBING or */
                             /* DGW_BC_PRESCRIBED                               */
  const int* face_orient;    /* NULL: every neighbour meets face f with its     */
                             /* face f^1, tangential coordinates aligned.  Else */
                             /* host int32 [n_cells][2*dim], 8 f' + o: the      */
                             /* neighbour's face f' and the orientation o that  */
                             /* maps the own tangential coordinates (s, t) (the */
                             /* other directions in increasing order) to the    */
                             /* neighbour's: bit 2 swaps them first, bit 0      */
                             /* reverses the first, bit 1 the second (2D: bit 0 */
                             /* reverses s).  Must be mutually consistent.      */
  dgw_material_fn material;  /* required                                        */
  void* material_ctx;
  int flux;                  /* DGW_FLUX_*                                      */
  int precision;             /* DGW_FP64 or DGW_FP32_SPLIT                      */
  int device;                /* HIP device ordinal or DGW_DEVICE_NONE           */
  int max_batch;             /* >= 1: largest B accepted by the stepping calls  */
  int storage_basis;         /* DGW_BASIS_GL (0, default) or DGW_BASIS_GAUSS    */
  const dgw_plane_wave* plane_waves;  /* host [n_plane_waves]; copied; the    */
                             /* exterior state of DGW_BC_PRESCRIBED faces       */
  int n_plane_waves;         /* 0..DGW_MAX_PLANE_WAVES, >= 1 if any face is     */
                             /* DGW_BC_PRESCRIBED                               */
} dgw_mesh_desc;

/* Builds the setup of Sec. 3 on the host in FP64: 1D Gauss / GL rules and
 * the basis-change, collocation-derivative, projection and embedding
 * matrices (Sec. 3.1-3.3); the curved map at every point set (cell Gauss
 * points, face Gauss points, the reduced Gauss sets of the degree reduction,
 * Sec. 3.3); the pre-computed metric w det(J) J^-1, the inverse mass factors
 * 1/(w det J rho) and rho c^2/(w det J), face area vectors w det J J^-T n and
 * the impedances rho c of both sides of every face point.  Validates
 * det J > 0 at every point and that the neighbour table is conforming
 * (DGW_EINVAL otherwise) and uploads everything to the device, which the
 * mesh owns.  *out is NULL on error. */
dgw_status dgw_mesh_create(const dgw_mesh_desc* desc, dgw_mesh** out);

/* Convenience: the periodic unit box [0,1]^dim with ncell^dim cells, each node
 * X moved to X + amp prod_j sin(2 pi X_j) in every coordinate, geometry degree
 * q = k, neighbours by periodic wrap.  Other fields (storage_basis included)
 * as in dgw_mesh_desc. */
dgw_status dgw_mesh_create_box(int dim, int ncell, int degree, double deform_amp,
                               dgw_material_fn material, void* material_ctx, int flux,
                               int precision, int device, int max_batch, int storage_basis,
                               dgw_mesh** out);

/* A ready material: rho = rho0, c(x) = clamp(c0 + amp nmodes^-1/2 sum_i
 * a_i cos(2 pi m_i.x + phi_i), cmin, cmax).  Pass dgw_material_fourier with a
 * dgw_fourier_material* as ctx; nmodes <= 16. */
typedef struct dgw_fourier_material {
  int nmodes;
  int m[16][3];
  double a[16];
  double phi[16];
  double c0, amp, cmin, cmax, rho0;
} dgw_fourier_material;
void dgw_material_fourier(const double* x, int64_t npts, int dim, double* rho, double* c,
                          void* ctx);

/* ---------------------------------------------------------------- b2 ---- */
void dgw_mesh_destroy(dgw_mesh* mesh);

typedef struct dgw_mesh_info {
  int dim, degree, n1d, nodes_per_cell, n_comp, geo_degree;
  int64_t n_cells;
  int64_t dofs;              /* per batch member: n_cells (d+1) n^d              */
  int64_t state_bytes;       /* per batch member (FP64)                          */
  int64_t lsrk_work_bytes;   /* per batch member, work buffer of dgw_step_lsrk   */
  int64_t ader_work_bytes;   /* per batch member, work buffer of dgw_step_ader   */
  int64_t device_bytes;      /* device memory owned by the mesh                  */
  int n_levels;              /* Gauss sets of the degree reduction (Sec. 3.3)    */
  int level_points[8];       /* points per direction of each set                 */
  double h_min;              /* min over cells of h_K (see dt_unit)              */
  double c_max;              /* max of c over all cell Gauss points              */
  double dt_unit;            /* min_K(h_K / c_K) / k^1.5: dt = Cr * dt_unit      */
                             /* (Sec. 2.3; h_K = min over the cell's Gauss points */
                             /*  of the smallest singular value of J)            */
  int precision, flux, max_batch, device;
} dgw_mesh_info;
dgw_status dgw_mesh_info_get(const dgw_mesh* mesh, dgw_mesh_info* info);

/* Copies setup data to host memory (synchronous), for inspection:
 *  DGW_GET_NODE_COORDS  [n_cells][np][dim]   physical GL node positions
 *  DGW_GET_CELL_METRIC  [n_cells][d*d+2][np] w detJ (J^-1)_{ba} at index b*d+a,
 *                                            then 1/(w detJ rho), rho c^2/(w detJ)
 *  DGW_GET_FACE         [n_cells][2d][d+2][n^(d-1)] area vector a (d), Z-, Z+
 *  DGW_GET_LEVEL(l)     [n_cells][d*d+2][m^d] same as the cell metric at the
 *                       l-th reduced Gauss set (l >= 1), m = level_points[l] */
enum { DGW_GET_NODE_COORDS = 0, DGW_GET_CELL_METRIC = 1, DGW_GET_FACE = 2, DGW_GET_LEVEL0 = 16 };
#define DGW_GET_LEVEL(l) (DGW_GET_LEVEL0 + (l))
dgw_status dgw_mesh_get(const dgw_mesh* mesh, int what, double* host_out, int64_t count);

/* ---------------------------------------------------------------- b3 ---- */
/* out = L u = -M^-1 K u (Sec. 2.1, eq. matrix-tc-sd) for B members, no source.
 * One fused launch: GL->G basis change, pointwise metric, transposed
 * collocation derivative, upwind face integrals with the neighbours' GL face
 * nodes, inverse mass by basis change (Sec. 3.1).  u, out: device
 * [B][n_cells][d+1][np]; must not alias (DGW_EINVAL).  1 <= B <= max_batch. */
dgw_status dgw_operator_apply(dgw_mesh* mesh, const double* u, double* out, int B, void* stream);

/* ---------------------------------------------------------------- sources */
/* Point sources s_i(t) delta(x - x_i) on the pressure equation, one per batch
 * member (member i gets source i), with a Ricker wavelet
 * s(t) = amp (1 - 2 a tau^2) exp(-a tau^2), a = (pi f)^2, tau = t - t0.
 * Not part of the paper.  Positions are located on the host by Newton
 * iteration on the cell maps (lowest cell index wins); DGW_EINVAL if a point
 * is outside the mesh. */
typedef struct dgw_source_desc {
  int n;                     /* number of sources = batch members they serve     */
  const double* position;    /* host [n][dim]                                     */
  const double* frequency;   /* host [n], peak frequency f                        */
  const double* t0;          /* host [n] or NULL (t0 = 1.2 / f)                   */
  const double* amplitude;   /* host [n] or NULL (1)                              */
} dgw_source_desc;
dgw_status dgw_sources_create(dgw_mesh* mesh, const dgw_source_desc* desc, dgw_sources** out);
void dgw_sources_destroy(dgw_sources* src);

/* ---------------------------------------------------------------- b4 ---- */
/* nsteps steps of the five-stage fourth-order 2N-storage Runge-Kutta scheme
 * (Sec. 2.2, LSRK4(5); Carpenter-Kennedy coefficients) from t0 with step dt:
 * du <- A_i du + dt (L u + s(t + c_i dt) g); u <- u + B_i du.  scheme
 * DGW_SCHEME_LSRK54: the vector update is fused into the operator sweep (one
 * launch per stage); the unfused variants above: see there.  u advances
 * in place; work: device buffer of B * lsrk_work_bytes (stage register and
 * the ping-pong copy that keeps neighbours reading the old stage).  src may
 * be NULL (else src->n >= B).  dt <= 0 or non-finite: DGW_EINVAL. */
dgw_status dgw_step_lsrk(dgw_mesh* mesh, int scheme, double t0, double dt, int nsteps,
                         double* u, double* work, int B, const dgw_sources* src, void* stream);

/* ---------------------------------------------------------------- b5 ---- */
/* nsteps ADER steps of order k+1 (Sec. 2.3, eq. ader): sweep 1 evaluates the
 * cell-local Taylor-Cauchy-Kowalevski sum I in the collocated Gauss basis
 * with the degree reduction every second derivative (Sec. 3.2-3.3, Alg. 3)
 * and writes it in the GL basis; sweep 2 applies u <- u + L(I) (+ the exact
 * time integral of the source).  Contract as dgw_step_lsrk;
 * work = B * ader_work_bytes.  flags: DGW_ADER_REDUCE or DGW_ADER_NOREDUCE. */
dgw_status dgw_step_ader(dgw_mesh* mesh, int flags, double t0, double dt, int nsteps, double* u,
                         double* work, int B, const dgw_sources* src, void* stream);

/* dgw_step_ader without a work argument and without any device allocation,
 * for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same steps, kernels and
 * results as dgw_step_ader; the work registers (I and the ping-pong state)
 * live in a 64 MiB static device array that each device running the call
 * holds until the process ends.  2 * B * state_bytes above 64 MiB (i.e. more
 * than 4 Mi state values per member times B): DGW_EINVAL before any launch.
 * Reduction periods other than the default need their reduced levels, which
 * one dgw_step_ader call with those flags builds; until then
 * DGW_EUNSUPPORTED.  The array is shared by every call on one device and
 * keeps the last call's contents (nothing in it needs clearing: each step
 * writes its registers before reading them), so calls that overlap on one
 * device race: serialize them (one stream, or events). */
dgw_status dgw_step_ader_noalloc(dgw_mesh* mesh, int flags, double t0, double dt, int nsteps,
                                 double* u, int B, const dgw_sources* src, void* stream);

/* Per-kernel timing of nsteps steps (the component breakdown of Sec. 4.3,
 * Table 3): like dgw_step_lsrk / dgw_step_ader, with a HIP event pair on
 * `stream` around every launch.  out->ms[i] is the mean duration of one launch
 * of component i, out->launches[i] the number of launches; components:
 * LSRK: 0 = fused operator + vector update; unfused LSRK: 0 = operator
 * sweep, 1 = the stage's vector update pass(es); ADER: 0 = TCK sweep, 1 =
 * fused operator + update, and for DGW_ADER_HDG 2 = the operator sweep that
 * stores L u.  Synchronous. */
typedef struct dgw_profile {
  int n;
  double ms[4];
  int64_t launches[4];
  char names[4][32];
} dgw_profile;
dgw_status dgw_step_profile(dgw_mesh* mesh, int scheme, int ader_flags, double t0, double dt, int nsteps,
                            double* u, double* work, int B, const dgw_sources* src, void* stream,
                            dgw_profile* out);

/* Energy (twice the acoustic energy) sum_K (v, rho v)_K + (p, p/(rho c^2))_K
 * per member, by Gauss quadrature; host_out[B]; synchronous on stream. */
dgw_status dgw_energy(dgw_mesh* mesh, const double* u, int B, double* host_out, void* stream);

/* Launch shape of the operator (which = 0) or TCK (which = 1) kernels:
 * cells per workgroup and threads per workgroup.  A positive cells_per_group
 * selects one of the two compiled shapes (the LDS tile must fit 160 KiB) for
 * the TCK, or for the operator with every epilogue; threads are fixed by the
 * kernel and the cell size (256; the operator 1024 for 9^3 points, the TCK
 * 512 for 8^3 and 1024 for 9^3): a positive input must equal that.  The
 * current shape is returned (for which = 0 the one of the plain operator);
 * which = 2 and 3 report the shape of the operator with the LSRK and with
 * the ADER update epilogue, which = 4, 5, 6 the batch members one workgroup
 * of the operator with the store, LSRK and ADER update epilogue processes (1,
 * or 8 for the member-block variant that loads a cell's geometry once for 8
 * members; 3D only) in cells_per_group (input cells_per_group must be 0).
 * dgw_autotune times the compiled shapes of the operator with each of its
 * epilogues (and, for B > 1 in 3D, the member-block variant of each) and of
 * the TCK on scratch buffers for batch size B and keeps
 * the fastest of each (per process, keyed by device architecture, d, k,
 * precision, storage basis, B and cell count).  When the environment
 * variable DGW_AUTOTUNE_CACHE names a file, results are looked up there
 * first and appended there as JSON lines
 * ({"key": ..., "op_store": s, "op_lsrk": s, "op_ader_update": s, "tck": 0|1, "ms": {...}},
 * s = 0..3: bit 0 the cells-per-workgroup choice, bit 1 the member block);
 * entries that no longer fit the LDS are ignored. */
dgw_status dgw_launch_shape(dgw_mesh* mesh, int which, int* cells_per_group, int* threads);
dgw_status dgw_autotune(dgw_mesh* mesh, int B, void* stream);

/* ---------------------------------------------------------------- b6 ---- */
typedef struct dgw_solve_desc {
  int scheme;                /* DGW_SCHEME_LSRK54, DGW_SCHEME_LSRK59 or ADER      */
  int ader_flags;
  double courant;            /* used when dt <= 0: dt = courant * dt_unit         */
  double dt;                 /* rounded down so that dt = (t_end-t0)/nsteps       */
  double t0, t_end;
  const dgw_sources* sources;/* may be NULL                                       */
  int use_graph;             /* capture one step in a hipGraph and replay it      */
  int autotune;              /* time the launch shapes once and keep the fastest  */
  int watchdog_every;        /* energy check of every member every N steps (0 = off) */
  double watchdog_growth;    /* DGW_EUNSTABLE if a member's energy is not finite, or
                                exceeds growth (default 10) times its initial energy;
                                members that start at rest are checked for a finite
                                energy only                                       */
  void* stream;
} dgw_solve_desc;
typedef struct dgw_solve_report {
  int64_t steps;
  double dt, wall_s, dof_steps_per_s;
  double energy0, energy_end;  /* member 0 */
} dgw_solve_report;
/* Synchronous solve of B members from t0 to t_end; work as for the scheme. */
dgw_status dgw_solve_batch(dgw_mesh* mesh, const dgw_solve_desc* desc, double* u, double* work,
                           int B, dgw_solve_report* report);

/* ---------------------------------------------------------------- b7 ---- */
typedef struct dgw_request {
  double arrival_s;          /* seconds after serving starts                       */
  int dim, ncell, degree;
  int scheme;                /* DGW_SCHEME_LSRK54, DGW_SCHEME_LSRK59 or ADER; else */
                             /* the result is DGW_EINVAL                            */
  int precision;
  double t_end, courant, deform_amp;
  dgw_fourier_material material;
  double ic_center[3], ic_width; /* Gaussian pressure pulse, v = 0                 */
} dgw_request;
typedef struct dgw_result {
  dgw_status status;
  double t_arrive, t_admit, t_done;  /* seconds since serving started              */
  int64_t steps, dofs;
  double energy0, energy_end;
  double* state_host;        /* optional caller buffer [dofs] for the final state  */
} dgw_result;
typedef struct dgw_server_desc {
  int device;
  double hbm_budget_bytes;   /* admission budget for all live requests             */
  int max_live;              /* most requests in flight (streams)                  */
  int realtime;              /* 1: honour arrival_s; 0: all arrive at 0            */
  int progress;              /* 1: one line on stderr per finished request         */
} dgw_server_desc;
typedef struct dgw_serve_report {
  int n_done, n_failed;
  double wall_s, p50_s, p99_s, dof_steps_per_s, max_wait_s;
} dgw_serve_report;
/* Replays a request trace: a request is admitted once it has arrived and its
 * device footprint fits the budget; admitted requests run concurrently on
 * their own streams, a chunk of about 1e7 DoF-steps per scheduling round
 * each, and retire when done; states at the GL nodes.  Requests larger than
 * the whole budget fail with DGW_ENOMEM in their result; the others
 * continue.  Synchronous. */
dgw_status dgw_serve(const dgw_server_desc* desc, const dgw_request* reqs, int n, dgw_result* out,
                     dgw_serve_report* report);

/* Footprint in bytes that dgw_serve charges a request (mesh + state + work). */
int64_t dgw_request_footprint(const dgw_request* req);

/* ---------------------------------------------------------------- b8 ---- */
const char* dgw_last_error(void);
const char* dgw_version(void);

/* 1D tables of the setup, for inspection: what = 0 Gauss points, 1 Gauss
 * weights, 2 GL points, 3 GL weights (n values each, on [0,1]); 4 S (GL->G,
 * n x n, S[q][j] = l^GL_j(xi^G_q)), 5 S^-1, 6 D (collocation derivative on
 * the Gauss points, D[q][j] = l^G_j'(xi^G_q)). */
dgw_status dgw_basis_1d(int n, int what, double* host_out);

/* Coefficients of the low-storage Runge-Kutta schemes in use (Sec. 2.2),
 * for inspection; host_out: caller-owned host buffer.  DGW_SCHEME_LSRK54:
 * 15 values A (5), B (5), c (5) of the 2N form; DGW_SCHEME_LSRK59: 26 values
 * alpha (8), b (9), c (9) of the 2R form (DGW_EDEVICE if its refinement did
 * not converge).  Other schemes or host_out NULL: DGW_EINVAL. */
dgw_status dgw_lsrk_coefficients(int scheme, double* host_out);

#ifdef __cplusplus
}
#endif
#endif /* DGW_H */
