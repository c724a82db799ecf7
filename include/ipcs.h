/*
 * ipcs.h -- C ABI of the MI355X (gfx950) incremental pressure-correction
 * (IPCS) solver for the incompressible Navier-Stokes equations with
 * Taylor-Hood elements: P2-P1 on triangles and tetrahedra, P3-P2 on
 * triangles.
 *
 * What is computed (arXiv 2605.25403, FEALPy.CFD):
 *   PDE      : Section 2.1, eq. (3): du/dt - nu Lap u + (u.grad)u + grad p = f,
 *              div u = 0, density rho = 1 unless set.
 *   Spaces   : Section 2.2.1, eqs. (4)-(5): V_h = continuous P2 per velocity
 *              component with Dirichlet data, Q_h = continuous P1 pressure;
 *              or P3 and P2 (Section 5.1, table "convergence_p3_p2").
 *   Scheme   : Section 2.2.1, eq. (9) (IPCS): momentum with explicit convection
 *              ((u^n.grad)u^n, v) and pressure p^n, pressure-increment Poisson,
 *              velocity correction. The Poisson right-hand side is taken as
 *              -(rho/dt)(div u*, q), the sign for which the correction makes
 *              u^{n+1} discretely divergence-free; the pressure is fixed by zero
 *              integral mean.
 *   Workflow : Section 4.2 (create mesh, choose spaces, choose method, run,
 *              read back) and the step decomposition of Section 3.2.3 (matrix,
 *              right-hand side and coefficient-update interfaces per step).
 *
 * Conventions
 *   - Every call returns IPCS_OK (0) or a negative status; nothing throws.
 *     ipcs_last_error() returns a thread-local message for the last failure on
 *     the calling thread (valid until the next call on that thread).
 *   - Handles are opaque and owned by the library; destroy calls accept NULL.
 *   - Host arrays passed in are copied; output buffers are caller-allocated and
 *     come with a capacity in elements; a buffer that is too small gives
 *     IPCS_E_INVALID and writes nothing.
 *   - Device memory: a run lives entirely inside one caller-provided device
 *     workspace (dev_ws, ws_bytes >= ipcs_run_workspace_bytes); the library
 *     never frees it. Besides small pinned host staging buffers, the only
 *     other allocation is ipcs_batch_step's stream-ordered one (hipMallocAsync,
 *     released with hipFreeAsync before it returns) for the descriptors of its
 *     shared launches; ipcs_batch_step_noalloc takes them from a fixed array
 *     instead. All device work of a run is issued on the HIP stream given at
 *     creation (or to the batch step).
 *   - Layout: velocity is component-major [dim][N2] (N2 velocity DOFs per
 *     component, N1 pressure DOFs; the numbering is stated at
 *     ipcs_mesh_unit_square_pair). All host-side fields are FP64, whatever
 *     the internal precision.
 *   - Threading: a run is not thread-safe; distinct runs may be driven from
 *     distinct threads.
 */
#ifndef IPCS_H
#define IPCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
  IPCS_OK = 0,
  IPCS_E_INVALID = -1,        /* bad argument, handle or buffer size          */
  IPCS_E_NOMEM = -2,          /* workspace too small / host allocation failed */
  IPCS_E_DEVICE = -3,         /* HIP runtime error                            */
  IPCS_E_NOT_CONVERGED = -4,  /* a Krylov solve hit maxit, or its tolerance is
                               * out of reach: three restarts in a row left
                               * the true residual b - A x above 90% of its
                               * least value so far                           */
  IPCS_E_BREAKDOWN = -5,      /* unrecoverable Krylov breakdown               */
  IPCS_E_NONFINITE = -6,      /* NaN/Inf met in a solve                       */
  IPCS_E_STATE = -7,          /* call not valid in the run's current state    */
  IPCS_E_CAPACITY = -8        /* admission refused (workspace budget)         */
};

const char* ipcs_last_error(void);

/* ---------------------------------------------------------------- mesh */
typedef struct ipcs_mesh_s* ipcs_mesh;

/* Taylor-Hood pairs (Section 2.2.1, eqs. (4)-(5); Section 4.2 takes P2-P1,
 * the higher-order study of Section 5.1, table "convergence_p3_p2", P3-P2).
 * The space and pattern names below keep the P2-P1 pair's vocabulary:
 * "P2" is the velocity space and "P1" the pressure space of the mesh's pair
 * (for IPCS_PAIR_P3P2: P3 velocity, P2 pressure). */
enum {
  IPCS_PAIR_P2P1 = 0,          /* triangles and tetrahedra                      */
  IPCS_PAIR_P3P2 = 1           /* triangles only                                */
};
enum { IPCS_SPACE_P1 = 1, IPCS_SPACE_P2 = 2 };   /* pressure, velocity space */
enum {                         /* sparsity patterns of the step's matrices      */
  IPCS_PATTERN_P2P2 = 0,       /* M, K, C, A (velocity x velocity)             */
  IPCS_PATTERN_P1P1 = 1,       /* Kp (pressure x pressure)                     */
  IPCS_PATTERN_P1P2 = 2,       /* D_c, divergence (pressure rows, velocity cols) */
  IPCS_PATTERN_P2P1 = 3        /* G_c, gradient (velocity rows, pressure cols) */
};

typedef struct {
  int32_t dim;                 /* 2 or 3                                       */
  int64_t nv, nc;              /* vertices, cells                              */
  int64_t n1, n2;              /* pressure and velocity DOFs per component     */
  int64_t nnz[4];              /* nnz of IPCS_PATTERN_* patterns               */
  int64_t nb2;                 /* boundary velocity nodes                      */
} ipcs_counts;

/* Unit square, nx x ny squares, each split by its SW-NE diagonal into two
 * counter-clockwise triangles; vertex (i,j) = (i/nx, j/ny) has index
 * j*(nx+1)+i (Section 2.2.1: conforming simplicial mesh T_h). */
int ipcs_mesh_unit_square(int32_t nx, int32_t ny, ipcs_mesh* out);
/* The same square with the DOF maps of a Taylor-Hood pair (IPCS_PAIR_*).
 * Numbering of every array that crosses this interface (fields, DOF
 * coordinates, cell DOF tables, boundary masks, patterns, matrices):
 * velocity DOFs (P2-P1) are the vertices in input order, then the edge
 * midpoints with the edges sorted by (lower, higher) vertex; velocity DOFs
 * (P3-P2) are the vertices, then two nodes per edge in that edge order (the
 * node at (2 x_lo + x_hi)/3, then the one at (x_lo + 2 x_hi)/3), then one node
 * per cell at its centroid, in cell order (triangles), or one node per face
 * at its centroid, the faces sorted by their (ascending) vertex triples
 * (tetrahedra). Pressure DOFs: P1, the vertices;
 * P2 (P3-P2 pair), the vertices, then the edge midpoints in edge order.
 * Internally the library numbers the non-vertex velocity nodes in
 * lexicographic order of their coordinates (last coordinate most
 * significant), so that neighbouring nodes have neighbouring indices; it
 * converts at this interface, outside any timed step. */
int ipcs_mesh_unit_square_pair(int32_t nx, int32_t ny, int32_t pair, ipcs_mesh* out);
/* Unit cube, nx*ny*nz cubes, each split into the 6 Kuhn tetrahedra around its
 * main diagonal; vertex (i,j,k) has index (k(ny+1)+j)(nx+1)+i. */
int ipcs_mesh_unit_cube(int32_t nx, int32_t ny, int32_t nz, ipcs_mesh* out);
/* The same cube with the DOF maps of a Taylor-Hood pair (IPCS_PAIR_*;
 * numbering as for ipcs_mesh_unit_square_pair). */
int ipcs_mesh_unit_cube_pair(int32_t nx, int32_t ny, int32_t nz, int32_t pair, ipcs_mesh* out);
/* Any conforming simplicial mesh: x[nv*dim] coordinates, cells[nc*(dim+1)]
 * vertex indices (0-based). Cells of negative orientation are accepted. */
int ipcs_mesh_from_arrays(int32_t dim, int64_t nv, const double* x, int64_t nc,
                          const int32_t* cells, ipcs_mesh* out);
/* The same with a Taylor-Hood pair (IPCS_PAIR_*). */
int ipcs_mesh_from_arrays_pair(int32_t dim, int64_t nv, const double* x, int64_t nc,
                               const int32_t* cells, int32_t pair, ipcs_mesh* out);
/* The mesh's Taylor-Hood pair (IPCS_PAIR_*). */
int ipcs_mesh_pair(ipcs_mesh m, int32_t* pair);
int ipcs_mesh_counts(ipcs_mesh m, ipcs_counts* out);
/* Coordinates of the DOFs of a space, [n*dim]. cap in doubles. */
int ipcs_mesh_dof_coords(ipcs_mesh m, int32_t space, double* out, int64_t cap);
/* Cell -> DOF table of a space, [nc * nloc] (P2 local order: vertices, then
 * edges v1v2, v2v0, v0v1 (2D) or 01,02,03,12,13,23 (3D); P3 local order:
 * vertices, then for each edge (a, b) of v1v2, v2v0, v0v1 the node nearer a
 * and the node nearer b, then the centroid). cap in int32s. */
int ipcs_mesh_cell_dofs(ipcs_mesh m, int32_t space, int32_t* out, int64_t cap);
/* Boundary flags of the velocity nodes (1 = on the boundary), [n2]. */
int ipcs_mesh_boundary(ipcs_mesh m, uint8_t* out, int64_t cap);
/* CSR pattern (row pointer [rows+1], sorted column indices [nnz]). */
int ipcs_mesh_pattern(ipcs_mesh m, int32_t which, int32_t* rowptr, int64_t cap_rows,
                      int32_t* col, int64_t cap_nnz);
/* Row partition of the pressure-pressure pattern IPCS_PATTERN_P1P1 (the rows
 * of Kp, the matrix of the pressure-increment Poisson problem, Section 2.2.1,
 * eq. (9), second line) into parts of at most rows_max rows (64..2048) that
 * the one-kernel-per-iteration Poisson CG uses (host data, for inspection;
 * ownership stays with the mesh, the arrays are copied out). Parts are compact
 * patches of pressure nodes (recursive coordinate bisection); rows are
 * renumbered part by part ("part order"). sizes[0..4]
 * receives nparts, the halo length, the number of SELL-64 slices, the number
 * of entries and the largest own + halo count of a part. With non-NULL
 * arrays also: perm[n1] (part-order row -> original row), part_ptr[nparts+1],
 * halo_ptr[nparts+1], halo[] (part-order rows each part reads from other
 * parts), slice_ptr[nparts+1] (first slice of each part), sptr[nslices+1]
 * (entry offsets; entry k of a part's local row l = 64 j + q sits at
 * sptr[slice_ptr[p] + j] + 64 k + q), lcol[] (local columns: < own for the
 * part's rows, own + h for halo[halo_ptr[p] + h]) and src[] (entry index in
 * the global SELL-64 layout of the pattern, -1 for padding). The arrays must
 * be all NULL or all non-NULL (halo may be NULL when sizes[1] is 0) and as
 * large as sizes[] says; IPCS_E_INVALID otherwise. */
int ipcs_mesh_p1_partition(ipcs_mesh m, int32_t rows_max, int64_t sizes[5], int32_t* perm,
                           int32_t* part_ptr, int32_t* halo_ptr, int32_t* halo,
                           int32_t* slice_ptr, int32_t* sptr, uint16_t* lcol, int32_t* src);
/* The degree-5 cell quadrature rule the kernels use for the P2-P1 pair, in
 * barycentric coordinates lam[nq*(dim+1)] with weights w[nq] summing to
 * 1/dim!. *nq receives the number of points; pass NULL buffers to query it.
 * (P3-P2 runs use the rule of ipcs_quadrature_rule_pair.) */
int ipcs_quadrature_rule(int32_t dim, int32_t* nq, double* lam, double* w, int64_t cap);
/* The cell rule of a Taylor-Hood pair, same conventions. IPCS_PAIR_P2P1: the
 * rule above. IPCS_PAIR_P3P2 (its convection integrand has degree 8):
 * triangles, the collapsed product of two 5-point Gauss-Legendre rules (25
 * points, exact to degree 8); tetrahedra, Stroud's conical product of 5-point
 * Gauss-Jacobi rules (125 points, exact to degree 9), point q = 25 i + 5 j + k
 * from the i-th, j-th and k-th nodes of the rules in x, y/(1-x) and
 * z/((1-x)(1-y/(1-x))). */
int ipcs_quadrature_rule_pair(int32_t dim, int32_t pair, int32_t* nq, double* lam, double* w,
                              int64_t cap);
void ipcs_mesh_destroy(ipcs_mesh m);

/* ---------------------------------------------------------------- runs */
typedef struct ipcs_run_s* ipcs_run;

/* Precision forms. IPCS_FP64: every value and operation in FP64.
 * IPCS_MIXED: quadrature, assembly arithmetic and stored matrix values in FP32
 * (cell geometry is formed in FP64 and then rounded); fields, Krylov vectors,
 * dot products, Jacobi diagonals and Dirichlet lifting in FP64, and SpMV
 * products accumulated in FP64. The divergence matrices D_c stay FP64: the
 * pressure right-hand side -(rho/dt) sum_c D_c U*_c cancels to within a
 * factor of about 1e7 of its terms' magnitudes on fine meshes, so FP32 values
 * would leave it dominated by their rounding. The pressure Poisson solve is an FP64
 * iterative refinement on the FP64 Kp, to ||r - Kp dP|| <= tol_ir ||r||,
 * around Jacobi-CG on Kp rounded to FP32. Each pass asks the inner CG for the
 * reduction still needed, but not below half of the reduction the previous
 * pass achieved, nor below tol_p; an inner breakdown (the rounded singular
 * Kp can be marginally indefinite) ends that pass at its last iterate and
 * sets a floor (1e-6, then 100 times higher) for later passes. At most 30
 * passes. The momentum and
 * correction solves run on the FP32 matrices to tol_mom / tol_corr. */
enum { IPCS_FP64 = 0, IPCS_MIXED = 1 };
/* Convection forms. IPCS_CONV_EXPLICIT: eq. (9) as printed, the convection
 * term with u^n on the right-hand side (b = (M/dt - C(U^n)) U^n - G P^n + F)
 * and the constant A = M/dt + nu K. IPCS_CONV_SEMI_IMPLICIT: the convection
 * operator moves into the momentum matrix, A^n = M/dt + nu K + C(U^n), with
 * its Dirichlet elimination and lifting re-formed every step, and
 * b = M U^n / dt - G P^n + F; BiCGStab then solves a nonsymmetric system
 * (Section 2.2.1, eq. (9), first line, with the convection term linearized
 * at u^n). */
enum { IPCS_CONV_EXPLICIT = 0, IPCS_CONV_SEMI_IMPLICIT = 1 };
/* Projection schemes of Section 2.2.1. IPCS_SCHEME_IPCS: eq. (9), the
 * incremental pressure correction (momentum with -(p^n, div v), Poisson for
 * the increment, P^{n+1} = P^n + dP). IPCS_SCHEME_CHORIN: the non-incremental
 * projection of Chorin and Temam stated before it (eq. (8)): no pressure term
 * in the momentum step, the Poisson solve gives P^{n+1} itself (shifted to
 * zero integral mean) and the correction uses it; the right-hand-side sign
 * is read as for IPCS. */
enum { IPCS_SCHEME_IPCS = 0, IPCS_SCHEME_CHORIN = 1 };
/* Start of the pressure Poisson solve (eq. (9), second line; Section 2.2.1
 * fixes the system, not the Krylov start). IPCS_START_ZERO: dP = 0 at every
 * step. IPCS_START_PREVIOUS: the previous step's dP (IPCS: the last
 * increment; Chorin-Temam: the last pressure), which the stopping test
 * ||r - Kp dP|| <= tol_p ||r|| judges the same way, so the result meets the
 * same tolerance (with a few percent fewer iterations on the Taylor-Green
 * and Beltrami problems, where dP changes by ~1e-3 of itself per step). In
 * the mixed form the first refinement pass's inner solve starts there (the
 * refinement itself still starts from dP = 0). The first step after
 * ipcs_run_create, ipcs_set_builtin_solution or ipcs_set_state starts from
 * 0, so a run resumed from a saved state differs from the uninterrupted one
 * within the tolerance (not bit for bit, as it does with IPCS_START_ZERO). */
enum { IPCS_START_ZERO = 0, IPCS_START_PREVIOUS = 1 };
/* Start of the momentum solve (eq. (9), first line; Section 2.2.1 fixes the
 * system, not the Krylov start), both judged by the same stopping test
 * ||b - A U*|| <= tol_mom ||b||. IPCS_MSTART_EXTRAPOLATED (default): the
 * extrapolation of the previous steps' tentative velocities to t^(n+1),
 * quadratic (3 U*^n - 3 U*^(n-1) + U*^(n-2)) once four steps have completed,
 * linear (2 U*^n - U*^(n-1)) after two or three, U^n before, counted since
 * ipcs_run_create, ipcs_set_builtin_solution, ipcs_set_state,
 * ipcs_set_viscosity, ipcs_set_time_step or a new forcing or Dirichlet
 * callback (each of which clears the history; a failed step keeps it). The
 * quadratic start leaves out the first step after a clear, whose tentative
 * velocity carries the scheme's initial layer. Its residual is O(dt^3) where
 * U^n's is O(dt) (at 512^2, dt = 1e-3: 4e-10 against 2e-5 of ||b||, 13
 * BiCGStab iterations against 39; linear: 2e-8, 22). A step then depends
 * on the previous tentative velocities as well as on (U^n, P^n): a run resumed
 * through ipcs_set_state differs from the uninterrupted one within the
 * tolerance, not bit for bit. IPCS_MSTART_STATE: U^n at every step, a step
 * is a function of (U^n, P^n, t) alone. Dirichlet rows start at their data
 * either way. */
enum { IPCS_MSTART_EXTRAPOLATED = 0, IPCS_MSTART_STATE = 1 };

typedef struct {
  double nu;            /* kinematic viscosity                                 */
  double rho;           /* density in the pressure steps (default 1)          */
  double dt;            /* time step                                           */
  double t0;            /* initial time                                        */
  int32_t precision;    /* IPCS_FP64 or IPCS_MIXED                             */
  int32_t convection;   /* IPCS_CONV_EXPLICIT (eq. (9)) or SEMI_IMPLICIT       */
  double tol_mom;       /* relative residual tolerance, momentum BiCGStab      */
  double tol_p;         /* pressure Poisson PCG (mixed: inner, see above)      */
  double tol_corr;      /* velocity-correction PCG                             */
  double tol_ir;        /* mixed form: FP64 iterative-refinement tolerance     */
  int32_t maxit;        /* iteration cap per solve                             */
  int32_t check_every;  /* most iterations a solve launches between two status
                         * polls near its expected end (fewer when one
                         * iteration costs more than a poll)                */
  int32_t callbacks;    /* 1: reserve staging for host-callback forcing        */
  int32_t poisson_part_rows; /* pressure Poisson CG form: 0 (default) one kernel
                           * per iteration on a row partition of Kp into parts
                           * of at most 384 rows, falling back to two kernels
                           * where a part's halo does not fit in LDS; 64..2048
                           * the same with that part size (IPCS_E_CAPACITY if
                           * it does not fit); -1 two kernels per iteration
                           * (SpMV, then the vector update)                  */
  int32_t scheme;       /* IPCS_SCHEME_IPCS (default) or IPCS_SCHEME_CHORIN    */
  int32_t poisson_s;    /* CG iterations per launch of the one-kernel Poisson
                         * CG: 1 (Chronopoulos-Gear CG) or 2 (s-step CG: two
                         * iterations of the same Jacobi-PCG per launch, from
                         * a basis of the matrix powers and one reduction of
                         * its Gram matrix; needs the part's second halo ring
                         * in LDS); 0 (default) chooses 1                    */
  int32_t poisson_start; /* IPCS_START_ZERO (default) or IPCS_START_PREVIOUS  */
  int32_t momentum_start; /* IPCS_MSTART_EXTRAPOLATED (default) or
                           * IPCS_MSTART_STATE                               */
} ipcs_params;

/* nu=0.01, rho=1, dt=1e-3, t0=0, FP64, explicit, tolerances 1e-12
 * (tol_ir 1e-10), maxit 20000, check_every 16, callbacks 0, the
 * extrapolated momentum start and the zero Poisson start. */
void ipcs_params_default(ipcs_params* p);

/* Device workspace a run of this mesh needs (its whole HBM footprint): the
 * matrices of eq. (9) (M, K, Kp, D_c, G_c, A, the convection matrix of
 * Section 2.2.1), the fields U^n, P^n, U*, dP (with the extrapolated
 * momentum start, also the three previous steps' U*) and the Krylov vectors of
 * the three solves. *bytes receives the size; IPCS_E_INVALID for a bad mesh or
 * parameters. The caller allocates it (device memory, 256-byte aligned). */
int ipcs_run_workspace_bytes(ipcs_mesh m, const ipcs_params* p, int64_t* bytes);
/* Sets up one IPCS run (the time loop of Section 2.2.1 on the spaces of
 * eqs. (4)-(5)): uploads the mesh data and assembles the constant matrices
 * of eq. (9) (M, K, Kp, D_c, G_c, A = M/dt + nu K with Dirichlet rows/columns
 * eliminated) on the device. dev_ws: the caller's device workspace of
 * ws_bytes bytes (IPCS_E_NOMEM if smaller than ipcs_run_workspace_bytes); it
 * stays owned by the caller and must outlive the run.
 * The initial state is zero until ipcs_set_state / ipcs_set_builtin_solution.
 * hip_stream is a hipStream_t (NULL = default stream). The mesh may be
 * destroyed afterwards. */
int ipcs_run_create(ipcs_mesh m, const ipcs_params* p, void* dev_ws, int64_t ws_bytes,
                    void* hip_stream, ipcs_run* out);
/* nu of eq. (1) and dt of eq. (9); A = M/dt + nu K is re-formed (and its
 * elimination and Jacobi diagonal) before the next step. IPCS_E_INVALID for
 * nu < 0 or dt <= 0. */
int ipcs_set_viscosity(ipcs_run r, double nu);
int ipcs_set_time_step(ipcs_run r, double dt);

/* Host callback evaluating a vector field at npts points x[npts*dim] at time
 * t into out[npts*dim]. */
typedef void (*ipcs_field_fn)(void* ctx, int32_t dim, int64_t npts, const double* x,
                              double t, double* out);
/* Body force f (eq. (3)); NULL means f = 0. Evaluated on the host at the
 * quadrature points every step (slow path, for tests); needs a run created
 * with params.callbacks = 1 (else IPCS_E_STATE). */
int ipcs_set_forcing(ipcs_run r, ipcs_field_fn f, void* ctx);
/* Dirichlet data g (the velocity on the boundary, H^1_0 lifting of V_h);
 * evaluated on the host at the boundary velocity nodes every step. */
int ipcs_set_dirichlet(ipcs_run r, ipcs_field_fn g, void* ctx);

enum {
  IPCS_SOL_TAYLOR_GREEN_2D = 1, /* prm = {k}; f = 0                               */
  IPCS_SOL_JOHN_2D = 2,         /* Section 5.1 benchmark; prm unused             */
  IPCS_SOL_BELTRAMI_3D = 3,     /* Ethier-Steinman, prm = {a, d}; f = 0           */
  IPCS_SOL_POLY_STEADY_2D = 4,  /* u=(y^2,x^2), p=x+y-1                           */
  IPCS_SOL_POLY_STEADY_3D = 5,  /* u=(y^2+z^2,z^2+x^2,x^2+y^2), p=x+y+z-3/2      */
  IPCS_SOL_POLY_CUBIC_2D = 6,   /* u=(x^3+2x^2y, -3x^2y-2xy^2), p=x^2-y^2+xy-1/4,
                                 * steady, f = (u.grad)u - nu Lap u + grad p: a
                                 * fixed point of the P3-P2 step                 */
  IPCS_SOL_STEADY_PAPER_2D = 7, /* the steady example of Section 4.2:
                                 * u = 10x^2(x-1)^2 y(y-1)(2y-1),
                                 * v = -10x(x-1)(2x-1) y^2(y-1)^2,
                                 * p = 10(2x-1)(2y-1), f = -nu Lap u + (u.grad)u
                                 * + grad p (steady solver only)                 */
  IPCS_SOL_POLY_CUBIC_3D = 8    /* u=(y^3+z^2, z^3+x^2, x^3+y^2),
                                 * p=xy+yz+zx-3/4, steady, f as for
                                 * IPCS_SOL_POLY_CUBIC_2D: a fixed point of the
                                 * P3-P2 step on tetrahedra                     */
};
/* Closed-form manufactured solution evaluated on the device: Dirichlet data,
 * forcing and the initial state U = I_h u(t), P = I_h p(t) shifted to zero
 * integral mean, at the run's current time. */
int ipcs_set_builtin_solution(ipcs_run r, int32_t kind, const double* prm, int32_t nprm);
/* Initial state / resume: u[dim*N2], p[N1] used as given, time t. */
int ipcs_set_state(ipcs_run r, const double* u, const double* p, double t);

typedef struct {
  int32_t status;           /* IPCS_OK or the failing status                    */
  int32_t it_mom[3];        /* BiCGStab iterations per component                */
  int32_t it_p;             /* Poisson PCG iterations (inner total, mixed form) */
  int32_t it_corr[3];       /* correction PCG iterations per component          */
  int32_t ir_outer;         /* mixed form: refinement sweeps of the Poisson     */
  int32_t failed_solve;     /* 0 none, 1 momentum, 2 pressure, 3 correction     */
  int32_t checks_p;         /* Poisson: true-residual checks b - A x (1: the
                             * recursive residual was confirmed at once; each
                             * further check follows a restart)                */
  int32_t reserved;
  double res_mom[3], res_p, res_corr[3];   /* final relative residuals         */
  double t;                 /* time reached                                     */
  float ms_asm, ms_mom, ms_p, ms_corr;     /* phase times (stream events)      */
} ipcs_step_stats;

/* Advance nsteps IPCS steps. stats may be NULL or hold nsteps entries. On a
 * failure the state stays at the last completed step and the status of the
 * failing solve is returned. */
int ipcs_advance(ipcs_run r, int32_t nsteps, ipcs_step_stats* stats);

enum { IPCS_PHASE_ASM = 0, IPCS_PHASE_MOMENTUM = 1, IPCS_PHASE_PRESSURE = 2,
       IPCS_PHASE_CORRECTION = 3 };
/* One sub-step of eq. (9) at a time (ASM: Dirichlet data, forcing, C(U^n) and
 * the momentum right-hand side; MOMENTUM: u*; PRESSURE: dP and its right-hand
 * side; CORRECTION: u^{n+1}, P^{n+1}, time advance). Phases must be called in
 * order; ipcs_advance is equivalent to the four in sequence. */
int ipcs_step_phase(ipcs_run r, int32_t phase, ipcs_step_stats* stats);

/* Read-back of the discrete solution of eq. (9) after the last step: the
 * velocity coefficients u_h in V_h (eq. (4)), [dim][N2] component-major, and
 * the pressure p_h in Q_h (eq. (5)), [N1], in the interface numbering, into
 * host memory of cap doubles (IPCS_E_INVALID if smaller); t^n. Synchronizes
 * the run's stream. */
int ipcs_get_velocity(ipcs_run r, double* u, int64_t cap);
int ipcs_get_pressure(ipcs_run r, double* p, int64_t cap);
int ipcs_get_time(ipcs_run r, double* t);

enum { IPCS_FIELD_U = 0, IPCS_FIELD_P = 1, IPCS_FIELD_USTAR = 2, IPCS_FIELD_DP = 3,
       IPCS_FIELD_RHS_MOM = 4, IPCS_FIELD_RHS_P = 5 };
/* Intermediate vectors of the current step (after the phase that makes them). */
int ipcs_get_field(ipcs_run r, int32_t which, double* out, int64_t cap);

enum { IPCS_MAT_M = 0, IPCS_MAT_K = 1, IPCS_MAT_KP = 2, IPCS_MAT_A = 3,
       IPCS_MAT_E = 4,          /* M/dt - C(U^n) (explicit form) or M/dt + C(U^n)
                                 * (semi-implicit), assembled in the ASM phase */
       IPCS_MAT_D0 = 8,         /* D_c = IPCS_MAT_D0 + c                          */
       IPCS_MAT_G0 = 12,        /* G_c = IPCS_MAT_G0 + c                          */
       IPCS_MAT_A_ELIM = 16,    /* momentum matrix, Dirichlet-eliminated (semi-
                                 * implicit: of the current step)             */
       IPCS_MAT_M_ELIM = 17 };
/* Copy a device matrix to the host as CSR (values in FP64). rowptr/col may be
 * NULL to fetch values only. */
int ipcs_export_matrix(ipcs_run r, int32_t which, int32_t* rowptr, int64_t cap_rows,
                       int32_t* col, double* val, int64_t cap_nnz);

/* One IPCS step (eq. (9)) for every run in runs[0..nruns) on one stream
 * (serving form). Assembly and right-hand sides are launched run by run; each
 * Krylov iteration of all runs is one set of shared launches, with per-run
 * scalars, reductions and stopping decisions, so every run's result is bitwise
 * the one it gets when stepped alone. Runs may differ in mesh, viscosity and
 * time step, and may mix the FP64 and mixed forms; they must share the
 * dimension and be between steps. A run whose solve fails keeps its state at
 * the last completed step (stats[i].status and failed_solve say which); the
 * others complete their step. Returns IPCS_OK or the first failure. stats may
 * be NULL or hold nruns entries; their phase times are the batch's. */
int ipcs_batch_step(ipcs_run* runs, int32_t nruns, void* hip_stream, ipcs_step_stats* stats);

/* Size of the fixed device array of ipcs_batch_step_noalloc, per GPU. */
#define IPCS_BATCH_SCRATCH_BYTES (16u << 20)
/* Most runs in one ipcs_batch_step_noalloc call. */
#define IPCS_BATCH_NOALLOC_MAX_RUNS 256
/* ipcs_batch_step for callers that cannot allocate memory (serving loops that
 * must not call hipMalloc, harnesses that forbid device or pinned-host
 * allocation once set up). It computes what ipcs_batch_step computes, with the
 * same kernels, block decompositions and reductions, so each run's result is
 * bitwise the same; it allocates nothing: the descriptors of each shared
 * Krylov solve go into a fixed device array of IPCS_BATCH_SCRATCH_BYTES that
 * every GPU the library runs on holds until the process ends, the status
 * polls into a fixed host array per GPU, and the batch's phase times are
 * taken with runs[0]'s own events. The runs must be on the current device.
 * Before any work it checks the batch: more than IPCS_BATCH_NOALLOC_MAX_RUNS
 * runs, or descriptors that need more than the array (runs with many blocks,
 * such as hundreds of the largest 2D meshes), give IPCS_E_CAPACITY and leave
 * every run as it was. Calls on one GPU share that GPU's arrays and each call
 * reuses them from solve to solve: two calls that overlap on one GPU (from
 * two host threads, or on two streams) race, and must not be made. */
int ipcs_batch_step_noalloc(ipcs_run* runs, int32_t nruns, void* hip_stream,
                            ipcs_step_stats* stats);

enum {                            /* kernels of the step, for the timing hooks       */
  IPCS_KERNEL_PCG_SPMV_P = 0,     /* Poisson CG: w = Kp u, partial u.w               */
  IPCS_KERNEL_PCG_UPDATE_P = 1,   /* Poisson CG: p, s, x, r, u updates; r.u, r.r     */
  IPCS_KERNEL_ASM_CONV = 2,       /* convection assembly E = M/dt -+ C(U^n): row-
                                   * owner (2D), or the cell-batched local matrices
                                   * (3D, first pass)                               */
  IPCS_KERNEL_BICG_SPMV = 3,      /* momentum BiCGStab: v = A phat, rhat.v           */
  IPCS_KERNEL_PCG_SPMV_M = 4,     /* correction CG: w = M u, u.w (all components)   */
  IPCS_KERNEL_BICG_SPMV_T = 5,    /* momentum BiCGStab: t = A shat, t.s, t.t, ...    */
  IPCS_KERNEL_BICG_UPDATE_S = 6,  /* momentum BiCGStab: s = r - alpha v, shat        */
  IPCS_KERNEL_BICG_UPDATE_X = 7,  /* momentum BiCGStab: x, r, p, phat updates; r.r   */
  IPCS_KERNEL_PCG_UPDATE_M = 8,   /* correction CG: p, s, x, r, u updates            */
  IPCS_KERNEL_PCG_FUSED_P = 9,    /* Poisson CG, one kernel per iteration: update,
                                   * halo recomputation, w = Kp u; r.u, r.r, w.u    */
  IPCS_KERNEL_ASM_SUM = 10,       /* convection assembly, second pass (3D): the
                                   * cells' local rows added into the matrix rows   */
  IPCS_NKERNEL = 11
};
/* Measurement hook (not part of the method): from the next call on, every
 * launch of a kernel whose bit (1 << IPCS_KERNEL_*) is set in mask is
 * bracketed by two HIP events on the run's stream, in the normal sequence of
 * the step; mask = 0 turns this off. Accumulated times are reset. */
int ipcs_kernel_timing(ipcs_run r, uint32_t mask);
/* Accumulated event time (ms) and launch count per kernel since the last
 * ipcs_kernel_timing call; ms and launches hold cap >= IPCS_NKERNEL entries. */
int ipcs_kernel_times(ipcs_run r, double* ms, int64_t* launches, int32_t cap);
/* Measurement hook (not part of the method): launches one of the step's
 * kernels nlaunch times back to back on the run's stream with the run's own
 * data and returns the mean duration per launch in microseconds, timed with
 * HIP events on that stream. Leaves the run's Krylov scratch vectors
 * undefined (the next solve re-initializes them); the solver states
 * (tolerances) are restored and U, P and t are not touched, so the run steps on
 * as before. Call between steps only. */
int ipcs_profile_kernel(ipcs_run r, int32_t kernel, int32_t nlaunch, double* us_per_launch);

/* The pressure Poisson CG form the run uses for Kp dP = r (eq. (9), second
 * line; measurement and inspection). *rows_max receives the part size
 * of its row partition (0: two kernels per iteration, no partition), *nparts
 * the number of parts, *halo_rows the summed halo sizes (the rows a part reads
 * from other parts, once per part), *lds_rows the largest own + halo count of
 * a part. Any output pointer may be NULL. */
int ipcs_poisson_partition(ipcs_run r, int32_t* rows_max, int32_t* nparts, int64_t* halo_rows,
                           int32_t* lds_rows);

void ipcs_run_destroy(ipcs_run r);

/* ---------------------------------------------------------------- steady */
/* The steady Navier-Stokes equations of Section 2.1 (-nu Lap u + (u.grad)u +
 * grad p = f, div u = 0, u = g on the boundary) with the P2-P1 pair, solved
 * by Newton's method: the Newton linearization of Section 2.2.1 without its
 * time-derivative term, run as in Section 4.2 (steps until the relative
 * change falls below a tolerance, 1e-10 in at most 10 steps there). Each
 * step solves the monolithic saddle-point system for the increment,
 *   [[nu K + C(U) + N(U), G], [D, 0]] (dU, dP) = (F - (nu K + C(U)) U - G P, -D U),
 * N_ce = (phi_j d_e u_c, phi_i), boundary velocity rows and columns
 * eliminated (the iterates carry the Dirichlet data), by flexible GMRES with
 * the block upper-triangular preconditioner [[A, G], [0, -(1/nu) diag(Mp 1)]]:
 * A, the velocity block, applied by a loose inner Jacobi-BiCGStab solve. The
 * pressure is fixed by zero integral mean after each step. The start is the
 * Dirichlet data on the boundary and zero elsewhere, P = 0. All device work
 * runs in the caller's workspace on the given stream. */
typedef struct ipcs_steady_s* ipcs_steady;
typedef struct {
  double nu;            /* kinematic viscosity                                 */
  double tol;           /* Newton: stop when ||(dU,dP)||_2 <= tol ||(U,P)||_2  */
  int32_t maxit;        /* Newton steps                                        */
  int32_t restart;      /* FGMRES basis length (2..512)                        */
  double lin_tol;       /* FGMRES relative residual of each Newton system      */
  int32_t lin_maxit;    /* FGMRES iterations per Newton system                 */
  int32_t inner_maxit;  /* inner BiCGStab iterations per preconditioner use   */
  double inner_tol;     /* inner BiCGStab relative tolerance                   */
} ipcs_steady_params;
/* nu = 1, tol = 1e-10, maxit = 10 (Section 4.2), restart 60, lin_tol 1e-12,
 * lin_maxit 3000, inner_maxit 2000, inner_tol 1e-2. */
void ipcs_steady_params_default(ipcs_steady_params* p);
typedef struct {
  int32_t status;       /* IPCS_OK or the failure                              */
  int32_t newton_steps;
  int32_t lin_it;       /* FGMRES iterations, summed over the steps            */
  int32_t inner_it;     /* inner BiCGStab iterations, summed                   */
  double rel_change;    /* ||(dU,dP)|| / ||(U,P)|| of the last step            */
  double res0, res;     /* ||residual|| at the first and at the last step      */
  float ms;             /* device time of the steps (stream events)            */
  int32_t reserved;
} ipcs_steady_stats;
/* Device workspace of a steady solve on this mesh (P2-P1 pair; the blocks of
 * the Newton system above, its monolithic layout, the FGMRES basis and the
 * inner solver's vectors). IPCS_E_INVALID for another pair or bad
 * parameters. */
int ipcs_steady_workspace_bytes(ipcs_mesh m, const ipcs_steady_params* p, int64_t* bytes);
/* Sets up a steady solve (Section 4.2's workflow) in the caller's workspace
 * of ws_bytes bytes (IPCS_E_NOMEM if smaller than the size above; it stays
 * owned by the caller and must outlive the solver): uploads the mesh and
 * assembles nu K, D_c, G_c and the lumped pressure mass. */
int ipcs_steady_create(ipcs_mesh m, const ipcs_steady_params* p, void* dev_ws,
                       int64_t ws_bytes, void* hip_stream, ipcs_steady* out);
/* Closed-form data on the device (IPCS_SOL_STEADY_PAPER_2D,
 * IPCS_SOL_POLY_STEADY_2D, IPCS_SOL_POLY_STEADY_3D): f and g; resets the
 * iterate to the start above. */
int ipcs_steady_set_builtin(ipcs_steady s, int32_t kind, const double* prm, int32_t nprm);
/* Iterate given by the caller: u[dim*N2] (Dirichlet data on the boundary
 * nodes), p[N1], interface numbering. */
int ipcs_steady_set_state(ipcs_steady s, const double* u, const double* p);
/* One Newton step; stats (may be NULL) accumulate. */
int ipcs_steady_step(ipcs_steady s, ipcs_steady_stats* stats);
/* Newton steps until the relative change is <= tol (IPCS_E_NOT_CONVERGED
 * after maxit steps). */
int ipcs_steady_solve(ipcs_steady s, ipcs_steady_stats* stats);
/* The current iterate, the discrete solution of the steady equations of
 * Section 2.1 once converged: velocity [dim][N2] and pressure [N1] in the
 * interface numbering, into host memory of cap doubles (IPCS_E_INVALID if
 * smaller). */
int ipcs_steady_get_velocity(ipcs_steady s, double* u, int64_t cap);
int ipcs_steady_get_pressure(ipcs_steady s, double* p, int64_t cap);
/* The last step's residual (right-hand side) or increment,
 * [dim*N2 + N1] in the interface numbering. */
enum { IPCS_STEADY_RESIDUAL = 0, IPCS_STEADY_INCREMENT = 1 };
int ipcs_steady_get_vector(ipcs_steady s, int32_t which, double* out, int64_t cap);
void ipcs_steady_destroy(ipcs_steady s);

#ifdef __cplusplus
}
#endif
#endif /* IPCS_H */
