/*
 * sem.h -- C ABI of the MI355X spectral-element Poisson solver.
 *
 * Method: Remacle, Gandham, Warburton, "GPU accelerated spectral finite
 * elements on all-hex meshes".  The library solves the model problem of
 * Section 2, c u - div(kappa grad u) = s (eq. (pde)), with homogeneous
 * Dirichlet data on a chosen node set and optional Neumann data, discretised
 * with order-N Gauss-Lobatto-Legendre (GLL) spectral elements on unstructured
 * hexahedra, by preconditioned conjugate gradients (Algorithm 1) with the
 * two-scale additive Schwarz preconditioner of Section 4 (overlapping
 * fast-diagonalisation patch solves plus an order-1 coarse correction).
 * kappa and c are constants by default (kappa = 1, c = 0: the Poisson
 * problem), or one value per element, or one value per local node.  Also: an
 * FP32-refined solve, batched solves of many meshes, backward Euler steps of
 * the heat equation of Section 6.2 and an aggregation-AMG coarse solver.
 *
 * Conventions shared by every entry point
 *   - Mesh input is host memory and is copied; the handle owns every buffer it
 *     allocates (host and device) until sem_mesh_destroy.
 *   - Vectors passed to the hot-path calls (sem_apply_A, sem_precond,
 *     sem_pcg_solve) are caller-owned DEVICE pointers of length n_global, in
 *     the global node numbering described at sem_mesh_numbering.  Work is
 *     enqueued on the caller's stream (a hipStream_t passed as void*, NULL =
 *     the null stream).  sem_apply_A and sem_precond return once enqueued;
 *     sem_pcg_solve synchronises its stream to return statistics.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Every function returns SEM_OK (0) or a negative status; no exception
 *     crosses the ABI.  sem_last_error() gives a thread-local message.
 *   - Supported orders: 2 <= N <= 15 (at N = 1 the extended 1D pencil of
 *     Section 4.2 has no Dirichlet point and is singular).
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_mesh_s* sem_mesh;

enum sem_status {
  SEM_OK = 0,
  SEM_EINVAL = -1,          /* bad argument (NULL pointer, size, vertex id out of range) */
  SEM_ENOMEM = -2,          /* host or device allocation failed */
  SEM_EMESH = -3,           /* invalid mesh: |J| <= 0 at a GLL node, face shared by > 2 hexes */
  SEM_ENOCONV = -4,         /* max_iter / max_outer reached; statistics are filled */
  SEM_EBREAKDOWN = -5,      /* p^T A p <= 0 or a non-finite scalar in PCG */
  SEM_EHIP = -6,            /* a HIP / runtime library call failed */
  SEM_EUNSUPPORTED = -7     /* order outside 2..15, or a call that needs a device on a host-only handle */
};

enum sem_dtype { SEM_F64 = 0, SEM_F32 = 1 };

/* parts of the two-scale preconditioner P = P^c + P^f (Section 4) */
enum sem_pc { SEM_PC_NONE = 0, SEM_PC_FINE = 1, SEM_PC_COARSE = 2, SEM_PC_TWOSCALE = 3 };

enum sem_solve_mode { SEM_SOLVE_FP64 = 0, SEM_SOLVE_FP32_REFINED = 1 };

typedef struct {
  int device;        /* HIP device ordinal (default 0) */
  int host_only;     /* 1: build the host tables only (numbering, geometry, patches) and
                        allocate nothing on a device; hot-path calls return SEM_EUNSUPPORTED */
  int build_fp32;    /* 1: also keep FP32 copies for SEM_F32 calls and the refined solve (default 1) */
  int autotune;      /* 1: time the operator kernel's tile candidates (elements per workgroup) on this
                        mesh at set-up and keep the fastest per dtype (default 1) */
  const char* tune_cache; /* optional text file of tuned tiles, read before and appended after tuning
                        (NULL: no file) */
} sem_setup_opts;

typedef struct {
  int mode;          /* sem_solve_mode */
  int pc;            /* sem_pc */
  double rtol;       /* stop when ||b - A x||_2 <= rtol ||b||_2; FP64 checks the recursive residual
                        each iteration, then confirms with the true residual and restarts from it
                        while it is above the tolerance */
  int max_iter;      /* FP64: iteration cap; refined: cap on inner iterations per outer step */
  int use_x0;        /* 1: start from the x passed in, else x = 0 */
  double inner_rtol; /* refined form: relative tolerance of each FP32 inner solve */
  int max_outer;     /* refined form: cap on outer (FP64 residual) steps */
  int check_every;   /* read the convergence scalar back every k iterations (>= 1) */
} sem_solve_opts;

typedef struct {
  int iterations;        /* total PCG iterations (inner iterations summed for the refined form) */
  int outer_iterations;  /* refined form: number of FP64 residual corrections; FP64: restarts
                            from the true residual */
  double rel_residual;   /* final ||r||_2 / ||b||_2 (the true FP64 residual when converged) */
  double solve_ms;       /* wall time of the solve on the host clock */
  double* history;       /* optional caller buffer for ||r_k|| / ||b|| (may be NULL) */
  int history_cap;
  int history_len;
} sem_solve_stats;

/* Default option values. */
void sem_default_setup_opts(sem_setup_opts* o);
void sem_default_solve_opts(sem_solve_opts* o);

/*
 * sem_mesh_setup -- build every table of the discretisation for one mesh.
 *   vtx   [n_vtx][3] vertex coordinates (host, row-major).
 *   hex   [n_hex][8] vertex ids per hexahedron in tensor order: local corner
 *         (a,b,c) in {0,1}^3 is entry a + 2b + 4c.  Any of the 24 proper
 *         orientations is accepted.
 *   order N of the GLL basis (Section 2.1), 2..15.
 * Builds: the canonical global numbering and gather tables (Section 2.2),
 * the geometric factors and lumped mass (Sections 2.3-2.4), the overlapping
 * patch table and 1D fast-diagonalisation basis (Section 4.2), and the
 * factorised order-1 coarse matrix (Section 4.1).  The default Dirichlet set
 * is the topological boundary (nodes on faces owned by one hexahedron).
 * Errors: SEM_EINVAL, SEM_EUNSUPPORTED (order), SEM_EMESH (|J| <= 0 at a GLL
 * node, a face shared by more than two hexahedra), SEM_ENOMEM, SEM_EHIP.
 */
int sem_mesh_setup(const double* vtx, int64_t n_vtx, const int64_t* hex, int64_t n_hex,
                   int order, const sem_setup_opts* opts, sem_mesh* out);

int sem_mesh_destroy(sem_mesh m);

/* n_global = number of global GLL nodes, n_local = n_hex (N+1)^3,
   n_vertices = number of mesh vertices referenced by the hexahedra. */
int sem_mesh_sizes(sem_mesh m, int64_t* n_global, int64_t* n_local, int64_t* n_vertices);

/*
 * sem_mesh_numbering -- the local-to-global table I_{l->g} of Section 2.2 (host out).
 *   l2g [n_hex][(N+1)^3], local node (i,j,k) at i + (N+1) j + (N+1)^2 k.
 * Canonical rule (the paper only asks for uniqueness): referenced vertices in
 * ascending vertex id; then edges (sorted vertex pairs, lexicographic), N-1 ids
 * each counted from the smaller vertex id; then faces (sorted 4-tuples,
 * lexicographic), (N-1)^2 ids each in the frame whose origin is the face's
 * smallest vertex id, p towards the smaller id of its two face-adjacent
 * corners, id offset (q-1)(N-1) + (p-1); then element interiors, (N-1)^3
 * per element, i fastest.
 */
int sem_mesh_numbering(sem_mesh m, int32_t* l2g_host);

/* Gather table I_{g->l} of eq. (gather) as CSR (host out): offsets [n_global+1],
   idx [n_local] = local indices, ascending within each global node. */
int sem_mesh_gs_csr(sem_mesh m, int64_t* offsets_host, int32_t* idx_host);

/* Overlapping patch table I^p of Section 4.2 (host out): [n_hex][(N+3)^3], patch
   node (i,j,k), -1 <= i,j,k <= N+1, at (i+1) + (N+3)(j+1) + (N+3)^2 (k+1);
   -1 marks a node outside the mesh (its residual is 0, its correction dropped). */
int sem_mesh_patch_table(sem_mesh m, int32_t* ip_host);

int sem_mesh_node_coords(sem_mesh m, double* xyz_host);   /* [n_global][3] */
int sem_mesh_lumped_mass(sem_mesh m, double* mass_host);  /* [n_global], m_N of Section 4.1 */
int sem_mesh_boundary_mask(sem_mesh m, uint8_t* mask_host); /* [n_global], 1 = Dirichlet */

/* Geometric factors (host out): G [n_hex][6][(N+1)^3] = entries (xx,xy,xz,yy,yz,zz) of
   rho_i rho_j rho_k |J| (J^T J)^{-1}, mass [n_hex][(N+1)^3] = rho_i rho_j rho_k |J|. */
int sem_mesh_geometry(sem_mesh m, double* G_host, double* mass_host);

/* Replace the Dirichlet set (host in, [n_global], 1 = Dirichlet).  Re-derives the
   coarse vertex set and refactors the coarse matrix.
   The Dirichlet set is state of the handle, not an argument of each hot-path
   call: the coarse space of Section 4.1 depends on it (its free vertices, the
   nested dissection of their graph and the factor of the coarse matrix), so a
   new set costs a new dissection and factorisation of the coarse matrix on the
   host and device, synchronously (the set-up's coarse part: tens of
   milliseconds on small meshes, seconds at tens of millions of nodes), while a
   fixed set costs nothing per call (the element kernels read it only for
   elements that touch it).  Calls enqueued before this one complete first. */
int sem_mesh_set_dirichlet(sem_mesh m, const uint8_t* mask_host);

/*
 * sem_apply_A -- y = mask(Q^T A_L Q u): the matrix-free stiffness action of
 * eq. (R) / Algorithm 2 followed by the gather of eq. (gather) and the zeroing
 * of Dirichlet nodes.  u, y: device vectors [n_global] of dtype (SEM_F64 /
 * SEM_F32); the input is used as given (not masked).  u and y must not alias.
 */
int sem_apply_A(sem_mesh m, const void* u_dev, void* y_dev, int dtype, void* stream);

/*
 * sem_precond -- z = mask(P^f r + P^c r), the two-scale preconditioner of
 * Section 4: pc selects the parts (sem_pc).  P^f: patch gather through I^p,
 * the fast-diagonalisation solve of eq. (z), additive scatter.  P^c: eq.
 * (coarse) with the exact inverse of the coarse matrix, always in FP64.
 * r, z: device vectors [n_global] of dtype; must not alias.
 */
int sem_precond(sem_mesh m, const void* r_dev, void* z_dev, int dtype, int pc, void* stream);

/* Coarse solve only: Z = A_c^{-1} R on the free vertices (device FP64 vectors
   [n_vertices] indexed by vertex global id; Dirichlet vertices give 0). */
int sem_coarse_solve(sem_mesh m, const double* R_dev, double* Z_dev, void* stream);

/*
 * sem_pcg_solve -- Algorithm 1 for A x = b (b, x device FP64 [n_global]).
 * SEM_SOLVE_FP64: every step in FP64.  SEM_SOLVE_FP32_REFINED: outer FP64
 * iterative refinement (true residual b - A x in FP64) around inner PCG solves
 * whose operator, gather and patch solves run in FP32, with FP64 dot products,
 * scalars and coarse solve.  Returns SEM_OK, SEM_ENOCONV (stats filled),
 * SEM_EBREAKDOWN, or an error.  Only the values of b on free nodes take part
 * (b is read as 0 on the Dirichlet set); ||b|| in the stopping rule is the norm
 * of those values.  b = 0 gives x = 0 and 0 iterations; with use_x0, a start
 * whose residual already meets the tolerance returns after 0 iterations.
 * After SEM_EBREAKDOWN x holds the last iterate with finite scalars.
 * Work vectors (5 of n_global FP64, and 5 FP32 for the refined form) are
 * allocated by the first solve that needs them and kept by the handle.
 */
int sem_pcg_solve(sem_mesh m, const double* b_dev, double* x_dev, const sem_solve_opts* o,
                  sem_solve_stats* st, void* stream);

/*
 * sem_pcg_solve_noalloc -- sem_pcg_solve for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, hosts that
 * forbid allocation after start-up).  Same arguments, results and statuses as
 * sem_pcg_solve; the work vectors, partial sums and scalars of the solve live
 * in one static device array of the library (128 MiB per device, held until
 * the process ends) instead of the handle's lazily allocated buffers, and the
 * call allocates nothing.  Needed: 40 bytes per global node (FP64), 60 with
 * SEM_SOLVE_FP32_REFINED, plus about 8 bytes per element (about 3.3 M and 2.2 M global nodes at
 * most); a larger mesh gives SEM_EINVAL and a message naming both sizes,
 * before any device work.  Everything the solve reads is built at set-up (the
 * coarse-solve graph, the side stream); if a later call on the handle dropped
 * one of them, the call fails with SEM_EINVAL instead of rebuilding it.  All
 * calls on one device share the array: calls that overlap in time on one
 * device (two host threads, or two streams) race and give wrong results.  Each
 * solve initialises the parts it reads; contents are not kept between calls.
 */
int sem_pcg_solve_noalloc(sem_mesh m, const double* b_dev, double* x_dev, const sem_solve_opts* o,
                          sem_solve_stats* st, void* stream);

/*
 * sem_mesh_set_coefficients -- constant kappa > 0 and c >= 0 of the model
 * problem c u - div(kappa grad u) = s (eq. (pde)).  Afterwards sem_apply_A
 * computes kappa times the stiffness action plus c m_N u (the GLL mass is
 * diagonal, Section 2.4), the patch solves use 1/(4 kappa (lambda_a/h_x^2 +
 * lambda_b/h_y^2 + lambda_c/h_z^2) + c) (eq. (z)), and the coarse matrix is
 * the order-1 operator with the same kappa and c (reassembled and
 * refactorised here; synchronises the device).  Defaults: kappa = 1, c = 0.
 * Errors: SEM_EINVAL (non-finite, kappa <= 0 or c < 0), SEM_ENOMEM, SEM_EHIP.
 */
int sem_mesh_set_coefficients(sem_mesh m, double kappa, double c);
/* Current constant (kappa, c) (host out); NaN while per-element or per-node values are in use. */
int sem_mesh_coefficients(sem_mesh m, double* kappa, double* c);

/*
 * sem_mesh_set_element_coefficients -- one kappa_e > 0 and c_e >= 0 per
 * element (host arrays [n_hex] in input element order; NULL: all 1, resp.
 * all 0), as in Algorithm 2: each element's local values become
 * kappa_e r_{ijk;e} + c_e m_{ijk;e} u_{ijk;e} before the gather; patch
 * solve s uses its own element's kappa_e, c_e in eq. (z); the coarse matrix
 * is assembled with them and refactorised (synchronises the device; uploads
 * the local mass m_{ijk;e}, [n_hex][(N+1)^3], when some c_e != 0).
 * sem_mesh_set_coefficients returns the handle to constant coefficients.
 * Errors: SEM_EINVAL (a value non-finite, kappa_e <= 0 or c_e < 0; nothing
 * is changed), SEM_ENOMEM, SEM_EHIP.
 */
int sem_mesh_set_element_coefficients(sem_mesh m, const double* kappa_host, const double* c_host);

/*
 * sem_mesh_set_node_coefficients -- kappa > 0 and c >= 0 at every local node
 * (host arrays [n_hex][(N+1)^3] in input element order, local index
 * i + (N+1) j + (N+1)^2 k; NULL: all 1, resp. all 0), as in eq. (R), where
 * each quadrature point carries its own kappa: the six factors G at node
 * (i,j,k) of element e are multiplied by kappa_{ijk;e} before the derivative
 * transposes, and c_{ijk;e} m_{ijk;e} u_{ijk;e} is added before the gather.
 * The device factors are replaced by the scaled ones (the host copy, and
 * sem_mesh_geometry, keep the plain G), and the operator kernel that rebuilds
 * G from the vertices reads kappa per local node (an [n_hex][(N+1)^3] copy on
 * the device, FP64 and FP32).  The patch solves and
 * the coarse matrix take one value per element: the mean over the reference
 * cube by the GLL rule, (1/8) sum rho_i rho_j rho_k v_{ijk;e} (refactorised
 * here; synchronises the device).  sem_mesh_set_coefficients and
 * sem_mesh_set_element_coefficients restore the plain factors.
 * Errors: SEM_EINVAL (a value non-finite, kappa <= 0 or c < 0; nothing is
 * changed), SEM_ENOMEM, SEM_EHIP.
 */
int sem_mesh_set_node_coefficients(sem_mesh m, const double* kappa_host, const double* c_host);

/*
 * sem_mesh_boundary_face_mass -- the Neumann term of eq. (pdeweak): for
 * du/dn = g on the boundary faces listed, the right-hand side gains
 * kappa g_N ws_N at each node, where (GLL rule on each face)
 *   ws_N = sum over the listed faces holding N of rho_p rho_q |dx/da x dx/db|
 * (a, b the face's two reference axes in increasing order).  faces_host:
 * [n_faces][2] pairs (element in input order, local face 2 axis + side:
 * xi-, xi+, eta-, eta+, zeta-, zeta+).  ws_host: [n_global] out (host),
 * overwritten.  Nodes of Neumann faces must be left out of the Dirichlet set
 * (sem_mesh_set_dirichlet).  Errors: SEM_EINVAL (NULL, an element or face
 * index out of range, a face that is not on the boundary).
 */
int sem_mesh_boundary_face_mass(sem_mesh m, const int64_t* faces_host, int64_t n_faces, double* ws_host);

/*
 * sem_mesh_set_coarse_solver -- P_0 of eq. (coarse).  SEM_COARSE_EXACT
 * (default): the exact inverse of the order-1 matrix (nested dissection,
 * FP64).  SEM_COARSE_AMG: one K-cycle of an aggregation-based algebraic
 * multigrid on it (Section 4.1, "Algebraic multigrid"): double pairwise
 * aggregation of the strong negative couplings (threshold 0.25), Galerkin
 * coarse matrices, damped Jacobi (omega = 2/3, one sweep before and one
 * after), two flexible-CG steps per level, the coarsest level (<= 400
 * unknowns) solved exactly; built on the host, applied on the device as one
 * captured graph, rebuilt whenever the coarse matrix changes.  P_0 is then
 * nonlinear and the PCG iterates differ from the exact case; the solution to
 * a given tolerance is the same.  Synchronises the device.
 * Errors: SEM_EINVAL (unknown solver), SEM_ENOMEM, SEM_EHIP, SEM_EMESH.
 */
enum sem_coarse_solver { SEM_COARSE_EXACT = 0, SEM_COARSE_AMG = 1 };
int sem_mesh_set_coarse_solver(sem_mesh m, int solver);

/* The AMG hierarchy the handle would build (host only, for checks): number
   of levels, the first `cap` level sizes (level 0 = free vertices), and, when
   agg0 != NULL and there are two levels or more, the aggregate of each level-0
   unknown ([level_sizes[0]], unknowns in ascending vertex id). */
int sem_mesh_amg_hierarchy(sem_mesh m, int64_t* level_sizes_host, int cap, int* n_levels, int32_t* agg0_host);

/*
 * sem_heat_step -- one backward Euler step of the heat equation (Section 6.2):
 * solves (kappa A + M / dt) u_next = M (u_prev / dt + q) with u = 0 on the
 * Dirichlet set, where M is the lumped mass m_N.  Sets the coefficients to
 * (kappa, 1/dt) first (the coarse matrix is refactorised only when they
 * change), forms the right-hand side on the device, copies u_prev to u_next
 * and runs sem_pcg_solve from it (o->use_x0 is forced to 1).
 *   u_prev [n_global] device FP64, the solution at the previous time;
 *   q      [n_global] device FP64 nodal source at the new time, or NULL (none);
 *   u_next [n_global] device FP64, out (may be u_prev; must not be q).
 * Returns what sem_pcg_solve returns; SEM_EINVAL for dt <= 0, kappa <= 0 or
 * NULL vectors.  Uses an internal right-hand-side buffer of the mesh handle:
 * calls on one handle must not overlap.
 */
int sem_heat_step(sem_mesh m, double kappa, double dt, const double* u_prev_dev, const double* q_dev,
                  double* u_next_dev, const sem_solve_opts* o, sem_solve_stats* st, void* stream);

/*
 * Batched solves: many independent meshes (of any orders in 2..15) solved
 * together.  Instances of one order share every kernel launch (their meshes
 * are concatenated into one disjoint union), scalars of Algorithm 1 are kept
 * per instance, and one PCG iteration of the whole batch is captured once in a
 * hipGraph and replayed.  Each instance uses its default Dirichlet set and
 * starts from x = 0; results match per-instance sem_pcg_solve calls.
 */
typedef struct sem_batch_s* sem_batch;

/* n instances; vtx[i] ([n_vtx[i]][3]) and hex[i] ([n_hex[i]][8]) are host arrays
   as for sem_mesh_setup, order[i] in 2..15.  Same errors as sem_mesh_setup. */
int sem_batch_setup(int n, const double* const* vtx, const int64_t* n_vtx, const int64_t* const* hex,
                    const int64_t* n_hex, const int* order, const sem_setup_opts* opts, sem_batch* out);

/* n_global[i] of every instance (host out, [n]). */
int sem_batch_sizes(sem_batch b, int64_t* n_global);

/* Solve A_i x_i = b_i for all instances.  b_dev, x_dev: host arrays of n device
   pointers (FP64, [n_global[i]] each, in each instance's own numbering; b is
   read as 0 on each instance's Dirichlet set).  As in sem_pcg_solve, the FP64
   form confirms each instance with its true residual b - A x and continues
   from it the instances still above their tolerance (outer_iterations counts
   these restarts).  st: optional array of n statistics.  Returns SEM_OK when
   every instance converged, SEM_ENOCONV or SEM_EBREAKDOWN otherwise
   (statistics filled). */
int sem_batch_solve(sem_batch b, const double* const* b_dev, double* const* x_dev, const sem_solve_opts* o,
                    sem_solve_stats* st, void* stream);

int sem_batch_destroy(sem_batch b);

/*
 * sem_time_apply_A -- run `reps` applications of sem_apply_A back to back on
 * `stream` with HIP events recorded around each of its two kernels (element
 * kernel, shared-node gather), synchronise, and return the mean duration of
 * each kernel in milliseconds.  Same arguments and errors as sem_apply_A;
 * reps >= 1.  For measurement and tuning.
 */
int sem_time_apply_A(sem_mesh m, const void* u_dev, void* y_dev, int dtype, int reps, void* stream,
                     double* ms_element, double* ms_gather);

/*
 * sem_stream_bench -- the device's achievable memory bandwidth with the
 * library's own streaming kernels, the ceiling against which the solver's
 * bandwidth-bound kernels are read (the paper's Section 6.1 reads its kernels
 * against the device bandwidth the same way).  a, b, c: caller-owned device
 * FP64 arrays of n entries each (n even, 16-byte aligned, no overlap); b and
 * c are overwritten.  Runs b = a (copy, 16 n bytes), c = a + 0.5 b (triad,
 * 24 n bytes) and a read-only sum of a (8 n bytes) on `stream`, reps timed
 * launches each for several grid sizes, synchronises, and returns the best
 * rate of each in gbs[0..2] (GB/s, 1e9 bytes).  SEM_EINVAL on bad arguments.
 */
int sem_stream_bench(const double* a_dev, double* b_dev, double* c_dev, int64_t n, int reps, void* stream,
                     double* gbs);

/* Tile of the operator kernel for dtype: elements per workgroup (1, 2, 4, 8;
   (N+1)^2 lanes each, at most 1024 lanes), 16 for the matrix-core kernel
   (N = 15 only, FP64 or FP32), or 32 for the kernel that rebuilds the geometric
   factors at every node from the element's 8 vertices instead of reading them
   (the r' kernel of Section 5.1 and Table 3; same factors up to rounding).  Chosen by the autotuner or the
   default for the order; sem_mesh_set_tile overrides it (SEM_EINVAL if not
   available). */
int sem_mesh_tile(sem_mesh m, int dtype, int* epb);
int sem_mesh_set_tile(sem_mesh m, int dtype, int epb);

/* Entries of the coarse factor that one exact coarse solve of Section 4.1
   reads: *fwd_entries of the stacked blocks [S^-1; W] of the nested-
   dissection fronts (forward sweep), *bwd_entries of the blocks W^T (backward
   sweep), FP64 each; both 0 before the first factorisation.  For byte counts
   (roofline of an iteration); SEM_EINVAL on a NULL argument. */
int sem_mesh_coarse_factor_size(sem_mesh m, int64_t* fwd_entries, int64_t* bwd_entries);

const char* sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
