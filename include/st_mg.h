/*
 * st_mg.h -- C ABI of the MI355X (gfx950) space-time multigrid library.
 *
 * Method: Gander & Neumueller, "Analysis of a new space-time parallel
 * multigrid algorithm for parabolic problems" (arXiv 1411.0519).
 * Problem (Sec. 1, eq. chap4_modelproblem): du/dt - Laplace(u) = f on
 * (0,1)^d x (0,T), u = 0 on the boundary, u(.,0) = u0.  Discretisation:
 * Q1 finite elements on the uniform grid with n interior nodes per
 * dimension (h = 1/(n+1)), discontinuous Galerkin of order p_t in time on N
 * slabs (tau = T/N) with the shifted Legendre basis
 * psi_l(t) = P_l(2 (t - t_{n-1})/tau - 1).  The all-at-once system
 * L u = F (eq. chap4_generalLinearSystem) has diagonal blocks
 * A = K_tau (x) M_h + M_tau (x) K_h and sub-diagonal blocks -N_tau (x) M_h.
 *
 * Solver (Sec. 2, Sec. 4): V-cycles (gamma = 1; W-cycles with gamma = 2) with nu1/nu2 damped
 * block-Jacobi steps u <- u + omega D^{-1}(F - L u) (eq. chap4_smoother),
 * D = diag{A} inverted exactly (eq. chap4_smootherExact) by fast
 * diagonalisation; restriction R = P^T with P from eq.
 * chap4_restrictionTime (time) and eq. chap4_spaceRestrictionProlongation
 * (space); full space-time coarsening iff mu_L = tau_L/h_L^2 >= mu*
 * (Remark chap4_remarkCriticalDiscretizationParameter), otherwise time
 * semi-coarsening; coarsest level = one time slab, solved exactly.
 * Optionally (Remark V-cycleApproxSpace, eq. chap4_smootherApprox) the exact
 * block inverse is replaced by one geometric multigrid cycle in space per
 * slab (damped block Jacobi in space, full weighting, linear interpolation),
 * the setting of the paper's numerical examples (Sec. 4).
 *
 * Conventions for every entry point:
 *  - return value: ST_OK (0) or a negative ST_E* code; st_mg_last_error()
 *    gives a message.  A handle may be used by one host thread at a time.
 *  - vectors are DEVICE pointers, contiguous, laid out
 *    [batch][slab][time dof l][z][y][x] (x fastest), batch-major; element
 *    type double for ST_FP64 and ST_MIXED, float for ST_FP32.  The caller
 *    owns every vector; the library only borrows them for the call.
 *  - `stream` is a hipStream_t (NULL = default stream).  All device work is
 *    enqueued on it; entry points that return host values (norms, iteration
 *    counts) synchronise that stream before returning.
 *  - "level" indices count from the finest (0) to the coarsest (nlev-1).
 */
#ifndef ST_MG_H
#define ST_MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct st_mg* st_mg_t;

enum {
  ST_OK = 0,
  ST_EINVAL = -1,      /* invalid argument or parameter combination        */
  ST_ENOMEM = -2,      /* host or device allocation failed                 */
  ST_EHIP = -3,        /* a HIP runtime call failed                        */
  ST_ENOCONV = -4,     /* maxit reached before rtol (u holds last iterate)  */
  ST_ESTATE = -5,      /* call not valid in the handle's state             */
  ST_EWORKSPACE = -6,  /* no workspace bound, or bound workspace too small */
  ST_ENAN = -7         /* residual norm became NaN or Inf                  */
};

enum {
  ST_COARSEN_AUTO = 0, /* Sec. 4 rule: full iff mu_L >= mu* and n_L > 1, else semi */
  ST_COARSEN_SEMI = 1, /* time semi-coarsening only                             */
  ST_COARSEN_FULL = 2  /* full space-time coarsening while n_L > 1, then semi   */
};

enum {
  ST_FP64 = 0,  /* every level in double                                          */
  ST_FP32 = 1,  /* every level in float, norms accumulated in double             */
  ST_MIXED = 2, /* double outer iterative refinement: fine residual and update in
                   double, inner V-cycle in float, coarsest solve in double       */
  ST_MIXED_BF16 = 3 /* as ST_MIXED, with the inner cycle's sine transforms on the
                   bf16 matrix cores (FP32 accumulation and storage)              */
};

enum {
  ST_SMOOTH_EXACT = 0,      /* D^{-1}: exact slab solves by fast diagonalisation  */
  ST_SMOOTH_SPATIAL_MG = 1  /* (I - M^x) D^{-1}: one spatial multigrid cycle per
                               slab (eq. chap4_smootherApprox); the coarsest level
                               and one-node levels stay exact                      */
};

typedef struct {
  int dim;          /* d in {1,2,3}                                              */
  int n;            /* interior nodes per dimension, n = 2^m - 1, 1 <= n <= 255  */
  double T;         /* final time > 0                                            */
  int N;            /* number of time slabs, a power of two                      */
  int pt;           /* DG order p_t, 0 <= p_t <= 47 (p_t <= 3: tuned kernels with
                       compile-time N_t; higher orders: runtime-N_t kernels)    */
  double omega;     /* damping omega_t of the block-Jacobi smoother (0,1]        */
  int nu1, nu2;     /* pre-/post-smoothing steps, >= 0                           */
  int coarsen;      /* ST_COARSEN_*                                              */
  double mu_star;   /* <= 0: computed from R(-3 mu*) = sqrt(2) - 1               */
  int precision;    /* ST_FP64 | ST_FP32 | ST_MIXED | ST_MIXED_BF16             */
  int batch;        /* number of right-hand sides b >= 1                         */
  int smoother;     /* ST_SMOOTH_EXACT | ST_SMOOTH_SPATIAL_MG                    */
  int nu1x, nu2x;   /* spatial cycle: pre-/post block-Jacobi steps, 0..16        */
  double omega_x;   /* spatial cycle: Jacobi damping in (0, 1]                   */
  int gamma;        /* cycle index (Sec. 2): 1 = V-cycle, 2 = W-cycle            */
} st_mg_params;

/* Fill defaults: d=1, n=31, T=1, N=16, p_t=1, omega=1/2, nu1=nu2=2 (Sec. 4,
 * Example chap4_example1), AUTO coarsening, FP64, batch 1, exact smoother;
 * spatial cycle (when selected) nu1x=nu2x=2, omega_x=2/3 (Sec. 4); V-cycle. */
void st_mg_default_params(st_mg_params* p);

/* Validate parameters, build the level hierarchy (Sec. 4 rule) and upload the
 * per-level constants (DST matrices, per-mode inverse blocks).  Allocates
 * only the constant tables; no vector workspace.  *out owned by the caller
 * until st_mg_destroy. */
int st_mg_setup(const st_mg_params* p, st_mg_t* out);

/* ---- P1 simplicial meshes (Sec. 4, Examples chap4_example1 and chap4_example2) ----
 * Space is discretised with conforming P1 elements on a coarse triangle (d = 2)
 * or tetrahedron (d = 3) mesh refined `refinements` times by red refinement
 * (every edge halved; a tetrahedron's inner octahedron cut along its shortest
 * diagonal, ties broken by the lexicographically smallest endpoint
 * coordinates).  Nodes on boundary faces (faces of one cell) carry the
 * homogeneous Dirichlet condition; the unknowns are the interior nodes ordered
 * along the Z-order (Morton) curve of their coordinates (each coordinate scaled
 * to the coarse mesh's bounding box and quantised to 21 bits in 3-D, 31 bits in
 * 2-D; bits interleaved with x lowest; ties by node number, where old vertices
 * come first and edge midpoints follow in the order a sweep over the cells,
 * local edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), meets them).  Level
 * transfers: nested interpolation in space (an edge node takes the mean of its
 * edge's ends), eq. chap4_restrictionTime in time, R = P^T.  The mesh size in
 * mu = tau/h^2 is h_L = h0 2^-L on refinement level L. */
typedef struct {
  int dim;              /* 2: triangles, 3: tetrahedra                            */
  int nnodes;           /* vertices of the coarse mesh, >= dim + 1                */
  int ncells;           /* cells of the coarse mesh, >= 1                         */
  const double* coords; /* HOST, nnodes x dim, row-major                          */
  const int* cells;     /* HOST, ncells x (dim + 1) vertex indices, each cell of
                           positive volume                                        */
  double h0;            /* coarse mesh size for the coarsening rule; <= 0: its
                           longest edge                                           */
} st_mesh;

/* Host-only query (no GPU needed): refinement level `level` (0..refinements)
 * of `coarse`.  nx = interior nodes, nnz = stored entries of the interior
 * M_h / K_h (CSR, one shared pattern, columns ascending).  Each output array
 * may be NULL; otherwise points (nx x dim), rowptr (nx + 1), col (nnz),
 * mval / kval (nnz) are filled.  ST_EINVAL for an invalid mesh (index out of
 * range, degenerate cell, dim mismatch) or level < 0; ST_ENOMEM when the
 * refined mesh would exceed 2^31 - 1 nodes or entries. */
int st_mesh_level(const st_mesh* coarse, int level, long long* nx, long long* nnz, double* points,
                  int* rowptr, int* col, double* mval, double* kval);

/* st_mg_setup for the P1 mesh `coarse` refined `refinements` (0..10) times:
 * the paper's inexact smoother is required (p->smoother = ST_SMOOTH_SPATIAL_MG:
 * node-block Jacobi in space, nu1x/nu2x steps damped by omega_x, down to the
 * coarse mesh, where each slab is solved exactly); p->n is ignored; p->dim must
 * equal coarse->dim; 0 <= p_t <= 3; precision ST_FP64, ST_FP32 or ST_MIXED.  The exact
 * slab solves of the coarse mesh and of the coarsest level use dense inverses
 * built at setup: N_t x (interior nodes) <= 1024 on both, else ST_EINVAL (refine
 * less, or use more time slabs so that space is coarsened further).  In the
 * per-level queries n_L reports the refinement level.  Vectors use the layout
 * [batch][slab][time dof l][interior node]. */
int st_mg_setup_mesh(const st_mg_params* p, const st_mesh* coarse, int refinements, st_mg_t* out);

int st_mg_destroy(st_mg_t h);
const char* st_mg_last_error(st_mg_t h);

/* Bytes of device workspace the solver needs (coarse-level vectors, the
 * fine residual, one transform buffer and reduction partials). */
int st_mg_workspace_bytes(st_mg_t h, size_t* bytes);
/* Bind caller-owned device memory (256-byte aligned, >= workspace bytes);
 * dptr == NULL asks the library to allocate and own it (freed by destroy). */
int st_mg_bind_workspace(st_mg_t h, void* dptr, size_t bytes);

/* Hierarchy description: number of levels, schedule string of nlev-1
 * characters 'f' (full) / 's' (semi) from fine to coarse, NUL-terminated
 * (cap >= nlev).  Per level: n_L, N_L, tau_L, mu_L = tau_L/h_L^2. */
int st_mg_levels(st_mg_t h, int* nlev, char* schedule, int cap);
int st_mg_level_info(st_mg_t h, int level, int* n, int* N, double* tau, double* mu);
/* Fine-level sizes: vector length per right-hand side (N N_t n^d) and the
 * nodal lengths of f (N n^d) and u0 (n^d) per right-hand side. */
int st_mg_sizes(st_mg_t h, long long* dof, long long* f_len, long long* u0_len);
/* Spatial unknowns per time dof on a level: n_L^d on the grid, the interior
 * nodes of the level's refinement on a P1 mesh. */
int st_mg_level_nx(st_mg_t h, int level, long long* nx);

/* Right-hand side from nodal data (Sec. 1 load vector; u0 enters slab 1
 * through N_tau (x) M_h, eq. (equation1) with n = 0):
 *   F[b][n][l] = (int_slab psi_l dt) M_h f[b][n],  F[b][0][l] += psi_l(t_0^+) M_h u0[b].
 * f: [b][N][n^d], u0: [b][n^d] (NULL = 0), both in the handle's vector type
 * (double for ST_MIXED).  F: fine vector. */
int st_mg_rhs(st_mg_t h, const void* f, const void* u0, void* F, void* stream);
/* Transpose of st_mg_rhs (for gradients): grad_f[b][n] = sum_l (int psi_l) M_h lam[b][n][l],
 * grad_u0[b] = sum_l psi_l(t_0^+) M_h lam[b][0][l].  Either output may be NULL. */
int st_mg_rhs_adjoint(st_mg_t h, const void* lam, void* grad_f, void* grad_u0, void* stream);

/* ---- level operators (finest = level 0); vectors sized for that level ----
 * prec selects the arithmetic (ST_FP64: double vectors, ST_FP32: float);
 * transpose != 0 applies L^T instead of L (the adjoint problem L^T lam = g). */
/* r = F - L u  (eq. chap4_smoother's defect); norms2 (nullable, host, batch
 * doubles) receives ||r_b||_2^2 per right-hand side. */
int st_mg_residual(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                   void* r, double* norms2, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * residual and norms as st_mg_residual, with its per-workgroup partial sums
 * and per-RHS sums kept in a static device array of the library instead of
 * the workspace.  Needs no bound workspace and calls no allocating routine
 * (no profiling events are recorded for it).  Limits: at most 2^20 partial
 * sums (level-0 residual workgroups per slab x N x batch; e.g. 8 x 1024 for
 * 63^3 x 1024 slabs) and batch <= 256, else ST_EINVAL before any device work.
 * The array (8 MiB + 2 KiB per GPU) lives until the process ends and is
 * shared by every handle on that GPU: calls that overlap on one GPU (other
 * streams or host threads) race on it; calls on one stream are ordered.  Every
 * partial sum is written before it is read, so nothing is cleared between
 * calls.  norms2 (nullable, host) as in st_mg_residual, level 0 only. */
int st_mg_residual_noalloc(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                           void* r, double* norms2, void* stream);
/* x = D^{-1} r, D = diag{A}: exact slab solves by fast diagonalisation. */
int st_mg_block_solve(st_mg_t h, int level, int prec, int transpose, const void* r, void* x,
                      void* stream);
/* x = (I - M^x) A^{-1} r on every slab: one geometric multigrid cycle in
 * space from the zero initial guess (Remark V-cycleApproxSpace): nu1x damped
 * block-Jacobi steps x <- x + omega_x (D^x)^{-1}(r - A x), D^x the N_t x N_t
 * blocks of A at each spatial node; defect restriction by full weighting
 * (R_x (x) I); the same cycle on the re-discretised A_{tau,2h} down to one
 * node, solved exactly; linear interpolation (P_x (x) I); nu2x steps, with
 * the handle's nu1x, nu2x, omega_x.  Needs a handle set up with
 * ST_SMOOTH_SPATIAL_MG (its workspace holds the cycle's vectors; ST_ESTATE
 * otherwise).  x and r must not overlap.  Levels with n = 1 give x = A^{-1} r. */
int st_mg_spatial_cycle(st_mg_t h, int level, int prec, int transpose, const void* r, void* x,
                        void* stream);
/* One damped block-Jacobi step u <- u + omega D^{-1}(F - L u), with D^{-1}
 * exact or approximated by the spatial cycle, as the handle's smoother says. */
int st_mg_smooth(st_mg_t h, int level, int prec, int transpose, void* u, const void* F,
                 void* stream);
/* F_c = R r_f = P^T r_f from level to level+1. */
int st_mg_restrict(st_mg_t h, int level, int prec, const void* r_fine, void* F_coarse, void* stream);
/* F_c = P^T (F - L u) from level to level+1 (eq. chap4_generalLinearSystem
 * followed by eq. chap4_restrictionTime and, on fully coarsened levels, eq.
 * chap4_spaceRestrictionProlongation): the pre-restriction defect of the
 * cycle.  On fully coarsened levels of dimension 2 or 3 with p_t <= 3 (n =
 * 2 n_c + 1) the residual kernel restricts its own output, so the fine defect
 * is never stored (its per-slab restricted parts use the level's workspace
 * defect buffer); elsewhere the residual goes through that buffer and is
 * restricted in a second pass.  u, F on the level, F_coarse on level+1, same
 * layout as every level vector. */
int st_mg_residual_restrict(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                            void* F_coarse, void* stream);
/* u_f += P e_c from level+1 to level. */
int st_mg_prolong_add(st_mg_t h, int level, int prec, const void* e_coarse, void* u_fine,
                      void* stream);

/* ---- cycles and solves on the finest level ----
 * (V stands for the handle's cycle: gamma coarse-grid cycles per level.)
 * One V-cycle u <- MG(u, F) (ST_MIXED: one refinement step: FP64 residual,
 * FP32 V-cycle for the correction, FP64 update).  relres (nullable, host,
 * batch doubles) receives ||F - L u_new|| / ||F - L u_old|| per RHS. */
int st_mg_vcycle(st_mg_t h, void* u, const void* F, double* relres, void* stream);
/* Repeat V-cycles until ||F - L u_k||_2 <= rtol ||F - L u_0||_2 for every
 * RHS or maxit cycles.  u is the initial guess on entry.  *iters = cycles
 * done; hist (nullable, host) receives (maxit+1) x batch relative residuals
 * (row k = after k cycles).  Returns ST_ENOCONV if maxit is reached. */
int st_mg_solve(st_mg_t h, void* u, const void* F, double rtol, int maxit, int* iters,
                double* hist, void* stream);
/* Adjoint solve L^T lam = g (backward in time, transposed blocks, same
 * hierarchy and transfers), lam in/out (initial guess), then the gradients
 * of J(f, u0) with dJ/du = g: grad_f and grad_u0 as in st_mg_rhs_adjoint
 * (each nullable).  Same stopping rule and outputs as st_mg_solve. */
int st_mg_adjoint(st_mg_t h, const void* g, void* lam, void* grad_f, void* grad_u0, double rtol,
                  int maxit, int* iters, double* hist, void* stream);

/* Graph mode: 1 = record one V-cycle per (u, F, transpose) as a hipGraph on
 * first use and replay it; 0 = launch kernels directly (default).  Graph mode
 * needs a non-NULL stream. */
int st_mg_set_graph(st_mg_t h, int enable);

/* Autotuner: per level, time one smoothing step with every applicable kernel
 * family (one-kernel small-level step with the slab in LDS; LDS-staged
 * transforms; register-resident transforms, once folded; the default family,
 * which at n = 63 and 127 (FP32 also 255) is the twice-folded register
 * transform with half the matrix-core work; in 2-D with N_t <= 2 at FP64
 * n = 63 and FP32 n = 63, 127, the slab-resident block solve, one workgroup
 * per slab running all twice-folded passes from LDS; in 2-D with N_t = 2 at n = 63, 127, the residual fused
 * with the forward twice-folded x pass) and keep the fastest.
 * With the spatial-cycle smoother the transforms serve only the coarsest
 * level and nothing is tuned.
 * u_scratch, F_scratch: two fine-level device vectors of the handle's vector
 * type whose contents are overwritten (may be NULL for ST_MIXED).  Needs a
 * bound workspace; synchronises the stream. */
int st_mg_autotune(st_mg_t h, void* u_scratch, void* F_scratch, void* stream);
/* Choice for one level: small (1/0), transform family (0 default, 1 LDS, 2 register once folded, 3 twice folded,
 * 4 slab-resident, 5 twice folded with the residual fused into the forward x pass, 6 x-mode-major slab-resident
 * (3-D), 7 the same with the residual fused into its forward x pass), tuned step ms. */
int st_mg_level_tuning(st_mg_t h, int level, int* small, int* impl, float* ms);

/* Launch shape of the twice-folded sine passes on one level (the autotuner
 * picks it per level, i.e. per n, precision, batch and slab count, after the
 * kernel family): waves per workgroup of the line passes (1, 2 or 4); a cap
 * on their grid in workgroups per compute unit (0 = one 16-line group per
 * wave; with a cap the workgroups are persistent and each wave loops over a
 * contiguous range of groups); column groups of 16 per workgroup of the
 * fused pass along the slowest axis (a power of two <= 4 / N_t; 0 = the
 * largest); its grid cap (as above).  Results do not depend on the shape
 * (every line is transformed by the same arithmetic).  set: ST_EINVAL for
 * values outside these ranges; drops a recorded graph. */
int st_mg_level_shape(st_mg_t h, int level, int* wpg, int* pass_per_cu, int* fused_cg, int* fused_per_cu);
int st_mg_set_level_shape(st_mg_t h, int level, int wpg, int pass_per_cu, int fused_cg, int fused_per_cu);

/* Per-kernel timing with HIP events recorded around every launch on the
 * launch stream (eager mode only; ST_ESTATE in graph mode).  start clears
 * previous records; read synchronises on the last event and returns the
 * summed duration (ms) and launch count of one kernel kind on one level
 * (level -1 = all levels). */
enum {
  ST_PROF_RESIDUAL = 0,   /* r = F - L u                                          */
  ST_PROF_PASS_FWD = 1,   /* forward sine-transform pass along x                  */
  ST_PROF_PASS_INV = 2,   /* inverse pass along x (applies the update)            */
  ST_PROF_FUSED = 3,      /* forward + per-mode time solve + inverse, slowest axis */
  ST_PROF_SMALL = 4,      /* whole smoothing step of a small level, one kernel     */
  ST_PROF_RESTRICT = 5, ST_PROF_PROLONG = 6, ST_PROF_OTHER = 7,
  ST_PROF_JACOBI = 8,     /* spatial cycle: block-Jacobi steps and defects        */
  ST_PROF_XFER_X = 9,     /* spatial cycle: restriction / prolongation in space   */
  ST_PROF_RESID_X = 10,   /* residual fused with the forward x pass               */
  ST_PROF_PASS_FWD_Y = 11, /* forward pass along another axis before the last    */
  ST_PROF_PASS_INV_Y = 12, /* inverse pass along such an axis                     */
  ST_PROF_RESID_RESTRICT = 13, /* residual and full restriction in one pass       */
  ST_PROF_KINDS = 14
};
int st_mg_profile_start(st_mg_t h);
int st_mg_profile_stop(st_mg_t h);
int st_mg_profile_read(st_mg_t h, int kind, int level, double* total_ms, int* count);

#ifdef __cplusplus
}
#endif

#endif /* ST_MG_H */
