// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stmg {

constexpr int NT_MAX = 4;          // compile-time time dofs of the tuned kernels (p_t <= 3)
constexpr int NT_BIG = 48;         // runtime time dofs of the high-order kernels (p_t <= 47)
constexpr int TILE_COLS = 64;      // columns per workgroup of the transform kernel

// Residual r = F - L u (or F - L^T u) on one level.  Time coefficients are
// already arranged for the direction: forward uses K_tau, N_tau = ca cb^T and
// the previous slab (dir = -1); the adjoint uses K_tau^T, N_tau^T = cb ca^T and
// the next slab (dir = +1).  M_tau is symmetric.
template <typename T>
struct ResidArgs {
  T K[NT_MAX * NT_MAX];   // K[l*NT + k]
  T M[NT_MAX * NT_MAX];
  T ca[NT_MAX];           // row factor of the coupling block
  T cb[NT_MAX];           // column factor (combination of the neighbour slab)
  T wm[3];                // 1-D mass stencil  h/6 * (1, 4, 1)
  T wk[3];                // 1-D stiffness stencil  1/h * (-1, 2, -1)
  int n;                  // interior nodes per dimension
  long long nx;           // n^d
  int N;                  // slabs
  int batch;
  int dir;                // -1 forward, +1 adjoint
};

// Restriction / prolongation between a fine level (Nf = 2 Nc slabs) and a coarse level.
template <typename T>
struct TransferArgs {
  T R1T[NT_MAX * NT_MAX];  // R1^T[l*NT + k]: fine slab 2m   <- coarse slab m
  T R2T[NT_MAX * NT_MAX];  // R2^T[l*NT + k]: fine slab 2m+1 <- coarse slab m
  int nf, nc;              // interior nodes per dimension (nc == nf for semi)
  long long nxf, nxc;
  int Nc;                  // coarse slabs
  int batch;
};

// Load vector from nodal data.
template <typename T>
struct RhsArgs {
  T ints[NT_MAX];   // int_slab psi_l dt
  T ca[NT_MAX];     // psi_l(t_0^+)
  T wm[3];
  int n;
  long long nx;
  int N;
  int batch;
};

enum { MODE_STORE = 0, MODE_ADD_SCALED = 1, MODE_SET_SCALED = 2 };

// ---- launchers (defined in stmg_kernels.hip) ----
template <typename Tin, typename Tout>
hipError_t launch_residual(int dim, int nt, const Tin* u, const Tin* F, Tout* r,
                           const ResidArgs<Tin>& a, double* partial, hipStream_t s);
// Rows per 2-D tile of the residual and spatial smoothing kernels (0: n too
// wide for one set of prefetched loads).
int residual_tile_rows(int nt, int n);
unsigned residual_blocks_per_slab(int dim, int n, long long nx, int nt, long long slabs);

// Folded DST-I transforms (stmg_transform.hip).  hb = transform_half_blocks(n);
// Sfrag = [dir fwd/inv][half odd/even][kb < hb][ib < 4 hb][64 lanes] fragments.
int transform_half_blocks(int n);
// Transform implementation: automatic choice, LDS-staged kernels only, or the
// FP64 register-resident kernels wherever their state fits.
enum { TRANSFORM_AUTO = 0, TRANSFORM_LDS = 1, TRANSFORM_REG = 2, TRANSFORM_REG2 = 3, TRANSFORM_SLAB = 4,
       TRANSFORM_XSLAB = 6 };
template <typename T>
hipError_t launch_dst_pass(int impl, int hb, bool xaxis, bool inverse, const T* in, T* out, const T* Sfrag,
                           int n, long long inner, long long ncols, T omega, int mode,
                           hipStream_t s);
template <typename T>
hipError_t launch_dst_fused(int impl, int hb, int nt, const T* in, T* out, const T* Sfrag, const T* G, int n,
                            long long inner, long long outer, int transpose, T omega, int mode,
                            hipStream_t s);
// BF16 matrix-core transforms on FP32 data (stmg_bf16.hip); F is the level's
// bf16 fragment table [dir][half][kb][c][lane][4], hb <= 8.
hipError_t launch_pass_bf16(int hb, bool inverse, const float* in, float* out, const void* F, int n, long long inner,
                            long long ncols, float omega, int mode, hipStream_t s);
hipError_t launch_fused_bf16(int hb, int nt, const float* in, float* out, const void* F, const float* G, int n,
                             long long inner, long long outer, int transpose, float omega, int mode, hipStream_t s);
template <typename T>
hipError_t launch_restrict(int dim, int nt, bool full, const T* rf, T* Fc, const TransferArgs<T>& a,
                           hipStream_t s);
template <typename T>
hipError_t launch_prolong(int dim, int nt, bool full, const T* ec, T* uf, const TransferArgs<T>& a,
                          hipStream_t s);
// Pre-restriction defect of a fully coarsened level (n = 2 n_c + 1) of
// dimension 2 or 3, N_t <= 4, without storing it: F_c = P^T (F - L u) through
// per-slab restricted parts in Hs (N slabs x N_t x n_c^d values), then their
// pair sums.  resid_restrict_shape is false where it does not apply.
struct ResRestrictShape {
  int tyc, zcc, nyt, nzt, bs, oit, sit;
  size_t lds;
};
bool resid_restrict_shape(int dim, int nt, int n, int nc, long long slabs, int tbytes, ResRestrictShape& sh);
template <typename T>
hipError_t launch_resid_restrict(int dim, int nt, const T* u, const T* F, T* Fc, T* Hs, const ResidArgs<T>& a,
                                 const TransferArgs<T>& t, hipStream_t s);
template <typename T>
hipError_t launch_rhs(int dim, int nt, const T* f, const T* u0, T* F, const RhsArgs<T>& a,
                      hipStream_t s);
template <typename T>
hipError_t launch_rhs_adjoint(int dim, int nt, const T* lam, T* gf, T* gu0, const RhsArgs<T>& a,
                              hipStream_t s);
template <typename T>
hipError_t launch_sumsq(const T* v, long long len, int batch, double* partial, unsigned gx,
                        hipStream_t s);
hipError_t launch_norm_final(const double* partial, long long per_batch, int batch, double* out,
                             hipStream_t s);
template <typename T>
hipError_t launch_fill(T* v, long long len, hipStream_t s);
// Idle one wave for about `microseconds` (capped at 5 ms) so that the launches
// queued behind it run without host-side gaps; used to time short sequences.
hipError_t launch_spin(double microseconds, hipStream_t s);
hipError_t launch_axpy_f32_f64(double* u, const float* e, long long len, hipStream_t s);
hipError_t launch_cast_f64_f32(const double* in, float* out, long long len, hipStream_t s);
hipError_t launch_cast_f32_f64(const float* in, double* out, long long len, hipStream_t s);

// ------------------------------------------------- spatial multigrid cycle
// Kernels of the inexact smoother (one geometric multigrid cycle in space per
// slab, no coupling between slabs).  The slab matrix A = K (x) M_h + M (x) K_h
// with K = K_tau (or K_tau^T for the adjoint) and M = M_tau; Dinv is the
// inverse N_t x N_t block of A at one spatial node (its transpose for the
// adjoint), which on a one-node level is A^{-1} itself.
enum { SP_JACOBI = 0, SP_DEFECT = 1 };
enum { UPD_NONE = 0, UPD_ADD = 1, UPD_SET = 2 };
template <typename T>
struct SpatialArgs {
  T K[NT_MAX * NT_MAX];
  T M[NT_MAX * NT_MAX];
  T Dinv[NT_MAX * NT_MAX];
  T wm[3];                // 1-D mass stencil  h/6 * (1, 4, 1)
  T wk[3];                // 1-D stiffness stencil  1/h * (-1, 2, -1)
  int n;                  // interior nodes per dimension
  long long nx;           // n^d
  long long slabs;        // batch * N
  T omega;                // Jacobi damping omega_x
  T scale;                // weight of the result in the output (UPD_ADD / UPD_SET)
  int op;                 // SP_JACOBI: y = x + omega Dinv (f - A x);  SP_DEFECT: y = f - A x
  int upd;                // UPD_NONE: out = y;  UPD_ADD: out = base + scale y;  UPD_SET: out = scale y
  int x_zero;             // x is treated as zero (x may be null)
};
template <typename T>
hipError_t launch_spatial(int dim, int nt, const T* x, const T* f, const T* base, T* out,
                          const SpatialArgs<T>& a, hipStream_t s);
// The coarse end of a spatial cycle in one kernel: one workgroup per slab runs
// the cycle from sub-level `first` (n_0 = n of that sub-level) down to one node
// and back with every sub-level vector in LDS.  Per sub-level j (0 = first):
// Dinv, stencil weights and n.  The result x of the first sub-level is written
// as out = x, scale*x or base + scale*x (upd as in SpatialArgs).
constexpr int TAIL_MAX = 8;
template <typename T>
struct TailArgs {
  T K[NT_MAX * NT_MAX];
  T M[NT_MAX * NT_MAX];
  T Dinv[TAIL_MAX][NT_MAX * NT_MAX];
  T wm[TAIL_MAX][3];
  T wk[TAIL_MAX][3];
  int n[TAIL_MAX];
  int levels;             // sub-levels in the tail (last has n = 1)
  long long slabs;
  T omega;
  T scale;
  int upd;
  int nu1, nu2;
};
// LDS bytes of the tail starting at n (0 if it does not fit the 64 KB budget).
size_t spatial_tail_lds(int dim, int n, int nt, size_t elem);
template <typename T>
hipError_t launch_spatial_tail(int dim, int nt, const T* f, const T* base, T* out, const TailArgs<T>& a,
                               hipStream_t s);
// Full weighting in space on every slab (time untouched): fc = (R_x (x) I) rf.
template <typename T>
hipError_t launch_restrict_space(int dim, int nt, const T* rf, T* fc, int nf, int nc, long long slabs,
                                 hipStream_t s);
// (Bi/tri)linear interpolation in space on every slab, added: uf += (P_x (x) I) ec.
template <typename T>
hipError_t launch_prolong_space(int dim, int nt, const T* ec, T* uf, int nf, int nc, long long slabs,
                                hipStream_t s);

// ------------------------------------------- high DG orders (N_t > NT_MAX)
// Time matrices in device memory (direction applied: K or K^T; ca/cb swapped
// for the adjoint).  stmg_generic.hip.
template <typename T>
struct GenArgs {
  const T* K;             // [nt*nt]
  const T* M;             // [nt*nt] M_tau / tau
  const T* ca;            // [nt]
  const T* cb;            // [nt]
  const T* ints;          // [nt] int_slab psi_l dt / tau
  T tau;
  T wm[3];
  T wk[3];
  int n;
  long long nx;
  int N;
  int batch;
  int dir;                // -1 forward, +1 adjoint
  int nt;
};
template <typename T>
struct GenTransfer {
  const T* R1T;           // [nt*nt]
  const T* R2T;
  int nf, nc;
  long long nxf, nxc;
  int Nc;
  int batch;
  int nt;
};
template <typename Tin, typename Tout>
hipError_t launch_residual_gen(int dim, const Tin* u, const Tin* F, Tout* r, const GenArgs<Tin>& a, double* partial,
                               hipStream_t s);
unsigned residual_gen_blocks_per_slab(long long nx);
template <typename T>
hipError_t launch_time_solve_gen(const T* in, T* out, const T* G, long long nx, int nt, long long slabs, int transpose,
                                 T omega, int mode, hipStream_t s);
template <typename T>
hipError_t launch_restrict_gen(int dim, bool full, const T* rf, T* Fc, const GenTransfer<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_prolong_gen(int dim, bool full, const T* ec, T* uf, const GenTransfer<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_rhs_gen(int dim, const T* f, const T* u0, T* F, const GenArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_rhs_adjoint_gen(int dim, const T* lam, T* gf, T* gu0, const GenArgs<T>& a, hipStream_t s);

}  // namespace stmg

namespace stmg {

// One damped block-Jacobi step on a small level, one workgroup per slab with
// the slab resident in LDS (stmg_smooth_small.hip).
template <typename T>
struct SmallArgs {
  ResidArgs<T> r;   // residual coefficients (direction included)
  T omega;
  int transpose;    // apply G^T in the per-mode solve
  int u_zero;       // u_in is treated as zero (u_in may be null)
  int s_lds;        // set by the launcher: the sine matrix is staged in LDS
};
// LDS bytes the small-level kernel needs (0 if the level does not qualify).
size_t smooth_small_lds(int dim, int n, long long nx, int nt, size_t elem);
template <typename T>
hipError_t launch_smooth_small(int dim, int nt, const T* u_in, T* u_out, const T* F, const T* Splain,
                               const T* G, const SmallArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_copy(const T* in, T* out, long long len, hipStream_t s);

}  // namespace stmg

namespace stmg {

// ------------------------------------------------- P1 meshes (stmg_mesh.hip)
constexpr int MESH_TILE = 512;   // rows per workgroup of the mesh kernels
// One refinement level on the device: the interior M_h and K_h in CSR with one
// shared pattern, and their diagonals [nx][2] = (M_ii, K_ii).
template <typename T>
struct MeshOp {
  const int* rowptr;
  const int* col;
  const T* mv;
  const T* kv;
  const T* diag;
  long long nx;
  // the same matrices column-major in ELL form for the hot kernels: entry e of
  // row i at e * nx + i (ecol, and emk holding (M_h, K_h) pairs), rows padded
  // to ew entries with column i and zero values
  const int* ecol;
  const T* emk;
  int ew;
  // halo of each MESH_TILE-row tile: the distinct columns its rows touch
  // (sorted), hcol[hoff[t] .. hoff[t+1]), at most hmax per tile; lcol[e * nx + i]
  // is the position of ecol[e * nx + i] in the halo of i's tile, ldiag[i] that
  // of node i itself
  const int* hoff;
  const int* hcol;
  const unsigned short* lcol;
  const unsigned short* ldiag;
  int hmax;
};
// Interpolation from the next coarser level: fine node i takes
// w[i] (e[p[2i]] + e[p[2i+1]]) over parents >= 0; its transpose as CSR over the
// coarse nodes (rrow, rcol: fine indices; weights w[rcol]).
struct MeshXfer {
  const int* p;
  const int* rrow;
  const int* rcol;
  long long nxf, nxc;
  // the transpose column-major in ELL form: entry e of coarse row I at
  // e * nxc + I (fine index, -1 for padding), rw entries per row
  const int* rell;
  int rw;
  // halo of each MESH_TILE-row coarse tile: the distinct fine nodes its rows of the
  // transpose touch (sorted), rhcol[rhoff[t] .. rhoff[t+1]), at most rhmax;
  // rloc[e * nxc + I] is the position of rell[e * nxc + I] in that halo
  const int* rhoff;
  const int* rhcol;
  const unsigned short* rloc;
  int rhmax;
};
// Residual r = F - L u on a mesh level; time coefficients as in ResidArgs.
template <typename T>
struct MeshResidArgs {
  MeshOp<T> op;
  T K[NT_MAX * NT_MAX];
  T M[NT_MAX * NT_MAX];
  T ca[NT_MAX];
  T cb[NT_MAX];
  int N;
  int batch;
  int dir;
};
template <typename Tin, typename Tout>
hipError_t launch_mesh_residual(int nt, const Tin* u, const Tin* F, Tout* r, const MeshResidArgs<Tin>& a,
                                double* partial, hipStream_t s);
unsigned mesh_blocks_per_slab(long long nx);
// Node-block Jacobi step or defect on every slab of a mesh level:
// y = x + omega D_i^{-1} (f - A x)_i with D_i = M_ii K + K_ii M (SP_JACOBI), or
// y = f - A x (SP_DEFECT); written as in SpatialArgs (upd, scale, base).
template <typename T>
struct MeshSmoothArgs {
  MeshOp<T> op;
  T K[NT_MAX * NT_MAX];
  T M[NT_MAX * NT_MAX];
  long long slabs;
  T omega;
  T scale;
  int op_kind;
  int upd;
  int x_zero;
};
template <typename T>
hipError_t launch_mesh_smooth(int nt, const T* x, const T* f, const T* base, T* out, const MeshSmoothArgs<T>& a,
                              hipStream_t s);
// fc = (P^T (x) I) rf per slab; uf += (P (x) I) ec per slab.
template <typename T>
hipError_t launch_mesh_restrict_space(int nt, const T* rf, T* fc, const MeshXfer& x, const T* w, long long slabs,
                                      hipStream_t s);
template <typename T>
hipError_t launch_mesh_prolong_space(int nt, const T* ec, T* uf, const MeshXfer& x, const T* w, long long slabs,
                                     hipStream_t s);
// Exact slab solve with a dense inverse (m = N_t nx <= 1024): y = Ainv f
// (Ainv^T f when trans), written as out = y, scale y or base + scale y.
template <typename T>
hipError_t launch_mesh_dense(const T* Ainv, int m, int trans, const T* f, const T* base, T* out, int upd, T scale,
                             long long slabs, hipStream_t s);
// Space-time transfers (eq. chap4_restrictionTime in time; space by the mesh
// interpolation when full, identity when semi).
template <typename T>
struct MeshTransferArgs {
  T R1T[NT_MAX * NT_MAX];
  T R2T[NT_MAX * NT_MAX];
  MeshXfer x;             // nxf == nxc for semi-coarsening
  const T* w;
  int full;
  int Nc;
  int batch;
};
template <typename T>
hipError_t launch_mesh_restrict(int nt, const T* rf, T* Fc, const MeshTransferArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_mesh_prolong(int nt, const T* ec, T* uf, const MeshTransferArgs<T>& a, hipStream_t s);
// Load vector and its transpose on the finest mesh level.
template <typename T>
struct MeshRhsArgs {
  MeshOp<T> op;
  T ints[NT_MAX];
  T ca[NT_MAX];
  int N;
  int batch;
};
template <typename T>
hipError_t launch_mesh_rhs(int nt, const T* f, const T* u0, T* F, const MeshRhsArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_mesh_rhs_adjoint(int nt, const T* lam, T* gf, T* gu0, const MeshRhsArgs<T>& a, hipStream_t s);

}  // namespace stmg

namespace stmg {

// ------------------------------------ coarse end of a cycle in one workgroup
// (stmg_coarse.hip).  Level 0 of the tail is the level the cycle is called on.
constexpr int CT_MAX = 10;
template <typename T>
struct CoarseLevel {
  T K[NT_MAX * NT_MAX];   // as ResidArgs (direction applied)
  T M[NT_MAX * NT_MAX];
  T ca[NT_MAX];
  T cb[NT_MAX];
  T wm[3];
  T wk[3];
  const T* gS;            // plain DST-I, n x n (device)
  const T* gG;            // per-mode inverse blocks in spectral order (device)
  int n, N, nx;
  float rn, rN, rnx;      // 1/n, 1/N, 1/nx for the index arithmetic
  int full;               // transition to the next tail level is full coarsening
  int offS, offG, offU, offF;   // LDS offsets in elements
};
template <typename T>
struct CoarseArgs {
  CoarseLevel<T> lv[CT_MAX];
  T R1T[NT_MAX * NT_MAX];
  T R2T[NT_MAX * NT_MAX];
  T omega;
  int levels;
  int nu1, nu2, gamma;
  int transpose;          // apply G^T
  int dir;                // -1 forward, +1 adjoint
  int offR, offQ;         // two scratch vectors of the largest tail level
};
// One cycle (with gamma coarse cycles below) on the tail's top level:
// u = cycle(u, F) (u treated as zero when u_zero), one workgroup, lds bytes.
template <typename T>
hipError_t launch_coarse_cycle(int dim, int nt, const CoarseArgs<T>* args, size_t lds, const T* F, T* u, int batch,
                               int u_zero, hipStream_t s);

}  // namespace stmg

namespace stmg {

// Twice-folded register transforms (stmg_transform2.hip), FP64 for n = 63,
// 127 and FP32 for n = 63, 127, 255: the x/y passes and the fused slowest-axis
// solve with half the matrix-core work of the once-folded ones; Sfrag2 is
// their fragment table.  The f32 instruction's accumulator rows are blocked
// (row 4 g + j in element j of lane group g) where the f64 one interleaves
// (g + 4 j), so the FP32 table stores output row twice_fold_row(i) at operand
// row i and both types share one register order.
// Per-mode time blocks from the 1-D eigenvalues (N_t <= 4): eig holds m_s then
// kappa_s of one axis in spectral order (2n values), K = K_tau, M = M_tau;
// the block of mode (s_1, .., s_d) is (mu K + nu M)^{-1} with mu = prod m and
// nu = sum_a kappa_a prod_{b != a} m_b.  eig == nullptr: read the table G.
template <typename T>
struct ModeEig {
  const T* eig;
  T K[NT_MAX * NT_MAX];
  T M[NT_MAX * NT_MAX];
};
// With bf16 (FP32 data only) Sfrag2 is the bf16 table of packed quadruples
// (v_mfma_f32_16x16x16_bf16 operands, rows permuted the same way).
bool twice_folded_ok(int n, int elem_bytes);
inline int twice_fold_row(int elem_bytes, int i) { return elem_bytes == 8 ? i : (i >> 2) + 4 * (i & 3); }
// Launch shape of the twice-folded pass kernels, chosen per level by the
// autotuner: waves per workgroup of the line passes (1, 2, 4), workgroups per
// compute unit when the grid is capped (persistent workgroups looping over
// contiguous ranges of tiles; 0 = one tile per wave / workgroup), column
// groups of 16 per workgroup of the fused pass (0 = 4 / N_t for N_t <= 2),
// and the compute-unit count the caps refer to.
struct PassShape {
  int wpg = 4;
  int pass_per_cu = 0;
  int fused_cg = 0;
  int fused_per_cu = 0;
  int cus = 0;
};
template <typename T>
hipError_t launch_pass_reg2(int n, bool inverse, const T* in, T* out, const T* Sfrag2, long long inner,
                            long long ncols, T omega, int mode, hipStream_t s, bool bf16 = false,
                            const PassShape& sh = PassShape{}, long long lps = 0);
// Slab-resident block solve with the twice-folded passes (one workgroup per
// 2-D slab, slab in LDS; FP64 n = 63, FP32 n = 63, 127; N_t <= 2): LDS bytes,
// 0 when the level does not qualify.  With me3 (dim 3) the blocks are the
// (slab, x-mode) planes of the x-mode-major layout [slab][kx][l][z][y] after
// the forward x pass, their per-mode blocks formed from the eigenvalues.
size_t slab_solve2_lds(int dim, int n, int nt, int elem_bytes);
template <typename T>
hipError_t launch_slab_solve2(int n, int nt, const T* src, T* dst, const T* Sfrag2, const T* G, long long slabs,
                              int transpose, T omega, int mode, hipStream_t s, const ModeEig<T>* me3 = nullptr);
// 2-D residual fused with the forward twice-folded x pass (N_t = 2, n = 63,
// 127): xhat = (S_x (x) I) (F - L u) in the layout of r; with `partial` the
// per-tile sums of r^2 in the residual kernel's layout.
bool resid_xfwd_ok(int dim, int n, int nt, int elem_bytes);
// 3-D residual fused with the forward x pass into the x-mode-major layout of
// the slab-resident solves (n = 63, 127; N_t <= 2); partial as in the residual
// (per-workgroup sums of r^2, its own tile count).
bool resid_xfwd3_ok(int n, int nt, int elem_bytes);
unsigned resid_xfwd3_blocks_per_slab(int n, int nt, long long slabs, int elem_bytes);
template <typename T>
hipError_t launch_resid_xfwd3(int n, int nt, const T* u, const T* F, T* xhat, const ResidArgs<T>& a,
                              const T* Sfrag2, double* partial, hipStream_t s);
template <typename T>
hipError_t launch_resid_xfwd(int n, const T* u, const T* F, T* xhat, const ResidArgs<T>& a, const T* Sfrag2,
                             double* partial, hipStream_t s);
template <typename T>
hipError_t launch_fused_pair2(int n, int nt, const T* in, T* out, const T* Sfrag2, const T* G, long long inner,
                              long long outer, int transpose, T omega, int mode, hipStream_t s, bool bf16 = false,
                              const ModeEig<T>* me = nullptr, const PassShape& sh = PassShape{});

}  // namespace stmg
