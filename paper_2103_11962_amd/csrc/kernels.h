// Launchers of the HIP kernels.  All launches are asynchronous on `st`.
//
// Vectors are regional (or composite) arrays with `ndof` values per node.  Launchers that take
// `lowp` run on the level's FP32 vectors and its low-precision coefficient copy (FP32, or BF16
// off-diagonals with FP32 centre blocks); otherwise vectors are FP64 with FP64 coefficients.
#pragma once
#include <atomic>

#include "internal.h"

namespace rmg {

// Kernel launches issued by the library in this process (counted by RMG_LAUNCH; read by
// rmg_kernel_launches).
extern std::atomic<int64_t> g_kernel_launches;

// Per-node operations applied after a regional stencil product z = A^(k) x.
enum class StencilOp {
  Matvec,          // y = Psi^T Psi A x
  Residual,        // r = b - Psi^T Psi A x
  ResidualScaled,  // r = (b - Psi^T Psi A x) / mult (input of the regional restriction)
  Cheb,            // r = b - Psi^T Psi A u; u_out = u + c1 (u - u_out) + c2 D~^-1 r, where u_out holds
                   // the iterate before u on entry (the previous correction is their difference)
  ChebFirst,       // u_out = u + c1 u + c2 D~^-1 r: the iterate before u was zero (the step after a
                   // zero-guess start), or c1 = 0 for a step with no previous correction
  CgQ,             // q = Psi^T Psi A p and partial sums of (p, q)
};

struct StencilArgs {
  StencilOp op;
  bool lowp = false;           // FP32 vectors, low-precision coefficients
  const void* x = nullptr;     // stencil input (u or p)
  void* out = nullptr;         // y / r / u_out / q
  const void* b = nullptr;     // right-hand side (Residual*, Cheb*)
  const void* dinv = nullptr;
  void* d = nullptr;           // Cheb*: shared rows' correction, stored for the interface kernel
  double c1 = 0.0, c2 = 0.0;
  double* partials = nullptr;  // CgQ / dot-fused variants: one double per block
  bool dot_rhs = false;        // Cheb*, FP64: also partial sums of (b, u_out) over the owned copies
  const void* dinv9 = nullptr; // Cheb, ChebFirst on 3-dof levels: nodal-block D~^-1 (9 per node), else null
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // when set, recorded around the stencil kernel only
};

// Runs the stencil kernel over all nodes and then the interface-group kernel.
// Returns the number of partial sums written (0 when no reduction was requested).
int64_t launch_stencil_op(const Level& L, const StencilArgs& a, hipStream_t st);

// Interface sum w = Psi^T Psi v on a level (FP64; v == w allowed).
void launch_interface_sum(const Level& L, const double* v, double* w, hipStream_t st);
// Region-local Gauss-Seidel sweep (kernels_gs.hip): delta = (D~/omega + L_k)^-1 r per region k
// (upper triangle, reverse order, when backward); every copy of an interface dof := their average.
// launch_gs_prepare copies the level's stencils and D~^-1 into the sweep's slot order (setup).
void launch_gs_prepare(Level& L, hipStream_t st);
void launch_gs_sweep(const Level& L, const double* r, double* delta, double omega, bool backward, hipStream_t st);
void launch_interface_avg(const Level& L, double* w, hipStream_t st);
// The same on explicit interface groups: every copy := sum (avg = false) or average of the copies.
void launch_group_reduce(const int64_t* gptr, const int* gcopy, int64_t ngroups, double* w, bool avg, hipStream_t st);

// Owner-masked composite dot product (FP64): partial sums written to `partials`; returns their count.
int64_t launch_dot(const Level& L, const double* a, const double* b, double* partials, hipStream_t st);

// Deterministic sum of `n` partials into scalars[slot].
void launch_reduce(const double* partials, int64_t n, double* scalars, int slot, hipStream_t st);

// Pointwise: u = c * dinv * b, the first Chebyshev step from a zero guess (the step after it runs
// as ChebFirst with its c1: its previous correction is u itself).
void launch_cheb_zero(const Level& L, bool lowp, const void* b, const void* dinv, double c, void* u, hipStream_t st,
                      const void* dinv9 = nullptr);

// Restriction level -> level+1 (input already divided by multiplicity), including coarse interface sum.
void launch_restrict(const Level& F, const Level& C, bool lowp, const void* r_scaled, void* w, hipStream_t st);
// Prolongation u += P ubar (level+1 -> level).
void launch_prolong_add(const Level& F, const Level& C, bool lowp, const void* ubar, void* u, hipStream_t st);
// Coarse-major restriction weights (F.rw, 125 per coarse node) from the stored weights F.pw.
void launch_build_rw(const Level& F, const Level& C, double* rw, hipStream_t st);
// Galerkin product per region (FP64): C.coef = R A P.
void launch_rap(const Level& F, Level& C, hipStream_t st);

// Point diagonal (centre coefficient of every dof) into a regional FP64 vector.
void launch_diag(const Level& L, double* out, hipStream_t st);
// out = 1 / in; flags[0] set to 1 if some entry is not finite or not positive.
void launch_recip_check(int64_t n, const double* in, double* out, int* flag, hipStream_t st);
// Power-method start vector (SplitMix64 counter generator, zero on Dirichlet nodes).
void launch_start_vector(const Level& L, int level, uint64_t seed, double* out, hipStream_t st);
// Pointwise helpers (FP64).
void launch_scale(int64_t n, const double* scalars, int slot, int mode, const double* x, double* y,
                  hipStream_t st);  // mode 0: y = x / sqrt(s); mode 1: y = x * s
void launch_mul(int64_t n, const double* a, const double* b, double* y, hipStream_t st);  // y = a*b
void launch_mul_block3(int64_t nodes, const double* D9, const double* x, double* y, hipStream_t st);
// Nodal-block D~^-1 of a 3-dof level into L.dinv9 (RMG_ERR_NUMERIC if a block is not positive definite).
void launch_block_diag(Level& L, hipStream_t st);
void launch_add(int64_t n, const double* x, double* y, hipStream_t st);  // y += x
void launch_log(int64_t n, const double* in, float* out, hipStream_t st);  // out = log(in), FP32
void launch_f64_to_f32(int64_t n, const double* in, float* out, hipStream_t st);
void launch_f32_to_f64(int64_t n, const float* in, double* out, hipStream_t st);
// Low-precision copy of a level's operator: coef_lo (FP32, or BF16 off-diagonals with FP32
// centre blocks whose diagonal keeps each row sum of the FP64 operator) and dinv_lo.
void launch_make_lowp(Level& L, int coef_type, hipStream_t st);

// Upper-half stencil copy of a 27-point 3D level (scalar or 3x3 blocks) whose FP64 operator is
// symmetric to rounding: L.coef_sym, or with lowp L.coef_lo_sym from the low-precision copy of a
// level that has L.coef_sym; returns false (and leaves the copy empty) otherwise.  The stencil
// kernels then stream 14 instead of 27 blocks per node.
bool launch_make_sym(Level& L, bool lowp, hipStream_t st, bool table);

// Composite <-> regional (FP64).
void launch_to_regional(const Level& L, const double* comp, double* reg, hipStream_t st);
void launch_to_composite(const Level& L, const double* reg, double* comp, int average, hipStream_t st);

// Coarsest level: gather owner copies, dense FP64 GEMV with the inverse, scatter to copies.
void launch_coarse_solve(const Level& L, bool lowp, const void* b, void* u, hipStream_t st);
// The coarse solve's halves: owner copies of b into L.cvec (FP64); L.cvec2 to every regional copy.
void launch_coarse_gather(const Level& L, bool lowp, const void* b, hipStream_t st);
void launch_coarse_scatter(const Level& L, bool lowp, void* u, hipStream_t st);
// y = A x, A row-major n x n (one wavefront per row).
void launch_dense_gemv(int n, const double* A, const double* x, double* y, hipStream_t st);
// In-place blocked Gauss-Jordan inversion of an SPD n x n matrix (row-major); synchronises st.
void launch_gauss_jordan(double* A, int n, hipStream_t st);
void launch_check_inverse(const double* A, int n, int* flag, hipStream_t st);

// Q1 assembly (scalar): Kref = 8x8 element matrix of the unit cube scaled by h.
void launch_assemble_q1_scalar(const Level& L, const double* Kref, const double* elem_coef, hipStream_t st);
// Q1 elasticity: Kdev = device 24x24 element matrix for E = 1, youngs_dev = E per region.
void launch_assemble_q1_elasticity(const Level& L, const double* Kdev, const double* youngs_dev, hipStream_t st);
// Dirichlet identity split 1/mult on shared Dirichlet nodes (after assembly).
void launch_dirichlet_split(const Level& L, hipStream_t st);
// Zero couplings that point outside each region box; flag non-finite values.
void launch_mask_stencil(const Level& L, int* flag, hipStream_t st);
// Region matrices from a composite stencil [npts][ncomp] on a tensor-product layout (Section 4 split).
void launch_split_composite(const Level& L, const double* comp, int* flag, hipStream_t st);
// Assembled composite CSR matrix -> composite stencil [L.npts][L.ncomp] (comp zeroed by the caller);
// flag bits: 1 non-finite value, 2 entry outside the stencil, 4 column out of range.
void launch_csr_to_stencil(const Level& L, const int64_t* rowptr, const int* colind, const double* vals,
                           double* comp, int* flag, hipStream_t st);
// Copy one region's stencil between a structure-of-arrays buffer [ncoef][region nodes] and the
// level's wave-tiled storage (to_level = 1: soa -> level).
void launch_region_stencil_io(const Level& L, int region, double* soa, int to_level, hipStream_t st);

// CG helpers (FP64).
// x += alpha p; r -= alpha q; partial sums of owner-masked (r, r); with u0 (scalar levels) also
// u0 = c0 * dinv * r, the V-cycle's zero-guess start from the new r (as launch_cheb_zero).
int64_t launch_cg_update(const Level& L, double* scalars, double* x, double* r, const double* p,
                         const double* q, double* partials, hipStream_t st, const double* dinv = nullptr,
                         double c0 = 0.0, double* u0 = nullptr);
// p = z + beta p.
void launch_cg_direction(int64_t n, double* scalars, const double* z, double* p, hipStream_t st);
// mode 0: alpha = rz / pq; mode 1: beta = rz_new / rz, rz = rz_new;
// mode 2 (flexible CG): beta = -alpha (z_new, q) / rz, rz = rz_new.
void launch_cg_scalars(double* scalars, int mode, hipStream_t st);
void launch_copy(int64_t n, const double* src, double* dst, hipStream_t st);
void launch_zero(int64_t n, double* dst, hipStream_t st);

// scalar slots
enum Slot { kRZ = 0, kPQ = 1, kRR = 2, kAlpha = 3, kBeta = 4, kRZnew = 5, kBB = 6, kTmp = 7, kTmp2 = 8, kZQ = 9,
            kNumSlots = 16 };

}  // namespace rmg
