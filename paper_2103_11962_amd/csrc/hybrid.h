// Structured/unstructured hybrid hierarchy (rmg_options.hybrid): host-side level description
// built by the planner in hybrid.cpp, and the device arrays the kernels of kernels_hybrid.hip read.
#pragma once

#include <array>
#include <memory>
#include <vector>

#include "internal.h"

namespace rmg {

// One region's matrix on a hybrid level (region-local columns, ascending, nonzeros only).
struct HRegionHost {
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<int64_t> comp;               // composite node of each row
  std::vector<std::array<int32_t, 3>> xyz; // composite lattice position, {-1,-1,-1} if none
  std::vector<uint8_t> free;               // 0 for Dirichlet rows (finest level only)
  int64_t n() const { return (int64_t)comp.size(); }
};

// Device arrays of one hybrid level.  Regional rows are numbered region by region.
struct HLevelDev {
  int64_t n = 0;
  int nreg = 0;
  // ELL in slices of 64 rows: the e-th stored entry of row i is at sptr[i / 64] + 64 e + i % 64,
  // e < (sptr[i / 64 + 1] - sptr[i / 64]) / 64; padding entries have column i and value 0
  DBuf sptr;   // int64 [nslices + 1]
  DBuf col;    // int32 regional column
  DBuf val;    // double
  DBuf dinv;   // double [n]: 1 / composite diagonal
  DBuf invm;   // double [n]: 1 / multiplicity
  int64_t ngroups = 0;
  DBuf gptr;   // int64 [ngroups + 1]: copies of each shared composite node, ascending region order
  DBuf gcopy;  // int32
  // Gauss-Seidel schedules, forward and backward: region k owns levels reg[k] .. reg[k+1]-1,
  // level v owns the schedule positions lv[v] .. lv[v+1]-1, position t updates row rows[t]; a
  // row's lower (forward) or upper (backward) neighbours lie on earlier levels.  The couplings a
  // position needs are stored by position in ELL slices of 64 positions: the e-th of position t
  // at tsptr[t / 64] + 64 e + t % 64, e < tcnt[t], so a wavefront loads them contiguously and
  // independently of its rows
  struct Sweep {
    DBuf reg, lv, rows, tsptr, tcnt, tcol, tval;
  } fwd, bwd;
  // transfers to the next level: coarse regional row of each row (-1: Dirichlet); the rows of
  // each coarse row (ascending)
  DBuf agg, cptr, crows;
  // work vectors
  DBuf b, u, r, d, y, b2, t;
  // coarsest level: inverse of the dense composite matrix, owner row of each composite node,
  // composite node of each row
  int nc = 0;
  DBuf ainv, owner, rowcomp, cvec, cvec2;
};

struct HLevel {
  std::vector<HRegionHost> regs;
  std::vector<int64_t> off;     // first regional row of each region, [nreg + 1]
  int64_t ncomp = 0;
  int shape[3] = {1, 1, 1};     // composite lattice extent per axis on this level
  std::vector<int32_t> agg;     // to the next level: coarse regional row of each row, -1 if none
  HLevelDev dev;
};

struct Hybrid {
  int dim = 3;
  unsigned mask = 0;
  std::vector<std::unique_ptr<HLevel>> lv;
};

// Staged plain aggregation of one matrix's free rows (roots, joins, leftovers; no interface
// stage), CSR with ascending columns: coarse index of every row (-1: not aggregated), numbered by
// each aggregate's smallest row.  Returns the number of aggregates.  (hybrid.cpp)
int64_t aggregate_plain(const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                        const std::vector<double>& val, const std::vector<uint8_t>& free, std::vector<int32_t>& agg);

// ---- kernels_hybrid.hip
// y = [[A]] x, region by region (no interface sum).
void launch_hyb_spmv(const HLevelDev& L, const double* x, double* y, hipStream_t st);
// out = (b - y) * invm (invm may be null: factor 1).
void launch_hyb_finish(int64_t n, const double* b, const double* y, const double* invm, double* out,
                       hipStream_t st);
// d = (D~/omega + L_k)^-1 r per region (upper triangle when backward), level-scheduled.
void launch_hyb_gs(const HLevelDev& L, const double* r, double* d, double omega, bool backward, hipStream_t st);
// u = (zero ? 0 : u) + omega D~^-1 r.
void launch_hyb_jacobi(int64_t n, double omega, const double* dinv, const double* r, double* u, bool zero,
                       hipStream_t st);
// bc[c] = sum of rs over the rows of coarse row c.
void launch_hyb_restrict(int64_t nc, const int64_t* cptr, const int* crows, const double* rs, double* bc,
                         hipStream_t st);
// u[i] += uc[agg[i]] for agg[i] >= 0.
void launch_hyb_prolong(int64_t n, const int* agg, const double* uc, double* u, hipStream_t st);
// z = Psi^T Abar^-1 (owner copies of b).
void launch_hyb_coarse(const HLevelDev& L, const double* b, double* z, hipStream_t st);

}  // namespace rmg
