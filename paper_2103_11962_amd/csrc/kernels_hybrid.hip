// Kernels of the structured/unstructured hybrid hierarchy (the paper's hybrid section, Table 5).
//
// Every level stores its region matrices as one block-diagonal sparse matrix over the regional
// rows (region by region), in ELL slices of 64 rows: a wavefront reads the e-th entry of its 64
// rows as one contiguous 64-element chunk, like the wave-tiled stencil arrays of the structured
// path.  Products are region-local; the interface sums and averages run on the level's interface
// groups (k_group_reduce).  Transfers are piecewise constant: restriction sums the (multiplicity-
// scaled) residual of each aggregate's rows, prolongation adds the coarse value to every row of
// the aggregate.  The region-local Gauss-Seidel sweep walks a precomputed dependency-level
// schedule per region with one block per region (a barrier between levels), which reproduces the
// sequential sweep's arithmetic.
#include "device_common.h"
#include "hybrid.h"
#include "kernels.h"

namespace rmg {

constexpr int kHybGsThreads = 1024;

__device__ __forceinline__ void ell_row(const int64_t* __restrict__ sptr, int64_t i, int64_t& base, int& width) {
  const int64_t s0 = sptr[i >> 6];
  width = (int)((sptr[(i >> 6) + 1] - s0) >> 6);
  base = s0 + (i & 63);
}

__global__ __launch_bounds__(kBlock) void k_hyb_spmv(int64_t n, const int64_t* __restrict__ sptr,
                                                     const int* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t base;
  int w;
  ell_row(sptr, i, base, w);
  double acc = 0.0;
  for (int e = 0; e < w; ++e) acc += val[base + 64 * e] * x[col[base + 64 * e]];
  y[i] = acc;
}

void launch_hyb_spmv(const HLevelDev& L, const double* x, double* y, hipStream_t st) {
  if (L.n == 0) return;
  RMG_LAUNCH(k_hyb_spmv, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, L.sptr.as<int64_t>(),
                     L.col.as<int>(), L.val.as<double>(), x, y);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_hyb_finish(int64_t n, const double* __restrict__ b,
                                                       const double* __restrict__ y, const double* __restrict__ invm,
                                                       double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double r = b[i] - y[i];
  out[i] = invm ? r * invm[i] : r;
}

void launch_hyb_finish(int64_t n, const double* b, const double* y, const double* invm, double* out,
                       hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_hyb_finish, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, b, y, invm, out);
  LAUNCH_CHECK();
}

// One block per region; the region's schedule levels in order, a barrier after each.  Position t
// of a level updates row rows[t] from its lower (upper) couplings stored at t; their neighbours'
// corrections were written on earlier levels.  The composite diagonal enters through dinv.
__global__ __launch_bounds__(kHybGsThreads) void k_hyb_gs(const int* __restrict__ reg, const int* __restrict__ lv,
                                                          const int* __restrict__ rows,
                                                          const int64_t* __restrict__ tsptr,
                                                          const int* __restrict__ tcnt, const int* __restrict__ tcol,
                                                          const double* __restrict__ tval,
                                                          const double* __restrict__ dinv,
                                                          const double* __restrict__ r, double* d, double omega) {
  const int k = blockIdx.x;
  for (int v = reg[k]; v < reg[k + 1]; ++v) {
    for (int t = lv[v] + (int)threadIdx.x; t < lv[v + 1]; t += kHybGsThreads) {
      const int i = rows[t];
      const int c = tcnt[t];
      const int64_t base = tsptr[t >> 6] + (t & 63);
      double acc = r[i];
      for (int e = 0; e < c; ++e) acc -= tval[base + 64 * e] * d[tcol[base + 64 * e]];
      d[i] = omega * acc * dinv[i];
    }
    __syncthreads();
  }
}

void launch_hyb_gs(const HLevelDev& L, const double* r, double* d, double omega, bool backward, hipStream_t st) {
  if (L.n == 0) return;
  const HLevelDev::Sweep& S = backward ? L.bwd : L.fwd;
  RMG_LAUNCH(k_hyb_gs, dim3(L.nreg), dim3(kHybGsThreads), 0, st, S.reg.as<int>(), S.lv.as<int>(),
                     S.rows.as<int>(), S.tsptr.as<int64_t>(), S.tcnt.as<int>(), S.tcol.as<int>(),
                     S.tval.as<double>(), L.dinv.as<double>(), r, d, omega);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_hyb_jacobi(int64_t n, double omega, const double* __restrict__ dinv,
                                                       const double* __restrict__ r, double* __restrict__ u,
                                                       int zero) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double c = omega * dinv[i] * r[i];
  u[i] = zero ? c : u[i] + c;
}

void launch_hyb_jacobi(int64_t n, double omega, const double* dinv, const double* r, double* u, bool zero,
                       hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_hyb_jacobi, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, omega, dinv, r, u, zero ? 1 : 0);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_hyb_restrict(int64_t nc, const int64_t* __restrict__ cptr,
                                                         const int* __restrict__ crows,
                                                         const double* __restrict__ rs, double* __restrict__ bc) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= nc) return;
  double s = 0.0;
  for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) s += rs[crows[e]];
  bc[c] = s;
}

void launch_hyb_restrict(int64_t nc, const int64_t* cptr, const int* crows, const double* rs, double* bc,
                         hipStream_t st) {
  if (nc == 0) return;
  RMG_LAUNCH(k_hyb_restrict, dim3(cdiv(nc, kBlock)), dim3(kBlock), 0, st, nc, cptr, crows, rs, bc);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_hyb_prolong(int64_t n, const int* __restrict__ agg,
                                                        const double* __restrict__ uc, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int a = agg[i];
  if (a >= 0) u[i] += uc[a];
}

void launch_hyb_prolong(int64_t n, const int* agg, const double* uc, double* u, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_hyb_prolong, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, agg, uc, u);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_hyb_gather(int nc, const int* __restrict__ owner,
                                                       const double* __restrict__ b, double* __restrict__ cv) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < nc) cv[c] = b[owner[c]];
}

__global__ __launch_bounds__(kBlock) void k_hyb_scatter(int64_t n, const int* __restrict__ rowcomp,
                                                        const double* __restrict__ cv, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) z[i] = cv[rowcomp[i]];
}

void launch_hyb_coarse(const HLevelDev& L, const double* b, double* z, hipStream_t st) {
  if (L.nc == 0) return;
  RMG_LAUNCH(k_hyb_gather, dim3(cdiv(L.nc, kBlock)), dim3(kBlock), 0, st, L.nc, L.owner.as<int>(), b,
                     L.cvec.as<double>());
  LAUNCH_CHECK();
  launch_dense_gemv(L.nc, L.ainv.as<double>(), L.cvec.as<double>(), L.cvec2.as<double>(), st);
  RMG_LAUNCH(k_hyb_scatter, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, L.rowcomp.as<int>(),
                     L.cvec2.as<double>(), z);
  LAUNCH_CHECK();
}

}  // namespace rmg
