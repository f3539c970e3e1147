// Kernels of the AMG coarse solver below the region hierarchy (Section 3.5): products with each
// level's composite matrix, smoothed prolongator and its transpose (ELL slices of 64 rows read one
// contiguous chunk per entry slot and wavefront; matrices with long rows, such as the transpose of
// the prolongator, in CSR with a wavefront per row), and the Chebyshev smoother's element-wise
// steps.  The levels are small (the coarse problem of the region hierarchy): L2-resident, latency
// bound; one thread per row.
#include "amg.h"
#include "device_common.h"

namespace rmg {

// y = M x (accumulate 0) or y += M x (accumulate 1); ELL, one thread per row.
__global__ __launch_bounds__(kBlock) void k_ell_apply(int64_t n, const int64_t* __restrict__ sptr,
                                                      const int* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t s0 = sptr[i >> 6];
  const int w = (int)((sptr[(i >> 6) + 1] - s0) >> 6);
  const int64_t base = s0 + (i & 63);
  double acc = 0.0;
  for (int e = 0; e < w; ++e) acc += val[base + 64 * e] * x[col[base + 64 * e]];
  y[i] = accumulate ? y[i] + acc : acc;
}

// The same for CSR with long rows: one wavefront per row; lane l sums entries l, l + 64, ... of
// the row, then the lanes combine in a fixed tree, so the result does not depend on timing.
constexpr int kWaveRows = kBlock / 64;

__global__ __launch_bounds__(kBlock) void k_csr_wave_apply(int64_t n, const int64_t* __restrict__ ptr,
                                                           const int* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ x, double* __restrict__ y,
                                                           int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * kWaveRows + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;  // whole wavefronts leave together
  double acc = 0.0;
  for (int64_t e = ptr[i] + lane; e < ptr[i + 1]; e += 64) acc += val[e] * x[col[e]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) y[i] = accumulate ? y[i] + acc : acc;
}

void launch_sp_apply(const SpDev& M, const double* x, double* y, bool accumulate, hipStream_t st) {
  if (M.n == 0) return;
  if (M.wave)
    RMG_LAUNCH(k_csr_wave_apply, dim3(cdiv(M.n, kWaveRows)), dim3(kBlock), 0, st, M.n, M.sptr.as<int64_t>(),
                       M.col.as<int>(), M.val.as<double>(), x, y, accumulate ? 1 : 0);
  else
    RMG_LAUNCH(k_ell_apply, dim3(cdiv(M.n, kBlock)), dim3(kBlock), 0, st, M.n, M.sptr.as<int64_t>(),
                       M.col.as<int>(), M.val.as<double>(), x, y, accumulate ? 1 : 0);
  LAUNCH_CHECK();
}

// First Chebyshev correction d = (1/theta) D^-1 r; u = d (zero) or u += d.
__global__ __launch_bounds__(kBlock) void k_amg_cheb_first(int64_t n, double inv_theta, const double* __restrict__ dinv,
                                                           const double* __restrict__ r, double* __restrict__ d,
                                                           double* __restrict__ u, int zero) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double di = inv_theta * (dinv[i] * r[i]);
  d[i] = di;
  u[i] = zero ? di : u[i] + di;
}

void launch_amg_cheb_first(int64_t n, double inv_theta, const double* dinv, const double* r, double* d, double* u,
                           bool zero, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_amg_cheb_first, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, inv_theta, dinv, r, d, u,
                     zero ? 1 : 0);
  LAUNCH_CHECK();
}

// Later Chebyshev steps, with y = A u: r = b - y, d = c1 d + c2 D^-1 r, u += d.
__global__ __launch_bounds__(kBlock) void k_amg_cheb_step(int64_t n, double c1, double c2,
                                                          const double* __restrict__ dinv,
                                                          const double* __restrict__ b, const double* __restrict__ y,
                                                          double* __restrict__ d, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double di = c1 * d[i] + c2 * (dinv[i] * (b[i] - y[i]));
  d[i] = di;
  u[i] += di;
}

void launch_amg_cheb_step(int64_t n, double c1, double c2, const double* dinv, const double* b, const double* y,
                          double* d, double* u, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_amg_cheb_step, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, c1, c2, dinv, b, y, d, u);
  LAUNCH_CHECK();
}

// r = b - y.
__global__ __launch_bounds__(kBlock) void k_amg_sub(int64_t n, const double* __restrict__ b,
                                                    const double* __restrict__ y, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) r[i] = b[i] - y[i];
}

void launch_amg_sub(int64_t n, const double* b, const double* y, double* r, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_amg_sub, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, b, y, r);
  LAUNCH_CHECK();
}

}  // namespace rmg
