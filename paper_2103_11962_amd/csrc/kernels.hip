// HIP kernels of the regional multigrid path for gfx950: interface sums, reductions,
// transfers, per-region Galerkin products, assembly, precision conversion, coarse solve and
// CG helpers.  The stencil operations live in kernels_stencil.hip.
//
// Work decomposition: every level keeps a table of BlockDesc (region, first local node); one
// 256-thread block processes 256 consecutive nodes of one region (x fastest), so vector streams
// are unit-stride and a block never straddles two regions.  Vectors hold `ndof` values per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.h"

namespace rmg {

std::atomic<int64_t> g_kernel_launches{0};

// ------------------------------------------------------- interface sum
template <int NDOF, class V>
__global__ __launch_bounds__(kBlock) void k_iface_sum(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                      int64_t ng, V* w) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t a0 = gptr[g], e = gptr[g + 1];
#pragma unroll
  for (int a = 0; a < NDOF; ++a) {
    V s = (V)0;
    for (int64_t c = a0; c < e; ++c) s += w[(int64_t)gcopy[c] * NDOF + a];
    for (int64_t c = a0; c < e; ++c) w[(int64_t)gcopy[c] * NDOF + a] = s;
  }
}

template <class V>
static void iface_sum_inplace(const Level& L, V* w, hipStream_t st) {
  if (L.ngroups == 0) return;
  const dim3 g(cdiv(L.ngroups, kBlock));
  if (L.ndof == 3)
    RMG_LAUNCH((k_iface_sum<3, V>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, w);
  else
    RMG_LAUNCH((k_iface_sum<1, V>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, w);
  LAUNCH_CHECK();
}

__global__ void k_copy(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

void launch_copy(int64_t n, const double* src, double* dst, hipStream_t st) {
  if (n == 0 || src == dst) return;
  RMG_LAUNCH(k_copy, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, src, dst);
  LAUNCH_CHECK();
}

void launch_interface_sum(const Level& L, const double* v, double* w, hipStream_t st) {
  if (v != w) launch_copy(L.ndofs(), v, w, st);
  iface_sum_inplace<double>(L, w, st);
}

// ------------------------------------------------------------ reductions
// Node blocks per block of the owner-masked dot products (kDescsPerBlock) and of the CG update
// (kUpdateDescs): each block sums that many consecutive node blocks, so the deterministic final
// reduction (one block) reads few partials.  The update, which also stores two vectors, runs
// fastest with two.
constexpr int kDescsPerBlock = 8;
constexpr int kUpdateDescs = 2;

static int64_t reduction_blocks(const Level& L, int per) { return cdiv((int64_t)L.blocks.size(), per); }

template <int NDOF>
__global__ __launch_bounds__(kBlock) void k_dot_nodes(LevelView L, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ partials) {
  double c = 0.0;
  for (int j = 0; j < kDescsPerBlock; ++j) {
    const int64_t d = (int64_t)blockIdx.x * kDescsPerBlock + j;
    if (d >= L.nblocks) break;
    const BlockDesc bd = L.blocks[d];
    const RegionGeo R = L.regs[bd.region];
    const int li = bd.start + (int)threadIdx.x;
    if (li < R.n) {
      int x, y, z;
      decompose(R, li, x, y, z);
      if (!is_shared(L, R, x, y, z)) {
        const int64_t gi = (R.off + li) * NDOF;
#pragma unroll
        for (int k = 0; k < NDOF; ++k) c += a[gi + k] * b[gi + k];
      }
    }
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <int NDOF>
__global__ __launch_bounds__(kBlock) void k_dot_groups(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                       int64_t ng, const double* __restrict__ a,
                                                       const double* __restrict__ b, double* __restrict__ partials) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double c = 0.0;
  if (g < ng) {
    const int64_t i = (int64_t)gcopy[gptr[g]] * NDOF;
#pragma unroll
    for (int k = 0; k < NDOF; ++k) c += a[i + k] * b[i + k];
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

static int64_t dot_groups(const Level& L, const double* a, const double* b, double* partials, hipStream_t st) {
  if (L.ngroups == 0) return 0;
  const int64_t ngb = cdiv(L.ngroups, kBlock);
  if (L.ndof == 3)
    RMG_LAUNCH(k_dot_groups<3>, dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, a, b, partials);
  else
    RMG_LAUNCH(k_dot_groups<1>, dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, a, b, partials);
  LAUNCH_CHECK();
  return ngb;
}

int64_t launch_dot(const Level& L, const double* a, const double* b, double* partials, hipStream_t st) {
  const int64_t nb = reduction_blocks(L, kDescsPerBlock);
  if (L.ndof == 3) RMG_LAUNCH(k_dot_nodes<3>, dim3(nb), dim3(kBlock), 0, st, L.view(), a, b, partials);
  else RMG_LAUNCH(k_dot_nodes<1>, dim3(nb), dim3(kBlock), 0, st, L.view(), a, b, partials);
  LAUNCH_CHECK();
  return nb + dot_groups(L, a, b, partials + nb, st);
}

constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double* __restrict__ partials, int64_t n,
                                                           double* scalars, int slot) {
  // eight strided sums per thread, so that eight loads are in flight
  double sj[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = threadIdx.x;
  for (; i + 7 * kReduceThreads < n; i += 8 * kReduceThreads) {
#pragma unroll
    for (int j = 0; j < 8; ++j) sj[j] += partials[i + j * kReduceThreads];
  }
  for (; i < n; i += kReduceThreads) sj[0] += partials[i];
  const double s = ((sj[0] + sj[1]) + (sj[2] + sj[3])) + ((sj[4] + sj[5]) + (sj[6] + sj[7]));
  __shared__ double sm[kReduceThreads];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) scalars[slot] = sm[0];
}

void launch_reduce(const double* partials, int64_t n, double* scalars, int slot, hipStream_t st) {
  RMG_LAUNCH(k_reduce, dim3(1), dim3(kReduceThreads), 0, st, partials, n, scalars, slot);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ pointwise
template <class V>
__global__ void k_cheb_zero(int64_t n, const V* __restrict__ b, const V* __restrict__ dinv, V c, V* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = c * (dinv[i] * b[i]);
}

// The same with the nodal-block D~^-1 of a 3-dof level (one row-major 3 x 3 block per node).
template <class V>
__global__ void k_cheb_zero_block3(int64_t nodes, const V* __restrict__ b, const V* __restrict__ dinv9, V c,
                                   V* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  const V* __restrict__ D = dinv9 + i * 9;
  const V b0 = b[3 * i], b1 = b[3 * i + 1], b2 = b[3 * i + 2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[3 * i + a] = c * (D[3 * a] * b0 + D[3 * a + 1] * b1 + D[3 * a + 2] * b2);
  }
}

void launch_cheb_zero(const Level& L, bool lowp, const void* b, const void* dinv, double c, void* u, hipStream_t st,
                      const void* dinv9) {
  const int64_t n = L.ndofs();
  if (dinv9) {
    RMG_REQUIRE(L.ndof == 3, RMG_ERR_ARG, "internal: nodal blocks on a scalar level");
    if (lowp)
      RMG_LAUNCH(k_cheb_zero_block3<float>, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, (const float*)b,
                 (const float*)dinv9, (float)c, (float*)u);
    else
      RMG_LAUNCH(k_cheb_zero_block3<double>, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, (const double*)b,
                 (const double*)dinv9, c, (double*)u);
    LAUNCH_CHECK();
    return;
  }
  if (lowp)
    RMG_LAUNCH(k_cheb_zero<float>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, (const float*)b,
                       (const float*)dinv, (float)c, (float*)u);
  else
    RMG_LAUNCH(k_cheb_zero<double>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, (const double*)b,
                       (const double*)dinv, c, (double*)u);
  LAUNCH_CHECK();
}

__global__ void k_scale(int64_t n, const double* scalars, int slot, int mode, const double* __restrict__ x,
                        double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = scalars[slot];
  const double f = mode == 0 ? 1.0 / sqrt(s) : s;
  y[i] = f * x[i];
}

void launch_scale(int64_t n, const double* scalars, int slot, int mode, const double* x, double* y,
                  hipStream_t st) {
  RMG_LAUNCH(k_scale, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, scalars, slot, mode, x, y);
  LAUNCH_CHECK();
}

__global__ void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] * b[i];
}

void launch_mul(int64_t n, const double* a, const double* b, double* y, hipStream_t st) {
  RMG_LAUNCH(k_mul, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, a, b, y);
  LAUNCH_CHECK();
}

// y = blockdiag(D) x with one row-major 3 x 3 block per node.
__global__ void k_mul_block3(int64_t nodes, const double* __restrict__ D9, const double* __restrict__ x,
                             double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  const double* __restrict__ D = D9 + i * 9;
  const double x0 = x[3 * i], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
#pragma unroll
  for (int a = 0; a < 3; ++a) y[3 * i + a] = D[3 * a] * x0 + D[3 * a + 1] * x1 + D[3 * a + 2] * x2;
}

void launch_mul_block3(int64_t nodes, const double* D9, const double* x, double* y, hipStream_t st) {
  RMG_LAUNCH(k_mul_block3, dim3(cdiv(nodes, kBlock)), dim3(kBlock), 0, st, nodes, D9, x, y);
  LAUNCH_CHECK();
}

// Nodal-block D~ of a 3-dof level (Section 3.2 smoother setup, block reading): column j of every
// node's centre block of [[A]], as a regional 3-vector per node, so that the interface sum adds
// the copies' blocks column by column.
__global__ __launch_bounds__(kBlock) void k_centre_column(LevelView L, const double* __restrict__ coef, int j,
                                                          double* __restrict__ col) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  const int64_t gi = R.off + li;
#pragma unroll
  for (int a = 0; a < 3; ++a) col[gi * 3 + a] = coef[coef_index(gi, (13 * 3 + a) * 3 + j, 27 * 9)];
}

// Inverse of each node's summed block (adjugate over the determinant); a block whose determinant
// is not positive and finite sets the flag.
__global__ void k_block_inv3(int64_t nodes, const double* __restrict__ c0, const double* __restrict__ c1,
                             const double* __restrict__ c2, double* __restrict__ D9, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  const double* col[3] = {c0, c1, c2};
  double B[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[a][j] = col[j][3 * i + a];
  const double k00 = B[1][1] * B[2][2] - B[1][2] * B[2][1], k01 = B[0][2] * B[2][1] - B[0][1] * B[2][2],
               k02 = B[0][1] * B[1][2] - B[0][2] * B[1][1];
  const double k10 = B[1][2] * B[2][0] - B[1][0] * B[2][2], k11 = B[0][0] * B[2][2] - B[0][2] * B[2][0],
               k12 = B[0][2] * B[1][0] - B[0][0] * B[1][2];
  const double k20 = B[1][0] * B[2][1] - B[1][1] * B[2][0], k21 = B[0][1] * B[2][0] - B[0][0] * B[2][1],
               k22 = B[0][0] * B[1][1] - B[0][1] * B[1][0];
  const double det = B[0][0] * k00 + B[0][1] * k10 + B[0][2] * k20;
  if (!(det > 0.0) || !isfinite(det)) atomicOr(flag, 1);
  const double r = 1.0 / det;
  double* __restrict__ D = D9 + i * 9;
  D[0] = k00 * r;
  D[1] = k01 * r;
  D[2] = k02 * r;
  D[3] = k10 * r;
  D[4] = k11 * r;
  D[5] = k12 * r;
  D[6] = k20 * r;
  D[7] = k21 * r;
  D[8] = k22 * r;
}

void launch_block_diag(Level& L, hipStream_t st) {
  RMG_REQUIRE(L.ndof == 3 && L.npts == 27, RMG_ERR_ARG, "nodal-block D~ needs a 3-dof 27-point level");
  const size_t nv = (size_t)L.ndofs();
  DBuf cols, flag;
  cols.alloc(sizeof(double) * 3 * nv);
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  double* c = cols.as<double>();
  for (int j = 0; j < 3; ++j) {
    RMG_LAUNCH(k_centre_column, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), j,
               c + j * nv);
    launch_interface_sum(L, c + j * nv, c + j * nv, st);
  }
  L.dinv9.alloc(sizeof(double) * 9 * (size_t)L.n);
  RMG_LAUNCH(k_block_inv3, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, c, c + nv, c + 2 * nv,
             L.dinv9.as<double>(), flag.as<int>());
  LAUNCH_CHECK();
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "a nodal block of the composite diagonal is not positive definite");
}

__global__ void k_add(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

void launch_add(int64_t n, const double* x, double* y, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_add, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, x, y);
  LAUNCH_CHECK();
}

__global__ void k_zero(int64_t n, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

void launch_zero(int64_t n, double* y, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_zero, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, y);
  LAUNCH_CHECK();
}

__global__ void k_f64_to_f32(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(int64_t n, const float* __restrict__ in, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

void launch_f64_to_f32(int64_t n, const double* in, float* out, hipStream_t st) {
  RMG_LAUNCH(k_f64_to_f32, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, in, out);
  LAUNCH_CHECK();
}
void launch_f32_to_f64(int64_t n, const float* in, double* out, hipStream_t st) {
  RMG_LAUNCH(k_f32_to_f64, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, in, out);
  LAUNCH_CHECK();
}

__global__ void k_recip_check(int64_t n, const double* __restrict__ in, double* __restrict__ out, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = in[i];
  if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
  out[i] = 1.0 / v;
}

void launch_recip_check(int64_t n, const double* in, double* out, int* flag, hipStream_t st) {
  RMG_LAUNCH(k_recip_check, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, in, out, flag);
  LAUNCH_CHECK();
}

// --------------------------------------------------------- diag / start
// Point diagonal: dof a of node i takes entry (a, a) of the centre block.
__global__ void k_diag(int64_t n, int ndof, int ncoef, int center, const double* __restrict__ coef,
                       double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ndof) return;
  const int64_t i = t / ndof;
  const int a = (int)(t - i * ndof);
  out[t] = coef[coef_index(i, center * ndof * ndof + a * ndof + a, ncoef)];
}

void launch_diag(const Level& L, double* out, hipStream_t st) {
  const int center = L.npts == 27 ? 13 : (L.npts == 9 ? 4 : 2);
  RMG_LAUNCH(k_diag, dim3(cdiv(L.ndofs(), kBlock)), dim3(kBlock), 0, st, L.n, L.ndof, L.ncoef(), center,
                     L.coef.as<double>(), out);
  LAUNCH_CHECK();
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): golden-ratio increment and the
// variant-13 finaliser; the counter of composite dof i on level l under seed s is
// i + (l << 40) + (s << 48), composite dofs numbered node-major, dof-minor.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_start_vector(LevelView L, int level, uint64_t seed,
                                                         double* __restrict__ out) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  const bool dn = is_dirichlet(L, gx, gy, gz);
  for (int a = 0; a < L.ndof; ++a) {
    double v = 0.0;
    if (!dn) {
      const uint64_t ctr = (uint64_t)(comp_index(L, gx, gy, gz) * L.ndof + a) + ((uint64_t)level << 40) + (seed << 48);
      const uint64_t r = splitmix64(ctr);
      v = 2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0;
    }
    out[(R.off + li) * L.ndof + a] = v;
  }
}

void launch_start_vector(const Level& L, int level, uint64_t seed, double* out, hipStream_t st) {
  RMG_LAUNCH(k_start_vector, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), level, seed, out);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ transfers
// Stored interpolation weights (learned or caller-given): 8 per fine node for the corners
// (ix, iy, iz) of its canonical coarse cell c = min(f / 3, coarse extent - 2), slot
// ix + 2 iy + 4 iz.  Returns P(f, C) for fine node f and coarse node C of the same region.
__device__ __forceinline__ double pweight(const double* __restrict__ pw, const RegionGeo& RF, const RegionGeo& RC,
                                          int fx, int fy, int fz, int X, int Y, int Z) {
  const int cx = min(fx / 3, RC.ex - 2), cy = min(fy / 3, RC.ey - 2), cz = RC.ez > 1 ? min(fz / 3, RC.ez - 2) : 0;
  const int ix = X - cx, iy = Y - cy, iz = Z - cz;
  if ((unsigned)ix > 1u || (unsigned)iy > 1u || (unsigned)iz > 1u) return 0.0;
  return pw[(RF.off + ((int64_t)fz * RF.ey + fy) * RF.ex + fx) * 8 + ix + 2 * iy + 4 * iz];
}

// One thread per coarse node: w = sum_f P_fC r_f over the fine nodes of the same region in the
// coarse intervals on either side of the node (at most two fine cells per side; r already divided
// by multiplicity), per dof.  Coarse Dirichlet nodes receive nothing (free fine nodes do not
// interpolate from them).
template <int DIM, int NDOF, class V>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelView F, LevelView C, const V* __restrict__ r,
                                                     V* __restrict__ w) {
  const BlockDesc bd = C.blocks[blockIdx.x];
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RC.n) return;
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const int64_t gi = RC.off + li;
  V acc[NDOF];
#pragma unroll
  for (int a = 0; a < NDOF; ++a) acc[a] = (V)0;
  if (!is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z)) {
    const V* __restrict__ rr = r + RF.off * NDOF;
    const int px = coarse_pos(X, RF.ex), py = coarse_pos(Y, RF.ey), pz = DIM == 3 ? coarse_pos(Z, RF.ez) : 0;
    int mxl, mxr, myl, myr, mzl = 0, mzr = 0;
    coarse_spans(X, RF.ex, RC.ex, mxl, mxr);
    coarse_spans(Y, RF.ey, RC.ey, myl, myr);
    if (DIM == 3) coarse_spans(Z, RF.ez, RC.ez, mzl, mzr);
    double wxs[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) wxs[t] = tap(t - 2, mxl, mxr);
    const int tzlo = DIM == 3 ? -2 : 0, tzhi = DIM == 3 ? 2 : 0;
#pragma unroll 1
    for (int tz = tzlo; tz <= tzhi; ++tz) {
      const int fz = pz + tz;
      if ((unsigned)fz >= (unsigned)RF.ez) continue;
      const double wz = DIM == 3 ? tap(tz, mzl, mzr) : 1.0;
      if (wz == 0.0) continue;
      for (int ty = -2; ty <= 2; ++ty) {
        const int fy = py + ty;
        if ((unsigned)fy >= (unsigned)RF.ey) continue;
        const double wy = tap(ty, myl, myr);
        if (wy == 0.0) continue;
        const double wzy = wz * wy;
        const int base = (fz * RF.ey + fy) * RF.ex;
#pragma unroll
        for (int tx = -2; tx <= 2; ++tx) {
          const int fx = px + tx;
          if ((unsigned)fx >= (unsigned)RF.ex) continue;
          const double wx = wxs[tx + 2];
          if (wx == 0.0) continue;
          const V wt = (V)(wzy * wx);
#pragma unroll
          for (int a = 0; a < NDOF; ++a) acc[a] += wt * rr[(int64_t)(base + fx) * NDOF + a];
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < NDOF; ++a) w[gi * NDOF + a] = acc[a];
}

// The same restriction by rows and planes (tiles of make_transfer_tiles): a block owns whole
// coarse rows (one thread per coarse node) and a few coarse planes of one region, walks the fine
// planes that reach them and stages each plane's fine rows in LDS with coalesced loads, so every
// fine value is read from memory once per block instead of once per coarse node that weights it.
// A fine plane adds to the two coarse planes whose intervals hold it; each coarse node's sum takes
// its terms in the order of k_restrict (planes, rows, then x ascending, zero weights skipped, the
// same weight products), so the two kernels give the same results bit for bit.
__device__ __forceinline__ bool dir_axis(unsigned mask, int bit, int g, int n) {
  return (((mask >> bit) & 1u) && g == 0) || (((mask >> (bit + 1)) & 1u) && g == n - 1);
}

template <int DIM, int NDOF, class V>
__global__ __launch_bounds__(kBlock) void k_restrict_planes(LevelView F, LevelView C, const Tile3* __restrict__ tiles,
                                                            int64_t stage_vals, const V* __restrict__ r,
                                                            V* __restrict__ w) {
  extern __shared__ double xfer_stage[];
  V* const stage0 = reinterpret_cast<V*>(xfer_stage);
  V* const stage1 = stage0 + stage_vals;
  const Tile3 T = tiles[xcd_item((int)blockIdx.x, (int)gridDim.x)];
  const RegionGeo RF = F.regs[T.region];
  const RegionGeo RC = C.regs[T.region];
  const int t = threadIdx.x;
  const int fy0 = max(coarse_pos(T.y0, RF.ey) - 2, 0);
  const int fy1 = min(coarse_pos(T.y0 + T.ty - 1, RF.ey) + 2, RF.ey - 1);
  const int fz0 = DIM == 3 ? max(coarse_pos(T.z0, RF.ez) - 2, 0) : 0;
  const int fz1 = DIM == 3 ? min(coarse_pos(T.z0 + T.nz - 1, RF.ez) + 2, RF.ez - 1) : 0;
  const int nval = (fy1 - fy0 + 1) * RF.ex * NDOF;
  const bool act = t < RC.ex * T.ty;
  const int X = act ? t % RC.ex : 0, Y = T.y0 + (act ? t / RC.ex : 0);
  const int px = coarse_pos(X, RF.ex), py = coarse_pos(Y, RF.ey);
  int mxl, mxr, myl, myr;
  coarse_spans(X, RF.ex, RC.ex, mxl, mxr);
  coarse_spans(Y, RF.ey, RC.ey, myl, myr);
  double wxs[5], wys[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    wxs[k] = tap(k - 2, mxl, mxr);
    wys[k] = tap(k - 2, myl, myr);
  }
  const bool dxy = dir_axis(C.mask, 0, RC.ox + X, C.cx) || dir_axis(C.mask, 2, RC.oy + Y, C.cy);
  V acc0[NDOF], acc1[NDOF];  // coarse planes zc and zc + 1
#pragma unroll
  for (int a = 0; a < NDOF; ++a) acc0[a] = acc1[a] = (V)0;
  int zc = fz0 / 3;
  auto flush = [&](int Z, const V* acc) {
    if (!act || Z < T.z0 || Z >= T.z0 + T.nz) return;
    const bool dir = dxy || dir_axis(C.mask, 4, RC.oz + Z, C.cz);
    const int64_t gi = (RC.off + ((int64_t)Z * RC.ey + Y) * RC.ex + X) * NDOF;
#pragma unroll
    for (int a = 0; a < NDOF; ++a) w[gi + a] = dir ? (V)0 : acc[a];
  };
  // a plane's staged rows pass through registers (fetched while the plane before is summed) into
  // one of two LDS buffers
  V pre[kXferStagePerThread];
  auto fetch = [&](int fz) {
    const V* __restrict__ src = r + (RF.off + ((int64_t)fz * RF.ey + fy0) * RF.ex) * NDOF;
#pragma unroll
    for (int j = 0; j < kXferStagePerThread; ++j) {
      const int i = t + j * kBlock;
      pre[j] = i < nval ? src[i] : (V)0;
    }
  };
  auto put = [&](V* __restrict__ dst) {
#pragma unroll
    for (int j = 0; j < kXferStagePerThread; ++j) {
      const int i = t + j * kBlock;
      if (i < nval) dst[i] = pre[j];
    }
  };
  fetch(fz0);
  put(stage0);
  for (int fz = fz0, buf = 0; fz <= fz1; ++fz, buf ^= 1) {
    if (fz < fz1) fetch(fz + 1);
    __syncthreads();  // this plane's rows are staged; the other buffer's readers are done
    const V* __restrict__ rows = buf ? stage1 : stage0;
    if (DIM == 3 && fz / 3 != zc) {  // coarse plane zc has all its terms
      flush(zc, acc0);
#pragma unroll
      for (int a = 0; a < NDOF; ++a) {
        acc0[a] = acc1[a];
        acc1[a] = (V)0;
      }
      zc = fz / 3;
    }
    double wz0 = 1.0, wz1 = 0.0;
    if (DIM == 3) {
      int ml, mr;
      coarse_spans(zc, RF.ez, RC.ez, ml, mr);
      wz0 = tap(fz - coarse_pos(zc, RF.ez), ml, mr);
      if (zc + 1 < RC.ez) {
        coarse_spans(zc + 1, RF.ez, RC.ez, ml, mr);
        wz1 = tap(fz - coarse_pos(zc + 1, RF.ez), ml, mr);
      }
    }
    if (act) {
#pragma unroll
      for (int ky = 0; ky < 5; ++ky) {
        const double wy = wys[ky];
        if (wy == 0.0) continue;
        const double wzy0 = wz0 * wy, wzy1 = wz1 * wy;
        const V* __restrict__ row = rows + (py + ky - 2 - fy0) * RF.ex * NDOF;
#pragma unroll
        for (int kx = 0; kx < 5; ++kx) {
          const double wx = wxs[kx];
          if (wx == 0.0) continue;
          const V w0 = (V)(wzy0 * wx), w1 = (V)(wzy1 * wx);
#pragma unroll
          for (int a = 0; a < NDOF; ++a) {
            const V v = row[(px + kx - 2) * NDOF + a];
            if (wz0 != 0.0) acc0[a] += w0 * v;
            if (wz1 != 0.0) acc1[a] += w1 * v;
          }
        }
      }
    }
    if (fz < fz1) put(buf ? stage0 : stage1);
  }
  flush(zc, acc0);
  if (DIM == 3 && zc + 1 < RC.ez) flush(zc + 1, acc1);
}

// Stored interpolation, coarse-major copy of the restriction weights: for every coarse node C the
// 125 weights P(3C + t, C), t in [-2, 2]^3 (slot (tz+2)*25 + (ty+2)*5 + tx+2), wave-tiled like the
// stencil coefficients so that the restriction streams them instead of gathering single slots of
// the fine nodes' weight records.  Zero outside the region box.
constexpr int kRestrictTaps = 125;

__global__ __launch_bounds__(kBlock) void k_build_rw(LevelView F, LevelView C, const double* __restrict__ pw,
                                                     double* __restrict__ rw) {
  const BlockDesc bd = C.blocks[blockIdx.x];
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RC.n) return;
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const int64_t gi = RC.off + li;
  for (int t = 0; t < kRestrictTaps; ++t) {
    const int fx = 3 * X + t % 5 - 2, fy = 3 * Y + (t / 5) % 5 - 2, fz = 3 * Z + t / 25 - 2;
    const bool in = (unsigned)fx < (unsigned)RF.ex && (unsigned)fy < (unsigned)RF.ey && (unsigned)fz < (unsigned)RF.ez;
    rw[coef_index(gi, t, kRestrictTaps)] = in ? pweight(pw, RF, RC, fx, fy, fz, X, Y, Z) : 0.0;
  }
}

void launch_build_rw(const Level& F, const Level& C, double* rw, hipStream_t st) {
  RMG_LAUNCH(k_build_rw, dim3(C.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), F.pw.as<double>(),
                     rw);
  LAUNCH_CHECK();
}

template <class V>
__global__ __launch_bounds__(kBlock) void k_restrict_rw(LevelView F, LevelView C, const V* __restrict__ r,
                                                        V* __restrict__ w, const double* __restrict__ rw) {
  const BlockDesc bd = C.blocks[blockIdx.x];
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RC.n) return;
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const int64_t gi = RC.off + li;
  V acc = (V)0;
  if (!is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z)) {
    const V* __restrict__ rr = r + RF.off;
    const double* __restrict__ wt = rw + coef_index(gi, 0, kRestrictTaps);  // slot t at wt[t * 64]
    for (int tz = -2; tz <= 2; ++tz) {
      const int fz = 3 * Z + tz;
      if ((unsigned)fz >= (unsigned)RF.ez) continue;
      for (int ty = -2; ty <= 2; ++ty) {
        const int fy = 3 * Y + ty;
        if ((unsigned)fy >= (unsigned)RF.ey) continue;
        const int base = (fz * RF.ey + fy) * RF.ex;
        const int t0 = (tz + 2) * 25 + (ty + 2) * 5;
#pragma unroll
        for (int tx = -2; tx <= 2; ++tx) {
          const int fx = 3 * X + tx;
          if ((unsigned)fx >= (unsigned)RF.ex) continue;
          acc += (V)wt[(t0 + tx + 2) * kTile] * rr[base + fx];
        }
      }
    }
  }
  w[gi] = acc;
}

template <int NDOF, class V>
static void restrict_t(const Level& F, const Level& C, const V* r, V* w, hipStream_t st) {
  const double* pw = F.pw.as<double>();
  if (!pw && !F.rtiles.empty()) {
    const dim3 g(F.rtiles.size()), b(kBlock);
    RMG_REQUIRE(F.rtile_vals <= (int64_t)kXferStagePerThread * kBlock, RMG_ERR_ARG,
                "internal: restriction tile stages more than its block holds");
    const size_t lds = 2 * sizeof(V) * (size_t)F.rtile_vals;
    if (F.dim == 3)
      RMG_LAUNCH((k_restrict_planes<3, NDOF, V>), g, b, lds, st, F.view(), C.view(), F.d_rtiles.as<Tile3>(),
                 F.rtile_vals, r, w);
    else
      RMG_LAUNCH((k_restrict_planes<2, NDOF, V>), g, b, lds, st, F.view(), C.view(), F.d_rtiles.as<Tile3>(),
                 F.rtile_vals, r, w);
    LAUNCH_CHECK();
    iface_sum_inplace<V>(C, w, st);
    return;
  }
  const dim3 g(C.blocks.size()), b(kBlock);
  if constexpr (NDOF == 1) {
    if (pw) {
      RMG_REQUIRE(F.dim == 3 && F.rw.p, RMG_ERR_ARG, "stored interpolation weights need a 3D level");
      RMG_LAUNCH((k_restrict_rw<V>), g, b, 0, st, F.view(), C.view(), r, w, F.rw.as<double>());
      LAUNCH_CHECK();
      iface_sum_inplace<V>(C, w, st);
      return;
    }
  }
  if (F.dim == 3)
    RMG_LAUNCH((k_restrict<3, NDOF, V>), g, b, 0, st, F.view(), C.view(), r, w);
  else
    RMG_LAUNCH((k_restrict<2, NDOF, V>), g, b, 0, st, F.view(), C.view(), r, w);
  LAUNCH_CHECK();
  iface_sum_inplace<V>(C, w, st);
}

void launch_restrict(const Level& F, const Level& C, bool lowp, const void* r_scaled, void* w, hipStream_t st) {
  if (lowp) {
    if (F.ndof == 3) restrict_t<3, float>(F, C, (const float*)r_scaled, (float*)w, st);
    else restrict_t<1, float>(F, C, (const float*)r_scaled, (float*)w, st);
  } else {
    if (F.ndof == 3) restrict_t<3, double>(F, C, (const double*)r_scaled, (double*)w, st);
    else restrict_t<1, double>(F, C, (const double*)r_scaled, (double*)w, st);
  }
}

// One thread per fine node: u += sum_C P_fC ubar_C over the (up to 2 per axis) coarse nodes of
// the coarse interval containing the node, per dof.  Stored weights are kept per canonical cell
// of the rate-3 lattice (extents 3^k + 1).
template <int DIM, int NDOF, class V, bool STORED>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView F, LevelView C, const V* __restrict__ ubar,
                                                        V* __restrict__ u, const double* __restrict__ pw) {
  const BlockDesc bd = F.blocks[blockIdx.x];
  const RegionGeo RF = F.regs[bd.region];
  const RegionGeo RC = C.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RF.n) return;
  int x, y, z;
  decompose(RF, li, x, y, z);
  const V* __restrict__ ub = ubar + RC.off * NDOF;
  V acc[NDOF];
#pragma unroll
  for (int a = 0; a < NDOF; ++a) acc[a] = (V)0;
  if constexpr (STORED) {
    const double* __restrict__ wv = pw + (RF.off + li) * 8;
    const int bx = min(x / 3, RC.ex - 2), by = min(y / 3, RC.ey - 2), bz = RC.ez > 1 ? min(z / 3, RC.ez - 2) : 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const double wt = wv[s];
      if (wt == 0.0) continue;
      const int X = bx + (s & 1), Y = by + ((s >> 1) & 1), Z = bz + ((s >> 2) & 1);
      acc[0] += (V)wt * ub[(int64_t)((Z * RC.ey + Y) * RC.ex + X)];
    }
    u[RF.off + li] += acc[0];
    return;
  }
  const bool fdir = is_dirichlet(F, RF.ox + x, RF.oy + y, RF.oz + z);
  int lx, ly, lz = 0;
  double ax0, ax1, ay0, ay1, az0 = 1.0, az1 = 0.0;
  bracket(x, RF.ex, RC.ex, lx, ax0, ax1);
  bracket(y, RF.ey, RC.ey, ly, ay0, ay1);
  if (DIM == 3) bracket(z, RF.ez, RC.ez, lz, az0, az1);
  // all 2 x 2 (x 2) candidates, unrolled: an absent one (zero weight, or a Dirichlet coarse node
  // seen from a free fine node) adds 0 to the sum, its index clamped into the box
  const double ax[2] = {ax0, ax1}, ay[2] = {ay0, ay1}, az[2] = {az0, az1};
#pragma unroll
  for (int iz = 0; iz < (DIM == 3 ? 2 : 1); ++iz) {
    const int Z = min(lz + iz, RC.ez - 1);
#pragma unroll
    for (int iy = 0; iy < 2; ++iy) {
      const int Y = min(ly + iy, RC.ey - 1);
      const double wzy = az[iz] * ay[iy];
#pragma unroll
      for (int ix = 0; ix < 2; ++ix) {
        const int X = min(lx + ix, RC.ex - 1);
        const bool off = !fdir && is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z);
        const V wt = off ? (V)0 : (V)(wzy * ax[ix]);
        const int64_t ci = (int64_t)((Z * RC.ey + Y) * RC.ex + X) * NDOF;
#pragma unroll
        for (int a = 0; a < NDOF; ++a) acc[a] += wt * ub[ci + a];
      }
    }
  }
  const int64_t fi = (RF.off + li) * NDOF;
#pragma unroll
  for (int a = 0; a < NDOF; ++a) u[fi + a] += acc[a];
}

// The same prolongation by rows and planes (tiles of make_transfer_tiles): a thread keeps one fine
// node's x and y interpolation (coarse candidates, weights, Dirichlet faces) and walks the tile's
// planes; per plane the block stages the coarse values its rows interpolate from (two coarse
// planes of the few coarse rows bracketing the tile's rows) in LDS with coalesced loads, so each
// is read from memory once per block rather than by every fine node next to it.  Terms, weights and
// their order are k_prolong_add's: the results are the same bit for bit.

template <int DIM, int NDOF, class V>
__global__ __launch_bounds__(kBlock) void k_prolong_rows(LevelView F, LevelView C, const Tile3* __restrict__ tiles,
                                                         const V* __restrict__ ubar, V* __restrict__ u) {
  __shared__ V stage[2][2 * kProlongStageXY * NDOF];  // two buffers of two coarse planes
  const Tile3 T = tiles[xcd_item((int)blockIdx.x, (int)gridDim.x)];
  const RegionGeo RF = F.regs[T.region];
  const RegionGeo RC = C.regs[T.region];
  const int t = threadIdx.x;
  const bool act = t < RF.ex * T.ty;
  const int x = act ? t % RF.ex : 0, y = T.y0 + (act ? t / RF.ex : 0);
  // coarse rows [cy0, cy1] bracket the tile's fine rows (at most three)
  int cy0, cy1;
  {
    double w0, w1;
    bracket(T.y0, RF.ey, RC.ey, cy0, w0, w1);
    bracket(T.y0 + T.ty - 1, RF.ey, RC.ey, cy1, w0, w1);
    cy1 = min(cy1 + 1, RC.ey - 1);
  }
  const int nrow = cy1 - cy0 + 1, nxy = nrow * RC.ex;
  const int nstage = (DIM == 3 ? 2 : 1) * nxy * NDOF;
  int lx, ly;
  double ax[2], ay[2];
  bracket(x, RF.ex, RC.ex, lx, ax[0], ax[1]);
  bracket(y, RF.ey, RC.ey, ly, ay[0], ay[1]);
  const bool fdxy = dir_axis(F.mask, 0, RF.ox + x, F.cx) || dir_axis(F.mask, 2, RF.oy + y, F.cy);
  int sxy[2][2];  // staged position (row - cy0, X) of each candidate
  bool dxy[2][2];
#pragma unroll
  for (int iy = 0; iy < 2; ++iy) {
    const int Y = min(ly + iy, RC.ey - 1);
#pragma unroll
    for (int ix = 0; ix < 2; ++ix) {
      const int X = min(lx + ix, RC.ex - 1);
      sxy[iy][ix] = (Y - cy0) * RC.ex + X;
      dxy[iy][ix] = dir_axis(C.mask, 0, RC.ox + X, C.cx) || dir_axis(C.mask, 2, RC.oy + Y, C.cy);
    }
  }
  const V* __restrict__ ub = ubar + RC.off * NDOF;
  for (int z = T.z0, buf = 0; z < T.z0 + T.nz; ++z, buf ^= 1) {
    int lz = 0;
    double az[2] = {1.0, 0.0};
    if (DIM == 3) bracket(z, RF.ez, RC.ez, lz, az[0], az[1]);
    // stage coarse planes lz and lz + 1 (clamped into the box) of rows cy0 .. cy1: [iz][row][X][dof]
    V* __restrict__ S = stage[buf];
    for (int i = t; i < nstage; i += kBlock) {
      const int iz = i / (nxy * NDOF), rem = i - iz * nxy * NDOF;
      const int Z = min(lz + iz, RC.ez - 1);
      S[i] = ub[((int64_t)Z * RC.ey + cy0) * RC.ex * NDOF + rem];
    }
    __syncthreads();  // staged; the other buffer's readers finished before the previous barrier
    if (act) {
      const bool fdir = fdxy || dir_axis(F.mask, 4, RF.oz + z, F.cz);
      V acc[NDOF];
#pragma unroll
      for (int a = 0; a < NDOF; ++a) acc[a] = (V)0;
#pragma unroll
      for (int iz = 0; iz < (DIM == 3 ? 2 : 1); ++iz) {
        const int Z = min(lz + iz, RC.ez - 1);
        const bool dz = dir_axis(C.mask, 4, RC.oz + Z, C.cz);
#pragma unroll
        for (int iy = 0; iy < 2; ++iy) {
          const double wzy = az[iz] * ay[iy];
#pragma unroll
          for (int ix = 0; ix < 2; ++ix) {
            const bool off = !fdir && (dz || dxy[iy][ix]);
            const V wt = off ? (V)0 : (V)(wzy * ax[ix]);
            const int si = (iz * nxy + sxy[iy][ix]) * NDOF;
#pragma unroll
            for (int a = 0; a < NDOF; ++a) acc[a] += wt * S[si + a];
          }
        }
      }
      const int64_t fi = (RF.off + ((int64_t)z * RF.ey + y) * RF.ex + x) * NDOF;
#pragma unroll
      for (int a = 0; a < NDOF; ++a) u[fi + a] += acc[a];
    }
  }
}

template <int NDOF, class V>
static void prolong_t(const Level& F, const Level& C, const V* ubar, V* u, hipStream_t st) {
  const double* pw = F.pw.as<double>();
  const dim3 g(F.blocks.size()), b(kBlock);
  if constexpr (NDOF == 1) {
    if (pw) {
      RMG_REQUIRE(F.dim == 3, RMG_ERR_ARG, "stored interpolation weights need a 3D level");
      RMG_LAUNCH((k_prolong_add<3, 1, V, true>), g, b, 0, st, F.view(), C.view(), ubar, u, pw);
      LAUNCH_CHECK();
      return;
    }
  }
  if (!F.ptiles.empty()) {
    const dim3 gt(F.ptiles.size());
    if (F.dim == 3)
      RMG_LAUNCH((k_prolong_rows<3, NDOF, V>), gt, b, 0, st, F.view(), C.view(), F.d_ptiles.as<Tile3>(), ubar, u);
    else
      RMG_LAUNCH((k_prolong_rows<2, NDOF, V>), gt, b, 0, st, F.view(), C.view(), F.d_ptiles.as<Tile3>(), ubar, u);
    LAUNCH_CHECK();
    return;
  }
  if (F.dim == 3)
    RMG_LAUNCH((k_prolong_add<3, NDOF, V, false>), g, b, 0, st, F.view(), C.view(), ubar, u, pw);
  else
    RMG_LAUNCH((k_prolong_add<2, NDOF, V, false>), g, b, 0, st, F.view(), C.view(), ubar, u, pw);
  LAUNCH_CHECK();
}

void launch_prolong_add(const Level& F, const Level& C, bool lowp, const void* ubar, void* u, hipStream_t st) {
  if (lowp) {
    if (F.ndof == 3) prolong_t<3, float>(F, C, (const float*)ubar, (float*)u, st);
    else prolong_t<1, float>(F, C, (const float*)ubar, (float*)u, st);
  } else {
    if (F.ndof == 3) prolong_t<3, double>(F, C, (const double*)ubar, (double*)u, st);
    else prolong_t<1, double>(F, C, (const double*)ubar, (double*)u, st);
  }
}

// ------------------------------------------------------------------ RAP
// Per-region Galerkin product [[Abar]] = P^T A^(k) P, one thread per coarse node C:
// Abar(C, C') = sum_{f, s} P(f, C) A(f, f+s) P(f+s, C') over the fine nodes f in the coarse
// intervals on either side of C (at most two fine cells per side) and their stencil neighbours
// f+s, whose coarse intervals give C' within one coarse node of C per axis (the coarse stencil
// keeps 27 points); blocks of NDOF x NDOF coefficients share the scalar weights.  Accumulators
// live in LDS (one column per thread).  Dirichlet reading: a Dirichlet coarse row only collects
// Dirichlet fine nodes; entries of a free row towards Dirichlet coarse nodes are zero.  STORED
// weights come from the fine nodes' records (rate-3 lattice, extents 3^k + 1).
// DIRONLY: only the Dirichlet coarse rows, thread t taking row list[t] (region, index) of nlist.
template <int NPTSF, int DIM, int NDOF, int BS, bool STORED, bool DIRONLY = false>
__global__ __launch_bounds__(BS) void k_rap(LevelView F, LevelView C, const double* __restrict__ coefF,
                                            double* __restrict__ coefC, const double* __restrict__ pw,
                                            const double* __restrict__ rw, const BlockDesc* __restrict__ list = nullptr,
                                            int64_t nlist = 0) {
  constexpr int NC = DIM == 3 ? 27 : 9;
  constexpr int NB = NDOF * NDOF;
  constexpr int SUB = kBlock / BS;
  __shared__ double acc[NC * NB][BS];
  const int tid = threadIdx.x;
#pragma unroll
  for (int o = 0; o < NC * NB; ++o) acc[o][tid] = 0.0;
  BlockDesc bd;
  int li;
  if constexpr (DIRONLY) {
    const int64_t t = (int64_t)blockIdx.x * BS + tid;
    if (t >= nlist) return;  // no block-wide synchronisation below: private LDS columns
    bd = list[t];
    li = bd.start;
  } else {
    bd = C.blocks[blockIdx.x / SUB];
    li = bd.start + (int)(blockIdx.x % SUB) * BS + tid;
  }
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  if (li >= RC.n) return;  // no block-wide synchronisation below: private LDS columns
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const bool cdir = is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z);
  if (DIRONLY && !cdir) return;  // the separable product wrote the free rows
  const int px = coarse_pos(X, RF.ex), py = coarse_pos(Y, RF.ey), pz = DIM == 3 ? coarse_pos(Z, RF.ez) : 0;
  int mxl, mxr, myl, myr, mzl = 0, mzr = 0;
  coarse_spans(X, RF.ex, RC.ex, mxl, mxr);
  coarse_spans(Y, RF.ey, RC.ey, myl, myr);
  if (DIM == 3) coarse_spans(Z, RF.ez, RC.ez, mzl, mzr);
  const int tzlo = DIM == 3 ? -2 : 0, tzhi = DIM == 3 ? 2 : 0;
  for (int tz = tzlo; tz <= tzhi; ++tz) {
    const int fz = pz + tz;
    if ((unsigned)fz >= (unsigned)RF.ez) continue;
    for (int ty = -2; ty <= 2; ++ty) {
      const int fy = py + ty;
      if ((unsigned)fy >= (unsigned)RF.ey) continue;
      for (int tx = -2; tx <= 2; ++tx) {
        const int fx = px + tx;
        if ((unsigned)fx >= (unsigned)RF.ex) continue;
        if (cdir && !is_dirichlet(F, RF.ox + fx, RF.oy + fy, RF.oz + fz)) continue;
        const double wf = STORED ? rw[coef_index(RC.off + li, (tz + 2) * 25 + (ty + 2) * 5 + tx + 2, 125)]
                                 : (DIM == 3 ? tap(tz, mzl, mzr) : 1.0) * tap(ty, myl, myr) * tap(tx, mxl, mxr);
        if (wf == 0.0) continue;
        const int64_t fi = RF.off + (fz * RF.ey + fy) * RF.ex + fx;
#pragma unroll
        for (int s = 0; s < NPTSF; ++s) {
          double a[NB];
          bool any = false;
#pragma unroll
          for (int ab = 0; ab < NB; ++ab) {
            a[ab] = coefF[coef_index(fi, s * NB + ab, NPTSF * NB)];
            any = any || a[ab] != 0.0;
          }
          if (!any) continue;
          int dx, dy, dz;
          stencil_offset<NPTSF>(s, dx, dy, dz);
          const int gx = fx + dx, gy = fy + dy, gz = fz + dz;
          if ((unsigned)gx >= (unsigned)RF.ex || (unsigned)gy >= (unsigned)RF.ey || (unsigned)gz >= (unsigned)RF.ez)
            continue;
          // the coarse interval holding the neighbour, per axis: nodes C + o0, C + o0 + 1 (the
          // neighbour lies within C's two intervals because f does and A couples adjacent nodes)
          int oxl, oyl, ozl = 0;
          double bx[2], by[2], bz[2] = {1.0, 0.0};
          interval_weights(tx + dx, mxl, mxr, oxl, bx[0], bx[1]);
          interval_weights(ty + dy, myl, myr, oyl, by[0], by[1]);
          if (DIM == 3) interval_weights(tz + dz, mzl, mzr, ozl, bz[0], bz[1]);
#pragma unroll
          for (int kz = 0; kz < (DIM == 3 ? 2 : 1); ++kz) {
            const int oz = ozl + kz;
            const double wz = bz[kz];
            if (wz == 0.0) continue;
#pragma unroll
            for (int ky = 0; ky < 2; ++ky) {
              const int oy = oyl + ky;
              const double wy = by[ky];
              if (wy == 0.0) continue;
#pragma unroll
              for (int kx = 0; kx < 2; ++kx) {
                const int ox = oxl + kx;
                const double wx = bx[kx];
                if (wx == 0.0) continue;
                const int oi = DIM == 3 ? (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1) : (oy + 1) * 3 + (ox + 1);
                double wo = wz * wy * wx;
                if constexpr (STORED) {
                  wo = pweight(pw, RF, RC, gx, gy, gz, X + ox, Y + oy, Z + oz);
                  if (wo == 0.0) continue;
                }
#pragma unroll
                for (int ab = 0; ab < NB; ++ab) acc[oi * NB + ab][tid] += (wf * a[ab]) * wo;
              }
            }
          }
        }
      }
    }
  }
  const int64_t gi = RC.off + li;
#pragma unroll
  for (int o = 0; o < NC; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
    const int Xn = X + ox, Yn = Y + oy, Zn = Z + oz;
    const bool inbox = (unsigned)Xn < (unsigned)RC.ex && (unsigned)Yn < (unsigned)RC.ey &&
                       (unsigned)Zn < (unsigned)RC.ez;
    const bool zero = !inbox || (!cdir && is_dirichlet(C, RC.ox + Xn, RC.oy + Yn, RC.oz + Zn));
#pragma unroll
    for (int ab = 0; ab < NB; ++ab)
      coefC[coef_index(gi, o * NB + ab, NC * NB)] = zero ? 0.0 : acc[o * NB + ab][tid];
  }
}

// ---------------------------------------------------- separable Galerkin product
// With the geometric interpolation the prolongator of a 3D region is the tensor product of one
// rate-3 interpolation per axis, P = Px (x) Py (x) Pz, so P^T A P = Qz^T Qy^T (Qx^T A Qx) Qy Qz with
// Qa interpolating along axis a only.  Each factor is a one-axis Galerkin product of a 27-point
// operator, which stays 27-point: along the coarsened axis an output node c sums the fine nodes f in
// its two intervals (weight P(f, c)) and each of their couplings (da, d1, d2) to f + da, split over
// the coarse nodes of f + da's interval (weights P(f + da, c + da')); the two other offsets pass
// through.  Three passes replace the 5 x 5 x 5 window of the generic product: about 400 multiply-adds
// per intermediate node against 27,000 per coarse node.  The passes use the full tensor weights;
// entries of free coarse rows towards Dirichlet coarse nodes are zeroed at the end, and Dirichlet
// coarse rows (which collect only Dirichlet fine nodes) come from the generic product.
template <int AX, bool LAST>
__global__ __launch_bounds__(kBlock) void k_rap_axis(const RegionGeo* __restrict__ gin, const RegionGeo* __restrict__ gout,
                                                     const BlockDesc* __restrict__ blocks, const double* __restrict__ sin_,
                                                     double* __restrict__ sout, LevelView C,
                                                     const double* __restrict__ sym, const double* __restrict__ table,
                                                     const int* __restrict__ served) {
  const BlockDesc bd = blocks[blockIdx.x];
  const RegionGeo RI = gin[bd.region], RO = gout[bd.region];
  // The x pass of a symmetric level takes the couplings its stencil operations apply: the stored
  // upper half and the neighbours' mirrored upper couplings (sym), or, in a region served by its
  // class tables, the same values from the table; otherwise the stored stencils.
  // (the region's table is copied to LDS once per block: every fine node reads 27 of its entries)
  __shared__ double stab[AX == 0 ? kClasses * kClassPts : 1];
  const bool use_tab = AX == 0 && table && served && served[bd.region];
  if (use_tab) {
    const double* __restrict__ tg = table + (int64_t)bd.region * kClasses * kClassPts;
    for (int e = threadIdx.x; e < kClasses * kClassPts; e += kBlock) stab[e] = tg[e];
    __syncthreads();
  }
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RO.n) return;
  int o[3];
  decompose(RO, li, o[0], o[1], o[2]);
  const int ein = AX == 0 ? RI.ex : (AX == 1 ? RI.ey : RI.ez);
  const int eout = AX == 0 ? RO.ex : (AX == 1 ? RO.ey : RO.ez);
  const int c = o[AX];
  bool cdir = false;
  if constexpr (LAST) {
    const RegionGeo RC = C.regs[bd.region];
    cdir = is_dirichlet(C, RC.ox + o[0], RC.oy + o[1], RC.oz + o[2]);
    if (cdir) return;  // Dirichlet coarse rows: the generic product
  }
  const int pos = coarse_pos(c, ein);
  int mL, mR;
  coarse_spans(c, ein, eout, mL, mR);
  double acc[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = 0.0;
  constexpr int kStride = AX == 0 ? 1 : (AX == 1 ? 3 : 9);  // stencil-index step of the coarsened axis
  // The products, with the couplings read by `get(fi, gi, tcb, s)`; each source is its own copy of
  // the loops, so that the loads of one fine node are issued together.
  auto accumulate = [&](auto get) {
#pragma unroll
    for (int t = -2; t <= 2; ++t) {
      const int f = pos + t;
      const double wf = tap(t, mL, mR);
      if ((unsigned)f >= (unsigned)ein || wf == 0.0) continue;
      int fi[3] = {o[0], o[1], o[2]};
      fi[AX] = f;
      const int64_t gi = RI.off + ((int64_t)fi[2] * RI.ey + fi[1]) * RI.ex + fi[0];
      const int tcb =
          use_tab ? ((axis_class(fi[2], RI.ez) * 5 + axis_class(fi[1], RI.ey)) * 5 + axis_class(fi[0], RI.ex)) * kClassPts
                  : 0;
#pragma unroll
      for (int da = -1; da <= 1; ++da) {
        if ((unsigned)(f + da) >= (unsigned)ein) continue;
        int o0;
        double w0, w1;
        interval_weights(t + da, mL, mR, o0, w0, w1);
#pragma unroll
        for (int q = 0; q < 9; ++q) {  // the two other offsets
          const int d1 = q % 3, d2 = q / 3;  // 0..2
          int sbase;
          if constexpr (AX == 0) sbase = d2 * 9 + d1 * 3;
          else if constexpr (AX == 1) sbase = d2 * 9 + d1;
          else sbase = d2 * 3 + d1;
          const double wa = wf * get(fi, gi, tcb, sbase + (da + 1) * kStride);
          acc[sbase + (o0 + 1) * kStride] += wa * w0;
          if (o0 + 2 <= 2) acc[sbase + (o0 + 2) * kStride] += wa * w1;
        }
      }
    }
  };
  if (use_tab) {
    accumulate([&](const int*, int64_t, int tcb, int sidx) { return stab[tcb + sidx]; });
  } else if (AX == 0 && sym) {
    accumulate([&](const int* fi, int64_t gi, int, int sidx) {
      if (sidx >= 13) return sym[coef_index(gi, sidx - 13, kSymPts)];
      // the neighbour's upper coupling towards this node, 0 outside the region
      int dx, dy, dz;
      stencil_offset<27>(sidx, dx, dy, dz);
      const bool in = (unsigned)(fi[0] + dx) < (unsigned)RI.ex && (unsigned)(fi[1] + dy) < (unsigned)RI.ey &&
                      (unsigned)(fi[2] + dz) < (unsigned)RI.ez;
      return in ? sym[coef_index(gi + dx + (int64_t)dy * RI.ex + (int64_t)dz * RI.ex * RI.ey, 13 - sidx, kSymPts)]
                : 0.0;
    });
  } else {
    accumulate([&](const int*, int64_t gi, int, int sidx) { return sin_[coef_index(gi, sidx, 27)]; });
  }
  const int64_t go = RO.off + li;
  if constexpr (LAST) {
    const RegionGeo RC = C.regs[bd.region];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int X = o[0] + q % 3 - 1, Y = o[1] + (q / 3) % 3 - 1, Z = o[2] + q / 9 - 1;
      const bool inbox = (unsigned)X < (unsigned)RO.ex && (unsigned)Y < (unsigned)RO.ey && (unsigned)Z < (unsigned)RO.ez;
      const bool zero = !inbox || is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z);
      sout[coef_index(go, q, 27)] = zero ? 0.0 : acc[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 27; ++q) sout[coef_index(go, q, 27)] = acc[q];
  }
}

// Separable product for a scalar 3D level with geometric interpolation: passes x, y, z through two
// intermediate grids (coarse along x; coarse along x and y), then the Dirichlet coarse rows.
static void launch_rap_separable(const Level& F, Level& C, hipStream_t st) {
  std::vector<RegionGeo> g1(F.regs), g2(F.regs);
  std::vector<BlockDesc> b1, b2;
  int64_t n1 = 0, n2 = 0;
  for (int k = 0; k < F.nreg; ++k) {
    g1[k].ex = C.regs[k].ex;
    g2[k].ex = C.regs[k].ex;
    g2[k].ey = C.regs[k].ey;
    for (RegionGeo* g : {&g1[k], &g2[k]}) g->n = g->ex * g->ey * g->ez;
    g1[k].off = n1;
    g2[k].off = n2;
    for (int s0 = 0; s0 < g1[k].n; s0 += kBlock) b1.push_back(BlockDesc{k, s0});
    for (int s0 = 0; s0 < g2[k].n; s0 += kBlock) b2.push_back(BlockDesc{k, s0});
    n1 += g1[k].n;
    n2 += g2[k].n;
  }
  DBuf dg1, dg2, db1, db2, s1, s2;
  dg1.alloc(sizeof(RegionGeo) * g1.size());
  dg2.alloc(sizeof(RegionGeo) * g2.size());
  db1.alloc(sizeof(BlockDesc) * b1.size());
  db2.alloc(sizeof(BlockDesc) * b2.size());
  RMG_HIP(hipMemcpyAsync(dg1.p, g1.data(), dg1.bytes, hipMemcpyHostToDevice, st));
  RMG_HIP(hipMemcpyAsync(dg2.p, g2.data(), dg2.bytes, hipMemcpyHostToDevice, st));
  RMG_HIP(hipMemcpyAsync(db1.p, b1.data(), db1.bytes, hipMemcpyHostToDevice, st));
  RMG_HIP(hipMemcpyAsync(db2.p, b2.data(), db2.bytes, hipMemcpyHostToDevice, st));
  s1.alloc(sizeof(double) * coef_elems(n1, 27));
  s2.alloc(sizeof(double) * coef_elems(n2, 27));
  const LevelView cv = C.view();
  const bool tables = F.class_table.p && F.class_table_ok.p;
  RMG_LAUNCH((k_rap_axis<0, false>), dim3(b1.size()), dim3(kBlock), 0, st, F.d_regs.as<RegionGeo>(),
             dg1.as<RegionGeo>(), db1.as<BlockDesc>(), F.coef.as<double>(), s1.as<double>(), cv,
             F.coef_sym.as<double>(), tables ? F.class_table.as<double>() : nullptr,
             tables ? F.class_table_ok.as<int>() : nullptr);
  RMG_LAUNCH((k_rap_axis<1, false>), dim3(b2.size()), dim3(kBlock), 0, st, dg1.as<RegionGeo>(),
             dg2.as<RegionGeo>(), db2.as<BlockDesc>(), s1.as<double>(), s2.as<double>(), cv, nullptr, nullptr,
             nullptr);
  RMG_LAUNCH((k_rap_axis<2, true>), dim3(C.blocks.size()), dim3(kBlock), 0, st, dg2.as<RegionGeo>(),
             C.d_regs.as<RegionGeo>(), C.d_blocks.as<BlockDesc>(), s2.as<double>(), C.coef.as<double>(), cv, nullptr,
             nullptr, nullptr);
  LAUNCH_CHECK();
  // Dirichlet coarse rows, one thread each from the list of them (rows or planes on a Dirichlet
  // face entirely, else the two end nodes of the row)
  std::vector<BlockDesc> drows;
  const unsigned m = C.mask;
  auto dir = [&](int g, int n, unsigned lo, unsigned hi) { return ((m & lo) && g == 0) || ((m & hi) && g == n - 1); };
  for (int k = 0; k < C.nreg; ++k) {
    const RegionGeo& R = C.regs[k];
    for (int z = 0; z < R.ez; ++z)
      for (int y = 0; y < R.ey; ++y) {
        const bool whole = dir(R.oz + z, C.comp[2], 16u, 32u) || dir(R.oy + y, C.comp[1], 4u, 8u);
        for (int x = 0; x < R.ex; x = (whole || x + 1 == R.ex || R.ex < 2) ? x + 1 : R.ex - 1)
          if (whole || dir(R.ox + x, C.comp[0], 1u, 2u)) drows.push_back(BlockDesc{k, (z * R.ey + y) * R.ex + x});
      }
  }
  if (!drows.empty()) {
    DBuf dl;
    dl.alloc(sizeof(BlockDesc) * drows.size());
    RMG_HIP(hipMemcpyAsync(dl.p, drows.data(), dl.bytes, hipMemcpyHostToDevice, st));
    RMG_LAUNCH((k_rap<27, 3, 1, kBlock, false, true>), dim3(cdiv((int64_t)drows.size(), kBlock)), dim3(kBlock), 0, st,
               F.view(), cv, F.coef.as<double>(), C.coef.as<double>(), nullptr, nullptr, dl.as<BlockDesc>(),
               (int64_t)drows.size());
    LAUNCH_CHECK();
    RMG_HIP(hipStreamSynchronize(st));  // before the list is released
  }
  // the intermediates are freed when this returns: wait for the passes that read them
  RMG_HIP(hipStreamSynchronize(st));
}

void launch_rap(const Level& F, Level& C, hipStream_t st) {
  const LevelView fv = F.view(), cv = C.view();
  const double* cf = F.coef.as<double>();
  double* cc = C.coef.as<double>();
  const double* pw = F.pw.as<double>();
  const double* rw = F.rw.as<double>();
  RMG_REQUIRE(!pw || (F.dim == 3 && F.ndof == 1 && rw), RMG_ERR_ARG,
              "stored interpolation weights need a scalar 3D level");
  if (F.ndof == 3) {
    RMG_REQUIRE(F.npts == 27, RMG_ERR_ARG, "3D levels need 27-point stencils");
    constexpr int BS = 32;
    RMG_LAUNCH((k_rap<27, 3, 3, BS, false>), dim3(C.blocks.size() * (kBlock / BS)), dim3(BS), 0, st, fv, cv,
                       cf, cc, pw, rw);
  } else if (F.dim == 3 && !pw && F.rap_separable) {
    RMG_REQUIRE(F.npts == 27, RMG_ERR_ARG, "3D levels need 27-point stencils");
    launch_rap_separable(F, C, st);
    return;
  } else if (F.dim == 3) {
    RMG_REQUIRE(F.npts == 27, RMG_ERR_ARG, "3D levels need 27-point stencils");
    if (pw)
      RMG_LAUNCH((k_rap<27, 3, 1, kBlock, true>), dim3(C.blocks.size()), dim3(kBlock), 0, st, fv, cv, cf, cc,
                         pw, rw);
    else
      RMG_LAUNCH((k_rap<27, 3, 1, kBlock, false>), dim3(C.blocks.size()), dim3(kBlock), 0, st, fv, cv, cf, cc,
                         pw, rw);
  } else if (F.npts == 9) {
    RMG_LAUNCH((k_rap<9, 2, 1, kBlock, false>), dim3(C.blocks.size()), dim3(kBlock), 0, st, fv, cv, cf, cc, pw,
                       rw);
  } else {
    RMG_LAUNCH((k_rap<5, 2, 1, kBlock, false>), dim3(C.blocks.size()), dim3(kBlock), 0, st, fv, cv, cf, cc, pw,
                       rw);
  }
  LAUNCH_CHECK();
}

// ------------------------------------------------- composite <-> regional
template <class V>
__global__ __launch_bounds__(kBlock) void k_to_regional(LevelView L, const double* __restrict__ comp,
                                                        V* __restrict__ reg) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int64_t ci = comp_index(L, R.ox + x, R.oy + y, R.oz + z) * L.ndof;
  for (int a = 0; a < L.ndof; ++a) reg[(R.off + li) * L.ndof + a] = (V)comp[ci + a];
}

void launch_to_regional(const Level& L, const double* comp, double* reg, hipStream_t st) {
  RMG_LAUNCH(k_to_regional<double>, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), comp, reg);
  LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_to_composite_nodes(LevelView L, const double* __restrict__ reg,
                                                               double* __restrict__ comp) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  if (is_shared(L, R, x, y, z)) return;
  const int64_t ci = comp_index(L, R.ox + x, R.oy + y, R.oz + z) * L.ndof;
  for (int a = 0; a < L.ndof; ++a) comp[ci + a] = reg[(R.off + li) * L.ndof + a];
}

__global__ __launch_bounds__(kBlock) void k_to_composite_groups(const int64_t* __restrict__ gptr,
                                                                const int* __restrict__ gcopy,
                                                                const int* __restrict__ gcomp, int64_t ng, int ndof,
                                                                const double* __restrict__ reg,
                                                                double* __restrict__ comp, int average) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t a0 = gptr[g], e = gptr[g + 1];
  for (int a = 0; a < ndof; ++a) {
    double v;
    if (average) {
      double s = 0.0;
      for (int64_t c = a0; c < e; ++c) s += reg[(int64_t)gcopy[c] * ndof + a];
      v = s / (double)(e - a0);
    } else {
      v = reg[(int64_t)gcopy[a0] * ndof + a];
    }
    comp[(int64_t)gcomp[g] * ndof + a] = v;
  }
}

void launch_to_composite(const Level& L, const double* reg, double* comp, int average, hipStream_t st) {
  RMG_LAUNCH(k_to_composite_nodes, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), reg, comp);
  LAUNCH_CHECK();
  if (L.ngroups > 0) {
    RMG_LAUNCH(k_to_composite_groups, dim3(cdiv(L.ngroups, kBlock)), dim3(kBlock), 0, st,
                       L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(), L.d_gcomp.as<int>(), L.ngroups, L.ndof, reg,
                       comp, average);
    LAUNCH_CHECK();
  }
}

// ------------------------------------------------------- coarse solve
template <class V>
__global__ void k_gather(int ncnode, int ndof, const int* __restrict__ owner, const V* __restrict__ reg,
                         double* __restrict__ c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncnode * ndof) return;
  const int i = t / ndof, a = t - i * ndof;
  c[t] = (double)reg[(int64_t)owner[i] * ndof + a];
}

// y = A x, A row-major n x n; one wavefront per row.
__global__ __launch_bounds__(256) void k_gemv(int n, const double* __restrict__ A, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* __restrict__ a = A + (int64_t)row * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * x[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[row] = s;
}

void launch_dense_gemv(int n, const double* A, const double* x, double* y, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_gemv, dim3(cdiv(n, 4)), dim3(256), 0, st, n, A, x, y);
  LAUNCH_CHECK();
}

void launch_coarse_gather(const Level& L, bool lowp, const void* b, hipStream_t st) {
  const int n = L.nc;
  const int ncnode = (int)L.ncomp;
  if (lowp)
    RMG_LAUNCH(k_gather<float>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, ncnode, L.ndof,
                       L.comp_owner.as<int>(), (const float*)b, L.cvec.as<double>());
  else
    RMG_LAUNCH(k_gather<double>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, ncnode, L.ndof,
                       L.comp_owner.as<int>(), (const double*)b, L.cvec.as<double>());
  LAUNCH_CHECK();
}

void launch_coarse_scatter(const Level& L, bool lowp, void* u, hipStream_t st) {
  if (lowp)
    RMG_LAUNCH(k_to_regional<float>, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(),
                       L.cvec2.as<double>(), (float*)u);
  else
    RMG_LAUNCH(k_to_regional<double>, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(),
                       L.cvec2.as<double>(), (double*)u);
  LAUNCH_CHECK();
}

void launch_coarse_solve(const Level& L, bool lowp, const void* b, void* u, hipStream_t st) {
  launch_coarse_gather(L, lowp, b, st);
  const int n = L.nc;
  RMG_LAUNCH(k_gemv, dim3(cdiv(n, 4)), dim3(256), 0, st, n, L.ainv.as<double>(), L.cvec.as<double>(),
                     L.cvec2.as<double>());
  LAUNCH_CHECK();
  launch_coarse_scatter(L, lowp, u, st);
}

// ------------------------------------------ coarse inverse: blocked Gauss-Jordan (SPD, in place)
// For a pivot panel P = [k0, k0 + nb) and the other indices R, one block step maps
//   A_PP -> X = A_PP^-1,  A_PR -> X A_PR,  A_RP -> -A_RP X,  A_RR -> A_RR - A_RP X A_PR,
// the block form of the scalar Gauss-Jordan step (no pivoting: every pivot block of an SPD matrix
// is SPD).  Four launches per panel: the panel inverse in LDS, T = A_RP X and W = X A_PR
// (stored nb x n), the rank-nb update of A_RR as a tiled GEMM, and the panel rows and columns.
constexpr int kGjB = 64;  // panel width

// The panel inverse: one 1024-thread block, lane j = column, 16 row groups of 4 rows each; per
// pivot k every thread reads the pivot row and column and its own entries from one LDS copy of
// the panel and writes the updated entries to the other (one barrier per pivot), the reciprocal
// of the pivot taken once.
constexpr int kGjPanelThreads = 1024;

__global__ __launch_bounds__(kGjPanelThreads) void k_gj_panel(int n, int k0, int nb, const double* __restrict__ A,
                                                              double* __restrict__ X) {
  constexpr int kRows = kGjPanelThreads / kGjB;  // row groups
  constexpr int kPer = kGjB / kRows;             // rows per thread
  __shared__ double s[2][kGjB][kGjB + 1];
  const int j = threadIdx.x % kGjB, i0 = threadIdx.x / kGjB;
  for (int i = i0; i < nb; i += kRows)
    if (j < nb) s[0][i][j] = A[(int64_t)(k0 + i) * n + k0 + j];
  __syncthreads();
  int cur = 0;
  for (int k = 0; k < nb; ++k) {
    const double rp = 1.0 / s[cur][k][k];
    if (j < nb) {
      const double rowk = s[cur][k][j];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const int i = i0 + kRows * r;
        if (i >= nb) continue;
        const double colk = s[cur][i][k];
        double v;
        if (i == k && j == k) v = rp;
        else if (i == k) v = rowk * rp;
        else if (j == k) v = -colk * rp;
        else v = s[cur][i][j] - colk * (rowk * rp);
        s[cur ^ 1][i][j] = v;
      }
    }
    cur ^= 1;
    __syncthreads();
  }
  for (int i = i0; i < nb; i += kRows)
    if (j < nb) X[i * kGjB + j] = s[cur][i][j];
}

// TT[q][i] = sum_p A[i][k0+p] X[p][q] (T transposed) and W[p][j] = sum_q X[p][q] A[k0+q][j], one
// thread per index i (= j) and per chunk of kGjChunk outputs q (p) (blockIdx.y), X in LDS.  Rows
// and columns inside the panel are computed but unused.
constexpr int kGjChunk = 8;

__global__ __launch_bounds__(kBlock) void k_gj_tw(int n, int k0, int nb, const double* __restrict__ A,
                                                  const double* __restrict__ X, double* __restrict__ TT,
                                                  double* __restrict__ W) {
  __shared__ double sx[kGjB][kGjB];  // X, zero outside nb x nb
  for (int e = threadIdx.x; e < kGjB * kGjB; e += kBlock) {
    const int r = e / kGjB, c = e % kGjB;
    sx[r][c] = (r < nb && c < nb) ? X[e] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  // fixed trip counts keep a[] in registers; entries beyond nb are zero
  double a[kGjB];
#pragma unroll
  for (int p = 0; p < kGjB; ++p) a[p] = p < nb ? A[(int64_t)i * n + k0 + p] : 0.0;  // row i, panel columns
  const int c0 = blockIdx.y * kGjChunk, c1 = min(nb, c0 + kGjChunk);
  for (int q = c0; q < c1; ++q) {
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < kGjB; ++p) t += a[p] * sx[p][q];
    TT[(int64_t)q * n + i] = t;
  }
#pragma unroll
  for (int q = 0; q < kGjB; ++q) a[q] = q < nb ? A[(int64_t)(k0 + q) * n + i] : 0.0;  // column i, panel rows
  for (int p = c0; p < c1; ++p) {
    double w = 0.0;
#pragma unroll
    for (int q = 0; q < kGjB; ++q) w += sx[p][q] * a[q];
    W[(int64_t)p * n + i] = w;
  }
}

// A_RR -= T A_PR over 64 x 64 output tiles: T and the panel rows staged in LDS, 4 x 4 outputs per
// thread (consecutive lanes own consecutive columns, so A is read and written coalesced).
__global__ __launch_bounds__(kBlock) void k_gj_rank(int n, int k0, int nb, double* __restrict__ A,
                                                    const double* __restrict__ TT) {
  const int bi = blockIdx.y * 64, bj = blockIdx.x * 64;
  const bool rows_in_panel = bi >= k0 && bi + 64 <= k0 + nb, cols_in_panel = bj >= k0 && bj + 64 <= k0 + nb;
  if (rows_in_panel || cols_in_panel) return;  // uniform over the block
  __shared__ double sT[kGjB][64];  // [q][row]
  __shared__ double sB[kGjB][64];  // [q][col]
  for (int e = threadIdx.x; e < nb * 64; e += kBlock) {
    const int q = e / 64, c = e - q * 64;
    sT[q][c] = bi + c < n ? TT[(int64_t)q * n + bi + c] : 0.0;
    sB[q][c] = bj + c < n ? A[(int64_t)(k0 + q) * n + bj + c] : 0.0;
  }
  __syncthreads();
  const int tj = threadIdx.x % 16, ti = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int q = 0; q < nb; ++q) {
    double t[4], v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) t[a] = sT[q][ti + 16 * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) v[b] = sB[q][tj + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += t[a] * v[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = bi + ti + 16 * a;
    if (i >= n || (i >= k0 && i < k0 + nb)) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = bj + tj + 16 * b;
      if (j >= n || (j >= k0 && j < k0 + nb)) continue;
      A[(int64_t)i * n + j] -= acc[a][b];
    }
  }
}

// Panel rows A[k0+p][j] = W[p][j] (j outside the panel) and the pivot block = X; one thread per
// (p, j), consecutive lanes on consecutive columns.
__global__ __launch_bounds__(kBlock) void k_gj_rows(int n, int k0, int nb, double* __restrict__ A,
                                                    const double* __restrict__ W, const double* __restrict__ X) {
  const int j = blockIdx.x * kBlock + threadIdx.x, p = blockIdx.y;
  if (j >= n) return;
  A[(int64_t)(k0 + p) * n + j] = (j >= k0 && j < k0 + nb) ? X[p * kGjB + (j - k0)] : W[(int64_t)p * n + j];
}

// Panel columns A[i][k0+q] = -T[i][q] (i outside the panel); one wavefront per row, lane q.
__global__ __launch_bounds__(kBlock) void k_gj_cols(int n, int k0, int nb, double* __restrict__ A,
                                                    const double* __restrict__ TT) {
  const int q = threadIdx.x & 63;
  const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (i >= n || q >= nb || (i >= k0 && i < k0 + nb)) return;
  A[(int64_t)i * n + k0 + q] = -TT[(int64_t)q * n + i];
}

void launch_gauss_jordan(double* A, int n, hipStream_t st) {
  if (n == 0) return;
  DBuf X, TT, W;
  X.alloc(sizeof(double) * kGjB * kGjB);
  TT.alloc(sizeof(double) * kGjB * (size_t)n);
  W.alloc(sizeof(double) * kGjB * (size_t)n);
  const int nt = (int)cdiv(n, 64);
  for (int k0 = 0; k0 < n; k0 += kGjB) {
    const int nb = std::min(kGjB, n - k0);
    RMG_LAUNCH(k_gj_panel, dim3(1), dim3(kGjPanelThreads), 0, st, n, k0, nb, A, X.as<double>());
    RMG_LAUNCH(k_gj_tw, dim3(cdiv(n, kBlock), cdiv(nb, kGjChunk)), dim3(kBlock), 0, st, n, k0, nb, A, X.as<double>(),
                       TT.as<double>(), W.as<double>());
    RMG_LAUNCH(k_gj_rank, dim3(nt, nt), dim3(kBlock), 0, st, n, k0, nb, A, TT.as<double>());
    RMG_LAUNCH(k_gj_rows, dim3(cdiv(n, kBlock), nb), dim3(kBlock), 0, st, n, k0, nb, A, W.as<double>(),
                       X.as<double>());
    RMG_LAUNCH(k_gj_cols, dim3(cdiv(n, kBlock / 64)), dim3(kBlock), 0, st, n, k0, nb, A, TT.as<double>());
  }
  LAUNCH_CHECK();
  RMG_HIP(hipStreamSynchronize(st));  // before the work buffers are released
}

__global__ void k_check_inverse(int n, const double* __restrict__ A, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = A[(int64_t)i * n + i];
  if (!(d > 0.0) || !isfinite(d)) atomicOr(flag, 1);
}

void launch_check_inverse(const double* A, int n, int* flag, hipStream_t st) {
  RMG_LAUNCH(k_check_inverse, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, A, flag);
  LAUNCH_CHECK();
}

// --------------------------------------------------------- Q1 assembly
struct Kmat {
  double k[64];
};

// One thread per node: sums the element matrices of the (up to 8) elements of its region
// that contain it; Dirichlet rows become identity rows and couplings to Dirichlet nodes are
// removed (symmetric elimination).  Element e's coefficient is elem_coef[e] or 1.
__global__ __launch_bounds__(kBlock) void k_assemble_q1(LevelView L, Kmat K, const double* __restrict__ ecoef,
                                                        double* __restrict__ coef) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  double acc[27];
#pragma unroll
  for (int s = 0; s < 27; ++s) acc[s] = 0.0;
  // element with lowest corner at node - a, node is its corner a
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const int exl = x - ax, eyl = y - ay, ezl = z - az;
    if (exl < 0 || eyl < 0 || ezl < 0 || exl > R.ex - 2 || eyl > R.ey - 2 || ezl > R.ez - 2) continue;
    double c = 1.0;
    if (ecoef) {
      const int64_t e = ((int64_t)(R.oz + ezl) * (L.cy - 1) + (R.oy + eyl)) * (L.cx - 1) + (R.ox + exl);
      c = ecoef[e];
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
      const int s = (bz - az + 1) * 9 + (by - ay + 1) * 3 + (bx - ax + 1);
      acc[s] += K.k[a * 8 + b] * c;
    }
  }
  const int64_t gi = R.off + li;
  const bool dn = is_dirichlet(L, gx, gy, gz);
#pragma unroll
  for (int s = 0; s < 27; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    double v = acc[s];
    const bool inbox = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                       (unsigned)(z + dz) < (unsigned)R.ez;
    if (!inbox) v = 0.0;
    if (dn) v = (s == 13) ? 1.0 : 0.0;
    else if (inbox && is_dirichlet(L, gx + dx, gy + dy, gz + dz)) v = 0.0;
    coef[coef_index(gi, s, 27)] = v;
  }
}

void launch_assemble_q1_scalar(const Level& L, const double* Kref, const double* elem_coef, hipStream_t st) {
  Kmat K;
  for (int i = 0; i < 64; ++i) K.k[i] = Kref[i];
  RMG_LAUNCH(k_assemble_q1, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), K, elem_coef,
                     L.coef.as<double>());
  LAUNCH_CHECK();
}

// Q1 isotropic elasticity, 3 dofs per node: one thread per node sums, for each of the 27
// neighbour offsets, the 3x3 blocks of the (up to 8) elements of its region that contain both
// nodes; Dirichlet nodes (all three components) become identity rows and couplings to them are
// removed.  K is the 24x24 element matrix for E = 1 (dof 3a+i = component i of corner a).
__global__ __launch_bounds__(kBlock) void k_assemble_q1_elast(LevelView L, const double* __restrict__ K,
                                                              const double* __restrict__ youngs,
                                                              double* __restrict__ coef) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  const double E = youngs[bd.region];
  const int64_t gi = R.off + li;
  const bool dn = is_dirichlet(L, gx, gy, gz);
#pragma unroll 1
  for (int s = 0; s < 27; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const int bx = ax + dx, by = ay + dy, bz = az + dz;
      if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
      const int exl = x - ax, eyl = y - ay, ezl = z - az;
      if (exl < 0 || eyl < 0 || ezl < 0 || exl > R.ex - 2 || eyl > R.ey - 2 || ezl > R.ez - 2) continue;
      const int b = bx + 2 * by + 4 * bz;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i * 3 + j] += E * K[(3 * a + i) * 24 + 3 * b + j];
    }
    const bool inbox = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                       (unsigned)(z + dz) < (unsigned)R.ez;
    const bool nbdir = inbox && is_dirichlet(L, gx + dx, gy + dy, gz + dz);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double v = acc[k];
      if (!inbox) v = 0.0;
      if (dn) v = (s == 13 && (k == 0 || k == 4 || k == 8)) ? 1.0 : 0.0;
      else if (nbdir) v = 0.0;
      coef[coef_index(gi, s * 9 + k, 243)] = v;
    }
  }
}

void launch_assemble_q1_elasticity(const Level& L, const double* Kdev, const double* youngs_dev, hipStream_t st) {
  RMG_LAUNCH(k_assemble_q1_elast, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), Kdev, youngs_dev,
                     L.coef.as<double>());
  LAUNCH_CHECK();
}

// Dirichlet rows of shared nodes: the identity is split 1/m over the m copies.
__global__ void k_dirichlet_split(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                  const int* __restrict__ gcomp, int64_t ng, LevelView L, int center,
                                  double* coef) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t ci = gcomp[g];
  const int gx = (int)(ci % L.cx), gy = (int)((ci / L.cx) % L.cy), gz = (int)(ci / ((int64_t)L.cx * L.cy));
  if (!is_dirichlet(L, gx, gy, gz)) return;
  const int64_t a0 = gptr[g], e = gptr[g + 1];
  const int nd = L.ndof, ncoef = L.npts * nd * nd;
  for (int64_t c = a0; c < e; ++c)
    for (int a = 0; a < nd; ++a)
      coef[coef_index(gcopy[c], center * nd * nd + a * nd + a, ncoef)] = 1.0 / (double)(e - a0);
}

void launch_dirichlet_split(const Level& L, hipStream_t st) {
  if (L.ngroups == 0) return;
  const int center = L.npts == 27 ? 13 : (L.npts == 9 ? 4 : 2);
  RMG_LAUNCH(k_dirichlet_split, dim3(cdiv(L.ngroups, kBlock)), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                     L.d_gcopy.as<int>(), L.d_gcomp.as<int>(), L.ngroups, L.view(), center, L.coef.as<double>());
  LAUNCH_CHECK();
}

template <int NPTS>
__global__ __launch_bounds__(kBlock) void k_mask_stencil(LevelView L, double* __restrict__ coef, int* flag) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int64_t gi = R.off + li;
  const int nb = L.ndof * L.ndof, ncoef = NPTS * nb;
  bool bad = false;
#pragma unroll
  for (int s = 0; s < NPTS; ++s) {
    int dx, dy, dz;
    stencil_offset<NPTS>(s, dx, dy, dz);
    const bool ok = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                    (unsigned)(z + dz) < (unsigned)R.ez;
    for (int ab = 0; ab < nb; ++ab) {
      double* c = coef + coef_index(gi, s * nb + ab, ncoef);
      if (!isfinite(*c)) bad = true;
      if (!ok) *c = 0.0;
    }
  }
  if (bad) atomicOr(flag, 1);
}

void launch_mask_stencil(const Level& L, int* flag, hipStream_t st) {
  const dim3 g(L.blocks.size());
  if (L.npts == 27) RMG_LAUNCH(k_mask_stencil<27>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  else if (L.npts == 9) RMG_LAUNCH(k_mask_stencil<9>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  else RMG_LAUNCH(k_mask_stencil<5>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  LAUNCH_CHECK();
}

// ------------------------------------------------- non-invasive split
template <int NPTS>
__global__ __launch_bounds__(kBlock) void k_split_composite(LevelView L, const double* __restrict__ comp,
                                                            int64_t ncomp, double* __restrict__ coef,
                                                            int* flag) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  const int mx = ((x == 0 && gx != 0) || (x == R.ex - 1 && gx != L.cx - 1)) ? 2 : 1;
  const int my = ((y == 0 && gy != 0) || (y == R.ey - 1 && gy != L.cy - 1)) ? 2 : 1;
  const int mz = ((z == 0 && gz != 0) || (z == R.ez - 1 && gz != L.cz - 1)) ? 2 : 1;
  const int64_t ci = comp_index(L, gx, gy, gz);
  const int64_t gi = R.off + li;
  constexpr int c = center_index<NPTS>();
  double rowsum = 0.0, offsum = 0.0;
  bool bad = false;
#pragma unroll
  for (int s = 0; s < NPTS; ++s) {
    int dx, dy, dz;
    stencil_offset<NPTS>(s, dx, dy, dz);
    const double a = comp[(int64_t)s * ncomp + ci];
    if (!isfinite(a)) bad = true;
    const bool indom = (unsigned)(gx + dx) < (unsigned)L.cx && (unsigned)(gy + dy) < (unsigned)L.cy &&
                       (unsigned)(gz + dz) < (unsigned)L.cz;
    if (indom) rowsum += a;
    if (s == c) continue;
    const bool inbox = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                       (unsigned)(z + dz) < (unsigned)R.ez;
    double v = 0.0;
    if (inbox) {
      const int q = (dx == 0 ? mx : 1) * (dy == 0 ? my : 1) * (dz == 0 ? mz : 1);
      v = a / (double)q;
      offsum += v;
    }
    coef[coef_index(gi, s, NPTS)] = v;
  }
  coef[coef_index(gi, c, NPTS)] = rowsum / (double)(mx * my * mz) - offsum;
  if (bad) atomicOr(flag, 1);
}

void launch_split_composite(const Level& L, const double* comp, int* flag, hipStream_t st) {
  const dim3 g(L.blocks.size());
  if (L.npts == 27)
    RMG_LAUNCH(k_split_composite<27>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  else if (L.npts == 9)
    RMG_LAUNCH(k_split_composite<9>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  else
    RMG_LAUNCH(k_split_composite<5>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  LAUNCH_CHECK();
}

// Assembled composite CSR matrix (rows and columns = composite nodes, x fastest) -> composite
// stencil [npts][ncomp] (zero-initialised by the caller), one thread per row; duplicate entries add
// up.  Flags: 1 a non-finite value, 2 an entry outside the stencil's neighbourhood, 4 a column
// index out of range (such entries are skipped).
template <int NPTS>
__global__ __launch_bounds__(kBlock) void k_csr_to_stencil(int cx, int cy, int cz, const int64_t* __restrict__ rowptr,
                                                           const int* __restrict__ colind,
                                                           const double* __restrict__ vals, double* __restrict__ comp,
                                                           int* flag) {
  const int64_t n = (int64_t)cx * cy * cz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gx = (int)(i % cx), gy = (int)((i / cx) % cy), gz = (int)(i / ((int64_t)cx * cy));
  int f = 0;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int j = colind[e];
    if (j < 0 || (int64_t)j >= n) {
      f |= 4;
      continue;
    }
    const int dx = j % cx - gx, dy = (j / cx) % cy - gy, dz = (int)(j / ((int64_t)cx * cy)) - gz;
    int s = -1;
    if (NPTS == 27 && abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) s = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1;
    if (NPTS == 9 && abs(dx) <= 1 && abs(dy) <= 1 && dz == 0) s = (dy + 1) * 3 + dx + 1;
    if (NPTS == 5 && dz == 0 && abs(dx) + abs(dy) <= 1) s = dy == -1 ? 0 : (dx == -1 ? 1 : (dx == 1 ? 3 : (dy == 1 ? 4 : 2)));
    if (s < 0) {
      f |= 2;
      continue;
    }
    const double v = vals[e];
    if (!isfinite(v)) f |= 1;
    comp[(int64_t)s * n + i] += v;
  }
  if (f) atomicOr(flag, f);
}

void launch_csr_to_stencil(const Level& L, const int64_t* rowptr, const int* colind, const double* vals,
                           double* comp, int* flag, hipStream_t st) {
  const dim3 g(cdiv(L.ncomp, kBlock)), b(kBlock);
  if (L.npts == 27)
    RMG_LAUNCH(k_csr_to_stencil<27>, g, b, 0, st, L.comp[0], L.comp[1], L.comp[2], rowptr, colind, vals, comp,
                       flag);
  else if (L.npts == 9)
    RMG_LAUNCH(k_csr_to_stencil<9>, g, b, 0, st, L.comp[0], L.comp[1], L.comp[2], rowptr, colind, vals, comp,
                       flag);
  else
    RMG_LAUNCH(k_csr_to_stencil<5>, g, b, 0, st, L.comp[0], L.comp[1], L.comp[2], rowptr, colind, vals, comp,
                       flag);
  LAUNCH_CHECK();
}

// Caller layout (structure of arrays over one region, [ncoef][nodes]) <-> wave-tiled storage.
__global__ void k_region_stencil_io(int64_t off, int nn, int ncoef, double* __restrict__ coef,
                                    double* __restrict__ soa, int to_level) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nn * ncoef) return;
  const int s = (int)(t / nn);
  const int i = (int)(t - (int64_t)s * nn);
  double* c = coef + coef_index(off + i, s, ncoef);
  if (to_level) *c = soa[t];
  else soa[t] = *c;
}

void launch_region_stencil_io(const Level& L, int region, double* soa, int to_level, hipStream_t st) {
  const RegionGeo& R = L.regs[region];
  const int64_t tot = (int64_t)R.n * L.ncoef();
  RMG_LAUNCH(k_region_stencil_io, dim3(cdiv(tot, kBlock)), dim3(kBlock), 0, st, R.off, R.n, L.ncoef(),
                     L.coef.as<double>(), soa, to_level);
  LAUNCH_CHECK();
}

// ------------------------------------------------- low-precision operator
// FP32: every coefficient rounded to float.  BF16: every coefficient rounded to bfloat16, plus
// an FP32 copy of the centre block whose diagonal entry of each dof row is set so that the row
// sum of the stored low-precision row equals the FP64 row sum (zero row sums, i.e. the constant
// null vector of the Laplacian and the translations of elasticity, survive the rounding).
template <int NDOF>
__global__ __launch_bounds__(kBlock) void k_make_lowp(int64_t n, const double* __restrict__ coef,
                                                      float* __restrict__ c32, uint16_t* __restrict__ cbf,
                                                      float* __restrict__ centre) {
  constexpr int NB = NDOF * NDOF, NCOEF = 27 * NB;
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  if (c32) {
    for (int k = 0; k < NCOEF; ++k) c32[coef_index(gi, k, NCOEF)] = (float)coef[coef_index(gi, k, NCOEF)];
    return;
  }
  double rowsum[NDOF], approx[NDOF];
#pragma unroll
  for (int a = 0; a < NDOF; ++a) rowsum[a] = approx[a] = 0.0;
  for (int s = 0; s < 27; ++s)
#pragma unroll
    for (int a = 0; a < NDOF; ++a)
#pragma unroll
      for (int b = 0; b < NDOF; ++b) {
        const int k = s * NB + a * NDOF + b;
        const double v = coef[coef_index(gi, k, NCOEF)];
        const uint16_t h = to_bf16((float)v);
        cbf[coef_index(gi, k, NCOEF)] = h;
        rowsum[a] += v;
        if (s == 13) {
          centre[gi * NB + a * NDOF + b] = (float)v;
          if (b != a) approx[a] += (double)(float)v;
        } else {
          approx[a] += (double)from_bf16(h);
        }
      }
#pragma unroll
  for (int a = 0; a < NDOF; ++a) centre[gi * NB + a * NDOF + a] = (float)(rowsum[a] - approx[a]);
}

void launch_make_lowp(Level& L, int coef_type, hipStream_t st) {
  RMG_REQUIRE(L.npts == 27, RMG_ERR_ARG, "low-precision levels need 27-point stencils");
  const size_t ne = coef_elems(L.n, L.ncoef());
  L.ct_lo = coef_type;
  float* c32 = nullptr;
  uint16_t* cbf = nullptr;
  float* centre = nullptr;
  if (coef_type == kCoefF32) {
    L.coef_lo.alloc(sizeof(float) * ne);
    c32 = L.coef_lo.as<float>();
  } else {
    L.coef_lo.alloc(sizeof(uint16_t) * ne);
    L.center_lo.alloc(sizeof(float) * (size_t)L.n * L.ndof * L.ndof);
    cbf = L.coef_lo.as<uint16_t>();
    centre = L.center_lo.as<float>();
  }
  const dim3 g(cdiv(L.n, kBlock));
  if (L.ndof == 3)
    RMG_LAUNCH(k_make_lowp<3>, g, dim3(kBlock), 0, st, L.n, L.coef.as<double>(), c32, cbf, centre);
  else
    RMG_LAUNCH(k_make_lowp<1>, g, dim3(kBlock), 0, st, L.n, L.coef.as<double>(), c32, cbf, centre);
  LAUNCH_CHECK();
  L.dinv_lo.alloc(sizeof(float) * (size_t)L.ndofs());
  launch_f64_to_f32(L.ndofs(), L.dinv.as<double>(), L.dinv_lo.as<float>(), st);
  L.dinv9_lo.release();
  if (L.dinv9.p) {
    L.dinv9_lo.alloc(sizeof(float) * 9 * (size_t)L.n);
    launch_f64_to_f32(9 * L.n, L.dinv9.as<double>(), L.dinv9_lo.as<float>(), st);
  }
}

// ------------------------------------------------------ symmetric half stencil
// Upper half (offsets 13..26, NDOF x NDOF blocks) of a 27-point level's stencils.  With a flag the
// FP64 operator is also checked: the flag is set unless every lower block equals the transposed
// upper block of the neighbour to rounding, |A(i, i+s)_ab - A(i+s, i)_ba| <= tol (d_i + d_j) with d
// the largest diagonal entry of a node's centre block, and couplings leaving the region are zero.
template <int NDOF, class C>
__global__ __launch_bounds__(kBlock) void k_make_sym(LevelView L, const C* __restrict__ coef, C* __restrict__ sym,
                                                     double tol, int* flag) {
  constexpr int NB = NDOF * NDOF, NC = 27 * NB, NS = kSymPts * NB;
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int64_t gi = R.off + li;
  for (int k = 0; k < NS; ++k) sym[coef_index(gi, k, NS)] = coef[coef_index(gi, 13 * NB + k, NC)];
  if (!flag) return;
  auto dmax = [&](int64_t g) {
    double d = 0.0;
    for (int a = 0; a < NDOF; ++a) d = fmax(d, fabs((double)coef[coef_index(g, 13 * NB + a * NDOF + a, NC)]));
    return d;
  };
  const double dii = dmax(gi);
  bool bad = false;
  for (int s = 0; s < 13; ++s) {
    int dx, dy, dz;
    stencil_offset<27>(s, dx, dy, dz);
    const bool in = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                    (unsigned)(z + dz) < (unsigned)R.ez;
    const int64_t gn = gi + dx + (int64_t)dy * R.ex + (int64_t)dz * R.ex * R.ey;
    const double djj = in ? dmax(gn) : 0.0;
    for (int a = 0; a < NDOF; ++a)
      for (int b = 0; b < NDOF; ++b) {
        const double v = (double)coef[coef_index(gi, s * NB + a * NDOF + b, NC)];
        if (!in) {
          if (v != 0.0) bad = true;
          continue;
        }
        const double m = (double)coef[coef_index(gn, (26 - s) * NB + b * NDOF + a, NC)];
        if (!(fabs(v - m) <= tol * (dii + djj))) bad = true;
      }
  }
  if (bad) atomicOr(flag, 1);
}

// Region tables of the symmetric 2.5D kernel.  Along an axis of extent e >= 5 a node's class is its
// coordinate on the two low layers (0, 1), 2 inside and 3, 4 on the two high layers; a node's class
// is (cz * 5 + cy) * 5 + cx.  A region's table holds, per class, the 27 couplings of the class's
// first node (x, y, z each 0, 1, 2, e - 2 or e - 1) as the streaming kernel reads them: its own
// upper couplings and its neighbours' upper couplings towards it, 0 towards neighbours outside the
// region.  The region is served when every node has its class's 27 couplings bit for bit; on a
// region whose operator is the same everywhere inside (one material, interface faces alike) that
// holds, and the tiles that serve it read no couplings from memory.
__device__ __forceinline__ bool same_bits(double a, double b) { return __double_as_longlong(a) == __double_as_longlong(b); }


// Coupling s of node (x, y, z) of region R, A(i, i + offset(s)), as the symmetric kernels read it.
template <int NDOF>
__device__ __forceinline__ double read_coupling(const RegionGeo& R, const double* __restrict__ sym, int x, int y,
                                                int z, int s, int a, int b) {
  constexpr int NB = NDOF * NDOF, NC = kSymPts * NB;
  const int64_t gi = R.off + ((int64_t)z * R.ey + y) * R.ex + x;
  if (s >= 13) return sym[coef_index(gi, (s - 13) * NB + a * NDOF + b, NC)];
  int dx, dy, dz;
  stencil_offset<27>(s, dx, dy, dz);
  if ((unsigned)(x + dx) >= (unsigned)R.ex || (unsigned)(y + dy) >= (unsigned)R.ey || (unsigned)(z + dz) >= (unsigned)R.ez)
    return 0.0;
  // a lower block is the transpose of the neighbour's upper block
  return sym[coef_index(gi + dx + (int64_t)dy * R.ex + (int64_t)dz * R.ex * R.ey, (13 - s) * NB + b * NDOF + a, NC)];
}

// One block per region, one thread per class; a class's row holds its 27 (blocks of) couplings in
// stencil order, each block row-major.
template <int NDOF>
__global__ __launch_bounds__(128) void k_class_table_ref(LevelView L, const double* __restrict__ sym,
                                                         double* __restrict__ table, int* __restrict__ ok) {
  constexpr int NB = NDOF * NDOF;
  const int k = blockIdx.x, c = threadIdx.x;
  const RegionGeo R = L.regs[k];
  const bool big = R.ex >= 5 && R.ey >= 5 && R.ez >= 5;
  if (c == 0) ok[k] = big ? 1 : 0;
  if (c >= kClasses) return;
  const int x = class_node(c % 5, R.ex), y = class_node(c / 5 % 5, R.ey), z = class_node(c / 25, R.ez);
  double* out = table + ((int64_t)k * kClasses + c) * kClassPts * NB;
  for (int s = 0; s < kClassPts; ++s)
    for (int e = 0; e < NB; ++e) out[s * NB + e] = big ? read_coupling<NDOF>(R, sym, x, y, z, s, e / NDOF, e % NDOF) : 0.0;
}

// One thread per node: a coupling that differs from its class's clears the region's flag.
template <int NDOF>
__global__ __launch_bounds__(kBlock) void k_class_table_check(LevelView L, const double* __restrict__ sym,
                                                              const double* __restrict__ table, int* __restrict__ ok) {
  constexpr int NB = NDOF * NDOF;
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n || !ok[bd.region]) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  const int c = (axis_class(z, R.ez) * 5 + axis_class(y, R.ey)) * 5 + axis_class(x, R.ex);
  const double* ref = table + ((int64_t)bd.region * kClasses + c) * kClassPts * NB;
  bool same = true;
  for (int s = 0; s < kClassPts; ++s)
    for (int e = 0; e < NB; ++e)
      same = same && same_bits(read_coupling<NDOF>(R, sym, x, y, z, s, e / NDOF, e % NDOF), ref[s * NB + e]);
  if (!same) ok[bd.region] = 0;
}

static void make_class_table(Level& L, hipStream_t st) {
  DBuf& tab = L.class_table;
  DBuf& ok = L.class_table_ok;
  const double* sym = static_cast<const double*>(L.coef_sym.p);
  const int nb = L.ndof * L.ndof;
  tab.alloc(sizeof(double) * kClasses * kClassPts * nb * L.nreg);
  ok.alloc(sizeof(int) * L.nreg);
  if (L.ndof == 3) {
    RMG_LAUNCH(k_class_table_ref<3>, dim3(L.nreg), dim3(128), 0, st, L.view(), sym, tab.as<double>(), ok.as<int>());
    RMG_LAUNCH(k_class_table_check<3>, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), sym,
               static_cast<const double*>(tab.p), ok.as<int>());
  } else {
    RMG_LAUNCH(k_class_table_ref<1>, dim3(L.nreg), dim3(128), 0, st, L.view(), sym, tab.as<double>(), ok.as<int>());
    RMG_LAUNCH(k_class_table_check<1>, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), sym,
               static_cast<const double*>(tab.p), ok.as<int>());
  }
  LAUNCH_CHECK();
  std::vector<int> flags(L.nreg);
  RMG_HIP(hipMemcpyAsync(flags.data(), ok.p, sizeof(int) * L.nreg, hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  int served = 0;
  for (int f : flags) served += f != 0;
  if (served == 0) {  // no region served: drop the tables, so the streaming kernel runs
    tab.release();
    ok.release();
    clear_split(L);
  } else if (L.use_tiles && L.tile_threads == kTileThreadsF64) {
    make_split(L, flags);
  } else {
    clear_split(L);  // node blocks: each block of a served region reads the tables
  }
}

template <int NDOF>
static void make_sym_t(Level& L, bool lowp, int* flag, hipStream_t st) {
  const size_t ne = coef_elems(L.n, kSymPts * NDOF * NDOF);
  const dim3 g(L.blocks.size()), b(kBlock);
  if (!lowp) {
    L.coef_sym.alloc(sizeof(double) * ne);
    RMG_LAUNCH((k_make_sym<NDOF, double>), g, b, 0, st, L.view(), L.coef.as<double>(), L.coef_sym.as<double>(),
                       1e-11, flag);
  } else if (L.ct_lo == kCoefF32) {
    L.coef_lo_sym.alloc(sizeof(float) * ne);
    RMG_LAUNCH((k_make_sym<NDOF, float>), g, b, 0, st, L.view(), L.coef_lo.as<float>(),
                       L.coef_lo_sym.as<float>(), 0.0, nullptr);
  } else {
    L.coef_lo_sym.alloc(sizeof(uint16_t) * ne);
    RMG_LAUNCH((k_make_sym<NDOF, uint16_t>), g, b, 0, st, L.view(), L.coef_lo.as<uint16_t>(),
                       L.coef_lo_sym.as<uint16_t>(), 0.0, nullptr);
  }
  LAUNCH_CHECK();
}

bool launch_make_sym(Level& L, bool lowp, hipStream_t st, bool table) {
  DBuf& out = lowp ? L.coef_lo_sym : L.coef_sym;
  out.release();
  if (!lowp) {
    L.class_table.release();
    L.class_table_ok.release();
    clear_split(L);
  }
  if (L.dim != 3 || L.npts != 27) return false;
  if (lowp) {
    // the low-precision copy rounds the same symmetric values: copy its upper half
    if (!L.coef_sym.p || L.ct_lo == kCoefF64) return false;
    if (L.ndof == 3) make_sym_t<3>(L, true, nullptr, st);
    else make_sym_t<1>(L, true, nullptr, st);
    return true;
  }
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  if (L.ndof == 3) make_sym_t<3>(L, false, flag.as<int>(), st);
  else make_sym_t<1>(L, false, flag.as<int>(), st);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  if (hflag) out.release();
  else if (table) make_class_table(L, st);
  return hflag == 0;
}

// ------------------------------------------------------------------ CG
// With u0 (scalar levels): also the V-cycle's zero-guess start from the new residual, u0 = c0 D~^-1 r,
// as k_cheb_zero computes it.
template <int NDOF>
__global__ __launch_bounds__(kBlock) void k_cg_update(LevelView L, const double* __restrict__ scalars,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      double* __restrict__ partials, const double* __restrict__ dinv,
                                                      double c0, double* __restrict__ u0,
                                                      const double* __restrict__ table, const int* __restrict__ table_ok) {
  const double alpha = scalars[kAlpha];
  double c = 0.0;
  for (int j = 0; j < kUpdateDescs; ++j) {
    const int64_t d = (int64_t)blockIdx.x * kUpdateDescs + j;
    if (d >= L.nblocks) break;
    const BlockDesc bd = L.blocks[d];
    const RegionGeo R = L.regs[bd.region];
    const int li = bd.start + (int)threadIdx.x;
    if (li < R.n) {
      int xx, yy, zz;
      decompose(R, li, xx, yy, zz);
      const bool own = !is_shared(L, R, xx, yy, zz);
#pragma unroll
      for (int a = 0; a < NDOF; ++a) {
        const int64_t gi = (R.off + li) * NDOF + a;
        x[gi] = x[gi] + alpha * p[gi];
        const double rn = r[gi] + (-alpha) * q[gi];
        r[gi] = rn;
        if (NDOF == 1 && u0) {
          // a one-region row of a region served by its class table: D~^-1 is 1 / its class's centre
          // coupling (the quotient the stored D~^-1 holds), so the row's D~^-1 is not read
          double di;
          if (table && own && table_ok[bd.region]) {
            const int cls = (axis_class(zz, R.ez) * 5 + axis_class(yy, R.ey)) * 5 + axis_class(xx, R.ex);
            di = 1.0 / table[((int64_t)bd.region * kClasses + cls) * kClassPts + 13];
          } else {
            di = dinv[gi];
          }
          u0[gi] = c0 * (di * rn);
        }
        if (own) c += rn * rn;
      }
    }
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int64_t launch_cg_update(const Level& L, double* scalars, double* x, double* r, const double* p, const double* q,
                         double* partials, hipStream_t st, const double* dinv, double c0, double* u0) {
  const int64_t nb = reduction_blocks(L, kUpdateDescs);
  RMG_REQUIRE(!u0 || (L.ndof == 1 && dinv), RMG_ERR_ARG, "internal: fused zero-guess start needs a scalar level");
  if (L.ndof == 3)
    RMG_LAUNCH(k_cg_update<3>, dim3(nb), dim3(kBlock), 0, st, L.view(), scalars, x, r, p, q, partials, nullptr,
               0.0, nullptr, nullptr, nullptr);
  else {
    // the class tables give D~^-1 of the served regions' one-region rows (when dinv is the level's own)
    const bool tab = u0 && dinv == L.dinv.as<double>() && L.npts == 27 && L.class_table.p && L.class_table_ok.p;
    RMG_LAUNCH(k_cg_update<1>, dim3(nb), dim3(kBlock), 0, st, L.view(), scalars, x, r, p, q, partials, dinv, c0,
               u0, tab ? L.class_table.as<double>() : nullptr, tab ? L.class_table_ok.as<int>() : nullptr);
  }
  LAUNCH_CHECK();
  return nb + dot_groups(L, r, r, partials + nb, st);
}

__global__ void k_cg_direction(int64_t n, const double* __restrict__ scalars, const double* __restrict__ z,
                               double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = scalars[kBeta];
  p[i] = z[i] + beta * p[i];
}

void launch_cg_direction(int64_t n, double* scalars, const double* z, double* p, hipStream_t st) {
  RMG_LAUNCH(k_cg_direction, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, scalars, z, p);
  LAUNCH_CHECK();
}

__global__ void k_cg_scalars(double* s, int mode) {
  if (mode == 0) {
    s[kAlpha] = s[kRZ] / s[kPQ];
  } else if (mode == 1) {
    s[kBeta] = s[kRZnew] / s[kRZ];
    s[kRZ] = s[kRZnew];
  } else {
    s[kBeta] = -s[kAlpha] * s[kZQ] / s[kRZ];
    s[kRZ] = s[kRZnew];
  }
}

void launch_cg_scalars(double* scalars, int mode, hipStream_t st) {
  RMG_LAUNCH(k_cg_scalars, dim3(1), dim3(1), 0, st, scalars, mode);
  LAUNCH_CHECK();
}

}  // namespace rmg
