// HIP kernels of the regional multigrid path for gfx950 (FP64, scalar PDEs).
//
// Work decomposition: every level keeps a table of BlockDesc (region, first
// local node); one 256-thread block processes 256 consecutive nodes of one
// region (x fastest), so coefficient and vector streams are unit-stride and
// a block never straddles two regions.  Interface nodes (nodes shared by
// several regions, Section 3.1) are finished by a second kernel over the
// level's interface groups: it sums the co-located partial results in
// ascending region order and writes the same final value to every copy
// (the Psi^T Psi operation, fused with whatever the node update needs).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace rmg {

// ------------------------------------------------------------------ helpers
template <int NPTS>
__device__ __forceinline__ void stencil_offset(int s, int& dx, int& dy, int& dz) {
  if constexpr (NPTS == 27) {
    dx = s % 3 - 1;
    dy = (s / 3) % 3 - 1;
    dz = s / 9 - 1;
  } else if constexpr (NPTS == 9) {
    dx = s % 3 - 1;
    dy = s / 3 - 1;
    dz = 0;
  } else {  // five-point: (0,-1) (-1,0) (0,0) (1,0) (0,1)
    dz = 0;
    dx = (s == 1) ? -1 : (s == 3 ? 1 : 0);
    dy = (s == 0) ? -1 : (s == 4 ? 1 : 0);
  }
}

template <int NPTS>
constexpr int center_index() {
  return NPTS == 27 ? 13 : (NPTS == 9 ? 4 : 2);
}

__device__ __forceinline__ bool is_dirichlet(const LevelView& L, int gx, int gy, int gz) {
  const unsigned m = L.mask;
  return ((m & 1u) && gx == 0) || ((m & 2u) && gx == L.cx - 1) || ((m & 4u) && gy == 0) ||
         ((m & 8u) && gy == L.cy - 1) || ((m & 16u) && gz == 0) || ((m & 32u) && gz == L.cz - 1);
}

// A node is shared with another region iff it lies on a face of its box that is not on the
// outer boundary of the domain (the boxes tile the domain's bounding box).
__device__ __forceinline__ bool is_shared(const LevelView& L, const RegionGeo& R, int x, int y, int z) {
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  return (x == 0 && gx != 0) || (x == R.ex - 1 && gx != L.cx - 1) || (y == 0 && gy != 0) ||
         (y == R.ey - 1 && gy != L.cy - 1) || (z == 0 && gz != 0) || (z == R.ez - 1 && gz != L.cz - 1);
}

__device__ __forceinline__ int64_t comp_index(const LevelView& L, int gx, int gy, int gz) {
  return ((int64_t)gz * L.cy + gy) * L.cx + gx;
}

__device__ __forceinline__ void decompose(const RegionGeo& R, int li, int& x, int& y, int& z) {
  x = li % R.ex;
  const int t = li / R.ex;
  y = t % R.ey;
  z = t / R.ey;
}

// Linear interpolation weight of a fine node at distance t (in fine cells) from a coarse node.
__device__ __forceinline__ double w1(int t) {
  t = t < 0 ? -t : t;
  return t == 0 ? 1.0 : (t == 1 ? 2.0 / 3.0 : (t == 2 ? 1.0 / 3.0 : 0.0));
}

__device__ __forceinline__ double block_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __shared__ double sm[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += sm[i];
  }
  return s;
}

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }


#define LAUNCH_CHECK() RMG_HIP(hipGetLastError())

// ------------------------------------------------------- stencil operations
struct OpParams {
  const double* x;
  double* out;
  const double* b;
  const double* dinv;
  double* d;
  double c1, c2;
  const double* dotw;
};

// Final update of a node once z = (Psi^T Psi A x) at that node is known; m = multiplicity.
// Returns this node's contribution to the fused reduction, if any.
template <StencilOp OP, bool DOT>
__device__ __forceinline__ double node_finish_x(const OpParams& p, int64_t gi, double z, int m, double xself);

template <StencilOp OP, bool DOT>
__device__ __forceinline__ double node_finish(const OpParams& p, int64_t gi, double z, int m) {
  if constexpr (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst || OP == StencilOp::CgQ)
    return node_finish_x<OP, DOT>(p, gi, z, m, p.x[gi]);
  else
    return node_finish_x<OP, DOT>(p, gi, z, m, 0.0);
}

// xself = the stencil input at this node (used by the Chebyshev update and the CG dot product).
template <StencilOp OP, bool DOT>
__device__ __forceinline__ double node_finish_x(const OpParams& p, int64_t gi, double z, int m, double xself) {
  if constexpr (OP == StencilOp::Matvec) {
    p.out[gi] = z;
    return 0.0;
  } else if constexpr (OP == StencilOp::Residual) {
    p.out[gi] = p.b[gi] - z;
    return 0.0;
  } else if constexpr (OP == StencilOp::ResidualScaled) {
    const double r = p.b[gi] - z;
    p.out[gi] = (m == 1) ? r : r / (double)m;
    return 0.0;
  } else if constexpr (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst) {
    const double r = p.b[gi] - z;
    double dd = p.c2 * (p.dinv[gi] * r);
    if constexpr (OP == StencilOp::Cheb) dd = p.c1 * p.d[gi] + dd;
    p.d[gi] = dd;
    const double u = xself + dd;
    p.out[gi] = u;
    if constexpr (DOT) return p.dotw[gi] * u;
    return 0.0;
  } else {  // CgQ
    p.out[gi] = z;
    return xself * z;
  }
}

template <int NPTS, StencilOp OP, bool DOT>
__global__ __launch_bounds__(kBlock) void k_stencil(LevelView L, const double* __restrict__ coef, OpParams p,
                                                    double* __restrict__ partials) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  double contrib = 0.0;
  if (li < R.n) {
    int x, y, z;
    decompose(R, li, x, y, z);
    const int64_t gi = R.off + li;
    const double* __restrict__ xr = p.x + R.off;
    const double* __restrict__ cf = coef + coef_index(gi, 0, NPTS);
    const int sy = R.ex, sz = R.ex * R.ey;
    const bool inner = x > 0 && x < R.ex - 1 && y > 0 && y < R.ey - 1 && (NPTS != 27 || (z > 0 && z < R.ez - 1));
    double acc = 0.0;
    if (inner) {
#pragma unroll
      for (int s = 0; s < NPTS; ++s) {
        int dx, dy, dz;
        stencil_offset<NPTS>(s, dx, dy, dz);
        acc += cf[s * kTile] * xr[li + dx + dy * sy + dz * sz];
      }
      contrib = node_finish<OP, DOT>(p, gi, acc, 1);
    } else {
#pragma unroll
      for (int s = 0; s < NPTS; ++s) {
        int dx, dy, dz;
        stencil_offset<NPTS>(s, dx, dy, dz);
        const bool ok = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                        (unsigned)(z + dz) < (unsigned)R.ez;
        if (ok) acc += cf[s * kTile] * xr[li + dx + dy * sy + dz * sz];
      }
      if (is_shared(L, R, x, y, z)) {
        p.out[gi] = acc;  // partial product; summed over the copies by k_iface
      } else {
        contrib = node_finish<OP, DOT>(p, gi, acc, 1);
      }
    }
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    const double s = block_sum(contrib);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}


// ------------------------------------------------ 3D stencil, 2.5D tiles
// A block owns a tile of ty x-rows (tx nodes each) of one region and marches nz planes in z.
// The input vector's planes pass through two LDS slots; each thread keeps its 3x3
// neighbourhood of planes z-1, z, z+1 in registers (rotated per plane), so it reads only the
// new plane from LDS, and the plane after next is prefetched from global memory into registers
// while the current plane is computed.  Neighbours outside the region box read 0 from LDS and
// have zero coefficients, so the 27-term sum needs no bounds branches.
constexpr int kT3 = 512;           // threads per 3D tile block
constexpr int kT3Plane = 1544;     // max (ty+2)(tx+2) over tx*ty <= 512
constexpr int kT3Fetch = (kT3Plane + kT3 - 1) / kT3;

template <StencilOp OP, bool DOT>
__global__ __launch_bounds__(kT3) void k_stencil3d(LevelView L, const Tile3* __restrict__ tiles,
                                                   const double* __restrict__ coef, OpParams p,
                                                   double* __restrict__ partials) {
  __shared__ double pl[2][kT3Plane];
  const Tile3 T = tiles[blockIdx.x];
  const RegionGeo R = L.regs[T.region];
  const int W = T.tx + 2, PL = (T.ty + 2) * W;
  const double* __restrict__ xr = p.x + R.off;
  const int t = threadIdx.x;
  const int ty = t / T.tx, tx = t - ty * T.tx;
  const int x = T.x0 + tx, y = T.y0 + ty;
  const bool active = ty < T.ty && x < R.ex && y < R.ey;
  const int sy = R.ex, sz = R.ex * R.ey;
  double pre[kT3Fetch];
  auto fetch = [&](int zz) {
#pragma unroll
    for (int k = 0; k < kT3Fetch; ++k) {
      const int idx = t + k * kT3;
      double v = 0.0;
      if (idx < PL) {
        const int r = idx / W;
        const int xx = T.x0 + idx - r * W - 1, yy = T.y0 - 1 + r;
        if ((unsigned)zz < (unsigned)R.ez && (unsigned)yy < (unsigned)R.ey && (unsigned)xx < (unsigned)R.ex)
          v = xr[zz * sz + yy * sy + xx];
      }
      pre[k] = v;
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int k = 0; k < kT3Fetch; ++k) {
      const int idx = t + k * kT3;
      if (idx < PL) pl[slot][idx] = pre[k];
    }
  };
  double rm[9], rc[9], rp[9];
  auto readn = [&](int slot, double* r) {
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int dx = j % 3 - 1, dy = j / 3 - 1;
      r[j] = pl[slot][(ty + 1 + dy) * W + tx + 1 + dx];
    }
  };
  const int z0 = T.z0, z1 = T.z0 + T.nz;
  fetch(z0 - 1);
  store(0);
  fetch(z0);
  store(1);
  __syncthreads();
  if (active) {
    readn(0, rm);
    readn(1, rc);
  }
  __syncthreads();
  fetch(z0 + 1);
  store(0);
  __syncthreads();
  double contrib = 0.0;
  for (int zz = z0; zz < z1; ++zz) {
    const int sp = (zz - z0) & 1;  // slot holding plane zz+1
    if (active) readn(sp, rp);
    fetch(zz + 2);
    if (active) {
      const int li = zz * sz + y * sy + x;
      const int64_t gi = R.off + li;
      const double* __restrict__ cf = coef + coef_index(gi, 0, 27);
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < 27; ++s) {
        const int j = s % 9, dz = s / 9 - 1;
        const double v = dz < 0 ? rm[j] : (dz == 0 ? rc[j] : rp[j]);
        acc += cf[s * kTile] * v;
      }
      const bool edge = x == 0 || x == R.ex - 1 || y == 0 || y == R.ey - 1 || zz == 0 || zz == R.ez - 1;
      if (edge && is_shared(L, R, x, y, zz)) p.out[gi] = acc;  // finished by k_iface
      else contrib += node_finish_x<OP, DOT>(p, gi, acc, 1, rc[4]);
    }
    store(sp ^ 1);  // plane zz+2 replaces plane zz
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      rm[j] = rc[j];
      rc[j] = rp[j];
    }
    __syncthreads();
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    double v = contrib;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __shared__ double sm[kT3 / 64];
    if ((t & 63) == 0) sm[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int i = 0; i < kT3 / 64; ++i) s += sm[i];
      partials[blockIdx.x] = s;
    }
  }
}

template <StencilOp OP, bool DOT>
__global__ __launch_bounds__(kBlock) void k_iface(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                  int64_t ng, OpParams p, double* __restrict__ partials) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double contrib = 0.0;
  if (g < ng) {
    const int64_t a = gptr[g], e = gptr[g + 1];
    const int m = (int)(e - a);
    double s = 0.0;
    for (int64_t c = a; c < e; ++c) s += p.out[gcopy[c]];
    for (int64_t c = a; c < e; ++c) {
      const double v = node_finish<OP, DOT>(p, gcopy[c], s, m);
      if (c == a) contrib = v;  // the first copy (lowest region) owns the composite dof
    }
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    const double s = block_sum(contrib);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

template <int NPTS, StencilOp OP, bool DOT>
static int64_t run_stencil(const Level& L, const OpParams& p, double* partials, hipStream_t st,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  const LevelView v = L.view();
  const bool tiled = NPTS == 27 && L.use_tiles;
  if (ev0) RMG_HIP(hipEventRecord(ev0, st));
  if (tiled)
    hipLaunchKernelGGL((k_stencil3d<OP, DOT>), dim3(L.tiles.size()), dim3(kT3), 0, st, v, L.d_tiles.as<Tile3>(),
                       L.coef.as<double>(), p, partials);
  else
    hipLaunchKernelGGL((k_stencil<NPTS, OP, DOT>), dim3(L.blocks.size()), dim3(kBlock), 0, st, v,
                       L.coef.as<double>(), p, partials);
  LAUNCH_CHECK();
  if (ev1) RMG_HIP(hipEventRecord(ev1, st));
  const int64_t nb = tiled ? (int64_t)L.tiles.size() : (int64_t)L.blocks.size();
  int64_t ngb = 0;
  if (L.ngroups > 0) {
    ngb = cdiv(L.ngroups, kBlock);
    hipLaunchKernelGGL((k_iface<OP, DOT>), dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, p, partials ? partials + nb : nullptr);
    LAUNCH_CHECK();
  }
  return (DOT || OP == StencilOp::CgQ) ? nb + ngb : 0;
}

template <int NPTS>
static int64_t dispatch_op(const Level& L, const StencilArgs& a, const OpParams& p, hipStream_t st) {
  const bool dot = a.dotw != nullptr;
  switch (a.op) {
    case StencilOp::Matvec: return run_stencil<NPTS, StencilOp::Matvec, false>(L, p, nullptr, st);
    case StencilOp::Residual: return run_stencil<NPTS, StencilOp::Residual, false>(L, p, nullptr, st);
    case StencilOp::ResidualScaled:
      return run_stencil<NPTS, StencilOp::ResidualScaled, false>(L, p, nullptr, st);
    case StencilOp::Cheb:
      return dot ? run_stencil<NPTS, StencilOp::Cheb, true>(L, p, a.partials, st, a.ev0, a.ev1)
                 : run_stencil<NPTS, StencilOp::Cheb, false>(L, p, nullptr, st, a.ev0, a.ev1);
    case StencilOp::ChebFirst:
      return dot ? run_stencil<NPTS, StencilOp::ChebFirst, true>(L, p, a.partials, st)
                 : run_stencil<NPTS, StencilOp::ChebFirst, false>(L, p, nullptr, st);
    case StencilOp::CgQ: return run_stencil<NPTS, StencilOp::CgQ, false>(L, p, a.partials, st, a.ev0, a.ev1);
  }
  return 0;
}

int64_t launch_stencil_op(const Level& L, const StencilArgs& a, hipStream_t st) {
  OpParams p{a.x, a.out, a.b, a.dinv, a.d, a.c1, a.c2, a.dotw};
  switch (L.npts) {
    case 27: return dispatch_op<27>(L, a, p, st);
    case 9: return dispatch_op<9>(L, a, p, st);
    case 5: return dispatch_op<5>(L, a, p, st);
  }
  fail(RMG_ERR_ARG, "unsupported stencil size");
}

// ------------------------------------------------------- interface sum
__global__ __launch_bounds__(kBlock) void k_iface_sum(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                      int64_t ng, const double* v, double* w) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t a = gptr[g], e = gptr[g + 1];
  double s = 0.0;
  for (int64_t c = a; c < e; ++c) s += v[gcopy[c]];
  for (int64_t c = a; c < e; ++c) w[gcopy[c]] = s;
}

__global__ void k_copy(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

void launch_copy(int64_t n, const double* src, double* dst, hipStream_t st) {
  if (n == 0 || src == dst) return;
  hipLaunchKernelGGL(k_copy, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, src, dst);
  LAUNCH_CHECK();
}

void launch_interface_sum(const Level& L, const double* v, double* w, hipStream_t st) {
  if (v != w) launch_copy(L.n, v, w, st);
  if (L.ngroups == 0) return;
  hipLaunchKernelGGL(k_iface_sum, dim3(cdiv(L.ngroups, kBlock)), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                     L.d_gcopy.as<int>(), L.ngroups, w, w);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ reductions
__global__ __launch_bounds__(kBlock) void k_dot_nodes(LevelView L, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ partials) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  double c = 0.0;
  if (li < R.n) {
    int x, y, z;
    decompose(R, li, x, y, z);
    if (!is_shared(L, R, x, y, z)) {
      const int64_t gi = R.off + li;
      c = a[gi] * b[gi];
    }
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_dot_groups(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                       int64_t ng, const double* __restrict__ a,
                                                       const double* __restrict__ b, double* __restrict__ partials) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double c = 0.0;
  if (g < ng) {
    const int i = gcopy[gptr[g]];
    c = a[i] * b[i];
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int64_t launch_dot(const Level& L, const double* a, const double* b, double* partials, hipStream_t st) {
  const LevelView v = L.view();
  const int64_t nb = (int64_t)L.blocks.size();
  hipLaunchKernelGGL(k_dot_nodes, dim3(nb), dim3(kBlock), 0, st, v, a, b, partials);
  LAUNCH_CHECK();
  int64_t ngb = 0;
  if (L.ngroups > 0) {
    ngb = cdiv(L.ngroups, kBlock);
    hipLaunchKernelGGL(k_dot_groups, dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, a, b, partials + nb);
    LAUNCH_CHECK();
  }
  return nb + ngb;
}

constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double* __restrict__ partials, int64_t n,
                                                           double* scalars, int slot) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kReduceThreads) s += partials[i];
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
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kReduceThreads), 0, st, partials, n, scalars, slot);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ pointwise
__global__ void k_cheb_zero(int64_t n, const double* __restrict__ b, const double* __restrict__ dinv, double c,
                            double* __restrict__ d, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = c * (dinv[i] * b[i]);
  d[i] = v;
  u[i] = v;
}

void launch_cheb_zero(const Level& L, const double* b, const double* dinv, double c, double* d, double* u,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_zero, dim3(cdiv(L.n, kBlock)), dim3(kBlock), 0, st, L.n, b, dinv, c, d, u);
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
  hipLaunchKernelGGL(k_scale, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, scalars, slot, mode, x, y);
  LAUNCH_CHECK();
}

__global__ void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] * b[i];
}

void launch_mul(int64_t n, const double* a, const double* b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_mul, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, a, b, y);
  LAUNCH_CHECK();
}

__global__ void k_zero(int64_t n, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

void launch_zero(int64_t n, double* y, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, y);
  LAUNCH_CHECK();
}

__global__ void k_sub_from(int64_t n, const double* __restrict__ b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b[i] - y[i];
}

void launch_sub_from(int64_t n, const double* b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_from, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, b, y);
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
  hipLaunchKernelGGL(k_recip_check, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, in, out, flag);
  LAUNCH_CHECK();
}

// --------------------------------------------------------- diag / start
template <int NPTS>
__global__ void k_diag(int64_t n, const double* __restrict__ coef, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = coef[coef_index(i, center_index<NPTS>(), NPTS)];
}

void launch_diag(const Level& L, double* out, hipStream_t st) {
  const dim3 g(cdiv(L.n, kBlock));
  if (L.npts == 27) hipLaunchKernelGGL(k_diag<27>, g, dim3(kBlock), 0, st, L.n, L.coef.as<double>(), out);
  else if (L.npts == 9) hipLaunchKernelGGL(k_diag<9>, g, dim3(kBlock), 0, st, L.n, L.coef.as<double>(), out);
  else hipLaunchKernelGGL(k_diag<5>, g, dim3(kBlock), 0, st, L.n, L.coef.as<double>(), out);
  LAUNCH_CHECK();
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): golden-ratio increment and the
// variant-13 finaliser; the counter of composite node i on level l under seed s is
// i + (l << 40) + (s << 48).
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
  double v = 0.0;
  if (!is_dirichlet(L, gx, gy, gz)) {
    const uint64_t ctr = (uint64_t)comp_index(L, gx, gy, gz) + ((uint64_t)level << 40) + (seed << 48);
    const uint64_t r = splitmix64(ctr);
    v = 2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0;
  }
  out[R.off + li] = v;
}

void launch_start_vector(const Level& L, int level, uint64_t seed, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_start_vector, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), level, seed, out);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------ transfers
// One thread per coarse node: w = sum_f P_fC r_f over the fine nodes of the same
// region within two fine cells per axis (r already divided by multiplicity).
// Coarse Dirichlet nodes receive nothing (free fine nodes do not interpolate from them).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelView F, LevelView C, const double* __restrict__ r,
                                                     double* __restrict__ w) {
  const BlockDesc bd = C.blocks[blockIdx.x];
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RC.n) return;
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const int64_t gi = RC.off + li;
  if (is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z)) {
    w[gi] = 0.0;
    return;
  }
  const double* __restrict__ rr = r + RF.off;
  double acc = 0.0;
  const int tzlo = DIM == 3 ? -2 : 0, tzhi = DIM == 3 ? 2 : 0;
  for (int tz = tzlo; tz <= tzhi; ++tz) {
    const int fz = 3 * Z + tz;
    if ((unsigned)fz >= (unsigned)RF.ez) continue;
    const double wz = w1(tz);
    for (int ty = -2; ty <= 2; ++ty) {
      const int fy = 3 * Y + ty;
      if ((unsigned)fy >= (unsigned)RF.ey) continue;
      const double wzy = wz * w1(ty);
      const int base = (fz * RF.ey + fy) * RF.ex;
#pragma unroll
      for (int tx = -2; tx <= 2; ++tx) {
        const int fx = 3 * X + tx;
        if ((unsigned)fx >= (unsigned)RF.ex) continue;
        acc += (wzy * w1(tx)) * rr[base + fx];
      }
    }
  }
  w[gi] = acc;
}

void launch_restrict(const Level& F, const Level& C, const double* r_scaled, double* w, hipStream_t st) {
  if (F.dim == 3)
    hipLaunchKernelGGL(k_restrict<3>, dim3(C.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), r_scaled, w);
  else
    hipLaunchKernelGGL(k_restrict<2>, dim3(C.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), r_scaled, w);
  LAUNCH_CHECK();
  launch_interface_sum(C, w, w, st);
}

// One thread per fine node: u += sum_C P_fC ubar_C over the (up to 2 per axis) coarse nodes
// of the coarse cell containing the node.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView F, LevelView C, const double* __restrict__ ubar,
                                                        double* __restrict__ u) {
  const BlockDesc bd = F.blocks[blockIdx.x];
  const RegionGeo RF = F.regs[bd.region];
  const RegionGeo RC = C.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RF.n) return;
  int x, y, z;
  decompose(RF, li, x, y, z);
  const bool fdir = is_dirichlet(F, RF.ox + x, RF.oy + y, RF.oz + z);
  const int cx = x / 3, tx = x - 3 * cx, cy = y / 3, ty = y - 3 * cy, cz = z / 3, tz = z - 3 * cz;
  const double* __restrict__ ub = ubar + RC.off;
  double acc = 0.0;
  const int nz = (DIM == 3 && tz) ? 2 : 1, ny = ty ? 2 : 1, nx = tx ? 2 : 1;
  for (int iz = 0; iz < nz; ++iz) {
    const double wz = DIM == 3 ? w1(tz - 3 * iz) : 1.0;
    for (int iy = 0; iy < ny; ++iy) {
      const double wzy = wz * w1(ty - 3 * iy);
      for (int ix = 0; ix < nx; ++ix) {
        const int X = cx + ix, Y = cy + iy, Z = cz + iz;
        if (!fdir && is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z)) continue;
        acc += (wzy * w1(tx - 3 * ix)) * ub[(Z * RC.ey + Y) * RC.ex + X];
      }
    }
  }
  u[RF.off + li] += acc;
}

void launch_prolong_add(const Level& F, const Level& C, const double* ubar, double* u, hipStream_t st) {
  if (F.dim == 3)
    hipLaunchKernelGGL(k_prolong_add<3>, dim3(F.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), ubar, u);
  else
    hipLaunchKernelGGL(k_prolong_add<2>, dim3(F.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), ubar, u);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------------ RAP
// Per-region Galerkin product [[Abar]] = P^T A^(k) P, one thread per coarse node C:
// Abar(C, C+o) = sum_{t, s} P(3C+t, C) A(3C+t, s) P(3C+t+s, C+o), with the fine node
// 3C+t within two cells of C and t+s-3o within two cells per axis.  Accumulators live
// in LDS (one column per thread).  Dirichlet reading: a Dirichlet coarse row only
// collects Dirichlet fine nodes; entries of a free row towards Dirichlet coarse nodes
// are zero.
constexpr int kRapBlock = kBlock;  // one block per BlockDesc; 27 x 256 doubles of LDS

template <int NPTSF, int DIM>
__global__ __launch_bounds__(kRapBlock) void k_rap(LevelView F, LevelView C, const double* __restrict__ coefF,
                                                   double* __restrict__ coefC) {
  constexpr int NC = DIM == 3 ? 27 : 9;
  __shared__ double acc[NC][kRapBlock];
  const int tid = threadIdx.x;
#pragma unroll
  for (int o = 0; o < NC; ++o) acc[o][tid] = 0.0;
  const BlockDesc bd = C.blocks[blockIdx.x];
  const RegionGeo RC = C.regs[bd.region];
  const RegionGeo RF = F.regs[bd.region];
  const int li = bd.start + tid;
  if (li >= RC.n) return;  // no block-wide synchronisation below: private LDS columns
  int X, Y, Z;
  decompose(RC, li, X, Y, Z);
  const bool cdir = is_dirichlet(C, RC.ox + X, RC.oy + Y, RC.oz + Z);
  const int tzlo = DIM == 3 ? -2 : 0, tzhi = DIM == 3 ? 2 : 0;
  for (int tz = tzlo; tz <= tzhi; ++tz) {
    const int fz = 3 * Z + tz;
    if ((unsigned)fz >= (unsigned)RF.ez) continue;
    for (int ty = -2; ty <= 2; ++ty) {
      const int fy = 3 * Y + ty;
      if ((unsigned)fy >= (unsigned)RF.ey) continue;
      for (int tx = -2; tx <= 2; ++tx) {
        const int fx = 3 * X + tx;
        if ((unsigned)fx >= (unsigned)RF.ex) continue;
        if (cdir && !is_dirichlet(F, RF.ox + fx, RF.oy + fy, RF.oz + fz)) continue;
        const double wf = (DIM == 3 ? w1(tz) : 1.0) * w1(ty) * w1(tx);
        const int64_t fi = RF.off + (fz * RF.ey + fy) * RF.ex + fx;
#pragma unroll
        for (int s = 0; s < NPTSF; ++s) {
          const double a = coefF[coef_index(fi, s, NPTSF)];
          if (a == 0.0) continue;
          int dx, dy, dz;
          stencil_offset<NPTSF>(s, dx, dy, dz);
          const double wa = wf * a;
          const int ux = tx + dx, uy = ty + dy, uz = tz + dz;
          const int oxl = ux <= -1 ? -1 : 0, oyl = uy <= -1 ? -1 : 0, ozl = uz <= -1 ? -1 : 0;
          for (int kz = 0; kz < (DIM == 3 ? 2 : 1); ++kz) {
            const int oz = DIM == 3 ? ozl + kz : 0;
            const double wz = DIM == 3 ? w1(uz - 3 * oz) : 1.0;
            if (wz == 0.0) continue;
            for (int ky = 0; ky < 2; ++ky) {
              const int oy = oyl + ky;
              const double wy = w1(uy - 3 * oy);
              if (wy == 0.0) continue;
              for (int kx = 0; kx < 2; ++kx) {
                const int ox = oxl + kx;
                const double wx = w1(ux - 3 * ox);
                if (wx == 0.0) continue;
                const int oi = DIM == 3 ? (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1) : (oy + 1) * 3 + (ox + 1);
                acc[oi][tid] += wa * (wz * wy * wx);
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
    double v = acc[o][tid];
    const int Xn = X + ox, Yn = Y + oy, Zn = Z + oz;
    const bool inbox = (unsigned)Xn < (unsigned)RC.ex && (unsigned)Yn < (unsigned)RC.ey &&
                       (unsigned)Zn < (unsigned)RC.ez;
    if (!inbox) v = 0.0;
    else if (!cdir && is_dirichlet(C, RC.ox + Xn, RC.oy + Yn, RC.oz + Zn)) v = 0.0;
    coefC[coef_index(gi, o, NC)] = v;
  }
}

void launch_rap(const Level& F, Level& C, hipStream_t st) {
  const dim3 g(C.blocks.size()), b(kRapBlock);
  if (F.dim == 3) {
    RMG_REQUIRE(F.npts == 27, RMG_ERR_ARG, "3D levels need 27-point stencils");
    hipLaunchKernelGGL((k_rap<27, 3>), g, b, 0, st, F.view(), C.view(), F.coef.as<double>(), C.coef.as<double>());
  } else if (F.npts == 9) {
    hipLaunchKernelGGL((k_rap<9, 2>), g, b, 0, st, F.view(), C.view(), F.coef.as<double>(), C.coef.as<double>());
  } else {
    hipLaunchKernelGGL((k_rap<5, 2>), g, b, 0, st, F.view(), C.view(), F.coef.as<double>(), C.coef.as<double>());
  }
  LAUNCH_CHECK();
}

// ------------------------------------------------- composite <-> regional
__global__ __launch_bounds__(kBlock) void k_to_regional(LevelView L, const double* __restrict__ comp,
                                                        double* __restrict__ reg) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= R.n) return;
  int x, y, z;
  decompose(R, li, x, y, z);
  reg[R.off + li] = comp[comp_index(L, R.ox + x, R.oy + y, R.oz + z)];
}

void launch_to_regional(const Level& L, const double* comp, double* reg, hipStream_t st) {
  hipLaunchKernelGGL(k_to_regional, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), comp, reg);
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
  comp[comp_index(L, R.ox + x, R.oy + y, R.oz + z)] = reg[R.off + li];
}

__global__ __launch_bounds__(kBlock) void k_to_composite_groups(const int64_t* __restrict__ gptr,
                                                                const int* __restrict__ gcopy,
                                                                const int* __restrict__ gcomp, int64_t ng,
                                                                const double* __restrict__ reg,
                                                                double* __restrict__ comp, int average) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t a = gptr[g], e = gptr[g + 1];
  double v;
  if (average) {
    double s = 0.0;
    for (int64_t c = a; c < e; ++c) s += reg[gcopy[c]];
    v = s / (double)(e - a);
  } else {
    v = reg[gcopy[a]];
  }
  comp[gcomp[g]] = v;
}

void launch_to_composite(const Level& L, const double* reg, double* comp, int average, hipStream_t st) {
  hipLaunchKernelGGL(k_to_composite_nodes, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), reg, comp);
  LAUNCH_CHECK();
  if (L.ngroups > 0) {
    hipLaunchKernelGGL(k_to_composite_groups, dim3(cdiv(L.ngroups, kBlock)), dim3(kBlock), 0, st,
                       L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(), L.d_gcomp.as<int>(), L.ngroups, reg, comp,
                       average);
    LAUNCH_CHECK();
  }
}

// ------------------------------------------------------- coarse solve
__global__ void k_gather(int n, const int* __restrict__ owner, const double* __restrict__ reg,
                         double* __restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = reg[owner[i]];
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

void launch_coarse_solve(const Level& L, const double* b, double* u, hipStream_t st) {
  const int n = L.nc;
  hipLaunchKernelGGL(k_gather, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, L.comp_owner.as<int>(), b,
                     L.cvec.as<double>());
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gemv, dim3(cdiv(n, 4)), dim3(256), 0, st, n, L.ainv.as<double>(), L.cvec.as<double>(),
                     L.cvec2.as<double>());
  LAUNCH_CHECK();
  launch_to_regional(L, L.cvec2.as<double>(), u, st);
}

__global__ void k_gj_save(int n, int k, const double* __restrict__ A, double* __restrict__ row,
                          double* __restrict__ col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    row[i] = A[(int64_t)k * n + i];
    col[i] = A[(int64_t)i * n + k];
  }
}

// In-place Gauss-Jordan step on pivot k (no pivoting; the matrix is SPD).
__global__ void k_gj_update(int n, int k, double* __restrict__ A, const double* __restrict__ row,
                            const double* __restrict__ col) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const double p = row[k];
  double* a = A + (int64_t)i * n + j;
  if (i == k && j == k) *a = 1.0 / p;
  else if (i == k) *a = row[j] / p;
  else if (j == k) *a = -col[i] / p;
  else *a -= col[i] * (row[j] / p);
}

void launch_gauss_jordan(double* A, int n, double* row, double* col, hipStream_t st) {
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_save, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, k, A, row, col);
    hipLaunchKernelGGL(k_gj_update, dim3(cdiv(n, kBlock), n), dim3(kBlock), 0, st, n, k, A, row, col);
  }
  LAUNCH_CHECK();
}

__global__ void k_check_inverse(int n, const double* __restrict__ A, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = A[(int64_t)i * n + i];
  if (!(d > 0.0) || !isfinite(d)) atomicOr(flag, 1);
}

void launch_check_inverse(const double* A, int n, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_inverse, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, A, flag);
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
  hipLaunchKernelGGL(k_assemble_q1, dim3(L.blocks.size()), dim3(kBlock), 0, st, L.view(), K, elem_coef,
                     L.coef.as<double>());
  LAUNCH_CHECK();
}

template <int NPTS>
__global__ void k_dirichlet_split(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                  const int* __restrict__ gcomp, int64_t ng, LevelView L, double* coef) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t ci = gcomp[g];
  const int gx = (int)(ci % L.cx), gy = (int)((ci / L.cx) % L.cy), gz = (int)(ci / ((int64_t)L.cx * L.cy));
  if (!is_dirichlet(L, gx, gy, gz)) return;
  const int64_t a = gptr[g], e = gptr[g + 1];
  for (int64_t c = a; c < e; ++c) coef[coef_index(gcopy[c], center_index<NPTS>(), NPTS)] = 1.0 / (double)(e - a);
}

void launch_dirichlet_split(const Level& L, hipStream_t st) {
  if (L.ngroups == 0) return;
  const dim3 g(cdiv(L.ngroups, kBlock));
  if (L.npts == 27)
    hipLaunchKernelGGL(k_dirichlet_split<27>, g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.d_gcomp.as<int>(), L.ngroups, L.view(), L.coef.as<double>());
  else if (L.npts == 9)
    hipLaunchKernelGGL(k_dirichlet_split<9>, g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.d_gcomp.as<int>(), L.ngroups, L.view(), L.coef.as<double>());
  else
    hipLaunchKernelGGL(k_dirichlet_split<5>, g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.d_gcomp.as<int>(), L.ngroups, L.view(), L.coef.as<double>());
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
  bool bad = false;
#pragma unroll
  for (int s = 0; s < NPTS; ++s) {
    int dx, dy, dz;
    stencil_offset<NPTS>(s, dx, dy, dz);
    double* c = coef + coef_index(gi, s, NPTS);
    const bool ok = (unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                    (unsigned)(z + dz) < (unsigned)R.ez;
    if (!isfinite(*c)) bad = true;
    if (!ok) *c = 0.0;
  }
  if (bad) atomicOr(flag, 1);
}

void launch_mask_stencil(const Level& L, int* flag, hipStream_t st) {
  const dim3 g(L.blocks.size());
  if (L.npts == 27) hipLaunchKernelGGL(k_mask_stencil<27>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  else if (L.npts == 9) hipLaunchKernelGGL(k_mask_stencil<9>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  else hipLaunchKernelGGL(k_mask_stencil<5>, g, dim3(kBlock), 0, st, L.view(), L.coef.as<double>(), flag);
  LAUNCH_CHECK();
}

// ------------------------------------------------- non-invasive split
// Region matrices from an assembled composite stencil on a tensor-product region layout
// (Section 4): an off-diagonal coupling is divided by q, the number of regions containing
// both end nodes; the diagonal of each region row is (row sum of A)/mult minus the region's
// split off-diagonals.  On a tensor layout a coupling along offset s is shared by
// prod_{d : s_d = 0} m_d regions, m_d = 2 on an inner slab boundary of axis d, else 1.
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
    hipLaunchKernelGGL(k_split_composite<27>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  else if (L.npts == 9)
    hipLaunchKernelGGL(k_split_composite<9>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  else
    hipLaunchKernelGGL(k_split_composite<5>, g, dim3(kBlock), 0, st, L.view(), comp, L.ncomp, L.coef.as<double>(), flag);
  LAUNCH_CHECK();
}

// Caller layout (structure of arrays over one region) <-> wave-tiled level storage.
__global__ void k_region_stencil_io(int64_t off, int nn, int npts, double* __restrict__ coef,
                                    double* __restrict__ soa, int to_level) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nn * npts) return;
  const int s = (int)(t / nn);
  const int i = (int)(t - (int64_t)s * nn);
  double* c = coef + coef_index(off + i, s, npts);
  if (to_level) *c = soa[t];
  else soa[t] = *c;
}

void launch_region_stencil_io(const Level& L, int region, double* soa, int to_level, hipStream_t st) {
  const RegionGeo& R = L.regs[region];
  const int64_t tot = (int64_t)R.n * L.npts;
  hipLaunchKernelGGL(k_region_stencil_io, dim3(cdiv(tot, kBlock)), dim3(kBlock), 0, st, R.off, R.n, L.npts,
                     L.coef.as<double>(), soa, to_level);
  LAUNCH_CHECK();
}

// ------------------------------------------------------------------ CG
__global__ __launch_bounds__(kBlock) void k_cg_update(LevelView L, const double* __restrict__ scalars,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      double* __restrict__ partials) {
  const BlockDesc bd = L.blocks[blockIdx.x];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  double c = 0.0;
  if (li < R.n) {
    const double alpha = scalars[kAlpha];
    const int64_t gi = R.off + li;
    x[gi] = x[gi] + alpha * p[gi];
    const double rn = r[gi] + (-alpha) * q[gi];
    r[gi] = rn;
    int xx, yy, zz;
    decompose(R, li, xx, yy, zz);
    if (!is_shared(L, R, xx, yy, zz)) c = rn * rn;
  }
  const double s = block_sum(c);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int64_t launch_cg_update(const Level& L, double* scalars, double* x, double* r, const double* p, const double* q,
                         double* partials, hipStream_t st) {
  const int64_t nb = (int64_t)L.blocks.size();
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kBlock), 0, st, L.view(), scalars, x, r, p, q, partials);
  LAUNCH_CHECK();
  int64_t ngb = 0;
  if (L.ngroups > 0) {
    ngb = cdiv(L.ngroups, kBlock);
    hipLaunchKernelGGL(k_dot_groups, dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(), L.d_gcopy.as<int>(),
                       L.ngroups, r, r, partials + nb);
    LAUNCH_CHECK();
  }
  return nb + ngb;
}

__global__ void k_cg_direction(int64_t n, const double* __restrict__ scalars, const double* __restrict__ z,
                               double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = scalars[kBeta];
  p[i] = z[i] + beta * p[i];
}

__global__ void k_cg_scalars(double* s, int mode) {
  if (mode == 0) {
    s[kAlpha] = s[kRZ] / s[kPQ];
  } else {
    s[kBeta] = s[kRZnew] / s[kRZ];
    s[kRZ] = s[kRZnew];
  }
}

void launch_cg_scalars(double* scalars, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(1), 0, st, scalars, mode);
  LAUNCH_CHECK();
}

void launch_cg_direction(int64_t n, double* scalars, const double* z, double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_direction, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, scalars, z, p);
  LAUNCH_CHECK();
}

}  // namespace rmg
