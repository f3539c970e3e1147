// Region-local Gauss-Seidel (Section 3.4, Algorithm 1) for gfx950.
//
// A sweep takes the composite residual r (computed beforehand with its interface sum, the sweep's
// only communication) and, in every region k independently, visits the region's dofs in
// lexicographic order (x fastest, then y, z; the dofs of a node in order), subtracting from r_i
// the couplings A^(k)_ij delta_j to dofs already visited and setting delta_i = omega r_i / d~_i.
// That is the triangular solve (D~/omega + L_k) delta_k = r_k; a backward sweep uses the upper
// triangle in reverse order.
//
// Lexicographic order is sequential, but a node only waits for its lower neighbours, and every
// lower neighbour of (x, y, z) lies on a smaller hyperplane x + WY y + WZ z (WY = 2, WZ = 4 for
// 9- and 27-point stencils, WY = 1 for the five-point one).  The nodes of one hyperplane are
// independent, so one block per region walks the hyperplanes in order with a barrier between
// them and updates each plane's nodes in parallel: the same arithmetic as the sequential sweep.
//
// Within a plane no two nodes are neighbours in x, so reading the regional arrays would give every
// lane its own cache line.  The sweep therefore works in "slot" order: plane t of a region owns
// slots pbase[t] + q, q = (z - z0(t)) * ycand + (y - ylo(t, z)) enumerating its (z, y) candidates
// (x follows from t).  At setup the level's stencils and D~^-1 are copied into slot order
// (k_gs_fill); a sweep reads them and the neighbours' corrections by slot, which for consecutive
// lanes are consecutive.  Only r and the regional output are touched once per node in regional
// order.  The corrections are read back from the slot array written by the same block before the
// barrier (all waves of a block share the CU's vector L1, and the barrier orders the accesses).
//
// After the sweep the copies of an interface node hold different corrections (each region saw only
// its own updates); k_group_reduce<AVG> replaces them by their average, so the regional vector
// stays the regional form of a composite one.
#include <vector>

#include "device_common.h"

namespace rmg {

constexpr int kGsThreads = 1024;

// Hyperplanes x + wy y + 4 z = t of a region box and the slots of their nodes.
struct GsPlanes {
  static constexpr int WZ = 4;
  int ex, ey, ez, wy, ycand, tmax;
  __host__ __device__ GsPlanes(int ex_, int ey_, int ez_, int wy_) : ex(ex_), ey(ey_), ez(ez_), wy(wy_) {
    const int c = (ex - 1) / wy + 1;  // y candidates of one (t, z): y in [ylo, ylo + c)
    ycand = ey < c ? ey : c;
    tmax = (ex - 1) + wy * (ey - 1) + WZ * (ez - 1);
  }
  __host__ __device__ int z0(int t) const {
    const int n = t - (ex - 1) - wy * (ey - 1);
    return n <= 0 ? 0 : (n + WZ - 1) / WZ;
  }
  __host__ __device__ int z1(int t) const {
    const int m = t / WZ;
    return m < ez - 1 ? m : ez - 1;
  }
  __host__ __device__ int count(int t) const {
    const int a = z0(t), b = z1(t);
    return b >= a ? (b - a + 1) * ycand : 0;
  }
  __host__ __device__ int ylo(int t, int z) const {
    const int n = t - WZ * z - (ex - 1);
    return n <= 0 ? 0 : (n + wy - 1) / wy;
  }
  // node of candidate q of plane t; false if the candidate lies outside the box
  __host__ __device__ bool node(int t, int q, int& x, int& y, int& z) const {
    z = z0(t) + q / ycand;
    y = ylo(t, z) + q % ycand;
    x = t - WZ * z - wy * y;
    return y < ey && x >= 0 && x < ex;
  }
  __host__ __device__ int slot(int t, int y, int z) const { return (z - z0(t)) * ycand + (y - ylo(t, z)); }
};

template <int NPTS>
constexpr int gs_wy() {
  return NPTS == 5 ? 1 : 2;
}

// Setup: the level's stencil blocks and D~^-1 in slot order (one block per region).
template <int NPTS, int NDOF>
__global__ __launch_bounds__(kGsThreads) void k_gs_fill(LevelView L, const int* __restrict__ rplane,
                                                        const int64_t* __restrict__ pbase,
                                                        const double* __restrict__ coef,
                                                        const double* __restrict__ dinv, double* __restrict__ cs,
                                                        double* __restrict__ ds_inv) {
  constexpr int NC = NPTS * NDOF * NDOF;
  const RegionGeo R = L.regs[blockIdx.x];
  const GsPlanes P(R.ex, R.ey, R.ez, gs_wy<NPTS>());
  const int64_t* __restrict__ pb = pbase + rplane[blockIdx.x];
  for (int t = 0; t <= P.tmax; ++t) {
    const int cnt = P.count(t);
    for (int q = threadIdx.x; q < cnt; q += kGsThreads) {
      int x, y, z;
      if (!P.node(t, q, x, y, z)) continue;
      const int64_t gi = R.off + x + (int64_t)R.ex * (y + (int64_t)R.ey * z);
      const int64_t p = pb[t] + q;
      for (int c = 0; c < NC; ++c) cs[coef_index(p, c, NC)] = coef[coef_index(gi, c, NC)];
#pragma unroll
      for (int a = 0; a < NDOF; ++a) ds_inv[p * NDOF + a] = dinv[gi * NDOF + a];
    }
  }
}

template <int NPTS, int NDOF, bool BACKWARD>
__global__ __launch_bounds__(kGsThreads) void k_gs_sweep(LevelView L, const int* __restrict__ rplane,
                                                         const int64_t* __restrict__ pbase,
                                                         const double* __restrict__ cs,
                                                         const double* __restrict__ ds_inv,
                                                         const double* __restrict__ r, double* __restrict__ delta,
                                                         double* ds, double omega) {
  constexpr int NB = NDOF * NDOF;
  constexpr int NC = NPTS * NB;
  constexpr int CEN = center_index<NPTS>();
  constexpr int WY = gs_wy<NPTS>();
  const RegionGeo R = L.regs[blockIdx.x];
  const GsPlanes P(R.ex, R.ey, R.ez, WY);
  const int64_t* __restrict__ pb = pbase + rplane[blockIdx.x];
  for (int step = 0; step <= P.tmax; ++step) {
    const int t = BACKWARD ? P.tmax - step : step;
    const int cnt = P.count(t);
    for (int q = threadIdx.x; q < cnt; q += kGsThreads) {
      int x, y, z;
      if (!P.node(t, q, x, y, z)) continue;
      const int64_t gi = R.off + x + (int64_t)R.ex * (y + (int64_t)R.ey * z);
      const int64_t p = pb[t] + q;
      const double* __restrict__ c = cs + coef_index(p, 0, NC);
      double dl[NDOF];
#pragma unroll
      for (int aa = 0; aa < NDOF; ++aa) {
        const int a = BACKWARD ? NDOF - 1 - aa : aa;
        double acc = r[gi * NDOF + a];
#pragma unroll
        for (int s = BACKWARD ? CEN + 1 : 0; s < (BACKWARD ? NPTS : CEN); ++s) {
          int dx, dy, dz;
          stencil_offset<NPTS>(s, dx, dy, dz);
          if ((unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
              (unsigned)(z + dz) < (unsigned)R.ez) {
            const int tn = t + dx + WY * dy + GsPlanes::WZ * dz;
            const int64_t pn = pb[tn] + P.slot(tn, y + dy, z + dz);
#pragma unroll
            for (int b = 0; b < NDOF; ++b) acc -= c[(s * NB + a * NDOF + b) * kTile] * ds[pn * NDOF + b];
          }
        }
        // dofs of the same node visited before this one
#pragma unroll
        for (int b = 0; b < NDOF; ++b)
          if (BACKWARD ? b > a : b < a) acc -= c[(CEN * NB + a * NDOF + b) * kTile] * dl[b];
        dl[a] = omega * acc * ds_inv[p * NDOF + a];
      }
#pragma unroll
      for (int a = 0; a < NDOF; ++a) {
        ds[p * NDOF + a] = dl[a];
        delta[gi * NDOF + a] = dl[a];
      }
    }
    __syncthreads();
  }
}

template <int NPTS, int NDOF>
static void gs_fill_launch(const Level& L, hipStream_t st) {
  RMG_LAUNCH((k_gs_fill<NPTS, NDOF>), dim3(L.nreg), dim3(kGsThreads), 0, st, L.view(), L.gs_rplane.as<int>(),
                     L.gs_pbase.as<int64_t>(), L.coef.as<double>(), L.dinv.as<double>(), L.gs_coef.as<double>(),
                     L.gs_dinv.as<double>());
  LAUNCH_CHECK();
}

void launch_gs_prepare(Level& L, hipStream_t st) {
  RMG_REQUIRE(L.ndof == 1 || L.npts == 27, RMG_ERR_ARG, "internal: Gauss-Seidel blocks need 27-point levels");
  const int wy = L.npts == 5 ? 1 : 2;
  std::vector<int32_t> rplane(L.nreg + 1, 0);
  std::vector<int64_t> pbase;
  int64_t slots = 0;
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    const GsPlanes P(R.ex, R.ey, R.ez, wy);
    rplane[k] = (int32_t)pbase.size();
    for (int t = 0; t <= P.tmax; ++t) {
      pbase.push_back(slots);
      slots += P.count(t);
    }
  }
  rplane[L.nreg] = (int32_t)pbase.size();
  pbase.push_back(slots);
  L.gs_rplane.alloc(sizeof(int32_t) * rplane.size());
  L.gs_pbase.alloc(sizeof(int64_t) * pbase.size());
  RMG_HIP(hipMemcpyAsync(L.gs_rplane.p, rplane.data(), sizeof(int32_t) * rplane.size(), hipMemcpyHostToDevice, st));
  RMG_HIP(hipMemcpyAsync(L.gs_pbase.p, pbase.data(), sizeof(int64_t) * pbase.size(), hipMemcpyHostToDevice, st));
  L.gs_coef.alloc(sizeof(double) * coef_elems(slots, L.ncoef()));
  L.gs_dinv.alloc(sizeof(double) * (size_t)slots * L.ndof);
  L.gs_d.alloc(sizeof(double) * (size_t)slots * L.ndof);
  if (L.npts == 27 && L.ndof == 3) gs_fill_launch<27, 3>(L, st);
  else if (L.npts == 27) gs_fill_launch<27, 1>(L, st);
  else if (L.npts == 9) gs_fill_launch<9, 1>(L, st);
  else gs_fill_launch<5, 1>(L, st);
  RMG_HIP(hipStreamSynchronize(st));  // the host tables above are released on return
}

template <int NPTS, int NDOF>
static void gs_launch(const Level& L, const double* r, double* delta, double omega, bool backward, hipStream_t st) {
  const LevelView V = L.view();
  const int* rp = L.gs_rplane.as<int>();
  const int64_t* pb = L.gs_pbase.as<int64_t>();
  const double* cs = L.gs_coef.as<double>();
  const double* di = L.gs_dinv.as<double>();
  double* ds = L.gs_d.as<double>();
  if (backward)
    RMG_LAUNCH((k_gs_sweep<NPTS, NDOF, true>), dim3(L.nreg), dim3(kGsThreads), 0, st, V, rp, pb, cs, di, r,
                       delta, ds, omega);
  else
    RMG_LAUNCH((k_gs_sweep<NPTS, NDOF, false>), dim3(L.nreg), dim3(kGsThreads), 0, st, V, rp, pb, cs, di, r,
                       delta, ds, omega);
  LAUNCH_CHECK();
}

void launch_gs_sweep(const Level& L, const double* r, double* delta, double omega, bool backward, hipStream_t st) {
  if (L.n == 0) return;
  RMG_REQUIRE(L.gs_pbase.p != nullptr, RMG_ERR_NOT_SETUP, "internal: Gauss-Seidel slot tables missing");
  if (L.npts == 27 && L.ndof == 3) gs_launch<27, 3>(L, r, delta, omega, backward, st);
  else if (L.npts == 27) gs_launch<27, 1>(L, r, delta, omega, backward, st);
  else if (L.npts == 9) gs_launch<9, 1>(L, r, delta, omega, backward, st);
  else gs_launch<5, 1>(L, r, delta, omega, backward, st);
}

// Every copy of an interface dof receives the sum (AVG: the average) of the copies, summed in
// ascending region order.
template <int NDOF, bool AVG>
__global__ __launch_bounds__(kBlock) void k_group_reduce(const int64_t* __restrict__ gptr,
                                                         const int* __restrict__ gcopy, int64_t ng, double* w) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t a0 = gptr[g], e = gptr[g + 1];
#pragma unroll
  for (int a = 0; a < NDOF; ++a) {
    double s = 0.0;
    for (int64_t c = a0; c < e; ++c) s += w[(int64_t)gcopy[c] * NDOF + a];
    if (AVG) s *= 1.0 / (double)(e - a0);
    for (int64_t c = a0; c < e; ++c) w[(int64_t)gcopy[c] * NDOF + a] = s;
  }
}

void launch_interface_avg(const Level& L, double* w, hipStream_t st) {
  if (L.ngroups == 0) return;
  const dim3 g(cdiv(L.ngroups, kBlock));
  if (L.ndof == 3)
    RMG_LAUNCH((k_group_reduce<3, true>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, w);
  else
    RMG_LAUNCH((k_group_reduce<1, true>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, w);
  LAUNCH_CHECK();
}

void launch_group_reduce(const int64_t* gptr, const int* gcopy, int64_t ngroups, double* w, bool avg, hipStream_t st) {
  if (ngroups == 0) return;
  const dim3 g(cdiv(ngroups, kBlock));
  if (avg)
    RMG_LAUNCH((k_group_reduce<1, true>), g, dim3(kBlock), 0, st, gptr, gcopy, ngroups, w);
  else
    RMG_LAUNCH((k_group_reduce<1, false>), g, dim3(kBlock), 0, st, gptr, gcopy, ngroups, w);
  LAUNCH_CHECK();
}

}  // namespace rmg
