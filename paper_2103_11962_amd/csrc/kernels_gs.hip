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
// The neighbours' corrections are read back from global memory written by the same block before
// the barrier (all waves of a block share the CU's vector L1, and the barrier orders the accesses).
//
// After the sweep the copies of an interface node hold different corrections (each region saw only
// its own updates); k_group_reduce<AVG> replaces them by their average, so the regional vector
// stays the regional form of a composite one.
#include "device_common.h"

namespace rmg {

constexpr int kGsThreads = 1024;

template <int NPTS, int NDOF, bool BACKWARD>
__global__ __launch_bounds__(kGsThreads) void k_gs_sweep(LevelView L, const double* __restrict__ coef,
                                                         const double* __restrict__ dinv,
                                                         const double* __restrict__ r, double* delta,
                                                         double omega) {
  constexpr int NB = NDOF * NDOF;
  constexpr int NC = NPTS * NB;
  constexpr int CEN = center_index<NPTS>();
  constexpr int WY = NPTS == 5 ? 1 : 2;
  constexpr int WZ = 4;
  const RegionGeo R = L.regs[blockIdx.x];
  const int tmax = (R.ex - 1) + WY * (R.ey - 1) + WZ * (R.ez - 1);
  // for a fixed z, the nodes of plane t have y in [ceil((t - WZ z - ex + 1) / WY), (t - WZ z) / WY]
  const int ycand = min(R.ey, (R.ex - 1) / WY + 1);
  const int sy = R.ex, sz = R.ex * R.ey;
  for (int step = 0; step <= tmax; ++step) {
    const int t = BACKWARD ? tmax - step : step;
    const int zlo_num = t - (R.ex - 1) - WY * (R.ey - 1);
    const int z0 = zlo_num <= 0 ? 0 : (zlo_num + WZ - 1) / WZ;
    const int z1 = min(R.ez - 1, t / WZ);
    const int cnt = z1 >= z0 ? (z1 - z0 + 1) * ycand : 0;
    for (int q = threadIdx.x; q < cnt; q += kGsThreads) {
      const int z = z0 + q / ycand;
      const int rem = t - WZ * z;  // x + WY y, >= 0
      const int ylo_num = rem - (R.ex - 1);
      const int y = (ylo_num <= 0 ? 0 : (ylo_num + WY - 1) / WY) + q % ycand;
      const int x = rem - WY * y;
      if (y >= R.ey || x < 0 || x >= R.ex) continue;
      const int li = x + sy * y + sz * z;
      const int64_t gi = R.off + li;
      const double* __restrict__ cf = coef + coef_index(gi, 0, NC);
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
            const int64_t nb = R.off + li + dx + dy * sy + dz * sz;
#pragma unroll
            for (int b = 0; b < NDOF; ++b) acc -= cf[(s * NB + a * NDOF + b) * kTile] * delta[nb * NDOF + b];
          }
        }
        // dofs of the same node visited before this one
#pragma unroll
        for (int b = 0; b < NDOF; ++b)
          if (BACKWARD ? b > a : b < a) acc -= cf[(CEN * NB + a * NDOF + b) * kTile] * dl[b];
        dl[a] = omega * acc * dinv[gi * NDOF + a];
      }
#pragma unroll
      for (int a = 0; a < NDOF; ++a) delta[gi * NDOF + a] = dl[a];
    }
    __syncthreads();
  }
}

template <int NPTS, int NDOF>
static void gs_launch(const Level& L, const double* r, double* delta, double omega, bool backward, hipStream_t st) {
  const LevelView V = L.view();
  const double* cf = L.coef.as<double>();
  const double* di = L.dinv.as<double>();
  if (backward)
    hipLaunchKernelGGL((k_gs_sweep<NPTS, NDOF, true>), dim3(L.nreg), dim3(kGsThreads), 0, st, V, cf, di, r, delta,
                       omega);
  else
    hipLaunchKernelGGL((k_gs_sweep<NPTS, NDOF, false>), dim3(L.nreg), dim3(kGsThreads), 0, st, V, cf, di, r, delta,
                       omega);
  LAUNCH_CHECK();
}

void launch_gs_sweep(const Level& L, const double* r, double* delta, double omega, bool backward, hipStream_t st) {
  if (L.n == 0) return;
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
    hipLaunchKernelGGL((k_group_reduce<3, true>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, w);
  else
    hipLaunchKernelGGL((k_group_reduce<1, true>), g, dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, w);
  LAUNCH_CHECK();
}

void launch_group_reduce(const int64_t* gptr, const int* gcopy, int64_t ngroups, double* w, bool avg, hipStream_t st) {
  if (ngroups == 0) return;
  const dim3 g(cdiv(ngroups, kBlock));
  if (avg)
    hipLaunchKernelGGL((k_group_reduce<1, true>), g, dim3(kBlock), 0, st, gptr, gcopy, ngroups, w);
  else
    hipLaunchKernelGGL((k_group_reduce<1, false>), g, dim3(kBlock), 0, st, gptr, gcopy, ngroups, w);
  LAUNCH_CHECK();
}

}  // namespace rmg
