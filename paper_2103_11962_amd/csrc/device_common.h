// Device-side helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace rmg {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

#define LAUNCH_CHECK() RMG_HIP(hipGetLastError())

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
__host__ __device__ constexpr int center_index() {
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

// Sum over a block of kBlock threads; the result is valid in thread 0.
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

// bfloat16 storage: the upper 16 bits of an IEEE float, rounded to nearest even.
__host__ __device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float from_bf16(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

template <class C>
struct CoefLoad;
template <>
struct CoefLoad<double> {
  __device__ static double get(const double* p) { return *p; }
};
template <>
struct CoefLoad<float> {
  __device__ static float get(const float* p) { return *p; }
};
template <>
struct CoefLoad<uint16_t> {
  __device__ static float get(const uint16_t* p) { return from_bf16(*p); }
};

}  // namespace rmg
