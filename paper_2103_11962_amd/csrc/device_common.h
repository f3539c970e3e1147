// Device-side helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace rmg {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

#define LAUNCH_CHECK() RMG_HIP(hipGetLastError())

// Every kernel launch of the library goes through RMG_LAUNCH, which counts it in
// g_kernel_launches (all handles and threads of the process).
#define RMG_LAUNCH(...)                                                  \
  do {                                                                   \
    ::rmg::g_kernel_launches.fetch_add(1, std::memory_order_relaxed);    \
    hipLaunchKernelGGL(__VA_ARGS__);                                     \
  } while (0)

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

// 1/m for a coarse interval of m = 1, 2 or 3 cells.  num * (1/m) equals num / m exactly for
// 0 <= num <= m (2 * (1/3) rounds like 2/3, 3 * (1/3) rounds to 1), with no division.
// Node class of a region's class tables along an axis of extent e >= 5: the coordinate on the two
// low layers (0, 1), 2 inside, 3 and 4 on the two high layers; and the first node of class c.
__device__ __forceinline__ int axis_class(int v, int e) { return v < 2 ? v : (v >= e - 2 ? v - e + 5 : 2); }
__device__ __forceinline__ int class_node(int c, int e) { return c <= 2 ? c : e - 5 + c; }

__device__ __forceinline__ double inv_span(int m) { return m == 3 ? 1.0 / 3.0 : (m == 2 ? 0.5 : 1.0); }

// Rate-3 coarsening of one region axis of e fine nodes into E coarse nodes: coarse node C sits at
// fine position min(3C, e - 1) (every third node from the region's first, and its last node).
// Fine node g (0 <= g < e) takes its interpolation from the coarse nodes lo (weight wlo) and, when
// whi != 0, lo + 1: lo = min(g / 3, E - 2) is the start of its coarse interval [p0, p1], p0 = 3 lo,
// p1 = min(3 lo + 3, e - 1), with linear weights (p1 - g) / (p1 - p0) and (g - p0) / (p1 - p0); a
// node at a coarse position takes that node alone (weight 1).  A degenerate axis (E = 1, the z
// axis of a 2D level) has one coarse node.
__device__ __forceinline__ void bracket(int g, int e, int E, int& lo, double& wlo, double& whi) {
  if (E < 2) {
    lo = 0;
    wlo = 1.0;
    whi = 0.0;
    return;
  }
  lo = min(g / 3, E - 2);
  const int p0 = 3 * lo, m = min(p0 + 3, e - 1) - p0, a = g - p0;
  const double inv = inv_span(m);
  const bool at_end = a == m;  // g is the interval's end node, the next coarse node
  lo += at_end ? 1 : 0;
  wlo = at_end ? 1.0 : (double)(m - a) * inv;
  whi = at_end ? 0.0 : (double)a * inv;
}

// Fine position of coarse node C on an axis of e fine nodes.
__device__ __forceinline__ int coarse_pos(int C, int e) { return min(3 * C, e - 1); }

// The coarse intervals on either side of coarse node C: mL cells to the left (0 for the first
// node), mR to the right (0 for the last); a degenerate axis (E = 1) has neither.
__device__ __forceinline__ void coarse_spans(int C, int e, int E, int& mL, int& mR) {
  const int p = coarse_pos(C, e);
  mL = C > 0 ? p - coarse_pos(C - 1, e) : 0;
  mR = C < E - 1 ? coarse_pos(C + 1, e) - p : 0;
}

// The two coarse nodes whose interval holds the fine node u cells from coarse node C (C's spans
// mL, mR; -mL <= u <= mR): C + o0 with weight w0 and C + o0 + 1 with weight w1.
__device__ __forceinline__ void interval_weights(int u, int mL, int mR, int& o0, double& w0, double& w1) {
  const bool neg = u < 0;
  o0 = neg ? -1 : 0;
  const int m = max(neg ? mL : mR, 1), a = neg ? mL + u : u;  // a: cells from the interval's start
  const double inv = inv_span(m);
  w0 = (double)(m - a) * inv;
  w1 = (double)a * inv;
}

// Weight of coarse node C for the fine node t cells from it (|t| <= 2), given its spans.
__device__ __forceinline__ double tap(int t, int mL, int mR) {
  const int m = t < 0 ? mL : mR, d = t < 0 ? -t : t;
  return t == 0 ? 1.0 : (d < m ? (double)(m - d) * inv_span(m) : 0.0);
}

// Work item of block b in a grid of n blocks.  The hardware deals consecutive blocks to the eight
// XCDs in turn, each with its own L2; this mapping gives every XCD a contiguous run of items, so
// neighbouring items (tiles, node blocks) that share data run on the same XCD and meet in its L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcds = 8;
  const int x = b % kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + min(x, r) + b / kXcds;
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
