// Learned prolongation weights: a small MLP (27 -> 64 -> 64 -> 208, ReLU, FP32) maps the
// centred log-coefficients of a coarse cell's 27 fine elements to one logit per (fine node,
// coarse corner) pair of the cell; a softmax over each node's corners gives its weights.
// Training, inference, data extraction and the assembly of per-node interpolation weights
// (averaging the predictions of all cells that share a node) run in the kernels below.
//
// Training kernels follow the textbook layer-by-layer backward pass: per-sample kernels for
// the forward pass, the loss and the activation gradients, and a split-N reduction of the
// weight gradients (fixed summation order, so gradients are deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "device_common.h"
#include "mlp.h"

namespace rmg {

// Non-corner fine nodes of a cell (x-fastest over the 4x4x4 cell nodes): position, number of
// corners, first logit, corner slots (ix + 2 iy + 4 iz).  Filled from cell_node_table.
__constant__ CellNode c_nodes[56];
__constant__ signed char c_pos2node[64];  // -1 for the 8 corners
__constant__ float c_kq1[64];              // Q1 Laplace element matrix of the unit cube (energy loss)

void cell_node_table(CellNode* nodes, signed char* pos2node) {
  int n = 0, off = 0;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) {
        const int c[3] = {i, j, k};
        const bool corner = (i == 0 || i == 3) && (j == 0 || j == 3) && (k == 0 || k == 3);
        pos2node[(k * 4 + j) * 4 + i] = corner ? (signed char)-1 : (signed char)n;
        if (corner) continue;
        CellNode& nd = nodes[n];
        nd.pos = (k * 4 + j) * 4 + i;
        nd.first = off;
        // per axis: an interior coordinate (1, 2) interpolates from both corners, 0 / 3 from one
        int opts[3][2] = {}, no[3];
        for (int d = 0; d < 3; ++d) {
          if (c[d] == 1 || c[d] == 2) {
            opts[d][0] = 0;
            opts[d][1] = 1;
            no[d] = 2;
          } else {
            opts[d][0] = c[d] == 0 ? 0 : 1;
            no[d] = 1;
          }
        }
        int nc = 0;
        for (int iz = 0; iz < no[2]; ++iz)
          for (int iy = 0; iy < no[1]; ++iy)
            for (int ix = 0; ix < no[0]; ++ix) nd.corner[nc++] = opts[0][ix] + 2 * opts[1][iy] + 4 * opts[2][iz];
        for (int q = nc; q < 8; ++q) nd.corner[q] = 0;
        nd.ncorner = nc;
        off += nc;
        ++n;
      }
  RMG_REQUIRE(n == 56 && off == kMlpOut, RMG_ERR_ARG, "internal: cell node table");
}

// Once per device (constant memory is per device); handles on other threads may call it too.
static void upload_tables() {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  RMG_HIP(hipGetDevice(&dev));
  RMG_REQUIRE(dev >= 0 && dev < 64, RMG_ERR_ARG, "device index beyond 63");
  std::lock_guard<std::mutex> lock(mu);
  if (done[dev]) return;
  CellNode nodes[56];
  signed char pos2node[64];
  cell_node_table(nodes, pos2node);
  RMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_nodes), nodes, sizeof(nodes)));
  RMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_pos2node), pos2node, sizeof(pos2node)));
  double K[64];
  q1_laplace_element(1.0, K);
  float Kf[64];
  for (int i = 0; i < 64; ++i) Kf[i] = (float)K[i];
  RMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_kq1), Kf, sizeof(Kf)));
  done[dev] = true;
}

// ------------------------------------------------------------------ forward
// Parameter layout: W1 [64][27], b1 [64], W2 [64][64], b2 [64], W3 [208][64], b3 [208].
__global__ __launch_bounds__(kBlock) void k_mlp_forward(int64_t n, const float* __restrict__ X,
                                                        const float* __restrict__ th, float* __restrict__ Z,
                                                        float* __restrict__ A1, float* __restrict__ A2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* W1 = th;
  const float* b1 = W1 + kMlpH * kMlpIn;
  const float* W2 = b1 + kMlpH;
  const float* b2 = W2 + kMlpH * kMlpH;
  const float* W3 = b2 + kMlpH;
  const float* b3 = W3 + kMlpOut * kMlpH;
  // hidden activations stay in registers: every loop that indexes them is fully unrolled
  float x[kMlpIn], h1[kMlpH], h2[kMlpH];
#pragma unroll
  for (int j = 0; j < kMlpIn; ++j) x[j] = X[i * kMlpIn + j];
#pragma unroll
  for (int r = 0; r < kMlpH; ++r) {
    float a = b1[r];
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) a += W1[r * kMlpIn + j] * x[j];
    if (A1) A1[i * kMlpH + r] = a;
    h1[r] = a > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int r = 0; r < kMlpH; ++r) {
    float a = b2[r];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) a += W2[r * kMlpH + j] * h1[j];
    if (A2) A2[i * kMlpH + r] = a;
    h2[r] = a > 0.f ? a : 0.f;
  }
  for (int r = 0; r < kMlpOut; ++r) {
    float a = b3[r];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) a += W3[r * kMlpH + j] * h2[j];
    Z[i * kMlpOut + r] = a;
  }
}

// Position (in the 4x4x4 cell nodes) of coarse corner slot s.
__device__ __forceinline__ int corner_pos(int s) { return 48 * ((s >> 2) & 1) + 12 * ((s >> 1) & 1) + 3 * (s & 1); }

// Softmax over the corners of node `nd` of a logit row (entries c >= nd.ncorner are left 0).
__device__ __forceinline__ void node_softmax(const float* z, const CellNode& nd, float (&w)[8]) {
  float m = z[nd.first];
#pragma unroll
  for (int c = 1; c < 8; ++c)
    if (c < nd.ncorner) m = fmaxf(m, z[nd.first + c]);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    w[c] = c < nd.ncorner ? expf(z[nd.first + c] - m) : 0.f;
    s += w[c];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) w[c] /= s;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Loss per sample and its gradient with respect to the logits, scaled by 1/n (the loss is a mean
// over samples), on the interpolation error delta_f = e_f - sum_c w_fc e_c (zero at the corners):
//   L2:      sum_f delta_f^2 / sum_f e_f^2;
//   ENERGY:  delta^T A_cell delta / (cbar sum_f e_f^2), A_cell = sum over the cell's 27 elements of
//            c_e K (Q1 Laplace, unit cube), c_e = exp(X_e), cbar the mean of the c_e.
// One wavefront per sample: lane p holds the error at cell node p (x fastest over the 4x4x4 nodes),
// the corner values and neighbouring errors arrive by lane shuffles, and each lane of a non-corner
// node evaluates that node's softmax, so rows of E, X, Z and dZ are read and written contiguously.
// Partial sums: one per block of kMlpLossSamples.
constexpr int kMlpLossSamples = kBlock / 64;

template <bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_mlp_loss(int64_t n, const float* __restrict__ Z,
                                                     const float* __restrict__ E, const float* __restrict__ X,
                                                     float* __restrict__ dZ, double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kMlpLossSamples + wid;
  float loss = 0.f;
  if (i < n) {  // uniform over the wavefront
    const float ep = E[i * 64 + lane];
    float norm = wave_sum(ep * ep);
    if (!(norm > 0.f)) norm = 1.f;
    float ec[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ec[q] = __shfl(ep, corner_pos(q), 64);
    const int node = c_pos2node[lane];
    float w[8], ev[8], delta = 0.f;
    CellNode nd{};
    if (node >= 0) {
      nd = c_nodes[node];
      node_softmax(Z + i * kMlpOut, nd, w);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) v = (c < nd.ncorner && nd.corner[c] == q) ? ec[q] : v;
        ev[c] = v;
      }
      float pred = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c) pred += w[c] * ev[c];
      delta = ep - pred;
    }
    float g;  // d loss / d delta at this lane's node
    if constexpr (ENERGY) {
      const float ce = lane < 27 ? expf(X[i * kMlpIn + lane]) : 0.f;
      const float cbar = wave_sum(ce) * (1.0f / 27.0f);
      const int px = lane & 3, py = (lane >> 2) & 3, pz = lane >> 4;
      float ad = 0.f;  // (A_cell delta) at this node: its elements, corner roles a, neighbours b
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int ex = px - (a & 1), ey = py - ((a >> 1) & 1), ez = pz - ((a >> 2) & 1);
        const bool valid = (unsigned)ex < 3u && (unsigned)ey < 3u && (unsigned)ez < 3u;
        const int e0x = valid ? ex : 0, e0y = valid ? ey : 0, e0z = valid ? ez : 0;
        const float c = __shfl(ce, e0x + 3 * e0y + 9 * e0z, 64);  // every lane takes part
        float sum = 0.f;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int nb = ((e0z + ((b >> 2) & 1)) * 4 + e0y + ((b >> 1) & 1)) * 4 + e0x + (b & 1);
          sum += c_kq1[a * 8 + b] * __shfl(delta, nb, 64);
        }
        if (valid) ad += c * sum;
      }
      const float enorm = cbar * norm;
      loss = wave_sum(delta * ad) / enorm;
      g = 2.f * ad / enorm;
    } else {
      loss = wave_sum(delta * delta) / norm;
      g = 2.f * delta / norm;
    }
    if (node >= 0) {
      const float dpred = -g;
      float sdw = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c) sdw += dpred * ev[c] * w[c];
      const float inv_n = 1.0f / (float)n;
      float* dz = dZ + i * kMlpOut;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < nd.ncorner) dz[nd.first + c] = w[c] * (dpred * ev[c] - sdw) * inv_n;
    }
  }
  __shared__ float sm[kMlpLossSamples];
  if (lane == 0) sm[wid] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kMlpLossSamples; ++k) s += (double)sm[k];
    partials[blockIdx.x] = s;
  }
}

// Activation gradients: D2 = (dZ W3) * [A2 > 0], D1 = (D2 W2) * [A1 > 0].
__global__ __launch_bounds__(kBlock) void k_mlp_backact(int64_t n, const float* __restrict__ dZ,
                                                        const float* __restrict__ A1, const float* __restrict__ A2,
                                                        const float* __restrict__ th, float* __restrict__ D1,
                                                        float* __restrict__ D2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* W2 = th + kMlpH * kMlpIn + kMlpH;
  const float* W3 = W2 + kMlpH * kMlpH + kMlpH;
  float d2[kMlpH];
#pragma unroll
  for (int k = 0; k < kMlpH; ++k) d2[k] = 0.f;
  for (int j = 0; j < kMlpOut; ++j) {
    const float g = dZ[i * kMlpOut + j];
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) d2[k] += g * W3[j * kMlpH + k];
  }
#pragma unroll
  for (int k = 0; k < kMlpH; ++k) {
    d2[k] = A2[i * kMlpH + k] > 0.f ? d2[k] : 0.f;
    D2[i * kMlpH + k] = d2[k];
  }
#pragma unroll 4
  for (int r = 0; r < kMlpH; ++r) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) a += d2[k] * W2[k * kMlpH + r];
    D1[i * kMlpH + r] = A1[i * kMlpH + r] > 0.f ? a : 0.f;
  }
}

// Weight gradients of one layer over a slice of samples, a small GEMM with a long reduction
// dimension: G[r][j] = sum_s D[s][r] H'[s][j] for j < C (H' = ReLU(H) when relu) and
// G[r][C] = sum_s D[s][r] (bias).  Tiles of kWgS samples are staged through LDS; each thread
// keeps an MR x MC register tile of G with rows r = tr + i TR and columns j = tc + k TC, so the
// lanes of a wavefront read 16 consecutive rows and 4 columns (broadcasts, no bank conflicts).
// One FP32 partial per block; the partials are summed in FP64 in block order.
constexpr int kWgS = 32;     // samples per LDS tile
constexpr int kWgBlocks = 512;

template <int R, int C, int MR, int MC>
__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t n, const float* __restrict__ D,
                                                   const float* __restrict__ H, int relu, int64_t per_block,
                                                   float* __restrict__ part) {
  constexpr int TR = R / MR, TC = 256 / TR, CP = MC * TC;
  static_assert(TR * MR == R && TR * TC == 256 && CP >= C, "tile shape");
  __shared__ float sD[kWgS][R];
  __shared__ float sH[kWgS][CP];
  const int tr = threadIdx.x % TR, tc = threadIdx.x / TR;
  float acc[MR][MC], accb[MR];
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    accb[i] = 0.f;
#pragma unroll
    for (int k = 0; k < MC; ++k) acc[i][k] = 0.f;
  }
  const int64_t s0 = (int64_t)blockIdx.x * per_block, s1 = min(n, s0 + per_block);
  for (int64_t t0 = s0; t0 < s1; t0 += kWgS) {
    const int ns = (int)min((int64_t)kWgS, s1 - t0);
    // rows of D and H are contiguous: the tile is one contiguous span of each
    for (int idx = threadIdx.x; idx < kWgS * R; idx += 256) {
      const int s = idx / R;
      sD[s][idx - s * R] = s < ns ? D[t0 * R + idx] : 0.f;
    }
    for (int idx = threadIdx.x; idx < kWgS * CP; idx += 256) {
      const int s = idx / CP, j = idx - s * CP;
      float v = (s < ns && j < C) ? H[(t0 + s) * C + j] : 0.f;
      if (relu) v = v > 0.f ? v : 0.f;
      sH[s][j] = v;
    }
    __syncthreads();
    for (int s = 0; s < kWgS; ++s) {
      float d[MR], h[MC];
#pragma unroll
      for (int i = 0; i < MR; ++i) d[i] = sD[s][tr + i * TR];
#pragma unroll
      for (int k = 0; k < MC; ++k) h[k] = sH[s][tc + k * TC];
#pragma unroll
      for (int i = 0; i < MR; ++i) {
        accb[i] += d[i];
#pragma unroll
        for (int k = 0; k < MC; ++k) acc[i][k] += d[i] * h[k];
      }
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * R * (C + 1);
#pragma unroll
  for (int i = 0; i < MR; ++i) {
    const int r = tr + i * TR;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      const int j = tc + k * TC;
      if (j < C) out[r * (C + 1) + j] = acc[i][k];
    }
    if (tc == 0) out[r * (C + 1) + C] = accb[i];
  }
}

// Sum the block partials into the flat gradient: W block at wofs (row-major R x C), bias at bofs.
// A block owns 64 outputs; its four wavefronts sum every fourth partial and the four sums are
// added in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_mlp_wgrad_reduce(int R, int C, int nblk, const float* __restrict__ part,
                                                             float* __restrict__ grad, int wofs, int bofs) {
  const int per = R * (C + 1);
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (t < per)
    for (int b = grp; b < nblk; b += kBlock / 64) s += (double)part[(int64_t)b * per + t];
  __shared__ double sm[kBlock / 64][64];
  sm[grp][lane] = s;
  __syncthreads();
  if (grp != 0 || t >= per) return;
  double tot = 0.0;
  for (int g = 0; g < kBlock / 64; ++g) tot += sm[g][lane];
  const int r = t / (C + 1), j = t - r * (C + 1);
  if (j < C) grad[wofs + r * C + j] = (float)tot;
  else grad[bofs + r] = (float)tot;
}

__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// --------------------------------------------------------------- launchers
void mlp_forward(int64_t n, const float* X, const float* theta, float* Z, float* A1, float* A2, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_mlp_forward, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, X, theta, Z, A1, A2);
  LAUNCH_CHECK();
}

int64_t mlp_loss_partials(int64_t n) { return cdiv(n, kMlpLossSamples); }

int64_t mlp_loss(int64_t n, const float* Z, const float* E, const float* X, int kind, float* dZ, double* partials,
                 hipStream_t st) {
  upload_tables();
  const int64_t nb = mlp_loss_partials(n);
  if (kind == 1)
    RMG_LAUNCH(k_mlp_loss<true>, dim3(nb), dim3(kBlock), 0, st, n, Z, E, X, dZ, partials);
  else
    RMG_LAUNCH(k_mlp_loss<false>, dim3(nb), dim3(kBlock), 0, st, n, Z, E, X, dZ, partials);
  LAUNCH_CHECK();
  return nb;
}

void mlp_backact(int64_t n, const float* dZ, const float* A1, const float* A2, const float* theta, float* D1,
                 float* D2, hipStream_t st) {
  RMG_LAUNCH(k_mlp_backact, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, dZ, A1, A2, theta, D1, D2);
  LAUNCH_CHECK();
}

int64_t mlp_grad_partials() { return (int64_t)kWgBlocks * kMlpOut * (kMlpH + 1); }

void mlp_weight_grads(int64_t n, const float* X, const float* A1, const float* A2, const float* dZ, const float* D1,
                      const float* D2, float* grad, float* part, hipStream_t st) {
  // samples per block: a whole number of LDS tiles, at most kWgBlocks blocks
  const int64_t per_block = cdiv(cdiv(n, std::min<int64_t>(kWgBlocks, cdiv(n, 256))), kWgS) * kWgS;
  const int nblk = (int)cdiv(n, per_block);
  const int ofs_b1 = kMlpH * kMlpIn, ofs_W2 = ofs_b1 + kMlpH, ofs_b2 = ofs_W2 + kMlpH * kMlpH,
            ofs_W3 = ofs_b2 + kMlpH, ofs_b3 = ofs_W3 + kMlpOut * kMlpH;
  auto reduce = [&](int R, int C, int wofs, int bofs) {
    RMG_LAUNCH(k_mlp_wgrad_reduce, dim3(cdiv(R * (C + 1), 64)), dim3(kBlock), 0, st, R, C, nblk, part, grad,
                       wofs, bofs);
    LAUNCH_CHECK();
  };
  RMG_LAUNCH((k_mlp_wgrad<kMlpOut, kMlpH, 13, 4>), dim3(nblk), dim3(256), 0, st, n, dZ, A2, 1, per_block,
                     part);
  LAUNCH_CHECK();
  reduce(kMlpOut, kMlpH, ofs_W3, ofs_b3);
  RMG_LAUNCH((k_mlp_wgrad<kMlpH, kMlpH, 4, 4>), dim3(nblk), dim3(256), 0, st, n, D2, A1, 1, per_block, part);
  LAUNCH_CHECK();
  reduce(kMlpH, kMlpH, ofs_W2, ofs_b2);
  RMG_LAUNCH((k_mlp_wgrad<kMlpH, kMlpIn, 4, 2>), dim3(nblk), dim3(256), 0, st, n, D1, X, 0, per_block, part);
  LAUNCH_CHECK();
  reduce(kMlpH, kMlpIn, 0, ofs_b1);
}

void mlp_adam(float* theta, const float* grad, float* m, float* v, int t, double lr, hipStream_t st) {
  const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
  RMG_LAUNCH(k_adam, dim3(cdiv(kMlpParams, kBlock)), dim3(kBlock), 0, st, kMlpParams, theta, grad, m, v,
                     (float)lr, c1, c2);
  LAUNCH_CHECK();
}

// ------------------------------------------------------- data extraction
// Cells of the finest level, region by region, x-fastest; cell_off[k] = first cell of region k.
__device__ __forceinline__ int cell_region(const int64_t* __restrict__ cell_off, int nreg, int64_t c) {
  int lo = 0, hi = nreg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell_off[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_cell_features(LevelView L, const int64_t* __restrict__ cell_off,
                                                          int64_t ncell, const float* __restrict__ logc,
                                                          float* __restrict__ X) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int k = cell_region(cell_off, L.nreg, c);
  const RegionGeo R = L.regs[k];
  const int ncx = (R.ex - 1) / 3, ncy = (R.ey - 1) / 3;
  const int64_t lc = c - cell_off[k];
  const int cx = (int)(lc % ncx), cy = (int)((lc / ncx) % ncy), cz = (int)(lc / ((int64_t)ncx * ncy));
  const int ecx = L.cx - 1, ecy = L.cy - 1;
  float v[27];
  float mean = 0.f;
#pragma unroll
  for (int e = 0; e < 27; ++e) {
    const int ex = R.ox + 3 * cx + e % 3, ey = R.oy + 3 * cy + (e / 3) % 3, ez = R.oz + 3 * cz + e / 9;
    v[e] = logc ? logc[((int64_t)ez * ecy + ey) * ecx + ex] : 0.f;
    mean += v[e];
  }
  mean *= (1.0f / 27.0f);
#pragma unroll
  for (int e = 0; e < 27; ++e) X[c * kMlpIn + e] = v[e] - mean;
}

__global__ __launch_bounds__(kBlock) void k_cell_targets(LevelView L, const int64_t* __restrict__ cell_off,
                                                         int64_t ncell, const double* __restrict__ e,
                                                         float* __restrict__ E) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int k = cell_region(cell_off, L.nreg, c);
  const RegionGeo R = L.regs[k];
  const int ncx = (R.ex - 1) / 3, ncy = (R.ey - 1) / 3;
  const int64_t lc = c - cell_off[k];
  const int cx = (int)(lc % ncx), cy = (int)((lc / ncx) % ncy), cz = (int)(lc / ((int64_t)ncx * ncy));
  for (int p = 0; p < 64; ++p) {
    const int x = 3 * cx + p % 4, y = 3 * cy + (p / 4) % 4, z = 3 * cz + p / 16;
    E[c * 64 + p] = (float)e[R.off + ((int64_t)z * R.ey + y) * R.ex + x];
  }
}

void cell_features(const Level& L, const int64_t* cell_off, int64_t ncell, const float* logc, float* X,
                   hipStream_t st) {
  RMG_LAUNCH(k_cell_features, dim3(cdiv(ncell, kBlock)), dim3(kBlock), 0, st, L.view(), cell_off, ncell, logc,
                     X);
  LAUNCH_CHECK();
}

void cell_targets(const Level& L, const int64_t* cell_off, int64_t ncell, const double* e, float* E, hipStream_t st) {
  RMG_LAUNCH(k_cell_targets, dim3(cdiv(ncell, kBlock)), dim3(kBlock), 0, st, L.view(), cell_off, ncell, e, E);
  LAUNCH_CHECK();
}

// ------------------------------------------------- learned weights per node
// One thread per fine node of the finest level: average the predictions of every cell (of any
// region) that contains the node, inject coarse corners, drop weights from Dirichlet coarse
// nodes to free fine nodes, and store them against the corners of the node's canonical cell.
// cellrow maps composite cells (x fastest) to logit rows.
__global__ __launch_bounds__(kBlock) void k_learned_weights(LevelView F, LevelView C, const float* __restrict__ Z,
                                                            const int* __restrict__ cellrow, double* __restrict__ pw) {
  const BlockDesc bd = F.blocks[blockIdx.x];
  const RegionGeo RF = F.regs[bd.region];
  const RegionGeo RC = C.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RF.n) return;
  int x, y, z;
  decompose(RF, li, x, y, z);
  const int gx = RF.ox + x, gy = RF.oy + y, gz = RF.oz + z;
  const int bx = min(x / 3, RC.ex - 2), by = min(y / 3, RC.ey - 2), bz = min(z / 3, RC.ez - 2);
  const int BX = RC.ox + bx, BY = RC.oy + by, BZ = RC.oz + bz;  // composite coarse index of the cell's corner 0
  double acc[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = 0.0;
  const bool fdir = is_dirichlet(F, gx, gy, gz);
  // slots are selected, never used as array indices, so the accumulators stay in registers
  if (gx % 3 == 0 && gy % 3 == 0 && gz % 3 == 0) {
    const int s = (gx / 3 - BX) + 2 * (gy / 3 - BY) + 4 * (gz / 3 - BZ);
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = q == s ? 1.0 : 0.0;
  } else {
    const int ncx = (F.cx - 1) / 3, ncy = (F.cy - 1) / 3, ncz = (F.cz - 1) / 3;
    int cnt = 0;
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          // candidate cell (composite cell index) containing the node
          const int cx = gx / 3 + dx, cy = gy / 3 + dy, cz = gz / 3 + dz;
          if (cx < 0 || cy < 0 || cz < 0 || cx >= ncx || cy >= ncy || cz >= ncz) continue;
          const int px = gx - 3 * cx, py = gy - 3 * cy, pz = gz - 3 * cz;
          if (px > 3 || py > 3 || pz > 3) continue;
          const int node = c_pos2node[(pz * 4 + py) * 4 + px];
          if (node < 0) continue;
          const CellNode nd = c_nodes[node];
          const float* zr = Z + (int64_t)cellrow[((int64_t)cz * ncy + cy) * ncx + cx] * kMlpOut;
          float w[8];
          node_softmax(zr, nd, w);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (k >= nd.ncorner) continue;
            const int cs = nd.corner[k];
            const int s = (cx + (cs & 1) - BX) + 2 * (cy + ((cs >> 1) & 1) - BY) + 4 * (cz + ((cs >> 2) & 1) - BZ);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += q == s ? (double)w[k] : 0.0;
          }
          ++cnt;
        }
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[s] /= (double)max(cnt, 1);
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int X = BX + (s & 1), Y = BY + ((s >> 1) & 1), Zc = BZ + ((s >> 2) & 1);
    double v = acc[s];
    if (!fdir && is_dirichlet(C, X, Y, Zc)) v = 0.0;
    pw[(RF.off + li) * 8 + s] = v;
  }
}

void learned_weights(const Level& F, const Level& C, const float* Z, const int* cellrow, double* pw, hipStream_t st) {
  upload_tables();
  RMG_LAUNCH(k_learned_weights, dim3(F.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), Z, cellrow,
                     pw);
  LAUNCH_CHECK();
}

// ------------------------------------------------ stored weight validation
// Violation flags (WeightFlag): non-finite weights, support beyond the node's face, edge or
// cell, a free fine node interpolating from a Dirichlet coarse node, and weights that do not sum
// to one where no admissible corner is a dropped Dirichlet node.
__global__ __launch_bounds__(kBlock) void k_check_weights(LevelView F, LevelView C, const double* __restrict__ pw,
                                                          int* flag) {
  const BlockDesc bd = F.blocks[blockIdx.x];
  const RegionGeo RF = F.regs[bd.region];
  const RegionGeo RC = C.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  if (li >= RF.n) return;
  int x, y, z;
  decompose(RF, li, x, y, z);
  const int bx = min(x / 3, RC.ex - 2), by = min(y / 3, RC.ey - 2), bz = min(z / 3, RC.ez - 2);
  const int t[3] = {x - 3 * bx, y - 3 * by, z - 3 * bz};
  const bool fdir = is_dirichlet(F, RF.ox + x, RF.oy + y, RF.oz + z);
  int f = 0;
  bool dropped = false;  // some admissible corner is a Dirichlet node (its weight is dropped)
  double sum = 0.0;
  for (int s = 0; s < 8; ++s) {
    const int b[3] = {s & 1, (s >> 1) & 1, (s >> 2) & 1};
    bool admissible = true;
    for (int d = 0; d < 3; ++d)
      if ((t[d] == 0 && b[d] == 1) || (t[d] == 3 && b[d] == 0)) admissible = false;
    const bool cdir = is_dirichlet(C, RC.ox + bx + b[0], RC.oy + by + b[1], RC.oz + bz + b[2]);
    if (admissible && cdir && !fdir) dropped = true;
    const double v = pw[(RF.off + li) * 8 + s];
    if (!isfinite(v)) f |= kWeightNonFinite;
    if (v == 0.0) continue;
    sum += v;
    if (!admissible) f |= kWeightSupport;
    if (cdir && !fdir) f |= kWeightDirichlet;
  }
  if (!dropped && !(fabs(sum - 1.0) <= 1e-6)) f |= kWeightSum;
  if (f) atomicOr(flag, f);
}

// Copies of a shared node must carry the same weight for every composite coarse corner.
__global__ __launch_bounds__(kBlock) void k_check_weight_copies(LevelView F, LevelView C,
                                                                const int64_t* __restrict__ gptr,
                                                                const int* __restrict__ gcopy,
                                                                const int* __restrict__ gcomp, int64_t ng,
                                                                const double* __restrict__ pw, int* flag) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ng) return;
  const int64_t ci = gcomp[g];
  const int gx = (int)(ci % F.cx), gy = (int)((ci / F.cx) % F.cy), gz = (int)(ci / ((int64_t)F.cx * F.cy));
  // composite weights of the first copy, keyed by composite corner offset from (gx/3, gy/3, gz/3) - 1
  double ref[27];
  for (int i = 0; i < 27; ++i) ref[i] = 0.0;
  for (int64_t c = gptr[g]; c < gptr[g + 1]; ++c) {
    const int gi = gcopy[c];
    int k = 0;
    while (k + 1 < F.nreg && F.regs[k + 1].off <= gi) ++k;
    const RegionGeo RF = F.regs[k], RC = C.regs[k];
    const int x = gx - RF.ox, y = gy - RF.oy, z = gz - RF.oz;
    const int bx = min(x / 3, RC.ex - 2), by = min(y / 3, RC.ey - 2), bz = min(z / 3, RC.ez - 2);
    double cur[27];
    for (int i = 0; i < 27; ++i) cur[i] = 0.0;
    for (int s = 0; s < 8; ++s) {
      const int X = RC.ox + bx + (s & 1) - gx / 3 + 1, Y = RC.oy + by + ((s >> 1) & 1) - gy / 3 + 1,
                Z = RC.oz + bz + ((s >> 2) & 1) - gz / 3 + 1;
      if ((unsigned)X > 2u || (unsigned)Y > 2u || (unsigned)Z > 2u) {
        if (pw[(int64_t)gi * 8 + s] != 0.0) atomicOr(flag, (int)kWeightSupport);
        continue;
      }
      cur[(Z * 3 + Y) * 3 + X] = pw[(int64_t)gi * 8 + s];
    }
    for (int i = 0; i < 27; ++i) {
      if (c == gptr[g]) ref[i] = cur[i];
      else if (cur[i] != ref[i]) atomicOr(flag, (int)kWeightCopies);
    }
  }
}

void check_weights(const Level& F, const Level& C, const double* pw, int* flag, hipStream_t st) {
  RMG_LAUNCH(k_check_weights, dim3(F.blocks.size()), dim3(kBlock), 0, st, F.view(), C.view(), pw, flag);
  LAUNCH_CHECK();
  if (F.ngroups > 0) {
    RMG_LAUNCH(k_check_weight_copies, dim3(cdiv(F.ngroups, kBlock)), dim3(kBlock), 0, st, F.view(), C.view(),
                       F.d_gptr.as<int64_t>(), F.d_gcopy.as<int>(), F.d_gcomp.as<int>(), F.ngroups, pw, flag);
    LAUNCH_CHECK();
  }
}

// Log of per-element coefficients (composite element grid) for the MLP features.
__global__ void k_log(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)log(in[i]);
}

void launch_log(int64_t n, const double* in, float* out, hipStream_t st) {
  if (n == 0) return;
  RMG_LAUNCH(k_log, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, n, in, out);
  LAUNCH_CHECK();
}

}  // namespace rmg
