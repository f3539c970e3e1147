// Regional stencil operations: the stencil product z = A^(k) x of every region fused with the
// node update it feeds (matvec, residual, Chebyshev step, CG product), followed by the
// interface-group kernel that sums the partial products of shared nodes over their copies in
// ascending region order (Psi^T Psi, Section 3.1 / the RegMatVec algorithm) and finishes them.
//
// Template parameters: NPTS stencil points, NDOF unknowns per node (3x3 coefficient blocks for
// elasticity), V vector type (double or float), C coefficient storage type (double, float or
// uint16_t = bfloat16; with bfloat16 the centre block comes from an FP32 array).
#include <type_traits>

#include "device_common.h"

namespace rmg {

template <class V>
struct OpP {
  const V* x;
  V* out;
  const V* b;
  const V* dinv;
  V* d;
  V c1, c2;
  const V* dinv9;  // NDOF 3 with nodal blocks: D~^-1 as one row-major 3 x 3 block per node, else null
};

// The Chebyshev / Jacobi update of the three dofs of node `node` with the nodal-block D~^-1:
// r = b - z, dd = c2 (D~^-1 r) (+ c1 dold), out = x + dd; dold the node's previous correction.
template <StencilOp OP, bool DOT, class V>
__device__ __forceinline__ double finish_block3_value(const OpP<V>& p, int64_t node, const V (&z)[3], const V (&xs)[3],
                                                      const V (&dold)[3], V (&out)[3], V (&dd)[3]) {
  const V* __restrict__ D = p.dinv9 + node * 9;
  V r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = p.b[node * 3 + a] - z[a];
  double c = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const V y = D[3 * a] * r[0] + D[3 * a + 1] * r[1] + D[3 * a + 2] * r[2];
    dd[a] = p.c2 * y;
    if constexpr (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst) dd[a] = fma(p.c1, dold[a], dd[a]);
    out[a] = xs[a] + dd[a];
    if constexpr (DOT) c += (double)p.b[node * 3 + a] * (double)out[a];
  }
  return c;
}

// Final update of dof i once z = (Psi^T Psi A x)_i is known; m = multiplicity of its node,
// xself = x_i: the value `out` the operation writes to p.out[i] and, for the Chebyshev steps, the
// new correction `dd`.  Returns the dof's contribution to the fused reduction, if any.
// OWN: the dof belongs to one region, whose centre coefficient `centre` is then the composite
// diagonal: the Chebyshev steps take 1 / centre (the same correctly rounded quotient as the stored
// D~^-1) instead of reading it.
// The Chebyshev steps keep no direction vector: the previous correction d_(k-1) = u_(k-1) - u_(k-2)
// is the difference of the step's input and the iterate before it, which the output buffer holds
// until the step overwrites it (the cycle's two buffers alternate), so a step reads u_(k-2) in
// place of d and writes only u_k.  The step after a zero-guess start (ChebFirst) has u_(k-2) = 0
// and reads nothing for it: its previous correction is u_(k-1) itself.  `dold` is the previous
// correction (shared dofs of a Cheb step: the stencil kernel leaves it in p.d for the interface
// kernel).
template <StencilOp OP, bool DOT, class V, bool OWN = false>
__device__ __forceinline__ double finish_value(const OpP<V>& p, int64_t i, V z, int m, V xself, V centre, V dold,
                                               V& out, V& dd) {
  if constexpr (OP == StencilOp::Matvec) {
    out = z;
    return 0.0;
  } else if constexpr (OP == StencilOp::Residual) {
    out = p.b[i] - z;
    return 0.0;
  } else if constexpr (OP == StencilOp::ResidualScaled) {
    const V r = p.b[i] - z;
    out = (m == 1) ? r : r / (V)m;
    return 0.0;
  } else if constexpr (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst) {
    const V bi = p.b[i];
    const V r = bi - z;
    const V di = OWN ? (V)1 / centre : p.dinv[i];
    dd = p.c2 * (di * r);
    dd = fma(p.c1, dold, dd);  // one rounding in every kernel
    out = xself + dd;
    if constexpr (DOT) return (double)bi * (double)out;
    return 0.0;
  } else {  // CgQ
    out = z;
    return (double)xself * (double)z;
  }
}

// The previous correction of a dof the stencil kernel finishes: x_i - u_(k-2), the latter read from
// the output buffer before it is overwritten (0 for the Jacobi steps, which have c1 = 0).
template <class V>
__device__ __forceinline__ V prev_correction(const OpP<V>& p, V xself, V uprev) {
  return p.c1 != (V)0 ? xself - uprev : (V)0;
}

// The same, written to dof i.
template <StencilOp OP, bool DOT, class V, bool OWN = false>
__device__ __forceinline__ double finish(const OpP<V>& p, int64_t i, V z, int m, V xself, V centre = (V)0) {
  V out, dd = (V)0, dold = (V)0;
  if constexpr (OP == StencilOp::Cheb) dold = prev_correction(p, xself, p.out[i]);
  if constexpr (OP == StencilOp::ChebFirst) dold = xself;
  const double c = finish_value<OP, DOT, V, OWN>(p, i, z, m, xself, centre, dold, out, dd);
  p.out[i] = out;
  return c;
}

// A shared dof's partial product goes to p.out for the interface kernel; a Chebyshev step first
// leaves its previous correction in p.d, since the partial replaces u_(k-2).
template <StencilOp OP, class V>
__device__ __forceinline__ void write_partial(const OpP<V>& p, int64_t i, V z, V xself, V uprev) {
  if constexpr (OP == StencilOp::Cheb) p.d[i] = prev_correction(p, xself, uprev);
  p.out[i] = z;
}

// The same with b_i and u_(k-2) (the output buffer's old value) already in registers (read a
// plane ahead); the arithmetic is finish_value's.
template <StencilOp OP, bool DOT, class V, bool OWN = false>
__device__ __forceinline__ double finish_pre(const OpP<V>& p, int64_t i, V z, int m, V xself, V centre, V bi, V uprev) {
  if constexpr (OP == StencilOp::Residual) {
    p.out[i] = bi - z;
    return 0.0;
  } else if constexpr (OP == StencilOp::ResidualScaled) {
    const V r = bi - z;
    p.out[i] = (m == 1) ? r : r / (V)m;
    return 0.0;
  } else if constexpr (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst) {
    const V r = bi - z;
    const V di = OWN ? (V)1 / centre : p.dinv[i];
    V dd = p.c2 * (di * r);
    if constexpr (OP == StencilOp::Cheb) dd = fma(p.c1, prev_correction(p, xself, uprev), dd);
    if constexpr (OP == StencilOp::ChebFirst) dd = fma(p.c1, xself, dd);
    const V out = xself + dd;
    p.out[i] = out;
    if constexpr (DOT) return (double)bi * (double)out;
    return 0.0;
  } else {
    return finish<OP, DOT, V, OWN>(p, i, z, m, xself, centre);
  }
}

// Coefficient (s, a, b) of node gi; the bfloat16 storage keeps its centre block in FP32.
template <int NPTS, int NDOF, class C>
__device__ __forceinline__ auto coefv(const C* __restrict__ cf, const float* __restrict__ centre, int64_t gi, int s,
                                      int a, int b) {
  if constexpr (sizeof(C) == 2) {
    if (s == center_index<NPTS>()) return centre[gi * NDOF * NDOF + a * NDOF + b];
  }
  return CoefLoad<C>::get(cf + (s * NDOF * NDOF + a * NDOF + b) * kTile);
}

// ---------------------------------------------------------------- node-parallel
// SYM (27-point levels whose operator is symmetric): `coef` holds the upper half of each stencil,
// kSymPts blocks per node; the block of a lower offset s is the transpose of the neighbour's
// upper block at offset 26 - s, read from the neighbour's record (consecutive lanes read
// consecutive records, and the record was streamed moments before by a nearby block).
// table (FP64 27-point symmetric levels, else null): the regions' class tables, used for the
// regions whose flag in table_ok is set: a node's 27 couplings (3 x 3 blocks on 3-dof levels) are
// its class's (the values the half stencil applies, bit for bit), read from the small table
// instead of from its own and its neighbours' records.
template <int NPTS, int NDOF, class V, class C, StencilOp OP, bool DOT, bool SYM>
__global__ __launch_bounds__(kBlock) void k_stencil(LevelView L, const C* __restrict__ coef,
                                                    const float* __restrict__ centre, OpP<V> p,
                                                    double* __restrict__ partials, const double* __restrict__ table,
                                                    const int* __restrict__ table_ok) {
  constexpr int NB = NDOF * NDOF;
  constexpr int NCOEF = SYM ? kSymPts * NB : NPTS * NB;
  constexpr bool kTab = NPTS == 27 && SYM && std::is_same<V, double>::value && std::is_same<C, double>::value;
  // every XCD runs a contiguous run of node blocks, so a block finds the records of the plane below
  // (its lower couplings on symmetric levels) in its own XCD's L2; its partial sum goes to the
  // node block's slot, as without the mapping
  const int blk = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const BlockDesc bd = L.blocks[blk];
  const RegionGeo R = L.regs[bd.region];
  const int li = bd.start + (int)threadIdx.x;
  double contrib = 0.0;
  if (li < R.n) {
    int x, y, z;
    decompose(R, li, x, y, z);
    const int64_t gi = R.off + li;
    const V* __restrict__ xr = p.x + R.off * NDOF;
    const C* __restrict__ cf = coef + coef_index(gi, 0, NCOEF);
    const int sy = R.ex, sz = R.ex * R.ey;
    const bool inner = x > 0 && x < R.ex - 1 && y > 0 && y < R.ey - 1 && (NPTS != 27 || (z > 0 && z < R.ez - 1));
    const bool tabbed = kTab && table && table_ok[bd.region];  // uniform over the block (one region)
    const double* __restrict__ tc =
        tabbed ? table + ((int64_t)bd.region * kClasses +
                          (axis_class(z, R.ez) * 5 + axis_class(y, R.ey)) * 5 + axis_class(x, R.ex)) * kClassPts * NB
               : nullptr;
    V acc[NDOF];
#pragma unroll
    for (int a = 0; a < NDOF; ++a) acc[a] = (V)0;
#pragma unroll
    for (int s = 0; s < NPTS; ++s) {
      int dx, dy, dz;
      stencil_offset<NPTS>(s, dx, dy, dz);
      const bool ok = inner || ((unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                                (unsigned)(z + dz) < (unsigned)R.ez);
      if (ok) {
        const int nb = li + dx + dy * sy + dz * sz;
        if constexpr (SYM) {
          if (kTab && tabbed) {
#pragma unroll
            for (int a = 0; a < NDOF; ++a)
#pragma unroll
              for (int b = 0; b < NDOF; ++b) acc[a] += (V)tc[(s * NDOF + a) * NDOF + b] * xr[nb * NDOF + b];
          } else if (s >= 13) {
#pragma unroll
            for (int a = 0; a < NDOF; ++a)
#pragma unroll
              for (int b = 0; b < NDOF; ++b) {
                V c;
                if (sizeof(C) == 2 && s == 13) c = (V)centre[gi * NB + a * NDOF + b];
                else c = (V)CoefLoad<C>::get(cf + ((s - 13) * NB + a * NDOF + b) * kTile);
                acc[a] += c * xr[nb * NDOF + b];
              }
          } else {
            const C* __restrict__ cn = coef + coef_index(R.off + nb, 0, NCOEF);
#pragma unroll
            for (int a = 0; a < NDOF; ++a)
#pragma unroll
              for (int b = 0; b < NDOF; ++b)
                acc[a] += (V)CoefLoad<C>::get(cn + ((13 - s) * NB + b * NDOF + a) * kTile) * xr[nb * NDOF + b];
          }
        } else {
#pragma unroll
          for (int a = 0; a < NDOF; ++a)
#pragma unroll
            for (int b = 0; b < NDOF; ++b)
              acc[a] += (V)coefv<NPTS, NDOF, C>(cf, centre, gi, s, a, b) * xr[nb * NDOF + b];
        }
      }
    }
    if (!inner && is_shared(L, R, x, y, z)) {
#pragma unroll
      for (int a = 0; a < NDOF; ++a)  // summed over copies by k_iface
        write_partial<OP, V>(p, gi * NDOF + a, acc[a], xr[li * NDOF + a], p.out[gi * NDOF + a]);
    } else {
      bool block = false;
      if constexpr (NDOF == 3 && (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst)) {
        if (p.dinv9) {
          V xs[3], dold[3], out[3], dd[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            xs[a] = xr[li * 3 + a];
            dold[a] = OP == StencilOp::Cheb ? prev_correction(p, xs[a], p.out[gi * 3 + a]) : xs[a];
          }
          contrib += finish_block3_value<OP, DOT, V>(p, gi, acc, xs, dold, out, dd);
#pragma unroll
          for (int a = 0; a < 3; ++a) p.out[gi * 3 + a] = out[a];
          block = true;
        }
      }
      if (!block) {
#pragma unroll
        for (int a = 0; a < NDOF; ++a) contrib += finish<OP, DOT, V>(p, gi * NDOF + a, acc[a], 1, xr[li * NDOF + a]);
      }
    }
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    const double s = block_sum(contrib);
    if (threadIdx.x == 0) partials[blk] = s;
  }
}

// ------------------------------------------------ 3D scalar stencil, 2.5D tiles
// A block owns a tile of ty x-rows (tx nodes each) of one region and marches nz planes in z.
// The input vector's planes pass through two LDS slots; each thread keeps its 3x3
// neighbourhood of planes z-1, z, z+1 in registers (rotated per plane), so it reads only the
// new plane from LDS, and the plane after next is prefetched from global memory into registers
// while the current plane is computed.  Neighbours outside the region box read 0 from LDS and
// have zero coefficients, so the 27-term sum needs no bounds branches.

// Grid = one block per tile, or (persistent launch) fewer blocks that stride over the tile list.
// SYM: the operator is symmetric and `coef` holds only the upper half of each stencil (offsets
// s = 13..26 of the 27-point order, kSymPts per node, wave-tiled); a lower coupling A(i, i+s),
// s < 13, is the upper coupling A(i+s, i) stored with node i+s at offset 26 - s.  Each thread
// streams its node's 14 couplings once and leaves the ones its neighbours need in LDS: the
// couplings towards z+1 for the next plane, the in-plane ones for this plane.  Only neighbours
// outside the tile (its edge rows, and plane z-1 of the tile's first plane) are read from memory,
// so HBM carries about 14 instead of 27 coefficients per node.
// NT threads per block (the level's tile_threads); tiles hold at most NT nodes.
template <int NT, class V, class C, StencilOp OP, bool DOT, bool SYM>
__global__ __launch_bounds__(NT) void k_stencil3d(LevelView L, const Tile3* __restrict__ tiles, int ntiles,
                                                  const C* __restrict__ coef, const float* __restrict__ centre,
                                                  OpP<V> p, double* __restrict__ partials) {
  constexpr int kT3 = NT;
  constexpr int kT3Plane = tile_plane_cap(NT);
  constexpr int kT3Fetch = (kT3Plane + kT3 - 1) / kT3;
  // Chebyshev steps compute D~^-1 of one-region nodes from the centre coefficient when it is stored
  // in the arithmetic's own type (FP64, or the FP32 copy); the BF16 storage's centre carries the
  // row-sum correction, so it keeps reading the stored reciprocal
  constexpr bool kOwnDiag = std::is_same<V, C>::value && (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst);
  __shared__ V pl[2][kT3Plane];
  // SYM: the previous plane's couplings towards z+1 (9 per tile node) and this plane's in-plane upper
  // couplings (4 per tile node), indexed by the tile-local node = thread index
  __shared__ C sprev[SYM ? 9 : 1][SYM ? kT3 : 1];
  __shared__ C srow[SYM ? 4 : 1][SYM ? kT3 : 1];
  const int t = threadIdx.x;
  double contrib = 0.0;
  // one tile per block: every XCD runs a contiguous run of tiles (xcd_item), so neighbouring
  // tiles' halo rows meet in its L2; persistent grids stride over the tiles
  const bool one = (int)gridDim.x == ntiles;
  for (int it = blockIdx.x; it < ntiles; it += gridDim.x) {
    const Tile3 T = tiles[one ? xcd_item(it, ntiles) : it];
    const RegionGeo R = L.regs[T.region];
    const int W = T.tx + 2, PL = (T.ty + 2) * W;
    const V* __restrict__ xr = p.x + R.off;
    const int ty = t / T.tx, tx = t - ty * T.tx;
    const int x = T.x0 + tx, y = T.y0 + ty;
    const bool active = ty < T.ty && x < R.ex && y < R.ey;
    const int sy = R.ex, sz = R.ex * R.ey;
    V pre[kT3Fetch];
    auto fetch = [&](int zz) {
#pragma unroll
      for (int k = 0; k < kT3Fetch; ++k) {
        const int idx = t + k * kT3;
        V v = (V)0;
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
    V rm[9], rc[9], rp[9];
    auto readn = [&](int slot, V* r) {
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int dx = j % 3 - 1, dy = j / 3 - 1;
        r[j] = pl[slot][(ty + 1 + dy) * W + tx + 1 + dx];
      }
    };
    const int z0 = T.z0, z1 = T.z0 + T.nz;
    // SYM: b and the old direction of this thread's node on the next plane, read a plane ahead
    constexpr bool kPreB = SYM && (OP == StencilOp::Residual || OP == StencilOp::ResidualScaled ||
                                   OP == StencilOp::Cheb || OP == StencilOp::ChebFirst);
    constexpr bool kPreD = SYM && OP == StencilOp::Cheb;
    V nb = (V)0, nd = (V)0;
    auto load_bd = [&](int z2) {
      if (active && z2 < z1) {
        const int64_t g = R.off + (int64_t)z2 * sz + (int64_t)y * sy + x;
        if constexpr (kPreB) nb = p.b[g];
        if constexpr (kPreD) nd = p.out[g];  // u_(k-2), see finish_value
      }
    };
    if constexpr (kPreB) load_bd(z0);
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
    for (int zz = z0; zz < z1; ++zz) {
      const int sp = (zz - z0) & 1;  // slot holding plane zz+1
      const V cb = nb, cd = nd;
      if constexpr (kPreB) load_bd(zz + 1);
      if (active) readn(sp, rp);
      fetch(zz + 2);
      // SYM: own upper couplings u[k] = A(i, i + offset(13 + k)); lower couplings lo[s] = A(i, i +
      // offset(s)) = A(i + offset(s), i), from LDS when the neighbour is a node of this tile (and,
      // for z-1, when this tile computed that plane), else from the neighbour's record in memory.
      V up[SYM ? kSymPts : 1], lo[SYM ? 13 : 1];
      if constexpr (SYM) {
        const int li = zz * sz + y * sy + x;
        const int64_t gi = R.off + li;
        const bool inner = x > 0 && x < R.ex - 1 && y > 0 && y < R.ey - 1 && zz > 0 && zz < R.ez - 1;
        auto nb_ok = [&](int dx, int dy, int dz) {
          return inner || ((unsigned)(x + dx) < (unsigned)R.ex && (unsigned)(y + dy) < (unsigned)R.ey &&
                           (unsigned)(zz + dz) < (unsigned)R.ez);
        };
        auto in_tile = [&](int dx, int dy) {
          return (unsigned)(tx + dx) < (unsigned)T.tx && (unsigned)(ty + dy) < (unsigned)T.ty;
        };
        auto mirror = [&](int s, int dx, int dy, int dz) {  // A(i + offset(s), i) from memory
          return (V)CoefLoad<C>::get(coef + coef_index(gi + dx + dy * sy + dz * sz, 13 - s, kSymPts));
        };
        if (active) {
          const C* __restrict__ cf = coef + coef_index(gi, 0, kSymPts);
#pragma unroll
          for (int k = 0; k < kSymPts; ++k) up[k] = (V)CoefLoad<C>::get(cf + k * kTile);
#pragma unroll
          for (int s = 0; s < 9; ++s) {  // z-1: the neighbour's coupling towards z+1
            const int dx = s % 3 - 1, dy = s / 3 - 1;
            V v = (V)0;
            if (nb_ok(dx, dy, -1)) v = (zz > z0 && in_tile(dx, dy)) ? (V)sprev[8 - s][t + dx + dy * T.tx] : mirror(s, dx, dy, -1);
            lo[s] = v;
          }
#pragma unroll
          for (int k = 1; k < 5; ++k) srow[k - 1][t] = (C)up[k];
        }
        __syncthreads();  // srow visible; every read of sprev done
        if (active) {
#pragma unroll
          for (int k = 5; k < kSymPts; ++k) sprev[k - 5][t] = (C)up[k];
#pragma unroll
          for (int s = 9; s < 13; ++s) {  // in-plane lower couplings
            int dx, dy, dz;
            stencil_offset<27>(s, dx, dy, dz);
            V v = (V)0;
            if (nb_ok(dx, dy, 0)) v = in_tile(dx, dy) ? (V)srow[12 - s][t + dx + dy * T.tx] : mirror(s, dx, dy, 0);
            lo[s] = v;
          }
        }
      }
      if (active) {
        const int li = zz * sz + y * sy + x;
        const int64_t gi = R.off + li;
        V acc = (V)0, ctr = (V)0;  // ctr: centre coefficient (the diagonal of a one-region node)
        if constexpr (SYM) {
          // stencil order, one rounding each (as k_stencil_table sums them)
#pragma unroll
          for (int s = 0; s < 27; ++s) {
            const int j = s % 9;
            acc = fma(s < 13 ? lo[s] : up[s - 13], s < 9 ? rm[j] : (s < 18 ? rc[j] : rp[j]), acc);
          }
          ctr = up[0];
        } else {
          const C* __restrict__ cf = coef + coef_index(gi, 0, 27);
#pragma unroll
          for (int s = 0; s < 27; ++s) {
            const int j = s % 9, dz = s / 9 - 1;
            const V v = dz < 0 ? rm[j] : (dz == 0 ? rc[j] : rp[j]);
            const V cv = (V)coefv<27, 1, C>(cf, centre, gi, s, 0, 0);
            if (s == 13) ctr = cv;
            acc += cv * v;
          }
        }
        const bool edge = x == 0 || x == R.ex - 1 || y == 0 || y == R.ey - 1 || zz == 0 || zz == R.ez - 1;
        if (edge && is_shared(L, R, x, y, zz)) {  // finished by k_iface
          if constexpr (kPreD) write_partial<OP, V>(p, gi, acc, rc[4], cd);
          else write_partial<OP, V>(p, gi, acc, rc[4], OP == StencilOp::Cheb ? p.out[gi] : (V)0);
        } else if constexpr (kPreB) contrib += finish_pre<OP, DOT, V, kOwnDiag>(p, gi, acc, 1, rc[4], ctr, cb, cd);
        else contrib += finish<OP, DOT, V, kOwnDiag>(p, gi, acc, 1, rc[4], ctr);
      }
      store(sp ^ 1);  // plane zz+2 replaces plane zz
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        rm[j] = rc[j];
        rc[j] = rp[j];
      }
      __syncthreads();
    }
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
      // one tile per block: the tile's slot, as without the mapping
      partials[one ? xcd_item((int)blockIdx.x, ntiles) : (int)blockIdx.x] = s;
    }
  }
}

// ------------------------------------------------------- region-table tiles

// Whole-region tiles of a region served by its class tables: ty full x-rows, nz planes.  The lanes
// of the rows' inner nodes (x in [2, ex - 2)) come first, padded to whole wavefronts, then the rows'
// four x-face nodes.  A node's couplings are its class's (scalar loads from the region's table): a
// wavefront takes the classes of its nodes one after the other, so one whose nodes share a class
// (every inner wavefront away from the y-faces) runs one pass.  No coupling is read per node.  The
// input vector's planes, whole rows with their halo, pass through two LDS slots; each plane is
// fetched four planes ahead into registers and b and u_(k-2) two planes ahead, so that two planes'
// loads are in flight while one is computed, and each plane read adds its products to the running
// sums of the three nodes it neighbours in z.  The kernel is held to 80 VGPRs (six waves per SIMD,
// three 8-wave blocks per CU), at the cost of one spilled register in the Chebyshev step; the
// variant that also sums (b, u_out) keeps five waves, where it needs no spill.  Blocks
// are mapped to tiles so that every XCD runs a contiguous run of tiles (xcd_item) and neighbouring
// tiles share their halo rows through its L2.  Every node sums its 27 products in stencil order with
// one rounding each, as k_stencil3d does, so the results are those of streaming every coupling bit
// for bit.
template <StencilOp OP, bool DOT>
__global__ __launch_bounds__(kTableThreads) __attribute__((amdgpu_waves_per_eu(DOT ? 5 : 6))) void k_stencil_table(LevelView L, const Tile3* __restrict__ tiles,
                                                                 const double* __restrict__ table, OpP<double> p,
                                                                 double* __restrict__ partials) {
  constexpr int NT = kTableThreads;
  constexpr int kPlane = 2 * NT;  // a tile's rows with their halo: two loads per lane (make_split)
  constexpr int kFetch = 2;
  constexpr bool kPreB = OP == StencilOp::Residual || OP == StencilOp::ResidualScaled || OP == StencilOp::Cheb ||
                         OP == StencilOp::ChebFirst;
  constexpr bool kPreD = OP == StencilOp::Cheb;
  constexpr int kXRows = 4 * kTableRows;  // x-face lanes: four a row
  __shared__ double pl[2][kPlane];
  __shared__ double xt[5][kClassPts][kXRows];  // the x-face lanes' couplings by z class
  const Tile3 T = tiles[xcd_item((int)blockIdx.x, (int)gridDim.x)];
  const RegionGeo R = L.regs[T.region];
  const double* __restrict__ tab = table + (int64_t)T.region * kClasses * kClassPts;
  const int t = threadIdx.x;
  // lane -> (row, x): inner-x lanes, padded to a wavefront boundary, then x-face lanes
  const int dxw = R.ex - 4, ndl = T.ty * dxw, pad = (ndl + 63) & ~63;
  int row = 0, x = 0;
  bool active = false;
  if (t < ndl) {
    row = t / dxw;
    x = 2 + t - row * dxw;
    active = true;
  } else if (t >= pad && t < pad + 4 * T.ty) {
    const int u = t - pad;
    row = u >> 2;
    x = (u & 3) < 2 ? (u & 3) : R.ex - 4 + (u & 3);
    active = true;
  }
  const int y = T.y0 + row;
  const int cxy = axis_class(y, R.ey) * 5 + axis_class(x, R.ex);
  const int W = R.ex + 2, PL = (T.ty + 2) * W;
  const int sy = R.ex, sz = R.ex * R.ey;
  const double* __restrict__ xr = p.x + R.off;
  // Loads are issued unconditionally (out-of-range positions read a valid element and are zeroed
  // when stored), so that the compiler counts the loads in flight exactly and waits only for the
  // plane it needs.
  auto fetch = [&](int zz, double(&pre)[kFetch]) {
    const int zc = min(max(zz, 0), R.ez - 1);
#pragma unroll
    for (int k = 0; k < kFetch; ++k) {
      const int idx = min(t + k * NT, PL - 1);
      const int r = idx / W;
      const int xx = min(max(idx - r * W - 1, 0), R.ex - 1), yy = min(max(T.y0 - 1 + r, 0), R.ey - 1);
      pre[k] = xr[(int64_t)zc * sz + (int64_t)yy * sy + xx];
    }
  };
  auto store = [&](int slot, int zz, const double(&pre)[kFetch]) {
#pragma unroll
    for (int k = 0; k < kFetch; ++k) {
      const int idx = t + k * NT;
      if (idx < PL) {
        const int r = idx / W;
        const int xx = idx - r * W - 1, yy = T.y0 - 1 + r;
        const bool in = (unsigned)zz < (unsigned)R.ez && (unsigned)yy < (unsigned)R.ey && (unsigned)xx < (unsigned)R.ex;
        pl[slot][idx] = in ? pre[k] : 0.0;
      }
    }
  };
  double v9[9];  // this lane's 3 x 3 neighbourhood on the plane read last
  auto readn = [&](int slot) {
#pragma unroll
    for (int j = 0; j < 9; ++j) v9[j] = pl[slot][(row + j / 3) * W + x + j % 3];
  };
  const int z0 = T.z0, z1 = T.z0 + T.nz;
  auto load_bd = [&](int z2, double& b2, double& d2) {  // inactive lanes and planes past the tile: a valid node
    const int64_t g = R.off + (int64_t)min(z2, z1 - 1) * sz + (int64_t)y * sy + x;
    if constexpr (kPreB) b2 = p.b[g];
    if constexpr (kPreD) d2 = p.out[g];  // u_(k-2), see finish_value
  };
  for (int e = t; e < 5 * kClassPts * kXRows; e += NT) {  // couplings of the x-face lanes' classes
    const int u = e % kXRows, s2 = e / kXRows % kClassPts, cz = e / (kXRows * kClassPts);
    const int yu = min(T.y0 + (u >> 2), R.ey - 1), xu = (u & 3) < 2 ? (u & 3) : R.ex - 4 + (u & 3);
    xt[cz][s2][u] = tab[((cz * 5 + axis_class(yu, R.ey)) * 5 + axis_class(xu, R.ex)) * kClassPts + s2];
  }
  // Running sums: once plane q has been added, a0 is node q - 1's sum, a1 node q's and a2 node
  // q + 1's.  A plane adds its nine values to the three nodes it neighbours in z (as their plane
  // z + 1, z and z - 1), so each node adds its 27 products in stencil order with one rounding each,
  // and only the plane read last is held in registers.
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, ctr = 0.0, xprev = 0.0;
  auto czc = [&](int z) { return min(max(axis_class(z, R.ez), 0), 4); };
  auto add_plane = [&](int q) {
    a2 = 0.0;
    if (t >= pad) {
      // the x-face wavefront (four classes a row): each lane reads its class's couplings from
      // the block's copy in LDS, nine at a time (the empty asm keeps the chunks' reads apart)
      const int u = t - pad;
      auto chunk = [&](const double* __restrict__ xc, double& acc) {
        double cf[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) cf[j] = xc[j * kXRows];
#pragma unroll
        for (int j = 0; j < 9; ++j) acc = fma(cf[j], v9[j], acc);
        __asm__ volatile("" ::: "memory");
      };
      chunk(&xt[czc(q - 1)][18][u], a0);
      chunk(&xt[czc(q)][9][u], a1);
      chunk(&xt[czc(q + 1)][0][u], a2);
      ctr = xt[czc(q - 1)][13][u];
    } else {
      // the classes of this wavefront's nodes, one after the other (the mask of lanes left and the
      // leading lane are wavefront-uniform, so every pass reads its class afresh)
      uint64_t left = __builtin_amdgcn_ballot_w64(true);
      while (left) {
        const int c = __builtin_amdgcn_readlane(cxy, (int)__builtin_ctzll(left));
        // the three classes' table offsets, in scalar registers the compiler cannot trade for
        // per-lane values below, so that the table is read with scalar loads
        int o0 = __builtin_amdgcn_readfirstlane((czc(q - 1) * 25 + c) * kClassPts);
        int o1 = __builtin_amdgcn_readfirstlane((czc(q) * 25 + c) * kClassPts);
        int o2 = __builtin_amdgcn_readfirstlane((czc(q + 1) * 25 + c) * kClassPts);
        __asm__ volatile("" : "+s"(o0), "+s"(o1), "+s"(o2));
        const bool mine = cxy == c;
        if (mine) {
          const double* __restrict__ t0 = tab + o0;
          const double* __restrict__ t1 = tab + o1;
          const double* __restrict__ t2 = tab + o2;
#pragma unroll
          for (int j = 0; j < 9; ++j) a0 = fma(t0[18 + j], v9[j], a0);
#pragma unroll
          for (int j = 0; j < 9; ++j) a1 = fma(t1[9 + j], v9[j], a1);
#pragma unroll
          for (int j = 0; j < 9; ++j) a2 = fma(t2[j], v9[j], a2);
          ctr = t0[13];
        }
        left &= ~__builtin_amdgcn_ballot_w64(mine);
      }
    }
  };
  auto shift = [&]() {
    a0 = a1;
    a1 = a2;
    xprev = v9[4];
  };
  double preA[kFetch], preB[kFetch];
  double nbA = 0.0, ndA = 0.0, nbB = 0.0, ndB = 0.0;
  load_bd(z0, nbA, ndA);
  load_bd(z0 + 1, nbB, ndB);
  fetch(z0 - 1, preA);
  fetch(z0, preB);
  store(0, z0 - 1, preA);
  store(1, z0, preB);
  __syncthreads();
  if (active) {  // planes z0 - 1 and z0: the first two thirds of node z0, the first of z0 + 1
    readn(0);
    add_plane(z0 - 1);
    shift();
    readn(1);
    add_plane(z0);
    shift();
  }
  __syncthreads();
  fetch(z0 + 1, preA);
  store(0, z0 + 1, preA);
  fetch(z0 + 2, preA);
  fetch(z0 + 3, preB);
  __syncthreads();
  double contrib = 0.0;
  // one plane: plane zz + 1 from LDS completes node zz; plane zz + 2 goes to LDS from the
  // registers that fetched it two planes ago, which then fetch plane zz + 4 (past the tile's last
  // plane it only keeps the loads in step: see the loop below)
  auto plane = [&](int zz, double(&pre)[kFetch], double& b2, double& d2) {
    const int sp = (zz - z0) & 1;  // slot holding plane zz + 1
    const bool work = active && zz < z1;
    if (work) readn(sp);
    if (zz + 2 <= z1) store(sp ^ 1, zz + 2, pre);  // plane zz + 2 replaces plane zz
    fetch(zz + 4, pre);
    const double cb = b2, cd = d2;
    load_bd(zz + 2, b2, d2);
    if (work) {
      add_plane(zz + 1);
      const int64_t gi = R.off + (int64_t)zz * sz + (int64_t)y * sy + x;
      const bool edge = x == 0 || x == R.ex - 1 || y == 0 || y == R.ey - 1 || zz == 0 || zz == R.ez - 1;
      if (edge && is_shared(L, R, x, y, zz)) write_partial<OP, double>(p, gi, a0, xprev, cd);  // finished by k_iface
      else if constexpr (kPreB) contrib += finish_pre<OP, DOT, double, true>(p, gi, a0, 1, xprev, ctr, cb, cd);
      else contrib += finish<OP, DOT, double, true>(p, gi, a0, 1, xprev, ctr);
      shift();
    }
    __syncthreads();
  };
  // Both halves run on every pass, also past the last plane, so that every pass issues the same
  // loads and the compiler's count of loads in flight stays exact around the loop.
  for (int zz = z0; zz < z1; zz += 2) {
    plane(zz, preA, nbA, ndA);
    plane(zz + 1, preB, nbB, ndB);
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    double v = contrib;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __shared__ double sm[NT / 64];
    if ((t & 63) == 0) sm[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int i = 0; i < NT / 64; ++i) s += sm[i];
      partials[blockIdx.x] = s;
    }
  }
}

// ----------------------------------------------------------- interface groups
// ng2: the first ng2 groups have two copies each (their copies start at 2 g, no gptr read).
template <int NDOF, class V, StencilOp OP, bool DOT>
__global__ __launch_bounds__(kBlock) void k_iface(const int64_t* __restrict__ gptr, const int* __restrict__ gcopy,
                                                  int64_t ng, int64_t ng2, OpP<V> p, double* __restrict__ partials) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double contrib = 0.0;
  if (g < ng) {
    const bool two = g < ng2;
    const int64_t a0 = two ? 2 * g : gptr[g], e = two ? a0 + 2 : gptr[g + 1];
    const int m = (int)(e - a0);
    bool block = false;
    if constexpr (NDOF == 3 && (OP == StencilOp::Cheb || OP == StencilOp::ChebFirst)) {
      if (p.dinv9) {  // nodal blocks: the node's three sums first, then the block update
        const int64_t n0 = gcopy[a0];
        V z[3], xs[3], dold[3], out[3], dd[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          V s = (V)0;
          for (int64_t c = a0; c < e; ++c) s += p.out[(int64_t)gcopy[c] * 3 + a];
          z[a] = s;
          xs[a] = p.x[n0 * 3 + a];
          // Cheb: left in p.d by the stencil kernel; ChebFirst: u_(k-1) itself
          dold[a] = OP == StencilOp::Cheb ? p.d[n0 * 3 + a] : xs[a];
        }
        contrib += finish_block3_value<OP, DOT, V>(p, n0, z, xs, dold, out, dd);
        for (int64_t c = a0; c < e; ++c) {
          const int64_t i = (int64_t)gcopy[c] * 3;
#pragma unroll
          for (int a = 0; a < 3; ++a) p.out[i + a] = out[a];
        }
        block = true;
      }
    }
#pragma unroll
    for (int a = 0; a < NDOF; ++a) {
      if (block) break;
      V s = (V)0;
      for (int64_t c = a0; c < e; ++c) s += p.out[(int64_t)gcopy[c] * NDOF + a];
      // the copies of a composite dof hold equal b, x, D~^-1 and previous correction (consistent
      // regional vectors), so the update is computed from the first copy (the lowest region, which
      // owns the dof) and written to every copy
      const int64_t i0 = (int64_t)gcopy[a0] * NDOF + a;
      V out, dd = (V)0;
      const V xs0 = p.x[i0];
      const V dold = OP == StencilOp::Cheb ? p.d[i0] : xs0;  // Cheb: left in p.d by the stencil kernel
      contrib += finish_value<OP, DOT, V>(p, i0, s, m, xs0, (V)0, dold, out, dd);
      for (int64_t c = a0; c < e; ++c) p.out[(int64_t)gcopy[c] * NDOF + a] = out;
    }
  }
  if constexpr (DOT || OP == StencilOp::CgQ) {
    const double s = block_sum(contrib);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ dispatch
template <int NPTS, int NDOF, class V, class C, StencilOp OP, bool DOT>
static int64_t run(const Level& L, const StencilArgs& a, hipStream_t st) {
  OpP<V> p{static_cast<const V*>(a.x), static_cast<V*>(a.out), static_cast<const V*>(a.b),
           static_cast<const V*>(a.dinv), static_cast<V*>(a.d), (V)a.c1, (V)a.c2,
           static_cast<const V*>(a.dinv9)};
  const C* coef = a.lowp ? L.coef_lo.as<C>() : L.coef.as<C>();
  const float* centre = L.center_lo.as<float>();
  const LevelView v = L.view();
  const bool tiled = NPTS == 27 && NDOF == 1 && L.use_tiles;
  const int ntiles = (int)L.tiles.size();
  const int grid3 = (L.tile_grid > 0 && L.tile_grid < ntiles) ? L.tile_grid : ntiles;
  int64_t nparts = grid3;  // partial sums written by the tiled launches
  if (a.ev0) RMG_HIP(hipEventRecord(a.ev0, st));
  if constexpr (NPTS == 27 && NDOF == 1) {
    if (tiled) {
      const C* sym = nullptr;
      const C* table = nullptr;
      if constexpr (std::is_same<V, C>::value) {
        sym = static_cast<const C*>(a.lowp ? L.coef_lo_sym.p : L.coef_sym.p);
        // the class tables serve the FP64 operator on 768-thread tiles
        if (!a.lowp && L.tile_threads == kTileThreadsF64 && L.class_table.p && L.class_table_ok.p)
          table = static_cast<const C*>(L.class_table.p);
      }
      bool split = false;
      if constexpr (std::is_same<V, double>::value && std::is_same<C, double>::value) {
        if (table && sym && L.tile_threads == kTileThreadsF64 && !L.table_tiles.empty()) {
          // region-table split: the served regions' whole-region tiles, then the other regions'
          // tiles, each with its own run of partial sums
          const int64_t nd = (int64_t)L.table_tiles.size(), no = (int64_t)L.other_tiles.size();
          RMG_REQUIRE(L.table_served.size() == (size_t)L.nreg, RMG_ERR_ARG, "internal: class tables without their split");
          RMG_LAUNCH((k_stencil_table<OP, DOT>), dim3(nd), dim3(kTableThreads), 0, st, v, L.d_table_tiles.as<Tile3>(),
                     table, p, a.partials);
          if (no > 0)
            RMG_LAUNCH((k_stencil3d<kTileThreadsF64, V, C, OP, DOT, true>), dim3(no), dim3(kTileThreadsF64), 0, st,
                       v, L.d_other_tiles.as<Tile3>(), (int)no, sym, centre, p,
                       a.partials ? a.partials + nd : nullptr);
          nparts = nd + no;
          split = true;
        }
      }
      auto launch3d = [&](auto nt) {
        constexpr int NT = decltype(nt)::value;
        if (sym) {
          if constexpr (std::is_same<V, C>::value) {
            RMG_LAUNCH((k_stencil3d<NT, V, C, OP, DOT, true>), dim3(grid3), dim3(NT), 0, st, v,
                               L.d_tiles.as<Tile3>(), ntiles, sym, centre, p, a.partials);
          }
        } else {
          RMG_LAUNCH((k_stencil3d<NT, V, C, OP, DOT, false>), dim3(grid3), dim3(NT), 0, st, v,
                             L.d_tiles.as<Tile3>(), ntiles, coef, centre, p, a.partials);
        }
      };
      if (split) {
      } else if constexpr (sizeof(V) == 8) {
        if (L.tile_threads == kTileThreadsF64) launch3d(std::integral_constant<int, kTileThreadsF64>());
        else launch3d(std::integral_constant<int, kTileThreadsF32>());
      } else {
        RMG_REQUIRE(L.tile_threads == kTileThreadsF32, RMG_ERR_ARG, "internal: FP32 tiles must be narrow");
        launch3d(std::integral_constant<int, kTileThreadsF32>());
      }
    }
  }
  if (!tiled) {
    const C* symc = static_cast<const C*>(a.lowp ? L.coef_lo_sym.p : L.coef_sym.p);
    // the class tables of an FP64 level run by node blocks
    const bool ntab = !a.lowp && NPTS == 27 && L.class_table.p && L.class_table_ok.p;
    const double* ntable = ntab ? L.class_table.as<double>() : nullptr;
    const int* ntable_ok = ntab ? L.class_table_ok.as<int>() : nullptr;
    auto node = [&](const LevelView& vk, int nblocks, double* part) {
      if constexpr (NPTS == 27) {
        if (symc) {
          RMG_LAUNCH((k_stencil<NPTS, NDOF, V, C, OP, DOT, true>), dim3(nblocks), dim3(kBlock), 0, st, vk,
                             symc, centre, p, part, ntable, ntable_ok);
          return;
        }
      }
      RMG_LAUNCH((k_stencil<NPTS, NDOF, V, C, OP, DOT, false>), dim3(nblocks), dim3(kBlock), 0, st, vk, coef,
                         centre, p, part, nullptr, nullptr);
    };
    if (L.per_region) {
      // unbatched: one launch per region over its slice of the block table (partials keep their slots)
      for (int k = 0; k < L.nreg; ++k) {
        const int b0 = L.region_block[k], b1 = L.region_block[k + 1];
        if (b1 == b0) continue;
        LevelView vk = v;
        vk.blocks = v.blocks + b0;
        vk.nblocks = b1 - b0;
        node(vk, b1 - b0, a.partials ? a.partials + b0 : nullptr);
      }
    } else {
      node(v, (int)L.blocks.size(), a.partials);
    }
  }
  LAUNCH_CHECK();
  if (a.ev1) RMG_HIP(hipEventRecord(a.ev1, st));
  const int64_t nb = tiled ? nparts : (int64_t)L.blocks.size();
  int64_t ngb = 0;
  if (L.ngroups > 0) {
    ngb = cdiv(L.ngroups, kBlock);
    RMG_LAUNCH((k_iface<NDOF, V, OP, DOT>), dim3(ngb), dim3(kBlock), 0, st, L.d_gptr.as<int64_t>(),
                       L.d_gcopy.as<int>(), L.ngroups, L.ngroups2, p, a.partials ? a.partials + nb : nullptr);
    LAUNCH_CHECK();
  }
  return (DOT || OP == StencilOp::CgQ) ? nb + ngb : 0;
}

// FP64: every operation.
template <int NPTS, int NDOF>
static int64_t ops_f64(const Level& L, const StencilArgs& a, hipStream_t st) {
  const bool dot = a.dot_rhs;
  switch (a.op) {
    case StencilOp::Matvec: return run<NPTS, NDOF, double, double, StencilOp::Matvec, false>(L, a, st);
    case StencilOp::Residual: return run<NPTS, NDOF, double, double, StencilOp::Residual, false>(L, a, st);
    case StencilOp::ResidualScaled:
      return run<NPTS, NDOF, double, double, StencilOp::ResidualScaled, false>(L, a, st);
    case StencilOp::Cheb:
      return dot ? run<NPTS, NDOF, double, double, StencilOp::Cheb, true>(L, a, st)
                 : run<NPTS, NDOF, double, double, StencilOp::Cheb, false>(L, a, st);
    case StencilOp::ChebFirst:
      return dot ? run<NPTS, NDOF, double, double, StencilOp::ChebFirst, true>(L, a, st)
                 : run<NPTS, NDOF, double, double, StencilOp::ChebFirst, false>(L, a, st);
    case StencilOp::CgQ: return run<NPTS, NDOF, double, double, StencilOp::CgQ, false>(L, a, st);
  }
  return 0;
}

// FP32 vectors: the V-cycle operations only.
template <int NDOF, class C>
static int64_t ops_f32(const Level& L, const StencilArgs& a, hipStream_t st) {
  RMG_REQUIRE(!a.dot_rhs, RMG_ERR_ARG, "internal: fused dot products need FP64 vectors");
  switch (a.op) {
    case StencilOp::Matvec: return run<27, NDOF, float, C, StencilOp::Matvec, false>(L, a, st);
    case StencilOp::ResidualScaled: return run<27, NDOF, float, C, StencilOp::ResidualScaled, false>(L, a, st);
    case StencilOp::Cheb: return run<27, NDOF, float, C, StencilOp::Cheb, false>(L, a, st);
    case StencilOp::ChebFirst: return run<27, NDOF, float, C, StencilOp::ChebFirst, false>(L, a, st);
    default: fail(RMG_ERR_ARG, "internal: operation not available in FP32");
  }
}

int64_t launch_stencil_op(const Level& L, const StencilArgs& a, hipStream_t st) {
  if (a.lowp) {
    RMG_REQUIRE(L.npts == 27 && L.ct_lo != kCoefF64, RMG_ERR_ARG, "internal: level has no low-precision copy");
    if (L.ndof == 1) return L.ct_lo == kCoefBF16 ? ops_f32<1, uint16_t>(L, a, st) : ops_f32<1, float>(L, a, st);
    return L.ct_lo == kCoefBF16 ? ops_f32<3, uint16_t>(L, a, st) : ops_f32<3, float>(L, a, st);
  }
  if (L.ndof == 3) {
    RMG_REQUIRE(L.npts == 27, RMG_ERR_ARG, "internal: block stencils are 27-point");
    return ops_f64<27, 3>(L, a, st);
  }
  switch (L.npts) {
    case 27: return ops_f64<27, 1>(L, a, st);
    case 9: return ops_f64<9, 1>(L, a, st);
    case 5: return ops_f64<5, 1>(L, a, st);
  }
  fail(RMG_ERR_ARG, "unsupported stencil size");
}

}  // namespace rmg
