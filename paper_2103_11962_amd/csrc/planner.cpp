// Host planner: region validation, level geometry, block tables, interface groups,
// and the coarsest-level composite operator.
#include <algorithm>
#include <memory>
#include <cmath>
#include <cstring>
#include <string>

#include "kernels.h"

namespace rmg {

DevAlloc& current_allocator() {
  thread_local DevAlloc a;
  return a;
}

void DBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) return;
  const DevAlloc& a = current_allocator();
  if (a.alloc) {
    p = a.alloc(nbytes, a.ctx);
    if (!p) fail(RMG_ERR_OOM, "device memory provider returned no memory for " + std::to_string(nbytes) + " bytes");
    from = a;
  } else {
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
      p = nullptr;
      fail(e == hipErrorOutOfMemory ? RMG_ERR_OOM : RMG_ERR_DEVICE,
           "hipMalloc of " + std::to_string(nbytes) + " bytes failed: " + hipGetErrorString(e));
    }
    from = DevAlloc();
  }
  bytes = nbytes;
}

void DBuf::release() {
  if (p) {
    if (from.free) from.free(p, from.ctx);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
  from = DevAlloc();
}

LevelView Level::view() const {
  LevelView v;
  v.regs = d_regs.as<RegionGeo>();
  v.blocks = d_blocks.as<BlockDesc>();
  v.nblocks = (int)blocks.size();
  v.nreg = nreg;
  v.n = n;
  v.cx = comp[0];
  v.cy = comp[1];
  v.cz = comp[2];
  v.mask = mask;
  v.npts = npts;
  v.ndof = ndof;
  return v;
}

static bool shared_node(const Level& L, const RegionGeo& R, int x, int y, int z) {
  const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
  return (x == 0 && gx != 0) || (x == R.ex - 1 && gx != L.comp[0] - 1) || (y == 0 && gy != 0) ||
         (y == R.ey - 1 && gy != L.comp[1] - 1) || (z == 0 && gz != 0) || (z == R.ez - 1 && gz != L.comp[2] - 1);
}

template <class T>
static void upload(DBuf& d, const std::vector<T>& v) {
  if (v.empty()) {
    d.release();
    return;
  }
  d.alloc(sizeof(T) * v.size());
  RMG_HIP(hipMemcpy(d.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
}

// 2.5D tiles of a 3D level: L.tile_threads-node tiles of whole (or that many nodes of) x-rows, `depth` planes deep,
// ordered largest first so a persistent launch hands out the costly tiles early.
void make_tiles(Level& L, int depth) {
  L.tiles.clear();
  L.tile_depth = depth;
  if (L.dim != 3) return;
  const int kThreads = L.tile_threads;
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    const int tx = std::min(R.ex, kThreads);
    const int tymax = std::min(R.ey, kThreads / tx);
    const int nty = (R.ey + tymax - 1) / tymax;  // tiles per column, rows shared out evenly
    for (int z0 = 0; z0 < R.ez; z0 += depth)
      for (int j = 0, y0 = 0; j < nty; ++j) {
        const int ty = R.ey / nty + (j < R.ey % nty ? 1 : 0);
        for (int x0 = 0; x0 < R.ex; x0 += tx)
          L.tiles.push_back(Tile3{k, x0, y0, z0, tx, ty, std::min(depth, R.ez - z0), 0});
        y0 += ty;
      }
  }
  std::stable_sort(L.tiles.begin(), L.tiles.end(), [](const Tile3& a, const Tile3& b) {
    return (int64_t)a.tx * a.ty * a.nz > (int64_t)b.tx * b.ty * b.nz;
  });
  for (const Tile3& T : L.tiles)
    RMG_REQUIRE((T.tx + 2) * (T.ty + 2) <= tile_plane_cap(kThreads) && T.tx * T.ty <= kThreads, RMG_ERR_ARG,
                "internal: tile too large");
  if (!L.tiles.empty()) {
    L.d_tiles.alloc(sizeof(Tile3) * L.tiles.size());
    RMG_HIP(hipMemcpy(L.d_tiles.p, L.tiles.data(), sizeof(Tile3) * L.tiles.size(), hipMemcpyHostToDevice));
  }
  if (!L.table_served.empty()) {  // a split exists: the regions it does not serve run these tiles
    L.other_tiles.clear();
    for (const Tile3& T : L.tiles)
      if (!L.table_served[T.region]) L.other_tiles.push_back(T);
    upload(L.d_other_tiles, L.other_tiles);
  }
}

void clear_split(Level& L) {
  L.table_served.clear();
  L.table_tiles.clear();
  L.other_tiles.clear();
  L.d_table_tiles.release();
  L.d_other_tiles.release();
}

// Lanes of a table tile of ty rows of extent ex: the rows' inner x-nodes (x in [2, ex - 2)) padded
// to whole wavefronts, then four x-face nodes per row.
static int table_lanes(int ex, int ty) { return ((ty * (ex - 4) + 63) & ~63) + 4 * ty; }

// Served regions (at least 5 nodes a side): whole-row tiles of ty rows, ty the most (at most
// kTableRows) whose lanes fit kTableThreads and whose plane with its halo takes two loads per lane,
// rows shared out evenly, and
// at most kTablePlanes planes (planes shared out evenly), largest first.
void make_split(Level& L, const std::vector<int>& served) {
  std::vector<int> keep = served;
  clear_split(L);
  L.table_served = keep;
  for (int k = 0; k < L.nreg; ++k) {
    if (!keep[k]) continue;
    const RegionGeo& R = L.regs[k];
    RMG_REQUIRE(R.ex >= 5 && R.ey >= 5 && R.ez >= 5, RMG_ERR_ARG, "internal: table region under 5 nodes a side");
    int tymax = 0;
    while (tymax < std::min(R.ey, kTableRows) && table_lanes(R.ex, tymax + 1) <= kTableThreads &&
           (R.ex + 2) * (tymax + 3) <= 2 * kTableThreads)
      ++tymax;
    RMG_REQUIRE(tymax >= 1, RMG_ERR_ARG, "internal: region row wider than a table tile");
    const int nty = (R.ey + tymax - 1) / tymax;
    const int ntz = (R.ez + kTablePlanes - 1) / kTablePlanes;
    for (int iz = 0, z0 = 0; iz < ntz; ++iz) {
      const int nz = R.ez / ntz + (iz < R.ez % ntz ? 1 : 0);
      for (int j = 0, y0 = 0; j < nty; ++j) {
        const int ty = R.ey / nty + (j < R.ey % nty ? 1 : 0);
        L.table_tiles.push_back(Tile3{k, 0, y0, z0, R.ex, ty, nz, 0});
        y0 += ty;
      }
      z0 += nz;
    }
  }
  for (const Tile3& T : L.table_tiles) {
    const RegionGeo& R = L.regs[T.region];
    RMG_REQUIRE(table_lanes(T.tx, T.ty) <= kTableThreads && T.ty <= kTableRows && (T.tx + 2) * (T.ty + 2) <= 2 * kTableThreads &&
                    T.x0 == 0 && T.tx == R.ex && T.y0 + T.ty <= R.ey && T.z0 + T.nz <= R.ez && T.nz >= 1,
                RMG_ERR_ARG, "internal: table tile does not fit its block");
  }
  for (const Tile3& T : L.tiles)
    if (!keep[T.region]) L.other_tiles.push_back(T);
  upload(L.d_table_tiles, L.table_tiles);
  upload(L.d_other_tiles, L.other_tiles);
}

// Transfer tiles.  Restriction: a block of kBlock threads owns whole coarse rows (one thread per
// coarse node, at most kBlock / EX rows) and up to kXferCoarsePlanes coarse planes, and stages per
// fine plane the fine rows that reach them (three per coarse row plus two on either side), at most
// kXferStagePerThread values per thread.  Prolongation: a block owns up to kBlock / ex whole fine rows
// (whose coarse rows fit its stage) and kXferFinePlanes fine planes.  Rows and planes are shared
// out evenly; on small levels tiles take fewer planes, then fewer rows, until the level has
// kXferMinTiles of them (or single rows and planes).
constexpr int kXferCoarsePlanes = 4;
constexpr int kXferFinePlanes = 8;
constexpr int64_t kXferStageBytes = 8 * kXferStagePerThread * kBlock;  // FP64 values staged per plane at most
constexpr size_t kXferMinTiles = 1024;

void make_transfer_tiles(Level& F, const Level& C, bool rows_and_planes) {
  F.rtiles.clear();
  F.ptiles.clear();
  F.rtile_vals = 0;
  auto cpos = [](int c, int e) { return std::min(3 * c, e - 1); };
  // start of the coarse interval of fine node g (the next coarse node for an interval's end node)
  auto lo_of = [](int g, int e, int E) {
    if (E < 2) return 0;
    int lo = std::min(g / 3, E - 2);
    const int p0 = 3 * lo, m = std::min(p0 + 3, e - 1) - p0;
    return g - p0 == m ? lo + 1 : lo;
  };
  bool ok = rows_and_planes && F.nreg == C.nreg && (F.dim == 2 || F.dim == 3);
  for (int k = 0; ok && k < F.nreg; ++k)
    if (C.regs[k].ex > kBlock || F.regs[k].ex > kBlock || C.regs[k].ex > kProlongStageXY) ok = false;
  // even shares of n items in parts of at most cap
  auto shares = [](int n, int cap) {
    const int parts = (n + cap - 1) / cap;
    std::vector<int> v(parts);
    for (int j = 0; j < parts; ++j) v[j] = n / parts + (j < n % parts ? 1 : 0);
    return v;
  };
  // restriction tiles with at most ny coarse rows (capped per region) and nz coarse planes
  auto build_r = [&](int nycap, int nzcap) {
    F.rtiles.clear();
    F.rtile_vals = 0;
    for (int k = 0; k < F.nreg; ++k) {
      const RegionGeo& RF = F.regs[k];
      const RegionGeo& RC = C.regs[k];
      auto rows = [&](int y0, int n) {
        return std::min(cpos(y0 + n - 1, RF.ey) + 2, RF.ey - 1) - std::max(cpos(y0, RF.ey) - 2, 0) + 1;
      };
      auto stage_bytes = [&](int n) { return (int64_t)std::min(3 * (n - 1) + 5, RF.ey) * RF.ex * F.ndof * 8; };
      int ny = std::min({RC.ey, kBlock / RC.ex, nycap});
      while (ny > 1 && stage_bytes(ny) > kXferStageBytes) --ny;
      if (stage_bytes(ny) > kXferStageBytes) return false;
      int z0 = 0;
      for (int nz : shares(RC.ez, F.dim == 3 ? nzcap : 1)) {
        int y0 = 0;
        for (int ty : shares(RC.ey, ny)) {
          F.rtiles.push_back(Tile3{k, 0, y0, z0, RC.ex, ty, nz, 0});
          F.rtile_vals = std::max(F.rtile_vals, (int64_t)rows(y0, ty) * RF.ex * F.ndof);
          y0 += ty;
        }
        z0 += nz;
      }
    }
    return true;
  };
  // prolongation tiles with at most fy fine rows (capped per region) and nz fine planes
  auto build_p = [&](int fycap, int nzcap) {
    F.ptiles.clear();
    for (int k = 0; k < F.nreg; ++k) {
      const RegionGeo& RF = F.regs[k];
      const RegionGeo& RC = C.regs[k];
      auto crows = [&](int y0, int n) {
        return std::min(lo_of(y0 + n - 1, RF.ey, RC.ey) + 1, RC.ey - 1) - lo_of(y0, RF.ey, RC.ey) + 1;
      };
      auto fits = [&](int n) {
        int y0 = 0;
        for (int ty : shares(RF.ey, n)) {
          if (crows(y0, ty) * RC.ex > kProlongStageXY) return false;
          y0 += ty;
        }
        return true;
      };
      int fy = std::min({RF.ey, std::max(1, kBlock / RF.ex), fycap});
      while (fy > 1 && !fits(fy)) --fy;
      if (!fits(fy)) return false;
      int z0 = 0;
      for (int nz : shares(RF.ez, F.dim == 3 ? nzcap : 1)) {
        int y0 = 0;
        for (int ty : shares(RF.ey, fy)) {
          F.ptiles.push_back(Tile3{k, 0, y0, z0, RF.ex, ty, nz, 0});
          y0 += ty;
        }
        z0 += nz;
      }
    }
    return true;
  };
  if (ok) {
    int ny = kBlock, nz = kXferCoarsePlanes;
    ok = build_r(ny, nz);
    while (ok && F.rtiles.size() < kXferMinTiles && (nz > 1 || ny > 1)) {
      if (nz > 1) nz /= 2;
      else ny = std::max(1, std::min(ny, kBlock) / 2);
      ok = build_r(ny, nz);
    }
  }
  if (ok) {
    int fy = kBlock, nz = kXferFinePlanes;
    ok = build_p(fy, nz);
    while (ok && F.ptiles.size() < kXferMinTiles && (nz > 1 || fy > 1)) {
      if (nz > 1) nz /= 2;
      else fy = std::max(1, std::min(fy, kBlock) / 2);
      ok = build_p(fy, nz);
    }
  }
  for (const Tile3& T : F.rtiles) {
    const RegionGeo& RC = C.regs[T.region];
    RMG_REQUIRE(T.tx * T.ty <= kBlock && T.y0 + T.ty <= RC.ey && T.z0 + T.nz <= RC.ez && T.ty >= 1 && T.nz >= 1,
                RMG_ERR_ARG, "internal: restriction tile does not fit its block");
  }
  for (const Tile3& T : F.ptiles) {
    const RegionGeo& RF = F.regs[T.region];
    RMG_REQUIRE(T.tx * T.ty <= kBlock && T.y0 + T.ty <= RF.ey && T.z0 + T.nz <= RF.ez && T.ty >= 1 && T.nz >= 1,
                RMG_ERR_ARG, "internal: prolongation tile does not fit its block");
  }
  if (!ok) {
    F.rtiles.clear();
    F.ptiles.clear();
    F.rtile_vals = 0;
  }
  upload(F.d_rtiles, F.rtiles);
  upload(F.d_ptiles, F.ptiles);
}

// Offsets, block table and interface groups of a level whose regs/comp are set.
void build_tables(Level& L) {
  int64_t off = 0;
  L.blocks.clear();
  L.region_block.assign(1, 0);
  for (int k = 0; k < L.nreg; ++k) {
    RegionGeo& R = L.regs[k];
    R.n = R.ex * R.ey * R.ez;
    R.off = off;
    off += R.n;
    for (int s = 0; s < R.n; s += kBlock) L.blocks.push_back(BlockDesc{k, s});
    L.region_block.push_back((int)L.blocks.size());
  }
  L.n = off;
  RMG_REQUIRE(L.n < (int64_t)1 << 31, RMG_ERR_ARG, "more than 2^31 regional nodes on one level");
  L.ncomp = (int64_t)L.comp[0] * L.comp[1] * L.comp[2];
  RMG_REQUIRE(L.ncomp < (int64_t)1 << 31, RMG_ERR_ARG, "more than 2^31 composite nodes");

  // Interface groups: (composite index, regional index) pairs of every shared surface node,
  // sorted by composite index; regional indices grow with the region id, so each group lists
  // its copies in ascending region order.
  std::vector<uint64_t> keys;
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    for (int z = 0; z < R.ez; ++z)
      for (int y = 0; y < R.ey; ++y) {
        const bool yz_face = (y == 0 || y == R.ey - 1 || z == 0 || z == R.ez - 1);
        for (int x = 0; x < R.ex; x += (yz_face ? 1 : std::max(1, R.ex - 1))) {
          if (!shared_node(L, R, x, y, z)) continue;
          const int64_t c = ((int64_t)(R.oz + z) * L.comp[1] + (R.oy + y)) * L.comp[0] + (R.ox + x);
          const int64_t ri = R.off + ((int64_t)z * R.ey + y) * R.ex + x;
          keys.push_back(((uint64_t)c << 32) | (uint64_t)ri);
        }
      }
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int64_t> gptr;
  std::vector<int32_t> gcopy, gcomp;
  gptr.push_back(0);
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    const uint64_t c = keys[i] >> 32;
    while (j < keys.size() && (keys[j] >> 32) == c) {
      gcopy.push_back((int32_t)(keys[j] & 0xffffffffu));
      ++j;
    }
    RMG_REQUIRE(j - i >= 2, RMG_ERR_SHAPE,
                "a node on an inner region face belongs to one region only: boxes do not conform");
    gcomp.push_back((int32_t)c);
    gptr.push_back((int64_t)gcopy.size());
    i = j;
  }
  // Order groups by multiplicity (faces, then edges, then corners) so a wavefront mostly sees
  // groups of one size.
  const int64_t ng = (int64_t)gcomp.size();
  std::vector<int64_t> order(ng);
  for (int64_t g = 0; g < ng; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return (gptr[a + 1] - gptr[a]) < (gptr[b + 1] - gptr[b]);
  });
  std::vector<int64_t> gptr2(1, 0);
  std::vector<int32_t> gcopy2, gcomp2;
  gcopy2.reserve(gcopy.size());
  for (int64_t g : order) {
    for (int64_t c = gptr[g]; c < gptr[g + 1]; ++c) gcopy2.push_back(gcopy[c]);
    gptr2.push_back((int64_t)gcopy2.size());
    gcomp2.push_back(gcomp[g]);
  }
  L.ngroups = ng;
  L.ngroups2 = 0;
  while (L.ngroups2 < ng && gptr2[L.ngroups2 + 1] - gptr2[L.ngroups2] == 2) ++L.ngroups2;
  // 2.5D tiles for the 3D stencil kernel, 21 planes deep by default; used when the level has
  // enough tiles to fill the GPU unless the options or the autotuner say otherwise.
  make_tiles(L, 21);
  L.use_tiles = L.tiles.size() >= kAutoTileMin;
  L.d_regs.alloc(sizeof(RegionGeo) * L.regs.size());
  RMG_HIP(hipMemcpy(L.d_regs.p, L.regs.data(), sizeof(RegionGeo) * L.regs.size(), hipMemcpyHostToDevice));
  L.d_blocks.alloc(sizeof(BlockDesc) * L.blocks.size());
  RMG_HIP(hipMemcpy(L.d_blocks.p, L.blocks.data(), sizeof(BlockDesc) * L.blocks.size(), hipMemcpyHostToDevice));
  if (ng > 0) {
    L.d_gptr.alloc(sizeof(int64_t) * gptr2.size());
    RMG_HIP(hipMemcpy(L.d_gptr.p, gptr2.data(), sizeof(int64_t) * gptr2.size(), hipMemcpyHostToDevice));
    L.d_gcopy.alloc(sizeof(int32_t) * gcopy2.size());
    RMG_HIP(hipMemcpy(L.d_gcopy.p, gcopy2.data(), sizeof(int32_t) * gcopy2.size(), hipMemcpyHostToDevice));
    L.d_gcomp.alloc(sizeof(int32_t) * gcomp2.size());
    RMG_HIP(hipMemcpy(L.d_gcomp.p, gcomp2.data(), sizeof(int32_t) * gcomp2.size(), hipMemcpyHostToDevice));
  }
}

// Region boxes must tile the bounding box of the domain: the element (cell) volumes add up
// to the bounding box volume and no two cell boxes intersect.
static void validate_tiling(int dim, int nreg, const std::vector<int32_t>& ext, const std::vector<int32_t>& org,
                            const int comp[3]) {
  int64_t vol = 0;
  for (int k = 0; k < nreg; ++k) {
    int64_t v = 1;
    for (int d = 0; d < dim; ++d) v *= ext[3 * k + d] - 1;
    vol += v;
  }
  int64_t total = 1;
  for (int d = 0; d < dim; ++d) total *= comp[d] - 1;
  RMG_REQUIRE(vol == total, RMG_ERR_SHAPE, "region boxes do not cover the domain exactly once");
  for (int a = 0; a < nreg; ++a)
    for (int b = a + 1; b < nreg; ++b) {
      bool overlap = true;
      for (int d = 0; d < dim; ++d) {
        const int lo = std::max(org[3 * a + d], org[3 * b + d]);
        const int hi = std::min(org[3 * a + d] + ext[3 * a + d] - 1, org[3 * b + d] + ext[3 * b + d] - 1);
        if (hi - lo <= 0) overlap = false;  // cell ranges [o, o+e-1) do not intersect
      }
      RMG_REQUIRE(!overlap, RMG_ERR_SHAPE,
                  "regions " + std::to_string(a) + " and " + std::to_string(b) + " overlap in more than an interface");
    }
}

void build_level0(rmg_handle* h) {
  std::unique_ptr<Level> L(new Level());  // owned here until the handle takes it
  L->dim = h->dim;
  L->nreg = h->nreg;
  L->npts = h->dim == 3 ? 27 : 9;
  L->ndof = h->ndof;
  L->mask = h->mask;
  L->comp[0] = L->comp[1] = L->comp[2] = 1;
  L->regs.resize(h->nreg);
  for (int k = 0; k < h->nreg; ++k) {
    RegionGeo& R = L->regs[k];
    R.ex = h->extent[3 * k + 0];
    R.ey = h->extent[3 * k + 1];
    R.ez = h->extent[3 * k + 2];
    R.ox = h->origin[3 * k + 0];
    R.oy = h->origin[3 * k + 1];
    R.oz = h->origin[3 * k + 2];
    R.pad = 0;
    L->comp[0] = std::max(L->comp[0], R.ox + R.ex);
    L->comp[1] = std::max(L->comp[1], R.oy + R.ey);
    L->comp[2] = std::max(L->comp[2], R.oz + R.ez);
  }
  validate_tiling(h->dim, h->nreg, h->extent, h->origin, L->comp);
  build_tables(*L);
  for (Level* old : h->levels) delete old;
  h->levels.clear();
  h->levels.push_back(L.release());
}

// Rate-3 coarsening of the region boxes (Section 3.2: each region's structured coarsening keeps
// coarse points on its interface).  Along each axis a region keeps every third node from its
// first one and its last node, (e + 1) / 3 + 1 nodes in all, so its last coarse interval spans 1,
// 2 or 3 cells.  The composite coarse lattice along an axis is the union of these positions; it
// must agree with each region's own positions on that region's range, so that co-located fine
// interface nodes interpolate from the same coarse nodes in every region (RMG_ERR_SHAPE
// otherwise).  Coarse origins index that lattice.  Extents 3^k + 1 at origins divisible by 3 give
// every third composite node.
void coarse_geometry(int dim, const std::vector<RegionGeo>& fine, std::vector<RegionGeo>& coarse, int comp[3]) {
  const size_t nreg = fine.size();
  coarse.assign(nreg, RegionGeo{});
  auto ext = [](RegionGeo& R, int d) -> int& { return d == 0 ? R.ex : (d == 1 ? R.ey : R.ez); };
  auto org = [](RegionGeo& R, int d) -> int& { return d == 0 ? R.ox : (d == 1 ? R.oy : R.oz); };
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) {
      for (RegionGeo& Q : coarse) {
        ext(Q, d) = 1;
        org(Q, d) = 0;
      }
      comp[d] = 1;
      continue;
    }
    std::vector<int> lattice;
    for (size_t k = 0; k < nreg; ++k) {
      RegionGeo R = fine[k];
      const int o = org(R, d), e = ext(R, d);
      for (int p = 0; p < e - 1; p += 3) lattice.push_back(o + p);
      lattice.push_back(o + e - 1);
    }
    std::sort(lattice.begin(), lattice.end());
    lattice.erase(std::unique(lattice.begin(), lattice.end()), lattice.end());
    for (size_t k = 0; k < nreg; ++k) {
      RegionGeo R = fine[k];
      const int o = org(R, d), e = ext(R, d), E = (e + 1) / 3 + 1;
      const size_t i0 = (size_t)(std::lower_bound(lattice.begin(), lattice.end(), o) - lattice.begin());
      bool same = i0 + E <= lattice.size();
      for (int j = 0; same && j < E; ++j) same = lattice[i0 + j] == o + std::min(3 * j, e - 1);
      RMG_REQUIRE(same, RMG_ERR_SHAPE,
                  "coarse points of region " + std::to_string(k) + " disagree with its neighbours' along axis " +
                      std::to_string(d));
      org(coarse[k], d) = (int)i0;
      ext(coarse[k], d) = E;
    }
    comp[d] = (int)lattice.size();
  }
}

Level* make_coarse_level(const Level& F) {
  std::unique_ptr<Level> C(new Level());  // released to the caller once complete
  C->dim = F.dim;
  C->nreg = F.nreg;
  C->npts = F.dim == 3 ? 27 : 9;
  C->ndof = F.ndof;
  C->mask = F.mask;
  coarse_geometry(F.dim, F.regs, C->regs, C->comp);
  build_tables(*C);
  return C.release();
}

// Coarsest level: Abar = Psi-bar [[Abar]] Psi-bar^T assembled densely on the host from the
// regional stencils, then inverted on the device (Section 3.5, direct solver).
void build_coarse_solver(rmg_handle* h, Level& L) {
  hipStream_t st = h->stream;
  const int nd = L.ndof, nb = nd * nd, ncoef = L.ncoef();
  const int64_t nc64 = L.ncomp * nd;
  RMG_REQUIRE(nc64 <= 20000, RMG_ERR_ARG, "coarsest composite problem too large for the dense solver");
  const int nc = (int)nc64;
  L.nc = nc;
  std::vector<double> coef(coef_elems(L.n, ncoef));
  RMG_HIP(hipMemcpyAsync(coef.data(), L.coef.p, sizeof(double) * coef.size(), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  L.abar_host.assign((size_t)nc * nc, 0.0);
  std::vector<int32_t> owner(L.ncomp, -1);
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    for (int z = 0; z < R.ez; ++z)
      for (int y = 0; y < R.ey; ++y)
        for (int x = 0; x < R.ex; ++x) {
          const int64_t li = ((int64_t)z * R.ey + y) * R.ex + x;
          const int64_t i = ((int64_t)(R.oz + z) * L.comp[1] + (R.oy + y)) * L.comp[0] + (R.ox + x);
          if (owner[i] < 0) owner[i] = (int32_t)(R.off + li);
          for (int s = 0; s < L.npts; ++s) {
            int dx, dy, dz;
            if (L.npts == 27) {
              dx = s % 3 - 1;
              dy = (s / 3) % 3 - 1;
              dz = s / 9 - 1;
            } else {
              dx = s % 3 - 1;
              dy = s / 3 - 1;
              dz = 0;
            }
            if (x + dx < 0 || x + dx >= R.ex || y + dy < 0 || y + dy >= R.ey || z + dz < 0 || z + dz >= R.ez) continue;
            const int64_t j = ((int64_t)(R.oz + z + dz) * L.comp[1] + (R.oy + y + dy)) * L.comp[0] + (R.ox + x + dx);
            for (int a = 0; a < nd; ++a)
              for (int b = 0; b < nd; ++b) {
                const double v = coef[coef_index(R.off + li, s * nb + a * nd + b, ncoef)];
                if (v != 0.0) L.abar_host[(size_t)(i * nd + a) * nc + (j * nd + b)] += v;
              }
          }
        }
  }
  L.ainv.alloc(sizeof(double) * (size_t)nc * nc);
  RMG_HIP(hipMemcpyAsync(L.ainv.p, L.abar_host.data(), sizeof(double) * (size_t)nc * nc, hipMemcpyHostToDevice, st));
  L.comp_owner.alloc(sizeof(int32_t) * owner.size());
  RMG_HIP(hipMemcpyAsync(L.comp_owner.p, owner.data(), sizeof(int32_t) * owner.size(), hipMemcpyHostToDevice, st));
  L.cvec.alloc(sizeof(double) * nc);
  L.cvec2.alloc(sizeof(double) * nc);
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  launch_gauss_jordan(L.ainv.as<double>(), nc, st);
  launch_check_inverse(L.ainv.as<double>(), nc, flag.as<int>(), st);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "coarsest composite operator is not symmetric positive definite");
}

}  // namespace rmg
