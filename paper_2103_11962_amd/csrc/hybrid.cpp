// Structured/unstructured hybrid hierarchy (the paper's structured/unstructured mesh hybrid
// section; Table 5): host planner and the cycle that drives the kernels of kernels_hybrid.hip.
//
// Coarsening is aggregation with piecewise-constant transfers (P^(k) has one 1 per aggregated row):
//  * structured region: every free node joins the aggregate of its nearest rate-3 coarse point
//    (per axis c = 3 floor((g + 1) / 3) in composite coordinates, moved one coarse step inward
//    where it would lie on a Dirichlet face; Dirichlet nodes are never aggregated);
//  * unstructured region: staged plain aggregation.  Stage I aggregates the region's interface
//    nodes by the structured rule (so every copy of an interface node lands in the same coarse
//    node in every region, as the Lemma on P requires); stage II makes a node whose free graph
//    neighbours are all unaggregated a root of an aggregate with them; stage III lets each node
//    still left join the neighbouring aggregate it has most couplings to (counted on the
//    aggregates as they stand when the stage starts; ties to the aggregate whose smallest member
//    comes first); stage IV starts, in order, an aggregate from each remaining node and its
//    unaggregated neighbours.
// A region's coarse nodes are ordered by the smallest row of their aggregate; coarse composite
// nodes are numbered by first sight, regions in order (nodes with a lattice position are one
// node in every region).  Region matrices of the next level are P^(k)T A^(k) P^(k) (the Theorem).
// The aggregation is sequential and runs here once per setup; the cycle runs on the device.
#include <algorithm>
#include <array>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "hybrid.h"
#include "kernels.h"

namespace rmg {

namespace {

// fn(k) for k in [0, n) on up to 16 host threads; each k writes only its own outputs and makes
// no HIP calls.  The first exception is rethrown on the calling thread.
template <class F>
void parallel_for(int64_t n, F&& fn) {
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  const int nt = (int)std::min<int64_t>(std::min<int64_t>(n, 16), hw);
  if (nt <= 1) {
    for (int64_t k = 0; k < n; ++k) fn(k);
    return;
  }
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex m;
  auto work = [&] {
    for (int64_t k; (k = next.fetch_add(1)) < n;) {
      try {
        fn(k);
      } catch (...) {
        std::lock_guard<std::mutex> g(m);
        if (!err) err = std::current_exception();
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (std::thread& t : pool) t.join();
  if (err) std::rethrow_exception(err);
}

int coarse_coord(int g, int axis, const int shape[3], unsigned mask) {
  int c = 3 * ((g + 1) / 3);
  if (((mask >> (2 * axis)) & 1u) && c == 0) c = 3;
  if (((mask >> (2 * axis + 1)) & 1u) && c == shape[axis] - 1) c = shape[axis] - 4;
  return c;
}

int64_t pack(const std::array<int32_t, 3>& p) {
  return ((int64_t)p[2] << 42) | ((int64_t)p[1] << 21) | (int64_t)p[0];
}

void host_offsets(int npts, int s, int& dx, int& dy, int& dz) {
  if (npts == 27) {
    dx = s % 3 - 1;
    dy = (s / 3) % 3 - 1;
    dz = s / 9 - 1;
  } else if (npts == 9) {
    dx = s % 3 - 1;
    dy = s / 3 - 1;
    dz = 0;
  } else {  // five-point order (0,-1) (-1,0) (0,0) (1,0) (0,1)
    dz = 0;
    dx = s == 1 ? -1 : (s == 3 ? 1 : 0);
    dy = s == 0 ? -1 : (s == 4 ? 1 : 0);
  }
}

// Setup upload of a host table; waits for the copy, so the table may die on return.
template <class T>
void upload(DBuf& d, const std::vector<T>& v, hipStream_t st) {
  d.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (v.empty()) return;
  RMG_HIP(hipMemcpyAsync(d.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  RMG_HIP(hipStreamSynchronize(st));
}

// The finest level's region matrices from the stencil level (nonzeros only, ascending columns).
void finest_level(rmg_handle* h, HLevel& H) {
  Level& L = *h->levels[0];
  hipStream_t st = h->stream;
  std::vector<double> coef(coef_elems(L.n, L.npts));
  RMG_HIP(hipMemcpyAsync(coef.data(), L.coef.p, sizeof(double) * coef.size(), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  for (int d = 0; d < 3; ++d) H.shape[d] = L.comp[d];
  H.ncomp = L.ncomp;
  H.regs.assign(L.nreg, HRegionHost());
  H.off.assign(L.nreg + 1, 0);
  const int cx = L.comp[0], cy = L.comp[1], cz = L.comp[2];
  parallel_for(L.nreg, [&](int64_t k) {
    const RegionGeo& R = L.regs[k];
    HRegionHost& G = H.regs[k];
    G.ptr.assign(1, 0);
    for (int z = 0; z < R.ez; ++z)
      for (int y = 0; y < R.ey; ++y)
        for (int x = 0; x < R.ex; ++x) {
          const int64_t li = ((int64_t)z * R.ey + y) * R.ex + x;
          for (int s = 0; s < L.npts; ++s) {
            int dx, dy, dz;
            host_offsets(L.npts, s, dx, dy, dz);
            if (x + dx < 0 || x + dx >= R.ex || y + dy < 0 || y + dy >= R.ey || z + dz < 0 || z + dz >= R.ez) continue;
            const double v = coef[coef_index(R.off + li, s, L.npts)];
            if (v == 0.0) continue;
            G.col.push_back((int32_t)(li + dx + (int64_t)dy * R.ex + (int64_t)dz * R.ex * R.ey));
            G.val.push_back(v);
          }
          G.ptr.push_back((int64_t)G.col.size());
          const int gx = R.ox + x, gy = R.oy + y, gz = R.oz + z;
          G.comp.push_back(((int64_t)gz * cy + gy) * cx + gx);
          G.xyz.push_back({gx, gy, gz});
          const unsigned m = L.mask;
          const bool dir = ((m & 1u) && gx == 0) || ((m & 2u) && gx == cx - 1) || ((m & 4u) && gy == 0) ||
                           ((m & 8u) && gy == cy - 1) || ((m & 16u) && gz == 0) || ((m & 32u) && gz == cz - 1);
          G.free.push_back(dir ? 0 : 1);
        }
  });
  for (int k = 0; k < L.nreg; ++k) H.off[k + 1] = H.off[k] + H.regs[k].n();
}

std::vector<int32_t> multiplicity(const HLevel& H) {
  std::vector<int32_t> m(H.ncomp, 0);
  for (const HRegionHost& G : H.regs)
    for (int64_t c : G.comp) ++m[c];
  return m;
}

// Aggregates of one region: coarse local index of every row (-1: Dirichlet) and the lattice
// position of every coarse node ({-1,-1,-1} for aggregates not formed by the structured rule).
void aggregate(const HRegionHost& G, bool unstructured, const std::vector<int32_t>& mult, const int shape[3],
               unsigned mask, int dim, std::vector<int32_t>& local, std::vector<std::array<int32_t, 3>>& cxyz) {
  const int64_t n = G.n();
  std::vector<int64_t> lab(n, -1);
  std::vector<std::array<int32_t, 3>> point;  // per label
  std::unordered_map<int64_t, int64_t> label_of_point;
  auto structured = [&](int64_t i) {
    std::array<int32_t, 3> cp = {0, 0, 0};
    for (int a = 0; a < dim; ++a) cp[a] = coarse_coord(G.xyz[i][a], a, shape, mask);
    auto it = label_of_point.find(pack(cp));
    if (it == label_of_point.end()) {
      it = label_of_point.emplace(pack(cp), (int64_t)point.size()).first;
      point.push_back(cp);
    }
    lab[i] = it->second;
  };
  auto for_neighbours = [&](int64_t i, auto&& fn) {
    for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e) {
      const int64_t j = G.col[e];
      if (j != i && G.val[e] != 0.0 && G.free[j]) fn(j);
    }
  };
  if (!unstructured) {
    for (int64_t i = 0; i < n; ++i)
      if (G.free[i]) structured(i);
  } else {
    for (int64_t i = 0; i < n; ++i)  // stage I: interface nodes
      if (G.free[i] && mult[G.comp[i]] >= 2) structured(i);
    const std::array<int32_t, 3> none = {-1, -1, -1};
    for (int64_t i = 0; i < n; ++i) {  // stage II: roots
      if (!G.free[i] || lab[i] >= 0) continue;
      bool all_free = true;
      for_neighbours(i, [&](int64_t j) { all_free = all_free && lab[j] < 0; });
      if (!all_free) continue;
      const int64_t a = (int64_t)point.size();
      point.push_back(none);
      lab[i] = a;
      for_neighbours(i, [&](int64_t j) { lab[j] = a; });
    }
    const std::vector<int64_t> snap = lab;  // stage III: joins
    std::vector<int64_t> first(point.size(), -1);
    for (int64_t i = 0; i < n; ++i)
      if (snap[i] >= 0 && first[snap[i]] < 0) first[snap[i]] = i;
    std::vector<std::pair<int64_t, int>> count;
    for (int64_t i = 0; i < n; ++i) {
      if (!G.free[i] || snap[i] >= 0) continue;
      count.clear();
      for_neighbours(i, [&](int64_t j) {
        if (snap[j] < 0) return;
        for (auto& c : count)
          if (c.first == snap[j]) {
            ++c.second;
            return;
          }
        count.push_back({snap[j], 1});
      });
      if (count.empty()) continue;
      int best = 0;
      for (auto& c : count) best = std::max(best, c.second);
      int64_t pick = -1;
      for (auto& c : count)
        if (c.second == best && (pick < 0 || first[c.first] < first[pick])) pick = c.first;
      lab[i] = pick;
    }
    for (int64_t i = 0; i < n; ++i) {  // stage IV: leftovers
      if (!G.free[i] || lab[i] >= 0) continue;
      const int64_t a = (int64_t)point.size();
      point.push_back(none);
      lab[i] = a;
      for_neighbours(i, [&](int64_t j) {
        if (lab[j] < 0) lab[j] = a;
      });
    }
  }
  // coarse nodes in order of their aggregate's smallest row
  std::vector<int32_t> cidx(point.size(), -1);
  local.assign(n, -1);
  cxyz.clear();
  for (int64_t i = 0; i < n; ++i) {
    if (lab[i] < 0) continue;
    if (cidx[lab[i]] < 0) {
      cidx[lab[i]] = (int32_t)cxyz.size();
      const std::array<int32_t, 3>& p = point[lab[i]];
      cxyz.push_back(p[0] < 0 ? p : std::array<int32_t, 3>{p[0] / 3, p[1] / 3, p[2] / 3});
    }
    local[i] = cidx[lab[i]];
  }
}

// Next level: aggregates of every region (global coarse rows in F.agg), numbering, Galerkin products.
void coarsen(const Hybrid& hy, HLevel& F, HLevel& C, const std::vector<int32_t>& kinds) {
  const int dim = hy.dim;
  for (int a = 0; a < dim; ++a)
    RMG_REQUIRE((F.shape[a] - 1) % 3 == 0 && F.shape[a] >= 7, RMG_ERR_SHAPE,
                "hybrid: composite extent - 1 must be divisible by 3 and at least 6 on every aggregated level");
  const std::vector<int32_t> mult = multiplicity(F);
  const int nreg = (int)F.regs.size();
  std::vector<std::vector<int32_t>> local(nreg);
  std::vector<std::vector<std::array<int32_t, 3>>> cxyz(nreg);
  parallel_for(nreg, [&](int64_t k) {
    aggregate(F.regs[k], kinds[k] != 0, mult, F.shape, hy.mask, dim, local[k], cxyz[k]);
  });
  for (int a = 0; a < 3; ++a) C.shape[a] = a < dim ? (F.shape[a] - 1) / 3 + 1 : 1;
  C.regs.assign(nreg, HRegionHost());
  C.off.assign(nreg + 1, 0);
  std::unordered_map<int64_t, int64_t> ids;
  int64_t next = 0;
  for (int k = 0; k < nreg; ++k) {
    HRegionHost& G = C.regs[k];
    for (const auto& p : cxyz[k]) {
      int64_t id;
      if (p[0] >= 0) {
        auto it = ids.find(pack(p));
        if (it == ids.end()) it = ids.emplace(pack(p), next++).first;
        id = it->second;
      } else {
        id = next++;
      }
      G.comp.push_back(id);
      G.xyz.push_back(p);
      G.free.push_back(1);
    }
    C.off[k + 1] = C.off[k] + G.n();
  }
  C.ncomp = next;
  F.agg.assign(F.off[nreg], -1);
  for (int k = 0; k < nreg; ++k)
    for (size_t i = 0; i < local[k].size(); ++i)
      if (local[k][i] >= 0) F.agg[F.off[k] + i] = (int32_t)(C.off[k] + local[k][i]);
  // Galerkin product per region: coarse row a sums the rows of its aggregate, columns mapped by P
  parallel_for(nreg, [&](int64_t k) {
    const HRegionHost& A = F.regs[k];
    HRegionHost& G = C.regs[k];
    const int64_t nc = G.n();
    std::vector<int64_t> rptr(nc + 1, 0);
    for (int32_t a : local[k])
      if (a >= 0) ++rptr[a + 1];
    for (int64_t a = 0; a < nc; ++a) rptr[a + 1] += rptr[a];
    std::vector<int64_t> rows(rptr[nc]), fill(rptr.begin(), rptr.end() - 1);
    for (int64_t i = 0; i < A.n(); ++i)
      if (local[k][i] >= 0) rows[fill[local[k][i]]++] = i;
    std::vector<double> acc(nc, 0.0);
    std::vector<int32_t> touched;
    std::vector<uint8_t> mark(nc, 0);
    G.ptr.assign(1, 0);
    for (int64_t a = 0; a < nc; ++a) {
      touched.clear();
      for (int64_t e = rptr[a]; e < rptr[a + 1]; ++e) {
        const int64_t i = rows[e];
        for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
          const int32_t b = local[k][A.col[q]];
          if (b < 0) continue;
          if (!mark[b]) {
            mark[b] = 1;
            touched.push_back(b);
          }
          acc[b] += A.val[q];
        }
      }
      std::sort(touched.begin(), touched.end());
      for (int32_t b : touched) {
        if (acc[b] != 0.0) {
          G.col.push_back(b);
          G.val.push_back(acc[b]);
        }
        acc[b] = 0.0;
        mark[b] = 0;
      }
      G.ptr.push_back((int64_t)G.col.size());
    }
  });
}

// Dependency levels of the forward (lower triangle) or backward (upper triangle) sweep of every
// region, flattened: region k owns levels reg[k] .. reg[k+1]-1, level v owns rows lv[v] .. lv[v+1]-1.
void gs_schedule(const HLevel& H, bool backward, std::vector<int32_t>& reg, std::vector<int32_t>& lv,
                 std::vector<int32_t>& rows) {
  const int nreg = (int)H.regs.size();
  std::vector<std::vector<int32_t>> order(nreg), bounds(nreg);  // per region: rows by level, level ends
  parallel_for(nreg, [&](int64_t k) {
    const HRegionHost& G = H.regs[k];
    const int64_t n = G.n();
    std::vector<int32_t> level(n, 0);
    int32_t nlev = 0;
    for (int64_t s = 0; s < n; ++s) {
      const int64_t i = backward ? n - 1 - s : s;
      int32_t l = 0;
      for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e) {
        const int64_t j = G.col[e];
        if (backward ? j > i : j < i) l = std::max(l, level[j] + 1);
      }
      level[i] = l;
      nlev = std::max(nlev, l + 1);
    }
    std::vector<int32_t> cnt(nlev + 1, 0);
    for (int32_t l : level) ++cnt[l + 1];
    for (int32_t l = 0; l < nlev; ++l) cnt[l + 1] += cnt[l];
    order[k].resize(n);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i) order[k][fill[level[i]]++] = (int32_t)(H.off[k] + i);
    bounds[k].assign(cnt.begin() + 1, cnt.end());
  });
  reg.assign(1, 0);
  lv.assign(1, 0);
  rows.clear();
  for (int k = 0; k < nreg; ++k) {
    const int32_t base = (int32_t)rows.size();
    rows.insert(rows.end(), order[k].begin(), order[k].end());
    for (int32_t b : bounds[k]) lv.push_back(base + b);
    reg.push_back((int32_t)lv.size() - 1);
  }
}

// Device arrays of one level (coarsest: the dense inverse instead of transfers).
void upload_level(rmg_handle* h, HLevel& H, bool coarsest, int64_t nc_next) {
  hipStream_t st = h->stream;
  HLevelDev& D = H.dev;
  const int nreg = (int)H.regs.size();
  const int64_t n = H.off[nreg];
  RMG_REQUIRE(n < ((int64_t)1 << 31), RMG_ERR_SHAPE, "hybrid: too many regional rows on one level");
  D.n = n;
  D.nreg = nreg;
  // ELL slices
  const int64_t ns = (n + 63) / 64;
  std::vector<int64_t> sptr(ns + 1, 0);
  std::vector<int32_t> rlen(n);
  std::vector<int64_t> rbeg(n);
  std::vector<int32_t> rreg(n);
  for (int k = 0; k < nreg; ++k)
    for (int64_t i = 0; i < H.regs[k].n(); ++i) {
      rbeg[H.off[k] + i] = H.regs[k].ptr[i];
      rlen[H.off[k] + i] = (int32_t)(H.regs[k].ptr[i + 1] - H.regs[k].ptr[i]);
      rreg[H.off[k] + i] = k;
    }
  for (int64_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int64_t i = s * 64; i < std::min(n, (s + 1) * 64); ++i) w = std::max(w, rlen[i]);
    sptr[s + 1] = sptr[s] + 64 * (int64_t)w;
  }
  std::vector<int32_t> col(sptr[ns], 0);
  std::vector<double> val(sptr[ns], 0.0);
  parallel_for(ns, [&](int64_t s) {
    const int64_t w = (sptr[s + 1] - sptr[s]) / 64;
    for (int64_t i = s * 64; i < std::min(n, (s + 1) * 64); ++i) {
      const HRegionHost& G = H.regs[rreg[i]];
      for (int64_t e = 0; e < w; ++e) {
        const int64_t at = sptr[s] + 64 * e + (i & 63);
        if (e < rlen[i]) {
          col[at] = (int32_t)(H.off[rreg[i]] + G.col[rbeg[i] + e]);
          val[at] = G.val[rbeg[i] + e];
        } else {
          col[at] = (int32_t)i;
        }
      }
    }
  });
  upload(D.sptr, sptr, st);
  upload(D.col, col, st);
  upload(D.val, val, st);
  // composite diagonal, multiplicity, interface groups
  const std::vector<int32_t> mult = multiplicity(H);
  std::vector<double> diag(H.ncomp, 0.0);
  std::vector<int64_t> rowcomp64(n);
  for (int k = 0; k < nreg; ++k) {
    const HRegionHost& G = H.regs[k];
    for (int64_t i = 0; i < G.n(); ++i) {
      rowcomp64[H.off[k] + i] = G.comp[i];
      for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e)
        if (G.col[e] == i) diag[G.comp[i]] += G.val[e];
    }
  }
  std::vector<double> dinv(n), invm(n);
  for (int64_t i = 0; i < n; ++i) {
    const double d = diag[rowcomp64[i]];
    RMG_REQUIRE(d > 0.0, RMG_ERR_NUMERIC, "hybrid: composite diagonal not positive");
    dinv[i] = 1.0 / d;
    invm[i] = 1.0 / (double)mult[rowcomp64[i]];
  }
  upload(D.dinv, dinv, st);
  upload(D.invm, invm, st);
  std::vector<int64_t> gstart(H.ncomp + 1, 0);
  for (int64_t c = 0; c < H.ncomp; ++c) gstart[c + 1] = gstart[c] + (mult[c] >= 2 ? mult[c] : 0);
  std::vector<int32_t> gcopy(gstart[H.ncomp]);
  std::vector<int64_t> gfill(gstart.begin(), gstart.end() - 1);
  for (int64_t i = 0; i < n; ++i)  // rows in region order: copies in ascending region order
    if (mult[rowcomp64[i]] >= 2) gcopy[gfill[rowcomp64[i]]++] = (int32_t)i;
  std::vector<int64_t> gptr(1, 0);
  for (int64_t c = 0; c < H.ncomp; ++c)
    if (mult[c] >= 2) gptr.push_back(gstart[c + 1]);
  D.ngroups = (int64_t)gptr.size() - 1;
  upload(D.gptr, gptr, st);
  upload(D.gcopy, gcopy, st);
  for (DBuf* v : {&D.b, &D.u, &D.r, &D.d, &D.y, &D.b2, &D.t}) v->alloc(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
  if (coarsest) {
    RMG_REQUIRE(H.ncomp <= 20000, RMG_ERR_ARG, "hybrid: coarsest composite problem too large for the dense solver");
    const int nc = (int)H.ncomp;
    D.nc = nc;
    std::vector<double> abar((size_t)nc * nc, 0.0);
    std::vector<int32_t> owner(nc, -1), rowcomp(n);
    for (int k = 0; k < nreg; ++k) {
      const HRegionHost& G = H.regs[k];
      for (int64_t i = 0; i < G.n(); ++i) {
        const int64_t gi = G.comp[i];
        rowcomp[H.off[k] + i] = (int32_t)gi;
        if (owner[gi] < 0) owner[gi] = (int32_t)(H.off[k] + i);
        for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e) abar[(size_t)gi * nc + G.comp[G.col[e]]] += G.val[e];
      }
    }
    upload(D.owner, owner, st);
    upload(D.rowcomp, rowcomp, st);
    D.ainv.alloc(sizeof(double) * (size_t)nc * nc);
    RMG_HIP(hipMemcpyAsync(D.ainv.p, abar.data(), sizeof(double) * abar.size(), hipMemcpyHostToDevice, st));
    RMG_HIP(hipStreamSynchronize(st));  // abar is a local table
    D.cvec.alloc(sizeof(double) * nc);
    D.cvec2.alloc(sizeof(double) * nc);
    launch_gauss_jordan(D.ainv.as<double>(), nc, st);
    DBuf flag;
    flag.alloc(sizeof(int));
    RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
    launch_check_inverse(D.ainv.as<double>(), nc, flag.as<int>(), st);
    int hflag = 0;
    RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    RMG_HIP(hipStreamSynchronize(st));
    RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "hybrid: coarsest composite matrix is singular");
    return;
  }
  for (int dir = 0; dir < 2; ++dir) {  // Gauss-Seidel schedules with their couplings by position
    const bool backward = dir == 1;
    HLevelDev::Sweep& S = backward ? D.bwd : D.fwd;
    std::vector<int32_t> reg, lv, rows;
    gs_schedule(H, backward, reg, lv, rows);
    std::vector<int32_t> tcnt(n);
    for (int64_t t = 0; t < n; ++t) {
      const int64_t i = rows[t];
      const HRegionHost& G = H.regs[rreg[i]];
      const int64_t li = i - H.off[rreg[i]];
      int32_t c = 0;
      for (int64_t e = G.ptr[li]; e < G.ptr[li + 1]; ++e) c += backward ? G.col[e] > li : G.col[e] < li;
      tcnt[t] = c;
    }
    std::vector<int64_t> tsptr(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
      int32_t w = 0;
      for (int64_t t = s * 64; t < std::min(n, (s + 1) * 64); ++t) w = std::max(w, tcnt[t]);
      tsptr[s + 1] = tsptr[s] + 64 * (int64_t)w;
    }
    std::vector<int32_t> tcol(tsptr[ns], 0);
    std::vector<double> tval(tsptr[ns], 0.0);
    parallel_for(ns, [&](int64_t s) {
      for (int64_t t = s * 64; t < std::min(n, (s + 1) * 64); ++t) {
        const int64_t i = rows[t];
        const HRegionHost& G = H.regs[rreg[i]];
        const int64_t li = i - H.off[rreg[i]];
        int64_t at = tsptr[s] + (t & 63);
        for (int64_t e = G.ptr[li]; e < G.ptr[li + 1]; ++e)
          if (backward ? G.col[e] > li : G.col[e] < li) {
            tcol[at] = (int32_t)(H.off[rreg[i]] + G.col[e]);
            tval[at] = G.val[e];
            at += 64;
          }
      }
    });
    upload(S.reg, reg, st);
    upload(S.lv, lv, st);
    upload(S.rows, rows, st);
    upload(S.tsptr, tsptr, st);
    upload(S.tcnt, tcnt, st);
    upload(S.tcol, tcol, st);
    upload(S.tval, tval, st);
  }
  // transfers: aggregate of every row; rows of every coarse row
  const int64_t nc = nc_next;
  std::vector<int64_t> cptr(nc + 1, 0);
  for (int32_t a : H.agg)
    if (a >= 0) ++cptr[a + 1];
  for (int64_t c = 0; c < nc; ++c) cptr[c + 1] += cptr[c];
  std::vector<int32_t> crows(cptr[nc]);
  std::vector<int64_t> cfill(cptr.begin(), cptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    if (H.agg[i] >= 0) crows[cfill[H.agg[i]]++] = (int32_t)i;
  upload(D.agg, H.agg, st);
  upload(D.cptr, cptr, st);
  upload(D.crows, crows, st);
  RMG_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------- cycle
void residual(const HLevelDev& L, const double* b, const double* u, double* out, bool scaled, hipStream_t st) {
  launch_hyb_spmv(L, u, L.y.as<double>(), st);
  launch_group_reduce(L.gptr.as<int64_t>(), L.gcopy.as<int>(), L.ngroups, L.y.as<double>(), false, st);
  launch_hyb_finish(L.n, b, L.y.as<double>(), scaled ? L.invm.as<double>() : nullptr, out, st);
}

void gs_sweep(const HLevelDev& L, const double* b, double* u, bool zero, bool backward, double omega, hipStream_t st) {
  if (zero) {  // u = 0: the residual is b, and the corrections are the new iterate
    launch_hyb_gs(L, b, u, omega, backward, st);
    launch_group_reduce(L.gptr.as<int64_t>(), L.gcopy.as<int>(), L.ngroups, u, true, st);
    return;
  }
  residual(L, b, u, L.r.as<double>(), false, st);
  launch_hyb_gs(L, L.r.as<double>(), L.d.as<double>(), omega, backward, st);
  launch_group_reduce(L.gptr.as<int64_t>(), L.gcopy.as<int>(), L.ngroups, L.d.as<double>(), true, st);
  launch_add(L.n, L.d.as<double>(), u, st);
}

void smooth(rmg_handle* h, const HLevelDev& L, const double* b, double* u, bool zero) {
  hipStream_t st = h->stream;
  const double w = h->opt.jacobi_omega;
  for (int it = 0; it < h->opt.cheb_degree; ++it) {
    const bool z0 = zero && it == 0;
    if (h->opt.smoother == 1) {
      if (z0) {
        launch_hyb_jacobi(L.n, w, L.dinv.as<double>(), b, u, true, st);
      } else {
        residual(L, b, u, L.r.as<double>(), false, st);
        launch_hyb_jacobi(L.n, w, L.dinv.as<double>(), L.r.as<double>(), u, false, st);
      }
    } else {
      gs_sweep(L, b, u, z0, false, w, st);
      if (h->opt.smoother == 4) gs_sweep(L, b, u, false, true, w, st);
    }
  }
}

void cycle(rmg_handle* h, int l, const double* b, double* z) {
  Hybrid& hy = *h->hy;
  const int last = (int)hy.lv.size() - 1;
  const HLevelDev& L = hy.lv[l]->dev;
  hipStream_t st = h->stream;
  if (l == last) {
    launch_hyb_coarse(L, b, z, st);
    return;
  }
  smooth(h, L, b, z, true);
  residual(L, b, z, L.r.as<double>(), true, st);  // divided by multiplicity (Section 3.3)
  const HLevelDev& C = hy.lv[l + 1]->dev;
  launch_hyb_restrict(C.n, L.cptr.as<int64_t>(), L.crows.as<int>(), L.r.as<double>(), C.b.as<double>(), st);
  launch_group_reduce(C.gptr.as<int64_t>(), C.gcopy.as<int>(), C.ngroups, C.b.as<double>(), false, st);
  cycle(h, l + 1, C.b.as<double>(), C.u.as<double>());
  if (h->opt.cycle_gamma == 2 && l + 1 < last) {  // W-cycle: a second coarse cycle on its residual
    residual(C, C.b.as<double>(), C.u.as<double>(), C.b2.as<double>(), false, st);
    cycle(h, l + 1, C.b2.as<double>(), C.t.as<double>());
    launch_add(C.n, C.t.as<double>(), C.u.as<double>(), st);
  }
  launch_hyb_prolong(L.n, L.agg.as<int>(), C.u.as<double>(), z, st);
  smooth(h, L, b, z, false);
}

const HLevel& level_of(rmg_handle* h, int level) {
  RMG_REQUIRE(h->hy != nullptr, RMG_ERR_NOT_SETUP, "no hybrid hierarchy");
  RMG_REQUIRE(level >= 0 && level < (int)h->hy->lv.size(), RMG_ERR_ARG, "level out of range");
  return *h->hy->lv[level];
}

}  // namespace

void hybrid_destroy(rmg_handle* h) {
  delete h->hy;
  h->hy = nullptr;
}

void hybrid_setup(rmg_handle* h) {
  hybrid_destroy(h);
  const rmg_options& o = h->opt;
  Level& L0 = *h->levels[0];
  RMG_REQUIRE(L0.ndof == 1, RMG_ERR_ARG, "hybrid hierarchy: scalar problems only");
  std::vector<int32_t> kinds = h->region_kind;
  if (kinds.size() != (size_t)L0.nreg) kinds.assign(L0.nreg, 0);
  auto* hy = new Hybrid();
  h->hy = hy;
  hy->dim = L0.dim;
  hy->mask = L0.mask;
  for (int l = 0; l < o.nlevels; ++l) hy->lv.push_back(std::make_unique<HLevel>());
  finest_level(h, *hy->lv[0]);
  for (int l = 0; l + 1 < o.nlevels; ++l) coarsen(*hy, *hy->lv[l], *hy->lv[l + 1], kinds);
  for (int l = 0; l < o.nlevels; ++l) {
    const bool last = l == o.nlevels - 1;
    upload_level(h, *hy->lv[l], last, last ? 0 : hy->lv[l + 1]->off.back());
  }
}

void hybrid_cycle(rmg_handle* h, const double* b, double* z) { cycle(h, 0, b, z); }

int64_t aggregate_plain(const std::vector<int64_t>& ptr, const std::vector<int32_t>& col,
                        const std::vector<double>& val, const std::vector<uint8_t>& free, std::vector<int32_t>& agg) {
  HRegionHost G;
  const int64_t n = (int64_t)free.size();
  G.ptr = ptr;
  G.col = col;
  G.val = val;
  G.free = free;
  G.comp.resize(n);
  for (int64_t i = 0; i < n; ++i) G.comp[i] = i;
  G.xyz.assign(n, {-1, -1, -1});
  const std::vector<int32_t> mult(n, 1);  // no interface: the structured stage never applies
  const int shape[3] = {1, 1, 1};
  std::vector<std::array<int32_t, 3>> cxyz;
  aggregate(G, true, mult, shape, 0u, 1, agg, cxyz);
  return (int64_t)cxyz.size();
}

}  // namespace rmg

// ------------------------------------------------------------------ C entry points
using namespace rmg;

rmg_status rmg_set_region_kinds(rmg_handle* h, const int32_t* kinds) {
  API_BEGIN
  RMG_REQUIRE(h && h->have_regions, RMG_ERR_NOT_SETUP, "regions not built");
  RMG_REQUIRE(kinds != nullptr, RMG_ERR_ARG, "null kinds");
  for (int k = 0; k < h->nreg; ++k)
    RMG_REQUIRE(kinds[k] == 0 || kinds[k] == 1, RMG_ERR_ARG, "region kinds must be 0 (structured) or 1 (unstructured)");
  h->region_kind.assign(kinds, kinds + h->nreg);
  API_END
}

rmg_status rmg_hybrid_level_info(rmg_handle* h, int level, int64_t* n_regional, int64_t* n_composite, int64_t* nnz) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  const HLevel& H = level_of(h, level);
  int64_t z = 0;
  for (const HRegionHost& G : H.regs) z += (int64_t)G.col.size();
  if (n_regional) *n_regional = H.off.back();
  if (n_composite) *n_composite = H.ncomp;
  if (nnz) *nnz = z;
  API_END
}

rmg_status rmg_hybrid_aggregates(rmg_handle* h, int level, int32_t* agg) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && agg != nullptr, RMG_ERR_ARG, "null argument");
  const HLevel& H = level_of(h, level);
  RMG_REQUIRE(level + 1 < (int)h->hy->lv.size(), RMG_ERR_ARG, "the coarsest level has no aggregates");
  std::copy(H.agg.begin(), H.agg.end(), agg);
  API_END
}

rmg_status rmg_hybrid_composite_ids(rmg_handle* h, int level, int64_t* comp) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && comp != nullptr, RMG_ERR_ARG, "null argument");
  const HLevel& H = level_of(h, level);
  for (size_t k = 0; k < H.regs.size(); ++k) std::copy(H.regs[k].comp.begin(), H.regs[k].comp.end(), comp + H.off[k]);
  API_END
}

rmg_status rmg_hybrid_matrix(rmg_handle* h, int level, int64_t* rowptr, int32_t* colind, double* values) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && rowptr && colind && values, RMG_ERR_ARG, "null argument");
  const HLevel& H = level_of(h, level);
  int64_t at = 0;
  rowptr[0] = 0;
  for (size_t k = 0; k < H.regs.size(); ++k) {
    const HRegionHost& G = H.regs[k];
    for (int64_t i = 0; i < G.n(); ++i) {
      for (int64_t e = G.ptr[i]; e < G.ptr[i + 1]; ++e, ++at) {
        colind[at] = (int32_t)(H.off[k] + G.col[e]);
        values[at] = G.val[e];
      }
      rowptr[H.off[k] + i + 1] = at;
    }
  }
  API_END
}
