// AMG coarse solver below the region hierarchy (Section 3.5, second coarse-level option): when
// the coarsest composite operator Abar is too large for a direct solver, the region cycle's coarse
// solve is one AMG V-cycle on Abar.  Smoothed aggregation, after the SA-AMG the section cites:
//  * aggregates: the staged plain aggregation of the hybrid hierarchy without its interface stage
//    (one composite matrix has no interfaces), on the graph of couplings |a_ij| >
//    1e-12 sqrt(a_ii a_jj) between free rows (rounding residue of a Galerkin product is no
//    coupling); Dirichlet rows are not aggregated;
//  * systems (3D elasticity): the near-null space from the region hierarchy, the six rigid-body
//    modes at the coarsest nodes' positions on the finest lattice; aggregation on the node graph
//    (blocks of Frobenius norm > 1e-12 sqrt(||A_II|| ||A_JJ||)), the tentative prolongator from a
//    thin QR of each aggregate's rows of the near-null space (diag R >= 0), coarse nodes = the
//    aggregates with six dofs each and near-null space R;
//  * tentative prolongator T (a 1 per aggregated row), smoothed P = (I - omega D^-1 A) T with
//    omega = 4 / (3 rho) and rho = max_i sum_j |a_ij| / a_ii (Gershgorin's bound on
//    lambda_max(D^-1 A));
//  * coarse operators P^T A P until a level has at most amg_coarse_size rows (or stops
//    shrinking); that level is inverted densely;
//  * V-cycle: the region levels' degree-K Chebyshev recurrence on [rho / eta, rho] before and after
//    each coarse correction.
// The hierarchy is built on the host once per setup; the cycle runs on the device, on the
// handle's stream, with no host synchronisation (it can be captured in a graph).
#include <algorithm>
#include <cmath>

#include "amg.h"
#include "hybrid.h"
#include "kernels.h"

namespace rmg {
namespace {

constexpr double kStrength = 1e-12;  // relative size below which an entry is no graph coupling
constexpr int kMaxAmgLevels = 20;
constexpr int kRigidModes = 6;       // near-null space of 3D elasticity

void spgemm(const Csr& X, const Csr& Y, Csr& Z);

void stencil_offset_host(int npts, int s, int& dx, int& dy, int& dz) {
  if (npts == 27) {
    dx = s % 3 - 1;
    dy = (s / 3) % 3 - 1;
    dz = s / 9 - 1;
  } else {
    dx = s % 3 - 1;
    dy = s / 3 - 1;
    dz = 0;
  }
}

// Abar = Psi-bar [[Abar]] Psi-bar^T of the coarsest region level in CSR (copies summed in
// ascending region order, exact zeros dropped), the free flag of every composite row, and the
// owner copy of every composite node (the lowest region containing it).
void composite_matrix(rmg_handle* h, const Level& L, Csr& A, std::vector<uint8_t>& free, std::vector<int32_t>& owner) {
  hipStream_t st = h->stream;
  const int nd = L.ndof, nc = L.ncoef();
  const int64_t n = L.ncomp * nd;
  std::vector<double> coef(coef_elems(L.n, nc));
  RMG_HIP(hipMemcpyAsync(coef.data(), L.coef.p, sizeof(double) * coef.size(), hipMemcpyDeviceToHost, st));
  RMG_HIP(hipStreamSynchronize(st));
  std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)n);
  owner.assign((size_t)L.ncomp, -1);
  const int cx = L.comp[0], cy = L.comp[1];
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    for (int z = 0; z < R.ez; ++z)
      for (int y = 0; y < R.ey; ++y)
        for (int x = 0; x < R.ex; ++x) {
          const int64_t li = ((int64_t)z * R.ey + y) * R.ex + x;
          const int64_t i = ((int64_t)(R.oz + z) * cy + (R.oy + y)) * cx + (R.ox + x);
          if (owner[i] < 0) owner[i] = (int32_t)(R.off + li);
          for (int s = 0; s < L.npts; ++s) {
            int dx, dy, dz;
            stencil_offset_host(L.npts, s, dx, dy, dz);
            if (x + dx < 0 || x + dx >= R.ex || y + dy < 0 || y + dy >= R.ey || z + dz < 0 || z + dz >= R.ez) continue;
            const int64_t j = ((int64_t)(R.oz + z + dz) * cy + (R.oy + y + dy)) * cx + (R.ox + x + dx);
            for (int a = 0; a < nd; ++a)
              for (int b = 0; b < nd; ++b) {  // block (a, b) of offset s
                const double v = coef[coef_index(R.off + li, (s * nd + a) * nd + b, nc)];
                if (v != 0.0) rows[i * nd + a].push_back({(int32_t)(j * nd + b), v});
              }
          }
        }
  }
  A.rows = A.cols = n;
  A.ptr.assign(1, 0);
  A.col.clear();
  A.val.clear();
  for (int64_t i = 0; i < n; ++i) {
    auto& r = rows[i];
    std::stable_sort(r.begin(), r.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t e = 0; e < r.size();) {
      const int32_t j = r[e].first;
      double acc = 0.0;
      for (; e < r.size() && r[e].first == j; ++e) acc += r[e].second;  // region order
      if (acc != 0.0) {
        A.col.push_back(j);
        A.val.push_back(acc);
      }
    }
    A.ptr.push_back((int64_t)A.col.size());
    std::vector<std::pair<int32_t, double>>().swap(r);
  }
  free.assign((size_t)n, 1);
  const unsigned m = L.mask;
  for (int64_t i = 0; i < L.ncomp; ++i) {
    const int gx = (int)(i % cx), gy = (int)((i / cx) % cy), gz = (int)(i / ((int64_t)cx * cy));
    const bool dir = ((m & 1u) && gx == 0) || ((m & 2u) && gx == cx - 1) || ((m & 4u) && gy == 0) ||
                     ((m & 8u) && gy == cy - 1) || ((m & 16u) && gz == 0) || ((m & 32u) && gz == L.comp[2] - 1);
    for (int a = 0; a < nd; ++a) free[i * nd + a] = dir ? 0 : 1;  // a Dirichlet node fixes all its dofs
  }
}

// Positions of the coarsest level's composite nodes (x fastest) on the finest lattice, relative
// to its centre: every coarse lattice line is the line of the level above at the region's coarse
// point min(3 X, extent - 1), followed up to level 0.
std::vector<double> finest_coordinates(rmg_handle* h) {
  const int nl = (int)h->levels.size();
  const Level& Lc = *h->levels[nl - 1];
  std::vector<std::vector<double>> axis(3);
  for (int d = 0; d < 3; ++d) {
    std::vector<int64_t> p((size_t)Lc.comp[d]);
    for (int64_t i = 0; i < Lc.comp[d]; ++i) p[(size_t)i] = i;
    for (int l = nl - 1; l >= 1; --l) {
      const Level& C = *h->levels[l];
      const Level& F = *h->levels[l - 1];
      std::vector<int64_t> line((size_t)C.comp[d], -1);
      for (int k = 0; k < C.nreg; ++k) {
        const int co[3] = {C.regs[k].ox, C.regs[k].oy, C.regs[k].oz}, ce[3] = {C.regs[k].ex, C.regs[k].ey, C.regs[k].ez};
        const int fo[3] = {F.regs[k].ox, F.regs[k].oy, F.regs[k].oz}, fe[3] = {F.regs[k].ex, F.regs[k].ey, F.regs[k].ez};
        for (int X = 0; X < ce[d]; ++X) line[(size_t)(co[d] + X)] = fo[d] + std::min(3 * X, fe[d] - 1);
      }
      for (auto& v : p) {
        RMG_REQUIRE(line[(size_t)v] >= 0, RMG_ERR_SHAPE, "internal: coarse lattice line without a fine line");
        v = line[(size_t)v];
      }
    }
    const double c = 0.5 * (h->levels[0]->comp[d] - 1);
    axis[d].resize(p.size());
    for (size_t i = 0; i < p.size(); ++i) axis[d][i] = (double)p[i] - c;
  }
  std::vector<double> X((size_t)Lc.ncomp * 3);
  for (int64_t i = 0; i < Lc.ncomp; ++i) {
    const int64_t gx = i % Lc.comp[0], gy = (i / Lc.comp[0]) % Lc.comp[1], gz = i / ((int64_t)Lc.comp[0] * Lc.comp[1]);
    X[(size_t)i * 3] = axis[0][(size_t)gx];
    X[(size_t)i * 3 + 1] = axis[1][(size_t)gy];
    X[(size_t)i * 3 + 2] = axis[2][(size_t)gz];
  }
  return X;
}

// Rigid-body modes (rows node-major, dof fastest; k = 6 columns, row-major): translations, then
// the rotations (-y, x, 0), (0, -z, y), (z, 0, -x).
std::vector<double> rigid_body_modes(const std::vector<double>& X) {
  const size_t n = X.size() / 3;
  std::vector<double> B(n * 3 * 6, 0.0);
  for (size_t i = 0; i < n; ++i) {
    const double x = X[i * 3], y = X[i * 3 + 1], z = X[i * 3 + 2];
    double* r0 = &B[(i * 3) * 6];
    double* r1 = &B[(i * 3 + 1) * 6];
    double* r2 = &B[(i * 3 + 2) * 6];
    r0[0] = r1[1] = r2[2] = 1.0;
    r0[3] = -y;
    r1[3] = x;
    r1[4] = -z;
    r2[4] = y;
    r0[5] = z;
    r2[5] = -x;
  }
  return B;
}

// Node graph of a system: nodes I, J (dof ranges nodes[I] .. nodes[I+1]) coupled when their block
// has Frobenius norm > kStrength sqrt(||A_II|| ||A_JJ||); free when all their rows are.
void node_graph(const Csr& A, const std::vector<int64_t>& nodes, const std::vector<uint8_t>& free,
                std::vector<int64_t>& ptr, std::vector<int32_t>& col, std::vector<double>& val,
                std::vector<uint8_t>& nfree) {
  const int64_t nn = (int64_t)nodes.size() - 1;
  std::vector<int32_t> node((size_t)A.rows);
  for (int64_t I = 0; I < nn; ++I)
    for (int64_t r = nodes[I]; r < nodes[I + 1]; ++r) node[(size_t)r] = (int32_t)I;
  std::vector<std::vector<std::pair<int32_t, double>>> sq((size_t)nn);  // squared block norms
  for (int64_t I = 0; I < nn; ++I) {
    auto& row = sq[(size_t)I];
    for (int64_t r = nodes[I]; r < nodes[I + 1]; ++r)
      for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) row.push_back({node[(size_t)A.col[e]], A.val[e] * A.val[e]});
    std::stable_sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    size_t w = 0;
    for (size_t e = 0; e < row.size();) {
      const int32_t J = row[e].first;
      double acc = 0.0;
      for (; e < row.size() && row[e].first == J; ++e) acc += row[e].second;
      row[w++] = {J, acc};
    }
    row.resize(w);
  }
  std::vector<double> dn((size_t)nn, 0.0);
  for (int64_t I = 0; I < nn; ++I)
    for (const auto& e : sq[(size_t)I])
      if (e.first == I) dn[(size_t)I] = std::sqrt(e.second);
  ptr.assign(1, 0);
  col.clear();
  val.clear();
  for (int64_t I = 0; I < nn; ++I) {
    for (const auto& e : sq[(size_t)I]) {
      const double f = std::sqrt(e.second);
      if (e.first == I || f > kStrength * std::sqrt(dn[(size_t)I] * dn[(size_t)e.first])) {
        col.push_back(e.first);
        val.push_back(f);
      }
    }
    ptr.push_back((int64_t)col.size());
  }
  nfree.assign((size_t)nn, 1);
  for (int64_t I = 0; I < nn; ++I)
    for (int64_t r = nodes[I]; r < nodes[I + 1]; ++r)
      if (!free[(size_t)r]) nfree[(size_t)I] = 0;
}

// Tentative prolongator of a system: per aggregate (its dofs ascending), B_a = Q R by modified
// Gram-Schmidt with a second pass (diag R > 0); Q fills the aggregate's k columns, R its k rows of
// the coarse near-null space Bc.  RMG_ERR_NUMERIC when an aggregate has fewer dofs than k or its
// rows of B are rank deficient.
void tentative_system(const std::vector<int32_t>& agg, int64_t na, const std::vector<int64_t>& nodes,
                      const std::vector<double>& B, int k, int64_t nrows, Csr& T, std::vector<double>& Bc) {
  std::vector<std::vector<int64_t>> members((size_t)na);
  for (size_t I = 0; I < agg.size(); ++I)
    if (agg[I] >= 0)
      for (int64_t r = nodes[I]; r < nodes[I + 1]; ++r) members[(size_t)agg[I]].push_back(r);
  std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)nrows);
  Bc.assign((size_t)na * k * k, 0.0);
  for (int64_t a = 0; a < na; ++a) {
    auto& dofs = members[(size_t)a];
    std::sort(dofs.begin(), dofs.end());
    const size_t m = dofs.size();
    RMG_REQUIRE(m >= (size_t)k, RMG_ERR_NUMERIC, "AMG: an aggregate has fewer dofs than the near-null space");
    std::vector<double> Q(m * k), R((size_t)k * k, 0.0);
    for (size_t i = 0; i < m; ++i)
      for (int j = 0; j < k; ++j) Q[i * k + j] = B[(size_t)dofs[i] * k + j];
    for (int j = 0; j < k; ++j) {
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < j; ++q) {
          double s = 0.0;
          for (size_t i = 0; i < m; ++i) s += Q[i * k + q] * Q[i * k + j];
          for (size_t i = 0; i < m; ++i) Q[i * k + j] -= s * Q[i * k + q];
          R[(size_t)q * k + j] += s;
        }
      double nrm = 0.0;
      for (size_t i = 0; i < m; ++i) nrm += Q[i * k + j] * Q[i * k + j];
      nrm = std::sqrt(nrm);
      RMG_REQUIRE(nrm > 0.0 && std::isfinite(nrm), RMG_ERR_NUMERIC, "AMG: near-null space rank deficient on an aggregate");
      R[(size_t)j * k + j] = nrm;
      for (size_t i = 0; i < m; ++i) Q[i * k + j] /= nrm;
    }
    for (size_t i = 0; i < m; ++i)
      for (int j = 0; j < k; ++j) rows[(size_t)dofs[i]].push_back({(int32_t)(a * k + j), Q[i * k + j]});
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Bc[((size_t)a * k + i) * k + j] = R[(size_t)i * k + j];
  }
  T.rows = nrows;
  T.cols = na * k;
  T.ptr.assign(1, 0);
  T.col.clear();
  T.val.clear();
  for (int64_t r = 0; r < nrows; ++r) {
    for (const auto& e : rows[(size_t)r]) {
      T.col.push_back(e.first);
      T.val.push_back(e.second);
    }
    T.ptr.push_back((int64_t)T.col.size());
  }
}

// P = T - omega D^-1 A T for a general T (exact zeros dropped, columns ascending).
void smooth_tentative(const Csr& A, const std::vector<double>& diag, const Csr& T, double omega, Csr& P) {
  Csr AT;
  spgemm(A, T, AT);
  P.rows = T.rows;
  P.cols = T.cols;
  P.ptr.assign(1, 0);
  P.col.clear();
  P.val.clear();
  for (int64_t i = 0; i < T.rows; ++i) {
    const double dinv = 1.0 / diag[(size_t)i];
    int64_t e = T.ptr[i], q = AT.ptr[i];
    while (e < T.ptr[i + 1] || q < AT.ptr[i + 1]) {
      const int32_t ce = e < T.ptr[i + 1] ? T.col[e] : INT32_MAX, cq = q < AT.ptr[i + 1] ? AT.col[q] : INT32_MAX;
      const int32_t c = std::min(ce, cq);
      const double t = ce == c ? T.val[e++] : 0.0;
      const double s = cq == c ? AT.val[q++] : 0.0;
      const double v = t - omega * (dinv * s);
      if (v != 0.0) {
        P.col.push_back(c);
        P.val.push_back(v);
      }
    }
    P.ptr.push_back((int64_t)P.col.size());
  }
}

std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d((size_t)A.rows, 0.0);
  for (int64_t i = 0; i < A.rows; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (A.col[e] == i) d[i] = A.val[e];
  return d;
}

// Z = X Y (sparse, ascending columns, exact zeros dropped).
void spgemm(const Csr& X, const Csr& Y, Csr& Z) {
  Z.rows = X.rows;
  Z.cols = Y.cols;
  Z.ptr.assign(1, 0);
  Z.col.clear();
  Z.val.clear();
  std::vector<double> acc((size_t)Y.cols, 0.0);
  std::vector<uint8_t> mark((size_t)Y.cols, 0);
  std::vector<int32_t> touched;
  for (int64_t i = 0; i < X.rows; ++i) {
    touched.clear();
    for (int64_t e = X.ptr[i]; e < X.ptr[i + 1]; ++e) {
      const int64_t k = X.col[e];
      const double x = X.val[e];
      for (int64_t q = Y.ptr[k]; q < Y.ptr[k + 1]; ++q) {
        const int32_t c = Y.col[q];
        if (!mark[c]) {
          mark[c] = 1;
          touched.push_back(c);
        }
        acc[c] += x * Y.val[q];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t c : touched) {
      if (acc[c] != 0.0) {
        Z.col.push_back(c);
        Z.val.push_back(acc[c]);
      }
      acc[c] = 0.0;
      mark[c] = 0;
    }
    Z.ptr.push_back((int64_t)Z.col.size());
  }
}

void transpose(const Csr& X, Csr& T) {
  T.rows = X.cols;
  T.cols = X.rows;
  T.ptr.assign((size_t)T.rows + 1, 0);
  for (int32_t c : X.col) ++T.ptr[c + 1];
  for (int64_t r = 0; r < T.rows; ++r) T.ptr[r + 1] += T.ptr[r];
  T.col.resize(X.col.size());
  T.val.resize(X.val.size());
  std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < X.rows; ++i)  // rows in order: ascending columns of T
    for (int64_t e = X.ptr[i]; e < X.ptr[i + 1]; ++e) {
      const int64_t at = fill[X.col[e]]++;
      T.col[at] = (int32_t)i;
      T.val[at] = X.val[e];
    }
}

// Aggregates of the free rows on the graph of non-negligible couplings.
int64_t aggregates(const Csr& A, const std::vector<double>& diag, const std::vector<uint8_t>& free,
                   std::vector<int32_t>& agg) {
  std::vector<int64_t> ptr(1, 0);
  std::vector<int32_t> col;
  std::vector<double> val;
  for (int64_t i = 0; i < A.rows; ++i) {
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int32_t j = A.col[e];
      if (j == i || std::fabs(A.val[e]) > kStrength * std::sqrt(std::fabs(diag[i] * diag[j]))) {
        col.push_back(j);
        val.push_back(A.val[e]);
      }
    }
    ptr.push_back((int64_t)col.size());
  }
  return aggregate_plain(ptr, col, val, free, agg);
}

// P = T - omega D^-1 A T (entries of a row in ascending coarse column, exact zeros dropped).
void smoothed_prolongator(const Csr& A, const std::vector<double>& diag, const std::vector<int32_t>& agg, int64_t nc,
                          double omega, Csr& P) {
  P.rows = A.rows;
  P.cols = nc;
  P.ptr.assign(1, 0);
  P.col.clear();
  P.val.clear();
  std::vector<double> s((size_t)nc, 0.0);
  std::vector<uint8_t> mark((size_t)nc, 0);
  std::vector<int32_t> touched;
  for (int64_t i = 0; i < A.rows; ++i) {
    touched.clear();
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {  // (A T)_ic, columns of A ascending
      const int32_t c = agg[A.col[e]];
      if (c < 0) continue;
      if (!mark[c]) {
        mark[c] = 1;
        touched.push_back(c);
      }
      s[c] += A.val[e];
    }
    if (agg[i] >= 0 && !mark[agg[i]]) {
      mark[agg[i]] = 1;
      touched.push_back(agg[i]);
    }
    std::sort(touched.begin(), touched.end());
    const double dinv = 1.0 / diag[i];
    for (int32_t c : touched) {
      const double t = agg[i] == c ? 1.0 : 0.0;
      const double v = t - omega * (dinv * s[c]);
      if (v != 0.0) {
        P.col.push_back(c);
        P.val.push_back(v);
      }
      s[c] = 0.0;
      mark[c] = 0;
    }
    P.ptr.push_back((int64_t)P.col.size());
  }
}

template <class T>
void upload(DBuf& d, const std::vector<T>& v, hipStream_t st) {
  d.alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) RMG_HIP(hipMemcpyAsync(d.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  RMG_HIP(hipStreamSynchronize(st));  // v may be a local table
}

void upload_sp(const Csr& M, SpDev& D, hipStream_t st) {
  const int64_t n = M.rows, ns = (n + 63) / 64;
  D.n = n;
  D.wave = M.nnz() > 32 * std::max<int64_t>(n, 1);
  if (D.wave) {  // long rows: plain CSR, a wavefront per row
    upload(D.sptr, M.ptr, st);
    upload(D.col, M.col, st);
    upload(D.val, M.val, st);
    return;
  }
  std::vector<int64_t> sptr((size_t)ns + 1, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int64_t w = 0;
    for (int64_t i = s * 64; i < std::min(n, (s + 1) * 64); ++i) w = std::max(w, M.ptr[i + 1] - M.ptr[i]);
    sptr[s + 1] = sptr[s] + 64 * w;
  }
  std::vector<int32_t> col((size_t)sptr[ns], 0);
  std::vector<double> val((size_t)sptr[ns], 0.0);
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t w = (sptr[s + 1] - sptr[s]) / 64;
    for (int64_t i = s * 64; i < std::min(n, (s + 1) * 64); ++i)
      for (int64_t e = 0; e < w; ++e) {
        const int64_t at = sptr[s] + 64 * e + (i & 63);
        const int64_t q = M.ptr[i] + e;
        col[at] = q < M.ptr[i + 1] ? M.col[q] : (int32_t)std::min<int64_t>(i, M.cols - 1);
        val[at] = q < M.ptr[i + 1] ? M.val[q] : 0.0;
      }
  }
  upload(D.sptr, sptr, st);
  upload(D.col, col, st);
  upload(D.val, val, st);
}

void cycle(rmg_handle* h, int l, const double* b, double* z) {
  Amg& amg = *h->amg;
  AmgLevel& L = *amg.lv[l];
  hipStream_t st = h->stream;
  const int64_t n = L.A.rows;
  if (l + 1 == (int)amg.lv.size()) {
    launch_dense_gemv(L.nc, L.ainv.as<double>(), b, z, st);
    return;
  }
  const int K = h->opt.cheb_degree;
  double* y = L.y.as<double>();
  double* d = L.d.as<double>();
  double* r = L.r.as<double>();
  const double* dinv = L.dinv.as<double>();
  auto chebyshev = [&](const double* r0, bool zero) {  // r0 = b - A z on entry
    launch_amg_cheb_first(n, L.inv_theta, dinv, r0, d, z, zero, st);
    for (int k = 1; k < K; ++k) {
      launch_sp_apply(L.dA, z, y, false, st);
      launch_amg_cheb_step(n, L.c1[k], L.c2[k], dinv, b, y, d, z, st);
    }
  };
  chebyshev(b, true);
  launch_sp_apply(L.dA, z, y, false, st);
  launch_amg_sub(n, b, y, r, st);
  AmgLevel& C = *amg.lv[l + 1];
  launch_sp_apply(L.dPt, r, C.b.as<double>(), false, st);
  cycle(h, l + 1, C.b.as<double>(), C.u.as<double>());
  launch_sp_apply(L.dP, C.u.as<double>(), z, true, st);
  launch_sp_apply(L.dA, z, y, false, st);
  launch_amg_sub(n, b, y, r, st);
  chebyshev(r, false);
}

const AmgLevel& amg_level(rmg_handle* h, int level) {
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  RMG_REQUIRE(h->amg != nullptr, RMG_ERR_NOT_SETUP, "no AMG coarse solver in the current hierarchy");
  RMG_REQUIRE(level >= 0 && level < (int)h->amg->lv.size(), RMG_ERR_ARG, "AMG level out of range");
  return *h->amg->lv[level];
}

}  // namespace

void amg_destroy(rmg_handle* h) {
  delete h->amg;
  h->amg = nullptr;
}

void amg_setup(rmg_handle* h, Level& L) {
  amg_destroy(h);
  RMG_REQUIRE(L.ndof == 1 || (L.ndof == 3 && L.dim == 3), RMG_ERR_ARG,
              "the AMG coarse solver handles scalar problems and 3D elasticity");
  hipStream_t st = h->stream;
  const rmg_options& o = h->opt;
  auto* amg = new Amg();
  h->amg = amg;
  Csr A;
  std::vector<uint8_t> free;
  std::vector<int32_t> owner;
  composite_matrix(h, L, A, free, owner);
  RMG_REQUIRE(A.rows < ((int64_t)1 << 31), RMG_ERR_SHAPE, "coarsest composite problem too large");
  L.nc = (int)A.rows;
  // systems: dof offsets of the nodes and the near-null space (rows x kRigidModes, row-major)
  const bool sys = L.ndof == 3;
  std::vector<int64_t> nodes;
  std::vector<double> B;
  if (sys) {
    nodes.resize((size_t)L.ncomp + 1);
    for (int64_t I = 0; I <= L.ncomp; ++I) nodes[(size_t)I] = 3 * I;
    B = rigid_body_modes(finest_coordinates(h));
  }
  upload(L.comp_owner, owner, st);
  L.cvec.alloc(sizeof(double) * (size_t)L.nc);
  L.cvec2.alloc(sizeof(double) * (size_t)L.nc);
  L.abar_host.clear();
  // levels: aggregate, smooth the tentative prolongator, Galerkin product
  for (;;) {
    amg->lv.push_back(std::make_unique<AmgLevel>());
    AmgLevel& V = *amg->lv.back();
    V.A = std::move(A);
    if (V.A.rows <= o.amg_coarse_size || (int)amg->lv.size() == kMaxAmgLevels) break;
    const std::vector<double> diag = diagonal(V.A);
    for (int64_t i = 0; i < V.A.rows; ++i)
      RMG_REQUIRE(diag[i] > 0.0, RMG_ERR_NUMERIC, "AMG: diagonal not positive");
    int64_t nc = 0;
    Csr T;
    std::vector<double> Bc;
    if (!sys) {
      nc = aggregates(V.A, diag, free, V.agg);
    } else {
      std::vector<int64_t> gp;
      std::vector<int32_t> gc;
      std::vector<double> gv;
      std::vector<uint8_t> nfree;
      node_graph(V.A, nodes, free, gp, gc, gv, nfree);
      const int64_t na = aggregate_plain(gp, gc, gv, nfree, V.agg);
      nc = na * kRigidModes;
      if (na > 0 && nc < V.A.rows) tentative_system(V.agg, na, nodes, B, kRigidModes, V.A.rows, T, Bc);
    }
    if (nc == 0 || nc >= V.A.rows) {
      V.agg.clear();
      break;
    }
    double rho = 0.0;
    for (int64_t i = 0; i < V.A.rows; ++i) {
      double s = 0.0;
      for (int64_t e = V.A.ptr[i]; e < V.A.ptr[i + 1]; ++e) s += std::fabs(V.A.val[e]);
      rho = std::max(rho, s / diag[i]);
    }
    V.rho = rho;
    V.omega = 4.0 / (3.0 * rho);
    if (!sys) smoothed_prolongator(V.A, diag, V.agg, nc, V.omega, V.P);
    else smooth_tentative(V.A, diag, T, V.omega, V.P);
    Csr AP, Pt;
    spgemm(V.A, V.P, AP);
    transpose(V.P, Pt);
    spgemm(Pt, AP, A);
    free.assign((size_t)nc, 1);
    if (sys) {  // the aggregates become the coarse nodes, with kRigidModes dofs each
      nodes.resize((size_t)nc / kRigidModes + 1);
      for (size_t I = 0; I < nodes.size(); ++I) nodes[I] = (int64_t)I * kRigidModes;
      B.swap(Bc);
    }
  }
  // device arrays
  const int nl = (int)amg->lv.size();
  for (int l = 0; l < nl; ++l) {
    AmgLevel& V = *amg->lv[l];
    const int64_t n = V.A.rows;
    for (DBuf* v : {&V.b, &V.u, &V.r, &V.d, &V.y}) v->alloc(sizeof(double) * (size_t)std::max<int64_t>(n, 1));
    if (l + 1 == nl) {  // dense inverse
      RMG_REQUIRE(n <= 20000, RMG_ERR_ARG, "AMG: the last level is too large for the dense solver");
      V.nc = (int)n;
      std::vector<double> dense((size_t)n * n, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t e = V.A.ptr[i]; e < V.A.ptr[i + 1]; ++e) dense[(size_t)i * n + V.A.col[e]] = V.A.val[e];
      V.ainv.alloc(sizeof(double) * dense.size());
      RMG_HIP(hipMemcpyAsync(V.ainv.p, dense.data(), sizeof(double) * dense.size(), hipMemcpyHostToDevice, st));
      RMG_HIP(hipStreamSynchronize(st));
      launch_gauss_jordan(V.ainv.as<double>(), V.nc, st);
      DBuf flag;
      flag.alloc(sizeof(int));
      RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
      launch_check_inverse(V.ainv.as<double>(), V.nc, flag.as<int>(), st);
      int hflag = 0;
      RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
      RMG_HIP(hipStreamSynchronize(st));
      RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "AMG: the last level's matrix is singular");
      continue;
    }
    upload_sp(V.A, V.dA, st);
    upload_sp(V.P, V.dP, st);
    Csr Pt;
    transpose(V.P, Pt);
    upload_sp(Pt, V.dPt, st);
    const std::vector<double> diag = diagonal(V.A);
    std::vector<double> dinv((size_t)n);
    for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / diag[i];
    upload(V.dinv, dinv, st);
    // Chebyshev on [rho / eta, rho] (the region levels' recurrence)
    const double alpha = V.rho / o.eig_ratio, beta = V.rho;
    const double theta = 0.5 * (alpha + beta), delta = 2.0 / (beta - alpha);
    double rc = 1.0 / (theta * delta);
    V.inv_theta = 1.0 / theta;
    V.c1.assign(o.cheb_degree, 0.0);
    V.c2.assign(o.cheb_degree, 0.0);
    for (int k = 1; k < o.cheb_degree; ++k) {
      const double rc_old = rc;
      rc = 1.0 / (2.0 * theta * delta - rc_old);
      V.c1[k] = rc * rc_old;
      V.c2[k] = 2.0 * rc * delta;
    }
  }
}

void amg_cycle(rmg_handle* h, const double* b, double* z) { cycle(h, 0, b, z); }

}  // namespace rmg

// ------------------------------------------------------------------ C entry points
using namespace rmg;

rmg_status rmg_amg_levels(rmg_handle* h, int* nlevels) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && nlevels != nullptr, RMG_ERR_ARG, "null argument");
  *nlevels = h->amg ? (int)h->amg->lv.size() : 0;
  API_END
}

rmg_status rmg_amg_level_info(rmg_handle* h, int level, int64_t* n, int64_t* nnz_a, int64_t* nnz_p) {
  API_BEGIN
  const AmgLevel& V = amg_level(h, level);
  if (n) *n = V.A.rows;
  if (nnz_a) *nnz_a = V.A.nnz();
  if (nnz_p) *nnz_p = V.P.nnz();
  API_END
}

rmg_status rmg_amg_matrix(rmg_handle* h, int level, int which, int64_t* rowptr, int32_t* colind, double* values) {
  API_BEGIN
  const AmgLevel& V = amg_level(h, level);
  RMG_REQUIRE(which == 0 || which == 1, RMG_ERR_ARG, "which must be 0 (matrix) or 1 (prolongator)");
  RMG_REQUIRE(rowptr && colind && values, RMG_ERR_ARG, "null argument");
  const Csr& M = which == 0 ? V.A : V.P;
  RMG_REQUIRE(which == 0 || !M.ptr.empty(), RMG_ERR_ARG, "the last AMG level has no prolongator");
  std::copy(M.ptr.begin(), M.ptr.end(), rowptr);
  std::copy(M.col.begin(), M.col.end(), colind);
  std::copy(M.val.begin(), M.val.end(), values);
  API_END
}
