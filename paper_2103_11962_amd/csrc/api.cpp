// C ABI of the regional multigrid library: validation, error mapping, entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"

namespace rmg {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(rmg_status code, const std::string& msg) { throw Error{code, msg}; }

// Reference Q1 Laplacian element matrix of a cube of side h: int grad phi_a . grad phi_b,
// 2x2x2 Gauss-Legendre quadrature, corner a = (a&1, (a>>1)&1, (a>>2)&1).
void q1_laplace_element(double h, double K[64]) {
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int i = 0; i < 64; ++i) K[i] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {g[qx], g[qy], g[qz]};
        double grad[8][3];
        for (int a = 0; a < 8; ++a) {
          const int c[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
          double f[3], df[3];
          for (int d = 0; d < 3; ++d) {
            f[d] = c[d] ? xi[d] : 1.0 - xi[d];
            df[d] = c[d] ? 1.0 : -1.0;
          }
          grad[a][0] = df[0] * f[1] * f[2];
          grad[a][1] = f[0] * df[1] * f[2];
          grad[a][2] = f[0] * f[1] * df[2];
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b)
            K[a * 8 + b] += 0.125 * h * (grad[a][0] * grad[b][0] + grad[a][1] * grad[b][1] + grad[a][2] * grad[b][2]);
      }
}

// Reference Q1 isotropic elasticity element matrix (E = 1, Poisson ratio nu, cube of side h):
// int B^T D B with Voigt strains (xx, yy, zz, yz, xz, xy), 2x2x2 Gauss-Legendre; dof 3a+i is
// displacement component i of corner a.
static void q1_elasticity_element(double nu, double h, double* K) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = 1.0 / (2.0 * (1.0 + nu));
  double D[6][6] = {};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D[i][j] = lam;
  for (int i = 0; i < 3; ++i) D[i][i] += 2.0 * mu;
  D[3][3] = D[4][4] = D[5][5] = mu;
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int i = 0; i < 576; ++i) K[i] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {g[qx], g[qy], g[qz]};
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          const int c[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
          double f[3], df[3];
          for (int d = 0; d < 3; ++d) {
            f[d] = c[d] ? xi[d] : 1.0 - xi[d];
            df[d] = c[d] ? 1.0 : -1.0;
          }
          const double gx = df[0] * f[1] * f[2] / h, gy = f[0] * df[1] * f[2] / h, gz = f[0] * f[1] * df[2] / h;
          B[0][3 * a + 0] = gx;
          B[1][3 * a + 1] = gy;
          B[2][3 * a + 2] = gz;
          B[3][3 * a + 1] = gz;
          B[3][3 * a + 2] = gy;
          B[4][3 * a + 0] = gz;
          B[4][3 * a + 2] = gx;
          B[5][3 * a + 0] = gy;
          B[5][3 * a + 1] = gx;
        }
        double DB[6][24];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 24; ++j) {
            double v = 0.0;
            for (int k = 0; k < 6; ++k) v += D[i][k] * B[k][j];
            DB[i][j] = v;
          }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double v = 0.0;
            for (int k = 0; k < 6; ++k) v += B[k][i] * DB[k][j];
            K[i * 24 + j] += 0.125 * h * h * h * v;
          }
      }
}

}  // namespace rmg

using namespace rmg;

void rmg_handle::drop_graphs() {
  if (graph_a) (void)hipGraphExecDestroy(graph_a);
  if (graph_b) (void)hipGraphExecDestroy(graph_b);
  graph_a = graph_b = nullptr;
  graph_b_ptr = graph_x_ptr = nullptr;
}

rmg_handle::~rmg_handle() {
  drop_graphs();
  rmg::hybrid_destroy(this);
  rmg::amg_destroy(this);
  if (gstream) (void)hipStreamDestroy(gstream);
  for (Level* L : levels) delete L;
  levels.clear();
  if (host_scalars) (void)hipHostFree(host_scalars);
}

void rmg::bind_handle(rmg_handle* h) {
  RMG_HIP(hipSetDevice(h->device));
  current_allocator() = h->alloc;
}

static void use_device(rmg_handle* h) {
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  bind_handle(h);
}

static Level& level_of(rmg_handle* h, int level) {
  RMG_REQUIRE(h->have_regions, RMG_ERR_NOT_SETUP, "regions not built");
  RMG_REQUIRE(level >= 0 && level < (int)h->levels.size(), RMG_ERR_ARG,
              "level " + std::to_string(level) + " does not exist");
  return *h->levels[level];
}

extern "C" {

void rmg_options_default(rmg_options* o) {
  if (!o) return;
  o->nlevels = 3;
  o->cheb_degree = 2;
  o->eig_ratio = 20.0;
  o->boost = 1.1;
  o->power_iters = 10;
  o->seed = 0;
  o->precision = RMG_PREC_FP64;
  o->stencil_kernel = 0;
  o->autotune = 0;
  o->use_graph = 0;
  o->autotune_cache = nullptr;
  o->smoother = 0;
  o->jacobi_omega = 0.6;
  o->symmetric = 1;
  o->batched = 1;
  o->judge_cycles = 10;
  o->hybrid = 0;
  o->cycle_gamma = 1;
  o->coarse_amg = 0;
  o->amg_coarse_size = 2000;
  o->region_table = 1;
  o->tile_planes = 0;
  o->galerkin_generic = 0;
  o->bf16_tolerance = 0.05;
  o->bf16_cycles = 10;
  o->block_diag = 0;
  o->transfer_rows = 1;
}

const char* rmg_last_error(void) { return g_last_error.c_str(); }

rmg_status rmg_create(rmg_handle** out, int device, void* stream, const rmg_allocator* alloc) {
  API_BEGIN
  RMG_REQUIRE(out != nullptr, RMG_ERR_ARG, "null output pointer");
  RMG_REQUIRE(!alloc || (alloc->alloc && alloc->free), RMG_ERR_ARG, "allocator needs both alloc and free");
  int ndev = 0;
  RMG_HIP(hipGetDeviceCount(&ndev));
  RMG_REQUIRE(device >= 0 && device < ndev, RMG_ERR_ARG, "no HIP device " + std::to_string(device));
  rmg_handle* h = new rmg_handle();
  h->device = device;
  h->stream = static_cast<hipStream_t>(stream);
  if (alloc) h->alloc = DevAlloc{alloc->alloc, alloc->free, alloc->ctx};
  rmg_options_default(&h->opt);
  try {
    bind_handle(h);
    h->scalars.alloc(sizeof(double) * kNumSlots);
    RMG_HIP(hipMemset(h->scalars.p, 0, sizeof(double) * kNumSlots));
    RMG_HIP(hipHostMalloc((void**)&h->host_scalars, sizeof(double) * kNumSlots, hipHostMallocDefault));
  } catch (...) {
    delete h;
    throw;
  }
  *out = h;
  API_END
}

rmg_status rmg_destroy(rmg_handle* h) {
  API_BEGIN
  if (!h) return RMG_OK;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  delete h;
  API_END
}

rmg_status rmg_build_regions(rmg_handle* h, int dim, int ndof, int nreg, const int32_t* extent,
                             const int32_t* origin, uint32_t mask) {
  API_BEGIN
  use_device(h);
  RMG_REQUIRE(dim == 2 || dim == 3, RMG_ERR_ARG, "dim must be 2 or 3");
  RMG_REQUIRE(ndof == 1 || (ndof == 3 && dim == 3), RMG_ERR_ARG, "ndof must be 1, or 3 with dim 3");
  RMG_REQUIRE(nreg >= 1 && extent && origin, RMG_ERR_ARG, "need nreg >= 1 and extent/origin arrays");
  RMG_REQUIRE(mask < (1u << (2 * dim)), RMG_ERR_ARG, "dirichlet mask has bits beyond 2*dim");
  h->have_regions = h->have_operator = h->have_hierarchy = false;
  hybrid_destroy(h);
  amg_destroy(h);
  h->region_kind.clear();
  h->user_pw.release();
  h->logc.release();
  if (h->pmode == RMG_P_STORED) h->pmode = RMG_P_GEOMETRIC;
  h->dim = dim;
  h->ndof = ndof;
  h->nreg = nreg;
  h->mask = mask;
  h->extent.assign(3 * (size_t)nreg, 1);
  h->origin.assign(3 * (size_t)nreg, 0);
  for (int k = 0; k < nreg; ++k)
    for (int d = 0; d < dim; ++d) {
      const int32_t e = extent[(size_t)k * dim + d], o = origin[(size_t)k * dim + d];
      RMG_REQUIRE(e >= 2 && o >= 0, RMG_ERR_SHAPE, "region extents must be >= 2 and origins >= 0");
      h->extent[3 * (size_t)k + d] = e;
      h->origin[3 * (size_t)k + d] = o;
    }
  build_level0(h);
  h->region_set.assign(nreg, false);
  Level& L = *h->levels[0];
  const size_t nb = sizeof(double) * (size_t)L.ndofs();
  h->cg_x.alloc(nb);
  h->cg_r.alloc(nb);
  h->cg_p.alloc(nb);
  h->cg_q.alloc(nb);
  h->cg_z.alloc(nb);
  h->cg_b.alloc(nb);
  h->partials.alloc(sizeof(double) * ((int64_t)L.blocks.size() + (L.ngroups + kBlock - 1) / kBlock + 16));
  h->have_regions = true;
  API_END
}

// Called once every argument of an operator-setting call has been checked, before level 0's
// operator buffers change: the hierarchy and the CG graphs recorded against the old operator stop
// being valid, so a call rejected later (non-finite values found on the device) leaves no
// hierarchy that reads half-replaced or freed buffers.
static void begin_operator_change(rmg_handle* h, Level& L) {
  h->have_hierarchy = false;
  h->have_operator = false;
  h->drop_graphs();
  L.coef_sym.release();  // the half stencils and class tables of the old operator
  L.coef_lo_sym.release();
  L.class_table.release();
  L.class_table_ok.release();
  clear_split(L);
}

rmg_status rmg_set_region_stencil(rmg_handle* h, int region, int npts, const double* coef, int on_device) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, 0);
  RMG_REQUIRE(region >= 0 && region < h->nreg, RMG_ERR_ARG, "region index out of range");
  RMG_REQUIRE(coef != nullptr, RMG_ERR_ARG, "null coefficient pointer");
  const bool ok = (h->dim == 3 && npts == 27) || (h->dim == 2 && (npts == 5 || npts == 9));
  RMG_REQUIRE(ok, RMG_ERR_ARG, "npts must be 27 in 3D and 5 or 9 in 2D");
  bool any = false;
  for (bool b : h->region_set) any = any || b;
  RMG_REQUIRE(!any || L.npts == npts, RMG_ERR_ARG, "all regions must use the same stencil size");
  begin_operator_change(h, L);
  h->region_set[region] = false;
  if (!any || L.npts != npts || !L.coef.p) {
    L.npts = npts;
    L.coef.alloc(sizeof(double) * coef_elems(L.n, L.ncoef()));
    RMG_HIP(hipMemsetAsync(L.coef.p, 0, sizeof(double) * coef_elems(L.n, L.ncoef()), h->stream));
  }
  const RegionGeo& R = L.regs[region];
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  DBuf soa;
  soa.alloc(sizeof(double) * (size_t)L.ncoef() * R.n);
  RMG_HIP(hipMemcpyAsync(soa.p, coef, sizeof(double) * (size_t)L.ncoef() * R.n, kind, h->stream));
  launch_region_stencil_io(L, region, soa.as<double>(), 1, h->stream);
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), h->stream));
  launch_mask_stencil(L, flag.as<int>(), h->stream);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "stencil has NaN or Inf entries");
  h->region_set[region] = true;
  h->logc.release();
  bool all = true;
  for (bool b : h->region_set) all = all && b;
  h->have_operator = all;
  API_END
}

// True when the region boxes are the products of per-axis slabs (a tensor-product layout).
static bool tensor_layout(const rmg_handle* h) {
  size_t combos = 1;
  std::vector<std::vector<std::pair<int, int>>> slabs(h->dim);
  for (int d = 0; d < h->dim; ++d) {
    for (int k = 0; k < h->nreg; ++k) {
      std::pair<int, int> iv{h->origin[3 * k + d], h->extent[3 * k + d]};
      bool found = false;
      for (auto& q : slabs[d]) found = found || q == iv;
      if (!found) slabs[d].push_back(iv);
    }
    // the slabs of one axis must form a chain sharing one node plane between neighbours
    std::sort(slabs[d].begin(), slabs[d].end());
    for (size_t i = 1; i < slabs[d].size(); ++i)
      if (slabs[d][i - 1].first + slabs[d][i - 1].second - 1 != slabs[d][i].first) return false;
    combos *= slabs[d].size();
  }
  // the tiling check already ran: boxes tile the domain without overlap, so a tensor layout
  // is exactly one with as many regions as slab combinations
  return combos == (size_t)h->nreg;
}

// Shared checks of the composite split (Section 4) for a stencil or CSR input.
static void check_composite_split(rmg_handle* h, int npts) {
  const bool ok = (h->dim == 3 && npts == 27) || (h->dim == 2 && (npts == 5 || npts == 9));
  RMG_REQUIRE(ok, RMG_ERR_ARG, "npts must be 27 in 3D and 5 or 9 in 2D");
  RMG_REQUIRE(h->ndof == 1, RMG_ERR_ARG, "the composite split handles scalar problems");
  RMG_REQUIRE(tensor_layout(h), RMG_ERR_SHAPE, "the composite split needs a tensor-product region layout");
}

// Region matrices from a device composite stencil [npts][ncomp].
static void split_into_regions(rmg_handle* h, Level& L, int npts, const double* src) {
  begin_operator_change(h, L);
  h->region_set.assign(h->nreg, false);
  L.npts = npts;
  L.coef.alloc(sizeof(double) * coef_elems(L.n, npts));
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), h->stream));
  launch_split_composite(L, src, flag.as<int>(), h->stream);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "composite stencil has NaN or Inf entries");
  h->region_set.assign(h->nreg, true);
  h->logc.release();
  h->have_operator = true;
}

rmg_status rmg_set_composite_stencil(rmg_handle* h, int npts, const double* coef, int on_device) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, 0);
  RMG_REQUIRE(coef != nullptr, RMG_ERR_ARG, "null coefficient pointer");
  check_composite_split(h, npts);
  DBuf tmp;
  const double* src = coef;
  if (!on_device) {
    tmp.alloc(sizeof(double) * (size_t)npts * L.ncomp);
    RMG_HIP(hipMemcpyAsync(tmp.p, coef, sizeof(double) * (size_t)npts * L.ncomp, hipMemcpyHostToDevice, h->stream));
    src = tmp.as<double>();
  }
  split_into_regions(h, L, npts, src);
  API_END
}

rmg_status rmg_set_composite_csr(rmg_handle* h, int npts, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                                 const double* values, int on_device) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, 0);
  RMG_REQUIRE(rowptr && (nnz == 0 || (colind && values)) && nnz >= 0, RMG_ERR_ARG, "null CSR array or nnz < 0");
  check_composite_split(h, npts);
  const int64_t n = L.ncomp;
  // row pointers are checked on the host before any kernel reads through them
  std::vector<int64_t> rp(n + 1);
  if (on_device) {
    RMG_HIP(hipMemcpyAsync(rp.data(), rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, h->stream));
    RMG_HIP(hipStreamSynchronize(h->stream));
  } else {
    std::copy(rowptr, rowptr + n + 1, rp.begin());
  }
  RMG_REQUIRE(rp[0] == 0 && rp[n] == nnz, RMG_ERR_ARG, "row pointers must start at 0 and end at nnz");
  for (int64_t i = 0; i < n; ++i)
    RMG_REQUIRE(rp[i + 1] >= rp[i], RMG_ERR_ARG, "row pointers must not decrease");
  DBuf drp, dci, dv, comp, flag;
  const int64_t* prp = rowptr;
  const int* pci = colind;
  const double* pv = values;
  if (!on_device) {
    drp.alloc(sizeof(int64_t) * (n + 1));
    RMG_HIP(hipMemcpyAsync(drp.p, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, h->stream));
    prp = drp.as<int64_t>();
    if (nnz > 0) {
      dci.alloc(sizeof(int32_t) * nnz);
      dv.alloc(sizeof(double) * nnz);
      RMG_HIP(hipMemcpyAsync(dci.p, colind, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, h->stream));
      RMG_HIP(hipMemcpyAsync(dv.p, values, sizeof(double) * nnz, hipMemcpyHostToDevice, h->stream));
      pci = dci.as<int>();
      pv = dv.as<double>();
    }
  }
  // the conversion reads the level's stencil size: from here on level 0 changes
  begin_operator_change(h, L);
  h->region_set.assign(h->nreg, false);
  L.npts = npts;
  comp.alloc(sizeof(double) * (size_t)npts * n);
  RMG_HIP(hipMemsetAsync(comp.p, 0, sizeof(double) * (size_t)npts * n, h->stream));
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), h->stream));
  launch_csr_to_stencil(L, prp, pci, pv, comp.as<double>(), flag.as<int>(), h->stream);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  RMG_REQUIRE(!(hflag & 4), RMG_ERR_ARG, "CSR column index out of range");
  RMG_REQUIRE(!(hflag & 2), RMG_ERR_SHAPE, "CSR entry outside the " + std::to_string(npts) + "-point neighbourhood");
  RMG_REQUIRE(!(hflag & 1), RMG_ERR_NUMERIC, "CSR values have NaN or Inf entries");
  split_into_regions(h, L, npts, comp.as<double>());
  API_END
}

rmg_status rmg_assemble_q1(rmg_handle* h, int pde, double hsize, const double* elem_coef, const double* youngs,
                           double nu) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, 0);
  RMG_REQUIRE(h->dim == 3, RMG_ERR_ARG, "Q1 assembly needs a 3D layout");
  RMG_REQUIRE(hsize > 0.0 && std::isfinite(hsize), RMG_ERR_ARG, "element size must be positive");
  RMG_REQUIRE(pde == RMG_PDE_LAPLACE || pde == RMG_PDE_DIFFUSION || pde == RMG_PDE_ELASTICITY, RMG_ERR_ARG,
              "unknown pde");
  RMG_REQUIRE((pde == RMG_PDE_ELASTICITY) == (h->ndof == 3), RMG_ERR_ARG,
              "elasticity needs ndof = 3, scalar problems ndof = 1");
  RMG_REQUIRE(pde != RMG_PDE_DIFFUSION || elem_coef != nullptr, RMG_ERR_ARG, "diffusion needs elem_coef");
  if (pde == RMG_PDE_ELASTICITY) {
    RMG_REQUIRE(youngs != nullptr, RMG_ERR_ARG, "elasticity needs Young's modulus per region");
    RMG_REQUIRE(nu > -1.0 && nu < 0.5, RMG_ERR_ARG, "Poisson ratio must lie in (-1, 0.5)");
    for (int k = 0; k < h->nreg; ++k)
      RMG_REQUIRE(youngs[k] > 0.0 && std::isfinite(youngs[k]), RMG_ERR_NUMERIC, "Young's moduli must be positive");
  }
  begin_operator_change(h, L);
  h->region_set.assign(h->nreg, false);
  L.npts = 27;
  L.coef.alloc(sizeof(double) * coef_elems(L.n, L.ncoef()));
  if (pde == RMG_PDE_ELASTICITY) {
    std::vector<double> K(576);
    q1_elasticity_element(nu, hsize, K.data());
    DBuf dK, dE;
    dK.alloc(sizeof(double) * 576);
    dE.alloc(sizeof(double) * h->nreg);
    RMG_HIP(hipMemcpyAsync(dK.p, K.data(), sizeof(double) * 576, hipMemcpyHostToDevice, h->stream));
    RMG_HIP(hipMemcpyAsync(dE.p, youngs, sizeof(double) * h->nreg, hipMemcpyHostToDevice, h->stream));
    launch_assemble_q1_elasticity(L, dK.as<double>(), dE.as<double>(), h->stream);
    RMG_HIP(hipStreamSynchronize(h->stream));
  } else {
    double K[64];
    q1_laplace_element(hsize, K);
    launch_assemble_q1_scalar(L, K, pde == RMG_PDE_DIFFUSION ? elem_coef : nullptr, h->stream);
  }
  // features of the learned interpolation: log of the element coefficients
  if (pde == RMG_PDE_DIFFUSION) {
    const int64_t nelem = (int64_t)(L.comp[0] - 1) * (L.comp[1] - 1) * (L.comp[2] - 1);
    h->logc.alloc(sizeof(float) * (size_t)nelem);
    launch_log(nelem, elem_coef, h->logc.as<float>(), h->stream);
  } else {
    h->logc.release();
  }
  launch_dirichlet_split(L, h->stream);
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), h->stream));
  launch_mask_stencil(L, flag.as<int>(), h->stream);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "assembled operator has NaN or Inf entries");
  h->region_set.assign(h->nreg, true);
  h->have_operator = true;
  API_END
}

rmg_status rmg_setup_hierarchy(rmg_handle* h, const rmg_options* opt) {
  API_BEGIN
  use_device(h);
  RMG_REQUIRE(opt != nullptr, RMG_ERR_ARG, "null options");
  RMG_REQUIRE(h->have_regions && h->have_operator, RMG_ERR_NOT_SETUP, "regions and operator must be set first");
  RMG_REQUIRE(opt->nlevels >= 2 && opt->nlevels <= 12, RMG_ERR_ARG, "nlevels must be in [2, 12]");
  RMG_REQUIRE(opt->cheb_degree >= 1 && opt->cheb_degree <= 16, RMG_ERR_ARG, "cheb_degree must be in [1, 16]");
  RMG_REQUIRE(opt->eig_ratio > 1.0 && opt->boost > 0.0, RMG_ERR_ARG, "need eig_ratio > 1 and boost > 0");
  RMG_REQUIRE(opt->power_iters >= 1, RMG_ERR_ARG, "power_iters must be >= 1");
  RMG_REQUIRE(opt->precision >= RMG_PREC_FP64 && opt->precision <= RMG_PREC_FP32_BF16_AUTO, RMG_ERR_ARG,
              "unknown precision");
  RMG_REQUIRE(opt->precision != RMG_PREC_FP32_BF16_AUTO ||
                  (std::isfinite(opt->bf16_tolerance) && opt->bf16_tolerance >= 0.0 && opt->bf16_cycles >= 1 &&
                   opt->bf16_cycles <= 1000),
              RMG_ERR_ARG, "bf16_tolerance must be finite and >= 0, bf16_cycles in [1, 1000]");
  RMG_REQUIRE(opt->precision == RMG_PREC_FP64 || h->dim == 3, RMG_ERR_ARG,
              "the low-precision V-cycle needs 27-point (3D) levels");
  RMG_REQUIRE(opt->stencil_kernel >= 0 && opt->stencil_kernel <= 3, RMG_ERR_ARG, "stencil_kernel must be 0..3");
  RMG_REQUIRE(opt->batched == 0 || opt->batched == 1, RMG_ERR_ARG, "batched must be 0 or 1");
  RMG_REQUIRE(opt->symmetric == 0 || opt->symmetric == 1, RMG_ERR_ARG, "symmetric must be 0 or 1");
  RMG_REQUIRE(opt->region_table == 0 || opt->region_table == 1, RMG_ERR_ARG, "region_table must be 0 or 1");
  RMG_REQUIRE(opt->tile_planes == 0 || opt->tile_planes == 21 || opt->tile_planes == 41, RMG_ERR_ARG,
              "tile_planes must be 0, 21 or 41");
  RMG_REQUIRE(opt->galerkin_generic == 0 || opt->galerkin_generic == 1, RMG_ERR_ARG,
              "galerkin_generic must be 0 or 1");
  RMG_REQUIRE(opt->block_diag == 0 || opt->block_diag == 1, RMG_ERR_ARG, "block_diag must be 0 or 1");
  RMG_REQUIRE(opt->transfer_rows == 0 || opt->transfer_rows == 1, RMG_ERR_ARG, "transfer_rows must be 0 or 1");
  RMG_REQUIRE(!opt->block_diag || (h->ndof == 3 && opt->smoother <= 1 && !opt->hybrid), RMG_ERR_ARG,
              "block_diag needs a 3-dof problem and the Chebyshev or Jacobi smoother");
  RMG_REQUIRE(opt->smoother >= 0 && opt->smoother <= 4, RMG_ERR_ARG,
              "smoother must be 0 (Chebyshev), 1 (Jacobi), 2 (Gauss-Seidel), 3 (forward/backward "
              "Gauss-Seidel) or 4 (symmetric Gauss-Seidel)");
  RMG_REQUIRE(opt->hybrid == 0 || opt->hybrid == 1, RMG_ERR_ARG, "hybrid must be 0 or 1");
  RMG_REQUIRE(opt->cycle_gamma == 1 || (opt->cycle_gamma == 2 && opt->hybrid == 1), RMG_ERR_ARG,
              "cycle_gamma must be 1, or 2 with the hybrid hierarchy");
  RMG_REQUIRE(!opt->hybrid || opt->smoother == 1 || opt->smoother == 2 || opt->smoother == 4, RMG_ERR_ARG,
              "the hybrid hierarchy smooths with Jacobi (1), Gauss-Seidel (2) or symmetric Gauss-Seidel (4)");
  RMG_REQUIRE(!opt->hybrid || opt->precision == RMG_PREC_FP64, RMG_ERR_ARG, "the hybrid hierarchy runs in FP64");
  RMG_REQUIRE(!opt->hybrid || h->pmode == RMG_P_GEOMETRIC, RMG_ERR_ARG,
              "the hybrid hierarchy builds its own transfers (no stored or learned interpolation)");
  RMG_REQUIRE(opt->smoother < 2 || opt->precision == RMG_PREC_FP64, RMG_ERR_ARG,
              "the Gauss-Seidel smoothers run in FP64 only");
  RMG_REQUIRE(opt->smoother == 0 || (opt->jacobi_omega > 0.0 && opt->jacobi_omega < 2.0), RMG_ERR_ARG,
              "jacobi_omega must lie in (0, 2)");
  RMG_REQUIRE(opt->judge_cycles >= 0 && opt->judge_cycles <= 1000, RMG_ERR_ARG, "judge_cycles must be in [0, 1000]");
  RMG_REQUIRE(opt->coarse_amg == 0 || opt->coarse_amg == 1, RMG_ERR_ARG, "coarse_amg must be 0 or 1");
  RMG_REQUIRE(!opt->coarse_amg || (opt->amg_coarse_size >= 1 && opt->amg_coarse_size <= 20000), RMG_ERR_ARG,
              "amg_coarse_size must be in [1, 20000]");
  RMG_REQUIRE(!opt->coarse_amg || !opt->hybrid, RMG_ERR_ARG,
              "the AMG coarse solver belongs to the geometric region hierarchy (not the hybrid one)");
  RMG_REQUIRE(!opt->coarse_amg || h->ndof == 1 || (h->ndof == 3 && h->dim == 3), RMG_ERR_ARG,
              "the AMG coarse solver handles scalar problems and 3D elasticity");
  h->opt = *opt;
  h->autotune_cache = opt->autotune_cache ? std::string(opt->autotune_cache) : std::string();
  h->opt.autotune_cache = nullptr;  // the caller's string is borrowed for this call only
  h->have_hierarchy = false;
  h->drop_graphs();
  const auto t0 = std::chrono::steady_clock::now();
  setup_hierarchy(h);
  RMG_HIP(hipStreamSynchronize(h->stream));
  h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  h->have_hierarchy = true;
  API_END
}

static void require_hierarchy(rmg_handle* h) {
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
}

rmg_status rmg_apply_vcycle(rmg_handle* h, const double* r, double* z, int layout) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(r && z && r != z, RMG_ERR_ARG, "r and z must be distinct non-null device pointers");
  RMG_REQUIRE(layout == RMG_LAYOUT_COMPOSITE || layout == RMG_LAYOUT_REGIONAL, RMG_ERR_ARG, "bad layout");
  Level& L = *h->levels[0];
  if (layout == RMG_LAYOUT_REGIONAL) {
    apply_preconditioner(h, r, z);
  } else {
    launch_to_regional(L, r, h->cg_b.as<double>(), h->stream);
    apply_preconditioner(h, h->cg_b.as<double>(), h->cg_z.as<double>());
    launch_to_composite(L, h->cg_z.as<double>(), z, 0, h->stream);
  }
  API_END
}

rmg_status rmg_solve(rmg_handle* h, const double* b, double* x, int layout, double rtol, int maxit,
                     rmg_solve_info* info) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(b && x && b != x, RMG_ERR_ARG, "b and x must be distinct non-null device pointers");
  RMG_REQUIRE(layout == RMG_LAYOUT_COMPOSITE || layout == RMG_LAYOUT_REGIONAL, RMG_ERR_ARG, "bad layout");
  RMG_REQUIRE(rtol > 0.0 && maxit >= 1, RMG_ERR_ARG, "need rtol > 0 and maxit >= 1");
  Level& L = *h->levels[0];
  rmg_status st = RMG_OK;
  if (layout == RMG_LAYOUT_REGIONAL) {
    pcg(h, b, x, rtol, maxit, info, &st);
  } else {
    launch_to_regional(L, b, h->cg_b.as<double>(), h->stream);
    launch_to_regional(L, x, h->cg_x.as<double>(), h->stream);
    pcg(h, h->cg_b.as<double>(), h->cg_x.as<double>(), rtol, maxit, info, &st);
    launch_to_composite(L, h->cg_x.as<double>(), x, 0, h->stream);
  }
  RMG_HIP(hipStreamSynchronize(h->stream));
  if (st != RMG_OK) return st;
  API_END
}

rmg_status rmg_mg_solve(rmg_handle* h, const double* b, double* x, int layout, double rtol, int maxit,
                        rmg_solve_info* info) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(b && x && b != x, RMG_ERR_ARG, "b and x must be distinct non-null device pointers");
  RMG_REQUIRE(layout == RMG_LAYOUT_COMPOSITE || layout == RMG_LAYOUT_REGIONAL, RMG_ERR_ARG, "bad layout");
  RMG_REQUIRE(rtol > 0.0 && maxit >= 1, RMG_ERR_ARG, "need rtol > 0 and maxit >= 1");
  Level& L = *h->levels[0];
  rmg_status st = RMG_OK;
  if (layout == RMG_LAYOUT_REGIONAL) {
    mg_solve(h, b, x, rtol, maxit, info, &st);
  } else {
    launch_to_regional(L, b, h->cg_b.as<double>(), h->stream);
    launch_to_regional(L, x, h->cg_x.as<double>(), h->stream);
    mg_solve(h, h->cg_b.as<double>(), h->cg_x.as<double>(), rtol, maxit, info, &st);
    launch_to_composite(L, h->cg_x.as<double>(), x, 0, h->stream);
  }
  RMG_HIP(hipStreamSynchronize(h->stream));
  if (st != RMG_OK) return st;
  API_END
}

rmg_status rmg_to_regional(rmg_handle* h, int level, const double* comp, double* reg) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  RMG_REQUIRE(comp && reg, RMG_ERR_ARG, "null pointer");
  launch_to_regional(L, comp, reg, h->stream);
  API_END
}

rmg_status rmg_to_composite(rmg_handle* h, int level, const double* reg, double* comp, int average) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  RMG_REQUIRE(comp && reg, RMG_ERR_ARG, "null pointer");
  launch_to_composite(L, reg, comp, average ? 1 : 0, h->stream);
  API_END
}

rmg_status rmg_regional_matvec(rmg_handle* h, int level, const double* v, double* z) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  RMG_REQUIRE(v && z && v != z, RMG_ERR_ARG, "v and z must be distinct non-null device pointers");
  RMG_REQUIRE(L.coef.p != nullptr && (level > 0 || h->have_operator), RMG_ERR_NOT_SETUP, "operator not set");
  StencilArgs a;
  a.op = StencilOp::Matvec;
  a.x = v;
  a.out = z;
  launch_stencil_op(L, a, h->stream);
  API_END
}

rmg_status rmg_interface_sum(rmg_handle* h, int level, const double* v, double* w) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  RMG_REQUIRE(v && w, RMG_ERR_ARG, "null pointer");
  launch_interface_sum(L, v, w, h->stream);
  API_END
}

rmg_status rmg_restrict(rmg_handle* h, int level, const double* r, double* w) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(level >= 0 && level + 1 < (int)h->levels.size(), RMG_ERR_ARG, "no coarser level");
  RMG_REQUIRE(r && w && r != w, RMG_ERR_ARG, "r and w must be distinct non-null device pointers");
  Level& F = *h->levels[level];
  Level& C = *h->levels[level + 1];
  {
    // r / mult on shared nodes: the ResidualScaled update with b = r and a zero product
    launch_zero(F.ndofs(), F.u2.as<double>(), h->stream);
    StencilArgs a;
    a.op = StencilOp::ResidualScaled;
    a.x = F.u2.as<double>();
    a.out = F.r.as<double>();
    a.b = r;
    launch_stencil_op(F, a, h->stream);
  }
  launch_restrict(F, C, false, F.r.as<double>(), w, h->stream);
  API_END
}

rmg_status rmg_prolongate_add(rmg_handle* h, int level, const double* ubar, double* u) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(level >= 0 && level + 1 < (int)h->levels.size(), RMG_ERR_ARG, "no coarser level");
  RMG_REQUIRE(ubar && u, RMG_ERR_ARG, "null pointer");
  launch_prolong_add(*h->levels[level], *h->levels[level + 1], false, ubar, u, h->stream);
  API_END
}

rmg_status rmg_smooth(rmg_handle* h, int level, const double* b, double* u) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(level >= 0 && level + 1 < (int)h->levels.size(), RMG_ERR_ARG, "the coarsest level has no smoother");
  RMG_REQUIRE(b && u && b != u, RMG_ERR_ARG, "b and u must be distinct non-null device pointers");
  smooth_zero_guess(h, level, b, u);
  API_END
}

rmg_status rmg_level_info(rmg_handle* h, int level, int64_t* n_regional, int64_t* n_composite, int* npts,
                          double* lambda_max) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  if (n_regional) *n_regional = L.n * h->ndof;
  if (n_composite) *n_composite = L.ncomp * h->ndof;
  if (npts) *npts = L.npts;
  if (lambda_max) *lambda_max = L.lambda;
  API_END
}

rmg_status rmg_level_kernel(rmg_handle* h, int level, int* kernel, int* coefs, int* coefs_lo) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  const bool tiled = L.use_tiles && L.ndof == 1 && L.npts == 27;
  if (kernel) *kernel = L.per_region ? 3 : (!tiled ? 0 : (L.tile_grid > 0 && L.tile_grid < (int)L.tiles.size() ? 2 : 1));
  const int nb = L.ndof * L.ndof;
  if (coefs) *coefs = L.coef_sym.p ? kSymPts * nb : L.ncoef();
  // the 2.5D kernel has no half-stencil path for BF16 storage
  const bool sym_lo = L.coef_lo_sym.p && !(tiled && L.ct_lo == kCoefBF16);
  if (coefs_lo) *coefs_lo = L.ct_lo == kCoefF64 ? 0 : (sym_lo ? kSymPts * nb : L.ncoef());
  API_END
}

rmg_status rmg_level_precision(rmg_handle* h, int level, int* coef_type, double* rho_fp32, double* rho_bf16) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  if (coef_type) *coef_type = L.ct_lo == kCoefF64 ? 0 : (L.ct_lo == kCoefF32 ? 1 : 2);
  if (rho_fp32) *rho_fp32 = L.rho_fp32;
  if (rho_bf16) *rho_bf16 = L.rho_bf16;
  API_END
}

rmg_status rmg_kernel_launches(int64_t* count) {
  API_BEGIN
  RMG_REQUIRE(count != nullptr, RMG_ERR_ARG, "null output");
  *count = g_kernel_launches.load(std::memory_order_relaxed);
  API_END
}

rmg_status rmg_level_tiles(rmg_handle* h, int level, int* ntiles, int* threads, int* planes) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  const bool tiled = L.use_tiles && L.ndof == 1 && L.npts == 27 && !L.per_region;
  if (ntiles) *ntiles = tiled ? (int)L.tiles.size() : 0;
  if (threads) *threads = tiled ? L.tile_threads : 0;
  if (planes) *planes = tiled ? L.tile_depth : 0;
  API_END
}

rmg_status rmg_level_transfer_tiles(rmg_handle* h, int level, int* restriction_tiles, int* prolongation_tiles) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  if (restriction_tiles) *restriction_tiles = (int)L.rtiles.size();
  if (prolongation_tiles) *prolongation_tiles = (int)L.ptiles.size();
  API_END
}

rmg_status rmg_level_table_regions(rmg_handle* h, int level, int* nregions) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  const DBuf& ok = L.class_table_ok;
  int count = 0;
  if (ok.p) {
    std::vector<int> flags(L.nreg);
    RMG_HIP(hipStreamSynchronize(h->stream));
    RMG_HIP(hipMemcpy(flags.data(), ok.p, sizeof(int) * L.nreg, hipMemcpyDeviceToHost));
    for (int f : flags) count += f != 0;
  }
  if (nregions) *nregions = count;
  API_END
}

rmg_status rmg_get_level_stencil(rmg_handle* h, int level, int region, double* host_out) {
  API_BEGIN
  use_device(h);
  Level& L = level_of(h, level);
  RMG_REQUIRE(region >= 0 && region < L.nreg && host_out, RMG_ERR_ARG, "bad region or null output");
  RMG_REQUIRE(L.coef.p != nullptr, RMG_ERR_NOT_SETUP, "no operator on this level");
  const RegionGeo& R = L.regs[region];
  DBuf soa;
  soa.alloc(sizeof(double) * (size_t)L.ncoef() * R.n);
  launch_region_stencil_io(L, region, soa.as<double>(), 0, h->stream);
  RMG_HIP(hipMemcpyAsync(host_out, soa.p, sizeof(double) * (size_t)L.ncoef() * R.n, hipMemcpyDeviceToHost,
                         h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  API_END
}

rmg_status rmg_get_coarse_matrix(rmg_handle* h, double* host_out) {
  API_BEGIN
  use_device(h);
  require_hierarchy(h);
  RMG_REQUIRE(host_out, RMG_ERR_ARG, "null output");
  Level& L = *h->levels.back();
  RMG_REQUIRE(!L.abar_host.empty(), RMG_ERR_NOT_SETUP, "no dense coarse matrix (the AMG coarse solver is in use)");
  std::memcpy(host_out, L.abar_host.data(), sizeof(double) * L.abar_host.size());
  API_END
}

rmg_status rmg_profile(rmg_handle* h, int enable) {
  API_BEGIN
  use_device(h);
  RMG_HIP(hipStreamSynchronize(h->stream));
  h->profiling = enable != 0;
  for (auto& t : h->timers) t.reset();
  API_END
}

rmg_status rmg_tune_report(rmg_handle* h, char* buf, int cap) {
  API_BEGIN
  RMG_REQUIRE(h && buf && cap > 0, RMG_ERR_ARG, "null handle or buffer");
  std::string all;
  for (const std::string& line : h->tune_report) all += line + "\n";
  const size_t n = std::min(all.size(), (size_t)cap - 1);
  std::memcpy(buf, all.data(), n);
  buf[n] = 0;
  API_END
}

rmg_status rmg_profile_query(rmg_handle* h, int kernel, int64_t* launches, double* total_ms) {
  API_BEGIN
  use_device(h);
  RMG_REQUIRE(kernel >= 0 && kernel < kNumTimed, RMG_ERR_ARG, "unknown timed kernel id");
  RMG_HIP(hipStreamSynchronize(h->stream));
  h->timers[kernel].harvest();
  if (launches) *launches = h->timers[kernel].count;
  if (total_ms) *total_ms = h->timers[kernel].total_ms;
  API_END
}

}  // extern "C"
