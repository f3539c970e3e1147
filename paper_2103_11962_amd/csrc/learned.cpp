// Host side of the stored and learned interpolation: weights for the finest level at setup and
// their validation, the MLP trainer (data, full-batch loss and gradient, Adam) and the entry
// points of both.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "kernels.h"
#include "mlp.h"

using namespace rmg;

struct rmg_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  DBuf theta, grad, m, v;  // float [kMlpParams]
  int t = 0;               // Adam steps taken since the parameters were set
  int loss_kind = 0;       // RMG_MLP_LOSS_*
  bool have_grad = false;
  int64_t n = 0, cap = 0;  // pairs held and capacity
  DBuf X, E;               // float [cap][27], [cap][64]
  int64_t wcap = 0;        // pairs the work arrays are sized for
  DBuf Z, A1, A2, dZ, D1, D2, partials, part, losses;
  int64_t loss_cap = 0;
};

namespace rmg {

// Coarse cells of a level, region by region (x fastest inside a region).
struct Cells {
  std::vector<int64_t> off;  // [nreg + 1]
  int64_t n = 0;
};

static Cells cells_of(const Level& L) {
  Cells c;
  c.off.assign(L.nreg + 1, 0);
  for (int k = 0; k < L.nreg; ++k) {
    const RegionGeo& R = L.regs[k];
    RMG_REQUIRE((R.ex - 1) % 3 == 0 && (R.ey - 1) % 3 == 0 && (R.ez - 1) % 3 == 0, RMG_ERR_SHAPE,
                "region extents must be 3 m + 1 for coarse cells");
    c.off[k + 1] = c.off[k] + (int64_t)((R.ex - 1) / 3) * ((R.ey - 1) / 3) * ((R.ez - 1) / 3);
  }
  c.n = c.off[L.nreg];
  return c;
}

// Setup upload of a host table; waits for the copy, so the table may die on return.
static void upload(DBuf& d, const void* host, size_t bytes, hipStream_t st) {
  d.alloc(bytes);
  RMG_HIP(hipMemcpyAsync(d.p, host, bytes, hipMemcpyHostToDevice, st));
  RMG_HIP(hipStreamSynchronize(st));
}

int validate_weights(rmg_handle* h, const Level& F, const Level& C) {
  DBuf flag;
  flag.alloc(sizeof(int));
  RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), h->stream));
  check_weights(F, C, F.pw.as<double>(), flag.as<int>(), h->stream);
  int hflag = 0;
  RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  return hflag;
}

// Learned weights: MLP logits for every coarse cell, then the per-node averaging kernel.
static void learned_weights_of(rmg_handle* h, Level& F, const Level& C) {
  hipStream_t st = h->stream;
  const Cells cells = cells_of(F);
  const int ncx = (F.comp[0] - 1) / 3, ncy = (F.comp[1] - 1) / 3, ncz = (F.comp[2] - 1) / 3;
  const int64_t ncomp_cells = (int64_t)ncx * ncy * ncz;
  RMG_REQUIRE(ncomp_cells == cells.n, RMG_ERR_SHAPE, "regions do not tile the coarse cells");
  RMG_REQUIRE(cells.n < (int64_t)1 << 31, RMG_ERR_ARG, "too many coarse cells");
  std::vector<int> cellrow(ncomp_cells, -1);
  for (int k = 0; k < F.nreg; ++k) {
    const RegionGeo& R = F.regs[k];
    const int nx = (R.ex - 1) / 3, ny = (R.ey - 1) / 3, nz = (R.ez - 1) / 3;
    int64_t row = cells.off[k];
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x, ++row) {
          const int64_t ci = ((int64_t)(R.oz / 3 + z) * ncy + (R.oy / 3 + y)) * ncx + (R.ox / 3 + x);
          RMG_REQUIRE(cellrow[ci] < 0, RMG_ERR_SHAPE, "coarse cell covered by two regions");
          cellrow[ci] = (int)row;
        }
  }
  const int64_t nelem = (int64_t)(F.comp[0] - 1) * (F.comp[1] - 1) * (F.comp[2] - 1);
  RMG_REQUIRE(!h->logc.p || h->logc.bytes == sizeof(float) * (size_t)nelem, RMG_ERR_ARG,
              "element coefficients do not match the finest level");
  RMG_REQUIRE((int)h->mlp_theta.size() == kMlpParams, RMG_ERR_ARG, "learned interpolation has no parameters");
  DBuf d_off, d_row, d_theta, X, Z;
  upload(d_off, cells.off.data(), sizeof(int64_t) * cells.off.size(), st);
  upload(d_row, cellrow.data(), sizeof(int) * cellrow.size(), st);
  upload(d_theta, h->mlp_theta.data(), sizeof(float) * kMlpParams, st);
  X.alloc(sizeof(float) * kMlpIn * (size_t)cells.n);
  Z.alloc(sizeof(float) * kMlpOut * (size_t)cells.n);
  cell_features(F, d_off.as<int64_t>(), cells.n, h->logc.as<float>(), X.as<float>(), st);
  mlp_forward(cells.n, X.as<float>(), d_theta.as<float>(), Z.as<float>(), nullptr, nullptr, st);
  learned_weights(F, C, Z.as<float>(), d_row.as<int>(), F.pw.as<double>(), st);
  RMG_HIP(hipStreamSynchronize(st));  // before the temporaries are freed
}

// Coarse-major restriction copy of valid stored weights.
static void build_restriction_weights(rmg_handle* h, Level& F, const Level& C) {
  F.rw.alloc(sizeof(double) * coef_elems(C.n, 125));
  launch_build_rw(F, C, F.rw.as<double>(), h->stream);
}

int prepare_stored_weights(rmg_handle* h, Level& F, const Level& C) {
  const size_t bytes = sizeof(double) * 8 * (size_t)F.n;
  F.pw.alloc(bytes);
  F.rw.release();
  if (h->pmode == RMG_P_STORED) {
    RMG_REQUIRE(h->user_pw.bytes == bytes, RMG_ERR_ARG, "stored interpolation weights do not match the finest level");
    RMG_HIP(hipMemcpyAsync(F.pw.p, h->user_pw.p, bytes, hipMemcpyDeviceToDevice, h->stream));
    const int flags = validate_weights(h, F, C);
    if (flags) {
      F.pw.release();
      fail(RMG_ERR_ARG, "stored interpolation weights are invalid (flags " + std::to_string(flags) + ")");
    }
    build_restriction_weights(h, F, C);
    return 0;
  }
  learned_weights_of(h, F, C);
  const int flags = validate_weights(h, F, C);
  if (flags) F.pw.release();  // fall back to the geometric interpolation
  else build_restriction_weights(h, F, C);
  return flags;
}

}  // namespace rmg

// ------------------------------------------------------------------ trainer
static void mlp_use(rmg_mlp* m) {
  RMG_REQUIRE(m != nullptr, RMG_ERR_ARG, "null trainer");
  RMG_HIP(hipSetDevice(m->device));
}

static void reserve_data(rmg_mlp* m, int64_t need) {
  if (need <= m->cap) return;
  const int64_t cap = std::max(need, m->cap + m->cap / 2);
  DBuf X, E;
  X.alloc(sizeof(float) * kMlpIn * (size_t)cap);
  E.alloc(sizeof(float) * 64 * (size_t)cap);
  if (m->n) {
    RMG_HIP(hipMemcpyAsync(X.p, m->X.p, sizeof(float) * kMlpIn * m->n, hipMemcpyDeviceToDevice, m->stream));
    RMG_HIP(hipMemcpyAsync(E.p, m->E.p, sizeof(float) * 64 * m->n, hipMemcpyDeviceToDevice, m->stream));
    RMG_HIP(hipStreamSynchronize(m->stream));
  }
  m->X.swap(X);
  m->E.swap(E);
  m->cap = cap;
}

static void reserve_work(rmg_mlp* m, int64_t n, int64_t nloss) {
  if (n > m->wcap) {
    m->Z.alloc(sizeof(float) * kMlpOut * (size_t)n);
    m->dZ.alloc(sizeof(float) * kMlpOut * (size_t)n);
    m->A1.alloc(sizeof(float) * kMlpH * (size_t)n);
    m->A2.alloc(sizeof(float) * kMlpH * (size_t)n);
    m->D1.alloc(sizeof(float) * kMlpH * (size_t)n);
    m->D2.alloc(sizeof(float) * kMlpH * (size_t)n);
    m->partials.alloc(sizeof(double) * (size_t)mlp_loss_partials(n));
    if (!m->part.p) m->part.alloc(sizeof(float) * (size_t)mlp_grad_partials());
    m->wcap = n;
  }
  if (nloss > m->loss_cap) {
    m->losses.alloc(sizeof(double) * (size_t)nloss);
    m->loss_cap = nloss;
  }
}

// Full-batch loss (into losses[slot]) and gradient (into grad) at the current parameters.
static void loss_grad(rmg_mlp* m, int slot) {
  const int64_t n = m->n;
  hipStream_t st = m->stream;
  const float* X = m->X.as<float>();
  float* Z = m->Z.as<float>();
  float* A1 = m->A1.as<float>();
  float* A2 = m->A2.as<float>();
  float* dZ = m->dZ.as<float>();
  float* D1 = m->D1.as<float>();
  float* D2 = m->D2.as<float>();
  mlp_forward(n, X, m->theta.as<float>(), Z, A1, A2, st);
  const int64_t np = mlp_loss(n, Z, m->E.as<float>(), X, m->loss_kind, dZ, m->partials.as<double>(), st);
  launch_reduce(m->partials.as<double>(), np, m->losses.as<double>(), slot, st);
  mlp_backact(n, dZ, A1, A2, m->theta.as<float>(), D1, D2, st);
  mlp_weight_grads(n, X, A1, A2, dZ, D1, D2, m->grad.as<float>(), m->part.as<float>(), st);
  m->have_grad = true;
}

static void adam(rmg_mlp* m, double lr) {
  ++m->t;
  mlp_adam(m->theta.as<float>(), m->grad.as<float>(), m->m.as<float>(), m->v.as<float>(), m->t, lr, m->stream);
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) on a counter; uniform in [-1, 1).
static double counter_uniform(uint64_t ctr) {
  uint64_t z = ctr + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return 2.0 * (double)(z >> 11) * 0x1p-53 - 1.0;
}

// Initial parameters: He-uniform hidden weights, output weights scaled by out_scale, zero hidden
// biases, and output biases equal to the log of the geometric (trilinear) weights, so that with
// small output weights every node starts at the geometric interpolation.
static void init_params(uint64_t seed, double out_scale, float* th) {
  constexpr uint64_t kStream = 96;  // counter stream of the initial parameters
  const uint64_t base = (kStream << 40) + (seed << 48);
  int o = 0;
  const int rows[3] = {kMlpH, kMlpH, kMlpOut}, cols[3] = {kMlpIn, kMlpH, kMlpH};
  for (int layer = 0; layer < 3; ++layer) {
    const double a = (layer == 2 ? out_scale : 1.0) * std::sqrt(6.0 / cols[layer]);
    for (int i = 0; i < rows[layer] * cols[layer]; ++i, ++o) th[o] = (float)(a * counter_uniform(base + o));
    if (layer < 2)
      for (int i = 0; i < rows[layer]; ++i) th[o++] = 0.0f;
  }
  CellNode nodes[56];
  signed char pos2node[64];
  cell_node_table(nodes, pos2node);
  for (const CellNode& nd : nodes) {
    const int p[3] = {nd.pos % 4, (nd.pos / 4) % 4, nd.pos / 16};
    for (int c = 0; c < nd.ncorner; ++c) {
      double w = 1.0;
      for (int d = 0; d < 3; ++d) {
        const int b = (nd.corner[c] >> d) & 1;
        w *= b ? p[d] / 3.0 : (3 - p[d]) / 3.0;
      }
      th[o + nd.first + c] = (float)std::log(w);
    }
  }
}

extern "C" {

rmg_status rmg_set_prolongator_weights(rmg_handle* h, const double* w, int on_device) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  bind_handle(h);
  if (!w) {
    h->user_pw.release();
    h->pmode = RMG_P_GEOMETRIC;
    return RMG_OK;
  }
  RMG_REQUIRE(h->have_regions, RMG_ERR_NOT_SETUP, "regions not built");
  RMG_REQUIRE(h->dim == 3 && h->ndof == 1, RMG_ERR_ARG, "stored interpolation weights need a scalar 3D problem");
  const Level& L = *h->levels[0];
  const size_t bytes = sizeof(double) * 8 * (size_t)L.n;
  h->user_pw.alloc(bytes);
  RMG_HIP(hipMemcpyAsync(h->user_pw.p, w, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  h->pmode = RMG_P_STORED;
  API_END
}

rmg_status rmg_set_learned_prolongator(rmg_handle* h, const float* theta) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  if (!theta) {
    h->mlp_theta.clear();
    h->pmode = RMG_P_GEOMETRIC;
    return RMG_OK;
  }
  h->mlp_theta.assign(theta, theta + kMlpParams);
  h->pmode = RMG_P_LEARNED;
  API_END
}

rmg_status rmg_prolongator_info(rmg_handle* h, int* kind, int* flags, double* rho_learned, double* rho_geometric) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr, RMG_ERR_ARG, "null handle");
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
  if (kind) *kind = h->p_used;
  if (flags) *flags = h->p_flags;
  if (rho_learned) *rho_learned = h->rho_learned;
  if (rho_geometric) *rho_geometric = h->rho_geometric;
  API_END
}

rmg_status rmg_get_prolongator_weights(rmg_handle* h, double* host_out) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && host_out != nullptr, RMG_ERR_ARG, "null handle or output");
  bind_handle(h);
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
  const Level& L = *h->levels[0];
  RMG_REQUIRE(L.pw.p != nullptr, RMG_ERR_ARG, "the hierarchy interpolates geometrically");
  RMG_HIP(hipMemcpyAsync(host_out, L.pw.p, L.pw.bytes, hipMemcpyDeviceToHost, h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
  API_END
}

rmg_status rmg_convergence_factor(rmg_handle* h, int cycles, double* rho) {
  API_BEGIN
  RMG_REQUIRE(h != nullptr && rho != nullptr, RMG_ERR_ARG, "null handle or output");
  bind_handle(h);
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
  RMG_REQUIRE(cycles >= 1 && cycles <= 10000, RMG_ERR_ARG, "cycles must be in [1, 10000]");
  *rho = convergence_factor(h, cycles);
  API_END
}

rmg_status rmg_mlp_create(rmg_mlp** out, int device, void* stream) {
  API_BEGIN
  RMG_REQUIRE(out != nullptr, RMG_ERR_ARG, "null output pointer");
  int ndev = 0;
  RMG_HIP(hipGetDeviceCount(&ndev));
  RMG_REQUIRE(device >= 0 && device < ndev, RMG_ERR_ARG, "no HIP device " + std::to_string(device));
  RMG_HIP(hipSetDevice(device));
  rmg_mlp* m = new rmg_mlp();
  m->device = device;
  m->stream = static_cast<hipStream_t>(stream);
  try {
    for (DBuf* b : {&m->theta, &m->grad, &m->m, &m->v}) {
      b->alloc(sizeof(float) * kMlpParams);
      RMG_HIP(hipMemsetAsync(b->p, 0, sizeof(float) * kMlpParams, m->stream));
    }
    RMG_HIP(hipStreamSynchronize(m->stream));
  } catch (...) {
    delete m;
    throw;
  }
  *out = m;
  API_END
}

rmg_status rmg_mlp_destroy(rmg_mlp* m) {
  API_BEGIN
  if (!m) return RMG_OK;
  (void)hipSetDevice(m->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  delete m;
  API_END
}

rmg_status rmg_mlp_set_params(rmg_mlp* m, const float* theta) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(theta != nullptr, RMG_ERR_ARG, "null parameters");
  RMG_HIP(hipMemcpyAsync(m->theta.p, theta, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->stream));
  RMG_HIP(hipMemsetAsync(m->m.p, 0, sizeof(float) * kMlpParams, m->stream));
  RMG_HIP(hipMemsetAsync(m->v.p, 0, sizeof(float) * kMlpParams, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  m->t = 0;
  m->have_grad = false;
  API_END
}

rmg_status rmg_mlp_init_params(rmg_mlp* m, uint64_t seed, double out_scale, float* theta_out) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(out_scale >= 0.0 && std::isfinite(out_scale), RMG_ERR_ARG, "out_scale must be finite and >= 0");
  RMG_REQUIRE(seed < (1ull << 16), RMG_ERR_ARG, "seed must be below 2^16");
  std::vector<float> th(kMlpParams);
  init_params(seed, out_scale, th.data());
  const rmg_status st = rmg_mlp_set_params(m, th.data());
  if (st != RMG_OK) return st;
  if (theta_out) std::copy(th.begin(), th.end(), theta_out);
  API_END
}

rmg_status rmg_mlp_set_loss(rmg_mlp* m, int kind) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(kind == RMG_MLP_LOSS_L2 || kind == RMG_MLP_LOSS_ENERGY, RMG_ERR_ARG, "unknown loss");
  m->loss_kind = kind;
  m->have_grad = false;
  API_END
}

rmg_status rmg_mlp_get_params(rmg_mlp* m, float* theta) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(theta != nullptr, RMG_ERR_ARG, "null output");
  RMG_HIP(hipMemcpyAsync(theta, m->theta.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  API_END
}

rmg_status rmg_mlp_add_data(rmg_mlp* m, int64_t n, const float* X, const float* E, int on_device) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(n >= 0 && (n == 0 || (X && E)), RMG_ERR_ARG, "need n >= 0 and X, E");
  if (n == 0) return RMG_OK;
  reserve_data(m, m->n + n);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  RMG_HIP(hipMemcpyAsync(m->X.as<float>() + m->n * kMlpIn, X, sizeof(float) * kMlpIn * n, kind, m->stream));
  RMG_HIP(hipMemcpyAsync(m->E.as<float>() + m->n * 64, E, sizeof(float) * 64 * n, kind, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  m->n += n;
  API_END
}

rmg_status rmg_mlp_add_samples(rmg_mlp* m, rmg_handle* h, int nsamples, uint64_t seed, int sweeps) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(h != nullptr && h->device == m->device, RMG_ERR_ARG, "handle on another device");
  RMG_REQUIRE(h->have_hierarchy, RMG_ERR_NOT_SETUP, "hierarchy not set up");
  RMG_REQUIRE(h->dim == 3 && h->ndof == 1, RMG_ERR_ARG, "training samples need a scalar 3D problem");
  RMG_REQUIRE(nsamples >= 1 && nsamples <= (1 << 20), RMG_ERR_ARG, "nsamples must be in [1, 2^20]");
  RMG_REQUIRE(sweeps >= 0 && sweeps <= 100000, RMG_ERR_ARG, "sweeps must be in [0, 100000]");
  RMG_REQUIRE(32 + (int64_t)nsamples < (1 << 24), RMG_ERR_ARG, "too many samples for the counter streams");
  Level& L = *h->levels[0];
  const Cells cells = cells_of(L);
  const int64_t total = (int64_t)nsamples * cells.n;
  RMG_HIP(hipStreamSynchronize(m->stream));
  reserve_data(m, m->n + total);
  hipStream_t st = h->stream;
  DBuf d_off, e, tmp, zero;
  upload(d_off, cells.off.data(), sizeof(int64_t) * cells.off.size(), st);
  e.alloc(sizeof(double) * (size_t)L.n);
  tmp.alloc(sizeof(double) * (size_t)L.n);
  zero.alloc(sizeof(double) * (size_t)L.n);
  launch_zero(L.n, zero.as<double>(), st);
  float* X0 = m->X.as<float>() + m->n * kMlpIn;
  cell_features(L, d_off.as<int64_t>(), cells.n, h->logc.as<float>(), X0, st);
  for (int s = 0; s < nsamples; ++s) {
    const int64_t row = m->n + (int64_t)s * cells.n;
    if (s > 0)
      RMG_HIP(hipMemcpyAsync(m->X.as<float>() + row * kMlpIn, X0, sizeof(float) * kMlpIn * cells.n,
                             hipMemcpyDeviceToDevice, st));
    launch_start_vector(L, 32 + s, seed, e.as<double>(), st);
    for (int k = 0; k < sweeps; ++k) smooth_iterate(h, 0, zero.as<double>(), e.as<double>(), tmp.as<double>());
    cell_targets(L, d_off.as<int64_t>(), cells.n, e.as<double>(), m->E.as<float>() + row * 64, st);
  }
  RMG_HIP(hipStreamSynchronize(st));
  m->n += total;
  API_END
}

rmg_status rmg_mlp_clear_data(rmg_mlp* m) {
  API_BEGIN
  mlp_use(m);
  m->n = 0;
  m->have_grad = false;
  API_END
}

rmg_status rmg_mlp_num_data(rmg_mlp* m, int64_t* n) {
  API_BEGIN
  RMG_REQUIRE(m != nullptr && n != nullptr, RMG_ERR_ARG, "null trainer or output");
  *n = m->n;
  API_END
}

rmg_status rmg_mlp_get_data(rmg_mlp* m, int64_t first, int64_t count, float* X, float* E) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(first >= 0 && count >= 0 && first + count <= m->n, RMG_ERR_ARG, "range outside the data");
  if (X)
    RMG_HIP(hipMemcpyAsync(X, m->X.as<float>() + first * kMlpIn, sizeof(float) * kMlpIn * count,
                           hipMemcpyDeviceToHost, m->stream));
  if (E)
    RMG_HIP(hipMemcpyAsync(E, m->E.as<float>() + first * 64, sizeof(float) * 64 * count, hipMemcpyDeviceToHost,
                           m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  API_END
}

rmg_status rmg_mlp_forward(rmg_mlp* m, int64_t n, const float* X, float* Z, int on_device) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(n >= 0 && (n == 0 || (X && Z)), RMG_ERR_ARG, "need n >= 0 and X, Z");
  if (n == 0) return RMG_OK;
  if (on_device) {
    mlp_forward(n, X, m->theta.as<float>(), Z, nullptr, nullptr, m->stream);
    return RMG_OK;
  }
  DBuf dX, dZ;
  upload(dX, X, sizeof(float) * kMlpIn * n, m->stream);
  dZ.alloc(sizeof(float) * kMlpOut * n);
  mlp_forward(n, dX.as<float>(), m->theta.as<float>(), dZ.as<float>(), nullptr, nullptr, m->stream);
  RMG_HIP(hipMemcpyAsync(Z, dZ.p, sizeof(float) * kMlpOut * n, hipMemcpyDeviceToHost, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  API_END
}

rmg_status rmg_mlp_loss_grad(rmg_mlp* m, double* loss, float* grad) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(m->n > 0, RMG_ERR_NOT_SETUP, "no training data");
  reserve_work(m, m->n, 1);
  loss_grad(m, 0);
  double l = 0.0;
  RMG_HIP(hipMemcpyAsync(&l, m->losses.p, sizeof(double), hipMemcpyDeviceToHost, m->stream));
  if (grad)
    RMG_HIP(hipMemcpyAsync(grad, m->grad.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  if (loss) *loss = l / (double)m->n;
  API_END
}

rmg_status rmg_mlp_adam_step(rmg_mlp* m, const float* grad, double lr) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(lr > 0.0 && std::isfinite(lr), RMG_ERR_ARG, "learning rate must be positive");
  if (grad) {
    RMG_HIP(hipMemcpyAsync(m->grad.p, grad, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->stream));
    m->have_grad = true;
  }
  RMG_REQUIRE(m->have_grad, RMG_ERR_NOT_SETUP, "no gradient");
  adam(m, lr);
  RMG_HIP(hipStreamSynchronize(m->stream));
  API_END
}

rmg_status rmg_mlp_train(rmg_mlp* m, int steps, double lr, double* loss_history) {
  API_BEGIN
  mlp_use(m);
  RMG_REQUIRE(m->n > 0, RMG_ERR_NOT_SETUP, "no training data");
  RMG_REQUIRE(steps >= 0 && steps <= 1000000, RMG_ERR_ARG, "steps must be in [0, 10^6]");
  RMG_REQUIRE(lr > 0.0 && std::isfinite(lr), RMG_ERR_ARG, "learning rate must be positive");
  if (steps == 0) return RMG_OK;
  reserve_work(m, m->n, steps);
  for (int s = 0; s < steps; ++s) {
    loss_grad(m, s);
    adam(m, lr);
  }
  std::vector<double> hist(steps);
  RMG_HIP(hipMemcpyAsync(hist.data(), m->losses.p, sizeof(double) * steps, hipMemcpyDeviceToHost, m->stream));
  RMG_HIP(hipStreamSynchronize(m->stream));
  if (loss_history)
    for (int s = 0; s < steps; ++s) loss_history[s] = hist[s] / (double)m->n;
  API_END
}

}  // extern "C"
