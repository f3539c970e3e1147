// Hierarchy setup, regional V-cycle and preconditioned CG (host orchestration of the kernels).
#include <algorithm>
#include <fstream>
#include <cmath>
#include <string>

#include "kernels.h"

namespace rmg {

void KernelTimer::acquire(hipEvent_t* e0, hipEvent_t* e1) {
  while (ev.size() < used + 2) {
    hipEvent_t e;
    RMG_HIP(hipEventCreate(&e));
    ev.push_back(e);
  }
  *e0 = ev[used];
  *e1 = ev[used + 1];
  used += 2;
}

void KernelTimer::harvest() {
  for (size_t i = 0; i + 1 < used; i += 2) {
    float ms = 0.f;
    RMG_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    total_ms += ms;
    ++count;
  }
  used = 0;
}

void KernelTimer::reset() {
  used = 0;
  count = 0;
  total_ms = 0.0;
}

KernelTimer::~KernelTimer() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

static int64_t partial_capacity(const Level& L) {
  // node blocks, 2.5D tiles or the region-table split (whole-region table tiles, other regions'
  // tiles), then the interface groups
  const int64_t split = (int64_t)(L.table_tiles.size() + L.tiles.size());
  return std::max({(int64_t)L.blocks.size(), (int64_t)L.tiles.size(), split}) + (L.ngroups + kBlock - 1) / kBlock + 16;
}

static double* scal(rmg_handle* h) { return h->scalars.as<double>(); }

static void read_scalars(rmg_handle* h) {
  RMG_HIP(hipMemcpyAsync(h->host_scalars, h->scalars.p, sizeof(double) * kNumSlots, hipMemcpyDeviceToHost,
                         h->stream));
  RMG_HIP(hipStreamSynchronize(h->stream));
}

static void dot(rmg_handle* h, const Level& L, const double* a, const double* b, int slot) {
  const int64_t np = launch_dot(L, a, b, h->partials.as<double>(), h->stream);
  launch_reduce(h->partials.as<double>(), np, scal(h), slot, h->stream);
}

// lambda_max(D~^-1 Psi^T Psi [[A]]) by power iteration: x <- x0/|x0|; y = D~^-1 A x,
// lambda = (x, y), x = y/|y| (Section 3.4; start vector from the counter generator).
static double power_method(rmg_handle* h, Level& L, int level) {
  hipStream_t st = h->stream;
  double* x = L.u.as<double>();
  double* y = L.u2.as<double>();
  double* t = L.r.as<double>();
  launch_start_vector(L, level, h->opt.seed, x, st);
  dot(h, L, x, x, kTmp);
  launch_scale(L.ndofs(), scal(h), kTmp, 0, x, x, st);
  for (int it = 0; it < h->opt.power_iters; ++it) {
    StencilArgs a;
    a.op = StencilOp::Matvec;
    a.x = x;
    a.out = t;
    launch_stencil_op(L, a, st);
    if (L.dinv9.p) launch_mul_block3(L.n, L.dinv9.as<double>(), t, y, st);
    else launch_mul(L.ndofs(), L.dinv.as<double>(), t, y, st);
    dot(h, L, x, y, kTmp2);
    dot(h, L, y, y, kTmp);
    launch_scale(L.ndofs(), scal(h), kTmp, 0, y, x, st);
  }
  read_scalars(h);
  return h->host_scalars[kTmp2];
}

static void chebyshev_coefficients(const rmg_options& o, Level& L) {
  if (o.smoother >= 1) {  // damped Jacobi: every step is d = omega D~^-1 r, u += d (unused by Gauss-Seidel)
    L.cheb_c1.assign(o.cheb_degree, 0.0);
    L.cheb_c2.assign(o.cheb_degree, o.jacobi_omega);
    return;
  }
  const double alpha = L.lambda / o.eig_ratio;
  const double beta = o.boost * L.lambda;
  const double theta = 0.5 * (alpha + beta);
  const double delta = 2.0 / (beta - alpha);
  L.cheb_c1.assign(o.cheb_degree, 0.0);
  L.cheb_c2.assign(o.cheb_degree, 0.0);
  double rho = 1.0 / (theta * delta);
  L.cheb_c2[0] = 1.0 / theta;  // first correction d = D~^-1 r / theta
  for (int k = 1; k < o.cheb_degree; ++k) {
    const double rho_old = rho;
    rho = 1.0 / (2.0 * theta * delta - rho_old);
    L.cheb_c1[k] = rho * rho_old;
    L.cheb_c2[k] = 2.0 * rho * delta;
  }
}

static void alloc_vectors(Level& L, bool with_b) {
  const size_t bytes = sizeof(double) * (size_t)L.ndofs();
  if (with_b) L.b.alloc(bytes);
  L.u.alloc(bytes);
  L.u2.alloc(bytes);
  L.d.alloc(bytes);
  L.r.alloc(bytes);
}

static void alloc_vectors_lowp(Level& L, bool with_b) {
  const size_t bytes = sizeof(float) * (size_t)L.ndofs();
  if (with_b) L.b32.alloc(bytes);
  L.u32.alloc(bytes);
  L.u232.alloc(bytes);
  L.d32.alloc(bytes);
  L.r32.alloc(bytes);
}

// ------------------------------------------------------------------- autotuner
// Candidate launch shapes of the scalar 3D stencil kernels on one level.
struct TuneChoice {
  int mode;   // 0 node-parallel, 1 one block per 2.5D tile, 2 persistent grid over the tiles
  int depth;  // planes per tile
  int grid;   // persistent grid size
};

static std::string tune_key(const Level& L, int level, int precision) {
  std::string k = "n" + std::to_string(L.n) + "_r" + std::to_string(L.nreg) + "_l" + std::to_string(level) + "_p" +
                  std::to_string(precision);
  for (int i = 0; i < std::min(L.nreg, 4); ++i)
    k += "_" + std::to_string(L.regs[i].ex) + "x" + std::to_string(L.regs[i].ey) + "x" + std::to_string(L.regs[i].ez);
  return k;
}

static void apply_choice(Level& L, const TuneChoice& c) {
  if (c.mode == 0) {
    L.use_tiles = false;
    L.tile_grid = 0;
    return;
  }
  if (L.tile_depth != c.depth) make_tiles(L, c.depth);
  L.use_tiles = true;
  L.tile_grid = c.mode == 2 ? c.grid : 0;
}

// Times the Chebyshev step on the level's own operator and scratch vectors (zero-filled) for
// every candidate and keeps the fastest.  Choices are cached in a text file when configured.
static void autotune_level(rmg_handle* h, Level& L, int level, bool lowp) {
  hipStream_t st = h->stream;
  const std::string key = tune_key(L, level, h->opt.precision);
  if (!h->autotune_cache.empty()) {
    std::ifstream in(h->autotune_cache);
    std::string k;
    TuneChoice c;
    while (in >> k >> c.mode >> c.depth >> c.grid) {
      if (k == key) {
        apply_choice(L, c);
        h->tune_report.push_back("level " + std::to_string(level) + " cached mode " + std::to_string(c.mode) +
                                 " depth " + std::to_string(c.depth) + " grid " + std::to_string(c.grid));
        return;
      }
    }
  }
  std::vector<TuneChoice> cands = {{0, 21, 0}, {1, 11, 0}, {1, 21, 0}, {1, 41, 0}, {2, 21, 256}, {2, 21, 512}, {2, 21, 1024}};
  const size_t vb = (lowp ? sizeof(float) : sizeof(double)) * (size_t)L.ndofs();
  void* vec[5] = {lowp ? L.u32.p : L.u.p, lowp ? L.u232.p : L.u2.p, lowp ? L.d32.p : L.d.p,
                  lowp ? L.r32.p : L.r.p, lowp ? L.b32.p : L.b.p};
  for (void* v : vec)
    if (v) RMG_HIP(hipMemsetAsync(v, 0, vb, st));
  const void* dinv = lowp ? L.dinv_lo.p : L.dinv.p;
  hipEvent_t e0, e1;
  RMG_HIP(hipEventCreate(&e0));
  RMG_HIP(hipEventCreate(&e1));
  double best = 1e30;
  TuneChoice bestc = cands[0];
  for (const TuneChoice& c : cands) {
    apply_choice(L, c);
    StencilArgs a;
    a.op = StencilOp::Cheb;
    a.lowp = lowp;
    a.x = vec[0];
    a.out = vec[1];
    a.b = vec[3];
    a.dinv = dinv;
    a.d = vec[2];
    a.c1 = 0.5;
    a.c2 = 0.5;
    launch_stencil_op(L, a, st);  // warm-up
    RMG_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) launch_stencil_op(L, a, st);
    RMG_HIP(hipEventRecord(e1, st));
    RMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    RMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      bestc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  apply_choice(L, bestc);
  h->tune_report.push_back("level " + std::to_string(level) + " mode " + std::to_string(bestc.mode) + " depth " +
                           std::to_string(bestc.depth) + " grid " + std::to_string(bestc.grid) + " step_ms " +
                           std::to_string(best / 3.0));
  if (!h->autotune_cache.empty()) {
    std::ofstream out(h->autotune_cache, std::ios::app);
    out << key << " " << bestc.mode << " " << bestc.depth << " " << bestc.grid << "\n";
  }
}

// Launch configuration, work vectors and symmetric half-stencil copy of one stencil level.
static void configure_level(rmg_handle* h, Level& L, bool with_b, bool sym) {
  const rmg_options& o = h->opt;
  const bool fp64 = o.precision == RMG_PREC_FP64;
  const int threads = fp64 ? kTileThreadsF64 : kTileThreadsF32;
  if (L.dim == 3 && (L.tile_depth != 21 || L.tile_threads != threads)) {
    L.tile_threads = threads;
    make_tiles(L, 21);
  }
  const size_t tiles21 = L.tiles.size();
  // FP64 tiles run one block per CU: on a level large enough for tiles, 41-plane tiles read two
  // halo planes per 41 instead of per 21, kept while they still give every CU four or more.
  if (o.tile_planes == 41 && L.dim == 3) {
    make_tiles(L, 41);
  } else if (o.tile_planes == 0 && L.dim == 3 && fp64 && tiles21 >= kAutoTileMin) {
    make_tiles(L, 41);
    if (L.tiles.size() < kDeepTileMin) make_tiles(L, 21);
  }
  L.tile_grid = 0;
  L.per_region = o.batched == 0;
  L.use_tiles = !L.per_region && L.ndof == 1 && !L.tiles.empty() &&
                (o.stencil_kernel >= 2 || (o.stencil_kernel == 0 && tiles21 >= kAutoTileMin));
  // persistent tiles: 4 blocks per CU, and at least two tiles per block
  if (L.use_tiles && o.stencil_kernel == 3) L.tile_grid = std::max(1, std::min(1024, (int)(L.tiles.size() + 1) / 2));
  alloc_vectors(L, with_b);
  L.ct_lo = kCoefF64;
  L.coef_lo.release();
  L.center_lo.release();
  L.coef_lo_sym.release();
  if (sym) {
    // class tables for the FP64 2.5D tiles and, on FP64 levels run by node blocks, for those blocks
    const bool tables = o.region_table != 0 && fp64 && L.npts == 27 &&
                        ((L.use_tiles && L.tile_threads == kTileThreadsF64) || (!L.use_tiles && !L.per_region));
    launch_make_sym(L, false, h->stream, tables);
  } else {
    L.coef_sym.release();
    L.class_table.release();
    L.class_table_ok.release();
    clear_split(L);
  }
}

void prepare_finest(rmg_handle* h) {
  Level* L0 = h->levels[0];
  for (size_t i = 1; i < h->levels.size(); ++i) delete h->levels[i];
  h->levels.resize(1);
  h->tune_report.clear();
  h->partials.alloc(sizeof(double) * partial_capacity(*L0));
  configure_level(h, *L0, false, h->opt.symmetric != 0);
  L0->pw.release();
  L0->rw.release();
  RMG_HIP(hipStreamSynchronize(h->stream));
}

// Levels 0 .. nlevels-1: smoother data, next level by per-region Galerkin product, and the
// coarsest level's direct solver.  `stored`: the finest level interpolates with stored (caller
// or learned) weights when they are valid; returns their validity flags (0 when valid or unused).
static int build_levels(rmg_handle* h, bool stored) {
  const rmg_options& o = h->opt;
  hipStream_t st = h->stream;
  Level* L0 = h->levels[0];
  for (size_t i = 1; i < h->levels.size(); ++i) delete h->levels[i];
  h->levels.resize(1);
  const bool lowp = o.precision != RMG_PREC_FP64;
  h->tune_report.clear();
  h->partials.alloc(sizeof(double) * partial_capacity(*L0));
  int pflags = 0;
  DBuf flag;
  flag.alloc(sizeof(int));
  for (int l = 0; l < o.nlevels; ++l) {
    Level& L = *h->levels[l];
    configure_level(h, L, l > 0, o.symmetric && l < o.nlevels - 1);  // (the coarsest is solved directly)
    if (lowp) alloc_vectors_lowp(L, true);  // level 0's b32 holds the FP32 copy of the CG residual
    if (l == o.nlevels - 1) {
      if (o.coarse_amg) amg_setup(h, L);  // Section 3.5: an AMG V-cycle instead of the direct solver
      else build_coarse_solver(h, L);
      break;
    }
    // D~ = Psi^T Psi diag([[A]]) (point diagonal), then its reciprocal (Section 3.2, smoother setup)
    L.dinv.alloc(sizeof(double) * (size_t)L.ndofs());
    launch_diag(L, L.r.as<double>(), st);
    launch_interface_sum(L, L.r.as<double>(), L.r.as<double>(), st);
    RMG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
    launch_recip_check(L.ndofs(), L.r.as<double>(), L.dinv.as<double>(), flag.as<int>(), st);
    int hflag = 0;
    RMG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    RMG_HIP(hipStreamSynchronize(st));
    RMG_REQUIRE(hflag == 0, RMG_ERR_NUMERIC, "composite diagonal not positive on level " + std::to_string(l));
    // block_diag: the nodal 3 x 3 blocks of D~, inverted per node, wherever D~^-1 enters
    if (o.block_diag) launch_block_diag(L, st);
    else L.dinv9.release();
    L.dinv9_lo.release();
    L.lambda = power_method(h, L, l);
    RMG_REQUIRE(std::isfinite(L.lambda) && L.lambda > 0.0, RMG_ERR_NUMERIC,
                "power method failed on level " + std::to_string(l));
    chebyshev_coefficients(o, L);
    if (o.smoother >= 2) launch_gs_prepare(L, st);
    else {
      L.gs_rplane.release();
      L.gs_pbase.release();
      L.gs_coef.release();
      L.gs_dinv.release();
      L.gs_d.release();
    }
    // next level: geometry, interpolation weights, then the per-region Galerkin product (FP64)
    Level* C = make_coarse_level(L);
    h->levels.push_back(C);
    make_transfer_tiles(L, *C, o.transfer_rows != 0);
    C->coef.alloc(sizeof(double) * coef_elems(C->n, C->ncoef()));
    if (l == 0) {
      if (stored) {
        pflags = prepare_stored_weights(h, L, *C);
      } else {
        L.pw.release();
        L.rw.release();
      }
    }
    L.rap_separable = o.galerkin_generic == 0;
    launch_rap(L, *C, st);
    // the V-cycle's copy of this level's operator, made after the Galerkin product used it
    if (lowp) {
      launch_make_lowp(L, (l == 0 && o.precision == RMG_PREC_FP32_BF16) ? kCoefBF16 : kCoefF32, st);
      if (o.symmetric) launch_make_sym(L, true, st, false);
    }
    if (o.autotune && !L.per_region && L.dim == 3 && L.ndof == 1 && L.npts == 27) autotune_level(h, L, l, lowp);
  }
  if (lowp) h->cg_z32.alloc(sizeof(float) * (size_t)L0->ndofs());
  RMG_HIP(hipStreamSynchronize(st));
  return pflags;
}

static void judge_learned(rmg_handle* h);
static void choose_bf16_levels(rmg_handle* h);

void setup_hierarchy(rmg_handle* h) {
  const rmg_options& o = h->opt;
  Level* L0 = h->levels[0];
  if (o.hybrid) {
    // the aggregation hierarchy checks its own composite lattice level by level (hybrid.cpp)
  } else if (h->pmode != RMG_P_GEOMETRIC) {
    // stored interpolation weights are kept per canonical cell of the uniform rate-3 lattice
    int64_t f = 1;
    for (int l = 1; l < o.nlevels; ++l) f *= 3;
    for (int k = 0; k < L0->nreg; ++k) {
      const RegionGeo& R = L0->regs[k];
      const int e[3] = {R.ex, R.ey, R.ez}, g[3] = {R.ox, R.oy, R.oz};
      for (int d = 0; d < L0->dim; ++d)
        RMG_REQUIRE((e[d] - 1) % f == 0 && g[d] % f == 0, RMG_ERR_SHAPE,
                    "region " + std::to_string(k) + ": extent-1 and origin must be divisible by 3^(nlevels-1) = " +
                        std::to_string(f));
    }
  } else {  // every level's coarse lattice must agree across interfaces: check before building
    std::vector<RegionGeo> fine = L0->regs, coarse;
    int comp[3];
    for (int l = 1; l < o.nlevels; ++l) {
      coarse_geometry(L0->dim, fine, coarse, comp);
      fine.swap(coarse);
    }
  }
  h->p_used = RMG_P_GEOMETRIC;
  h->rho_learned = h->rho_geometric = -1.0;
  h->p_flags = 0;
  hybrid_destroy(h);
  amg_destroy(h);
  if (o.hybrid) {  // aggregation hierarchy of the structured/unstructured hybrid
    prepare_finest(h);
    hybrid_setup(h);
    return;
  }
  const bool stored = h->pmode != RMG_P_GEOMETRIC;
  RMG_REQUIRE(!stored || (L0->dim == 3 && L0->ndof == 1), RMG_ERR_ARG,
              "stored or learned interpolation needs a scalar 3D problem");
  h->p_flags = build_levels(h, stored);
  if (stored && h->p_flags == 0) h->p_used = h->pmode;
  if (h->p_used == RMG_P_LEARNED && o.judge_cycles > 0) judge_learned(h);
  if (o.precision == RMG_PREC_FP32_BF16_AUTO) choose_bf16_levels(h);
}

// The judge: keep the learned hierarchy only if it converges faster than the geometric one.
static void judge_learned(rmg_handle* h) {
  const rmg_options& o = h->opt;
  Level* L0 = h->levels[0];
  const double rl = convergence_factor(h, o.judge_cycles);
  std::vector<Level*> learned(h->levels.begin() + 1, h->levels.end());
  h->levels.resize(1);
  DBuf pw, rw;
  pw.swap(L0->pw);
  rw.swap(L0->rw);
  try {
    build_levels(h, false);
  } catch (...) {
    for (Level* l : learned) delete l;
    throw;
  }
  const double rg = convergence_factor(h, o.judge_cycles);
  h->rho_learned = rl;
  h->rho_geometric = rg;
  if (rl < rg) {
    for (size_t i = 1; i < h->levels.size(); ++i) delete h->levels[i];
    h->levels.resize(1);
    h->levels.insert(h->levels.end(), learned.begin(), learned.end());
    L0->pw.swap(pw);
    L0->rw.swap(rw);
  } else {
    for (Level* l : learned) delete l;
    h->p_used = RMG_P_GEOMETRIC;
    h->p_flags = RMG_PW_JUDGED_WORSE;
  }
}

// Low-precision copy of a level's stencil for the V-cycle, as build_levels makes it.
static void set_level_lowp(rmg_handle* h, Level& L, int coef_type) {
  launch_make_lowp(L, coef_type, h->stream);
  if (h->opt.symmetric) launch_make_sym(L, true, h->stream, false);
}

// Per-level BF16 (RMG_PREC_FP32_BF16_AUTO): the convergence factor of bf16_cycles stationary
// V-cycles with every level in FP32 is the reference; finest level first, each smoothed 27-point
// level is switched to BF16 off-diagonals and kept there when the factor, measured with the finer
// levels as already decided, stays within (1 + bf16_tolerance) of the reference.
static void choose_bf16_levels(rmg_handle* h) {
  const rmg_options& o = h->opt;
  const int nl = (int)h->levels.size();
  for (Level* L : h->levels) L->rho_fp32 = L->rho_bf16 = -1.0;
  const double ref = convergence_factor(h, o.bf16_cycles);
  RMG_REQUIRE(std::isfinite(ref), RMG_ERR_NUMERIC, "convergence factor of the FP32 V-cycle is not finite");
  for (int l = 0; l < nl - 1; ++l) {
    Level& L = *h->levels[l];
    if (L.npts != 27 || L.ct_lo != kCoefF32) continue;
    set_level_lowp(h, L, kCoefBF16);
    const double rho = convergence_factor(h, o.bf16_cycles);
    L.rho_fp32 = ref;
    L.rho_bf16 = rho;
    if (!(std::isfinite(rho) && rho <= ref * (1.0 + o.bf16_tolerance))) set_level_lowp(h, L, kCoefF32);
  }
  RMG_HIP(hipStreamSynchronize(h->stream));
}

// Buffers of one level for the FP64 or the FP32 V-cycle.
struct Bufs {
  void *b, *u, *u2, *d, *r;
  const void* dinv;
  const void* dinv9;  // nodal-block D~^-1 (block_diag), else null
};

static Bufs bufs(Level& L, bool lowp) {
  if (lowp) return {L.b32.p, L.u32.p, L.u232.p, L.d32.p, L.r32.p, L.dinv_lo.p, L.dinv9_lo.p};
  return {L.b.p, L.u.p, L.u2.p, L.d.p, L.r.p, L.dinv.p, L.dinv9.p};
}

// Kinds of Chebyshev step: the iterate before uin is in uout (Next), is zero (AfterZero: the step
// after the zero-guess start), or there is no previous correction (Start: smoothing an iterate).
enum class ChebKind { Next, AfterZero, Start };

// One Chebyshev step uin -> uout; with dot (FP64), also the partial sums of (b, uout) over the
// owned copies into h->partials, whose count it returns.
static int64_t cheb_step(rmg_handle* h, Level& L, bool lowp, int k, ChebKind kind, const void* b, const void* uin,
                         void* uout, bool dot = false) {
  const Bufs B = bufs(L, lowp);
  StencilArgs a;
  a.op = kind == ChebKind::Next ? StencilOp::Cheb : StencilOp::ChebFirst;
  a.lowp = lowp;
  a.x = uin;
  a.out = uout;
  a.b = b;
  a.dinv = B.dinv;
  a.dinv9 = B.dinv9;
  a.d = B.d;
  a.c1 = kind == ChebKind::Start ? 0.0 : L.cheb_c1[k];
  a.c2 = L.cheb_c2[k];
  if (dot) {
    a.dot_rhs = true;
    a.partials = h->partials.as<double>();
  }
  if (h->profiling && &L == h->levels[0] && kind == ChebKind::Next && !dot)
    h->timers[kTimedCheb].acquire(&a.ev0, &a.ev1);
  return launch_stencil_op(L, a, h->stream);
}

// Region-local Gauss-Seidel (Section 3.4, Algorithm 1), cheb_degree sweeps on u in place (FP64).
// Each sweep: the composite residual r = b - A u with its interface sum, the region sweeps into d,
// the average of the copies of every interface dof, u += d.  zero: u is 0 on entry, so the first
// residual is b and the first sweep writes its corrections straight into u.
static void gs_sweep(rmg_handle* h, Level& L, const double* b, double* u, bool zero, bool backward) {
  hipStream_t st = h->stream;
  const double omega = h->opt.jacobi_omega;
  if (zero) {
    launch_gs_sweep(L, b, u, omega, backward, st);
    launch_interface_avg(L, u, st);
    return;
  }
  StencilArgs a;
  a.op = StencilOp::Residual;
  a.x = u;
  a.out = L.r.p;
  a.b = b;
  launch_stencil_op(L, a, st);
  launch_gs_sweep(L, L.r.as<double>(), L.d.as<double>(), omega, backward, st);
  launch_interface_avg(L, L.d.as<double>(), st);
  launch_add(L.ndofs(), L.d.as<double>(), u, st);
}

// smoother 4 (symmetric Gauss-Seidel): every iteration a forward then a backward sweep.
static void gs_smooth(rmg_handle* h, Level& L, const double* b, double* u, bool zero, bool backward) {
  for (int k = 0; k < h->opt.cheb_degree; ++k) {
    gs_sweep(h, L, b, u, zero && k == 0, backward && h->opt.smoother != 4);
    if (h->opt.smoother == 4) gs_sweep(h, L, b, u, false, true);
  }
}

void smooth_zero_guess(rmg_handle* h, int level, const double* b, double* u_out) {
  RMG_REQUIRE(h->hy == nullptr, RMG_ERR_ARG, "per-level smoothing is not available on the hybrid hierarchy");
  Level& L = *h->levels[level];
  hipStream_t st = h->stream;
  if (h->opt.smoother >= 2) {
    gs_smooth(h, L, b, u_out, true, false);
    return;
  }
  const int K = h->opt.cheb_degree;
  void* buf[2] = {L.u.p, u_out};
  launch_cheb_zero(L, false, b, L.dinv.p, L.cheb_c2[0], buf[0], st, L.dinv9.p);
  int cur = 0;
  for (int k = 1; k < K; ++k) {
    cheb_step(h, L, false, k, k == 1 ? ChebKind::AfterZero : ChebKind::Next, b, buf[cur], buf[1 - cur]);
    cur = 1 - cur;
  }
  if (buf[cur] != u_out) launch_copy(L.ndofs(), (const double*)buf[cur], u_out, st);
}

void smooth_iterate(rmg_handle* h, int level, const double* b, double* u, double* tmp) {
  Level& L = *h->levels[level];
  RMG_REQUIRE(h->opt.smoother < 2, RMG_ERR_ARG, "smooth_iterate: Chebyshev or Jacobi smoother only");
  void* buf[2] = {u, tmp};
  int cur = 0;
  for (int k = 0; k < h->opt.cheb_degree; ++k) {
    cheb_step(h, L, false, k, k == 0 ? ChebKind::Start : ChebKind::Next, b, buf[cur], buf[1 - cur]);
    cur = 1 - cur;
  }
  if (cur) launch_copy(L.ndofs(), tmp, u, h->stream);
}

// Counter stream of the start vector of rmg_convergence_factor (power-method streams are the level
// numbers, training errors 32 + sample).
constexpr int kRhoStream = 63;

double convergence_factor(rmg_handle* h, int cycles, double* work) {
  Level& L = *h->levels[0];
  hipStream_t st = h->stream;
  const int64_t n = L.ndofs();
  DBuf own;
  if (!work) {
    own.alloc(sizeof(double) * 4 * (size_t)n);
    work = own.as<double>();
  }
  // work: the zero right-hand side, the iterate, its residual and the correction, n each
  double* zero = work;
  double* x = work + n;
  double* r = work + 2 * n;
  double* z = work + 3 * n;
  launch_zero(n, zero, st);
  launch_start_vector(L, kRhoStream, h->opt.seed, x, st);
  auto residual = [&] {
    StencilArgs a;
    a.op = StencilOp::Residual;
    a.x = x;
    a.out = r;
    a.b = zero;
    launch_stencil_op(L, a, st);
  };
  residual();
  dot(h, L, r, r, kTmp);
  read_scalars(h);
  const double r0 = std::sqrt(h->host_scalars[kTmp]);
  for (int c = 0; c < cycles; ++c) {
    apply_preconditioner(h, r, z);
    launch_add(n, z, x, st);
    residual();
  }
  dot(h, L, r, r, kTmp);
  read_scalars(h);
  const double rk = std::sqrt(h->host_scalars[kTmp]);
  if (!(r0 > 0.0)) return 0.0;
  return std::pow(rk / r0, 1.0 / cycles);
}

// Per-level preconditioner time (rmg_profile on; never inside a captured graph, where profiling is
// switched off): an event pair around a level's own launches.  begin returns the closing event.
static hipEvent_t level_span_begin(rmg_handle* h, int level) {
  if (!h->profiling || !h->timing_levels) return nullptr;
  hipEvent_t e0, e1;
  h->level_timers[level].acquire(&e0, &e1);
  RMG_HIP(hipEventRecord(e0, h->stream));
  return e1;
}

static void level_span_end(rmg_handle* h, hipEvent_t e1) {
  if (e1) RMG_HIP(hipEventRecord(e1, h->stream));
}

static void level_times_reset(rmg_handle* h) {
  for (auto& t : h->level_timers) t.reset();
  h->timing_levels = true;
}

// After a stream synchronisation: the solve's per-level totals into info.
static void level_times_report(rmg_handle* h, rmg_solve_info* info) {
  h->timing_levels = false;
  for (int l = 0; l < 12; ++l) {
    h->level_timers[l].harvest();
    if (info) info->level_ms[l] = h->level_timers[l].total_ms;
  }
}

void mg_solve(rmg_handle* h, const double* b, double* x, double rtol, int maxit, rmg_solve_info* info,
              rmg_status* status) {
  Level& L = *h->levels[0];
  hipStream_t st = h->stream;
  const int64_t n = L.ndofs();
  double* r = h->cg_r.as<double>();
  double* z = h->cg_z.as<double>();
  hipEvent_t e0, e1;
  RMG_HIP(hipEventCreate(&e0));
  RMG_HIP(hipEventCreate(&e1));
  level_times_reset(h);
  RMG_HIP(hipEventRecord(e0, st));
  auto residual = [&] {
    StencilArgs a;
    a.op = StencilOp::Residual;
    a.x = x;
    a.out = r;
    a.b = b;
    launch_stencil_op(L, a, st);
  };
  int hist_len = 0;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_len < info->history_cap) info->history[hist_len] = v;
    ++hist_len;
  };
  *status = RMG_OK;
  dot(h, L, b, b, kBB);
  residual();
  dot(h, L, r, r, kRR);
  read_scalars(h);
  const double bnorm = std::sqrt(h->host_scalars[kBB]);
  double rel = bnorm > 0.0 ? std::sqrt(h->host_scalars[kRR]) / bnorm : 0.0;
  push_hist(rel);
  int it = 0;
  bool converged = bnorm == 0.0 || rel <= rtol;
  if (bnorm == 0.0) launch_zero(n, x, st);
  while (!converged && it < maxit) {
    apply_preconditioner(h, r, z);
    launch_add(n, z, x, st);
    residual();
    dot(h, L, r, r, kRR);
    read_scalars(h);
    ++it;
    const double rr = h->host_scalars[kRR];
    if (!std::isfinite(rr)) {
      *status = RMG_ERR_BREAKDOWN;
      set_last_error("multigrid iteration diverged (non-finite residual)");
      break;
    }
    rel = std::sqrt(rr) / bnorm;
    push_hist(rel);
    converged = rel <= rtol;
  }
  RMG_HIP(hipEventRecord(e1, st));
  RMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  RMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  level_times_report(h, info);
  if (*status == RMG_OK && !converged) {
    *status = RMG_ERR_NOT_CONVERGED;
    set_last_error("multigrid did not reach rtol within maxit cycles");
  }
  if (info) {
    info->iterations = it;
    info->converged = converged ? 1 : 0;
    info->relres = rel;
    info->true_relres = rel;  // the residual is recomputed from x every cycle
    info->solve_ms = ms;
    info->history_len = hist_len;
    info->setup_ms = h->setup_ms;
  }
}

void vcycle(rmg_handle* h, int level, bool lowp, const void* b, void* z, int dot_slot, bool start_ready) {
  const int nl = (int)h->levels.size();
  Level& L = *h->levels[level];
  hipStream_t st = h->stream;
  if (level == nl - 1) {
    hipEvent_t span = level_span_begin(h, level);
    if (h->amg) {
      launch_coarse_gather(L, lowp, b, st);
      amg_cycle(h, L.cvec.as<double>(), L.cvec2.as<double>());
      launch_coarse_scatter(L, lowp, z, st);
    } else {
      launch_coarse_solve(L, lowp, b, z, st);
    }
    level_span_end(h, span);
    return;
  }
  hipEvent_t span = level_span_begin(h, level);
  if (h->opt.smoother >= 2) {  // region-local Gauss-Seidel (FP64 only), in place on z
    double* u = static_cast<double*>(z);
    gs_smooth(h, L, static_cast<const double*>(b), u, true, false);
    StencilArgs a;
    a.op = StencilOp::ResidualScaled;
    a.x = u;
    a.out = L.r.p;
    a.b = b;
    launch_stencil_op(L, a, st);
    Level& C = *h->levels[level + 1];
    launch_restrict(L, C, false, L.r.p, C.b.p, st);
    level_span_end(h, span);
    vcycle(h, level + 1, false, C.b.p, C.u2.p);
    span = level_span_begin(h, level);
    launch_prolong_add(L, C, false, C.u2.p, u, st);
    gs_smooth(h, L, static_cast<const double*>(b), u, false, h->opt.smoother == 3);
    level_span_end(h, span);
    return;
  }
  const int K = h->opt.cheb_degree;
  const Bufs B = bufs(L, lowp);
  // ping-pong buffers arranged so that the last post-smoothing step writes z
  void* buf[2] = {B.u, z};
  // the zero-guess start (already in B.u when the CG update wrote it from the new residual)
  if (!start_ready) launch_cheb_zero(L, lowp, b, B.dinv, L.cheb_c2[0], buf[0], st, B.dinv9);
  int cur = 0;
  for (int k = 1; k < K; ++k) {
    cheb_step(h, L, lowp, k, k == 1 ? ChebKind::AfterZero : ChebKind::Next, b, buf[cur], buf[1 - cur]);
    cur = 1 - cur;
  }
  // residual divided by multiplicity, restriction and coarse interface sum (Section 3.3)
  StencilArgs a;
  a.op = StencilOp::ResidualScaled;
  a.lowp = lowp;
  a.x = buf[cur];
  a.out = B.r;
  a.b = b;
  launch_stencil_op(L, a, st);
  Level& C = *h->levels[level + 1];
  const Bufs BC = bufs(C, lowp);
  launch_restrict(L, C, lowp, B.r, BC.b, st);
  level_span_end(h, span);
  vcycle(h, level + 1, lowp, BC.b, BC.u2);
  span = level_span_begin(h, level);
  launch_prolong_add(L, C, lowp, BC.u2, buf[cur], st);
  for (int k = 0; k < K; ++k) {
    // the last step also sums (b, z) when asked (the CG inner product (r, z))
    const bool dot = k == K - 1 && dot_slot >= 0 && !lowp;
    const int64_t np =
        cheb_step(h, L, lowp, k, k == 0 ? ChebKind::Start : ChebKind::Next, b, buf[cur], buf[1 - cur], dot);
    if (dot) launch_reduce(h->partials.as<double>(), np, scal(h), dot_slot, st);
    cur = 1 - cur;
  }
  level_span_end(h, span);
  RMG_REQUIRE(buf[cur] == z, RMG_ERR_ARG, "internal: V-cycle buffer parity");
}

// z = M^-1 r with the configured precision (FP64 regional vectors in and out); with slot >= 0 also
// (r, z) into that scalar slot, summed by the V-cycle's last Chebyshev step where it has one.
// start_ready: the finest level's zero-guess start is already in its u (fused_start_ok).
static void precondition(rmg_handle* h, const double* r, double* z, int slot = -1, bool start_ready = false) {
  Level& L = *h->levels[0];
  if (h->hy) {
    hybrid_cycle(h, r, z);
  } else if (h->opt.precision == RMG_PREC_FP64) {
    const bool fused = slot >= 0 && h->opt.smoother <= 1 && h->levels.size() > 1;
    vcycle(h, 0, false, r, z, fused ? slot : -1, start_ready);
    if (fused) return;
  } else {
    launch_f64_to_f32(L.ndofs(), r, L.b32.as<float>(), h->stream);
    vcycle(h, 0, true, L.b32.p, h->cg_z32.p);
    launch_f32_to_f64(L.ndofs(), h->cg_z32.as<float>(), z, h->stream);
  }
  if (slot >= 0) dot(h, L, r, z, slot);
}

void apply_preconditioner(rmg_handle* h, const double* r, double* z) { precondition(h, r, z); }

// Preconditioned CG (textbook Hestenes-Stiefel).  With a low-precision V-cycle, or the hybrid
// cycle, the preconditioner is only approximately a fixed symmetric operator, so the flexible
// (Polak-Ribiere) coefficient beta = (z_new, r_new - r_old) / (z_old, r_old) =
// -alpha (z_new, q) / (z_old, r_old) is used; the residual, the update and all inner products
// stay in FP64.
// Runs `body` under stream capture and instantiates the resulting graph.
template <class F>
static hipGraphExec_t capture_graph(hipStream_t st, F&& body) {
  hipGraph_t g = nullptr;
  RMG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(st, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  RMG_HIP(hipStreamEndCapture(st, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  RMG_HIP(err);
  return e;
}

// While alive, the handle's work goes to its private capture stream, ordered after (and, on
// exit, before) the caller's stream.
struct GraphStream {
  rmg_handle* h;
  hipStream_t user;
  GraphStream(rmg_handle* hh) : h(hh), user(hh->stream) {
    if (!h->gstream) RMG_HIP(hipStreamCreate(&h->gstream));
    hipEvent_t ev;
    RMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    RMG_HIP(hipEventRecord(ev, user));
    RMG_HIP(hipStreamWaitEvent(h->gstream, ev, 0));
    (void)hipEventDestroy(ev);
    h->stream = h->gstream;
  }
  ~GraphStream() {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(ev, h->gstream);
      (void)hipStreamWaitEvent(user, ev, 0);
      (void)hipEventDestroy(ev);
    }
    h->stream = user;
  }
};

// Whether the CG update can also write the FP64 V-cycle's zero-guess start on the finest level
// (scalar Chebyshev or Jacobi smoothing with the point D~ below a coarser level).
static bool fused_start_ok(rmg_handle* h) {
  const Level& L = *h->levels[0];
  return !h->hy && h->opt.precision == RMG_PREC_FP64 && h->opt.smoother <= 1 && h->levels.size() > 1 &&
         L.ndof == 1 && !L.dinv9.p && L.u.p && L.dinv.p;
}

static void pcg_impl(rmg_handle* h, const double* b, double* x, double rtol, int maxit, rmg_solve_info* info,
                     rmg_status* status) {
  Level& L = *h->levels[0];
  hipStream_t st = h->stream;
  const int64_t n = L.ndofs();
  // the hybrid cycle's region-local sweeps average the interface copies: not exactly symmetric
  const bool flexible = h->opt.precision != RMG_PREC_FP64 || h->hy != nullptr;
  const bool graphs = h->opt.use_graph != 0;
  // the CG update also writes the V-cycle's zero-guess start from the new residual
  const bool fused_start = fused_start_ok(h);
  double* r = h->cg_r.as<double>();
  double* p = h->cg_p.as<double>();
  double* q = h->cg_q.as<double>();
  double* z = h->cg_z.as<double>();
  double* part = h->partials.as<double>();
  hipEvent_t e0, e1;
  RMG_HIP(hipEventCreate(&e0));
  RMG_HIP(hipEventCreate(&e1));
  level_times_reset(h);
  RMG_HIP(hipEventRecord(e0, st));
  *status = RMG_OK;
  int hist_len = 0;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_len < info->history_cap) info->history[hist_len] = v;
    ++hist_len;
  };
  // first half of an iteration: q = A p, alpha, x and r updates, (r, r)
  auto body_a = [&](bool timed) {
    StencilArgs a;
    a.op = StencilOp::CgQ;
    a.x = p;
    a.out = q;
    a.partials = part;
    if (timed) h->timers[kTimedCgQ].acquire(&a.ev0, &a.ev1);
    const int64_t np = launch_stencil_op(L, a, st);
    launch_reduce(part, np, scal(h), kPQ, st);
    launch_cg_scalars(scal(h), 0, st);
    const int64_t nu = fused_start ? launch_cg_update(L, scal(h), x, r, p, q, part, st, L.dinv.as<double>(),
                                                      L.cheb_c2[0], L.u.as<double>())
                                   : launch_cg_update(L, scal(h), x, r, p, q, part, st);
    launch_reduce(part, nu, scal(h), kRR, st);
  };
  // second half: z = M^-1 r, beta, p update
  auto body_b = [&]() {
    precondition(h, r, z, kRZnew, fused_start);
    if (flexible) {
      dot(h, L, z, q, kZQ);
      launch_cg_scalars(scal(h), 2, st);
    } else {
      launch_cg_scalars(scal(h), 1, st);
    }
    launch_cg_direction(n, scal(h), z, p, st);
  };
  // r = b - A x0
  {
    StencilArgs a;
    a.op = StencilOp::Residual;
    a.x = x;
    a.out = r;
    a.b = b;
    launch_stencil_op(L, a, st);
  }
  dot(h, L, b, b, kBB);
  read_scalars(h);
  const double bnorm = std::sqrt(h->host_scalars[kBB]);
  int it = 0;
  double rel = 1.0;
  bool converged = false;
  // out = b - A x and its relative norm (true_rel)
  double true_rel = -1.0;
  auto true_residual = [&](double* out) {
    StencilArgs a;
    a.op = StencilOp::Residual;
    a.x = x;
    a.out = out;
    a.b = b;
    launch_stencil_op(L, a, st);
    dot(h, L, out, out, kTmp);
    read_scalars(h);
    true_rel = std::sqrt(h->host_scalars[kTmp]) / bnorm;
  };
  push_hist(1.0);
  if (bnorm == 0.0) {
    launch_zero(n, x, st);
    rel = 0.0;
    converged = true;
  } else {
    precondition(h, r, z, kRZ);
    launch_copy(n, z, p, st);
    if (graphs && (!h->graph_a || h->graph_b_ptr != b || h->graph_x_ptr != x)) {
      h->drop_graphs();
      const bool prof = h->profiling;
      h->profiling = false;  // no event records inside graphs
      h->graph_a = capture_graph(st, [&] { body_a(false); });
      h->graph_b = capture_graph(st, body_b);
      h->profiling = prof;
      h->graph_b_ptr = b;
      h->graph_x_ptr = x;
    }
    while (it < maxit) {
      if (graphs) RMG_HIP(hipGraphLaunch(h->graph_a, st));
      else body_a(h->profiling);
      ++it;
      read_scalars(h);
      if (h->profiling) {
        for (auto& t : h->timers) t.harvest();
        for (auto& t : h->level_timers) t.harvest();
      }
      const double rz = h->host_scalars[kRZ], pq = h->host_scalars[kPQ], rr = h->host_scalars[kRR];
      if (!(pq > 0.0) || !(rz > 0.0) || !std::isfinite(rr)) {
        *status = RMG_ERR_BREAKDOWN;
        set_last_error("CG breakdown: (r,z) = " + std::to_string(rz) + ", (p,Ap) = " + std::to_string(pq));
        rel = std::sqrt(std::fabs(rr)) / bnorm;
        break;
      }
      rel = std::sqrt(rr) / bnorm;
      push_hist(rel);
      if (rel <= rtol) {
        // the tolerance is on the system's relative residual: the recursively updated r is
        // accepted only if b - A x agrees, else CG goes on from the true residual
        true_residual(r);
        if (true_rel <= rtol) {
          converged = true;
          break;
        }
        // CG goes on from the true residual: the zero-guess start the update wrote is stale
        if (fused_start && it < maxit) {
          Level& L0 = *h->levels[0];
          launch_cheb_zero(L0, false, r, L0.dinv.p, L0.cheb_c2[0], L0.u.p, st);
        }
      }
      if (it >= maxit) break;
      if (graphs) RMG_HIP(hipGraphLaunch(h->graph_b, st));
      else body_b();
    }
  }
  RMG_HIP(hipEventRecord(e1, st));
  RMG_HIP(hipEventSynchronize(e1));
  if (!converged && bnorm > 0.0) true_residual(q);  // reported true residual of the last iterate
  if (h->profiling)
    for (auto& t : h->timers) t.harvest();
  level_times_report(h, info);
  float ms = 0.f;
  RMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (*status == RMG_OK && !converged) {
    *status = RMG_ERR_NOT_CONVERGED;
    set_last_error("CG did not reach rtol within maxit iterations");
  }
  if (info) {
    info->iterations = it;
    info->converged = converged ? 1 : 0;
    info->relres = rel;
    info->true_relres = bnorm > 0.0 ? true_rel : 0.0;
    info->solve_ms = ms;
    info->history_len = hist_len;
    info->setup_ms = h->setup_ms;
  }
}

void pcg(rmg_handle* h, const double* b, double* x, double rtol, int maxit, rmg_solve_info* info,
         rmg_status* status) {
  if (h->opt.use_graph) {
    GraphStream gs(h);
    pcg_impl(h, b, x, rtol, maxit, info, status);
  } else {
    pcg_impl(h, b, x, rtol, maxit, info, status);
  }
}

}  // namespace rmg
