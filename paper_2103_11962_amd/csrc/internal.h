// Internal data structures of the regional multigrid library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <string>
#include <utility>
#include <vector>

#include "../../include/regmg.h"

namespace rmg {

// ---------------------------------------------------------------- errors
struct Error {
  rmg_status code;
  std::string msg;
};
[[noreturn]] void fail(rmg_status code, const std::string& msg);
void set_last_error(const std::string& msg);

#define RMG_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      ::rmg::fail(e_ == hipErrorOutOfMemory ? RMG_ERR_OOM : RMG_ERR_DEVICE,                \
                  std::string(#call " failed: ") + hipGetErrorString(e_));                 \
  } while (0)

#define RMG_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) ::rmg::fail(code, msg); \
  } while (0)

// Device memory provider of the entry point running on this thread (empty: hipMalloc/hipFree).
struct DevAlloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
DevAlloc& current_allocator();
// Restores the thread's provider when an entry point returns; bind_handle(h) selects h's device
// and provider for the rest of the entry point.
struct AllocatorScope {
  DevAlloc saved;
  AllocatorScope() : saved(current_allocator()) { current_allocator() = DevAlloc(); }
  ~AllocatorScope() { current_allocator() = saved; }
};

// Body of a C entry point: library errors become a status and the thread's last error.
#define API_BEGIN             \
  try {                       \
    rmg::AllocatorScope alloc_scope_;
#define API_END                                   \
  }                                               \
  catch (const rmg::Error& e) {                   \
    rmg::set_last_error(e.msg);                   \
    return e.code;                                \
  }                                               \
  catch (const std::exception& e) {               \
    rmg::set_last_error(e.what());                \
    return RMG_ERR_ARG;                           \
  }                                               \
  return RMG_OK;

// ------------------------------------------------------- device geometry
// One region on one level.  2D problems use ez = oz = 0 extents of 1.
struct RegionGeo {
  int ex, ey, ez;     // node extents
  int ox, oy, oz;     // composite coordinates of local node (0,0,0)
  int64_t off;        // first node of the region in the level's regional vector
  int n;              // ex*ey*ez
  int pad;
};

// A block of consecutive nodes of one region: the unit of work of node-parallel kernels.
struct BlockDesc {
  int region;
  int start;  // first local node index
};

constexpr int kBlock = 256;  // threads per block for node-parallel kernels
constexpr int kProlongStageXY = 384;  // coarse nodes per plane a prolongation tile stages at most
constexpr int kXferStagePerThread = 12;  // fine values per thread a restriction tile stages per plane at most

constexpr size_t kAutoTileMin = 2048;  // 2.5D tiles needed on a level before they are used by default
constexpr size_t kDeepTileMin = 1024;  // 41-plane FP64 tiles needed before they replace 21-plane ones

// Threads per 2.5D tile block.  The FP64 kernel needs about 150 VGPRs (3 waves per SIMD), so a
// 768-thread block (12 waves) is the widest that fits and one block runs per CU; the FP32 kernel
// needs about 93 (5 waves per SIMD), where five 256-thread blocks (20 waves) run per CU (two
// 512-thread blocks, 16 waves, took 6% longer per step on a 113M-row level).  A level whose
// V-cycle runs in FP32 uses the narrow tiles for every operation.
constexpr int kTileThreadsF64 = 768;
constexpr int kTileThreadsF32 = 256;
// Threads per whole-region tile of a table region (k_stencil_table): the inner x-nodes of a few rows
// padded to whole wavefronts plus their rows' four x-face nodes; planes and rows per tile at most.
// Five rows of 82 nodes fill 468 of 512 lanes; at six waves per SIMD three 8-wave blocks run per CU
// (on C2: 284 us per Chebyshev step, against 307 us for four rows in 384 threads, 288 us for eight
// rows in 768, 312 us for seven in 640).
constexpr int kTableThreads = 512;
constexpr int kTablePlanes = 41;
constexpr int kTableRows = 5;
// Largest (tx + 2)(ty + 2) over tiles of at most nt nodes (tx * ty <= nt): the single row, ty = 1.
constexpr int tile_plane_cap(int nt) { return 3 * (nt + 2); }
// Region tables: a node's class along an axis of extent e >= 5 is its coordinate on the two low
// layers (0, 1), 2 inside, and 3, 4 on the two high layers; a node's class is (cz * 5 + cy) * 5 + cx,
// and a served region keeps, per class, the 27 couplings in stencil order that every node of the
// class has.
constexpr int kClasses = 125;
constexpr int kClassPts = 27;

// A 2.5D tile of a 3D region: ty x-rows of tx nodes starting at (x0, y0), planes z0 .. z0+nz-1.
struct Tile3 {
  int region, x0, y0, z0, tx, ty, nz, pad;
};

// Stencil coefficients are stored wave-tiled: the npts coefficients of 64 consecutive regional
// nodes form one contiguous chunk laid out [s][lane], so a wavefront streams one contiguous
// block of memory instead of npts separate streams.
constexpr int kTile = 64;
__host__ __device__ __forceinline__ int64_t coef_index(int64_t gi, int s, int npts) {
  return ((gi >> 6) * npts + s) * kTile + (gi & (kTile - 1));
}
inline size_t coef_elems(int64_t n, int npts) { return (size_t)((n + kTile - 1) / kTile) * kTile * npts; }
constexpr int kSymPts = 14;  // upper half of a symmetric 27-point stencil: offsets 13..26

// Everything a kernel needs to know about a level, passed by value.
struct LevelView {
  const RegionGeo* regs;
  const BlockDesc* blocks;
  int nblocks;
  int nreg;
  int64_t n;         // regional nodes on the level
  int cx, cy, cz;    // composite node extents
  unsigned mask;     // Dirichlet faces
  int npts;          // stencil points stored (5, 9 or 27)
  int ndof;          // unknowns per node (1, or 3 for elasticity)
};

// Device buffer owned by the library.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevAlloc from;  // the provider p came from
  void alloc(size_t nbytes);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
  void swap(DBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(from, o.from);
  }
  ~DBuf() { release(); }
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
};

// Coefficient storage types of a level's low-precision copy.
enum CoefType { kCoefF64 = 0, kCoefF32 = 1, kCoefBF16 = 2 };

struct Level {
  int dim = 3;
  int npts = 27;
  int ndof = 1;
  int nreg = 0;
  unsigned mask = 0;   // Dirichlet faces
  int comp[3] = {1, 1, 1};
  int64_t n = 0;       // regional nodes
  int64_t ncomp = 0;   // composite nodes
  std::vector<RegionGeo> regs;
  std::vector<BlockDesc> blocks;
  std::vector<int> region_block;  // [nreg + 1]: first block of each region (blocks are region-major)
  DBuf d_regs, d_blocks;
  std::vector<Tile3> tiles;  // 2.5D tiles of a 3D level (empty in 2D)
  DBuf d_tiles;
  bool use_tiles = false;    // run 27-point stencil operations with the 2.5D kernel
  int tile_depth = 21;       // planes per tile
  int tile_threads = kTileThreadsF64;  // threads per 2.5D tile block (tiles hold at most this many nodes)
  int tile_grid = 0;         // > 0: persistent launch of this many blocks looping over the tiles
  bool rap_separable = true; // scalar 3D geometric Galerkin product as three one-axis products
  bool per_region = false;   // stencil operations launch the node-parallel kernel once per region
  // interface groups: copies of each shared composite node, ascending region order
  int64_t ngroups = 0;
  int64_t ngroups2 = 0;  // the first ngroups2 groups have two copies (groups are ordered by size)
  DBuf d_gptr;    // int64 [ngroups+1]
  DBuf d_gcopy;   // int32 regional node indices
  DBuf d_gcomp;   // int32 composite node index of each group
  // operator (FP64, wave-tiled, ncoef() values per node: npts blocks of ndof x ndof)
  DBuf coef;
  DBuf coef_sym;     // symmetric scalar 27-point levels: the upper half (kSymPts per node), else empty
  // Region tables (FP64 levels run by 768-thread 2.5D tiles, else empty): per region the
  // kClasses x kClassPts couplings of its node classes, and a flag that every node of the region
  // has its class's couplings bit for bit (the couplings the streaming kernel reads: its own upper
  // ones and its neighbours' mirrored ones, 0 towards neighbours outside the region).
  DBuf class_table, class_table_ok;
  // With the tables: the served regions run whole-row tiles that take every coupling from the
  // tables (k_stencil_table), the other regions the level's streaming 2.5D tiles.  Built with the
  // tables (make_split), refreshed when the tiles change.
  std::vector<int> table_served;     // per region: 1 when the tables serve it
  std::vector<Tile3> table_tiles;    // whole-row tiles of the served regions (k_stencil_table)
  std::vector<Tile3> other_tiles;    // the level's 2.5D tiles of the regions not served
  DBuf d_table_tiles, d_other_tiles;
  // Transfers to the next level by rows and planes (make_transfer_tiles; empty: one thread per
  // node).  Restriction tiles hold coarse rows y0 .. y0+ty-1 and planes z0 .. z0+nz-1 of a region
  // (tx = the coarse row length), prolongation tiles fine rows and planes; rtile_vals is the most
  // fine values (nodes times ndof) a restriction tile stages per plane.
  std::vector<Tile3> rtiles, ptiles;  // a prolongation tile's rows reach at most kProlongStageXY coarse nodes a plane
  DBuf d_rtiles, d_ptiles;
  int64_t rtile_vals = 0;
  DBuf dinv;      // double [n * ndof]: 1 / point diagonal of the composite operator
  DBuf dinv9;     // block_diag (3-dof levels): inverse nodal 3 x 3 blocks of D~, double [n][9] row-major
  DBuf dinv9_lo;  // its FP32 copy for the low-precision V-cycle
  DBuf pw;        // stored interpolation weights to the next level, double [n][8] (null: geometric)
  DBuf rw;        // with pw: the same weights per coarse node (125 taps, wave-tiled) for the restriction
  // region-local Gauss-Seidel (smoothers 2-4): the level's stencils and D~^-1 copied into the
  // sweep's hyperplane order ("slots"), so that a wavefront's loads are contiguous
  DBuf gs_rplane;  // int32 [nreg + 1]: first plane of each region in gs_pbase
  DBuf gs_pbase;   // int64: first slot of every plane of every region, then one past the last
  DBuf gs_coef;    // double, wave-tiled by slot: ncoef() values per slot
  DBuf gs_dinv;    // double [slots * ndof]
  DBuf gs_d;       // double [slots * ndof]: the sweep's corrections by slot
  double lambda = 0.0;
  std::vector<double> cheb_c1, cheb_c2;  // per Chebyshev step: direction and residual factors
  // work vectors (regional): b (rhs), u / u2 (ping-pong), d (Chebyshev direction), r (residual)
  DBuf b, u, u2, d, r;
  // low-precision V-cycle copy (FP32 vectors; FP32 or BF16 coefficients)
  int ct_lo = kCoefF64;  // kCoefF64: no copy
  // per-level BF16 decision (RMG_PREC_FP32_BF16_AUTO): factor with every level FP32, with this
  // level BF16; -1 where not tried
  double rho_fp32 = -1.0, rho_bf16 = -1.0;
  DBuf coef_lo;          // float or uint16 (bf16), wave-tiled like coef
  DBuf center_lo;        // bf16 storage only: FP32 centre blocks [n][ndof*ndof]
  DBuf coef_lo_sym;      // FP32 storage of a symmetric level: the upper half, else empty
  DBuf dinv_lo, b32, u32, u232, d32, r32;
  // coarsest level: composite inverse and owner map (nc = composite dofs)
  int nc = 0;
  DBuf ainv;       // double [nc][nc]
  DBuf comp_owner; // int32 [ncomp] regional node index of the owner copy
  DBuf cvec, cvec2;  // double [nc]
  std::vector<double> abar_host;  // dense composite coarse operator (for inspection)

  int ncoef() const { return npts * ndof * ndof; }
  int64_t ndofs() const { return n * ndof; }
  LevelView view() const;
};

}  // namespace rmg

namespace rmg {
// Event-pair timing of selected finest-level kernels (enabled on request).
struct KernelTimer {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t used = 0;
  int64_t count = 0;
  double total_ms = 0.0;
  void acquire(hipEvent_t* e0, hipEvent_t* e1);
  void harvest();  // after a stream synchronisation: accumulate and recycle
  void reset();
  ~KernelTimer();
};
enum TimedKernel { kTimedCheb = 0, kTimedCgQ = 1, kNumTimed = 2 };
}  // namespace rmg

namespace rmg {
struct Hybrid;  // hybrid.cpp
struct Amg;     // amg.cpp
}

struct rmg_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int dim = 0, ndof = 1, nreg = 0;
  unsigned mask = 0;
  std::vector<int32_t> extent, origin;  // finest level, [nreg][3] (2D padded)
  bool have_regions = false, have_operator = false, have_hierarchy = false;
  std::vector<bool> region_set;
  rmg_options opt{};
  std::vector<rmg::Level*> levels;
  // CG work vectors (finest level, regional)
  rmg::DBuf cg_x, cg_r, cg_p, cg_q, cg_z, cg_b, tmp_a, tmp_b;
  rmg::DBuf cg_z32;     // FP32 output of the low-precision V-cycle
  rmg::DBuf partials;   // double partial sums
  rmg::DBuf scalars;    // double device scalars
  double* host_scalars = nullptr;  // pinned
  bool profiling = false;
  std::string autotune_cache;
  std::vector<std::string> tune_report;  // one line per tuned level
  // CG iteration graphs (use_graph): valid for the recorded (b, x) pointers until the next setup
  hipStream_t gstream = nullptr;
  hipGraphExec_t graph_a = nullptr, graph_b = nullptr;
  const void* graph_b_ptr = nullptr;
  const void* graph_x_ptr = nullptr;
  void drop_graphs();
  rmg::KernelTimer timers[rmg::kNumTimed];
  rmg::KernelTimer level_timers[12];  // per region level, reset at the start of every solve
  bool timing_levels = false;         // a solve with profiling on is running
  // finest-level interpolation requested for the next setup (RMG_P_*) and its inputs
  int pmode = 0;
  rmg::DBuf user_pw;             // caller weights, double [n][8]
  std::vector<float> mlp_theta;  // parameters of the learned interpolation
  rmg::DBuf logc;                // float log of the per-element coefficients (diffusion), or empty
  // interpolation of the current hierarchy
  int p_used = 0, p_flags = 0;
  double rho_learned = -1.0, rho_geometric = -1.0;
  // structured/unstructured hybrid: region kinds (0 structured, 1 unstructured) and the hierarchy
  std::vector<int32_t> region_kind;
  rmg::Hybrid* hy = nullptr;
  rmg::Amg* amg = nullptr;  // AMG coarse solver below the region hierarchy (coarse_amg = 1)
  rmg::DevAlloc alloc;     // device memory provider (empty: hipMalloc)
  double setup_ms = 0.0;   // wall time of the last rmg_setup_hierarchy
  ~rmg_handle();
};

namespace rmg {

// api.cpp: select h's device and memory provider for the rest of the current entry point.
void bind_handle(rmg_handle* h);
// api.cpp: Q1 Laplace element matrix of a cube of side h (2x2x2 Gauss-Legendre), corners ax + 2 ay + 4 az.
void q1_laplace_element(double h, double K[64]);

// planner.cpp
void build_level0(rmg_handle* h);
// Coarse region boxes and composite lattice extents of the next level; RMG_ERR_SHAPE when the
// regions' coarse points disagree on an interface.
void coarse_geometry(int dim, const std::vector<RegionGeo>& fine, std::vector<RegionGeo>& coarse, int comp[3]);
Level* make_coarse_level(const Level& fine);
void build_tables(Level& L);
void make_tiles(Level& L, int depth);
// Region-table split of a level whose table flags are `served` (per region): whole-row tiles of the
// served regions and the remaining regions' tiles (also rebuilt by make_tiles while a split exists).
void make_split(Level& L, const std::vector<int>& served);
// Row-and-plane tiles of the transfers between F and the next level C (F.rtiles, F.ptiles), or
// none when `rows` is false or a region's rows are too long for them.
void make_transfer_tiles(Level& F, const Level& C, bool rows);
void clear_split(Level& L);
void build_coarse_solver(rmg_handle* h, Level& L);

// amg.cpp: AMG coarse solver on the coarsest region level's composite operator (Section 3.5).
// amg_setup builds it from L's stencils (L.nc, comp_owner, cvec, cvec2 set as for the direct
// solver); amg_cycle runs one V-cycle z = M^-1 b on composite vectors of L.nc entries.
void amg_setup(rmg_handle* h, Level& L);
void amg_cycle(rmg_handle* h, const double* b, double* z);
void amg_destroy(rmg_handle* h);

// solver.cpp
void setup_hierarchy(rmg_handle* h);
// z = V_level(b) with zero initial guess; z must not be one of the level's work vectors.
// lowp: FP32 vectors and the levels' low-precision operators (b, z are float*), else FP64.
// dot_slot >= 0 (FP64, Chebyshev or Jacobi smoother, not the coarsest level): (b, z) over the
// owned copies, summed by the last smoothing step, goes to that scalar slot.
// start_ready: the level's zero-guess start u_0 = c D~^-1 b is already in its u (written by the CG
// update), so the cycle does not compute it.
void vcycle(rmg_handle* h, int level, bool lowp, const void* b, void* z, int dot_slot = -1, bool start_ready = false);
// z = M^-1 r (one V-cycle in the configured precision); FP64 regional vectors.
void apply_preconditioner(rmg_handle* h, const double* r, double* z);
void pcg(rmg_handle* h, const double* b, double* x, double rtol, int maxit, rmg_solve_info* info,
         rmg_status* st);
// Multigrid as a solver: x <- x + V(b - A x) (regional FP64 vectors).
void mg_solve(rmg_handle* h, const double* b, double* x, double rtol, int maxit, rmg_solve_info* info,
              rmg_status* st);
void smooth_zero_guess(rmg_handle* h, int level, const double* b, double* u_out);
// u <- S(b, u): one degree-K Chebyshev application from the current iterate (tmp: work vector).
void smooth_iterate(rmg_handle* h, int level, const double* b, double* u, double* tmp);
// Convergence factor of `cycles` stationary V-cycles on A x = 0 (FP64 outer iteration).
// work: device memory for 4 n_regional doubles, or nullptr (then allocated for the call).
double convergence_factor(rmg_handle* h, int cycles, double* work = nullptr);

// solver.cpp: finest-level work vectors and launch configuration for the outer CG / MG loop.
void prepare_finest(rmg_handle* h);

// hybrid.cpp: the structured/unstructured hybrid hierarchy (rmg_options.hybrid = 1).
void hybrid_setup(rmg_handle* h);
void hybrid_destroy(rmg_handle* h);
// z = cycle_0(b) with zero initial guess (regional FP64 vectors of the finest level).
void hybrid_cycle(rmg_handle* h, const double* b, double* z);

// learned.cpp
// Stored weights of the finest level for the next coarse level C (caller or learned); returns the
// validity flags (0: valid, weights in F.pw).  Releases F.pw when the interpolation is geometric.
int prepare_stored_weights(rmg_handle* h, Level& F, const Level& C);
int validate_weights(rmg_handle* h, const Level& F, const Level& C);

}  // namespace rmg
