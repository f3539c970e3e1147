// Learned interpolation weights: MLP sizes, the cell-node table and the kernel launchers.
#pragma once
#include "internal.h"

namespace rmg {

constexpr int kMlpIn = 27;    // centred log-coefficients of a coarse cell's 3x3x3 fine elements
constexpr int kMlpH = 64;     // two hidden layers (ReLU)
constexpr int kMlpOut = 208;  // one logit per (non-corner fine node, admissible coarse corner)
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;
static_assert(kMlpParams == RMG_MLP_NPARAM, "parameter count");

// A non-corner fine node of a cell: position in the 4x4x4 cell nodes (x fastest), first logit,
// number of coarse corners it interpolates from (2 on an edge, 4 on a face, 8 inside) and their
// slots ix + 2 iy + 4 iz.
struct CellNode {
  int pos, first, ncorner;
  int corner[8];
};

// The 56 non-corner nodes of a cell and, per cell position (x fastest), its node or -1 at corners.
void cell_node_table(CellNode* nodes, signed char* pos2node);

// Z = MLP(X) for n samples; A1, A2 (pre-activations, [n][64]) are stored when non-null.
void mlp_forward(int64_t n, const float* X, const float* theta, float* Z, float* A1, float* A2, hipStream_t st);
// Loss partial sums (one double per block of samples; mlp_loss_partials(n) of them, also the
// returned count) and dZ = dloss/dZ / n.
int64_t mlp_loss_partials(int64_t n);
// kind 0: interpolation error in L2; 1: in the energy norm of the cell's local operator (needs X).
int64_t mlp_loss(int64_t n, const float* Z, const float* E, const float* X, int kind, float* dZ, double* partials,
                 hipStream_t st);
// Activation gradients of the two hidden layers.
void mlp_backact(int64_t n, const float* dZ, const float* A1, const float* A2, const float* theta, float* D1,
                 float* D2, hipStream_t st);
// Weight gradients (flat, parameter order) from the activation gradients; part holds
// mlp_grad_partials() floats.
int64_t mlp_grad_partials();
void mlp_weight_grads(int64_t n, const float* X, const float* A1, const float* A2, const float* dZ, const float* D1,
                      const float* D2, float* grad, float* part, hipStream_t st);
// Adam step t (from 1).
void mlp_adam(float* theta, const float* grad, float* m, float* v, int t, double lr, hipStream_t st);

// Training data and inference inputs of a scalar 3D finest level.  Cells are numbered region by
// region, x fastest; cell_off[k] is region k's first cell (device int64 [nreg + 1]).
void cell_features(const Level& L, const int64_t* cell_off, int64_t ncell, const float* logc, float* X,
                   hipStream_t st);
void cell_targets(const Level& L, const int64_t* cell_off, int64_t ncell, const double* e, float* E, hipStream_t st);
// Stored weights [n][8] of the finest level from logits Z; cellrow maps composite cells to rows of Z.
void learned_weights(const Level& F, const Level& C, const float* Z, const int* cellrow, double* pw, hipStream_t st);
// OR of violation flags of stored weights into *flag (see kWeight* below).
void check_weights(const Level& F, const Level& C, const double* pw, int* flag, hipStream_t st);

enum WeightFlag {
  kWeightNonFinite = 1,   // NaN or Inf
  kWeightSupport = 2,     // weight towards a coarse node off the fine node's face, edge or cell
  kWeightDirichlet = 4,   // free fine node interpolating from a Dirichlet coarse node
  kWeightCopies = 8,      // copies of a shared fine node carry different weights
  kWeightSum = 16,        // weights not summing to one although no Dirichlet weight was dropped
};
static_assert(kWeightNonFinite == RMG_PW_NONFINITE && kWeightSupport == RMG_PW_SUPPORT &&
                  kWeightDirichlet == RMG_PW_DIRICHLET && kWeightCopies == RMG_PW_COPIES && kWeightSum == RMG_PW_SUM,
              "flag values of the C interface");

}  // namespace rmg
