// AMG coarse solver below the region hierarchy (Section 3.5, rmg_options.coarse_amg): host levels
// built by amg.cpp and the device arrays the kernels of kernels_amg.hip read.
#pragma once

#include <memory>
#include <vector>

#include "internal.h"

namespace rmg {

// Host matrix in CSR, ascending columns.
struct Csr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// Device matrix.  Short rows (at most 32 entries on average): ELL slices of 64 rows, the e-th
// stored entry of row i at sptr[i / 64] + 64 e + i % 64, e < (sptr[i / 64 + 1] - sptr[i / 64]) / 64,
// padding entries with a valid column and value 0; one thread per row.  Long rows (wave): CSR
// (sptr = row pointers), one wavefront per row, its lanes reading the row contiguously.
struct SpDev {
  int64_t n = 0;
  bool wave = false;
  DBuf sptr, col, val;
};

struct AmgLevel {
  Csr A;                     // composite matrix of this level
  Csr P;                     // smoothed prolongator to the next level (empty on the last level)
  std::vector<int32_t> agg;  // aggregate of every row, -1 if none
  double rho = 0.0;          // Gershgorin bound on lambda_max(D^-1 A)
  double omega = 0.0;        // prolongator smoothing weight 4 / (3 rho)
  // device
  SpDev dA, dP, dPt;
  DBuf dinv, b, u, r, d, y;
  double inv_theta = 0.0;      // Chebyshev: first correction (1/theta) D^-1 r
  std::vector<double> c1, c2;  // Chebyshev step k >= 1: d = c1[k] d + c2[k] D^-1 r
  int nc = 0;                  // last level: rows of the dense inverse
  DBuf ainv;
};

struct Amg {
  std::vector<std::unique_ptr<AmgLevel>> lv;
};

// ---- kernels_amg.hip
// y = M x, or y += M x when accumulate.
void launch_sp_apply(const SpDev& M, const double* x, double* y, bool accumulate, hipStream_t st);
// d = inv_theta D^-1 r; u = d (zero) or u += d.
void launch_amg_cheb_first(int64_t n, double inv_theta, const double* dinv, const double* r, double* d, double* u,
                           bool zero, hipStream_t st);
// d = c1 d + c2 D^-1 (b - y); u += d.
void launch_amg_cheb_step(int64_t n, double c1, double c2, const double* dinv, const double* b, const double* y,
                          double* d, double* u, hipStream_t st);
// r = b - y.
void launch_amg_sub(int64_t n, const double* b, const double* y, double* r, hipStream_t st);

}  // namespace rmg
