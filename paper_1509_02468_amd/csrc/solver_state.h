// Device-resident solver state (one small struct per solver call).
#pragma once

#include <cstdint>

namespace gsf {

struct CgState {
  double rho;    // r^T r of the current residual (z-space)
  double rho0;
  double res0;
  double floor;  // breakdown floor (tau ||z0||)^2
  double tol;    // requested tolerance (<= 0: run kmax steps)
  double tol2;   // tol^2 rho0, or -1
  double tau;    // breakdown tau of the data precision
  double alpha, beta, pq;
  double rhob[2];  // r^T r by step parity (step k reads rhob[k & 1]; the fused CG kernels)
  int32_t active;
  int32_t status;
  int32_t iters;
  int32_t k;     // 1-based index of the next step
  int32_t pad;
};

// Block CG: one state per column (the columns are independent CG runs that
// share each apply) and whether any column is still running.
struct BlockCgState {
  CgState col[8];
  int32_t m;
  int32_t active;  // some column still active
  int32_t pad[2];
};

struct LobpcgState {
  double theta[8];
  double res[8];       // residual norms of the current X
  double yx[9];        // Y^T W (constraint projection coefficients); the output's X^T z0 and Y^T z0 (m + 1)
  double yz[8];        // Y^T T(R) (learned preconditioner)
  double ynorm_inv;    // 1 / ||sqrt(d)||
  double tol;
  double drop_tol;
  double zero_tol;
  int32_t m;
  int32_t ns;          // columns in the current trial basis (m, 2m or 3m)
  int32_t active;
  int32_t status;
  int32_t iters;
  int32_t dropped;
  int32_t have_p;      // P block valid
  int32_t nkept;       // kept columns of the last Rayleigh-Ritz
  int32_t start_failed;  // the start block had rank < m
  int32_t kept[24];
  int32_t tuse[8];     // column j uses T(r_j) this step (else T = I)
  int32_t fallbacks;   // column-steps that fell back to T = I
  int32_t pad2;
  double cid[64];      // m x m identity coefficients: the residual of a refreshed AX
};

}  // namespace gsf
