// Argument blocks and launchers of the LOBPCG kernels.
#pragma once

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {

// first-stage split of the Gram partial reduction: the reduction launch sums
// kGramPerChunk partials per chunk, the Rayleigh-Ritz workgroup the chunks
// (4 / 8 / 16 chunks: 9.48-9.50 / 9.38-9.45 / 9.44-9.47 ms per joint CG50 +
// LOBPCG50 call at 1024^2 in alternating runs on one GPU; equal at 4096^2)
constexpr int kGramChunks = 8;
constexpr int kGramDirect = 16;     // at most this many Gram workgroups: no reduction launch
static_assert(kGramChunks <= kGramDirect, "the Rayleigh-Ritz workgroup sums at most kGramDirect values per entry");
// level-2 buffer: kGramChunks x (up to 7 tiles) x 256 chunk sums, then the
// previous update's reduced residual sums (8 values, at kGramFinSlot)
constexpr int kGramFinSlot = kGramChunks * 7 * 256;
constexpr int kGramLevel2Doubles = kGramFinSlot + 32;
// workgroups of the Gram kernel (at most), compared in alternating runs on one
// GPU: 256 / 384 / 512 / 768 / 1024 took 9.63 / 9.55 / 9.41-9.43 / 9.45 /
// 9.46-9.47 ms per joint CG50 + LOBPCG50 call at 1024^2 and 2.76 / 2.87 /
// 2.73-2.76 / 2.73-2.75 / 2.84-2.85 ms per LOBPCG step at 4096^2, m = 8
constexpr int kGramBlocks = 512;
constexpr int kGramPerChunk = kGramBlocks / kGramChunks;  // partials per chunk

struct LobArgs {
  int prec;
  int64_t n, rows, cols;
  int ndim, m, constraint;
  const void* x0;
  const void* sqd;
  void *X, *W, *P, *AX, *AW, *AP;
  const double* C;     // ns x m coefficients of the last Rayleigh-Ritz step
  double* vpart;       // per-workgroup partial sums
  LobpcgState* st;
  void* xout;
  void* ritz;          // nullable
};

struct StartDegrees {
  int a[8];  // row (2D) degree of phi_j
  int b[8];  // column / sample degree of phi_j
};

struct GramArgs {
  const void* S[3];
  const void* AS[3];
  int ns, m;
  int64_t n;
  int nparts;          // workgroups of the Gram kernel
  double* partials;    // nparts x tiles x 256
  double* level2;      // kGramChunks x tiles x 256
  const int* active;   // nullable
};

struct RRArgs {
  double* C;
  double* theta;
  LobpcgState* st;     // nullable
  double drop_tol, zero_tol;
  // nullable: per-workgroup partials of the previous update (stride values
  // per workgroup, residual norms first) to finalize before the Rayleigh-Ritz
  // step, in place of a separate finalize launch (no constraint)
  const double* fin_partials;
  int fin_nparts, fin_stride;
  double* gram_out;    // nullable: GA then GB (ns x ns)
  int* kept_out;       // nullable
  int* nkept_out;      // nullable
  int init;            // 1 for the start-block Rayleigh-Ritz
};

int gram_tiles_total(int ns);
gsf_status lob_launch_ynorm(const LobArgs& a, int nb, hipStream_t s);
struct CgStepArgs;
// which: 0 start block, 1 update + finalize, 2 output dots, 3 output,
// 4 update without the finalize (see RRArgs::fin_partials), 5 the finalize alone,
// 6 / 7 the residual of a recomputed AX with / without the finalize (a.C = I).
// cg_direction (nullable, same precision; which = 1 or 4 only): a CG
// direction phase run as extra workgroups of the update launch (the joint
// CG + LOBPCG driver).
gsf_status lob_launch_mkernel(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg,
                              hipStream_t s, const CgStepArgs* cg_direction = nullptr);
gsf_status lob_launch_project(const LobArgs& a, void* B, int nb, hipStream_t s);
// Gram partials, their reduction and the Rayleigh-Ritz step.  cg_update
// (nullable): a CG update phase run as extra workgroups of the Rayleigh-Ritz
// launch (the joint CG + LOBPCG driver).
gsf_status lob_launch_gram(const GramArgs& g, const RRArgs& r, int prec, hipStream_t s,
                           const CgStepArgs* cg_update = nullptr);
gsf_status lob_launch_rr_only(const double* G, int ns, int m, const RRArgs& r, hipStream_t s);
gsf_status launch_lob_state_init(LobpcgState* dst, const LobpcgState& v, hipStream_t s);
gsf_status launch_cg_state_init(CgState* dst, const CgState& v, hipStream_t s);

}  // namespace gsf
