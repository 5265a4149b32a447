// Block linear algebra and solver-state declarations (FP64, N x L row-major).
#pragma once

#include "internal.h"

namespace mbbs {

constexpr int GRAM_MAXPAIR = 3;
constexpr int GRAM_MAXBLK = 1024;
constexpr int COMBO_MAXIN = 4;
constexpr int LMAX_SOLVER = 16;   // keeps the update kernel within 64 KiB of LDS

// Up to three products X_p^H Y_p in one pass; diag[p] = 1 keeps only the
// diagonal (enough for traces and column norms).
struct GramArgs {
  int npair;
  int diag[GRAM_MAXPAIR];
  const double2* X[GRAM_MAXPAIR];
  const double2* Y[GRAM_MAXPAIR];
};
struct GramOut {
  double2* G[GRAM_MAXPAIR];   // L x L results (device)
};

// out = sum_k T_k(in_k): mode 0 identity, 1 complex scalar *coef, 2 right
// multiplication by the L x L matrix coef.
struct ComboArgs {
  int nin;
  int mode[COMBO_MAXIN];
  const double2* in[COMBO_MAXIN];
  const double2* coef[COMBO_MAXIN];
};

// Device-side solver state.
enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXITER = 2, ST_BREAKDOWN = 3 };
struct SolverState {
  int frozen;      // nonzero: every iteration kernel returns at once
  int status;      // ST_*
  int iter;        // iterations started
  int maxiter;
  int reason;      // breakdown: 1 Cholesky, 2 LU pivot, 3 zeta, 4 non-finite residual
  int hist_len;    // entries written to the residual history
  int pad[2];
  double tol2;     // tol^2
};
constexpr int HIST_CAP = 4096;   // residual-history entries kept on the device

// Pointers to every small device array the coefficient kernels touch.
struct SolverDev {
  SolverState* state;
  double* rnorm2;     // ||r_i||^2 (L)
  double* bnorm2;     // ||b_i||^2 (L)
  double2* Gpp;       // P^H P
  double2* Gpp2;      // second CholQR pass Gram
  double2* ginv;      // gamma^{-1}
  double2* RtV;
  double2* RtR;
  double2* RtZ;
  double2* ZT;        // diagonal of Z^H T
  double2* ZZ;        // diagonal of Z^H Z
  double2* lu;        // LU factors of R~^H V
  int* piv;
  double2* alpha;
  double2* nalpha;
  double2* beta;
  double2* C1;        // ginv * beta
  double2* C2;        // -zeta * beta
  double2* zeta;
  double2* nzeta;
  double2* one;       // constant 1 (scalar coefficient)
  double* hist;       // max_i ||r_i||^2/||b_i||^2 after each iteration (HIST_CAP)
  int qr_passes;      // 0: no QR (gamma = 1), 1: Cholesky QR, 2: CholQR2
};

// A batch of systems solved together: every N x L block holds the systems one
// after the other (rows [s N, (s + 1) N) for system s), and every small
// per-system array is repeated per system (L x L matrices every L*L entries,
// length-L vectors every L, scalars and solver states every 1, histories
// every HIST_CAP).  The streaming kernels take the system from blockIdx.y,
// the one-workgroup coefficient kernels from blockIdx.x; a system whose flag
// frozen[s * fstride] is set is skipped.  A single system is n = 1.
struct SysBatch {
  int n = 1;
  int fstride = 0;
};
static_assert(sizeof(SolverState) == SOLVER_FLAG_STRIDE * sizeof(int), "solver state record layout");

// The pointers of system s in a batch laid out as above.
__host__ __device__ inline SolverDev sys_view(SolverDev d, int s, int L) {
  const size_t LL = (size_t)L * L;
  d.state += s;
  d.rnorm2 += (size_t)s * L; d.bnorm2 += (size_t)s * L;
  d.Gpp += s * LL; d.Gpp2 += s * LL; d.ginv += s * LL; d.RtV += s * LL; d.RtR += s * LL; d.RtZ += s * LL;
  d.ZT += s * LL; d.ZZ += s * LL; d.lu += s * LL; d.alpha += s * LL; d.nalpha += s * LL; d.beta += s * LL;
  d.C1 += s * LL; d.C2 += s * LL;
  d.piv += (size_t)s * L;
  d.zeta += s; d.nzeta += s; d.one += s;
  d.hist += (size_t)s * HIST_CAP;
  return d;
}

int gram_blocks(size_t N, int L);
size_t gram_partial_bytes(size_t N, int L, int nsys = 1);
int launch_gram(int L, size_t N, const GramArgs& a, const GramOut& o, double2* partial, const int* frozen,
                hipStream_t st, SysBatch sb = SysBatch());
int launch_combo(int L, size_t N, const ComboArgs& a, double2* out, int gram_mode, const GramOut* o,
                 double2* partial, const int* frozen, hipStream_t st, SysBatch sb = SysBatch());
// which: 0 CholQR factor, 1 second CholQR pass, 2 alpha, 3 zeta/beta; one
// workgroup per system
int launch_coef(int which, int L, const SolverDev& d, hipStream_t st, int nsys = 1);
// Loop test of Alg. 1 on the current ||r_i||^2 (sets frozen and the status
// once it stops the iteration) and the residual-history entry of the
// iteration just finished, per system.
int launch_loop_test(int L, const SolverDev& d, hipStream_t st, int nsys = 1);
// b = a on n_per_sys entries of every system whose flag is clear.
int launch_copy_sys(const double2* a, double2* b, size_t n_per_sys, const int* frozen, hipStream_t st, SysBatch sb);
int launch_fill(double2* p, size_t n, double2 v, hipStream_t st);
int launch_chol_standalone(int L, const double2* G, double2* gam, double2* ginv, int* ok, hipStream_t st);
int launch_matmul_small(int L, const double2* A, const double2* B, double2* C, hipStream_t st);
int launch_lu_standalone(int L, int m, const double2* G, const double2* R, double2* X, int* ok, hipStream_t st);
int launch_copy(const double2* a, double2* b, size_t n, hipStream_t st);

}  // namespace mbbs
