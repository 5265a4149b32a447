// Modified block BiCGSTAB (Alg. 1, and the memory-saving Alg. 2) driven from
// the host with every coefficient computed on the device: the host only
// enqueues iterations (optionally captured in a HIP graph of k iterations)
// and reads a small state record after each batch.  The loop test of Alg. 1
// (continue while max_i ||r_i||/||b_i|| > tol) runs on the device on R_0 and
// after step 4.10 of each iteration, where the new residual norms are formed;
// once it fails, the device sets `frozen`, step 4.12 and every later kernel of
// the batch return at once, and the host sees the stop after the iteration
// that caused it.  After the recursive residual converges, the true residual
// B - A X is checked in FP64 and the iteration restarts from it if needed.
//
// A batch handle (several same-shape systems stacked along t) runs the same
// iteration for all of its systems in every launch: each system has its own
// state record, coefficients and flag, a stopped system is skipped by every
// kernel, and the host takes the true-residual and restart decisions per
// system once every system of the batch has stopped.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "blas.h"

namespace mbbs {

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Work {
  // FP64 N x L blocks of every system (Bp: the right-hand side times
  // (1 + T)^{-1} with clover)
  double2 *R, *P, *Rt, *V, *T, *Z, *U, *S, *Bp;
  SapBuffers sap;
  double2* partial;
  SolverDev d;
  double* trnorm2;   // true residual norms^2 (nsys x L)
  double2* mone;     // constant -1 (nsys)
};

// Per-system small arrays, laid out as sys_view expects.
size_t small_bytes(int L, int nsys) {
  const size_t LL = (size_t)L * L * sizeof(double2) * nsys;
  const size_t vec = (size_t)L * sizeof(double) * nsys;
  return al(sizeof(SolverState) * nsys) + 3 * al(vec) + 16 * al(LL) + al((size_t)L * sizeof(int) * nsys) +
         4 * al(sizeof(double2) * nsys) + al((size_t)HIST_CAP * sizeof(double) * nsys);
}

size_t block_bytes(const mbbs_lattice_s* lat, int L) { return al((size_t)lat->g.V * 12 * L * sizeof(double2)); }

int nblocks_needed(const mbbs_solve_params& p) {
  // R, P, Rt, V, Z, U always; T unless memsave; S only with a preconditioner
  int n = 6;
  if (!p.memsave) n += 1;
  if (p.precond) n += 1;
  return n;
}
int nblocks_needed(const mbbs_lattice_s* lat, const mbbs_solve_params& p) {
  return nblocks_needed(p) + (lat->gk.clov ? 1 : 0);
}

size_t rows_per_system(const mbbs_lattice_s* lat) { return (size_t)(lat->g.V / lat->nsys) * 12; }

size_t workspace_bytes(const mbbs_lattice_s* lat, int L, const mbbs_solve_params& p) {
  size_t b = nblocks_needed(lat, p) * block_bytes(lat, L);
  if (p.precond) b += al(sap_buffer_bytes(lat, L, p.sap_prec, p.domain_solver == 1));
  b += al(gram_partial_bytes(rows_per_system(lat), L, lat->nsys));
  b += small_bytes(L, lat->nsys);
  return b;
}

int bind(const mbbs_lattice_s* lat, int L, const mbbs_solve_params& p, void* ws, size_t bytes, Work& w) {
  MBBS_CHECK(ws != nullptr && bytes >= workspace_bytes(lat, L, p), "solver workspace too small");
  char* q = (char*)ws;
  const size_t B = block_bytes(lat, L);
  const int ns = lat->nsys;
  auto take = [&](size_t n) { char* r = q; q += al(n); return r; };
  w.R = (double2*)take(B);
  w.P = (double2*)take(B);
  w.Rt = (double2*)take(B);
  w.V = (double2*)take(B);
  w.Z = (double2*)take(B);
  w.U = (double2*)take(B);
  w.T = p.memsave ? w.R : (double2*)take(B);
  w.S = p.precond ? (double2*)take(B) : w.T;
  w.Bp = lat->gk.clov ? (double2*)take(B) : nullptr;
  if (p.precond) {
    const bool ssor = p.domain_solver == 1;
    const size_t sb = sap_buffer_bytes(lat, L, p.sap_prec, ssor);
    MBBS_TRY(sap_bind(lat, L, p.sap_prec, take(sb), sb, &w.sap, ssor));
    w.sap.nssor = p.nssor;
    w.sap.ssor_omega = p.ssor_omega;
  }
  w.partial = (double2*)take(gram_partial_bytes(rows_per_system(lat), L, ns));
  const size_t LL = (size_t)L * L * sizeof(double2) * ns;
  const size_t vec = (size_t)L * sizeof(double) * ns;
  SolverDev& d = w.d;
  d.state = (SolverState*)take(sizeof(SolverState) * ns);
  d.rnorm2 = (double*)take(vec);
  d.bnorm2 = (double*)take(vec);
  w.trnorm2 = (double*)take(vec);
  d.Gpp = (double2*)take(LL);
  d.Gpp2 = (double2*)take(LL);
  d.ginv = (double2*)take(LL);
  d.RtV = (double2*)take(LL);
  d.RtR = (double2*)take(LL);
  d.RtZ = (double2*)take(LL);
  d.ZT = (double2*)take(LL);
  d.ZZ = (double2*)take(LL);
  d.lu = (double2*)take(LL);
  d.alpha = (double2*)take(LL);
  d.nalpha = (double2*)take(LL);
  d.beta = (double2*)take(LL);
  d.C1 = (double2*)take(LL);
  d.C2 = (double2*)take(LL);
  take(LL);
  take(LL);
  d.piv = (int*)take((size_t)L * sizeof(int) * ns);
  d.zeta = (double2*)take(sizeof(double2) * ns);
  d.nzeta = (double2*)take(sizeof(double2) * ns);
  d.one = (double2*)take(sizeof(double2) * ns);
  w.mone = (double2*)take(sizeof(double2) * ns);
  d.hist = (double*)take((size_t)HIST_CAP * sizeof(double) * ns);
  d.qr_passes = p.qr_passes;
  return MBBS_OK;
}

// Column norms^2 of a block through a diagonal Gram product into dst (L doubles
// per system as the real parts of the diagonal, gathered by a tiny kernel).
__global__ void k_diag_real(int L, const double2* __restrict__ G, double* __restrict__ out, const int* frozen,
                            int fstride) {
  const int sys = blockIdx.x;
  if (frozen && frozen[sys * fstride]) return;
  for (int i = threadIdx.x; i < L; i += blockDim.x) out[(size_t)sys * L + i] = G[(size_t)sys * L * L + i * L + i].x;
}

struct Ctx {
  const mbbs_lattice_s* lat;
  int L;
  int nsys;
  size_t N;          // rows per system
  size_t NL;         // complex entries of one stacked N x L block (all systems)
  SysBatch sb;
  mbbs_solve_params p;
  Work w;
  const double2* B;
  double2* X;
  hipStream_t st;
  Profiler* prof;
  const int* frozen;  // first system's flag; the others follow at sb.fstride
};

int col_norms(Ctx& c, const double2* A, double* out, const int* frozen) {
  GramArgs g{};
  g.npair = 1;
  g.diag[0] = 1;
  g.X[0] = A;
  g.Y[0] = A;
  GramOut o{};
  o.G[0] = c.w.d.Gpp2;  // scratch L x L per system
  if (c.prof) c.prof->begin(MBBS_K_GRAM);
  MBBS_TRY(launch_gram(c.L, c.N, g, o, c.w.partial, frozen, c.st, c.sb));
  hipLaunchKernelGGL(k_diag_real, dim3(c.nsys), dim3(64), 0, c.st, c.L, (const double2*)c.w.d.Gpp2, out, frozen,
                     c.sb.fstride);
  if (c.prof) c.prof->end();
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

// A applied in FP64 to every system whose flag (if given) is clear.
int dslash64(Ctx& c, const double2* in, double2* out, const int* frozen) {
  if (c.prof) c.prof->begin(MBBS_K_DSLASH64);
  int rc = launch_dslash(c.lat, c.L, P64, P64, LEX, false, in, nullptr, out, nullptr, 0, c.lat->g.V, frozen, c.st);
  if (c.prof) c.prof->end();
  return rc;
}

int combo(Ctx& c, ComboArgs a, double2* out, int gm, double2* gout, const int* frozen) {
  GramOut o{};
  o.G[0] = gout;
  if (c.prof) c.prof->begin(gm ? MBBS_K_GRAM : MBBS_K_UPDATE);
  int rc = launch_combo(c.L, c.N, a, out, gm, &o, c.w.partial, frozen, c.st, c.sb);
  if (c.prof) c.prof->end();
  return rc;
}

int gram(Ctx& c, const GramArgs& g, const GramOut& o, const int* frozen) {
  if (c.prof) c.prof->begin(MBBS_K_GRAM);
  int rc = launch_gram(c.L, c.N, g, o, c.w.partial, frozen, c.st, c.sb);
  if (c.prof) c.prof->end();
  return rc;
}

int precondition(Ctx& c, const double2* in, const double2* gam, double2* out) {
  if (c.p.precond) return sap_apply(c.lat, c.w.sap, c.p.ncy, c.p.nmr, in, gam, out, c.frozen, c.st, c.prof);
  // M = 1: out = in * gam (gam may be null only when out aliases in)
  if (gam == nullptr) return MBBS_OK;
  ComboArgs a{};
  a.nin = 1;
  a.mode[0] = 2; a.in[0] = in; a.coef[0] = gam;
  return combo(c, a, out, 0, nullptr, c.frozen);
}

int coef(Ctx& c, int which) {
  if (c.prof) c.prof->begin(MBBS_K_SMALL);
  int rc = launch_coef(which, c.L, c.w.d, c.st, c.nsys);
  if (c.prof) c.prof->end();
  return rc;
}

// One iteration of Alg. 1 (or Alg. 2), every step on the device.
int enqueue_iteration(Ctx& c) {
  Work& w = c.w;
  SolverDev& d = w.d;
  const int* fz = c.frozen;
  // 4.1 (Cholesky QR factor of P, folded into the consumers)
  MBBS_TRY(coef(c, 0));
  if (c.p.qr_passes == 2) {
    ComboArgs a{};
    a.nin = 1; a.mode[0] = 2; a.in[0] = w.P; a.coef[0] = d.ginv;
    MBBS_TRY(combo(c, a, w.U, 2, d.Gpp2, fz));
    MBBS_TRY(coef(c, 1));
  }
  // 4.2 U = M (P gamma^{-1});  4.3 V = A U
  MBBS_TRY(precondition(c, w.P, d.ginv, w.U));
  MBBS_TRY(dslash64(c, w.U, w.V, fz));
  // 4.4 alpha from R~^H V and R~^H R
  {
    GramArgs g{};
    g.npair = 2;
    g.X[0] = w.Rt; g.Y[0] = w.V;
    g.X[1] = w.Rt; g.Y[1] = w.R;
    GramOut o{};
    o.G[0] = d.RtV; o.G[1] = d.RtR;
    MBBS_TRY(gram(c, g, o, fz));
  }
  MBBS_TRY(coef(c, 2));
  // 4.5 T = R - V alpha   (Alg. 2: R <- R - V alpha, X <- X + U alpha)
  {
    ComboArgs a{};
    a.nin = 2;
    a.mode[0] = 0; a.in[0] = w.R;
    a.mode[1] = 2; a.in[1] = w.V; a.coef[1] = d.nalpha;
    MBBS_TRY(combo(c, a, w.T, 0, nullptr, fz));
  }
  if (c.p.memsave) {
    ComboArgs a{};
    a.nin = 2;
    a.mode[0] = 0; a.in[0] = c.X;
    a.mode[1] = 2; a.in[1] = w.U; a.coef[1] = d.alpha;
    MBBS_TRY(combo(c, a, c.X, 0, nullptr, fz));
  }
  // 4.6 S = M T;  4.7 Z = A S
  if (c.p.precond) MBBS_TRY(precondition(c, w.T, nullptr, w.S));
  MBBS_TRY(dslash64(c, w.S, w.Z, fz));
  // 4.8 / 4.11: R~^H Z, Tr(Z^H T), Tr(Z^H Z)
  {
    GramArgs g{};
    g.npair = 3;
    g.X[0] = w.Rt; g.Y[0] = w.Z;
    g.diag[1] = 1; g.X[1] = w.Z; g.Y[1] = w.T;
    g.diag[2] = 1; g.X[2] = w.Z; g.Y[2] = w.Z;
    GramOut o{};
    o.G[0] = d.RtZ; o.G[1] = d.ZT; o.G[2] = d.ZZ;
    MBBS_TRY(gram(c, g, o, fz));
  }
  MBBS_TRY(coef(c, 3));
  // 4.9 X <- X + U alpha + zeta S   (Alg. 2: X <- X + zeta S)
  {
    ComboArgs a{};
    a.nin = c.p.memsave ? 2 : 3;
    a.mode[0] = 0; a.in[0] = c.X;
    a.mode[1] = 1; a.in[1] = w.S; a.coef[1] = d.zeta;
    if (!c.p.memsave) { a.mode[2] = 2; a.in[2] = w.U; a.coef[2] = d.alpha; }
    MBBS_TRY(combo(c, a, c.X, 0, nullptr, fz));
  }
  // 4.10 R = T - zeta Z, with ||r_i||^2 for the loop test
  {
    ComboArgs a{};
    a.nin = 2;
    a.mode[0] = 0; a.in[0] = w.T;
    a.mode[1] = 1; a.in[1] = w.Z; a.coef[1] = d.nzeta;
    MBBS_TRY(combo(c, a, w.R, 1, d.Gpp2, fz));
    if (c.prof) c.prof->begin(MBBS_K_SMALL);
    hipLaunchKernelGGL(k_diag_real, dim3(c.nsys), dim3(64), 0, c.st, c.L, (const double2*)d.Gpp2, d.rnorm2, fz,
                       c.sb.fstride);
    MBBS_HIP(hipGetLastError());
    // loop test on the new residual: a stop skips step 4.12
    MBBS_TRY(launch_loop_test(c.L, d, c.st, c.nsys));
    if (c.prof) c.prof->end();
  }
  // 4.12 P <- R + (Q - zeta V) beta = R + P (gamma^{-1} beta) - V (zeta beta), with P^H P
  {
    ComboArgs a{};
    a.nin = 3;
    a.mode[0] = 0; a.in[0] = w.R;
    a.mode[1] = 2; a.in[1] = w.P; a.coef[1] = d.C1;
    a.mode[2] = 2; a.in[2] = w.V; a.coef[2] = d.C2;
    MBBS_TRY(combo(c, a, w.P, 2, d.Gpp, fz));
  }
  return MBBS_OK;
}

// R = B - A X (or B when X = 0), P = R, R~ (= R unless given), the norms of
// R and P^H P, for every system whose flag is clear (the others keep theirs).
int start(Ctx& c, bool x_zero, bool set_rt) {
  Work& w = c.w;
  const int* fz = c.frozen;
  if (x_zero) {
    MBBS_TRY(launch_copy_sys(c.B, w.R, c.N * c.L, fz, c.st, c.sb));
  } else {
    MBBS_TRY(dslash64(c, c.X, w.V, fz));
    ComboArgs a{};
    a.nin = 2;
    a.mode[0] = 0; a.in[0] = c.B;
    a.mode[1] = 1; a.in[1] = w.V; a.coef[1] = w.mone;
    MBBS_TRY(combo(c, a, w.R, 0, nullptr, fz));
  }
  MBBS_TRY(launch_copy_sys(w.R, w.P, c.N * c.L, fz, c.st, c.sb));
  if (set_rt)
    MBBS_TRY(launch_copy_sys(c.p.rtilde ? (const double2*)c.p.rtilde : w.R, w.Rt, c.N * c.L, fz, c.st, c.sb));
  MBBS_TRY(col_norms(c, w.R, w.d.rnorm2, fz));
  {
    GramArgs g{};
    g.npair = 1;
    g.X[0] = w.P; g.Y[0] = w.P;
    GramOut o{};
    o.G[0] = w.d.Gpp;
    MBBS_TRY(gram(c, g, o, fz));
  }
  return MBBS_OK;
}

// True residual T = B - A X and its column norms, every system.
int true_residual(Ctx& c) {
  Work& w = c.w;
  double2* t = w.T == w.R ? w.Z : w.T;
  MBBS_TRY(dslash64(c, c.X, w.V, nullptr));
  ComboArgs a{};
  a.nin = 2;
  a.mode[0] = 0; a.in[0] = c.B;
  a.mode[1] = 1; a.in[1] = w.V; a.coef[1] = w.mone;
  MBBS_TRY(combo(c, a, t, 0, nullptr, nullptr));
  MBBS_TRY(col_norms(c, t, w.trnorm2, nullptr));
  return MBBS_OK;
}

}  // namespace

// Host-visible parts of one (batch of) systems' solve, shared with the
// batched driver.  Per-system vectors have nsys entries.
struct SolveJob {
  Ctx c;
  std::vector<SolverState> hs;   // last state records read back
  std::vector<int> restarts, rc;
  std::vector<char> done;
  std::vector<long long> n_outer;
  int ndone = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void init(int n) {
    hs.assign(n, SolverState{});
    restarts.assign(n, 0);
    rc.assign(n, MBBS_OK);
    done.assign(n, 0);
    n_outer.assign(n, 0);
    ndone = 0;
  }
  void finish(int s, int code) {
    if (done[s]) return;
    done[s] = 1;
    rc[s] = code;
    ++ndone;
  }
};

// Copy device memory to the host in stream order (the caller's stream may be
// non-blocking with respect to the legacy default stream).
static int read_dev(Ctx& c, void* dst, const void* src, size_t n) {
  MBBS_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c.st));
  MBBS_HIP(hipStreamSynchronize(c.st));
  return MBBS_OK;
}

static SolverState fresh_state(const Ctx& c, bool stopped) {
  SolverState s{};
  s.maxiter = c.p.maxiter;
  s.tol2 = c.p.tol * c.p.tol;
  s.frozen = stopped ? 1 : 0;
  s.status = ST_RUNNING;
  return s;
}

// Per-system validity of B (a zero or non-finite column is rejected).
static bool bad_rhs(const double* bn, int L, int* col) {
  for (int i = 0; i < L; ++i)
    if (!(bn[i] > 0) || !std::isfinite(bn[i])) { *col = i; return true; }
  return false;
}

static int job_init(SolveJob& j) {
  Ctx& c = j.c;
  const int ns = c.nsys;
  MBBS_TRY(launch_fill(c.w.d.one, ns, make_double2(1, 0), c.st));
  MBBS_TRY(launch_fill(c.w.mone, ns, make_double2(-1, 0), c.st));
  if (!c.p.x0_is_guess) MBBS_TRY(launch_fill(c.X, c.NL, make_double2(0, 0), c.st));
  // ||b_i||^2 of every system
  MBBS_TRY(col_norms(c, c.B, c.w.d.bnorm2, nullptr));
  std::vector<double> bn((size_t)ns * c.L);
  MBBS_TRY(read_dev(c, bn.data(), c.w.d.bnorm2, bn.size() * sizeof(double)));
  std::vector<SolverState> s(ns);
  for (int k = 0; k < ns; ++k) {
    int col = 0;
    const bool bad = bad_rhs(&bn[(size_t)k * c.L], c.L, &col);
    if (bad) {
      set_error("right-hand side column " + std::to_string(col) + (ns > 1 ? " of system " + std::to_string(k) : "") +
                (bn[(size_t)k * c.L + col] > 0 ? " is not finite" : " is zero"));
      j.finish(k, MBBS_EINVAL);
    }
    s[k] = fresh_state(c, bad);
  }
  if (j.ndone == ns) return MBBS_EINVAL;
  MBBS_HIP(hipMemcpyAsync(c.w.d.state, s.data(), sizeof(SolverState) * ns, hipMemcpyHostToDevice, c.st));
  MBBS_TRY(start(c, !c.p.x0_is_guess, true));
  for (int k = 0; k < ns; ++k)
    if (!j.done[k]) j.n_outer[k] += c.p.x0_is_guess ? 1 : 0;
  MBBS_TRY(launch_loop_test(c.L, c.w.d, c.st, ns));   // R_0 may already satisfy the test
  MBBS_HIP(hipStreamSynchronize(c.st));
  return MBBS_OK;
}

// Host decision once every system has stopped: the true residual of each
// system still open decides success, failure or a restart from it.
// *restarted receives the number of systems restarted (their records in
// j.hs are reset to running).
static int decide(SolveJob& j, const double* tn, const double* bn, int* restarted) {
  Ctx& c = j.c;
  const int ns = c.nsys;
  std::vector<SolverState> s = j.hs;
  int nr = 0;
  for (int k = 0; k < ns; ++k) {
    if (j.done[k]) continue;
    j.n_outer[k] += 1;
    double worst = 0;
    bool finite = true;
    for (int i = 0; i < c.L; ++i) {
      const double r = tn[(size_t)k * c.L + i] / bn[(size_t)k * c.L + i];
      finite = finite && std::isfinite(r);
      worst = std::max(worst, r);
    }
    const bool ok = finite && worst <= c.p.tol * c.p.tol;
    const SolverState& h = j.hs[k];
    if (h.status == ST_BREAKDOWN) {
      if (!ok) set_error("block BiCGSTAB breakdown (" +
                         std::string(h.reason == 1 ? "P^H P not positive definite" :
                                     h.reason == 2 ? "singular R~^H V" :
                                     h.reason == 4 ? "non-finite residual" : "non-finite zeta") + ")" +
                         (ns > 1 ? " in system " + std::to_string(k) : ""));
      j.finish(k, ok ? MBBS_OK : MBBS_EBREAKDOWN);
    } else if (ok) {
      j.finish(k, MBBS_OK);
    } else if (h.status == ST_MAXITER || j.restarts[k] >= c.p.max_restarts || h.iter >= c.p.maxiter) {
      j.finish(k, MBBS_NOT_CONVERGED);
    } else {
      // restart from the true residual: R = B - A X, P = R, keep R~
      j.restarts[k] += 1;
      j.n_outer[k] += 1;
      s[k].frozen = 0;
      s[k].status = ST_RUNNING;
      ++nr;
    }
  }
  *restarted = nr;
  if (nr) j.hs = s;
  return MBBS_OK;
}

// After a batch of iterations: read the states; once every system has
// stopped, check the true residuals and restart the systems that need it.
static int job_check(SolveJob& j) {
  Ctx& c = j.c;
  const int ns = c.nsys;
  MBBS_TRY(read_dev(c, j.hs.data(), c.w.d.state, sizeof(SolverState) * ns));
  for (int k = 0; k < ns; ++k)
    if (!j.hs[k].frozen) return MBBS_OK;
  MBBS_TRY(true_residual(c));
  std::vector<double> tn((size_t)ns * c.L), bn((size_t)ns * c.L);
  MBBS_TRY(read_dev(c, tn.data(), c.w.trnorm2, tn.size() * sizeof(double)));
  MBBS_TRY(read_dev(c, bn.data(), c.w.d.bnorm2, bn.size() * sizeof(double)));
  int nr = 0;
  MBBS_TRY(decide(j, tn.data(), bn.data(), &nr));
  if (nr == 0) return MBBS_OK;
  MBBS_HIP(hipMemcpyAsync(c.w.d.state, j.hs.data(), sizeof(SolverState) * ns, hipMemcpyHostToDevice, c.st));
  MBBS_TRY(start(c, false, false));
  MBBS_HIP(hipStreamSynchronize(c.st));
  return MBBS_OK;
}

static int job_enqueue(SolveJob& j, int k) {
  for (int i = 0; i < k; ++i) MBBS_TRY(enqueue_iteration(j.c));
  return MBBS_OK;
}

// Per-system result records (info has nsys entries).
static void job_fill_info(SolveJob& j, mbbs_solve_info* info, double seconds) {
  if (!info) return;
  Ctx& c = j.c;
  const int ns = c.nsys;
  std::vector<double> tn((size_t)ns * c.L), rn((size_t)ns * c.L), bn((size_t)ns * c.L);
  const bool norms = read_dev(c, tn.data(), c.w.trnorm2, tn.size() * sizeof(double)) == MBBS_OK &&
                     read_dev(c, rn.data(), c.w.d.rnorm2, rn.size() * sizeof(double)) == MBBS_OK &&
                     read_dev(c, bn.data(), c.w.d.bnorm2, bn.size() * sizeof(double)) == MBBS_OK;
  for (int k = 0; k < ns; ++k) {
    mbbs_solve_info* in = info + k;
    in->status = j.rc[k];
    in->iterations = j.hs[k].iter;
    in->restarts = j.restarts[k];
    in->n_dslash_outer = 2ll * j.hs[k].iter + j.n_outer[k];
    in->n_sap = c.p.precond ? 2ll * j.hs[k].iter : 0;
    in->seconds = seconds;
    if (norms) {
      for (int i = 0; i < c.L; ++i) {
        const size_t e = (size_t)k * c.L + i;
        if (in->true_res) in->true_res[i] = std::sqrt(tn[e] / bn[e]);
        if (in->rec_res) in->rec_res[i] = std::sqrt(rn[e] / bn[e]);
      }
    }
    if (c.prof) {
      for (int q = 0; q < MBBS_K_COUNT; ++q) {
        in->kernel_ms[q] = c.prof->ms[q];
        in->kernel_launches[q] = c.prof->launches[q];
      }
    }
    in->history_len = 0;
    const int nh = std::min(std::min(j.hs[k].hist_len, HIST_CAP), in->history_cap);
    if (in->res_history && nh > 0) {
      std::vector<double> h(nh);
      if (read_dev(c, h.data(), c.w.d.hist + (size_t)k * HIST_CAP, nh * sizeof(double)) == MBBS_OK) {
        for (int i = 0; i < nh; ++i) in->res_history[i] = std::sqrt(h[i]);
        in->history_len = nh;
      }
    }
  }
}

static int validate(const mbbs_lattice_s* lat, int L, const mbbs_solve_params* p) {
  MBBS_CHECK(lat != nullptr && p != nullptr, "null argument");
  MBBS_CHECK(L >= 1 && L <= LMAX_SOLVER, "L must be in 1..16 for the solver");
  MBBS_CHECK(p->tol > 0 && std::isfinite(p->tol), "tol must be positive");
  MBBS_CHECK(p->maxiter >= 0, "maxiter must be >= 0");
  MBBS_CHECK(p->qr_passes >= 0 && p->qr_passes <= 2, "qr_passes must be 0 (no QR), 1 or 2");
  MBBS_CHECK(p->sap_prec >= 0 && p->sap_prec <= 2, "bad sap_prec");
  if (p->precond) {
    MBBS_CHECK(p->domain_solver == 0 || p->domain_solver == 1, "domain_solver must be 0 (MR) or 1 (SSOR)");
    MBBS_CHECK(p->ncy >= 1, "SAP needs ncy >= 1");
    if (p->domain_solver == 0) MBBS_CHECK(p->nmr >= 1, "MR domain solves need nmr >= 1");
    else {
      MBBS_CHECK(p->nssor == 0 || p->nssor == 1, "N_SSOR must be 0 or 1");
      MBBS_CHECK(std::isfinite(p->ssor_omega) && p->ssor_omega > 0 && p->ssor_omega < 2,
                 "SSOR omega must lie in (0, 2)");
    }
  }
  return MBBS_OK;
}

static void ctx_setup(Ctx& c, const mbbs_lattice_s* lat, int L, const mbbs_solve_params& p, const double* B,
                      double* X) {
  c.lat = lat;
  c.L = L;
  c.nsys = lat->nsys;
  c.N = rows_per_system(lat);
  c.NL = (size_t)lat->g.V * 12 * L;
  c.sb.n = lat->nsys;
  c.sb.fstride = SOLVER_FLAG_STRIDE;
  c.p = p;
  c.B = (const double2*)B;
  c.X = (double2*)X;
  c.prof = nullptr;
}

static int solve_impl(mbbs_lattice_t lat, int L, const double* B_dev, double* X_dev, const mbbs_solve_params* params,
                      void* ws, size_t ws_bytes, mbbs_solve_info* info, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  MBBS_TRY(validate(lat, L, params));
  MBBS_CHECK(B_dev && X_dev && B_dev != X_dev, "B and X must be distinct device blocks");
  SolveJob j;
  Ctx& c = j.c;
  ctx_setup(c, lat, L, *params, B_dev, X_dev);
  j.init(c.nsys);
  c.st = (hipStream_t)stream;
  Profiler prof;
  MBBS_TRY(bind(lat, L, c.p, ws, ws_bytes, c.w));
  c.frozen = &c.w.d.state->frozen;
  if (c.w.Bp) {   // clover: solve A X = (1 + T)^{-1} B
    MBBS_TRY(launch_clover_apply(lat, L, c.B, c.w.Bp, c.st));
    c.B = c.w.Bp;
  }
  if (c.p.profile) {
    prof.on = true;
    prof.st = c.st;
    for (int i = 0; i < 2 * Profiler::CAP; ++i) (void)hipEventCreate(&prof.ev[i]);
    c.prof = &prof;
  }
  int rc = job_init(j);
  const int k = std::max(1, c.p.graph_iters);
  const bool use_graph = c.p.graph_iters > 1 && c.st != nullptr && !c.p.profile;
  while (rc == MBBS_OK && j.ndone < c.nsys) {
    if (use_graph) {
      if (!j.exec) {
        if (hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal) != hipSuccess) { rc = MBBS_EHIP; break; }
        int erc = job_enqueue(j, k);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c.st, &g);
        if (erc < 0 || e != hipSuccess) { rc = erc < 0 ? erc : MBBS_EHIP; set_error("graph capture failed"); break; }
        j.graph = g;
        if (hipGraphInstantiate(&j.exec, g, nullptr, nullptr, 0) != hipSuccess) {
          set_error("graph instantiation failed");
          rc = MBBS_EHIP;
          break;
        }
      }
      if (hipGraphLaunch(j.exec, c.st) != hipSuccess) { set_error("graph launch failed"); rc = MBBS_EHIP; break; }
    } else {
      rc = job_enqueue(j, k);
      if (rc < 0) break;
    }
    if (prof.on) prof.flush();
    rc = job_check(j);
  }
  if (j.exec) (void)hipGraphExecDestroy(j.exec);
  if (j.graph) (void)hipGraphDestroy(j.graph);
  if (prof.on) prof.flush();
  (void)hipStreamSynchronize(c.st);
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc < 0) {
    // a call that failed before or while iterating: nothing is reported as solved
    if (info)
      for (int s = 0; s < c.nsys; ++s) info[s].status = j.done[s] ? j.rc[s] : rc;
  } else {
    job_fill_info(j, info, secs);
    // the call's status: the worst over the systems
    for (int s = 0; s < c.nsys; ++s) {
      if (j.rc[s] < 0) rc = std::min(rc, j.rc[s]);
      else if (rc == MBBS_OK && j.rc[s] == MBBS_NOT_CONVERGED) rc = MBBS_NOT_CONVERGED;
    }
  }
  if (prof.on)
    for (int i = 0; i < 2 * Profiler::CAP; ++i) (void)hipEventDestroy(prof.ev[i]);
  return rc;
}

// ---------------------------------------------------------------- batched
// Batched driver.  Jobs (each a lattice handle: one system, or a batch of
// same-shape systems fused into every launch) are spread over up to
// BATCH_LANES internal streams (largest first, each to the least loaded
// lane); each lane is an independent chain on its own hardware queue, so the
// latency-bound launches of small jobs overlap.  The host never waits for a
// whole round: it polls one event per job and, as soon as a job's previous
// batch of k iterations (and the copy of its state records) has drained,
// decides on the host what that job does next (more iterations, a
// true-residual check, restarts, stop) and enqueues it behind whatever its
// lane still holds.
constexpr int BATCH_LANES = 4;

enum BatchPhase { PH_INIT = 0, PH_ITER = 1, PH_TRUE = 2 };

// Host-side mirror of the small device records one job reports back (pinned
// memory, written by asynchronous copies): nsys states, then nsys x L true
// and right-hand-side norms.
struct HostRec {
  SolverState* st;
  double* tn;
  double* bn;
};

struct BatchJob {
  SolveJob j;
  int lane = 0;
  int phase = PH_INIT;
  bool pending = false;
  hipEvent_t ev = nullptr;
  HostRec h{};
  void* pinned = nullptr;
};

static int batch_record(BatchJob& b) {
  MBBS_HIP(hipEventRecord(b.ev, b.j.c.st));
  b.pending = true;
  return MBBS_OK;
}

// Set-up without host synchronisation: constants, X = 0, ||b_i||^2 (back to
// the host for its check).
static int batch_init(BatchJob& b) {
  Ctx& c = b.j.c;
  if (c.w.Bp) {   // clover: solve A X = (1 + T)^{-1} B
    MBBS_TRY(launch_clover_apply(c.lat, c.L, c.B, c.w.Bp, c.st));
    c.B = c.w.Bp;
  }
  MBBS_TRY(launch_fill(c.w.d.one, c.nsys, make_double2(1, 0), c.st));
  MBBS_TRY(launch_fill(c.w.mone, c.nsys, make_double2(-1, 0), c.st));
  if (!c.p.x0_is_guess) MBBS_TRY(launch_fill(c.X, c.NL, make_double2(0, 0), c.st));
  MBBS_TRY(col_norms(c, c.B, c.w.d.bnorm2, nullptr));
  MBBS_HIP(hipMemcpyAsync(b.h.bn, c.w.d.bnorm2, (size_t)c.nsys * c.L * sizeof(double), hipMemcpyDeviceToHost, c.st));
  b.phase = PH_INIT;
  return batch_record(b);
}

// k iterations (replayed from a per-job graph when graph_iters > 1), then the
// state records back to the host.
static int batch_iterate(BatchJob& b, int k) {
  SolveJob& j = b.j;
  Ctx& c = j.c;
  if (k > 1) {
    if (!j.exec) {
      MBBS_HIP(hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal));
      int erc = job_enqueue(j, k);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c.st, &g);
      if (erc < 0) return erc;
      MBBS_CHECK(e == hipSuccess, "graph capture failed");
      j.graph = g;
      MBBS_CHECK(hipGraphInstantiate(&j.exec, g, nullptr, nullptr, 0) == hipSuccess, "graph instantiation failed");
    }
    MBBS_HIP(hipGraphLaunch(j.exec, c.st));
  } else {
    MBBS_TRY(job_enqueue(j, 1));
  }
  MBBS_HIP(hipMemcpyAsync(b.h.st, c.w.d.state, sizeof(SolverState) * c.nsys, hipMemcpyDeviceToHost, c.st));
  b.phase = PH_ITER;
  return batch_record(b);
}

static int batch_true(BatchJob& b) {
  Ctx& c = b.j.c;
  MBBS_TRY(true_residual(c));
  MBBS_HIP(hipMemcpyAsync(b.h.tn, c.w.trnorm2, (size_t)c.nsys * c.L * sizeof(double), hipMemcpyDeviceToHost, c.st));
  b.phase = PH_TRUE;
  return batch_record(b);
}

// The host's decision once a job's pending work has drained.
static int batch_step(BatchJob& b, int k) {
  SolveJob& j = b.j;
  Ctx& c = j.c;
  const int ns = c.nsys;
  if (b.phase == PH_INIT) {
    for (int s = 0; s < ns; ++s) {
      int col = 0;
      const bool bad = bad_rhs(&b.h.bn[(size_t)s * c.L], c.L, &col);
      if (bad) {
        set_error("right-hand side column " + std::to_string(col) + " is zero or not finite");
        j.finish(s, MBBS_EINVAL);
      }
      b.h.st[s] = fresh_state(c, bad);
    }
    if (j.ndone == ns) return MBBS_OK;
    MBBS_HIP(hipMemcpyAsync(c.w.d.state, b.h.st, sizeof(SolverState) * ns, hipMemcpyHostToDevice, c.st));
    MBBS_TRY(start(c, !c.p.x0_is_guess, true));
    for (int s = 0; s < ns; ++s)
      if (!j.done[s]) j.n_outer[s] += c.p.x0_is_guess ? 1 : 0;
    MBBS_TRY(launch_loop_test(c.L, c.w.d, c.st, ns));
    return batch_iterate(b, k);
  }
  if (b.phase == PH_ITER) {
    for (int s = 0; s < ns; ++s) j.hs[s] = b.h.st[s];
    for (int s = 0; s < ns; ++s)
      if (!j.hs[s].frozen) return batch_iterate(b, k);
    return batch_true(b);
  }
  // PH_TRUE: the same decisions as the single-call driver
  int nr = 0;
  MBBS_TRY(decide(j, b.h.tn, b.h.bn, &nr));
  if (nr == 0) return MBBS_OK;
  for (int s = 0; s < ns; ++s) b.h.st[s] = j.hs[s];
  MBBS_HIP(hipMemcpyAsync(c.w.d.state, b.h.st, sizeof(SolverState) * ns, hipMemcpyHostToDevice, c.st));
  MBBS_TRY(start(c, false, false));
  return batch_iterate(b, k);
}

static int batched_impl(int njob, const mbbs_lattice_t* lats, const int* Ls, const double* const* B, double* const* X,
                        const mbbs_solve_params* params, void* ws, size_t ws_bytes, mbbs_solve_info* infos,
                        void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  MBBS_CHECK(njob >= 1 && lats && Ls && B && X && params, "null argument");
  hipStream_t caller = (hipStream_t)stream;
  std::vector<BatchJob> jobs(njob);
  // lanes: largest jobs first, each to the least loaded lane
  const int nl = std::min(njob, BATCH_LANES);
  std::vector<int> order(njob);
  for (int i = 0; i < njob; ++i) order[i] = i;
  for (int i = 0; i < njob; ++i) MBBS_TRY(validate(lats[i], Ls[i], &params[i]));
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)lats[a]->g.V * Ls[a] > (double)lats[b]->g.V * Ls[b];
  });
  std::vector<double> load(nl, 0.0);
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    jobs[i].lane = l;
    load[l] += (double)lats[i]->g.V * Ls[i];
  }
  // infos: one record per system, jobs in argument order
  std::vector<int> first(njob, 0);
  for (int i = 1; i < njob; ++i) first[i] = first[i - 1] + lats[i - 1]->nsys;
  char* q = (char*)ws;
  size_t left = ws_bytes;
  for (int i = 0; i < njob; ++i) {
    const size_t need = workspace_bytes(lats[i], Ls[i], params[i]);
    MBBS_CHECK(q != nullptr && left >= need, "batched workspace too small");
    Ctx& c = jobs[i].j.c;
    mbbs_solve_params p = params[i];
    p.profile = 0;
    MBBS_CHECK(B[i] && X[i] && B[i] != X[i], "B and X must be distinct device blocks");
    ctx_setup(c, lats[i], Ls[i], p, B[i], X[i]);
    jobs[i].j.init(c.nsys);
    MBBS_TRY(bind(lats[i], Ls[i], c.p, q, need, c.w));
    c.frozen = &c.w.d.state->frozen;
    q += al(need);
    left -= std::min(left, al(need));
  }
  // resources, released on every exit path below
  std::vector<hipStream_t> lanes(nl, nullptr);
  hipEvent_t fork = nullptr;
  int rc = MBBS_OK;
  auto fail = [&](int code, const char* msg) { if (rc >= 0) { rc = code; set_error(msg); } };
  for (int i = 0; i < njob && rc >= 0; ++i) {
    BatchJob& b = jobs[i];
    const int ns = b.j.c.nsys, L = b.j.c.L;
    const size_t bytes = sizeof(SolverState) * ns + 2 * sizeof(double) * ns * L;
    if (hipHostMalloc(&b.pinned, bytes, hipHostMallocDefault) != hipSuccess) {
      fail(MBBS_ENOMEM, "pinned host memory for the batched state records");
      break;
    }
    b.h.st = (SolverState*)b.pinned;
    b.h.tn = (double*)((char*)b.pinned + sizeof(SolverState) * ns);
    b.h.bn = b.h.tn + (size_t)ns * L;
  }
  for (int l = 0; l < nl && rc >= 0; ++l)
    if (hipStreamCreateWithFlags(&lanes[l], hipStreamNonBlocking) != hipSuccess) fail(MBBS_EHIP, "stream creation");
  if (rc >= 0 && (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
                  hipEventRecord(fork, caller) != hipSuccess))
    fail(MBBS_EHIP, "event creation");
  for (int l = 0; l < nl && rc >= 0; ++l)
    if (hipStreamWaitEvent(lanes[l], fork, 0) != hipSuccess) fail(MBBS_EHIP, "stream wait");
  for (int i = 0; i < njob && rc >= 0; ++i) {
    BatchJob& b = jobs[i];
    b.j.c.st = lanes[b.lane];
    if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) fail(MBBS_EHIP, "event creation");
  }
  // set-up of every job, then the polling loop
  for (int i = 0; i < njob && rc >= 0; ++i) {
    const int e = batch_init(jobs[i]);
    if (e < 0) rc = e;
  }
  auto job_done = [](const BatchJob& b) { return b.j.ndone == b.j.c.nsys; };
  int remaining = njob;
  while (rc >= 0 && remaining > 0) {
    bool progress = false;
    for (int i = 0; i < njob && rc >= 0; ++i) {
      BatchJob& b = jobs[i];
      if (job_done(b) || !b.pending) continue;
      const hipError_t e = hipEventQuery(b.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) { fail(MBBS_EHIP, "batched solve: device error"); break; }
      b.pending = false;
      progress = true;
      const int k = std::max(1, b.j.c.p.graph_iters);
      const int s = batch_step(b, k);
      if (s < 0) { rc = s; break; }
      if (job_done(b)) --remaining;
    }
    if (!progress) std::this_thread::yield();
  }
  for (int l = 0; l < nl; ++l)
    if (lanes[l]) (void)hipStreamSynchronize(lanes[l]);
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = MBBS_OK;
  for (int i = 0; i < njob; ++i) {
    SolveJob& j = jobs[i].j;
    mbbs_solve_info* in = infos ? infos + first[i] : nullptr;
    if (rc >= 0) job_fill_info(j, in, secs);
    else if (in)
      for (int s = 0; s < j.c.nsys; ++s) in[s].status = j.done[s] ? j.rc[s] : rc;
    for (int s = 0; s < j.c.nsys; ++s) {
      if (j.rc[s] < 0) worst = std::min(worst, j.rc[s]);
      else if (worst == MBBS_OK && j.rc[s] == MBBS_NOT_CONVERGED) worst = MBBS_NOT_CONVERGED;
    }
    if (j.exec) (void)hipGraphExecDestroy(j.exec);
    if (j.graph) (void)hipGraphDestroy(j.graph);
    if (jobs[i].ev) (void)hipEventDestroy(jobs[i].ev);
    if (jobs[i].pinned) (void)hipHostFree(jobs[i].pinned);
  }
  // the caller's stream sees every lane's work as complete
  for (int l = 0; l < nl; ++l)
    if (lanes[l]) (void)hipStreamDestroy(lanes[l]);
  if (fork) (void)hipEventDestroy(fork);
  return rc < 0 ? rc : worst;
}

}  // namespace mbbs

using namespace mbbs;

extern "C" void mbbs_solve_params_default(mbbs_solve_params* p) {
  if (!p) return;
  p->tol = 1e-10;
  p->maxiter = 1000;
  p->max_restarts = 3;
  p->ncy = 4;
  p->nmr = 4;
  p->sap_prec = MBBS_FP32;
  p->x0_is_guess = 0;
  p->qr_passes = 1;
  p->graph_iters = 1;
  p->precond = 1;
  p->memsave = 0;
  p->profile = 0;
  p->domain_solver = 0;
  p->nssor = 1;
  p->ssor_omega = 1.26;
  p->rtilde = nullptr;
}

extern "C" int mbbs_solve_workspace_size(mbbs_lattice_t lat, int L, const mbbs_solve_params* params, size_t* bytes) {
  MBBS_TRY(validate(lat, L, params));
  MBBS_CHECK(bytes != nullptr, "null argument");
  *bytes = workspace_bytes(lat, L, *params);
  return MBBS_OK;
}

extern "C" int mbbs_solve(mbbs_lattice_t lat, int L, const double* B_dev, double* X_dev,
                          const mbbs_solve_params* params, void* ws_dev, size_t ws_bytes, mbbs_solve_info* info,
                          void* stream) {
  return solve_impl(lat, L, B_dev, X_dev, params, ws_dev, ws_bytes, info, stream);
}

extern "C" int mbbs_solve_batched_workspace_size(int nsys, const mbbs_lattice_t* lats, const int* Ls,
                                                 const mbbs_solve_params* params, size_t* bytes) {
  MBBS_CHECK(nsys >= 1 && lats && Ls && params && bytes, "null argument");
  size_t t = 0;
  for (int i = 0; i < nsys; ++i) {
    MBBS_TRY(validate(lats[i], Ls[i], &params[i]));
    t += al(workspace_bytes(lats[i], Ls[i], params[i]));
  }
  *bytes = t;
  return MBBS_OK;
}

extern "C" int mbbs_solve_batched(int nsys, const mbbs_lattice_t* lats, const int* Ls, const double* const* B_dev,
                                  double* const* X_dev, const mbbs_solve_params* params, void* ws_dev,
                                  size_t ws_bytes, mbbs_solve_info* infos, void* stream) {
  return batched_impl(nsys, lats, Ls, B_dev, X_dev, params, ws_dev, ws_bytes, infos, stream);
}
