// Tall-skinny block linear algebra of Alg. 1 in FP64 on N x L blocks stored
// row-major (right-hand side fastest):
//  - Gram products X^H Y (steps 4.1 via P^H P, 4.4, 4.8, 4.11), fixed-order
//    two-stage reductions so results are bit-reproducible run to run;
//  - block updates out = sum_k in_k C_k with L x L (or scalar) coefficients
//    (steps 4.5, 4.9, 4.10, 4.12), optionally fused with the Gram product or
//    the column norms of their output;
//  - one-workgroup coefficient kernels: Cholesky QR factor, LU with partial
//    pivoting and the alpha/beta/zeta solves.
// Every kernel of the iteration returns at once while the solver's device
// flag `frozen` is set (converged, iteration cap or breakdown).
#include "blas.h"

namespace mbbs {

// Sum v over threadIdx.y (fixed tree) for each threadIdx.x; result valid in y == 0.
__device__ inline double2 block_reduce_y(double2* sh, cplx<double> v, int j, int y, int L, int S) {
  __syncthreads();
  sh[(size_t)y * L + j] = make_double2(v.re, v.im);
  __syncthreads();
  for (int st = 1; st < S; st <<= 1) {
    if ((y % (2 * st)) == 0 && y + st < S) {
      double2 u = sh[(size_t)y * L + j], w = sh[(size_t)(y + st) * L + j];
      sh[(size_t)y * L + j] = make_double2(u.x + w.x, u.y + w.y);
    }
    __syncthreads();
  }
  return sh[j];
}

// ---------------------------------------------------------------- Gram
// Thread (j, y): column j of X, row y of the block's current row tile.  Each
// block accumulates sum_n conj(X[n,j]) Y[n,:] over its rows (Y rows staged in
// LDS), reduces over y in LDS and writes its partial Gram matrices.  The pair
// count NP and the column bound LMAX are compile-time so that the
// accumulators stay in registers.
template <int LMAX, int NF, int ND, bool EXACT = false>
__global__ void __launch_bounds__(256) k_gram(int L, size_t N, GramArgs a, double2* __restrict__ partial,
                                              const int* __restrict__ frozen, int fstride) {
  if constexpr (EXACT) L = LMAX;   // L known at compile time: immediate offsets, no column bounds
  // pairs 0..NF-1 are full products, NF..NF+ND-1 diagonal-only
  constexpr int NP = NF + ND;
  const int sys = blockIdx.y;
  if (frozen && frozen[sys * fstride]) return;
  // the system's rows: [sys N, sys N + N) of the stacked blocks
  const size_t nbeg = (size_t)sys * N, nend = nbeg + N;
  extern __shared__ double2 sh[];  // [2][GRAM_MAXPAIR][S][L] Y rows, reused for the reduction
  const int j = threadIdx.x, y = threadIdx.y, S = blockDim.y;
  cplx<double> acc[NF > 0 ? NF : 1][LMAX];
  cplx<double> dacc[ND > 0 ? ND : 1];
#pragma unroll
  for (int p = 0; p < (NF > 0 ? NF : 1); ++p)
#pragma unroll
    for (int q = 0; q < LMAX; ++q) acc[p][q] = cmake(0.0, 0.0);
#pragma unroll
  for (int p = 0; p < (ND > 0 ? ND : 1); ++p) dacc[p] = cmake(0.0, 0.0);
  const size_t stride = (size_t)gridDim.x * S;
  int buf = 0;   // two row buffers: one barrier per row tile
  // the next row tile's values are loaded while the current one is summed
  // (twice the bytes in flight per wave: the pass is bound by memory latency)
  double2 xn[NP], yn[NP];
  auto fetch = [&](size_t n) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      xn[p] = make_double2(0, 0);
      yn[p] = make_double2(0, 0);
      if (n < nend) {
        xn[p] = a.X[p][n * L + j];
        yn[p] = a.Y[p][n * L + j];
      }
    }
  };
  fetch(nbeg + (size_t)blockIdx.x * S + y);
  for (size_t n0 = nbeg + (size_t)blockIdx.x * S; n0 < nend; n0 += stride, buf ^= 1) {
    cplx<double> xv[NP];
    double2 yv[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      xv[p] = cmake(xn[p].x, xn[p].y);
      yv[p] = yn[p];
    }
    fetch(n0 + stride + y);
    double2* rows = sh + (size_t)buf * GRAM_MAXPAIR * S * L;
#pragma unroll
    for (int p = 0; p < NF; ++p) rows[((size_t)p * S + y) * L + j] = yv[p];
#pragma unroll
    for (int p = NF; p < NP; ++p) dacc[p - NF] = dacc[p - NF] + cdot(xv[p], cmake(yv[p].x, yv[p].y));
    if constexpr (NF > 0) {
      // the buffer written here was last read two tiles ago, before the
      // barrier of the previous tile
      __syncthreads();
#pragma unroll
      for (int p = 0; p < NF; ++p)
#pragma unroll
        for (int q = 0; q < LMAX; ++q) {
          if (q < L) {
            double2 ye = rows[((size_t)p * S + y) * L + q];
            acc[p][q] = acc[p][q] + cdot(xv[p], cmake(ye.x, ye.y));
          }
        }
    }
  }
  // reduce over y one output column at a time: sh reused as [S][L]
  partial += (size_t)blockIdx.y * gridDim.x * GRAM_MAXPAIR * L * L;   // the system's partials
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    double2* out = partial + ((size_t)blockIdx.x * GRAM_MAXPAIR + p) * L * L;
#pragma unroll
    for (int q = 0; q < LMAX; ++q) {
      if (q < L) {
        double2 r = block_reduce_y(sh, acc[p][q], j, y, L, S);
        if (y == 0) out[j * L + q] = r;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < ND; ++p) {
    double2* out = partial + ((size_t)blockIdx.x * GRAM_MAXPAIR + NF + p) * L * L;
    double2 r = block_reduce_y(sh, dacc[p], j, y, L, S);
    if (y == 0)
      for (int qq = 0; qq < L; ++qq) out[j * L + qq] = qq == j ? r : make_double2(0, 0);
  }
}

// Sum the block partials in a fixed tree: one block per output entry.
__global__ void __launch_bounds__(256) k_gram_finish(int L, int nblk, const double2* __restrict__ partial,
                                                     GramOut o, const int* __restrict__ frozen, int fstride) {
  const int sys = blockIdx.y;
  if (frozen && frozen[sys * fstride]) return;
  partial += (size_t)sys * nblk * GRAM_MAXPAIR * L * L;
  __shared__ double2 red[256];
  const int e = blockIdx.x;  // (pair, i, j)
  const int p = e / (L * L), ij = e % (L * L);
  double2 s = make_double2(0, 0);
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    double2 v = partial[((size_t)b * GRAM_MAXPAIR + p) * L * L + ij];
    s.x += v.x; s.y += v.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[threadIdx.x].x += red[threadIdx.x + st].x;
      red[threadIdx.x].y += red[threadIdx.x + st].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) o.G[p][(size_t)sys * L * L + ij] = red[0];
}

// ---------------------------------------------------------------- block update
// out[n, j] = sum_k T_k(in_k)[n, j], T_k = identity, complex scalar (device),
// or right multiplication by an L x L matrix (device, row-major).  Matrix
// inputs stage their rows in LDS before any output is written, so an output
// may alias one of the inputs.  Optionally accumulates the Gram matrix (or
// only the column norms) of the output, as GRAM partials.
template <int LMAX, int GM, bool EXACT = false>
__global__ void __launch_bounds__(256) k_combo(int L, size_t N, ComboArgs a, double2* __restrict__ out,
                                               double2* __restrict__ partial, const int* __restrict__ frozen,
                                               int fstride) {
  if constexpr (EXACT) L = LMAX;
  const int sys = blockIdx.y;
  if (frozen && frozen[sys * fstride]) return;
  // the system's rows and coefficients: offsets added where the argument
  // block is read (writing to it would move it to scratch memory)
  const size_t roff = (size_t)sys * N * L;
  out += roff;
  if (partial) partial += (size_t)sys * gridDim.x * GRAM_MAXPAIR * L * L;
  extern __shared__ double2 sh[];  // [nmat][S][L] rows, then [nmat][L][L] coefficients
  const int j = threadIdx.x, y = threadIdx.y, S = blockDim.y;
  const int tid = y * L + j, nthr = L * S;
  const int nin = a.nin;
  double2* mats = sh + (size_t)COMBO_MAXIN * S * L;
  for (int k = 0; k < nin; ++k)
    if (a.mode[k] == 2)
      for (int e = tid; e < L * L; e += nthr) mats[(size_t)k * L * L + e] = a.coef[k][(size_t)sys * L * L + e];
  cplx<double> g[LMAX];
#pragma unroll
  for (int q = 0; q < LMAX; ++q) g[q] = cmake(0.0, 0.0);
  // rows are staged through LDS only for matrix inputs (and for the output
  // Gram); without them the rows are independent and need no barriers
  bool anymat = false;
  for (int k = 0; k < nin; ++k) anymat = anymat || a.mode[k] == 2;
  const bool staged = anymat || GM == 2;
  const size_t stride = (size_t)gridDim.x * S;
  // the next row tile's inputs are loaded while the current one is combined
  // (more bytes in flight per wave: the pass is bound by memory latency)
  double2 vn[COMBO_MAXIN];
  auto fetch = [&](size_t n) {
#pragma unroll
    for (int k = 0; k < COMBO_MAXIN; ++k) {
      vn[k] = make_double2(0, 0);
      if (k < nin && n < N) vn[k] = a.in[k][roff + n * L + j];
    }
  };
  fetch((size_t)blockIdx.x * S + y);
  for (size_t n0 = (size_t)blockIdx.x * S; n0 < N; n0 += stride) {
    const size_t n = n0 + y;
    double2 vc[COMBO_MAXIN];
#pragma unroll
    for (int k = 0; k < COMBO_MAXIN; ++k) vc[k] = vn[k];
    fetch(n0 + stride + y);
    if (staged) __syncthreads();
    cplx<double> acc = cmake(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < COMBO_MAXIN; ++k) {
      if (k >= nin) break;
      if (a.mode[k] == 2) {
        sh[((size_t)k * S + y) * L + j] = vc[k];   // zero past the last row
      } else if (n < N) {
        const double2 v = vc[k];
        if (a.mode[k] == 0) acc = acc + cmake(v.x, v.y);
        else acc = acc + cmake(a.coef[k][sys].x, a.coef[k][sys].y) * cmake(v.x, v.y);
      }
    }
    if (anymat) __syncthreads();
    for (int k = 0; k < nin; ++k) {
      if (a.mode[k] != 2) continue;
      const double2* row = sh + ((size_t)k * S + y) * L;
      const double2* m = mats + (size_t)k * L * L;
      for (int q = 0; q < L; ++q) acc = acc + cmake(row[q].x, row[q].y) * cmake(m[q * L + j].x, m[q * L + j].y);
    }
    if (n < N) out[n * L + j] = make_double2(acc.re, acc.im);
    if constexpr (GM == 1) {
      g[0] = g[0] + cmake(norm2(acc), 0.0);
    } else if constexpr (GM == 2) {
      // exchange the output row through LDS (slot of input 0 is free now)
      __syncthreads();
      double2* orow = sh + ((size_t)(COMBO_MAXIN - 1) * S + y) * L;
      orow[j] = n < N ? make_double2(acc.re, acc.im) : make_double2(0, 0);
      __syncthreads();
      cplx<double> xv = n < N ? acc : cmake(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < LMAX; ++q)
        if (q < L) g[q] = g[q] + cdot(xv, cmake(orow[q].x, orow[q].y));
    }
  }
  if constexpr (GM != 0) {
    const int nq = GM == 1 ? 1 : L;
    double2* o = partial + (size_t)blockIdx.x * GRAM_MAXPAIR * L * L;
#pragma unroll
    for (int q = 0; q < LMAX; ++q) {
      if (q < nq) {
        double2 r = block_reduce_y(sh, g[q], j, y, L, S);
        if (y == 0) {
          if (GM == 1) {
            for (int qq = 0; qq < L; ++qq) o[j * L + qq] = qq == j ? r : make_double2(0, 0);
          } else {
            o[j * L + q] = r;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- small L x L
// Complex L x L helpers executed by one workgroup (matrices in LDS).
__device__ inline cplx<double> ld2(const double2* p, int i) { return cmake(p[i].x, p[i].y); }
__device__ inline void st2(double2* p, int i, cplx<double> v) { p[i] = make_double2(v.re, v.im); }

// Upper Cholesky G = gamma^H gamma (positive real diagonal) by thread 0, then
// gamma^{-1} column-parallel.  Returns false (via flag) if not positive definite.
__device__ bool chol_inv(int L, double2* G, double2* ginv) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    for (int i = 0; i < L && ok; ++i) {
      double d = G[i * L + i].x;
      for (int k = 0; k < i; ++k) d -= norm2(ld2(G, k * L + i));
      if (!(d > 0) || !isfinite(d)) { ok = 0; break; }
      d = sqrt(d);
      st2(G, i * L + i, cmake(d, 0.0));
      for (int jj = i + 1; jj < L; ++jj) {
        cplx<double> s = ld2(G, i * L + jj);
        for (int k = 0; k < i; ++k) s = s - cdot(ld2(G, k * L + i), ld2(G, k * L + jj));
        st2(G, i * L + jj, (1.0 / d) * s);
      }
      for (int jj = 0; jj < i; ++jj) st2(G, i * L + jj, cmake(0.0, 0.0));
    }
  }
  __syncthreads();
  if (!ok) return false;
  // inverse of upper-triangular gamma: solve gamma * ginv[:, c] = e_c, column c per thread
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    for (int i = L - 1; i >= 0; --i) {
      cplx<double> s = cmake(i == c ? 1.0 : 0.0, 0.0);
      for (int k = i + 1; k < L; ++k) s = s - ld2(G, i * L + k) * ld2(ginv, k * L + c);
      st2(ginv, i * L + c, (1.0 / G[i * L + i].x) * s);
    }
  }
  __syncthreads();
  return true;
}

// LU with partial pivoting (pivot: largest |Re|+|Im|, first one on ties), in
// place, thread 0.  Returns false on an exactly zero or non-finite pivot.
__device__ bool lu_factor(int L, double2* A, int* piv) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    for (int kk = 0; kk < L; ++kk) {
      int p = kk;
      double best = -1;
      for (int i = kk; i < L; ++i) {
        double v = fabs(A[i * L + kk].x) + fabs(A[i * L + kk].y);
        if (v > best) { best = v; p = i; }
      }
      piv[kk] = p;
      if (!(best > 0) || !isfinite(best)) { ok = 0; break; }
      if (p != kk)
        for (int c = 0; c < L; ++c) { double2 t = A[kk * L + c]; A[kk * L + c] = A[p * L + c]; A[p * L + c] = t; }
      cplx<double> d = ld2(A, kk * L + kk);
      double dn = norm2(d);
      cplx<double> dinv = cmake(d.re / dn, -d.im / dn);
      for (int i = kk + 1; i < L; ++i) {
        cplx<double> f = ld2(A, i * L + kk) * dinv;
        st2(A, i * L + kk, f);
        for (int c = kk + 1; c < L; ++c) st2(A, i * L + c, ld2(A, i * L + c) - f * ld2(A, kk * L + c));
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// Solve (LU) X = sgn * Rhs for m right-hand sides (row-major L x m), column-parallel.
__device__ void lu_solve(int L, int m, const double2* A, const int* piv, const double2* R, double2* X, double sgn) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    for (int i = 0; i < L; ++i) X[i * m + c] = make_double2(sgn * R[i * m + c].x, sgn * R[i * m + c].y);
    for (int k = 0; k < L; ++k) {
      int p = piv[k];
      if (p != k) { double2 t = X[k * m + c]; X[k * m + c] = X[p * m + c]; X[p * m + c] = t; }
    }
    for (int i = 0; i < L; ++i) {
      cplx<double> s = ld2(X, i * m + c);
      for (int k = 0; k < i; ++k) s = s - ld2(A, i * L + k) * ld2(X, k * m + c);
      st2(X, i * m + c, s);
    }
    for (int i = L - 1; i >= 0; --i) {
      cplx<double> s = ld2(X, i * m + c);
      for (int k = i + 1; k < L; ++k) s = s - ld2(A, i * L + k) * ld2(X, k * m + c);
      cplx<double> d = ld2(A, i * L + i);
      double dn = norm2(d);
      st2(X, i * m + c, s * cmake(d.re / dn, -d.im / dn));
    }
  }
  __syncthreads();
}

// Loop test of Alg. 1 (iterate while max_i ||r_i||/||b_i|| > tol), run after
// step 4.10 has formed the new column norms, so that a stop is visible to the
// host before it enqueues another iteration; also run once on R_0.
__global__ void k_loop_test(int L, SolverDev d) {
  d = sys_view(d, blockIdx.x, L);   // one workgroup per system
  SolverState* S = d.state;
  if (S->frozen) return;
  if (threadIdx.x != 0) return;
  double worst = 0;
  int bad = 0;
  for (int i = 0; i < L; ++i) {
    const double r = d.rnorm2[i] / d.bnorm2[i];
    if (!isfinite(r)) bad = 1;
    worst = fmax(worst, r);
  }
  if (S->iter >= 1 && S->iter <= HIST_CAP) {
    d.hist[S->iter - 1] = bad ? (double)NAN : worst;
    S->hist_len = S->iter;
  }
  if (bad) {
    S->frozen = 1;
    S->status = ST_BREAKDOWN;
    S->reason = 4;
  } else if (worst <= S->tol2) {
    S->frozen = 1;
    S->status = ST_CONVERGED;
  } else if (S->iter >= S->maxiter) {
    S->frozen = 1;
    S->status = ST_MAXITER;
  }
}

// Step 4.1: Cholesky QR factor of P (gamma^{-1} for the consumers); with
// qr_passes = 0 the QR step is left out (gamma = 1, the unmodified block
// BiCGSTAB the paper's QR is compared against).  Counts the iteration.
__global__ void k_coef_qr(int L, SolverDev d) {
  d = sys_view(d, blockIdx.x, L);   // one workgroup per system
  SolverState* S = d.state;
  if (S->frozen) return;
  extern __shared__ double2 sm[];
  double2* G = sm;
  double2* gi = sm + L * L;
  if (d.qr_passes == 0) {
    for (int e = threadIdx.x; e < L * L; e += blockDim.x)
      d.ginv[e] = make_double2(e / L == e % L ? 1.0 : 0.0, 0.0);
    if (threadIdx.x == 0) S->iter += 1;
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) G[e] = d.Gpp[e];
  __syncthreads();
  bool ok = chol_inv(L, G, gi);
  if (!ok) {
    if (threadIdx.x == 0) { S->frozen = 1; S->status = ST_BREAKDOWN; S->reason = 1; }
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) d.ginv[e] = gi[e];
  if (threadIdx.x == 0) S->iter += 1;
}

// Optional second Cholesky-QR pass: Gpp2 = (P g1^{-1})^H (P g1^{-1}) was
// accumulated by the caller; fold its factor into ginv = g1^{-1} g2^{-1}.
__global__ void k_coef_qr2(int L, SolverDev d) {
  d = sys_view(d, blockIdx.x, L);   // one workgroup per system
  SolverState* S = d.state;
  if (S->frozen) return;
  extern __shared__ double2 sm[];
  double2* G = sm;
  double2* gi = sm + L * L;
  double2* g1 = sm + 2 * L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) { G[e] = d.Gpp2[e]; g1[e] = d.ginv[e]; }
  __syncthreads();
  bool ok = chol_inv(L, G, gi);
  if (!ok) {
    if (threadIdx.x == 0) { S->frozen = 1; S->status = ST_BREAKDOWN; S->reason = 1; }
    return;
  }
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    int i = e / L, j = e % L;
    cplx<double> s = cmake(0.0, 0.0);
    for (int k = 0; k < L; ++k) s = s + ld2(g1, i * L + k) * ld2(gi, k * L + j);
    st2(d.ginv, e, s);
  }
}

// Step 4.4: LU of R~^H V, alpha = (R~^H V)^{-1} R~^H R; also -alpha.
__global__ void k_coef_alpha(int L, SolverDev d) {
  d = sys_view(d, blockIdx.x, L);   // one workgroup per system
  SolverState* S = d.state;
  if (S->frozen) return;
  extern __shared__ double2 sm[];
  double2* A = sm;
  double2* X = sm + L * L;
  __shared__ int piv[64];
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) A[e] = d.RtV[e];
  __syncthreads();
  if (!lu_factor(L, A, piv)) {
    if (threadIdx.x == 0) { S->frozen = 1; S->status = ST_BREAKDOWN; S->reason = 2; }
    return;
  }
  lu_solve(L, L, A, piv, d.RtR, X, 1.0);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    d.lu[e] = A[e];
    d.alpha[e] = X[e];
    d.nalpha[e] = make_double2(-X[e].x, -X[e].y);
  }
  for (int e = threadIdx.x; e < L; e += blockDim.x) d.piv[e] = piv[e];
}

// Steps 4.8 and 4.11: zeta = Tr(Z^H T)/Tr(Z^H Z); beta = -(R~^H V)^{-1} R~^H Z;
// coefficients of the fused updates: C1 = ginv * beta, C2 = -zeta * beta.
__global__ void k_coef_zeta(int L, SolverDev d) {
  d = sys_view(d, blockIdx.x, L);   // one workgroup per system
  SolverState* S = d.state;
  if (S->frozen) return;
  extern __shared__ double2 sm[];
  double2* B = sm;
  __shared__ int piv[64];
  __shared__ double zt_re, zt_im, zz;
  if (threadIdx.x == 0) {
    zt_re = zt_im = zz = 0;
    for (int i = 0; i < L; ++i) {
      zt_re += d.ZT[i * L + i].x;
      zt_im += d.ZT[i * L + i].y;
      zz += d.ZZ[i * L + i].x;
    }
  }
  for (int e = threadIdx.x; e < L; e += blockDim.x) piv[e] = d.piv[e];
  __syncthreads();
  const double zr = zt_re / zz, zi = zt_im / zz;
  if (!(zz > 0) || !isfinite(zr) || !isfinite(zi)) {
    if (threadIdx.x == 0) { S->frozen = 1; S->status = ST_BREAKDOWN; S->reason = 3; }
    return;
  }
  lu_solve(L, L, d.lu, piv, d.RtZ, B, -1.0);
  const cplx<double> z = cmake(zr, zi);
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    int i = e / L, jj = e % L;
    cplx<double> s = cmake(0.0, 0.0);
    for (int k = 0; k < L; ++k) s = s + ld2(d.ginv, i * L + k) * ld2(B, k * L + jj);
    st2(d.C1, e, s);
    st2(d.C2, e, cmake(-1.0, 0.0) * (z * ld2(B, e)));
    d.beta[e] = B[e];
  }
  if (threadIdx.x == 0) {
    d.zeta[0] = make_double2(zr, zi);
    d.nzeta[0] = make_double2(-zr, -zi);
  }
}

// ---------------------------------------------------------------- utilities
__global__ void k_fill(double2* __restrict__ p, size_t n, double2 v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_copy(const double2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}
__global__ void k_copy_sys(const double2* __restrict__ a, double2* __restrict__ b, size_t n, const int* __restrict__ frozen,
                           int fstride) {
  const int sys = blockIdx.y;
  if (frozen && frozen[sys * fstride]) return;
  a += (size_t)sys * n;
  b += (size_t)sys * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// Precision conversions of whole blocks (lexicographic order).
template <int P>
__global__ void __launch_bounds__(256) k_conv_to(size_t nsites, int L, const double2* __restrict__ x,
                                                 typename Store<P>::Elem* __restrict__ y, float* __restrict__ ys) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= nsites * L) return;
  const size_t s = t / L;
  const int j = t % L;
  if constexpr (Store<P>::scaled) {
    float m = 0;
    for (int e = 0; e < 12; ++e) {
      double2 v = x[(s * 12 + e) * L + j];
      m = fmaxf(m, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
    }
    ys[s * L + j] = m;
    float inv = m > 0 ? 1.0f / m : 0.0f;
    for (int e = 0; e < 12; ++e) {
      double2 v = x[(s * 12 + e) * L + j];
      Store<P>::st(y, (s * 12 + e) * L + j, cmake<float>((float)v.x * inv, (float)v.y * inv));
    }
  } else {
    using R = typename Store<P>::Real;
    for (int e = 0; e < 12; ++e) {
      double2 v = x[(s * 12 + e) * L + j];
      Store<P>::st(y, (s * 12 + e) * L + j, cmake<R>((R)v.x, (R)v.y));
    }
  }
}
template <int P>
__global__ void __launch_bounds__(256) k_conv_from(size_t nsites, int L, const typename Store<P>::Elem* __restrict__ x,
                                                   const float* __restrict__ xs, double2* __restrict__ y) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= nsites * L) return;
  const size_t s = t / L;
  const int j = t % L;
  double sc = 1;
  if constexpr (Store<P>::scaled) sc = xs[s * L + j];
  for (int e = 0; e < 12; ++e) {
    auto v = Store<P>::ld(x, (s * 12 + e) * L + j);
    y[(s * 12 + e) * L + j] = make_double2((double)v.re * sc, (double)v.im * sc);
  }
}

// ---------------------------------------------------------------- host side
static int gram_rows_per_block(int L) {
  int S = 256 / L;
  if (S < 1) S = 1;
  // power of two not required; keep within 256 threads
  return S;
}

int gram_blocks(size_t N, int L) {
  const int S = gram_rows_per_block(L);
  size_t nb = (N + S - 1) / S;
  return (int)(nb < GRAM_MAXBLK ? nb : GRAM_MAXBLK);
}

size_t gram_partial_bytes(size_t N, int L, int nsys) {
  return (size_t)nsys * gram_blocks(N, L) * GRAM_MAXPAIR * L * L * sizeof(double2);
}

template <int LMAX>
static void launch_gram_l(int L, size_t N, const GramArgs& a, double2* partial, const int* frozen, hipStream_t st,
                          SysBatch sb) {
  const int S = gram_rows_per_block(L);
  const int nb = gram_blocks(N, L);
  const size_t shb = 2 * (size_t)GRAM_MAXPAIR * S * L * sizeof(double2);
  int nf = 0;
  while (nf < a.npair && !a.diag[nf]) ++nf;
  const int nd = a.npair - nf;
  const dim3 grd(nb, sb.n);
#define GL(F, D)                                                                                         \
  do {                                                                                                   \
    if (L == LMAX)                                                                                       \
      hipLaunchKernelGGL((k_gram<LMAX, F, D, true>), grd, dim3(L, S), shb, st, L, N, a, partial, frozen, sb.fstride); \
    else                                                                                                 \
      hipLaunchKernelGGL((k_gram<LMAX, F, D>), grd, dim3(L, S), shb, st, L, N, a, partial, frozen, sb.fstride);     \
  } while (0)
  if (nf == 1 && nd == 0) GL(1, 0);
  else if (nf == 2 && nd == 0) GL(2, 0);
  else if (nf == 1 && nd == 2) GL(1, 2);
  else if (nf == 0 && nd == 1) GL(0, 1);
  else if (nf == 3 && nd == 0) GL(3, 0);
  else if (nf == 1 && nd == 1) GL(1, 1);
  else if (nf == 0 && nd == 2) GL(0, 2);
  else GL(0, 3);
#undef GL
}

int launch_gram(int L, size_t N, const GramArgs& a, const GramOut& o, double2* partial, const int* frozen,
                hipStream_t st, SysBatch sb) {
  MBBS_CHECK(L >= 1 && L <= LMAX_SOLVER, "L out of range for block linear algebra");
  MBBS_CHECK(a.npair >= 1 && a.npair <= GRAM_MAXPAIR, "bad Gram pair count");
  if (L <= 4) launch_gram_l<4>(L, N, a, partial, frozen, st, sb);
  else if (L <= 8) launch_gram_l<8>(L, N, a, partial, frozen, st, sb);
  else if (L <= 12) launch_gram_l<12>(L, N, a, partial, frozen, st, sb);
  else launch_gram_l<16>(L, N, a, partial, frozen, st, sb);
  MBBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_finish, dim3(a.npair * L * L, sb.n), dim3(256), 0, st, L, gram_blocks(N, L), partial, o,
                     frozen, sb.fstride);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

template <int LMAX, int GM>
static void launch_combo_l(int L, size_t N, const ComboArgs& a, double2* out, double2* partial, const int* frozen,
                           hipStream_t st, SysBatch sb) {
  const int S = gram_rows_per_block(L);
  const int nb = gram_blocks(N, L);
  const size_t shb = ((size_t)COMBO_MAXIN * S * L + (size_t)COMBO_MAXIN * L * L) * sizeof(double2);
  const dim3 grd(nb, sb.n);
  if (L == LMAX)
    hipLaunchKernelGGL((k_combo<LMAX, GM, true>), grd, dim3(L, S), shb, st, L, N, a, out, partial, frozen, sb.fstride);
  else
    hipLaunchKernelGGL((k_combo<LMAX, GM>), grd, dim3(L, S), shb, st, L, N, a, out, partial, frozen, sb.fstride);
}

int launch_combo(int L, size_t N, const ComboArgs& a, double2* out, int gram_mode, const GramOut* o,
                 double2* partial, const int* frozen, hipStream_t st, SysBatch sb) {
  MBBS_CHECK(L >= 1 && L <= LMAX_SOLVER, "L out of range for block linear algebra");
#define CL(LM)                                                                                   \
  do {                                                                                           \
    if (gram_mode == 0) launch_combo_l<LM, 0>(L, N, a, out, partial, frozen, st, sb);            \
    else if (gram_mode == 1) launch_combo_l<LM, 1>(L, N, a, out, partial, frozen, st, sb);       \
    else launch_combo_l<LM, 2>(L, N, a, out, partial, frozen, st, sb);                           \
  } while (0)
  if (L <= 4) CL(4);
  else if (L <= 8) CL(8);
  else if (L <= 12) CL(12);
  else CL(16);
#undef CL
  MBBS_HIP(hipGetLastError());
  if (gram_mode != 0) {
    hipLaunchKernelGGL(k_gram_finish, dim3(L * L, sb.n), dim3(256), 0, st, L, gram_blocks(N, L), partial, *o, frozen,
                       sb.fstride);
    MBBS_HIP(hipGetLastError());
  }
  return MBBS_OK;
}

int launch_coef(int which, int L, const SolverDev& d, hipStream_t st, int nsys) {
  const size_t sh = 3 * (size_t)L * L * sizeof(double2);
  switch (which) {
    case 0: hipLaunchKernelGGL(k_coef_qr, dim3(nsys), dim3(64), sh, st, L, d); break;
    case 1: hipLaunchKernelGGL(k_coef_qr2, dim3(nsys), dim3(64), sh, st, L, d); break;
    case 2: hipLaunchKernelGGL(k_coef_alpha, dim3(nsys), dim3(64), sh, st, L, d); break;
    default: hipLaunchKernelGGL(k_coef_zeta, dim3(nsys), dim3(64), sh, st, L, d); break;
  }
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_loop_test(int L, const SolverDev& d, hipStream_t st, int nsys) {
  hipLaunchKernelGGL(k_loop_test, dim3(nsys), dim3(64), 0, st, L, d);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_copy_sys(const double2* a, double2* b, size_t n_per_sys, const int* frozen, hipStream_t st, SysBatch sb) {
  if (n_per_sys == 0) return MBBS_OK;
  int nb = (int)((n_per_sys + 255) / 256);
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_copy_sys, dim3(nb, sb.n), dim3(256), 0, st, a, b, n_per_sys, frozen, sb.fstride);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_fill(double2* p, size_t n, double2 v, hipStream_t st) {
  if (n == 0) return MBBS_OK;
  int nb = (int)((n + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, st, p, n, v);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_copy(const double2* a, double2* b, size_t n, hipStream_t st) {
  if (n == 0) return MBBS_OK;
  int nb = (int)((n + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, st, a, b, n);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_convert_to(int prec, size_t nsites, int L, const double2* x, void* y, float* ys, hipStream_t st) {
  const size_t n = nsites * L;
  if (n == 0) return MBBS_OK;
  dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (prec) {
    case P64: hipLaunchKernelGGL(k_conv_to<P64>, g, b, 0, st, nsites, L, x, (double2*)y, ys); break;
    case P32: hipLaunchKernelGGL(k_conv_to<P32>, g, b, 0, st, nsites, L, x, (float2*)y, ys); break;
    case P16: hipLaunchKernelGGL(k_conv_to<P16>, g, b, 0, st, nsites, L, x, (__half2*)y, ys); break;
    default: set_error("bad precision"); return MBBS_EINVAL;
  }
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int launch_convert_from(int prec, size_t nsites, int L, const void* x, const float* xs, double2* y, hipStream_t st) {
  const size_t n = nsites * L;
  if (n == 0) return MBBS_OK;
  dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (prec) {
    case P64: hipLaunchKernelGGL(k_conv_from<P64>, g, b, 0, st, nsites, L, (const double2*)x, xs, y); break;
    case P32: hipLaunchKernelGGL(k_conv_from<P32>, g, b, 0, st, nsites, L, (const float2*)x, xs, y); break;
    case P16: hipLaunchKernelGGL(k_conv_from<P16>, g, b, 0, st, nsites, L, (const __half2*)x, xs, y); break;
    default: set_error("bad precision"); return MBBS_EINVAL;
  }
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

}  // namespace mbbs

namespace mbbs {

// Standalone Cholesky factor + inverse (for the CholQR entry point):
// G (in) -> gamma (out, upper) and ginv; *ok = 0 if not positive definite.
__global__ void k_chol_standalone(int L, const double2* __restrict__ G, double2* __restrict__ gam,
                                  double2* __restrict__ ginv, int* __restrict__ ok) {
  extern __shared__ double2 sm[];
  double2* A = sm;
  double2* gi = sm + L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) A[e] = G[e];
  __syncthreads();
  bool good = chol_inv(L, A, gi);
  if (threadIdx.x == 0) *ok = good ? 1 : 0;
  if (!good) return;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) { gam[e] = A[e]; ginv[e] = gi[e]; }
}

// gam_out = g2 * g1 (combined R factor of two CholQR passes).
__global__ void k_matmul_small(int L, const double2* __restrict__ A, const double2* __restrict__ B,
                               double2* __restrict__ C) {
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
    int i = e / L, j = e % L;
    cplx<double> s = cmake(0.0, 0.0);
    for (int k = 0; k < L; ++k) s = s + ld2(A, i * L + k) * ld2(B, k * L + j);
    st2(C, e, s);
  }
}

__global__ void k_lu_standalone(int L, int m, const double2* __restrict__ G, const double2* __restrict__ R,
                                double2* __restrict__ X, int* __restrict__ ok) {
  extern __shared__ double2 sm[];
  double2* A = sm;
  double2* Rs = sm + L * L;
  double2* Xs = Rs + (size_t)L * m;
  __shared__ int piv[64];
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) A[e] = G[e];
  for (int e = threadIdx.x; e < L * m; e += blockDim.x) Rs[e] = R[e];
  __syncthreads();
  bool good = lu_factor(L, A, piv);
  if (threadIdx.x == 0) *ok = good ? 1 : 0;
  if (!good) return;
  lu_solve(L, m, A, piv, Rs, Xs, 1.0);
  for (int e = threadIdx.x; e < L * m; e += blockDim.x) X[e] = Xs[e];
}

int launch_chol_standalone(int L, const double2* G, double2* gam, double2* ginv, int* ok, hipStream_t st) {
  hipLaunchKernelGGL(k_chol_standalone, dim3(1), dim3(64), 2 * (size_t)L * L * sizeof(double2), st, L, G, gam, ginv, ok);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}
int launch_matmul_small(int L, const double2* A, const double2* B, double2* C, hipStream_t st) {
  hipLaunchKernelGGL(k_matmul_small, dim3(1), dim3(256), 0, st, L, A, B, C);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}
int launch_lu_standalone(int L, int m, const double2* G, const double2* R, double2* X, int* ok, hipStream_t st) {
  const size_t sh = ((size_t)L * L + 2 * (size_t)L * m) * sizeof(double2);
  hipLaunchKernelGGL(k_lu_standalone, dim3(1), dim3(64), sh, st, L, m, G, R, X, ok);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

}  // namespace mbbs
