// Multi-RHS Wilson hopping kernels (Sec. 2.1, block hopping-term equation):
// one thread owns one site and C consecutive right-hand sides, loads each of
// the 8 links once and applies it to all C columns (the link reuse across
// right-hand sides the paper builds its cache tuning on), accumulating the
// spin-projected hops in registers.  Variants: full operator, the
// domain-restricted (Dirichlet) operator of Sec. 2.2, the SAP residual
// eta - A psi, and the MR domain step with its per-domain reductions.
#include "stencil.h"
#include "tile.h"

namespace mbbs {

// ---------------------------------------------------------------- kernels
// Thread layout: threadIdx.x = column chunk (C columns each), threadIdx.y =
// site within the block; blocks cover consecutive sites of the field order.
template <int PIN, int POUT, int PL, int C, int ORDER, bool BLOCKED, bool PAIR = false, int LT = 0>
__global__ void __launch_bounds__(256) k_dslash(GeomK k, double kappa, int L,
                                                const typename Store<PIN>::Elem* __restrict__ in,
                                                const float* __restrict__ in_s,
                                                typename Store<POUT>::Elem* __restrict__ out,
                                                float* __restrict__ out_s,
                                                const LinkElem<PL>* __restrict__ U, int s0, int n,
                                                int bpt, int ngroups, const int* __restrict__ frozen) {
  // LT > 0: L known at compile time, so element offsets become immediates
  if constexpr (LT > 0) L = LT;
  using R = typename Store<PL>::Real;
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  if (i >= n) return;
  const int col0 = (grp * blockDim.x + threadIdx.x) * C;
  // lexicographic fields are walked tile by tile (whole lattice, s0 = 0)
  const SiteCtx c = ORDER == LEX ? site_ctx_tiled(k, i) : site_ctx<DM>(k, s0 + i);
  if (sys_frozen(k, frozen, c.sys)) return;
  const int s = c.s;
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  hop_sum<PIN, PL, C, ORDER, BLOCKED ? INSIDE : ALL, R, PAIR>(k, c, in, in_s, U, L, col0, acc);
  if (k.clov) clover_apply<ORDER, C, R>(k, s, acc);
  const R kap = (R)kappa_of(k, c, kappa);
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const size_t base = (size_t)s * 12 * L + col0 + q;
    cplx<R> v[4][3];
    load_spinor<PIN, R>(in, in_s, base, L, (size_t)s * L + col0 + q, v);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[sp][a] = v[sp][a] - kap * acc[sp][a][q];
    if (k.nt_store) store_spinor<POUT, R, true>(out, out_s, base, L, (size_t)s * L + col0 + q, v);
    else store_spinor<POUT, R>(out, out_s, base, L, (size_t)s * L + col0 + q, v);
  }
}

// SAP residual on the sites of one colour: r = eta - (psi - kappa H psi).
// mode 0: psi = 0 everywhere (first half-sweep): r = eta.
// mode 1: psi = 0 on this colour (second half-sweep of the first cycle): only
//         hops leaving the domain see a nonzero psi, r = eta + kappa H_out psi.
// mode 2: general case.
template <int PR, int PPSI, int PL, int C, bool PAIR = false, int LT = 0>
__global__ void __launch_bounds__(256) k_sap_resid(GeomK k, double kappa, int L, int s0, int n, int mode,
                                                   const typename Store<PR>::Elem* __restrict__ eta,
                                                   const float* __restrict__ eta_s,
                                                   const typename Store<PPSI>::Elem* __restrict__ psi,
                                                   typename Store<PR>::Elem* __restrict__ r,
                                                   float* __restrict__ r_s,
                                                   const LinkElem<PL>* __restrict__ U, int bpt,
                                                   int ngroups, const int* __restrict__ frozen) {
  if constexpr (LT > 0) L = LT;
  using R = typename Store<PL>::Real;
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  if (i >= n) return;
  const int s = s0 + i;
  const int col0 = (grp * blockDim.x + threadIdx.x) * C;
  const SiteCtx c = site_ctx<DM>(k, s);
  if (sys_frozen(k, frozen, c.sys)) return;
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  if (mode != 0) {
    if (mode == 1) hop_sum<PPSI, PL, C, DM, OUTSIDE, R, PAIR>(k, c, psi, nullptr, U, L, col0, acc);
    else hop_sum<PPSI, PL, C, DM, ALL, R, PAIR>(k, c, psi, nullptr, U, L, col0, acc);
    if (k.clov) clover_apply<DM, C, R>(k, s, acc);
  }
  const R kap = (R)kappa_of(k, c, kappa);
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const size_t base = (size_t)s * 12 * L + col0 + q;
    const size_t sidx = (size_t)s * L + col0 + q;
    cplx<R> e[4][3];
    load_spinor<PR, R>(eta, eta_s, base, L, sidx, e);
    if (mode != 0) {
      cplx<R> p[4][3];
      if (mode == 2) {
        load_spinor<PPSI, R>(psi, nullptr, base, L, sidx, p);
      } else {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) p[sp][a] = cmake<R>(0, 0);
      }
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) e[sp][a] = e[sp][a] - p[sp][a] + kap * acc[sp][a][q];
    }
    store_spinor<PR, R>(r, r_s, base, L, sidx, e);
  }
}

// MR step, part 1: w = A_DD r on one colour's domains, plus per-block sums of
// <w, r> and <w, w> per column.
template <int PR, int PL, int C, bool PAIR = false, int LT = 0>
__global__ void __launch_bounds__(256) k_mr_dslash(GeomK k, double kappa, int L, int s0, int n,
                                                   const typename Store<PR>::Elem* __restrict__ r,
                                                   const float* __restrict__ r_s,
                                                   typename Store<PR>::Elem* __restrict__ w,
                                                   float* __restrict__ w_s,
                                                   const LinkElem<PL>* __restrict__ U,
                                                   double* __restrict__ partial, int bpt, int ngroups,
                                                   const int* __restrict__ frozen) {
  if constexpr (LT > 0) L = LT;
  using R = typename Store<PL>::Real;
  extern __shared__ double red[];  // [3][blockDim.y][blockDim.x*C]
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  const int s = s0 + i;  // blocks never straddle domains
  const int colg = grp * blockDim.x * C;           // first column of the group
  const int col0 = colg + threadIdx.x * C;
  const SiteCtx c = site_ctx<DM>(k, s);
  // a block lies in one domain, hence one system: the test is block-uniform
  if (sys_frozen(k, frozen, c.sys)) return;
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  hop_sum<PR, PL, C, DM, INSIDE, R, PAIR>(k, c, r, r_s, U, L, col0, acc);
  if (k.clov) clover_apply<DM, C, R>(k, s, acc);
  const R kap = (R)kappa_of(k, c, kappa);
  const int ny = blockDim.y, nx = blockDim.x * C;
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const size_t base = (size_t)s * 12 * L + col0 + q;
    const size_t sidx = (size_t)s * L + col0 + q;
    cplx<R> v[4][3];
    load_spinor<PR, R>(r, r_s, base, L, sidx, v);
    double wr_re = 0, wr_im = 0, ww = 0;
    cplx<R> wv[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        wv[sp][a] = v[sp][a] - kap * acc[sp][a][q];
      }
    store_spinor<PR, R>(w, w_s, base, L, sidx, wv);
    if constexpr (Store<PR>::scaled) {
      // use the stored (rounded) w so that the update sees the same vector
      load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
    }
    R a_re = 0, a_im = 0, a_ww = 0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // <w, r> and <w, w> as FMA chains
        const cplx<R> x = wv[sp][a], y = v[sp][a];
        a_re = fmar(x.re, y.re, fmar(x.im, y.im, a_re));
        a_im = fmar(x.re, y.im, fmar(-x.im, y.re, a_im));
        a_ww = fmar(x.re, x.re, fmar(x.im, x.im, a_ww));
      }
    wr_re = a_re; wr_im = a_im; ww = a_ww;
    const int col = threadIdx.x * C + q;             // column within the group
    red[(0 * ny + threadIdx.y) * nx + col] = wr_re;
    red[(1 * ny + threadIdx.y) * nx + col] = wr_im;
    red[(2 * ny + threadIdx.y) * nx + col] = ww;
  }
  __syncthreads();
  // sum over the block's sites in fixed order, one thread per column chunk
  const int rel = i - threadIdx.y;                        // first site of the block in its colour
  const int dom = rel / k.g.Vb;                           // domain rank within the colour
  const int nblk = k.g.Vb / ny;
  const int bid = (rel % k.g.Vb) / ny;                    // block index inside the domain
  if (threadIdx.y == 0) {
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int col = threadIdx.x * C + q;
      double a0 = 0, a1 = 0, a2 = 0;
      for (int y = 0; y < ny; ++y) {
        a0 += red[(0 * ny + y) * nx + col];
        a1 += red[(1 * ny + y) * nx + col];
        a2 += red[(2 * ny + y) * nx + col];
      }
      double* pp = partial + (((size_t)dom * nblk + bid) * L + colg + col) * 3;
      pp[0] = a0; pp[1] = a1; pp[2] = a2;
    }
  }
}

// MR step, part 1b: per domain of the colour (one block each), sum the block
// partials in fixed order and form omega = <w, r> / <w, w> (0 if <w, w> = 0).
// A separate launch: the kernel boundary makes every block's partial visible
// without device-wide fences (which on this chip write back and invalidate the
// per-XCD L2 caches).
__global__ void __launch_bounds__(256) k_mr_omega(GeomK k, int L, int nblk, const double* __restrict__ partial,
                                                  double* __restrict__ omega, const int* __restrict__ frozen) {
  const int dom = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  __shared__ double red[3 * 256];
  const int G = nthr / L > 0 ? nthr / L : 1;
  const double* pp = partial + ((size_t)dom * nblk) * L * 3;
  for (int e = tid; e < G * L; e += nthr) {
    const int g = e / L, col = e % L;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int bb = g; bb < nblk; bb += G) {
      a0 += pp[((size_t)bb * L + col) * 3 + 0];
      a1 += pp[((size_t)bb * L + col) * 3 + 1];
      a2 += pp[((size_t)bb * L + col) * 3 + 2];
    }
    red[(0 * G + g) * L + col] = a0;
    red[(1 * G + g) * L + col] = a1;
    red[(2 * G + g) * L + col] = a2;
  }
  __syncthreads();
  for (int col = tid; col < L; col += nthr) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int gg = 0; gg < G; ++gg) {
      s0 += red[(0 * G + gg) * L + col];
      s1 += red[(1 * G + gg) * L + col];
      s2 += red[(2 * G + gg) * L + col];
    }
    double o_re = 0, o_im = 0;
    if (s2 > 0) { o_re = s0 / s2; o_im = s1 / s2; }
    omega[((size_t)dom * L + col) * 2 + 0] = o_re;
    omega[((size_t)dom * L + col) * 2 + 1] = o_im;
  }
}

// MR step, part 2: psi += omega r ; r -= omega w  (per domain and column).
template <int PR, int PPSI>
__global__ void __launch_bounds__(256) k_mr_update(GeomK k, int L, int s0, int n,
                                                   typename Store<PR>::Elem* __restrict__ r,
                                                   float* __restrict__ r_s,
                                                   const typename Store<PR>::Elem* __restrict__ w,
                                                   const float* __restrict__ w_s,
                                                   typename Store<PPSI>::Elem* __restrict__ psi,
                                                   const double* __restrict__ omega, int update_r,
                                                   int assign, const int* __restrict__ frozen) {
  using R = typename Store<PR>::Real;
  const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
  if (s >= s0 + n) return;
  const int col = threadIdx.x;
  const int dom = (s - (s >= k.g.Vh ? k.g.Vh : 0)) / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  const cplx<R> om = cmake<R>((R)omega[((size_t)dom * L + col) * 2], (R)omega[((size_t)dom * L + col) * 2 + 1]);
  const size_t base = (size_t)s * 12 * L + col;
  const size_t sidx = (size_t)s * L + col;
  cplx<R> rv[4][3];
  load_spinor<PR, R>(r, r_s, base, L, sidx, rv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      mr_psi_update<PPSI, R>(psi, base + (size_t)(3 * sp + a) * L, mr_mul(om, rv[sp][a]), assign);
  if (!update_r) return;
  cplx<R> wv[4][3];
  load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) rv[sp][a] = rv[sp][a] - mr_mul(om, wv[sp][a]);
  store_spinor<PR, R>(r, r_s, base, L, sidx, rv);
}

// The whole MR domain solve of one colour in one launch: one workgroup per
// domain runs the nmr steps (w = A_DD r, omega = <w, r> / <w, w>,
// psi += omega r, r -= omega w) with the domain-wide sums and the step-to-step
// dependence handled inside the workgroup (barriers only).  Thread t owns
// column t % L of the sites t / L, t / L + SPB, ... of its domain, so its
// per-column sums need no atomics and are combined in fixed order.
// r, w and psi are read and written by other threads of the workgroup
// between barriers, so they carry no restrict / const qualifiers here.
template <int PR> constexpr int mr_fused_threads() { return PR == P64 ? 512 : 1024; }

template <int PR, int PPSI, int PL>
__global__ void __launch_bounds__(mr_fused_threads<PR>()) k_mr_fused(GeomK k, double kappa, int L, int s0, int spb, int nmr,
                                                   int assign_first, typename Store<PR>::Elem* r, float* r_s,
                                                   typename Store<PR>::Elem* w, float* w_s,
                                                   typename Store<PPSI>::Elem* psi,
                                                   const LinkElem<PL>* __restrict__ U,
                                                   const int* __restrict__ frozen) {
  // one workgroup per domain, hence one system: the test is block-uniform
  const int sys = sys_of_domain(k, blockIdx.x);
  if (sys_frozen(k, frozen, sys)) return;
  using R = typename Store<PR>::Real;
  using RP = typename Store<PPSI>::Real;
  __shared__ double red[3][1024];
  __shared__ double om_sh[2 * 16];
  const int t = threadIdx.x;
  const int T = spb * L;
  const bool active = t < T;
  const int col = t % L, j = t / L;
  const int base_site = s0 + blockIdx.x * k.g.Vb;
  const R kap = (R)(k.kap ? k.kap[sys] : kappa);
  for (int it = 0; it < nmr; ++it) {
    double sr = 0, si = 0, sw = 0;
    if (active) {
      for (int loc = j; loc < k.g.Vb; loc += spb) {
        const int s = base_site + loc;
        const SiteCtx c = site_ctx<DM>(k, s);
        cplx<R> acc[4][3][1];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) acc[sp][a][0] = cmake<R>(0, 0);
        hop_sum<PR, PL, 1, DM, INSIDE, R>(k, c, r, r_s, U, L, col, acc);
        if (k.clov) clover_apply<DM, 1, R>(k, s, acc);
        const size_t base = (size_t)s * 12 * L + col;
        const size_t sidx = (size_t)s * L + col;
        cplx<R> v[4][3], wv[4][3];
        load_spinor<PR, R>(r, r_s, base, L, sidx, v);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) wv[sp][a] = v[sp][a] - kap * acc[sp][a][0];
        store_spinor<PR, R>(w, w_s, base, L, sidx, wv);
        if constexpr (Store<PR>::scaled) load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
        R a_re = 0, a_im = 0, a_ww = 0;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const cplx<R> x = wv[sp][a], y = v[sp][a];
            a_re = fmar(x.re, y.re, fmar(x.im, y.im, a_re));
            a_im = fmar(x.re, y.im, fmar(-x.im, y.re, a_im));
            a_ww = fmar(x.re, x.re, fmar(x.im, x.im, a_ww));
          }
        sr += a_re; si += a_im; sw += a_ww;
      }
    }
    red[0][t] = sr; red[1][t] = si; red[2][t] = sw;
    __syncthreads();
    if (t < L) {
      double a0 = 0, a1 = 0, a2 = 0;
      for (int jj = 0; jj < spb; ++jj) {
        a0 += red[0][jj * L + t];
        a1 += red[1][jj * L + t];
        a2 += red[2][jj * L + t];
      }
      om_sh[2 * t] = a2 > 0 ? a0 / a2 : 0.0;
      om_sh[2 * t + 1] = a2 > 0 ? a1 / a2 : 0.0;
    }
    __syncthreads();
    if (active) {
      const cplx<R> om = cmake<R>((R)om_sh[2 * col], (R)om_sh[2 * col + 1]);
      const bool assign = assign_first && it == 0, update_r = it + 1 < nmr;
      for (int loc = j; loc < k.g.Vb; loc += spb) {
        const int s = base_site + loc;
        const size_t base = (size_t)s * 12 * L + col;
        const size_t sidx = (size_t)s * L + col;
        cplx<R> rv[4][3];
        load_spinor<PR, R>(r, r_s, base, L, sidx, rv);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const size_t i = base + (size_t)(3 * sp + a) * L;
            cplx<R> d = om * rv[sp][a];
            if (assign) {
              Store<PPSI>::st(psi, i, cplx<RP>{(RP)d.re, (RP)d.im});
            } else {
              auto pv = Store<PPSI>::ld(psi, i);
              Store<PPSI>::st(psi, i, cplx<RP>{(RP)(pv.re + (RP)d.re), (RP)(pv.im + (RP)d.im)});
            }
          }
        if (update_r) {
          cplx<R> wv[4][3];
          load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
#pragma unroll
          for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) rv[sp][a] = rv[sp][a] - om * wv[sp][a];
          store_spinor<PR, R>(r, r_s, base, L, sidx, rv);
        }
      }
    }
    __syncthreads();
  }
}

// MR step, part 2, FP32 storage: the same update as a flat stream over the
// n*12*L complex entries of the colour, two adjacent entries (float4) per
// thread, for full-width coalesced loads and stores.  Entry e of site s,
// column j sits at (s*12 + e)*L + j, so both entries of a pair share the
// site (L even) and the domain.
__global__ void __launch_bounds__(256) k_mr_update_flat(GeomK k, int L, int s0, int n, float4* __restrict__ r,
                                                        const float4* __restrict__ w, float4* __restrict__ psi,
                                                        const double* __restrict__ omega, int update_r, int assign,
                                                        const int* __restrict__ frozen) {
  const size_t npair = (size_t)n * 6 * L;             // n*12*L entries, two per thread
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= npair) return;
  const size_t e0 = 2 * q;                             // first entry, relative to the colour
  const int col = (int)(e0 % L);
  const int s = (int)(e0 / (12 * (size_t)L));          // site within the colour
  const int dom = s / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  const double* om = omega + ((size_t)dom * L + col) * 2;
  const cplx<float> o0 = cmake((float)om[0], (float)om[1]), o1 = cmake((float)om[2], (float)om[3]);
  const size_t g = (size_t)s0 * 6 * L + q;             // float4 index in the whole field
  const float4 rv = r[g];
  const cplx<float> d0 = mr_mul(o0, cmake(rv.x, rv.y)), d1 = mr_mul(o1, cmake(rv.z, rv.w));
  if (assign) {
    psi[g] = make_float4(d0.re, d0.im, d1.re, d1.im);
  } else {
    const float4 p = psi[g];
    psi[g] = make_float4(p.x + d0.re, p.y + d0.im, p.z + d1.re, p.w + d1.im);
  }
  if (!update_r) return;
  const float4 wv = w[g];
  const cplx<float> m0 = mr_mul(o0, cmake(wv.x, wv.y)), m1 = mr_mul(o1, cmake(wv.z, wv.w));
  r[g] = make_float4(rv.x - m0.re, rv.y - m0.im, rv.z - m1.re, rv.w - m1.im);
}

// MR with psi formed once per domain solve (the MR steps of Sec. 2.2, with
// the sum psi = sum_k omega_k r_k regrouped).  Since r_k = r_0 - sum_{j<k}
// omega_j w_j,  sum_{k<n} omega_k r_k = c r_0 - sum_{j<n-1} e_j w_j  with
// c = sum_k omega_k and e_j = omega_j sum_{k>j} omega_k.  Between steps only
// r_{k+1} = r_k - omega_k w_k is formed; psi is read and written once, from r_0
// and the kept w_j, instead of at every step.
constexpr int MR_ONCE_MAX = 4;   // MR steps per domain solve in that form

struct MrOnceArgs {
  const void* r0;
  const float* r0_s;
  const void* w[MR_ONCE_MAX - 1];
  const float* w_s[MR_ONCE_MAX - 1];
};

// c and e_j of one domain and column from the steps' omega (stride apart).
__device__ __forceinline__ void mr_once_coefs(const double* omega, size_t stride, size_t idx, int nmr,
                                              cplx<double>& c, cplx<double> (&e)[MR_ONCE_MAX - 1]) {
  cplx<double> om[MR_ONCE_MAX];
#pragma unroll
  for (int k = 0; k < MR_ONCE_MAX; ++k)
    om[k] = k < nmr ? cmake(omega[k * stride + idx], omega[k * stride + idx + 1]) : cmake(0.0, 0.0);
  c = cmake(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < MR_ONCE_MAX; ++k) c = c + om[k];
  cplx<double> tail = cmake(0.0, 0.0);
#pragma unroll
  for (int j = MR_ONCE_MAX - 2; j >= 0; --j) {
    tail = tail + om[j + 1];
    e[j] = om[j] * tail;
  }
}

// r_out = r_in - omega w on one colour (r_out may be r_in).
template <int PR>
__global__ void __launch_bounds__(256) k_mr_rstep(GeomK k, int L, int s0, int n,
                                                  const typename Store<PR>::Elem* r_in, const float* r_in_s,
                                                  const typename Store<PR>::Elem* __restrict__ w,
                                                  const float* __restrict__ w_s, typename Store<PR>::Elem* r_out,
                                                  float* r_out_s, const double* __restrict__ omega,
                                                  const int* __restrict__ frozen) {
  using R = typename Store<PR>::Real;
  const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
  if (s >= s0 + n) return;
  const int col = threadIdx.x;
  const int dom = (s - (s >= k.g.Vh ? k.g.Vh : 0)) / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  const cplx<R> om = cmake<R>((R)omega[((size_t)dom * L + col) * 2], (R)omega[((size_t)dom * L + col) * 2 + 1]);
  const size_t base = (size_t)s * 12 * L + col;
  const size_t sidx = (size_t)s * L + col;
  cplx<R> rv[4][3], wv[4][3];
  load_spinor<PR, R>(r_in, r_in_s, base, L, sidx, rv);
  load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) rv[sp][a] = rv[sp][a] - mr_mul(om, wv[sp][a]);
  store_spinor<PR, R>(r_out, r_out_s, base, L, sidx, rv);
}

// The same for FP32 storage as a flat stream of float4 (two columns).
__global__ void __launch_bounds__(256) k_mr_rstep_flat(GeomK k, int L, int s0, int n, const float4* r_in,
                                                       const float4* __restrict__ w, float4* r_out,
                                                       const double* __restrict__ omega,
                                                       const int* __restrict__ frozen) {
  const size_t npair = (size_t)n * 6 * L;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= npair) return;
  const size_t e0 = 2 * q;
  const int col = (int)(e0 % L);
  const int s = (int)(e0 / (12 * (size_t)L));
  const int dom = s / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  const double* om = omega + ((size_t)dom * L + col) * 2;
  const cplx<float> o0 = cmake((float)om[0], (float)om[1]), o1 = cmake((float)om[2], (float)om[3]);
  const size_t g = (size_t)s0 * 6 * L + q;
  const float4 rv = r_in[g], wv = w[g];
  const cplx<float> m0 = mr_mul(o0, cmake(wv.x, wv.y)), m1 = mr_mul(o1, cmake(wv.z, wv.w));
  r_out[g] = make_float4(rv.x - m0.re, rv.y - m0.im, rv.z - m1.re, rv.w - m1.im);
}

// psi (+)= c r_0 - sum_{j<nmr-1} e_j w_j on one colour (assign: =).
template <int PR, int PPSI>
__global__ void __launch_bounds__(256) k_mr_psi_once(GeomK k, int L, int s0, int n, MrOnceArgs a,
                                                     typename Store<PPSI>::Elem* __restrict__ psi,
                                                     const double* __restrict__ omega, size_t ostride, int nmr,
                                                     int assign, const int* __restrict__ frozen) {
  using R = typename Store<PR>::Real;
  using E = typename Store<PR>::Elem;
  const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
  if (s >= s0 + n) return;
  const int col = threadIdx.x;
  const int dom = (s - (s >= k.g.Vh ? k.g.Vh : 0)) / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  cplx<double> cd, ed[MR_ONCE_MAX - 1];
  mr_once_coefs(omega, ostride, ((size_t)dom * L + col) * 2, nmr, cd, ed);
  const size_t base = (size_t)s * 12 * L + col;
  const size_t sidx = (size_t)s * L + col;
  cplx<R> v[4][3], acc[4][3];
  load_spinor<PR, R>((const E*)a.r0, a.r0_s, base, L, sidx, v);
  const cplx<R> c = cmake<R>((R)cd.re, (R)cd.im);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[sp][q] = mr_mul(c, v[sp][q]);
#pragma unroll
  for (int j = 0; j < MR_ONCE_MAX - 1; ++j) {
    if (j >= nmr - 1) break;
    const cplx<R> e = cmake<R>((R)ed[j].re, (R)ed[j].im);
    load_spinor<PR, R>((const E*)a.w[j], a.w_s[j], base, L, sidx, v);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[sp][q] = acc[sp][q] - mr_mul(e, v[sp][q]);
  }
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int q = 0; q < 3; ++q) mr_psi_update<PPSI, R>(psi, base + (size_t)(3 * sp + q) * L, acc[sp][q], assign);
}

// The same for FP32 storage and FP32 psi as a flat stream of float4.
__global__ void __launch_bounds__(256) k_mr_psi_once_flat(GeomK k, int L, int s0, int n, MrOnceArgs a,
                                                          float4* __restrict__ psi, const double* __restrict__ omega,
                                                          size_t ostride, int nmr, int assign,
                                                          const int* __restrict__ frozen) {
  const size_t npair = (size_t)n * 6 * L;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= npair) return;
  const size_t e0 = 2 * q;
  const int col = (int)(e0 % L);
  const int s = (int)(e0 / (12 * (size_t)L));
  const int dom = s / k.g.Vb;
  if (sys_frozen(k, frozen, sys_of_domain(k, dom))) return;
  cplx<double> cd0, cd1, ed0[MR_ONCE_MAX - 1], ed1[MR_ONCE_MAX - 1];
  mr_once_coefs(omega, ostride, ((size_t)dom * L + col) * 2, nmr, cd0, ed0);
  mr_once_coefs(omega, ostride, ((size_t)dom * L + col + 1) * 2, nmr, cd1, ed1);
  const size_t g = (size_t)s0 * 6 * L + q;
  const float4 r0 = ((const float4*)a.r0)[g];
  cplx<float> d0 = mr_mul(cmake((float)cd0.re, (float)cd0.im), cmake(r0.x, r0.y));
  cplx<float> d1 = mr_mul(cmake((float)cd1.re, (float)cd1.im), cmake(r0.z, r0.w));
#pragma unroll
  for (int j = 0; j < MR_ONCE_MAX - 1; ++j) {
    if (j >= nmr - 1) break;
    const float4 wv = ((const float4*)a.w[j])[g];
    d0 = d0 - mr_mul(cmake((float)ed0[j].re, (float)ed0[j].im), cmake(wv.x, wv.y));
    d1 = d1 - mr_mul(cmake((float)ed1[j].re, (float)ed1[j].im), cmake(wv.z, wv.w));
  }
  if (assign) {
    psi[g] = make_float4(d0.re, d0.im, d1.re, d1.im);
  } else {
    const float4 p = psi[g];
    psi[g] = make_float4(p.x + d0.re, p.y + d0.im, p.z + d1.re, p.w + d1.im);
  }
}

// ---------------------------------------------------------------- split-wave kernels
// Block = (IPB items) x (P hop groups); item = (site, column), IPB = S * L is a
// multiple of the wave size so every wave belongs to one hop group.  Group h
// sums its hops (hop_group), the P partial sums meet in LDS, and group h then
// finishes spins h*(4/P) .. h*(4/P)+4/P-1 of every item.  Compared with one
// thread per site doing all eight hops, a site has P times more loads in
// flight and P times fewer sites are resident per CU, so the neighbour data
// of the resident sites fits the XCD's L2 better.
template <typename R>
struct SplitSmem {
  cplx<R>* xs;    // [P][IPB][12] partial hop sums
  R* mx;          // [P][IPB] partial maxima (FP16 storage scale)
};
template <typename R>
__device__ __forceinline__ SplitSmem<R> split_smem(int P, int IPB) {
  extern __shared__ unsigned char smem_raw[];
  SplitSmem<R> m;
  m.xs = (cplx<R>*)smem_raw;
  m.mx = (R*)(smem_raw + (size_t)P * IPB * 12 * sizeof(cplx<R>));
  return m;
}

// Final value of this group's spins: v = base + coef * (sum over groups).
template <int P, typename R>
__device__ __forceinline__ void split_total(const SplitSmem<R>& m, int h, int item, int IPB,
                                            cplx<R> (&tot)[4 / P][3]) {
  constexpr int NS = 4 / P;
#pragma unroll
  for (int t = 0; t < NS; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> sum = cmake<R>(0, 0);
#pragma unroll
      for (int g = 0; g < P; ++g) sum = sum + m.xs[((size_t)g * IPB + item) * 12 + 3 * (h * NS + t) + a];
      tot[t][a] = sum;
    }
}

template <int P, typename R>
__device__ __forceinline__ void split_publish(const SplitSmem<R>& m, int h, int item, int IPB,
                                              const cplx<R> (&acc)[4][3][1]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) m.xs[((size_t)h * IPB + item) * 12 + 3 * sp + a] = acc[sp][a][0];
}

// Store this group's spins of one (site, column); FP16 storage exchanges the
// groups' maxima first so that all of them use the same scale.
template <int POUT, int P, typename R, bool NT = false>
__device__ __forceinline__ void split_store(const SplitSmem<R>& m, int h, int item, int IPB, bool active,
                                            typename Store<POUT>::Elem* out, float* out_s, size_t base, int L,
                                            size_t sidx, cplx<R> (&v)[4 / P][3]) {
  constexpr int NS = 4 / P;
  if constexpr (Store<POUT>::scaled) {
    R mloc = 0;
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int a = 0; a < 3; ++a) mloc = fmaxf(mloc, fmaxf(fabsf(v[t][a].re), fabsf(v[t][a].im)));
    m.mx[(size_t)h * IPB + item] = mloc;
    __syncthreads();
    R mx = 0;
#pragma unroll
    for (int g = 0; g < P; ++g) mx = fmaxf(mx, m.mx[(size_t)g * IPB + item]);
    if (!active) return;
    if (h == 0) out_s[sidx] = mx;
    const R inv = mx > 0 ? (R)1 / mx : (R)0;
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if constexpr (NT) Store<POUT>::st_nt(out, base + (size_t)(3 * (h * NS + t) + a) * L, inv * v[t][a]);
        else Store<POUT>::st(out, base + (size_t)(3 * (h * NS + t) + a) * L, inv * v[t][a]);
      }
  } else {
    if (!active) return;
    using RO = typename Store<POUT>::Real;
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if constexpr (NT) Store<POUT>::st_nt(out, base + (size_t)(3 * (h * NS + t) + a) * L, cplx<RO>{(RO)v[t][a].re, (RO)v[t][a].im});
        else Store<POUT>::st(out, base + (size_t)(3 * (h * NS + t) + a) * L, cplx<RO>{(RO)v[t][a].re, (RO)v[t][a].im});
      }
  }
}

// This group's spins of one stored (site, column) spinor.
template <int PIN, int P, typename R>
__device__ __forceinline__ void split_load(const typename Store<PIN>::Elem* in, const float* in_s, size_t base,
                                           int L, size_t sidx, int h, cplx<R> (&v)[4 / P][3]) {
  constexpr int NS = 4 / P;
  R sc = 1;
  if constexpr (Store<PIN>::scaled) sc = (R)in_s[sidx];
#pragma unroll
  for (int t = 0; t < NS; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      auto e = Store<PIN>::ld(in, base + (size_t)(3 * (h * NS + t) + a) * L);
      v[t][a] = cmake<R>((R)e.re * sc, (R)e.im * sc);
    }
}

template <int PIN, int POUT, int PL, int ORDER, bool BLOCKED, int P>
__global__ void __launch_bounds__(768) k_dslash_split(GeomK k, double kappa, int L,
                                                       const typename Store<PIN>::Elem* __restrict__ in,
                                                       const float* __restrict__ in_s,
                                                       typename Store<POUT>::Elem* __restrict__ out,
                                                       float* __restrict__ out_s,
                                                       const LinkElem<PL>* __restrict__ U, int s0, int n, int S,
                                                       const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  const int IPB = blockDim.x, h = threadIdx.y, item = threadIdx.x;
  const int lsite = item / L, col = item - lsite * L;
  const SplitSmem<R> m = split_smem<R>(P, IPB);
  const PersistRange pr = persist_range((n + S - 1) / S);
  for (int lb = pr.first; lb < pr.end; lb += pr.step) {
  const int i = lb * S + lsite;
  const bool active = i < n;
  const SiteCtx c = ORDER == LEX ? site_ctx_tiled(k, active ? i : 0) : site_ctx<DM>(k, s0 + (active ? i : 0));
  cplx<R> acc[4][3][1];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[sp][a][0] = cmake<R>(0, 0);
  if (active) hop_group<PIN, PL, ORDER, BLOCKED ? INSIDE : ALL, P, R>(h, k, c, in, in_s, U, L, col, acc);
  split_publish<P, R>(m, h, item, IPB, acc);
  __syncthreads();
  cplx<R> tot[4 / P][3], v[4 / P][3];
  split_total<P, R>(m, h, item, IPB, tot);
  const size_t base = (size_t)c.s * 12 * L + col, sidx = (size_t)c.s * L + col;
  if (active) split_load<PIN, P, R>(in, in_s, base, L, sidx, h, v);
  const R kap = (R)kappa;
#pragma unroll
  for (int t = 0; t < 4 / P; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[t][a] = v[t][a] - kap * tot[t][a];
  if (k.nt_store) split_store<POUT, P, R, true>(m, h, item, IPB, active, out, out_s, base, L, sidx, v);
  else split_store<POUT, P, R>(m, h, item, IPB, active, out, out_s, base, L, sidx, v);
  __syncthreads();   // the exchange area is reused by the next logical block
  }
}

// Split-wave SAP residual on one colour (modes as in k_sap_resid).
template <int PR, int PPSI, int PL, int P>
__global__ void __launch_bounds__(768) k_sap_resid_split(GeomK k, double kappa, int L, int s0, int n, int mode,
                                                          const typename Store<PR>::Elem* __restrict__ eta,
                                                          const float* __restrict__ eta_s,
                                                          const typename Store<PPSI>::Elem* __restrict__ psi,
                                                          typename Store<PR>::Elem* __restrict__ r,
                                                          float* __restrict__ r_s,
                                                          const LinkElem<PL>* __restrict__ U, int S,
                                                          const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  const int IPB = blockDim.x, h = threadIdx.y, item = threadIdx.x;
  const int lsite = item / L, col = item - lsite * L;
  const SplitSmem<R> m = split_smem<R>(P, IPB);
  const PersistRange pr = persist_range((n + S - 1) / S);
  for (int lb = pr.first; lb < pr.end; lb += pr.step) {
  const int i = lb * S + lsite;
  const bool active = i < n;
  const int s = s0 + (active ? i : 0);
  cplx<R> acc[4][3][1];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[sp][a][0] = cmake<R>(0, 0);
  if (active && mode != 0) {
    const SiteCtx c = site_ctx<DM>(k, s);
    if (mode == 1) hop_group<PPSI, PL, DM, OUTSIDE, P, R>(h, k, c, psi, nullptr, U, L, col, acc);
    else hop_group<PPSI, PL, DM, ALL, P, R>(h, k, c, psi, nullptr, U, L, col, acc);
  }
  split_publish<P, R>(m, h, item, IPB, acc);
  __syncthreads();
  cplx<R> tot[4 / P][3], e[4 / P][3], pv[4 / P][3];
  split_total<P, R>(m, h, item, IPB, tot);
  const size_t base = (size_t)s * 12 * L + col, sidx = (size_t)s * L + col;
  if (active) {
    split_load<PR, P, R>(eta, eta_s, base, L, sidx, h, e);
    if (mode == 2) split_load<PPSI, P, R>(psi, nullptr, base, L, sidx, h, pv);
  }
  const R kap = (R)kappa;
#pragma unroll
  for (int t = 0; t < 4 / P; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (mode == 2) e[t][a] = e[t][a] - pv[t][a];
      if (mode != 0) e[t][a] = e[t][a] + kap * tot[t][a];
    }
  split_store<PR, P, R>(m, h, item, IPB, active, r, r_s, base, L, sidx, e);
  __syncthreads();
  }
}

// Split-wave MR step, part 1: w = A_DD r on one colour plus per-block sums of
// <w, r> and <w, w> per column.  S divides the block volume, so a block never
// straddles two domains.
template <int PR, int PL, int P>
__global__ void __launch_bounds__(768) k_mr_dslash_split(GeomK k, double kappa, int L, int s0, int n,
                                                          const typename Store<PR>::Elem* __restrict__ r,
                                                          const float* __restrict__ r_s,
                                                          typename Store<PR>::Elem* __restrict__ w,
                                                          float* __restrict__ w_s,
                                                          const LinkElem<PL>* __restrict__ U,
                                                          double* __restrict__ partial, int S,
                                                          const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  const int IPB = blockDim.x, h = threadIdx.y, item = threadIdx.x;
  const int lsite = item / L, col = item - lsite * L;
  const SplitSmem<R> m = split_smem<R>(P, IPB);
  const PersistRange pr = persist_range(n / S);
  for (int lb = pr.first; lb < pr.end; lb += pr.step) {
  const int i = lb * S + lsite;
  const int s = s0 + i;
  const SiteCtx c = site_ctx<DM>(k, s);
  cplx<R> acc[4][3][1];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[sp][a][0] = cmake<R>(0, 0);
  hop_group<PR, PL, DM, INSIDE, P, R>(h, k, c, r, r_s, U, L, col, acc);
  split_publish<P, R>(m, h, item, IPB, acc);
  __syncthreads();
  cplx<R> tot[4 / P][3], rv[4 / P][3], wv[4 / P][3];
  split_total<P, R>(m, h, item, IPB, tot);
  const size_t base = (size_t)s * 12 * L + col, sidx = (size_t)s * L + col;
  split_load<PR, P, R>(r, r_s, base, L, sidx, h, rv);
  const R kap = (R)kappa;
#pragma unroll
  for (int t = 0; t < 4 / P; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) wv[t][a] = rv[t][a] - kap * tot[t][a];
  split_store<PR, P, R>(m, h, item, IPB, true, w, w_s, base, L, sidx, wv);
  if constexpr (Store<PR>::scaled) {
    __syncthreads();   // make the stored halves visible to this thread's reload
    split_load<PR, P, R>(w, w_s, base, L, sidx, h, wv);
  }
  double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int t = 0; t < 4 / P; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> d = cdot(wv[t][a], rv[t][a]);
      a0 += d.re; a1 += d.im; a2 += norm2(wv[t][a]);
    }
  // reduce over (group, site) per column in fixed order, reusing the exchange area
  __syncthreads();
  double* red = (double*)m.xs;   // [3][P][IPB]
  red[(0 * P + h) * IPB + item] = a0;
  red[(1 * P + h) * IPB + item] = a1;
  red[(2 * P + h) * IPB + item] = a2;
  __syncthreads();
  if (h == 0 && lsite == 0) {
    double s0v = 0, s1v = 0, s2v = 0;
    for (int g = 0; g < P; ++g)
      for (int y = 0; y < S; ++y) {
        s0v += red[(0 * P + g) * IPB + y * L + col];
        s1v += red[(1 * P + g) * IPB + y * L + col];
        s2v += red[(2 * P + g) * IPB + y * L + col];
      }
    const int dom = i / k.g.Vb, nblk = k.g.Vb / S, bid = (i % k.g.Vb) / S;
    double* pp = partial + (((size_t)dom * nblk + bid) * L + col) * 3;
    pp[0] = s0v; pp[1] = s1v; pp[2] = s2v;
  }
  __syncthreads();
  }
}

// ---------------------------------------------------------------- host side
GeomK make_geomk(const Geom& g, int nsys) {
  GeomK k;
  k.g = g;
  k.nsys = nsys;
  k.tsys = g.d[3] / nsys;
  k.ndt = g.nd[3] / nsys;
  k.Vsys = g.V / nsys;
  k.ftsys = make_fastdiv(k.tsys);
  k.fndt = make_fastdiv(k.ndt);
  k.kap = nullptr;
  k.fstride = SOLVER_FLAG_STRIDE;
  for (int m = 0; m < 4; ++m) {
    k.fd[m] = make_fastdiv(g.d[m]);
    k.fb[m] = make_fastdiv(g.b[m]);
  }
  k.fnd0 = make_fastdiv(g.nd[0]);
  for (int m = 0; m < 4; ++m) k.fnd[m] = make_fastdiv(g.nd[m]);
  k.fVb = make_fastdiv(g.Vb);
  k.nt_store = 0;
  for (int o = 0; o < 2; ++o) { k.cinv64[o] = nullptr; k.cinv32[o] = nullptr; }
  k.clov = 0;
  k.lstride[0] = 1;
  k.stride[0] = 1;
  for (int m = 1; m < 4; ++m) {
    k.lstride[m] = k.lstride[m - 1] * g.b[m - 1];
    k.stride[m] = k.stride[m - 1] * g.d[m - 1];
  }
  return k;
}

// Sites per block so that blockDim = (L/C, S) has about `target` threads and S
// divides `vdiv` (so blocks never straddle SAP domains when vdiv = Vb).
static int sites_per_block(int nchunk, int vdiv, int target = 256) {
  int best = 1;
  for (int s = 1; s * nchunk <= target; ++s)
    if (vdiv % s == 0) best = s;
  return best;
}

// Launch plan of a stencil kernel over `nsites` sites (a multiple of the
// SAP block volume): C columns per thread, column groups of gw columns,
// S sites per block, bpt blocks per tile.
struct Plan {
  int C, gw, nchunk, ngroups, S, bpt, nblocks;
};
static Plan make_plan(const mbbs_lattice_s* lat, int L, int prec, int nsites) {
  Plan p;
  p.C = pick_chunk(lat, L, prec);
  p.gw = lat->group_cols[prec];
  if (p.gw <= 0 || p.gw % p.C || L % p.gw) p.gw = L;
  p.nchunk = p.gw / p.C;
  p.ngroups = L / p.gw;
  p.S = sites_per_block(p.nchunk, lat->g.Vb, lat->block_threads[prec]);
  p.bpt = lat->g.Vb / p.S;
  p.nblocks = (nsites / lat->g.Vb) * p.ngroups * p.bpt;
  return p;
}

// Sites per block of a split-wave launch: S divides the block volume, S*L is
// a multiple of the wave size and at most 256, P*S*L <= 768 threads, and the
// exchange area fits the 160 KiB LDS.  0 if no such S exists.
static int split_sites(const mbbs_lattice_s* lat, int L, int prec, int P) {
  const size_t rb = prec == P64 ? 8 : 4;
  int best = 0;
  for (int S = 1; S * L <= 256; ++S) {
    if (lat->g.Vb % S || (S * L) % 64 || P * S * L > 768) continue;
    const size_t smem = (size_t)P * S * L * (24 * rb + rb);
    if (smem > 160 * 1024) continue;
    best = S;
  }
  return best;
}
static size_t split_smem_bytes(int prec, int P, int S, int L) {
  const size_t rb = prec == P64 ? 8 : 4;
  return (size_t)P * S * L * (24 * rb + rb);
}
// Grid of a split-wave launch: one block per logical block (rounded up to a
// multiple of 8 for the XCD mapping), or, with the persistent-blocks knob, a
// fixed number of resident blocks per CU that loop over their XCD's range.
static int split_grid(const mbbs_lattice_s* lat, int prec, int P, int S, int L, int nlb) {
  (void)prec; (void)P; (void)S; (void)L;
  int g = ((nlb + 7) / 8) * 8;
  if (lat->persist_blocks > 0 && 256 * lat->persist_blocks < g) g = 256 * lat->persist_blocks;
  return g < 8 ? 8 : g;
}

// Allow dynamic LDS above the 64 KiB default for a kernel (once per kernel).
static void allow_lds(const void* fn) {
  static const void* seen[64];
  static int nseen = 0;
  for (int i = 0; i < nseen; ++i)
    if (seen[i] == fn) return;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (nseen < 64) seen[nseen++] = fn;
}

template <int PIN, int POUT, int PL, int P>
static int dslash_split_launch(const mbbs_lattice_s* lat, int L, int order, bool blocked, const void* in,
                               const float* in_s, void* out, float* out_s, int s0, int n, int S, const int* frozen,
                               hipStream_t st) {
  const void* U;
  if (order == LEX) U = PL == P64 ? (const void*)lat->U64 : PL == P32 ? (const void*)lat->U32 : (const void*)lat->U16;
  else U = PL == P64 ? (const void*)lat->U64dm : PL == P32 ? (const void*)lat->U32dm : (const void*)lat->U16dm;
  using EI = typename Store<PIN>::Elem;
  using EO = typename Store<POUT>::Elem;
  using EL = LinkElem<PL>;
  const size_t smem = split_smem_bytes(PL, P, S, L);
  dim3 blk(S * L, P), grd(split_grid(lat, PL, P, S, L, ceil_div(n, S)));
  GeomK gk = lat->gk;
  gk.nt_store = lat->nt_store[PL];
#define SL(ORD, BLK)                                                                                    \
  do {                                                                                                  \
    auto fn = k_dslash_split<PIN, POUT, PL, ORD, BLK, P>;                                               \
    allow_lds((const void*)fn);                                                                         \
    hipLaunchKernelGGL(fn, grd, blk, smem, st, gk, lat->kappa, L, (const EI*)in, in_s, (EO*)out,        \
                       out_s, (const EL*)U, s0, n, S, frozen);                                          \
  } while (0)
  if (order == LEX) { if (blocked) SL(LEX, true); else SL(LEX, false); }
  else { if (blocked) SL(DM, true); else SL(DM, false); }
#undef SL
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

template <int PIN, int POUT, int PL, int C>
static int dslash_dispatch_order(const mbbs_lattice_s* lat, int L, int order, bool blocked,
                                 const void* in, const float* in_s, void* out, float* out_s,
                                 int s0, int n, const int* frozen, hipStream_t st) {
  const Plan pl = make_plan(lat, L, PL, n);
  dim3 blk(pl.nchunk, pl.S);
  dim3 grd(pl.nblocks);
  const void* U;
  if (order == LEX) U = PL == P64 ? (const void*)lat->U64 : PL == P32 ? (const void*)lat->U32 : (const void*)lat->U16;
  else U = PL == P64 ? (const void*)lat->U64dm : PL == P32 ? (const void*)lat->U32dm : (const void*)lat->U16dm;
  using EI = typename Store<PIN>::Elem;
  using EO = typename Store<POUT>::Elem;
  using EL = LinkElem<PL>;
  GeomK gk = lat->gk;
  gk.nt_store = lat->nt_store[PL];
#define MBBS_LAUNCH(ORD, BLK)                                                                   \
  hipLaunchKernelGGL((k_dslash<PIN, POUT, PL, C, ORD, BLK>), grd, blk, (size_t)lat->lds_pad_kb * 1024, st,     \
                     gk, lat->kappa, L,                                                                     \
                     (const EI*)in, in_s, (EO*)out, out_s, (const EL*)U, s0, n, pl.bpt, pl.ngroups, frozen)
  if (order == LEX) {
    if (blocked) MBBS_LAUNCH(LEX, true);
    else if (C <= 2 && L == 12) {   // the common block width, with compile-time element offsets
      if constexpr (C <= 2) {
        if (lat->hop_pair[PL])
          hipLaunchKernelGGL((k_dslash<PIN, POUT, PL, C, LEX, false, true, 12>), grd, blk,
                             (size_t)lat->lds_pad_kb * 1024, st, gk, lat->kappa, L, (const EI*)in, in_s, (EO*)out,
                             out_s, (const EL*)U, s0, n, pl.bpt, pl.ngroups, frozen);
        else
          hipLaunchKernelGGL((k_dslash<PIN, POUT, PL, C, LEX, false, false, 12>), grd, blk,
                             (size_t)lat->lds_pad_kb * 1024, st, gk, lat->kappa, L, (const EI*)in, in_s, (EO*)out,
                             out_s, (const EL*)U, s0, n, pl.bpt, pl.ngroups, frozen);
      }
    } else if (lat->hop_pair[PL])
      hipLaunchKernelGGL((k_dslash<PIN, POUT, PL, C, LEX, false, true>), grd, blk, (size_t)lat->lds_pad_kb * 1024, st,
                         gk, lat->kappa, L, (const EI*)in, in_s, (EO*)out, out_s, (const EL*)U, s0, n, pl.bpt,
                         pl.ngroups, frozen);
    else MBBS_LAUNCH(LEX, false);
  } else {
    if (blocked) MBBS_LAUNCH(DM, true); else MBBS_LAUNCH(DM, false);
  }
#undef MBBS_LAUNCH
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

template <int PIN, int POUT, int PL>
static int dslash_dispatch_c(const mbbs_lattice_s* lat, int L, int order, bool blocked,
                             const void* in, const float* in_s, void* out, float* out_s, int s0,
                             int n, const int* frozen, hipStream_t st) {
  if constexpr (PIN == POUT && PIN == PL) {
    TileArgs T;
    const bool whole = order == LEX ? (s0 == 0 && n == lat->g.V) : (s0 % lat->g.Vb == 0 && n % lat->g.Vb == 0);
    // the tiled kernels move two FP32 columns as one 16-byte access: both
    // fields 16-byte aligned, else the column-by-column kernel below
    const bool al = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
    if (whole && al && tile_plan(lat, L, PL, &T))
      return launch_dslash_tiled(lat, L, PL, order, blocked, T, in, in_s, out, out_s, s0, n, frozen, st);
  }
  const int P = lat->nsys == 1 ? lat->split[PL] : 0;   // the split kernels serve single systems only
  if ((P == 2 || P == 4) && !lat->gk.clov) {   // the split kernels have no clover step
    const int S = split_sites(lat, L, PL, P);
    if (S > 0) {
      if (P == 4) return dslash_split_launch<PIN, POUT, PL, 4>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, S, frozen, st);
      return dslash_split_launch<PIN, POUT, PL, 2>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, S, frozen, st);
    }
  }
  switch (pick_chunk(lat, L, PL)) {
    case 4: return dslash_dispatch_order<PIN, POUT, PL, 4>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
    case 3: return dslash_dispatch_order<PIN, POUT, PL, 3>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
    case 2: return dslash_dispatch_order<PIN, POUT, PL, 2>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
    default: return dslash_dispatch_order<PIN, POUT, PL, 1>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
  }
}

int launch_dslash(const mbbs_lattice_s* lat, int L, int prec_in, int prec_out, int order,
                  bool blocked, const void* in, const float* in_s, void* out, float* out_s,
                  int s0, int n, const int* frozen, hipStream_t st) {
  if (n <= 0) return MBBS_OK;
  if (prec_in == P64 && prec_out == P64)
    return dslash_dispatch_c<P64, P64, P64>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
  if (prec_in == P32 && prec_out == P64)
    return dslash_dispatch_c<P32, P64, P64>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
  if (prec_in == P32 && prec_out == P32)
    return dslash_dispatch_c<P32, P32, P32>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
  if (prec_in == P16 && prec_out == P16)
    return dslash_dispatch_c<P16, P16, P16>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, frozen, st);
  set_error("unsupported precision combination");
  return MBBS_EINVAL;
}

// ---------------------------------------------------------------- SAP host
// Whether the MR steps of this precision fold the previous step's update in.
static bool folded_mr(const mbbs_lattice_s* lat, int prec) { return lat->tile[prec] == 2 && prec != P16; }

// Whether MR domain solves form psi once (needs a second r and three more w).
static bool once_mr(const mbbs_lattice_s* lat, int prec) { return lat->mr_once[prec] == 1; }

static size_t sap_bytes(const mbbs_lattice_s* lat, int L, int prec, bool ssor, bool folded, bool once = false) {
  const size_t V = lat->g.V;
  const size_t elem = prec == P64 ? 16 : prec == P32 ? 8 : 4;
  const size_t field = V * 12 * L * elem;
  const size_t scales = prec == P16 ? V * L * sizeof(float) : 0;
  const size_t psi = V * 12 * L * (prec == P64 ? 16 : 8);
  const size_t ndc = lat->g.ndom / 2;             // domains per colour
  const size_t nblk = lat->g.Vh;                  // upper bound on blocks per colour
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  // eta, r, w; x2 (SSOR); a second r and w for the folded MR update (tiled,
  // setting 2: included only while that setting is on)
  // psi once: a second r (r2) and w2 plus wx[0], wx[1]
  const size_t nf = ssor ? 4 : (once ? 7 : (folded ? 5 : 3));
  return al(field) * nf + al(scales) * nf + al(psi) + al(nblk * L * 3 * sizeof(double)) +
         al(ndc * L * 2 * sizeof(double) * MR_ONCE_MAX);
}

size_t sap_buffer_bytes(const mbbs_lattice_s* lat, int L, int prec, bool ssor) {
  return sap_bytes(lat, L, prec, ssor, !ssor && folded_mr(lat, prec), !ssor && once_mr(lat, prec));
}

int sap_bind(const mbbs_lattice_s* lat, int L, int prec, void* ws, size_t bytes, SapBuffers* b, bool ssor) {
  // the folded MR update's buffers are bound only if the workspace holds
  // them (sized while that setting was on); otherwise the MR steps run unfolded
  const bool folded = !ssor && folded_mr(lat, prec);
  MBBS_CHECK(ws != nullptr && bytes >= sap_bytes(lat, L, prec, ssor, false), "SAP workspace too small");
  const size_t V = lat->g.V;
  const size_t elem = prec == P64 ? 16 : prec == P32 ? 8 : 4;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* p = (char*)ws;
  const size_t field = al(V * 12 * L * elem);
  const size_t scales = al(prec == P16 ? V * L * sizeof(float) : 0);
  b->L = L;
  b->prec = prec;
  b->eta = p; p += field;
  b->r = p; p += field;
  b->w = p; p += field;
  b->eta_s = prec == P16 ? (float*)p : nullptr; p += scales;
  b->r_s = prec == P16 ? (float*)p : nullptr; p += scales;
  b->w_s = prec == P16 ? (float*)p : nullptr; p += scales;
  b->psi = p; p += al(V * 12 * L * (prec == P64 ? 16 : 8));
  b->partial = (double*)p; p += al((size_t)lat->g.Vh * L * 3 * sizeof(double));
  b->omega = (double*)p; p += al((size_t)(lat->g.ndom / 2) * L * 2 * sizeof(double) * MR_ONCE_MAX);
  b->ssor = ssor ? 1 : 0;
  b->x2 = nullptr;
  b->x2_s = nullptr;
  if (ssor) {
    b->x2 = p; p += field;
    b->x2_s = prec == P16 ? (float*)p : nullptr; p += scales;
  } else if (once_mr(lat, prec) && bytes >= sap_bytes(lat, L, prec, false, false, true)) {
    b->r2 = p; p += field;
    b->r2_s = prec == P16 ? (float*)p : nullptr; p += scales;
    b->w2 = p; p += field;
    b->w2_s = prec == P16 ? (float*)p : nullptr; p += scales;
    for (int j = 0; j < 2; ++j) {
      b->wx[j] = p; p += field;
      b->wx_s[j] = prec == P16 ? (float*)p : nullptr; p += scales;
    }
  } else if (folded && bytes >= sap_bytes(lat, L, prec, false, true)) {
    b->r2 = p; p += field;
    b->r2_s = nullptr; p += scales;
    b->w2 = p; p += field;
    b->w2_s = nullptr; p += scales;
  }
  return MBBS_OK;
}

// Sites per pass of the fused MR kernel: the largest divisor of the block
// volume with at most `tmax` threads (one per site and column), preferring
// whole waves.
static int mr_fused_spb(int Vb, int L, int tmax) {
  int best = 0, best_w = 0;
  for (int s = 1; s <= Vb && s * L <= tmax; ++s) {
    if (Vb % s) continue;
    best = s;
    if ((s * L) % 64 == 0) best_w = s;
  }
  // whole waves unless that halves the threads or more
  return (best_w > 0 && 2 * best_w > best) ? best_w : best;
}
static bool use_mr_fused(const mbbs_lattice_s* lat, int L) {
  if (L > 16) return false;   // omega of at most 16 columns in LDS
  if (lat->mr_fused >= 0) return lat->mr_fused == 1;
  return (size_t)lat->g.Vb * L <= 2048;
}

template <int PR, int PPSI, int PL>
static int sap_cycles(const mbbs_lattice_s* lat, const SapBuffers& b, int ncy, int nmr,
                      const int* frozen, hipStream_t st, Profiler* prof) {
  using ER = typename Store<PR>::Elem;
  using EP = typename Store<PPSI>::Elem;
  using EL = LinkElem<PL>;
  const int L = b.L;
  const Geom& g = lat->g;
  const EL* U = PL == P64 ? (const EL*)lat->U64dm : PL == P32 ? (const EL*)lat->U32dm : (const EL*)lat->U16dm;
  const Plan pl = make_plan(lat, L, PL, g.Vh);
  const int C = pl.C, S = pl.S;
  const int Su = sites_per_block(L, g.Vb);
  const size_t red_bytes = 3 * (size_t)S * pl.gw * sizeof(double);
  for (int cy = 0; cy < ncy; ++cy) {
    for (int col = 0; col < 2; ++col) {
      const int s0 = col * g.Vh, n = g.Vh;
      if (b.ssor) {   // the residual is formed inside the SSOR launch
        if (prof) prof->begin(MBBS_K_SSOR);
        MBBS_TRY(ssor_colour(lat, b, col, cy == 0, cy > 0 ? 2 : col, frozen, st));
        if (prof) prof->end();
        continue;
      }
      const int P = lat->nsys == 1 ? lat->split[PL] : 0;   // the split kernels serve single systems only
      const int SS = ((P == 2 || P == 4) && !lat->gk.clov) ? split_sites(lat, L, PL, P) : 0;
      // psi formed once: r_0 is only read, so on the first colour of the first
      // cycle (psi = 0, r_0 = eta) the domain solve reads eta itself
      const bool once_form = !use_mr_fused(lat, L) && lat->mr_once[PL] && nmr <= MR_ONCE_MAX && b.r2 && b.w2 &&
                             b.wx[0] && b.wx[1];
      const bool r_is_eta = once_form && cy == 0 && col == 0;
      void* r0 = r_is_eta ? b.eta : b.r;
      float* r0_s = r_is_eta ? b.eta_s : b.r_s;
      if (!r_is_eta) {
      if (prof) prof->begin(MBBS_K_SAP_RES);
      TileArgs TR;
      const bool tres = cy > 0 && (((uintptr_t)b.psi | (uintptr_t)b.r | (uintptr_t)b.eta) & 15) == 0 &&
                        tile_plan_resid(lat, L, PL, &TR);
      if (tres) {
        // general case with psi staged per tile in LDS
        MBBS_TRY(launch_resid_tiled(lat, L, PL, TR, b.eta, b.eta_s, b.psi, b.r, b.r_s, s0, n, frozen, st));
      } else if (SS > 0) {
        const size_t smem = split_smem_bytes(PL, P, SS, L);
        const int mode = cy > 0 ? 2 : col;
        if (P == 4) {
          auto fn = k_sap_resid_split<PR, PPSI, PL, 4>;
          allow_lds((const void*)fn);
          hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 4, SS, L, ceil_div(n, SS))), dim3(SS * L, 4), smem, st,
                             lat->gk, lat->kappa, L, s0, n, mode, (const ER*)b.eta, b.eta_s, (const EP*)b.psi, (ER*)b.r, b.r_s, U, SS, frozen);
        } else {
          auto fn = k_sap_resid_split<PR, PPSI, PL, 2>;
          allow_lds((const void*)fn);
          hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 2, SS, L, ceil_div(n, SS))), dim3(SS * L, 2), smem, st,
                             lat->gk, lat->kappa, L, s0, n, mode, (const ER*)b.eta, b.eta_s, (const EP*)b.psi, (ER*)b.r, b.r_s, U, SS, frozen);
        }
      } else {
#define RES(CC, PV)                                                                                  \
  if (L == 12)                                                                                       \
    hipLaunchKernelGGL((k_sap_resid<PR, PPSI, PL, CC, PV, 12>), dim3(pl.nblocks), dim3(pl.nchunk, S),        \
                       (size_t)lat->lds_pad_kb * 1024, st,                                                   \
                       lat->gk, lat->kappa, L, s0, n, cy > 0 ? 2 : col, (const ER*)b.eta,              \
                       b.eta_s, (const EP*)b.psi, (ER*)b.r, b.r_s, U, pl.bpt, pl.ngroups, frozen);      \
  else                                                                                               \
  hipLaunchKernelGGL((k_sap_resid<PR, PPSI, PL, CC, PV>), dim3(pl.nblocks), dim3(pl.nchunk, S),              \
                     (size_t)lat->lds_pad_kb * 1024, st,                                                     \
                     lat->gk, lat->kappa, L, s0, n, cy > 0 ? 2 : col, (const ER*)b.eta,                \
                     b.eta_s, (const EP*)b.psi, (ER*)b.r, b.r_s, U, pl.bpt, pl.ngroups, frozen)
      const bool pr = lat->hop_pair[PL] != 0;
      switch (C) {
        case 4: hipLaunchKernelGGL((k_sap_resid<PR, PPSI, PL, 4>), dim3(pl.nblocks), dim3(pl.nchunk, S),
                                   (size_t)lat->lds_pad_kb * 1024, st, lat->gk, lat->kappa, L, s0, n,
                                   cy > 0 ? 2 : col, (const ER*)b.eta, b.eta_s, (const EP*)b.psi, (ER*)b.r,
                                   b.r_s, U, pl.bpt, pl.ngroups, frozen); break;
        case 3: hipLaunchKernelGGL((k_sap_resid<PR, PPSI, PL, 3>), dim3(pl.nblocks), dim3(pl.nchunk, S),
                                   (size_t)lat->lds_pad_kb * 1024, st, lat->gk, lat->kappa, L, s0, n,
                                   cy > 0 ? 2 : col, (const ER*)b.eta, b.eta_s, (const EP*)b.psi, (ER*)b.r,
                                   b.r_s, U, pl.bpt, pl.ngroups, frozen); break;
        case 2: if (pr) RES(2, true); else RES(2, false); break;
        default: if (pr) RES(1, true); else RES(1, false);
      }
#undef RES
      }
      if (prof) prof->end();
      MBBS_HIP(hipGetLastError());
      }

      if (use_mr_fused(lat, L)) {
        const int spb = mr_fused_spb(g.Vb, L, mr_fused_threads<PR>());
        if (prof) prof->begin(MBBS_K_MR_DSLASH);
        hipLaunchKernelGGL((k_mr_fused<PR, PPSI, PL>), dim3(g.ndom / 2), dim3(spb * L), 0, st, lat->gk, lat->kappa,
                           L, s0, spb, nmr, (int)(cy == 0), (ER*)b.r, b.r_s, (ER*)b.w, b.w_s, (EP*)b.psi, U,
                           frozen);
        if (prof) prof->end();
        MBBS_HIP(hipGetLastError());
        continue;
      }
      TileArgs T;
      const bool tiled = ((uintptr_t)b.r & 15) == 0 && ((uintptr_t)b.w & 15) == 0 && tile_plan(lat, L, PL, &T);
      const size_t ostride = (size_t)(g.ndom / 2) * L * 2;   // doubles per step's omega
      // one MR stencil step w = A_DD r on this colour, then its omega (per domain and column) into om
      auto stencil_step = [&](const void* rr, const float* rr_s, void* ww, float* ww_s, double* om) -> int {
        int nblk_dom = g.Vb / S;
        if (tiled) {
          nblk_dom = T.tpd;
          MBBS_TRY(launch_mr_dslash_tiled(lat, L, PL, T, rr, rr_s, ww, ww_s, s0, n, b.partial, frozen, st));
        } else if (SS > 0) {
          nblk_dom = g.Vb / SS;
          const size_t smem = split_smem_bytes(PL, P, SS, L);
          if (P == 4) {
            auto fn = k_mr_dslash_split<PR, PL, 4>;
            allow_lds((const void*)fn);
            hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 4, SS, L, n / SS)), dim3(SS * L, 4), smem, st, lat->gk,
                               lat->kappa, L, s0, n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, SS, frozen);
          } else {
            auto fn = k_mr_dslash_split<PR, PL, 2>;
            allow_lds((const void*)fn);
            hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 2, SS, L, n / SS)), dim3(SS * L, 2), smem, st, lat->gk,
                               lat->kappa, L, s0, n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, SS, frozen);
          }
        } else {
#define MRD(CC, PV)                                                                                   \
  if (L == 12)                                                                                        \
    hipLaunchKernelGGL((k_mr_dslash<PR, PL, CC, PV, 12>), dim3(pl.nblocks), dim3(pl.nchunk, S),             \
                       red_bytes + (size_t)lat->lds_pad_kb * 1024, st, lat->gk,                              \
                       lat->kappa, L, s0, n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, pl.bpt,      \
                       pl.ngroups, frozen);                                                                \
  else                                                                                                \
  hipLaunchKernelGGL((k_mr_dslash<PR, PL, CC, PV>), dim3(pl.nblocks), dim3(pl.nchunk, S),                   \
                     red_bytes + (size_t)lat->lds_pad_kb * 1024, st, lat->gk,                                \
                     lat->kappa, L, s0, n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, pl.bpt,        \
                     pl.ngroups, frozen)
          const bool pr = lat->hop_pair[PL] != 0;
          switch (C) {
            case 4: hipLaunchKernelGGL((k_mr_dslash<PR, PL, 4>), dim3(pl.nblocks), dim3(pl.nchunk, S),
                                       red_bytes + (size_t)lat->lds_pad_kb * 1024, st, lat->gk, lat->kappa, L, s0,
                                       n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, pl.bpt, pl.ngroups,
                                       frozen); break;
            case 3: hipLaunchKernelGGL((k_mr_dslash<PR, PL, 3>), dim3(pl.nblocks), dim3(pl.nchunk, S),
                                       red_bytes + (size_t)lat->lds_pad_kb * 1024, st, lat->gk, lat->kappa, L, s0,
                                       n, (const ER*)rr, rr_s, (ER*)ww, ww_s, U, b.partial, pl.bpt, pl.ngroups,
                                       frozen); break;
            case 2: if (pr) MRD(2, true); else MRD(2, false); break;
            default: if (pr) MRD(1, true); else MRD(1, false);
          }
#undef MRD
        }
        MBBS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_mr_omega, dim3(g.ndom / 2), dim3(256), 0, st, lat->gk, L, nblk_dom,
                           (const double*)b.partial, om, frozen);
        MBBS_HIP(hipGetLastError());
        return MBBS_OK;
      };
      if (once_form) {
        // psi formed once: r_0 stays in b.r (or is eta), r_1, r_2, ... overwrite
        // r2, the steps' A r are kept (w_0 .. w_{nmr-1}), each step's omega kept
        void* wb[MR_ONCE_MAX] = {b.w, b.w2, b.wx[0], b.wx[1]};
        float* wbs[MR_ONCE_MAX] = {b.w_s, b.w2_s, b.wx_s[0], b.wx_s[1]};
        for (int it = 0; it < nmr; ++it) {
          const void* rin = it == 0 ? r0 : b.r2;
          float* rin_s = it == 0 ? r0_s : b.r2_s;
          // the last step's A r only feeds its omega: the tiled step need not store it
          const bool keep = it + 1 < nmr || !tiled;
          if (prof) prof->begin(MBBS_K_MR_DSLASH);
          MBBS_TRY(stencil_step(rin, rin_s, keep ? wb[it] : nullptr, keep ? wbs[it] : nullptr,
                                b.omega + it * ostride));
          if (prof) prof->end();
          if (it + 1 == nmr) break;
          if (prof) prof->begin(MBBS_K_MR_UPDATE);
          if constexpr (PR == P32) {
            if (L % 2 == 0) {
              const size_t npair = (size_t)n * 6 * L;
              hipLaunchKernelGGL(k_mr_rstep_flat, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, st, lat->gk,
                                 L, s0, n, (const float4*)rin, (const float4*)wb[it], (float4*)b.r2,
                                 b.omega + it * ostride, frozen);
            } else {
              hipLaunchKernelGGL((k_mr_rstep<PR>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0, n,
                                 (const ER*)rin, rin_s, (const ER*)wb[it], wbs[it], (ER*)b.r2, b.r2_s,
                                 b.omega + it * ostride, frozen);
            }
          } else {
            hipLaunchKernelGGL((k_mr_rstep<PR>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0, n,
                               (const ER*)rin, rin_s, (const ER*)wb[it], wbs[it], (ER*)b.r2, b.r2_s,
                               b.omega + it * ostride, frozen);
          }
          if (prof) prof->end();
          MBBS_HIP(hipGetLastError());
        }
        MrOnceArgs oa{};
        oa.r0 = r0; oa.r0_s = r0_s;
        for (int j = 0; j < MR_ONCE_MAX - 1; ++j) { oa.w[j] = wb[j]; oa.w_s[j] = wbs[j]; }
        if (prof) prof->begin(MBBS_K_MR_UPDATE);
        if constexpr (PR == P32 && PPSI == P32) {
          if (L % 2 == 0) {
            const size_t npair = (size_t)n * 6 * L;
            hipLaunchKernelGGL(k_mr_psi_once_flat, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, st, lat->gk,
                               L, s0, n, oa, (float4*)b.psi, (const double*)b.omega, ostride, nmr, (int)(cy == 0),
                               frozen);
          } else {
            hipLaunchKernelGGL((k_mr_psi_once<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0,
                               n, oa, (EP*)b.psi, (const double*)b.omega, ostride, nmr, (int)(cy == 0), frozen);
          }
        } else {
          hipLaunchKernelGGL((k_mr_psi_once<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0,
                             n, oa, (EP*)b.psi, (const double*)b.omega, ostride, nmr, (int)(cy == 0), frozen);
        }
        if (prof) prof->end();
        MBBS_HIP(hipGetLastError());
        continue;
      }
      if (tiled && lat->tile[PL] == 2 && PL != P16 && b.r2 && b.w2) {
        // each step folds the previous step's update in; the steps alternate
        // between two residual / A r buffers; psi's last update follows
        void* rb[2] = {b.r, b.r2};
        void* wb[2] = {b.w, b.w2};
        float* rbs[2] = {b.r_s, b.r2_s};
        float* wbs[2] = {b.w_s, b.w2_s};
        for (int it = 0; it < nmr; ++it) {
          if (prof) prof->begin(MBBS_K_MR_DSLASH);
          const int c = it & 1, o = c ^ 1;
          if (it == 0) {
            MBBS_TRY(launch_mr_dslash_tiled(lat, L, PL, T, rb[0], rbs[0], wb[0], wbs[0], s0, n, b.partial, frozen, st));
          } else {
            MBBS_TRY(launch_mr_fused_tiled(lat, L, PL, T, rb[o], rbs[o], wb[o], wbs[o], rb[c], rbs[c], wb[c], wbs[c],
                                           b.psi, b.omega, cy == 0 && it == 1, s0, n, b.partial, frozen, st));
          }
          hipLaunchKernelGGL(k_mr_omega, dim3(g.ndom / 2), dim3(256), 0, st, lat->gk, L, T.tpd,
                             (const double*)b.partial, b.omega, frozen);
          if (prof) prof->end();
          MBBS_HIP(hipGetLastError());
        }
        if (prof) prof->begin(MBBS_K_MR_UPDATE);
        const int c = (nmr - 1) & 1;
        const int assign = cy == 0 && nmr == 1;
        if constexpr (PR == P32 && PPSI == P32) {
          const size_t npair = (size_t)n * 6 * L;
          hipLaunchKernelGGL(k_mr_update_flat, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, st, lat->gk, L, s0,
                             n, (float4*)rb[c], (const float4*)wb[c], (float4*)b.psi, b.omega, 0, assign, frozen);
        } else {
          hipLaunchKernelGGL((k_mr_update<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0, n,
                             (ER*)rb[c], rbs[c], (const ER*)wb[c], wbs[c], (EP*)b.psi, b.omega, 0, assign, frozen);
        }
        if (prof) prof->end();
        MBBS_HIP(hipGetLastError());
        continue;
      }
      for (int it = 0; it < nmr; ++it) {
        if (prof) prof->begin(MBBS_K_MR_DSLASH);
        MBBS_TRY(stencil_step(b.r, b.r_s, b.w, b.w_s, b.omega));
        if (prof) prof->end();
        if (prof) prof->begin(MBBS_K_MR_UPDATE);
        if constexpr (PR == P32 && PPSI == P32) {
          if (L % 2 == 0) {
            const size_t npair = (size_t)n * 6 * L;
            hipLaunchKernelGGL(k_mr_update_flat, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, st, lat->gk,
                               L, s0, n, (float4*)b.r, (const float4*)b.w, (float4*)b.psi, b.omega,
                               (int)(it + 1 < nmr), (int)(cy == 0 && it == 0), frozen);
          } else {
            hipLaunchKernelGGL((k_mr_update<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0,
                               n, (ER*)b.r, b.r_s, (const ER*)b.w, b.w_s, (EP*)b.psi, b.omega,
                               (int)(it + 1 < nmr), (int)(cy == 0 && it == 0), frozen);
          }
        } else {
          hipLaunchKernelGGL((k_mr_update<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0,
                             n, (ER*)b.r, b.r_s, (const ER*)b.w, b.w_s, (EP*)b.psi, b.omega,
                             (int)(it + 1 < nmr), (int)(cy == 0 && it == 0), frozen);
        }
        if (prof) prof->end();
        MBBS_HIP(hipGetLastError());
      }
    }
  }
  return MBBS_OK;
}

// Conversion kernels between the FP64 lexicographic block and the SAP
// domain-major storage.  to_sap optionally right-multiplies by an L x L
// matrix first (the Cholesky-QR factor gamma^{-1}, folded into the copy).
template <int PR, int LT = 0>
__global__ void __launch_bounds__(256) k_to_sap(GeomK k, int L, const double2* __restrict__ in,
                                                const double2* __restrict__ gam,
                                                typename Store<PR>::Elem* __restrict__ out,
                                                float* __restrict__ out_s, const int* __restrict__ frozen) {
  if constexpr (LT > 0) L = LT;
  using R = typename Store<PR>::Real;
  // with gamma: [L][L] gamma, then the block's sites' 12 L input values
  // ([site][12][L], staged once: every column of a row reads all of it)
  extern __shared__ double2 gsh[];
  __shared__ int lsh[256];
  // a block never straddles two systems (its site count divides a system's
  // half volume), so the system, its flag and its gamma are block-uniform
  const int sys = site_ctx<DM>(k, min((int)(blockIdx.x * blockDim.y), k.g.V - 1)).sys;
  if (sys_frozen(k, frozen, sys)) return;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x, nthr = blockDim.x * blockDim.y;
  const int s = blockIdx.x * blockDim.y + threadIdx.y;  // domain-major index
  double2* ish = gsh + L * L;
  if (gam) {
    for (int e = tid; e < L * L; e += nthr) gsh[e] = gam[(size_t)sys * L * L + e];
    for (int y = tid; y < (int)blockDim.y; y += nthr) {
      const int sy = blockIdx.x * blockDim.y + y;
      lsh[y] = sy < k.g.V ? lex_of(k, site_ctx<DM>(k, sy)) : -1;
    }
    __syncthreads();
    const int row = 12 * L, tot = (int)blockDim.y * row;
    // NB loads of a thread are in flight before its LDS writes; past the end
    // a slot repeats the last element (same bytes, same place)
    constexpr int NB = 8;
    for (int f0 = tid; f0 < tot; f0 += NB * nthr) {
      double2 buf[NB];
      int ff[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        ff[q] = min(f0 + q * nthr, tot - 1);
        const int y = ff[q] / row, w = ff[q] - y * row;
        buf[q] = in[(size_t)max(lsh[y], 0) * row + w];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) ish[ff[q]] = buf[q];
    }
    __syncthreads();
  }
  if (s >= k.g.V) return;
  const int j = threadIdx.x;
  cplx<double> v[4][3];
  if (gam) {
    const double2* xr = ish + (size_t)threadIdx.y * 12 * L;
    if constexpr (LT > 0) {
      // column j of gamma in registers: only the rows come from LDS
      cplx<double> gc[LT];
#pragma unroll
      for (int m = 0; m < LT; ++m) gc[m] = cmake(gsh[m * L + j].x, gsh[m * L + j].y);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cplx<double> acc = cmake(0.0, 0.0);
#pragma unroll
          for (int m = 0; m < LT; ++m) {
            const double2 e = xr[(3 * sp + a) * L + m];
            acc = acc + cmake(e.x, e.y) * gc[m];
          }
          v[sp][a] = acc;
        }
    } else {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          cplx<double> acc = cmake(0.0, 0.0);
          for (int m = 0; m < L; ++m) {
            double2 e = xr[(3 * sp + a) * L + m], gg = gsh[m * L + j];
            acc = acc + cmake(e.x, e.y) * cmake(gg.x, gg.y);
          }
          v[sp][a] = acc;
        }
    }
  } else {
    const int ls = lex_of(k, site_ctx<DM>(k, s));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double2 e = in[((size_t)ls * 12 + 3 * sp + a) * L + j];
        v[sp][a] = cmake(e.x, e.y);
      }
  }
  cplx<R> vr[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) vr[sp][a] = cmake<R>((R)v[sp][a].re, (R)v[sp][a].im);
  store_spinor<PR, R>(out, out_s, (size_t)s * 12 * L + j, L, (size_t)s * L + j, vr);
}

template <int PPSI, int LT = 0>
__global__ void __launch_bounds__(256) k_from_sap(GeomK k, int L, const typename Store<PPSI>::Elem* __restrict__ in,
                                                  double2* __restrict__ out, const int* __restrict__ frozen) {
  if constexpr (LT > 0) L = LT;
  const int s = blockIdx.x * blockDim.y + threadIdx.y;
  if (s >= k.g.V) return;
  const int j = threadIdx.x;
  const SiteCtx c = site_ctx<DM>(k, s);
  if (sys_frozen(k, frozen, c.sys)) return;
  const int ls = lex_of(k, c);
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    auto v = Store<PPSI>::ld(in, ((size_t)s * 12 + e) * L + j);
    out[((size_t)ls * 12 + e) * L + j] = make_double2((double)v.re, (double)v.im);
  }
}

// FP32 psi to the FP64 block, even L: a block takes FROM_SITES consecutive
// domain-major sites, finds their lexicographic rows once, then streams each
// site's 12 L values as 16-byte loads (two complex) and 32-byte stores.
constexpr int FROM_SITES = 16;
__global__ void __launch_bounds__(256) k_from_sap_flat(GeomK k, int L, const float4* __restrict__ in,
                                                       double2* __restrict__ out, const int* __restrict__ frozen) {
  __shared__ int lsh[FROM_SITES];
  const int s0 = blockIdx.x * FROM_SITES;
  if (threadIdx.x < FROM_SITES) {
    const int s = s0 + threadIdx.x;
    int ls = -1;
    if (s < k.g.V) {
      const SiteCtx c = site_ctx<DM>(k, s);
      if (!sys_frozen(k, frozen, c.sys)) ls = lex_of(k, c);
    }
    lsh[threadIdx.x] = ls;
  }
  __syncthreads();
  const int per = 6 * L;   // float4 units per site
  const int tot = min(FROM_SITES, k.g.V - s0) * per;
  // a thread's loads are in flight together before its stores (past the end
  // a slot reloads the last unit and stores nothing)
  constexpr int NB = 6;
  for (int u0 = threadIdx.x; u0 < tot; u0 += NB * blockDim.x) {
    float4 v[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int u = min(u0 + q * (int)blockDim.x, tot - 1);
      v[q] = in[(size_t)s0 * per + u];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int u = u0 + q * (int)blockDim.x;
      if (u >= tot) continue;
      const int y = u / per, w = u - y * per;
      if (lsh[y] < 0) continue;
      double2* o = out + (size_t)lsh[y] * 12 * L + 2 * w;
      o[0] = make_double2((double)v[q].x, (double)v[q].y);
      o[1] = make_double2((double)v[q].z, (double)v[q].w);
    }
  }
}

int sap_to(const mbbs_lattice_s* lat, const SapBuffers& b, const double2* in, const double2* gam, void* dst,
           float* dst_s, const int* frozen, hipStream_t st) {
  const int L = b.L;
  const Geom& g = lat->g;
  // a batch: blocks stay inside one system's half volume (per-system gamma)
  const int S = sites_per_block(L, lat->nsys > 1 ? g.V / (2 * lat->nsys) : g.V);
  const size_t gsh = gam ? ((size_t)L * L + (size_t)S * 12 * L) * sizeof(double2) : 0;
  const bool l12 = L == 12;   // compile-time row offsets for the common block width
  switch (b.prec) {
    case P64:
      if (l12) hipLaunchKernelGGL((k_to_sap<P64, 12>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (double2*)dst, nullptr, frozen);
      else hipLaunchKernelGGL((k_to_sap<P64>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (double2*)dst, nullptr, frozen);
      break;
    case P32:
      if (l12) hipLaunchKernelGGL((k_to_sap<P32, 12>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (float2*)dst, nullptr, frozen);
      else hipLaunchKernelGGL((k_to_sap<P32>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (float2*)dst, nullptr, frozen);
      break;
    default:
      if (l12) hipLaunchKernelGGL((k_to_sap<P16, 12>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (__half2*)dst, dst_s, frozen);
      else hipLaunchKernelGGL((k_to_sap<P16>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (__half2*)dst, dst_s, frozen);
      break;
  }
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int sap_from(const mbbs_lattice_s* lat, const SapBuffers& b, double2* out, const int* frozen, hipStream_t st) {
  const int L = b.L;
  const Geom& g = lat->g;
  const int S = sites_per_block(L, g.V);
  if (b.prec == P64) {
    if (L == 12) hipLaunchKernelGGL((k_from_sap<P64, 12>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const double2*)b.psi, out, frozen);
    else hipLaunchKernelGGL((k_from_sap<P64>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const double2*)b.psi, out, frozen);
  } else if (L % 2 == 0 && ((uintptr_t)b.psi & 15) == 0 && ((uintptr_t)out & 15) == 0) {
    hipLaunchKernelGGL(k_from_sap_flat, dim3(ceil_div(g.V, FROM_SITES)), dim3(256), 0, st, lat->gk, L,
                       (const float4*)b.psi, out, frozen);
  } else {
    if (L == 12) hipLaunchKernelGGL((k_from_sap<P32, 12>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const float2*)b.psi, out, frozen);
    else hipLaunchKernelGGL((k_from_sap<P32>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const float2*)b.psi, out, frozen);
  }
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int sap_apply(const mbbs_lattice_s* lat, const SapBuffers& b, int ncy, int nmr, const double2* in,
              const double2* gam, double2* out, const int* frozen, hipStream_t st, Profiler* prof) {
  if (prof) prof->begin(MBBS_K_CONVERT);
  MBBS_TRY(sap_to(lat, b, in, gam, b.eta, b.eta_s, frozen, st));
  if (prof) prof->end();
  // psi needs no clearing: the first domain solve of the first cycle assigns it.
  int rc;
  switch (b.prec) {
    case P64: rc = sap_cycles<P64, P64, P64>(lat, b, ncy, nmr, frozen, st, prof); break;
    case P32: rc = sap_cycles<P32, P32, P32>(lat, b, ncy, nmr, frozen, st, prof); break;
    default: rc = sap_cycles<P16, P32, P16>(lat, b, ncy, nmr, frozen, st, prof); break;
  }
  if (rc < 0) return rc;
  if (prof) prof->begin(MBBS_K_CONVERT);
  MBBS_TRY(sap_from(lat, b, out, frozen, st));
  if (prof) prof->end();
  return MBBS_OK;
}

}  // namespace mbbs
