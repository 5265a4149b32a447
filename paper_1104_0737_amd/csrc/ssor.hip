// SSOR approximate domain inverse of the SAP preconditioner (Sec. 2.2, SSOR
// equations), with the paper's naming: on a domain A_DD = 1 - Lf - Ub, Lf the
// forward in-domain hops, Ub the backward ones, and
//   B = (1 - w Ub)^{-1} [ sum_{j=0}^{N} (1 - A^S)^j ] (1 - w Lf)^{-1},
//   A^S = (1/w) [ (1 - w Lf)^{-1} + (1 - w Ub)^{-1} + (w - 2) (1 - w Lf)^{-1} (1 - w Ub)^{-1} ].
// For N = 1 (the paper's setting) B r takes four triangular sweeps:
//   t = F r,  u = G t,  c = F (t + (w - 2) u),  y = G (2 t - (u + c) / w),
// with F = (1 - w Lf)^{-1}, G = (1 - w Ub)^{-1}, since A^S t = (u + c) / w;
// N = 0 is y = G F r.  Inside SAP the residual r = eta - A psi of the domain
// is formed in the first sweep, site by site, instead of by a separate pass.
//
// A triangular solve x = in + w Lf x is a wavefront: a forward hop raises the
// hyperplane index h = l_0 + l_1 + l_2 + l_3 of the local coordinates by one,
// so all sites of a hyperplane are independent once the hyperplane above is
// done.  One workgroup owns one domain and walks its hyperplanes (top down
// for F, bottom up for G) with a barrier between them; the fields stay in
// global memory (the domain's working set stays in the CU's caches), items
// are (site of the hyperplane, column) pairs spread over the workgroup.
#include "stencil.h"

namespace mbbs {

template <int PR> constexpr int ssor_threads() { return PR == P64 ? 512 : 768; }

// The fields one launch touches (SAP storage precision PR, psi in PPSI).
template <int PR, int PPSI>
struct SsorFields {
  typename Store<PR>::Elem *eta, *r, *a, *b;
  float *eta_s, *r_s, *a_s, *b_s;
  typename Store<PPSI>::Elem* psi;
};

// One sweep.  MODE: input, destination, and what else happens
//   0: in = r                        -> a               (t = F r; blocked B)
//   5: in = eta - A psi at the site  -> a               (t = F r, r the SAP residual,
//                                                        computed on the fly: rmode 0 eta,
//                                                        1 outside hops only, 2 all)
//   1: in = a                        -> b               (u = G t)
//   6: in = a + (w - 2) b            -> r, and a <- 2a - (b + c)/w   (c, then s in place of t)
//   7: in = a                        -> b, psi (+)= y   (y = G s, N = 1)
//   4: in = a                        -> b, psi (+)= y   (y = G t, N = 0)
// The destination of a sweep is also what its hops read (the neighbours'
// results, one hyperplane earlier in the sweep).  In-place writes (a in
// mode 6, b in mode 7) touch only the item's own site, which no other item
// of the sweep reads.
template <int PR, int PPSI, int PL, bool FWD, int MODE>
__device__ __forceinline__ void ssor_sweep(const GeomK& k, int L, int base_site, double kappa, double omega,
                                           const SsorFields<PR, PPSI>& f, int rmode, bool assign,
                                           const LinkElem<PL>* __restrict__ U,
                                           const int* __restrict__ hp_loc, const int* __restrict__ hp_off, int nh) {
  using R = typename Store<PR>::Real;
  using RP = typename Store<PPSI>::Real;
  typename Store<PR>::Elem* X = MODE == 0 || MODE == 5 ? f.a : MODE == 6 ? f.r : f.b;
  float* X_s = MODE == 0 || MODE == 5 ? f.a_s : MODE == 6 ? f.r_s : f.b_s;
  const R wkr = (R)(omega * kappa), om = (R)omega, kap = (R)kappa;
  for (int step = 0; step < nh; ++step) {
    const int h = FWD ? nh - 1 - step : step;
    const int o0 = hp_off[h], nsite = hp_off[h + 1] - o0;
    for (int i = threadIdx.x; i < nsite * L; i += blockDim.x) {
      const int j = i / L, col = i - j * L;
      const int s = base_site + hp_loc[o0 + j];
      const SiteCtx c = site_ctx<DM>(k, s);
      const size_t base = (size_t)s * 12 * L + col, sidx = (size_t)s * L + col;
      cplx<R> acc[4][3][1];
      cplx<R> in[4][3];
      if constexpr (MODE == 5) {
        // the SAP residual eta - (psi - kappa (1+T)^-1 H psi) at this site
        load_spinor<PR, R>(f.eta, f.eta_s, base, L, sidx, in);
        if (rmode != 0) {
#pragma unroll
          for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[sp][q][0] = cmake<R>(0, 0);
          if (rmode == 1) hop_sum<PPSI, PL, 1, DM, OUTSIDE, R>(k, c, f.psi, nullptr, U, L, col, acc);
          else hop_sum<PPSI, PL, 1, DM, ALL, R>(k, c, f.psi, nullptr, U, L, col, acc);
          if (k.clov) clover_apply<DM, 1, R>(k, s, acc);
          cplx<R> p[4][3];
          if (rmode == 2) {
            load_spinor<PPSI, R>(f.psi, nullptr, base, L, sidx, p);
          } else {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
              for (int q = 0; q < 3; ++q) p[sp][q] = cmake<R>(0, 0);
          }
#pragma unroll
          for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int q = 0; q < 3; ++q) in[sp][q] = in[sp][q] - p[sp][q] + kap * acc[sp][q][0];
        }
      }
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[sp][q][0] = cmake<R>(0, 0);
      // FP32 / FP16 storage: two directions' loads in flight; FP64 would spill
      if constexpr (PR == P64) hop_sum<PR, PL, 1, DM, FWD ? FWD_IN : BWD_IN, R>(k, c, X, X_s, U, L, col, acc);
      else hop_sense_sum<PR, PL, 1, DM, FWD ? FWD_IN : BWD_IN, R>(k, c, X, X_s, U, L, col, acc);
      if (k.clov) clover_apply<DM, 1, R>(k, s, acc);
      cplx<R> t[4][3], u[4][3];
      if constexpr (MODE == 0) {
        load_spinor<PR, R>(f.r, f.r_s, base, L, sidx, in);
      } else if constexpr (MODE == 1 || MODE == 4 || MODE == 7) {
        load_spinor<PR, R>(f.a, f.a_s, base, L, sidx, in);
      } else if constexpr (MODE == 6) {
        load_spinor<PR, R>(f.a, f.a_s, base, L, sidx, t);
        load_spinor<PR, R>(f.b, f.b_s, base, L, sidx, u);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) in[sp][q] = t[sp][q] + (om - (R)2) * u[sp][q];
      }
      cplx<R> v[4][3];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int q = 0; q < 3; ++q) v[sp][q] = in[sp][q] + wkr * acc[sp][q][0];
      store_spinor<PR, R>(X, X_s, base, L, sidx, v);
      if constexpr (MODE == 6) {
        // s = 2 t - (u + c) / w, with c as stored (what the hops of this sweep read)
        if constexpr (Store<PR>::scaled) load_spinor<PR, R>(X, X_s, base, L, sidx, v);
        const R inv = (R)1 / om;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) t[sp][q] = (R)2 * t[sp][q] - inv * (u[sp][q] + v[sp][q]);
        store_spinor<PR, R>(f.a, f.a_s, base, L, sidx, t);
      }
      if constexpr (MODE == 4 || MODE == 7) {
        // psi gets the value as stored (FP16 storage: rounded), as the hops see it
        if constexpr (Store<PR>::scaled) load_spinor<PR, R>(X, X_s, base, L, sidx, v);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const size_t e = base + (size_t)(3 * sp + q) * L;
            if (assign) {
              Store<PPSI>::st(f.psi, e, cplx<RP>{(RP)v[sp][q].re, (RP)v[sp][q].im});
            } else {
              auto pv = Store<PPSI>::ld(f.psi, e);
              Store<PPSI>::st(f.psi, e, cplx<RP>{(RP)(pv.re + (RP)v[sp][q].re), (RP)(pv.im + (RP)v[sp][q].im)});
            }
          }
      }
    }
    __syncthreads();
  }
}

// One workgroup per domain of the colour starting at s0 (domain-major order).
// rmode < 0: r holds the input; 0, 1, 2: the input is the SAP residual,
// formed in the first sweep (modes as in the SAP residual kernel).  The
// fields are written and read by other threads of the workgroup between
// barriers: no restrict / const qualifiers on them.
template <int PR, int PPSI, int PL, int LT = 0>
__global__ void __launch_bounds__(ssor_threads<PR>()) k_ssor(GeomK k, double kappa, int L, int s0, double omega,
                                                             int nssor, int assign, int rmode,
                                                             SsorFields<PR, PPSI> f,
                                                             const LinkElem<PL>* __restrict__ U,
                                                             const int* __restrict__ hp_loc,
                                                             const int* __restrict__ hp_off, int nh,
                                                             const int* __restrict__ frozen) {
  // one workgroup per domain, hence one system: block-uniform test and kappa
  const int sys = sys_of_domain(k, blockIdx.x);
  if (sys_frozen(k, frozen, sys)) return;
  if (k.kap) kappa = k.kap[sys];
  if constexpr (LT > 0) L = LT;   // compile-time element offsets for the common block width
  const int base_site = s0 + blockIdx.x * k.g.Vb;
  if (rmode < 0)
    ssor_sweep<PR, PPSI, PL, true, 0>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
  else
    ssor_sweep<PR, PPSI, PL, true, 5>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
  if (nssor == 0) {
    ssor_sweep<PR, PPSI, PL, false, 4>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
    return;
  }
  ssor_sweep<PR, PPSI, PL, false, 1>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
  ssor_sweep<PR, PPSI, PL, true, 6>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
  ssor_sweep<PR, PPSI, PL, false, 7>(k, L, base_site, kappa, omega, f, rmode, assign, U, hp_loc, hp_off, nh);
}

template <int PR, int PPSI, int PL>
static int ssor_launch(const mbbs_lattice_s* lat, const SapBuffers& b, int colour, bool assign, int rmode,
                       const int* frozen, hipStream_t st) {
  using ER = typename Store<PR>::Elem;
  using EP = typename Store<PPSI>::Elem;
  using EL = LinkElem<PL>;
  const Geom& g = lat->g;
  const EL* U = PL == P64 ? (const EL*)lat->U64dm : PL == P32 ? (const EL*)lat->U32dm : (const EL*)lat->U16dm;
  const int want = ((lat->hp_max * b.L + 63) / 64) * 64;
  const int T = std::max(64, std::min(ssor_threads<PR>(), want));
  SsorFields<PR, PPSI> f;
  f.eta = (ER*)b.eta; f.eta_s = b.eta_s;
  f.r = (ER*)b.r; f.r_s = b.r_s;
  f.a = (ER*)b.w; f.a_s = b.w_s;
  f.b = (ER*)b.x2; f.b_s = b.x2_s;
  f.psi = (EP*)b.psi;
  if (b.L == 12)
    hipLaunchKernelGGL((k_ssor<PR, PPSI, PL, 12>), dim3(g.ndom / 2), dim3(T), 0, st, lat->gk, lat->kappa, b.L,
                       colour * g.Vh, b.ssor_omega, b.nssor, (int)assign, rmode, f, U, (const int*)lat->hp_loc,
                       (const int*)lat->hp_off, lat->nh, frozen);
  else
    hipLaunchKernelGGL((k_ssor<PR, PPSI, PL>), dim3(g.ndom / 2), dim3(T), 0, st, lat->gk, lat->kappa, b.L,
                       colour * g.Vh, b.ssor_omega, b.nssor, (int)assign, rmode, f, U, (const int*)lat->hp_loc,
                       (const int*)lat->hp_off, lat->nh, frozen);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int ssor_colour(const mbbs_lattice_s* lat, const SapBuffers& b, int colour, bool assign, int rmode,
                const int* frozen, hipStream_t st) {
  MBBS_CHECK(b.ssor && b.x2 != nullptr, "SAP buffers bound without the SSOR field");
  MBBS_CHECK(b.nssor == 0 || b.nssor == 1, "N_SSOR must be 0 or 1");
  switch (b.prec) {
    case P64: return ssor_launch<P64, P64, P64>(lat, b, colour, assign, rmode, frozen, st);
    case P32: return ssor_launch<P32, P32, P32>(lat, b, colour, assign, rmode, frozen, st);
    default: return ssor_launch<P16, P32, P16>(lat, b, colour, assign, rmode, frozen, st);
  }
}

int ssor_blocked_apply(const mbbs_lattice_s* lat, const SapBuffers& b, const double2* in, double2* out,
                       hipStream_t st) {
  // r holds the input on both colours; each colour's launch reads only its
  // own domains, and psi of each colour is assigned by its launch
  MBBS_TRY(sap_to(lat, b, in, nullptr, b.r, b.r_s, nullptr, st));
  MBBS_TRY(ssor_colour(lat, b, 0, true, -1, nullptr, st));
  MBBS_TRY(ssor_colour(lat, b, 1, true, -1, nullptr, st));
  return sap_from(lat, b, out, nullptr, st);
}

}  // namespace mbbs
