// SSOR approximate domain inverse of the SAP preconditioner (Sec. 2.2, SSOR
// equations), with the paper's naming: on a domain A_DD = 1 - Lf - Ub, Lf the
// forward in-domain hops, Ub the backward ones, and
//   B = (1 - w Ub)^{-1} [ sum_{j=0}^{N} (1 - A^S)^j ] (1 - w Lf)^{-1},
//   A^S = (1/w) [ (1 - w Lf)^{-1} + (1 - w Ub)^{-1} + (w - 2) (1 - w Lf)^{-1} (1 - w Ub)^{-1} ].
// For N = 1 (the paper's setting) B r takes four triangular sweeps:
//   t = F r,  u = G t,  c = F (t + (w - 2) u),  y = G (2 t - (u + c) / w),
// with F = (1 - w Lf)^{-1}, G = (1 - w Ub)^{-1}, since A^S t = (u + c) / w;
// N = 0 is y = G F r.
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

template <int PR> constexpr int ssor_threads() { return PR == P64 ? 512 : 1024; }

// One sweep.  MODE: input and destination of the result
//   0: in = r                     -> a              (t = F r)
//   1: in = a                     -> b              (u = G t)
//   2: in = a + (w - 2) b         -> r              (c = F (t + (w-2) u))
//   3: in = 2 a - (b + r) / w     -> b, psi (+)= y  (y = G s, N = 1)
//   4: in = a                     -> b, psi (+)= y  (y = G t, N = 0)
// The destination of a sweep is also what its hops read (the neighbours'
// results, one hyperplane earlier in the sweep).  In mode 3 each item reads
// b at its own site before overwriting it with y; the hops only read sites of
// earlier hyperplanes, which already hold y.
template <int PR, int PPSI, int PL, bool FWD, int MODE>
__device__ __forceinline__ void ssor_sweep(const GeomK& k, int L, int base_site, double wk, double omega,
                                           typename Store<PR>::Elem* r, float* r_s,
                                           typename Store<PR>::Elem* a, float* a_s,
                                           typename Store<PR>::Elem* b, float* b_s,
                                           typename Store<PPSI>::Elem* psi, bool assign,
                                           const LinkElem<PL>* __restrict__ U,
                                           const int* __restrict__ hp_loc, const int* __restrict__ hp_off, int nh) {
  using R = typename Store<PR>::Real;
  using RP = typename Store<PPSI>::Real;
  typename Store<PR>::Elem* X = MODE == 0 ? a : MODE == 2 ? r : b;
  float* X_s = MODE == 0 ? a_s : MODE == 2 ? r_s : b_s;
  const R wkr = (R)wk, om = (R)omega;
  for (int step = 0; step < nh; ++step) {
    const int h = FWD ? nh - 1 - step : step;
    const int o0 = hp_off[h], nsite = hp_off[h + 1] - o0;
    for (int i = threadIdx.x; i < nsite * L; i += blockDim.x) {
      const int j = i / L, col = i - j * L;
      const int s = base_site + hp_loc[o0 + j];
      const SiteCtx c = site_ctx<DM>(k, s);
      cplx<R> acc[4][3][1];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[sp][q][0] = cmake<R>(0, 0);
      hop_sum<PR, PL, 1, DM, FWD ? FWD_IN : BWD_IN, R>(k, c, X, X_s, U, L, col, acc);
      if (k.clov) clover_apply<DM, 1, R>(k, s, acc);
      const size_t base = (size_t)s * 12 * L + col, sidx = (size_t)s * L + col;
      cplx<R> in[4][3];
      if constexpr (MODE == 0) {
        load_spinor<PR, R>(r, r_s, base, L, sidx, in);
      } else if constexpr (MODE == 1 || MODE == 4) {
        load_spinor<PR, R>(a, a_s, base, L, sidx, in);
      } else if constexpr (MODE == 2) {
        cplx<R> t[4][3], u[4][3];
        load_spinor<PR, R>(a, a_s, base, L, sidx, t);
        load_spinor<PR, R>(b, b_s, base, L, sidx, u);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) in[sp][q] = t[sp][q] + (om - (R)2) * u[sp][q];
      } else {
        cplx<R> t[4][3], u[4][3], cc[4][3];
        load_spinor<PR, R>(a, a_s, base, L, sidx, t);
        load_spinor<PR, R>(b, b_s, base, L, sidx, u);
        load_spinor<PR, R>(r, r_s, base, L, sidx, cc);
        const R inv = (R)1 / om;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) in[sp][q] = (R)2 * t[sp][q] - inv * (u[sp][q] + cc[sp][q]);
      }
      cplx<R> v[4][3];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int q = 0; q < 3; ++q) v[sp][q] = in[sp][q] + wkr * acc[sp][q][0];
      store_spinor<PR, R>(X, X_s, base, L, sidx, v);
      if constexpr (MODE == 3 || MODE == 4) {
        // psi gets the value as stored (FP16 storage: rounded), as the hops see it
        if constexpr (Store<PR>::scaled) load_spinor<PR, R>(X, X_s, base, L, sidx, v);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const size_t e = base + (size_t)(3 * sp + q) * L;
            if (assign) {
              Store<PPSI>::st(psi, e, cplx<RP>{(RP)v[sp][q].re, (RP)v[sp][q].im});
            } else {
              auto pv = Store<PPSI>::ld(psi, e);
              Store<PPSI>::st(psi, e, cplx<RP>{(RP)(pv.re + (RP)v[sp][q].re), (RP)(pv.im + (RP)v[sp][q].im)});
            }
          }
      }
    }
    __syncthreads();
  }
}

// One workgroup per domain of the colour starting at s0 (domain-major order).
// r, a, b and psi are written and read by other threads of the workgroup
// between barriers: no restrict / const qualifiers on them.
template <int PR, int PPSI, int PL>
__global__ void __launch_bounds__(ssor_threads<PR>()) k_ssor(GeomK k, double kappa, int L, int s0, double omega,
                                                             int nssor, int assign,
                                                             typename Store<PR>::Elem* r, float* r_s,
                                                             typename Store<PR>::Elem* a, float* a_s,
                                                             typename Store<PR>::Elem* b, float* b_s,
                                                             typename Store<PPSI>::Elem* psi,
                                                             const LinkElem<PL>* __restrict__ U,
                                                             const int* __restrict__ hp_loc,
                                                             const int* __restrict__ hp_off, int nh,
                                                             const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  const int base_site = s0 + blockIdx.x * k.g.Vb;
  const double wk = omega * kappa;
  ssor_sweep<PR, PPSI, PL, true, 0>(k, L, base_site, wk, omega, r, r_s, a, a_s, b, b_s, psi, assign, U, hp_loc,
                                    hp_off, nh);
  if (nssor == 0) {
    ssor_sweep<PR, PPSI, PL, false, 4>(k, L, base_site, wk, omega, r, r_s, a, a_s, b, b_s, psi, assign, U, hp_loc,
                                       hp_off, nh);
    return;
  }
  ssor_sweep<PR, PPSI, PL, false, 1>(k, L, base_site, wk, omega, r, r_s, a, a_s, b, b_s, psi, assign, U, hp_loc,
                                     hp_off, nh);
  ssor_sweep<PR, PPSI, PL, true, 2>(k, L, base_site, wk, omega, r, r_s, a, a_s, b, b_s, psi, assign, U, hp_loc,
                                    hp_off, nh);
  ssor_sweep<PR, PPSI, PL, false, 3>(k, L, base_site, wk, omega, r, r_s, a, a_s, b, b_s, psi, assign, U, hp_loc,
                                     hp_off, nh);
}

template <int PR, int PPSI, int PL>
static int ssor_launch(const mbbs_lattice_s* lat, const SapBuffers& b, int colour, bool assign, const int* frozen,
                       hipStream_t st) {
  using ER = typename Store<PR>::Elem;
  using EP = typename Store<PPSI>::Elem;
  using EL = LinkElem<PL>;
  const Geom& g = lat->g;
  const EL* U = PL == P64 ? (const EL*)lat->U64dm : PL == P32 ? (const EL*)lat->U32dm : (const EL*)lat->U16dm;
  const int want = ((lat->hp_max * b.L + 63) / 64) * 64;
  const int T = std::max(64, std::min(ssor_threads<PR>(), want));
  hipLaunchKernelGGL((k_ssor<PR, PPSI, PL>), dim3(g.ndom / 2), dim3(T), 0, st, lat->gk, lat->kappa, b.L,
                     colour * g.Vh, b.ssor_omega, b.nssor, (int)assign, (ER*)b.r, b.r_s, (ER*)b.w, b.w_s,
                     (ER*)b.x2, b.x2_s, (EP*)b.psi, U, (const int*)lat->hp_loc, (const int*)lat->hp_off, lat->nh,
                     frozen);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int ssor_colour(const mbbs_lattice_s* lat, const SapBuffers& b, int colour, bool assign, const int* frozen,
                hipStream_t st) {
  MBBS_CHECK(b.ssor && b.x2 != nullptr, "SAP buffers bound without the SSOR field");
  MBBS_CHECK(b.nssor == 0 || b.nssor == 1, "N_SSOR must be 0 or 1");
  switch (b.prec) {
    case P64: return ssor_launch<P64, P64, P64>(lat, b, colour, assign, frozen, st);
    case P32: return ssor_launch<P32, P32, P32>(lat, b, colour, assign, frozen, st);
    default: return ssor_launch<P16, P32, P16>(lat, b, colour, assign, frozen, st);
  }
}

int ssor_blocked_apply(const mbbs_lattice_s* lat, const SapBuffers& b, const double2* in, double2* out,
                       hipStream_t st) {
  // r holds the input on both colours; each colour's launch reads only its
  // own domains, and psi of each colour is assigned by its launch
  MBBS_TRY(sap_to(lat, b, in, nullptr, b.r, b.r_s, nullptr, st));
  MBBS_TRY(ssor_colour(lat, b, 0, true, nullptr, st));
  MBBS_TRY(ssor_colour(lat, b, 1, true, nullptr, st));
  return sap_from(lat, b, out, nullptr, st);
}

}  // namespace mbbs
