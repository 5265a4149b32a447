// Clover term and its site-diagonal (Jacobi) inverse for the O(a)-improved
// Wilson operator of Sec. 2.2, whose matrix is divided by (I + clover term)
// before the domain decomposition.  The paper does not write the term out;
// the form used (Sheikholeslami-Wohlert in the hopping normalisation
// A = 1 - kappa H):
//   Q_{mu nu}(x): the four plaquettes of the (mu, nu) plane that start and end
//                 at x, each traversed mu first, then nu,
//   F_{mu nu} = (Q - Q^dagger) / 8,   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
//   T(x) = i c_sw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
//   A = (1 + T)^{-1} D = 1 - kappa (1 + T)^{-1} H.
// In the chiral basis sigma_{mu nu} is block diagonal over spins {0,1} and
// {2,3}: sigma_{kl} = -eps_{klm} s_m in both blocks and sigma_{k3} = +/- s_k
// (s_m the Pauli matrices, k, l, m spatial).  So 1 + T is two hermitian 6 x 6
// blocks, 1 + i c_sw kappa [[Bz, Bx - i By], [Bx + i By, -Bz]] with
// Bx = -F_12 +/- F_03, By = F_02 +/- F_13, Bz = -F_01 +/- F_23.  Their
// inverses are stored packed per site and block: 6 real diagonal entries,
// then the 15 entries (i, j), i < j, row by row, as (re, im): 72 reals a site.
#include "stencil.h"

namespace mbbs {

namespace {

struct M3 { cplx<double> m[3][3]; };

__device__ M3 link(const double2* U, int site, int mu) {
  M3 r;
  const double2* p = U + ((size_t)site * 4 + mu) * 9;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) r.m[a][b] = cmake(p[a * 3 + b].x, p[a * 3 + b].y);
  return r;
}
__device__ M3 mul(const M3& a, const M3& b) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> s = cmake(0.0, 0.0);
      for (int l = 0; l < 3; ++l) s = s + a.m[i][l] * b.m[l][j];
      r.m[i][j] = s;
    }
  return r;
}
__device__ M3 dag(const M3& a) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = conj(a.m[j][i]);
  return r;
}
__device__ M3 add(const M3& a, const M3& b, double sb = 1.0) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][j] + sb * b.m[i][j];
  return r;
}

// Site of x + a*mu + b*nu with periodic wrap.
__device__ int shifted(const Geom& g, const int (&x)[4], int mu, int a, int nu, int b) {
  Coord c;
  for (int m = 0; m < 4; ++m) c.c[m] = x[m];
  c.c[mu] = (c.c[mu] + a + g.d[mu]) % g.d[mu];
  c.c[nu] = (c.c[nu] + b + g.d[nu]) % g.d[nu];
  return lex_site(g, c);
}

__device__ M3 field_strength(const Geom& g, const double2* U, const int (&x)[4], int s, int mu, int nu) {
  const int xpm = shifted(g, x, mu, 1, nu, 0), xpn = shifted(g, x, mu, 0, nu, 1);
  const int xmm = shifted(g, x, mu, -1, nu, 0), xmn = shifted(g, x, mu, 0, nu, -1);
  const int xmm_pn = shifted(g, x, mu, -1, nu, 1), xmm_mn = shifted(g, x, mu, -1, nu, -1);
  const int xpm_mn = shifted(g, x, mu, 1, nu, -1);
  // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
  M3 q = mul(mul(link(U, s, mu), link(U, xpm, nu)), mul(dag(link(U, xpn, mu)), dag(link(U, s, nu))));
  // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
  q = add(q, mul(mul(link(U, s, nu), dag(link(U, xmm_pn, mu))), mul(dag(link(U, xmm, nu)), link(U, xmm, mu))));
  // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
  q = add(q, mul(mul(dag(link(U, xmm, mu)), dag(link(U, xmm_mn, nu))), mul(link(U, xmm_mn, mu), link(U, xmn, nu))));
  // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
  q = add(q, mul(mul(dag(link(U, xmn, nu)), link(U, xmn, mu)), mul(link(U, xpm_mn, nu), dag(link(U, s, mu)))));
  M3 f = add(q, dag(q), -1.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) f.m[i][j] = 0.125 * f.m[i][j];
  return f;
}

// Invert a 6 x 6 complex matrix in place by Gauss-Jordan elimination with
// partial pivoting (|re| + |im|).  Returns false on a pivot below 1e-12.
__device__ bool invert6(cplx<double> (&a)[6][6], cplx<double> (&inv)[6][6]) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) inv[i][j] = cmake(i == j ? 1.0 : 0.0, 0.0);
  for (int c = 0; c < 6; ++c) {
    int p = c;
    double best = fabs(a[c][c].re) + fabs(a[c][c].im);
    for (int r = c + 1; r < 6; ++r) {
      const double v = fabs(a[r][c].re) + fabs(a[r][c].im);
      if (v > best) { best = v; p = r; }
    }
    if (!(best > 1e-12)) return false;
    if (p != c)
      for (int j = 0; j < 6; ++j) {
        cplx<double> t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t;
        t = inv[c][j]; inv[c][j] = inv[p][j]; inv[p][j] = t;
      }
    const cplx<double> d = a[c][c];
    const double dn = norm2(d);
    const cplx<double> di = cmake(d.re / dn, -d.im / dn);
    for (int j = 0; j < 6; ++j) { a[c][j] = a[c][j] * di; inv[c][j] = inv[c][j] * di; }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const cplx<double> f = a[r][c];
      for (int j = 0; j < 6; ++j) {
        a[r][j] = a[r][j] - f * a[c][j];
        inv[r][j] = inv[r][j] - f * inv[c][j];
      }
    }
  }
  return true;
}

__global__ void __launch_bounds__(64) k_clover(GeomK k, const double2* __restrict__ U, double cskap,
                                               double* __restrict__ c64, float* __restrict__ c32,
                                               double* __restrict__ c64dm, float* __restrict__ c32dm,
                                               int* __restrict__ bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= k.g.V) return;
  const SiteCtx c = site_ctx<LEX>(k, s);
  const int x[4] = {c.x[0], c.x[1], c.x[2], c.x[3]};
  Coord cx;
  for (int m = 0; m < 4; ++m) cx.c[m] = x[m];
  const int sdm = dm_index(k.g, cx);
  const M3 F01 = field_strength(k.g, U, x, s, 0, 1), F02 = field_strength(k.g, U, x, s, 0, 2);
  const M3 F03 = field_strength(k.g, U, x, s, 0, 3), F12 = field_strength(k.g, U, x, s, 1, 2);
  const M3 F13 = field_strength(k.g, U, x, s, 1, 3), F23 = field_strength(k.g, U, x, s, 2, 3);
  for (int blk = 0; blk < 2; ++blk) {
    const double sg = blk == 0 ? 1.0 : -1.0;
    cplx<double> a[6][6], inv[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        // Bx = +/-F03 - F12, By = F02 +/- F13, Bz = +/-F23 - F01 (upper / lower block)
        const cplx<double> bx = sg * F03.m[i][j] - F12.m[i][j];
        const cplx<double> by = F02.m[i][j] + sg * F13.m[i][j];
        const cplx<double> bz = sg * F23.m[i][j] - F01.m[i][j];
        // [[Bz, Bx - i By], [Bx + i By, -Bz]]
        const cplx<double> iby = cmake(-by.im, by.re);
        const cplx<double> blkm[2][2] = {{bz, bx - iby}, {bx + iby, cmake(-bz.re, -bz.im)}};
        for (int u = 0; u < 2; ++u)
          for (int v = 0; v < 2; ++v) {
            const cplx<double> t = blkm[u][v];
            // 1 + i cskap t
            a[3 * u + i][3 * v + j] = cmake((3 * u + i == 3 * v + j ? 1.0 : 0.0) - cskap * t.im, cskap * t.re);
          }
      }
    if (!invert6(a, inv)) *bad = 1;
    double pk[36];
    for (int i = 0; i < 6; ++i) pk[i] = inv[i][i].re;
    int o = 6;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) { pk[o++] = inv[i][j].re; pk[o++] = inv[i][j].im; }
    for (int e = 0; e < 36; ++e) {
      c64[(size_t)s * 72 + blk * 36 + e] = pk[e];
      c32[(size_t)s * 72 + blk * 36 + e] = (float)pk[e];
      c64dm[(size_t)sdm * 72 + blk * 36 + e] = pk[e];
      c32dm[(size_t)sdm * 72 + blk * 36 + e] = (float)pk[e];
    }
  }
}

// Unpack the FP64 lexicographic inverse to full 12 x 12 complex site matrices
// (row 3*spin + colour), for checks.
__global__ void k_clover_unpack(int V, const double* __restrict__ c64, double2* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  for (int e = 0; e < 144; ++e) out[(size_t)s * 144 + e] = make_double2(0, 0);
  for (int blk = 0; blk < 2; ++blk) {
    const double* pk = c64 + (size_t)s * 72 + blk * 36;
    const int o0 = 6 * blk;
    for (int i = 0; i < 6; ++i) out[(size_t)s * 144 + (o0 + i) * 12 + o0 + i] = make_double2(pk[i], 0);
    int o = 6;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        const double re = pk[o++], im = pk[o++];
        out[(size_t)s * 144 + (o0 + i) * 12 + o0 + j] = make_double2(re, im);
        out[(size_t)s * 144 + (o0 + j) * 12 + o0 + i] = make_double2(re, -im);
      }
  }
}

// out = (1 + T)^{-1} in on an FP64 lexicographic N x L block.
__global__ void __launch_bounds__(256) k_clover_apply(GeomK k, int L, const double2* __restrict__ in,
                                                      double2* __restrict__ out) {
  const int s = blockIdx.x * blockDim.y + threadIdx.y;
  if (s >= k.g.V) return;
  const int col = threadIdx.x;
  cplx<double> v[4][3][1];
  for (int sp = 0; sp < 4; ++sp)
    for (int a = 0; a < 3; ++a) {
      const double2 e = in[((size_t)s * 12 + 3 * sp + a) * L + col];
      v[sp][a][0] = cmake(e.x, e.y);
    }
  clover_apply<LEX, 1, double>(k, s, v);
  for (int sp = 0; sp < 4; ++sp)
    for (int a = 0; a < 3; ++a)
      out[((size_t)s * 12 + 3 * sp + a) * L + col] = make_double2(v[sp][a][0].re, v[sp][a][0].im);
}

}  // namespace

int launch_clover_apply(const mbbs_lattice_s* lat, int L, const double2* in, double2* out, hipStream_t st) {
  const int S = std::max(1, 256 / L);
  hipLaunchKernelGGL(k_clover_apply, dim3(ceil_div(lat->g.V, S)), dim3(L, S), 0, st, lat->gk, L, in, out);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

int clover_build(mbbs_lattice_s* lat, double csw, hipStream_t st) {
  const size_t V = lat->g.V;
  auto release = [&]() {
    (void)hipFree(lat->cl64); (void)hipFree(lat->cl32); (void)hipFree(lat->cl64dm); (void)hipFree(lat->cl32dm);
    lat->cl64 = lat->cl64dm = nullptr;
    lat->cl32 = lat->cl32dm = nullptr;
    for (int o = 0; o < 2; ++o) { lat->gk.cinv64[o] = nullptr; lat->gk.cinv32[o] = nullptr; }
    lat->gk.clov = 0;
    lat->csw = 0;
  };
  release();
  if (csw == 0.0) return MBBS_OK;
  if (hipMalloc(&lat->cl64, V * 72 * sizeof(double)) != hipSuccess ||
      hipMalloc(&lat->cl64dm, V * 72 * sizeof(double)) != hipSuccess ||
      hipMalloc(&lat->cl32, V * 72 * sizeof(float)) != hipSuccess ||
      hipMalloc(&lat->cl32dm, V * 72 * sizeof(float)) != hipSuccess) {
    release();
    set_error("out of device memory for the clover inverse");
    return MBBS_ENOMEM;
  }
  int* bad = nullptr;
  if (hipMalloc(&bad, sizeof(int)) != hipSuccess) { release(); set_error("out of device memory"); return MBBS_ENOMEM; }
  int hbad = 0;
  bool ok = hipMemsetAsync(bad, 0, sizeof(int), st) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_clover, dim3(ceil_div((int)V, 64)), dim3(64), 0, st, lat->gk, (const double2*)lat->U64,
                       csw * lat->kappa, lat->cl64, lat->cl32, lat->cl64dm, lat->cl32dm, bad);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
  }
  (void)hipFree(bad);
  if (!ok) { release(); set_error("clover construction failed"); return MBBS_EHIP; }
  if (hbad) { release(); set_error("1 + clover term is singular at some site"); return MBBS_EBREAKDOWN; }
  lat->gk.cinv64[LEX] = lat->cl64;
  lat->gk.cinv64[DM] = lat->cl64dm;
  lat->gk.cinv32[LEX] = lat->cl32;
  lat->gk.cinv32[DM] = lat->cl32dm;
  lat->gk.clov = 1;
  lat->csw = csw;
  return MBBS_OK;
}

int clover_unpack(const mbbs_lattice_s* lat, double2* out, hipStream_t st) {
  MBBS_CHECK(lat->gk.clov, "no clover term set on this lattice");
  hipLaunchKernelGGL(k_clover_unpack, dim3(ceil_div(lat->g.V, 64)), dim3(64), 0, st, lat->g.V,
                     (const double*)lat->cl64, out);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

}  // namespace mbbs
