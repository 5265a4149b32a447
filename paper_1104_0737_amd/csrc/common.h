// Shared device/host definitions: complex arithmetic, storage formats,
// lattice geometry and the Wilson hop in the chiral gamma basis.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>

namespace mbbs {

// ------------------------------------------------------------------ complex
template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmake(R a, R b) { return cplx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cdot(cplx<R> a, cplx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ R norm2(cplx<R> a) { return a.re * a.re + a.im * a.im; }

// Fused multiply-adds, written out so that a complex multiply-accumulate is
// four FMAs (the compiler contracts a*b - c*d + s into mul + fma + add).
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// s + a * b
template <typename R>
__device__ __forceinline__ cplx<R> cmac(cplx<R> s, cplx<R> a, cplx<R> b) {
  return {fmar(-a.im, b.im, fmar(a.re, b.re, s.re)), fmar(a.im, b.re, fmar(a.re, b.im, s.im))};
}
// s + conj(a) * b
template <typename R>
__device__ __forceinline__ cplx<R> cmac_conj(cplx<R> s, cplx<R> a, cplx<R> b) {
  return {fmar(a.im, b.im, fmar(a.re, b.re, s.re)), fmar(-a.im, b.re, fmar(a.re, b.im, s.im))};
}

// Multiply by one of the units +1, +i, -1, -i (code 0..3).
template <int U, typename R>
__device__ __forceinline__ cplx<R> unit_mul(cplx<R> a) {
  if constexpr (U == 0) return a;
  else if constexpr (U == 1) return {-a.im, a.re};
  else if constexpr (U == 2) return {-a.re, -a.im};
  else return {a.im, -a.re};
}

// ------------------------------------------------------------------ precision
enum Prec { P64 = 0, P32 = 1, P16 = 2 };

// Storage traits of a spinor field.  Real = arithmetic type.  Elem = stored
// complex element.  P16 keeps one float scale per (site, column).
template <int P> struct Store;
template <> struct Store<P64> {
  using Real = double;
  using Elem = double2;
  static constexpr bool scaled = false;
  __device__ __forceinline__ static cplx<double> ld(const Elem* p, size_t i) {
    double2 v = p[i];
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(Elem* p, size_t i, cplx<double> v) { p[i] = make_double2(v.re, v.im); }
  __device__ __forceinline__ static void st_nt(Elem* p, size_t i, cplx<double> v) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 x = {v.re, v.im};
    __builtin_nontemporal_store(x, (v2*)(p + i));
  }
};
template <> struct Store<P32> {
  using Real = float;
  using Elem = float2;
  static constexpr bool scaled = false;
  __device__ __forceinline__ static cplx<float> ld(const Elem* p, size_t i) {
    float2 v = p[i];
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(Elem* p, size_t i, cplx<float> v) { p[i] = make_float2(v.re, v.im); }
  __device__ __forceinline__ static void st_nt(Elem* p, size_t i, cplx<float> v) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    v2 x = {v.re, v.im};
    __builtin_nontemporal_store(x, (v2*)(p + i));
  }
};
template <> struct Store<P16> {
  using Real = float;
  using Elem = __half2;
  static constexpr bool scaled = true;
  __device__ __forceinline__ static cplx<float> ld(const Elem* p, size_t i) {
    float2 v = __half22float2(p[i]);
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(Elem* p, size_t i, cplx<float> v) {
    p[i] = __floats2half2_rn(v.re, v.im);
  }
  __device__ __forceinline__ static void st_nt(Elem* p, size_t i, cplx<float> v) {
    __half2 h = __floats2half2_rn(v.re, v.im);
    unsigned u;
    __builtin_memcpy(&u, &h, sizeof(u));
    __builtin_nontemporal_store(u, (unsigned*)(p + i));
  }
};

// Link storage: same element types; links are never scaled (|U_ab| <= 1).
template <int P> using LinkElem = typename Store<P>::Elem;

// ------------------------------------------------------------------ geometry
// Site order: site = x + Lx*(y + Ly*(z + Lz*t)).  Domain-major order (SAP):
// colour-0 domains by id, then colour-1 domains, local lexicographic inside.
// Because the number of domains along x is even, the k-th domain of a colour
// in id order is one of the pair (2k, 2k+1): its rank is id >> 1.
struct Geom {
  int d[4];        // extents
  int b[4];        // SAP block
  int nd[4];       // domains per direction
  int V, Vh, Vb;   // volume, V/2, block volume
  int ndom;        // number of domains
  double ph[4][2]; // boundary phases
};

struct Coord { int c[4]; };

__host__ __device__ __forceinline__ Coord lex_coord(const Geom& g, int s) {
  Coord r;
  r.c[0] = s % g.d[0]; s /= g.d[0];
  r.c[1] = s % g.d[1]; s /= g.d[1];
  r.c[2] = s % g.d[2];
  r.c[3] = s / g.d[2];
  return r;
}
__host__ __device__ __forceinline__ int lex_site(const Geom& g, const Coord& x) {
  return x.c[0] + g.d[0] * (x.c[1] + g.d[1] * (x.c[2] + g.d[2] * x.c[3]));
}
__host__ __device__ __forceinline__ int domain_id(const Geom& g, const Coord& x) {
  return x.c[0] / g.b[0] + g.nd[0] * (x.c[1] / g.b[1] + g.nd[1] * (x.c[2] / g.b[2] + g.nd[2] * (x.c[3] / g.b[3])));
}
__host__ __device__ __forceinline__ int domain_colour(const Geom& g, const Coord& x) {
  return (x.c[0] / g.b[0] + x.c[1] / g.b[1] + x.c[2] / g.b[2] + x.c[3] / g.b[3]) & 1;
}
__host__ __device__ __forceinline__ int local_index(const Geom& g, const Coord& x) {
  return x.c[0] % g.b[0] + g.b[0] * (x.c[1] % g.b[1] + g.b[1] * (x.c[2] % g.b[2] + g.b[2] * (x.c[3] % g.b[3])));
}
__host__ __device__ __forceinline__ int dm_index(const Geom& g, const Coord& x) {
  return domain_colour(g, x) * g.Vh + (domain_id(g, x) >> 1) * g.Vb + local_index(g, x);
}
// Inverse of dm_index.
__host__ __device__ __forceinline__ Coord dm_coord(const Geom& g, int i) {
  int colour = i >= g.Vh;
  int rem = i - colour * g.Vh;
  int k = rem / g.Vb;
  int loc = rem - k * g.Vb;
  int id = 2 * k;
  int dc0 = id % g.nd[0], t = id / g.nd[0];
  int dc1 = t % g.nd[1]; t /= g.nd[1];
  int dc2 = t % g.nd[2];
  int dc3 = t / g.nd[2];
  if (((dc0 + dc1 + dc2 + dc3) & 1) != colour) dc0 += 1;
  Coord r;
  r.c[0] = dc0 * g.b[0] + loc % g.b[0]; loc /= g.b[0];
  r.c[1] = dc1 * g.b[1] + loc % g.b[1]; loc /= g.b[1];
  r.c[2] = dc2 * g.b[2] + loc % g.b[2];
  r.c[3] = dc3 * g.b[3] + loc / g.b[2];
  return r;
}

// Neighbour of x along mu (dir = +1 forward, -1 backward), wrapped; `wrapped`
// tells whether the hop crossed the lattice boundary.
__host__ __device__ __forceinline__ Coord hop(const Geom& g, Coord x, int mu, int dir, bool& wrapped) {
  int v = x.c[mu] + dir;
  wrapped = false;
  if (v == g.d[mu]) { v = 0; wrapped = true; }
  if (v < 0) { v = g.d[mu] - 1; wrapped = true; }
  x.c[mu] = v;
  return x;
}
// True when the hop from x along (mu, dir) leaves x's SAP domain.
__host__ __device__ __forceinline__ bool leaves_domain(const Geom& g, const Coord& x, int mu, int dir) {
  int r = x.c[mu] % g.b[mu];
  return dir > 0 ? (r == g.b[mu] - 1) : (r == 0);
}

// ------------------------------------------------------------------ spin
// Chiral basis, gamma_k = [[0,-i s_k],[i s_k,0]] (mu = k-1), gamma_4 = [[0,1],[1,0]].
// (1 -/+ gamma_mu) has rank 2: the upper half h = (h0, h1) is
//   h0 = psi0 + A0 * psi[P0], h1 = psi1 + A1 * psi[P1]
// and after the colour multiply chi = W h the lower half of the result is
//   out2 += B0 * chi[Q0], out3 += B1 * chi[Q1].
// Unit codes: 0 = +1, 1 = +i, 2 = -1, 3 = -i.  Table for the "minus" sign
// (forward hop); the "plus" sign (backward hop) negates A and B.
struct SpinRule { int P0, A0, P1, A1, Q0, B0, Q1, B1; };
__host__ __device__ constexpr SpinRule spin_rule(int mu, int fwd) {
  // mu 0: h = (psi0 + i psi3, psi1 + i psi2), lower = (-i chi1, -i chi0)
  // mu 1: h = (psi0 + psi3, psi1 - psi2),     lower = (-chi1, +chi0)
  // mu 2: h = (psi0 + i psi2, psi1 - i psi3), lower = (-i chi0, +i chi1)
  // mu 3: h = (psi0 - psi2, psi1 - psi3),     lower = (-chi0, -chi1)
  return fwd ? (mu == 0 ? SpinRule{3, 1, 2, 1, 1, 3, 0, 3}
              : mu == 1 ? SpinRule{3, 0, 2, 2, 1, 2, 0, 0}
              : mu == 2 ? SpinRule{2, 1, 3, 3, 0, 3, 1, 1}
                        : SpinRule{2, 2, 3, 2, 0, 2, 1, 2})
             : (mu == 0 ? SpinRule{3, 3, 2, 3, 1, 1, 0, 1}
              : mu == 1 ? SpinRule{3, 2, 2, 0, 1, 0, 0, 2}
              : mu == 2 ? SpinRule{2, 3, 3, 1, 0, 1, 1, 3}
                        : SpinRule{2, 0, 3, 0, 0, 0, 1, 0});
}

template <int U, typename R>
__device__ __forceinline__ cplx<R> add_unit(cplx<R> a, cplx<R> b) { return a + unit_mul<U>(b); }

// Runtime-code variant (codes are compile-time constants after unrolling).
template <typename R>
__device__ __forceinline__ cplx<R> umul(int u, cplx<R> a) {
  switch (u & 3) {
    case 0: return a;
    case 1: return {-a.im, a.re};
    case 2: return {-a.re, -a.im};
    default: return {a.im, -a.re};
  }
}

// Host-side helpers -----------------------------------------------------------
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace mbbs
