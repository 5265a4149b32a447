// Multi-RHS Wilson hopping kernels (Sec. 2.1, block hopping-term equation):
// one thread owns one site and C consecutive right-hand sides, loads each of
// the 8 links once and applies it to all C columns (the link reuse across
// right-hand sides the paper builds its cache tuning on), accumulating the
// spin-projected hops in registers.  Variants: full operator, the
// domain-restricted (Dirichlet) operator of Sec. 2.2, the SAP residual
// eta - A psi, and the MR domain step with its per-domain reductions.
#include "internal.h"
#include "sitectx.h"

namespace mbbs {

template <typename R>
struct Mat3 { cplx<R> m[3][3]; };

template <int PL, typename R>
__device__ __forceinline__ Mat3<R> load_link(const LinkElem<PL>* U, int site, int mu) {
  Mat3<R> u;
  const LinkElem<PL>* p = U + ((size_t)site * 4 + mu) * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      auto v = Store<PL>::ld(p, a * 3 + b);
      u.m[a][b] = cmake<R>((R)v.re, (R)v.im);
    }
  return u;
}

// Which hops a kernel sums: every hop, only hops inside the SAP domain
// (Dirichlet operator A_DD), or only hops that leave it (coupling to the
// neighbouring domains).
enum Hops { ALL = 0, INSIDE = 1, OUTSIDE = 2 };

// One hop (MU, FWD) of the hopping term for the C columns of a thread:
// acc[spin][colour][k] += (1 -/+ gamma_mu) W psi_nb (W = U or U^dagger).
// `token` chains consecutive hops: each hop's addresses depend on the
// previous hop's accumulator (an empty asm), so its loads are not hoisted
// above it; one hop's data in flight per thread keeps register pressure low.
// Whether hop (MU, FWD) is excluded by the HOPS selection.
template <int ORDER, int HOPS, int MU, int FWD>
__device__ __forceinline__ bool hop_skipped(const GeomK& k, const SiteCtx& c) {
  if constexpr (HOPS == ALL) {
    return false;
  } else {
    int r = (ORDER == DM) ? c.l[MU] : (c.x[MU] % k.g.b[MU]);
    bool leaves = FWD ? (r == k.g.b[MU] - 1) : (r == 0);
    return HOPS == INSIDE ? leaves : !leaves;
  }
}

template <int PIN, int PL, int C, int ORDER, int HOPS, int MU, int FWD, typename R>
__device__ __forceinline__ void hop_body(const GeomK& k, const SiteCtx& c, int sn, int ls,
                                         const typename Store<PIN>::Elem* __restrict__ in,
                                         const float* __restrict__ in_s,
                                         const LinkElem<PL>* __restrict__ U, int L, int col0,
                                         cplx<R> (&acc)[4][3][C], R& token);

template <int PIN, int PL, int C, int ORDER, int HOPS, int MU, int FWD, typename R>
__device__ __forceinline__ void hop_one(const GeomK& k, const SiteCtx& c,
                                        const typename Store<PIN>::Elem* __restrict__ in,
                                        const float* __restrict__ in_s,
                                        const LinkElem<PL>* __restrict__ U, int L, int col0,
                                        cplx<R> (&acc)[4][3][C], R& token) {
  if (hop_skipped<ORDER, HOPS, MU, FWD>(k, c)) return;
  int sn = neighbour<ORDER>(k, c, MU, FWD ? 1 : -1);
  int ls = FWD ? c.s : sn;
  asm volatile("" : "+v"(sn), "+v"(ls) : "v"(token));
  hop_body<PIN, PL, C, ORDER, HOPS, MU, FWD, R>(k, c, sn, ls, in, in_s, U, L, col0, acc, token);
}

// Raw register image of the data one hop reads: C columns of the neighbour's
// spinor and the link, kept in storage format until every load of the hop
// has been issued.
template <int P> struct RawT;
template <> struct RawT<P64> { using T = double; static constexpr int per = 2; };
template <> struct RawT<P32> { using T = float; static constexpr int per = 2; };
template <> struct RawT<P16> { using T = unsigned; static constexpr int per = 1; };

template <int P>
__device__ __forceinline__ void raw_split(typename Store<P>::Elem e, typename RawT<P>::T* r) {
  if constexpr (P == P16) {
    __builtin_memcpy(r, &e, sizeof(unsigned));
  } else {
    r[0] = e.x; r[1] = e.y;
  }
}
template <int P, typename R>
__device__ __forceinline__ cplx<R> raw_join(const typename RawT<P>::T* r) {
  if constexpr (P == P16) {
    __half2 h;
    __builtin_memcpy(&h, r, sizeof(unsigned));
    float2 f = __half22float2(h);
    return cmake<R>((R)f.x, (R)f.y);
  } else {
    return cmake<R>((R)r[0], (R)r[1]);
  }
}

// One asm consuming every value a hop loads: all of the hop's loads are
// issued before its first wait (left alone, the compiler sinks each column's
// loads to just before their use: one memory round trip per column).
template <typename T, int NS, typename U, int NL>
__device__ __forceinline__ void pin_regs(T (&s)[NS], U (&l)[NL]) {
  if constexpr (NS == 12 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 12 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else if constexpr (NS == 24 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 24 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else if constexpr (NS == 36 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 36 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else if constexpr (NS == 48 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 48 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else if constexpr (NS == 72 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]), "+v"(s[48]), "+v"(s[49]), "+v"(s[50]), "+v"(s[51]), "+v"(s[52]), "+v"(s[53]), "+v"(s[54]), "+v"(s[55]), "+v"(s[56]), "+v"(s[57]), "+v"(s[58]), "+v"(s[59]), "+v"(s[60]), "+v"(s[61]), "+v"(s[62]), "+v"(s[63]), "+v"(s[64]), "+v"(s[65]), "+v"(s[66]), "+v"(s[67]), "+v"(s[68]), "+v"(s[69]), "+v"(s[70]), "+v"(s[71]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 72 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]), "+v"(s[48]), "+v"(s[49]), "+v"(s[50]), "+v"(s[51]), "+v"(s[52]), "+v"(s[53]), "+v"(s[54]), "+v"(s[55]), "+v"(s[56]), "+v"(s[57]), "+v"(s[58]), "+v"(s[59]), "+v"(s[60]), "+v"(s[61]), "+v"(s[62]), "+v"(s[63]), "+v"(s[64]), "+v"(s[65]), "+v"(s[66]), "+v"(s[67]), "+v"(s[68]), "+v"(s[69]), "+v"(s[70]), "+v"(s[71]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else if constexpr (NS == 96 && NL == 9) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]), "+v"(s[48]), "+v"(s[49]), "+v"(s[50]), "+v"(s[51]), "+v"(s[52]), "+v"(s[53]), "+v"(s[54]), "+v"(s[55]), "+v"(s[56]), "+v"(s[57]), "+v"(s[58]), "+v"(s[59]), "+v"(s[60]), "+v"(s[61]), "+v"(s[62]), "+v"(s[63]), "+v"(s[64]), "+v"(s[65]), "+v"(s[66]), "+v"(s[67]), "+v"(s[68]), "+v"(s[69]), "+v"(s[70]), "+v"(s[71]), "+v"(s[72]), "+v"(s[73]), "+v"(s[74]), "+v"(s[75]), "+v"(s[76]), "+v"(s[77]), "+v"(s[78]), "+v"(s[79]), "+v"(s[80]), "+v"(s[81]), "+v"(s[82]), "+v"(s[83]), "+v"(s[84]), "+v"(s[85]), "+v"(s[86]), "+v"(s[87]), "+v"(s[88]), "+v"(s[89]), "+v"(s[90]), "+v"(s[91]), "+v"(s[92]), "+v"(s[93]), "+v"(s[94]), "+v"(s[95]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]));
  } else if constexpr (NS == 96 && NL == 18) {
    asm volatile("" : "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]), "+v"(s[4]), "+v"(s[5]), "+v"(s[6]), "+v"(s[7]), "+v"(s[8]), "+v"(s[9]), "+v"(s[10]), "+v"(s[11]), "+v"(s[12]), "+v"(s[13]), "+v"(s[14]), "+v"(s[15]), "+v"(s[16]), "+v"(s[17]), "+v"(s[18]), "+v"(s[19]), "+v"(s[20]), "+v"(s[21]), "+v"(s[22]), "+v"(s[23]), "+v"(s[24]), "+v"(s[25]), "+v"(s[26]), "+v"(s[27]), "+v"(s[28]), "+v"(s[29]), "+v"(s[30]), "+v"(s[31]), "+v"(s[32]), "+v"(s[33]), "+v"(s[34]), "+v"(s[35]), "+v"(s[36]), "+v"(s[37]), "+v"(s[38]), "+v"(s[39]), "+v"(s[40]), "+v"(s[41]), "+v"(s[42]), "+v"(s[43]), "+v"(s[44]), "+v"(s[45]), "+v"(s[46]), "+v"(s[47]), "+v"(s[48]), "+v"(s[49]), "+v"(s[50]), "+v"(s[51]), "+v"(s[52]), "+v"(s[53]), "+v"(s[54]), "+v"(s[55]), "+v"(s[56]), "+v"(s[57]), "+v"(s[58]), "+v"(s[59]), "+v"(s[60]), "+v"(s[61]), "+v"(s[62]), "+v"(s[63]), "+v"(s[64]), "+v"(s[65]), "+v"(s[66]), "+v"(s[67]), "+v"(s[68]), "+v"(s[69]), "+v"(s[70]), "+v"(s[71]), "+v"(s[72]), "+v"(s[73]), "+v"(s[74]), "+v"(s[75]), "+v"(s[76]), "+v"(s[77]), "+v"(s[78]), "+v"(s[79]), "+v"(s[80]), "+v"(s[81]), "+v"(s[82]), "+v"(s[83]), "+v"(s[84]), "+v"(s[85]), "+v"(s[86]), "+v"(s[87]), "+v"(s[88]), "+v"(s[89]), "+v"(s[90]), "+v"(s[91]), "+v"(s[92]), "+v"(s[93]), "+v"(s[94]), "+v"(s[95]),
                 "+v"(l[0]), "+v"(l[1]), "+v"(l[2]), "+v"(l[3]), "+v"(l[4]), "+v"(l[5]), "+v"(l[6]), "+v"(l[7]), "+v"(l[8]), "+v"(l[9]), "+v"(l[10]), "+v"(l[11]), "+v"(l[12]), "+v"(l[13]), "+v"(l[14]), "+v"(l[15]), "+v"(l[16]), "+v"(l[17]));
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) asm volatile("" : "+v"(s[i]));
#pragma unroll
    for (int i = 0; i < NL; ++i) asm volatile("" : "+v"(l[i]));
  }
}

template <int PIN, int PL, int C>
struct HopData {
  typename RawT<PIN>::T sp[C * 12 * RawT<PIN>::per];   // column-major: column q at q * 12 * per
  typename RawT<PL>::T lk[9 * RawT<PL>::per];
  float sc[C];
};

template <int PIN, int PL, int C, int MU>
__device__ __forceinline__ void hop_load(int sn, int ls, const typename Store<PIN>::Elem* __restrict__ in,
                                         const float* __restrict__ in_s, const LinkElem<PL>* __restrict__ U,
                                         int L, int col0, HopData<PIN, PL, C>& d) {
  // the link first: loads complete in order, and the arithmetic on the first
  // spinor elements needs the link
  const LinkElem<PL>* lp = U + ((size_t)ls * 4 + MU) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) raw_split<PL>(lp[e], &d.lk[e * RawT<PL>::per]);
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const size_t base = (size_t)sn * 12 * L + col0 + q;
#pragma unroll
    for (int e = 0; e < 12; ++e) raw_split<PIN>(in[base + (size_t)e * L], &d.sp[(q * 12 + e) * RawT<PIN>::per]);
    if constexpr (Store<PIN>::scaled) d.sc[q] = in_s[(size_t)sn * L + col0 + q];
  }
}

// With one column per thread the loads of a hop are issued together anyway,
// and consuming each value as it arrives overlaps the tail of the loads with
// arithmetic: pin only from two columns on.
template <int PIN, int PL, int C>
__device__ __forceinline__ void hop_pin(HopData<PIN, PL, C>& d) {
  if constexpr (C > 1) pin_regs(d.sp, d.lk);
}

// The hop's arithmetic on loaded data.
template <int PIN, int PL, int C, int HOPS, int MU, int FWD, typename R>
__device__ __forceinline__ void hop_compute(const GeomK& k, const SiteCtx& c, const HopData<PIN, PL, C>& d,
                                            cplx<R> (&acc)[4][3][C]) {
  const bool wrap = FWD ? (c.x[MU] == k.g.d[MU] - 1) : (c.x[MU] == 0);
  cplx<R> ph = cmake<R>((R)1, (R)0);
  if (HOPS != INSIDE && wrap) ph = cmake<R>((R)k.g.ph[MU][0], (R)(FWD ? k.g.ph[MU][1] : -k.g.ph[MU][1]));
  Mat3<R> u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u.m[a][b] = raw_join<PL, R>(&d.lk[(a * 3 + b) * RawT<PL>::per]);
  constexpr SpinRule sr = spin_rule(MU, FWD);
#pragma unroll
  for (int q = 0; q < C; ++q) {
    cplx<R> p[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) p[sp][a] = raw_join<PIN, R>(&d.sp[(q * 12 + 3 * sp + a) * RawT<PIN>::per]);
    if constexpr (Store<PIN>::scaled) {
      const R sc = (R)d.sc[q];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) p[sp][a] = sc * p[sp][a];
    }
    cplx<R> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      h0[a] = p[0][a] + unit_mul<sr.A0>(p[sr.P0][a]);
      h1[a] = p[1][a] + unit_mul<sr.A1>(p[sr.P1][a]);
    }
    if (HOPS != INSIDE && wrap) {
#pragma unroll
      for (int a = 0; a < 3; ++a) { h0[a] = ph * h0[a]; h1[a] = ph * h1[a]; }
    }
    cplx<R> x0[3], x1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<R> s0 = cmake<R>(0, 0), s1 = cmake<R>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (FWD) {  // U h
          s0 = s0 + u.m[a][b] * h0[b];
          s1 = s1 + u.m[a][b] * h1[b];
        } else {              // U^dagger h
          s0 = s0 + cdot(u.m[b][a], h0[b]);
          s1 = s1 + cdot(u.m[b][a], h1[b]);
        }
      }
      x0[a] = s0; x1[a] = s1;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc[0][a][q] = acc[0][a][q] + x0[a];
      acc[1][a][q] = acc[1][a][q] + x1[a];
      acc[2][a][q] = acc[2][a][q] + unit_mul<sr.B0>(sr.Q0 ? x1[a] : x0[a]);
      acc[3][a][q] = acc[3][a][q] + unit_mul<sr.B1>(sr.Q1 ? x1[a] : x0[a]);
    }
  }
}

// Materialise the accumulators at a hop boundary (otherwise the additions are
// deferred and every hop's partial result stays live) and pass the token on.
template <int C, typename R>
__device__ __forceinline__ void hop_settle(cplx<R> (&acc)[4][3][C], R& token) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) asm volatile("" : "+v"(acc[sp][a][q].re), "+v"(acc[sp][a][q].im));
  token = acc[0][0][0].re;
}

template <int PIN, int PL, int C, int ORDER, int HOPS, int MU, int FWD, typename R>
__device__ __forceinline__ void hop_body(const GeomK& k, const SiteCtx& c, int sn, int ls,
                                         const typename Store<PIN>::Elem* __restrict__ in,
                                         const float* __restrict__ in_s,
                                         const LinkElem<PL>* __restrict__ U, int L, int col0,
                                         cplx<R> (&acc)[4][3][C], R& token) {
  HopData<PIN, PL, C> d;
  hop_load<PIN, PL, C, MU>(sn, ls, in, in_s, U, L, col0, d);
  hop_pin(d);
  hop_compute<PIN, PL, C, HOPS, MU, FWD, R>(k, c, d, acc);
  hop_settle(acc, token);
}

// Both hops of direction MU.  PAIR: the backward hop's addresses do not wait
// for the forward hop, so both hops' loads can be in flight together.
template <int PIN, int PL, int C, int ORDER, int HOPS, int MU, typename R, bool PAIR = false>
__device__ __forceinline__ void hop_dir(const GeomK& k, const SiteCtx& c, const typename Store<PIN>::Elem* in,
                                        const float* in_s, const LinkElem<PL>* U, int L, int col0,
                                        cplx<R> (&acc)[4][3][C], R& token) {
  if constexpr (PAIR) {
    const bool sf = hop_skipped<ORDER, HOPS, MU, 1>(k, c), sb = hop_skipped<ORDER, HOPS, MU, 0>(k, c);
    int snf = neighbour<ORDER>(k, c, MU, 1), snb = neighbour<ORDER>(k, c, MU, -1);
    int lsf = c.s, lsb = snb;
    asm volatile("" : "+v"(snf), "+v"(lsf), "+v"(snb), "+v"(lsb) : "v"(token));
    HopData<PIN, PL, C> df, db;
    if (!sf) hop_load<PIN, PL, C, MU>(snf, lsf, in, in_s, U, L, col0, df);
    if (!sb) hop_load<PIN, PL, C, MU>(snb, lsb, in, in_s, U, L, col0, db);
    if (!sf) hop_pin(df);
    if (!sb) hop_pin(db);
    if (!sf) hop_compute<PIN, PL, C, HOPS, MU, 1, R>(k, c, df, acc);
    if (!sb) hop_compute<PIN, PL, C, HOPS, MU, 0, R>(k, c, db, acc);
    hop_settle(acc, token);
  } else {
    hop_one<PIN, PL, C, ORDER, HOPS, MU, 1, R>(k, c, in, in_s, U, L, col0, acc, token);
    hop_one<PIN, PL, C, ORDER, HOPS, MU, 0, R>(k, c, in, in_s, U, L, col0, acc, token);
  }
}

// All eight hops.
template <int PIN, int PL, int C, int ORDER, int HOPS, typename R, bool PAIR = false>
__device__ __forceinline__ void hop_sum(const GeomK& k, const SiteCtx& c,
                                        const typename Store<PIN>::Elem* __restrict__ in,
                                        const float* __restrict__ in_s,
                                        const LinkElem<PL>* __restrict__ U, int L, int col0,
                                        cplx<R> (&acc)[4][3][C]) {
  R token = 0;
  hop_dir<PIN, PL, C, ORDER, HOPS, 0, R, PAIR>(k, c, in, in_s, U, L, col0, acc, token);
  hop_dir<PIN, PL, C, ORDER, HOPS, 1, R, PAIR>(k, c, in, in_s, U, L, col0, acc, token);
  hop_dir<PIN, PL, C, ORDER, HOPS, 2, R, PAIR>(k, c, in, in_s, U, L, col0, acc, token);
  hop_dir<PIN, PL, C, ORDER, HOPS, 3, R, PAIR>(k, c, in, in_s, U, L, col0, acc, token);
}

// The hops of group h when the eight hops are split over P wave-uniform
// groups (P = 4: direction h; P = 2: directions 2h and 2h+1).
template <int PIN, int PL, int ORDER, int HOPS, int P, typename R>
__device__ __forceinline__ void hop_group(int h, const GeomK& k, const SiteCtx& c,
                                          const typename Store<PIN>::Elem* in, const float* in_s,
                                          const LinkElem<PL>* U, int L, int col, cplx<R> (&acc)[4][3][1]) {
  R token = 0;
  if constexpr (P == 4) {
    switch (h) {
      case 0: hop_dir<PIN, PL, 1, ORDER, HOPS, 0, R>(k, c, in, in_s, U, L, col, acc, token); break;
      case 1: hop_dir<PIN, PL, 1, ORDER, HOPS, 1, R>(k, c, in, in_s, U, L, col, acc, token); break;
      case 2: hop_dir<PIN, PL, 1, ORDER, HOPS, 2, R>(k, c, in, in_s, U, L, col, acc, token); break;
      default: hop_dir<PIN, PL, 1, ORDER, HOPS, 3, R>(k, c, in, in_s, U, L, col, acc, token); break;
    }
  } else if constexpr (P == 2) {
    if (h == 0) {
      hop_dir<PIN, PL, 1, ORDER, HOPS, 0, R>(k, c, in, in_s, U, L, col, acc, token);
      hop_dir<PIN, PL, 1, ORDER, HOPS, 1, R>(k, c, in, in_s, U, L, col, acc, token);
    } else {
      hop_dir<PIN, PL, 1, ORDER, HOPS, 2, R>(k, c, in, in_s, U, L, col, acc, token);
      hop_dir<PIN, PL, 1, ORDER, HOPS, 3, R>(k, c, in, in_s, U, L, col, acc, token);
    }
  } else {
    hop_sum<PIN, PL, 1, ORDER, HOPS, R>(k, c, in, in_s, U, L, col, acc);
  }
}

// Store one (site, column) spinor; P16 computes the per-(site, column) scale.
template <int POUT, typename R, bool NT = false>
__device__ __forceinline__ void store_spinor(typename Store<POUT>::Elem* out, float* out_s,
                                             size_t base, int L, size_t sidx, cplx<R> (&v)[4][3]) {
  if constexpr (Store<POUT>::scaled) {
    R m = 0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) m = fmaxf(m, fmaxf(fabsf(v[sp][a].re), fabsf(v[sp][a].im)));
    R inv = m > 0 ? (R)1 / m : (R)0;
    out_s[sidx] = m;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if constexpr (NT) Store<POUT>::st_nt(out, base + (size_t)(3 * sp + a) * L, inv * v[sp][a]);
        else Store<POUT>::st(out, base + (size_t)(3 * sp + a) * L, inv * v[sp][a]);
      }
  } else {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cplx<typename Store<POUT>::Real> o{(typename Store<POUT>::Real)v[sp][a].re,
                                                 (typename Store<POUT>::Real)v[sp][a].im};
        if constexpr (NT) Store<POUT>::st_nt(out, base + (size_t)(3 * sp + a) * L, o);
        else Store<POUT>::st(out, base + (size_t)(3 * sp + a) * L, o);
      }
  }
}

template <int PIN, typename R>
__device__ __forceinline__ void load_spinor(const typename Store<PIN>::Elem* in, const float* in_s,
                                            size_t base, int L, size_t sidx, cplx<R> (&v)[4][3]) {
  R sc = 1;
  if constexpr (Store<PIN>::scaled) sc = (R)in_s[sidx];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      auto e = Store<PIN>::ld(in, base + (size_t)(3 * sp + a) * L);
      v[sp][a] = cmake<R>((R)e.re * sc, (R)e.im * sc);
    }
}

// ---------------------------------------------------------------- kernels
// Thread layout: threadIdx.x = column chunk (C columns each), threadIdx.y =
// site within the block; blocks cover consecutive sites of the field order.
template <int PIN, int POUT, int PL, int C, int ORDER, bool BLOCKED, bool PAIR = false>
__global__ void __launch_bounds__(256) k_dslash(GeomK k, double kappa, int L,
                                                const typename Store<PIN>::Elem* __restrict__ in,
                                                const float* __restrict__ in_s,
                                                typename Store<POUT>::Elem* __restrict__ out,
                                                float* __restrict__ out_s,
                                                const LinkElem<PL>* __restrict__ U, int s0, int n,
                                                int bpt, int ngroups, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  if (i >= n) return;
  const int col0 = (grp * blockDim.x + threadIdx.x) * C;
  // lexicographic fields are walked tile by tile (whole lattice, s0 = 0)
  const SiteCtx c = ORDER == LEX ? site_ctx_tiled(k, i) : site_ctx<DM>(k, s0 + i);
  const int s = c.s;
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  hop_sum<PIN, PL, C, ORDER, BLOCKED ? INSIDE : ALL, R, PAIR>(k, c, in, in_s, U, L, col0, acc);
  const R kap = (R)kappa;
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
template <int PR, int PPSI, int PL, int C>
__global__ void __launch_bounds__(256) k_sap_resid(GeomK k, double kappa, int L, int s0, int n, int mode,
                                                   const typename Store<PR>::Elem* __restrict__ eta,
                                                   const float* __restrict__ eta_s,
                                                   const typename Store<PPSI>::Elem* __restrict__ psi,
                                                   typename Store<PR>::Elem* __restrict__ r,
                                                   float* __restrict__ r_s,
                                                   const LinkElem<PL>* __restrict__ U, int bpt,
                                                   int ngroups, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  if (i >= n) return;
  const int s = s0 + i;
  const int col0 = (grp * blockDim.x + threadIdx.x) * C;
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  if (mode != 0) {
    const SiteCtx c = site_ctx<DM>(k, s);
    if (mode == 1) hop_sum<PPSI, PL, C, DM, OUTSIDE, R>(k, c, psi, nullptr, U, L, col0, acc);
    else hop_sum<PPSI, PL, C, DM, ALL, R>(k, c, psi, nullptr, U, L, col0, acc);
  }
  const R kap = (R)kappa;
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
template <int PR, int PL, int C>
__global__ void __launch_bounds__(256) k_mr_dslash(GeomK k, double kappa, int L, int s0, int n,
                                                   const typename Store<PR>::Elem* __restrict__ r,
                                                   const float* __restrict__ r_s,
                                                   typename Store<PR>::Elem* __restrict__ w,
                                                   float* __restrict__ w_s,
                                                   const LinkElem<PL>* __restrict__ U,
                                                   double* __restrict__ partial, int bpt, int ngroups,
                                                   const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PL>::Real;
  extern __shared__ double red[];  // [3][blockDim.y][blockDim.x*C]
  int i, grp;
  decompose(xcd_block(blockIdx.x, gridDim.x), bpt, ngroups, blockDim.y, i, grp);
  const int s = s0 + i;  // blocks never straddle domains
  const int colg = grp * blockDim.x * C;           // first column of the group
  const int col0 = colg + threadIdx.x * C;
  const SiteCtx c = site_ctx<DM>(k, s);
  cplx<R> acc[4][3][C];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[sp][a][q] = cmake<R>(0, 0);
  hop_sum<PR, PL, C, DM, INSIDE, R>(k, c, r, r_s, U, L, col0, acc);
  const R kap = (R)kappa;
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
        cplx<R> d = cdot(wv[sp][a], v[sp][a]);
        a_re += d.re; a_im += d.im; a_ww += norm2(wv[sp][a]);
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
__global__ void __launch_bounds__(256) k_mr_omega(int L, int nblk, const double* __restrict__ partial,
                                                  double* __restrict__ omega, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  __shared__ double red[3 * 256];
  const int dom = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
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
  if (frozen && *frozen) return;
  using R = typename Store<PR>::Real;
  using RP = typename Store<PPSI>::Real;
  const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
  if (s >= s0 + n) return;
  const int col = threadIdx.x;
  const int dom = (s - (s >= k.g.Vh ? k.g.Vh : 0)) / k.g.Vb;
  const cplx<R> om = cmake<R>((R)omega[((size_t)dom * L + col) * 2], (R)omega[((size_t)dom * L + col) * 2 + 1]);
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
  if (!update_r) return;
  cplx<R> wv[4][3];
  load_spinor<PR, R>(w, w_s, base, L, sidx, wv);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) rv[sp][a] = rv[sp][a] - om * wv[sp][a];
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
  if (frozen && *frozen) return;
  using R = typename Store<PR>::Real;
  using RP = typename Store<PPSI>::Real;
  __shared__ double red[3][1024];
  __shared__ double om_sh[2 * 16];
  const int t = threadIdx.x;
  const int T = spb * L;
  const bool active = t < T;
  const int col = t % L, j = t / L;
  const int base_site = s0 + blockIdx.x * k.g.Vb;
  const R kap = (R)kappa;
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
            cplx<R> d = cdot(wv[sp][a], v[sp][a]);
            a_re += d.re; a_im += d.im; a_ww += norm2(wv[sp][a]);
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
GeomK make_geomk(const Geom& g) {
  GeomK k;
  k.g = g;
  for (int m = 0; m < 4; ++m) {
    k.fd[m] = make_fastdiv(g.d[m]);
    k.fb[m] = make_fastdiv(g.b[m]);
  }
  k.fnd0 = make_fastdiv(g.nd[0]);
  for (int m = 0; m < 4; ++m) k.fnd[m] = make_fastdiv(g.nd[m]);
  k.fVb = make_fastdiv(g.Vb);
  k.nt_store = 0;
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
  p.C = pick_chunk(L, prec);
  p.gw = lat->group_cols[prec];
  if (p.gw <= 0 || p.gw % p.C || L % p.gw) p.gw = L;
  p.nchunk = p.gw / p.C;
  p.ngroups = L / p.gw;
  p.S = sites_per_block(p.nchunk, lat->g.Vb, lat->block_threads);
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
    else if (lat->hop_pair[PL])
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
  const int P = lat->split[PL];
  if (P == 2 || P == 4) {
    const int S = split_sites(lat, L, PL, P);
    if (S > 0) {
      if (P == 4) return dslash_split_launch<PIN, POUT, PL, 4>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, S, frozen, st);
      return dslash_split_launch<PIN, POUT, PL, 2>(lat, L, order, blocked, in, in_s, out, out_s, s0, n, S, frozen, st);
    }
  }
  switch (pick_chunk(L, PL)) {
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
size_t sap_buffer_bytes(const mbbs_lattice_s* lat, int L, int prec) {
  const size_t V = lat->g.V;
  const size_t elem = prec == P64 ? 16 : prec == P32 ? 8 : 4;
  const size_t field = V * 12 * L * elem;
  const size_t scales = prec == P16 ? V * L * sizeof(float) : 0;
  const size_t psi = V * 12 * L * (prec == P64 ? 16 : 8);
  const size_t ndc = lat->g.ndom / 2;             // domains per colour
  const size_t nblk = lat->g.Vh;                  // upper bound on blocks per colour
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return al(field) * 3 + al(scales) * 3 + al(psi) + al(nblk * L * 3 * sizeof(double)) +
         al(ndc * L * 2 * sizeof(double));
}

int sap_bind(const mbbs_lattice_s* lat, int L, int prec, void* ws, size_t bytes, SapBuffers* b) {
  const size_t need = sap_buffer_bytes(lat, L, prec);
  MBBS_CHECK(ws != nullptr && bytes >= need, "SAP workspace too small");
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
  b->omega = (double*)p;
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
      const int P = lat->split[PL];
      const int SS = (P == 2 || P == 4) ? split_sites(lat, L, PL, P) : 0;
      if (prof) prof->begin(MBBS_K_SAP_RES);
      if (SS > 0) {
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
#define RES(CC)                                                                                      \
  hipLaunchKernelGGL((k_sap_resid<PR, PPSI, PL, CC>), dim3(pl.nblocks), dim3(pl.nchunk, S),                  \
                     (size_t)lat->lds_pad_kb * 1024, st,                                                     \
                     lat->gk, lat->kappa, L, s0, n, cy > 0 ? 2 : col, (const ER*)b.eta,                \
                     b.eta_s, (const EP*)b.psi, (ER*)b.r, b.r_s, U, pl.bpt, pl.ngroups, frozen)
      switch (C) { case 4: RES(4); break; case 3: RES(3); break; case 2: RES(2); break; default: RES(1); }
#undef RES
      }
      if (prof) prof->end();
      MBBS_HIP(hipGetLastError());
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
      for (int it = 0; it < nmr; ++it) {
        if (prof) prof->begin(MBBS_K_MR_DSLASH);
        int nblk_dom = g.Vb / S;
        if (SS > 0) {
          nblk_dom = g.Vb / SS;
          const size_t smem = split_smem_bytes(PL, P, SS, L);
          if (P == 4) {
            auto fn = k_mr_dslash_split<PR, PL, 4>;
            allow_lds((const void*)fn);
            hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 4, SS, L, n / SS)), dim3(SS * L, 4), smem, st, lat->gk,
                               lat->kappa, L, s0, n,
                               (const ER*)b.r, b.r_s, (ER*)b.w, b.w_s, U, b.partial, SS, frozen);
          } else {
            auto fn = k_mr_dslash_split<PR, PL, 2>;
            allow_lds((const void*)fn);
            hipLaunchKernelGGL(fn, dim3(split_grid(lat, PL, 2, SS, L, n / SS)), dim3(SS * L, 2), smem, st, lat->gk,
                               lat->kappa, L, s0, n,
                               (const ER*)b.r, b.r_s, (ER*)b.w, b.w_s, U, b.partial, SS, frozen);
          }
        } else {
#define MRD(CC)                                                                                       \
  hipLaunchKernelGGL((k_mr_dslash<PR, PL, CC>), dim3(pl.nblocks), dim3(pl.nchunk, S),                       \
                     red_bytes + (size_t)lat->lds_pad_kb * 1024, st, lat->gk,                                \
                     lat->kappa, L, s0, n, (const ER*)b.r, b.r_s, (ER*)b.w, b.w_s, U, b.partial, pl.bpt,   \
                     pl.ngroups, frozen)
        switch (C) { case 4: MRD(4); break; case 3: MRD(3); break; case 2: MRD(2); break; default: MRD(1); }
#undef MRD
        }
        MBBS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_mr_omega, dim3(g.ndom / 2), dim3(256), 0, st, L, nblk_dom, (const double*)b.partial,
                           b.omega, frozen);
        if (prof) prof->end();
        MBBS_HIP(hipGetLastError());
        if (prof) prof->begin(MBBS_K_MR_UPDATE);
        hipLaunchKernelGGL((k_mr_update<PR, PPSI>), dim3(ceil_div(n, Su)), dim3(L, Su), 0, st, lat->gk, L, s0,
                           n, (ER*)b.r, b.r_s, (const ER*)b.w, b.w_s, (EP*)b.psi, b.omega,
                           (int)(it + 1 < nmr), (int)(cy == 0 && it == 0), frozen);
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
template <int PR>
__global__ void __launch_bounds__(256) k_to_sap(GeomK k, int L, const double2* __restrict__ in,
                                                const double2* __restrict__ gam,
                                                typename Store<PR>::Elem* __restrict__ out,
                                                float* __restrict__ out_s, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  using R = typename Store<PR>::Real;
  extern __shared__ double2 gsh[];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if (gam) {
    for (int e = tid; e < L * L; e += blockDim.x * blockDim.y) gsh[e] = gam[e];
    __syncthreads();
  }
  const int s = blockIdx.x * blockDim.y + threadIdx.y;  // domain-major index
  if (s >= k.g.V) return;
  const int j = threadIdx.x;
  const SiteCtx c = site_ctx<DM>(k, s);
  Coord x;
  for (int m = 0; m < 4; ++m) x.c[m] = c.x[m];
  const int ls = lex_site(k.g, x);
  cplx<double> v[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t row = ((size_t)ls * 12 + 3 * sp + a) * L;
      if (gam) {
        cplx<double> acc = cmake(0.0, 0.0);
        for (int m = 0; m < L; ++m) {
          double2 e = in[row + m], gg = gsh[m * L + j];
          acc = acc + cmake(e.x, e.y) * cmake(gg.x, gg.y);
        }
        v[sp][a] = acc;
      } else {
        double2 e = in[row + j];
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

template <int PPSI>
__global__ void __launch_bounds__(256) k_from_sap(GeomK k, int L, const typename Store<PPSI>::Elem* __restrict__ in,
                                                  double2* __restrict__ out, const int* __restrict__ frozen) {
  if (frozen && *frozen) return;
  const int s = blockIdx.x * blockDim.y + threadIdx.y;
  if (s >= k.g.V) return;
  const int j = threadIdx.x;
  const SiteCtx c = site_ctx<DM>(k, s);
  Coord x;
  for (int m = 0; m < 4; ++m) x.c[m] = c.x[m];
  const int ls = lex_site(k.g, x);
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    auto v = Store<PPSI>::ld(in, ((size_t)s * 12 + e) * L + j);
    out[((size_t)ls * 12 + e) * L + j] = make_double2((double)v.re, (double)v.im);
  }
}

int sap_apply(const mbbs_lattice_s* lat, const SapBuffers& b, int ncy, int nmr, const double2* in,
              const double2* gam, double2* out, const int* frozen, hipStream_t st, Profiler* prof) {
  const int L = b.L;
  const Geom& g = lat->g;
  const int S = sites_per_block(L, g.V);
  if (prof) prof->begin(MBBS_K_CONVERT);
  const size_t gsh = gam ? (size_t)L * L * sizeof(double2) : 0;
  switch (b.prec) {
    case P64: hipLaunchKernelGGL((k_to_sap<P64>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (double2*)b.eta, nullptr, frozen); break;
    case P32: hipLaunchKernelGGL((k_to_sap<P32>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (float2*)b.eta, nullptr, frozen); break;
    default: hipLaunchKernelGGL((k_to_sap<P16>), dim3(ceil_div(g.V, S)), dim3(L, S), gsh, st, lat->gk, L, in, gam, (__half2*)b.eta, b.eta_s, frozen); break;
  }
  if (prof) prof->end();
  MBBS_HIP(hipGetLastError());
  // psi needs no clearing: the first MR step of the first cycle assigns it.
  int rc;
  switch (b.prec) {
    case P64: rc = sap_cycles<P64, P64, P64>(lat, b, ncy, nmr, frozen, st, prof); break;
    case P32: rc = sap_cycles<P32, P32, P32>(lat, b, ncy, nmr, frozen, st, prof); break;
    default: rc = sap_cycles<P16, P32, P16>(lat, b, ncy, nmr, frozen, st, prof); break;
  }
  if (rc < 0) return rc;
  if (prof) prof->begin(MBBS_K_CONVERT);
  if (b.prec == P64)
    hipLaunchKernelGGL((k_from_sap<P64>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const double2*)b.psi, out, frozen);
  else
    hipLaunchKernelGGL((k_from_sap<P32>), dim3(ceil_div(g.V, S)), dim3(L, S), 0, st, lat->gk, L, (const float2*)b.psi, out, frozen);
  if (prof) prof->end();
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

}  // namespace mbbs
