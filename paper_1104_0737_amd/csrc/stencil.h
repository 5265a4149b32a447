// Stencil building blocks shared by the operator, SAP and SSOR kernels: one
// thread owns one site and C consecutive right-hand sides, loads each link
// once and applies it to all C columns (the link reuse across right-hand
// sides of Sec. 2.1's block hopping-term equation), accumulating the
// spin-projected hops in registers.
#pragma once

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
// FWD_IN / BWD_IN: only the forward / only the backward hops inside the
// domain (the two triangular parts of A_DD used by the SSOR sweeps).
enum Hops { ALL = 0, INSIDE = 1, OUTSIDE = 2, FWD_IN = 3, BWD_IN = 4 };

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
  } else if constexpr ((HOPS == FWD_IN && !FWD) || (HOPS == BWD_IN && FWD)) {
    return true;
  } else {
    int r = (ORDER == DM) ? c.l[MU] : (c.x[MU] % k.g.b[MU]);
    bool leaves = FWD ? (r == k.g.b[MU] - 1) : (r == 0);
    return HOPS == OUTSIDE ? !leaves : leaves;
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

// The 9 elements of link (site ls, direction MU) in storage format.  The four
// links of a site are contiguous and the site's record is 16-byte aligned
// (288 bytes in FP32, 144 in FP16 storage), so a link is read with 16-byte
// loads of the aligned window that holds it (5 loads for 72 bytes in FP32, 3
// for 36 in FP16; FP64 elements are 16 bytes already) instead of one load
// per element: fewer memory instructions for the same cache lines.
template <int PL, int MU>
__device__ __forceinline__ void link_load(const LinkElem<PL>* __restrict__ U, int ls,
                                          typename RawT<PL>::T* __restrict__ lk) {
  if constexpr (PL == P32) {
    constexpr int off = MU & 1;                       // window starts 8 bytes early for odd MU
    const float4* w = (const float4*)(U + (size_t)ls * 36 + 9 * MU - off);
    float win[20];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const float4 v = w[i];
      win[4 * i] = v.x; win[4 * i + 1] = v.y; win[4 * i + 2] = v.z; win[4 * i + 3] = v.w;
    }
#pragma unroll
    for (int e = 0; e < 18; ++e) lk[e] = win[2 * off + e];
  } else if constexpr (PL == P16) {
    constexpr int off = (9 * MU) & 3;                 // window: 12 elements from a 16-byte boundary
    const uint4* w = (const uint4*)(U + (size_t)ls * 36 + 9 * MU - off);
    unsigned win[12];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const uint4 v = w[i];
      win[4 * i] = v.x; win[4 * i + 1] = v.y; win[4 * i + 2] = v.z; win[4 * i + 3] = v.w;
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) lk[e] = win[off + e];
  } else {
    const LinkElem<PL>* lp = U + ((size_t)ls * 4 + MU) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) raw_split<PL>(lp[e], &lk[e * RawT<PL>::per]);
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
  link_load<PL, MU>(U, ls, d.lk);
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
  const bool wrap = FWD ? (c.x[MU] == wrap_extent(k, MU) - 1) : (c.x[MU] == 0);
  cplx<R> ph = cmake<R>((R)1, (R)0);
  constexpr bool may_wrap = HOPS == ALL || HOPS == OUTSIDE;   // in-domain hops never cross the boundary
  if (may_wrap && wrap) ph = cmake<R>((R)k.g.ph[MU][0], (R)(FWD ? k.g.ph[MU][1] : -k.g.ph[MU][1]));
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
    if (may_wrap && wrap) {
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
          s0 = cmac(s0, u.m[a][b], h0[b]);
          s1 = cmac(s1, u.m[a][b], h1[b]);
        } else {              // U^dagger h
          s0 = cmac_conj(s0, u.m[b][a], h0[b]);
          s1 = cmac_conj(s1, u.m[b][a], h1[b]);
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

// Two hops of one sense (forward if F) in directions MU1 and MU2, with the
// loads of both in flight together.
template <int PIN, int PL, int C, int ORDER, int HOPS, int MU1, int MU2, int F, typename R>
__device__ __forceinline__ void hop_two_dirs(const GeomK& k, const SiteCtx& c, const typename Store<PIN>::Elem* in,
                                             const float* in_s, const LinkElem<PL>* U, int L, int col0,
                                             cplx<R> (&acc)[4][3][C], R& token) {
  const bool s1 = hop_skipped<ORDER, HOPS, MU1, F>(k, c), s2 = hop_skipped<ORDER, HOPS, MU2, F>(k, c);
  int sn1 = neighbour<ORDER>(k, c, MU1, F ? 1 : -1), sn2 = neighbour<ORDER>(k, c, MU2, F ? 1 : -1);
  int ls1 = F ? c.s : sn1, ls2 = F ? c.s : sn2;
  asm volatile("" : "+v"(sn1), "+v"(ls1), "+v"(sn2), "+v"(ls2) : "v"(token));
  HopData<PIN, PL, C> d1, d2;
  if (!s1) hop_load<PIN, PL, C, MU1>(sn1, ls1, in, in_s, U, L, col0, d1);
  if (!s2) hop_load<PIN, PL, C, MU2>(sn2, ls2, in, in_s, U, L, col0, d2);
  if (!s1) hop_pin(d1);
  if (!s2) hop_pin(d2);
  if (!s1) hop_compute<PIN, PL, C, HOPS, MU1, F, R>(k, c, d1, acc);
  if (!s2) hop_compute<PIN, PL, C, HOPS, MU2, F, R>(k, c, d2, acc);
  hop_settle(acc, token);
}

// The four hops of one sense (HOPS = FWD_IN or BWD_IN: the triangular parts
// of A_DD), as two pairs of directions with each pair's loads in flight.
template <int PIN, int PL, int C, int ORDER, int HOPS, typename R>
__device__ __forceinline__ void hop_sense_sum(const GeomK& k, const SiteCtx& c,
                                              const typename Store<PIN>::Elem* __restrict__ in,
                                              const float* __restrict__ in_s,
                                              const LinkElem<PL>* __restrict__ U, int L, int col0,
                                              cplx<R> (&acc)[4][3][C]) {
  static_assert(HOPS == FWD_IN || HOPS == BWD_IN, "one-sense hop sets only");
  constexpr int F = HOPS == FWD_IN ? 1 : 0;
  R token = 0;
  hop_two_dirs<PIN, PL, C, ORDER, HOPS, 0, 1, F, R>(k, c, in, in_s, U, L, col0, acc, token);
  hop_two_dirs<PIN, PL, C, ORDER, HOPS, 2, 3, F, R>(k, c, in, in_s, U, L, col0, acc, token);
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

// acc <- (1 + T(s))^{-1} acc for the C columns of a thread (clover, Jacobi
// preconditioned).  The inverse is two hermitian 6 x 6 blocks (spins {0,1}
// and {2,3}, row 3*spin' + colour), packed: 6 real diagonal entries, then
// (i, j), i < j, row by row as (re, im).  Rows are read one at a time.
template <int ORDER, int C, typename R>
__device__ __forceinline__ void clover_apply(const GeomK& k, int s, cplx<R> (&acc)[4][3][C]) {
  const R* m;
  if constexpr (sizeof(R) == 8) m = (const R*)k.cinv64[ORDER] + (size_t)s * 72;
  else m = (const R*)k.cinv32[ORDER] + (size_t)s * 72;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const R* p = m + 36 * blk;
    cplx<R> out[6][C];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
      for (int q = 0; q < C; ++q) out[i][q] = p[i] * acc[2 * blk + i / 3][i % 3][q];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        if (j == i) continue;
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        const int o = 6 + 2 * (lo * 6 - lo * (lo + 1) / 2 + (hi - lo - 1));
        const cplx<R> e = cmake<R>(p[o], i < j ? p[o + 1] : -p[o + 1]);
#pragma unroll
        for (int q = 0; q < C; ++q) out[i][q] = out[i][q] + e * acc[2 * blk + j / 3][j % 3][q];
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int q = 0; q < C; ++q) acc[2 * blk + i / 3][i % 3][q] = out[i][q];
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

// The MR step's updates (Sec. 2.2, minimal residual domain solver): omega * r
// for psi and r - omega * w for the residual.  The products are written with
// explicit FMAs, so every kernel that performs the step rounds alike.
template <typename R>
__device__ __forceinline__ cplx<R> mr_mul(cplx<R> a, cplx<R> b) {
  return {fmar(a.re, b.re, -(a.im * b.im)), fmar(a.re, b.im, a.im * b.re)};
}
// psi_i = d (assign) or psi_i + d.
template <int PPSI, typename R>
__device__ __forceinline__ void mr_psi_update(typename Store<PPSI>::Elem* psi, size_t i, cplx<R> d, bool assign) {
  using RP = typename Store<PPSI>::Real;
  if (assign) {
    Store<PPSI>::st(psi, i, cplx<RP>{(RP)d.re, (RP)d.im});
  } else {
    const auto pv = Store<PPSI>::ld(psi, i);
    Store<PPSI>::st(psi, i, cplx<RP>{(RP)(pv.re + (RP)d.re), (RP)(pv.im + (RP)d.im)});
  }
}

}  // namespace mbbs
