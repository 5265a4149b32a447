// Per-thread site context and neighbour arithmetic shared by the stencil
// kernels and the index-table builder (so the exported tables certify the
// very index computations the kernels perform).
#pragma once

#include "internal.h"

namespace mbbs {

// Per-thread site context: coordinates and, in domain-major order, the
// domain coordinates and local coordinates (computed once, hops are then
// incremental).
// In a batch of systems stacked along t, x[3] is the t coordinate inside the
// site's own system `sys` and dc[3] the domain coordinate in the stack.
struct SiteCtx {
  int s;        // index in the field's order
  int x[4];     // coordinates inside the site's system
  int l[4];     // local coordinates in the domain (DM order)
  int dc[4];    // domain coordinates (DM order; dc[3] counts over the stack)
  int colour;
  int loc;      // local index (DM order)
  int sys;      // system of a stacked batch (0 for a single system)
};

template <int ORDER>
__device__ __forceinline__ SiteCtx site_ctx(const GeomK& k, int s) {
  SiteCtx c;
  c.s = s;
  if constexpr (ORDER == LEX) {
    uint32_t q = s;
    uint32_t q1 = fdiv(q, k.fd[0]); c.x[0] = q - q1 * k.g.d[0];
    uint32_t q2 = fdiv(q1, k.fd[1]); c.x[1] = q1 - q2 * k.g.d[1];
    uint32_t q3 = fdiv(q2, k.fd[2]); c.x[2] = q2 - q3 * k.g.d[2];
    c.sys = fdiv(q3, k.ftsys);
    c.x[3] = q3 - c.sys * k.tsys;
    c.colour = 0; c.loc = 0;
    for (int m = 0; m < 4; ++m) { c.l[m] = 0; c.dc[m] = 0; }
  } else {
    c.colour = s >= k.g.Vh;
    uint32_t rem = s - c.colour * k.g.Vh;
    uint32_t kk = fdiv(rem, k.fVb);
    uint32_t loc = rem - kk * k.g.Vb;
    c.loc = loc;
    uint32_t id = 2 * kk;
    uint32_t t0 = fdiv(id, k.fnd0);
    int d0 = id - t0 * k.g.nd[0];
    int d1 = t0 % k.g.nd[1];
    uint32_t t1 = t0 / k.g.nd[1];
    int d2 = t1 % k.g.nd[2];
    int d3 = t1 / k.g.nd[2];
    if (((d0 + d1 + d2 + d3) & 1) != c.colour) d0 += 1;
    c.dc[0] = d0; c.dc[1] = d1; c.dc[2] = d2; c.dc[3] = d3;
    uint32_t q1 = fdiv(loc, k.fb[0]); c.l[0] = loc - q1 * k.g.b[0];
    uint32_t q2 = fdiv(q1, k.fb[1]); c.l[1] = q1 - q2 * k.g.b[1];
    uint32_t q3 = fdiv(q2, k.fb[2]); c.l[2] = q2 - q3 * k.g.b[2];
    c.l[3] = q3;
    c.sys = fdiv(d3, k.fndt);
    for (int m = 0; m < 3; ++m) c.x[m] = c.dc[m] * k.g.b[m] + c.l[m];
    c.x[3] = (d3 - c.sys * k.ndt) * k.g.b[3] + c.l[3];
  }
  return c;
}

// Lexicographic context of the i-th site of a tiled traversal: tiles are the
// SAP blocks in lexicographic order of the domain grid, sites inside a tile
// in local lexicographic order.  Used to walk lexicographic fields tile by
// tile so that a tile's neighbour data stays in one XCD's L2.
__device__ __forceinline__ SiteCtx site_ctx_tiled(const GeomK& k, int i) {
  SiteCtx c;
  const uint32_t tile = fdiv(i, k.fVb);
  const uint32_t loc = i - tile * k.g.Vb;
  uint32_t q = tile, r;
  int tc[4], lc[4];
  r = fdiv(q, k.fnd[0]); tc[0] = q - r * k.g.nd[0]; q = r;
  r = fdiv(q, k.fnd[1]); tc[1] = q - r * k.g.nd[1]; q = r;
  r = fdiv(q, k.fnd[2]); tc[2] = q - r * k.g.nd[2]; tc[3] = r;
  q = loc;
  r = fdiv(q, k.fb[0]); lc[0] = q - r * k.g.b[0]; q = r;
  r = fdiv(q, k.fb[1]); lc[1] = q - r * k.g.b[1]; q = r;
  r = fdiv(q, k.fb[2]); lc[2] = q - r * k.g.b[2]; lc[3] = r;
  for (int m = 0; m < 4; ++m) {
    c.x[m] = tc[m] * k.g.b[m] + lc[m];
    c.l[m] = lc[m];
    c.dc[m] = tc[m];
  }
  c.s = c.x[0] + k.stride[1] * c.x[1] + k.stride[2] * c.x[2] + k.stride[3] * c.x[3];
  c.sys = fdiv(tc[3], k.fndt);
  c.x[3] -= c.sys * k.tsys;
  c.colour = 0;
  c.loc = loc;
  return c;
}

// Lexicographic index (over the stack) of a site context of either order.
__device__ __forceinline__ int lex_of(const GeomK& k, const SiteCtx& c) {
  return c.x[0] + k.stride[1] * c.x[1] + k.stride[2] * c.x[2] + k.stride[3] * (c.x[3] + c.sys * k.tsys);
}

// Extent along mu inside one system (t hops wrap at the system's own extent).
__device__ __forceinline__ int wrap_extent(const GeomK& k, int mu) { return mu == 3 ? k.tsys : k.g.d[mu]; }

// The hopping parameter of the site's system (a batch keeps one per system).
__device__ __forceinline__ double kappa_of(const GeomK& k, const SiteCtx& c, double kappa) {
  return k.kap ? k.kap[c.sys] : kappa;
}

// System of the dom-th domain of one colour (each colour's domains are
// ordered system by system, ndom / (2 nsys) of them per system).
__device__ __forceinline__ int sys_of_domain(const GeomK& k, int dom) {
  return k.nsys == 1 ? 0 : dom / (k.g.ndom / (2 * k.nsys));
}

// Whether the site's system has stopped iterating (solver flag, may be null).
__device__ __forceinline__ bool sys_frozen(const GeomK& k, const int* frozen, int sys) {
  return frozen && frozen[sys * k.fstride];
}

// Neighbour index of the site along (mu, dir) in the field's order.
template <int ORDER>
__device__ __forceinline__ int neighbour(const GeomK& k, const SiteCtx& c, int mu, int dir) {
  if constexpr (ORDER == LEX) {
    const int ext = wrap_extent(k, mu);
    int v = c.x[mu] + dir;
    if (v == ext) return c.s - (ext - 1) * k.stride[mu];
    if (v < 0) return c.s + (ext - 1) * k.stride[mu];
    return c.s + dir * k.stride[mu];
  } else {
    int lv = c.l[mu] + dir;
    if (lv >= 0 && lv < k.g.b[mu]) return c.s + dir * k.lstride[mu];
    int dc[4] = {c.dc[0], c.dc[1], c.dc[2], c.dc[3]};
    // the domain grid wraps inside the site's system (t: ndt domains from sys * ndt)
    const int lo = mu == 3 ? c.sys * k.ndt : 0, nd = mu == 3 ? k.ndt : k.g.nd[mu];
    int nv = dc[mu] + dir;
    dc[mu] = nv < lo ? lo + nd - 1 : (nv == lo + nd ? lo : nv);
    int nl = dir > 0 ? 0 : k.g.b[mu] - 1;
    int loc = c.loc + (nl - c.l[mu]) * k.lstride[mu];
    int id = dc[0] + k.g.nd[0] * (dc[1] + k.g.nd[1] * (dc[2] + k.g.nd[2] * dc[3]));
    return (1 - c.colour) * k.g.Vh + (id >> 1) * k.g.Vb + loc;
  }
}

}  // namespace mbbs
