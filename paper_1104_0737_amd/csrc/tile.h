// LDS-tiled stencil launches: a workgroup owns one tile (a sub-block of a SAP
// domain) and all L columns or a group of them, stages the tile's input
// spinors in LDS, and reads from global memory only the neighbours outside
// the tile.
#pragma once

#include "internal.h"

namespace mbbs {

struct TileArgs {
  int t[4];        // tile extents (each divides the SAP block extent; powers of two)
  int lt[4];       // their base-2 logarithms
  int tstr[4];     // strides of the tile-local lexicographic index
  int ts;          // sites per tile
  int tpd;         // tiles per domain
  int lg;          // columns per workgroup (a divisor of L)
  int ng;          // workgroups per tile: L / lg
  unsigned lds;    // dynamic LDS bytes per workgroup
};

// Columns per thread of the tiled kernels: 1 in FP64, 2 otherwise.
inline int tile_cols(int prec) { return prec == P64 ? 1 : 2; }

// Whether the tiled kernels serve this lattice, L and precision (the knob is
// on, L fits the kernel's column split, a tile shape fits LDS and one
// workgroup), with the tile shape in *out.
bool tile_plan(const mbbs_lattice_s* lat, int L, int prec, TileArgs* out);

// out = in - kappa H in on sites [s0, s0 + n) of order `order` (whole domains;
// LEX: the whole lattice), all hops or in-domain hops only (blocked); input
// and output of precision `prec`.
int launch_dslash_tiled(const mbbs_lattice_s* lat, int L, int prec, int order, bool blocked, const TileArgs& T,
                        const void* in, const float* in_s, void* out, float* out_s, int s0, int n,
                        const int* frozen, hipStream_t st);

// MR step, part 1, on one colour's domains (domain-major sites [s0, s0 + n)):
// w = A_DD r and per tile and column the sums (<w, r>.re, <w, r>.im, <w, w>)
// into partial[((dom * tpd + tile) * L + col) * 3 + m].
int launch_mr_dslash_tiled(const mbbs_lattice_s* lat, int L, int prec, const TileArgs& T, const void* r,
                           const float* r_s, void* w, float* w_s, int s0, int n, double* partial, const int* frozen,
                           hipStream_t st);

// The SAP residual on one colour's domains (domain-major sites [s0, s0 + n)),
// general case: r = eta - psi + kappa H psi over all hops (with the clover
// step when set), psi staged in LDS.  prec is the SAP storage precision of
// eta and r; psi is FP64 for FP64 and FP32 otherwise.
bool tile_plan_resid(const mbbs_lattice_s* lat, int L, int prec, TileArgs* out);
int launch_resid_tiled(const mbbs_lattice_s* lat, int L, int prec, const TileArgs& T, const void* eta,
                       const float* eta_s, const void* psi, void* r, float* r_s, int s0, int n, const int* frozen,
                       hipStream_t st);

// MR step with the previous step's update folded in, on one colour's domains:
// psi (+)= omega r_old (assign: =), r_new = r_old - omega w_old, then
// w_new = A_DD r_new and the partials as launch_mr_dslash_tiled.  omega holds
// the previous step's values per domain and column; r_new / w_new must not
// alias r_old / w_old (other tiles still read those).
int launch_mr_fused_tiled(const mbbs_lattice_s* lat, int L, int prec, const TileArgs& T, const void* r_old,
                          const float* r_old_s, const void* w_old, const float* w_old_s, void* r_new, float* r_new_s,
                          void* w_new, float* w_new_s, void* psi, const double* omega, bool assign, int s0, int n,
                          double* partial, const int* frozen, hipStream_t st);

}  // namespace mbbs
