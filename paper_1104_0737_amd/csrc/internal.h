// Internal host-side declarations shared by the library's translation units.
#pragma once

#include <string>
#include <vector>

#include "common.h"
#include "../../include/mbbs.h"

namespace mbbs {

// Error reporting: a thread-local message plus a status code.
void set_error(const std::string& msg);
const char* last_error();

#define MBBS_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::mbbs::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
      return MBBS_EHIP;                                                           \
    }                                                                             \
  } while (0)

#define MBBS_CHECK(cond, msg)                                                     \
  do {                                                                            \
    if (!(cond)) {                                                                \
      ::mbbs::set_error(msg);                                                     \
      return MBBS_EINVAL;                                                         \
    }                                                                             \
  } while (0)

#define MBBS_TRY(call)                                                            \
  do {                                                                            \
    int r_ = (call);                                                              \
    if (r_ < 0) return r_;                                                        \
  } while (0)

// Unsigned division by a runtime constant: q = umulhi(n, mul) >> shift
// (Granlund-Montgomery round-up method), exact for 0 <= n < 2^31.
struct FastDiv {
  uint32_t d, mul, shift;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0, 0};
  if (d == 1) { f.mul = 0; f.shift = 0; return f; }
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.shift = l - 1;
  f.mul = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  if (f.d == 1) return n;
  uint32_t t = __umulhi(n, f.mul);
  return (t + ((n - t) >> 1)) >> f.shift;
}

// Geometry plus the fast dividers and strides the kernels need.
struct GeomK {
  Geom g;
  FastDiv fd[4];     // extents
  FastDiv fb[4];     // block sizes
  FastDiv fnd0;      // domains along x
  FastDiv fnd[4];    // domains along each direction
  FastDiv fVb;       // block volume
  int lstride[4];    // local strides inside a domain
  int stride[4];     // lexicographic strides
  int nt_store;      // operator output written with nontemporal stores
  // clover (Jacobi preconditioned): (1 + T)^{-1} per site, packed (72 reals),
  // indexed [order]; clov = 0 means the plain Wilson operator
  const double* cinv64[2];
  const float* cinv32[2];
  int clov;
  // A batch of nsys independent systems of one shape is stacked along t:
  // system s owns t in [s * tsys, (s + 1) * tsys) and its t hops wrap inside
  // that range; its hopping parameter is kap[s] (device) and its solver flag
  // frozen[s * fstride].  A single system has nsys = 1, tsys = g.d[3].
  int nsys;
  int tsys;          // t extent of one system
  int ndt;           // domains along t per system
  int Vsys;          // sites per system
  FastDiv ftsys, fndt;
  const double* kap; // per-system kappa (device), null: the kernel's scalar kappa
  int fstride;       // ints between consecutive systems' solver flags
};
GeomK make_geomk(const Geom& g, int nsys = 1);
// ints between consecutive solver state records (the flag `frozen` is the
// first field of each; checked against the record's layout in blas.h)
constexpr int SOLVER_FLAG_STRIDE = 10;

// Workgroups are dealt to the 8 XCDs of the chip in turn (block b runs on XCD
// b mod 8).  Remap so that XCD x processes one contiguous run of logical
// blocks, in order: spatial neighbours then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

}  // namespace mbbs

struct mbbs_lattice_s {
  mbbs::Geom g;      // for a batch: the stacked geometry (t extent nsys * tsys)
  mbbs::GeomK gk;
  double kappa;      // a batch keeps its systems' values in kap_dev / kap_host
  int nsys = 1;      // systems stacked along t (1: a single lattice)
  double* kap_dev = nullptr;
  std::vector<double> kap_host;
  int device;
  double2* U64 = nullptr;     // lexicographic links (FP64), [site][mu][a][b]
  float2* U32 = nullptr;
  __half2* U16 = nullptr;
  double2* U64dm = nullptr;   // domain-major links
  float2* U32dm = nullptr;
  __half2* U16dm = nullptr;
  // launch tuning (set through mbbs_lattice_tune): columns per column group
  // of the stencil kernels per precision (0: all columns in one group) and
  // the target number of threads per block
  int group_cols[3] = {0, 0, 0};
  int block_threads[3] = {256, 256, 256};   // target threads per block, per precision
  int lds_pad_kb = 0;   // extra LDS per stencil block: caps resident blocks per CU
  int split[3] = {0, 0, 0};  // hop groups per site (0/1: one thread does all 8 hops)
  int persist_blocks = 0;    // resident blocks per CU of persistent split kernels (0: not persistent)
  int mr_fused = -1;         // SAP domain solve in one launch per colour: -1 auto, 0 off, 1 on
  int hop_pair[3] = {0, 0, 0};  // operator: both hops of a direction in flight at once
  int nt_store[3] = {0, 0, 0};  // operator: nontemporal output stores
  int chunk[3] = {0, 0, 0};     // columns per thread of the stencil kernels (0: automatic)
  int tile[3] = {0, 0, 0};      // LDS-tiled operator and MR kernels: 0 off, 1 on, 2 on with the MR update fused,
                                // 3 on with tiles of at most half the LDS
  int tile_lg[3] = {0, 0, 0};   // columns per tiled workgroup (0: all L)
  int mr_once[3] = {0, 0, 0};   // MR domain solves form psi once from r_0 and the steps' A r (1) or step by step (0)
  // SSOR wavefront order inside a domain: local indices sorted by the
  // hyperplane h = l_0 + l_1 + l_2 + l_3 (then by local index); hyperplane h
  // holds entries hp_off[h] .. hp_off[h+1]-1 (device arrays)
  double* cl64 = nullptr;    // (1 + T)^{-1}, packed, lexicographic / domain-major
  float* cl32 = nullptr;
  double* cl64dm = nullptr;
  float* cl32dm = nullptr;
  double csw = 0;
  int* hp_loc = nullptr;
  int* hp_off = nullptr;
  int nh = 0;          // number of hyperplanes, sum_mu (b_mu - 1) + 1
  int hp_max = 0;      // sites in the largest hyperplane
};

namespace mbbs {

// ---------------------------------------------------------------- launchers
// Field order of a kernel's sites.
enum Order { LEX = 0, DM = 1 };

// out = in - kappa * H(in) on sites [s0, s0 + n) (order `order`), all hops
// (blocked = false) or in-domain hops only (blocked = true).
int launch_dslash(const mbbs_lattice_s* lat, int L, int prec_in, int prec_out, int order,
                  bool blocked, const void* in, const float* in_s, void* out, float* out_s,
                  int s0, int n, const int* frozen, hipStream_t st);

// SAP pieces (domain-major order, colour c sites [c*Vh, (c+1)*Vh)).
struct SapBuffers {
  int L, prec;             // prec of r, w, eta; psi is FP64 for P64 else FP32
  void* eta; float* eta_s;
  void* r;   float* r_s;
  void* w;   float* w_s;
  void* psi;               // double2 or float2
  double* partial;         // per block, per column: (wr.re, wr.im, ww)
  double* omega;           // per domain-of-colour, per column: complex step
  // domain solver: MR (ssor = 0) or SSOR with nssor correction terms and
  // relaxation ssor_omega; SSOR needs one more field x2
  int ssor = 0, nssor = 1;
  double ssor_omega = 1.0;
  void* x2 = nullptr; float* x2_s = nullptr;
  // MR with the update folded into the next step (tiled kernels): second
  // residual and A r buffers, the steps alternate between the two.  MR with
  // psi formed once per domain solve: r2 holds r_1, r_2, ... and w, w2,
  // wx[0], wx[1] keep the steps' A r
  void* r2 = nullptr; float* r2_s = nullptr;
  void* w2 = nullptr; float* w2_s = nullptr;
  void* wx[2] = {nullptr, nullptr}; float* wx_s[2] = {nullptr, nullptr};
};
size_t sap_buffer_bytes(const mbbs_lattice_s* lat, int L, int prec, bool ssor = false);
int sap_bind(const mbbs_lattice_s* lat, int L, int prec, void* ws, size_t bytes, SapBuffers* b, bool ssor = false);
// Clover: build (1 + T)^{-1} from the lattice's links (csw = 0 removes it);
// out = (1 + T)^{-1} in on an FP64 lexicographic block; unpack to 12 x 12.
int clover_build(mbbs_lattice_s* lat, double csw, hipStream_t st);
int launch_clover_apply(const mbbs_lattice_s* lat, int L, const double2* in, double2* out, hipStream_t st);
int clover_unpack(const mbbs_lattice_s* lat, double2* out, hipStream_t st);

// FP64 lexicographic block -> SAP storage of b.prec (dst, dst_s), optionally
// right-multiplied by gam; SAP psi -> FP64 lexicographic block.
int sap_to(const mbbs_lattice_s* lat, const SapBuffers& b, const double2* in, const double2* gam, void* dst,
           float* dst_s, const int* frozen, hipStream_t st);
int sap_from(const mbbs_lattice_s* lat, const SapBuffers& b, double2* out, const int* frozen, hipStream_t st);
// SSOR domain inverse B on every domain of one colour: psi (+)= B r on those
// domains (assign: psi = B r).  rmode < 0: r holds the input; 0, 1, 2: the
// input is the SAP residual eta - A psi (modes of the SAP residual kernel),
// formed inside the first sweep.  r, w and x2 are overwritten.
int ssor_colour(const mbbs_lattice_s* lat, const SapBuffers& b, int colour, bool assign, int rmode,
                const int* frozen, hipStream_t st);
// out = B in on every domain (both colours), FP64 lexicographic blocks.
int ssor_blocked_apply(const mbbs_lattice_s* lat, const SapBuffers& b, const double2* in, double2* out,
                       hipStream_t st);
// Full preconditioner application.  `in` is an FP64 lexicographic block;
// if gam != nullptr, in is right-multiplied by the L x L matrix gam (device,
// row-major) first.  out (FP64 lexicographic) receives psi.  `frozen` (device
// int, may be null) makes every kernel a no-op when nonzero.
int sap_apply(const mbbs_lattice_s* lat, const SapBuffers& b, int ncy, int nmr,
              const double2* in, const double2* gam, double2* out, const int* frozen,
              hipStream_t st, struct Profiler* prof);

// Conversions between the FP64 ABI block and the precision storages.
int launch_convert_to(int prec, size_t nsites, int L, const double2* x, void* y, float* ys,
                      hipStream_t st);
int launch_convert_from(int prec, size_t nsites, int L, const void* x, const float* xs,
                        double2* y, hipStream_t st);

// Index tables.
int build_table(const mbbs_lattice_s* lat, int which, int32_t* dev_out, hipStream_t st);
size_t table_entries(const mbbs_lattice_s* lat, int which);

// Kernel-class timing with HIP events (solver profile mode).
struct Profiler {
  static constexpr int CAP = 512;
  bool on = false;
  hipStream_t st = nullptr;
  hipEvent_t ev[2 * CAP];
  int cls[CAP];
  int n = 0;
  double ms[MBBS_K_COUNT] = {0};
  long long launches[MBBS_K_COUNT] = {0};
  void begin(int k);
  void end();
  void flush();
};

// Launch configuration helpers.
inline int pick_chunk(const mbbs_lattice_s* lat, int L, int prec) {
  // columns per thread: amortise link loads and index work over columns
  const int forced = lat->chunk[prec];
  if (forced >= 1 && forced <= 4 && L % forced == 0) return forced;
  int cmax = prec == P64 ? 1 : 2;
  for (int c = cmax; c > 1; --c)
    if (L % c == 0) return c;
  return 1;
}

// Persistent launches: gridDim.x blocks (a multiple of 8) walk `nlb` logical
// blocks.  Block b runs on XCD x = b mod 8 and takes the logical blocks of
// that XCD's contiguous range [x*nlb/8, (x+1)*nlb/8) with stride gridDim.x/8,
// so the blocks resident on one XCD always work on neighbouring sites.
struct PersistRange {
  int first, end, step;
};
__device__ __forceinline__ PersistRange persist_range(int nlb) {
  const int x = blockIdx.x & 7, j = blockIdx.x >> 3, per = gridDim.x >> 3;
  PersistRange r;
  r.first = (int)(((long long)x * nlb) / 8) + j;
  r.end = (int)(((long long)(x + 1) * nlb) / 8);
  r.step = per;
  return r;
}

// Decomposition of a stencil launch into (tile, column group, site block):
// logical block lb covers sites [t*Vb + b*S, +S) of the traversal and the
// column group g; blocks of one tile's column group are consecutive so that
// they run together on one XCD.
__device__ __forceinline__ void decompose(int lb, int bpt, int ngroups, int S, int& site, int& g) {
  const int per_tile = ngroups * bpt;
  const int t = lb / per_tile;
  const int rem = lb - t * per_tile;
  g = rem / bpt;
  const int b = rem - g * bpt;
  site = (t * bpt + b) * S + (int)threadIdx.y;
}

}  // namespace mbbs
