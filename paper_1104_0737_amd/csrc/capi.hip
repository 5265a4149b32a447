// C-ABI entry points for the operator, the SAP preconditioner and the block
// linear algebra (the solver's own entry points live with the solver).
#include <cmath>
#include <mutex>
#include <vector>

#include "blas.h"

using namespace mbbs;

namespace {

int prec_ok(int p) { return p == MBBS_FP64 || p == MBBS_FP32 || p == MBBS_FP16S; }
size_t elem_bytes(int p) { return p == MBBS_FP64 ? 16 : p == MBBS_FP32 ? 8 : 4; }

// Device scratch owned by one call (only the accuracy-check entry points use it).
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n ? n : 1) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

}  // namespace

extern "C" int mbbs_apply_dirac_raw(mbbs_lattice_t lat, int L, int prec, const void* X, const float* Xs, void* Y,
                                    float* Ys, void* stream) {
  MBBS_CHECK(lat && X && Y && X != Y, "null or aliased arguments");
  MBBS_CHECK(L >= 1 && L <= 256, "L must be in 1..256");
  MBBS_CHECK(prec_ok(prec), "bad precision");
  MBBS_CHECK(prec != MBBS_FP16S || (Xs && Ys), "FP16S needs scale arrays");
  return launch_dslash(lat, L, prec, prec, LEX, false, X, Xs, Y, Ys, 0, lat->g.V, nullptr, (hipStream_t)stream);
}

static int apply_generic(mbbs_lattice_t lat, int L, const double* X, double* Y, int prec, bool blocked, void* stream) {
  MBBS_CHECK(lat && X && Y && X != Y, "null or aliased arguments");
  MBBS_CHECK(L >= 1 && L <= 256, "L must be in 1..256");
  MBBS_CHECK(prec_ok(prec), "bad precision");
  hipStream_t st = (hipStream_t)stream;
  if (prec == MBBS_FP64)
    return launch_dslash(lat, L, P64, P64, LEX, blocked, X, nullptr, Y, nullptr, 0, lat->g.V, nullptr, st);
  Scratch s;
  const size_t V = lat->g.V;
  void* a = s.get(V * 12 * L * elem_bytes(prec));
  void* b = s.get(V * 12 * L * elem_bytes(prec));
  float* as = prec == MBBS_FP16S ? (float*)s.get(V * L * sizeof(float)) : nullptr;
  float* bs = prec == MBBS_FP16S ? (float*)s.get(V * L * sizeof(float)) : nullptr;
  if (!a || !b || (prec == MBBS_FP16S && (!as || !bs))) {
    set_error("out of device memory");
    return MBBS_ENOMEM;
  }
  MBBS_TRY(launch_convert_to(prec, V, L, (const double2*)X, a, as, st));
  MBBS_TRY(launch_dslash(lat, L, prec, prec, LEX, blocked, a, as, b, bs, 0, lat->g.V, nullptr, st));
  MBBS_TRY(launch_convert_from(prec, V, L, b, bs, (double2*)Y, st));
  MBBS_HIP(hipStreamSynchronize(st));
  return MBBS_OK;
}

extern "C" int mbbs_apply_dirac(mbbs_lattice_t lat, int L, const double* X, double* Y, int prec, void* stream) {
  return apply_generic(lat, L, X, Y, prec, false, stream);
}

extern "C" int mbbs_apply_blocked(mbbs_lattice_t lat, int L, const double* X, double* Y, int prec, void* stream) {
  return apply_generic(lat, L, X, Y, prec, true, stream);
}

extern "C" int mbbs_convert_to(int prec, size_t nsites, int L, const double* X, void* Y, float* Ys, void* stream) {
  MBBS_CHECK(X && Y && L >= 1 && prec_ok(prec), "bad arguments");
  MBBS_CHECK(prec != MBBS_FP16S || Ys, "FP16S needs a scale array");
  return launch_convert_to(prec, nsites, L, (const double2*)X, Y, Ys, (hipStream_t)stream);
}

extern "C" int mbbs_convert_from(int prec, size_t nsites, int L, const void* X, const float* Xs, double* Y,
                                 void* stream) {
  MBBS_CHECK(X && Y && L >= 1 && prec_ok(prec), "bad arguments");
  MBBS_CHECK(prec != MBBS_FP16S || Xs, "FP16S needs a scale array");
  return launch_convert_from(prec, nsites, L, X, Xs, (double2*)Y, (hipStream_t)stream);
}

extern "C" int mbbs_sap_workspace_size(mbbs_lattice_t lat, int L, int prec, size_t* bytes) {
  MBBS_CHECK(lat && bytes && L >= 1 && prec_ok(prec), "bad arguments");
  *bytes = sap_buffer_bytes(lat, L, prec);
  return MBBS_OK;
}

extern "C" int mbbs_sap_apply(mbbs_lattice_t lat, int L, const double* X, double* Y, int ncy, int nmr, int prec,
                              void* ws, size_t ws_bytes, void* stream) {
  MBBS_CHECK(lat && X && Y && X != Y, "null or aliased arguments");
  MBBS_CHECK(L >= 1 && L <= 64, "L must be in 1..64");
  MBBS_CHECK(ncy >= 1 && nmr >= 1, "ncy and nmr must be >= 1");
  MBBS_CHECK(prec_ok(prec), "bad precision");
  SapBuffers b;
  MBBS_TRY(sap_bind(lat, L, prec, ws, ws_bytes, &b));
  return sap_apply(lat, b, ncy, nmr, (const double2*)X, nullptr, (double2*)Y, nullptr, (hipStream_t)stream, nullptr);
}

static int ssor_args(mbbs_lattice_t lat, int L, int nssor, double omega, int prec) {
  MBBS_CHECK(lat != nullptr, "null lattice");
  MBBS_CHECK(L >= 1 && L <= 64, "L must be in 1..64");
  MBBS_CHECK(nssor == 0 || nssor == 1, "N_SSOR must be 0 or 1");
  MBBS_CHECK(std::isfinite(omega) && omega > 0 && omega < 2, "SSOR omega must lie in (0, 2)");
  MBBS_CHECK(prec_ok(prec), "bad precision");
  return MBBS_OK;
}

extern "C" int mbbs_ssor_workspace_size(mbbs_lattice_t lat, int L, int prec, size_t* bytes) {
  MBBS_CHECK(lat && bytes, "null argument");
  MBBS_CHECK(L >= 1 && L <= 64, "L must be in 1..64");
  MBBS_CHECK(prec_ok(prec), "bad precision");
  *bytes = sap_buffer_bytes(lat, L, prec, true);
  return MBBS_OK;
}

extern "C" int mbbs_sap_apply_ssor(mbbs_lattice_t lat, int L, const double* X, double* Y, int ncy, int nssor,
                                   double omega, int prec, void* ws, size_t ws_bytes, void* stream) {
  MBBS_TRY(ssor_args(lat, L, nssor, omega, prec));
  MBBS_CHECK(X && Y && X != Y, "null or aliased arguments");
  MBBS_CHECK(ncy >= 1, "ncy must be >= 1");
  SapBuffers b;
  MBBS_TRY(sap_bind(lat, L, prec, ws, ws_bytes, &b, true));
  b.nssor = nssor;
  b.ssor_omega = omega;
  return sap_apply(lat, b, ncy, 0, (const double2*)X, nullptr, (double2*)Y, nullptr, (hipStream_t)stream, nullptr);
}

extern "C" int mbbs_apply_ssor_blocked(mbbs_lattice_t lat, int L, const double* X, double* Y, int nssor,
                                       double omega, int prec, void* ws, size_t ws_bytes, void* stream) {
  MBBS_TRY(ssor_args(lat, L, nssor, omega, prec));
  MBBS_CHECK(X && Y && X != Y, "null or aliased arguments");
  SapBuffers b;
  MBBS_TRY(sap_bind(lat, L, prec, ws, ws_bytes, &b, true));
  b.nssor = nssor;
  b.ssor_omega = omega;
  return ssor_blocked_apply(lat, b, (const double2*)X, (double2*)Y, (hipStream_t)stream);
}

extern "C" int mbbs_gram_workspace_size(size_t N, int L, size_t* bytes) {
  MBBS_CHECK(bytes && L >= 1 && L <= LMAX_SOLVER, "bad arguments");
  *bytes = gram_partial_bytes(N, L);
  return MBBS_OK;
}

extern "C" int mbbs_gram(size_t N, int L, const double* X, const double* Y, double* G, void* ws, size_t ws_bytes,
                         void* stream) {
  MBBS_CHECK(X && Y && G && L >= 1 && L <= LMAX_SOLVER, "bad arguments");
  MBBS_CHECK(ws && ws_bytes >= gram_partial_bytes(N, L), "Gram workspace too small");
  GramArgs a{};
  a.npair = 1;
  a.X[0] = (const double2*)X;
  a.Y[0] = (const double2*)Y;
  GramOut o{};
  o.G[0] = (double2*)G;
  return launch_gram(L, N, a, o, (double2*)ws, nullptr, (hipStream_t)stream);
}

// ---------------------------------------------------------------- no allocation
// Static device scratch of mbbs_gram_noalloc: the per-block partial Gram
// matrices (at most GRAM_MAXBLK blocks x GRAM_MAXPAIR products x 16 x 16
// complex doubles, 12 MiB).  Each device the library runs on holds its own
// copy until the process ends.  In host code `scratch` is only a stand-in
// for the symbol: its device address, per device, comes from
// hipGetSymbolAddress and is the only form passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES =
    (size_t)GRAM_MAXBLK * GRAM_MAXPAIR * LMAX_SOLVER * LMAX_SOLVER * sizeof(double2);
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up once per device (with
// that device current) on the first call there.
int scratch_address(double2** out) {
  int dev = -1;
  MBBS_HIP(hipGetDevice(&dev));
  MBBS_CHECK(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return MBBS_EHIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = (double2*)g_scratch_dev[dev];
  return MBBS_OK;
}
}  // namespace

extern "C" int mbbs_gram_noalloc(size_t N, int L, const double* X, const double* Y, double* G, void* stream) {
  MBBS_CHECK(X && Y && G, "null argument");
  MBBS_CHECK(L >= 1 && L <= LMAX_SOLVER, "L must be in 1..16 (the static scratch holds 16 x 16 partials)");
  MBBS_CHECK(gram_partial_bytes(N, L) <= NOALLOC_SCRATCH_BYTES, "Gram partials exceed the static scratch");
  double2* partial = nullptr;
  MBBS_TRY(scratch_address(&partial));
  // every block writes its own partial before the finishing pass reads it:
  // nothing in the scratch has to start at zero
  GramArgs a{};
  a.npair = 1;
  a.X[0] = (const double2*)X;
  a.Y[0] = (const double2*)Y;
  GramOut o{};
  o.G[0] = (double2*)G;
  return launch_gram(L, N, a, o, partial, nullptr, (hipStream_t)stream);
}

extern "C" int mbbs_cholqr(size_t N, int L, const double* P, double* Q, double* gamma, int passes, void* ws,
                           size_t ws_bytes, void* stream) {
  MBBS_CHECK(P && Q && gamma && L >= 1 && L <= LMAX_SOLVER, "bad arguments");
  MBBS_CHECK(passes == 1 || passes == 2, "passes must be 1 or 2");
  const size_t LL = (size_t)L * L * sizeof(double2);
  const size_t need = gram_partial_bytes(N, L) + 5 * LL + 256;
  MBBS_CHECK(ws && ws_bytes >= need, "CholQR workspace too small (Gram partials + 5 L x L + 256 bytes)");
  hipStream_t st = (hipStream_t)stream;
  double2* partial = (double2*)ws;
  char* q = (char*)ws + gram_partial_bytes(N, L);
  double2* G = (double2*)q;
  double2* g1 = (double2*)(q + LL);
  double2* gi = (double2*)(q + 2 * LL);
  double2* g2 = (double2*)(q + 3 * LL);
  double2* gtmp = (double2*)(q + 4 * LL);
  int* ok = (int*)(q + 5 * LL);
  const double2* src = (const double2*)P;
  for (int pass = 0; pass < passes; ++pass) {
    GramArgs a{};
    a.npair = 1;
    a.X[0] = src;
    a.Y[0] = src;
    GramOut o{};
    o.G[0] = G;
    MBBS_TRY(launch_gram(L, N, a, o, partial, nullptr, st));
    MBBS_TRY(launch_chol_standalone(L, G, pass == 0 ? g1 : g2, gi, ok, st));
    int hok = 0;
    MBBS_HIP(hipMemcpyAsync(&hok, ok, sizeof(int), hipMemcpyDeviceToHost, st));
    MBBS_HIP(hipStreamSynchronize(st));
    if (!hok) {
      set_error("P^H P is not numerically positive definite");
      return MBBS_EBREAKDOWN;
    }
    ComboArgs c{};
    c.nin = 1;
    c.mode[0] = 2;
    c.in[0] = src;
    c.coef[0] = gi;
    MBBS_TRY(launch_combo(L, N, c, (double2*)Q, 0, nullptr, nullptr, nullptr, st));
    src = (const double2*)Q;
  }
  if (passes == 2) {
    MBBS_TRY(launch_matmul_small(L, g2, g1, gtmp, st));
    MBBS_HIP(hipMemcpyAsync(gamma, gtmp, LL, hipMemcpyDeviceToDevice, st));
  } else {
    MBBS_HIP(hipMemcpyAsync(gamma, g1, LL, hipMemcpyDeviceToDevice, st));
  }
  return MBBS_OK;
}

extern "C" int mbbs_lu_solve(int L, int m, const double* G, const double* R, double* X, void* stream) {
  MBBS_CHECK(G && R && X && L >= 1 && L <= 32 && m >= 1 && m <= 32, "bad arguments (L, m in 1..32)");
  hipStream_t st = (hipStream_t)stream;
  int* ok = nullptr;
  MBBS_HIP(hipMalloc(&ok, sizeof(int)));
  int rc = launch_lu_standalone(L, m, (const double2*)G, (const double2*)R, (double2*)X, ok, st);
  int hok = 0;
  if (rc == MBBS_OK && (hipMemcpyAsync(&hok, ok, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
    rc = MBBS_EHIP;
  (void)hipFree(ok);
  if (rc == MBBS_OK && !hok) {
    set_error("zero pivot in the LU factorisation");
    return MBBS_EBREAKDOWN;
  }
  return rc;
}
