// Lattice handle: geometry validation, device copies of the links in every
// precision and site order the kernels read, index tables, error strings and
// the kernel-class profiler.
#include <cmath>
#include <cstring>
#include <string>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "tile.h"
#include "sitectx.h"

namespace mbbs {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

// Link copies: lexicographic FP32/FP16 and domain-major FP64/FP32/FP16.
__global__ void k_links(GeomK k, const double2* __restrict__ U, float2* __restrict__ U32, __half2* __restrict__ U16,
                        double2* __restrict__ U64dm, float2* __restrict__ U32dm, __half2* __restrict__ U16dm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // domain-major position
  if (i >= k.g.V) return;
  const SiteCtx c = site_ctx<DM>(k, i);
  const int s = lex_of(k, c);
  for (int e = 0; e < 36; ++e) {
    const double2 v = U[(size_t)i * 36 + e];  // lexicographic site i
    U32[(size_t)i * 36 + e] = make_float2((float)v.x, (float)v.y);
    U16[(size_t)i * 36 + e] = __floats2half2_rn((float)v.x, (float)v.y);
    const double2 w = U[(size_t)s * 36 + e];  // site at domain-major position i
    U64dm[(size_t)i * 36 + e] = w;
    U32dm[(size_t)i * 36 + e] = make_float2((float)w.x, (float)w.y);
    U16dm[(size_t)i * 36 + e] = __floats2half2_rn((float)w.x, (float)w.y);
  }
}

// All per-site tables, from the kernels' own index functions.
__global__ void k_tables(GeomK k, int which, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const Geom& g = k.g;
  if (which == MBBS_TAB_LOCAL_NB) {
    if (i >= g.Vb) return;
    // local site i of the first colour-0 domain (domain id 0, position i)
    const SiteCtx c = site_ctx<DM>(k, i);
    for (int mu = 0; mu < 4; ++mu)
      for (int s = 0; s < 2; ++s) {
        const int dir = s ? -1 : 1;
        const int lv = c.l[mu] + dir;
        out[(size_t)i * 8 + 2 * mu + s] = (lv >= 0 && lv < g.b[mu]) ? neighbour<DM>(k, c, mu, dir) - (i - c.loc) : -1;
      }
    return;
  }
  if (i >= g.V) return;
  if (which == MBBS_TAB_DM_NEIGHBOUR || which == MBBS_TAB_DM_SITE) {
    const SiteCtx c = site_ctx<DM>(k, i);
    if (which == MBBS_TAB_DM_SITE) {
      out[i] = lex_of(k, c);
      return;
    }
    for (int mu = 0; mu < 4; ++mu) {
      out[(size_t)i * 8 + 2 * mu] = neighbour<DM>(k, c, mu, 1);
      out[(size_t)i * 8 + 2 * mu + 1] = neighbour<DM>(k, c, mu, -1);
    }
    return;
  }
  const SiteCtx c = site_ctx<LEX>(k, i);
  Coord x;
  for (int m = 0; m < 4; ++m) x.c[m] = c.x[m];
  switch (which) {
    case MBBS_TAB_COORD:
      for (int m = 0; m < 4; ++m) out[(size_t)i * 4 + m] = c.x[m];
      break;
    case MBBS_TAB_NEIGHBOUR:
      for (int mu = 0; mu < 4; ++mu) {
        out[(size_t)i * 8 + 2 * mu] = neighbour<LEX>(k, c, mu, 1);
        out[(size_t)i * 8 + 2 * mu + 1] = neighbour<LEX>(k, c, mu, -1);
      }
      break;
    case MBBS_TAB_BOUNDARY: {
      int f = 0;
      for (int mu = 0; mu < 4; ++mu) {
        if (c.x[mu] == wrap_extent(k, mu) - 1) f |= 1 << (2 * mu);
        if (c.x[mu] == 0) f |= 1 << (2 * mu + 1);
      }
      out[i] = f;
      break;
    }
    case MBBS_TAB_PARITY: out[i] = (c.x[0] + c.x[1] + c.x[2] + c.x[3]) & 1; break;
    case MBBS_TAB_EO: out[i] = ((c.x[0] + c.x[1] + c.x[2] + c.x[3]) & 1) * g.Vh + (i >> 1); break;
    case MBBS_TAB_DOMAIN: out[i] = domain_id(g, x); break;
    case MBBS_TAB_COLOUR: out[i] = domain_colour(g, x); break;
    case MBBS_TAB_LOCAL: out[i] = local_index(g, x); break;
    case MBBS_TAB_DM_INDEX: out[i] = dm_index(g, x); break;
    default: break;
  }
}

size_t table_entries(const mbbs_lattice_s* lat, int which) {
  const size_t V = lat->g.V;
  switch (which) {
    case MBBS_TAB_COORD: return 4 * V;
    case MBBS_TAB_NEIGHBOUR: case MBBS_TAB_DM_NEIGHBOUR: return 8 * V;
    case MBBS_TAB_LOCAL_NB: return 8 * (size_t)lat->g.Vb;
    case MBBS_TAB_HYPERPLANE: return (size_t)lat->g.Vb + lat->nh + 1;
    default: return V;
  }
}

int build_table(const mbbs_lattice_s* lat, int which, int32_t* dev_out, hipStream_t st) {
  if (which == MBBS_TAB_HYPERPLANE) {   // the arrays the SSOR kernels read
    MBBS_HIP(hipMemcpyAsync(dev_out, lat->hp_loc, lat->g.Vb * sizeof(int), hipMemcpyDeviceToDevice, st));
    MBBS_HIP(hipMemcpyAsync(dev_out + lat->g.Vb, lat->hp_off, (lat->nh + 1) * sizeof(int), hipMemcpyDeviceToDevice,
                            st));
    return MBBS_OK;
  }
  const int n = which == MBBS_TAB_LOCAL_NB ? lat->g.Vb : lat->g.V;
  hipLaunchKernelGGL(k_tables, dim3(ceil_div(n, 256)), dim3(256), 0, st, lat->gk, which, dev_out);
  MBBS_HIP(hipGetLastError());
  return MBBS_OK;
}

// ---------------------------------------------------------------- profiler
void Profiler::begin(int k) {
  if (!on || n >= CAP) return;
  cls[n] = k;
  (void)hipEventRecord(ev[2 * n], st);
}
void Profiler::end() {
  if (!on || n >= CAP) return;
  (void)hipEventRecord(ev[2 * n + 1], st);
  ++n;
  if (n == CAP) flush();
}
void Profiler::flush() {
  if (!on || n == 0) return;
  (void)hipEventSynchronize(ev[2 * n - 1]);
  for (int i = 0; i < n; ++i) {
    float t = 0;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ms[cls[i]] += t;
    launches[cls[i]] += 1;
  }
  n = 0;
}

}  // namespace mbbs

using namespace mbbs;

// A lattice handle for nsys >= 1 systems of one shape: with nsys > 1 the
// systems are stacked along t (system s owns t in [s Lt, (s + 1) Lt), its t
// hops wrap inside that range) and every kernel of the handle treats them
// as independent systems with hopping parameters kappa[s].
static int lattice_create(const int dims[4], const int block[4], int nsys, const double* const* U_dev,
                          const double* kappa, const double phase[8], void* stream, mbbs_lattice_t* out) {
  MBBS_CHECK(dims && block && U_dev && kappa && phase && out, "null argument");
  MBBS_CHECK(nsys >= 1, "a batch needs at least one system");
  Geom g;
  long long V = 1;
  for (int m = 0; m < 4; ++m) {
    MBBS_CHECK(dims[m] >= 2 && dims[m] % 2 == 0, "every extent must be even and >= 2");
    MBBS_CHECK(block[m] >= 1 && dims[m] % block[m] == 0, "extent not divisible by the SAP block");
    MBBS_CHECK((dims[m] / block[m]) % 2 == 0, "the number of domains along each direction must be even");
    const double a = phase[2 * m], b = phase[2 * m + 1];
    MBBS_CHECK(std::fabs(std::sqrt(a * a + b * b) - 1.0) < 1e-12, "boundary phases must have modulus 1");
    const int stack = m == 3 ? nsys : 1;
    g.d[m] = dims[m] * stack;
    g.b[m] = block[m];
    g.nd[m] = dims[m] / block[m] * stack;
    g.ph[m][0] = a;
    g.ph[m][1] = b;
    V *= dims[m];
  }
  const long long Vsys = V;
  V *= nsys;
  MBBS_CHECK(V * 12 < (1ll << 31), "lattice (batch) too large for 32-bit site indexing");
  for (int s = 0; s < nsys; ++s) {
    MBBS_CHECK(std::isfinite(kappa[s]), "kappa must be finite");
    MBBS_CHECK(U_dev[s] != nullptr, "null link array");
  }
  g.V = (int)V;
  g.Vh = g.V / 2;
  g.Vb = block[0] * block[1] * block[2] * block[3];
  g.ndom = g.V / g.Vb;
  auto* lat = new mbbs_lattice_s();
  lat->g = g;
  lat->gk = make_geomk(g, nsys);
  lat->kappa = kappa[0];
  lat->nsys = nsys;
  (void)hipGetDevice(&lat->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)V * 36, nsys_links = (size_t)Vsys * 36;
  auto fail = [&](int rc) { mbbs_lattice_destroy(lat); return rc; };
  if (nsys > 1) {
    lat->kap_host.assign(kappa, kappa + nsys);
    if (hipMalloc(&lat->kap_dev, nsys * sizeof(double)) != hipSuccess) {
      set_error("out of device memory for the batch's kappa values");
      return fail(MBBS_ENOMEM);
    }
    if (hipMemcpy(lat->kap_dev, kappa, nsys * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("kappa copy failed");
      return fail(MBBS_EHIP);
    }
    lat->gk.kap = lat->kap_dev;
  }
  if (hipMalloc(&lat->U64, n * sizeof(double2)) != hipSuccess || hipMalloc(&lat->U32, n * sizeof(float2)) != hipSuccess ||
      hipMalloc(&lat->U16, n * sizeof(__half2)) != hipSuccess ||
      hipMalloc(&lat->U64dm, n * sizeof(double2)) != hipSuccess ||
      hipMalloc(&lat->U32dm, n * sizeof(float2)) != hipSuccess ||
      hipMalloc(&lat->U16dm, n * sizeof(__half2)) != hipSuccess) {
    set_error("out of device memory for link copies");
    return fail(MBBS_ENOMEM);
  }
  for (int s = 0; s < nsys; ++s) {
    if (hipMemcpyAsync(lat->U64 + (size_t)s * nsys_links, U_dev[s], nsys_links * sizeof(double2),
                       hipMemcpyDeviceToDevice, st) != hipSuccess) {
      set_error("link copy failed");
      return fail(MBBS_EHIP);
    }
  }
  hipLaunchKernelGGL(k_links, dim3(ceil_div(V, 256)), dim3(256), 0, st, lat->gk, (const double2*)lat->U64, lat->U32,
                     lat->U16, lat->U64dm, lat->U32dm, lat->U16dm);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    set_error("link conversion failed");
    return fail(MBBS_EHIP);
  }
  // SSOR wavefront order (counting sort of the local sites by hyperplane)
  {
    const int nh = (g.b[0] - 1) + (g.b[1] - 1) + (g.b[2] - 1) + (g.b[3] - 1) + 1;
    std::vector<int> cnt(nh + 1, 0), loc(g.Vb), hsite(g.Vb);
    for (int l = 0; l < g.Vb; ++l) {
      const int l0 = l % g.b[0], l1 = (l / g.b[0]) % g.b[1], l2 = (l / (g.b[0] * g.b[1])) % g.b[2],
                l3 = l / (g.b[0] * g.b[1] * g.b[2]);
      hsite[l] = l0 + l1 + l2 + l3;
      cnt[hsite[l] + 1] += 1;
    }
    for (int h = 0; h < nh; ++h) {
      lat->hp_max = std::max(lat->hp_max, cnt[h + 1]);
      cnt[h + 1] += cnt[h];
    }
    std::vector<int> off(cnt), pos(cnt.begin(), cnt.end() - 1);
    for (int l = 0; l < g.Vb; ++l) loc[pos[hsite[l]]++] = l;
    lat->nh = nh;
    if (hipMalloc(&lat->hp_loc, g.Vb * sizeof(int)) != hipSuccess ||
        hipMalloc(&lat->hp_off, (nh + 1) * sizeof(int)) != hipSuccess) {
      set_error("out of device memory for the wavefront tables");
      return fail(MBBS_ENOMEM);
    }
    if (hipMemcpy(lat->hp_loc, loc.data(), g.Vb * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(lat->hp_off, off.data(), (nh + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("wavefront table copy failed");
      return fail(MBBS_EHIP);
    }
  }
  *out = lat;
  return MBBS_OK;
}

extern "C" int mbbs_lattice_create(const int dims[4], const int block[4], const double* U_dev, double kappa,
                                   const double phase[8], void* stream, mbbs_lattice_t* out) {
  return lattice_create(dims, block, 1, &U_dev, &kappa, phase, stream, out);
}

extern "C" int mbbs_lattice_create_batch(int nsys, const int dims[4], const int block[4], const double* const* U_dev,
                                         const double* kappa, const double phase[8], void* stream,
                                         mbbs_lattice_t* out) {
  return lattice_create(dims, block, nsys, U_dev, kappa, phase, stream, out);
}

extern "C" int mbbs_lattice_nsys(mbbs_lattice_t lat, int* nsys) {
  MBBS_CHECK(lat != nullptr && nsys != nullptr, "null argument");
  *nsys = lat->nsys;
  return MBBS_OK;
}

extern "C" int mbbs_lattice_destroy(mbbs_lattice_t lat) {
  if (!lat) return MBBS_OK;
  (void)hipFree(lat->U64);
  (void)hipFree(lat->U32);
  (void)hipFree(lat->U16);
  (void)hipFree(lat->U64dm);
  (void)hipFree(lat->U32dm);
  (void)hipFree(lat->U16dm);
  (void)hipFree(lat->hp_loc);
  (void)hipFree(lat->hp_off);
  (void)hipFree(lat->cl64);
  (void)hipFree(lat->cl32);
  (void)hipFree(lat->cl64dm);
  (void)hipFree(lat->cl32dm);
  (void)hipFree(lat->kap_dev);
  delete lat;
  return MBBS_OK;
}

extern "C" int mbbs_lattice_set_clover(mbbs_lattice_t lat, double csw, void* stream) {
  MBBS_CHECK(lat != nullptr, "null lattice");
  MBBS_CHECK(std::isfinite(csw), "c_sw must be finite");
  MBBS_CHECK(lat->nsys == 1, "the clover term is available on single-system handles only");
  return clover_build(lat, csw, (hipStream_t)stream);
}

extern "C" int mbbs_lattice_clover_inverse(mbbs_lattice_t lat, double* out_dev, void* stream) {
  MBBS_CHECK(lat != nullptr && out_dev != nullptr, "null argument");
  MBBS_TRY(clover_unpack(lat, (double2*)out_dev, (hipStream_t)stream));
  MBBS_HIP(hipStreamSynchronize((hipStream_t)stream));
  return MBBS_OK;
}

extern "C" int mbbs_apply_clover_inverse(mbbs_lattice_t lat, int L, const double* X, double* Y, void* stream) {
  MBBS_CHECK(lat && X && Y, "null argument");
  MBBS_CHECK(L >= 1 && L <= 256, "L must be in 1..256");
  MBBS_CHECK(lat->gk.clov, "no clover term set on this lattice");
  return launch_clover_apply(lat, L, (const double2*)X, (double2*)Y, (hipStream_t)stream);
}

extern "C" int mbbs_lattice_tune(mbbs_lattice_t lat, int knob, int value) {
  MBBS_CHECK(lat != nullptr, "null lattice");
  switch (knob) {
    case MBBS_TUNE_GROUP_FP64:
    case MBBS_TUNE_GROUP_FP32:
    case MBBS_TUNE_GROUP_FP16S:
      MBBS_CHECK(value >= 0 && value <= 64, "column group out of range");
      lat->group_cols[knob] = value;
      return MBBS_OK;
    case MBBS_TUNE_BLOCK_THREADS:
      MBBS_CHECK(value >= 32 && value <= 256, "threads per block must be in 32..256");
      for (int p = 0; p < 3; ++p) lat->block_threads[p] = value;
      return MBBS_OK;
    case MBBS_TUNE_BLOCK_THREADS_FP64:
    case MBBS_TUNE_BLOCK_THREADS_FP32:
    case MBBS_TUNE_BLOCK_THREADS_FP16S:
      MBBS_CHECK(value >= 32 && value <= 256, "threads per block must be in 32..256");
      lat->block_threads[knob - MBBS_TUNE_BLOCK_THREADS_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_SPLIT_FP64:
    case MBBS_TUNE_SPLIT_FP32:
    case MBBS_TUNE_SPLIT_FP16S:
      MBBS_CHECK(value == 0 || value == 1 || value == 2 || value == 4, "split must be 0, 1, 2 or 4");
      lat->split[knob - MBBS_TUNE_SPLIT_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_PERSIST_BLOCKS:
      MBBS_CHECK(value >= 0 && value <= 16, "persistent blocks per CU must be in 0..16");
      lat->persist_blocks = value;
      return MBBS_OK;
    case MBBS_TUNE_NT_STORE_FP64:
    case MBBS_TUNE_NT_STORE_FP32:
    case MBBS_TUNE_NT_STORE_FP16S:
      MBBS_CHECK(value == 0 || value == 1, "nontemporal store flag must be 0 or 1");
      lat->nt_store[knob - MBBS_TUNE_NT_STORE_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_HOP_PAIR_FP64:
    case MBBS_TUNE_HOP_PAIR_FP32:
    case MBBS_TUNE_HOP_PAIR_FP16S:
      MBBS_CHECK(value == 0 || value == 1, "hop pairing must be 0 or 1");
      lat->hop_pair[knob - MBBS_TUNE_HOP_PAIR_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_CHUNK_FP64:
    case MBBS_TUNE_CHUNK_FP32:
    case MBBS_TUNE_CHUNK_FP16S:
      MBBS_CHECK(value >= 0 && value <= 4, "columns per thread must be 0 (automatic) or 1..4");
      lat->chunk[knob - MBBS_TUNE_CHUNK_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_TILE_FP64:
    case MBBS_TUNE_TILE_FP32:
    case MBBS_TUNE_TILE_FP16S:
      MBBS_CHECK(value >= 0 && value <= 3, "tiled stencil setting must be 0, 1, 2 or 3");
      // the folded MR update is withdrawn for FP16 storage: its only run did not finish
      MBBS_CHECK(!(value == 2 && knob == MBBS_TUNE_TILE_FP16S), "folded MR update not available for FP16 storage");
      lat->tile[knob - MBBS_TUNE_TILE_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_TILE_COLS_FP64:
    case MBBS_TUNE_TILE_COLS_FP32:
    case MBBS_TUNE_TILE_COLS_FP16S:
      MBBS_CHECK(value >= 0 && value <= 256, "columns per tiled workgroup must be in 0..256");
      lat->tile_lg[knob - MBBS_TUNE_TILE_COLS_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_MR_ONCE_FP64:
    case MBBS_TUNE_MR_ONCE_FP32:
    case MBBS_TUNE_MR_ONCE_FP16S:
      MBBS_CHECK(value == 0 || value == 1, "psi-once MR must be 0 or 1");
      lat->mr_once[knob - MBBS_TUNE_MR_ONCE_FP64] = value;
      return MBBS_OK;
    case MBBS_TUNE_MR_FUSED:
      MBBS_CHECK(value >= -1 && value <= 1, "fused MR must be -1 (auto), 0 or 1");
      lat->mr_fused = value;
      return MBBS_OK;
    case MBBS_TUNE_LDS_PAD_KB:
      MBBS_CHECK(value >= 0 && value <= 64, "LDS pad must be in 0..64 KiB");
      lat->lds_pad_kb = value;
      return MBBS_OK;
    default:
      set_error("unknown tuning knob");
      return MBBS_EINVAL;
  }
}

extern "C" int mbbs_lattice_tile_shape(mbbs_lattice_t lat, int L, int prec, int32_t* t4) {
  MBBS_CHECK(lat != nullptr && t4 != nullptr, "null argument");
  MBBS_CHECK(L >= 1 && L <= 256, "L must be in 1..256");
  MBBS_CHECK(prec >= P64 && prec <= P16, "unknown precision");
  TileArgs T;
  const bool on = tile_plan(lat, L, prec, &T);
  for (int m = 0; m < 4; ++m) t4[m] = on ? T.t[m] : 0;
  return MBBS_OK;
}

extern "C" int mbbs_lattice_table_size(mbbs_lattice_t lat, int which, size_t* count) {
  MBBS_CHECK(lat && count, "null argument");
  MBBS_CHECK(which >= 0 && which < MBBS_TAB_COUNT, "unknown table");
  *count = table_entries(lat, which);
  return MBBS_OK;
}

extern "C" int mbbs_lattice_table(mbbs_lattice_t lat, int which, int32_t* out, size_t count) {
  MBBS_CHECK(lat && out, "null argument");
  MBBS_CHECK(which >= 0 && which < MBBS_TAB_COUNT, "unknown table");
  const size_t n = table_entries(lat, which);
  MBBS_CHECK(count >= n, "output buffer too small for the table");
  int32_t* d = nullptr;
  MBBS_HIP(hipMalloc(&d, n * sizeof(int32_t)));
  int rc = build_table(lat, which, d, nullptr);
  if (rc == MBBS_OK && hipMemcpy(out, d, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("table copy failed");
    rc = MBBS_EHIP;
  }
  (void)hipFree(d);
  return rc;
}

extern "C" const char* mbbs_last_error(void) { return last_error(); }
