// C ABI of the tau = 1 lattice BGK scheme (include/maclab.h, maclab_bgk_*):
// validation, workspace layout, boundary bookkeeping and launch sequencing.
// The kernels are in kernels_bgk.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <string>

#include "internal.h"

using namespace maclab;

struct maclab_bgk_s {
  maclab_config cfg;
  int q = 0, d = 0;
  bool fp64 = false;
  int64_t nx = 0, ny = 0, nz = 0, N = 0, plane = 0;
  size_t state_bytes = 0, staging_bytes = 0;
  hipStream_t stream = nullptr;
  char* state[2] = {nullptr, nullptr};
  int cur = 0;
  char* staging = nullptr;
  FaceValues fv;
  double e = 0, dt = 0;
  int64_t steps = 0;
  std::string err;
};

namespace {

thread_local std::string g_bgk_err;

constexpr size_t kAlign = 256;
constexpr size_t kStagingMax = size_t(8) << 20;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int fail(maclab_bgk_t h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(maclab_bgk_t h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_bgk_err = buf;
  return code;
}

#define HIP_TRY(h, expr)                                                                              \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail((h), MACLAB_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

struct BgkLayout {
  int q, d;
  bool fp64;
  int64_t N, plane;
  size_t state_bytes, staging_bytes, workspace_bytes;
};

int bgk_layout(const maclab_config* c, BgkLayout* L, std::string* why) {
  if (!c) {
    *why = "config is NULL";
    return MACLAB_EINVAL;
  }
  if (c->lattice != MACLAB_D2Q9 && c->lattice != MACLAB_D3Q19) {
    *why = "lattice must be MACLAB_D2Q9 (9) or MACLAB_D3Q19 (19)";
    return MACLAB_EUNSUPPORTED;
  }
  if (c->precision != MACLAB_FP64 && c->precision != MACLAB_FP32) {
    *why = "the population scheme stores FP64 or FP32 populations";
    return MACLAB_EUNSUPPORTED;
  }
  if (!(c->dx > 0) || !isfinite(c->dx) || !(c->nu > 0) || !isfinite(c->nu) || !(c->rho_ref > 0) ||
      !isfinite(c->rho_ref)) {
    *why = "dx, nu and rho_ref must be finite and positive";
    return MACLAB_EINVAL;
  }
  for (int i = 0; i < 3; ++i)
    if (!isfinite(c->body_force[i])) {
      *why = "body_force must be finite";
      return MACLAB_EINVAL;
    }
  const int d = c->lattice == MACLAB_D2Q9 ? 2 : 3;
  for (int i = 0; i < 3; ++i)
    if (c->n[i] < 1 || c->n[i] > (int64_t(1) << 24)) {
      *why = "node counts must be in [1, 2^24]";
      return MACLAB_EINVAL;
    }
  if (d == 2 && c->n[2] != 1) {
    *why = "D2Q9 needs n[2] == 1";
    return MACLAB_EINVAL;
  }
  const int64_t nxy = c->n[0] * c->n[1];
  if (nxy > (int64_t(1) << 34) || nxy * c->n[2] > (int64_t(1) << 34)) {
    *why = "lattice too large";
    return MACLAB_EINVAL;
  }
  L->q = c->lattice;
  L->d = d;
  L->fp64 = c->precision == MACLAB_FP64;
  L->N = nxy * c->n[2];
  L->plane = (int64_t)round_up((size_t)L->N, 512) + 256;
  const size_t t = L->fp64 ? 8 : 4;
  L->state_bytes = (size_t)L->q * (size_t)L->plane * t;
  L->staging_bytes = std::min(kStagingMax, round_up(sizeof(double) * 4 * (size_t)L->N, kAlign));
  L->workspace_bytes = 2 * round_up(L->state_bytes, kAlign) + L->staging_bytes;
  return MACLAB_OK;
}

BgkParams bgk_params(const maclab_bgk_t h) {
  BgkParams p;
  p.nx = h->nx;
  p.ny = h->ny;
  p.nz = h->nz;
  p.plane = h->plane;
  for (int ax = 0; ax < 3; ++ax) p.fixed[ax] = h->fv.kind[2 * ax] == MACLAB_BC_FIXED;
  p.rho_ref = h->cfg.rho_ref;
  for (int i = 0; i < 3; ++i) p.g[i] = i < h->d ? h->dt * h->cfg.body_force[i] / h->e : 0.0;
  return p;
}

int impose(maclab_bgk_t h) {
  HIP_TRY(h, launch_bgk_impose(h->q, h->fp64, h->state[0], h->state[1], bgk_params(h), h->fv, h->e, h->stream));
  return MACLAB_OK;
}

// Nodes per host-transfer chunk: rho and d velocity planes of FP64 fit in
// the staging area.
int64_t chunk_nodes(const maclab_bgk_t h) { return (int64_t)(h->staging_bytes / (sizeof(double) * (h->d + 1))); }

}  // namespace

extern "C" {

size_t maclab_bgk_workspace_bytes(const maclab_config* cfg) {
  BgkLayout L;
  std::string why;
  return bgk_layout(cfg, &L, &why) == MACLAB_OK ? L.workspace_bytes : 0;
}

int maclab_bgk_init(const maclab_config* cfg, maclab_bgk_t* out) {
  if (!out) return fail(nullptr, MACLAB_EINVAL, "out is NULL");
  *out = nullptr;
  BgkLayout L;
  std::string why;
  const int rc = bgk_layout(cfg, &L, &why);
  if (rc != MACLAB_OK) return fail(nullptr, rc, "maclab_bgk_init: %s", why.c_str());
  if (!cfg->workspace) return fail(nullptr, MACLAB_EWORKSPACE, "maclab_bgk_init: workspace is NULL");
  if ((uintptr_t)cfg->workspace % kAlign)
    return fail(nullptr, MACLAB_EWORKSPACE, "maclab_bgk_init: workspace must be %zu-byte aligned", kAlign);
  if (cfg->workspace_bytes < L.workspace_bytes)
    return fail(nullptr, MACLAB_EWORKSPACE, "maclab_bgk_init: workspace has %zu bytes, needs %zu",
                cfg->workspace_bytes, L.workspace_bytes);
  maclab_bgk_t h = new (std::nothrow) maclab_bgk_s();
  if (!h) return fail(nullptr, MACLAB_EINVAL, "maclab_bgk_init: out of host memory");
  h->cfg = *cfg;
  h->q = L.q;
  h->d = L.d;
  h->fp64 = L.fp64;
  h->nx = cfg->n[0];
  h->ny = cfg->n[1];
  h->nz = cfg->n[2];
  h->N = L.N;
  h->plane = L.plane;
  h->state_bytes = L.state_bytes;
  h->staging_bytes = L.staging_bytes;
  h->stream = (hipStream_t)cfg->stream;
  char* ws = (char*)cfg->workspace;
  const size_t sb = round_up(L.state_bytes, kAlign);
  h->state[0] = ws;
  h->state[1] = ws + sb;
  h->staging = ws + 2 * sb;
  for (int f = 0; f < 6; ++f) {
    h->fv.kind[f] = MACLAB_BC_PERIODIC;
    h->fv.rho[f] = cfg->rho_ref;
    for (int c = 0; c < 3; ++c) h->fv.u[f][c] = 0.0;
  }
  h->e = 6.0 * cfg->nu / cfg->dx;  // Eq. (6)
  h->dt = cfg->dx / h->e;          // text after Eq. (6)
  // at rest: every population is its weight times rho_ref, a zero deviation
  const hipError_t e1 = hipMemsetAsync(ws, 0, 2 * sb, h->stream);
  if (e1 != hipSuccess) {
    const int code = fail(nullptr, MACLAB_EHIP, "maclab_bgk_init: hipMemsetAsync: %s", hipGetErrorString(e1));
    delete h;
    return code;
  }
  *out = h;
  return MACLAB_OK;
}

int maclab_bgk_set_bc(maclab_bgk_t h, int face, int kind, double rho_b, const double* u_b) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (face < 0 || face > 5) return fail(h, MACLAB_EINVAL, "face %d out of range", face);
  if (face / 2 >= h->d) return fail(h, MACLAB_EINVAL, "face %d does not exist in 2D", face);
  if (kind != MACLAB_BC_PERIODIC && kind != MACLAB_BC_FIXED)
    return fail(h, MACLAB_EINVAL, "the population scheme supports periodic and fixed faces only (kind %d)", kind);
  if (kind == MACLAB_BC_FIXED) {
    if (!u_b) return fail(h, MACLAB_EINVAL, "u_b is NULL");
    if (!(rho_b > 0) || !isfinite(rho_b)) return fail(h, MACLAB_EINVAL, "rho_b must be finite and positive");
    for (int c = 0; c < h->d; ++c)
      if (!isfinite(u_b[c])) return fail(h, MACLAB_EINVAL, "u_b must be finite");
    h->fv.rho[face] = rho_b;
    for (int c = 0; c < 3; ++c) h->fv.u[face][c] = c < h->d ? u_b[c] : 0.0;
  }
  h->fv.kind[face] = kind;
  return impose(h);
}

int maclab_bgk_set_fields(maclab_bgk_t h, const double* rho, const double* u, int on_device) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!rho || !u) return fail(h, MACLAB_EINVAL, "rho and u must not be NULL");
  const int64_t N = h->N;
  char* dst = h->state[h->cur];
  if (on_device) {
    HIP_TRY(h, launch_bgk_encode(h->q, h->fp64, dst, h->plane, rho, u, u + N, h->d == 3 ? u + 2 * N : u, 0, N,
                                 h->cfg.rho_ref, h->e, h->stream));
  } else {
    const int64_t chunk = chunk_nodes(h);
    double* st = (double*)h->staging;
    for (int64_t off = 0; off < N; off += chunk) {
      const int64_t cnt = std::min(chunk, N - off);
      HIP_TRY(h, hipMemcpyAsync(st, rho + off, sizeof(double) * cnt, hipMemcpyHostToDevice, h->stream));
      for (int c = 0; c < h->d; ++c)
        HIP_TRY(h, hipMemcpyAsync(st + (1 + c) * chunk, u + c * N + off, sizeof(double) * cnt, hipMemcpyHostToDevice,
                                  h->stream));
      double* s = st;
      HIP_TRY(h, launch_bgk_encode(h->q, h->fp64, dst, h->plane, s, s + chunk, s + 2 * chunk,
                                   h->d == 3 ? s + 3 * chunk : s + chunk, off, cnt, h->cfg.rho_ref, h->e, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));  // staging is reused
    }
  }
  HIP_TRY(h, hipMemcpyAsync(h->state[h->cur ^ 1], dst, h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
  return impose(h);
}

int maclab_bgk_step(maclab_bgk_t h, int64_t n) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, MACLAB_EINVAL, "negative step count");
  for (int ax = 0; ax < h->d; ++ax) {
    if (h->fv.kind[2 * ax] != h->fv.kind[2 * ax + 1])
      return fail(h, MACLAB_EINVAL, "faces of axis %d differ (both must be periodic or both fixed)", ax);
    const int64_t m = ax == 0 ? h->nx : (ax == 1 ? h->ny : h->nz);
    if (h->fv.kind[2 * ax] == MACLAB_BC_FIXED && m < 3)
      return fail(h, MACLAB_EINVAL, "fixed faces on axis %d need at least 3 nodes", ax);
  }
  const BgkParams p = bgk_params(h);
  for (int64_t s = 0; s < n; ++s) {
    HIP_TRY(h, launch_bgk_step(h->q, h->fp64, p, h->state[h->cur], h->state[h->cur ^ 1], h->stream));
    h->cur ^= 1;
    ++h->steps;
  }
  return MACLAB_OK;
}

int maclab_bgk_get_fields(maclab_bgk_t h, double* rho, double* u, int on_device) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!rho || !u) return fail(h, MACLAB_EINVAL, "rho and u must not be NULL");
  const int64_t N = h->N;
  const char* src = h->state[h->cur];
  if (on_device) {
    HIP_TRY(h, launch_bgk_decode(h->q, h->fp64, src, h->plane, rho, u, u + N, h->d == 3 ? u + 2 * N : u, 0, N,
                                 h->cfg.rho_ref, h->e, h->stream));
    return MACLAB_OK;
  }
  const int64_t chunk = chunk_nodes(h);
  double* st = (double*)h->staging;
  for (int64_t off = 0; off < N; off += chunk) {
    const int64_t cnt = std::min(chunk, N - off);
    HIP_TRY(h, launch_bgk_decode(h->q, h->fp64, src, h->plane, st, st + chunk, st + 2 * chunk,
                                 h->d == 3 ? st + 3 * chunk : st + chunk, off, cnt, h->cfg.rho_ref, h->e, h->stream));
    HIP_TRY(h, hipMemcpyAsync(rho + off, st, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
    for (int c = 0; c < h->d; ++c)
      HIP_TRY(h, hipMemcpyAsync(u + c * N + off, st + (1 + c) * chunk, sizeof(double) * cnt, hipMemcpyDeviceToHost,
                                h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
  }
  return MACLAB_OK;
}

size_t maclab_bgk_state_bytes(maclab_bgk_t h) { return h ? h->state_bytes : 0; }

int maclab_bgk_save_state(maclab_bgk_t h, void* dst_device) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!dst_device) return fail(h, MACLAB_EINVAL, "dst is NULL");
  HIP_TRY(h, hipMemcpyAsync(dst_device, h->state[h->cur], h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
  return MACLAB_OK;
}

void maclab_bgk_destroy(maclab_bgk_t h) { delete h; }

const char* maclab_bgk_last_error(maclab_bgk_t h) { return h ? h->err.c_str() : g_bgk_err.c_str(); }

}  // extern "C"
