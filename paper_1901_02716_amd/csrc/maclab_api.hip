// C ABI of the MacLAB library (include/maclab.h): validation, workspace
// layout, parameter map, boundary bookkeeping and launch sequencing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace maclab;

namespace {
// Which kernel advances the lattice and how it is tiled. kernel 0: general;
// 1: fast D3Q19, LDS exchange; 2: fast D3Q19, independent wavefronts;
// 3: fast D2Q9.
struct Plan {
  int kernel = 0;
  FastShape s3;
  Fast2DShape s2;
};
}  // namespace

struct maclab_s {
  maclab_config cfg;
  Layout L;
  hipStream_t stream = nullptr;
  char* state[2] = {nullptr, nullptr};
  int cur = 0;
  double* partials = nullptr;
  double* result = nullptr;  // kDiagValues doubles after the partials
  char* staging = nullptr;
  double* gslots = nullptr;  // force-adjoint slots (adjoint_slots(L) x 4), then 4 doubles of fold result
  FaceValues fv;
  double e = 0, dt = 0;
  int64_t steps = 0;
  int cus = 256;               // compute units of the device
  int device = 0;              // HIP device the handle was created on
  Plan plan;                   // kernel and tiling of the step
  bool plan_set = false;       // chosen by maclab_set_tiling / maclab_autotune
  int adj_kernel = -1;         // reverse step: -1 automatic, 0 general, 3 fast D2Q9
  Fast2DShape adj2;            // its tiling when set explicitly
  bool view = false;           // one lattice of a batch: memory owned by the batch
  std::string err;
};

namespace {

thread_local std::string g_err;

// ------------------------------------------------ allocation-free scratch
// The reduction partials and result of maclab_diagnostics_noalloc live in
// this fixed device array instead of the caller's workspace: (kDiagBlocks +
// 1) rows of kDiagValues doubles, 65.6 KB on every device the library runs
// on, held until the process ends. In host code `scratch` names a host-side
// stand-in, not device memory: host code uses only the per-device address
// that hipGetSymbolAddress returns (device_scratch).
constexpr size_t kScratchDoubles = (size_t)(kDiagBlocks + 1) * kDiagValues;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Looks up (once per device, with that device current) the device address
// of `scratch`; returns the HIP status of the lookup.
hipError_t device_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr size_t kStagingMax = size_t(8) << 20;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int fail(maclab_t h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(maclab_t h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h)
    h->err = buf;
  else
    g_err = buf;
  return code;
}

#define HIP_TRY(h, expr)                                                                              \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail((h), MACLAB_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

// Validates the configuration and fills the layout. Pure host arithmetic.
int make_layout(const maclab_config* c, Layout* L, std::string* why) {
  if (!c) {
    *why = "config is NULL";
    return MACLAB_EINVAL;
  }
  if (c->lattice != MACLAB_D2Q9 && c->lattice != MACLAB_D3Q19) {
    *why = "lattice must be MACLAB_D2Q9 (9) or MACLAB_D3Q19 (19)";
    return MACLAB_EUNSUPPORTED;
  }
  if (c->precision < MACLAB_FP64 || c->precision > MACLAB_S16) {
    *why = "precision must be FP64, FP32, HILO or S16";
    return MACLAB_EUNSUPPORTED;
  }
  if (!(c->dx > 0) || !isfinite(c->dx) || !(c->nu > 0) || !isfinite(c->nu)) {
    *why = "dx and nu must be finite and positive";
    return MACLAB_EINVAL;
  }
  if (!(c->rho_ref > 0) || !isfinite(c->rho_ref)) {
    *why = "rho_ref must be finite and positive";
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
  // each count is at most 2^24, so n[0] n[1] fits; test it before the third
  // factor can overflow
  const int64_t nxy = c->n[0] * c->n[1];
  const int64_t N = nxy > (int64_t(1) << 34) ? nxy : nxy * c->n[2];
  if (N > (int64_t(1) << 34)) {
    *why = "lattice too large";
    return MACLAB_EINVAL;
  }
  L->q = c->lattice;
  L->d = d;
  L->precision = c->precision;
  L->bytes = c->precision == MACLAB_FP64 ? 8 : (c->precision == MACLAB_S16 ? 2 : 4);
  L->nx = c->n[0];
  L->ny = c->n[1];
  L->nz = c->n[2];
  L->N = N;
  // D2Q9 rows start on 128-byte boundaries: the fast D2Q9 kernel moves rows
  // segment by segment, and rows that straddle cache lines cost it about a
  // third of its rate. A D3Q19 row is padded to the next row width of the
  // fast D3Q19 kernel (64, 128 or 256 nodes, one wavefront per row) when that
  // adds at most an eighth, so that lattices such as 251^3 run on it.
  if (d == 2) {
    L->px = (int64_t)round_up((size_t)L->nx, (size_t)(128 / L->bytes));
  } else {
    L->px = L->nx;
    for (int64_t w : {64, 128, 256})
      if (w >= L->nx) {
        if (8 * w <= 9 * L->nx) L->px = w;
        break;
      }
  }
  // 256 elements past a multiple of 512: the field planes of a power-of-two
  // lattice then do not start at addresses that differ only in their high
  // bits, which costs about 2% in a 256^3 step
  L->plane = (int64_t)round_up((size_t)(L->px * L->ny * L->nz), 512) + 256;
  L->state_bytes = (size_t)(d + 1) * (size_t)L->plane * (size_t)L->bytes;
  L->partial_bytes = round_up(sizeof(double) * (kDiagBlocks + 1) * kDiagValues, kAlign);
  L->staging_bytes = std::min(kStagingMax, round_up(sizeof(double) * (size_t)N, kAlign));
  L->adjoint_bytes = round_up(sizeof(double) * 4 * (size_t)(adjoint_slots(*L) + 1), kAlign);
  L->workspace_bytes =
      2 * round_up(L->state_bytes, kAlign) + L->partial_bytes + L->staging_bytes + L->adjoint_bytes;
  return MACLAB_OK;
}

StepParams make_params(const maclab_t h) {
  StepParams p{};
  p.nx = h->L.nx;
  p.ny = h->L.ny;
  p.nz = h->L.nz;
  p.px = h->L.px;
  p.plane = h->L.plane;
  for (int ax = 0; ax < 3; ++ax) p.fixed[ax] = h->fv.kind[2 * ax] != MACLAB_BC_PERIODIC;
  p.rho_ref = h->cfg.rho_ref;
  for (int i = 0; i < 3; ++i) p.g[i] = (i < h->L.d) ? h->dt * h->cfg.body_force[i] / h->e : 0.0;
  p.seed = h->cfg.seed;
  p.step = (uint64_t)h->steps;
  p.sr_key = sr_key(p.seed, p.step);
  return p;
}

int check_faces(maclab_t h) {
  for (int ax = 0; ax < h->L.d; ++ax) {
    if ((h->fv.kind[2 * ax] == MACLAB_BC_PERIODIC) != (h->fv.kind[2 * ax + 1] == MACLAB_BC_PERIODIC))
      return fail(h, MACLAB_EINVAL, "faces of axis %d differ (both must be periodic or both bounded)", ax);
    const int64_t n = ax == 0 ? h->L.nx : (ax == 1 ? h->L.ny : h->L.nz);
    if (h->fv.kind[2 * ax] != MACLAB_BC_PERIODIC && n < 3)
      return fail(h, MACLAB_EINVAL, "bounded faces on axis %d need at least 3 nodes", ax);
  }
  return MACLAB_OK;
}

int impose(maclab_t h) {
  HIP_TRY(h, launch_impose_bc(h->L, h->state[0], h->state[1], h->fv, h->cfg.rho_ref, h->e, h->stream));
  HIP_TRY(h, launch_derive_faces(h->L, h->state[0], h->fv, h->stream));
  HIP_TRY(h, launch_derive_faces(h->L, h->state[1], h->fv, h->stream));
  return MACLAB_OK;
}

// Reverse mode covers periodic and fixed faces.
int reverse_supported(maclab_t h) {
  if (h->view) return fail(h, MACLAB_EUNSUPPORTED, "reverse mode is not available on a lattice of a batch");
  if (has_derived_faces(h->fv))
    return fail(h, MACLAB_EUNSUPPORTED, "reverse mode covers periodic and fixed faces only");
  return MACLAB_OK;
}

char* plane_ptr(maclab_t h, int buf, int field) {
  return h->state[buf] + (size_t)field * (size_t)h->L.plane * (size_t)h->L.bytes;
}

bool plan_valid(const Layout& L, const StepParams& p, const Plan& pl) {
  switch (pl.kernel) {
    case 0: return true;
    case 1:
    case 2: return fast_step_supported(L, p) && pl.s3.kind == pl.kernel - 1 && fast_shape_valid(L, p, pl.s3);
    case 3: return fast2d_supported(L, p) && fast2d_shape_valid(L, p, pl.s2);
  }
  return false;
}

Plan plan_default(const Layout& L, const StepParams& p, int cus) {
  Plan pl;
  if (fast_step_supported(L, p)) {
    pl.s3 = fast_default_shape(L, p, cus);
    pl.kernel = 1 + pl.s3.kind;
  } else if (fast2d_supported(L, p)) {
    pl.s2 = fast2d_default_shape(L, p, cus);
    if (fast2d_shape_valid(L, p, pl.s2)) pl.kernel = 3;
  }
  return pl;
}

int plan_candidates(const Layout& L, const StepParams& p, int cus, Plan* out, int max_out) {
  int n = 0;
  out[n++] = plan_default(L, p, cus);
  if (fast_step_supported(L, p)) {
    FastShape c[80];
    const int m = fast_candidates(L, p, cus, c, 80);
    for (int i = 0; i < m && n < max_out; ++i) {
      Plan pl;
      pl.kernel = 1 + c[i].kind;
      pl.s3 = c[i];
      out[n++] = pl;
    }
  } else if (fast2d_supported(L, p)) {
    Fast2DShape c[48];
    const int m = fast2d_candidates(L, p, cus, c, 48);
    for (int i = 0; i < m && n < max_out; ++i) {
      Plan pl;
      pl.kernel = 3;
      pl.s2 = c[i];
      out[n++] = pl;
    }
  }
  return n;
}

hipError_t launch_plan(const Layout& L, const StepParams& p, const Plan& pl, const void* src, void* dst,
                       hipStream_t s) {
  switch (pl.kernel) {
    case 1:
    case 2: return launch_step_fast(L, src, dst, p, pl.s3, s);
    case 3: return launch_step_fast2d(L, src, dst, p, pl.s2, s);
  }
  return launch_step_generic(L, src, dst, p, s);
}

const Plan& current_plan(maclab_t h, const StepParams& p) {
  if (!(h->plan_set && plan_valid(h->L, p, h->plan))) {
    h->plan = plan_default(h->L, p, h->cus);
    h->plan_set = false;
  }
  return h->plan;
}

}  // namespace

extern "C" {

size_t maclab_workspace_bytes(const maclab_config* cfg) {
  Layout L;
  std::string why;
  if (make_layout(cfg, &L, &why) != MACLAB_OK) return 0;
  return L.workspace_bytes;
}

int maclab_init(const maclab_config* cfg, maclab_t* out) {
  if (!out) return fail(nullptr, MACLAB_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  std::string why;
  int rc = make_layout(cfg, &L, &why);
  if (rc != MACLAB_OK) return fail(nullptr, rc, "maclab_init: %s", why.c_str());
  if (!cfg->workspace) return fail(nullptr, MACLAB_EWORKSPACE, "maclab_init: workspace is NULL");
  if ((uintptr_t)cfg->workspace % kAlign)
    return fail(nullptr, MACLAB_EWORKSPACE, "maclab_init: workspace must be %zu-byte aligned", kAlign);
  if (cfg->workspace_bytes < L.workspace_bytes)
    return fail(nullptr, MACLAB_EWORKSPACE, "maclab_init: workspace has %zu bytes, needs %zu",
                cfg->workspace_bytes, L.workspace_bytes);
  maclab_t h = new (std::nothrow) maclab_s();
  if (!h) return fail(nullptr, MACLAB_EINVAL, "maclab_init: out of host memory");
  h->cfg = *cfg;
  h->L = L;
  h->stream = (hipStream_t)cfg->stream;
  char* ws = (char*)cfg->workspace;
  const size_t sb = round_up(L.state_bytes, kAlign);
  h->state[0] = ws;
  h->state[1] = ws + sb;
  h->partials = (double*)(ws + 2 * sb);
  h->result = h->partials + (size_t)kDiagBlocks * kDiagValues;
  h->staging = ws + 2 * sb + L.partial_bytes;
  h->gslots = (double*)(ws + 2 * sb + L.partial_bytes + L.staging_bytes);
  for (int f = 0; f < 6; ++f) {
    h->fv.kind[f] = MACLAB_BC_PERIODIC;
    h->fv.rho[f] = cfg->rho_ref;
    for (int c = 0; c < 3; ++c) h->fv.u[f][c] = 0.0;
  }
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      h->device = dev;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        h->cus = cus;
      // the address of the allocation-free entry points' scratch array on
      // this device (once per device; the entry point reports a failure)
      double* unused = nullptr;
      (void)device_scratch(dev, &unused);
    }
  }
  h->e = 6.0 * cfg->nu / cfg->dx;  // Eq. (6)
  h->dt = cfg->dx / h->e;          // text after Eq. (6)
  // state at rest: zero deviation and zero velocity in every codec
  hipError_t e1 = hipMemsetAsync(ws, 0, 2 * sb, h->stream);
  if (e1 != hipSuccess) {
    int code = fail(nullptr, MACLAB_EHIP, "maclab_init: hipMemsetAsync: %s", hipGetErrorString(e1));
    delete h;
    return code;
  }
  *out = h;
  return MACLAB_OK;
}

int maclab_set_bc(maclab_t h, int face, int kind, double rho_b, const double* u_b) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (face < 0 || face > 5) return fail(h, MACLAB_EINVAL, "face %d out of range", face);
  if (face / 2 >= h->L.d) return fail(h, MACLAB_EINVAL, "face %d does not exist in 2D", face);
  if (kind < MACLAB_BC_PERIODIC || kind > MACLAB_BC_PRESSURE)
    return fail(h, MACLAB_EINVAL, "unknown boundary kind %d", kind);
  if ((kind == MACLAB_BC_RHO_NEUMANN || kind == MACLAB_BC_PRESSURE) && h->view)
    return fail(h, MACLAB_EUNSUPPORTED, "a lattice of a batch has periodic and fixed faces only");
  if (kind != MACLAB_BC_PERIODIC) {
    if (!u_b) return fail(h, MACLAB_EINVAL, "u_b is NULL");
    if (!(rho_b > 0) || !isfinite(rho_b)) return fail(h, MACLAB_EINVAL, "rho_b must be finite and positive");
    for (int c = 0; c < h->L.d; ++c)
      if (!isfinite(u_b[c])) return fail(h, MACLAB_EINVAL, "u_b must be finite");
  }
  h->fv.kind[face] = kind;
  if (kind != MACLAB_BC_PERIODIC) {
    h->fv.rho[face] = rho_b;
    for (int c = 0; c < 3; ++c) h->fv.u[face][c] = c < h->L.d ? u_b[c] : 0.0;
  }
  return impose(h);
}

int maclab_set_fields(maclab_t h, const double* rho, const double* u, int on_device) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!rho || !u) return fail(h, MACLAB_EINVAL, "rho and u must not be NULL");
  const Layout& L = h->L;
  const double offsets[4] = {h->cfg.rho_ref, 0, 0, 0};
  const double muls[4] = {1.0, 1.0 / h->e, 1.0 / h->e, 1.0 / h->e};
  for (int f = 0; f <= L.d; ++f) {
    const double* src = f == 0 ? rho : u + (size_t)(f - 1) * (size_t)L.N;
    if (on_device) {
      HIP_TRY(h, launch_encode(L, plane_ptr(h, h->cur, f), src, 0, L.N, offsets[f], muls[f], f, h->stream));
    } else {
      const int64_t chunk = (int64_t)(L.staging_bytes / sizeof(double));
      for (int64_t off = 0; off < L.N; off += chunk) {
        const int64_t cnt = std::min(chunk, L.N - off);
        HIP_TRY(h, hipMemcpyAsync(h->staging, src + off, sizeof(double) * cnt, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, launch_encode(L, plane_ptr(h, h->cur, f), (const double*)h->staging, off,
                                 cnt, offsets[f], muls[f], f, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));  // staging is reused
      }
    }
  }
  // the other buffer gets the same state, so fixed nodes agree in both
  HIP_TRY(h, hipMemcpyAsync(h->state[h->cur ^ 1], h->state[h->cur], L.state_bytes, hipMemcpyDeviceToDevice,
                            h->stream));
  return impose(h);
}

int maclab_step(maclab_t h, int64_t n) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, MACLAB_EINVAL, "negative step count");
  int rc = check_faces(h);
  if (rc) return rc;
  StepParams p = make_params(h);
  const Plan pl = current_plan(h, p);
  for (int64_t s = 0; s < n; ++s) {
    p.step = (uint64_t)h->steps;
    p.sr_key = sr_key(p.seed, p.step);
    const void* src = h->state[h->cur];
    void* dst = h->state[h->cur ^ 1];
    HIP_TRY(h, launch_plan(h->L, p, pl, src, dst, h->stream));
    HIP_TRY(h, launch_derive_faces(h->L, dst, h->fv, h->stream));
    h->cur ^= 1;
    ++h->steps;
  }
  return MACLAB_OK;
}

int maclab_diagnostics(maclab_t h, double out[7]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out) return fail(h, MACLAB_EINVAL, "out is NULL");
  HIP_TRY(h, launch_diagnostics(h->L, h->state[h->cur], h->cfg.rho_ref, h->e, h->partials, h->result,
                                h->stream));
  double r[kDiagValues];
  HIP_TRY(h, hipMemcpyAsync(r, h->result, sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < 7; ++i) out[i] = r[i];
  return MACLAB_OK;
}

int maclab_diagnostics_noalloc(maclab_t h, double* out_dev) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out_dev) return fail(h, MACLAB_EINVAL, "out_dev is NULL");
  // the reduction writes one row of partials per workgroup (at most
  // kDiagBlocks), then a result row; all of it must fit the scratch array
  const int64_t want = (h->L.N + 255) / 256;
  const int64_t rows = std::min<int64_t>(std::max<int64_t>(want, 1), kDiagBlocks) + 1;
  if ((size_t)rows * kDiagValues > kScratchDoubles)
    return fail(h, MACLAB_EWORKSPACE, "diagnostics need %lld scratch doubles, the array holds %zu",
                (long long)rows * kDiagValues, kScratchDoubles);
  double* base = nullptr;
  HIP_TRY(h, device_scratch(h->device, &base));
  double* partials = base;
  double* result = base + (size_t)kDiagBlocks * kDiagValues;
  HIP_TRY(h, launch_diagnostics(h->L, h->state[h->cur], h->cfg.rho_ref, h->e, partials, result, h->stream));
  HIP_TRY(h, hipMemcpyAsync(out_dev, result, 7 * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return MACLAB_OK;
}

int maclab_residual(maclab_t h, double out[3]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out) return fail(h, MACLAB_EINVAL, "out is NULL");
  HIP_TRY(h, launch_residual(h->L, h->state[h->cur ^ 1], h->state[h->cur], h->partials, h->result, h->stream));
  double r[3];
  HIP_TRY(h, hipMemcpyAsync(r, h->result, sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  out[0] = r[0] * h->e;  // u = e u~
  out[1] = r[1];
  out[2] = r[2];
  return MACLAB_OK;
}

int maclab_step_until(maclab_t h, double tol, int64_t max_steps, int64_t check_every, int64_t* done,
                      double resid[3]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!(tol >= 0) || max_steps < 0 || check_every < 1)
    return fail(h, MACLAB_EINVAL, "need tol >= 0, max_steps >= 0 and check_every >= 1");
  int64_t k = 0;
  double r[3] = {0, 0, 0};
  if (done) *done = 0;
  while (k < max_steps) {
    const int64_t m = std::min(check_every, max_steps - k);
    int rc = maclab_step(h, m);
    if (rc) return rc;
    k += m;
    if (done) *done = k;
    rc = maclab_residual(h, r);
    if (rc) return rc;
    if (resid)
      for (int i = 0; i < 3; ++i) resid[i] = r[i];
    if (r[2] > 0) return fail(h, MACLAB_ENONFINITE, "%.0f non-finite nodes after %lld steps", r[2], (long long)h->steps);
    if (r[0] < tol) break;
  }
  return MACLAB_OK;
}

int maclab_step_checked(maclab_t h, int64_t n, int64_t check_every, int64_t* done) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (check_every < 1) return fail(h, MACLAB_EINVAL, "check_every must be >= 1");
  int64_t k = 0;
  if (done) *done = 0;
  while (k < n) {
    const int64_t m = std::min(check_every, n - k);
    int rc = maclab_step(h, m);
    if (rc) return rc;
    k += m;
    if (done) *done = k;
    double d[7];
    rc = maclab_diagnostics(h, d);
    if (rc) return rc;
    if (d[6] > 0 || !(d[5] < 1.0))
      return fail(h, MACLAB_ENONFINITE, "step %lld: %.0f non-finite nodes, max |u|/e = %g", (long long)h->steps,
                  d[6], d[5]);
  }
  return MACLAB_OK;
}

int maclab_get_fields(maclab_t h, double* rho, double* u, int on_device) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!rho || !u) return fail(h, MACLAB_EINVAL, "rho and u must not be NULL");
  const Layout& L = h->L;
  const double offsets[4] = {h->cfg.rho_ref, 0, 0, 0};
  const double muls[4] = {1.0, h->e, h->e, h->e};
  for (int f = 0; f <= L.d; ++f) {
    double* dst = f == 0 ? rho : u + (size_t)(f - 1) * (size_t)L.N;
    if (on_device) {
      HIP_TRY(h, launch_decode(L, dst, plane_ptr(h, h->cur, f), 0, L.N, offsets[f], muls[f], f, h->stream));
    } else {
      const int64_t chunk = (int64_t)(L.staging_bytes / sizeof(double));
      for (int64_t off = 0; off < L.N; off += chunk) {
        const int64_t cnt = std::min(chunk, L.N - off);
        HIP_TRY(h, launch_decode(L, (double*)h->staging, plane_ptr(h, h->cur, f), off, cnt,
                                 offsets[f], muls[f], f, h->stream));
        HIP_TRY(h, hipMemcpyAsync(dst + off, h->staging, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
      }
    }
  }
  return MACLAB_OK;
}

int maclab_params(maclab_t h, double out[6]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out) return fail(h, MACLAB_EINVAL, "out is NULL");
  double umax = 0;
  for (int f = 0; f < 2 * h->L.d; ++f) {
    // faces that hold their velocity (a pressure face takes it from the flow)
    if (h->fv.kind[f] != MACLAB_BC_FIXED && h->fv.kind[f] != MACLAB_BC_RHO_NEUMANN) continue;
    double s = 0;
    for (int c = 0; c < h->L.d; ++c) s += h->fv.u[f][c] * h->fv.u[f][c];
    umax = std::max(umax, sqrt(s));
  }
  out[0] = h->e;
  out[1] = h->dt;
  out[2] = umax * h->cfg.dx / h->cfg.nu;
  out[3] = out[2] / 6.0;
  out[4] = (double)h->steps;
  out[5] = (double)h->steps * h->dt;
  return MACLAB_OK;
}

size_t maclab_state_bytes(maclab_t h) { return h ? h->L.state_bytes : 0; }

int maclab_save_state(maclab_t h, void* dst) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!dst) return fail(h, MACLAB_EINVAL, "dst is NULL");
  HIP_TRY(h, hipMemcpyAsync(dst, h->state[h->cur], h->L.state_bytes, hipMemcpyDeviceToDevice, h->stream));
  return MACLAB_OK;
}

int maclab_load_state(maclab_t h, const void* src) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!src) return fail(h, MACLAB_EINVAL, "src is NULL");
  HIP_TRY(h, hipMemcpyAsync(h->state[0], src, h->L.state_bytes, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->state[1], src, h->L.state_bytes, hipMemcpyDeviceToDevice, h->stream));
  return MACLAB_OK;
}

int maclab_get_tiling(maclab_t h, int out[5]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out) return fail(h, MACLAB_EINVAL, "out is NULL");
  StepParams p = make_params(h);
  const Plan& pl = current_plan(h, p);
  out[0] = pl.kernel;
  out[1] = out[2] = out[3] = out[4] = 0;
  if (pl.kernel == 1 || pl.kernel == 2) {
    out[1] = pl.s3.W;
    out[2] = pl.s3.nyb;
    out[3] = pl.s3.nzb;
    out[4] = pl.s3.pf;
  } else if (pl.kernel == 3) {
    out[1] = pl.s2.kx;
    out[2] = (int)((h->L.nx + 64 * pl.s2.kx - 1) / (64 * pl.s2.kx));
    out[3] = pl.s2.nband;
  }
  return MACLAB_OK;
}

int maclab_set_tiling(maclab_t h, int kernel, int W, int nyb, int nzb, int pf) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  StepParams p = make_params(h);
  Plan pl;
  pl.kernel = kernel;
  if (kernel == 1 || kernel == 2) {
    if (!fast_step_supported(h->L, p))
      return fail(h, MACLAB_EUNSUPPORTED, "the fast D3Q19 kernels do not handle this lattice");
    pl.s3 = FastShape{W, nyb, nzb, pf, kernel - 1};
  } else if (kernel == 3) {
    if (!fast2d_supported(h->L, p))
      return fail(h, MACLAB_EUNSUPPORTED, "the fast D2Q9 kernel does not handle this lattice");
    pl.s2.kx = W;
    pl.s2.nband = nzb;
  } else if (kernel != 0) {
    return fail(h, MACLAB_EINVAL, "kernel must be 0 (general), 1, 2 (D3Q19) or 3 (D2Q9)");
  }
  if (!plan_valid(h->L, p, pl))
    return fail(h, MACLAB_EINVAL, "invalid tiling kernel=%d W=%d nyb=%d nzb=%d pf=%d", kernel, W, nyb, nzb, pf);
  h->plan = pl;
  h->plan_set = true;
  return MACLAB_OK;
}

int maclab_autotune(maclab_t h, int reps, double* best_ms) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (reps < 1) return fail(h, MACLAB_EINVAL, "reps must be >= 1");
  int rc = check_faces(h);
  if (rc) return rc;
  StepParams p = make_params(h);
  const void* src = h->state[h->cur];
  void* dst = h->state[h->cur ^ 1];  // scratch output: the state is not advanced
  Plan cand[96];
  const int nc = plan_candidates(h->L, p, h->cus, cand, 96);
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0));
  hipError_t ee = hipEventCreate(&e1);
  if (ee != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(h, MACLAB_EHIP, "hipEventCreate: %s", hipGetErrorString(ee));
  }
  double best = 1e300;
  int best_i = 0;
  hipError_t err = hipSuccess;
  for (int i = 0; i < nc && err == hipSuccess; ++i) {
    if ((err = launch_plan(h->L, p, cand[i], src, dst, h->stream)) != hipSuccess) break;  // warm-up
    double total = 0;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
      // A time step reads a source that the step before has just written
      // with write-through stores, part of which the memory-side cache may
      // still hold, and nothing else. Launches repeated from one source would
      // find other data there (the source they read before). So before each
      // timed launch the source is copied to the spare buffer and back
      // (untimed; the same bytes, stored the way a step stores them).
      if ((err = launch_stream_copy(src, dst, h->L.state_bytes, h->stream)) != hipSuccess) break;
      if ((err = launch_stream_copy(dst, h->state[h->cur], h->L.state_bytes, h->stream)) != hipSuccess) break;
      if ((err = hipEventRecord(e0, h->stream)) != hipSuccess) break;
      if ((err = launch_plan(h->L, p, cand[i], src, dst, h->stream)) != hipSuccess) break;
      if ((err = hipEventRecord(e1, h->stream)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      total += ms;
    }
    if (err != hipSuccess) break;
    const double per = total / reps;
    if (per < best) {
      best = per;
      best_i = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(h, MACLAB_EHIP, "maclab_autotune: %s", hipGetErrorString(err));
  h->plan = cand[best_i];
  h->plan_set = true;
  if (best_ms) *best_ms = best;
  return MACLAB_OK;
}

int maclab_set_body_force(maclab_t h, const double* G) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!G) return fail(h, MACLAB_EINVAL, "G is NULL");
  for (int c = 0; c < 3; ++c)
    if (!isfinite(G[c])) return fail(h, MACLAB_EINVAL, "body force must be finite");
  for (int c = 0; c < 3; ++c) h->cfg.body_force[c] = G[c];
  return MACLAB_OK;
}

int maclab_step_external(maclab_t h, const void* src, void* dst, int64_t step_index) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!src || !dst || src == dst) return fail(h, MACLAB_EINVAL, "src and dst must be distinct device buffers");
  int rc = check_faces(h);
  if (rc) return rc;
  StepParams p = make_params(h);
  p.step = (uint64_t)step_index;
  p.sr_key = sr_key(p.seed, p.step);
  const Plan pl = current_plan(h, p);
  HIP_TRY(h, launch_plan(h->L, p, pl, src, dst, h->stream));
  bool any_bounded = false;
  for (int f = 0; f < 6; ++f) any_bounded |= h->fv.kind[f] != MACLAB_BC_PERIODIC;
  if (any_bounded) HIP_TRY(h, launch_impose_bc(h->L, dst, dst, h->fv, h->cfg.rho_ref, h->e, h->stream));
  HIP_TRY(h, launch_derive_faces(h->L, dst, h->fv, h->stream));
  return MACLAB_OK;
}

int maclab_copy(maclab_t h, const void* src, void* dst, size_t bytes) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!src || !dst) return fail(h, MACLAB_EINVAL, "src and dst must be device pointers");
  if (((uintptr_t)src | (uintptr_t)dst | bytes) & 15)
    return fail(h, MACLAB_EINVAL, "src, dst and bytes must be multiples of 16");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(h, MACLAB_EINVAL, "src and dst overlap");
  HIP_TRY(h, launch_stream_copy(src, dst, bytes, h->stream));
  return MACLAB_OK;
}

size_t maclab_adjoint_bytes(maclab_t h) {
  if (!h) return 0;
  const size_t t = h->L.precision == MACLAB_FP64 ? sizeof(double) : sizeof(float);
  return (size_t)(h->L.d + 1) * (size_t)h->L.plane * t;
}

int maclab_adjoint_seed(maclab_t h, const void* state_T, const double* dLdu, void* adj) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (int rc_ = reverse_supported(h)) return rc_;
  if (!state_T || !dLdu || !adj) return fail(h, MACLAB_EINVAL, "state_T, dLdu and adj must be device pointers");
  int rc = check_faces(h);
  if (rc) return rc;
  const StepParams p = make_params(h);
  HIP_TRY(h, launch_adjoint_seed(h->L, state_T, dLdu, adj, p, h->e, h->stream));
  return MACLAB_OK;
}

int maclab_adjoint_reset(maclab_t h) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (int rc_ = reverse_supported(h)) return rc_;
  HIP_TRY(h, launch_zero_doubles(h->gslots, (int64_t)(h->L.adjoint_bytes / sizeof(double)), h->stream));
  return MACLAB_OK;
}

namespace {
// The reverse step's kernel: the fast D2Q9 one where it applies.
bool adjoint_fast2d(maclab_t h, const StepParams& p, Fast2DShape* sh) {
  if (h->adj_kernel == 0 || !adjoint2d_supported(h->L, p)) return false;
  *sh = h->adj_kernel == 3 ? h->adj2 : adjoint2d_default_shape(h->L, p, h->cus);
  return adjoint2d_shape_valid(h->L, p, *sh);
}

int adjoint_one(maclab_t h, const StepParams& p, const void* state_n, const void* adj_np1, void* adj_n) {
  Fast2DShape sh;
  if (adjoint_fast2d(h, p, &sh))
    HIP_TRY(h, launch_adjoint_fast2d(h->L, state_n, adj_np1, adj_n, p, sh, h->gslots, h->stream));
  else
    HIP_TRY(h, launch_adjoint_step(h->L, state_n, adj_np1, adj_n, p, h->gslots, h->stream));
  return MACLAB_OK;
}
}  // namespace

int maclab_set_adjoint_tiling(maclab_t h, int kernel, int kx, int nband) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (kernel == -1 || kernel == 0) {
    h->adj_kernel = kernel;
    return MACLAB_OK;
  }
  if (kernel != 3) return fail(h, MACLAB_EINVAL, "adjoint kernel must be -1, 0 or 3");
  const StepParams p = make_params(h);
  if (!adjoint2d_supported(h->L, p)) return fail(h, MACLAB_EUNSUPPORTED, "the fast D2Q9 adjoint does not handle this lattice");
  Fast2DShape sh;
  sh.kx = kx;
  sh.nband = nband;
  if (!adjoint2d_shape_valid(h->L, p, sh))
    return fail(h, MACLAB_EINVAL, "invalid adjoint tiling kx=%d nband=%d (kx in {1,2}, 1 <= nband <= ceil(ny/4))", kx,
                nband);
  h->adj_kernel = 3;
  h->adj2 = sh;
  return MACLAB_OK;
}

int maclab_get_adjoint_tiling(maclab_t h, int out[3]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (!out) return fail(h, MACLAB_EINVAL, "out is NULL");
  const StepParams p = make_params(h);
  Fast2DShape sh;
  if (adjoint_fast2d(h, p, &sh)) {
    out[0] = 3;
    out[1] = sh.kx;
    out[2] = sh.nband;
  } else {
    out[0] = 0;
    out[1] = out[2] = 0;
  }
  return MACLAB_OK;
}

int maclab_adjoint_step(maclab_t h, const void* state_n, const void* adj_np1, void* adj_n) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (int rc_ = reverse_supported(h)) return rc_;
  if (!state_n || !adj_np1 || !adj_n || adj_np1 == adj_n)
    return fail(h, MACLAB_EINVAL, "state and adjoint buffers must be device pointers, adj_np1 != adj_n");
  int rc = check_faces(h);
  if (rc) return rc;
  const StepParams p = make_params(h);
  return adjoint_one(h, p, state_n, adj_np1, adj_n);
}

int maclab_adjoint_segment(maclab_t h, const void* ckpt, void* states, int64_t nsteps, int64_t step_index,
                           void* adj_a, void* adj_b, int* which) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (int rc_ = reverse_supported(h)) return rc_;
  if (!ckpt || !adj_a || !adj_b || !which || adj_a == adj_b || (*which != 0 && *which != 1))
    return fail(h, MACLAB_EINVAL, "ckpt, adj_a, adj_b (distinct) and which (0 or 1) are required");
  if (nsteps < 1 || step_index < 0) return fail(h, MACLAB_EINVAL, "nsteps must be >= 1 and step_index >= 0");
  if (nsteps > 1 && !states) return fail(h, MACLAB_EINVAL, "states is NULL");
  int rc = check_faces(h);
  if (rc) return rc;
  const size_t sb = h->L.state_bytes;
  auto slot = [&](int64_t n) -> const void* {  // state at step step_index + n
    return n == 0 ? ckpt : (const void*)((const char*)states + (size_t)(n - 1) * sb);
  };
  // recompute the states after the checkpoint
  for (int64_t n = 1; n < nsteps; ++n) {
    rc = maclab_step_external(h, slot(n - 1), (void*)slot(n), step_index + n - 1);
    if (rc) return rc;
  }
  void* adj[2] = {adj_a, adj_b};
  int cur = *which;
  const StepParams p = make_params(h);
  for (int64_t n = nsteps - 1; n >= 0; --n) {
    rc = adjoint_one(h, p, slot(n), adj[cur], adj[cur ^ 1]);
    if (rc) return rc;
    cur ^= 1;
  }
  *which = cur;
  return MACLAB_OK;
}

int maclab_adjoint_result(maclab_t h, const void* state0, const void* adj0, double* dLdu0, double* dLdrho0,
                          double dLdG[3]) {
  if (!h) return fail(nullptr, MACLAB_EINVAL, "handle is NULL");
  if (int rc_ = reverse_supported(h)) return rc_;
  if (!adj0) return fail(h, MACLAB_EINVAL, "adj0 is NULL");
  if (dLdu0) {
    if (!state0) return fail(h, MACLAB_EINVAL, "state0 is NULL");
    HIP_TRY(h, launch_adjoint_result(h->L, state0, adj0, dLdu0, dLdrho0, h->cfg.rho_ref, h->e, h->stream));
  }
  if (dLdG) {
    const int64_t ns = adjoint_slots(h->L);
    double* fold = h->gslots + 4 * ns;
    HIP_TRY(h, launch_adjoint_fold(h->gslots, ns, fold, h->stream));
    double g[4];
    HIP_TRY(h, hipMemcpyAsync(g, fold, sizeof(double) * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    // g = dt G / e per step, so dL/dG = (dt / e) sum_steps sum_x Mbar
    for (int c = 0; c < 3; ++c) dLdG[c] = c < h->L.d ? g[c] * h->dt / h->e : 0.0;
  }
  return MACLAB_OK;
}

void maclab_destroy(maclab_t h) {
  if (h && !h->view) delete h;  // a batch's lattices go with the batch
}

const char* maclab_last_error(maclab_t h) { return h ? h->err.c_str() : g_err.c_str(); }

}  // extern "C"

// ===================================================================== batch
// Many D2Q9 lattices in one state allocation, advanced by one launch per step
// over a table of work items (lattice, x-segment, band of rows); a run of
// steps is captured once in a HIP graph and replayed.

struct maclab_batch_s {
  int count = 0;
  int precision = 0;
  double rho_ref = 1.0;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;  // the caller's
  hipStream_t priv = nullptr;    // graph capture and replay (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<maclab_s*> lat;
  std::vector<int64_t> base;     // element offset of each lattice in a state buffer
  char* state[2] = {nullptr, nullptr};
  size_t state_bytes = 0;        // of one state buffer (all lattices)
  double* partials = nullptr;    // shared reduction partials (device)
  Lattice2D* table = nullptr;    // device
  int4* items = nullptr;         // device
  int64_t max_items = 0;
  int kx = 1, rows = 16;
  int nitems = 0;
  bool uploaded = false;
  int up_kx = 0, up_rows = 0;
  std::vector<Lattice2D> table_host;
  std::vector<int4> items_host;
  int graph_steps = 32;          // steps per captured graph (even; 0: no graph)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int cus = 256;
  int device = 0;
  std::string err;
};

namespace {

int bfail(maclab_batch_t b, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int bfail(maclab_batch_t b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b)
    b->err = buf;
  else
    g_err = buf;
  return code;
}

#define BHIP_TRY(b, expr)                                                                             \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return bfail((b), MACLAB_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

constexpr int kBatchRowsMin = 4;

struct BatchLayout {
  std::vector<Layout> L;
  std::vector<size_t> off;  // byte offset of each lattice in a state buffer
  size_t states = 0, partial = 0, staging = 0, adjoint = 0, table = 0, items = 0, total = 0;
  int64_t max_items = 0;
};

int batch_layout(const maclab_config* cfgs, int count, BatchLayout* B, std::string* why) {
  if (!cfgs || count < 1) {
    *why = "need at least one lattice";
    return MACLAB_EINVAL;
  }
  B->L.resize(count);
  B->off.resize(count);
  for (int i = 0; i < count; ++i) {
    const maclab_config& c = cfgs[i];
    std::string w;
    const int rc = make_layout(&c, &B->L[i], &w);
    if (rc != MACLAB_OK) {
      *why = "lattice " + std::to_string(i) + ": " + w;
      return rc;
    }
    if (c.lattice != MACLAB_D2Q9) {
      *why = "lattice " + std::to_string(i) + ": a batch holds D2Q9 lattices only";
      return MACLAB_EUNSUPPORTED;
    }
    if (c.precision != cfgs[0].precision || c.rho_ref != cfgs[0].rho_ref || c.seed != cfgs[0].seed ||
        c.stream != cfgs[0].stream) {
      *why = "lattice " + std::to_string(i) + ": precision, rho_ref, seed and stream must match lattice 0";
      return MACLAB_EINVAL;
    }
    if (c.n[0] >= (int64_t(1) << 20) || c.n[1] >= (int64_t(1) << 20)) {
      *why = "lattice " + std::to_string(i) + ": extents must be below 2^20";
      return MACLAB_EINVAL;
    }
    B->off[i] = B->states;
    B->states += round_up(B->L[i].state_bytes, kAlign);
    B->partial = std::max(B->partial, B->L[i].partial_bytes);
    B->staging = std::max(B->staging, B->L[i].staging_bytes);
    B->adjoint = std::max(B->adjoint, B->L[i].adjoint_bytes);
    B->max_items += ((B->L[i].nx + 63) / 64) * ((B->L[i].ny + kBatchRowsMin - 1) / kBatchRowsMin);
  }
  if (B->max_items > (int64_t(1) << 30)) {
    *why = "too many work items";
    return MACLAB_EINVAL;
  }
  B->table = round_up(sizeof(Lattice2D) * (size_t)count, kAlign);
  B->items = round_up(sizeof(int4) * (size_t)B->max_items, kAlign);
  B->total = 2 * B->states + B->partial + B->staging + B->adjoint + B->table + B->items;
  return MACLAB_OK;
}

// Lattice table and work items of a tiling, from the lattices' current
// faces and body forces.
int batch_plan(maclab_batch_t b, int kx, int rows, std::vector<Lattice2D>* table, std::vector<int4>* items) {
  if (kx != 1 && kx != 2) return bfail(b, MACLAB_EINVAL, "kx must be 1 or 2");
  if (rows < kBatchRowsMin) return bfail(b, MACLAB_EINVAL, "rows per work item must be >= %d", kBatchRowsMin);
  table->assign(b->count, Lattice2D{});
  items->clear();
  // Lattices largest first, so the tail of a launch is made of small ones;
  // the items of one lattice in row order (bands, and the x-segments of a
  // band), so that neighbouring bands run at about the same time on one XCD
  // and the rows each reads beside its own come from that XCD's L2. (Sorting
  // the items themselves by size scattered the bands of a lattice, and a
  // batch step then read 1.39 times the bytes of its fields.)
  std::vector<int> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return b->lat[a]->L.nx * b->lat[a]->L.ny > b->lat[c]->L.nx * b->lat[c]->L.ny;
  });
  for (int i : order) {
    maclab_s* h = b->lat[i];
    const int rc = check_faces(h);
    if (rc) return bfail(b, rc, "lattice %d: %s", i, h->err.c_str());
    const StepParams p = make_params(h);
    if (!fast2d_supported(h->L, p))
      return bfail(b, MACLAB_EUNSUPPORTED,
                   "lattice %d: not a fast D2Q9 lattice (a field plane must be under 2 GiB)", i);
    if (!p.fixed[0] && h->L.nx % kx != 0)
      return bfail(b, MACLAB_EINVAL, "lattice %d: periodic x extent %lld is not a multiple of kx = %d", i,
                   (long long)h->L.nx, kx);
    Lattice2D& t = (*table)[i];
    t.nx = (int)h->L.nx;
    t.ny = (int)h->L.ny;
    t.pitch = (int)h->L.px;
    t.xper = !p.fixed[0];
    t.yper = !p.fixed[1];
    t.gx = p.g[0];
    t.gy = p.g[1];
    t.base = b->base[i];
    t.plane = h->L.plane;
    const int nseg = (t.nx + 64 * kx - 1) / (64 * kx);
    const int ylo = p.fixed[1] ? 1 : 0, nyo = p.fixed[1] ? t.ny - 2 : t.ny;
    const int nb = (nyo + rows - 1) / rows;
    for (int band = 0; band < nb; ++band) {
      const int y0 = ylo + (int)((int64_t)band * nyo / nb), y1 = ylo + (int)((int64_t)(band + 1) * nyo / nb);
      for (int sg = 0; sg < nseg; ++sg) items->push_back(make_int4(i, sg * 64 * kx, y0, y1));
    }
  }
  if ((int64_t)items->size() > b->max_items) return bfail(b, MACLAB_EINVAL, "too many work items for the workspace");
  return MACLAB_OK;
}

void drop_graph(maclab_batch_t b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

bool same_lattice(const Lattice2D& a, const Lattice2D& c) {
  return a.nx == c.nx && a.ny == c.ny && a.pitch == c.pitch && a.xper == c.xper && a.yper == c.yper &&
         a.gx == c.gx && a.gy == c.gy && a.base == c.base && a.plane == c.plane;
}

// Makes the device tables match the current tiling, faces and forces.
int batch_sync(maclab_batch_t b) {
  std::vector<Lattice2D> table;
  std::vector<int4> items;
  int rc = batch_plan(b, b->kx, b->rows, &table, &items);
  if (rc) return rc;
  bool same = b->uploaded && b->up_kx == b->kx && b->up_rows == b->rows && table.size() == b->table_host.size();
  for (size_t i = 0; same && i < table.size(); ++i) same = same_lattice(table[i], b->table_host[i]);
  if (same) return MACLAB_OK;
  drop_graph(b);
  b->table_host.swap(table);
  b->items_host.swap(items);
  BHIP_TRY(b, hipMemcpyAsync(b->table, b->table_host.data(), sizeof(Lattice2D) * b->table_host.size(),
                             hipMemcpyHostToDevice, b->stream));
  if (!b->items_host.empty())
    BHIP_TRY(b, hipMemcpyAsync(b->items, b->items_host.data(), sizeof(int4) * b->items_host.size(),
                               hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));  // the host copies may change before the next sync
  b->nitems = (int)b->items_host.size();
  b->uploaded = true;
  b->up_kx = b->kx;
  b->up_rows = b->rows;
  return MACLAB_OK;
}

int batch_consistent(maclab_batch_t b) {
  for (int i = 1; i < b->count; ++i)
    if (b->lat[i]->cur != b->lat[0]->cur || b->lat[i]->steps != b->lat[0]->steps)
      return bfail(b, MACLAB_EINVAL, "lattice %d was stepped on its own; the batch steps all lattices together", i);
  return MACLAB_OK;
}

void batch_advance(maclab_batch_t b, int64_t n) {
  for (maclab_s* h : b->lat) {
    h->cur ^= (int)(n & 1);
    h->steps += n;
  }
}

int batch_launch(maclab_batch_t b, hipStream_t s, int cur, int64_t step) {
  const uint32_t key = sr_key(b->seed, (uint64_t)step);
  BHIP_TRY(b, launch_step_fast2d_items(b->precision, b->kx, b->state[cur], b->state[cur ^ 1], b->table, b->items,
                                       b->nitems, b->rho_ref, key, b->state_bytes >= kStreamStoreBytes, s));
  return MACLAB_OK;
}

}  // namespace

extern "C" {

size_t maclab_batch_workspace_bytes(const maclab_config* cfgs, int count) {
  BatchLayout B;
  std::string why;
  if (batch_layout(cfgs, count, &B, &why) != MACLAB_OK) return 0;
  return B.total;
}

int maclab_batch_init(const maclab_config* cfgs, int count, void* workspace, size_t workspace_bytes,
                      maclab_batch_t* out) {
  if (!out) return bfail(nullptr, MACLAB_EINVAL, "out is NULL");
  *out = nullptr;
  BatchLayout B;
  std::string why;
  int rc = batch_layout(cfgs, count, &B, &why);
  if (rc) return bfail(nullptr, rc, "maclab_batch_init: %s", why.c_str());
  if (!workspace || (uintptr_t)workspace % kAlign)
    return bfail(nullptr, MACLAB_EWORKSPACE, "maclab_batch_init: workspace must be %zu-byte aligned device memory",
                 kAlign);
  if (workspace_bytes < B.total)
    return bfail(nullptr, MACLAB_EWORKSPACE, "maclab_batch_init: workspace has %zu bytes, needs %zu",
                 workspace_bytes, B.total);
  maclab_batch_t b = new (std::nothrow) maclab_batch_s();
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "maclab_batch_init: out of host memory");
  b->count = count;
  b->precision = cfgs[0].precision;
  b->rho_ref = cfgs[0].rho_ref;
  b->seed = cfgs[0].seed;
  b->stream = (hipStream_t)cfgs[0].stream;
  b->max_items = B.max_items;
  char* ws = (char*)workspace;
  b->state[0] = ws;
  b->state[1] = ws + B.states;
  b->state_bytes = B.states;
  char* shared = ws + 2 * B.states;
  double* partials = (double*)shared;
  b->partials = partials;
  char* staging = shared + B.partial;
  double* gslots = (double*)(staging + B.staging);
  b->table = (Lattice2D*)(shared + B.partial + B.staging + B.adjoint);
  b->items = (int4*)((char*)b->table + B.table);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    b->device = dev;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      b->cus = cus;
    double* unused = nullptr;
    (void)device_scratch(dev, &unused);
  }
  b->lat.reserve(count);
  b->base.resize(count);
  const int bytes = B.L[0].bytes;
  for (int i = 0; i < count; ++i) {
    maclab_s* h = new (std::nothrow) maclab_s();
    if (!h) {
      maclab_batch_destroy(b);
      return bfail(nullptr, MACLAB_EINVAL, "maclab_batch_init: out of host memory");
    }
    h->view = true;
    h->cfg = cfgs[i];
    h->cfg.workspace = nullptr;
    h->cfg.workspace_bytes = 0;
    h->L = B.L[i];
    h->stream = b->stream;
    h->state[0] = b->state[0] + B.off[i];
    h->state[1] = b->state[1] + B.off[i];
    h->partials = partials;
    h->result = partials + (size_t)kDiagBlocks * kDiagValues;
    h->staging = staging;
    h->L.staging_bytes = B.staging;
    h->gslots = gslots;
    for (int f = 0; f < 6; ++f) {
      h->fv.kind[f] = MACLAB_BC_PERIODIC;
      h->fv.rho[f] = cfgs[i].rho_ref;
      for (int c = 0; c < 3; ++c) h->fv.u[f][c] = 0.0;
    }
    h->cus = b->cus;
    h->device = b->device;
    h->e = 6.0 * cfgs[i].nu / cfgs[i].dx;  // Eq. (6)
    h->dt = cfgs[i].dx / h->e;
    b->lat.push_back(h);
    b->base[i] = (int64_t)(B.off[i] / (size_t)bytes);
  }
  hipError_t e1 = hipMemsetAsync(ws, 0, 2 * B.states, b->stream);
  if (e1 == hipSuccess) e1 = hipStreamCreateWithFlags(&b->priv, hipStreamNonBlocking);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e1 != hipSuccess) {
    rc = bfail(nullptr, MACLAB_EHIP, "maclab_batch_init: %s", hipGetErrorString(e1));
    maclab_batch_destroy(b);
    return rc;
  }
  // two nodes per lane only if every lattice is wide enough for it and of
  // even width (an odd periodic row cannot be split in pairs)
  b->kx = 2;
  for (int i = 0; i < count; ++i)
    if (B.L[i].nx < 128 || B.L[i].nx % 2) b->kx = 1;
  *out = b;
  return MACLAB_OK;
}

maclab_t maclab_batch_lattice(maclab_batch_t b, int index) {
  if (!b || index < 0 || index >= b->count) return nullptr;
  return b->lat[index];
}

int maclab_batch_count(maclab_batch_t b) { return b ? b->count : 0; }

int maclab_batch_step(maclab_batch_t b, int64_t n) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  if (n < 0) return bfail(b, MACLAB_EINVAL, "negative step count");
  int rc = batch_consistent(b);
  if (!rc) rc = batch_sync(b);
  if (rc) return rc;
  int64_t done = 0;
  const bool graphs = b->graph_steps > 0 && b->precision != MACLAB_S16;  // S16 keys every step's rounding
  if (graphs && n >= b->graph_steps + (b->lat[0]->cur & 1)) {
    if (b->lat[0]->cur & 1) {  // the graph starts from buffer 0
      rc = batch_launch(b, b->stream, 1, b->lat[0]->steps);
      if (rc) return rc;
      batch_advance(b, 1);
      done = 1;
    }
    if (!b->exec) {
      BHIP_TRY(b, hipStreamBeginCapture(b->priv, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < b->graph_steps; ++k) {
        rc = batch_launch(b, b->priv, k & 1, 0);
        if (rc) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(b->priv, &g);
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
      }
      BHIP_TRY(b, hipStreamEndCapture(b->priv, &b->graph));
      BHIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    const int64_t reps = (n - done) / b->graph_steps;
    BHIP_TRY(b, hipEventRecord(b->ev_in, b->stream));
    BHIP_TRY(b, hipStreamWaitEvent(b->priv, b->ev_in, 0));
    for (int64_t r = 0; r < reps; ++r) BHIP_TRY(b, hipGraphLaunch(b->exec, b->priv));
    BHIP_TRY(b, hipEventRecord(b->ev_out, b->priv));
    BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->ev_out, 0));
    batch_advance(b, reps * b->graph_steps);
    done += reps * b->graph_steps;
  }
  for (; done < n; ++done) {
    rc = batch_launch(b, b->stream, b->lat[0]->cur, b->lat[0]->steps);
    if (rc) return rc;
    batch_advance(b, 1);
  }
  return MACLAB_OK;
}

int maclab_batch_step_separate(maclab_batch_t b, int64_t n) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  if (n < 0) return bfail(b, MACLAB_EINVAL, "negative step count");
  int rc = batch_consistent(b);
  if (rc) return rc;
  std::vector<Fast2DShape> shapes(b->count);
  for (int i = 0; i < b->count; ++i) {
    maclab_s* h = b->lat[i];
    rc = check_faces(h);
    if (rc) return bfail(b, rc, "lattice %d: %s", i, h->err.c_str());
    const StepParams p = make_params(h);
    if (!fast2d_supported(h->L, p)) return bfail(b, MACLAB_EUNSUPPORTED, "lattice %d: not a fast D2Q9 lattice", i);
    shapes[i] = fast2d_default_shape(h->L, p, b->cus);
  }
  for (int64_t k = 0; k < n; ++k) {
    for (int i = 0; i < b->count; ++i) {
      maclab_s* h = b->lat[i];
      StepParams p = make_params(h);
      BHIP_TRY(b, launch_step_fast2d(h->L, h->state[h->cur], h->state[h->cur ^ 1], p, shapes[i], b->stream));
    }
    batch_advance(b, 1);
  }
  return MACLAB_OK;
}

int maclab_batch_get_tiling(maclab_batch_t b, int out[3]) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  if (!out) return bfail(b, MACLAB_EINVAL, "out is NULL");
  const int rc = batch_sync(b);
  if (rc) return rc;
  out[0] = b->kx;
  out[1] = b->rows;
  out[2] = b->nitems;
  return MACLAB_OK;
}

int maclab_batch_set_tiling(maclab_batch_t b, int kx, int rows) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  std::vector<Lattice2D> t;
  std::vector<int4> it;
  int rc = batch_plan(b, kx, rows, &t, &it);  // validates
  if (rc) return rc;
  b->kx = kx;
  b->rows = rows;
  return batch_sync(b);
}

int maclab_batch_set_graph(maclab_batch_t b, int steps_per_graph) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  if (steps_per_graph < 0 || steps_per_graph % 2 || steps_per_graph > 4096)
    return bfail(b, MACLAB_EINVAL, "steps per graph must be 0 or an even number up to 4096");
  if (steps_per_graph != b->graph_steps) drop_graph(b);
  b->graph_steps = steps_per_graph;
  return MACLAB_OK;
}

int maclab_batch_autotune(maclab_batch_t b, int reps, double* best_ms) {
  if (!b) return bfail(nullptr, MACLAB_EINVAL, "batch is NULL");
  if (reps < 1) return bfail(b, MACLAB_EINVAL, "reps must be >= 1");
  int rc = batch_consistent(b);
  if (rc) return rc;
  hipEvent_t e0, e1;
  BHIP_TRY(b, hipEventCreate(&e0));
  hipError_t ee = hipEventCreate(&e1);
  if (ee != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, MACLAB_EHIP, "hipEventCreate: %s", hipGetErrorString(ee));
  }
  const int kx0 = b->kx, rows0 = b->rows;
  double best = 1e300;
  int bkx = kx0, brows = rows0;
  const int cur = b->lat[0]->cur;
  for (int kx : {1, 2}) {
    for (int rows : {4, 8, 16, 32, 64, 128}) {
      std::vector<Lattice2D> t;
      std::vector<int4> it;
      if (batch_plan(b, kx, rows, &t, &it) != MACLAB_OK) continue;
      b->kx = kx;
      b->rows = rows;
      rc = batch_sync(b);
      // the spare buffer takes the output: the state is not advanced. Before
      // each timed launch an untimed pass reads the spare buffer, so that the
      // launch finds its source out of the caches, as a time step does.
      if (!rc) rc = batch_launch(b, b->stream, cur, b->lat[0]->steps);
      hipError_t he = hipSuccess;
      double total = 0;
      for (int r = 0; !rc && he == hipSuccess && r < reps; ++r) {
        he = launch_touch(b->state[cur ^ 1], b->state_bytes, (uint32_t*)b->partials, 0x9e3779b9u, b->stream);
        if (he == hipSuccess) he = hipEventRecord(e0, b->stream);
        if (he == hipSuccess) rc = batch_launch(b, b->stream, cur, b->lat[0]->steps);
        if (!rc && he == hipSuccess) he = hipEventRecord(e1, b->stream);
        if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0;
        if (!rc && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        total += ms;
      }
      if (rc || he != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        return bfail(b, MACLAB_EHIP, "autotune timing: %s", hipGetErrorString(he));
      }
      const double per = total / reps;
      if (per < best) {
        best = per;
        bkx = kx;
        brows = rows;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->kx = bkx;
  b->rows = brows;
  rc = batch_sync(b);
  if (rc) return rc;
  if (best_ms) *best_ms = best;
  return MACLAB_OK;
}

void maclab_batch_destroy(maclab_batch_t b) {
  if (!b) return;
  drop_graph(b);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->priv) (void)hipStreamDestroy(b->priv);
  for (maclab_s* h : b->lat) delete h;
  delete b;
}

const char* maclab_batch_last_error(maclab_batch_t b) { return b ? b->err.c_str() : g_err.c_str(); }

}  // extern "C"
