// The lattice BGK scheme the paper starts from, Eq. (1) with relaxation time
// tau = 1, on gfx950: the Q populations of every node are stored, and a step
// streams them and relaxes them fully to the local equilibrium Eq. (2),
//
//   f_a(x + c_a, t + 1) = f_a(x, t) - (f_a(x, t) - f_eq_a(x, t)) / tau
//                       = f_eq_a(x, t)                         (tau = 1).
//
// This is the scheme MacLAB replaces: with tau = 1 the stored populations
// are exactly the equilibria of the macroscopic state, so they carry nothing
// that rho and u do not (Methods, Eqs. (9)-(10)). Both schemes give the same
// rho and u up to rounding; this one moves 2 Q values per node and step
// instead of 2 (d + 1).
//
// Storage: Q planes of `plane` elements, node (i, j, k) at i + nx (j + ny k)
// (no row padding), holding the post-collision populations as deviations
// F_a - w_a rho_ref (FP64 or FP32), so that sums of them stay small, as in
// the MacLAB state. Fixed (boundary) nodes hold f_eq(rho_b, u_b) in both
// buffers and are never written by a step.
#include "internal.h"

namespace maclab {

namespace {

// One wavefront per x-row (lanes stride over the row), four rows per
// workgroup. The step pulls: destination x gathers population a from its
// upstream node x - c_a, so every stored population is read exactly once per
// step (no halo re-reads; neighbouring rows share only cache lines).
template <int Q, class T>
__global__ __launch_bounds__(256) void bgk_step_kernel(const T* __restrict__ src, T* __restrict__ dst, BgkParams p) {
  using Lt = Lattice<Q>;
  const int64_t rows = p.ny * p.nz;
  // workgroups go to the eight XCDs in turn: give each XCD a contiguous
  // range of row groups, so neighbouring rows share its L2
  const int64_t nb = gridDim.x, bid = blockIdx.x;
  const int64_t per = nb >> 3, rem = nb & 7, xcd = bid & 7;
  const int64_t grp = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int64_t row = grp * 4 + threadIdx.y;
  if (row >= rows) return;
  const int64_t j = row % p.ny, k = row / p.ny;
  if ((p.fixed[1] && (j == 0 || j == p.ny - 1)) || (p.fixed[2] && (k == 0 || k == p.nz - 1))) return;
  // upstream rows (an interior node of a fixed axis never wraps)
  const int64_t jr[3] = {j + 1 < p.ny ? j + 1 : 0, j, j > 0 ? j - 1 : p.ny - 1};  // index 1 - c_y
  const int64_t kr[3] = {k + 1 < p.nz ? k + 1 : 0, k, k > 0 ? k - 1 : p.nz - 1};
  const T rho_ref = (T)p.rho_ref;
  const T g[3] = {(T)p.g[0], (T)p.g[1], (T)p.g[2]};
  for (int64_t i = threadIdx.x; i < p.nx; i += 64) {
    if (p.fixed[0] && (i == 0 || i == p.nx - 1)) continue;
    const int64_t ir[3] = {i + 1 < p.nx ? i + 1 : 0, i, i > 0 ? i - 1 : p.nx - 1};
    // stream: the populations arriving at x; their density deviation and
    // momentum (Eqs. (4)-(5) in population form)
    T f[Q];
    T r = 0, m[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int64_t s = ir[1 + Lt::cx[a]] + p.nx * (jr[1 + Lt::cy[a]] + p.ny * kr[1 + Lt::cz[a]]);
      f[a] = src[(int64_t)a * p.plane + s];
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      r += f[a];
      m[0] += (T)Lt::cx[a] * f[a];
      m[1] += (T)Lt::cy[a] * f[a];
      m[2] += (T)Lt::cz[a] * f[a];
    }
    // collide with tau = 1: the new populations are the equilibria of the
    // new state (the body force of test 2 enters the momentum)
    const T rho = rho_ref + r;
    const T inv = (T)1 / rho;
    const T u0 = (m[0] + g[0]) * inv, u1 = (m[1] + g[1]) * inv, u2 = (m[2] + g[2]) * inv;
    const T uu = u0 * u0 + u1 * u1 + u2 * u2;
    const int64_t x = i + p.nx * (j + p.ny * k);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const T cu = (T)Lt::cx[a] * u0 + (T)Lt::cy[a] * u1 + (T)Lt::cz[a] * u2;
      const T phim1 = (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu;  // phi_a - 1
      // w_a (rho phi_a - rho_ref) = w_a (r + rho (phi_a - 1))
      __builtin_nontemporal_store((T)Lt::wnum[a] * (r + rho * phim1) * (T)(1.0 / 36.0), &dst[(int64_t)a * p.plane + x]);
    }
  }
}

// Populations of the state (rho, u) given as FP64 physical fields of dense
// nodes first .. first+count-1: F_a - w_a rho_ref = w_a (drho + rho (phi_a - 1))
// with phi_a of Eq. (2) at u~ = u / e.
template <int Q, class T>
__global__ void bgk_encode_kernel(T* dst, int64_t plane, const double* __restrict__ rho,
                                  const double* __restrict__ ux, const double* __restrict__ uy,
                                  const double* __restrict__ uz, int64_t first, int64_t count, double rho_ref,
                                  double inv_e) {
  using Lt = Lattice<Q>;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[s];
    const double u[3] = {ux[s] * inv_e, uy[s] * inv_e, Q == 19 ? uz[s] * inv_e : 0.0};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < Q; ++a) {
      const double cu = Lt::cx[a] * u[0] + Lt::cy[a] * u[1] + Lt::cz[a] * u[2];
      const double phim1 = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
      dst[(int64_t)a * plane + first + s] = (T)(Lt::wnum[a] / 36.0 * ((r - rho_ref) + r * phim1));
    }
  }
}

// The moments of the stored populations (the state they are the equilibria
// of): rho = rho_ref + sum_a F^_a, u = e (sum_a c_a F^_a) / rho, as FP64.
template <int Q, class T>
__global__ void bgk_decode_kernel(const T* __restrict__ src, int64_t plane, double* rho, double* ux, double* uy,
                                  double* uz, int64_t first, int64_t count, double rho_ref, double e) {
  using Lt = Lattice<Q>;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += (int64_t)gridDim.x * blockDim.x) {
    double r = 0, m[3] = {0, 0, 0};
    for (int a = 0; a < Q; ++a) {
      const double f = (double)src[(int64_t)a * plane + first + s];
      r += f;
      m[0] += Lt::cx[a] * f;
      m[1] += Lt::cy[a] * f;
      m[2] += Lt::cz[a] * f;
    }
    const double rh = rho_ref + r;
    rho[s] = rh;
    ux[s] = e * m[0] / rh;
    uy[s] = e * m[1] / rh;
    if (Q == 19) uz[s] = e * m[2] / rh;
  }
}

// Fixed nodes of both buffers get f_eq(rho_b, u_b); a node on several fixed
// faces takes the values of the lowest-numbered one.
template <int Q, class T>
__global__ void bgk_impose_kernel(T* b0, T* b1, BgkParams p, FaceValues fv, double e) {
  using Lt = Lattice<Q>;
  const int64_t N = p.nx * p.ny * p.nz;
  const int64_t n[3] = {p.nx, p.ny, p.nz};
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx[3] = {x % p.nx, (x / p.nx) % p.ny, x / (p.nx * p.ny)};
    int face = -1;
    for (int f = 0; f < 6 && face < 0; ++f) {
      if (fv.kind[f] != MACLAB_BC_FIXED) continue;
      const int ax = f / 2;
      if (idx[ax] == ((f & 1) ? n[ax] - 1 : 0)) face = f;
    }
    if (face < 0) continue;
    const double r = fv.rho[face];
    const double u[3] = {fv.u[face][0] / e, fv.u[face][1] / e, Q == 19 ? fv.u[face][2] / e : 0.0};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < Q; ++a) {
      const double cu = Lt::cx[a] * u[0] + Lt::cy[a] * u[1] + Lt::cz[a] * u[2];
      const double phim1 = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
      const T v = (T)(Lt::wnum[a] / 36.0 * ((r - p.rho_ref) + r * phim1));
      b0[(int64_t)a * p.plane + x] = v;
      b1[(int64_t)a * p.plane + x] = v;
    }
  }
}

template <int Q, class T>
hipError_t step_qt(const BgkParams& p, const void* src, void* dst, hipStream_t s) {
  const int64_t groups = (p.ny * p.nz + 3) / 4;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((bgk_step_kernel<Q, T>), dim3((unsigned)groups), dim3(64, 4), 0, s, (const T*)src, (T*)dst, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bgk_step(int q, bool fp64, const BgkParams& p, const void* src, void* dst, hipStream_t s) {
  if (q == 9) return fp64 ? step_qt<9, double>(p, src, dst, s) : step_qt<9, float>(p, src, dst, s);
  return fp64 ? step_qt<19, double>(p, src, dst, s) : step_qt<19, float>(p, src, dst, s);
}

hipError_t launch_bgk_encode(int q, bool fp64, void* dst, int64_t plane, const double* rho, const double* ux,
                             const double* uy, const double* uz, int64_t first, int64_t count, double rho_ref,
                             double e, hipStream_t s) {
  const unsigned b = blocks_256(count);
  const double ie = 1.0 / e;
  if (q == 9) {
    if (fp64)
      hipLaunchKernelGGL((bgk_encode_kernel<9, double>), dim3(b), dim3(256), 0, s, (double*)dst, plane, rho, ux, uy,
                         uz, first, count, rho_ref, ie);
    else
      hipLaunchKernelGGL((bgk_encode_kernel<9, float>), dim3(b), dim3(256), 0, s, (float*)dst, plane, rho, ux, uy,
                         uz, first, count, rho_ref, ie);
  } else {
    if (fp64)
      hipLaunchKernelGGL((bgk_encode_kernel<19, double>), dim3(b), dim3(256), 0, s, (double*)dst, plane, rho, ux, uy,
                         uz, first, count, rho_ref, ie);
    else
      hipLaunchKernelGGL((bgk_encode_kernel<19, float>), dim3(b), dim3(256), 0, s, (float*)dst, plane, rho, ux, uy,
                         uz, first, count, rho_ref, ie);
  }
  return hipGetLastError();
}

hipError_t launch_bgk_decode(int q, bool fp64, const void* src, int64_t plane, double* rho, double* ux, double* uy,
                             double* uz, int64_t first, int64_t count, double rho_ref, double e, hipStream_t s) {
  const unsigned b = blocks_256(count);
  if (q == 9) {
    if (fp64)
      hipLaunchKernelGGL((bgk_decode_kernel<9, double>), dim3(b), dim3(256), 0, s, (const double*)src, plane, rho,
                         ux, uy, uz, first, count, rho_ref, e);
    else
      hipLaunchKernelGGL((bgk_decode_kernel<9, float>), dim3(b), dim3(256), 0, s, (const float*)src, plane, rho,
                         ux, uy, uz, first, count, rho_ref, e);
  } else {
    if (fp64)
      hipLaunchKernelGGL((bgk_decode_kernel<19, double>), dim3(b), dim3(256), 0, s, (const double*)src, plane, rho,
                         ux, uy, uz, first, count, rho_ref, e);
    else
      hipLaunchKernelGGL((bgk_decode_kernel<19, float>), dim3(b), dim3(256), 0, s, (const float*)src, plane, rho,
                         ux, uy, uz, first, count, rho_ref, e);
  }
  return hipGetLastError();
}

hipError_t launch_bgk_impose(int q, bool fp64, void* b0, void* b1, const BgkParams& p, const FaceValues& fv, double e,
                             hipStream_t s) {
  const unsigned b = blocks_256(p.nx * p.ny * p.nz);
  if (q == 9) {
    if (fp64)
      hipLaunchKernelGGL((bgk_impose_kernel<9, double>), dim3(b), dim3(256), 0, s, (double*)b0, (double*)b1, p, fv, e);
    else
      hipLaunchKernelGGL((bgk_impose_kernel<9, float>), dim3(b), dim3(256), 0, s, (float*)b0, (float*)b1, p, fv, e);
  } else {
    if (fp64)
      hipLaunchKernelGGL((bgk_impose_kernel<19, double>), dim3(b), dim3(256), 0, s, (double*)b0, (double*)b1, p, fv,
                         e);
    else
      hipLaunchKernelGGL((bgk_impose_kernel<19, float>), dim3(b), dim3(256), 0, s, (float*)b0, (float*)b1, p, fv, e);
  }
  return hipGetLastError();
}

}  // namespace maclab
