// Reverse mode of the MacLAB step for gfx950.
//
// For a loss L on later states, let (rhobar', ubar') be the adjoint of the
// new state (rho', u~') at node x (lattice units). The step
//   rho'(x) = sum_a F_a(x - c_a),  m'(x) = sum_a c_a F_a(x - c_a),
//   u~'(x)  = (m'(x) + g) / rho'(x),  F_a = w_a rho phi_a(u~)   (Eqs. (2), (4), (5))
// is reversed node by node:
//   Mbar(x) = ubar'(x) / rho'(x),   Rbar(x) = rhobar'(x) - ubar'(x).u~'(x) / rho'(x),
//   gbar   += sum_x Mbar(x),
//   Fbar_a(y) = Rbar(y + c_a) + c_a . Mbar(y + c_a),
//   rhobar(y) = sum_a Fbar_a w_a phi_a(u~(y)),
//   ubar(y)   = rho(y) sum_a Fbar_a w_a (3 c_a + 9 (c_a.u~) c_a - 3 u~).
// Fixed nodes hold constants: their Rbar, Mbar and own adjoint are zero.
// The gather from the downstream nodes y + c_a needs no atomics. The force
// adjoint is summed per workgroup in FP64 into a slot that the same
// workgroup updates every step, so its value does not depend on timing.
#include "internal.h"

namespace maclab {

template <int Q, class C>
__global__ __launch_bounds__(256) void adjoint_generic_kernel(const typename C::elem* __restrict__ sn,
                                                              const typename C::elem* __restrict__ sn1,
                                                              const typename C::T* __restrict__ an1,
                                                              typename C::T* __restrict__ an, StepParams p,
                                                              double* __restrict__ gslots) {
  using Lat = Lattice<Q>;
  using T = typename C::T;
  constexpr int D = Lat::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  const int64_t k = blockIdx.z;
  const bool inside = i < p.nx && j < p.ny;
  const T rho_ref = (T)p.rho_ref;
  auto is_fixed = [&](int64_t a, int64_t b, int64_t c) {
    return (p.fixed[0] && (a == 0 || a == p.nx - 1)) || (p.fixed[1] && (b == 0 || b == p.ny - 1)) ||
           (p.fixed[2] && (c == 0 || c == p.nz - 1));
  };
  auto wrap = [](int64_t v, int64_t n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  // Rbar and Mbar at node x (zero at fixed nodes)
  auto downstream = [&](int64_t xi, int64_t xj, int64_t xk, T& Rb, T (&Mb)[3]) {
    Mb[0] = Mb[1] = Mb[2] = (T)0;
    Rb = (T)0;
    if (is_fixed(xi, xj, xk)) return;
    const int64_t x = xi + p.nx * (xj + p.ny * xk);
    const T r1 = rho_ref + C::dec(sn1[x], 0);
    const T inv = (T)1 / r1;
    T dot = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const T ub = an1[(1 + c) * p.plane + x];
      Mb[c] = ub * inv;
      dot += ub * C::dec(sn1[(1 + c) * p.plane + x], 1 + c);
    }
    Rb = an1[x] - dot * inv;
  };

  double gpart[3] = {0, 0, 0};
  if (inside) {
    const int64_t y = i + p.nx * (j + p.ny * k);
    T rb = 0, ub[3] = {0, 0, 0};
    if (!is_fixed(i, j, k)) {
      const T rho = rho_ref + C::dec(sn[y], 0);
      T u[3] = {0, 0, 0};
#pragma unroll
      for (int c = 0; c < D; ++c) u[c] = C::dec(sn[(1 + c) * p.plane + y], 1 + c);
      const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const int cx = Lat::cx[a], cy = Lat::cy[a], cz = Lat::cz[a];
        T Rb, Mb[3];
        downstream(wrap(i + cx, p.nx), wrap(j + cy, p.ny), wrap(k + cz, p.nz), Rb, Mb);
        if (a == 0) {
          for (int c = 0; c < D; ++c) gpart[c] = (double)Mb[c];
        }
        const T Fb = Rb + (T)cx * Mb[0] + (T)cy * Mb[1] + (T)cz * Mb[2];
        const T G = (T)Lat::wnum[a] / (T)36 * Fb;
        const T cu = (T)cx * u[0] + (T)cy * u[1] + (T)cz * u[2];
        rb += G * ((T)1 + (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
        const T s = (T)3 + (T)9 * cu;
        ub[0] += G * rho * (s * (T)cx - (T)3 * u[0]);
        ub[1] += G * rho * (s * (T)cy - (T)3 * u[1]);
        ub[2] += G * rho * (s * (T)cz - (T)3 * u[2]);
      }
    }
    an[y] = rb;
#pragma unroll
    for (int c = 0; c < D; ++c) an[(1 + c) * p.plane + y] = ub[c];
  }
  // per-workgroup FP64 sum of Mbar over its nodes, added to this
  // workgroup's own slot
  __shared__ double red[3][4];
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = gpart[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (t < 3) {
    const double s = ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
    const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    gslots[b * 4 + t] += s;
  }
}

// Adjoint of the state for a loss with derivative dLdu (physical velocity,
// FP64, d planes of N): ubar = e dL/du, rhobar = 0.
template <class T>
__global__ void adjoint_seed_kernel(const double* __restrict__ dLdu, T* __restrict__ adj, int64_t N, int64_t plane,
                                    int d, double e) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  adj[x] = (T)0;
  for (int c = 0; c < d; ++c) adj[(1 + c) * plane + x] = (T)(e * dLdu[c * N + x]);
}

// dL/du0 = ubar / e, dL/drho0 = rhobar (FP64 outputs, SoA as the fields).
template <class T>
__global__ void adjoint_result_kernel(const T* __restrict__ adj, double* __restrict__ dLdu, double* __restrict__ dLdrho,
                                      int64_t N, int64_t plane, int d, double e) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  if (dLdrho) dLdrho[x] = (double)adj[x];
  for (int c = 0; c < d; ++c) dLdu[c * N + x] = (double)adj[(1 + c) * plane + x] / e;
}

// Folds the per-workgroup slots in a fixed order: out[c] = sum_b slots[b][c].
__global__ __launch_bounds__(256) void adjoint_fold_kernel(const double* __restrict__ slots, int64_t nslots,
                                                           double* __restrict__ out) {
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = 0; c < 3; ++c) {
    double v = 0;
    for (int64_t b = threadIdx.x; b < nslots; b += blockDim.x) v += slots[b * 4 + c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) out[threadIdx.x] = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) +
                                          red[threadIdx.x][3];
}

// ---------------------------------------------------------------- launchers
int64_t adjoint_slots(const Layout& L) {
  return ((L.nx + 63) / 64) * ((L.ny + 3) / 4) * L.nz;
}

hipError_t launch_adjoint_step(const Layout& L, const void* sn, const void* sn1, const void* an1, void* an,
                               const StepParams& p, double* gslots, hipStream_t s) {
  const dim3 block(64, 4, 1);
  const dim3 grid((unsigned)((L.nx + 63) / 64), (unsigned)((L.ny + 3) / 4), (unsigned)L.nz);
  auto go = [&](auto codec) {
    using C = decltype(codec);
    using E = typename C::elem;
    using T = typename C::T;
    if (L.q == 9)
      hipLaunchKernelGGL((adjoint_generic_kernel<9, C>), grid, block, 0, s, (const E*)sn, (const E*)sn1,
                         (const T*)an1, (T*)an, p, gslots);
    else
      hipLaunchKernelGGL((adjoint_generic_kernel<19, C>), grid, block, 0, s, (const E*)sn, (const E*)sn1,
                         (const T*)an1, (T*)an, p, gslots);
    return hipGetLastError();
  };
  switch (L.precision) {
    case MACLAB_FP64: return go(CodecF64{});
    case MACLAB_FP32: return go(CodecF32{});
    case MACLAB_HILO: return go(CodecHILO{});
    case MACLAB_S16: return go(CodecS16{});
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_seed(const Layout& L, const double* dLdu, void* adj, double e, hipStream_t s) {
  const unsigned blocks = (unsigned)((L.N + 255) / 256);
  if (L.precision == MACLAB_FP64)
    hipLaunchKernelGGL(adjoint_seed_kernel<double>, dim3(blocks), dim3(256), 0, s, dLdu, (double*)adj, L.N, L.plane,
                       L.d, e);
  else
    hipLaunchKernelGGL(adjoint_seed_kernel<float>, dim3(blocks), dim3(256), 0, s, dLdu, (float*)adj, L.N, L.plane,
                       L.d, e);
  return hipGetLastError();
}

hipError_t launch_adjoint_result(const Layout& L, const void* adj, double* dLdu, double* dLdrho, double e,
                                 hipStream_t s) {
  const unsigned blocks = (unsigned)((L.N + 255) / 256);
  if (L.precision == MACLAB_FP64)
    hipLaunchKernelGGL(adjoint_result_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)adj, dLdu, dLdrho,
                       L.N, L.plane, L.d, e);
  else
    hipLaunchKernelGGL(adjoint_result_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)adj, dLdu, dLdrho,
                       L.N, L.plane, L.d, e);
  return hipGetLastError();
}

hipError_t launch_adjoint_fold(const double* slots, int64_t nslots, double* out, hipStream_t s) {
  hipLaunchKernelGGL(adjoint_fold_kernel, dim3(1), dim3(256), 0, s, slots, nslots, out);
  return hipGetLastError();
}

}  // namespace maclab
