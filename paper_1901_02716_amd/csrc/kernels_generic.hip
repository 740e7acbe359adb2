// General-shape kernels of the MacLAB library for gfx950: the step for any
// node counts and boundary kinds, the field codecs, boundary imposition and
// the FP64 diagnostics reduction.
//
// The step is the gather of the paper's Eqs. (4)-(5): the new density and
// momentum of node x are the sums over links a of the equilibrium f_eq_a
// (Eq. (2)) evaluated at the upstream node x - c_a. It is computed in
// deviation form: with rho = rho_ref + drho and phi_a the bracket of Eq. (2),
//   F^_a = f_eq_a - w_a rho_ref = w_a [drho + rho (phi_a - 1)],
// and because sum_a w_a = 1 and sum_a w_a c_a = 0,
//   drho' = sum_a F^_a(x - c_a),   m' = sum_a c_a F^_a(x - c_a),
// which is Eqs. (4)-(5) exactly while only small numbers are summed.
// The new lattice velocity is u~' = (m' + g) / (rho_ref + drho').
#include "internal.h"

#include <algorithm>

namespace maclab {

template <class C>
__device__ __forceinline__ typename C::T load_field(const typename C::elem* base, int64_t plane, int f,
                                                    int64_t node) {
  return C::dec(base[f * plane + node], f);
}

template <class C>
__device__ __forceinline__ void store_field(typename C::elem* base, int64_t plane, int f, int64_t node,
                                            typename C::T v, uint32_t node_bits) {
  base[f * plane + node] = C::enc(v, f, node_bits);
}

__device__ __forceinline__ int64_t wrap_idx(int64_t v, int64_t n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// One thread per destination node; the upstream values come through the
// cache. Handles every shape, periodic wrap on any axis and fixed faces.
template <int Q, class C>
__global__ __launch_bounds__(256) void step_generic_kernel(const typename C::elem* __restrict__ src,
                                                           typename C::elem* __restrict__ dst,
                                                           StepParams p) {
  using Lat = Lattice<Q>;
  using T = typename C::T;
  constexpr int D = Lat::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  const int64_t k = blockIdx.z;
  if (i >= p.nx || j >= p.ny) return;
  if ((p.fixed[0] && (i == 0 || i == p.nx - 1)) || (p.fixed[1] && (j == 0 || j == p.ny - 1)) ||
      (p.fixed[2] && (k == 0 || k == p.nz - 1)))
    return;  // fixed nodes hold their values in both buffers
  const T rho_ref = (T)p.rho_ref;
  T drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int cx = Lat::cx[a], cy = Lat::cy[a], cz = Lat::cz[a];
    const int64_t si = wrap_idx(i - cx, p.nx);
    const int64_t sj = wrap_idx(j - cy, p.ny);
    const int64_t sk = wrap_idx(k - cz, p.nz);
    const int64_t s = si + p.px * (sj + p.ny * sk);
    const T dr = load_field<C>(src, p.plane, 0, s);
    const T ux = load_field<C>(src, p.plane, 1, s);
    const T uy = load_field<C>(src, p.plane, 2, s);
    T uz = 0;
    if constexpr (D == 3) uz = load_field<C>(src, p.plane, 3, s);
    const T rho = rho_ref + dr;
    const T cu = (T)cx * ux + (T)cy * uy + (T)cz * uz;
    const T uu = ux * ux + uy * uy + uz * uz;
    // 36 F^_a with the integer weight numerators (w_a = wnum_a / 36)
    const T F = (T)Lat::wnum[a] * (dr + rho * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu));
    drho += F;
    if (cx) mx += (T)cx * F;
    if (cy) my += (T)cy * F;
    if (cz) mz += (T)cz * F;
  }
  // drho' = r / 36, u~' = (m + 36 g) / (36 rho_ref + r)
  const T inv = (T)1 / ((T)36 * rho_ref + drho);
  const int64_t x = i + p.px * (j + p.ny * k);
  uint32_t bits = 0;
  if constexpr (needs_rng<C>::value) bits = sr_node_bits(p.sr_key, i + p.nx * (j + p.ny * k));
  store_field<C>(dst, p.plane, 0, x, div36(drho), bits);
  store_field<C>(dst, p.plane, 1, x, (mx + (T)(36.0 * p.g[0])) * inv, bits);
  store_field<C>(dst, p.plane, 2, x, (my + (T)(36.0 * p.g[1])) * inv, bits);
  if constexpr (D == 3) store_field<C>(dst, p.plane, 3, x, (mz + (T)(36.0 * p.g[2])) * inv, bits);
}

// Writes what each bounded face holds into both buffers: (rho_b, u_b) on a
// fixed face, u_b on a face with a zero-gradient density, rho_b on a pressure
// face. A node on several bounded faces belongs to the lowest-numbered one.
// The other values of the last two kinds come from derive_faces_kernel.
template <class C>
__global__ void impose_bc_kernel(typename C::elem* b0, typename C::elem* b1, int64_t nx, int64_t ny,
                                 int64_t nz, int64_t px, int64_t plane, int d, FaceValues fv, double rho_ref,
                                 double e) {
  const int64_t N = nx * ny * nz;
  const int64_t n[3] = {nx, ny, nz};
  for (int64_t di = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; di < N; di += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx[3] = {di % nx, (di / nx) % ny, di / (nx * ny)};
    const int64_t x = stored_index(di, nx, px);
    int face = -1;
    for (int f = 0; f < 6 && face < 0; ++f) {
      if (fv.kind[f] == MACLAB_BC_PERIODIC) continue;
      const int ax = f / 2;
      if (idx[ax] == ((f & 1) ? n[ax] - 1 : 0)) face = f;
    }
    if (face < 0) continue;
    typename C::elem v[4];
    v[0] = C::enc_nearest((typename C::T)(fv.rho[face] - rho_ref), 0);
    for (int c = 0; c < d; ++c) v[1 + c] = C::enc_nearest((typename C::T)(fv.u[face][c] / e), 1 + c);
    const int first = fv.kind[face] == MACLAB_BC_RHO_NEUMANN ? 1 : 0;
    const int last = fv.kind[face] == MACLAB_BC_PRESSURE ? 0 : d;
    for (int f = first; f <= last; ++f) {
      b0[f * plane + x] = v[f];
      b1[f * plane + x] = v[f];
    }
  }
}

// The values of faces with a zero normal gradient: after a step, every node
// owned by a face with a zero-gradient density takes the stored density of
// its nearest interior node (each index on a bounded axis moved into
// 1 .. n-2), and every node of a pressure face that node's stored velocity.
// Stored elements are copied bit for bit (the same codec on both sides). One
// thread per node of a face (blockIdx.y = face); the nodes read are interior
// nodes, which this kernel never writes.
template <class E>
__global__ void derive_faces_kernel(E* buf, int64_t nx, int64_t ny, int64_t nz, int64_t px, int64_t plane, int d,
                                    FaceValues fv) {
  const int face = blockIdx.y;
  const int kind = fv.kind[face];
  if (kind != MACLAB_BC_RHO_NEUMANN && kind != MACLAB_BC_PRESSURE) return;
  const int64_t n[3] = {nx, ny, nz};
  const int ax = face / 2, ab = ax == 0 ? 1 : 0, ac = ax == 2 ? 1 : 2;
  const int64_t count = n[ab] * n[ac];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx[3];
    idx[ax] = (face & 1) ? n[ax] - 1 : 0;
    idx[ab] = t % n[ab];
    idx[ac] = t / n[ab];
    bool owned = true;  // by no lower-numbered bounded face
    for (int g = 0; g < face; ++g) {
      if (fv.kind[g] == MACLAB_BC_PERIODIC) continue;
      if (idx[g / 2] == ((g & 1) ? n[g / 2] - 1 : 0)) owned = false;
    }
    if (!owned) continue;
    int64_t in[3];
    for (int a = 0; a < 3; ++a) {
      in[a] = idx[a];
      if (fv.kind[2 * a] == MACLAB_BC_PERIODIC) continue;
      in[a] = in[a] < 1 ? 1 : (in[a] > n[a] - 2 ? n[a] - 2 : in[a]);
    }
    const int64_t x = idx[0] + px * (idx[1] + ny * idx[2]);
    const int64_t s = in[0] + px * (in[1] + ny * in[2]);
    if (kind == MACLAB_BC_RHO_NEUMANN) {
      buf[x] = buf[s];
    } else {
      for (int f = 1; f <= d; ++f) buf[f * plane + x] = buf[f * plane + s];
    }
  }
}

// Physical float64 -> stored: value = (src - offset) * mul, rounded to nearest;
// src[i] is dense node first + i of the plane at dst.
template <class C>
__global__ void encode_kernel(typename C::elem* dst, const double* __restrict__ src, int64_t first, int64_t count,
                              int64_t nx, int64_t px, double offset, double mul, int field) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[stored_index(first + i, nx, px)] = C::enc_nearest((typename C::T)((src[i] - offset) * mul), field);
}

// Stored -> physical float64: dst = offset + mul * value; dst[i] is dense
// node first + i of the plane at src.
template <class C>
__global__ void decode_kernel(double* dst, const typename C::elem* __restrict__ src, int64_t first, int64_t count,
                              int64_t nx, int64_t px, double offset, double mul, int field) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = offset + mul * (double)C::dec(src[stored_index(first + i, nx, px)], field);
}

// ------------------------------------------------------------ diagnostics
// Mass, momentum and kinetic energy in FP64 (the conserved moments of the
// equilibrium, Methods, Eqs. (14)-(15)), max |u~| and the non-finite count.
// Each block reduces its grid-stride share with 64-lane wavefront shuffles,
// then across waves through LDS, and writes one partial row; a single block
// then folds the rows in a fixed order, so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

template <class C>
__global__ __launch_bounds__(256) void diag_partial_kernel(const typename C::elem* __restrict__ s,
                                                           int64_t N, int64_t nx, int64_t px, int64_t plane,
                                                           int d, double rho_ref, double e,
                                                           double* __restrict__ partials) {
  double acc[kDiagValues] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t di = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; di < N;
       di += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = stored_index(di, nx, px);
    const double rho = rho_ref + (double)C::dec(s[x], 0);
    double ut[3] = {0, 0, 0};
    bool finite = isfinite(rho);
    for (int c = 0; c < d; ++c) {
      ut[c] = (double)C::dec(s[(1 + c) * plane + x], 1 + c);
      finite = finite && isfinite(ut[c]);
    }
    if (!finite) {
      acc[6] += 1.0;
      continue;
    }
    const double uu = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    acc[0] += rho;
    for (int c = 0; c < 3; ++c) acc[1 + c] += rho * e * ut[c];
    acc[4] += 0.5 * rho * e * e * uu;
    acc[5] = fmax(acc[5], sqrt(uu));
  }
  __shared__ double red[kDiagValues][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < kDiagValues; ++v) {
    const double r = (v == 5) ? wave_max(acc[v]) : wave_sum(acc[v]);
    if (lane == 0) red[v][wave] = r;
  }
  __syncthreads();
  if (threadIdx.x < kDiagValues) {
    const int v = threadIdx.x;
    double r = red[v][0];
    for (int w = 1; w < 4; ++w) r = (v == 5) ? fmax(r, red[v][w]) : r + red[v][w];
    partials[(int64_t)blockIdx.x * kDiagValues + v] = r;
  }
}

__global__ __launch_bounds__(256) void diag_final_kernel(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out) {
  __shared__ double red[kDiagValues][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < kDiagValues; ++v) {
    double acc = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double x = partials[(int64_t)b * kDiagValues + v];
      acc = (v == 5) ? fmax(acc, x) : acc + x;
    }
    const double r = (v == 5) ? wave_max(acc) : wave_sum(acc);
    if (lane == 0) red[v][wave] = r;
  }
  __syncthreads();
  if (threadIdx.x < kDiagValues) {
    const int v = threadIdx.x;
    double r = red[v][0];
    for (int w = 1; w < 4; ++w) r = (v == 5) ? fmax(r, red[v][w]) : r + red[v][w];
    out[v] = r;
  }
}

// Change over the last step (recipe step (v): the run goes on until a
// solution is reached): per block, the largest |u~_i(b) - u~_i(a)| over nodes
// and components, the largest |drho(b) - drho(a)|, and the count of nodes
// non-finite in b. Maxima do not depend on the order of the reduction.
template <class C>
__global__ __launch_bounds__(256) void residual_partial_kernel(const typename C::elem* __restrict__ a,
                                                               const typename C::elem* __restrict__ b, int64_t N,
                                                               int64_t nx, int64_t px, int64_t plane, int d,
                                                               double* __restrict__ partials) {
  double du = 0, dr = 0, bad = 0;
  for (int64_t di = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; di < N;
       di += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = stored_index(di, nx, px);
    const double rb = (double)C::dec(b[x], 0);
    bool finite = isfinite(rb);
    double m = 0;
    for (int c = 1; c <= d; ++c) {
      const double ub = (double)C::dec(b[c * plane + x], c);
      finite = finite && isfinite(ub);
      m = fmax(m, fabs(ub - (double)C::dec(a[c * plane + x], c)));
    }
    if (!finite) {
      bad += 1.0;
      continue;
    }
    du = fmax(du, m);
    dr = fmax(dr, fabs(rb - (double)C::dec(a[x], 0)));
  }
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  du = wave_max(du);
  dr = wave_max(dr);
  bad = wave_sum(bad);
  if (lane == 0) {
    red[0][wave] = du;
    red[1][wave] = dr;
    red[2][wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int v = threadIdx.x;
    double r = red[v][0];
    for (int w = 1; w < 4; ++w) r = v < 2 ? fmax(r, red[v][w]) : r + red[v][w];
    partials[(int64_t)blockIdx.x * 4 + v] = r;
  }
}

__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ partials, int nblocks,
                                                             double* __restrict__ out) {
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < 3; ++v) {
    double acc = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double x = partials[(int64_t)b * 4 + v];
      acc = v < 2 ? fmax(acc, x) : acc + x;
    }
    const double r = v < 2 ? wave_max(acc) : wave_sum(acc);
    if (lane == 0) red[v][wave] = r;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int v = threadIdx.x;
    double r = red[v][0];
    for (int w = 1; w < 4; ++w) r = v < 2 ? fmax(r, red[v][w]) : r + red[v][w];
    out[v] = r;
  }
}

// ---------------------------------------------------------------- launchers
template <class F>
static hipError_t dispatch_codec(int precision, F&& f) {
  switch (precision) {
    case MACLAB_FP64: return f(CodecF64{});
    case MACLAB_FP32: return f(CodecF32{});
    case MACLAB_HILO: return f(CodecHILO{});
    case MACLAB_S16: return f(CodecS16{});
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_generic(const Layout& L, const void* src, void* dst, const StepParams& p,
                               hipStream_t s) {
  const dim3 block(64, 4, 1);
  const dim3 grid((unsigned)((L.nx + 63) / 64), (unsigned)((L.ny + 3) / 4), (unsigned)L.nz);
  return dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    using E = typename C::elem;
    if (L.q == 9)
      hipLaunchKernelGGL((step_generic_kernel<9, C>), grid, block, 0, s, (const E*)src, (E*)dst, p);
    else
      hipLaunchKernelGGL((step_generic_kernel<19, C>), grid, block, 0, s, (const E*)src, (E*)dst, p);
    return hipGetLastError();
  });
}

hipError_t launch_impose_bc(const Layout& L, void* b0, void* b1, const FaceValues& fv, double rho_ref,
                            double e, hipStream_t s) {
  const unsigned blocks = blocks_256(L.N);
  return dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    using E = typename C::elem;
    hipLaunchKernelGGL((impose_bc_kernel<C>), dim3(blocks), dim3(256), 0, s, (E*)b0, (E*)b1, L.nx, L.ny,
                       L.nz, L.px, L.plane, L.d, fv, rho_ref, e);
    return hipGetLastError();
  });
}

bool has_derived_faces(const FaceValues& fv) {
  for (int f = 0; f < 6; ++f)
    if (fv.kind[f] == MACLAB_BC_RHO_NEUMANN || fv.kind[f] == MACLAB_BC_PRESSURE) return true;
  return false;
}

hipError_t launch_derive_faces(const Layout& L, void* buf, const FaceValues& fv, hipStream_t s) {
  if (!has_derived_faces(fv)) return hipSuccess;
  const int64_t big = std::max(L.nx * L.ny, std::max(L.ny * L.nz, L.nx * L.nz));
  const dim3 grid(blocks_256(big), 2 * L.d);
  switch (L.bytes) {
    case 2:
      hipLaunchKernelGGL((derive_faces_kernel<uint16_t>), grid, dim3(256), 0, s, (uint16_t*)buf, L.nx, L.ny, L.nz,
                         L.px, L.plane, L.d, fv);
      break;
    case 4:
      hipLaunchKernelGGL((derive_faces_kernel<uint32_t>), grid, dim3(256), 0, s, (uint32_t*)buf, L.nx, L.ny, L.nz,
                         L.px, L.plane, L.d, fv);
      break;
    default:
      hipLaunchKernelGGL((derive_faces_kernel<uint64_t>), grid, dim3(256), 0, s, (uint64_t*)buf, L.nx, L.ny, L.nz,
                         L.px, L.plane, L.d, fv);
  }
  return hipGetLastError();
}

hipError_t launch_encode(const Layout& L, void* dst, const double* src, int64_t first, int64_t count,
                         double offset, double mul, int field, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = blocks_256(count);
  return dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL((encode_kernel<C>), dim3(blocks), dim3(256), 0, s, (typename C::elem*)dst, src, first,
                       count, L.nx, L.px, offset, mul, field);
    return hipGetLastError();
  });
}

hipError_t launch_decode(const Layout& L, double* dst, const void* src, int64_t first, int64_t count,
                         double offset, double mul, int field, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = blocks_256(count);
  return dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL((decode_kernel<C>), dim3(blocks), dim3(256), 0, s, dst,
                       (const typename C::elem*)src, first, count, L.nx, L.px, offset, mul, field);
    return hipGetLastError();
  });
}

hipError_t launch_diagnostics(const Layout& L, const void* state, double rho_ref, double e, double* partials,
                              double* result, hipStream_t s) {
  const int64_t want = (L.N + 255) / 256;
  const int blocks = (int)(want < kDiagBlocks ? (want > 0 ? want : 1) : kDiagBlocks);
  hipError_t err = dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL((diag_partial_kernel<C>), dim3(blocks), dim3(256), 0, s,
                       (const typename C::elem*)state, L.N, L.nx, L.px, L.plane, L.d, rho_ref, e, partials);
    return hipGetLastError();
  });
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, partials, blocks, result);
  return hipGetLastError();
}

// Streaming copy in the access forms of the step kernels, to measure the
// memory rate a step can reach: 16-byte non-temporal loads and device-scope
// (sc1) stores, the fastest copy of a state buffer measured on the device
// (a 268 MB buffer back and forth: 79.7 us with four workgroups of 256 per
// CU, 85.5 us with non-temporal stores, 89.6 us with 8192 workgroups). It
// moves the bytes of a step with none of its arithmetic. blockIdx.y selects
// a chunk of at most kCopyChunk bytes, which one buffer resource addresses.
constexpr int64_t kCopyChunk = int64_t(1) << 30;
__global__ void stream_copy_kernel(const char* __restrict__ src, char* __restrict__ dst, int64_t bytes) {
  typedef uint32_t w4 __attribute__((ext_vector_type(4)));
  const int64_t base = (int64_t)blockIdx.y * kCopyChunk;
  const int64_t left = bytes - base;
  const int len = (int)(left < kCopyChunk ? left : kCopyChunk);
  const buf_t rs = make_buf(src + base, len), rd = make_buf(dst + base, len);
  const int stride = (int)(gridDim.x * blockDim.x) * 16;
  for (int off = (int)(blockIdx.x * blockDim.x + threadIdx.x) * 16; off < len; off += stride)
    buf_store<w4, kStoreDevice>(buf_load<w4, kStoreStream>(rs, off), rd, off);
}

hipError_t launch_residual(const Layout& L, const void* prev, const void* cur, double* partials, double* result,
                           hipStream_t s) {
  const int64_t want = (L.N + 255) / 256;
  const int blocks = (int)(want < kDiagBlocks ? (want > 0 ? want : 1) : kDiagBlocks);
  hipError_t err = dispatch_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL((residual_partial_kernel<C>), dim3(blocks), dim3(256), 0, s, (const typename C::elem*)prev,
                       (const typename C::elem*)cur, L.N, L.nx, L.px, L.plane, L.d, partials);
    return hipGetLastError();
  });
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, s, partials, blocks, result);
  return hipGetLastError();
}

__global__ void touch_kernel(const uint4* __restrict__ p, int64_t n16, uint32_t* __restrict__ sink, uint32_t key) {
  uint32_t acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const uint4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == key) sink[0] = acc;
}

hipError_t launch_touch(const void* buf, size_t bytes, uint32_t* sink, uint32_t key, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  const int64_t want = (n16 + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(touch_kernel, dim3(blocks), dim3(256), 0, s, (const uint4*)buf, n16, sink, key);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 16) return hipErrorInvalidValue;
  const int64_t chunks = ((int64_t)bytes + kCopyChunk - 1) / kCopyChunk;
  const int64_t want = ((int64_t)(bytes < (size_t)kCopyChunk ? bytes : (size_t)kCopyChunk) / 16 + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks, (unsigned)chunks), dim3(256), 0, s, (const char*)src,
                     (char*)dst, (int64_t)bytes);
  return hipGetLastError();
}

}  // namespace maclab
