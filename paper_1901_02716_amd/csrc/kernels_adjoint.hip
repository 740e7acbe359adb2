// Reverse mode of the MacLAB step for gfx950.
//
// The step (Eqs. (2), (4), (5), lattice units)
//   rho'(x) = sum_a F_a(x - c_a),  u~'(x) = (sum_a c_a F_a(x - c_a) + g) / rho'(x),
//   F_a(y)  = w_a rho(y) phi_a(u~(y)),  phi_a = 1 + 3 c.u + 4.5 (c.u)^2 - 1.5 |u|^2,
// is reversed node by node. For a loss L, write (rhobar, ubar) for its
// derivatives with respect to (rho, u~) of one state. The adjoint buffers do
// not hold (rhobar, ubar) but the pair the previous step needs,
//   Mbar = ubar / rho,   Rbar = rhobar - Mbar . u~        (zero at fixed nodes),
// because with it the reverse step reads only u~ of the older state:
//   Fbar_a(y) = Rbar'(y + c_a) + c_a . Mbar'(y + c_a),
//   S0 = sum_a w_a Fbar_a, S1 = sum_a w_a c_a Fbar_a, S2 = sum_a w_a c_a c_a Fbar_a,
//   rhobar(y) = S0 (1 - 1.5 |u|^2) + 3 u.S1 + 4.5 u.S2.u,
//   ubar(y)   = rho(y) (3 S1 + 9 S2 u - 3 u S0),
// so that Mbar(y) = 3 S1 + 9 S2 u - 3 u S0 and Rbar(y) = S0 (1 + 1.5 |u|^2) -
// 4.5 u.S2.u: rho(y) cancels. The force enters every step as g = dt G / e, so
// dL/dg accumulates sum_x Mbar'(x) over the nodes and steps; it is summed per
// wavefront or workgroup in FP64 into a slot that the same wavefront or
// workgroup updates every step, so its value does not depend on timing.
// The gather from the downstream nodes y + c_a needs no atomics.
#include "internal.h"

namespace maclab {

namespace {

__device__ __forceinline__ bool node_fixed(const StepParams& p, int64_t i, int64_t j, int64_t k) {
  return (p.fixed[0] && (i == 0 || i == p.nx - 1)) || (p.fixed[1] && (j == 0 || j == p.ny - 1)) ||
         (p.fixed[2] && (k == 0 || k == p.nz - 1));
}

template <class T, int KX>
struct alignas(sizeof(T) * KX) RowVecT {
  T v[KX];
};

// Sums a per-lane FP64 value over a 64-lane wavefront (result in lane 0).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

}  // namespace

// ------------------------------------------------------- any lattice, any size
// One thread per node y; grid (nx/64, ny/4, nz), block (64, 4).
template <int Q, class C>
__global__ __launch_bounds__(256) void adjoint_generic_kernel(const typename C::elem* __restrict__ sn,
                                                              const typename C::T* __restrict__ bn1,
                                                              typename C::T* __restrict__ bn, StepParams p,
                                                              double* __restrict__ gslots) {
  using Lat = Lattice<Q>;
  using T = typename C::T;
  constexpr int D = Lat::D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  const int64_t k = blockIdx.z;
  const bool inside = i < p.nx && j < p.ny;
  auto wrap = [](int64_t v, int64_t n) { return v < 0 ? v + n : (v >= n ? v - n : v); };

  double gpart[3] = {0, 0, 0};
  if (inside) {
    const int64_t y = i + p.px * (j + p.ny * k);
#pragma unroll
    for (int c = 0; c < D; ++c) gpart[c] = (double)bn1[(1 + c) * p.plane + y];
    T rb = 0, mb[3] = {0, 0, 0}, u[3] = {0, 0, 0};
    const bool fixed = node_fixed(p, i, j, k);
    if (!fixed) {
#pragma unroll
      for (int c = 0; c < D; ++c) u[c] = C::dec(sn[(1 + c) * p.plane + y], 1 + c);
      const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const int cx = Lat::cx[a], cy = Lat::cy[a], cz = Lat::cz[a];
        // a non-fixed node has all its neighbours on the lattice (or wrapped)
        const int64_t x = wrap(i + cx, p.nx) + p.px * (wrap(j + cy, p.ny) + p.ny * wrap(k + cz, p.nz));
        T Fb = bn1[x];
        if (cx) Fb += (T)cx * bn1[p.plane + x];
        if (cy) Fb += (T)cy * bn1[2 * p.plane + x];
        if (cz) Fb += (T)cz * bn1[3 * p.plane + x];
        const T G = (T)Lat::wnum[a] / (T)36 * Fb;
        const T cu = (T)cx * u[0] + (T)cy * u[1] + (T)cz * u[2];
        rb += G * ((T)1 + (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
        const T s = (T)3 + (T)9 * cu;
        mb[0] += G * (s * (T)cx - (T)3 * u[0]);
        mb[1] += G * (s * (T)cy - (T)3 * u[1]);
        mb[2] += G * (s * (T)cz - (T)3 * u[2]);
      }
      rb -= mb[0] * u[0] + mb[1] * u[1] + mb[2] * u[2];
    }
    bn[y] = rb;
#pragma unroll
    for (int c = 0; c < D; ++c) bn[(1 + c) * p.plane + y] = mb[c];
  }
  __shared__ double red[3][4];
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = wave_sum(gpart[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (t < 3) {
    const double s = ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
    const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    gslots[b * 4 + t] += s;
  }
}

// ------------------------------------------------------------- fast D2Q9
// One wavefront per (x-segment of 64*KX nodes, band of rows), marching up the
// rows as the forward kernel does. The D2Q9 weights factor as w = wx(c_x)
// wy(c_y) with wx = wy = (1, 4, 1)/6, so every moment S is a 3-point sum in x
// of each adjoint row followed by a 3-point sum in y. Per source row and
// node the x pass gives (times 6, with L/R the left/right neighbours)
//   a0 = P_L + 4P + P_R + (Mx_R - Mx_L)   b0 = My_L + 4My + My_R
//   a1 = (P_R - P_L) + (Mx_R + Mx_L)      b1 = My_R - My_L
//   a2 = P_L + P_R + (Mx_R - Mx_L)        b2 = My_L + My_R
// (P = Rbar', Mx, My = Mbar'), and for destination row j, with rows m = j-1,
// c = j, p = j+1, the moments times 36 are
//   S0 = (a0-b0)_m + 4 a0_c + (a0+b0)_p   S2yy = (a0-b0)_m + (a0+b0)_p
//   S1y = (a0+b0)_p - (a0-b0)_m           S1x = (a1-b1)_m + 4 a1_c + (a1+b1)_p
//   S2xy = (a1+b1)_p - (a1-b1)_m          S2xx = (a2-b2)_m + 4 a2_c + (a2+b2)_p.
// Every row of the lattice is written, fixed rows and columns with zeros.
struct Adj2DParams {
  int nx, ny;
  int64_t pitch;  // elements between rows
  int64_t plane;
  int xper, yper;
  int nseg, nband, nitems;
  int aligned;
};

template <class C, int KX>
__global__ __launch_bounds__(256) void adjoint_d2q9_fast(const typename C::elem* __restrict__ sn,
                                                         const typename C::T* __restrict__ bn1,
                                                         typename C::T* __restrict__ bn, Adj2DParams p,
                                                         double* __restrict__ gslots) {
#pragma clang fp contract(off)
  using T = typename C::T;
  constexpr int SW = 64 * KX;
  const int lane = threadIdx.x & 63;
  // XCD-aware numbering (workgroups go to the eight XCDs in turn): XCD k
  // takes a contiguous range of (segment, band) items, so neighbouring bands
  // share their boundary rows through its L2
  const int nblk = (int)gridDim.x, bid = (int)blockIdx.x;
  const int per = nblk >> 3, rem = nblk & 7, xcd = bid & 7;
  const int lblk = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int g = __builtin_amdgcn_readfirstlane(lblk * 4 + (int)(threadIdx.x >> 6));
  if (g >= p.nitems) return;
  const int seg = g % p.nseg, band = g / p.nseg;
  const int x0 = seg * SW;
  const int y0 = (int)((int64_t)band * p.ny / p.nband);
  const int y1 = (int)((int64_t)(band + 1) * p.ny / p.nband);
  const int xb = x0 + KX * lane;
  const bool wrap_dpp = p.xper && x0 == 0 && p.nx == SW;  // one segment spans a periodic row
  const bool vec = p.aligned && xb + KX <= p.nx;           // the lane's nodes are one vector
  // On a periodic axis the lanes past the end of the row read its first nodes
  // again, so that the last node's right neighbour is in the next lane (the
  // extent is a multiple of KX); they store nothing and add nothing to dL/dG.
  const int xw = p.xper ? xb % p.nx : xb;
  const bool vload = p.aligned && (p.xper || xb + KX <= p.nx);
  // the node beside the segment that lanes 0 and 63 read (wrapped on a
  // periodic axis; none beyond a fixed face)
  int hx = lane == 0 ? x0 - 1 : x0 + SW;
  if (p.xper) hx = ((hx % p.nx) + p.nx) % p.nx;
  const bool hok = !wrap_dpp && (lane == 0 || lane == 63) && hx >= 0 && hx < p.nx;
  bool node_in[KX];  // the lane's nodes that are nodes of the row (not wrapped copies)
#pragma unroll
  for (int e = 0; e < KX; ++e) node_in[e] = xb + e < p.nx;

  T P[KX], Mx[KX], My[KX];
  T hP = 0, hMx = 0, hMy = 0;  // node beside the segment (lanes 0 and 63)
  T ux[KX], uy[KX];            // u~ of the destination row that completes next
  auto load_row = [&](int r) {
    int rr = r;
    bool valid = true;
    if (r < 0 || r >= p.ny) {
      if (p.yper)
        rr = r < 0 ? r + p.ny : r - p.ny;
      else
        valid = false;
    }
#pragma unroll
    for (int e = 0; e < KX; ++e) P[e] = Mx[e] = My[e] = (T)0;
    hP = hMx = hMy = (T)0;
    if (!valid) return;  // outside a fixed face: nothing flows from there
    const int64_t rb = p.pitch * rr;
    if (vload) {
      using V = RowVecT<T, KX>;
      const V a = *reinterpret_cast<const V*>(bn1 + rb + xw);
      const V b = *reinterpret_cast<const V*>(bn1 + p.plane + rb + xw);
      const V c = *reinterpret_cast<const V*>(bn1 + 2 * p.plane + rb + xw);
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        P[e] = a.v[e];
        Mx[e] = b.v[e];
        My[e] = c.v[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        const int x = p.xper ? (xb + e) % p.nx : xb + e;
        if (x < p.nx) {
          P[e] = bn1[rb + x];
          Mx[e] = bn1[p.plane + rb + x];
          My[e] = bn1[2 * p.plane + rb + x];
        }
      }
    }
    if (hok) {
      hP = bn1[rb + hx];
      hMx = bn1[p.plane + rb + hx];
      hMy = bn1[2 * p.plane + rb + hx];
    }
  };
  auto load_u = [&](int j) {
    const int64_t rb = p.pitch * j;
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      int x = xb + e;
      x = x < p.nx ? x : p.nx - 1;  // lanes past a ragged end read a valid node
      ux[e] = C::dec(sn[p.plane + rb + x], 1);
      uy[e] = C::dec(sn[2 * p.plane + rb + x], 2);
    }
  };

  // pending destination rows: m-row sums (a-b) of row r-2 (for row r-1) and
  // of row r-1 (for row r); c-row values a of row r-1 (for row r-1)
  T m0[KX], m1[KX], m2[KX], n0[KX], n1[KX], n2[KX], c0[KX], c1[KX], c2[KX];
#pragma unroll
  for (int e = 0; e < KX; ++e) m0[e] = m1[e] = m2[e] = n0[e] = n1[e] = n2[e] = c0[e] = c1[e] = c2[e] = (T)0;
  double gx = 0, gy = 0;
  const T k36 = (T)(1.0 / 36.0);

  load_row(y0 - 1);
  for (int r = y0 - 1; r <= y1; ++r) {
    // x pass of source row r
    T a0[KX], a1[KX], a2[KX], b0[KX], b1[KX], b2[KX];
    {
      T inP = dpp_from_left(P[KX - 1]), inMx = dpp_from_left(Mx[KX - 1]), inMy = dpp_from_left(My[KX - 1]);
      T inPr = dpp_from_right(P[0]), inMxr = dpp_from_right(Mx[0]), inMyr = dpp_from_right(My[0]);
      if (!wrap_dpp && lane == 0) {
        inP = hP;
        inMx = hMx;
        inMy = hMy;
      }
      if (!wrap_dpp && lane == 63) {
        inPr = hP;
        inMxr = hMx;
        inMyr = hMy;
      }
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        const int el = e > 0 ? e - 1 : 0, er = e + 1 < KX ? e + 1 : KX - 1;
        const T PL = e == 0 ? inP : P[el], PR = e == KX - 1 ? inPr : P[er];
        const T XL = e == 0 ? inMx : Mx[el], XR = e == KX - 1 ? inMxr : Mx[er];
        const T YL = e == 0 ? inMy : My[el], YR = e == KX - 1 ? inMyr : My[er];
        const T sP = PL + PR, dX = XR - XL, sY = YL + YR;
        a2[e] = sP + dX;
        a0[e] = fma_t((T)4, P[e], a2[e]);
        a1[e] = (PR - PL) + (XR + XL);
        b0[e] = fma_t((T)4, My[e], sY);
        b1[e] = YR - YL;
        b2[e] = sY;
      }
    }
    if (r >= y0 && r < y1) {
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        if (node_in[e]) {
          gx += (double)Mx[e];
          gy += (double)My[e];
        }
      }
    }
    T vx[KX], vy[KX];
    const bool complete = r - 1 >= y0;
    if (complete) {
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        vx[e] = ux[e];
        vy[e] = uy[e];
      }
    }
    if (r < y1) {
      load_row(r + 1);
      if (r >= y0) load_u(r);  // destination row r completes after source row r + 1
    }
    if (complete) {
      const int j = r - 1;
      const int64_t rb = p.pitch * j;
      const bool row_fixed = !p.yper && (j == 0 || j == p.ny - 1);
      RowVecT<T, KX> oR, oX, oY;
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        const T pa0 = a0[e] + b0[e], pa1 = a1[e] + b1[e], pa2 = a2[e] + b2[e];
        const T S2yy = (m0[e] + pa0) * k36;
        const T S1y = (pa0 - m0[e]) * k36;
        const T S0 = fma_t((T)4, c0[e], m0[e] + pa0) * k36;
        const T S2xy = (pa1 - m1[e]) * k36;
        const T S1x = fma_t((T)4, c1[e], m1[e] + pa1) * k36;
        const T S2xx = fma_t((T)4, c2[e], m2[e] + pa2) * k36;
        const T u = vx[e], v = vy[e];
        const T uu = fma_t(u, u, v * v);
        const T su = fma_t(S2xx, u, S2xy * v), sv = fma_t(S2xy, u, S2yy * v);
        const T quad = fma_t(u, su, v * sv);
        const T R = fma_t(S0, fma_t((T)1.5, uu, (T)1), (T)-4.5 * quad);
        const T X = fma_t((T)3, S1x, fma_t((T)9, su, (T)-3 * u * S0));
        const T Y = fma_t((T)3, S1y, fma_t((T)9, sv, (T)-3 * v * S0));
        const int x = xb + e;
        const bool fixed = row_fixed || (!p.xper && (x == 0 || x == p.nx - 1));
        oR.v[e] = fixed ? (T)0 : R;
        oX.v[e] = fixed ? (T)0 : X;
        oY.v[e] = fixed ? (T)0 : Y;
      }
      if (vec) {
        *reinterpret_cast<RowVecT<T, KX>*>(bn + rb + xb) = oR;
        *reinterpret_cast<RowVecT<T, KX>*>(bn + p.plane + rb + xb) = oX;
        *reinterpret_cast<RowVecT<T, KX>*>(bn + 2 * p.plane + rb + xb) = oY;
      } else {
#pragma unroll
        for (int e = 0; e < KX; ++e) {
          const int x = xb + e;
          if (x < p.nx) {
            bn[rb + x] = oR.v[e];
            bn[p.plane + rb + x] = oX.v[e];
            bn[2 * p.plane + rb + x] = oY.v[e];
          }
        }
      }
    }
    // roll: row r becomes the c row of destination r and the m row of r + 1
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      m0[e] = n0[e];
      m1[e] = n1[e];
      m2[e] = n2[e];
      n0[e] = a0[e] - b0[e];
      n1[e] = a1[e] - b1[e];
      n2[e] = a2[e] - b2[e];
      c0[e] = a0[e];
      c1[e] = a1[e];
      c2[e] = a2[e];
    }
  }
  gx = wave_sum(gx);
  gy = wave_sum(gy);
  if (lane == 0) {
    gslots[(int64_t)g * 4 + 0] += gx;
    gslots[(int64_t)g * 4 + 1] += gy;
  }
}

// --------------------------------------------------------- seed and result
// Terminal adjoint for a loss with derivative dLdu (physical velocity, FP64,
// d planes of N): ubar = e dL/du, rhobar = 0, stored as Mbar = ubar / rho,
// Rbar = -Mbar . u~; zero at fixed nodes.
template <class C>
__global__ void adjoint_seed_kernel(const typename C::elem* __restrict__ sT, const double* __restrict__ dLdu,
                                    typename C::T* __restrict__ adj, StepParams p, int d, double e) {
  using T = typename C::T;
  const int64_t N = p.nx * p.ny * p.nz;
  for (int64_t di = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; di < N; di += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = di % p.nx, j = (di / p.nx) % p.ny, k = di / (p.nx * p.ny);
    const int64_t x = stored_index(di, p.nx, p.px);
    if (node_fixed(p, i, j, k)) {
      for (int c = 0; c <= d; ++c) adj[c * p.plane + x] = (T)0;
      continue;
    }
    const T inv = (T)1 / ((T)p.rho_ref + C::dec(sT[x], 0));
    T R = 0;
    for (int c = 0; c < d; ++c) {
      const T M = (T)(e * dLdu[c * N + di]) * inv;
      adj[(1 + c) * p.plane + x] = M;
      R -= M * C::dec(sT[(1 + c) * p.plane + x], 1 + c);
    }
    adj[x] = R;
  }
}

// dL/du0 = rho Mbar / e, dL/drho0 = Rbar + Mbar . u~ (FP64, SoA as the fields).
template <class C>
__global__ void adjoint_result_kernel(const typename C::elem* __restrict__ s0, const typename C::T* __restrict__ adj,
                                      double* __restrict__ dLdu, double* __restrict__ dLdrho, int64_t N,
                                      int64_t nx, int64_t px, int64_t plane, int d, double rho_ref, double e) {
  for (int64_t di = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; di < N; di += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = stored_index(di, nx, px);
    const double rho = rho_ref + (double)C::dec(s0[x], 0);
    double rb = (double)adj[x];
    for (int c = 0; c < d; ++c) {
      const double M = (double)adj[(1 + c) * plane + x];
      dLdu[c * N + di] = rho * M / e;
      rb += M * (double)C::dec(s0[(1 + c) * plane + x], 1 + c);
    }
    if (dLdrho) dLdrho[di] = rb;
  }
}

// Folds the slots in a fixed order: out[c] = sum_b slots[b][c].
__global__ __launch_bounds__(256) void adjoint_fold_kernel(const double* __restrict__ slots, int64_t nslots,
                                                           double* __restrict__ out) {
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = 0; c < 3; ++c) {
    double v = 0;
    for (int64_t b = threadIdx.x; b < nslots; b += blockDim.x) v += slots[b * 4 + c];
    v = wave_sum(v);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) out[threadIdx.x] = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) +
                                          red[threadIdx.x][3];
}

// Clears FP64 accumulators with a kernel (no memset node when captured).
__global__ void zero_doubles_kernel(double* __restrict__ dst, int64_t count) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += (int64_t)gridDim.x * blockDim.x)
    dst[x] = 0.0;
}

// ---------------------------------------------------------------- launchers
int64_t adjoint_slots(const Layout& L) {
  // the generic kernel's workgroups; the fast D2Q9 kernel uses at most
  // ceil(nx/64) x ceil(ny/4) wavefronts
  return ((L.nx + 63) / 64) * ((L.ny + 3) / 4) * L.nz;
}

template <class F>
static hipError_t by_codec(int precision, F&& go) {
  switch (precision) {
    case MACLAB_FP64: return go(CodecF64{});
    case MACLAB_FP32: return go(CodecF32{});
    case MACLAB_HILO: return go(CodecHILO{});
    case MACLAB_S16: return go(CodecS16{});
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_step(const Layout& L, const void* sn, const void* an1, void* an, const StepParams& p,
                               double* gslots, hipStream_t s) {
  const dim3 block(64, 4, 1);
  const dim3 grid((unsigned)((L.nx + 63) / 64), (unsigned)((L.ny + 3) / 4), (unsigned)L.nz);
  return by_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    using E = typename C::elem;
    using T = typename C::T;
    if (L.q == 9)
      hipLaunchKernelGGL((adjoint_generic_kernel<9, C>), grid, block, 0, s, (const E*)sn, (const T*)an1, (T*)an, p,
                         gslots);
    else
      hipLaunchKernelGGL((adjoint_generic_kernel<19, C>), grid, block, 0, s, (const E*)sn, (const T*)an1, (T*)an,
                         p, gslots);
    return hipGetLastError();
  });
}

bool adjoint2d_supported(const Layout& L, const StepParams& p) {
  return L.q == 9 && L.ny >= 3 && L.nx >= (p.fixed[0] ? 3 : 1);
}

bool adjoint2d_shape_valid(const Layout& L, const StepParams& p, const Fast2DShape& sh) {
  if (!adjoint2d_supported(L, p) || (sh.kx != 1 && sh.kx != 2) || sh.nband < 1) return false;
  if (sh.nband > (L.ny + 3) / 4) return false;  // slot budget, and at least ~4 rows per band
  if (!p.fixed[0] && L.nx % sh.kx != 0) return false;  // a periodic wrap may not split a lane's nodes
  return true;
}

Fast2DShape adjoint2d_default_shape(const Layout& L, const StepParams& p, int cus) {
  Fast2DShape sh;
  sh.kx = L.nx >= 128 ? 2 : 1;
  while (!p.fixed[0] && L.nx % sh.kx != 0) sh.kx /= 2;
  const int nseg = (int)((L.nx + 64 * sh.kx - 1) / (64 * sh.kx));
  int nband = (8 * cus + nseg - 1) / nseg;
  const int maxb = (int)((L.ny + 3) / 4);
  sh.nband = nband > maxb ? maxb : (nband < 1 ? 1 : nband);
  return sh;
}

hipError_t launch_adjoint_fast2d(const Layout& L, const void* sn, const void* an1, void* an, const StepParams& p,
                                 const Fast2DShape& sh, double* gslots, hipStream_t s) {
  if (!adjoint2d_shape_valid(L, p, sh)) return hipErrorInvalidValue;
  Adj2DParams ap{};
  ap.nx = (int)L.nx;
  ap.ny = (int)L.ny;
  ap.pitch = L.px;
  ap.plane = L.plane;
  ap.xper = !p.fixed[0];
  ap.yper = !p.fixed[1];
  ap.nseg = (int)((L.nx + 64 * sh.kx - 1) / (64 * sh.kx));
  ap.nband = sh.nband;
  ap.nitems = ap.nseg * ap.nband;
  ap.aligned = (L.px % sh.kx) == 0;
  const unsigned blocks = (unsigned)((ap.nitems + 3) / 4);
  return by_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    using E = typename C::elem;
    using T = typename C::T;
    if (sh.kx == 1)
      hipLaunchKernelGGL((adjoint_d2q9_fast<C, 1>), dim3(blocks), dim3(256), 0, s, (const E*)sn, (const T*)an1,
                         (T*)an, ap, gslots);
    else
      hipLaunchKernelGGL((adjoint_d2q9_fast<C, 2>), dim3(blocks), dim3(256), 0, s, (const E*)sn, (const T*)an1,
                         (T*)an, ap, gslots);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_seed(const Layout& L, const void* sT, const double* dLdu, void* adj, const StepParams& p,
                               double e, hipStream_t s) {
  const unsigned blocks = blocks_256(L.N);
  return by_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL(adjoint_seed_kernel<C>, dim3(blocks), dim3(256), 0, s, (const typename C::elem*)sT, dLdu,
                       (typename C::T*)adj, p, L.d, e);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_result(const Layout& L, const void* s0, const void* adj, double* dLdu, double* dLdrho,
                                 double rho_ref, double e, hipStream_t s) {
  const unsigned blocks = blocks_256(L.N);
  return by_codec(L.precision, [&](auto codec) {
    using C = decltype(codec);
    hipLaunchKernelGGL(adjoint_result_kernel<C>, dim3(blocks), dim3(256), 0, s, (const typename C::elem*)s0,
                       (const typename C::T*)adj, dLdu, dLdrho, L.N, L.nx, L.px, L.plane, L.d, rho_ref, e);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_fold(const double* slots, int64_t nslots, double* out, hipStream_t s) {
  hipLaunchKernelGGL(adjoint_fold_kernel, dim3(1), dim3(256), 0, s, slots, nslots, out);
  return hipGetLastError();
}

hipError_t launch_zero_doubles(double* dst, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(blocks_256(count)), dim3(256), 0, s, dst, count);
  return hipGetLastError();
}

}  // namespace maclab
