// Fast D3Q19 MacLAB step for gfx950 (lattices whose x extent is 64, 128 or
// 256 nodes; FP32 arithmetic; FP32, split-bf16 or scaled-binary16 storage).
//
// Work decomposition
//  - A wavefront owns one whole x-row: lane l holds the KX = nx/64 nodes
//    x = KX*l .. KX*l + KX-1, so every field row is one coalesced vector load.
//  - A workgroup is W output rows (y) plus one halo row on each side, one
//    wavefront per row, marching in z over a chunk of planes (2.5-D blocking).
//  - Each node computes the equilibria of its 19 links once (Eq. (2), in the
//    deviation form F^_a = f_eq_a - w_a rho_ref, scaled by 36) and pushes them
//    to the node x + c_a:
//      * links with c_y = 0 stay in the wavefront: the x shift is an in-lane
//        register move or a DPP wave rotate (wave_ror / wave_rol) across lanes;
//        the z shift is a rolling set of three plane accumulators;
//      * links with c_y = +-1 go through LDS to the neighbouring row's
//        wavefront, which reads them at x, x-1 or x+1.
//  - After source plane z is pushed, destination plane z-1 holds the full
//    gathers of Eqs. (4)-(5) and is finalised: rho' = rho_ref + drho',
//    u~' = (m' + g) / rho', and stored (fixed nodes are skipped).
//  - Workgroups are numbered so that each XCD gets a contiguous band of tiles
//    (neighbouring tiles share halo rows through that XCD's L2).
#include "internal.h"

namespace maclab {

struct Fast3DParams {
  int ny, nz;
  int ylo, yhi, zlo, zhi;  // output rows / planes, inclusive
  int yper, zper, xwall;
  int zc;                  // output planes per workgroup
  int nyb, nblocks;        // workgroups along y, total
  int64_t plane;           // elements per field plane
  float rho_ref, gx, gy, gz;
  uint64_t seed, step;
};

// ----------------------------------------------------------- row load/store
template <class C, int KX>
struct alignas(sizeof(typename C::elem) * KX) RowVec {
  typename C::elem v[KX];
};

template <class C, int KX>
__device__ __forceinline__ void load_row(const typename C::elem* __restrict__ p, int field, float (&out)[KX]) {
  const RowVec<C, KX> r = *reinterpret_cast<const RowVec<C, KX>*>(p);
#pragma unroll
  for (int e = 0; e < KX; ++e) out[e] = (float)C::dec(r.v[e], field);
}

template <class C, int KX>
__device__ __forceinline__ typename C::elem enc_one(float v, int field, int64_t node, const Fast3DParams& p) {
  uint32_t r = 0;
  if constexpr (needs_rng<C>::value) r = sr_bits(p.seed, p.step, node, field);
  return C::enc(v, field, r);
}

// Stores one row of one field; with x walls the first node of lane 0 and the
// last node of lane 63 (the wall nodes) are left untouched.
template <class C, int KX>
__device__ __forceinline__ void store_row(typename C::elem* __restrict__ p, int field, const float (&v)[KX],
                                          int64_t node0, int lane, bool xwall, const Fast3DParams& pr) {
  RowVec<C, KX> r;
#pragma unroll
  for (int e = 0; e < KX; ++e) r.v[e] = enc_one<C, KX>(v[e], field, node0 + e, pr);
  if (xwall && (lane == 0 || lane == 63)) {
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      const bool wall = (lane == 0 && e == 0) || (lane == 63 && e == KX - 1);
      if (!wall) p[e] = r.v[e];
    }
  } else {
    *reinterpret_cast<RowVec<C, KX>*>(p) = r;
  }
}

// Lane l receives the value of lane l-1 (lane 0 that of lane 63).
__device__ __forceinline__ float from_left_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C, 0xF, 0xF, false));
}
// Lane l receives the value of lane l+1 (lane 63 that of lane 0).
__device__ __forceinline__ float from_right_lane(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, false));
}

template <int KX>
struct PlaneAcc {
  float r[KX], mx[KX], my[KX], mz[KX];  // 36 * (drho', m')
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int e = 0; e < KX; ++e) r[e] = mx[e] = my[e] = mz[e] = 0.f;
  }
};

// Pushes one source row (the KX nodes of this lane) into the three plane
// accumulators of this wavefront and into this wavefront's LDS rows.
// acc_m: destination plane z-1, acc_c: plane z, acc_p: plane z+1.
template <int KX>
__device__ __forceinline__ void push_row(const float (&dr)[KX], const float (&ux)[KX], const float (&uy)[KX],
                                         const float (&uz)[KX], float rho_ref, PlaneAcc<KX>& acc_m,
                                         PlaneAcc<KX>& acc_c, PlaneAcc<KX>& acc_p, float* __restrict__ up,
                                         float* __restrict__ dn, int lane) {
  constexpr int NX = 64 * KX;
  // values leaving the lane through its right / left edge
  float out_r0 = 0.f, out_r1 = 0.f, out_r2 = 0.f;  // (1,0,0), (1,0,1), (1,0,-1) of the last node
  float out_l0 = 0.f, out_l1 = 0.f, out_l2 = 0.f;  // (-1,0,0), (-1,0,1), (-1,0,-1) of the first node
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    // equilibria of the 19 links, times 36, in deviation form (Eq. (2))
    const float rho = rho_ref + dr[e];
    const float tx = 3.f * ux[e], ty = 3.f * uy[e], tz = 3.f * uz[e];
    const float bx = rho * tx, by = rho * ty, bz = rho * tz;  // 3 rho u
    const float qxx = 0.5f * bx * tx, qyy = 0.5f * by * ty, qzz = 0.5f * bz * tz;  // 4.5 rho u_i^2
    const float qxy = bx * ty, qxz = bx * tz, qyz = by * tz;                      // 9 rho u_i u_j
    const float a = dr[e] - (qxx + qyy + qzz) * (1.f / 3.f);                       // drho - 1.5 rho |u|^2
    const float sx = a + qxx, sy = a + qyy, sz = a + qzz;
    const float f0 = 12.f * a;
    const float fxp = 2.f * (sx + bx), fxm = 2.f * (sx - bx);
    const float fyp = 2.f * (sy + by), fym = 2.f * (sy - by);
    const float fzp = 2.f * (sz + bz), fzm = 2.f * (sz - bz);
    float p, m, u, v;
    // xy edges
    p = sx + qyy + qxy; m = sx + qyy - qxy; u = bx + by; v = bx - by;
    const float f_pp0 = p + u, f_mm0 = p - u, f_pm0 = m + v, f_mp0 = m - v;
    // xz edges
    p = sx + qzz + qxz; m = sx + qzz - qxz; u = bx + bz; v = bx - bz;
    const float f_p0p = p + u, f_m0m = p - u, f_p0m = m + v, f_m0p = m - v;
    // yz edges
    p = sy + qzz + qyz; m = sy + qzz - qyz; u = by + bz; v = by - bz;
    const float f_0pp = p + u, f_0mm = p - u, f_0pm = m + v, f_0mp = m - v;

    // c_y = 0 links: plane z (rest, +-x), plane z+1 (+z, +-x+z), plane z-1
    acc_c.r[e] += f0;
    const float tzp = fzp, tzm = fzm;
    acc_p.r[e] += tzp;
    acc_p.mz[e] += tzp;
    acc_m.r[e] += tzm;
    acc_m.mz[e] -= tzm;
    if (e + 1 < KX) {
      acc_c.r[e + 1] += fxp;
      acc_c.mx[e + 1] += fxp;
      acc_p.r[e + 1] += f_p0p;
      acc_p.mx[e + 1] += f_p0p;
      acc_p.mz[e + 1] += f_p0p;
      acc_m.r[e + 1] += f_p0m;
      acc_m.mx[e + 1] += f_p0m;
      acc_m.mz[e + 1] -= f_p0m;
    } else {
      out_r0 = fxp;
      out_r1 = f_p0p;
      out_r2 = f_p0m;
    }
    if (e > 0) {
      acc_c.r[e - 1] += fxm;
      acc_c.mx[e - 1] -= fxm;
      acc_p.r[e - 1] += f_m0p;
      acc_p.mx[e - 1] -= f_m0p;
      acc_p.mz[e - 1] += f_m0p;
      acc_m.r[e - 1] += f_m0m;
      acc_m.mx[e - 1] -= f_m0m;
      acc_m.mz[e - 1] -= f_m0m;
    } else {
      out_l0 = fxm;
      out_l1 = f_m0p;
      out_l2 = f_m0m;
    }
    // c_y = +1 links to the next row, c_y = -1 links to the previous row;
    // LDS rows are stored transposed (node KX*l + e at e*64 + l) so that a
    // wavefront touches 64 consecutive words
    const int x = e * 64 + lane;
    up[0 * NX + x] = fyp;
    up[1 * NX + x] = f_pp0;
    up[2 * NX + x] = f_mp0;
    up[3 * NX + x] = f_0pp;
    up[4 * NX + x] = f_0pm;
    dn[0 * NX + x] = fym;
    dn[1 * NX + x] = f_pm0;
    dn[2 * NX + x] = f_mm0;
    dn[3 * NX + x] = f_0mp;
    dn[4 * NX + x] = f_0mm;
  }
  // cross-lane x shifts: the last node's +x links enter the next lane's first
  // node, the first node's -x links enter the previous lane's last node
  const float in_r0 = from_left_lane(out_r0), in_r1 = from_left_lane(out_r1), in_r2 = from_left_lane(out_r2);
  const float in_l0 = from_right_lane(out_l0), in_l1 = from_right_lane(out_l1), in_l2 = from_right_lane(out_l2);
  acc_c.r[0] += in_r0;
  acc_c.mx[0] += in_r0;
  acc_p.r[0] += in_r1;
  acc_p.mx[0] += in_r1;
  acc_p.mz[0] += in_r1;
  acc_m.r[0] += in_r2;
  acc_m.mx[0] += in_r2;
  acc_m.mz[0] -= in_r2;
  acc_c.r[KX - 1] += in_l0;
  acc_c.mx[KX - 1] -= in_l0;
  acc_p.r[KX - 1] += in_l1;
  acc_p.mx[KX - 1] -= in_l1;
  acc_p.mz[KX - 1] += in_l1;
  acc_m.r[KX - 1] += in_l2;
  acc_m.mx[KX - 1] -= in_l2;
  acc_m.mz[KX - 1] -= in_l2;
}

// Adds the c_y = +-1 links arriving from the rows below (`from_below`, sent
// with c_y = +1) and above (`from_above`, c_y = -1).
template <int KX>
__device__ __forceinline__ void pull_rows(const float* __restrict__ from_below, const float* __restrict__ from_above,
                                          PlaneAcc<KX>& acc_m, PlaneAcc<KX>& acc_c, PlaneAcc<KX>& acc_p,
                                          int lane) {
  constexpr int NX = 64 * KX;
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    // transposed positions of nodes x, x-1 and x+1 (periodic across the row)
    const int x = e * 64 + lane;
    const int xl = e > 0 ? (e - 1) * 64 + lane : (KX - 1) * 64 + ((lane + 63) & 63);
    const int xr = e < KX - 1 ? (e + 1) * 64 + lane : ((lane + 1) & 63);
    const float a0 = from_below[0 * NX + x], a1 = from_below[1 * NX + xl], a2 = from_below[2 * NX + xr];
    const float a3 = from_below[3 * NX + x], a4 = from_below[4 * NX + x];
    const float b0 = from_above[0 * NX + x], b1 = from_above[1 * NX + xl], b2 = from_above[2 * NX + xr];
    const float b3 = from_above[3 * NX + x], b4 = from_above[4 * NX + x];
    const float sa = a0 + a1 + a2, sb = b0 + b1 + b2;
    acc_c.r[e] += sa + sb;
    acc_c.my[e] += sa - sb;
    acc_c.mx[e] += (a1 - a2) + (b1 - b2);
    const float s3 = a3 + b3, s4 = a4 + b4;
    acc_p.r[e] += s3;
    acc_p.mz[e] += s3;
    acc_p.my[e] += a3 - b3;
    acc_m.r[e] += s4;
    acc_m.mz[e] -= s4;
    acc_m.my[e] += a4 - b4;
  }
}

template <class C, int KX, int W>
__global__ __launch_bounds__(64 * (W + 2)) void step_d3q19_fast(const typename C::elem* __restrict__ src,
                                                               typename C::elem* __restrict__ dst, Fast3DParams p) {
  constexpr int NX = 64 * KX;
  constexpr int ROWS = W + 2;
  __shared__ float lds[2 * ROWS * 5 * NX];
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  float* up = lds + wv * 5 * NX;               // this wave's c_y = +1 links
  float* dn = lds + (ROWS + wv) * 5 * NX;      // this wave's c_y = -1 links
  const float* from_below = lds + (wv > 0 ? wv - 1 : 0) * 5 * NX;
  const float* from_above = lds + (ROWS + (wv + 1 < ROWS ? wv + 1 : wv)) * 5 * NX;

  // XCD-aware tile numbering: XCD k (= blockIdx.x mod 8) gets a contiguous band
  const int bid = blockIdx.x;
  const int per = p.nblocks >> 3, rem = p.nblocks & 7, xcd = bid & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int by = tile % p.nyb, bz = tile / p.nyb;

  const int y0 = p.ylo + by * W;
  int yrow = y0 - 1 + wv;
  const bool out_row = wv >= 1 && wv <= W && yrow <= p.yhi;
  if (p.yper)
    yrow = (yrow % p.ny + p.ny) % p.ny;
  else
    yrow = yrow < 0 ? 0 : (yrow > p.ny - 1 ? p.ny - 1 : yrow);
  const int z0 = p.zlo + bz * p.zc;
  const int z1 = min(z0 + p.zc, p.zhi + 1);  // output planes [z0, z1)
  const int xbase = lane * KX;
  const int64_t nx = NX;
  const int64_t plane = p.plane;

  float dr[KX], ux[KX], uy[KX], uz[KX];
  auto zwrap = [&](int z) { return p.zper ? (z + p.nz) % p.nz : z; };
  auto load_plane = [&](int z) {
    const int64_t base = nx * ((int64_t)yrow + (int64_t)p.ny * zwrap(z)) + xbase;
    load_row<C, KX>(src + base, 0, dr);
    load_row<C, KX>(src + plane + base, 1, ux);
    load_row<C, KX>(src + 2 * plane + base, 2, uy);
    load_row<C, KX>(src + 3 * plane + base, 3, uz);
  };

  // One source plane: push its links, exchange the c_y = +-1 links through
  // LDS, then finalise destination plane zs-1. am / ac / ap are the
  // accumulators of destination planes zs-1, zs, zs+1.
  auto source_plane = [&](int zs, PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
    push_row<KX>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    if (zs < z1) load_plane(zs + 1);  // prefetch the next source plane
    __syncthreads();
    if (out_row) pull_rows<KX>(from_below, from_above, am, ac, ap, lane);
    __syncthreads();
    const int zd = zs - 1;
    if (out_row && zd >= z0) {
      float r[KX], vx[KX], vy[KX], vz[KX];
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        const float drn = am.r[e] * (1.f / 36.f);
        const float inv = __builtin_amdgcn_rcpf(p.rho_ref + drn);  // v_rcp_f32, 1 ulp
        r[e] = drn;
        vx[e] = (am.mx[e] * (1.f / 36.f) + p.gx) * inv;
        vy[e] = (am.my[e] * (1.f / 36.f) + p.gy) * inv;
        vz[e] = (am.mz[e] * (1.f / 36.f) + p.gz) * inv;
      }
      const int64_t node0 = nx * ((int64_t)yrow + (int64_t)p.ny * zwrap(zd)) + xbase;
      store_row<C, KX>(dst + node0, 0, r, node0, lane, p.xwall, p);
      store_row<C, KX>(dst + plane + node0, 1, vx, node0, lane, p.xwall, p);
      store_row<C, KX>(dst + 2 * plane + node0, 2, vy, node0, lane, p.xwall, p);
      store_row<C, KX>(dst + 3 * plane + node0, 3, vz, node0, lane, p.xwall, p);
    }
    am.zero();  // becomes destination plane zs+2
  };

  // source planes z0-1 .. z1, three at a time so the accumulator roles
  // rotate at compile time
  PlaneAcc<KX> a0, a1, a2;
  a0.zero();
  a1.zero();
  a2.zero();
  load_plane(z0 - 1);
  for (int zs = z0 - 1; zs <= z1; zs += 3) {
    source_plane(zs, a0, a1, a2);
    if (zs + 1 > z1) break;
    source_plane(zs + 1, a1, a2, a0);
    if (zs + 2 > z1) break;
    source_plane(zs + 2, a2, a0, a1);
  }
}

// ------------------------------------------------------------------ launch
constexpr int kFastW = 6;     // output rows per workgroup
constexpr int kFastZc = 32;   // output planes per workgroup

bool fast_step_supported(const Layout& L, const StepParams& p) {
  if (L.q != 19) return false;
  if (L.precision != MACLAB_FP32 && L.precision != MACLAB_HILO && L.precision != MACLAB_S16) return false;
  if (L.nx != 64 && L.nx != 128 && L.nx != 256) return false;
  if (L.ny < 3 || L.nz < 3) return false;
  (void)p;
  return true;
}

template <class C, int KX>
static hipError_t launch_fast_kx(const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  const dim3 block(64, kFastW + 2, 1);
  hipLaunchKernelGGL((step_d3q19_fast<C, KX, kFastW>), dim3(fp.nblocks), block, 0, s, (const E*)src, (E*)dst, fp);
  return hipGetLastError();
}

template <class C>
static hipError_t launch_fast_codec(const Layout& L, const void* src, void* dst, const Fast3DParams& fp,
                                    hipStream_t s) {
  switch (L.nx) {
    case 64: return launch_fast_kx<C, 1>(src, dst, fp, s);
    case 128: return launch_fast_kx<C, 2>(src, dst, fp, s);
    case 256: return launch_fast_kx<C, 4>(src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_fast(const Layout& L, const void* src, void* dst, const StepParams& p, hipStream_t s) {
  Fast3DParams fp;
  fp.ny = (int)L.ny;
  fp.nz = (int)L.nz;
  fp.yper = !p.fixed[1];
  fp.zper = !p.fixed[2];
  fp.xwall = p.fixed[0];
  fp.ylo = fp.yper ? 0 : 1;
  fp.yhi = fp.yper ? fp.ny - 1 : fp.ny - 2;
  fp.zlo = fp.zper ? 0 : 1;
  fp.zhi = fp.zper ? fp.nz - 1 : fp.nz - 2;
  fp.zc = kFastZc;
  fp.nyb = (fp.yhi - fp.ylo + 1 + kFastW - 1) / kFastW;
  const int nzb = (fp.zhi - fp.zlo + 1 + kFastZc - 1) / kFastZc;
  fp.nblocks = fp.nyb * nzb;
  fp.plane = L.plane;
  fp.rho_ref = (float)p.rho_ref;
  fp.gx = (float)p.g[0];
  fp.gy = (float)p.g[1];
  fp.gz = (float)p.g[2];
  fp.seed = p.seed;
  fp.step = p.step;
  switch (L.precision) {
    case MACLAB_FP32: return launch_fast_codec<CodecF32>(L, src, dst, fp, s);
    case MACLAB_HILO: return launch_fast_codec<CodecHILO>(L, src, dst, fp, s);
    case MACLAB_S16: return launch_fast_codec<CodecS16>(L, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace maclab
