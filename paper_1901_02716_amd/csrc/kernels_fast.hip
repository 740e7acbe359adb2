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
  int ylo, nyo;            // first output row, number of output rows
  int zlo, nzo;            // first output plane, number of output planes
  int yper, zper, xwall;
  int nyb, nzb, nblocks;   // workgroups along y and z, total
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
    // the new state is not read again in this step: stream it past the caches
    constexpr int B = (int)sizeof(RowVec<C, KX>);
    if constexpr (B == 16) {
      typedef uint32_t w4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(__builtin_bit_cast(w4, r), reinterpret_cast<w4*>(p));
    } else if constexpr (B == 8) {
      typedef uint32_t w2 __attribute__((ext_vector_type(2)));
      __builtin_nontemporal_store(__builtin_bit_cast(w2, r), reinterpret_cast<w2*>(p));
    } else if constexpr (B == 4) {
      __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, r), reinterpret_cast<uint32_t*>(p));
    } else {
      *reinterpret_cast<RowVec<C, KX>*>(p) = r;
    }
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
// MODE 0: an output row (everything); MODE 1: the halo row below the tile
// (only its c_y = +1 links are needed); MODE 2: the halo row above (c_y = -1).
// Floating-point contraction is off and every FMA is written out, so a link
// value has the same bits whichever wavefront (output or halo) computes it,
// and the result does not depend on the tiling.
template <int KX, int MODE>
__device__ __forceinline__ void push_row(const float (&dr)[KX], const float (&ux)[KX], const float (&uy)[KX],
                                         const float (&uz)[KX], float rho_ref, PlaneAcc<KX>& acc_m,
                                         PlaneAcc<KX>& acc_c, PlaneAcc<KX>& acc_p, float* __restrict__ up,
                                         float* __restrict__ dn, int lane) {
#pragma clang fp contract(off)
  constexpr int NX = 64 * KX;
  // values leaving the lane through its right / left edge (axis links are
  // carried as halves: the link value is twice the carried number)
  float out_r0 = 0.f, out_r1 = 0.f, out_r2 = 0.f;  // (1,0,0)/2, (1,0,1), (1,0,-1) of the last node
  float out_l0 = 0.f, out_l1 = 0.f, out_l2 = 0.f;  // (-1,0,0)/2, (-1,0,1), (-1,0,-1) of the first node
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    // equilibria of the 19 links, times 36, in deviation form (Eq. (2)):
    // 36 F^_a = wnum_a [a + c.b + sum_i c_i^2 q_ii + sum_{i<j} c_i c_j q_ij]
    const float rho = rho_ref + dr[e];
    const float tx = 3.f * ux[e], ty = 3.f * uy[e], tz = 3.f * uz[e];
    const float bx = rho * tx, by = rho * ty, bz = rho * tz;                      // 3 rho u
    const float qxx = bx * (1.5f * ux[e]), qyy = by * (1.5f * uy[e]), qzz = bz * (1.5f * uz[e]);  // 4.5 rho u_i^2
    const float qxy = bx * ty, qxz = bx * tz, qyz = by * tz;                      // 9 rho u_i u_j
    const float a = __builtin_fmaf(qxx + qyy + qzz, -1.f / 3.f, dr[e]);           // drho - 1.5 rho |u|^2
    const float sx = a + qxx, sy = a + qyy, sz = a + qzz;
    const float f0 = 12.f * a;
    // axis links, halved: 36 F^ = 2 (s_i +- b_i)
    const float hxp = sx + bx, hxm = sx - bx;
    const float hyp = sy + by, hym = sy - by;
    const float hzp = sz + bz, hzm = sz - bz;
    float p, m, u, v;
    // xy edges
    p = (sx + qyy) + qxy; m = (sx + qyy) - qxy; u = bx + by; v = bx - by;
    const float f_pp0 = p + u, f_mm0 = p - u, f_pm0 = m + v, f_mp0 = m - v;
    // xz edges
    p = (sx + qzz) + qxz; m = (sx + qzz) - qxz; u = bx + bz; v = bx - bz;
    const float f_p0p = p + u, f_m0m = p - u, f_p0m = m + v, f_m0p = m - v;
    // yz edges
    p = (sy + qzz) + qyz; m = (sy + qzz) - qyz; u = by + bz; v = by - bz;
    const float f_0pp = p + u, f_0mm = p - u, f_0pm = m + v, f_0mp = m - v;

    if constexpr (MODE == 0) {
      // c_y = 0 links: plane z (rest, +-x), plane z+1 (+z, +-x+z), plane z-1
      acc_c.r[e] += f0;
      acc_p.r[e] = __builtin_fmaf(2.f, hzp, acc_p.r[e]);
      acc_p.mz[e] = __builtin_fmaf(2.f, hzp, acc_p.mz[e]);
      acc_m.r[e] = __builtin_fmaf(2.f, hzm, acc_m.r[e]);
      acc_m.mz[e] = __builtin_fmaf(-2.f, hzm, acc_m.mz[e]);
      if (e + 1 < KX) {
        acc_c.r[e + 1] = __builtin_fmaf(2.f, hxp, acc_c.r[e + 1]);
        acc_c.mx[e + 1] = __builtin_fmaf(2.f, hxp, acc_c.mx[e + 1]);
        acc_p.r[e + 1] += f_p0p;
        acc_p.mx[e + 1] += f_p0p;
        acc_p.mz[e + 1] += f_p0p;
        acc_m.r[e + 1] += f_p0m;
        acc_m.mx[e + 1] += f_p0m;
        acc_m.mz[e + 1] -= f_p0m;
      } else {
        out_r0 = hxp;
        out_r1 = f_p0p;
        out_r2 = f_p0m;
      }
      if (e > 0) {
        acc_c.r[e - 1] = __builtin_fmaf(2.f, hxm, acc_c.r[e - 1]);
        acc_c.mx[e - 1] = __builtin_fmaf(-2.f, hxm, acc_c.mx[e - 1]);
        acc_p.r[e - 1] += f_m0p;
        acc_p.mx[e - 1] -= f_m0p;
        acc_p.mz[e - 1] += f_m0p;
        acc_m.r[e - 1] += f_m0m;
        acc_m.mx[e - 1] -= f_m0m;
        acc_m.mz[e - 1] -= f_m0m;
      } else {
        out_l0 = hxm;
        out_l1 = f_m0p;
        out_l2 = f_m0m;
      }
    }
    // c_y = +1 links to the next row, c_y = -1 links to the previous row
    // (the axis link halved); LDS rows are stored transposed (node KX*l + e
    // at e*64 + l) so that a wavefront touches 64 consecutive words
    const int x = e * 64 + lane;
    if constexpr (MODE != 2) {
      up[0 * NX + x] = hyp;
      up[1 * NX + x] = f_pp0;
      up[2 * NX + x] = f_mp0;
      up[3 * NX + x] = f_0pp;
      up[4 * NX + x] = f_0pm;
    }
    if constexpr (MODE != 1) {
      dn[0 * NX + x] = hym;
      dn[1 * NX + x] = f_pm0;
      dn[2 * NX + x] = f_mm0;
      dn[3 * NX + x] = f_0mp;
      dn[4 * NX + x] = f_0mm;
    }
  }
  if constexpr (MODE != 0) return;
  // cross-lane x shifts: the last node's +x links enter the next lane's first
  // node, the first node's -x links enter the previous lane's last node
  const float in_r0 = from_left_lane(out_r0), in_r1 = from_left_lane(out_r1), in_r2 = from_left_lane(out_r2);
  const float in_l0 = from_right_lane(out_l0), in_l1 = from_right_lane(out_l1), in_l2 = from_right_lane(out_l2);
  acc_c.r[0] = __builtin_fmaf(2.f, in_r0, acc_c.r[0]);
  acc_c.mx[0] = __builtin_fmaf(2.f, in_r0, acc_c.mx[0]);
  acc_p.r[0] += in_r1;
  acc_p.mx[0] += in_r1;
  acc_p.mz[0] += in_r1;
  acc_m.r[0] += in_r2;
  acc_m.mx[0] += in_r2;
  acc_m.mz[0] -= in_r2;
  acc_c.r[KX - 1] = __builtin_fmaf(2.f, in_l0, acc_c.r[KX - 1]);
  acc_c.mx[KX - 1] = __builtin_fmaf(-2.f, in_l0, acc_c.mx[KX - 1]);
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
#pragma clang fp contract(off)
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
    const float sa = __builtin_fmaf(2.f, a0, a1 + a2), sb = __builtin_fmaf(2.f, b0, b1 + b2);
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
  (void)W;

  // XCD-aware tile numbering: XCD k (= blockIdx.x mod 8) gets a contiguous band
  const int bid = blockIdx.x;
  const int per = p.nblocks >> 3, rem = p.nblocks & 7, xcd = bid & 7;
  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int by = tile % p.nyb, bz = tile / p.nyb;

  // balanced ranges: block (by, bz) owns output rows [y0, y1) and planes [z0, z1)
  const int y0 = p.ylo + (int)((int64_t)by * p.nyo / p.nyb);
  const int y1 = p.ylo + (int)((int64_t)(by + 1) * p.nyo / p.nyb);
  const int z0 = p.zlo + (int)((int64_t)bz * p.nzo / p.nzb);
  const int z1 = p.zlo + (int)((int64_t)(bz + 1) * p.nzo / p.nzb);
  const int rows = y1 - y0;  // <= W
  // wave 0: halo row y0-1; waves 1..rows: output rows; wave rows+1: halo row
  // y1; any further waves idle (they only join the barriers)
  const int mode = wv == 0 ? 1 : (wv <= rows ? 0 : (wv == rows + 1 ? 2 : 3));
  const bool out_row = mode == 0;
  int yrow = y0 - 1 + wv;
  if (p.yper)
    yrow = (yrow % p.ny + p.ny) % p.ny;
  else
    yrow = yrow < 0 ? 0 : (yrow > p.ny - 1 ? p.ny - 1 : yrow);
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
    if (mode == 0)
      push_row<KX, 0>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    else if (mode == 1)
      push_row<KX, 1>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    else if (mode == 2)
      push_row<KX, 2>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    if (zs < z1 && mode != 3) load_plane(zs + 1);  // prefetch the next source plane
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
        vx[e] = __builtin_fmaf(am.mx[e], 1.f / 36.f, p.gx) * inv;
        vy[e] = __builtin_fmaf(am.my[e], 1.f / 36.f, p.gy) * inv;
        vz[e] = __builtin_fmaf(am.mz[e], 1.f / 36.f, p.gz) * inv;
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
  if (mode != 3) load_plane(z0 - 1);
  for (int zs = z0 - 1; zs <= z1; zs += 3) {
    source_plane(zs, a0, a1, a2);
    if (zs + 1 > z1) break;
    source_plane(zs + 1, a1, a2, a0);
    if (zs + 2 > z1) break;
    source_plane(zs + 2, a2, a0, a1);
  }
}

// ------------------------------------------------------------------ launch
static const int kFastW[] = {4, 6, 8, 10, 12};

bool fast_step_supported(const Layout& L, const StepParams& p) {
  if (L.q != 19) return false;
  if (L.precision != MACLAB_FP32 && L.precision != MACLAB_HILO && L.precision != MACLAB_S16) return false;
  if (L.nx != 64 && L.nx != 128 && L.nx != 256) return false;
  if (L.ny < 3 || L.nz < 3) return false;
  (void)p;
  return true;
}

static void output_ranges(const Layout& L, const StepParams& p, int* nyo, int* nzo) {
  *nyo = p.fixed[1] ? (int)L.ny - 2 : (int)L.ny;
  *nzo = p.fixed[2] ? (int)L.nz - 2 : (int)L.nz;
}

bool fast_shape_valid(const Layout& L, const StepParams& p, const FastShape& sh) {
  int nyo, nzo;
  output_ranges(L, p, &nyo, &nzo);
  bool w_ok = false;
  for (int w : kFastW) w_ok |= (w == sh.W);
  if (!w_ok || sh.nyb < 1 || sh.nzb < 1 || sh.nyb > nyo || sh.nzb > nzo) return false;
  return (nyo + sh.nyb - 1) / sh.nyb <= sh.W;
}

// One workgroup per CU with equal tiles: the widest W whose row blocks leave
// enough z-chunks to fill the device.
FastShape fast_default_shape(const Layout& L, const StepParams& p, int cus) {
  int nyo, nzo;
  output_ranges(L, p, &nyo, &nzo);
  FastShape sh;
  sh.W = 8;
  sh.nyb = (nyo + sh.W - 1) / sh.W;
  sh.nzb = cus / sh.nyb;
  if (sh.nzb < 1) sh.nzb = 1;
  if (sh.nzb > nzo) sh.nzb = nzo;
  return sh;
}

int fast_candidates(const Layout& L, const StepParams& p, int cus, FastShape* out, int max_out) {
  int nyo, nzo;
  output_ranges(L, p, &nyo, &nzo);
  int n = 0;
  for (int w : kFastW) {
    const int nyb = (nyo + w - 1) / w;
    for (int mult : {1, 2}) {
      int nzb = mult * cus / nyb;
      if (nzb < 1) nzb = 1;
      if (nzb > nzo) nzb = nzo;
      FastShape sh{w, nyb, nzb};
      bool dup = false;
      for (int i = 0; i < n; ++i) dup |= out[i].W == w && out[i].nyb == nyb && out[i].nzb == nzb;
      if (!dup && n < max_out && fast_shape_valid(L, p, sh)) out[n++] = sh;
    }
  }
  return n;
}

template <class C, int KX, int W>
static hipError_t launch_fast_w(const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  const dim3 block(64, W + 2, 1);
  hipLaunchKernelGGL((step_d3q19_fast<C, KX, W>), dim3(fp.nblocks), block, 0, s, (const E*)src, (E*)dst, fp);
  return hipGetLastError();
}

template <class C, int KX>
static hipError_t launch_fast_kx(int W, const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  switch (W) {
    case 4: return launch_fast_w<C, KX, 4>(src, dst, fp, s);
    case 6: return launch_fast_w<C, KX, 6>(src, dst, fp, s);
    case 8: return launch_fast_w<C, KX, 8>(src, dst, fp, s);
    case 10: return launch_fast_w<C, KX, 10>(src, dst, fp, s);
    case 12: return launch_fast_w<C, KX, 12>(src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

template <class C>
static hipError_t launch_fast_codec(const Layout& L, int W, const void* src, void* dst, const Fast3DParams& fp,
                                    hipStream_t s) {
  switch (L.nx) {
    case 64: return launch_fast_kx<C, 1>(W, src, dst, fp, s);
    case 128: return launch_fast_kx<C, 2>(W, src, dst, fp, s);
    case 256: return launch_fast_kx<C, 4>(W, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_fast(const Layout& L, const void* src, void* dst, const StepParams& p, const FastShape& sh,
                            hipStream_t s) {
  if (!fast_shape_valid(L, p, sh)) return hipErrorInvalidValue;
  Fast3DParams fp;
  fp.ny = (int)L.ny;
  fp.nz = (int)L.nz;
  fp.yper = !p.fixed[1];
  fp.zper = !p.fixed[2];
  fp.xwall = p.fixed[0];
  output_ranges(L, p, &fp.nyo, &fp.nzo);
  fp.ylo = fp.yper ? 0 : 1;
  fp.zlo = fp.zper ? 0 : 1;
  fp.nyb = sh.nyb;
  fp.nzb = sh.nzb;
  fp.nblocks = sh.nyb * sh.nzb;
  fp.plane = L.plane;
  fp.rho_ref = (float)p.rho_ref;
  fp.gx = (float)p.g[0];
  fp.gy = (float)p.g[1];
  fp.gz = (float)p.g[2];
  fp.seed = p.seed;
  fp.step = p.step;
  switch (L.precision) {
    case MACLAB_FP32: return launch_fast_codec<CodecF32>(L, sh.W, src, dst, fp, s);
    case MACLAB_HILO: return launch_fast_codec<CodecHILO>(L, sh.W, src, dst, fp, s);
    case MACLAB_S16: return launch_fast_codec<CodecS16>(L, sh.W, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace maclab
