// Fast D3Q19 MacLAB step for gfx950 (rows of 64, 128 or 256 nodes, or rows
// between fixed x faces padded to one of those widths; FP32 arithmetic; FP32,
// split-bf16 or scaled-binary16 storage).
//
// Work decomposition
//  - A wavefront owns one whole x-row: lane l holds the KX = px/64 nodes
//    x = KX*l .. KX*l + KX-1 (px the row pitch), so every field row is one
//    coalesced vector load.
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
//    u~' = (m' + g) / rho', and stored: rows and planes of fixed faces are
//    never written, and a fixed node at either end of a row is written back
//    with its unchanged stored value.
//  - Workgroups are numbered so that each XCD gets a contiguous band of tiles
//    (neighbouring tiles share halo rows through that XCD's L2); rows that no
//    other workgroup reads are loaded non-temporally, to leave L2 to those.
#include "internal.h"

#include <type_traits>

namespace maclab {

struct Fast3DParams {
  int ny, nz;
  int ylo, nyo;            // first output row, number of output rows
  int zlo, nzo;            // first output plane, number of output planes
  int yper, zper, xwall;
  int nxd;                 // nodes per row (the row pitch is 64 KX, nxd < 64 KX only with fixed x faces)
  int nyb, nzb, nblocks;   // workgroups along y and z, total
  int64_t plane;           // elements per field plane
  float rho_ref;
  float g36x, g36y, g36z;  // 36 dt G / e
  uint32_t sr_key;         // S16 rounding key of this step
};

// ----------------------------------------------------------- row load/store
template <class C, int KX>
struct alignas(sizeof(typename C::elem) * KX) RowVec {
  typename C::elem v[KX];
};

// Loads one row of one field as stored (times the codec's storage scale).
template <class C, int KX>
__device__ __forceinline__ void load_row(const typename C::elem* __restrict__ p, int field, float (&out)[KX]) {
  const RowVec<C, KX> r = *reinterpret_cast<const RowVec<C, KX>*>(p);
#pragma unroll
  for (int e = 0; e < KX; ++e) out[e] = (float)C::dec_scaled(r.v[e], field);
}

// Stores one encoded row of one field; with x walls the first node of lane 0
// and the last node of lane 63 (the wall nodes) are left untouched.
template <class C, int KX>
__device__ __forceinline__ void store_row(typename C::elem* __restrict__ p, const RowVec<C, KX>& r, int lane,
                                          bool xwall) {
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

template <int KX>
struct PlaneAcc {
  float r[KX], mx[KX], my[KX], mz[KX];  // 36 * (drho', m')
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int e = 0; e < KX; ++e) r[e] = mx[e] = my[e] = mz[e] = 0.f;
  }
};

// Finalises the KX nodes of one row of destination plane accumulators a and
// encodes them: drho' = r / 36 and u~' = (m + 36 g) / (36 rho_ref + r)
// (Eqs. (4)-(5) with the sums carried times 36). The accumulators hold the
// sums times K = the codec's density scale (a power of two; see node_links),
// so K drho' = div36(a.r) and S u~' = S (a.m + 36 K g) / (36 K rho_ref + a.r)
// for the velocity scale S: every scale is exact, and the stored values
// carry them. Node e of the lane (dense node index node0 + e) draws its own
// rounding bits, sr_node_bits(key, node0 + e), the bits every kernel gives
// that node in that step, so the rounding decisions of neighbouring nodes are
// independent.
template <class C, int KX>
__device__ __forceinline__ void finalize_row(const PlaneAcc<KX>& a, float rho_ref, float g36x, float g36y, float g36z,
                                             uint32_t key, int64_t node0, RowVec<C, KX> (&o)[4]) {
#pragma clang fp contract(off)
  constexpr float K = C::kScaleRho;
  float v[4][KX];
  uint32_t bits[KX];
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    const float inv = recip_f32(K * (36.f * rho_ref) + a.r[e]) * C::kScaleU;
    v[0][e] = div36(a.r[e]);
    v[1][e] = (a.mx[e] + K * g36x) * inv;
    v[2][e] = (a.my[e] + K * g36y) * inv;
    v[3][e] = (a.mz[e] + K * g36z) * inv;
    bits[e] = needs_rng<C>::value ? sr_node_bits(key, node0 + e) : 0u;
  }
  if constexpr (sizeof(typename C::elem) == 2 && KX % 2 == 0) {
    struct Words { uint32_t w[KX / 2]; };
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      Words w;
#pragma unroll
      for (int e = 0; e < KX; e += 2) w.w[e / 2] = C::enc2_scaled(v[f][e], v[f][e + 1], f, bits[e], bits[e + 1]);
      o[f] = __builtin_bit_cast(RowVec<C, KX>, w);
    }
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int e = 0; e < KX; ++e) o[f].v[e] = C::enc_scaled(v[f][e], f, bits[e]);
  }
}

// The 19 link values of one node, times 36, in deviation form (Eq. (2)):
//   36 F^_a = wnum_a [a + c.b + sum_i c_i^2 q_ii + sum_{i<j} c_i c_j q_ij]
// with a = drho - 1.5 rho |u|^2, b = 3 rho u, q_ii = 4.5 rho u_i^2,
// q_ij = 9 rho u_i u_j. The six axis links are carried halved (h = F/2).
struct Links {
  float f0, hxp, hxm, hyp, hym, hzp, hzm;
  float pp0, mm0, pm0, mp0;  // (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0)
  float p0p, m0m, p0m, m0p;  // (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
  float zpp, zmm, zpm, zmp;  // (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
};

// Contraction is off and every FMA is written out, so a link value has the
// same bits whichever wavefront (output or halo row) computes it and the
// result does not depend on the tiling.
//
// The inputs are the stored fields times the codec's storage scales, d =
// K drho and v = S u~ (K, S powers of two; 1 for FP32 storage), and every
// link value comes out times K: with r3 = (3 K / S) rho each b and each
// product c_ij = b_i v_j carries K resp. K S, and the constants that multiply
// the c_ij are divided by S. Powers of two commute with every rounding, so
// the scaled links are K times the unscaled ones, bit for bit.
template <class C>
__device__ __forceinline__ void node_links(float dr, float ux, float uy, float uz, float rho_ref, Links& L) {
#pragma clang fp contract(off)
  constexpr float K = C::kScaleRho, S = C::kScaleU;
  const float rho = K == 1.f ? rho_ref + dr : __builtin_fmaf(dr, 1.f / K, rho_ref);
  const float r3 = (3.f * K / S) * rho;
  const float bx = r3 * ux, by = r3 * uy, bz = r3 * uz;    // 3 rho u          (times K)
  const float cxx = bx * ux, cyy = by * uy, czz = bz * uz;  // 3 rho u_i^2      (times K S; q_ii = 1.5 c_ii)
  const float cxy = bx * uy, cxz = bx * uz, cyz = by * uz;  // 3 rho u_i u_j    (times K S; q_ij = 3 c_ij)
  const float a = __builtin_fmaf((cxx + cyy) + czz, -0.5f / S, dr);
  const float sx = __builtin_fmaf(cxx, 1.5f / S, a), sy = __builtin_fmaf(cyy, 1.5f / S, a),
              sz = __builtin_fmaf(czz, 1.5f / S, a);
  L.f0 = 12.f * a;
  L.hxp = sx + bx;
  L.hxm = sx - bx;
  L.hyp = sy + by;
  L.hym = sy - by;
  L.hzp = sz + bz;
  L.hzm = sz - bz;
  float t, p, m, u, v;
  t = __builtin_fmaf(cyy, 1.5f / S, sx);  // a + q_xx + q_yy
  p = __builtin_fmaf(cxy, 3.f / S, t);
  m = __builtin_fmaf(cxy, -3.f / S, t);
  u = bx + by;
  v = bx - by;
  L.pp0 = p + u;
  L.mm0 = p - u;
  L.pm0 = m + v;
  L.mp0 = m - v;
  t = __builtin_fmaf(czz, 1.5f / S, sx);  // a + q_xx + q_zz
  p = __builtin_fmaf(cxz, 3.f / S, t);
  m = __builtin_fmaf(cxz, -3.f / S, t);
  u = bx + bz;
  v = bx - bz;
  L.p0p = p + u;
  L.m0m = p - u;
  L.p0m = m + v;
  L.m0p = m - v;
  t = __builtin_fmaf(czz, 1.5f / S, sy);  // a + q_yy + q_zz
  p = __builtin_fmaf(cyz, 3.f / S, t);
  m = __builtin_fmaf(cyz, -3.f / S, t);
  u = by + bz;
  v = by - bz;
  L.zpp = p + u;
  L.zmm = p - u;
  L.zpm = m + v;
  L.zmp = m - v;
}

// Pushes one source row (the KX nodes of this lane).
// MODE 0 (output row): c_y = 0 links go into the plane accumulators of this
// wavefront -- am (destination plane z-1), ac (plane z), ap (plane z+1, which
// this call is the first to touch, so it is assigned) -- and c_y = +-1 links
// into this wavefront's LDS rows. MODE 1 / 2 (halo row below / above the
// tile): only the c_y = +1 / -1 links, to LDS.
template <int KX>
__device__ __forceinline__ void own_row_links(const float (&f0)[KX], const float (&hzp)[KX], const float (&hzm)[KX],
                                              const float (&hxp)[KX], const float (&p0p)[KX], const float (&p0m)[KX],
                                              const float (&hxm)[KX], const float (&m0p)[KX], const float (&m0m)[KX],
                                              PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap);

template <class C, int KX, int MODE>
__device__ __forceinline__ void push_row(const float (&dr)[KX], const float (&ux)[KX], const float (&uy)[KX],
                                         const float (&uz)[KX], float rho_ref, PlaneAcc<KX>& am,
                                         PlaneAcc<KX>& ac, PlaneAcc<KX>& ap, float* __restrict__ up,
                                         float* __restrict__ dn, int lane) {
#pragma clang fp contract(off)
  constexpr int NX = 64 * KX;
  // c_y = 0 links kept per node: rest, +-z, and the four links that move in x
  float f0[KX], hzp[KX], hzm[KX];
  float hxp[KX], p0p[KX], p0m[KX];  // move to x+1
  float hxm[KX], m0p[KX], m0m[KX];  // move to x-1
  // c_y = +1 links (to the next row) and c_y = -1 links (to the previous row)
  float hyp[KX], pp0[KX], mp0[KX], zpp[KX], zpm[KX];
  float hym[KX], pm0[KX], mm0[KX], zmp[KX], zmm[KX];
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    Links L;
    node_links<C>(dr[e], ux[e], uy[e], uz[e], rho_ref, L);
    hyp[e] = L.hyp;
    pp0[e] = L.pp0;
    mp0[e] = L.mp0;
    zpp[e] = L.zpp;
    zpm[e] = L.zpm;
    hym[e] = L.hym;
    pm0[e] = L.pm0;
    mm0[e] = L.mm0;
    zmp[e] = L.zmp;
    zmm[e] = L.zmm;
    f0[e] = L.f0;
    hzp[e] = L.hzp;
    hzm[e] = L.hzm;
    hxp[e] = L.hxp;
    p0p[e] = L.p0p;
    p0m[e] = L.p0m;
    hxm[e] = L.hxm;
    m0p[e] = L.m0p;
    m0m[e] = L.m0m;
  }
  // What node x of the neighbouring row receives in the plane of the source
  // (the axis link of node x, the +x-moving diagonal of node x-1 and the
  // -x-moving one of node x+1) is combined here into its density and x
  // momentum contributions s and d; the +-z diagonals go as they are. LDS rows
  // are stored transposed (node KX*l + e at e*64 + l) so that a wavefront
  // touches 64 consecutive words.
  auto send = [&](float* __restrict__ buf, const float (&h)[KX], const float (&ep)[KX], const float (&em)[KX],
                  const float (&vp)[KX], const float (&vm)[KX]) {
    const float in_ep = dpp_from_left(ep[KX - 1]), in_em = dpp_from_right(em[0]);
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      const float a = e > 0 ? ep[e - 1] : in_ep, b = e < KX - 1 ? em[e + 1] : in_em;
      const int x = e * 64 + lane;
      buf[0 * NX + x] = __builtin_fmaf(2.f, h[e], a + b);
      buf[1 * NX + x] = a - b;
      buf[2 * NX + x] = vp[e];
      buf[3 * NX + x] = vm[e];
    }
  };
  if constexpr (MODE != 2) send(up, hyp, pp0, mp0, zpp, zpm);
  if constexpr (MODE != 1) send(dn, hym, pm0, mm0, zmp, zmm);
  if constexpr (MODE == 0) own_row_links<KX>(f0, hzp, hzm, hxp, p0p, p0m, hxm, m0p, m0m, am, ac, ap);
}

// The c_y = 0 links of a row into the plane accumulators: rest, +-z, and the
// links moving in x, which cross to the neighbouring lane at the lane edges.
// Plane z+1 (ap) is first touched here, so it is assigned.
template <int KX>
__device__ __forceinline__ void own_row_links(const float (&f0)[KX], const float (&hzp)[KX], const float (&hzm)[KX],
                                              const float (&hxp)[KX], const float (&p0p)[KX], const float (&p0m)[KX],
                                              const float (&hxm)[KX], const float (&m0p)[KX], const float (&m0m)[KX],
                                              PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
#pragma clang fp contract(off)
  const float in_hxp = dpp_from_left(hxp[KX - 1]), in_p0p = dpp_from_left(p0p[KX - 1]),
              in_p0m = dpp_from_left(p0m[KX - 1]);
  const float in_hxm = dpp_from_right(hxm[0]), in_m0p = dpp_from_right(m0p[0]), in_m0m = dpp_from_right(m0m[0]);
#pragma unroll
  for (int d = 0; d < KX; ++d) {
    // links arriving at node d from d-1 (moving +x) and d+1 (moving -x)
    const float Phx = d > 0 ? hxp[d - 1] : in_hxp, Pzp = d > 0 ? p0p[d - 1] : in_p0p,
                Pzm = d > 0 ? p0m[d - 1] : in_p0m;
    const float Mhx = d < KX - 1 ? hxm[d + 1] : in_hxm, Mzp = d < KX - 1 ? m0p[d + 1] : in_m0p,
                Mzm = d < KX - 1 ? m0m[d + 1] : in_m0m;
    // plane z: rest and +-x
    const float A = Phx + Mhx, B = Phx - Mhx;
    ac.r[d] += __builtin_fmaf(2.f, A, f0[d]);
    ac.mx[d] = __builtin_fmaf(2.f, B, ac.mx[d]);
    // plane z+1: +z, +x+z, -x+z (first contributions to this plane)
    const float sp = __builtin_fmaf(2.f, hzp[d], Pzp + Mzp);
    ap.r[d] = sp;
    ap.mz[d] = sp;
    ap.mx[d] = Pzp - Mzp;
    // plane z-1: -z, +x-z, -x-z
    const float sm = __builtin_fmaf(2.f, hzm[d], Pzm + Mzm);
    am.r[d] += sm;
    am.mz[d] -= sm;
    am.mx[d] += Pzm - Mzm;
  }
}

// Adds the c_y = +1 links arriving from the row below (S = +1) or the c_y =
// -1 links from the row above (S = -1) to the plane accumulators. For node d
// the arriving links are h (the axis link, halved), ep from node d-1 (moving
// +x), em from node d+1 (moving -x), and vp / vm (moving +z / -z). The y
// momentum of plane z+1 is first touched by the row below, so it is assigned.
template <int KX, int S>
__device__ __forceinline__ void add_row_links(float h, float ep_from_left, float em_from_right, float vp, float vm,
                                              int d, PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
#pragma clang fp contract(off)
  const float s = __builtin_fmaf(2.f, h, ep_from_left + em_from_right);
  ac.r[d] += s;
  ac.mx[d] += ep_from_left - em_from_right;
  ap.r[d] += vp;
  ap.mz[d] += vp;
  am.r[d] += vm;
  am.mz[d] -= vm;
  if constexpr (S > 0) {
    ac.my[d] += s;
    ap.my[d] = vp;
    am.my[d] += vm;
  } else {
    ac.my[d] -= s;
    ap.my[d] -= vp;
    am.my[d] -= vm;
  }
}

// Adds the contributions sent through LDS by the rows below (c_y = +1 links,
// S = +1) and above (c_y = -1 links, S = -1): s and d in the plane of the
// source, vp / vm moving to planes z+1 / z-1. The y momentum of plane z+1 is
// first touched by the row below, so it is assigned.
template <int KX, int S>
__device__ __forceinline__ void add_sent(float s, float d, float vp, float vm, int e, PlaneAcc<KX>& am,
                                         PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
#pragma clang fp contract(off)
  ac.r[e] += s;
  ac.mx[e] += d;
  ap.r[e] += vp;
  ap.mz[e] += vp;
  am.r[e] += vm;
  am.mz[e] -= vm;
  if constexpr (S > 0) {
    ac.my[e] += s;
    ap.my[e] = vp;
    am.my[e] += vm;
  } else {
    ac.my[e] -= s;
    ap.my[e] -= vp;
    am.my[e] -= vm;
  }
}

template <int KX>
__device__ __forceinline__ void pull_rows(const float* __restrict__ from_below, const float* __restrict__ from_above,
                                          PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap, int lane) {
  constexpr int NX = 64 * KX;
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    const int x = e * 64 + lane;
    add_sent<KX, 1>(from_below[0 * NX + x], from_below[1 * NX + x], from_below[2 * NX + x], from_below[3 * NX + x], e,
                    am, ac, ap);
    add_sent<KX, -1>(from_above[0 * NX + x], from_above[1 * NX + x], from_above[2 * NX + x], from_above[3 * NX + x], e,
                     am, ac, ap);
  }
}

template <int KX>
struct RowData {
  float dr[KX], ux[KX], uy[KX], uz[KX];
};

// Raw (stored) elements of one row of the four fields.
template <class C, int KX>
struct RawRow {
  RowVec<C, KX> f[4];
};

// c ? a : b on the bit patterns. A plain conditional between two elements of
// one row is turned by the compiler into a load at a selected index, which
// puts 16-bit rows in scratch memory.
template <class E>
__device__ __forceinline__ E pick_bits(bool c, E a, E b) {
  using U = std::conditional_t<sizeof(E) == 2, uint16_t, std::conditional_t<sizeof(E) == 4, uint32_t, uint64_t>>;
  static_assert(sizeof(U) == sizeof(E), "element size");
  const U m = (U)0 - (U)c;
  return __builtin_bit_cast(E, (U)((__builtin_bit_cast(U, a) & m) | (__builtin_bit_cast(U, b) & (U)~m)));
}

// PF: source planes loaded ahead (1 or 2).
//
// Memory goes through buffer resources of the four field planes, and every
// wavefront of the workgroup -- output, halo or idle -- issues the same four
// row loads and four row stores in every plane step: a wavefront without a
// row to load or to store (a halo row never stores, an idle wave neither
// loads nor stores, the first two planes of a tile complete no plane of it)
// uses an out-of-range offset, so the load reads zero and the store is
// dropped. With the same sequence of memory operations on every path the
// compiler's wait for a plane's loads lets the previous plane's stores stay in
// flight. Wall nodes of a stored row are written back with the raw values of
// the source row of the same plane, loaded one step before. PADX: the rows
// hold fewer than 64 KX nodes (fixed x faces); the lanes past the last node
// read the row padding and keep it, like the walls, from the raw row.
template <class C, int KX, int W, int PF, bool PADX>
__global__ __launch_bounds__(64 * (W + 2)) void step_d3q19_fast(const typename C::elem* __restrict__ src,
                                                               typename C::elem* __restrict__ dst, Fast3DParams p) {
  using E = typename C::elem;
  using V = RowVec<C, KX>;
  constexpr int NX = 64 * KX;
  constexpr int ROWS = W + 2;
  constexpr int EB = (int)sizeof(E);
  // LDS slots of 4 x NX words: ROWS-1 upward slots (rows 0..ROWS-2 send to
  // the next row) and ROWS-1 downward slots (rows 1..ROWS-1 send to the
  // previous row). With two such sets (when they fit in the 160 KB of LDS),
  // source planes alternate between them and one barrier per plane suffices:
  // a set is written again only two planes later, after every wavefront has
  // passed the barrier that follows its reads of that set.
  constexpr int SLOTS = 2 * (ROWS - 1) * 4 * NX;
  constexpr bool DB = 2 * SLOTS * 4 <= 160 * 1024;
  __shared__ float lds[(DB ? 2 : 1) * SLOTS];
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int s_up = wv < ROWS - 1 ? wv : ROWS - 2;  // slot this row sends up to (unused by the top row)
  const int s_dn = wv > 0 ? wv - 1 : 0;            // ... and down to (unused by the bottom row)
  float* const up0 = lds + s_up * 4 * NX;
  float* const dn0 = lds + (ROWS - 1 + s_dn) * 4 * NX;
  const float* const below0 = lds + s_dn * 4 * NX;             // sent up by row wv-1
  const float* const above0 = lds + (ROWS - 1 + s_up) * 4 * NX;  // sent down by row wv+1

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

  buf_t rs[4], rd[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    rs[f] = make_buf(src + f * p.plane, p.plane * EB);
    rd[f] = make_buf(dst + f * p.plane, p.plane * EB);
  }
  auto zwrap = [&](int z) { return p.zper ? (z + p.nz) % p.nz : z; };
  auto row_off = [&](int z) { return (int)((nx * ((int64_t)yrow + (int64_t)p.ny * zwrap(z)) + xbase) * EB); };
  // An output row other than the first and last of the tile (which the tiles
  // beside it in y read as halo rows, at about the same time) is loaded
  // non-temporally, so it does not take L2 space from the rows that are read
  // twice. (The planes a tile shares with its z neighbours are read at the
  // start of one tile and the end of the other, too far apart for L2 to keep
  // them, so they are loaded the same way.) With a one-plane prefetch every
  // wavefront issues both loads, one of them out of range; with a two-plane
  // prefetch of 32-bit rows it branches on its (uniform) row role; padded
  // rows and 16-bit rows at two planes are loaded cached.
  auto load_plane = [&](int z, bool valid, RawRow<C, KX>& b) {
    const int off = valid && mode != 3 ? row_off(z) : kOutOfRange;
    if constexpr (PF == 1 && !PADX) {
      const bool once = mode == 0 && wv >= 2 && wv <= rows - 1;
      const int oc = once ? kOutOfRange : off, on = once ? off : kOutOfRange;
#pragma unroll
      for (int f = 0; f < 4; ++f) b.f[f] = buf_or(buf_load<V>(rs[f], oc), buf_load<V, 2>(rs[f], on));
    } else if constexpr (PF == 2 && !PADX && EB == 4) {
      // with two planes in flight there are no registers for both load
      // forms: the wavefront picks one with a branch that is uniform across
      // it, so no wait for outstanding loads is needed where the paths join.
      // (For 16-bit rows, whose loads are half as wide, non-temporal loads
      // at this depth were slower: they stay cached.)
      const bool once = __builtin_amdgcn_readfirstlane((int)(mode == 0 && wv >= 2 && wv <= rows - 1)) != 0;
      if (once) {
#pragma unroll
        for (int f = 0; f < 4; ++f) b.f[f] = buf_load<V, 2>(rs[f], off);
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) b.f[f] = buf_load<V>(rs[f], off);
      }
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) b.f[f] = buf_load<V>(rs[f], off);
    }
  };
  const bool wall_lane = p.xwall && (lane == 0 || lane == 63);
  // raw wall elements (element 0 of lane 0, element KX-1 of lane 63) of the
  // row being pushed and of the row pushed one step before; with PADX the
  // whole raw rows
  E wcur[4], wprev[4];
  V rcur[4], rprev[4];

  // One source plane: push its links, exchange the c_y = +-1 links through
  // LDS, then finalise destination plane zs-1 (STORE) or issue the same stores
  // out of range. am / ac / ap are the accumulators of destination planes
  // zs-1, zs, zs+1; b holds plane zs and is refilled with plane zs+PF.
  auto source_plane = [&](auto store_c, int zs, PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap,
                          RawRow<C, KX>& b, int set) {
    constexpr bool STORE = decltype(store_c)::value;
    const int so = DB ? set * SLOTS : 0;
    float* const up = up0 + so;
    float* const dn = dn0 + so;
    float dr[KX], ux[KX], uy[KX], uz[KX];
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      dr[e] = (float)C::dec_scaled(b.f[0].v[e], 0);
      ux[e] = (float)C::dec_scaled(b.f[1].v[e], 1);
      uy[e] = (float)C::dec_scaled(b.f[2].v[e], 2);
      uz[e] = (float)C::dec_scaled(b.f[3].v[e], 3);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if constexpr (PADX) {
        rprev[f] = rcur[f];
        rcur[f] = b.f[f];
      } else {
        wprev[f] = wcur[f];
        wcur[f] = pick_bits(lane == 0, b.f[f].v[0], b.f[f].v[KX - 1]);
      }
    }
    if (mode == 0)
      push_row<C, KX, 0>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    else if (mode == 1)
      push_row<C, KX, 1>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    else if (mode == 2)
      push_row<C, KX, 2>(dr, ux, uy, uz, p.rho_ref, am, ac, ap, up, dn, lane);
    load_plane(zs + PF, zs + PF <= z1, b);
    __syncthreads();
    if (out_row) pull_rows<KX>(below0 + so, above0 + so, am, ac, ap, lane);
    if constexpr (!DB) __syncthreads();
    const int zd = zs - 1;
    V o[4] = {};
    if (STORE && out_row) {
      // dense index of the lane's first node (the stochastic rounding numbers
      // nodes without the row padding)
      const int64_t node0 = (int64_t)p.nxd * ((int64_t)yrow + (int64_t)p.ny * zwrap(zd)) + xbase;
      finalize_row<C, KX>(am, p.rho_ref, p.g36x, p.g36y, p.g36z, p.sr_key, node0, o);
      if constexpr (PADX) {
#pragma unroll
        for (int e = 0; e < KX; ++e) {
          const int x = xbase + e;
          if (x == 0 || x >= p.nxd - 1) {
#pragma unroll
            for (int f = 0; f < 4; ++f) o[f].v[e] = rprev[f].v[e];
          }
        }
      } else if (wall_lane) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          if (lane == 0)
            o[f].v[0] = wprev[f];
          else
            o[f].v[KX - 1] = wprev[f];
        }
      }
    }
    const int off = STORE && out_row ? row_off(zd) : kOutOfRange;
    // the new state is not read again in this step. Device-scope stores (sc1)
    // write through L2, so nothing of the new state is left dirty there for
    // the end of the kernel to write back, and the memory-side cache may keep
    // what the next step reads first: FP32 256^3 97.9 -> 93.3 us against
    // non-temporal stores (a plain copy of the same bytes: 85.5 -> 79.7 us).
#pragma unroll
    for (int f = 0; f < 4; ++f) buf_store<V, kStoreDevice>(o[f], rd[f], off);
  };

  // Source planes z0-1 .. z1 (z1 >= z0 + 1); the first two complete no plane
  // of the tile. Accumulator roles rotate with period 3 and the prefetch
  // buffers with period PF, so six planes per trip. The destination planes
  // z0-2 and z0-1 start from zero; plane zs+1 is assigned by the push of
  // plane zs.
  using NoStore = std::integral_constant<bool, false>;
  using Store = std::integral_constant<bool, true>;
  PlaneAcc<KX> a0, a1, a2;
  a0.zero();
  a1.zero();
  RawRow<C, KX> b0, b1;
  load_plane(z0 - 1, true, b0);
  if constexpr (PF == 2) load_plane(z0, true, b1);
  RawRow<C, KX>& c1 = PF == 2 ? b1 : b0;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    wcur[f] = E{};
    rcur[f] = V{};
  }
  source_plane(NoStore{}, z0 - 1, a0, a1, a2, b0, 0);
  source_plane(NoStore{}, z0, a1, a2, a0, c1, 1);
  for (int zs = z0 + 1; zs <= z1; zs += 6) {
    source_plane(Store{}, zs, a2, a0, a1, b0, 0);
    if (zs + 1 > z1) break;
    source_plane(Store{}, zs + 1, a0, a1, a2, c1, 1);
    if (zs + 2 > z1) break;
    source_plane(Store{}, zs + 2, a1, a2, a0, b0, 0);
    if (zs + 3 > z1) break;
    source_plane(Store{}, zs + 3, a2, a0, a1, c1, 1);
    if (zs + 4 > z1) break;
    source_plane(Store{}, zs + 4, a0, a1, a2, b0, 0);
    if (zs + 5 > z1) break;
    source_plane(Store{}, zs + 5, a1, a2, a0, c1, 1);
  }
}

// ----------------------------------------------- barrier-free variant
// Each wavefront owns one output x-row and a z-range and works alone, with
// no LDS and no barriers: per source plane it reads its own row and the rows
// below and above (the neighbouring rows come from the caches), evaluates the
// c_y = 0 links of its own row and, of the neighbouring rows, only the links
// that reach it. Link values and the order of every sum are those of the
// exchange kernel above, so both kernels give the same bits.
template <class C, int KX, int S>
__device__ __forceinline__ void neighbour_row(const RowData<KX>& b, float rho_ref, PlaneAcc<KX>& am,
                                              PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
  float h[KX], ep[KX], em[KX], vp[KX], vm[KX];
#pragma unroll
  for (int e = 0; e < KX; ++e) {
    Links L;
    node_links<C>(b.dr[e], b.ux[e], b.uy[e], b.uz[e], rho_ref, L);
    if constexpr (S > 0) {
      h[e] = L.hyp;
      ep[e] = L.pp0;
      em[e] = L.mp0;
      vp[e] = L.zpp;
      vm[e] = L.zpm;
    } else {
      h[e] = L.hym;
      ep[e] = L.pm0;
      em[e] = L.mm0;
      vp[e] = L.zmp;
      vm[e] = L.zmm;
    }
  }
  const float in_ep = dpp_from_left(ep[KX - 1]);
  const float in_em = dpp_from_right(em[0]);
#pragma unroll
  for (int d = 0; d < KX; ++d) {
    const float epl = d > 0 ? ep[d - 1] : in_ep;
    const float emr = d < KX - 1 ? em[d + 1] : in_em;
    add_row_links<KX, S>(h[d], epl, emr, vp[d], vm[d], d, am, ac, ap);
  }
}

template <class C, int KX, int NWV>
__global__ __launch_bounds__(64 * NWV) void step_d3q19_indep(const typename C::elem* __restrict__ src,
                                                             typename C::elem* __restrict__ dst, Fast3DParams p) {
  const int lane = threadIdx.x;
  const int wv = threadIdx.y;
  const int bid = blockIdx.x;
  const int per = p.nblocks >> 3, rem = p.nblocks & 7, xcd = bid & 7;
  const int blk = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int64_t g = (int64_t)blk * NWV + wv;  // wavefront index: row fastest
  if (g >= (int64_t)p.nyo * p.nzb) return;
  const int row = (int)(g % p.nyo), zc = (int)(g / p.nyo);
  const int y = p.ylo + row;
  const int z0 = p.zlo + (int)((int64_t)zc * p.nzo / p.nzb);
  const int z1 = p.zlo + (int)((int64_t)(zc + 1) * p.nzo / p.nzb);
  auto ywrap = [&](int v) { return p.yper ? (v + p.ny) % p.ny : v; };
  const int yb = ywrap(y - 1), ya = ywrap(y + 1);
  const int xbase = lane * KX;
  constexpr int64_t nx = 64 * KX;
  const int64_t plane = p.plane;
  auto zwrap = [&](int z) { return p.zper ? (z + p.nz) % p.nz : z; };
  auto load = [&](int yy, int z, RowData<KX>& b) {
    const int64_t base = nx * ((int64_t)yy + (int64_t)p.ny * zwrap(z)) + xbase;
    load_row<C, KX>(src + base, 0, b.dr);
    load_row<C, KX>(src + plane + base, 1, b.ux);
    load_row<C, KX>(src + 2 * plane + base, 2, b.uy);
    load_row<C, KX>(src + 3 * plane + base, 3, b.uz);
  };

  RowData<KX> own, below, above;
  auto source_plane = [&](int zs, PlaneAcc<KX>& am, PlaneAcc<KX>& ac, PlaneAcc<KX>& ap) {
    {
      float f0[KX], hzp[KX], hzm[KX], hxp[KX], p0p[KX], p0m[KX], hxm[KX], m0p[KX], m0m[KX];
#pragma unroll
      for (int e = 0; e < KX; ++e) {
        Links L;
        node_links<C>(own.dr[e], own.ux[e], own.uy[e], own.uz[e], p.rho_ref, L);
        f0[e] = L.f0;
        hzp[e] = L.hzp;
        hzm[e] = L.hzm;
        hxp[e] = L.hxp;
        p0p[e] = L.p0p;
        p0m[e] = L.p0m;
        hxm[e] = L.hxm;
        m0p[e] = L.m0p;
        m0m[e] = L.m0m;
      }
      if (zs < z1) load(y, zs + 1, own);
      own_row_links<KX>(f0, hzp, hzm, hxp, p0p, p0m, hxm, m0p, m0m, am, ac, ap);
    }
    neighbour_row<C, KX, 1>(below, p.rho_ref, am, ac, ap);
    if (zs < z1) load(yb, zs + 1, below);
    neighbour_row<C, KX, -1>(above, p.rho_ref, am, ac, ap);
    if (zs < z1) load(ya, zs + 1, above);
    const int zd = zs - 1;
    if (zd >= z0) {
      const int64_t node0 = nx * ((int64_t)y + (int64_t)p.ny * zwrap(zd)) + xbase;
      RowVec<C, KX> o[4];
      finalize_row<C, KX>(am, p.rho_ref, p.g36x, p.g36y, p.g36z, p.sr_key, node0, o);
#pragma unroll
      for (int f = 0; f < 4; ++f) store_row<C, KX>(dst + f * plane + node0, o[f], lane, p.xwall);
    }
  };

  PlaneAcc<KX> a0, a1, a2;
  a0.zero();
  a1.zero();
  load(y, z0 - 1, own);
  load(yb, z0 - 1, below);
  load(ya, z0 - 1, above);
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
  // one wavefront per row of 64, 128 or 256 nodes; a shorter row (padded to
  // that pitch) only between fixed x faces, since a periodic row wraps through
  // the wavefront's lanes
  if (L.px != 64 && L.px != 128 && L.px != 256) return false;
  if (L.px != L.nx && !p.fixed[0]) return false;
  if (L.ny < 3 || L.nz < 3) return false;
  if (L.plane * L.bytes >= (int64_t(1) << 31)) return false;  // buffer offsets are 31-bit
  return true;
}

static void output_ranges(const Layout& L, const StepParams& p, int* nyo, int* nzo) {
  *nyo = p.fixed[1] ? (int)L.ny - 2 : (int)L.ny;
  *nzo = p.fixed[2] ? (int)L.nz - 2 : (int)L.nz;
}

bool fast_shape_valid(const Layout& L, const StepParams& p, const FastShape& sh) {
  int nyo, nzo;
  output_ranges(L, p, &nyo, &nzo);
  if (sh.kind == 1) {
    // the independent kernel keeps three row buffers and three plane
    // accumulators per lane: it fits the register file only at nx = 64
    if (L.nx != 64) return false;
    const bool w_ok = sh.W == 1 || sh.W == 2 || sh.W == 4 || sh.W == 8;
    return w_ok && sh.nyb == 1 && sh.pf == 1 && sh.nzb >= 1 && sh.nzb <= nzo;
  }
  if (sh.kind != 0) return false;
  bool w_ok = false;
  for (int w : kFastW) w_ok |= (w == sh.W);
  if (!w_ok || (sh.pf != 1 && sh.pf != 2) || sh.nyb < 1 || sh.nzb < 1 || sh.nyb > nyo || sh.nzb > nzo)
    return false;
  if (sh.pf == 2 && sh.W > 10) return false;  // the two-plane buffer would not fit in registers
  if (sh.pf == 2 && L.px != L.nx) return false;  // padded rows: one-plane prefetch only
  return (nyo + sh.nyb - 1) / sh.nyb <= sh.W;
}

// One workgroup per CU with equal tiles: the widest W whose row blocks leave
// enough z-chunks to fill the device.
FastShape fast_default_shape(const Layout& L, const StepParams& p, int cus) {
  int nyo, nzo;
  output_ranges(L, p, &nyo, &nzo);
  FastShape sh;
  sh.W = 8;
  sh.pf = 1;
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
  // independent wavefronts: about 8, 12, 16 or 24 per CU
  for (int w : {2, 4, 8}) {
    for (int per_cu : {8, 12, 16, 24}) {
      int nzb = (per_cu * cus + nyo - 1) / nyo;
      if (nzb > nzo) nzb = nzo;
      if (nzb < 1) nzb = 1;
      FastShape sh{w, 1, nzb, 1, 1};
      bool dup = false;
      for (int i = 0; i < n; ++i) dup |= out[i].kind == 1 && out[i].W == w && out[i].nzb == nzb;
      if (!dup && n < max_out && fast_shape_valid(L, p, sh)) out[n++] = sh;
    }
  }
  for (int w : kFastW) {
    const int nyb = (nyo + w - 1) / w;
    // about one and two workgroups per CU, and a few z-chunk counts just
    // below one per CU (fewer, longer chunks fill and drain less)
    for (int eighths : {6, 7, 8, 16}) {
      int nzb = eighths * cus / (8 * nyb);
      if (nzb < 1) nzb = 1;
      if (nzb > nzo) nzb = nzo;
      for (int pf : {1, 2}) {
        FastShape sh{w, nyb, nzb, pf, 0};
        bool dup = false;
        for (int i = 0; i < n; ++i)
          dup |= out[i].kind == 0 && out[i].W == w && out[i].nyb == nyb && out[i].nzb == nzb && out[i].pf == pf;
        if (!dup && n < max_out && fast_shape_valid(L, p, sh)) out[n++] = sh;
      }
    }
  }
  return n;
}

template <class C, int KX, int W, int PF, bool PADX>
static hipError_t launch_fast_w(const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  const dim3 block(64, W + 2, 1);
  hipLaunchKernelGGL((step_d3q19_fast<C, KX, W, PF, PADX>), dim3(fp.nblocks), block, 0, s, (const E*)src, (E*)dst,
                     fp);
  return hipGetLastError();
}

template <class C, int KX, int PF, bool PADX>
static hipError_t launch_fast_pf(int W, const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  switch (W) {
    case 4: return launch_fast_w<C, KX, 4, PF, PADX>(src, dst, fp, s);
    case 6: return launch_fast_w<C, KX, 6, PF, PADX>(src, dst, fp, s);
    case 8: return launch_fast_w<C, KX, 8, PF, PADX>(src, dst, fp, s);
    case 10: return launch_fast_w<C, KX, 10, PF, PADX>(src, dst, fp, s);
    case 12:
      if constexpr (PF == 1) return launch_fast_w<C, KX, 12, PF, PADX>(src, dst, fp, s);
      break;
  }
  return hipErrorInvalidValue;
}

template <class C, int KX, int NWV>
static hipError_t launch_indep_w(const void* src, void* dst, const Fast3DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  if constexpr (KX == 1) {
    hipLaunchKernelGGL((step_d3q19_indep<C, KX, NWV>), dim3(fp.nblocks), dim3(64, NWV, 1), 0, s, (const E*)src,
                       (E*)dst, fp);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <class C, int KX>
static hipError_t launch_fast_kx(const FastShape& sh, const void* src, void* dst, const Fast3DParams& fp,
                                 hipStream_t s) {
  if (sh.kind == 1) {
    switch (sh.W) {
      case 1: return launch_indep_w<C, KX, 1>(src, dst, fp, s);
      case 2: return launch_indep_w<C, KX, 2>(src, dst, fp, s);
      case 4: return launch_indep_w<C, KX, 4>(src, dst, fp, s);
      case 8: return launch_indep_w<C, KX, 8>(src, dst, fp, s);
    }
    return hipErrorInvalidValue;
  }
  if (fp.nxd != 64 * KX) {
    // padded rows: the two-plane prefetch variant is not built for them
    if (sh.pf != 1) return hipErrorInvalidValue;
    return launch_fast_pf<C, KX, 1, true>(sh.W, src, dst, fp, s);
  }
  return sh.pf == 2 ? launch_fast_pf<C, KX, 2, false>(sh.W, src, dst, fp, s)
                    : launch_fast_pf<C, KX, 1, false>(sh.W, src, dst, fp, s);
}

template <class C>
static hipError_t launch_fast_codec(const Layout& L, const FastShape& sh, const void* src, void* dst,
                                    const Fast3DParams& fp, hipStream_t s) {
  switch (L.px) {
    case 64: return launch_fast_kx<C, 1>(sh, src, dst, fp, s);
    case 128: return launch_fast_kx<C, 2>(sh, src, dst, fp, s);
    case 256: return launch_fast_kx<C, 4>(sh, src, dst, fp, s);
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
  fp.nxd = (int)L.nx;
  output_ranges(L, p, &fp.nyo, &fp.nzo);
  fp.ylo = fp.yper ? 0 : 1;
  fp.zlo = fp.zper ? 0 : 1;
  fp.nyb = sh.nyb;
  fp.nzb = sh.nzb;
  if (sh.kind == 1) {
    const int64_t waves = (int64_t)fp.nyo * sh.nzb;
    fp.nblocks = (int)((waves + sh.W - 1) / sh.W);
  } else {
    fp.nblocks = sh.nyb * sh.nzb;
  }
  fp.plane = L.plane;
  fp.rho_ref = (float)p.rho_ref;
  fp.g36x = (float)(36.0 * p.g[0]);
  fp.g36y = (float)(36.0 * p.g[1]);
  fp.g36z = (float)(36.0 * p.g[2]);
  fp.sr_key = p.sr_key;
  switch (L.precision) {
    case MACLAB_FP32: return launch_fast_codec<CodecF32>(L, sh, src, dst, fp, s);
    case MACLAB_HILO: return launch_fast_codec<CodecHILO>(L, sh, src, dst, fp, s);
    case MACLAB_S16: return launch_fast_codec<CodecS16>(L, sh, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace maclab
