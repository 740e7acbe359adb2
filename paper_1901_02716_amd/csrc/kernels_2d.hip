// Fast D2Q9 MacLAB step for gfx950, for one lattice or a batch of lattices.
//
// Work decomposition
//  - A work item is (lattice, x-segment, band of rows). One wavefront takes
//    one item: lane l holds the KX consecutive nodes x0 + KX*l .. + KX-1 of
//    the segment (64*KX nodes wide) and the wavefront marches up the rows of
//    its band, keeping three rolling row accumulators (rows y-1, y, y+1).
//  - The weights are a tensor product (36 w = 6 w_x 6 w_y), so each node
//    computes the six moments of its equilibrium (Eq. (2), deviation form,
//    times 36) and the gather runs as an x pass (three values sent to each
//    x neighbour: an in-lane move or a DPP wave rotate across lanes) and a
//    y pass (the rolling row accumulators); see moments2 / send2. At the
//    edges of a segment that does not span the whole row, the two lanes at
//    the edges also take the moments of the node just outside it.
//  - After source row y is pushed, destination row y-1 holds the gathers of
//    Eqs. (4)-(5): rho' = rho_ref + drho', u~' = (m' + g) / rho'.
//  - There is no LDS and no barrier; every wavefront works alone.
//  - Contraction is off and every FMA is written out, so results do not
//    depend on the segmentation or banding.
#include "internal.h"

#include <type_traits>

namespace maclab {

struct Fast2DParams {
  const Lattice2D* lat;  // device array (batch) ...
  Lattice2D one;         // ... or this single lattice when lat == nullptr
  const int4* items;     // device array of work items {lattice, x0, y0, y1} ...
  int nseg, nband;       // ... or, when items == nullptr, segments x bands of `one`
  int nyo, ylo;          //     (output rows nyo from ylo, split into nband bands)
  int nitems;
  double rho_ref;
  uint32_t sr_key;
};

// The D2Q9 weights are a tensor product, 36 w_a = (6 w_x(c_x)) (6 w_y(c_y))
// with 6 w(0) = 4 and 6 w(+-1) = 1, and the link values of Eq. (2) in the
// deviation form F^_a = f_eq_a - w_a rho_ref are, times 36,
//   36 F^_a = (6 w_x)(6 w_y) [a + c_x bx + c_y by + 1.5 (c_x^2 cxx + c_y^2 cyy) + 3 c_x c_y cxy]
// with rho = rho_ref + drho, bx = 3 rho u_x, by = 3 rho u_y, cxx = bx u_x,
// cyy = by u_y, cxy = bx u_y and a = drho - (cxx + cyy) / 2. So the gather of
// Eqs. (4)-(5) runs as a pass along x and a pass along y over the six
// moments of each node instead of over its nine links. Along x, node x
// receives from x-1 and x+1 (c_x = +1 from the left, -1 from the right)
//   R0 = a + bx + 1.5 cxx,  R1 = by + 3 cxy,  R2 = cyy   (sent to the right)
//   L0 = a - bx + 1.5 cxx,  L1 = by - 3 cxy,  L2 = cyy   (sent to the left)
// and forms, per power of c_y, the x-gathered density (T) and x momentum (U)
// terms of its row:
//   T0 = 4 a + R0' + L0',  T1 = 4 by + R1' + L1',  T2 = 1.5 (4 cyy + R2' + L2')
//   U0 = R0' - L0',        U1 = R1' - L1',         U2 = 1.5 (R2' - L2').
// Along y the row above receives T0 + T1 + T2 (density and y momentum) and
// U0 + U1 + U2 (x momentum), the row below T0 - T1 + T2 (density, minus y
// momentum) and U0 - U1 + U2, and the row itself 4 T0 and 4 U0: together
// 36 drho' and 36 m' of Eqs. (4)-(5).
template <class T>
struct Mom2 {
  T a, bx, by, cxx, cyy, cxy;
};

template <class T>
__device__ __forceinline__ void moments2(T dr, T ux, T uy, T rho_ref, Mom2<T>& M) {
#pragma clang fp contract(off)
  const T rho = rho_ref + dr;
  const T r3 = (T)3 * rho;
  M.bx = r3 * ux;
  M.by = r3 * uy;
  M.cxx = M.bx * ux;
  M.cyy = M.by * uy;
  M.cxy = M.bx * uy;
  M.a = fma_t(M.cxx + M.cyy, (T)-0.5, dr);
}

// What a node sends along x: to the right (R0, R1; R2 = cyy) and to the
// left (L0, L1; L2 = cyy).
template <class T>
struct Send2 {
  T r0, r1, l0, l1, c2;
};

template <class T>
__device__ __forceinline__ Send2<T> send2(const Mom2<T>& M) {
#pragma clang fp contract(off)
  Send2<T> S;
  const T s = fma_t(M.cxx, (T)1.5, M.a);
  S.r0 = s + M.bx;
  S.l0 = s - M.bx;
  S.r1 = fma_t(M.cxy, (T)3, M.by);
  S.l1 = fma_t(M.cxy, (T)-3, M.by);
  S.c2 = M.cyy;
  return S;
}

template <class E, int KX>
struct alignas(sizeof(E) * KX) RowVec2 {
  E v[KX];
};

template <class T, int KX>
struct RowAcc2 {
  T r[KX], mx[KX], my[KX];  // 36 * (drho', m')
};

// Wavefronts per SIMD the register budget must allow (keeps the scheduler
// from spending registers on hoisting).
template <class C, int KX>
struct Occupancy2D {
  static constexpr int value = sizeof(typename C::T) == 8 ? (KX > 1 ? 2 : 3) : 4;
};

// Memory access of one wavefront goes through buffer resources of the three
// field planes of its lattice, and every wavefront issues the same sequence of
// loads and stores in every row step: lanes without a node (past the end of
// the row, the halo of an interior lane, a row past the band) use an
// out-of-range offset. The compiler's wait for a row's loads then only has to
// let the previous row's stores stay in flight. Rows start on a boundary of
// at least 128 bytes (the row pitch), so a lane moves its KX nodes with one
// vector access per field.
//
// NT: stores stream past the caches (non-temporal), for a state buffer
// larger than the device's memory-side cache, where stores that stay in the
// caches only evict what the step still has to read (the 512-cavity batch
// step: 325 us cached, 283 us streamed, 321 us device-scope). Otherwise they
// are device-scope stores (sc1), which write through L2 and leave the new
// state in the memory-side cache for the next step, with nothing dirty in L2
// for the end of the kernel to write back (1024^2 FP64 cavity: 10.3 us
// cached, 8.9 us device-scope; 2048^2 FP32: 16.2, 15.1; 24.8 streamed).
template <class C, int KX, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occupancy2D<C, KX>::value)))
void step_d2q9_fast(const typename C::elem* __restrict__ src, typename C::elem* __restrict__ dst, Fast2DParams p) {
  using T = typename C::T;
  using E = typename C::elem;
  using V = RowVec2<E, KX>;
  constexpr int SW = 64 * KX;
  constexpr int EB = (int)sizeof(E);
  const int lane = threadIdx.x & 63;
  // XCD-aware numbering: workgroups go to the eight XCDs in turn (blockIdx.x
  // mod 8), so XCD k is given a contiguous range of work items -- the bands
  // of a lattice next to each other, whose boundary rows its L2 then shares.
  // The work item is uniform across the wavefront: keep it in scalar registers.
  const int nblk = (int)gridDim.x, bid = (int)blockIdx.x;
  const int per = nblk >> 3, rem = nblk & 7, xcd = bid & 7;
  const int lblk = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
  const int g = __builtin_amdgcn_readfirstlane(lblk * 4 + (int)(threadIdx.x >> 6));
  if (g >= p.nitems) return;
  Lattice2D lt;
  int x0, y0, y1;
  if (p.items) {
    const int4 it = p.items[g];
    lt = p.lat[it.x];
    x0 = it.y;
    y0 = it.z;
    y1 = it.w;
  } else {
    lt = p.one;
    const int seg = g % p.nseg, band = g / p.nseg;
    x0 = seg * SW;
    y0 = p.ylo + (int)((int64_t)band * p.nyo / p.nband);
    y1 = p.ylo + (int)((int64_t)(band + 1) * p.nyo / p.nband);
  }
  const int64_t pbytes = lt.plane * EB;
  buf_t rs[3], rd[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    rs[f] = make_buf(src + lt.base + f * lt.plane, pbytes);
    rd[f] = make_buf(dst + lt.base + f * lt.plane, pbytes);
  }
  const T rho_ref = (T)p.rho_ref;
  const int xb = x0 + KX * lane;
  // the segment spans the row (one wavefront): neighbours wrap through DPP;
  // otherwise the edge lanes evaluate the node just outside the segment
  // (wrapping on a periodic axis). On a periodic axis the lanes past the end
  // of the row load its first nodes again, so the last node's right
  // neighbour is in the next lane (the extent is a multiple of KX).
  const bool full_row = x0 == 0 && lt.nx == SW;
  const bool need_left = !full_row && (x0 > 0 || lt.xper);
  const bool need_right = !full_row && (x0 + SW < lt.nx || lt.xper);
  int hx = lane == 0 ? x0 - 1 : x0 + SW;
  hx = ((hx % lt.nx) + lt.nx) % lt.nx;
  const int xl = lt.xper ? xb % lt.nx : xb;  // the position this lane loads
  const bool in_row = lt.xper || xb < lt.nx;
  const bool halo_lane = (lane == 0 && need_left) || (lane == 63 && need_right);
  auto ywrap = [&](int y) { return lt.yper ? (y + lt.ny) % lt.ny : y; };

  // raw rows: a ring of five slots, row y in slot (y - y0 + 1) mod 5: the
  // source row being pushed, the row before it (whose wall nodes are stored
  // back unchanged) and three rows in flight. Slots are chosen at compile
  // time, so no row is copied between registers.
  V ring[5][3];
  E hring[5][3];
  auto load_row = [&](int y, bool valid, V (&ld)[3], E (&hld)[3]) {
    const int rb = (int)((int64_t)lt.pitch * ywrap(y) * EB);
    const int off = valid && in_row ? rb + xl * EB : kOutOfRange;
#pragma unroll
    for (int f = 0; f < 3; ++f) ld[f] = buf_load<V>(rs[f], off);
    const int hoff = valid && halo_lane ? rb + hx * EB : kOutOfRange;
#pragma unroll
    for (int f = 0; f < 3; ++f) hld[f] = buf_load<E>(rs[f], hoff);
  };

  RowAcc2<T, KX> A0, A1, A2;
#pragma unroll
  for (int e = 0; e < KX; ++e) A0.r[e] = A0.mx[e] = A0.my[e] = A1.r[e] = A1.mx[e] = A1.my[e] = (T)0;

  // Source row ys into rows ys-1 (am), ys (ac), ys+1 (ap, first touched here);
  // then destination row ys-1 is complete and stored (STORE), or the same
  // stores are issued out of range (the first row of the band).
  // Destination node d needs its own links (rest, +-y), the +x-moving links
  // of node d-1 (P) and the -x-moving links of node d+1 (M); it is completed
  // as soon as node d+1 has been evaluated, so few link values stay live.
  auto source_row = [&](auto store_c, auto slot_c, int ys, RowAcc2<T, KX>& am, RowAcc2<T, KX>& ac,
                        RowAcc2<T, KX>& ap) {
#pragma clang fp contract(off)
    constexpr bool STORE = decltype(store_c)::value;
    constexpr int SL = decltype(slot_c)::value;
    const V(&cur)[3] = ring[SL];
    const V(&prev)[3] = ring[(SL + 4) % 5];
    const E(&hv)[3] = hring[SL];
    T dr[KX], ux[KX], uy[KX];
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      dr[e] = C::dec(cur[0].v[e], 0);
      ux[e] = C::dec(cur[1].v[e], 1);
      uy[e] = C::dec(cur[2].v[e], 2);
    }
    Mom2<T> M[KX];
    Send2<T> S[KX];
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      moments2<T>(dr[e], ux[e], uy[e], rho_ref, M[e]);
      S[e] = send2<T>(M[e]);
    }
    // the node beside the segment (meaningful on the edge lanes only)
    Mom2<T> HM;
    moments2<T>(C::dec(hv[0], 0), C::dec(hv[1], 1), C::dec(hv[2], 2), rho_ref, HM);
    const Send2<T> H = send2<T>(HM);
    load_row(ys + 3, ys + 3 <= y1, ring[(SL + 3) % 5], hring[(SL + 3) % 5]);  // row ys - 2's slot
    // what enters the lane's first node from the left and its last node from the right
    T in_r0 = dpp_from_left(S[KX - 1].r0), in_r1 = dpp_from_left(S[KX - 1].r1),
      in_r2 = dpp_from_left(S[KX - 1].c2);
    T in_l0 = dpp_from_right(S[0].l0), in_l1 = dpp_from_right(S[0].l1), in_l2 = dpp_from_right(S[0].c2);
    if (lane == 0 && need_left) {
      in_r0 = H.r0;
      in_r1 = H.r1;
      in_r2 = H.c2;
    }
    if (lane == 63 && need_right) {
      in_l0 = H.l0;
      in_l1 = H.l1;
      in_l2 = H.c2;
    }
#pragma unroll
    for (int q = 0; q < KX; ++q) {
      const T r0 = q > 0 ? S[q - 1].r0 : in_r0, r1 = q > 0 ? S[q - 1].r1 : in_r1, r2 = q > 0 ? S[q - 1].c2 : in_r2;
      const T l0 = q < KX - 1 ? S[q + 1].l0 : in_l0, l1 = q < KX - 1 ? S[q + 1].l1 : in_l1,
              l2 = q < KX - 1 ? S[q + 1].c2 : in_l2;
      // the x pass of node q ...
      const T t0 = fma_t((T)4, M[q].a, r0 + l0), u0 = r0 - l0;
      const T t1 = fma_t((T)4, M[q].by, r1 + l1), u1 = r1 - l1;
      const T t2 = fma_t((T)4, M[q].cyy, r2 + l2), u2 = r2 - l2;
      // ... and the y pass: rows ys+1 (first touched here), ys and ys-1
      const T pt = fma_t((T)1.5, t2, t0), pu = fma_t((T)1.5, u2, u0);
      const T up = pt + t1, dn = pt - t1;
      const T qup = pu + u1, qdn = pu - u1;
      ap.r[q] = up;
      ap.my[q] = up;
      ap.mx[q] = qup;
      ac.r[q] = fma_t((T)4, t0, ac.r[q]);
      ac.mx[q] = fma_t((T)4, u0, ac.mx[q]);
      am.r[q] += dn;
      am.my[q] -= dn;
      am.mx[q] += qdn;
    }
    const int yd = ys - 1;
    const int rb = STORE ? (int)((int64_t)lt.pitch * ywrap(yd) * EB) : 0;
    V o[3];
#pragma unroll
    for (int q = 0; q < KX; ++q) {
      // drho' = r / 36, u~' = (m / 36 + g) / (rho_ref + r / 36) = (m + 36 g) / (36 rho_ref + r)
      const T drn = div36(am.r[q]);
      const T den = (T)36 * rho_ref + am.r[q];
      T inv;
      if constexpr (sizeof(T) == 4)
        inv = recip_f32(den);
      else
        inv = (T)1 / den;
      const T vx = (am.mx[q] + (T)(36.0 * lt.gx)) * inv;
      const T vy = (am.my[q] + (T)(36.0 * lt.gy)) * inv;
      uint32_t bits = 0;
      if constexpr (needs_rng<C>::value) bits = sr_node_bits(p.sr_key, (int64_t)lt.nx * ywrap(yd) + xb + q);
      o[0].v[q] = C::enc(drn, 0, bits);
      o[1].v[q] = C::enc(vx, 1, bits);
      o[2].v[q] = C::enc(vy, 2, bits);
    }
    // a wall node keeps its stored value (the row before holds it unchanged),
    // and so does the row padding a lane's last nodes may reach
#pragma unroll
    for (int q = 0; q < KX; ++q) {
      const int x = xb + q;
      if (x >= lt.nx || (!lt.xper && (x == 0 || x == lt.nx - 1))) {
#pragma unroll
        for (int f = 0; f < 3; ++f) o[f].v[q] = prev[f].v[q];
      }
    }
    const int off = STORE && xb < lt.nx ? rb + xb * EB : kOutOfRange;
#pragma unroll
    for (int f = 0; f < 3; ++f) buf_store<V, NT ? kStoreStream : kStoreDevice>(o[f], rd[f], off);
  };

  using NoStore = std::integral_constant<bool, false>;
  using Store = std::integral_constant<bool, true>;
  auto slot = [](auto k) { return std::integral_constant<int, decltype(k)::value>{}; };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  using S4 = std::integral_constant<int, 4>;
  // source rows y0-1 .. y1 (y1 >= y0 + 1); the first two complete no row of
  // the band. Accumulator roles rotate with period 3 and ring slots with
  // period 5: fifteen rows per trip.
  load_row(y0 - 1, true, ring[0], hring[0]);
  load_row(y0, true, ring[1], hring[1]);
  load_row(y0 + 1, true, ring[2], hring[2]);
#pragma unroll
  for (int f = 0; f < 3; ++f) ring[4][f] = V{};  // the row before the first (never stored)
  source_row(NoStore{}, slot(S0{}), y0 - 1, A0, A1, A2);
  source_row(NoStore{}, slot(S1{}), y0, A1, A2, A0);
  for (int ys = y0 + 1; ys <= y1; ys += 15) {
    source_row(Store{}, S2{}, ys, A2, A0, A1);
    if (ys + 1 > y1) break;
    source_row(Store{}, S3{}, ys + 1, A0, A1, A2);
    if (ys + 2 > y1) break;
    source_row(Store{}, S4{}, ys + 2, A1, A2, A0);
    if (ys + 3 > y1) break;
    source_row(Store{}, S0{}, ys + 3, A2, A0, A1);
    if (ys + 4 > y1) break;
    source_row(Store{}, S1{}, ys + 4, A0, A1, A2);
    if (ys + 5 > y1) break;
    source_row(Store{}, S2{}, ys + 5, A1, A2, A0);
    if (ys + 6 > y1) break;
    source_row(Store{}, S3{}, ys + 6, A2, A0, A1);
    if (ys + 7 > y1) break;
    source_row(Store{}, S4{}, ys + 7, A0, A1, A2);
    if (ys + 8 > y1) break;
    source_row(Store{}, S0{}, ys + 8, A1, A2, A0);
    if (ys + 9 > y1) break;
    source_row(Store{}, S1{}, ys + 9, A2, A0, A1);
    if (ys + 10 > y1) break;
    source_row(Store{}, S2{}, ys + 10, A0, A1, A2);
    if (ys + 11 > y1) break;
    source_row(Store{}, S3{}, ys + 11, A1, A2, A0);
    if (ys + 12 > y1) break;
    source_row(Store{}, S4{}, ys + 12, A2, A0, A1);
    if (ys + 13 > y1) break;
    source_row(Store{}, S0{}, ys + 13, A0, A1, A2);
    if (ys + 14 > y1) break;
    source_row(Store{}, S1{}, ys + 14, A1, A2, A0);
  }
}

// ------------------------------------------------------------------ launch
bool fast2d_supported(const Layout& L, const StepParams& p) {
  if (L.q != 9 || L.ny < 3) return false;
  if (L.plane * L.bytes >= (int64_t(1) << 31)) return false;  // buffer offsets are 31-bit
  return p.fixed[0] ? L.nx >= 3 : L.nx >= 1;
}

// Wider segments need more registers than a wavefront can hold without
// spilling (three rolling rows of accumulators per node).
static bool kx_ok(int kx) { return kx == 1 || kx == 2; }

bool fast2d_shape_valid(const Layout& L, const StepParams& p, const Fast2DShape& sh) {
  if (!kx_ok(sh.kx) || sh.nband < 1) return false;
  if (L.px % sh.kx != 0) return false;  // a lane's KX nodes are one vector access
  const int nyo = p.fixed[1] ? (int)L.ny - 2 : (int)L.ny;
  if (sh.nband > nyo) return false;
  if (!p.fixed[0] && L.nx % sh.kx != 0) return false;  // a periodic wrap may not split a lane's nodes
  return true;
}

Fast2DShape fast2d_default_shape(const Layout& L, const StepParams& p, int cus) {
  Fast2DShape sh;
  sh.kx = L.nx >= 128 ? 2 : 1;
  while (!p.fixed[0] && L.nx % sh.kx != 0) sh.kx /= 2;
  const int nseg = (int)((L.nx + 64 * sh.kx - 1) / (64 * sh.kx));
  const int nyo = p.fixed[1] ? (int)L.ny - 2 : (int)L.ny;
  int nband = (8 * cus + nseg - 1) / nseg;  // about 8 wavefronts per CU
  if (nband > nyo / 4) nband = nyo / 4;      // at least four rows per band
  if (nband < 1) nband = 1;
  sh.nband = nband;
  return sh;
}

int fast2d_candidates(const Layout& L, const StepParams& p, int cus, Fast2DShape* out, int max_out) {
  int n = 0;
  const int nyo = p.fixed[1] ? (int)L.ny - 2 : (int)L.ny;
  for (int kx : {1, 2}) {
    for (int per_cu : {4, 8, 16, 32}) {
      Fast2DShape sh;
      sh.kx = kx;
      const int nseg = (int)((L.nx + 64 * kx - 1) / (64 * kx));
      int nband = (per_cu * cus + nseg - 1) / nseg;
      if (nband > nyo) nband = nyo;
      sh.nband = nband;
      bool dup = false;
      for (int i = 0; i < n; ++i) dup |= out[i].kx == kx && out[i].nband == nband;
      if (!dup && n < max_out && fast2d_shape_valid(L, p, sh)) out[n++] = sh;
    }
  }
  return n;
}

template <class C, int KX, bool NT>
static hipError_t launch2d_kx(const void* src, void* dst, const Fast2DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  const unsigned blocks = (unsigned)((fp.nitems + 3) / 4);
  hipLaunchKernelGGL((step_d2q9_fast<C, KX, NT>), dim3(blocks), dim3(256), 0, s, (const E*)src, (E*)dst, fp);
  return hipGetLastError();
}

template <class C, bool NT>
static hipError_t launch2d_codec(int kx, const void* src, void* dst, const Fast2DParams& fp, hipStream_t s) {
  if (kx == 1) return launch2d_kx<C, 1, NT>(src, dst, fp, s);
  if (kx == 2) return launch2d_kx<C, 2, NT>(src, dst, fp, s);
  return hipErrorInvalidValue;
}

template <bool NT>
static hipError_t launch2d_nt(int precision, int kx, const void* src, void* dst, const Fast2DParams& fp,
                              hipStream_t s) {
  switch (precision) {
    case MACLAB_FP64: return launch2d_codec<CodecF64, NT>(kx, src, dst, fp, s);
    case MACLAB_FP32: return launch2d_codec<CodecF32, NT>(kx, src, dst, fp, s);
    case MACLAB_HILO: return launch2d_codec<CodecHILO, NT>(kx, src, dst, fp, s);
    case MACLAB_S16: return launch2d_codec<CodecS16, NT>(kx, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

static hipError_t launch2d(int precision, int kx, const void* src, void* dst, const Fast2DParams& fp,
                           bool stream_stores, hipStream_t s) {
  return stream_stores ? launch2d_nt<true>(precision, kx, src, dst, fp, s)
                       : launch2d_nt<false>(precision, kx, src, dst, fp, s);
}

hipError_t launch_step_fast2d_items(int precision, int kx, const void* src, void* dst, const Lattice2D* lat,
                                    const int4* items, int nitems, double rho_ref, uint32_t sr_key,
                                    bool stream_stores, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  Fast2DParams fp{};
  fp.lat = lat;
  fp.items = items;
  fp.nitems = nitems;
  fp.nseg = 1;
  fp.nband = 1;
  fp.rho_ref = rho_ref;
  fp.sr_key = sr_key;
  return launch2d(precision, kx, src, dst, fp, stream_stores, s);
}

hipError_t launch_step_fast2d(const Layout& L, const void* src, void* dst, const StepParams& p,
                              const Fast2DShape& sh, hipStream_t s) {
  if (!fast2d_shape_valid(L, p, sh)) return hipErrorInvalidValue;
  Fast2DParams fp{};
  fp.lat = nullptr;
  fp.items = nullptr;
  Lattice2D& lt = fp.one;
  lt.nx = (int)L.nx;
  lt.ny = (int)L.ny;
  lt.pitch = (int)L.px;
  lt.xper = !p.fixed[0];
  lt.yper = !p.fixed[1];
  lt.gx = p.g[0];
  lt.gy = p.g[1];
  lt.base = 0;
  lt.plane = L.plane;
  fp.nseg = (int)((L.nx + 64 * sh.kx - 1) / (64 * sh.kx));
  fp.nyo = p.fixed[1] ? lt.ny - 2 : lt.ny;
  fp.ylo = p.fixed[1] ? 1 : 0;
  fp.nband = sh.nband;
  fp.nitems = fp.nseg * fp.nband;
  fp.rho_ref = p.rho_ref;
  fp.sr_key = p.sr_key;
  return launch2d(L.precision, sh.kx, src, dst, fp, L.state_bytes >= kStreamStoreBytes, s);
}

}  // namespace maclab
