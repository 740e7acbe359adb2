// Fast D2Q9 MacLAB step for gfx950, for one lattice or a batch of lattices.
//
// Work decomposition
//  - A work item is (lattice, x-segment, band of rows). One wavefront takes
//    one item: lane l holds the KX consecutive nodes x0 + KX*l .. + KX-1 of
//    the segment (64*KX nodes wide) and the wavefront marches up the rows of
//    its band, keeping three rolling row accumulators (rows y-1, y, y+1).
//  - Each node computes the equilibria of its 9 links once (Eq. (2) in the
//    deviation form F^_a = f_eq_a - w_a rho_ref, times 36) and pushes them to
//    x + c_a: the y shift is the rolling accumulator, the x shift an in-lane
//    move or a DPP wave rotate across lanes. At the edges of a segment that
//    does not span the whole row, the two lanes at the edges also evaluate
//    the links of the neighbouring node outside the segment.
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

template <class T>
struct Links2 {
  T f0, qxp, qxm, qyp, qym;  // rest, and the axis links divided by 4
  T pp, mm, pm, mp;          // (1,1) (-1,-1) (1,-1) (-1,1)
};

// The 9 link values of one node, times 36: 36 F^_a = wnum_a [a + c.b +
// sum_i c_i^2 q_ii + c_x c_y q_xy] with a = drho - 1.5 rho |u|^2, b = 3 rho u,
// q_ii = 4.5 rho u_i^2, q_xy = 9 rho u_x u_y (wnum = 16, 4, 1).
template <class T>
__device__ __forceinline__ void links2(T dr, T ux, T uy, T rho_ref, Links2<T>& L) {
#pragma clang fp contract(off)
  const T rho = rho_ref + dr;
  const T r3 = (T)3 * rho;
  const T bx = r3 * ux, by = r3 * uy;
  const T cxx = bx * ux, cyy = by * uy, cxy = bx * uy;  // 3 rho u_i u_j
  const T a = fma_t(cxx + cyy, (T)-0.5, dr);
  const T sx = fma_t(cxx, (T)1.5, a), sy = fma_t(cyy, (T)1.5, a);
  L.f0 = (T)16 * a;
  L.qxp = sx + bx;
  L.qxm = sx - bx;
  L.qyp = sy + by;
  L.qym = sy - by;
  const T t = fma_t(cyy, (T)1.5, sx);
  const T p = fma_t(cxy, (T)3, t), m = fma_t(cxy, (T)-3, t);
  const T u = bx + by, v = bx - by;
  L.pp = p + u;
  L.mm = p - u;
  L.pm = m + v;
  L.mp = m - v;
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
template <class C, int KX>
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

  // raw rows: a ring of three rows in flight (row y in slot (y - y0 + 1) mod
  // 3), the source row being pushed (cur) and the row before it (prev, whose
  // wall nodes are stored back unchanged)
  V ring[3][3], cur[3], prev[3];
  E hring[3][3];
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
  auto source_row = [&](auto store_c, int ys, RowAcc2<T, KX>& am, RowAcc2<T, KX>& ac, RowAcc2<T, KX>& ap,
                        V (&ld)[3], E (&hld)[3]) {
#pragma clang fp contract(off)
    constexpr bool STORE = decltype(store_c)::value;
    T dr[KX], ux[KX], uy[KX];
    E hv[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      prev[f] = cur[f];
      cur[f] = ld[f];
      hv[f] = hld[f];
    }
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      dr[e] = C::dec(cur[0].v[e], 0);
      ux[e] = C::dec(cur[1].v[e], 1);
      uy[e] = C::dec(cur[2].v[e], 2);
    }
    T of0[KX], oyp[KX], oym[KX];   // own links of node e
    T pq[KX], ppp[KX], ppm[KX];    // P links of node e: (1,0)/4, (1,1), (1,-1)
    T mq[KX], mmp[KX], mmm[KX];    // M links of node e: (-1,0)/4, (-1,1), (-1,-1)
    auto complete = [&](int q, T Pq, T Ppp, T Ppm, T Mq, T Mmp, T Mmm) {
      // row ys: rest, +-x
      ac.r[q] += fma_t((T)4, Pq + Mq, of0[q]);
      ac.mx[q] = fma_t((T)4, Pq - Mq, ac.mx[q]);
      // row ys+1: +y, +x+y, -x+y
      const T sp = fma_t((T)4, oyp[q], Ppp + Mmp);
      ap.r[q] = sp;
      ap.my[q] = sp;
      ap.mx[q] = Ppp - Mmp;
      // row ys-1: -y, +x-y, -x-y
      const T sm = fma_t((T)4, oym[q], Ppm + Mmm);
      am.r[q] += sm;
      am.my[q] -= sm;
      am.mx[q] += Ppm - Mmm;
    };
#pragma unroll
    for (int e = 0; e < KX; ++e) {
      Links2<T> L;
      links2<T>(dr[e], ux[e], uy[e], rho_ref, L);
      of0[e] = L.f0;
      oyp[e] = L.qyp;
      oym[e] = L.qym;
      pq[e] = L.qxp;
      ppp[e] = L.pp;
      ppm[e] = L.pm;
      mq[e] = L.qxm;
      mmp[e] = L.mp;
      mmm[e] = L.mm;
      if (e >= 2) complete(e - 1, pq[e - 2], ppp[e - 2], ppm[e - 2], mq[e], mmp[e], mmm[e]);
    }
    Links2<T> H;
    links2<T>(C::dec(hv[0], 0), C::dec(hv[1], 1), C::dec(hv[2], 2), rho_ref, H);  // meaningful on halo lanes only
    load_row(ys + 3, ys + 3 <= y1, ld, hld);  // the slot just consumed takes row ys + 3
    // links entering the lane's first node from the left and last node from the right
    T in_q = dpp_from_left(pq[KX - 1]), in_pp = dpp_from_left(ppp[KX - 1]), in_pm = dpp_from_left(ppm[KX - 1]);
    T in_mq = dpp_from_right(mq[0]), in_mp = dpp_from_right(mmp[0]), in_mm = dpp_from_right(mmm[0]);
    if (lane == 0 && need_left) {
      in_q = H.qxp;
      in_pp = H.pp;
      in_pm = H.pm;
    }
    if (lane == 63 && need_right) {
      in_mq = H.qxm;
      in_mp = H.mp;
      in_mm = H.mm;
    }
    if constexpr (KX == 1) {
      complete(0, in_q, in_pp, in_pm, in_mq, in_mp, in_mm);
    } else {
      complete(0, in_q, in_pp, in_pm, mq[1], mmp[1], mmm[1]);
      complete(KX - 1, pq[KX - 2], ppp[KX - 2], ppm[KX - 2], in_mq, in_mp, in_mm);
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
    for (int f = 0; f < 3; ++f) buf_store<V>(o[f], rd[f], off);
  };

  using NoStore = std::integral_constant<bool, false>;
  using Store = std::integral_constant<bool, true>;
  // source rows y0-1 .. y1 (y1 >= y0 + 1); the first two complete no row of
  // the band
  load_row(y0 - 1, true, ring[0], hring[0]);
  load_row(y0, true, ring[1], hring[1]);
  load_row(y0 + 1, true, ring[2], hring[2]);
#pragma unroll
  for (int f = 0; f < 3; ++f) cur[f] = ring[0][f];
  source_row(NoStore{}, y0 - 1, A0, A1, A2, ring[0], hring[0]);
  source_row(NoStore{}, y0, A1, A2, A0, ring[1], hring[1]);
  for (int ys = y0 + 1; ys <= y1; ys += 3) {
    source_row(Store{}, ys, A2, A0, A1, ring[2], hring[2]);
    if (ys + 1 > y1) break;
    source_row(Store{}, ys + 1, A0, A1, A2, ring[0], hring[0]);
    if (ys + 2 > y1) break;
    source_row(Store{}, ys + 2, A1, A2, A0, ring[1], hring[1]);
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

template <class C, int KX>
static hipError_t launch2d_kx(const void* src, void* dst, const Fast2DParams& fp, hipStream_t s) {
  using E = typename C::elem;
  const unsigned blocks = (unsigned)((fp.nitems + 3) / 4);
  hipLaunchKernelGGL((step_d2q9_fast<C, KX>), dim3(blocks), dim3(256), 0, s, (const E*)src, (E*)dst, fp);
  return hipGetLastError();
}

template <class C>
static hipError_t launch2d_codec(int kx, const void* src, void* dst, const Fast2DParams& fp, hipStream_t s) {
  if (kx == 1) return launch2d_kx<C, 1>(src, dst, fp, s);
  if (kx == 2) return launch2d_kx<C, 2>(src, dst, fp, s);
  return hipErrorInvalidValue;
}

static hipError_t launch2d(int precision, int kx, const void* src, void* dst, const Fast2DParams& fp,
                           hipStream_t s) {
  switch (precision) {
    case MACLAB_FP64: return launch2d_codec<CodecF64>(kx, src, dst, fp, s);
    case MACLAB_FP32: return launch2d_codec<CodecF32>(kx, src, dst, fp, s);
    case MACLAB_HILO: return launch2d_codec<CodecHILO>(kx, src, dst, fp, s);
    case MACLAB_S16: return launch2d_codec<CodecS16>(kx, src, dst, fp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_fast2d_items(int precision, int kx, const void* src, void* dst, const Lattice2D* lat,
                                    const int4* items, int nitems, double rho_ref, uint32_t sr_key, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  Fast2DParams fp{};
  fp.lat = lat;
  fp.items = items;
  fp.nitems = nitems;
  fp.nseg = 1;
  fp.nband = 1;
  fp.rho_ref = rho_ref;
  fp.sr_key = sr_key;
  return launch2d(precision, kx, src, dst, fp, s);
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
  return launch2d(L.precision, sh.kx, src, dst, fp, s);
}

}  // namespace maclab
