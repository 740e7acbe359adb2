// Device-side building blocks of the MacLAB step for gfx950: lattice tables,
// the per-step parameter block, storage codecs and the stochastic-rounding
// hash. Everything here is GPU code of this library; it shares nothing with
// the CPU oracle used by the tests.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace maclab {

// ---------------------------------------------------------------- lattices
// Unit velocities c_a = e_a / e and weights. D2Q9 in the order listed with
// Eq. (1) of the paper, weights 4/9, 1/9, 1/36 (with Eq. (2)); D3Q19 in the
// order listed at the start of the numerical tests, weights 1/3, 1/18, 1/36.
template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
  static constexpr int D = 2;
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int wnum[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};  // w = wnum / 36
};

template <>
struct Lattice<19> {
  static constexpr int D = 3;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, -1, 1};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int wnum[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
};

// ------------------------------------------------------------- parameters
// Everything a step kernel needs, passed by value. Lattice units: the stored
// velocity is u~ = u / e and g = dt G / e is the per-step velocity increment
// of the body force (test 2 of the paper, with G = -dp/dx).
struct StepParams {
  int64_t nx, ny, nz;   // node counts
  int64_t px;           // elements between consecutive rows (>= nx)
  int64_t plane;        // elements between consecutive planes of one buffer
  int fixed[3];         // 1 if both faces of the axis are fixed (Dirichlet)
  double rho_ref;       // density the stored deviation refers to
  double g[3];          // dt * G / e
  uint64_t seed;        // S16 stochastic rounding
  uint64_t step;        // index of the step being computed
  uint32_t sr_key;      // sr_key(seed, step): rounding key of this step
};

// Node (i, j, k) is stored at i + px (j + ny k). The dense index d = i + nx (j
// + ny k) numbers the nodes without the row padding (the order of the fields
// a caller passes in and gets back, and the node numbers of the stochastic
// rounding); this returns the stored position of dense index d.
__device__ __forceinline__ int64_t stored_index(int64_t d, int64_t nx, int64_t px) {
  return px == nx ? d : (d / nx) * px + d % nx;
}

// --------------------------------------------------------- storage codecs
// A codec maps the compute type T to the stored element and back. Field index
// 0 is the density deviation rho - rho_ref, fields 1..D are u~.
__device__ __forceinline__ float bits_f32(uint32_t b) { return __uint_as_float(b); }

struct CodecF64 {
  using elem = double;
  using T = double;
  static constexpr int bytes = 8;
  static constexpr T kScaleRho = 1, kScaleU = 1;
  __device__ static T dec(elem s, int) { return s; }
  __device__ static T dec_scaled(elem s, int) { return s; }
  __device__ static elem enc(T v, int, uint32_t) { return v; }
  __device__ static elem enc_scaled(T v, int, uint32_t) { return v; }
  __device__ static elem enc_nearest(T v, int field) { return enc(v, field, 0u); }
};

struct CodecF32 {
  using elem = float;
  using T = float;
  static constexpr int bytes = 4;
  static constexpr T kScaleRho = 1, kScaleU = 1;
  __device__ static T dec(elem s, int) { return s; }
  __device__ static T dec_scaled(elem s, int) { return s; }
  __device__ static elem enc(T v, int, uint32_t) { return v; }
  __device__ static elem enc_scaled(T v, int, uint32_t) { return v; }
  __device__ static elem enc_nearest(T v, int field) { return enc(v, field, 0u); }
};

// Split bfloat16: hi = bf16(v), lo = bf16(v - hi), packed as (hi << 16) | lo
// (gfx950 converts with v_cvt_pk_bf16_f32, round to nearest even).
struct CodecHILO {
  using elem = uint32_t;
  using T = float;
  static constexpr int bytes = 4;
  static constexpr T kScaleRho = 1, kScaleU = 1;
  __device__ static T dec(elem s, int) {
    return bits_f32(s & 0xffff0000u) + bits_f32(s << 16);
  }
  __device__ static T dec_scaled(elem s, int field) { return dec(s, field); }
  __device__ static elem enc(T v, int, uint32_t) {
    const __bf16 hi = (__bf16)v;
    const __bf16 lo = (__bf16)(v - (float)hi);
    return ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16) | (uint32_t)__builtin_bit_cast(uint16_t, lo);
  }
  __device__ static elem enc_scaled(T v, int field, uint32_t bits) { return enc(v, field, bits); }
  __device__ static elem enc_nearest(T v, int field) { return enc(v, field, 0u); }
};

// Scaled binary16 with stochastic rounding: the value times 2^10 (density
// deviation) or 2^6 (velocity) is rounded to one of its two neighbouring
// binary16 values, up with probability equal to the fraction that binary16
// drops. Each stored node draws 32 random bits per step (`node_bits`, from a
// counter-based generator over the node index and the step).
struct CodecS16 {
  using elem = uint16_t;
  using T = float;
  static constexpr int bytes = 2;
  static constexpr T kScaleRho = 1024.0f, kScaleU = 64.0f;
  __device__ static float scale(int field) { return field == 0 ? kScaleRho : kScaleU; }
  __device__ static float inv_scale(int field) { return field == 0 ? (1.0f / kScaleRho) : (1.0f / kScaleU); }
  __device__ static T dec(elem s, int field) {
    _Float16 h = __builtin_bit_cast(_Float16, s);
    return (float)h * inv_scale(field);
  }
  // the stored value itself: the field times scale(field)
  __device__ static T dec_scaled(elem s, int) { return (float)__builtin_bit_cast(_Float16, s); }
  // The rounding conversion (v_cvt_sr_f16_f32) rounds up with probability
  // equal to the discarded fraction, drawn from the high bits of its random
  // operand; field f uses the node's 32 random bits rotated by 8 f.
  __device__ static uint32_t field_bits(uint32_t node_bits, int field) {
    return field == 0 ? node_bits : ((node_bits << (8 * field)) | (node_bits >> (32 - 8 * field)));
  }
  // `vs` is the value already multiplied by scale(field).
  __device__ static elem enc_scaled(T vs, int field, uint32_t node_bits) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 h = {};
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, vs, field_bits(node_bits, field), false);
    return __builtin_bit_cast(uint16_t, h.x);
  }
  __device__ static elem enc(T v, int field, uint32_t node_bits) {
    return enc_scaled(v * scale(field), field, node_bits);
  }
  // Two neighbouring scaled values of one field converted into the low and
  // high halves of one 32-bit word (the same bits as two enc_scaled calls).
  __device__ static uint32_t enc2_scaled(T a, T b, int field, uint32_t bits_a, uint32_t bits_b) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 h = {};
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, a, field_bits(bits_a, field), false);
    h = __builtin_amdgcn_cvt_sr_f16_f32(h, b, field_bits(bits_b, field), true);
    return __builtin_bit_cast(uint32_t, h);
  }
  // Round to nearest (fields set from outside the time loop).
  __device__ static elem enc_nearest(T v, int field) {
    const _Float16 h = (_Float16)(v * scale(field));
    return __builtin_bit_cast(uint16_t, h);
  }
};

// Counter-based random bits for CodecS16: a 32-bit integer finaliser of a
// Weyl sequence over the node index, offset by a key that mixes the seed and
// the step (computed once per launch on the host). The finaliser is the
// xorshift-multiply hash "lowbias32" published by C. Wellons (hash-prospector,
// 2018); the Weyl increments 0x9e3779b9 / 0x9e3779b1 are 2^32 divided by the
// golden ratio (Knuth's multiplicative hashing). Every node draws its own
// 32 bits per step.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__host__ __device__ __forceinline__ uint32_t sr_key(uint64_t seed, uint64_t step) {
  return mix32((uint32_t)seed ^ mix32((uint32_t)(seed >> 32) + (uint32_t)step * 0x9e3779b9u));
}

__device__ __forceinline__ uint32_t sr_node_bits(uint32_t key, int64_t node) {
  return mix32((uint32_t)node * 0x9e3779b1u + key);
}

template <class C>
struct needs_rng { static constexpr bool value = false; };
template <>
struct needs_rng<CodecS16> { static constexpr bool value = true; };

// ----------------------------------------------------------- reciprocal
// 1/x in FP32: the hardware estimate (v_rcp_f32, up to 1 ulp off, and not
// symmetric about the exact value) refined by one Newton step, so that the
// error stays within about half an ulp and does not build up as a drift over
// many steps of u~ = m / rho.
__device__ __forceinline__ float recip_f32(float x) {
#pragma clang fp contract(off)
  const float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// x / 36 for the link sums, which carry the weights times 36: the product
// with the rounded constant 1/36 (which is 2.4e-8 too large in FP32) is
// corrected by one residual step, so that no bias of that size is applied to
// the density in every step.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
__device__ __forceinline__ T div36(T x) {
#pragma clang fp contract(off)
  const T c = (T)(1.0 / 36.0);
  const T q = x * c;
  const T e = fma_t((T)-36, q, x);
  return fma_t(e, c, q);
}


// ------------------------------------------------------ cross-lane moves
// DPP wave rotates: lane l receives the value of lane l-1 (lane 0 that of
// lane 63), or of lane l+1 (lane 63 that of lane 0). A rotate gives every
// lane a source, so bound_ctrl (zero for lanes without one) changes no value;
// set, it lets the compiler drop the unused "old" operand (a register move
// per rotate where the result cannot be folded into the instruction using it).
__device__ __forceinline__ float dpp_from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF, true));
}
__device__ __forceinline__ double dpp_from_left(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) & 0xffffffff), 0x13C, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) >> 32), 0x13C, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double dpp_from_right(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) & 0xffffffff), 0x134, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) >> 32), 0x134, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------- buffer addressing
// Raw buffer loads and stores through a buffer resource of one field plane.
// A byte offset of kOutOfRange lies past every resource (resources are kept
// below 2^31 bytes): such a load returns zero and such a store is dropped by
// the hardware's range check, so lanes without a node still execute the same
// memory instructions as the others and every wavefront issues the same
// sequence of memory operations whatever its position.
constexpr int kOutOfRange = (int)0x80000000;
using buf_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ buf_t make_buf(const void* base, int64_t bytes) {
  // stride 0 (raw), range `bytes`, gfx9 data format word
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int BYTES>
struct BufIO;
template <>
struct BufIO<2> {
  using U = unsigned short;
  template <int AUX>
  __device__ static U load(buf_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX); }
  template <int AUX>
  __device__ static void store(U v, buf_t r, int off) { __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, AUX); }
};
template <>
struct BufIO<4> {
  using U = unsigned int;
  template <int AUX>
  __device__ static U load(buf_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX); }
  template <int AUX>
  __device__ static void store(U v, buf_t r, int off) { __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, AUX); }
};
template <>
struct BufIO<8> {
  typedef unsigned int U __attribute__((ext_vector_type(2)));
  template <int AUX>
  __device__ static U load(buf_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX); }
  template <int AUX>
  __device__ static void store(U v, buf_t r, int off) { __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, AUX); }
};
template <>
struct BufIO<16> {
  typedef unsigned int U __attribute__((ext_vector_type(4)));
  template <int AUX>
  __device__ static U load(buf_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX); }
  template <int AUX>
  __device__ static void store(U v, buf_t r, int off) { __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, AUX); }
};

// Cache-policy words of buffer loads and stores (gfx950): sc0 = 1, nt = 2,
// sc1 = 16. Non-temporal (nt) accesses stream past the caches; a
// device-scope store (sc1) writes through L2 to memory.
constexpr int kStoreStream = 2;
constexpr int kStoreDevice = 16;

// Loads / stores a trivially copyable V (2, 4, 8 or 16 bytes) at a byte offset;
// AUX is the cache-policy word (2: non-temporal).
template <class V, int AUX = 0>
__device__ __forceinline__ V buf_load(buf_t r, int off) {
  return __builtin_bit_cast(V, BufIO<sizeof(V)>::template load<AUX>(r, off));
}
// Bitwise or of two loaded values: of a load and an out-of-range load (which
// reads zero), the loaded value.
template <class V>
__device__ __forceinline__ V buf_or(const V& a, const V& b) {
  using U = typename BufIO<sizeof(V)>::U;
  const U r = (U)(__builtin_bit_cast(U, a) | __builtin_bit_cast(U, b));
  return __builtin_bit_cast(V, r);
}
template <class V, int AUX = 0>
__device__ __forceinline__ void buf_store(const V& v, buf_t r, int off) {
  BufIO<sizeof(V)>::template store<AUX>(__builtin_bit_cast(typename BufIO<sizeof(V)>::U, v), r, off);
}

}  // namespace maclab
