// Host-side declarations shared by the library's translation units: the
// handle, and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/maclab.h"
#include "device.h"

namespace maclab {

// Values of the six faces as the kernels see them (physical units except
// where noted).
struct FaceValues {
  int kind[6];
  double rho[6];
  double u[6][3];
};

struct Layout {
  int q = 0, d = 0, precision = 0, bytes = 0;
  int64_t nx = 0, ny = 0, nz = 0, N = 0;
  int64_t px = 0;             // elements between rows (nx, or nx rounded up to 128 bytes for D2Q9)
  int64_t plane = 0;          // elements between field planes (px ny nz rounded up, plus 256)
  size_t state_bytes = 0;     // (d + 1) planes
  size_t partial_bytes = 0;   // reduction partials
  size_t staging_bytes = 0;   // host transfer staging
  size_t adjoint_bytes = 0;   // per-workgroup FP64 slots of the force adjoint (+ fold result)
  size_t workspace_bytes = 0;
};

// A state buffer at least this large does not fit in the device's 256 MB
// last-level (memory-side) cache: what one step writes is evicted before the
// next step reads it, so the D2Q9 step streams its stores past the caches.
constexpr size_t kStreamStoreBytes = size_t(256) << 20;

constexpr int kDiagBlocks = 1024;  // partial sums of the diagnostics reduction
constexpr int kDiagValues = 8;     // M, Px, Py, Pz, E, max|u~|, non-finite, pad

// Workgroups of 256 for a per-element kernel over `count` elements. A grid
// dimension holds fewer than 2^32 work-items, and lattices may have more
// nodes, so these kernels stride over the elements and the grid is capped.
inline unsigned blocks_256(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < (int64_t(1) << 20) ? (b > 0 ? b : 1) : (int64_t(1) << 20));
}

// Launchers (kernels_generic.hip). All enqueue on `s` and return the launch
// status.
hipError_t launch_step_generic(const Layout& L, const void* src, void* dst, const StepParams& p,
                               hipStream_t s);
hipError_t launch_impose_bc(const Layout& L, void* buf0, void* buf1, const FaceValues& fv, double rho_ref,
                            double e, hipStream_t s);
// Faces with a zero normal gradient (MACLAB_BC_RHO_NEUMANN: density;
// MACLAB_BC_PRESSURE: velocity) copy it from their nearest interior nodes in
// `buf`; nothing is launched when no face is of those kinds.
bool has_derived_faces(const FaceValues& fv);
hipError_t launch_derive_faces(const Layout& L, void* buf, const FaceValues& fv, hipStream_t s);
// Dense nodes first .. first+count-1 of one field plane (dense index: x
// fastest over nx, no row padding) from / to FP64 arrays of count values.
hipError_t launch_encode(const Layout& L, void* plane_dst, const double* src, int64_t first, int64_t count,
                         double offset, double mul, int field, hipStream_t s);
hipError_t launch_decode(const Layout& L, double* dst, const void* plane_src, int64_t first, int64_t count,
                         double offset, double mul, int field, hipStream_t s);
// Largest change of u~ and of drho from state `prev` to state `cur` and the
// count of non-finite nodes in `cur`, into result[0..2] (FP64, in storage
// units); partials holds kDiagBlocks x 4 doubles.
hipError_t launch_residual(const Layout& L, const void* prev, const void* cur, double* partials, double* result,
                           hipStream_t s);
// Streaming copy of `bytes` (a multiple of 16; 16-byte aligned, disjoint).
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// Reads `bytes` (a multiple of 16, 16-byte aligned) with ordinary cached loads
// and keeps nothing (`sink` is written only if the data hash equals `key`,
// so the loads stay): it fills the caches with this buffer.
hipError_t launch_touch(const void* buf, size_t bytes, uint32_t* sink, uint32_t key, hipStream_t s);
hipError_t launch_diagnostics(const Layout& L, const void* state, double rho_ref, double e, double* partials,
                              double* result, hipStream_t s);

// Fast D3Q19 path (kernels_fast.hip). `supported` tells whether the fast
// kernels handle the layout; a FastShape selects one and its tiling.
// kind 0 (LDS exchange): W output rows per workgroup (one wavefront each,
// plus two halo rows), nyb x nzb workgroups with balanced ranges, pf source
// planes loaded ahead. kind 1 (independent wavefronts): W wavefronts per
// workgroup, each owning one row and one of nzb balanced z-chunks (nyb = 1,
// pf = 1).
struct FastShape {
  int W = 8, nyb = 1, nzb = 1;
  int pf = 1;
  int kind = 0;
};
bool fast_step_supported(const Layout& L, const StepParams& p);
bool fast_shape_valid(const Layout& L, const StepParams& p, const FastShape& sh);
FastShape fast_default_shape(const Layout& L, const StepParams& p, int cus);
int fast_candidates(const Layout& L, const StepParams& p, int cus, FastShape* out, int max_out);
hipError_t launch_step_fast(const Layout& L, const void* src, void* dst, const StepParams& p, const FastShape& sh,
                            hipStream_t s);

// Fast D2Q9 path (kernels_2d.hip): one wavefront per (x-segment of 64*kx
// nodes, band of rows); nband bands per segment.
struct Fast2DShape {
  int kx = 4, nband = 1;
};
bool fast2d_supported(const Layout& L, const StepParams& p);
bool fast2d_shape_valid(const Layout& L, const StepParams& p, const Fast2DShape& sh);
Fast2DShape fast2d_default_shape(const Layout& L, const StepParams& p, int cus);
int fast2d_candidates(const Layout& L, const StepParams& p, int cus, Fast2DShape* out, int max_out);
hipError_t launch_step_fast2d(const Layout& L, const void* src, void* dst, const StepParams& p,
                              const Fast2DShape& sh, hipStream_t s);

// Where one lattice of a batch lives in memory and how its boundaries behave
// (elements relative to the batch's state buffer).
struct Lattice2D {
  int nx, ny, pitch;  // node counts; elements between rows (>= nx)
  int xper, yper;     // periodic axes (else both faces fixed)
  double gx, gy;      // dt G / e
  int64_t base;       // element offset of the lattice's first field plane
  int64_t plane;      // elements between field planes
};
// A batch step: work item {lattice, x0, y0, y1} of a device table, one
// wavefront each, all lattices in one launch (every pitch a multiple of kx).
// stream_stores: non-temporal stores (a state buffer of kStreamStoreBytes or
// more).
hipError_t launch_step_fast2d_items(int precision, int kx, const void* src, void* dst, const Lattice2D* lat,
                                    const int4* items, int nitems, double rho_ref, uint32_t sr_key,
                                    bool stream_stores, hipStream_t s);

// Reverse mode (kernels_adjoint.hip). Adjoint buffers hold (Rbar, Mbar) in
// the compute type, d + 1 planes of `plane` elements.
int64_t adjoint_slots(const Layout& L);
hipError_t launch_adjoint_step(const Layout& L, const void* sn, const void* an1, void* an, const StepParams& p,
                               double* gslots, hipStream_t s);
bool adjoint2d_supported(const Layout& L, const StepParams& p);
bool adjoint2d_shape_valid(const Layout& L, const StepParams& p, const Fast2DShape& sh);
Fast2DShape adjoint2d_default_shape(const Layout& L, const StepParams& p, int cus);
hipError_t launch_adjoint_fast2d(const Layout& L, const void* sn, const void* an1, void* an, const StepParams& p,
                                 const Fast2DShape& sh, double* gslots, hipStream_t s);
hipError_t launch_adjoint_seed(const Layout& L, const void* sT, const double* dLdu, void* adj, const StepParams& p,
                               double e, hipStream_t s);
hipError_t launch_adjoint_result(const Layout& L, const void* s0, const void* adj, double* dLdu, double* dLdrho,
                                 double rho_ref, double e, hipStream_t s);
hipError_t launch_adjoint_fold(const double* slots, int64_t nslots, double* out, hipStream_t s);
hipError_t launch_zero_doubles(double* dst, int64_t count, hipStream_t s);

// Lattice BGK with tau = 1, populations stored (kernels_bgk.hip): Q planes
// of `plane` elements, dense rows, FP64 or FP32 deviations F_a - w_a rho_ref.
struct BgkParams {
  int64_t nx, ny, nz;   // node counts
  int64_t plane;        // elements between population planes
  int fixed[3];         // 1 if both faces of the axis are fixed
  double rho_ref;       // density the stored deviations refer to
  double g[3];          // dt G / e
};
hipError_t launch_bgk_step(int q, bool fp64, const BgkParams& p, const void* src, void* dst, hipStream_t s);
hipError_t launch_bgk_encode(int q, bool fp64, void* dst, int64_t plane, const double* rho, const double* ux,
                             const double* uy, const double* uz, int64_t first, int64_t count, double rho_ref,
                             double e, hipStream_t s);
hipError_t launch_bgk_decode(int q, bool fp64, const void* src, int64_t plane, double* rho, double* ux, double* uy,
                             double* uz, int64_t first, int64_t count, double rho_ref, double e, hipStream_t s);
hipError_t launch_bgk_impose(int q, bool fp64, void* b0, void* b1, const BgkParams& p, const FaceValues& fv, double e,
                             hipStream_t s);

}  // namespace maclab
