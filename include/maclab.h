/*
 * maclab.h -- C ABI of the MI355X (gfx950) MacLAB library.
 *
 * The library advances the macroscopic lattice Boltzmann method of
 * J. G. Zhou, "Macroscopic Lattice Boltzmann Method (MacLAB)",
 * arXiv:1901.02716: with relaxation time tau = 1 the populations after a
 * step are the previous equilibria of the upstream neighbours (Methods,
 * Eqs. (9)-(10)), so only the density and velocity are stored and one step is
 *
 *   rho(x, t) = sum_a f_eq_a(x - e_a dt, t - dt)                  Eq. (4)
 *   u(x, t)   = 1/rho(x, t) sum_a e_a f_eq_a(x - e_a dt, t - dt)  Eq. (5)
 *
 * with f_eq of Eq. (2), particle speed e = 6 nu / dx (Eq. (6)) and time step
 * dt = dx / e. A problem is stated as the paper states it (recipe steps
 * (i)-(v) after Eq. (6)): a lattice, node counts, the lattice size dx, the
 * viscosity nu, macroscopic boundary values and the initial rho and u.
 *
 * Conventions
 *  - Every function returns an int status: MACLAB_OK (0) or a negative code.
 *    No C++ exception crosses this interface. maclab_last_error(h) returns a
 *    handle-owned message valid until the next call on h; with h == NULL it
 *    returns the message of the last failed call on this thread that had no
 *    handle (for example a rejected maclab_init).
 *  - Fields are SoA float64 arrays in physical units: rho has N = nx*ny*nz
 *    entries, u has d planes of N entries (u_x plane, then u_y, then u_z),
 *    node (i, j, k) at index i + nx*(j + ny*k). d = 2 for D2Q9, 3 for D3Q19.
 *  - Ownership: the caller owns every device buffer (including the workspace)
 *    and the stream; the library owns only the opaque handle and never frees
 *    caller memory. The workspace must outlive the handle.
 *  - Ordering: calls are ordered on the configured HIP stream. Only calls that
 *    return data to host memory (get_fields / set_fields with on_device = 0,
 *    diagnostics, params) synchronise that stream. A handle is not
 *    thread-safe; distinct handles are independent.
 */
#ifndef MACLAB_H
#define MACLAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MACLAB_OK 0
#define MACLAB_EINVAL -1       /* an argument or the configuration is invalid */
#define MACLAB_EUNSUPPORTED -2 /* lattice / precision / shape not supported */
#define MACLAB_EHIP -3         /* HIP runtime error; message names it */
#define MACLAB_EWORKSPACE -4   /* workspace missing or too small */
#define MACLAB_ENONFINITE -5   /* a checked step found NaN/Inf or |u|/e >= 1 */

/* Lattices (main text: D2Q9 with Eq. (1); D3Q19 in the numerical tests). */
enum { MACLAB_D2Q9 = 9, MACLAB_D3Q19 = 19 };

/* Storage of (rho - rho_ref, u / e) between steps. Arithmetic is FP64 for
 * MACLAB_FP64 and FP32 for the others.
 *  FP64 : 8 bytes per value.
 *  FP32 : 4 bytes per value.
 *  HILO : bfloat16 pair (hi, lo) with value = hi + lo, packed in 4 bytes.
 *  S16  : IEEE binary16 of a power-of-two scaled value (2^10 for the density
 *         deviation, 2^6 for the velocity), stored with stochastic rounding
 *         driven by a counter-based hash of (seed, step, node, field);
 *         2 bytes per value. */
enum { MACLAB_FP64 = 0, MACLAB_FP32 = 1, MACLAB_HILO = 2, MACLAB_S16 = 3 };

/* Faces and boundary kinds. A fixed face holds its physical (rho_b, u_b) on
 * every node of the face ("physical variables can directly be retained as
 * the boundary conditions", abstract (i); recipe step (iv)). The paper gives
 * no density for a wall and no inflow or outflow condition; two more kinds
 * of bounded face generalise the pressure-gradient term of test 2:
 *  MACLAB_BC_RHO_NEUMANN: the face holds u_b, and its density has a zero
 *    normal gradient: after every step it takes the new density of the
 *    nearest interior node (a wall that neither adds nor removes mass
 *    through a held density);
 *  MACLAB_BC_PRESSURE: the face holds rho_b, i.e. the pressure
 *    p = rho_b e^2 / 3 (Methods), and its velocity has a zero normal
 *    gradient: after every step it takes the new velocity of the nearest
 *    interior node (a pressure inlet or outlet).
 * The nearest interior node moves every index on a bounded axis into
 * 1 .. n-2. Both faces of an axis must be periodic, or both bounded (any mix
 * of the three bounded kinds). A node on several bounded faces belongs to
 * the lowest-numbered face (XLO < XHI < YLO < YHI < ZLO < ZHI), so side
 * walls own the edges and corners of a lid on the highest face. Reverse mode
 * and batches take periodic and fixed faces only. */
enum { MACLAB_XLO = 0, MACLAB_XHI, MACLAB_YLO, MACLAB_YHI, MACLAB_ZLO, MACLAB_ZHI };
enum { MACLAB_BC_PERIODIC = 0, MACLAB_BC_FIXED = 1, MACLAB_BC_RHO_NEUMANN = 2, MACLAB_BC_PRESSURE = 3 };

typedef struct maclab_s* maclab_t;

typedef struct {
  int32_t lattice;        /* MACLAB_D2Q9 or MACLAB_D3Q19 */
  int32_t precision;      /* MACLAB_FP64 / FP32 / HILO / S16 */
  int64_t n[3];           /* node counts including boundary nodes; n[2] = 1 for D2Q9 */
  double dx;              /* lattice size [m] (> 0) */
  double nu;              /* kinematic viscosity [m^2/s] (> 0) */
  double body_force[3];   /* uniform body force per unit volume G = -grad p [N/m^3] */
  double rho_ref;         /* reference density of the stored deviation (e.g. 1.0) */
  uint64_t seed;          /* stochastic-rounding stream (S16 only) */
  void* stream;           /* hipStream_t the library enqueues on; NULL = default stream */
  void* workspace;        /* caller-owned device memory, 256-byte aligned */
  size_t workspace_bytes; /* >= maclab_workspace_bytes(cfg) */
} maclab_config;

/* Bytes of workspace the configuration needs (two state buffers, reduction
 * partials, a host-transfer staging area). Pure host arithmetic; returns 0
 * for an invalid configuration. */
size_t maclab_workspace_bytes(const maclab_config* cfg);

/* Validates cfg, derives e = 6 nu / dx (Eq. (6)) and dt = dx / e, and binds
 * the workspace. All faces start periodic and the state starts at rest
 * (rho = rho_ref, u = 0). Invalid configurations return MACLAB_EINVAL (or
 * MACLAB_EWORKSPACE / MACLAB_EUNSUPPORTED) before any HIP call. */
int maclab_init(const maclab_config* cfg, maclab_t* out);

/* Sets face `face` to `kind`. A bounded face holds density rho_b and / or
 * velocity u_b[0..d-1] (physical units) as its kind says; the held values
 * are written into the state at once and never updated by maclab_step, the
 * others are taken from the interior now and after every step.
 * MACLAB_EUNSUPPORTED for RHO_NEUMANN or PRESSURE on a lattice of a batch. */
int maclab_set_bc(maclab_t h, int face, int kind, double rho_b, const double* u_b);

/* Loads physical rho (N values) and u (d*N values) into the state, then
 * re-imposes the fixed-face values. on_device = 1: device pointers;
 * on_device = 0: host pointers (copied through the staging area; syncs). */
int maclab_set_fields(maclab_t h, const double* rho, const double* u, int on_device);

/* Enqueues n time steps (Eqs. (4)-(5) plus the body force of test 2: the
 * new lattice velocity is (sum_a c_a f_eq_a + dt G / e) / rho'). Asynchronous.
 * Returns MACLAB_EINVAL if the face kinds of an axis differ. */
int maclab_step(maclab_t h, int64_t n);

/* Like maclab_step, but after every `check_every` steps reduces the state
 * and stops early with MACLAB_ENONFINITE when a value is non-finite or the
 * largest |u|/e reaches 1 (the validity condition of the equilibrium: Mach
 * number much smaller than one). *done receives the steps completed.
 * Synchronises at every check. */
int maclab_step_checked(maclab_t h, int64_t n, int64_t check_every, int64_t* done);

/* Writes physical rho (N values) and u (d*N values). on_device = 0 means
 * host destinations and synchronises. */
int maclab_get_fields(maclab_t h, double* rho, double* u, int on_device);

/* FP64 reductions over all nodes, written to host out[7]: mass sum rho,
 * momentum sum rho u (x, y, z), kinetic energy 1/2 sum rho |u|^2, max |u|/e,
 * number of nodes holding a non-finite value (excluded from the sums).
 * Deterministic (fixed reduction order). Synchronises. */
int maclab_diagnostics(maclab_t h, double out[7]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * reductions of maclab_diagnostics, enqueued on the handle's stream, with
 * the 7 doubles written to caller device memory out_dev (same order and
 * values) and without synchronising. Its reduction partials live in a fixed
 * 65.6 KB device array of the library (one per device, held until the
 * process ends, its address looked up when the first handle on the device
 * is created), not in the workspace; it calls no allocating routine. Every
 * call on one device shares that array: calls that overlap in time on one
 * device (different streams or threads) race and must be ordered by the
 * caller. MACLAB_EWORKSPACE if a reduction would not fit the array (cannot
 * happen with the library's fixed reduction width), MACLAB_EHIP if the
 * array's address cannot be obtained. */
int maclab_diagnostics_noalloc(maclab_t h, double* out_dev);

/* Host out[6]: particle speed e, time step dt, lattice Reynolds number
 * R_le = max_fixed |u_b| dx / nu (main text, stability remark after
 * Eq. (6)), Mach number R_le / 6, steps taken, simulated time steps * dt. */
int maclab_params(maclab_t h, double out[6]);

/* Native state: the d+1 stored planes of the current step in storage format,
 * maclab_state_bytes(h) bytes. In a plane, node (i, j, k) sits at element
 * i + px (j + ny k): for D2Q9 px is nx rounded up to a multiple of 128 bytes
 * (so every row starts on a 128-byte boundary); for D3Q19 it is the next of
 * 64, 128, 256 when that is at most nx + nx/8, else nx. The
 * plane stride is px ny nz rounded up to 512, plus 256 elements. The library
 * gives no result that depends on the padding (row ends and plane ends) and
 * keeps it zero in its own buffers. save copies the state to caller device memory; load
 * restores it bitwise into both ping-pong buffers (including 16-bit
 * storage), so a run resumed from a saved state repeats the original bit for
 * bit (for S16 the rounding stream is keyed by the step counter, which load
 * leaves unchanged). Stream-ordered, asynchronous. */
size_t maclab_state_bytes(maclab_t h);
int maclab_save_state(maclab_t h, void* dst_device);
int maclab_load_state(maclab_t h, const void* src_device);

/* Kernel and tiling of the step. out[5] = {kernel, W, nyb, nzb, pf}.
 *  kernel 0: general kernel (any shape and boundaries; no tiling).
 *  kernel 1: fast D3Q19, LDS exchange (row pitch 64, 128 or 256: x extent
 *    64, 128 or 256, or between fixed x faces an extent padded to one of
 *    them; FP32 arithmetic): one wavefront per x-row marches in z;
 *    workgroups of W output rows (W in {4,6,8,10,12}) plus two halo rows
 *    exchange the y-links through LDS; nyb x nzb workgroups with balanced
 *    (y, z) ranges; pf (1 or 2, 2 only with W <= 10 and unpadded rows)
 *    source planes loaded ahead. Needs ceil(rows / nyb) <= W.
 *  kernel 2: fast D3Q19, independent wavefronts (x extent 64 only): each
 *    wavefront owns one row and one of nzb balanced z-chunks and evaluates
 *    the links of the neighbouring rows it needs itself (no LDS, no
 *    barriers); W in {1,2,4,8} wavefronts per workgroup; nyb = pf = 1.
 *  kernel 3: fast D2Q9 (walled x of any extent, or periodic x whose extent
 *    is a multiple of W): one wavefront per (x-segment of 64*W nodes,
 *    band of rows), W in {1,2}; nzb bands; nyb (reported: segments per
 *    row) and pf are ignored.
 * set_tiling validates (nyb <= rows, nzb <= planes or bands <= rows) and
 * returns MACLAB_EUNSUPPORTED when the kernel does not handle the lattice.
 * Kernels 1 and 2 and every valid tiling of a kernel give bitwise identical
 * results. */
int maclab_get_tiling(maclab_t h, int out[5]);
int maclab_set_tiling(maclab_t h, int kernel, int W, int nyb, int nzb, int pf);

/* Times the candidate tilings of this lattice (each launched `reps` times
 * from the current state into the spare buffer, so the simulation does not
 * advance; before each timed launch an untimed pass reads the spare buffer,
 * so that the launch finds its source out of the caches, as a step does)
 * and keeps the fastest; *best_ms (may be NULL) receives its time per step.
 * The spare buffer then holds the state one step ahead, so until the next
 * step maclab_residual gives the change over that step. Synchronises. */
int maclab_autotune(maclab_t h, int reps, double* best_ms);

/* Replaces the uniform body force G (physical units) for subsequent steps. */
int maclab_set_body_force(maclab_t h, const double* G);

/* One step from the native state at src to dst (both caller-owned device
 * buffers of maclab_state_bytes; dst receives the fixed-face values too; the
 * padding at plane ends is left as it was, and a D2Q9 row's padding may
 * receive src's),
 * with the rounding stream of step `step_index`. The handle's own state and
 * step counter are untouched. Used to recompute a trajectory segment from a
 * checkpoint. */
int maclab_step_external(maclab_t h, const void* src, void* dst, int64_t step_index);

/* Reverse mode (the chain rule through Eqs. (2), (4), (5) and the
 * body-force term of test 2, for a loss L on later velocities). An adjoint
 * vector is caller-owned device memory of maclab_adjoint_bytes: d+1 planes
 * of the handle's plane stride, FP64 for MACLAB_FP64 storage and FP32
 * otherwise. For the state at step n it holds not (dL/drho, dL/du~) but the
 * pair the reverse step needs, Mbar = (dL/du~) / rho and Rbar = dL/drho -
 * Mbar . u~ (zero at fixed nodes, whose values do not depend on the past).
 *  seed:    from the native state at the last step T (as saved) and the
 *           derivative dLdu of the loss with respect to the physical
 *           velocity at T (device FP64, d*N, SoA like the fields), writes
 *           the adjoint at T.
 *  reset:   zeroes the FP64 accumulator of the body-force derivative.
 *  step:    from the state at step n and the adjoint at n+1, writes the
 *           adjoint at n and adds step n+1's force contribution to the
 *           accumulator. adj_np1 and adj_n must differ.
 *  segment: the reverse sweep over steps step_index .. step_index+nsteps-1
 *           from a checkpoint: recomputes the states at step_index+1 ..
 *           step_index+nsteps-1 from `ckpt` (the state at step_index) into
 *           `states` (nsteps-1 consecutive slots of maclab_state_bytes;
 *           NULL when nsteps = 1), then applies `step` nsteps times, ping-
 *           ponging between adj_a and adj_b: on entry adj[*which] (adj_a for
 *           0, adj_b for 1) holds the adjoint at step_index+nsteps, on
 *           return adj[*which] holds the adjoint at step_index.
 *  result:  from the state and the adjoint at step 0 writes dL/du0 (device
 *           FP64, d*N) and, if dLdrho0 is not NULL, dL/drho0 (device FP64,
 *           N); dLdG (host, may be NULL) receives dL/dG from the
 *           accumulator. Synchronises when dLdG is requested.
 * The force accumulator is summed per wavefront or workgroup in FP64 into
 * slots each owned by one of them, folded in a fixed order, so results are
 * reproducible. It lives in the handle on purpose, rather than as a partial
 * buffer the caller passes to every step and reduces itself: the sum over a
 * whole reverse sweep then has one fixed folding order, whatever the
 * checkpoint schedule. Stream-ordered; every buffer must stay valid until the
 * stream reaches the call. */
size_t maclab_adjoint_bytes(maclab_t h);
int maclab_adjoint_seed(maclab_t h, const void* state_T, const double* dLdu, void* adj);
int maclab_adjoint_reset(maclab_t h);
int maclab_adjoint_step(maclab_t h, const void* state_n, const void* adj_np1, void* adj_n);
int maclab_adjoint_segment(maclab_t h, const void* ckpt, void* states, int64_t nsteps, int64_t step_index,
                           void* adj_a, void* adj_b, int* which);
int maclab_adjoint_result(maclab_t h, const void* state0, const void* adj0, double* dLdu0, double* dLdrho0,
                          double dLdG[3]);

/* Kernel of the reverse step. kernel -1: automatic (the default); 0: the
 * general kernel (any lattice); 3: the fast D2Q9 kernel (walled x of any
 * extent, or periodic x whose extent is a multiple of kx): one
 * wavefront per (x-segment of 64*kx nodes, kx in {1,2}, band of rows),
 * 1 <= nband <= ceil(ny/4). get writes {kernel, kx, nband} of the kernel
 * the reverse step uses. EUNSUPPORTED when kernel 3 does not handle the
 * lattice, EINVAL for an invalid tiling. */
int maclab_set_adjoint_tiling(maclab_t h, int kernel, int kx, int nband);
int maclab_get_adjoint_tiling(maclab_t h, int out[3]);

/* ----------------------------------------------------------------- batch
 * Many independent D2Q9 lattices (for instance lid-driven cavities of
 * different sizes and Reynolds numbers, test 3 of the paper) advanced
 * together. Each lattice is described by its own maclab_config (lattice
 * must be MACLAB_D2Q9; precision, rho_ref, seed and stream must match those
 * of lattice 0; the workspace fields are ignored) and lives in one caller-
 * owned workspace of maclab_batch_workspace_bytes (256-byte aligned device
 * memory; 0 means an invalid description). A full maclab_config per
 * lattice, rather than arrays of sizes and viscosities, is deliberate: each
 * lattice keeps every per-lattice option of a single handle (its own dx,
 * nu, body force and faces), validated by the same code as maclab_init.
 *  lattice:       a handle for lattice `index`, owned by the batch (NULL if
 *                 out of range). Use it with maclab_set_bc, set_fields,
 *                 get_fields, diagnostics, params, save_state and load_state
 *                 like a handle of its own; maclab_destroy ignores it and
 *                 reverse mode returns MACLAB_EUNSUPPORTED. Those calls share
 *                 the batch's scratch, so they must not overlap in time.
 *  step:          n steps of every lattice (Eqs. (4)-(5) with each
 *                 lattice's faces and force): one launch per step over a
 *                 table of work items {lattice, x-segment of 64*kx nodes,
 *                 band of `rows` rows}: lattices largest first, the items
 *                 of one lattice in row order. Runs of
 *                 steps_per_graph steps are captured once in a HIP graph
 *                 and replayed on a private stream ordered after and before
 *                 the caller's stream (not for MACLAB_S16, whose rounding is
 *                 keyed per step). Results are bitwise those of stepping each
 *                 lattice with maclab_step on the fast D2Q9 kernel.
 *                 MACLAB_EINVAL if a lattice was stepped on its own.
 *  step_separate: the same n steps as one launch per lattice per step (the
 *                 schedule a loop over single lattices would use).
 *  get_tiling:    out[3] = {kx, rows, work items}. set_tiling: kx in {1,2},
 *                 rows >= 4 (a periodic x extent must be a multiple of
 *                 kx). autotune: times every candidate (each launched
 *                 `reps` times into the spare buffers, so nothing advances;
 *                 an untimed pass over the spare buffers before each timed
 *                 launch leaves the source out of the caches, as in a step),
 *                 keeps the fastest; *best_ms (may be NULL) gets its time per
 *                 step. set_graph: steps per captured graph, even, 0 for none
 *                 (default 32). */
typedef struct maclab_batch_s* maclab_batch_t;
size_t maclab_batch_workspace_bytes(const maclab_config* cfgs, int count);
int maclab_batch_init(const maclab_config* cfgs, int count, void* workspace, size_t workspace_bytes,
                      maclab_batch_t* out);
maclab_t maclab_batch_lattice(maclab_batch_t b, int index);
int maclab_batch_count(maclab_batch_t b);
int maclab_batch_step(maclab_batch_t b, int64_t n);
int maclab_batch_step_separate(maclab_batch_t b, int64_t n);
int maclab_batch_get_tiling(maclab_batch_t b, int out[3]);
int maclab_batch_set_tiling(maclab_batch_t b, int kx, int rows);
int maclab_batch_set_graph(maclab_batch_t b, int steps_per_graph);
int maclab_batch_autotune(maclab_batch_t b, int reps, double* best_ms);
void maclab_batch_destroy(maclab_batch_t b);
const char* maclab_batch_last_error(maclab_batch_t b);

/* Calibration: copies `bytes` from src to dst (caller device memory, 16-byte
 * aligned, not overlapping; bytes a multiple of 16) on the handle's stream
 * with non-temporal 16-byte loads and device-scope (write-through) stores,
 * the access forms of the step kernels and the fastest copy form measured on
 * the device. Copying a state buffer back and forth moves the bytes of a step
 * without its arithmetic, which gives the memory rate a step can reach on
 * the device. Asynchronous. MACLAB_EINVAL for a NULL or misaligned pointer
 * or a size that is not a multiple of 16. */
int maclab_copy(maclab_t h, const void* src, void* dst, size_t bytes);

/* Steady state (recipe step (v): the computation is repeated until a
 * solution is reached). maclab_residual gives the change over the last step
 * from the two ping-pong buffers, which hold the last two states:
 * out[0] = max over nodes and components of |u_i(n) - u_i(n-1)| (physical
 * units), out[1] = max |rho(n) - rho(n-1)|, out[2] = the count of nodes of
 * state n holding a non-finite value (not counted in out[0], out[1]). After
 * init, set_fields or load_state, before any step, both buffers hold the same
 * state and the change is 0. Synchronises.
 * maclab_step_until steps in blocks of check_every steps and evaluates the
 * residual after each block, until out[0] < tol or max_steps steps are done;
 * *done (may be NULL) receives the steps taken and resid (may be NULL) the
 * last residual. MACLAB_OK whether or not it converged (compare resid[0]
 * with tol); MACLAB_ENONFINITE as soon as a check finds non-finite nodes;
 * MACLAB_EINVAL for tol < 0, max_steps < 0 or check_every < 1. */
int maclab_residual(maclab_t h, double out[3]);
int maclab_step_until(maclab_t h, double tol, int64_t max_steps, int64_t check_every, int64_t* done,
                      double resid[3]);

/* ----------------------------------------------- lattice BGK with tau = 1
 * The population scheme the paper starts from: Eq. (1), the lattice BGK
 * equation, with relaxation time tau = 1, so that a step streams the Q
 * populations of every node and relaxes them fully to the equilibrium of
 * Eq. (2):  f_a(x + c_a, t + 1) = f_eq_a(rho(x, t), u(x, t)),  with
 * rho = sum_a f_a and rho u = sum_a e_a f_a (+ dt G, the body force of
 * test 2, as in maclab_step). The Methods show that with tau = 1 this gives
 * the same rho and u as the MacLAB step (Eqs. (9)-(10)); it stores Q values
 * per node instead of d + 1, which is the memory the paper's method saves
 * (abstract, advantage (ii)). A handle of its own:
 *  - cfg as for maclab_init; precision MACLAB_FP64 or MACLAB_FP32 (the
 *    populations are stored and computed in that type), else
 *    MACLAB_EUNSUPPORTED. maclab_bgk_workspace_bytes returns 0 for an
 *    invalid or unsupported configuration.
 *  - State: two buffers of Q planes, node (i, j, k) at i + nx (j + ny k) of a
 *    plane (no row padding), plane stride maclab_bgk_state_bytes / (Q x
 *    element size), holding the post-collision populations as deviations
 *    f_a - w_a rho_ref. save_state copies the current buffer to caller device
 *    memory (stream-ordered).
 *  - set_bc: periodic or fixed faces only (MACLAB_EINVAL otherwise); a fixed
 *    node holds f_eq(rho_b, u_b) and is never updated, the lowest-numbered
 *    face owning edges and corners, as in maclab_set_bc.
 *  - set_fields: the populations become f_eq of the given physical (rho, u)
 *    (SoA FP64, as for maclab_set_fields); get_fields returns the moments
 *    of the stored populations, rho = sum_a f_a and u = sum_a e_a f_a / rho.
 *    Host pointers (on_device = 0) synchronise the stream.
 *  - step: n steps, stream-ordered and asynchronous; MACLAB_EINVAL if the
 *    faces of an axis differ.
 * The workspace is caller-owned device memory (256-byte aligned); the handle
 * owns nothing else on the device. */
typedef struct maclab_bgk_s* maclab_bgk_t;
size_t maclab_bgk_workspace_bytes(const maclab_config* cfg);
int maclab_bgk_init(const maclab_config* cfg, maclab_bgk_t* out);
int maclab_bgk_set_bc(maclab_bgk_t h, int face, int kind, double rho_b, const double* u_b);
int maclab_bgk_set_fields(maclab_bgk_t h, const double* rho, const double* u, int on_device);
int maclab_bgk_step(maclab_bgk_t h, int64_t n);
int maclab_bgk_get_fields(maclab_bgk_t h, double* rho, double* u, int on_device);
size_t maclab_bgk_state_bytes(maclab_bgk_t h);
int maclab_bgk_save_state(maclab_bgk_t h, void* dst_device);
void maclab_bgk_destroy(maclab_bgk_t h);
const char* maclab_bgk_last_error(maclab_bgk_t h);

/* Releases the handle (not the caller's memory). NULL is ignored. */
void maclab_destroy(maclab_t h);

const char* maclab_last_error(maclab_t h);

#ifdef __cplusplus
}
#endif

#endif /* MACLAB_H */
