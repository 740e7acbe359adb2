/*
 * MacLAB oracle: a plain, single-threaded, FP64 CPU implementation of the
 * macroscopic lattice Boltzmann time step of J. G. Zhou, "Macroscopic
 * Lattice Boltzmann Method (MacLAB)", arXiv:1901.02716.
 *
 * TEST INFRASTRUCTURE. This file is the correctness reference for the GPU
 * library and nothing else: only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the GPU path, and the GPU path never calls it.
 *
 * It is deliberately slow and literal. Everything is done in physical units,
 * in the paper's notation:
 *   e_a   = e * c_a                    particle velocity of link a
 *   f_eq  = w_a rho (1 + 3 e_a.u/e^2 + 9/2 (e_a.u)^2/e^4 - 3/2 u.u/e^2)
 *                                       main text, Eq. (2) [feq-full]
 *   rho(x,t)  = sum_a f_eq_a(x - e_a dt, t - dt)        Eq. (4) [mlb-p.1]
 *   u_i(x,t)  = 1/rho(x,t) sum_a e_ai f_eq_a(x - e_a dt, t - dt)
 *                                                       Eq. (5) [mlb-u.1]
 *   e  = 6 nu / dx                                      Eq. (6) [mlb-viscosity]
 *   dt = dx / e                                         text after Eq. (6)
 * A node x - e_a dt is the neighbouring lattice node x - c_a (main text,
 * after Eq. (6)); periodic axes wrap (numerical tests 1, 2 and 4).
 *
 * Readings of the paper this file takes (each one is listed in the design
 * notes of the repository):
 *  - Eq. (5) sums e_{aj}; the Methods derivation, Eqs. (12)-(13), shows the
 *    component is e_{ai}. The oracle uses e_{ai}.
 *  - Test 2 adds a pressure-gradient term "+dx/(e rho) dp/dx" to Eq. (5).
 *    With dp/dx < 0 that literal sign drives the flow towards -x, which
 *    contradicts the analytic profile Eq. (8) [Couette-PreGrad]. The oracle
 *    adds  + dt * G / rho'  with G = -dp/dx (a body force per unit volume),
 *    using dx/e = dt; rho' is the newly gathered density.
 *  - Fixed boundary nodes hold their physical rho and u ("no calculations
 *    are needed", test 2; abstract, advantage (i)). A node on several fixed
 *    faces takes the values of the face with the lowest index in the order
 *    XLO, XHI, YLO, YHI, ZLO, ZHI (so side walls own the edges and corners
 *    of a lid on the highest face).
 *  - Both faces of an axis are either periodic or bounded (fixed or one of
 *    the two kinds below, in any mix).
 *  - The paper never gives the density on a wall (only "no calculations are
 *    needed" there) nor an inflow/outflow condition; two further kinds of
 *    bounded face generalise test 2:
 *      RHO_NEUMANN: the face holds its velocity u_b, and its density has a
 *        zero normal gradient: after every step it takes the new density of
 *        the nearest interior node;
 *      PRESSURE: the face holds its density rho_b (the pressure
 *        p = rho e^2 / 3 of the Methods), and its velocity has a zero normal
 *        gradient: after every step it takes the new velocity of the
 *        nearest interior node.
 *    The nearest interior node of a boundary node moves every index on a
 *    bounded axis into 1 .. n-2 (for a node on one face, its neighbour along
 *    the normal; for an edge or a corner, the diagonal one).
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fPIC -shared (no threads, no
 * SIMD intrinsics, no FMA contraction).
 */
#include <stddef.h>
#include <tgmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The arithmetic type. FP64 is the oracle; a build with
 * -DORACLE_REAL="long double" (x87 extended precision, 64-bit significand)
 * runs the same steps with 11 more bits, which separates the FP64 oracle's
 * own rounding from a GPU path's in long runs of slow flows. Problem
 * parameters stay double; every field and every operation is `real`. */
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

/* sizeof(real): 8 for the FP64 oracle, 16 for the extended build. */
int oracle_real_bytes(void) { return (int)sizeof(real); }

#define ORACLE_PERIODIC 0
#define ORACLE_FIXED 1
#define ORACLE_RHO_NEUMANN 2
#define ORACLE_PRESSURE 3

/* Problem statement: lattice, node counts, dx, nu (main text, recipe step
 * (i)), a uniform body force, and per-face boundary kind and values. */
typedef struct {
  int32_t q;          /* 9 = D2Q9, 19 = D3Q19 */
  int32_t reserved;
  int64_t n[3];       /* node counts including boundary nodes; n[2] = 1 in 2D */
  double dx;          /* lattice size [m] */
  double nu;          /* kinematic viscosity [m^2/s] */
  double G[3];        /* body force per unit volume, G = -grad p [N/m^3] */
  int32_t face_kind[6];
  double face_rho[6];
  double face_u[6][3];
} oracle_problem;

/* ---- Lattices ------------------------------------------------------------
 * D2Q9: velocities listed with Eq. (1) [lb.1], in that order; weights 4/9,
 * 1/9 and 1/36 given with Eq. (2).
 * D3Q19: velocities and weights 1/3, 1/18, 1/36 listed at the start of the
 * numerical tests, in that order. */
static const int D2Q9_C[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const real D2Q9_W[9] = {(real)4 / 9,  (real)1 / 9,  (real)1 / 9,
                                 (real)1 / 9,  (real)1 / 9,  (real)1 / 36,
                                 (real)1 / 36, (real)1 / 36, (real)1 / 36};

static const int D3Q19_C[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {-1, 1, 0},
    {1, -1, 0}, {0, 1, 1},   {0, -1, -1}, {0, -1, 1}, {0, 1, -1},
    {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1}};
static const real D3Q19_W[19] = {
    (real)1 / 3,  (real)1 / 18, (real)1 / 18, (real)1 / 18, (real)1 / 18,
    (real)1 / 18, (real)1 / 18, (real)1 / 36, (real)1 / 36, (real)1 / 36,
    (real)1 / 36, (real)1 / 36, (real)1 / 36, (real)1 / 36, (real)1 / 36,
    (real)1 / 36, (real)1 / 36, (real)1 / 36, (real)1 / 36};

static int lattice_dims(int q) { return q == 9 ? 2 : (q == 19 ? 3 : 0); }

static const int (*lattice_c(int q))[3] { return q == 9 ? D2Q9_C : D3Q19_C; }

static const real* lattice_w(int q) { return q == 9 ? D2Q9_W : D3Q19_W; }

/* Copies the velocity set (q x 3 ints) and weights (q reals) out. */
int oracle_lattice(int q, int* c_out, real* w_out) {
  if (lattice_dims(q) == 0) return -1;
  const int(*c)[3] = lattice_c(q);
  const real* w = lattice_w(q);
  for (int a = 0; a < q; ++a) {
    for (int i = 0; i < 3; ++i) c_out[3 * a + i] = c[a][i];
    w_out[a] = w[a];
  }
  return 0;
}

/* Eq. (6) [mlb-viscosity]: particle speed from viscosity and lattice size. */
real oracle_particle_speed(double nu, double dx) { return 6.0 * (real)nu / (real)dx; }

/* Text after Eq. (6): the time step is no longer free, dt = dx / e. */
real oracle_time_step(double nu, double dx) {
  return (real)dx / oracle_particle_speed(nu, dx);
}

/* Eq. (2) [feq-full] for link a, in physical units with e_a = e c_a. */
real oracle_feq(int q, int a, real rho, const real* u, real e) {
  const int(*c)[3] = lattice_c(q);
  const real* w = lattice_w(q);
  const int d = lattice_dims(q);
  real eu = 0.0, uu = 0.0;
  for (int i = 0; i < d; ++i) {
    real ea_i = e * (real)c[a][i];
    eu += ea_i * u[i];
    uu += u[i] * u[i];
  }
  real e2 = e * e;
  return w[a] * rho *
         (1.0 + 3.0 * eu / e2 + 4.5 * eu * eu / (e2 * e2) - 1.5 * uu / e2);
}

/* ---- Geometry helpers ----------------------------------------------------*/
static int validate(const oracle_problem* p) {
  int d = lattice_dims(p->q);
  if (d == 0) return -1;
  if (!(p->dx > 0.0) || !(p->nu > 0.0)) return -1;
  for (int ax = 0; ax < 3; ++ax) {
    if (p->n[ax] < 1) return -1;
    int lo = p->face_kind[2 * ax], hi = p->face_kind[2 * ax + 1];
    if (lo < ORACLE_PERIODIC || lo > ORACLE_PRESSURE) return -1;
    if (hi < ORACLE_PERIODIC || hi > ORACLE_PRESSURE) return -1;
    if ((lo == ORACLE_PERIODIC) != (hi == ORACLE_PERIODIC)) return -1;
    if (ax >= d && (p->n[ax] != 1 || lo != ORACLE_PERIODIC)) return -1;
    if (lo != ORACLE_PERIODIC && p->n[ax] < 3) return -1;
  }
  return 0;
}

/* Index of the lowest-numbered bounded (non-periodic) face the node lies on,
 * or -1: that face owns the node. */
static int fixed_face(const oracle_problem* p, int64_t i, int64_t j,
                      int64_t k) {
  const int64_t idx[3] = {i, j, k};
  for (int f = 0; f < 6; ++f) {
    if (p->face_kind[f] == ORACLE_PERIODIC) continue;
    int ax = f / 2;
    int64_t at = (f % 2 == 0) ? 0 : p->n[ax] - 1;
    if (idx[ax] == at) return f;
  }
  return -1;
}

static int64_t wrap(int64_t v, int64_t n) {
  int64_t r = v % n;
  return r < 0 ? r + n : r;
}

/* The nearest interior node of node (i, j, k): every index on a bounded
 * axis moved into 1 .. n-2. */
static int64_t interior_of(const oracle_problem* p, int64_t i, int64_t j,
                           int64_t k) {
  int64_t idx[3] = {i, j, k};
  for (int ax = 0; ax < 3; ++ax) {
    if (p->face_kind[2 * ax] == ORACLE_PERIODIC) continue;
    if (idx[ax] < 1) idx[ax] = 1;
    if (idx[ax] > p->n[ax] - 2) idx[ax] = p->n[ax] - 2;
  }
  return idx[0] + p->n[0] * (idx[1] + p->n[1] * idx[2]);
}

/* The values a face holds: all of (rho_b, u_b) on a fixed face, u_b on a
 * RHO_NEUMANN face, rho_b on a PRESSURE face. */
static void hold_face_values(const oracle_problem* p, real* rho, real* u) {
  const int d = lattice_dims(p->q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int f = fixed_face(p, i, j, k);
        if (f < 0) continue;
        int64_t x = i + nx * (j + ny * k);
        if (p->face_kind[f] != ORACLE_RHO_NEUMANN) rho[x] = p->face_rho[f];
        if (p->face_kind[f] != ORACLE_PRESSURE)
          for (int c = 0; c < d; ++c) u[c * N + x] = p->face_u[f][c];
      }
}

/* The zero-normal-gradient values: the density of a RHO_NEUMANN node and the
 * velocity of a PRESSURE node are those of its nearest interior node. */
static void copy_from_interior(const oracle_problem* p, real* rho,
                               real* u) {
  const int d = lattice_dims(p->q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int f = fixed_face(p, i, j, k);
        if (f < 0 || p->face_kind[f] == ORACLE_FIXED) continue;
        int64_t x = i + nx * (j + ny * k);
        int64_t s = interior_of(p, i, j, k);
        if (p->face_kind[f] == ORACLE_RHO_NEUMANN)
          rho[x] = rho[s];
        else
          for (int c = 0; c < d; ++c) u[c * N + x] = u[c * N + s];
      }
}

/* Writes the boundary values into every boundary node: what each face
 * holds, then the values its kind takes from the interior. */
int oracle_impose_boundary(const oracle_problem* p, real* rho, real* u) {
  if (validate(p)) return -1;
  hold_face_values(p, rho, u);
  copy_from_interior(p, rho, u);
  return 0;
}

/* Eqs. (4)-(5) at one non-fixed node (i, j, k): gathers the equilibria of
 * the upstream nodes and returns the new density and velocity. */
static void update_node(const oracle_problem* p, real e, real dt,
                        const real* rho, const real* u, int64_t i,
                        int64_t j, int64_t k, real* rho_out,
                        real* u_out) {
  const int q = p->q, d = lattice_dims(q);
  const int(*c)[3] = lattice_c(q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  real r = 0.0;
  real m[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < q; ++a) {
    /* Source node x - e_a dt = x - c_a. */
    int64_t si = wrap(i - c[a][0], nx);
    int64_t sj = wrap(j - c[a][1], ny);
    int64_t sk = wrap(k - c[a][2], nz);
    int64_t s = si + nx * (sj + ny * sk);
    real us[3] = {0.0, 0.0, 0.0};
    for (int cc = 0; cc < d; ++cc) us[cc] = u[cc * N + s];
    real f = oracle_feq(q, a, rho[s], us, e);
    r += f;                                     /* Eq. (4) */
    for (int cc = 0; cc < d; ++cc) m[cc] += e * (real)c[a][cc] * f;
  }
  *rho_out = r;
  for (int cc = 0; cc < d; ++cc) {
    /* Eq. (5) plus the body-force term of test 2 (sign per G). */
    u_out[cc] = m[cc] / r + dt * p->G[cc] / r;
  }
}

/* One MacLAB step from (rho, u) into (rho_new, u_new). */
static void step_once(const oracle_problem* p, real e, real dt,
                      const real* rho, const real* u, real* rho_new,
                      real* u_new) {
  const int d = lattice_dims(p->q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const int64_t x = i + nx * (j + ny * k);
        if (fixed_face(p, i, j, k) >= 0) {
          /* Recipe step (iv): boundary nodes keep their physical values. */
          rho_new[x] = rho[x];
          for (int cc = 0; cc < d; ++cc) u_new[cc * N + x] = u[cc * N + x];
          continue;
        }
        real un[3];
        update_node(p, e, dt, rho, u, i, j, k, &rho_new[x], un);
        for (int cc = 0; cc < d; ++cc) u_new[cc * N + x] = un[cc];
      }
  /* faces with a zero-normal-gradient quantity take it from the new state */
  copy_from_interior(p, rho_new, u_new);
}

/* One step evaluated only at the listed nodes (flat indices): rho_out[s] and
 * u_out[c * count + s] receive the values after the step. Fixed nodes keep
 * their values. For checking large lattices on a sample of nodes. */
int oracle_step_at(const oracle_problem* p, const real* rho,
                   const real* u, const int64_t* nodes, int64_t count,
                   real* rho_out, real* u_out) {
  if (validate(p) || count < 0) return -1;
  const int d = lattice_dims(p->q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  const real e = oracle_particle_speed(p->nu, p->dx);
  const real dt = p->dx / e;
  for (int64_t s = 0; s < count; ++s) {
    const int64_t x = nodes[s];
    if (x < 0 || x >= N) return -1;
    const int64_t i = x % nx, j = (x / nx) % ny, k = x / (nx * ny);
    real un[3] = {0.0, 0.0, 0.0};
    const int f = fixed_face(p, i, j, k);
    if (f >= 0) {
      rho_out[s] = rho[x];
      for (int cc = 0; cc < d; ++cc) un[cc] = u[cc * N + x];
      if (p->face_kind[f] != ORACLE_FIXED) {
        /* the copied quantity is the new value at the nearest interior node */
        const int64_t t = interior_of(p, i, j, k);
        real rt, ut[3] = {0.0, 0.0, 0.0};
        update_node(p, e, dt, rho, u, t % nx, (t / nx) % ny, t / (nx * ny), &rt, ut);
        if (p->face_kind[f] == ORACLE_RHO_NEUMANN)
          rho_out[s] = rt;
        else
          for (int cc = 0; cc < d; ++cc) un[cc] = ut[cc];
      }
    } else {
      update_node(p, e, dt, rho, u, i, j, k, &rho_out[s], un);
    }
    for (int cc = 0; cc < d; ++cc) u_out[cc * count + s] = un[cc];
  }
  return 0;
}

/* Advances (rho, u) in place by `steps` time steps. rho has N = nx*ny*nz
 * entries, u has d planes of N entries (component-major), x fastest.
 * Boundary values must already be in the arrays (oracle_impose_boundary).
 * Returns 0, or -1 on an invalid problem, -2 on allocation failure. */
int oracle_run(const oracle_problem* p, real* rho, real* u,
               int64_t steps) {
  if (validate(p) || steps < 0) return -1;
  const int d = lattice_dims(p->q);
  const int64_t N = p->n[0] * p->n[1] * p->n[2];
  const real e = oracle_particle_speed(p->nu, p->dx);
  const real dt = p->dx / e;
  real* r2 = (real*)malloc(sizeof(real) * (size_t)N);
  real* u2 = (real*)malloc(sizeof(real) * (size_t)(N * d));
  if (!r2 || !u2) {
    free(r2);
    free(u2);
    return -2;
  }
  for (int64_t s = 0; s < steps; ++s) {
    step_once(p, e, dt, rho, u, r2, u2);
    memcpy(rho, r2, sizeof(real) * (size_t)N);
    memcpy(u, u2, sizeof(real) * (size_t)(N * d));
  }
  free(r2);
  free(u2);
  return 0;
}

/* ---- Diagnostics ---------------------------------------------------------
 * Mass M = sum rho, momentum P = sum rho u, kinetic energy
 * E = 1/2 sum rho |u|^2 over all nodes (the conserved moments of the
 * equilibrium, Methods, Eqs. (14)-(15)), the largest |u|/e (the Mach number
 * the paper's validity condition refers to), and the number of nodes holding
 * a non-finite value. Sums use Neumaier's compensated summation. */
typedef struct {
  real s, c;
} neumaier;

static void nsum_add(neumaier* a, real v) {
  real t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

int oracle_diagnostics(const oracle_problem* p, const real* rho,
                       const real* u, real* out7) {
  if (validate(p)) return -1;
  const int d = lattice_dims(p->q);
  const int64_t N = p->n[0] * p->n[1] * p->n[2];
  const real e = oracle_particle_speed(p->nu, p->dx);
  neumaier M = {0, 0}, P[3] = {{0, 0}, {0, 0}, {0, 0}}, E = {0, 0};
  real umax = 0.0, bad = 0.0;
  for (int64_t x = 0; x < N; ++x) {
    int finite = isfinite(rho[x]);
    real uu = 0.0;
    for (int c = 0; c < d; ++c) {
      finite = finite && isfinite(u[c * N + x]);
      uu += u[c * N + x] * u[c * N + x];
    }
    if (!finite) {
      bad += 1.0;
      continue;
    }
    nsum_add(&M, rho[x]);
    for (int c = 0; c < d; ++c) nsum_add(&P[c], rho[x] * u[c * N + x]);
    nsum_add(&E, 0.5 * rho[x] * uu);
    real m = sqrt(uu) / e;
    if (m > umax) umax = m;
  }
  out7[0] = M.s + M.c;
  for (int c = 0; c < 3; ++c) out7[1 + c] = P[c].s + P[c].c;
  out7[4] = E.s + E.c;
  out7[5] = umax;
  out7[6] = bad;
  return 0;
}

/* ---- Reverse-mode derivative ---------------------------------------------
 * Gradient of L = sum_x sum_i (u_i(x, T) - u_target_i(x))^2 (u after `steps`
 * steps) with respect to the initial velocity u(x, 0) and the body force G,
 * by the chain rule applied backwards through the steps above, written in
 * the same physical units:
 *   m'(x)   = sum_a e_a f_a(x - c_a) + dt G,      u'(x) = m'(x) / rho'(x)
 *     -> mbar(x) = ubar'(x) / rho'(x),
 *        rbar_tot(x) = rhobar'(x) - ubar'(x) . u'(x) / rho'(x),
 *        Gbar += dt sum_x mbar(x)
 *   rho'(x) = sum_a f_a(x - c_a),  m' = sum_a e_a f_a(x - c_a)
 *     -> fbar_a(y) = rbar_tot(y + c_a) + e_a . mbar(y + c_a)
 *   f_a(y)  = w_a rho (1 + 3 e_a.u/e^2 + 9/2 (e_a.u)^2/e^4 - 3/2 u.u/e^2)
 *     -> rhobar(y) = sum_a fbar_a f_a / rho,
 *        ubar(y)   = sum_a fbar_a w_a rho (3 e_a/e^2 + 9 (e_a.u) e_a/e^4
 *                                          - 3 u/e^2)
 * Fixed nodes hold constants: nothing flows through them (their rbar_tot
 * and mbar are zero, and their own adjoint is zero).
 * The whole trajectory is stored (steps + 1 states): for small problems only.
 * Outputs: grad_u0 (d planes of N), grad_G[3], loss[1]. Returns 0, -1 on an
 * invalid problem, -2 on allocation failure. */
int oracle_adjoint_run(const oracle_problem* p, const real* rho0,
                       const real* u0, int64_t steps,
                       const real* u_target, real* grad_u0,
                       real* grad_G, real* loss) {
  if (validate(p) || steps < 0) return -1;
  /* reverse mode covers periodic and fixed faces */
  for (int f = 0; f < 6; ++f)
    if (p->face_kind[f] == ORACLE_RHO_NEUMANN || p->face_kind[f] == ORACLE_PRESSURE) return -1;
  const int q = p->q, d = lattice_dims(q);
  const int(*c)[3] = lattice_c(q);
  const real* w = lattice_w(q);
  const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const int64_t N = nx * ny * nz;
  const real e = oracle_particle_speed(p->nu, p->dx);
  const real dt = p->dx / e;
  const size_t S = (size_t)(N * (d + 1));
  real* traj = (real*)malloc(sizeof(real) * S * (size_t)(steps + 1));
  real* rb = (real*)malloc(sizeof(real) * (size_t)N);      /* rhobar */
  real* ub = (real*)malloc(sizeof(real) * (size_t)(N * d)); /* ubar */
  real* rt = (real*)malloc(sizeof(real) * (size_t)N);      /* rbar_tot */
  real* mb = (real*)malloc(sizeof(real) * (size_t)(N * d)); /* mbar */
  if (!traj || !rb || !ub || !rt || !mb) {
    free(traj); free(rb); free(ub); free(rt); free(mb);
    return -2;
  }
  /* forward, keeping every state: state n = [rho (N) | u (d N)] */
  memcpy(traj, rho0, sizeof(real) * (size_t)N);
  memcpy(traj + N, u0, sizeof(real) * (size_t)(N * d));
  oracle_impose_boundary(p, traj, traj + N);
  for (int64_t s = 0; s < steps; ++s) {
    real* cur = traj + S * (size_t)s;
    real* nxt = traj + S * (size_t)(s + 1);
    step_once(p, e, dt, cur, cur + N, nxt, nxt + N);
  }
  /* loss and its derivative with respect to the final velocity */
  const real* fin = traj + S * (size_t)steps;
  real L = 0.0;
  for (int64_t x = 0; x < N; ++x) {
    rb[x] = 0.0;
    for (int cc = 0; cc < d; ++cc) {
      real diff = fin[N + cc * N + x] - u_target[cc * N + x];
      L += diff * diff;
      ub[cc * N + x] = 2.0 * diff;
    }
  }
  *loss = L;
  for (int cc = 0; cc < 3; ++cc) grad_G[cc] = 0.0;
  for (int64_t s = steps - 1; s >= 0; --s) {
    const real* cur = traj + S * (size_t)s;       /* state n     */
    const real* nxt = traj + S * (size_t)(s + 1); /* state n + 1 */
    /* through u' = m' / rho' */
    for (int64_t k = 0; k < nz; ++k)
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const int64_t x = i + nx * (j + ny * k);
          if (fixed_face(p, i, j, k) >= 0) {
            rt[x] = 0.0;
            for (int cc = 0; cc < d; ++cc) mb[cc * N + x] = 0.0;
            continue;
          }
          real r1 = nxt[x], dot = 0.0;
          for (int cc = 0; cc < d; ++cc) {
            mb[cc * N + x] = ub[cc * N + x] / r1;
            dot += ub[cc * N + x] * nxt[N + cc * N + x];
            grad_G[cc] += dt * mb[cc * N + x];
          }
          rt[x] = rb[x] - dot / r1;
        }
    /* through the gather and the equilibrium at the upstream nodes */
    for (int64_t k = 0; k < nz; ++k)
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const int64_t y = i + nx * (j + ny * k);
          real rho = cur[y];
          real uu[3] = {0.0, 0.0, 0.0};
          for (int cc = 0; cc < d; ++cc) uu[cc] = cur[N + cc * N + y];
          real rbar = 0.0, ubar[3] = {0.0, 0.0, 0.0};
          for (int a = 0; a < q; ++a) {
            int64_t xi = wrap(i + c[a][0], nx);
            int64_t xj = wrap(j + c[a][1], ny);
            int64_t xk = wrap(k + c[a][2], nz);
            int64_t x = xi + nx * (xj + ny * xk);
            real fbar = rt[x];
            for (int cc = 0; cc < d; ++cc) fbar += e * (real)c[a][cc] * mb[cc * N + x];
            real f = oracle_feq(q, a, rho, uu, e);
            rbar += fbar * f / rho;
            real eu = 0.0;
            for (int cc = 0; cc < d; ++cc) eu += e * (real)c[a][cc] * uu[cc];
            for (int cc = 0; cc < d; ++cc) {
              real ea = e * (real)c[a][cc];
              ubar[cc] += fbar * w[a] * rho *
                          (3.0 * ea / (e * e) + 9.0 * eu * ea / (e * e * e * e) -
                           3.0 * uu[cc] / (e * e));
            }
          }
          if (fixed_face(p, i, j, k) >= 0) {
            rbar = 0.0;
            for (int cc = 0; cc < d; ++cc) ubar[cc] = 0.0;
          }
          rb[y] = rbar;
          for (int cc = 0; cc < d; ++cc) ub[cc * N + y] = ubar[cc];
        }
  }
  memcpy(grad_u0, ub, sizeof(real) * (size_t)(N * d));
  free(traj); free(rb); free(ub); free(rt); free(mb);
  return 0;
}
