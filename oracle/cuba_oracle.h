/*
 * cuba_oracle.h -- CPU oracle for the per-time-step particle-in-cell (PIC)
 * Boltzmann update of "CuBA - a CUDA implementation of BAMPS"
 * (Cardoso, Bicudo, Eilhauer, Bouras; arXiv:1208.0961).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, sequential FP64
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, constant or helper with the HIP library; the two
 * meet only through the seeded input generator and through their outputs.
 *
 * All arrays are indexed by particle id (the index in the caller's arrays);
 * the oracle never permutes them.  Every floating-point expression is
 * written in the evaluation order that defines the method's result; build
 * with -O2 -ffp-contract=off and without -ffast-math.
 */
#ifndef CUBA_ORACLE_H
#define CUBA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem definition (Sec. 2 of the paper: box, cells, sigma, test-particle
 * ratio, time step).  Walls sit at 0 and box[d] on each axis. */
typedef struct {
  double box[3];     /* Lx, Ly, Lz [fm]                                   */
  int32_t cells[3];  /* nx, ny, nz; cell edge dx_d = L_d / n_d            */
  double sigma;      /* total isotropic cross section [fm^2]              */
  double r_test;     /* test particles per physical particle              */
  double dt;         /* time step [fm/c]                                  */
  uint64_t seed;     /* Philox key: low word = key[0], high word = key[1] */
} orc_params;

/* Optional per-step record used by the parity tests.  Any pointer may be
 * NULL.  cand / claim hold (cell, a, b) triples with a < b local canonical
 * indices; counts are written to n_cand / n_claim even when the arrays are
 * too small (then only the first *_cap triples are stored). */
typedef struct {
  uint32_t *cell;     /* [n]   cell of each particle (by id)             */
  uint32_t *perm;     /* [n]   ids in canonical (cell, id) order          */
  uint32_t *offsets;  /* [C+1] start of each cell in perm                 */
  uint32_t *cand;     /* [3*cand_cap]  every pair with u < P22, judged on
                         the momenta the cell held before its collisions   */
  int64_t cand_cap;
  int64_t n_cand;
  uint32_t *claim;    /* [3*claim_cap] pairs that scattered, in order     */
  int64_t claim_cap;
  int64_t n_claim;
} orc_trace;

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,  /* bad parameters                                  */
  ORC_ERANGE = -2,  /* particle outside the box, non-finite, |p| = 0,
                       or a cell too full for a 32-bit pair index       */
  ORC_ENOMEM = -3
};

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): one block of four
 * 32-bit words for counter ctr and key key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Uniform in [0,1) with 53 bits: ((hi:lo) >> 11) * 2^-53. */
double orc_u53(uint32_t lo, uint32_t hi);

/* Derived constants: cell edges, cell volume and K = sigma/r_test*dt/V. */
void orc_constants(const orc_params *p, double dx[3], double *vcell,
                   double *kfac);

/* Parameter and state checks; ORC_OK or a negative code. */
int orc_check(const orc_params *p, int64_t n, const double *x,
              const double *y, const double *z, const double *px,
              const double *py, const double *pz);

/* One time step with index t, in place.  nthreads > 1 spreads the
 * (independent) cells over POSIX threads; the result does not depend on
 * it.  A trace needs nthreads == 1. */
int orc_step(const orc_params *p, int64_t n, double *x, double *y, double *z,
             double *px, double *py, double *pz, uint32_t t, int nthreads,
             orc_trace *tr);

/* nsteps steps with indices t0, t0+1, ... */
int orc_run(const orc_params *p, int64_t n, double *x, double *y, double *z,
            double *px, double *py, double *pz, uint32_t t0, int32_t nsteps,
            int nthreads);

/* Lab-frame profiles over the nx slabs along x [GeV/fm^3]:
 * T00[ix] = sum E / (r_test dx Ly Lz), T0x[ix] = sum p_x / (same). */
void orc_observe(const orc_params *p, int64_t n, const double *x,
                 const double *px, const double *py, const double *pz,
                 double *T00, double *T0x);

/* Moments of the distribution over the nx slabs along x (the observables of
 * the sigma scan, Sec. 5 / Fig. 3: the approach to ideal hydrodynamics):
 * T00, T0x as orc_observe, T^xx[ix] = sum p_x^2 / E / (r_test dx Ly Lz)
 * [GeV/fm^3] and the density n[ix] = count / (r_test dx Ly Lz) [fm^-3] of
 * physical particles. */
void orc_observe_moments(const orc_params *p, int64_t n, const double *x,
                         const double *px, const double *py, const double *pz,
                         double *T00, double *T0x, double *Txx, double *nd);

/* Rest frame of each slab (the Landau frame of the t-x block of T^{mu nu},
 * a reading: transverse flow is absent in the tube): the energy density e
 * and velocity v with T^{mu nu} u_nu = e u^mu, u = gamma (1, v):
 *   e = ((T00 - Txx) + sqrt((T00 + Txx - 2|T0x|)(T00 + Txx + 2|T0x|))) / 2,
 *   v = T0x / (e + Txx).
 * For an ideal fluid (T00 = (e+p) g^2 - p, T0x = (e+p) g^2 v,
 * Txx = (e+p) g^2 v^2 + p) this returns its e and v. */
void orc_landau(int32_t nx, const double *T00, const double *T0x, const double *Txx,
                double *e, double *v);

/* The collision of one cell with caller-supplied uniforms (for brute-force
 * tests of the claim rule).  The cell's members, in canonical order, are
 * given by their momenta (updated in place).  u_acc[k] is the acceptance
 * uniform of pair k (lexicographic index); u_kin[2k], u_kin[2k+1] are the
 * polar and azimuthal uniforms of its outgoing direction.  Accepted pairs
 * are written to acc_a/acc_b (capacity n/2); returns their count. */
int orc_collide_cell_with_uniforms(int32_t nc, double *px, double *py,
                                   double *pz, double kfac,
                                   const double *u_acc, const double *u_kin,
                                   int32_t *acc_a, int32_t *acc_b);

/* The CM-frame 2->2 kinematics of one accepted pair, in place. */
void orc_scatter_pair(double *pa, double *pb, double uc, double uphi);

#ifdef __cplusplus
}
#endif
#endif
