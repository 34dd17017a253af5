/*
 * cuba_oracle.c -- CPU oracle for the per-time-step PIC Boltzmann update of
 * arXiv:1208.0961 ("CuBA - a CUDA implementation of BAMPS").
 *
 * TEST INFRASTRUCTURE ONLY (see cuba_oracle.h).  Plain sequential FP64 code
 * written from the method's description; shares nothing with the HIP path.
 *
 * One step, in the order the method prescribes (Sec. 2):
 *   1. free streaming, Eq. (2):        x_d <- x_d + (p_d / E) dt,  E = |p|
 *   2. elastic reflection at the six walls of the box (end of Sec. 2)
 *   3. cell of each particle, cells of volume dx dy dz (Sec. 2, PIC method)
 *   4. particles of each cell listed in ascending id (a stable counting sort)
 *   5. every same-cell pair (a < b, lexicographic) is tested with
 *      P22 = v_rel sigma / r_test * dt / V_cell, v_rel = s / (2 E1 E2),
 *      Eq. (3) with the test-particle rescaling of Sec. 2; a particle
 *      scatters at most once per step: a pair whose member has already
 *      scattered in this step is skipped (a reading: the paper is silent)
 *   6. an accepted pair is boosted to its CM frame, given an isotropic
 *      direction there with |p*| = sqrt(s)/2, and boosted back (Sec. 2).
 *
 * Random numbers are Philox4x32-10 blocks keyed by the seed, with counter
 * (pair index k, cell c, step t, purpose): purpose 0 decides acceptance,
 * purpose 1 draws the outgoing direction.  This keyed choice is a reading
 * (the paper says only "Monte-Carlo"); it makes the result independent of
 * the order in which pairs are evaluated.
 */
#include "cuba_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4.2): ten rounds of two       */
/* 32x32->64 multiplies; the key is bumped by the Weyl constants between   */
/* rounds.                                                                  */
/* ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

double orc_u53(uint32_t lo, uint32_t hi) {
  uint64_t bits = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)bits * 0x1p-53;
}

/* ---------------------------------------------------------------------- */
/* Constants and checks                                                    */
/* ---------------------------------------------------------------------- */
void orc_constants(const orc_params *p, double dx[3], double *vcell,
                   double *kfac) {
  for (int d = 0; d < 3; ++d) dx[d] = p->box[d] / (double)p->cells[d];
  double v = (dx[0] * dx[1]) * dx[2];
  if (vcell) *vcell = v;
  /* Eq. (3) with N_test read as r_test: K = ((sigma / r_test) * dt) / V */
  if (kfac) *kfac = ((p->sigma / p->r_test) * p->dt) / v;
}

static double energy(double px, double py, double pz) {
  return sqrt((px * px + py * py) + pz * pz);
}

int orc_check(const orc_params *p, int64_t n, const double *x,
              const double *y, const double *z, const double *px,
              const double *py, const double *pz) {
  double dx[3], v, kf;
  if (n < 0) return ORC_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!(isfinite(p->box[d]) && p->box[d] > 0.0)) return ORC_EINVAL;
    if (p->cells[d] < 1) return ORC_EINVAL;
  }
  if (!(isfinite(p->sigma) && p->sigma >= 0.0)) return ORC_EINVAL;
  if (!(isfinite(p->r_test) && p->r_test > 0.0)) return ORC_EINVAL;
  if (!(isfinite(p->dt) && p->dt > 0.0)) return ORC_EINVAL;
  orc_constants(p, dx, &v, &kf);
  /* Sec. 5: dt is chosen below the cell size (at most one cell per step). */
  for (int d = 0; d < 3; ++d)
    if (!(p->dt < dx[d])) return ORC_EINVAL;
  /* v_rel <= 2, so P22 <= 2K must stay a probability. */
  if (!(2.0 * kf <= 1.0)) return ORC_EINVAL;
  const double *r[3] = {x, y, z};
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) {
      double q = r[d][i];
      if (!(isfinite(q) && q >= 0.0 && q <= p->box[d])) return ORC_ERANGE;
    }
    if (!(isfinite(px[i]) && isfinite(py[i]) && isfinite(pz[i])))
      return ORC_ERANGE;
    if (!(energy(px[i], py[i], pz[i]) > 0.0)) return ORC_ERANGE;
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Kinematics of an accepted pair (Sec. 2): boost to the CM frame, choose  */
/* an isotropic direction there, boost back.                               */
/* ---------------------------------------------------------------------- */
void orc_scatter_pair(double *pa, double *pb, double uc, double uphi) {
  const double two_pi = 6.283185307179586;
  double ea = energy(pa[0], pa[1], pa[2]);
  double eb = energy(pb[0], pb[1], pb[2]);
  double dot = (pa[0] * pb[0] + pa[1] * pb[1]) + pa[2] * pb[2];
  double e12 = ea * eb;
  /* Mandelstam s = 2 (E1 E2 - p1.p2) for massless particles.  For a small
   * opening angle the difference cancels; there the identity
   * (E1E2)^2 - (p1.p2)^2 = |p1 x p2|^2 gives the same s without it. */
  double s;
  if (dot > 0.0) {
    double cx = pa[1] * pb[2] - pa[2] * pb[1];
    double cy = pa[2] * pb[0] - pa[0] * pb[2];
    double cz = pa[0] * pb[1] - pa[1] * pb[0];
    double cross2 = (cx * cx + cy * cy) + cz * cz;
    s = (2.0 * cross2) / (e12 + dot);
  } else {
    s = 2.0 * (e12 - dot);
  }
  if (!(s > 0.0)) return; /* collinear pair: no CM frame, leave unchanged */
  double et = ea + eb;
  double ptot[3] = {pa[0] + pb[0], pa[1] + pb[1], pa[2] + pb[2]};
  double rs = sqrt(s);
  double gamma = et / rs;
  double beta[3] = {ptot[0] / et, ptot[1] / et, ptot[2] / et};
  double estar = rs * 0.5;

  /* isotropic direction in the CM frame, axes parallel to the lab axes */
  double cth = 2.0 * uc - 1.0;
  double sth = sqrt((1.0 - cth) * (1.0 + cth));
  double phi = two_pi * uphi;
  double dir[3] = {sth * cos(phi), sth * sin(phi), cth};
  double q[3] = {estar * dir[0], estar * dir[1], estar * dir[2]};

  /* boost back: p = q + beta (gamma^2/(gamma+1) (beta.q) + gamma E*) */
  double g2 = (gamma * gamma) / (gamma + 1.0);
  double bq = (beta[0] * q[0] + beta[1] * q[1]) + beta[2] * q[2];
  double fa = g2 * bq + gamma * estar;
  double fb = g2 * (-bq) + gamma * estar;
  for (int d = 0; d < 3; ++d) {
    pa[d] = q[d] + beta[d] * fa;
    pb[d] = (-q[d]) + beta[d] * fb;
  }
}

/* ---------------------------------------------------------------------- */
/* The collision of one cell.                                               */
/* ---------------------------------------------------------------------- */
typedef struct {
  /* acceptance uniform of pair k */
  double (*u_acc)(const void *ctx, uint64_t k);
  /* polar and azimuthal uniforms of pair k's outgoing direction */
  void (*u_kin)(const void *ctx, uint64_t k, double *uc, double *uphi);
  const void *ctx;
} draws_t;

typedef struct {
  uint32_t key[2];
  uint32_t cell;
  uint32_t step;
} philox_draws_ctx;

static double philox_u_acc(const void *vctx, uint64_t k) {
  const philox_draws_ctx *c = (const philox_draws_ctx *)vctx;
  uint32_t ctr[4] = {(uint32_t)k, c->cell, c->step, 0u}, w[4];
  orc_philox4x32_10(ctr, c->key, w);
  return orc_u53(w[0], w[1]);
}

static void philox_u_kin(const void *vctx, uint64_t k, double *uc,
                         double *uphi) {
  const philox_draws_ctx *c = (const philox_draws_ctx *)vctx;
  uint32_t ctr[4] = {(uint32_t)k, c->cell, c->step, 1u}, w[4];
  orc_philox4x32_10(ctr, c->key, w);
  *uc = orc_u53(w[0], w[1]);
  *uphi = orc_u53(w[2], w[3]);
}

typedef struct {
  const double *u_acc;
  const double *u_kin;
} array_draws_ctx;

static double array_u_acc(const void *vctx, uint64_t k) {
  return ((const array_draws_ctx *)vctx)->u_acc[k];
}

static void array_u_kin(const void *vctx, uint64_t k, double *uc,
                        double *uphi) {
  const array_draws_ctx *c = (const array_draws_ctx *)vctx;
  *uc = c->u_kin[2 * k];
  *uphi = c->u_kin[2 * k + 1];
}

/* Lexicographic index of pair (a, b), a < b, among the n(n-1)/2 pairs. */
static uint64_t pair_index(uint64_t a, uint64_t b, uint64_t nc) {
  return a * (2 * nc - a - 1) / 2 + (b - a - 1);
}

/* Eq. (3): does pair (a, b) collide, given its acceptance uniform u? */
static int pair_accepts(const double *pa, const double *pb, double kfac,
                        double u) {
  double ea = energy(pa[0], pa[1], pa[2]);
  double eb = energy(pb[0], pb[1], pb[2]);
  double dot = (pa[0] * pb[0] + pa[1] * pb[1]) + pa[2] * pb[2];
  double e12 = ea * eb;
  double s = 2.0 * (e12 - dot);
  double vrel = s / (2.0 * e12);
  double p22 = vrel * kfac;
  return u < p22;
}

/* Collide the nc members of one cell.  mom[3*j..] is the momentum of the
 * member with canonical index j, read and written through the accessor
 * arrays mx/my/mz at indices ids[j].  claimed is scratch of size nc. */
typedef struct {
  double *px, *py, *pz;
} mom_arrays;

static void get_p(const mom_arrays *m, int64_t i, double p[3]) {
  p[0] = m->px[i];
  p[1] = m->py[i];
  p[2] = m->pz[i];
}

static void set_p(const mom_arrays *m, int64_t i, const double p[3]) {
  m->px[i] = p[0];
  m->py[i] = p[1];
  m->pz[i] = p[2];
}

static int collide_cell(int64_t nc, const int64_t *ids, const mom_arrays *m,
                        double kfac, const draws_t *dr, unsigned char *claimed,
                        uint32_t cell, orc_trace *tr, int32_t *acc_a,
                        int32_t *acc_b) {
  int nacc = 0;
  if (nc < 2) return 0;
  /* Record only: every pair with u < P22 on the momenta before any of the
   * cell's collisions (what the claim rule below chooses among). */
  if (tr) {
    for (int64_t a = 0; a + 1 < nc; ++a) {
      for (int64_t b = a + 1; b < nc; ++b) {
        double pa[3], pb[3];
        uint64_t k = pair_index((uint64_t)a, (uint64_t)b, (uint64_t)nc);
        get_p(m, ids[a], pa);
        get_p(m, ids[b], pb);
        if (pair_accepts(pa, pb, kfac, dr->u_acc(dr->ctx, k))) {
          if (tr->cand && tr->n_cand < tr->cand_cap) {
            tr->cand[3 * tr->n_cand + 0] = cell;
            tr->cand[3 * tr->n_cand + 1] = (uint32_t)a;
            tr->cand[3 * tr->n_cand + 2] = (uint32_t)b;
          }
          tr->n_cand++;
        }
      }
    }
  }
  memset(claimed, 0, (size_t)nc);
  for (int64_t a = 0; a + 1 < nc; ++a) {
    for (int64_t b = a + 1; b < nc; ++b) {
      if (claimed[a] || claimed[b]) continue; /* at most one scattering */
      double pa[3], pb[3];
      uint64_t k = pair_index((uint64_t)a, (uint64_t)b, (uint64_t)nc);
      get_p(m, ids[a], pa);
      get_p(m, ids[b], pb);
      if (!pair_accepts(pa, pb, kfac, dr->u_acc(dr->ctx, k))) continue;
      double uc, uphi;
      dr->u_kin(dr->ctx, k, &uc, &uphi);
      orc_scatter_pair(pa, pb, uc, uphi);
      set_p(m, ids[a], pa);
      set_p(m, ids[b], pb);
      claimed[a] = 1;
      claimed[b] = 1;
      if (acc_a) {
        acc_a[nacc] = (int32_t)a;
        acc_b[nacc] = (int32_t)b;
      }
      nacc++;
      if (tr) {
        if (tr->claim && tr->n_claim < tr->claim_cap) {
          tr->claim[3 * tr->n_claim + 0] = cell;
          tr->claim[3 * tr->n_claim + 1] = (uint32_t)a;
          tr->claim[3 * tr->n_claim + 2] = (uint32_t)b;
        }
        tr->n_claim++;
      }
    }
  }
  return nacc;
}

int orc_collide_cell_with_uniforms(int32_t nc, double *px, double *py,
                                   double *pz, double kfac,
                                   const double *u_acc, const double *u_kin,
                                   int32_t *acc_a, int32_t *acc_b) {
  if (nc < 0) return ORC_EINVAL;
  int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
  unsigned char *claimed = (unsigned char *)malloc((size_t)nc + 1);
  if (!ids || !claimed) {
    free(ids);
    free(claimed);
    return ORC_ENOMEM;
  }
  for (int32_t j = 0; j < nc; ++j) ids[j] = j;
  array_draws_ctx actx = {u_acc, u_kin};
  draws_t dr = {array_u_acc, array_u_kin, &actx};
  mom_arrays m = {px, py, pz};
  int nacc = collide_cell(nc, ids, &m, kfac, &dr, claimed, 0u, NULL, acc_a,
                          acc_b);
  free(ids);
  free(claimed);
  return nacc;
}

/* ---------------------------------------------------------------------- */
/* Streaming, reflection, binning                                          */
/* ---------------------------------------------------------------------- */
static void stream_reflect(const orc_params *p, int64_t n, double *x,
                           double *y, double *z, double *px, double *py,
                           double *pz) {
  double *r[3] = {x, y, z};
  double *q[3] = {px, py, pz};
  for (int64_t i = 0; i < n; ++i) {
    double e = energy(px[i], py[i], pz[i]);
    for (int d = 0; d < 3; ++d) {
      /* Eq. (2): x <- x + c^2 p_x / E dt  (c = 1); E = 0 does not move */
      if (e != 0.0) {
        double v = q[d][i] / e;
        r[d][i] = r[d][i] + v * p->dt;
      }
      /* elastic reflection: mirror the overshoot, flip the normal p */
      double L = p->box[d];
      if (r[d][i] < 0.0) {
        r[d][i] = -r[d][i];
        q[d][i] = -q[d][i];
      } else if (r[d][i] > L) {
        r[d][i] = 2.0 * L - r[d][i];
        q[d][i] = -q[d][i];
      }
    }
  }
}

static int32_t axis_cell(double xd, double dxd, int32_t nd) {
  int32_t i = (int32_t)floor(xd / dxd);
  if (i < 0) i = 0;
  if (i > nd - 1) i = nd - 1;
  return i;
}

static uint32_t cell_of(const orc_params *p, const double dx[3], double xx,
                        double yy, double zz) {
  int32_t ix = axis_cell(xx, dx[0], p->cells[0]);
  int32_t iy = axis_cell(yy, dx[1], p->cells[1]);
  int32_t iz = axis_cell(zz, dx[2], p->cells[2]);
  return (uint32_t)(((int64_t)ix * p->cells[1] + iy) * p->cells[2] + iz);
}

/* ---------------------------------------------------------------------- */
/* Threads over cells (timing only; the result does not depend on them)   */
/* ---------------------------------------------------------------------- */
typedef struct {
  const orc_params *p;
  const int64_t *list;
  const int64_t *off;
  int64_t ncells;
  mom_arrays m;
  double kfac;
  uint32_t t;
  int64_t max_occ;
  int64_t chunk; /* cells taken per grab */
  int64_t next;  /* shared cursor, guarded by mu */
  pthread_mutex_t mu;
} collide_job;

static void *collide_worker(void *arg) {
  collide_job *J = (collide_job *)arg;
  unsigned char *claimed = (unsigned char *)malloc((size_t)J->max_occ + 1);
  philox_draws_ctx pctx;
  pctx.key[0] = (uint32_t)J->p->seed;
  pctx.key[1] = (uint32_t)(J->p->seed >> 32);
  pctx.step = J->t;
  draws_t dr = {philox_u_acc, philox_u_kin, &pctx};
  for (;;) {
    int64_t c0, c1;
    pthread_mutex_lock(&J->mu);
    c0 = J->next;
    J->next += J->chunk;
    pthread_mutex_unlock(&J->mu);
    if (c0 >= J->ncells) break;
    c1 = c0 + J->chunk < J->ncells ? c0 + J->chunk : J->ncells;
    for (int64_t c = c0; c < c1; ++c) {
      pctx.cell = (uint32_t)c;
      collide_cell(J->off[c + 1] - J->off[c], J->list + J->off[c], &J->m,
                   J->kfac, &dr, claimed, (uint32_t)c, NULL, NULL, NULL);
    }
  }
  free(claimed);
  return NULL;
}

/* ---------------------------------------------------------------------- */
/* One step                                                                */
/* ---------------------------------------------------------------------- */
int orc_step(const orc_params *p, int64_t n, double *x, double *y, double *z,
             double *px, double *py, double *pz, uint32_t t, int nthreads,
             orc_trace *tr) {
  double dx[3], vcell, kfac;
  int64_t ncells =
      (int64_t)p->cells[0] * (int64_t)p->cells[1] * (int64_t)p->cells[2];
  if (tr && nthreads > 1) return ORC_EINVAL;
  orc_constants(p, dx, &vcell, &kfac);

  /* 1-2: free streaming and wall reflection */
  stream_reflect(p, n, x, y, z, px, py, pz);

  /* 3-4: cells and a stable counting sort by cell (ids ascending) */
  uint32_t *cell = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n + 1));
  int64_t *off = (int64_t *)calloc((size_t)(ncells + 1), sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncells + 1));
  int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!cell || !off || !fill || !list) {
    free(cell);
    free(off);
    free(fill);
    free(list);
    return ORC_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    cell[i] = cell_of(p, dx, x[i], y[i], z[i]);
    off[cell[i] + 1]++;
  }
  int64_t max_occ = 0;
  for (int64_t c = 0; c < ncells; ++c) {
    if (off[c + 1] > max_occ) max_occ = off[c + 1];
    off[c + 1] += off[c];
  }
  /* the pair index must fit the 32-bit counter word */
  if (max_occ > 92681) {
    free(cell);
    free(off);
    free(fill);
    free(list);
    return ORC_ERANGE;
  }
  memcpy(fill, off, sizeof(int64_t) * (size_t)ncells);
  for (int64_t i = 0; i < n; ++i) list[fill[cell[i]]++] = i;
  if (tr) {
    if (tr->cell)
      for (int64_t i = 0; i < n; ++i) tr->cell[i] = cell[i];
    if (tr->perm)
      for (int64_t j = 0; j < n; ++j) tr->perm[j] = (uint32_t)list[j];
    if (tr->offsets)
      for (int64_t c = 0; c <= ncells; ++c) tr->offsets[c] = (uint32_t)off[c];
    tr->n_cand = 0;
    tr->n_claim = 0;
  }

  /* 5-6: collisions, cell by cell (cells are independent) */
  mom_arrays m = {px, py, pz};
  if (nthreads <= 1) {
    unsigned char *claimed = (unsigned char *)malloc((size_t)max_occ + 1);
    philox_draws_ctx pctx;
    pctx.key[0] = (uint32_t)p->seed;
    pctx.key[1] = (uint32_t)(p->seed >> 32);
    pctx.step = t;
    draws_t dr = {philox_u_acc, philox_u_kin, &pctx};
    for (int64_t c = 0; c < ncells; ++c) {
      pctx.cell = (uint32_t)c;
      collide_cell(off[c + 1] - off[c], list + off[c], &m, kfac, &dr, claimed,
                   (uint32_t)c, tr, NULL, NULL);
    }
    free(claimed);
  } else {
    collide_job J;
    J.p = p;
    J.list = list;
    J.off = off;
    J.ncells = ncells;
    J.m = m;
    J.kfac = kfac;
    J.t = t;
    J.max_occ = max_occ;
    J.next = 0;
    J.chunk = ncells / (16 * (int64_t)nthreads);
    if (J.chunk < 1) J.chunk = 1;
    if (J.chunk > 64) J.chunk = 64;
    pthread_mutex_init(&J.mu, NULL);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; ++i)
      pthread_create(&th[i], NULL, collide_worker, &J);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
  }
  free(cell);
  free(off);
  free(fill);
  free(list);
  return ORC_OK;
}

int orc_run(const orc_params *p, int64_t n, double *x, double *y, double *z,
            double *px, double *py, double *pz, uint32_t t0, int32_t nsteps,
            int nthreads) {
  for (int32_t s = 0; s < nsteps; ++s) {
    int rc = orc_step(p, n, x, y, z, px, py, pz, t0 + (uint32_t)s, nthreads,
                      NULL);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Observables: the energy-density profile of Fig. 2 (lab-frame T^00) and  */
/* the momentum-density profile T^0x, per slab of cells along x.           */
/* ---------------------------------------------------------------------- */
/* Slab moments: sums over the particles of each x-slab, then divided by
 * the slab's physical volume (r_test dx Ly Lz), as the profiles of Sec. 5. */
void orc_observe_moments(const orc_params *p, int64_t n, const double *x,
                         const double *px, const double *py, const double *pz,
                         double *T00, double *T0x, double *Txx, double *nd) {
  double dx[3];
  orc_constants(p, dx, NULL, NULL);
  int32_t nx = p->cells[0];
  for (int32_t i = 0; i < nx; ++i) T00[i] = T0x[i] = Txx[i] = nd[i] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t ix = axis_cell(x[i], dx[0], nx);
    double e = energy(px[i], py[i], pz[i]);
    T00[ix] += e;
    T0x[ix] += px[i];
    Txx[ix] += (px[i] * px[i]) / e;
    nd[ix] += 1.0;
  }
  double vol = ((p->r_test * dx[0]) * p->box[1]) * p->box[2];
  for (int32_t i = 0; i < nx; ++i) {
    T00[i] = T00[i] / vol;
    T0x[i] = T0x[i] / vol;
    Txx[i] = Txx[i] / vol;
    nd[i] = nd[i] / vol;
  }
}

/* The timelike eigenvector of T^mu_nu restricted to t and x: with the
 * metric (+,-), T^mu_nu u^nu = e u^mu has the eigenvalues
 * ((T00 - Txx) +- sqrt((T00 + Txx)^2 - 4 T0x^2)) / 2; the larger one is the
 * rest-frame energy density, and the x-row gives T0x - Txx v = e v. */
void orc_landau(int32_t nx, const double *T00, const double *T0x, const double *Txx,
                double *e, double *v) {
  for (int32_t i = 0; i < nx; ++i) {
    /* (T00 + Txx)^2 - 4 T0x^2 as a product of two factors (no squares of
     * large numbers); rounding can make it slightly negative at v -> 1 */
    double a = T00[i] + Txx[i];
    double b = 2.0 * fabs(T0x[i]);
    double disc = (a - b) * (a + b);
    if (disc < 0.0) disc = 0.0;
    double ei = ((T00[i] - Txx[i]) + sqrt(disc)) / 2.0;
    double den = ei + Txx[i];
    e[i] = ei;
    v[i] = den > 0.0 ? T0x[i] / den : 0.0;
  }
}

void orc_observe(const orc_params *p, int64_t n, const double *x,
                 const double *px, const double *py, const double *pz,
                 double *T00, double *T0x) {
  double dx[3];
  orc_constants(p, dx, NULL, NULL);
  int32_t nx = p->cells[0];
  for (int32_t i = 0; i < nx; ++i) {
    T00[i] = 0.0;
    T0x[i] = 0.0;
  }
  for (int64_t i = 0; i < n; ++i) {
    int32_t ix = axis_cell(x[i], dx[0], nx);
    T00[ix] += energy(px[i], py[i], pz[i]);
    T0x[ix] += px[i];
  }
  double vol = ((p->r_test * dx[0]) * p->box[1]) * p->box[2];
  for (int32_t i = 0; i < nx; ++i) {
    T00[i] = T00[i] / vol;
    T0x[i] = T0x[i] / vol;
  }
}
