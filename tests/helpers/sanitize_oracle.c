/* Drives every entry point of the C oracle, valid and invalid calls, so that
 * a build under AddressSanitizer and UndefinedBehaviorSanitizer reports any
 * out-of-bounds access, use of freed memory, overflow or misaligned access in
 * it.  Exits non-zero on a failed check; the sanitizers abort on a finding. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cuba_oracle.h"

static uint64_t g_lcg = 0x9E3779B97F4A7C15ull;
static double unit(void) { /* (0, 1] */
  g_lcg = g_lcg * 6364136223846793005ull + 1442695040888963407ull;
  return ((double)(g_lcg >> 11) + 1.0) * 0x1p-53;
}

#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      return 1;                                                      \
    }                                                                \
  } while (0)

static double total_energy(int64_t n, const double *px, const double *py, const double *pz) {
  double e = 0.0;
  for (int64_t i = 0; i < n; ++i) e += sqrt(px[i] * px[i] + py[i] * py[i] + pz[i] * pz[i]);
  return e;
}

int main(void) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.box[0] = 4.0; p.box[1] = 1.0; p.box[2] = 1.0;
  p.cells[0] = 20; p.cells[1] = 2; p.cells[2] = 3;  /* ragged: 120 cells */
  p.sigma = 0.4; p.r_test = 40.0; p.dt = 0.02; p.seed = 0x1234567890abcdefull;
  const int64_t n = 3001;
  double *r[6];
  for (int k = 0; k < 6; ++k) {
    r[k] = (double *)malloc((size_t)n * sizeof(double));
    CHECK(r[k] != NULL);
  }
  for (int64_t i = 0; i < n; ++i) {
    r[0][i] = p.box[0] * (1.0 - unit());
    r[1][i] = p.box[1] * (1.0 - unit());
    r[2][i] = p.box[2] * (1.0 - unit());
    const double e = -0.35 * log(unit() * unit() * unit());
    const double c = 2.0 * unit() - 1.0, s = sqrt((1.0 - c) * (1.0 + c));
    const double phi = 6.283185307179586 * unit();
    r[3][i] = e * s * cos(phi);
    r[4][i] = e * s * sin(phi);
    r[5][i] = e * c + 1e-300;
  }
  r[0][0] = 0.0;        /* on the walls */
  r[0][1] = p.box[0];
  r[1][2] = p.box[1];
  CHECK(orc_check(&p, n, r[0], r[1], r[2], r[3], r[4], r[5]) == ORC_OK);

  /* invalid parameters and states */
  orc_params q = p;
  q.dt = 1.0;
  CHECK(orc_check(&q, n, r[0], r[1], r[2], r[3], r[4], r[5]) == ORC_EINVAL);
  q = p;
  q.cells[1] = 0;
  CHECK(orc_check(&q, n, r[0], r[1], r[2], r[3], r[4], r[5]) == ORC_EINVAL);
  const double keep = r[0][5];
  r[0][5] = -1e-9;
  CHECK(orc_check(&p, n, r[0], r[1], r[2], r[3], r[4], r[5]) == ORC_ERANGE);
  r[0][5] = NAN;
  CHECK(orc_check(&p, n, r[0], r[1], r[2], r[3], r[4], r[5]) == ORC_ERANGE);
  r[0][5] = keep;

  const int64_t ncell = (int64_t)p.cells[0] * p.cells[1] * p.cells[2];
  uint32_t *cell = (uint32_t *)malloc((size_t)n * 4), *perm = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *offs = (uint32_t *)malloc((size_t)(ncell + 1) * 4);
  uint32_t *cand = (uint32_t *)malloc(3 * 8 * 4), *claim = (uint32_t *)malloc(3 * 4 * 4);
  CHECK(cell && perm && offs && cand && claim);
  const double e0 = total_energy(n, r[3], r[4], r[5]);
  for (uint32_t t = 0; t < 6; ++t) {
    /* small candidate and claim buffers: counts past the capacity */
    orc_trace tr;
    memset(&tr, 0, sizeof tr);
    tr.cell = cell; tr.perm = perm; tr.offsets = offs;
    tr.cand = cand; tr.cand_cap = 8; tr.claim = claim; tr.claim_cap = 4;
    CHECK(orc_step(&p, n, r[0], r[1], r[2], r[3], r[4], r[5], t, 1, &tr) == ORC_OK);
    CHECK(offs[ncell] == (uint32_t)n);
  }
  CHECK(orc_run(&p, n, r[0], r[1], r[2], r[3], r[4], r[5], 6, 10, 4) == ORC_OK);
  const double e1 = total_energy(n, r[3], r[4], r[5]);
  CHECK(fabs(e1 - e0) <= 1e-11 * e0);

  double T00[20], T0x[20], Txx[20], nd[20], e[20], v[20];
  orc_observe(&p, n, r[0], r[3], r[4], r[5], T00, T0x);
  orc_observe_moments(&p, n, r[0], r[3], r[4], r[5], T00, T0x, Txx, nd);
  orc_landau(20, T00, T0x, Txx, e, v);
  for (int k = 0; k < 20; ++k) CHECK(isfinite(e[k]) && isfinite(v[k]));

  /* one cell with injected uniforms; every pair accepted */
  double cx[6], cy[6], cz[6], ua[15], uk[30];
  int32_t aa[3], bb[3];
  for (int i = 0; i < 6; ++i) {
    cx[i] = unit();
    cy[i] = unit() - 0.5;
    cz[i] = 0.1 * i + 0.01;
  }
  for (int k = 0; k < 15; ++k) ua[k] = 0.0;
  for (int k = 0; k < 30; ++k) uk[k] = unit();
  CHECK(orc_collide_cell_with_uniforms(6, cx, cy, cz, 0.5, ua, uk, aa, bb) == 3);
  double pa[3] = {1.0, 0.0, 0.0}, pb[3] = {-1.0, 0.0, 0.0};
  orc_scatter_pair(pa, pb, 0.25, 0.75);
  CHECK(fabs(pa[0] + pb[0]) < 1e-15 && fabs(pa[1] + pb[1]) < 1e-15);

  uint32_t ctr[4] = {0xFFFFFFFFu, 1u, 2u, 3u}, key[2] = {5u, 6u}, w[4];
  orc_philox4x32_10(ctr, key, w);
  CHECK(orc_u53(0xFFFFFFFFu, 0xFFFFFFFFu) < 1.0 && orc_u53(0u, 0u) == 0.0);

  for (int k = 0; k < 6; ++k) free(r[k]);
  free(cell); free(perm); free(offs); free(cand); free(claim);
  printf("oracle sanitizer run ok\n");
  return 0;
}
