// device.hpp -- per-particle and per-pair device arithmetic of the PIC
// Boltzmann step (arXiv:1208.0961, Sec. 2) for gfx950.
//
// Every floating-point expression is evaluated in the order fixed by the
// determinism contract in include/cuba.h; the library is built with
// -ffp-contract=off so that no multiply-add is fused, and relies on the
// correctly rounded FP64 division and square root of the AMDGPU backend.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cuba {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The round keys
// key + r * (golden-ratio Weyl constants) are wave-uniform, so the compiler
// keeps them in scalar registers; so are the counter words for cell, step
// and purpose, which lets it scalarise the first two rounds' uniform halves.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t w0, w1, w2, w3;
};

constexpr uint32_t kMulA = 0xD2511F53u;  // multiplies word 0
constexpr uint32_t kMulB = 0xCD9E8D57u;  // multiplies word 2
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 VALU instruction (3-input bit op, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One Philox round with round keys ka, kb.
__device__ __forceinline__ void philox_round(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                             uint32_t &x3, uint32_t ka, uint32_t kb) {
  const uint64_t pa = (uint64_t)x0 * kMulA;
  const uint64_t pb = (uint64_t)x2 * kMulB;
  const uint32_t y0 = xor3((uint32_t)(pb >> 32), x1, ka);
  const uint32_t y2 = xor3((uint32_t)(pa >> 32), x3, kb);
  x1 = (uint32_t)pb;
  x3 = (uint32_t)pa;
  x0 = y0;
  x2 = y2;
}

__device__ __forceinline__ Words4 philox10(uint32_t x0, uint32_t x1, uint32_t x2,
                                           uint32_t x3, uint32_t key0,
                                           uint32_t key1) {
#pragma unroll
  for (uint32_t r = 0; r < 10; ++r)
    philox_round(x0, x1, x2, x3, key0 + r * kWeylA, key1 + r * kWeylB);
  return Words4{x0, x1, x2, x3};
}

// Word w1 of the same block, computing only what w1 depends on: rounds 1-6
// in full; then round 7 needs hi(A) and B, round 8 lo(A) and hi(B), round 9
// hi(A), round 10 lo(B).  16 vector multiplies instead of 20 (fewer when
// the counter's cell, step and purpose words are wave-uniform).
__device__ __forceinline__ uint32_t philox10_w1(uint32_t x0, uint32_t x1, uint32_t x2,
                                                uint32_t x3, uint32_t key0,
                                                uint32_t key1) {
#pragma unroll
  for (uint32_t r = 0; r < 6; ++r)
    philox_round(x0, x1, x2, x3, key0 + r * kWeylA, key1 + r * kWeylB);
  {  // round 7
    const uint32_t ha = __umulhi(x0, kMulA);
    const uint64_t pb = (uint64_t)x2 * kMulB;
    const uint32_t y0 = xor3((uint32_t)(pb >> 32), x1, key0 + 6u * kWeylA);
    x2 = xor3(ha, x3, key1 + 6u * kWeylB);
    x1 = (uint32_t)pb;
    x0 = y0;
  }
  {  // round 8
    const uint32_t la = x0 * kMulA;
    const uint32_t hb = __umulhi(x2, kMulB);
    x0 = xor3(hb, x1, key0 + 7u * kWeylA);
    x3 = la;
  }
  // round 9, then the low half of round 10's second product
  x2 = xor3(__umulhi(x0, kMulA), x3, key1 + 8u * kWeylB);
  return x2 * kMulB;
}

// 53-bit uniform in [0, 1) from two words (hi:lo).
__device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t bits = ((((uint64_t)hi) << 32) | lo) >> 11;
  return (double)bits * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Geometry and the single-particle update (Eq. (2) and the walls).
// ---------------------------------------------------------------------------
struct Geometry {
  double L[3];   // box edges
  double dx[3];  // cell edges L_d / n_d
  int32_t n[3];  // cells per axis
  double dt;
};

__device__ __forceinline__ double norm3(double a, double b, double c) {
  return __builtin_sqrt((a * a + b * b) + c * c);
}

// Free streaming over dt, then specular reflection at the walls 0 and L_d.
template <bool kStream>
__device__ __forceinline__ void advance(const Geometry &g, double &x, double &y,
                                        double &z, double &px, double &py,
                                        double &pz) {
  if (kStream) {
    const double e = norm3(px, py, pz);
    if (e != 0.0) {
      const double vx = px / e, vy = py / e, vz = pz / e;
      x = x + vx * g.dt;
      y = y + vy * g.dt;
      z = z + vz * g.dt;
    }
    if (x < 0.0) {
      x = -x;
      px = -px;
    } else if (x > g.L[0]) {
      x = 2.0 * g.L[0] - x;
      px = -px;
    }
    if (y < 0.0) {
      y = -y;
      py = -py;
    } else if (y > g.L[1]) {
      y = 2.0 * g.L[1] - y;
      py = -py;
    }
    if (z < 0.0) {
      z = -z;
      pz = -pz;
    } else if (z > g.L[2]) {
      z = 2.0 * g.L[2] - z;
      pz = -pz;
    }
  }
}

__device__ __forceinline__ int32_t axis_index(double q, double d, int32_t n) {
  int32_t i = (int32_t)__builtin_floor(q / d);
  i = i < 0 ? 0 : i;
  return i > n - 1 ? n - 1 : i;
}

// x-major cell id.
__device__ __forceinline__ uint32_t cell_id(const Geometry &g, double x, double y,
                                           double z) {
  const int32_t ix = axis_index(x, g.dx[0], g.n[0]);
  const int32_t iy = axis_index(y, g.dx[1], g.n[1]);
  const int32_t iz = axis_index(z, g.dx[2], g.n[2]);
  return (uint32_t)((ix * g.n[1] + iy) * g.n[2] + iz);
}

// ---------------------------------------------------------------------------
// Pairs of an n-member cell: lexicographic index k <-> (a, b), a < b.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t row_start(uint32_t a, uint32_t n) {
  return a * (2u * n - a - 1u) / 2u;
}

__device__ __forceinline__ void pair_of_index(uint32_t k, uint32_t n, uint32_t &a,
                                              uint32_t &b) {
  const double m = 2.0 * (double)n - 1.0;
  double r = (m - __builtin_sqrt(m * m - 8.0 * (double)k)) * 0.5;
  int32_t ai = (int32_t)r;
  ai = ai < 0 ? 0 : ai;
  ai = ai > (int32_t)n - 2 ? (int32_t)n - 2 : ai;
  uint32_t aa = (uint32_t)ai;
  while (aa > 0 && row_start(aa, n) > k) --aa;
  while (aa + 1 <= n - 2 && row_start(aa + 1, n) <= k) ++aa;
  a = aa;
  b = k - row_start(aa, n) + aa + 1u;
}

// The same map for cells of any size up to the 32-bit pair-index limit,
// in 64-bit integer arithmetic (n (2n - a - 1) exceeds 32 bits above
// 46 341 members).
__device__ __forceinline__ uint64_t row_start64(uint64_t a, uint64_t n) {
  return a * (2u * n - a - 1u) / 2u;
}

__device__ __forceinline__ void pair_of_index64(uint64_t k, uint64_t n, uint32_t &a,
                                                uint32_t &b) {
  const double m = 2.0 * (double)n - 1.0;
  const double r = (m - __builtin_sqrt(m * m - 8.0 * (double)k)) * 0.5;
  int64_t ai = (int64_t)r;
  ai = ai < 0 ? 0 : ai;
  ai = ai > (int64_t)n - 2 ? (int64_t)n - 2 : ai;
  uint64_t aa = (uint64_t)ai;
  while (aa > 0 && row_start64(aa, n) > k) --aa;
  while (aa + 1 <= n - 2 && row_start64(aa + 1, n) <= k) ++aa;
  a = (uint32_t)aa;
  b = (uint32_t)(k - row_start64(aa, n) + aa + 1u);
}

// ---------------------------------------------------------------------------
// Eq. (3): the pair's acceptance probability P22 = K s / (2 E1 E2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double p22(double ax, double ay, double az, double bx,
                                      double by, double bz, double kfac) {
  const double ea = norm3(ax, ay, az);
  const double eb = norm3(bx, by, bz);
  const double dot = (ax * bx + ay * by) + az * bz;
  const double e12 = ea * eb;
  const double s = 2.0 * (e12 - dot);
  const double vrel = s / (2.0 * e12);
  return vrel * kfac;
}

// ---------------------------------------------------------------------------
// 2 -> 2 kinematics: CM boost, isotropic direction, boost back (Sec. 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scatter_pair(double &ax, double &ay, double &az,
                                             double &bx, double &by, double &bz,
                                             double uc, double uphi) {
  const double ea = norm3(ax, ay, az);
  const double eb = norm3(bx, by, bz);
  const double dot = (ax * bx + ay * by) + az * bz;
  const double e12 = ea * eb;
  double s;
  if (dot > 0.0) {
    // small opening angle: s = 2 |pa x pb|^2 / (E1E2 + pa.pb), no cancellation
    const double cx = ay * bz - az * by;
    const double cy = az * bx - ax * bz;
    const double cz = ax * by - ay * bx;
    const double c2 = (cx * cx + cy * cy) + cz * cz;
    s = (2.0 * c2) / (e12 + dot);
  } else {
    s = 2.0 * (e12 - dot);
  }
  if (!(s > 0.0)) return;  // collinear: no CM frame
  const double et = ea + eb;
  const double Px = ax + bx, Py = ay + by, Pz = az + bz;
  const double rs = __builtin_sqrt(s);
  const double gamma = et / rs;
  const double btx = Px / et, bty = Py / et, btz = Pz / et;
  const double estar = rs * 0.5;

  const double cth = 2.0 * uc - 1.0;
  const double sth = __builtin_sqrt((1.0 - cth) * (1.0 + cth));
  // phi = 2 pi uphi: sin and cos of pi * (2 uphi), whose argument needs no
  // range reduction (the oracle rounds 2 pi uphi first and calls sin, cos;
  // the two differ by ulps)
  double sphi, cphi;
  sincospi(2.0 * uphi, &sphi, &cphi);
  const double qx = estar * (sth * cphi);
  const double qy = estar * (sth * sphi);
  const double qz = estar * cth;

  const double g2 = (gamma * gamma) / (gamma + 1.0);
  const double bq = (btx * qx + bty * qy) + btz * qz;
  const double fa = g2 * bq + gamma * estar;
  const double fb = g2 * (-bq) + gamma * estar;
  ax = qx + btx * fa;
  ay = qy + bty * fa;
  az = qz + btz * fa;
  bx = (-qx) + btx * fb;
  by = (-qy) + bty * fb;
  bz = (-qz) + btz * fb;
}

}  // namespace cuba
