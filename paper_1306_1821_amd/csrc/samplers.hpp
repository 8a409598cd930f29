// Scalar float64 samplers for the Gibbs blocks, one thread per draw.
//
// chi^2_beta = 2 Gamma(beta/2): Marsaglia & Tsang (2000), attempt j on Philox
//   block j (words 0,1 -> normal by Box-Muller cosine branch, word 2 -> the
//   acceptance uniform, word 3 -> U^(1/a) boost when a < 1).
// GIG(p, A, B), density ~ x^(p-1) exp(-(A x + B/x)/2): ratio of uniforms with
//   mode shift (Dagpunar 1989, Lehner 1989) on h(z) ~ z^(lam-1) exp(-om/2 (z+1/z)),
//   lam = |p|, om = sqrt(A B), x = sqrt(B/A) z^(sign p); the rectangle's v
//   extremes are the roots of d/dz [ln|z - m| + ln h(z)/2] on either side of the
//   mode m, found by bisection; attempt j on block j (word 0 -> u, word 1 -> v).
#pragma once
#include "rng.hpp"

namespace hmcsamp {

constexpr int kMaxAttempts = 256;

// Returns a Gamma(a, 1) variate, or -1 if no attempt was accepted.
__device__ inline double gamma_mt(double a, uint64_t seed, uint32_t chain, uint32_t draw,
                                  uint32_t sub) {
  const bool boost = a < 1.0;
  const double aa = boost ? a + 1.0 : a;
  const double d = aa - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  for (int j = 0; j < kMaxAttempts; ++j) {
    hmcrng::U4 w = hmcrng::block(seed, chain, hmcrng::kChi2, draw, sub, (uint32_t)j);
    double x, unused;
    hmcrng::box_muller(w.w[0], w.w[1], &x, &unused);
    const double t = 1.0 + c * x;
    if (t <= 0.0) continue;
    const double v = t * t * t;
    const double u = hmcrng::uniform(w.w[2]);
    if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) {
      double g = d * v;
      if (boost) g *= pow(hmcrng::uniform(w.w[3]), 1.0 / a);
      return g;
    }
  }
  return -1.0;
}

struct GigBox {
  double lam, om, m, vm, vp;
};

__device__ inline double gig_lh(const GigBox& b, double z) {
  const double d = z - b.m;
  return (b.lam - 1.0) * log1p(d / b.m) - 0.5 * b.om * d * (1.0 - 1.0 / (z * b.m));
}

__device__ inline double gig_F(const GigBox& b, double z) {
  return 1.0 / (z - b.m) + 0.5 * ((b.lam - 1.0) / z - 0.5 * b.om * (1.0 - 1.0 / (z * z)));
}

__device__ inline double gig_bisect(const GigBox& b, double lo, double hi) {
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (gig_F(b, mid) > 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

__device__ inline GigBox gig_box(double lam, double om) {
  GigBox b;
  b.lam = lam;
  b.om = om;
  b.m = ((lam - 1.0) + sqrt((lam - 1.0) * (lam - 1.0) + om * om)) / om;
  double step = b.m;
  for (int i = 0; i < 2000 && gig_F(b, b.m + step) > 0.0; ++i) step *= 2.0;
  const double zp = gig_bisect(b, b.m, b.m + step);
  double lo = 0.5 * b.m;
  for (int i = 0; i < 2000 && gig_F(b, lo) < 0.0; ++i) lo *= 0.5;
  const double zm = gig_bisect(b, lo, b.m);
  b.vp = (zp - b.m) * exp(0.5 * gig_lh(b, zp));
  b.vm = (zm - b.m) * exp(0.5 * gig_lh(b, zm));
  return b;
}

// Returns a GIG(p, A, B) variate, or -1 if no attempt was accepted.
__device__ inline double gig(double p, double A, double B, uint64_t seed, uint32_t chain,
                             uint32_t draw, uint32_t sub) {
  const GigBox b = gig_box(fabs(p), sqrt(A * B));
  for (int j = 0; j < kMaxAttempts; ++j) {
    hmcrng::U4 w = hmcrng::block(seed, chain, hmcrng::kGig, draw, sub, (uint32_t)j);
    const double u = hmcrng::uniform(w.w[0]);
    const double v = b.vm + (b.vp - b.vm) * hmcrng::uniform(w.w[1]);
    const double z = v / u + b.m;
    if (z <= 0.0) continue;
    if (log(u) <= 0.5 * gig_lh(b, z)) {
      const double s = sqrt(B / A);
      return p >= 0.0 ? s * z : s / z;
    }
  }
  return -1.0;
}

}  // namespace hmcsamp
