// The gradient-side update of PDRQS1 (thesis §4.4) at one pixel, shared by
// its own kernel and by the forward projector's launch, whose extra
// workgroups run it alongside the projection (both read u only).
#pragma once
#include "common.hpp"

namespace ctpd {

// Pointwise projection onto the Euclidean ball of the given radius (§3.3).
__device__ inline void ball_project(float q1, float q2, float radius, float &w1, float &w2) {
  const float nrm = sqrtf(q1 * q1 + q2 * q2);
  const float sc = (nrm > radius) ? radius / nrm : 1.f;
  w1 = q1 * sc;
  w2 = q2 * sc;
}

// v2 = vb2 + st nabla u, w = proj_radius(2 v2 - vb2), vb2 <- vb2 + w - v2,
// s2 = vb2 + st nabla u for the next iteration.  mode 1: only s2 = vb2 +
// st nabla u.  mode 2: also store w.  mode 4: Algorithm CP's dual step.
// mode 5: ADMM's z-step (§4.6).  q2out: 2 v2 - vb2; ubar: the u >= 0
// resolvent (§4.5).  Pointers are those of problem 0 of a batch; z selects.
__device__ inline void tv_update_px(const TvArgs &a, int i, int j, int z) {
  const int n = a.n;
  const size_t nn = (size_t)n * n;
  const size_t o = (size_t)j * n + i;
  const float *u = a.u + z * nn;
  float *vb2 = a.vb2 + z * 2 * nn;
  float *s2 = a.s2 + z * 2 * nn;
  const float c = u[o];
  const float g1 = (i < n - 1) ? (u[o + 1] - c) * a.inv_h : 0.f;
  const float g2 = (j < n - 1) ? (u[o + n] - c) * a.inv_h : 0.f;
  const float b1 = vb2[o], b2 = vb2[o + nn];
  const float st = a.st, radius = a.radius;
  if (a.mode == 5) {
    // ADMM z-step and multiplier update, gradient block: s = nabla u + eta_v,
    // v = soft(s, radius), eta_v <- s - v, and the next u-step's residual
    // term (v - eta_v) - nabla u = 2 v - s - nabla u
    const float t1 = g1 + b1, t2 = g2 + b2;
    const float nq = sqrtf(t1 * t1 + t2 * t2);
    const float sc = nq > radius ? 1.f - radius / nq : 0.f;
    const float v1 = sc * t1, v2 = sc * t2;
    vb2[o] = t1 - v1;
    vb2[o + nn] = t2 - v2;
    s2[o] = 2.f * v1 - t1 - g1;
    s2[o + nn] = 2.f * v2 - t2 - g2;
    return;
  }
  if (a.mode == 1) {
    s2[o] = fmaf(st, g1, b1);
    s2[o + nn] = fmaf(st, g2, b2);
    return;
  }
  if (a.mode == 4) {
    float w1, w2;
    ball_project(fmaf(st, g1, b1), fmaf(st, g2, b2), radius, w1, w2);
    vb2[o] = w1;
    vb2[o + nn] = w2;
    return;
  }
  const float v1 = fmaf(st, g1, b1), v2 = fmaf(st, g2, b2);
  float w1, w2;
  ball_project(2.f * v1 - b1, 2.f * v2 - b2, radius, w1, w2);
  if (a.q2out != nullptr) {
    float *q2 = a.q2out + z * 2 * nn;
    q2[o] = 2.f * v1 - b1;
    q2[o + nn] = 2.f * v2 - b2;
  }
  if (a.ubar != nullptr) {
    float *ub = a.ubar + z * nn;
    const float x = ub[o];
    ub[o] = x + fmaxf(2.f * c - x, 0.f) - c;
  }
  const float n1 = b1 + w1 - v1, n2 = b2 + w2 - v2;
  vb2[o] = n1;
  vb2[o + nn] = n2;
  s2[o] = fmaf(st, g1, n1);
  s2[o + nn] = fmaf(st, g2, n2);
  if (a.mode == 2) {
    float *w = a.wout + z * 2 * nn;
    w[o] = w1;
    w[o + nn] = w2;
  }
}

}  // namespace ctpd
