// Narrow phase of the contact set: the distance d_c of each point-triangle
// and edge-edge pair (the barrier argument of Section 3.1), its closest
// features and the gradient n = grad d_c that the projected contact Hessian
// of Section 4.1 uses.  One thread per pair; the outputs are the d and grad
// arrays of a contact stencil set.
#include "kernels.hpp"

namespace mas {

namespace {

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 axpy(double s, V3 a, V3 b) { return {fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z)}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double clamp01(double v) { return fmin(1.0, fmax(0.0, v)); }

// weight s of the closest point a + s (b - a) of a segment to p
__device__ __forceinline__ double seg_weight(V3 p, V3 a, V3 b) {
  const V3 e = b - a;
  const double ee = dot(e, e);
  return ee > 0.0 ? clamp01(dot(p - a, e) / ee) : 0.0;
}

// Closest point of triangle (a, b, c) to p, located by the Voronoi regions
// of its vertices, edges and face (Ericson, Real-Time Collision Detection,
// 2005, Section 5.1.5); w receives its barycentric weights.  Types: 0-2
// vertex a, b, c; 3 edge ab, 4 edge bc, 5 edge ca; 6 face.  A triangle
// without area that reaches the face case takes the nearest of its sides.
__device__ int pt_closest(V3 p, V3 a, V3 b, V3 c, double w[3]) {
  const V3 ab = b - a, ac = c - a;
  const V3 ap = p - a;
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) {
    w[0] = 1.0, w[1] = 0.0, w[2] = 0.0;
    return 0;
  }
  const V3 bp = p - b;
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) {
    w[0] = 0.0, w[1] = 1.0, w[2] = 0.0;
    return 1;
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    const double s = d1 / (d1 - d3);
    w[0] = 1.0 - s, w[1] = s, w[2] = 0.0;
    return 3;
  }
  const V3 cp = p - c;
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) {
    w[0] = 0.0, w[1] = 0.0, w[2] = 1.0;
    return 2;
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    const double s = d2 / (d2 - d6);
    w[0] = 1.0 - s, w[1] = 0.0, w[2] = s;
    return 5;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && d4 - d3 >= 0.0 && d5 - d6 >= 0.0) {
    const double s = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    w[0] = 0.0, w[1] = 1.0 - s, w[2] = s;
    return 4;
  }
  const double den = va + vb + vc;
  if (den > 0.0) {
    const double v = vb / den, u = vc / den;
    w[0] = 1.0 - v - u, w[1] = v, w[2] = u;
    return 6;
  }
  // no area: the nearest side
  const V3 T[3] = {a, b, c};
  double best = INFINITY;
  int ty = 3;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = k, j = (k + 1) % 3;
    const double s = seg_weight(p, T[i], T[j]);
    const V3 q = axpy(s, T[j] - T[i], T[i]);
    const double dd = dot(p - q, p - q);
    if (dd < best) {
      best = dd;
      w[0] = w[1] = w[2] = 0.0;
      w[i] = 1.0 - s;
      w[j] = s;
      ty = s == 0.0 ? i : (s == 1.0 ? j : 3 + k);
    }
  }
  return ty;
}

// Closest points a0 + s (a1 - a0) and b0 + t (b1 - b0) of two segments
// (unconstrained stationary point, then clamped to the square edge by edge;
// parallel segments start from s = 0).  Type 3 f(s) + f(t), f = 0 at the
// first vertex, 1 at the second, 2 inside.
__device__ int ee_closest(V3 a0, V3 a1, V3 b0, V3 b1, double& s, double& t) {
  const V3 u = a1 - a0, v = b1 - b0, r = a0 - b0;
  const double a = dot(u, u), e = dot(v, v), f = dot(v, r);
  if (a == 0.0 && e == 0.0) {
    s = t = 0.0;
  } else if (a == 0.0) {
    s = 0.0;
    t = clamp01(f / e);
  } else {
    const double c = dot(u, r);
    if (e == 0.0) {
      t = 0.0;
      s = clamp01(-c / a);
    } else {
      const double b = dot(u, v);
      const double den = a * e - b * b;
      s = den > 1e-14 * a * e ? clamp01((b * f - c * e) / den) : 0.0;
      t = (b * s + f) / e;
      if (t < 0.0) {
        t = 0.0;
        s = clamp01(-c / a);
      } else if (t > 1.0) {
        t = 1.0;
        s = clamp01((b - c) / a);
      }
    }
  }
  const int fs = s == 0.0 ? 0 : (s == 1.0 ? 1 : 2);
  const int ft = t == 0.0 ? 0 : (t == 1.0 ? 1 : 2);
  return 3 * fs + ft;
}

}  // namespace

__global__ __launch_bounds__(256) void k_contact_dist(int64_t N, int64_t m, const int32_t* pairs,
                                                      const uint8_t* kind, const double* x, double* dist,
                                                      double* grad, uint8_t* type, uint32_t* err) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int4 iv = reinterpret_cast<const int4*>(pairs)[i];
  const int v[4] = {iv.x, iv.y, iv.z, iv.w};
  if (!(v[0] >= 0 && v[0] < N && v[1] >= 0 && v[1] < N && v[2] >= 0 && v[2] < N && v[3] >= 0 && v[3] < N)) {
    dist[i] = NAN;
    if (type) type[i] = 255;
    if (grad)
      for (int q = 0; q < 12; ++q) grad[12 * i + q] = 0.0;
    atomicOr(err, ERRB_INDEX);
    return;
  }
  V3 X[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) X[j] = {x[3 * int64_t(v[j])], x[3 * int64_t(v[j]) + 1], x[3 * int64_t(v[j]) + 2]};
  double wt[4];  // weights of the closest points, second primitive negated
  V3 c1, c2;
  int ty;
  if (kind[i] == 0) {
    double w[3];
    ty = pt_closest(X[0], X[1], X[2], X[3], w);
    wt[0] = 1.0, wt[1] = -w[0], wt[2] = -w[1], wt[3] = -w[2];
    c1 = X[0];
    c2 = {w[0] * X[1].x + w[1] * X[2].x + w[2] * X[3].x, w[0] * X[1].y + w[1] * X[2].y + w[2] * X[3].y,
          w[0] * X[1].z + w[1] * X[2].z + w[2] * X[3].z};
  } else {
    double s, t;
    ty = ee_closest(X[0], X[1], X[2], X[3], s, t);
    wt[0] = 1.0 - s, wt[1] = s, wt[2] = -(1.0 - t), wt[3] = -t;
    c1 = axpy(s, X[1] - X[0], X[0]);
    c2 = axpy(t, X[3] - X[2], X[2]);
  }
  const V3 dv = c1 - c2;
  const double d = sqrt(dot(dv, dv));
  dist[i] = d;
  if (type) type[i] = uint8_t(ty);
  if (grad) {
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    const V3 n = {dv.x * inv, dv.y * inv, dv.z * inv};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      grad[12 * i + 3 * j] = wt[j] * n.x;
      grad[12 * i + 3 * j + 1] = wt[j] * n.y;
      grad[12 * i + 3 * j + 2] = wt[j] * n.z;
    }
  }
}

mas_status launch_contact_distances(Ctx& c, const double* x, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                    double* dist, double* grad, uint8_t* type) {
  ProfScope ps(c, MAS_T_CONTACT);
  if (m > 0)
    k_contact_dist<<<dim3((m + 255) / 256), dim3(256), 0, c.s>>>(c.N, m, pairs, kind, x, dist, grad, type,
                                                                  c.err);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
