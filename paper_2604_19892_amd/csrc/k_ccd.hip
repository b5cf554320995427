// Conservative CCD of point-triangle and edge-edge pairs (supplement
// Section 3): the relative-displacement lower bound, the coplanarity cubic
// and the safe-side bisection of its first sign change, one thread per
// pair, then the per-subdomain minimum of Algorithm 1.
#include "kernels.hpp"

namespace mas {

namespace {

struct Cubic {
  double d, c, b, a;  // f(t) = a t^3 + b t^2 + c t + d
};

__device__ __forceinline__ double cub(const Cubic& f, double t) { return ((f.a * t + f.b) * t + f.c) * t + f.d; }

__device__ __forceinline__ int sgn(double v) { return int(v > 0.0) - int(v < 0.0); }

// Sixteen halvings of [xs, xu] that keep f(xs) on the side of ys
// (supplement Algorithm 1; ys follows xs when xs advances).
__device__ double safe_bisect(const Cubic& f, double xs, double xu, double ys) {
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const double xm = 0.5 * (xs + xu), ym = cub(f, xm);
    if (sgn(ys) != sgn(ym)) {
      xu = xm;
    } else {
      xs = xm;
      ys = ym;
    }
  }
  return xs;
}

// Supplement Algorithm 2: [max(0, al), 1] is cut at the critical points of f
// (roots of 3 a t^2 + 2 b t + c, from the cancellation-free form of the
// quadratic formula) into monotonic pieces; the first piece whose ends
// differ in sign is bisected, or its start returned when it begins past al.
__device__ double cubic_safe(const Cubic& f, double al) {
  if (al >= 1.0) return 1.0;
  double x = fmax(0.0, al);
  double y = cub(f, x);
  if (y == 0.0) return x;
  const double y1 = cub(f, 1.0);
  const double disc = f.b * f.b - 3.0 * f.a * f.c;
  if (disc > 0.0) {
    const double q = -(f.b + copysign(sqrt(disc), f.b));
    const double r1 = f.a != 0.0 ? q / (3.0 * f.a) : INFINITY;
    const double r2 = q != 0.0 ? f.c / q : INFINITY;
    const double xa = fmin(r1, r2), xb = fmax(r1, r2);
    if (x < xa && xa < 1.0) {
      const double ya = cub(f, xa);
      if (sgn(y) != sgn(ya)) return safe_bisect(f, x, xa, y);
      x = xa;
      y = ya;
    }
    if (x < xb && xb < 1.0) {
      const double yb = cub(f, xb);
      if (sgn(y) != sgn(yb)) return x > al ? x : safe_bisect(f, x, xb, y);
      x = xb;
      y = yb;
    }
  } else if (disc == 0.0 && f.a != 0.0) {
    const double xi = -f.b / (3.0 * f.a);
    if (x < xi && xi < 1.0) {
      const double yi = cub(f, xi);
      if (sgn(y) != sgn(yi)) return safe_bisect(f, x, xi, y);
      x = xi;
      y = yi;
    }
  }
  if (sgn(y) != sgn(y1)) return x > al ? x : safe_bisect(f, x, 1.0, y);
  return 1.0;
}

__device__ __forceinline__ void cross3(const double* u, const double* v, double* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

__device__ __forceinline__ double dot3(const double* u, const double* v) {
  return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

}  // namespace

__global__ __launch_bounds__(256) void k_ccd_pairs(int64_t N, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                                   const double* dist, const double* x, const double* p,
                                                   double* alpha_pair, double* alpha, uint32_t* err) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int v[4] = {-1, -1, -1, -1};
  double step = 1.0;
  bool ok = i < m;
  if (ok) {
    const int4 iv = reinterpret_cast<const int4*>(pairs)[i];
    ok = iv.x >= 0 && iv.x < N && iv.y >= 0 && iv.y < N && iv.z >= 0 && iv.z < N && iv.w >= 0 && iv.w < N;
    if (!ok) {
      // a vertex id outside [0, N): no step for this pair, reported by the error flag
      if (alpha_pair) alpha_pair[i] = 0.0;
      atomicOr(err, ERRB_INDEX);
    }
  }
  if (ok) {
    const int4 iv = reinterpret_cast<const int4*>(pairs)[i];
    v[0] = iv.x;
    v[1] = iv.y;
    v[2] = iv.z;
    v[3] = iv.w;
    double xv[4][3], pv[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xv[j][q] = x[3 * int64_t(v[j]) + q];
        pv[j][q] = p[3 * int64_t(v[j]) + q];
      }
    // largest relative displacement of a vertex pair across the primitives
    auto rel2 = [&](int s, int t) {
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) r += (pv[s][q] - pv[t][q]) * (pv[s][q] - pv[t][q]);
      return r;
    };
    double l2;
    if (kind[i] == 0) l2 = fmax(fmax(rel2(0, 1), rel2(0, 2)), rel2(0, 3));
    else l2 = fmax(fmax(rel2(0, 2), rel2(0, 3)), fmax(rel2(1, 2), rel2(1, 3)));
    const double l = sqrt(l2);
    const double al = l > 0.0 ? dist[i] / l : INFINITY;
    // f(t) = A(t) . (B(t) x C(t)) with A = x1 - x0 + t (p1 - p0), B, C alike
    double a0[3], a1[3], b0[3], b1[3], c0[3], c1[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a0[q] = xv[1][q] - xv[0][q];
      a1[q] = pv[1][q] - pv[0][q];
      b0[q] = xv[2][q] - xv[0][q];
      b1[q] = pv[2][q] - pv[0][q];
      c0[q] = xv[3][q] - xv[0][q];
      c1[q] = pv[3][q] - pv[0][q];
    }
    double b0c0[3], b1c0[3], b0c1[3], b1c1[3];
    cross3(b0, c0, b0c0);
    cross3(b1, c0, b1c0);
    cross3(b0, c1, b0c1);
    cross3(b1, c1, b1c1);
    Cubic f;
    f.d = dot3(a0, b0c0);
    f.c = dot3(a1, b0c0) + dot3(a0, b1c0) + dot3(a0, b0c1);
    f.b = dot3(a1, b1c0) + dot3(a1, b0c1) + dot3(a0, b1c1);
    f.a = dot3(a1, b1c1);
    step = cubic_safe(f, al);
    if (alpha_pair) alpha_pair[i] = step;
  }
  if (!alpha) return;
  const bool has = step < 1.0;
  if (__ballot(has) == 0) return;  // uniform
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sd = v[j] >> 5;
    const long long key = (has && v[j] >= 0) ? (long long)sd : -1ll;
    wave_min_pos(key, alpha + (key >= 0 ? sd : 0), step);
  }
}

mas_status launch_ccd(Ctx& c, const double* x, const double* p, int64_t m, const int32_t* pairs,
                      const uint8_t* kind, const double* dist, double* alpha_pair, double* alpha) {
  ProfScope ps(c, MAS_T_CCD);
  const int64_t D = c.lv[0].nsub;
  if (alpha) fill_f64(c, alpha, D, 1.0);
  if (m > 0)
    k_ccd_pairs<<<dim3((m + 255) / 256), dim3(256), 0, c.s>>>(c.N, m, pairs, kind, dist, x, p, alpha_pair,
                                                                alpha, c.err);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
