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

// Conservative step of one pair along the vertex displacements pv (supplement
// Eqs. (29), (31) for the lower bound alpha_l = d_min / l, d_min = 0.9 dist,
// then Algorithm 2 on the coplanarity
// cubic f(t) = A(t) . (B(t) x C(t)), A = x1 - x0 + t (p1 - p0), B, C alike).
__device__ double pair_step(const double (&xv)[4][3], const double (&pv)[4][3], int kind, double dist) {
  // largest relative displacement of a vertex pair across the primitives
  auto rel2 = [&](int s, int t) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) r += (pv[s][q] - pv[t][q]) * (pv[s][q] - pv[t][q]);
    return r;
  };
  double l2;
  if (kind == 0) l2 = fmax(fmax(rel2(0, 1), rel2(0, 2)), rel2(0, 3));
  else l2 = fmax(fmax(rel2(0, 2), rel2(0, 3)), fmax(rel2(1, 2), rel2(1, 3)));
  const double l = sqrt(l2);
  // d_min = 0.9 dist: a root before alpha_l is then a crossing of the plane
  // away from the other primitive (the pair is at least 0.1 dist apart
  // there), and a pair meeting exactly at dist / l is still found
  const double al = l > 0.0 ? 0.9 * dist / l : INFINITY;
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
  return cubic_safe(f, al);
}

// the pair's four vertex ids if all lie in [0, N) (else false and the
// error flag)
__device__ __forceinline__ bool pair_ids(int64_t N, const int32_t* pairs, int64_t i, int (&v)[4], uint32_t* err) {
  const int4 iv = reinterpret_cast<const int4*>(pairs)[i];
  const bool ok = iv.x >= 0 && iv.x < N && iv.y >= 0 && iv.y < N && iv.z >= 0 && iv.z < N && iv.w >= 0 && iv.w < N;
  if (!ok) {
    atomicOr(err, ERRB_INDEX);
    return false;
  }
  v[0] = iv.x;
  v[1] = iv.y;
  v[2] = iv.z;
  v[3] = iv.w;
  return true;
}

__global__ __launch_bounds__(256) void k_ccd_pairs(int64_t N, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                                   const double* dist, const double* x, const double* p,
                                                   double* alpha_pair, double* alpha, uint32_t* err) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int v[4] = {-1, -1, -1, -1};
  double step = 1.0;
  bool ok = i < m;
  if (ok) {
    ok = pair_ids(N, pairs, i, v, err);
    // a vertex id outside [0, N): no step for this pair, reported by the error flag
    if (!ok && alpha_pair) alpha_pair[i] = 0.0;
  }
  if (ok) {
    double xv[4][3], pv[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xv[j][q] = x[3 * int64_t(v[j]) + q];
        pv[j][q] = p[3 * int64_t(v[j]) + q];
      }
    step = pair_step(xv, pv, kind[i], dist[i]);
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

// ---------------------------------------------------------------------------
// Per-subdomain safe steps on point-triangle / edge-edge pairs (Algorithm 1's
// ConservativeCCD with per-subdomain alpha_d; Section 4.4).  A pair spanning
// subdomains with different steps moves its vertices by different fractions
// of p, which the CCD along p does not cover; those motions are checked
// with the CCD along the actual displacements and damped, as for the affine
// stencils (see k_pncg.hip).  scal2[0]: max |p_v| (bits), scal2[1]: the
// smallest alpha_d (bits).

__global__ void k_ccd_init(int64_t D, double* a0, uint64_t* half, uint32_t* rounds, unsigned long long* scal2) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < D) {
    a0[i] = 1.0;
    half[i] = 0ull;
  }
  if (i <= SAFE_ROUNDS) rounds[i] = 0u;
  if (i == 0) {
    scal2[0] = 0ull;
    scal2[1] = (unsigned long long)__double_as_longlong(1.0);
  }
}

// largest |p_v| over the vertices (non-negative doubles order like their bits)
__global__ __launch_bounds__(256) void k_pmax(int64_t N, const double* p, unsigned long long* pmax) {
  double mx = 0.0;
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < N; v += int64_t(gridDim.x) * blockDim.x) {
    const double a = p[3 * v], b = p[3 * v + 1], c = p[3 * v + 2];
    mx = fmax(mx, sqrt(a * a + b * b + c * c));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0 && mx > 0.0) atomicMax(pmax, (unsigned long long)__double_as_longlong(mx));
}

// alpha_d <= radius / (2 max |p_v|): no two vertices approach each other by
// more than the candidate radius, so pairs farther apart than it (left out
// of the candidates) cannot meet under any steps up to alpha_d; the
// smallest alpha_d goes to scal2[1]
__global__ void k_ccd_cap(int64_t D, double radius, double* a0, unsigned long long* scal2) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const double pm = __longlong_as_double((long long)scal2[0]);
  const double cap = pm > 0.0 ? fmin(1.0, radius / (2.0 * pm)) : 1.0;
  double a = INFINITY;
  if (i < D) {
    a = fmin(a0[i], cap);
    a0[i] = a;
  }
  for (int o = 32; o > 0; o >>= 1) a = fmin(a, __shfl_xor(a, o));
  if ((threadIdx.x & 63) == 0 && a < 1.0) atomicMin(&scal2[1], (unsigned long long)__double_as_longlong(a));
}

// Damping round r < SAFE_ROUNDS: a pair whose vertices, each moved by its
// own subdomain's step, would reach coplanarity (the CCD along those
// displacements finds a root before 1) marks its subdomains for halving
// (bit r of half) and is counted in rounds[r].  A round after one that found
// nothing returns at once; round SAFE_ROUNDS only counts.
__global__ __launch_bounds__(256) void k_ccd_round(int r, int64_t N, int64_t m, const int32_t* pairs,
                                                   const uint8_t* kind, const double* dist, const double* x,
                                                   const double* p, const double* a0, uint64_t* half,
                                                   uint32_t* rounds, uint32_t* err) {
  if (r > 0 && rounds[r - 1] == 0u) return;  // uniform: written by the previous launch
  const uint64_t mask = (1ull << r) - 1ull;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  bool viol = false;
  int v[4] = {-1, -1, -1, -1};
  if (i < m && pair_ids(N, pairs, i, v, err)) {
    double xv[4][3], pv[4][3];
    double s0 = -1.0;
    bool mixed = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t h = __hip_atomic_load(half + (v[j] >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & mask;
      const double sj = ldexp(a0[v[j] >> 5], -__popcll(h));
      mixed |= (j > 0 && sj != s0);
      s0 = j == 0 ? sj : s0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xv[j][q] = x[3 * int64_t(v[j]) + q];
        pv[j][q] = sj * p[3 * int64_t(v[j]) + q];
      }
    }
    // a pair moving with one step was covered by the CCD along p
    viol = mixed && pair_step(xv, pv, kind[i], dist[i]) < 1.0;
    if (viol && r < SAFE_ROUNDS) {
#pragma unroll
      for (int j = 0; j < 4; ++j) atomicOr(reinterpret_cast<unsigned long long*>(half + (v[j] >> 5)), 1ull << r);
    }
  }
  const unsigned long long b = __ballot(viol);
  if (b != 0 && (threadIdx.x & 63) == 0) atomicAdd(rounds + r, uint32_t(__popcll(b)));
}

// the damped steps, or, if the last round still found a pair, the smallest
// step for every subdomain (one common step along p, which the CCD covers)
__global__ void k_ccd_final(int64_t D, const double* a0, const uint64_t* half, const uint32_t* rounds,
                            const unsigned long long* scal2, double* alpha) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= D) return;
  alpha[i] = rounds[SAFE_ROUNDS] != 0u ? __longlong_as_double((long long)scal2[1])
                                        : ldexp(a0[i], -__popcll(half[i]));
}

mas_status launch_ccd_safe_step(Ctx& c, const double* x, const double* p, double radius, int64_t m,
                                const int32_t* pairs, const uint8_t* kind, const double* dist, double scale,
                                double* alpha, double* x_out) {
  ProfScope ps(c, MAS_T_CCD);
  const int64_t D = c.lv[0].nsub;
  const dim3 gD((std::max<int64_t>(D, SAFE_ROUNDS + 1) + 255) / 256), b256(256);
  unsigned long long* scal2 = reinterpret_cast<unsigned long long*>(c.scal + 8);
  k_ccd_init<<<gD, b256, 0, c.s>>>(D, c.alpha0, c.ahalf, c.around, scal2);
  k_pmax<<<dim3(std::min<int64_t>((c.N + 255) / 256, int64_t(c.n_cu) * 4)), b256, 0, c.s>>>(c.N, p, scal2);
  if (m > 0) {
    const dim3 g((m + 255) / 256);
    k_ccd_pairs<<<g, b256, 0, c.s>>>(c.N, m, pairs, kind, dist, x, p, nullptr, c.alpha0, c.err);
    k_ccd_cap<<<gD, b256, 0, c.s>>>(D, radius, c.alpha0, scal2);
    for (int r = 0; r <= SAFE_ROUNDS; ++r)
      k_ccd_round<<<g, b256, 0, c.s>>>(r, c.N, m, pairs, kind, dist, x, p, c.alpha0, c.ahalf, c.around, c.err);
  } else {
    k_ccd_cap<<<gD, b256, 0, c.s>>>(D, radius, c.alpha0, scal2);
  }
  k_ccd_final<<<gD, b256, 0, c.s>>>(D, c.alpha0, c.ahalf, c.around, scal2, c.alpha);
  HIPCHK(hipGetLastError());
  return launch_step_with(c, x, p, scale, alpha, x_out);
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
