// Narrow phase of the contact set: the distance d_c of each point-triangle
// and edge-edge pair (the barrier argument of Section 3.1), its closest
// features and the gradient n = grad d_c that the projected contact Hessian
// of Section 4.1 uses.  One thread per pair; the outputs are the d and grad
// arrays of a contact stencil set.
#include <cstring>

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

// Distance of pair X (point-triangle or edge-edge), the closest-point
// weights (second primitive negated) and the unit vector n from the second
// closest point to the first (zero at d = 0); returns the type.
__device__ int pair_geometry(const V3 (&X)[4], int kind, double& d, double (&wt)[4], V3& n) {
  V3 c1, c2;
  int ty;
  if (kind == 0) {
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
  d = sqrt(dot(dv, dv));
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  n = {dv.x * inv, dv.y * inv, dv.z * inv};
  return ty;
}

__device__ __forceinline__ V3 load_v3(const double* x, int v) {
  return {x[3 * int64_t(v)], x[3 * int64_t(v) + 1], x[3 * int64_t(v) + 2]};
}

__device__ __forceinline__ void store_grad(double* grad, int64_t i, const double (&wt)[4], V3 n) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    grad[12 * i + 3 * j] = wt[j] * n.x;
    grad[12 * i + 3 * j + 1] = wt[j] * n.y;
    grad[12 * i + 3 * j + 2] = wt[j] * n.z;
  }
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
  for (int j = 0; j < 4; ++j) X[j] = load_v3(x, v[j]);
  double d, wt[4];
  V3 n;
  const int ty = pair_geometry(X, kind[i], d, wt, n);
  dist[i] = d;
  if (type) type[i] = uint8_t(ty);
  if (grad) store_grad(grad, i, wt, n);
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

// ---------------------------------------------------------------------------
// Broad phase of ComputeConstraintSet (Algorithm 1): a uniform grid of
// cells of side h = (largest primitive extent) + 2 dhat, hashed into
// buckets.  Every triangle and every edge is entered into each cell its
// box, grown by dhat, overlaps (at most two cells per axis at this h).  A
// point probes its own cell: a triangle within dhat of it has a grown box
// containing it, so it is entered there, once.  An edge probes the cells
// of its own box and keeps a partner edge only in the cell holding the
// lower corner of the overlap of its own box and the partner's grown box,
// so each pair is found once.  Candidates whose boxes are dhat or more apart are dropped, the
// rest go through the narrow phase and are kept when d < dhat.  Results
// are appended through one counter, one atomic per wavefront for up to
// four pairs per lane (their order is not fixed).
namespace {

constexpr int CELL_BITS = 21;  // per axis in the cell key (cells wrap every 2^21)

__device__ __forceinline__ uint64_t cell_key(int64_t cx, int64_t cy, int64_t cz) {
  const uint64_t m = (1ull << CELL_BITS) - 1;
  return ((uint64_t(cx) & m) << (2 * CELL_BITS)) | ((uint64_t(cy) & m) << CELL_BITS) | (uint64_t(cz) & m);
}

__device__ __forceinline__ int64_t cell_of(double v, double h) { return int64_t(floor(v / h)); }

struct Box {
  double lo[3], hi[3];
};

template <int NV>
__device__ __forceinline__ Box prim_box(const double* x, const int32_t* ids, int64_t p) {
  Box b;
  for (int a = 0; a < 3; ++a) b.lo[a] = b.hi[a] = x[3 * int64_t(ids[NV * p]) + a];
#pragma unroll
  for (int j = 1; j < NV; ++j)
    for (int a = 0; a < 3; ++a) {
      const double v = x[3 * int64_t(ids[NV * p + j]) + a];
      b.lo[a] = fmin(b.lo[a], v);
      b.hi[a] = fmax(b.hi[a], v);
    }
  return b;
}

// squared distance between boxes a and b
__device__ __forceinline__ double box_dist2(const Box& a, const Box& b) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double g = fmax(0.0, fmax(a.lo[q] - b.hi[q], b.lo[q] - a.hi[q]));
    s += g * g;
  }
  return s;
}

// Identity of a pair found by the constraint set: the kind (tag 2
// point-triangle, 3 edge-edge, in bits 60-63) and the indices of its two
// primitives in the caller's lists (the vertex's index in verts and the
// triangle's in tris, or the two edges' indices in edges, the smaller
// first), 30 bits each.  The lists are fixed across calls, so a pair keeps
// its key from one contact set to the next.
__device__ __forceinline__ uint64_t pair_key(int kind, int64_t a, int64_t b) {
  return (uint64_t(2 + kind) << 60) | (uint64_t(a) << 30) | uint64_t(b);
}

__device__ __forceinline__ void append_pair(unsigned long long* count, int64_t cap, const int (&v)[4], int kind,
                                            double d, const double (&wt)[4], V3 n, int32_t* pairs, uint8_t* kinds,
                                            double* dist, double* grad, uint64_t* keys, uint64_t key) {
  const unsigned long long slot = atomicAdd(count, 1ull);
  if (int64_t(slot) >= cap) return;
  const int64_t i = int64_t(slot);
  reinterpret_cast<int4*>(pairs)[i] = make_int4(v[0], v[1], v[2], v[3]);
  kinds[i] = uint8_t(kind);
  dist[i] = d;
  if (grad) store_grad(grad, i, wt, n);
  if (keys) keys[i] = key;
}

}  // namespace

// Checks every id against N and every coordinate for finiteness (misc[2]:
// bit 0 a bad id, bit 1 a non-finite coordinate) before anything else
// reads them; misc[0] receives the largest axis extent of a triangle or
// edge and misc[3] the largest |coordinate|, both as the bits of a
// non-negative double (their order is the order of the values).
__global__ __launch_bounds__(256) void k_cs_prep(int64_t N, int64_t nt, const int32_t* tris, int64_t ne,
                                                 const int32_t* edges, int64_t nv, const int32_t* verts,
                                                 const double* x, unsigned long long* misc) {
  __shared__ double se[4], sa[4];
  __shared__ unsigned long long sb[4];
  double e = 0.0, amax = 0.0;
  unsigned long long bad = 0;
  const int64_t total = nt + ne + nv;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t* ids;
    int nid;
    if (i < nt) ids = tris + 3 * i, nid = 3;
    else if (i < nt + ne) ids = edges + 2 * (i - nt), nid = 2;
    else ids = verts + (i - nt - ne), nid = 1;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool ok = true;
    for (int j = 0; j < nid; ++j) {
      const int v = ids[j];
      if (!(v >= 0 && v < N)) {
        bad |= 1ull;
        ok = false;
        continue;
      }
      for (int a = 0; a < 3; ++a) {
        const double c = x[3 * int64_t(v) + a];
        if (!isfinite(c)) {
          bad |= 2ull;
          ok = false;
        }
        lo[a] = fmin(lo[a], c);
        hi[a] = fmax(hi[a], c);
      }
    }
    if (ok) {
      for (int a = 0; a < 3; ++a) amax = fmax(amax, fmax(fabs(lo[a]), fabs(hi[a])));
      if (nid > 1) e = fmax(e, fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2])));
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    e = fmax(e, __shfl_xor(e, o));
    amax = fmax(amax, __shfl_xor(amax, o));
    bad |= __shfl_xor(bad, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) se[w] = e, sa[w] = amax, sb[w] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q) e = fmax(e, se[q]), amax = fmax(amax, sa[q]), bad |= sb[q];
    if (e > 0.0) atomicMax(&misc[0], (unsigned long long)__double_as_longlong(e));
    if (bad) atomicOr(&misc[2], bad);
    if (amax > 0.0) atomicMax(&misc[3], (unsigned long long)__double_as_longlong(amax));
  }
}

// enters every primitive into the cells of its grown box: FILL = false
// counts per bucket, FILL = true takes slots from the bucket cursors
template <int NV, bool FILL>
__global__ __launch_bounds__(256) void k_cs_insert(int64_t n, const int32_t* ids, const double* x, double h,
                                                   double dhat, uint64_t hmask, int32_t* cnt, uint64_t* ekey,
                                                   int32_t* eid, uint32_t* err) {
  const int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (p >= n) return;
  const Box b = prim_box<NV>(x, ids, p);
  int64_t c0[3], c1[3];
  for (int a = 0; a < 3; ++a) {
    c0[a] = cell_of(b.lo[a] - dhat, h);
    c1[a] = cell_of(b.hi[a] + dhat, h);
    if (c1[a] - c0[a] > 2 || c1[a] < c0[a]) {  // cannot happen with h >= extent + 2 dhat; never loop long
      atomicOr(err, ERRB_INDEX);
      return;
    }
  }
  for (int64_t cx = c0[0]; cx <= c1[0]; ++cx)
    for (int64_t cy = c0[1]; cy <= c1[1]; ++cy)
      for (int64_t cz = c0[2]; cz <= c1[2]; ++cz) {
        const uint64_t k = cell_key(cx, cy, cz);
        const uint64_t bkt = key_hash(k) & hmask;
        if constexpr (!FILL) {
          atomicAdd(&cnt[bkt], 1);
        } else {
          const int slot = atomicAdd(&cnt[bkt], 1);
          ekey[slot] = k;
          eid[slot] = int32_t(p);
        }
      }
}

// Up to HITS pairs a lane has found are appended together with those of
// the other lanes at the next point the whole wavefront reaches: one atomic
// per wavefront instead of one per pair (pairs beyond HITS take their own).
// The lane keeps only the partner's index and recomputes the geometry when
// it writes.
constexpr int HITS = 4;

__device__ __forceinline__ void push_hit(int (&hb)[HITS], int j) {
#pragma unroll
  for (int q = HITS - 1; q > 0; --q) hb[q] = hb[q - 1];
  hb[0] = j;
}

// First output slot of this lane's nb pairs; every lane of the wavefront calls.
__device__ __forceinline__ int64_t wave_reserve(int nb, unsigned long long* count) {
  const int lane = threadIdx.x & 63;
  int incl = nb;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const int total = __shfl(incl, 63);
  unsigned long long base = 0;
  if (total > 0 && lane == 63) base = atomicAdd(count, (unsigned long long)total);
  base = __shfl(base, 63);
  return int64_t(base) + incl - nb;
}

__device__ __forceinline__ void write_pair(int64_t slot, int64_t cap, const int (&q)[4], int kind, const double* x,
                                           int32_t* pairs, uint8_t* kinds, double* dist, double* grad,
                                           uint64_t* keys, uint64_t key) {
  if (slot >= cap) return;
  if (keys) keys[slot] = key;
  const V3 X[4] = {load_v3(x, q[0]), load_v3(x, q[1]), load_v3(x, q[2]), load_v3(x, q[3])};
  double d, wt[4];
  V3 n;
  pair_geometry(X, kind, d, wt, n);
  reinterpret_cast<int4*>(pairs)[slot] = make_int4(q[0], q[1], q[2], q[3]);
  kinds[slot] = uint8_t(kind);
  dist[slot] = d;
  if (grad) store_grad(grad, slot, wt, n);
}

__global__ __launch_bounds__(256) void k_cs_query_pt(int64_t nv, const int32_t* verts, const int32_t* tris,
                                                     const double* x, double h, double dhat, uint64_t hmask,
                                                     const int32_t* off, const uint64_t* ekey, const int32_t* eid,
                                                     int64_t cap, int32_t* pairs, uint8_t* kinds, double* dist,
                                                     double* grad, uint64_t* keys, unsigned long long* count) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int v = 0, e0 = 0, e1 = 0;
  V3 P{};
  uint64_t k = 0;
  if (i < nv) {
    v = verts[i];
    P = load_v3(x, v);
    k = cell_key(cell_of(P.x, h), cell_of(P.y, h), cell_of(P.z, h));
    const uint64_t bkt = key_hash(k) & hmask;
    e0 = off[bkt];
    e1 = off[bkt + 1];
  }
  const Box pb = {{P.x, P.y, P.z}, {P.x, P.y, P.z}};
  const double dh2 = dhat * dhat;
  int hb[HITS] = {0, 0, 0, 0};
  int nb = 0;
  for (int e = e0; e < e1; ++e) {
    if (ekey[e] != k) continue;
    const int t = eid[e];
    const int tv[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (tv[0] == v || tv[1] == v || tv[2] == v) continue;
    if (!(box_dist2(pb, prim_box<3>(x, tris, t)) < dh2)) continue;
    const int q[4] = {v, tv[0], tv[1], tv[2]};
    const V3 X[4] = {P, load_v3(x, tv[0]), load_v3(x, tv[1]), load_v3(x, tv[2])};
    double d, wt[4];
    V3 n;
    pair_geometry(X, 0, d, wt, n);
    if (d < dhat) {
      if (nb < HITS) {
        push_hit(hb, t);
        ++nb;
      } else {
        append_pair(count, cap, q, 0, d, wt, n, pairs, kinds, dist, grad, keys, pair_key(0, i, t));
      }
    }
  }
  const int64_t s0 = wave_reserve(nb, count);
#pragma unroll
  for (int q = 0; q < HITS; ++q) {
    if (q < nb) {
      const int t = hb[q];
      const int ids[4] = {v, tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
      write_pair(s0 + q, cap, ids, 0, x, pairs, kinds, dist, grad, keys, pair_key(0, i, t));
    }
  }
}

__global__ __launch_bounds__(256) void k_cs_query_ee(int64_t ne, const int32_t* edges, const double* x, double h,
                                                     double dhat, uint64_t hmask, const int32_t* off,
                                                     const uint64_t* ekey, const int32_t* eid, int64_t cap,
                                                     int32_t* pairs, uint8_t* kinds, double* dist, double* grad,
                                                     uint64_t* keys, unsigned long long* count, uint32_t* err) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int a0 = 0, a1 = 0, ncell = 0;
  int64_t c0[3] = {0, 0, 0}, span[3] = {1, 1, 1};
  Box ab{};
  if (i < ne) {
    a0 = edges[2 * i];
    a1 = edges[2 * i + 1];
    ab = prim_box<2>(x, edges, i);
    ncell = 1;
    for (int a = 0; a < 3; ++a) {
      c0[a] = cell_of(ab.lo[a], h);
      span[a] = cell_of(ab.hi[a], h) - c0[a] + 1;
      if (span[a] > 3 || span[a] < 1) {  // as in k_cs_insert
        atomicOr(err, ERRB_INDEX);
        ncell = 0;
        span[a] = 1;
      }
    }
    if (ncell) ncell = int(span[0] * span[1] * span[2]);
  }
  const double dh2 = dhat * dhat;
  // one cell per step for every lane, so that the appends after each step
  // are reached by the whole wavefront
  for (int cell = 0; __ballot(cell < ncell) != 0ull; ++cell) {
    int hb[HITS] = {0, 0, 0, 0};
    int nb = 0;
    if (cell < ncell) {
      const int64_t cx = c0[0] + cell % span[0], cy = c0[1] + (cell / span[0]) % span[1],
                    cz = c0[2] + cell / (span[0] * span[1]);
      const uint64_t k = cell_key(cx, cy, cz);
      const uint64_t bkt = key_hash(k) & hmask;
      for (int e = off[bkt]; e < off[bkt + 1]; ++e) {
        if (ekey[e] != k) continue;
        const int j = eid[e];
        if (j <= i) continue;
        const int b0 = edges[2 * j], b1 = edges[2 * j + 1];
        if (b0 == a0 || b0 == a1 || b1 == a0 || b1 == a1) continue;
        const Box bb = prim_box<2>(x, edges, j);
        if (!(box_dist2(ab, bb) < dh2)) continue;
        // report from the cell of the lower corner of the overlap of the own box and the grown partner box
        const int64_t rx = cell_of(fmax(ab.lo[0], bb.lo[0] - dhat), h);
        const int64_t ry = cell_of(fmax(ab.lo[1], bb.lo[1] - dhat), h);
        const int64_t rz = cell_of(fmax(ab.lo[2], bb.lo[2] - dhat), h);
        if (rx != cx || ry != cy || rz != cz) continue;
        const int q[4] = {a0, a1, b0, b1};
        const V3 X[4] = {load_v3(x, a0), load_v3(x, a1), load_v3(x, b0), load_v3(x, b1)};
        double d, wt[4];
        V3 n;
        pair_geometry(X, 1, d, wt, n);
        if (d < dhat) {
          if (nb < HITS) {
            push_hit(hb, j);
            ++nb;
          } else {
            append_pair(count, cap, q, 1, d, wt, n, pairs, kinds, dist, grad, keys, pair_key(1, i, j));
          }
        }
      }
    }
    const int64_t s0 = wave_reserve(nb, count);
#pragma unroll
    for (int q = 0; q < HITS; ++q) {
      if (q < nb) {
        const int j = hb[q];
        const int ids[4] = {a0, a1, edges[2 * j], edges[2 * j + 1]};
        write_pair(s0 + q, cap, ids, 1, x, pairs, kinds, dist, grad, keys, pair_key(1, i, j));
      }
    }
  }
}

// the tables were allocated by mas_create; a request beyond them is an
// argument error
static mas_status check_table(const Ctx::CellTable& t, int64_t H, int64_t E) {
  return (H + 1 > t.h_cap || E > t.e_cap) ? MAS_ERR_INVALID_ARG : MAS_OK;
}

static int64_t pow2_at_least(int64_t n) {
  int64_t H = 1024;
  while (H < n) H <<= 1;
  return H;
}

mas_status launch_constraint_set(Ctx& c, const double* x, double dhat, int64_t nv, const int32_t* verts, int64_t nt,
                                 const int32_t* tris, int64_t ne, const int32_t* edges, int64_t cap, int32_t* pairs,
                                 uint8_t* kind, double* dist, double* grad, uint64_t* key, int64_t* count) {
  ProfScope ps(c, MAS_T_CSET);
  *count = 0;
  if (nt > c.cfg.max_tris || ne > c.cfg.max_edges) return MAS_ERR_INVALID_ARG;
  HIPCHK(hipMemsetAsync(c.cs_misc, 0, 4 * sizeof(unsigned long long), c.s));
  if (nt + ne == 0) return MAS_OK;
  const int64_t prep_grid = std::min<int64_t>((nt + ne + nv + 255) / 256, int64_t(c.n_cu) * 8);
  k_cs_prep<<<dim3(prep_grid), dim3(256), 0, c.s>>>(c.N, nt, tris, ne, edges, nv, verts, x, c.cs_misc);
  unsigned long long misc[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(misc, c.cs_misc, sizeof(misc), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  if (misc[2] & 1ull) return MAS_ERR_INVALID_ARG;
  if (misc[2] & 2ull) return MAS_ERR_NONFINITE;
  double ext, amax;
  std::memcpy(&ext, &misc[0], sizeof(ext));
  std::memcpy(&amax, &misc[3], sizeof(amax));
  const double h = ext + 2.0 * dhat;
  // cell indices |x| / h must stay far inside int64
  if (!(h > 0.0) || !std::isfinite(h) || amax / h > 1e15) return MAS_ERR_INVALID_ARG;
  const int64_t n[2] = {nt, ne};
  const int32_t* ids[2] = {tris, edges};
  int64_t H[2];
  int32_t total[2] = {0, 0};
  for (int k = 0; k < 2; ++k) {
    H[k] = pow2_at_least(2 * n[k]);
    mas_status st = check_table(c.cs[k], H[k], 0);
    if (st != MAS_OK) return st;
    HIPCHK(hipMemsetAsync(c.cs[k].cnt, 0, sizeof(int32_t) * (H[k] + 1), c.s));
    if (n[k] == 0) continue;
    const dim3 g((n[k] + 255) / 256);
    if (k == 0)
      k_cs_insert<3, false><<<g, dim3(256), 0, c.s>>>(n[k], ids[k], x, h, dhat, uint64_t(H[k] - 1), c.cs[k].cnt,
                                                       nullptr, nullptr, c.err);
    else
      k_cs_insert<2, false><<<g, dim3(256), 0, c.s>>>(n[k], ids[k], x, h, dhat, uint64_t(H[k] - 1), c.cs[k].cnt,
                                                       nullptr, nullptr, c.err);
    mas_status s2 = exclusive_scan_i32(c, c.cs[k].cnt, c.cs[k].off, H[k] + 1);
    if (s2 != MAS_OK) return s2;
    HIPCHK(hipMemcpyAsync(&total[k], c.cs[k].off + H[k], sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
  }
  HIPCHK(hipStreamSynchronize(c.s));
  for (int k = 0; k < 2; ++k) {
    if (n[k] == 0) continue;
    if (total[k] < 0) return MAS_ERR_INVALID_ARG;  // more than 2^31 cell entries
    mas_status st = check_table(c.cs[k], H[k], std::max<int64_t>(total[k], 1));
    if (st != MAS_OK) return st;
    HIPCHK(hipMemcpyAsync(c.cs[k].cnt, c.cs[k].off, sizeof(int32_t) * H[k], hipMemcpyDeviceToDevice, c.s));
    const dim3 g((n[k] + 255) / 256);
    if (k == 0)
      k_cs_insert<3, true><<<g, dim3(256), 0, c.s>>>(n[k], ids[k], x, h, dhat, uint64_t(H[k] - 1), c.cs[k].cnt,
                                                      c.cs[k].key, c.cs[k].id, c.err);
    else
      k_cs_insert<2, true><<<g, dim3(256), 0, c.s>>>(n[k], ids[k], x, h, dhat, uint64_t(H[k] - 1), c.cs[k].cnt,
                                                      c.cs[k].key, c.cs[k].id, c.err);
  }
  unsigned long long* cnt = c.cs_misc + 1;
  if (nv > 0 && nt > 0)
    k_cs_query_pt<<<dim3((nv + 255) / 256), dim3(256), 0, c.s>>>(nv, verts, tris, x, h, dhat, uint64_t(H[0] - 1),
                                                                  c.cs[0].off, c.cs[0].key, c.cs[0].id, cap, pairs,
                                                                  kind, dist, grad, key, cnt);
  if (ne > 1)
    k_cs_query_ee<<<dim3((ne + 255) / 256), dim3(256), 0, c.s>>>(ne, edges, x, h, dhat, uint64_t(H[1] - 1),
                                                                  c.cs[1].off, c.cs[1].key, c.cs[1].id, cap, pairs,
                                                                  kind, dist, grad, key, cnt, c.err);
  HIPCHK(hipGetLastError());
  unsigned long long found = 0;
  HIPCHK(hipMemcpyAsync(&found, cnt, sizeof(found), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  *count = int64_t(found);
  return MAS_OK;
}

}  // namespace mas
