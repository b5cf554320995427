// Preconditioner apply z = P g (supplement Eq. (4)): restriction to every
// coarse level, coarse block products, then one workgroup per level-0
// subdomain applies its inverse block, the Woodbury correction (Section 4.1)
// and adds the coarse corrections of the subdomain's vertices.
#include <algorithm>

#include "kernels.hpp"

namespace mas {

// Restriction C_(l) g (supplement Section 1.3), level by level: the value
// of node a at level l (component c) is the sum over its 32 children at
// level l - 1 (level 0: the vertices).
__global__ void k_restrict(int64_t n_child, int64_t nodes, const double* child, double* out) {
  const int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (q >= 3 * nodes) return;
  const int64_t a = q / 3;
  const int c = int(q % 3);
  const int64_t v0 = SUB * a, v1 = min<int64_t>(v0 + SUB, n_child);
  double s = 0;
  for (int64_t v = v0; v < v1; ++v) s += child[3 * v + c];
  out[q] = s;
}

// ---------------------------------------------------------------------------
// y = B x for one stored block, 128 threads, thread t on tile t of the tiled
// layout.  The tile's units are loaded straight into registers (every
// wavefront access is one contiguous 512-byte piece); x goes through LDS;
// each tile produces a row-side and a column-side partial of six sums
// (diagonal pairs only row sides), collected in LDS as part[b][s] for row
// tile b and partner tile s, 16 per row tile, and summed by threads 0..95.
// 16-bit blocks hold B_ij / (sig_i sig_j): x is scaled by sig before and y
// after.  Arithmetic in float64.
constexpr int PB = 102;  // doubles per row tile in part[] (16 x 6, padded against bank conflicts)

template <int P>
__device__ __forceinline__ double decode_entry(uint2 w, int e) {
  if constexpr (P == MAS_F64) {
    return __hiloint2double(int(w.y), int(w.x));
  } else if constexpr (P == MAS_F32) {
    return double(__uint_as_float((e & 1) ? w.y : w.x));
  } else {
    const uint32_t h2 = (e & 2) ? w.y : w.x;
    const uint16_t h = uint16_t((e & 1) ? (h2 >> 16) : (h2 & 0xffffu));
    return double((P == MAS_BF16) ? bf16_to_f32(h) : f16_to_f32(h));
  }
}

// Entry e of this thread's tile: from the registers loaded up front, or
// (STREAM) loaded from memory where it is used, which keeps the registers
// of a rarely taken wide path from setting the occupancy of the kernel.
template <int P, bool STREAM>
__device__ __forceinline__ double tile_entry(const uint2 (&u)[STREAM ? 1 : tile_ud(P)], const uint2* s2, int t,
                                             int e) {
  if constexpr (STREAM) return decode_entry<P>(ld_once(s2 + tile_unit(P, t, e / tile_epu(P))), e);
  else return decode_entry<P>(u[e / tile_epu(P)], e);
}

template <int P, bool STREAM = false>
__device__ __forceinline__ double block_apply(const unsigned char* slot, const float* scale_d, double xv, int bi,
                                              int bj, double* xs, double* part) {
  constexpr int UO = tile_uo(P), UD = tile_ud(P);
  constexpr bool q16 = (P == MAS_BF16 || P == MAS_F16);
  const int t = threadIdx.x;
  const bool diag = t >= 120;
  uint2 u[STREAM ? 1 : UD];
  const uint2* s2 = reinterpret_cast<const uint2*>(slot);
  if constexpr (!STREAM) {
#pragma unroll
    for (int k = 0; k < UD; ++k) {
      u[k] = make_uint2(0u, 0u);
      if (k < UO || diag) u[k] = ld_once(s2 + tile_unit(P, t, k));
    }
  }
  float sg = 1.0f;
  if (t < BD) {
    if (q16) sg = scale_d[t];
    xs[t] = q16 ? xv * double(sg) : xv;
  }
  __syncthreads();
  if (!diag) {
    double xi[6], xj[6], y[6], w[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      xi[q] = xs[6 * bi + q];
      xj[q] = xs[6 * bj + q];
      w[q] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double a = tile_entry<P, STREAM>(u, s2, t, 6 * r + q);
        acc += a * xj[q];
        w[q] += a * xi[r];
      }
      y[r] = acc;
    }
    double* pr = part + bi * PB + 6 * bj;
    double* pc = part + bj * PB + 6 * bi;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      pr[q] = y[q];
      pc[q] = w[q];
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = 2 * (t - 120) + h;
      double xb[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) xb[q] = xs[6 * b + q];
      double* pd = part + b * PB + 6 * b;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          acc += tile_entry<P, STREAM>(u, s2, t, 21 * h + (r >= q ? r * (r + 1) / 2 + q : q * (q + 1) / 2 + r)) *
                 xb[q];
        pd[r] = acc;
      }
    }
  }
  __syncthreads();
  double z = 0.0;
  if (t < BD) {
    const double* pz = part + (t / 6) * PB + t % 6;
#pragma unroll
    for (int s = 0; s < 16; ++s) z += pz[6 * s];
    if (q16) z *= double(sg);
  }
  return z;
}

// WIDE = false: float64 blocks (promoted ones when a narrower format was
// requested) take the streamed path.
template <bool WIDE = true>
__device__ __forceinline__ double block_apply_any(int P, const unsigned char* slot, const float* scale_d, double xv,
                                                  int bi, int bj, double* xs, double* part) {
  switch (P) {
    case MAS_F64: return block_apply<MAS_F64, !WIDE>(slot, scale_d, xv, bi, bj, xs, part);
    case MAS_F32: return block_apply<MAS_F32>(slot, scale_d, xv, bi, bj, xs, part);
    case MAS_BF16: return block_apply<MAS_BF16>(slot, scale_d, xv, bi, bj, xs, part);
    default: return block_apply<MAS_F16>(slot, scale_d, xv, bi, bj, xs, part);
  }
}

struct CoarseBlocks {
  int L;
  int64_t first[MAXL + 1];  // prefix of subdomain counts over levels 1..L-1
  int64_t nodes[MAXL];
  const void* blk[MAXL];
  const uint8_t* bprec[MAXL];
  const float* scale[MAXL];
  const double* r[MAXL];
  double* c[MAXL];
};

__global__ __launch_bounds__(NTILE) void k_apply_coarse(CoarseBlocks cb) {
  __shared__ double xs[BD];
  __shared__ __align__(16) double part[16 * PB];
  const int64_t gb = blockIdx.x;
  int l = 1;
  while (l + 1 < cb.L && gb >= cb.first[l + 1]) ++l;
  const int64_t d = gb - cb.first[l];
  const int t = threadIdx.x;
  int bi = 0, bj = 0;
  if (t < 120) tile_rc(t, bi, bj);
  const int64_t a = SUB * d + t / 3;
  const double xv = (t < BD && a < cb.nodes[l]) ? cb.r[l][BD * d + t] : 0.0;
  const unsigned char* slot = reinterpret_cast<const unsigned char*>(cb.blk[l]) + d * BLK_STRIDE;
  const double v = block_apply_any(cb.bprec[l][d], slot, cb.scale[l] + BD * d, xv, bi, bj, xs, part);
  if (t < BD && a < cb.nodes[l]) cb.c[l][BD * d + t] = v;
}

struct FineArgs {
  int64_t N;
  const void* blk;
  const uint8_t* bprec;
  const float* scale;
  const double* g;
  double* z;
  const int32_t* rank;  // nullptr: no Woodbury update
  int K;
  const SlotCol* slots;
  const double* W;
  const double* Lcap;
  int L;
  const double* c[MAXL];
  uint32_t* err;
};

// One workgroup per level-0 subdomain d: z_d = B_d g_d, minus the Woodbury
// correction W_d C_d^-1 U_d^T B_d g_d where the subdomain was updated, plus
// the coarse corrections of its vertices.
template <bool WIDE>
__global__ __launch_bounds__(NTILE, WIDE ? 4 : 5) void k_apply_l0(FineArgs fa) {
  __shared__ double xs[BD];
  __shared__ __align__(16) double part[16 * PB];
  // Woodbury scratch sized by K: factor, r, lambda, slot columns
  extern __shared__ __align__(16) double wdyn[];
  const int K = fa.K;
  double* Lf = wdyn;
  double* rr = Lf + K * (K + 1) / 2;
  double* lam = rr + K;
  SlotCol* sl = reinterpret_cast<SlotCol*>(lam + K + ((K * (K + 1) / 2 + 2 * K) & 1));
  double* zb = part;  // the base product, after the partials are consumed
  const int64_t d = blockIdx.x;
  const int t = threadIdx.x;
  const int r = fa.rank ? fa.rank[d] : 0;
  if (r > 0) {
    const double* Lm = fa.Lcap + d * (K * (K + 1) / 2);
    for (int q = t; q < r * (r + 1) / 2; q += blockDim.x) Lf[q] = Lm[q];
    if (t < r) sl[t] = fa.slots[d * K + t];
  }
  int bi = 0, bj = 0;
  if (t < 120) tile_rc(t, bi, bj);
  const int64_t v = SUB * d + t / 3;
  double xv = 0.0, corr = 0.0;
  if (t < BD && v < fa.N) {
    xv = fa.g[BD * d + t];
    if (!isfinite(xv)) atomicOr(fa.err, ERRB_NONFINITE);
#pragma unroll
    for (int l = 1; l < MAXL; ++l)
      if (l < fa.L) corr += fa.c[l][3 * (v >> (5 * l)) + t % 3];
  }
  const unsigned char* slot = reinterpret_cast<const unsigned char*>(fa.blk) + d * BLK_STRIDE;
  double zv = block_apply_any<WIDE>(fa.bprec[d], slot, fa.scale + BD * d, xv, bi, bj, xs, part);
  if (r > 0) {
    __syncthreads();
    if (t < BD) zb[t] = zv;
    __syncthreads();
    // r_j = u_j^T z_base over the stencil vertices inside the subdomain
    if (t < r) {
      double acc = 0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int lv = sl[t].lv[s];
        if (lv < 0) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc += sl[t].u[3 * s + a] * zb[3 * lv + a];
      }
      rr[t] = acc;
    }
    __syncthreads();
    if (t == 0) {
      // (L L^T) lambda = r: forward substitution in place in rr, then backward
      for (int i = 0; i < r; ++i) {
        double y = rr[i];
        for (int k = 0; k < i; ++k) y -= Lf[pk(i, k)] * rr[k];
        rr[i] = y / Lf[pk(i, i)];
      }
      for (int i = r - 1; i >= 0; --i) {
        double y = rr[i];
        for (int k = i + 1; k < r; ++k) y -= Lf[pk(k, i)] * lam[k];
        lam[i] = y / Lf[pk(i, i)];
      }
    }
    __syncthreads();
    if (t < BD) {
      const double* Wd = fa.W + d * K * BD;
      double acc = 0;
      for (int j = 0; j < r; ++j) acc += Wd[j * BD + t] * lam[j];
      zv -= acc;
    }
  }
  if (t < BD && v < fa.N) fa.z[BD * d + t] = zv + corr;
}

mas_status launch_apply(Ctx& c, const double* g, double* z) {
  if (c.cfg.precond == MAS_PRECOND_BJ3) return launch_bj_apply(c, g, z);
  ProfScope ps(c, MAS_T_APPLY);
  if (c.L > 1) {
    for (int l = 1; l < c.L; ++l) {
      const int64_t n = c.lv[l].nodes;
      k_restrict<<<dim3((3 * n + 255) / 256), dim3(256), 0, c.s>>>(c.lv[l - 1].nodes, n,
                                                                   l == 1 ? g : c.lv[l - 1].r, c.lv[l].r);
    }
    CoarseBlocks cb{};
    cb.L = c.L;
    cb.first[1] = 0;
    for (int l = 1; l < c.L; ++l) {
      cb.first[l + 1] = cb.first[l] + c.lv[l].nsub;
      cb.nodes[l] = c.lv[l].nodes;
      cb.blk[l] = c.lv[l].blk;
      cb.bprec[l] = c.lv[l].bprec;
      cb.scale[l] = c.lv[l].scale;
      cb.r[l] = c.lv[l].r;
      cb.c[l] = c.lv[l].c;
    }
    int64_t total = cb.first[c.L];
    k_apply_coarse<<<dim3(total), dim3(NTILE), 0, c.s>>>(cb);
  }
  FineArgs fa{};
  fa.N = c.N;
  fa.blk = c.lv[0].blk;
  fa.bprec = c.lv[0].bprec;
  fa.scale = c.lv[0].scale;
  fa.g = g;
  fa.z = z;
  fa.rank = c.have_update && c.K > 0 ? c.rank : nullptr;
  fa.K = c.K;
  fa.slots = c.slots;
  fa.W = c.W;
  fa.Lcap = c.Lcap;
  fa.L = c.L;
  for (int l = 1; l < c.L; ++l) fa.c[l] = c.lv[l].c;
  fa.err = c.err;
  prof_begin(c, MAS_T_APPLY_L0);
  const int K = std::max(c.K, 1);
  const size_t wlds = sizeof(double) * size_t(K * (K + 1) / 2 + 2 * K + 1) + sizeof(SlotCol) * size_t(K);
  if (c.lv[0].prec == MAS_F64)
    k_apply_l0<true><<<dim3(c.lv[0].nsub), dim3(NTILE), wlds, c.s>>>(fa);
  else
    k_apply_l0<false><<<dim3(c.lv[0].nsub), dim3(NTILE), wlds, c.s>>>(fa);
  prof_end(c, MAS_T_APPLY_L0);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
