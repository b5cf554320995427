// 3x3 block-Jacobi comparison preconditioner (precond = MAS_PRECOND_BJ3):
// the preconditioner that MAS is measured against in the paper's
// preconditioner-efficacy study (Section 5).  Each vertex keeps the packed
// lower 3x3 diagonal block of H~ = H_base + U U^T and its inverse; applying
// it is one 3x3 product per vertex.  H_base's vertex blocks are read from
// the level-0 assembly (every tet, base contact and the mass touching a
// vertex land in its subdomain's block), so no separate assembly pass is
// needed; the update columns add u_j u_j^T to each of their vertices.
#include "common.hpp"
#include "kernels.hpp"

namespace mas {

// packed lower 3x3: (00, 10, 11, 20, 21, 22)
__global__ void k_bj_base(int64_t N, const double* __restrict__ acc0, double* __restrict__ bj) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  const double* blk = acc0 + (v >> 5) * int64_t(PK);
  const int r = 3 * int(v & 31);
  double* o = bj + 6 * v;
  o[0] = blk[pk(r, r)];
  o[1] = blk[pk(r + 1, r)];
  o[2] = blk[pk(r + 1, r + 1)];
  o[3] = blk[pk(r + 2, r)];
  o[4] = blk[pk(r + 2, r + 1)];
  o[5] = blk[pk(r + 2, r + 2)];
}

// the update columns: u_j u_j^T into the block of each vertex j of column c
__global__ void k_bj_cols(int64_t m, const int32_t* __restrict__ Uidx, const double* __restrict__ U,
                          const double* __restrict__ dS, double* bj) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= m || !(dS[c] > 0.0)) return;  // zero column (not stored)
  const int4 iv = reinterpret_cast<const int4*>(Uidx)[c];
  const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (vi[j] < 0) continue;
    const double* u = U + 12 * c + 3 * j;
    const double u0 = u[0], u1 = u[1], u2 = u[2];
    double* o = bj + 6 * int64_t(vi[j]);
    unsafeAtomicAdd(o + 0, u0 * u0);
    unsafeAtomicAdd(o + 1, u1 * u0);
    unsafeAtomicAdd(o + 2, u1 * u1);
    unsafeAtomicAdd(o + 3, u2 * u0);
    unsafeAtomicAdd(o + 4, u2 * u1);
    unsafeAtomicAdd(o + 5, u2 * u2);
  }
}

// B^-1 = L^-T L^-1 from the Cholesky factor L of B (float64).  A block that
// is not positive definite gets a zero inverse and sets ERRB_NOT_SPD.
__global__ void k_bj_invert(int64_t N, const double* __restrict__ bj, double* __restrict__ bjinv, uint32_t* err) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  const double* b = bj + 6 * v;
  double* o = bjinv + 6 * v;
  const double a00 = b[0], a10 = b[1], a11 = b[2], a20 = b[3], a21 = b[4], a22 = b[5];
  bool ok = a00 > 0.0;
  const double l00 = sqrt(a00);
  const double l10 = a10 / l00, l20 = a20 / l00;
  const double e1 = a11 - l10 * l10;
  ok = ok && e1 > 0.0;
  const double l11 = sqrt(e1);
  const double l21 = (a21 - l20 * l10) / l11;
  const double e2 = a22 - l20 * l20 - l21 * l21;
  ok = ok && e2 > 0.0 && isfinite(e2);
  if (!ok) {
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = 0.0;
    atomicOr(err, ERRB_NOT_SPD);
    return;
  }
  const double l22 = sqrt(e2);
  // M = L^-1 (lower)
  const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
  const double m10 = -l10 * m00 * m11;
  const double m21 = -l21 * m11 * m22;
  const double m20 = -(l20 * m00 + l21 * m10) * m22;
  o[0] = m00 * m00 + m10 * m10 + m20 * m20;
  o[1] = m11 * m10 + m21 * m20;
  o[2] = m11 * m11 + m21 * m21;
  o[3] = m22 * m20;
  o[4] = m22 * m21;
  o[5] = m22 * m22;
}

// z_i = B_i^-1 g_i
__global__ void k_bj_apply(int64_t N, const double* __restrict__ bjinv, const double* __restrict__ g,
                           double* __restrict__ z, uint32_t* err) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  const double* q = bjinv + 6 * v;
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
  const double g0 = g[3 * v], g1 = g[3 * v + 1], g2 = g[3 * v + 2];
  if (!isfinite(g0) || !isfinite(g1) || !isfinite(g2)) atomicOr(err, ERRB_NONFINITE);
  z[3 * v] = q0 * g0 + q1 * g1 + q3 * g2;
  z[3 * v + 1] = q1 * g0 + q2 * g1 + q4 * g2;
  z[3 * v + 2] = q3 * g0 + q4 * g1 + q5 * g2;
}

static inline dim3 vgrid(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

mas_status launch_bj_build(Ctx& c) {
  k_bj_base<<<vgrid(c.N), dim3(256), 0, c.s>>>(c.N, c.lv[0].acc, c.bj);
  k_bj_invert<<<vgrid(c.N), dim3(256), 0, c.s>>>(c.N, c.bj, c.bjinv, c.err);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status launch_bj_update(Ctx& c, int64_t m) {
  k_bj_base<<<vgrid(c.N), dim3(256), 0, c.s>>>(c.N, c.lv[0].acc, c.bj);
  if (m > 0) k_bj_cols<<<vgrid(m), dim3(256), 0, c.s>>>(m, c.Uidx, c.U, c.dS, c.bj);
  k_bj_invert<<<vgrid(c.N), dim3(256), 0, c.s>>>(c.N, c.bj, c.bjinv, c.err);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status launch_bj_apply(Ctx& c, const double* g, double* z) {
  ProfScope ps(c, MAS_T_APPLY);
  k_bj_apply<<<vgrid(c.N), dim3(256), 0, c.s>>>(c.N, c.bjinv, g, z, c.err);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
