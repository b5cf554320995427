// RebuildMAS: the frozen element Hessians, the base contact set, level-0
// subdomain blocks (assembled and inverted inside one workgroup) and the
// Galerkin coarse blocks of every level.
#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

// ---------------------------------------------------------------------------
// Element snapshot: per tet the 9x9 tangent of h^2 V Psi with its negative
// eigenvalues clamped, packed (45), followed by Dm^-1 (9).  AoSoA layout:
// tile t/64, component, lane t%64 - one wavefront reads a component with one
// coalesced 512-byte (f64) access.
__global__ __launch_bounds__(64) void k_elem_hess(int64_t T, int64_t Tpad, const int32_t* tets,
                                                  const double* geo, const double* x, double h,
                                                  double* hf64, float* hf32) {
  int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= Tpad) return;
  double H[45];
  double Dmi[9];
  if (t < T) {
    double xe[12];
    for (int j = 0; j < 4; ++j) {
      int v = tets[4 * t + j];
      for (int a = 0; a < 3; ++a) xe[3 * j + a] = x[3 * v + a];
    }
    const double* g = geo + 12 * t;
#pragma unroll
    for (int q = 0; q < 9; ++q) Dmi[q] = g[q];
    double F[3][3];
    def_grad(xe, Dmi, F);
    snh_tangent_psd(F, g[10], g[11], H);
    double s = h * h * g[9];
#pragma unroll
    for (int q = 0; q < 45; ++q) H[q] *= s;
  } else {
#pragma unroll
    for (int q = 0; q < 45; ++q) H[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) Dmi[q] = 0.0;
  }
  int64_t base = (t / TILE) * (EH * TILE) + (t % TILE);
#pragma unroll
  for (int q = 0; q < 45; ++q) hf64[base + q * TILE] = H[q];
#pragma unroll
  for (int q = 0; q < 9; ++q) hf64[base + (45 + q) * TILE] = Dmi[q];
  if (hf32) {
#pragma unroll
    for (int q = 0; q < 45; ++q) hf32[base + q * TILE] = float(H[q]);
#pragma unroll
    for (int q = 0; q < 9; ++q) hf32[base + (45 + q) * TILE] = float(Dmi[q]);
  }
}

mas_status launch_elem_hessians(Ctx& c, const double* x_base) {
  k_elem_hess<<<dim3(c.Tpad / TILE), dim3(TILE), 0, c.s>>>(c.T, c.Tpad, c.tets, c.geo, x_base,
                                                            c.cfg.h, c.hf64, c.hf32);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

__device__ inline void load_snapshot(const double* hf64, int64_t t, double* H, double* Dmi) {
  int64_t base = (t / TILE) * (EH * TILE) + (t % TILE);
#pragma unroll
  for (int q = 0; q < 45; ++q) H[q] = hf64[base + q * TILE];
#pragma unroll
  for (int q = 0; q < 9; ++q) Dmi[q] = hf64[base + (45 + q) * TILE];
}

// ---------------------------------------------------------------------------
// Base contact set: copy, stiffness k = kappa b''(d) and columns sqrt(k) n.
__global__ void k_base_copy(int64_t m, const uint64_t* key, const int32_t* idx, const double* d,
                            const double* grad, double kappa, double dhat, uint64_t* bkey,
                            int32_t* biota, double* bk, double* bgrad, int32_t* bidx, double* bu,
                            uint32_t* err) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= m) return;
  double b, b1, b2;
  double di = d[i];
  if (!isfinite(di)) atomicOr(err, ERRB_NONFINITE);
  barrier3(di, dhat, &b, &b1, &b2);
  double k = kappa * b2;
  bk[i] = k;
  bkey[i] = key[i];
  biota[i] = int32_t(i);
  double sk = sqrt(k);
  for (int q = 0; q < 12; ++q) {
    double n = grad[12 * i + q];
    bgrad[12 * i + q] = n;
    bu[12 * i + q] = sk * n;
  }
  for (int q = 0; q < 4; ++q) bidx[4 * i + q] = idx[4 * i + q];
}

static mas_status grow_base(Ctx& c, int64_t m) {
  if (m <= c.mb_cap) return MAS_OK;
  int64_t cap = m + m / 4 + 1024;
  hipFree(c.bkey); hipFree(c.bkey_sorted); hipFree(c.biota); hipFree(c.bperm);
  hipFree(c.bk); hipFree(c.bgrad); hipFree(c.bidx); hipFree(c.bu); hipFree(c.bc_list);
  for (int l = 1; l < c.L; ++l) {
    hipFree(c.lv[l].xc_list);
    c.lv[l].xc_list = nullptr;
    if (hipMalloc(&c.lv[l].xc_list, 16 * cap) != hipSuccess) return MAS_ERR_OOM;
  }
  bool ok = hipMalloc(&c.bkey, 8 * cap) == hipSuccess && hipMalloc(&c.bkey_sorted, 8 * cap) == hipSuccess &&
            hipMalloc(&c.biota, 4 * cap) == hipSuccess && hipMalloc(&c.bperm, 4 * cap) == hipSuccess &&
            hipMalloc(&c.bk, 8 * cap) == hipSuccess && hipMalloc(&c.bgrad, 96 * cap) == hipSuccess &&
            hipMalloc(&c.bidx, 16 * cap) == hipSuccess && hipMalloc(&c.bu, 96 * cap) == hipSuccess &&
            hipMalloc(&c.bc_list, 16 * cap) == hipSuccess;
  if (!ok) return MAS_ERR_OOM;
  c.mb_cap = cap;
  return MAS_OK;
}

mas_status launch_base_contacts(Ctx& c, const mas_contacts* b) {
  int64_t m = b ? b->m : 0;
  mas_status st = grow_base(c, m > 0 ? m : 1);
  if (st != MAS_OK) return st;
  c.mb = m;
  if (m > 0) {
    int bs = 256;
    k_base_copy<<<dim3((m + bs - 1) / bs), dim3(bs), 0, c.s>>>(
        m, b->key, b->idx, b->d, b->grad, c.cfg.kappa, c.cfg.dhat, c.bkey, c.biota, c.bk, c.bgrad,
        c.bidx, c.bu, c.err);
    HIPCHK(hipGetLastError());
    st = sort_keys(c, m, c.bkey, c.bkey_sorted, c.biota, c.bperm);
    if (st != MAS_OK) return st;
  }
  st = bucket_by_subdomain(c, 0, m, c.bidx, c.bk, c.bgrad, c.bc_cnt, c.bc_off, c.bc_list);
  if (st != MAS_OK) return st;
  for (int l = 1; l < c.L; ++l) {
    Level& Lv = c.lv[l];
    st = bucket_by_subdomain(c, l, m, c.bidx, c.bk, c.bgrad, Lv.xc_cnt, Lv.xc_off, Lv.xc_list);
    if (st != MAS_OK) return st;
  }
  return MAS_OK;
}

// ---------------------------------------------------------------------------
// 1/x: hardware reciprocal refined by two Newton steps (x positive, normal)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Inverse of a small SPD block (W = 1, 2, 3) by cofactors.  pivot receives
// the first non-positive leading minor (or the last one if all are positive).
template <int W>
__device__ __forceinline__ bool small_spd_inv(const double (&a)[W][W], double (&m)[W][W], double& pivot) {
  if constexpr (W == 1) {
    pivot = a[0][0];
    m[0][0] = rcp_nr(a[0][0]);
    return a[0][0] > 0.0 && isfinite(a[0][0]);
  } else if constexpr (W == 2) {
    const double det = a[0][0] * a[1][1] - a[1][0] * a[1][0];
    pivot = a[0][0] > 0.0 ? det : a[0][0];
    const double id = rcp_nr(det);
    m[0][0] = a[1][1] * id;
    m[1][1] = a[0][0] * id;
    m[0][1] = m[1][0] = -a[1][0] * id;
    return a[0][0] > 0.0 && det > 0.0 && isfinite(det);
  } else {
    const double c00 = a[1][1] * a[2][2] - a[2][1] * a[2][1];
    const double c10 = a[2][1] * a[2][0] - a[1][0] * a[2][2];
    const double c20 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    const double det = a[0][0] * c00 + a[1][0] * c10 + a[2][0] * c20;
    const double m2 = a[0][0] * a[1][1] - a[1][0] * a[1][0];
    pivot = !(a[0][0] > 0.0) ? a[0][0] : (!(m2 > 0.0) ? m2 : det);
    const double id = rcp_nr(det);
    m[0][0] = c00 * id;
    m[1][0] = m[0][1] = c10 * id;
    m[2][0] = m[0][2] = c20 * id;
    m[1][1] = (a[0][0] * a[2][2] - a[2][0] * a[2][0]) * id;
    m[2][1] = m[1][2] = (a[2][0] * a[1][0] - a[0][0] * a[2][1]) * id;
    m[2][2] = m2 * id;
    return a[0][0] > 0.0 && m2 > 0.0 && det > 0.0 && isfinite(det);
  }
}

// In-place inverse of an SPD 96x96 matrix held packed-lower in LDS with the
// symmetric sweep operator (Goodnight 1979), which maps A to -A^-1 once every
// pivot has been swept; sweeping a set K of pivots at once is
//   A_ij -= A_iK A_KK^-1 A_Kj,  A_iK <- A_iK A_KK^-1,  A_KK <- -A_KK^-1.
// The matrix is first scaled to unit diagonal (sc = diag^-1/2).  Thread
// t < 136 keeps the 6x6 tile (ti, tj), ti >= tj, of a 16x16 tile grid in
// registers; per panel of W pivots the W pivot columns pass through LDS (a
// double buffer that reuses A's storage, one barrier per panel).  All three
// updates are one rank-W product R -= P Q^T with P the panel, its KK part
// lowered by I, and Q = P A_KK^-1; it leaves the diagonal of A_KK too large by
// exactly 2, and no later panel reads those entries, so 2 is taken off at the
// end.  With unit diagonal, the diagonal of -A^-1 is at most -1 and the shift
// costs no accuracy.
template <int W>
__device__ __forceinline__ void spd_invert_lds(double* A, double* sc, uint32_t* err, DiagRec* dg, int source,
                                               int level, int64_t index) {
  const int tid = threadIdx.x;
  const bool act = tid < 136;
  int ti = 0, tj = 0;
  if (act) {
    ti = int((sqrt(8.0 * tid + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tid) ++ti;
    while (ti * (ti + 1) / 2 > tid) --ti;
    tj = tid - ti * (ti + 1) / 2;
  }
  if (tid < BD) sc[tid] = 1.0 / sqrt(A[pk(tid, tid)]);
  __syncthreads();
  double R[6][6];
  if (act) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q) R[r][q] = A[pks(6 * ti + r, 6 * tj + q)] * sc[6 * ti + r] * sc[6 * tj + q];
  }
  __syncthreads();
  int bad_k = -1;
  double bad_v = 0.0;
  for (int kb = 0; kb < BD / 6; ++kb) {
#pragma unroll
    for (int sub = 0; sub < 6 / W; ++sub) {
      const int co = sub * W;
      double* P = A + ((kb * (6 / W) + sub) & 1) * (W * BD);
      if (act) {
        if (tj == kb) {
#pragma unroll
          for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c < W; ++c)
              P[c * BD + 6 * ti + r] = (ti == kb && r == co + c) ? R[r][co + c] - 1.0 : R[r][co + c];
        } else if (ti == kb) {
#pragma unroll
          for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int c = 0; c < W; ++c) P[c * BD + 6 * tj + q] = R[co + c][q];
        }
      }
      __syncthreads();
      const int k0 = 6 * kb + co;
      double a[W][W], M[W][W], pivot;
#pragma unroll
      for (int c = 0; c < W; ++c)
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) a[c][c2] = P[c2 * BD + k0 + c] + (c == c2 ? 1.0 : 0.0);
      if (!small_spd_inv<W>(a, M, pivot) && bad_k < 0) {
        bad_k = k0;
        bad_v = pivot;
      }
      if (act) {
        double ci[6][W], Q[6][W];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int c = 0; c < W; ++c) ci[r][c] = P[c * BD + 6 * ti + r];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          double pj[W];
#pragma unroll
          for (int c = 0; c < W; ++c) pj[c] = P[c * BD + 6 * tj + q];
#pragma unroll
          for (int c = 0; c < W; ++c) {
            double t = 0.0;
#pragma unroll
            for (int c2 = 0; c2 < W; ++c2) t += pj[c2] * M[c2][c];
            Q[q][c] = t;
          }
        }
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int c = 0; c < W; ++c) R[r][q] -= ci[r][c] * Q[q][c];
      }
    }
  }
  if (bad_k >= 0 && tid == 0) {
    atomicOr(err, ERRB_NOT_SPD);
    diag_report(dg, source, level, index, bad_k, bad_v);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int i = 6 * ti + r, j = 6 * tj + q;
        if (i >= j) A[pk(i, j)] = ((i == j) ? 2.0 - R[r][q] : -R[r][q]) * sc[i] * sc[j];
      }
  }
  __syncthreads();
}

// Store an inverted block (LDS, packed f64) at precision P in slot d, in the
// tiled layout of the block products (writes in storage order).
// 16-bit storage keeps A_ij / (sigma_i sigma_j) with sigma_i = sqrt(A_ii).
template <int P>
__device__ __forceinline__ void store_block(const double* A, void* out, float* scale_out, int64_t d, float* sig) {
  const int tid = threadIdx.x;
  unsigned char* slot = reinterpret_cast<unsigned char*>(out) + d * BLK_STRIDE;
  constexpr bool q16 = (P == MAS_BF16 || P == MAS_F16);
  if (q16) {
    for (int i = tid; i < BD; i += blockDim.x) {
      float s = float(sqrt(A[pk(i, i)]));
      sig[i] = s;
      scale_out[d * BD + i] = s;
    }
    __syncthreads();
  }
  for (int pos = tid; pos < blk_positions(P); pos += blockDim.x) {
    int i = 0, j = 0;
    const double v = blk_entry_of(P, pos, i, j) ? A[pk(i, j)] : 0.0;
    if (P == MAS_F64) {
      reinterpret_cast<double*>(slot)[pos] = v;
    } else if (P == MAS_F32) {
      reinterpret_cast<float*>(slot)[pos] = float(v);
    } else {
      const float f = float(v / (double(sig[i]) * double(sig[j])));
      reinterpret_cast<uint16_t*>(slot)[pos] = (P == MAS_BF16) ? f32_to_bf16(f) : f32_to_f16(f);
    }
  }
}

// place a 3x3 block (pair of local nodes li, lj) into the packed lower matrix
__device__ inline void add_block_lds(double* A, int li, int lj, bool diag, const double b[3][3]) {
  if (diag) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q <= a; ++q) atomicAdd(&A[pk(3 * li + a, 3 * li + q)], b[a][q]);
  } else if (li > lj) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) atomicAdd(&A[pk(3 * li + a, 3 * lj + q)], b[a][q]);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) atomicAdd(&A[pk(3 * lj + q, 3 * li + a)], b[a][q]);
  }
}

// Sum of the 3x3 blocks of a packed symmetric block (rows of nodes >= valid
// excluded): the diagonal block of the level-(l+1) node the subdomain forms,
// since C_(l+1) = C_hat C_(l) sums node blocks (supplement Eq. (3)).
__device__ __forceinline__ void block_node_sum(const double* A, int valid, double* out9) {
  __shared__ double red[9][4];
  double s9[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) s9[q] = 0.0;
  for (int e = threadIdx.x; e < PK; e += blockDim.x) {
    int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    while (i * (i + 1) / 2 > e) --i;
    const int j = e - i * (i + 1) / 2;
    if (i / 3 >= valid || j / 3 >= valid) continue;
    const double v = A[e];
    const int a = i % 3, b = j % 3;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (q == 3 * a + b) s9[q] += v;
      if (i != j && q == 3 * b + a) s9[q] += v;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double t = wave_sum(s9[q]);
    if (lane == 0) red[q][w] = t;
  }
  __syncthreads();
  if (threadIdx.x < 9) out9[threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] +
                                           red[threadIdx.x][3];
}

// ---------------------------------------------------------------------------
// Level 0: one workgroup per subdomain d accumulates S_d H_base S_d^T in LDS
// (mass, every tet touching d, every base contact touching d) and writes it
// packed in float64 to the assembly buffer.  Tets are staged through LDS in
// batches; each work item is then one (tet, vertex pair).
__constant__ int8_t c_pair_i[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
__constant__ int8_t c_pair_j[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
constexpr int TB = 24;  // tets staged per batch

__global__ __launch_bounds__(256) void k_assemble_l0(int64_t N, const int32_t* tets, const double* mass,
                                                     const double* hf64, const int32_t* tet_off,
                                                     const int32_t* tet_list, const double* bk,
                                                     const double* bgrad, const int32_t* bidx,
                                                     const int32_t* bc_off, const int32_t* bc_list,
                                                     double* acc) {
  __shared__ double A[PK];
  __shared__ double snap[TB][EH];
  __shared__ int32_t tv[TB][4];
  const int64_t d = blockIdx.x;
  const int tid = threadIdx.x;
  for (int e = tid; e < PK; e += blockDim.x) A[e] = 0.0;
  __syncthreads();
  if (tid < BD) {
    int64_t v = SUB * d + tid / 3;
    A[pk(tid, tid)] = (v < N) ? mass[v] : 1.0;
  }
  const int t0 = tet_off[d], nt = tet_off[d + 1] - t0;
  for (int b0 = 0; b0 < nt; b0 += TB) {
    const int nb = min(TB, nt - b0);
    __syncthreads();
    for (int q = tid; q < nb * EH; q += blockDim.x) {
      const int k = q / EH, c = q % EH;
      const int64_t t = tet_list[t0 + b0 + k];
      snap[k][c] = hf64[(t / TILE) * (EH * TILE) + c * TILE + (t % TILE)];
    }
    if (tid < 4 * nb) {
      const int k = tid / 4;
      tv[k][tid % 4] = tets[4 * int64_t(tet_list[t0 + b0 + k]) + tid % 4];
    }
    __syncthreads();
    for (int w = tid; w < 10 * nb; w += blockDim.x) {
      const int k = w / 10, pr = w % 10;
      const int i = c_pair_i[pr], j = c_pair_j[pr];
      const int vi = tv[k][i], vj = tv[k][j];
      if ((vi >> 5) != d || (vj >> 5) != d) continue;
      const double* H = snap[k];
      const double* Dmi = snap[k] + 45;
      double coef[4][3];
      dfdx_coef(Dmi, coef);
      double ci[3], cj[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        ci[b] = (i == 0) ? coef[0][b] : (i == 1) ? coef[1][b] : (i == 2) ? coef[2][b] : coef[3][b];
        cj[b] = (j == 0) ? coef[0][b] : (j == 1) ? coef[1][b] : (j == 2) ? coef[2][b] : coef[3][b];
      }
      double blk[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int ap = 0; ap < 3; ++ap) {
          double sum = 0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int bp = 0; bp < 3; ++bp) sum += ci[b] * H[p9(3 * b + a, 3 * bp + ap)] * cj[bp];
          blk[a][ap] = sum;
        }
      add_block_lds(A, vi & 31, vj & 31, i == j, blk);
    }
  }
  const int c0 = bc_off[d], nc = bc_off[d + 1] - c0;
  for (int w = tid; w < 10 * nc; w += blockDim.x) {
    const int64_t ci = bc_list[c0 + w / 10];
    const int pr = w % 10;
    const int i = c_pair_i[pr], j = c_pair_j[pr];
    const int vi = bidx[4 * ci + i], vj = bidx[4 * ci + j];
    if (vi < 0 || vj < 0 || (vi >> 5) != d || (vj >> 5) != d) continue;
    const double k = bk[ci];
    const double* n = bgrad + 12 * ci;
    double blk[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) blk[a][q] = k * n[3 * i + a] * n[3 * j + q];
    add_block_lds(A, vi & 31, vj & 31, i == j, blk);
  }
  __syncthreads();
  double* out = acc + d * PK;
  for (int e = tid; e < PK; e += blockDim.x) out[e] = A[e];
}

constexpr int INV_W = 1;  // pivots per panel of the block sweep

// Inverts the packed float64 blocks of one level (rows of nodes beyond the
// node count are identity) and stores each in the requested precision, or a
// wider one when kappa = max_i M_ii B_ii exceeds guard / (20 eps): the spectral
// norm of the rounding error of a unit-diagonal 96x96 matrix is about 20 eps,
// and 1/kappa bounds its smallest eigenvalue from above.
__global__ __launch_bounds__(256) void k_invert_blocks(int64_t nodes, const double* acc, void* blk, float* scale,
                                                       uint8_t* bprec, int req, double guard, uint32_t* err,
                                                       DiagRec* dg, int level, double* ndiag_next) {
  __shared__ double A[PK];
  __shared__ double sc[BD];
  __shared__ double mdiag[BD];
  __shared__ float sig[BD];
  __shared__ int chosen;
  const int64_t d = blockIdx.x;
  const double* src = acc + d * PK;
  for (int e = threadIdx.x; e < PK; e += blockDim.x) A[e] = src[e];
  __syncthreads();
  if (threadIdx.x < BD) {
    int64_t a = SUB * d + threadIdx.x / 3;
    if (a >= nodes) A[pk(threadIdx.x, threadIdx.x)] = 1.0;
    mdiag[threadIdx.x] = A[pk(threadIdx.x, threadIdx.x)];
  }
  __syncthreads();
  if (ndiag_next) block_node_sum(A, int(min<int64_t>(SUB, nodes - SUB * d)), ndiag_next + 9 * d);
  spd_invert_lds<INV_W>(A, sc, err, dg, level == 0 ? 1 : 2, level, d);
  if (threadIdx.x < 64) {
    double k1 = mdiag[threadIdx.x] * A[pk(threadIdx.x, threadIdx.x)];
    if (threadIdx.x < BD - 64) {
      int i2 = threadIdx.x + 64;
      k1 = fmax(k1, mdiag[i2] * A[pk(i2, i2)]);
    }
    for (int o = 32; o > 0; o >>= 1) k1 = fmax(k1, __shfl_xor(k1, o));
    if (threadIdx.x == 0) {
      int p = req;
      while (guard > 0.0 && p != MAS_F64 && !(k1 <= guard / (20.0 * prec_eps(p))))
        p = (p == MAS_F32) ? MAS_F64 : MAS_F32;
      chosen = p;
      bprec[d] = uint8_t(p);
    }
  }
  __syncthreads();
  switch (chosen) {
    case MAS_F64: store_block<MAS_F64>(A, blk, scale, d, sig); break;
    case MAS_F32: store_block<MAS_F32>(A, blk, scale, d, sig); break;
    case MAS_BF16: store_block<MAS_BF16>(A, blk, scale, d, sig); break;
    default: store_block<MAS_F16>(A, blk, scale, d, sig);
  }
}

static void launch_invert(Ctx& c, int l) {
  Level& Lv = c.lv[l];
  k_invert_blocks<<<dim3(Lv.nsub), dim3(256), 0, c.s>>>(Lv.nodes, Lv.acc, Lv.blk, Lv.scale, Lv.bprec, Lv.prec,
                                                         c.cfg.prec_guard, c.err, c.diag, l,
                                                         l + 1 < c.L ? c.lv[l + 1].ndiag : nullptr);
}

mas_status launch_level0_build(Ctx& c) {
  Level& L0 = c.lv[0];
  k_assemble_l0<<<dim3(L0.nsub), dim3(256), 0, c.s>>>(c.N, c.tets, c.mass, c.hf64, c.tet_off, c.tet_list, c.bk,
                                                      c.bgrad, c.bidx, c.bc_off, c.bc_list, L0.acc);
  launch_invert(c, 0);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ---------------------------------------------------------------------------
// Coarse level l: A_(l) = C_(l) H_base C_(l)^T on the 32 nodes of each
// level-l subdomain S.  The diagonal node blocks come from the level below
// (block sums taken while inverting it).  The rest are pairs of different
// nodes of S, which only tets and base contacts with at least two nodes in S
// produce: a tet contributes chat_s^T Hf chat_u, where chat_s sums the dF/dx
// coefficients of its vertices in node s; a contact k nhat_s nhat_u^T with
// nhat_s the sum of its n_j in node s.  The items of S are split over
// `splits` workgroups that accumulate in LDS (one LDS atomic per distinct
// node pair and wavefront) and add their nonzero entries to the block.

// adds b (node pair ls > lu) to A, summed first over the lanes of the
// wavefront with the same pair while such groups are large; key < 0: nothing
// to add.  Uniform control flow.
__device__ __forceinline__ void wave_add_pair(double* A, int key, const double (&b)[3][3]) {
  const int lane = threadIdx.x & 63;
  while (true) {
    const unsigned long long act = __ballot(key >= 0);
    if (act == 0) break;
    const int leader = __ffsll(act) - 1;
    const int lk = __shfl(key, leader);
    const bool mine = key == lk;
    if (__popcll(__ballot(mine)) < 4) {  // mostly distinct pairs: add directly
      if (key >= 0) {
        const int ls = key >> 5, lu = key & 31;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int q = 0; q < 3; ++q) atomicAdd(&A[pk(3 * ls + a, 3 * lu + q)], b[a][q]);
      }
      break;
    }
    double t[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) t[a][q] = wave_sum(mine ? b[a][q] : 0.0);
    if (lane == leader) {
      const int ls = lk >> 5, lu = lk & 31;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 3; ++q) atomicAdd(&A[pk(3 * ls + a, 3 * lu + q)], t[a][q]);
    }
    if (mine) key = -1;
  }
}

// the first index j' <= j of a stencil vertex in the same node as j
__device__ __forceinline__ void node_leaders(const int (&nd)[4], int (&lead)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lead[j] = j;
#pragma unroll
    for (int i = 3; i >= 0; --i)
      if (i < j && nd[i] == nd[j]) lead[j] = i;
  }
}

__global__ __launch_bounds__(256) void k_assemble_coarse(int l, int64_t nodes, int splits, const double* ndiag,
                                                         const int32_t* tets, const double* hf64,
                                                         const int32_t* xt_off, const int32_t* xt_list,
                                                         const double* bk, const double* bgrad, const int32_t* bidx,
                                                         const int32_t* xc_off, const int32_t* xc_list,
                                                         double* acc) {
  __shared__ double A[PK];
  const int64_t S = blockIdx.x;
  const int part = blockIdx.y;
  const int tid = threadIdx.x;
  const int ns = 5 * l;
  for (int e = tid; e < PK; e += blockDim.x) A[e] = 0.0;
  __syncthreads();
  if (part == 0 && tid < SUB) {
    const int64_t a = SUB * S + tid;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = 0; y <= x; ++y)
        A[pk(3 * tid + x, 3 * tid + y)] = (a < nodes) ? ndiag[9 * a + 3 * x + y] : (x == y ? 1.0 : 0.0);
  }
  __syncthreads();
  {
    const int o = xt_off[S], n = xt_off[S + 1] - o;
    const int lo = o + int(int64_t(n) * part / splits), hi = o + int(int64_t(n) * (part + 1) / splits);
    for (int w0 = lo; w0 < hi; w0 += blockDim.x) {
      const int w = w0 + tid;
      const bool ok = w < hi;
      const int64_t t = ok ? xt_list[w] : 0;
      int nd[4], lead[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) nd[j] = ok ? (tets[4 * t + j] >> ns) : -1;
      node_leaders(nd, lead);
      double H[45], Dmi[9], coef[4][3];
      load_snapshot(hf64, t, H, Dmi);
      dfdx_coef(Dmi, coef);
      double ch[4][3];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double sum = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (lead[j] == s) sum += coef[j][b];
          ch[s][b] = sum;
        }
#pragma unroll
      for (int s = 1; s < 4; ++s)
#pragma unroll
        for (int u = 0; u < s; ++u) {
          const bool act = ok && lead[s] == s && lead[u] == u && (nd[s] >> 5) == S && (nd[u] >> 5) == S;
          const int ls = nd[s] & 31, lu = nd[u] & 31;
          const bool sw = ls < lu;  // store the pair with the larger local node first
          double b[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int ap = 0; ap < 3; ++ap) {
              double sum = 0;
#pragma unroll
              for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                for (int bp = 0; bp < 3; ++bp) sum += ch[s][bb] * H[p9(3 * bb + a, 3 * bp + ap)] * ch[u][bp];
              b[a][ap] = sum;
            }
          if (sw) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int q = 0; q < a; ++q) {
                const double x = b[a][q];
                b[a][q] = b[q][a];
                b[q][a] = x;
              }
          }
          wave_add_pair(A, act ? (sw ? (lu << 5) | ls : (ls << 5) | lu) : -1, b);
        }
    }
  }
  {
    const int o = xc_off[S], n = xc_off[S + 1] - o;
    const int lo = o + int(int64_t(n) * part / splits), hi = o + int(int64_t(n) * (part + 1) / splits);
    for (int w0 = lo; w0 < hi; w0 += blockDim.x) {
      const int w = w0 + tid;
      const bool ok = w < hi;
      const int64_t ci = ok ? xc_list[w] : 0;
      const double k = ok ? bk[ci] : 0.0;
      const double* n = bgrad + 12 * ci;
      int v[4], nd[4], lead[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = ok ? bidx[4 * ci + j] : -1;
        nd[j] = v[j] >= 0 ? (v[j] >> ns) : -1 - j;
      }
      node_leaders(nd, lead);
      double nh[4][3];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double sum = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (lead[j] == s && v[j] >= 0) sum += n[3 * j + a];
          nh[s][a] = sum;
        }
#pragma unroll
      for (int s = 1; s < 4; ++s)
#pragma unroll
        for (int u = 0; u < s; ++u) {
          const bool act = lead[s] == s && lead[u] == u && v[s] >= 0 && v[u] >= 0 && (nd[s] >> 5) == S &&
                           (nd[u] >> 5) == S;
          const int ls = nd[s] & 31, lu = nd[u] & 31;
          const bool sw = ls < lu;
          double b[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < 3; ++q) b[a][q] = sw ? k * nh[u][a] * nh[s][q] : k * nh[s][a] * nh[u][q];
          wave_add_pair(A, act ? (sw ? (lu << 5) | ls : (ls << 5) | lu) : -1, b);
        }
    }
  }
  __syncthreads();
  double* out = acc + S * PK;
  if (splits == 1) {
    for (int e = tid; e < PK; e += blockDim.x) out[e] = A[e];
  } else {
    for (int e = tid; e < PK; e += blockDim.x)
      if (A[e] != 0.0) unsafeAtomicAdd(&out[e], A[e]);
  }
}

__global__ void k_zero(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

mas_status launch_coarse_build(Ctx& c) {
  for (int l = 1; l < c.L; ++l) {
    Level& Lv = c.lv[l];
    const int sp = Lv.splits;
    if (sp > 1) k_zero<<<dim3(1024), dim3(256), 0, c.s>>>(Lv.acc, Lv.nsub * PK);
    k_assemble_coarse<<<dim3(Lv.nsub, sp), dim3(256), 0, c.s>>>(l, Lv.nodes, sp, Lv.ndiag, c.tets, c.hf64,
                                                                Lv.xt_off, Lv.xt_list, c.bk, c.bgrad, c.bidx,
                                                                Lv.xc_off, Lv.xc_list, Lv.acc);
    launch_invert(c, l);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
