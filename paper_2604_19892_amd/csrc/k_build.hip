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
    snh_tangent(F, g[10], g[11], H);
    psd_project9(H);
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
  return bucket_by_subdomain(c, m, c.bidx, c.bk, c.bgrad, c.bc_cnt, c.bc_off, c.bc_list);
}

// ---------------------------------------------------------------------------
// In-place inverse of an SPD 96x96 matrix held packed-lower in LDS, using the
// symmetric sweep operator (Goodnight 1979): sweeping every pivot k maps A to
// -A^-1.  The matrix lives in registers during the sweeps: thread t < 136
// owns the 6x6 tile (ti, tj), ti >= tj, of a 16x16 tile grid; per pivot only
// the pivot column passes through LDS (double-buffered, one barrier a step).
__device__ void spd_invert_lds(double* A, double (*colbuf)[BD], uint32_t* err) {
  const int tid = threadIdx.x;
  const bool act = tid < 136;
  int ti = 0, tj = 0;
  if (act) {
    ti = int((sqrt(8.0 * tid + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tid) ++ti;
    while (ti * (ti + 1) / 2 > tid) --ti;
    tj = tid - ti * (ti + 1) / 2;
  }
  double R[6][6];
  if (act) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q) R[r][q] = A[pks(6 * ti + r, 6 * tj + q)];
  }
  bool bad = false;
  for (int k = 0; k < BD; ++k) {
    double* col = colbuf[k & 1];
    const int kb = k / 6, kr = k % 6;
    if (act) {
      if (tj == kb) {
#pragma unroll
        for (int r = 0; r < 6; ++r)
          if (6 * ti + r >= k) col[6 * ti + r] = R[r][kr];
      }
      if (ti == kb) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (6 * tj + q < k) col[6 * tj + q] = R[kr][q];
      }
    }
    __syncthreads();
    const double dk = col[k];
    bad |= !(dk > 0.0) || !isfinite(dk);
    const double inv = 1.0 / dk;
    if (act) {
      double ci[6], cj[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) ci[r] = col[6 * ti + r];
#pragma unroll
      for (int q = 0; q < 6; ++q) cj[q] = col[6 * tj + q] * inv;
      if (ti != kb && tj != kb) {
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int q = 0; q < 6; ++q) R[r][q] -= ci[r] * cj[q];
      } else {
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const int i = 6 * ti + r, j = 6 * tj + q;
            if (i == k && j == k) R[r][q] = -inv;
            else if (i == k) R[r][q] = cj[q];
            else if (j == k) R[r][q] = ci[r] * inv;
            else R[r][q] -= ci[r] * cj[q];
          }
      }
    }
  }
  if (bad && tid == 0) atomicOr(err, ERRB_NOT_SPD);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int i = 6 * ti + r, j = 6 * tj + q;
        if (i >= j) A[pk(i, j)] = -R[r][q];
      }
  }
  __syncthreads();
}

// Store an inverted block (LDS, packed f64) at the requested precision.
// 16-bit storage keeps A_ij / (sigma_i sigma_j) with sigma_i = sqrt(A_ii).
template <int P>
__device__ void store_block(const double* A, void* out, float* scale_out, int64_t d, float* sig) {
  const int tid = threadIdx.x;
  const size_t stride = blk_elems(P);
  if (P == MAS_F64) {
    double* o = reinterpret_cast<double*>(out) + d * stride;
    for (int e = tid; e < PK; e += blockDim.x) o[e] = A[e];
  } else if (P == MAS_F32) {
    float* o = reinterpret_cast<float*>(out) + d * stride;
    for (int e = tid; e < PK; e += blockDim.x) o[e] = float(A[e]);
  } else {
    for (int i = tid; i < BD; i += blockDim.x) {
      float s = float(sqrt(A[pk(i, i)]));
      sig[i] = s;
      scale_out[d * BD + i] = s;
    }
    __syncthreads();
    uint16_t* o = reinterpret_cast<uint16_t*>(out) + d * stride;
    for (int e = tid; e < PK; e += blockDim.x) {
      int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      while (i * (i + 1) / 2 > e) --i;
      int j = e - i * (i + 1) / 2;
      float v = float(A[e] / (double(sig[i]) * double(sig[j])));
      o[e] = (P == MAS_BF16) ? f32_to_bf16(v) : f32_to_f16(v);
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

__device__ inline void add_block_global(double* A, int li, int lj, bool diag, const double b[3][3]) {
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

// ---------------------------------------------------------------------------
// Level 0: one workgroup per subdomain d assembles S_d H_base S_d^T in LDS
// (mass, every tet touching d, every base contact touching d), inverts it and
// stores it.  Rows of vertices beyond N are identity.
template <int P>
__global__ __launch_bounds__(256) void k_build_l0(int64_t N, const int32_t* tets, const double* mass,
                                                  const double* hf64, const int32_t* tet_off,
                                                  const int32_t* tet_list, const double* bk,
                                                  const double* bgrad, const int32_t* bidx,
                                                  const int32_t* bc_off, const int32_t* bc_list,
                                                  void* blk, float* scale, uint32_t* err) {
  __shared__ double A[PK];
  __shared__ double colbuf[2][BD];
  __shared__ float sig[BD];
  const int64_t d = blockIdx.x;
  const int tid = threadIdx.x;
  for (int e = tid; e < PK; e += blockDim.x) A[e] = 0.0;
  __syncthreads();
  if (tid < BD) {
    int64_t v = SUB * d + tid / 3;
    A[pk(tid, tid)] = (v < N) ? mass[v] : 1.0;
  }
  __syncthreads();
  for (int e = tet_off[d] + tid; e < tet_off[d + 1]; e += blockDim.x) {
    int64_t t = tet_list[e];
    int v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = tets[4 * t + j];
    double H[45], Dmi[9], coef[4][3];
    load_snapshot(hf64, t, H, Dmi);
    dfdx_coef(Dmi, coef);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        if ((v[i] >> 5) != d || (v[j] >> 5) != d) continue;
        double b[3][3];
        elem_block(H, coef, i, j, b);
        add_block_lds(A, v[i] & 31, v[j] & 31, i == j, b);
      }
  }
  for (int e = bc_off[d] + tid; e < bc_off[d + 1]; e += blockDim.x) {
    int64_t ci = bc_list[e];
    double k = bk[ci];
    const double* n = bgrad + 12 * ci;
    int v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = bidx[4 * ci + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        if (v[i] < 0 || v[j] < 0 || (v[i] >> 5) != d || (v[j] >> 5) != d) continue;
        double b[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int q = 0; q < 3; ++q) b[a][q] = k * n[3 * i + a] * n[3 * j + q];
        add_block_lds(A, v[i] & 31, v[j] & 31, i == j, b);
      }
  }
  __syncthreads();
  spd_invert_lds(A, colbuf, err);
  store_block<P>(A, blk, scale, d, sig);
}

mas_status launch_level0_build(Ctx& c) {
  Level& L0 = c.lv[0];
  dim3 g(L0.nsub), b(256);
  switch (L0.prec) {
    case MAS_F64:
      k_build_l0<MAS_F64><<<g, b, 0, c.s>>>(c.N, c.tets, c.mass, c.hf64, c.tet_off, c.tet_list, c.bk,
                                            c.bgrad, c.bidx, c.bc_off, c.bc_list, L0.blk, L0.scale, c.err);
      break;
    case MAS_F32:
      k_build_l0<MAS_F32><<<g, b, 0, c.s>>>(c.N, c.tets, c.mass, c.hf64, c.tet_off, c.tet_list, c.bk,
                                            c.bgrad, c.bidx, c.bc_off, c.bc_list, L0.blk, L0.scale, c.err);
      break;
    case MAS_BF16:
      k_build_l0<MAS_BF16><<<g, b, 0, c.s>>>(c.N, c.tets, c.mass, c.hf64, c.tet_off, c.tet_list, c.bk,
                                             c.bgrad, c.bidx, c.bc_off, c.bc_list, L0.blk, L0.scale, c.err);
      break;
    default:
      k_build_l0<MAS_F16><<<g, b, 0, c.s>>>(c.N, c.tets, c.mass, c.hf64, c.tet_off, c.tet_list, c.bk,
                                            c.bgrad, c.bidx, c.bc_off, c.bc_list, L0.blk, L0.scale, c.err);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ---------------------------------------------------------------------------
// Coarse levels.  A_(l) = C_(l) H_base C_(l)^T: a term S_e^T H_e S_e restricted
// to level-l nodes sums the coefficients of vertices that share a node, so
// the element contributes  chat_s^T Hf chat_t  per node pair (s, t), where
// chat_s = sum of dF/dx coefficients of its vertices in node s.  Elements whose
// vertices all share one node contribute nothing (translations are in the
// kernel of H_e); the same holds for contacts through nhat_s = sum of n_j.

struct CoarseArgs {
  int L;                    // number of levels
  double* acc[MAXL];        // packed f64 accumulation per level (index 1..L-1)
};

__global__ void k_coarse_tets(int64_t T, const int32_t* tets, const double* hf64, CoarseArgs ca) {
  int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= T) return;
  int v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = tets[4 * t + j];
  bool loaded = false;
  double H[45], Dmi[9], coef[4][3];
  for (int l = 1; l < ca.L; ++l) {
    int nd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) nd[j] = v[j] >> (5 * l);
    if (nd[0] == nd[1] && nd[0] == nd[2] && nd[0] == nd[3]) continue;
    if (!loaded) {
      load_snapshot(hf64, t, H, Dmi);
      dfdx_coef(Dmi, coef);
      loaded = true;
    }
    int lead[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      lead[j] = j;
#pragma unroll
      for (int i = 3; i >= 0; --i)
        if (i < j && nd[i] == nd[j]) lead[j] = i;
    }
    double ch[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double acc = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (lead[j] == s) acc += coef[j][b];
        ch[s][b] = acc;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u <= s; ++u) {
        if (lead[s] != s || lead[u] != u) continue;
        int a_s = nd[s], a_u = nd[u];
        if ((a_s >> 5) != (a_u >> 5)) continue;
        double b[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int ap = 0; ap < 3; ++ap) {
            double acc = 0;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
#pragma unroll
              for (int bp = 0; bp < 3; ++bp) acc += ch[s][bb] * H[p9(3 * bb + a, 3 * bp + ap)] * ch[u][bp];
            b[a][ap] = acc;
          }
        double* A = ca.acc[l] + int64_t(a_s >> 5) * PK;
        add_block_global(A, a_s & 31, a_u & 31, s == u, b);
      }
  }
}

__global__ void k_coarse_contacts(int64_t m, const double* bk, const double* bgrad, const int32_t* bidx,
                                  CoarseArgs ca) {
  int64_t ci = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (ci >= m) return;
  double k = bk[ci];
  if (!(k > 0.0)) return;
  int v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = bidx[4 * ci + j];
  const double* n = bgrad + 12 * ci;
  for (int l = 1; l < ca.L; ++l) {
    int nd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) nd[j] = v[j] >= 0 ? (v[j] >> (5 * l)) : -1 - j;
    int lead[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      lead[j] = j;
#pragma unroll
      for (int i = 3; i >= 0; --i)
        if (i < j && nd[i] == nd[j]) lead[j] = i;
    }
    double nh[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double acc = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (lead[j] == s && v[j] >= 0) acc += n[3 * j + a];
        nh[s][a] = acc;
      }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u <= s; ++u) {
        if (lead[s] != s || lead[u] != u || v[s] < 0 || v[u] < 0) continue;
        int a_s = nd[s], a_u = nd[u];
        if ((a_s >> 5) != (a_u >> 5)) continue;
        double b[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int q = 0; q < 3; ++q) b[a][q] = k * nh[s][a] * nh[u][q];
        double* A = ca.acc[l] + int64_t(a_s >> 5) * PK;
        add_block_global(A, a_s & 31, a_u & 31, s == u, b);
      }
  }
}

// node masses of level l from level l-1 (or vertex) masses; adds them to the
// diagonal of the level-l accumulation
__global__ void k_coarse_mass(int64_t nodes, int64_t child_n, const double* child_mass,
                              double* node_mass, double* acc) {
  int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (a >= nodes) return;
  double s = 0;
  for (int64_t q = SUB * a; q < SUB * a + SUB && q < child_n; ++q) s += child_mass[q];
  node_mass[a] = s;
  double* A = acc + (a >> 5) * PK;
  int la = int(a & 31);
#pragma unroll
  for (int c3 = 0; c3 < 3; ++c3) A[pk(3 * la + c3, 3 * la + c3)] += s;
}

template <int P>
__global__ __launch_bounds__(256) void k_coarse_invert(int64_t nodes, const double* acc, void* blk,
                                                       uint32_t* err) {
  __shared__ double A[PK];
  __shared__ double colbuf[2][BD];
  __shared__ float sig[BD];
  const int64_t d = blockIdx.x;
  const double* src = acc + d * PK;
  for (int e = threadIdx.x; e < PK; e += blockDim.x) A[e] = src[e];
  __syncthreads();
  if (threadIdx.x < BD) {
    int64_t a = SUB * d + threadIdx.x / 3;
    if (a >= nodes) A[pk(threadIdx.x, threadIdx.x)] = 1.0;
  }
  __syncthreads();
  spd_invert_lds(A, colbuf, err);
  store_block<P>(A, blk, nullptr, d, sig);
}

mas_status launch_coarse_build(Ctx& c) {
  if (c.L < 2) return MAS_OK;
  CoarseArgs ca{};
  ca.L = c.L;
  for (int l = 1; l < c.L; ++l) {
    ca.acc[l] = c.lv[l].acc;
    HIPCHK(hipMemsetAsync(c.lv[l].acc, 0, sizeof(double) * PK * c.lv[l].nsub, c.s));
  }
  // masses: level-1 nodes from vertices, then upward; r buffers hold node masses
  const double* child = c.mass;
  int64_t child_n = c.N;
  for (int l = 1; l < c.L; ++l) {
    int64_t nodes = c.lv[l].nodes;
    k_coarse_mass<<<dim3((nodes + 255) / 256), dim3(256), 0, c.s>>>(nodes, child_n, child, c.lv[l].r,
                                                                   c.lv[l].acc);
    child = c.lv[l].r;
    child_n = nodes;
  }
  k_coarse_tets<<<dim3((c.T + 255) / 256), dim3(256), 0, c.s>>>(c.T, c.tets, c.hf64, ca);
  if (c.mb > 0)
    k_coarse_contacts<<<dim3((c.mb + 255) / 256), dim3(256), 0, c.s>>>(c.mb, c.bk, c.bgrad, c.bidx, ca);
  for (int l = 1; l < c.L; ++l) {
    Level& Lv = c.lv[l];
    if (Lv.prec == MAS_F64)
      k_coarse_invert<MAS_F64><<<dim3(Lv.nsub), dim3(256), 0, c.s>>>(Lv.nodes, Lv.acc, Lv.blk, c.err);
    else
      k_coarse_invert<MAS_F32><<<dim3(Lv.nsub), dim3(256), 0, c.s>>>(Lv.nodes, Lv.acc, Lv.blk, c.err);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
