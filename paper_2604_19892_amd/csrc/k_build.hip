// RebuildMAS: the frozen element Hessians, the base contact set, level-0
// subdomain blocks (assembled and inverted inside one workgroup) and the
// Galerkin coarse blocks of every level.
#include <algorithm>

#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

// ---------------------------------------------------------------------------
// Element snapshots: per tet the 9x9 tangent of h^2 V Psi with its negative
// eigenvalues clamped, packed (45), followed by Dm^-1 (9), in the chunked
// tile layout of snap_load.  One thread per range entry: it writes the
// entry's copy (float32 or float64), read by the Hessian-vector product and,
// on the tet's home entry, by the block assembly.
__global__ __launch_bounds__(64) void k_elem_hess(int64_t nent, int64_t nent_pad, const int32_t* rl_t,
                                                  const int32_t* rl_tv, const double* rl_geo, const double* x,
                                                  double h, double* hr64, float* hr32) {
  const int64_t w = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (w >= nent_pad) return;
  double e[EH];
#pragma unroll
  for (int q = 0; q < EH; ++q) e[q] = 0.0;
  if (w < nent) {
    const int4 tv = reinterpret_cast<const int4*>(rl_tv)[w];
    const int v[4] = {tv.x, tv.y, tv.z, tv.w};
    double xe[12];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) xe[3 * j + a] = x[3 * v[j] + a];
    double g[12];
    geo_load(rl_geo, w, g);
    double F[3][3];
    def_grad(xe, g, F);
    double H[45];
    snh_tangent_psd(F, g[10], g[11], H);
    const double s = h * h * g[9];
#pragma unroll
    for (int q = 0; q < 45; ++q) e[q] = H[q] * s;
#pragma unroll
    for (int q = 0; q < 9; ++q) e[45 + q] = g[q];
  }
  if (hr32) {
    float4* p32 = reinterpret_cast<float4*>(hr32) + (w / TILE) * (SNAP_NC32 * TILE) + (w % TILE);
#pragma unroll
    for (int c = 0; c < SNAP_NC32; ++c) {
      float vv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) vv[k] = (4 * c + k < EH) ? float(e[4 * c + k]) : 0.0f;
      st_once(p32 + c * TILE, make_float4(vv[0], vv[1], vv[2], vv[3]));
    }
  } else {
    double2* p64 = reinterpret_cast<double2*>(hr64) + (w / TILE) * (SNAP_NC64 * TILE) + (w % TILE);
#pragma unroll
    for (int c = 0; c < SNAP_NC64; ++c) st_once(p64 + c * TILE, make_double2(e[2 * c], e[2 * c + 1]));
  }
}

mas_status launch_elem_hessians(Ctx& c, const double* x_base) {
  k_elem_hess<<<dim3(c.nent_pad / TILE), dim3(TILE), 0, c.s>>>(c.nent, c.nent_pad, c.rl_t, c.rl_tv, c.rl_geo,
                                                               x_base, c.cfg.h, c.hr64, c.hr32);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ---------------------------------------------------------------------------
// Base contact set: copy, stiffness k = kappa b''(d) and columns sqrt(k) n.
// Each wavefront takes 64 stencils; the 12-wide rows are copied by the whole
// wavefront in 64-element strides so that every store is contiguous.
__global__ __launch_bounds__(256) void k_base_copy(int64_t m, const uint64_t* key, const int32_t* idx,
                                                   const double* d, const double* grad, double kappa, double dhat,
                                                   uint64_t* bkey, double* bk, uint8_t* bpm, double* bgrad,
                                                   int32_t* bidx, double* bu, uint32_t* err) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t w0 = i - lane;  // first stencil of this wavefront
  double sk = 0.0;
  if (i < m) {
    double b, b1, b2;
    const double di = d[i];
    if (!isfinite(di)) atomicOr(err, ERRB_NONFINITE);
    barrier3(di, dhat, &b, &b1, &b2);
    const double k = kappa * b2;
    bk[i] = k;
    bkey[i] = key[i];
    sk = sqrt(k);
#pragma unroll
    for (int q = 0; q < 4; ++q) bidx[4 * i + q] = idx[4 * i + q];
  }
  // part masks (part_mask) of the wavefront's stencils, gathered from the
  // copy below: entry e is vertex (e mod 12) / 3 of stencil e / 12
  __shared__ uint32_t pmw[256];
  uint32_t* pw = pmw + (threadIdx.x & ~63);
  pw[lane] = 0u;
  wave_sync();
  const int64_t n12 = 12 * (min<int64_t>(m, w0 + 64) - w0);
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int e = q * 64 + lane;
    const double s = __shfl(sk, e / 12);
    if (e < n12) {
      const double n = grad[12 * w0 + e];
      bgrad[12 * w0 + e] = n;
      bu[12 * w0 + e] = s * n;
      if (n != 0.0) atomicOr(&pw[e / 12], 1u << ((e % 12) / 3));
    }
  }
  wave_sync();
  if (i < m) bpm[i] = sk > 0.0 ? uint8_t(pw[lane]) : uint8_t(0);
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Inserts the keys of the base contacts with k > 0 into the table (it has at
// least twice as many slots as keys, so every probe sequence meets a free
// slot).  A base contact with k = 0 classifies a current one exactly as
// absence does (dS = k either way), so it is left out.  A key already
// present keeps its first entry.
__global__ void k_hash_insert(int64_t m, const uint64_t* key, const double* bk, uint64_t* hkey, int32_t* hval,
                              int64_t mask) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= m || !(bk[i] > 0.0)) return;
  const uint64_t k = key[i];
  int64_t h = int64_t(key_hash(k) & uint64_t(mask));
  while (true) {
    const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(hkey + h),
                                              (unsigned long long)HKEY_EMPTY, (unsigned long long)k);
    if (prev == HKEY_EMPTY) {
      hval[h] = int32_t(i);
      return;
    }
    if (prev == k) return;
    h = (h + 1) & mask;
  }
}

mas_status launch_base_contacts(Ctx& c, const mas_contacts* b) {
  int64_t m = b ? b->m : 0;
  if (m > c.mb_cap) return MAS_ERR_INVALID_ARG;  // checked by mas_build before any launch
  c.mb = m;
  // the part of the key table in use: a power of two of at least twice the
  // base contacts (the table was allocated for max_contacts)
  c.hsize = 1024;
  while (c.hsize < 2 * m) c.hsize *= 2;
  mas_status st = MAS_OK;
  if (m > 0) {
    int bs = 256;
    k_base_copy<<<dim3((m + bs - 1) / bs), dim3(bs), 0, c.s>>>(
        m, b->key, b->idx, b->d, b->grad, c.cfg.kappa, c.cfg.dhat, c.bkey, c.bk, c.bpm, c.bgrad,
        c.bidx, c.bu, c.err);
    k_fill_u64<<<dim3(std::min<int64_t>(1024, (c.hsize + 255) / 256)), dim3(256), 0, c.s>>>(c.hkey, c.hsize,
                                                                                             HKEY_EMPTY);
    k_hash_insert<<<dim3((m + 255) / 256), dim3(256), 0, c.s>>>(m, c.bkey, c.bk, c.hkey, c.hval, c.hsize - 1);
    HIPCHK(hipGetLastError());
  }
  st = bucket_by_subdomain(c, m, c.bidx, c.bpm, c.bc_cnt, c.bc_off, c.bc_list);
  if (st != MAS_OK) return st;
  return bucket_stencils(c, 1, c.vrange, c.nrange, m, c.bidx, c.bpm, c.rc_cnt, c.rc_off, c.rc_list);
}

// ---------------------------------------------------------------------------

// place a 3x3 block (pair of local nodes li, lj) into the packed lower matrix
template <bool DET>
__device__ inline void add_block_lds(double* A, int* Acnt, int pass, int li, int lj, bool diag,
                                     const double b[3][3]) {
  if (diag) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q <= a; ++q) acc_term<DET>(A, Acnt, pk(3 * li + a, 3 * li + q), b[a][q], pass);
  } else if (li > lj) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc_term<DET>(A, Acnt, pk(3 * li + a, 3 * lj + q), b[a][q], pass);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc_term<DET>(A, Acnt, pk(3 * lj + q, 3 * li + a), b[a][q], pass);
  }
}

// ---------------------------------------------------------------------------
// Level 0 and the coupling blocks of the coarse levels.  One workgroup per
// level-0 subdomain d accumulates S_d H_base S_d^T in LDS (mass, every tet
// and base contact touching d) and writes it packed in float64 to the level-0
// assembly buffer.  The same pass yields the off-diagonal node blocks of
// every coarse level A_(l) = C_(l) H C_(l)^T (supplement Eq. (3)): a vertex
// pair (a in d, b outside d) adds H_ab to exactly one of them, at the level l
// where a and b first share a subdomain, node pair (a >> 5l, b >> 5l); the
// workgroup of the larger node takes it (the lower block).  Level 1's node is
// d itself, so its row of blocks is complete here and written directly;
// deeper levels are summed per workgroup in LDS and added with atomics.  The
// diagonal node blocks come later: level 1's from the block sums taken while
// level 0 is inverted, deeper ones from k_node_sums.  One thread per tet (or contact): it forms
// G_j = Hf (c_j x I) once per vertex j and the 3x3 blocks c_i^T G_j of the
// pairs it has to deliver.
struct L0Args {
  int64_t N;
  int L;
  const double* mass;
  const float* h32;       // entry snapshots (one of the two is set)
  const double* h64;
  const int32_t* tet_off;  // subdomain -> its tet records
  const int32_t* l0_tv;    // per record: the tet's four vertices
  const int32_t* l0_home;  // per record: the entry holding the tet's home snapshot
  const double* bk;
  const double* bgrad;
  const int32_t* bidx;
  const int32_t* bc_off;
  const int32_t* bc_list;
  double* acc[MAXL];
  double* coup;  // deterministic mode: deep-level coupling tables per subdomain
};

// Where the pair (vi, vj) of a stencil touching subdomain d goes: 0 = level 0
// block, l >= 1 = coupling table of level l (node of the outside vertex in
// *nb, *flip if vj is the vertex in d), -1 = nowhere.
__device__ __forceinline__ int route_pair(int64_t d, int L, int vi, int vj, int* nb, bool* flip) {
  const bool in_i = (vi >> 5) == d, in_j = (vj >> 5) == d;
  if (in_i && in_j) return 0;
  if (in_i == in_j) return -1;
  const int a = in_i ? vi : vj, b = in_i ? vj : vi;
  *flip = !in_i;
  for (int l = 1; l < L; ++l) {
    if ((a >> (5 * (l + 1))) == (b >> (5 * (l + 1)))) {
      if ((a >> (5 * l)) < (b >> (5 * l))) return -1;
      *nb = (b >> (5 * l)) & 31;
      return l;
    }
  }
  return -1;
}

template <bool DET>
__device__ __forceinline__ void add_coupling(double* T, int* Tcnt, int pass, int l, int nb, bool flip,
                                             const double (&b)[3][3]) {
  const int e = ((l - 1) * SUB + nb) * 9;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) acc_term<DET>(T, Tcnt, e + 3 * x + y, flip ? b[y][x] : b[x][y], pass);
}

constexpr int L0_THREADS = 128;

// DET: the sums of A and of the coupling tables are taken with the two-pass
// fixed-point accumulation (so that they do not depend on the order of the
// LDS atomics), and the deep-level tables go to a.coup, to be summed over
// the subdomains in ascending order by k_coup_reduce.
template <typename TH, bool DET>
__global__ __launch_bounds__(L0_THREADS) void k_assemble_l0(L0Args a) {
  __shared__ __align__(16) double A[PK];
  extern __shared__ double T[];  // (L - 1) x 32 node blocks of 9; DET: then the counts of A and T
  const int64_t d = xcd_block(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int nT = (a.L - 1) * SUB * 9;
  int* Acnt = DET ? reinterpret_cast<int*>(T + nT) : nullptr;
  int* Tcnt = DET ? Acnt + PK : nullptr;
  for (int e = tid; e < PK; e += blockDim.x) A[e] = 0.0;
  for (int e = tid; e < nT; e += blockDim.x) T[e] = 0.0;
  if (DET) {
    for (int e = tid; e < PK; e += blockDim.x) Acnt[e] = 0;
    for (int e = tid; e < nT; e += blockDim.x) Tcnt[e] = 0;
  }
  __syncthreads();
  for (int pass = DET ? 0 : 1; pass < 2; ++pass) {
  // the lumped mass (identity on padded rows) goes in before any tet or
  // stencil adds to the diagonal
  if (tid < BD) {
    int64_t v = SUB * d + tid / 3;
    const double mv = (v < a.N) ? a.mass[v] : 1.0;
    if (DET) acc_term<DET>(A, Acnt, pk(tid, tid), mv, pass);
    else A[pk(tid, tid)] = mv;
  }
  __syncthreads();
  const int t0 = a.tet_off[d], t1 = a.tet_off[d + 1];
  for (int w = t0 + tid; w < t1; w += blockDim.x) {
    const int4 tv = reinterpret_cast<const int4*>(a.l0_tv)[w];
    const int v[4] = {tv.x, tv.y, tv.z, tv.w};
    int dest[4][4], nbr[4][4];
    bool flip[4][4], need[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      need[j] = false;
#pragma unroll
      for (int i = j; i < 4; ++i) {
        nbr[i][j] = 0;
        flip[i][j] = false;
        dest[i][j] = route_pair(d, a.L, v[i], v[j], &nbr[i][j], &flip[i][j]);
        need[j] |= dest[i][j] >= 0;
      }
    }
    if (!(need[0] || need[1] || need[2] || need[3])) continue;
    constexpr int NH = sizeof(TH) == 8 ? EH : 4 * SNAP_NC32;
    TH H[NH];
    if constexpr (sizeof(TH) == 8) snap_load<false>(a.h64, a.l0_home[w], H);
    else snap_load<false>(a.h32, a.l0_home[w], H);
    double coef[4][3];
    {
      double dm[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) dm[q] = double(H[45 + q]);
      dfdx_coef(dm, coef);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!need[j]) continue;
      double G[9][3];  // G[3b + x][y] = sum_b' Hf(3b + x, 3b' + y) c_j[b']
#pragma unroll
      for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int y = 0; y < 3; ++y)
          G[r][y] = double(H[p9(r, y)]) * coef[j][0] + double(H[p9(r, 3 + y)]) * coef[j][1] +
                    double(H[p9(r, 6 + y)]) * coef[j][2];
#pragma unroll
      for (int i = j; i < 4; ++i) {
        if (dest[i][j] < 0) continue;
        double blk[3][3];
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y)
            blk[x][y] = coef[i][0] * G[x][y] + coef[i][1] * G[3 + x][y] + coef[i][2] * G[6 + x][y];
        if (dest[i][j] == 0) add_block_lds<DET>(A, Acnt, pass, v[i] & 31, v[j] & 31, i == j, blk);
        else add_coupling<DET>(T, Tcnt, pass, dest[i][j], nbr[i][j], flip[i][j], blk);
      }
    }
  }
  const int c0 = a.bc_off[d], c1 = a.bc_off[d + 1];
  for (int w = c0 + tid; w < c1; w += blockDim.x) {
    const int64_t ci = a.bc_list[w];
    int v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = a.bidx[4 * ci + j];
    const double k = a.bk[ci];
    const double* n = a.bgrad + 12 * ci;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (v[j] < 0) continue;
#pragma unroll
      for (int i = j; i < 4; ++i) {
        if (v[i] < 0) continue;
        int nbr = 0;
        bool flip = false;
        const int dest = route_pair(d, a.L, v[i], v[j], &nbr, &flip);
        if (dest < 0) continue;
        double blk[3][3];
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) blk[x][y] = k * n[3 * i + x] * n[3 * j + y];
        if (dest == 0) add_block_lds<DET>(A, Acnt, pass, v[i] & 31, v[j] & 31, i == j, blk);
        else add_coupling<DET>(T, Tcnt, pass, dest, nbr, flip, blk);
      }
    }
  }
  __syncthreads();
  if (DET) {
    if (pass == 0) {
      for (int e = tid; e < PK; e += blockDim.x) fx_mid(&A[e], &Acnt[e]);
      for (int e = tid; e < nT; e += blockDim.x) fx_mid(&T[e], &Tcnt[e]);
    } else {
      for (int e = tid; e < PK; e += blockDim.x) A[e] = fx_get(&A[e], &Acnt[e]);
      for (int e = tid; e < nT; e += blockDim.x) T[e] = fx_get(&T[e], &Tcnt[e]);
    }
    __syncthreads();
  }
  }  // passes
  {
    // 16-byte stores (PK is even, every block starts on 16 bytes), not
    // kept in the caches: the inversion reads each block once
    const double2* src2 = reinterpret_cast<const double2*>(A);
    double2* out2 = reinterpret_cast<double2*>(a.acc[0] + d * PK);
    for (int e = tid; e < PK / 2; e += blockDim.x) st_once(out2 + e, src2[e]);
  }
  if (DET && a.L > 2) {
    // the deep-level tables of this subdomain, zeros included
    double* cp = a.coup + d * int64_t(nT - SUB * 9);
    for (int q = SUB * 9 + tid; q < nT; q += blockDim.x) cp[q - SUB * 9] = T[q];
  }
  if (a.L > 1) {
    // level 1: the blocks (d, u), u < d, of row d of subdomain d >> 5
    const int ld = int(d & 31);
    double* o1 = a.acc[1] + (d >> 5) * PK;
    for (int q = tid; q < 9 * ld; q += blockDim.x) {
      const int u = q / 9, x = (q % 9) / 3, y = q % 3;
      o1[pk(3 * ld + x, 3 * u + y)] = T[u * 9 + 3 * x + y];
    }
    // deeper levels: only the tables this subdomain touched
    for (int q = SUB * 9 + tid; !DET && q < nT; q += blockDim.x) {
      const double val = T[q];
      if (val == 0.0) continue;
      const int l = q / (SUB * 9) + 1, u = (q / 9) % SUB, x = (q % 9) / 3, y = q % 3;
      const int na = int((d >> (5 * (l - 1))) & 31);
      unsafeAtomicAdd(&a.acc[l][(d >> (5 * l)) * PK + pk(3 * na + x, 3 * u + y)], val);
    }
  }
}

// Level l >= 2: the diagonal node block of node s (subdomain s of level
// l - 1) is the sum of all 3x3 node blocks of that subdomain's block, both
// triangles, rows of real nodes only (C_(l) sums the nodes of s).  One
// workgroup per subdomain reads the packed block (entry e = tid + 256 k is
// (i, j), tracked from one to the next) and keeps the sum
// as W + W^T: entry (i, j < i) adds to W[3 (i mod 3) + j mod 3], a diagonal
// entry half of itself.
constexpr int NS_T = 256;
__global__ __launch_bounds__(NS_T) void k_node_sums(int64_t nodes_prev, const double* acc_prev, double* acc_l) {
  __shared__ double red[NS_T / 64][9];
  const int64_t s = blockIdx.x;
  const int tid = threadIdx.x;
  const int nv = 3 * int(min<int64_t>(SUB, nodes_prev - SUB * s));
  const double* A = acc_prev + s * PK;
  double W[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) W[t] = 0.0;
  // every load first (they are independent), then the bins
  constexpr int NE = (PK + NS_T - 1) / NS_T;
  double vals[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) vals[k] = tid + NS_T * k < PK ? A[tid + NS_T * k] : 0.0;
  int i = 0, j = tid;
  while (j > i) j -= ++i;
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    if (i < nv) {
      const double val = vals[k];
      const int k9 = 3 * (i % 3) + j % 3;
      const double wv = j == i ? 0.5 * val : val;
#pragma unroll
      for (int t = 0; t < 9; ++t)
        if (k9 == t) W[t] += wv;
    }
    j += NS_T;
    while (j > i && i < BD) j -= ++i;
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const double v = wave_sum(W[t]);
    if ((tid & 63) == 0) red[tid >> 6][t] = v;
  }
  __syncthreads();
  if (tid < 9 && tid / 3 >= tid % 3) {
    const int x = tid / 3, y = tid % 3;
    double sum = 0.0;
    for (int w = 0; w < NS_T / 64; ++w) sum += red[w][3 * x + y] + red[w][3 * y + x];
    const int ln = int(s & 31);
    acc_l[(s >> 5) * PK + pk(3 * ln + x, 3 * ln + y)] = sum;
  }
}

__global__ void k_zero(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// Deterministic mode: the coupling blocks of level l >= 2 summed over the
// level-0 subdomains in ascending order.  Row node na of level-l subdomain
// P is the level-(l-1) subdomain s = 32 P + na, whose level-0 subdomains
// d in [s 32^(l-1), (s + 1) 32^(l-1)) each wrote their table for it; only
// the blocks (na, u < na) of the lower triangle exist.
__global__ void k_coup_reduce(int l, int L, int64_t D0, int64_t nsub_prev, const double* coup, double* acc_l) {
  const int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t s = q / (SUB * 9);
  if (s >= nsub_prev) return;
  const int r = int(q % (SUB * 9));
  const int u = r / 9, x = (r % 9) / 3, y = r % 3;
  const int na = int(s & 31);
  if (u >= na) return;
  const int sh = 5 * (l - 1);
  const int64_t d0 = s << sh, d1 = min<int64_t>(D0, (s + 1) << sh);
  const int64_t stride = int64_t(L - 2) * SUB * 9;
  double sum = 0.0;
  for (int64_t dd = d0; dd < d1; ++dd) sum += coup[dd * stride + (l - 2) * SUB * 9 + r];
  acc_l[(s >> 5) * PK + pk(3 * na + x, 3 * u + y)] = sum;
}

mas_status launch_level0_build(Ctx& c) {
  Level& L0 = c.lv[0];
  for (int l = 2; l < c.L; ++l) k_zero<<<dim3(256), dim3(256), 0, c.s>>>(c.lv[l].acc, c.lv[l].nsub * PK);
  L0Args a{};
  a.N = c.N;
  a.L = c.L;
  a.mass = c.mass;
  a.h32 = c.hr32;
  a.h64 = c.hr64;
  a.tet_off = c.tet_off;
  a.l0_tv = c.l0_tv;
  a.l0_home = c.l0_home;
  a.bk = c.bk;
  a.bgrad = c.bgrad;
  a.bidx = c.bidx;
  a.bc_off = c.bc_off;
  a.bc_list = c.bc_list;
  for (int l = 0; l < c.L; ++l) a.acc[l] = c.lv[l].acc;
  a.coup = c.coup;
  const size_t nT = size_t(std::max(c.L - 1, 1)) * SUB * 9;
  if (c.cfg.deterministic) {
    const size_t lds = sizeof(double) * nT + sizeof(int) * (PK + nT);
    if (c.hr32)
      k_assemble_l0<float, true><<<dim3(L0.nsub), dim3(L0_THREADS), lds, c.s>>>(a);
    else
      k_assemble_l0<double, true><<<dim3(L0.nsub), dim3(L0_THREADS), lds, c.s>>>(a);
    for (int l = 2; l < c.L; ++l) {
      const int64_t n = c.lv[l - 1].nsub * int64_t(SUB * 9);
      k_coup_reduce<<<dim3((n + 255) / 256), dim3(256), 0, c.s>>>(l, c.L, L0.nsub, c.lv[l - 1].nsub, c.coup,
                                                                   c.lv[l].acc);
    }
  } else {
    const size_t lds = sizeof(double) * nT;
    if (c.hr32)
      k_assemble_l0<float, false><<<dim3(L0.nsub), dim3(L0_THREADS), lds, c.s>>>(a);
    else
      k_assemble_l0<double, false><<<dim3(L0.nsub), dim3(L0_THREADS), lds, c.s>>>(a);
  }
  if (c.cfg.precond == MAS_PRECOND_BJ3) return launch_bj_build(c);  // no MAS level is inverted
  // level 0, whose inversion completes level 1's diagonal node blocks; the
  // deeper diagonal node blocks are sums over the level below; then every
  // coarse level in one launch (their blocks are few, each a long chain)
  launch_invert_mfma(c, 0, 1, c.L > 1 ? c.lv[1].acc : nullptr);
  for (int l = 2; l < c.L; ++l)
    k_node_sums<<<dim3(c.lv[l - 1].nsub), dim3(NS_T), 0, c.s>>>(c.lv[l - 1].nodes, c.lv[l - 1].acc, c.lv[l].acc);
  if (c.L > 1) launch_invert_mfma(c, 1, c.L, nullptr);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
