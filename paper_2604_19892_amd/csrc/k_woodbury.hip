// Sparse-Input Woodbury update of the level-0 blocks: classification of the
// current contacts against the base set, localized Top-K per subdomain and
// the capacitance factors I + U_d^T B_d U_d.
#include <algorithm>

#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

// Each current contact: k = kappa b''(d); looked up by key in the base set.
//   not found            -> dS = k
//   found, cos < cos_rot -> dS = k          (rotated normal, treated as new)
//   found, k > k_base    -> dS = k - k_base (stiffening)
//   otherwise            -> dS = 0          (softening)
// The column u = sqrt(dS) n enters the untruncated U.
// A contact with k = 0 (d >= dhat) has dS = 0 whatever the base holds, so it
// is not looked up, and a column with dS = 0 is not stored (readers of U
// test dS first).  The lookup first tries the same position in the base
// set (contact sets that keep their order between build and update), then
// the base-key hash table.
// Per workgroup the counts of the branches taken (active, new, rotated,
// stiffened, softened) go to part[5 * block + q]; they are summed only when
// the counters are read.
constexpr int CLS_T = 256;

__global__ __launch_bounds__(CLS_T) void k_classify(int64_t m, const uint64_t* key, const int32_t* idx,
                                                    const double* d, const double* grad, double kappa, double dhat,
                                                    double cos_rot, int64_t mb, const uint64_t* bkey,
                                                    const uint64_t* hkey, const int32_t* hval, int64_t hmask,
                                                    const double* bk, const double* bgrad, double* U, int32_t* Uidx,
                                                    double* dS, uint8_t* upm, uint64_t* ckey, uint32_t* err,
                                                    int32_t* part) {
  __shared__ int cnt[5];
  if (threadIdx.x < 5) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  int branch = -1;  // 1 new, 2 rotated, 3 stiffened, 4 softened
  if (i < m) {
    double b, b1, b2;
    const double di = d[i];
    if (!isfinite(di)) atomicOr(err, ERRB_NONFINITE);
    barrier3(di, dhat, &b, &b1, &b2);
    const double k = kappa * b2;
    const uint64_t kk = key[i];
    ckey[i] = kk;
    reinterpret_cast<int4*>(Uidx)[i] = reinterpret_cast<const int4*>(idx)[i];
    if (!(k > 0.0)) {
      dS[i] = 0.0;  // the column is zero and is not stored: readers test dS first
      upm[i] = 0;
    } else {
      double n[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) n[q] = grad[12 * i + q];
      double s = k;
      branch = 1;
      int64_t bi = -1;
      if (i < mb && bkey[i] == kk) {
        bi = i;
      } else if (mb > 0) {
        // probe the base-key table until the key or a free slot
        int64_t h = int64_t(key_hash(kk) & uint64_t(hmask));
        while (true) {
          const uint64_t hk = hkey[h];
          if (hk == kk) {
            bi = hval[h];
            break;
          }
          if (hk == HKEY_EMPTY) break;
          h = (h + 1) & hmask;
        }
      }
      if (bi >= 0) {
        double dot = 0, nn = 0, bb = 0;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
          const double nb = bgrad[12 * bi + q];
          dot += n[q] * nb;
          nn += n[q] * n[q];
          bb += nb * nb;
        }
        const double cosang = dot / (sqrt(nn) * sqrt(bb));
        if (cosang < cos_rot) {
          s = k;
          branch = 2;
        } else if (k > bk[bi]) {
          s = k - bk[bi];
          branch = 3;
        } else {
          s = 0.0;
          branch = 4;
        }
      }
      if (!(s > 0.0)) s = 0.0;
      dS[i] = s;
      uint8_t pm = 0;
      if (s > 0.0) {
        const double sq = sqrt(s);
        double u[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
          u[q] = sq * n[q];
          U[12 * i + q] = u[q];
        }
        pm = part_mask(u);
      }
      upm[i] = pm;
    }
  }
  if (part) {
    if (branch > 0) {
      atomicAdd(&cnt[0], 1);
      atomicAdd(&cnt[branch], 1);
    }
    __syncthreads();
    if (threadIdx.x < 5) part[5 * int64_t(blockIdx.x) + threadIdx.x] = cnt[threadIdx.x];
  }
}

// ranking order: larger dS first, then smaller key
__device__ inline bool ranks_before(double s1, uint64_t k1, double s2, uint64_t k2) {
  return s1 > s2 || (s1 == s2 && k1 < k2);
}

// One wavefront per subdomain: K rounds of a wave-wide arg-best.  Lists of
// up to 64 * TOPK_R candidates are held in registers (TOPK_R per lane) and a
// pick is struck out by its holder; longer lists are rescanned from memory
// each round for the best candidate ranked after the previous pick.
constexpr int TOPK_R = 8;

__device__ __forceinline__ void wave_best(double& bs, unsigned long long& bkey, int& bc) {
  for (int o = 32; o > 0; o >>= 1) {
    const double os = __shfl_xor(bs, o);
    const unsigned long long ok = __shfl_xor(bkey, o);
    const int oc = __shfl_xor(bc, o);
    if (oc >= 0 && (bc < 0 || ranks_before(os, ok, bs, bkey))) {
      bs = os;
      bkey = ok;
      bc = oc;
    }
  }
}

__device__ __forceinline__ void topk_emit(int64_t d, int K, int r, int bc, int lane, const int32_t* Uidx,
                                          const double* U, int32_t* sel, SlotCol* slots) {
  SlotCol* sc = slots + d * K + r;
  if (lane == 0) sel[d * K + r] = bc;
  if (lane < 12) sc->u[lane] = U[12 * int64_t(bc) + lane];
  if (lane < 4) {
    const int v = Uidx[4 * int64_t(bc) + lane];
    sc->lv[lane] = (v >= 0 && (v >> 5) == d) ? (v & 31) : -1;
  }
}

__global__ __launch_bounds__(64, 6) void k_topk(int K, const int32_t* off, const int32_t* list,
                                             const double* dS, const uint64_t* key, const int32_t* Uidx,
                                             const double* U, int32_t* rank, int32_t* sel,
                                             SlotCol* slots) {
  const int64_t d = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = off[d], e = off[d + 1];
  int r = 0;
  if (e - b <= 64 * TOPK_R) {
    double s[TOPK_R];
    unsigned long long kk[TOPK_R];
    int cc[TOPK_R];
#pragma unroll
    for (int q = 0; q < TOPK_R; ++q) {
      const int w = b + lane + 64 * q;
      cc[q] = -1;
      s[q] = 0.0;
      kk[q] = 0;
      if (w < e) {
        cc[q] = list[w];
        s[q] = dS[cc[q]];
        kk[q] = key[cc[q]];
      }
    }
    for (; r < K; ++r) {
      double bs = 0.0;
      unsigned long long bkey = 0;
      int bc = -1;
#pragma unroll
      for (int q = 0; q < TOPK_R; ++q) {
        if (cc[q] >= 0 && (bc < 0 || ranks_before(s[q], kk[q], bs, bkey))) {
          bs = s[q];
          bkey = kk[q];
          bc = cc[q];
        }
      }
      wave_best(bs, bkey, bc);
      if (bc < 0) break;
#pragma unroll
      for (int q = 0; q < TOPK_R; ++q)
        if (cc[q] == bc) cc[q] = -1;
      topk_emit(d, K, r, bc, lane, Uidx, U, sel, slots);
    }
  } else {
    double ps = 0.0;
    uint64_t pkey = 0;
    bool first = true;
    for (; r < K; ++r) {
      double bs = 0.0;
      unsigned long long bkey = 0;
      int bc = -1;
      for (int q = b + lane; q < e; q += 64) {
        const int c = list[q];
        const double sv = dS[c];
        const uint64_t kv = key[c];
        if (!first && !ranks_before(ps, pkey, sv, kv)) continue;
        if (bc < 0 || ranks_before(sv, kv, bs, bkey)) {
          bs = sv;
          bkey = kv;
          bc = c;
        }
      }
      wave_best(bs, bkey, bc);
      if (bc < 0) break;
      topk_emit(d, K, r, bc, lane, Uidx, U, sel, slots);
      ps = bs;
      pkey = bkey;
      first = false;
    }
  }
  if (lane == 0) {
    rank[d] = r;
    for (int q = r; q < K; ++q) sel[d * K + q] = -1;
  }
}

// Histogram of the per-subdomain ranks: LDS counts per workgroup, then one
// global atomic per bin and workgroup (a global atomic per subdomain would
// serialise on the K + 1 addresses).
__global__ __launch_bounds__(256) void k_rank_hist(int64_t D, int K, const int32_t* rank, int32_t* hist) {
  __shared__ int h[MAXK + 1];
  for (int q = threadIdx.x; q <= K; q += blockDim.x) h[q] = 0;
  __syncthreads();
  for (int64_t d = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; d < D; d += int64_t(gridDim.x) * blockDim.x)
    atomicAdd(&h[rank[d]], 1);
  __syncthreads();
  for (int q = threadIdx.x; q <= K; q += blockDim.x)
    if (h[q]) atomicAdd(&hist[q], h[q]);
}

template <int P>
__device__ __forceinline__ double block_entry(const unsigned char* A, const float* sig, int i, int j) {
  const int e = blk_pos(P, i, j);
  if (P == MAS_F64) return reinterpret_cast<const double*>(A)[e];
  if (P == MAS_F32) return double(reinterpret_cast<const float*>(A)[e]);
  uint16_t h = reinterpret_cast<const uint16_t*>(A)[e];
  float v = (P == MAS_BF16) ? bf16_to_f32(h) : f16_to_f32(h);
  return double(v) * double(sig[i]) * double(sig[j]);
}

// W[:, j] = B_d u_j: a gather of at most 12 columns of B_d
template <int P>
__device__ __forceinline__ void gather_w(const unsigned char* As, const float* sig, const SlotCol* sl, int r,
                                         double (*Ws)[BD]) {
  for (int q = threadIdx.x; q < r * BD; q += blockDim.x) {
    int j = q / BD, i = q % BD;
    double acc = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int lv = sl[j].lv[s];
      if (lv < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) acc += block_entry<P>(As, sig, i, 3 * lv + a) * sl[j].u[3 * s + a];
    }
    Ws[j][i] = acc;
  }
}

// One workgroup per subdomain with rank r > 0: W = B_d U_d (96 x r), the
// capacitance C = I + U_d^T W and its float64 Cholesky factor (right-looking,
// on the first wavefront).  Blocks
// stored in 32 or 16 bits are staged in LDS, float64 blocks are read in
// place; W, C and the slot columns live in dynamic LDS sized by K.
constexpr size_t CAP_STAGE = blk_elems(MAS_F32) * 4;

__global__ __launch_bounds__(256) void k_capacitance(int K, const void* blk, const uint8_t* bprec,
                                                     const float* scale, int32_t* rank, const SlotCol* slots,
                                                     double* W, double* Lcap, uint32_t* err, DiagRec* dg) {
  __shared__ __align__(16) unsigned char As[CAP_STAGE];
  __shared__ float sig[BD];
  extern __shared__ __align__(16) double cdyn[];
  double(*Ws)[BD] = reinterpret_cast<double(*)[BD]>(cdyn);
  double* Cm = cdyn + K * BD;
  SlotCol* sl = reinterpret_cast<SlotCol*>(Cm + K * K);
  const int64_t d = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = rank[d];
  if (r == 0) return;
  const int P = bprec[d];
  const unsigned char* src = reinterpret_cast<const unsigned char*>(blk) + d * BLK_STRIDE;
  if (P != MAS_F64) {
    const int nbytes = int(blk_elems(P) * prec_size(P));
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* dst = reinterpret_cast<uint4*>(As);
    for (int q = tid; q < nbytes / 16; q += blockDim.x) dst[q] = s4[q];
  }
  if (P == MAS_BF16 || P == MAS_F16) {
    if (tid < BD) sig[tid] = scale[d * BD + tid];
  }
  for (int q = tid; q < r; q += blockDim.x) sl[q] = slots[d * K + q];
  __syncthreads();
  switch (P) {
    case MAS_F64: gather_w<MAS_F64>(src, sig, sl, r, Ws); break;
    case MAS_F32: gather_w<MAS_F32>(As, sig, sl, r, Ws); break;
    case MAS_BF16: gather_w<MAS_BF16>(As, sig, sl, r, Ws); break;
    default: gather_w<MAS_F16>(As, sig, sl, r, Ws);
  }
  __syncthreads();
  for (int q = tid; q < r * r; q += blockDim.x) {
    int j = q / r, k = q % r;
    double acc = (j == k) ? 1.0 : 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int lv = sl[j].lv[s];
      if (lv < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) acc += sl[j].u[3 * s + a] * Ws[k][3 * lv + a];
    }
    Cm[j * r + k] = acc;
  }
  __syncthreads();
  // C = L L^T in place (lower triangle), float64, by the first wavefront
  // alone (r <= K is small: the steps order themselves within the
  // wavefront, no workgroup barrier) while the others write W.  Column j of
  // L depends on the leading (j + 1) x (j + 1) part of C only, so a pivot
  // that is not positive ends the factor there: the subdomain keeps its
  // first j columns (the ones of largest dS) and the rank drops to j.
  if (tid < 64) {
    int rk = r;
    for (int j = 0; j < r; ++j) {
      const double djj = Cm[j * r + j];  // the same value in every lane
      if (!(djj > 0.0) || !isfinite(djj)) {
        if (tid == 0) diag_report(dg + MAXL, 3, 0, d, j, djj);
        rk = j;
        break;
      }
      const double ljj = sqrt(djj);
      wave_sync();
      for (int i = j + 1 + tid; i < r; i += 64) Cm[i * r + j] /= ljj;
      if (tid == 0) Cm[j * r + j] = ljj;
      wave_sync();
      const int nr = r - j - 1;
      for (int q = tid; q < nr * nr; q += 64) {
        const int i = j + 1 + q / nr, k = j + 1 + q % nr;
        if (k <= i) Cm[i * r + k] -= Cm[i * r + j] * Cm[k * r + j];
      }
      wave_sync();
    }
    if (tid == 0 && rk < r) {
      atomicOr(err, ERRB_RANK);
      rank[d] = rk;
    }
    double* L = Lcap + d * (K * (K + 1) / 2);
    for (int q = tid; q < rk * rk; q += 64) {
      const int i = q / rk, j = q % rk;
      if (j <= i) L[pk(i, j)] = Cm[i * r + j];
    }
  } else {
    // all r columns (the apply reads only the first rank[d] of them)
    for (int q = tid - 64; q < r * BD; q += blockDim.x - 64) {
      const int j = q / BD, i = q % BD;
      W[(d * K + j) * BD + i] = Ws[j][i];
    }
  }
}

mas_status launch_woodbury(Ctx& c, const mas_contacts* cur, int32_t* rank_hist) {
  ProfScope ps(c, MAS_T_UPDATE);
  int64_t m = cur ? cur->m : 0;
  if (m > c.mc_cap) return MAS_ERR_INVALID_ARG;  // checked by mas_woodbury_update
  mas_status st = MAS_OK;
  c.mc = m;
  c.cls_blocks = (m + CLS_T - 1) / CLS_T;
  if (m > 0) {
    k_classify<<<dim3(c.cls_blocks), dim3(CLS_T), 0, c.s>>>(
        m, cur->key, cur->idx, cur->d, cur->grad, c.cfg.kappa, c.cfg.dhat, c.cfg.cos_rot, c.mb,
        c.bkey, c.hkey, c.hval, c.hsize - 1, c.bk, c.bgrad, c.U, c.Uidx, c.dS, c.upm, c.ckey, c.err, c.cls_part);
    HIPCHK(hipGetLastError());
  }
  const int64_t D = c.lv[0].nsub;
  if (c.cfg.precond == MAS_PRECOND_BJ3) {
    // the vertex blocks of H~ instead of Top-K and capacitance
    if (rank_hist) {
      fill_i32(c, rank_hist, c.K + 1, 0);
      fill_i32(c, rank_hist, 1, int32_t(D));
    }
    return launch_bj_update(c, m);
  }
  st = bucket_by_subdomain(c, m, c.Uidx, c.upm, c.cand_cnt, c.cand_off, c.cand_list);
  if (st != MAS_OK) return st;
  if (rank_hist) fill_i32(c, rank_hist, c.K + 1, 0);
  if (c.K == 0) {
    fill_i32(c, c.rank, D, 0);
    if (rank_hist) fill_i32(c, rank_hist, 1, int32_t(D));
    return MAS_OK;
  }
  k_topk<<<dim3(D), dim3(64), 0, c.s>>>(c.K, c.cand_off, c.cand_list, c.dS, c.ckey, c.Uidx, c.U, c.rank,
                                        c.sel, c.slots);
  Level& L0 = c.lv[0];
  {
    ProfScope pc(c, MAS_T_CAPACITANCE);
    const size_t cap_lds = sizeof(double) * (size_t(c.K) * BD + size_t(c.K) * c.K) + sizeof(SlotCol) * c.K;
    k_capacitance<<<dim3(D), dim3(256), cap_lds, c.s>>>(c.K, L0.blk, L0.bprec, L0.scale, c.rank, c.slots, c.W,
                                                        c.Lcap, c.err, c.diag);
  }
  // after the capacitance factors, which may lower a rank
  if (rank_hist)
    k_rank_hist<<<dim3(std::min<int64_t>(64, (D + 255) / 256)), dim3(256), 0, c.s>>>(D, c.K, c.rank, rank_hist);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
