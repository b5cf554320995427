// Preconditioner apply z = P g: restriction to every coarse level, coarse
// block solves, then one workgroup per level-0 subdomain streams its inverse
// block through LDS, applies the Woodbury correction and adds the coarse
// corrections of the subdomain's vertices.
#include <algorithm>

#include "kernels.hpp"

namespace mas {

// r_1[3a+c] = sum of g over the 32 vertices of level-1 node a; levels >= 2
// accumulate those sums into their nodes (zeroed beforehand).
struct RestrictArgs {
  int L;
  double* r[MAXL];
};

__global__ void k_restrict(int64_t N, int64_t nodes1, const double* g, RestrictArgs ra) {
  int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (q >= 3 * nodes1) return;
  int64_t a = q / 3;
  int c = int(q % 3);
  double s = 0;
  int64_t v0 = SUB * a;
  int64_t v1 = v0 + SUB < N ? v0 + SUB : N;
  for (int64_t v = v0; v < v1; ++v) s += g[3 * v + c];
  ra.r[1][q] = s;
  for (int l = 2; l < ra.L; ++l) atomicAdd(&ra.r[l][3 * (a >> (5 * (l - 1))) + c], s);
}

template <int P>
__device__ __forceinline__ double lds_entry(const unsigned char* As, int e) {
  if (P == MAS_F64) return reinterpret_cast<const double*>(As)[e];
  if (P == MAS_F32) return double(reinterpret_cast<const float*>(As)[e]);
  uint16_t h = reinterpret_cast<const uint16_t*>(As)[e];
  return double((P == MAS_BF16) ? bf16_to_f32(h) : f16_to_f32(h));
}

// y_row = sum_j A(row, j) x_j for a packed-lower symmetric block in LDS; the
// 192 threads split each row into two halves of 48 columns.
template <int P>
__device__ __forceinline__ double row_half(const unsigned char* As, const double* x, int row, int half) {
  double acc = 0;
  const int j0 = 48 * half;
  const int br = row * (row + 1) / 2;
#pragma unroll 8
  for (int jj = 0; jj < 48; ++jj) {
    const int j = j0 + jj;
    const int e = (j <= row) ? br + j : j * (j + 1) / 2 + row;
    acc += lds_entry<P>(As, e) * x[j];
  }
  return acc;
}

__device__ __forceinline__ int slot_bytes(int P) { return int(blk_elems(P) * prec_size(P)); }

// the 192 row-halves of a block product, in the block's stored precision
__device__ __forceinline__ void block_rows(int P, const unsigned char* As, const double* x, double (*part)[BD]) {
  const int tid = threadIdx.x;
  if (tid >= 2 * BD) return;
  const int row = tid % BD, half = tid / BD;
  double v;
  switch (P) {
    case MAS_F64: v = row_half<MAS_F64>(As, x, row, half); break;
    case MAS_F32: v = row_half<MAS_F32>(As, x, row, half); break;
    case MAS_BF16: v = row_half<MAS_BF16>(As, x, row, half); break;
    default: v = row_half<MAS_F16>(As, x, row, half);
  }
  part[half][row] = v;
}

__device__ __forceinline__ void load_slot(const void* blk, int64_t d, int P, unsigned char* As) {
  const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(blk) + d * BLK_STRIDE);
  uint4* dst = reinterpret_cast<uint4*>(As);
  const int n = slot_bytes(P) / 16;
  for (int q = threadIdx.x; q < n; q += blockDim.x) dst[q] = src[q];
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

__global__ __launch_bounds__(256) void k_apply_coarse(CoarseBlocks cb) {
  __shared__ __align__(16) unsigned char As[BLK_STRIDE];
  __shared__ double x[BD];
  __shared__ double part[2][BD];
  __shared__ float sig[BD];
  int64_t gb = blockIdx.x;
  int l = 1;
  while (l + 1 < cb.L && gb >= cb.first[l + 1]) ++l;
  const int64_t d = gb - cb.first[l];
  const int tid = threadIdx.x;
  const int P = cb.bprec[l][d];
  const bool q16 = (P == MAS_BF16 || P == MAS_F16);
  load_slot(cb.blk[l], d, P, As);
  if (tid < BD) {
    int64_t a = SUB * d + tid / 3;
    double xv = a < cb.nodes[l] ? cb.r[l][BD * d + tid] : 0.0;
    if (q16) {
      sig[tid] = cb.scale[l][BD * d + tid];
      xv *= double(sig[tid]);
    }
    x[tid] = xv;
  }
  __syncthreads();
  block_rows(P, As, x, part);
  __syncthreads();
  if (tid < BD) {
    int64_t a = SUB * d + tid / 3;
    double v = part[0][tid] + part[1][tid];
    if (q16) v *= double(sig[tid]);
    if (a < cb.nodes[l]) cb.c[l][BD * d + tid] = v;
  }
}

struct FineArgs {
  int64_t N;
  int64_t D;
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
};

constexpr int PF = (BLK_STRIDE / 16 + 255) / 256;  // 16-byte prefetch registers per thread

// Persistent workgroups stream the level-0 blocks.  While block d is applied
// from LDS, everything block d + grid needs from memory (the block, its
// slice of g, the coarse corrections of its vertices and its rank) is
// already loading into registers, so the HBM latency overlaps the LDS work.
// Updated subdomains fetch their Woodbury data (slot columns, capacitance
// factor, W) in one batch.
__global__ __launch_bounds__(256) void k_apply_l0(FineArgs fa) {
  __shared__ __align__(16) unsigned char As[BLK_STRIDE];
  __shared__ double x[BD];
  __shared__ double part[2][BD];
  __shared__ double zb[BD];
  __shared__ double rr[MAXK];
  __shared__ double lam[MAXK];
  __shared__ double Lf[MAXK * (MAXK + 1) / 2];
  __shared__ SlotCol sl[MAXK];
  __shared__ float sig[BD];
  const int tid = threadIdx.x;
  const int K = fa.K;
  int P = 0, Pn = 0, rn = 0;
  double gn = 0.0, cn[MAXL - 1];
  float sn = 1.0f;
#pragma unroll
  for (int l = 0; l < MAXL - 1; ++l) cn[l] = 0.0;
  int64_t d = blockIdx.x;
  static_assert(PF == 10, "prefetch registers are spelled out for 10 chunks");
  uint4 p0, p1, p2, p3, p4, p5, p6, p7, p8, p9;
#define MAS_PF1(R, Q) \
  if (tid + 256 * (Q) < n_) R = src_[tid + 256 * (Q)];
#define MAS_PREFETCH(dd)                                                                                   \
  do {                                                                                                     \
    Pn = fa.bprec[dd];                                                                                     \
    rn = fa.rank ? fa.rank[dd] : 0;                                                                        \
    const int n_ = slot_bytes(Pn) / 16;                                                                    \
    const uint4* src_ =                                                                                    \
        reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(fa.blk) + (dd) * BLK_STRIDE); \
    MAS_PF1(p0, 0) MAS_PF1(p1, 1) MAS_PF1(p2, 2) MAS_PF1(p3, 3) MAS_PF1(p4, 4)                              \
    MAS_PF1(p5, 5) MAS_PF1(p6, 6) MAS_PF1(p7, 7) MAS_PF1(p8, 8) MAS_PF1(p9, 9)                              \
    if (tid < BD) {                                                                                        \
      const int64_t v_ = SUB * (dd) + tid / 3;                                                             \
      gn = v_ < fa.N ? fa.g[BD * (dd) + tid] : 0.0;                                                        \
      sn = fa.scale[BD * (dd) + tid];                                                                      \
      if (v_ < fa.N) {                                                                                     \
        _Pragma("unroll") for (int l_ = 1; l_ < MAXL; ++l_) if (l_ < fa.L) cn[l_ - 1] =                    \
            fa.c[l_][3 * (v_ >> (5 * l_)) + tid % 3];                                                      \
      }                                                                                                    \
    }                                                                                                      \
  } while (0)
#define MAS_ST1(R, Q) \
  if (tid + 256 * (Q) < n) dst[tid + 256 * (Q)] = R;
  if (d < fa.D) MAS_PREFETCH(d);
  for (; d < fa.D; d += gridDim.x) {
    P = Pn;
    const int r = rn;
    const bool q16 = (P == MAS_BF16 || P == MAS_F16);
    double corr = 0.0;
#pragma unroll
    for (int l = 0; l < MAXL - 1; ++l) corr += cn[l];
    {
      const int n = slot_bytes(P) / 16;
      uint4* dst = reinterpret_cast<uint4*>(As);
      MAS_ST1(p0, 0) MAS_ST1(p1, 1) MAS_ST1(p2, 2) MAS_ST1(p3, 3) MAS_ST1(p4, 4)
      MAS_ST1(p5, 5) MAS_ST1(p6, 6) MAS_ST1(p7, 7) MAS_ST1(p8, 8) MAS_ST1(p9, 9)
    }
    if (tid < BD) {
      if (q16) sig[tid] = sn;
      x[tid] = q16 ? gn * double(sn) : gn;
    }
    if (r > 0) {
      // Woodbury data of this subdomain, all loads in flight together
      const int nl = r * (r + 1) / 2;
      const double* Lm = fa.Lcap + d * (K * (K + 1) / 2);
      for (int q = tid; q < nl; q += blockDim.x) Lf[q] = Lm[q];
      if (tid < r) sl[tid] = fa.slots[d * K + tid];
    }
    __syncthreads();
    if (d + gridDim.x < fa.D) MAS_PREFETCH(d + gridDim.x);
    block_rows(P, As, x, part);
    __syncthreads();
    double zv = 0.0;
    if (tid < BD) {
      zv = part[0][tid] + part[1][tid];
      if (q16) zv *= double(sig[tid]);
      zb[tid] = zv;
    }
    if (r > 0) {
      __syncthreads();
      // r_j = u_j^T z_base over the stencil vertices inside the subdomain
      if (tid < r) {
        double acc = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          int lv = sl[tid].lv[s];
          if (lv < 0) continue;
#pragma unroll
          for (int a = 0; a < 3; ++a) acc += sl[tid].u[3 * s + a] * zb[3 * lv + a];
        }
        rr[tid] = acc;
      }
      __syncthreads();
      if (tid == 0) {
        // (L L^T) lambda = r: forward substitution in place in rr, then backward
        for (int i = 0; i < r; ++i) {
          double v = rr[i];
          for (int k = 0; k < i; ++k) v -= Lf[pk(i, k)] * rr[k];
          rr[i] = v / Lf[pk(i, i)];
        }
        for (int i = r - 1; i >= 0; --i) {
          double v = rr[i];
          for (int k = i + 1; k < r; ++k) v -= Lf[pk(k, i)] * lam[k];
          lam[i] = v / Lf[pk(i, i)];
        }
      }
      __syncthreads();
      if (tid < BD) {
        const double* Wd = fa.W + d * K * BD;
        double acc = 0;
        for (int j = 0; j < r; ++j) acc += Wd[j * BD + tid] * lam[j];
        zv -= acc;
      }
    }
    if (tid < BD) {
      const int64_t v = SUB * d + tid / 3;
      if (v < fa.N) fa.z[BD * d + tid] = zv + corr;
    }
    __syncthreads();
  }
#undef MAS_PREFETCH
#undef MAS_PF1
#undef MAS_ST1
}

mas_status launch_apply(Ctx& c, const double* g, double* z) {
  ProfScope ps(c, MAS_T_APPLY);
  if (c.L > 1) {
    RestrictArgs ra{};
    ra.L = c.L;
    for (int l = 1; l < c.L; ++l) ra.r[l] = c.lv[l].r;
    for (int l = 2; l < c.L; ++l) HIPCHK(hipMemsetAsync(c.lv[l].r, 0, sizeof(double) * 3 * c.lv[l].nodes, c.s));
    int64_t n1 = c.lv[1].nodes;
    k_restrict<<<dim3((3 * n1 + 255) / 256), dim3(256), 0, c.s>>>(c.N, n1, g, ra);
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
    k_apply_coarse<<<dim3(total), dim3(256), 0, c.s>>>(cb);
  }
  FineArgs fa{};
  fa.N = c.N;
  fa.D = c.lv[0].nsub;
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
  prof_begin(c, MAS_T_APPLY_L0);
  const int64_t grid = std::min<int64_t>(c.lv[0].nsub, int64_t(c.n_cu) * 3);
  k_apply_l0<<<dim3(grid), dim3(256), 0, c.s>>>(fa);
  prof_end(c, MAS_T_APPLY_L0);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
