// Preconditioner apply z = P g: restriction to every coarse level, coarse
// block solves, then one workgroup per level-0 subdomain streams its inverse
// block through LDS, applies the Woodbury correction and adds the coarse
// corrections of the subdomain's vertices.
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
__device__ inline double lds_entry(const unsigned char* As, int e) {
  if (P == MAS_F64) return reinterpret_cast<const double*>(As)[e];
  if (P == MAS_F32) return double(reinterpret_cast<const float*>(As)[e]);
  uint16_t h = reinterpret_cast<const uint16_t*>(As)[e];
  return double((P == MAS_BF16) ? bf16_to_f32(h) : f16_to_f32(h));
}

// y_row = sum_j A(row, j) x_j for a packed-lower symmetric block in LDS; the
// 192 threads split each row into two halves of 48 columns.
template <int P>
__device__ inline double row_half(const unsigned char* As, const double* x, int row, int half) {
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

struct CoarseBlocks {
  int L;
  int prec;
  int64_t first[MAXL + 1];  // prefix of subdomain counts over levels 1..L-1
  int64_t nodes[MAXL];
  const void* blk[MAXL];
  const double* r[MAXL];
  double* c[MAXL];
};

template <int P>
__global__ __launch_bounds__(256) void k_apply_coarse(CoarseBlocks cb) {
  constexpr size_t E = blk_elems(P);
  constexpr size_t ES = prec_size(P);
  __shared__ __align__(16) unsigned char As[E * ES];
  __shared__ double x[BD];
  __shared__ double part[2][BD];
  int64_t gb = blockIdx.x;
  int l = 1;
  while (l + 1 < cb.L && gb >= cb.first[l + 1]) ++l;
  const int64_t d = gb - cb.first[l];
  const int tid = threadIdx.x;
  {
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(cb.blk[l]) + d * E * ES);
    uint4* dst = reinterpret_cast<uint4*>(As);
    for (int q = tid; q < int(E * ES / 16); q += blockDim.x) dst[q] = src[q];
  }
  if (tid < BD) {
    int64_t a = SUB * d + tid / 3;
    x[tid] = a < cb.nodes[l] ? cb.r[l][BD * d + tid] : 0.0;
  }
  __syncthreads();
  if (tid < 2 * BD) part[tid / BD][tid % BD] = row_half<P>(As, x, tid % BD, tid / BD);
  __syncthreads();
  if (tid < BD) {
    int64_t a = SUB * d + tid / 3;
    if (a < cb.nodes[l]) cb.c[l][BD * d + tid] = part[0][tid] + part[1][tid];
  }
}

struct FineArgs {
  int64_t N;
  const void* blk;
  const float* scale;
  const double* g;
  double* z;
  const int32_t* rank;  // nullptr: no Woodbury update
  int K;
  const SlotCol* slots;
  const void* W;
  const double* Lcap;
  int L;
  const double* c[MAXL];
};

template <int P>
__global__ __launch_bounds__(256) void k_apply_l0(FineArgs fa) {
  constexpr size_t E = blk_elems(P);
  constexpr size_t ES = prec_size(P);
  constexpr bool Q16 = (P == MAS_BF16 || P == MAS_F16);
  __shared__ __align__(16) unsigned char As[E * ES];
  __shared__ double x[BD];
  __shared__ double part[2][BD];
  __shared__ double zb[BD];
  __shared__ double rr[MAXK];
  __shared__ double lam[MAXK];
  __shared__ float sig[BD];
  const int64_t d = blockIdx.x;
  const int tid = threadIdx.x;
  {
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(fa.blk) + d * E * ES);
    uint4* dst = reinterpret_cast<uint4*>(As);
    for (int q = tid; q < int(E * ES / 16); q += blockDim.x) dst[q] = src[q];
  }
  if (tid < BD) {
    int64_t v = SUB * d + tid / 3;
    double gv = v < fa.N ? fa.g[BD * d + tid] : 0.0;
    if (Q16) {
      float s = fa.scale[BD * d + tid];
      sig[tid] = s;
      gv *= double(s);
    }
    x[tid] = gv;
  }
  __syncthreads();
  if (tid < 2 * BD) part[tid / BD][tid % BD] = row_half<P>(As, x, tid % BD, tid / BD);
  __syncthreads();
  if (tid < BD) {
    double v = part[0][tid] + part[1][tid];
    if (Q16) v *= double(sig[tid]);
    zb[tid] = v;
  }
  const int r = fa.rank ? fa.rank[d] : 0;
  if (r > 0) {
    __syncthreads();
    // r_j = u_j^T z_base over the stencil vertices inside the subdomain
    if (tid < r) {
      const SlotCol& sc = fa.slots[d * fa.K + tid];
      double acc = 0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int lv = sc.lv[s];
        if (lv < 0) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc += sc.u[3 * s + a] * zb[3 * lv + a];
      }
      rr[tid] = acc;
    }
    __syncthreads();
    if (tid == 0) {
      // (L L^T) lambda = r: forward substitution in place in rr, then backward
      const double* Lm = fa.Lcap + d * (fa.K * (fa.K + 1) / 2);
      for (int i = 0; i < r; ++i) {
        double v = rr[i];
        for (int k = 0; k < i; ++k) v -= Lm[pk(i, k)] * rr[k];
        rr[i] = v / Lm[pk(i, i)];
      }
      for (int i = r - 1; i >= 0; --i) {
        double v = rr[i];
        for (int k = i + 1; k < r; ++k) v -= Lm[pk(k, i)] * lam[k];
        lam[i] = v / Lm[pk(i, i)];
      }
    }
    __syncthreads();
    if (tid < BD) {
      double acc = 0;
      if (P == MAS_F64) {
        const double* Wd = reinterpret_cast<const double*>(fa.W) + d * fa.K * BD;
        for (int j = 0; j < r; ++j) acc += Wd[j * BD + tid] * lam[j];
      } else {
        const float* Wd = reinterpret_cast<const float*>(fa.W) + d * fa.K * BD;
        for (int j = 0; j < r; ++j) acc += double(Wd[j * BD + tid]) * lam[j];
      }
      zb[tid] -= acc;
    }
  }
  if (tid < BD) {
    int64_t v = SUB * d + tid / 3;
    if (v < fa.N) {
      double out = zb[tid];
      const int c = tid % 3;
      for (int l = 1; l < fa.L; ++l) out += fa.c[l][3 * (v >> (5 * l)) + c];
      fa.z[BD * d + tid] = out;
    }
  }
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
      cb.r[l] = c.lv[l].r;
      cb.c[l] = c.lv[l].c;
    }
    int64_t total = cb.first[c.L];
    if (c.lv[1].prec == MAS_F64) k_apply_coarse<MAS_F64><<<dim3(total), dim3(256), 0, c.s>>>(cb);
    else k_apply_coarse<MAS_F32><<<dim3(total), dim3(256), 0, c.s>>>(cb);
  }
  FineArgs fa{};
  fa.N = c.N;
  fa.blk = c.lv[0].blk;
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
  dim3 gr(c.lv[0].nsub), bl(256);
  prof_begin(c, MAS_T_APPLY_L0);
  switch (c.lv[0].prec) {
    case MAS_F64: k_apply_l0<MAS_F64><<<gr, bl, 0, c.s>>>(fa); break;
    case MAS_F32: k_apply_l0<MAS_F32><<<gr, bl, 0, c.s>>>(fa); break;
    case MAS_BF16: k_apply_l0<MAS_BF16><<<gr, bl, 0, c.s>>>(fa); break;
    default: k_apply_l0<MAS_F16><<<gr, bl, 0, c.s>>>(fa);
  }
  prof_end(c, MAS_T_APPLY_L0);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
