// Matrix-free product with the frozen Hessian snapshot:
//   y = M v + sum_e S_e^T H_e S_e v + sum_{c in base} k_c n_c (n_c^T v)
//       [+ sum_c u_c (u_c^T v) for the current update columns].
// H_e is never formed: each tet stores its projected 9x9 tangent (45) and
// Dm^-1 (9) and applies B^T Hf B v on the fly, which moves 54 values per tet
// instead of the 78 of a packed 12x12.
#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

__global__ void k_mass_mul(int64_t n3, const double* mass, const double* v, double* y) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  y[i] = mass[i / 3] * v[i];
}

// Each workgroup applies SW_CHUNK consecutive tets (sorted by smallest
// vertex) and scatters through an LDS window starting at the chunk's first
// smallest vertex.
template <typename TH>
__global__ __launch_bounds__(256) void k_hv_tets(int64_t N, int64_t T, const int32_t* tets, const TH* hf,
                                                 const double* v, double* y) {
  __shared__ double win[3 * SW_WIN];
  const int64_t t0 = int64_t(blockIdx.x) * SW_CHUNK;
  const int4 f4 = reinterpret_cast<const int4*>(tets)[t0];
  const int vbase = min(min(f4.x, f4.y), min(f4.z, f4.w));
  for (int e = threadIdx.x; e < 3 * SW_WIN; e += blockDim.x) win[e] = 0.0;
  __syncthreads();
  for (int k = 0; k < SW_CHUNK; k += 256) {
    const int64_t t = t0 + k + threadIdx.x;
    if (t >= T) break;
    TH H[sizeof(TH) == 8 ? EH : 4 * SNAP_NC32];
    snap_load(hf, t, H);
    const int4 tv = reinterpret_cast<const int4*>(tets)[t];
    const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
    double ve[12];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) ve[3 * j + a] = v[3 * vi[j] + a];
    double f[12];
    elem_hv<TH>(H, H + 45, ve, f);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) sw_add(win, y, vbase, vi[j], a, f[3 * j + a]);
  }
  __syncthreads();
  sw_flush(win, y, vbase, N);
}

// rank-one stencil columns: y += u (u^T v), scattered through an LDS window
// (columns in the order given; sorted by smallest vertex they stay local)
__global__ __launch_bounds__(256) void k_hv_cols(int64_t N, int64_t m, const int32_t* idx, const double* u,
                                                 const double* v, double* y) {
  __shared__ double win[3 * SW_WIN];
  const int64_t c0 = int64_t(blockIdx.x) * SW_CHUNK;
  int vbase;
  {
    const int4 f4 = reinterpret_cast<const int4*>(idx)[c0];
    int mn = INT32_MAX;
    if (f4.x >= 0) mn = min(mn, f4.x);
    if (f4.y >= 0) mn = min(mn, f4.y);
    if (f4.z >= 0) mn = min(mn, f4.z);
    if (f4.w >= 0) mn = min(mn, f4.w);
    vbase = (mn == INT32_MAX) ? 0 : mn;
  }
  for (int e = threadIdx.x; e < 3 * SW_WIN; e += blockDim.x) win[e] = 0.0;
  __syncthreads();
  for (int k = 0; k < SW_CHUNK; k += 256) {
    const int64_t i = c0 + k + threadIdx.x;
    if (i >= m) break;
    const int4 iv = reinterpret_cast<const int4*>(idx)[i];
    const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    double uu[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) uu[q] = u[12 * i + q];
    double w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) w += uu[3 * j + a] * v[3 * vi[j] + a];
    }
    if (w == 0.0) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) sw_add(win, y, vbase, vi[j], a, w * uu[3 * j + a]);
    }
  }
  __syncthreads();
  sw_flush(win, y, vbase, N);
}

mas_status launch_hessvec(Ctx& c, const double* v, double* y, int with_update) {
  ProfScope ps(c, MAS_T_HESSVEC);
  int64_t n3 = 3 * c.N;
  k_mass_mul<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, c.mass, v, y);
  if (c.T > 0) {
    ProfScope pt(c, MAS_T_HV_TETS);
    dim3 g((c.T + SW_CHUNK - 1) / SW_CHUNK), b(256);
    if (c.hf32)
      k_hv_tets<float><<<g, b, 0, c.s>>>(c.N, c.T, c.tets, c.hf32, v, y);
    else
      k_hv_tets<double><<<g, b, 0, c.s>>>(c.N, c.T, c.tets, c.hf64, v, y);
  }
  if (c.mb > 0)
    k_hv_cols<<<dim3((c.mb + SW_CHUNK - 1) / SW_CHUNK), dim3(256), 0, c.s>>>(c.N, c.mb, c.bidx, c.bu, v, y);
  if (with_update && c.have_update && c.mc > 0)
    k_hv_cols<<<dim3((c.mc + SW_CHUNK - 1) / SW_CHUNK), dim3(256), 0, c.s>>>(c.N, c.mc, c.Uidx, c.U, v, y);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
