// Matrix-free product with the frozen Hessian snapshot (H~ of Section 4.1):
//   y = M v + sum_e S_e^T H_e S_e v + sum_{c in base} k_c n_c (n_c^T v)
//       [+ sum_c u_c (u_c^T v) for the current update columns].
// H_e is never formed: each tet stores its projected 9x9 tangent (45) and
// Dm^-1 (9) and applies B^T Hf B v on the fly, which moves 54 values per tet
// instead of the 78 of a packed 12x12.
#include <algorithm>

#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

// Owner-computes product over the vertex ranges: the workgroup of range r
// applies every tet and every base stencil touching r, keeps only the rows of
// its own vertices (LDS accumulation) and writes y for them together with
// the mass term, so no output is ever written by two workgroups.  A tet
// touching k ranges has k entries (about 1.3 on the test scenes), each with
// its own copy of the snapshot, so a workgroup streams contiguous data.  The
// range's own part of v is staged in LDS once and read from there by every
// entry (only the vertices of other ranges are gathered from memory).  One
// workgroup per compute unit (the two 48 KB LDS arrays);
// resident workgroups take ranges from a counter (dynamic balance) and each
// exits once the counter has passed the last range.
// float64 snapshots take 512 threads, so that their larger per-thread state
// stays in registers.
template <typename TH>
constexpr int hv_threads() {
  return sizeof(TH) == 8 ? 512 : 1024;
}

// DET: the rows are summed with the two-pass fixed-point accumulation, so
// that they do not depend on the order of the LDS atomics (every tet and
// stencil of the range is applied twice).
template <typename TH, bool DET>
__global__ __launch_bounds__(hv_threads<TH>()) void k_hv_range(int64_t nrange, const int32_t* rbeg,
                                                                const int32_t* rt_off, const int32_t* rl_tv,
                                                                const TH* hr, const int32_t* bidx, const double* bu,
                                                                const int32_t* rc_off, const int32_t* rc_list,
                                                                const double* mass, const double* v, double* y,
                                                                uint32_t* ctr, uint32_t* err) {
  __shared__ double win[3 * RANGE_MAX];
  __shared__ double vs[3 * RANGE_MAX];
  __shared__ int aux[DET ? 3 * RANGE_MAX : 1];
  __shared__ int64_t cur;
  constexpr int NH = sizeof(TH) == 8 ? EH : 4 * SNAP_NC32;
  while (true) {
    if (threadIdx.x == 0) cur = atomicAdd(ctr, 1u);
    __syncthreads();
    const int64_t r = cur;
    if (r >= nrange) break;  // every workgroup ends here once the counter passes nrange
    const int v0 = rbeg[r], nv = rbeg[r + 1] - v0;
    for (int e = threadIdx.x; e < 3 * nv; e += blockDim.x) {
      win[e] = 0.0;
      if (DET) aux[e] = 0;
      const double ve = v[3 * int64_t(v0) + e];
      if (!isfinite(ve)) atomicOr(err, ERRB_NONFINITE);
      vs[e] = ve;
    }
    __syncthreads();
    for (int pass = DET ? 0 : 1; pass < 2; ++pass) {
    const int t0 = rt_off[r], t1 = rt_off[r + 1];
    for (int w = t0 + threadIdx.x; w < t1; w += blockDim.x) {
      const int4 tv = reinterpret_cast<const int4*>(rl_tv)[w];
      const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
      TH H[NH];
      snap_load(hr, w, H);
      double ve[12];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int lv = vi[j] - v0;
        if (lv >= 0 && lv < nv) {
#pragma unroll
          for (int a = 0; a < 3; ++a) ve[3 * j + a] = vs[3 * lv + a];
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a) ve[3 * j + a] = v[3 * vi[j] + a];
        }
      }
      double f[12];
      elem_hv<TH>(H, H + 45, ve, f);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int lv = vi[j] - v0;
        if (lv >= 0 && lv < nv) {
#pragma unroll
          for (int a = 0; a < 3; ++a) acc_term<DET>(win, aux, 3 * lv + a, f[3 * j + a], pass);
        }
      }
    }
    const int c0 = rc_off[r], c1 = rc_off[r + 1];
    for (int w = c0 + threadIdx.x; w < c1; w += blockDim.x) {
      const int64_t i = rc_list[w];
      const int4 iv = reinterpret_cast<const int4*>(bidx)[i];
      const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
      double uu[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) uu[q] = bu[12 * i + q];
      double s = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (vi[j] < 0) continue;
        const int lv = vi[j] - v0;
        const bool own = lv >= 0 && lv < nv;
#pragma unroll
        for (int a = 0; a < 3; ++a) s += uu[3 * j + a] * (own ? vs[3 * lv + a] : v[3 * vi[j] + a]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int lv = vi[j] - v0;
        if (vi[j] >= 0 && lv >= 0 && lv < nv) {
#pragma unroll
          for (int a = 0; a < 3; ++a) acc_term<DET>(win, aux, 3 * lv + a, s * uu[3 * j + a], pass);
        }
      }
    }
    __syncthreads();
    if (DET) {
      for (int e = threadIdx.x; e < 3 * nv; e += blockDim.x) {
        if (pass == 0) fx_mid(&win[e], &aux[e]);
        else win[e] = fx_get(&win[e], &aux[e]);
      }
      __syncthreads();
    }
    }  // passes
    for (int e = threadIdx.x; e < 3 * nv; e += blockDim.x) {
      const int64_t q = 3 * int64_t(v0) + e;
      y[q] = mass[q / 3] * vs[e] + win[e];
    }
    __syncthreads();
  }
}

// rank-one stencil columns: y += u (u^T v), scattered through an LDS window
// (columns in the order given; sorted by smallest vertex they stay local)
__global__ __launch_bounds__(256) void k_hv_cols(int64_t N, int64_t m, const int32_t* idx, const double* u,
                                                 const double* dS, const double* v, double* y) {
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
    if (!(dS[i] > 0.0)) continue;  // zero column (not stored)
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

// Deterministic mode: y[3 v + a] += (u_c . v) u_c[3 j + a] over the
// incidences (c, j) of vertex v in ascending order (lists built from the
// update columns with dS > 0).
__global__ __launch_bounds__(256) void k_hv_cols_gather(int64_t N, const int32_t* off, const int32_t* list,
                                                        const int32_t* idx, const double* u, const double* v,
                                                        double* y) {
  const int64_t vv = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (vv >= N) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = off[vv]; q < off[vv + 1]; ++q) {
    const int64_t slot = list[q];
    const int64_t ci = slot >> 2;
    const int j = int(slot & 3);
    const int4 iv = reinterpret_cast<const int4*>(idx)[ci];
    const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (vi[k] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) w += u[12 * ci + 3 * k + a] * v[3 * int64_t(vi[k]) + a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] += w * u[12 * ci + 3 * j + a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) y[3 * vv + a] += acc[a];
}

template <bool DET>
static void launch_hv_range(Ctx& c, const double* v, double* y) {
  const int64_t grid = std::min<int64_t>(c.nrange, int64_t(c.n_cu));
  if (c.hr32)
    k_hv_range<float, DET><<<dim3(grid), dim3(hv_threads<float>()), 0, c.s>>>(
        c.nrange, c.rbeg, c.rt_off, c.rl_tv, c.hr32, c.bidx, c.bu, c.rc_off, c.rc_list, c.mass, v, y, c.ctr, c.err);
  else
    k_hv_range<double, DET><<<dim3(grid), dim3(hv_threads<double>()), 0, c.s>>>(
        c.nrange, c.rbeg, c.rt_off, c.rl_tv, c.hr64, c.bidx, c.bu, c.rc_off, c.rc_list, c.mass, v, y, c.ctr, c.err);
}

mas_status launch_hessvec(Ctx& c, const double* v, double* y, int with_update) {
  ProfScope ps(c, MAS_T_HESSVEC);
  k_set_u32<<<dim3(1), dim3(1), 0, c.s>>>(c.ctr, 0u);
  {
    ProfScope pt(c, MAS_T_HV_TETS);
    if (c.cfg.deterministic) launch_hv_range<true>(c, v, y);
    else launch_hv_range<false>(c, v, y);
  }
  if (with_update && c.have_update && c.mc > 0) {
    if (c.cfg.deterministic) {
      mas_status st = build_incidence(c, c.mc, c.Uidx, c.dS);
      if (st != MAS_OK) return st;
      k_hv_cols_gather<<<dim3((c.N + 255) / 256), dim3(256), 0, c.s>>>(c.N, c.inc_off, c.inc_list, c.Uidx, c.U, v,
                                                                        y);
    } else {
      k_hv_cols<<<dim3((c.mc + SW_CHUNK - 1) / SW_CHUNK), dim3(256), 0, c.s>>>(c.N, c.mc, c.Uidx, c.U, c.dS, v,
                                                                                y);
    }
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
