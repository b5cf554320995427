// Bucketing of contact stencils into per-subdomain and per-range lists.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace mas {

// buckets (map ? map[v] : v / div) of the vertices of stencil i (w[i] > 0)
// whose part of vec12 is nonzero; returns the count and writes them to out[4]
__device__ inline int stencil_buckets(int div, const int32_t* map, int64_t i, const int32_t* idx, const double* w,
                                      const double* vec12, int out[4]) {
  int n = 0;
  if (!(w[i] > 0.0)) return 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = idx[4 * i + j];
    if (v < 0) continue;
    const double* u = vec12 + 12 * i + 3 * j;
    if (u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0) continue;
    const int d = map ? map[v] : v / div;
    bool dup = false;
    for (int q = 0; q < n; ++q) dup |= (out[q] == d);
    if (!dup) out[n++] = d;
  }
  return n;
}

// Counting and filling aggregate over the wavefront: lanes with the same
// bucket share one atomic (stencils arrive sorted by their smallest vertex,
// so neighbouring lanes mostly share buckets, which at coarse levels are
// few).  Every lane runs the loops, including those past the end.
__global__ __launch_bounds__(256) void k_bucket_count(int div, const int32_t* map, int64_t m, const int32_t* idx, const double* w,
                                                      const double* vec12, int32_t* cnt) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  int b[4];
  const int n = (i < m) ? stencil_buckets(div, map, i, idx, w, vec12, b) : 0;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int key = q < n ? b[q] : -1;
    while (true) {
      const unsigned long long act = __ballot(key >= 0);
      if (act == 0) break;
      const int leader = __ffsll(act) - 1;
      const int lk = __shfl(key, leader);
      const unsigned long long match = __ballot(key == lk);
      if (lane == leader) atomicAdd(&cnt[lk], __popcll(match));
      if (key == lk) key = -1;
    }
  }
}

__global__ __launch_bounds__(256) void k_bucket_fill(int div, const int32_t* map, int64_t m, const int32_t* idx, const double* w,
                                                     const double* vec12, int32_t* cursor, int32_t* list) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  int b[4];
  const int n = (i < m) ? stencil_buckets(div, map, i, idx, w, vec12, b) : 0;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int key = q < n ? b[q] : -1;
    while (true) {
      const unsigned long long act = __ballot(key >= 0);
      if (act == 0) break;
      const int leader = __ffsll(act) - 1;
      const int lk = __shfl(key, leader);
      const unsigned long long match = __ballot(key == lk);
      int base = 0;
      if (lane == leader) base = atomicAdd(&cursor[lk], __popcll(match));
      base = __shfl(base, leader);
      if (key == lk) {
        list[base + __popcll(match & below)] = int32_t(i);
        key = -1;
      }
    }
  }
}

// The order of items inside a bucket follows the atomics of the fill pass;
// every consumer is order independent up to the rounding order of sums (Top-K
// ranks by a total order, block assembly adds with atomics).

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

mas_status ensure_cub(Ctx& c, size_t bytes) {
  if (bytes <= c.cub_bytes) return MAS_OK;
  if (c.cub_tmp) HIPCHK(hipFree(c.cub_tmp));
  c.cub_tmp = nullptr;
  c.cub_bytes = 0;
  if (hipMalloc(&c.cub_tmp, bytes) != hipSuccess) return MAS_ERR_OOM;
  c.cub_bytes = bytes;
  return MAS_OK;
}

mas_status exclusive_scan_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n1) {
  size_t bytes = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, int(n1), c.s));
  mas_status st = ensure_cub(c, bytes);
  if (st != MAS_OK) return st;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(c.cub_tmp, bytes, in, out, int(n1), c.s));
  return MAS_OK;
}

mas_status bucket_stencils(Ctx& c, int div, const int32_t* map, int64_t D, int64_t m, const int32_t* idx, const double* w,
                           const double* vec12, int32_t* cnt, int32_t* off, int32_t* list) {
  HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (D + 1), c.s));
  if (m > 0) {
    int bs = 256;
    int64_t gs = (m + bs - 1) / bs;
    k_bucket_count<<<dim3(gs), dim3(bs), 0, c.s>>>(div, map, m, idx, w, vec12, cnt);
  }
  size_t bytes = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, cnt, off, int(D + 1), c.s));
  mas_status st = ensure_cub(c, bytes);
  if (st != MAS_OK) return st;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(c.cub_tmp, bytes, cnt, off, int(D + 1), c.s));
  if (m > 0) {
    // reuse cnt as the fill cursor
    HIPCHK(hipMemcpyAsync(cnt, off, sizeof(int32_t) * D, hipMemcpyDeviceToDevice, c.s));
    int bs = 256;
    int64_t gs = (m + bs - 1) / bs;
    k_bucket_fill<<<dim3(gs), dim3(bs), 0, c.s>>>(div, map, m, idx, w, vec12, cnt, list);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status bucket_by_subdomain(Ctx& c, int64_t m, const int32_t* idx, const double* w, const double* vec12,
                               int32_t* cnt, int32_t* off, int32_t* list) {
  return bucket_stencils(c, SUB, nullptr, c.lv[0].nsub, m, idx, w, vec12, cnt, off, list);
}

}  // namespace mas
