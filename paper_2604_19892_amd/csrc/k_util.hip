// Bucketing of contact stencils into per-subdomain and per-range lists, and
// the exclusive prefix sum they are built with.
#include <algorithm>

#include "kernels.hpp"

namespace mas {

// buckets (map ? map[v] : v / div) of the vertices j of stencil i with bit j
// of pm[i] set; returns the count and writes them to out[4]
__device__ inline int stencil_buckets(int div, const int32_t* map, int64_t i, const int32_t* idx, const uint8_t* pm,
                                      int out[4]) {
  int n = 0;
  const unsigned mask = pm[i];
  if (mask == 0u) return 0;
  const int4 iv = reinterpret_cast<const int4*>(idx)[i];
  const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = vi[j];
    if (v < 0 || !((mask >> j) & 1u)) continue;
    const int d = map ? map[v] : v / div;
    bool dup = false;
    for (int q = 0; q < n; ++q) dup |= (out[q] == d);
    if (!dup) out[n++] = d;
  }
  return n;
}

// Counting and filling aggregate over the workgroup: each of its (up to
// 4 x 256) bucket keys goes into an LDS hash table by linear probing, which
// gives the key's slot and the item's rank among the workgroup's items of
// that bucket; one global atomic per distinct key then adds the slot's
// count (count pass) or reserves its run of list positions (fill pass).
// Stencils arrive sorted by their smallest vertex, so the keys of a
// stencil's other vertices are scattered; a per-key loop over the
// wavefront would serialise on them.
constexpr int BK_T = 256;
constexpr int BK_HASH = 2048;  // > 4 keys x 256 items: at most half full

__device__ inline int bk_slot(int* hkey, int key) {
  int h = int((uint32_t(key) * 2654435761u) >> 21) & (BK_HASH - 1);
  while (true) {
    const int old = atomicCAS(&hkey[h], -1, key);
    if (old == -1 || old == key) return h;
    h = (h + 1) & (BK_HASH - 1);
  }
}

__global__ __launch_bounds__(BK_T) void k_bucket_count(int div, const int32_t* map, int64_t m, const int32_t* idx,
                                                       const uint8_t* pm, int32_t* cnt) {
  __shared__ int hkey[BK_HASH];
  __shared__ int hcnt[BK_HASH];
  for (int q = threadIdx.x; q < BK_HASH; q += BK_T) {
    hkey[q] = -1;
    hcnt[q] = 0;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * int64_t(BK_T) + threadIdx.x;
  int b[4];
  const int n = (i < m) ? stencil_buckets(div, map, i, idx, pm, b) : 0;
  for (int q = 0; q < n; ++q) atomicAdd(&hcnt[bk_slot(hkey, b[q])], 1);
  __syncthreads();
  for (int q = threadIdx.x; q < BK_HASH; q += BK_T)
    if (hkey[q] >= 0) atomicAdd(&cnt[hkey[q]], hcnt[q]);
}

__global__ __launch_bounds__(BK_T) void k_bucket_fill(int div, const int32_t* map, int64_t m, const int32_t* idx,
                                                      const uint8_t* pm, int32_t* cursor, int32_t* list) {
  __shared__ int hkey[BK_HASH];
  __shared__ int hcnt[BK_HASH];
  for (int q = threadIdx.x; q < BK_HASH; q += BK_T) {
    hkey[q] = -1;
    hcnt[q] = 0;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * int64_t(BK_T) + threadIdx.x;
  int b[4], slot[4], rank[4];
  const int n = (i < m) ? stencil_buckets(div, map, i, idx, pm, b) : 0;
  for (int q = 0; q < n; ++q) {
    slot[q] = bk_slot(hkey, b[q]);
    rank[q] = atomicAdd(&hcnt[slot[q]], 1);
  }
  __syncthreads();
  // the run of each distinct key (hcnt now holds its first list position)
  for (int q = threadIdx.x; q < BK_HASH; q += BK_T)
    if (hkey[q] >= 0) hcnt[q] = atomicAdd(&cursor[hkey[q]], hcnt[q]);
  __syncthreads();
  for (int q = 0; q < n; ++q) list[hcnt[slot[q]] + rank[q]] = int32_t(i);
}

// The order of items inside a bucket follows the atomics of the fill pass;
// every consumer is order independent up to the rounding order of sums (Top-K
// ranks by a total order, block assembly adds with atomics).

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_copy_i32(const int32_t* src, int32_t* dst, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

void fill_f64(Ctx& c, double* p, int64_t n, double v) {
  if (n <= 0) return;
  k_fill_f64<<<dim3(std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, c.s>>>(p, n, v);
}

void fill_i32(Ctx& c, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return;
  k_fill_i32<<<dim3(std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, c.s>>>(p, n, v);
}

// ------------------------------------------------------------ prefix sums
// Exclusive scan of int32 counts in tiles of SCAN_N items: each tile is
// scanned in one workgroup (SCAN_IPT consecutive items per thread, thread
// totals scanned across the wavefront with shuffles, wavefront totals in
// LDS) and writes its total; the totals are scanned the same way
// (recursively) and added back.  Integer sums, so the result does not depend
// on any order.
constexpr int SCAN_T = 256, SCAN_IPT = 8, SCAN_N = SCAN_T * SCAN_IPT;

__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const int32_t* in, int32_t* out, int64_t n, int32_t* tsum) {
  __shared__ int32_t s[SCAN_N];
  __shared__ int32_t wsum[SCAN_T / 64];
  const int64_t base = int64_t(blockIdx.x) * SCAN_N;
  for (int q = threadIdx.x; q < SCAN_N; q += SCAN_T) {
    const int64_t i = base + q;
    s[q] = i < n ? in[i] : 0;
  }
  __syncthreads();
  int32_t loc[SCAN_IPT];
  int32_t tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) {
    loc[k] = tot;
    tot += s[threadIdx.x * SCAN_IPT + k];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = tot;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t u = __shfl_up(inc, o);
    if (lane >= o) inc += u;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t ex = inc - tot;
  for (int q = 0; q < w; ++q) ex += wsum[q];
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) s[threadIdx.x * SCAN_IPT + k] = ex + loc[k];
  if (threadIdx.x == SCAN_T - 1) tsum[blockIdx.x] = ex + tot;
  __syncthreads();
  for (int q = threadIdx.x; q < SCAN_N; q += SCAN_T) {
    const int64_t i = base + q;
    if (i < n) out[i] = s[q];
  }
}

__global__ void k_scan_add(int32_t* out, int64_t n, const int32_t* tsum) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) out[i] += tsum[i / SCAN_N];
}

int64_t scan_scratch_elems(int64_t n) {
  int64_t tot = 0;
  while (n > 1) {
    n = (n + SCAN_N - 1) / SCAN_N;
    tot += n + 64;
  }
  return tot + 64;
}

static void scan_rec(Ctx& c, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp) {
  const int64_t nb = (n + SCAN_N - 1) / SCAN_N;
  k_scan_tile<<<dim3(nb), dim3(SCAN_T), 0, c.s>>>(in, out, n, tmp);
  if (nb > 1) {
    scan_rec(c, tmp, tmp, nb, tmp + nb + 64);
    k_scan_add<<<dim3((n + 255) / 256), dim3(256), 0, c.s>>>(out, n, tmp);
  }
}

mas_status exclusive_scan_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n1) {
  if (n1 <= 0) return MAS_OK;
  if (n1 > c.scan_cap) return MAS_ERR_INVALID_ARG;
  scan_rec(c, in, out, n1, c.scan_tmp);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status bucket_stencils(Ctx& c, int div, const int32_t* map, int64_t D, int64_t m, const int32_t* idx,
                           const uint8_t* pm, int32_t* cnt, int32_t* off, int32_t* list) {
  fill_i32(c, cnt, D + 1, 0);
  if (m > 0) k_bucket_count<<<dim3((m + BK_T - 1) / BK_T), dim3(BK_T), 0, c.s>>>(div, map, m, idx, pm, cnt);
  mas_status st = exclusive_scan_i32(c, cnt, off, D + 1);
  if (st != MAS_OK) return st;
  if (m > 0) {
    // reuse cnt as the fill cursor
    k_copy_i32<<<dim3(std::min<int64_t>((D + 255) / 256, 4096)), dim3(256), 0, c.s>>>(off, cnt, D);
    k_bucket_fill<<<dim3((m + BK_T - 1) / BK_T), dim3(BK_T), 0, c.s>>>(div, map, m, idx, pm, cnt, list);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ------------------------------------------------- vertex incidence lists
// Deterministic mode: for every vertex v the slots 4 c + j of the stencils
// c (with w[c] > 0 when w is given) whose vertex j is v, in ascending order:
// counted with integer atomics, placed by an exclusive scan and a fill in
// atomic order, then each vertex's list sorted by its own thread (lists are
// short: the contacts of one vertex).
__global__ void k_inc_count(int64_t m, const int32_t* idx, const double* w, int32_t* cnt) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= 4 * m) return;
  const int v = idx[i];
  if (v >= 0 && (!w || w[i >> 2] > 0.0)) atomicAdd(&cnt[v], 1);
}

__global__ void k_inc_fill(int64_t m, const int32_t* idx, const double* w, int32_t* cursor, int32_t* list) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= 4 * m) return;
  const int v = idx[i];
  if (v >= 0 && (!w || w[i >> 2] > 0.0)) list[atomicAdd(&cursor[v], 1)] = int32_t(i);
}

__global__ void k_inc_sort(int64_t N, const int32_t* off, int32_t* list) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  const int b = off[v], e = off[v + 1];
  for (int q = b + 1; q < e; ++q) {
    const int32_t key = list[q];
    int p = q - 1;
    while (p >= b && list[p] > key) {
      list[p + 1] = list[p];
      --p;
    }
    list[p + 1] = key;
  }
}

mas_status build_incidence(Ctx& c, int64_t m, const int32_t* idx, const double* w) {
  if (m > c.cfg.max_contacts) return MAS_ERR_INVALID_ARG;
  fill_i32(c, c.inc_cnt, c.N + 1, 0);
  const dim3 g((4 * m + 255) / 256), b(256);
  if (m > 0) k_inc_count<<<g, b, 0, c.s>>>(m, idx, w, c.inc_cnt);
  mas_status st = exclusive_scan_i32(c, c.inc_cnt, c.inc_off, c.N + 1);
  if (st != MAS_OK) return st;
  if (m > 0) {
    k_copy_i32<<<dim3(std::min<int64_t>((c.N + 255) / 256, 4096)), b, 0, c.s>>>(c.inc_off, c.inc_cnt, c.N);
    k_inc_fill<<<g, b, 0, c.s>>>(m, idx, w, c.inc_cnt, c.inc_list);
    k_inc_sort<<<dim3((c.N + 255) / 256), b, 0, c.s>>>(c.N, c.inc_off, c.inc_list);
  }
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status bucket_by_subdomain(Ctx& c, int64_t m, const int32_t* idx, const uint8_t* pm, int32_t* cnt,
                               int32_t* off, int32_t* list) {
  return bucket_stencils(c, SUB, nullptr, c.lv[0].nsub, m, idx, pm, cnt, off, list);
}

}  // namespace mas
