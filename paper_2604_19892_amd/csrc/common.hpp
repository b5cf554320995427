// Shared types of the MAS-PNCG HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <cmath>

#include <vector>

#include "maspncg.h"

namespace mas {

constexpr int SUB = 32;                 // vertices (nodes) per subdomain
constexpr int BD = 96;                  // block dimension (3 DOFs x 32)
constexpr int PK = BD * (BD + 1) / 2;   // packed lower-triangular entries (4656)
constexpr int MAXL = 6;                 // maximum MAS levels
constexpr int MAXK = 32;                // maximum Woodbury rank per subdomain
constexpr int MAX_SCENES = 1024;        // scenes of one context (batched form)
constexpr int SAFE_ROUNDS = 16;         // safe-step damping rounds (device side, no host sync)
constexpr int EH = 54;                  // per-tet snapshot: 45 (9x9 packed) + 9 (Dm^-1)
constexpr int TILE = 64;                // tets per AoSoA tile (one wavefront)
// Vertex ranges of the owner-computes products: range r owns the vertices
// [rbeg[r], rbeg[r+1]) (at most RANGE_MAX of them) and writes their outputs
// without atomics.  Ranges are cut so that each is touched by about
// RANGE_TETS tets; resident workgroups take ranges from a counter until all
// are done.
constexpr int RANGE_MAX = 2048;
constexpr int RANGE_TETS = 4096;
constexpr int SNAP_NC64 = EH / 2;       // 16-byte chunks per float64 snapshot (27)
constexpr int SNAP_NC32 = (EH + 3) / 4; // 16-byte chunks per float32 snapshot (14, 2 entries padding)

// sticky device error bits
constexpr uint32_t ERRB_NOT_SPD = 1u;
constexpr uint32_t ERRB_NONFINITE = 2u;
constexpr uint32_t ERRB_RANK = 4u;
constexpr uint32_t ERRB_INDEX = 8u;  // a pair named a vertex id outside [0, N)

// packed lower-triangular index, i >= j
__host__ __device__ inline int pk(int i, int j) { return i * (i + 1) / 2 + j; }
__host__ __device__ inline int pks(int i, int j) { return i >= j ? pk(i, j) : pk(j, i); }

// symmetric 9x9 packed index (upper storage is the same as lower by symmetry)
__host__ __device__ inline constexpr int p9(int i, int j) {
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

__host__ __device__ inline constexpr size_t prec_size(int p) {
  return p == MAS_F64 ? 8 : (p == MAS_F32 ? 4 : 2);
}
// elements per stored block: packed size rounded up to a 256-byte multiple
__host__ __device__ inline constexpr size_t blk_elems(int p) {
  return (PK + 256 / prec_size(p) - 1) / (256 / prec_size(p)) * (256 / prec_size(p));
}

// every block occupies a slot of the float64 size; its stored precision is
// recorded per block
constexpr size_t BLK_STRIDE = blk_elems(MAS_F64) * 8;

// Data streamed once per pass in whole-wavefront pieces (stored blocks,
// element snapshots, rest geometry) is loaded and stored with the non-temporal
// hint, so the stream does not displace the vectors that are gathered
// through the caches.
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 ld_once(const uint2* p) {
  const nt_u2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p));
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_once(const float4* p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_once(const double2* p) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_once(uint2* p, uint2 v) {
  __builtin_nontemporal_store(nt_u2{v.x, v.y}, reinterpret_cast<nt_u2*>(p));
}
__device__ __forceinline__ void st_once(float4* p, float4 v) {
  __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_f4*>(p));
}
__device__ __forceinline__ void st_once(double2* p, double2 v) {
  __builtin_nontemporal_store(nt_d2{v.x, v.y}, reinterpret_cast<nt_d2*>(p));
}

// Element snapshot layout (45 packed tangent entries, then Dm^-1): per tile
// of 64 tets, 16-byte chunk c of every tet of the tile lies contiguously
// (chunk-major, then tet), so a wavefront reads one chunk of 64 tets as one
// 1 KiB access.
// NT = false: plain loads, for gathers of scattered entries whose cache
// lines other threads of the workgroup may read next.
template <bool NT = true>
__device__ __forceinline__ void snap_load(const double* hf, int64_t t, double (&e)[EH]) {
  const double2* p = reinterpret_cast<const double2*>(hf) + (t / TILE) * (SNAP_NC64 * TILE) + (t % TILE);
#pragma unroll
  for (int c = 0; c < SNAP_NC64; ++c) {
    const double2 v = NT ? ld_once(p + c * TILE) : p[c * TILE];
    e[2 * c] = v.x;
    e[2 * c + 1] = v.y;
  }
}
template <bool NT = true>
__device__ __forceinline__ void snap_load(const float* hf, int64_t t, float (&e)[4 * SNAP_NC32]) {
  const float4* p = reinterpret_cast<const float4*>(hf) + (t / TILE) * (SNAP_NC32 * TILE) + (t % TILE);
#pragma unroll
  for (int c = 0; c < SNAP_NC32; ++c) {
    const float4 v = NT ? ld_once(p + c * TILE) : p[c * TILE];
    e[4 * c] = v.x;
    e[4 * c + 1] = v.y;
    e[4 * c + 2] = v.z;
    e[4 * c + 3] = v.w;
  }
}

// Per-tet rest data (Dm^-1 row-major, V, mu, lam): 12 doubles in the same
// chunked tile layout (6 chunks of 2).
constexpr int GEO_NC = 6;
__device__ __forceinline__ void geo_load(const double* geo, int64_t t, double (&g)[12]) {
  const double2* p = reinterpret_cast<const double2*>(geo) + (t / TILE) * (GEO_NC * TILE) + (t % TILE);
#pragma unroll
  for (int c = 0; c < GEO_NC; ++c) {
    const double2 v = ld_once(p + c * TILE);
    g[2 * c] = v.x;
    g[2 * c + 1] = v.y;
  }
}
__device__ __forceinline__ void geo_store(double* geo, int64_t t, const double (&g)[12]) {
  double2* p = reinterpret_cast<double2*>(geo) + (t / TILE) * (GEO_NC * TILE) + (t % TILE);
#pragma unroll
  for (int c = 0; c < GEO_NC; ++c) p[c * TILE] = make_double2(g[2 * c], g[2 * c + 1]);
}

// Stored block layout.  A symmetric 96x96 block is cut into 6x6 tiles: the
// 120 tiles (bi, bj), bi > bj, numbered t = bi (bi - 1) / 2 + bj with their 36
// entries row-major, and the 16 diagonal tiles in pairs (2m, 2m + 1) with 21
// packed-lower entries each, numbered t = 120 + m.  A block product runs 128
// threads, thread t on tile t.  Each tile's entries are cut into 8-byte
// units; unit k of the 64 tiles of a wavefront are stored next to each other,
// so every unit is one contiguous 512-byte access.  The diagonal pairs (lanes
// 56..63 of the second wavefront) have a few more units, stored last.
constexpr int NTILE = 128;
__host__ __device__ inline constexpr int tile_epu(int P) { return 8 / int(prec_size(P)); }
__host__ __device__ inline constexpr int tile_uo(int P) { return 36 / tile_epu(P); }
__host__ __device__ inline constexpr int tile_ud(int P) { return (42 + tile_epu(P) - 1) / tile_epu(P); }
__host__ __device__ inline constexpr int blk_positions(int P) {
  return (128 * tile_uo(P) + 8 * (tile_ud(P) - tile_uo(P))) * tile_epu(P);
}
// index of unit k of tile t
__host__ __device__ inline int tile_unit(int P, int t, int k) {
  const int uo = tile_uo(P);
  if (t < 64) return k * 64 + t;
  if (k < uo) return 64 * uo + k * 64 + (t - 64);
  return 128 * uo + (k - uo) * 8 + (t - 120);
}
// row/column tile of off-diagonal tile t < 120
__host__ __device__ inline void tile_rc(int t, int& bi, int& bj) {
  bi = 1;
  while ((bi + 1) * bi / 2 <= t) ++bi;
  bj = t - bi * (bi - 1) / 2;
}
// storage position (in entries) of A(i, j)
__host__ __device__ inline int blk_pos(int P, int i, int j) {
  if (i < j) {
    const int x = i;
    i = j;
    j = x;
  }
  const int bi = i / 6, bj = j / 6, r = i % 6, q = j % 6;
  int t, e;
  if (bi > bj) {
    t = bi * (bi - 1) / 2 + bj;
    e = 6 * r + q;
  } else {
    t = 120 + bi / 2;
    e = 21 * (bi & 1) + r * (r + 1) / 2 + q;
  }
  const int epu = tile_epu(P);
  return tile_unit(P, t, e / epu) * epu + e % epu;
}
// the entry (i >= j) held at storage position pos; false for padding
__host__ __device__ inline bool blk_entry_of(int P, int pos, int& i, int& j) {
  const int epu = tile_epu(P), uo = tile_uo(P);
  const int u = pos / epu, sub = pos % epu;
  int t, k;
  if (u < 64 * uo) {
    t = u % 64;
    k = u / 64;
  } else if (u < 128 * uo) {
    t = 64 + (u - 64 * uo) % 64;
    k = (u - 64 * uo) / 64;
  } else {
    t = 120 + (u - 128 * uo) % 8;
    k = uo + (u - 128 * uo) / 8;
  }
  int e = k * epu + sub;
  if (t < 120) {
    int bi, bj;
    tile_rc(t, bi, bj);
    i = 6 * bi + e / 6;
    j = 6 * bj + e % 6;
    return true;
  }
  if (e >= 42) return false;
  const int b = 2 * (t - 120) + (e >= 21 ? 1 : 0);
  if (e >= 21) e -= 21;
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  i = 6 * b + r;
  j = 6 * b + e - r * (r + 1) / 2;
  return true;
}

static_assert(blk_positions(MAS_F64) <= int(blk_elems(MAS_F64)) && blk_positions(MAS_F32) <= int(blk_elems(MAS_F32)) &&
                  blk_positions(MAS_BF16) <= int(blk_elems(MAS_BF16)),
              "tiled blocks fit their slots");

// unit roundoff of each storage format
__host__ __device__ inline constexpr double prec_eps(int p) {
  return p == MAS_F64 ? 1.1102230246251565e-16
                      : (p == MAS_F32 ? 5.9604644775390625e-08 : (p == MAS_F16 ? 4.8828125e-04 : 3.90625e-03));
}

// ------------------------------------------------------------ 16-bit floats
// bfloat16: upper half of an IEEE binary32; rounding to nearest even.
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);  // inf / nan
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}
__host__ __device__ inline float f16_to_f32(uint16_t h) {
  _Float16 v;
  memcpy(&v, &h, 2);
  return float(v);
}
__host__ __device__ inline uint16_t f32_to_f16(float f) {
  _Float16 v = _Float16(f);
  uint16_t h;
  memcpy(&h, &v, 2);
  return h;
}

// positive doubles order like their bit patterns: atomic min through uint64
__device__ inline void atomic_min_pos(double* a, double v) {
  atomicMin(reinterpret_cast<unsigned long long*>(a), (unsigned long long)__double_as_longlong(v));
}

// Bit j set when vertex j of a stencil carries a nonzero part of its
// 12-vector u (the bucket passes then read one byte instead of u).
__device__ inline uint8_t part_mask(const double (&u)[12]) {
  uint8_t pm = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (u[3 * j] != 0.0 || u[3 * j + 1] != 0.0 || u[3 * j + 2] != 0.0) pm |= uint8_t(1u << j);
  return pm;
}

// first device-side failure of one source, written once (source: 1 level-0
// build, 2 coarse build, 3 capacitance).  The context holds DIAG_SLOTS of
// them: slot l for the blocks of level l, slot MAXL for the capacitance, so
// that a failure of a level-0 block is reported before the coarse failures
// it causes, whichever block reached its record first.
struct DiagRec {
  uint32_t flag;
  int32_t source;
  int32_t level;
  int32_t step;
  int64_t index;
  double value;
};

constexpr int DIAG_SLOTS = MAXL + 1;

__device__ inline void diag_report(DiagRec* dg, int source, int level, int64_t index, int step,
                                   double value) {
  if (!dg) return;
  if (atomicCAS(&dg->flag, 0u, 1u) == 0u) {
    dg->source = source;
    dg->level = level;
    dg->index = index;
    dg->step = step;
    dg->value = value;
  }
}

// Logical workgroup index for L2 locality: workgroups are dealt to the
// eight XCDs (each with its own L2) in turn, so workgroup b runs on XCD
// b mod 8.  This bijection of [0, G) gives every XCD a contiguous run of
// logical indices, so neighbouring work that reads the same cache lines
// (gathers of shared vertices, entries of one vertex range) meets in one L2
// instead of fetching the lines once per XCD.
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
  const int64_t q = G / NXCD, r = G % NXCD, x = b % NXCD, k = b / NXCD;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Base-key table: linear probing from a SplitMix64-finalised hash (Steele,
// Lea and Flood 2014; the finaliser constants as Vigna published them).
constexpr uint64_t HKEY_EMPTY = ~uint64_t(0);
__host__ __device__ inline uint64_t key_hash(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

struct SlotCol {        // one column of U_d restricted to its subdomain
  int32_t lv[4];        // local vertex (0..31) of each stencil vertex, -1 if outside
  double u[12];
};

struct Level {
  int64_t nodes = 0;    // level-l nodes (level 0: vertices)
  int64_t nsub = 0;     // D_l
  int prec = MAS_F64;      // requested storage precision
  void* blk = nullptr;     // nsub slots of BLK_STRIDE bytes
  uint8_t* bprec = nullptr;  // stored precision of each block
  float* scale = nullptr;  // nsub * 96 row scales (16-bit storage)
  double* acc = nullptr;   // packed FP64 assembly of every block of the level
  double* r = nullptr;     // restricted residual 3*nodes (levels >= 1)
  double* c = nullptr;     // coarse correction 3*nodes (levels >= 1)
};

struct Prof;  // host-side kernel timers (api.hip)

struct Ctx {
  hipStream_t s = nullptr;
  Prof* prof = nullptr;
  mas_config cfg{};
  int64_t N = 0, T = 0, Tpad = 0;
  int n_cu = 256;                  // compute units of the device
  int L = 1, K = 8;
  Level lv[MAXL];

  // mesh, library order
  int32_t* tets = nullptr;     // 4T
  double* geo = nullptr;       // 12T: Dm^-1 (9, row-major), vol, mu, lam
  double* mass = nullptr;      // N
  int32_t* tet_off = nullptr;  // D0+1, level-0 subdomain d -> its tet records [tet_off[d], tet_off[d+1])
  int32_t* l0_tv = nullptr;    // 4 per record: the vertices of a tet touching the subdomain
  int32_t* l0_home = nullptr;  // per record: the range entry holding that tet's home snapshot copy
  int rmax = 0;                // largest range (vertices)
  int64_t nrange = 0;          // vertex ranges
  int32_t* rbeg = nullptr;     // nrange+1 range starts
  int32_t* vrange = nullptr;   // N: range of each vertex
  uint32_t* ctr = nullptr;     // work counters of the range kernels (4)
  int32_t* rt_off = nullptr;   // nrange+1, range -> its entries [rt_off[r], rt_off[r+1])
  int64_t nent = 0, nent_pad = 0;  // entries: (range, tet touching it), range-major
  int32_t* rl_t = nullptr;     // tet of each entry, bit 31 set on the entry of its smallest vertex's range
  int32_t* rl_tv = nullptr;    // 4 vertices of the entry's tet
  double* rl_geo = nullptr;    // rest data per entry (chunked tile layout over entries)
  double* hr64 = nullptr;      // element snapshot per entry, float64 Hessian storage
  float* hr32 = nullptr;       // element snapshot per entry, float32 Hessian storage

  bool built = false;

  // base contact set (capacity cfg.max_contacts, allocated at create)
  int64_t mb = 0, mb_cap = 0;
  uint64_t* bkey = nullptr;        // mb, input order
  uint64_t* hkey = nullptr;        // hcap: open-addressing table of the base keys (HKEY_EMPTY: free)
  int32_t* hval = nullptr;         // hcap: base index of each stored key
  int64_t hcap = 0;                // allocated slots: a power of two, at least twice max_contacts
  int64_t hsize = 1024;            // slots in use: a power of two, at least twice the base contacts
  double* bk = nullptr;            // mb stiffness
  uint8_t* bpm = nullptr;          // mb: bit j set when vertex j carries a nonzero part of bgrad and k > 0
  double* bgrad = nullptr;         // 12 mb
  int32_t* bidx = nullptr;         // 4 mb
  double* bu = nullptr;            // 12 mb, sqrt(k) n
  int32_t* bc_cnt = nullptr;       // D0
  int32_t* bc_off = nullptr;       // D0+1
  int32_t* bc_list = nullptr;      // 4 mb
  int32_t* rc_cnt = nullptr;       // nrange+1: range -> base stencils touching it
  int32_t* rc_off = nullptr;
  int32_t* rc_list = nullptr;      // 4 mb

  // current update (untruncated U) and the localized Woodbury data
  // (capacity cfg.max_contacts)
  int64_t mc = 0, mc_cap = 0;
  double* U = nullptr;             // 12 mc
  int32_t* Uidx = nullptr;         // 4 mc
  double* dS = nullptr;            // mc
  uint8_t* upm = nullptr;          // mc: bit j set when vertex j carries a nonzero part of U (dS > 0)
  uint64_t* ckey = nullptr;        // mc
  int32_t* cand_cnt = nullptr;     // D0
  int32_t* cand_off = nullptr;     // D0+1
  int32_t* cand_list = nullptr;    // 4 mc
  int32_t* rank = nullptr;         // D0
  int32_t* sel = nullptr;          // D0*K
  SlotCol* slots = nullptr;        // D0*K
  double* W = nullptr;             // D0*K*96, float64
  double* Lcap = nullptr;          // D0*K*(K+1)/2
  bool have_update = false;

  // scenes of the batched form: library vertex -> scene, the first vertex
  // range of each scene (ranges are cut at scene starts), per-scene scratch
  int S = 1;
  std::vector<int64_t> scene_v;  // host, S + 1 library vertex offsets
  int32_t* seg = nullptr;        // N
  int64_t* scene_r = nullptr;    // S + 1
  double* sc_acc = nullptr;      // 8 S

  // 3x3 block-Jacobi comparison preconditioner (precond = MAS_PRECOND_BJ3):
  // per vertex the packed lower 3x3 block of H~ (6 doubles) and its inverse
  double* bj = nullptr;            // 6N
  double* bjinv = nullptr;         // 6N

  // scratch
  double* partials = nullptr;      // reductions
  int n_partial_blocks = 1024;
  double* scal = nullptr;          // small device scalars (mu, nu, ...)
  double* fixed_ws = nullptr;      // this device's address of the library's fixed workspace array
  double* alpha = nullptr;         // D0, step sizes of the last safe step
  double* alpha0 = nullptr;        // D0, step sizes before damping
  double* alpha_mix = nullptr;     // D0, step sizes safe for any mix of steps (fallback)
  uint64_t* ahalf = nullptr;       // D0, bit r: subdomain halved in damping round r
  uint32_t* around = nullptr;      // SAFE_ROUNDS violation counts of the damping rounds
  uint32_t* err = nullptr;         // sticky error bits
  DiagRec* diag = nullptr;         // DIAG_SLOTS first-failure records
  mas_iter_stats* stats = nullptr; // per-iteration counters (device)
  // deterministic mode: vertex incidence lists of a stencil set (for
  // each vertex its (stencil, slot) pairs 4 c + j in ascending order) and
  // the deep-level coupling blocks of every level-0 subdomain
  int32_t* inc_cnt = nullptr;      // N + 1 counts, then fill cursors
  int32_t* inc_off = nullptr;      // N + 1
  int32_t* inc_list = nullptr;     // 4 max_contacts
  double* coup = nullptr;          // D0 x (L - 2) x 32 x 9 (levels >= 2), when L > 2
  int32_t* cls_part = nullptr;     // branch counts of the classification, 5 per workgroup
  int64_t cls_blocks = 0;          // workgroups of the last classification
  int32_t* scan_tmp = nullptr;     // block sums of the exclusive scans
  int64_t scan_cap = 0;            // longest scan the scratch serves

  // broad phase of the contact set: one spatial hash table per primitive
  // kind (triangles, edges), sized at create for cfg.max_tris / max_edges
  struct CellTable {
    int32_t* cnt = nullptr;  // H + 1 bucket counts, then fill cursors
    int32_t* off = nullptr;  // H + 1 bucket offsets
    uint64_t* key = nullptr; // entries: cell key
    int32_t* id = nullptr;   // entries: primitive index
    int64_t h_cap = 0, e_cap = 0;
  } cs[2];
  unsigned long long* cs_misc = nullptr;  // [0] largest primitive extent (bits), [1] pair count
};

// Scatter through an LDS window.  A workgroup handles a chunk of items
// sorted by their smallest vertex; vertices in [vbase, vbase + SW_WIN) are
// accumulated in LDS, the others (and finally the window) are added to the
// global vector with atomics, which cuts global atomics several-fold.
constexpr int SW_WIN = 1024;

constexpr int SW_CHUNK = 1024;

// (the two branches use different atomic scopes so that they stay an LDS
// atomic and a global atomic rather than being merged into one generic one)
__device__ __forceinline__ void sw_add(double* win, double* y, int vbase, int v, int a, double val) {
  const int lv = v - vbase;
  if (lv >= 0 && lv < SW_WIN)
    __hip_atomic_fetch_add(&win[3 * lv + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_fetch_add(&y[3 * int64_t(v) + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void sw_flush(const double* win, double* y, int vbase, int64_t N) {
  for (int e = threadIdx.x; e < 3 * SW_WIN; e += blockDim.x) {
    const double val = win[e];
    if (val != 0.0 && int64_t(vbase) + e / 3 < N) atomicAdd(&y[3 * int64_t(vbase) + e], val);
  }
}

// Orders the LDS accesses of one wavefront's lanes at this point: a
// wavefront's LDS operations execute in program order, so it is enough that
// the compiler moves no memory access across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront aggregation of atomics: lanes whose key matches the lowest
// pending lane's key combine their values (one shuffle reduction per
// distinct key) and only that lane issues the atomic.  Every lane of the
// wavefront must call these together (uniform control flow); key < 0 marks
// a lane with nothing to add.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// atomic min of a positive double per key (address addr of the leader)
__device__ __forceinline__ void wave_min_pos(long long key, double* addr, double val) {
  const int lane = threadIdx.x & 63;
  bool pending = key >= 0;
  while (true) {
    const unsigned long long act = __ballot(pending);
    if (act == 0) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const long long lk = __shfl(key, leader);
    const bool mine = pending && key == lk;
    const double m = wave_min(mine ? val : INFINITY);
    if (lane == leader) atomic_min_pos(addr, m);
    if (mine) pending = false;
  }
}

// ------------------------------------------------------ deterministic sums
// Order-independent accumulation (deterministic mode).  A sum whose terms
// arrive through atomics in no fixed order is taken in two passes over the
// same terms.  Pass 0 records per destination entry the largest |term| (the
// bits of a non-negative double order like its value) and the number of
// terms; from these the entry's quantum 2^e is the power of two with
// max * count < 2^(62 + e), so every partial sum fits an int64.  Pass 1 adds
// each term rounded once to a multiple of 2^e, as an integer: integer
// addition is associative, so the result is the same whatever order the
// atomics take.  The error of an entry is at most count^2 * max * 2^-62, no
// more than float64 accumulation's own worst case (count^2 * max * 2^-53
// relative to the partial sums).  An entry that saw a non-finite term
// reads back as NaN.
constexpr int FX_NONFINITE = -100000;  // exponent marker of an entry with a non-finite term

__device__ __forceinline__ void fx_note(double* slot, int* cnt, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(slot), (unsigned long long)__double_as_longlong(fabs(v)));
  atomicAdd(cnt, 1);
}
// after pass 0: the entry's exponent (stored over its count); the slot is
// cleared to an integer zero
__device__ __forceinline__ void fx_mid(double* slot, int* cnt) {
  const unsigned long long bits = *reinterpret_cast<unsigned long long*>(slot);
  const double mx = __longlong_as_double((long long)bits);
  int e = 0;
  if (!isfinite(mx)) {
    e = FX_NONFINITE;
  } else if (mx > 0.0) {
    frexp(mx * double(*cnt), &e);  // mx * cnt < 2^e
    e -= 62;
  }
  *cnt = e;
  *reinterpret_cast<long long*>(slot) = 0;
}
__device__ __forceinline__ void fx_add(double* slot, const int* ex, double v) {
  if (*ex == FX_NONFINITE) return;
  atomicAdd(reinterpret_cast<unsigned long long*>(slot), (unsigned long long)llrint(ldexp(v, -*ex)));
}
__device__ __forceinline__ double fx_get(const double* slot, const int* ex) {
  if (*ex == FX_NONFINITE) return NAN;
  return ldexp(double(*reinterpret_cast<const long long*>(slot)), *ex);
}
// one term into an LDS accumulator: plain float atomics (fast mode) or the
// pass of the two-pass fixed-point sum (DET)
template <bool DET>
__device__ __forceinline__ void acc_term(double* win, int* aux, int e, double v, int pass) {
  if constexpr (!DET) {
    atomicAdd(&win[e], v);
  } else {
    if (pass == 0) fx_note(&win[e], &aux[e], v);
    else fx_add(&win[e], &aux[e], v);
  }
}

// Records a HIP event pair around its scope when timers are enabled.
void prof_begin(Ctx& c, int timer);
void prof_end(Ctx& c, int timer);
struct ProfScope {
  Ctx& c;
  int t;
  ProfScope(Ctx& c_, int t_) : c(c_), t(t_) { prof_begin(c, t); }
  ~ProfScope() { prof_end(c, t); }
};

}  // namespace mas

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return MAS_ERR_HIP;         \
  } while (0)
