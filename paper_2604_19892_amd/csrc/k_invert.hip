// Inversion of the MAS subdomain blocks on the matrix cores (FP64 MFMA).
//
// Each 96x96 symmetric positive definite block (the Schwarz subdomain matrix
// S_d (C H C^T) S_d^T of a level, supplement Eqs. (1)-(4)) is inverted by one
// wavefront with the blocked symmetric sweep operator (Goodnight 1979):
// sweeping the 16x16 pivot block K of A maps
//   A_KK -> -A_KK^-1,  A_KI -> A_KK^-1 A_KI,  A_IJ -> A_IJ - A_IK A_KK^-1 A_KJ,
// and after the six pivot blocks the matrix is -A^-1.  The pivot block enters
// through its Cholesky factor A_KK = L L^T and G = L^-1: with Z_I = G A_KI,
// the update is the Gram product Z_I^T Z_J, the new row K is G^T Z_I and the
// pivot block -G^T G.  (Forming A_KK^-1 explicitly and multiplying by it
// loses about four more digits on blocks with condition numbers near 1e11,
// which stiff barrier contacts produce; the Gram form keeps the scalar
// sweep's accuracy.)  The block is scaled to unit diagonal first and held
// negated (T = -A), so every product accumulates with a plus sign and T ends
// as the inverse.  The 21 tiles of the block (the six diagonal tiles in full,
// one orientation of each off-diagonal pair) stay in the wavefront's
// registers from load to store; the products are v_mfma_f64_16x16x4f64; L^-1
// comes from one elimination pass over [A_KK | I] with lane broadcasts.
#include "kernels.hpp"

namespace mas {

typedef double d4 __attribute__((ext_vector_type(4)));

// A 16x16 tile in accumulator layout: lane l = c + 16 q (c = l & 15,
// q = l >> 4) holds the entries (q + 4 v, c), v = 0..3.  In that layout a
// tile Z is the B operand of the 16x16x4 product for k = 4 s..4 s + 3 as its
// element s, and the A operand of Z^T likewise, so
//   tmul(Y, Z, acc) = acc + Y^T Z
// needs no data movement.
__device__ __forceinline__ d4 tmul(const d4 Y, const d4 Z, d4 acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[0], Z[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[1], Z[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[2], Z[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[3], Z[3], acc, 0, 0, 0);
  return acc;
}

// Lane reads and broadcasts of doubles: readlane (wave-uniform result) and
// the DPP row broadcast row_newbcast:P (lane c + 16 q receives lane P + 16 q).
__device__ __forceinline__ double read_lane(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}
template <int P>
__device__ __forceinline__ double row_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + P, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + P, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(a): the hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double a) {
  double r = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}

// G = L^-1 for the Cholesky factor L L^T = X of a symmetric positive
// definite 16x16 tile (accumulator layout), by eliminating on [X | I] with
// L^-1 from the left: pivot p divides row p by sqrt(x_pp) and takes
// (x_rp / x_pp) row p from every row r > p, on both halves; the left half
// ends as L^T, the right half (G, identity on entry) as L^-1.  The first
// pivot that is not positive and finite goes to *bad / *badv.
template <int P>
__device__ __forceinline__ void chol_inv_pivot(d4& X, d4& G, int c, int q, int* bad, double* badv) {
  // rows q + 4 v: all above the pivot for v < vp (untouched), all below it
  // for v > vp, and row P itself or rows on either side for v = vp
  constexpr int vp = P >> 2, qp = P & 3;
  const double app = read_lane(X[vp], P + 16 * qp);
  const double ax = __shfl(X[vp], c + 16 * qp);  // row P of the left half
  const double ag = __shfl(G[vp], c + 16 * qp);  // row P of the right half
  const bool first_bad = *bad < 0 && !(app > 0.0 && isfinite(app));
  *badv = first_bad ? app : *badv;
  *bad = first_bad ? P : *bad;
  const double rs = rsqrt_nr(app), ia = rs * rs;
#pragma unroll
  for (int v = vp; v < 4; ++v) {
    const double f = row_bcast<P>(X[v]) * ia;  // x_rP / x_PP
    const double xn = fma(-f, ax, X[v]);
    const double gn = fma(-f, ag, G[v]);
    if (v == vp) {
      X[v] = q == qp ? ax * rs : (q > qp ? xn : X[v]);
      G[v] = q == qp ? ag * rs : (q > qp ? gn : G[v]);
    } else {
      X[v] = xn;
      G[v] = gn;
    }
  }
}

template <int P = 0>
__device__ __forceinline__ void chol_inv16(d4& X, d4& G, int c, int q, int* bad, double* badv) {
  chol_inv_pivot<P>(X, G, c, q, bad, badv);
  if constexpr (P < 15) chol_inv16<P + 1>(X, G, c, q, bad, badv);
}

constexpr int TPAD = 17;  // LDS row of a tile (16 + 1 against bank conflicts)

__device__ __forceinline__ void tile_put(double* buf, const d4& Y, int c, int q) {
#pragma unroll
  for (int v = 0; v < 4; ++v) buf[(q + 4 * v) * TPAD + c] = Y[v];
}
// the transpose of the tile put into buf, in accumulator layout
__device__ __forceinline__ d4 tile_get_t(const double* buf, int c, int q) {
  d4 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r[v] = buf[c * TPAD + q + 4 * v];
  return r;
}

// the stored image of a 32- or 16-bit block, staged in LDS
constexpr int IMG_DOUBLES = int(blk_elems(MAS_F32) * 4 / 8);
static_assert(blk_elems(MAS_BF16) * 2 <= blk_elems(MAS_F32) * 4, "16-bit image fits the 32-bit one");
static_assert(6 * 16 * TPAD <= IMG_DOUBLES, "transpose buffers fit the image space");

template <int P>
__device__ __forceinline__ void store_entry(unsigned char* slot, int i, int j, double val) {
  const int pos = blk_pos(P, i, j);
  if constexpr (P == MAS_F64) reinterpret_cast<double*>(slot)[pos] = val;
  else if constexpr (P == MAS_F32) reinterpret_cast<float*>(slot)[pos] = float(val);
  else if constexpr (P == MAS_BF16) reinterpret_cast<uint16_t*>(slot)[pos] = f32_to_bf16(float(val));
  else reinterpret_cast<uint16_t*>(slot)[pos] = f32_to_f16(float(val));
}

// Final tiles (every off-diagonal pair in its lower orientation) to the
// stored layout of the block products; 16-bit storage keeps
// B_ij / (sig_i sig_j).
template <int P>
__device__ __forceinline__ void store_block(unsigned char* slot, const d4 (&T)[6][6], const double* sc,
                                            const float* sig, int c, int q) {
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const int j = 16 * a + c;
    const double scj = sc[j];
    const double gj = (P == MAS_BF16 || P == MAS_F16) ? double(sig[j]) : 1.0;
#pragma unroll
    for (int b = a; b < 6; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * b + q + 4 * v;
        if (b == a && i < j) continue;
        double val = T[a][b][v] * sc[i] * scj;
        if constexpr (P == MAS_BF16 || P == MAS_F16) val /= double(sig[i]) * gj;
        store_entry<P>(slot, i, j, val);
      }
    }
  }
}

// State of the factorization of a pivot block in progress: left half X,
// right half G (identity on entry), first failing pivot.
struct Factor {
  d4 X, G;
  int bad;
  double badv;
};

__device__ __forceinline__ Factor factor_begin(const d4& TKK, int c, int q) {
  Factor f;
  f.X = -TKK;
#pragma unroll
  for (int v = 0; v < 4; ++v) f.G[v] = (q + 4 * v == c) ? 1.0 : 0.0;
  f.bad = -1;
  f.badv = 0.0;
  return f;
}

// The tile products of step K after the pivot block of step K + 1: item n
// of the update T_IJ += Z_I^T Z_J over the pairs I <= J outside row and
// column K (row-major, the pair (K + 1, K + 1) excluded, it comes first),
// then the five tiles G^T Z_I of row K, then G^T G.
constexpr int upd_count(int K) { return K < 5 ? 14 : 15; }
constexpr int upd_pair(int K, int n, bool want_j) {
  int m = 0;
  for (int I = 0; I < 6; ++I) {
    if (I == K) continue;
    for (int J = I; J < 6; ++J) {
      if (J == K || (I == K + 1 && J == K + 1)) continue;
      if (m == n) return want_j ? J : I;
      ++m;
    }
  }
  return -1;
}
constexpr int panel_index(int K, int n) { return n < K ? n : n + 1; }  // the n-th I != K

template <int K, int N>
__device__ __forceinline__ void step_item(d4 (&T)[6][6], const d4 (&Z)[6], const d4& G, Factor& f, int c,
                                          int q) {
  constexpr int NU = upd_count(K);
  const d4 zero = {0.0, 0.0, 0.0, 0.0};
  if constexpr (N < NU) {
    constexpr int I = upd_pair(K, N, false), J = upd_pair(K, N, true);
    // a pair {I, J} (I < J) is held as (J, I) once step J has passed
    if constexpr (J == I) T[I][I] = tmul(Z[I], Z[I], T[I][I]);
    else if constexpr (K > J) T[I][J] = tmul(Z[J], Z[I], T[I][J]);
    else T[I][J] = tmul(Z[I], Z[J], T[I][J]);
  } else if constexpr (N < NU + 5) {
    constexpr int I = panel_index(K, N - NU);
    if constexpr (I < K) T[I][K] = tmul(G, Z[I], zero);
    else T[K][I] = tmul(G, Z[I], zero);
  } else {
    T[K][K] = tmul(G, G, zero);
  }
  if constexpr (K < 5 && N < 16) {
    chol_inv_pivot<N>(f.X, f.G, c, q, &f.bad, &f.badv);
    // issue order: each of the item's four products followed by a share of
    // the pivot's lane exchanges and arithmetic, so the wave issues them
    // while the matrix unit works (a wave issues in order, and a run of
    // products would hold it until the last one starts)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x080, 2, 0);  // LDS exchanges
      __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);  // VALU
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (N < NU + 5) step_item<K, N + 1>(T, Z, G, f, c, q);
}

// Sweep of pivot block K (see the top of the file), given G = L^-1 of its
// pivot block.  Tiles of pairs {a, K}, a < K, turn to orientation (K, a)
// first, through LDS.  The pivot block of step K + 1 is updated first; its
// 16 elimination pivots are then issued one after each independent tile
// product of the rest of the step, so that the lane exchanges and the
// scalar chain of the factorization run beside the matrix products.
template <int K>
__device__ __forceinline__ void sweep_step(d4 (&T)[6][6], d4& G, double (*tb)[16 * TPAD], int c, int q,
                                           int* bad, double* badv) {
  if constexpr (K > 0) {
#pragma unroll
    for (int a = 0; a < K; ++a) tile_put(tb[a + 1], T[a][K], c, q);
  }
  tile_put(tb[0], G, c, q);
  __syncthreads();
  if constexpr (K > 0) {
#pragma unroll
    for (int a = 0; a < K; ++a) T[a][K] = tile_get_t(tb[a + 1], c, q);
  }
  const d4 GT = tile_get_t(tb[0], c, q);
  __syncthreads();
  const d4 zero = {0.0, 0.0, 0.0, 0.0};
  // Z_I = G T_KI for the panel tiles (orientation (K, I))
  d4 Z[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    if (I == K) continue;
    Z[I] = tmul(GT, I < K ? T[I][K] : T[K][I], zero);
  }
  Factor f;
  if constexpr (K < 5) {
    T[K + 1][K + 1] = tmul(Z[K + 1], Z[K + 1], T[K + 1][K + 1]);
    f = factor_begin(T[K + 1][K + 1], c, q);
  }
  step_item<K, 0>(T, Z, G, f, c, q);
  if constexpr (K < 5) {
    const bool first = *bad < 0 && f.bad >= 0;
    *badv = first ? f.badv : *badv;
    *bad = first ? 16 * (K + 1) + f.bad : *bad;
    G = f.G;
  }
}

template <int P = 0>
__device__ __forceinline__ void factor_all(Factor& f, int c, int q) {
  chol_inv_pivot<P>(f.X, f.G, c, q, &f.bad, &f.badv);
  if constexpr (P < 15) factor_all<P + 1>(f, c, q);
}

// One wavefront per block, two wavefronts per SIMD (the 21 tiles need about
// 170 of a wave's 256 registers; the compiler keeps the rest of the working
// set within the limit with a few hundred bytes of spills outside the sweep,
// which stay in the caches: 1.44 ms instead of 1.92 ms at one wave per SIMD
// for the 35,625 level-0 blocks of the puffer scene, the second wave issuing
// while the first waits on its lane exchanges).  One launch covers the
// levels [lo, hi), the highest first.  acc: the packed lower float64 blocks
// of each level (rows and columns of nodes beyond the node count are
// identity).  Stored in the requested precision, or a wider one when
// kappa = max_i M_ii B_ii exceeds guard / (20 eps) (the spectral norm of the
// rounding error of a unit-diagonal 96x96 matrix is about 20 eps, and
// 1/kappa bounds its smallest eigenvalue from above).  With acc_next, the
// sum of all 3x3 node blocks of the block (before inversion) becomes the
// diagonal block of node d at the next level (C_(l+1) sums the nodes of d).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_invert_mfma(InvLevels iv, double guard,
                                                                                             uint32_t* err, DiagRec* dg) {
  // transposes during the steps; the stored image of a 32- or 16-bit block
  // at the end
  __shared__ __align__(16) double lds[IMG_DOUBLES];
  double(*tb)[16 * TPAD] = reinterpret_cast<double(*)[16 * TPAD]>(lds);
  __shared__ double sc[BD];
  __shared__ float sig[BD];
  // block -> (level, subdomain): levels hi - 1, ..., lo
  int level = iv.lo;
  int64_t d = blockIdx.x;
  for (int q = iv.hi - 1; q > iv.lo; --q) {
    if (d < iv.nsub[q]) {
      level = q;
      break;
    }
    d -= iv.nsub[q];
  }
  const int64_t nodes = iv.nodes[level];
  const int req = iv.prec[level];
  uint8_t* bprec = iv.bprec[level];
  float* scale = iv.scale[level];
  double* acc_next = iv.acc_next;
  const int l = threadIdx.x, c = l & 15, q = l >> 4;
  const double* src = iv.acc[level] + d * PK;
  const int nv = 3 * int(min<int64_t>(SUB, nodes - SUB * d));  // rows of real nodes
  d4 T[6][6];
  // node-bin sums of the raw block: row bin (a + v + q) mod 3, column bin
  // (b + c) mod 3; kept by (a + v) mod 3 and b mod 3 (compile-time), the
  // lane's q and c are added at the end
  double sD[3][3], sO[3][3];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int w = 0; w < 3; ++w) sD[u][w] = sO[u][w] = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * a + q + 4 * v, j = 16 * b + c;
        const double x = (i < nv && j < nv) ? src[i >= j ? pk(i, j) : pk(j, i)] : 0.0;
        T[a][b][v] = x;
        if (b == a) sD[(a + v) % 3][b % 3] += x;
        else sO[(a + v) % 3][b % 3] += x;
      }
  if (acc_next) {
    double s9[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) s9[t] = 0.0;
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        const int x = (u + q) % 3, y = (w + c) % 3;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          if (t == 3 * x + y) s9[t] += sD[u][w] + sO[u][w];
          if (t == 3 * y + x) s9[t] += sO[u][w];
        }
      }
#pragma unroll
    for (int t = 0; t < 9; ++t) s9[t] = wave_sum(s9[t]);
    const int ln = int(d & 31);
#pragma unroll
    for (int t = 0; t < 9; ++t)
      if (l == t && t / 3 >= t % 3) acc_next[(d >> 5) * PK + pk(3 * ln + t / 3, 3 * ln + t % 3)] = s9[t];
  }
  // identity on padded rows; unit-diagonal scaling sc_i = a_ii^-1/2
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (q + 4 * v == c) {
        const int i = 16 * a + c;
        if (i >= nv) T[a][a][v] = 1.0;
        sc[i] = 1.0 / sqrt(T[a][a][v]);
      }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double si = sc[16 * a + q + 4 * v];
#pragma unroll
      for (int b = a; b < 6; ++b) T[a][b][v] *= -si * sc[16 * b + c];
    }
  int bad = -1;
  double badv = 0.0;
  Factor f0 = factor_begin(T[0][0], c, q);
  factor_all(f0, c, q);
  bad = f0.bad;
  badv = f0.badv;
  d4 G = f0.G;
  sweep_step<0>(T, G, tb, c, q, &bad, &badv);
  sweep_step<1>(T, G, tb, c, q, &bad, &badv);
  sweep_step<2>(T, G, tb, c, q, &bad, &badv);
  sweep_step<3>(T, G, tb, c, q, &bad, &badv);
  sweep_step<4>(T, G, tb, c, q, &bad, &badv);
  sweep_step<5>(T, G, tb, c, q, &bad, &badv);
  if (bad >= 0 && l == 0) {
    atomicOr(err, ERRB_NOT_SPD);
    diag_report(dg + level, level == 0 ? 1 : 2, level, d, bad, badv);
  }
  // T = S^-1 of the scaled block S; kappa = max_i of its diagonal
  double kap = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (q + 4 * v == c) kap = fmax(kap, T[a][a][v]);
  for (int o = 32; o > 0; o >>= 1) kap = fmax(kap, __shfl_xor(kap, o));
  int P = req;
  while (guard > 0.0 && P != MAS_F64 && !(kap <= guard / (20.0 * prec_eps(P))))
    P = (P == MAS_F32) ? MAS_F64 : MAS_F32;
  if (l == 0) bprec[d] = uint8_t(P);
  unsigned char* slot = reinterpret_cast<unsigned char*>(iv.blk[level]) + d * BLK_STRIDE;
  if (P == MAS_BF16 || P == MAS_F16) {
    // sig_i = sqrt(B_ii), B_ii = T_ii sc_i^2
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (q + 4 * v == c) {
          const int i = 16 * a + c;
          const float s = float(sqrt(T[a][a][v] * sc[i] * sc[i]));
          sig[i] = s;
          scale[d * BD + i] = s;
        }
    __syncthreads();
  }
  if (P == MAS_F64) {
    store_block<MAS_F64>(slot, T, sc, sig, c, q);
    return;
  }
  // 32- and 16-bit blocks: the image in LDS (the transpose buffers are free
  // after the last step's barrier), then 16-byte stores of the whole slot
  unsigned char* img = reinterpret_cast<unsigned char*>(lds);
  switch (P) {
    case MAS_F32: store_block<MAS_F32>(img, T, sc, sig, c, q); break;
    case MAS_BF16: store_block<MAS_BF16>(img, T, sc, sig, c, q); break;
    default: store_block<MAS_F16>(img, T, sc, sig, c, q);
  }
  __syncthreads();
  const int n16 = int(blk_elems(P) * prec_size(P) / 16);
  const float4* src4 = reinterpret_cast<const float4*>(lds);
  float4* dst4 = reinterpret_cast<float4*>(slot);
  for (int k = l; k < n16; k += 64) st_once(dst4 + k, src4[k]);
}

void launch_invert_mfma(Ctx& c, int lo, int hi, double* acc_next) {
  InvLevels iv{};
  iv.lo = lo;
  iv.hi = hi;
  iv.acc_next = acc_next;
  int64_t nb = 0;
  for (int l = lo; l < hi; ++l) {
    const Level& Lv = c.lv[l];
    iv.nsub[l] = Lv.nsub;
    iv.nodes[l] = Lv.nodes;
    iv.acc[l] = Lv.acc;
    iv.blk[l] = Lv.blk;
    iv.scale[l] = Lv.scale;
    iv.bprec[l] = Lv.bprec;
    iv.prec[l] = Lv.prec;
    nb += Lv.nsub;
  }
  if (nb > 0) k_invert_mfma<<<dim3(nb), dim3(64), 0, c.s>>>(iv, c.cfg.prec_guard, c.err, c.diag);
}

}  // namespace mas
