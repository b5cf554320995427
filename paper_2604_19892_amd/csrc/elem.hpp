// Per-tetrahedron device math: deformation gradient, stable Neo-Hookean
// energy / stress / tangent, the PSD projection of the 9x9 tangent, and the
// products of the frozen element Hessian with vectors.
//
// Conventions.  F = Ds Dm^-1 with Ds = [x1-x0, x2-x0, x3-x0] (columns).
// vec(F) is column-major: entry (a,b) sits at 3b + a.  The 9x9 tangent is
// stored packed symmetric (45 entries, index p9).  Dm^-1 is row-major.
#pragma once

#include "common.hpp"

namespace mas {

struct M3 {
  double m[3][3];
};

__device__ inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// F[a][b] = sum_c (x_{c+1} - x_0)[a] Dminv[c][b]
__device__ inline void def_grad(const double* xe /*12*/, const double* Dmi /*9*/, double F[3][3]) {
  double ds[3][3];  // ds[c][a]
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) ds[c][a] = xe[3 * (c + 1) + a] - xe[a];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      F[a][b] = ds[0][a] * Dmi[0 * 3 + b] + ds[1][a] * Dmi[1 * 3 + b] + ds[2][a] * Dmi[2 * 3 + b];
}

__device__ inline double det3(const double F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
         F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// cofactor dJ/dF as columns: cof[:,0] = f1 x f2, cof[:,1] = f2 x f0, cof[:,2] = f0 x f1
__device__ inline void cofactor3(const double F[3][3], double C[3][3]) {
  double f0[3] = {F[0][0], F[1][0], F[2][0]};
  double f1[3] = {F[0][1], F[1][1], F[2][1]};
  double f2[3] = {F[0][2], F[1][2], F[2][2]};
  double c0[3], c1[3], c2[3];
  cross3(f1, f2, c0);
  cross3(f2, f0, c1);
  cross3(f0, f1, c2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C[a][0] = c0[a];
    C[a][1] = c1[a];
    C[a][2] = c2[a];
  }
}

// Psi(F) = mu/2 (tr F^T F - 3) - mu (J - 1) + lam/2 (J - 1)^2
__device__ inline double snh_energy(const double F[3][3], double mu, double lam) {
  double ic = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ic += F[a][b] * F[a][b];
  double J = det3(F);
  return 0.5 * mu * (ic - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) * (J - 1.0);
}

// P = mu F + (lam (J-1) - mu) cof(F)
__device__ inline void snh_stress(const double F[3][3], double mu, double lam, double P[3][3]) {
  double C[3][3];
  cofactor3(F, C);
  double s = lam * (det3(F) - 1.0) - mu;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) P[a][b] = mu * F[a][b] + s * C[a][b];
}

// Lower-triangle of d2Psi/dF2 = mu I + lam g g^T + (lam (J-1) - mu) d2J/dF2,
// g = vec(cof F).  d2J/dF2 couples column blocks b != b' through the skew
// matrix of the third column: block(0,1) = -[f2]x, block(0,2) = [f1]x,
// block(1,2) = -[f0]x (and the transposes).
__device__ inline void snh_tangent(const double F[3][3], double mu, double lam, double H[45]) {
  double C[3][3];
  cofactor3(F, C);
  double g[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) g[3 * b + a] = C[a][b];
  double s = lam * (det3(F) - 1.0) - mu;
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) H[p9(i, j)] = lam * g[i] * g[j] + (i == j ? mu : 0.0);
  // skew blocks: [a]x (r,c) entries: (0,1)=-a2 (0,2)=a1 (1,0)=a2 (1,2)=-a0 (2,0)=-a1 (2,1)=a0
  // block(bi,bj) for bi>bj in the lower triangle:
  //   (1,0) =  [f2]x, (2,0) = -[f1]x, (2,1) = [f0]x
  const double f[3][3] = {{F[0][0], F[1][0], F[2][0]}, {F[0][1], F[1][1], F[2][1]},
                          {F[0][2], F[1][2], F[2][2]}};
  auto add_skew = [&](int bi, int bj, const double* a, double sign) {
    double S[3][3] = {{0, -a[2], a[1]}, {a[2], 0, -a[0]}, {-a[1], a[0], 0}};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) H[p9(3 * bi + r, 3 * bj + c)] += s * sign * S[r][c];
  };
  add_skew(1, 0, f[2], 1.0);
  add_skew(2, 0, f[1], -1.0);
  add_skew(2, 1, f[0], 1.0);
}

// One Jacobi rotation of a symmetric 3x3 A zeroing A[P][Q]; V accumulates
// the rotations (columns are eigenvectors).
template <int P, int Q>
__device__ __forceinline__ void jacobi3_rot(double (&A)[3][3], double (&V)[3][3]) {
  constexpr int R = 3 - P - Q;
  const double apq = A[P][Q];
  if (apq == 0.0) return;
  const double theta = (A[Q][Q] - A[P][P]) / (2.0 * apq);
  const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0);
  const double sn = t * c;
  A[P][P] -= t * apq;
  A[Q][Q] += t * apq;
  A[P][Q] = A[Q][P] = 0.0;
  const double arp = A[R][P], arq = A[R][Q];
  A[R][P] = A[P][R] = c * arp - sn * arq;
  A[R][Q] = A[Q][R] = sn * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vkp = V[k][P], vkq = V[k][Q];
    V[k][P] = c * vkp - sn * vkq;
    V[k][Q] = sn * vkp + c * vkq;
  }
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi: on return the diagonal
// of A holds the eigenvalues and V the eigenvectors (columns).
__device__ inline void jacobi3(double (&A)[3][3], double (&V)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (!(off > 1e-36 * dia)) break;
    jacobi3_rot<0, 1>(A, V);
    jacobi3_rot<0, 2>(A, V);
    jacobi3_rot<1, 2>(A, V);
  }
}

// Givens rotation on rows P, Q of B zeroing B[Q][C] (B[P][C] >= 0 after);
// U accumulates the transposed rotations so that U B stays invariant.
template <int P, int Q, int C>
__device__ __forceinline__ void givens3(double (&B)[3][3], double (&U)[3][3]) {
  const double a = B[P][C], b = B[Q][C];
  const double r = sqrt(a * a + b * b);
  const double c = (r > 0.0) ? a / r : 1.0, sn = (r > 0.0) ? b / r : 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double bp = B[P][k], bq = B[Q][k];
    B[P][k] = c * bp + sn * bq;
    B[Q][k] = -sn * bp + c * bq;
    const double up = U[k][P], uq = U[k][Q];
    U[k][P] = c * up + sn * uq;
    U[k][Q] = -sn * up + c * uq;
  }
}

// Rotation-variant SVD F = U diag(sig) V^T with U, V proper rotations and
// sig[0] >= sig[1] >= |sig[2]|, sig[2] < 0 for inverted F: V from the
// eigenvectors of F^T F, then U and sig from a Givens QR of F V (the diagonal
// of R; it carries the sign of det F), following McAdams et al. (2011).
__device__ inline void svd3_rv(const double (&F)[3][3], double (&U)[3][3], double (&sig)[3], double (&V)[3][3]) {
  double S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
  jacobi3(S, V);
  double ev[3] = {S[0][0], S[1][1], S[2][2]};
  auto cswap = [&](int i, int j) {
    if (ev[i] < ev[j]) {
      const double e = ev[i];
      ev[i] = ev[j];
      ev[j] = e;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double v = V[k][i];
        V[k][i] = V[k][j];
        V[k][j] = v;
      }
    }
  };
  cswap(0, 1);
  cswap(0, 2);
  cswap(1, 2);
  const double dv = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                    V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                    V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
  if (dv < 0.0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k][2] = -V[k][2];
  }
  double B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[i][j] = (i == j) ? 1.0 : 0.0;
  givens3<0, 1, 0>(B, U);
  givens3<0, 2, 0>(B, U);
  givens3<1, 2, 1>(B, U);
  sig[0] = B[0][0];
  sig[1] = B[1][1];
  sig[2] = B[2][2];
}

// H -= lam q q^T (packed 9x9)
__device__ __forceinline__ void sub_rank1_9(double (&H)[45], double lam, const double (&q)[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) H[p9(i, j)] -= lam * q[i] * q[j];
}

// The SNH tangent with its negative eigenvalues clamped to zero.  Its
// eigenvectors are known in closed form from the rotation-variant SVD of F
// (Smith, de Goes and Kim 2019): for each axis k a twist and a flip mode
// (u_i v_j^T -/+ u_j v_i^T)/sqrt2 with eigenvalues mu + s sig_k and
// mu - s sig_k, s = lam (J - 1) - mu, and three scaling modes
// sum_i w_i u_i v_i^T from the 3x3 matrix mu I + lam d d^T + s d2J/dsig2.
// The clamped tangent is the full tangent minus its negative modes.
__device__ inline void snh_tangent_psd(const double F[3][3], double mu, double lam, double (&H)[45]) {
  snh_tangent(F, mu, lam, H);
  const double (&Fr)[3][3] = *reinterpret_cast<const double(*)[3][3]>(F);
  double U[3][3], V[3][3], sg[3];
  svd3_rv(Fr, U, sg, V);
  const double s = lam * (det3(F) - 1.0) - mu;
  const double r2 = 0.70710678118654752440;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    const double et = mu + s * sg[k], ef = mu - s * sg[k];
    if (et < 0.0) {
      double q[9];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) q[3 * b + a] = r2 * (U[a][i] * V[b][j] - U[a][j] * V[b][i]);
      sub_rank1_9(H, et, q);
    }
    if (ef < 0.0) {
      double q[9];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) q[3 * b + a] = r2 * (U[a][i] * V[b][j] + U[a][j] * V[b][i]);
      sub_rank1_9(H, ef, q);
    }
  }
  const double d[3] = {sg[1] * sg[2], sg[0] * sg[2], sg[0] * sg[1]};
  double A3[3][3], W[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A3[i][j] = lam * d[i] * d[j] + (i == j ? mu : s * sg[3 - i - j]);
  jacobi3(A3, W);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double e = A3[m][m];
    if (e < 0.0) {
      double q[9];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          q[3 * b + a] = W[0][m] * U[a][0] * V[b][0] + W[1][m] * U[a][1] * V[b][1] + W[2][m] * U[a][2] * V[b][2];
      sub_rank1_9(H, e, q);
    }
  }
}

// f = B^T Hf B v for one tet.  Hf: 45 packed entries (already scaled by
// h^2 V_e), Dmi: Dm^-1 row-major, v: 12 values (4 vertex triples).
template <typename TH>
__device__ inline void elem_hv(const TH* Hf, const TH* Dmi, const double* v, double* f) {
  double w[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double acc = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc += (v[3 * (c + 1) + a] - v[a]) * double(Dmi[3 * c + b]);
      w[3 * b + a] = acc;
    }
  double t[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double acc = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) acc += double(Hf[p9(i, j)]) * w[j];
    t[i] = acc;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s0 = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) acc += t[3 * b + a] * double(Dmi[3 * c + b]);
      f[3 * (c + 1) + a] = acc;
      s0 += acc;
    }
    f[a] = -s0;
  }
}

// coef[j][b] = d F_ab / d x_{j,a}
__device__ inline void dfdx_coef(const double* Dmi, double coef[4][3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    coef[1][b] = Dmi[0 * 3 + b];
    coef[2][b] = Dmi[1 * 3 + b];
    coef[3][b] = Dmi[2 * 3 + b];
    coef[0][b] = -(coef[1][b] + coef[2][b] + coef[3][b]);
  }
}

// 3x3 block (i,j) of the 12x12 element Hessian B^T Hf B:
// out[a][a'] = sum_{b,b'} coef[i][b] Hf(3b+a, 3b'+a') coef[j][b']
__device__ inline void elem_block(const double* Hf, const double coef[4][3], int i, int j,
                                  double out[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int ap = 0; ap < 3; ++ap) {
      double acc = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int bp = 0; bp < 3; ++bp) acc += coef[i][b] * Hf[p9(3 * b + a, 3 * bp + ap)] * coef[j][bp];
      out[a][ap] = acc;
    }
}

// barrier b(d) = -(d - dhat)^2 ln(d/dhat) on 0 < d < dhat and derivatives
__device__ inline void barrier3(double d, double dhat, double* b, double* b1, double* b2) {
  if (d > 0.0 && d < dhat) {
    double r = d - dhat;
    double L = log(d / dhat);
    *b = -r * r * L;
    *b1 = -2.0 * r * L - r * r / d;
    *b2 = -2.0 * L - 4.0 * r / d + (r * r) / (d * d);
  } else {
    *b = 0.0;
    *b1 = 0.0;
    *b2 = 0.0;
  }
}

}  // namespace mas
