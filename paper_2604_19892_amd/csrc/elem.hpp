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

// Clamp the eigenvalues of a symmetric 9x9 matrix (packed) at zero, in
// place.  Cyclic Jacobi rotations (Golub & Van Loan, Sec. 8.5) accumulate the
// eigenvectors; the projection V max(Lambda, 0) V^T is rebuilt from them.
__device__ inline void psd_project9(double A[45]) {
  double V[9][9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  double fro = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) fro += (i == j ? 1.0 : 2.0) * A[p9(i, j)] * A[p9(i, j)];
  const double tol = 1e-30 * fro;
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) off += A[p9(i, j)] * A[p9(i, j)];
    if (off <= tol) break;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
#pragma unroll
      for (int q = p + 1; q < 9; ++q) {
        double apq = A[p9(p, q)];
        if (apq != 0.0) {
          double theta = (A[p9(q, q)] - A[p9(p, p)]) / (2.0 * apq);
          double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          double c = 1.0 / sqrt(t * t + 1.0);
          double s = t * c;
          A[p9(p, p)] -= t * apq;
          A[p9(q, q)] += t * apq;
          A[p9(p, q)] = 0.0;
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            if (k == p || k == q) continue;
            double akp = A[p9(k, p)], akq = A[p9(k, q)];
            A[p9(k, p)] = c * akp - s * akq;
            A[p9(k, q)] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
      }
    }
  }
  double lam[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) lam[i] = fmax(A[p9(i, i)], 0.0);
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double acc = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc += V[i][k] * lam[k] * V[j][k];
      A[p9(i, j)] = acc;
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
