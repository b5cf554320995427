// Setup kernels: element rest quantities and lumped masses, the inertial
// target x~ and affine stencil distances.
#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

// Dm = [X1-X0, X2-X0, X3-X0]; Dm^-1 rows are the cross products of its
// columns over det(Dm); V = det/6; mu, lam from Young's modulus and Poisson's
// ratio; tmass[t] = rho V / 4, the share each of its vertices receives.
__global__ void k_rest(int64_t T, const int32_t* tets, const double* X, const double* rho,
                       const double* E, const double* nu, double* geo, double* tmass) {
  int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= T) return;
  int v[4];
  double p[4][3];
  for (int j = 0; j < 4; ++j) {
    v[j] = tets[4 * t + j];
    for (int a = 0; a < 3; ++a) p[j][a] = X[3 * v[j] + a];
  }
  double e1[3], e2[3], e3[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = p[1][a] - p[0][a];
    e2[a] = p[2][a] - p[0][a];
    e3[a] = p[3][a] - p[0][a];
  }
  double c23[3], c31[3], c12[3];
  cross3(e2, e3, c23);
  cross3(e3, e1, c31);
  cross3(e1, e2, c12);
  double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  double g[12];
  double id = 1.0 / det;
  for (int a = 0; a < 3; ++a) {
    g[0 * 3 + a] = c23[a] * id;
    g[1 * 3 + a] = c31[a] * id;
    g[2 * 3 + a] = c12[a] * id;
  }
  double vol = det / 6.0;
  double Ev = E[t], nv = nu[t];
  g[9] = vol;
  g[10] = Ev / (2.0 * (1.0 + nv));
  g[11] = Ev * nv / ((1.0 + nv) * (1.0 - 2.0 * nv));
  geo_store(geo, t, g);
  tmass[t] = rho[t] * vol * 0.25;
}

// Lumped mass of each vertex: the shares of its tets summed in ascending tet
// order (voff/vt: vertex -> touching tets), so the masses do not depend on
// the order in which threads run.
__global__ void k_lumped_mass(int64_t N, const int32_t* voff, const int32_t* vt, const double* tmass,
                              double* mass) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  double m = 0.0;
  for (int32_t q = voff[v]; q < voff[v + 1]; ++q) m += tmass[vt[q]];
  mass[v] = m;
}

// rest data copied to the range-major entries (padding entries zero)
__global__ void k_geo_entries(int64_t nent, int64_t nent_pad, const int32_t* rl_t, const double* geo,
                              double* rl_geo) {
  const int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (w >= nent_pad) return;
  double g[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) g[q] = 0.0;
  if (w < nent) geo_load(geo, rl_t[w] & 0x7fffffff, g);
  geo_store(rl_geo, w, g);
}

mas_status launch_rest(Ctx& c, const double* X, const double* rho, const double* E, const double* nu,
                       double* tmass, const int32_t* voff, const int32_t* vt) {
  int bs = 256;
  k_rest<<<dim3((c.T + bs - 1) / bs), dim3(bs), 0, c.s>>>(c.T, c.tets, X, rho, E, nu, c.geo, tmass);
  k_lumped_mass<<<dim3((c.N + bs - 1) / bs), dim3(bs), 0, c.s>>>(c.N, voff, vt, tmass, c.mass);
  k_geo_entries<<<dim3((c.nent_pad + bs - 1) / bs), dim3(bs), 0, c.s>>>(c.nent, c.nent_pad, c.rl_t, c.geo,
                                                                        c.rl_geo);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

__global__ void k_inertial(int64_t n3, const double* xt, const double* vt, double h, double g0,
                           double g1, double g2, double* out) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  int a = int(i % 3);
  double g = a == 0 ? g0 : (a == 1 ? g1 : g2);
  out[i] = xt[i] + h * vt[i] + h * h * g;
}

mas_status launch_inertial(Ctx& c, const double* xt, const double* vt, double* xtil) {
  int64_t n3 = 3 * c.N;
  int bs = 256;
  k_inertial<<<dim3((n3 + bs - 1) / bs), dim3(bs), 0, c.s>>>(
      n3, xt, vt, c.cfg.h, c.cfg.gravity[0], c.cfg.gravity[1], c.cfg.gravity[2], xtil);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// implicit Euler: v = (x_new - x_old) / h, x~ = x_new + h v + h^2 g
__global__ void k_next_frame(int64_t n3, const double* xn, const double* xo, double h, double g0, double g1,
                             double g2, double* v, double* xtil) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  const int a = int(i % 3);
  const double g = a == 0 ? g0 : (a == 1 ? g1 : g2);
  const double vi = (xn[i] - xo[i]) / h;
  if (v) v[i] = vi;
  if (xtil) xtil[i] = xn[i] + h * vi + h * h * g;
}

mas_status launch_next_frame(Ctx& c, const double* xn, const double* xo, double* v, double* xtil) {
  const int64_t n3 = 3 * c.N;
  k_next_frame<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, xn, xo, c.cfg.h, c.cfg.gravity[0],
                                                             c.cfg.gravity[1], c.cfg.gravity[2], v, xtil);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

__global__ void k_stencil_distance(int64_t m, const double* x, const int32_t* idx,
                                   const double* grad, const double* off, double* d) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double acc = 0;
  for (int j = 0; j < 4; ++j) {
    int v = idx[4 * i + j];
    if (v < 0) continue;
    for (int a = 0; a < 3; ++a) acc += grad[12 * i + 3 * j + a] * x[3 * v + a];
  }
  d[i] = acc - off[i];
}

mas_status launch_stencil_distance(Ctx& c, const double* x, int64_t m, const int32_t* idx,
                                   const double* grad, const double* off, double* d) {
  if (m == 0) return MAS_OK;
  int bs = 256;
  k_stencil_distance<<<dim3((m + bs - 1) / bs), dim3(bs), 0, c.s>>>(m, x, idx, grad, off, d);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
