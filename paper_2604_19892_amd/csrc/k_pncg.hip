// Per-iteration kernels around the preconditioner: energy and gradient of
// the incremental potential, the 2x2 subspace step with its fallback and the
// restart ratio, and the per-subdomain safe step.
#include <algorithm>

#include "kernels.hpp"
#include "elem.hpp"

namespace mas {

constexpr int RB = 256;  // reduction block size

// sums NV values across the block; thread 0 writes out[v * nblk + blockIdx.x]
template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double* out, int nblk) {
  __shared__ double sh[NV][RB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) sh[q][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0;
      for (int i = 0; i < RB / 64; ++i) s += sh[q][i];
      out[q * nblk + blockIdx.x] = s;
    }
  }
}

// ----------------------------------------------------------- energy / grad
// Inertia and elasticity, owner-computes over the vertex ranges: workgroup r
// takes its vertices' inertia term M (x - x~) and every tet touching r (its
// range-major entries), accumulates the elastic gradient h^2 V P Dm^-T of its
// own vertices in LDS and writes g for them (no atomics).  A tet's energy
// h^2 V Psi(F) is counted by its home entry (the range of its smallest
// vertex).  Energies are reduced per
// range in a fixed order (part rows 0 and 1, one slot per range).  The
// range's own part of x is staged in LDS and read from there by every
// entry; one 1024-thread workgroup per compute unit (two 48 KB LDS arrays).
constexpr int EGT = 1024;
__global__ __launch_bounds__(EGT) void k_eg_range(int64_t nrange, const int32_t* rbeg, const int32_t* rl_t,
                                                  const int32_t* rl_tv, const double* rl_geo, const int32_t* rt_off,
                                                  const double* mass, const double* x, const double* xt, double h2,
                                                  double* g, double* part, int nblk, uint32_t* ctr) {
  __shared__ double win[3 * RANGE_MAX];
  __shared__ double xs[3 * RANGE_MAX];
  __shared__ double red[2][EGT / 64];
  __shared__ int64_t cur;
  const bool grad = g != nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // partial slots past the last range stay zero
  for (int64_t q = nrange + blockIdx.x * int64_t(EGT) + threadIdx.x; q < nblk; q += int64_t(gridDim.x) * EGT) {
    part[q] = 0.0;
    part[nblk + q] = 0.0;
  }
  while (true) {
    if (threadIdx.x == 0) cur = atomicAdd(ctr, 1u);
    __syncthreads();
    const int64_t r = cur;
    if (r >= nrange) break;  // every workgroup ends here once the counter passes nrange
    double e[2] = {0.0, 0.0};
    const int v0 = rbeg[r], nv = rbeg[r + 1] - v0;
    for (int q = threadIdx.x; q < 3 * nv; q += EGT) {
      win[q] = 0.0;
      xs[q] = x[3 * int64_t(v0) + q];
    }
    for (int lv = threadIdx.x; lv < nv; lv += EGT) {
      const double m = mass[v0 + lv];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double dx = x[3 * int64_t(v0 + lv) + a] - xt[3 * int64_t(v0 + lv) + a];
        e[0] += 0.5 * m * dx * dx;
      }
    }
    __syncthreads();
    const int t0 = rt_off[r], t1 = rt_off[r + 1];
    for (int w = t0 + threadIdx.x; w < t1; w += EGT) {
      const int4 tv = reinterpret_cast<const int4*>(rl_tv)[w];
      const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
      const bool own_e = rl_t[w] < 0;  // home entry of the tet
      bool touch[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) touch[j] = grad && vi[j] >= v0 && vi[j] < v0 + nv;
      double xe[12];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int lv = vi[j] - v0;
        if (lv >= 0 && lv < nv) {
#pragma unroll
          for (int a = 0; a < 3; ++a) xe[3 * j + a] = xs[3 * lv + a];
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a) xe[3 * j + a] = x[3 * vi[j] + a];
        }
      }
      double gm[12];
      geo_load(rl_geo, w, gm);
      double F[3][3];
      def_grad(xe, gm, F);
      const double s = h2 * gm[9];
      if (own_e) e[1] += s * snh_energy(F, gm[10], gm[11]);
      if (touch[0] || touch[1] || touch[2] || touch[3]) {
        double P[3][3];
        snh_stress(F, gm[10], gm[11], P);
        double f0[3] = {0, 0, 0};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            double acc = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) acc += P[a][b] * gm[3 * cc + b];
            acc *= s;
            f0[a] -= acc;
            if (touch[cc + 1]) atomicAdd(&win[3 * (vi[cc + 1] - v0) + a], acc);
          }
        }
        if (touch[0]) {
#pragma unroll
          for (int a = 0; a < 3; ++a) atomicAdd(&win[3 * (vi[0] - v0) + a], f0[a]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double t = wave_sum(e[q]);
      if (lane == 0) red[q][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      double t = 0.0;
      for (int i = 0; i < EGT / 64; ++i) t += red[threadIdx.x][i];
      part[threadIdx.x * int64_t(nblk) + r] = t;
    }
    if (grad) {
      for (int q = threadIdx.x; q < 3 * nv; q += EGT) {
        const int64_t gq = 3 * int64_t(v0) + q;
        g[gq] = mass[gq / 3] * (xs[q] - xt[gq]) + win[q];
      }
    }
    __syncthreads();
  }
}

// kappa b(d) and kappa b'(d) grad d; a non-positive distance flags +inf.
// Chunks of SW_CHUNK stencils scatter through an LDS window (stencils sorted
// by smallest vertex stay local).
__global__ __launch_bounds__(RB) void k_eg_contacts(int64_t N, int64_t m, const int32_t* idx, const double* d,
                                                    const double* grad, double kappa, double dhat, double* g,
                                                    double* part, int nblk) {
  __shared__ double win[3 * SW_WIN];
  __shared__ double win2[3 * SW_WIN];
  double e[2] = {0.0, 0.0};
  const bool gr = g != nullptr;
  for (int64_t chunk = blockIdx.x; chunk * SW_CHUNK < m; chunk += nblk) {
    const int64_t c0 = chunk * SW_CHUNK;
    // two windows: from the smallest vertex of the chunk's first stencil,
    // and around its largest one (a contact's two sides lie far apart in
    // the vertex order); vertices in neither go to memory
    int vbase, vbase2;
    {
      const int4 f4 = reinterpret_cast<const int4*>(idx)[c0];
      int mn = INT32_MAX, mx = -1;
      const int fv[4] = {f4.x, f4.y, f4.z, f4.w};
      for (int j = 0; j < 4; ++j)
        if (fv[j] >= 0) mn = min(mn, fv[j]), mx = max(mx, fv[j]);
      vbase = (mn == INT32_MAX) ? 0 : mn;
      vbase2 = max(vbase + SW_WIN, mx - SW_WIN / 4);
    }
    if (gr) {
      for (int q = threadIdx.x; q < 3 * SW_WIN; q += RB) win[q] = 0.0, win2[q] = 0.0;
      __syncthreads();
    }
    for (int k = 0; k < SW_CHUNK; k += RB) {
      const int64_t i = c0 + k + threadIdx.x;
      if (i >= m) break;
      const double di = d[i];
      if (!(di > 0.0)) {
        e[1] += 1.0;
        continue;
      }
      if (di >= dhat) continue;
      double b, b1, b2;
      barrier3(di, dhat, &b, &b1, &b2);
      e[0] += kappa * b;
      if (gr) {
        const double s = kappa * b1;
        const int4 iv = reinterpret_cast<const int4*>(idx)[i];
        const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (vi[j] < 0) continue;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double val = s * grad[12 * i + 3 * j + a];
            const int l2 = vi[j] - vbase2;
            if (l2 >= 0 && l2 < SW_WIN)
              __hip_atomic_fetch_add(&win2[3 * l2 + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
              sw_add(win, g, vbase, vi[j], a, val);
          }
        }
      }
    }
    if (gr) {
      __syncthreads();
      sw_flush(win, g, vbase, N);
      sw_flush(win2, g, vbase2, N);
      __syncthreads();
    }
  }
  block_reduce_store<2>(e, part, nblk);
}

// sums NV rows of nblk partials with one block of RB threads in a fixed order;
// the totals land in tot[0..NV) (LDS)
template <int NV>
__device__ inline void sum_partials(const double* part, int nblk, double* tot) {
  __shared__ double red[NV][RB];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0;
    for (int i = threadIdx.x; i < nblk; i += RB) s += part[q * nblk + i];
    red[q][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < NV) tot[threadIdx.x] = red[threadIdx.x][0];
  __syncthreads();
}

__global__ __launch_bounds__(RB) void k_eg_finalize(const double* part, int nblk, double* E) {
  __shared__ double tot[4];
  sum_partials<4>(part, nblk, tot);
  if (threadIdx.x == 0) *E = tot[3] > 0 ? INFINITY : (tot[0] + tot[1]) + tot[2];
}

mas_status launch_energy_grad(Ctx& c, const double* x, const double* xt, const mas_contacts* ct,
                              double* E, double* g) {
  ProfScope ps(c, MAS_T_ENERGY);
  const int nb = c.n_partial_blocks;
  double* part = c.partials;  // [0]: inertia [1]: elastic [2]: barrier [3]: infeasible count
  k_set_u32<<<dim3(1), dim3(1), 0, c.s>>>(c.ctr + 1, 0u);
  k_eg_range<<<dim3(std::min<int64_t>(c.nrange, int64_t(c.n_cu))), dim3(EGT), 0, c.s>>>(
      c.nrange, c.rbeg, c.rl_t, c.rl_tv, c.rl_geo, c.rt_off, c.mass, x, xt, c.cfg.h * c.cfg.h, g, part, nb, c.ctr + 1);
  int64_t m = ct ? ct->m : 0;
  if (m > 0) {
    // writes part[2*nb..] (energy) and part[3*nb..] (infeasible count)
    k_eg_contacts<<<dim3(nb), dim3(RB), 0, c.s>>>(c.N, m, ct->idx, ct->d, ct->grad, c.cfg.kappa, c.cfg.dhat,
                                                   g, part + 2 * nb, nb);
  } else {
    HIPCHK(hipMemsetAsync(part + 2 * nb, 0, sizeof(double) * 2 * nb, c.s));
  }
  k_eg_finalize<<<dim3(1), dim3(RB), 0, c.s>>>(part, nb, E);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ------------------------------------------------------------ subspace step
// per block: g.z, g.p, g.zp, z.vz, z.vp, p.vp, g.g, z.z and over the update
// columns (u.z)^2, (u.z)(u.p), (u.p)^2
constexpr int NS = 11;

__global__ __launch_bounds__(RB) void k_ss_reduce(int64_t n3, const double* g, const double* z,
                                                  const double* zp, const double* p, const double* vz,
                                                  const double* vp, int use_p, int64_t m,
                                                  const int32_t* Uidx, const double* U, const double* dS,
                                                  double* part, int nblk) {
  double s[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) s[q] = 0.0;
  for (int64_t i = blockIdx.x * int64_t(RB) + threadIdx.x; i < n3; i += int64_t(nblk) * RB) {
    double gi = g[i], zi = z[i], vzi = vz[i];
    s[0] += gi * zi;
    if (zp) s[2] += gi * zp[i];
    s[3] += zi * vzi;
    s[6] += gi * gi;
    s[7] += zi * zi;
    if (use_p) {
      double pi = p[i], vpi = vp[i];
      s[1] += gi * pi;
      s[4] += zi * vpi;
      s[5] += pi * vpi;
    }
  }
  for (int64_t c = blockIdx.x * int64_t(RB) + threadIdx.x; c < m; c += int64_t(nblk) * RB) {
    if (!(dS[c] > 0.0)) continue;  // zero column (not stored)
    const int4 iv = reinterpret_cast<const int4*>(Uidx)[c];
    int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    double xz = 0, xp = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double u = U[12 * c + 3 * j + a];
        xz += u * z[3 * vi[j] + a];
        if (use_p) xp += u * p[3 * vi[j] + a];
      }
    }
    s[8] += xz * xz;
    s[9] += xz * xp;
    s[10] += xp * xp;
  }
  block_reduce_store<NS>(s, part, nblk);
}

__global__ __launch_bounds__(RB) void k_ss_finalize(const double* part, int nblk, int restart, int has_zp,
                                                    double eps_sing, double eps_abs, double delta,
                                                    mas_step_out* out, double* scal) {
  __shared__ double s[NS];
  sum_partials<NS>(part, nblk, s);
  if (threadIdx.x != 0) return;
  double gz = s[0], gp = s[1], gzp = s[2];
  double A11 = s[3] + s[8], A12 = s[4] + s[9], A22 = s[5] + s[10];
  double mu, nu;
  int fb = 0;
  if (restart) {
    if (A11 > 0) {
      mu = gz / A11;
      nu = 0.0;
    } else {
      mu = 1.0;
      nu = 0.0;
      fb = 1;
    }
  } else {
    double det = A11 * A22 - A12 * A12;
    if (fabs(det) < eps_sing * fmax(A11 * A22, eps_abs)) {
      mu = 1.0;
      nu = 0.0;
      fb = 1;
    } else {
      mu = (gz * A22 - A12 * gp) / det;
      nu = (A12 * gz - A11 * gp) / det;
    }
  }
  double r = has_zp ? fabs(gzp) / gz : 0.0;
  mas_step_out o;
  o.mu = mu;
  o.nu = nu;
  o.r = r;
  o.gz = gz;
  o.gp = gp;
  o.gzp = gzp;
  o.A11 = A11;
  o.A12 = A12;
  o.A22 = A22;
  o.gnorm2 = s[6];
  o.znorm2 = s[7];
  o.fallback = fb;
  o.restart_next = (r > delta) ? 1 : 0;
  o.restart_used = restart ? 1 : 0;
  o.reserved = 0;
  if (out) *out = o;
  scal[0] = mu;
  scal[1] = nu;
}

// p <- -mu z + nu p;  v_p <- -mu v_z + nu v_p  (H_base is linear)
__global__ void k_ss_update(int64_t n3, const double* z, const double* vz, double* p, double* vp,
                            const double* scal) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  const double mu = scal[0], nu = scal[1];
  if (nu == 0.0) {
    p[i] = -mu * z[i];
    vp[i] = -mu * vz[i];
  } else {
    p[i] = -mu * z[i] + nu * p[i];
    vp[i] = -mu * vz[i] + nu * vp[i];
  }
}

mas_status launch_subspace(Ctx& c, const double* g, const double* z, const double* zp,
                           const double* vz, double* p, double* vp, int restart, mas_step_out* out) {
  ProfScope ps(c, MAS_T_SUBSPACE);
  const int nb = c.n_partial_blocks;
  int64_t n3 = 3 * c.N;
  int64_t m = (c.have_update) ? c.mc : 0;
  k_ss_reduce<<<dim3(nb), dim3(RB), 0, c.s>>>(n3, g, z, zp, p, vz, vp, restart ? 0 : 1, m, c.Uidx, c.U,
                                              c.dS, c.partials, nb);
  k_ss_finalize<<<dim3(1), dim3(RB), 0, c.s>>>(c.partials, nb, restart, zp != nullptr, c.cfg.eps_sing,
                                               c.cfg.eps_abs, c.cfg.restart_delta, out, c.scal);
  k_ss_update<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, z, vz, p, vp, c.scal);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ------------------------------------------------------------- safe step
__global__ void k_alpha_init(int64_t D, double* alpha) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < D) alpha[i] = 1.0;
}

// alpha_c = min(1, 0.9 d / s) for a stencil closing at the rate
// s = -sum_j grad_j . p_j > 0, to every subdomain the stencil touches
__global__ __launch_bounds__(256) void k_alpha_stencils(int64_t m, const int32_t* idx, const double* grad,
                                                        const double* d, const double* p, double* alpha) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int vi[4] = {-1, -1, -1, -1};
  double a = INFINITY;
  if (i < m) {
    const int4 iv = reinterpret_cast<const int4*>(idx)[i];
    vi[0] = iv.x; vi[1] = iv.y; vi[2] = iv.z; vi[3] = iv.w;
    double s = 0;  // closing rate of the stencil along p
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
#pragma unroll
      for (int q = 0; q < 3; ++q) s -= grad[12 * i + 3 * j + q] * p[3 * vi[j] + q];
    }
    if (s > 0.0) a = fmax(fmin(1.0, 0.9 * d[i] / s), 0.0);
  }
  const bool has = a < 1.0;
  if (__ballot(has) == 0) return;  // uniform
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sd = vi[j] >> 5;
    const long long key = (has && vi[j] >= 0) ? (long long)sd : -1ll;
    wave_min_pos(key, alpha + (key >= 0 ? sd : 0), a);
  }
}

__global__ void k_step(int64_t n3, const double* x, const double* p, const double* alpha, double scale,
                       double* xo) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  xo[i] = x[i] + scale * alpha[(i / 3) >> 5] * p[i];
}

// A stencil whose vertices, each moved with its own subdomain's step, would
// close to below 0.05 of its distance marks the subdomains it touches.
__global__ __launch_bounds__(256) void k_alpha_check(int64_t m, const int32_t* idx, const double* grad,
                                                     const double* d, const double* p, const double* alpha,
                                                     uint8_t* mark, uint32_t* count) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  bool viol = false;
  if (i < m) {
    const double di = d[i];
    if (di > 0.0) {
      const int4 iv = reinterpret_cast<const int4*>(idx)[i];
      const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
      double dn = di;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (vi[j] < 0) continue;
        double dot = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) dot += grad[12 * i + 3 * j + q] * p[3 * vi[j] + q];
        dn += alpha[vi[j] >> 5] * dot;
      }
      if (dn < 0.05 * di) {
        viol = true;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (vi[j] >= 0) mark[vi[j] >> 5] = 1;
      }
    }
  }
  const unsigned long long b = __ballot(viol);
  if (b != 0 && (threadIdx.x & 63) == 0) atomicAdd(count, uint32_t(__popcll(b)));
}

__global__ void k_alpha_halve(int64_t D, double* alpha, uint8_t* mark) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < D && mark[i]) {
    alpha[i] *= 0.5;
    mark[i] = 0;
  }
}

mas_status launch_safe_step(Ctx& c, const double* x, const double* p, const mas_contacts* cand,
                            double scale, double* alpha, double* x_out) {
  const int64_t D = c.lv[0].nsub;
  if (cand) {
    k_alpha_init<<<dim3((D + 255) / 256), dim3(256), 0, c.s>>>(D, c.alpha);
    if (cand->m > 0) {
      const dim3 g((cand->m + 255) / 256), b(256);
      k_alpha_stencils<<<g, b, 0, c.s>>>(cand->m, cand->idx, cand->grad, cand->d, p, c.alpha);
      // subdomains moving at different steps: halve the steps of the
      // subdomains of any stencil the combined motion would close
      for (int round = 0; round < SAFE_ROUNDS; ++round) {
        k_set_u32<<<dim3(1), dim3(1), 0, c.s>>>(c.ctr + 2, 0u);
        k_alpha_check<<<g, b, 0, c.s>>>(cand->m, cand->idx, cand->grad, cand->d, p, c.alpha, c.amark, c.ctr + 2);
        uint32_t nv = 0;
        HIPCHK(hipMemcpyAsync(&nv, c.ctr + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, c.s));
        HIPCHK(hipStreamSynchronize(c.s));
        if (nv == 0) break;
        k_alpha_halve<<<dim3((D + 255) / 256), dim3(256), 0, c.s>>>(D, c.alpha, c.amark);
      }
    }
  }
  int64_t n3 = 3 * c.N;
  k_step<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, x, p, c.alpha, scale, x_out);
  if (alpha) HIPCHK(hipMemcpyAsync(alpha, c.alpha, sizeof(double) * D, hipMemcpyDeviceToDevice, c.s));
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
