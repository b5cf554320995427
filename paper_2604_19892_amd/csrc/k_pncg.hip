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
// DET: the gradient rows are summed with the two-pass fixed-point
// accumulation (the element stresses are evaluated twice).
constexpr int EGT = 1024;
template <bool DET>
__global__ __launch_bounds__(EGT) void k_eg_range(int64_t nrange, const int32_t* rbeg, const int32_t* rl_t,
                                                  const int32_t* rl_tv, const double* rl_geo, const int32_t* rt_off,
                                                  const double* mass, const double* x, const double* xt, double h2,
                                                  double* g, double* part, int nblk, uint32_t* ctr) {
  __shared__ double win[3 * RANGE_MAX];
  __shared__ double xs[3 * RANGE_MAX];
  __shared__ int aux[DET ? 3 * RANGE_MAX : 1];
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
      if (DET) aux[q] = 0;
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
    for (int pass = (DET && grad) ? 0 : 1; pass < 2; ++pass) {
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
      if (own_e && pass == 1) e[1] += s * snh_energy(F, gm[10], gm[11]);
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
            if (touch[cc + 1]) acc_term<DET>(win, aux, 3 * (vi[cc + 1] - v0) + a, acc, pass);
          }
        }
        if (touch[0]) {
#pragma unroll
          for (int a = 0; a < 3; ++a) acc_term<DET>(win, aux, 3 * (vi[0] - v0) + a, f0[a], pass);
        }
      }
    }
    if (DET && grad) {
      __syncthreads();
      for (int q = threadIdx.x; q < 3 * nv; q += EGT) {
        if (pass == 0) fx_mid(&win[q], &aux[q]);
        else win[q] = fx_get(&win[q], &aux[q]);
      }
      __syncthreads();
    }
    }  // passes
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

// LDS hash of the far side of a chunk's contacts: slot of vertex v (linear
// probing, at most FAR_PROBES probes), or -1 when the table is too full
constexpr int FAR_SLOTS = 1024;
constexpr int FAR_PROBES = 16;
__device__ inline int far_slot(int* hk, int v) {
  int h = int((uint32_t(v) * 2654435761u) >> 22) & (FAR_SLOTS - 1);
  for (int p = 0; p < FAR_PROBES; ++p) {
    const int old = atomicCAS(&hk[h], -1, v);
    if (old == -1 || old == v) return h;
    h = (h + 1) & (FAR_SLOTS - 1);
  }
  return -1;
}

// kappa b(d) and kappa b'(d) grad d; a non-positive distance flags +inf.
// Chunks of SW_CHUNK stencils scatter through an LDS window (stencils sorted
// by smallest vertex stay local) and, for the vertices outside it (a
// contact's other side lies far away in the vertex order), an LDS hash
// table that is added to g once per distinct vertex.
__global__ __launch_bounds__(RB) void k_eg_contacts(int64_t N, int64_t m, const int32_t* idx, const double* d,
                                                    const double* grad, double kappa, double dhat, double* g,
                                                    double* part, int nblk) {
  __shared__ double win[3 * SW_WIN];
  __shared__ int hk[FAR_SLOTS];
  __shared__ double hv[3 * FAR_SLOTS];
  double e[2] = {0.0, 0.0};
  const bool gr = g != nullptr;
  for (int64_t chunk = blockIdx.x; chunk * SW_CHUNK < m; chunk += nblk) {
    const int64_t c0 = chunk * SW_CHUNK;
    // the window starts at the smallest vertex of the chunk's first stencil
    int vbase;
    {
      const int4 f4 = reinterpret_cast<const int4*>(idx)[c0];
      int mn = INT32_MAX;
      const int fv[4] = {f4.x, f4.y, f4.z, f4.w};
      for (int j = 0; j < 4; ++j)
        if (fv[j] >= 0) mn = min(mn, fv[j]);
      vbase = (mn == INT32_MAX) ? 0 : mn;
    }
    if (gr) {
      for (int q = threadIdx.x; q < 3 * SW_WIN; q += RB) win[q] = 0.0;
      for (int q = threadIdx.x; q < FAR_SLOTS; q += RB) {
        hk[q] = -1;
        hv[3 * q] = hv[3 * q + 1] = hv[3 * q + 2] = 0.0;
      }
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
          const int lv = vi[j] - vbase;
          const bool near = lv >= 0 && lv < SW_WIN;
          const int fs = near ? -1 : far_slot(hk, vi[j]);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double val = s * grad[12 * i + 3 * j + a];
            if (near)
              __hip_atomic_fetch_add(&win[3 * lv + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else if (fs >= 0)
              __hip_atomic_fetch_add(&hv[3 * fs + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
              __hip_atomic_fetch_add(&g[3 * int64_t(vi[j]) + a], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    if (gr) {
      __syncthreads();
      sw_flush(win, g, vbase, N);
      for (int q = threadIdx.x; q < FAR_SLOTS; q += RB) {
        const int v = hk[q];
        if (v < 0) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (hv[3 * q + a] != 0.0) atomicAdd(&g[3 * int64_t(v) + a], hv[3 * q + a]);
      }
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

// Deterministic mode: g[3 v + a] += kappa b'(d_c) grad_c[3 j + a] over the
// incidences (c, j) of vertex v in ascending order (0 < d_c < dhat).
__global__ __launch_bounds__(256) void k_eg_contacts_gather(int64_t N, const int32_t* off, const int32_t* list,
                                                            const double* d, const double* grad, double kappa,
                                                            double dhat, double* g) {
  const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (v >= N) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = off[v]; q < off[v + 1]; ++q) {
    const int64_t slot = list[q];
    const int64_t ci = slot >> 2;
    const double di = d[ci];
    if (!(di > 0.0) || di >= dhat) continue;
    double b, b1, b2;
    barrier3(di, dhat, &b, &b1, &b2);
    const double s = kappa * b1;
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] += s * grad[12 * ci + 3 * (slot & 3) + a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) g[3 * v + a] += acc[a];
}

mas_status launch_energy_grad(Ctx& c, const double* x, const double* xt, const mas_contacts* ct,
                              double* E, double* g) {
  ProfScope ps(c, MAS_T_ENERGY);
  const int nb = c.n_partial_blocks;
  double* part = c.partials;  // [0]: inertia [1]: elastic [2]: barrier [3]: infeasible count
  const bool det = c.cfg.deterministic != 0;
  k_set_u32<<<dim3(1), dim3(1), 0, c.s>>>(c.ctr + 1, 0u);
  const dim3 gr(std::min<int64_t>(c.nrange, int64_t(c.n_cu)));
  if (det)
    k_eg_range<true><<<gr, dim3(EGT), 0, c.s>>>(c.nrange, c.rbeg, c.rl_t, c.rl_tv, c.rl_geo, c.rt_off, c.mass, x, xt,
                                                c.cfg.h * c.cfg.h, g, part, nb, c.ctr + 1);
  else
    k_eg_range<false><<<gr, dim3(EGT), 0, c.s>>>(c.nrange, c.rbeg, c.rl_t, c.rl_tv, c.rl_geo, c.rt_off, c.mass, x,
                                                 xt, c.cfg.h * c.cfg.h, g, part, nb, c.ctr + 1);
  int64_t m = ct ? ct->m : 0;
  if (m > 0) {
    // writes part[2*nb..] (energy) and part[3*nb..] (infeasible count); in
    // deterministic mode the gradient terms come from the ordered gather
    k_eg_contacts<<<dim3(nb), dim3(RB), 0, c.s>>>(c.N, m, ct->idx, ct->d, ct->grad, c.cfg.kappa, c.cfg.dhat,
                                                   det ? nullptr : g, part + 2 * nb, nb);
    if (det && g) {
      mas_status st = build_incidence(c, m, ct->idx, nullptr);
      if (st != MAS_OK) return st;
      k_eg_contacts_gather<<<dim3((c.N + 255) / 256), dim3(256), 0, c.s>>>(c.N, c.inc_off, c.inc_list, ct->d,
                                                                            ct->grad, c.cfg.kappa, c.cfg.dhat, g);
    }
  } else {
    fill_f64(c, part + 2 * nb, 2 * nb, 0.0);
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

// the 2x2 solve from the sums s[NS] (thread-local); writes out (nullable)
// and returns mu, nu in scal[0], scal[1]
__device__ void ss_solve(const double* s, int restart, int has_zp, double eps_sing, double eps_abs, double delta,
                         mas_step_out* out, double* scal);

__global__ __launch_bounds__(RB) void k_ss_finalize(const double* part, int nblk, int restart, int has_zp,
                                                    double eps_sing, double eps_abs, double delta,
                                                    mas_step_out* out, double* scal) {
  __shared__ double s[NS];
  sum_partials<NS>(part, nblk, s);
  if (threadIdx.x != 0) return;
  ss_solve(s, restart, has_zp, eps_sing, eps_abs, delta, out, scal);
}

__device__ void ss_solve(const double* s, int restart, int has_zp, double eps_sing, double eps_abs, double delta,
                         mas_step_out* out, double* scal) {
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

int64_t subspace_workspace_elems(const Ctx& c) { return int64_t(NS) * c.n_partial_blocks + 2; }

// part: NS x n_partial_blocks per-block partial sums; scal: mu and nu.  Every
// entry is written before it is read, so neither needs clearing.
mas_status launch_subspace_ws(Ctx& c, const double* g, const double* z, const double* zp, const double* vz,
                              double* p, double* vp, int restart, mas_step_out* out, double* part,
                              double* scal) {
  const int nb = c.n_partial_blocks;
  int64_t n3 = 3 * c.N;
  int64_t m = (c.have_update) ? c.mc : 0;
  k_ss_reduce<<<dim3(nb), dim3(RB), 0, c.s>>>(n3, g, z, zp, p, vz, vp, restart ? 0 : 1, m, c.Uidx, c.U,
                                              c.dS, part, nb);
  k_ss_finalize<<<dim3(1), dim3(RB), 0, c.s>>>(part, nb, restart, zp != nullptr, c.cfg.eps_sing,
                                               c.cfg.eps_abs, c.cfg.restart_delta, out, scal);
  k_ss_update<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, z, vz, p, vp, scal);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status launch_subspace(Ctx& c, const double* g, const double* z, const double* zp,
                           const double* vz, double* p, double* vp, int restart, mas_step_out* out) {
  ProfScope ps(c, MAS_T_SUBSPACE);
  return launch_subspace_ws(c, g, z, zp, vz, p, vp, restart, out, c.partials, c.scal);
}

// ------------------------------------------------- comparison direction rules
// Classic preconditioned nonlinear CG directions of the search-direction
// study (Section 5): d = -z + beta d_prev with the Fletcher-Reeves,
// conjugate-descent or Dai-Kou beta, and the step p = alpha d with alpha
// minimising the quadratic model g^T p + 1/2 p^T H~ p along d.  The
// subspace step's reduction supplies g.z, g.d_prev, g.z_prev and the H~
// products of z and d_prev; three more sums bring in g_prev.

// per block: g_prev.z, g_prev.z_prev, g_prev.d_prev
__global__ __launch_bounds__(RB) void k_beta_reduce(int64_t n3, const double* gq, const double* z,
                                                    const double* zq, const double* d, double* part, int nblk) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * int64_t(RB) + threadIdx.x; i < n3; i += int64_t(nblk) * RB) {
    const double a = gq[i];
    s[0] += a * z[i];
    s[1] += a * zq[i];
    s[2] += a * d[i];
  }
  block_reduce_store<3>(s, part, nblk);
}

__global__ __launch_bounds__(RB) void k_beta_finalize(const double* part, const double* part3, int nblk, int rule,
                                                      int restart, int has_zp, double delta, mas_step_out* out,
                                                      double* scal) {
  __shared__ double s[NS];
  __shared__ double t[3];
  sum_partials<NS>(part, nblk, s);
  if (!restart) sum_partials<3>(part3, nblk, t);  // restart is uniform over the block
  if (threadIdx.x != 0) return;
  const double gz = s[0], gd = s[1], gzp = s[2];
  const double A11 = s[3] + s[8], A12 = s[4] + s[9], A22 = s[5] + s[10];
  double beta = 0.0;
  int fb = 0;
  if (!restart) {
    const double qz = t[0], qzp = t[1], qd = t[2];  // g_prev . (z, z_prev, d_prev)
    double den = 0.0, b = 0.0;
    if (rule == MAS_BETA_FR) {
      den = qzp;
      b = gz / den;
    } else if (rule == MAS_BETA_CD) {
      den = -qd;
      b = gz / den;
    } else {  // Dai-Kou: y = g - g_prev, P y = z - z_prev
      den = gd - qd;                       // d_prev . y
      const double yz = gz - qz;           // y . z
      const double yPy = gz - gzp - qz + qzp;
      b = yz / den - (yPy / den) * (gd / den);
    }
    if (den > 0.0) beta = b;
    else fb = 1;
  }
  double gdn = -gz + beta * gd;  // g . d
  if (!restart && !(gdn < 0.0)) {
    beta = 0.0;
    fb = 1;
    gdn = -gz;
  }
  const double dHd = beta == 0.0 ? A11 : A11 - 2.0 * beta * A12 + beta * beta * A22;
  double alpha;
  if (dHd > 0.0) {
    alpha = -gdn / dHd;
  } else {
    alpha = 1.0;
    fb = 1;
  }
  const double r = has_zp ? fabs(gzp) / gz : 0.0;
  mas_step_out o;
  o.mu = alpha;
  o.nu = beta;
  o.r = r;
  o.gz = gz;
  o.gp = gd;
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
  scal[0] = alpha;
  scal[1] = beta;
}

// d <- -z + beta d;  v_d <- -v_z + beta v_d;  p = alpha d
__global__ void k_beta_update(int64_t n3, const double* z, const double* vz, double* d, double* vd, double* p,
                              const double* scal) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  const double alpha = scal[0], beta = scal[1];
  double dn, vn;
  if (beta == 0.0) {
    dn = -z[i];
    vn = -vz[i];
  } else {
    dn = -z[i] + beta * d[i];
    vn = -vz[i] + beta * vd[i];
  }
  d[i] = dn;
  vd[i] = vn;
  p[i] = alpha * dn;
}

mas_status launch_beta(Ctx& c, int rule, const double* g, const double* gq, const double* z, const double* zq,
                       const double* vz, double* d, double* vd, int restart, double* p, mas_step_out* out) {
  ProfScope ps(c, MAS_T_SUBSPACE);
  const int nb = c.n_partial_blocks;
  const int64_t n3 = 3 * c.N;
  const int64_t m = (c.have_update) ? c.mc : 0;
  double* part = c.partials;
  double* part3 = c.partials + int64_t(NS) * nb;  // rows NS..NS+2 of the 16-row workspace
  k_ss_reduce<<<dim3(nb), dim3(RB), 0, c.s>>>(n3, g, z, zq, d, vz, vd, restart ? 0 : 1, m, c.Uidx, c.U, c.dS,
                                              part, nb);
  if (!restart) k_beta_reduce<<<dim3(nb), dim3(RB), 0, c.s>>>(n3, gq, z, zq, d, part3, nb);
  k_beta_finalize<<<dim3(1), dim3(RB), 0, c.s>>>(part, part3, nb, rule, restart, zq != nullptr,
                                                 c.cfg.restart_delta, out, c.scal);
  k_beta_update<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, z, vz, d, vd, p, c.scal);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// ------------------------------------------------------------- safe step
__global__ void k_alpha_init(int64_t D, double* a0, double* amix, uint64_t* half, uint32_t* rounds) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < D) {
    a0[i] = 1.0;
    amix[i] = 1.0;
    half[i] = 0ull;
  }
  if (i <= SAFE_ROUNDS) rounds[i] = 0u;
}

// alpha_c = min(1, 0.9 d / s) for a stencil closing at the rate
// s = -sum_j grad_j . p_j > 0, to every subdomain the stencil touches
// (alpha); and the fallback bound min(1, 0.9 d / sum_j max(0, -grad_j . p_j)),
// which holds for any mix of per-vertex steps up to it (amix)
__global__ __launch_bounds__(256) void k_alpha_stencils(int64_t m, const int32_t* idx, const double* grad,
                                                        const double* d, const double* p, double* alpha,
                                                        double* amix) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int vi[4] = {-1, -1, -1, -1};
  double a = INFINITY, am = INFINITY;
  if (i < m) {
    const int4 iv = reinterpret_cast<const int4*>(idx)[i];
    vi[0] = iv.x; vi[1] = iv.y; vi[2] = iv.z; vi[3] = iv.w;
    double s = 0;   // closing rate of the stencil along p
    double sp = 0;  // sum of the vertices' own closing rates
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) dot += grad[12 * i + 3 * j + q] * p[3 * vi[j] + q];
      s -= dot;
      sp += fmax(0.0, -dot);
    }
    if (s > 0.0) a = fmax(fmin(1.0, 0.9 * d[i] / s), 0.0);
    if (sp > 0.0) am = fmax(fmin(1.0, 0.9 * d[i] / sp), 0.0);
  }
  const bool has = a < 1.0, hasm = am < 1.0;
  if (__ballot(has || hasm) == 0) return;  // uniform
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sd = vi[j] >> 5;
    const long long key = (has && vi[j] >= 0) ? (long long)sd : -1ll;
    wave_min_pos(key, alpha + (key >= 0 ? sd : 0), a);
    const long long keym = (hasm && vi[j] >= 0) ? (long long)sd : -1ll;
    wave_min_pos(keym, amix + (keym >= 0 ? sd : 0), am);
  }
}

// Step of subdomain s in damping round r: a0 halved once for every earlier
// round that marked it (bit q of half[s] for q < r; bits of round r itself,
// set concurrently, are masked off, so the value does not depend on the
// order of the atomics).
__device__ __forceinline__ double alpha_round(const double* a0, const uint64_t* half, int s, uint64_t mask) {
  const uint64_t h = __hip_atomic_load(half + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & mask;
  return ldexp(a0[s], -__popcll(h));
}

// Damping round r < SAFE_ROUNDS: a stencil whose vertices, each moved with
// its own subdomain's step, would close to below 0.05 of its distance marks
// its subdomains for halving (bit r) and is counted in rounds[r].  A round
// after one that found nothing returns at once.  Round SAFE_ROUNDS only
// counts what is left.
__global__ __launch_bounds__(256) void k_alpha_round(int r, int64_t m, const int32_t* idx, const double* grad,
                                                     const double* d, const double* p, const double* a0,
                                                     uint64_t* half, uint32_t* rounds) {
  if (r > 0 && rounds[r - 1] == 0u) return;  // uniform: written by the previous launch
  const uint64_t mask = (1ull << r) - 1ull;
  // a bounded grid (most rounds find nothing and return at once, so their
  // cost is the dispatch); each workgroup walks a contiguous run of
  // stencils, runs placed by xcd_block
  const int64_t per = (m + int64_t(gridDim.x) * 256 - 1) / (int64_t(gridDim.x) * 256) * 256;
  const int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * per;
  uint32_t nviol = 0;
  for (int64_t i = b0 + threadIdx.x; i < min(m, b0 + per); i += blockDim.x) {
    const double di = d[i];
    if (!(di > 0.0)) continue;
    const int4 iv = reinterpret_cast<const int4*>(idx)[i];
    const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    double dn = di;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) dot += grad[12 * i + 3 * j + q] * p[3 * vi[j] + q];
      dn += alpha_round(a0, half, vi[j] >> 5, mask) * dot;
    }
    if (dn < 0.05 * di) {
      ++nviol;
      if (r < SAFE_ROUNDS) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (vi[j] >= 0) atomicOr(reinterpret_cast<unsigned long long*>(half + (vi[j] >> 5)), 1ull << r);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) nviol += __shfl_xor(nviol, o);
  if (nviol != 0 && (threadIdx.x & 63) == 0) atomicAdd(rounds + r, nviol);
}

// the damped steps, or, if the last round still found a stencil closing
// below 0.05 d, the bound for any mix of steps for every subdomain
__global__ void k_alpha_final(int64_t D, const double* a0, const double* amix, const uint64_t* half,
                              const uint32_t* rounds, double* alpha) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= D) return;
  alpha[i] = rounds[SAFE_ROUNDS] != 0u ? amix[i] : ldexp(a0[i], -__popcll(half[i]));
}

__global__ void k_step(int64_t n3, const double* x, const double* p, const double* alpha, double scale,
                       double* xo) {
  int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  xo[i] = x[i] + scale * alpha[(i / 3) >> 5] * p[i];
}

__global__ void k_copy_f64(const double* src, double* dst, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// x_out = x + scale alpha_{sub(v)} p_v with the step sizes in c.alpha (and a
// copy of them to alpha when given)
mas_status launch_step_with(Ctx& c, const double* x, const double* p, double scale, double* alpha,
                            double* x_out) {
  const int64_t D = c.lv[0].nsub;
  const int64_t n3 = 3 * c.N;
  k_step<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, x, p, c.alpha, scale, x_out);
  if (alpha)
    k_copy_f64<<<dim3(std::min<int64_t>((D + 255) / 256, 1024)), dim3(256), 0, c.s>>>(c.alpha, alpha, D);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

mas_status launch_safe_step(Ctx& c, const double* x, const double* p, const mas_contacts* cand,
                            double scale, double* alpha, double* x_out) {
  const int64_t D = c.lv[0].nsub;
  const dim3 gD((std::max<int64_t>(D, SAFE_ROUNDS + 1) + 255) / 256), b256(256);
  if (cand) {
    k_alpha_init<<<gD, b256, 0, c.s>>>(D, c.alpha0, c.alpha_mix, c.ahalf, c.around);
    if (cand->m > 0) {
      const dim3 g((cand->m + 255) / 256);
      k_alpha_stencils<<<g, b256, 0, c.s>>>(cand->m, cand->idx, cand->grad, cand->d, p, c.alpha0, c.alpha_mix);
      // subdomains moving at different steps: halve the steps of the
      // subdomains of any stencil the combined motion would close
      const dim3 gr(unsigned(std::min<int64_t>(g.x, 4 * int64_t(c.n_cu))));
      for (int r = 0; r <= SAFE_ROUNDS; ++r)
        k_alpha_round<<<gr, b256, 0, c.s>>>(r, cand->m, cand->idx, cand->grad, cand->d, p, c.alpha0, c.ahalf,
                                            c.around);
    }
    k_alpha_final<<<gD, b256, 0, c.s>>>(D, c.alpha0, c.alpha_mix, c.ahalf, c.around, c.alpha);
  }
  int64_t n3 = 3 * c.N;
  k_step<<<dim3((n3 + 255) / 256), b256, 0, c.s>>>(n3, x, p, c.alpha, scale, x_out);
  if (alpha) k_copy_f64<<<dim3(std::min<int64_t>((D + 255) / 256, 1024)), b256, 0, c.s>>>(c.alpha, alpha, D);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}


// ------------------------------------------------------------------ scenes
// Batched form: independent scenes in one context.  Library vertices are
// ordered scene by scene and no vertex range crosses a scene, so per-range
// partial sums add up to per-scene sums in a fixed order; the terms of the
// update columns and of the contacts go to their scene through LDS and one
// atomic per scene and workgroup.  Scratch: sc_acc[0, 3S) the xi sums,
// [3S, 5S) the per-scene mu and nu, [5S, 7S) the contact energies.

// per range: the vector sums 0..7 of the 2x2 system over the range's DOFs
__global__ __launch_bounds__(RB) void k_ss_reduce_rng(const int32_t* rbeg, const int32_t* seg, const double* g,
                                                      const double* z, const double* zp, const double* p,
                                                      const double* vz, const double* vp, const int32_t* restart,
                                                      double* part, int nrange) {
  const int r = blockIdx.x;
  const int64_t i0 = 3 * int64_t(rbeg[r]), i1 = 3 * int64_t(rbeg[r + 1]);
  const bool use_p = restart[seg[rbeg[r]]] == 0;
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RB) {
    const double gi = g[i], zi = z[i], vzi = vz[i];
    s[0] += gi * zi;
    if (zp) s[2] += gi * zp[i];
    s[3] += zi * vzi;
    s[6] += gi * gi;
    s[7] += zi * zi;
    if (use_p) {
      const double pi = p[i], vpi = vp[i];
      s[1] += gi * pi;
      s[4] += zi * vpi;
      s[5] += pi * vpi;
    }
  }
  block_reduce_store<8>(s, part, nrange);
}

// (u.z)^2, (u.z)(u.p), (u.p)^2 of the update columns, per scene
__global__ __launch_bounds__(RB) void k_ss_xi_scenes(int64_t m, const int32_t* Uidx, const double* U,
                                                     const double* dS, const double* z, const double* p,
                                                     const int32_t* seg, const int32_t* restart, int S,
                                                     double* acc) {
  extern __shared__ double la[];
  for (int q = threadIdx.x; q < 3 * S; q += RB) la[q] = 0.0;
  __syncthreads();
  for (int64_t c = blockIdx.x * int64_t(RB) + threadIdx.x; c < m; c += int64_t(gridDim.x) * RB) {
    if (!(dS[c] > 0.0)) continue;
    const int4 iv = reinterpret_cast<const int4*>(Uidx)[c];
    const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    int sc = -1;
#pragma unroll
    for (int j = 3; j >= 0; --j)
      if (vi[j] >= 0) sc = seg[vi[j]];
    if (sc < 0) continue;
    const bool use_p = restart[sc] == 0;
    double xz = 0.0, xp = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (vi[j] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u = U[12 * c + 3 * j + a];
        xz += u * z[3 * vi[j] + a];
        if (use_p) xp += u * p[3 * vi[j] + a];
      }
    }
    __hip_atomic_fetch_add(&la[3 * sc], xz * xz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&la[3 * sc + 1], xz * xp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&la[3 * sc + 2], xp * xp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 3 * S; q += RB)
    if (la[q] != 0.0) atomicAdd(&acc[q], la[q]);
}

// per scene (one workgroup each): its ranges' sums in a fixed order, the
// xi sums, and the 2x2 solve
__global__ __launch_bounds__(RB) void k_ss_final_scenes(const int64_t* scene_r, const double* part, int nrange,
                                                        const double* acc, const int32_t* restart, int has_zp,
                                                        double eps_sing, double eps_abs, double delta,
                                                        mas_step_out* out, double* scal) {
  __shared__ double red[8][RB];
  const int sc = blockIdx.x;
  const int64_t r0 = scene_r[sc], r1 = scene_r[sc + 1];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double t = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += RB) t += part[q * int64_t(nrange) + r];
    red[q][threadIdx.x] = t;
  }
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double s[NS];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = red[q][0];
  s[8] = acc[3 * sc];
  s[9] = acc[3 * sc + 1];
  s[10] = acc[3 * sc + 2];
  ss_solve(s, restart[sc], has_zp, eps_sing, eps_abs, delta, out ? out + sc : nullptr, scal + 2 * sc);
}

__global__ void k_ss_update_scenes(int64_t n3, const int32_t* seg, const double* z, const double* vz, double* p,
                                   double* vp, const double* scal) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  const int sc = seg[i / 3];
  const double mu = scal[2 * sc], nu = scal[2 * sc + 1];
  if (nu == 0.0) {
    p[i] = -mu * z[i];
    vp[i] = -mu * vz[i];
  } else {
    p[i] = -mu * z[i] + nu * p[i];
    vp[i] = -mu * vz[i] + nu * vp[i];
  }
}

mas_status launch_subspace_scenes(Ctx& c, const double* g, const double* z, const double* zp, const double* vz,
                                  double* p, double* vp, const int32_t* restart, mas_step_out* out) {
  ProfScope ps(c, MAS_T_SUBSPACE);
  const int S = c.S, nr = int(c.nrange);
  const int64_t n3 = 3 * c.N;
  double* xi = c.sc_acc;
  double* scal = c.sc_acc + 3 * S;
  fill_f64(c, xi, 3 * S, 0.0);
  k_ss_reduce_rng<<<dim3(nr), dim3(RB), 0, c.s>>>(c.rbeg, c.seg, g, z, zp, p, vz, vp, restart, c.partials, nr);
  const int64_t m = c.have_update ? c.mc : 0;
  if (m > 0)
    k_ss_xi_scenes<<<dim3(unsigned(std::min<int64_t>((m + RB - 1) / RB, 1024))), dim3(RB),
                     sizeof(double) * 3 * S, c.s>>>(m, c.Uidx, c.U, c.dS, z, p, c.seg, restart, S, xi);
  k_ss_final_scenes<<<dim3(S), dim3(RB), 0, c.s>>>(c.scene_r, c.partials, nr, xi, restart, zp != nullptr,
                                                   c.cfg.eps_sing, c.cfg.eps_abs, c.cfg.restart_delta, out, scal);
  k_ss_update_scenes<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, c.seg, z, vz, p, vp, scal);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

// barrier energy and infeasible count of the contacts, per scene
__global__ __launch_bounds__(RB) void k_eg_contacts_scenes(int64_t m, const int32_t* idx, const double* d,
                                                           double kappa, double dhat, const int32_t* seg, int S,
                                                           double* acc) {
  extern __shared__ double la[];
  for (int q = threadIdx.x; q < 2 * S; q += RB) la[q] = 0.0;
  __syncthreads();
  for (int64_t c = blockIdx.x * int64_t(RB) + threadIdx.x; c < m; c += int64_t(gridDim.x) * RB) {
    const int4 iv = reinterpret_cast<const int4*>(idx)[c];
    const int vi[4] = {iv.x, iv.y, iv.z, iv.w};
    int sc = -1;
#pragma unroll
    for (int j = 3; j >= 0; --j)
      if (vi[j] >= 0) sc = seg[vi[j]];
    if (sc < 0) continue;
    const double di = d[c];
    if (!(di > 0.0)) {
      __hip_atomic_fetch_add(&la[2 * sc + 1], 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else if (di < dhat) {
      double b, b1, b2;
      barrier3(di, dhat, &b, &b1, &b2);
      __hip_atomic_fetch_add(&la[2 * sc], kappa * b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 2 * S; q += RB)
    if (la[q] != 0.0) atomicAdd(&acc[q], la[q]);
}

// per scene: inertia and elasticity of its ranges (fixed order) plus its
// contacts; +inf if one of its contacts is not at a positive distance
__global__ __launch_bounds__(RB) void k_eg_final_scenes(const int64_t* scene_r, const double* part, int nblk,
                                                        const double* acc, double* E) {
  __shared__ double red[RB];
  const int sc = blockIdx.x;
  double t = 0.0;
  for (int64_t r = scene_r[sc] + threadIdx.x; r < scene_r[sc + 1]; r += RB) t += part[r] + part[nblk + r];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[sc] = acc[2 * sc + 1] > 0.0 ? INFINITY : red[0] + acc[2 * sc];
}

mas_status launch_energy_grad_scenes(Ctx& c, const double* x, const double* xt, const mas_contacts* ct,
                                     double* E, double* g) {
  const int S = c.S;
  mas_status st = launch_energy_grad(c, x, xt, ct, c.scal + 32, g);
  if (st != MAS_OK) return st;
  double* eacc = c.sc_acc + 5 * S;
  fill_f64(c, eacc, 2 * S, 0.0);
  const int64_t m = ct ? ct->m : 0;
  if (m > 0)
    k_eg_contacts_scenes<<<dim3(unsigned(std::min<int64_t>((m + RB - 1) / RB, 1024))), dim3(RB),
                           sizeof(double) * 2 * S, c.s>>>(m, ct->idx, ct->d, c.cfg.kappa, c.cfg.dhat, c.seg, S,
                                                          eacc);
  k_eg_final_scenes<<<dim3(S), dim3(RB), 0, c.s>>>(c.scene_r, c.partials, c.n_partial_blocks, eacc, E);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

__global__ void k_step_scenes(int64_t n3, const int32_t* seg, const double* x, const double* p, const double* alpha,
                              const double* scale, double* xo) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n3) return;
  const int64_t v = i / 3;
  xo[i] = x[i] + scale[seg[v]] * alpha[v >> 5] * p[i];
}

mas_status launch_step_scenes(Ctx& c, const double* x, const double* p, const double* scale, double* x_out) {
  const int64_t n3 = 3 * c.N;
  k_step_scenes<<<dim3((n3 + 255) / 256), dim3(256), 0, c.s>>>(n3, c.seg, x, p, c.alpha, scale, x_out);
  HIPCHK(hipGetLastError());
  return MAS_OK;
}

}  // namespace mas
