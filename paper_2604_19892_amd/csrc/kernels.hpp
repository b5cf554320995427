// Host-side launchers of the library kernels (one definition per .hip file).
#pragma once

#include "common.hpp"

namespace mas {

// k_util.hip -----------------------------------------------------------
// Buckets stencils into per-level-0-subdomain lists: the distinct
// subdomains (v >> 5) of the vertices j with bit j of pm[i] set (part_mask
// of the stencil's 12-vector, zero for a stencil left out).
mas_status bucket_by_subdomain(Ctx& c, int64_t m, const int32_t* idx, const uint8_t* pm, int32_t* cnt,
                               int32_t* off, int32_t* list);
// the same into D buckets map[v] (map non-null) or v / div
mas_status bucket_stencils(Ctx& c, int div, const int32_t* map, int64_t D, int64_t m, const int32_t* idx,
                           const uint8_t* pm, int32_t* cnt, int32_t* off, int32_t* list);

// deterministic mode: per-vertex incidence lists (c.inc_off, c.inc_list) of
// the stencils with w[c] > 0 (all when w is null), each list ascending
mas_status build_incidence(Ctx& c, int64_t m, const int32_t* idx, const double* w);
// out[0..n1) = exclusive prefix sums of in[0..n1) (in == out allowed);
// n1 must not exceed c.scan_cap
mas_status exclusive_scan_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n1);
// scratch (int32 elements) that scans of up to n items need
int64_t scan_scratch_elems(int64_t n);
// one-thread store of a counter (graph-capturable, unlike a memset)
__global__ void k_set_u32(uint32_t* p, uint32_t v);
// p[0..n) = v with a fill kernel (graph-capturable, unlike a memset)
void fill_i32(Ctx& c, int32_t* p, int64_t n, int32_t v);
void fill_f64(Ctx& c, double* p, int64_t n, double v);

// k_invert.hip ---------------------------------------------------------
// the blocks of the levels [lo, hi), for one inversion launch
struct InvLevels {
  int lo, hi;
  int64_t nsub[MAXL], nodes[MAXL];
  const double* acc[MAXL];
  void* blk[MAXL];
  float* scale[MAXL];
  uint8_t* bprec[MAXL];
  int prec[MAXL];
  double* acc_next;  // when set, the node-block sums of each block go there
};
// inverts the assembled blocks of the levels [lo, hi) (FP64 MFMA) in one
// launch and stores them in their chosen precision; with acc_next (a launch
// of one level l), completes the diagonal node blocks of level l + 1
void launch_invert_mfma(Ctx& c, int lo, int hi, double* acc_next);

// k_setup.hip ----------------------------------------------------------
mas_status launch_rest(Ctx& c, const double* X, const double* rho, const double* E, const double* nu,
                       double* tmass, const int32_t* voff, const int32_t* vt);
mas_status launch_inertial(Ctx& c, const double* xt, const double* vt, double* xtil);
mas_status launch_next_frame(Ctx& c, const double* xn, const double* xo, double* v, double* xtil);
mas_status launch_stencil_distance(Ctx& c, const double* x, int64_t m, const int32_t* idx,
                                   const double* grad, const double* off, double* d);

// k_build.hip ----------------------------------------------------------
mas_status launch_elem_hessians(Ctx& c, const double* x_base);
mas_status launch_base_contacts(Ctx& c, const mas_contacts* b);
// the blocks of every level: assembly, coarse diagonal node blocks, inversion
mas_status launch_level0_build(Ctx& c);

// k_woodbury.hip -------------------------------------------------------
mas_status launch_woodbury(Ctx& c, const mas_contacts* cur, int32_t* rank_hist);

// k_apply.hip ----------------------------------------------------------
mas_status launch_apply(Ctx& c, const double* g, double* z);

// k_jacobi.hip ---------------------------------------------------------
// 3x3 block-Jacobi comparison preconditioner (precond = MAS_PRECOND_BJ3)
mas_status launch_bj_build(Ctx& c);
mas_status launch_bj_update(Ctx& c, int64_t m);
mas_status launch_bj_apply(Ctx& c, const double* g, double* z);

// k_hessvec.hip --------------------------------------------------------
mas_status launch_hessvec(Ctx& c, const double* v, double* y, int with_update);

// k_pncg.hip -----------------------------------------------------------
mas_status launch_energy_grad(Ctx& c, const double* x, const double* xt, const mas_contacts* ct,
                              double* E, double* g);
mas_status launch_subspace(Ctx& c, const double* g, const double* z, const double* zp,
                           const double* vz, double* p, double* vp, int restart, mas_step_out* out);
// the subspace step with its reduction workspace given by the caller:
// subspace_workspace_elems(c) doubles, partials first, then mu and nu
int64_t subspace_workspace_elems(const Ctx& c);
mas_status launch_subspace_ws(Ctx& c, const double* g, const double* z, const double* zp, const double* vz,
                              double* p, double* vp, int restart, mas_step_out* out, double* part,
                              double* scal);
// batched form: per-scene step scalars, energies and step scales
mas_status launch_subspace_scenes(Ctx& c, const double* g, const double* z, const double* zp, const double* vz,
                                  double* p, double* vp, const int32_t* restart, mas_step_out* out);
mas_status launch_energy_grad_scenes(Ctx& c, const double* x, const double* xt, const mas_contacts* ct,
                                     double* E, double* g);
mas_status launch_step_scenes(Ctx& c, const double* x, const double* p, const double* scale, double* x_out);
// comparison direction rules (rule: MAS_BETA_FR, MAS_BETA_CD, MAS_BETA_DK)
mas_status launch_beta(Ctx& c, int rule, const double* g, const double* g_prev, const double* z,
                       const double* z_prev, const double* vz, double* d, double* vd, int restart, double* p,
                       mas_step_out* out);
mas_status launch_safe_step(Ctx& c, const double* x, const double* p, const mas_contacts* cand,
                            double scale, double* alpha, double* x_out);
mas_status launch_step_with(Ctx& c, const double* x, const double* p, double scale, double* alpha,
                            double* x_out);

// k_ccd.hip ------------------------------------------------------------
mas_status launch_ccd_safe_step(Ctx& c, const double* x, const double* p, double radius, int64_t m,
                                const int32_t* pairs, const uint8_t* kind, const double* dist, double scale,
                                double* alpha, double* x_out);
mas_status launch_ccd(Ctx& c, const double* x, const double* p, int64_t m, const int32_t* pairs,
                      const uint8_t* kind, const double* dist, double* alpha_pair, double* alpha);
mas_status launch_contact_distances(Ctx& c, const double* x, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                    double* dist, double* grad, uint8_t* type);
mas_status launch_constraint_set(Ctx& c, const double* x, double dhat, int64_t nv, const int32_t* verts, int64_t nt,
                                 const int32_t* tris, int64_t ne, const int32_t* edges, int64_t cap, int32_t* pairs,
                                 uint8_t* kind, double* dist, double* grad, uint64_t* key, int64_t* count);

}  // namespace mas
