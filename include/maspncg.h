/*
 * maspncg.h - C ABI of the MAS-PNCG hot path for AMD MI355X (gfx950).
 *
 * The library computes the data-parallel core of one iteration of the
 * multilevel-preconditioned nonlinear conjugate gradient method for
 * Incremental Potential Contact (MAS-PNCG):
 *
 *   mas_build            RebuildMAS of Algorithm 1: Hessian snapshot and all
 *                        MAS levels (Section 3.3, supplement Section 1)
 *   mas_woodbury_update  contact classification, localized Top-K and the
 *                        per-subdomain capacitance factors (Section 4.1)
 *   mas_apply            z = P g with Woodbury-updated level 0 and frozen
 *                        coarse levels (Section 4.1.2, assembly of z_{k+1})
 *   hess_vec             y = H_base v (+ U U^T v) (Eq. for H~ in Section 4.1;
 *                        supplement Eqs. (11)-(15))
 *   pncg_subspace_step   2x2 subspace minimisation, fallback and restart
 *                        ratio (Sections 4.2-4.3; supplement Section 2)
 *
 * plus the supporting calls an iteration needs (energy and gradient of the
 * incremental potential, Section 3.1; per-subdomain safe step of Algorithm 1
 * for affine contact stencils).
 *
 * Conventions shared by every call
 * --------------------------------
 * Vertex numbering.  mas_create sorts the vertices by a 63-bit Morton code of
 * their rest positions (21 bits per axis, normalised to the bounding box,
 * ties kept in input order) and returns perm[new] = old.  Every vector and
 * every contact vertex index passed afterwards uses that library order.
 * Level-0 subdomain d holds vertices [32 d, 32 d + 32); a level-l node is a
 * run of 32^l consecutive vertices; a level-l subdomain is 32 consecutive
 * level-l nodes.  Blocks are 96 x 96 (3 DOFs per vertex or node).
 *
 * Vectors.  Device float64 arrays of length 3N, xyz interleaved per vertex.
 *
 * Contacts.  An affine distance stencil over up to four vertices:
 * key (identity, uint64; unique within a set and different from
 * 0xffffffffffffffff, which marks free slots of the library's key table),
 * idx[4] (library vertex ids, -1 padded), d (current distance) and
 * grad[12] = dd/dx.  Contacts with d >= dhat carry zero stiffness.  All
 * contact arrays are device pointers.
 *
 * Memory ownership.  The caller owns every pointer it passes.  The library
 * copies what it keeps (mesh at mas_create, the base contact set at
 * mas_build, the update columns at mas_woodbury_update) and frees its own
 * memory in mas_destroy.  Calls never free caller memory.
 *
 * Streams.  Every call is enqueued on the stream given to mas_create and
 * returns without synchronising, except where stated.  Scalar outputs are
 * written to device memory.
 *
 * Errors.  Invalid arguments and call-order mistakes return immediately
 * (MAS_ERR_INVALID_ARG, MAS_ERR_STATE).  Conditions detected by kernels
 * (non-positive pivot, non-finite input, rank overflow) set a sticky device
 * error word that mas_sync_status reports.  No call aborts the process.
 * A context is bound to one stream and is not thread-safe.
 */
#ifndef MASPNCG_H
#define MASPNCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MAS_OK = 0,
  MAS_ERR_INVALID_ARG = 1,
  MAS_ERR_STATE = 2,
  MAS_ERR_OOM = 3,
  MAS_ERR_HIP = 4,
  MAS_ERR_NOT_SPD = 5,
  MAS_ERR_NONFINITE = 6,
  MAS_ERR_RANK = 7
} mas_status;

/* Storage precision of the level-0 inverse blocks (block_prec) and of the
 * element Hessian snapshot (hess_prec: MAS_F64 or MAS_F32).  Blocks are
 * always assembled and inverted in float64 (supplement Section 1.1) and then
 * stored in the requested form when that form can hold them: with
 * kappa_d = max_i (M_d)_ii (B_d)_ii (a lower bound on the condition number of
 * the Jacobi-scaled block), a block is kept in a format of unit roundoff eps
 * only if kappa_d <= prec_guard / (20 eps); otherwise it is promoted
 * (BF16/FP16 -> FP32 -> FP64), so no stored block loses definiteness.  BF16
 * and FP16 blocks carry a per-row symmetric scaling sigma_i = B_ii^1/2.
 * Products with stored blocks accumulate in float64. */
typedef enum { MAS_F64 = 0, MAS_F32 = 1, MAS_BF16 = 2, MAS_F16 = 3 } mas_prec;

typedef struct {
  int32_t num_levels;   /* MAS levels including level 0, 1..6 (supplement 1.2) */
  int32_t max_rank;     /* Top-K per subdomain, 0..32 (Section 4.1.1, K = 8) */
  double cos_rot;       /* cosine of the rotation threshold (25 degrees) */
  double restart_delta; /* restart threshold delta (Section 4.3, 0.3) */
  double eps_sing;      /* relative singularity tolerance (supplement 2.4.3) */
  double eps_abs;       /* absolute floor of the singularity test */
  double kappa;         /* barrier stiffness: B = kappa sum_c b(d_c) */
  double dhat;          /* barrier activation distance */
  double h;             /* time step */
  double gravity[3];    /* external acceleration used for x~ */
  int32_t block_prec;   /* requested mas_prec of level-0 blocks */
  int32_t coarse_prec;  /* requested mas_prec of levels >= 1 */
  int32_t hess_prec;    /* MAS_F64 or MAS_F32 element Hessian snapshot */
  int32_t deterministic; /* 1: every sum in a fixed order, so that repeated calls
                            on the same inputs give bitwise equal results (the
                            sums of the fast mode follow the order of atomics) */
  double prec_guard;    /* promotion threshold factor (default 0.5; 0: never promote) */
  /* Capacities.  All device memory is allocated by mas_create; no later call
   * allocates.  0 picks the default shown. */
  int64_t max_contacts; /* largest base or current contact set (max(2 N, 65536)) */
  int64_t max_tris;     /* largest triangle list of mas_constraint_set (2 N + 64) */
  int64_t max_edges;    /* largest edge list of mas_constraint_set (3 N + 64) */
  int32_t precond;      /* MAS_PRECOND_MAS (the method) or MAS_PRECOND_BJ3 */
  int32_t hierarchy;    /* MAS_HIER_MORTON or MAS_HIER_CONNECTIVITY */
} mas_config;

/* Vertex order that defines the hierarchy (a level-l node is a run of 32^l
 * consecutive vertices, a subdomain a run of 32 nodes).  MAS_HIER_MORTON:
 * Morton order of the rest positions.  MAS_HIER_CONNECTIVITY: the
 * connectivity-aware hierarchy of supplement Section 1.2 (greedy
 * aggregation over the graph of vertices that share a tet): vertices
 * numbered component by component (Morton order inside); each cluster of
 * 32 nodes grows from the smallest unassigned node by the smallest
 * unassigned node adjacent to its members (else the smallest unassigned
 * node); the clusters of level l are the nodes of level l + 1, aggregated
 * the same way; a partial node closes the last cluster.  The mesh's
 * contact links are edges of the graph too (the reconnection of supplement
 * Section 1.2, taken once: the order is computed by mas_create on the host
 * and fixes the data layout, so contacts that form later do not regroup
 * it). */
#define MAS_HIER_MORTON 0
#define MAS_HIER_CONNECTIVITY 1

/* Preconditioner of a context.  MAS_PRECOND_BJ3 is the comparison
 * preconditioner of the ablation study (Section 5, preconditioner
 * efficacy): the 3x3 block-Jacobi inverse of H~ (each vertex's diagonal
 * block of H_base, plus that of U U^T after mas_woodbury_update), inverted
 * by Cholesky in float64.  In that mode mas_build assembles the level-0
 * blocks but inverts no MAS level, mas_woodbury_update classifies (for H~)
 * and rebuilds the vertex blocks instead of Top-K and capacitance, and
 * mas_apply returns z_i = B_i^-1 g_i; mas_get_block and the MAS queries
 * have nothing to report.  Not combinable with deterministic mode. */
#define MAS_PRECOND_MAS 0
#define MAS_PRECOND_BJ3 1

/* Tetrahedral mesh, host pointers, original vertex numbering.  tets must
 * have positive orientation at rest. */
typedef struct {
  int64_t num_vertices;
  int64_t num_tets;
  const double* rest_x;   /* 3N */
  const int32_t* tets;    /* 4T */
  const double* density;  /* T */
  const double* youngs;   /* T */
  const double* poisson;  /* T */
  /* Contact links for the connectivity-aware hierarchy (supplement Section
   * 1.2, reconnection: primitives in close proximity join the adjacency
   * graph): num_links pairs of original vertex ids (2 * num_links int32,
   * host), read by mas_create and mas_vertex_order only when the hierarchy
   * is MAS_HIER_CONNECTIVITY; may be 0 / NULL. */
  int64_t num_links;
  const int32_t* links;
  /* Independent scenes in one mesh (the batched form): scene s owns the
   * original vertices [scene_offsets[s], scene_offsets[s + 1]) (host,
   * num_scenes + 1 entries, 0 first, num_vertices last, increasing); no tet
   * or link may join two scenes.  num_scenes 0 or 1 (and NULL offsets):
   * one scene.  The library then orders vertices scene by scene (Morton
   * order inside each; MAS_HIER_MORTON only), cuts its vertex ranges at
   * scene starts, and the *_scenes calls below take per-scene scalars.
   * Coarse MAS nodes are runs of 32^l library vertices and may span the end
   * of one scene and the start of the next (P stays SPD on the union). */
  int32_t num_scenes;
  const int64_t* scene_offsets;
} mas_mesh;

/* Contact stencils, device pointers, library vertex numbering. */
typedef struct {
  int64_t m;
  const uint64_t* key;    /* m */
  const int32_t* idx;     /* 4m, -1 padded */
  const double* d;        /* m */
  const double* grad;     /* 12m */
} mas_contacts;

/* Scalars written by pncg_subspace_step (device memory). */
typedef struct {
  double mu, nu;          /* p_{k+1} = -mu z + nu p_k */
  double r;               /* restart ratio |g^T z_prev| / (g^T z) */
  double gz, gp, gzp;     /* g^T z, g^T p_k, g^T z_prev */
  double A11, A12, A22;   /* entries of the 2x2 system (supplement Eq. (19)) */
  double gnorm2, znorm2;  /* squared norms of g and z */
  int32_t fallback;       /* 1 if mu = 1, nu = 0 was taken */
  int32_t restart_next;   /* r > restart_delta */
  int32_t restart_used;   /* the restart form (nu = 0) was used */
  int32_t reserved;
} mas_step_out;

/* Counters of the last mas_woodbury_update and mas_safe_step (host copy,
 * filled by mas_read_stats).  The classification follows Section 4.1.1:
 * a current contact with k > 0 is new (no base entry with k > 0), rotated
 * (its normal turned past the rotation threshold; dS = k), stiffened
 * (dS = k - k_base > 0) or softened (dS = 0). */
typedef struct {
  int64_t contacts;        /* current contacts of the last mas_woodbury_update */
  int64_t active;          /* of them with k > 0 (d < dhat) */
  int64_t n_new, n_rotated, n_stiffened, n_softened;
  int64_t rank_sum;        /* sum over level-0 subdomains of the kept rank r_d */
  int32_t rank_max;        /* largest r_d */
  int32_t safe_rounds;     /* damping rounds of the last mas_safe_step that damped a subdomain */
  int64_t safe_left;       /* stencils still closing below 0.05 d after the last round
                              (> 0: the any-mix fallback bound was taken) */
  int64_t alpha_hist[8];   /* level-0 subdomains by the last safe step alpha_d: [0] alpha = 1,
                              [i] alpha in [2^-i, 2^(1-i)) for i = 1..6, [7] alpha < 2^-6 */
} mas_iter_stats;

/* Fills cfg with the paper's stated defaults (K = 8, 25 degrees, delta = 0.3,
 * eps_sing = 1e-12) and float64 storage. */
void mas_default_config(mas_config* cfg);

/* Creates a context: Morton order, element rest quantities (Dm^-1, volume,
 * Lame parameters from Young's modulus and Poisson's ratio, lumped masses),
 * subdomain tables.  perm_out (host, N) receives perm[new] = old.
 * Allocates all device memory the context will use, sized by the mesh and
 * the capacities of cfg; no later call allocates.  stream may be NULL
 * (default). */
mas_status mas_create(const mas_config* cfg, const mas_mesh* mesh, void* hip_stream,
                      void** ctx_out, int32_t* perm_out);

mas_status mas_destroy(void* ctx);

/* RebuildMAS (Algorithm 1; supplement Section 1).  At x_base (device, 3N):
 * per-tet SNH Hessians with eigenvalues of d2Psi/dF2 clamped at zero, the
 * base contact set (copied; k = kappa b''(d), n = grad), level-0 blocks
 * S_d H_base S_d^T and Galerkin coarse blocks of every level, all inverted in
 * float64 and stored at the configured precision.  Clears the Woodbury
 * update.  A non-positive pivot sets MAS_ERR_NOT_SPD.  base->m must not
 * exceed max_contacts (MAS_ERR_INVALID_ARG). */
mas_status mas_build(void* ctx, const double* x_base, const mas_contacts* base);

/* Sparse-Input Woodbury update (Section 4.1).  Classifies every current
 * contact against the base set by key (new, rotated: cos < cos_rot, stiffening,
 * softening), keeps the untruncated update columns u = sqrt(dS) n for
 * hess_vec and the subspace step, selects per level-0 subdomain the max_rank
 * candidates of largest dS (ties: smaller key first), and factors the
 * capacitance I + U_d^T B_d U_d in float64.  rank_hist (device, max_rank+1
 * int32, nullable) receives the histogram of per-subdomain ranks.
 * curr->m must not exceed max_contacts (MAS_ERR_INVALID_ARG).  A
 * capacitance pivot that is not positive (rounding, in exact arithmetic the
 * matrix is SPD) drops that column and the later ones, which rank lowest by
 * dS: the subdomain keeps the factor of its leading columns, and the next
 * mas_sync_status returns MAS_ERR_RANK naming the subdomain.  A non-finite
 * distance sets MAS_ERR_NONFINITE. */
mas_status mas_woodbury_update(void* ctx, const mas_contacts* curr, int32_t* rank_hist);
/* (W_d = B_d U_d is kept in float64: its product with C_d^-1 cancels against
 * B_d along stiff contact directions.) */

/* z = P g (device vectors, 3N, must not alias): level-0 blocks with the
 * Woodbury correction z_d = B_d g_d - W_d C_d^-1 U_d^T B_d g_d, plus
 * C_(l)^T M_(l)^-1 C_(l) g for every coarse level.  A non-finite entry of g
 * sets MAS_ERR_NONFINITE. */
mas_status mas_apply(void* ctx, const double* g, double* z);

/* y = H_base v, plus U U^T v when with_update != 0 (device, 3N, no alias).
 * H_base = M + sum_e S_e^T H_e S_e + sum_{c in base} k_c n_c n_c^T frozen at
 * the last mas_build.  A non-finite entry of v sets MAS_ERR_NONFINITE. */
mas_status hess_vec(void* ctx, const double* v, double* y, int32_t with_update);

/* 2x2 subspace step (Section 4.2; supplement Section 2.4).  Inputs g, z,
 * z_prev, v_z = H_base z; in/out p (p_k -> p_{k+1}) and v_p (H_base p_k ->
 * H_base p_{k+1}, updated by linearity).  restart != 0 takes mu = g^T z /
 * z^T H~ z, nu = 0 (Algorithm 1).  z_prev may be NULL (r = 0).  out is a
 * device pointer.  Singular systems fall back to mu = 1, nu = 0. */
mas_status pncg_subspace_step(void* ctx, const double* g, const double* z, const double* z_prev,
                              const double* v_z, double* p, double* v_p, int32_t restart,
                              mas_step_out* out);

/* pncg_subspace_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the reduction
 * workspace (11 per-block partial sums for each of max(1024, vertex ranges)
 * blocks, then mu and nu) lives in a fixed 768 KiB device array that the
 * library's code object holds on each device (up to 98,304 doubles, enough
 * for about 8,900 vertex ranges, on the order of 10M vertices); the call
 * makes no allocation and no host synchronisation.  A context needing more
 * gives MAS_ERR_INVALID_ARG; before mas_build MAS_ERR_STATE.  Every call on
 * one device shares that array (it keeps the last call's contents, and every
 * entry is written before it is read): calls that overlap in time on one
 * device, from contexts on different streams, race and must be ordered by
 * the caller. */
mas_status pncg_subspace_step_noalloc(void* ctx, const double* g, const double* z, const double* z_prev,
                                      const double* v_z, double* p, double* v_p, int32_t restart,
                                      mas_step_out* out);

/* Direction rules of the search-direction comparison (Section 5): classic
 * preconditioned nonlinear CG, d = -z + beta d_prev, beta by
 *   MAS_BETA_FR  Fletcher-Reeves    g^T z / (g_prev^T z_prev)
 *   MAS_BETA_CD  conjugate descent  g^T z / (-d_prev^T g_prev)
 *   MAS_BETA_DK  Dai-Kou            y^T z / (d^T y) - (y^T (z - z_prev) /
 *                d^T y) (d^T g) / (d^T y), y = g - g_prev
 * (the published formulas with g^T g replaced by g^T z; the paper names the
 * rules without printing them), then p = alpha d with alpha = -g^T d /
 * d^T H~ d.  Inputs g, z, v_z = H_base z, z_prev (may be NULL on a restart:
 * r = 0) and, unless restart != 0, g_prev (device, 3N; g_prev is not read on
 * a restart); in/out d (d_prev -> d) and v_d (H_base d, updated by
 * linearity); out p (3N, the step for the safe step).  restart != 0 takes
 * beta = 0 (the same step as pncg_subspace_step's restart form).  A
 * non-positive denominator or a d that is not a descent direction gives
 * d = -z; d^T H~ d <= 0 gives alpha = 1; either sets out->fallback.  out
 * (device) holds alpha in mu and beta in nu; r and restart_next as for the
 * subspace step.  Bad rule or missing g_prev / z_prev: MAS_ERR_INVALID_ARG. */
#define MAS_BETA_FR 1
#define MAS_BETA_CD 2
#define MAS_BETA_DK 3
mas_status pncg_beta_step(void* ctx, int32_t rule, const double* g, const double* g_prev, const double* z,
                          const double* z_prev, const double* v_z, double* d, double* v_d, int32_t restart,
                          double* p, mas_step_out* out);

/* Per-scene forms of the iteration for a mesh of several scenes (the same
 * calls serve one scene).  Each scene takes its own 2x2 step (Section 4.2;
 * supplement Section 2.4) from sums over its own vertices and update
 * columns:
 *   pncg_subspace_step_scenes: as pncg_subspace_step, with restart (device
 *     int32, num_scenes) and out (device, num_scenes) per scene; z_prev may be
 *     NULL (r = 0);
 *   mas_energy_grad_scenes: E (device, num_scenes) per scene and the gradient
 *     g (device, 3N, nullable) as mas_energy_grad;
 *   mas_step_scenes: x_out = x + scale_s alpha_d p with the per-subdomain steps
 *     of the last mas_safe_step and a scale per scene (device, num_scenes);
 *   mas_scenes: the scene count and, if voff is not NULL, the library vertex
 *     offset of each scene (host int64, num_scenes + 1).
 * Not available in deterministic mode (MAS_ERR_STATE). */
mas_status pncg_subspace_step_scenes(void* ctx, const double* g, const double* z, const double* z_prev,
                                     const double* v_z, double* p, double* v_p, const int32_t* restart,
                                     mas_step_out* out);
mas_status mas_energy_grad_scenes(void* ctx, const double* x, const double* x_tilde, const mas_contacts* c,
                                  double* E, double* g);
mas_status mas_step_scenes(void* ctx, const double* x, const double* p, const double* scale, double* x_out);
mas_status mas_scenes(void* ctx, int32_t* num_scenes, int64_t* voff);

/* Incremental potential (Section 3.1) at x: E (device scalar) and, if g is
 * not NULL, its gradient (device, 3N).  Contacts with d <= 0 make E = +inf.
 * In deterministic mode c->m must not exceed max_contacts when g is given
 * (the contact terms are gathered per vertex in ascending contact order). */
mas_status mas_energy_grad(void* ctx, const double* x, const double* x_tilde,
                           const mas_contacts* c, double* E, double* g);

/* x~ = x^t + h v^t + h^2 gravity (device vectors). */
mas_status mas_inertial_target(void* ctx, const double* x_t, const double* v_t, double* x_tilde);

/* The next time step of implicit Euler (Algorithm 1's inputs x^t, v^t): after
 * a step from x_old to x_new, v = (x_new - x_old) / h and
 * x~ = x_new + h v + h^2 gravity.  Device vectors of 3N; v or x_tilde may be
 * NULL; x_new and x_old may not alias the outputs. */
mas_status mas_next_frame(void* ctx, const double* x_new, const double* x_old, double* v, double* x_tilde);

/* Distances of affine stencils d = grad . x[idx] - off (device arrays). */
mas_status mas_stencil_distance(void* ctx, const double* x, int64_t m, const int32_t* idx,
                                const double* grad, const double* off, double* d_out);

/* Per-subdomain safe steps for affine stencils (cand; Section 4.4 and
 * supplement Section 3, relative displacement of the stencil's vertices):
 * a stencil closing at the rate s_c = -sum_j grad_cj . p_j > 0 allows
 * alpha_c = max(0, min(1, 0.9 d_c / s_c)); alpha_d = min(1, min over stencils
 * touching subdomain d).  Vertices of one stencil in different subdomains
 * move with different steps: in up to 16 damping rounds, run on the device
 * without host synchronisation (a round after one that found nothing does
 * no work), every subdomain of a stencil whose distance would fall below
 * 0.05 d_c under the mixed steps has its step halved.  Writes
 * x_out = x + scale * alpha_{sub(v)} p_v (device, 3N).  If a stencil is
 * still closing below 0.05 d_c after the last round, every subdomain takes
 * instead the bound that holds for any mix of steps: a stencil allows
 * min(1, 0.9 d_c / sum_j max(0, -grad_cj . p_j)), alpha_d the smallest over
 * the stencils touching d, so no stencil comes below 0.1 d_c; the number of
 * such stencils is mas_iter_stats.safe_left.
 * cand == NULL reuses the step sizes of the previous call (line-search
 * halving only changes scale).  alpha (device, D_0, nullable) receives the
 * step sizes.  cand->m must not exceed max_contacts. */
mas_status mas_safe_step(void* ctx, const double* x, const double* p, const mas_contacts* cand,
                         double scale, double* alpha, double* x_out);

/* Conservative CCD of point-triangle and edge-edge pairs (supplement
 * Section 3.4, Algorithms 1 and 2).  Per pair: the lower bound
 * alpha_l = d_min / l, d_min = 0.9 dist (the supplement leaves d_min open;
 * the margin makes a root before alpha_l a crossing of the plane away from
 * the other primitive, and finds a pair that meets exactly at dist / l),
 * with l the largest relative displacement along p of a
 * vertex of one primitive and a vertex of the other (supplement Eqs. (29),
 * (31)); then the coplanarity cubic f(t), the signed volume of the four
 * vertices at x + t p, is cut at its critical points into monotonic pieces
 * on [max(0, alpha_l), 1] and the first piece whose ends differ in sign is
 * bisected 16 times toward the safe side (a piece entered past alpha_l
 * returns its start); 1 if no piece changes sign.
 * x, p: device 3N.  pairs: device int32 4m, library vertex ids,
 * point-triangle (P, T0, T1, T2) or edge-edge (E1a, E1b, E2a, E2b); kind:
 * device uint8 m, 0 = point-triangle, 1 = edge-edge; dist: device float64 m,
 * the pairs' current distances (a lower bound is safe).  alpha_pair
 * (device float64 m, nullable) receives the pair steps; alpha (device
 * float64 D_0, nullable) receives per level-0 subdomain the smallest step
 * of the pairs with a vertex in it, 1 where there is none (Algorithm 1's
 * per-subdomain alpha_d).  A pair with a vertex id outside [0, N) gets
 * step 0, takes no part in alpha, and the next mas_sync_status returns
 * MAS_ERR_INVALID_ARG. */
mas_status mas_ccd_steps(void* ctx, const double* x, const double* p, int64_t m, const int32_t* pairs,
                         const uint8_t* kind, const double* dist, double* alpha_pair, double* alpha);

/* Per-subdomain safe steps on point-triangle and edge-edge pairs (Algorithm
 * 1: ConservativeCCD giving {alpha_d}, x + sum_d S_d^T alpha_d S_d p;
 * Section 4.4).  alpha_d starts as the smallest mas_ccd_steps step along p
 * of the candidate pairs with a vertex in subdomain d, capped at
 * radius / (2 max_v |p_v|): candidates must include every pair closer than
 * radius, and the cap keeps pairs farther apart from meeting under any
 * steps.  Vertices of one pair in subdomains with different steps move by
 * different fractions of p: in up to 16 damping rounds on the device, a
 * pair whose CCD along its vertices' actual displacements finds a root
 * before 1 halves the steps of its subdomains; if one is left after the last
 * round, every subdomain takes the smallest alpha_d (one common step along
 * p, which the CCD covers), counted in mas_iter_stats.safe_left.  Writes
 * x_out = x + scale alpha_{sub(v)} p_v (device 3N, 0 <= scale <= 1); alpha
 * (device D_0, nullable) receives the steps; mas_safe_step with cand = NULL
 * reuses them with another scale.  pairs, kind, dist (device, m >= 0) as
 * for mas_ccd_steps (dist: current distances, a lower bound is safe).
 * MAS_ERR_INVALID_ARG for radius <= 0, scale outside [0, 1] or null
 * arrays. */
mas_status mas_ccd_safe_step(void* ctx, const double* x, const double* p, double radius, int64_t m,
                             const int32_t* pairs, const uint8_t* kind, const double* dist, double scale,
                             double* alpha, double* x_out);

/* Narrow phase of the contact set: per point-triangle or edge-edge pair the
 * distance d_c that the barrier of Section 3.1 takes, and its gradient
 * n = grad d_c of the projected contact Hessian (Section 4.1; the update
 * columns u = sqrt(k) n of supplement Eq. (11)).  d_c is the unsigned
 * Euclidean distance between the two primitives; grad d_c = w_j n_hat on
 * the vertices of the first primitive and -w_j n_hat on those of the
 * second, with w the weights of the closest points (1 for the point, barycentric on the triangle, 1 - s and s
 * on an edge) and n_hat the unit vector from the second closest point to the
 * first; it is zero where d_c = 0.  Parallel edges have many closest pairs:
 * the one on the first edge's first vertex or on a segment end is taken.
 * x: device 3N.  pairs, kind: as for mas_ccd_steps.  dist: device float64
 * m.  grad (device float64 12m, vertex-major: 12 i + 3 j + axis; nullable)
 * and dist together are the d and grad of a mas_contacts set over the same
 * idx.  type (device uint8 m, nullable) receives the closest features:
 * point-triangle 0-2 vertex T0, T1, T2, 3 edge T0T1, 4 edge T1T2, 5 edge
 * T2T0, 6 face; edge-edge 3 a + b with a, b = 0 first vertex, 1 second
 * vertex, 2 interior of the first and second edge.  A pair with a vertex id
 * outside [0, N) gets dist = NaN, grad = 0, type = 255, and the next
 * mas_sync_status returns MAS_ERR_INVALID_ARG. */
mas_status mas_contact_distances(void* ctx, const double* x, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                 double* dist, double* grad, uint8_t* type);

/* ComputeConstraintSet of Algorithm 1: every point-triangle pair (a surface
 * vertex and a surface triangle not containing it) and every edge-edge
 * pair (two surface edges without a common vertex, once, the edge listed
 * first in edges first) with distance d_c < dhat (d_c, n = grad d_c and
 * the layouts as for mas_contact_distances).  Broad phase: a hashed
 * uniform grid of cell side (largest axis extent of a triangle or edge) +
 * 2 dhat; narrow phase as mas_contact_distances.
 * x: device 3N.  verts (device int32 nv), tris (device int32 3nt), edges
 * (device int32 2ne): library vertex ids.  Outputs, device, capacity cap:
 * pairs int32 4cap (P, T0, T1, T2 or E1a, E1b, E2a, E2b), kind uint8 cap
 * (0 point-triangle, 1 edge-edge), dist float64 cap, grad float64 12cap
 * (nullable), key uint64 cap (nullable): the contact's identity for the
 * classification of Section 4.1.1, tag 2 (point-triangle) or 3 (edge-edge)
 * in bits 60-63, then 30 bits each for the two primitives' indices in the
 * lists given (the vertex's index in verts and the triangle's in tris, or
 * the two edges' indices in edges, the smaller first), so a pair keeps its
 * key across calls over the same lists (nv, nt, ne < 2^30).  *count (host)
 * receives the number of pairs found; only the
 * first min(count, cap) are written, in no fixed order (call again with a
 * larger cap when count > cap).  Synchronises the stream (it reads the
 * largest primitive extent, which sets the cell side, and the table sizes
 * back).  The grid tables are allocated by mas_create for max_tris and
 * max_edges primitives with up to 8 cell entries each.  Errors:
 * MAS_ERR_INVALID_ARG for nt > max_tris, ne > max_edges, more cell entries
 * than the tables hold, an id outside [0, N),
 * dhat <= 0, or coordinates so large against the cell side that cell
 * indices would exceed 1e15; MAS_ERR_NONFINITE for a non-finite
 * coordinate of a listed vertex; both before any pair is written. */
mas_status mas_constraint_set(void* ctx, const double* x, double dhat, int64_t nv, const int32_t* verts, int64_t nt,
                              const int32_t* tris, int64_t ne, const int32_t* edges, int64_t cap, int32_t* pairs,
                              uint8_t* kind, double* dist, double* grad, uint64_t* key, int64_t* count);

/* Synchronises the stream and returns the sticky device error (and clears
 * it); msg (nullable) receives a description. */
mas_status mas_sync_status(void* ctx, char* msg, int32_t msg_len);

/* Synchronises the stream and fills *out (host) from the device counters
 * of the last mas_woodbury_update and mas_safe_step. */
mas_status mas_read_stats(void* ctx, mas_iter_stats* out);

/* Sizes: N, T, number of levels, D_l for l < 6. */
mas_status mas_query(void* ctx, int64_t* N, int64_t* T, int32_t* levels, int64_t* nsub /*6*/);

/* The vertex order mas_create would use for this mesh (host only, no
 * device call, no context): perm_out (host, N) receives perm[new] = old
 * vertex id for the hierarchy kind (MAS_HIER_MORTON or
 * MAS_HIER_CONNECTIVITY, supplement Section 1.2) and num_levels (1..6).
 * Only num_vertices, num_tets, rest_x, tets and the links of the mesh are
 * read. */
mas_status mas_vertex_order(const mas_mesh* mesh, int32_t num_levels, int32_t hierarchy, int32_t* perm_out);

/* Number of blocks of level l stored in each precision by the last
 * mas_build (counts[4] indexed by mas_prec, host). */
mas_status mas_block_precisions(void* ctx, int32_t level, int64_t* counts);

/* Copies block d of level l, dequantised to float64, as a dense 96x96
 * row-major host array (for verification). */
mas_status mas_get_block(void* ctx, int32_t level, int64_t d, double* out_host);

/* Copies the Top-K selection: per level-0 subdomain its rank (host int32 D_0)
 * and the selected current-contact indices (host int32 D_0 x max_rank, -1 when
 * unused), in ranking order. */
mas_status mas_get_selection(void* ctx, int32_t* rank_host, int32_t* sel_host);

/* Kernel timers.  While enabled, the library records a HIP event pair on its
 * stream around the named kernel (or call) every time it runs, so that
 * durations are measured on the stream the kernels are launched on. */
typedef enum {
  MAS_T_APPLY_L0 = 0,     /* level-0 block apply kernel of mas_apply */
  MAS_T_APPLY = 1,        /* the whole mas_apply call */
  MAS_T_HV_TETS = 2,      /* element kernel of hess_vec */
  MAS_T_HESSVEC = 3,      /* the whole hess_vec call */
  MAS_T_UPDATE = 4,       /* the whole mas_woodbury_update call */
  MAS_T_CAPACITANCE = 5,  /* capacitance kernel of mas_woodbury_update */
  MAS_T_BUILD = 6,        /* the whole mas_build call */
  MAS_T_ENERGY = 7,       /* the whole mas_energy_grad call */
  MAS_T_SUBSPACE = 8,     /* the whole pncg_subspace_step call */
  MAS_T_CCD = 9,          /* the whole mas_ccd_steps call */
  MAS_T_CONTACT = 10,     /* the whole mas_contact_distances call */
  MAS_T_CSET = 11,        /* the whole mas_constraint_set call */
  MAS_T_COUNT = 12
} mas_timer;

/* Enables (1) or disables (0) the kernel timers; enabling clears them. */
mas_status mas_profile_enable(void* ctx, int32_t enable);

/* Restricts the timers recorded while enabled to those whose bit (1 << t)
 * is set in mask (default: all).  Each timed launch adds an event pair to
 * the stream, so a timed region that must not be slowed down records only
 * the timers it reports. */
mas_status mas_profile_select(void* ctx, uint32_t mask);

/* Synchronises the stream and returns the summed duration (ms) and number of
 * timed launches of one timer since the last read, then clears it. */
mas_status mas_profile_read(void* ctx, int32_t timer, double* total_ms, int64_t* count);

/* Returns a static string naming a status code. */
const char* mas_status_string(mas_status s);

#ifdef __cplusplus
}
#endif

#endif /* MASPNCG_H */
