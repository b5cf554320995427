// C ABI entry points: argument checks, context lifetime, call order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <numeric>
#include <queue>
#include <new>
#include <vector>

#include "kernels.hpp"

namespace mas {

struct Prof {
  bool on = false;
  uint32_t mask = 0xffffffffu;  // timers recorded while on (bit t: timer t)
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> done[MAS_T_COUNT];
  hipEvent_t open[MAS_T_COUNT] = {};
};

static hipEvent_t prof_take(Prof& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(Ctx& c, int t) {
  if (!c.prof || !c.prof->on || t < 0 || t >= MAS_T_COUNT || !((c.prof->mask >> t) & 1u)) return;
  hipEvent_t e = prof_take(*c.prof);
  if (!e) return;
  hipEventRecord(e, c.s);
  c.prof->open[t] = e;
}

void prof_end(Ctx& c, int t) {
  if (!c.prof || !c.prof->on || t < 0 || t >= MAS_T_COUNT || !c.prof->open[t]) return;
  hipEvent_t e = prof_take(*c.prof);
  if (!e) return;
  hipEventRecord(e, c.s);
  c.prof->done[t].push_back({c.prof->open[t], e});
  c.prof->open[t] = nullptr;
}

}  // namespace mas

using namespace mas;

// Fixed workspace of pncg_subspace_step_noalloc: the per-block partial sums
// of the subspace step's reductions and its two scalars, in device memory
// that the code object itself holds (each device that loads the library has
// its own copy until the process ends), so that call allocates nothing.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// kernels only ever receive the address from hipGetSymbolAddress, looked up
// once per device by mas_create with that device current.
constexpr int64_t SCRATCH_DOUBLES = 98304;  // 768 KiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[MAX_DEVICES] = {};

// this device's address of `scratch` (the current device)
mas_status scratch_address(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return MAS_ERR_HIP;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MAS_ERR_HIP;
    scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = scratch_dev[dev];
  return MAS_OK;
}

}  // namespace

namespace {

Ctx* as_ctx(void* p) { return reinterpret_cast<Ctx*>(p); }

template <typename T>
mas_status dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess) return MAS_ERR_OOM;
  return MAS_OK;
}

mas_status dalloc_bytes(void** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(p, n) != hipSuccess) return MAS_ERR_OOM;
  return MAS_OK;
}

// 63-bit Morton code of positions normalised to the bounding box, 21 bits
// per axis; x bits at positions 3b, y at 3b+1, z at 3b+2.
void morton_order(const double* X, int64_t N, std::vector<int32_t>& perm) {
  double lo[3], hi[3], ext[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = X[a];
    hi[a] = X[a];
  }
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], X[3 * i + a]);
      hi[a] = std::max(hi[a], X[3 * i + a]);
    }
  for (int a = 0; a < 3; ++a) {
    ext[a] = hi[a] - lo[a];
    if (!(ext[a] > 0)) ext[a] = 1.0;
  }
  std::vector<uint64_t> code(N);
  for (int64_t i = 0; i < N; ++i) {
    uint64_t c = 0;
    for (int a = 0; a < 3; ++a) {
      double t = (X[3 * i + a] - lo[a]) / ext[a] * 2097151.0;
      double f = std::floor(t);
      if (f < 0) f = 0;
      if (f > 2097151.0) f = 2097151.0;
      uint64_t q = uint64_t(f);
      for (int b = 0; b < 21; ++b) c |= ((q >> b) & 1ull) << (3 * b + a);
    }
    code[i] = c;
  }
  perm.resize(N);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t p, int32_t q) { return code[p] < code[q]; });
}

// Connectivity-aware order (supplement Section 1.2: greedy aggregation over
// the graph of nodes that share an element).  Level-0 nodes are the
// vertices, numbered component by component of the tet graph (components
// in the order of their smallest Morton rank, Morton order inside); a
// cluster grows from the smallest unassigned node by the smallest
// unassigned node adjacent to its members (else the smallest unassigned
// node) to SUB nodes; the clusters of level l are the nodes of level l+1,
// adjacent when some of their members are.  A node with fewer than SUB^l
// vertices (only the last can be) stays out of the growth and closes the
// last cluster, so every level-l node but the last holds SUB^l vertices.
// The vertex order expands the top-level clusters in order, members in the
// order they were added.
struct Graph {
  std::vector<int64_t> off;  // n + 1
  std::vector<int32_t> adj;  // sorted, unique neighbour lists
};

static void graph_from_pairs(int64_t n, std::vector<uint64_t>& pairs, Graph& g) {
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  g.off.assign(n + 1, 0);
  g.adj.resize(pairs.size());
  for (uint64_t e : pairs) ++g.off[(e >> 32) + 1];
  for (int64_t i = 0; i < n; ++i) g.off[i + 1] += g.off[i];
  for (size_t k = 0; k < pairs.size(); ++k) g.adj[k] = int32_t(pairs[k] & 0xffffffffu);
}

// clusters of nodes 0..n-1: members in the order added; cl_off has one
// entry per cluster plus one
static void aggregate_graph(const Graph& g, int64_t n, bool partial_last, std::vector<int64_t>& cl_off,
                            std::vector<int32_t>& members) {
  const int64_t limit = partial_last ? n - 1 : n;
  std::vector<uint8_t> assigned(n, 0);
  cl_off.assign(1, 0);
  members.clear();
  members.reserve(n);
  int64_t nxt = 0;
  std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> cand;
  for (int64_t seed = 0; seed < limit; ++seed) {
    if (assigned[seed]) continue;
    while (!cand.empty()) cand.pop();
    int64_t u = seed;
    int count = 0;
    while (true) {
      members.push_back(int32_t(u));
      assigned[u] = 1;
      ++count;
      for (int64_t k = g.off[u]; k < g.off[u + 1]; ++k) {
        const int32_t w = g.adj[k];
        if (w < limit && !assigned[w]) cand.push(w);
      }
      if (count == SUB) break;
      int64_t next = -1;
      while (!cand.empty()) {
        const int32_t w = cand.top();
        cand.pop();
        if (!assigned[w]) {
          next = w;
          break;
        }
      }
      if (next < 0) {
        while (nxt < limit && assigned[nxt]) ++nxt;
        if (nxt >= limit) break;
        next = nxt;
      }
      u = next;
    }
    cl_off.push_back(int64_t(members.size()));
  }
  if (partial_last) {
    const int64_t nc = int64_t(cl_off.size()) - 1;
    if (nc > 0 && cl_off[nc] - cl_off[nc - 1] < SUB) {
      members.push_back(int32_t(n - 1));
      cl_off[nc] += 1;
    } else {
      members.push_back(int32_t(n - 1));
      cl_off.push_back(int64_t(members.size()));
    }
  }
}

void connectivity_order(const double* X, int64_t N, const int32_t* tets, int64_t T, const int32_t* links,
                        int64_t nlinks, int L, std::vector<int32_t>& perm) {
  std::vector<int32_t> mperm;
  morton_order(X, N, mperm);
  std::vector<int64_t> mrank(N);
  for (int64_t i = 0; i < N; ++i) mrank[mperm[i]] = i;
  // components of the tet graph (union-find)
  std::vector<int64_t> par(N);
  std::iota(par.begin(), par.end(), 0);
  auto find = [&](int64_t a) {
    while (par[a] != a) {
      par[a] = par[par[a]];
      a = par[a];
    }
    return a;
  };
  auto unite = [&](int64_t a, int64_t b) {
    a = find(a);
    b = find(b);
    if (a != b) par[std::max(a, b)] = std::min(a, b);
  };
  for (int64_t t = 0; t < T; ++t)
    for (int j = 1; j < 4; ++j) unite(tets[4 * t], tets[4 * t + j]);
  for (int64_t k = 0; k < nlinks; ++k) unite(links[2 * k], links[2 * k + 1]);
  std::vector<int64_t> first(N, N);  // smallest Morton rank of each component (at its root)
  for (int64_t v = 0; v < N; ++v) {
    const int64_t r = find(v);
    first[r] = std::min(first[r], mrank[v]);
  }
  // level-0 node ids: (component's smallest rank, rank)
  std::vector<int32_t> node_vertex(mperm);
  std::stable_sort(node_vertex.begin(), node_vertex.end(),
                   [&](int32_t a, int32_t b) { return first[find(a)] < first[find(b)]; });
  std::vector<int32_t> vertex_node(N);
  for (int64_t i = 0; i < N; ++i) vertex_node[node_vertex[i]] = int32_t(i);
  Graph g;
  {
    std::vector<uint64_t> pairs;
    pairs.reserve(size_t(12) * T);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const uint64_t u = uint64_t(vertex_node[tets[4 * t + a]]), w = uint64_t(vertex_node[tets[4 * t + b]]);
          if (u != w) pairs.push_back((u << 32) | w);
        }
    for (int64_t k = 0; k < nlinks; ++k) {
      const uint64_t u = uint64_t(vertex_node[links[2 * k]]), w = uint64_t(vertex_node[links[2 * k + 1]]);
      if (u != w) {
        pairs.push_back((u << 32) | w);
        pairs.push_back((w << 32) | u);
      }
    }
    graph_from_pairs(N, pairs, g);
  }
  std::vector<std::vector<int64_t>> offs(L);
  std::vector<std::vector<int32_t>> mems(L);
  std::vector<int64_t> size(N, 1);
  int64_t n = N, full = 1;
  for (int l = 0; l < L; ++l) {
    const bool partial = n > 0 && size[n - 1] < full;
    aggregate_graph(g, n, partial, offs[l], mems[l]);
    const int64_t nc = int64_t(offs[l].size()) - 1;
    std::vector<int64_t> csize(nc, 0);
    std::vector<int32_t> cid(n);
    for (int64_t c = 0; c < nc; ++c)
      for (int64_t k = offs[l][c]; k < offs[l][c + 1]; ++k) {
        cid[mems[l][k]] = int32_t(c);
        csize[c] += size[mems[l][k]];
      }
    if (l + 1 < L) {
      std::vector<uint64_t> pairs;
      for (int64_t u = 0; u < n; ++u)
        for (int64_t k = g.off[u]; k < g.off[u + 1]; ++k) {
          const int32_t a = cid[u], b = cid[g.adj[k]];
          if (a != b) pairs.push_back((uint64_t(a) << 32) | uint64_t(b));
        }
      Graph h;
      graph_from_pairs(nc, pairs, h);
      g = std::move(h);
    }
    size = std::move(csize);
    n = nc;
    full *= SUB;
  }
  // expand the top-level clusters down to level-0 nodes
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  for (int l = L - 1; l >= 0; --l) {
    std::vector<int32_t> next;
    next.reserve(mems[l].size());
    for (int32_t c : order)
      for (int64_t k = offs[l][c]; k < offs[l][c + 1]; ++k) next.push_back(mems[l][k]);
    order = std::move(next);
  }
  perm.resize(N);
  for (int64_t i = 0; i < N; ++i) perm[i] = node_vertex[order[i]];
}

mas_status valid_contacts(const mas_contacts* c) {
  if (!c) return MAS_OK;
  if (c->m < 0) return MAS_ERR_INVALID_ARG;
  if (c->m > 0 && (!c->key || !c->idx || !c->d || !c->grad)) return MAS_ERR_INVALID_ARG;
  if (c->m > INT32_MAX / 4) return MAS_ERR_INVALID_ARG;
  return MAS_OK;
}

}  // namespace

extern "C" {

void mas_default_config(mas_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->num_levels = 2;
  cfg->max_rank = 8;
  cfg->cos_rot = std::cos(25.0 * M_PI / 180.0);
  cfg->restart_delta = 0.3;
  cfg->eps_sing = 1e-12;
  cfg->eps_abs = 1e-300;
  cfg->kappa = 1.0;
  cfg->dhat = 1e-3;
  cfg->h = 0.01;
  cfg->gravity[2] = -9.81;
  cfg->block_prec = MAS_F64;
  cfg->coarse_prec = MAS_F64;
  cfg->hess_prec = MAS_F64;
  cfg->prec_guard = 0.5;
}

const char* mas_status_string(mas_status s) {
  switch (s) {
    case MAS_OK: return "ok";
    case MAS_ERR_INVALID_ARG: return "invalid argument";
    case MAS_ERR_STATE: return "call out of order";
    case MAS_ERR_OOM: return "device allocation failed";
    case MAS_ERR_HIP: return "HIP runtime error";
    case MAS_ERR_NOT_SPD: return "non-positive pivot (matrix not SPD)";
    case MAS_ERR_NONFINITE: return "non-finite input";
    case MAS_ERR_RANK: return "capacitance rank reduced (trailing update columns dropped)";
  }
  return "unknown status";
}

mas_status mas_destroy(void* p) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx* c = as_ctx(p);
  hipStreamSynchronize(c->s);
  void* ptrs[] = {c->tets, c->geo, c->mass, c->tet_off, c->l0_tv, c->l0_home, c->rt_off, c->rbeg, c->vrange, c->ctr, c->rl_t, c->rl_tv,
                  c->rl_geo, c->hr64, c->hr32, c->rc_cnt, c->rc_off, c->rc_list, c->bkey,
                  c->hkey, c->hval, c->bk, c->bpm, c->bgrad, c->bidx, c->bu, c->bc_cnt,
                  c->bc_off, c->bc_list, c->U, c->Uidx, c->dS, c->upm, c->ckey, c->cand_cnt, c->cand_off,
                  c->cand_list, c->rank, c->sel, c->slots, c->W, c->Lcap, c->partials, c->scal,
                  c->alpha, c->alpha0, c->alpha_mix, c->ahalf, c->around, c->err, c->diag, c->cls_part, c->scan_tmp,
                  c->inc_cnt, c->inc_off, c->inc_list, c->coup, c->bj, c->bjinv, c->seg, c->scene_r, c->sc_acc};
  for (void* q : ptrs)
    if (q) hipFree(q);
  for (auto& t : c->cs) {
    void* tp[] = {t.cnt, t.off, t.key, t.id};
    for (void* q : tp)
      if (q) hipFree(q);
  }
  if (c->cs_misc) hipFree(c->cs_misc);
  for (int l = 0; l < MAXL; ++l) {
    Level& L = c->lv[l];
    void* lp[] = {L.blk, L.bprec, L.scale, L.acc, L.r, L.c};
    for (void* q : lp)
      if (q) hipFree(q);
  }
  if (c->prof) {
    for (int t = 0; t < MAS_T_COUNT; ++t)
      for (auto& pr : c->prof->done[t]) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
      }
    for (hipEvent_t e : c->prof->pool) hipEventDestroy(e);
    delete c->prof;
  }
  delete c;
  return MAS_OK;
}

mas_status mas_create(const mas_config* cfg, const mas_mesh* mesh, void* hip_stream, void** ctx_out,
                      int32_t* perm_out) {
  if (!cfg || !mesh || !ctx_out) return MAS_ERR_INVALID_ARG;
  *ctx_out = nullptr;
  const int64_t N = mesh->num_vertices, T = mesh->num_tets;
  if (N <= 0 || T < 0 || N > (int64_t(1) << 30) || T > (int64_t(1) << 29)) return MAS_ERR_INVALID_ARG;
  if (!mesh->rest_x || (T > 0 && (!mesh->tets || !mesh->density || !mesh->youngs || !mesh->poisson)))
    return MAS_ERR_INVALID_ARG;
  if (cfg->num_levels < 1 || cfg->num_levels > MAXL) return MAS_ERR_INVALID_ARG;
  if (cfg->max_rank < 0 || cfg->max_rank > MAXK) return MAS_ERR_INVALID_ARG;
  if (cfg->block_prec < MAS_F64 || cfg->block_prec > MAS_F16) return MAS_ERR_INVALID_ARG;
  if (cfg->coarse_prec < MAS_F64 || cfg->coarse_prec > MAS_F16) return MAS_ERR_INVALID_ARG;
  if (!(cfg->prec_guard >= 0)) return MAS_ERR_INVALID_ARG;
  if (cfg->hess_prec != MAS_F64 && cfg->hess_prec != MAS_F32) return MAS_ERR_INVALID_ARG;
  if (!(cfg->dhat > 0) || !(cfg->h > 0) || !(cfg->kappa >= 0)) return MAS_ERR_INVALID_ARG;
  if (cfg->deterministic != 0 && cfg->deterministic != 1) return MAS_ERR_INVALID_ARG;
  if (cfg->precond != MAS_PRECOND_MAS && cfg->precond != MAS_PRECOND_BJ3) return MAS_ERR_INVALID_ARG;
  if (cfg->precond == MAS_PRECOND_BJ3 && cfg->deterministic) return MAS_ERR_INVALID_ARG;
  if (cfg->hierarchy != MAS_HIER_MORTON && cfg->hierarchy != MAS_HIER_CONNECTIVITY) return MAS_ERR_INVALID_ARG;
  if (cfg->max_contacts < 0 || cfg->max_tris < 0 || cfg->max_edges < 0) return MAS_ERR_INVALID_ARG;
  if (cfg->max_contacts > INT32_MAX / 4 || cfg->max_tris > INT32_MAX / 8 || cfg->max_edges > INT32_MAX / 8)
    return MAS_ERR_INVALID_ARG;
  for (int64_t t = 0; t < 4 * T; ++t)
    if (mesh->tets[t] < 0 || mesh->tets[t] >= N) return MAS_ERR_INVALID_ARG;
  if (mesh->num_links < 0 || (mesh->num_links > 0 && !mesh->links)) return MAS_ERR_INVALID_ARG;
  for (int64_t k = 0; k < 2 * mesh->num_links; ++k)
    if (mesh->links[k] < 0 || mesh->links[k] >= N) return MAS_ERR_INVALID_ARG;
  // scenes: contiguous original vertex ranges that no tet or link joins
  const int S = mesh->num_scenes > 1 ? mesh->num_scenes : 1;
  std::vector<int32_t> vscene(N, 0);
  if (S > 1) {
    const int64_t* so = mesh->scene_offsets;
    if (!so || S > MAX_SCENES || cfg->hierarchy != MAS_HIER_MORTON || so[0] != 0 || so[S] != N)
      return MAS_ERR_INVALID_ARG;
    for (int q = 0; q < S; ++q) {
      if (so[q + 1] <= so[q]) return MAS_ERR_INVALID_ARG;
      for (int64_t v = so[q]; v < so[q + 1]; ++v) vscene[v] = q;
    }
    for (int64_t t = 0; t < T; ++t)
      for (int j = 1; j < 4; ++j)
        if (vscene[mesh->tets[4 * t + j]] != vscene[mesh->tets[4 * t]]) return MAS_ERR_INVALID_ARG;
    for (int64_t k = 0; k < mesh->num_links; ++k)
      if (vscene[mesh->links[2 * k]] != vscene[mesh->links[2 * k + 1]]) return MAS_ERR_INVALID_ARG;
  }

  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return MAS_ERR_OOM;
  c->s = reinterpret_cast<hipStream_t>(hip_stream);
  c->cfg = *cfg;
  if (c->cfg.max_contacts == 0) c->cfg.max_contacts = std::max<int64_t>(2 * N, 65536);
  if (c->cfg.max_tris == 0) c->cfg.max_tris = 2 * N + 64;
  if (c->cfg.max_edges == 0) c->cfg.max_edges = 3 * N + 64;
  c->N = N;
  c->T = T;
  c->Tpad = (T + TILE - 1) / TILE * TILE;
  if (c->Tpad == 0) c->Tpad = TILE;
  c->L = cfg->num_levels;
  c->K = cfg->max_rank;
  if (scratch_address(&c->fixed_ws) != MAS_OK) {
    delete c;
    return MAS_ERR_HIP;
  }
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        prop.multiProcessorCount > 0)
      c->n_cu = prop.multiProcessorCount;
  }
  mas_status st = MAS_OK;
#define TRY(x)                 \
  do {                         \
    st = (x);                  \
    if (st != MAS_OK) {        \
      mas_destroy(c);          \
      return st;               \
    }                          \
  } while (0)

  // Morton order and renumbered, locality-sorted tets
  std::vector<int32_t> perm;
  if (cfg->hierarchy == MAS_HIER_CONNECTIVITY)
    connectivity_order(mesh->rest_x, N, mesh->tets, T, mesh->links, mesh->num_links, cfg->num_levels, perm);
  else
    morton_order(mesh->rest_x, N, perm);
  c->S = S;
  c->scene_v.assign(S + 1, 0);
  if (S > 1) {
    // scene by scene, Morton order inside each
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return vscene[a] < vscene[b]; });
    for (int q = 0; q <= S; ++q) c->scene_v[q] = mesh->scene_offsets[q];
  } else {
    c->scene_v[1] = N;
  }
  std::vector<int32_t> rank(N);
  for (int64_t i = 0; i < N; ++i) rank[perm[i]] = int32_t(i);
  std::vector<int32_t> torder(T);
  std::vector<int32_t> tmin(T);
  for (int64_t t = 0; t < T; ++t) {
    int32_t m = INT32_MAX;
    for (int j = 0; j < 4; ++j) m = std::min(m, rank[mesh->tets[4 * t + j]]);
    tmin[t] = m;
  }
  std::iota(torder.begin(), torder.end(), 0);
  std::stable_sort(torder.begin(), torder.end(), [&](int32_t a, int32_t b) { return tmin[a] < tmin[b]; });
  std::vector<int32_t> tets(4 * T);
  std::vector<double> rho(T), E(T), nu(T);
  for (int64_t i = 0; i < T; ++i) {
    int64_t t = torder[i];
    for (int j = 0; j < 4; ++j) tets[4 * i + j] = rank[mesh->tets[4 * t + j]];
    rho[i] = mesh->density[t];
    E[i] = mesh->youngs[t];
    nu[i] = mesh->poisson[t];
  }
  std::vector<double> Xl(3 * N);
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) Xl[3 * i + a] = mesh->rest_x[3 * int64_t(perm[i]) + a];

  // levels
  int64_t nodes = N;
  for (int l = 0; l < c->L; ++l) {
    c->lv[l].nodes = nodes;
    c->lv[l].nsub = (nodes + SUB - 1) / SUB;
    c->lv[l].prec = (l == 0) ? cfg->block_prec : cfg->coarse_prec;
    nodes = c->lv[l].nsub;
  }
  const int64_t D0 = c->lv[0].nsub;

  // bucket (v / div) -> tets touching it, ascending tet order
  auto tet_buckets = [&](int div, int64_t nb, std::vector<int32_t>& off, std::vector<int32_t>& list) {
    auto buckets = [&](int64_t t, int* ds) {
      int n = 0;
      for (int j = 0; j < 4; ++j) {
        const int d = tets[4 * t + j] / div;
        bool dup = false;
        for (int q = 0; q < n; ++q) dup |= ds[q] == d;
        if (!dup) ds[n++] = d;
      }
      return n;
    };
    off.assign(nb + 1, 0);
    int ds[4];
    for (int64_t t = 0; t < T; ++t) {
      const int n = buckets(t, ds);
      for (int q = 0; q < n; ++q) off[ds[q] + 1]++;
    }
    for (int64_t d = 0; d < nb; ++d) off[d + 1] += off[d];
    list.assign(std::max<int32_t>(off[nb], 1), 0);
    std::vector<int32_t> cur(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
      const int n = buckets(t, ds);
      for (int q = 0; q < n; ++q) list[cur[ds[q]]++] = int32_t(t);
    }
  };
  std::vector<int32_t> toff, tlist, roff, rlist;
  tet_buckets(SUB, D0, toff, tlist);
  // vertex ranges: cut greedily in vertex order so that each range is
  // touched by about RANGE_TETS tets and spans at most RANGE_MAX vertices
  std::vector<int32_t> rbeg, vrange(N);
  // vertex -> touching tets, ascending tet order (ranges; lumped masses)
  std::vector<int32_t> voff(N + 1, 0), vt(std::max<int64_t>(4 * T, 1));
  {
    for (int64_t q = 0; q < 4 * T; ++q) voff[tets[q] + 1]++;
    for (int64_t v = 0; v < N; ++v) voff[v + 1] += voff[v];
    std::vector<int32_t> cur(voff.begin(), voff.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int j = 0; j < 4; ++j) vt[cur[tets[4 * t + j]]++] = int32_t(t);
    const int64_t target = RANGE_TETS;
    std::vector<int32_t> mark(T, -1);
    int64_t cnt = 0;
    int32_t r = 0, start = 0;
    rbeg.push_back(0);
    for (int64_t v = 0; v < N; ++v) {
      int64_t add = 0;
      for (int32_t q = voff[v]; q < voff[v + 1]; ++q) add += mark[vt[q]] != r;
      const bool scene_start = std::binary_search(c->scene_v.begin(), c->scene_v.end(), int64_t(v));
      if (v > start && (cnt + add > target || v - start >= RANGE_MAX || scene_start)) {
        ++r;
        start = int32_t(v);
        rbeg.push_back(start);
        cnt = 0;
        add = voff[v + 1] - voff[v];
      }
      for (int32_t q = voff[v]; q < voff[v + 1]; ++q) mark[vt[q]] = r;
      cnt += add;
      vrange[v] = r;
    }
    rbeg.push_back(int32_t(N));
    c->nrange = int64_t(rbeg.size()) - 1;
    c->rmax = 0;
    for (int64_t q = 0; q < c->nrange; ++q) c->rmax = std::max(c->rmax, rbeg[q + 1] - rbeg[q]);
  }
  {
    // range -> touching tets, ascending tet order
    roff.assign(c->nrange + 1, 0);
    auto ranges = [&](int64_t t, int* ds) {
      int n = 0;
      for (int j = 0; j < 4; ++j) {
        const int d = vrange[tets[4 * t + j]];
        bool dup = false;
        for (int q = 0; q < n; ++q) dup |= ds[q] == d;
        if (!dup) ds[n++] = d;
      }
      return n;
    };
    int ds[4];
    for (int64_t t = 0; t < T; ++t) {
      const int n = ranges(t, ds);
      for (int q = 0; q < n; ++q) roff[ds[q] + 1]++;
    }
    for (int64_t d = 0; d < c->nrange; ++d) roff[d + 1] += roff[d];
    rlist.assign(std::max<int32_t>(roff[c->nrange], 1), 0);
    std::vector<int32_t> cur(roff.begin(), roff.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
      const int n = ranges(t, ds);
      for (int q = 0; q < n; ++q) rlist[cur[ds[q]]++] = int32_t(t);
    }
  }

  // device memory
  TRY(dalloc(&c->tets, 4 * T));
  TRY(dalloc(&c->geo, 12 * c->Tpad));
  TRY(dalloc(&c->mass, N));
  TRY(dalloc(&c->tet_off, D0 + 1));
  TRY(dalloc(&c->l0_tv, 4 * tlist.size()));
  TRY(dalloc(&c->l0_home, tlist.size()));
  TRY(dalloc(&c->rt_off, c->nrange + 1));
  TRY(dalloc(&c->rbeg, c->nrange + 1));
  {
    // scenes: library vertex -> scene, first range of each scene
    std::vector<int32_t> segh(N);
    for (int q = 0; q < S; ++q)
      for (int64_t v = c->scene_v[q]; v < c->scene_v[q + 1]; ++v) segh[v] = q;
    std::vector<int64_t> sr(S + 1);
    for (int q = 0; q < S; ++q) sr[q] = vrange[c->scene_v[q]];
    sr[S] = c->nrange;
    TRY(dalloc(&c->seg, N));
    TRY(dalloc(&c->scene_r, S + 1));
    TRY(dalloc(&c->sc_acc, 8 * S));
    HIPCHK(hipMemcpy(c->seg, segh.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->scene_r, sr.data(), (S + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  TRY(dalloc(&c->vrange, N));
  TRY(dalloc(&c->ctr, 4));
  HIPCHK(hipMemcpy(c->rbeg, rbeg.data(), rbeg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->vrange, vrange.data(), vrange.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  c->nent = int64_t(roff[c->nrange]);
  c->nent_pad = std::max<int64_t>((c->nent + TILE - 1) / TILE * TILE, TILE);
  TRY(dalloc(&c->rl_t, c->nent_pad));
  TRY(dalloc(&c->rl_tv, 4 * c->nent_pad));
  TRY(dalloc(&c->rl_geo, 12 * c->nent_pad));
  TRY(dalloc(&c->rc_cnt, c->nrange + 1));
  TRY(dalloc(&c->rc_off, c->nrange + 1));
  if (cfg->hess_prec == MAS_F32) TRY(dalloc(&c->hr32, 4 * SNAP_NC32 * c->nent_pad));
  else TRY(dalloc(&c->hr64, EH * c->nent_pad));
  for (int l = 0; l < c->L; ++l) {
    Level& L = c->lv[l];
    TRY(dalloc_bytes(&L.blk, L.nsub * BLK_STRIDE));
    TRY(dalloc(&L.bprec, L.nsub));
    TRY(dalloc(&L.scale, L.nsub * BD));
    TRY(dalloc(&L.acc, L.nsub * PK));
    if (l > 0) {
      TRY(dalloc(&L.r, 3 * L.nodes));
      TRY(dalloc(&L.c, 3 * L.nodes));
    }
  }
  TRY(dalloc(&c->bc_cnt, D0 + 1));
  TRY(dalloc(&c->bc_off, D0 + 1));
  TRY(dalloc(&c->cand_cnt, D0 + 1));
  TRY(dalloc(&c->cand_off, D0 + 1));
  int Kk = std::max(c->K, 1);
  TRY(dalloc(&c->rank, D0));
  TRY(dalloc(&c->sel, D0 * Kk));
  TRY(dalloc(&c->slots, D0 * Kk));
  TRY(dalloc(&c->W, size_t(D0) * Kk * BD));
  TRY(dalloc(&c->Lcap, D0 * (Kk * (Kk + 1) / 2)));
  c->n_partial_blocks = int(std::max<int64_t>(1024, c->nrange));
  TRY(dalloc(&c->partials, 16 * c->n_partial_blocks));
  TRY(dalloc(&c->scal, 64));
  TRY(dalloc(&c->alpha, D0));
  TRY(dalloc(&c->alpha0, D0));
  TRY(dalloc(&c->alpha_mix, D0));
  if (cfg->precond == MAS_PRECOND_BJ3) {
    TRY(dalloc(&c->bj, 6 * N));
    TRY(dalloc(&c->bjinv, 6 * N));
  }
  TRY(dalloc(&c->ahalf, D0));
  TRY(dalloc(&c->around, SAFE_ROUNDS + 1));
  TRY(dalloc(&c->err, 1));
  TRY(dalloc(&c->diag, DIAG_SLOTS));
  // contact sets: capacity max_contacts, key table twice that (power of two)
  {
    const int64_t cap = std::max<int64_t>(c->cfg.max_contacts, 1);
    c->mb_cap = c->mc_cap = cap;
    c->hcap = 1024;
    while (c->hcap < 2 * cap) c->hcap *= 2;
    TRY(dalloc(&c->bkey, cap));
    TRY(dalloc(&c->hkey, c->hcap));
    TRY(dalloc(&c->hval, c->hcap));
    TRY(dalloc(&c->bk, cap));
    TRY(dalloc(&c->bpm, cap));
    TRY(dalloc(&c->bgrad, 12 * cap));
    TRY(dalloc(&c->bidx, 4 * cap));
    TRY(dalloc(&c->bu, 12 * cap));
    TRY(dalloc(&c->bc_list, 4 * cap));
    TRY(dalloc(&c->rc_list, 4 * cap));
    TRY(dalloc(&c->U, 12 * cap));
    TRY(dalloc(&c->Uidx, 4 * cap));
    TRY(dalloc(&c->dS, cap));
    TRY(dalloc(&c->upm, cap));
    TRY(dalloc(&c->ckey, cap));
    TRY(dalloc(&c->cand_list, 4 * cap));
    TRY(dalloc(&c->cls_part, 5 * ((cap + 255) / 256)));
  }
  // constraint-set grid tables: buckets a power of two of at least twice the
  // primitives, up to 8 cell entries per primitive
  {
    const int64_t np[2] = {c->cfg.max_tris, c->cfg.max_edges};
    for (int k = 0; k < 2; ++k) {
      Ctx::CellTable& t = c->cs[k];
      int64_t H = 1024;
      while (H < 2 * np[k]) H <<= 1;
      t.h_cap = H + 1;
      t.e_cap = std::max<int64_t>(8 * np[k], 1);
      TRY(dalloc(&t.cnt, t.h_cap));
      TRY(dalloc(&t.off, t.h_cap));
      TRY(dalloc(&t.key, t.e_cap));
      TRY(dalloc(&t.id, t.e_cap));
    }
    TRY(dalloc(&c->cs_misc, 4));
  }
  // deterministic mode: vertex incidence lists and the per-subdomain
  // deep-level coupling tables
  if (c->cfg.deterministic) {
    TRY(dalloc(&c->inc_cnt, N + 1));
    TRY(dalloc(&c->inc_off, N + 1));
    TRY(dalloc(&c->inc_list, 4 * std::max<int64_t>(c->cfg.max_contacts, 1)));
    if (c->L > 2) TRY(dalloc(&c->coup, size_t(D0) * (c->L - 2) * SUB * 9));
  }
  // scratch of the exclusive scans: the longest scan is a bucket table (or
  // the vertex counts of the incidence lists)
  c->scan_cap = std::max<int64_t>({D0 + 1, c->nrange + 1, c->cs[0].h_cap, c->cs[1].h_cap, N + 1});
  TRY(dalloc(&c->scan_tmp, scan_scratch_elems(c->scan_cap)));
  HIPCHK(hipMemsetAsync(c->err, 0, sizeof(uint32_t), c->s));
  HIPCHK(hipMemsetAsync(c->diag, 0, sizeof(DiagRec) * DIAG_SLOTS, c->s));
  HIPCHK(hipMemsetAsync(c->rank, 0, sizeof(int32_t) * D0, c->s));
  HIPCHK(hipMemsetAsync(c->alpha, 0, sizeof(double) * D0, c->s));
  HIPCHK(hipMemsetAsync(c->around, 0, sizeof(uint32_t) * (SAFE_ROUNDS + 1), c->s));

  HIPCHK(hipMemcpyAsync(c->tets, tets.data(), 4 * T * sizeof(int32_t), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->tet_off, toff.data(), (D0 + 1) * sizeof(int32_t), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->rt_off, roff.data(), roff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->s));
  {
    // entries: tet id (home flag in bit 31) and its vertices
    std::vector<int32_t> et(c->nent_pad, 0), etv(4 * c->nent_pad, 0), th(c->Tpad, 0);
    for (int64_t r = 0; r < c->nrange; ++r)
      for (int32_t w = roff[r]; w < roff[r + 1]; ++w) {
        const int64_t t = rlist[w];
        int vmin = tets[4 * t];
        for (int j = 0; j < 4; ++j) {
          etv[4 * w + j] = tets[4 * t + j];
          vmin = std::min(vmin, tets[4 * t + j]);
        }
        const bool home = vrange[vmin] == r;
        et[w] = int32_t(t) | (home ? int32_t(0x80000000u) : 0);
        if (home) th[t] = w;
      }
    HIPCHK(hipMemcpy(c->rl_t, et.data(), et.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->rl_tv, etv.data(), etv.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    // level-0 records: the tet's vertices and its home entry side by side, so
    // that the block assembly reads them without a chain of gathers
    std::vector<int32_t> rtv(4 * tlist.size()), rh(tlist.size());
    for (size_t w = 0; w < tlist.size(); ++w) {
      const int64_t t = tlist[w];
      for (int j = 0; j < 4; ++j) rtv[4 * w + j] = tets[4 * t + j];
      rh[w] = th[t];
    }
    HIPCHK(hipMemcpy(c->l0_tv, rtv.data(), rtv.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->l0_home, rh.data(), rh.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  double *dX = nullptr, *drho = nullptr, *dE = nullptr, *dnu = nullptr, *dmq = nullptr;
  int32_t *dvoff = nullptr, *dvt = nullptr;
  TRY(dalloc(&dX, 3 * N));
  TRY(dalloc(&drho, T));
  TRY(dalloc(&dE, T));
  TRY(dalloc(&dnu, T));
  TRY(dalloc(&dmq, T));
  TRY(dalloc(&dvoff, N + 1));
  TRY(dalloc(&dvt, vt.size()));
  HIPCHK(hipMemcpyAsync(dX, Xl.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(drho, rho.data(), T * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(dE, E.data(), T * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(dnu, nu.data(), T * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(dvoff, voff.data(), (N + 1) * sizeof(int32_t), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(dvt, vt.data(), vt.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->s));
  st = launch_rest(*c, dX, drho, dE, dnu, dmq, dvoff, dvt);
  hipStreamSynchronize(c->s);
  hipFree(dX);
  hipFree(drho);
  hipFree(dE);
  hipFree(dnu);
  hipFree(dmq);
  hipFree(dvoff);
  hipFree(dvt);
  if (st != MAS_OK) {
    mas_destroy(c);
    return st;
  }
  // empty bucket lists until the first build
  TRY(bucket_by_subdomain(*c, 0, nullptr, nullptr, c->bc_cnt, c->bc_off, nullptr));
  TRY(bucket_stencils(*c, 1, c->vrange, c->nrange, 0, nullptr, nullptr, c->rc_cnt, c->rc_off, nullptr));
  HIPCHK(hipStreamSynchronize(c->s));
  if (perm_out) std::memcpy(perm_out, perm.data(), N * sizeof(int32_t));
  *ctx_out = c;
#undef TRY
  return MAS_OK;
}

mas_status mas_build(void* p, const double* x_base, const mas_contacts* base) {
  if (!p || !x_base) return MAS_ERR_INVALID_ARG;
  mas_status st = valid_contacts(base);
  if (st != MAS_OK) return st;
  Ctx& c = *as_ctx(p);
  if (base && base->m > c.mb_cap) return MAS_ERR_INVALID_ARG;
  ProfScope ps(c, MAS_T_BUILD);
  if ((st = launch_elem_hessians(c, x_base)) != MAS_OK) return st;
  if ((st = launch_base_contacts(c, base)) != MAS_OK) return st;
  if ((st = launch_level0_build(c)) != MAS_OK) return st;
  c.built = true;
  c.have_update = false;
  c.mc = 0;
  return MAS_OK;
}

mas_status mas_woodbury_update(void* p, const mas_contacts* cur, int32_t* rank_hist) {
  if (!p) return MAS_ERR_INVALID_ARG;
  mas_status st = valid_contacts(cur);
  if (st != MAS_OK) return st;
  Ctx& c = *as_ctx(p);
  if (!c.built) return MAS_ERR_STATE;
  if (cur && cur->m > c.mc_cap) return MAS_ERR_INVALID_ARG;
  if ((st = launch_woodbury(c, cur, rank_hist)) != MAS_OK) return st;
  c.have_update = true;
  return MAS_OK;
}

mas_status mas_apply(void* p, const double* g, double* z) {
  if (!p || !g || !z || g == z) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built) return MAS_ERR_STATE;
  return launch_apply(c, g, z);
}

mas_status hess_vec(void* p, const double* v, double* y, int32_t with_update) {
  if (!p || !v || !y || v == y) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built) return MAS_ERR_STATE;
  return launch_hessvec(c, v, y, with_update);
}

mas_status pncg_subspace_step(void* p, const double* g, const double* z, const double* z_prev,
                              const double* v_z, double* pk_, double* v_p, int32_t restart,
                              mas_step_out* out) {
  if (!p || !g || !z || !v_z || !pk_ || !v_p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built) return MAS_ERR_STATE;
  return launch_subspace(c, g, z, z_prev, v_z, pk_, v_p, restart, out);
}

mas_status pncg_subspace_step_noalloc(void* p, const double* g, const double* z, const double* z_prev,
                                      const double* v_z, double* pk_, double* v_p, int32_t restart,
                                      mas_step_out* out) {
  if (!p || !g || !z || !v_z || !pk_ || !v_p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built || !c.fixed_ws) return MAS_ERR_STATE;
  const int64_t need = subspace_workspace_elems(c);
  if (need > SCRATCH_DOUBLES) return MAS_ERR_INVALID_ARG;
  return launch_subspace_ws(c, g, z, z_prev, v_z, pk_, v_p, restart, out, c.fixed_ws, c.fixed_ws + need - 2);
}

mas_status pncg_beta_step(void* p, int32_t rule, const double* g, const double* g_prev, const double* z,
                          const double* z_prev, const double* v_z, double* d, double* v_d, int32_t restart,
                          double* step, mas_step_out* out) {
  if (!p || !g || !z || !v_z || !d || !v_d || !step) return MAS_ERR_INVALID_ARG;
  if (rule != MAS_BETA_FR && rule != MAS_BETA_CD && rule != MAS_BETA_DK) return MAS_ERR_INVALID_ARG;
  if (!restart && (!g_prev || !z_prev)) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built) return MAS_ERR_STATE;
  return launch_beta(c, rule, g, restart ? nullptr : g_prev, z, z_prev, v_z, d, v_d, restart, step, out);
}

mas_status pncg_subspace_step_scenes(void* p, const double* g, const double* z, const double* z_prev,
                                     const double* v_z, double* pk_, double* v_p, const int32_t* restart,
                                     mas_step_out* out) {
  if (!p || !g || !z || !v_z || !pk_ || !v_p || !restart) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.built || c.cfg.deterministic) return MAS_ERR_STATE;
  return launch_subspace_scenes(c, g, z, z_prev, v_z, pk_, v_p, restart, out);
}

mas_status mas_energy_grad_scenes(void* p, const double* x, const double* x_tilde, const mas_contacts* ct,
                                  double* E, double* g) {
  if (!p || !x || !x_tilde || !E) return MAS_ERR_INVALID_ARG;
  mas_status st = valid_contacts(ct);
  if (st != MAS_OK) return st;
  Ctx& c = *as_ctx(p);
  if (c.cfg.deterministic) return MAS_ERR_STATE;
  return launch_energy_grad_scenes(c, x, x_tilde, ct, E, g);
}

mas_status mas_step_scenes(void* p, const double* x, const double* pk_, const double* scale, double* x_out) {
  if (!p || !x || !pk_ || !scale || !x_out || x == x_out) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (c.cfg.deterministic) return MAS_ERR_STATE;
  return launch_step_scenes(c, x, pk_, scale, x_out);
}

mas_status mas_scenes(void* p, int32_t* num_scenes, int64_t* voff) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (num_scenes) *num_scenes = c.S;
  if (voff) std::copy(c.scene_v.begin(), c.scene_v.end(), voff);
  return MAS_OK;
}

mas_status mas_energy_grad(void* p, const double* x, const double* x_tilde, const mas_contacts* ct,
                           double* E, double* g) {
  if (!p || !x || !x_tilde || !E) return MAS_ERR_INVALID_ARG;
  mas_status st = valid_contacts(ct);
  if (st != MAS_OK) return st;
  Ctx& c = *as_ctx(p);
  // the ordered gather of deterministic mode lists the contacts per vertex
  if (c.cfg.deterministic && g && ct && ct->m > c.cfg.max_contacts) return MAS_ERR_INVALID_ARG;
  return launch_energy_grad(c, x, x_tilde, ct, E, g);
}

mas_status mas_ccd_safe_step(void* p, const double* x, const double* pdir, double radius, int64_t m,
                             const int32_t* pairs, const uint8_t* kind, const double* dist, double scale,
                             double* alpha, double* x_out) {
  if (!p || !x || !pdir || !x_out || m < 0 || !(radius > 0.0) || !std::isfinite(radius)) return MAS_ERR_INVALID_ARG;
  if (m > 0 && (!pairs || !kind || !dist)) return MAS_ERR_INVALID_ARG;
  if (!(scale >= 0.0) || !(scale <= 1.0)) return MAS_ERR_INVALID_ARG;
  return launch_ccd_safe_step(*as_ctx(p), x, pdir, radius, m, pairs, kind, dist, scale, alpha, x_out);
}

mas_status mas_next_frame(void* p, const double* x_new, const double* x_old, double* v, double* x_tilde) {
  if (!p || !x_new || !x_old || (!v && !x_tilde)) return MAS_ERR_INVALID_ARG;
  if (v == x_new || v == x_old || x_tilde == x_new || x_tilde == x_old || (v && v == x_tilde))
    return MAS_ERR_INVALID_ARG;
  return launch_next_frame(*as_ctx(p), x_new, x_old, v, x_tilde);
}

mas_status mas_inertial_target(void* p, const double* x_t, const double* v_t, double* x_tilde) {
  if (!p || !x_t || !v_t || !x_tilde) return MAS_ERR_INVALID_ARG;
  return launch_inertial(*as_ctx(p), x_t, v_t, x_tilde);
}

mas_status mas_stencil_distance(void* p, const double* x, int64_t m, const int32_t* idx,
                                const double* grad, const double* off, double* d_out) {
  if (!p || !x || m < 0 || (m > 0 && (!idx || !grad || !off || !d_out))) return MAS_ERR_INVALID_ARG;
  return launch_stencil_distance(*as_ctx(p), x, m, idx, grad, off, d_out);
}

mas_status mas_safe_step(void* p, const double* x, const double* pv, const mas_contacts* cand,
                         double scale, double* alpha, double* x_out) {
  if (!p || !x || !pv || !x_out) return MAS_ERR_INVALID_ARG;
  mas_status st = valid_contacts(cand);
  if (st != MAS_OK) return st;
  return launch_safe_step(*as_ctx(p), x, pv, cand, scale, alpha, x_out);
}

mas_status mas_ccd_steps(void* p, const double* x, const double* pv, int64_t m, const int32_t* pairs,
                         const uint8_t* kind, const double* dist, double* alpha_pair, double* alpha) {
  if (!p || !x || !pv || m < 0) return MAS_ERR_INVALID_ARG;
  if (m > 0 && (!pairs || !kind || !dist)) return MAS_ERR_INVALID_ARG;
  return launch_ccd(*as_ctx(p), x, pv, m, pairs, kind, dist, alpha_pair, alpha);
}

mas_status mas_contact_distances(void* p, const double* x, int64_t m, const int32_t* pairs, const uint8_t* kind,
                                 double* dist, double* grad, uint8_t* type) {
  if (!p || !x || m < 0) return MAS_ERR_INVALID_ARG;
  if (m > 0 && (!pairs || !kind || !dist)) return MAS_ERR_INVALID_ARG;
  return launch_contact_distances(*as_ctx(p), x, m, pairs, kind, dist, grad, type);
}

mas_status mas_constraint_set(void* p, const double* x, double dhat, int64_t nv, const int32_t* verts, int64_t nt,
                              const int32_t* tris, int64_t ne, const int32_t* edges, int64_t cap, int32_t* pairs,
                              uint8_t* kind, double* dist, double* grad, uint64_t* key, int64_t* count) {
  if (!p || !x || !count || !(dhat > 0.0) || !std::isfinite(dhat) || nv < 0 || nt < 0 || ne < 0 || cap < 0)
    return MAS_ERR_INVALID_ARG;
  if ((nv > 0 && !verts) || (nt > 0 && !tris) || (ne > 0 && !edges)) return MAS_ERR_INVALID_ARG;
  if (cap > 0 && (!pairs || !kind || !dist)) return MAS_ERR_INVALID_ARG;
  if (nt > INT32_MAX || ne > INT32_MAX || cap > INT32_MAX) return MAS_ERR_INVALID_ARG;
  return launch_constraint_set(*as_ctx(p), x, dhat, nv, verts, nt, tris, ne, edges, cap, pairs, kind, dist, grad,
                               key, count);
}

mas_status mas_sync_status(void* p, char* msg, int32_t msg_len) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  hipError_t e = hipStreamSynchronize(c.s);
  mas_status st = MAS_OK;
  DiagRec dg{};
  if (e != hipSuccess) {
    st = MAS_ERR_HIP;
  } else {
    uint32_t bits = 0;
    DiagRec slots[DIAG_SLOTS];
    if (hipMemcpy(&bits, c.err, sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess) st = MAS_ERR_HIP;
    if (hipMemcpy(slots, c.diag, sizeof(slots), hipMemcpyDeviceToHost) != hipSuccess) st = MAS_ERR_HIP;
    hipMemset(c.err, 0, sizeof(uint32_t));
    hipMemset(c.diag, 0, sizeof(slots));
    // the lowest level that failed (its failures cause the ones above)
    for (int q = 0; q < DIAG_SLOTS && !dg.flag; ++q)
      if (slots[q].flag) dg = slots[q];
    if (bits & ERRB_NOT_SPD) st = MAS_ERR_NOT_SPD;
    else if (bits & ERRB_NONFINITE) st = MAS_ERR_NONFINITE;
    else if (bits & ERRB_RANK) st = MAS_ERR_RANK;
    else if (bits & ERRB_INDEX) st = MAS_ERR_INVALID_ARG;
  }
  if (msg && msg_len > 0) {
    static const char* src[] = {"?", "level-0 block", "coarse block", "capacitance (columns from this step on dropped)"};
    if (st == MAS_ERR_HIP)
      std::snprintf(msg, msg_len, "%s: %s", mas_status_string(st), hipGetErrorString(e));
    else if (dg.flag)
      std::snprintf(msg, msg_len, "%s: %s (level %d, subdomain %lld, step %d, pivot %.6g)",
                    mas_status_string(st), src[dg.source >= 1 && dg.source <= 3 ? dg.source : 0], dg.level,
                    (long long)dg.index, dg.step, dg.value);
    else
      std::snprintf(msg, msg_len, "%s", mas_status_string(st));
  }
  return st;
}

mas_status mas_read_stats(void* p, mas_iter_stats* out) {
  if (!p || !out) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  std::memset(out, 0, sizeof(*out));
  HIPCHK(hipStreamSynchronize(c.s));
  const int64_t D0 = c.lv[0].nsub;
  out->contacts = c.have_update ? c.mc : 0;
  if (c.have_update && c.cls_blocks > 0) {
    std::vector<int32_t> part(5 * c.cls_blocks);
    HIPCHK(hipMemcpy(part.data(), c.cls_part, part.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t b = 0; b < c.cls_blocks; ++b) {
      out->active += part[5 * b];
      out->n_new += part[5 * b + 1];
      out->n_rotated += part[5 * b + 2];
      out->n_stiffened += part[5 * b + 3];
      out->n_softened += part[5 * b + 4];
    }
  }
  if (c.have_update && c.K > 0) {
    std::vector<int32_t> rk(D0);
    HIPCHK(hipMemcpy(rk.data(), c.rank, D0 * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t r : rk) {
      out->rank_sum += r;
      out->rank_max = std::max(out->rank_max, r);
    }
  }
  uint32_t rounds[SAFE_ROUNDS + 1];
  HIPCHK(hipMemcpy(rounds, c.around, sizeof(rounds), hipMemcpyDeviceToHost));
  for (int r = 0; r < SAFE_ROUNDS; ++r) out->safe_rounds += rounds[r] > 0;
  out->safe_left = rounds[SAFE_ROUNDS];
  std::vector<double> al(D0);
  HIPCHK(hipMemcpy(al.data(), c.alpha, D0 * sizeof(double), hipMemcpyDeviceToHost));
  for (double a : al) {
    int bin = 7;
    if (a >= 1.0) bin = 0;
    else
      for (int i = 1; i <= 6; ++i)
        if (a >= std::ldexp(1.0, -i)) {
          bin = i;
          break;
        }
    out->alpha_hist[bin]++;
  }
  return MAS_OK;
}

mas_status mas_vertex_order(const mas_mesh* mesh, int32_t num_levels, int32_t hierarchy, int32_t* perm_out) {
  if (!mesh || !perm_out || !mesh->rest_x) return MAS_ERR_INVALID_ARG;
  const int64_t N = mesh->num_vertices, T = mesh->num_tets;
  if (N <= 0 || T < 0 || N > (int64_t(1) << 30) || (T > 0 && !mesh->tets)) return MAS_ERR_INVALID_ARG;
  if (num_levels < 1 || num_levels > MAXL) return MAS_ERR_INVALID_ARG;
  if (hierarchy != MAS_HIER_MORTON && hierarchy != MAS_HIER_CONNECTIVITY) return MAS_ERR_INVALID_ARG;
  for (int64_t t = 0; t < 4 * T; ++t)
    if (mesh->tets[t] < 0 || mesh->tets[t] >= N) return MAS_ERR_INVALID_ARG;
  std::vector<int32_t> perm;
  if (mesh->num_links < 0 || (mesh->num_links > 0 && !mesh->links)) return MAS_ERR_INVALID_ARG;
  for (int64_t k = 0; k < 2 * mesh->num_links; ++k)
    if (mesh->links[k] < 0 || mesh->links[k] >= N) return MAS_ERR_INVALID_ARG;
  if (hierarchy == MAS_HIER_CONNECTIVITY)
    connectivity_order(mesh->rest_x, N, mesh->tets, T, mesh->links, mesh->num_links, num_levels, perm);
  else
    morton_order(mesh->rest_x, N, perm);
  if (mesh->num_scenes > 1) {
    // scene by scene, as mas_create orders them
    const int S = mesh->num_scenes;
    const int64_t* so = mesh->scene_offsets;
    if (!so || S > MAX_SCENES || hierarchy != MAS_HIER_MORTON || so[0] != 0 || so[S] != N)
      return MAS_ERR_INVALID_ARG;
    std::vector<int32_t> vscene(N, 0);
    for (int q = 0; q < S; ++q) {
      if (so[q + 1] <= so[q]) return MAS_ERR_INVALID_ARG;
      for (int64_t v = so[q]; v < so[q + 1]; ++v) vscene[v] = q;
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return vscene[a] < vscene[b]; });
  }
  std::copy(perm.begin(), perm.end(), perm_out);
  return MAS_OK;
}

mas_status mas_query(void* p, int64_t* N, int64_t* T, int32_t* levels, int64_t* nsub) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (N) *N = c.N;
  if (T) *T = c.T;
  if (levels) *levels = c.L;
  if (nsub)
    for (int l = 0; l < MAXL; ++l) nsub[l] = l < c.L ? c.lv[l].nsub : 0;
  return MAS_OK;
}

mas_status mas_get_block(void* p, int32_t level, int64_t d, double* out) {
  if (!p || !out) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (level < 0 || level >= c.L || d < 0 || d >= c.lv[level].nsub) return MAS_ERR_INVALID_ARG;
  if (!c.built || c.cfg.precond != MAS_PRECOND_MAS) return MAS_ERR_STATE;
  Level& L = c.lv[level];
  uint8_t p8 = 0;
  HIPCHK(hipStreamSynchronize(c.s));
  HIPCHK(hipMemcpy(&p8, L.bprec + d, 1, hipMemcpyDeviceToHost));
  const int P = p8;
  std::vector<unsigned char> raw(BLK_STRIDE);
  std::vector<float> sig(BD, 1.0f);
  HIPCHK(hipMemcpy(raw.data(), reinterpret_cast<unsigned char*>(L.blk) + d * BLK_STRIDE, BLK_STRIDE,
                   hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(sig.data(), L.scale + d * BD, BD * sizeof(float), hipMemcpyDeviceToHost));
  for (int i = 0; i < BD; ++i)
    for (int j = 0; j <= i; ++j) {
      const int e = blk_pos(P, i, j);
      double v;
      if (P == MAS_F64) v = reinterpret_cast<double*>(raw.data())[e];
      else if (P == MAS_F32) v = reinterpret_cast<float*>(raw.data())[e];
      else {
        uint16_t h = reinterpret_cast<uint16_t*>(raw.data())[e];
        float f = P == MAS_BF16 ? bf16_to_f32(h) : f16_to_f32(h);
        v = double(f) * sig[i] * sig[j];
      }
      out[i * BD + j] = v;
      out[j * BD + i] = v;
    }
  return MAS_OK;
}

mas_status mas_block_precisions(void* p, int32_t level, int64_t* counts) {
  if (!p || !counts) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (level < 0 || level >= c.L) return MAS_ERR_INVALID_ARG;
  if (!c.built || c.cfg.precond != MAS_PRECOND_MAS) return MAS_ERR_STATE;
  Level& L = c.lv[level];
  std::vector<uint8_t> pr(L.nsub);
  HIPCHK(hipStreamSynchronize(c.s));
  HIPCHK(hipMemcpy(pr.data(), L.bprec, L.nsub, hipMemcpyDeviceToHost));
  for (int q = 0; q < 4; ++q) counts[q] = 0;
  for (uint8_t v : pr) counts[v & 3]++;
  return MAS_OK;
}

mas_status mas_profile_enable(void* p, int32_t enable) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.prof) c.prof = new (std::nothrow) Prof();
  if (!c.prof) return MAS_ERR_OOM;
  HIPCHK(hipStreamSynchronize(c.s));
  for (int t = 0; t < MAS_T_COUNT; ++t) {
    for (auto& pr : c.prof->done[t]) {
      c.prof->pool.push_back(pr.first);
      c.prof->pool.push_back(pr.second);
    }
    c.prof->done[t].clear();
    c.prof->open[t] = nullptr;
  }
  c.prof->on = enable != 0;
  return MAS_OK;
}

mas_status mas_profile_select(void* p, uint32_t mask) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  if (!c.prof) c.prof = new (std::nothrow) Prof();
  if (!c.prof) return MAS_ERR_OOM;
  c.prof->mask = mask;
  return MAS_OK;
}

mas_status mas_profile_read(void* p, int32_t timer, double* total_ms, int64_t* count) {
  if (!p || timer < 0 || timer >= MAS_T_COUNT) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  double tot = 0;
  int64_t n = 0;
  if (c.prof) {
    HIPCHK(hipStreamSynchronize(c.s));
    for (auto& pr : c.prof->done[timer]) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
      tot += ms;
      ++n;
      c.prof->pool.push_back(pr.first);
      c.prof->pool.push_back(pr.second);
    }
    c.prof->done[timer].clear();
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = n;
  return MAS_OK;
}

mas_status mas_get_selection(void* p, int32_t* rank_host, int32_t* sel_host) {
  if (!p) return MAS_ERR_INVALID_ARG;
  Ctx& c = *as_ctx(p);
  const int64_t D0 = c.lv[0].nsub;
  HIPCHK(hipStreamSynchronize(c.s));
  if (!c.have_update || c.K == 0 || c.cfg.precond != MAS_PRECOND_MAS) {
    if (rank_host) std::memset(rank_host, 0, D0 * sizeof(int32_t));
    if (sel_host) std::fill(sel_host, sel_host + D0 * c.K, -1);
    return MAS_OK;
  }
  if (rank_host) HIPCHK(hipMemcpy(rank_host, c.rank, D0 * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (sel_host) HIPCHK(hipMemcpy(sel_host, c.sel, D0 * c.K * sizeof(int32_t), hipMemcpyDeviceToHost));
  return MAS_OK;
}

}  // extern "C"
