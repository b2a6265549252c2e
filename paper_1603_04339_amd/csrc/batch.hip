// Batched CheFSI over several (cell, k) problems: the Chebyshev filters of all
// problems advance together; every recurrence step is one launch of the projections of
// all problems, one stencil launch over all problems and one launch of the projector
// scatters of all problems (each with per-problem arguments in a device table; the
// scatter runs inside the stencil step for problems with fused tables), and the whole
// sequence is captured once into a HIP graph.  The coefficients (which change with the
// filter bounds of every pass) live in device tables rewritten before each replay, so
// the captured graph is reused unchanged.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "devmath.hpp"

namespace sparc {

static size_t al256(size_t b) { return ((b + 255) / 256) * 256; }

}  // namespace sparc

using namespace sparc;

struct sparc_filter_plan {
  sparc_ctx* ctx;
  sparc_dtype dt;
  int n_o, tile, n_prob, max_deg;
  int dir;   // some problem has a Dirichlet direction
  std::vector<sparc_ham*> H;
  std::vector<void*> X, W, alpha;
  std::vector<char> fused;        // the problem applies its projectors inside the step
  std::vector<int64_t> ldx;
  std::vector<int> n_s, deg;
  // per step: participating problems, their table and work-group offsets
  std::vector<std::vector<int>> members;
  std::vector<int64_t> total_wg;
  std::vector<size_t> table_off;  // byte offset of step j's table in the device/host table buffer
  std::vector<size_t> wg_off;     // int offset of step j's offsets
  char* dev_tables;
  int* dev_wg;
  double* dev_a;                  // [max_deg][n_prob] scatter scale per step
  std::vector<size_t> nl_lds;     // dynamic LDS of step j's launch
  // projections and scatters of step j: argument blocks [max_deg][n_prob] and
  // work-group offsets [max_deg][n_prob + 1] (device, then host copies)
  NlBatchArgs* dev_gather;
  NlBatchArgs* dev_scatter;
  int* dev_goff;
  int* dev_soff;
  std::vector<NlBatchArgs> host_gather, host_scatter;
  std::vector<int> host_goff, host_soff, n_gather, n_scatter;
  std::vector<int64_t> gather_wg, scatter_wg;
  int maxp;
  std::vector<char> host_tables;
  std::vector<int> host_wg;
  std::vector<double> host_a;
  size_t table_bytes;
  bool use_graph;
  hipStream_t cap_stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace sparc {

// the step sequence of all problems (enqueued directly, or recorded into the graph)
static int plan_enqueue(sparc_filter_plan* P) {
  const size_t eb = elem_bytes(P->dt);
  for (int j = 0; j < P->max_deg; ++j) {
    const auto& mem = P->members[j];
    // projections of the step input (all problems, one launch)
    const size_t t0 = (size_t)j * P->n_prob, o0 = (size_t)j * (P->n_prob + 1);
    SPARC_TRY(nl_gather_batched(P->ctx, P->dt, P->maxp, P->dev_gather + t0, P->dev_goff + o0, P->n_gather[j],
                                P->gather_wg[j]));
    SPARC_TRY(step_table_launch(P->ctx, P->dt, P->n_o, P->tile, P->dev_tables + P->table_off[j],
                                P->dev_wg + P->wg_off[j], (int)mem.size(), P->total_wg[j], P->dir, P->nl_lds[j]));
    // projector scatters of the problems that do not apply them inside the step (one launch)
    SPARC_TRY(nl_scatter_batched(P->ctx, P->dt, P->dev_scatter + t0, P->dev_soff + o0, P->n_scatter[j],
                                 P->scatter_wg[j], P->dev_a + (size_t)j * P->n_prob));
  }
  // Y_m of an odd degree sits in the work block
  for (int p = 0; p < P->n_prob; ++p)
    if ((P->deg[p] - 1) % 2 == 0)
      SPARC_HIP(hipMemcpy2DAsync(P->X[p], P->ldx[p] * eb, P->W[p], P->H[p]->n_d * eb, P->H[p]->n_d * eb, P->n_s[p],
                                 hipMemcpyDeviceToDevice, P->ctx->stream));
  return SPARC_OK;
}

// host tables for the given bounds (pointers fixed, coefficients per problem)
static int plan_tables(sparc_filter_plan* P, const double* lcut, const double* lmax) {
  std::vector<StepDesc> d;
  std::vector<sparc_ham*> hs;
  for (int j = 0; j < P->max_deg; ++j) {
    d.clear();
    hs.clear();
    P->n_gather[j] = P->n_scatter[j] = 0;
    P->gather_wg[j] = P->scatter_wg[j] = 0;
    for (int p : P->members[j]) {
      const double c = 0.5 * (lmax[p] + lcut[p]), e = 0.5 * (lmax[p] - lcut[p]);
      StepDesc s;
      s.n_s = P->n_s[p];
      const int64_t nd = P->H[p]->n_d;
      if (j == 0) {
        s.x = P->X[p]; s.ldx = P->ldx[p];
        s.z = nullptr; s.ldz = 0;
        s.out = P->W[p]; s.ldo = nd;
        s.a = 1.0 / e; s.b = -c / e; s.c = 0.0;
      } else {
        const bool x_in_w = (j - 1) % 2 == 0;  // Y_j in W for odd j
        s.x = x_in_w ? P->W[p] : P->X[p];
        s.ldx = x_in_w ? nd : P->ldx[p];
        s.out = x_in_w ? P->X[p] : P->W[p];
        s.ldo = x_in_w ? P->ldx[p] : nd;
        s.z = s.out; s.ldz = s.ldo;
        s.a = 2.0 / e; s.b = -2.0 * c / e; s.c = -1.0;
      }
      s.alpha = P->fused[p] ? P->alpha[p] : nullptr;
      P->host_a[(size_t)j * P->n_prob + p] = s.a;
      d.push_back(s);
      hs.push_back(P->H[p]);
      // projections of Y_j and (separate form) the scatter into Y_{j+1}
      NlBatchArgs nb;
      int gw = 0, sw = 0;
      nl_batch_args(P->H[p], s.x, s.ldx, s.out, s.ldo, s.n_s, P->alpha[p], p, &nb, &gw, &sw);
      if (gw > 0) {
        P->host_gather[(size_t)j * P->n_prob + P->n_gather[j]] = nb;
        P->host_goff[(size_t)j * (P->n_prob + 1) + P->n_gather[j]] = (int)P->gather_wg[j];
        P->gather_wg[j] += gw;
        P->n_gather[j]++;
      }
      if (sw > 0 && !P->fused[p]) {
        P->host_scatter[(size_t)j * P->n_prob + P->n_scatter[j]] = nb;
        P->host_soff[(size_t)j * (P->n_prob + 1) + P->n_scatter[j]] = (int)P->scatter_wg[j];
        P->scatter_wg[j] += sw;
        P->n_scatter[j]++;
      }
    }
    P->host_goff[(size_t)j * (P->n_prob + 1) + P->n_gather[j]] = (int)P->gather_wg[j];
    P->host_soff[(size_t)j * (P->n_prob + 1) + P->n_scatter[j]] = (int)P->scatter_wg[j];
    P->nl_lds[j] = 0;
    if (d.empty()) continue;
    int64_t tot = step_table_build(hs.data(), d.data(), (int)d.size(), P->tile,
                                   P->host_tables.data() + P->table_off[j], P->host_wg.data() + P->wg_off[j],
                                   &P->nl_lds[j]);
    if (tot < 0) return fail(SPARC_EINVAL, "filter plan: bad dtype");
    P->total_wg[j] = tot;
  }
  return SPARC_OK;
}

// Stencil tile of a plan when the context autotunes: every shape is timed on the plan's
// own batched step over all problems, in the recurrence's memory pattern (X_p read,
// W_p read and written: x = X_p, z = out = W_p), three launches back to back after a
// warm-up, best of two such runs; X is only read and W is workspace.  The choice is
// kept per set of problem shapes.
static std::mutex g_plan_tune_mu;
static std::map<std::vector<int>, int> g_plan_tune;

static int plan_tune_tile(sparc_filter_plan* P) {
  std::vector<int> key;
  for (int p = 0; p < P->n_prob; ++p) {
    const sparc_ham* h = P->H[p];
    key.insert(key.end(), {h->grid.n[0], h->grid.n[1], h->grid.n[2], P->n_s[p], (int)h->dtype, h->grid.n_o,
                           dirichlet_mask(h->grid)});
  }
  {
    std::lock_guard<std::mutex> lk(g_plan_tune_mu);
    auto it = g_plan_tune.find(key);
    if (it != g_plan_tune.end()) { P->tile = it->second; return SPARC_OK; }
  }
  sparc_ctx* ctx = P->ctx;
  const int n = P->n_prob;
  std::vector<StepDesc> d(n);
  std::vector<sparc_ham*> hs(P->H);
  hipEvent_t e0, e1;
  SPARC_HIP(hipEventCreate(&e0));
  SPARC_HIP(hipEventCreate(&e1));
  const bool timing = ctx->timing;
  ctx->timing = false;
  int best = P->tile, rc = SPARC_OK;
  float best_ms = 1e30f;
  char* tab = P->host_tables.data() + P->table_off[0];
  int* wg = P->host_wg.data() + P->wg_off[0];
  // step 0 has every problem as a member: its table and offsets hold n blocks
  const size_t tab_bytes = (P->max_deg > 1 ? P->table_off[1] : P->table_bytes) - P->table_off[0];
  for (int t = 0; t < tile_shape_count() && rc == SPARC_OK; ++t) {
    if (tile_shape_threads(t) > 1024) continue;
    for (int p = 0; p < n; ++p) {
      StepDesc& s = d[p];
      const int64_t nd = P->H[p]->n_d;
      s.n_s = P->n_s[p];
      s.x = P->X[p]; s.ldx = P->ldx[p];
      s.z = P->W[p]; s.ldz = nd;
      s.out = P->W[p]; s.ldo = nd;
      s.a = 0.05; s.b = 0.0; s.c = 0.0;
      s.alpha = nl_step_fused(P->H[p], t) ? P->alpha[p] : nullptr;
    }
    size_t lds = 0;
    const int64_t tot = step_table_build(hs.data(), d.data(), n, t, tab, wg, &lds);
    if (tot < 0) { rc = fail(SPARC_EINVAL, "filter plan: bad dtype"); break; }
    hipError_t e = hipMemcpyAsync(P->dev_tables + P->table_off[0], tab, tab_bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(P->dev_wg + P->wg_off[0], wg, (size_t)(n + 1) * sizeof(int), hipMemcpyHostToDevice,
                         ctx->stream);
    if (e != hipSuccess) { rc = fail(SPARC_EDEVICE, "filter plan: %s", hipGetErrorString(e)); break; }
    auto launch = [&]() {
      return step_table_launch(ctx, P->dt, P->n_o, t, P->dev_tables + P->table_off[0], P->dev_wg + P->wg_off[0], n,
                               tot, P->dir, lds);
    };
    rc = launch();  // warm-up
    float t_best = 1e30f;
    for (int r = 0; r < 2 && rc == SPARC_OK; ++r) {
      hipEventRecord(e0, ctx->stream);
      for (int q = 0; q < 3 && rc == SPARC_OK; ++q) rc = launch();
      hipEventRecord(e1, ctx->stream);
      if (rc != SPARC_OK) break;
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      t_best = std::min(t_best, ms);
    }
    if (rc == SPARC_OK && t_best < best_ms) { best_ms = t_best; best = t; }
  }
  ctx->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SPARC_OK) return rc;
  P->tile = best;
  std::lock_guard<std::mutex> lk(g_plan_tune_mu);
  g_plan_tune[key] = best;
  return SPARC_OK;
}

}  // namespace sparc

extern "C" {

size_t sparc_filter_plan_workspace_bytes(int32_t n_prob, sparc_ham* const* H, const int32_t* n_s, const int32_t* degree) {
  if (n_prob < 1 || !H || !n_s || !degree) return 0;
  size_t b = 0;
  int max_deg = 0;
  for (int p = 0; p < n_prob; ++p) {
    if (!H[p]) return 0;
    b += al256((size_t)H[p]->n_d * n_s[p] * elem_bytes(H[p]->dtype));
    b += al256(alpha_bytes(H[p], n_s[p]));
    max_deg = std::max(max_deg, degree[p]);
  }
  b += al256((size_t)max_deg * n_prob * step_args_bytes(H[0]->dtype));
  b += al256((size_t)max_deg * (n_prob + 1) * sizeof(int));
  b += al256((size_t)max_deg * n_prob * sizeof(double));
  b += 2 * al256((size_t)max_deg * n_prob * sizeof(NlBatchArgs));
  b += 2 * al256((size_t)max_deg * (n_prob + 1) * sizeof(int));
  return b;
}

int sparc_filter_plan_create(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X, const int64_t* ldx,
                             const int32_t* n_s, const int32_t* degree, int32_t use_graph, void* work,
                             size_t work_bytes, sparc_filter_plan** out) {
  if (!ctx || !H || !X || !ldx || !n_s || !degree || !out) return fail(SPARC_EINVAL, "filter plan: null argument");
  *out = nullptr;
  if (n_prob < 1) return fail(SPARC_EINVAL, "filter plan: n_prob < 1");
  for (int p = 0; p < n_prob; ++p) {
    if (!H[p] || !X[p]) return fail(SPARC_EINVAL, "filter plan: problem %d has a null pointer", p);
    if (H[p]->ctx != ctx) return fail(SPARC_EINVAL, "filter plan: problem %d belongs to another context", p);
    if (H[p]->dtype != H[0]->dtype || H[p]->grid.n_o != H[0]->grid.n_o)
      return fail(SPARC_EINVAL, "filter plan: all problems need the same dtype and stencil order");
    if (n_s[p] < 1 || ldx[p] < H[p]->n_d) return fail(SPARC_ESHAPE, "filter plan: problem %d has a bad n_s or ld", p);
    if (degree[p] < 1) return fail(SPARC_EINVAL, "filter plan: problem %d has degree < 1", p);
  }
  size_t need = sparc_filter_plan_workspace_bytes(n_prob, H, n_s, degree);
  if (!work || work_bytes < need) return fail(SPARC_ENOMEM, "filter plan: workspace %zu < %zu bytes", work_bytes, need);
  sparc_filter_plan* P = new sparc_filter_plan();
  P->ctx = ctx;
  P->dt = H[0]->dtype;
  P->n_o = H[0]->grid.n_o;
  P->n_prob = n_prob;
  P->max_deg = *std::max_element(degree, degree + n_prob);
  P->H.assign(H, H + n_prob);
  P->X.assign(X, X + n_prob);
  P->ldx.assign(ldx, ldx + n_prob);
  P->n_s.assign(n_s, n_s + n_prob);
  P->deg.assign(degree, degree + n_prob);
  char* w = (char*)work;
  for (int p = 0; p < n_prob; ++p) {
    P->W.push_back(w);
    w += al256((size_t)H[p]->n_d * n_s[p] * elem_bytes(P->dt));
    P->alpha.push_back(w);
    w += al256(alpha_bytes(H[p], n_s[p]));
  }
  const size_t ab = step_args_bytes(P->dt);
  P->table_bytes = (size_t)P->max_deg * n_prob * ab;
  P->dev_tables = w;
  w += al256(P->table_bytes);
  P->dev_wg = (int*)w;
  w += al256((size_t)P->max_deg * (n_prob + 1) * sizeof(int));
  P->dev_a = (double*)w;
  w += al256((size_t)P->max_deg * n_prob * sizeof(double));
  P->dev_gather = (NlBatchArgs*)w;
  w += al256((size_t)P->max_deg * n_prob * sizeof(NlBatchArgs));
  P->dev_scatter = (NlBatchArgs*)w;
  w += al256((size_t)P->max_deg * n_prob * sizeof(NlBatchArgs));
  P->dev_goff = (int*)w;
  w += al256((size_t)P->max_deg * (n_prob + 1) * sizeof(int));
  P->dev_soff = (int*)w;
  P->host_gather.assign((size_t)P->max_deg * n_prob, NlBatchArgs{});
  P->host_scatter.assign((size_t)P->max_deg * n_prob, NlBatchArgs{});
  P->host_goff.assign((size_t)P->max_deg * (n_prob + 1), 0);
  P->host_soff.assign((size_t)P->max_deg * (n_prob + 1), 0);
  P->n_gather.assign(P->max_deg, 0);
  P->n_scatter.assign(P->max_deg, 0);
  P->gather_wg.assign(P->max_deg, 0);
  P->scatter_wg.assign(P->max_deg, 0);
  P->maxp = 0;
  for (int p = 0; p < n_prob; ++p) P->maxp = std::max(P->maxp, H[p]->max_proj_per_atom);
  P->nl_lds.assign(P->max_deg, 0);
  P->members.resize(P->max_deg);
  P->total_wg.assign(P->max_deg, 0);
  size_t toff = 0, woff = 0;
  for (int j = 0; j < P->max_deg; ++j) {
    for (int p = 0; p < n_prob; ++p)
      if (degree[p] > j) P->members[j].push_back(p);
    P->table_off.push_back(toff);
    P->wg_off.push_back(woff);
    toff += P->members[j].size() * ab;
    woff += P->members[j].size() + 1;
  }
  P->host_tables.assign(P->table_bytes, 0);
  P->host_wg.assign((size_t)P->max_deg * (n_prob + 1), 0);
  P->host_a.assign((size_t)P->max_deg * n_prob, 0.0);
  // stencil tile: autotuned on the largest problem when the context asks for it
  int big = 0;
  for (int p = 1; p < n_prob; ++p)
    if ((double)H[p]->n_d * n_s[p] > (double)H[big]->n_d * n_s[big]) big = p;
  P->tile = heuristic_tile(H[big]->grid.n[0], H[big]->grid.n[1], elem_bytes(P->dt));
  P->dir = 0;
  for (int p = 0; p < n_prob; ++p) P->dir |= dirichlet_mask(H[p]->grid) != 0 ? 1 : 0;
  if (ctx->autotune) {
    int rc = plan_tune_tile(P);
    if (rc != SPARC_OK) { delete P; return rc; }
  }
  for (int p = 0; p < n_prob; ++p) P->fused.push_back(nl_step_fused(H[p], P->tile) ? 1 : 0);
  P->use_graph = use_graph != 0;
  P->cap_stream = nullptr;
  P->graph = nullptr;
  P->exec = nullptr;
  if (P->use_graph) {
    // capture on a private stream (the context's stream may be the default stream)
    std::vector<double> lc(n_prob, 0.0), lm(n_prob, 1.0);
    int rc = plan_tables(P, lc.data(), lm.data());
    hipError_t e = hipSuccess;
    if (rc == SPARC_OK) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (rc == SPARC_OK && e == hipSuccess) {
      hipStream_t saved = ctx->stream;
      const bool timing = ctx->timing;
      ctx->stream = P->cap_stream;
      ctx->timing = false;
      e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = plan_enqueue(P);
        hipError_t e2 = hipStreamEndCapture(P->cap_stream, &P->graph);
        if (rc == SPARC_OK && e2 != hipSuccess) e = e2;
      }
      ctx->stream = saved;
      ctx->timing = timing;
      if (rc == SPARC_OK && e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    }
    if (rc != SPARC_OK || e != hipSuccess) {
      sparc_filter_plan_destroy(P);
      if (rc != SPARC_OK) return rc;
      return fail(SPARC_EDEVICE, "filter plan: graph capture failed: %s", hipGetErrorString(e));
    }
  }
  *out = P;
  return SPARC_OK;
}

int sparc_filter_plan_run(sparc_filter_plan* P, const double* lambda_cut, const double* lambda_max) {
  if (!P || !lambda_cut || !lambda_max) return fail(SPARC_EINVAL, "filter plan run: null argument");
  for (int p = 0; p < P->n_prob; ++p)
    if (!(lambda_max[p] > lambda_cut[p]) || !std::isfinite(lambda_max[p]) || !std::isfinite(lambda_cut[p]))
      return fail(SPARC_EINVAL, "filter plan run: problem %d needs finite lambda_max > lambda_cut", p);
  SPARC_TRY(plan_tables(P, lambda_cut, lambda_max));
  hipStream_t s = P->ctx->stream;
  SPARC_HIP(hipMemcpyAsync(P->dev_tables, P->host_tables.data(), P->table_bytes, hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(P->dev_wg, P->host_wg.data(), P->host_wg.size() * sizeof(int), hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(P->dev_a, P->host_a.data(), P->host_a.size() * sizeof(double), hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(P->dev_gather, P->host_gather.data(), P->host_gather.size() * sizeof(NlBatchArgs),
                           hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(P->dev_scatter, P->host_scatter.data(), P->host_scatter.size() * sizeof(NlBatchArgs),
                           hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(P->dev_goff, P->host_goff.data(), P->host_goff.size() * sizeof(int), hipMemcpyHostToDevice,
                           s));
  SPARC_HIP(hipMemcpyAsync(P->dev_soff, P->host_soff.data(), P->host_soff.size() * sizeof(int), hipMemcpyHostToDevice,
                           s));
  if (P->use_graph) {
    int t = timer_begin(P->ctx, "filter_graph");
    SPARC_HIP(hipGraphLaunch(P->exec, s));
    timer_end(P->ctx, t);
    // the host tables must stay unchanged until the uploads above have been consumed
    SPARC_HIP(hipStreamSynchronize(s));
    return SPARC_OK;
  }
  int rc = plan_enqueue(P);
  if (rc == SPARC_OK) SPARC_HIP(hipStreamSynchronize(s));
  return rc;
}

void sparc_filter_plan_destroy(sparc_filter_plan* P) {
  if (!P) return;
  if (P->exec) hipGraphExecDestroy(P->exec);
  if (P->graph) hipGraphDestroy(P->graph);
  if (P->cap_stream) hipStreamDestroy(P->cap_stream);
  delete P;
}

int chebyshev_filter_batched(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X, const int64_t* ldx,
                             const int32_t* n_s, const int32_t* degree, const double* lambda_cut,
                             const double* lambda_max, void* work, size_t work_bytes) {
  sparc_filter_plan* P = nullptr;
  SPARC_TRY(sparc_filter_plan_create(ctx, n_prob, H, X, ldx, n_s, degree, 0, work, work_bytes, &P));
  int rc = sparc_filter_plan_run(P, lambda_cut, lambda_max);
  sparc_filter_plan_destroy(P);
  return rc;
}

int rayleigh_ritz_batched(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X, const int64_t* ldx,
                          const int32_t* n_s, sparc_gemm_mode mode, double* const* ritz_dev, void* work,
                          size_t work_bytes) {
  if (!ctx || !H || !X || !ldx || !n_s || !ritz_dev) return fail(SPARC_EINVAL, "rayleigh_ritz_batched: null argument");
  if (n_prob < 1) return fail(SPARC_EINVAL, "rayleigh_ritz_batched: n_prob < 1");
  for (int p = 0; p < n_prob; ++p) {
    if (!H[p] || H[p]->ctx != ctx) return fail(SPARC_EINVAL, "rayleigh_ritz_batched: problem %d has no/another context", p);
    int32_t info = 0;
    SPARC_TRY(rayleigh_ritz(H[p], X[p], ldx[p], n_s[p], mode, ritz_dev[p], work, work_bytes, &info));
  }
  return SPARC_OK;
}

size_t sparc_rr_batched_workspace_bytes(int32_t n_prob, sparc_ham* const* H, const int32_t* n_s) {
  size_t b = 0;
  for (int p = 0; p < n_prob; ++p) b = std::max(b, sparc_workspace_bytes(H[p], n_s[p], SPARC_OP_RR));
  return b;
}

int sparc_ctx_set_autotune(sparc_ctx* ctx, int enable) {
  if (!ctx) return fail(SPARC_EINVAL, "sparc_ctx_set_autotune: ctx is NULL");
  ctx->autotune = enable != 0;
  return SPARC_OK;
}

}  // extern "C"
