// Batched dense t-SVD: many independent problems of uneven shape in one
// engine launch (Gram, reduction, power iteration) and a grouped finish.
//
// The method per problem is the single-problem one (Algorithm 1 on the Gram
// of Algorithm 2/3): only the scheduling differs.
//   Engine: one persistent launch whose workgroups take work items from one
//           list in order: per problem (queued longest first) its Gram units
//           (split-K chunk x triangle tile, the unit shape per Gram-dimension
//           class from the context's tuning), the reduction of each
//           tile's chunk partials into B, and the seats of its power team; a
//           team runs the single-problem body (a team is to one problem what
//           the whole grid is to a single call).  Later problems' Gram units
//           run beside earlier problems' teams.
//   Finish: one grouped FP64 product launch per side, then sigma and scale/sign.
//
// A problem's team size depends only on its own Gram dimension and the
// context's team_kib, a member's rows only on its rank in the team, and the
// Gram chunking only on the problem's contraction length, so its result does
// not depend on which other problems share the batch: a problem solved alone
// and in any mix gives the same bits.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "batched.h"
#include "common.h"

namespace tsvd {

namespace {

// Gram-dimension class of the per-class unit shapes: 0 for d <= 128, c for
// 2^(6+c) < d <= 2^(7+c), the last class for anything larger
int gram_class(int64_t d) {
  int c = 0;
  while (c < TSVD_GRAM_CLASSES - 1 && d > ((int64_t)128 << c)) c++;
  return c;
}

// library choice of the tile edge: 128 in every class.  A 128-edge tile
// does twice the MFMA work of a 64-edge one per panel load; even up to
// d = 128, where three 64-edge tiles skip a quarter of the square, they load
// each panel twice and measured slower (64 batched problems, d <= 128: 4.25
// against 4.4-4.7 ms per call)
int default_tile(int) { return 128; }

// workgroups a problem's power iteration runs on: enough to hold its Gram at
// team_kib per CU, at least 4 rows per workgroup
int wanted_team(int64_t d, int num_cu, int team_kib) {
  const double bytes = 4.0 * (double)d * (double)d;
  int64_t g = (int64_t)ceil(bytes / (team_kib * 1024.0));
  g = std::max<int64_t>(1, std::min<int64_t>(g, num_cu));
  g = std::min<int64_t>(g, (d + 3) / 4);
  return (int)std::max<int64_t>(g, 1);
}

// relative duration of a problem on its team: k triplets of GEMVs over the
// d x d Gram split g ways, with a floor for the exchange latency
double team_cost(int64_t d, int k, int g) { return (double)k * std::max((double)d * (double)d / g, 65536.0); }

}  // namespace

tsvd_status batch_plan(tsvd_ctx* ctx, int count, const tsvd_problem* probs, BatchPlan& bp, int team_cap) {
  const int cap = team_cap > 0 ? std::min(team_cap, ctx->num_cu) : ctx->num_cu;
  // default: 256 KiB of the problem's Gram per member, about what a member
  // holds on chip (LDS rows plus register rows) up to a dimension of 8192
  const int team_kib = ctx->tuning.team_kib > 0 ? ctx->tuning.team_kib : 256;
  const int64_t kc_default = ctx->tuning.group_kchunk > 0 ? ctx->tuning.group_kchunk : 2048;
  bp.count = count;
  bp.P.assign(count, ProbPlan());
  for (int i = 0; i < count; i++) {
    const tsvd_problem& q = probs[i];
    const tsvd_opts& o = q.opts;
    ProbPlan& p = bp.P[i];
    if (!q.A || !q.U || !q.S || !q.V || !o.v0) return fail(ctx, TSVD_ERR_INVALID_ARG, "problem %d: null pointer", i);
    if (q.m < 1 || q.n < 1 || q.lda < q.n || q.ldu < q.m || q.ldv < q.n)
      return fail(ctx, TSVD_ERR_INVALID_ARG, "problem %d: bad shape or leading dimension", i);
    if (q.dtype != TSVD_F32) return fail(ctx, TSVD_ERR_UNSUPPORTED, "problem %d: the batched path takes FP32 A", i);
    const int mode = gram_mode(o.gram, TSVD_F32);
    if (mode != MODE_FP32 && mode != MODE_BF16X3)
      return fail(ctx, TSVD_ERR_UNSUPPORTED, "problem %d: gram must be AUTO, FP32 or BF16X3", i);
    if (o.branch != 0 && o.branch != 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "problem %d: bad branch", i);
    const int64_t mn = std::min(q.m, q.n);
    const int k = o.k == -1 ? (int)mn : o.k;
    if (k < 1 || k > mn)
      return fail(ctx, TSVD_ERR_INVALID_ARG, "problem %d: k=%d outside [1, %lld]", i, o.k, (long long)mn);
    if (o.fixed_iters)
      for (int l = 0; l < k; l++)
        if (o.fixed_iters[l] < 1) return fail(ctx, TSVD_ERR_INVALID_ARG, "problem %d: fixed_iters[%d] < 1", i, l);
    p.right = right_side(q.m, q.n, o.branch);
    p.side = p.right ? TSVD_SIDE_RIGHT : TSVD_SIDE_LEFT;
    p.mode = mode;
    p.d = p.right ? q.n : q.m;
    p.K = p.right ? q.m : q.n;
    p.k = k;
    p.ldb = (p.d + 3) & ~(int64_t)3;
    if (p.d > 32768)
      return fail(ctx, TSVD_ERR_UNSUPPORTED, "problem %d: Gram dimension %lld too large for the batched path", i,
                  (long long)p.d);
    // Gram work units: the class's tile edge, split-K chunks of about the
    // class's contraction rows, the chunk count capped so that the partials
    // would fill at most 4096 tiles of edge 128 (the same bytes for edge 64):
    // the chunking, and so every result bit, does not depend on the edge
    const int cls = gram_class(p.d);
    p.bm = ctx->tuning.group_tile[cls] > 0 ? ctx->tuning.group_tile[cls] : default_tile(cls);
    const int64_t kc_target = ctx->tuning.group_kchunk_cls[cls] > 0 ? ctx->tuning.group_kchunk_cls[cls] : kc_default;
    p.nt = (int)((p.d + p.bm - 1) / p.bm);
    p.T = p.nt * (p.nt + 1) / 2;
    const int64_t nt128 = (p.d + 127) / 128, T128 = nt128 * (nt128 + 1) / 2;
    int64_t S = std::max<int64_t>(1, (p.K + kc_target / 2) / kc_target);
    S = std::min<int64_t>(S, std::max<int64_t>(1, 4096 / T128));
    int64_t kchunk = (p.K + S - 1) / S;
    kchunk = (kchunk + 31) / 32 * 32;
    p.S = (int)((p.K + kchunk - 1) / kchunk);
    p.kchunk = kchunk;
    const int64_t M = p.right ? q.m : q.n;
    p.nb = (int)((M + 127) / 128);
    p.G = wanted_team(p.d, cap, team_kib);
    // the engine kernel's own static LDS comes out of the per-workgroup budget
    if (power_plan(4, (int)p.d, p.k, ctx->num_cu, ctx->max_lds - engine_static_lds(), p.G, &p.pp))
      return fail(ctx, TSVD_ERR_UNSUPPORTED, "problem %d: d=%lld too large for the LDS-resident iterate", i,
                  (long long)p.d);
    p.G = p.pp.G;
    // per-problem workspace: B, the split-K partial tiles, the finish's column sums
    size_t off = 0;
    auto take = [&](size_t b) { off = align256(off); const size_t o2 = off; off += b; return o2; };
    p.off_B = take((size_t)p.d * p.ldb * 4);
    p.off_partial = take((size_t)p.S * p.T * p.bm * p.bm * 4);
    p.off_ssq = take((size_t)(p.nb + 2) * p.k * 8);
    p.ws_bytes = align256(off);
  }
  // power queue, longest first (stable: ties keep the caller's order)
  bp.queue.resize(count);
  std::iota(bp.queue.begin(), bp.queue.end(), 0);
  std::stable_sort(bp.queue.begin(), bp.queue.end(), [&](int x, int y) {
    return team_cost(bp.P[x].d, bp.P[x].k, bp.P[x].G) > team_cost(bp.P[y].d, bp.P[y].k, bp.P[y].G);
  });
  // the engine runs on every CU the cap allows (the Gram units of the whole
  // batch are spread over them; every team fits)
  bp.grid = cap;
  int64_t items = 0;
  for (auto& p : bp.P) items += (int64_t)p.S * p.T + p.T + p.G;
  if (items > (int64_t)1 << 30) return fail(ctx, TSVD_ERR_UNSUPPORTED, "batch too large (%lld work items)", (long long)items);
  bp.nitems = (int)items;

  // batch-level workspace: descriptors, statuses and iteration logs, then the
  // cleared region (queue counters and every problem's exchange buffers)
  size_t off = 0;
  auto take = [&](size_t b) { off = align256(off); const size_t o2 = off; off += b; return o2; };
  bp.off_gjobs = take((size_t)count * sizeof(GramJob));
  bp.off_pargs = take((size_t)count * sizeof(PowerArgs));
  bp.off_items = take((size_t)bp.nitems * sizeof(EngineItem));
  bp.off_fjobs = take((size_t)count * sizeof(FinishJob));
  bp.total_k = 0;
  for (auto& p : bp.P) bp.total_k += p.k;
  bp.off_fixed = take(bp.total_k * sizeof(int));
  bp.desc_bytes = off;  // everything above is uploaded in one copy
  bp.off_status = take((size_t)count * 4 * sizeof(int));
  bp.off_iters = take(bp.total_k * sizeof(int));
  bp.off_lambda = take(bp.total_k * sizeof(double));
  bp.off_zero = align256(off);
  bp.off_ctr = take((size_t)(4 * count + 1) * sizeof(int));
  for (auto& p : bp.P) {
    const size_t dpad = (size_t)((p.d + 3) & ~3), pw = (size_t)2 * (p.k + 2);
    p.ex_words = 2 * dpad + 2 * (size_t)p.G * pw + 8 * dpad;  // x (2 parities), partials, v and w
    p.off_ex = take(p.ex_words * 8);
  }
  bp.zero_words = (align256(off) - bp.off_zero) / 8;
  for (auto& p : bp.P) p.off_kscr = take((size_t)p.G * 2 * (p.k + 2) * 8);
  bp.batch_ws_bytes = align256(off) + 256;
  return TSVD_OK;
}

tsvd_status batch_enqueue(tsvd_ctx* ctx, const tsvd_problem* probs, BatchPlan& bp, char* bbase,
                          char* const* pbase, hipStream_t stream, hipEvent_t* ev, char* hpin, int* exit_flags,
                          int exit_id) {
  const int count = bp.count;
  if (hpin) {
    bp.desc = hpin;
    bp.hs = (int*)(hpin + align256(bp.desc_bytes));
    bp.hit = (int*)((char*)bp.hs + align256((size_t)count * 16));
    bp.hl = (double*)((char*)bp.hit + align256(bp.total_k * 4));
  } else {
    bp.desc_v.assign(bp.desc_bytes, 0);
    bp.hs_v.assign((size_t)count * 4, 0);
    bp.hit_v.assign(bp.total_k, 0);
    bp.hl_v.assign(bp.total_k, 0.0);
    bp.desc = bp.desc_v.data();
    bp.hs = bp.hs_v.data();
    bp.hit = bp.hit_v.data();
    bp.hl = bp.hl_v.data();
  }
  memset(bp.desc, 0, bp.desc_bytes);
  char* h = bp.desc;
  GramJob* gj = (GramJob*)(h + bp.off_gjobs);
  PowerArgs* pa = (PowerArgs*)(h + bp.off_pargs);
  FinishJob* fj = (FinishJob*)(h + bp.off_fjobs);
  std::vector<size_t> kofs(count);
  {
    size_t ko = 0;
    for (int i = 0; i < count; i++) { kofs[i] = ko; ko += bp.P[i].k; }
  }

  // one Gram job per problem (job i is problem i)
  for (int i = 0; i < count; i++) {
    const ProbPlan& p = bp.P[i];
    const tsvd_problem& q = probs[i];
    GramJob& j = gj[i];
    j.A = q.A; j.m = q.m; j.n = q.n; j.lda = q.lda; j.side = p.side; j.mode = p.mode;
    j.nt = p.nt; j.T = p.T; j.S = p.S; j.kchunk = p.kchunk; j.bm = p.bm;
    j.vec_ok = (((uintptr_t)q.A & 15) == 0) && (q.lda % 4 == 0);
    j.partial = pbase[i] + p.off_partial;
    j.B = pbase[i] + p.off_B;
    j.ldb = p.ldb;
  }
  // the engine's work list: per problem in power-queue order, its Gram units,
  // its tile reductions, then the seats of its team
  {
    EngineItem* it = (EngineItem*)(h + bp.off_items);
    int64_t n = 0;
    for (int qi = 0; qi < count; qi++) {
      const int i = bp.queue[qi];
      const ProbPlan& p = bp.P[i];
      for (int u = 0; u < p.S * p.T; u++) it[n++] = EngineItem{ITEM_GRAM, i, u, i, p.G, 0, 0, 0};
      for (int t = 0; t < p.T; t++) it[n++] = EngineItem{ITEM_REDUCE, i, t, i, p.G, 0, 0, 0};
      for (int r = 0; r < p.G; r++) it[n++] = EngineItem{ITEM_POWER, i, r, i, p.G, 0, 0, 0};
    }
    if (n != bp.nitems) return fail(ctx, TSVD_ERR_INTERNAL, "work list size %lld != %d", (long long)n, bp.nitems);
  }
  int* d_status = (int*)(bbase + bp.off_status);
  for (int i = 0; i < count; i++) {
    const ProbPlan& p = bp.P[i];
    const tsvd_problem& q = probs[i];
    PowerArgs& a = pa[i];
    memset(&a, 0, sizeof a);
    a.B = pbase[i] + p.off_B;
    a.ldb = p.ldb;
    a.d = (int)p.d;
    a.k = p.k;
    a.eps = q.opts.eps;
    a.max_iter = q.opts.max_iter > 0 ? q.opts.max_iter : 10000;
    a.fixed_iters = q.opts.fixed_iters ? (const int*)(bbase + bp.off_fixed) + kofs[i] : nullptr;
    a.v0 = q.opts.v0;
    a.X = p.right ? q.V : q.U;
    a.ldx = p.right ? q.ldv : q.ldu;
    a.lambda = (double*)(bbase + bp.off_lambda) + kofs[i];
    a.iters = (int*)(bbase + bp.off_iters) + kofs[i];
    a.status = d_status + 4 * i;
    a.rpb = p.pp.rpb;
    a.cache_rows = p.pp.cache_rows;
    a.ldsB = p.pp.ldsB;
    a.vec_ok = 1;  // B is 256-byte aligned with ldb a multiple of 4
    a.spin_limit = (int64_t)1 << 21;
    const int64_t dpad = (p.d + 3) & ~(int64_t)3;
    a.pw = 2 * (p.k + 2);
    a.xwords = dpad;  // FP32 iterate: one word per element
    a.vstride = 2 * dpad;
    a.xex = (uint64_t*)(bbase + p.off_ex);
    a.pex = a.xex + 2 * a.xwords;
    a.vex = a.pex + (int64_t)2 * p.G * a.pw;
    a.wex = a.vex + 2 * a.vstride;
    a.kscr = (double*)(bbase + p.off_kscr);
  }
  for (int i = 0; i < count; i++)
    if (probs[i].opts.fixed_iters)
      memcpy((int*)(h + bp.off_fixed) + kofs[i], probs[i].opts.fixed_iters, (size_t)bp.P[i].k * 4);
  // finish jobs grouped by side
  bp.fcount[0] = bp.fcount[1] = 0;
  bp.funits[0] = bp.funits[1] = 0;
  bp.fcols[0] = bp.fcols[1] = 0;
  {
    int fi = 0;
    for (int side : {0, 1})
      for (int i = 0; i < count; i++) {
        const ProbPlan& p = bp.P[i];
        if (p.side != side) continue;
        const tsvd_problem& q = probs[i];
        FinishJob& f = fj[fi++];
        f.A = q.A; f.m = q.m; f.n = q.n; f.lda = q.lda; f.side = p.side; f.k = p.k;
        f.U = q.U; f.ldu = q.ldu; f.V = q.V; f.ldv = q.ldv; f.S = q.S;
        f.ssq = (double*)(pbase[i] + p.off_ssq);
        f.kdone = d_status + 4 * i;  // status[0] = k_done
        f.nb = p.nb;
        f.ubegin = bp.funits[side];
        f.cbegin = bp.fcols[side];
        bp.funits[side] += (int64_t)f.nb * ((f.k + 63) / 64);
        bp.fcols[side] += f.k;
        bp.fcount[side]++;
      }
  }

  // ---- device work
  if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  if (hipMemcpyAsync(bbase, h, bp.desc_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "copy descriptors");
  if (int rc = zero_bytes_launch(d_status, (size_t)count * 16, stream)) return from_internal(ctx, rc, "clear status");
  {
    // every problem's U, V and S, one launch per side group
    const FinishJob* dfj0 = (const FinishJob*)(bbase + bp.off_fjobs);
    int rc = finish_grouped_zero_launch(dfj0, bp.fcount[0], bp.fcols[0], stream);
    if (!rc) rc = finish_grouped_zero_launch(dfj0 + bp.fcount[0], bp.fcount[1], bp.fcols[1], stream);
    if (rc) return from_internal(ctx, rc, "clear outputs");
  }
  if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  size_t lds = 0;
  for (auto& p : bp.P) lds = std::max(lds, p.pp.lds_bytes);
  {
    const int rc = engine_launch((const EngineItem*)(bbase + bp.off_items), bp.nitems,
                                 (const GramJob*)(bbase + bp.off_gjobs), (const PowerArgs*)(bbase + bp.off_pargs),
                                 (int*)(bbase + bp.off_ctr), count, bp.grid, lds, (uint64_t*)(bbase + bp.off_zero),
                                 bp.zero_words, stream, exit_flags, exit_id);
    if (rc == -2) return fail(ctx, TSVD_ERR_UNSUPPORTED, "batched engine kernel does not fit on a CU");
    if (rc) return from_internal(ctx, rc, "batched engine");
  }
  if (ev && hipEventRecord(ev[2], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  {
    const FinishJob* dfj = (const FinishJob*)(bbase + bp.off_fjobs);
    int64_t rows[2] = {0, 0};
    for (int i = 0; i < count; i++) rows[bp.P[i].side] = std::max(rows[bp.P[i].side], std::max(probs[i].m, probs[i].n));
    int rc = finish_grouped_launch(0, dfj, bp.fcount[0], bp.funits[0], bp.fcols[0], rows[0], stream);
    if (!rc)
      rc = finish_grouped_launch(1, dfj + bp.fcount[0], bp.fcount[1], bp.funits[1], bp.fcols[1], rows[1], stream);
    if (rc) return from_internal(ctx, rc, "grouped finish");
  }
  if (ev && hipEventRecord(ev[3], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  // small results to the host (valid once the stream has completed)
  if (hipMemcpyAsync(bp.hs, d_status, (size_t)count * 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(bp.hit, bbase + bp.off_iters, bp.total_k * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(bp.hl, bbase + bp.off_lambda, bp.total_k * 8, hipMemcpyDeviceToHost, stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "batched readback");
  return TSVD_OK;
}

tsvd_status batch_problem_result(const BatchPlan& bp, const tsvd_problem& q, int i, tsvd_info* info) {
  const ProbPlan& p = bp.P[i];
  const int* s = &bp.hs[(size_t)4 * i];
  tsvd_status si = TSVD_OK;
  if (s[2] == ERR_SPIN) si = TSVD_ERR_INTERNAL;
  else if (s[2] == ERR_NONFINITE) si = TSVD_ERR_NONFINITE;
  else if (s[2] == ERR_BADSTART) si = TSVD_ERR_INVALID_ARG;
  else if (!s[1] && !q.opts.fixed_iters && q.opts.eps > 0) si = TSVD_ERR_NOT_CONVERGED;
  if (info) {
    size_t ko = 0;
    for (int j = 0; j < i; j++) ko += bp.P[j].k;
    info->k_done = s[0];
    info->converged = s[1];
    info->rank_deficient = s[3];
    info->branch_right = p.right ? 1 : 0;
    if (info->iters) memcpy(info->iters, &bp.hit[ko], (size_t)p.k * 4);
    if (info->lambda) memcpy(info->lambda, &bp.hl[ko], (size_t)p.k * 8);
    info->h2d_bytes = 0;
    info->latency_ms = 0;
    info->t_stream_copy_ms = 0;
    info->t_stream_compute_ms = 0;
    info->t_stream_overlap_ms = 0;
  }
  return si;
}

}  // namespace tsvd

using namespace tsvd;

extern "C" {

tsvd_status tsvd_dense_batched(tsvd_ctx* ctx, int32_t count, const tsvd_problem* probs, int64_t hbm_budget,
                               tsvd_info* infos, int32_t* statuses, void* stream_) {
  if (!ctx) return TSVD_ERR_INVALID_ARG;
  if (count < 0 || (count > 0 && !probs)) return fail(ctx, TSVD_ERR_INVALID_ARG, "bad count or null problems");
  if (count == 0) return TSVD_OK;
  if (hbm_budget < 0) return fail(ctx, TSVD_ERR_INVALID_ARG, "hbm_budget < 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "hipSetDevice");
  hipStream_t stream = (hipStream_t)stream_;
  BatchPlan bp;
  tsvd_status st = batch_plan(ctx, count, probs, bp, ctx->tuning.power_blocks);
  if (st) return st;
  size_t need = bp.batch_ws_bytes;
  std::vector<size_t> poff(count);
  for (int i = 0; i < count; i++) {
    poff[i] = need;
    need += bp.P[i].ws_bytes;
  }
  st = ensure_ws(ctx, need, hbm_budget);
  if (st) return st;
  char* base = (char*)ctx->ws;
  std::vector<char*> pbase(count);
  for (int i = 0; i < count; i++) pbase[i] = base + poff[i];
  st = batch_enqueue(ctx, probs, bp, base, pbase.data(), stream, ctx->ev);
  if (st) return st;
  if (hipStreamSynchronize(stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "batched run: %s", hipGetErrorString(hipGetLastError()));
  float tg = 0, te = 0, tf = 0, tt = 0;
  (void)hipEventElapsedTime(&tg, ctx->ev[0], ctx->ev[1]);
  (void)hipEventElapsedTime(&te, ctx->ev[1], ctx->ev[2]);
  (void)hipEventElapsedTime(&tf, ctx->ev[2], ctx->ev[3]);
  (void)hipEventElapsedTime(&tt, ctx->ev[0], ctx->ev[3]);
  tsvd_status first_bad = TSVD_OK;
  int first_idx = -1;
  for (int i = 0; i < count; i++) {
    tsvd_info* in = infos ? &infos[i] : nullptr;
    const tsvd_status si = batch_problem_result(bp, probs[i], i, in);
    if (in) {
      in->t_gram_ms = tg;
      in->t_eig_ms = te;
      in->t_final_ms = tf;
      in->t_total_ms = tt;
      in->workspace_bytes = (int64_t)need;
    }
    if (statuses) statuses[i] = si;
    if (si != TSVD_OK && first_bad == TSVD_OK) { first_bad = si; first_idx = i; }
  }
  if (first_bad != TSVD_OK)
    return fail(ctx, first_bad, "problem %d of the batch: %s", first_idx, tsvd_status_string(first_bad));
  return TSVD_OK;
}

}  // extern "C"
