// Batched dense t-SVD: many independent problems of uneven shape in a few
// grouped launches (Gram, power iteration, finishing product).
//
// The method per problem is the single-problem one (Algorithm 1 on the Gram
// of Algorithm 2/3): only the scheduling differs.
//   Gram:   one launch per (Gram mode, side) whose workgroups are the
//           (problem, split-K chunk, 128x128 triangle tile) units of every
//           problem, then one deterministic reduction launch.
//   Power:  cooperative launches ("rounds"); in each, the CUs are split into
//           teams and every team solves its list of problems one after the
//           other with its own exchange buffers (a team is to one problem what
//           the whole grid is to a single call).
//   Finish: one grouped FP64 product launch per side, then sigma and scale/sign.
//
// A problem's team size depends only on its own Gram dimension and the
// context's team_kib (teams host only problems of their own size), and its
// Gram chunking only on its own contraction length, so its result does not
// depend on which other problems share the batch: a problem solved alone and
// in any mix gives the same bits.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "batched.h"
#include "common.h"

namespace tsvd {

namespace {

constexpr int kTile = 128;  // grouped Gram tile edge

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

// Rounds of teams.  Problems are taken longest first; each joins the
// least-loaded team of its own size in the current round if that finishes no
// later than the round's longest team, else opens a new team while CUs remain,
// else waits for the next round.
void plan_rounds(std::vector<ProbPlan>& P, int num_cu, std::vector<RoundPlan>& rounds) {
  std::vector<int> todo(P.size());
  std::iota(todo.begin(), todo.end(), 0);
  std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) {
    return team_cost(P[a].d, P[a].k, P[a].G) > team_cost(P[b].d, P[b].k, P[b].G);
  });
  while (!todo.empty()) {
    RoundPlan r;
    int free_cu = num_cu;
    double longest = 0.0;
    std::vector<int> later;
    for (int i : todo) {
      const double c = team_cost(P[i].d, P[i].k, P[i].G);
      int best = -1;
      double best_end = 1e300;
      for (size_t t = 0; t < r.teams.size(); t++) {
        if (r.teams[t].size != P[i].G) continue;
        const double end = r.teams[t].load + c;
        if (end < best_end) { best_end = end; best = (int)t; }
      }
      if (best >= 0 && best_end <= std::max(longest, c)) {
        r.teams[best].probs.push_back(i);
        r.teams[best].load = best_end;
        longest = std::max(longest, best_end);
      } else if (free_cu >= P[i].G) {
        TeamPlan t;
        t.size = P[i].G;
        t.first = num_cu - free_cu;
        free_cu -= P[i].G;
        t.probs.push_back(i);
        t.load = c;
        longest = std::max(longest, c);
        r.teams.push_back(t);
      } else if (best >= 0) {
        r.teams[best].probs.push_back(i);
        r.teams[best].load = best_end;
        longest = std::max(longest, best_end);
      } else {
        later.push_back(i);
      }
    }
    r.grid = 0;
    for (auto& t : r.teams) r.grid = std::max(r.grid, t.first + t.size);
    rounds.push_back(std::move(r));
    todo.swap(later);
  }
}

}  // namespace

tsvd_status batch_plan(tsvd_ctx* ctx, int count, const tsvd_problem* probs, BatchPlan& bp) {
  const int team_kib = ctx->tuning.team_kib > 0 ? ctx->tuning.team_kib : 128;
  const int64_t kc_target = ctx->tuning.group_kchunk > 0 ? ctx->tuning.group_kchunk : 2048;
  bp.count = count;
  bp.P.assign(count, ProbPlan());
  bp.rounds.clear();
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
    // Gram split-K: chunks of about kc_target contraction rows, at most 4096
    // partial tiles per problem
    p.nt = (int)((p.d + kTile - 1) / kTile);
    p.T = p.nt * (p.nt + 1) / 2;
    int64_t S = std::max<int64_t>(1, (p.K + kc_target / 2) / kc_target);
    S = std::min<int64_t>(S, std::max<int64_t>(1, 4096 / p.T));
    int64_t kchunk = (p.K + S - 1) / S;
    kchunk = (kchunk + 31) / 32 * 32;
    p.S = (int)((p.K + kchunk - 1) / kchunk);
    p.kchunk = kchunk;
    const int64_t M = p.right ? q.m : q.n;
    p.nb = (int)((M + 127) / 128);
    p.G = wanted_team(p.d, ctx->num_cu, team_kib);
    if (power_plan(4, (int)p.d, p.k, ctx->num_cu, ctx->max_lds, p.G, &p.pp))
      return fail(ctx, TSVD_ERR_UNSUPPORTED, "problem %d: d=%lld too large for the LDS-resident iterate", i,
                  (long long)p.d);
    p.G = p.pp.G;
    // per-problem workspace: B, the split-K partial tiles, the finish's column sums
    size_t off = 0;
    auto take = [&](size_t b) { off = align256(off); const size_t o2 = off; off += b; return o2; };
    p.off_B = take((size_t)p.d * p.ldb * 4);
    p.off_partial = take((size_t)p.S * p.T * kTile * kTile * 4);
    p.off_ssq = take((size_t)p.nb * p.k * 8);
    p.ws_bytes = align256(off);
  }
  plan_rounds(bp.P, ctx->num_cu, bp.rounds);

  // batch-level workspace: descriptors, statuses and iteration logs, team buffers
  size_t off = 0;
  auto take = [&](size_t b) { off = align256(off); const size_t o2 = off; off += b; return o2; };
  int nteams = 0, ntob = 0;
  for (auto& r : bp.rounds) { nteams += (int)r.teams.size(); ntob += r.grid; }
  bp.nteams = nteams;
  bp.ntob = ntob;
  bp.off_gjobs = take((size_t)count * sizeof(GramJob));
  bp.off_pargs = take((size_t)count * sizeof(PowerArgs));
  bp.off_order = take((size_t)count * sizeof(int));
  bp.off_teams = take((size_t)nteams * sizeof(PowerTeam));
  bp.off_tob = take((size_t)ntob * sizeof(int));
  bp.off_fjobs = take((size_t)count * sizeof(FinishJob));
  bp.total_k = 0;
  for (auto& p : bp.P) bp.total_k += p.k;
  bp.off_fixed = take(bp.total_k * sizeof(int));
  bp.desc_bytes = off;  // everything above is uploaded in one copy
  bp.off_status = take((size_t)count * 4 * sizeof(int));
  bp.off_iters = take(bp.total_k * sizeof(int));
  bp.off_lambda = take(bp.total_k * sizeof(double));
  bp.off_ex = align256(off);
  for (auto& r : bp.rounds)
    for (auto& t : r.teams) {
      for (int i : t.probs) {
        t.dpad_max = std::max(t.dpad_max, (int)((bp.P[i].d + 3) & ~3));
        t.k_max = std::max(t.k_max, bp.P[i].k);
      }
      const size_t xw = (size_t)t.dpad_max, pw = (size_t)2 * (t.k_max + 2), vs = (size_t)2 * t.dpad_max;
      t.off_ex = take((2 * xw + 2 * (size_t)t.size * pw + 4 * vs) * 8);
    }
  bp.ex_words = (align256(off) - bp.off_ex) / 8;
  for (auto& r : bp.rounds)
    for (auto& t : r.teams) t.off_kscr = take((size_t)t.size * 2 * (t.k_max + 2) * 8);
  bp.batch_ws_bytes = align256(off) + 256;
  return TSVD_OK;
}

tsvd_status batch_enqueue(tsvd_ctx* ctx, const tsvd_problem* probs, BatchPlan& bp, char* bbase,
                          char* const* pbase, hipStream_t stream, hipEvent_t* ev, char* hpin) {
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
  int* ord = (int*)(h + bp.off_order);
  PowerTeam* pt = (PowerTeam*)(h + bp.off_teams);
  int* tob = (int*)(h + bp.off_tob);
  FinishJob* fj = (FinishJob*)(h + bp.off_fjobs);
  std::vector<size_t> kofs(count);
  {
    size_t ko = 0;
    for (int i = 0; i < count; i++) { kofs[i] = ko; ko += bp.P[i].k; }
  }

  // Gram jobs grouped by (mode, side): contiguous runs, one launch each
  bp.ggroups.clear();
  {
    int gi = 0;
    for (int mode : {MODE_BF16X3, MODE_FP32})
      for (int side : {0, 1}) {
        BatchPlan::Group g{mode, side, gi, 0, 0, 0};
        for (int i = 0; i < count; i++) {
          const ProbPlan& p = bp.P[i];
          if (p.mode != mode || p.side != side) continue;
          const tsvd_problem& q = probs[i];
          GramJob& j = gj[gi++];
          j.A = q.A; j.m = q.m; j.n = q.n; j.lda = q.lda; j.side = side;
          j.nt = p.nt; j.T = p.T; j.S = p.S; j.kchunk = p.kchunk;
          j.vec_ok = (((uintptr_t)q.A & 15) == 0) && (q.lda % 4 == 0);
          j.partial = pbase[i] + p.off_partial;
          j.B = pbase[i] + p.off_B;
          j.ldb = p.ldb;
          j.ubegin = g.units;
          j.rbegin = g.runits;
          g.units += (int64_t)p.S * p.T;
          g.runits += (int64_t)16 * p.T;
          g.count++;
        }
        if (g.count) bp.ggroups.push_back(g);
      }
  }
  // teams, round by round
  {
    int oi = 0, ti = 0, bi = 0;
    for (auto& r : bp.rounds) {
      r.team0 = ti;
      r.tob0 = bi;
      for (int b = 0; b < r.grid; b++) tob[bi + b] = -1;
      for (auto& tp : r.teams) {
        PowerTeam& d = pt[ti];
        d.first = tp.first;
        d.size = tp.size;
        d.pbegin = oi;
        for (int i : tp.probs) ord[oi++] = i;
        d.pend = oi;
        d.xwords = tp.dpad_max;  // FP32 iterate: one word per element
        d.pw = 2 * (tp.k_max + 2);
        d.vstride = (int64_t)2 * tp.dpad_max;
        d.xex = (uint64_t*)(bbase + tp.off_ex);
        d.pex = d.xex + 2 * d.xwords;
        d.vex = d.pex + (size_t)2 * tp.size * d.pw;
        d.wex = d.vex + 2 * d.vstride;
        d.kscr = (double*)(bbase + tp.off_kscr);
        for (int b = 0; b < tp.size; b++) tob[bi + tp.first + b] = ti - r.team0;
        ti++;
      }
      bi += r.grid;
    }
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
    // exchange buffers, pw, xwords and vstride come from the team at run time
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
  if (hipMemsetAsync(d_status, 0, (size_t)count * 16, stream) != hipSuccess)
    return fail(ctx, TSVD_ERR_HIP, "memset status");
  for (int i = 0; i < count; i++) {
    const tsvd_problem& q = probs[i];
    const ProbPlan& p = bp.P[i];
    if (hipMemset2DAsync(q.U, q.ldu * 8, 0, q.m * 8, p.k, stream) != hipSuccess ||
        hipMemset2DAsync(q.V, q.ldv * 8, 0, q.n * 8, p.k, stream) != hipSuccess ||
        hipMemsetAsync(q.S, 0, (size_t)p.k * 8, stream) != hipSuccess)
      return fail(ctx, TSVD_ERR_HIP, "memset outputs of problem %d", i);
  }
  for (auto& g : bp.ggroups) {
    const int rc = syrk_grouped_launch(g.mode, g.side, (const GramJob*)(bbase + bp.off_gjobs) + g.first, g.count,
                                       g.units, g.runits, stream);
    if (rc) return from_internal(ctx, rc, "grouped gram");
  }
  if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  size_t lds = 0;
  for (auto& p : bp.P) lds = std::max(lds, p.pp.lds_bytes);
  for (size_t r = 0; r < bp.rounds.size(); r++) {
    const RoundPlan& rp = bp.rounds[r];
    const int rc = power_team_launch((const PowerArgs*)(bbase + bp.off_pargs), (const int*)(bbase + bp.off_order),
                                     (const PowerTeam*)(bbase + bp.off_teams) + rp.team0,
                                     (const int*)(bbase + bp.off_tob) + rp.tob0, rp.grid, lds,
                                     (uint64_t*)(bbase + bp.off_ex), r == 0 ? bp.ex_words : 0, stream);
    if (rc == -2) return fail(ctx, TSVD_ERR_UNSUPPORTED, "team power kernel does not fit on a CU");
    if (rc) return from_internal(ctx, rc, "team power iteration");
  }
  if (ev && hipEventRecord(ev[2], stream) != hipSuccess) return fail(ctx, TSVD_ERR_HIP, "event");
  {
    const FinishJob* dfj = (const FinishJob*)(bbase + bp.off_fjobs);
    int rc = finish_grouped_launch(0, dfj, bp.fcount[0], bp.funits[0], bp.fcols[0], stream);
    if (!rc) rc = finish_grouped_launch(1, dfj + bp.fcount[0], bp.fcount[1], bp.funits[1], bp.fcols[1], stream);
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
  tsvd_status st = batch_plan(ctx, count, probs, bp);
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
