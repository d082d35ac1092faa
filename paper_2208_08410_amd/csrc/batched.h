// Planning and enqueueing of a batch of dense problems (shared by the batched
// entry point and the server).
#pragma once

#include <vector>

#include "ctx.h"
#include "internal.h"

namespace tsvd {

struct ProbPlan {
  bool right = true;
  int side = 0, mode = 0;
  int64_t d = 0, K = 0;
  int k = 0;
  int64_t ldb = 0;
  int bm = 0;                 // Gram tile edge (64 or 128)
  int nt = 0, T = 0, S = 0;   // Gram tiles per side, triangle tiles, split-K chunks
  int64_t kchunk = 0;
  int G = 0;                  // power team size (workgroups)
  PowerPlan pp = {};
  int nb = 0;                 // finish row tiles
  // per-problem workspace: offsets from the problem's base, total bytes
  size_t off_B = 0, off_partial = 0, off_ssq = 0, ws_bytes = 0;
  // power exchange buffers and scratch, in the batch workspace
  size_t off_ex = 0, ex_words = 0, off_kscr = 0;
};

struct BatchPlan {
  int count = 0;
  std::vector<ProbPlan> P;
  std::vector<int> queue;   // power queue: problem indices, longest first
  int grid = 0;             // engine workgroups
  int nitems = 0;           // engine work items (Gram units, reductions, team seats)
  // batch workspace layout
  size_t off_gjobs = 0, off_pargs = 0, off_items = 0, off_fjobs = 0, desc_bytes = 0;
  size_t off_status = 0, off_iters = 0, off_lambda = 0, off_fixed = 0;
  size_t off_zero = 0, zero_words = 0, off_ctr = 0;  // cleared by the engine launch
  size_t batch_ws_bytes = 0;
  size_t total_k = 0;
  // filled by batch_enqueue (host copies live until the stream completes)
  int fcount[2] = {0, 0};
  int64_t funits[2] = {0, 0}, fcols[2] = {0, 0};
  std::vector<char> desc_v;
  std::vector<int> hs_v, hit_v;
  std::vector<double> hl_v;
  char* desc = nullptr;  // host copies: in the vectors above, or in caller-given pinned memory
  int *hs = nullptr, *hit = nullptr;
  double* hl = nullptr;
  // pinned host bytes batch_enqueue needs when given a pinned staging area
  size_t host_bytes() const { return align256(desc_bytes) + align256((size_t)count * 16) + align256(total_k * 4) +
                                     align256(total_k * 8); }
};

// validate the problems and plan tiles, teams and workspace sizes; team_cap
// (0 = the CU count) bounds every team and the engine launch's grid
tsvd_status batch_plan(tsvd_ctx* ctx, int count, const tsvd_problem* probs, BatchPlan& bp, int team_cap = 0);
// enqueue the whole batch on `stream` (asynchronous).  bbase: batch workspace
// (bp.batch_ws_bytes); pbase[i]: problem i's workspace (bp.P[i].ws_bytes).
// ev (optional, 4 events) marks start / before the engine launch (the clears
// done) / after it (Gram, reductions and power iterations) / end.
// hpin (optional): pinned host memory of bp.host_bytes() for the descriptor
// upload and the result readback, so that no copy waits on the host; without
// it, pageable vectors are used.  The small results land in bp.hs / hit / hl
// once the stream has completed.
// exit_flags / exit_id: passed to the engine launch (its workgroups report
// their exit there, for the server's CU accounting)
tsvd_status batch_enqueue(tsvd_ctx* ctx, const tsvd_problem* probs, BatchPlan& bp, char* bbase, char* const* pbase,
                          hipStream_t stream, hipEvent_t* ev, char* hpin = nullptr, int* exit_flags = nullptr,
                          int exit_id = 0);
// status and info of problem i after the stream has completed
tsvd_status batch_problem_result(const BatchPlan& bp, const tsvd_problem& q, int i, tsvd_info* info);

}  // namespace tsvd
