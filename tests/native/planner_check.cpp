// Host-only run of the planner (aln_api.cpp) under AddressSanitizer and
// UndefinedBehaviorSanitizer, through a context without a device: random
// batches of every shape class under every mode, pruning rule and width,
// with and without CIGAR, planned, described and destroyed; the description
// must cover every pair once with disjoint traceback regions and CIGAR
// slots inside the footprint.  Bad arguments must come back as statuses.
// Prints OK.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "aln.h"

static int fail(const char *what, long long a, long long b) {
  std::printf("FAIL %s %lld %lld\n", what, a, b);
  return 1;
}

int main(int argc, char **argv) {
  std::mt19937_64 rng(argc > 1 ? std::atoi(argv[1]) : 1);
  auto rnd = [&](int n) { return n > 0 ? (int)(rng() % (uint64_t)n) : 0; };
  aln_ctx *ctx = nullptr;
  if (aln_create_host(&ctx, 0, 0) != ALN_OK || !ctx) return fail("create_host", 0, 0);
  aln_ctx *bad = nullptr;
  if (aln_create_host(&bad, -1, 0) != ALN_E_INVAL) return fail("negative cus accepted", 0, 0);
  int planned = 0, folded = 0;
  for (int round = 0; round < 300; ++round) {
    const int A = rnd(3) == 0 ? 20 : 4;
    std::vector<int32_t> mat(A * A);
    const bool mm = rnd(2);
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b)
        mat[a * A + b] = a == b ? 1 + rnd(4) : (mm ? -2 : -1 - rnd(3));
    aln_scoring sc{A, mat.data(), -rnd(8), -rnd(4)};
    int32_t sid = -1;
    if (aln_set_scoring(ctx, &sc, &sid) != ALN_OK) return fail("set_scoring", round, 0);
    const int n = rnd(5) == 0 ? 0 : 1 + rnd(300);
    std::vector<int32_t> ql(n), rl(n);
    for (int p = 0; p < n; ++p) {
      const int cls = rnd(6);
      ql[p] = cls == 0 ? 0 : cls == 1 ? 1 : cls == 2 ? rnd(5000) : rnd(900);
      rl[p] = cls == 0 ? rnd(3) : cls == 3 ? 1 : rnd(900);
    }
    aln_params p{};
    p.prune = rnd(5);
    // mostly valid combinations: X-drop / Z-drop extend, search global
    p.mode = (p.prune == ALN_XDROP || p.prune == ALN_ZDROP) && rnd(4) ? ALN_EXTEND
             : p.prune == ALN_SEARCH && rnd(4)                        ? ALN_GLOBAL
                                                                      : rnd(3);
    if (p.prune == ALN_SEARCH && rnd(4)) { // penalties
      for (int a = 0; a < A; ++a)
        for (int b = 0; b < A; ++b) mat[a * A + b] = a == b ? 0 : -1 - rnd(3) * (a > b ? 0 : 0);
      for (int a = 0; a < A; ++a)
        for (int b = 0; b < A; ++b) mat[a * A + b] = a == b ? 0 : mat[0 * A + 1];
      aln_scoring pen{A, mat.data(), -rnd(6), -1 - rnd(3)};
      if (aln_set_scoring(ctx, &pen, &sid) != ALN_OK) return fail("set_scoring 2", round, 0);
      p.want_cigar = 0;
    }
    p.band_w = rnd(6) == 0 ? -1 : rnd(400);
    p.xdrop = rnd(8) == 0 ? -1 : rnd(200);
    p.width = rnd(3);
    if (p.prune != ALN_SEARCH) p.want_cigar = rnd(2);
    aln_plan *plan = nullptr;
    aln_footprint fp{};
    const aln_status st = aln_plan_create(ctx, sid, &p, n, ql.data(), rl.data(), &plan, &fp);
    if (st != ALN_OK) {
      if (plan) return fail("plan on error", round, st);
      if (st != ALN_E_INVAL && st != ALN_E_UNSUPPORTED) return fail("status", round, st);
      continue;
    }
    int32_t nl = 0;
    const int64_t nt = aln_plan_describe(plan, nullptr, 0, &nl, nullptr, 0);
    if (nt < 0) return fail("describe", round, nt);
    std::vector<aln_launch_info> L(std::max(nl, 1));
    std::vector<aln_task_info> T(std::max<int64_t>(nt, 1));
    if (aln_plan_describe(plan, L.data(), nl, &nl, T.data(), nt) != nt) return fail("describe 2", round, nt);
    std::vector<int> seen(n, 0);
    for (int64_t k = 0; k < nt; ++k) {
      const aln_task_info &t = T[k];
      if (t.pair < 0 || t.pair >= n || t.launch < 0 || t.launch >= nl) return fail("task", round, k);
      seen[t.pair]++;
    }
    for (int q = 0; q < n; ++q)
      if (seen[q] != 1) return fail("pair not once", round, q);
    if (p.want_cigar && p.prune != ALN_SEARCH) {
      std::vector<std::pair<int64_t, int64_t>> tb, cg;
      for (int64_t k = 0; k < nt; ++k) {
        tb.push_back({T[k].tb_off, T[k].tb_off + T[k].tb_bytes});
        cg.push_back({T[k].cigar_off, T[k].cigar_off + T[k].cigar_cap});
      }
      std::sort(tb.begin(), tb.end());
      std::sort(cg.begin(), cg.end());
      for (size_t k = 0; k < tb.size(); ++k) {
        if (tb[k].first < 0 || tb[k].second > (int64_t)fp.traceback_bytes) return fail("tb range", round, k);
        if (k && tb[k - 1].second > tb[k].first) return fail("tb overlap", round, k);
        if (cg[k].first < 0 || cg[k].second > (int64_t)fp.cigar_words) return fail("cigar range", round, k);
        if (k && cg[k - 1].second > cg[k].first) return fail("cigar overlap", round, k);
      }
    }
    if (fp.workspace_bytes < fp.traceback_bytes) return fail("workspace", round, 0);
    aln_plan_destroy(plan);
    ++planned;
  }
  // folding plans
  aln_fold_params fpar{};
  fpar.pair[0 * 4 + 3] = fpar.pair[3 * 4 + 0] = 1;
  fpar.pair[1 * 4 + 2] = fpar.pair[2 * 4 + 1] = 1;
  fpar.min_loop = 3;
  fpar.xdrop = 2;
  fpar.warmup = 15;
  for (int round = 0; round < 40; ++round) {
    const int n = rnd(300);
    std::vector<int32_t> len(n);
    for (int k = 0; k < n; ++k) len[k] = round % 4 == 3 ? rnd(600) : rnd(500); // some too long
    aln_plan *plan = nullptr;
    aln_footprint fp{};
    const aln_status st = aln_fold_plan_create(ctx, &fpar, n, len.data(), &plan, &fp);
    if (st != ALN_OK) {
      if (st != ALN_E_UNSUPPORTED || plan) return fail("fold status", round, st);
      continue;
    }
    const int64_t nt = aln_plan_describe(plan, nullptr, 0, nullptr, nullptr, 0);
    if (nt != n) return fail("fold tasks", round, nt);
    aln_plan_destroy(plan);
    ++folded;
  }
  if (planned < 100 || folded < 20) return fail("too few plans", planned, folded);
  aln_destroy(ctx);
  std::printf("OK\n");
  return 0;
}
