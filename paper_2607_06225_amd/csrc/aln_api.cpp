// aln_api.cpp -- host runtime behind include/aln.h.
//
// Planning happens on the host from the pairs' lengths: each pair gets a
// kernel and a tile shape, pairs of one shape are ordered longest first
// (largest cell count first, so the tail of a launch is short work), and the
// workspace is laid out as [task lists | traceback codes].  Executing a plan
// uploads the task lists from pinned memory and enqueues the kernels on the
// caller's stream; nothing is allocated on that path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "runtime.h"

using alnk::DevScoring;
using alnk::PairTask;
using namespace alnrt;


namespace {


#define HIP_TRY(ctx, call)                                                       \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail((ctx), ALN_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Rows per lane for the strip kernel: fewest padded cells plus a per-step
// overhead of about eight cells per lane.
int choose_strip_rows(int32_t M, int32_t N) {
  static const int cand[] = {8, 16, 24, 32};
  int best = 16;
  double best_cost = 1e300;
  for (int R : cand) {
    const int64_t HS = 64LL * R;
    const int64_t ns = (M + HS - 1) / HS;
    const double cost = (double)ns * (double)(N + 63) * 64.0 * (double)(R + 8);
    if (cost < best_cost) {
      best_cost = cost;
      best = R;
    }
  }
  return best;
}

hipEvent_t pool_event(aln_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` (which enqueues one kernel on `st`); with profiling on, the
// launch is bracketed by events recorded on the same stream.
template <class F>
hipError_t timed_launch(aln_ctx *ctx, const char *name, hipStream_t st, F &&launch) {
  if (!ctx->profiling) return launch();
  hipEvent_t a = pool_event(ctx), b = pool_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  (void)hipEventRecord(a, st);
  hipError_t e = launch();
  (void)hipEventRecord(b, st);
  ctx->timed.push_back({name, a, b});
  return e;
}

} // namespace

aln_status alnrt::fail(aln_ctx *ctx, aln_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

extern "C" {

int32_t aln_abi_version(void) { return ALN_ABI_VERSION; }

aln_status aln_create(aln_ctx **ctx, int32_t device) {
  if (!ctx) return ALN_E_INVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return ALN_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return ALN_E_DEVICE;
  aln_ctx *c = new (std::nothrow) aln_ctx;
  if (!c) return ALN_E_NOMEM;
  c->device = device;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
    c->cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) ==
          hipSuccess && v > 0)
    c->lds_per_cu = v;
  if (alnrt::scratch_init(c) != ALN_OK) {
    delete c;
    return ALN_E_DEVICE;
  }
  *ctx = c;
  return ALN_OK;
}

aln_status aln_create_host(aln_ctx **ctx, int32_t cus, int32_t lds_per_cu) {
  if (!ctx || cus < 0 || lds_per_cu < 0) return ALN_E_INVAL;
  *ctx = nullptr;
  aln_ctx *c = new (std::nothrow) aln_ctx;
  if (!c) return ALN_E_NOMEM;
  c->device = -1;
  if (cus > 0) c->cus = cus;
  if (lds_per_cu > 0) c->lds_per_cu = lds_per_cu;
  *ctx = c;
  return ALN_OK;
}

void aln_destroy(aln_ctx *ctx) {
  if (!ctx) return;
  if (ctx->device < 0) {
    delete ctx;
    return;
  }
  (void)hipSetDevice(ctx->device);
  for (DevScoring *d : ctx->dsc) (void)hipFree(d);
  for (auto &t : ctx->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
}

aln_status aln_set_profiling(aln_ctx *ctx, int32_t enable) {
  if (!ctx) return ALN_E_INVAL;
  ctx->profiling = enable != 0;
  return ALN_OK;
}

int32_t aln_kernel_times(aln_ctx *ctx, const char **names, double *ms, int64_t *launches,
                         int32_t max) {
  if (!ctx || max < 0 || (max > 0 && (!names || !ms || !launches))) return ALN_E_INVAL;
  (void)hipSetDevice(ctx->device);
  int32_t nout = 0;
  for (auto &t : ctx->timed) {
    float el = 0.f;
    (void)hipEventSynchronize(t.b);
    (void)hipEventElapsedTime(&el, t.a, t.b);
    int32_t k = 0;
    while (k < nout && strcmp(names[k], t.name) != 0) ++k;
    if (k == nout) {
      if (nout == max) continue;
      names[nout] = t.name;
      ms[nout] = 0.0;
      launches[nout] = 0;
      ++nout;
    }
    ms[k] += el;
    launches[k] += 1;
    ctx->event_pool.push_back(t.a);
    ctx->event_pool.push_back(t.b);
  }
  ctx->timed.clear();
  return nout;
}

const char *aln_last_error(const aln_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

aln_status aln_set_scoring(aln_ctx *ctx, const aln_scoring *sc, int32_t *scoring_id) {
  if (!ctx || !sc || !scoring_id || !sc->matrix) return fail(ctx, ALN_E_INVAL, "null argument");
  const int A = sc->alphabet;
  if (A < 1 || A > alnk::kMaxAlphabet)
    return fail(ctx, ALN_E_INVAL, "alphabet %d outside 1..%d", A, alnk::kMaxAlphabet);
  if (sc->gap_open > 0 || sc->gap_extend > 0 || sc->gap_open < -1024 || sc->gap_extend < -1024)
    return fail(ctx, ALN_E_INVAL, "gap penalties must lie in [-1024, 0]");
  DevScoring h;
  memset(&h, 0, sizeof h);
  h.alphabet = A;
  h.gap_open = sc->gap_open;
  h.gap_extend = sc->gap_extend;
  h.max_s = -(1 << 30);
  h.min_s = 1 << 30;
  bool mm = true;
  for (int a = 0; a < A; ++a)
    for (int b = 0; b < A; ++b) {
      const int v = sc->matrix[a * A + b];
      if (v < -127 || v > 127)
        return fail(ctx, ALN_E_INVAL, "substitution score %d outside [-127, 127]", v);
      h.mat[a * alnk::kMaxAlphabet + b] = v;
      h.max_s = std::max(h.max_s, v);
      h.min_s = std::min(h.min_s, v);
      const int ref = (a == b) ? sc->matrix[0] : (A > 1 ? sc->matrix[1] : 0);
      if (v != ref) mm = false;
    }
  h.match_mismatch = mm ? 1 : 0;
  h.match = sc->matrix[0];
  h.mismatch = A > 1 ? sc->matrix[1] : 0;
  for (int a = 0; a < A; ++a) {
    uint32_t w = 0;
    for (int b = 0; b < 4; ++b) {
      const int v = (b < A) ? h.mat[a * alnk::kMaxAlphabet + b] : -128;
      w |= ((uint32_t)(v & 0xff)) << (8 * b);
    }
    h.rowtab[a] = w;
  }
  if (ctx->device < 0) { // no device: the host mirror only
    ctx->dsc.push_back(nullptr);
    ctx->hsc.push_back(h);
    *scoring_id = (int32_t)ctx->dsc.size() - 1;
    return ALN_OK;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  DevScoring *d = nullptr;
  HIP_TRY(ctx, hipMalloc(&d, sizeof(DevScoring)));
  hipError_t e = hipMemcpy(d, &h, sizeof h, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(ctx, ALN_E_DEVICE, "hipMemcpy scoring: %s", hipGetErrorString(e));
  }
  ctx->dsc.push_back(d);
  ctx->hsc.push_back(h);
  *scoring_id = (int32_t)ctx->dsc.size() - 1;
  return ALN_OK;
}

} // extern "C"

// Resident wavefronts per CU of the sixteen-sides X-drop kernel: the
// device's occupancy, or three per SIMD (its register count) without one.
static int lanes_waves_per_cu(const aln_ctx *ctx, bool tb) {
  return ctx->device < 0 ? 12 : alnk::xdrop_lanes_waves_per_cu(tb);
}

// Interior cells (1 <= i <= M, 1 <= j <= N) of the static band: row i keeps
// floor(iN/M) - w <= j <= floor(iN/M) + w.  Rows whose band is clipped by
// column 1 or column N are counted one by one (the centre floor(iN/M) is
// non-decreasing in i, so they form a prefix and a suffix of the rows); every
// other row holds 2w + 1 cells.
static int64_t band_cells(int64_t M, int64_t N, int64_t w) {
  if (M <= 0 || N <= 0) return 0;
  if (w >= std::max(M, N)) return M * N;
  auto centre = [&](int64_t i) { return i * N / M; };
  auto row = [&](int64_t i) {
    const int64_t lo = std::max<int64_t>(1, centre(i) - w), hi = std::min(N, centre(i) + w);
    return hi >= lo ? hi - lo + 1 : 0;
  };
  // last row clipped on the left (centre <= w), first clipped on the right
  int64_t a = 0, lo = 1, hi = M;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) / 2;
    if (centre(mid) <= w) { a = mid; lo = mid + 1; } else { hi = mid - 1; }
  }
  int64_t b = M + 1;
  lo = 1;
  hi = M;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) / 2;
    if (centre(mid) + w > N) { b = mid; hi = mid - 1; } else { lo = mid + 1; }
  }
  int64_t total = 0;
  if (b <= a + 1) {
    for (int64_t i = 1; i <= M; ++i) total += row(i);
    return total;
  }
  for (int64_t i = 1; i <= a; ++i) total += row(i);
  for (int64_t i = b; i <= M; ++i) total += row(i);
  return total + (b - a - 1) * (2 * w + 1);
}

aln_status alnrt::plan_build(aln_ctx *ctx, int32_t scoring_id, const aln_params *params, int32_t n,
                             const int32_t *q_len_host, const int32_t *r_len_host,
                             aln_plan **plan) {
  if (!ctx || !params || !plan || n < 0 || (n > 0 && (!q_len_host || !r_len_host)))
    return fail(ctx, ALN_E_INVAL, "null argument or negative n");
  *plan = nullptr;
  if (scoring_id < 0 || scoring_id >= (int32_t)ctx->dsc.size())
    return fail(ctx, ALN_E_INVAL, "unknown scoring id %d", scoring_id);
  const aln_params &p = *params;
  if (p.mode < ALN_GLOBAL || p.mode > ALN_EXTEND) return fail(ctx, ALN_E_INVAL, "bad mode");
  if (p.prune < ALN_FULL || p.prune > ALN_SEARCH) return fail(ctx, ALN_E_INVAL, "bad prune");
  if (p.prune == ALN_BAND && p.band_w < 0) return fail(ctx, ALN_E_INVAL, "band_w < 0");
  const bool dyn_prune = p.prune == ALN_XDROP || p.prune == ALN_ZDROP;
  if (dyn_prune && (p.xdrop < 0 || p.mode != ALN_EXTEND))
    return fail(ctx, ALN_E_INVAL, "XDROP / ZDROP need mode EXTEND and a threshold >= 0");
  if (p.width < ALN_W_AUTO || p.width > ALN_W_I32) return fail(ctx, ALN_E_INVAL, "bad width");
  const DevScoring &hs = ctx->hsc[scoring_id];
  const int64_t per_step = (int64_t)std::abs(hs.gap_open) + std::abs(hs.gap_extend) + 128;
  if (p.prune == ALN_SEARCH) {
    if (p.mode != ALN_GLOBAL || p.want_cigar)
      return fail(ctx, ALN_E_UNSUPPORTED, "SEARCH is GLOBAL, score only, without CIGAR");
    if (!hs.match_mismatch || hs.match != 0 || hs.mismatch >= 0 || hs.gap_open > 0 ||
        hs.gap_extend >= 0)
      return fail(ctx, ALN_E_UNSUPPORTED,
                  "SEARCH needs penalties: match 0, one mismatch score < 0, open <= 0, extend < 0");
  }

  aln_plan *pl = new (std::nothrow) aln_plan;
  if (!pl) return fail(ctx, ALN_E_NOMEM, "plan allocation");
  pl->ctx = ctx;
  pl->scoring_id = scoring_id;
  pl->p = p;
  pl->n = n;
  pl->qlen.assign(q_len_host, q_len_host + n);
  pl->rlen.assign(r_len_host, r_len_host + n);
  const bool small = hs.alphabet <= 4;

  int32_t maxM = 0, maxN = 0;
  for (int32_t i = 0; i < n; ++i) {
    maxM = std::max(maxM, pl->qlen[i]);
    maxN = std::max(maxN, pl->rlen[i]);
  }
  // score-major search: one workgroup per pair, longest first, both
  // sequences and the furthest-row arrays in LDS.  Unit edit costs: four
  // wavefronts share a pair when two rows fit in LDS, else one wavefront
  // updates a single row in place.  Gap-affine penalties: four wavefronts
  // over rings of past H, E and F rows.
  if (p.prune == ALN_SEARCH) {
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return (int64_t)pl->qlen[a] + pl->rlen[a] > (int64_t)pl->qlen[b] + pl->rlen[b];
    });
    LaunchDesc L{};
    L.kind = K_SEARCH;
    L.mode = ALN_GLOBAL;
    L.first = 0;
    L.count = n;
    L.lds_bnd = (int32_t)align_up((uint64_t)maxM + 20, 16);  // query codes + padding
    L.lds_prof = (int32_t)align_up((uint64_t)maxN + 20, 16); // reference codes + padding
    L.lds_f = (int32_t)align_up(((uint64_t)maxM + maxN + 1) * 2, 16); // int16 rows
    if (maxM > 32767 || (int64_t)L.lds_bnd + L.lds_prof + L.lds_f > 160 * 1024) {
      delete pl;
      return fail(ctx, ALN_E_UNSUPPORTED, "SEARCH needs M <= 32767 and the longest M plus the longest N of the batch <= about 54000");
    }
    L.waves = (int64_t)L.lds_bnd + L.lds_prof + 2 * (int64_t)L.lds_f <= 160 * 1024 ? 4 : 1;
    const bool unit = hs.mismatch == -1 && hs.gap_open == 0 && hs.gap_extend == -1;
    if (!unit) { // gap-affine: rings of past score rows, four wavefronts
      L.pen_x = -hs.mismatch;
      L.pen_o = -hs.gap_open;
      L.pen_e = -hs.gap_extend;
      L.ring_h = std::max(L.pen_x, L.pen_o + L.pen_e) + 1;
      L.ring_e = L.pen_e + 1;
      L.waves = 4;
      const int64_t lds = (int64_t)L.lds_bnd + L.lds_prof +
                          (int64_t)(L.ring_h + 2 * L.ring_e) * L.lds_f;
      if (lds > 160 * 1024) {
        delete pl;
        return fail(ctx, ALN_E_UNSUPPORTED,
                    "gap-affine SEARCH keeps %d score rows of %d bytes in LDS: %lld bytes > 160 KB",
                    L.ring_h + 2 * L.ring_e, L.lds_f, (long long)lds);
      }
      // First pass: rows of diagonals -dcap..dcap, dcap as large as lets four
      // workgroups share a CU; pairs whose range outgrows it run again with
      // full rows.  Skipped when capped rows would not be shorter.
      const int64_t nrows = L.ring_h + 2 * L.ring_e;
      const int64_t per_row = (40 * 1024 - (int64_t)L.lds_bnd - L.lds_prof) / nrows;
      const int64_t cap = (per_row / 2 - 1) / 2;
      if (cap >= 16 && 2 * cap + 1 < (int64_t)maxM + maxN + 1) {
        L.dcap = (int32_t)cap;
        L.lds_fc = (int32_t)align_up((uint64_t)(2 * cap + 1) * 2, 16);
        if ((int64_t)L.lds_bnd + L.lds_prof + nrows * L.lds_fc > 40 * 1024) { // rounding
          L.dcap -= 8;
          L.lds_fc = (int32_t)align_up((uint64_t)(2 * L.dcap + 1) * 2, 16);
        }
      }
    }
    for (int32_t i : order) {
      PairTask t;
      memset(&t, 0, sizeof t);
      t.pair = i;
      t.tb_off = -1;
      pl->tasks.push_back(t);
    }
    pl->launches.push_back(L);
    pl->tasks_bytes = align_up(sizeof(PairTask) * std::max<size_t>(pl->tasks.size(), 1));
    pl->upload_bytes = sizeof(PairTask) * pl->tasks.size();
    pl->tb_base = pl->tasks_bytes;
    pl->tb_bytes = 0;
    pl->ws_bytes = pl->tasks_bytes;
    pl->cigar_words = 0;
    *plan = pl;
    return ALN_OK;
  }

  // packed int16 Smith-Waterman: LOCAL, full matrix, score + end cell
  const int rerun_rows = 16;
  const int32_t rerun_bnd = (int32_t)align_up((uint64_t)(maxN + 1) * 8, 16);
  const int32_t rerun_prof = small ? 0 : (int32_t)align_up((uint64_t)hs.alphabet * 64 * rerun_rows, 16);
  const bool use_sw16 = p.mode == ALN_LOCAL && p.prune == ALN_FULL && !p.want_cigar &&
                        p.width != ALN_W_I32 && n > 0 && hs.alphabet < alnk::kMaxAlphabet &&
                        maxN <= 65535 - 63 && maxM < (1 << 20) &&
                        4LL * (rerun_bnd + rerun_prof) <= 160 * 1024;
  if (use_sw16) {
    // rows per lane: forced while the autotuner measures, else the
    // ALN_SW16_ROWS override, else the autotuner's choice, else 16
    int tile = 16;
    if (ctx->tuning.valid) tile = ctx->tuning.sw16_rows;
    if (const char *ev = getenv("ALN_SW16_ROWS")) {
      const int r = atoi(ev);
      if (r == 4 || r == 8 || r == 12 || r == 16) tile = r;
    }
    if (ctx->force_sw16_rows) tile = ctx->force_sw16_rows;
    const int R = tile;
    pl->sw16_rows = R;
    const int32_t HS = 16 * R, HW = 64 * R; // strip heights: 16-lane group, wide item
    auto nstr = [](int32_t m, int32_t hs) { return (m + hs - 1) / hs; };
    // pairs sorted by strips, then columns, longest first; consecutive
    // pairs share a task (the two 16-bit halves), so the halves match
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      const int sa = nstr(pl->qlen[a], HS), sb = nstr(pl->qlen[b], HS);
      if (sa != sb) return sa > sb;
      return pl->rlen[a] > pl->rlen[b];
    });
    struct TaskDim {
      int32_t pa, pb, mmax, nmax;
    };
    std::vector<TaskDim> td;
    for (int32_t q = 0; q < n; q += 2) {
      TaskDim t{order[q], q + 1 < n ? order[q + 1] : -1, pl->qlen[order[q]], pl->rlen[order[q]]};
      if (t.pb >= 0) {
        t.mmax = std::max(t.mmax, pl->qlen[t.pb]);
        t.nmax = std::max(t.nmax, pl->rlen[t.pb]);
      }
      td.push_back(t);
    }
    const int32_t nt = (int32_t)td.size();
    // Serial column steps of one wavefront: a group of four tasks on 16-lane
    // groups runs the largest strip count times the widest reference (plus
    // the lane skew); a wide item runs one task in 64*R-row strips.
    auto steps_narrow = [&](const std::vector<int32_t> &grp) {
      int32_t ns = 0, nm = 0;
      for (int32_t k : grp) {
        ns = std::max(ns, nstr(td[k].mmax, HS));
        nm = std::max(nm, td[k].nmax);
      }
      return (int64_t)ns * (nm + 15);
    };
    auto steps_wide = [&](int32_t k) { return (int64_t)nstr(td[k].mmax, HW) * (td[k].nmax + 63); };
    // Load model: one wavefront per item; LDS bounds the wavefronts per CU.
    // A lone wavefront keeps its SIMD about 4/5 busy, so a second one on the
    // same SIMD adds about a quarter of a wavefront's rate.
    const size_t lds16 = alnk::sw16_lds_bytes(R, hs.alphabet);
    const int wpc = (int)std::max<size_t>(1, std::min<size_t>(16, (size_t)ctx->lds_per_cu / lds16));
    const double capacity =
        (double)ctx->cus * (std::min(wpc, 4) + 0.25 * std::min(std::max(wpc - 4, 0), 4));
    int64_t total = 0;
    for (int32_t k = 0; k < nt; k += 4) {
      std::vector<int32_t> grp;
      for (int32_t q = k; q < std::min(nt, k + 4); ++q) grp.push_back(q);
      total += steps_narrow(grp);
    }
    // A task whose own strips take longer than most of a wave slot's share
    // of the launch would finish last: it runs wide.
    int wide_pct = ctx->tuning.valid && ctx->tuning.sw16_wide_pct ? ctx->tuning.sw16_wide_pct : 80;
    if (ctx->force_sw16_wide_pct) wide_pct = ctx->force_sw16_wide_pct;
    const double wide_above =
        wide_pct < 0 ? 1e300 : wide_pct / 100.0 * (double)total / capacity;
    struct Item {
      int64_t steps;
      std::vector<int32_t> tasks;
      bool wide;
    };
    std::vector<Item> items;
    std::vector<int32_t> grp;
    auto close_group = [&] {
      if (grp.empty()) return;
      items.push_back(Item{steps_narrow(grp), grp, false});
      grp.clear();
    };
    for (int32_t k = 0; k < nt; ++k) {
      if ((double)nstr(td[k].mmax, HS) * (td[k].nmax + 15) > wide_above) {
        items.push_back(Item{steps_wide(k), {k}, true});
        continue;
      }
      grp.push_back(k);
      if (grp.size() == 4) close_group();
    }
    close_group();
    // longest item first: workgroups are dispatched in index order
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &b) { return a.steps > b.steps; });
    pl->sw16_wide = 0;
    uint64_t bnd_bytes = 0;
    std::vector<uint64_t> bnd_rel;
    LaunchDesc L{};
    L.kind = K_SW16;
    L.rows = R;
    L.mode = ALN_LOCAL;
    L.first = 0;
    for (const Item &it : items) {
      pl->sw16_items.push_back(
          alnk::Sw16Item{(int32_t)pl->sw16_tasks.size(), it.wide ? -1 : (int32_t)it.tasks.size()});
      pl->sw16_wide += it.wide;
      for (int32_t k : it.tasks) {
        const TaskDim &d = td[k];
        alnk::Sw16Task t;
        t.pa = d.pa;
        t.pb = d.pb;
        t.nstrips = nstr(d.mmax, it.wide ? HW : HS);
        t.nmax = d.nmax;
        t.bnd_off = 0;
        bnd_rel.push_back(t.nstrips > 1 ? bnd_bytes : ~0ULL);
        if (t.nstrips > 1) bnd_bytes += align_up((uint64_t)(t.nmax + 1) * 8);
        pl->sw16_tasks.push_back(t);
        // the same pairs one by one (per-pair runs, always wide), sharing the
        // task's boundary row: a pair alone never has more strips, nor more
        // columns, than its task
        for (int h = 0; h < 2; ++h) {
          const int32_t pp = h ? t.pb : t.pa;
          if (pp < 0) continue;
          alnk::Sw16Task u;
          u.pa = pp;
          u.pb = -1;
          u.nstrips = nstr(pl->qlen[pp], HW);
          u.nmax = pl->rlen[pp];
          u.bnd_off = (int64_t)(pl->sw16_tasks.size() - 1); // task index, resolved below
          pl->sw16_single.push_back(u);
          pl->sw16_single_rows.push_back(R);
        }
      }
    }
    L.count = (int32_t)pl->sw16_tasks.size();
    pl->launches.push_back(L);
    // workspace: [sw16 tasks | items | single tasks | rerun counter | rerun queue |
    //             boundary rows]
    pl->sw16_off = 0;
    pl->sw16_items_off = align_up(sizeof(alnk::Sw16Task) * pl->sw16_tasks.size());
    pl->sw16_single_off =
        pl->sw16_items_off + align_up(sizeof(alnk::Sw16Item) * pl->sw16_items.size());
    pl->rerun_cnt_off = pl->sw16_single_off + align_up(sizeof(alnk::Sw16Task) * pl->sw16_single.size());
    pl->rerun_off = pl->rerun_cnt_off + kAlign;
    const uint64_t bnd_base = pl->rerun_off + align_up(sizeof(PairTask) * (size_t)n);
    for (size_t k = 0; k < pl->sw16_tasks.size(); ++k)
      pl->sw16_tasks[k].bnd_off = bnd_rel[k] == ~0ULL ? 0 : (int64_t)(bnd_base + bnd_rel[k]);
    for (alnk::Sw16Task &u : pl->sw16_single) u.bnd_off = pl->sw16_tasks[(size_t)u.bnd_off].bnd_off;
    pl->rerun.kind = K_RERUN;
    pl->rerun.rows = rerun_rows;
    pl->rerun.mode = ALN_LOCAL;
    pl->rerun.tb = false;
    pl->rerun.small = small;
    pl->rerun.first = 0;
    pl->rerun.count = n;
    pl->rerun.lds_bnd = rerun_bnd;
    pl->rerun.lds_prof = rerun_prof;
    for (int32_t i = 0; i < n; ++i) pl->cells += (int64_t)pl->qlen[i] * pl->rlen[i];
    pl->upload_bytes = pl->rerun_cnt_off;
    pl->tasks_bytes = bnd_base + bnd_bytes;
    pl->tb_base = pl->tasks_bytes;
    pl->tb_bytes = 0;
    pl->ws_bytes = pl->tasks_bytes;
    pl->cigar_words = 0;
    *plan = pl;
    return ALN_OK;
  }

  // ---- per-pair kernel choice: full-matrix strips, or the antidiagonal
  // kernel (band, X-drop) with a window of 64*RD diagonals
  struct Item {
    int32_t pair;
    int kind;
    int rows;
    double cost;
    int waves = 1; // full matrix / band strips: wavefronts per pair (strip pipeline)
    int ring = 0;  // band strips: columns of the LDS boundary ring
  };
  std::vector<Item> items;
  items.reserve(n);
  static const int kDiagRows[] = {2, 4, 8, 10, 16, 32};
  int srows = ctx->tuning.valid ? ctx->tuning.strip_rows : 0;
  if (ctx->force_strip_rows >= 0) srows = ctx->force_strip_rows;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t M = pl->qlen[i], N = pl->rlen[i];
    if (M < 0 || N < 0) {
      delete pl;
      return fail(ctx, ALN_E_INVAL, "negative length at pair %d", i);
    }
    if ((int64_t)(M + (int64_t)N) * per_step >= (1LL << 29)) {
      delete pl;
      return fail(ctx, ALN_E_UNSUPPORTED, "pair %d too long for int32 scores", i);
    }
    Item it{i, K_STRIP, 0, 0.0};
    const bool band_is_full = p.prune == ALN_BAND && (M == 0 || p.band_w >= std::max(M, N));
    if (p.prune == ALN_FULL || band_is_full) {
      it.rows = srows ? srows : choose_strip_rows(M, N);
      it.cost = (double)M * N;
      pl->cells += (int64_t)M * N;
    } else {
      it.kind = K_DIAG;
      if (p.mode != ALN_GLOBAL && (int64_t)std::max(hs.max_s, 1) * std::min(M, N) >= (1 << 20)) {
        delete pl;
        return fail(ctx, ALN_E_UNSUPPORTED, "pair %d: best score may exceed 2^20", i);
      }
      if (p.prune == ALN_BAND) {
        const int64_t w = p.band_w;
        // strips (band_kernel 2..5: one or four wavefronts per pair, 4 or 2
        // rows per lane): a strip's columns and 10 spare ones fit one LDS ring
        // of at most 2048, and the pipeline's stamps s*(N+1) + column fit 31
        // bits
        int bk = ctx->force_band_kernel
                     ? ctx->force_band_kernel
                     : (ctx->tuning.valid ? ctx->tuning.band_kernel : 0);
        if (bk == 0) bk = 2 * w + 1 >= 256 ? 5 : 1; // wide bands: strips, four wavefronts of 2 rows
        const int brows = (bk == 4 || bk == 5) ? 2 : 4;
        const int64_t cols = M > 0 && N > 0 ? alnk::band_strip_cols(M, N, (int32_t)std::min<int64_t>(w, 1 << 28), brows) : 0;
        const int64_t ring = std::max<int64_t>(64, (cols + 10 + 15) / 16 * 16);
        const int64_t nsb = (M + 64LL * brows - 1) / (64LL * brows);
        const bool strip_fit = M > 0 && N > 0 && ring <= 2048 && w < (1 << 28) &&
                               nsb * ((int64_t)N + 1) + N < (1LL << 31);
        if (bk >= 2 && strip_fit) {
          it.kind = K_BAND;
          it.rows = brows;
          it.waves = (bk == 3 || bk == 5) ? alnk::kStripPipeWaves : 1;
          it.ring = (int)ring;
          it.cost = (double)nsb * (double)(cols + 63) * brows;
        } else {
          int64_t width = 2 * w + 6 + ((2 * w + 2) * std::abs((int64_t)N - M) + M - 1) / std::max(M, 1);
          width = std::min<int64_t>(width, 2LL * std::min(M, N) + 6);
          it.rows = 0;
          for (int r : kDiagRows)
            if (64LL * r - 6 >= width && (!p.want_cigar || r <= 16)) { it.rows = r; break; }
          if (it.rows == 0) {
            delete pl;
            return fail(ctx, ALN_E_UNSUPPORTED, "pair %d: band of %lld diagonals exceeds the window",
                        i, (long long)width);
          }
          it.cost = (double)(M + N) * it.rows;
        }
        pl->cells += band_cells(M, N, p.band_w);
      } else {
        it.rows = ctx->tuning.valid ? ctx->tuning.xdrop_rows : 4;
        if (ctx->force_xdrop_rows) it.rows = ctx->force_xdrop_rows;
        it.cost = (double)(M + N);
      }
    }
    items.push_back(it);
  }
  // Strip pipeline: when the full-matrix pairs are too few to give every
  // SIMD a wavefront of its own, a pair of several strips runs on the
  // wavefronts of one workgroup, its strips handed down through LDS -- unless
  // a fixed strip height is tuned or forced.  By default, with at most three
  // quarters of a wavefront per SIMD, four wavefronts of 4 rows per lane
  // (256-row strips).  Tuned tiles ask for it (4) or for eight wavefronts of
  // 2 rows (2; 128-row strips, two wavefronts per SIMD of the CU: measured
  // 3% slower on 1 kbp pairs, where each strip's start behind the one above
  // sets the pace).  Boundary buffers hold whole rows, which bounds N.
  //
  // In the automatic choice the pipelined pairs run on the band strips with a
  // band past the matrix (the same four-wavefront schedule, 256-row strips):
  // that kernel's rotating lane-0 feeds and eight-step code stores take
  // about 18% less time on 1 kbp pairs.  Its LDS ring holds a strip's
  // columns and 10 more, so N <= 2038.
  pl->strip_band_w = p.prune == ALN_BAND ? p.band_w : (1 << 28);
  if (srows == 0 || srows == 2 || srows == 4) {
    int64_t n_full = 0;
    for (const Item &it : items) n_full += it.kind == K_STRIP;
    const int64_t simds = 4LL * ctx->cus;
    int R = 0, G = 0;
    if (srows == 2) {
      R = 2;
      G = alnk::kStripPipeWaves2;
    } else if (srows == 4 || n_full * 4 <= simds * 3) {
      R = 4;
      G = alnk::kStripPipeWaves;
    }
    for (Item &it : items) {
      if (it.kind != K_STRIP || G == 0) continue;
      const int32_t M = pl->qlen[it.pair], N = pl->rlen[it.pair];
      const uint64_t bnd = align_up((uint64_t)(N + 1) * 8, 16);
      const uint64_t prof = small ? 0 : align_up((uint64_t)hs.alphabet * 64 * R, 16);
      if ((srows == 0 || srows == 2) && M > 64 * R && N <= 2038 &&
          pl->strip_band_w >= std::max(M, N)) {
        const int64_t ring = std::max<int64_t>(64, ((int64_t)N + 10 + 15) / 16 * 16);
        it.kind = K_BAND;
        it.rows = R;
        it.waves = G;
        it.ring = (int)ring;
        it.cost = (double)((M + 64LL * R - 1) / (64LL * R)) * (double)(N + 63) * R;
      } else if (M > 64 * R && alnk::strip_lds_bytes(G, (int)bnd, (int)prof, N) <= 160 * 1024) {
        it.rows = R;
        it.waves = G;
      } else if (srows != 0) {
        it.rows = choose_strip_rows(M, N); // a one-strip pair, or one too wide for the LDS
      }
    }
  }
  // X-drop without traceback under match / mismatch scoring on a small
  // alphabet runs on the sixteen-sides-per-wavefront kernel when its
  // arithmetic fits: offset-frame scores in one byte, the out-of-range
  // penalty (-128) below every threshold (X < 128 + 2|e|), end cells in 16
  // bits and keys (score << 6) in 31.  Z-drop too, scores only, when tuned
  // (its form masks removed and out-of-range cells itself, so Z has no
  // bound).
  const bool zd = p.prune == ALN_ZDROP;
  const bool lanes_fit =
      (p.prune == ALN_XDROP || zd) && hs.match_mismatch && hs.alphabet <= 4 &&
      (zd || (int64_t)p.xdrop <= 127 - 2LL * hs.gap_extend) && hs.match - 2 * hs.gap_extend <= 127 &&
      hs.mismatch - 2 * hs.gap_extend >= -128 && maxM <= 65535 && maxN <= 65535 &&
      ((int64_t)maxM + maxN) * (1 - hs.gap_extend + std::max(hs.match, 0)) < (1LL << 23);
  const bool lanes_ok = lanes_fit && !p.want_cigar;
  std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
    if (a.kind != b.kind) return a.kind < b.kind;
    if (a.waves != b.waves) return a.waves < b.waves;
    if (a.rows != b.rows) return a.rows < b.rows;
    return a.cost > b.cost;
  });
  uint64_t tb_off = 0, cg_off = 0;
  for (size_t k = 0; k < items.size();) {
    size_t e = k;
    int32_t grpN = 0, grpRing = 0;
    bool multi = false;
    while (e < items.size() && items[e].kind == items[k].kind && items[e].rows == items[k].rows &&
           items[e].waves == items[k].waves) {
      grpN = std::max(grpN, pl->rlen[items[e].pair]);
      grpRing = std::max(grpRing, items[e].ring);
      if (items[e].kind == K_STRIP && pl->qlen[items[e].pair] > 64 * items[e].rows) multi = true;
      ++e;
    }
    LaunchDesc L{};
    L.kind = items[k].kind;
    L.rows = items[k].rows;
    L.mode = p.mode;
    if (L.kind == K_DIAG && dyn_prune) {
      // Z-drop takes the sixteen-sides form only when tuned: its regions
      // often outgrow the 64-cell window (at Z = 100, e = -2 nearly every
      // side, 345 ms against 300 on the one-side kernel)
      L.sides = ctx->tuning.valid ? ctx->tuning.xdrop_sides : ((lanes_ok && !zd) ? 16 : 1);
      if (ctx->force_xdrop_sides) L.sides = ctx->force_xdrop_sides;
      if (L.sides == 16 && !lanes_ok) L.sides = 1;
      if (L.sides == 4 && L.rows != 8) L.sides = 1;
      if (L.sides == 16) {
        const int64_t want = ((int64_t)(e - k) + 15) / 16;
        const int64_t fit = (int64_t)ctx->cus * lanes_waves_per_cu(ctx, false);
        L.grid = (int)std::max<int64_t>(1, std::min(want, fit));
      }
    }
    L.tb = p.want_cigar != 0 && !dyn_prune; // X-drop codes come from a second pass
    L.small = small;
    L.first = (int32_t)pl->tasks.size();
    L.count = (int32_t)(e - k);
    L.waves = items[k].waves;
    if (L.kind == K_BAND) {
      L.lds_bnd = grpRing * 8;
      L.lds_prof = small ? 0 : (int32_t)align_up((uint64_t)hs.alphabet * 64 * L.rows, 16);
      L.max_n = grpN;
    }
    if (L.kind == K_STRIP) {
      L.lds_bnd = multi ? (int32_t)align_up((uint64_t)(grpN + 1) * 8, 16) : 0;
      L.lds_prof = small ? 0 : (int32_t)align_up((uint64_t)hs.alphabet * 64 * L.rows, 16);
      L.max_n = grpN;
      if (alnk::strip_lds_bytes(L.waves, L.lds_bnd, L.lds_prof, L.max_n) > 160 * 1024) {
        delete pl;
        return fail(ctx, ALN_E_UNSUPPORTED,
                    "full-matrix pairs with N = %d and M > %d need more LDS than a CU has", grpN,
                    64 * L.rows);
      }
    }
    for (size_t q = k; q < e; ++q) {
      const int32_t i = items[q].pair;
      const int32_t M = pl->qlen[i], N = pl->rlen[i];
      PairTask t;
      memset(&t, 0, sizeof t);
      t.pair = i;
      t.rows = L.rows;
      t.tb_off = -1;
      if (p.want_cigar && !dyn_prune) {
        uint64_t bytes;
        if (L.kind == K_STRIP) {
          const int64_t ns = (M + 64LL * L.rows - 1) / (64LL * L.rows);
          bytes = (uint64_t)ns * (uint64_t)(N + 63) * 64ULL * (uint64_t)(L.rows / 2);
        } else if (L.kind == K_BAND) {
          const int64_t ns = (M + 64LL * L.rows - 1) / (64LL * L.rows);
          bytes = (uint64_t)ns * 64ULL *
                  (uint64_t)alnk::band_code_steps(M, N, pl->strip_band_w, L.rows) *
                  (uint64_t)(L.rows / 2);
        } else {
          const uint64_t nk = (uint64_t)M + N + 1;
          bytes = (nk + 63) / 64 * 64 * 4 + ((uint64_t)(M + N) / 2 + 1) * 64 * 8;
        }
        t.tb_off = (int64_t)tb_off;
        tb_off += align_up(bytes);
        t.cigar_off = (int64_t)cg_off;
        t.cigar_cap = M + N + 1;
        cg_off += (uint64_t)(M + N + 1);
      }
      pl->tasks.push_back(t);
    }
    pl->launches.push_back(L);
    k = e;
  }
  // X-drop / Z-drop with CIGAR: a second task list, one task per pair with
  // 4 diagonals per lane, for the traceback pass and the walk.  Codes take 2
  // bytes per lane and antidiagonal pair, plus the window base per
  // antidiagonal; the pass stops at the end cell's antidiagonal.
  if (dyn_prune && p.want_cigar) {
    pl->xtb_first = (int32_t)pl->tasks.size();
    pl->xtb_count = n;
    // the sixteen-sides kernel writes the codes where its arithmetic fits,
    // unless a tuned tile other than its own asks for the one-side pass
    const int tuned_sides = ctx->force_xdrop_sides
                                ? ctx->force_xdrop_sides
                                : (ctx->tuning.valid ? ctx->tuning.xdrop_sides : 16);
    pl->xtb_lanes = lanes_fit && !zd && tuned_sides == 16;
    if (pl->xtb_lanes) {
      const int64_t want = ((int64_t)n + 15) / 16;
      const int64_t fit = (int64_t)ctx->cus * lanes_waves_per_cu(ctx, true);
      pl->xtb_grid = (int)std::max<int64_t>(1, std::min(want, fit));
    }
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return (int64_t)pl->qlen[a] + pl->rlen[a] > (int64_t)pl->qlen[b] + pl->rlen[b];
    });
    for (int32_t i : order) {
      const int32_t M = pl->qlen[i], N = pl->rlen[i];
      PairTask t;
      memset(&t, 0, sizeof t);
      t.pair = i;
      t.rows = 4;
      const uint64_t nk = (uint64_t)M + N + 1;
      const uint64_t bytes = (nk + 63) / 64 * 64 * 4 + ((uint64_t)(M + N) / 2 + 1) * 64 * 2;
      t.tb_off = (int64_t)tb_off;
      tb_off += align_up(bytes);
      t.cigar_off = (int64_t)cg_off;
      t.cigar_cap = M + N + 1;
      cg_off += (uint64_t)(M + N + 1);
      pl->tasks.push_back(t);
    }
    pl->first_diag_tb = pl->xtb_first;
    pl->n_diag_tb = n;
  }
  // walk ranges: strip tasks come first (kind order), then antidiagonal tasks
  if (p.want_cigar && !dyn_prune) {
    for (const LaunchDesc &L : pl->launches) {
      if (L.kind == K_STRIP) pl->n_strip_tb += L.count;
      if (L.kind == K_DIAG) {
        if (pl->n_diag_tb == 0) pl->first_diag_tb = L.first;
        pl->n_diag_tb += L.count;
      }
      if (L.kind == K_BAND) {
        if (pl->n_band_tb == 0) pl->first_band_tb = L.first;
        pl->n_band_tb += L.count;
      }
    }
  }
  pl->xdrop = dyn_prune; // X-drop or Z-drop: widening queues
  pl->tasks_bytes = align_up(sizeof(PairTask) * std::max<size_t>(pl->tasks.size(), 1));
  pl->upload_bytes = sizeof(PairTask) * pl->tasks.size();
  if (pl->xdrop) {
    pl->widen_cnt_off = pl->tasks_bytes;
    pl->widen_off[0] = pl->widen_cnt_off + kAlign;
    pl->widen_off[1] = pl->widen_off[0] + align_up(sizeof(PairTask) * (size_t)std::max(n, 1));
    pl->widen_off[2] = pl->widen_off[1] + align_up(sizeof(PairTask) * (size_t)std::max(n, 1));
    pl->tasks_bytes = pl->widen_off[2] + (pl->xtb_lanes ? align_up(sizeof(PairTask) * (size_t)std::max(n, 1)) : 0);
  }
  pl->tb_base = pl->tasks_bytes;
  pl->tb_bytes = tb_off;
  pl->ws_bytes = pl->tb_base + pl->tb_bytes;
  pl->cigar_words = cg_off;
  *plan = pl;
  return ALN_OK;
}

void alnrt::plan_stage(const aln_plan *pl, void *dst) {
  uint8_t *d = static_cast<uint8_t *>(dst);
  if (pl->fold) {
    memcpy(d, pl->fold_tasks.data(), sizeof(alnk::FoldTask) * pl->fold_tasks.size());
    return;
  }
  if (!pl->sw16_tasks.empty()) {
    memcpy(d + pl->sw16_off, pl->sw16_tasks.data(), sizeof(alnk::Sw16Task) * pl->sw16_tasks.size());
    memcpy(d + pl->sw16_items_off, pl->sw16_items.data(),
           sizeof(alnk::Sw16Item) * pl->sw16_items.size());
    memcpy(d + pl->sw16_single_off, pl->sw16_single.data(),
           sizeof(alnk::Sw16Task) * pl->sw16_single.size());
  } else if (!pl->tasks.empty()) {
    memcpy(d, pl->tasks.data(), sizeof(PairTask) * pl->tasks.size());
  }
}

extern "C" {

aln_status aln_plan_create(aln_ctx *ctx, int32_t scoring_id, const aln_params *params, int32_t n,
                           const int32_t *q_len_host, const int32_t *r_len_host, aln_plan **plan,
                           aln_footprint *fp) {
  aln_plan *pl = nullptr;
  aln_status st = plan_build(ctx, scoring_id, params, n, q_len_host, r_len_host, &pl);
  if (st != ALN_OK) return st;
  if (alnrt::plan_alloc_staging(pl) != ALN_OK) {
    delete pl;
    return fail(ctx, ALN_E_NOMEM, "staging for %llu bytes", (unsigned long long)pl->upload_bytes);
  }
  plan_stage(pl, pl->pinned);
  if (fp) {
    fp->workspace_bytes = pl->ws_bytes;
    fp->traceback_bytes = pl->tb_bytes;
    fp->cigar_words = pl->cigar_words;
    fp->cells = pl->cells;
  }
  *plan = pl;
  return ALN_OK;
}

void aln_plan_destroy(aln_plan *plan) {
  if (!plan) return;
  if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->pinned && plan->own_pinned) {
    if (plan->host_staging) std::free(plan->pinned);
    else (void)hipHostFree(plan->pinned);
  }
  delete plan;
}

} // extern "C"

aln_status alnrt::exec_check(aln_ctx *ctx, aln_plan *plan, const aln_batch *b, void *d_ws,
                             uint64_t ws_bytes, aln_result *d_res, uint32_t *d_cigar,
                             uint64_t cigar_words) {
  if (!ctx || !plan || !b || plan->ctx != ctx) return fail(ctx, ALN_E_INVAL, "bad context or plan");
  if (plan->fold) return fail(ctx, ALN_E_INVAL, "a folding plan runs with aln_fold_execute");
  if (b->n != plan->n) return fail(ctx, ALN_E_INVAL, "batch has %d pairs, plan %d", b->n, plan->n);
  if (plan->n == 0) return ALN_OK;
  if (!d_res || !b->q_off || !b->q_len || !b->r_off || !b->r_len)
    return fail(ctx, ALN_E_INVAL, "null device pointer");
  if (!d_ws || ws_bytes < plan->ws_bytes)
    return fail(ctx, ALN_E_CAPACITY, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes,
                (unsigned long long)plan->ws_bytes);
  if (plan->p.want_cigar && (!d_cigar || cigar_words < plan->cigar_words))
    return fail(ctx, ALN_E_CAPACITY, "CIGAR buffer %llu < %llu words",
                (unsigned long long)cigar_words, (unsigned long long)plan->cigar_words);
  if (ctx->device < 0) return fail(ctx, ALN_E_DEVICE, "the context has no device");
  return ALN_OK;
}

aln_status alnrt::plan_alloc_staging(aln_plan *pl) {
  const size_t bytes = (size_t)std::max<uint64_t>(pl->upload_bytes, 1);
  if (pl->ctx->device < 0) {
    pl->pinned = std::malloc(bytes);
    pl->host_staging = true;
    return pl->pinned ? ALN_OK : ALN_E_NOMEM;
  }
  return hipHostMalloc(&pl->pinned, bytes, hipHostMallocDefault) == hipSuccess ? ALN_OK
                                                                               : ALN_E_NOMEM;
}

extern "C" {

static aln_status run_plan(aln_ctx *ctx, aln_plan *plan, const aln_batch *b, void *d_ws,
                           aln_result *d_res, uint32_t *d_cigar, hipStream_t st, bool per_pair) {
  if (plan->n == 0) return ALN_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  PairTask *dtasks = reinterpret_cast<PairTask *>(ws);
  if (plan->upload_bytes)
    HIP_TRY(ctx, hipMemcpyAsync(ws, plan->pinned, plan->upload_bytes, hipMemcpyHostToDevice, st));
  alnk::BatchPtrs bp{b->q, b->q_off, b->q_len, b->r, b->r_off, b->r_len};
  const DevScoring *dsc = ctx->dsc[plan->scoring_id];
  const DevScoring &hsc = ctx->hsc[plan->scoring_id];
  const bool sw16 = !plan->sw16_tasks.empty();
  int32_t *rerun_cnt = sw16 ? reinterpret_cast<int32_t *>(ws + plan->rerun_cnt_off) : nullptr;
  PairTask *rerun_q = sw16 ? reinterpret_cast<PairTask *>(ws + plan->rerun_off) : nullptr;

  int32_t *widen_cnt = plan->xdrop ? reinterpret_cast<int32_t *>(ws + plan->widen_cnt_off) : nullptr;
  // counters: sw16 re-run queue; X-drop widening queues (2), the lanes
  // kernel's work queue (2) and its queue of pairs for the one-side pass with
  // codes (1)
  alnk::ValidateArgs va{bp, plan->n, hsc.alphabet, d_res, sw16 ? rerun_cnt : widen_cnt,
                        sw16 ? 1 : (plan->xdrop ? 5 : 0)};
  HIP_TRY(ctx, timed_launch(ctx, "validate", st, [&] { return alnk::launch_validate(va, st); }));

  if (!plan->launches.empty() && plan->launches[0].kind == K_SEARCH) {
    const LaunchDesc &L = plan->launches[0];
    alnk::SearchArgs sa{bp,      dtasks,  L.count, d_res,    L.lds_bnd, L.lds_prof, L.lds_f,
                        L.waves, L.pen_x, L.pen_o, L.pen_e, L.ring_h,  L.ring_e,  0, 0};
    // gap-affine with a diagonal cap: a capped pass, then full rows for the
    // pairs it flagged
    std::pair<const char *, alnk::SearchArgs> passes[2];
    int npass = 0;
    if (L.pen_x > 0 && L.dcap > 0) {
      alnk::SearchArgs c = sa;
      c.lds_f = L.lds_fc;
      c.dcap = L.dcap;
      passes[npass++] = {"search_affine", c};
      sa.pass = 1;
      passes[npass++] = {"search_affine_wide", sa};
    } else {
      passes[npass++] = {L.pen_x > 0 ? "search_affine" : "search", sa};
    }
    for (int ip = 0; ip < npass; ++ip) {
      alnk::SearchArgs &x = passes[ip].second;
      if (!per_pair) {
        HIP_TRY(ctx, timed_launch(ctx, passes[ip].first, st, [&] { return alnk::launch_search(x, st); }));
      } else {
        for (int32_t k = 0; k < L.count; ++k) {
          x.tasks = dtasks + k;
          x.ntasks = 1;
          HIP_TRY(ctx, alnk::launch_search(x, st));
        }
      }
    }
    return ALN_OK;
  }

  if (sw16) {
    alnk::Sw16Args a16;
    a16.b = bp;
    a16.sc = dsc;
    a16.sc_alphabet = hsc.alphabet;
    a16.ws = ws;
    a16.res = d_res;
    a16.rerun_count = rerun_cnt;
    a16.rerun = rerun_q;
    a16.rerun_threshold = 32767 - std::max(hsc.max_s, 0);
    if (!per_pair) {
      for (const LaunchDesc &L : plan->launches) {
        if (L.kind != K_SW16) continue;
        a16.tasks = reinterpret_cast<const alnk::Sw16Task *>(ws + plan->sw16_off) + L.first;
        a16.ntasks = L.count;
        a16.items = reinterpret_cast<const alnk::Sw16Item *>(ws + plan->sw16_items_off);
        a16.nitems = (int32_t)plan->sw16_items.size();
        HIP_TRY(ctx, timed_launch(ctx, "sw16", st, [&] {
                  return alnk::launch_sw16(L.rows, a16, st);
                }));
      }
    } else {
      for (size_t k = 0; k < plan->sw16_single.size(); ++k) {
        a16.tasks = reinterpret_cast<const alnk::Sw16Task *>(ws + plan->sw16_single_off) + k;
        a16.ntasks = 1;
        a16.items = nullptr;
        a16.nitems = 0;
        HIP_TRY(ctx, alnk::launch_sw16(plan->sw16_single_rows[k], a16, st));
      }
    }
    const LaunchDesc &L = plan->rerun;
    alnk::StripArgs sa;
    sa.b = bp;
    sa.tasks = rerun_q;
    sa.ntasks = L.count;
    sa.dyn_ntasks = rerun_cnt;
    sa.mode = L.mode;
    sa.sc = dsc;
    sa.tb = nullptr;
    sa.res = d_res;
    sa.lds_bnd = L.lds_bnd;
    sa.lds_prof = L.lds_prof;
    sa.waves = 1;
    sa.max_n = 0;
    HIP_TRY(ctx, timed_launch(ctx, "strip_i32_rerun", st, [&] {
              return alnk::launch_strip(L.rows, L.mode, false, L.small, sa, st);
            }));
    return ALN_OK;
  }

  auto diag_args = [&](const PairTask *tasks, int32_t ntasks, const int32_t *dyn, int widen_rows,
                       int32_t *wcnt, PairTask *wq) {
    alnk::DiagArgs da;
    da.b = bp;
    da.tasks = tasks;
    da.ntasks = ntasks;
    da.dyn_ntasks = dyn;
    da.band_w = plan->p.band_w;
    da.xdrop = plan->p.xdrop;
    da.sc = dsc;
    da.tb = ws + plan->tb_base;
    da.res = d_res;
    da.widen_count = wcnt;
    da.widen = wq;
    da.widen_rows = widen_rows;
    da.match_mismatch = hsc.match_mismatch;
    return da;
  };
  PairTask *wq0 = plan->xdrop ? reinterpret_cast<PairTask *>(ws + plan->widen_off[0]) : nullptr;
  bool zd_lanes = false; // Z-drop on the sixteen-sides kernel
  for (const LaunchDesc &L : plan->launches)
    zd_lanes = zd_lanes || (L.kind == K_DIAG && L.sides == 16 && plan->p.prune == ALN_ZDROP);
  PairTask *wq1 = plan->xdrop ? reinterpret_cast<PairTask *>(ws + plan->widen_off[1]) : nullptr;
  PairTask *wq2 = plan->xtb_lanes ? reinterpret_cast<PairTask *>(ws + plan->widen_off[2]) : nullptr;
  if (plan->xtb_lanes) {
    // codes from the sixteen-sides kernel; pairs whose region outgrows its
    // window are recomputed with codes by the one-side pass (queue 2)
    alnk::XdlArgs xa;
    xa.zdrop = 0;
    xa.b = bp;
    xa.tasks = dtasks + plan->xtb_first;
    xa.ntasks = plan->xtb_count;
    xa.queue = widen_cnt + 2;
    xa.xdrop = plan->p.xdrop;
    xa.gap_open = hsc.gap_open;
    xa.gap_extend = hsc.gap_extend;
    xa.match = hsc.match;
    xa.mismatch = hsc.mismatch;
    xa.res = d_res;
    xa.widen_count = widen_cnt + 4;
    xa.widen = wq2;
    xa.widen_rows = 4;
    xa.tb = ws + plan->tb_base;
    if (!per_pair) {
      HIP_TRY(ctx, timed_launch(ctx, "xdrop_lanes_tb", st, [&] {
                return alnk::launch_xdrop_lanes(true, xa, plan->xtb_grid, st);
              }));
    } else {
      for (int32_t k = 0; k < plan->xtb_count; ++k) {
        xa.tasks = dtasks + plan->xtb_first + k;
        xa.ntasks = 1;
        HIP_TRY(ctx, alnk::launch_xdrop_lanes(true, xa, 1, st));
      }
    }
    alnk::DiagArgs d = diag_args(wq2, plan->n, widen_cnt + 4, 16, widen_cnt, wq0);
    HIP_TRY(ctx, timed_launch(ctx, "xdrop_tb", st, [&] {
              return alnk::launch_diag(4, ALN_EXTEND, plan->p.prune, true, d, st);
            }));
  } else if (plan->xtb_count > 0) {
    // X-drop / Z-drop with CIGAR: one pass per pair computes the results and
    // writes the traceback codes; regions that outgrow its window go to the
    // widening queue below (score only) and the walk decides their CIGAR
    auto xtb = [&](int32_t first, int32_t count) {
      alnk::DiagArgs d = diag_args(dtasks + first, count, nullptr, 16, widen_cnt, wq0);
      return alnk::launch_diag(4, ALN_EXTEND, plan->p.prune, true, d, st);
    };
    const char *fam = plan->p.prune == ALN_ZDROP ? "zdrop_tb" : "xdrop_tb";
    if (!per_pair) {
      HIP_TRY(ctx, timed_launch(ctx, fam, st, [&] { return xtb(plan->xtb_first, plan->xtb_count); }));
    } else {
      for (int32_t k = 0; k < plan->xtb_count; ++k) HIP_TRY(ctx, xtb(plan->xtb_first + k, 1));
    }
  }
  for (const LaunchDesc &L : plan->launches) {
    if (L.kind == K_DIAG) {
      if (plan->xtb_count > 0) continue; // the traceback pass above replaces it
      const int widen_rows = plan->xdrop ? (zd_lanes ? 4 : 16) : 0;
      if (L.sides == 16) {
        alnk::XdlArgs xa;
        xa.tb = nullptr;
        xa.zdrop = plan->p.prune == ALN_ZDROP ? 1 : 0;
        xa.b = bp;
        xa.tasks = dtasks + L.first;
        xa.ntasks = L.count;
        xa.queue = widen_cnt + 2;
        xa.xdrop = plan->p.xdrop;
        xa.gap_open = hsc.gap_open;
        xa.gap_extend = hsc.gap_extend;
        xa.match = hsc.match;
        xa.mismatch = hsc.mismatch;
        xa.res = d_res;
        xa.widen_count = widen_cnt;
        xa.widen = wq0;
        xa.widen_rows = widen_rows;
        if (!per_pair) {
          HIP_TRY(ctx, timed_launch(ctx, xa.zdrop ? "zdrop_lanes" : "xdrop_lanes", st, [&] {
                    return alnk::launch_xdrop_lanes(false, xa, L.grid, st);
                  }));
        } else {
          for (int32_t k = 0; k < L.count; ++k) {
            xa.tasks = dtasks + L.first + k;
            xa.ntasks = 1;
            HIP_TRY(ctx, alnk::launch_xdrop_lanes(false, xa, 1, st));
          }
        }
        continue;
      }
      auto go = [&](const alnk::DiagArgs &da) {
        return L.sides == 4 ? alnk::launch_xdrop_group(plan->p.prune, da, st)
                            : alnk::launch_diag(L.rows, L.mode, plan->p.prune, L.tb, da, st);
      };
      if (!per_pair) {
        alnk::DiagArgs da = diag_args(dtasks + L.first, L.count, nullptr, widen_rows, widen_cnt, wq0);
        const char *fam = plan->p.prune == ALN_ZDROP ? "zdrop" : (plan->xdrop ? "xdrop" : "diag_band");
        HIP_TRY(ctx, timed_launch(ctx, fam, st, [&] { return go(da); }));
      } else {
        for (int32_t k = 0; k < L.count; ++k) {
          alnk::DiagArgs da = diag_args(dtasks + L.first + k, 1, nullptr, widen_rows, widen_cnt, wq0);
          HIP_TRY(ctx, go(da));
        }
      }
      continue;
    }
    alnk::StripArgs sa;
    sa.b = bp;
    sa.dyn_ntasks = nullptr;
    sa.mode = L.mode;
    sa.sc = dsc;
    sa.tb = ws + plan->tb_base;
    sa.res = d_res;
    sa.lds_bnd = L.lds_bnd;
    sa.lds_prof = L.lds_prof;
    sa.waves = L.waves;
    sa.max_n = L.max_n;
    sa.band_w = plan->strip_band_w;
    sa.ring_cols = L.lds_bnd / 8;
    if (L.kind == K_BAND) {
      if (!per_pair) {
        sa.tasks = dtasks + L.first;
        sa.ntasks = L.count;
        HIP_TRY(ctx, timed_launch(ctx, "band_strip", st, [&] {
                  return alnk::launch_band_strip(L.rows, L.mode, L.tb, L.small, sa, st);
                }));
      } else {
        for (int32_t k = 0; k < L.count; ++k) {
          sa.tasks = dtasks + L.first + k;
          sa.ntasks = 1;
          HIP_TRY(ctx, alnk::launch_band_strip(L.rows, L.mode, L.tb, L.small, sa, st));
        }
      }
      continue;
    }
    if (!per_pair) {
      sa.tasks = dtasks + L.first;
      sa.ntasks = L.count;
      HIP_TRY(ctx, timed_launch(ctx, "strip_i32", st, [&] {
                return alnk::launch_strip(L.rows, L.mode, L.tb, L.small, sa, st);
              }));
    } else {
      for (int32_t k = 0; k < L.count; ++k) {
        sa.tasks = dtasks + L.first + k;
        sa.ntasks = 1;
        HIP_TRY(ctx, alnk::launch_strip(L.rows, L.mode, L.tb, L.small, sa, st));
      }
    }
  }
  if (plan->xdrop) {
    // pairs whose surviving region outgrew their window: 1024 diagonals, then
    // 2048.  Z-drop from the sixteen-sides kernel (64 cells) first tries the
    // one-side kernel's 256 diagonals: Z-drop regions often reach about 100
    // cells, and that window holds them at a quarter of the wider one's cost.
    const int pr = plan->p.prune;
    const char *fam = pr == ALN_ZDROP ? "zdrop_wide" : "xdrop_wide";
    alnk::DiagArgs d1 = diag_args(wq0, plan->n, widen_cnt, 32, widen_cnt + 1, wq1);
    HIP_TRY(ctx, timed_launch(ctx, fam, st, [&] {
              return alnk::launch_diag(zd_lanes ? 4 : 16, ALN_EXTEND, pr, false, d1, st);
            }));
    alnk::DiagArgs d2 = diag_args(wq1, plan->n, widen_cnt + 1, 0, nullptr, nullptr);
    HIP_TRY(ctx, timed_launch(ctx, fam, st, [&] {
              return alnk::launch_diag(32, ALN_EXTEND, pr, false, d2, st);
            }));
  }
  if (plan->p.want_cigar) {
    alnk::WalkArgs wa;
    wa.b = bp;
    wa.mode = plan->p.mode;
    wa.layout = 0;
    wa.diag_stride = plan->xtb_lanes ? 1 : (plan->xtb_count > 0 ? 2 : 8);
    wa.dyn_ntasks = nullptr;
    wa.band_w = plan->p.band_w;
    wa.sc = dsc;
    wa.tb = ws + plan->tb_base;
    wa.res = d_res;
    wa.cigar = d_cigar;
    auto walk = [&](int layout, const PairTask *tasks, int32_t nt) -> hipError_t {
      wa.tasks = tasks;
      wa.ntasks = nt;
      wa.layout = layout;
      wa.band_w = layout == 2 ? plan->strip_band_w : plan->p.band_w;
      return layout == 1 ? alnk::launch_walk_diag(wa, st) : alnk::launch_walk(layout, wa, st);
    };
    if (!per_pair) {
      HIP_TRY(ctx, timed_launch(ctx, "walk", st, [&] { return walk(0, dtasks, plan->n_strip_tb); }));
      HIP_TRY(ctx, timed_launch(ctx, "walk", st, [&] {
                return walk(1, dtasks + plan->first_diag_tb, plan->n_diag_tb);
              }));
      HIP_TRY(ctx, timed_launch(ctx, "walk", st, [&] {
                return walk(2, dtasks + plan->first_band_tb, plan->n_band_tb);
              }));
    } else {
      for (int32_t k = 0; k < plan->n_strip_tb; ++k) HIP_TRY(ctx, walk(0, dtasks + k, 1));
      for (int32_t k = 0; k < plan->n_diag_tb; ++k)
        HIP_TRY(ctx, walk(1, dtasks + plan->first_diag_tb + k, 1));
      for (int32_t k = 0; k < plan->n_band_tb; ++k)
        HIP_TRY(ctx, walk(2, dtasks + plan->first_band_tb + k, 1));
    }
    if (plan->xtb_lanes) { // the pairs the one-side pass recomputed, in its layout
      wa.diag_stride = 2;
      wa.dyn_ntasks = widen_cnt + 4;
      HIP_TRY(ctx, timed_launch(ctx, "walk", st, [&] { return walk(1, wq2, plan->n); }));
    }
  }
  return ALN_OK;
}

aln_status aln_execute(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch, void *d_ws,
                       uint64_t ws_bytes, aln_result *d_res, uint32_t *d_cigar,
                       uint64_t cigar_words, void *stream) {
  aln_status st = exec_check(ctx, plan, batch, d_ws, ws_bytes, d_res, d_cigar, cigar_words);
  if (st != ALN_OK) return st;
  return run_plan(ctx, plan, batch, d_ws, d_res, d_cigar, (hipStream_t)stream, false);
}

aln_status aln_execute_per_pair(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch, void *d_ws,
                                uint64_t ws_bytes, aln_result *d_res, uint32_t *d_cigar,
                                uint64_t cigar_words, void *stream) {
  aln_status st = exec_check(ctx, plan, batch, d_ws, ws_bytes, d_res, d_cigar, cigar_words);
  if (st != ALN_OK) return st;
  return run_plan(ctx, plan, batch, d_ws, d_res, d_cigar, (hipStream_t)stream, true);
}

aln_status aln_graph_capture(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch, void *d_ws,
                             uint64_t ws_bytes, aln_result *d_res, uint32_t *d_cigar,
                             uint64_t cigar_words, void *stream) {
  aln_status st = exec_check(ctx, plan, batch, d_ws, ws_bytes, d_res, d_cigar, cigar_words);
  if (st != ALN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (s == nullptr) return fail(ctx, ALN_E_INVAL, "graph capture needs a non-default stream");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (plan->gexec) {
    (void)hipGraphExecDestroy(plan->gexec);
    plan->gexec = nullptr;
  }
  if (plan->graph) {
    (void)hipGraphDestroy(plan->graph);
    plan->graph = nullptr;
  }
  HIP_TRY(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = run_plan(ctx, plan, batch, d_ws, d_res, d_cigar, s, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != ALN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(ctx, ALN_E_DEVICE, "end capture: %s", hipGetErrorString(e));
  plan->graph = g;
  HIP_TRY(ctx, hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
  HIP_TRY(ctx, hipGraphLaunch(plan->gexec, s));
  return ALN_OK;
}

int64_t aln_plan_describe(const aln_plan *plan, aln_launch_info *launches, int32_t max_launches,
                          int32_t *n_launches, aln_task_info *tasks, int64_t max_tasks) {
  if (!plan || max_launches < 0 || max_tasks < 0) return ALN_E_INVAL;
  int32_t nl = 0;
  int64_t nt = 0;
  auto add_launch = [&](const char *fam, int tile, int sides, int64_t first, int64_t count) {
    if (launches && nl < max_launches) {
      aln_launch_info &L = launches[nl];
      memset(&L, 0, sizeof L);
      std::snprintf(L.family, sizeof L.family, "%s", fam);
      L.tile = tile;
      L.sides = sides;
      L.first = (int32_t)first;
      L.count = (int32_t)count;
    }
    ++nl;
  };
  auto add_task = [&](int32_t launch, int32_t pair, int64_t tb_off, int64_t tb_bytes,
                      int64_t cigar_off, int32_t cigar_cap, int32_t tile) {
    if (tasks && nt < max_tasks) {
      aln_task_info &T = tasks[nt];
      T.launch = launch;
      T.pair = pair;
      T.tb_off = tb_off;
      T.tb_bytes = tb_bytes;
      T.cigar_off = cigar_off;
      T.cigar_cap = cigar_cap;
      T.tile = tile;
    }
    ++nt;
  };
  // traceback bytes of a task: up to the next reservation (offsets grow in
  // task order), the last up to the end of the traceback area
  std::vector<int64_t> tb_end(plan->tasks.size(), (int64_t)plan->tb_bytes);
  {
    int64_t next = (int64_t)plan->tb_bytes;
    for (size_t k = plan->tasks.size(); k-- > 0;) {
      if (plan->tasks[k].tb_off >= 0) {
        tb_end[k] = next;
        next = plan->tasks[k].tb_off;
      }
    }
  }
  auto pair_tasks = [&](int32_t launch, int64_t first, int64_t count) {
    for (int64_t k = first; k < first + count; ++k) {
      const alnk::PairTask &t = plan->tasks[(size_t)k];
      const bool tb = t.tb_off >= 0 && plan->p.want_cigar;
      add_task(launch, t.pair, tb ? t.tb_off : -1, tb ? tb_end[(size_t)k] - t.tb_off : 0,
               plan->p.want_cigar ? t.cigar_off : -1, plan->p.want_cigar ? t.cigar_cap : 0, t.rows);
    }
  };
  if (plan->fold) {
    for (const auto &F : plan->fold_launches) {
      const int32_t id = nl;
      add_launch("fold", F.stride, F.elt, F.first, F.count);
      for (int32_t k = F.first; k < F.first + F.count; ++k)
        add_task(id, plan->fold_tasks[(size_t)k].seq, -1, 0, -1, 0, F.stride);
    }
  } else if (plan->xtb_count > 0) {
    const int32_t id = nl;
    const char *fam = plan->xtb_lanes ? "xdrop_lanes_tb"
                                      : (plan->p.prune == ALN_ZDROP ? "zdrop_tb" : "xdrop_tb");
    add_launch(fam, 4, plan->xtb_lanes ? 16 : 1, plan->xtb_first, plan->xtb_count);
    pair_tasks(id, plan->xtb_first, plan->xtb_count);
  } else {
    for (const LaunchDesc &L : plan->launches) {
      const int32_t id = nl;
      if (L.kind == K_SW16) {
        add_launch("sw16", L.rows, 2, L.first, L.count);
        for (int32_t k = L.first; k < L.first + L.count; ++k) {
          const alnk::Sw16Task &t = plan->sw16_tasks[(size_t)k];
          add_task(id, t.pa, -1, 0, -1, 0, L.rows);
          if (t.pb >= 0) add_task(id, t.pb, -1, 0, -1, 0, L.rows);
        }
        continue;
      }
      const char *fam = "strip_i32";
      if (L.kind == K_SEARCH) fam = L.pen_x > 0 ? "search_affine" : "search";
      if (L.kind == K_BAND) fam = "band_strip";
      if (L.kind == K_DIAG) {
        if (plan->p.prune == ALN_BAND) fam = "diag_band";
        else if (plan->p.prune == ALN_ZDROP)
          fam = L.sides == 16 ? "zdrop_lanes" : (L.sides == 4 ? "zdrop_group" : "zdrop");
        else fam = L.sides == 16 ? "xdrop_lanes" : (L.sides == 4 ? "xdrop_group" : "xdrop");
      }
      add_launch(fam, L.rows, (L.kind == K_STRIP || L.kind == K_BAND) ? L.waves : L.sides, L.first,
                 L.count);
      pair_tasks(id, L.first, L.count);
    }
  }
  if (n_launches) *n_launches = nl;
  return nt;
}

aln_status aln_graph_launch(aln_ctx *ctx, aln_plan *plan, void *stream) {
  if (!ctx || !plan || !plan->gexec) return fail(ctx, ALN_E_INVAL, "no captured graph");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipGraphLaunch(plan->gexec, (hipStream_t)stream));
  return ALN_OK;
}

} // extern "C"

aln_status alnrt::plan_run(aln_ctx *ctx, aln_plan *plan, const aln_batch *b, void *d_ws,
                           aln_result *d_res, uint32_t *d_cigar, hipStream_t st, bool per_pair) {
  return run_plan(ctx, plan, b, d_ws, d_res, d_cigar, st, per_pair);
}

// ------------------------------------------------------------------ folding

extern "C" {

aln_status aln_fold_plan_create(aln_ctx *ctx, const aln_fold_params *params, int32_t n,
                                const int32_t *len_host, aln_plan **plan, aln_footprint *fp) {
  if (!ctx || !params || !plan || n < 0 || (n > 0 && !len_host))
    return fail(ctx, ALN_E_INVAL, "null argument or negative n");
  *plan = nullptr;
  const aln_fold_params &p = *params;
  int maxpair = 0;
  for (int k = 0; k < 16; ++k) {
    if (p.pair[k] < 0 || p.pair[k] > 127) return fail(ctx, ALN_E_INVAL, "pair scores must be 0..127");
    maxpair = std::max(maxpair, p.pair[k]);
  }
  if (p.min_loop < 0 || p.warmup < 0) return fail(ctx, ALN_E_INVAL, "min_loop and warmup >= 0");
  if (p.block != 0 && p.block != 256 && p.block != 512 && p.block != 1024)
    return fail(ctx, ALN_E_INVAL, "block must be 0, 256, 512 or 1024");
  // LDS of one CU, less the kernel's few static words
  const int64_t lds_max = std::min<int64_t>(ctx->lds_per_cu, 160 * 1024) - 256;
  // Per sequence: the row stride of its folded triangle (the smallest of
  // kFoldStrides above its length) and the element width (one byte when
  // every score fits 0..253 -- 255 marks minus infinity -- else two).
  struct Cls {
    int elt, stride;
  };
  std::vector<Cls> cls(n);
  for (int32_t s = 0; s < n; ++s) {
    const int32_t L = len_host[s];
    if (L < 0) return fail(ctx, ALN_E_INVAL, "negative length");
    int stride = 0;
    for (int sc : alnk::kFoldStrides)
      if (L + 1 <= sc) {
        stride = sc;
        break;
      }
    const int64_t maxF = (int64_t)maxpair * (L / 2);
    const bool u8 = stride && maxF <= 253 && (int64_t)alnk::fold_lds_bytes(1, stride, L) <= lds_max;
    const bool i16 =
        stride && maxF <= 32767 && (int64_t)alnk::fold_lds_bytes(2, stride, L) <= lds_max;
    if (!u8 && !i16)
      return fail(ctx, ALN_E_UNSUPPORTED,
                  "sequence %d (%d nt): longer than 511, or its triangle does not fit LDS, or "
                  "its scores could exceed 32767", s, L);
    cls[s] = Cls{u8 ? 1 : 2, stride};
  }
  aln_plan *pl = new (std::nothrow) aln_plan;
  if (!pl) return fail(ctx, ALN_E_NOMEM, "plan allocation");
  pl->ctx = ctx;
  pl->n = n;
  pl->fold = true;
  pl->fold_p = p;
  pl->qlen.assign(len_host, len_host + n);
  // one launch per (stride, width), the widest rows first; within a launch
  // the longest sequence first (LPT).  Threads per workgroup so that the
  // workgroups LDS lets share a CU hold about 16 wavefronts.
  int64_t cells = 0;
  for (int si = 3; si >= 0; --si) {
    for (int elt = 2; elt >= 1; --elt) {
      const int stride = alnk::kFoldStrides[si];
      std::vector<int32_t> idx;
      int32_t max_n = 0;
      for (int32_t s = 0; s < n; ++s)
        if (cls[s].stride == stride && cls[s].elt == elt) {
          idx.push_back(s);
          max_n = std::max(max_n, len_host[s]);
        }
      if (idx.empty()) continue;
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int32_t x, int32_t y) { return len_host[x] > len_host[y]; });
      const int64_t lds = (int64_t)alnk::fold_lds_bytes(elt, stride, max_n);
      const int64_t per_cu = std::max<int64_t>(1, lds_max / std::max<int64_t>(lds, 1));
      aln_plan::FoldLaunch L;
      L.elt = elt;
      L.stride = stride;
      L.block = p.block ? p.block : (per_cu >= 4 ? 256 : (per_cu >= 2 ? 512 : 1024));
      L.first = (int32_t)pl->fold_tasks.size();
      L.count = (int32_t)idx.size();
      L.max_n = max_n;
      for (int32_t s : idx) {
        pl->fold_tasks.push_back(alnk::FoldTask{s, len_host[s]});
        cells += (int64_t)len_host[s] * (len_host[s] - 1) / 2;
      }
      pl->fold_launches.push_back(L);
    }
  }
  pl->upload_bytes = sizeof(alnk::FoldTask) * pl->fold_tasks.size();
  pl->tasks_bytes = align_up(std::max<uint64_t>(pl->upload_bytes, 1));
  pl->ws_bytes = pl->tasks_bytes;
  pl->cells = cells;
  if (alnrt::plan_alloc_staging(pl) != ALN_OK) {
    delete pl;
    return fail(ctx, ALN_E_NOMEM, "staging");
  }
  plan_stage(pl, pl->pinned);
  if (fp) {
    fp->workspace_bytes = pl->ws_bytes;
    fp->traceback_bytes = 0;
    fp->cigar_words = 0;
    fp->cells = cells;
  }
  *plan = pl;
  return ALN_OK;
}

aln_status aln_fold_execute(aln_ctx *ctx, aln_plan *plan, const aln_fold_batch *b, void *d_ws,
                            uint64_t ws_bytes, aln_fold_result *d_res, void *stream) {
  if (!ctx || !plan || !b || plan->ctx != ctx || !plan->fold)
    return fail(ctx, ALN_E_INVAL, "bad context or folding plan");
  if (b->n != plan->n) return fail(ctx, ALN_E_INVAL, "batch has %d sequences, plan %d", b->n, plan->n);
  if (plan->n == 0) return ALN_OK;
  if (!d_res || !b->x || !b->off || !b->len) return fail(ctx, ALN_E_INVAL, "null device pointer");
  if (!d_ws || ws_bytes < plan->ws_bytes)
    return fail(ctx, ALN_E_CAPACITY, "workspace %llu < %llu bytes", (unsigned long long)ws_bytes,
                (unsigned long long)plan->ws_bytes);
  if (ctx->device < 0) return fail(ctx, ALN_E_DEVICE, "the context has no device");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemcpyAsync(d_ws, plan->pinned, plan->upload_bytes, hipMemcpyHostToDevice, st));
  alnk::FoldArgs a;
  a.x = b->x;
  a.off = b->off;
  a.len = b->len;
  for (int k = 0; k < 16; ++k) a.pair[k] = plan->fold_p.pair[k];
  a.min_loop = plan->fold_p.min_loop;
  a.xdrop = plan->fold_p.xdrop;
  a.warmup = plan->fold_p.warmup;
  a.res = d_res;
  const alnk::FoldTask *tasks = static_cast<const alnk::FoldTask *>(d_ws);
  for (const aln_plan::FoldLaunch &L : plan->fold_launches) {
    a.tasks = tasks + L.first;
    a.ntasks = L.count;
    a.max_n = L.max_n;
    HIP_TRY(ctx, timed_launch(ctx, "fold", st, [&] {
              return alnk::launch_fold(L.elt, L.block, L.stride, a, st);
            }));
  }
  return ALN_OK;
}

} // extern "C"
