// autotune.cpp -- choose tiles by timing candidates on the caller's batch.
//
// Which tile is fastest depends on the length mix and on the device: a
// shorter strip wastes fewer padded rows but pays more per step, and a
// launch lasts as long as its longest pair.  Rather than predict that, the
// tuner plans the batch once per candidate tile of the kernel family it
// uses, runs each plan (one warm-up, then the faster of two timed runs) and
// keeps the fastest.  Every candidate computes the same results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "runtime.h"

namespace {

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Plan and time the batch with the context's current forced tile.  Returns
// ms, or a negative value if the planner rejects the tile; device errors
// are returned through *err.
double time_candidate(aln_ctx *ctx, int32_t sid, const aln_params &prm, const aln_batch *b,
                      const int32_t *ql, const int32_t *rl, hipStream_t st, aln_status *err) {
  aln_plan *pl = nullptr;
  aln_footprint fp{};
  const aln_status ps = aln_plan_create(ctx, sid, &prm, b->n, ql, rl, &pl, &fp);
  if (ps == ALN_E_UNSUPPORTED) return -1.0; // this tile cannot run these pairs
  if (ps != ALN_OK) {
    *err = ps;
    return -1.0;
  }
  DevBuf ws, res, cig;
  if (hipMalloc(&ws.p, std::max<uint64_t>(fp.workspace_bytes, 1)) != hipSuccess ||
      hipMalloc(&res.p, sizeof(aln_result) * (size_t)std::max(b->n, 1)) != hipSuccess ||
      (fp.cigar_words && hipMalloc(&cig.p, 4 * fp.cigar_words) != hipSuccess)) {
    aln_plan_destroy(pl);
    *err = alnrt::fail(ctx, ALN_E_NOMEM, "autotune: device buffers");
    return -1.0;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = -1.0;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, st);
      *err = aln_execute(ctx, pl, b, ws.p, fp.workspace_bytes, (aln_result *)res.p,
                         (uint32_t *)cig.p, fp.cigar_words, st);
      (void)hipEventRecord(e1, st);
      if (*err != ALN_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        *err = alnrt::fail(ctx, ALN_E_DEVICE, "autotune: run failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && (best < 0 || ms < best)) best = ms;
    }
  } else {
    *err = alnrt::fail(ctx, ALN_E_DEVICE, "autotune: events");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  aln_plan_destroy(pl);
  return *err == ALN_OK ? best : -1.0;
}

// Time each candidate (set through `force`), return the fastest (or
// `fallback` when none runs) and record the times.
template <class F>
int pick(const int *cands, int nc, double *ms_out, int fallback, F &&time_with) {
  int best = fallback;
  double best_ms = 1e300;
  for (int c = 0; c < nc; ++c) {
    const double ms = time_with(cands[c]);
    ms_out[c] = ms;
    if (ms > 0 && ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  return best;
}

} // namespace

extern "C" {

aln_status aln_autotune(aln_ctx *ctx, int32_t scoring_id, const aln_params *params,
                        const aln_batch *batch, const int32_t *q_len_host,
                        const int32_t *r_len_host, void *stream) {
  if (!ctx || !params || !batch || (batch->n > 0 && (!q_len_host || !r_len_host)))
    return alnrt::fail(ctx, ALN_E_INVAL, "null argument");
  if (scoring_id < 0 || scoring_id >= (int32_t)ctx->dsc.size())
    return alnrt::fail(ctx, ALN_E_INVAL, "unknown scoring id %d", scoring_id);
  if (batch->n == 0) return ALN_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return alnrt::fail(ctx, ALN_E_DEVICE, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const aln_params &p = *params;
  aln_tuning t = ctx->tuning;
  if (!t.valid) {
    t = aln_tuning{};
    t.sw16_rows = 16;
    t.strip_rows = 0;
    t.xdrop_rows = 4;
    t.xdrop_sides = 1;
  }
  aln_status err = ALN_OK;
  auto run = [&]() {
    return time_candidate(ctx, scoring_id, p, batch, q_len_host, r_len_host, st, &err);
  };
  const bool local_full = p.mode == ALN_LOCAL && p.prune == ALN_FULL && !p.want_cigar &&
                          p.width != ALN_W_I32;
  if (p.prune == ALN_XDROP || p.prune == ALN_ZDROP) {
    // X-drop and Z-drop share the kernel family and its tile choice;
    // candidates rows x sides: 4x1, 4x16, 8x1, 8x4 (encoded rows +
    // 100*(sides-1)); 4x16 is the sixteen-sides kernel where the plan
    // qualifies, else 4x1
    static const int c[4] = {4, 1504, 8, 308};
    const int best = pick(c, 4, t.xdrop_ms, 4, [&](int code) {
      ctx->force_xdrop_rows = code % 100;
      ctx->force_xdrop_sides = code / 100 + 1;
      const double ms = run();
      ctx->force_xdrop_rows = 0;
      ctx->force_xdrop_sides = 0;
      return ms;
    });
    t.xdrop_rows = best % 100;
    t.xdrop_sides = best / 100 + 1;
  } else if (local_full) {
    // rows per lane x the wide-item threshold; sw16_ms keeps each tile's
    // best time over the thresholds
    static const int c[4] = {16, 12, 8, 4};
    static const int wp[4] = {25, 40, 60, 80};
    int wide_of[17] = {0};
    t.sw16_rows = pick(c, 4, t.sw16_ms, 16, [&](int r) {
      double wms[4];
      ctx->force_sw16_rows = r;
      wide_of[r] = pick(wp, 4, wms, 80, [&](int pct) {
        ctx->force_sw16_wide_pct = pct;
        const double ms = run();
        ctx->force_sw16_wide_pct = 0;
        return ms;
      });
      ctx->force_sw16_rows = 0;
      double ms = -1.0;
      for (double x : wms)
        if (x > 0 && (ms < 0 || x < ms)) ms = x;
      return ms;
    });
    t.sw16_wide_pct = wide_of[t.sw16_rows] ? wide_of[t.sw16_rows] : 80;
  } else if (p.prune == ALN_FULL) {
    static const int c[7] = {0, 2, 4, 8, 16, 24, 32};
    t.strip_rows = pick(c, 7, t.strip_ms, 0, [&](int r) {
      ctx->force_strip_rows = r;
      const double ms = run();
      ctx->force_strip_rows = -1;
      return ms;
    });
  } else if (p.prune == ALN_BAND) {
    // antidiagonal windows, or strips with one or four wavefronts per pair
    // and 4 or 2 rows per lane
    static const int c[5] = {1, 2, 3, 4, 5};
    t.band_kernel = pick(c, 5, t.band_ms, 0, [&](int k) {
      ctx->force_band_kernel = k;
      const double ms = run();
      ctx->force_band_kernel = 0;
      return ms;
    });
  } else {
    return ALN_OK;
  }
  if (err != ALN_OK) return err;
  t.valid = 1;
  ctx->tuning = t;
  return ALN_OK;
}

aln_status aln_get_tuning(const aln_ctx *ctx, aln_tuning *tuning) {
  if (!ctx || !tuning) return ALN_E_INVAL;
  *tuning = ctx->tuning;
  return ALN_OK;
}

aln_status aln_set_tuning(aln_ctx *ctx, const aln_tuning *tuning) {
  if (!ctx || !tuning) return ALN_E_INVAL;
  if (tuning->valid) {
    const int s = tuning->sw16_rows, r = tuning->strip_rows, x = tuning->xdrop_rows;
    const int xs = tuning->xdrop_sides, w = tuning->sw16_wide_pct;
    if (!(s == 4 || s == 8 || s == 12 || s == 16) ||
        !(r == 0 || r == 2 || r == 4 || r == 8 || r == 16 || r == 24 || r == 32) ||
        !(x == 2 || x == 4 || x == 8) ||
        !(xs == 1 || (xs == 4 && x == 8) || (xs == 16 && x == 4)) || w < -1 || w > 10000 ||
        tuning->band_kernel < 0 || tuning->band_kernel > 5)
      return alnrt::fail(ctx, ALN_E_INVAL, "tile choice outside the kernels' tiles");
  }
  ctx->tuning = *tuning;
  return ALN_OK;
}

} // extern "C"
