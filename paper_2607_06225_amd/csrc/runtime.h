// runtime.h -- host-side state shared by the execution API (aln_api.cpp) and
// the request server (server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "aln.h"
#include "internal.h"

struct aln_ctx {
  int device = 0; // -1: a context without a device (aln_create_host)
  int cus = 256;                // compute units, and LDS bytes per CU (planner's load model)
  int lds_per_cu = 160 * 1024;
  std::string err;
  std::vector<alnk::DevScoring *> dsc; // device copies, owned
  std::vector<alnk::DevScoring> hsc;   // host mirrors
  // kernel timing (aln_set_profiling)
  bool profiling = false;
  struct TimedLaunch {
    const char *name;
    hipEvent_t a, b;
  };
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  // autotuning: the tiles chosen by aln_autotune, and the tile the tuner
  // forces while it measures a candidate (sw16/xdrop 0, strips -1: none)
  aln_tuning tuning{};
  int force_sw16_rows = 0;
  int force_strip_rows = -1;
  int force_xdrop_rows = 0;
  int force_xdrop_sides = 0;
  int force_sw16_wide_pct = 0;
  int force_band_kernel = 0;
  // device address of the fixed workspace of aln_execute_noalloc (this device)
  void *scratch = nullptr;
};

namespace alnrt {

enum Kind { K_STRIP = 0, K_SW16 = 1, K_RERUN = 2, K_DIAG = 3, K_SEARCH = 4, K_BAND = 5 };

struct LaunchDesc {
  int kind;
  int rows;
  int mode;
  bool tb;
  bool small;
  int32_t first; // first task of this launch
  int32_t count;
  int32_t lds_bnd;
  int32_t lds_prof;
  int sides = 1; // X-drop: extension sides per wavefront (16: the persistent lanes kernel)
  int grid = 0;  // X-drop lanes kernel: wavefronts of the persistent grid
  int waves = 1; // full matrix: wavefronts per pair (strip pipeline)
  int max_n = 0; // largest reference length of the launch
  int32_t lds_f = 0;  // search: LDS bytes of one furthest-row array
  int32_t pen_x = 0, pen_o = 0, pen_e = 0, ring_h = 0, ring_e = 0; // gap-affine SEARCH
  int32_t dcap = 0, lds_fc = 0; // gap-affine: first-pass diagonal cap and its row bytes
};

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

// Record a formatted message as ctx's last error and return st.
aln_status fail(aln_ctx *ctx, aln_status st, const char *fmt, ...);

} // namespace alnrt

struct aln_plan {
  aln_ctx *ctx = nullptr;
  int32_t scoring_id = 0;
  aln_params p{};
  int32_t n = 0;
  std::vector<int32_t> qlen, rlen;
  std::vector<alnk::PairTask> tasks;
  std::vector<alnrt::LaunchDesc> launches;
  // packed int16 path
  std::vector<alnk::Sw16Task> sw16_tasks;    // two pairs per task
  std::vector<alnk::Sw16Task> sw16_single;   // one pair per task (per-pair runs)
  std::vector<int> sw16_single_rows;         // tile of each single task
  std::vector<alnk::Sw16Item> sw16_items;    // one wavefront each, longest first
  int32_t sw16_wide = 0;                     // items running one task on 64 lanes
  int sw16_rows = 16;
  uint64_t sw16_off = 0, sw16_items_off = 0, sw16_single_off = 0, rerun_cnt_off = 0, rerun_off = 0;
  alnrt::LaunchDesc rerun{};
  // X-drop widening queues: counters (ws offset) and two queues of n tasks
  uint64_t widen_cnt_off = 0, widen_off[3] = {0, 0, 0};
  // X-drop with CIGAR on the sixteen-sides kernel (codes 32 B per antidiagonal);
  // pairs that outgrow its window go to the one-side pass with codes (queue 2)
  bool xtb_lanes = false;
  int xtb_grid = 0;
  bool xdrop = false;
  int32_t n_strip_tb = 0, first_diag_tb = 0, n_diag_tb = 0; // walk ranges
  int32_t first_band_tb = 0, n_band_tb = 0;
  // band strips' half-width: the band's, or for full-matrix pairs on band
  // strips a width past every pair's (the band then covers the matrix)
  int32_t strip_band_w = 0;
  int32_t xtb_first = 0, xtb_count = 0; // X-drop / Z-drop traceback-pass tasks
  uint64_t upload_bytes = 0; // task lists copied to the front of the workspace
  uint64_t tasks_bytes = 0;
  uint64_t tb_base = 0;
  uint64_t tb_bytes = 0;
  uint64_t ws_bytes = 0;
  uint64_t cigar_words = 0;
  int64_t cells = 0;
  void *pinned = nullptr;   // host staging of the task lists
  bool own_pinned = true;   // false: staging belongs to the server slot
  bool host_staging = false; // staging in plain host memory (a context without a device)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // RNA folding plans (aln_fold_plan_create): parameters, tasks in launch
  // order and one launch per LDS size class
  bool fold = false;
  aln_fold_params fold_p{};
  std::vector<alnk::FoldTask> fold_tasks;
  struct FoldLaunch {
    int elt;    // bytes per triangle element
    int stride; // row stride of the folded triangle (elements)
    int block;  // threads per workgroup
    int32_t first, count, max_n;
  };
  std::vector<FoldLaunch> fold_launches;
};

namespace alnrt {

// Plan a batch from host lengths (kernel choice, buckets, workspace layout).
// Host work only; no pinned staging is allocated (pl->pinned stays null).
aln_status plan_build(aln_ctx *ctx, int32_t scoring_id, const aln_params *params, int32_t n,
                      const int32_t *q_len_host, const int32_t *r_len_host, aln_plan **out);
// Write the plan's upload image (plan->upload_bytes bytes) to dst.
void plan_stage(const aln_plan *pl, void *dst);
// Look up the device address of the fixed no-allocation workspace on
// ctx->device (current) and keep it in ctx->scratch.
aln_status scratch_init(aln_ctx *ctx);
// host staging of a plan's task lists: pinned, or plain memory without a device
aln_status plan_alloc_staging(aln_plan *pl);
// Argument checks shared by the execute entry points.
aln_status exec_check(aln_ctx *ctx, aln_plan *plan, const aln_batch *b, void *d_ws,
                      uint64_t ws_bytes, aln_result *d_res, uint32_t *d_cigar,
                      uint64_t cigar_words);
// Enqueue the plan on `st` (upload from pl->pinned, then the kernels).
aln_status plan_run(aln_ctx *ctx, aln_plan *plan, const aln_batch *b, void *d_ws,
                    aln_result *d_res, uint32_t *d_cigar, hipStream_t st, bool per_pair);

} // namespace alnrt
