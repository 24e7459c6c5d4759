"""Thin ctypes binding of libaln_hip.so (include/aln.h).

Argument marshalling only: every alignment step runs in the HIP library.
PyTorch supplies device memory (tensors) and streams.  Importing this module
does not touch the GPU; the first Context() loads the library and raises if
it has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaln_hip.so")

GLOBAL, LOCAL, EXTEND = 0, 1, 2
FULL, BAND, XDROP, ZDROP, SEARCH = 0, 1, 2, 3, 4
W_AUTO, W_I16, W_I32 = 0, 1, 2
NOALLOC_WORKSPACE_BYTES = 64 << 20  # ALN_NOALLOC_WORKSPACE_BYTES
R_OK, R_UNREACHABLE, R_CIGAR_CAP, R_BAD_SYMBOL, R_TOO_WIDE, R_INTERNAL = 0, 1, 2, 3, 4, 5
E_INVAL, E_NOMEM, E_DEVICE, E_CAPACITY, E_UNSUPPORTED = -1, -2, -3, -4, -5
F_I16_RERUN, F_WIDENED = 1, 2
OP_I, OP_D, OP_EQ, OP_X = 1, 2, 7, 8

RESULT_DTYPE = np.dtype([
    ("score", "<i4"), ("q_end", "<i4"), ("r_end", "<i4"), ("q_begin", "<i4"),
    ("r_begin", "<i4"), ("status", "<i4"), ("flags", "<i4"), ("cigar_len", "<i4"),
    ("cells", "<i8"), ("cigar_off", "<i8")])
assert RESULT_DTYPE.itemsize == 48


class AlnError(RuntimeError):
    pass


class _Scoring(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_int32), ("matrix", ctypes.c_void_p),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("band_w", ctypes.c_int32), ("xdrop", ctypes.c_int32),
                ("width", ctypes.c_int32), ("want_cigar", ctypes.c_int32)]


class _Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("q", ctypes.c_void_p), ("q_off", ctypes.c_void_p),
                ("q_len", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("r_off", ctypes.c_void_p), ("r_len", ctypes.c_void_p)]


class _FoldParams(ctypes.Structure):
    _fields_ = [("pair", ctypes.c_int32 * 16), ("min_loop", ctypes.c_int32),
                ("xdrop", ctypes.c_int32), ("warmup", ctypes.c_int32),
                ("block", ctypes.c_int32)]


class _FoldBatch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("x", ctypes.c_void_p), ("off", ctypes.c_void_p),
                ("len", ctypes.c_void_p)]


FOLD_RESULT_DTYPE = np.dtype([("score", "<i4"), ("i", "<i4"), ("j", "<i4"), ("full", "<i4"),
                              ("cells", "<i8"), ("terms", "<i8"), ("status", "<i4"),
                              ("reserved", "<i4")])
assert FOLD_RESULT_DTYPE.itemsize == 40


class _Footprint(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("traceback_bytes", ctypes.c_uint64),
                ("cigar_words", ctypes.c_uint64), ("cells", ctypes.c_int64)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("max_batch_pairs", ctypes.c_int32),
                ("hbm_budget", ctypes.c_uint64), ("max_batch_cells", ctypes.c_int64),
                ("class_streams", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("scoring_id", ctypes.c_int32), ("params", _Params),
                ("q", ctypes.c_void_p), ("q_len", ctypes.c_int32),
                ("r", ctypes.c_void_p), ("r_len", ctypes.c_int32),
                ("tag", ctypes.c_uint64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("admission_waits", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("peak_arena_bytes", ctypes.c_uint64),
                ("cells", ctypes.c_int64), ("peak_inflight", ctypes.c_int32),
                ("streams", ctypes.c_int32)]


COMPLETION_DTYPE = np.dtype(
    [("id", "<u8"), ("tag", "<u8")] + [(n, RESULT_DTYPE.fields[n][0]) for n in RESULT_DTYPE.names]
    + [("error", "<i4"), ("batch_pairs", "<i4"), ("batch_id", "<u8"),
       ("t_submit", "<f8"), ("t_launch", "<f8"), ("t_done", "<f8")])
assert COMPLETION_DTYPE.itemsize == 104

class _LaunchInfo(ctypes.Structure):
    _fields_ = [("family", ctypes.c_char * 24), ("tile", ctypes.c_int32),
                ("sides", ctypes.c_int32), ("first", ctypes.c_int32), ("count", ctypes.c_int32)]


TASK_INFO_DTYPE = np.dtype([("launch", np.int32), ("pair", np.int32), ("tb_off", np.int64),
                            ("tb_bytes", np.int64), ("cigar_off", np.int64),
                            ("cigar_cap", np.int32), ("tile", np.int32)])


class _Tuning(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int32), ("sw16_rows", ctypes.c_int32),
                ("strip_rows", ctypes.c_int32), ("xdrop_rows", ctypes.c_int32),
                ("xdrop_sides", ctypes.c_int32), ("sw16_wide_pct", ctypes.c_int32),
                ("sw16_ms", ctypes.c_double * 4), ("strip_ms", ctypes.c_double * 7),
                ("xdrop_ms", ctypes.c_double * 4), ("band_kernel", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("band_ms", ctypes.c_double * 5)]


SW16_TILES, STRIP_TILES = (16, 12, 8, 4), (0, 2, 4, 8, 16, 24, 32)
XDROP_TILES = ("4x1", "4x16", "8x1", "8x4")  # window cells per lane x sides per wavefront
# antidiagonal windows; strips of 4 rows per lane, 1 or 4 waves a pair; of 2 rows
BAND_KERNELS = ("diag", "strip1", "strip4", "strip1_r2", "strip4_r2")


_lib = None

# every symbol include/aln.h declares
EXPORTS = [
    "aln_abi_version", "aln_create", "aln_create_host", "aln_destroy", "aln_last_error",
    "aln_set_scoring", "aln_plan_create", "aln_plan_describe", "aln_plan_destroy", "aln_execute",
    "aln_execute_noalloc", "aln_execute_per_pair", "aln_graph_capture", "aln_graph_launch",
    "aln_set_profiling", "aln_kernel_times", "aln_autotune", "aln_get_tuning", "aln_set_tuning",
    "aln_valu_probe", "aln_fold_plan_create", "aln_fold_execute",
    "aln_server_create", "aln_server_destroy", "aln_server_submit", "aln_server_poll",
    "aln_server_drain", "aln_server_clock", "aln_server_get_stats", "aln_server_last_error",
]


def load_library(path=LIB_PATH):
    """Load libaln_hip.so and declare its signatures (no GPU call)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise AlnError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "aln_abi_version": ([], I32),
        "aln_create": ([P, I32], I32),
        "aln_create_host": ([P, I32, I32], I32),
        "aln_plan_describe": ([P, P, I32, P, P, ctypes.c_int64], ctypes.c_int64),
        "aln_destroy": ([P], None),
        "aln_last_error": ([P], ctypes.c_char_p),
        "aln_set_scoring": ([P, P, P], I32),
        "aln_plan_create": ([P, I32, P, I32, P, P, P, P], I32),
        "aln_plan_destroy": ([P], None),
        "aln_execute": ([P, P, P, P, U64, P, P, U64, P], I32),
        "aln_execute_noalloc": ([P, P, P, P, P, U64, P], I32),
        "aln_execute_per_pair": ([P, P, P, P, U64, P, P, U64, P], I32),
        "aln_graph_capture": ([P, P, P, P, U64, P, P, U64, P], I32),
        "aln_graph_launch": ([P, P, P], I32),
        "aln_set_profiling": ([P, I32], I32),
        "aln_kernel_times": ([P, P, P, P, I32], I32),
        "aln_autotune": ([P, I32, P, P, P, P, P], I32),
        "aln_get_tuning": ([P, P], I32),
        "aln_set_tuning": ([P, P], I32),
        "aln_valu_probe": ([P, I32, I32, I32, I32, P], I32),
        "aln_fold_plan_create": ([P, P, I32, P, P, P], I32),
        "aln_fold_execute": ([P, P, P, P, U64, P, P], I32),
        "aln_server_create": ([P, P, P], I32),
        "aln_server_destroy": ([P], None),
        "aln_server_submit": ([P, P, P], I32),
        "aln_server_poll": ([P, P, I32, P, U64, P, I32], I32),
        "aln_server_drain": ([P, I32], I32),
        "aln_server_clock": ([P], ctypes.c_double),
        "aln_server_get_stats": ([P, P], I32),
        "aln_server_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    def __init__(self, ctx, handle, fp, n, params):
        self.ctx = ctx
        self.handle = handle
        self.workspace_bytes = int(fp.workspace_bytes)
        self.traceback_bytes = int(fp.traceback_bytes)
        self.cigar_words = int(fp.cigar_words)
        self.cells = int(fp.cells)
        self.n = n
        self.params = params

    def describe(self):
        """(launches, tasks) of aln_plan_describe: a list of dicts and an
        ndarray of TASK_INFO_DTYPE."""
        nl = ctypes.c_int32()
        nt = int(self.ctx.lib.aln_plan_describe(self.handle, None, 0, ctypes.byref(nl), None, 0))
        if nt < 0:
            raise AlnError(f"aln_plan_describe failed ({nt})")
        L = (_LaunchInfo * max(nl.value, 1))()
        tasks = np.zeros(nt, dtype=TASK_INFO_DTYPE)
        self.ctx.lib.aln_plan_describe(self.handle, L, nl.value, ctypes.byref(nl),
                                       tasks.ctypes.data, nt)
        launches = [dict(family=L[k].family.decode(), tile=int(L[k].tile), sides=int(L[k].sides),
                         first=int(L[k].first), count=int(L[k].count)) for k in range(nl.value)]
        return launches, tasks

    def close(self):
        if self.handle is not None:
            self.ctx.lib.aln_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceBatch:
    """A workloads.Batch copied to device tensors, in the layout aln_batch names."""

    def __init__(self, batch, device="cuda"):
        import torch
        self.src = batch
        self.n = batch.n
        self.q = torch.from_numpy(np.ascontiguousarray(batch.q)).to(device)
        self.q_off = torch.from_numpy(np.ascontiguousarray(batch.q_off)).to(device)
        self.q_len = torch.from_numpy(np.ascontiguousarray(batch.q_len)).to(device)
        self.r = torch.from_numpy(np.ascontiguousarray(batch.r)).to(device)
        self.r_off = torch.from_numpy(np.ascontiguousarray(batch.r_off)).to(device)
        self.r_len = torch.from_numpy(np.ascontiguousarray(batch.r_len)).to(device)
        self.q_len_host = np.ascontiguousarray(batch.q_len, dtype=np.int32)
        self.r_len_host = np.ascontiguousarray(batch.r_len, dtype=np.int32)
        self.c = _Batch(self.n, self.q.data_ptr(), self.q_off.data_ptr(), self.q_len.data_ptr(),
                        self.r.data_ptr(), self.r_off.data_ptr(), self.r_len.data_ptr())


class Context:
    lib_path = LIB_PATH

    def __init__(self, device=0):
        self.lib = load_library()
        self.device = device
        # PyTorch holds the device memory and streams this binding uses: let
        # it set the device up first (a process whose first HIP call came from
        # the library has been seen to leave PyTorch without devices)
        try:
            import torch
            torch.cuda.init()
        except (ImportError, RuntimeError):
            pass
        h = ctypes.c_void_p()
        self._check(self.lib.aln_create(ctypes.byref(h), int(device)), None)
        self.handle = h

    @classmethod
    def host(cls, cus=0, lds_per_cu=0):
        """A context without a device (aln_create_host): planning and
        footprints only; anything that would run on a device raises."""
        self = cls.__new__(cls)
        self.lib = load_library()
        self.device = -1
        h = ctypes.c_void_p()
        self.handle = None
        self._check(self.lib.aln_create_host(ctypes.byref(h), int(cus), int(lds_per_cu)), None)
        self.handle = h
        return self

    def _check(self, rc, handle="self"):
        if rc != 0:
            msg = b""
            if handle is not None and getattr(self, "handle", None) is not None:
                msg = self.lib.aln_last_error(self.handle) or b""
            raise AlnError(f"aln call failed ({rc}): {msg.decode(errors='replace')}")

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.aln_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scoring(self, matrix, gap_open, gap_extend):
        mat = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
        A = int(mat.shape[0])
        sc = _Scoring(A, mat.ctypes.data, int(gap_open), int(gap_extend))
        sid = ctypes.c_int32()
        self._check(self.lib.aln_set_scoring(self.handle, ctypes.byref(sc), ctypes.byref(sid)))
        return int(sid.value)

    def plan(self, scoring_id, q_len_host, r_len_host, mode, prune=FULL, band_w=0, xdrop=0,
             width=W_AUTO, want_cigar=False):
        ql = np.ascontiguousarray(q_len_host, dtype=np.int32)
        rl = np.ascontiguousarray(r_len_host, dtype=np.int32)
        params = _Params(int(mode), int(prune), int(band_w), int(xdrop), int(width),
                         1 if want_cigar else 0)
        h = ctypes.c_void_p()
        fp = _Footprint()
        self._check(self.lib.aln_plan_create(self.handle, int(scoring_id), ctypes.byref(params),
                                             int(ql.size), ql.ctypes.data, rl.ctypes.data,
                                             ctypes.byref(h), ctypes.byref(fp)))
        return Plan(self, h, fp, int(ql.size), params)

    def _exec(self, fn, plan, dbatch, ws, res, cigar, stream):
        self._check(fn(self.handle, plan.handle, ctypes.byref(dbatch.c), _ptr(ws),
                       int(ws.numel()) if ws is not None else 0, _ptr(res), _ptr(cigar),
                       int(cigar.numel()) if cigar is not None else 0, _stream_handle(stream)))

    def execute(self, plan, dbatch, ws, res, cigar=None, stream=None):
        self._exec(self.lib.aln_execute, plan, dbatch, ws, res, cigar, stream)

    def execute_noalloc(self, plan, dbatch, res, cigar=None, stream=None):
        """aln_execute on the library's fixed per-GPU workspace (no allocation)."""
        self._check(self.lib.aln_execute_noalloc(
            self.handle, plan.handle, ctypes.byref(dbatch.c), _ptr(res), _ptr(cigar),
            int(cigar.numel()) if cigar is not None else 0, _stream_handle(stream)))

    def execute_per_pair(self, plan, dbatch, ws, res, cigar=None, stream=None):
        self._exec(self.lib.aln_execute_per_pair, plan, dbatch, ws, res, cigar, stream)

    def graph_capture(self, plan, dbatch, ws, res, cigar=None, stream=None):
        self._exec(self.lib.aln_graph_capture, plan, dbatch, ws, res, cigar, stream)

    def graph_launch(self, plan, stream=None):
        self._check(self.lib.aln_graph_launch(self.handle, plan.handle, _stream_handle(stream)))

    def autotune(self, scoring_id, dbatch, mode, prune=FULL, band_w=0, xdrop=0, width=W_AUTO,
                 want_cigar=False, stream=None, cache=None, scoring=None):
        """Time every candidate tile of the kernel family this batch uses on
        the batch itself (a DeviceBatch; pass a sample of a large workload)
        and keep the fastest for later plans of this context.

        cache: path of a JSON tuning cache (tuning_cache.py); with
        scoring=(matrix, gap_open, gap_extend) a cached choice for the same
        device, library, scoring, parameters and batch shape is applied
        without timing, and a new one is stored.  The result carries
        "cached": True when it came from the file."""
        key = None
        if cache is not None and scoring is not None:
            from . import tuning_cache
            import torch
            prop = torch.cuda.get_device_properties(self.device)
            dev = f"{prop.name}/{getattr(prop, 'gcnArchName', '')}"
            key = tuning_cache.make_key(self.lib_path, dev, scoring[0], scoring[1], scoring[2],
                                        mode, prune, band_w, xdrop, width, want_cigar,
                                        dbatch.q_len_host, dbatch.r_len_host)
            hit = tuning_cache.lookup(cache, key)
            if hit is not None:
                self.set_tuning(hit)
                return dict(self.tuning(), cached=True)
        params = _Params(int(mode), int(prune), int(band_w), int(xdrop), int(width),
                         1 if want_cigar else 0)
        ql = dbatch.q_len_host
        rl = dbatch.r_len_host
        self._check(self.lib.aln_autotune(self.handle, int(scoring_id), ctypes.byref(params),
                                          ctypes.byref(dbatch.c), ql.ctypes.data, rl.ctypes.data,
                                          _stream_handle(stream)))
        t = self.tuning()
        if key is not None:
            from . import tuning_cache
            tuning_cache.store(cache, key, {k: v for k, v in t.items() if not k.endswith("_ms")})
        return dict(t, cached=False)

    def tuning(self):
        t = _Tuning()
        self._check(self.lib.aln_get_tuning(self.handle, ctypes.byref(t)))
        return {"valid": bool(t.valid), "sw16_rows": int(t.sw16_rows),
                "strip_rows": int(t.strip_rows), "xdrop_rows": int(t.xdrop_rows),
                "xdrop_sides": int(t.xdrop_sides), "sw16_wide_pct": int(t.sw16_wide_pct),
                "sw16_ms": dict(zip(SW16_TILES, map(float, t.sw16_ms))),
                "strip_ms": dict(zip(STRIP_TILES, map(float, t.strip_ms))),
                "xdrop_ms": dict(zip(XDROP_TILES, map(float, t.xdrop_ms))),
                "band_kernel": int(t.band_kernel),
                "band_ms": dict(zip(BAND_KERNELS, map(float, t.band_ms)))}

    def set_tuning(self, tuning):
        t = _Tuning()
        t.valid = 1 if tuning.get("valid", True) else 0
        t.sw16_rows = int(tuning.get("sw16_rows", 16))
        t.strip_rows = int(tuning.get("strip_rows", 0))
        t.xdrop_rows = int(tuning.get("xdrop_rows", 4))
        t.xdrop_sides = int(tuning.get("xdrop_sides", 1))
        t.sw16_wide_pct = int(tuning.get("sw16_wide_pct", 0))
        t.band_kernel = int(tuning.get("band_kernel", 0))
        self._check(self.lib.aln_set_tuning(self.handle, ctypes.byref(t)))

    def set_profiling(self, enable):
        self._check(self.lib.aln_set_profiling(self.handle, 1 if enable else 0))

    def kernel_times(self, max_families=16):
        """{family: (total_ms, launches)} since the last call (profiling on)."""
        names = (ctypes.c_char_p * max_families)()
        ms = (ctypes.c_double * max_families)()
        cnt = (ctypes.c_int64 * max_families)()
        k = self.lib.aln_kernel_times(self.handle, names, ms, cnt, max_families)
        if k < 0:
            raise AlnError(f"aln_kernel_times failed ({k})")
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}


PROBE_OPS = ("v_add_u32", "v_max_i32", "v_max3_i32", "v_cmp_gt_i32", "v_cndmask_b32",
             "v_pk_max_i16", "v_pk_add_u16", "v_lshl_or_b32", "v_add3_u32", "v_mov_b32_dpp",
             "v_max_i32_dpp", "v_add_u32_sdwa", "v_perm_b32", "v_alignbyte_b32", "v_bfe_u32",
             "v_addc_co_u32")


def valu_probe(ctx, op, dependent=False, waves_per_simd=4, iters=2000):
    """aln_valu_probe: issue rate (wave instructions per SIMD per cycle) of one
    instruction class with every SIMD busy, and the shader clock under that
    load (GHz).  Returns a dict."""
    out = (ctypes.c_double * 6)()
    k = PROBE_OPS.index(op) if isinstance(op, str) else int(op)
    ctx._check(ctx.lib.aln_valu_probe(ctx.handle, k, 1 if dependent else 0, int(waves_per_simd),
                                      int(iters), out))
    ms, cyc, ticks, waves, instr, simds = list(out)
    return dict(op=PROBE_OPS[k], dependent=bool(dependent), waves_per_simd=int(waves_per_simd),
                ms=ms, clock_ghz=0.1 * cyc / ticks if ticks else None,
                issue_per_simd_cycle=instr * waves_per_simd / cyc if cyc else None,
                cycles_per_instr_one_wave=cyc / instr if instr else None,
                wall_rate_per_simd_ns=instr * waves / simds / (ms * 1e6) if ms else None)


class FoldDeviceBatch:
    """A workloads.FoldBatch copied to device tensors (aln_fold_batch)."""

    def __init__(self, fb, device="cuda"):
        import torch
        self.src = fb
        self.n = fb.n
        self.x = torch.from_numpy(np.ascontiguousarray(fb.x)).to(device)
        self.off = torch.from_numpy(np.ascontiguousarray(fb.off)).to(device)
        self.len = torch.from_numpy(np.ascontiguousarray(fb.length)).to(device)
        self.len_host = np.ascontiguousarray(fb.length, dtype=np.int32)
        self.c = _FoldBatch(self.n, self.x.data_ptr(), self.off.data_ptr(), self.len.data_ptr())


def fold_params(pair, min_loop=0, xdrop=-1, warmup=15, block=0):
    p = _FoldParams()
    flat = np.asarray(pair, dtype=np.int32).reshape(16)
    for k in range(16):
        p.pair[k] = int(flat[k])
    p.min_loop, p.xdrop, p.warmup, p.block = int(min_loop), int(xdrop), int(warmup), int(block)
    return p


def fold_plan(ctx, fb, len_host=None, block=0):
    """aln_fold_plan_create for a workloads.FoldBatch (its parameters and lengths)."""
    lens = np.ascontiguousarray(fb.length if len_host is None else len_host, dtype=np.int32)
    params = fold_params(fb.pair, fb.min_loop, fb.xdrop, fb.warmup, block)
    h = ctypes.c_void_p()
    fp = _Footprint()
    ctx._check(ctx.lib.aln_fold_plan_create(ctx.handle, ctypes.byref(params), int(lens.size),
                                            lens.ctypes.data, ctypes.byref(h), ctypes.byref(fp)))
    return Plan(ctx, h, fp, int(lens.size), params)


def fold_execute(ctx, plan, fdb, ws, res, stream=None):
    ctx._check(ctx.lib.aln_fold_execute(ctx.handle, plan.handle, ctypes.byref(fdb.c), _ptr(ws),
                                        int(ws.numel()), _ptr(res), _stream_handle(stream)))


def fold(ctx, fb, stream=None, block=0):
    """Plan and run one workloads.FoldBatch; returns the results ndarray."""
    import torch
    plan = fold_plan(ctx, fb, block=block)
    fdb = FoldDeviceBatch(fb)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    res = torch.zeros(max(fb.n, 1) * FOLD_RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    fold_execute(ctx, plan, fdb, ws, res, stream=stream)
    torch.cuda.synchronize()
    out = np.frombuffer(res.cpu().numpy().tobytes(), dtype=FOLD_RESULT_DTYPE, count=fb.n).copy()
    plan.close()
    return out


class Buffers:
    """Device buffers for one plan: workspace (uint8), results, CIGAR words."""

    def __init__(self, plan, device="cuda"):
        import torch
        self.ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=device)
        self.res = torch.zeros(max(plan.n, 1) * RESULT_DTYPE.itemsize, dtype=torch.uint8,
                               device=device)
        self.cigar = (torch.zeros(max(plan.cigar_words, 1), dtype=torch.int32, device=device)
                      if plan.params.want_cigar else None)

    def results(self, n):
        raw = self.res.cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=RESULT_DTYPE, count=n).copy()

    def cigars(self, res):
        if self.cigar is None:
            return None
        words = self.cigar.cpu().numpy().view(np.uint32)
        return [words[int(r["cigar_off"]): int(r["cigar_off"]) + int(r["cigar_len"])].copy()
                for r in res]


def align(ctx, batch, scoring_id=None, width=W_AUTO, mode=None, per_pair=False, graph=False,
          stream=None, dbatch=None):
    """Plan and run one workloads.Batch; returns (results ndarray, cigars or None)."""
    import torch
    if scoring_id is None:
        scoring_id = ctx.set_scoring(batch.matrix, batch.gap_open, batch.gap_extend)
    plan = ctx.plan(scoring_id, batch.q_len, batch.r_len, batch.mode if mode is None else mode,
                    batch.prune, batch.band_w, batch.xdrop, width, batch.want_cigar)
    db = dbatch if dbatch is not None else DeviceBatch(batch)
    buf = Buffers(plan)
    if graph:
        s = stream or torch.cuda.Stream()
        ctx.graph_capture(plan, db, buf.ws, buf.res, buf.cigar, stream=s)
        s.synchronize()
    elif per_pair:
        ctx.execute_per_pair(plan, db, buf.ws, buf.res, buf.cigar, stream=stream)
    else:
        ctx.execute(plan, db, buf.ws, buf.res, buf.cigar, stream=stream)
    torch.cuda.synchronize()
    res = buf.results(batch.n)
    cig = buf.cigars(res)
    plan.close()
    return res, cig


class Server:
    """Continuous-batching request server (include/aln.h, aln_server_*).

    Scorings must be set on ``ctx`` before the server is created.  submit()
    copies the sequences; poll() returns (completions ndarray of
    COMPLETION_DTYPE, list of CIGAR arrays or None per completion)."""

    def __init__(self, ctx, streams=4, max_batch_pairs=1024, hbm_budget=0, max_batch_cells=0,
                 class_streams=0):
        self.ctx = ctx
        self.lib = ctx.lib
        cfg = _ServerCfg(int(streams), int(max_batch_pairs), int(hbm_budget),
                         int(max_batch_cells), int(class_streams), 0)
        h = ctypes.c_void_p()
        ctx._check(self.lib.aln_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._max_cigar = 1
        self._comp = (ctypes.c_uint8 * (COMPLETION_DTYPE.itemsize * 256))()
        self._cig = np.zeros(1 << 16, dtype=np.uint32)

    def _err(self, rc):
        msg = self.lib.aln_server_last_error(self.handle) or b""
        return AlnError(f"aln_server call failed ({rc}): {msg.decode(errors='replace')}")

    def submit(self, scoring_id, q, r, mode, prune=FULL, band_w=0, xdrop=0, width=W_AUTO,
               want_cigar=False, tag=0):
        qa = np.ascontiguousarray(q, dtype=np.uint8)
        ra = np.ascontiguousarray(r, dtype=np.uint8)
        req = _Request(int(scoring_id),
                       _Params(int(mode), int(prune), int(band_w), int(xdrop), int(width),
                               1 if want_cigar else 0),
                       qa.ctypes.data if qa.size else None, int(qa.size),
                       ra.ctypes.data if ra.size else None, int(ra.size), int(tag))
        rid = ctypes.c_uint64()
        rc = self.lib.aln_server_submit(self.handle, ctypes.byref(req), ctypes.byref(rid))
        if rc != 0:
            raise self._err(rc)
        if want_cigar:
            self._max_cigar = max(self._max_cigar, qa.size + ra.size + 1)
        return int(rid.value)

    def poll(self, max_n=256, wait_us=0):
        max_n = min(int(max_n), 256)
        need = self._max_cigar * max_n
        if self._cig.size < need:
            self._cig = np.zeros(need, dtype=np.uint32)
        used = ctypes.c_uint64()
        k = self.lib.aln_server_poll(self.handle, self._comp, max_n, self._cig.ctypes.data,
                                     int(self._cig.size), ctypes.byref(used), int(wait_us))
        if k < 0:
            raise self._err(k)
        comp = np.frombuffer(bytes(self._comp)[: k * COMPLETION_DTYPE.itemsize],
                             dtype=COMPLETION_DTYPE).copy()
        cigs = [self._cig[int(c["cigar_off"]): int(c["cigar_off"]) + int(c["cigar_len"])].copy()
                if c["cigar_len"] > 0 else None for c in comp]
        return comp, cigs

    def drain(self, timeout_ms=-1):
        rc = self.lib.aln_server_drain(self.handle, int(timeout_ms))
        if rc != 0:
            raise self._err(rc)

    def clock(self):
        return float(self.lib.aln_server_clock(self.handle))

    def stats(self):
        st = _ServerStats()
        rc = self.lib.aln_server_get_stats(self.handle, ctypes.byref(st))
        if rc != 0:
            raise self._err(rc)
        return {n: int(getattr(st, n)) for n, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.aln_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

