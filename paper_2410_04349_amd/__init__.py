"""Python binding of libhb, the MI355X rule-based blocking library.

Argument marshalling only: every step on the data runs in libhb's HIP
kernels.  PyTorch supplies device memory (an allocator callback backed by
its caching allocator) and the stream.  The functions carry the names of
the C entry points declared in include/hb.h.

The in-tree shared library must exist (built by `build.py`); importing
this package without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhb.so")

HB_OK = 0
HB_ERR_INVALID_ARG = 1
HB_ERR_TYPE = 2
HB_ERR_UNBLOCKABLE = 3
HB_ERR_LIMIT = 4
HB_ERR_OOM = 5
HB_ERR_CAPACITY = 6
HB_ERR_HIP = 7
HB_ERR_STALE_ID = 8
HB_ERR_STATE = 9

HB_PLAN_GIVEN = 0
HB_PLAN_HEURISTIC = 1
HB_PLAN_LEARNED = 2

_COLTYPE = {"string": 0, "categorical": 1, "int64": 2}
_OP = {"eq": 0, "ed": 1, "jaccard": 2, "absdiff": 3, "eq_const": 4, "eq_cross": 5, "ed_cross": 6,
       "jaccard_cross": 7, "contain": 8}
HB_PLAN_CHEAPEST, HB_PLAN_SELECTIVE, HB_PLAN_RANDOM_PREDS, HB_PLAN_RANDOM_RULES = 3, 4, 5, 6
_PLAN = {"given": HB_PLAN_GIVEN, "heuristic": HB_PLAN_HEURISTIC, "learned": HB_PLAN_LEARNED,
         "cheapest": HB_PLAN_CHEAPEST, "selective": HB_PLAN_SELECTIVE,
         "random_preds": HB_PLAN_RANDOM_PREDS, "random_rules": HB_PLAN_RANDOM_RULES}

EXPORTED = [
    "hb_create", "hb_destroy", "hb_last_error", "hb_version", "hb_load_relation", "hb_load_relation_async",
    "hb_release_relation",
    "hb_compile_rules", "hb_partition", "hb_match", "hb_match_noalloc", "hb_set_rows_per_wave", "hb_set_sparse_rows", "hb_set_pack_small_blocks", "hb_set_learned_min_saving", "hb_ruleset_estimates", "hb_ruleset_buckets",
    "hb_epg_path", "hb_plan_path", "hb_profile_enable", "hb_profile_query", "hb_profile_bytes", "hb_profile_reset", "hb_last_match_stats",
    "hb_match_work", "hb_costmodel_init", "hb_costmodel_set_params", "hb_costmodel_get_params",
    "hb_costmodel_train", "hb_costmodel_predict", "hb_costmodel_trace", "hb_costmodel_adam_step",
    "hb_costmodel_save", "hb_costmodel_load", "hb_costmodel_select", "hb_set_cost_estimate",
    "hb_log_collect", "hb_pair_log_collect", "hb_batch_create", "hb_batch_run", "hb_batch_result", "hb_batch_info_get",
    "hb_batch_destroy",
]

HB_BATCH_GRAPH = 1
HB_BATCH_AUTOTUNE = 2
HB_BATCH_FORM = {"streams": 0x100, "multi": 0x200, "persistent": 0x300}

HB_MLP_PARAMS = 5378
HB_MODEL_BLOCK, HB_MODEL_PAIR = 0, 1
_MODEL = {"block": HB_MODEL_BLOCK, "pair": HB_MODEL_PAIR}
HB_COST_STATIC, HB_COST_PAIR_NET = 0, 1
_COST = {"static": HB_COST_STATIC, "pair_net": HB_COST_PAIR_NET}

OP_KINDS = ["eq_value", "absdiff", "eq_string_filter", "ed_filter", "jaccard_filter", "eq_string",
            "edit_distance", "jaccard"]


class HbJob(ctypes.Structure):
    _fields_ = [("rel_id", ctypes.c_uint32), ("ruleset_id", ctypes.c_uint32)]


class HbBatchInfo(ctypes.Structure):
    _fields_ = [("n_jobs", ctypes.c_uint32), ("n_partitions", ctypes.c_uint32), ("work_items", ctypes.c_uint64),
                ("form", ctypes.c_int32),
                ("grid", ctypes.c_uint32), ("grab", ctypes.c_uint32), ("occupancy", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("graph", ctypes.c_int32), ("n_tuned", ctypes.c_uint32),
                ("tune_ms", ctypes.c_double * 32), ("fallback_blocks", ctypes.c_uint64)]


class HbColumn(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("bytes", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("valid", ctypes.c_void_p)]


class HbPred(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("attr", ctypes.c_uint32), ("k", ctypes.c_int64),
                ("q", ctypes.c_uint32), ("num", ctypes.c_uint32), ("den", ctypes.c_uint32),
                ("d", ctypes.c_int64), ("attr_b", ctypes.c_uint32), ("side", ctypes.c_int32),
                ("c", ctypes.c_int64)]


class HbRule(ctypes.Structure):
    _fields_ = [("n_preds", ctypes.c_uint32), ("preds", ctypes.POINTER(HbPred))]


class HbMatchStats(ctypes.Structure):
    _fields_ = [("candidate_pairs", ctypes.c_uint64), ("matched_pairs", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("learned_blocks", ctypes.c_uint64), ("fallback_blocks", ctypes.c_uint64),
                ("learned_plans", ctypes.c_uint64), ("predicted_heuristic", ctypes.c_double),
                ("predicted_chosen", ctypes.c_double)]


class HbWorkStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("matched", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("waves", ctypes.c_uint64 * 8), ("lanes", ctypes.c_uint64 * 8), ("passed", ctypes.c_uint64 * 8),
                ("work", ctypes.c_uint64 * 8), ("lane_ops", ctypes.c_double), ("batch_ops", ctypes.c_double),
                ("issued_ops", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libhb.so is not built ({LIB_PATH}); run paper_2410_04349_amd/build.py")
    # torch bundles its own HIP runtime under the same soname as the system
    # one libhb links against; loading torch first makes the process use a
    # single runtime whichever module the caller imports first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    sig = {
        "hb_create": (I32, [ctypes.POINTER(P), ctypes.c_int, ALLOC_FN, FREE_FN, P, P]),
        "hb_destroy": (None, [P]),
        "hb_last_error": (ctypes.c_char_p, [P]),
        "hb_version": (ctypes.c_char_p, []),
        "hb_load_relation": (I32, [P, U32, U32, ctypes.POINTER(HbColumn), ctypes.c_int, ctypes.POINTER(U32)]),
        "hb_load_relation_async": (I32, [P, U32, U32, ctypes.POINTER(HbColumn), ctypes.c_int, ctypes.POINTER(U32)]),
        "hb_release_relation": (I32, [P, U32]),
        "hb_compile_rules": (I32, [P, U32, U32, ctypes.POINTER(HbRule), ctypes.POINTER(U32)]),
        "hb_partition": (I32, [P, U32, U32, ctypes.POINTER(U64)]),
        "hb_match": (I32, [P, U32, U32, I32, P, ctypes.c_int, U64, ctypes.POINTER(U64)]),
        "hb_match_noalloc": (I32, [P, U32, U32, I32, P, U64, ctypes.POINTER(U64)]),
        "hb_set_rows_per_wave": (I32, [P, U32]),
        "hb_set_sparse_rows": (I32, [P, U32]),
        "hb_set_pack_small_blocks": (I32, [P, ctypes.c_int]),
        "hb_set_learned_min_saving": (I32, [P, ctypes.c_float]),
        "hb_ruleset_estimates": (I32, [P, U32, P, P, U32, ctypes.POINTER(U32)]),
        "hb_ruleset_buckets": (I32, [P, U32, U32, P, ctypes.POINTER(U64)]),
        "hb_epg_path": (I32, [U32, P, P, U32, P, P, P, P, ctypes.POINTER(U32)]),
        "hb_plan_path": (I32, [U32, U32, P, P, U32, P, P, P, P, ctypes.POINTER(U32)]),
        "hb_profile_enable": (I32, [P, ctypes.c_int]),
        "hb_profile_query": (I32, [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U64)]),
        "hb_profile_bytes": (I32, [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]),
        "hb_profile_reset": (I32, [P]),
        "hb_last_match_stats": (I32, [P, ctypes.POINTER(HbMatchStats)]),
        "hb_match_work": (I32, [P, U32, U32, I32, ctypes.POINTER(HbWorkStats)]),
        "hb_costmodel_init": (I32, [P, U64]),
        "hb_costmodel_set_params": (I32, [P, P, U32]),
        "hb_costmodel_get_params": (I32, [P, P, U32]),
        "hb_costmodel_train": (I32, [P, P, P, U64, ctypes.c_int, U32, U32, ctypes.c_float,
                                     ctypes.POINTER(ctypes.c_float)]),
        "hb_costmodel_predict": (I32, [P, P, U64, ctypes.c_int, P, ctypes.c_int]),
        "hb_costmodel_trace": (I32, [P, P, P, U32, P, U64]),
        "hb_costmodel_adam_step": (I32, [P, P, ctypes.c_float]),
        "hb_costmodel_save": (I32, [P, ctypes.c_char_p]),
        "hb_costmodel_load": (I32, [P, ctypes.c_char_p]),
        "hb_log_collect": (I32, [P, U32, U32, U32, U64, P, P, P, P, U64, ctypes.POINTER(U64)]),
        "hb_pair_log_collect": (I32, [P, U32, U32, U32, U64, P, P, P, U64, ctypes.POINTER(U64)]),
        "hb_costmodel_select": (I32, [P, I32]),
        "hb_set_cost_estimate": (I32, [P, I32, U32, U64]),
        "hb_batch_create": (I32, [P, ctypes.POINTER(HbJob), U32, I32, U32, ctypes.POINTER(U32)]),
        "hb_batch_run": (I32, [P, U32, ctypes.POINTER(U64)]),
        "hb_batch_result": (I32, [P, U32, U32, P, ctypes.c_int, U64, ctypes.POINTER(U64)]),
        "hb_batch_info_get": (I32, [P, U32, ctypes.POINTER(HbBatchInfo)]),
        "hb_batch_destroy": (I32, [P, U32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load_lib()


class HbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hb status {status}: {message}")
        self.status = status
        self.message = message


def _ptr(a) -> Optional[int]:
    """Address of a numpy array or a torch tensor (None passes through)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


class Context:
    """An hb_ctx on one device; device memory comes from torch's caching
    allocator (allocator='torch') or hipMallocAsync (allocator='hip')."""

    def __init__(self, device: int = 0, allocator: str = "torch", stream=None):
        self.device = device
        self._held = {}
        self.alloc_calls = 0   # device allocations the library asked for
        self._alloc_cb = ALLOC_FN(0)
        self._free_cb = FREE_FN(0)
        if allocator == "torch":
            import torch

            def _alloc(nbytes, user):
                self.alloc_calls += 1
                try:
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
                except RuntimeError:
                    return None
                p = t.data_ptr()
                self._held[p] = t
                return p

            def _free(p, user):
                self._held.pop(p, None)

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
        if stream is None and allocator == "torch":
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        st = _lib.hb_create(ctypes.byref(h), device, self._alloc_cb, self._free_cb, None,
                            ctypes.c_void_p(stream) if stream else None)
        if st != HB_OK:
            raise HbError(st, "hb_create failed")
        self.h = h

    def check(self, st: int):
        if st != HB_OK:
            raise HbError(st, _lib.hb_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            _lib.hb_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hb_create(device: int = 0, allocator: str = "torch", stream=None) -> Context:
    return Context(device, allocator, stream)


def hb_destroy(ctx: Context) -> None:
    ctx.close()


def hb_version() -> str:
    return _lib.hb_version().decode()


def hb_last_error(ctx: Context) -> str:
    return _lib.hb_last_error(ctx.h).decode()


def _columns(columns):
    arr = (HbColumn * len(columns))()
    for k, c in enumerate(columns):
        data = getattr(c, "data", None)
        if data is not None and len(data) == 0:
            data = None
        arr[k] = HbColumn(_COLTYPE[c.type], _ptr(c.offsets), _ptr(data), _ptr(c.values), _ptr(c.valid))
    return arr


def hb_load_relation(ctx: Context, columns: Sequence, n_rows: int, on_device: bool = False) -> int:
    """columns: objects with .type ('string'|'categorical'|'int64') and
    .offsets/.data (strings), .values (others), .valid (optional bitmap);
    numpy arrays for host input, torch device tensors for device input."""
    rid = ctypes.c_uint32()
    ctx.check(_lib.hb_load_relation(ctx.h, n_rows, len(columns), _columns(columns), int(on_device),
                                    ctypes.byref(rid)))
    return rid.value


def hb_load_relation_async(ctx: Context, columns: Sequence, n_rows: int, on_device: bool = False) -> int:
    """As hb_load_relation, returning once the copies are queued on the
    context's copy stream; the arrays must stay alive and unchanged until
    the relation's first use (pinned host memory for an asynchronous copy)."""
    rid = ctypes.c_uint32()
    ctx.check(_lib.hb_load_relation_async(ctx.h, n_rows, len(columns), _columns(columns), int(on_device),
                                          ctypes.byref(rid)))
    return rid.value


def hb_release_relation(ctx: Context, rel_id: int) -> None:
    ctx.check(_lib.hb_release_relation(ctx.h, rel_id))


def _c_rules(rules):
    keep = []
    crules = (HbRule * len(rules))()
    for r, rule in enumerate(rules):
        preds = (HbPred * max(1, len(rule)))()
        for x, p in enumerate(rule):
            preds[x] = HbPred(_OP[p.op], p.attr, p.k, p.q, p.num, p.den, p.d, getattr(p, "attr_b", 0),
                              getattr(p, "side", 0), getattr(p, "c", 0))
        keep.append(preds)
        crules[r] = HbRule(len(rule), ctypes.cast(preds, ctypes.POINTER(HbPred)))
    return crules, keep


def hb_compile_rules(ctx: Context, rel_id: int, rules) -> int:
    """rules: list of rules, each a list of predicates with fields
    op ('eq'|'ed'|'jaccard'|'absdiff'|'eq_const'|'eq_cross'|'ed_cross'),
    attr, k, q, num, den, d, attr_b (t.A = s.B, t.A ~ s.B), side and c
    (t.A = c: side 0; s.A = c: side 1)."""
    crules, keep = _c_rules(rules)
    rs = ctypes.c_uint32()
    ctx.check(_lib.hb_compile_rules(ctx.h, rel_id, len(rules), crules, ctypes.byref(rs)))
    return rs.value


def hb_partition(ctx: Context, rel_id: int, ruleset_id: int) -> int:
    n = ctypes.c_uint64()
    ctx.check(_lib.hb_partition(ctx.h, rel_id, ruleset_id, ctypes.byref(n)))
    return n.value


def hb_match(ctx: Context, rel_id: int, ruleset_id: int, plan="heuristic", out=None, capacity: int = None):
    """Ca(D) as sorted packed uint64 (i << 32) | j.  With out=None a host
    numpy array is returned (sized by the capacity protocol); with a torch
    device tensor `out` (uint64/int64) the pairs are written there and the
    count is returned."""
    pl = _PLAN[plan] if isinstance(plan, str) else int(plan)
    n = ctypes.c_uint64()
    if out is not None:
        cap = out.numel() if capacity is None else capacity
        ctx.check(_lib.hb_match(ctx.h, rel_id, ruleset_id, pl, ctypes.c_void_p(out.data_ptr()), 1, cap,
                                ctypes.byref(n)))
        return n.value
    st = _lib.hb_match(ctx.h, rel_id, ruleset_id, pl, None, 0, 0, ctypes.byref(n))
    if st == HB_OK:
        return np.zeros(0, dtype=np.uint64)
    if st != HB_ERR_CAPACITY:
        ctx.check(st)
    buf = np.zeros(max(1, n.value), dtype=np.uint64)
    ctx.check(_lib.hb_match(ctx.h, rel_id, ruleset_id, pl, ctypes.c_void_p(buf.ctypes.data), 0, len(buf),
                            ctypes.byref(n)))
    return buf[: n.value]


def hb_match_noalloc(ctx: Context, rel_id: int, ruleset_id: int, plan, out, capacity: int = None) -> int:
    """hb_match into the torch device tensor `out` (uint64/int64) without any
    device allocation (see include/hb.h); returns the pair count."""
    pl = _PLAN[plan] if isinstance(plan, str) else int(plan)
    n = ctypes.c_uint64()
    cap = out.numel() if capacity is None else capacity
    ctx.check(_lib.hb_match_noalloc(ctx.h, rel_id, ruleset_id, pl, ctypes.c_void_p(out.data_ptr()), cap,
                                    ctypes.byref(n)))
    return n.value


def hb_set_rows_per_wave(ctx: Context, rows: int) -> None:
    ctx.check(_lib.hb_set_rows_per_wave(ctx.h, rows))


def hb_set_pack_small_blocks(ctx: Context, on: bool) -> None:
    ctx.check(_lib.hb_set_pack_small_blocks(ctx.h, int(on)))


def hb_set_sparse_rows(ctx: Context, max_rows: int) -> None:
    ctx.check(_lib.hb_set_sparse_rows(ctx.h, max_rows))


def hb_set_learned_min_saving(ctx: Context, min_saving: float) -> None:
    ctx.check(_lib.hb_set_learned_min_saving(ctx.h, min_saving))


def hb_ruleset_estimates(ctx: Context, ruleset_id: int) -> Tuple[np.ndarray, np.ndarray]:
    n = ctypes.c_uint32()
    ctx.check(_lib.hb_ruleset_estimates(ctx.h, ruleset_id, None, None, 0, ctypes.byref(n)))
    sp = np.zeros(n.value, dtype=np.float64)
    cost = np.zeros(n.value, dtype=np.float64)
    ctx.check(_lib.hb_ruleset_estimates(ctx.h, ruleset_id, ctypes.c_void_p(sp.ctypes.data),
                                        ctypes.c_void_p(cost.ctypes.data), n.value, ctypes.byref(n)))
    return sp, cost


def hb_ruleset_buckets(ctx: Context, ruleset_id: int, pred: int) -> Tuple[np.ndarray, int]:
    counts = np.zeros(1024, dtype=np.uint64)
    n = ctypes.c_uint64()
    ctx.check(_lib.hb_ruleset_buckets(ctx.h, ruleset_id, pred, ctypes.c_void_p(counts.ctypes.data),
                                      ctypes.byref(n)))
    return counts, n.value


def hb_epg_path(sp: Sequence[float], cost: Sequence[float], rules: Sequence[Sequence[int]]):
    """Pure host: [(rule, [pred ids])] in sequential-path order."""
    return hb_plan_path("heuristic", sp, cost, rules)


def hb_plan_path(plan, sp: Sequence[float], cost: Sequence[float], rules: Sequence[Sequence[int]]):
    """Pure host: the path of `plan` (any but "learned"): [(rule, [pred ids])]."""
    pl = _PLAN[plan] if isinstance(plan, str) else int(plan)
    sp = np.ascontiguousarray(sp, dtype=np.float64)
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    lens = np.array([len(r) for r in rules], dtype=np.uint32)
    flat = np.array([p for r in rules for p in r], dtype=np.uint32)
    if flat.size == 0:
        flat = np.zeros(1, dtype=np.uint32)
    out_rules = np.zeros(max(1, len(rules)), dtype=np.uint32)
    out_preds = np.zeros(max(1, int(lens.sum())), dtype=np.uint32)
    n = ctypes.c_uint32()
    st = _lib.hb_plan_path(pl, len(sp), ctypes.c_void_p(sp.ctypes.data), ctypes.c_void_p(cost.ctypes.data),
                           len(rules), ctypes.c_void_p(lens.ctypes.data), ctypes.c_void_p(flat.ctypes.data),
                           ctypes.c_void_p(out_rules.ctypes.data), ctypes.c_void_p(out_preds.ctypes.data),
                           ctypes.byref(n))
    if st != HB_OK:
        raise HbError(st, "hb_plan_path failed")
    res = []
    o = 0
    for r in out_rules[: len(rules)]:
        k = len(set(rules[int(r)]))
        res.append((int(r), [int(x) for x in out_preds[o:o + k]]))
        o += k
    return res


def hb_profile_enable(ctx: Context, on: bool = True) -> None:
    ctx.check(_lib.hb_profile_enable(ctx.h, int(on)))


def hb_profile_query(ctx: Context, name: str) -> Tuple[float, int]:
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    ctx.check(_lib.hb_profile_query(ctx.h, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def hb_profile_bytes(ctx: Context, name: str) -> float:
    b = ctypes.c_double()
    ctx.check(_lib.hb_profile_bytes(ctx.h, name.encode(), ctypes.byref(b)))
    return b.value


def hb_profile_reset(ctx: Context) -> None:
    ctx.check(_lib.hb_profile_reset(ctx.h))


def hb_last_match_stats(ctx: Context) -> dict:
    s = HbMatchStats()
    ctx.check(_lib.hb_last_match_stats(ctx.h, ctypes.byref(s)))
    return {"candidate_pairs": s.candidate_pairs, "matched_pairs": s.matched_pairs, "tiles": s.tiles,
            "launches": s.launches, "learned_blocks": s.learned_blocks, "fallback_blocks": s.fallback_blocks,
            "learned_plans": s.learned_plans, "predicted_heuristic": s.predicted_heuristic,
            "predicted_chosen": s.predicted_chosen}


def hb_match_work(ctx: Context, rel_id: int, ruleset_id: int, plan="heuristic") -> dict:
    """Counters of one instrumented evaluation pass (see include/hb.h)."""
    pl = _PLAN[plan] if isinstance(plan, str) else int(plan)
    w = HbWorkStats()
    ctx.check(_lib.hb_match_work(ctx.h, rel_id, ruleset_id, pl, ctypes.byref(w)))
    per_op = {}
    for k, name in enumerate(OP_KINDS):
        per_op[name] = {"waves": w.waves[k], "lanes": w.lanes[k], "passed": w.passed[k], "work": w.work[k]}
    return {"pairs": w.pairs, "matched": w.matched, "launches": w.launches, "lane_ops": w.lane_ops,
            "batch_ops": w.batch_ops, "issued_ops": w.issued_ops, "per_op": per_op}


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def hb_costmodel_init(ctx: Context, seed: int) -> None:
    ctx.check(_lib.hb_costmodel_init(ctx.h, seed))


def hb_costmodel_set_params(ctx: Context, params) -> None:
    p = _f32(params)
    ctx.check(_lib.hb_costmodel_set_params(ctx.h, ctypes.c_void_p(p.ctypes.data), p.size))


def hb_costmodel_get_params(ctx: Context) -> np.ndarray:
    p = np.zeros(HB_MLP_PARAMS, dtype=np.float32)
    ctx.check(_lib.hb_costmodel_get_params(ctx.h, ctypes.c_void_p(p.ctypes.data), p.size))
    return p


def hb_costmodel_train(ctx: Context, x, t, epochs: int, batch: int, lr: float) -> float:
    x, t = _f32(x), _f32(t)
    loss = ctypes.c_float()
    ctx.check(_lib.hb_costmodel_train(ctx.h, ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(t.ctypes.data),
                                      x.shape[0], 0, epochs, batch, lr, ctypes.byref(loss)))
    return loss.value


def hb_costmodel_predict(ctx: Context, x) -> np.ndarray:
    x = _f32(x)
    y = np.zeros((x.shape[0], 2), dtype=np.float32)
    ctx.check(_lib.hb_costmodel_predict(ctx.h, ctypes.c_void_p(x.ctypes.data), x.shape[0], 0,
                                        ctypes.c_void_p(y.ctypes.data), 0))
    return y


def hb_costmodel_trace(ctx: Context, x, t) -> dict:
    x, t = _f32(x), _f32(t)
    n = x.shape[0]
    total = n * (6 * 64 + 4) + HB_MLP_PARAMS
    out = np.zeros(total, dtype=np.float32)
    ctx.check(_lib.hb_costmodel_trace(ctx.h, ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(t.ctypes.data), n,
                                      ctypes.c_void_p(out.ctypes.data), total))
    res = {}
    o = 0
    for name, cols in (("z1", 64), ("h1", 64), ("z2", 64), ("h2", 64), ("y", 2), ("dy", 2), ("dz2", 64),
                       ("dz1", 64)):
        res[name] = out[o:o + n * cols].reshape(n, cols)
        o += n * cols
    res["grad"] = out[o:o + HB_MLP_PARAMS]
    return res


def hb_costmodel_adam_step(ctx: Context, grads, lr: float) -> None:
    g = _f32(grads)
    ctx.check(_lib.hb_costmodel_adam_step(ctx.h, ctypes.c_void_p(g.ctypes.data), lr))


def hb_costmodel_save(ctx: Context, path: str) -> None:
    ctx.check(_lib.hb_costmodel_save(ctx.h, os.fsencode(path)))


def hb_costmodel_load(ctx: Context, path: str) -> None:
    ctx.check(_lib.hb_costmodel_load(ctx.h, os.fsencode(path)))


def hb_costmodel_select(ctx: Context, which) -> None:
    """"block" (the learned plan's model) or "pair" (the per-pair network of
    the estimated cost): the model the hb_costmodel_* calls act on."""
    ctx.check(_lib.hb_costmodel_select(ctx.h, _MODEL[which] if isinstance(which, str) else int(which)))


def hb_set_cost_estimate(ctx: Context, source, samples: int = 1024, seed: int = 0x48425041) -> None:
    """"static" or "pair_net": where hb_compile_rules takes predicate costs."""
    ctx.check(_lib.hb_set_cost_estimate(ctx.h, _COST[source] if isinstance(source, str) else int(source),
                                        samples, seed))


def hb_pair_log_collect(ctx: Context, rel_id: int, ruleset_id: int, samples: int, seed: int) -> dict:
    """Per-pair logging pass (see include/hb.h): features [n x 16], labels
    [n x 2] (satisfied, log2(1 + cycles) / 16), rows predicate-major, and
    pairs [samples x 2] (i, j)."""
    n = ctypes.c_uint64()
    st = _lib.hb_pair_log_collect(ctx.h, rel_id, ruleset_id, samples, seed, None, None, None, 0, ctypes.byref(n))
    if st not in (HB_OK, HB_ERR_CAPACITY):
        ctx.check(st)
    rows = n.value
    f = np.zeros((max(rows, 1), 16), dtype=np.float32)
    lab = np.zeros((max(rows, 1), 2), dtype=np.float32)
    pairs = np.zeros((max(samples, 1), 2), dtype=np.uint32)
    ctx.check(_lib.hb_pair_log_collect(ctx.h, rel_id, ruleset_id, samples, seed, ctypes.c_void_p(f.ctypes.data),
                                       ctypes.c_void_p(lab.ctypes.data), ctypes.c_void_p(pairs.ctypes.data), rows,
                                       ctypes.byref(n)))
    return {"features": f[:rows], "labels": lab[:rows], "pairs": pairs[:samples] if rows else pairs[:0]}


def hb_log_collect(ctx: Context, rel_id: int, ruleset_id: int, samples: int, seed: int) -> dict:
    """Logging pass (see include/hb.h): features [n x 16], labels [n x 2],
    meta [n x 3] (key index, block, predicate id), counts [n x 4] (pairs
    sampled, pairs satisfying, cycles, pairs passing the first step)."""
    n = ctypes.c_uint64()
    st = _lib.hb_log_collect(ctx.h, rel_id, ruleset_id, samples, seed, None, None, None, None, 0, ctypes.byref(n))
    if st not in (HB_OK, HB_ERR_CAPACITY):
        ctx.check(st)
    rows = n.value
    f = np.zeros((max(rows, 1), 16), dtype=np.float32)
    lab = np.zeros((max(rows, 1), 2), dtype=np.float32)
    meta = np.zeros((max(rows, 1), 3), dtype=np.uint32)
    cnt = np.zeros((max(rows, 1), 4), dtype=np.uint64)
    ctx.check(_lib.hb_log_collect(ctx.h, rel_id, ruleset_id, samples, seed, ctypes.c_void_p(f.ctypes.data),
                                  ctypes.c_void_p(lab.ctypes.data), ctypes.c_void_p(meta.ctypes.data),
                                  ctypes.c_void_p(cnt.ctypes.data), rows, ctypes.byref(n)))
    return {"features": f[:rows], "labels": lab[:rows], "meta": meta[:rows], "counts": cnt[:rows]}


# ------------------------------------------------------------ batches

def hb_batch_create(ctx: Context, jobs, plan="heuristic", graph: bool = True, autotune: bool = False,
                    form=None) -> int:
    """jobs: sequence of (rel_id, ruleset_id), each partitioned; form: None
    (tuned or remembered), "streams", "multi" or "persistent"."""
    arr = (HbJob * max(1, len(jobs)))(*[HbJob(int(r), int(s)) for r, s in jobs])
    pl = _PLAN[plan] if isinstance(plan, str) else int(plan)
    flags = (HB_BATCH_GRAPH if graph else 0) | (HB_BATCH_AUTOTUNE if autotune else 0)
    if form is not None:
        flags |= HB_BATCH_FORM[form]
    bid = ctypes.c_uint32()
    ctx.check(_lib.hb_batch_create(ctx.h, arr, len(jobs), pl, flags, ctypes.byref(bid)))
    return bid.value


def hb_batch_run(ctx: Context, batch_id: int) -> int:
    n = ctypes.c_uint64()
    ctx.check(_lib.hb_batch_run(ctx.h, batch_id, ctypes.byref(n)))
    return n.value


def hb_batch_result(ctx: Context, batch_id: int, job: int, out=None):
    """Job `job`'s sorted packed pairs: a host numpy array, or written into
    the torch device tensor `out` (count returned)."""
    n = ctypes.c_uint64()
    if out is not None:
        ctx.check(_lib.hb_batch_result(ctx.h, batch_id, job, ctypes.c_void_p(out.data_ptr()), 1, out.numel(),
                                       ctypes.byref(n)))
        return n.value
    st = _lib.hb_batch_result(ctx.h, batch_id, job, None, 0, 0, ctypes.byref(n))
    if st == HB_OK:
        return np.zeros(0, dtype=np.uint64)
    if st != HB_ERR_CAPACITY:
        ctx.check(st)
    buf = np.zeros(max(1, n.value), dtype=np.uint64)
    ctx.check(_lib.hb_batch_result(ctx.h, batch_id, job, ctypes.c_void_p(buf.ctypes.data), 0, len(buf),
                                   ctypes.byref(n)))
    return buf[: n.value]


def hb_batch_info(ctx: Context, batch_id: int) -> dict:
    i = HbBatchInfo()
    ctx.check(_lib.hb_batch_info_get(ctx.h, batch_id, ctypes.byref(i)))
    return {"n_jobs": i.n_jobs, "n_partitions": i.n_partitions, "work_items": i.work_items,
            "form": ["streams", "multi", "persistent"][i.form], "grid": i.grid,
            "grab": i.grab, "occupancy": i.occupancy, "lds_bytes": i.lds_bytes, "graph": bool(i.graph),
            "tune_ms": list(i.tune_ms[: i.n_tuned]), "fallback_blocks": i.fallback_blocks}


def hb_batch_destroy(ctx: Context, batch_id: int) -> None:
    ctx.check(_lib.hb_batch_destroy(ctx.h, batch_id))
