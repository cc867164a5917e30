"""Python binding of libhtri (ctypes).  Argument marshalling only: every
step of the computation runs in the HIP library.  PyTorch provides device
memory (through the allocator callback) and the stream.

Names follow the C ABI in include/htri.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtri.so")

HTRI_OK = 0
HTRI_DEDUPE_EDGES = 1
HTRI_INPUT_ON_DEVICE = 2
HTRI_OUTPUT_ON_DEVICE = 4
HTRI_ORDER_INPUT = 8
HTRI_WIDE_TILE_KEYS = 256
HTRI_COUNT_NO_WINDOW = 16
HTRI_COUNT_WINDOW_ALWAYS = 32
HTRI_COUNT_INCLUSION_CLASSES = 64
HTRI_COUNT_OWNER_PROBE = 128
HTRI_COUNT_DENSE_TTT = 512
HTRI_COUNT_COMMON_VERTEX = 1024
HTRI_COUNT_SPARSE_TTT = 2048
HTRI_SAMPLE_EXACT_INCLUSION = 1
HTRI_IMPORTANCE_TOTAL = 1
_WINDOW_FLAGS = {"auto": 0, "off": HTRI_COUNT_NO_WINDOW, "always": HTRI_COUNT_WINDOW_ALWAYS,
                 "inclusion_classes": HTRI_COUNT_INCLUSION_CLASSES, "dense_ttt": HTRI_COUNT_DENSE_TTT,
                 "common_vertex": HTRI_COUNT_COMMON_VERTEX, "sparse_ttt": HTRI_COUNT_SPARSE_TTT}
HTRI_MODEL_NUM_PARAMS = 5313
ALL_PATTERNS = 0x1FFFFE

STATUS = {0: "HTRI_OK", -1: "HTRI_E_INVALID", -2: "HTRI_E_RANGE", -3: "HTRI_E_EMPTY_EDGE",
          -4: "HTRI_E_DUPLICATE_EDGE", -5: "HTRI_E_OOM", -6: "HTRI_E_DEVICE", -7: "HTRI_E_OVERFLOW",
          -8: "HTRI_E_STATE", -9: "HTRI_E_UNSUPPORTED"}


class HtriError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        super().__init__(f"{where}: {STATUS.get(code, code)}" + (f" ({msg})" if msg else ""))
        self.code = code


_P = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class SampleParams(ctypes.Structure):
    _fields_ = [("budget_fraction", ctypes.c_double), ("num_samples", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("proposal", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("defensive_mix", ctypes.c_double),
                ("pool_factor", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("partners", ctypes.c_int32), ("order", ctypes.c_int32)]

    def as_tuple(self):
        return (int(self.chunk), int(self.partners), int(self.order))


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libhtri.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                          "(python -m paper_2504_02271_amd.build) first")
    # torch supplies device memory and streams; load its HIP runtime first so
    # that the library binds to the same one
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "htri_graph_load": ([_P, _i64, _P, _i32, _u32, _P, _P, ctypes.POINTER(_P)], ctypes.c_int),
        "htri_graph_info": ([_P, _P], ctypes.c_int),
        "htri_graph_edge_map": ([_P, _P], ctypes.c_int),
        "htri_graph_csr": ([_P, _P, _P], ctypes.c_int),
        "htri_build_wedges": ([_P, _P], ctypes.c_int),
        "htri_get_wedges": ([_P, _P, _P, _P], ctypes.c_int),
        "htri_count_patterns": ([_P, _u32, _P, _P, _P, _u32], ctypes.c_int),
        "htri_last_timings": ([_P, _P], ctypes.c_int),
        "htri_clear_wedges": ([_P], ctypes.c_int),
        "htri_closure_stats": ([_P, _P], ctypes.c_int),
        "htri_enumerate": ([_P, _i32, _i64, _P, _P, _u32], ctypes.c_int),
        "htri_clustering_coefficient": ([_P, _i64, _P, _P], ctypes.c_int),
        "htri_get_wedge_list": ([_P, _P, _i64, _P, _P, _P], ctypes.c_int),
        "htri_count_per_edge_patterns": ([_P, _P, _P, _u32], ctypes.c_int),
        "htri_local_clustering": ([_P, _P, _P, _u32], ctypes.c_int),
        "htri_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "htri_last_error": ([_P], ctypes.c_char_p),
        "htri_graph_free": ([_P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _optional = {
        "htri_estimate": ([_P, ctypes.POINTER(SampleParams), _P, _P, _P], ctypes.c_int),
        "htri_subgraph": ([_P, ctypes.c_double, _u64, _i32, ctypes.POINTER(_P), _P, _P, _P], ctypes.c_int),
        "htri_close_wedges": ([_P, _P, _i64, _P], ctypes.c_int),
        "htri_wedge_features": ([_P, _P], ctypes.c_int),
        "htri_proposal_scores": ([_P, _P, _P, _i64, _P], ctypes.c_int),
        "htri_wedge_importance": ([_P, _P, _u32, _P], ctypes.c_int),
        "htri_estimate_uniform_noalloc": ([_P, _i64, _u64, _P, _P], ctypes.c_int),
        "htri_adv_split": ([_i64, _i64, _i64, _P], ctypes.c_int),
        "htri_model_save": ([_P, ctypes.c_char_p], ctypes.c_int),
        "htri_model_load": ([_P, ctypes.c_char_p], ctypes.c_int),
        "htri_model_last_error": ([_P], ctypes.c_char_p),
        "htri_model_create": ([_u64, _P, ctypes.POINTER(_P)], ctypes.c_int),
        "htri_model_free": ([_P], None),
        "htri_model_get_params": ([_P, _P], ctypes.c_int),
        "htri_model_set_params": ([_P, _P], ctypes.c_int),
        "htri_model_forward": ([_P, _P, _i64, _P], ctypes.c_int),
        "htri_model_loss_grad": ([_P, _P, _P, _i64, _P, _P], ctypes.c_int),
        "htri_model_train": ([_P, _P, _P, _i64, _i32, _i32, ctypes.c_float, _u64, _P], ctypes.c_int),
        "htri_batch_load": ([_i32, _P, _P, _P, _P, _u32, ctypes.POINTER(_P)], ctypes.c_int),
        "htri_batch_info": ([_P, _P], ctypes.c_int),
        "htri_batch_count": ([_P, ctypes.POINTER(Schedule), _i32, _P, _P], ctypes.c_int),
        "htri_batch_autotune": ([_P, _i32, ctypes.POINTER(Schedule), _P], ctypes.c_int),
        "htri_batch_count_per_graph": ([_P, ctypes.POINTER(Schedule), _P, _P], ctypes.c_int),
        "htri_batch_count_full": ([_P, ctypes.POINTER(Schedule), _P, _P], ctypes.c_int),
        "htri_batch_size_classes": ([_P, _P], ctypes.c_int),
        "htri_batch_autotune_classes": ([_P, _i32, ctypes.c_char_p, _P, _P, _P], ctypes.c_int),
        "htri_batch_count_classes": ([_P, _P, _i32, _P, _P], ctypes.c_int),
        "htri_batch_count_full_per_graph": ([_P, ctypes.POINTER(Schedule), _P, _P], ctypes.c_int),
        "htri_batch_last_error": ([_P], ctypes.c_char_p),
        "htri_batch_free": ([_P], None),
    }
    for name, (args, res) in _optional.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, where: str, handle=None):
    if rc != HTRI_OK:
        msg = load_library().htri_last_error(handle)
        raise HtriError(rc, where, msg.decode() if msg else "")


# ---------------------------------------------------------------- torch glue

class TorchMemory:
    """Device memory from torch's caching allocator, handed to the library
    through the htri_allocator callbacks; the stream is torch's current one."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        alloc_fn = torch.cuda.caching_allocator_alloc
        delete_fn = torch.cuda.caching_allocator_delete

        def _alloc(nbytes, stream, ctx):
            try:
                return alloc_fn(int(nbytes), device, stream)
            except Exception:
                return None

        def _free(ptr, stream, ctx):
            # may run during interpreter shutdown, after torch is torn down
            try:
                if ptr:
                    delete_fn(ptr)
            except Exception:
                pass

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = Allocator(self._alloc_cb, self._free_cb, None)

    def stream_handle(self) -> int:
        return int(self.torch.cuda.current_stream(self.device).cuda_stream)


_default_mem: Optional[TorchMemory] = None


def default_memory() -> TorchMemory:
    global _default_mem
    if _default_mem is None:
        _default_mem = TorchMemory(0)
    return _default_mem


# ---------------------------------------------------------------- graph

class Graph:
    """A hypergraph resident on the GPU (htri_graph)."""

    def __init__(self, handle, mem: Optional[TorchMemory]):
        self._h = handle
        self._mem = mem            # keeps the allocator callbacks alive
        self._lib = load_library()
        info = np.zeros(4, np.int64)
        _check(self._lib.htri_graph_info(self._h, _ptr(info)), "htri_graph_info", self._h)
        self.num_edges, self.removed, self.nnz, self.num_vertices = (int(x) for x in info)
        self.summary: Optional[np.ndarray] = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.htri_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def edge_map(self) -> np.ndarray:
        out = np.zeros(self.num_edges, np.int64)
        _check(self._lib.htri_graph_edge_map(self._h, _ptr(out)), "htri_graph_edge_map", self._h)
        return out

    def csr(self) -> Tuple[np.ndarray, np.ndarray]:
        off = np.zeros(self.num_edges + 1, np.int64)
        mem = np.zeros(self.nnz, np.int32)
        _check(self._lib.htri_graph_csr(self._h, _ptr(off), _ptr(mem)), "htri_graph_csr", self._h)
        return off, mem

    def build_wedges(self) -> np.ndarray:
        s = np.zeros(6, np.int64)
        _check(self._lib.htri_build_wedges(self._h, _ptr(s)), "htri_build_wedges", self._h)
        self.summary = s
        return s

    @property
    def num_wedges(self) -> int:
        if self.summary is None:
            self.build_wedges()
        return int(self.summary[0])

    def get_wedges(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        nw = self.num_wedges
        src = np.zeros(nw, np.int32)
        dst = np.zeros(nw, np.int32)
        om = np.zeros(nw, np.int32)
        _check(self._lib.htri_get_wedges(self._h, _ptr(src), _ptr(dst), _ptr(om)), "htri_get_wedges", self._h)
        return src, dst, om

    def subgraph(self, sigma: float, seed: int = 0, fixed_size: bool = False):
        """Sub-hypergraph for sigma-sampling: (Graph, kept normalised ids
        ascending, triangle scale).  fixed_size: exactly round(sigma*m)
        hyperedges, else each kept with probability sigma.  Counts or
        estimates on the subgraph times the scale are unbiased here."""
        kept = np.zeros(max(self.num_edges, 1), np.int32)
        n = ctypes.c_int64(0)
        scale = ctypes.c_double(0.0)
        h = ctypes.c_void_p()
        _check(self._lib.htri_subgraph(self._h, float(sigma), int(seed) & (2**64 - 1), 1 if fixed_size else 0,
                                       ctypes.byref(h), _ptr(kept), ctypes.byref(n), ctypes.byref(scale)),
               "htri_subgraph", self._h)
        return Graph(h, self._mem), kept[: n.value].copy(), float(scale.value)

    def get_wedge_list(self, idx) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(src, dst, omega) of the listed hyperwedges (indices in get_wedges order)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        n = idx.shape[0]
        src = np.zeros(n, np.int32)
        dst = np.zeros(n, np.int32)
        om = np.zeros(n, np.int32)
        _check(self._lib.htri_get_wedge_list(self._h, _ptr(idx), n, _ptr(src), _ptr(dst), _ptr(om)),
               "htri_get_wedge_list", self._h)
        return src, dst, om

    def count_patterns(self, mask: int = 0, per_edge: bool = False, per_wedge: bool = False,
                       device_out: bool = False, window: str = "auto", probe: str = "middle"):
        """Returns (counts int64[21], per_edge or None, per_wedge or None).
        With device_out the per-edge/per-wedge results are torch tensors on the GPU.
        window: "auto" (dense top-rank window when it pays), "off", "always", or
        "inclusion_classes" (patterns 1-8 only, searched around the inclusion
        hyperwedges; no per_wedge).
        probe: "middle" (each hyperwedge (r, j) probes the rest of N+(r)
        against N+(j); the library falls back to "owner" when its lists do
        not fit) or "owner" (each partner's N+(j) against N+(r))."""
        counts = np.zeros(21, np.int64)
        pe = pw = None
        if probe not in ("middle", "owner"):
            raise ValueError(f"probe must be 'middle' or 'owner', not {probe!r}")
        flags = _WINDOW_FLAGS[window] | (HTRI_COUNT_OWNER_PROBE if probe == "owner" else 0)
        if device_out:
            import torch
            flags |= HTRI_OUTPUT_ON_DEVICE
            if per_edge:
                pe = torch.empty(self.num_edges, dtype=torch.int64, device="cuda")
            if per_wedge:
                pw = torch.empty(self.num_wedges, dtype=torch.int32, device="cuda")
            pe_p = pe.data_ptr() if pe is not None else None
            pw_p = pw.data_ptr() if pw is not None else None
        else:
            if per_edge:
                pe = np.zeros(self.num_edges, np.int64)
            if per_wedge:
                pw = np.zeros(self.num_wedges, np.int32)
            pe_p = _ptr(pe)
            pw_p = _ptr(pw)
        _check(self._lib.htri_count_patterns(self._h, mask, _ptr(counts), pe_p, pw_p, flags),
               "htri_count_patterns", self._h)
        return counts, pe, pw

    def count_per_edge_patterns(self, device_out: bool = False):
        """(counts int64[21], per-hyperedge per-pattern counts int64[m, 21]);
        device_out: the per-hyperedge counts as a torch tensor on the GPU."""
        counts = np.zeros(21, np.int64)
        if device_out:
            import torch
            out = torch.empty((max(self.num_edges, 1), 21), dtype=torch.int64, device="cuda")
            _check(self._lib.htri_count_per_edge_patterns(self._h, _ptr(counts), out.data_ptr(),
                                                          HTRI_OUTPUT_ON_DEVICE),
                   "htri_count_per_edge_patterns", self._h)
            return counts, out[: self.num_edges]
        out = np.zeros((max(self.num_edges, 1), 21), np.int64)
        _check(self._lib.htri_count_per_edge_patterns(self._h, _ptr(counts), _ptr(out), 0),
               "htri_count_per_edge_patterns", self._h)
        return counts, out[: self.num_edges]

    def local_clustering(self, epsilon=None) -> np.ndarray:
        """Local clustering coefficient of every hyperedge (float64[m])."""
        e = None if epsilon is None else np.ascontiguousarray(epsilon, dtype=np.float64)
        if e is not None and e.shape != (21,):
            raise ValueError("epsilon holds 21 weights (index 0 unused)")
        out = np.zeros(max(self.num_edges, 1), np.float64)
        _check(self._lib.htri_local_clustering(self._h, _ptr(e), _ptr(out), 0), "htri_local_clustering", self._h)
        return out[: self.num_edges]

    def enumerate(self, pattern: int, capacity: int = 1 << 20):
        """(triples int32 [min(found, capacity), 3] of normalised ids, found)."""
        capacity = int(capacity)
        out = np.zeros((max(capacity, 1), 3), np.int32)
        found = ctypes.c_int64(0)
        _check(self._lib.htri_enumerate(self._h, int(pattern), capacity, _ptr(out), ctypes.byref(found), 0),
               "htri_enumerate", self._h)
        return out[: min(found.value, capacity)], int(found.value)

    def clear_wedges(self) -> None:
        _check(self._lib.htri_clear_wedges(self._h), "htri_clear_wedges", self._h)
        self.summary = None

    def closure_stats(self) -> np.ndarray:
        """[S, probed entries, work items, Omega mask words, closure blocks,
        window rows, window wedges, S outside the window, wedges outside,
        mask words outside, window bitmap words read, window hits enumerated,
        middle-centric probing (1/0), in-list hyperwedges, in-list mask
        words, hashed entries staged]"""
        out = np.zeros(16, np.int64)
        _check(self._lib.htri_closure_stats(self._h, _ptr(out)), "htri_closure_stats", self._h)
        return out

    def estimate(self, budget: float = 0.01, num_samples: int = 0, seed: int = 0, proposal: int = 0,
                 model: "Optional[Model]" = None, defensive_mix: float = 0.1, pool_factor: float = 0.0,
                 exact_inclusion: bool = False):
        """Hyperwedge-sampling estimate: (est float64[21], stderr float64[21], device ms).
        exact_inclusion: close every inclusion hyperwedge exactly, sample the rest."""
        p = SampleParams(float(budget), int(num_samples), int(seed) & 0xFFFFFFFFFFFFFFFF, int(proposal),
                         HTRI_SAMPLE_EXACT_INCLUSION if exact_inclusion else 0,
                         model._h if model is not None else None, float(defensive_mix), float(pool_factor))
        est = np.zeros(21, np.float64)
        se = np.zeros(21, np.float64)
        ms = ctypes.c_double(0.0)
        _check(self._lib.htri_estimate(self._h, ctypes.byref(p), _ptr(est), _ptr(se), ctypes.byref(ms)),
               "htri_estimate", self._h)
        return est, se, float(ms.value)

    def estimate_uniform_noalloc(self, num_samples: int, seed: int = 0, est=None, stderr=None):
        """The uniform estimate computed without device allocation by the
        library, into caller tensors (float64[21] on the GPU; created here
        when not given).  Only enqueued on the handle's stream."""
        import torch
        if est is None:
            est = torch.zeros(21, dtype=torch.float64, device="cuda")
        if stderr is None:
            stderr = torch.zeros(21, dtype=torch.float64, device="cuda")
        _check(self._lib.htri_estimate_uniform_noalloc(self._h, int(num_samples), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                       ctypes.c_void_p(est.data_ptr()),
                                                       ctypes.c_void_p(stderr.data_ptr())),
               "htri_estimate_uniform_noalloc", self._h)
        return est, stderr

    def close_wedges(self, idx) -> np.ndarray:
        """Per-pattern closure counts int64[n, 21] of the listed wedges (get_wedges order)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros((idx.shape[0], 21), np.int64)
        _check(self._lib.htri_close_wedges(self._h, _ptr(idx), idx.shape[0], _ptr(out)),
               "htri_close_wedges", self._h)
        return out

    def proposal_scores(self, model: "Model", idx=None) -> np.ndarray:
        """float64 score of the learned proposal for the listed hyperwedges
        (get_wedges order; None = every hyperwedge)."""
        if idx is None:
            n = self.num_wedges
            idx_p = None
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            n = idx.shape[0]
            idx_p = _ptr(idx)
        out = np.zeros(max(n, 1), np.float64)
        _check(self._lib.htri_proposal_scores(self._h, model._h, idx_p, n, _ptr(out)),
               "htri_proposal_scores", self._h)
        return out[:n]

    def wedge_importance(self, counts, with_total: bool = False):
        """The learned proposal's training target log1p(u(w)) of every
        hyperwedge: float32 [|wedges|] torch tensor on the GPU."""
        import torch
        c = np.ascontiguousarray(counts, dtype=np.int64)
        out = torch.empty(max(self.num_wedges, 1), dtype=torch.float32, device="cuda")
        if self.num_wedges:
            _check(self._lib.htri_wedge_importance(self._h, _ptr(c), HTRI_IMPORTANCE_TOTAL if with_total else 0,
                                                   ctypes.c_void_p(out.data_ptr())), "htri_wedge_importance", self._h)
        return out[: self.num_wedges]

    def wedge_features(self):
        """float32 [|wedges|, 16] torch tensor on the GPU."""
        import torch
        x = torch.empty((max(self.num_wedges, 1), 16), dtype=torch.float32, device="cuda")
        if self.num_wedges:
            _check(self._lib.htri_wedge_features(self._h, ctypes.c_void_p(x.data_ptr())),
                   "htri_wedge_features", self._h)
        return x[: self.num_wedges]

    def last_timings(self) -> np.ndarray:
        """ms: [wedges, schedule, closure, reduce, window part, probing part]"""
        ms = np.zeros(6, np.float64)
        _check(self._lib.htri_last_timings(self._h, _ptr(ms)), "htri_last_timings", self._h)
        return ms


def adv_split(n_inter: int, n_incl: int, alpha: int) -> np.ndarray:
    """Appro-adv's draws per class: [alpha1 (TTT), alpha2 (CCC), alpha3 (TTC), alpha4 (TCC)]."""
    out = np.zeros(4, np.int64)
    _check(load_library().htri_adv_split(int(n_inter), int(n_incl), int(alpha), _ptr(out)), "htri_adv_split")
    return out


def clustering_coefficient(counts, connected_triples: int, epsilon=None) -> float:
    """Def. 5.1 from per-pattern counts (int64[21]) and W (summary[3]);
    epsilon: None (all 1) or 21 weights in [0, 1] (index 0 unused)."""
    lib = load_library()
    c = np.ascontiguousarray(counts, dtype=np.int64)
    e = None if epsilon is None else np.ascontiguousarray(epsilon, dtype=np.float64)
    if c.shape != (21,) or (e is not None and e.shape != (21,)):
        raise ValueError("counts and epsilon hold 21 entries")
    out = ctypes.c_double(0.0)
    _check(lib.htri_clustering_coefficient(_ptr(c), int(connected_triples), _ptr(e), ctypes.byref(out)),
           "htri_clustering_coefficient")
    return float(out.value)


def graph_load(offsets, members, num_vertices: int, flags: int = HTRI_DEDUPE_EDGES,
               mem: Optional[TorchMemory] = None, use_torch: bool = True) -> Graph:
    """Load a hypergraph (host numpy arrays, or torch CUDA tensors with
    HTRI_INPUT_ON_DEVICE) and normalise it on the GPU."""
    lib = load_library()
    if use_torch and mem is None:
        mem = default_memory()
    stream = mem.stream_handle() if mem is not None else None
    alloc = ctypes.byref(mem.struct) if mem is not None else None
    h = ctypes.c_void_p()
    if flags & HTRI_INPUT_ON_DEVICE:
        off_p = ctypes.c_void_p(offsets.data_ptr())
        mem_p = ctypes.c_void_p(members.data_ptr())
        m = int(offsets.shape[0]) - 1
    else:
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        members = np.ascontiguousarray(members, dtype=np.int32)
        off_p, mem_p = _ptr(offsets), _ptr(members)
        m = offsets.shape[0] - 1
    rc = lib.htri_graph_load(off_p, m, mem_p, int(num_vertices), flags, alloc, stream, ctypes.byref(h))
    _check(rc, "htri_graph_load", None)
    return Graph(h, mem)


# ---------------------------------------------------------------- model

class Model:
    """The proposal network (htri_model): 16 -> 64 -> 64 -> 1, ReLU, float32."""

    def __init__(self, seed: int = 0, mem: Optional[TorchMemory] = None):
        self._lib = load_library()
        mem = mem or default_memory()
        h = ctypes.c_void_p()
        _check(self._lib.htri_model_create(int(seed), mem.stream_handle(), ctypes.byref(h)), "htri_model_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.htri_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(HTRI_MODEL_NUM_PARAMS, np.float32)
        _check(self._lib.htri_model_get_params(self._h, _ptr(out)), "htri_model_get_params")
        return out

    def set_params(self, params: np.ndarray) -> None:
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.shape == (HTRI_MODEL_NUM_PARAMS,)
        _check(self._lib.htri_model_set_params(self._h, _ptr(params)), "htri_model_set_params")

    def _merr(self, rc, where):
        if rc != HTRI_OK:
            msg = self._lib.htri_model_last_error(self._h)
            raise HtriError(rc, where, msg.decode() if msg else "")

    def save(self, path: str) -> None:
        """Raw float32 parameters at path, JSON metadata at path + '.json'."""
        self._merr(self._lib.htri_model_save(self._h, os.fsencode(path)), "htri_model_save")

    def load(self, path: str) -> None:
        self._merr(self._lib.htri_model_load(self._h, os.fsencode(path)), "htri_model_load")

    def forward(self, x):
        import torch
        x = x.contiguous()
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(self._lib.htri_model_forward(self._h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                            ctypes.c_void_p(out.data_ptr())), "htri_model_forward")
        return out

    def loss_grad(self, x, y):
        x = x.contiguous()
        y = y.contiguous()
        g = np.zeros(HTRI_MODEL_NUM_PARAMS, np.float32)
        L = ctypes.c_double(0.0)
        _check(self._lib.htri_model_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                              x.shape[0], ctypes.byref(L), _ptr(g)), "htri_model_loss_grad")
        return float(L.value), g

    def train(self, x, y, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0) -> float:
        x = x.contiguous()
        y = y.contiguous()
        L = ctypes.c_double(0.0)
        _check(self._lib.htri_model_train(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                          x.shape[0], int(steps), int(batch), float(lr), int(seed),
                                          ctypes.byref(L)), "htri_model_train")
        return float(L.value)


# ---------------------------------------------------------------- batch

class Batch:
    """Many hypergraphs counted in one persistent launch (htri_batch)."""

    def __init__(self, graphs, flags: int = HTRI_DEDUPE_EDGES):
        self._lib = load_library()
        n = len(graphs)
        self._keep = []
        offs = (ctypes.c_void_p * max(n, 1))()
        mems = (ctypes.c_void_p * max(n, 1))()
        ne = np.zeros(max(n, 1), np.int64)
        nv = np.zeros(max(n, 1), np.int32)
        for q, g in enumerate(graphs):
            o = np.ascontiguousarray(g.offsets, dtype=np.int64)
            m = np.ascontiguousarray(g.members, dtype=np.int32)
            self._keep += [o, m]
            offs[q] = o.ctypes.data
            mems[q] = m.ctypes.data
            ne[q] = o.shape[0] - 1
            nv[q] = g.num_vertices
        h = ctypes.c_void_p()
        rc = self._lib.htri_batch_load(n, offs, _ptr(ne), mems, _ptr(nv), flags, ctypes.byref(h))
        _check(rc, "htri_batch_load", None)
        self._h = h
        self.count = n
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.htri_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, where):
        if rc != HTRI_OK:
            msg = self._lib.htri_batch_last_error(self._h)
            raise HtriError(rc, where, msg.decode() if msg else "")

    def wedges(self) -> np.ndarray:
        out = np.zeros(self.count, np.int64)
        self._err(self._lib.htri_batch_info(self._h, _ptr(out)), "htri_batch_info")
        return out

    def count_patterns(self, schedule=(512, 256, 0), use_graph: bool = True):
        sc = Schedule(*schedule)
        out = np.zeros((self.count, 21), np.int64)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_count(self._h, ctypes.byref(sc), 1 if use_graph else 0, _ptr(out),
                                             ctypes.byref(ms)), "htri_batch_count")
        return out, float(ms.value)

    def autotune(self, repeats: int = 2):
        sc = Schedule(0, 0, 0)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_autotune(self._h, int(repeats), ctypes.byref(sc), ctypes.byref(ms)),
                  "htri_batch_autotune")
        return sc.as_tuple(), float(ms.value)

    def count_per_graph(self, schedule=(512, 256, 0)):
        sc = Schedule(*schedule)
        out = np.zeros((self.count, 21), np.int64)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_count_per_graph(self._h, ctypes.byref(sc), _ptr(out), ctypes.byref(ms)),
                  "htri_batch_count_per_graph")
        return out, float(ms.value)

    def count_full(self, schedule=(512, 256, 0)):
        """Step 1 + items + closure of every graph in one captured HIP-graph
        replay: (counts int64[count, 21], device ms)."""
        sc = Schedule(*schedule)
        out = np.zeros((self.count, 21), np.int64)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_count_full(self._h, ctypes.byref(sc), _ptr(out), ctypes.byref(ms)),
                  "htri_batch_count_full")
        return out, float(ms.value)

    def count_full_per_graph(self, schedule=(512, 256, 0)):
        """The same hot path issued graph by graph: (counts, wall ms)."""
        sc = Schedule(*schedule)
        out = np.zeros((self.count, 21), np.int64)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_count_full_per_graph(self._h, ctypes.byref(sc), _ptr(out), ctypes.byref(ms)),
                  "htri_batch_count_full_per_graph")
        return out, float(ms.value)

    def size_classes(self) -> np.ndarray:
        """Size class (0, 1, 2 by hyperwedges: < 2^18, < 2^21, more) of every graph."""
        out = np.zeros(max(self.count, 1), np.int32)
        self._err(self._lib.htri_batch_size_classes(self._h, _ptr(out)), "htri_batch_size_classes")
        return out[: self.count]

    def autotune_classes(self, repeats: int = 2, cache_path: Optional[str] = None):
        """Fastest schedule per size class: ([3 schedules], [3 ms], from_cache)."""
        best = (Schedule * 3)()
        ms = np.zeros(3, np.float64)
        hit = ctypes.c_int32(0)
        path = os.fsencode(cache_path) if cache_path else None
        self._err(self._lib.htri_batch_autotune_classes(self._h, int(repeats), path, best, _ptr(ms),
                                                        ctypes.byref(hit)), "htri_batch_autotune_classes")
        return [b.as_tuple() for b in best], ms.tolist(), bool(hit.value)

    def count_classes(self, schedules, use_graph: bool = True):
        """Counts with one schedule per size class: (counts int64[count, 21], device ms)."""
        sc = (Schedule * 3)(*[Schedule(*t) for t in schedules])
        out = np.zeros((self.count, 21), np.int64)
        ms = ctypes.c_double(0.0)
        self._err(self._lib.htri_batch_count_classes(self._h, sc, 1 if use_graph else 0, _ptr(out),
                                                     ctypes.byref(ms)), "htri_batch_count_classes")
        return out, float(ms.value)
