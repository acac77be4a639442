"""Python binding of libfrustration (ctypes): argument marshalling only.

Every step of the sweep and of graphL runs in the HIP kernels of the library;
PyTorch only provides device memory (the workspace and the I/O tensors) and
the stream.  There is no CPU fallback: if the library is missing or no GPU is
present, construction fails with an error.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfrustration.so")

ERRORS = {
    0: "FI_OK", -1: "FI_EINVAL", -2: "FI_EASYM", -3: "FI_ESELFLOOP", -4: "FI_EDUP",
    -5: "FI_ESIGN", -6: "FI_ERANGE", -7: "FI_EUNSORTED", -8: "FI_ECAPACITY",
    -9: "FI_EDEVICE", -10: "FI_EDEPTH", -11: "FI_ECOLLISION", -12: "FI_EWORKSPACE",
    -13: "FI_EORDER",
}
SYMBOLS = (
    "fi_graph_workspace_size", "fi_graph_create", "fi_graph_destroy", "fi_graph_info",
    "fi_graph_status", "fi_sweep", "fi_sweep_range", "fi_min_frustration", "fi_cloud_size",
    "fi_cloud_read", "fi_cloud_reset", "fi_cloud_load", "fi_tree_state", "fi_count",
    "fi_graphl_forward", "fi_graphl_backward", "fi_graphl_step", "fi_round_count",
    "fi_batch_workspace_size", "fi_batch_create", "fi_batch_sweep", "fi_set_schedule",
    "fi_get_schedule", "fi_prof_enable", "fi_prof_read", "fi_strerror",
    "fi_bcloud_workspace_size", "fi_bcloud_fmax_for", "fi_bcloud_create", "fi_bcloud_destroy",
    "fi_bcloud_reset", "fi_bcloud_merge", "fi_sweep_bounded", "fi_bcloud_size", "fi_bcloud_read",
    "fi_bcloud_min", "fi_bcloud_stats", "fi_edge_list", "fi_switch_list", "fi_sweep_stats",
    "fi_graphl_descend", "fi_graphl_aux_size", "fi_graphl_scales", "fi_set_sampler",
    "fi_get_sampler", "fi_clean_workspace_size", "fi_clean", "fi_clean_no_alloc",
    "fi_batch_cloud_read", "fi_prof_phases", "fi_probe_gather",
)
CLEAN_NO_ALLOC_MAX_ENTRIES = 1_000_000  # FI_CLEAN_NO_ALLOC_MAX_ENTRIES


class FrustrationError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}")


class CloudEntry(ctypes.Structure):
    _fields_ = [("key_hi", ctypes.c_uint64), ("key_lo", ctypes.c_uint64),
                ("freq", ctypes.c_uint64), ("switches", ctypes.c_uint64),
                ("first_tree", ctypes.c_uint64)]


class Schedule(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("heavy", ctypes.c_int32), ("batch", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfrustration.so and declare its C signatures (no GPU needed)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                              "or python paper_2311_00869_amd/_build.py")
        L = ctypes.CDLL(path)
        c = ctypes
        vp, i32, i64, u64, sz = c.c_void_p, c.c_int32, c.c_int64, c.c_uint64, c.c_size_t
        P = c.POINTER
        sig = {
            "fi_graph_workspace_size": ([i32, i64, i64, P(sz)], c.c_int),
            "fi_graph_create": ([i32, i64, vp, vp, vp, i64, vp, sz, vp, P(vp)], c.c_int),
            "fi_graph_destroy": ([vp], None),
            "fi_graph_info": ([vp, P(i32), P(i32)], c.c_int),
            "fi_graph_status": ([vp, vp], c.c_int),
            "fi_sweep": ([vp, i64, u64, vp], c.c_int),
            "fi_sweep_range": ([vp, i64, i64, u64, vp, vp], c.c_int),
            "fi_min_frustration": ([vp, P(u64), P(u64), vp], c.c_int),
            "fi_cloud_size": ([vp, P(i64), vp], c.c_int),
            "fi_cloud_read": ([vp, vp, i64, P(i64), vp], c.c_int),
            "fi_cloud_reset": ([vp, vp], c.c_int),
            "fi_cloud_load": ([vp, vp, i64, vp], c.c_int),
            "fi_tree_state": ([vp, u64, i64, vp, vp, vp], c.c_int),
            "fi_count": ([vp, vp, i32, vp, vp], c.c_int),
            "fi_graphl_forward": ([vp, vp, i32, vp, vp], c.c_int),
            "fi_graphl_backward": ([vp, vp, i32, vp, vp, vp], c.c_int),
            "fi_graphl_step": ([vp, vp, i32, c.c_float, vp, vp], c.c_int),
            "fi_round_count": ([vp, vp, i32, vp, vp, vp], c.c_int),
            "fi_batch_workspace_size": ([i32, vp, vp, i64, P(sz)], c.c_int),
            "fi_batch_create": ([i32, vp, vp, vp, vp, vp, i64, vp, sz, vp, P(vp)], c.c_int),
            "fi_batch_sweep": ([vp, i64, u64, vp, vp, vp], c.c_int),
            "fi_set_schedule": ([vp, P(Schedule)], c.c_int),
            "fi_get_schedule": ([vp, P(Schedule)], c.c_int),
            "fi_prof_enable": ([vp, c.c_int], c.c_int),
            "fi_prof_read": ([vp, c.c_int, P(c.c_double), P(i64)], c.c_int),
            "fi_strerror": ([c.c_int], c.c_char_p),
            "fi_bcloud_workspace_size": ([i64, i64, P(sz)], c.c_int),
            "fi_bcloud_fmax_for": ([sz, i64, P(i64)], c.c_int),
            "fi_bcloud_create": ([i64, i64, vp, sz, vp, P(vp)], c.c_int),
            "fi_bcloud_destroy": ([vp], None),
            "fi_bcloud_reset": ([vp, vp], c.c_int),
            "fi_bcloud_merge": ([vp, vp, i64, i64, vp], c.c_int),
            "fi_sweep_bounded": ([vp, vp, i64, i64, u64, i64, vp], c.c_int),
            "fi_bcloud_size": ([vp, P(i64), vp], c.c_int),
            "fi_bcloud_read": ([vp, vp, i64, P(i64), vp], c.c_int),
            "fi_bcloud_min": ([vp, P(u64), P(u64), vp], c.c_int),
            "fi_bcloud_stats": ([vp, P(i64), P(i64), vp], c.c_int),
            "fi_edge_list": ([vp, vp, vp], c.c_int),
            "fi_switch_list": ([vp, vp, vp, i64, vp, vp], c.c_int),
            "fi_sweep_stats": ([vp, i64, i64, u64, vp, vp, vp], c.c_int),
            "fi_graphl_descend": ([vp, vp, vp, i32, c.c_float, i64, i32, vp, sz, vp], c.c_int),
            "fi_graphl_aux_size": ([vp, i32, P(sz)], c.c_int),
            "fi_graphl_scales": ([vp, vp, i32, vp, vp], c.c_int),
            "fi_set_sampler": ([vp, i32], c.c_int),
            "fi_clean_workspace_size": ([i32, i64, P(sz)], c.c_int),
            "fi_clean": ([i32, i64, vp, vp, vp, vp, sz, vp, vp, vp, P(i64), vp], c.c_int),
            "fi_clean_no_alloc": ([i32, i64, vp, vp, vp, vp, vp, vp, P(i64), vp], c.c_int),
            "fi_batch_cloud_read": ([vp, i32, vp, i64, P(i64), vp], c.c_int),
            "fi_prof_phases": ([vp, vp, i64], c.c_int),
            "fi_probe_gather": ([vp, i64, vp, i64, vp, vp], c.c_int),
            "fi_get_sampler": ([vp, P(i32)], c.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return L


def _check(rc: int, where: str):
    if rc != 0:
        raise FrustrationError(rc, where)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libfrustration needs a ROCm GPU; none is visible")


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


def nwords(n: int) -> int:
    return (n + 63) // 64


def words_to_numpy(t) -> np.ndarray:
    """int64 device words -> numpy uint64."""
    return t.detach().cpu().numpy().view(np.uint64)


def probe_gather(idx, records, sink, stream=None):
    """Measurement aid (fi_probe_gather): read the first 32 bytes of the 64-byte
    record idx[e] of records for every e, as one dense pull level gathers its
    neighbours.  idx: int32 device tensor; records: a device tensor of
    64 * n_records bytes; sink: a device tensor of at least 4 bytes."""
    lib = load_library()
    if idx.dtype != torch.int32 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous int32 tensor")
    nbytes = records.numel() * records.element_size()
    if nbytes % 64 or not records.is_contiguous() or sink.numel() * sink.element_size() < 4:
        raise ValueError("records must hold whole 64-byte records; sink at least 4 bytes")
    _check(lib.fi_probe_gather(_ptr(idx), idx.numel(), _ptr(records), nbytes // 64, _ptr(sink),
                               _stream_ptr(stream)), "probe_gather")


def clean(n: int, src, dst, sign, device="cuda", stream=None, no_alloc: bool = False):
    """The paper's input cleaning on the GPU (fi_clean): a raw signed edge
    list -> (row_ptr, col, sign) device tensors of a simple symmetric signed
    graph, and the counts of what was kept and dropped.  no_alloc=True calls
    fi_clean_no_alloc, whose workspace is the library's own device array (up
    to CLEAN_NO_ALLOC_MAX_ENTRIES entries)."""
    _require_gpu()
    lib = load_library()
    dev = torch.device(device)
    s = _dev(src, torch.int32, dev)
    d = _dev(dst, torch.int32, dev)
    g = _dev(sign, torch.int32, dev)
    E = int(s.numel())
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(2 * E, 1), dtype=torch.int32, device=dev)
    sg = torch.empty(max(2 * E, 1), dtype=torch.int8, device=dev)
    counts = (ctypes.c_int64 * 5)()
    if no_alloc:
        with torch.cuda.device(dev):
            _check(lib.fi_clean_no_alloc(int(n), E, _ptr(s), _ptr(d), _ptr(g), _ptr(rp), _ptr(col),
                                         _ptr(sg), counts, _stream_ptr(stream)), "clean_no_alloc")
    else:
        size = ctypes.c_size_t()
        _check(lib.fi_clean_workspace_size(int(n), E, ctypes.byref(size)), "clean_workspace_size")
        raw = torch.empty(size.value + 256, dtype=torch.uint8, device=dev)
        ptr = (raw.data_ptr() + 255) // 256 * 256
        with torch.cuda.device(dev):
            _check(lib.fi_clean(int(n), E, _ptr(s), _ptr(d), _ptr(g), ctypes.c_void_p(ptr), size.value,
                                _ptr(rp), _ptr(col), _ptr(sg), counts, _stream_ptr(stream)), "clean")
    nnz = 2 * counts[0]
    names = ("kept", "invalid", "self_loops", "duplicates", "inconsistent_pairs")
    return rp, col[:nnz], sg[:nnz], dict(zip(names, [int(x) for x in counts]))


class Graph:
    """A signed graph resident on the GPU with its frustration cloud.

    row_ptr / col / sign: symmetric sorted CSR (numpy or torch).  The
    workspace is one torch uint8 tensor owned by this object.
    """

    def __init__(self, row_ptr, col, sign, cloud_capacity: int = 4096, device="cuda",
                 stream=None):
        _require_gpu()
        self.lib = load_library()
        self.device = torch.device(device)
        rp = _dev(row_ptr, torch.int32, self.device)
        cl = _dev(col, torch.int32, self.device)
        sg = _dev(sign, torch.int8, self.device)
        self.n = int(rp.numel() - 1)
        self.nnz = int(cl.numel())
        self.m = self.nnz // 2
        self.nwords = nwords(self.n)
        self.cloud_capacity = int(cloud_capacity)
        size = ctypes.c_size_t(0)
        _check(self.lib.fi_graph_workspace_size(self.n, self.nnz, self.cloud_capacity,
                                                ctypes.byref(size)), "workspace_size")
        self.ws_bytes = int(size.value)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.fi_graph_create(self.n, self.nnz, _ptr(rp), _ptr(cl), _ptr(sg),
                                          self.cloud_capacity, ctypes.c_void_p(self._ws_ptr),
                                          self.ws_bytes, _stream_ptr(stream), ctypes.byref(h))
        _check(rc, "graph_create")
        self.handle = h
        del rp, cl, sg

    # ---------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            self.lib.fi_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        c, i = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.fi_graph_info(self.handle, ctypes.byref(c), ctypes.byref(i)), "info")
        return int(c.value), int(i.value)

    def status(self, stream=None):
        _check(self.lib.fi_graph_status(self.handle, _stream_ptr(stream)), "status")

    # ---------------------------------------------------------------- sweep
    def sweep(self, K: int, seed: int, stream=None):
        _check(self.lib.fi_sweep(self.handle, int(K), seed & (2**64 - 1), _stream_ptr(stream)), "sweep")

    def sweep_range(self, t0: int, t1: int, seed: int, tree_switches: bool = False, stream=None):
        out = torch.empty(max(t1 - t0, 1), dtype=torch.int64, device=self.device) if tree_switches else None
        _check(self.lib.fi_sweep_range(self.handle, int(t0), int(t1), seed & (2**64 - 1), _ptr(out),
                                       _stream_ptr(stream)), "sweep_range")
        return None if out is None else out[: t1 - t0]

    def min_frustration(self, stream=None):
        s, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.fi_min_frustration(self.handle, ctypes.byref(s), ctypes.byref(t),
                                           _stream_ptr(stream)), "min_frustration")
        return int(s.value), int(t.value)

    def cloud_size(self, stream=None) -> int:
        k = ctypes.c_int64()
        _check(self.lib.fi_cloud_size(self.handle, ctypes.byref(k), _stream_ptr(stream)), "cloud_size")
        return int(k.value)

    def cloud(self, stream=None) -> np.ndarray:
        """uint64 [E, 5]: key_hi, key_lo, freq, switches, first_tree (sorted by key)."""
        size = self.cloud_size(stream)
        buf = (CloudEntry * max(size, 1))()
        written = ctypes.c_int64()
        _check(self.lib.fi_cloud_read(self.handle, buf, size, ctypes.byref(written),
                                      _stream_ptr(stream)), "cloud_read")
        arr = np.ctypeslib.as_array(buf).view(np.uint64).reshape(-1, 5)[:size].copy()
        return arr

    def sweep_bounded(self, cloud: "BoundedCloud", t0: int, t1: int, seed: int, chunk: int = 0,
                      stream=None):
        """Alg. alg-scale over trees t0 .. t1-1 into ``cloud`` (empties this
        graph's own cloud, which stages each chunk)."""
        _check(self.lib.fi_sweep_bounded(self.handle, cloud.handle, int(t0), int(t1),
                                         seed & (2**64 - 1), int(chunk), _stream_ptr(stream)),
               "sweep_bounded")

    def edge_list(self, stream=None):
        """int32 [m, 2]: the undirected edges (u < v) in increasing order."""
        out = torch.empty((max(self.m, 1), 2), dtype=torch.int32, device=self.device)
        _check(self.lib.fi_edge_list(self.handle, _ptr(out), _stream_ptr(stream)), "edge_list")
        return out[: self.m]

    def switch_list(self, bits, cap=None, stream=None):
        """Edges a state frustrates (the edges to switch), int32 [k, 2] in
        edge-list order.  ``bits``: int64 device words, set bit = -1."""
        b = bits.to(device=self.device, dtype=torch.int64).contiguous()
        cap = self.m if cap is None else int(cap)
        out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self.lib.fi_switch_list(self.handle, _ptr(b), _ptr(out), cap, _ptr(cnt),
                                       _stream_ptr(stream)), "switch_list")
        k = int(cnt.item())
        return out[: min(k, cap)], k

    def sweep_stats(self, t0: int, t1: int, seed: int, vertex_minus=None, edge_switched=None,
                    stream=None):
        """Trees t0 .. t1-1 into the cloud, adding per-vertex and per-edge
        counts to the given int64 tensors (new zero tensors if None)."""
        if vertex_minus is None:
            vertex_minus = torch.zeros(max(self.n, 1), dtype=torch.int64, device=self.device)
        if edge_switched is None:
            edge_switched = torch.zeros(max(self.m, 1), dtype=torch.int64, device=self.device)
        _check(self.lib.fi_sweep_stats(self.handle, int(t0), int(t1), seed & (2**64 - 1),
                                       _ptr(vertex_minus), _ptr(edge_switched),
                                       _stream_ptr(stream)), "sweep_stats")
        return vertex_minus[: self.n], edge_switched[: self.m]

    def cloud_reset(self, stream=None):
        _check(self.lib.fi_cloud_reset(self.handle, _stream_ptr(stream)), "cloud_reset")

    def cloud_load(self, entries, stream=None):
        e = np.ascontiguousarray(entries, dtype=np.uint64).reshape(-1, 5)
        _check(self.lib.fi_cloud_load(self.handle, e.ctypes.data_as(ctypes.c_void_p), e.shape[0],
                                      _stream_ptr(stream)), "cloud_load")

    def tree_state(self, seed: int, t: int, stream=None):
        """(canonical words as numpy uint64 [nwords], switches) of tree t."""
        bits = torch.zeros(max(self.nwords, 1), dtype=torch.int64, device=self.device)
        sw = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self.lib.fi_tree_state(self.handle, seed & (2**64 - 1), int(t), _ptr(bits), _ptr(sw),
                                      _stream_ptr(stream)), "tree_state")
        return words_to_numpy(bits)[: self.nwords], int(sw.item())

    def count(self, bits, stream=None):
        """Exact frustration counts of B states given as int64 words [B, nwords]."""
        b = bits.to(device=self.device, dtype=torch.int64).contiguous().reshape(-1, self.nwords)
        out = torch.zeros(b.shape[0], dtype=torch.int64, device=self.device)
        _check(self.lib.fi_count(self.handle, _ptr(b), b.shape[0], _ptr(out), _stream_ptr(stream)), "count")
        return out

    # ---------------------------------------------------------------- graphL
    def graphl_forward(self, gamma, stream=None):
        g = gamma.contiguous()
        R = g.shape[1]
        loss = torch.empty(R, dtype=torch.float64, device=self.device)
        _check(self.lib.fi_graphl_forward(self.handle, _ptr(g), R, _ptr(loss), _stream_ptr(stream)),
               "graphl_forward")
        return loss

    def graphl_backward(self, gamma, grad_loss=None, stream=None):
        g = gamma.contiguous()
        R = g.shape[1]
        w = None if grad_loss is None else grad_loss.to(dtype=torch.float64).contiguous()
        out = torch.empty_like(g)
        _check(self.lib.fi_graphl_backward(self.handle, _ptr(g), R, _ptr(w), _ptr(out),
                                           _stream_ptr(stream)), "graphl_backward")
        return out

    def graphl_step(self, gamma, alpha: float, out=None, stream=None):
        g = gamma.contiguous()
        R = g.shape[1]
        if out is None:
            out = torch.empty_like(g)
        _check(self.lib.fi_graphl_step(self.handle, _ptr(g), R, float(alpha), _ptr(out),
                                       _stream_ptr(stream)), "graphl_step")
        return out

    def graphl_descend(self, gamma0, steps: int, alpha: float = 0.001, rescale_log2: int = 0,
                       out=None, stream=None):
        """Alg. alg-gradient's update loop with the power-of-two overflow
        policy.  Returns (Gamma, scales): the true iterate is
        Gamma * 2**scales (``scales()`` turns the handle into int32 [n, R])."""
        R = gamma0.shape[1]
        g = out if out is not None else torch.empty((self.n, R), dtype=torch.float32,
                                                    device=self.device)
        g.copy_(gamma0)
        work = torch.empty_like(g)
        size = ctypes.c_size_t()
        _check(self.lib.fi_graphl_aux_size(self.handle, R, ctypes.byref(size)), "graphl_aux_size")
        raw = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (raw.data_ptr() + 255) // 256 * 256
        _check(self.lib.fi_graphl_descend(self.handle, _ptr(g), _ptr(work), R, float(alpha),
                                          int(steps), int(rescale_log2), ctypes.c_void_p(ptr),
                                          size.value, _stream_ptr(stream)), "graphl_descend")
        graph = self

        class Scales:
            def __call__(self_, stream=None):
                o = torch.empty((max(graph.n, 1), R), dtype=torch.int32, device=graph.device)
                _check(graph.lib.fi_graphl_scales(graph.handle, ctypes.c_void_p(ptr), R, _ptr(o),
                                                  _stream_ptr(stream)), "graphl_scales")
                return o[: graph.n]

        sc = Scales()
        sc.buffer = raw
        return g, sc

    def round_count(self, gamma, return_bits: bool = False, stream=None):
        g = gamma.contiguous()
        R = g.shape[1]
        counts = torch.empty(R, dtype=torch.int64, device=self.device)
        bits = torch.empty((R, max(self.nwords, 1)), dtype=torch.int64, device=self.device) if return_bits else None
        _check(self.lib.fi_round_count(self.handle, _ptr(g), R, _ptr(counts), _ptr(bits),
                                       _stream_ptr(stream)), "round_count")
        return (counts, bits) if return_bits else counts

    SAMPLERS = {"bfs": 0, "rdfs": 1, "hybrid": 2, "kruskal": 3}

    def set_sampler(self, sampler="bfs"):
        """Tree sampler: "bfs", "rdfs", "hybrid" (Alg. alg-hybrid) or "kruskal"."""
        code = self.SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
        _check(self.lib.fi_set_sampler(self.handle, code), "set_sampler")

    def get_sampler(self) -> str:
        out = ctypes.c_int32()
        _check(self.lib.fi_get_sampler(self.handle, ctypes.byref(out)), "get_sampler")
        return {v: k for k, v in self.SAMPLERS.items()}[out.value]

    # ---------------------------------------------------------------- tuning / timing
    def set_schedule(self, path=0, block=256, grid=0, heavy=512, batch=4):
        s = Schedule(path, block, grid, heavy, batch)
        _check(self.lib.fi_set_schedule(self.handle, ctypes.byref(s)), "set_schedule")

    def get_schedule(self):
        s = Schedule()
        _check(self.lib.fi_get_schedule(self.handle, ctypes.byref(s)), "get_schedule")
        return dict(path=s.path, block=s.block, grid=s.grid, heavy=s.heavy, batch=s.batch)

    def prof_enable(self, on=True):
        _check(self.lib.fi_prof_enable(self.handle, 1 if on else 0), "prof_enable")

    def prof_read(self, kernel=0):
        ms, k = ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.fi_prof_read(self.handle, kernel, ctypes.byref(ms), ctypes.byref(k)), "prof_read")
        return float(ms.value), int(k.value)

    PHASES = {0: "start", 1: "reset", 2: "roots", 3: "big roots", 4: "lists", 5: "pull",
              6: "split rows", 7: "counts+keys", 8: "insert"}

    def phase_log(self, records: int = 1 << 16):
        """Turn the multi-tree kernel's phase log on (a zeroed device buffer
        of `records` records) or, with records=0, off.  Returns the buffer."""
        if records <= 0:
            _check(self.lib.fi_prof_phases(self.handle, None, 0), "prof_phases")
            self._plog = None
            return None
        self._plog = torch.zeros(2 + 2 * records, dtype=torch.int64, device=self.device)
        _check(self.lib.fi_prof_phases(self.handle, _ptr(self._plog), self._plog.numel()),
               "prof_phases")
        return self._plog

    def phase_records(self):
        """The logged (phase, level, microseconds since the previous record)
        of every record after a launch start, in order."""
        log = self._plog.cpu().numpy().view(np.uint64)
        k = min(int(log[0]), (log.size - 2) // 2)
        tags, t = log[2:2 + 2 * k:2], log[3:3 + 2 * k:2].astype(np.int64)
        out = []
        for i in range(1, k):
            ph, lv = int(tags[i]) >> 32, int(tags[i]) & 0xFFFFFFFF
            if ph != 0:
                out.append((ph, lv, (t[i] - t[i - 1]) / 100.0))
        return out


class BoundedCloud:
    """Memory-bound frustration cloud of Alg. alg-scale: the F_max best
    states by (switch count, first tree), each with its full count.

    Fill it with ``graph.sweep_bounded(cloud, t0, t1, seed)``, or with
    ``graph.sweep_range`` over consecutive chunks and ``merge``.  The graph's
    cloud_capacity must not exceed ``staging``.
    """

    def __init__(self, f_max: int, staging: int = 8192, device="cuda", stream=None):
        _require_gpu()
        self.lib = load_library()
        self.device = torch.device(device)
        self.f_max, self.staging = int(f_max), int(staging)
        size = ctypes.c_size_t(0)
        _check(self.lib.fi_bcloud_workspace_size(self.f_max, self.staging, ctypes.byref(size)),
               "bcloud_workspace_size")
        self.ws_bytes = int(size.value)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.fi_bcloud_create(self.f_max, self.staging, ctypes.c_void_p(ptr),
                                           self.ws_bytes, _stream_ptr(stream), ctypes.byref(h))
        _check(rc, "bcloud_create")
        self.handle = h

    @staticmethod
    def fmax_for(cap_bytes: int, staging: int = 8192) -> int:
        """Largest F_max whose workspace fits in cap_bytes."""
        out = ctypes.c_int64()
        _check(load_library().fi_bcloud_fmax_for(int(cap_bytes), int(staging), ctypes.byref(out)),
               "bcloud_fmax_for")
        return int(out.value)

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            self.lib.fi_bcloud_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        _check(self.lib.fi_bcloud_reset(self.handle, _stream_ptr(stream)), "bcloud_reset")

    def merge(self, graph: "Graph", t0: int, t1: int, stream=None):
        _check(self.lib.fi_bcloud_merge(graph.handle, self.handle, int(t0), int(t1),
                                        _stream_ptr(stream)), "bcloud_merge")

    def size(self, stream=None) -> int:
        k = ctypes.c_int64()
        _check(self.lib.fi_bcloud_size(self.handle, ctypes.byref(k), _stream_ptr(stream)),
               "bcloud_size")
        return int(k.value)

    def entries(self, stream=None) -> np.ndarray:
        """uint64 [E, 5]: key_hi, key_lo, freq, switches, first_tree (sorted by key)."""
        size = self.size(stream)
        buf = (CloudEntry * max(size, 1))()
        written = ctypes.c_int64()
        _check(self.lib.fi_bcloud_read(self.handle, buf, size, ctypes.byref(written),
                                       _stream_ptr(stream)), "bcloud_read")
        return np.ctypeslib.as_array(buf).view(np.uint64).reshape(-1, 5)[:size].copy()

    def min_frustration(self, stream=None):
        s, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.fi_bcloud_min(self.handle, ctypes.byref(s), ctypes.byref(t),
                                      _stream_ptr(stream)), "bcloud_min")
        return int(s.value), int(t.value)

    def stats(self, stream=None):
        """(trees merged, entries dropped)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.fi_bcloud_stats(self.handle, ctypes.byref(a), ctypes.byref(b),
                                        _stream_ptr(stream)), "bcloud_stats")
        return int(a.value), int(b.value)


class BatchGraph:
    """Many independent signed graphs of uneven size swept in the same
    launches, each with its own vertex ids, cloud and minimum.

    graphs: a sequence of (row_ptr, col, sign) CSR triples (or objects with
    those attributes).  They are concatenated on the host, uploaded once and
    validated, packed and split into components on the GPU.
    """

    def __init__(self, graphs, cloud_capacity_per_graph: int = 1024, device="cuda", stream=None):
        _require_gpu()
        self.lib = load_library()
        self.device = torch.device(device)
        rps, cols, sgns = [], [], []
        vo, no = [0], [0]
        for gr in graphs:
            if isinstance(gr, (tuple, list)):
                rp, cl, sg = gr
            else:
                rp, cl, sg = gr.row_ptr, gr.col, gr.sign
            rp = np.asarray(rp, dtype=np.int32)
            cl = np.asarray(cl, dtype=np.int32)
            sg = np.asarray(sg, dtype=np.int8)
            rps.append(rp)
            cols.append(cl)
            sgns.append(sg)
            vo.append(vo[-1] + rp.size - 1)
            no.append(no[-1] + cl.size)
        self.G = len(rps)
        if self.G < 1:
            raise FrustrationError(-1, "batch_create")
        self.vertex_offsets = np.asarray(vo, dtype=np.int64)
        self.nnz_offsets = np.asarray(no, dtype=np.int64)
        self.cloud_capacity = int(cloud_capacity_per_graph)
        rp_all = torch.from_numpy(np.concatenate(rps)).to(self.device)
        col_all = torch.from_numpy(np.concatenate(cols) if no[-1] else np.zeros(1, np.int32)).to(self.device)
        sg_all = torch.from_numpy(np.concatenate(sgns) if no[-1] else np.zeros(1, np.int8)).to(self.device)
        vop = self.vertex_offsets.ctypes.data_as(ctypes.c_void_p)
        nop = self.nnz_offsets.ctypes.data_as(ctypes.c_void_p)
        size = ctypes.c_size_t(0)
        _check(self.lib.fi_batch_workspace_size(self.G, vop, nop, self.cloud_capacity,
                                                ctypes.byref(size)), "batch_workspace_size")
        self.ws_bytes = int(size.value)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.fi_batch_create(self.G, vop, nop, _ptr(rp_all), _ptr(col_all), _ptr(sg_all),
                                          self.cloud_capacity, ctypes.c_void_p(self._ws_ptr),
                                          self.ws_bytes, _stream_ptr(stream), ctypes.byref(h))
        _check(rc, "batch_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            self.lib.fi_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep_into(self, trees: int, seed: int, min_out, distinct_out=None, stream=None):
        """Launch-only form (no host synchronisation), usable under HIP graph
        capture: min_out int64 [G, 2] receives (switches, first tree) per
        graph, distinct_out int64 [G] the number of distinct states."""
        _check(self.lib.fi_batch_sweep(self.handle, int(trees), seed & (2**64 - 1), _ptr(min_out),
                                       _ptr(distinct_out) if distinct_out is not None else None,
                                       _stream_ptr(stream)), "batch_sweep")

    def sweep(self, trees: int, seed: int, stream=None):
        """Sweep `trees` trees of every graph; returns (min [G, 2], distinct [G])
        as int64 device tensors, after checking the sticky error bits."""
        mn = torch.empty((self.G, 2), dtype=torch.int64, device=self.device)
        ds = torch.empty(self.G, dtype=torch.int64, device=self.device)
        self.sweep_into(trees, seed, mn, ds, stream)
        self.status(stream)
        return mn, ds

    def status(self, stream=None):
        _check(self.lib.fi_graph_status(self.handle, _stream_ptr(stream)), "batch_status")

    def cloud(self, graph: int, stream=None) -> np.ndarray:
        """Graph `graph`'s cloud after the last sweep: uint64 [E, 5] rows
        (key_hi, key_lo, freq, switches, first_tree) sorted by key."""
        n = ctypes.c_int64(0)
        _check(self.lib.fi_batch_cloud_read(self.handle, int(graph), None, 0, ctypes.byref(n),
                                            _stream_ptr(stream)), "batch_cloud_read")
        buf = (CloudEntry * max(n.value, 1))()
        _check(self.lib.fi_batch_cloud_read(self.handle, int(graph), buf, n.value, ctypes.byref(n),
                                            _stream_ptr(stream)), "batch_cloud_read")
        return np.array([[e.key_hi, e.key_lo, e.freq, e.switches, e.first_tree] for e in buf[: n.value]],
                        dtype=np.uint64).reshape(-1, 5)

    def set_schedule(self, block=256, grid=0, path=0):
        """path 0: 64 trees of a graph per workgroup pass when at least 16 trees
        per graph are swept, else one workgroup per tree; 1: one workgroup per
        tree; 4: 64 trees per pass."""
        s = Schedule(path, block, grid, 512, 1)
        _check(self.lib.fi_set_schedule(self.handle, ctypes.byref(s)), "set_schedule")

    def get_schedule(self):
        s = Schedule()
        _check(self.lib.fi_get_schedule(self.handle, ctypes.byref(s)), "get_schedule")
        return dict(block=s.block, grid=s.grid, path=s.path)

    def prof_enable(self, on=True):
        _check(self.lib.fi_prof_enable(self.handle, 1 if on else 0), "prof_enable")

    def prof_read(self, kernel=0):
        ms, k = ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.fi_prof_read(self.handle, kernel, ctypes.byref(ms), ctypes.byref(k)), "prof_read")
        return float(ms.value), int(k.value)


class GraphLLoss(torch.autograd.Function):
    """L_r = sum over edges (1 - e_ij G_ir G_jr) / 2 (Eq. eq-loss_imbalance_new) for
    every restart column r; forward and backward are the library's kernels."""

    @staticmethod
    def forward(ctx, gamma, graph):
        ctx.graph = graph
        ctx.save_for_backward(gamma)
        return graph.graphl_forward(gamma)

    @staticmethod
    def backward(ctx, grad_loss):
        (gamma,) = ctx.saved_tensors
        return ctx.graph.graphl_backward(gamma, grad_loss), None


def graphl_loss(graph: Graph, gamma):
    return GraphLLoss.apply(gamma, graph)


def graphl_descent(graph: Graph, gamma0, steps: int, alpha: float = 0.001):
    """Alg. alg-gradient's update loop with the fused step kernel (ping-pong
    buffers); returns the final Gamma."""
    a = gamma0.contiguous().clone()
    b = torch.empty_like(a)
    for _ in range(steps):
        graph.graphl_step(a, alpha, out=b)
        a, b = b, a
    return a
