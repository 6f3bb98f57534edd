"""Python binding of libmsf.so, the MI355X minimum spanning forest library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/msf.h``.  PyTorch provides
device memory and the current stream.  There is no CPU fallback: if the
library is not built, importing the binding's entry points raises.

    import paper_2302_12199_amd as msf
    mask, total, stats = msf.compute(u, v, w, n)      # u, v, w: int32 CUDA tensors
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so libmsf.so binds to the HIP runtime torch uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsf.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EWORKSPACE, EINTERNAL = 0, -1, -2, -3, -4, -5, -6
ALGOS = {"boruvka": 0, "filter": 1}
PIVOTS = {"median": 0, "quantile": 1, "mlp": 2}
ROUND0 = {"auto": 0, "edges": 1, "buckets": 2}
DEDUP = {"auto": 0, "never": 1, "exact": 2, "local": 3}
MAX_TRACE = 64


class Options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("pivot", ctypes.c_int32),
                ("quantile", ctypes.c_float), ("sample_size", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("sparse_degree", ctypes.c_int32),
                ("min_split_edges", ctypes.c_int32), ("round0", ctypes.c_int32),
                ("dedup_policy", ctypes.c_int32), ("split_retries", ctypes.c_int32),
                ("defer_edges", ctypes.c_int32), ("tail_threshold", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("total_weight", ctypes.c_uint64), ("msf_edges", ctypes.c_uint64),
                ("rounds", ctypes.c_uint32), ("levels", ctypes.c_uint32),
                ("base_cases", ctypes.c_uint32), ("pivot_q_used", ctypes.c_float),
                ("round_live", ctypes.c_uint64 * MAX_TRACE),
                ("round_edges", ctypes.c_uint64 * MAX_TRACE),
                ("round_found", ctypes.c_uint64 * MAX_TRACE),
                ("filtered_in", ctypes.c_uint64), ("filtered_out", ctypes.c_uint64),
                ("split_edges", ctypes.c_uint64 * MAX_TRACE),
                ("split_pivot", ctypes.c_uint64 * MAX_TRACE),
                ("split_light", ctypes.c_uint64 * MAX_TRACE),
                ("split_kept", ctypes.c_uint64 * MAX_TRACE),
                ("split_q", ctypes.c_float * MAX_TRACE),
                ("top_features", ctypes.c_float * 16),
                ("split_features", (ctypes.c_float * 16) * MAX_TRACE),
                ("round_vertices", ctypes.c_uint64 * MAX_TRACE),
                ("split_attempts", ctypes.c_uint32 * MAX_TRACE),
                ("split_deferred_in", ctypes.c_uint64 * MAX_TRACE),
                ("pivot_retries", ctypes.c_uint32), ("deferrals", ctypes.c_uint32)]

    def to_dict(self):
        r = min(self.rounds, MAX_TRACE)
        return {"total_weight": int(self.total_weight), "msf_edges": int(self.msf_edges),
                "rounds": int(self.rounds), "levels": int(self.levels),
                "base_cases": int(self.base_cases), "pivot_q_used": float(self.pivot_q_used),
                "round_live": [int(x) for x in self.round_live[:r]],
                "round_edges": [int(x) for x in self.round_edges[:r]],
                "round_found": [int(x) for x in self.round_found[:r]],
                "round_vertices": [int(x) for x in self.round_vertices[:r]],
                "filtered_in": int(self.filtered_in), "filtered_out": int(self.filtered_out),
                "splits": [{"edges": int(self.split_edges[i]), "pivot": int(self.split_pivot[i]),
                            "light": int(self.split_light[i]), "kept": int(self.split_kept[i]),
                            "q": float(self.split_q[i]),
                            "attempts": int(self.split_attempts[i]),
                            "deferred_in": int(self.split_deferred_in[i]),
                            "features": [float(x) for x in self.split_features[i]]}
                           for i in range(min(self.levels, MAX_TRACE))],
                "top_features": [float(x) for x in self.top_features],
                "pivot_retries": int(self.pivot_retries), "deferrals": int(self.deferrals)}


class MSFError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        text = _lib().msf_status_string(status).decode() if _LIB else str(status)
        super().__init__(f"msf status {status} ({text}){': ' + detail if detail else ''}")


_LIB = None

# Exported C symbols (each declared in include/msf.h).
SYMBOLS = ("msf_workspace_bytes", "msf_compute", "msf_compute_noalloc", "msf_status_string", "msf_last_error",
           "msf_version", "msf_profile_enable", "msf_profile_reset", "msf_profile_read",
           "msf_batched_workspace_bytes", "msf_compute_batched", "msf_batched_graph_create",
           "msf_batched_graph_launch", "msf_batched_graph_destroy", "msf_batched_autotune",
           "msf_wall_clock_khz", "msf_pivot_model_load", "msf_pivot_model_clear",
           "msf_pivot_model_loaded", "msf_mlp_param_count", "msf_mlp_forward", "msf_mlp_grad",
           "msf_mlp_adam")


class BatchOptions(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("lds_vertices", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("coop_edges", ctypes.c_int32),
                ("wave_edges", ctypes.c_int32), ("hot_min", ctypes.c_int32),
                ("wave_min", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        lib.msf_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(Options)]
        lib.msf_workspace_bytes.restype = sz
        lib.msf_compute.argtypes = [vp, vp, vp, i64, i64, vp, ctypes.POINTER(ctypes.c_uint64),
                                    vp, sz, vp, ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        lib.msf_compute.restype = ctypes.c_int
        lib.msf_compute_noalloc.argtypes = [vp, vp, vp, i64, i64, vp,
                                            ctypes.POINTER(ctypes.c_uint64), vp,
                                            ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        lib.msf_compute_noalloc.restype = ctypes.c_int
        lib.msf_status_string.argtypes = [ctypes.c_int]
        lib.msf_status_string.restype = ctypes.c_char_p
        lib.msf_last_error.restype = ctypes.c_char_p
        lib.msf_version.restype = ctypes.c_int
        lib.msf_profile_enable.argtypes = [ctypes.c_int]
        bo = ctypes.POINTER(BatchOptions)
        lib.msf_batched_workspace_bytes.argtypes = [i64, i64, bo]
        lib.msf_batched_workspace_bytes.restype = sz
        lib.msf_compute_batched.argtypes = [vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, sz,
                                            vp, bo]
        lib.msf_batched_graph_create.argtypes = [vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, vp,
                                                 vp, sz, bo, ctypes.POINTER(vp)]
        lib.msf_batched_graph_launch.argtypes = [vp, vp]
        lib.msf_batched_graph_destroy.argtypes = [vp]
        lib.msf_pivot_model_load.argtypes = [vp, sz]
        lib.msf_mlp_forward.argtypes = [vp, vp, i64, vp, ctypes.c_int, vp]
        lib.msf_mlp_grad.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp, vp, vp]
        lib.msf_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_int, vp]
        lib.msf_batched_autotune.argtypes = [vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, vp, sz, vp,
                                             bo, ctypes.POINTER(ctypes.c_float)]
        lib.msf_profile_read.argtypes = [ctypes.POINTER(KernelProfile), ctypes.c_int]
        _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (raises if libmsf.so is not built)."""
    return _lib()


def make_options(algo="boruvka", pivot="median", quantile=0.5, seed=1, sample_size=0,
                 sparse_degree=0, min_split_edges=0, round0="auto", dedup="auto",
                 split_retries=0, defer_edges=0, tail_threshold=0):
    o = Options()
    o.tail_threshold = int(tail_threshold)
    o.split_retries = int(split_retries)
    o.defer_edges = int(defer_edges)
    o.round0 = ROUND0[round0] if isinstance(round0, str) else int(round0)
    o.dedup_policy = DEDUP[dedup] if isinstance(dedup, str) else int(dedup)
    o.algo = ALGOS[algo] if isinstance(algo, str) else int(algo)
    o.pivot = PIVOTS[pivot] if isinstance(pivot, str) else int(pivot)
    o.quantile = float(quantile)
    o.seed = int(seed)
    o.sample_size = int(sample_size)
    o.sparse_degree = int(sparse_degree)
    o.min_split_edges = int(min_split_edges)
    return o


def workspace_bytes(m, n, **opts):
    o = make_options(**opts)
    return int(_lib().msf_workspace_bytes(int(m), int(n), ctypes.byref(o)))


def _dev_i32(t, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype == torch.uint32:
        t = t.view(torch.int32)
    if t.dtype != torch.int32:
        raise TypeError(f"{name} must be int32 (or uint32 for w)")
    return t.contiguous()


def compute(u, v, w, n, *, workspace=None, mask_out=None, stream=None, **opts):
    """MSF of the graph (u[e], v[e], w[e]) on vertices [0, n).

    Returns (mask, total, stats): mask is a uint8 CUDA tensor (1 = MSF edge),
    total the 64-bit MSF weight (Python int) and stats a dict (msf.h msf_stats).
    ``workspace`` may be a uint8 CUDA tensor of at least workspace_bytes(m, n)
    bytes; otherwise torch allocates one for the call.
    """
    lib = _lib()
    u, v, w = _dev_i32(u, "u"), _dev_i32(v, "v"), _dev_i32(w, "w")
    m = u.numel()
    if v.numel() != m or w.numel() != m:
        raise ValueError("u, v, w must have the same length")
    o = make_options(**opts)
    dev = u.device
    if mask_out is None:
        mask_out = torch.empty(max(m, 1), dtype=torch.uint8, device=dev)[:m]
    need = int(lib.msf_workspace_bytes(m, int(n), ctypes.byref(o)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    total = ctypes.c_uint64(0)
    st = Stats()
    rc = lib.msf_compute(u.data_ptr(), v.data_ptr(), w.data_ptr(), m, int(n),
                         mask_out.data_ptr(), ctypes.byref(total), workspace.data_ptr(),
                         workspace.numel(), ctypes.c_void_p(s.cuda_stream), ctypes.byref(o),
                         ctypes.byref(st))
    if rc != OK:
        raise MSFError(rc, lib.msf_last_error().decode(errors="replace"))
    return mask_out, int(total.value), st.to_dict()


NOALLOC_SCRATCH_BYTES = 128 << 20      # MSF_NOALLOC_SCRATCH_BYTES in msf.h


def compute_noalloc(u, v, w, n, *, mask_out, stream=None, **opts):
    """MSF through msf_compute_noalloc: the library's static per-GPU scratch
    is the workspace, so the call allocates nothing (``mask_out`` must be
    given).  Same results as compute(); raises MSFError(EWORKSPACE) when the
    graph needs more than NOALLOC_SCRATCH_BYTES of workspace."""
    lib = _lib()
    u, v, w = _dev_i32(u, "u"), _dev_i32(v, "v"), _dev_i32(w, "w")
    m = u.numel()
    if v.numel() != m or w.numel() != m or mask_out.numel() < m:
        raise ValueError("u, v, w, mask_out lengths differ")
    o = make_options(**opts)
    s = stream if stream is not None else torch.cuda.current_stream(u.device)
    total = ctypes.c_uint64(0)
    st = Stats()
    rc = lib.msf_compute_noalloc(u.data_ptr(), v.data_ptr(), w.data_ptr(), m, int(n),
                                 mask_out.data_ptr(), ctypes.byref(total),
                                 ctypes.c_void_p(s.cuda_stream), ctypes.byref(o),
                                 ctypes.byref(st))
    if rc != OK:
        raise MSFError(rc, lib.msf_last_error().decode(errors="replace"))
    return mask_out, int(total.value), st.to_dict()


def profile_enable(on=True):
    _lib().msf_profile_enable(1 if on else 0)


def profile_reset():
    _lib().msf_profile_reset()


def profile_read():
    """{kernel family: {"launches", "ms", "bytes"}} accumulated since the last reset."""
    buf = (KernelProfile * 64)()
    k = _lib().msf_profile_read(buf, 64)
    return {buf[i].name.decode(): {"launches": int(buf[i].launches), "ms": float(buf[i].total_ms),
                                   "bytes": float(buf[i].bytes)} for i in range(k)}


def make_batch_options(block=0, lds_vertices=0, workgroups=0, coop_edges=0, wave_edges=0,
                       hot_min=0, wave_min=0):
    o = BatchOptions()
    o.block, o.lds_vertices, o.workgroups = int(block), int(lds_vertices), int(workgroups)
    o.coop_edges, o.wave_edges = int(coop_edges), int(wave_edges)
    o.hot_min, o.wave_min = int(hot_min), int(wave_min)
    return o


class Batch:
    """Device buffers of one batch of graphs plus the batched entry points.

    u, v, w: concatenated int32 CUDA tensors with LOCAL vertex ids per graph;
    edge_off, vert_off: int64 offsets (numpy or CUDA tensors) of length G + 1.
    order defaults to largest graph first (by edge count).
    """

    def __init__(self, u, v, w, edge_off, vert_off, order="largest_first", options=None):
        import numpy as np
        self.lib = _lib()
        self.u, self.v, self.w = _dev_i32(u, "u"), _dev_i32(v, "v"), _dev_i32(w, "w")
        dev = self.u.device
        eo = np.asarray(edge_off.cpu() if isinstance(edge_off, torch.Tensor) else edge_off,
                        np.int64)
        vo = np.asarray(vert_off.cpu() if isinstance(vert_off, torch.Tensor) else vert_off,
                        np.int64)
        self.G = len(eo) - 1
        self.max_n = int((vo[1:] - vo[:-1]).max()) if self.G > 0 else 0
        self.eoff = torch.from_numpy(eo).to(dev)
        self.voff = torch.from_numpy(vo).to(dev)
        if order == "largest_first":
            o = np.argsort(-(eo[1:] - eo[:-1]), kind="stable").astype(np.int32)
            self.order = torch.from_numpy(o).to(dev)
        elif order is None:
            self.order = None
        else:
            self.order = torch.as_tensor(order, dtype=torch.int32, device=dev)
        self.options = options if options is not None else make_batch_options()
        m = int(eo[-1]) if self.G > 0 else 0
        self.mask = torch.empty(max(m, 1), dtype=torch.uint8, device=dev)
        self.totals = torch.empty(max(self.G, 1), dtype=torch.int64, device=dev)
        # [g] finish, [G] batch start, [G + 1 + g] start of graph g
        self.ticks = torch.empty(2 * self.G + 1, dtype=torch.int64, device=dev)
        need = max(int(self.lib.msf_batched_workspace_bytes(self.G, self.max_n, None)),
                   int(self.lib.msf_batched_workspace_bytes(self.G, self.max_n,
                                                           ctypes.byref(self.options))))
        self.workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        self._graph = None

    def _args(self):
        return (self.u.data_ptr(), self.v.data_ptr(), self.w.data_ptr(), self.eoff.data_ptr(),
                self.voff.data_ptr(), self.G, self.max_n,
                self.order.data_ptr() if self.order is not None else None,
                self.mask.data_ptr(), self.totals.data_ptr())

    def launch(self, stream=None):
        """Stream-ordered launch (no synchronisation)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.u.device)
        rc = self.lib.msf_compute_batched(*self._args(), self.ticks.data_ptr(),
                                          self.workspace.data_ptr(), self.workspace.numel(),
                                          ctypes.c_void_p(s.cuda_stream),
                                          ctypes.byref(self.options))
        if rc != OK:
            raise MSFError(rc, self.lib.msf_last_error().decode(errors="replace"))

    def capture(self):
        """Captures the launch into a hipGraph once; returns self."""
        if self._graph is None:
            h = ctypes.c_void_p()
            rc = self.lib.msf_batched_graph_create(*self._args(), self.ticks.data_ptr(),
                                                   self.workspace.data_ptr(),
                                                   self.workspace.numel(),
                                                   ctypes.byref(self.options), ctypes.byref(h))
            if rc != OK:
                raise MSFError(rc, self.lib.msf_last_error().decode(errors="replace"))
            self._graph = h
        return self

    def replay(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.u.device)
        rc = self.lib.msf_batched_graph_launch(self._graph, ctypes.c_void_p(s.cuda_stream))
        if rc != OK:
            raise MSFError(rc, self.lib.msf_last_error().decode(errors="replace"))

    def autotune(self, stream=None):
        """Times every candidate configuration; adopts and returns the fastest."""
        s = stream if stream is not None else torch.cuda.current_stream(self.u.device)
        best = BatchOptions()
        ms = ctypes.c_float()
        rc = self.lib.msf_batched_autotune(*self._args(), self.workspace.data_ptr(),
                                           self.workspace.numel(), ctypes.c_void_p(s.cuda_stream),
                                           ctypes.byref(best), ctypes.byref(ms))
        if rc != OK:
            raise MSFError(rc, self.lib.msf_last_error().decode(errors="replace"))
        self.options = best
        if self._graph is not None:
            self.close()
        return {"block": best.block, "lds_vertices": best.lds_vertices,
                "coop_edges": best.coop_edges, "wave_edges": best.wave_edges,
                "hot_min": best.hot_min, "wave_min": best.wave_min, "ms": ms.value}

    def close(self):
        if self._graph is not None:
            self.lib.msf_batched_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- pivot network

MLP_IN, MLP_H = 16, 64
MLP_PARAMS = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1
MODEL_MAGIC, MODEL_VERSION = 0x5046534d, 1
DEFAULT_MODEL = os.path.join(_HERE, "data", "pivot_mlp.bin")


def init_pivot_params(seed=0):
    """He-initialised FP32 network parameters (biases zero), flat in the
    load layout W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, (2.0 / MLP_IN) ** 0.5, MLP_H * MLP_IN), np.zeros(MLP_H),
             rng.normal(0, (2.0 / MLP_H) ** 0.5, MLP_H * MLP_H), np.zeros(MLP_H),
             rng.normal(0, (1.0 / MLP_H) ** 0.5, MLP_H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def model_blob(params):
    """Serialises FP32 parameters (length MLP_PARAMS) into the load format."""
    import numpy as np
    p = np.ascontiguousarray(params, np.float32)
    if p.shape != (MLP_PARAMS,):
        raise ValueError(f"expected {MLP_PARAMS} parameters")
    hdr = np.array([MODEL_MAGIC, MODEL_VERSION, MLP_IN, MLP_H], np.uint32)
    return hdr.tobytes() + p.tobytes()


def load_pivot_model(blob_or_path=None):
    """Loads a pivot network (bytes or a file path; default: the shipped one)."""
    if blob_or_path is None:
        blob_or_path = DEFAULT_MODEL
    blob = open(blob_or_path, "rb").read() if isinstance(blob_or_path, str) else bytes(blob_or_path)
    buf = ctypes.create_string_buffer(blob, len(blob))
    rc = _lib().msf_pivot_model_load(buf, len(blob))
    if rc != OK:
        raise MSFError(rc, "bad pivot model")


def clear_pivot_model():
    _lib().msf_pivot_model_clear()


def pivot_model_loaded():
    return bool(_lib().msf_pivot_model_loaded())


def mlp_forward(params, x, bf16=True):
    """params: FP32 CUDA tensor [MLP_PARAMS]; x: FP32 CUDA tensor [B, 16] -> z [B]."""
    B = x.shape[0]
    z = torch.empty(B, dtype=torch.float32, device=x.device)
    s = torch.cuda.current_stream(x.device)
    rc = _lib().msf_mlp_forward(params.data_ptr(), x.contiguous().data_ptr(), B, z.data_ptr(),
                                1 if bf16 else 0, ctypes.c_void_p(s.cuda_stream))
    if rc != OK:
        raise MSFError(rc)
    return z


def mlp_grad(params, x, target, bf16=True):
    """Gradient of mean (z - target)^2 / 2; returns (grad [MLP_PARAMS], loss tensor [1])."""
    B = x.shape[0]
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    s = torch.cuda.current_stream(x.device)
    rc = _lib().msf_mlp_grad(params.data_ptr(), x.contiguous().data_ptr(),
                             target.contiguous().data_ptr(), B, 1 if bf16 else 0, g.data_ptr(),
                             loss.data_ptr(), ctypes.c_void_p(s.cuda_stream))
    if rc != OK:
        raise MSFError(rc)
    return g, loss


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    s = torch.cuda.current_stream(params.device)
    rc = _lib().msf_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), lr,
                             beta1, beta2, eps, step, ctypes.c_void_p(s.cuda_stream))
    if rc != OK:
        raise MSFError(rc)


def wall_clock_khz():
    return int(_lib().msf_wall_clock_khz())


def compute_raw(u_ptr, v_ptr, w_ptr, m, n, mask_ptr, workspace_ptr=0, workspace_bytes=0,
                stream=0, options=None, stats=None):
    """Direct C-ABI call on raw device pointers; returns (status, total)."""
    total = ctypes.c_uint64(0)
    rc = _lib().msf_compute(u_ptr, v_ptr, w_ptr, int(m), int(n), mask_ptr, ctypes.byref(total),
                            workspace_ptr or None, int(workspace_bytes), stream or None,
                            ctypes.byref(options) if options is not None else None,
                            ctypes.byref(stats) if stats is not None else None)
    return rc, int(total.value)
