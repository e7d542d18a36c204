"""Thin ctypes binding of the C ABI in include/ldpc.h (argument marshalling only).

Every step of decoding runs in the HIP kernels of libldpc_hip.so; this module
only converts Python/PyTorch arguments to pointers and sizes.  PyTorch is used
for device memory and streams.  There is no fallback: if the library is
missing the import of this module's functions raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libldpc_hip.so")

# status codes (ldpc_status)
OK, E_INVAL, E_RANGE, E_DUP_EDGE, E_NOMEM, E_DEVICE, E_UNSUPPORTED = range(7)
# decode flags
NO_EARLY_STOP = 1 << 0
MSG_FP16 = 1 << 1
MSG_BF16 = 1 << 2
MSG_Q8 = 1 << 6          # 8-bit fixed-point messages: steps of 1/2, saturating at +-63.5
LANE_SLOTS_1 = 1 << 3
LANE_SLOTS_2 = 1 << 4
LANE_SLOTS_4 = 1 << 5
COMPACT_TAIL = 1 << 7    # decode/simulate: move the last running frames into smaller slot ranges (device-driven)
# graph flags
GRAPH_HOST_ONLY = 1 << 0

EXPORTED = ("ldpc_graph_create", "ldpc_graph_create_qc", "ldpc_graph_destroy", "ldpc_graph_info", "ldpc_graph_arrays",
            "ldpc_decode_workspace_size", "ldpc_decode", "ldpc_decode_rule", "ldpc_decode_profiled",
            "ldpc_decode_noalloc", "ldpc_simulate_workspace_size", "ldpc_simulate", "ldpc_simulate_rule",
            "ldpc_status_str", "ldpc_last_error", "ldpc_engine_create", "ldpc_engine_destroy", "ldpc_engine_info",
            "ldpc_engine_submit", "ldpc_engine_capacity", "ldpc_engine_step", "ldpc_engine_poll",
            "ldpc_engine_run", "ldpc_engine_stream", "ldpc_engine_autotune", "ldpc_server_create", "ldpc_server_submit",
            "ldpc_server_poll", "ldpc_server_result", "ldpc_server_stats", "ldpc_server_destroy")


class Frame(ctypes.Structure):
    """ldpc_frame: device pointers of one queued frame."""
    _fields_ = [("llr", ctypes.c_void_p), ("bits", ctypes.c_void_p), ("ok", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("llr_out", ctypes.c_void_p), ("done", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("lane_slots", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("max_requests", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("rule_param", ctypes.c_float), ("iters_per_step", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Rule(ctypes.Structure):
    """ldpc_rule: check rule kind and parameter."""
    _fields_ = [("kind", ctypes.c_int32), ("param", ctypes.c_float), ("reserved", ctypes.c_int32 * 2)]


# check rules by name: (kind, default parameter); "ms" is the normalized rule with alpha = 1
RULE_SUM_PRODUCT, RULE_MIN_SUM_NORMALIZED, RULE_MIN_SUM_OFFSET = 0, 1, 2
RULES = {"sp": (RULE_SUM_PRODUCT, 0.0), "ms": (RULE_MIN_SUM_NORMALIZED, 1.0),
         "nms": (RULE_MIN_SUM_NORMALIZED, 0.75), "oms": (RULE_MIN_SUM_OFFSET, 0.25)}


def make_rule(rule=None, param=None):
    """A Rule from a name in RULES (None: sum-product) and an optional parameter."""
    if isinstance(rule, Rule):
        return rule
    kind, default = RULES["sp" if rule is None else rule]
    return Rule(kind, default if (param is None or rule == "ms") else float(param))


class EngineOpts(ctypes.Structure):
    _fields_ = [("lane_slots", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("no_compaction", ctypes.c_int32), ("iters_per_step", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("rule_param", ctypes.c_float), ("reserved", ctypes.c_int32 * 2)]


class LdpcError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        super().__init__(f"{func}: {detail} (status {status})")
        self.status = status


_lib = None


def load_library():
    """Load libldpc_hip.so (built in-tree by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: torch ships its own HIP runtime under the same soname
    # (libamdhip64.so.7).  Loaded first, it is the one this library binds to;
    # loaded second, it would be a second runtime that sees no devices.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1609_01567_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.ldpc_graph_create.argtypes = [I32, I32, I64, P, P, U32, ctypes.POINTER(P)]
    lib.ldpc_graph_create_qc.argtypes = [I32, I32, I32, P, U32, ctypes.POINTER(P)]
    lib.ldpc_graph_destroy.argtypes = [P]
    lib.ldpc_graph_info.argtypes = [P, P, P, P, P, P, P]
    lib.ldpc_graph_arrays.argtypes = [P, P, P, P, P, P]
    lib.ldpc_decode_workspace_size.argtypes = [P, I32, U32, ctypes.POINTER(ctypes.c_size_t)]
    lib.ldpc_decode.argtypes = [P, P, I32, I32, U32, P, P, P, P, P, ctypes.c_size_t, P]
    lib.ldpc_decode_rule.argtypes = [P, P, I32, I32, U32, P, P, P, P, P, P, ctypes.c_size_t, P]
    lib.ldpc_decode_profiled.argtypes = [P, P, I32, I32, U32, P, P, P, P, P, ctypes.c_size_t, P, P, P, P]
    lib.ldpc_decode_noalloc.argtypes = [P, P, I32, I32, U32, P, P, P, P, P]
    lib.ldpc_simulate_workspace_size.argtypes = [P, I32, U32, ctypes.POINTER(ctypes.c_size_t)]
    lib.ldpc_simulate.argtypes = [P, I32, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, I32, U32, P, P, P,
                                  ctypes.c_size_t, P]
    lib.ldpc_simulate_rule.argtypes = [P, I32, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, I32, U32, P, P, P,
                                       P, ctypes.c_size_t, P]
    for f in ("ldpc_graph_create", "ldpc_graph_create_qc", "ldpc_graph_destroy", "ldpc_graph_info", "ldpc_graph_arrays",
              "ldpc_decode_workspace_size", "ldpc_decode", "ldpc_decode_rule", "ldpc_decode_profiled",
              "ldpc_decode_noalloc", "ldpc_simulate_workspace_size", "ldpc_simulate", "ldpc_simulate_rule"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ldpc_engine_create.argtypes = [P, I32, P, P, I32, U32, P, ctypes.POINTER(P)]
    lib.ldpc_engine_destroy.argtypes = [P]
    lib.ldpc_engine_info.argtypes = [P, P, P]
    lib.ldpc_engine_submit.argtypes = [P, I32, P, I32, P]
    lib.ldpc_engine_capacity.argtypes = [P, I32, P]
    lib.ldpc_engine_step.argtypes = [P, I32]
    lib.ldpc_engine_poll.argtypes = [P, P, P]
    lib.ldpc_engine_run.argtypes = [P, I32, P]
    lib.ldpc_engine_stream.argtypes = [P, ctypes.POINTER(P)]
    lib.ldpc_engine_autotune.argtypes = [P, I32, P, P, I32, U32, P, P, P]
    lib.ldpc_engine_autotune.restype = ctypes.c_int
    lib.ldpc_server_create.argtypes = [P, I32, P, I32, U32, I64, I64, P, ctypes.POINTER(P)]
    lib.ldpc_server_submit.argtypes = [P, I32, P, I32, ctypes.POINTER(I64)]
    lib.ldpc_server_poll.argtypes = [P, P, I32, ctypes.POINTER(I32), I32]
    lib.ldpc_server_result.argtypes = [P, I64, P, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.ldpc_server_stats.argtypes = [P, P]
    lib.ldpc_server_destroy.argtypes = [P]
    for f in ("ldpc_server_create", "ldpc_server_submit", "ldpc_server_poll", "ldpc_server_result",
              "ldpc_server_stats", "ldpc_server_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    for f in ("ldpc_engine_create", "ldpc_engine_destroy", "ldpc_engine_info", "ldpc_engine_submit",
              "ldpc_engine_capacity", "ldpc_engine_step", "ldpc_engine_poll", "ldpc_engine_run",
              "ldpc_engine_stream"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ldpc_status_str.argtypes = [ctypes.c_int]
    lib.ldpc_status_str.restype = ctypes.c_char_p
    lib.ldpc_last_error.argtypes = []
    lib.ldpc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, func: str):
    if status != OK:
        lib = load_library()
        raise LdpcError(status, func, lib.ldpc_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Graph:
    """Tanner graph of a binary parity-check matrix (ldpc_graph_create)."""

    def __init__(self, m: int, n: int, rows, cols, host_only: bool = False):
        lib = load_library()
        self._lib = lib
        self._h = ctypes.c_void_p()
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        if rows.shape != cols.shape or rows.ndim != 1:
            raise ValueError("rows and cols must be 1-D arrays of equal length")
        _check(lib.ldpc_graph_create(int(m), int(n), rows.size, _np_ptr(rows), _np_ptr(cols),
                                     GRAPH_HOST_ONLY if host_only else 0, ctypes.byref(self._h)),
               "ldpc_graph_create")
        self.m, self.n, self.nnz = int(m), int(n), int(rows.size)
        self.host_only = host_only

    @classmethod
    def from_code(cls, code, host_only: bool = False) -> "Graph":
        return cls(code.m, code.n, code.rows, code.cols, host_only=host_only)

    @classmethod
    def from_qc(cls, Z: int, shifts, host_only: bool = False) -> "Graph":
        """ldpc_graph_create_qc: the code lifted from an [mb][nb] shift table (-1: zero block) by Z."""
        shifts = np.ascontiguousarray(shifts, dtype=np.int32)
        if shifts.ndim != 2:
            raise ValueError("shifts must be a 2-D [mb][nb] array")
        self = cls.__new__(cls)
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        mb, nb = shifts.shape
        _check(self._lib.ldpc_graph_create_qc(int(mb), int(nb), int(Z), _np_ptr(shifts),
                                              GRAPH_HOST_ONLY if host_only else 0, ctypes.byref(self._h)),
               "ldpc_graph_create_qc")
        self.m, self.n, self.nnz = int(mb * Z), int(nb * Z), int((shifts >= 0).sum()) * int(Z)
        self.host_only = host_only
        return self

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph has been closed")
        return self._h

    def info(self) -> dict:
        vals = [ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(),
                ctypes.c_int64()]
        _check(self._lib.ldpc_graph_info(self.handle, *[ctypes.byref(v) for v in vals]), "ldpc_graph_info")
        keys = ("m", "n", "nnz", "max_check_deg", "max_bit_deg", "device_bytes")
        return {k: int(v.value) for k, v in zip(keys, vals)}

    def arrays(self) -> dict:
        out = dict(row_ptr=np.zeros(self.m + 1, np.int32), col_idx=np.zeros(self.nnz, np.int32),
                   col_ptr=np.zeros(self.n + 1, np.int32), row_idx=np.zeros(self.nnz, np.int32),
                   csr_to_csc=np.zeros(self.nnz, np.int32))
        _check(self._lib.ldpc_graph_arrays(self.handle, *[_np_ptr(out[k]) for k in
                                                          ("row_ptr", "col_idx", "col_ptr", "row_idx", "csr_to_csc")]),
               "ldpc_graph_arrays")
        return out

    def close(self):
        if self._h:
            self._lib.ldpc_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(graph: Graph, frames: int, flags: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(graph._lib.ldpc_decode_workspace_size(graph.handle, int(frames), int(flags), ctypes.byref(out)),
           "ldpc_decode_workspace_size")
    return int(out.value)


@dataclasses.dataclass
class DecodeResult:
    bits: "object"     # torch.uint8 [F][n] on the device
    ok: "object"       # torch.uint8 [F]
    iters: "object"    # torch.int32 [F]
    llr: "object"      # torch.float32 [F][n] or None


class Workspace:
    """Caller-owned device workspace (a torch uint8 tensor, 256-byte aligned)."""

    def __init__(self, nbytes: int, device=None):
        import torch
        self.nbytes = int(nbytes)
        self._t = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        base = self._t.data_ptr()
        self.ptr = (base + 255) // 256 * 256

    def fits(self, nbytes: int) -> bool:
        return nbytes <= self.nbytes


def _prepare(graph: Graph, llr, flags: int, want_llr: bool, workspace, stream, out):
    import torch
    if llr.dtype != torch.float32 or not llr.is_cuda or llr.dim() != 2 or not llr.is_contiguous():
        raise ValueError("llr must be a contiguous float32 CUDA tensor [frames][n]")
    F, n = llr.shape
    if n != graph.n:
        raise ValueError("llr width does not match the graph")
    dev = llr.device
    if out is None:
        out = DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device=dev),
                           ok=torch.empty(F, dtype=torch.uint8, device=dev),
                           iters=torch.empty(F, dtype=torch.int32, device=dev),
                           llr=torch.empty((F, n), dtype=torch.float32, device=dev) if want_llr else None)
    need = workspace_size(graph, F, flags)
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    args = (graph.handle, ctypes.c_void_p(llr.data_ptr()), int(F))
    outs = (ctypes.c_void_p(out.bits.data_ptr()), ctypes.c_void_p(out.ok.data_ptr()),
            ctypes.c_void_p(out.iters.data_ptr()),
            ctypes.c_void_p(out.llr.data_ptr()) if out.llr is not None else None,
            ctypes.c_void_p(workspace.ptr), ctypes.c_size_t(workspace.nbytes),
            ctypes.c_void_p(stream.cuda_stream))
    return out, workspace, args, outs


def decode(graph: Graph, llr, max_iter: int, flags: int = 0, want_llr: bool = False,
           workspace: Workspace | None = None, stream=None, out: DecodeResult | None = None, rule=None,
           rule_param=None) -> DecodeResult:
    """Enqueue ldpc_decode on `stream` (default: torch's current stream) and return the output tensors.

    `llr` is a contiguous float32 CUDA tensor [F][n].  The call does not
    synchronize; read the outputs after the stream reaches this point (torch
    does that for you when you use them on the same stream).  `rule` selects
    the check rule by name ("sp", "ms", "nms", "oms"; None is sum-product) with
    an optional `rule_param`; any rule goes through ldpc_decode_rule.
    """
    out, workspace, args, outs = _prepare(graph, llr, flags, want_llr, workspace, stream, out)
    if rule is None:
        _check(graph._lib.ldpc_decode(*args, int(max_iter), int(flags), *outs), "ldpc_decode")
    else:
        r = make_rule(rule, rule_param)
        _check(graph._lib.ldpc_decode_rule(*args, int(max_iter), int(flags), ctypes.byref(r), *outs),
               "ldpc_decode_rule")
    out._workspace = workspace   # keep the workspace alive until the stream has consumed it
    return out


def decode_profiled(graph: Graph, llr, max_iter: int, flags: int = 0, want_llr: bool = False,
                    workspace: Workspace | None = None, stream=None, out: DecodeResult | None = None):
    """ldpc_decode_profiled: decode, wait, and return (result, timings in ms)."""
    out, workspace, args, outs = _prepare(graph, llr, flags, want_llr, workspace, stream, out)
    check_ms = np.zeros(max_iter, np.float32)
    bit_ms = np.zeros(max_iter, np.float32)
    edge_ms = np.zeros(2, np.float32)
    _check(graph._lib.ldpc_decode_profiled(*args, int(max_iter), int(flags), *outs, _np_ptr(check_ms),
                                           _np_ptr(bit_ms), _np_ptr(edge_ms)), "ldpc_decode_profiled")
    out._workspace = workspace
    return out, dict(check_ms=check_ms, bit_ms=bit_ms, edge_ms=edge_ms)


# bytes of the library's static per-device decode state (ldpc_decode_noalloc)
NOALLOC_SCRATCH_BYTES = 128 << 20


def decode_noalloc(graph: Graph, llr, max_iter: int, flags: int = 0, want_llr: bool = False, stream=None,
                   out: DecodeResult | None = None) -> DecodeResult:
    """Enqueue ldpc_decode_noalloc: the decode state lives in the library's static device array.

    Pass preallocated `out` tensors to keep the call free of allocation.  Calls
    on one device share that array: serialize them (e.g. on one stream).
    """
    import torch
    if llr.dtype != torch.float32 or not llr.is_cuda or llr.dim() != 2 or not llr.is_contiguous():
        raise ValueError("llr must be a contiguous float32 CUDA tensor [frames][n]")
    F, n = llr.shape
    if n != graph.n:
        raise ValueError("llr width does not match the graph")
    dev = llr.device
    if out is None:
        out = DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device=dev),
                           ok=torch.empty(F, dtype=torch.uint8, device=dev),
                           iters=torch.empty(F, dtype=torch.int32, device=dev),
                           llr=torch.empty((F, n), dtype=torch.float32, device=dev) if want_llr else None)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    _check(graph._lib.ldpc_decode_noalloc(
        graph.handle, ctypes.c_void_p(llr.data_ptr()), int(F), int(max_iter), int(flags),
        ctypes.c_void_p(out.bits.data_ptr()), ctypes.c_void_p(out.ok.data_ptr()),
        ctypes.c_void_p(out.iters.data_ptr()),
        ctypes.c_void_p(out.llr.data_ptr()) if out.llr is not None else None,
        ctypes.c_void_p(stream.cuda_stream)), "ldpc_decode_noalloc")
    return out


SIM_FIELDS = ("frames", "frame_errors", "bit_errors", "undetected", "iterations")


def simulate_workspace_size(graph: Graph, frames: int, flags: int = 0) -> int:
    n = ctypes.c_size_t()
    _check(graph._lib.ldpc_simulate_workspace_size(graph.handle, int(frames), int(flags), ctypes.byref(n)),
           "ldpc_simulate_workspace_size")
    return int(n.value)


def simulate(graph: Graph, frames: int, ebn0_db: float, seed: int, max_iter: int, flags: int = 0,
             first_frame: int = 0, counts=None, want_llr: bool = False, workspace: Workspace | None = None,
             stream=None, rule=None, rule_param=None):
    """Enqueue ldpc_simulate (all-zero codeword over BPSK/AWGN, noise drawn on the device).

    `counts` is a CUDA int64 tensor of 5 counters (SIM_FIELDS), added to;
    a zeroed one is made when None.  Returns (counts, llr or None); read them
    after the stream reaches this point.  `rule` / `rule_param` as in decode()
    (through ldpc_simulate_rule).
    """
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    if counts is None:
        counts = torch.zeros(len(SIM_FIELDS), dtype=torch.int64, device=dev)
    if counts.dtype != torch.int64 or not counts.is_cuda or counts.numel() != len(SIM_FIELDS):
        raise ValueError("counts must be a CUDA int64 tensor of 5 counters")
    llr = torch.empty((frames, graph.n), dtype=torch.float32, device=dev) if want_llr else None
    need = simulate_workspace_size(graph, frames, flags)
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    head = (graph.handle, int(frames), float(ebn0_db), int(seed) & (2 ** 64 - 1), int(first_frame), int(max_iter),
            int(flags))
    tail = (ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(llr.data_ptr()) if llr is not None else None,
            ctypes.c_void_p(workspace.ptr), ctypes.c_size_t(workspace.nbytes), ctypes.c_void_p(stream.cuda_stream))
    if rule is None:
        _check(graph._lib.ldpc_simulate(*head, *tail), "ldpc_simulate")
    else:
        r = make_rule(rule, rule_param)
        _check(graph._lib.ldpc_simulate_rule(*head, ctypes.byref(r), *tail), "ldpc_simulate_rule")
    counts._workspace = workspace   # keep the workspace alive until the stream has consumed it
    return counts, llr


def sim_counts(counts) -> dict:
    """The 5 counters of a simulate() run as a dict (synchronizes on the tensor)."""
    return dict(zip(SIM_FIELDS, (int(x) for x in counts.cpu().tolist())))


class Engine:
    """Batched decoder with continuous refill (ldpc_engine_*) over several graphs."""

    def __init__(self, graphs, slots, queue_cap, max_iter: int, flags: int = 0, lane_slots: int = 0,
                 graph_steps: int = 0, repack: bool = True, iters_per_step: int = 0, rule=None, rule_param=None):
        lib = load_library()
        self._lib = lib
        self.graphs = list(graphs)
        ng = len(self.graphs)
        hs = (ctypes.c_void_p * ng)(*[g.handle.value for g in self.graphs])
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        qc = np.ascontiguousarray(queue_cap, dtype=np.int32)
        if sl.size != ng or qc.size != ng:
            raise ValueError("one slot count and one queue capacity per graph")
        r = make_rule(rule, rule_param)
        opts = EngineOpts(lane_slots, graph_steps, 0 if repack else 1, iters_per_step, r.kind, r.param)
        self._h = ctypes.c_void_p()
        _check(lib.ldpc_engine_create(hs, ng, _np_ptr(sl), _np_ptr(qc), int(max_iter), int(flags),
                                      ctypes.byref(opts), ctypes.byref(self._h)), "ldpc_engine_create")
        self.max_iter, self.flags, self.ngraphs = int(max_iter), int(flags), ng
        self._keep = []   # tensors referenced by queued frames

    @property
    def handle(self):
        if not self._h:
            raise ValueError("engine has been closed")
        return self._h

    def info(self) -> dict:
        b = ctypes.c_int64()
        sl = np.zeros(self.ngraphs, np.int32)
        _check(self._lib.ldpc_engine_info(self.handle, ctypes.byref(b), _np_ptr(sl)), "ldpc_engine_info")
        return {"device_bytes": int(b.value), "slots": sl.tolist()}

    def capacity(self, graph: int) -> int:
        v = ctypes.c_int32()
        _check(self._lib.ldpc_engine_capacity(self.handle, int(graph), ctypes.byref(v)), "ldpc_engine_capacity")
        return int(v.value)

    def submit(self, graph: int, frames, stream=None):
        """Queue frames: a sequence of Frame structs (device pointers)."""
        arr = (Frame * len(frames))(*frames)
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self._lib.ldpc_engine_submit(self.handle, int(graph), arr, len(frames), st), "ldpc_engine_submit")

    def step(self, replays: int = 1):
        _check(self._lib.ldpc_engine_step(self.handle, int(replays)), "ldpc_engine_step")

    def poll(self):
        r = np.zeros(self.ngraphs, np.int64)
        p = np.zeros(self.ngraphs, np.int64)
        _check(self._lib.ldpc_engine_poll(self.handle, _np_ptr(r), _np_ptr(p)), "ldpc_engine_poll")
        return r, p

    def run(self, max_replays: int = 0) -> int:
        n = ctypes.c_int64()
        _check(self._lib.ldpc_engine_run(self.handle, int(max_replays), ctypes.byref(n)), "ldpc_engine_run")
        self._keep.clear()
        return int(n.value)

    def close(self):
        if self._h:
            self._lib.ldpc_engine_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def frames_for(llr, bits, ok, iters, llr_out=None, done=None):
    """Frame descriptors for row f of [F][n] tensors (outputs preallocated)."""
    F, n = llr.shape
    out = []
    for f in range(F):
        out.append(Frame(llr.data_ptr() + 4 * n * f, bits.data_ptr() + n * f, ok.data_ptr() + f,
                         iters.data_ptr() + 4 * f,
                         (llr_out.data_ptr() + 4 * n * f) if llr_out is not None else None,
                         done.data_ptr() if done is not None else None))
    return out


def decode_batch(engine: Engine, jobs, want_llr: bool = False, max_replays: int = 0):
    """Decode jobs [(graph_index, llr [F][n] float32 CUDA tensor), ...] with `engine`.

    Every frame is queued (the queues must hold them), the engine runs until
    all have finished (or max_replays replays; then LdpcError), and one
    DecodeResult per job is returned.
    """
    import torch
    torch.cuda.synchronize()
    results = []
    for gi, llr in jobs:
        if llr.dtype != torch.float32 or not llr.is_cuda or llr.dim() != 2 or not llr.is_contiguous():
            raise ValueError("llr must be a contiguous float32 CUDA tensor [frames][n]")
        F, n = llr.shape
        if n != engine.graphs[gi].n:
            raise ValueError("llr width does not match the graph")
        res = DecodeResult(bits=torch.empty((F, n), dtype=torch.uint8, device=llr.device),
                           ok=torch.empty(F, dtype=torch.uint8, device=llr.device),
                           iters=torch.empty(F, dtype=torch.int32, device=llr.device),
                           llr=torch.empty((F, n), dtype=torch.float32, device=llr.device) if want_llr else None)
        engine.submit(gi, frames_for(llr, res.bits, res.ok, res.iters, res.llr))
        results.append(res)
    engine.run(max_replays)
    _, pending = engine.poll()
    if pending.any():
        raise LdpcError(E_DEVICE, "decode_batch", f"frames still pending after {max_replays} replays: {pending}")
    return results


def autotune(graphs, frame_lists, max_iter: int, flags: int = 0) -> dict:
    """ldpc_engine_autotune over the given frames (lists of Frame per graph)."""
    lib = load_library()
    ng = len(graphs)
    hs = (ctypes.c_void_p * ng)(*[g.handle.value for g in graphs])
    arrays = [(Frame * len(fl))(*fl) for fl in frame_lists]
    ptrs = (ctypes.c_void_p * ng)(*[ctypes.cast(a, ctypes.c_void_p).value for a in arrays])
    counts = np.array([len(fl) for fl in frame_lists], np.int32)
    slots = np.zeros(ng, np.int32)
    opts = EngineOpts()
    ms = ctypes.c_float()
    _check(lib.ldpc_engine_autotune(hs, ng, ptrs, _np_ptr(counts), int(max_iter), int(flags), _np_ptr(slots),
                                    ctypes.byref(opts), ctypes.byref(ms)), "ldpc_engine_autotune")
    return {"slots": slots.tolist(), "lane_slots": int(opts.lane_slots), "graph_steps": int(opts.graph_steps),
            "iters_per_step": int(opts.iters_per_step), "ms": float(ms.value)}


class Server:
    """Request-serving loop (ldpc_server_*): host LLRs in, host results out."""

    STAT_KEYS = ("submitted", "admitted", "completed", "frames_completed", "waiting", "in_flight",
                 "device_bytes_in_use", "device_bytes_peak")

    def __init__(self, graphs, slots, max_iter: int, flags: int = 0, hbm_budget: int = 1 << 30,
                 host_budget: int = 1 << 28, lane_slots: int = 0, graph_steps: int = 0, max_requests: int = 0,
                 rule=None, rule_param=None, iters_per_step: int = 0):
        lib = load_library()
        self._lib = lib
        self.graphs = list(graphs)
        ng = len(self.graphs)
        hs = (ctypes.c_void_p * ng)(*[g.handle.value for g in self.graphs])
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        r = make_rule(rule, rule_param)
        opts = ServerOpts(lane_slots, graph_steps, max_requests, r.kind, r.param, iters_per_step)
        self._h = ctypes.c_void_p()
        _check(lib.ldpc_server_create(hs, ng, _np_ptr(sl), int(max_iter), int(flags), int(hbm_budget),
                                      int(host_budget), ctypes.byref(opts), ctypes.byref(self._h)),
               "ldpc_server_create")
        self._frames = {}

    def submit(self, graph: int, llr: np.ndarray) -> int:
        llr = np.ascontiguousarray(llr, dtype=np.float32)
        if llr.ndim != 2 or llr.shape[1] != self.graphs[graph].n:
            raise ValueError("llr must be [frames][n] for the graph")
        rid = ctypes.c_int64()
        _check(self._lib.ldpc_server_submit(self._h, int(graph), _np_ptr(llr), llr.shape[0], ctypes.byref(rid)),
               "ldpc_server_submit")
        self._frames[int(rid.value)] = (llr.shape[0], self.graphs[graph].n)
        return int(rid.value)

    def poll(self, wait_ms: int = 0, max_ids: int = 4096):
        ids = np.zeros(max_ids, np.int64)
        cnt = ctypes.c_int32()
        _check(self._lib.ldpc_server_poll(self._h, _np_ptr(ids), max_ids, ctypes.byref(cnt), int(wait_ms)),
               "ldpc_server_poll")
        return ids[: cnt.value].tolist()

    def result(self, rid: int, want_bits: bool = True):
        """(bits [F][n] or None, ok [F], iters [F], latency seconds); releases the request."""
        F, n = self._frames.pop(rid)
        bits = np.zeros((F, n), np.uint8) if want_bits else None
        ok = np.zeros(F, np.uint8)
        iters = np.zeros(F, np.int32)
        lat = ctypes.c_double()
        _check(self._lib.ldpc_server_result(self._h, int(rid), _np_ptr(bits) if want_bits else None, _np_ptr(ok),
                                            _np_ptr(iters), ctypes.byref(lat)), "ldpc_server_result")
        return bits, ok, iters, float(lat.value)

    def stats(self) -> dict:
        st = np.zeros(8, np.int64)
        _check(self._lib.ldpc_server_stats(self._h, _np_ptr(st)), "ldpc_server_stats")
        return dict(zip(self.STAT_KEYS, st.tolist()))

    def close(self):
        if self._h:
            self._lib.ldpc_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
