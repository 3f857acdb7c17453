"""ctypes binding of ``libhyperflow.so`` (C ABI in ``include/hyperflow.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Inputs may be numpy arrays (host memory) or torch CUDA/HIP tensors
(device memory, passed by ``data_ptr()``); PyTorch is used only for device
memory and streams.  There is no fallback: if the library is missing the
first call raises.

The C entry points are exposed under their own names
(``flow_problem_create``, ``maxflow_solve``, ``mincut_source_side``,
``flow_batch_solve``, ``flow_batch_create``, ``flow_batch_run``,
``flow_batch_tune``, ``flow_batch_get_config``, ``flow_batch_destroy``,
``flow_problem_reset``, ``flow_problem_sink_side``, ``flow_problem_pierce``,
``flow_problem_flowcutter``, ``flow_problem_stats``,
``flow_problem_kernel_times``, ``flow_problem_destroy``, ``fp_last_error``)
plus small owner classes :class:`FlowProblem` and :class:`FlowBatch`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhyperflow.so")

FP_OK = 0
STATUS = {
    0: "FP_OK",
    -1: "FP_ERR_INVALID",
    -2: "FP_ERR_OVERFLOW",
    -3: "FP_ERR_STATE",
    -4: "FP_ERR_DEVICE",
    -5: "FP_ERR_OOM",
    -6: "FP_ERR_ABORTED",
}


class HyperflowError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class Options(ctypes.Structure):
    _fields_ = [
        ("relabel_factor_x16", ctypes.c_int32),
        ("round_budget", ctypes.c_int32),
        ("debug_checks", ctypes.c_int32),
        ("tail_threshold", ctypes.c_int32),
        ("group_lanes", ctypes.c_int32),
        ("big_degree", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("gr_interval", ctypes.c_int32),
        ("stale_rounds", ctypes.c_int32),
        ("bottom_up_min", ctypes.c_int32),
        ("bfs_arc_parallel", ctypes.c_int32),
        ("pull_min", ctypes.c_int32),
        ("tail_gr_interval", ctypes.c_int32),
        ("bfs_flat", ctypes.c_int32),
        ("bfs_marks", ctypes.c_int32),
        ("relabel_blocking", ctypes.c_int32),
        ("bfs_xcd", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int64),
        ("tail_rounds", ctypes.c_int64),
        ("relabels", ctypes.c_int64),
        ("global_relabels", ctypes.c_int64),
        ("bfs_levels", ctypes.c_int64),
        ("restarts", ctypes.c_int64),
        ("host_syncs", ctypes.c_int64),
        ("flow_value", ctypes.c_int64),
        ("alg_bytes", ctypes.c_int64),
        ("reserved", ctypes.c_int64 * 7),
    ]


class BatchConfig(ctypes.Structure):
    _fields_ = [
        ("group_lanes", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("gr_interval", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
        ("streams", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("union_pins", ctypes.c_int32),
        ("wg_threads", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if not k.startswith("reserved")}


class CutterResult(ctypes.Structure):
    _fields_ = [
        ("flow", ctypes.c_int64),
        ("source_weight", ctypes.c_int64),
        ("sink_weight", ctypes.c_int64),
        ("iterations", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("side", ctypes.c_int32),
        ("augmenting", ctypes.c_int32),
        ("first_balanced", ctypes.c_int32),
        ("slice_iterations", ctypes.c_int32),
        ("resumable", ctypes.c_int32),
        ("reserved32", ctypes.c_int32),
        ("reserved", ctypes.c_int64 * 2),
    ]


class CutterStep(ctypes.Structure):
    _fields_ = [
        ("side", ctypes.c_int32),
        ("node", ctypes.c_int32),
        ("flow", ctypes.c_int64),
        ("source_weight", ctypes.c_int64),
        ("sink_weight", ctypes.c_int64),
        ("count", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


CUTTER_STATUS = {0: "balanced", 1: "infeasible", 2: "cap"}

EXPORTED = [
    "flow_problem_create",
    "maxflow_solve",
    "mincut_source_side",
    "flow_batch_solve",
    "flow_batch_create",
    "flow_batch_run",
    "flow_batch_tune",
    "flow_batch_get_config",
    "flow_batch_destroy",
    "flow_problem_reset",
    "flow_problem_sink_side",
    "flow_problem_pierce",
    "flow_problem_flowcutter",
    "flow_problem_flowcutter_continue",
    "flow_problem_terminals",
    "flow_problem_stats",
    "flow_problem_kernel_times",
    "flow_problem_export_state",
    "flow_problem_destroy",
    "maxflow_mincut_noalloc",
    "flow_regions_build",
    "flow_regions_info",
    "flow_regions_export",
    "flow_regions_problem",
    "flow_regions_solve",
    "flow_regions_source_side",
    "flow_regions_destroy",
    "flow_partition_create",
    "flow_partition_apply",
    "flow_partition_get",
    "flow_partition_refine",
    "flow_partition_destroy",
    "scorer_create",
    "scorer_fit_normalization",
    "scorer_gradient",
    "scorer_train",
    "scorer_predict",
    "scorer_get_params",
    "scorer_set_params",
    "scorer_destroy",
    "flow_release_cached_memory",
    "fp_last_error",
]

SCORER_PARAMS = 5057

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2201_01556_amd.build`")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.flow_problem_create.argtypes = [i32, i32, vp, vp, vp, vp, i32, vp, i32, i32,
                                        ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    lib.flow_problem_create.restype = ctypes.c_int
    lib.maxflow_solve.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.maxflow_solve.restype = ctypes.c_int
    lib.mincut_source_side.argtypes = [vp, vp, i32, vp, vp]
    lib.mincut_source_side.restype = ctypes.c_int
    lib.flow_batch_solve.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp]
    lib.flow_batch_solve.restype = ctypes.c_int
    lib.flow_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, vp,
                                      ctypes.POINTER(BatchConfig), vp, ctypes.POINTER(vp)]
    lib.flow_batch_create.restype = ctypes.c_int
    lib.flow_batch_run.argtypes = [vp, vp, i32, vp, vp]
    lib.flow_batch_run.restype = ctypes.c_int
    lib.flow_batch_tune.argtypes = [vp, vp, ctypes.c_char_p, ctypes.POINTER(BatchConfig)]
    lib.flow_batch_tune.restype = ctypes.c_int
    lib.flow_batch_get_config.argtypes = [vp, ctypes.POINTER(BatchConfig)]
    lib.flow_batch_get_config.restype = ctypes.c_int
    lib.flow_batch_destroy.argtypes = [vp]
    lib.flow_batch_destroy.restype = None
    lib.flow_problem_reset.argtypes = [vp]
    lib.flow_problem_reset.restype = ctypes.c_int
    lib.flow_problem_pierce.argtypes = [vp, i32, vp, i32, vp]
    lib.flow_problem_pierce.restype = ctypes.c_int
    lib.flow_problem_sink_side.argtypes = [vp, vp, i32, vp]
    lib.flow_problem_sink_side.restype = ctypes.c_int
    lib.flow_problem_flowcutter.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, i32, i32, i32,
                                            vp, i32, vp, ctypes.POINTER(CutterResult), vp]
    lib.flow_problem_flowcutter.restype = ctypes.c_int
    lib.flow_problem_flowcutter_continue.argtypes = [vp, i32, vp, i32, vp,
                                                     ctypes.POINTER(CutterResult), vp]
    lib.flow_problem_flowcutter_continue.restype = ctypes.c_int
    lib.flow_problem_terminals.argtypes = [vp, vp, i32, vp]
    lib.flow_problem_terminals.restype = ctypes.c_int
    lib.flow_problem_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.flow_problem_stats.restype = ctypes.c_int
    lib.flow_problem_kernel_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p),
                                              vp, vp, vp]
    lib.flow_problem_kernel_times.restype = i32
    lib.flow_problem_export_state.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.flow_problem_export_state.restype = ctypes.c_int
    lib.flow_problem_destroy.argtypes = [vp]
    lib.flow_problem_destroy.restype = None
    lib.maxflow_mincut_noalloc.argtypes = [i32, i32, vp, vp, vp, vp, i32, vp, i32, i32, vp,
                                           ctypes.POINTER(ctypes.c_int64), vp, vp]
    lib.maxflow_mincut_noalloc.restype = ctypes.c_int
    lib.flow_regions_build.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, i32, vp, vp, i32, i32,
                                       vp, ctypes.POINTER(vp)]
    lib.flow_regions_build.restype = ctypes.c_int
    lib.flow_regions_info.argtypes = [vp, i32, vp]
    lib.flow_regions_info.restype = ctypes.c_int
    lib.flow_regions_export.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.flow_regions_export.restype = ctypes.c_int
    lib.flow_regions_problem.argtypes = [vp, i32, ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    lib.flow_regions_problem.restype = ctypes.c_int
    lib.flow_regions_solve.argtypes = [vp, vp, vp, vp]
    lib.flow_regions_solve.restype = ctypes.c_int
    lib.flow_regions_source_side.argtypes = [vp, i32, i32, vp, vp]
    lib.flow_regions_source_side.restype = ctypes.c_int
    lib.flow_regions_destroy.argtypes = [vp]
    lib.flow_regions_destroy.restype = None
    lib.flow_partition_create.argtypes = [i32, i32, vp, vp, vp, vp, vp, i32, i32, vp,
                                          ctypes.POINTER(vp)]
    lib.flow_partition_create.restype = ctypes.c_int
    lib.flow_partition_apply.argtypes = [vp, vp, ctypes.POINTER(vp), vp, ctypes.c_int64, vp,
                                         vp, vp, vp]
    lib.flow_partition_apply.restype = ctypes.c_int
    lib.flow_partition_get.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.flow_partition_get.restype = ctypes.c_int
    lib.flow_partition_refine.argtypes = [vp, ctypes.POINTER(RefineConfig), vp,
                                          ctypes.POINTER(RefineResult), vp]
    lib.flow_partition_refine.restype = ctypes.c_int
    lib.flow_partition_destroy.argtypes = [vp]
    lib.flow_partition_destroy.restype = None
    lib.scorer_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
    lib.scorer_create.restype = ctypes.c_int
    lib.scorer_fit_normalization.argtypes = [vp, vp, i32, i32, vp]
    lib.scorer_fit_normalization.restype = ctypes.c_int
    lib.scorer_gradient.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    lib.scorer_gradient.restype = ctypes.c_int
    lib.scorer_train.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp]
    lib.scorer_train.restype = ctypes.c_int
    lib.scorer_predict.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.scorer_predict.restype = ctypes.c_int
    lib.scorer_get_params.argtypes = [vp, vp, vp]
    lib.scorer_get_params.restype = ctypes.c_int
    lib.scorer_set_params.argtypes = [vp, vp, vp]
    lib.scorer_set_params.restype = ctypes.c_int
    lib.scorer_destroy.argtypes = [vp]
    lib.scorer_destroy.restype = None
    lib.fp_last_error.argtypes = []
    lib.fp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def fp_last_error() -> str:
    return load_library().fp_last_error().decode()


def _check(status: int):
    if status != FP_OK:
        raise HyperflowError(status, fp_last_error())


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _is_device_tensor(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, dtype):
    """(pointer, memkind, keepalive) of an int32 / uint8 array or tensor."""
    if _is_device_tensor(a):
        import torch
        want = {np.int32: torch.int32, np.uint8: torch.uint8}[dtype]
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"device tensor must be contiguous {want}")
        return a.data_ptr(), 1, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, 0, arr


def flow_problem_create(num_vertices, net_offsets, pins, net_weights, sources, sinks,
                        options: Options | None = None, stream=None):
    """Create a problem handle; inputs all host (numpy) or all device (torch)."""
    lib = load_library()
    args = [_ptr(a, np.int32) for a in (net_offsets, pins, net_weights, sources, sinks)]
    kinds = {k for _, k, _ in args}
    if len(kinds) != 1:
        raise TypeError("inputs must be all host arrays or all device tensors")
    mem_kind = kinds.pop()
    num_nets = len(net_offsets) - 1
    h = ctypes.c_void_p()
    st = lib.flow_problem_create(int(num_vertices), int(num_nets), args[0][0], args[1][0],
                                 args[2][0], args[3][0], len(sources), args[4][0], len(sinks),
                                 mem_kind, ctypes.byref(options) if options else None,
                                 _stream_ptr(stream), ctypes.byref(h))
    _check(st)
    return h


def maxflow_solve(handle, stream=None) -> int:
    f = ctypes.c_int64()
    _check(load_library().maxflow_solve(handle, _stream_ptr(stream), ctypes.byref(f)))
    return int(f.value)


def mincut_source_side(handle, num_vertices, num_nets, vertex_side=None, net_side=None,
                       stream=None, want_nets=True):
    """Minimal source side.  With no output buffers given, returns host numpy
    arrays (vertex_side, net_side); device tensors are filled in place."""
    lib = load_library()
    if vertex_side is None:
        vertex_side = np.zeros(max(num_vertices, 1), dtype=np.uint8)
        if want_nets and net_side is None:
            net_side = np.zeros(max(num_nets, 1), dtype=np.uint8)
    vp, vk, _ = _ptr(vertex_side, np.uint8)
    np_ = None
    if net_side is not None:
        np_, nk, _ = _ptr(net_side, np.uint8)
        if nk != vk:
            raise TypeError("vertex_side and net_side must be in the same memory")
    _check(lib.mincut_source_side(handle, _stream_ptr(stream), vk, vp, np_))
    if vk == 0:
        vs = np.asarray(vertex_side)[:num_vertices]
        ns = np.asarray(net_side)[:num_nets] if net_side is not None else None
        return vs, ns
    return vertex_side, net_side


def flow_batch_solve(handles, skip=None, stream=None) -> np.ndarray:
    lib = load_library()
    n = len(handles)
    arr = _handle_array(handles)
    flows = np.zeros(max(n, 1), dtype=np.int64)
    sk = None
    if skip is not None:
        skip_arr = np.ascontiguousarray(skip, dtype=np.uint8)
        sk = skip_arr.ctypes.data
    _check(lib.flow_batch_solve(arr, n, sk, _stream_ptr(stream), flows.ctypes.data))
    return flows[:n]


def _handle_array(handles):
    n = len(handles)
    return (ctypes.c_void_p * max(n, 1))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                           for h in handles])


def flow_batch_create(handles, vertex_sides=None, net_sides=None,
                      config: BatchConfig | None = None, stream=None):
    """Plan a batch.  ``vertex_sides`` / ``net_sides``: lists of device
    uint8 tensors (one per problem) that ``flow_batch_run(with_cut=1)``
    fills, or None."""
    lib = load_library()
    n = len(handles)
    arr = _handle_array(handles)

    def ptrs(bufs):
        if bufs is None:
            return None, None
        if len(bufs) != n:
            raise ValueError("one output buffer per problem")
        out = []
        for b in bufs:
            if b is None:
                out.append(0)
                continue
            p, kind, _ = _ptr(b, np.uint8)
            if kind != 1:
                raise TypeError("batch cut outputs must be device tensors")
            out.append(p)
        a = (ctypes.c_void_p * max(n, 1))(*out)
        return a, a
    vs, _ = ptrs(vertex_sides)
    ns, _ = ptrs(net_sides)
    h = ctypes.c_void_p()
    _check(lib.flow_batch_create(arr, n, vs, ns, ctypes.byref(config) if config else None,
                                 _stream_ptr(stream), ctypes.byref(h)))
    return h


def flow_batch_run(batch, count: int, skip=None, with_cut: bool = False,
                   stream=None) -> np.ndarray:
    flows = np.zeros(max(count, 1), dtype=np.int64)
    sk = None
    if skip is not None:
        skip_arr = np.ascontiguousarray(skip, dtype=np.uint8)
        if skip_arr.shape[0] != count:
            raise ValueError("skip needs one entry per problem")
        sk = skip_arr.ctypes.data
    _check(load_library().flow_batch_run(batch, sk, 1 if with_cut else 0, _stream_ptr(stream),
                                         flows.ctypes.data))
    return flows[:count]


def flow_batch_tune(batch, cache_path: str | None = None, stream=None) -> dict:
    c = BatchConfig()
    _check(load_library().flow_batch_tune(batch, _stream_ptr(stream),
                                          cache_path.encode() if cache_path else None,
                                          ctypes.byref(c)))
    return c.as_dict()


def flow_batch_get_config(batch) -> dict:
    c = BatchConfig()
    _check(load_library().flow_batch_get_config(batch, ctypes.byref(c)))
    return c.as_dict()


def flow_batch_destroy(batch):
    if batch:
        load_library().flow_batch_destroy(batch)


def flow_problem_reset(handle):
    _check(load_library().flow_problem_reset(handle))


def flow_problem_sink_side(handle, num_vertices, vertex_side=None, stream=None):
    """Maximal sink side (vertices that reach a sink in the residual
    network).  Host numpy array unless a device tensor is given."""
    if vertex_side is None:
        vertex_side = np.zeros(max(num_vertices, 1), dtype=np.uint8)
    vp, vk, _ = _ptr(vertex_side, np.uint8)
    _check(load_library().flow_problem_sink_side(handle, _stream_ptr(stream), vk, vp))
    if vk == 0:
        return np.asarray(vertex_side)[:num_vertices]
    return vertex_side


def flow_problem_flowcutter(handle, num_vertices, vertex_weights, max_source_weight,
                            max_sink_weight, max_iterations=100000, vertex_side=None,
                            stream=None, want_trace=True, bulk_percent=0,
                            most_balanced=False):
    """FlowCutter on the handle's current terminals.  Returns (result dict,
    source side X, trace list of (side, node, flow, c(S_r), c(T_r))); the
    dict's "counts" lists the vertices pierced per iteration."""
    lib = load_library()
    vw = np.ascontiguousarray(vertex_weights, dtype=np.int32)
    if vw.shape[0] != num_vertices:
        raise ValueError("one weight per vertex")
    if vertex_side is None:
        vertex_side = np.zeros(max(num_vertices, 1), dtype=np.uint8)
    vp, vk, _ = _ptr(vertex_side, np.uint8)
    res = CutterResult()
    steps = (CutterStep * max(int(max_iterations), 1))() if want_trace else None
    _check(lib.flow_problem_flowcutter(handle, vw.ctypes.data, int(max_source_weight),
                                       int(max_sink_weight), int(max_iterations),
                                       int(bulk_percent), int(bool(most_balanced)),
                                       _stream_ptr(stream), vk, vp,
                                       ctypes.byref(res),
                                       ctypes.cast(steps, ctypes.c_void_p) if steps else None))
    return _cutter_out(res, steps, vertex_side, vk, num_vertices)


def _cutter_out(res, steps, vertex_side, vk, num_vertices):
    out = dict(flow=int(res.flow), source_weight=int(res.source_weight),
               sink_weight=int(res.sink_weight), iterations=int(res.iterations),
               status=CUTTER_STATUS.get(res.status, str(res.status)), side=int(res.side),
               augmenting=int(res.augmenting), first_balanced=int(res.first_balanced),
               slice_iterations=int(res.slice_iterations), resumable=bool(res.resumable))
    trace = []
    n = int(res.slice_iterations)
    if steps is not None:
        trace = [(int(t.side), int(t.node), int(t.flow), int(t.source_weight),
                  int(t.sink_weight)) for t in steps[:n]]
        out["counts"] = [int(t.count) for t in steps[:n]]
    x = np.asarray(vertex_side)[:num_vertices] if vk == 0 else vertex_side
    return out, x, trace


def flow_problem_flowcutter_continue(handle, num_vertices, max_iterations=100000,
                                     vertex_side=None, stream=None, want_trace=True):
    """Resume the handle's FlowCutter run after its last call stopped at its
    iteration limit; same return values as flow_problem_flowcutter, the
    trace holding this call's iterations."""
    lib = load_library()
    if vertex_side is None:
        vertex_side = np.zeros(max(num_vertices, 1), dtype=np.uint8)
    vp, vk, _ = _ptr(vertex_side, np.uint8)
    res = CutterResult()
    steps = (CutterStep * max(int(max_iterations), 1))() if want_trace else None
    _check(lib.flow_problem_flowcutter_continue(
        handle, int(max_iterations), _stream_ptr(stream), vk, vp, ctypes.byref(res),
        ctypes.cast(steps, ctypes.c_void_p) if steps else None))
    return _cutter_out(res, steps, vertex_side, vk, num_vertices)


def flow_problem_terminals(handle, num_vertices, roles=None, stream=None):
    """Current terminal roles per vertex (0 free, 1 source, 2 sink)."""
    if roles is None:
        roles = np.zeros(max(num_vertices, 1), dtype=np.uint8)
    vp, vk, _ = _ptr(roles, np.uint8)
    _check(load_library().flow_problem_terminals(handle, _stream_ptr(stream), vk, vp))
    if vk == 0:
        return np.asarray(roles)[:num_vertices]
    return roles


def flow_problem_pierce(handle, side: int, vertices, stream=None):
    v = np.ascontiguousarray(vertices, dtype=np.int32)
    _check(load_library().flow_problem_pierce(handle, int(side), v.ctypes.data, len(v),
                                              _stream_ptr(stream)))


def flow_problem_stats(handle) -> dict:
    s = Stats()
    _check(load_library().flow_problem_stats(handle, ctypes.byref(s)))
    return {k: int(getattr(s, k)) for k, _ in Stats._fields_ if k != "reserved"}


def flow_problem_kernel_times(handle) -> list:
    lib = load_library()
    n = 32
    names = (ctypes.c_char_p * n)()
    launches = np.zeros(n, dtype=np.int64)
    ms = np.zeros(n, dtype=np.float64)
    by = np.zeros(n, dtype=np.float64)
    k = lib.flow_problem_kernel_times(handle, n, names, launches.ctypes.data, ms.ctypes.data,
                                      by.ctypes.data)
    if k < 0:
        _check(k)
    return [dict(kernel=names[i].decode(), launches=int(launches[i]), ms=float(ms[i]),
                 bytes=float(by[i])) for i in range(k)]


def flow_problem_export_state(handle, num_vertices, num_nets, num_pins, stream=None):
    """Host copies of the flow state: dict with f_in, f_out (per pin slot),
    f_b (per net), labels and excess (vertices, then e_in / e_out of each
    net interleaved)."""
    P, E, M = num_pins, num_nets, num_vertices + 2 * num_nets
    out = dict(f_in=np.zeros(max(P, 1), np.int32), f_out=np.zeros(max(P, 1), np.int32),
               f_b=np.zeros(max(E, 1), np.int32), labels=np.zeros(max(M, 1), np.int32),
               excess=np.zeros(max(M, 1), np.int32))
    _check(load_library().flow_problem_export_state(
        handle, _stream_ptr(stream), out["f_in"].ctypes.data, out["f_out"].ctypes.data,
        out["f_b"].ctypes.data, out["labels"].ctypes.data, out["excess"].ctypes.data))
    out["f_in"], out["f_out"] = out["f_in"][:P], out["f_out"][:P]
    out["f_b"] = out["f_b"][:E]
    out["labels"], out["excess"] = out["labels"][:M], out["excess"][:M]
    return out


def maxflow_mincut_noalloc(num_vertices, net_offsets, pins, net_weights, sources, sinks,
                           vertex_side=None, net_side=None, stream=None):
    """Flow value and minimal source side in one call that allocates nothing
    (device state in the library's fixed scratch array).  Inputs and outputs
    share one memory kind: host numpy arrays, or CUDA tensors throughout.
    Returns (flow, vertex_side, net_side)."""
    lib = load_library()
    ptrs = [_ptr(a, np.int32) for a in (net_offsets, pins, net_weights, sources, sinks)]
    kinds = {k for _, k, _ in ptrs}
    num_nets = len(ptrs[0][2]) - 1
    if vertex_side is None:
        vertex_side = np.zeros(max(num_vertices, 1), dtype=np.uint8)
    if net_side is None:
        net_side = np.zeros(max(num_nets, 1), dtype=np.uint8)
    vp_, vk, _ = _ptr(vertex_side, np.uint8)
    np_, nk, _ = _ptr(net_side, np.uint8)
    kinds |= {vk, nk}
    if len(kinds) != 1:
        raise ValueError("inputs and outputs must all be host arrays or all device tensors")
    F = ctypes.c_int64(0)
    _check(lib.maxflow_mincut_noalloc(int(num_vertices), num_nets, ptrs[0][0], ptrs[1][0],
                                      ptrs[2][0], ptrs[3][0], len(ptrs[3][2]), ptrs[4][0],
                                      len(ptrs[4][2]), kinds.pop(), _stream_ptr(stream),
                                      ctypes.byref(F), vp_, np_))
    if vk == 0:
        vertex_side = np.asarray(vertex_side)[:num_vertices]
        net_side = np.asarray(net_side)[:num_nets]
    return int(F.value), vertex_side, net_side


def flow_problem_destroy(handle):
    if handle:
        load_library().flow_problem_destroy(handle)


REGION_INFO = ("n", "num_vertices", "num_nets", "num_pins", "cut_before", "boundary",
               "weight_i", "weight_j", "bin_2", "bin_4", "bin_8", "bin_16", "bin_64",
               "bin_256", "bin_more", "merged")


def flow_regions_build(num_vertices, net_offsets, pins, net_weights, vertex_weights, blocks,
                       k, pairs, caps, merge_identical=True, stream=None):
    """Build the flow problems of block pairs on the device; hypergraph,
    vertex weights and blocks all host (numpy) or all device (torch);
    ``pairs`` (count x 2 block ids) and ``caps`` (count x 2 weight caps) are
    host arrays.  Returns the handle."""
    lib = load_library()
    arrs = [_ptr(a, np.int32) for a in (net_offsets, pins, net_weights, vertex_weights, blocks)]
    kinds = {m for _, m, _ in arrs}
    if len(kinds) != 1:
        raise TypeError("hypergraph, vertex weights and blocks must share one memory kind")
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1)
    cp = np.ascontiguousarray(caps, dtype=np.int64).reshape(-1)
    if pr.shape[0] != cp.shape[0] or pr.shape[0] % 2:
        raise ValueError("pairs and caps need two entries per pair")
    num_nets = len(net_offsets) - 1
    out = ctypes.c_void_p()
    _check(lib.flow_regions_build(int(num_vertices), int(num_nets), *[a[0] for a in arrs],
                                  int(k), pr.shape[0] // 2, pr.ctypes.data, cp.ctypes.data,
                                  1 if merge_identical else 0, kinds.pop(), _stream_ptr(stream),
                                  ctypes.byref(out)))
    return out.value


def flow_regions_info(handle, pair) -> dict:
    lib = load_library()
    info = np.zeros(16, dtype=np.int64)
    _check(lib.flow_regions_info(handle, int(pair), info.ctypes.data))
    return {k: int(v) for k, v in zip(REGION_INFO, info)}


def flow_regions_export(handle, pair, stream=None) -> dict:
    """Pair ``pair``'s problem copied to the host."""
    lib = load_library()
    inf = flow_regions_info(handle, pair)
    n, ne, npins = inf["n"], inf["num_nets"], inf["num_pins"]
    bufs = dict(net_offsets=np.empty(ne + 1, np.int32), pins=np.empty(max(npins, 1), np.int32),
                net_weights=np.empty(max(ne, 1), np.int32), vertex_weights=np.empty(n + 2, np.int32),
                vertex_ids=np.empty(max(n, 1), np.int32), net_ids=np.empty(max(ne, 1), np.int32))
    _check(lib.flow_regions_export(handle, int(pair), 0, _stream_ptr(stream),
                                   *[b.ctypes.data for b in bufs.values()]))
    bufs["pins"] = bufs["pins"][:npins]
    bufs["net_weights"] = bufs["net_weights"][:ne]
    bufs["vertex_ids"] = bufs["vertex_ids"][:n]
    bufs["net_ids"] = bufs["net_ids"][:ne]
    bufs["info"] = inf
    return bufs


def flow_regions_problem(handle, pair, options: Options | None = None, stream=None):
    lib = load_library()
    out = ctypes.c_void_p()
    _check(lib.flow_regions_problem(handle, int(pair),
                                    ctypes.byref(options) if options is not None else None,
                                    _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def flow_regions_destroy(handle):
    if handle:
        load_library().flow_regions_destroy(handle)


class FlowRegions:
    """Owner of the device-built flow problems of block pairs."""

    def __init__(self, num_vertices, net_offsets, pins, net_weights, vertex_weights, blocks, k,
                 pairs, caps, merge_identical=True, stream=None):
        self.stream = stream
        self.pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        self.count = len(self.pairs)
        self.handle = flow_regions_build(num_vertices, net_offsets, pins, net_weights,
                                         vertex_weights, blocks, k, pairs, caps, merge_identical,
                                         stream)

    def info(self, pair) -> dict:
        return flow_regions_info(self.handle, pair)

    def export(self, pair) -> dict:
        return flow_regions_export(self.handle, pair, self.stream)

    def features(self, cuts, block_weights) -> np.ndarray:
        """The learned scorer's 12 integer features of every pair (int64,
        count x 12) from the statistics the device construction computed:
        the pair's cut weight (``cuts``), region pins, boundary vertices, the
        7 net-size bins, then c(V_i) and c(V_j) (``block_weights``)."""
        cuts = np.asarray(cuts, dtype=np.int64).reshape(-1)
        bw = np.asarray(block_weights, dtype=np.int64)
        if len(cuts) != self.count:
            raise ValueError("one cut weight per pair")
        keys = ("num_pins", "boundary", "bin_2", "bin_4", "bin_8", "bin_16", "bin_64",
                "bin_256", "bin_more")
        out = np.empty((self.count, 12), dtype=np.int64)
        for q in range(self.count):
            inf = self.info(q)
            i, j = self.pairs[q]
            out[q] = [cuts[q], *[inf[k] for k in keys], bw[i], bw[j]]
        return out

    def solve(self, skip=None):
        """Minimum cuts of the pairs not skipped, as union networks built from
        the regions (flow_regions_solve); flows of skipped pairs are -1."""
        lib = load_library()
        flows = np.zeros(max(self.count, 1), np.int64)
        sk = None
        if skip is not None:
            sk = np.ascontiguousarray(skip, dtype=np.uint8)
            if sk.shape[0] != self.count:
                raise ValueError("one skip flag per pair")
        _check(lib.flow_regions_solve(self.handle, sk.ctypes.data if sk is not None else None,
                                      _stream_ptr(self.stream), flows.ctypes.data))
        return flows[:self.count]

    def source_side(self, pair):
        """Pair ``pair``'s minimal source side of the last solve (host)."""
        lib = load_library()
        n = self.info(pair)["n"]
        out = np.zeros(max(n, 1), np.uint8)
        _check(lib.flow_regions_source_side(self.handle, int(pair), 0, _stream_ptr(self.stream),
                                            out.ctypes.data))
        return out[:n]

    def problem(self, pair, options: Options | None = None, **opts) -> "FlowProblem":
        if options is None and opts:
            options = Options(**opts)
        inf = self.info(pair)
        return FlowProblem._adopt(flow_regions_problem(self.handle, pair, options, self.stream),
                                  inf["num_vertices"], inf["num_nets"], self.stream)

    def close(self):
        if self.handle:
            flow_regions_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MOVE_STATUS = {0: "not tried", 1: "applied", 2: "unbalanced", 3: "reverted"}


class RefineConfig(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int32), ("min_cut", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("eps_percent", ctypes.c_int32),
                ("min_improvement_ppm", ctypes.c_int32), ("max_pairs", ctypes.c_int32),
                ("merge_identical", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RefineResult(ctypes.Structure):
    _fields_ = [("objective_before", ctypes.c_int64), ("objective_after", ctypes.c_int64),
                ("moves", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("pairs_tried", ctypes.c_int32), ("pairs_applied", ctypes.c_int32),
                ("pairs_reverted", ctypes.c_int32), ("pairs_unbalanced", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class FlowPartition:
    """Owner of a k-way partition on the device to which block-pair results
    are applied (flow_partition_*)."""

    def __init__(self, num_vertices, net_offsets, pins, net_weights, vertex_weights, blocks, k,
                 stream=None):
        lib = load_library()
        arrs = [_ptr(a, np.int32)
                for a in (net_offsets, pins, net_weights, vertex_weights, blocks)]
        kinds = {m for _, m, _ in arrs}
        if len(kinds) != 1:
            raise TypeError("hypergraph, vertex weights and blocks must share one memory kind")
        self.stream = stream
        self.num_vertices = int(num_vertices)
        self.k = int(k)
        out = ctypes.c_void_p()
        _check(lib.flow_partition_create(int(num_vertices), len(net_offsets) - 1,
                                         *[a[0] for a in arrs], int(k), kinds.pop(),
                                         _stream_ptr(stream), ctypes.byref(out)))
        self.handle = out.value

    def apply(self, regions: "FlowRegions", vertex_sides, expected_gains, lmax):
        """Apply pair q's source side ``vertex_sides[q]`` (device uint8
        tensors; None = the sides of the regions' last solve) in pair order;
        returns (status, gains, moved) arrays."""
        lib = load_library()
        n = regions.count
        ptrs = None
        if vertex_sides is not None:
            ptrs = (ctypes.c_void_p * max(n, 1))()
            for q in range(n):
                ptrs[q] = _ptr(vertex_sides[q], np.uint8)[0]
        g = np.ascontiguousarray(expected_gains, dtype=np.int64)
        if g.shape[0] != n:
            raise ValueError("one expected gain per pair")
        st = np.zeros(max(n, 1), np.int32)
        gains = np.zeros(max(n, 1), np.int64)
        moved = np.zeros(max(n, 1), np.int32)
        _check(lib.flow_partition_apply(self.handle, regions.handle, ptrs, g.ctypes.data,
                                        int(lmax), _stream_ptr(self.stream), st.ctypes.data,
                                        gains.ctypes.data, moved.ctypes.data))
        return st[:n], gains[:n], moved[:n]

    def refine(self, max_rounds=16, min_cut=10, alpha=16, eps_percent=3,
               min_improvement_ppm=1000, max_pairs=0, merge_identical=True):
        """Refinement rounds on the device (flow_partition_refine); returns
        (result dict, objective after each round, first entry before)."""
        lib = load_library()
        max_rounds = int(max_rounds) or 16
        cfg = RefineConfig(int(max_rounds), int(min_cut), int(alpha), int(eps_percent),
                           int(min_improvement_ppm), int(max_pairs), int(bool(merge_identical)),
                           0)
        res = RefineResult()
        traj = np.full(int(max_rounds) + 1, -1, np.int64)
        _check(lib.flow_partition_refine(self.handle, ctypes.byref(cfg), _stream_ptr(self.stream),
                                         ctypes.byref(res), traj.ctypes.data))
        out = {name: int(getattr(res, name)) for name, _ in RefineResult._fields_
               if name != "reserved"}
        return out, traj[:out["rounds"] + 1]

    def get(self):
        """(blocks, block weights, objective sum w(e) (lambda(e) - 1))."""
        lib = load_library()
        blocks = np.empty(self.num_vertices, np.int32)
        bw = np.empty(self.k, np.int64)
        obj = ctypes.c_int64()
        _check(lib.flow_partition_get(self.handle, 0, _stream_ptr(self.stream),
                                      blocks.ctypes.data, bw.ctypes.data, ctypes.byref(obj)))
        return blocks, bw, int(obj.value)

    def close(self):
        if self.handle:
            load_library().flow_partition_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FlowProblem:
    """Owner of one problem handle."""

    def __init__(self, num_vertices, net_offsets, pins, net_weights, sources, sinks,
                 options: Options | None = None, stream=None, **opts):
        if options is None and opts:
            options = Options(**opts)
        self.num_vertices = int(num_vertices)
        self.num_nets = len(net_offsets) - 1
        self.stream = stream
        self.handle = flow_problem_create(num_vertices, net_offsets, pins, net_weights,
                                          sources, sinks, options, stream)

    @classmethod
    def _adopt(cls, handle, num_vertices, num_nets, stream=None):
        """Wrap a handle created elsewhere (the caller gives up its ownership)."""
        self = cls.__new__(cls)
        self.num_vertices = int(num_vertices)
        self.num_nets = int(num_nets)
        self.stream = stream
        self.handle = handle
        return self

    @classmethod
    def from_hypergraph(cls, hg, device: bool = False, **opts):
        arrays = (hg.net_offsets, hg.pins, hg.net_weights, hg.sources, hg.sinks)
        if device:
            import torch
            arrays = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays)
            torch.cuda.synchronize()
        return cls(hg.num_vertices, *arrays, **opts)

    def solve(self) -> int:
        return maxflow_solve(self.handle, self.stream)

    def source_side(self, vertex_side=None, net_side=None):
        return mincut_source_side(self.handle, self.num_vertices, self.num_nets, vertex_side,
                                  net_side, self.stream)

    def reset(self):
        flow_problem_reset(self.handle)

    def pierce(self, side: int, vertices):
        flow_problem_pierce(self.handle, side, vertices, self.stream)

    def sink_side(self, vertex_side=None):
        return flow_problem_sink_side(self.handle, self.num_vertices, vertex_side, self.stream)

    def flowcutter(self, vertex_weights, max_source_weight, max_sink_weight,
                   max_iterations=100000, vertex_side=None, want_trace=True, bulk_percent=0,
                   most_balanced=False):
        return flow_problem_flowcutter(self.handle, self.num_vertices, vertex_weights,
                                       max_source_weight, max_sink_weight, max_iterations,
                                       vertex_side, self.stream, want_trace, bulk_percent,
                                       most_balanced)

    def flowcutter_continue(self, max_iterations=100000, vertex_side=None, want_trace=True):
        return flow_problem_flowcutter_continue(self.handle, self.num_vertices, max_iterations,
                                                vertex_side, self.stream, want_trace)

    def terminals(self, roles=None):
        return flow_problem_terminals(self.handle, self.num_vertices, roles, self.stream)

    def stats(self) -> dict:
        return flow_problem_stats(self.handle)

    def export_state(self, num_pins: int) -> dict:
        return flow_problem_export_state(self.handle, self.num_vertices, self.num_nets,
                                         num_pins, self.stream)

    def kernel_times(self) -> list:
        return flow_problem_kernel_times(self.handle)

    def close(self):
        if self.handle:
            flow_problem_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FlowBatch:
    """Owner of a batch plan over :class:`FlowProblem` objects (which must
    outlive it).  With ``with_cut=True`` device side buffers are allocated
    for every problem (``vertex_sides[i]``, ``net_sides[i]``)."""

    def __init__(self, problems, with_cut: bool = False, config: BatchConfig | None = None,
                 stream=None, **cfg):
        if config is None and cfg:
            config = BatchConfig(**cfg)
        self.problems = list(problems)
        self.stream = stream
        self.vertex_sides = self.net_sides = None
        if with_cut:
            import torch
            self.vertex_sides = [torch.zeros(max(p.num_vertices, 1), dtype=torch.uint8,
                                             device="cuda") for p in self.problems]
            self.net_sides = [torch.zeros(max(p.num_nets, 1), dtype=torch.uint8, device="cuda")
                              for p in self.problems]
            torch.cuda.synchronize()
        self.handle = flow_batch_create([p.handle for p in self.problems], self.vertex_sides,
                                        self.net_sides, config, stream)

    def run(self, skip=None, with_cut: bool = False) -> np.ndarray:
        return flow_batch_run(self.handle, len(self.problems), skip, with_cut, self.stream)

    def tune(self, cache_path: str | None = None) -> dict:
        return flow_batch_tune(self.handle, cache_path, self.stream)

    def config(self) -> dict:
        return flow_batch_get_config(self.handle)

    def sides(self, i: int):
        """Host copies of problem i's (vertex_side, net_side) after a run
        with the cut."""
        p = self.problems[i]
        return (self.vertex_sides[i][:p.num_vertices].cpu().numpy(),
                self.net_sides[i][:p.num_nets].cpu().numpy())

    def close(self):
        if self.handle:
            flow_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scorer:
    """Owner of a learned pruning scorer (MLP 12 -> 64 -> 64 -> 1 on the
    device).  Features: int64 [n x 12] host arrays; labels float 0/1."""

    def __init__(self, init_params, stream=None):
        self.stream = stream
        p = np.ascontiguousarray(init_params, dtype=np.float32)
        if p.shape != (SCORER_PARAMS,):
            raise ValueError(f"need {SCORER_PARAMS} parameters")
        h = ctypes.c_void_p()
        _check(load_library().scorer_create(p.ctypes.data, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def _feats(features):
        f = np.ascontiguousarray(features, dtype=np.int64)
        if f.ndim != 2 or f.shape[1] != 12:
            raise ValueError("features must be n x 12")
        return f

    def fit_normalization(self, features):
        f = self._feats(features)
        _check(load_library().scorer_fit_normalization(self.handle, f.ctypes.data, f.shape[0], 0,
                                                       _stream_ptr(self.stream)))

    def gradient(self, features, labels):
        f = self._feats(features)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        g = np.zeros(SCORER_PARAMS, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check(load_library().scorer_gradient(self.handle, f.ctypes.data, y.ctypes.data,
                                              f.shape[0], 0, _stream_ptr(self.stream),
                                              g.ctypes.data, loss.ctypes.data))
        return float(loss[0]), g

    def train(self, features, labels, steps, lr=1e-3):
        f = self._feats(features)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(load_library().scorer_train(self.handle, f.ctypes.data, y.ctypes.data, f.shape[0],
                                           0, int(steps), float(lr), _stream_ptr(self.stream),
                                           losses.ctypes.data))
        return losses[:steps]

    def predict(self, features):
        f = self._feats(features)
        p = np.zeros(f.shape[0], dtype=np.float32)
        _check(load_library().scorer_predict(self.handle, f.ctypes.data, f.shape[0], 0,
                                             _stream_ptr(self.stream), p.ctypes.data))
        return p

    def params(self):
        p = np.zeros(SCORER_PARAMS, dtype=np.float32)
        ms = np.zeros(24, dtype=np.float64)
        _check(load_library().scorer_get_params(self.handle, p.ctypes.data, ms.ctypes.data))
        return p, ms

    def set_params(self, params, mean_std=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        ms = None if mean_std is None else np.ascontiguousarray(mean_std, dtype=np.float64)
        _check(load_library().scorer_set_params(self.handle, p.ctypes.data,
                                                None if ms is None else ms.ctypes.data))

    def close(self):
        if self.handle:
            load_library().scorer_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
