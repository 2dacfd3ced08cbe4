"""ctypes binding of libft (include/ft.h).

The functions ``ft_*`` mirror the C entry points one to one and only marshal
arguments: every step of the transfer runs in the HIP library.  PyTorch
supplies device memory and the current stream.  ``Target`` and ``Source`` are
small conveniences that keep the mesh tensors in the layouts the library
expects (structure-of-arrays coordinates, int32 connectivity).

The library must be built (``python -m paper_2603_00538_amd.build``); there is
no fallback: loading fails loudly if ``libft.so`` is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libft.so")

FT_OK, FT_E_ARG, FT_E_MESH, FT_E_ORDER, FT_E_DEVICE, FT_E_NOCONV, FT_E_NONFINITE, FT_E_OOM, FT_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FT_F64, FT_F32, FT_SPLIT_F16, FT_SPLIT_BF16 = 0, 1, 2, 3
FT_BATCH_GRAPH = 1
FT_SAMPLING_PLAIN, FT_SAMPLING_STRATIFIED = 0, 1
FT_ALPHA_FIXED, FT_ALPHA_ELEMENT = 0, 1
FT_VALUES_FIELD_MAJOR, FT_VALUES_ELEMENT_TILES = 0, 1
STATUS_NAMES = {0: "FT_OK", -1: "FT_E_ARG", -2: "FT_E_MESH", -3: "FT_E_ORDER", -4: "FT_E_DEVICE",
                -5: "FT_E_NOCONV", -6: "FT_E_NONFINITE", -7: "FT_E_OOM", -8: "FT_E_UNSUPPORTED"}

EXPORTED = ["ft_target_create", "ft_target_create_p2", "ft_target_destroy", "ft_target_get_info", "ft_query_count", "ft_sample_points",
            "ft_consume_queries", "ft_consume_queries_noalloc", "ft_transfer_p1",
            "ft_transfer_supermesh", "ft_project", "ft_source_create_p1", "ft_source_eval",
            "ft_source_eval_queries", "ft_source_eval_tiles", "ft_source_autotune", "ft_source_stats", "ft_batch_create", "ft_batch_run", "ft_batch_autotune", "ft_batch_variant",
            "ft_batch_destroy", "ft_batch_consume_run",
            "ft_plan_create", "ft_plan_transfer", "ft_plan_destroy",
            "ft_source_destroy", "ft_source_get_info", "ft_source_integral", "ft_samples_for_tolerance",
            "ft_allocate_samples", "ft_budget_for_tolerance", "ft_sample_points_adaptive",
            "ft_consume_queries_adaptive", "ft_transfer_p1_adaptive", "ft_last_error"]


class SampleCfg(ctypes.Structure):
    _fields_ = [("samples_per_elem", ctypes.c_int32), ("n_fields", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("alpha_mode", ctypes.c_int32), ("values_layout", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SolveCfg(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("refine_steps", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("sum_b", ctypes.c_double), ("int_x", ctypes.c_double), ("cons_defect", ctypes.c_double),
                ("rel_resid", ctypes.c_double), ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_nonfinite", ctypes.c_int64), ("n_out_of_domain", ctypes.c_int64),
                ("sum_b_stderr", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TargetInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("n_inverted", ctypes.c_int64), ("order", ctypes.c_int32)]


class Allocation(ctypes.Structure):
    _fields_ = [("total", ctypes.c_int64), ("weight_sum", ctypes.c_double), ("predicted_stderr", ctypes.c_double)]


class SourceInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_fields", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_elems", ctypes.c_int64), ("bins", ctypes.c_int32 * 3), ("n_registrations", ctypes.c_int64)]


class FtError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libft.so (once); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2603_00538_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ft_target_create": (I32, [I32, I64, P, I64, P, P, ctypes.POINTER(P)]),
        "ft_target_create_p2": (I32, [I32, I64, P, I64, P, P, ctypes.POINTER(P)]),
        "ft_target_destroy": (I32, [P]),
        "ft_target_get_info": (I32, [P, ctypes.POINTER(TargetInfo)]),
        "ft_query_count": (I64, [P, I32]),
        "ft_sample_points": (I32, [P, ctypes.POINTER(SampleCfg), P, P]),
        "ft_consume_queries": (I32, [P, ctypes.POINTER(SampleCfg), P, P]),
        "ft_consume_queries_noalloc": (I32, [P, ctypes.POINTER(SampleCfg), P, P]),
        "ft_transfer_p1": (I32, [P, P, ctypes.POINTER(SampleCfg), P]),
        "ft_transfer_supermesh": (I32, [P, P, P, P]),
        "ft_project": (I32, [P, ctypes.POINTER(SolveCfg), P, P, ctypes.POINTER(Report), P]),
        "ft_source_create_p1": (I32, [I32, I64, P, I64, P, I32, P, P, P, ctypes.POINTER(P)]),
        "ft_source_eval": (I32, [P, I64, P, I64, I32, P, I64, P, P]),
        "ft_source_eval_queries": (I32, [P, I64, I64, P, I64, I32, P, I64, P, P]),
        "ft_source_autotune": (I32, [P, I64, I64, P, I64, I32, I32, P, P, P]),
        "ft_source_eval_tiles": (I32, [P, I64, I64, I32, P, I64, I32, P, P, P]),
        "ft_source_stats": (I32, [P, ctypes.POINTER(I64), P]),
        "ft_source_destroy": (I32, [P]),
        "ft_source_get_info": (I32, [P, ctypes.POINTER(SourceInfo)]),
        "ft_source_integral": (I32, [P, ctypes.POINTER(D), P]),
        "ft_batch_create": (I32, [I32, P, P, ctypes.POINTER(SampleCfg), I32, P, ctypes.POINTER(P)]),
        "ft_batch_run": (I32, [P, ctypes.POINTER(SolveCfg), P, P, ctypes.POINTER(Report), P, P]),
        "ft_batch_destroy": (I32, [P]),
        "ft_batch_consume_run": (I32, [P, ctypes.POINTER(SolveCfg), P, P, P, ctypes.POINTER(Report), P, P]),
        "ft_batch_autotune": (I32, [P, ctypes.c_char_p, ctypes.POINTER(I32), P]),
        "ft_batch_variant": (I32, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "ft_plan_create": (I32, [P, P, ctypes.POINTER(SampleCfg), P, ctypes.POINTER(P)]),
        "ft_plan_transfer": (I32, [P, P, P]),
        "ft_plan_destroy": (I32, [P]),
        "ft_samples_for_tolerance": (I32, [ctypes.POINTER(Report), I32, D]),
        "ft_allocate_samples": (I32, [P, I32, I64, I32, I32, P, ctypes.POINTER(Allocation), P]),
        "ft_budget_for_tolerance": (I64, [D, D, D]),
        "ft_sample_points_adaptive": (I32, [P, ctypes.POINTER(SampleCfg), P, I64, P, P]),
        "ft_consume_queries_adaptive": (I32, [P, ctypes.POINTER(SampleCfg), P, I64, P, P]),
        "ft_transfer_p1_adaptive": (I32, [P, P, ctypes.POINTER(SampleCfg), P, I64, P]),
        "ft_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, fn: str, allow=()):
    if status != FT_OK and status not in allow:
        raise FtError(status, fn, load().ft_last_error().decode())
    return status


# ------------------------------------------------------------------ C entry points
def ft_target_create(dim, n_nodes, coords_ptr, n_elems, conn_ptr, stream):
    h = ctypes.c_void_p()
    _check(load().ft_target_create(dim, n_nodes, coords_ptr, n_elems, conn_ptr, stream, ctypes.byref(h)),
           "ft_target_create")
    return h


def ft_target_create_p2(dim, n_nodes, coords_ptr, n_elems, conn_ptr, stream):
    h = ctypes.c_void_p()
    _check(load().ft_target_create_p2(dim, n_nodes, coords_ptr, n_elems, conn_ptr, stream, ctypes.byref(h)),
           "ft_target_create_p2")
    return h


def ft_target_destroy(h):
    return load().ft_target_destroy(h)


def ft_target_get_info(h) -> TargetInfo:
    info = TargetInfo()
    _check(load().ft_target_get_info(h, ctypes.byref(info)), "ft_target_get_info")
    return info


def ft_query_count(h, samples_per_elem):
    return load().ft_query_count(h, samples_per_elem)


def ft_sample_points(h, cfg: SampleCfg, points_ptr, stream):
    return _check(load().ft_sample_points(h, ctypes.byref(cfg), points_ptr, stream), "ft_sample_points")


def ft_consume_queries(h, cfg: SampleCfg, values_ptr, stream):
    return _check(load().ft_consume_queries(h, ctypes.byref(cfg), values_ptr, stream), "ft_consume_queries")


def ft_consume_queries_noalloc(h, cfg: SampleCfg, values_ptr, stream):
    return _check(load().ft_consume_queries_noalloc(h, ctypes.byref(cfg), values_ptr, stream),
                  "ft_consume_queries_noalloc")


def ft_transfer_p1(h, src, cfg: SampleCfg, stream):
    return _check(load().ft_transfer_p1(h, src, ctypes.byref(cfg), stream), "ft_transfer_p1")


def ft_transfer_supermesh(h, src, area_ptr, stream):
    return _check(load().ft_transfer_supermesh(h, src, area_ptr, stream), "ft_transfer_supermesh")


def ft_project(h, cfg: SolveCfg, x_ptr, b_ptr, n_fields, stream, allow=(FT_E_NOCONV, FT_E_NONFINITE)):
    reps = (Report * n_fields)()
    st = _check(load().ft_project(h, ctypes.byref(cfg), x_ptr, b_ptr, reps, stream), "ft_project", allow)
    return st, [r.as_dict() for r in reps]


def ft_batch_create(targets, sources, cfgs, flags, stream):
    K = len(targets)
    th = (ctypes.c_void_p * K)(*targets)
    sh = (ctypes.c_void_p * K)(*sources)
    cf = (SampleCfg * K)(*cfgs)
    out = ctypes.c_void_p()
    _check(load().ft_batch_create(K, th, sh, cf, flags, stream, ctypes.byref(out)), "ft_batch_create")
    return out


def ft_batch_run(h, cfg: SolveCfg, x_ptrs, b_ptrs, stream, n_systems=None, allow=(FT_E_NOCONV, FT_E_NONFINITE)):
    K = len(x_ptrs)
    xs = (ctypes.c_void_p * K)(*x_ptrs)
    bs = (ctypes.c_void_p * K)(*b_ptrs) if b_ptrs is not None else None
    R = n_systems or K   # one report per field of every transfer
    reps = (Report * R)()
    sts = (ctypes.c_int32 * R)()
    st = _check(load().ft_batch_run(h, ctypes.byref(cfg), xs, bs, reps, sts, stream), "ft_batch_run", allow)
    return st, [r.as_dict() for r in reps], list(sts)


def ft_batch_consume_run(h, cfg: SolveCfg, value_ptrs, x_ptrs, b_ptrs, stream, n_systems,
                         allow=(FT_E_NOCONV, FT_E_NONFINITE)):
    K = len(x_ptrs)
    vs = (ctypes.c_void_p * K)(*value_ptrs)
    xs = (ctypes.c_void_p * K)(*x_ptrs)
    bs = (ctypes.c_void_p * K)(*b_ptrs) if b_ptrs is not None else None
    reps = (Report * n_systems)()
    sts = (ctypes.c_int32 * n_systems)()
    st = _check(load().ft_batch_consume_run(h, ctypes.byref(cfg), vs, xs, bs, reps, sts, stream),
                "ft_batch_consume_run", allow)
    return st, [r.as_dict() for r in reps], list(sts)


def ft_source_autotune(h, n_nodes, n_points, points_ptr, ld, precision, candidates, stream):
    cand = (ctypes.c_int32 * len(candidates))(*candidates)
    out = (ctypes.c_int32 * 3)()
    _check(load().ft_source_autotune(h, n_nodes, n_points, points_ptr, ld, precision, len(candidates), cand, out,
                                     stream), "ft_source_autotune")
    return list(out)


def ft_plan_create(t, s, cfg: SampleCfg, stream):
    out = ctypes.c_void_p()
    _check(load().ft_plan_create(t, s, ctypes.byref(cfg), stream, ctypes.byref(out)), "ft_plan_create")
    return out


def ft_plan_transfer(h, values_ptr, stream):
    return _check(load().ft_plan_transfer(h, values_ptr, stream), "ft_plan_transfer")


def ft_plan_destroy(h):
    return _check(load().ft_plan_destroy(h), "ft_plan_destroy")


def ft_batch_autotune(h, cache_path, stream):
    n = ctypes.c_int32(0)
    _check(load().ft_batch_autotune(h, cache_path.encode() if cache_path else None, ctypes.byref(n), stream),
           "ft_batch_autotune")
    return n.value


def ft_batch_variant(h, k):
    g, p = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().ft_batch_variant(h, k, ctypes.byref(g), ctypes.byref(p)), "ft_batch_variant")
    return g.value, p.value


def ft_batch_destroy(h):
    return _check(load().ft_batch_destroy(h), "ft_batch_destroy")


def ft_samples_for_tolerance(report, samples_per_elem, rel_tol):
    """Samples per element for a target standard error of sum b (-1: the
    report carries no estimate).  report: a Report or its dict form."""
    if isinstance(report, dict):
        r = Report()
        for k, _ in Report._fields_:
            setattr(r, k, report[k])
        report = r
    return int(load().ft_samples_for_tolerance(ctypes.byref(report), samples_per_elem, rel_tol))


def ft_source_create_p1(dim, n_nodes, coords_ptr, n_elems, conn_ptr, n_fields, values_ptr, bins, stream):
    h = ctypes.c_void_p()
    b = None
    if bins is not None:
        b = (ctypes.c_int32 * 3)(*[int(v) for v in list(bins) + [0] * (3 - len(bins))])
    _check(load().ft_source_create_p1(dim, n_nodes, coords_ptr, n_elems, conn_ptr, n_fields, values_ptr, b, stream,
                                      ctypes.byref(h)), "ft_source_create_p1")
    return h


def ft_source_eval(h, n_points, points_ptr, ld, precision, values_ptr, ld_out, ids_ptr, stream):
    return _check(load().ft_source_eval(h, n_points, points_ptr, ld, precision, values_ptr, ld_out, ids_ptr, stream),
                  "ft_source_eval")


def ft_source_eval_queries(h, n_nodes, n_points, points_ptr, ld, precision, values_ptr, ld_out, ids_ptr, stream):
    return _check(load().ft_source_eval_queries(h, n_nodes, n_points, points_ptr, ld, precision, values_ptr, ld_out,
                                                ids_ptr, stream), "ft_source_eval_queries")


def ft_source_eval_tiles(h, n_nodes, n_elems, N, points_ptr, ld, precision, values_ptr, ids_ptr, stream):
    return _check(load().ft_source_eval_tiles(h, n_nodes, n_elems, N, points_ptr, ld, precision, values_ptr,
                                              ids_ptr, stream), "ft_source_eval_tiles")


def ft_source_stats(h, stream):
    n = ctypes.c_int64()
    _check(load().ft_source_stats(h, ctypes.byref(n), stream), "ft_source_stats")
    return n.value


def ft_source_destroy(h):
    return load().ft_source_destroy(h)


def ft_source_integral(h, n_fields, stream):
    out = (ctypes.c_double * n_fields)()
    _check(load().ft_source_integral(h, out, stream), "ft_source_integral")
    return list(out)


def ft_source_get_info(h) -> SourceInfo:
    info = SourceInfo()
    _check(load().ft_source_get_info(h, ctypes.byref(info)), "ft_source_get_info")
    return info


# ------------------------------------------------------------------ torch conveniences
def ft_allocate_samples(h, field, budget, n_min, n_max, offsets_ptr, stream) -> Allocation:
    a = Allocation()
    _check(load().ft_allocate_samples(h, field, budget, n_min, n_max, offsets_ptr, ctypes.byref(a), stream),
           "ft_allocate_samples")
    return a


def ft_budget_for_tolerance(weight_sum, sum_b, rel_tol):
    """Total samples for which the Neyman prediction reaches rel_tol |sum_b| (-1: invalid arguments)."""
    return int(load().ft_budget_for_tolerance(weight_sum, sum_b, rel_tol))


def ft_sample_points_adaptive(h, cfg: SampleCfg, offsets_ptr, total, points_ptr, stream):
    return _check(load().ft_sample_points_adaptive(h, ctypes.byref(cfg), offsets_ptr, total, points_ptr, stream),
                  "ft_sample_points_adaptive")


def ft_consume_queries_adaptive(h, cfg: SampleCfg, offsets_ptr, total, values_ptr, stream):
    return _check(load().ft_consume_queries_adaptive(h, ctypes.byref(cfg), offsets_ptr, total, values_ptr, stream),
                  "ft_consume_queries_adaptive")


def ft_transfer_p1_adaptive(h, src, cfg: SampleCfg, offsets_ptr, total, stream):
    return _check(load().ft_transfer_p1_adaptive(h, src, ctypes.byref(cfg), offsets_ptr, total, stream),
                  "ft_transfer_p1_adaptive")


def _torch():
    import torch
    return torch


def current_stream():
    return _torch().cuda.current_stream().cuda_stream


def _device_ptr(t, name, dtype=None, shape0=None):
    """Data pointer of a contiguous CUDA tensor (raises instead of passing a wrong layout)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (got strides {tuple(t.stride())})")
    if dtype is not None and t.dtype not in dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtype}")
    if shape0 is not None and t.shape[0] != shape0:
        raise ValueError(f"{name} has leading size {t.shape[0]}, expected {shape0}")
    return t.data_ptr()


def _soa(coords, device):
    """(n, d) array/tensor -> contiguous (d, n) float64 device tensor."""
    torch = _torch()
    t = torch.as_tensor(coords, dtype=torch.float64)
    return t.t().contiguous().to(device)


@dataclass
class Transfer:
    """Result of one transfer (device tensors and host reports)."""
    x: object
    b: object
    reports: list
    status: int


class Target:
    """A target mesh on the device (ft_target_create / ft_target_create_p2 ...
    ft_target_destroy).  order 2: conn lists each element's vertices, then its
    edge nodes (ft_target_create_p2)."""

    def __init__(self, coords, conn, device="cuda", order=1):
        torch = _torch()
        self.dim = int(coords.shape[1])
        self.order = int(order)
        self.coords = _soa(coords, device)                                  # (d, n)
        self.conn = torch.as_tensor(conn, dtype=torch.int32).contiguous().to(device)
        self.n_nodes = int(coords.shape[0])
        self.n_elems = int(conn.shape[0])
        create = ft_target_create_p2 if self.order == 2 else ft_target_create
        self.handle = create(self.dim, self.n_nodes, self.coords.data_ptr(), self.n_elems, self.conn.data_ptr(),
                             current_stream())

    def close(self):
        if getattr(self, "handle", None):
            ft_target_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return ft_target_get_info(self.handle)

    def query_count(self, N):
        return ft_query_count(self.handle, N)

    def sample_points(self, cfg: SampleCfg, out=None):
        torch = _torch()
        Q = self.query_count(cfg.samples_per_elem)
        dt = torch.float64 if cfg.precision == FT_F64 else torch.float32
        if out is None:
            out = torch.empty((self.dim, Q), dtype=dt, device=self.coords.device)
        if out.numel() < self.dim * Q:
            raise ValueError(f"points buffer holds {out.numel()} values, needs {self.dim * Q}")
        ft_sample_points(self.handle, cfg, _device_ptr(out, "points", (dt,)), current_stream())
        return out

    def consume(self, cfg: SampleCfg, values, noalloc=False):
        """ft_consume_queries, or ft_consume_queries_noalloc with noalloc=True."""
        torch = _torch()
        dt = torch.float64 if cfg.precision == FT_F64 else torch.float32
        Q = self.query_count(cfg.samples_per_elem)
        if values.numel() < cfg.n_fields * Q:
            raise ValueError(f"values hold {values.numel()} entries, need {cfg.n_fields * Q}")
        fn = ft_consume_queries_noalloc if noalloc else ft_consume_queries
        fn(self.handle, cfg, _device_ptr(values, "values", (dt,)), current_stream())

    def allocate_samples(self, budget, field=0, n_min=2, n_max=1 << 20, offsets=None):
        """ft_allocate_samples after a pilot transfer: (offsets int64 (E+1,) device
        tensor, Allocation) for `budget` samples in all."""
        torch = _torch()
        if offsets is None:
            offsets = torch.empty(self.n_elems + 1, dtype=torch.int64, device=self.coords.device)
        if offsets.numel() < self.n_elems + 1:
            raise ValueError(f"offsets hold {offsets.numel()} entries, need {self.n_elems + 1}")
        a = ft_allocate_samples(self.handle, field, int(budget), n_min, n_max,
                                _device_ptr(offsets, "offsets", (torch.int64,)), current_stream())
        return offsets, a

    def sample_points_adaptive(self, cfg: SampleCfg, offsets, total, out=None):
        """ft_sample_points_adaptive: the list of per-element counts, (dim, n_nodes + total)."""
        torch = _torch()
        Q = self.n_nodes + int(total)
        dt = torch.float64 if cfg.precision == FT_F64 else torch.float32
        if out is None:
            out = torch.empty((self.dim, Q), dtype=dt, device=self.coords.device)
        if out.numel() < self.dim * Q:
            raise ValueError(f"points buffer holds {out.numel()} values, needs {self.dim * Q}")
        ft_sample_points_adaptive(self.handle, cfg, _device_ptr(offsets, "offsets", (torch.int64,)), int(total),
                                  _device_ptr(out, "points", (dt,)), current_stream())
        return out

    def consume_adaptive(self, cfg: SampleCfg, offsets, total, values):
        """ft_consume_queries_adaptive for values [F][n_nodes + total]."""
        torch = _torch()
        dt = torch.float64 if cfg.precision == FT_F64 else torch.float32
        Q = self.n_nodes + int(total)
        if values.numel() < cfg.n_fields * Q:
            raise ValueError(f"values hold {values.numel()} entries, need {cfg.n_fields * Q}")
        ft_consume_queries_adaptive(self.handle, cfg, _device_ptr(offsets, "offsets", (torch.int64,)), int(total),
                                    _device_ptr(values, "values", (dt,)), current_stream())

    def transfer_from_adaptive(self, source, cfg: SampleCfg, offsets, total):
        """ft_transfer_p1_adaptive: the fused route with per-element counts."""
        torch = _torch()
        ft_transfer_p1_adaptive(self.handle, source.handle, cfg, _device_ptr(offsets, "offsets", (torch.int64,)),
                                int(total), current_stream())

    def transfer_from(self, source, cfg: SampleCfg):
        """Fused steps 1 and 3-6 from a built-in Source (no query list in memory)."""
        ft_transfer_p1(self.handle, source.handle, cfg, current_stream())

    def transfer_supermesh(self, source, area=None):
        """Exact load vector by mesh intersection (ft_transfer_supermesh); returns
        the per-element intersection areas when area=True."""
        torch = _torch()
        out = None
        if area:
            out = torch.empty(self.n_elems, dtype=torch.float64, device=self.coords.device)
        ft_transfer_supermesh(self.handle, source.handle,
                              _device_ptr(out, "area", (torch.float64,)) if out is not None else None,
                              current_stream())
        return out

    def project(self, n_fields=1, rtol=1e-14, max_iter=500, want_b=True, x=None, b=None, refine_steps=0):
        torch = _torch()
        if x is None:
            x = torch.empty((n_fields, self.n_nodes), dtype=torch.float64, device=self.coords.device)
        if want_b and b is None:
            b = torch.empty((n_fields, self.n_nodes), dtype=torch.float64, device=self.coords.device)
        f64 = (torch.float64,)
        st, reps = ft_project(self.handle, SolveCfg(rtol, max_iter, refine_steps), _device_ptr(x, "x", f64, n_fields),
                              _device_ptr(b, "b", f64, n_fields) if want_b else None, n_fields, current_stream())
        return Transfer(x, b, reps, st)


class Source:
    """Mesh-backed P1 source with uniform-grid localization (ft_source_*)."""

    def __init__(self, coords, conn, nodal_values, bins=None, device="cuda"):
        torch = _torch()
        self.dim = int(coords.shape[1])
        self.coords = _soa(coords, device)
        self.conn = torch.as_tensor(conn, dtype=torch.int32).contiguous().to(device)
        v = torch.as_tensor(nodal_values, dtype=torch.float64)
        if v.ndim == 1:
            v = v[None, :]
        self.values = v.contiguous().to(device)
        self.n_fields = int(self.values.shape[0])
        self.n_nodes = int(coords.shape[0])
        self.handle = ft_source_create_p1(self.dim, int(coords.shape[0]), self.coords.data_ptr(), int(conn.shape[0]),
                                          self.conn.data_ptr(), self.n_fields, self.values.data_ptr(), bins,
                                          current_stream())

    def close(self):
        if getattr(self, "handle", None):
            ft_source_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, points, out=None, ids=None, start=0, count=None):
        """Evaluate points[:, start:start+count] of a (d, ld) device tensor into out[:, start:start+count].

        Returns out, (F, ld) in the dtype of points.  The range form lets a
        caller evaluate blocks of a query list separately (e.g. the node block
        and the sample block), with the list's leading dimension.
        """
        torch = _torch()
        if points.ndim != 2 or points.shape[0] != self.dim:
            raise ValueError(f"points must have shape ({self.dim}, n)")
        ld = int(points.shape[1])
        count = ld - start if count is None else int(count)
        if start < 0 or count < 0 or start + count > ld:
            raise ValueError("start/count out of range")
        prec = FT_F32 if points.dtype == torch.float32 else FT_F64
        if out is None:
            out = torch.empty((self.n_fields, ld), dtype=points.dtype, device=points.device)
        if out.ndim != 2 or out.shape[0] != self.n_fields or out.shape[1] < start + count or out.dtype != points.dtype:
            raise ValueError("out must have shape (n_fields, >= start + count) and the dtype of points")
        if ids is not None and (ids.dtype != torch.int32 or ids.numel() < start + count):
            raise ValueError("ids must be int32 with at least start + count entries")
        isz = points.element_size()
        ft_source_eval(self.handle, count, _device_ptr(points, "points", (torch.float32, torch.float64)) + start * isz,
                       ld, prec, _device_ptr(out, "out") + start * isz, int(out.shape[1]),
                       (_device_ptr(ids, "ids") + start * 4) if ids is not None else None, current_stream())
        return out

    def eval_query_list(self, points, n_nodes, out=None, ids=None):
        """Evaluate a transfer's whole (d, Q) query list in one launch, its node block
        and its sample block in separate wavefronts (ft_source_eval_queries)."""
        torch = _torch()
        if points.ndim != 2 or points.shape[0] != self.dim:
            raise ValueError(f"points must have shape ({self.dim}, n)")
        ld = int(points.shape[1])
        if not 0 <= n_nodes <= ld:
            raise ValueError("n_nodes out of range")
        prec = FT_F32 if points.dtype == torch.float32 else FT_F64
        if out is None:
            out = torch.empty((self.n_fields, ld), dtype=points.dtype, device=points.device)
        if out.ndim != 2 or out.shape[0] != self.n_fields or out.shape[1] < ld or out.dtype != points.dtype:
            raise ValueError("out must have shape (n_fields, >= Q) and the dtype of points")
        if ids is not None and (ids.dtype != torch.int32 or ids.numel() < ld):
            raise ValueError("ids must be int32 with at least Q entries")
        ft_source_eval_queries(self.handle, int(n_nodes), ld, _device_ptr(points, "points", (torch.float32, torch.float64)),
                               ld, prec, _device_ptr(out, "out"), int(out.shape[1]),
                               _device_ptr(ids, "ids") if ids is not None else None, current_stream())
        return out

    def eval_tiles(self, points, n_nodes, n_elems, N, out=None, ids=None):
        """Evaluate a transfer's (d, Q) query list, values as element tiles
        (FT_VALUES_ELEMENT_TILES): a flat tensor of F*Q values."""
        torch = _torch()
        if points.ndim != 2 or points.shape[0] != self.dim:
            raise ValueError(f"points must have shape ({self.dim}, n)")
        Q = n_nodes + n_elems * N
        ld = int(points.shape[1])
        if ld < Q:
            raise ValueError("points hold fewer than n_nodes + n_elems * N queries")
        prec = FT_F32 if points.dtype == torch.float32 else FT_F64
        if out is None:
            out = torch.empty(self.n_fields * Q, dtype=points.dtype, device=points.device)
        if out.numel() < self.n_fields * Q or out.dtype != points.dtype:
            raise ValueError("out must hold n_fields * Q values of the dtype of points")
        if ids is not None and (ids.dtype != torch.int32 or ids.numel() < Q):
            raise ValueError("ids must be int32 with at least Q entries")
        ft_source_eval_tiles(self.handle, int(n_nodes), int(n_elems), int(N),
                             _device_ptr(points, "points", (torch.float32, torch.float64)), ld, prec,
                             _device_ptr(out, "out"), _device_ptr(ids, "ids") if ids is not None else None,
                             current_stream())
        return out

    def autotune(self, points, n_nodes, candidates):
        """Pick the bin grid that evaluates this (d, Q) query sample fastest; returns the cells per axis."""
        torch = _torch()
        prec = FT_F32 if points.dtype == torch.float32 else FT_F64
        ptr = _device_ptr(points, "points", (torch.float32, torch.float64))
        return ft_source_autotune(self.handle, int(n_nodes), int(points.shape[1]), ptr, int(points.shape[1]), prec,
                                  list(candidates), current_stream())

    @property
    def info(self):
        return ft_source_get_info(self.handle)

    def integral(self):
        """Exact integral of each field over the source mesh (ft_source_integral)."""
        return ft_source_integral(self.handle, self.n_fields, current_stream())

    def take_out_of_domain(self):
        return ft_source_stats(self.handle, current_stream())


class Batch:
    """Many built-in-source transfers run together (ft_batch_create / ft_batch_run).

    targets, sources: Target and Source objects (kept alive by the batch);
    cfgs: one SampleCfg per transfer.  run() returns, per transfer, the
    solution x (device tensor, (n,) for one field, (F, n) for F > 1) and the
    load vector b, the reports and statuses (one per field, transfer by
    transfer).
    """

    def __init__(self, targets, sources, cfgs, graph=False):
        """sources=None: a batch for caller values (consume_run only)."""
        self.targets = list(targets)
        self.sources = list(sources) if sources is not None else [None] * len(self.targets)
        self.cfgs = list(cfgs)
        self.handle = ft_batch_create([t.handle for t in self.targets],
                                      [s.handle if s is not None else None for s in self.sources],
                                      self.cfgs, FT_BATCH_GRAPH if graph else 0, current_stream())

    def _outputs(self, xs, bs, want_b):
        torch = _torch()
        dev = self.targets[0].coords.device

        def shape(t, c):
            return (t.n_nodes,) if c.n_fields == 1 else (c.n_fields, t.n_nodes)
        if xs is None:
            xs = [torch.empty(shape(t, c), dtype=torch.float64, device=dev) for t, c in zip(self.targets, self.cfgs)]
        if want_b and bs is None:
            bs = [torch.empty(shape(t, c), dtype=torch.float64, device=dev) for t, c in zip(self.targets, self.cfgs)]
        f64 = (torch.float64,)
        xp = [_device_ptr(x, "x", f64) for x in xs]
        bp = [_device_ptr(b, "b", f64) for b in bs] if want_b else None
        return xs, bs, xp, bp

    def run(self, rtol=1e-14, max_iter=60, xs=None, bs=None, want_b=True):
        xs, bs, xp, bp = self._outputs(xs, bs, want_b)
        st, reps, sts = ft_batch_run(self.handle, SolveCfg(rtol, max_iter), xp, bp, current_stream(),
                                     n_systems=sum(c.n_fields for c in self.cfgs))
        return xs, bs, reps, sts, st

    def consume_run(self, values, rtol=1e-14, max_iter=60, xs=None, bs=None, want_b=True):
        """ft_batch_consume_run: values[k] holds transfer k's query values (its
        target sampled with cfgs[k] beforehand)."""
        torch = _torch()
        vp = [_device_ptr(v, "values", (torch.float64, torch.float32)) for v in values]
        xs, bs, xp, bp = self._outputs(xs, bs, want_b)
        st, reps, sts = ft_batch_consume_run(self.handle, SolveCfg(rtol, max_iter), vp, xp, bp, current_stream(),
                                             sum(c.n_fields for c in self.cfgs))
        return xs, bs, reps, sts, st

    def autotune(self, cache_path=None):
        """ft_batch_autotune: returns the number of transfer kinds timed (0: all from the cache)."""
        return ft_batch_autotune(self.handle, cache_path, current_stream())

    def variant(self, k):
        """(lanes per element, samples per lane) of transfer k's element stage."""
        return ft_batch_variant(self.handle, k)

    def close(self):
        if getattr(self, "handle", None):
            ft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Setup/online split (ft_plan_create / ft_plan_transfer): localize once,
    then transfer new nodal values of the source field as often as needed."""

    def __init__(self, target, source, cfg: SampleCfg):
        self.target, self.source, self.cfg = target, source, cfg
        self.handle = ft_plan_create(target.handle, source.handle, cfg, current_stream())

    def transfer(self, nodal_values=None):
        """nodal_values: (F, n_source_nodes) float64 device tensor, or None for the source's own.
        Follow with target.project()."""
        torch = _torch()
        ptr = None
        if nodal_values is not None:
            if tuple(nodal_values.shape) != (self.cfg.n_fields, self.source.n_nodes):
                raise ValueError(f"nodal_values must have shape ({self.cfg.n_fields}, {self.source.n_nodes})")
            ptr = _device_ptr(nodal_values, "nodal_values", (torch.float64,))
        ft_plan_transfer(self.handle, ptr, current_stream())

    def close(self):
        if getattr(self, "handle", None):
            ft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
