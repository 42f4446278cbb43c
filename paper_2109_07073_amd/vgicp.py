"""ctypes binding of libvgicp.so (C ABI in include/vgicp.h).

Argument marshalling only: every step of voxelization, linearization, cost
evaluation and overlap runs in the library's HIP kernels.  Device memory and
streams come from PyTorch-ROCm tensors; clouds are passed as tensors
xyz float32 (3, n) (coordinate planes) and cov float32 (n, 6) (per point
xx, xy, xz, yy, yz, zz) on the GPU.

The library must be built (python -m paper_2109_07073_amd.build); importing
this module without it raises ImportError.  There is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvgicp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vgicp.h")

OK, EINVAL, ENOMEM, ERANGE, ENONFINITE, EHIP, EFULL = 0, -1, -2, -3, -4, -5, -6
REQ = {"linearize": 0, "evaluate": 1, "overlap": 2}
GATE = {"above": 0, "at_least": 1}
SUBMAP = {0: "start", 1: "skip", 2: "insert", 3: "close"}
ACC = {"mixed": 0, "f32": 1, "f64": 2, "f32_comp": 3}
KERNELS = {"linearize": 0, "reduce": 1, "overlap": 2, "evaluate": 3}
SCHED = {"batched": 0, "per_factor": 1}
RESID = {"f64": 0, "f32": 1}
FUSED = {"f64": 0, "f32": 1}
FORM = {"auto": 0, "source": 1, "pair": 2}
LAYOUT = {"grouped": 0, "interleaved": 1, "balanced": 2}
NOALLOC_MAX_TILES = 32768      # VGICP_NOALLOC_MAX_TILES


class VgicpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class CCloud(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("cov", ctypes.c_void_p), ("n", ctypes.c_int64)]


class CFactor(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("tgt", ctypes.c_int32),
                ("pose_i", ctypes.c_int32), ("pose_j", ctypes.c_int32)]


class CServerRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_poses", ctypes.c_int32), ("n", ctypes.c_int64),
                ("factors", ctypes.c_void_p), ("h_poses", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("b", ctypes.c_void_p), ("e", ctypes.c_void_p),
                ("inliers", ctypes.c_void_p), ("overlap", ctypes.c_void_p)]


class COpts(ctypes.Structure):
    _fields_ = [("accum", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("resid", ctypes.c_int32),
                ("fp64_kappa", ctypes.c_float), ("fused", ctypes.c_int32),
                ("form", ctypes.c_int32)]


class CSubmapRules(ctypes.Structure):
    _fields_ = [("skip_above", ctypes.c_double), ("close_below", ctypes.c_double),
                ("max_frames", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", ctypes.c_int64), ("max_batch_factors", ctypes.c_int32),
                ("max_batch_points", ctypes.c_int32), ("max_batch_poses", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("tile_points", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("opts", COpts)]


_vp, _i32, _i64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_P = ctypes.POINTER

_PROTOS = {
    "vgicp_version": (ctypes.c_int, []),
    "vgicp_last_error": (ctypes.c_char_p, [_vp]),
    "vgicp_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, _P(_vp)]),
    "vgicp_ctx_set_stream": (ctypes.c_int, [_vp, _vp]),
    "vgicp_ctx_synchronize": (ctypes.c_int, [_vp]),
    "vgicp_ctx_destroy": (ctypes.c_int, [_vp]),
    "vgicp_ctx_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vgicp_ctx_read_timing": (ctypes.c_int, [_vp, ctypes.c_int, _P(_dbl), _P(_i64)]),
    "vgicp_ctx_reset_timing": (ctypes.c_int, [_vp]),
    "vgicp_voxelize": (ctypes.c_int, [_vp, _P(CCloud), _dbl, _P(_vp)]),
    "vgicp_map_info": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_dbl)]),
    "vgicp_map_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "vgicp_map_free": (ctypes.c_int, [_vp]),
    "vgicp_factorset_create": (ctypes.c_int, [_vp, _P(CCloud), _i32, _P(_vp), _i32, _P(CFactor),
                                              _i64, _i32, _i32, _P(_vp)]),
    "vgicp_factorset_info": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i32)]),
    "vgicp_factorset_destroy": (ctypes.c_int, [_vp]),
    "vgicp_factorset_graph_count": (ctypes.c_int, [_vp, _P(_i64)]),
    "vgicp_factorset_pairs": (ctypes.c_int, [_vp, _P(_i64), _vp]),
    "vgicp_factorset_tune": (ctypes.c_int, [_vp, _vp, _vp, _P(COpts), _vp, _vp, _vp, _vp, _vp,
                                            _i32, _P(_i32), _P(_dbl)]),
    "vgicp_assemble_system": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vgicp_validate_factors": (ctypes.c_int, [_i32, _i32, _i32, _P(CFactor), _i64]),
    "vgicp_linearize_factors": (ctypes.c_int, [_vp, _vp, _vp, _P(COpts), _vp, _vp, _vp, _vp, _vp]),
    "vgicp_evaluate_errors": (ctypes.c_int, [_vp, _vp, _vp, _P(COpts), _vp, _vp]),
    "vgicp_linearize_factors_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _P(COpts), _vp, _vp, _vp,
                                                       _vp, _vp]),
    "vgicp_overlap": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vgicp_server_create": (ctypes.c_int, [ctypes.c_int, _P(CServerConfig), _P(_vp)]),
    "vgicp_server_destroy": (ctypes.c_int, [_vp]),
    "vgicp_server_last_error": (ctypes.c_char_p, [_vp]),
    "vgicp_server_add_frame": (ctypes.c_int, [_vp, _vp, _vp, _i64, _dbl, _P(_i32)]),
    "vgicp_server_remove_frame": (ctypes.c_int, [_vp, _i32]),
    "vgicp_factorset_fp64_points": (ctypes.c_int, [_vp, _vp, _P(_i64)]),
    "vgicp_factorset_check": (ctypes.c_int, [_vp, _vp, _P(_i64), _P(_i64), _P(_i64)]),
    "vgicp_factorset_reorder": (ctypes.c_int, [_vp, _vp, _vp]),
    "vgicp_factorset_set_grid": (ctypes.c_int, [_vp, _vp, _i32]),
    "vgicp_factorset_time_kernel": (ctypes.c_int, [_vp, _vp, _vp, _P(COpts), _i32, _i32, _P(_dbl)]),
    "vgicp_factorset_grid": (ctypes.c_int, [_vp, _P(_i32)]),
    "vgicp_factorset_form": (ctypes.c_int, [_vp, _P(_i32)]),
    "vgicp_factorset_set_layout": (ctypes.c_int, [_vp, _vp, _i32]),
    "vgicp_factorset_layout": (ctypes.c_int, [_vp, _P(_i32)]),
    "vgicp_server_memory": (ctypes.c_int, [_vp, _P(_i64), _P(_i64)]),
    "vgicp_server_submit": (ctypes.c_int, [_vp, ctypes.c_int, _P(CFactor), _i64, _vp, _i32, _vp,
                                           _vp, _vp, _vp, _vp, _P(_i64)]),
    "vgicp_server_submit_many": (ctypes.c_int, [_vp, _P(CServerRequest), _i32, _P(_i64)]),
    "vgicp_server_poll": (ctypes.c_int, [_vp, _i64, _P(ctypes.c_int)]),
    "vgicp_server_wait": (ctypes.c_int, [_vp, _i64, _P(_dbl)]),
    "vgicp_server_stats": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i64)]),
    "vgicp_connect": (ctypes.c_int, [_vp, _P(CCloud), _vp, _P(_vp), _vp, _i32, _dbl, _i32, _vp,
                                     _vp, _vp, _P(_i32)]),
    "vgicp_submap_step": (ctypes.c_int, [_vp, _P(CSubmapRules), _P(CCloud), _vp, _vp, _vp, _vp,
                                         _vp, _i32, _P(_i32), _P(_dbl), _P(_dbl)]),
    "vgicp_server_connect": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _i32, _dbl, _i32, _vp, _vp,
                                            _vp, _P(_i32)]),
    "vgicp_server_submap_step": (ctypes.c_int, [_vp, _P(CSubmapRules), _i32, _vp, _i32, _vp, _i32,
                                                _vp, _i32, _P(_i32), _P(_dbl), _P(_dbl)]),
}


def header_symbols() -> list[str]:
    """Entry points declared in include/vgicp.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vgicp_\w+)\s*\(", text, re.M)))


def load_library() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2109_07073_amd.build`")
    # PyTorch-ROCm ships its own libamdhip64.so.7 / libhsa-runtime64.so.1.  Loading
    # torch first makes the dynamic loader bind libvgicp.so to that same runtime
    # (matched by SONAME), so torch's device pointers and streams are valid in
    # the library.  Two HIP runtimes in one process do not share devices.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def lib() -> ctypes.CDLL:
    return _lib


def _err(ctx_ptr) -> str:
    m = _lib.vgicp_last_error(ctx_ptr)
    return m.decode() if m else ""


def _check(code: int, ctx_ptr=None):
    if code != OK:
        raise VgicpError(code, _err(ctx_ptr))


def validate_factors(n_sources: int, n_maps: int, n_poses: int, factors) -> None:
    """Host-only validation of a factor list (no device needed)."""
    arr, n = _factor_array(factors)
    _check(_lib.vgicp_validate_factors(n_sources, n_maps, n_poses, arr, n))


class _FactorRows:
    """(n, 4) int32 rows viewed as a vgicp_factor array (same layout: four
    int32 fields); keeps the buffer alive while the pointer is in use."""

    def __init__(self, factors):
        f = np.asarray(factors, dtype=np.int32).reshape(-1, 4)
        self.rows = np.ascontiguousarray(f if f.shape[0] else np.zeros((1, 4), np.int32))
        self.n = int(f.shape[0])
        self._as_parameter_ = self.rows.ctypes.data_as(ctypes.POINTER(CFactor))


assert ctypes.sizeof(CFactor) == 16


def _factor_array(factors):
    rows = _FactorRows(factors)
    return rows, rows.n


# ---------------------------------------------------------------- torch glue

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_tensor(t, dtype, shape=None, name="tensor", on_gpu=True):
    """Check a tensor the library reads or writes: dtype, shape, contiguity,
    then (unless on_gpu is False) that it lives on the GPU; ValueError on the
    first mismatch, before anything reaches the library."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if on_gpu and not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    return t


def _check_outputs(out, specs):
    """`out` must hold a tensor for every (key, dtype, shape) of `specs`."""
    if not isinstance(out, dict):
        raise ValueError("out must be a dict of tensors")
    for key, dtype, shape in specs:
        if key not in out:
            raise ValueError(f"out is missing '{key}'")
        _dev_tensor(out[key], dtype, shape, f"out['{key}']", on_gpu=False)
    for key, dtype, shape in specs:
        _dev_tensor(out[key], dtype, shape, f"out['{key}']")
    return out


def _graph_needs_out(use_graph, out):
    if use_graph and out is None:
        raise ValueError("use_graph=True needs out=: a graph is captured per output pointer "
                         "set, so fresh outputs on every call would capture a new graph each "
                         "time")


def cloud_to_device(xyz, cov, device="cuda"):
    """(n,3)/(n,6) float32 host arrays -> device tensors xyz (3,n), cov (n,6)."""
    torch = _torch()
    x = torch.from_numpy(np.ascontiguousarray(np.asarray(xyz, np.float32).reshape(-1, 3).T))
    c = torch.from_numpy(np.ascontiguousarray(np.asarray(cov, np.float32).reshape(-1, 6)))
    return x.to(device).contiguous(), c.to(device).contiguous()


def _pad16(k: int) -> int:
    return (k + 15) & ~15


def clouds_to_device(clouds, device="cuda"):
    """Upload many (xyz (n,3), cov (n,6)) host clouds into one device buffer and
    return views xyz (3,n) / cov (n,6) per cloud (each array starts on a
    64-byte boundary), plus the buffer."""
    torch = _torch()
    sizes = [int(np.asarray(x).reshape(-1, 3).shape[0]) for x, _ in clouds]
    total = int(sum(_pad16(3 * n) + _pad16(6 * n) for n in sizes))
    host = np.zeros(max(total, 1), dtype=np.float32)
    views, off = [], 0
    for (x, c), n in zip(clouds, sizes):
        oc = off + _pad16(3 * n)
        host[off:off + 3 * n] = np.asarray(x, np.float32).reshape(-1, 3).T.reshape(-1)
        host[oc:oc + 6 * n] = np.asarray(c, np.float32).reshape(-1)
        views.append((off, oc, n))
        off = oc + _pad16(6 * n)
    buf = torch.from_numpy(host).to(device)
    out = [(buf[o:o + 3 * n].view(3, n), buf[oc:oc + 6 * n].view(n, 6)) for o, oc, n in views]
    return out, buf


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(_lib.vgicp_ctx_create(self.device, _stream_handle(self.stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        self.stream = stream
        _check(_lib.vgicp_ctx_set_stream(self._h, _stream_handle(stream)), self._h)

    def synchronize(self):
        _check(_lib.vgicp_ctx_synchronize(self._h), self._h)

    def set_timing(self, enable: bool = True):
        """Bracket each kernel launch (outside graphs) with HIP events."""
        _check(_lib.vgicp_ctx_set_timing(self._h, int(bool(enable))), self._h)

    def reset_timing(self):
        _check(_lib.vgicp_ctx_reset_timing(self._h), self._h)

    def read_timing(self, kernel: str):
        """(total milliseconds, launches) of a kernel kind since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib.vgicp_ctx_read_timing(self._h, KERNELS[kernel], ctypes.byref(ms),
                                          ctypes.byref(n)), self._h)
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.vgicp_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VoxelMap:
    def __init__(self, ctx: Context, handle):
        self._ctx = ctx
        self._h = handle
        nv, cap, nb, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(_lib.vgicp_map_info(handle, ctypes.byref(nv), ctypes.byref(cap), ctypes.byref(nb),
                                   ctypes.byref(r)))
        self.n_voxels, self.capacity = nv.value, cap.value
        self.device_bytes, self.resolution = nb.value, r.value

    @property
    def handle(self):
        return self._h

    def export(self):
        """Voxels in ordinal order: keys int32 (V,3), mean (V,3), cov (V,6), count (V,)."""
        torch = _torch()
        V = self.n_voxels
        dev = f"cuda:{self._ctx.device}"
        keys = torch.empty((V, 3), dtype=torch.int32, device=dev)
        mean = torch.empty((V, 3), dtype=torch.float32, device=dev)
        cov = torch.empty((V, 6), dtype=torch.float32, device=dev)
        cnt = torch.empty((V,), dtype=torch.int32, device=dev)
        _check(_lib.vgicp_map_export(self._ctx.handle, self._h, keys.data_ptr(), mean.data_ptr(),
                                     cov.data_ptr(), cnt.data_ptr()), self._ctx.handle)
        return {"keys": keys, "mean": mean, "cov": cov, "count": cnt}

    def free(self):
        if getattr(self, "_h", None):
            _lib.vgicp_map_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def voxelize(ctx: Context, xyz, cov, resolution: float) -> VoxelMap:
    """Voxel map of a device cloud (xyz (3,n), cov (n,6) float32 tensors)."""
    torch = _torch()
    n = int(xyz.shape[1]) if xyz.dim() == 2 else -1
    _dev_tensor(xyz, torch.float32, (3, n), "xyz")
    _dev_tensor(cov, torch.float32, (n, 6), "cov")
    c = CCloud(xyz.data_ptr() if n else None, cov.data_ptr() if n else None, n)
    h = ctypes.c_void_p()
    _check(_lib.vgicp_voxelize(ctx.handle, ctypes.byref(c), float(resolution), ctypes.byref(h)),
           ctx.handle)
    return VoxelMap(ctx, h)


class FactorSet:
    """Factor list bound to its source clouds and target maps.

    sources: list of (xyz (3,n), cov (n,6)) device tensors, read only while the
    set is created (the library keeps its own Morton-ordered copy of each cloud a
    factor uses); maps: list of VoxelMap (kept alive here); factors: (F, 4) rows
    (src, tgt, pose_i, pose_j)."""

    def __init__(self, ctx: Context, sources, maps, factors, n_poses: int, tile_points: int = 0):
        torch = _torch()
        self._ctx = ctx
        sources = list(sources)
        self._maps = list(maps)
        cl = (CCloud * max(1, len(sources)))()
        for k, (x, c) in enumerate(sources):
            n = int(x.shape[1])
            _dev_tensor(x, torch.float32, (3, n), f"sources[{k}].xyz")
            _dev_tensor(c, torch.float32, (n, 6), f"sources[{k}].cov")
            cl[k] = CCloud(x.data_ptr() if n else None, c.data_ptr() if n else None, n)
        mp = (ctypes.c_void_p * max(1, len(self._maps)))()
        for k, m in enumerate(self._maps):
            mp[k] = m.handle
        arr, nf = _factor_array(factors)
        self.factors = np.asarray(factors, dtype=np.int32).reshape(-1, 4).copy()
        self.n_poses = int(n_poses)
        h = ctypes.c_void_p()
        _check(_lib.vgicp_factorset_create(ctx.handle, cl, len(sources), mp, len(self._maps),
                                           arr, nf, self.n_poses, int(tile_points), ctypes.byref(h)),
               ctx.handle)
        self._h = h
        a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib.vgicp_factorset_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                         ctypes.byref(d)))
        self.n_factors, self.n_tiles, self.total_points = a.value, b.value, c.value
        self.tile_points = d.value
        self.source_sizes = np.array([int(sources[s][0].shape[1]) for s in self.factors[:, 0]],
                                     dtype=np.int64)
        n = ctypes.c_int64()
        _check(_lib.vgicp_factorset_pairs(h, ctypes.byref(n), None))
        self.pairs = np.zeros((n.value, 2), dtype=np.int32)
        if n.value:
            _check(_lib.vgicp_factorset_pairs(h, ctypes.byref(n),
                                              self.pairs.ctypes.data_as(ctypes.c_void_p)))

    @property
    def handle(self):
        return self._h

    def graph_count(self) -> int:
        """HIP graphs the factor set holds for graph replay (at most 8)."""
        n = ctypes.c_int64()
        _check(_lib.vgicp_factorset_graph_count(self._h, ctypes.byref(n)))
        return n.value

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.vgicp_factorset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _opts(accum: str, schedule: str, use_graph: bool, resid: str = "f64",
          fp64_kappa: float = 0.0, fused: str = "f64", form: str = "auto") -> COpts:
    if accum not in ACC:
        raise ValueError(f"accum must be one of {sorted(ACC)}")
    if schedule not in SCHED:
        raise ValueError(f"schedule must be one of {sorted(SCHED)}")
    if resid not in RESID:
        raise ValueError(f"resid must be one of {sorted(RESID)}")
    if fused not in FUSED:
        raise ValueError(f"fused must be one of {sorted(FUSED)}")
    if form not in FORM:
        raise ValueError(f"form must be one of {sorted(FORM)}")
    return COpts(ACC[accum], SCHED[schedule], int(bool(use_graph)), RESID[resid],
                 float(fp64_kappa), FUSED[fused], FORM[form])


def _check_poses(fs: FactorSet, poses):
    torch = _torch()
    return _dev_tensor(poses, torch.float64, (fs.n_poses, 12), "poses")


def linearize_factors(ctx: Context, fs: FactorSet, poses, accum: str = "mixed",
                      schedule: str = "batched", use_graph: bool = False,
                      with_corr: bool = False, out=None, resid: str = "f64",
                      fp64_kappa: float = 0.0, fused: str = "f64", form: str = "auto"):
    """Hessian factors of every factor at `poses` (float64 (P, 12) device).
    Returns dict of device tensors H (F,12,12), b (F,12), e (F,), inliers (F,)
    and corr (total_points,) when asked.  `out` may supply the same dict of
    preallocated tensors (needed for graph replay with stable pointers).
    `form`: "source" (21 + 6 + 1 source-frame sums expanded per factor),
    "pair" (Eqs. (5)-(6) term by term, 78 + 12 + 1 sums) or "auto" (the
    factor set's form, see tune_tiles)."""
    torch = _torch()
    _graph_needs_out(use_graph, out)
    F = fs.n_factors
    specs = [("H", torch.float64, (F, 12, 12)), ("b", torch.float64, (F, 12)),
             ("e", torch.float64, (F,)), ("inliers", torch.int64, (F,))]
    if out is not None:
        _check_outputs(out, specs)
    _check_poses(fs, poses)
    dev = f"cuda:{ctx.device}"
    if out is None:
        out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device=dev),
               "b": torch.empty((F, 12), dtype=torch.float64, device=dev),
               "e": torch.empty((F,), dtype=torch.float64, device=dev),
               "inliers": torch.empty((F,), dtype=torch.int64, device=dev)}
        if with_corr:
            out["corr"] = torch.empty((fs.total_points,), dtype=torch.int32, device=dev)
    corr = out.get("corr")
    if corr is not None:
        _dev_tensor(corr, torch.int32, (fs.total_points,), "out['corr']")
    o = _opts(accum, schedule, use_graph, resid, fp64_kappa, fused, form)
    _check(_lib.vgicp_linearize_factors(ctx.handle, fs.handle, poses.data_ptr(), ctypes.byref(o),
                                        out["H"].data_ptr(), out["b"].data_ptr(),
                                        out["e"].data_ptr(), out["inliers"].data_ptr(),
                                        corr.data_ptr() if corr is not None else None),
           ctx.handle)
    return out


def linearize_factors_noalloc(ctx: Context, fs: FactorSet, poses, out, accum: str = "mixed",
                              schedule: str = "batched", resid: str = "f64",
                              fp64_kappa: float = 0.0, fused: str = "f64"):
    """linearize_factors into caller-owned `out` (H, b, e, inliers and
    optionally corr, as linearize_factors returns them) through
    vgicp_linearize_factors_noalloc: the library allocates nothing during the
    call (its per-tile partials live in a fixed per-device array), so the
    factor set may have at most NOALLOC_MAX_TILES tiles, and calls that overlap
    on one device race."""
    torch = _torch()
    F = fs.n_factors
    if out is None:
        raise ValueError("linearize_factors_noalloc needs caller-owned outputs in `out`")
    _check_outputs(out, [("H", torch.float64, (F, 12, 12)), ("b", torch.float64, (F, 12)),
                         ("e", torch.float64, (F,)), ("inliers", torch.int64, (F,))])
    corr = out.get("corr")
    if corr is not None:
        _dev_tensor(corr, torch.int32, (fs.total_points,), "out['corr']")
    _check_poses(fs, poses)
    o = _opts(accum, schedule, False, resid, fp64_kappa, fused)
    _check(_lib.vgicp_linearize_factors_noalloc(
        ctx.handle, fs.handle, poses.data_ptr(), ctypes.byref(o), out["H"].data_ptr(),
        out["b"].data_ptr(), out["e"].data_ptr(), out["inliers"].data_ptr(),
        corr.data_ptr() if corr is not None else None), ctx.handle)
    return out


def evaluate_errors(ctx: Context, fs: FactorSet, poses, accum: str = "mixed",
                    schedule: str = "batched", use_graph: bool = False, out=None,
                    resid: str = "f64", fp64_kappa: float = 0.0, fused: str = "f64"):
    """Matching cost e (F,) and inliers (F,) without Jacobians."""
    torch = _torch()
    _graph_needs_out(use_graph, out)
    F = fs.n_factors
    if out is not None:
        _check_outputs(out, [("e", torch.float64, (F,)), ("inliers", torch.int64, (F,))])
    _check_poses(fs, poses)
    dev = f"cuda:{ctx.device}"
    if out is None:
        out = {"e": torch.empty((F,), dtype=torch.float64, device=dev),
               "inliers": torch.empty((F,), dtype=torch.int64, device=dev)}
    o = _opts(accum, schedule, use_graph, resid, fp64_kappa, fused)
    _check(_lib.vgicp_evaluate_errors(ctx.handle, fs.handle, poses.data_ptr(), ctypes.byref(o),
                                      out["e"].data_ptr(), out["inliers"].data_ptr()), ctx.handle)
    return out


def overlap(ctx: Context, fs: FactorSet, poses, out=None):
    """Overlap hit counts (F,) int64 and rates (F,) float64 (Eqs. (7)-(8))."""
    torch = _torch()
    F = fs.n_factors
    if out is not None:
        _check_outputs(out, [("hits", torch.int64, (F,)), ("overlap", torch.float64, (F,))])
    _check_poses(fs, poses)
    dev = f"cuda:{ctx.device}"
    if out is None:
        out = {"hits": torch.empty((F,), dtype=torch.int64, device=dev),
               "overlap": torch.empty((F,), dtype=torch.float64, device=dev)}
    _check(_lib.vgicp_overlap(ctx.handle, fs.handle, poses.data_ptr(), out["hits"].data_ptr(),
                              out["overlap"].data_ptr()), ctx.handle)
    return out


def tune_tiles(ctx: Context, fs: FactorSet, poses, candidates=None, accum: str = "mixed",
               resid: str = "f64", fp64_kappa: float = 0.0, fused: str = "f64",
               form: str = "auto"):
    """Time a linearization round per candidate tile size, grid, tile-table
    layout (grouped and balanced, and interleaved when factors share source
    copies) and (with form "auto") form,
    and keep the fastest (vgicp_factorset_tune).  Returns (tile_points, ms per
    round); grid(fs), layout_of(fs) and form_of(fs) give the rest."""
    torch = _torch()
    _check_poses(fs, poses)
    dev = f"cuda:{ctx.device}"
    F = fs.n_factors
    H = torch.empty((max(F, 1), 12, 12), dtype=torch.float64, device=dev)
    b = torch.empty((max(F, 1), 12), dtype=torch.float64, device=dev)
    e = torch.empty((max(F, 1),), dtype=torch.float64, device=dev)
    inl = torch.empty((max(F, 1),), dtype=torch.int64, device=dev)
    o = _opts(accum, "batched", False, resid, fp64_kappa, fused, form)
    cand = None
    n = 0
    if candidates is not None:
        c = np.ascontiguousarray(np.asarray(candidates, dtype=np.int32).reshape(-1))
        cand, n = c.ctypes.data_as(ctypes.c_void_p), c.size
    best, ms = ctypes.c_int32(), ctypes.c_double()
    _check(_lib.vgicp_factorset_tune(ctx.handle, fs.handle, poses.data_ptr(), ctypes.byref(o),
                                     H.data_ptr(), b.data_ptr(), e.data_ptr(), inl.data_ptr(),
                                     cand, n, ctypes.byref(best), ctypes.byref(ms)), ctx.handle)
    _refresh_tiles(fs)
    return best.value, ms.value


def time_kernel(ctx: Context, fs: FactorSet, poses, kernel: str = "linearize", reps: int = 20,
                accum: str = "mixed", resid: str = "f64", fp64_kappa: float = 0.0,
                fused: str = "f64", form: str = "auto") -> float:
    """Mean device milliseconds of one launch of a round's `kernel`
    ("linearize", "evaluate" or "overlap") over the whole factor set, from
    `reps` back-to-back launches between one pair of HIP events
    (vgicp_factorset_time_kernel)."""
    _check_poses(fs, poses)
    if kernel not in ("linearize", "evaluate", "overlap"):
        raise ValueError("kernel must be linearize, evaluate or overlap")
    o = _opts(accum, "batched", False, resid, fp64_kappa, fused, form)
    ms = ctypes.c_double()
    _check(_lib.vgicp_factorset_time_kernel(ctx.handle, fs.handle, poses.data_ptr(), ctypes.byref(o),
                                            KERNELS[kernel], int(reps), ctypes.byref(ms)),
           ctx.handle)
    return ms.value


def set_grid(ctx: Context, fs: FactorSet, persist_blocks: int):
    """Grid of the factor set's launches: 0 = one workgroup per tile, a
    multiple of 8 = a persistent grid of that many workgroups
    (vgicp_factorset_set_grid).  Results are the same bits on either grid."""
    _check(_lib.vgicp_factorset_set_grid(ctx.handle, fs.handle, int(persist_blocks)), ctx.handle)


def grid(fs: FactorSet) -> int:
    """The factor set's persistent-grid size, 0 for one workgroup per tile."""
    g = ctypes.c_int32()
    _check(_lib.vgicp_factorset_grid(fs.handle, ctypes.byref(g)))
    return g.value


def set_layout(ctx: Context, fs: FactorSet, layout: str):
    """Tile-table layout: "grouped" (factors by target map, each factor's
    tiles consecutive), "interleaved" (the factors reading one source copy
    side by side, tile by tile) or "balanced" (the grouped order in one run of
    about equal points per XCD, the factors ending a run cut into quarter-size
    tiles) (vgicp_factorset_set_layout).  Grouped and interleaved give the
    same bits; balanced changes the FP32 summation order of the factors it
    cuts shorter (integer outputs are the same)."""
    if layout not in LAYOUT:
        raise ValueError(f"layout must be one of {sorted(LAYOUT)}")
    _check(_lib.vgicp_factorset_set_layout(ctx.handle, fs.handle, LAYOUT[layout]), ctx.handle)
    _refresh_tiles(fs)


def layout_of(fs: FactorSet) -> str:
    """The factor set's tile-table layout ("grouped", "interleaved" or
    "balanced")."""
    v = ctypes.c_int32()
    _check(_lib.vgicp_factorset_layout(fs.handle, ctypes.byref(v)))
    return {v2: k for k, v2 in LAYOUT.items()}[v.value]


def _refresh_tiles(fs: FactorSet):
    a, nt, c3, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.vgicp_factorset_info(fs.handle, ctypes.byref(a), ctypes.byref(nt),
                                     ctypes.byref(c3), ctypes.byref(d)))
    fs.n_tiles, fs.tile_points = nt.value, d.value


def form_of(fs: FactorSet) -> str:
    """The form "auto" calls use on this factor set ("source" unless
    tune_tiles chose "pair")."""
    f = ctypes.c_int32()
    _check(_lib.vgicp_factorset_form(fs.handle, ctypes.byref(f)))
    return {v: k for k, v in FORM.items()}[f.value]


def reorder_by_target(ctx: Context, fs: FactorSet, poses):
    """Give every factor its own copy of its source points in the order of the
    target voxels they fall in at `poses` (vgicp_factorset_reorder);
    synchronizes.  Results change only by FP32 summation order."""
    torch = _torch()
    _check_poses(fs, poses)
    _check(_lib.vgicp_factorset_reorder(ctx.handle, fs.handle, poses.data_ptr()), ctx.handle)


def fp64_points(ctx: Context, fs: FactorSet) -> int:
    """Correspondences of the last linearize / evaluate call on `fs` whose
    fused covariance was formed in FP64: all inliers with fused="f64", those
    the fp64_kappa gate picked with fused="f32" (synchronizes)."""
    n = ctypes.c_int64()
    _check(_lib.vgicp_factorset_fp64_points(ctx.handle, fs.handle, ctypes.byref(n)), ctx.handle)
    return n.value


def check_inputs(ctx: Context, fs: FactorSet) -> dict:
    """vgicp_factorset_check: source points with a non-finite coordinate or
    covariance entry (counted at creation) and the degenerate correspondences
    of the last linearize / evaluate call (synchronizes)."""
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.vgicp_factorset_check(ctx.handle, fs.handle, ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c)), ctx.handle)
    return {"nonfinite_points": a.value, "nonfinite_covs": b.value, "degenerate_hits": c.value}


def assemble_system(ctx: Context, fs: FactorSet, H, b, out=None, with_offdiag: bool = True):
    """Global system blocks from per-factor H (F,12,12) and b (F,12) device
    float64 tensors: Hdiag (P,6,6), bvec (P,6) and, when asked, Hoff (K,6,6)
    for the pose pairs fs.pairs (K,2) (Sec. III-D)."""
    torch = _torch()
    dev = f"cuda:{ctx.device}"
    F, P, K = fs.n_factors, fs.n_poses, fs.pairs.shape[0]
    _dev_tensor(H, torch.float64, (F, 12, 12), "H")
    _dev_tensor(b, torch.float64, (F, 12), "b")
    if out is None:
        out = {"Hdiag": torch.empty((P, 6, 6), dtype=torch.float64, device=dev),
               "bvec": torch.empty((P, 6), dtype=torch.float64, device=dev)}
        if with_offdiag:
            out["Hoff"] = torch.empty((K, 6, 6), dtype=torch.float64, device=dev)
    _dev_tensor(out["Hdiag"], torch.float64, (P, 6, 6), "Hdiag")
    _dev_tensor(out["bvec"], torch.float64, (P, 6), "bvec")
    hoff = out.get("Hoff")
    if hoff is not None:
        _dev_tensor(hoff, torch.float64, (K, 6, 6), "Hoff")
    _check(_lib.vgicp_assemble_system(ctx.handle, fs.handle, H.data_ptr() if F else None,
                                      b.data_ptr() if F else None,
                                      out["Hdiag"].data_ptr() if P else None,
                                      out["bvec"].data_ptr() if P else None,
                                      hoff.data_ptr() if (hoff is not None and K) else None),
           ctx.handle)
    return out


# ------------------------------------------------------ keyframe control


def _pose12(p, name="pose"):
    a = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1))
    if a.shape != (12,):
        raise ValueError(f"{name} must hold 12 values (R row-major, then t)")
    return a


def _poses_n12(p, n, name="poses"):
    a = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1, 12))
    if a.shape[0] != n:
        raise ValueError(f"{name} must be ({n}, 12)")
    return a


def _rules(skip_above=0.95, close_below=0.10, max_frames=15):
    return CSubmapRules(float(skip_above), float(close_below), int(max_frames), 0)


def connect(ctx: Context, xyz, pose, maps, map_poses, threshold: float = 0.025,
            rule: str = "above"):
    """Overlap-gated factor creation (Sec. III-C): the overlap of the device
    cloud xyz (3, n) at `pose` (12,) against every map at map_poses (k, 12),
    and which of them `threshold` admits (rule "above": overlap > threshold,
    the paper's; "at_least": >=).  Returns dict of host arrays hits (k,),
    overlap (k,), admitted (k,) bool."""
    torch = _torch()
    n = int(xyz.shape[1]) if xyz.dim() == 2 else -1
    _dev_tensor(xyz, torch.float32, (3, n), "xyz")
    maps = list(maps)
    k = len(maps)
    P = _pose12(pose)
    MP = _poses_n12(map_poses, k, "map_poses")
    if rule not in GATE:
        raise ValueError(f"rule must be one of {sorted(GATE)}")
    c = CCloud(xyz.data_ptr() if n else None, None, n)
    mp = (ctypes.c_void_p * max(1, k))(*[m.handle for m in maps])
    hits = np.zeros(max(k, 1), np.int64)
    ov = np.zeros(max(k, 1), np.float64)
    adm = np.zeros(max(k, 1), np.int32)
    na = ctypes.c_int32()
    _check(_lib.vgicp_connect(ctx.handle, ctypes.byref(c), P.ctypes.data, mp, MP.ctypes.data, k,
                              float(threshold), GATE[rule], hits.ctypes.data, ov.ctypes.data,
                              adm.ctypes.data, ctypes.byref(na)), ctx.handle)
    return {"hits": hits[:k], "overlap": ov[:k], "admitted": adm[:k].astype(bool)}


def submap_step(ctx: Context, xyz, pose, first=None, first_pose=None, last=None,
                last_pose=None, n_submap: int = 0, skip_above: float = 0.95,
                close_below: float = 0.10, max_frames: int = 15):
    """Local-mapping decision (Sec. III-B) for the device cloud xyz (3, n) at
    `pose` arriving at a submap of n_submap frames whose first and last frames
    have maps `first` and `last` at their poses.  Returns (decision,
    overlap_first, overlap_last) with decision one of "start", "skip",
    "insert", "close"."""
    torch = _torch()
    n = int(xyz.shape[1]) if xyz.dim() == 2 else -1
    _dev_tensor(xyz, torch.float32, (3, n), "xyz")
    r = _rules(skip_above, close_below, max_frames)
    c = CCloud(xyz.data_ptr() if n else None, None, n)
    P = _pose12(pose)
    if n_submap > 0:
        FP, LP = _pose12(first_pose, "first_pose"), _pose12(last_pose, "last_pose")
        fh, lh, fp, lp = first.handle, last.handle, FP.ctypes.data, LP.ctypes.data
    else:
        fh = lh = fp = lp = None
    d, of, ol = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.vgicp_submap_step(ctx.handle, ctypes.byref(r), ctypes.byref(c), P.ctypes.data,
                                  fh, fp, lh, lp, int(n_submap), ctypes.byref(d),
                                  ctypes.byref(of), ctypes.byref(ol)), ctx.handle)
    return SUBMAP[d.value], of.value, ol.value


# ---------------------------------------------------------------- serving


class ServerRequest:
    """A submitted request: host output arrays are filled when it completes.
    `out` (a finished request of the same kind and size) lends its arrays, so
    that an optimizer's repeated rounds reuse their host buffers; the arrays
    serve one request in flight at a time."""

    def __init__(self, server, kind, n, out=None, pending=()):
        self.server = server
        self.kind = kind
        if out is not None:
            if out.kind != kind or out.inliers.shape[0] != n or out.ticket in server._inflight:
                raise ValueError("out must be a finished request of the same kind and size")
            # one set of host arrays serves one request in flight at a time
            holders = list(server._inflight.values()) + list(pending)
            if any(r.inliers is out.inliers for r in holders):
                raise ValueError("out's arrays are already lent to a request in flight")
            self.inliers, self.e, self.H, self.b, self.overlap = (out.inliers, out.e, out.H,
                                                                  out.b, out.overlap)
        else:
            self.inliers = np.zeros(n, dtype=np.int64)
            self.e = np.zeros(n, dtype=np.float64)
            self.H = np.zeros((n, 12, 12), dtype=np.float64) if kind == "linearize" else None
            self.b = np.zeros((n, 12), dtype=np.float64) if kind == "linearize" else None
            self.overlap = np.zeros(n, dtype=np.float64) if kind == "overlap" else None
        self.ticket = None
        self.latency_ms = None

    def done(self) -> bool:
        d = ctypes.c_int()
        _check_srv(_lib.vgicp_server_poll(self.server._h, self.ticket, ctypes.byref(d)), self.server)
        return bool(d.value)

    def wait(self):
        lat = ctypes.c_double()
        try:
            _check_srv(_lib.vgicp_server_wait(self.server._h, self.ticket, ctypes.byref(lat)),
                       self.server)
        finally:
            self.server._inflight.pop(self.ticket, None)
        self.latency_ms = lat.value
        return self


def _check_srv(code, server):
    if code != OK:
        msg = _lib.vgicp_server_last_error(server._h if server is not None else None)
        raise VgicpError(code, msg.decode() if msg else "")


class Server:
    """Continuous-batching server over resident keyframes (vgicp_server_*).

    Frames are host clouds (xyz (n,3), cov (n,6) float32) copied to the device
    and voxelized once; requests over frame ids and host poses are batched by
    the library's worker thread."""

    def __init__(self, device=0, memory_budget_bytes=0, max_batch_factors=4096,
                 max_batch_points=1 << 27, max_batch_poses=65536, inflight=2, tile_points=0,
                 accum="mixed", resid="f64", fp64_kappa=0.0, fused="f64"):
        cfg = CServerConfig(int(memory_budget_bytes), int(max_batch_factors), int(max_batch_points),
                            int(max_batch_poses), int(inflight), int(tile_points), 0,
                            _opts(accum, "batched", False, resid, fp64_kappa, fused))
        h = ctypes.c_void_p()
        code = _lib.vgicp_server_create(int(device), ctypes.byref(cfg), ctypes.byref(h))
        if code != OK:
            raise VgicpError(code, "vgicp_server_create failed")
        self._h = h
        # Submitted requests own the host arrays the worker writes into: keep
        # them alive until they are waited for or the server is closed.
        self._inflight = {}

    def add_frame(self, xyz, cov, resolution: float) -> int:
        x = np.ascontiguousarray(np.asarray(xyz, np.float32).reshape(-1, 3).T)
        c = np.ascontiguousarray(np.asarray(cov, np.float32).reshape(-1, 6))
        fid = ctypes.c_int32()
        _check_srv(_lib.vgicp_server_add_frame(self._h, x.ctypes.data, c.ctypes.data, x.shape[1],
                                               float(resolution), ctypes.byref(fid)), self)
        return fid.value

    def remove_frame(self, frame_id: int):
        _check_srv(_lib.vgicp_server_remove_frame(self._h, int(frame_id)), self)

    def memory(self):
        used, budget = ctypes.c_int64(), ctypes.c_int64()
        _check_srv(_lib.vgicp_server_memory(self._h, ctypes.byref(used), ctypes.byref(budget)), self)
        return used.value, budget.value

    def submit(self, kind: str, factors, poses, out: ServerRequest = None) -> ServerRequest:
        arr, n = _factor_array(factors)
        p = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 12))
        r = ServerRequest(self, kind, n, out)
        t = ctypes.c_int64()
        ptr = lambda a: a.ctypes.data if a is not None else None  # noqa: E731
        r._keep = (arr, p)
        _check_srv(_lib.vgicp_server_submit(self._h, REQ[kind], arr, n, p.ctypes.data, p.shape[0],
                                            ptr(r.H), ptr(r.b), ptr(r.e), ptr(r.inliers),
                                            ptr(r.overlap), ctypes.byref(t)), self)
        r.ticket = t.value
        self._inflight[r.ticket] = r
        return r

    def submit_many(self, requests) -> list:
        """Queue several requests at once (vgicp_server_submit_many), so that
        requests of one kind share a batch: `requests` is a sequence of
        (kind, factors, poses) or (kind, factors, poses, out) as for submit.
        All or nothing; returns the ServerRequests in order."""
        items = [tuple(r) + (None,) * (4 - len(r)) for r in requests]
        reqs = (CServerRequest * max(len(items), 1))()
        out, keep = [], []
        ptr = lambda a: a.ctypes.data if a is not None else None  # noqa: E731
        for q, (kind, factors, poses, prev) in enumerate(items):
            arr, n = _factor_array(factors)
            p = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(-1, 12))
            r = ServerRequest(self, kind, n, prev, pending=out)
            r._keep = (arr, p)
            reqs[q] = CServerRequest(REQ[kind], p.shape[0], n, arr.rows.ctypes.data, p.ctypes.data,
                                     ptr(r.H), ptr(r.b), ptr(r.e), ptr(r.inliers),
                                     ptr(r.overlap))
            out.append(r)
        tickets = (ctypes.c_int64 * max(len(items), 1))()
        _check_srv(_lib.vgicp_server_submit_many(self._h, reqs, len(items), tickets), self)
        for q, r in enumerate(out):
            r.ticket = tickets[q]
            self._inflight[r.ticket] = r
        return out

    def connect(self, frame: int, pose, candidates, candidate_poses, threshold: float = 0.025,
                rule: str = "above"):
        """vgicp_server_connect: overlap of resident frame `frame` at `pose`
        against the resident frames `candidates` at candidate_poses, batched
        with the server's other requests.  Returns dict hits, overlap,
        admitted (host arrays)."""
        cand = np.ascontiguousarray(np.asarray(candidates, np.int32).reshape(-1))
        k = cand.size
        P = _pose12(pose)
        CP = _poses_n12(candidate_poses, k, "candidate_poses")
        if rule not in GATE:
            raise ValueError(f"rule must be one of {sorted(GATE)}")
        hits = np.zeros(max(k, 1), np.int64)
        ov = np.zeros(max(k, 1), np.float64)
        adm = np.zeros(max(k, 1), np.int32)
        na = ctypes.c_int32()
        _check_srv(_lib.vgicp_server_connect(self._h, int(frame), P.ctypes.data, cand.ctypes.data,
                                             CP.ctypes.data, k, float(threshold), GATE[rule],
                                             hits.ctypes.data, ov.ctypes.data, adm.ctypes.data,
                                             ctypes.byref(na)), self)
        return {"hits": hits[:k], "overlap": ov[:k], "admitted": adm[:k].astype(bool)}

    def submap_step(self, frame: int, pose, first: int = -1, first_pose=None, last: int = -1,
                    last_pose=None, n_submap: int = 0, skip_above: float = 0.95,
                    close_below: float = 0.10, max_frames: int = 15):
        """vgicp_server_submap_step over resident frames; returns (decision,
        overlap_first, overlap_last)."""
        r = _rules(skip_above, close_below, max_frames)
        P = _pose12(pose)
        if n_submap > 0:
            FP, LP = _pose12(first_pose, "first_pose"), _pose12(last_pose, "last_pose")
            fp, lp = FP.ctypes.data, LP.ctypes.data
        else:
            fp = lp = None
        d, of, ol = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        _check_srv(_lib.vgicp_server_submap_step(self._h, ctypes.byref(r), int(frame), P.ctypes.data,
                                                 int(first), fp, int(last), lp, int(n_submap),
                                                 ctypes.byref(d), ctypes.byref(of),
                                                 ctypes.byref(ol)), self)
        return SUBMAP[d.value], of.value, ol.value

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check_srv(_lib.vgicp_server_stats(self._h, *[ctypes.byref(x) for x in v]), self)
        return {"batches": v[0].value, "requests": v[1].value,
                "max_requests_per_batch": v[2].value, "max_inflight": v[3].value}

    def close(self):
        """Finish every submitted request, then free the server."""
        if getattr(self, "_h", None):
            _lib.vgicp_server_destroy(self._h)
            self._h = None
            self._inflight.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
