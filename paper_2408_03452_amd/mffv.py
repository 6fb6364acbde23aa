"""Python binding of libmffv (ctypes): the C entry points under the same names.

Only argument marshalling happens here: tensors become device pointers, the
torch stream becomes a ``hipStream_t``, negative return codes become
:class:`MffvError`. Every step of the solver runs in the HIP library, which
must have been built (``paper_2408_03452_amd.build``); importing a missing or
broken library raises immediately instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime that libmffv then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmffv.so")

OK = 0
NOT_CONVERGED = 1
EINVAL = -1
ENOMEM = -2
EHIP = -3
EBREAKDOWN = -4
ESTATE = -5

FP32, FP64, FP32_IR = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_LEARNED = 0, 1, 2


class MffvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mffv error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("net", ctypes.c_void_p), ("single_reduction", ctypes.c_int),
                ("nn_every", ctypes.c_int), ("timing", ctypes.c_int),
                ("async_", ctypes.c_int),   # mffv_opts.async (a Python keyword)
                ("nn_smooth", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("ci", ctypes.c_int), ("remap", ctypes.c_int), ("vec", ctypes.c_int),
                ("blocks", ctypes.c_int), ("apply_us", ctypes.c_double),
                ("candidates", ctypes.c_int), ("phase_a_us", ctypes.c_double),
                ("seg", ctypes.c_int), ("apply_ci", ctypes.c_int), ("apply_remap", ctypes.c_int),
                ("apply_seg", ctypes.c_int), ("apply_blocks", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("ir_steps", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("ms", ctypes.c_double),
                ("phase_a_us", ctypes.c_double), ("phase_b_us", ctypes.c_double),
                ("precond_us", ctypes.c_double), ("timed_iters", ctypes.c_int),
                ("single_reduction", ctypes.c_int), ("nn_layer_us", ctypes.c_double * 4),
                ("nn_timed", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: (list(v) if k == "nn_layer_us" else v)
                for k, v in ((k, getattr(self, k)) for k, _ in self._fields_)}


_lib = None
_P = ctypes.c_void_p


def _declare(lib):
    sig = {
        "mffv_version": (ctypes.c_char_p, []),
        "mffv_last_error": (ctypes.c_char_p, []),
        "mffv_default_opts": (None, [ctypes.POINTER(Opts)]),
        "mffv_create_grid": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                                            ctypes.POINTER(_P)]),
        "mffv_destroy_grid": (None, [_P]),
        "mffv_perm_to_trans": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                                              ctypes.c_double, _P, _P, _P, _P]),
        "mffv_set_transmissibility": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_float, _P, _P,
                                                     _P]),
        "mffv_apply": (ctypes.c_int, [_P, _P, _P]),
        "mffv_apply_f64": (ctypes.c_int, [_P, _P, _P]),
        "mffv_true_residual": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
        "mffv_true_residual_noalloc": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
        # info: a host mffv_info (array) or, with opts.async, a device array
        "mffv_cg_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(Opts), _P]),
        "mffv_cg_solve_f64": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(Opts),
                                             ctypes.POINTER(Info)]),
        "mffv_cg_solve_batched": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int,
                                                 ctypes.POINTER(_P), ctypes.POINTER(_P),
                                                 ctypes.POINTER(Opts), _P]),
        "mffv_create_grid_faces": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.POINTER(_P)]),
        "mffv_set_face_transmissibility": (ctypes.c_int, [_P, _P, _P, ctypes.c_float, _P, _P, _P]),
        "mffv_face_order": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P]),
        "mffv_step_rhs": (ctypes.c_int, [_P, _P, _P, ctypes.c_float, _P, _P, _P, _P, _P]),
        "mffv_time_steps": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_float, _P, _P, _P, _P,
                                           ctypes.POINTER(Opts), _P]),
        "mffv_copy_probe": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
        "mffv_stream_probe": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P), ctypes.c_int,
                                             ctypes.c_int64, _P]),
        "mffv_net_num_params": (ctypes.c_int, []),
        "mffv_net_create": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
        "mffv_net_destroy": (None, [_P]),
        "mffv_net_get_params": (ctypes.c_int, [_P, _P, _P]),
        "mffv_net_set_params": (ctypes.c_int, [_P, _P]),
        "mffv_net_set_activation": (ctypes.c_int, [_P, ctypes.c_int]),
        "mffv_net_set_loss": (ctypes.c_int, [_P, ctypes.c_int]),
        "mffv_set_nn_run": (ctypes.c_int, [ctypes.c_int]),
        "mffv_nn_forward": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P,
                                           _P]),
        "mffv_nn_time_layers": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                               ctypes.c_int, _P, _P]),
        "mffv_nn_smooth_sample": (ctypes.c_int, [_P, ctypes.c_double, _P, _P]),
        "mffv_nn_loss_grad": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
        "mffv_nn_train_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_float,
                                              ctypes.POINTER(ctypes.c_double)]),
        "mffv_grid_feature": (ctypes.c_int, [_P, _P]),
        "mffv_set_launch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "mffv_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(TuneResult)]),
        "mffv_set_batched_launch": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
        "mffv_set_batched_watchdog": (ctypes.c_int, [ctypes.c_double]),
        "mffv_set_batched_rebalance": (ctypes.c_int, [ctypes.c_int]),
        "mffv_autotune_batched": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int,
                                                 ctypes.POINTER(_P), ctypes.POINTER(_P),
                                                 ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_double)]),
        "mffv_harvest_pair": (ctypes.c_int, [_P, _P, _P, _P, _P, _P,
                                             ctypes.POINTER(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def lib():
    """The loaded libmffv (raises if it is not built)."""
    global _lib
    if _lib is None:
        path = os.environ.get("MFFV_LIBRARY", LIB_PATH)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_2408_03452_amd.build` (hipcc, gfx950)")
        _lib = _declare(ctypes.CDLL(path))
    return _lib


def version() -> str:
    return lib().mffv_version().decode()


def last_error() -> str:
    return lib().mffv_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise MffvError(rc, last_error())
    return rc


def _ptr(t, dtype=None, n=None, name="array"):
    """Device pointer of a tensor (or None / int passthrough)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def default_opts(**kw) -> Opts:
    """mffv_opts with the library defaults; ``net=`` takes a :class:`Net`."""
    o = Opts()
    lib().mffv_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "net":
            o._net = v
            v = v.handle if v is not None else None
        setattr(o, k, v)
    return o


class Grid:
    """Owning wrapper of an ``mffv_grid*``."""

    def __init__(self, handle: int, shape, stream_ptr: int):
        self.handle = handle
        self.shape = tuple(shape)
        self.n = shape[0] * shape[1] * shape[2]
        self.stream_ptr = stream_ptr

    def close(self):
        if self.handle:
            lib().mffv_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_grid(nx: int, ny: int, nz: int, stream=None) -> Grid:
    h = _P()
    s = _stream(stream)
    _check(lib().mffv_create_grid(nx, ny, nz, s, ctypes.byref(h)))
    return Grid(h.value, (nx, ny, nz), s)


def destroy_grid(grid: Grid) -> None:
    grid.close()


def create_grid_faces(n: int, face_k, face_l, stream=None) -> Grid:
    """Face-list grid of n cells; face_k/face_l are host integer arrays of the
    cells each face joins (copied)."""
    import numpy as np
    fk = np.ascontiguousarray(face_k, dtype=np.int32)
    fl = np.ascontiguousarray(face_l, dtype=np.int32)
    if fk.shape != fl.shape or fk.ndim != 1:
        raise ValueError("face_k and face_l must be 1-D arrays of the same length")
    s = _stream(stream)
    h = _P()
    _check(lib().mffv_create_grid_faces(int(n), int(fk.size), fk.ctypes.data if fk.size else None,
                                        fl.ctypes.data if fl.size else None, s, ctypes.byref(h)))
    g = Grid(h.value, (int(n), 1, 1), s)
    g.nfaces = int(fk.size)
    return g


def face_order(n: int, face_k, face_l):
    """Reverse Cuthill-McKee numbering of a face-list mesh (mffv_face_order):
    a host int32 array, the new number of every cell."""
    import numpy as np
    fk = np.ascontiguousarray(face_k, dtype=np.int32)
    fl = np.ascontiguousarray(face_l, dtype=np.int32)
    out = np.empty(int(n), dtype=np.int32)
    _check(lib().mffv_face_order(int(n), int(fk.size), fk.ctypes.data if fk.size else None,
                                 fl.ctypes.data if fl.size else None, out.ctypes.data))
    return out


def set_face_transmissibility(grid: Grid, T, accum=None, accum_scalar=0.0, dmask=None, pD=None,
                              b_out=None) -> None:
    n = grid.n
    _check(lib().mffv_set_face_transmissibility(
        grid.handle, _ptr(T, torch.float32, getattr(grid, "nfaces", None), "T"),
        _ptr(accum, torch.float32, n, "accum"),
        float(accum_scalar), _ptr(dmask, torch.uint8, n, "dmask"), _ptr(pD, torch.float32, n, "pD"),
        _ptr(b_out, torch.float32, n, "b_out")))


def perm_to_trans(nx, ny, nz, k, kz_ratio, tx, ty, tz, stream=None) -> None:
    n = nx * ny * nz
    _check(lib().mffv_perm_to_trans(nx, ny, nz, _ptr(k, torch.float64, n, "k"), kz_ratio,
                                    _ptr(tx, torch.float32, n, "tx"),
                                    _ptr(ty, torch.float32, n, "ty"),
                                    _ptr(tz, torch.float32, n, "tz"), _stream(stream)))


def set_transmissibility(grid: Grid, tx, ty, tz, accum=None, accum_scalar=0.0, dmask=None,
                         pD=None, b_out=None) -> None:
    n = grid.n
    _check(lib().mffv_set_transmissibility(
        grid.handle, _ptr(tx, torch.float32, n, "tx"), _ptr(ty, torch.float32, n, "ty"),
        _ptr(tz, torch.float32, n, "tz"), _ptr(accum, torch.float32, n, "accum"),
        float(accum_scalar), _ptr(dmask, torch.uint8, n, "dmask"),
        _ptr(pD, torch.float32, n, "pD"), _ptr(b_out, torch.float32, n, "b_out")))


def apply(grid: Grid, x, y) -> None:
    _check(lib().mffv_apply(grid.handle, _ptr(x, torch.float32, grid.n, "x"),
                            _ptr(y, torch.float32, grid.n, "y")))


def apply_f64(grid: Grid, x, y) -> None:
    _check(lib().mffv_apply_f64(grid.handle, _ptr(x, torch.float64, grid.n, "x"),
                                _ptr(y, torch.float64, grid.n, "y")))


def true_residual(grid: Grid, b, x, r_out=None) -> float:
    rel = ctypes.c_double()
    _check(lib().mffv_true_residual(grid.handle, _ptr(b, torch.float32, grid.n, "b"),
                                    _ptr(x, torch.float64, grid.n, "x"),
                                    _ptr(r_out, torch.float64, grid.n, "r_out"),
                                    ctypes.byref(rel)))
    return rel.value


def true_residual_noalloc(grid: Grid, b, x, r_out) -> float:
    """mffv_true_residual without allocation (r_out required)."""
    rel = ctypes.c_double()
    _check(lib().mffv_true_residual_noalloc(grid.handle, _ptr(b, torch.float32, grid.n, "b"),
                                            _ptr(x, torch.float64, grid.n, "x"),
                                            _ptr(r_out, torch.float64, grid.n, "r_out"),
                                            ctypes.byref(rel)))
    return rel.value


def _device_infos(ns: int, like):
    """A device array of ns mffv_info structs (for opts.async_)."""
    return torch.zeros(ns * ctypes.sizeof(Info), dtype=torch.uint8, device=like.device)


def infos_from_device(arr) -> list:
    """Read the device mffv_info array of an asynchronous solve (synchronizes)."""
    host = arr.detach().cpu().numpy().tobytes()
    size = ctypes.sizeof(Info)
    return [Info.from_buffer_copy(host[i * size:(i + 1) * size]).as_dict() for i in range(len(host) // size)]


def cg_solve(grid: Grid, b, x, opts: Opts | None = None):
    """Returns (status, info dict); raises MffvError on errors. With
    ``opts.async_`` the solve is only enqueued (capture-safe once its plan
    exists) and the second item is a device array for infos_from_device."""
    bp = _ptr(b, torch.float32, grid.n, "b")
    xp = _ptr(x, torch.float32, grid.n, "x")
    if opts is not None and opts.async_:
        dinfo = _device_infos(1, x)
        rc = lib().mffv_cg_solve(grid.handle, bp, xp, ctypes.byref(opts), dinfo.data_ptr())
        return _check(rc), dinfo
    info = Info()
    rc = lib().mffv_cg_solve(grid.handle, bp, xp, ctypes.byref(opts) if opts is not None else None,
                             ctypes.addressof(info))
    return _check(rc), info.as_dict()


def cg_solve_f64(grid: Grid, b, x, opts: Opts | None = None):
    info = Info()
    rc = lib().mffv_cg_solve_f64(grid.handle, _ptr(b, torch.float64, grid.n, "b"),
                                 _ptr(x, torch.float64, grid.n, "x"),
                                 ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(info))
    return _check(rc), info.as_dict()


def cg_solve_batched(grids, b, x, opts: Opts | None = None):
    """Solve len(grids) systems in one launch; returns (status, [info dict])."""
    ns = len(grids)
    if len(b) != ns or len(x) != ns:
        raise ValueError("grids, b and x must have the same length")
    G = (_P * ns)(*[g.handle for g in grids])
    B = (_P * ns)(*[_ptr(bb, torch.float32, g.n, "b") for bb, g in zip(b, grids)])
    X = (_P * ns)(*[_ptr(xx, torch.float32, g.n, "x") for xx, g in zip(x, grids)])
    if opts is not None and opts.async_:
        # only enqueued: the infos land in device memory (read with infos_from_device)
        dinfo = _device_infos(ns, x[0])
        rc = lib().mffv_cg_solve_batched(G, ns, B, X, ctypes.byref(opts), dinfo.data_ptr())
        return _check(rc), dinfo
    infos = (Info * ns)()
    rc = lib().mffv_cg_solve_batched(G, ns, B, X, ctypes.byref(opts) if opts is not None else None,
                                     ctypes.addressof(infos))
    return _check(rc), [i.as_dict() for i in infos]


def step_rhs(grid: Grid, b, p_old, rhs, c=None, c_scalar=0.0, wi=None, pw=None, q=None) -> None:
    """Right-hand side of one backward-Euler step with wells (mffv_step_rhs)."""
    n = grid.n
    _check(lib().mffv_step_rhs(grid.handle, _ptr(b, torch.float32, n, "b"), _ptr(c, torch.float32, n, "c"),
                               float(c_scalar), _ptr(p_old, torch.float32, n, "p_old"),
                               _ptr(wi, torch.float32, n, "wi"), _ptr(pw, torch.float32, n, "pw"),
                               _ptr(q, torch.float32, n, "q"), _ptr(rhs, torch.float32, n, "rhs")))


def time_steps(grid: Grid, nsteps: int, b, p, c=None, c_scalar=0.0, wi=None, pw=None, q=None,
               opts: Opts | None = None):
    """nsteps backward-Euler steps in place on p (mffv_time_steps); returns
    (status, per-step info dicts). The operator's accumulation must be c + wi."""
    n = grid.n
    infos = (Info * max(nsteps, 1))()
    rc = lib().mffv_time_steps(grid.handle, int(nsteps), _ptr(b, torch.float32, n, "b"),
                               _ptr(c, torch.float32, n, "c"), float(c_scalar),
                               _ptr(wi, torch.float32, n, "wi"), _ptr(pw, torch.float32, n, "pw"),
                               _ptr(q, torch.float32, n, "q"), _ptr(p, torch.float32, n, "p"),
                               ctypes.byref(opts) if opts is not None else None, ctypes.addressof(infos))
    return _check(rc), [infos[i].as_dict() for i in range(nsteps)]


def set_launch(grid: Grid, ci: int, remap: int, seg: int = 0) -> None:
    """ci planes per block, remap 0/1, seg: 0 default, -1 flat, else row-segment length."""
    _check(lib().mffv_set_launch(grid.handle, ci, remap, seg))


def autotune(grid: Grid, cache_path: str | None = None) -> dict:
    out = TuneResult()
    _check(lib().mffv_autotune(grid.handle, cache_path.encode() if cache_path else None,
                               ctypes.byref(out)))
    return out.as_dict()


def set_batched_launch(blocks_per_cu: int, items_per_block: int) -> None:
    _check(lib().mffv_set_batched_launch(blocks_per_cu, items_per_block))


def set_batched_watchdog(seconds: float) -> None:
    """Limit of one per-system wait of the batched kernel (0: fail at once)."""
    _check(lib().mffv_set_batched_watchdog(float(seconds)))


def set_batched_rebalance(on: bool) -> None:
    """Block shares of repeated batched solves follow the last solve's iterations (default on)."""
    _check(lib().mffv_set_batched_rebalance(1 if on else 0))


def autotune_batched(grids, b, x, opts: Opts | None = None) -> dict:
    ns = len(grids)
    G = (_P * ns)(*[g.handle for g in grids])
    B = (_P * ns)(*[_ptr(bb, torch.float32, g.n, "b") for bb, g in zip(b, grids)])
    X = (_P * ns)(*[_ptr(xx, torch.float32, g.n, "x") for xx, g in zip(x, grids)])
    bpc, ipb, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().mffv_autotune_batched(G, ns, B, X, ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(bpc), ctypes.byref(ipb), ctypes.byref(ms)))
    return {"blocks_per_cu": bpc.value, "items_per_block": ipb.value, "ms": ms.value}


def stream_probe(ins, outs, stream=None) -> None:
    """Streaming probe (mffv_stream_probe): every tensor of outs receives the
    sum of the tensors of ins (FP32 device tensors of one length)."""
    n = ins[0].numel()
    I = (_P * len(ins))(*[_ptr(t, torch.float32, n, "in") for t in ins])
    O = (_P * len(outs))(*[_ptr(t, torch.float32, n, "out") for t in outs])
    _check(lib().mffv_stream_probe(I, len(ins), O, len(outs), n, _stream(stream)))


def copy_probe(dst, src, nbytes: int, stream=None) -> None:
    _check(lib().mffv_copy_probe(_ptr(dst), _ptr(src), nbytes, _stream(stream)))


# --- learned preconditioner ------------------------------------------------


class Net:
    """Owning wrapper of an ``mffv_net*`` (network weights on the device)."""

    def __init__(self, handle: int):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().mffv_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def net_num_params() -> int:
    return lib().mffv_net_num_params()


def _host_f32(a, n, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    if a.size != n:
        raise ValueError(f"{name} must have {n} values")
    return a


def net_create(params=None) -> Net:
    h = _P()
    n = net_num_params()
    arr = None if params is None else _host_f32(params, n, "params")
    _check(lib().mffv_net_create(None if arr is None else arr.ctypes.data, ctypes.byref(h)))
    net = Net(h.value)
    net._keep = arr
    return net


def net_set_activation(net: Net, relu: bool) -> None:
    _check(lib().mffv_net_set_activation(net.handle, 1 if relu else 0))


def net_set_loss(net: Net, kind: int) -> None:
    _check(lib().mffv_net_set_loss(net.handle, int(kind)))


def set_nn_run(run: int) -> None:
    """Planes per block of the network's marching convolutions (0: automatic)."""
    _check(lib().mffv_set_nn_run(int(run)))


def net_destroy(net: Net) -> None:
    net.close()


def net_get_params(net: Net):
    """(params, grads) as host float32 arrays."""
    import numpy as np
    n = net_num_params()
    p = np.empty(n, dtype=np.float32)
    g = np.empty(n, dtype=np.float32)
    _check(lib().mffv_net_get_params(net.handle, p.ctypes.data, g.ctypes.data))
    return p, g


def net_set_params(net: Net, params) -> None:
    arr = _host_f32(params, net_num_params(), "params")
    _check(lib().mffv_net_set_params(net.handle, arr.ctypes.data))


def nn_forward(net: Net, shape, r_hat, feat, out, stream=None) -> None:
    nx, ny, nz = shape
    n = nx * ny * nz
    _check(lib().mffv_nn_forward(net.handle, nx, ny, nz, _ptr(r_hat, torch.float32, n, "r_hat"),
                                 _ptr(feat, torch.float32, n, "feat"),
                                 _ptr(out, torch.float32, n, "out"), _stream(stream)))


def nn_smooth_sample(grid: Grid, omega: float, r_hat, out) -> None:
    """out = (I - omega A~) r_hat on the unknown cells (the residual the network sees between the sweeps)."""
    _check(lib().mffv_nn_smooth_sample(grid.handle, float(omega), _ptr(r_hat, torch.float32, grid.n, "r_hat"),
                                       _ptr(out, torch.float32, grid.n, "out")))


def nn_time_layers(net: Net, shape, r_hat, feat, reps: int = 20, stream=None) -> list:
    """Mean microseconds per launch of each of the four layers (back-to-back launches)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    us = (ctypes.c_double * 4)()
    _check(lib().mffv_nn_time_layers(net.handle, nx, ny, nz, _ptr(r_hat, torch.float32, n, "r_hat"),
                                     _ptr(feat, torch.float32, n, "feat"), int(reps), ctypes.addressof(us),
                                     _stream(stream)))
    return list(us)


def nn_loss_grad(net: Net, grid: Grid, r_hat, target) -> float:
    """Energy-norm loss of one pair on the grid's operator; the gradient stays in the net."""
    loss = ctypes.c_double()
    n = grid.n
    _check(lib().mffv_nn_loss_grad(net.handle, grid.handle, _ptr(r_hat, torch.float32, n, "r_hat"),
                                   _ptr(target, torch.float32, n, "target"), ctypes.byref(loss)))
    return loss.value


def nn_train_step(net: Net, grid: Grid, r_hat, target, lr: float, want_loss: bool = False):
    loss = ctypes.c_double()
    n = grid.n
    _check(lib().mffv_nn_train_step(net.handle, grid.handle, _ptr(r_hat, torch.float32, n, "r_hat"),
                                    _ptr(target, torch.float32, n, "target"), float(lr),
                                    ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def grid_feature(grid: Grid, feat) -> None:
    _check(lib().mffv_grid_feature(grid.handle, _ptr(feat, torch.float32, grid.n, "feat")))


def harvest_pair(grid: Grid, b, x, x_star, r_hat, target) -> float:
    """Fill the scaled (r_hat, target) pair for iterate x; returns the scale s."""
    s = ctypes.c_float()
    n = grid.n
    _check(lib().mffv_harvest_pair(grid.handle, _ptr(b, torch.float32, n, "b"),
                                   _ptr(x, torch.float32, n, "x"),
                                   _ptr(x_star, torch.float64, n, "x_star"),
                                   _ptr(r_hat, torch.float32, n, "r_hat"),
                                   _ptr(target, torch.float32, n, "target"), ctypes.byref(s)))
    return s.value
