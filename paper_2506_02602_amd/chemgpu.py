"""Thin ctypes binding of ``libchemgpu.so`` (argument marshalling only).

Every function forwards to the C entry point of the same name in
``include/chemgpu.h``; device buffers are torch tensors on the GPU (their
``data_ptr()`` is passed through) and the stream is torch's current HIP stream
unless one is given.  There is no fallback: if the built library is missing
the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libchemgpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")

# torch ships its own HIP runtime under the same SONAME (libamdhip64.so.7);
# loading torch first makes the library bind to that copy, so the process
# holds one runtime and torch's device memory and streams are usable here.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

CHEM_OK = 0
CELL_OK, CELL_MAXSTEPS, CELL_NONFINITE, CELL_H_UNDERFLOW = 0, 1, 2, 3


class chem_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int32),
                ("chunk_steps", C.c_int32), ("block_size", C.c_int32),
                ("fixed_steps", C.c_int32),
                ("tail_steps", C.c_int32),
                ("scheme", C.c_int32),
                ("tail_cap", C.c_int32),
                ("pool_order", C.c_int32)]


class chem_box(C.Structure):
    _fields_ = [("state", C.c_void_p), ("ld", C.c_int64), ("n_cells", C.c_int64),
                ("dt", C.c_double), ("n_sub", C.c_int32), ("level", C.c_int32),
                ("status", C.c_void_p), ("counts", C.c_void_p)]


class ChemError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.chem_last_error().decode()
        super().__init__(f"{where}: {_lib.chem_strerror(code).decode()} ({code}): {msg}")
        self.code = code


_P = C.c_void_p
_lib.chem_strerror.argtypes = [C.c_int]
_lib.chem_strerror.restype = C.c_char_p
_lib.chem_last_error.argtypes = []
_lib.chem_last_error.restype = C.c_char_p
_lib.chem_mech_load.argtypes = [C.c_char_p, C.POINTER(_P)]
_lib.chem_mech_load.restype = C.c_int
_lib.chem_mech_query.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_uint64)]
_lib.chem_mech_query.restype = C.c_int
_lib.chem_mech_free.argtypes = [_P]
_lib.chem_mech_free.restype = None
_lib.chem_workspace_reserve.argtypes = [_P, C.c_int64]
_lib.chem_workspace_reserve.restype = C.c_int
_lib.chem_set_kernel_timing.argtypes = [_P, C.c_int32]
_lib.chem_set_kernel_timing.restype = C.c_int
_lib.chem_kernel_times.argtypes = [_P, C.POINTER(C.c_float), C.c_int32]
_lib.chem_kernel_times.restype = C.c_int
_lib.chem_integrate.argtypes = [_P, _P, C.c_int64, C.c_int64, C.c_double,
                                C.POINTER(chem_opts), _P, _P, _P]
_lib.chem_integrate.restype = C.c_int
_lib.chem_integrate_batched.argtypes = [_P, C.POINTER(chem_box), C.c_int32, C.POINTER(chem_opts), _P]
_lib.chem_integrate_batched.restype = C.c_int
_lib.chem_graph_capture_batched.argtypes = [_P, C.POINTER(chem_box), C.c_int32,
                                            C.POINTER(chem_opts), _P, C.POINTER(_P)]
_lib.chem_graph_capture_batched.restype = C.c_int
_lib.chem_graph_launch.argtypes = [_P, _P]
_lib.chem_graph_launch.restype = C.c_int
_lib.chem_graph_destroy.argtypes = [_P]
_lib.chem_graph_destroy.restype = None
_lib.chem_autotune.argtypes = [_P, C.POINTER(chem_box), C.c_int32, C.POINTER(chem_opts), C.c_int32,
                               C.c_char_p, _P, C.POINTER(chem_opts)]
_lib.chem_autotune.restype = C.c_int


def _check(rc, where):
    if rc != CHEM_OK:
        raise ChemError(rc, where)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


SCHEMES = {"lsrk": 0, "rkf45": 1, "ros4": 2}


def make_opts(rtol=0.0, atol=0.0, max_steps=0, chunk_steps=0, block_size=0, fixed_steps=0,
              tail_steps=0, scheme="lsrk", tail_cap=0, pool_order=0):
    return chem_opts(rtol, atol, max_steps, chunk_steps, block_size, fixed_steps, tail_steps,
                     SCHEMES[scheme] if isinstance(scheme, str) else int(scheme), tail_cap,
                     pool_order)


class Mechanism:
    """Owns a ``chem_mech`` handle.

    The library's integration calls allocate nothing: they run on the
    workspace that ``chem_workspace_reserve`` allocated and return
    CHEM_ECAPACITY past it.  With ``auto_reserve`` (the default) the wrappers
    below grow the reservation before a call on more cells than it holds (a
    reservation that grows waits for the device first); a caller that wants a
    fixed footprint reserves once up front, or sets ``auto_reserve = False``
    and gets the library's error instead."""

    def __init__(self, path: str, reserve: int = 0, auto_reserve: bool = True):
        h = _P()
        _check(_lib.chem_mech_load(path.encode(), C.byref(h)), "chem_mech_load")
        self.handle = h
        ns, nr, hsh = C.c_int32(), C.c_int32(), C.c_uint64()
        _check(_lib.chem_mech_query(h, C.byref(ns), C.byref(nr), C.byref(hsh)), "chem_mech_query")
        self.n_species, self.n_reactions, self.hash = ns.value, nr.value, hsh.value
        self.path = path
        self.reserved = -1
        self.auto_reserve = auto_reserve
        if reserve:
            chem_workspace_reserve(self, reserve)

    def close(self):
        if getattr(self, "handle", None):
            _lib.chem_mech_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chem_mech_load(path: str, reserve: int = 0) -> Mechanism:
    return Mechanism(path, reserve=reserve)


def chem_workspace_reserve(mech: Mechanism, max_cells: int) -> None:
    _check(_lib.chem_workspace_reserve(mech.handle, int(max_cells)), "chem_workspace_reserve")
    mech.reserved = max(mech.reserved, int(max_cells))


def _reserve_for(mech: Mechanism, n: int) -> None:
    if mech.auto_reserve and n > mech.reserved:
        chem_workspace_reserve(mech, n)


def chem_set_kernel_timing(mech: Mechanism, on: bool = True) -> None:
    _check(_lib.chem_set_kernel_timing(mech.handle, 1 if on else 0), "chem_set_kernel_timing")


def chem_kernel_times(mech: Mechanism) -> dict:
    """Durations (ms) of the last timed call's launches (waits for it);
    `total` the whole flow step."""
    ms = (C.c_float * 5)()
    _check(_lib.chem_kernel_times(mech.handle, ms, 5), "chem_kernel_times")
    return {"persistent": ms[0], "tail_sort": ms[1], "coop": ms[2], "resume": ms[3],
            "total": ms[4]}


_lib.chem_tail_stats.argtypes = [_P, C.POINTER(C.c_int64), C.c_int32]
_lib.chem_tail_stats.restype = C.c_int


def chem_tail_stats(mech: Mechanism) -> dict:
    """Tail list of the last timed call: cells handed over, of them finished
    by the cooperative kernel, and the steps that kernel took."""
    out = (C.c_int64 * 3)()
    _check(_lib.chem_tail_stats(mech.handle, out, 3), "chem_tail_stats")
    return {"handed_over": out[0], "cooperative": out[1], "cooperative_steps": out[2]}


def chem_integrate(mech: Mechanism, state, dt: float, opts: chem_opts | None = None,
                   stream=None, status=None, counts=None, n_cells=None) -> None:
    """state: float64 CUDA tensor [N+3, ld] (rows T, Y.., rho, h), updated in place."""
    ld = state.shape[1]
    n = ld if n_cells is None else int(n_cells)
    assert state.dtype.itemsize == 8 and state.is_contiguous() and state.shape[0] == mech.n_species + 3
    if status is not None:
        assert status.numel() >= n and status.element_size() == 4
    if counts is not None:
        assert counts.numel() >= 2 * n and counts.element_size() == 4
    o = opts if opts is not None else make_opts()
    _reserve_for(mech, n)
    _check(_lib.chem_integrate(mech.handle, _ptr(state), ld, n, float(dt), C.byref(o),
                               _stream(stream), _ptr(status), _ptr(counts)), "chem_integrate")


_lib.chem_integrate_noalloc.argtypes = [_P, _P, C.c_int64, C.c_int64, C.c_double,
                                        C.POINTER(chem_opts), _P, _P, _P]
_lib.chem_integrate_noalloc.restype = C.c_int
NOALLOC_MAX_CELLS = 1 << 20


def chem_integrate_noalloc(mech: Mechanism, state, dt: float, opts: chem_opts | None = None,
                           stream=None, status=None, counts=None, n_cells=None) -> None:
    """As chem_integrate, on the library's fixed scratch array (no workspace,
    no allocation; at most NOALLOC_MAX_CELLS cells; calls overlapping on one
    GPU race)."""
    ld = state.shape[1]
    n = ld if n_cells is None else int(n_cells)
    assert state.dtype.itemsize == 8 and state.is_contiguous() and state.shape[0] == mech.n_species + 3
    if status is not None:
        assert status.numel() >= n and status.element_size() == 4
    if counts is not None:
        assert counts.numel() >= 2 * n and counts.element_size() == 4
    o = opts if opts is not None else make_opts()
    _check(_lib.chem_integrate_noalloc(mech.handle, _ptr(state), ld, n, float(dt), C.byref(o),
                                       _stream(stream), _ptr(status), _ptr(counts)),
           "chem_integrate_noalloc")


_lib.surrogate_create.argtypes = [_P, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(_P)]
_lib.surrogate_query.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
_lib.surrogate_get_params.argtypes = [_P, _P, _P]
_lib.surrogate_set_params.argtypes = [_P, _P, _P]
_lib.surrogate_make_pairs.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_double, _P, _P, _P, _P]
_lib.surrogate_train.argtypes = [_P, _P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                                 _P, _P]
_lib.surrogate_forward.argtypes = [_P, _P, C.c_int64, _P, _P]
_lib.surrogate_grad.argtypes = [_P, _P, _P, C.c_int32, _P, C.POINTER(C.c_float), _P]
_lib.surrogate_infer.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_double, C.POINTER(C.c_double),
                                 C.c_int32, C.POINTER(chem_opts), _P, _P, _P, _P, _P,
                                 C.POINTER(C.c_int64)]
_lib.surrogate_reserve.argtypes = [_P, C.c_int64]
_lib.surrogate_graph_capture.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_double,
                                         C.POINTER(C.c_double), C.POINTER(chem_opts), _P,
                                         C.POINTER(_P)]
_lib.surrogate_autotune.argtypes = [_P, _P, _P, C.c_int64, C.c_int64, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(chem_opts), C.c_int32,
                                    C.c_char_p, _P, C.POINTER(chem_opts)]
_lib.surrogate_save.argtypes = [_P, C.c_char_p]
_lib.surrogate_load.argtypes = [_P, C.c_char_p, C.POINTER(_P)]
_lib.surrogate_free.argtypes = [_P]
_lib.surrogate_free.restype = None
for _n in ("surrogate_create", "surrogate_query", "surrogate_get_params", "surrogate_set_params",
           "surrogate_make_pairs", "surrogate_train", "surrogate_forward", "surrogate_grad",
           "surrogate_infer", "surrogate_save", "surrogate_load", "surrogate_reserve"):
    getattr(_lib, _n).restype = C.c_int

TRUST_HULL, TRUST_ELEM, TRUST_POS, TRUST_ENERGY, TRUST_NONFINITE = 1, 2, 4, 8, 16


class Surrogate:
    """Owns a ``chem_surr`` handle (see include/chemgpu.h)."""

    def __init__(self, mech: Mechanism, seed: int = 0, handle=None):
        self.mech = mech
        if handle is None:
            h = _P()
            _check(_lib.surrogate_create(mech.handle, 128, 3, int(seed), C.byref(h)),
                   "surrogate_create")
            handle = h
        self.handle = handle
        self.reserved = -1
        ni, no, P = C.c_int32(), C.c_int32(), C.c_int64()
        _check(_lib.surrogate_query(self.handle, C.byref(ni), C.byref(no), C.byref(P)),
               "surrogate_query")
        self.n_in, self.n_out, self.n_params = ni.value, no.value, P.value

    @property
    def norm_size(self):
        return 4 * self.n_in + 2 * self.n_out

    def get_params(self):
        import numpy as np
        th = np.zeros(self.n_params, np.float32)
        nm = np.zeros(self.norm_size, np.float32)
        _check(_lib.surrogate_get_params(self.handle, th.ctypes.data, nm.ctypes.data),
               "surrogate_get_params")
        return th, nm

    def set_params(self, theta=None, norm=None):
        import numpy as np
        th = None if theta is None else np.ascontiguousarray(theta, np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        _check(_lib.surrogate_set_params(self.handle, None if th is None else th.ctypes.data,
                                         None if nm is None else nm.ctypes.data),
               "surrogate_set_params")

    def close(self):
        if getattr(self, "handle", None):
            _lib.surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_create(mech: Mechanism, seed: int = 0) -> Surrogate:
    return Surrogate(mech, seed)


def surrogate_make_pairs(mech: Mechanism, before, after, dt=0.0, dt_cells=None, X=None, Y=None,
                         stream=None):
    import torch
    n = before.shape[1]
    if X is None:
        X = torch.empty((n, mech.n_species + 3), dtype=torch.float32, device=before.device)
    if Y is None:
        Y = torch.empty((n, mech.n_species + 1), dtype=torch.float32, device=before.device)
    _check(_lib.surrogate_make_pairs(mech.handle, before.data_ptr(), after.data_ptr(), n, n,
                                     float(dt), _ptr(dt_cells), X.data_ptr(), Y.data_ptr(),
                                     _stream(stream)), "surrogate_make_pairs")
    return X, Y


def surrogate_train(s: Surrogate, X, Y, epochs=1, batch=4096, lr=1e-3, seed=0, stream=None):
    import numpy as np
    loss = np.zeros(max(epochs, 1), np.float32)
    _check(_lib.surrogate_train(s.handle, X.data_ptr(), Y.data_ptr(), X.shape[0], int(epochs),
                                int(batch), float(lr), int(seed), _stream(stream), loss.ctypes.data),
           "surrogate_train")
    return loss[:epochs]


def surrogate_forward(s: Surrogate, X, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((X.shape[0], s.n_out), dtype=torch.float32, device=X.device)
    _check(_lib.surrogate_forward(s.handle, X.data_ptr(), X.shape[0], out.data_ptr(),
                                  _stream(stream)), "surrogate_forward")
    return out


def surrogate_grad(s: Surrogate, Xn, Yn, grad=None, stream=None):
    import torch
    if grad is None:
        grad = torch.empty(s.n_params, dtype=torch.float32, device=Xn.device)
    loss = C.c_float()
    _check(_lib.surrogate_grad(s.handle, Xn.data_ptr(), Yn.data_ptr(), Xn.shape[0], grad.data_ptr(),
                               C.byref(loss), _stream(stream)), "surrogate_grad")
    return grad, loss.value


def surrogate_reserve(s: Surrogate, max_cells: int) -> None:
    _check(_lib.surrogate_reserve(s.handle, int(max_cells)), "surrogate_reserve")
    s.reserved = max(s.reserved, int(max_cells))


def surrogate_infer(s: Surrogate, mech: Mechanism, state, dt, trust, fallback=True, opts=None,
                    stream=None, trust_code=None, out_std=None, status=None, counts=None,
                    n_cells=None, want_count=False):
    ld = state.shape[1]
    n = ld if n_cells is None else int(n_cells)
    if fallback:
        _reserve_for(mech, n)
        if mech.auto_reserve and n > s.reserved:
            surrogate_reserve(s, n)
    tr = (C.c_double * 4)(*[float(x) for x in trust])
    o = opts if opts is not None else make_opts()
    cnt = C.c_int64(-1)
    _check(_lib.surrogate_infer(s.handle, mech.handle, state.data_ptr(), ld, n, float(dt), tr,
                                1 if fallback else 0, C.byref(o), _stream(stream), _ptr(trust_code),
                                _ptr(out_std), _ptr(status), _ptr(counts),
                                C.byref(cnt) if want_count else None), "surrogate_infer")
    return cnt.value if want_count else None


def surrogate_autotune(s: Surrogate, mech: Mechanism, state, dt, trust, base=None, reps=3,
                       cache_path=None, stream=None, n_cells=None) -> chem_opts:
    """Launch for surrogate_infer's FP64 fallback, tuned on whole surrogate
    steps over `state` (restored on return)."""
    ld = state.shape[1]
    n = ld if n_cells is None else int(n_cells)
    tr = (C.c_double * 4)(*[float(x) for x in trust])
    o = base if base is not None else make_opts()
    best = chem_opts()
    _reserve_for(mech, n)
    if mech.auto_reserve and n > s.reserved:
        surrogate_reserve(s, n)
    _check(_lib.surrogate_autotune(s.handle, mech.handle, state.data_ptr(), ld, n, float(dt), tr,
                                   C.byref(o), int(reps),
                                   cache_path.encode() if cache_path else None, _stream(stream),
                                   C.byref(best)), "surrogate_autotune")
    return best


def surrogate_graph_capture(s: Surrogate, mech: Mechanism, state, dt, trust, opts=None,
                            stream=None, n_cells=None) -> Graph:
    """One surrogate step with fallback on `state`, captured (``chem_graph``)."""
    ld = state.shape[1]
    n = ld if n_cells is None else int(n_cells)
    tr = (C.c_double * 4)(*[float(x) for x in trust])
    o = opts if opts is not None else make_opts()
    h = _P()
    _check(_lib.surrogate_graph_capture(s.handle, mech.handle, state.data_ptr(), ld, n, float(dt),
                                        tr, C.byref(o), _stream(stream), C.byref(h)),
           "surrogate_graph_capture")
    return Graph(mech, [state, s], handle=h)


def surrogate_save(s: Surrogate, path: str) -> None:
    _check(_lib.surrogate_save(s.handle, path.encode()), "surrogate_save")


def surrogate_load(mech: Mechanism, path: str) -> Surrogate:
    h = _P()
    _check(_lib.surrogate_load(mech.handle, path.encode(), C.byref(h)), "surrogate_load")
    return Surrogate(mech, handle=h)


def make_boxes(boxes):
    """boxes: list of dicts with keys state (CUDA float64 [N+3, ld]), dt,
    n_sub (default 1), level (default 0), status, counts (optional tensors),
    n_cells (default ld)."""
    arr = (chem_box * max(len(boxes), 1))()
    for i, b in enumerate(boxes):
        st = b["state"]
        ld = st.shape[1]
        arr[i] = chem_box(st.data_ptr(), ld, int(b.get("n_cells", ld)), float(b["dt"]),
                          int(b.get("n_sub", 1)), int(b.get("level", 0)),
                          _ptr(b.get("status")), _ptr(b.get("counts")))
    return arr


def chem_integrate_batched(mech: Mechanism, boxes, opts: chem_opts | None = None,
                           stream=None) -> None:
    arr = make_boxes(boxes)
    o = opts if opts is not None else make_opts()
    _reserve_for(mech, sum(int(arr[i].n_cells) for i in range(len(boxes))))
    _check(_lib.chem_integrate_batched(mech.handle, arr, len(boxes), C.byref(o),
                                       _stream(stream)), "chem_integrate_batched")


class Graph:
    """A captured batched call or surrogate step (``chem_graph``)."""

    def __init__(self, mech: Mechanism, boxes, opts: chem_opts | None = None, stream=None,
                 handle=None):
        if handle is not None:
            self.handle = handle
            self._keep = boxes
            return
        arr = make_boxes(boxes)
        o = opts if opts is not None else make_opts()
        h = _P()
        _check(_lib.chem_graph_capture_batched(mech.handle, arr, len(boxes), C.byref(o),
                                               _stream(stream), C.byref(h)),
               "chem_graph_capture_batched")
        self.handle = h
        self._keep = boxes

    def launch(self, stream=None):
        _check(_lib.chem_graph_launch(self.handle, _stream(stream)), "chem_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            _lib.chem_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chem_graph_capture_batched(mech, boxes, opts=None, stream=None) -> Graph:
    return Graph(mech, boxes, opts, stream)


def chem_autotune(mech: Mechanism, boxes, base: chem_opts | None = None, reps: int = 3,
                  cache_path: str | None = None, stream=None) -> chem_opts:
    arr = make_boxes(boxes)
    o = base if base is not None else make_opts()
    best = chem_opts()
    _reserve_for(mech, sum(int(arr[i].n_cells) for i in range(len(boxes))))
    _check(_lib.chem_autotune(mech.handle, arr, len(boxes), C.byref(o), int(reps),
                              cache_path.encode() if cache_path else None, _stream(stream),
                              C.byref(best)), "chem_autotune")
    return best


_lib.chem_react_conserved.argtypes = [_P, _P, C.c_int64, C.c_int64, C.c_double,
                                      C.POINTER(chem_opts), _P, _P, _P]


def chem_react_conserved(mech: Mechanism, cons, dt: float, opts: chem_opts | None = None,
                         status=None, counts=None, stream=None, n_cells: int | None = None):
    """Reaction step on conserved rows (rho, rho u, rho v, rho w, rho E,
    rho Y_1..rho Y_N, T, h) of a [N+7, ld] float64 device tensor, in place."""
    ld = cons.shape[1]
    n = ld if n_cells is None else int(n_cells)
    assert cons.dtype.itemsize == 8 and cons.is_contiguous() and cons.shape[0] == mech.n_species + 7
    if status is not None:
        assert status.numel() >= n and status.element_size() == 4
    if counts is not None:
        assert counts.numel() >= 2 * n and counts.element_size() == 4
    o = opts if opts is not None else make_opts()
    _reserve_for(mech, n)
    _check(_lib.chem_react_conserved(mech.handle, _ptr(cons), ld, n, float(dt), C.byref(o),
                                     _stream(stream), _ptr(status), _ptr(counts)),
           "chem_react_conserved")


_lib.chem_eval_exp.argtypes = [_P, _P, C.c_int64, _P]


def chem_eval_exp(x, stream=None):
    """e^x on the device with the exponential the rate evaluation uses."""
    import torch
    y = torch.empty_like(x)
    _check(_lib.chem_eval_exp(x.data_ptr(), y.data_ptr(), x.numel(), _stream(stream)),
           "chem_eval_exp")
    return y


_lib.chem_eval_math.restype = C.c_int
_lib.chem_eval_math.argtypes = [C.c_int32, _P, _P, C.c_int64, _P]
MATH_FNS = {"exp_cw": 0, "log_atanh": 2, "exp_tab": 3}


def chem_eval_math(fn, x, stream=None):
    """fn(x) on the device with one of the integrators' own elementary
    functions ("exp_cw", "log_atanh", "exp_tab")."""
    import torch
    y = torch.empty_like(x)
    _check(_lib.chem_eval_math(MATH_FNS[fn], x.data_ptr(), y.data_ptr(), x.numel(),
                               _stream(stream)), "chem_eval_math")
    return y


def exported_symbols():
    """Names declared in include/chemgpu.h that this library must export."""
    return ["chem_mech_load", "chem_mech_query", "chem_mech_free", "chem_workspace_reserve",
            "chem_integrate", "chem_integrate_batched", "chem_graph_capture_batched",
            "chem_graph_launch", "chem_graph_destroy", "chem_autotune", "chem_strerror",
            "chem_last_error", "surrogate_create", "surrogate_query", "surrogate_get_params",
            "surrogate_set_params", "surrogate_make_pairs", "surrogate_train", "surrogate_forward",
            "surrogate_grad", "surrogate_infer", "surrogate_save", "surrogate_load",
            "surrogate_free", "chem_eval_exp", "chem_eval_math", "chem_react_conserved",
            "chem_set_kernel_timing", "chem_kernel_times", "surrogate_reserve",
            "chem_integrate_noalloc", "chem_tail_stats", "surrogate_autotune",
            "surrogate_graph_capture"]
