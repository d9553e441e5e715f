"""ctypes binding of ``libbbe.so`` (C ABI in ``include/bbe.h``).

Argument marshalling only: every step of the race model runs in the HIP
kernels of the library.  PyTorch supplies device memory (CUDA tensors) and
the stream (``torch.cuda.current_stream()``).  There is no fallback: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbe.so")

OK, EINVAL, ENOMEM, EDEVICE = 0, -1, -2, -3
MAX_COMPETITORS = 20
UNRANKED = 0xFF
TICK_LIMIT = 1 << 20


class BBEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Competitor(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float), ("hi", ctypes.c_float), ("pref", ctypes.c_float),
                ("rho", ctypes.c_float), ("theta", ctypes.c_float)]


class State(ctypes.Structure):
    _fields_ = [("tick", ctypes.c_uint32), ("pos", ctypes.c_void_p),
                ("prev_step", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("race", ctypes.c_void_p), ("state", ctypes.POINTER(State)),
                ("sim_begin", ctypes.c_uint32), ("n_sims", ctypes.c_uint32),
                ("request", ctypes.c_uint32), ("stop_after", ctypes.c_int)]


PLAN_AUTOTUNE = 1


_lib = None

# (name, restype, argtypes) of every exported function declared in include/*.h
_P, _I, _U32, _U64, _F = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
SIGNATURES = {
    "bbe_race_init": (_I, [_P, _I, _F, _P]),
    "bbe_race_free": (None, [_P]),
    "bbe_race_n": (_I, [_P]),
    "bbe_race_set_pace": (_I, [_P, _P, _P]),
    "bbe_pref_from_factors": (_I, [_P, _I, _P, _P, _I, _P]),
    "bbe_race_sim": (_I, [_P, _P, _U32, _U32, _U64, _U32, _I, _P, _P, _P, _P]),
    "bbe_win_probs": (_I, [_P, _I, _I, _I, _P, _P]),
    "bbe_race_prefix": (_I, [_P, _P, _U64, _U32, _U32, _F, _P, _P, _P, _P]),
    "bbe_rank_counts": (_I, [_P, _U32, _I, _P, _P]),
    "bbe_order_pmf": (_I, [_P, _U32, _I, _P, _P]),
    "bbe_batch_plan_create": (_I, [_P, _I, _U64, _P, _P, _P, ctypes.c_uint, _P, _P]),
    "bbe_batch_plan_launch": (_I, [_P, _P]),
    "bbe_batch_plan_set_states": (_I, [_P, _P, _P]),
    "bbe_batch_plan_info": (_I, [_P, _P, _P, _P, _P]),
    "bbe_batch_plan_free": (None, [_P]),
    "bbe_prefix_batch": (_I, [_P, _P, _P, _I, _U64, _P, _P, _P, _P]),
    "bbe_prefix_batch_noalloc": (_I, [_P, _P, _P, _I, _U64, _P, _P, _P, _P]),
    "bbe_mlp_create": (_I, [_P, _I, _P]),
    "bbe_mlp_free": (None, [_P]),
    "bbe_mlp_get_params": (_I, [_P, _P]),
    "bbe_mlp_save": (_I, [_P, ctypes.c_char_p]),
    "bbe_mlp_save_checkpoint": (_I, [_P, ctypes.c_char_p]),
    "bbe_mlp_load": (_I, [ctypes.c_char_p, _I, _P]),
    "bbe_mlp_forward": (_I, [_P, _P, _P, _I, _P, _P, _P, _P]),
    "bbe_mlp_forward_hidden": (_I, [_P, _P, _P, _I, _P, _P, _P]),
    "bbe_mlp_loss_grad": (_I, [_P, _P, _P, _P, _I, _P, _P, _P]),
    "bbe_mlp_adam_step": (_I, [_P, _P, _F, _P]),
    "bbe_mlp_train_step": (_I, [_P, _P, _P, _P, _I, _F, _P, _P]),
    "bbe_encode_states": (_I, [_P, _P, _P, _P, _I, _F, _F, _P, _P, _P, _P, _P]),
    "bbe_race_advance": (_I, [_P, _P, _U64, _U32, _U32, _U32, _P, _P, _P, _P]),
    "bbe_race_trace": (_I, [_P, _P, _U64, _U32, _U32, _U32, _P, _P, _P]),
    "bbe_bettors_create": (_I, [_P, _P, _I, _P]),
    "bbe_bettors_free": (None, [_P]),
    "bbe_bettors_count": (_I, [_P, _P]),
    "bbe_bettor_views": (_I, [_P, _P, _U32, _I, _F, _U32, _U32, _U32, _U64, _P, _P, _P]),
    "bbe_rp_views": (_I, [_P, _I, _I, _I, _P, _P, _P]),
    "bbe_last_error": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BBEError(EDEVICE, f"{LIB_PATH} not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise BBEError(rc, lib().bbe_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Race:
    """A validated race: n competitors (rows lo, hi, pref, rho, theta, and
    optionally the time term gamma, tau of the responsiveness) on a track of
    length ``track_len``."""

    def __init__(self, comp, track_len: float):
        comp = np.asarray(comp, dtype=np.float32)
        if comp.ndim != 2 or comp.shape[1] not in (5, 7):
            raise BBEError(EINVAL, "comp must be [n, 5] or [n, 7]")
        self.n = int(comp.shape[0])
        self.comp = np.ascontiguousarray(comp[:, :5])
        self.pace = (np.ascontiguousarray(comp[:, 5]), np.ascontiguousarray(comp[:, 6])) \
            if comp.shape[1] == 7 else None
        self.track_len = float(track_len)
        # rows of 5 float32 are bbe_competitor structs
        h = ctypes.c_void_p()
        _check(lib().bbe_race_init(self.comp.ctypes.data if self.n else None, self.n,
                                   self.track_len, ctypes.byref(h)))
        self._h = h
        if self.pace is not None:
            _check(lib().bbe_race_set_pace(h, self.pace[0].ctypes.data, self.pace[1].ctypes.data))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bbe_race_free(h)
            self._h = None


def _state_struct(state, n):
    """(tick, pos, prev) host arrays -> (State, keepalive)."""
    if state is None:
        return None, None
    t, pos, prev = state
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    prev = np.ascontiguousarray(prev, dtype=np.float32)
    if pos.shape != (n,) or prev.shape != (n,):
        raise BBEError(EINVAL, "state arrays must have n entries")
    st = State(int(t), pos.ctypes.data, prev.ctypes.data)
    return st, (pos, prev)


def race_sim(race: Race, n_sims: int, seed: int, request: int = 0, state=None,
             sim_begin: int = 0, stop_after: int | None = None, orders=None, wins=None,
             steps=None, stream=None):
    """Enqueue ``bbe_race_sim``.  ``orders`` (uint8 [n_sims, n]), ``wins``
    (int64 [n]) and ``steps`` (int64 [1]) are CUDA tensors or None."""
    st, keep = _state_struct(state, race.n)
    stop_after = race.n if stop_after is None else int(stop_after)
    _check(lib().bbe_race_sim(race.handle, ctypes.byref(st) if st is not None else None,
                              sim_begin, n_sims, seed, request, stop_after, _dptr(orders),
                              _dptr(wins), _dptr(steps), _stream(stream)))
    del keep


def win_probs(wins, probs, n: int | None = None, stream=None):
    """Enqueue ``bbe_win_probs`` over a 1-D or 2-D int64 CUDA tensor."""
    w2 = wins.reshape(1, -1) if wins.dim() == 1 else wins
    rows, stride = w2.shape
    n = stride if n is None else n
    _check(lib().bbe_win_probs(_dptr(w2), rows, n, stride, _dptr(probs), _stream(stream)))


ORDER_PMF_MAX_N = 7


def rank_counts(orders, n: int, counts, stream=None):
    """Enqueue ``bbe_rank_counts``: orders uint8 CUDA tensor [n_sims, n],
    counts int64 CUDA tensor [n, n] (overwritten)."""
    n_sims = int(orders.shape[0]) if orders is not None else 0
    _check(lib().bbe_rank_counts(_dptr(orders), n_sims, n, _dptr(counts), _stream(stream)))


def order_pmf(orders, n: int, counts, stream=None):
    """Enqueue ``bbe_order_pmf``: orders uint8 CUDA tensor [n_sims, n],
    counts int64 CUDA tensor [n!] (overwritten)."""
    n_sims = int(orders.shape[0]) if orders is not None else 0
    _check(lib().bbe_order_pmf(_dptr(orders), n_sims, n, _dptr(counts), _stream(stream)))


def race_prefix(race: Race, seed: int, request: int, sim: int, target: float, tick_out,
                pos_out, prev_out, state=None, stream=None):
    st, keep = _state_struct(state, race.n)
    _check(lib().bbe_race_prefix(race.handle, ctypes.byref(st) if st is not None else None, seed,
                                 request, sim, float(target), _dptr(tick_out), _dptr(pos_out),
                                 _dptr(prev_out), _stream(stream)))
    del keep


def _request_array(specs):
    """specs: sequence of (race, state or None, sim_begin, n_sims, request,
    stop_after) -> (ctypes array, keepalive)."""
    keep = []
    arr = (Request * len(specs))()
    for i, (race, state, sim_begin, n_sims, request, stop_after) in enumerate(specs):
        st, k = _state_struct(state, race.n)
        keep.append((st, k, race))
        arr[i].race = race.handle
        arr[i].state = ctypes.pointer(st) if st is not None else None
        arr[i].sim_begin = int(sim_begin)
        arr[i].n_sims = int(n_sims)
        arr[i].request = int(request) & 0xFFFFFFFF
        arr[i].stop_after = int(stop_after or 0)
    return arr, keep


_STATE_DT = np.dtype([("tick", "<u4"), ("pad", "<u4"), ("pos", "<u8"), ("prev", "<u8")])
_REQ_DT = np.dtype([("race", "<u8"), ("state", "<u8"), ("sim_begin", "<u4"), ("n_sims", "<u4"),
                    ("request", "<u4"), ("stop_after", "<i4")])
assert _STATE_DT.itemsize == ctypes.sizeof(State)
assert _REQ_DT.itemsize == ctypes.sizeof(Request)


class RequestTable:
    """Many requests as one packed bbe_request array, built with numpy (no
    per-request Python objects).  ``races``: one Race per request;
    ``n_sims``, ``requests``, ``stop_after``, ``sim_begin``: scalars or
    per-request arrays; in-play states as ``tick`` uint32 [B] and ``pos`` /
    ``prev`` float32 [B, m] with m >= every race's n (row r's first n
    entries are request r's state), or all three None (start of race)."""

    def __init__(self, races, n_sims, requests, stop_after=0, sim_begin=0, tick=None, pos=None,
                 prev=None):
        B = len(races)
        self.races = list(races)
        self.req = np.zeros(B, _REQ_DT)
        self.req["race"] = np.fromiter((r.handle.value for r in self.races), np.uint64, B)
        self.req["sim_begin"] = sim_begin
        self.req["n_sims"] = n_sims
        self.req["request"] = np.asarray(requests, np.int64) & 0xFFFFFFFF
        self.req["stop_after"] = stop_after
        self.st = self.pos = self.prev = None
        if tick is not None:
            self.pos = np.ascontiguousarray(pos, dtype=np.float32)
            self.prev = np.ascontiguousarray(prev, dtype=np.float32)
            nmax = max((r.n for r in self.races), default=0)
            if self.pos.shape != self.prev.shape or self.pos.ndim != 2 or \
                    self.pos.shape[0] != B or self.pos.shape[1] < nmax:
                raise BBEError(EINVAL, "pos/prev must be [n_requests, >= n] arrays")
            self.st = np.zeros(B, _STATE_DT)
            self.st["tick"] = np.asarray(tick, np.uint32)
            rows = np.arange(B, dtype=np.uint64)
            self.st["pos"] = np.uint64(self.pos.ctypes.data) + rows * np.uint64(self.pos.strides[0])
            self.st["prev"] = np.uint64(self.prev.ctypes.data) + \
                rows * np.uint64(self.prev.strides[0])
            self.req["state"] = np.uint64(self.st.ctypes.data) + \
                rows * np.uint64(_STATE_DT.itemsize)

    def __len__(self):
        return len(self.req)

    @property
    def ptr(self):
        return self.req.ctypes.data


def _requests(specs):
    """(pointer, count, keepalive) for a RequestTable or a list of specs."""
    if isinstance(specs, RequestTable):
        return specs.ptr, len(specs), specs
    arr, keep = _request_array(specs)
    return arr, len(specs), keep


class BatchPlan:
    """A plan over uneven requests (``bbe_batch_plan_*``).  Outputs are CUDA
    tensors bound at creation: ``wins`` int64 [n_reqs, 20], optional
    ``probs`` float64 [n_reqs, 20] and ``steps`` int64 [1]."""

    def __init__(self, specs, seed: int, wins, probs=None, steps=None, autotune=True,
                 stream=None):
        arr, n_reqs, keep = _requests(specs)
        h = ctypes.c_void_p()
        self.n_reqs = n_reqs
        self._outs = (wins, probs, steps)
        _check(lib().bbe_batch_plan_create(arr, n_reqs, seed, _dptr(wins), _dptr(probs),
                                           _dptr(steps), PLAN_AUTOTUNE if autotune else 0,
                                           _stream(stream), ctypes.byref(h)))
        del keep
        self._h = h

    def launch(self, stream=None):
        _check(lib().bbe_batch_plan_launch(self._h, _stream(stream)))

    def set_states(self, tick, pos, prev, stream=None):
        """``bbe_batch_plan_set_states``: new start states for every request,
        tick uint32 [B] and pos / prev float32 [B, m] (m >= each race's n)."""
        pos = np.ascontiguousarray(pos, dtype=np.float32)
        prev = np.ascontiguousarray(prev, dtype=np.float32)
        tick = np.ascontiguousarray(tick, dtype=np.uint32)
        B = tick.shape[0]
        if B != self.n_reqs or pos.shape != prev.shape or pos.ndim != 2 or pos.shape[0] != B:
            raise BBEError(EINVAL, "tick [n_requests] and pos/prev [n_requests, m] arrays")
        st = np.zeros(B, _STATE_DT)
        rows = np.arange(B, dtype=np.uint64)
        st["tick"] = tick
        st["pos"] = np.uint64(pos.ctypes.data) + rows * np.uint64(pos.strides[0])
        st["prev"] = np.uint64(prev.ctypes.data) + rows * np.uint64(prev.strides[0])
        _check(lib().bbe_batch_plan_set_states(self._h, st.ctypes.data, _stream(stream)))

    def info(self):
        v = [ctypes.c_int() for _ in range(4)]
        _check(lib().bbe_batch_plan_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(waves_per_block=v[0].value, grid=v[1].value, sims_per_item=v[2].value,
                    n_items=v[3].value)

    def free(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bbe_batch_plan_free(h)
        self._h = None

    def __del__(self):
        self.free()


def prefix_batch(specs, sims, targets, seed, tick_out, pos_out, prev_out, stream=None):
    """Batched in-play states: specs (a list or a RequestTable) as for
    BatchPlan (n_sims etc. ignored)."""
    arr, n_reqs, keep = _requests(specs)
    sims = np.ascontiguousarray(sims, dtype=np.uint32)
    targets = np.ascontiguousarray(targets, dtype=np.float32)
    if sims.shape != (n_reqs,) or targets.shape != (n_reqs,):
        raise BBEError(EINVAL, "sims and targets need one entry per request")
    _check(lib().bbe_prefix_batch(arr, sims.ctypes.data, targets.ctypes.data, n_reqs, seed,
                                  _dptr(tick_out), _dptr(pos_out), _dptr(prev_out),
                                  _stream(stream)))
    del keep


PREFIX_NOALLOC_MAX = 4096


def prefix_batch_noalloc(specs, sims, targets, seed, tick_out, pos_out, prev_out, stream=None):
    """``bbe_prefix_batch_noalloc``: as prefix_batch, with the request
    descriptors in the library's fixed per-GPU workspace (at most
    PREFIX_NOALLOC_MAX requests; calls must not overlap on one GPU)."""
    arr, n_reqs, keep = _requests(specs)
    sims = np.ascontiguousarray(sims, dtype=np.uint32)
    targets = np.ascontiguousarray(targets, dtype=np.float32)
    if sims.shape != (n_reqs,) or targets.shape != (n_reqs,):
        raise BBEError(EINVAL, "sims and targets need one entry per request")
    _check(lib().bbe_prefix_batch_noalloc(arr, sims.ctypes.data, targets.ctypes.data, n_reqs,
                                          seed, _dptr(tick_out), _dptr(pos_out),
                                          _dptr(prev_out), _stream(stream)))
    del keep


MLP_NPARAMS = 177_940


class Mlp:
    """The surrogate network (``bbe_mlp_*``).  Tensors are CUDA tensors:
    x int16/uint16-bits [B, 160], n_valid int32 [B], target float32 [B, 20]."""

    def __init__(self, params, max_batch: int):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAMS,):
            raise BBEError(EINVAL, f"params must have {MLP_NPARAMS} values")
        h = ctypes.c_void_p()
        _check(lib().bbe_mlp_create(p.ctypes.data, int(max_batch), ctypes.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)

    def params(self) -> np.ndarray:
        out = np.empty(MLP_NPARAMS, dtype=np.float32)
        _check(lib().bbe_mlp_get_params(self._h, out.ctypes.data))
        return out

    def save(self, path: str):
        _check(lib().bbe_mlp_save(self._h, os.fsencode(path)))

    def save_checkpoint(self, path: str):
        """``bbe_mlp_save_checkpoint``: parameters, Adam moments and step
        count (``load`` resumes training from it exactly)."""
        _check(lib().bbe_mlp_save_checkpoint(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str, max_batch: int) -> "Mlp":
        h = ctypes.c_void_p()
        _check(lib().bbe_mlp_load(os.fsencode(path), int(max_batch), ctypes.byref(h)))
        m = cls.__new__(cls)
        m._h = h
        m.max_batch = int(max_batch)
        return m

    def forward(self, x, n_valid, probs=None, entropy=None, logits=None, stream=None):
        _check(lib().bbe_mlp_forward(self._h, _dptr(x), _dptr(n_valid), int(x.shape[0]),
                                     _dptr(probs), _dptr(entropy), _dptr(logits),
                                     _stream(stream)))

    def forward_hidden(self, x, n_valid, hidden, logits=None, stream=None):
        """``bbe_mlp_forward_hidden``: hidden int16/uint16-bits CUDA tensor
        [3, B, 256] receives h1, h2, h3."""
        if tuple(hidden.shape) != (3, int(x.shape[0]), 256):
            raise BBEError(EINVAL, "hidden must be [3, batch, 256]")
        _check(lib().bbe_mlp_forward_hidden(self._h, _dptr(x), _dptr(n_valid), int(x.shape[0]),
                                            _dptr(hidden), _dptr(logits), _stream(stream)))

    def loss_grad(self, x, n_valid, target, loss, grad=None, stream=None):
        _check(lib().bbe_mlp_loss_grad(self._h, _dptr(x), _dptr(n_valid), _dptr(target),
                                       int(x.shape[0]), _dptr(loss), _dptr(grad),
                                       _stream(stream)))

    def adam_step(self, lr: float, grad=None, stream=None):
        _check(lib().bbe_mlp_adam_step(self._h, _dptr(grad), float(lr), _stream(stream)))

    def train_step(self, x, n_valid, target, lr: float, loss, stream=None):
        _check(lib().bbe_mlp_train_step(self._h, _dptr(x), _dptr(n_valid), _dptr(target),
                                        int(x.shape[0]), float(lr), _dptr(loss), _stream(stream)))

    def free(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bbe_mlp_free(h)
        self._h = None

    def __del__(self):
        self.free()


def encode_states(comp, n, pos, prev, track_len: float, dt: float, x, slot=None, probs=None,
                  target=None, stream=None):
    """Enqueue ``bbe_encode_states`` on CUDA tensors."""
    _check(lib().bbe_encode_states(_dptr(comp), _dptr(n), _dptr(pos), _dptr(prev),
                                   int(n.shape[0]), float(track_len), float(dt), _dptr(x),
                                   _dptr(slot), _dptr(probs), _dptr(target), _stream(stream)))


def race_advance(race: Race, seed: int, request: int, sim: int, n_ticks: int, tick_out,
                 pos_out, prev_out, state=None, stream=None):
    st, keep = _state_struct(state, race.n)
    _check(lib().bbe_race_advance(race.handle, ctypes.byref(st) if st is not None else None,
                                  seed, request, sim, int(n_ticks), _dptr(tick_out),
                                  _dptr(pos_out), _dptr(prev_out), _stream(stream)))
    del keep


def race_trace(race: Race, seed: int, request: int, sim: int, max_rows: int, trace, n_rows,
               state=None, stream=None):
    """Enqueue ``bbe_race_trace``: trace float32 CUDA tensor [max_rows, n],
    n_rows int32 (uint32 bits) CUDA tensor [1]."""
    st, keep = _state_struct(state, race.n)
    _check(lib().bbe_race_trace(race.handle, ctypes.byref(st) if st is not None else None,
                                seed, request, sim, int(max_rows), _dptr(trace), _dptr(n_rows),
                                _stream(stream)))
    del keep


BETTOR_KINDS = {"ZI": 0, "LW": 1, "UD": 2, "LinEx": 3}


class Bettors:
    """A population of cheap in-play bettors (``bbe_bettors_*``): kinds uint8
    (``BETTOR_KINDS``) and parameters float32, host arrays."""

    def __init__(self, kinds, params):
        k = np.ascontiguousarray(kinds, dtype=np.uint8)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if k.ndim != 1 or p.shape != k.shape:
            raise BBEError(EINVAL, "kinds and params must be 1-D arrays of equal length")
        h = ctypes.c_void_p()
        _check(lib().bbe_bettors_create(k.ctypes.data, p.ctypes.data, int(k.shape[0]),
                                        ctypes.byref(h)))
        self._h = h
        self.n = int(k.shape[0])

    def per_kind(self) -> np.ndarray:
        out = np.zeros(4, dtype=np.uint32)
        _check(lib().bbe_bettors_count(self._h, out.ctypes.data))
        return out

    def views(self, trace, n_rows: int, track_len: float, t0: int, seed: int, first_row: int,
              n_eval: int, views=None, counts=None, stream=None):
        """Enqueue ``bbe_bettor_views``: trace float32 CUDA tensor [>= n_rows, n];
        views uint8 [n_eval, n_bettors] and/or counts int32 (uint32 bits)
        [n_eval, n] CUDA tensors."""
        _check(lib().bbe_bettor_views(self._h, _dptr(trace), int(n_rows), int(trace.shape[1]),
                                      float(track_len), int(t0), int(first_row), int(n_eval),
                                      seed, _dptr(views), _dptr(counts), _stream(stream)))

    def free(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bbe_bettors_free(h)
        self._h = None

    def __del__(self):
        self.free()


def rp_views(wins, n: int, views=None, counts=None, stream=None):
    """Enqueue ``bbe_rp_views``: wins int64 CUDA tensor [B, stride]; views
    uint8 [B] and/or counts int32 (uint32 bits) [n]."""
    _check(lib().bbe_rp_views(_dptr(wins), int(wins.shape[0]), int(n), int(wins.shape[1]),
                              _dptr(views), _dptr(counts), _stream(stream)))


def pref_from_factors(factors, prefs, sens) -> np.ndarray:
    """``bbe_pref_from_factors`` on host arrays: factors [F], prefs and sens
    [n, F]; returns P [n] (float32)."""
    f = np.ascontiguousarray(factors, dtype=np.float32)
    p = np.ascontiguousarray(prefs, dtype=np.float32)
    w = np.ascontiguousarray(sens, dtype=np.float32)
    if p.ndim != 2 or p.shape != w.shape or p.shape[1] != f.shape[0]:
        raise BBEError(EINVAL, "prefs and sens must be [n, F] with F = len(factors)")
    out = np.empty(p.shape[0], dtype=np.float32)
    _check(lib().bbe_pref_from_factors(f.ctypes.data, int(f.shape[0]), p.ctypes.data,
                                       w.ctypes.data, int(p.shape[0]), out.ctypes.data))
    return out
