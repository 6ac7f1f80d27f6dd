"""Python binding of libframrir.so (the C ABI in include/framrir.h).

Argument marshalling only: torch supplies device memory and streams, ctypes
passes raw pointers.  Every step of the method runs in the library's HIP
kernels; if the library is missing this module raises instead of falling back.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libframrir.so")

FRAMRIR_TAPS = 81
FRAMRIR_FLAG_MULTIRATE = 1
NOALLOC_SCRATCH_BYTES = 64 << 20      # FRAMRIR_NOALLOC_SCRATCH_BYTES


class FramrirError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__(f"framrir error {code}: {detail}")
        self.code = code


class Room(ctypes.Structure):
    _fields_ = [("size", ctypes.c_double * 3), ("rt60", ctypes.c_double), ("fs", ctypes.c_double),
                ("c", ctypes.c_double), ("r_override", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("n_src", ctypes.c_int32), ("n_mic", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("tau", ctypes.c_double), ("img_lo", ctypes.c_int32),
                ("img_hi", ctypes.c_int32), ("taps", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Launch(ctypes.Structure):
    _fields_ = [("lds_bytes", ctypes.c_int32), ("wg_threads", ctypes.c_int32), ("grid_wgs", ctypes.c_int32),
                ("max_mic_group", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("bwd_wg_threads", ctypes.c_int32), ("bwd_grid_wgs", ctypes.c_int32), ("render_path", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_rooms", ctypes.c_int32), ("n_src", ctypes.c_int32), ("n_mic", ctypes.c_int32),
                ("n_items", ctypes.c_int32), ("n_img", ctypes.c_int64), ("out_floats", ctypes.c_int64),
                ("desc_bytes", ctypes.c_int64), ("ws_bytes", ctypes.c_int64), ("ws_bwd_bytes", ctypes.c_int64),
                ("max_T", ctypes.c_int32), ("max_img", ctypes.c_int32), ("early_floats", ctypes.c_int64),
                ("n_chan", ctypes.c_int32), ("multirate", ctypes.c_int32), ("mr_floats", ctypes.c_int64),
                ("ws_mr_bytes", ctypes.c_int64), ("fir_blocks", ctypes.c_int64)]


DEFAULT_PARAMS = dict(alpha=0.25, beta=1.0, a=-2.0, b=2.0, tau=0.25, img_lo=1024, img_hi=4096)
DEFAULT_LAUNCH = dict(lds_bytes=131072, wg_threads=1024, grid_wgs=0, max_mic_group=8, waves_per_simd=4,
                      bwd_wg_threads=0, bwd_grid_wgs=0, render_path=0)
RENDER_SCATTER, RENDER_MOMENTS = 0, 1

EXPORTS = {
    "framrir_plan_create": (ctypes.c_int, [ctypes.POINTER(Room), ctypes.c_int32, ctypes.POINTER(Params),
                                           ctypes.POINTER(Launch), ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "framrir_plan_destroy": (None, [ctypes.c_void_p]),
    "framrir_plan_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "framrir_plan_get_arrays": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 7),
    "framrir_plan_desc": (ctypes.c_void_p, [ctypes.c_void_p]),
    "framrir_draw": (ctypes.c_int, [ctypes.c_void_p] * 6),
    "framrir_render": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_forward": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_forward_noalloc": (ctypes.c_int, [ctypes.c_void_p] * 8),
    "framrir_forward_early": (ctypes.c_int, [ctypes.c_void_p] * 10 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_prepare": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                               ctypes.c_void_p]),
    "framrir_render_prepared": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_render_backward": (ctypes.c_int, [ctypes.c_void_p] * 11 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_render_backward_prepared": (ctypes.c_int, [ctypes.c_void_p] * 9 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_render_backward_draws": (ctypes.c_int, [ctypes.c_void_p] * 10 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_render_backward_draws_prepared": (ctypes.c_int,
                                               [ctypes.c_void_p] * 8 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_workspace_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_plan_get_early": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "framrir_early": (ctypes.c_int, [ctypes.c_void_p] * 8),
    "framrir_forward_multirate": (ctypes.c_int, [ctypes.c_void_p] * 9 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_multirate_filter": (ctypes.c_int, [ctypes.c_void_p] * 5 + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_spatial_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "framrir_spatialize": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_int32] + [ctypes.c_void_p] * 4
                           + [ctypes.c_size_t, ctypes.c_void_p]),
    "framrir_philox4x32": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p]),
    "framrir_cbrt_rn": (ctypes.c_int, [ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_void_p]),
    "framrir_host_cbrt_rn": (ctypes.c_int, [ctypes.c_void_p] * 2 + [ctypes.c_int64]),
    "framrir_host_sqrt_rn": (ctypes.c_int, [ctypes.c_void_p] * 2 + [ctypes.c_int64]),
    "framrir_host_philox4x32": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int64]),
    "framrir_last_error_detail": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
    "framrir_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "framrir_version": (ctypes.c_int, []),
    "framrir_arch_supported": (ctypes.c_int, [ctypes.c_char_p]),
    "framrir_handle_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "framrir_handle_destroy": (None, [ctypes.c_void_p]),
    "framrir_size_class": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]),
    "framrir_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_double)]),
    "framrir_tune_lookup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def lib():
    """Loads libframrir.so (built in-tree).  torch is imported first so that
    the library binds to the HIP runtime torch already loaded."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2304_08052_amd.build")
        so = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(so, name)
            fn.restype = res
            fn.argtypes = args
        _lib = so
    return _lib


def _check(rc):
    if rc != 0:
        buf = ctypes.create_string_buffer(1024)
        lib().framrir_last_error_detail(buf, 1024)
        raise FramrirError(rc, buf.value.decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def room_structs(batch):
    """The batch as the C ABI takes it: (framrir_room array, n_rooms, src
    [sum n_src, 3] FP64, mic [sum n_mic, 3] FP64), contiguous host arrays."""
    n = len(batch["rt60"])
    rooms = (Room * n)()
    for b in range(n):
        rm = rooms[b]
        for k in range(3):
            rm.size[k] = float(batch["size"][b][k])
        rm.rt60 = float(batch["rt60"][b])
        rm.fs = float(batch["fs"][b])
        rm.c = float(batch["c"][b])
        rm.r_override = float(batch["r_override"][b])
        rm.seed = int(batch["seed"][b])
        rm.n_src = int(batch["n_src"][b])
        rm.n_mic = int(batch["n_mic"][b])
    src = np.ascontiguousarray(batch["src"], dtype=np.float64)
    mic = np.ascontiguousarray(batch["mic"], dtype=np.float64)
    return rooms, n, src, mic


def params_struct(params=None, multirate=False):
    prm = dict(DEFAULT_PARAMS, **(params or {}))
    return prm, Params(prm["alpha"], prm["beta"], prm["a"], prm["b"], prm["tau"], prm["img_lo"], prm["img_hi"],
                       FRAMRIR_TAPS, FRAMRIR_FLAG_MULTIRATE if multirate else 0)


LAUNCH_FIELDS = ("lds_bytes", "wg_threads", "grid_wgs", "max_mic_group", "waves_per_simd", "bwd_wg_threads",
                 "bwd_grid_wgs", "render_path")


def launch_struct(launch=None):
    lau = dict(DEFAULT_LAUNCH, **(launch or {}))
    return lau, Launch(*(int(lau[k]) for k in LAUNCH_FIELDS))


def launch_dict(la):
    return {k: int(getattr(la, k)) for k in LAUNCH_FIELDS}


def arch_supported(gcn_arch_name):
    """framrir_arch_supported: does a device of this gcnArchName run the library."""
    return bool(lib().framrir_arch_supported(gcn_arch_name.encode()))


def size_class(batch):
    """framrir_size_class: the tuning-cache key of a batch."""
    rooms, n, _, _ = room_structs(batch)
    buf = ctypes.create_string_buffer(256)
    _check(lib().framrir_size_class(rooms, n, buf, 256))
    return buf.value.decode()


class Handle:
    """framrir_handle of one device: architecture check, the allocation-free
    entry point's scratch, and the tuning caches (paths: the writable cache
    first, then read-only fallbacks)."""

    def __init__(self, device=0, cache_paths=()):
        h = ctypes.c_void_p()
        _check(lib().framrir_handle_create(int(device), ":".join(cache_paths).encode(), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.framrir_handle_destroy(h)
            self._h = None

    def tune(self, batch, candidates=None, reps=5, params=None, size_class=None):
        """framrir_tune: (best launch dict, median ms of its forward)."""
        rooms, n, src, mic = room_structs(batch)
        _, p = params_struct(params)
        cands = None
        if candidates:
            cands = (Launch * len(candidates))(*(launch_struct(c)[1] for c in candidates))
        best = Launch()
        ms = ctypes.c_double()
        _check(lib().framrir_tune(self._h, rooms, n, ctypes.byref(p), _np_ptr(src), _np_ptr(mic),
                                  size_class.encode() if size_class else None, cands,
                                  len(candidates) if candidates else 0, int(reps), ctypes.byref(best),
                                  ctypes.byref(ms)))
        return launch_dict(best), float(ms.value)

    def lookup(self, size_class):
        """framrir_tune_lookup: (launch dict, found)."""
        out = Launch()
        found = ctypes.c_int32()
        _check(lib().framrir_tune_lookup(self._h, size_class.encode(), ctypes.byref(out), ctypes.byref(found)))
        return launch_dict(out), bool(found.value)


class Plan:
    """Host plan of a batch plus its descriptor blob on the device.

    batch: dict with size (B,3), rt60, fs, c, r_override, seed, n_src, n_mic,
    src (sum n_src, 3), mic (sum n_mic, 3) -- see workloads.py."""

    def __init__(self, batch, params=None, launch=None, device="cuda", multirate=False):
        """device="cpu" plans and keeps the blob in host memory (no GPU calls).
        multirate=True plans the paper-literal multi-rate rendering
        (forward_multirate only)."""
        import torch
        L = lib()
        rooms, n, self.src, self.mic = room_structs(batch)
        prm, p = params_struct(params, multirate)
        lau, la = launch_struct(launch)
        handle = ctypes.c_void_p()
        _check(L.framrir_plan_create(rooms, n, ctypes.byref(p), ctypes.byref(la), _np_ptr(self.src),
                                     _np_ptr(self.mic), ctypes.byref(handle)))
        self._h = handle
        self.params = prm
        self.launch = lau
        info = PlanInfo()
        _check(L.framrir_plan_get_info(self._h, ctypes.byref(info)))
        self.info = info
        self.n_rooms = info.n_rooms
        self.T = np.zeros(n, dtype=np.int32)
        self.out_off = np.zeros(n + 1, dtype=np.int64)
        self.r = np.zeros(n, dtype=np.float64)
        self.n_img = np.zeros(info.n_src, dtype=np.int32)
        self.img_off = np.zeros(info.n_src + 1, dtype=np.int64)
        self.rrmax = np.zeros(info.n_src, dtype=np.float64)
        self.d0 = np.zeros(info.n_src, dtype=np.float64)
        _check(L.framrir_plan_get_arrays(self._h, _np_ptr(self.T), _np_ptr(self.out_off), _np_ptr(self.r),
                                         _np_ptr(self.n_img), _np_ptr(self.img_off), _np_ptr(self.rrmax),
                                         _np_ptr(self.d0)))
        self.early_off = np.zeros(n + 1, dtype=np.int64)
        self.early_width = np.zeros(n, dtype=np.int32)
        self.chan_off = np.zeros(n + 1, dtype=np.int32)
        _check(L.framrir_plan_get_early(self._h, _np_ptr(self.early_off), _np_ptr(self.early_width),
                                        _np_ptr(self.chan_off)))
        self.n_src = np.asarray(batch["n_src"], dtype=np.int64)
        self.n_mic = np.asarray(batch["n_mic"], dtype=np.int64)
        self.src_off = np.concatenate([[0], np.cumsum(self.n_src)])
        self.mic_off = np.concatenate([[0], np.cumsum(self.n_mic)])
        blob = ctypes.string_at(L.framrir_plan_desc(self._h), info.desc_bytes)
        self.device = torch.device(device)
        self.desc = torch.from_numpy(np.frombuffer(blob, dtype=np.uint8).copy()).to(self.device)
        self.src_dev = torch.from_numpy(self.src).to(self.device)
        self.mic_dev = torch.from_numpy(self.mic).to(self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.framrir_plan_destroy(h)
            self._h = None

    # ---- buffers -----------------------------------------------------------
    def empty_table(self):
        import torch
        return torch.empty((self.info.n_img, 4), dtype=torch.float64, device=self.device)

    def empty_out(self):
        import torch
        return torch.empty(self.info.out_floats, dtype=torch.float32, device=self.device)

    def workspace(self, backward=False):
        """Render (or backward) workspace, initialised for its first call."""
        import torch
        n = self.info.ws_bwd_bytes if backward else self.info.ws_bytes
        return torch.zeros(n, dtype=torch.uint8, device=self.device)

    def _ck(self, t, kind):
        """Device pointer of t for the C ABI after checking what the call reads
        or writes through it: dtype, contiguity, at least the plan's element
        count for that argument, and that it lives on a GPU (a wrong dtype
        would otherwise be read with the wrong element size)."""
        if t is None:
            return None
        import torch
        i = self.info
        dtype, numel = {
            "desc": (torch.uint8, None), "ws": (torch.uint8, None),
            "table": (torch.float64, 4 * i.n_img), "aux": (torch.float64, 8 * i.n_img),
            "words": (torch.int32, 4 * i.n_img),
            "mic": (torch.float64, 3 * i.n_mic), "src": (torch.float64, 3 * i.n_src), "r": (torch.float64, i.n_rooms),
            "out": (torch.float32, i.out_floats), "gm": (torch.float32, 3 * i.n_mic),
            "gs": (torch.float32, 3 * i.n_src),
            "gr": (torch.float32, i.n_rooms), "inter": (torch.float32, i.mr_floats),
            "early": (torch.float32, i.early_floats), "start": (torch.int32, i.n_chan)}[kind]
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{kind}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype != dtype:
            raise TypeError(f"{kind}: dtype {t.dtype}, the library reads {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{kind}: tensor is not contiguous")
        if numel is not None and t.numel() < numel:
            raise ValueError(f"{kind}: {t.numel()} elements, the plan needs {numel}")
        if t.device.type != "cuda":
            raise ValueError(f"{kind}: tensor on {t.device}, the library takes device memory")
        return ctypes.c_void_p(t.data_ptr())

    # ---- device calls ------------------------------------------------------
    # Every device call takes an optional desc: a device copy of another
    # plan's descriptor blob launched with this plan's shapes (see stream.py).
    def draw(self, table=None, aux=False, words=False, stream=None, desc=None):
        import torch
        table = self.empty_table() if table is None else table
        aux_t = torch.empty((self.info.n_img, 8), dtype=torch.float64, device=self.device) if aux else None
        w_t = torch.empty((self.info.n_img, 4), dtype=torch.int32, device=self.device) if words else None
        desc = self.desc if desc is None else desc
        _check(lib().framrir_draw(self._h, self._ck(desc, "desc"), self._ck(table, "table"), self._ck(aux_t, "aux"),
                                  self._ck(w_t, "words"), _stream(stream)))
        return table, aux_t, w_t

    def render(self, table, mic=None, src=None, r=None, out=None, ws=None, stream=None, desc=None):
        out = self.empty_out() if out is None else out
        ws = self.workspace() if ws is None else ws
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_render(self._h, self._ck(desc, "desc"), self._ck(table, "table"), self._ck(mic, "mic"),
                                    self._ck(src, "src"), self._ck(r, "r"), self._ck(out, "out"), self._ck(ws, "ws"),
                                    ws.numel(), _stream(stream)))
        return out

    def forward(self, table=None, mic=None, src=None, r=None, out=None, ws=None, stream=None, desc=None):
        """framrir_forward; table=False draws without exporting the table
        (returned as None)."""
        table = self.empty_table() if table is None else (None if table is False else table)
        out = self.empty_out() if out is None else out
        ws = self.workspace() if ws is None else ws
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_forward(self._h, self._ck(desc, "desc"), self._ck(table, "table"), self._ck(mic, "mic"),
                                     self._ck(src, "src"), self._ck(r, "r"), self._ck(out, "out"), self._ck(ws, "ws"),
                                     ws.numel(), _stream(stream)))
        return out, table

    def forward_early(self, table=None, mic=None, src=None, r=None, out=None, early=None, start=None, ws=None,
                      stream=None, desc=None):
        """framrir_forward_early: the forward and the Eq. 9 windows from the
        same pass; returns (out, table, early, start) (table=False: no table)."""
        import torch
        table = self.empty_table() if table is None else (None if table is False else table)
        out = self.empty_out() if out is None else out
        early = torch.empty(self.info.early_floats, dtype=torch.float32, device=self.device) if early is None \
            else early
        start = torch.empty(self.info.n_chan, dtype=torch.int32, device=self.device) if start is None else start
        ws = self.workspace() if ws is None else ws
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_forward_early(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                           self._ck(mic, "mic"), self._ck(src, "src"), self._ck(r, "r"),
                                           self._ck(out, "out"), self._ck(early, "early"), self._ck(start, "start"),
                                           self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        return out, table, early, start

    def forward_noalloc(self, table, out, mic=None, src=None, r=None, stream=None, desc=None):
        """framrir_forward_noalloc: the forward with the library's static
        device scratch as its workspace (no allocation in the call; the
        caller passes the table, or None, and the output)."""
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_forward_noalloc(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                             self._ck(mic, "mic"), self._ck(src, "src"), self._ck(r, "r"),
                                             self._ck(out, "out"), _stream(stream)))
        return out, table

    def prepare(self, table, mic=None, src=None, r=None, ws=None, draw=False, stream=None, desc=None):
        """framrir_prepare: per-source scales and row order (and the draws when draw=True)."""
        ws = self.workspace() if ws is None else ws
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_prepare(self._h, self._ck(desc, "desc"), self._ck(table, "table"), self._ck(mic, "mic"),
                                     self._ck(src, "src"), self._ck(r, "r"), int(draw), self._ck(ws, "ws"), ws.numel(),
                                     _stream(stream)))
        return ws

    def render_prepared(self, table, mic=None, src=None, r=None, out=None, ws=None, stream=None, desc=None):
        """framrir_render_prepared: the render kernel alone (after prepare)."""
        out = self.empty_out() if out is None else out
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_render_prepared(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                             self._ck(mic, "mic"), self._ck(src, "src"), self._ck(r, "r"),
                                             self._ck(out, "out"), self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        return out

    def backward(self, table, grad_out, mic=None, src=None, r=None, ws=None, grads=None, stream=None, desc=None,
                 prepared=False):
        """framrir_render_backward; with prepared=True framrir_render_backward_prepared,
        reusing the preparation a forward / render / prepare call left in ws
        (a backward-size workspace), and table / src are not read."""
        import torch
        if prepared and ws is None:
            raise ValueError("prepared=True needs the workspace the forward ran on")
        ws = self.workspace(backward=True) if ws is None else ws
        desc = self.desc if desc is None else desc
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        if grads is None:
            grads = (torch.empty((self.info.n_mic, 3), dtype=torch.float32, device=self.device),
                     torch.empty((self.info.n_src, 3), dtype=torch.float32, device=self.device),
                     torch.empty(self.info.n_rooms, dtype=torch.float32, device=self.device))
        gm, gs, gr = grads
        if prepared:
            _check(lib().framrir_render_backward_prepared(self._h, self._ck(desc, "desc"), self._ck(mic, "mic"),
                                                          self._ck(r, "r"), self._ck(grad_out, "out"),
                                                          self._ck(gm, "gm"), self._ck(gs, "gs"), self._ck(gr, "gr"),
                                                          self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        else:
            _check(lib().framrir_render_backward(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                                 self._ck(mic, "mic"), self._ck(src, "src"), self._ck(r, "r"),
                                                 self._ck(grad_out, "out"), self._ck(gm, "gm"), self._ck(gs, "gs"),
                                                 self._ck(gr, "gr"), self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        return gm, gs, gr

    def backward_draws(self, table, grad_out, ws=None, grads=None, stream=None, desc=None, prepared=False):
        """framrir_render_backward_draws (prepared=True: ..._draws_prepared,
        reusing the preparation of a forward with r = None in ws): the gradient
        with the images moving with the plan's positions and r."""
        import torch
        if prepared and ws is None:
            raise ValueError("prepared=True needs the workspace the forward ran on")
        ws = self.workspace(backward=True) if ws is None else ws
        desc = self.desc if desc is None else desc
        if grads is None:
            grads = (torch.empty((self.info.n_mic, 3), dtype=torch.float32, device=self.device),
                     torch.empty((self.info.n_src, 3), dtype=torch.float32, device=self.device),
                     torch.empty(self.info.n_rooms, dtype=torch.float32, device=self.device))
        gm, gs, gr = grads
        if prepared:
            _check(lib().framrir_render_backward_draws_prepared(self._h, self._ck(desc, "desc"), _ptr(self.mic_dev),
                                                                self._ck(grad_out, "out"), self._ck(gm, "gm"),
                                                                self._ck(gs, "gs"), self._ck(gr, "gr"),
                                                                self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        else:
            _check(lib().framrir_render_backward_draws(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                                       _ptr(self.mic_dev), _ptr(self.src_dev),
                                                       self._ck(grad_out, "out"), self._ck(gm, "gm"),
                                                       self._ck(gs, "gs"), self._ck(gr, "gr"), self._ck(ws, "ws"),
                                                       ws.numel(), _stream(stream)))
        return gm, gs, gr

    def forward_multirate(self, table=None, mic=None, src=None, r=None, inter=None, out=None, ws=None,
                          stream=None, desc=None):
        """framrir_forward_multirate: draws, the render at r_l fs on the high-rate
        grid, the 80 Hz high-pass and the decimation to fs.  Returns
        (out [out_floats], table, inter [mr_floats]: the intermediate signal
        at r_l fs)."""
        import torch
        table = self.empty_table() if table is None else table
        out = self.empty_out() if out is None else out
        inter = torch.empty(self.info.mr_floats, dtype=torch.float32, device=self.device) if inter is None \
            else inter
        ws = torch.zeros(self.info.ws_mr_bytes, dtype=torch.uint8, device=self.device) if ws is None else ws
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_forward_multirate(self._h, self._ck(desc, "desc"), self._ck(table, "table"),
                                               self._ck(mic, "mic"), self._ck(src, "src"), self._ck(r, "r"),
                                               self._ck(inter, "inter"), self._ck(out, "out"), self._ck(ws, "ws"),
                                               ws.numel(), _stream(stream)))
        return out, table, inter

    def multirate_filter(self, inter, out=None, ws=None, stream=None, desc=None):
        """framrir_multirate_filter: high-pass and decimation of inter[:mr_floats]."""
        import torch
        out = self.empty_out() if out is None else out
        ws = torch.zeros(self.info.ws_mr_bytes, dtype=torch.uint8, device=self.device) if ws is None else ws
        desc = self.desc if desc is None else desc
        _check(lib().framrir_multirate_filter(self._h, self._ck(desc, "desc"), self._ck(inter, "inter"),
                                              self._ck(out, "out"), self._ck(ws, "ws"), ws.numel(), _stream(stream)))
        return out

    def spatial_workspace_bytes(self, n_samples):
        n = ctypes.c_size_t(0)
        _check(lib().framrir_spatial_workspace(self._h, int(n_samples), ctypes.byref(n)))
        return int(n.value)

    def spatialize(self, rir, sig, sir_db, snr_db, images=None, mix=None, gains=None, ws=None, stream=None,
                   desc=None):
        """framrir_spatialize: rooms of 3 sources (speakers 0, 1, noise 2); sig
        [n_src, N] FP32 dry signals, sir_db / snr_db [n_rooms] FP32; returns
        (images [n_chan, N], mix [n_mic, N], gains [n_src])."""
        import torch
        n = int(sig.shape[-1])
        assert sig.dtype == torch.float32 and sig.is_contiguous() and sig.numel() == self.info.n_src * n
        images = torch.empty((self.info.n_chan, n), dtype=torch.float32, device=self.device) if images is None \
            else images
        mix = torch.empty((self.info.n_mic, n), dtype=torch.float32, device=self.device) if mix is None else mix
        gains = torch.empty(self.info.n_src, dtype=torch.float32, device=self.device) if gains is None else gains
        if ws is None:
            ws = torch.empty(self.spatial_workspace_bytes(n), dtype=torch.uint8, device=self.device)
        desc = self.desc if desc is None else desc
        _check(lib().framrir_spatialize(self._h, _ptr(desc), _ptr(rir), _ptr(sig), _ptr(sir_db), _ptr(snr_db), n,
                                        _ptr(images), _ptr(mix), _ptr(gains), _ptr(ws), ws.numel(),
                                        _stream(stream)))
        return images, mix, gains

    def early(self, out, early=None, start=None, mic=None, src=None, stream=None, desc=None):
        """framrir_early: the Eq. 9 windows of rendered RIRs `out`; returns
        (early [early_floats] FP32, start [n_chan] int32)."""
        import torch
        early = torch.empty(self.info.early_floats, dtype=torch.float32, device=self.device) if early is None \
            else early
        start = torch.empty(self.info.n_chan, dtype=torch.int32, device=self.device) if start is None else start
        mic = self.mic_dev if mic is None else mic
        src = self.src_dev if src is None else src
        desc = self.desc if desc is None else desc
        _check(lib().framrir_early(self._h, self._ck(desc, "desc"), self._ck(mic, "mic"), self._ck(src, "src"),
                                   self._ck(out, "out"), self._ck(early, "early"), self._ck(start, "start"),
                                   _stream(stream)))
        return early, start

    def early_view(self, early, b):
        """[S_b, M_b, W_b] view of room b's early windows."""
        w = int(self.early_width[b])
        return early[self.early_off[b]:self.early_off[b + 1]].view(int(self.n_src[b]), int(self.n_mic[b]), w)

    # ---- views -------------------------------------------------------------
    def room_view(self, out, b):
        """[S_b, M_b, T_b] view of room b in the packed output."""
        s, m, t = int(self.n_src[b]), int(self.n_mic[b]), int(self.T[b])
        o = int(self.out_off[b])
        return out[o:o + s * m * t].view(s, m, t)

    def source_rows(self, table, s):
        """Image-table rows of global source s."""
        return table[int(self.img_off[s]):int(self.img_off[s + 1])]


def philox4x32(ctr, key, stream=None):
    """Device Philox4x32-10: ctr int32 [n,4], key int32 [n,2] (bit patterns)."""
    import torch
    out = torch.empty_like(ctr)
    _check(lib().framrir_philox4x32(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0], _stream(stream)))
    return out


def cbrt_rn(x, stream=None):
    """Device correctly rounded cube root of an FP64 tensor."""
    import torch
    y = torch.empty_like(x)
    _check(lib().framrir_cbrt_rn(_ptr(x), _ptr(y), x.numel(), _stream(stream)))
    return y


def host_cbrt_rn(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _check(lib().framrir_host_cbrt_rn(_np_ptr(x), _np_ptr(y), x.size))
    return y


def host_sqrt_rn(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _check(lib().framrir_host_sqrt_rn(_np_ptr(x), _np_ptr(y), x.size))
    return y


def host_philox4x32(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    _check(lib().framrir_host_philox4x32(_np_ptr(ctr), _np_ptr(key), _np_ptr(out), ctr.shape[0]))
    return out


def split_rooms(batch):
    """One single-room batch per room (same arrays, sliced)."""
    out = []
    so = mo = 0
    for b in range(len(batch["rt60"])):
        ns, nm = int(batch["n_src"][b]), int(batch["n_mic"][b])
        one = {k: batch[k][b:b + 1] for k in ("size", "rt60", "fs", "c", "r_override", "seed", "n_src", "n_mic")}
        one["src"] = batch["src"][so:so + ns]
        one["mic"] = batch["mic"][mo:mo + nm]
        out.append(one)
        so += ns
        mo += nm
    return out


class PerRoom:
    """The plain per-room launch path: one plan and one draw + render launch
    sequence per room, the rooms one after another on one stream, writing
    into slices of the same packed output as the batched path.  Same kernels;
    no cross-room persistence and no graph."""

    def __init__(self, batch, params=None, launch=None):
        self.plans = [Plan(one, params, launch) for one in split_rooms(batch)]
        self.tables = [p.empty_table() for p in self.plans]
        self.ws = [p.workspace() for p in self.plans]
        sizes = [p.info.out_floats for p in self.plans]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)])

    def forward(self, out, stream=None):
        for p, t, w, o0, o1 in zip(self.plans, self.tables, self.ws, self.offsets[:-1], self.offsets[1:]):
            p.forward(table=t, out=out[int(o0):int(o1)], ws=w, stream=stream)
        return out


def simulate(batch, params=None, launch=None):
    """Batched forward: returns (packed FP32 RIRs on the device, plan, table)."""
    plan = Plan(batch, params, launch)
    out, table = plan.forward()
    return out, plan, table


def _autograd():
    import torch

    class RenderFn(torch.autograd.Function):
        """Render with the image table held fixed; differentiable in the
        microphone positions, source positions and per-room r."""

        @staticmethod
        def forward(ctx, mic, src, r, plan, table):
            out = plan.render(table, mic=mic.contiguous(), src=src.contiguous(), r=r.contiguous())
            ctx.plan = plan
            ctx.table = table
            ctx.save_for_backward(mic, src, r)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            mic, src, r = ctx.saved_tensors
            gm, gs, gr = ctx.plan.backward(ctx.table, grad_out.contiguous().float(), mic=mic.contiguous(),
                                           src=src.contiguous(), r=r.contiguous())
            return gm.to(mic.dtype), gs.to(src.dtype), gr.to(r.dtype), None, None

    return RenderFn


_RENDER_FN = None


def render_differentiable(plan, table, mic, src, r):
    """Autograd entry: RIRs as a function of mic [n_mic,3], src [n_src,3]
    and r [n_rooms] (FP64 tensors), draws held fixed."""
    global _RENDER_FN
    if _RENDER_FN is None:
        _RENDER_FN = _autograd()
    return _RENDER_FN.apply(mic, src, r, plan, table)
