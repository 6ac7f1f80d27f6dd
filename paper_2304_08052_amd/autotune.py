"""Launch-shape tuning through the library's handle: argument marshalling
only.  The search over candidate shapes (scatter and bin-moment renders),
the timing of each candidate's forward with HIP events, the size classes and
the JSON cache all live in the C library (framrir_handle_create,
framrir_tune, framrir_tune_lookup, framrir_size_class).

Caches: $FRAMRIR_TUNE_CACHE (else ~/.cache/framrir/tune.json) is the one
tuning writes; tune_cache.json beside this module (entries measured on
MI355X) is read after it.  Keys are "architecture|size class".
"""
import os

from . import framrir as fr

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

_HANDLES = {}


def cache_path():
    return os.environ.get("FRAMRIR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "framrir", "tune.json"))


def handle(writable=True):
    """The handle of the current device, with the writable cache first (or
    none: writable=False) and the shipped cache after it."""
    import torch
    dev = torch.cuda.current_device()
    path = cache_path() if writable else ""
    key = (dev, path)
    if key not in _HANDLES:
        if path:
            os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        _HANDLES[key] = fr.Handle(dev, (path, SHIPPED))
    return _HANDLES[key]


def size_class(batch):
    return fr.size_class(batch)


def tune(batch, candidates=None, reps=5, params=None, store=True, size_class=None):
    """framrir_tune on this batch: (best launch, median ms of its forward);
    candidates None = the library's search."""
    return handle(writable=store).tune(batch, candidates=candidates, reps=reps, params=params,
                                       size_class=size_class)


def launch_for(batch, tune_if_missing=False, params=None):
    """The cached launch of this batch's size class (or the default)."""
    launch, found = handle().lookup(fr.size_class(batch))
    if not found and tune_if_missing:
        return tune(batch, params=params)[0]
    return launch


def stream_class(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max):
    """Size class of a fixed-capacity graph step (stream.GraphStream): its
    launch shape serves every batch the capacity admits."""
    return f"stream:rooms={n_rooms};src<={n_src_max};mics<={n_mic_max};rt60<={rt60_max:g};fs<={fs_max:g}"


def launch_for_stream(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max):
    """The cached launch of a graph step of this capacity (or the default)."""
    return handle().lookup(stream_class(n_rooms, n_src_max, n_mic_max, rt60_max, fs_max))[0]
