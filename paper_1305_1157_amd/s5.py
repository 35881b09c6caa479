"""Python binding of the S^5 C-ABI (``include/s5.h``): argument marshalling only.

Device memory and streams come from PyTorch; every step of the sort runs in the
HIP kernels of ``libs5.so``.  There is no fallback: if the library is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime that libs5.so must share)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libs5.so")

S5_OK, S5_ERR_INVALID, S5_ERR_NOMEM, S5_ERR_HIP, S5_ERR_DEVICE = 0, -1, -2, -3, -4
S5_ERR_TOO_LARGE = -5
STATIC_SCRATCH_BYTES = 64 << 20  # S5_STATIC_SCRATCH_BYTES
SPLIT_SAMPLED, SPLIT_LEARNED = 0, 1
CLASSIFY_UNROLL, CLASSIFY_EQUAL, CLASSIFY_JUMP = 0, 1, 2
ALPHABET_BYTES, ALPHABET_AUTO = 0, 1
DISTRIBUTE_ONE_PASS, DISTRIBUTE_TWO_PASS = 0, 1

EXPORTS = ("s5_sort", "s5_sort_ex", "s5_sort_static", "s5_workspace_bytes", "s5_sort_batched",
           "s5_classify_ex",
           "s5_sort_batched_tuned", "s5_stats_get",
           "s5_strerror", "s5_release", "s5_prefix_keys", "s5_classify", "s5_profile_enable",
           "s5_profile_only",
           "s5_profile_read", "s5_mlp_train", "s5_mlp_grad", "s5_mlp_eval", "s5_mlp_propose",
           "s5_debug_limit_capacity", "s5_debug_count_writes", "s5_debug_miss_publish")


class Config(ctypes.Structure):
    _fields_ = [("splitters", ctypes.c_uint32), ("oversample", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("base_threshold", ctypes.c_uint32), ("splitter_mode", ctypes.c_uint32),
                ("imbalance_bound", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("graph_levels", ctypes.c_uint32), ("classifier", ctypes.c_uint32),
                ("alphabet", ctypes.c_uint32), ("distribution", ctypes.c_uint32)]


class SetTuning(ctypes.Structure):
    """Per-set parameters of ``sort_batched(..., tuning=...)`` (0 = the config's value)."""
    _fields_ = [("splitters", ctypes.c_uint16), ("base_threshold", ctypes.c_uint16),
                ("tile", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("fallbacks", ctypes.c_uint32),
                ("moved_M", ctypes.c_uint64), ("max_bucket", ctypes.c_uint64),
                ("entropy_bits", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t),
                ("base_items", ctypes.c_uint64), ("segments", ctypes.c_uint64),
                ("char_bits", ctypes.c_uint32), ("alphabet_retries", ctypes.c_uint32),
                ("learned_proposals", ctypes.c_uint32), ("root_depth", ctypes.c_uint32),
                ("imbalance_mean", ctypes.c_double), ("imbalance_max", ctypes.c_double),
                ("moved_one_bucket", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelProfile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("items", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_double)]


class S5Error(RuntimeError):
    pass


_lib = None
_wlib = None
WCHECK_PATH = os.path.join(_PKG, "libs5_wcheck.so")


def load(path: str = LIB_PATH):
    """Load ``libs5.so`` (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        _lib = _open(path)
    return _lib


def load_wcheck():
    """The write-check build ``libs5_wcheck.so`` (every output write counted;
    tests only), with the same entry points."""
    global _wlib
    if _wlib is None:
        _wlib = _open(WCHECK_PATH)
    return _wlib


def _open(path: str):
    if not os.path.exists(path):
        raise S5Error(f"S^5 HIP library not built: {path} is missing "
                      "(run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    lib.s5_sort.argtypes = [P, P, U32, P, P, P]
    lib.s5_sort_ex.argtypes = [P, U64, P, U32, P, P, ctypes.POINTER(Config), P, ctypes.c_size_t, P]
    lib.s5_sort_static.argtypes = [P, U64, P, U32, P, P, ctypes.POINTER(Config), P]
    lib.s5_workspace_bytes.argtypes = [U32, ctypes.POINTER(Config)]
    lib.s5_workspace_bytes.restype = ctypes.c_size_t
    lib.s5_sort_batched.argtypes = [P, U64, P, P, U32, P, P, ctypes.POINTER(Config), P]
    lib.s5_sort_batched_tuned.argtypes = [P, U64, P, P, U32, ctypes.POINTER(SetTuning), P, P,
                                          ctypes.POINTER(Config), P]
    lib.s5_stats_get.argtypes = [P, ctypes.POINTER(Stats)]
    lib.s5_strerror.argtypes = [ctypes.c_int]
    lib.s5_strerror.restype = ctypes.c_char_p
    lib.s5_release.argtypes = []
    lib.s5_release.restype = None
    lib.s5_prefix_keys.argtypes = [P, P, U32, U32, P, P]
    lib.s5_classify.argtypes = [P, U32, P, U32, P, P]
    lib.s5_classify_ex.argtypes = [P, U32, P, U32, U32, P, P]
    lib.s5_mlp_train.argtypes = [P, U32, U32, ctypes.c_float, U64, P, P]
    lib.s5_mlp_grad.argtypes = [P, P, U32, P, P]
    lib.s5_mlp_eval.argtypes = [P, P, U32, U64, U64, P, P]
    lib.s5_mlp_propose.argtypes = [P, P, U32, U32, ctypes.c_float, P, P, P, P]
    lib.s5_profile_enable.argtypes = [ctypes.c_int]
    lib.s5_profile_only.argtypes = [ctypes.c_char_p]
    lib.s5_profile_only.restype = ctypes.c_int
    lib.s5_profile_read.argtypes = [ctypes.POINTER(KernelProfile), U32, ctypes.POINTER(U32)]
    lib.s5_debug_limit_capacity.argtypes = [U32, U32]
    lib.s5_debug_count_writes.argtypes = [P, P, U64, P, P, P]
    lib.s5_debug_miss_publish.argtypes = [ctypes.c_int]
    for f in ("s5_debug_limit_capacity", "s5_debug_count_writes", "s5_debug_miss_publish",
              "s5_sort", "s5_sort_ex",
              "s5_sort_static", "s5_sort_batched", "s5_classify_ex", "s5_sort_batched_tuned", "s5_stats_get",
              "s5_prefix_keys",
              "s5_classify", "s5_profile_enable", "s5_profile_read", "s5_mlp_train", "s5_mlp_grad",
              "s5_mlp_eval", "s5_mlp_propose"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _check(rc: int):
    if rc != S5_OK:
        raise S5Error(f"S^5 call failed: {load().s5_strerror(rc).decode()} ({rc})")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_out(out_perm: torch.Tensor, out_lcp: torch.Tensor, n: int):
    if out_perm.numel() < n or out_lcp.numel() < n:
        raise ValueError(f"out_perm and out_lcp need at least {n} entries")


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_config(splitters=0, oversample=0, unroll=0, tile=0, base_threshold=0,
                splitter_mode=SPLIT_SAMPLED, imbalance_bound=0.0, seed=0,
                graph_levels=0, classifier=CLASSIFY_UNROLL, alphabet=ALPHABET_BYTES,
                distribution=DISTRIBUTE_ONE_PASS) -> Config:
    return Config(splitters, oversample, unroll, tile, base_threshold, splitter_mode,
                  imbalance_bound, seed, graph_levels, classifier, alphabet, distribution)


def sort(chars: torch.Tensor, offsets: torch.Tensor, cfg: Config | None = None,
         out_perm: torch.Tensor | None = None, out_lcp: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None, stream=None):
    """Sort the strings at ``offsets`` (uint64) in the arena ``chars`` (uint8).

    Returns ``(perm, lcp)`` as uint32 device tensors.
    """
    lib = load()
    n = offsets.numel()
    dev = offsets.device
    if out_perm is None:
        out_perm = torch.empty(n, dtype=torch.uint32, device=dev)
    if out_lcp is None:
        out_lcp = torch.empty(n, dtype=torch.uint32, device=dev)
    _check_out(out_perm, out_lcp, n)
    ws, wsb = None, 0
    if workspace is not None:
        # a workspace smaller than workspace_bytes(n, cfg) is rejected by the
        # library (S5_ERR_NOMEM) before any device work
        ws, wsb = _dev(workspace, torch.uint8, "workspace"), workspace.numel()
    rc = lib.s5_sort_ex(_dev(chars, torch.uint8, "chars"), chars.numel(),
                        _dev(offsets, torch.uint64, "offsets"), n,
                        _dev(out_perm, torch.uint32, "out_perm"),
                        _dev(out_lcp, torch.uint32, "out_lcp"),
                        ctypes.byref(cfg) if cfg is not None else None, ws, wsb, _stream(stream))
    _check(rc)
    return out_perm, out_lcp


def sort_static(chars: torch.Tensor, offsets: torch.Tensor, out_perm: torch.Tensor,
                out_lcp: torch.Tensor, cfg: Config | None = None, stream=None) -> int:
    """``s5_sort_static``: the sort with its workspace in the library's static
    scratch array (no allocation).  The caller passes the outputs; returns the
    status code (``S5_ERR_TOO_LARGE`` if the sort does not fit the array)."""
    _check_out(out_perm, out_lcp, offsets.numel())
    return int(load().s5_sort_static(_dev(chars, torch.uint8, "chars"), chars.numel(),
                                     _dev(offsets, torch.uint64, "offsets"), offsets.numel(),
                                     _dev(out_perm, torch.uint32, "out_perm"),
                                     _dev(out_lcp, torch.uint32, "out_lcp"),
                                     ctypes.byref(cfg) if cfg is not None else None,
                                     _stream(stream)))


def sort_plain(chars: torch.Tensor, offsets: torch.Tensor, out_perm: torch.Tensor,
               out_lcp: torch.Tensor, stream=None):
    """The 6-argument entry point ``s5_sort`` (internal workspace pool, defaults)."""
    _check_out(out_perm, out_lcp, offsets.numel())
    _check(load().s5_sort(_dev(chars, torch.uint8, "chars"),
                          _dev(offsets, torch.uint64, "offsets"), offsets.numel(),
                          _dev(out_perm, torch.uint32, "out_perm"),
                          _dev(out_lcp, torch.uint32, "out_lcp"), _stream(stream)))
    return out_perm, out_lcp


def make_tuning(rows) -> ctypes.Array:
    """Host array of SetTuning from (splitters, base_threshold, tile) rows."""
    arr = (SetTuning * len(rows))()
    for i, (v, t, tile) in enumerate(rows):
        arr[i] = SetTuning(v, t, tile)
    return arr


def sort_batched(chars: torch.Tensor, offsets: torch.Tensor, set_begin: torch.Tensor,
                 cfg: Config | None = None, tuning=None, out_perm: torch.Tensor | None = None,
                 out_lcp: torch.Tensor | None = None, stream=None):
    """Sort every set ``offsets[set_begin[s]:set_begin[s+1]]`` on its own (one
    graph launch for all sets; ``tuning``: per-set parameters from
    ``make_tuning``).

    Returns set-local ``perm`` and ``lcp`` (0 at each set's first slot)."""
    lib = load()
    n = offsets.numel()
    if out_perm is None:
        out_perm = torch.empty(n, dtype=torch.uint32, device=offsets.device)
    if out_lcp is None:
        out_lcp = torch.empty(n, dtype=torch.uint32, device=offsets.device)
    _check_out(out_perm, out_lcp, n)
    num_sets = set_begin.numel() - 1
    if num_sets < 0:
        raise ValueError("set_begin needs num_sets + 1 entries")
    if tuning is not None and len(tuning) != num_sets:
        raise ValueError("tuning needs one entry per set")
    if num_sets and int(set_begin[-1]) > n:  # the sets would read past offsets
        raise ValueError("set_begin[-1] exceeds the number of offsets")
    rc = lib.s5_sort_batched_tuned(_dev(chars, torch.uint8, "chars"), chars.numel(),
                                   _dev(offsets, torch.uint64, "offsets"),
                                   _dev(set_begin, torch.uint64, "set_begin"), num_sets, tuning,
                                   _dev(out_perm, torch.uint32, "out_perm"),
                                   _dev(out_lcp, torch.uint32, "out_lcp"),
                                   ctypes.byref(cfg) if cfg is not None else None, _stream(stream))
    _check(rc)
    return out_perm, out_lcp


def workspace_bytes(n: int, cfg: Config | None = None) -> int:
    return int(load().s5_workspace_bytes(n, ctypes.byref(cfg) if cfg is not None else None))


def stats(stream=None) -> dict:
    st = Stats()
    rc = load().s5_stats_get(_stream(stream), ctypes.byref(st))
    _check(rc)
    return st.as_dict()


def prefix_keys(chars: torch.Tensor, offsets: torch.Tensor, depth: int = 0, stream=None):
    """uint64 keys: the 8 bytes of every string at ``depth``, big-endian, zero-padded."""
    n = offsets.numel()
    keys = torch.empty(n, dtype=torch.uint64, device=offsets.device)
    _check(load().s5_prefix_keys(_dev(chars, torch.uint8, "chars"),
                                 _dev(offsets, torch.uint64, "offsets"), n, depth,
                                 _dev(keys, torch.uint64, "keys"), _stream(stream)))
    return keys


def classify(keys: torch.Tensor, splitters: torch.Tensor, variant: int = CLASSIFY_UNROLL,
             stream=None):
    """Ternary bucket (uint16) of every key against sorted splitters (2^d - 1 of them)."""
    n = keys.numel()
    out = torch.empty(n, dtype=torch.uint16, device=keys.device)
    _check(load().s5_classify_ex(_dev(keys, torch.uint64, "keys"), n,
                                 _dev(splitters, torch.uint64, "splitters"), splitters.numel(),
                                 variant, _dev(out, torch.uint16, "out"), _stream(stream)))
    return out


def release():
    load().s5_release()


def profile_enable(on: bool = True):
    """Turn per-kernel HIP-event timing on or off (clears the accumulators)."""
    _check(load().s5_profile_enable(1 if on else 0))


def profile_only(kernel: str | None = None):
    """Time only the launches of ``kernel`` (None: every kernel)."""
    _check(load().s5_profile_only(kernel.encode() if kernel else None))


def profile_read() -> dict:
    """Per-kernel totals since the last ``profile_enable``: name -> dict."""
    arr = (KernelProfile * 32)()
    cnt = ctypes.c_uint32(0)
    _check(load().s5_profile_read(arr, 32, ctypes.byref(cnt)))
    out = {}
    for i in range(min(cnt.value, 32)):
        e = arr[i]
        out[e.name.decode()] = {"launches": e.launches, "total_ms": e.total_ms,
                                "items": e.items, "alg_bytes": e.alg_bytes}
    return out


N_MLP_PARAMS = 1377


def mlp_train(sorted_keys: torch.Tensor, steps: int, lr: float, seed: int, stream=None):
    """Train the learned-splitter model on sorted uint64 keys; returns 1377 float32 params."""
    out = torch.empty(N_MLP_PARAMS, dtype=torch.float32, device=sorted_keys.device)
    _check(load().s5_mlp_train(_dev(sorted_keys, torch.uint64, "sorted_keys"), sorted_keys.numel(),
                               steps, lr, seed, _dev(out, torch.float32, "out"), _stream(stream)))
    return out


def mlp_grad(params: torch.Tensor, sorted_keys: torch.Tensor, stream=None):
    out = torch.empty(N_MLP_PARAMS, dtype=torch.float32, device=sorted_keys.device)
    _check(load().s5_mlp_grad(_dev(params, torch.float32, "params"),
                              _dev(sorted_keys, torch.uint64, "sorted_keys"), sorted_keys.numel(),
                              _dev(out, torch.float32, "out"), _stream(stream)))
    return out


def mlp_eval(params: torch.Tensor, keys: torch.Tensor, lo: int = 0, hi: int = 2**64 - 1,
             stream=None):
    """Model output for every key, features scaled by the byte-wise range (lo, hi)."""
    out = torch.empty(keys.numel(), dtype=torch.float32, device=keys.device)
    _check(load().s5_mlp_eval(_dev(params, torch.float32, "params"), _dev(keys, torch.uint64, "keys"),
                              keys.numel(), lo, hi, _dev(out, torch.float32, "out"),
                              _stream(stream)))
    return out


def mlp_propose(params: torch.Tensor, sorted_keys: torch.Tensor, v: int, beta: float = 4.0,
                stream=None):
    """The learned splitter proposal for a model and its sorted sample: returns
    ``(splitters uint64[v], model outputs float32[m], rejected uint32[1])``."""
    m = sorted_keys.numel()
    dev = sorted_keys.device
    spl = torch.empty(v, dtype=torch.uint64, device=dev)
    y = torch.empty(m, dtype=torch.float32, device=dev)
    rej = torch.empty(1, dtype=torch.uint32, device=dev)
    _check(load().s5_mlp_propose(_dev(params, torch.float32, "params"),
                                 _dev(sorted_keys, torch.uint64, "sorted_keys"), m, v, beta,
                                 _dev(spl, torch.uint64, "splitters"),
                                 _dev(y, torch.float32, "cdf"), _dev(rej, torch.uint32, "reject"),
                                 _stream(stream)))
    return spl, y, rej
