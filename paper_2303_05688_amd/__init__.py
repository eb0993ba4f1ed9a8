"""MI355X (gfx950) ASCI determinant search: Python binding of libasci.so.

Argument marshalling only: every step of the search runs in the HIP library.
Device arrays are torch tensors on a ROCm device (PyTorch provides device
memory and streams); work is queued on torch's current stream.  Importing this
package raises if the library has not been built (see ``build.py``); there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# One HIP runtime per process.  PyTorch-ROCm carries its own libamdhip64 with
# the same soname as the system one; loading torch first makes libasci.so bind
# to that copy.  Loaded the other way round, the process would hold two HIP
# runtimes, and the second one to initialise finds no device.
import torch  # noqa: E402,F401  (device memory and streams come from torch)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasci.so")

ASCI_OK, ASCI_EINVAL, ASCI_ENOMEM, ASCI_EDEVICE = 0, -1, -2, -3
ASCI_EAGAIN = 1


class AsciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % ({-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE"}.get(code, "?"), code, msg))
        self.code = code


class Options(C.Structure):
    _fields_ = [("ncore", C.c_int64), ("eps", C.c_double), ("constraint_level", C.c_int32),
                ("ecore", C.c_double), ("pair_buffer_bytes", C.c_int64), ("split_pairs", C.c_int64)]


class LoopOptions(C.Structure):
    _fields_ = [("ncore", C.c_int64), ("ntdets", C.c_int64), ("max_iter", C.c_int32), ("e_tol", C.c_double),
                ("davidson_subspace", C.c_int32), ("davidson_max_iter", C.c_int32), ("davidson_tol", C.c_double),
                ("pt2", C.c_int32), ("search", Options)]


class LoopIter(C.Structure):
    _fields_ = [("ndets", C.c_int64), ("candidates", C.c_int64), ("nnz", C.c_int64), ("energy", C.c_double),
                ("davidson_resid", C.c_double), ("davidson_iters", C.c_int32), ("search_ms", C.c_double),
                ("select_ms", C.c_double), ("hbuild_ms", C.c_double), ("davidson_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("h", C.c_void_p), ("eri", C.c_void_p), ("norb", C.c_int), ("nalpha", C.c_int),
                ("nbeta", C.c_int), ("dets", C.c_void_p), ("coeffs", C.c_void_p), ("ndets", C.c_int64),
                ("E0", C.c_double), ("k", C.c_int64), ("opt", Options), ("out_dets", C.c_void_p),
                ("out_scores", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("count", C.c_int64), ("latency_ms", C.c_double), ("run_ms", C.c_double),
                ("contributions", C.c_int64)]


class AsyncResult(C.Structure):
    _fields_ = [("count", C.c_int64), ("status", C.c_int32), ("flags", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("rejected", C.c_int64), ("max_running", C.c_int64), ("peak_bytes", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("wall_s", C.c_double),
                ("contributions", C.c_int64), ("bypassed", C.c_int64), ("held_results", C.c_int64)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libasci.so is not built: run `python paper_2303_05688_amd/build.py` "
                      "(or __graft_entry__.build()) first")

_lib = C.CDLL(LIB_PATH)
_vp, _dp, _up, _ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.POINTER(C.c_int64)
_lib.asci_version.restype = C.c_int
_lib.asci_strerror.restype = C.c_char_p
_lib.asci_strerror.argtypes = [C.c_int]
_lib.asci_last_error.restype = C.c_char_p
_lib.asci_options_default.argtypes = [C.POINTER(Options)]
_lib.asci_ctx_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
_lib.asci_ctx_destroy.argtypes = [_vp]
_lib.asci_search.argtypes = [_dp, _dp, C.c_int, C.c_int, C.c_int, _up, _dp, C.c_int64, C.c_double, C.c_int64,
                             C.POINTER(Options), _up, _dp, _ip]
_lib.asci_search_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double,
                                    C.c_int64, C.POINTER(Options), _vp, _vp, _ip, _vp]
_lib.asci_search_device_noalloc.argtypes = [_vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double,
                                            C.c_int64, C.POINTER(Options), _vp, _vp, _ip, _vp]
_lib.asci_candidates_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64,
                                        C.c_double, C.POINTER(Options), C.c_int64, _vp, _vp, _vp, _ip, _vp]
_lib.asci_class_counts_device.argtypes = [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64,
                                          C.POINTER(Options), C.c_int64, _up, _ip, _ip, _vp]
_lib.asci_pt2_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double,
                                 C.POINTER(Options), _dp, _ip, _vp]
_lib.asci_energy_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double,
                                    _dp, _vp]
_lib.asci_balance_classes.argtypes = [_ip, C.c_int64, C.c_int32, C.POINTER(C.c_int32), _ip]
_lib.asci_hmat_build_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, C.c_int64, C.c_double,
                                        C.POINTER(C.c_void_p), _vp]
_lib.asci_hmat_info.argtypes = [_vp, _ip, _ip]
_lib.asci_hmat_export.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.asci_hmat_matvec_device.argtypes = [_vp, _vp, _vp, _vp]
_lib.asci_hmat_destroy.restype = None
_lib.asci_hmat_destroy.argtypes = [_vp]
_lib.asci_davidson_device.argtypes = [_vp, _vp, _vp, C.c_int32, C.c_int32, C.c_double, _dp, _vp, _dp,
                                      C.POINTER(C.c_int32), _vp]
_lib.asci_loop_options_default.restype = None
_lib.asci_loop_options_default.argtypes = [C.POINTER(LoopOptions)]
_lib.asci_loop_step_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64, C.c_double,
                                       C.POINTER(LoopOptions), _vp, _vp, _ip, C.POINTER(LoopIter), _vp]
_lib.asci_run_device.argtypes = [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _vp, _vp, C.c_int64,
                                 C.POINTER(LoopOptions), _vp, _vp, _ip, _dp, _dp, C.POINTER(LoopIter),
                                 C.POINTER(C.c_int32), _vp]

_lib.asci_ctx_set_profiling.argtypes = [_vp, C.c_int]
_lib.asci_ctx_profile_only.argtypes = [_vp, C.c_char_p]
_lib.asci_ctx_set_param.argtypes = [_vp, C.c_char_p, C.c_int64]
_lib.asci_ctx_get_param.argtypes = [_vp, C.c_char_p, _ip]
_lib.asci_ctx_profile_entry.argtypes = [_vp, C.c_int, C.c_char_p, C.c_int, _dp, _ip, _dp]

_lib.asci_request_footprint.restype = C.c_int64
_lib.asci_request_footprint.argtypes = [C.POINTER(Request)]
_lib.asci_search_batch.argtypes = [_vp, C.POINTER(Request), C.c_int, C.POINTER(Result), _vp]
_lib.asci_autotune.argtypes = [_vp, C.POINTER(Request), C.c_int, _ip, _ip]
_lib.asci_server_create.argtypes = [C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_void_p)]
_lib.asci_server_create_fake.argtypes = [C.c_int64, C.c_int, C.c_double, C.POINTER(C.c_void_p)]
_lib.asci_server_submit.argtypes = [_vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
_lib.asci_server_poll.argtypes = [_vp, C.c_uint64, C.POINTER(Result)]
_lib.asci_server_footprint.restype = C.c_int64
_lib.asci_server_footprint.argtypes = [_vp, C.POINTER(Request)]
_lib.asci_server_wait.argtypes = [_vp, C.c_uint64, C.POINTER(Result)]
_lib.asci_server_get_stats.argtypes = [_vp, C.POINTER(ServerStats)]
_lib.asci_server_destroy.argtypes = [_vp]
_lib.asci_server_set_param.argtypes = [_vp, C.c_char_p, C.c_double]
_lib.asci_search_async.argtypes = [_vp, C.POINTER(Request), _vp, _vp]
_lib.asci_request_async_bytes.argtypes = [_vp, C.POINTER(Request), _ip]
_lib.asci_tune_shapes.argtypes = [_vp, C.POINTER(Request), C.c_int, C.POINTER(C.c_int)]
_lib.asci_tune_record.argtypes = [C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_int]
_lib.asci_tune_lookup.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, C.POINTER(C.c_int)]
_lib.asci_tune_save.argtypes = [C.c_char_p]
_lib.asci_tune_load.argtypes = [C.c_char_p, C.POINTER(C.c_int)]
_lib.asci_tune_arch.argtypes = [C.c_int, C.c_char_p, C.c_int]

EXPORTS = ["asci_version", "asci_strerror", "asci_last_error", "asci_options_default", "asci_ctx_create",
           "asci_ctx_destroy", "asci_ctx_set_param", "asci_ctx_get_param", "asci_ctx_set_profiling",
           "asci_ctx_profile_only", "asci_ctx_profile_entry", "asci_search",
           "asci_search_device", "asci_candidates_device", "asci_pt2_device", "asci_class_counts_device",
           "asci_energy_device", "asci_balance_classes", "asci_hmat_build_device", "asci_hmat_info",
           "asci_hmat_export", "asci_hmat_matvec_device", "asci_hmat_destroy", "asci_davidson_device",
           "asci_loop_options_default", "asci_loop_step_device", "asci_run_device",
           "asci_request_footprint", "asci_search_batch", "asci_autotune", "asci_server_create",
           "asci_server_create_fake", "asci_server_submit", "asci_server_footprint", "asci_server_poll",
           "asci_server_wait", "asci_server_set_param", "asci_search_device_noalloc", "asci_search_async",
           "asci_request_async_bytes", "asci_tune_shapes", "asci_tune_record", "asci_tune_lookup",
           "asci_tune_clear", "asci_tune_save", "asci_tune_load", "asci_tune_arch",
           "asci_server_get_stats", "asci_server_destroy"]


def lib():
    return _lib


def _check(rc):
    if rc != ASCI_OK:
        raise AsciError(rc, _lib.asci_last_error().decode())


def options(ncore=0, eps=0.0, ecore=0.0, pair_buffer_bytes=0, constraint_level=3, split_pairs=0):
    o = Options()
    _lib.asci_options_default(C.byref(o))
    o.ncore, o.eps, o.ecore = int(ncore), float(eps), float(ecore)
    o.pair_buffer_bytes, o.constraint_level = int(pair_buffer_bytes), int(constraint_level)
    o.split_pairs = int(split_pairs)
    return o


class Context:
    """One asci_ctx (device workspace) per device."""

    _cache = {}

    def __init__(self, device=0):
        self.device = device
        self.ptr = C.c_void_p()
        _check(_lib.asci_ctx_create(device, C.byref(self.ptr)))

    @classmethod
    def get(cls, device=0):
        if device not in cls._cache:
            cls._cache[device] = cls(device)
        return cls._cache[device]

    def set_param(self, name, value):
        _check(_lib.asci_ctx_set_param(self.ptr, name.encode(), int(value)))

    def get_param(self, name):
        v = C.c_int64()
        _check(_lib.asci_ctx_get_param(self.ptr, name.encode(), C.byref(v)))
        return v.value

    def set_profiling(self, enable=True, only=None):
        """Per-kernel timing; `only` restricts the events to one kernel name."""
        _check(_lib.asci_ctx_profile_only(self.ptr, (only or "").encode()))
        _check(_lib.asci_ctx_set_profiling(self.ptr, int(bool(enable))))

    def profile(self):
        """{kernel name: (total ms, launches, algorithmic bytes)} since profiling was enabled."""
        out = {}
        i = 0
        buf = C.create_string_buffer(64)
        ms, nl, by = C.c_double(), C.c_int64(), C.c_double()
        while _lib.asci_ctx_profile_entry(self.ptr, i, buf, 64, C.byref(ms), C.byref(nl), C.byref(by)) == 0:
            out[buf.value.decode()] = (ms.value, nl.value, by.value)
            i += 1
        return out

    def close(self):
        """Free the context (its device workspace) now."""
        if self.ptr:
            _lib.asci_ctx_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _torch():
    import torch
    return torch


def _dev(t, dtype):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a tensor on a ROCm device")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("expected a contiguous %s tensor" % dtype)
    return t.data_ptr()


def _stream(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dets_tensor(dets):
    torch = _torch()
    if dets.dtype == torch.uint64:
        return dets
    if dets.dtype == torch.int64:
        return dets.view(torch.uint64)
    raise TypeError("determinants must be uint64 (or int64 bit patterns)")


def search(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, k, ncore=0, eps=0.0, ecore=0.0,
           pair_buffer_bytes=0, constraint_level=3, split_pairs=0, ctx=None):
    """ASCI search on device tensors: returns (dets[m, 2] uint64, scores[m] float64)
    on the same device, ordered by |score| descending, ties by key ascending."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    out_d = torch.empty((int(k), 2), dtype=torch.uint64, device=h.device)
    out_s = torch.empty((int(k),), dtype=torch.float64, device=h.device)
    cnt = C.c_int64(0)
    o = options(ncore, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs)
    _check(_lib.asci_search_device(ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                                   _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0],
                                   float(E0), int(k), C.byref(o), out_d.data_ptr(), out_s.data_ptr(),
                                   C.byref(cnt), _stream(dev)))
    m = cnt.value
    return out_d[:m], out_s[:m]


def search_noalloc(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, k, out_dets, out_scores, ncore=0, eps=0.0,
                   ecore=0.0, constraint_level=3, split_pairs=0):
    """asci_search_device_noalloc into caller-owned outputs (out_dets[k, 2]
    uint64, out_scores[k] float64 device tensors); returns the count.  The
    call allocates no device memory."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    dets = _dets_tensor(dets)
    if out_dets.shape[0] < int(k) or out_scores.shape[0] < int(k):
        raise ValueError("outputs shorter than k")
    cnt = C.c_int64(0)
    o = options(ncore, eps, ecore, 0, constraint_level, split_pairs)
    _check(_lib.asci_search_device_noalloc(_dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                                           _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0],
                                           float(E0), int(k), C.byref(o), _dev(out_dets, torch.uint64),
                                           _dev(out_scores, torch.float64), C.byref(cnt), _stream(dev)))
    return cnt.value


def candidates(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0,
               pair_buffer_bytes=0, constraint_level=3, split_pairs=0, ctx=None):
    """Every candidate, ascending key: (dets[U, 2], N_a[U], A_a[U]) on the device."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    o = options(ncore, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs)
    cnt = C.c_int64(0)
    args = (ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
            _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0], float(E0), C.byref(o))
    rc = _lib.asci_candidates_device(*args, 0, None, None, None, C.byref(cnt), _stream(dev))
    if rc not in (ASCI_OK, ASCI_ENOMEM) or (rc == ASCI_ENOMEM and cnt.value == 0):
        _check(rc)
    U = cnt.value
    out_d = torch.empty((max(U, 1), 2), dtype=torch.uint64, device=h.device)
    out_n = torch.empty((max(U, 1),), dtype=torch.float64, device=h.device)
    out_s = torch.empty((max(U, 1),), dtype=torch.float64, device=h.device)
    _check(_lib.asci_candidates_device(*args, U, out_d.data_ptr(), out_n.data_ptr(), out_s.data_ptr(),
                                       C.byref(cnt), _stream(dev)))
    return out_d[:U], out_n[:U], out_s[:U]


def pt2(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, ncore=0, eps=0.0, ecore=0.0, pair_buffer_bytes=0,
        constraint_level=3, split_pairs=0, ctx=None):
    """Second-order energy of the candidates: (E_PT2, number of candidates)."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    e, cnt = C.c_double(), C.c_int64()
    o = options(ncore, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs)
    _check(_lib.asci_pt2_device(ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                                _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0], float(E0),
                                C.byref(o), C.byref(e), C.byref(cnt), _stream(dev)))
    return e.value, cnt.value


def class_counts(norb, nalpha, nbeta, dets, coeffs, ncore=0, constraint_level=3, split_pairs=0, ctx=None):
    """Non-empty constraint classes (level 3 = triplets; split_pairs > 0 splits the
    heavy ones): (masks uint64[m] ascending, pair counts int64[m]) as numpy arrays."""
    torch = _torch()
    dev = dets.device.index if dets.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    o = options(ncore, constraint_level=constraint_level, split_pairs=split_pairs)
    cnt = C.c_int64(0)
    cap = 1
    for _ in range(2):
        masks = np.zeros(cap, dtype=np.uint64)
        counts = np.zeros(cap, dtype=np.int64)
        rc = _lib.asci_class_counts_device(ctx.ptr, norb, nalpha, nbeta, _dev(dets, torch.uint64),
                                           _dev(coeffs, torch.float64), dets.shape[0], C.byref(o), cap,
                                           masks.ctypes.data_as(_up), counts.ctypes.data_as(_ip), C.byref(cnt),
                                           _stream(dev))
        if rc == ASCI_OK:
            return masks[:cnt.value], counts[:cnt.value]
        if rc != ASCI_ENOMEM:
            _check(rc)
        cap = cnt.value
    _check(rc)


def balance_classes(counts, npe):
    """Alg. 3's greedy static load balance: (owner int32[m], load int64[npe])."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    owner = np.zeros(len(counts), dtype=np.int32)
    load = np.zeros(int(npe), dtype=np.int64)
    _check(_lib.asci_balance_classes(counts.ctypes.data_as(_ip), len(counts), int(npe),
                                     owner.ctypes.data_as(C.POINTER(C.c_int32)), load.ctypes.data_as(_ip)))
    return owner, load


def pairs_per_det(norb, nalpha, nbeta):
    """Singles and doubles of one determinant (the closed-form pair count per core)."""
    va, vb = norb - nalpha, norb - nbeta
    c2 = lambda x: x * (x - 1) // 2  # noqa: E731
    return nalpha * va + nbeta * vb + c2(nalpha) * c2(va) + c2(nbeta) * c2(vb) + nalpha * va * nbeta * vb


def class_skew(counts, npes=(8, 64, 256, 1024)):
    """Skew statistics of a class partition (the single-GPU analogue of the
    per-element pair counts by constraint level): number of non-empty classes,
    the largest class over the mean, and for each element count P the largest
    Alg. 3 load over the mean load (1 = perfect balance) and the share of all
    pairs in the single largest class (indivisible work)."""
    counts = np.asarray(counts, dtype=np.int64)
    nz = counts[counts > 0]
    tot = int(nz.sum())
    out = {"classes": int(len(nz)), "pairs": tot,
           "max_over_mean": float(nz.max() / nz.mean()) if len(nz) else 0.0,
           "largest_share": float(nz.max() / tot) if tot else 0.0, "imbalance": {}}
    for p in npes:
        _, load = balance_classes(nz, p)
        out["imbalance"][int(p)] = float(load.max() / (tot / p)) if tot else 0.0
    return out


def energy(h, eri, norb, nalpha, nbeta, dets, coeffs, ecore=0.0, ctx=None):
    """<C|H|C> over the given determinants, computed on the device."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    e = C.c_double(0.0)
    _check(_lib.asci_energy_device(ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                                   _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0],
                                   float(ecore), C.byref(e), _stream(dev)))
    return e.value


def search_host(h, eri, norb, nalpha, nbeta, dets, coeffs, E0, k, ncore=0, eps=0.0, ecore=0.0,
                pair_buffer_bytes=0, constraint_level=3, split_pairs=0):
    """The host-buffer entry point (asci_search): numpy in, numpy out."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    out_d = np.zeros((int(k), 2), dtype=np.uint64)
    out_s = np.zeros(int(k), dtype=np.float64)
    cnt = C.c_int64(0)
    o = options(ncore, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs)
    _check(_lib.asci_search(h.ctypes.data_as(_dp), eri.ctypes.data_as(_dp), norb, nalpha, nbeta,
                            dets.ctypes.data_as(_up), coeffs.ctypes.data_as(_dp), len(coeffs), float(E0), int(k),
                            C.byref(o), out_d.ctypes.data_as(_up), out_s.ctypes.data_as(_dp), C.byref(cnt)))
    m = cnt.value
    return out_d[:m], out_s[:m]


# ---------------------------------------------------------------- batch and serving


class SearchRequest:
    """A device-side search request; allocates its outputs (k results) on the
    device and keeps references to every buffer it names."""

    def __init__(self, h, eri, norb, nalpha, nbeta, dets, coeffs, E0, k, ncore=0, eps=0.0, ecore=0.0,
                 pair_buffer_bytes=0, constraint_level=3, split_pairs=0):
        torch = _torch()
        dets = _dets_tensor(dets)
        self.keep = (h, eri, dets, coeffs)
        self.out_dets = torch.empty((int(k), 2), dtype=torch.uint64, device=h.device)
        self.out_scores = torch.empty((int(k),), dtype=torch.float64, device=h.device)
        self.c = Request(_dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                         _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0], float(E0), int(k),
                         options(ncore, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs), self.out_dets.data_ptr(),
                         self.out_scores.data_ptr())

    def result(self, count):
        return self.out_dets[:count], self.out_scores[:count]


def search_async(req, result=None, ctx=None, stream=None):
    """Queue a SearchRequest with nothing read back (asci_search_async) on
    `stream` (a torch.cuda.Stream, default the current one).  result: a device
    int64 tensor of 2 elements that receives (count, status | flags << 32);
    returned.  Read it after synchronising the stream (async_status)."""
    torch = _torch()
    dev = req.out_dets.device
    ctx = ctx or Context.get(dev.index if dev.index is not None else torch.cuda.current_device())
    if result is None:
        result = torch.zeros(2, dtype=torch.int64, device=dev)
    st = stream.cuda_stream if stream is not None else _stream(dev.index if dev.index is not None else 0)
    _check(_lib.asci_search_async(ctx.ptr, C.byref(req.c), result.data_ptr(), st))
    return result


def graph_capable(req, ctx=None):
    """Whether a SearchRequest is inside the asynchronous search's scope (and so
    runs in the captured graph of a batch)."""
    torch = _torch()
    dev = req.out_dets.device
    ctx = ctx or Context.get(dev.index if dev.index is not None else torch.cuda.current_device())
    v = C.c_int64()
    _check(_lib.asci_request_async_bytes(ctx.ptr, C.byref(req.c), C.byref(v)))
    return v.value


def async_status(result):
    """(count, status, flags) of an asci_async_result held in a 2-element int64 tensor."""
    r = result.cpu().tolist()
    count, word = int(r[0]), int(r[1]) & 0xFFFFFFFFFFFFFFFF
    status = word & 0xFFFFFFFF
    if status >= 1 << 31:
        status -= 1 << 32
    return count, status, word >> 32


def tune_shapes(requests, ctx=None):
    """Time each distinct request shape with finish_cap 4096 / 2048 / 1024 and
    record the fastest (process-wide); returns the number of shapes timed."""
    torch = _torch()
    ctx = ctx or Context.get(torch.cuda.current_device())
    arr = (Request * len(requests))(*[r.c for r in requests])
    n = C.c_int()
    _check(_lib.asci_tune_shapes(ctx.ptr, arr, len(requests), C.byref(n)))
    return n.value


def tune_record(arch, norb, nalpha, bucket, finish_cap):
    _check(_lib.asci_tune_record(arch.encode(), norb, nalpha, bucket, finish_cap))


def tune_lookup(device, norb, nalpha, pairs):
    v = C.c_int()
    _check(_lib.asci_tune_lookup(device, norb, nalpha, int(pairs), C.byref(v)))
    return v.value


def tune_arch(device=0):
    """The architecture name the per-shape tuning table keys device's entries by."""
    buf = C.create_string_buffer(128)
    _check(_lib.asci_tune_arch(device, buf, 128))
    return buf.value.decode()


def tune_clear():
    _check(_lib.asci_tune_clear())


def tune_save(path):
    _check(_lib.asci_tune_save(str(path).encode()))


def tune_load(path):
    n = C.c_int()
    _check(_lib.asci_tune_load(str(path).encode(), C.byref(n)))
    return n.value


def fake_request(norb, nalpha, nbeta, ndets, k):
    """A request with no buffers, for the fake (host-only) server."""
    return Request(None, None, norb, nalpha, nbeta, None, None, ndets, 0.0, k, options(), None, None)


def footprint(req):
    c = req.c if isinstance(req, SearchRequest) else req
    return _lib.asci_request_footprint(C.byref(c))


def search_batch(requests, ctx=None):
    """Run SearchRequests as one batch; returns the list of Result structs."""
    torch = _torch()
    ctx = ctx or Context.get(torch.cuda.current_device())
    arr = (Request * len(requests))(*[r.c for r in requests])
    res = (Result * len(requests))()
    rc = _lib.asci_search_batch(ctx.ptr, arr, len(requests), res, _stream(torch.cuda.current_device()))
    if rc != ASCI_OK:
        raise AsciError(rc, "batch: " + ", ".join(str(r.status) for r in res))
    return list(res)


def autotune(sample_requests, ctx=None):
    """Per-shape tuning of the sample's shapes (asci_autotune): returns the batch
    slots (unchanged) and the finish capacity recorded for the largest request."""
    torch = _torch()
    ctx = ctx or Context.get(torch.cuda.current_device())
    arr = (Request * len(sample_requests))(*[r.c for r in sample_requests])
    bs, bc = C.c_int64(), C.c_int64()
    _check(_lib.asci_autotune(ctx.ptr, arr, len(sample_requests), C.byref(bs), C.byref(bc)))
    return {"batch_slots": bs.value, "finish_cap": bc.value}


class Server:
    """Continuous-batching request loop (asci_server_*)."""

    def __init__(self, device=0, hbm_budget=None, slots=4, fake_ns_per_byte=None):
        self.ptr = C.c_void_p()
        if fake_ns_per_byte is not None:
            _check(_lib.asci_server_create_fake(int(hbm_budget), int(slots), float(fake_ns_per_byte),
                                                C.byref(self.ptr)))
        else:
            if hbm_budget is None:
                torch = _torch()
                free, _ = torch.cuda.mem_get_info(device)
                hbm_budget = int(free * 0.7)
            _check(_lib.asci_server_create(int(device), int(hbm_budget), int(slots), C.byref(self.ptr)))
        self.requests = {}

    def submit(self, req):
        c = req.c if isinstance(req, SearchRequest) else req
        t = C.c_uint64()
        rc = _lib.asci_server_submit(self.ptr, C.byref(c), C.byref(t))
        self.requests[t.value] = req
        if rc not in (ASCI_OK, ASCI_ENOMEM):
            _check(rc)
        return t.value

    def footprint(self, req):
        c = req.c if isinstance(req, SearchRequest) else req
        return _lib.asci_server_footprint(self.ptr, C.byref(c))

    def poll(self, ticket):
        """The result once the request has completed (handed over once), else None."""
        r = Result()
        rc = _lib.asci_server_poll(self.ptr, ticket, C.byref(r))
        if rc == ASCI_OK:
            self.requests.pop(ticket, None)
            return r
        if rc != ASCI_EAGAIN:
            _check(rc)
        return None

    def wait(self, ticket):
        r = Result()
        _check(_lib.asci_server_wait(self.ptr, ticket, C.byref(r)))
        self.requests.pop(ticket, None)
        return r

    def set_param(self, name, value):
        _check(_lib.asci_server_set_param(self.ptr, name.encode(), float(value)))

    def stats(self):
        st = ServerStats()
        _check(_lib.asci_server_get_stats(self.ptr, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.ptr:
            _lib.asci_server_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- variational step and the ASCI loop


class HMat:
    """H over a determinant set (device CSR built by the double loop)."""

    def __init__(self, h, eri, norb, nalpha, nbeta, dets, ecore=0.0, ctx=None):
        torch = _torch()
        dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
        self.ctx = ctx or Context.get(dev)
        self.device = h.device
        self._dev = dev
        dets = _dets_tensor(dets)
        self.ptr = C.c_void_p()
        _check(_lib.asci_hmat_build_device(self.ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb,
                                           nalpha, nbeta, _dev(dets, torch.uint64), dets.shape[0], float(ecore),
                                           C.byref(self.ptr), _stream(dev)))
        nr, nz = C.c_int64(), C.c_int64()
        _check(_lib.asci_hmat_info(self.ptr, C.byref(nr), C.byref(nz)))
        self.nrows, self.nnz = nr.value, nz.value

    def export(self):
        """(rowptr int64[n+1], cols int32[nnz], vals float64[nnz]) device tensors."""
        torch = _torch()
        rp = torch.empty(self.nrows + 1, dtype=torch.int64, device=self.device)
        cols = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        vals = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.device)
        _check(_lib.asci_hmat_export(self.ptr, rp.data_ptr(), cols.data_ptr(), vals.data_ptr(), _stream(self._dev)))
        return rp, cols[: self.nnz], vals[: self.nnz]

    def matvec(self, x):
        torch = _torch()
        y = torch.empty(self.nrows, dtype=torch.float64, device=self.device)
        _check(_lib.asci_hmat_matvec_device(self.ptr, _dev(x, torch.float64), y.data_ptr(), _stream(self._dev)))
        return y

    def close(self):
        if self.ptr:
            _lib.asci_hmat_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def davidson(H, guess=None, max_subspace=24, max_iter=200, tol=1e-8):
    """Lowest eigenpair of an HMat (Alg. 5, shifted-Jacobi preconditioner):
    (energy, vector tensor, residual norm, iterations)."""
    torch = _torch()
    vec = torch.empty(H.nrows, dtype=torch.float64, device=H.device)
    e, r, it = C.c_double(), C.c_double(), C.c_int32()
    g = _dev(guess, torch.float64) if guess is not None else None
    _check(_lib.asci_davidson_device(H.ctx.ptr, H.ptr, g, int(max_subspace), int(max_iter), float(tol), C.byref(e),
                                     vec.data_ptr(), C.byref(r), C.byref(it), _stream(H._dev)))
    return e.value, vec, r.value, it.value


def loop_options(ntdets, ncore=0, max_iter=10, e_tol=1e-6, davidson_subspace=24, davidson_max_iter=200,
                 davidson_tol=1e-8, pt2=False, eps=0.0, ecore=0.0, constraint_level=3, split_pairs=0,
                 pair_buffer_bytes=0):
    o = LoopOptions()
    _lib.asci_loop_options_default(C.byref(o))
    o.ncore, o.ntdets, o.max_iter, o.e_tol = int(ncore), int(ntdets), int(max_iter), float(e_tol)
    o.davidson_subspace, o.davidson_max_iter = int(davidson_subspace), int(davidson_max_iter)
    o.davidson_tol, o.pt2 = float(davidson_tol), int(bool(pt2))
    o.search = options(0, eps, ecore, pair_buffer_bytes, constraint_level, split_pairs)
    return o


def loop_step(h, eri, norb, nalpha, nbeta, dets, coeffs, Ek, opts, ctx=None):
    """One iteration of Alg. 1: (dets, coeffs, info dict) of psi_{k+1}."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets = _dets_tensor(dets)
    out_d = torch.empty((opts.ntdets, 2), dtype=torch.uint64, device=h.device)
    out_c = torch.empty(opts.ntdets, dtype=torch.float64, device=h.device)
    nn = C.c_int64()
    info = LoopIter()
    _check(_lib.asci_loop_step_device(ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha,
                                      nbeta, _dev(dets, torch.uint64), _dev(coeffs, torch.float64), dets.shape[0],
                                      float(Ek), C.byref(opts), out_d.data_ptr(), out_c.data_ptr(), C.byref(nn),
                                      C.byref(info), _stream(dev)))
    return out_d[: nn.value], out_c[: nn.value], info.as_dict()


def run(h, eri, norb, nalpha, nbeta, dets0, coeffs0, opts, ctx=None):
    """Alg. 1 from (dets0, coeffs0): dict with dets, coeffs (device), energy,
    pt2 and the per-iteration records."""
    torch = _torch()
    dev = h.device.index if h.device.index is not None else torch.cuda.current_device()
    ctx = ctx or Context.get(dev)
    dets0 = _dets_tensor(dets0)
    cap = max(int(opts.ntdets), dets0.shape[0])
    out_d = torch.empty((cap, 2), dtype=torch.uint64, device=h.device)
    out_c = torch.empty(cap, dtype=torch.float64, device=h.device)
    nn, e, p, ni = C.c_int64(), C.c_double(), C.c_double(), C.c_int32()
    recs = (LoopIter * max(1, int(opts.max_iter)))()
    _check(_lib.asci_run_device(ctx.ptr, _dev(h, torch.float64), _dev(eri, torch.float64), norb, nalpha, nbeta,
                                _dev(dets0, torch.uint64), _dev(coeffs0, torch.float64), dets0.shape[0],
                                C.byref(opts), out_d.data_ptr(), out_c.data_ptr(), C.byref(nn), C.byref(e),
                                C.byref(p), recs, C.byref(ni), _stream(dev)))
    return {"dets": out_d[: nn.value], "coeffs": out_c[: nn.value], "energy": e.value, "pt2": p.value,
            "iterations": [recs[i].as_dict() for i in range(ni.value)]}
