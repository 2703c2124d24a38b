"""Python binding of libprojmotif (PROJECTION motif finding on MI355X / gfx950).

Argument marshalling only: every function below forwards to the C ABI of
``include/projmotif.h`` with the same name; every step of the path runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  Importing
fails loudly when ``libprojmotif.so`` has not been built (there is no CPU
fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libprojmotif.so")

PM_OK, PM_EINVAL, PM_ERANGE, PM_ECAPACITY, PM_EDEVICE = 0, -1, -2, -3, -4
PM_STATUS_BAD_SYMBOL, PM_STATUS_BAD_MASK, PM_STATUS_CAPACITY = 1, 2, 4
PM_DNA, PM_PROTEIN = 4, 20
PM_FP64, PM_FP32, PM_F16X2, PM_F16 = 0, 1, 2, 3

DNA_CODE_ORDER = "ACTG"
PROTEIN_CODE_ORDER = "ARNDCQEGHILKMFPSTWYV"

EXPORTS = [
    "pm_version", "pm_last_error", "pm_packed_words", "pm_pack", "pm_masks_from_seed",
    "pm_auto_params", "projection_hash", "pm_select_workspace", "bucket_select",
    "bucket_profile", "theta_init", "em_refine", "em_best", "projection_run",
    "pm_batch_check", "projection_hash_batch", "bucket_select_batch", "bucket_profile_batch",
    "pm_em_batch_workspace", "pm_em_workspace", "em_refine_batch", "em_best_batch",
    "triage_features", "pm_triage_packed_bytes", "triage_pack", "triage_forward", "pm_triage_workspace",
    "triage_train_step", "pm_triage_select_workspace", "triage_select", "triage_fallback_select",
    "triage_merge_best", "em_autotune", "em_tuning", "em_set_tuning",
    "pm_hash_select_workspace", "bucket_hash_select", "pm_hash_select_batch_workspace", "bucket_hash_select_batch",
    "pm_hash_select_scratch_bytes", "bucket_hash_select_noalloc",
    "pm_sort_select_workspace", "bucket_sort_select", "pm_sort_select_batch_workspace", "bucket_sort_select_batch",
    "em_refine_model", "projection_run_range", "gibbs_refine",
    "projection_hash_select", "projection_hash_select_batch",
]

PM_TRIAGE_PARAMS, PM_TRIAGE_INPUTS = 88577, 87


class PmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class pm_seqs(C.Structure):
    _fields_ = [("alphabet", C.c_int32), ("t", C.c_int32), ("n_total", C.c_int64),
                ("n_min", C.c_int32), ("n_max", C.c_int32), ("offsets", C.c_void_p),
                ("packed", C.c_void_p)]


class pm_bucket(C.Structure):
    _fields_ = [("trial", C.c_uint32), ("key", C.c_uint32), ("size", C.c_uint32),
                ("first", C.c_uint32)]


class pm_inst(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("packed", C.c_void_p), ("n_total", C.c_int64),
                ("x", C.c_int64), ("key_base", C.c_int64), ("t", C.c_int32), ("n_min", C.c_int32),
                ("m", C.c_int32), ("first_item", C.c_int32)]


class pm_batch(C.Structure):
    _fields_ = [("alphabet", C.c_int32), ("l", C.c_int32), ("k", C.c_int32), ("P", C.c_int32),
                ("items", C.c_int32), ("inst", C.c_void_p), ("inst_host", C.c_void_p),
                ("item_inst", C.c_void_p)]


class pm_problem(C.Structure):
    _fields_ = [("alphabet", C.c_int32), ("t", C.c_int32), ("seqs", C.POINTER(C.c_char_p)),
                ("n", C.POINTER(C.c_int32)), ("l", C.c_int32), ("d", C.c_int32),
                ("k", C.c_int32), ("s", C.c_int32), ("m", C.c_int32),
                ("masks", C.POINTER(C.c_uint32)), ("seed", C.c_uint64),
                ("bg", C.POINTER(C.c_double))]


class pm_options(C.Structure):
    _fields_ = [("em_iters", C.c_int32), ("beta", C.c_double), ("precision", C.c_int32),
                ("batched", C.c_int32), ("triage", C.c_int32), ("triage_frac", C.c_double),
                ("triage_weights", C.c_char_p), ("stream", C.c_void_p)]


class pm_result(C.Structure):
    _fields_ = [("consensus", C.c_char_p), ("sites", C.POINTER(C.c_int32)),
                ("theta", C.POINTER(C.c_double)), ("J", C.c_double), ("llr", C.c_double),
                ("best_trial", C.c_int32), ("best_key", C.c_uint32), ("n_enriched", C.c_int64),
                ("n_refined", C.c_int64), ("fallback_used", C.c_int32),
                ("k", C.c_int32), ("s", C.c_int32), ("m", C.c_int32)]


_lib = None


def lib():
    """Load libprojmotif.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1605_06904_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, dbl, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64,
                                      C.c_double, C.c_size_t)
    sig = {
        "pm_version": (C.c_char_p, []),
        "pm_last_error": (C.c_char_p, []),
        "pm_packed_words": (i64, [i32, i64]),
        "pm_pack": (C.c_int, [i32, P, i64, P, P, P]),
        "pm_masks_from_seed": (C.c_int, [u64, i32, i32, i32, P]),
        "pm_auto_params": (C.c_int, [i32, i32, i64, i32, i32, dbl, P, P, P]),
        "projection_hash": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, i32, P, P, P, P]),
        "pm_select_workspace": (sz, [i32, i32, i32, i64]),
        "bucket_select": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, P, i32, u32, P, i64, P, i64,
                                    P, P, sz, P, P]),
        "bucket_profile": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, i64, P, P, P]),
        "theta_init": (C.c_int, [i32, i32, P, i64, P, P, dbl, P, P]),
        "em_refine": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, P, i32, dbl, i32, P, P, P,
                                P, P, sz, P]),
        "pm_em_workspace": (sz, [C.POINTER(pm_seqs), i32, i32]),
        "em_best": (C.c_int, [P, i64, P, i32, P, i32, i32, P, P, P]),
        "projection_run": (C.c_int, [C.POINTER(pm_problem), i32, C.POINTER(pm_options),
                                     C.POINTER(pm_result)]),
        "projection_run_range": (C.c_int, [C.POINTER(pm_problem), i32, i32, C.POINTER(pm_options),
                                           C.POINTER(pm_result), P]),
        "pm_batch_check": (C.c_int, [C.POINTER(pm_batch)]),
        "projection_hash_batch": (C.c_int, [C.POINTER(pm_batch), P, P, P, P, P]),
        "bucket_select_batch": (C.c_int, [C.POINTER(pm_batch), P, P, u32, P, i64, P, i64, P, P, sz,
                                          P, P]),
        "bucket_profile_batch": (C.c_int, [C.POINTER(pm_batch), P, P, i64, i64, P, P, P]),
        "pm_em_batch_workspace": (sz, [C.POINTER(pm_batch), i32]),
        "em_refine_batch": (C.c_int, [C.POINTER(pm_batch), P, P, P, i64, P, i32, dbl, i32, P, P, P,
                                      P, P, sz, P]),
        "em_best_batch": (C.c_int, [C.POINTER(pm_batch), P, P, i64, P, i32, P, P, P, P]),
        "triage_features": (C.c_int, [i32, P, i64, P, P, P, P, P, P]),
        "pm_triage_packed_bytes": (sz, []),
        "triage_pack": (C.c_int, [P, P, P]),
        "triage_forward": (C.c_int, [P, P, i64, P, P, P]),
        "pm_triage_workspace": (sz, [i32]),
        "triage_train_step": (C.c_int, [P, P, P, i32, P, P, i32, C.c_float, P, P, P, sz, P]),
        "pm_triage_select_workspace": (sz, [i32, i64]),
        "triage_select": (C.c_int, [C.c_void_p, P, P, i64, P, dbl, P, i32, i32, P, P, P, P, P, P, sz, P]),
        "triage_fallback_select": (C.c_int, [C.c_void_p, P, i64, P, P, P, P, P, i32, dbl, P, i32, i32, P, P,
                                             P, P, P, P, P, P, sz, P]),
        "triage_merge_best": (C.c_int, [i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P, P]),
        "em_autotune": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, i32, dbl, i32, P, P, P, sz, P, P]),
        "em_tuning": (C.c_int, [i32, i32]),
        "em_set_tuning": (C.c_int, [i32, i32, i32]),
        "pm_hash_select_workspace": (sz, [C.POINTER(pm_seqs), i32, i32, i32]),
        "bucket_hash_select": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, i32, u32, P, i64, P, i64, P, P, sz, P,
                                         P]),
        "pm_hash_select_batch_workspace": (sz, [C.POINTER(pm_batch)]),
        "bucket_hash_select_batch": (C.c_int, [C.POINTER(pm_batch), P, u32, P, i64, P, i64, P, P, sz, P, P]),
        "em_refine_model": (C.c_int, [C.POINTER(pm_seqs), i32, i32, dbl, P, P, i64, P, i32, dbl, i32, P, P, P, P,
                                      P, P]),
        "gibbs_refine": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, P, i32, dbl, u64, P, P, P, P]),
        "pm_sort_select_workspace": (sz, [C.POINTER(pm_seqs), i32, i32, i32]),
        "bucket_sort_select": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, i32, u32, P, i64, P, i64, P, P, sz, P,
                                         P]),
        "pm_sort_select_batch_workspace": (sz, [C.POINTER(pm_batch)]),
        "bucket_sort_select_batch": (C.c_int, [C.POINTER(pm_batch), P, u32, P, i64, P, i64, P, P, sz, P, P]),
        "projection_hash_select": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, i32, P, P, u32, P, i64, P, i64,
                                             P, P, sz, P, P]),
        "projection_hash_select_batch": (C.c_int, [C.POINTER(pm_batch), P, P, P, u32, P, i64, P, i64, P, P, sz,
                                                   P, P]),
        "pm_hash_select_scratch_bytes": (sz, []),
        "bucket_hash_select_noalloc": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, i32, u32, P, i64, P, i64, P, P,
                                                 P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != PM_OK:
        raise PmError(rc, lib().pm_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device (or host) address of a tensor, or None."""
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------- C ABI names
def pm_version() -> str:
    return lib().pm_version().decode()


def pm_last_error() -> str:
    return lib().pm_last_error().decode()


def pm_packed_words(alphabet: int, n_total: int) -> int:
    return int(lib().pm_packed_words(alphabet, n_total))


def pm_pack(alphabet, ascii, n_total, packed, status=None, stream=None):
    _check(lib().pm_pack(alphabet, _ptr(ascii), n_total, _ptr(packed), _ptr(status), _stream(stream)))


def pm_masks_from_seed(seed: int, l: int, k: int, m: int):
    import numpy as np
    out = np.zeros(max(m, 1), dtype=np.uint32)
    _check(lib().pm_masks_from_seed(seed, l, k, m, out.ctypes.data))
    return out[:m]


def pm_auto_params(alphabet: int, t: int, x: int, l: int, d: int, q: float = 0.95):
    k, s, m = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().pm_auto_params(alphabet, t, x, l, d, q, C.byref(k), C.byref(s), C.byref(m)))
    return k.value, s.value, m.value


def projection_hash(S: "Seqs", l, k, masks, m, keys=None, counts=None, status=None, stream=None):
    _check(lib().projection_hash(C.byref(S.c), l, k, _ptr(masks), m, _ptr(keys), _ptr(counts),
                                 _ptr(status), _stream(stream)))


def pm_select_workspace(alphabet: int, k: int, m: int, cap_buckets: int) -> int:
    return int(lib().pm_select_workspace(alphabet, k, m, cap_buckets))


def bucket_select(S, l, k, keys, counts, m, s, buckets, cap_buckets, members, cap_members, n_out,
                  ws, ws_bytes, status=None, stream=None):
    _check(lib().bucket_select(C.byref(S.c), l, k, _ptr(keys), _ptr(counts), m, s, _ptr(buckets),
                               cap_buckets, _ptr(members), cap_members, _ptr(n_out), _ptr(ws),
                               ws_bytes, _ptr(status), _stream(stream)))


def projection_hash_select(S, l, k, masks, m, keys, counts, s, buckets, cap_buckets, members, cap_members,
                           n_out, ws, ws_bytes, status=None, stream=None):
    _check(lib().projection_hash_select(C.byref(S.c), l, k, _ptr(masks), m, _ptr(keys), _ptr(counts), s,
                                        _ptr(buckets), cap_buckets, _ptr(members), cap_members, _ptr(n_out),
                                        _ptr(ws), ws_bytes, _ptr(status), _stream(stream)))


def pm_hash_select_workspace(S, l: int, k: int, m: int) -> int:
    return int(lib().pm_hash_select_workspace(C.byref(S.c), l, k, m))


def bucket_hash_select(S, l, k, masks, m, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                       status=None, stream=None):
    _check(lib().bucket_hash_select(C.byref(S.c), l, k, _ptr(masks), m, s, _ptr(buckets), cap_buckets,
                                    _ptr(members), cap_members, _ptr(n_out), _ptr(ws), ws_bytes, _ptr(status),
                                    _stream(stream)))


def pm_sort_select_workspace(S, l: int, k: int, m: int) -> int:
    return int(lib().pm_sort_select_workspace(C.byref(S.c), l, k, m))


def bucket_sort_select(S, l, k, masks, m, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                       status=None, stream=None):
    _check(lib().bucket_sort_select(C.byref(S.c), l, k, _ptr(masks), m, s, _ptr(buckets), cap_buckets,
                                    _ptr(members), cap_members, _ptr(n_out), _ptr(ws), ws_bytes, _ptr(status),
                                    _stream(stream)))


def pm_sort_select_batch_workspace(B) -> int:
    return int(lib().pm_sort_select_batch_workspace(C.byref(B.c)))


def bucket_sort_select_batch(B, masks, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                             status=None, stream=None):
    _check(lib().bucket_sort_select_batch(C.byref(B.c), _ptr(masks), s, _ptr(buckets), cap_buckets, _ptr(members),
                                          cap_members, _ptr(n_out), _ptr(ws), ws_bytes, _ptr(status),
                                          _stream(stream)))


def pm_hash_select_scratch_bytes() -> int:
    return int(lib().pm_hash_select_scratch_bytes())


def bucket_hash_select_noalloc(S, l, k, masks, m, s, buckets, cap_buckets, members, cap_members, n_out, status=None,
                               stream=None):
    _check(lib().bucket_hash_select_noalloc(C.byref(S.c), l, k, _ptr(masks), m, s, _ptr(buckets), cap_buckets,
                                            _ptr(members), cap_members, _ptr(n_out), _ptr(status), _stream(stream)))


def pm_hash_select_batch_workspace(B) -> int:
    return int(lib().pm_hash_select_batch_workspace(C.byref(B.c)))


def bucket_hash_select_batch(B, masks, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                             status=None, stream=None):
    _check(lib().bucket_hash_select_batch(C.byref(B.c), _ptr(masks), s, _ptr(buckets), cap_buckets, _ptr(members),
                                          cap_members, _ptr(n_out), _ptr(ws), ws_bytes, _ptr(status),
                                          _stream(stream)))


def bucket_profile(S, l, buckets, members, cap_members, B, n_dev, profile, stream=None):
    _check(lib().bucket_profile(C.byref(S.c), l, _ptr(buckets), _ptr(members), cap_members, B,
                                _ptr(n_dev), _ptr(profile), _stream(stream)))


def theta_init(alphabet, l, profile, B, n_dev, bg, beta, theta0, stream=None):
    _check(lib().theta_init(alphabet, l, _ptr(profile), B, _ptr(n_dev), _ptr(bg), beta,
                            _ptr(theta0), _stream(stream)))


def pm_em_workspace(S, l: int, precision: int) -> int:
    return int(lib().pm_em_workspace(C.byref(S.c), l, precision))


def _em_ws(S, l, precision, ws, like):
    """The workspace argument of em_refine / em_autotune: the caller's tensor,
    False for none (tables built inside the EM kernel), or None for a fresh
    one of pm_em_workspace bytes on `like`'s device."""
    if ws is False:
        return None, 0
    if ws is None:
        nbytes = pm_em_workspace(S, l, precision)
        if nbytes == 0:
            return None, 0
        import torch
        ws = torch.empty(nbytes, dtype=torch.uint8, device=like.device)
    return ws, ws.numel() * ws.element_size()


def em_refine(S, l, theta0, bg, B, n_dev, iters, beta, precision, theta_out, J_out, llr_out=None,
              sites_out=None, stream=None, ws=None):
    ws, ws_bytes = _em_ws(S, l, precision, ws, theta0)
    _check(lib().em_refine(C.byref(S.c), l, _ptr(theta0), _ptr(bg), B, _ptr(n_dev), iters, beta,
                           precision, _ptr(theta_out), _ptr(J_out), _ptr(llr_out), _ptr(sites_out),
                           _ptr(ws), ws_bytes, _stream(stream)))


def gibbs_refine(S, l, theta0, bg, B, n_dev, sweeps, beta, seed, theta_out, F_out=None, sites_out=None,
                 stream=None):
    _check(lib().gibbs_refine(C.byref(S.c), l, _ptr(theta0), _ptr(bg), B, _ptr(n_dev), sweeps, beta, seed,
                              _ptr(theta_out), _ptr(F_out), _ptr(sites_out), _stream(stream)))


PM_OOPS, PM_ZOOPS, PM_TCM = 0, 1, 2


def em_refine_model(S, l, model, mix0, theta0, bg, B, n_dev, iters, beta, precision, theta_out, mix_out, J_out,
                    llr_out=None, sites_out=None, stream=None):
    _check(lib().em_refine_model(C.byref(S.c), l, model, mix0, _ptr(theta0), _ptr(bg), B, _ptr(n_dev), iters, beta,
                                 precision, _ptr(theta_out), _ptr(mix_out), _ptr(J_out), _ptr(llr_out),
                                 _ptr(sites_out), _stream(stream)))


def em_autotune(S, l, theta0, bg, B, iters, beta, precision, theta_out, J_out, stream=None, ws=None) -> int:
    ws, ws_bytes = _em_ws(S, l, precision, ws, theta0)
    choice = C.c_int32(0)
    _check(lib().em_autotune(C.byref(S.c), l, _ptr(theta0), _ptr(bg), B, iters, beta, precision, _ptr(theta_out),
                             _ptr(J_out), _ptr(ws), ws_bytes, C.byref(choice), _stream(stream)))
    return choice.value


def em_tuning(l: int, precision: int) -> int:
    v = lib().em_tuning(l, precision)
    if v < 0:
        _check(v)
    return v


def em_set_tuning(l: int, precision: int, shape: int) -> None:
    _check(lib().em_set_tuning(l, precision, shape))


def em_best(J, B, n_dev, iters, theta, alphabet, l, best_out, consensus_out=None, stream=None):
    _check(lib().em_best(_ptr(J), B, _ptr(n_dev), iters, _ptr(theta), alphabet, l, _ptr(best_out),
                         _ptr(consensus_out), _stream(stream)))


def pm_batch_check(B: "Batch"):
    _check(lib().pm_batch_check(C.byref(B.c)))


def projection_hash_batch(B: "Batch", masks, keys=None, counts=None, status=None, stream=None):
    _check(lib().projection_hash_batch(C.byref(B.c), _ptr(masks), _ptr(keys), _ptr(counts), _ptr(status),
                                       _stream(stream)))


def bucket_select_batch(B, keys, counts, s, buckets, cap_buckets, members, cap_members, n_out, ws,
                        ws_bytes, status=None, stream=None):
    _check(lib().bucket_select_batch(C.byref(B.c), _ptr(keys), _ptr(counts), s, _ptr(buckets), cap_buckets,
                                     _ptr(members), cap_members, _ptr(n_out), _ptr(ws), ws_bytes,
                                     _ptr(status), _stream(stream)))


def projection_hash_select_batch(B, masks, keys, counts, s, buckets, cap_buckets, members, cap_members, n_out,
                                 ws, ws_bytes, status=None, stream=None):
    _check(lib().projection_hash_select_batch(C.byref(B.c), _ptr(masks), _ptr(keys), _ptr(counts), s,
                                              _ptr(buckets), cap_buckets, _ptr(members), cap_members,
                                              _ptr(n_out), _ptr(ws), ws_bytes, _ptr(status), _stream(stream)))


def bucket_profile_batch(B, buckets, members, cap_members, Bcap, n_dev, profile, stream=None):
    _check(lib().bucket_profile_batch(C.byref(B.c), _ptr(buckets), _ptr(members), cap_members, Bcap,
                                      _ptr(n_dev), _ptr(profile), _stream(stream)))


def pm_em_batch_workspace(B, precision: int) -> int:
    return int(lib().pm_em_batch_workspace(C.byref(B.c), precision))


def em_refine_batch(B, buckets, theta0, bg, Bcap, n_dev, iters, beta, precision, theta_out, J_out,
                    llr_out=None, sites_out=None, ws=None, ws_bytes=0, stream=None):
    _check(lib().em_refine_batch(C.byref(B.c), _ptr(buckets), _ptr(theta0), _ptr(bg), Bcap, _ptr(n_dev),
                                 iters, beta, precision, _ptr(theta_out), _ptr(J_out), _ptr(llr_out),
                                 _ptr(sites_out), _ptr(ws), ws_bytes, _stream(stream)))


def em_best_batch(B, buckets, J, Bcap, n_dev, iters, theta, best_out, consensus_out=None, stream=None):
    _check(lib().em_best_batch(C.byref(B.c), _ptr(buckets), _ptr(J), Bcap, _ptr(n_dev), iters, _ptr(theta),
                               _ptr(best_out), _ptr(consensus_out), _stream(stream)))


def _batch_ptr(B):
    return None if B is None else C.addressof(B.c)


def triage_features(l, profile, B, n_dev, bg, mu, sd, feat, stream=None):
    _check(lib().triage_features(l, _ptr(profile), B, _ptr(n_dev), _ptr(bg), _ptr(mu), _ptr(sd), _ptr(feat),
                                 _stream(stream)))


def pm_triage_packed_bytes() -> int:
    return int(lib().pm_triage_packed_bytes())


def triage_pack(params, packed, stream=None):
    _check(lib().triage_pack(_ptr(params), _ptr(packed), _stream(stream)))


def triage_forward(packed, feat, B, n_dev, score, stream=None):
    _check(lib().triage_forward(_ptr(packed), _ptr(feat), B, _ptr(n_dev), _ptr(score), _stream(stream)))


def pm_triage_workspace(N: int) -> int:
    return int(lib().pm_triage_workspace(N))


def triage_train_step(params, adam_m, adam_v, step, X, target, N, lr, loss_out=None, grads_out=None, ws=None,
                      ws_bytes=0, stream=None):
    _check(lib().triage_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), step, _ptr(X), _ptr(target), N, lr,
                                   _ptr(loss_out), _ptr(grads_out), _ptr(ws), ws_bytes, _stream(stream)))


def pm_triage_select_workspace(P: int, B: int) -> int:
    return int(lib().pm_triage_select_workspace(P, B))


def triage_select(Bt, buckets, score, B, n_dev, frac, theta0, alphabet, l, taken, sel_buckets, sel_theta0,
                  sel_index, n_sel, ws, ws_bytes, stream=None):
    _check(lib().triage_select(_batch_ptr(Bt), _ptr(buckets), _ptr(score), B, _ptr(n_dev), frac, _ptr(theta0),
                               alphabet, l, _ptr(taken), _ptr(sel_buckets), _ptr(sel_theta0), _ptr(sel_index),
                               _ptr(n_sel), _ptr(ws), ws_bytes, _stream(stream)))


def triage_fallback_select(Bt, buckets, B, n_dev, sel1, n_sel1, best, J, iters, threshold, theta0, alphabet, l,
                           taken, sel_buckets, sel_theta0, sel_index, n_sel, fell_back, z_out, ws, ws_bytes,
                           stream=None):
    _check(lib().triage_fallback_select(_batch_ptr(Bt), _ptr(buckets), B, _ptr(n_dev), _ptr(sel1), _ptr(n_sel1),
                                        _ptr(best), _ptr(J), iters, threshold, _ptr(theta0), alphabet, l, _ptr(taken),
                                        _ptr(sel_buckets), _ptr(sel_theta0), _ptr(sel_index), _ptr(n_sel),
                                        _ptr(fell_back), _ptr(z_out), _ptr(ws), ws_bytes, _stream(stream)))


def triage_merge_best(P, alphabet, l, iters, best1, index1, J1, theta1, best2, index2, J2, theta2, best_out,
                      consensus_out=None, stream=None):
    _check(lib().triage_merge_best(P, alphabet, l, iters, _ptr(best1), _ptr(index1), _ptr(J1), _ptr(theta1),
                                   _ptr(best2), _ptr(index2), _ptr(J2), _ptr(theta2), _ptr(best_out),
                                   _ptr(consensus_out), _stream(stream)))


@dataclass
class Problem:
    """One motif-finding problem (Alg. 2 INPUT): sequences, alphabet, l, d;
    k, s, m <= 0 are chosen by pm_auto_params; masks None are drawn from seed;
    bg None is the input composition."""
    seqs: Sequence[str]
    alphabet: int
    l: int
    d: int = 0
    k: int = 0
    s: int = 0
    m: int = 0
    masks: object = None
    seed: int = 0
    bg: object = None


def _fill_problem(pr, P, keep):
    import numpy as np
    t = len(pr.seqs)
    raw = [x.encode("ascii") for x in pr.seqs]
    arr = (C.c_char_p * t)(*raw)
    ns = (C.c_int32 * t)(*[len(x) for x in raw])
    keep += [raw, arr, ns]
    P.alphabet, P.t, P.seqs, P.n = pr.alphabet, t, C.cast(arr, C.POINTER(C.c_char_p)), ns
    P.l, P.d, P.k, P.s, P.m, P.seed = pr.l, pr.d, pr.k, pr.s, pr.m, pr.seed
    if pr.masks is not None:
        mk = np.ascontiguousarray(pr.masks, dtype=np.uint32)
        keep.append(mk)
        P.masks = mk.ctypes.data_as(C.POINTER(C.c_uint32))
        P.m = len(mk)
    if pr.bg is not None:
        bgv = np.ascontiguousarray(pr.bg, dtype=np.float64)
        keep.append(bgv)
        P.bg = bgv.ctypes.data_as(C.POINTER(C.c_double))


def _result_buffers(R, A, t, l):
    import numpy as np
    cons = C.create_string_buffer(l + 1)
    sites = np.zeros(t, dtype=np.int32)
    theta = np.zeros((A, l), dtype=np.float64)
    R.consensus = C.cast(cons, C.c_char_p)
    R.sites = sites.ctypes.data_as(C.POINTER(C.c_int32))
    R.theta = theta.ctypes.data_as(C.POINTER(C.c_double))
    return cons, sites, theta


def _options(em_iters, beta, precision, batched, triage, triage_frac, triage_weights, stream):
    O = pm_options()
    O.em_iters, O.beta, O.precision = em_iters, beta, precision
    O.batched, O.triage, O.triage_frac = int(bool(batched)), int(bool(triage)), triage_frac
    if triage:
        path = triage_weights or default_triage_bin_path()
        O.triage_weights = path.encode()
    O.stream = _stream(stream) if stream is not None else None
    return O


def _results(Rs, outs):
    res = []
    for R, (cons, sites, theta) in zip(Rs, outs):
        res.append(dict(consensus=cons.value.decode(), sites=sites, theta=theta, J=R.J, llr=R.llr,
                        best_trial=R.best_trial, best_key=R.best_key, n_enriched=R.n_enriched,
                        n_refined=R.n_refined, fallback_used=bool(R.fallback_used), k=R.k, s=R.s, m=R.m))
    return res


def projection_run(problems, em_iters: int = 5, beta: float = 1.0, precision: int = PM_FP64,
                   batched: bool = False, triage: bool = False, triage_frac: float = 0.05,
                   triage_weights: Optional[str] = None, stream=None) -> list:
    """Host in, host out: the whole path on every problem (synchronous).
    `problems` is a Problem or a list of them; returns one dict per problem.
    triage_weights defaults to the shipped weights file when triage is on."""
    if isinstance(problems, Problem):
        problems = [problems]
    n = len(problems)
    keep = []  # buffers the C structures point into
    Ps = (pm_problem * n)()
    Rs = (pm_result * n)()
    outs = []
    for pr, P, R in zip(problems, Ps, Rs):
        _fill_problem(pr, P, keep)
        outs.append(_result_buffers(R, pr.alphabet, len(pr.seqs), pr.l))
    O = _options(em_iters, beta, precision, batched, triage, triage_frac, triage_weights, stream)
    _check(lib().projection_run(Ps, n, C.byref(O), Rs))
    return _results(Rs, outs)


def projection_run_range(problem, l_minus: int, l_plus: int, em_iters: int = 5, beta: float = 1.0,
                         precision: int = PM_FP64, batched: bool = False, triage: bool = False,
                         triage_frac: float = 0.05, triage_weights: Optional[str] = None, stream=None):
    """One problem at every motif length l_minus..l_plus (problem.l is
    ignored): (one dict per length, the chosen length or -1)."""
    keep = []
    P = pm_problem()
    _fill_problem(problem, P, keep)
    n = l_plus - l_minus + 1
    Rs = (pm_result * max(n, 1))()
    outs = [_result_buffers(R, problem.alphabet, len(problem.seqs), l_minus + q) for q, R in enumerate(Rs)]
    O = _options(em_iters, beta, precision, batched, triage, triage_frac, triage_weights, stream)
    chosen = C.c_int32(-1)
    _check(lib().projection_run_range(C.byref(P), l_minus, l_plus, C.byref(O), Rs, C.byref(chosen)))
    return _results(Rs, outs), chosen.value


# ----------------------------------------------------------------- device data
class Seqs:
    """Sequences resident on the GPU: ASCII staged, then packed by pm_pack."""

    def __init__(self, alphabet: int, seqs: Sequence[str], device="cuda", stream=None):
        import numpy as np
        import torch
        self.alphabet = alphabet
        self.t = len(seqs)
        lens = [len(x) for x in seqs]
        self.lens = lens
        raw = np.frombuffer("".join(seqs).encode("ascii"), dtype=np.uint8)
        off = np.zeros(self.t + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        self.n_total = int(off[-1])
        self.ascii = torch.from_numpy(raw.copy()).to(device)
        self.offsets = torch.from_numpy(off).to(device)
        self.packed = torch.zeros(pm_packed_words(alphabet, self.n_total), dtype=torch.int32,
                                  device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        pm_pack(alphabet, self.ascii, self.n_total, self.packed, self.status, stream)
        self.c = pm_seqs(alphabet, self.t, self.n_total, min(lens), max(lens),
                         self.offsets.data_ptr(), self.packed.data_ptr())

    def nwin(self, l: int) -> int:
        return self.n_total - self.t * (l - 1)

    def check_status(self):
        v = int(self.status.item())
        if v & PM_STATUS_BAD_SYMBOL:
            raise PmError(PM_EINVAL, "a sequence holds a symbol outside the alphabet")


def code_order(alphabet: int) -> str:
    return DNA_CODE_ORDER if alphabet == 4 else PROTEIN_CODE_ORDER


@dataclass
class PassBuffers:
    """Device buffers of one pass of the path (hash -> select -> EM -> best)."""
    keys: object
    counts: object
    status: object
    n_out: object
    buckets: object
    members: object
    ws: object
    profile: object
    theta0: object
    theta: object
    J: object
    llr: object
    sites: object
    best: object
    consensus: object
    cap_b: int
    cap_m: int


class Pipeline:
    """One instance, one fixed shape: allocate once, then run whole passes
    on a stream with no host synchronisation inside a pass."""

    def __init__(self, S: Seqs, l: int, k: int, s: int, masks, iters: int, beta: float,
                 precision: int, bg, cap_b: int, cap_m: int, device="cuda"):
        import numpy as np
        import torch
        self.S, self.l, self.k, self.s, self.iters, self.beta = S, l, k, s, iters, beta
        self.precision = precision
        A = S.alphabet
        self.m = len(masks)
        self.x = S.nwin(l)
        self.nb = A ** k
        dev = device
        self.masks = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).to(dev)
        self.bg = torch.as_tensor(np.asarray(bg, dtype=np.float64), device=dev)
        ws_bytes = pm_select_workspace(A, k, self.m, cap_b)
        AL = A * l
        z = lambda *shape, dt=torch.int32: torch.zeros(*shape, dtype=dt, device=dev)
        self.b = PassBuffers(
            keys=z(self.m, self.x), counts=z(self.m, self.nb), status=z(1), n_out=z(2, dt=torch.int64),
            buckets=z(max(cap_b, 1), 4), members=z(max(cap_m, 1)), ws=z((ws_bytes + 3) // 4),
            profile=z(max(cap_b, 1), A, l), theta0=z(max(cap_b, 1), A, l, dt=torch.float64),
            theta=z(max(cap_b, 1), A, l, dt=torch.float64), J=z(max(cap_b, 1), iters + 1, dt=torch.float64),
            llr=z(max(cap_b, 1), iters + 1, dt=torch.float64), sites=z(max(cap_b, 1), S.t),
            best=z(1, dt=torch.int64), consensus=torch.zeros(l + 1, dtype=torch.uint8, device=dev),
            cap_b=cap_b, cap_m=cap_m)
        self.ws_bytes = ws_bytes
        # one-hot tables of the matrix-core EM (empty for the other forms)
        self.em_ws = torch.empty(max(pm_em_workspace(S, l, precision), 1), dtype=torch.uint8, device=dev)

    def hash(self, stream=None):
        b = self.b
        projection_hash(self.S, self.l, self.k, self.masks, self.m, b.keys, b.counts, b.status, stream)

    def select(self, stream=None):
        b = self.b
        bucket_select(self.S, self.l, self.k, b.keys, b.counts, self.m, self.s, b.buckets, b.cap_b,
                      b.members, b.cap_m, b.n_out, b.ws, self.ws_bytes, b.status, stream)

    def hash_select(self, stream=None):
        """hash() then select() in one call (the same outputs): the hash pass
        also forms the selection's bitmap and totals."""
        b = self.b
        projection_hash_select(self.S, self.l, self.k, self.masks, self.m, b.keys, b.counts, self.s, b.buckets,
                               b.cap_b, b.members, b.cap_m, b.n_out, b.ws, self.ws_bytes, b.status, stream)

    def refine(self, stream=None):
        b, A = self.b, self.S.alphabet
        bucket_profile(self.S, self.l, b.buckets, b.members, b.cap_m, b.cap_b, b.n_out, b.profile, stream)
        theta_init(A, self.l, b.profile, b.cap_b, b.n_out, self.bg, self.beta, b.theta0, stream)
        em_refine(self.S, self.l, b.theta0, self.bg, b.cap_b, b.n_out, self.iters, self.beta,
                  self.precision, b.theta, b.J, b.llr, b.sites, stream, ws=self.em_ws)
        em_best(b.J, b.cap_b, b.n_out, self.iters, b.theta, A, self.l, b.best, b.consensus, stream)

    def run(self, stream=None):
        self.hash_select(stream)
        self.refine(stream)

    def result(self) -> dict:
        """Copy the answer back (synchronises)."""
        b = self.b
        nb_, nm_ = [int(v) for v in b.n_out.cpu()]
        st = int(b.status.item())
        best = int(b.best.item())
        out = dict(n_buckets=nb_, n_members=nm_, status=st, best=best)
        if best >= 0:
            out["consensus"] = bytes(b.consensus.cpu().numpy()[: self.l]).decode()
            out["sites"] = b.sites[best].cpu().numpy()
            out["J"] = float(b.J[best, -1].item())
            out["bucket"] = b.buckets[best].cpu().numpy().view("uint32")
        return out


# ----------------------------------------------------------------- batches
class Batch:
    """Many instances of one shape class (alphabet, l, k) on the GPU.

    Every instance's ASCII is padded with code-0 letters to a whole number of
    packed words plus the four padding words pm_pack appends, so one pm_pack
    over the concatenation gives each instance its own aligned, zero-padded
    packed region; offsets are per instance (local symbol numbers)."""

    def __init__(self, alphabet: int, l: int, k: int, instances: Sequence[Sequence[str]], masks,
                 device="cuda", stream=None):
        import numpy as np
        import torch
        self.alphabet, self.l, self.k = alphabet, l, k
        self.P = len(instances)
        per = 16 if alphabet == 4 else 6
        masks = [np.ascontiguousarray(mk, dtype=np.uint32) for mk in masks]
        if len(masks) != self.P:
            raise ValueError("one mask table per instance")
        chunks, offs, word_base, off_base = [], [], [], []
        wb = ob = 0
        self.t, self.x, self.n_total, self.m = [], [], [], []
        for seqs, mk in zip(instances, masks):
            lens = [len(q) for q in seqs]
            n = sum(lens)
            nw = pm_packed_words(alphabet, n)
            chunks.append("".join(seqs) + "A" * (nw * per - n))
            o = np.zeros(len(seqs) + 1, dtype=np.int64)
            o[1:] = np.cumsum(lens)
            offs.append(o)
            word_base.append(wb)
            off_base.append(ob)
            wb += nw
            ob += len(seqs) + 1
            self.t.append(len(seqs))
            self.n_total.append(n)
            self.x.append(n - len(seqs) * (l - 1))
            self.m.append(len(mk))
        self.n_min = [min(len(q) for q in seqs) for seqs in instances]
        raw = np.frombuffer("".join(chunks).encode("ascii"), dtype=np.uint8)
        self.ascii = torch.from_numpy(raw.copy()).to(device)
        self.packed = torch.zeros(pm_packed_words(alphabet, len(raw)), dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        pm_pack(alphabet, self.ascii, len(raw), self.packed, self.status, stream)
        self.offsets = torch.from_numpy(np.concatenate(offs)).to(device)
        self.items = int(sum(self.m))
        self.masks = torch.from_numpy(np.concatenate(masks).view(np.int32)).to(device)
        first, key = 0, 0
        tab = (pm_inst * self.P)()
        item_inst = np.zeros(self.items, dtype=np.int32)
        self.first_item, self.key_base = [], []
        for p in range(self.P):
            e = tab[p]
            e.offsets = self.offsets.data_ptr() + 8 * off_base[p]
            e.packed = self.packed.data_ptr() + 4 * word_base[p]
            e.n_total, e.x, e.key_base = self.n_total[p], self.x[p], key
            e.t, e.n_min, e.m, e.first_item = self.t[p], self.n_min[p], self.m[p], first
            item_inst[first:first + self.m[p]] = p
            self.first_item.append(first)
            self.key_base.append(key)
            first += self.m[p]
            key += self.m[p] * self.x[p]
        self.keys_total = key
        self.tab_host = tab
        self.tab = torch.frombuffer(bytearray(bytes(tab)), dtype=torch.uint8).to(device)
        self.item_inst = torch.from_numpy(item_inst).to(device)
        self.c = pm_batch(alphabet, l, k, self.P, self.items, self.tab.data_ptr(),
                          C.cast(tab, C.c_void_p), self.item_inst.data_ptr())
        pm_batch_check(self)

    @property
    def t_max(self) -> int:
        return max(self.t)


class BatchPipeline:
    """All instances of a Batch through the whole path in one set of launches
    per step (hash, select, profiles, theta^0, EM, per-instance best), with
    fixed buffers, so the pass can be captured in a HIP graph."""

    def __init__(self, B: Batch, s: int, iters: int, beta: float, precision: int, bg, cap_b: int,
                 cap_m: int, device="cuda"):
        import numpy as np
        import torch
        self.B, self.s, self.iters, self.beta, self.precision = B, s, iters, beta, precision
        A, l = B.alphabet, B.l
        self.nb = A ** B.k
        dev = device
        self.bg = torch.as_tensor(np.asarray(bg, dtype=np.float64), device=dev)
        self.ws_bytes = pm_select_workspace(A, B.k, B.items, cap_b)
        self.em_ws_bytes = pm_em_batch_workspace(B, precision)
        cb = max(cap_b, 1)
        z = lambda *shape, dt=torch.int32: torch.zeros(*shape, dtype=dt, device=dev)
        self.b = PassBuffers(
            keys=z(B.keys_total), counts=z(B.items, self.nb), status=z(1), n_out=z(2, dt=torch.int64),
            buckets=z(cb, 4), members=z(max(cap_m, 1)), ws=z((self.ws_bytes + 3) // 4),
            profile=z(cb, A, l), theta0=z(cb, A, l, dt=torch.float64), theta=z(cb, A, l, dt=torch.float64),
            J=z(cb, iters + 1, dt=torch.float64), llr=z(cb, iters + 1, dt=torch.float64),
            sites=z(cb, B.t_max), best=z(B.P, dt=torch.int64),
            consensus=torch.zeros(B.P, l + 1, dtype=torch.uint8, device=dev), cap_b=cap_b, cap_m=cap_m)
        self.em_ws = z((self.em_ws_bytes + 3) // 4)

    def hash(self, stream=None):
        b = self.b
        projection_hash_batch(self.B, self.B.masks, b.keys, b.counts, b.status, stream)

    def select(self, stream=None):
        b = self.b
        bucket_select_batch(self.B, b.keys, b.counts, self.s, b.buckets, b.cap_b, b.members, b.cap_m,
                            b.n_out, b.ws, self.ws_bytes, b.status, stream)

    def hash_select(self, stream=None):
        """hash() then select() in one call (the same outputs)."""
        b = self.b
        projection_hash_select_batch(self.B, self.B.masks, b.keys, b.counts, self.s, b.buckets, b.cap_b,
                                     b.members, b.cap_m, b.n_out, b.ws, self.ws_bytes, b.status, stream)

    def profile(self, stream=None):
        b = self.b
        bucket_profile_batch(self.B, b.buckets, b.members, b.cap_m, b.cap_b, b.n_out, b.profile, stream)
        theta_init(self.B.alphabet, self.B.l, b.profile, b.cap_b, b.n_out, self.bg, self.beta, b.theta0,
                   stream)

    def refine(self, stream=None):
        b = self.b
        em_refine_batch(self.B, b.buckets, b.theta0, self.bg, b.cap_b, b.n_out, self.iters, self.beta,
                        self.precision, b.theta, b.J, b.llr, b.sites, self.em_ws, self.em_ws_bytes, stream)

    def best(self, stream=None):
        b = self.b
        em_best_batch(self.B, b.buckets, b.J, b.cap_b, b.n_out, self.iters, b.theta, b.best, b.consensus,
                      stream)

    def run(self, stream=None):
        self.hash_select(stream)
        self.profile(stream)
        self.refine(stream)
        self.best(stream)

    def results(self) -> list:
        """Per-instance answers (synchronises)."""
        b, l = self.b, self.B.l
        best = b.best.cpu().numpy()
        cons = b.consensus.cpu().numpy()
        J = b.J[:, -1].cpu().numpy()
        sites = b.sites.cpu().numpy()
        out = []
        for p in range(self.B.P):
            r = dict(best=int(best[p]))
            if best[p] >= 0:
                r["consensus"] = bytes(cons[p, :l]).decode()
                r["J"] = float(J[best[p]])
                r["sites"] = sites[best[p], : self.B.t[p]].copy()
            out.append(r)
        return out


def size_batch(B: Batch, s: int, device="cuda"):
    """Bucket and member counts of a batch (one hash + select pass with zero
    capacities; synchronises)."""
    P0 = BatchPipeline(B, s, 0, 1.0, PM_FP64, [1.0 / B.alphabet] * B.alphabet, 0, 0, device)
    P0.hash()
    P0.select()
    nb_, nm_ = [int(v) for v in P0.b.n_out.cpu()]
    return nb_, nm_


# ----------------------------------------------------------------- triage
class Triage:
    """A trained triage network on the GPU: FP32 parameters, their packed
    BF16 serving form, the feature standardisation and the fallback
    threshold (best J(theta^iters) per sequence)."""

    def __init__(self, params, mu, sd, threshold: float, device="cuda", meta=None):
        import numpy as np
        import torch
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32), device=device).contiguous()
        assert self.params.numel() == PM_TRIAGE_PARAMS
        self.mu = torch.as_tensor(np.asarray(mu, dtype=np.float32), device=device).contiguous()
        self.sd = torch.as_tensor(np.asarray(sd, dtype=np.float32), device=device).contiguous()
        self.threshold = float(threshold)
        self.meta = dict(meta or {})
        self.packed = torch.zeros(pm_triage_packed_bytes(), dtype=torch.uint8, device=device)
        self.repack()

    def repack(self, stream=None):
        triage_pack(self.params, self.packed, stream)

    @classmethod
    def load(cls, path: str, device="cuda"):
        import json
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            return cls(z["params"], z["mu"], z["sd"], float(z["threshold"]), device, meta)

    def save_bin(self, path: str):
        """The weights in the file format projection_run reads."""
        write_triage_bin(path, self.params.cpu().numpy(), self.mu.cpu().numpy(), self.sd.cpu().numpy(),
                         self.threshold, self.meta.get("thresholds_by_l", {}))

    def save(self, path: str):
        import json
        import numpy as np
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu.cpu().numpy(), sd=self.sd.cpu().numpy(),
                 threshold=np.float64(self.threshold), meta=json.dumps(self.meta))

    def threshold_for(self, l: int) -> float:
        """Fallback threshold (z-score of the triaged winner's objective among
        the refined buckets of its instance) for motif length l: the
        per-length value from training when there is one, else the pooled one."""
        per = self.meta.get("thresholds_by_l", {})
        return float(per.get(str(l), per.get(l, self.threshold)))

    def score(self, l, profile, B, n_dev, bg, feat, score, stream=None):
        triage_features(l, profile, B, n_dev, bg, self.mu, self.sd, feat, stream)
        triage_forward(self.packed, feat, B, n_dev, score, stream)


def default_triage_path() -> str:
    return os.path.join(PKG, "triage_weights.npz")


def write_triage_bin(path: str, params, mu, sd, threshold: float, thresholds_by_l: dict):
    """Triage weights in the format projection_run reads (include/projmotif.h):
    "PMTRIAG1", the sizes, FP32 parameters, mu and sd, the pooled fallback
    threshold and the per-motif-length thresholds."""
    import struct
    import numpy as np
    per = {int(k): float(v) for k, v in thresholds_by_l.items()}
    with open(path, "wb") as f:
        f.write(b"PMTRIAG1")
        f.write(struct.pack("<ii", PM_TRIAGE_PARAMS, PM_TRIAGE_INPUTS))
        for a, n in ((params, PM_TRIAGE_PARAMS), (mu, PM_TRIAGE_INPUTS), (sd, PM_TRIAGE_INPUTS)):
            v = np.ascontiguousarray(a, dtype="<f4").reshape(-1)
            assert v.size == n
            f.write(v.tobytes())
        f.write(struct.pack("<di", float(threshold), len(per)))
        for l in sorted(per):
            f.write(struct.pack("<id", l, per[l]))


def convert_triage_npz(npz_path: str, bin_path: str):
    """The binary weights file of a training output (.npz)."""
    import json
    import numpy as np
    with np.load(npz_path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        write_triage_bin(bin_path, z["params"], z["mu"], z["sd"], float(z["threshold"]),
                         meta.get("thresholds_by_l", {}))


def default_triage_bin_path() -> str:
    """The shipped weights in the file format projection_run reads."""
    return os.path.join(PKG, "triage_weights.bin")


class TriagedBatchPipeline(BatchPipeline):
    """BatchPipeline with learned triage: after theta^0, the network scores
    every bucket, EM refines the top `frac` of each instance, instances whose
    winner is weak fall back to refining all their other buckets, and the
    better winner is kept.  All on device, no host synchronisation."""

    def __init__(self, B: Batch, s: int, iters: int, beta: float, precision: int, bg, cap_b: int, cap_m: int,
                 triage: Triage, frac: float = 0.05, device="cuda"):
        import torch
        super().__init__(B, s, iters, beta, precision, bg, cap_b, cap_m, device)
        self.tri, self.frac = triage, frac
        self.threshold = triage.threshold_for(B.l)
        A, l = B.alphabet, B.l
        cb = max(cap_b, 1)
        z = lambda *shape, dt=torch.int32: torch.zeros(*shape, dtype=dt, device=device)
        self.feat = z(cb, PM_TRIAGE_INPUTS, dt=torch.float32)
        self.score_buf = z(cb, dt=torch.float32)
        self.taken = z(cb, dt=torch.uint8)
        self.sel_ws_bytes = pm_triage_select_workspace(B.P, cb)
        self.sel_ws = z((self.sel_ws_bytes + 7) // 8, dt=torch.int64)
        self.fell_back = z(B.P)
        self.z = z(B.P, dt=torch.float64)
        self.lists = []
        for _ in range(2):
            self.lists.append(dict(
                buckets=z(cb, 4), theta0=z(cb, A, l, dt=torch.float64), index=z(cb, dt=torch.int64),
                n=z(1, dt=torch.int64), theta=z(cb, A, l, dt=torch.float64), J=z(cb, iters + 1, dt=torch.float64),
                llr=z(cb, iters + 1, dt=torch.float64), sites=z(cb, B.t_max), best=z(B.P, dt=torch.int64)))

    def _refine_list(self, L, stream):
        em_refine_batch(self.B, L["buckets"], L["theta0"], self.bg, self.b.cap_b, L["n"], self.iters, self.beta,
                        self.precision, L["theta"], L["J"], L["llr"], L["sites"], self.em_ws, self.em_ws_bytes,
                        stream)
        em_best_batch(self.B, L["buckets"], L["J"], self.b.cap_b, L["n"], self.iters, L["theta"], L["best"], None,
                      stream)

    def score_buckets(self, stream=None):
        """Scores of every bucket into score_buf: the network's (a subclass
        may rank the buckets another way)."""
        b, B = self.b, self.B
        self.tri.score(B.l, b.profile, b.cap_b, b.n_out, self.bg, self.feat, self.score_buf, stream)

    def triage(self, stream=None):
        b, B = self.b, self.B
        self.score_buckets(stream)
        L1, L2 = self.lists
        triage_select(B, b.buckets, self.score_buf, b.cap_b, b.n_out, self.frac, b.theta0, B.alphabet, B.l,
                      self.taken, L1["buckets"], L1["theta0"], L1["index"], L1["n"], self.sel_ws, self.sel_ws_bytes,
                      stream)
        self._refine_list(L1, stream)
        triage_fallback_select(B, b.buckets, b.cap_b, b.n_out, L1["buckets"], L1["n"], L1["best"], L1["J"],
                               self.iters, self.threshold, b.theta0, B.alphabet, B.l, self.taken, L2["buckets"],
                               L2["theta0"], L2["index"], L2["n"], self.fell_back, self.z, self.sel_ws,
                               self.sel_ws_bytes, stream)
        self._refine_list(L2, stream)
        triage_merge_best(B.P, B.alphabet, B.l, self.iters, L1["best"], L1["index"], L1["J"], L1["theta"],
                          L2["best"], L2["index"], L2["J"], L2["theta"], b.best, b.consensus, stream)

    def run(self, stream=None):
        self.hash_select(stream)
        self.profile(stream)
        self.triage(stream)

    def results(self) -> list:
        """Per-instance answers (synchronises); sites from the list that won."""
        import numpy as np
        b, l = self.b, self.B.l
        best = b.best.cpu().numpy()
        cons = b.consensus.cpu().numpy()
        L1, L2 = self.lists
        i1, i2 = L1["index"].cpu().numpy(), L2["index"].cpu().numpy()
        bb1, bb2 = L1["best"].cpu().numpy(), L2["best"].cpu().numpy()
        fb = self.fell_back.cpu().numpy()
        zz = self.z.cpu().numpy()
        n1, n2 = int(L1["n"].item()), int(L2["n"].item())
        out = []
        for p in range(self.B.P):
            r = dict(best=int(best[p]), fell_back=bool(fb[p]), z=float(zz[p]))
            if best[p] >= 0:
                r["consensus"] = bytes(cons[p, :l]).decode()
                if bb1[p] >= 0 and i1[bb1[p]] == best[p]:
                    L, w = L1, bb1[p]
                else:
                    L, w = L2, bb2[p]
                r["J"] = float(L["J"][w, -1].item())
                r["sites"] = L["sites"][w, : self.B.t[p]].cpu().numpy()
            out.append(r)
        self.refined = n1 + n2
        return out
