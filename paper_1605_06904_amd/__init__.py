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
PM_FP64, PM_FP32, PM_F16X2 = 0, 1, 2

DNA_CODE_ORDER = "ACTG"
PROTEIN_CODE_ORDER = "ARNDCQEGHILKMFPSTWYV"

EXPORTS = [
    "pm_version", "pm_last_error", "pm_packed_words", "pm_pack", "pm_masks_from_seed",
    "pm_auto_params", "projection_hash", "pm_select_workspace", "bucket_select",
    "bucket_profile", "theta_init", "em_refine", "em_best", "projection_run",
]


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


class pm_problem(C.Structure):
    _fields_ = [("alphabet", C.c_int32), ("t", C.c_int32), ("seqs", C.POINTER(C.c_char_p)),
                ("n", C.POINTER(C.c_int32)), ("l", C.c_int32), ("d", C.c_int32),
                ("k", C.c_int32), ("s", C.c_int32), ("m", C.c_int32),
                ("masks", C.POINTER(C.c_uint32)), ("seed", C.c_uint64),
                ("bg", C.POINTER(C.c_double))]


class pm_options(C.Structure):
    _fields_ = [("em_iters", C.c_int32), ("beta", C.c_double), ("precision", C.c_int32),
                ("stream", C.c_void_p)]


class pm_result(C.Structure):
    _fields_ = [("consensus", C.c_char_p), ("sites", C.POINTER(C.c_int32)),
                ("theta", C.POINTER(C.c_double)), ("J", C.c_double), ("llr", C.c_double),
                ("best_trial", C.c_int32), ("best_key", C.c_uint32), ("n_enriched", C.c_int64),
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
        "pm_select_workspace": (sz, [i32, i64]),
        "bucket_select": (C.c_int, [C.POINTER(pm_seqs), i32, i32, P, P, i32, u32, P, i64, P, i64,
                                    P, P, sz, P, P]),
        "bucket_profile": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, i64, P, P, P]),
        "theta_init": (C.c_int, [i32, i32, P, i64, P, P, dbl, P, P]),
        "em_refine": (C.c_int, [C.POINTER(pm_seqs), i32, P, P, i64, P, i32, dbl, i32, P, P, P,
                                P, P]),
        "em_best": (C.c_int, [P, i64, P, i32, P, i32, i32, P, P, P]),
        "projection_run": (C.c_int, [C.POINTER(pm_problem), C.POINTER(pm_options),
                                     C.POINTER(pm_result)]),
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


def pm_select_workspace(m: int, cap_buckets: int) -> int:
    return int(lib().pm_select_workspace(m, cap_buckets))


def bucket_select(S, l, k, keys, counts, m, s, buckets, cap_buckets, members, cap_members, n_out,
                  ws, ws_bytes, status=None, stream=None):
    _check(lib().bucket_select(C.byref(S.c), l, k, _ptr(keys), _ptr(counts), m, s, _ptr(buckets),
                               cap_buckets, _ptr(members), cap_members, _ptr(n_out), _ptr(ws),
                               ws_bytes, _ptr(status), _stream(stream)))


def bucket_profile(S, l, buckets, members, cap_members, B, n_dev, profile, stream=None):
    _check(lib().bucket_profile(C.byref(S.c), l, _ptr(buckets), _ptr(members), cap_members, B,
                                _ptr(n_dev), _ptr(profile), _stream(stream)))


def theta_init(alphabet, l, profile, B, n_dev, bg, beta, theta0, stream=None):
    _check(lib().theta_init(alphabet, l, _ptr(profile), B, _ptr(n_dev), _ptr(bg), beta,
                            _ptr(theta0), _stream(stream)))


def em_refine(S, l, theta0, bg, B, n_dev, iters, beta, precision, theta_out, J_out, llr_out=None,
              sites_out=None, stream=None):
    _check(lib().em_refine(C.byref(S.c), l, _ptr(theta0), _ptr(bg), B, _ptr(n_dev), iters, beta,
                           precision, _ptr(theta_out), _ptr(J_out), _ptr(llr_out), _ptr(sites_out),
                           _stream(stream)))


def em_best(J, B, n_dev, iters, theta, alphabet, l, best_out, consensus_out=None, stream=None):
    _check(lib().em_best(_ptr(J), B, _ptr(n_dev), iters, _ptr(theta), alphabet, l, _ptr(best_out),
                         _ptr(consensus_out), _stream(stream)))


def projection_run(seqs: Sequence[str], alphabet: int, l: int, d: int = 0, k: int = 0, s: int = 0,
                   m: int = 0, masks=None, seed: int = 0, bg=None, em_iters: int = 5,
                   beta: float = 1.0, precision: int = PM_FP64, stream=None) -> dict:
    """Host in, host out: the whole path on one instance (synchronous)."""
    import numpy as np
    t = len(seqs)
    raw = [x.encode("ascii") for x in seqs]
    arr = (C.c_char_p * t)(*raw)
    ns = (C.c_int32 * t)(*[len(x) for x in raw])
    P = pm_problem()
    P.alphabet, P.t, P.seqs, P.n = alphabet, t, C.cast(arr, C.POINTER(C.c_char_p)), ns
    P.l, P.d, P.k, P.s, P.m, P.seed = l, d, k, s, m, seed
    mk = None
    if masks is not None:
        mk = np.ascontiguousarray(masks, dtype=np.uint32)
        P.masks = mk.ctypes.data_as(C.POINTER(C.c_uint32))
        P.m = len(mk)
    bgv = None
    if bg is not None:
        bgv = np.ascontiguousarray(bg, dtype=np.float64)
        P.bg = bgv.ctypes.data_as(C.POINTER(C.c_double))
    O = pm_options()
    O.em_iters, O.beta, O.precision = em_iters, beta, precision
    O.stream = _stream(stream) if stream is not None else None
    cons = C.create_string_buffer(l + 1)
    sites = np.zeros(t, dtype=np.int32)
    theta = np.zeros((alphabet, l), dtype=np.float64)
    R = pm_result()
    R.consensus = C.cast(cons, C.c_char_p)
    R.sites = sites.ctypes.data_as(C.POINTER(C.c_int32))
    R.theta = theta.ctypes.data_as(C.POINTER(C.c_double))
    _check(lib().projection_run(C.byref(P), C.byref(O), C.byref(R)))
    return dict(consensus=cons.value.decode(), sites=sites, theta=theta, J=R.J, llr=R.llr,
                best_trial=R.best_trial, best_key=R.best_key, n_enriched=R.n_enriched,
                k=R.k, s=R.s, m=R.m)


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
        ws_bytes = pm_select_workspace(self.m, cap_b)
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

    def hash(self, stream=None):
        b = self.b
        projection_hash(self.S, self.l, self.k, self.masks, self.m, b.keys, b.counts, b.status, stream)

    def select(self, stream=None):
        b = self.b
        bucket_select(self.S, self.l, self.k, b.keys, b.counts, self.m, self.s, b.buckets, b.cap_b,
                      b.members, b.cap_m, b.n_out, b.ws, self.ws_bytes, b.status, stream)

    def refine(self, stream=None):
        b, A = self.b, self.S.alphabet
        bucket_profile(self.S, self.l, b.buckets, b.members, b.cap_m, b.cap_b, b.n_out, b.profile, stream)
        theta_init(A, self.l, b.profile, b.cap_b, b.n_out, self.bg, self.beta, b.theta0, stream)
        em_refine(self.S, self.l, b.theta0, self.bg, b.cap_b, b.n_out, self.iters, self.beta,
                  self.precision, b.theta, b.J, b.llr, b.sites, stream)
        em_best(b.J, b.cap_b, b.n_out, self.iters, b.theta, A, self.l, b.best, b.consensus, stream)

    def run(self, stream=None):
        self.hash(stream)
        self.select(stream)
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
