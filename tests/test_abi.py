"""The C-ABI library: it loads, exports every declared entry point, and its
host-side helpers and argument checks behave -- all without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "projmotif.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\([^;]*\)\s*;", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 14
    L = C.CDLL(pm.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pm.EXPORTS) == names


def test_version_and_error_string():
    assert "gfx950" in pm.pm_version()
    assert pm.pm_last_error() == ""


def test_packed_words():
    assert pm.pm_packed_words(4, 0) == 4
    assert pm.pm_packed_words(4, 16) == 5
    assert pm.pm_packed_words(4, 17) == 6
    assert pm.pm_packed_words(20, 6) == 5
    assert pm.pm_packed_words(20, 7) == 6
    assert pm.pm_packed_words(5, 7) == -1


@pytest.mark.parametrize("seed,l,k,m", [(1, 15, 7, 50), (99, 18, 8, 20), (5, 32, 9, 10), (0, 4, 4, 3)])
def test_seeded_masks_match_oracle(seed, l, k, m):
    """Both sides implement the Park-Miller generator from its definition."""
    assert np.array_equal(pm.pm_masks_from_seed(seed, l, k, m), oracle.masks_from_seed(seed, l, k, m))


@pytest.mark.parametrize("A,t,n,l,d", [(4, 20, 600, 15, 4), (4, 20, 1000, 18, 6), (20, 30, 1000, 20, 6),
                                       (4, 50, 2000, 21, 7), (4, 20, 600, 8, 1)])
def test_auto_params_match_oracle(A, t, n, l, d):
    x = t * (n - l + 1)
    assert pm.pm_auto_params(A, t, x, l, d) == oracle.auto_params(l, d, t, x, A)


def test_auto_params_rejects_unreachable_threshold():
    with pytest.raises(pm.PmError):
        pm.pm_auto_params(4, 20, 20 * 593, 8, 2)


def _fake_seqs(**kw):
    f = dict(alphabet=4, t=2, n_total=20, n_min=10, n_max=10, offsets=0x1000, packed=0x2000)
    f.update(kw)
    return pm.pm_seqs(**f)


class _S:
    def __init__(self, c):
        self.c = c


@pytest.mark.parametrize("kw,l,k", [
    (dict(alphabet=5), 4, 2),       # bad alphabet
    (dict(t=0), 4, 2),              # no sequences
    (dict(n_min=3), 4, 2),          # a sequence shorter than l
    ({}, 33, 2),                    # l too large
    ({}, 4, 5),                     # k > l
    ({}, 4, 0),                     # k < 1
    (dict(n_total=25), 4, 2),       # inconsistent lengths
    (dict(offsets=0), 4, 2),        # NULL offsets
])
def test_projection_hash_rejects_bad_arguments_before_any_launch(kw, l, k):
    S = _S(_fake_seqs(**kw))
    rc = pm.lib().projection_hash(C.byref(S.c), l, k, 0x3000, 4, 0x4000, 0x5000, None, None)
    assert rc == pm.PM_EINVAL
    assert pm.pm_last_error()


def test_projection_hash_range_errors():
    S = _S(_fake_seqs(n_total=40, n_min=20, n_max=20))
    # DNA keys must fit 32 bits; protein k <= 7
    assert pm.lib().projection_hash(C.byref(S.c), 20, 17, 0x3000, 1, 0x4000, None, None, None) == pm.PM_ERANGE
    # counts beyond 2^24 bins
    assert pm.lib().projection_hash(C.byref(S.c), 20, 13, 0x3000, 1, None, 0x5000, None, None) == pm.PM_ERANGE
    S2 = _S(_fake_seqs(alphabet=20, n_total=40, n_min=20, n_max=20))
    assert pm.lib().projection_hash(C.byref(S2.c), 20, 8, 0x3000, 1, 0x4000, None, None, None) == pm.PM_ERANGE


def test_other_entry_points_validate():
    S = _S(_fake_seqs())
    L = pm.lib()
    # keys/counts missing
    assert L.bucket_select(C.byref(S.c), 4, 2, None, 0x1, 1, 2, 0x1, 1, 0x1, 1, 0x1, 0x1, 1 << 20,
                           None, None) == pm.PM_EINVAL
    # workspace too small
    assert L.bucket_select(C.byref(S.c), 4, 2, 0x1, 0x1, 1, 2, 0x1, 1, 0x1, 1, 0x1, 0x1, 8,
                           None, None) == pm.PM_EINVAL
    # hash + selection in one call: keys and counts both required, the
    # selection's workspace and |Sigma|^k limit
    ws = pm.pm_select_workspace(4, 2, 1, 1)
    assert L.projection_hash_select(C.byref(S.c), 4, 2, 0x3000, 1, None, 0x5000, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1000, ws, None, None) == pm.PM_EINVAL
    assert L.projection_hash_select(C.byref(S.c), 4, 2, 0x3000, 1, 0x4000, None, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1000, ws, None, None) == pm.PM_EINVAL
    assert L.projection_hash_select(C.byref(S.c), 4, 2, 0x3000, 1, 0x4000, 0x5000, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1000, ws - 8, None, None) == pm.PM_EINVAL
    assert L.projection_hash_select(C.byref(S.c), 4, 2, 0x3000, 1, 0x4000, 0x5000, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1004, ws, None, None) == pm.PM_EINVAL  # workspace not 8-byte aligned
    assert L.projection_hash_select(C.byref(S.c), 4, 2, 0x3000, 0, 0x4000, 0x5000, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1000, ws, None, None) == pm.PM_EINVAL  # no trials
    S3 = _S(_fake_seqs(n_total=40, n_min=20, n_max=20))
    assert L.projection_hash_select(C.byref(S3.c), 20, 10, 0x3000, 1, 0x4000, 0x5000, 2, 0x1, 1, 0x1, 1, 0x1,
                                    0x1000, 1 << 30, None, None) == pm.PM_ERANGE  # 4^10 bins
    # selection workspace: per-trial totals and bitmap of |Sigma|^k / 64 words;
    # 0 outside the count-table range (|Sigma|^k <= 2^19)
    assert pm.pm_select_workspace(4, 9, 10, 100) > pm.pm_select_workspace(4, 8, 10, 100) > 0
    assert pm.pm_select_workspace(4, 8, 10, 200) == pm.pm_select_workspace(4, 8, 10, 100)  # cursors in LDS
    assert pm.pm_select_workspace(4, 10, 10, 100) == 0
    assert pm.pm_select_workspace(20, 5, 10, 100) == 0
    assert pm.pm_select_workspace(20, 4, 10, 100) > 0
    assert pm.pm_select_workspace(3, 4, 10, 100) == 0
    assert L.theta_init(5, 4, 0x1, 1, None, 0x1, 1.0, 0x1, None) == pm.PM_EINVAL
    assert L.theta_init(4, 4, 0x1, 1, None, 0x1, -1.0, 0x1, None) == pm.PM_EINVAL
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, 3, 1.0, 7, 0x1, 0x1, None, None,
                       None, 0, None) == pm.PM_EINVAL
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, -1, 1.0, 0, 0x1, 0x1, None, None,
                       None, 0, None) == pm.PM_EINVAL
    # matrix-core workspace: one-hot tables of t + ceil(x/32) window pairs of
    # 1 KB + (4 ceil(l/4) + 12) x 64 B (t=2, n=10+10, l=4: x=14, 3 pairs of 2 KB)
    assert L.pm_em_workspace(C.byref(S.c), 4, pm.PM_F16X2) == 3 * 2048
    assert L.pm_em_workspace(C.byref(S.c), 4, pm.PM_FP64) == 0
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, 3, 1.0, pm.PM_F16X2, 0x1, 0x1, None, None,
                       0x1000, 3 * 2048 - 1, None) == pm.PM_EINVAL
    assert L.em_best(0x1, 1, None, 0, 0x1, 4, 40, 0x1, None, None) == pm.PM_EINVAL
    # nothing to do is fine and launches nothing
    assert L.em_refine(C.byref(S.c), 4, None, None, 0, None, 3, 1.0, 0, None, None, None, None,
                       None, 0, None) == pm.PM_OK


def test_projection_run_rejects_bad_problem():
    """Host-side checks of projection_run fail before any device call."""
    with pytest.raises(pm.PmError, match="problem 0"):
        pm.projection_run(pm.Problem(["ACGT", "ACG"], 4, 4))          # a sequence shorter than l
    with pytest.raises(pm.PmError, match="problem 1"):
        pm.projection_run([pm.Problem(["ACGTACGT"], 4, 4, k=2, s=2, masks=np.array([0b11])),
                           pm.Problem(["ACGTACGT"], 4, 4, k=2, s=2, masks=np.array([0b111]))])  # wrong popcount
    with pytest.raises(pm.PmError, match="never occurs"):
        pm.projection_run(pm.Problem(["AAAAAAAA"], 4, 4, k=2, s=2, masks=np.array([0b11])))  # bg from composition
    with pytest.raises(pm.PmError, match="triage"):
        pm.projection_run(pm.Problem(["ACGTACGT"], 4, 4, k=2, s=2, masks=np.array([0b11])), triage=True,
                          triage_weights="/nonexistent/triage.bin")
    L = pm.lib()
    assert L.projection_run(None, 0, None, None) == pm.PM_EINVAL


def test_triage_weights_file_round_trip(tmp_path):
    """The shipped binary weights equal the training output they came from,
    in the layout the header documents."""
    import json
    import struct
    with np.load(pm.default_triage_path(), allow_pickle=False) as z:
        params, mu, sd, thr = z["params"], z["mu"], z["sd"], float(z["threshold"])
        per = json.loads(str(z["meta"])).get("thresholds_by_l", {})
    raw = open(pm.default_triage_bin_path(), "rb").read()
    assert raw[:8] == b"PMTRIAG1"
    assert struct.unpack_from("<ii", raw, 8) == (pm.PM_TRIAGE_PARAMS, pm.PM_TRIAGE_INPUTS)
    o = 16
    for a, n in ((params, pm.PM_TRIAGE_PARAMS), (mu, 87), (sd, 87)):
        assert np.array_equal(np.frombuffer(raw, dtype="<f4", count=n, offset=o), a.astype(np.float32))
        o += 4 * n
    t0, nl = struct.unpack_from("<di", raw, o)
    assert t0 == thr and nl == len(per)
    o += 12
    got = {}
    for _ in range(nl):
        l, v = struct.unpack_from("<id", raw, o)
        got[l] = v
        o += 12
    assert o == len(raw) and got == {int(k): float(v) for k, v in per.items()}
    pm.convert_triage_npz(pm.default_triage_path(), str(tmp_path / "w.bin"))
    assert open(tmp_path / "w.bin", "rb").read() == raw


def _fake_batch(P=3, l=11, k=5, m=(2, 3, 1), x_fix=None, first_fix=None):
    tab = (pm.pm_inst * P)()
    item = key = 0
    for p in range(P):
        e = tab[p]
        e.offsets, e.packed = 0x1000 + 64 * p, 0x8000 + 4096 * p
        e.t, e.n_min = 2 + p, 20
        e.n_total = e.t * 20
        e.x = e.n_total - e.t * (l - 1)
        e.m, e.first_item, e.key_base = m[p], item, key
        item += m[p]
        key += m[p] * e.x
    if x_fix is not None:
        tab[x_fix].x += 1
    if first_fix is not None:
        tab[first_fix].first_item += 1
    b = pm.pm_batch(4, l, k, P, item, 0x10000, C.cast(tab, C.c_void_p), 0x20000)
    return b, tab


def test_batch_check_host_only():
    """The batch table is checked on the host (no device access)."""
    L = pm.lib()
    b, tab = _fake_batch()
    assert L.pm_batch_check(C.byref(b)) == pm.PM_OK
    for bad in (dict(x_fix=1), dict(first_fix=2)):
        b2, tab2 = _fake_batch(**bad)
        assert L.pm_batch_check(C.byref(b2)) == pm.PM_EINVAL
        assert pm.pm_last_error()
    b3, tab3 = _fake_batch()
    b3.items += 1
    assert L.pm_batch_check(C.byref(b3)) == pm.PM_EINVAL
    b4, tab4 = _fake_batch()
    b4.k = 12
    assert L.pm_batch_check(C.byref(b4)) == pm.PM_EINVAL


def test_batch_and_triage_entry_points_validate():
    L = pm.lib()
    b, tab = _fake_batch()
    # hash: keys and counts both missing
    assert L.projection_hash_batch(C.byref(b), 0x1, None, None, None, None) == pm.PM_EINVAL
    # select: workspace too small
    assert L.bucket_select_batch(C.byref(b), 0x1, 0x1, 2, 0x1, 10, 0x1, 10, 0x1, 0x1, 8, None,
                                 None) == pm.PM_EINVAL
    # EM: the matrix-core forms are DNA only; a too-small plan workspace
    S = _S(_fake_seqs(alphabet=20))
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, 3, 1.0, pm.PM_F16X2, 0x1, 0x1, None, None,
                       None, 0, None) == pm.PM_EINVAL
    # the protein matrix-core form takes l <= 24
    S25 = _S(_fake_seqs(alphabet=20, n_total=60, n_min=30, n_max=30))
    assert L.em_refine(C.byref(S25.c), 25, 0x1, 0x1, 1, None, 3, 1.0, pm.PM_F16, 0x1, 0x1, None, None,
                       None, 0, None) == pm.PM_ERANGE
    assert L.em_refine_batch(C.byref(b), 0x1, 0x1, 0x1, 10, None, 2, 1.0, pm.PM_F16X2, 0x1, 0x1, None,
                             None, 0x1, 8, None) == pm.PM_EINVAL
    # batch workspace: plan (4P+1 int64) and first slots (P+1 int64), each
    # rounded to 256 B, then the tables: instances t = 2, 3, 4 with x = 20, 30,
    # 40 at l = 11 take 3 + 4 + 6 window pairs of 1 KB + 24 x 64 B
    assert L.pm_em_batch_workspace(C.byref(b), pm.PM_F16X2) == 256 + 256 + 13 * 2560
    assert L.pm_em_batch_workspace(C.byref(b), pm.PM_FP32) == 0
    # triage: l above 21, frac outside (0, 1], workspace sizes
    assert L.triage_features(22, 0x1, 1, None, 0x1, None, None, 0x1, None) == pm.PM_EINVAL
    assert L.triage_features(15, 0x1, 1, None, 0x1, 0x1, None, 0x1, None) == pm.PM_EINVAL  # mu without sd
    ws = pm.pm_triage_select_workspace(3, 100)
    assert L.triage_select(C.addressof(b), 0x1, 0x1, 100, None, 0.0, 0x1, 4, 11, None, 0x1, 0x1, None, 0x1,
                           0x1, ws, None) == pm.PM_EINVAL
    assert L.triage_select(C.addressof(b), 0x1, 0x1, 100, None, 0.05, 0x1, 4, 12, None, 0x1, 0x1, None, 0x1,
                           0x1, ws, None) == pm.PM_EINVAL  # l differs from the batch
    assert L.triage_train_step(0x1, None, None, 0, 0x1, 0x1, 16, 1e-3, None, None, 0x1,
                               pm.pm_triage_workspace(16), None) == pm.PM_EINVAL  # Adam needs moments
    assert L.triage_train_step(0x1, None, None, 0, 0x1, 0x1, 16, 0.0, None, None, 0x1, 8,
                               None) == pm.PM_EINVAL  # workspace too small
    assert pm.pm_triage_packed_bytes() == (16 * 3 * 64 + 16 * 8 * 64) * 16 + (3 * 256 + 1) * 4
    assert pm.PM_TRIAGE_PARAMS == 87 * 256 + 256 + 256 * 256 + 256 + 256 + 1
