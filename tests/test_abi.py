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
    assert L.theta_init(5, 4, 0x1, 1, None, 0x1, 1.0, 0x1, None) == pm.PM_EINVAL
    assert L.theta_init(4, 4, 0x1, 1, None, 0x1, -1.0, 0x1, None) == pm.PM_EINVAL
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, 3, 1.0, 7, 0x1, 0x1, None, None,
                       None) == pm.PM_EINVAL
    assert L.em_refine(C.byref(S.c), 4, 0x1, 0x1, 1, None, -1, 1.0, 0, 0x1, 0x1, None, None,
                       None) == pm.PM_EINVAL
    assert L.em_best(0x1, 1, None, 0, 0x1, 4, 40, 0x1, None, None) == pm.PM_EINVAL
    # nothing to do is fine and launches nothing
    assert L.em_refine(C.byref(S.c), 4, None, None, 0, None, 3, 1.0, 0, None, None, None, None,
                       None) == pm.PM_OK


def test_projection_run_rejects_bad_problem():
    with pytest.raises(pm.PmError):
        pm.projection_run(["ACGT", "ACG"], 4, 4)          # a sequence shorter than l
    with pytest.raises(pm.PmError):
        pm.projection_run(["ACGTACGT"], 4, 4, k=2, s=2, masks=np.array([0b111]))  # wrong popcount
