"""The allocation-free fused selection (bucket_hash_select_noalloc) against
the workspace form (bucket_hash_select) through the C ABI: two calls in a row
on one device, the second on a smaller instance, each compared with the
workspace form on the same input (bucket records bit-exact, every bucket's
members equal as a set, totals equal); and the size limit refused before
anything runs."""
import sys

import numpy as np
import pytest

import paper_1605_06904_amd as pm
from synth import planted_instance, projection_masks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def _lists(S, l, k, masks, s, noalloc):
    m = len(masks)
    dm = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if noalloc:
        run = lambda bk, cb, mem, cm: pm.bucket_hash_select_noalloc(S, l, k, dm, m, s, bk, cb, mem, cm, n_out, st)
    else:
        nbytes = pm.pm_hash_select_workspace(S, l, k, m)
        ws = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")
        run = lambda bk, cb, mem, cm: pm.bucket_hash_select(S, l, k, dm, m, s, bk, cb, mem, cm, n_out, ws, nbytes,
                                                            st)
    run(None, 0, None, 0)
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in n_out.cpu()]
    bk = torch.full((max(nb_, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(nm_, 1),), -1, dtype=torch.int32, device="cuda")
    st.zero_()  # the sizing call flags its zero capacities
    run(bk, nb_, mem, nm_)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert [int(v) for v in n_out.cpu()] == [nb_, nm_]
    return bk.cpu().numpy().view(np.uint32)[:nb_], mem.cpu().numpy().view(np.uint32)[:nm_]


def _same(a, b):
    bk_a, mem_a = a
    bk_b, mem_b = b
    assert np.array_equal(bk_a, bk_b)
    assert len(mem_a) == len(mem_b)
    for rec in bk_a:
        f, n = int(rec[3]), int(rec[2])
        assert np.array_equal(np.sort(mem_a[f:f + n]), np.sort(mem_b[f:f + n]))


def test_noalloc_matches_workspace_form_on_two_calls():
    rng = np.random.default_rng(77)
    # a larger instance (several tiles, two histogram slices), then a smaller one
    cases = [(planted_instance(rng, 20, 1000, 18, 6), 18, 8, 4, 300),
             (planted_instance(rng, 7, 250, 12, 2), 12, 6, 3, 21)]
    for inst, l, k, s, m in cases:
        masks = projection_masks(rng, l, k, m)
        S = pm.Seqs(4, inst.seqs)
        say(f"noalloc t={len(inst.seqs)} l={l} k={k} s={s} m={m}")
        ref = _lists(S, l, k, masks, s, noalloc=False)
        got = _lists(S, l, k, masks, s, noalloc=True)
        assert len(ref[0]) > 0
        _same(got, ref)


def test_noalloc_rejects_more_trials_than_the_scratch_holds():
    rng = np.random.default_rng(5)
    inst = planted_instance(rng, 4, 120, 10, 2)
    S = pm.Seqs(4, inst.seqs)
    per = 4 * 8  # bytes per trial-slice entry
    m = (pm.pm_hash_select_scratch_bytes() - 256) // per + 1
    masks = projection_masks(rng, 10, 5, m)
    dm = torch.from_numpy(masks.view(np.int32)).cuda()
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert pm.pm_hash_select_workspace(S, 10, 5, m) > pm.pm_hash_select_scratch_bytes()
    with pytest.raises(pm.PmError) as e:
        pm.bucket_hash_select_noalloc(S, 10, 5, dm, m, 3, None, 0, None, 0, n_out)
    assert e.value.code == pm.PM_ERANGE
    assert "scratch" in str(e.value)
    # the same call one trial-slice inside the limit runs
    m_ok = m - 1
    pm.bucket_hash_select_noalloc(S, 10, 5, dm, m_ok, 3, None, 0, None, 0, n_out)
    torch.cuda.synchronize()
    assert int(n_out[0].item()) >= 0
